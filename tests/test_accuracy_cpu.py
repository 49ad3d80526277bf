"""The accuracy study's measures and generator (CPU)."""
import numpy as np

from paper_2402_16712_amd import accuracy as A
from paper_2402_16712_amd import workloads as wl


def test_discordance_is_a_line_distance():
    v = np.array([3.0, -4.0, 0.0])
    assert A.discordance(v, v) == 0.0
    assert A.discordance(v, -2.5 * v) == 0.0                 # direction sign and scale
    assert A.discordance(v, np.array([4.0, 3.0, 0.0])) == 1.0  # orthogonal
    # 60 degrees: 1 - cos = 1/2
    assert abs(A.discordance([1.0, 0.0], [0.5, np.sqrt(3.0) / 2]) - 0.5) < 1e-15
    assert A.discordance(v, np.zeros(3)) == 1.0


def test_sparsity_share():
    assert A.sparsity([0.0, 1.0, 0.0, -2.0]) == 0.5
    assert A.sparsity([1.0, 0.0]) == 0.5


def test_generator_recipe():
    X, v = wl.accuracy_matrix(400, 30, 0)
    assert X.shape == (400, 30) and X.flags.f_contiguous
    assert abs(np.linalg.norm(v) - 1.0) < 1e-12 and np.all(v != 0.0)
    # rank one plus Laplace(0, 1) noise: the residual off the true line has
    # the noise's mean absolute value 1 (per entry), the scores span +-100
    alpha = X @ v
    R = X - np.outer(alpha, v)
    assert 0.85 < np.mean(np.abs(R)) < 1.15
    assert np.max(np.abs(alpha)) > 80.0
    X2, v2 = wl.accuracy_matrix(400, 30, 0)
    assert np.array_equal(X, X2) and np.array_equal(v, v2)
