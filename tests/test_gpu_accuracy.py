"""The accuracy study of Algorithm 1 at a reduced size: the library's fits
along the penalty grid equal the oracle's, and the curves behave as the
study describes (a dense, nearly exact line at lambda = 0; fewer nonzero
coordinates and a larger discordance as lambda grows)."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2402_16712_amd import accuracy as A
from paper_2402_16712_amd import workloads as wl

pytestmark = pytest.mark.gpu


def test_accuracy_curves_reduced():
    import torch
    from paper_2402_16712_amd import binding as B
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = B.Context(0)
    try:
        X, v = wl.accuracy_matrix(600, 200, 0)
        X1, _ = wl.accuracy_matrix(600, 200, 1)
        top = max(wl.max_column_mass(X), wl.max_column_mass(X1))
        lam = np.linspace(0.0, top, 16)                     # up to every v_k = 0
        res = A.run(c, [(600, 200)], lam, [0, 1])["600x200"]
        g = c.fit_path(B.device_matrix(X), lam)
        torch.cuda.synchronize()
        V = g["V"].cpu().numpy()
    finally:
        c.close()
    r = O.fit_path(X, lam)
    assert V.tobytes() == r["V"].tobytes()
    d, s = np.array(res["discordance"]), np.array(res["sparsity"])
    assert s[0] == 1.0 and d[0] < 0.01
    assert np.all(np.diff(s) <= 1e-12)                      # sparser as lambda grows
    assert s[-1] == 1.0 / 200 and d[-1] > d[0]             # lambda >= every column mass: v* = e_j
