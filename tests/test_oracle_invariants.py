"""Oracle invariants that hold exactly (bit for bit) or to rounding, and the
shape of the solution path (|v_k| non-increasing, z_j concave in lambda)."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2402_16712_amd import workloads as wl


def _prob(seed):
    p = wl.small_fit(seed)
    return p.X, float(p.lambdas[0])


@pytest.mark.parametrize("seed", [0, 1])
def test_row_sign_flip_is_bit_identical(seed):
    X, lam = _prob(seed)
    a = O.fit(X, lam)
    Y = X.copy(order="F")
    flip = np.random.default_rng(seed).random(X.shape[0]) < 0.5
    Y[flip, :] *= -1.0
    b = O.fit(Y, lam)
    assert a["j"] == b["j"]
    assert a["v"].tobytes() == b["v"].tobytes()
    assert a["z_all"].tobytes() == b["z_all"].tobytes()
    assert (a["row"] == b["row"]).all()


@pytest.mark.parametrize("s", [-3, 5])
def test_power_of_two_scaling_is_exact(s):
    X, lam = _prob(2)
    a = O.fit(X, lam)
    b = O.fit(np.asfortranarray(X * 2.0 ** s), lam * 2.0 ** s)
    assert a["j"] == b["j"] and (a["row"] == b["row"]).all()
    assert a["v"].tobytes() == b["v"].tobytes()
    assert (a["z_all"] * 2.0 ** s).tobytes() == b["z_all"].tobytes()


def test_column_negation_negates_v():
    X, lam = _prob(3)
    a = O.fit(X, lam)
    k = (a["j"] + 1) % X.shape[1]
    Y = X.copy(order="F")
    Y[:, k] *= -1.0
    b = O.fit(Y, lam)
    assert a["j"] == b["j"]
    assert b["v"][k] == -a["v"][k] or (a["v"][k] == 0 and b["v"][k] == 0)
    assert a["z_all"].tobytes() == b["z_all"].tobytes()


def test_row_permutation_to_rounding():
    X, lam = _prob(4)
    a = O.fit(X, lam)
    perm = np.random.default_rng(1).permutation(X.shape[0])
    b = O.fit(np.asfortranarray(X[perm]), lam)
    assert a["j"] == b["j"]
    assert (a["v"] == b["v"]).all()
    np.testing.assert_allclose(a["z_all"], b["z_all"], rtol=1e-12)


def test_path_shape():
    X, _ = _prob(5)
    big = float(np.abs(X).sum(0).max())
    lams = np.linspace(0.0, big, 41)
    for j in (0, 7, 13):
        f = O.fit_j(X, j, lams)
        absv = np.abs(f["V"])
        assert (np.diff(absv, axis=0) <= 0).all(), "|v_k(lambda)| must not grow"
        z = f["ZJ"]
        second = z[2:] - 2 * z[1:-1] + z[:-2]
        assert (second <= 1e-9 * z.max()).all(), "z_j(lambda) must be concave"
        assert np.count_nonzero(f["V"][-1]) == 1


def test_path_equals_fits():
    X, _ = _prob(6)
    lams = wl.log_lambdas(float(np.abs(X).sum(0).max()), 6)
    p = O.fit_path(X, lams)
    for t, lam in enumerate(lams):
        f = O.fit(X, lam)
        assert f["j"] == p["J"][t] and f["obj"] == p["OBJ"][t]
        assert f["v"].tobytes() == p["V"][t].tobytes()


def test_status_codes():
    X, lam = _prob(0)
    Y = X.copy(order="F")
    Y[3, 4] = np.nan
    with pytest.raises(O.OracleError) as e:
        O.fit(Y, lam)
    assert e.value.code == O.ENONFINITE
    with pytest.raises(O.OracleError) as e:
        O.fit(X, -1.0)
    assert e.value.code == O.EINVAL
    # overflowing selected ratio: tiny x_ij under huge x_ik
    Z = np.asfortranarray(np.array([[1e-300, 1e300], [2e-300, 3e300], [1e-300, 2e300]]))
    r = O.fit_j(Z, 0, [0.0])
    assert r["status"] == O.ERANGE and np.isinf(r["V"][0, 1])


def test_all_zero_column_gives_unit_vector():
    X = wl.random_small(3, 10, 4)
    X[:, 2] = 0.0
    f = O.fit_j(X, 2, [0.5])
    assert f["V"][0].tolist() == [0.0, 0.0, 1.0, 0.0]
    assert abs(f["ZJ"][0] - (np.abs(X).sum() + 0.5)) < 1e-12 * f["ZJ"][0]
