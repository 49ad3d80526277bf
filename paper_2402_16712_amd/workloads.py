"""Seeded synthetic inputs for the sparse robust l1 line fit.

This module only draws numbers: it holds none of the method's arithmetic, so
both the CPU oracle (tests) and the HIP path (tests, smoke, bench) take their
inputs from here.  Every draw comes from numpy's Philox-4x32-10 counter-based
generator keyed by an explicit integer seed, so a (recipe, seed) pair names
one matrix on every machine.

Recipe (the paper's simulation setting, Sec. "Experiments with Synthetic
Data", is a rank-one signal plus heavy-tailed noise plus gross outliers):

    X = u l^T + E
    u ~ N(0, 1)^n                       latent scores
    l : s loadings ~ U[-1, 1] at s random positions, zero elsewhere
    E ~ Laplace(0, b) iid               (b = 0.1)
    outlier rows (chosen without replacement) replaced by iid
        N(0, sigma_out^2) entries
    a fraction of entries (chosen without replacement) set to exactly +0.0

X is returned column-major (numpy order='F'), the layout the library takes:
x(i, k) = X[i + k * ld] with ld = n.
"""
from __future__ import annotations

import dataclasses

import numpy as np

LAPLACE_B = 0.1


def _rng(*key: int) -> np.random.Generator:
    # Philox keyed by the seed words: counter based, stable across platforms.
    words = [int(k) & 0xFFFFFFFFFFFFFFFF for k in key]
    ss = np.random.SeedSequence(words)
    return np.random.Generator(np.random.Philox(ss))


def rank_one_matrix(n: int, m: int, s: int, n_outlier_rows: int,
                    outlier_sigma: float, zero_frac: float, seed,
                    laplace_b: float = LAPLACE_B) -> np.ndarray:
    """One n x m FP64 matrix of the recipe above (column-major)."""
    if isinstance(seed, (tuple, list)):
        rng = _rng(*seed)
    else:
        rng = _rng(seed)
    u = rng.standard_normal(n)
    load = np.zeros(m)
    s = int(min(max(s, 0), m))
    if s:
        pos = rng.choice(m, size=s, replace=False)
        load[pos] = rng.uniform(-1.0, 1.0, size=s)
    X = np.outer(u, load) + rng.laplace(0.0, laplace_b, size=(n, m))
    n_out = int(min(max(n_outlier_rows, 0), n))
    if n_out:
        rows = rng.choice(n, size=n_out, replace=False)
        X[rows, :] = outlier_sigma * rng.standard_normal((n_out, m))
    nz = int(round(zero_frac * n * m))
    if nz:
        flat = rng.choice(n * m, size=nz, replace=False)
        X.reshape(-1)[flat] = 0.0
    return np.asfortranarray(X)


def max_column_mass(X: np.ndarray) -> float:
    """Lambda-scale of a workload: max_j sum_i |x_ij| (numpy's own sum)."""
    return float(np.abs(X).sum(axis=0).max()) if X.size else 0.0


def log_lambdas(big: float, L: int, lo_exp: float = -3.0) -> np.ndarray:
    """L values big * 10^(lo_exp + (-lo_exp) t/(L-1)), t = 0..L-1 (last = big)."""
    if L == 1:
        return np.array([big])
    t = np.arange(L, dtype=np.float64)
    lam = big * 10.0 ** (lo_exp + (-lo_exp) * t / (L - 1))
    lam[-1] = big
    return lam


# ---------------------------------------------------------------- workloads

@dataclasses.dataclass
class Problem:
    X: np.ndarray            # n x m FP64, column-major
    lambdas: np.ndarray      # L FP64 penalties
    name: str

    @property
    def n(self) -> int:
        return self.X.shape[0]

    @property
    def m(self) -> int:
        return self.X.shape[1]


def small_fit(seed: int = 0) -> Problem:
    """n=200 x m=20: 4 nonzero loadings, 10 rows (5%) replaced by N(0,100^2)
    outliers, no exact zeros, lambda = 0.1 * max column mass."""
    X = rank_one_matrix(200, 20, 4, 10, 100.0, 0.0, (0, seed))
    lam = 0.1 * max_column_mass(X)
    return Problem(X, np.array([lam]), f"fit-200x20-seed{seed}")


def large_fit(seed: int = 0, n: int = 2000, m: int = 2000) -> Problem:
    """n x m (2000 x 2000): 10% of m nonzero loadings, 10% outlier rows
    replaced by 20*N(0,1), 1% exact zeros, lambda = 0.05 * max column mass."""
    X = rank_one_matrix(n, m, max(1, m // 10), n // 10, 20.0, 0.01, (1, seed, n, m))
    lam = 0.05 * max_column_mass(X)
    return Problem(X, np.array([lam]), f"fit-{n}x{m}-seed{seed}")


def lambda_path(seed: int = 0, n: int = 2000, m: int = 2000, L: int = 64) -> Problem:
    """Same matrix recipe as large_fit; L penalties log-spaced from
    1e-3 * Lambda to Lambda, Lambda = max column mass."""
    X = rank_one_matrix(n, m, max(1, m // 10), n // 10, 20.0, 0.01, (1, seed, n, m))
    return Problem(X, log_lambdas(max_column_mass(X), L), f"path-{n}x{m}x{L}-seed{seed}")


def uneven_batch(batch_seed: int = 12345, B: int = 512, L: int = 16,
                 n_range=(50, 4000), m_range=(10, 500)) -> list[Problem]:
    """B independent matrices, n ~ U{n_range}, m ~ U{m_range}, sparsity
    round(0.1 m), outlier fraction ~ U[0.05, 0.15], 1% zeros, L log-spaced
    penalties per matrix."""
    rng = _rng(3, batch_seed)
    ns = rng.integers(n_range[0], n_range[1] + 1, size=B)
    ms = rng.integers(m_range[0], m_range[1] + 1, size=B)
    fr = rng.uniform(0.05, 0.15, size=B)
    out = []
    for b in range(B):
        n, m = int(ns[b]), int(ms[b])
        X = rank_one_matrix(n, m, max(1, int(round(0.1 * m))), int(round(fr[b] * n)),
                            20.0, 0.01, (4, batch_seed, b))
        out.append(Problem(X, log_lambdas(max_column_mass(X), L), f"batch{batch_seed}-{b}-{n}x{m}"))
    return out


def ranker_matrix(index: int, n: int | None = None, m: int | None = None,
                  n_range=(500, 4000), m_range=(50, 500)) -> Problem:
    """Training / evaluation matrices for the candidate ranker: sizes drawn
    from the given ranges unless fixed, same recipe, lambda = 0.05 * mass."""
    rng = _rng(5, index)
    if n is None:
        n = int(rng.integers(n_range[0], n_range[1] + 1))
    if m is None:
        m = int(rng.integers(m_range[0], m_range[1] + 1))
    X = rank_one_matrix(n, m, max(1, m // 10), n // 10, 20.0, 0.01, (6, index, n, m))
    return Problem(X, np.array([0.05 * max_column_mass(X)]), f"rank{index}-{n}x{m}")


def random_small(seed: int, n: int, m: int, integer: bool = False,
                 zero_frac: float = 0.0, span: int = 5) -> np.ndarray:
    """Tiny dense matrices for exhaustive checks: iid N(0,1) entries, or
    integers in [-span, span] (many exact ties among ratios)."""
    rng = _rng(7, seed, n, m, int(integer))
    if integer:
        X = rng.integers(-span, span + 1, size=(n, m)).astype(np.float64)
    else:
        X = rng.standard_normal((n, m))
    nz = int(round(zero_frac * n * m))
    if nz:
        X.reshape(-1)[rng.choice(n * m, size=nz, replace=False)] = 0.0
    return np.asfortranarray(X)


def rank_one_matrix_torch(n: int, m: int, s: int, n_outlier_rows: int, outlier_sigma: float,
                          zero_frac: float, seed: int, device="cuda:0", laplace_b: float = LAPLACE_B):
    """The same recipe as rank_one_matrix, drawn on the GPU with torch's
    seeded Philox generator (for the large training and evaluation sets of
    the candidate ranker).  Returns a column-major (n, m) FP64 device tensor
    (strides (1, n))."""
    import torch
    g = torch.Generator(device=device)
    g.manual_seed(int(seed) & 0x7FFFFFFFFFFFFFFF)
    f64 = torch.float64
    u = torch.randn(n, generator=g, device=device, dtype=f64)
    load = torch.zeros(m, device=device, dtype=f64)
    s = int(min(max(s, 0), m))
    if s:
        pos = torch.randperm(m, generator=g, device=device)[:s]
        load[pos] = torch.rand(s, generator=g, device=device, dtype=f64) * 2.0 - 1.0
    # Laplace(0, b) by inversion of a uniform on (-1/2, 1/2)
    U = torch.rand((m, n), generator=g, device=device, dtype=f64) - 0.5
    noise = -laplace_b * torch.sign(U) * torch.log1p(-2.0 * U.abs())
    XT = load[:, None] * u[None, :] + noise                       # (m, n): column k is row k
    n_out = int(min(max(n_outlier_rows, 0), n))
    if n_out:
        rows = torch.randperm(n, generator=g, device=device)[:n_out]
        XT[:, rows] = outlier_sigma * torch.randn((m, n_out), generator=g, device=device, dtype=f64)
    nz = int(round(zero_frac * n * m))
    if nz:
        flat = torch.randperm(n * m, generator=g, device=device)[:nz]
        XT.view(-1)[flat] = 0.0
    return XT.t()


def ranker_matrix_torch(index: int, n=None, m=None, n_range=(500, 4000), m_range=(50, 500),
                        device="cuda:0"):
    """Ranker training / evaluation matrix `index` on the GPU: sizes from the
    ranges unless fixed, 10% of m nonzero loadings, 10% outlier rows replaced
    by 20*N(0,1), 1% zeros, lambda = 0.05 * max column mass."""
    import torch
    rng = _rng(8, index)
    if n is None:
        n = int(rng.integers(n_range[0], n_range[1] + 1))
    if m is None:
        m = int(rng.integers(m_range[0], m_range[1] + 1))
    X = rank_one_matrix_torch(n, m, max(1, m // 10), n // 10, 20.0, 0.01, 1_000_003 * index + 17, device)
    lam = 0.05 * float(X.abs().sum(dim=0).max())
    return X, lam


def accuracy_matrix(n: int, m: int, seed: int, noise_b: float = 1.0):
    """The simulation of the paper's study of Algorithm 1 as lambda varies
    (Sec. 3, "Effect of Varying m and n on Error and Sparsity"): a dense true
    direction v with coordinates ~ U(-1, 1) scaled to unit l2 norm, scores
    alpha ~ U(-100, 100), x_i = alpha_i v + Laplace(0, noise_b) noise, no
    outliers.  Returns (X n x m column-major, v)."""
    rng = _rng(10, seed, n, m)
    v = rng.uniform(-1.0, 1.0, size=m)
    v = v / np.sqrt(np.sum(v * v))
    alpha = rng.uniform(-100.0, 100.0, size=n)
    X = np.outer(alpha, v) + rng.laplace(0.0, noise_b, size=(n, m))
    return np.asfortranarray(X), v
