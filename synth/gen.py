"""Seeded generators (inputs only; no view-maintenance arithmetic)."""

from __future__ import annotations

import numpy as np

# Spawn-key purposes: the second element of every key.
KEY_A = 1
KEY_UPDATES = 2
KEY_ROWS = 3
KEY_GRAPH = 4
KEY_SPECTRAL = 5
KEY_INT = 6
KEY_GENERAL = 7


def rng(seed: int, *key: int) -> np.random.Generator:
    """PCG64 generator for stream `key` under `seed`."""
    ss = np.random.SeedSequence(int(seed), spawn_key=tuple(int(k) for k in key))
    return np.random.Generator(np.random.PCG64(ss))


def spectral_norm_estimate(A: np.ndarray, seed: int = 0) -> float:
    """Largest singular value of A.

    Exact (LAPACK SVD) for n <= 1024.  Above that, ARPACK's implicitly
    restarted Lanczos (scipy svds, k = 1) from a seeded Gaussian start vector,
    converged to a relative tolerance of 1e-8; the result is a deterministic
    function of (A, seed) and agrees with the SVD to ~1e-15 on these
    matrices.
    """
    n = A.shape[0]
    if n <= 1024:
        return float(np.linalg.norm(A, 2))
    from scipy.sparse.linalg import svds
    v0 = rng(seed, KEY_SPECTRAL, n).standard_normal(min(A.shape))
    return float(svds(A, k=1, v0=v0, tol=1e-8, return_singular_vectors=False)[0])


def gaussian_matrix(n: int, seed: int = 0, config: int = 0, view: int = 0,
                    target_norm: float | None = 0.9) -> np.ndarray:
    """n x n FP64 matrix with i.i.d. N(0, 1/n) entries, rescaled to spectral
    norm `target_norm` (no rescaling when target_norm is None)."""
    g = rng(seed, config, KEY_A, view)
    A = g.standard_normal((n, n))
    A *= 1.0 / np.sqrt(n)
    if target_norm is not None and n > 0:
        s = spectral_norm_estimate(A, seed=seed)
        A *= target_norm / s
    return A


def update_factors(n: int, r: int, count: int, seed: int = 0, config: int = 0,
                   view: int = 0, sigma: float | None = None) -> tuple[np.ndarray, np.ndarray]:
    """`count` update factor pairs (U_t, V_t), each n x r, FP64.

    Entries are i.i.d. N(0, sigma) with standard deviation sigma
    (default 1e-2 / sqrt(n)).  Returns arrays of shape (count, n, r).
    """
    if sigma is None:
        sigma = 1e-2 / np.sqrt(max(n, 1))
    g = rng(seed, config, KEY_UPDATES, view)
    U = g.standard_normal((count, n, r)) * sigma
    V = g.standard_normal((count, n, r)) * sigma
    return U, V


def zipf_rows(n: int, count: int, s: float, seed: int = 0, config: int = 0,
              view: int = 0) -> np.ndarray:
    """`count` row indices in [0, n) whose frequencies follow a Zipf law with
    exponent s over a seeded permutation of the rows (s = 0 is uniform)."""
    g = rng(seed, config, KEY_ROWS, view)
    ranks = np.arange(1, n + 1, dtype=np.float64)
    w = ranks ** (-float(s))
    w /= w.sum()
    perm = g.permutation(n)
    draws = g.choice(n, size=count, p=w)
    return perm[draws]


def row_updates(n: int, count: int, s: float = 0.0, seed: int = 0,
                config: int = 0, view: int = 0,
                sigma: float | None = None) -> tuple[np.ndarray, np.ndarray]:
    """Rank-1 row updates: u_t = e_{i_t} and v_t a random row change.

    Row indices follow zipf_rows(s).  Returns (U, V) of shape (count, n, 1).
    """
    if sigma is None:
        sigma = 1e-2 / np.sqrt(max(n, 1))
    rows = zipf_rows(n, count, s, seed, config, view)
    g = rng(seed, config, KEY_UPDATES, view, 1)
    U = np.zeros((count, n, 1))
    U[np.arange(count), rows, 0] = 1.0
    V = g.standard_normal((count, n, 1)) * sigma
    return U, V


def random_dag(n: int, p: float, seed: int = 0) -> np.ndarray:
    """0/1 adjacency matrix (FP64) of a random DAG: edge a->b with
    probability p for a < b (topological order = index order)."""
    g = rng(seed, 0, KEY_GRAPH, n)
    M = (g.random((n, n)) < p).astype(np.float64)
    return np.triu(M, 1)


def integer_matrix(shape, lo: int, hi: int, seed: int = 0, tag: int = 0) -> np.ndarray:
    """Integer-valued FP64 array with entries uniform in [lo, hi]."""
    g = rng(seed, 0, KEY_INT, tag)
    return g.integers(lo, hi + 1, size=shape).astype(np.float64)


def round_to(x: np.ndarray, dtype) -> np.ndarray:
    """Round once to `dtype` (e.g. np.float32) and return the rounded values
    as an array of that dtype (C-contiguous)."""
    return np.ascontiguousarray(np.asarray(x, dtype=dtype))


def general_operands(n: int, p: int, seed: int = 0, config: int = 0,
                     view: int = 0) -> tuple[np.ndarray, np.ndarray]:
    """T_0 and B of the general form T_{i+1} = A T_i + B, both n x p FP64:
    T_0 with i.i.d. N(0, 1) entries, B with i.i.d. N(0, 0.01) entries (so
    that with a spectral norm of A near 0.9 the fixed point B / (I - A) is
    of the size of T_0)."""
    g = rng(seed, config, KEY_GENERAL, view)
    T0 = g.standard_normal((n, p))
    B = g.standard_normal((n, p)) * 0.1
    return T0, B


def regression_problem(n: int, p: int, samples: int, seed: int = 0,
                       config: int = 0) -> tuple[np.ndarray, np.ndarray, float]:
    """Gradient-descent linear regression as a general form (the regression
    experiment of Sec. 7): theta_{i+1} = theta_i - eta X^T (X theta_i - Y)
    is T_{i+1} = A T_i + B with A = I - eta X^T X and B = eta X^T Y.
    X (samples x n) and Y (samples x p) have i.i.d. N(0, 1) entries; eta is
    1 / ||X||_2^2, which puts the spectrum of A in [0, 1).  Returns
    (A, B, eta), FP64."""
    g = rng(seed, config, KEY_GENERAL, 1)
    X = g.standard_normal((samples, n))
    Y = g.standard_normal((samples, p))
    s = float(np.linalg.norm(X, 2)) if min(X.shape) <= 1024 else spectral_norm_estimate(X, seed=seed)
    eta = 1.0 / (s * s)
    A = np.eye(n) - eta * (X.T @ X)
    B = eta * (X.T @ Y)
    return A, B, eta


def regression_rows(n: int, count: int, eta: float, seed: int = 0,
                    config: int = 0) -> tuple[np.ndarray, np.ndarray]:
    """New training rows x_t as rank-1 changes of A = I - eta X^T X:
    Delta A = (-eta x_t) x_t^T.  x_t has i.i.d. N(0, 1) entries.  Returns
    (U, V) of shape (count, n, 1)."""
    g = rng(seed, config, KEY_GENERAL, 2)
    x = g.standard_normal((count, n, 1))
    return -eta * x, x.copy()
