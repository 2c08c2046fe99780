"""Seeded synthetic ridge problems shaped like the paper's workloads.

This module only generates inputs (X, y, lambda); it contains none of the
solver's arithmetic. Both the HIP library's callers and the CPU oracle's
tests consume what it returns.

Recipes (numpy PCG64, ``data_seed`` fixed per workload):

* dense:   X_ij ~ N(0, 1), optionally times a per-column scale exp(s * xi_j)
           with xi_j ~ N(0, 1) (log-normal column norms), optionally with a
           fraction of columns replaced by 0.9 * (a random partner column)
           + sqrt(1 - 0.81) * fresh noise (correlated pairs);
* csr:     exactly ``nnz`` distinct positions drawn uniformly over the n x d
           grid (row and column counts then follow Poisson-like laws),
           values N(0, 1);
* targets: y = X w* + noise_scale * N(0, 1) with w* ~ N(0, 1);
* kernel points: n points in d dimensions drawn around n / 10 cluster centres
           (centres N(0, I), offsets spread * N(0, I)), each coordinate then
           standardised; targets y = sin(P v) + 0.1 N(0, 1) with v ~ N(0, I / d).

The paper's own datasets (Boston, California Housing, RCV1, YearPredictionMSD)
are not used; these synthetic matrices stand in for them.
"""
from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp

DATA_SEED_BASE = 2105055650


@dataclass
class Problem:
    name: str
    X: object            # numpy array (n x d) or scipy.sparse.csr_matrix
    y: np.ndarray        # FP64 [n]
    lam: float
    w_star: np.ndarray   # the generating weights (not the ridge solution)


def dense_matrix(n, d, rng, dtype=np.float64, col_log_sigma=0.0, corr_frac=0.0, corr_rho=0.9):
    X = rng.standard_normal((n, d), dtype=np.float64 if dtype == np.float64 else np.float32)
    if corr_frac > 0.0:
        ncorr = int(round(corr_frac * d))
        cols = rng.choice(d, size=ncorr, replace=False)
        for j in cols:
            p = int(rng.integers(0, d - 1))
            p = p + 1 if p >= j else p
            g = rng.standard_normal(n).astype(X.dtype)
            X[:, j] = corr_rho * X[:, p] + np.sqrt(1.0 - corr_rho ** 2) * g
    if col_log_sigma > 0.0:
        scale = np.exp(col_log_sigma * rng.standard_normal(d))
        X *= scale.astype(X.dtype)[None, :]
    return np.ascontiguousarray(X.astype(dtype, copy=False))


def csr_matrix(n, d, nnz, rng, dtype=np.float32):
    lin = rng.choice(n * d, size=nnz, replace=False)
    lin.sort()
    rows = lin // d
    cols = (lin % d).astype(np.int32)
    vals = rng.standard_normal(nnz).astype(dtype)
    indptr = np.zeros(n + 1, dtype=np.int64)
    np.add.at(indptr, rows + 1, 1)
    indptr = np.cumsum(indptr)
    X = sp.csr_matrix((vals, cols, indptr), shape=(n, d))
    X.has_sorted_indices = True
    return X


def targets(X, rng, noise=0.01):
    d = X.shape[1]
    w_star = rng.standard_normal(d)
    Xw = np.asarray(X @ w_star.astype(np.float64) if sp.issparse(X)
                    else X.astype(np.float64, copy=False) @ w_star).ravel()
    y = Xw + noise * rng.standard_normal(X.shape[0])
    return y, w_star


def make_dense(n, d, lam, seed, dtype=np.float64, col_log_sigma=0.0, corr_frac=0.0, name=None):
    rng = np.random.Generator(np.random.PCG64(seed))
    X = dense_matrix(n, d, rng, dtype, col_log_sigma, corr_frac)
    y, w_star = targets(X, rng)
    return Problem(name or f"dense_{n}x{d}", X, y, lam, w_star)


def make_csr(n, d, density, lam, seed, dtype=np.float32, name=None):
    rng = np.random.Generator(np.random.PCG64(seed))
    nnz = int(round(density * n * d))
    X = csr_matrix(n, d, nnz, rng, dtype)
    y, w_star = targets(X, rng)
    return Problem(name or f"csr_{n}x{d}", X, y, lam, w_star)


@dataclass
class KernelProblem:
    name: str
    P: np.ndarray        # n x d points, FP64
    y: np.ndarray        # FP64 [n]
    lam: float
    sigma: float         # Gaussian kernel width


def make_points(n, d, lam, sigma, seed, clusters=None, spread=0.3, name=None):
    rng = np.random.Generator(np.random.PCG64(seed))
    nc = clusters if clusters else max(1, n // 10)
    centres = rng.standard_normal((nc, d))
    label = rng.integers(0, nc, size=n)
    P = centres[label] + spread * rng.standard_normal((n, d))
    P = (P - P.mean(axis=0)) / P.std(axis=0)
    v = rng.standard_normal(d) / np.sqrt(d)
    y = np.sin(P @ v) + 0.1 * rng.standard_normal(n)
    return KernelProblem(name or f"points_{n}x{d}", np.ascontiguousarray(P), y, lam, sigma)


# The workloads, with reduced shape-alike variants for fast tests.
def dense_primal(scale=1.0, seed=DATA_SEED_BASE + 0):
    """X 2000 x 500 FP64 N(0,1), lambda = 1e-2 (subsample sketch, tau = 50)."""
    n, d = int(2000 * scale), int(500 * scale)
    return make_dense(n, d, 1e-2, seed, np.float64, name=f"dense_primal_{n}x{d}")


def sparse_csr(scale=1.0, seed=DATA_SEED_BASE + 1):
    """CSR X 100000 x 20000 FP32, density 0.1%, lambda = 1e-3 (count / SubCount, tau = 500)."""
    n, d = int(100000 * scale), int(20000 * scale)
    return make_csr(n, d, 1e-3, 1e-3, seed, np.float32, name=f"csr_{n}x{d}")


def dense_mixed(scale=1.0, seed=DATA_SEED_BASE + 2):
    """X 50000 x 8192 FP32, N(0,1) times log-normal(0,1) column scales, lambda = 1e-1."""
    n, d = int(50000 * scale), int(8192 * scale)
    return make_dense(n, d, 1e-1, seed, np.float32, col_log_sigma=1.0, name=f"dense_mixed_{n}x{d}")


def dense_learned(scale=1.0, seed=DATA_SEED_BASE + 4):
    """X 200000 x 4096 FP32, log-normal(0,2) column norms, 5% correlated columns, lambda = 1e-2."""
    n, d = int(200000 * scale), int(4096 * scale)
    return make_dense(n, d, 1e-2, seed, np.float32, col_log_sigma=2.0, corr_frac=0.05,
                      name=f"dense_learned_{n}x{d}")


def kernel_california(scale=1.0, seed=DATA_SEED_BASE + 5):
    """20640 points in 8 dimensions (the shape of the California Housing kernel problem),
    Gaussian kernel sigma = 0.5, lambda = 1e-6 (subsample sketch, tau = m / 4)."""
    n = int(20640 * scale)
    return make_points(n, 8, 1e-6, 0.5, seed, name=f"kernel_california_{n}x8")


def kernel_boston(seed=DATA_SEED_BASE + 6):
    """506 points in 13 dimensions (the shape of the Boston kernel problem), sigma = 0.5
    sqrt(13 / 8) (the same typical kernel values as in 8 dimensions), lambda = 1e-6
    (tau = floor(m / 4) = 126)."""
    return make_points(506, 13, 1e-6, 0.5 * np.sqrt(13.0 / 8.0), seed, name="kernel_boston_506x13")


def accel_points(seed=DATA_SEED_BASE + 7):
    """The acceleration experiment's problem: kernel ridge with sigma = 0.5 and lambda = 1/n on
    the rows of a random sparse 2000 x 500 matrix of density 0.25 (values uniform on [0, 1),
    exactly round(0.25 n d) distinct uniform positions), as dense points; subsample tau =
    floor(m^(2/3)) = 158."""
    n, d = 2000, 500
    rng = np.random.Generator(np.random.PCG64(seed))
    X = csr_matrix(n, d, int(round(0.25 * n * d)), rng, np.float64)
    X.data = rng.random(X.nnz)
    P = np.ascontiguousarray(X.toarray())
    y = rng.standard_normal(n)
    return KernelProblem("accel_sparse_2000x500", P, y, 1.0 / n, 0.5)


def batched_tau(m):
    """Sketch size of a batched problem: a multiple of 64 near m^(2/3), clamped to [64, 512]
    and to m (the per-problem rule of the batched workload)."""
    t = 64.0 * np.floor(m ** (2.0 / 3.0) / 64.0 + 0.5)
    return int(min(min(512.0, max(64.0, t)), m))


def _batched_one(p, n, d, dense, nrhs, seed, density):
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, p])))
    if dense:
        X = rng.standard_normal((n, d), dtype=np.float32)
    else:
        X = csr_matrix(n, d, int(round(density * n * d)), rng, np.float32)
    W = rng.standard_normal((d, nrhs))
    if dense:
        Y = np.empty((n, nrhs))
        for r0 in range(0, n, 4096):  # FP64 products without an FP64 copy of X
            Y[r0:r0 + 4096] = X[r0:r0 + 4096].astype(np.float64) @ W
    else:
        Y = np.asarray(X @ W)
    Y += 0.01 * rng.standard_normal((n, nrhs))
    return X, Y


def batched(count=64, scale=1.0, seed=DATA_SEED_BASE + 3, nrhs=4, nlambda=16, density=0.005,
            workers=8, cap_factor=50):
    """Ragged batch: n ~ U{2000..40000}, d ~ U{500..8000} (times `scale`); the first half dense
    N(0,1) FP32, the second half CSR at 0.5% density with N(0,1) values; lambda grid
    10^(-4 + 5 i / (nlambda - 1)); nrhs right-hand sides Y = X W* + 0.01 N(0,1), W* ~ N(0,1);
    per-problem iteration cap cap_factor * m / tau (m = min(n, d), tau = batched_tau(m)).
    Returns a list of dicts (X, y, lambdas, max_iter, kind)."""
    import concurrent.futures
    rng = np.random.Generator(np.random.PCG64(seed))
    ns = rng.integers(2000, 40001, size=count)
    ds = rng.integers(500, 8001, size=count)
    lams = 10.0 ** (-4.0 + 5.0 * np.arange(nlambda) / max(1, nlambda - 1))
    shapes = [(p, max(8, int(ns[p] * scale)), max(8, int(ds[p] * scale)), p < count // 2)
              for p in range(count)]
    with concurrent.futures.ThreadPoolExecutor(max(1, workers)) as ex:
        data = list(ex.map(lambda s: _batched_one(s[0], s[1], s[2], s[3], nrhs, seed, density), shapes))
    out = []
    for (p, n, d, dense), (X, Y) in zip(shapes, data):
        m = min(n, d)
        tau = batched_tau(m)
        out.append(dict(X=X, y=Y, lambdas=lams, max_iter=max(1, int(cap_factor * m / tau)),
                        kind="dense" if dense else "csr", n=n, d=d, tau=tau))
    return out
