"""The ridge linear system A w = b (Sec. 2.1).

Ridge regression min_w 1/2 ||X w - y||^2 + lambda/2 ||w||^2 (eq:ridge) is solved
through its stationarity system. Both forms are written A = Z Z^T + lambda I:

* primal (eq:linear):     A = X^T X + lambda I,  b = X^T y,  Z = X^T,  m = d;
* dual   (eq:duallinear): A = X X^T + lambda I,  b = y,      Z = X,    m = n,
  and the weights are recovered as w = X^T alpha.

The form rule of Sec. 2.1 picks the primal when d <= n and the dual otherwise
(eq:Axb: m is the smaller dimension of X).

Kernel ridge regression (Sec. 2.2, eq:kernelridge) is the system A = K (K + lambda I),
b = K y for a symmetric kernel matrix K (the Gaussian kernel of eq:Gausskernel here),
whose solution is the dual coefficient vector alpha (m = n).

Part of the oracle: test infrastructure only.
"""
from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp


@dataclass
class RidgeSystem:
    X: object          # n x d, numpy array or scipy sparse matrix, FP64
    Z: object          # m x K with A = Z Z^T + lambda I
    b: np.ndarray      # right-hand side, FP64 [m]
    lam: float
    form: str          # "primal" | "dual"

    @property
    def m(self):
        return self.Z.shape[0]

    def matvec(self, v):
        """A v = Z (Z^T v) + lambda v."""
        return np.asarray(self.Z @ (self.Z.T @ v)).ravel() + self.lam * v

    def dense_A(self):
        Zd = self.Z.toarray() if sp.issparse(self.Z) else self.Z
        return Zd @ Zd.T + self.lam * np.eye(self.m)

    def weights(self, x):
        """Ridge weights from the solution x of A x = b (Lemma A.1: w = X^T alpha)."""
        if self.form == "primal":
            return np.asarray(x, dtype=np.float64).copy()
        return np.asarray(self.X.T @ x).ravel()


def choose_form(n, d):
    """Primal when d <= n, dual when n < d (Sec. 2.1)."""
    return "primal" if d <= n else "dual"


def ridge_system(X, y, lam, form="auto"):
    if sp.issparse(X):
        X = sp.csr_matrix(X, dtype=np.float64)
    else:
        X = np.asarray(X, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64).ravel()
    n, d = X.shape
    if y.shape[0] != n:
        raise ValueError("y must have n entries")
    if not lam > 0:
        raise ValueError("lambda must be positive")
    if form == "auto":
        form = choose_form(n, d)
    if form == "primal":
        Z = X.T.tocsr() if sp.issparse(X) else np.ascontiguousarray(X.T)
        b = np.asarray(X.T @ y).ravel()
    elif form == "dual":
        Z = X
        b = y.copy()
    else:
        raise ValueError(f"unknown form {form!r}")
    return RidgeSystem(X=X, Z=Z, b=b, lam=float(lam), form=form)


# ---------------------------------------------------------------- kernel ridge (Sec. 2.2)
def rbf_kernel(P, sigma, rows=None):
    """Gaussian kernel matrix (eq:Gausskernel): K_ij = exp(-||p_i - p_j||^2 / (2 sigma^2)),
    the squared distance summed from the coordinate differences. rows: only those rows
    (K[rows, :]); computed in blocks of rows to bound memory."""
    P = np.asarray(P, dtype=np.float64)
    idx = np.arange(P.shape[0]) if rows is None else np.asarray(rows)
    out = np.empty((idx.size, P.shape[0]))
    for s in range(0, idx.size, 256):
        blk = P[idx[s:s + 256]]
        diff = blk[:, None, :] - P[None, :, :]
        out[s:s + 256] = np.exp(-np.sum(diff * diff, axis=2) / (2.0 * sigma * sigma))
    return out


@dataclass
class KernelSystem:
    """Kernel ridge regression (eq:kernelridge): A = K^T (K + lambda I) and b = K^T y with
    K symmetric positive semidefinite, m = n. The solution is the dual coefficient vector
    alpha; predictions at the training points are K alpha."""
    Kmat: np.ndarray   # m x m
    b: np.ndarray
    lam: float
    y: np.ndarray
    form: str = "kernel"

    @property
    def m(self):
        return self.Kmat.shape[0]

    def matvec(self, v):
        """A v = K (K v) + lambda K v."""
        Kv = self.Kmat @ v
        return self.Kmat @ Kv + self.lam * Kv

    def sketched_AS(self, S):
        """A S = K (K S) + lambda K S (m x tau, dense)."""
        KS = np.asarray(self.Kmat @ S)
        return self.Kmat @ KS + self.lam * KS

    def dense_A(self):
        return self.Kmat.T @ (self.Kmat + self.lam * np.eye(self.m))

    def weights(self, x):
        return np.asarray(x, dtype=np.float64).copy()


def gram_system(Kmat, y, lam):
    """A kernel ridge system for a given symmetric kernel matrix (eq:kernelridge)."""
    Kmat = np.asarray(Kmat, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64).ravel()
    if Kmat.ndim != 2 or Kmat.shape[0] != Kmat.shape[1] or y.shape[0] != Kmat.shape[0]:
        raise ValueError("K must be m x m and y must have m entries")
    if not lam > 0:
        raise ValueError("lambda must be positive")
    return KernelSystem(Kmat=Kmat, b=Kmat.T @ y, lam=float(lam), y=y)


def kernel_system(P, y, lam, sigma):
    """Kernel ridge system for points P (n x d) with the Gaussian kernel of width sigma."""
    if not sigma > 0:
        raise ValueError("sigma must be positive")
    return gram_system(rbf_kernel(P, sigma), y, lam)
