"""The ridge linear system A w = b (Sec. 2.1).

Ridge regression min_w 1/2 ||X w - y||^2 + lambda/2 ||w||^2 (eq:ridge) is solved
through its stationarity system. Both forms are written A = Z Z^T + lambda I:

* primal (eq:linear):     A = X^T X + lambda I,  b = X^T y,  Z = X^T,  m = d;
* dual   (eq:duallinear): A = X X^T + lambda I,  b = y,      Z = X,    m = n,
  and the weights are recovered as w = X^T alpha.

The form rule of Sec. 2.1 picks the primal when d <= n and the dual otherwise
(eq:Axb: m is the smaller dimension of X).

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
