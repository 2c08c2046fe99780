"""Least-norm solution of the sketched system (eq:sketched_system, Alg. 1 and 2).

The paper leaves the routine behind ``least_norm_solution`` unstated. The
sketched matrix S^T A S is symmetric positive semi-definite, and positive
definite on the columns of S that are nonzero (A = B + lambda I with
lambda > 0). Reading used here: a Cholesky factorisation G = L L^T of the lower
triangle of G restricted to the nonzero columns of S, followed by one forward
and one backward substitution. A zero column of S (an empty count bucket)
makes the matching row and column of G and entry of S^T r zero; the
pseudo-inverse solution sets that entry of delta to zero, which is what the
restriction does.

Part of the oracle: test infrastructure only.
"""
import numpy as np


class NotPositiveDefinite(ArithmeticError):
    pass


def cholesky_lower(G):
    """L with L L^T = G, reading only the lower triangle of G (column by column)."""
    G = np.asarray(G, dtype=np.float64)
    n = G.shape[0]
    L = np.zeros_like(G)
    for j in range(n):
        d = G[j, j] - np.dot(L[j, :j], L[j, :j])
        if not d > 0.0:
            raise NotPositiveDefinite(f"pivot {j} is {d!r}")
        L[j, j] = np.sqrt(d)
        if j + 1 < n:
            L[j + 1:, j] = (G[j + 1:, j] - L[j + 1:, :j] @ L[j, :j]) / L[j, j]
    return L


def forward_substitution(L, b):
    """x with L x = b, L lower triangular."""
    n = L.shape[0]
    x = np.zeros(n)
    for i in range(n):
        x[i] = (b[i] - np.dot(L[i, :i], x[:i])) / L[i, i]
    return x


def backward_substitution_transposed(L, b):
    """x with L^T x = b, L lower triangular."""
    n = L.shape[0]
    x = np.zeros(n)
    for i in range(n - 1, -1, -1):
        x[i] = (b[i] - np.dot(L[i + 1:, i], x[i + 1:])) / L[i, i]
    return x


def least_norm_solution(G, rho, active=None):
    """delta = G^dagger rho for the sketched system, via Cholesky on the active block."""
    G = np.asarray(G, dtype=np.float64)
    rho = np.asarray(rho, dtype=np.float64)
    tau = G.shape[0]
    if active is None:
        active = np.ones(tau, dtype=bool)
    sel = np.flatnonzero(active)
    delta = np.zeros(tau)
    if sel.size == 0:
        return delta
    Gs = G[np.ix_(sel, sel)]
    L = cholesky_lower(Gs)
    y = forward_substitution(L, rho[sel])
    delta[sel] = backward_substitution_transposed(L, y)
    return delta
