"""Pins of the oracle's kernel ridge system (Sec. 2.2, eq:kernelridge, eq:Gausskernel):

* the Gaussian kernel on hand-computed distances, symmetry, unit diagonal, positive
  semidefiniteness, and the row-block form against the whole matrix;
* the kernel trick: with the linear kernel K = X X^T, the coefficients alpha solving
  K (K + lambda I) alpha = K y give X^T alpha = the primal ridge weights (X^T X + lambda I)^{-1} X^T y;
* A S from the sketched products equals columns C of K (K + lambda I) formed directly;
* a full sketch (tau = m) without momentum solves the system in one step, and the solution
  is (K + lambda I)^{-1} y when K is nonsingular;
* the projection property S^T r^{k+1} = 0 (gamma = 1, beta = 0) and convergence of a
  small clustered problem to the direct solution.
"""
import math

import numpy as np
import pytest

from oracle import sketch as sk
from oracle.problem import gram_system, kernel_system, rbf_kernel
from oracle.solver import Options, init_state, sketched_products, solve, step
from paper_2105_05565_amd import inputs


def test_gaussian_kernel_hand_values():
    P = np.array([[0.0, 0.0], [3.0, 4.0], [0.0, 1.0]])
    K = rbf_kernel(P, 1.0)
    want = np.array([[1.0, math.exp(-12.5), math.exp(-0.5)],
                     [math.exp(-12.5), 1.0, math.exp(-9.0)],
                     [math.exp(-0.5), math.exp(-9.0), 1.0]])
    assert np.allclose(K, want, rtol=1e-15, atol=0)
    K2 = rbf_kernel(P, 2.0)
    assert K2[0, 1] == pytest.approx(math.exp(-25.0 / 8.0), rel=1e-15)


def test_gaussian_kernel_structure():
    p = inputs.make_points(300, 5, 1e-3, 0.7, seed=3)
    K = rbf_kernel(p.P, p.sigma)
    assert np.array_equal(K, K.T)
    assert np.all(np.diag(K) == 1.0)
    assert np.all((K > 0) & (K <= 1.0))
    assert np.linalg.eigvalsh(K).min() > -1e-12
    rows = np.array([7, 0, 299, 150])
    assert np.array_equal(rbf_kernel(p.P, p.sigma, rows=rows), K[rows])


def test_kernel_trick_linear_kernel_gives_primal_ridge():
    rng = np.random.default_rng(4)
    X = rng.standard_normal((20, 30))
    y = rng.standard_normal(20)
    lam = 0.3
    sysm = gram_system(X @ X.T, y, lam)
    st = solve(sysm, Options(sketch="subsample", tau=7, momentum="heuristic", tol=1e-12, max_iter=200000))
    w_primal = np.linalg.solve(X.T @ X + lam * np.eye(30), X.T @ y)
    assert np.allclose(X.T @ st.w, w_primal, rtol=1e-8, atol=1e-10)


def test_sketched_products_equal_direct_columns():
    p = inputs.make_points(90, 4, 0.05, 0.8, seed=5)
    sysm = kernel_system(p.P, p.y, p.lam, p.sigma)
    s = sk.draw_subsample(3, 0, 4, sysm.m, 17)
    _, AS, G, _ = sketched_products(sysm, s)
    K = rbf_kernel(p.P, p.sigma)
    A = K @ (K + p.lam * np.eye(90))
    assert np.allclose(AS, A[:, s.rows], rtol=1e-12, atol=1e-13)
    assert np.allclose(G, A[np.ix_(s.rows, s.rows)], rtol=1e-12, atol=1e-13)


def test_full_sketch_one_step_is_the_direct_solution():
    p = inputs.make_points(60, 3, 0.1, 0.6, seed=6)
    sysm = kernel_system(p.P, p.y, p.lam, p.sigma)
    st = init_state(sysm)
    step(sysm, st, Options(sketch="subsample", tau=60, momentum="none"))
    K = rbf_kernel(p.P, p.sigma)
    alpha = np.linalg.solve(K + p.lam * np.eye(60), p.y)
    assert np.allclose(st.w, alpha, rtol=1e-8, atol=1e-10)


def test_projection_property_and_convergence():
    p = inputs.make_points(150, 6, 1e-3, 0.5, seed=8)
    sysm = kernel_system(p.P, p.y, p.lam, p.sigma)
    st = init_state(sysm)
    opts = Options(sketch="subsample", tau=40, momentum="none", seed=2)
    for _ in range(5):
        _, s, _ = step(sysm, st, opts)
        assert np.abs(st.r[s.rows]).max() <= 1e-10 * np.abs(sysm.b).max()
    st = solve(sysm, Options(sketch="subsample", tau=40, momentum="heuristic", tol=1e-10, seed=2,
                             max_iter=100000))
    K = rbf_kernel(p.P, p.sigma)
    alpha = np.linalg.solve(K + p.lam * np.eye(150), p.y)
    A = K @ (K + p.lam * np.eye(150))
    kappa = np.linalg.cond(A)
    assert np.linalg.norm(st.w - alpha) <= 2 * kappa * 1e-10 * np.linalg.norm(alpha)
    assert np.linalg.norm(A @ st.w - sysm.b) <= 1.01e-10 * np.linalg.norm(sysm.b)
