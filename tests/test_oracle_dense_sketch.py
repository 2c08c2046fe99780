"""Pins of the oracle's dense sketches (Def. 4.1 Gaussian, Def. 4.4 SRHT):

* SRHT: the closed-form entries equal I_C H D / sqrt(tau m') built from scipy's Hadamard
  matrix (Sylvester construction), truncated to the first m rows (zero padding of A);
  S^T S = I / tau when m is a power of 2; C is a uniform tau-subset of [0, m') (chi^2 over
  all subsets) and the signs are balanced;
* Gaussian: entries pass a Kolmogorov-Smirnov test against N(0, 1), have unit variance,
  and distinct columns / iterations are uncorrelated;
* the iteration with these sketches: a square Gaussian sketch (tau = m) solves the
  system in one step, S^T r^{k+1} = 0 after every step without momentum, and solves
  converge to the direct solution.
"""
import itertools

import numpy as np
import pytest
import scipy.linalg
import scipy.stats

from oracle import sketch as sk
from oracle.problem import kernel_system, ridge_system
from oracle.solver import Options, init_state, solve, step
from paper_2105_05565_amd import inputs


@pytest.mark.parametrize("m,tau", [(8, 3), (13, 5), (64, 64), (100, 30), (506, 126)])
def test_srht_matches_explicit_hadamard(m, tau):
    C, d, mp = sk.srht_parts(3, 1, 7, m, tau)
    assert mp >= m and mp < 2 * m and (mp & (mp - 1)) == 0
    H = scipy.linalg.hadamard(mp).astype(np.float64)
    dp = np.concatenate([d, np.ones(mp - m)])
    St = H[C, :] @ np.diag(dp) / np.sqrt(tau * mp)
    S = sk.srht_matrix(3, 1, 7, m, tau)
    assert np.array_equal(S, St.T[:m])


def test_srht_orthogonal_columns_at_power_of_two():
    S = sk.srht_matrix(5, 0, 2, 128, 40)
    assert np.allclose(S.T @ S, np.eye(40) / 40, rtol=0, atol=1e-15)


def test_srht_subset_uniform_and_signs_balanced():
    counts = {}
    signs = []
    for k in range(6000):
        C, d, mp = sk.srht_parts(11, 0, k, 7, 2)   # m' = 8, 28 subsets
        counts[tuple(C)] = counts.get(tuple(C), 0) + 1
        signs.append(d)
    assert len(counts) == len(list(itertools.combinations(range(8), 2)))
    obs = np.array(list(counts.values()), dtype=float)
    assert scipy.stats.chisquare(obs).pvalue > 1e-3
    s = np.concatenate(signs)
    assert abs(s.mean()) < 0.03


def test_gaussian_entries_standard_normal_and_independent():
    S = np.concatenate([sk.gaussian_matrix(2, 0, k, 997, 37) for k in range(6)], axis=0)
    z = S.ravel()
    assert scipy.stats.kstest(z, "norm").pvalue > 1e-3
    assert abs(z.mean()) < 0.02 and abs(z.var() - 1.0) < 0.02
    corr = np.corrcoef(S.T)
    off = corr[~np.eye(37, dtype=bool)]
    assert np.abs(off).max() < 0.05
    a, b = sk.gaussian_matrix(2, 0, 0, 997, 37), sk.gaussian_matrix(2, 0, 1, 997, 37)
    assert abs(np.corrcoef(a.ravel(), b.ravel())[0, 1]) < 0.02


def test_square_gaussian_sketch_solves_in_one_step():
    p = inputs.make_dense(60, 20, 0.1, seed=4)
    system = ridge_system(p.X, p.y, p.lam, "primal")
    st = init_state(system)
    step(system, st, Options(sketch="gaussian", tau=20, momentum="none"))
    wstar = np.linalg.solve(system.dense_A(), system.b)
    assert np.allclose(st.w, wstar, rtol=1e-8, atol=1e-11)


@pytest.mark.parametrize("kind", ["gaussian", "srht"])
def test_projection_and_convergence(kind):
    # m = 60 of m' = 64: the truncated Hadamard columns stay independent (with heavy
    # truncation an SRHT draw can have dependent columns and a singular S^T A S)
    p = inputs.make_dense(150, 60, 0.5, seed=6)
    system = ridge_system(p.X, p.y, p.lam, "primal")
    st = init_state(system)
    opts = Options(sketch=kind, tau=9, momentum="none", seed=3)
    for _ in range(6):
        _, s, _ = step(system, st, opts)
        Sm = s.matrix().toarray()
        assert np.abs(Sm.T @ st.r).max() <= 1e-12 * np.abs(system.b).max()
    st = solve(system, Options(sketch=kind, tau=12, momentum="heuristic", seed=3, tol=1e-10, max_iter=50000))
    wstar = np.linalg.solve(system.dense_A(), system.b)
    assert np.linalg.norm(st.w - wstar) <= 1e-7 * np.linalg.norm(wstar)
    q = inputs.make_points(62, 5, 1e-1, 0.3, seed=6)
    ks = kernel_system(q.P, q.y, q.lam, q.sigma)
    st = solve(ks, Options(sketch=kind, tau=18, momentum="none", seed=4, tol=1e-9, max_iter=50000))
    assert st.history[-1] <= 1e-9
