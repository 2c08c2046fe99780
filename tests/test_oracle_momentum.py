"""Pins of the oracle's theoretical momentum rule (Sec. 6, Thm 6.2, Cor 6.3,
eq:parameterswitchtheory), written from the paper's formulas independently of
oracle/solver.py:

* the switch index is the first k at which the constant-eta momentum of Cor 6.3 reaches
  the threshold (brute-force scan);
* gamma_k, beta_k satisfy eq:etalambdatogammbetagen with zeta_k of eq:zeta_kaptheo summed
  term by term here, across the switch, and the identity eq:soj9so9sj4ap;
* before the switch they equal the closed forms of eq:cst_eta_lambda_to_gamma_beta_formula;
* heavy ball with these parameters equals the iterate-averaging form (Prop 6.1) for the
  non-constant eta_k sequence;
* Thm 6.2 / Cor 6.3: the mean last-iterate squared residual over seeded runs stays below
  ||w^0 - w*||_A^2 / (lambda_min(E[H]) sum_{t<=k} eta_t (1 - eta_t)), with E[H] from every
  tau-subset of a tiny problem.
"""
import itertools

import numpy as np
import pytest

from oracle import sketch as sk
from oracle.problem import ridge_system
from oracle.solver import SWITCH_NEVER, Options, init_state, schedule, step, theory_switch
from paper_2105_05565_amd import inputs


def _beta_cst(eta, k):
    return 1.0 - (2.0 - eta) / ((k + 1) * (1.0 - eta) + 1.0)


@pytest.mark.parametrize("eta,thr", [(0.995, 0.5), (0.99, 0.5), (0.9, 0.3), (0.995, 0.7), (0.5, 0.99)])
def test_switch_is_first_crossing(eta, thr):
    k = 0
    while _beta_cst(eta, k) < thr:
        k += 1
    assert theory_switch(eta, thr) == k
    assert theory_switch(1.0, 0.5) == SWITCH_NEVER and theory_switch(0.9, 1.0) == SWITCH_NEVER


def _eta_seq(eta, K, n):
    return [eta if t < K else 1.0 for t in range(n)]


def _zeta(etas, k):
    s = 0.0
    for t in range(k):
        s += etas[t] * (1.0 - etas[t])
    return s / etas[k]


@pytest.mark.parametrize("eta,thr", [(0.995, 0.5), (0.9, 0.3)])
def test_parameters_follow_zeta_form_across_switch(eta, thr):
    opts = Options(momentum="theory", eta=eta, beta_max=thr)
    K = theory_switch(eta, thr)
    n = K + 60
    etas = _eta_seq(eta, K, n + 2)
    for k in range(n):
        g, b = schedule(opts, k)
        zk, zk1 = _zeta(etas, k), _zeta(etas, k + 1)
        assert g == pytest.approx(etas[k] / (zk1 + 1.0), rel=1e-12)
        assert b == pytest.approx(zk / (zk1 + 1.0), rel=1e-12, abs=1e-15)
        # eq:soj9so9sj4ap
        assert etas[k] * (1.0 + zk - etas[k]) == pytest.approx(etas[k + 1] * zk1, rel=1e-12, abs=1e-15)
    # the paper: beta rises from 0 to about 0.5 while gamma falls from about 1 to 0.5
    if (eta, thr) == (0.995, 0.5):
        assert schedule(opts, 0)[1] == 0.0 and schedule(opts, 0)[0] > 0.99
        for k in (K, K + 10, 10 * K):
            g, b = schedule(opts, k)
            assert abs(g - 0.5) < 1e-4 and abs(b - 0.5) < 1e-4


def test_before_switch_equals_corollary_6_3():
    eta = 0.995
    opts = Options(momentum="theory", eta=eta)
    K = theory_switch(eta, 0.5)
    for k in range(K - 1):
        g, b = schedule(opts, k)
        d = (k + 1) * (1.0 - eta) + 1.0
        assert g == pytest.approx(eta / d, rel=1e-12)
        assert b == pytest.approx(1.0 - (2.0 - eta) / d, rel=1e-12, abs=1e-15)


def test_heavy_ball_equals_iterate_averaging_with_switch():
    """Prop 6.1 holds for any eta_k: the oracle's heavy ball with the theory schedule
    against eq:zupdateap / eq:iterateavap written here (W = A)."""
    p = inputs.make_dense(60, 24, 0.3, seed=11)
    sysm = ridge_system(p.X, p.y, p.lam, "primal")
    A = sysm.dense_A()
    eta, thr = 0.9, 0.3
    K = theory_switch(eta, thr)
    etas = _eta_seq(eta, K, 40)
    opts = Options(sketch="subsample", tau=6, momentum="theory", eta=eta, beta_max=thr)
    st = init_state(sysm)
    w = np.zeros(sysm.m)
    z = w.copy()  # z^{-1} = w^0
    for k in range(K + 12):
        s = sk.draw_subsample(1, 0, k, sysm.m, 6)
        S = s.matrix().toarray()
        grad = S @ np.linalg.solve(S.T @ A @ S, S.T @ (A @ w - sysm.b))  # eq:grad with W = A
        z = z - etas[k] * grad
        a = 1.0 / (_zeta(etas, k + 1) + 1.0)
        w = (1.0 - a) * w + a * z
        step(sysm, st, opts, sketch=s)
        assert np.allclose(st.w, w, rtol=1e-9, atol=1e-12), k


def test_last_iterate_bound_theorem_6_2():
    """Thm 6.2 (here in the constant-eta regime of Cor 6.3: eta = 0.5 with the switch far
    beyond the checked iterations): E ||A w^k - b||^2 <= ||w^0 - w*||_A^2 /
    (lambda_min(E[H]) sum_{t<=k} eta_t (1 - eta_t))."""
    m, tau = 6, 2
    p = inputs.make_dense(10, m, 0.5, seed=5)
    sysm = ridge_system(p.X, p.y, p.lam, "primal")
    A = sysm.dense_A()
    subsets = list(itertools.combinations(range(m), tau))
    EH = np.zeros((m, m))
    for C in subsets:
        I_C = np.eye(m)[:, C]
        EH += I_C @ np.linalg.inv(I_C.T @ A @ I_C) @ I_C.T / len(subsets)
    lam_min = np.linalg.eigvalsh(EH).min()
    wstar = np.linalg.solve(A, sysm.b)
    e0 = wstar @ A @ wstar  # w^0 = 0
    eta, thr = 0.5, 0.99
    assert theory_switch(eta, thr) > 100
    checks = {10: 0.0, 40: 0.0, 100: 0.0}
    runs = 300
    for seed in range(runs):
        st = init_state(sysm)
        opts = Options(sketch="subsample", tau=tau, momentum="theory", eta=eta, beta_max=thr, seed=2000 + seed)
        for k in range(1, 101):
            step(sysm, st, opts)
            if k in checks:
                res = A @ st.w - sysm.b
                checks[k] += res @ res / runs
    for k, mean in checks.items():
        bound = e0 / (lam_min * (k + 1) * eta * (1.0 - eta))
        assert mean <= bound, (k, mean, bound)
