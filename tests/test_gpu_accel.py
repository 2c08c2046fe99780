"""GPU: accelerated sketch-and-project (Alg. 3) against the oracle's accelerated method.

* mu = nu = 1 reproduces the GPU's plain method (no momentum) bit for bit;
* FP64 trajectories of w, v, r_w, r_v to 1e-10 entry by entry over 50 iterations for the subsample
  sketch (primal, dual, kernel ridge) and the count and SubCount sketches (both CSR
  routes), with lookahead batches of 3 so that batch boundaries (where the next sketch is
  applied to r_z) are crossed;
* a solve with conservative parameters stops on ||r_v|| and reaches the direct solution.
"""
import numpy as np
import pytest

from oracle.accel import accel_init, accel_step
from oracle.problem import kernel_system, ridge_system
from oracle.solver import Options
from paper_2105_05565_amd import inputs, rs
from parity_util import assert_state_close, assert_vec_close

pytestmark = pytest.mark.gpu

TRAJ_TOL = 1e-10


def _rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


@pytest.mark.parametrize("kind", ["subsample", "count"])
def test_mu_nu_one_equals_plain_method(kind):
    p = inputs.make_csr(400, 150, 0.04, 0.05, seed=3) if kind == "count" else inputs.make_dense(300, 130, 0.05, seed=1)
    tau = 23 if kind == "count" else 37
    A = rs.Solver(p.X, p.y, p.lam, tau=tau, sketch=kind, form="primal", tol=0.0, seed=5, accel=(1.0, 1.0))
    P = rs.Solver(p.X, p.y, p.lam, tau=tau, sketch=kind, form="primal", tol=0.0, seed=5, momentum="none")
    for c in (1, 4, 30):
        A.step(c)
        P.step(c)
        xa, va, ra, rva = A.state()
        xp, _, rp, _ = P.state()
        assert np.array_equal(xa, xp) and np.array_equal(va, xp)
        assert np.array_equal(ra, rp) and np.array_equal(rva, rp)
    A.close()
    P.close()


CASES = {
    "dense-primal": dict(kind="subsample", tau=37, form="primal", route="auto"),
    "dense-dual": dict(kind="subsample", tau=45, form="dual", route="auto"),
    "csr-count-arows": dict(kind="count", tau=23, form="primal", route="arows"),
    "csr-count-scatter": dict(kind="count", tau=23, form="primal", route="scatter"),
    "csr-subcount": dict(kind="subcount", tau=20, form="primal", route="arows"),
    "kernel": dict(kind="subsample", tau=60, form=None, route="auto"),
}


@pytest.mark.parametrize("case", sorted(CASES))
@pytest.mark.parametrize("mu,nu", [(0.01, 10.0), (0.2, 3.0)])
def test_accelerated_trajectory(case, mu, nu):
    c = CASES[case]
    kw = dict(tau=c["tau"], sketch=c["kind"], tol=0.0, seed=7, accel=(mu, nu), lookahead=3,
              sparse_route=c["route"])
    if case == "kernel":
        p = inputs.make_points(240, 6, 1e-3, 0.5, seed=41)
        system = kernel_system(p.P, p.y, p.lam, p.sigma)
        S = rs.Solver(p.P, p.y, p.lam, kernel_sigma=p.sigma, **kw)
    else:
        if c["kind"] == "subsample":
            p = inputs.make_dense(300, 130, 0.05, seed=1) if c["form"] == "primal" \
                else inputs.make_dense(110, 260, 0.05, seed=2)
        else:
            p = inputs.make_csr(400, 150, 0.04, 0.05, seed=3)
        system = ridge_system(p.X, p.y, p.lam, c["form"])
        S = rs.Solver(p.X, p.y, p.lam, form=c["form"], **kw)
    opts = Options(sketch=c["kind"], tau=c["tau"], seed=7, tol=0.0,
                   sum_size=0)
    st = accel_init(system)
    done = 0
    for ck in (1, 2, 3, 7, 20, 50):
        while st.k < ck:
            accel_step(system, st, opts, mu, nu)
        S.step(ck - done)
        done = ck
        assert_state_close(S.state(), [("w", st.w), ("v", st.v), ("r_w", st.r_w), ("r_v", st.r_v)], TRAJ_TOL,
                           f"accel {case} mu={mu} nu={nu} k={ck}")
    np.testing.assert_allclose(S.history(), st.history[:done + 1], rtol=1e-9, atol=0)
    S.close()


def test_accelerated_solve_reaches_direct_solution():
    p = inputs.make_dense(400, 100, 0.1, seed=8)
    system = ridge_system(p.X, p.y, p.lam, "primal")
    S = rs.Solver(p.X, p.y, p.lam, tau=20, form="primal", tol=1e-10, seed=3, max_iter=200000,
                  accel=(1e-3, 50.0))
    w, st, rep = S.solve()
    assert st == rs.RS_OK and rep.rel_res <= 1e-10
    wstar = np.linalg.solve(system.dense_A(), system.b)
    assert _rel(w, wstar) <= 1e-6
    hist = S.history()
    assert hist[-1] <= 1e-10 < hist[-2]
    S.close()
