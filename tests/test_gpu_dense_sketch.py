"""GPU: dense sketches (Gaussian, Def. 4.1; SRHT, Def. 4.4) and the count / SubCount sketches on
dense data, which all take the dense-S products T = Z^T S, A S = Z T + lambda S (kernel ridge:
+ lambda K S), G = S^T A S on FP64 MFMA.

* the sketch: S recovered from the GPU's A S (S = A^{-1} A S on small systems) equals the
  oracle's draw (SRHT and count to rounding of the solve, Gaussian also within the last
  bits of the transcendental functions);
* A S against the oracle's sketched product;
* FP64 trajectories to 1e-10 over 50 iterations, entry by entry (x, x_prev, r, r_prev): primal,
  dual, kernel ridge, ragged tiles;
* a converged solve reaches the direct solution.
SRHT problems use m close below a power of 2 (m' / m < 1.1), where the truncated Hadamard
columns stay independent. The SRHT's T = Z^T S and G = S^T AS come from its fast Walsh-Hadamard
transform (m' <= 16384), the other sketches' from FP64 MFMA products with the explicit S.
"""
import numpy as np
import pytest

from oracle import sketch as osk
from oracle.problem import kernel_system, ridge_system
from oracle.solver import Options, init_state, sketched_products, step
from paper_2105_05565_amd import inputs, rs
from parity_util import assert_state_close, assert_vec_close

pytestmark = pytest.mark.gpu

TRAJ_TOL = 1e-10


def _rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


@pytest.mark.parametrize("kind", ["gaussian", "srht", "count", "subcount"])
def test_dense_sketch_products_and_draw(kind):
    p = inputs.make_dense(300, 120, 0.5, seed=51)
    system = ridge_system(p.X, p.y, p.lam, "primal")
    tau = 24
    S = rs.Solver(p.X, p.y, p.lam, tau=tau, sketch=kind, form="primal", tol=0.0, seed=9, momentum="none",
                  subcount_k=3 if kind == "subcount" else 0)
    S.step(1)
    AS, Ginv = S.products()
    sk = osk.draw(kind, 9, 0, 0, 120, tau, sum_size=3 if kind == "subcount" else 0)
    _, AS_o, G_o, _ = sketched_products(system, sk)
    assert_vec_close(AS.ravel(), AS_o.ravel(), 1e-12, f"{kind} AS")
    S_gpu = np.linalg.solve(system.dense_A(), AS)
    assert np.abs(S_gpu - sk.matrix().toarray()).max() <= 1e-9 * np.abs(sk.signs).max()
    active = np.abs(sk.matrix().toarray()).sum(axis=0) > 0
    Gi = Ginv[np.ix_(active, active)]
    assert _rel(Gi @ G_o[np.ix_(active, active)], np.eye(active.sum())) <= 1e-9
    S.close()


CASES = {
    "primal": dict(n=300, d=120, tau=24, form="primal", seed=52),
    "dual": dict(n=124, d=260, tau=31, form="dual", seed=53),
    "ragged": dict(n=701, d=250, tau=130, form="primal", seed=54),  # partial 128 x 128 tiles
}


@pytest.mark.parametrize("case", sorted(CASES))
@pytest.mark.parametrize("kind", ["gaussian", "srht", "count"])
def test_dense_sketch_trajectory(case, kind):
    c = CASES[case]
    p = inputs.make_dense(c["n"], c["d"], 0.05, seed=c["seed"])
    system = ridge_system(p.X, p.y, p.lam, c["form"])
    opts = Options(sketch=kind, tau=c["tau"], momentum="heuristic", seed=5, tol=0.0)
    st = init_state(system)
    S = rs.Solver(p.X, p.y, p.lam, tau=c["tau"], sketch=kind, form=c["form"], tol=0.0, seed=5, lookahead=7)
    done = 0
    for ck in (1, 2, 9, 30, 50):
        while st.k < ck:
            step(system, st, opts)
        S.step(ck - done)
        done = ck
        assert_state_close(S.state(), [("x", st.w), ("x_prev", st.w_prev), ("r", st.r), ("r_prev", st.r_prev)],
                           TRAJ_TOL, f"{kind}/{case} k={ck}")
    np.testing.assert_allclose(S.history(), st.history[:done + 1], rtol=1e-9, atol=0)
    S.close()


@pytest.mark.parametrize("kind", ["gaussian", "srht", "count", "subcount"])
def test_kernel_dense_sketch_trajectory(kind):
    p = inputs.make_points(250, 6, 1e-3, 0.5, seed=55)
    system = kernel_system(p.P, p.y, p.lam, p.sigma)
    opts = Options(sketch=kind, tau=40, momentum="heuristic", seed=6, tol=0.0, sum_size=0)
    st = init_state(system)
    S = rs.Solver(p.P, p.y, p.lam, tau=40, sketch=kind, tol=0.0, seed=6, kernel_sigma=p.sigma)
    for _ in range(50):
        step(system, st, opts)
    S.step(50)
    assert_state_close(S.state(), [("x", st.w), ("x_prev", st.w_prev), ("r", st.r), ("r_prev", st.r_prev)],
                       TRAJ_TOL, f"kernel {kind} k=50")
    S.close()


def test_srht_fast_transform_largest_padding():
    """The SRHT's fast transform at its largest LDS-resident padding: 9000 kernel-ridge points
    (m' = 16384, one column of Z per workgroup, 144 KB of LDS). T = Z^T S and G = S^T AS come from
    the Walsh-Hadamard butterflies; AS and G^{-1} against the oracle's products of the explicit
    SRHT matrix, entry by entry."""
    p = inputs.make_points(9000, 8, 1e-3, 0.5, seed=57)
    system = kernel_system(p.P, p.y, p.lam, p.sigma)
    tau = 60
    S = rs.Solver(p.P, p.y, p.lam, tau=tau, sketch="srht", tol=0.0, seed=4, momentum="none",
                  kernel_sigma=p.sigma)
    S.step(1)
    AS, Ginv = S.products()
    S.close()
    sk = osk.draw("srht", 4, 0, 0, 9000, tau)
    _, AS_o, G_o, _ = sketched_products(system, sk)
    assert_vec_close(AS.ravel(), AS_o.ravel(), 1e-11, "SRHT m'=16384 AS")
    err = np.abs(Ginv[:tau, :tau] @ G_o - np.eye(tau)).max()
    assert err <= 4 * tau * 2.0 ** -53 * np.linalg.cond(G_o), err


@pytest.mark.parametrize("kind", ["gaussian", "srht"])
def test_dense_sketch_solve_reaches_direct_solution(kind):
    p = inputs.make_dense(500, 120, 0.1, seed=56)
    system = ridge_system(p.X, p.y, p.lam, "primal")
    S = rs.Solver(p.X, p.y, p.lam, tau=20, sketch=kind, form="primal", tol=1e-10, seed=3, max_iter=50000)
    w, st, rep = S.solve()
    assert st == rs.RS_OK
    wstar = np.linalg.solve(system.dense_A(), system.b)
    assert _rel(w, wstar) <= 1e-7
    S.close()


@pytest.mark.parametrize("call", ["step", "solve"])
def test_singular_sketched_system_reports_status(call):
    """A sketched system that is singular reaches the non-positive-pivot path. An SRHT draw over
    m = 300 coordinates (padded to m' = 512, Def. 4.4) with tau = 250 keeps about 60 column pairs
    (j, j + 256) whose truncated Hadamard columns agree on the first 256 rows and can only be told
    apart on the 44 rows beyond: S has rank 223 < tau, so S^T A S is singular although A is
    positive definite. The oracle's Cholesky meets a non-positive pivot on this draw; the library
    returns RS_ESINGULAR through the C ABI (rs_step and rs_solve), its kernels end normally,
    rs_last_error names the pivot, and the handle can still be reset and destroyed."""
    from oracle.linalg import NotPositiveDefinite, cholesky_lower
    m, tau, seed = 300, 250, 1
    p = inputs.make_dense(400, m, 0.05, seed=7)
    system = ridge_system(p.X, p.y, p.lam, "primal")
    sk = osk.draw("srht", seed, 0, 0, m, tau)
    assert np.linalg.matrix_rank(sk.matrix().toarray()) < tau
    _, _, G_o, _ = sketched_products(system, sk)
    with pytest.raises(NotPositiveDefinite):
        cholesky_lower(G_o)
    S = rs.Solver(p.X, p.y, p.lam, tau=tau, sketch="srht", form="primal", tol=1e-6, seed=seed,
                  momentum="none", max_iter=50)
    lib = rs.load()
    if call == "step":
        rel = rs.ctypes.c_double(0.0)
        st = lib.rs_step(S.h, 1, rs.ctypes.byref(rel))
    else:
        rep = rs.rs_report()
        st = lib.rs_solve(S.h, None, rs.ctypes.byref(rep))
    assert st == rs.RS_ESINGULAR, (st, rs.status_string(st))
    assert "pivot" in rs.last_error(S.h)
    assert rs.status_string(st) == "sketched system not positive definite"
    S.reset(seed + 1)
    S.close()
