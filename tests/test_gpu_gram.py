"""GPU: the formed-A route for the subsample sketch (rs_options.dense_route = 1).

A = Z Z^T + lambda I (kernel ridge: K K + lambda K) is formed once by the product kernel
with every coordinate as one sketch, and each sketch's AS is gathered from its columns.
Checked as the product route is: FP64 products and 50-iteration trajectories against the
oracle entry by entry (1e-12, 1e-10), BF16 products within the dot-product bound (plain and
kernel ridge), kernel ridge against the product route, and the combinations it does not
serve are rejected.
"""
import numpy as np
import pytest

from oracle import sketch as osk
from oracle.problem import kernel_system, ridge_system
from oracle.solver import Options, init_state, sketched_products, step
from paper_2105_05565_amd import inputs, rs
from parity_util import assert_state_close, assert_vec_close

pytestmark = pytest.mark.gpu

U_BF16, U_FP32 = 2.0 ** -8, 2.0 ** -24


@pytest.mark.parametrize("form,n,d", [("primal", 700, 230), ("dual", 230, 700)])
def test_gram_route_fp64_products_and_trajectory(form, n, d):
    p = inputs.make_dense(n, d, 0.05, seed=91)
    system = ridge_system(p.X, p.y, p.lam, form)
    tau = 29
    S = rs.Solver(p.X, p.y, p.lam, tau=tau, sketch="subsample", form=form, tol=0.0, seed=6, lookahead=5,
                  dense_route="gram")
    opts = Options(sketch="subsample", tau=tau, momentum="heuristic", seed=6, tol=0.0)
    st = init_state(system)
    for c in (1, 7, 30, 50):
        while st.k < c:
            step(system, st, opts)
        S.step(c - S.k)
        assert_state_close(S.state(), [("x", st.w), ("x_prev", st.w_prev), ("r", st.r), ("r_prev", st.r_prev)],
                           1e-10, f"formed A {form} k={c}")
    AS, _ = S.products()
    s = osk.draw_subsample(6, 0, 49, system.m, tau)
    _, AS_or, _, _ = sketched_products(system, s)
    assert_vec_close(AS.ravel(), AS_or.ravel(), 1e-12, "formed A: AS")
    S.close()


def test_gram_route_mixed_products_within_bound():
    p = inputs.make_dense(900, 300, 0.1, seed=92, dtype=np.float32, col_log_sigma=1.0)
    system = ridge_system(p.X, p.y, p.lam, "primal")
    tau = 40
    S = rs.Solver(p.X, p.y, p.lam, tau=tau, sketch="subsample", tol=0.0, seed=5, precision="mixed",
                  lookahead=3, dense_route="gram")
    S.step(3)
    AS, Gi = S.products()
    s = osk.draw_subsample(5, 0, 2, system.m, tau)
    _, AS_or, _, _ = sketched_products(system, s)
    Z = np.asarray(system.Z, dtype=np.float64)
    C = s.rows
    bound = (2 * U_BF16 + Z.shape[1] * U_FP32) * (np.abs(Z) @ np.abs(Z[C]).T) + 1e-30
    assert np.all(np.abs(AS - AS_or) <= bound)
    Gm = np.tril(AS[C]) + np.tril(AS[C], -1).T
    assert np.allclose(Gi @ Gm, np.eye(tau), atol=1e-8)
    S.close()
    T = rs.Solver(p.X, p.y, p.lam, tau=tau, sketch="subsample", tol=1e-8, seed=5, precision="mixed",
                  dense_route="gram", max_iter=100000)
    _, st, rep = T.solve()
    assert st == rs.RS_OK and rep.rel_res_true <= 1e-8 * 1.001
    T.close()


def test_gram_route_kernel_ridge_matches_product_route():
    p = inputs.make_points(400, 8, 1e-2, 0.5, seed=93)
    kw = dict(tau=50, kernel_sigma=p.sigma, tol=0.0, seed=7, lookahead=4)
    A = rs.Solver(p.P, p.y, p.lam, dense_route="gram", **kw)
    B = rs.Solver(p.P, p.y, p.lam, **kw)
    A.step(25)
    B.step(25)
    assert_state_close(A.state(), list(zip(("x", "x_prev", "r", "r_prev"), B.state())), 1e-10,
                       "formed A vs products, kernel ridge")
    A.close()
    B.close()


def test_gram_route_kernel_ridge_mixed_products_within_bound():
    """Kernel ridge with BF16 products on the formed-A route: A = K K + lambda K formed once
    from the BF16 kernel matrix (FP32 accumulation), each sketch's AS gathered from it. Its
    entries against the oracle's FP64 K (K S) + lambda K S within the dot-product bound
    (2 u_bf16 + n u_fp32) (|K| |K_C|^T) plus the FP32 rounding of the stored entries, and
    against the product route's AS of the same sketch within twice that bound; a mixed solve
    stops on the FP64-refreshed residual."""
    p = inputs.make_points(700, 8, 1e-2, 0.5, seed=96)
    system = kernel_system(p.P, p.y, p.lam, p.sigma)
    tau = 64
    kw = dict(tau=tau, kernel_sigma=p.sigma, tol=0.0, seed=5, precision="mixed", lookahead=3)
    A = rs.Solver(p.P, p.y, p.lam, dense_route="gram", **kw)
    B = rs.Solver(p.P, p.y, p.lam, **kw)
    A.step(3)
    B.step(3)
    AS_a, Gi = A.products()
    AS_b, _ = B.products()
    A.close()
    B.close()
    sketch = osk.draw_subsample(5, 0, 2, 700, tau)
    _, AS_o, _, _ = sketched_products(system, sketch)
    K = system.Kmat
    C = sketch.rows
    bound = (2 * U_BF16 + 700 * U_FP32) * (np.abs(K) @ np.abs(K[C]).T) + 2 * U_FP32 * np.abs(AS_o) + 1e-30
    err = np.abs(AS_a - AS_o)
    assert np.all(err <= bound), float((err / bound).max())
    assert np.all(np.abs(AS_a - AS_b) <= 2 * bound)
    Gm = np.tril(AS_a[C]) + np.tril(AS_a[C], -1).T
    kappa = np.linalg.cond(Gm)
    assert np.abs(Gi @ Gm - np.eye(tau)).max() <= 4 * tau * 2.0 ** -53 * kappa
    T = rs.Solver(p.P, p.y, p.lam, tau=tau, kernel_sigma=p.sigma, tol=1e-8, seed=5, precision="mixed",
                  dense_route="gram", max_iter=100000)
    _, st, rep = T.solve()
    assert st == rs.RS_OK and rep.rel_res_true <= 1e-8 * 1.001
    T.close()


def test_gram_route_rejections():
    p = inputs.make_csr(300, 120, 0.05, 0.05, seed=94)
    with pytest.raises(rs.RsError) as e:
        rs.Solver(p.X, p.y, p.lam, tau=20, sketch="count", dense_route="gram")
    assert e.value.status == rs.RS_EUNSUPPORTED
    q = inputs.make_dense(300, 120, 0.05, seed=95)
    with pytest.raises(rs.RsError) as e:
        rs.Solver(q.X, q.y, q.lam, tau=20, sketch="gaussian", dense_route="gram")
    assert e.value.status == rs.RS_EUNSUPPORTED
