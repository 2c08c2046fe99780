"""GPU parity: the HIP library (through the C ABI) against the CPU FP64 oracle.

* sketches: bit-exact (coordinates, buckets, signs) for every kind;
* trajectories: x^k, x^{k-1}, r^k, r^{k-1} entry by entry within 1e-10 relative (plus 1e-10
  times the vector's largest entry) for k <= 50, FP64;
* converged weights against a direct solve; primal/dual agreement.
Shapes are chosen to span several tiles with ragged tails (m, tau not multiples of
the 64 x 64 product tiles or of the 32 x 32 factorisation tiles).
"""
import os

import numpy as np
import pytest
import scipy.sparse as sp

from oracle import sketch as osk
from oracle.problem import ridge_system
from oracle.solver import Options, init_state, step
from paper_2105_05565_amd import inputs, rs
from parity_util import assert_state_close, assert_vec_close

pytestmark = pytest.mark.gpu

TRAJ_TOL = 1e-10


def _oracle_sketch_triplets(kind, seed, pid, k, m, tau, sub_k):
    s = osk.draw(kind, seed, pid, k, m, tau, sum_size=sub_k)
    order = np.lexsort((s.rows, s.cols))
    return s.rows[order], s.cols[order], s.signs[order]


def _sorted(rows, cols, signs):
    order = np.lexsort((rows, cols))
    return rows[order], cols[order], signs[order]


def _dense(n, d, lam, seed):
    return inputs.make_dense(n, d, lam, seed=seed)


def _csr(n, d, density, lam, seed, dtype=np.float64):
    return inputs.make_csr(n, d, density, lam, seed=seed, dtype=dtype)


@pytest.mark.parametrize("n,d,tau", [(300, 130, 37), (200, 64, 64), (500, 97, 1), (120, 90, 90)])
def test_subsample_sketch_bit_exact(n, d, tau):
    p = _dense(n, d, 0.1, seed=n + d)
    S = rs.Solver(p.X, p.y, p.lam, tau=tau, sketch="subsample", form="primal", momentum="none",
                  tol=0.0, seed=7, problem_id=3)
    for k in range(6):
        S.step(1)
        got = S.last_sketch()
        exp = _oracle_sketch_triplets("subsample", 7, 3, k, d, tau, 0)
        for g, e in zip(got, exp):
            assert np.array_equal(g, e), (k, g[:10], e[:10])
    S.close()


@pytest.mark.parametrize("kind,sub_k", [("count", 0), ("subcount", 3), ("subcount", 0)])
@pytest.mark.parametrize("n,d,tau", [(400, 150, 20), (300, 211, 33)])
def test_sparse_sketches_bit_exact(kind, sub_k, n, d, tau):
    p = _csr(n, d, 0.05, 0.1, seed=d)
    S = rs.Solver(p.X, p.y, p.lam, tau=tau, sketch=kind, form="primal", momentum="none", tol=0.0,
                  seed=11, problem_id=1, subcount_k=sub_k)
    kk = sub_k if sub_k > 0 else osk.subcount_k(d, tau)
    for k in range(5):
        S.step(1)
        got = _sorted(*S.last_sketch())
        exp = _oracle_sketch_triplets(kind, 11, 1, k, d, tau, kk)
        for g, e in zip(got, exp):
            assert np.array_equal(g, e), (kind, k)
    S.close()


def test_count_sketch_bit_exact_large_m():
    """m = 20000 coordinates (the sparse workload's primal size), several iterations."""
    p = _csr(2000, 20000, 0.002, 1e-3, seed=5, dtype=np.float32)
    S = rs.Solver(p.X, p.y, p.lam, tau=500, sketch="count", form="primal", momentum="none",
                  tol=0.0, seed=3, lookahead=4)
    S.step(4)
    got = _sorted(*S.last_sketch())
    exp = _oracle_sketch_triplets("count", 3, 0, 3, 20000, 500, 0)
    for g, e in zip(got, exp):
        assert np.array_equal(g, e)
    S.close()


def _oracle_trajectory(system, opts, checkpoints):
    """The oracle's (x, x_prev, r, r_prev) at each checkpoint, and its residual history."""
    st = init_state(system)
    out = {}
    for c in checkpoints:
        while st.k < c:
            step(system, st, opts)
        out[c] = (st.w.copy(), st.w_prev.copy(), st.r.copy(), st.r_prev.copy())
    return out, list(st.history)


def _trajectory_check(X, y, lam, *, form, kind, tau, momentum, sub_k=0, iters=50, checkpoints=None,
                      lookahead=0, seed=5, route="auto", oracle=None):
    """Advance the GPU solve and the oracle to each checkpoint and compare x^k, x^{k-1}, r^k and
    r^{k-1} entry by entry (relative TRAJ_TOL, absolute TRAJ_TOL times the vector's largest
    entry), then the residual history. oracle: a precomputed _oracle_trajectory result for the
    same problem, options and checkpoints (shared by several routes)."""
    checkpoints = checkpoints or [1, 2, 3, 7, 20, iters]
    if oracle is None:
        system = ridge_system(X, y, lam, form)
        opts = Options(sketch=kind, tau=tau, sum_size=sub_k if sub_k else 0, momentum=momentum, seed=seed,
                       tol=0.0)
        oracle = _oracle_trajectory(system, opts, checkpoints)
    ref, ref_hist = oracle
    S = rs.Solver(X, y, lam, tau=tau, sketch=kind, form=form, momentum=momentum, tol=0.0, seed=seed,
                  subcount_k=sub_k, lookahead=lookahead, sparse_route=route)
    done = 0
    worst = 0.0
    for c in checkpoints:
        S.step(c - done)
        done = c
        assert S.k == c
        w, wp, r, rp = ref[c]
        worst = max(worst, assert_state_close(
            S.state(), [("x", w), ("x_prev", wp), ("r", r), ("r_prev", rp)], TRAJ_TOL,
            f"{kind}/{form}/{route} k={c}"))
    hist = S.history()
    np.testing.assert_allclose(hist, ref_hist[:len(hist)], rtol=1e-9, atol=0)
    S.close()
    return worst


@pytest.mark.parametrize("momentum", ["none", "heuristic", "constant"])
@pytest.mark.parametrize("form", ["primal", "dual"])
def test_dense_subsample_trajectory(momentum, form):
    if form == "primal":
        p = _dense(300, 130, 0.05, seed=1)
        tau = 37
    else:
        p = _dense(110, 260, 0.05, seed=2)
        tau = 45
    _trajectory_check(p.X, p.y, p.lam, form=form, kind="subsample", tau=tau, momentum=momentum)


@pytest.mark.parametrize("n,d,tau", [(301, 130, 37), (701, 300, 150)])
def test_dense_subsample_trajectory_ragged_tiles(n, d, tau):
    # K = n odd: rows of Z are not 16-byte aligned (element-wise panel loads); m = 300 and
    # tau = 150 leave partial 128 x 128 product tiles in both directions
    p = _dense(n, d, 0.05, seed=n)
    _trajectory_check(p.X, p.y, p.lam, form="primal", kind="subsample", tau=tau, momentum="heuristic")


@pytest.mark.parametrize("case", ["dense-subsample", "csr-count-arows", "csr-subcount-scatter"])
def test_theory_momentum_trajectory_across_switch(case):
    """Theoretical momentum rule (eq:parameterswitchtheory): gamma_k falls and beta_k rises
    until the switch at k = 201 (eta 0.995, threshold 0.5), then both stay at 0.5; the
    checkpoints straddle the switch. The problems converge slowly enough that r stays far
    above rounding level at k = 240."""
    if case == "dense-subsample":
        p = inputs.make_dense(600, 300, 0.05, seed=600, col_log_sigma=1.0)
        kind, tau, route = "subsample", 10, "auto"
    elif case == "csr-count-arows":
        p = _csr(400, 150, 0.04, 0.05, seed=3)
        kind, tau, route = "count", 23, "arows"
    else:
        p = _csr(600, 300, 0.02, 0.05, seed=7)
        kind, tau, route = "subcount", 20, "scatter"
    _trajectory_check(p.X, p.y, p.lam, form="primal", kind=kind, tau=tau, momentum="theory",
                      checkpoints=[1, 7, 150, 200, 201, 202, 240], route=route)


def test_dense_subsample_trajectory_f32_colmajor_input():
    p = _dense(260, 70, 0.2, seed=9)
    Xf = np.asfortranarray(p.X.astype(np.float32))
    _trajectory_check(Xf, p.y, p.lam, form="primal", kind="subsample", tau=20, momentum="heuristic")


@pytest.mark.parametrize("route", ["scatter", "arows"])
@pytest.mark.parametrize("kind,sub_k", [("count", 0), ("subcount", 2)])
@pytest.mark.parametrize("form", ["primal", "dual"])
def test_sparse_trajectory(kind, sub_k, form, route):
    if form == "primal":
        p = _csr(400, 150, 0.04, 0.05, seed=3)
        tau = 23
    else:
        p = _csr(150, 400, 0.04, 0.05, seed=4)
        tau = 29
    _trajectory_check(p.X, p.y, p.lam, form=form, kind=kind, tau=tau, momentum="heuristic", sub_k=sub_k,
                      route=route)


@pytest.mark.parametrize("route", ["scatter", "arows"])
def test_sparse_ragged_rows_and_empty_columns(route):
    """CSR rows of very different lengths (one dense row, empty rows and columns), tau larger than
    one 64-column chunk, lookahead batches of 3."""
    rng = np.random.default_rng(21)
    n, d = 600, 230
    X = sp.random(n, d, density=0.02, random_state=5, format="lil")
    X[7, :] = rng.standard_normal(d)           # a dense row of X: a dense row of Z Z^T's pattern
    X[:, 11] = 0.0                             # an empty column
    X[40:45, :] = 0.0                          # empty rows
    X = sp.csr_matrix(X)
    y = rng.standard_normal(n)
    _trajectory_check(X, y, 0.3, form="primal", kind="count", tau=70, momentum="heuristic", lookahead=3,
                      route=route, checkpoints=[1, 4, 10])


def test_lookahead_batches_do_not_change_results():
    p = _dense(300, 130, 0.05, seed=1)
    outs = []
    for la in (1, 7, 64):
        S = rs.Solver(p.X, p.y, p.lam, tau=37, sketch="subsample", momentum="heuristic", tol=0.0,
                      lookahead=la)
        S.step(30)
        outs.append(S.state()[0])
        S.close()
    assert np.array_equal(outs[0], outs[1]) and np.array_equal(outs[0], outs[2])


def test_dense_primal_full_size_trajectory():
    """The dense primal workload at full size: X 2000 x 500, tau = 50, 50 iterations."""
    p = inputs.dense_primal()
    for momentum in ("none", "heuristic"):
        _trajectory_check(p.X, p.y, p.lam, form="primal", kind="subsample", tau=50, momentum=momentum,
                          checkpoints=[1, 10, 50])


@pytest.mark.timeout(900)
@pytest.mark.parametrize("workload,tau", [("dense_mixed", 1024), ("dense_learned", 512)])
def test_dense_large_full_size_first_iterations_fp64(workload, tau):
    """The large dense workloads at full size on the FP64 path (X 50000 x 8192 with log-normal(0,1)
    column scales, tau = 1024; X 200000 x 4096 with log-normal(0,2) columns and 5% correlated
    ones, tau = 512; primal, heuristic momentum): the first ten iterations against the oracle,
    entry by entry."""
    p = getattr(inputs, workload)()
    print(f"[dense full size fp64] {workload} tau={tau}", flush=True)
    _trajectory_check(p.X, p.y, p.lam, form="primal", kind="subsample", tau=tau, momentum="heuristic",
                      checkpoints=[1, 3, 10])


@pytest.mark.timeout(900)
@pytest.mark.parametrize("kind,sub_k", [("count", 0), ("subcount", 4)])
def test_sparse_full_size_trajectory(kind, sub_k):
    """The sparse workload at full size (CSR 100000 x 20000, 0.1%, tau = 500, primal, heuristic
    momentum): 50 iterations against the oracle, entry by entry, on both routes (the rows of
    Z Z^T and the scatter of CSR columns), count and SubCount (s = 4 tau)."""
    p = inputs.sparse_csr()
    checkpoints = [1, 3, 10, 25, 50]
    system = ridge_system(p.X, p.y, p.lam, "primal")
    opts = Options(sketch=kind, tau=500, sum_size=sub_k, momentum="heuristic", seed=5, tol=0.0)
    print(f"[sparse full size] {kind}: oracle, 50 iterations", flush=True)
    ref = _oracle_trajectory(system, opts, checkpoints)
    for route in ("arows", "scatter"):
        print(f"[sparse full size] {kind} route={route}", flush=True)
        _trajectory_check(p.X, p.y, p.lam, form="primal", kind=kind, tau=500, momentum="heuristic",
                          sub_k=sub_k, checkpoints=checkpoints, route=route, oracle=ref)


@pytest.mark.timeout(900)
def test_sparse_dual_full_size_trajectory():
    """The sparse workload in the dual form at full size (m = n = 100000 coordinates, K = 20000,
    count sketch tau = 500): ten iterations against the oracle, entry by entry, on both routes
    (the rows of X X^T hold about 2e8 entries, beyond the LDS bucket map: the packed-map kernel)."""
    p = inputs.sparse_csr()
    checkpoints = [1, 2, 5, 10]
    system = ridge_system(p.X, p.y, p.lam, "dual")
    opts = Options(sketch="count", tau=500, momentum="heuristic", seed=5, tol=0.0)
    print("[dual full size] oracle, 10 iterations", flush=True)
    ref = _oracle_trajectory(system, opts, checkpoints)
    for route in ("arows", "scatter"):
        print(f"[dual full size] route={route}", flush=True)
        _trajectory_check(p.X, p.y, p.lam, form="dual", kind="count", tau=500, momentum="heuristic",
                          checkpoints=checkpoints, route=route, oracle=ref)


def test_sparse_packed_bucket_map():
    """m = 45000 coordinates (dual form): the 16-bit bucket map no longer fits LDS beside eight
    accumulators, so the rows of X X^T take the kernel with three 10-bit codes per word."""
    p = _csr(45000, 3000, 0.002, 0.05, seed=45)
    for kind, sub_k in (("count", 0), ("subcount", 10)):
        _trajectory_check(p.X, p.y, p.lam, form="dual", kind=kind, tau=100, momentum="heuristic", sub_k=sub_k,
                          checkpoints=[1, 5, 20], route="arows")


def test_solve_converges_to_direct_solution():
    p = _dense(400, 120, 0.1, seed=4)
    S = rs.Solver(p.X, p.y, p.lam, tau=30, sketch="subsample", momentum="heuristic", tol=1e-10,
                  max_iter=20000)
    w, st, rep = S.solve()
    assert st == rs.RS_OK and rep.rel_res <= 1e-10
    A = p.X.T @ p.X + p.lam * np.eye(120)
    w_direct = np.linalg.solve(A, p.X.T @ p.y)
    assert np.linalg.norm(w - w_direct) <= 1e-8 * np.linalg.norm(w_direct)
    # stop iteration equals the first k with ||r^k|| / ||r^0|| <= tol
    hist = S.history()
    assert hist[-1] <= 1e-10 and np.all(hist[:-1] > 1e-10)
    S.close()


def test_dual_weights_match_primal():
    p = _csr(120, 300, 0.05, 0.3, seed=8)
    wd, st1, _ = rs.Solver(p.X, p.y, p.lam, tau=25, sketch="count", form="dual", tol=1e-11,
                           max_iter=200000).solve()
    wp, st2, _ = rs.Solver(p.X, p.y, p.lam, tau=25, sketch="count", form="primal", tol=1e-11,
                           max_iter=200000).solve()
    assert st1 == rs.RS_OK and st2 == rs.RS_OK
    assert np.linalg.norm(wd - wp) <= 1e-7 * np.linalg.norm(wp)


def test_not_converged_status():
    p = _dense(300, 130, 0.05, seed=1)
    S = rs.Solver(p.X, p.y, p.lam, tau=5, max_iter=3, tol=1e-12)
    w, st, rep = S.solve()
    assert st == rs.RS_NOT_CONVERGED and rep.iters == 3
    S.close()


def test_device_inputs_from_torch():
    import torch
    p = _dense(300, 130, 0.05, seed=1)
    Xd = torch.from_numpy(p.X).cuda()
    yd = torch.from_numpy(p.y).cuda()
    S1 = rs.Solver(Xd, yd, p.lam, tau=37, tol=0.0, stream=torch.cuda.current_stream().cuda_stream)
    S2 = rs.Solver(p.X, p.y, p.lam, tau=37, tol=0.0)
    S1.step(10)
    S2.step(10)
    assert np.array_equal(S1.state()[0], S2.state()[0])
    rowptr = torch.from_numpy(sp.csr_matrix(p.X).indptr.astype(np.int64)).cuda()
    assert rowptr.is_cuda


@pytest.mark.parametrize("case", ["dense_primal", "dense_dual", "csr_count_arows", "csr_subcount_dual_scatter",
                                  "kernel", "mixed", "gaussian"])
def test_report_true_residual_matches_oracle(case):
    """rs_report.rel_res_true, the FP64 residual of the returned iterate formed from the data,
    against ||A x - b|| / ||b|| formed by the oracle for the same x: the two differ at most
    by 4 gamma_n || |Z| (|Z^T| |x|) + lambda |x| + |b| || / ||b|| (two dot-product orders,
    Higham Sec. 3.1; kernel ridge: |K| (|K| |x|) + lambda |K| |x| + |b|)."""
    from oracle.problem import kernel_system
    kw = dict(tol=1e-8, seed=3, max_iter=100000)
    if case == "kernel":
        p = inputs.make_points(300, 6, 1e-2, 0.5, seed=81)
        system = kernel_system(p.P, p.y, p.lam, p.sigma)
        S = rs.Solver(p.P, p.y, p.lam, tau=40, kernel_sigma=p.sigma, **kw)
    else:
        form = "dual" if "dual" in case else "primal"
        if case.startswith("csr"):
            p = _csr(500, 220, 0.03, 0.05, seed=82) if form == "primal" else _csr(220, 500, 0.03, 0.05, seed=83)
            kind = "count" if "subcount" not in case else "subcount"
            route = "arows" if "arows" in case else "scatter"
            S = rs.Solver(p.X, p.y, p.lam, tau=25, sketch=kind, form=form, subcount_k=2, sparse_route=route, **kw)
        else:
            dt = np.float32 if case == "mixed" else np.float64
            p = inputs.make_dense(400, 150, 0.05, seed=84, dtype=dt) if form == "primal" else \
                inputs.make_dense(150, 400, 0.05, seed=85)
            sketch = "gaussian" if case == "gaussian" else "subsample"
            S = rs.Solver(p.X, p.y, p.lam, tau=30, sketch=sketch, form=form,
                          precision="mixed" if case == "mixed" else "fp64", **kw)
        system = ridge_system(p.X, p.y, p.lam, form)
    _, st, rep = S.solve()
    assert st == rs.RS_OK
    x = S.state()[0]
    S.close()
    r = system.matvec(x) - system.b
    nb = np.linalg.norm(system.b)
    if case == "kernel":
        K = np.abs(system.Kmat)
        mag = K @ (K @ np.abs(x)) + p.lam * (K @ np.abs(x)) + np.abs(system.b)
        n = K.shape[0]
    else:
        Z = system.Z.toarray() if hasattr(system.Z, "toarray") else np.asarray(system.Z)
        Z = np.abs(Z)
        mag = Z @ (Z.T @ np.abs(x)) + p.lam * np.abs(x) + np.abs(system.b)
        n = max(Z.shape)
    gamma = n * 2.0 ** -53 / (1 - n * 2.0 ** -53)
    bound = 4 * gamma * np.linalg.norm(mag) / nb
    assert abs(rep.rel_res_true - np.linalg.norm(r) / nb) <= bound, (rep.rel_res_true, np.linalg.norm(r) / nb, bound)
    if case == "mixed":  # the stop test there uses the FP64-refreshed residual
        assert rep.rel_res_true <= 1e-8 * 1.001
