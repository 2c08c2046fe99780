"""GPU: batched lock-step solves (problems of different shapes x lambda grid x right-hand sides).

Slot (p, l, q) of a batch draws the sketch sequence of the single solve with
problem_id = p (same Philox key), so its trajectory is the single solve's up to the
rounding of forming A(lambda) S as B S + lambda S: checked to 1e-10 against the single
GPU solve and against the oracle. Captured-graph replays equal direct launches bit
for bit; converged weights match a direct solve; per-problem caps and resets behave.
"""
import numpy as np
import pytest

from oracle.problem import ridge_system
from oracle.solver import Options, init_state, step
from paper_2105_05565_amd import inputs, rs
from parity_util import assert_state_close, assert_vec_close

pytestmark = pytest.mark.gpu

LAMS = [0.05, 0.5, 2.0]


def _problems():
    rng = np.random.default_rng(11)
    out = []
    specs = [("dense", 300, 130, 37, np.float64), ("dense", 110, 260, 0, np.float32),
             ("csr", 400, 150, 23, np.float64), ("csr", 150, 400, 30, np.float32)]
    for i, (kind, n, d, tau, dt) in enumerate(specs):
        if kind == "dense":
            X = inputs.make_dense(n, d, 0.1, seed=100 + i, dtype=dt).X
        else:
            X = inputs.make_csr(n, d, 0.04, 0.1, seed=100 + i, dtype=dt).X
        y = rng.standard_normal((n, 2))
        out.append(dict(X=X, y=y, lambdas=LAMS, tau=tau))
    return out


def _single(pr, p, l, q, iters, seed, tol=0.0):
    tau = pr["tau"] if pr["tau"] else 64
    sketch = "count" if hasattr(pr["X"], "tocsr") else "subsample"
    S = rs.Solver(pr["X"], pr["y"][:, q], pr["lambdas"][l], tau=tau, sketch=sketch, tol=tol, seed=seed,
                  problem_id=p, max_iter=100000)
    return S


def _rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def test_batch_matches_single_solves_and_oracle():
    probs = _problems()
    N = 25
    B = rs.Batch(probs, tol=0.0, seed=4, graph_iters=4)
    B.step(N)
    assert B.k == N
    for p, pr in enumerate(probs):
        info = B.info(p)
        assert info.slots == 6
        for l in range(3):
            for q in range(2):
                j = l * 2 + q
                x, xp, r, rp = B.state(p, j)
                S = _single(pr, p, l, q, N, seed=4)
                S.step(N)
                xs, xps, rs_, rps = S.state()
                S.close()
                assert_state_close((x, xp, r, rp), [("x", xs), ("x_prev", xps), ("r", rs_), ("r_prev", rps)],
                                   1e-10, f"slot ({p}, {j}) vs single solve")
    # oracle, one slot per problem
    for p, pr in enumerate(probs):
        l, q = p % 3, (p + 1) % 2
        system = ridge_system(pr["X"], pr["y"][:, q], pr["lambdas"][l])
        sketch = "count" if hasattr(pr["X"], "tocsr") else "subsample"
        tau = pr["tau"] if pr["tau"] else 64
        opts = Options(sketch=sketch, tau=tau, momentum="heuristic", tol=0.0, max_iter=N, seed=4,
                       problem_id=p)
        st = init_state(system)
        for _ in range(N):
            step(system, st, opts)
        assert_state_close(B.state(p, l * 2 + q), [("x", st.w), ("x_prev", st.w_prev), ("r", st.r),
                                                   ("r_prev", st.r_prev)], 1e-10, f"problem {p} vs oracle")
    B.close()


def test_batch_theory_momentum_across_switch_matches_oracle():
    """The schedule table of a batch under the theoretical momentum rule: 230 iterations
    cross its switch at k = 201; one slot per problem against the oracle."""
    probs = _problems()
    N = 230
    B = rs.Batch(probs, momentum="theory", tol=0.0, seed=6, graph_iters=8)
    B.step(N)
    for p, pr in enumerate(probs):
        l, q = (p + 2) % 3, p % 2
        system = ridge_system(pr["X"], pr["y"][:, q], pr["lambdas"][l])
        sketch = "count" if hasattr(pr["X"], "tocsr") else "subsample"
        tau = pr["tau"] if pr["tau"] else 64
        opts = Options(sketch=sketch, tau=tau, momentum="theory", tol=0.0, max_iter=N, seed=6, problem_id=p)
        st = init_state(system)
        for _ in range(N):
            step(system, st, opts)
        assert_state_close(B.state(p, l * 2 + q), [("x", st.w), ("x_prev", st.w_prev), ("r", st.r),
                                                   ("r_prev", st.r_prev)], 1e-10, f"problem {p} vs oracle (theory)")
    B.close()


def test_default_tau_rule():
    probs = _problems()
    B = rs.Batch(probs[:2], tol=0.0)
    assert B.info(0).tau == 37
    assert B.info(1).tau == 64  # m = 110: 64 round(110^(2/3) / 64) = 0 -> clamped to 64
    B.close()


def test_graph_replay_equals_direct_launches():
    probs = _problems()
    A = rs.Batch(probs, tol=0.0, seed=2, graph_iters=4)
    D = rs.Batch(probs, tol=0.0, seed=2, graph_iters=-1)
    A.step(10)
    D.step(10)
    for p in range(len(probs)):
        for j in (0, 5):
            for u, v in zip(A.state(p, j), D.state(p, j)):
                assert np.array_equal(u, v), (p, j)
    A.close()
    D.close()


def test_converged_batch_matches_direct_solution_and_single_stop_iterations():
    probs = _problems()
    tol = 1e-8
    B = rs.Batch(probs, tol=tol, seed=3)
    st, rep = B.solve()
    assert st == rs.RS_OK and rep.converged == rep.solves == 24
    for p, pr in enumerate(probs):
        stop, rel = B.slots(p)
        assert np.all(stop > 0) and np.all(rel <= tol)
        W = B.weights(p)
        for l in range(3):
            for q in range(2):
                j = l * 2 + q
                system = ridge_system(pr["X"], pr["y"][:, q], pr["lambdas"][l])
                A = system.dense_A()
                w_direct = system.weights(np.linalg.solve(A, system.b))
                kappa = np.linalg.cond(A)
                assert _rel(W[j], w_direct) <= 2 * kappa * tol, (p, j)
                S = _single(pr, p, l, q, 0, seed=3, tol=tol)
                w1, st1, rep1 = S.solve()
                S.close()
                assert abs(rep1.iters - stop[j]) <= 1, (p, j, rep1.iters, stop[j])
    B.close()


def test_caps_and_not_converged():
    probs = _problems()
    probs[1]["max_iter"] = 5
    B = rs.Batch(probs, tol=1e-10, seed=1)
    st, rep = B.solve()
    assert st == rs.RS_NOT_CONVERGED
    assert B.info(1).iters == 5
    stop, rel = B.slots(1)
    assert np.all(stop == -1) and np.all(rel > 1e-10)
    for p in (0, 2, 3):
        assert np.all(B.slots(p)[0] > 0)
    B.close()


def test_reset_and_autotune():
    probs = _problems()
    B = rs.Batch(probs, tol=0.0, seed=5, autotune=True)
    t = B.tuning()
    assert t["tuned"] == 1 and t["dense_tk"] == 16 and t["dense_ms"] > 0
    B.step(8)
    first = [B.state(p, 3)[0] for p in range(4)]
    B.reset(6)
    B.step(8)
    C = rs.Batch(probs, tol=0.0, seed=6)
    C.step(8)
    for p in range(4):
        assert _rel(B.state(p, 3)[0], C.state(p, 3)[0]) <= 1e-12
    B.reset(5)
    B.step(8)
    for p in range(4):
        assert _rel(B.state(p, 3)[0], first[p]) <= 1e-14
    B.close()
    C.close()


@pytest.mark.timeout(900)
def test_batched_full_size_sampled_slots():
    """The batched workload at full size, built as the benchmark builds it (64 problems,
    n ~ U{2000..40000}, d ~ U{500..8000}, half dense and half CSR at 0.5%, 16 lambdas x 4
    right-hand sides, autotuned launch shapes, torch's current stream): one slot of each of four
    problems (dense and CSR, primal and dual form where the batch has one) against the oracle's
    solve to 1e-10, entry by entry, after 3 and after 10 lock steps."""
    import torch
    from oracle.problem import choose_form
    probs = inputs.batched()
    stream = torch.cuda.current_stream().cuda_stream
    B = rs.Batch(probs, tol=0.0, seed=1, autotune=True, stream=stream)
    N = 10
    picks = []
    for kind in ("dense", "csr"):
        for form in ("primal", "dual"):
            cands = [p for p, pr in enumerate(probs)
                     if pr["kind"] == kind and choose_form(pr["n"], pr["d"]) == form]
            if cands:
                picks.append(cands[len(cands) // 2])
    assert len(picks) >= 2
    ref = {}
    for p in picks:
        pr = probs[p]
        l, q = p % len(pr["lambdas"]), p % pr["y"].shape[1]
        print(f"[batched full size] problem {p} {pr['kind']} n={pr['n']} d={pr['d']} tau={pr['tau']}",
              flush=True)
        system = ridge_system(pr["X"], pr["y"][:, q], pr["lambdas"][l])
        opts = Options(sketch="subsample" if pr["kind"] == "dense" else "count", tau=pr["tau"],
                       momentum="heuristic", tol=0.0, max_iter=N, seed=1, problem_id=p)
        st = init_state(system)
        ref[p] = {}
        for c in (3, N):
            while st.k < c:
                step(system, st, opts)
            ref[p][c] = [("x", st.w.copy()), ("x_prev", st.w_prev.copy()), ("r", st.r.copy()),
                         ("r_prev", st.r_prev.copy())]
    for c in (3, N):
        B.step(c - B.k)
        assert B.k == c
        for p in picks:
            pr = probs[p]
            l, q = p % len(pr["lambdas"]), p % pr["y"].shape[1]
            assert_state_close(B.state(p, l * pr["y"].shape[1] + q), ref[p][c], 1e-10,
                               f"full-size batch problem {p} k={c}")
    B.close()


# ---- mixed precision (BF16 products for the dense problems, FP64 refresh) ----

def _refresh_bound(system, x):
    """Dot-product bound of two FP64 summation orders of Z (Z^T x) + lambda x - b."""
    Za = np.abs(np.asarray(system.Z.todense()) if hasattr(system.Z, "todense") else system.Z)
    n = max(Za.shape)
    gamma = n * 2.0 ** -53 / (1 - n * 2.0 ** -53)
    return 4 * gamma * (Za @ (Za.T @ np.abs(x)) + system.lam * np.abs(x) + np.abs(system.b))


def test_mixed_batch_refresh_recomputes_true_residual():
    """After R lock steps (refresh interval R) a dense problem's r^R and r^{R-1} are the FP64
    residuals A x - b of its iterates x^R and x^{R-1} (within the dot-product bound of the two
    summation orders), for every slot; the CSR problems, whose products stay FP64, follow the
    FP64 batch bit for bit."""
    probs = _problems()
    R = 5
    M = rs.Batch(probs, tol=0.0, seed=4, precision="mixed", refresh_every=R, graph_iters=4)
    F = rs.Batch(probs, tol=0.0, seed=4, graph_iters=4)
    M.step(R)
    F.step(R)
    for p, pr in enumerate(probs):
        for l in range(3):
            for q in range(2):
                j = l * 2 + q
                x, xp, r, rp = M.state(p, j)
                if hasattr(pr["X"], "tocsr"):
                    for u, v in zip((x, xp, r, rp), F.state(p, j)):
                        assert np.array_equal(u, v), (p, j)
                    continue
                system = ridge_system(pr["X"], pr["y"][:, q], pr["lambdas"][l])
                for xx, rr, what in ((x, r, "r^R"), (xp, rp, "r^{R-1}")):
                    true = system.matvec(xx) - system.b
                    err = np.abs(rr - true)
                    bound = _refresh_bound(system, xx)
                    assert np.all(err <= bound), (p, j, what, float((err / bound).max()))
    M.close()
    F.close()


def test_mixed_batch_converges_and_stops_only_at_refreshes():
    """A mixed batch solved to tol: every slot converges; a dense problem's slots stop only at
    refresh iterations (multiples of R) and reach the direct solution within 2 kappa tol; the
    CSR problems stop where the FP64 batch stops."""
    probs = _problems()
    tol, R = 1e-8, 10
    M = rs.Batch(probs, tol=tol, seed=3, precision="mixed", refresh_every=R)
    F = rs.Batch(probs, tol=tol, seed=3)
    st, rep = M.solve()
    assert st == rs.RS_OK and rep.converged == rep.solves == 24
    F.solve()
    for p, pr in enumerate(probs):
        stop, rel = M.slots(p)
        assert np.all(stop > 0) and np.all(rel <= tol)
        if hasattr(pr["X"], "tocsr"):
            assert np.array_equal(stop, F.slots(p)[0]), p
            continue
        assert np.all(stop % R == 0), (p, stop)
        W = M.weights(p)
        for l in range(3):
            for q in range(2):
                j = l * 2 + q
                system = ridge_system(pr["X"], pr["y"][:, q], pr["lambdas"][l])
                A = system.dense_A()
                w_direct = system.weights(np.linalg.solve(A, system.b))
                assert _rel(W[j], w_direct) <= 2 * np.linalg.cond(A) * tol, (p, j)
    M.close()
    F.close()


def test_mixed_batch_graph_replay_equals_direct_launches():
    """Replays of the captured mixed sequence (the refresh kernels run every iteration and act
    only at refresh iterations) equal direct launches bit for bit across two refreshes."""
    probs = _problems()
    A = rs.Batch(probs, tol=0.0, seed=2, precision="mixed", refresh_every=5, graph_iters=4)
    D = rs.Batch(probs, tol=0.0, seed=2, precision="mixed", refresh_every=5, graph_iters=-1)
    A.step(12)
    D.step(12)
    for p in range(len(probs)):
        for j in (0, 5):
            for u, v in zip(A.state(p, j), D.state(p, j)):
                assert np.array_equal(u, v), (p, j)
    A.close()
    D.close()
