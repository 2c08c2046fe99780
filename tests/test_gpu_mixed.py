"""GPU: sketched products against the oracle (FP64) and the mixed-precision path
(BF16 products with FP32 accumulation on dense data, FP32-stored AS on CSR data, FP64
Cholesky, periodic FP64 refresh).

The BF16 products are bounded by the standard dot-product error bound (Higham,
Accuracy and Stability, Sec. 3.1) applied to BF16-rounded inputs accumulated in
FP32: |AS_gpu - AS| <= (2 u_bf16 + K u_fp32) (|Z| |Z_C|^T) elementwise, u_bf16 = 2^-8,
u_fp32 = 2^-24 (unit roundoffs of round-to-nearest).
"""
import numpy as np
import pytest

from oracle import sketch as osk
from oracle.problem import ridge_system
from oracle.solver import sketched_products
from paper_2105_05565_amd import inputs, rs

pytestmark = pytest.mark.gpu

U_BF16 = 2.0 ** -8
U_FP32 = 2.0 ** -24


def _oracle_products(p, form, kind, k, tau, sub_k=0, seed=5):
    system = ridge_system(p.X, p.y, p.lam, form)
    s = osk.draw(kind, seed, 0, k, system.m, tau, sum_size=sub_k)
    S, AS, G, active = sketched_products(system, s)
    return system, s, AS, G, active


@pytest.mark.parametrize("kind,form,route", [("subsample", "primal", "auto"), ("subsample", "dual", "auto"),
                                             ("count", "primal", "scatter"), ("subcount", "dual", "scatter"),
                                             ("count", "primal", "arows"), ("subcount", "dual", "arows"),
                                             ("count", "dual", "arows")])
def test_fp64_products_match_oracle(kind, form, route):
    if kind == "subsample":
        p = inputs.make_dense(300, 130, 0.05, seed=1) if form == "primal" else inputs.make_dense(110, 260, 0.05, seed=2)
        tau = 37
    else:
        p = inputs.make_csr(400, 150, 0.04, 0.05, seed=3) if form == "primal" else inputs.make_csr(150, 400, 0.04, 0.05, seed=4)
        tau = 23
    S = rs.Solver(p.X, p.y, p.lam, tau=tau, sketch=kind, form=form, tol=0.0, seed=5, subcount_k=2,
                  sparse_route=route)
    S.step(3)
    AS, Gi = S.products()
    _, s, AS_or, G_or, active = _oracle_products(p, form, kind, 2, tau, sub_k=2)
    assert np.allclose(AS, AS_or, rtol=1e-12, atol=1e-12 * np.abs(AS_or).max())
    G = G_or.copy()
    for b in np.flatnonzero(~active):
        G[b, b] = 1.0
    assert np.allclose(Gi @ G, np.eye(tau), atol=1e-10)
    S.close()


def _bf16(a):
    """Round float32 values to the nearest BF16 (ties to even), returned as float64."""
    u = np.ascontiguousarray(a, dtype=np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


@pytest.mark.parametrize("n,d,tau,form", [(700, 300, 37, "primal"), (300, 700, 41, "dual"),
                                          (1200, 513, 64, "primal"), (8192, 300, 37, "primal"),
                                          (8192, 600, 37, "primal")])
def test_mixed_products_within_bound(n, d, tau, form):
    """The last two cases (m = 300 and 600, K = 8192: two and three 256 x 256 tiles per launch) run
    the launch split over K into 4 ranges summed into a workspace and added in order; with three
    tiles the 12 (range, tile) pairs leave workgroups of the 8-XCD layout idle."""
    p = inputs.make_dense(n, d, 0.1, seed=n + d, dtype=np.float32, col_log_sigma=1.0)
    S = rs.Solver(p.X, p.y, p.lam, tau=tau, sketch="subsample", form=form, tol=0.0, seed=5,
                  precision="mixed", lookahead=3)
    S.step(3)
    AS, Gi = S.products()
    system, s, AS_or, _, _ = _oracle_products(p, form, "subsample", 2, tau)
    Z = np.asarray(system.Z, dtype=np.float64)
    K = Z.shape[1]
    C = s.rows
    bound = (2 * U_BF16 + K * U_FP32) * (np.abs(Z) @ np.abs(Z[C]).T) + 1e-30
    err = np.abs(AS - AS_or)
    assert np.all(err <= bound), float((err / bound).max())
    # against the product of BF16-rounded data: only FP32 accumulation error remains
    Zb = _bf16(Z.astype(np.float32))
    AS_b = Zb @ Zb[C].T
    AS_b[C, np.arange(tau)] += p.lam
    bound_b = K * U_FP32 * (np.abs(Zb) @ np.abs(Zb[C]).T) + 1e-6 * p.lam
    assert np.all(np.abs(AS - AS_b) <= bound_b)
    # G^{-1} inverts the sketched matrix the GPU formed (lower triangle of AS[C, :])
    Gm = np.tril(AS[C]) + np.tril(AS[C], -1).T
    assert np.allclose(Gi @ Gm, np.eye(tau), atol=1e-8)
    S.close()


def test_mixed_sketches_bit_exact():
    p = inputs.make_dense(700, 300, 0.1, seed=3, dtype=np.float32)
    S = rs.Solver(p.X, p.y, p.lam, tau=37, sketch="subsample", tol=0.0, seed=9, precision="mixed")
    for k in range(3):
        S.step(1)
        rows, cols, signs = S.last_sketch()
        exp = osk.draw_subsample(9, 0, k, 300, 37)
        assert np.array_equal(rows, exp.rows) and np.array_equal(cols, exp.cols)
    S.close()


def test_mixed_refresh_recomputes_true_residual():
    p = inputs.make_dense(900, 300, 0.1, seed=4, dtype=np.float32, col_log_sigma=1.0)
    system = ridge_system(p.X, p.y, p.lam, "primal")
    S = rs.Solver(p.X, p.y, p.lam, tau=40, sketch="subsample", tol=0.0, seed=2, precision="mixed",
                  refresh_every=10, lookahead=16)
    for steps in (10, 20, 40):
        S.step(steps - S.k)
        x, xp, r, rp = S.state()
        for xx, rr in ((x, r), (xp, rp)):
            true = system.matvec(xx) - system.b
            assert np.linalg.norm(rr - true) <= 1e-12 * np.linalg.norm(system.b)
    S.close()


@pytest.mark.parametrize("form", ["primal", "dual"])
def test_mixed_converges_to_fp64_solution(form):
    if form == "primal":
        p = inputs.make_dense(2000, 400, 0.1, seed=7, dtype=np.float32, col_log_sigma=1.0)
    else:
        p = inputs.make_dense(400, 2000, 0.1, seed=8, dtype=np.float32, col_log_sigma=1.0)
    system = ridge_system(p.X, p.y, p.lam, form)
    S = rs.Solver(p.X, p.y, p.lam, tau=64, sketch="subsample", form=form, tol=1e-8, seed=3,
                  precision="mixed", max_iter=200000)
    w, st, rep = S.solve()
    assert st == rs.RS_OK
    x = S.state()[0]
    true_rel = np.linalg.norm(system.matvec(x) - system.b) / np.linalg.norm(system.b)
    assert true_rel <= 1e-8 * 1.0001
    A = system.dense_A()
    w_direct = system.weights(np.linalg.solve(A, system.b))
    kappa = np.linalg.cond(A)
    rel_err = np.linalg.norm(w - w_direct) / np.linalg.norm(w_direct)
    assert rel_err <= 2 * kappa * 1e-8, (rel_err, kappa)
    S.close()


@pytest.mark.parametrize("kind,sub_k", [("count", 0), ("subcount", 3)])
@pytest.mark.parametrize("form", ["primal", "dual"])
def test_csr_mixed_products_within_fp32_bound(kind, sub_k, form):
    """CSR data in mixed precision: the bucket sums of AS are formed in FP64 from the rows of
    Z Z^T and stored in FP32, so each entry is within u_fp32 |AS| of the exact product (plus
    FP64 summation error); G = S^T AS is summed in FP64 from the stored entries, so
    G_gpu = G + E with |E| <= |S|^T (u_fp32 |AS|), and the returned G^{-1} inverts G to
    ||G^{-1}|| ||E|| (plus FP64 rounding)."""
    p = inputs.make_csr(500, 220, 0.03, 0.05, seed=61) if form == "primal" else \
        inputs.make_csr(220, 500, 0.03, 0.05, seed=62)
    tau = 25
    S = rs.Solver(p.X, p.y, p.lam, tau=tau, sketch=kind, form=form, subcount_k=sub_k, tol=0.0, seed=5,
                  precision="mixed", lookahead=3)
    S.step(3)
    AS, Gi = S.products()
    S.close()
    system, s, AS_or, G_or, active = _oracle_products(p, form, kind, 2, tau, sub_k)
    bound = U_FP32 * np.abs(AS_or) + 1e-13 * np.abs(AS_or).max()
    err = np.abs(AS - AS_or)
    assert np.all(err <= bound), float((err / bound).max())
    Sabs = np.abs(s.matrix().toarray())
    Eb = Sabs.T @ (U_FP32 * np.abs(AS_or))
    G = G_or.copy()
    for b in np.flatnonzero(~active):
        G[b, b] = 1.0
    resid = np.linalg.norm(Gi @ G - np.eye(tau), 2)
    assert resid <= 1.01 * np.linalg.norm(Gi, 2) * np.linalg.norm(Eb) + 1e-10, resid


@pytest.mark.parametrize("kind", ["count", "subcount"])
def test_csr_mixed_refresh_recomputes_true_residual(kind):
    """Every refresh_every iterations r^k and r^{k-1} are recomputed in FP64 from the CSR data
    (Z^T x, then Z (Z^T x)): they equal A x - b formed by the oracle for the GPU's iterates."""
    p = inputs.make_csr(900, 300, 0.02, 0.05, seed=63, dtype=np.float32)
    system = ridge_system(p.X, p.y, p.lam, "primal")
    S = rs.Solver(p.X, p.y, p.lam, tau=30, sketch=kind, subcount_k=2, tol=0.0, seed=2, precision="mixed",
                  refresh_every=10, lookahead=16)
    for steps in (10, 20, 40):
        S.step(steps - S.k)
        x, xp, r, rp = S.state()
        for xx, rr in ((x, r), (xp, rp)):
            true = system.matvec(xx) - system.b
            assert np.linalg.norm(rr - true) <= 1e-12 * np.linalg.norm(system.b)
    S.close()


@pytest.mark.parametrize("kind", ["count", "subcount"])
def test_csr_mixed_stops_only_on_refreshed_residual(kind):
    """A mixed CSR solve stops at the first refresh whose FP64 residual is <= tol. With
    refreshes only every refresh_every iterations the stop iteration is a multiple of it; with
    the early refresh (the default) it is that or the end of a lookahead batch whose last
    tracked estimate had reached tol, no later than the first. Either way the reported and
    recomputed residuals are <= tol and the weights reach the direct solution within 2 kappa tol."""
    p = inputs.make_csr(2000, 400, 0.02, 0.1, seed=64, dtype=np.float32)
    system = ridge_system(p.X, p.y, p.lam, "primal")
    tol = 1e-8
    A = system.dense_A()
    w_direct = np.linalg.solve(A, system.b)
    iters = {}
    for early in (False, True):
        S = rs.Solver(p.X, p.y, p.lam, tau=40, sketch=kind, subcount_k=3, tol=tol, seed=3, precision="mixed",
                      max_iter=200000, refresh_every=20, refresh_early=early)
        w, st, rep = S.solve()
        assert st == rs.RS_OK
        hist = S.history()
        if early:
            assert rep.iters % 20 == 0 or hist[rep.iters - 1] <= tol
        else:
            assert rep.iters % 20 == 0
        assert rep.rel_res <= tol and rep.rel_res_true <= tol * 1.0001
        assert hist[rep.iters] <= tol
        assert np.linalg.norm(w - w_direct) <= 2 * np.linalg.cond(A) * tol * np.linalg.norm(w_direct)
        iters[early] = rep.iters
        S.close()
    assert iters[True] <= iters[False]


@pytest.mark.parametrize("lookahead", [2, 5])
def test_dense_mixed_early_refresh(lookahead):
    """Dense mixed solve with small lookahead batches: the early refresh stops at the first
    batch end whose tracked estimate reached tol and whose FP64 residual meets it (never
    later than the refresh_every schedule), at a true residual <= tol."""
    p = inputs.make_dense(2000, 400, 0.1, seed=7, dtype=np.float32, col_log_sigma=1.0)
    system = ridge_system(p.X, p.y, p.lam, "primal")
    tol = 1e-8
    iters = {}
    for early in (False, True):
        S = rs.Solver(p.X, p.y, p.lam, tau=64, sketch="subsample", tol=tol, seed=3, precision="mixed",
                      max_iter=200000, lookahead=lookahead, refresh_early=early)
        w, st, rep = S.solve()
        assert st == rs.RS_OK
        hist = S.history()
        x = S.state()[0]
        true_rel = np.linalg.norm(system.matvec(x) - system.b) / np.linalg.norm(system.b)
        assert true_rel <= tol * 1.0001 and rep.rel_res <= tol and hist[rep.iters] <= tol
        if early:
            assert rep.iters % 20 == 0 or (rep.iters % lookahead == 0 and hist[rep.iters - 1] <= tol)
        else:
            assert rep.iters % 20 == 0
        iters[early] = rep.iters
        S.close()
    assert iters[True] <= iters[False]


def test_csr_mixed_rejections():
    p = inputs.make_csr(100, 40, 0.1, 0.1, seed=1)
    with pytest.raises(rs.RsError) as e:
        rs.Solver(p.X, p.y, p.lam, tau=5, sketch="count", precision="mixed", sparse_route="scatter")
    assert e.value.status == rs.RS_EUNSUPPORTED
    with pytest.raises(rs.RsError) as e:
        rs.Solver(p.X, p.y, p.lam, tau=5, sketch="count", precision="mixed", accel=(0.5, 1.5))
    assert e.value.status == rs.RS_EUNSUPPORTED


@pytest.mark.timeout(600)
def test_csr_mixed_full_size_sampled():
    """The sparse workload at full size in mixed precision, launched as the benchmark launches it
    (CSR 100000 x 20000, count sketch tau = 500, default lookahead and pipeline): 48 sampled rows
    of the 20th sketch's AS within the FP32 bound against the oracle's FP64 rows, and the
    refreshed r^20, r^19 against the oracle's A x - b for the GPU's iterates within
    4 gamma_n (|Z| (|Z^T| |x|) + lambda |x| + |b|)."""
    p = inputs.sparse_csr()
    system = ridge_system(p.X, p.y, p.lam, "primal")
    print("[csr mixed full size] count tau=500", flush=True)
    S = rs.Solver(p.X, p.y, p.lam, tau=500, sketch="count", tol=0.0, seed=1, precision="mixed")
    S.step(20)
    AS, _ = S.products()
    x, xp, r, rp = S.state()
    S.close()
    sk = osk.draw("count", 1, 0, 19, system.m, 500)
    rng = np.random.default_rng(5)
    rows = np.sort(rng.choice(system.m, 48, replace=False))
    Zr = system.Z[rows]
    AS_o = np.asarray((Zr @ (system.Z.T @ sk.matrix())).todense()) + system.lam * sk.matrix().toarray()[rows]
    bound = U_FP32 * np.abs(AS_o) + 1e-13 * np.abs(AS_o).max()
    assert np.all(np.abs(AS[rows] - AS_o) <= bound)
    Za = abs(system.Z)
    n = system.Z.shape[1]
    gamma = n * 2.0 ** -53 / (1 - n * 2.0 ** -53)
    for xx, rr in ((x, r), (xp, rp)):
        true = system.matvec(xx) - system.b
        mag = Za @ (Za.T @ np.abs(xx)) + system.lam * np.abs(xx) + np.abs(system.b)
        assert np.all(np.abs(rr - true) <= 4 * gamma * mag)


@pytest.mark.parametrize("tau,kind", [(130, "subsample"), (300, "subsample"), (700, "subsample"),
                                      (257, "count")])
def test_tiled_factorisation_inverse(tau, kind):
    """G^{-1} from the device-wide tiled factorisation (tau > 64) inverts the oracle's G."""
    if kind == "subsample":
        p = inputs.make_dense(1500, 800, 0.5, seed=tau)
    else:
        p = inputs.make_csr(3000, 900, 0.01, 0.5, seed=tau)
    S = rs.Solver(p.X, p.y, p.lam, tau=tau, sketch=kind, form="primal", tol=0.0, seed=5, lookahead=5)
    S.step(5)
    AS, Gi = S.products()
    _, s, AS_or, G_or, active = _oracle_products(p, "primal", kind, 4, tau)
    G = G_or.copy()
    for b in np.flatnonzero(~active):
        G[b, b] = 1.0
    err = np.abs(Gi @ G - np.eye(tau)).max()
    assert err <= 1e-9, err
    assert np.allclose(Gi, Gi.T, rtol=0, atol=1e-12 * np.abs(Gi).max())
    S.close()


@pytest.mark.parametrize("workload,tau", [("dense_mixed", 1024), ("dense_learned", 512)])
def test_mixed_full_size_sampled(workload, tau):
    """The BF16 workloads at full size, launched as the benchmark launches them (device inputs
    on torch's current stream, default lookahead and preparation pipeline; uniform sampling):
    X 50000 x 8192 with log-normal(0,1) column scales, tau = 1024, and X 200000 x 4096 with
    log-normal(0,2) columns and 5% correlated ones, tau = 512, both primal. Checked: the
    third sketch bit-exact; 96 sampled rows of its AS against the oracle's FP64 rows within
    the BF16/FP32 bound; G^{-1} inverting the sketched matrix the GPU formed, within the
    bound of an inverse through Cholesky (Higham, Sec. 14.3); and after 20 iterations the
    refreshed residual and the previous one equal to A x - b from the oracle's FP64 system,
    within the dot-product bound of the two summation orders (each side's error in
    Z (Z^T x) + lambda x - Z y is within 2 gamma_n (|Z| (|Z^T| |x| + |y|) + lambda |x|), as
    d < n)."""
    import torch
    p = getattr(inputs, workload)()
    n, d = p.X.shape
    print(f"[mixed full size] {workload} n={n} d={d} tau={tau}", flush=True)
    X = torch.from_numpy(p.X).cuda()
    y = torch.from_numpy(p.y).cuda()
    stream = torch.cuda.current_stream().cuda_stream
    S = rs.Solver(X, y, p.lam, tau=tau, sketch="subsample", form="primal", tol=0.0, seed=1,
                  precision="mixed", stream=stream)
    S.step(3)
    rows, cols, _ = S.last_sketch()
    exp = osk.draw_subsample(1, 0, 2, d, tau)
    assert np.array_equal(rows, exp.rows) and np.array_equal(cols, exp.cols)
    AS, Gi = S.products()
    system = ridge_system(p.X, p.y, p.lam, "primal")
    Z = system.Z  # d x n, FP64
    C = exp.rows
    rng = np.random.default_rng(11)
    idx = np.unique(np.concatenate([rng.choice(d, 64, replace=False), C[:32]]))
    ZC = Z[C]
    AS_or = Z[idx] @ ZC.T
    AS_or[idx[:, None] == C[None, :]] += p.lam
    bound = (2 * U_BF16 + n * U_FP32) * (np.abs(Z[idx]) @ np.abs(ZC).T) + 1e-30
    err = np.abs(AS[idx] - AS_or)
    assert np.all(err <= bound), float((err / bound).max())
    Gm = np.tril(AS[C]) + np.tril(AS[C], -1).T
    kappa = np.linalg.cond(Gm)
    assert np.abs(Gi @ Gm - np.eye(tau)).max() <= 4 * tau * 2.0 ** -53 * kappa, kappa
    del ZC, AS, Gi, Gm
    S.step(20 - S.k)
    x, xp, r, rp = S.state()
    gamma_n = n * 2.0 ** -53 / (1 - n * 2.0 ** -53)
    for xx, rr in ((x, r), (xp, rp)):
        true = system.matvec(xx) - system.b
        mag = np.abs(Z) @ (np.abs(system.X) @ np.abs(xx) + np.abs(p.y)) + p.lam * np.abs(xx)
        assert np.all(np.abs(rr - true) <= 4 * gamma_n * mag)
    S.close()
