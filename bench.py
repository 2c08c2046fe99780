#!/usr/bin/env python3
"""Benchmark: time to relative residual 1e-6 of sketch-and-project on one MI355X.

A step is one full solve (x^0 = 0 until ||r^k|| / ||r^0|| <= 1e-6). The default workload is the
largest one that fits one GPU: dense X 200000 x 4096 (FP32, log-normal(0,2) column scales, 5% of
the columns correlated at 0.9 with a random partner), lambda = 1e-2, primal form, subsample
sketch tau = 512 whose coordinates come from the learned proposal (an MLP trained on traces of
200 seeded uniform solves before the timed region), BF16 products with FP32 accumulation, FP64
factorisations and an FP64 residual refresh every 20 iterations, heuristic momentum. The timed
steps are the held-out seeds 201, 202, ...; the same seeds are also solved with uniform sampling
(BF16) and by the plain FP64 solver (uniform sampling, FP64 products), the tuned-vs-plain
comparison. --workload selects the other workloads (the sparse count-sketch workload, CSR
100000 x 20000 at 0.1%, tau = 500: sparse_count). The data and its device layouts stay resident
in HBM.

Prints one JSON line with the metric, a roofline entry for the kernel that dominates the solve
(algorithmic flops or bytes per launch over its HIP-event duration, on the stream it runs on),
a per-kernel breakdown and the CPU oracle's time on a bounded sample.
"""
import argparse
import hashlib
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0       # MI355X HBM3E
FP64_PEAK_TFS = 78.6        # MI355X FP64 (vector and matrix)
BF16_PEAK_TFS = 2500.0      # MI355X dense BF16 MFMA

WORKLOADS = {
    "sparse_count": dict(kind="csr", gen="sparse_csr", sketch="count", tau=500, sub_k=0, precision="fp64",
                         name="csr_100000x20000_density0.001_count_tau500_primal"),
    "sparse_count_dual": dict(kind="csr", gen="sparse_csr", sketch="count", tau=500, sub_k=0, precision="fp64",
                              form="dual", fixed_iters=200,
                              name="csr_100000x20000_density0.001_count_tau500_dual_200iterations"),
    "sparse_subcount": dict(kind="csr", gen="sparse_csr", sketch="subcount", tau=500, sub_k=4,
                            precision="fp64",
                            name="csr_100000x20000_density0.001_subcount_s2000_tau500_primal"),
    "sparse_count_mixed": dict(kind="csr", gen="sparse_csr", sketch="count", tau=500, sub_k=0, precision="mixed",
                               name="csr_100000x20000_density0.001_count_tau500_primal_fp32AS_refresh20"),
    "sparse_subcount_mixed": dict(kind="csr", gen="sparse_csr", sketch="subcount", tau=500, sub_k=4,
                                  precision="mixed",
                                  name="csr_100000x20000_density0.001_subcount_s2000_tau500_primal_fp32AS_refresh20"),
    "dense_primal": dict(kind="dense", gen="dense_primal", sketch="subsample", tau=50, sub_k=0,
                         precision="fp64", name="dense_2000x500_subsample_tau50_primal"),
    "dense_mixed": dict(kind="dense", gen="dense_mixed", sketch="subsample", tau=1024, sub_k=0,
                        precision="mixed",
                        name="dense_50000x8192_lognormal1_subsample_tau1024_primal_bf16_refresh20"),
    "dense_mixed_fp64": dict(kind="dense", gen="dense_mixed", sketch="subsample", tau=1024, sub_k=0,
                             precision="fp64",
                             name="dense_50000x8192_lognormal1_subsample_tau1024_primal_fp64"),
    "dense_learned": dict(kind="dense", gen="dense_learned", sketch="subsample", tau=512, sub_k=0,
                          precision="mixed",
                          name="dense_200000x4096_lognormal2_corr0.05_subsample_tau512_primal_bf16_learned"),
    "kernel_california": dict(kind="kernel", gen="kernel_california", sketch="subsample", tau=5160, sub_k=0,
                              precision="fp64",
                              name="kernel_rbf_20640x8_sigma0.5_lambda1e-6_subsample_tau5160"),
    "kernel_california_mixed": dict(kind="kernel", gen="kernel_california", sketch="subsample", tau=5160, sub_k=0,
                                    precision="mixed",
                                    name="kernel_rbf_20640x8_sigma0.5_lambda1e-6_subsample_tau5160_bf16_refresh20"),
    "accel_grid": dict(kind="kernel", sketch="subsample", tau=158, sub_k=0, precision="fp64",
                       name="accel_grid_kernel_rbf_2000_sigma0.5_lambda1/n_tau158_tol1e-4"),
    "sketch_compare": dict(kind="kernel", sketch="subsample", tau=126, sub_k=0, precision="fp64",
                           name="sketches_kernel_boston_506x13_tau126_and_dense_2000x500_tau50"),
    "batched": dict(kind="batch", precision="fp64",
                    name="batched_64problems_n2000-40000_d500-8000_half_csr0.005_16lambda_4rhs"),
}


def kernel_source_sha(files):
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, "paper_2105_05565_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def algorithmic_bytes(cls, wl, n, d, nnz, m, K, tau, nsel, a_nnz=0, slots=1):
    """Minimum HBM bytes one sketch (iteration) needs in each kernel class (FP64 layouts)."""
    if cls == "as":
        if wl["kind"] == "csr":
            # CSR of Z and of Z^T (FP32 value + int32 column each) read once, row pointers,
            # bucket map, AS written once (FP64, or FP32 in mixed precision), G = S^T A S written
            # once (FP64)
            elt = 4 if wl["precision"] == "mixed" else 8
            return 2 * nnz * 8 + (m + 1) * 8 + (K + 1) * 8 + m * 4 + m * tau * elt + tau * tau * 8
        if wl.get("gram"):
            # formed A: the tau gathered entries of each of its m rows read, AS written
            elt = 4 if wl["precision"] == "mixed" else 8
            return 2 * m * tau * elt + tau * 4
        # dense subsample: Z read once (m x K) + gathered rows (tau x K) + AS written; kernel
        # ridge also reads the gathered columns K[:, C] for the shift lambda K S
        elt = 2 if wl["precision"] == "mixed" else 8
        shift = m * tau * 8 if wl["kind"] == "kernel" else 0
        return m * K * elt + tau * K * elt + m * tau * (4 if wl["precision"] == "mixed" else 8) + shift
    if cls == "g":
        # G = S^T AS from the member rows of AS (FP64, or FP32 in mixed precision), their bucket
        # codes and indices, the bucket offsets; G written
        elt = 4 if wl["precision"] == "mixed" else 8
        return nsel * tau * elt + nsel * (4 + 4) + (tau + 1) * 4 + tau * tau * 8
    if cls == "update":
        # AS read, bucket map, x^k, x^{k-1}, r^k, r^{k-1} read, two vectors written, delta
        return m * tau * (4 if wl["precision"] == "mixed" else 8) + m * 4 + 4 * m * 8 + 2 * m * 8 + tau * 8
    if cls == "delta":
        return tau * tau * 8 + nsel * (4 + 4 + 8) + tau * 4 + tau * 8
    if cls == "sketch":
        return m * (8 + 4) + nsel * 4 + (tau + 1) * 4
    if cls == "chol":
        return 3 * tau * tau * 8
    if cls == "iters":
        return (algorithmic_bytes("delta", wl, n, d, nnz, m, K, tau, nsel)
                + algorithmic_bytes("update", wl, n, d, nnz, m, K, tau, nsel))
    return 0


def make_problem(wl):
    from paper_2105_05565_amd import inputs
    return getattr(inputs, wl["gen"])()


def cpu_baseline(p, wl, gpu_iters_median, sample_s, momentum="heuristic", threads=1):
    """The oracle on the first iterations of the seed-1 solve, with `threads` BLAS threads
    (None: all of the host's)."""
    from threadpoolctl import threadpool_limits

    from oracle.problem import ridge_system
    from oracle.solver import Options, init_state, step
    with threadpool_limits(limits=threads):
        if wl["kind"] == "kernel":
            from oracle.problem import kernel_system
            system = kernel_system(p.P, p.y, p.lam, p.sigma)
        else:
            system = ridge_system(p.X, p.y, p.lam, wl.get("form", "primal"))
        st = init_state(system)
        opts = Options(sketch=wl["sketch"], tau=wl["tau"], sum_size=wl["sub_k"], momentum=momentum,
                       seed=1, tol=1e-6)
        t0 = time.perf_counter()
        while (st.k == 0 or time.perf_counter() - t0 < sample_s) and st.history[-1] > 1e-6:
            step(system, st, opts)
        el = time.perf_counter() - t0
        from threadpoolctl import threadpool_info
        blas = max([int(i.get("num_threads", 1)) for i in threadpool_info()] or [1])
    per_iter = el / st.k
    # the dense oracle's products are BLAS GEMMs (all the threads the limit allows); the CSR
    # oracle's products are scipy sparse products, which run on one thread whatever the limit
    cores = 1 if wl["kind"] == "csr" else blas
    return {"value": per_iter * gpu_iters_median, "unit": "s", "cores": cores, "kind": "oracle",
            "sample": (f"extrapolated: first {st.k} iterations of the seed-1 solve on the full workload "
                       f"({el:.1f} s, {per_iter:.3f} s/iteration, {cores} thread(s)) times the GPU's median "
                       f"iteration count {gpu_iters_median:.0f}; sketches are bit-identical"),
            "s_per_iter": per_iter}


def kernel_table(prof, wl, workload, n, d, nnz, m, K, nsel, total, a_nnz=0):
    """Per-class timings (HIP events) with algorithmic bytes, and the roofline entry of the
    class that dominates the timed solves."""
    kernels = {}
    for cls, v in prof.items():
        if v["launches"] == 0:
            continue
        spl = v["slots"] / v["launches"]
        b = algorithmic_bytes(cls, wl, n, d, nnz, m, K, wl["tau"], nsel, a_nnz, spl) * spl
        avg_ms = v["ms"] / v["launches"]
        kernels[cls] = {"total_ms": round(v["ms"], 3), "launches": v["launches"],
                        "slots_per_launch": round(v["slots"] / v["launches"], 2),
                        "avg_ms": round(avg_ms, 5), "alg_bytes_per_launch": int(b),
                        "gbs": round(b / (avg_ms * 1e-3) / 1e9, 1) if avg_ms > 0 else None,
                        "share_of_timed": round(v["ms"] / (total * 1e3), 4)}
    dom = max((c for c in kernels if c != "iters"), key=lambda c: kernels[c]["total_ms"])
    kd = kernels[dom]
    achieved = kd["gbs"]
    def arows_name():
        # which A-rows kernel the library picks: 16-bit bucket map in LDS, packed 10-bit map, or global map
        if 2 * m + 64 * wl["tau"] <= 96 * 1024 and wl["tau"] < 16383:
            return "k_as_arows_lds"
        if wl["tau"] <= 511 and (m + 2) // 3 * 4 + 32 * wl["tau"] <= 156 * 1024:
            return "k_as_arows_packed"
        return "k_as_arows"
    as_name = (arows_name() if a_nnz else "k_as_sparse_bucket") if wl["kind"] == "csr" \
        else ("k_gram_gather" if wl.get("gram") else wl.get("as_kernel", "k_as_dense_f64_128"))
    roofline = {"kernel": {"as": as_name, "g": "k_g_from_as",
                           "update": "k_update", "chol": "k_chol_inverse", "delta": "k_delta",
                           "iters": "k_delta+k_update sequence",
                           "sketch": "k_sketch_count" if wl["sketch"] == "count" else "k_sketch_select"}[dom],
                "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4) if achieved else None, "traffic": None,
                "alg_bytes_per_launch": kd["alg_bytes_per_launch"], "avg_launch_ms": kd["avg_ms"]}
    if wl["kind"] in ("dense", "kernel") and dom == "as" and not wl.get("gram"):
        # a dense sketch takes two products per sketch (T = Z^T S, then Z T)
        flops = 2.0 * m * wl["tau"] * K * kd["slots_per_launch"] * wl.get("as_products", 1)
        tfs = flops / (kd["avg_ms"] * 1e-3) / 1e12
        peak = BF16_PEAK_TFS if wl["precision"] == "mixed" else FP64_PEAK_TFS
        if wl["precision"] == "mixed":
            # the library's K split for launches with fewer 256 x 256 tiles than compute units
            # (bf16_split_factor): doubling while tiles * split * 2 <= 256 and every K range
            # keeps >= 32 stages of 64; the split form adds an in-order reduction launch
            ntiles = -(-m // 256) * -(-int(kd["slots_per_launch"] * wl["tau"]) // 256)
            nk, split = -(-K // 64), 1
            while ntiles * split * 2 <= 256 and nk >= split * 2 * 32:
                split *= 2
            mixed_name = "k_as_dense_bf16_split+k_splitk_reduce" if split > 1 else "k_as_dense_bf16"
        roofline.update({"kernel": mixed_name if wl["precision"] == "mixed" else as_name,
                         "bound": "mfma", "achieved": round(tfs, 1), "peak": peak, "unit": "TFLOP/s",
                         "frac": round(tfs / peak, 4), "alg_flops_per_launch": flops,
                         "hbm_gbs_algorithmic": kd["gbs"]})
    if dom == "chol":
        # explicit inverse of each tau x tau sketched system: factorisation tau^3 / 3, triangular
        # inverse tau^3 / 3, U U^T tau^3 / 3 flop on FP64 MFMA; the device-wide tiled kernels serve
        # tau >= 128 with fewer than 128 sketches per launch
        tau = wl["tau"]
        ldg = (tau + 63) // 64 * 64
        flops = float(tau) ** 3 * kd["slots_per_launch"]
        tfs = flops / (kd["avg_ms"] * 1e-3) / 1e12
        tiled = ldg >= 128 and kd["slots_per_launch"] < 128
        # the library's tiled form (chol_multi_mode): fused steps, panel + update, or the
        # factor steps followed by the inverse-by-distance and U U^T chains
        nt, ns = ldg // 64, kd["slots_per_launch"]
        tiled_name = ("k_chol_assemble+k_chol_diag0+k_chol_step" if ns * nt * nt <= 512 else
                      "k_chol_assemble+k_chol_diag0+k_chol_panel+k_chol_narrow+k_chol_update" if ns * nt ** 3 <= 4e6 else
                      "k_chol_assemble+k_chol_diag0+k_chol_panel+k_chol_narrow+k_chol_update+k_chol_ll_inverse+k_chol_lauum")
        roofline.update({"kernel": tiled_name if tiled else "k_chol_inverse",
                         "bound": "mfma", "achieved": round(tfs, 1), "peak": FP64_PEAK_TFS, "unit": "TFLOP/s",
                         "frac": round(tfs / FP64_PEAK_TFS, 4), "alg_flops_per_launch": flops,
                         "hbm_gbs_algorithmic": kd["gbs"]})
    traffic_file = os.path.join(ROOT, "profiles",
                                f"traffic_{roofline['kernel'].replace('+', '_')}_{workload}.json")
    if os.path.exists(traffic_file):
        tf = json.load(open(traffic_file))
        src = {"k_as_sparse_bucket": ["k_sparse.hip"], "k_update": ["k_update.hip"],
               "k_as_dense_f64_128": ["k_dense.hip"], "k_as_arows_lds": ["k_sparse_a.hip"],
               "k_as_dense_bf16": ["k_dense_bf16.hip"],
               "k_as_dense_bf16_split+k_splitk_reduce": ["k_dense_bf16.hip"],
               "k_g_from_as": ["k_sparse_a.hip"]
               }.get(roofline["kernel"], [])
        if src and tf.get("source_sha") == kernel_source_sha(src):
            roofline["traffic"] = tf["hbm_bytes_per_launch_scaled"] * kd["slots_per_launch"] / tf["slots_per_launch"]

    return kernels, roofline


def batch_weights(pr):
    """Relative per-iteration work of one batched problem (for extrapolating samples)."""
    m, K = min(pr["n"], pr["d"]), max(pr["n"], pr["d"])
    if pr["kind"] == "dense":
        return 2.0 * m * K * pr["tau"]
    return float(pr["X"].nnz) * pr["tau"] + m * pr["tau"]


def main_batched(args):
    import numpy as np
    import torch

    from paper_2105_05565_amd import inputs, rs

    wl = WORKLOADS["batched"]
    torch.cuda.set_device(0)
    print(f"[bench] generating {wl['name']}", file=sys.stderr, flush=True)
    probs = inputs.batched(scale=args.scale, cap_factor=args.cap_factor)
    stream = torch.cuda.current_stream().cuda_stream
    t0 = time.perf_counter()
    mixed = args.batch_precision == "mixed"
    B = rs.Batch(probs, tol=1e-6, seed=1, autotune=True, stream=stream, max_iter=args.max_iter,
                 momentum=args.momentum, precision=args.batch_precision)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    tune = B.tuning()
    print(f"[bench] batch built in {setup_s:.1f} s, tuning {tune}", file=sys.stderr, flush=True)
    for w in range(args.warmup):
        B.reset(10000 + w)
        B.solve()
        print(f"[bench] warmup {w} done: {B.k} lock-step iterations", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    times, conv, steps_k = [], [], []
    for i in range(args.steps):
        ti = time.perf_counter()
        B.reset(i + 1)
        st, rep = B.solve()
        times.append(time.perf_counter() - ti)
        conv.append(rep.converged / rep.solves)
        steps_k.append(rep.iters)
        print(f"[bench] step {i}: {rep.iters} lock-step iterations, {rep.converged}/{rep.solves} "
              f"converged, {times[-1]:.2f} s", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    total = time.perf_counter() - t_start
    # iterations per slot of the last solve (cap for slots that did not converge)
    slot_iters = []
    for p, pr in enumerate(probs):
        stop, _ = B.slots(p)
        slot_iters.append(np.where(stop >= 0, stop, pr["max_iter"]))
    n_solves = sum(len(v) for v in slot_iters)
    solve_iters = int(sum(int(v.sum()) for v in slot_iters))
    dense_flops = sum(batch_weights(pr) for pr in probs if pr["kind"] == "dense")
    T = total / args.steps
    peak = BF16_PEAK_TFS if mixed else FP64_PEAK_TFS
    roofline = {"kernel": "k_as_dense_bf16_tab" if mixed else "k_as_dense_f64_tab", "bound": "mfma",
                "achieved": None, "peak": peak,
                "unit": "TFLOP/s", "frac": None, "traffic": None,
                "alg_flops_per_launch": dense_flops, "avg_launch_ms": tune["dense_ms"],
                "note": "launch duration timed with HIP events by the tuner on the first iteration "
                        "(every problem active)"}
    if tune["dense_ms"] > 0:
        tfs = dense_flops / (tune["dense_ms"] * 1e-3) / 1e12
        roofline.update({"achieved": round(tfs, 2), "frac": round(tfs / peak, 4)})

    # converged fraction and median stop iteration per lambda (slot j = l * nrhs + q)
    nl = len(probs[0]["lambdas"])
    nrhs = probs[0]["y"].shape[1]
    per_lambda = []
    for l in range(nl):
        stops = np.concatenate([B.slots(p)[0][l * nrhs:(l + 1) * nrhs] for p in range(len(probs))])
        conv_l = stops >= 0
        per_lambda.append({"lambda": float(probs[0]["lambdas"][l]), "converged_fraction": round(float(conv_l.mean()), 4),
                           "median_stop_iteration": float(np.median(stops[conv_l])) if conv_l.any() else None})
    B.close()

    fp64_batch = None
    if mixed:
        # the same batch with FP64 products (and no refresh), one solve of the first timed seed
        print("[bench] the FP64 batch, one solve", file=sys.stderr, flush=True)
        F = rs.Batch(probs, tol=1e-6, seed=1, autotune=True, stream=stream, max_iter=args.max_iter,
                     momentum=args.momentum)
        torch.cuda.synchronize()
        ti = time.perf_counter()
        st_f, rep_f = F.solve()
        torch.cuda.synchronize()
        fp64_batch = {"seconds": round(time.perf_counter() - ti, 3), "lock_step_iters": rep_f.iters,
                      "converged_fraction": round(rep_f.converged / rep_f.solves, 4), "seed": 1,
                      "mixed_seconds_same_seed": round(times[0], 3)}
        F.close()

    # the plain FP64 single-solve path: full solves (to 1e-6 or the problem's cap) of a stratified
    # subset -- 8 problems spread over the per-iteration work (4 dense, 4 CSR), 4 lambdas each,
    # right-hand side 0 -- timed one by one; the seconds per unit of work and iteration of each kind
    # scale to every slot of the batch with the iterations that slot took there
    order = sorted(range(len(probs)), key=lambda p: batch_weights(probs[p]))
    subset = [p for kind in ("dense", "csr") for p in
              [q for q in order if probs[q]["kind"] == kind][::8][:4]]
    lam_idx = [0, nl // 3, (2 * nl) // 3, nl - 1]
    rate = {"dense": [0.0, 0.0], "csr": [0.0, 0.0]}  # seconds, work * iterations
    full = []
    for p in subset:
        pr = probs[p]
        for l in lam_idx:
            S = rs.Solver(pr["X"], pr["y"][:, 0], float(pr["lambdas"][l]), tau=pr["tau"],
                          sketch="subsample" if pr["kind"] == "dense" else "count", tol=1e-6, seed=1,
                          problem_id=p, max_iter=pr["max_iter"], stream=stream, momentum=args.momentum)
            torch.cuda.synchronize()
            ts = time.perf_counter()
            _, st1, rep1 = S.solve()
            torch.cuda.synchronize()
            el = time.perf_counter() - ts
            S.close()
            rate[pr["kind"]][0] += el
            rate[pr["kind"]][1] += batch_weights(pr) * rep1.iters
            full.append({"problem": p, "kind": pr["kind"], "lambda": float(pr["lambdas"][l]), "seconds": round(el, 4),
                         "iterations": rep1.iters, "converged": st1 == rs.RS_OK})
    plain = 0.0
    for pr, it in zip(probs, slot_iters):
        sec, work = rate[pr["kind"]]
        plain += float(it.sum()) * batch_weights(pr) * sec / work

    out = {
        "metric": "time-to-rel-residual 1e-6", "value": round(T, 4), "unit": "s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(T * 1e3, 1),
        "higher_is_better": False, "scaling": "weak", "vs_baseline": None, "dtype": "bf16" if mixed else "f64",
        "data": "synthetic",
        "config": {"workload": wl["name"], "problems": len(probs), "lambdas": 16, "rhs": 4,
                   "precision": args.batch_precision, "refresh_every": 20 if mixed else None,
                   "solves": n_solves, "dense": sum(pr["kind"] == "dense" for pr in probs),
                   "tau_rule": "64 round(m^(2/3) / 64) clamped to [64, 512]", "cap": f"{args.cap_factor:g} m / tau",
                   "tol": 1e-6, "momentum": args.momentum, "graph_iters": tune["graph_iters"]},
        "converged_fraction": round(statistics.median(conv), 4),
        "lock_step_iters_median": statistics.median(steps_k),
        "solve_iterations": solve_iters,
        "solve_iterations_per_s": round(solve_iters / T, 1),
        "time_s_all": [round(t, 4) for t in times],
        "setup_s": round(setup_s, 2),
        "tuning": tune,
        "roofline": roofline,
        "per_lambda": per_lambda,
        "fp64_batch": fp64_batch,
        "plain_fp64_single_solves": {
            "value": round(plain, 1), "unit": "s",
            "sample": (f"{len(full)} full single solves (to 1e-6 or the cap) of a stratified subset: problems "
                       f"{subset} (4 dense, 4 CSR, spread over the per-iteration work) x lambdas "
                       f"{[float(probs[0]['lambdas'][l]) for l in lam_idx]} x right-hand side 0; their seconds per "
                       "unit of work and iteration, per kind, scaled by every slot's work and the iterations it "
                       "took in the batch"),
            "full_solves": full},
    }
    if not args.no_cpu_baseline:
        print("[bench] timing the CPU oracle on a bounded sample", file=sys.stderr, flush=True)
        from threadpoolctl import threadpool_limits

        from oracle.problem import ridge_system
        from oracle.solver import Options, init_state, step
        per = {}
        with threadpool_limits(limits=1):
            for p in (0, len(probs) // 2):
                pr = probs[p]
                system = ridge_system(pr["X"], pr["y"][:, 0], float(pr["lambdas"][8]))
                st = init_state(system)
                opts = Options(sketch="subsample" if pr["kind"] == "dense" else "count", tau=pr["tau"],
                               momentum=args.momentum, seed=1, problem_id=p, tol=0.0)
                ts = time.perf_counter()
                while st.k == 0 or (time.perf_counter() - ts < args.cpu_sample_s / 2 and st.k < 50):
                    step(system, st, opts)
                per[pr["kind"]] = ((time.perf_counter() - ts) / st.k, batch_weights(pr), st.k)
        est = 0.0
        for pr, it in zip(probs, slot_iters):
            t_it, w0, _ = per[pr["kind"]]
            est += float(it.sum()) * t_it * batch_weights(pr) / w0
        out["cpu_baseline"] = {
            "value": round(est, 1), "unit": "s", "cores": 1, "kind": "oracle",
            "sample": (f"{per['dense'][2]} iterations of one solve of problem 0 (dense, "
                       f"{per['dense'][0]:.3f} s/iteration) and {per['csr'][2]} of problem 32 (CSR, "
                       f"{per['csr'][0]:.4f} s/iteration), 1 thread, scaled by per-problem work to the "
                       f"{solve_iters} solve-iterations of the batch")}
    print(json.dumps(out))


def main_learned(args):
    """Learned proposal: train on traces of uniform solves (seeds 1..N), then time held-out
    solves (seeds 201..) with the learned proposal; uniform, A_jj / Tr A and plain FP64
    solves of the same held-out seeds are reported beside it."""
    import numpy as np
    import torch

    from paper_2105_05565_amd import rs

    wl = WORKLOADS["dense_learned"]
    torch.cuda.set_device(0)
    print(f"[bench] generating {wl['name']}", file=sys.stderr, flush=True)
    p = make_problem(wl)
    n, d = p.X.shape
    X = torch.from_numpy(p.X).cuda()
    y = torch.from_numpy(p.y).cuda()
    stream = torch.cuda.current_stream().cuda_stream
    tau = wl["tau"]
    kw = dict(tau=tau, sketch="subsample", form="primal", momentum="heuristic", tol=1e-6, precision="mixed",
              max_iter=args.max_iter, stream=stream)

    t0 = time.perf_counter()
    U = rs.Solver(X, y, p.lam, trace_every=2, trace_capacity=400000, lookahead=8, **kw)
    tr_iters = []
    for sd in range(1, args.train_solves + 1):
        U.reset(sd)
        _, _, rep = U.solve()
        tr_iters.append(rep.iters)
        if sd % max(1, args.train_solves // 20) == 0:
            print(f"[bench] trace solve {sd}/{args.train_solves}: {rep.iters} iterations", file=sys.stderr,
                  flush=True)
    T = rs.Trainer(tau, init_seed=1)
    T.add_traces(U)
    records = T.records
    U.close()
    # the listwise cross-entropy over all records before and after training, and its floor
    # (the mean entropy of the records' targets, reached only if softmax(s) matched them)
    loss_before, loss_floor = T.evaluate()
    losses = T.fit(10, batch=16, lr=1e-3, shuffle_seed=7)
    loss_after, _ = T.evaluate()
    params = T.params()
    T.close()
    train_s = time.perf_counter() - t0
    print(f"[bench] trained on {records} records from {args.train_solves} solves in {train_s:.1f} s; "
          f"loss {loss_before:.4f} -> {loss_after:.4f} (floor {loss_floor:.4f}); "
          f"epoch losses {[round(v, 4) for v in losses]}", file=sys.stderr, flush=True)

    look = args.lookahead if args.lookahead > 0 else 2

    def run(sampler, seeds, profile=0, **extra):
        S = rs.Solver(X, y, p.lam, sampler=sampler, profile=profile, **{**kw, **extra})
        if sampler == "learned":
            S.set_sampler_params(params)
        times, iters, rels, sts = [], [], [], []
        for sd in seeds:
            S.reset(sd)
            torch.cuda.synchronize()
            ti = time.perf_counter()
            _, st, rep = S.solve()
            times.append(time.perf_counter() - ti)
            iters.append(rep.iters)
            rels.append(rep.rel_res)
            sts.append(st)
        prof = S.profile() if profile else None
        S.close()
        return times, iters, rels, sts, prof

    # the timed solves record HIP events around the product launches only (profile 3): the
    # roofline needs those, and every event in the stream costs a few microseconds; the
    # breakdown over all phases comes from an untimed solve afterwards (profile 1)
    S = rs.Solver(X, y, p.lam, sampler="learned", profile=3, lookahead=look, **kw)
    S.set_sampler_params(params)
    for w in range(args.warmup):
        S.reset(10000 + w)
        S.solve()
    S.profile(clear=True)
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    times, iters, rels_true = [], [], []
    for i in range(args.steps):
        ti = time.perf_counter()
        S.reset(201 + i)
        _, st, rep = S.solve()
        times.append(time.perf_counter() - ti)
        iters.append(rep.iters)
        rels_true.append(rep.rel_res_true)
        print(f"[bench] step {i}: {rep.iters} iterations, {times[-1]*1e3:.1f} ms, rel {rep.rel_res:.2e}",
              file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    total = time.perf_counter() - t_start
    prof = S.profile()
    S.close()
    T_step = total / args.steps
    m, K = d, n
    kernels, roofline = kernel_table(prof, wl, "dense_learned", n, d, n * d, m, K, tau, total)
    B = rs.Solver(X, y, p.lam, sampler="learned", profile=1, lookahead=look, **kw)
    B.set_sampler_params(params)
    B.reset(201)
    torch.cuda.synchronize()
    tb = time.perf_counter()
    B.solve()
    torch.cuda.synchronize()
    tb = time.perf_counter() - tb
    breakdown, _ = kernel_table(B.profile(), wl, "dense_learned", n, d, n * d, m, K, tau, tb)
    B.close()

    seeds = list(range(201, 201 + args.steps))
    print("[bench] uniform sampling, BF16 products, same seeds", file=sys.stderr, flush=True)
    ut, ui, ur, _, _ = run("uniform", seeds)
    print("[bench] A_jj / Tr A sampling, one seed", file=sys.stderr, flush=True)
    dt, di, dr, dst, _ = run("diag", seeds[:1], max_iter=min(args.max_iter, 3000))
    nf = max(1, min(args.fp64_solves, len(seeds)))
    print(f"[bench] plain FP64 solver (uniform sampling, FP64 products), {nf} seeds", file=sys.stderr,
          flush=True)
    pt, pi, pr_, pst, _ = run("uniform", seeds[:nf], precision="fp64")
    out = {
        "metric": "time-to-rel-residual 1e-6", "value": round(T_step, 6), "unit": "s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(T_step * 1e3, 3),
        "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
        "dtype": "bf16", "data": "synthetic",
        "config": {"workload": wl["name"], "n": n, "d": d, "form": "primal", "sketch": "subsample (learned proposal)",
                   "tau": tau, "lambda": p.lam, "momentum": "heuristic", "tol": 1e-6, "precision": "mixed",
                   "lookahead": look, "train_solves": args.train_solves, "held_out_seeds": seeds},
        "iters_median": statistics.median(iters),
        "time_s_all": [round(t, 4) for t in times],
        "phases_untimed_solve": {"seed": 201, "seconds": round(tb, 4), "per_phase": breakdown},
        # per result: ||A w - b|| / ||b|| of each timed solve's iterate, recomputed in FP64 from the data
        "final_rel_res_true_max": max(rels_true),
        "training": {"records": records, "seconds": round(train_s, 1),
                     "trace_solve_iters_median": statistics.median(tr_iters),
                     "epoch_loss": [round(v, 4) for v in losses],
                     "loss_before": round(loss_before, 4), "loss_after": round(loss_after, 4),
                     "loss_floor": round(loss_floor, 4)},
        "compare_same_seeds": {
            "uniform_mixed": {"seeds": len(seeds), "time_s_median": round(statistics.median(ut), 4),
                              "iters_median": statistics.median(ui)},
            "diag_mixed": {"seeds": 1, "time_s": round(dt[0], 4), "iters": di[0], "rel_res": dr[0],
                           "converged": dst[0] == 0, "cap": min(args.max_iter, 3000)},
            "uniform_fp64_plain": {"seeds": nf, "time_s_median": round(statistics.median(pt), 4),
                                   "iters_median": statistics.median(pi), "rel_res_max": max(pr_),
                                   "all_converged": all(s == 0 for s in pst),
                                   "learned_time_s_median_same_seeds": round(statistics.median(times[:nf]), 4)},
        },
        "speedup_vs_uniform_mixed": round(statistics.median(ut) / statistics.median(times), 3),
        "speedup_vs_plain_fp64": round(statistics.median(pt) / statistics.median(times[:nf]), 2),
        "roofline": roofline,
        "kernels": kernels,
    }
    if not args.no_cpu_baseline:
        print("[bench] timing the CPU oracle on a bounded sample", file=sys.stderr, flush=True)
        cb = cpu_baseline(p, wl, statistics.median(iters), args.cpu_sample_s, threads=None)
        cb.pop("s_per_iter")
        cb["sample"] = cb["sample"].replace("; sketches are bit-identical", "") + (
            "; the oracle's per-iteration cost with uniform sketches (the proposal's MLP adds ~1e-4 of "
            "an iteration's flops)")
        out["cpu_baseline"] = cb
    print(json.dumps(out))


def main_sketches(args):
    """The sketch comparison (Sec. 8.2): subsample, count, SubCount, Gaussian and SRHT sketches with
    the heuristic momentum on the kernel problem shaped like Boston (506 points, tau = 126,
    lambda = 1e-6) and on the dense workload (2000 x 500, tau = 50); median time and iterations
    to relative residual 1e-6 over seeded solves."""
    import numpy as np
    import torch

    from paper_2105_05565_amd import inputs, rs

    wl = WORKLOADS["sketch_compare"]
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream().cuda_stream
    runs = max(1, args.steps)
    kinds = ["subsample", "count", "subcount", "gaussian", "srht"]
    pb = inputs.kernel_boston()
    pd = inputs.dense_primal()
    problems = [("kernel_boston_506x13", pb, 126), ("dense_2000x500", pd, 50)]
    results = {}
    prof_first = None
    for pname, p, tau in problems:
        kern = pname.startswith("kernel")
        X = torch.from_numpy(p.P if kern else p.X).cuda()
        y = torch.from_numpy(p.y).cuda()
        res = {}
        for kind in kinds:
            kw = dict(kernel_sigma=p.sigma) if kern else dict(form="primal")
            S = rs.Solver(X, y, p.lam, tau=tau, sketch=kind, tol=1e-6, max_iter=args.max_iter, seed=1,
                          stream=stream, profile=1, **kw)
            S.reset(1000)
            S.solve()
            S.profile(clear=True)
            ts, its = [], []
            for r in range(runs):
                S.reset(r + 1)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                _, st, rep = S.solve()
                ts.append(time.perf_counter() - t0)
                its.append(rep.iters if st == rs.RS_OK else -1)
            prof = S.profile()
            S.close()
            res[kind] = {"median_s": round(statistics.median(ts), 6), "median_iters": statistics.median(its),
                         "all_converged": min(its) >= 0,
                         "ms_per_iter": round(1e3 * sum(ts) / max(1, sum(i for i in its if i > 0)), 4)}
            if prof_first is None and kind == "gaussian":
                prof_first = (prof, sum(ts), p, tau, kern)
            print(f"[bench] {pname} {kind}: {res[kind]}", file=sys.stderr, flush=True)
        results[pname] = res
    prof, total, p, tau, kern = prof_first
    n = p.P.shape[0]
    wl_k = dict(wl, tau=tau, as_products=2, as_kernel="k_gemm_f64")
    kernels, roofline = kernel_table(prof, wl_k, "sketch_compare", n, p.P.shape[1], n * p.P.shape[1], n, n, tau, total)
    T = results["kernel_boston_506x13"]["subsample"]["median_s"]
    out = {
        "metric": "time-to-rel-residual 1e-6 by sketch (value: subsample on the Boston-shaped kernel problem)",
        "value": T, "unit": "s", "n_gpus": 1, "steps": runs, "warmup": 1, "ms_per_step": round(T * 1e3, 4),
        "higher_is_better": False, "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": wl["name"], "momentum": "heuristic", "tol": 1e-6, "runs": runs},
        "results": results, "roofline_gaussian_kernel": roofline, "kernels_gaussian_kernel": kernels,
    }
    print(json.dumps(out))


def main_accel(args):
    """Accelerated method (Alg. 3) over a (mu, nu) grid with 0 < mu <= 1/nu <= 1, on the
    acceleration experiment's kernel problem (rows of a random sparse 2000 x 500 matrix,
    sigma = 0.5, lambda = 1/n) and on a clustered 2000-point kernel problem; median time to
    relative residual 1e-4 over seeded solves, against the plain method."""
    import numpy as np
    import torch

    from paper_2105_05565_amd import inputs, rs

    wl = WORKLOADS["accel_grid"]
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream().cuda_stream
    tol, tau, runs = 1e-4, wl["tau"], args.accel_runs
    cap = min(args.max_iter, 10000)  # cells that do not reach tol within it count as not converged
    mus = [1.0, 0.3, 0.1, 0.03, 0.01, 0.003, 0.001]
    nus = [1.0, 1.5, 2.0, 3.0, 5.0, 10.0, 30.0, 100.0, 300.0, 1000.0]
    grid = [(mu, nu) for mu in mus for nu in nus if nu <= 1.0 / mu]
    problems = [("sparse_2000x500_density0.25", inputs.accel_points()),
                ("clustered_2000x8", inputs.make_points(2000, 8, 1.0 / 2000, 0.5, seed=inputs.DATA_SEED_BASE + 8))]
    results = {}
    t_all = time.perf_counter()
    for pname, p in problems:
        P = torch.from_numpy(p.P).cuda()
        y = torch.from_numpy(p.y).cuda()

        def run(**kw):
            S = rs.Solver(P, y, p.lam, tau=tau, tol=tol, max_iter=cap, kernel_sigma=p.sigma,
                          stream=stream, **kw)
            S.reset(1000)
            S.solve()  # warmup
            ts, its = [], []
            for r in range(runs):
                S.reset(r + 1)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                _, st, rep = S.solve()
                ts.append(time.perf_counter() - t0)
                its.append(rep.iters if st == rs.RS_OK else -1)
            S.close()
            return statistics.median(ts), statistics.median(its), min(its)

        plain = run(momentum="none")
        heur = run(momentum="heuristic")
        cells = []
        for mu, nu in grid:
            t, it, worst = run(accel=(mu, nu))
            cells.append({"mu": mu, "nu": nu, "median_s": round(t, 6), "median_iters": it,
                          "all_converged": worst >= 0})
        ok = [c for c in cells if c["all_converged"]]
        best = min(ok, key=lambda c: c["median_s"]) if ok else None
        results[pname] = {"plain_s": round(plain[0], 6), "plain_iters": plain[1],
                          "heuristic_s": round(heur[0], 6), "heuristic_iters": heur[1],
                          "best": best, "grid": cells}
        print(f"[bench] {pname}: plain {plain[0]*1e3:.2f} ms / {plain[1]} it, best "
              f"{best}", file=sys.stderr, flush=True)
    total = time.perf_counter() - t_all

    # roofline of the product kernel from one profiled solve at the best cell (first problem)
    pname, p = problems[0]
    best = results[pname]["best"] or {"mu": 1.0, "nu": 1.0}
    S = rs.Solver(torch.from_numpy(p.P).cuda(), torch.from_numpy(p.y).cuda(), p.lam, tau=tau, tol=tol,
                  max_iter=cap, kernel_sigma=p.sigma, stream=stream, profile=1,
                  accel=(best["mu"], best["nu"]))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, _, rep = S.solve()
    torch.cuda.synchronize()
    prof = S.profile()
    S.close()
    n = p.P.shape[0]
    kernels, roofline = kernel_table(prof, wl, "accel_grid", n, p.P.shape[1], n * p.P.shape[1], n, n, tau,
                                     time.perf_counter() - t0)
    T = results[pname]["best"]["median_s"] if results[pname]["best"] else None
    out = {
        "metric": "time-to-rel-residual 1e-4, best (mu, nu) of the grid", "value": T, "unit": "s",
        "n_gpus": 1, "steps": runs, "warmup": 1, "ms_per_step": round(T * 1e3, 4) if T else None,
        "higher_is_better": False, "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": wl["name"], "n": n, "tau": tau, "sigma": p.sigma, "lambda": p.lam, "tol": tol,
                   "runs_per_cell": runs, "grid_cells": len(grid)},
        "problems": results, "grid_wall_s": round(total, 2), "roofline": roofline, "kernels": kernels,
    }
    if not args.no_cpu_baseline:
        from threadpoolctl import threadpool_limits

        from oracle.accel import accel_init, accel_step
        from oracle.problem import kernel_system
        from oracle.solver import Options
        with threadpool_limits(limits=1):
            system = kernel_system(p.P, p.y, p.lam, p.sigma)
            st = accel_init(system)
            opts = Options(sketch="subsample", tau=tau, seed=1, tol=tol)
            ts = time.perf_counter()
            while st.history[-1] > tol and st.k < cap and \
                    (st.k == 0 or time.perf_counter() - ts < args.cpu_sample_s):
                accel_step(system, st, opts, best["mu"], best["nu"])
            el = time.perf_counter() - ts
        per = el / st.k
        med_it = results[pname]["best"]["median_iters"] if results[pname]["best"] else st.k
        out["cpu_baseline"] = {"value": round(per * med_it, 4), "unit": "s", "cores": 1, "kind": "oracle",
                               "sample": f"{st.k} iterations of the seed-1 accelerated solve at the best cell "
                                         f"({el:.1f} s, 1 thread), scaled to the GPU's median iteration count "
                                         f"{med_it}"}
    print(json.dumps(out))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="dense_learned", choices=sorted(WORKLOADS))
    ap.add_argument("--lookahead", type=int, default=0)
    ap.add_argument("--momentum", default="heuristic", choices=["heuristic", "theory", "none"],
                    help="momentum schedule (the learned-sampler workload keeps the heuristic one)")
    ap.add_argument("--no-pipeline", action="store_true",
                    help="prepare each lookahead batch on the solver's stream (no overlap with iterating)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample-s", type=float, default=15.0)
    ap.add_argument("--sparse-route", default="auto", choices=["auto", "scatter", "arows"],
                    help="CSR workloads: how AS is formed (auto picks the rows of Z Z^T when they fit)")
    ap.add_argument("--accel-runs", type=int, default=10,
                    help="accel_grid: seeded solves per (mu, nu) cell")
    ap.add_argument("--train-solves", type=int, default=200,
                    help="dense_learned only: seeded uniform solves whose traces train the proposal")
    ap.add_argument("--fp64-solves", type=int, default=5,
                    help="dense_learned only: held-out seeds also solved by the plain FP64 solver")
    ap.add_argument("--scale", type=float, default=1.0,
                    help="batched workload only: shrink n and d (shape-alike smaller batch)")
    ap.add_argument("--cap-factor", type=float, default=100.0,
                    help="batched workload only: per-problem iteration cap cap_factor * m / tau")
    ap.add_argument("--max-iter", type=int, default=200000,
                    help="iteration cap per solve (a capped run reports per-iteration throughput)")
    ap.add_argument("--dense-route", default="products", choices=["products", "gram"],
                    help="subsample sketch on dense data: per-sketch MFMA products, or A formed once "
                         "at creation and its columns gathered per sketch")
    ap.add_argument("--batch-precision", default="mixed", choices=["mixed", "fp64"],
                    help="batched workload: BF16 products for the dense problems with an FP64 refresh every "
                         "20 iterations (then one FP64 batch solve is timed beside it), or FP64 throughout")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain device-to-device copy of 1 GiB five times (the known-size "
                         "reference for HBM traffic counters)")
    args = ap.parse_args()
    if args.calibrate_copy:
        import torch
        nbytes = 1 << 30
        src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": nbytes, "copy_bytes_written": nbytes, "dispatches": 5}))
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the solver is single-GPU.",
              file=sys.stderr)
        sys.exit(2)

    if args.workload == "batched":
        return main_batched(args)
    if args.workload == "dense_learned":
        return main_learned(args)
    if args.workload == "accel_grid":
        return main_accel(args)
    if args.workload == "sketch_compare":
        return main_sketches(args)

    import numpy as np
    import torch

    from paper_2105_05565_amd import rs

    wl = WORKLOADS[args.workload]
    if args.dense_route == "gram":
        if wl["kind"] == "csr" or wl["sketch"] != "subsample":
            raise SystemExit("--dense-route gram serves the subsample sketch on dense data or kernel ridge")
        wl = {**wl, "gram": True, "name": wl["name"] + "_formedA"}
    torch.cuda.set_device(0)
    print(f"[bench] generating {wl['name']}", file=sys.stderr, flush=True)
    p = make_problem(wl)
    kern = wl["kind"] == "kernel"
    n, d = p.P.shape if kern else p.X.shape
    if kern:
        X = torch.from_numpy(p.P).cuda()
        nnz = n * d
    elif wl["kind"] == "csr":
        X = (torch.from_numpy(p.X.indptr.astype(np.int64)).cuda(),
             torch.from_numpy(p.X.indices.astype(np.int32)).cuda(),
             torch.from_numpy(p.X.data).cuda(), (n, d))
        nnz = int(p.X.nnz)
    else:
        X = torch.from_numpy(p.X).cuda()
        nnz = n * d
    y = torch.from_numpy(p.y).cuda()
    stream = torch.cuda.current_stream().cuda_stream
    torch.cuda.synchronize()

    form = wl.get("form", "primal")
    fixed = wl.get("fixed_iters", 0)  # throughput at a fixed iteration count instead of time to 1e-6
    tol = 0.0 if fixed else 1e-6
    max_iter = fixed if fixed else args.max_iter
    t0 = time.perf_counter()
    S = rs.Solver(X, y, p.lam, tau=wl["tau"], sketch=wl["sketch"], form=form, momentum=args.momentum,
                  subcount_k=wl["sub_k"], tol=tol, max_iter=max_iter, seed=1,
                  precision=wl["precision"], lookahead=args.lookahead, profile=1, stream=stream,
                  sparse_route=args.sparse_route, pipeline=not args.no_pipeline,
                  kernel_sigma=p.sigma if kern else None, dense_route=args.dense_route)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    route, a_nnz = rs.rs_get_route(S.h)
    m, K = (n, n) if kern else ((n, d) if form == "dual" else (d, n))
    nsel = {"count": m, "subcount": wl["tau"] * max(wl["sub_k"], 1), "subsample": wl["tau"]}[wl["sketch"]]

    for w in range(args.warmup):
        S.reset(10000 + w)
        S.solve()
        print(f"[bench] warmup {w} done: {S.k} iterations", file=sys.stderr, flush=True)
    S.profile(clear=True)

    torch.cuda.synchronize()
    t_start = time.perf_counter()
    times, iters, rels_true = [], [], []
    for i in range(args.steps):
        ti = time.perf_counter()
        S.reset(i + 1)
        _, st, rep = S.solve()
        times.append(time.perf_counter() - ti)
        iters.append(rep.iters)
        rels_true.append(rep.rel_res_true)
        if st != rs.RS_OK and not fixed:
            print(f"[bench] step {i} did not converge: {rep.rel_res:.3e}", file=sys.stderr, flush=True)
        print(f"[bench] step {i}: {rep.iters} iterations, {times[-1]*1e3:.1f} ms", file=sys.stderr,
              flush=True)
    torch.cuda.synchronize()
    total = time.perf_counter() - t_start
    prof = S.profile()
    S.close()

    # one more solve, untimed, with every launch bracketed by events (per-launch breakdown);
    # skipped when one solve takes more than 10 s
    prof2 = {}
    if total / args.steps <= 10.0:
        S2 = rs.Solver(X, y, p.lam, tau=wl["tau"], sketch=wl["sketch"], form=form, momentum=args.momentum,
                       subcount_k=wl["sub_k"], tol=tol, max_iter=max_iter, seed=1,
                       precision=wl["precision"], lookahead=args.lookahead, profile=2, stream=stream,
                       sparse_route=args.sparse_route, pipeline=not args.no_pipeline,
                       kernel_sigma=p.sigma if kern else None, dense_route=args.dense_route)
        S2.solve()
        prof2 = S2.profile()
        S2.close()

    # context, untimed for the metric: the theoretical momentum rule (eq:parameterswitchtheory)
    # on the same workload and seeds, when a solve is short
    alt = None
    if args.momentum == "heuristic" and total / args.steps <= 5.0 and not fixed:
        S3 = rs.Solver(X, y, p.lam, tau=wl["tau"], sketch=wl["sketch"], form="primal", momentum="theory",
                       subcount_k=wl["sub_k"], tol=1e-6, max_iter=args.max_iter, seed=1,
                       precision=wl["precision"], lookahead=args.lookahead, stream=stream,
                       sparse_route=args.sparse_route, pipeline=not args.no_pipeline,
                       kernel_sigma=p.sigma if kern else None, dense_route=args.dense_route)
        S3.solve()
        t3, i3 = [], []
        for i in range(min(args.steps, 3)):
            S3.reset(i + 1)
            torch.cuda.synchronize()
            ti = time.perf_counter()
            _, st3, rep3 = S3.solve()
            torch.cuda.synchronize()
            t3.append(time.perf_counter() - ti)
            i3.append(rep3.iters if st3 == rs.RS_OK else -1)
        S3.close()
        alt = {"momentum": "theory", "time_s_median": round(statistics.median(t3), 6),
               "iters_median": statistics.median(i3), "solves": len(t3)}

    T = total / args.steps
    tot_iters = sum(iters)
    kernels, roofline = kernel_table(prof, wl, args.workload, n, d, nnz, m, K, nsel, total, a_nnz)
    solve_level = None
    if wl["kind"] == "csr":
        # the whole iteration's algorithmic bytes: CSR(Z) and CSR(Z^T) read (value + column),
        # AS written and read back by the update, G written, six iterate/residual vectors
        elt = 4 if wl["precision"] == "mixed" else 8
        per_it = 2 * nnz * 8 + 2 * m * wl["tau"] * elt + wl["tau"] ** 2 * 8 + 6 * m * 8
        gbs = per_it * tot_iters / total / 1e9
        solve_level = {"bytes_per_iteration": per_it, "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS,
                       "unit": "GB/s", "frac": round(gbs / HBM_PEAK_GBS, 4),
                       "us_per_iteration": round(total / tot_iters * 1e6, 2),
                       "floor_us_per_iteration": round(per_it / (HBM_PEAK_GBS * 1e9) * 1e6, 2)}

    metric, value, unit, hib = "time-to-rel-residual 1e-6", round(T, 6), "s", False
    if fixed:
        metric, value, unit, hib = f"iterations/s over {fixed} iterations", round(tot_iters / total, 1), "it/s", True
    out = {
        "metric": metric, "value": value, "unit": unit, "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(T * 1e3, 3),
        "higher_is_better": hib, "scaling": "weak", "vs_baseline": None,
        # CSR mixed precision sums in FP64 and stores AS in FP32; dense mixed multiplies BF16 on MFMA
        "dtype": "bf16" if wl["precision"] == "mixed" and wl["kind"] != "csr" else "f64",
        "data": "synthetic",
        "config": {"workload": wl["name"], "n": n, "d": d, "nnz": nnz, "form": "kernel" if kern else form,
                   "sketch": wl["sketch"], "tau": wl["tau"], "subcount_k": wl["sub_k"],
                   "lambda": p.lam, "momentum": args.momentum, "tol": tol,
                   "precision": wl["precision"], "max_iter": args.max_iter,
                   "sparse_route": {0: None, 1: "scatter", 2: "arows"}[route],
                   "a_nnz": a_nnz or None,
                   "pipeline": not args.no_pipeline and wl.get("sampler", "uniform") != "learned"},
        "iters_per_s": round(tot_iters / total, 1),
        "iters_median": statistics.median(iters),
        "time_s_quartiles": [round(q, 6) for q in statistics.quantiles(times, n=4)] if len(times) > 1 else times,
        # per result: ||A w - b|| / ||b|| of each timed solve's iterate, recomputed in FP64 from the data
        "final_rel_res_true_max": max(rels_true),
        "setup_s": round(setup_s, 4),
        "roofline": roofline,
        "solve_level_hbm": solve_level,
        "kernels": kernels,
        "other_momentum_untimed": alt,
        "kernels_per_launch_untimed": {c: {"avg_ms": round(v["ms"] / v["launches"], 5),
                                           "launches": v["launches"]}
                                       for c, v in prof2.items() if v["launches"]},
    }
    if not args.no_cpu_baseline:
        print("[bench] timing the CPU oracle on a bounded sample", file=sys.stderr, flush=True)
        cb = cpu_baseline(p, wl, statistics.median(iters), args.cpu_sample_s, args.momentum,
                          threads=1 if wl["kind"] == "csr" else None)
        per_iter = cb.pop("s_per_iter")
        if fixed:
            cb["value"], cb["unit"] = round(1.0 / per_iter, 3), "it/s"
        out["cpu_baseline"] = cb
    print(json.dumps(out))


if __name__ == "__main__":
    main()
