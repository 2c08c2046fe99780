"""CPU: bench.py's host-side bookkeeping (roofline arithmetic, kernel naming, traffic lookup,
the one-GPU guard), checked on synthetic HIP-event profiles without a device."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def _prof(**classes):
    prof = {c: {"launches": 0, "slots": 0, "ms": 0.0} for c in ("sketch", "as", "chol", "iters")}
    for c, (launches, slots, ms) in classes.items():
        prof[c] = {"launches": launches, "slots": slots, "ms": ms}
    return prof


def test_learned_workload_roofline_is_the_split_product_on_bf16_peak():
    wl = bench.WORKLOADS["dense_learned"]
    n, d = 200000, 4096
    # 21 product launches of 2 sketches at 1.5 ms each dominate the solve
    prof = _prof(**{"as": (21, 42, 31.5), "chol": (21, 42, 4.6), "sketch": (21, 42, 1.5), "iters": (21, 42, 3.3)})
    kernels, roof = bench.kernel_table(prof, wl, "dense_learned", n, d, n * d, d, n, 512, 0.0437)
    assert roof["kernel"] == "k_as_dense_bf16_split+k_splitk_reduce"  # 16 x 4 tiles: split over K
    flops = 2.0 * d * 512 * n * 2
    assert roof["alg_flops_per_launch"] == pytest.approx(flops)
    assert roof["achieved"] == pytest.approx(flops / 1.5e-3 / 1e12, abs=0.05)
    assert roof["peak"] == bench.BF16_PEAK_TFS and roof["unit"] == "TFLOP/s" and roof["bound"] == "mfma"
    assert roof["frac"] == pytest.approx(roof["achieved"] / bench.BF16_PEAK_TFS, abs=1e-4)
    assert kernels["as"]["share_of_timed"] == pytest.approx(31.5 / 43.7, abs=1e-4)
    # HBM traffic: the committed counter summary, only while it was taken on the current source
    tf = json.load(open(os.path.join(ROOT, "profiles",
                                     "traffic_k_as_dense_bf16_split_k_splitk_reduce_dense_learned.json")))
    if tf["source_sha"] == bench.kernel_source_sha(["k_dense_bf16.hip"]):
        assert roof["traffic"] == pytest.approx(tf["hbm_bytes_per_launch_scaled"])
    else:
        assert roof["traffic"] is None


def test_whole_k_launch_keeps_the_plain_product_name():
    wl = bench.WORKLOADS["dense_mixed"]
    n, d = 50000, 8192
    prof = _prof(**{"as": (15, 480, 15 * 23.4), "chol": (15, 480, 30.0), "iters": (15, 480, 100.0)})
    _, roof = bench.kernel_table(prof, wl, "dense_mixed", n, d, n * d, d, n, 1024, 0.40)
    assert roof["kernel"] == "k_as_dense_bf16"  # 32 x 128 tiles fill the chip without a split


@pytest.mark.parametrize("tau,slots,name", [
    (512, 2, "k_chol_assemble+k_chol_diag0+k_chol_step"),
    (1024, 31, "k_chol_assemble+k_chol_diag0+k_chol_panel+k_chol_narrow+k_chol_update"),
    (5184, 31, "k_chol_assemble+k_chol_diag0+k_chol_panel+k_chol_narrow+k_chol_update+k_chol_ll_inverse+"
               "k_chol_lauum"),
])
def test_factorisation_roofline_names_the_tiled_form(tau, slots, name):
    wl = dict(bench.WORKLOADS["dense_mixed"], gram=True, tau=tau)
    prof = _prof(**{"chol": (10, 10 * slots, 10 * 2.0), "as": (10, 10 * slots, 1.0), "iters": (10, 10 * slots, 1.0)})
    _, roof = bench.kernel_table(prof, wl, "dense_mixed", 50000, 8192, 0, 8192, 50000, tau, 0.05)
    assert roof["kernel"] == name
    assert roof["alg_flops_per_launch"] == pytest.approx(float(tau) ** 3 * slots)
    assert roof["peak"] == bench.FP64_PEAK_TFS


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=300)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
