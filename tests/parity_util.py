"""Element-wise comparison helpers shared by the GPU parity tests.

A vector from the HIP path matches the oracle's to relative tolerance tol when every entry
satisfies |got_i - exp_i| <= tol * |exp_i| + tol * max_j |exp_j|: relative where the entry is
of the vector's own scale, and absolute at tol times the largest entry where it is small (a
coordinate that the two rounding orders both leave near zero). This is stricter than a
norm-wise ||got - exp|| / ||exp|| <= tol by up to the square root of the vector's length.
"""
import numpy as np


def assert_vec_close(got, exp, tol, what=""):
    got = np.asarray(got, dtype=np.float64)
    exp = np.asarray(exp, dtype=np.float64)
    assert got.shape == exp.shape, (what, got.shape, exp.shape)
    scale = float(np.max(np.abs(exp))) if exp.size else 0.0
    err = np.abs(got - exp)
    lim = tol * np.abs(exp) + tol * scale
    bad = err > lim
    if np.any(bad):
        i = int(np.argmax(err - lim))
        raise AssertionError(
            f"{what}: {int(bad.sum())} of {exp.size} entries outside tol {tol:g}; worst at {i}: "
            f"got {got[i]!r} expected {exp[i]!r} (|diff| {err[i]:.3e}, limit {lim[i]:.3e}, "
            f"max |expected| {scale:.3e})")
    return float(np.max(err / np.maximum(lim / tol, 1e-300))) if exp.size else 0.0


def assert_state_close(gpu_state, oracle_pairs, tol, what=""):
    """gpu_state: sequence of arrays; oracle_pairs: matching sequence of (name, array)."""
    worst = 0.0
    for g, (name, e) in zip(gpu_state, oracle_pairs):
        worst = max(worst, assert_vec_close(g, e, tol, f"{what} {name}"))
    return worst
