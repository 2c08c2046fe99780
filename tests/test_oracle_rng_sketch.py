"""Pins for the oracle's random draws and sketch constructions (CPU only)."""
import itertools
import json
import math
import os

import numpy as np
import pytest
import scipy.stats

from oracle import sketch as sk
from oracle.philox import philox4x64_10

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_settings.json")


def _numpy_block(counter, key):
    """numpy's Philox advances its 256-bit counter before producing a block."""
    v = sum(int(c) << (64 * i) for i, c in enumerate(counter))
    v = (v - 1) % (1 << 256)
    prev = [(v >> (64 * i)) & ((1 << 64) - 1) for i in range(4)]
    g = np.random.Philox(key=np.array(key, dtype=np.uint64), counter=np.array(prev, dtype=np.uint64))
    return [int(x) for x in g.random_raw(4)]


@pytest.mark.parametrize("counter,key", [
    ((0, 0, 0, 0), (0, 0)),
    ((1, 0, 0, 0), (5, 7)),
    ((123456789, 42, 3, 1), (2105055650, 17)),
    ((2**64 - 1, 2**63, 4, 2**32 + 5), (2**64 - 1, 1)),
])
def test_philox_matches_numpy_library(counter, key):
    mine = [int(x) for x in philox4x64_10(*[np.uint64(c) for c in counter], *key)]
    assert mine == _numpy_block(counter, key)


def test_philox_vectorised_equals_scalar():
    i = np.arange(1000, dtype=np.uint64)
    vec = philox4x64_10(i, np.uint64(7), np.uint64(1), np.uint64(0), 11, 3)
    for j in (0, 1, 499, 999):
        one = philox4x64_10(np.uint64(j), np.uint64(7), np.uint64(1), np.uint64(0), 11, 3)
        assert all(int(vec[t][j]) == int(one[t]) for t in range(4))


def test_subsample_is_sorted_distinct_subset():
    s = sk.draw_subsample(3, 0, 5, 1000, 77)
    assert s.rows.shape == (77,)
    assert np.all(np.diff(s.rows) > 0)
    assert s.rows.min() >= 0 and s.rows.max() < 1000
    S = s.matrix().toarray()
    assert np.array_equal(S, np.eye(1000)[:, s.rows])


def test_subsample_matches_bruteforce_selection():
    m, tau = 40, 9
    w0, _, _, _ = philox4x64_10(np.arange(m, dtype=np.uint64), np.uint64(2), np.uint64(sk.TAG_SUBSAMPLE),
                                np.uint64(0), 5, 1)
    pairs = sorted((int(w0[i]), i) for i in range(m))
    expect = sorted(i for _, i in pairs[:tau])
    assert list(sk.draw_subsample(5, 1, 2, m, tau).rows) == expect


def test_subsample_uniform_over_subsets():
    """eq:subsample: every tau-subset has probability 1 / binom(m, tau)."""
    m, tau, trials = 5, 2, 6000
    counts = {c: 0 for c in itertools.combinations(range(m), tau)}
    for k in range(trials):
        counts[tuple(sk.draw_subsample(9, 0, k, m, tau).rows)] += 1
    obs = np.array(list(counts.values()))
    chi2 = scipy.stats.chisquare(obs).pvalue
    assert chi2 > 1e-4


def test_count_sketch_hash_and_signs():
    m, tau = 20000, 500
    s = sk.draw_count(1, 0, 3, m, tau)
    assert s.cols.min() >= 0 and s.cols.max() < tau
    hist = np.bincount(s.cols, minlength=tau)
    assert scipy.stats.chisquare(hist).pvalue > 1e-4
    npos = int((s.signs > 0).sum())
    assert abs(npos - m / 2) < 5 * math.sqrt(m / 4)
    # one nonzero per row of S, equal to the sign
    S = s.matrix()
    assert S.nnz == m and np.all(np.abs(S.data) == 1)


def test_subcount_matches_product_of_factors():
    """Def. 4.3: S^T = Sigma D I_C built from its three factors (eq:Sigmacount)."""
    m, tau, kk = 30, 4, 3
    s = sk.draw_subcount(4, 2, 1, m, tau, sum_size=kk)
    ssz = kk * tau
    chosen = s.rows                         # ascending key order = the order of I_C's rows
    I_C = np.zeros((ssz, m))
    I_C[np.arange(ssz), chosen] = 1.0
    D = np.diag(s.signs)
    Sigma = np.zeros((tau, ssz))
    for b in range(tau):
        Sigma[b, b * kk:(b + 1) * kk] = 1.0
    St = Sigma @ D @ I_C
    assert np.array_equal(s.matrix().toarray().T, St)
    assert len(set(chosen.tolist())) == ssz


def test_subcount_golden_example_and_rule():
    g = json.load(open(GOLDEN))
    ex = g["subcount_example"]
    s = sk.draw_subcount(1, 0, 0, 10, ex["tau"], sum_size=ex["k"])
    assert s.rows.shape[0] == ex["s"]
    assert np.all(np.bincount(s.cols, minlength=ex["tau"]) == ex["k"])
    # the paper's default rule
    assert sk.subcount_k(1000, 100) == 10      # 10 tau <= m
    assert sk.subcount_k(506, 126) == 4        # else floor(m / tau)
    assert sk.subcount_k(999, 100) == 9


def test_subcount_with_all_rows_is_signed_permutation():
    m = 12
    s = sk.draw_subcount(2, 0, 0, m, m, sum_size=1)
    S = s.matrix().toarray()
    assert np.array_equal(np.abs(S) @ np.abs(S).T, np.eye(m))


def test_weighted_keys_exact_and_selection():
    m, tau = 64, 10
    u = sk.uniform_keys_weighted(3, 0, 4, m)
    assert np.all((u > 0) & (u < 1))
    w0, _, _, _ = philox4x64_10(np.arange(m, dtype=np.uint64), np.uint64(4), np.uint64(sk.TAG_WEIGHTED),
                                np.uint64(0), 3, 0)
    # exactness: u * 2^52 - 0.5 recovers the integer W0 >> 12
    assert np.array_equal((u * 2.0 ** 52 - 0.5).astype(np.uint64), w0 >> np.uint64(12))
    q = np.linspace(1.0, 2.0, m).astype(np.float32)
    s = sk.draw_weighted(3, 0, 4, q, tau)
    keys = u / q.astype(np.float64)
    expect = sorted(i for _, i in sorted((keys[i], i) for i in range(m))[:tau])
    assert list(s.rows) == expect


def test_weighted_inclusion_follows_proposal():
    """Heavier q means more frequent inclusion; equal q gives the uniform subsample law."""
    m, tau, trials = 8, 2, 4000
    q = np.array([8, 1, 1, 1, 1, 1, 1, 1], dtype=np.float32)
    hits = np.zeros(m)
    for k in range(trials):
        hits[sk.draw_weighted(1, 0, k, q, tau).rows] += 1
    assert hits[0] > 2.5 * hits[1:].mean()
    qu = np.ones(m, dtype=np.float32)
    hits_u = np.zeros(m)
    for k in range(trials):
        hits_u[sk.draw_weighted(1, 0, k, qu, tau).rows] += 1
    assert scipy.stats.chisquare(hits_u).pvalue > 1e-4


def test_paper_sketch_sizes():
    g = json.load(open(GOLDEN))
    for e in g["sketch_sizes"]:
        m = e["m"]
        val = {"floor(m/4)": m // 4, "m/4": m / 4, "ceil(m^(2/3))": math.ceil(m ** (2 / 3)),
               "floor(m^(2/3))": math.floor(m ** (2 / 3))}[e["rule"]]
        assert val == e["tau"], e
