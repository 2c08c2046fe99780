"""Sketch draws S_k ~ D for sketch-and-project (Sec. 4), from Philox4x64-10.

Random-stream convention (shared by every implementation of the method in
this repository, each written independently):

* key     = (seed, problem_id)
* counter = (i, k, tag, slot): coordinate index i, iteration k, a tag naming
  the draw (1 subsample, 2 count, 3 SubCount, 4 weighted subsample) and a
  solve slot (0 unless a caller asks for per-solve streams).
* W0..W3 are the four 64-bit output words of that block.

Draws:

* Subsample (Def. 4.2, eq:subsample): C is the set of tau coordinates with the
  smallest pairs (W0_i, i) in lexicographic order. Every tau-subset is then
  equally likely, as eq:subsample requires. S = I_C with its columns in
  ascending coordinate order.
* Count (Sec. 4.2): every row i is sent to bucket h(i) = floor(hi32(W0_i) * tau
  / 2^32) with sign sigma_i = -1 if W1_i is odd else +1, i.e. each row of A
  has its sign flipped with probability 1/2 and is added to a uniformly drawn
  row of S^T A.
* SubCount (Def. 4.3, eq:Sigmacount): S^T = Sigma D I_C. The s = k*tau
  coordinates with the smallest (W0_i, i) (tag 3) are kept in ascending key
  order, i.e. in random order; the coordinate of rank p lands in bucket
  floor(p / k) (k contiguous rows summed) with sign from W1_i.
* Weighted subsample (a distribution D other than uniform, Sec. 3 and the
  non-uniform sampling of Sec. 7): u_i = ((W0_i >> 12) + 0.5) * 2^-52 and
  key_i = u_i / q_i in IEEE FP64; the tau smallest (key_i, i) are kept.

Part of the oracle: test infrastructure only.
"""
from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp

from .philox import philox4x64_10

TAG_SUBSAMPLE = 1
TAG_COUNT = 2
TAG_SUBCOUNT = 3
TAG_WEIGHTED = 4


def _blocks(seed, problem_id, k, tag, slot, m):
    i = np.arange(m, dtype=np.uint64)
    return philox4x64_10(i, np.uint64(k), np.uint64(tag), np.uint64(slot),
                         np.uint64(seed), np.uint64(problem_id))


def _smallest(keys, count):
    """Indices of the `count` smallest (key, index) pairs, in ascending key order."""
    idx = np.arange(keys.shape[0])
    order = np.lexsort((idx, keys))  # primary: key, ties: lower index first
    return order[:count]


def subcount_k(m, tau):
    """Sum size k of the SubCount sketch when the caller gives none (Sec. 4.2):
    k = 10 if 10*tau <= m, else floor(m / tau); then s = k * tau."""
    if 10 * tau <= m:
        return 10
    return m // tau


@dataclass
class Sketch:
    kind: str            # "subsample" | "count" | "subcount" | "weighted"
    m: int
    tau: int
    rows: np.ndarray     # int64: coordinates carrying a nonzero of S
    cols: np.ndarray     # int64: the column (bucket) of S for each of `rows`
    signs: np.ndarray    # float64: the value (+1/-1) of S at (rows, cols)

    def matrix(self):
        """S as an m x tau sparse matrix (CSR)."""
        return sp.csr_matrix((self.signs, (self.rows, self.cols)), shape=(self.m, self.tau))


def draw_subsample(seed, problem_id, k, m, tau, slot=0):
    """Uniform tau-subset C (eq:subsample); S = I_C, columns in ascending index."""
    if not (1 <= tau <= m):
        raise ValueError("subsample needs 1 <= tau <= m")
    w0, _, _, _ = _blocks(seed, problem_id, k, TAG_SUBSAMPLE, slot, m)
    C = np.sort(_smallest(w0, tau)).astype(np.int64)
    return Sketch("subsample", m, tau, C, np.arange(tau, dtype=np.int64), np.ones(tau))


def draw_count(seed, problem_id, k, m, tau, slot=0):
    """Count sketch (Sec. 4.2): hash h(i) in [0, tau) and sign sigma_i per row."""
    if tau < 1:
        raise ValueError("count sketch needs tau >= 1")
    w0, w1, _, _ = _blocks(seed, problem_id, k, TAG_COUNT, slot, m)
    h = ((w0 >> np.uint64(32)) * np.uint64(tau)) >> np.uint64(32)
    sigma = np.where((w1 & np.uint64(1)) == 1, -1.0, 1.0)
    return Sketch("count", m, tau, np.arange(m, dtype=np.int64), h.astype(np.int64), sigma)


def draw_subcount(seed, problem_id, k, m, tau, sum_size=0, slot=0):
    """SubCount sketch (Def. 4.3): S^T = Sigma D I_C with s = sum_size * tau."""
    kk = sum_size if sum_size > 0 else subcount_k(m, tau)
    s = kk * tau
    if kk < 1 or s > m:
        raise ValueError("SubCount needs 1 <= k and k * tau <= m")
    w0, w1, _, _ = _blocks(seed, problem_id, k, TAG_SUBCOUNT, slot, m)
    chosen = _smallest(w0, s).astype(np.int64)          # ascending key order = random order
    rank = np.arange(s, dtype=np.int64)
    bucket = rank // kk                                   # Sigma sums k contiguous rows
    sigma = np.where((w1[chosen] & np.uint64(1)) == 1, -1.0, 1.0)
    return Sketch("subcount", m, tau, chosen, bucket, sigma)


def uniform_keys_weighted(seed, problem_id, k, m, slot=0):
    """u_i = ((W0_i >> 12) + 0.5) * 2^-52, exactly representable in FP64, in (0, 1)."""
    w0, _, _, _ = _blocks(seed, problem_id, k, TAG_WEIGHTED, slot, m)
    return ((w0 >> np.uint64(12)).astype(np.float64) + 0.5) * 2.0 ** -52


def draw_weighted(seed, problem_id, k, q, tau, slot=0):
    """Subsample with inclusion driven by a proposal q > 0: the tau smallest u_i / q_i."""
    q = np.asarray(q)
    m = q.shape[0]
    if not (1 <= tau <= m):
        raise ValueError("weighted subsample needs 1 <= tau <= m")
    u = uniform_keys_weighted(seed, problem_id, k, m, slot)
    keys = u / q.astype(np.float64)
    C = np.sort(_smallest(keys, tau)).astype(np.int64)
    return Sketch("weighted", m, tau, C, np.arange(tau, dtype=np.int64), np.ones(tau))


def draw(kind, seed, problem_id, k, m, tau, sum_size=0, slot=0, q=None):
    if kind == "subsample":
        return draw_subsample(seed, problem_id, k, m, tau, slot)
    if kind == "count":
        return draw_count(seed, problem_id, k, m, tau, slot)
    if kind == "subcount":
        return draw_subcount(seed, problem_id, k, m, tau, sum_size, slot)
    if kind == "weighted":
        return draw_weighted(seed, problem_id, k, q, tau, slot)
    raise ValueError(f"unknown sketch kind {kind!r}")
