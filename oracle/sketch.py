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
* Gaussian (Def. 4.1): S_ic ~ N(0, 1) i.i.d. Entry (i, c) comes from the block with
  counter (i * G + c // 4, k, 6, slot), G = ceil(tau / 4): uniforms
  u = ((W >> 11) + 0.5) * 2^-53 and the Box-Muller transform of the pairs (W0, W1)
  (columns 4g, 4g + 1) and (W2, W3) (columns 4g + 2, 4g + 3):
  sqrt(-2 ln u_a) cos(2 pi u_b), sqrt(-2 ln u_a) sin(2 pi u_b).
* SRHT (Def. 4.4): S^T = I_C H_{m'} D / sqrt(tau m') with m' = 2^ceil(log2 m) and A
  padded with zero rows, so S holds the first m rows of D H_{m'} I_C^T / sqrt(tau m'):
  S_ic = d_i (-1)^popcount(i & C_c) / sqrt(tau m'). C: the tau smallest (W0_j, j) over
  j < m' (tag 7), ascending; d_i = -1 if W1_i (same block) is odd, else +1.

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
TAG_GAUSSIAN = 6
TAG_SRHT = 7


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
    kind: str            # "subsample" | "count" | "subcount" | "weighted" | "gaussian" | "srht"
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


def _dense_sketch(kind, S):
    m, tau = S.shape
    rows = np.repeat(np.arange(m, dtype=np.int64), tau)
    cols = np.tile(np.arange(tau, dtype=np.int64), m)
    return Sketch(kind, m, tau, rows, cols, S.reshape(-1).copy())


def gaussian_matrix(seed, problem_id, k, m, tau, slot=0):
    """The m x tau Gaussian sketch (Def. 4.1) as a dense array."""
    if tau < 1 or m < 1:
        raise ValueError("Gaussian sketch needs m, tau >= 1")
    G = (tau + 3) // 4
    j = (np.arange(m, dtype=np.uint64)[:, None] * np.uint64(G) + np.arange(G, dtype=np.uint64)[None, :]).ravel()
    w = philox4x64_10(j, np.uint64(k), np.uint64(TAG_GAUSSIAN), np.uint64(slot), np.uint64(seed),
                      np.uint64(problem_id))
    u = [((x >> np.uint64(11)).astype(np.float64) + 0.5) * 2.0 ** -53 for x in w]
    r01, t01 = np.sqrt(-2.0 * np.log(u[0])), 2.0 * np.pi * u[1]
    r23, t23 = np.sqrt(-2.0 * np.log(u[2])), 2.0 * np.pi * u[3]
    z = np.stack([r01 * np.cos(t01), r01 * np.sin(t01), r23 * np.cos(t23), r23 * np.sin(t23)], axis=1)
    return z.reshape(m, 4 * G)[:, :tau].copy()


def draw_gaussian(seed, problem_id, k, m, tau, slot=0):
    return _dense_sketch("gaussian", gaussian_matrix(seed, problem_id, k, m, tau, slot))


def srht_padded_size(m):
    """m' = 2^ceil(log2 m) (Sec. 4.3: A is padded with zero rows to a power of 2)."""
    return 1 << max(0, int(m - 1).bit_length())


def srht_parts(seed, problem_id, k, m, tau, slot=0):
    """(C, d, m') of the SRHT sketch: C ascending in [0, m'), signs d for the first m rows."""
    mp = srht_padded_size(m)
    if not (1 <= tau <= mp):
        raise ValueError("SRHT needs 1 <= tau <= m'")
    w0, w1, _, _ = _blocks(seed, problem_id, k, TAG_SRHT, slot, mp)
    C = np.sort(_smallest(w0, tau)).astype(np.int64)
    d = np.where((w1[:m] & np.uint64(1)) == 1, -1.0, 1.0)
    return C, d, mp


def srht_matrix(seed, problem_id, k, m, tau, slot=0):
    """The m x tau SRHT sketch (Def. 4.4) as a dense array, from the closed form of the
    Sylvester Hadamard entries H_ij = (-1)^popcount(i & j)."""
    C, d, mp = srht_parts(seed, problem_id, k, m, tau, slot)
    i = np.arange(m, dtype=np.int64)[:, None]
    bits = np.bitwise_and(i, C[None, :])
    par = np.zeros(bits.shape, dtype=np.int64)
    while np.any(bits):
        par ^= bits & 1
        bits >>= 1
    H = 1.0 - 2.0 * par
    return d[:, None] * H * (1.0 / np.sqrt(float(tau) * float(mp)))


def draw_srht(seed, problem_id, k, m, tau, slot=0):
    return _dense_sketch("srht", srht_matrix(seed, problem_id, k, m, tau, slot))


def draw(kind, seed, problem_id, k, m, tau, sum_size=0, slot=0, q=None):
    if kind == "subsample":
        return draw_subsample(seed, problem_id, k, m, tau, slot)
    if kind == "count":
        return draw_count(seed, problem_id, k, m, tau, slot)
    if kind == "subcount":
        return draw_subcount(seed, problem_id, k, m, tau, sum_size, slot)
    if kind == "weighted":
        return draw_weighted(seed, problem_id, k, q, tau, slot)
    if kind == "gaussian":
        return draw_gaussian(seed, problem_id, k, m, tau, slot)
    if kind == "srht":
        return draw_srht(seed, problem_id, k, m, tau, slot)
    raise ValueError(f"unknown sketch kind {kind!r}")
