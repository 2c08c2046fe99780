// Device-wide blocked FP64 Cholesky and inverse of the sketched matrices G = S^T A S
// of a lookahead batch (least-norm solution of eq:sketched_system, delta = G^{-1} rho).
//
// The single-workgroup factorisation (k_chol.hip) runs one sketch per compute unit,
// which leaves most of the chip idle when a batch holds few sketches. Here every
// 64 x 64 tile of every sketch is a workgroup, and the sequential structure of a
// right-looking algorithm is carried by kernel boundaries on the stream. With nt tiles
// per side, the factorisation, the inverse W = L^{-1} and the product G^{-1} = W^T W all
// advance together, one block column per launch, in nt + 1 launches:
//
//   assemble (+ diag0)     G assembled on and below the diagonal (gathered rows of AS for
//                          the subsample sketch, identity padding and empty buckets); tile (0, 0) factored in
//                          LDS, X_0 = L_00^{-1} stored (by the assembly's workgroup of that
//                          tile, or in a launch of its own when many sketches are assembled)
//   step s = 1 .. nt, k = s - 1, one workgroup per item:
//     F  (s <= l <= i)     G_il -= L_ik L_lk^T with L_ik = G_ik X_k^T formed in the
//                          workgroup; the item (s, s) then factors G_ss in LDS: X_s
//     I  (i >= s, j <= k)  T_ij (+)= L_ik W_kj, where W_kj = -X_k T_kj (j < k) or X_k
//                          (j = k); T_ij = sum_{t=j}^{i-1} L_it W_tj is what row i of
//                          W = L^{-1} needs: W_ij = -X_i T_ij
//     A  (j <= i <= k)     (G^{-1})_ij (+)= W_ki^T W_kj, both W blocks formed from T in
//                          the workgroup; the last step also writes the upper triangle
//
// L itself is never stored: every item forms the L and W blocks it reads from G, X and T,
// which are final by the time it runs (G_ik after step k - 1, X_k in step k, T_kj after
// step k - 1). T lives in the tiles of U below the diagonal, G^{-1} over G: in step s the
// tiles read by one item are written by none, each written tile by one item only.
#include "chol_tiles.h"
#include "dev_common.h"
#include "rs_internal.h"

namespace rs {
namespace {

using namespace chol;

struct MultiArgs {
  double* G;      // [slots][ldg][ldg]
  double* U;      // [slots][ldg][ldg]  T_ij in the tiles below the diagonal
  double* X;      // [slots][nt][64][64]  X_k = L_kk^{-1}
  int64_t ldg;
  int32_t nt, tau, kind;
  const void* AS;
  int32_t as_f32;
  int64_t ldas, m;
  const int32_t* members;
  const int32_t* offs;
  int32_t* status;
  const int32_t* done;
  int32_t nslots;
  int32_t xcd;  // 1: the items of a sketch on one XCD (see item_of_block)
};

// Sketch and item of this workgroup. Plain layout: grid (items, nslots). XCD layout (many
// sketches): a 1-D grid of 8 * ceil(nslots / 8) * items workgroups; workgroup b runs on XCD
// b % 8, sketches are dealt round-robin to the XCDs and each XCD takes its sketches' items
// one sketch after the other, so the tiles a sketch's items share stay in that XCD's L2.
// Returns false for the padding workgroups of the XCD layout.
__device__ __forceinline__ bool item_of_block(const MultiArgs& a, int items, int64_t* slot, int* item) {
  if (!a.xcd) {
    *slot = blockIdx.y;
    *item = blockIdx.x;
    return true;
  }
  const int b = blockIdx.x, q = b >> 3;
  *slot = (b & 7) + 8 * (q / items);
  *item = q % items;
  return *slot < a.nslots;
}

__device__ __forceinline__ double* tile(double* base, int64_t ld, int i, int j) {
  return base + (int64_t)i * NB * ld + (int64_t)j * NB;
}

// Linear index -> (i, j) with lo <= j <= i (row-major over i).
__device__ __forceinline__ void lower_pair(int idx, int lo, int* i, int* j) {
  int row = lo, width = 1;
  while (idx >= width) {
    idx -= width;
    ++row;
    ++width;
  }
  *i = row;
  *j = lo + idx;
}

// X_s <- ta (64 x 64 from LDS), and its transpose into the diagonal tile U_ss (the form the
// inverse by distance reads).
__device__ __forceinline__ void store_x(double* X, double* Uss, int64_t ldg, const double* ta) {
  for (int e = threadIdx.x; e < NB * NB; e += kThreads) {
    const int r = e >> 6, c = e & 63;
    X[e] = ta[r * LDT + c];
    Uss[(int64_t)r * ldg + c] = ta[c * LDT + r];
  }
}

// FACTOR0: the workgroup of tile (0, 0) also factors it (dynamic LDS: two tiles for every
// workgroup, so only with few sketches); otherwise k_chol_diag0 does, in a launch of its own.
// Only the tiles on and below the diagonal (grid: nt (nt + 1) / 2 x 1 x slots): the steps read
// G below the diagonal and write G^{-1} over both triangles at the end.
template <bool FACTOR0>
__global__ __launch_bounds__(kThreads) void k_chol_assemble(MultiArgs a) {
  extern __shared__ __align__(16) double lds[];
  __shared__ int bad;
  if (*a.done) return;
  const int64_t slot = blockIdx.z;
  int ti, tj;
  lower_pair(blockIdx.x, 0, &ti, &tj);
  const bool first = FACTOR0 && ti == 0 && tj == 0;
  double* G = a.G + slot * a.ldg * a.ldg;
  const int32_t* offs = a.offs + slot * (a.tau + 1);
  const int32_t* members = a.members + slot * a.tau;  // subsample: nsel = tau
  // the 16 values of this thread first (their loads in flight together), then the stores
  constexpr int kPer = NB * NB / kThreads;
  double v[kPer];
  bool wr[kPer];
#pragma unroll
  for (int q = 0; q < kPer; ++q) {
    const int e = threadIdx.x + kThreads * q, r = e >> 6, c = e & 63;
    const int64_t gr = (int64_t)ti * NB + r, gc = (int64_t)tj * NB + c;
    wr[q] = true;
    if (gr >= a.tau || gc >= a.tau) {
      v[q] = (gr == gc) ? 1.0 : 0.0;
    } else if (a.kind == kSubsample) {
      const int64_t src = (slot * a.m + members[gr]) * a.ldas + gc;
      v[q] = a.as_f32 ? (double)((const float*)a.AS)[src] : ((const double*)a.AS)[src];
    } else if (gr == gc && offs[gr + 1] == offs[gr]) {
      v[q] = 1.0;  // empty bucket: zero row and column of S^T A S
    } else {
      wr[q] = false;  // formed already (S^T A S summed from AS)
      v[q] = first ? G[gr * a.ldg + gc] : 0.0;
    }
  }
#pragma unroll
  for (int q = 0; q < kPer; ++q) {
    const int e = threadIdx.x + kThreads * q, r = e >> 6, c = e & 63;
    if (wr[q]) G[((int64_t)ti * NB + r) * a.ldg + (int64_t)tj * NB + c] = v[q];
    if (first) lds[r * LDT + c] = v[q];
  }
  if (!first) return;
  if (threadIdx.x == 0) bad = 0;
  __syncthreads();
  factor_diag_tile(lds, lds + NB * LDT, &bad);
  store_x(a.X + slot * a.nt * NB * NB, a.U + slot * a.ldg * a.ldg, a.ldg, lds + NB * LDT);
  if (threadIdx.x == 0) a.status[slot] = bad;
}

// Tile (0, 0) of every sketch factored in LDS: X_0 and U_00, and the sketch's status.
__global__ __launch_bounds__(kThreads) void k_chol_diag0(MultiArgs a) {
  extern __shared__ __align__(16) double lds[];
  __shared__ int bad;
  if (*a.done) return;
  const int64_t slot = blockIdx.x;
  if (threadIdx.x == 0) bad = 0;
  load_tile(lds, a.G + slot * a.ldg * a.ldg, a.ldg, false);
  __syncthreads();
  factor_diag_tile(lds, lds + NB * LDT, &bad);
  store_x(a.X + slot * a.nt * NB * NB, a.U + slot * a.ldg * a.ldg, a.ldg, lds + NB * LDT);
  if (threadIdx.x == 0) a.status[slot] = bad;
}

// Items of step s: F first (its item 0 is the diagonal tile (s, s), the longest), then I,
// then A. LDS: tx, ta, tb (64 x LDT each).
__global__ __launch_bounds__(kThreads) void k_chol_step(MultiArgs a, int s) {
  extern __shared__ __align__(16) double lds[];
  double* tx = lds;
  double* ta = lds + NB * LDT;
  double* tb = lds + 2 * NB * LDT;
  __shared__ int bad;
  if (*a.done) return;
  const int nt = a.nt, k = s - 1;
  const int nF = (nt - s) * (nt - s + 1) / 2, nI = (nt - s) * s;
  int64_t slot;
  int item;
  if (!item_of_block(a, nF + nI + s * (s + 1) / 2, &slot, &item)) return;
  double* G = a.G + slot * a.ldg * a.ldg;
  double* U = a.U + slot * a.ldg * a.ldg;
  const double* Xk = a.X + (slot * nt + k) * NB * NB;
  if (item < nF) {
    // F: G_il -= L_ik L_lk^T
    int i, l;
    lower_pair(item, s, &i, &l);
    double* Gil = tile(G, a.ldg, i, l);
    Acc g;
    acc_load(g, Gil, a.ldg);
    load_tile(tx, Xk, NB, false);
    load_tile(ta, tile(G, a.ldg, i, k), a.ldg, false);
    if (l != i) load_tile(tb, tile(G, a.ldg, l, k), a.ldg, false);
    __syncthreads();
    Acc c1, c2;
    acc_zero(c1);
    tile_mma(c1, ta, tx);  // L_ik
    if (l != i) {
      acc_zero(c2);
      tile_mma(c2, tb, tx);  // L_lk
    }
    __syncthreads();
    acc_for_each(c1, [&](int r, int cc, double v) { ta[r * LDT + cc] = v; });
    if (l != i) acc_for_each(c2, [&](int r, int cc, double v) { tb[r * LDT + cc] = v; });
    __syncthreads();
    Acc c3;
    acc_zero(c3);
    tile_mma(c3, ta, l != i ? tb : ta);
    if (i == s && l == s) {
      // the diagonal tile of step s is now final: factor it
      if (threadIdx.x == 0) bad = 0;
      __syncthreads();
#pragma unroll
      for (int u = 0; u < 2; ++u)
#pragma unroll
        for (int w = 0; w < 2; ++w) g.v[u][w] -= c3.v[u][w];
      acc_for_each(g, [&](int r, int cc, double v) { tx[r * LDT + cc] = v; });
      __syncthreads();
      factor_diag_tile(tx, ta, &bad);
      store_x(a.X + (slot * nt + s) * NB * NB, tile(U, a.ldg, s, s), a.ldg, ta);
      if (threadIdx.x == 0 && bad) a.status[slot] = 1;
    } else {
#pragma unroll
      for (int u = 0; u < 2; ++u)
#pragma unroll
        for (int w = 0; w < 2; ++w) g.v[u][w] -= c3.v[u][w];
      acc_for_each(g, [&](int r, int cc, double v) { Gil[(int64_t)r * a.ldg + cc] = v; });
    }
    return;
  }
  item -= nF;
  if (item < nI) {
    // I: T_ij (+)= L_ik W_kj
    const int i = s + item / s, j = item % s;
    double* Tij = tile(U, a.ldg, i, j);
    Acc g;
    if (j < k) acc_load(g, Tij, a.ldg);
    load_tile(tx, Xk, NB, false);
    load_tile(ta, tile(G, a.ldg, i, k), a.ldg, false);
    if (j < k)
      load_tile(tb, tile(U, a.ldg, k, j), a.ldg, true);  // T_kj^T
    else
      load_tile(tb, Xk, NB, true);  // W_kk^T = X_k^T
    __syncthreads();
    Acc c1, c2;
    acc_zero(c1);
    tile_mma(c1, ta, tx);  // L_ik
    if (j < k) {
      acc_zero(c2);
      tile_mma(c2, tx, tb);  // X_k T_kj = -W_kj
    }
    __syncthreads();
    acc_for_each(c1, [&](int r, int cc, double v) { ta[r * LDT + cc] = v; });
    if (j < k) acc_for_each(c2, [&](int r, int cc, double v) { tb[cc * LDT + r] = -v; });  // W_kj^T
    __syncthreads();
    Acc c3;
    acc_zero(c3);
    tile_mma(c3, ta, tb);  // L_ik W_kj
    if (j < k) {
#pragma unroll
      for (int u = 0; u < 2; ++u)
#pragma unroll
        for (int w = 0; w < 2; ++w) c3.v[u][w] += g.v[u][w];
    }
    acc_for_each(c3, [&](int r, int cc, double v) { Tij[(int64_t)r * a.ldg + cc] = v; });
    return;
  }
  item -= nI;
  {
    // A: (G^{-1})_ij (+)= W_ki^T W_kj for j <= i <= k
    int i, j;
    lower_pair(item, 0, &i, &j);
    double* Gij = tile(G, a.ldg, i, j);
    Acc g;
    if (i < k) acc_load(g, Gij, a.ldg);
    load_tile(tx, Xk, NB, false);
    if (i < k) load_tile(ta, tile(U, a.ldg, k, i), a.ldg, true);  // T_ki^T
    if (j < k && j != i) load_tile(tb, tile(U, a.ldg, k, j), a.ldg, true);
    __syncthreads();
    Acc c1, c2;
    if (i < k) {
      acc_zero(c1);
      tile_mma(c1, tx, ta);  // X_k T_ki = -W_ki
    }
    if (j < k && j != i) {
      acc_zero(c2);
      tile_mma(c2, tx, tb);  // -W_kj
    }
    __syncthreads();
    // operands of W_ki^T W_kj: ta[r][t] = W_ki[t][r], tb[c][t] = W_kj[t][c]
    if (i < k)
      acc_for_each(c1, [&](int r, int cc, double v) { ta[cc * LDT + r] = -v; });
    else
      for (int e = threadIdx.x; e < NB * NB; e += kThreads)
        ta[(e & 63) * LDT + (e >> 6)] = tx[(e >> 6) * LDT + (e & 63)];  // W_kk = X_k
    if (j < k && j != i) acc_for_each(c2, [&](int r, int cc, double v) { tb[cc * LDT + r] = -v; });
    __syncthreads();
    Acc c3;
    acc_zero(c3);
    tile_mma(c3, ta, j != i ? tb : ta);
    if (i < k) {
#pragma unroll
      for (int u = 0; u < 2; ++u)
#pragma unroll
        for (int w = 0; w < 2; ++w) c3.v[u][w] += g.v[u][w];
    }
    double* Gji = tile(G, a.ldg, j, i);
    const bool last = s == nt, mirror = last && i != j;
    acc_for_each(c3, [&](int r, int cc, double v) {
      Gij[(int64_t)r * a.ldg + cc] = v;
      if (mirror) Gji[(int64_t)cc * a.ldg + r] = v;
    });
  }
}

// Work-optimal form of the same steps, two launches per step (no block is formed twice).
// Panel of step s (k = s - 1): L_ik = G_ik X_k^T stored over G_ik (i >= s), and row k of W
// (mode 1), stored transposed over T_kj: U_kj <- W_kj^T = -(X_k T_kj)^T (j < k). The item
// of L_sk then brings the diagonal tile up to date, G_ss - L_sk L_sk^T (and - L_s,kx L_s,kx^T
// for kx >= 0, the column whose update of G_ss was deferred to here: the update launches
// leave the diagonal tile out), and factors it: X_s, U_ss = X_s^T. LDS: two tiles.
__global__ __launch_bounds__(kThreads) void k_chol_panel(MultiArgs a, int s, int items, int kx) {
  extern __shared__ __align__(16) double lds[];
  double* tx = lds;
  double* ta = lds + NB * LDT;
  __shared__ int bad;
  if (*a.done) return;
  const int nt = a.nt, k = s - 1;
  int64_t slot;
  int item;
  if (!item_of_block(a, items, &slot, &item)) return;
  double* G = a.G + slot * a.ldg * a.ldg;
  double* U = a.U + slot * a.ldg * a.ldg;
  const double* Xk = a.X + (slot * nt + k) * NB * NB;
  const bool lpanel = item < nt - s;
  double* dst = lpanel ? tile(G, a.ldg, s + item, k) : tile(U, a.ldg, k, item - (nt - s));
  const bool diag = lpanel && item == 0;
  Acc g;
  if (diag) acc_load(g, tile(G, a.ldg, s, s), a.ldg);
  load_tile(tx, Xk, NB, false);
  load_tile(ta, dst, a.ldg, !lpanel);  // G_ik, or T_kj^T
  __syncthreads();
  Acc c;
  acc_zero(c);
  if (lpanel) {
    tile_mma(c, ta, tx);  // L_ik = G_ik X_k^T
    acc_for_each(c, [&](int r, int cc, double v) { dst[(int64_t)r * a.ldg + cc] = v; });
  } else {
    tile_mma(c, tx, ta);  // X_k T_kj = -W_kj, stored as W_kj^T
    acc_for_each(c, [&](int r, int cc, double v) { dst[(int64_t)cc * a.ldg + r] = -v; });
  }
  if (!diag) return;
  if (threadIdx.x == 0) bad = 0;
  __syncthreads();  // ta, tx read by every wave
  acc_for_each(c, [&](int r, int cc, double v) { ta[r * LDT + cc] = v; });
  __syncthreads();
  Acc c2;
  acc_zero(c2);
  tile_mma(c2, ta, ta);  // L_sk L_sk^T
  if (kx >= 0) tile_mma_global(c2, tile(G, a.ldg, s, kx), tile(G, a.ldg, s, kx), a.ldg);  // + L_s,kx L_s,kx^T
#pragma unroll
  for (int u = 0; u < 2; ++u)
#pragma unroll
    for (int w = 0; w < 2; ++w) g.v[u][w] -= c2.v[u][w];
  acc_for_each(g, [&](int r, int cc, double v) { tx[r * LDT + cc] = v; });
  __syncthreads();
  factor_diag_tile(tx, ta, &bad);
  store_x(a.X + (slot * nt + s) * NB * NB, tile(U, a.ldg, s, s), a.ldg, ta);
  if (threadIdx.x == 0 && bad) a.status[slot] = 1;
}

// Updates from the stored panels of columns k_lo .. s - 1 (one, or two when a pair of steps
// shares the launch, so that each target is read and written once for both), the tile
// products straight from global memory (no LDS, so that many items share a compute unit):
// F (s <= l <= i, (s, s) left to the next panel): G_il -= sum_k L_ik L_lk^T;
// I (i >= s, j < s): T_ij (+)= sum_{k >= max(k_lo, j)} L_ik W_kj (the k = j term is the first);
// A (j <= i < s): (G^{-1})_ij (+)= sum_{k >= max(k_lo, i)} W_ki^T W_kj (the k = i term is the
// first). W_kj^T is read from U_kj (U_kk = X_k^T).
__global__ __launch_bounds__(kThreads) void k_chol_update(MultiArgs a, int s, int items, int k_lo) {
  if (*a.done) return;
  const int nt = a.nt;
  const int nF = (nt - s) * (nt - s + 1) / 2 - (s < nt ? 1 : 0), nI = (nt - s) * s;
  int64_t slot;
  int item;
  if (!item_of_block(a, items, &slot, &item)) return;
  double* G = a.G + slot * a.ldg * a.ldg;
  double* U = a.U + slot * a.ldg * a.ldg;
  const int64_t ld = a.ldg;
  Acc g, c;
  acc_zero(c);
  if (item < nF) {
    int i, l;
    lower_pair(item + 1, s, &i, &l);  // pair 0 is (s, s)
    double* Gil = tile(G, ld, i, l);
    acc_load(g, Gil, ld);
    for (int k = k_lo; k < s; ++k) tile_mma_global(c, tile(G, ld, i, k), tile(G, ld, l, k), ld);
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
      for (int w = 0; w < 2; ++w) g.v[u][w] -= c.v[u][w];
    acc_for_each(g, [&](int r, int cc, double v) { Gil[(int64_t)r * ld + cc] = v; });
    return;
  }
  item -= nF;
  if (item < nI) {
    const int i = s + item / s, j = item % s;
    const bool first = j >= k_lo;
    double* Tij = tile(U, ld, i, j);
    if (!first) acc_load(g, Tij, ld);
    for (int k = max(k_lo, j); k < s; ++k) tile_mma_global(c, tile(G, ld, i, k), tile(U, ld, k, j), ld);
    if (!first) {
#pragma unroll
      for (int u = 0; u < 2; ++u)
#pragma unroll
        for (int w = 0; w < 2; ++w) c.v[u][w] += g.v[u][w];
    }
    acc_for_each(c, [&](int r, int cc, double v) { Tij[(int64_t)r * ld + cc] = v; });
    return;
  }
  item -= nI;
  int i, j;
  lower_pair(item, 0, &i, &j);
  const bool first = i >= k_lo;
  double* Gij = tile(G, ld, i, j);
  if (!first) acc_load(g, Gij, ld);
  for (int k = max(k_lo, i); k < s; ++k) tile_mma_global(c, tile(U, ld, k, i), tile(U, ld, k, j), ld);
  if (!first) {
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
      for (int w = 0; w < 2; ++w) c.v[u][w] += g.v[u][w];
  }
  double* Gji = tile(G, ld, j, i);
  const bool mirror = s == nt && i != j;
  acc_for_each(c, [&](int r, int cc, double v) {
    Gij[(int64_t)r * ld + cc] = v;
    if (mirror) Gji[(int64_t)cc * ld + r] = v;
  });
}

// The part of step s's update (k = s - 1) that the next panel needs before a paired update
// applies the rest together with step s + 1's: column s of G, G_is -= L_ik L_sk^T (i > s),
// and, with trow, row s of T, T_sj (+)= L_sk W_kj (j <= k; the j = k term is the first).
__global__ __launch_bounds__(kThreads) void k_chol_narrow(MultiArgs a, int s, int items, int trow) {
  if (*a.done) return;
  const int nt = a.nt, k = s - 1, nFc = nt - s - 1;
  int64_t slot;
  int item;
  if (!item_of_block(a, items, &slot, &item)) return;
  double* G = a.G + slot * a.ldg * a.ldg;
  double* U = a.U + slot * a.ldg * a.ldg;
  const int64_t ld = a.ldg;
  Acc g, c;
  acc_zero(c);
  if (item < nFc) {
    double* Gis = tile(G, ld, s + 1 + item, s);
    acc_load(g, Gis, ld);
    tile_mma_global(c, tile(G, ld, s + 1 + item, k), tile(G, ld, s, k), ld);
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
      for (int w = 0; w < 2; ++w) g.v[u][w] -= c.v[u][w];
    acc_for_each(g, [&](int r, int cc, double v) { Gis[(int64_t)r * ld + cc] = v; });
    return;
  }
  if (!trow) return;
  const int j = item - nFc;
  double* Tsj = tile(U, ld, s, j);
  if (j < k) acc_load(g, Tsj, ld);
  tile_mma_global(c, tile(G, ld, s, k), tile(U, ld, k, j), ld);
  if (j < k) {
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
      for (int w = 0; w < 2; ++w) c.v[u][w] += g.v[u][w];
  }
  acc_for_each(c, [&](int r, int cc, double v) { Tsj[(int64_t)r * ld + cc] = v; });
}

// Inverse by distance d = i - j after the factorisation (mode 2): W_ij = -X_i sum_{k=j}^{i-1}
// L_ik W_kj as one chain of tile products per workgroup, stored transposed as U_ji (U = W^T),
// L_ik read from the tiles of G below the diagonal.
__global__ __launch_bounds__(kThreads) void k_chol_ll_inverse(MultiArgs a, int d) {
  extern __shared__ __align__(16) double lds[];
  double* tt = lds;
  double* tx = lds + NB * LDT;
  if (*a.done) return;
  int64_t slot;
  int j;
  if (!item_of_block(a, a.nt - d, &slot, &j)) return;
  const int i = j + d;
  double* G = a.G + slot * a.ldg * a.ldg;
  double* U = a.U + slot * a.ldg * a.ldg;
  Acc c;
  acc_zero(c);
  for (int k = j; k < i; ++k) tile_mma_global(c, tile(G, a.ldg, i, k), tile(U, a.ldg, j, k), a.ldg);
  // T = sum_k L_ik W_kj; U_ji = W_ij^T = -T^T X_i^T
  acc_for_each(c, [&](int r, int cc, double v) { tt[cc * LDT + r] = v; });
  load_tile(tx, a.X + (slot * a.nt + i) * NB * NB, NB, false);
  __syncthreads();
  Acc c2;
  acc_zero(c2);
  tile_mma(c2, tt, tx);
  double* Uji = tile(U, a.ldg, j, i);
  acc_for_each(c2, [&](int r, int cc, double v) { Uji[(int64_t)r * a.ldg + cc] = -v; });
}

// G^{-1} = U U^T (mode 2): tile (i, j) = sum_{k >= i} U_ik U_jk^T as one chain per
// workgroup, written to both triangles.
__global__ __launch_bounds__(kThreads) void k_chol_lauum(MultiArgs a) {
  if (*a.done) return;
  int64_t slot;
  int item, i, j;
  if (!item_of_block(a, a.nt * (a.nt + 1) / 2, &slot, &item)) return;
  lower_pair(item, 0, &i, &j);
  double* G = a.G + slot * a.ldg * a.ldg;
  double* U = a.U + slot * a.ldg * a.ldg;
  Acc c;
  acc_zero(c);
  for (int kt = i; kt < a.nt; ++kt) tile_mma_global(c, tile(U, a.ldg, i, kt), tile(U, a.ldg, j, kt), a.ldg);
  double* Gij = tile(G, a.ldg, i, j);
  double* Gji = tile(G, a.ldg, j, i);
  acc_for_each(c, [&](int r, int cc, double v) {
    Gij[(int64_t)r * a.ldg + cc] = v;
    if (i != j) Gji[(int64_t)cc * a.ldg + r] = v;
  });
}

}  // namespace

size_t chol_multi_x_bytes(int64_t ldg) { return sizeof(double) * (size_t)(ldg / NB) * NB * NB; }

// Measured on tau = 256 .. 5184 with 2 .. 31 sketches: the fused steps lead while a step's
// items fit on the chip about twice (tau = 512, 2 sketches: 199 us against 276 and 422),
// mode 1 in between (tau = 1024, 31 sketches: 1.76 ms against 3.38 and 2.00; tau = 2048, 16:
// 5.56 ms against 12.9 and 6.43), mode 2 once the tile products outweigh every chain
// (tau = 5184, 31 sketches: 138 ms against 146 and 397).
int chol_multi_mode(int64_t nt, int64_t nslots) {
  if (nslots * nt * nt <= 512) return 0;
  return nslots * nt * nt * nt > 4000000 ? 2 : 1;
}

// The XCD layout keeps a sketch's tiles in one L2; it pays with 8 or more sketches whose
// matrices are not far larger than the L2 (tau = 1024, 31 sketches: 1.92 ms against 2.15;
// tau = 5184: 165 ms against 161).
int chol_multi_xcd(int64_t nt, int64_t nslots) { return nslots >= 8 && nt <= 40 ? 1 : 0; }

// mode 0: one launch per step, each workgroup forming the L and W blocks it reads (three
// tile products per item, nt + 1 launches: the shortest chain); mode 1: panel and update
// launches per step (one tile product per item, a third of the work, 2 nt + 2 launches);
// mode 2: panel and update launches for the factorisation alone, then the inverse by
// distance and U U^T as chains of products accumulated in registers (each output tile
// written once: the least memory traffic, for large tau).
hipError_t launch_chol_multi_mode(double* G, double* U, double* X, int64_t ldg, int32_t tau,
                                  int32_t nslots, int32_t kind, const void* AS, int32_t as_f32,
                                  int64_t ldas, int64_t m, const int32_t* members, const int32_t* offs,
                                  int32_t* status, const int32_t* done, int mode, int xcd, hipStream_t s) {
  if (ldg % NB != 0) return hipErrorInvalidValue;
  MultiArgs a{G, U, X, ldg, (int32_t)(ldg / NB), tau, kind, AS, as_f32, ldas, m, members, offs,
              status, done, nslots, xcd >= 0 ? xcd : chol_multi_xcd(ldg / NB, nslots)};
  const int nt = a.nt;
  const size_t two = sizeof(double) * 2 * NB * LDT;
  const size_t three = sizeof(double) * 3 * NB * LDT;
  hipError_t e = hipFuncSetAttribute((const void*)k_chol_diag0, hipFuncAttributeMaxDynamicSharedMemorySize, (int)two);
  if (e == hipSuccess)
    e = hipFuncSetAttribute((const void*)k_chol_assemble<true>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)two);
  if (e == hipSuccess)
    e = hipFuncSetAttribute((const void*)k_chol_step, hipFuncAttributeMaxDynamicSharedMemorySize, (int)three);
  if (e == hipSuccess)
    e = hipFuncSetAttribute((const void*)k_chol_panel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)two);
  if (e == hipSuccess)
    e = hipFuncSetAttribute((const void*)k_chol_ll_inverse, hipFuncAttributeMaxDynamicSharedMemorySize, (int)two);
  if (e != hipSuccess) return e;
  if (mode == 0) {
    hipLaunchKernelGGL(k_chol_assemble<true>, dim3(nt * (nt + 1) / 2, 1, nslots), dim3(kThreads), two, s, a);
  } else {
    hipLaunchKernelGGL(k_chol_assemble<false>, dim3(nt * (nt + 1) / 2, 1, nslots), dim3(kThreads), 0, s, a);
    hipLaunchKernelGGL(k_chol_diag0, dim3(nslots), dim3(kThreads), two, s, a);
  }
  // grid of `items` work items per sketch in the layout item_of_block expects
  auto grid = [&](int items) {
    return a.xcd ? dim3((unsigned)(8 * ((nslots + 7) / 8) * items)) : dim3(items, nslots);
  };
  if (mode == 0) {
    for (int st = 1; st <= nt; ++st) {
      const int items = (nt - st) * (nt - st + 1) / 2 + (nt - st) * st + st * (st + 1) / 2;
      hipLaunchKernelGGL(k_chol_step, grid(items), dim3(kThreads), three, s, a, st);
    }
  } else {
    // Steps in pairs (st, st + 1): panel st, the narrow part of update st, panel st + 1 (its
    // diagonal tile also takes column st - 1's term), then one update for both columns; a
    // last unpaired step takes its own update. Mode 2 stops before step nt (no W, no G^{-1}).
    const int last = mode == 1 ? nt : nt - 1;
    auto nupd = [&](int st) {  // update items of step st (the diagonal tile left out)
      const int nF = (nt - st) * (nt - st + 1) / 2 - (st < nt ? 1 : 0);
      return mode == 1 ? nF + (nt - st) * st + st * (st + 1) / 2 : nF;
    };
    auto npanel = [&](int st) { return mode == 1 ? nt - 1 : nt - st; };
    int st = 1;
    while (st <= last) {
      if (st + 1 <= last) {
        const int nnar = (nt - st - 1) + (mode == 1 ? st : 0);
        hipLaunchKernelGGL(k_chol_panel, grid(npanel(st)), dim3(kThreads), two, s, a, st, npanel(st), -1);
        if (nnar > 0)
          hipLaunchKernelGGL(k_chol_narrow, grid(nnar), dim3(kThreads), 0, s, a, st, nnar, mode == 1 ? 1 : 0);
        hipLaunchKernelGGL(k_chol_panel, grid(npanel(st + 1)), dim3(kThreads), two, s, a, st + 1, npanel(st + 1),
                           st - 1);
        const int nu = nupd(st + 1);
        if (nu > 0) hipLaunchKernelGGL(k_chol_update, grid(nu), dim3(kThreads), 0, s, a, st + 1, nu, st - 1);
        st += 2;
      } else {
        hipLaunchKernelGGL(k_chol_panel, grid(npanel(st)), dim3(kThreads), two, s, a, st, npanel(st), -1);
        const int nu = nupd(st);
        if (nu > 0) hipLaunchKernelGGL(k_chol_update, grid(nu), dim3(kThreads), 0, s, a, st, nu, st - 1);
        st += 1;
      }
    }
  }
  if (mode == 2) {
    for (int d = 1; d < nt; ++d)
      hipLaunchKernelGGL(k_chol_ll_inverse, grid(nt - d), dim3(kThreads), two, s, a, d);
    hipLaunchKernelGGL(k_chol_lauum, grid(nt * (nt + 1) / 2), dim3(kThreads), 0, s, a);
  }
  return hipGetLastError();
}

hipError_t launch_chol_multi(double* G, double* U, double* X, int64_t ldg, int32_t tau,
                             int32_t nslots, int32_t kind, const void* AS, int32_t as_f32,
                             int64_t ldas, int64_t m, const int32_t* members, const int32_t* offs,
                             int32_t* status, const int32_t* done, hipStream_t s) {
  return launch_chol_multi_mode(G, U, X, ldg, tau, nslots, kind, AS, as_f32, ldas, m, members, offs, status,
                                done, chol_multi_mode(ldg / NB, nslots), -1, s);
}

}  // namespace rs
