// Device-wide blocked FP64 Cholesky and inverse of the sketched matrices G = S^T A S
// of a lookahead batch (least-norm solution of eq:sketched_system, delta = G^{-1} rho).
//
// The single-workgroup factorisation (k_chol.hip) runs one sketch per compute unit,
// which leaves most of the chip idle when a batch holds few sketches. Here every
// 64 x 64 tile of every sketch is a workgroup, and the sequential structure of a
// right-looking algorithm is carried by kernel boundaries on the stream: the diagonal
// factorisation of step j never waits for a chain of tile products, because the trailing
// update of step j - 1 (one tile product per workgroup, all tiles at once) has already
// brought G_jj up to date:
//
//   assemble               G (gathered rows of AS for the subsample sketch), identity
//                          padding and empty buckets; U <- 0
//   for j = 0 .. nt-1:
//     diag(j)              G_jj = L_jj L_jj^T factored in LDS; X_jj = L_jj^{-1} stored,
//                          and U_jj = X_jj^T
//     panel(j)             L_ij = G_ij X_jj^T for i > j, over G_ij
//     trail(j)             G_il -= L_ij L_lj^T for j < l <= i
//   for d = 1 .. nt-1:
//     ll_inverse(d)        W = L^{-1} by distance d = i - j: W_ij = -X_ii sum_{k=j}^{i-1} L_ik W_kj,
//                          stored transposed as U_ji (U = L^{-T}, so W_kj = U_jk^T)
//   lauum                  G^{-1} = U U^T: tile (i, j) = sum_{k >= i} U_ik U_jk^T
//
// Tile products read their operands straight from global memory (they are shared by many
// workgroups and stay in L2), so that many workgroups fit on a compute unit.
#include "chol_tiles.h"
#include "dev_common.h"
#include "rs_internal.h"

namespace rs {
namespace {

using namespace chol;

struct MultiArgs {
  double* G;      // [slots][ldg][ldg]
  double* U;      // [slots][ldg][ldg]
  double* X;      // [slots][nt][64][64]  L_kk^{-1}
  int64_t ldg;
  int32_t nt, tau, kind;
  const void* AS;
  int32_t as_f32;
  int64_t ldas, m;
  const int32_t* members;
  const int32_t* offs;
  int32_t* status;
  const int32_t* done;
};

__device__ __forceinline__ double* tile(double* base, int64_t ld, int i, int j) {
  return base + (int64_t)i * NB * ld + (int64_t)j * NB;
}

__global__ __launch_bounds__(kThreads) void k_chol_assemble(MultiArgs a) {
  if (*a.done) return;
  const int64_t slot = blockIdx.z;
  const int ti = blockIdx.y, tj = blockIdx.x;
  double* G = a.G + slot * a.ldg * a.ldg;
  double* U = a.U + slot * a.ldg * a.ldg;
  const int32_t* offs = a.offs + slot * (a.tau + 1);
  const int32_t* members = a.members + slot * a.tau;  // subsample: nsel = tau
  for (int e = threadIdx.x; e < NB * NB; e += kThreads) {
    const int r = e >> 6, c = e & 63;
    const int64_t gr = (int64_t)ti * NB + r, gc = (int64_t)tj * NB + c;
    double* g = G + gr * a.ldg + gc;
    if (gr >= a.tau || gc >= a.tau) {
      *g = (gr == gc) ? 1.0 : 0.0;
    } else if (a.kind == kSubsample) {
      const int64_t src = (slot * a.m + members[gr]) * a.ldas + gc;
      *g = a.as_f32 ? (double)((const float*)a.AS)[src] : ((const double*)a.AS)[src];
    } else if (gr == gc && offs[gr + 1] == offs[gr]) {
      *g = 1.0;  // empty bucket: zero row and column of S^T A S
    }
    U[gr * a.ldg + gc] = 0.0;
  }
  if (ti == 0 && tj == 0 && threadIdx.x == 0) a.status[slot] = 0;
}

// Linear index -> (i, j) with lo <= j <= i < nt (row-major over i).
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

// Step j's diagonal tile (already updated by the trailing updates of steps < j) factored in
// LDS: X_jj = L_jj^{-1} kept for the panel and the inverse, U_jj = X_jj^T.
__global__ __launch_bounds__(kThreads) void k_chol_diag(MultiArgs a, int j) {
  extern __shared__ __align__(16) double lds[];
  double* ta = lds;
  double* td = lds + NB * LDT;
  double* col = lds + 2 * NB * LDT;
  __shared__ int bad;
  if (*a.done) return;
  const int64_t slot = blockIdx.x;
  double* G = a.G + slot * a.ldg * a.ldg;
  double* U = a.U + slot * a.ldg * a.ldg;
  if (threadIdx.x == 0) bad = 0;
  load_tile(td, tile(G, a.ldg, j, j), a.ldg, false);
  __syncthreads();
  factor_diag_tile(td, ta, col, &bad);
  double* Ujj = tile(U, a.ldg, j, j);
  double* Xj = a.X + (slot * a.nt + j) * NB * NB;
  for (int e = threadIdx.x; e < NB * NB; e += kThreads) {
    const int r = e >> 6, cc = e & 63;
    Ujj[(int64_t)r * a.ldg + cc] = ta[cc * LDT + r];
    Xj[e] = ta[r * LDT + cc];
  }
  if (threadIdx.x == 0 && bad) a.status[slot] = 1;
}

// L_ij = G_ij X_jj^T for the tiles i > j of column j (G_ij already updated), over G_ij.
__global__ __launch_bounds__(kThreads) void k_chol_panel(MultiArgs a, int j) {
  extern __shared__ __align__(16) double lds[];
  double* tp = lds;
  double* tx = lds + NB * LDT;
  if (*a.done) return;
  const int64_t slot = blockIdx.y;
  const int i = j + 1 + (int)blockIdx.x;
  double* G = a.G + slot * a.ldg * a.ldg;
  double* Gij = tile(G, a.ldg, i, j);
  load_tile(tp, Gij, a.ldg, false);
  load_tile(tx, a.X + (slot * a.nt + j) * NB * NB, NB, false);
  __syncthreads();
  Acc c;
  acc_zero(c);
  tile_mma(c, tp, tx);  // G_ij X_jj^T
  acc_for_each(c, [&](int r, int cc, double v) { Gij[(int64_t)r * a.ldg + cc] = v; });
}

// Trailing update of step j: G_il -= L_ij L_lj^T for every j < l <= i < nt, one tile per
// workgroup (each element read and written by one lane).
__global__ __launch_bounds__(kThreads) void k_chol_trail(MultiArgs a, int j) {
  if (*a.done) return;
  const int64_t slot = blockIdx.y;
  int i, l;
  lower_pair(blockIdx.x, j + 1, &i, &l);
  double* G = a.G + slot * a.ldg * a.ldg;
  Acc c;
  acc_zero(c);
  tile_mma_global(c, tile(G, a.ldg, i, j), tile(G, a.ldg, l, j), a.ldg);
  double* Gil = tile(G, a.ldg, i, l);
  acc_for_each(c, [&](int r, int cc, double v) { Gil[(int64_t)r * a.ldg + cc] -= v; });
}

__global__ __launch_bounds__(kThreads) void k_chol_ll_inverse(MultiArgs a, int d) {
  extern __shared__ __align__(16) double lds[];
  double* tt = lds;
  double* tx = lds + NB * LDT;
  if (*a.done) return;
  const int64_t slot = blockIdx.y;
  const int j = (int)blockIdx.x, i = j + d;
  double* G = a.G + slot * a.ldg * a.ldg;
  double* U = a.U + slot * a.ldg * a.ldg;
  Acc c;
  acc_zero(c);
  for (int k = j; k < i; ++k) tile_mma_global(c, tile(G, a.ldg, i, k), tile(U, a.ldg, j, k), a.ldg);
  // T = sum_k L_ik W_kj; U_ji = W_ij^T = -T^T X_ii^T
  acc_for_each(c, [&](int r, int cc, double v) { tt[cc * LDT + r] = v; });
  load_tile(tx, a.X + (slot * a.nt + i) * NB * NB, NB, false);
  __syncthreads();
  Acc c2;
  acc_zero(c2);
  tile_mma(c2, tt, tx);
  double* Uji = tile(U, a.ldg, j, i);
  acc_for_each(c2, [&](int r, int cc, double v) { Uji[(int64_t)r * a.ldg + cc] = -v; });
}

__global__ __launch_bounds__(kThreads) void k_chol_lauum(MultiArgs a) {
  if (*a.done) return;
  const int64_t slot = blockIdx.y;
  int i, j;
  lower_pair(blockIdx.x, 0, &i, &j);
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

hipError_t launch_chol_multi(double* G, double* U, double* X, int64_t ldg, int32_t tau,
                             int32_t nslots, int32_t kind, const void* AS, int32_t as_f32,
                             int64_t ldas, int64_t m, const int32_t* members, const int32_t* offs,
                             int32_t* status, const int32_t* done, hipStream_t s) {
  if (ldg % NB != 0) return hipErrorInvalidValue;
  MultiArgs a{G, U, X, ldg, (int32_t)(ldg / NB), tau, kind, AS, as_f32, ldas, m, members, offs,
              status, done};
  const int nt = a.nt;
  const size_t diag_bytes = sizeof(double) * (3 * NB * LDT + NB);
  const size_t pair_bytes = sizeof(double) * 2 * NB * LDT;
  hipError_t e = hipFuncSetAttribute((const void*)k_chol_diag, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)diag_bytes);
  if (e == hipSuccess)
    e = hipFuncSetAttribute((const void*)k_chol_panel, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)pair_bytes);
  if (e == hipSuccess)
    e = hipFuncSetAttribute((const void*)k_chol_ll_inverse, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)pair_bytes);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_chol_assemble, dim3(nt, nt, nslots), dim3(kThreads), 0, s, a);
  for (int j = 0; j < nt; ++j) {
    hipLaunchKernelGGL(k_chol_diag, dim3(nslots), dim3(kThreads), diag_bytes, s, a, j);
    const int below = nt - j - 1;
    if (below > 0) {
      hipLaunchKernelGGL(k_chol_panel, dim3(below, nslots), dim3(kThreads), pair_bytes, s, a, j);
      hipLaunchKernelGGL(k_chol_trail, dim3(below * (below + 1) / 2, nslots), dim3(kThreads), 0, s, a, j);
    }
  }
  for (int d = 1; d < nt; ++d)
    hipLaunchKernelGGL(k_chol_ll_inverse, dim3(nt - d, nslots), dim3(kThreads), pair_bytes, s, a, d);
  hipLaunchKernelGGL(k_chol_lauum, dim3(nt * (nt + 1) / 2, nslots), dim3(kThreads), 0, s, a);
  return hipGetLastError();
}

}  // namespace rs
