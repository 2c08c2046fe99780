// Device-wide blocked FP64 Cholesky and inverse of the sketched matrices G = S^T A S
// of a lookahead batch (least-norm solution of eq:sketched_system, delta = G^{-1} rho).
//
// The single-workgroup factorisation (k_chol.hip) runs one sketch per compute unit,
// which leaves most of the chip idle when a batch holds few sketches. Here every
// 64 x 64 tile of every sketch is a workgroup, and the sequential structure of the
// right-looking algorithm is carried by kernel boundaries on the stream:
//
//   assemble               G (gathered rows of AS for the subsample sketch), identity
//                          padding and empty buckets; U <- 0
//   for k = 0 .. nt-1:
//     diag_panel(k)        each workgroup factors G_kk = L_kk L_kk^T in LDS (redundantly)
//                          and forms X = L_kk^{-1}; workgroup k stores X and U_kk = X^T,
//                          workgroup i > k stores the panel L_ik = G_ik X^T, and
//                          workgroup j < k finishes U_jk <- U_jk X^T   (U = (L^{-1})^T)
//     trailing(k)          G_ij -= L_ik L_jk^T for k < j <= i, and the inverse step
//                          U_ji -= U_jk L_ik^T for i > k, j <= k
//   lauum                  G^{-1} = U U^T: tile (i, j) = sum_{k >= i} U_ik U_jk^T
//
// The inverse step uses W = L^{-1} computed right-looking (W_k* <- L_kk^{-1} W_k*,
// W_i* -= L_ik W_k* for i > k), stored transposed as U so that every tile product
// reads both operands row-major.
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

__global__ __launch_bounds__(kThreads) void k_chol_diag_panel(MultiArgs a, int kt) {
  extern __shared__ __align__(16) double lds[];
  double* ta = lds;
  double* tb = lds + NB * LDT;
  double* td = lds + 2 * NB * LDT;
  double* col = lds + 3 * NB * LDT;
  __shared__ int bad;
  if (*a.done) return;
  const int64_t slot = blockIdx.y;
  double* G = a.G + slot * a.ldg * a.ldg;
  double* U = a.U + slot * a.ldg * a.ldg;
  if (threadIdx.x == 0) bad = 0;
  // G_kk is only read in this launch (L_kk itself is not needed later), so every
  // workgroup can factor it.
  load_tile(td, tile(G, a.ldg, kt, kt), a.ldg, false);
  __syncthreads();
  factor_diag_tile(td, ta, col, &bad);
  const int npanel = a.nt - kt;
  if ((int)blockIdx.x >= npanel) {
    // finish column kt of U: U_jk <- U_jk X^T for j < kt (all updates were applied)
    const int j = (int)blockIdx.x - npanel;
    double* Ujk = tile(U, a.ldg, j, kt);
    load_tile(tb, Ujk, a.ldg, false);
    __syncthreads();
    Acc c;
    acc_zero(c);
    tile_mma(c, tb, ta);
    acc_for_each(c, [&](int r, int cc, double v) { Ujk[(int64_t)r * a.ldg + cc] = v; });
    return;
  }
  const int it = kt + (int)blockIdx.x;
  if (it == kt) {
    double* Ukk = tile(U, a.ldg, kt, kt);
    double* Xk = a.X + (slot * a.nt + kt) * NB * NB;
    for (int e = threadIdx.x; e < NB * NB; e += kThreads) {
      const int r = e >> 6, c = e & 63;
      Ukk[(int64_t)r * a.ldg + c] = ta[c * LDT + r];
      Xk[e] = ta[r * LDT + c];
    }
    if (threadIdx.x == 0 && bad) a.status[slot] = 1;
    return;
  }
  // panel: L_ik = G_ik X^T  (C = a b^T with a = G_ik, b = X)
  double* Gik = tile(G, a.ldg, it, kt);
  load_tile(tb, Gik, a.ldg, false);
  __syncthreads();
  Acc c;
  acc_zero(c);
  tile_mma(c, tb, ta);
  acc_for_each(c, [&](int r, int cc, double v) { Gik[(int64_t)r * a.ldg + cc] = v; });
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

// Operands are read straight from global memory (they are shared by many workgroups and stay
// in L2); without LDS many workgroups fit on a compute unit to cover the load latency.
__global__ __launch_bounds__(kThreads) void k_chol_trailing(MultiArgs a, int kt, int ntrail) {
  if (*a.done) return;
  const int64_t slot = blockIdx.y;
  double* G = a.G + slot * a.ldg * a.ldg;
  double* U = a.U + slot * a.ldg * a.ldg;
  int idx = blockIdx.x;
  Acc c;
  acc_zero(c);
  if (idx < ntrail) {
    // G_ij -= L_ik L_jk^T, kt < j <= i
    int i, j;
    lower_pair(idx, kt + 1, &i, &j);
    tile_mma_global(c, tile(G, a.ldg, i, kt), tile(G, a.ldg, j, kt), a.ldg);
    double* Gij = tile(G, a.ldg, i, j);
    acc_for_each(c, [&](int r, int cc, double v) { Gij[(int64_t)r * a.ldg + cc] -= v; });
    return;
  }
  // inverse step: U_ji -= U_jk L_ik^T for i > kt, j <= kt (column i is finished by
  // diag_panel(i), which scales it by X_ii^T)
  idx -= ntrail;
  const int i = kt + 1 + idx / (kt + 1), j = idx % (kt + 1);
  double* Uji = tile(U, a.ldg, j, i);
  tile_mma_global(c, tile(U, a.ldg, j, kt), tile(G, a.ldg, i, kt), a.ldg);  // U_jk L_ik^T
  acc_for_each(c, [&](int r, int cc, double v) { Uji[(int64_t)r * a.ldg + cc] -= v; });
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
  hipError_t e = hipFuncSetAttribute((const void*)k_chol_diag_panel,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)diag_bytes);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_chol_assemble, dim3(nt, nt, nslots), dim3(kThreads), 0, s, a);
  for (int kt = 0; kt < nt; ++kt) {
    hipLaunchKernelGGL(k_chol_diag_panel, dim3(nt, nslots), dim3(kThreads), diag_bytes, s, a, kt);
    const int rest = nt - kt - 1;
    const int ntrail = rest * (rest + 1) / 2;
    const int ninv = rest * (kt + 1);
    if (ntrail + ninv > 0)
      hipLaunchKernelGGL(k_chol_trailing, dim3(ntrail + ninv, nslots), dim3(kThreads), 0, s, a, kt, ntrail);
  }
  hipLaunchKernelGGL(k_chol_lauum, dim3(nt * (nt + 1) / 2, nslots), dim3(kThreads), 0, s, a);
  return hipGetLastError();
}

}  // namespace rs
