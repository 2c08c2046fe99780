// FP64 Cholesky factorisation and inverse of the sketched matrix G = S^T A S.
//
// The least-norm solution of G delta = S^T r (eq:sketched_system) is computed as
// delta = G^{-1} rho with G^{-1} = L^{-T} L^{-1} from the Cholesky factor L of the
// lower triangle of G. The factorisation does not depend on the iterate, so it is
// computed ahead for a batch of sketches, one workgroup per sketch, and the
// per-iteration critical path keeps a single matrix-vector product.
//
// A column of S that is zero (an empty count bucket) makes the matching row and
// column of G zero and rho_b = 0; the diagonal entry is set to 1 so that delta_b = 0,
// which equals the pseudo-inverse solution. Padding to a multiple of 64 is the
// identity as well.
//
// Blocked algorithm on 64 x 64 tiles (4 waves, FP64 MFMA 16x16x4 for tile products,
// operands staged in LDS), with U = L^{-T} (upper triangular) kept instead of L^{-1}
// so that every tile product reads its operands row-major:
//   1. right-looking Cholesky: factor the diagonal tile and invert it in LDS,
//      panel L_ik = G_ik U_kk, trailing update G_ij -= L_ik L_jk^T;
//   2. U_ji = -(sum_{k=j}^{i-1} U_jk L_ik^T) U_ii for i > j  (U = (L^{-1})^T);
//   3. G^{-1} = U U^T, tile (i, j) = sum_{k >= max(i,j)} U_ik U_jk^T, both triangles.
#include "chol_tiles.h"
#include "dev_common.h"
#include "rs_internal.h"

namespace rs {
namespace {

using namespace chol;

// Phases 1-3 on the assembled, padded ldg x ldg matrix G (lower triangle read):
// G <- G^{-1} (both triangles), U <- L^{-T}. LDS: ta, tb, td (64 x LDT each), col (64).
__device__ __forceinline__ void factor_invert(double* __restrict__ G, double* __restrict__ U,
                                              int64_t ldg, double* ta, double* tb, double* td,
                                              double* col, int* bad_flag) {
  const int tid = threadIdx.x;
  const int nt = (int)(ldg / NB);
  int& bad = *bad_flag;
  // Phase 1: Cholesky (lower triangle of G in place) and U_kk = L_kk^{-T}.
  for (int kt = 0; kt < nt; ++kt) {
    double* Gkk = G + (int64_t)kt * NB * ldg + kt * NB;
    load_tile(td, Gkk, ldg, false);
    __syncthreads();
    for (int c = 0; c < NB; ++c) {
      if (tid < NB) {
        double piv = td[c * LDT + c];
        if (!(piv > 0.0) || !(piv < INFINITY)) {
          if (tid == c) bad = 1;
          piv = 1.0;
        }
        const double sq = sqrt(piv);
        col[tid] = (tid == c) ? sq : (tid > c ? td[tid * LDT + c] / sq : 0.0);
      }
      __syncthreads();
      for (int e = tid; e < NB * NB; e += kThreads) {
        const int r = e >> 6, cc = e & 63;
        if (cc == c && r >= c) td[r * LDT + c] = col[r];
        else if (cc > c && r >= cc) td[r * LDT + cc] -= col[r] * col[cc];
      }
      __syncthreads();
    }
    // X = L_kk^{-1} row by row (row i needs rows < i): thread j owns column j, ta[i][j] = X[i][j]
    if (tid < NB) {
      const int j = tid;
      for (int i = 0; i < NB; ++i) {
        double s = (i == j) ? 1.0 : 0.0;
        for (int t = j; t < i; ++t) s -= td[i * LDT + t] * ta[t * LDT + j];
        ta[i * LDT + j] = (i >= j) ? s / td[i * LDT + i] : 0.0;
      }
    }
    __syncthreads();
    // write L_kk (upper part zero) and U_kk = X^T; tb[c][k] = U_kk[k][c] = X[c][k] for the panel
    double* Ukk = U + (int64_t)kt * NB * ldg + kt * NB;
    for (int e = tid; e < NB * NB; e += kThreads) {
      const int r = e >> 6, c = e & 63;
      Gkk[(int64_t)r * ldg + c] = (c <= r) ? td[r * LDT + c] : 0.0;
      Ukk[(int64_t)r * ldg + c] = ta[c * LDT + r];
      tb[r * LDT + c] = ta[r * LDT + c];
    }
    __syncthreads();
    // panel: L_ik = G_ik U_kk
    for (int it = kt + 1; it < nt; ++it) {
      double* Gik = G + (int64_t)it * NB * ldg + kt * NB;
      load_tile(ta, Gik, ldg, false);
      __syncthreads();
      Acc c;
      acc_zero(c);
      tile_mma(c, ta, tb);
      __syncthreads();
      acc_for_each(c, [&](int r, int cc, double v) { Gik[(int64_t)r * ldg + cc] = v; });
      __syncthreads();
    }
    // trailing update: G_ij -= L_ik L_jk^T for kt < jt <= it
    for (int jt = kt + 1; jt < nt; ++jt) {
      load_tile(tb, G + (int64_t)jt * NB * ldg + kt * NB, ldg, false);  // tb[c][k] = L_jk[c][k]
      for (int it = jt; it < nt; ++it) {
        load_tile(ta, G + (int64_t)it * NB * ldg + kt * NB, ldg, false);
        __syncthreads();
        Acc c;
        acc_zero(c);
        tile_mma(c, ta, tb);
        double* Gij = G + (int64_t)it * NB * ldg + jt * NB;
        acc_for_each(c, [&](int r, int cc, double v) { Gij[(int64_t)r * ldg + cc] -= v; });
        __syncthreads();
      }
    }
  }

  // Phase 2: U_ji = -(sum_{k=j}^{i-1} U_jk L_ik^T) U_ii for i > j.
  for (int jt = 0; jt < nt; ++jt) {
    for (int it = jt + 1; it < nt; ++it) {
      Acc c;
      acc_zero(c);
      for (int kt = jt; kt < it; ++kt) {
        load_tile(ta, U + (int64_t)jt * NB * ldg + kt * NB, ldg, false);  // ta = U_jk
        load_tile(tb, G + (int64_t)it * NB * ldg + kt * NB, ldg, false);  // tb[c][k] = L_ik[c][k]
        __syncthreads();
        tile_mma(c, ta, tb);
        __syncthreads();
      }
      acc_for_each(c, [&](int r, int cc, double v) { ta[r * LDT + cc] = v; });
      load_tile(tb, U + (int64_t)it * NB * ldg + it * NB, ldg, true);  // tb[c][k] = U_ii[k][c]
      __syncthreads();
      Acc o;
      acc_zero(o);
      tile_mma(o, ta, tb);
      double* Uji = U + (int64_t)jt * NB * ldg + it * NB;
      acc_for_each(o, [&](int r, int cc, double v) { Uji[(int64_t)r * ldg + cc] = -v; });
      __syncthreads();
    }
  }

  // Phase 3: G^{-1} = U U^T, tile (i, j) = sum_{k >= i} U_ik U_jk^T for i >= j.
  for (int it = 0; it < nt; ++it) {
    for (int jt = 0; jt <= it; ++jt) {
      Acc c;
      acc_zero(c);
      for (int kt = it; kt < nt; ++kt) {
        load_tile(ta, U + (int64_t)it * NB * ldg + kt * NB, ldg, false);  // ta = U_ik
        load_tile(tb, U + (int64_t)jt * NB * ldg + kt * NB, ldg, false);  // tb[c][k] = U_jk[c][k]
        __syncthreads();
        tile_mma(c, ta, tb);
        __syncthreads();
      }
      double* Gij = G + (int64_t)it * NB * ldg + jt * NB;
      double* Gji = G + (int64_t)jt * NB * ldg + it * NB;
      acc_for_each(c, [&](int r, int cc, double v) {
        Gij[(int64_t)r * ldg + cc] = v;
        if (jt != it) Gji[(int64_t)cc * ldg + r] = v;
      });
      __syncthreads();
    }
  }
}

template <typename ASV>
__global__ __launch_bounds__(kThreads) void k_chol_inverse(double* __restrict__ Gall,
                                                           double* __restrict__ Uall, int64_t ldg,
                                                           int32_t tau, int32_t kind,
                                                           const ASV* __restrict__ ASall,
                                                           int64_t ldas, int64_t m,
                                                           const int32_t* __restrict__ members_all,
                                                           const int32_t* __restrict__ offs_all,
                                                           int32_t* __restrict__ status,
                                                           const int32_t* __restrict__ done) {
  extern __shared__ __align__(16) double lds[];
  double* ta = lds;                  // [64][65]
  double* tb = lds + NB * LDT;       // [64][65]
  double* td = lds + 2 * NB * LDT;   // [64][65]
  double* col = lds + 3 * NB * LDT;  // [64]
  __shared__ int bad;
  if (*done) return;
  const int tid = threadIdx.x;
  const int64_t slot = blockIdx.x;
  double* G = Gall + slot * ldg * ldg;
  double* U = Uall + slot * ldg * ldg;
  const int32_t* offs = offs_all + slot * (tau + 1);
  if (tid == 0) bad = 0;

  // Phase 0: assemble G (subsample: rows C of AS), padding and empty buckets.
  if (kind == kSubsample) {
    const int32_t* members = members_all + slot * tau;
    const ASV* AS = ASall + slot * m * ldas;
    for (int64_t e = tid; e < (int64_t)tau * tau; e += kThreads) {
      const int64_t c = e / tau, cc = e % tau;
      G[c * ldg + cc] = (double)AS[(int64_t)members[c] * ldas + cc];
    }
  }
  for (int64_t e = tid; e < ldg * ldg; e += kThreads) {
    const int64_t r = e / ldg, c = e % ldg;
    if (r >= tau || c >= tau) G[e] = (r == c) ? 1.0 : 0.0;
  }
  __syncthreads();
  if (kind != kSubsample) {
    for (int bkt = tid; bkt < tau; bkt += kThreads)
      if (offs[bkt + 1] == offs[bkt]) G[(int64_t)bkt * ldg + bkt] = 1.0;
  }
  __syncthreads();

  factor_invert(G, U, ldg, ta, tb, td, col, &bad);
  if (tid == 0) status[slot] = bad;
}


// Grouped form (batched solves): job = one (problem, lambda) pair sharing the
// problem's product B S = Z (Z^T S) (no lambda term), so that
// S^T A(lambda) S = S^T B S + lambda S^T S. Subsample: rows C of B S plus lambda I;
// count: G0 = S^T B S plus lambda diag(bucket sizes) (S^T S for a count sketch), the
// diagonal of an empty bucket set to 1. Persistent grid striding over the jobs.
__global__ __launch_bounds__(kThreads) void k_chol_tab(const CholJob* __restrict__ jobs, int32_t njobs) {
  extern __shared__ __align__(16) double lds[];
  double* ta = lds;
  double* tb = lds + NB * LDT;
  double* td = lds + 2 * NB * LDT;
  double* col = lds + 3 * NB * LDT;
  __shared__ int bad;
  const int tid = threadIdx.x;
  for (int32_t t = blockIdx.x; t < njobs; t += gridDim.x) {
    const CholJob& j = jobs[t];
    if (*j.done) continue;  // uniform across the workgroup
    double* G = j.G;
    const int64_t ldg = j.ldg;
    const int tau = j.tau;
    if (tid == 0) bad = 0;
    for (int64_t e = tid; e < ldg * ldg; e += kThreads) {
      const int64_t r = e / ldg, c = e % ldg;
      double v;
      if (r >= tau || c >= tau) {
        v = (r == c) ? 1.0 : 0.0;
      } else if (j.kind == kSubsample) {
        v = j.BS[(int64_t)j.members[r] * j.ldas + c];
        if (r == c) v += j.lam;
      } else {
        v = j.G0[r * ldg + c];
        if (r == c) {
          const int cnt = j.offs[r + 1] - j.offs[r];
          v = cnt == 0 ? 1.0 : v + j.lam * (double)cnt;
        }
      }
      G[e] = v;
    }
    __syncthreads();
    factor_invert(G, j.U, ldg, ta, tb, td, col, &bad);
    if (tid == 0 && bad) *j.status = 1;  // sticky until the host clears it
    __syncthreads();
  }
}

template <typename ASV>
hipError_t chol_launch(double* G, double* W, int64_t ldg, int32_t tau, int32_t nslots, int32_t kind,
                       const ASV* AS, int64_t ldas, int64_t m, const int32_t* members,
                       const int32_t* offs, int32_t* status, const int32_t* done, hipStream_t s) {
  if (ldg % NB != 0) return hipErrorInvalidValue;
  const size_t bytes = sizeof(double) * (3 * NB * LDT + NB);
  hipError_t e = hipFuncSetAttribute((const void*)k_chol_inverse<ASV>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_chol_inverse<ASV>, dim3(nslots), dim3(kThreads), bytes, s, G, W, ldg, tau,
                     kind, AS, ldas, m, members, offs, status, done);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_chol_inverse(double* G, double* W, int64_t ldg, int32_t tau, int32_t nslots,
                               int32_t kind, const void* AS, int32_t as_f32, int64_t ldas, int64_t m,
                               const int32_t* members, const int32_t* offs, int32_t* status,
                               const int32_t* done, hipStream_t s) {
  if (as_f32)
    return chol_launch<float>(G, W, ldg, tau, nslots, kind, (const float*)AS, ldas, m, members, offs,
                              status, done, s);
  return chol_launch<double>(G, W, ldg, tau, nslots, kind, (const double*)AS, ldas, m, members, offs,
                             status, done, s);
}

hipError_t launch_chol_tab(const CholJob* jobs, int32_t njobs, int32_t grid, hipStream_t s) {
  if (njobs <= 0) return hipSuccess;
  grid = grid < 1 ? 1 : (grid > njobs ? njobs : grid);
  const size_t bytes = sizeof(double) * (3 * NB * LDT + NB);
  hipError_t e = hipFuncSetAttribute((const void*)k_chol_tab, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)bytes);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_chol_tab, dim3(grid), dim3(kThreads), bytes, s, jobs, njobs);
  return hipGetLastError();
}

}  // namespace rs
