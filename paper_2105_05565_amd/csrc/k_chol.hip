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
// which equals the pseudo-inverse solution. Padding to a multiple of 32 is the
// identity as well.
//
// Blocked algorithm on 32 x 32 tiles staged in LDS (256 threads, each owning a
// 1 x 4 strip of a tile):
//   1. right-looking Cholesky: factor diagonal tile, panel solve, trailing update;
//   2. W = L^{-1}: inverted diagonal tiles, W_ij = -W_ii sum_{k=j}^{i-1} L_ik W_kj;
//   3. G^{-1} = W^T W, written to both triangles.
#include "dev_common.h"
#include "rs_internal.h"

namespace rs {
namespace {

constexpr int NB = 32;
constexpr int kThreads = 256;

struct CholLds {
  double a[NB][NB + 1];
  double b[NB][NB + 1];
  double d[NB][NB + 1];
  int bad;
};

__device__ __forceinline__ void load_tile(double (*dst)[NB + 1], const double* src, int64_t ld,
                                          bool trans) {
  for (int e = threadIdx.x; e < NB * NB; e += kThreads) {
    const int r = e >> 5, c = e & 31;
    dst[r][c] = trans ? src[(int64_t)c * ld + r] : src[(int64_t)r * ld + c];
  }
}

// acc (this thread's 1 x 4 strip) += A * B with A, B in LDS.
__device__ __forceinline__ void tile_fma(double acc[4], double (*A)[NB + 1], double (*B)[NB + 1]) {
  const int r = threadIdx.x >> 3, c4 = (threadIdx.x & 7) * 4;
#pragma unroll 8
  for (int k = 0; k < NB; ++k) {
    const double av = A[r][k];
#pragma unroll
    for (int q = 0; q < 4; ++q) acc[q] += av * B[k][c4 + q];
  }
}

__device__ __forceinline__ void store_strip(double* dst, int64_t ld, const double acc[4]) {
  const int r = threadIdx.x >> 3, c4 = (threadIdx.x & 7) * 4;
#pragma unroll
  for (int q = 0; q < 4; ++q) dst[(int64_t)r * ld + c4 + q] = acc[q];
}

__device__ __forceinline__ void add_strip(double* dst, int64_t ld, const double acc[4], double alpha) {
  const int r = threadIdx.x >> 3, c4 = (threadIdx.x & 7) * 4;
#pragma unroll
  for (int q = 0; q < 4; ++q) dst[(int64_t)r * ld + c4 + q] += alpha * acc[q];
}

__global__ __launch_bounds__(kThreads) void k_chol_inverse(double* __restrict__ Gall,
                                                           double* __restrict__ Wall, int64_t ldg,
                                                           int32_t tau, int32_t kind,
                                                           const double* __restrict__ ASall, int64_t m,
                                                           const int32_t* __restrict__ members_all,
                                                           const int32_t* __restrict__ offs_all,
                                                           int32_t* __restrict__ status,
                                                           const int32_t* __restrict__ done) {
  __shared__ CholLds S;
  if (*done) return;
  const int tid = threadIdx.x;
  const int64_t slot = blockIdx.x;
  double* G = Gall + slot * ldg * ldg;
  double* W = Wall + slot * ldg * ldg;
  const int32_t* offs = offs_all + slot * (tau + 1);
  const int nt = (int)(ldg / NB);
  if (tid == 0) S.bad = 0;

  // Phase 0: assemble G (subsample: rows C of AS), padding and empty buckets.
  if (kind == kSubsample) {
    const int32_t* members = members_all + slot * tau;
    const double* AS = ASall + slot * m * tau;
    for (int64_t e = tid; e < (int64_t)tau * tau; e += kThreads) {
      const int64_t c = e / tau, cc = e % tau;
      G[c * ldg + cc] = AS[(int64_t)members[c] * tau + cc];
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

  // Phase 1: Cholesky, lower triangle in place.
  for (int kt = 0; kt < nt; ++kt) {
    double* Gkk = G + (int64_t)kt * NB * ldg + kt * NB;
    load_tile(S.d, Gkk, ldg, false);
    __syncthreads();
    for (int c = 0; c < NB; ++c) {
      if (tid == 0) {
        double piv = S.d[c][c];
        if (!(piv > 0.0) || !(piv < INFINITY)) {
          S.bad = 1;
          piv = 1.0;
        }
        S.d[c][c] = sqrt(piv);
      }
      __syncthreads();
      if (tid > c && tid < NB) S.d[tid][c] /= S.d[c][c];
      __syncthreads();
      for (int e = tid; e < NB * NB; e += kThreads) {
        const int r = e >> 5, cc = e & 31;
        if (cc > c && r >= cc) S.d[r][cc] -= S.d[r][c] * S.d[cc][c];
      }
      __syncthreads();
    }
    // zero the strict upper part; invert the diagonal tile into S.a (one column per thread)
    for (int e = tid; e < NB * NB; e += kThreads) {
      const int r = e >> 5, c = e & 31;
      if (c > r) S.d[r][c] = 0.0;
    }
    __syncthreads();
    if (tid < NB) {
      const int j = tid;
      for (int i = 0; i < NB; ++i) {
        double s = (i == j) ? 1.0 : 0.0;
        for (int t = j; t < i; ++t) s -= S.d[i][t] * S.a[t][j];
        S.a[i][j] = (i >= j) ? s / S.d[i][i] : 0.0;
      }
    }
    __syncthreads();
    for (int e = tid; e < NB * NB; e += kThreads) {
      const int r = e >> 5, c = e & 31;
      Gkk[(int64_t)r * ldg + c] = S.d[r][c];
      W[((int64_t)kt * NB + r) * ldg + kt * NB + c] = S.a[r][c];
    }
    __syncthreads();
    // panel: L_ik = G_ik * (L_kk^{-1})^T
    for (int e = tid; e < NB * NB; e += kThreads) {
      const int r = e >> 5, c = e & 31;
      S.b[r][c] = S.a[c][r];
    }
    __syncthreads();
    for (int it = kt + 1; it < nt; ++it) {
      double* Gik = G + (int64_t)it * NB * ldg + kt * NB;
      load_tile(S.a, Gik, ldg, false);
      __syncthreads();
      double acc[4] = {0.0, 0.0, 0.0, 0.0};
      tile_fma(acc, S.a, S.b);
      __syncthreads();
      store_strip(Gik, ldg, acc);
      __syncthreads();
    }
    // trailing update: G_ij -= L_ik L_jk^T for kt < jt <= it
    for (int jt = kt + 1; jt < nt; ++jt) {
      load_tile(S.b, G + (int64_t)jt * NB * ldg + kt * NB, ldg, true);
      for (int it = jt; it < nt; ++it) {
        load_tile(S.a, G + (int64_t)it * NB * ldg + kt * NB, ldg, false);
        __syncthreads();
        double acc[4] = {0.0, 0.0, 0.0, 0.0};
        tile_fma(acc, S.a, S.b);
        add_strip(G + (int64_t)it * NB * ldg + jt * NB, ldg, acc, -1.0);
        __syncthreads();
      }
    }
  }

  // Phase 2: W = L^{-1} below the diagonal tiles (diagonal tiles were stored above).
  for (int jt = 0; jt < nt; ++jt) {
    for (int it = jt + 1; it < nt; ++it) {
      double acc[4] = {0.0, 0.0, 0.0, 0.0};
      for (int kt = jt; kt < it; ++kt) {
        load_tile(S.a, G + (int64_t)it * NB * ldg + kt * NB, ldg, false);  // L_ik
        load_tile(S.b, W + (int64_t)kt * NB * ldg + jt * NB, ldg, false);  // W_kj
        __syncthreads();
        tile_fma(acc, S.a, S.b);
        __syncthreads();
      }
      {
        const int r = tid >> 3, c4 = (tid & 7) * 4;
#pragma unroll
        for (int q = 0; q < 4; ++q) S.d[r][c4 + q] = acc[q];
      }
      load_tile(S.a, W + (int64_t)it * NB * ldg + it * NB, ldg, false);  // W_ii
      __syncthreads();
      double out[4] = {0.0, 0.0, 0.0, 0.0};
      tile_fma(out, S.a, S.d);
#pragma unroll
      for (int q = 0; q < 4; ++q) out[q] = -out[q];
      store_strip(W + (int64_t)it * NB * ldg + jt * NB, ldg, out);
      __syncthreads();
    }
  }

  // Phase 3: G^{-1} = W^T W (both triangles of G).
  for (int it = 0; it < nt; ++it) {
    for (int jt = 0; jt <= it; ++jt) {
      double acc[4] = {0.0, 0.0, 0.0, 0.0};
      for (int kt = it; kt < nt; ++kt) {
        load_tile(S.a, W + (int64_t)kt * NB * ldg + it * NB, ldg, true);   // W_ki^T
        load_tile(S.b, W + (int64_t)kt * NB * ldg + jt * NB, ldg, false);  // W_kj
        __syncthreads();
        tile_fma(acc, S.a, S.b);
        __syncthreads();
      }
      const int r = tid >> 3, c4 = (tid & 7) * 4;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        G[((int64_t)it * NB + r) * ldg + jt * NB + c4 + q] = acc[q];
        if (jt != it) G[((int64_t)jt * NB + c4 + q) * ldg + it * NB + r] = acc[q];
      }
      __syncthreads();
    }
  }
  if (tid == 0) status[slot] = S.bad;
}

}  // namespace

hipError_t launch_chol_inverse(double* G, double* W, int64_t ldg, int32_t tau, int32_t nslots,
                               int32_t kind, const double* AS, int64_t m, const int32_t* members,
                               const int32_t* offs, int32_t* status, const int32_t* done,
                               hipStream_t s) {
  if (ldg % NB != 0) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_chol_inverse, dim3(nslots), dim3(kThreads), 0, s, G, W, ldg, tau, kind, AS,
                     m, members, offs, status, done);
  return hipGetLastError();
}

}  // namespace rs
