// 64 x 64 FP64 tile helpers for the sketched-matrix factorisation kernels:
// LDS staging and tile products on FP64 MFMA (16x16x4), 4 waves per workgroup.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace rs {
namespace chol {

constexpr int NB = 64;
constexpr int LDT = NB + 1;  // LDS row stride (odd: fewer bank conflicts)
constexpr int kThreads = 256;

typedef double d4v __attribute__((ext_vector_type(4)));

struct Acc {
  d4v v[2][2];
};

__device__ __forceinline__ void acc_zero(Acc& c) {
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) c.v[i][j] = d4v{0.0, 0.0, 0.0, 0.0};
}

// dst[r][c] = src[r * ld + c]  (trans: src[c * ld + r]) for a 64 x 64 tile.
__device__ __forceinline__ void load_tile(double* dst, const double* src, int64_t ld, bool trans) {
  for (int e = threadIdx.x; e < NB * NB; e += kThreads) {
    const int r = e >> 6, c = e & 63;
    dst[r * LDT + c] = trans ? src[(int64_t)c * ld + r] : src[(int64_t)r * ld + c];
  }
}

// C += A * B^T with A = a[r][k], B = b[c][k] (both 64 x 64 in LDS), K = 64.
// Wave w owns rows 32 (w / 2) .. +32 and columns 32 (w % 2) .. +32 of C.
__device__ __forceinline__ void tile_mma(Acc& c, const double* a, const double* b) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wr = (wave >> 1) * 32, wc = (wave & 1) * 32;
  const int l16 = lane & 15, lk = lane >> 4;
#pragma unroll 4
  for (int k4 = 0; k4 < NB; k4 += 4) {
    double av[2], bv[2];
#pragma unroll
    for (int i = 0; i < 2; ++i) av[i] = a[(wr + i * 16 + l16) * LDT + k4 + lk];
#pragma unroll
    for (int j = 0; j < 2; ++j) bv[j] = b[(wc + j * 16 + l16) * LDT + k4 + lk];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j)
        c.v[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[i], bv[j], c.v[i][j], 0, 0, 0);
  }
}

// Visit the accumulator elements: f(row, col, value) with (row, col) inside the tile.
// 16x16x4 FP64 MFMA result layout: lane l, element v -> row 4 v + l / 16, column l % 16.
template <class F>
__device__ __forceinline__ void acc_for_each(const Acc& c, F f) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wr = (wave >> 1) * 32, wc = (wave & 1) * 32;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v)
        f(wr + i * 16 + 4 * v + (lane >> 4), wc + j * 16 + (lane & 15), c.v[i][j][v]);
}

// Factor the 64 x 64 tile in td (LDS, lower triangle read) in place: td <- L (upper part
// zeroed) with L L^T = td, and ta <- X = L^{-1} (lower). col: 64 doubles of LDS scratch.
// A pivot that is not positive and finite is replaced by 1 and reported through *bad.
__device__ __forceinline__ void factor_diag_tile(double* td, double* ta, double* col, int* bad) {
  const int tid = threadIdx.x;
  for (int c = 0; c < NB; ++c) {
    if (tid < NB) {
      double piv = td[c * LDT + c];
      if (!(piv > 0.0) || !(piv < INFINITY)) {
        if (tid == c) *bad = 1;
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
  for (int e = tid; e < NB * NB; e += kThreads) {
    const int r = e >> 6, c = e & 63;
    if (c > r) td[r * LDT + c] = 0.0;
  }
  __syncthreads();
  // X = L^{-1} row by row (row i needs rows < i): thread j owns column j
  if (tid < NB) {
    const int j = tid;
    for (int i = 0; i < NB; ++i) {
      double s = (i == j) ? 1.0 : 0.0;
      for (int t = j; t < i; ++t) s -= td[i * LDT + t] * ta[t * LDT + j];
      ta[i * LDT + j] = (i >= j) ? s / td[i * LDT + i] : 0.0;
    }
  }
  __syncthreads();
}

}  // namespace chol
}  // namespace rs
