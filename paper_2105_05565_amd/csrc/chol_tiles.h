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

// C += A * B^T with A, B 64 x 64 tiles read straight from global memory (row stride ld, rows
// 32-byte aligned), no LDS: wave w owns rows 32 (w / 2) .. +32 and columns 32 (w % 2) .. +32 of
// C. A lane reads 4 consecutive k values of one row at once; the four 4-deep MFMA steps of a
// 16-wide chunk q then take k = 16 q + 4 g + s in lane group g = lane / 16 at step s, the same
// k for A and B, so every k term enters the sum once (in another order than tile_mma).
__device__ __forceinline__ void tile_mma_global(Acc& c, const double* __restrict__ A, const double* __restrict__ B,
                                                int64_t ld) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wr = (wave >> 1) * 32, wc = (wave & 1) * 32;
  const int l16 = lane & 15, g = lane >> 4;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    double4 av[2], bv[2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
      av[i] = *reinterpret_cast<const double4*>(A + (int64_t)(wr + i * 16 + l16) * ld + 16 * q + 4 * g);
#pragma unroll
    for (int j = 0; j < 2; ++j)
      bv[j] = *reinterpret_cast<const double4*>(B + (int64_t)(wc + j * 16 + l16) * ld + 16 * q + 4 * g);
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        c.v[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[i].x, bv[j].x, c.v[i][j], 0, 0, 0);
        c.v[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[i].y, bv[j].y, c.v[i][j], 0, 0, 0);
        c.v[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[i].z, bv[j].z, c.v[i][j], 0, 0, 0);
        c.v[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[i].w, bv[j].w, c.v[i][j], 0, 0, 0);
      }
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

// acc (16 x 16) += A B^T over K = 16 on FP64 MFMA, A(row, k) = pa[row * sar + k * sac],
// B(col, k) = pb[col * sbr + k * sbc]. Result element v of lane l: row 4 v + l / 16,
// column l % 16.
__device__ __forceinline__ void mma16(d4v& acc, const double* pa, int sar, int sac, const double* pb, int sbr,
                                      int sbc) {
  const int lane = threadIdx.x & 63, l16 = lane & 15, lk = lane >> 4;
#pragma unroll
  for (int k4 = 0; k4 < 16; k4 += 4) {
    const double av = pa[l16 * sar + (k4 + lk) * sac];
    const double bv = pb[l16 * sbr + (k4 + lk) * sbc];
    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc, 0, 0, 0);
  }
}

__device__ __forceinline__ double* blk16(double* t, int i, int j) { return t + (i * 16) * LDT + j * 16; }

// The value of v in lane l (a compile-time lane after unrolling), as a wave-uniform scalar.
__device__ __forceinline__ double lane_value(double v, int l) {
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), l);
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), l);
  return __hiloint2double(hi, lo);
}

// Factor the 64 x 64 tile in td (LDS, lower triangle read) in place: td <- L (upper part
// zeroed) with L L^T = td, and ta <- X = L^{-1} (lower, upper part zeroed). A pivot that
// is not positive and finite is replaced by 1 and reported through *bad. col: LDS scratch
// (unused). Called by all threads of the workgroup.
//
// Blocked on 16 x 16 sub-blocks, right-looking: wave 0 factors and inverts the diagonal
// block in registers (lane r holds row r, column values read as scalars from their lane), the
// panel L_ik = A_ik X_kk^T and the trailing update A_ij -= L_ik L_jk^T are FP64 MFMA
// products spread over the waves. Then X_ij = -X_ii sum_{k=j}^{i-1} L_ik X_kj by
// distance i - j, the partial sums parked in the unused upper blocks of td.
__device__ __forceinline__ void factor_diag_tile(double* td, double* ta, double* col, int* bad) {
  (void)col;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  constexpr int kNW = kThreads / 64;
  for (int kb = 0; kb < 4; ++kb) {
    if (wave == 0) {
      // rows of the diagonal block in lanes 0-15 (lanes >= 16 carry copies, not stored)
      const int r = lane & 15;
      double* D = blk16(td, kb, kb);
      double d[16];
#pragma unroll
      for (int c = 0; c < 16; ++c) d[c] = D[r * LDT + c];
      int badl = 0;
#pragma unroll
      for (int c = 0; c < 16; ++c) {
        double piv = lane_value(d[c], c);
        if (!(piv > 0.0) || !(piv < INFINITY)) {
          badl = 1;
          piv = 1.0;
        }
        const double sq = sqrt(piv);
        const double l = r > c ? d[c] / sq : (r == c ? sq : 0.0);
        d[c] = l;
#pragma unroll
        for (int cc = c + 1; cc < 16; ++cc) d[cc] -= l * lane_value(l, cc);
      }
      // X_kk = L_kk^{-1}: lane j solves for column j (rows i < j come out zero)
      const int j = r;
      double x[16];
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        double s = (i == j) ? 1.0 : 0.0;
#pragma unroll
        for (int t = 0; t < i; ++t) s -= lane_value(d[t], i) * x[t];
        x[i] = s / lane_value(d[i], i);
      }
      if (lane < 16) {
        double* X = blk16(ta, kb, kb);
#pragma unroll
        for (int c = 0; c < 16; ++c) {
          D[r * LDT + c] = c <= r ? d[c] : 0.0;
          X[c * LDT + j] = x[c];
        }
        if (badl) *bad = 1;
      }
    }
    __syncthreads();
    // panel: L_ik = A_ik X_kk^T
    for (int i = kb + 1 + wave; i < 4; i += kNW) {
      d4v acc = {0.0, 0.0, 0.0, 0.0};
      double* Aik = blk16(td, i, kb);
      mma16(acc, Aik, LDT, 1, blk16(ta, kb, kb), LDT, 1);
#pragma unroll
      for (int v = 0; v < 4; ++v) Aik[(4 * v + (lane >> 4)) * LDT + (lane & 15)] = acc[v];
    }
    __syncthreads();
    // trailing: A_ij -= L_ik L_jk^T for kb < j <= i
    {
      int q = 0;
      for (int i = kb + 1; i < 4; ++i)
        for (int j = kb + 1; j <= i; ++j, ++q) {
          if (q % kNW != wave) continue;
          d4v acc = {0.0, 0.0, 0.0, 0.0};
          mma16(acc, blk16(td, i, kb), LDT, 1, blk16(td, j, kb), LDT, 1);
          double* Aij = blk16(td, i, j);
#pragma unroll
          for (int v = 0; v < 4; ++v) Aij[(4 * v + (lane >> 4)) * LDT + (lane & 15)] -= acc[v];
        }
    }
    __syncthreads();
  }
  // X below the diagonal blocks, by distance dd = i - j
  for (int dd = 1; dd < 4; ++dd) {
    // T_ij = sum_{k=j}^{i-1} L_ik X_kj, parked in td block (j, i)
    for (int j = wave; j + dd < 4; j += kNW) {
      const int i = j + dd;
      d4v acc = {0.0, 0.0, 0.0, 0.0};
      for (int k = j; k < i; ++k) mma16(acc, blk16(td, i, k), LDT, 1, blk16(ta, k, j), 1, LDT);
      double* T = blk16(td, j, i);
#pragma unroll
      for (int v = 0; v < 4; ++v) T[(4 * v + (lane >> 4)) * LDT + (lane & 15)] = acc[v];
    }
    __syncthreads();
    // X_ij = -X_ii T_ij
    for (int j = wave; j + dd < 4; j += kNW) {
      const int i = j + dd;
      d4v acc = {0.0, 0.0, 0.0, 0.0};
      mma16(acc, blk16(ta, i, i), LDT, 1, blk16(td, j, i), 1, LDT);
      double* X = blk16(ta, i, j);
#pragma unroll
      for (int v = 0; v < 4; ++v) X[(4 * v + (lane >> 4)) * LDT + (lane & 15)] = -acc[v];
    }
    __syncthreads();
  }
  // zero the blocks above the diagonal in both tiles
  for (int e = tid; e < NB * NB; e += kThreads) {
    const int r = e >> 6, c = e & 63;
    if ((c >> 4) > (r >> 4)) {
      td[r * LDT + c] = 0.0;
      ta[r * LDT + c] = 0.0;
    }
  }
  __syncthreads();
}

}  // namespace chol
}  // namespace rs
