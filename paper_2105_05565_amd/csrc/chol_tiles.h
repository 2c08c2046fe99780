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

// dst[r][c] = src[r * ld + c]  (trans: src[c * ld + r]) for a 64 x 64 tile (src and ld
// even, so that a pair of neighbouring elements is one 16-byte load). Each thread issues
// its 8 loads before the first LDS store, so the tile costs one memory latency.
__device__ __forceinline__ void load_tile(double* dst, const double* src, int64_t ld, bool trans) {
  double2 v[8];
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const int e = threadIdx.x + kThreads * q, r = e >> 5, c = 2 * (e & 31);
    v[q] = *reinterpret_cast<const double2*>(src + (int64_t)r * ld + c);
  }
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const int e = threadIdx.x + kThreads * q, r = e >> 5, c = 2 * (e & 31);
    if (trans) {
      dst[c * LDT + r] = v[q].x;
      dst[(c + 1) * LDT + r] = v[q].y;
    } else {
      dst[r * LDT + c] = v[q].x;
      dst[r * LDT + c + 1] = v[q].y;
    }
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

// c <- the 64 x 64 tile at src (row stride ld) in the accumulator layout of acc_for_each.
__device__ __forceinline__ void acc_load(Acc& c, const double* src, int64_t ld) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wr = (wave >> 1) * 32, wc = (wave & 1) * 32;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v)
        c.v[i][j][v] = src[(int64_t)(wr + i * 16 + 4 * v + (lane >> 4)) * ld + wc + j * 16 + (lane & 15)];
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

// The value of v in lane l of this lane's 16-lane row (DPP row_newbcast), for a lane index
// that is a constant once the caller's loops are unrolled.
template <int L>
__device__ __forceinline__ double row_bcast_c(double v) {
  const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), 0x150 + L, 0xf, 0xf, true);
  const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), 0x150 + L, 0xf, 0xf, true);
  return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double row_bcast(double v, int l) {
  switch (l) {
    case 0: return row_bcast_c<0>(v);
    case 1: return row_bcast_c<1>(v);
    case 2: return row_bcast_c<2>(v);
    case 3: return row_bcast_c<3>(v);
    case 4: return row_bcast_c<4>(v);
    case 5: return row_bcast_c<5>(v);
    case 6: return row_bcast_c<6>(v);
    case 7: return row_bcast_c<7>(v);
    case 8: return row_bcast_c<8>(v);
    case 9: return row_bcast_c<9>(v);
    case 10: return row_bcast_c<10>(v);
    case 11: return row_bcast_c<11>(v);
    case 12: return row_bcast_c<12>(v);
    case 13: return row_bcast_c<13>(v);
    case 14: return row_bcast_c<14>(v);
    default: return row_bcast_c<15>(v);
  }
}

// x^{-1/2}: the hardware estimate (relative error about 5e-8) refined by two Newton steps
// y <- y + y (1/2 - x y^2 / 2), which brings it within an ulp or so.
__device__ __forceinline__ double rsqrt_refined(double x) {
  double y = __builtin_amdgcn_rsq(x);
  const double h = 0.5 * x;
  double e = fma(-h * y, y, 0.5);
  y = fma(y, e, y);
  e = fma(-h * y, y, 0.5);
  return fma(y, e, y);
}

// Wave 0 factors the 16 x 16 diagonal block kb of td in registers and inverts it in the same
// sweep: lane r holds row r (the four 16-lane rows of the wave hold the same block), pivot c is
// L_cc = sqrt(a_cc) from one reciprocal square root, the entries of column c reach the other
// lanes by row broadcasts, and lane j carries column j of the inverse (x_c = s_c / L_cc, then
// s_i -= L_ic x_c). L_kk goes back to td (lower triangle), X_kk = L_kk^{-1} to ta.
__device__ __forceinline__ void factor_block16(double* td, double* ta, int kb, int* bad) {
  const int lane = threadIdx.x & 63, r = lane & 15;
  double* D = blk16(td, kb, kb);
  double d[16], s[16];
#pragma unroll
  for (int c = 0; c < 16; ++c) {
    d[c] = D[r * LDT + c];
    s[c] = c == r ? 1.0 : 0.0;
  }
  int badl = 0;
#pragma unroll
  for (int c = 0; c < 16; ++c) {
    double piv = row_bcast(d[c], c);
    if (!(piv > 0.0) || !(piv < INFINITY)) {
      badl = 1;
      piv = 1.0;
    }
    const double rs = rsqrt_refined(piv);
    // lane c: sqrt(piv) (when the pivot was replaced, 1); lanes above c carry values of the
    // upper triangle that are never read
    const double l = r == c ? piv * rs : d[c] * rs;
    d[c] = l;
    const double x = s[c] * rs;
    s[c] = x;
#pragma unroll
    for (int cc = c + 1; cc < 16; ++cc) {
      const double lc = row_bcast(l, cc);
      d[cc] -= l * lc;
      s[cc] -= lc * x;
    }
  }
  if (lane < 16) {
    double* X = blk16(ta, kb, kb);
#pragma unroll
    for (int c = 0; c < 16; ++c) {
      if (c <= r) D[r * LDT + c] = d[c];
      X[c * LDT + r] = s[c];
    }
    if (badl) *bad = 1;
  }
}

// Factor the 64 x 64 tile in td (LDS, lower triangle read) in place: the lower triangle of
// td <- L with L L^T = td (the part above the diagonal is left undefined), and ta <- X =
// L^{-1} (lower triangular, zeros above the diagonal). A pivot that is not positive and
// finite is replaced by 1 and reported through *bad. Called by all threads of the workgroup.
//
// Blocked on 16 x 16 sub-blocks, right-looking, with the diagonal blocks on wave 0
// (factor_block16). After block kb is factored the waves form, on FP64 MFMA, the panel
// L_ik = A_ik X_kk^T and the blocks X_kj = -X_kk T_kj of row kb of X; then the trailing
// update A_ij -= L_ik L_jk^T together with the partial sums T_ij = sum_{t=j}^{kb} L_it X_tj
// (kept in the blocks of ta below the diagonal), during which wave 0 updates the next
// diagonal block first and factors it while waves 1-3 update the rest.
__device__ __forceinline__ void factor_diag_tile(double* td, double* ta, int* bad) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  for (int kb = 0; kb < 4; ++kb) {
    // Diagonal block kb on wave 0: its last update (by L_{kb,kb-1}, step kb - 1's item 0),
    // then its factorisation. Waves 1-3 meanwhile take the rest of step kb - 1's trailing
    // update, A_ij -= L_ik L_jk^T (k < j <= i) and T_ij (+)= L_ik X_kj (i > k >= j) with
    // k = kb - 1; before the first block they clear the blocks of ta above the diagonal.
    if (wave == 0) {
      if (kb > 0) {
        d4v acc = {0.0, 0.0, 0.0, 0.0};
        double* L1 = blk16(td, kb, kb - 1);
        mma16(acc, L1, LDT, 1, L1, LDT, 1);
        double* A11 = blk16(td, kb, kb);
#pragma unroll
        for (int v = 0; v < 4; ++v) A11[(4 * v + (lane >> 4)) * LDT + (lane & 15)] -= acc[v];
        // the block's rows come back to other lanes of this wave through LDS
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      }
      factor_block16(td, ta, kb, bad);
    } else if (kb == 0) {
      for (int e = tid - 64; e < 6 * 256; e += kThreads - 64) {
        const int b = e >> 8, w = e & 255;
        const int bi = b < 3 ? 0 : (b < 5 ? 1 : 2);
        const int bj = b < 3 ? b + 1 : (b < 5 ? b - 1 : 3);
        ta[(16 * bi + (w >> 4)) * LDT + 16 * bj + (w & 15)] = 0.0;
      }
    } else {
      const int k = kb - 1;
      const int nA = (3 - k) * (4 - k) / 2, nT = (3 - k) * (k + 1);
      // item 0, the diagonal block (kb, kb), is wave 0's
      for (int it = wave; it < nA + nT; it += kThreads / 64 - 1) {
        d4v acc = {0.0, 0.0, 0.0, 0.0};
        if (it < nA) {
          int i = k + 1, j = it;
          while (j >= i - k) {
            j -= i - k;
            ++i;
          }
          j += k + 1;
          mma16(acc, blk16(td, i, k), LDT, 1, blk16(td, j, k), LDT, 1);
          double* Aij = blk16(td, i, j);
#pragma unroll
          for (int v = 0; v < 4; ++v) Aij[(4 * v + (lane >> 4)) * LDT + (lane & 15)] -= acc[v];
        } else {
          const int t = it - nA, i = k + 1 + t / (k + 1), j = t % (k + 1);
          mma16(acc, blk16(td, i, k), LDT, 1, blk16(ta, k, j), 1, LDT);
          double* Tij = blk16(ta, i, j);
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            double* p = Tij + (4 * v + (lane >> 4)) * LDT + (lane & 15);
            *p = j == k ? acc[v] : *p + acc[v];
          }
        }
      }
    }
    __syncthreads();
    // panel L_ik = A_ik X_kk^T (i > kb) and row kb of X: X_kj = -X_kk T_kj (j < kb)
    if (wave < 3) {
      d4v acc = {0.0, 0.0, 0.0, 0.0};
      if (wave < 3 - kb) {
        double* Aik = blk16(td, kb + 1 + wave, kb);
        mma16(acc, Aik, LDT, 1, blk16(ta, kb, kb), LDT, 1);
#pragma unroll
        for (int v = 0; v < 4; ++v) Aik[(4 * v + (lane >> 4)) * LDT + (lane & 15)] = acc[v];
      } else {
        double* Tkj = blk16(ta, kb, wave - (3 - kb));
        mma16(acc, blk16(ta, kb, kb), LDT, 1, Tkj, 1, LDT);
#pragma unroll
        for (int v = 0; v < 4; ++v) Tkj[(4 * v + (lane >> 4)) * LDT + (lane & 15)] = -acc[v];
      }
    }
    __syncthreads();
  }
}

}  // namespace chol
}  // namespace rs
