// Dense sketches (Gaussian, Def. 4.1; SRHT, Def. 4.4) and the products they need.
//
// A dense S (m x tau, row-major, row stride ldas, zero padding columns) turns the
// sketched products into general contractions: T = Z^T S (K x tau), A S = Z T + lambda S
// (kernel ridge: + lambda T, since K S = K^T S), G = S^T A S. They run on one FP64 MFMA
// GEMM (128 x 128 tiles, 4 waves of 64 x 64, 16-deep panels with the next panel loaded
// into registers while the current one is multiplied), batched over lookahead slots.
// The iteration needs rho = S^T r (k_rho_dense_*: per row block partial sums, then a
// fixed-order sum over the blocks) and x -= gamma S delta next to r -= gamma AS delta
// (k_update_dense). The SRHT skips the explicit-S products where it can: T = Z^T S and
// G = S^T (AS) come from the fast Walsh-Hadamard transform of Z and of AS (k_srht_apply).
#include <algorithm>

#include "dev_common.h"
#include "rs_internal.h"

namespace rs {
namespace {

typedef double d4v __attribute__((ext_vector_type(4)));

constexpr int kThreads = 256;
constexpr int kGT = 128, kGK = 16;

__device__ __forceinline__ double unit_open(uint64_t w) {  // ((w >> 11) + 0.5) 2^-53 in (0, 1)
  return ((double)(w >> 11) + 0.5) * 0x1p-53;
}

// S[slot] (m x ldas): entry (i, c) from the Philox block (i G + c / 4, k, 6, 0), G = ceil(tau / 4);
// Box-Muller on the pairs (W0, W1) -> columns 4g, 4g+1 and (W2, W3) -> 4g+2, 4g+3.
__global__ __launch_bounds__(kThreads) void k_sketch_gauss(double* __restrict__ S, int64_t m, int32_t tau,
                                                           int64_t ldas, uint64_t seed, uint64_t pid, int64_t k0,
                                                           int32_t* __restrict__ offs, const int32_t* __restrict__ done) {
  if (*done) return;
  const int slot = blockIdx.y;
  const int64_t G = (tau + 3) / 4, ngrp = ldas / 4;
  const uint64_t k = (uint64_t)(k0 + slot);
  double* Ss = S + (int64_t)slot * m * ldas;
  for (int64_t e = (int64_t)blockIdx.x * kThreads + threadIdx.x; e < m * ngrp; e += (int64_t)gridDim.x * kThreads) {
    const int64_t i = e / ngrp, g = e % ngrp;
    double z[4] = {0.0, 0.0, 0.0, 0.0};
    if (g < G) {
      const Philox4 w = philox4x64_10((uint64_t)(i * G + g), k, kTagGaussian, 0, seed, pid);
      const double u0 = unit_open(w.v0), u1 = unit_open(w.v1), u2 = unit_open(w.v2), u3 = unit_open(w.v3);
      const double r01 = sqrt(-2.0 * log(u0)), t01 = 2.0 * M_PI * u1;
      const double r23 = sqrt(-2.0 * log(u2)), t23 = 2.0 * M_PI * u3;
      z[0] = r01 * cos(t01);
      z[1] = r01 * sin(t01);
      z[2] = r23 * cos(t23);
      z[3] = r23 * sin(t23);
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int64_t c = 4 * g + q;
      Ss[i * ldas + c] = c < tau ? z[q] : 0.0;
    }
  }
  // every column is a bucket of its own (no empty bucket for the factorisation)
  if (blockIdx.x == 0)
    for (int c = threadIdx.x; c <= tau; c += kThreads) offs[(int64_t)slot * (tau + 1) + c] = c;
}

// SRHT S[slot] (m x ldas) from C (members, ascending in [0, m')) and the signs
// d_i = -1 if W1 of the block (i, k, 7, 0) is odd: S_ic = d_i (-1)^popcount(i & C_c) scale.
__global__ __launch_bounds__(kThreads) void k_srht_fill(double* __restrict__ S, int64_t m, int32_t tau, int64_t ldas,
                                                        const int32_t* __restrict__ members, uint64_t seed,
                                                        uint64_t pid, int64_t k0, double scale,
                                                        const int32_t* __restrict__ done) {
  extern __shared__ int32_t cl[];  // [tau]
  if (*done) return;
  const int slot = blockIdx.y;
  const uint64_t k = (uint64_t)(k0 + slot);
  for (int c = threadIdx.x; c < tau; c += kThreads) cl[c] = members[(int64_t)slot * tau + c];
  __syncthreads();
  double* Ss = S + (int64_t)slot * m * ldas;
  for (int64_t i = blockIdx.x; i < m; i += gridDim.x) {
    const Philox4 w = philox4x64_10((uint64_t)i, k, kTagSrht, 0, seed, pid);
    const double di = (w.v1 & 1ull) ? -1.0 : 1.0;
    for (int c = threadIdx.x; c < (int)ldas; c += kThreads) {
      double v = 0.0;
      if (c < tau) {
        const double h = (__popcll((unsigned long long)(i & (int64_t)cl[c])) & 1) ? -1.0 : 1.0;
        v = di * h * scale;
      }
      Ss[i * ldas + c] = v;
    }
  }
}

// Dense form of a sparse sketch (count, SubCount on dense data): row i of S[slot] is zero except
// S[i][hmap_i >> 1] = -1 if hmap_i is odd, else +1 (hmap_i < 0: no entry).
__global__ __launch_bounds__(kThreads) void k_sketch_densify(double* __restrict__ S, const int32_t* __restrict__ hmap,
                                                             int64_t m, int64_t ldas, const int32_t* __restrict__ done) {
  if (*done) return;
  const int slot = blockIdx.y;
  double* Ss = S + (int64_t)slot * m * ldas;
  const int32_t* hm = hmap + (int64_t)slot * m;
  for (int64_t e = (int64_t)blockIdx.x * kThreads + threadIdx.x; e < m * ldas; e += (int64_t)gridDim.x * kThreads) {
    const int64_t i = e / ldas, c = e % ldas;
    const int32_t code = hm[i];
    Ss[e] = (code >= 0 && (code >> 1) == c) ? ((code & 1) ? -1.0 : 1.0) : 0.0;
  }
}

// C(i, j) = sum_k A(i, k) B(k, j) (+ lam E(i, j)), A(i, k) = AT ? A[k lda + i] : A[i lda + k],
// B(k, j) = B[k ldb + j]; slot blockIdx.z offsets every operand by its slot stride.
template <bool AT>
__global__ __launch_bounds__(kThreads, 2) void k_gemm_f64(GemmF64Args g) {
  __shared__ double As[kGT][kGK + 1];
  __shared__ double Bs[kGT][kGK + 1];  // Bs[j][k] = B(k, j)
  if (g.done && *g.done) return;
  const int64_t slot = blockIdx.z;
  const double* __restrict__ A = g.A + slot * g.sA;
  const double* __restrict__ B = g.B + slot * g.sB;
  double* __restrict__ C = g.C + slot * g.sC;
  const double* __restrict__ E = g.E ? g.E + slot * g.sE : nullptr;
  const int64_t i0 = (int64_t)blockIdx.x * kGT, j0 = (int64_t)blockIdx.y * kGT;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wr = (wave >> 1) * 64, wc = (wave & 1) * 64;
  d4v acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = d4v{0.0, 0.0, 0.0, 0.0};
  // Loads of a 128 x 16 panel of each operand, 8 elements per thread. A (row-major):
  // thread t reads rows t / 16 + 16 u at column t % 16; A (transposed) and B: element
  // (t % 128) of rows t / 128 + 2 u, which are contiguous in memory.
  double ra[8], rb[8];
  const int a_r = AT ? (tid & 127) : (tid >> 4), a_k = AT ? (tid >> 7) : (tid & 15);
  const int b_c = tid & 127, b_k = tid >> 7;
  const bool a_in = AT ? (i0 + a_r < g.M) : true;
  const bool b_in = j0 + b_c < g.N;
  auto gload = [&](int64_t k0) {
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      if (AT) {
        const int64_t k = k0 + a_k + 2 * u;
        ra[u] = (a_in && k < g.Kd) ? A[k * g.lda + i0 + a_r] : 0.0;
      } else {
        const int64_t i = i0 + a_r + 16 * u, k = k0 + a_k;
        ra[u] = (i < g.M && k < g.Kd) ? A[i * g.lda + k] : 0.0;
      }
      const int64_t kr = k0 + b_k + 2 * u;
      rb[u] = (b_in && kr < g.Kd) ? B[kr * g.ldb + j0 + b_c] : 0.0;
    }
  };
  auto lstore = [&]() {
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      if (AT)
        As[a_r][a_k + 2 * u] = ra[u];
      else
        As[a_r + 16 * u][a_k] = ra[u];
      Bs[b_c][b_k + 2 * u] = rb[u];
    }
  };
  gload(0);
  lstore();
  __syncthreads();
  for (int64_t k0 = 0; k0 < g.Kd; k0 += kGK) {
    const bool more = k0 + kGK < g.Kd;
    if (more) gload(k0 + kGK);
#pragma unroll
    for (int k4 = 0; k4 < kGK; k4 += 4) {
      double a[4], b[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) a[i] = As[wr + i * 16 + (lane & 15)][k4 + (lane >> 4)];
#pragma unroll
      for (int j = 0; j < 4; ++j) b[j] = Bs[wc + j * 16 + (lane & 15)][k4 + (lane >> 4)];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b[j], acc[i][j], 0, 0, 0);
    }
    __syncthreads();
    if (more) {
      lstore();
      __syncthreads();
    }
  }
  // D layout of the 16x16x4 FP64 MFMA: lane l, element v -> row 4 v + l / 16, column l % 16.
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t row = i0 + wr + i * 16 + v * 4 + (lane >> 4);
        const int64_t col = j0 + wc + j * 16 + (lane & 15);
        if (row < g.M && col < g.N) {
          double val = acc[i][j][v];
          if (E) val += g.lam * E[row * g.lde + col];
          C[row * g.ldc + col] = val;
        }
      }
}

// part[b][c] = sum over rows i of block b (in order) of S[i][c] r[i]
__global__ __launch_bounds__(kThreads) void k_rho_dense_part(const double* __restrict__ S, int64_t ldas, int32_t tau,
                                                             int64_t m, const double* __restrict__ r, int32_t nblk,
                                                             double* __restrict__ part,
                                                             const DevFlags* __restrict__ flags) {
  if (flags->done) return;
  const int64_t per = (m + nblk - 1) / nblk;
  const int64_t i0 = min(m, (int64_t)blockIdx.x * per), i1 = min(m, i0 + per);
  for (int c = threadIdx.x; c < tau; c += kThreads) {
    double s = 0.0;
    for (int64_t i = i0; i < i1; ++i) s += S[i * ldas + c] * r[i];
    part[(int64_t)blockIdx.x * tau + c] = s;
  }
}

__global__ __launch_bounds__(kThreads) void k_rho_dense_sum(const double* __restrict__ part, int32_t nblk, int32_t tau,
                                                            double* __restrict__ rho,
                                                            const DevFlags* __restrict__ flags) {
  if (flags->done) return;
  const int c = blockIdx.x * kThreads + threadIdx.x;
  if (c >= tau) return;
  double s = 0.0;
  for (int b = 0; b < nblk; ++b) s += part[(int64_t)b * tau + c];
  rho[c] = s;
}

// x^{k+1} = (1 + beta) x^k - beta x^{k-1} - gamma S delta, r^{k+1} likewise with AS delta, over
// ceil(m / npart) rows per workgroup (one wave per row), plus the partial sums of ||r^{k+1}||^2.
__global__ __launch_bounds__(kThreads) void k_update_dense(const double* __restrict__ AS, const double* __restrict__ S,
                                                           int64_t ldas, int32_t tau, const double* __restrict__ delta,
                                                           int64_t m, const double* __restrict__ x,
                                                           double* __restrict__ xo, const double* __restrict__ r,
                                                           double* __restrict__ ro, double gamma, double beta,
                                                           double* __restrict__ partials, int32_t npart,
                                                           const DevFlags* __restrict__ flags) {
  extern __shared__ __align__(16) double dl[];  // [ldas]
  __shared__ double scratch[16];
  if (flags->done) return;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  for (int c = tid; c < (int)ldas; c += kThreads) dl[c] = c < tau ? delta[c] : 0.0;
  __syncthreads();
  const int64_t per = (m + npart - 1) / npart;
  const int64_t j0 = min(m, (int64_t)blockIdx.x * per), j1 = min(m, j0 + per);
  const int half = (int)(ldas >> 1);
  double ss = 0.0;
  for (int64_t j = j0 + wave; j < j1; j += kThreads / 64) {
    const double2* a2 = reinterpret_cast<const double2*>(AS + j * ldas);
    const double2* s2 = reinterpret_cast<const double2*>(S + j * ldas);
    double sa = 0.0, sd = 0.0;
    for (int c2 = lane; c2 < half; c2 += 64) {
      const double2 a = a2[c2], b = s2[c2];
      const double d0 = dl[2 * c2], d1 = dl[2 * c2 + 1];
      sa += a.x * d0 + a.y * d1;
      sd += b.x * d0 + b.y * d1;
    }
    sa = wave_sum(sa);
    sd = wave_sum(sd);
    if (lane == 0) {
      const double onepb = 1.0 + beta;
      const double rn = onepb * r[j] - beta * ro[j] - gamma * sa;
      const double xn = onepb * x[j] - beta * xo[j] - gamma * sd;
      ro[j] = rn;
      xo[j] = xn;
      ss += rn * rn;
    }
  }
  ss = block_sum(ss, scratch);
  if (tid == 0) partials[blockIdx.x] = ss;
}

// The SRHT applied by its fast transform (Def. 4.4): for every column j of Y (m x ncols, row
// stride ldy) and every sketch column c, OUT(j, c) = sum_{i < m} S_ic Y_ij with
// S_ic = scale d_i (-1)^popcount(i & C_c), i.e. the entries C_c of H_{m'} (D Y_j) where the column
// D Y_j is zero-padded to m' = 2^lg rows. A workgroup loads JB consecutive columns (times the
// signs d_i) into LDS, runs the in-place Walsh-Hadamard butterflies on all of them (two stages
// per pass: quads (b, b + h, b + 2h, b + 3h)), and writes the tau selected rows. Reading Y once
// replaces the 2 m ncols tau flop of multiplying it by an explicit S. The signs are read back
// from the slot's explicit S (column 0: d_i = sign(S_i0) (-1)^popcount(i & C_0)), so both forms
// use the same draw. OUT(j, c) is stored at OUT[j ldo + c] (trans_out = 0) or OUT[c ldo + j].
__global__ __launch_bounds__(kThreads) void k_srht_apply(
    const double* __restrict__ Y, int64_t ldy, int64_t sY, int64_t m, int64_t ncols, int32_t lg, int32_t jbl,
    const double* __restrict__ S, int64_t lds, int64_t sS, const int32_t* __restrict__ members, int32_t tau,
    double scale, double* __restrict__ OUT, int64_t ldo, int64_t sO, int32_t trans_out,
    const int32_t* __restrict__ done) {
  extern __shared__ __align__(16) double buf[];  // [m'][JB], then m' sign bytes
  if (*done) return;
  const int64_t slot = blockIdx.y;
  const int64_t mp = (int64_t)1 << lg;
  const int JB = 1 << jbl;
  const int64_t j0 = (int64_t)blockIdx.x * JB;
  signed char* sgn = reinterpret_cast<signed char*>(buf + mp * JB);
  const double* Ys = Y + slot * sY;
  const double* Ss = S + slot * sS;
  const int32_t* Cs = members + slot * (int64_t)tau;
  const int64_t c0 = Cs[0];
  for (int64_t i = threadIdx.x; i < m; i += kThreads) {
    const bool hneg = __popcll((unsigned long long)(i & c0)) & 1;
    sgn[i] = ((Ss[i * lds] < 0.0) != hneg) ? -1 : 1;
  }
  __syncthreads();
  for (int64_t e = threadIdx.x; e < mp * JB; e += kThreads) {
    const int64_t i = e >> jbl, j = j0 + (e & (JB - 1));
    buf[e] = (i < m && j < ncols) ? (double)sgn[i] * Ys[i * ldy + j] : 0.0;
  }
  __syncthreads();
  int64_t h = 1;
  int rem = lg;
  for (; rem >= 2; rem -= 2, h <<= 2) {
    for (int64_t q = threadIdx.x; q < (mp >> 2) * JB; q += kThreads) {
      const int64_t t = q >> jbl, j = q & (JB - 1);
      const int64_t b = (t / h) * 4 * h + t % h;
      double* p0 = buf + b * JB + j;
      const int64_t hs = h * JB;
      const double a0 = p0[0], a1 = p0[hs], a2 = p0[2 * hs], a3 = p0[3 * hs];
      const double s01 = a0 + a1, d01 = a0 - a1, s23 = a2 + a3, d23 = a2 - a3;
      p0[0] = s01 + s23;
      p0[2 * hs] = s01 - s23;
      p0[hs] = d01 + d23;
      p0[3 * hs] = d01 - d23;
    }
    __syncthreads();
  }
  if (rem == 1) {
    for (int64_t q = threadIdx.x; q < (mp >> 1) * JB; q += kThreads) {
      const int64_t t = q >> jbl, j = q & (JB - 1);
      const int64_t b = (t / h) * 2 * h + t % h;
      double* p0 = buf + b * JB + j;
      const double a0 = p0[0], a1 = p0[h * JB];
      p0[0] = a0 + a1;
      p0[h * JB] = a0 - a1;
    }
    __syncthreads();
  }
  double* Os = OUT + slot * sO;
  for (int64_t e = threadIdx.x; e < (int64_t)JB * tau; e += kThreads) {
    const int64_t jj = e / tau, c = e % tau, j = j0 + jj;
    if (j >= ncols) continue;
    const double v = scale * buf[(int64_t)Cs[c] * JB + jj];
    if (trans_out)
      Os[c * ldo + j] = v;
    else
      Os[j * ldo + c] = v;
  }
}

}  // namespace

hipError_t launch_sketch_gauss(double* S, int64_t m, int32_t tau, int64_t ldas, uint64_t seed, uint64_t pid,
                               int64_t k0, int32_t nslots, int32_t* offs, const int32_t* done, hipStream_t s) {
  if (nslots <= 0) return hipSuccess;
  if (ldas % 4 != 0 || ldas < tau || nslots > 65535) return hipErrorInvalidValue;
  const int64_t work = m * (ldas / 4);
  unsigned gx = (unsigned)std::min<int64_t>((work + kThreads - 1) / kThreads, 4096);
  if (gx == 0) gx = 1;
  hipLaunchKernelGGL(k_sketch_gauss, dim3(gx, (unsigned)nslots), dim3(kThreads), 0, s, S, m, tau, ldas, seed, pid,
                     k0, offs, done);
  return hipGetLastError();
}

hipError_t launch_srht_fill(double* S, int64_t m, int32_t tau, int64_t ldas, const int32_t* members, uint64_t seed,
                            uint64_t pid, int64_t k0, int64_t mpad, int32_t nslots, const int32_t* done,
                            hipStream_t s) {
  if (nslots <= 0) return hipSuccess;
  if (ldas < tau || nslots > 65535 || mpad < m) return hipErrorInvalidValue;
  const double scale = 1.0 / sqrt((double)tau * (double)mpad);
  const unsigned gx = (unsigned)std::min<int64_t>(m, 2048);
  hipLaunchKernelGGL(k_srht_fill, dim3(gx, (unsigned)nslots), dim3(kThreads), sizeof(int32_t) * tau, s, S, m, tau,
                     ldas, members, seed, pid, k0, scale, done);
  return hipGetLastError();
}

hipError_t launch_gemm_f64(const GemmF64Args& g, bool a_trans, int32_t nslots, hipStream_t s) {
  if (nslots <= 0 || g.M <= 0 || g.N <= 0) return hipSuccess;
  const int64_t gx = (g.M + kGT - 1) / kGT, gy = (g.N + kGT - 1) / kGT;
  if (gx > 0x7fffffff || gy > 65535 || nslots > 65535) return hipErrorInvalidValue;
  if (a_trans)
    hipLaunchKernelGGL((k_gemm_f64<true>), dim3((unsigned)gx, (unsigned)gy, (unsigned)nslots), dim3(kThreads), 0, s, g);
  else
    hipLaunchKernelGGL((k_gemm_f64<false>), dim3((unsigned)gx, (unsigned)gy, (unsigned)nslots), dim3(kThreads), 0, s,
                       g);
  return hipGetLastError();
}

hipError_t launch_sketch_densify(double* S, const int32_t* hmap, int64_t m, int64_t ldas, int32_t nslots,
                                 const int32_t* done, hipStream_t s) {
  if (nslots <= 0) return hipSuccess;
  if (nslots > 65535) return hipErrorInvalidValue;
  const unsigned gx = (unsigned)std::min<int64_t>((m * ldas + kThreads - 1) / kThreads, 4096);
  hipLaunchKernelGGL(k_sketch_densify, dim3(gx, (unsigned)nslots), dim3(kThreads), 0, s, S, hmap, m, ldas, done);
  return hipGetLastError();
}

int32_t rho_dense_blocks() { return 64; }

hipError_t launch_rho_dense(const double* S, int64_t ldas, int32_t tau, int64_t m, const double* r, double* part,
                            double* rho, const DevFlags* flags, hipStream_t s) {
  const int32_t nblk = rho_dense_blocks();
  hipLaunchKernelGGL(k_rho_dense_part, dim3(nblk), dim3(kThreads), 0, s, S, ldas, tau, m, r, nblk, part, flags);
  hipLaunchKernelGGL(k_rho_dense_sum, dim3((unsigned)((tau + kThreads - 1) / kThreads)), dim3(kThreads), 0, s, part,
                     nblk, tau, rho, flags);
  return hipGetLastError();
}

hipError_t launch_update_dense(const double* AS, const double* S, int64_t ldas, int32_t tau, const double* delta,
                               int64_t m, const double* x, double* x_prev_out, const double* r, double* r_prev_out,
                               double gamma, double beta, double* partials, int32_t npart, const DevFlags* flags,
                               hipStream_t s) {
  if (ldas % 2 != 0 || npart <= 0) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_update_dense, dim3((unsigned)npart), dim3(kThreads), sizeof(double) * ldas, s, AS, S, ldas, tau,
                     delta, m, x, x_prev_out, r, r_prev_out, gamma, beta, partials, npart, flags);
  return hipGetLastError();
}

int64_t srht_fast_max_mpad() { return 16384; }

hipError_t launch_srht_apply(const double* Y, int64_t ldy, int64_t sY, int64_t m, int64_t ncols, int64_t mpad,
                             const double* S, int64_t lds, int64_t sS, const int32_t* members, int32_t tau,
                             double* OUT, int64_t ldo, int64_t sO, int32_t trans_out, int32_t nslots,
                             const int32_t* done, hipStream_t s) {
  if (nslots <= 0 || ncols <= 0) return hipSuccess;
  int lg = 0;
  while (((int64_t)1 << lg) < mpad) ++lg;
  if (((int64_t)1 << lg) != mpad || mpad < m || mpad > srht_fast_max_mpad() || tau < 1 || tau > mpad ||
      nslots > 65535)
    return hipErrorInvalidValue;
  // JB columns per workgroup: at most 16, and at most 16384 / m' so that the LDS image stays <= 128 KB
  int jbl = 0;
  while (jbl < 4 && ((int64_t)2 << jbl) * mpad <= 16384) ++jbl;
  const int64_t JB = (int64_t)1 << jbl;
  const size_t bytes = sizeof(double) * (size_t)mpad * JB + (size_t)mpad;
  static bool attr_set = false;
  if (!attr_set) {
    hipError_t e = hipFuncSetAttribute((const void*)k_srht_apply, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)(sizeof(double) * 16384 + 16384));
    if (e != hipSuccess) return e;
    attr_set = true;
  }
  const int64_t gx = (ncols + JB - 1) / JB;
  if (gx > 0x7fffffff) return hipErrorInvalidValue;
  const double scale = 1.0 / sqrt((double)tau * (double)mpad);
  hipLaunchKernelGGL(k_srht_apply, dim3((unsigned)gx, (unsigned)nslots), dim3(kThreads), bytes, s, Y, ldy, sY, m,
                     ncols, (int32_t)lg, (int32_t)jbl, S, lds, sS, members, tau, scale, OUT, ldo, sO, trans_out, done);
  return hipGetLastError();
}

}  // namespace rs
