// Dense products for the subsample sketch and setup helpers (CDNA4, wave64).
//
// For S = I_C, A S = Z (Z^T I_C) + lambda I_C = Z Z[C,:]^T + lambda I_C: an m x tau
// contraction over K whose second operand is the gathered rows C of Z. Several
// lookahead sketches share the first operand, so one launch contracts Z against
// [Z[C_0,:]; Z[C_1,:]; ...] (N = slots * tau columns) on FP64 MFMA (16x16x4).
// Kernel ridge (Sec. 2.2) stores the symmetric kernel matrix as Z (m = K): then
// A S = K (K + lambda I) I_C = Z Z[C,:]^T + lambda Z[:,C], the same contraction with the
// shift taken from the gathered columns.
#include "dev_common.h"
#include "rs_internal.h"

namespace rs {
namespace {

typedef double d4v __attribute__((ext_vector_type(4)));

// 128 x 128 tile of AS on 4 waves (each 64 x 64 as 4 x 4 FP64 MFMA blocks of 16 x 16):
// twice the flops per staged byte of the 64 x 64 tile. The next 16-deep K panel of both
// operands is loaded into registers (16-byte loads when rows are 16-byte aligned) while
// the current one is multiplied from LDS.
constexpr int kBT = 128, kBK = 16;
struct DenseLds128 {
  double As[kBT][kBK + 1];
  double Bs[kBT][kBK + 1];
  int64_t brow[kBT];
};

__device__ __forceinline__ void as_dense_tile128(const double* __restrict__ Z, int64_t ldz, int64_t m,
                                                 int64_t K, const int32_t* __restrict__ members,
                                                 int32_t tau, int64_t ntot, int64_t ldas, double lam,
                                                 int32_t lam_kernel, double* __restrict__ AS, int64_t row0,
                                                 int64_t n0, DenseLds128& L) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wr = (wave >> 1) * 64, wc = (wave & 1) * 64;
  if (tid < kBT) {
    const int64_t n = n0 + tid;
    L.brow[tid] = n < ntot ? (int64_t)members[n] : -1;  // members is [slot][tau]
  }
  __syncthreads();
  d4v acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = d4v{0.0, 0.0, 0.0, 0.0};

  // element pair e = tid + 256 u (u < 4) of a 128 x 16 panel: row e / 8, columns 2 (e % 8) + {0, 1}
  const bool vec = (ldz & 1) == 0;
  int64_t arow[4], brw[4];
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int r = (tid + 256 * u) >> 3;
    arow[u] = row0 + r < m ? row0 + r : -1;
    brw[u] = L.brow[r];
  }
  const int kc = 2 * (tid & 7);
  double2 ra[4], rb[4];
  auto gload = [&](int64_t kk) {
    const int64_t k = kk + kc;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      double2 va = make_double2(0.0, 0.0), vb = make_double2(0.0, 0.0);
      if (vec && k + 1 < K) {
        if (arow[u] >= 0) va = *reinterpret_cast<const double2*>(Z + arow[u] * ldz + k);
        if (brw[u] >= 0) vb = *reinterpret_cast<const double2*>(Z + brw[u] * ldz + k);
      } else {
        if (arow[u] >= 0 && k < K) va.x = Z[arow[u] * ldz + k];
        if (arow[u] >= 0 && k + 1 < K) va.y = Z[arow[u] * ldz + k + 1];
        if (brw[u] >= 0 && k < K) vb.x = Z[brw[u] * ldz + k];
        if (brw[u] >= 0 && k + 1 < K) vb.y = Z[brw[u] * ldz + k + 1];
      }
      ra[u] = va;
      rb[u] = vb;
    }
  };
  auto lstore = [&]() {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int r = (tid + 256 * u) >> 3;
      L.As[r][kc] = ra[u].x;
      L.As[r][kc + 1] = ra[u].y;
      L.Bs[r][kc] = rb[u].x;
      L.Bs[r][kc + 1] = rb[u].y;
    }
  };
  gload(0);
  lstore();
  __syncthreads();
  for (int64_t kk = 0; kk < K; kk += kBK) {
    const bool more = kk + kBK < K;
    if (more) gload(kk + kBK);
#pragma unroll
    for (int k4 = 0; k4 < kBK; k4 += 4) {
      double a[4], b[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) a[i] = L.As[wr + i * 16 + (lane & 15)][k4 + (lane >> 4)];
#pragma unroll
      for (int j = 0; j < 4; ++j) b[j] = L.Bs[wc + j * 16 + (lane & 15)][k4 + (lane >> 4)];
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
        const int64_t row = row0 + wr + i * 16 + v * 4 + (lane >> 4);
        const int col = wc + j * 16 + (lane & 15);
        const int64_t n = n0 + col;
        if (row < m && n < ntot) {
          const int64_t slot = n / tau, c = n % tau;
          double val = acc[i][j][v];
          if (lam_kernel)
            val += lam * Z[L.brow[col] * ldz + row];  // lambda K[row, C_c] (K symmetric)
          else if (row == L.brow[col])
            val += lam;
          AS[(slot * m + row) * ldas + c] = val;
        }
      }
  __syncthreads();  // brow is rewritten by the next tile of a persistent workgroup
}

__global__ __launch_bounds__(256, 2) void k_as_dense_f64_128(const double* __restrict__ Z, int64_t ldz,
                                                             int64_t m, int64_t K,
                                                             const int32_t* __restrict__ members,
                                                             int32_t tau, int64_t ldas, int32_t nslots,
                                                             double lam, int32_t lam_kernel,
                                                             double* __restrict__ AS,
                                                             const int32_t* __restrict__ done) {
  __shared__ DenseLds128 L;
  if (*done) return;
  as_dense_tile128(Z, ldz, m, K, members, tau, (int64_t)nslots * tau, ldas, lam, lam_kernel, AS,
                   (int64_t)blockIdx.x * kBT, (int64_t)blockIdx.y * kBT, L);
}

// Grouped form over a ragged table of (job, 128-row tile, 128-column tile) entries; a
// fixed grid of workgroups strides over the table (persistent launch).
__global__ __launch_bounds__(256, 2) void k_as_dense_f64_tab(const DenseJob* __restrict__ jobs,
                                                             const DenseTile* __restrict__ tiles,
                                                             int32_t ntiles) {
  __shared__ DenseLds128 L;
  for (int32_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
    const DenseTile tl = tiles[t];
    const DenseJob& j = jobs[tl.job];
    if (*j.done) continue;  // uniform across the workgroup
    as_dense_tile128(j.Z, j.ldz, j.m, j.K, j.members, j.tau, j.tau, j.ldas, j.lam, 0, j.AS,
                     (int64_t)tl.tm * kBT, (int64_t)tl.tn * kBT, L);
  }
}

__global__ void k_transpose_to_f64(const void* __restrict__ src, int32_t is_f32, int64_t rows,
                                   int64_t cols, int64_t lds, double* __restrict__ dst, int64_t ldd) {
  __shared__ double tile[32][33];
  const int64_t r0 = (int64_t)blockIdx.y * 32, c0 = (int64_t)blockIdx.x * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 256 threads: 32 x 8
  for (int yy = ty; yy < 32; yy += 8) {
    const int64_t r = r0 + yy, c = c0 + tx;
    double v = 0.0;
    if (r < rows && c < cols)
      v = is_f32 ? (double)((const float*)src)[r * lds + c] : ((const double*)src)[r * lds + c];
    tile[yy][tx] = v;
  }
  __syncthreads();
  for (int yy = ty; yy < 32; yy += 8) {
    const int64_t c = c0 + yy, r = r0 + tx;  // dst[c][r] = src[r][c]
    if (c < cols && r < rows) dst[c * ldd + r] = tile[tx][yy];
  }
}

__global__ void k_copy_to_f64(const void* __restrict__ src, int32_t is_f32, int64_t rows,
                              int64_t cols, int64_t lds, double* __restrict__ dst, int64_t ldd) {
  for (int64_t r = blockIdx.y; r < rows; r += gridDim.y)
    for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < cols;
         c += (int64_t)gridDim.x * blockDim.x)
      dst[r * ldd + c] =
          is_f32 ? (double)((const float*)src)[r * lds + c] : ((const double*)src)[r * lds + c];
}

// out[j] = sum_k Z[j][k] v[k]: one wave per row, fixed-order reduction.
__global__ void k_gemv_rows(const double* __restrict__ Z, int64_t ldz, int64_t m, int64_t K,
                            const double* __restrict__ v, double* __restrict__ out) {
  const int lane = threadIdx.x & 63;
  const int64_t row = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (row >= m) return;
  double s = 0.0;
  for (int64_t k = lane; k < K; k += 64) s += Z[row * ldz + k] * v[k];
  s = wave_sum(s);
  if (lane == 0) out[row] = s;
}

// out[k] = sum_j Z[j][k] v[j]: one thread per column k, rows in order.
__global__ void k_gemv_cols(const double* __restrict__ Z, int64_t ldz, int64_t m, int64_t K,
                            const double* __restrict__ v, double* __restrict__ out) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= K) return;
  double s = 0.0;
  for (int64_t j = 0; j < m; ++j) s += Z[j * ldz + k] * v[j];
  out[k] = s;
}

// Gaussian kernel matrix (eq:Gausskernel) of points P (n x d, row-major FP64):
// Kout[i][j] = exp(-sum_t (P[i][t] - P[j][t])^2 / denom), denom = 2 sigma^2, one 64 x 64
// tile per workgroup, 32 coordinates at a time staged in LDS; every thread owns a 4 x 4
// block. The squares are summed in coordinate order, so Kout is exactly symmetric.
constexpr int kRbfT = 64, kRbfD = 32;
__global__ __launch_bounds__(256) void k_rbf_gram(const double* __restrict__ P, int64_t n, int64_t d,
                                                  double denom, double* __restrict__ Kout, int64_t ldk) {
  __shared__ double pi[kRbfT][kRbfD + 1];
  __shared__ double pj[kRbfT][kRbfD + 1];
  const int tid = threadIdx.x;
  const int64_t i0 = (int64_t)blockIdx.y * kRbfT, j0 = (int64_t)blockIdx.x * kRbfT;
  const int ti = (tid >> 4) * 4, tj = (tid & 15) * 4;
  double acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = 0.0;
  for (int64_t t0 = 0; t0 < d; t0 += kRbfD) {
    for (int e = tid; e < kRbfT * kRbfD; e += 256) {
      const int r = e / kRbfD, c = e % kRbfD;
      const int64_t t = t0 + c;
      pi[r][c] = (i0 + r < n && t < d) ? P[(i0 + r) * d + t] : 0.0;
      pj[r][c] = (j0 + r < n && t < d) ? P[(j0 + r) * d + t] : 0.0;
    }
    __syncthreads();
    const int tn = (int)(d - t0 < kRbfD ? d - t0 : kRbfD);
    for (int c = 0; c < tn; ++c) {
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) {
          const double df = pi[ti + a][c] - pj[tj + b][c];
          acc[a][b] += df * df;
        }
    }
    __syncthreads();
  }
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const int64_t i = i0 + ti + a, j = j0 + tj + b;
      if (i < n && j < n) Kout[i * ldk + j] = exp(-acc[a][b] / denom);
    }
}

__global__ void k_vec_to_f64(const void* __restrict__ src, int32_t is_f32, int64_t n,
                             double* __restrict__ dst) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = is_f32 ? (double)((const float*)src)[i] : ((const double*)src)[i];
}

}  // namespace

namespace {
// One wave per row of AS: the row of the formed A is read at the sketch's coordinates
// (ascending, so the reads of a wave fall in a few lines) and written contiguously.
template <typename T>
__global__ __launch_bounds__(256) void k_gram_gather(const T* __restrict__ A, int64_t lda, int64_t m,
                                                     const int32_t* __restrict__ members, int64_t nsel,
                                                     int32_t tau, int64_t ldas, T* __restrict__ AS,
                                                     const int32_t* __restrict__ done) {
  if (*done) return;
  const int64_t slot = blockIdx.y;
  const int64_t row = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (row >= m) return;
  const int lane = threadIdx.x & 63;
  const int32_t* mem = members + slot * nsel;
  const T* a = A + row * lda;
  T* out = AS + (slot * m + row) * ldas;
  for (int c = lane; c < tau; c += 64) out[c] = a[mem[c]];
}
}  // namespace

hipError_t launch_gram_gather(const void* A, int32_t f32, int64_t lda, int64_t m, const int32_t* members,
                              int64_t nsel, int32_t tau, int64_t ldas, int32_t nslots, void* AS,
                              const int32_t* done, hipStream_t s) {
  if (tau > nsel || tau > ldas || lda < m || nslots < 1) return hipErrorInvalidValue;
  const dim3 grid((unsigned)((m + 3) / 4), (unsigned)nslots);
  if (f32)
    hipLaunchKernelGGL(k_gram_gather<float>, grid, dim3(256), 0, s, (const float*)A, lda, m, members, nsel, tau,
                       ldas, (float*)AS, done);
  else
    hipLaunchKernelGGL(k_gram_gather<double>, grid, dim3(256), 0, s, (const double*)A, lda, m, members, nsel,
                       tau, ldas, (double*)AS, done);
  return hipGetLastError();
}

hipError_t launch_as_dense_f64(const double* Z, int64_t ldz, int64_t m, int64_t K,
                               const int32_t* members, int32_t tau, int64_t ldas, int32_t nslots,
                               double lam, int32_t lam_kernel, double* AS, const int32_t* done,
                               hipStream_t s) {
  const int64_t ntot = (int64_t)nslots * tau;
  if (lam_kernel && K != m) return hipErrorInvalidValue;
  dim3 grid((unsigned)((m + kBT - 1) / kBT), (unsigned)((ntot + kBT - 1) / kBT));
  hipLaunchKernelGGL(k_as_dense_f64_128, grid, dim3(256), 0, s, Z, ldz, m, K, members, tau, ldas,
                     nslots, lam, lam_kernel, AS, done);
  return hipGetLastError();
}

hipError_t launch_transpose_to_f64(const void* src, int32_t src_is_f32, int64_t rows, int64_t cols,
                                   int64_t lds, double* dst, int64_t ldd, hipStream_t s) {
  dim3 grid((unsigned)((cols + 31) / 32), (unsigned)((rows + 31) / 32));
  hipLaunchKernelGGL(k_transpose_to_f64, grid, dim3(256), 0, s, src, src_is_f32, rows, cols, lds,
                     dst, ldd);
  return hipGetLastError();
}

hipError_t launch_copy_to_f64(const void* src, int32_t src_is_f32, int64_t rows, int64_t cols,
                              int64_t lds, double* dst, int64_t ldd, hipStream_t s) {
  if (rows == 0) return hipSuccess;
  unsigned gx = (unsigned)((cols + 255) / 256);
  if (gx > 64) gx = 64;
  dim3 grid(gx, (unsigned)(rows < 65535 ? rows : 65535));
  hipLaunchKernelGGL(k_copy_to_f64, grid, dim3(256), 0, s, src, src_is_f32, rows, cols, lds, dst,
                     ldd);
  return hipGetLastError();
}

hipError_t launch_gemv_rows(const double* Z, int64_t ldz, int64_t m, int64_t K, const double* v,
                            double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_gemv_rows, dim3((unsigned)((m + 3) / 4)), dim3(256), 0, s, Z, ldz, m, K, v,
                     out);
  return hipGetLastError();
}

hipError_t launch_gemv_cols(const double* Z, int64_t ldz, int64_t m, int64_t K, const double* v,
                            double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_gemv_cols, dim3((unsigned)((K + 255) / 256)), dim3(256), 0, s, Z, ldz, m, K,
                     v, out);
  return hipGetLastError();
}

hipError_t launch_vec_to_f64(const void* src, int32_t src_is_f32, int64_t n, double* dst,
                             hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_vec_to_f64, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, src,
                     src_is_f32, n, dst);
  return hipGetLastError();
}

hipError_t launch_rbf_gram(const double* P, int64_t n, int64_t d, double sigma, double* Kout, int64_t ldk,
                           hipStream_t s) {
  if (n <= 0) return hipSuccess;
  if (d < 1 || ldk < n || !(sigma > 0.0)) return hipErrorInvalidValue;
  const unsigned t = (unsigned)((n + kRbfT - 1) / kRbfT);
  if (t > 65535) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_rbf_gram, dim3(t, t), dim3(256), 0, s, P, n, d, 2.0 * sigma * sigma, Kout, ldk);
  return hipGetLastError();
}

hipError_t launch_as_dense_f64_tab(const DenseJob* jobs, const DenseTile* tiles, int32_t ntiles,
                                   int32_t tk, int32_t grid, hipStream_t s) {
  if (ntiles <= 0) return hipSuccess;
  grid = grid < 1 ? 1 : (grid > ntiles ? ntiles : grid);
  if (tk != kBK) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_as_dense_f64_tab, dim3(grid), dim3(256), 0, s, jobs, tiles, ntiles);
  return hipGetLastError();
}

}  // namespace rs
