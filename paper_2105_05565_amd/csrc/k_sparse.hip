// Count and SubCount sketch products for CSR data (Sec. 4.2).
//
// With Z the m x K operand of A = Z Z^T + lambda I (primal Z = X^T, dual Z = X):
//
//   AS[j, :] = sum_{i in row j of Z} Z_ji T[i, :] + lambda s_j e_{h(j)},
//   T[i, :]  = sum_{j' in row i of Z^T} s_j' Z_j'i e_{h(j')}          (T = Z^T S),
//
// where h(j) is the bucket (column of S) holding coordinate j and s_j its sign.
// Each row of AS is built by one wavefront as a signed scatter-add of CSR entries
// into tau bucket accumulators staged in LDS. Buckets are processed by one
// workgroup each, so the sketched matrix G = S^T A S, whose row b is
// sum_{j in bucket b} s_j AS[j, :], is accumulated in registers alongside the rows
// (no global atomics; fixed reduction order). For SubCount the coordinates outside
// the sketch still need their rows of AS; a second kernel builds those rows.
#include <hipcub/hipcub.hpp>

#include "dev_common.h"
#include "rs_internal.h"

namespace rs {
namespace {

constexpr int kWaves = 4;
constexpr int kMaxTauChunks = 32;  // tau <= 2048

// One wavefront: acc[0 .. tau) <- row j of AS (acc is this wave's LDS slice).
__device__ __forceinline__ void scatter_row(int64_t j, const int64_t* __restrict__ zr_ptr,
                                            const int32_t* __restrict__ zr_col,
                                            const double* __restrict__ zr_val,
                                            const int64_t* __restrict__ zt_ptr,
                                            const int32_t* __restrict__ zt_col,
                                            const double* __restrict__ zt_val,
                                            const int32_t* __restrict__ hmap, int32_t tau,
                                            double lam, double* acc, int lane) {
  for (int c = lane; c < tau; c += 64) acc[c] = 0.0;
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  const int64_t p0 = zr_ptr[j], p1 = zr_ptr[j + 1];
  for (int64_t p = p0 + lane; p < p1; p += 64) {
    const int64_t i = zr_col[p];
    const double zv = zr_val[p];
    const int64_t q0 = zt_ptr[i], q1 = zt_ptr[i + 1];
    for (int64_t q = q0; q < q1; ++q) {
      const int code = hmap[zt_col[q]];
      if (code >= 0) {
        double v = zv * zt_val[q];
        if (code & 1) v = -v;
        atomicAdd(&acc[code >> 1], v);
      }
    }
  }
  const int cj = hmap[j];
  if (lane == 0 && cj >= 0) atomicAdd(&acc[cj >> 1], (cj & 1) ? -lam : lam);
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__global__ __launch_bounds__(kWaves * 64) void k_as_sparse_bucket(
    const int64_t* __restrict__ zr_ptr, const int32_t* __restrict__ zr_col,
    const double* __restrict__ zr_val, const int64_t* __restrict__ zt_ptr,
    const int32_t* __restrict__ zt_col, const double* __restrict__ zt_val, int64_t m, int32_t tau,
    double lam, const int32_t* __restrict__ hmap_all, const int32_t* __restrict__ members_all,
    const int32_t* __restrict__ offs_all, int64_t nsel, double* __restrict__ AS,
    double* __restrict__ G, int64_t ldg, const int32_t* __restrict__ done) {
  extern __shared__ __align__(16) double lds[];  // [kWaves][tau]
  if (*done) return;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int b = blockIdx.x;
  const int64_t slot = blockIdx.y;
  const int32_t* hmap = hmap_all + slot * m;
  const int32_t* members = members_all + slot * nsel;
  const int32_t* offs = offs_all + slot * (tau + 1);
  double* acc = lds + wave * tau;
  double gp[kMaxTauChunks];
#pragma unroll
  for (int t = 0; t < kMaxTauChunks; ++t) gp[t] = 0.0;

  const int p0 = offs[b], p1 = offs[b + 1];
  for (int p = p0 + wave; p < p1; p += kWaves) {
    const int64_t j = members[p];
    scatter_row(j, zr_ptr, zr_col, zr_val, zt_ptr, zt_col, zt_val, hmap, tau, lam, acc, lane);
    const double sj = (hmap[j] & 1) ? -1.0 : 1.0;
    double* out = AS + (slot * m + j) * tau;
#pragma unroll
    for (int t = 0; t < kMaxTauChunks; ++t) {
      const int c = lane + 64 * t;
      if (c < tau) {
        const double v = acc[c];
        out[c] = v;
        gp[t] += sj * v;
      }
    }
    __builtin_amdgcn_wave_barrier();
  }
  __syncthreads();
#pragma unroll
  for (int t = 0; t < kMaxTauChunks; ++t) {
    const int c = lane + 64 * t;
    if (c < tau) acc[c] = gp[t];
  }
  __syncthreads();
  double* grow = G + (slot * ldg + b) * ldg;
  for (int c = tid; c < tau; c += kWaves * 64) {
    double v = 0.0;
    for (int w = 0; w < kWaves; ++w) v += lds[w * tau + c];
    grow[c] = v;
  }
}

// Rows of AS for coordinates outside the sketch (SubCount); one wavefront per row.
__global__ __launch_bounds__(kWaves * 64) void k_as_sparse_rows(
    const int64_t* __restrict__ zr_ptr, const int32_t* __restrict__ zr_col,
    const double* __restrict__ zr_val, const int64_t* __restrict__ zt_ptr,
    const int32_t* __restrict__ zt_col, const double* __restrict__ zt_val, int64_t m, int32_t tau,
    double lam, const int32_t* __restrict__ hmap_all, double* __restrict__ AS,
    const int32_t* __restrict__ done) {
  extern __shared__ __align__(16) double lds[];
  if (*done) return;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t slot = blockIdx.y;
  const int64_t j = (int64_t)blockIdx.x * kWaves + wave;
  if (j >= m) return;
  const int32_t* hmap = hmap_all + slot * m;
  if (hmap[j] >= 0) return;  // member rows come from the bucket kernel
  double* acc = lds + wave * tau;
  scatter_row(j, zr_ptr, zr_col, zr_val, zt_ptr, zt_col, zt_val, hmap, tau, lam, acc, lane);
  double* out = AS + (slot * m + j) * tau;
  for (int c = lane; c < tau; c += 64) out[c] = acc[c];
}

__global__ void k_spmv_csr(const int64_t* __restrict__ ptr, const int32_t* __restrict__ col,
                           const double* __restrict__ val, int64_t rows, const double* __restrict__ v,
                           double* __restrict__ out) {
  const int lane = threadIdx.x & 63;
  const int64_t r = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (r >= rows) return;
  double s = 0.0;
  for (int64_t p = ptr[r] + lane; p < ptr[r + 1]; p += 64) s += val[p] * v[col[p]];
  s = wave_sum(s);
  if (lane == 0) out[r] = s;
}

// ---- CSR transpose (setup) ----
__global__ void k_expand_rows(const int64_t* __restrict__ ptr, int64_t rows, int32_t* __restrict__ row_of) {
  const int64_t r = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (r >= rows) return;
  for (int64_t p = ptr[r] + lane; p < ptr[r + 1]; p += 64) row_of[p] = (int32_t)r;
}

__global__ void k_iota(int32_t* __restrict__ v, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) v[i] = (int32_t)i;
}

__global__ void k_gather_transposed(const int32_t* __restrict__ perm, const int32_t* __restrict__ row_of,
                                    const void* __restrict__ val, int32_t is_f32, int64_t nnz,
                                    int32_t* __restrict__ tcol, double* __restrict__ tval) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nnz) return;
  const int32_t p = perm[i];
  tcol[i] = row_of[p];
  tval[i] = is_f32 ? (double)((const float*)val)[p] : ((const double*)val)[p];
}

// tptr[c] = number of sorted keys < c (binary search on the sorted column keys).
__global__ void k_row_ptr_from_sorted(const int32_t* __restrict__ keys, int64_t nnz, int64_t cols,
                                      int64_t* __restrict__ tptr) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c > cols) return;
  int64_t lo = 0, hi = nnz;
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if (keys[mid] < c) lo = mid + 1; else hi = mid;
  }
  tptr[c] = lo;
}

}  // namespace

hipError_t launch_as_sparse_f64(const int64_t* zr_ptr, const int32_t* zr_col, const double* zr_val,
                                const int64_t* zt_ptr, const int32_t* zt_col, const double* zt_val,
                                int64_t m, int32_t tau, int32_t nslots, int32_t kind, double lam,
                                const int32_t* hmap, const int32_t* members, const int32_t* offs,
                                int64_t nsel, double* AS, double* G, int64_t ldg,
                                const int32_t* done, hipStream_t s) {
  if (tau > 64 * kMaxTauChunks) return hipErrorInvalidValue;
  const size_t bytes = sizeof(double) * kWaves * (size_t)tau;
  hipError_t e = hipFuncSetAttribute((const void*)k_as_sparse_bucket,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_as_sparse_bucket, dim3(tau, nslots), dim3(kWaves * 64), bytes, s, zr_ptr,
                     zr_col, zr_val, zt_ptr, zt_col, zt_val, m, tau, lam, hmap, members, offs, nsel,
                     AS, G, ldg, done);
  e = hipGetLastError();
  if (e != hipSuccess || kind != kSubcount) return e;
  e = hipFuncSetAttribute((const void*)k_as_sparse_rows,
                          hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_as_sparse_rows, dim3((unsigned)((m + kWaves - 1) / kWaves), nslots),
                     dim3(kWaves * 64), bytes, s, zr_ptr, zr_col, zr_val, zt_ptr, zt_col, zt_val, m,
                     tau, lam, hmap, AS, done);
  return hipGetLastError();
}

hipError_t launch_spmv_csr(const int64_t* ptr, const int32_t* col, const double* val, int64_t rows,
                           const double* v, double* out, hipStream_t s) {
  if (rows == 0) return hipSuccess;
  hipLaunchKernelGGL(k_spmv_csr, dim3((unsigned)((rows + 3) / 4)), dim3(256), 0, s, ptr, col, val,
                     rows, v, out);
  return hipGetLastError();
}

hipError_t csr_transpose(const int64_t* ptr, const int32_t* col, const void* val, int32_t val_is_f32,
                         int64_t rows, int64_t cols, int64_t nnz, int64_t* tptr, int32_t* tcol,
                         double* tval, hipStream_t s) {
  if (nnz == 0) {
    return hipMemsetAsync(tptr, 0, sizeof(int64_t) * (cols + 1), s);
  }
  int32_t *row_of = nullptr, *keys_out = nullptr, *idx_in = nullptr, *idx_out = nullptr;
  void* tmp = nullptr;
  size_t tmp_bytes = 0;
  hipError_t e = hipMalloc(&row_of, sizeof(int32_t) * nnz);
  if (e == hipSuccess) e = hipMalloc(&keys_out, sizeof(int32_t) * nnz);
  if (e == hipSuccess) e = hipMalloc(&idx_in, sizeof(int32_t) * nnz);
  if (e == hipSuccess) e = hipMalloc(&idx_out, sizeof(int32_t) * nnz);
  int end_bit = 1;
  while (end_bit < 31 && (1ll << end_bit) <= cols) ++end_bit;
  if (e == hipSuccess)
    e = hipcub::DeviceRadixSort::SortPairs(nullptr, tmp_bytes, col, keys_out, idx_in, idx_out,
                                           (int)nnz, 0, end_bit, s);
  if (e == hipSuccess) e = hipMalloc(&tmp, tmp_bytes);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k_expand_rows, dim3((unsigned)((rows + 3) / 4)), dim3(256), 0, s, ptr, rows,
                       row_of);
    hipLaunchKernelGGL(k_iota, dim3((unsigned)((nnz + 255) / 256)), dim3(256), 0, s, idx_in, nnz);
    e = hipcub::DeviceRadixSort::SortPairs(tmp, tmp_bytes, col, keys_out, idx_in, idx_out, (int)nnz,
                                           0, end_bit, s);
  }
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k_gather_transposed, dim3((unsigned)((nnz + 255) / 256)), dim3(256), 0, s,
                       idx_out, row_of, val, val_is_f32, nnz, tcol, tval);
    hipLaunchKernelGGL(k_row_ptr_from_sorted, dim3((unsigned)((cols + 1 + 255) / 256)), dim3(256),
                       0, s, keys_out, nnz, cols, tptr);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  (void)hipFree(row_of);
  (void)hipFree(keys_out);
  (void)hipFree(idx_in);
  (void)hipFree(idx_out);
  (void)hipFree(tmp);
  return e;
}

}  // namespace rs
