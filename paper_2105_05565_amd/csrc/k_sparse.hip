// Count and SubCount sketch products for CSR data (Sec. 4.2).
//
// With Z the m x K operand of A = Z Z^T + lambda I (primal Z = X^T, dual Z = X):
//
//   AS[j, :] = sum_{i in row j of Z} Z_ji T[i, :] + lambda s_j e_{h(j)},
//   T[i, :]  = sum_{j' in row i of Z^T} s_j' Z_j'i e_{h(j')}          (T = Z^T S),
//
// where h(j) is the bucket (column of S) holding coordinate j and s_j its sign.
// Per sketch, one streaming pass stores T entry by entry, aligned with CSR(Z^T), as
// (bucket, signed value). Each row of AS is then built by one wavefront as a signed
// scatter-add of Z_ji T[i, :] into tau bucket accumulators staged in LDS; the wave
// splits into 16-lane groups that each walk one row of T (coalesced segments).
// Buckets are processed by one workgroup each, so G = S^T A S,
// whose row b is sum_{j in bucket b} s_j AS[j, :], is accumulated alongside the
// rows in LDS (no global atomics; fixed reduction order across waves). For SubCount
// the coordinates outside the sketch still need their rows of AS; a second kernel
// builds those rows.
//
// CSR values are held in the input precision (FP32 inputs stay FP32: exactly
// representable, and their pairwise products are exact in FP64); every product and
// sum is formed in FP64.
#include <hipcub/hipcub.hpp>

#include <algorithm>

#include "dev_common.h"
#include "rs_internal.h"

namespace rs {
namespace {

constexpr int kWaves = 8;

// Entry of T = Z^T S aligned with CSR(Z^T): bucket code of the column (-1: outside the
// sketch) and the signed value s_j' Z_j'i.
template <typename V>
struct TEntry;
template <>
struct __align__(8) TEntry<float> {
  int32_t code;
  float val;
};
template <>
struct __align__(16) TEntry<double> {
  int64_t code;
  double val;
};

// T[slot][q] for every entry q of CSR(Z^T): one pass per sketch, coalesced apart from
// the bucket-map lookup.
template <typename V>
__global__ void k_build_t(const int32_t* __restrict__ zt_col, const V* __restrict__ zt_val,
                          int64_t nnz, const int32_t* __restrict__ hmap_all, int64_t m,
                          TEntry<V>* __restrict__ T, const int32_t* __restrict__ done) {
  if (*done) return;
  const int64_t slot = blockIdx.y;
  const int32_t* hmap = hmap_all + slot * m;
  TEntry<V>* t = T + slot * nnz;
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < nnz;
       q += (int64_t)gridDim.x * blockDim.x) {
    const int code = hmap[zt_col[q]];
    const V v = zt_val[q];
    TEntry<V> e;
    e.code = code < 0 ? -1 : (code >> 1);
    e.val = (code & 1) ? -v : v;
    t[q] = e;
  }
}

struct RowLds {  // per-wave staging of one chunk (<= 64 entries) of row j of Z
  int64_t q0[64];
  int32_t len[64];
  double zv[64];
};

// One wavefront: acc[0 .. tau) <- row j of AS. The wave splits into four 16-lane
// groups; group g walks entries p = g, g + 4, ... of the current chunk of row j and
// its lanes stride over the matching row of Z^T (coalesced 16-entry segments).
template <typename V>
__device__ __forceinline__ void scatter_row(int64_t j, const int64_t* __restrict__ zr_ptr,
                                            const int32_t* __restrict__ zr_col,
                                            const V* __restrict__ zr_val,
                                            const int64_t* __restrict__ zt_ptr,
                                            const TEntry<V>* __restrict__ T, int code_j, int32_t tau,
                                            double lam, double* acc, RowLds* rl, int lane) {
  for (int c = lane; c < tau; c += 64) acc[c] = 0.0;
  const int grp = lane >> 4, sub = lane & 15;
  const int64_t p0 = zr_ptr[j], p1 = zr_ptr[j + 1];
  for (int64_t pb = p0; pb < p1; pb += 64) {
    const int64_t p = pb + lane;
    const int cnt = (int)min<int64_t>(64, p1 - pb);
    if (p < p1) {
      const int64_t i = zr_col[p];
      const int64_t q0 = zt_ptr[i];
      rl->q0[lane] = q0;
      rl->len[lane] = (int)(zt_ptr[i + 1] - q0);
      rl->zv[lane] = (double)zr_val[p];
    }
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    for (int e = grp; e < cnt; e += 4) {
      const int64_t q0 = rl->q0[e];
      const int len = rl->len[e];
      const double zv = rl->zv[e];
      for (int t = sub; t < len; t += 32) {
        const TEntry<V> a = T[q0 + t];
        const bool two = t + 16 < len;
        TEntry<V> b;
        if (two) b = T[q0 + t + 16];
        if (a.code >= 0) atomicAdd(&acc[a.code], zv * (double)a.val);
        if (two && b.code >= 0) atomicAdd(&acc[b.code], zv * (double)b.val);
      }
    }
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
  }
  if (lane == 0 && code_j >= 0) atomicAdd(&acc[code_j >> 1], (code_j & 1) ? -lam : lam);
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
}

// One workgroup per bucket b of a sketch: its member rows of AS and row b of G.
// NCH = number of 64-column chunks of tau held per lane for the G partial sums.
template <typename V, int NCH>
__device__ __forceinline__ void bucket_body(
    const int64_t* __restrict__ zr_ptr, const int32_t* __restrict__ zr_col,
    const V* __restrict__ zr_val, const int64_t* __restrict__ zt_ptr,
    const TEntry<V>* __restrict__ T_all, int64_t nnz, int64_t m, int32_t tau, int64_t ldas,
    double lam, const int32_t* __restrict__ hmap_all, const int32_t* __restrict__ members_all,
    const int32_t* __restrict__ offs_all, int64_t nsel, double* __restrict__ AS,
    double* __restrict__ G, int64_t ldg, int b, int64_t slot, double* lds, RowLds* rls) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int32_t* hmap = hmap_all + slot * m;
  const int32_t* members = members_all + slot * nsel;
  const int32_t* offs = offs_all + slot * (tau + 1);
  const TEntry<V>* T = T_all + slot * nnz;
  double* acc = lds + wave * tau;
  double gp[NCH];
#pragma unroll
  for (int t = 0; t < NCH; ++t) gp[t] = 0.0;

  const int p0 = offs[b], p1 = offs[b + 1];
  for (int p = p0 + wave; p < p1; p += kWaves) {
    const int64_t j = members[p];
    const int cj = hmap[j];
    scatter_row<V>(j, zr_ptr, zr_col, zr_val, zt_ptr, T, cj, tau, lam, acc, &rls[wave], lane);
    const double sj = (cj & 1) ? -1.0 : 1.0;
    double* out = AS + (slot * m + j) * ldas;
#pragma unroll
    for (int t = 0; t < NCH; ++t) {
      const int c = lane + 64 * t;
      if (c < tau) {
        const double v = acc[c];
        out[c] = v;
        gp[t] += sj * v;
      }
    }
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
  }
  __syncthreads();
#pragma unroll
  for (int t = 0; t < NCH; ++t) {
    const int c = lane + 64 * t;
    if (c < tau) acc[c] = gp[t];
  }
  __syncthreads();
  double* grow = G + (slot * ldg + b) * ldg;
  for (int c = tid; c < tau; c += kWaves * 64) {
    double v = 0.0;
#pragma unroll
    for (int w = 0; w < kWaves; ++w) v += lds[w * tau + c];
    grow[c] = v;
  }
  __syncthreads();  // lds is reused by the next bucket of a persistent workgroup
}

template <typename V, int NCH>
__global__ __launch_bounds__(kWaves * 64) void k_as_sparse_bucket(
    const int64_t* __restrict__ zr_ptr, const int32_t* __restrict__ zr_col,
    const V* __restrict__ zr_val, const int64_t* __restrict__ zt_ptr,
    const TEntry<V>* __restrict__ T_all, int64_t nnz, int64_t m, int32_t tau, int64_t ldas,
    double lam, const int32_t* __restrict__ hmap_all, const int32_t* __restrict__ members_all,
    const int32_t* __restrict__ offs_all, int64_t nsel, double* __restrict__ AS,
    double* __restrict__ G, int64_t ldg, const int32_t* __restrict__ done) {
  extern __shared__ __align__(16) double lds[];  // acc [kWaves][tau]
  __shared__ RowLds rls[kWaves];
  if (*done) return;
  bucket_body<V, NCH>(zr_ptr, zr_col, zr_val, zt_ptr, T_all, nnz, m, tau, ldas, lam, hmap_all,
                      members_all, offs_all, nsel, AS, G, ldg, blockIdx.x, blockIdx.y, lds, rls);
}

// Grouped forms (batched solves, FP64 values): T for every job (blockIdx.y = job), then
// a persistent grid striding over the ragged table of (job, bucket) pairs.
__global__ void k_build_t_tab(const SparseJob* __restrict__ jobs) {
  const SparseJob& j = jobs[blockIdx.y];
  if (*j.done) return;
  TEntry<double>* t = static_cast<TEntry<double>*>(j.tbuf);
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < j.nnz;
       q += (int64_t)gridDim.x * blockDim.x) {
    const int code = j.hmap[j.zt_col[q]];
    const double v = j.zt_val[q];
    TEntry<double> e;
    e.code = code < 0 ? -1 : (code >> 1);
    e.val = (code & 1) ? -v : v;
    t[q] = e;
  }
}

template <int NCH>
__global__ __launch_bounds__(kWaves * 64) void k_as_sparse_bucket_tab(
    const SparseJob* __restrict__ jobs, const int32_t* __restrict__ items, int32_t nitems) {
  extern __shared__ __align__(16) double lds[];  // acc [kWaves][max tau]
  __shared__ RowLds rls[kWaves];
  for (int32_t t = blockIdx.x; t < nitems; t += gridDim.x) {
    const int32_t job = items[2 * t], b = items[2 * t + 1];
    const SparseJob& j = jobs[job];
    if (*j.done) continue;  // uniform across the workgroup
    bucket_body<double, NCH>(j.zr_ptr, j.zr_col, j.zr_val, j.zt_ptr,
                             static_cast<const TEntry<double>*>(j.tbuf), j.nnz, j.m, j.tau, j.ldas,
                             j.lam, j.hmap, j.members, j.offs, j.nsel, j.AS, j.G, j.ldg, b, 0, lds,
                             rls);
  }
}

// Rows of AS for coordinates outside the sketch (SubCount); one wavefront per row.
template <typename V>
__global__ __launch_bounds__(kWaves * 64) void k_as_sparse_rows(
    const int64_t* __restrict__ zr_ptr, const int32_t* __restrict__ zr_col,
    const V* __restrict__ zr_val, const int64_t* __restrict__ zt_ptr,
    const TEntry<V>* __restrict__ T_all, int64_t nnz, int64_t m, int32_t tau, int64_t ldas,
    double lam, const int32_t* __restrict__ hmap_all, double* __restrict__ AS,
    const int32_t* __restrict__ done) {
  extern __shared__ __align__(16) double lds[];
  __shared__ RowLds rls[kWaves];
  if (*done) return;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t slot = blockIdx.y;
  const int64_t j = (int64_t)blockIdx.x * kWaves + wave;
  if (j >= m) return;
  const int32_t* hmap = hmap_all + slot * m;
  const int cj = hmap[j];
  if (cj >= 0) return;  // member rows come from the bucket kernel
  double* acc = lds + wave * tau;
  scatter_row<V>(j, zr_ptr, zr_col, zr_val, zt_ptr, T_all + slot * nnz, cj, tau, lam, acc,
                 &rls[wave], lane);
  double* out = AS + (slot * m + j) * ldas;
  for (int c = lane; c < tau; c += 64) out[c] = acc[c];
}

template <typename V>
__global__ void k_spmv_csr(const int64_t* __restrict__ ptr, const int32_t* __restrict__ col,
                           const V* __restrict__ val, int64_t rows, const double* __restrict__ v,
                           double* __restrict__ out) {
  const int lane = threadIdx.x & 63;
  const int64_t r = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (r >= rows) return;
  double s = 0.0;
  for (int64_t p = ptr[r] + lane; p < ptr[r + 1]; p += 64) s += (double)val[p] * v[col[p]];
  s = wave_sum(s);
  if (lane == 0) out[r] = s;
}

// Two sparse products sharing each row's pass: o0 = M v0, o1 = M v1 (FP64 accumulation), one
// wave per row; skipped once the solve has stopped.
template <typename V>
__global__ void k_spmv_pair(const int64_t* __restrict__ ptr, const int32_t* __restrict__ col,
                            const V* __restrict__ val, int64_t rows, const double* __restrict__ v0,
                            const double* __restrict__ v1, double* __restrict__ o0, double* __restrict__ o1,
                            const DevFlags* __restrict__ flags) {
  if (flags->done) return;
  const int lane = threadIdx.x & 63;
  const int64_t r = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (r >= rows) return;
  double s0 = 0.0, s1 = 0.0;
  for (int64_t p = ptr[r] + lane; p < ptr[r + 1]; p += 64) {
    const double a = (double)val[p];
    const int32_t c = col[p];
    s0 += a * v0[c];
    s1 += a * v1[c];
  }
  s0 = wave_sum(s0);
  s1 = wave_sum(s1);
  if (lane == 0) {
    o0[r] = s0;
    o1[r] = s1;
  }
}

constexpr int kRefreshRows = 1024;  // rows per workgroup of the residual kernel

// r = t0 + lambda x - b, rp = t1 + lambda xp - b; partial sums of ||r||^2 per workgroup.
__global__ __launch_bounds__(256) void k_resid_pair(const double* __restrict__ t0, const double* __restrict__ t1,
                                                    const double* __restrict__ x, const double* __restrict__ xp,
                                                    const double* __restrict__ b, double lam, int64_t m,
                                                    double* __restrict__ r, double* __restrict__ rp,
                                                    double* __restrict__ partials,
                                                    const DevFlags* __restrict__ flags) {
  __shared__ double scratch[16];
  if (flags->done) return;
  const int64_t j0 = (int64_t)blockIdx.x * kRefreshRows, j1 = min(m, j0 + kRefreshRows);
  double ss = 0.0;
  for (int64_t j = j0 + threadIdx.x; j < j1; j += blockDim.x) {
    const double rn = t0[j] + lam * x[j] - b[j];
    r[j] = rn;
    rp[j] = t1[j] + lam * xp[j] - b[j];
    ss += rn * rn;
  }
  ss = block_sum(ss, scratch);
  if (threadIdx.x == 0) partials[blockIdx.x] = ss;
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

template <typename V>
__global__ void k_gather_transposed(const int32_t* __restrict__ perm, const int32_t* __restrict__ row_of,
                                    const V* __restrict__ val, int64_t nnz, int32_t* __restrict__ tcol,
                                    V* __restrict__ tval) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nnz) return;
  const int32_t p = perm[i];
  tcol[i] = row_of[p];
  tval[i] = val[p];
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

template <typename V, int NCH>
hipError_t bucket_launch(const int64_t* zr_ptr, const int32_t* zr_col, const V* zr_val,
                         const int64_t* zt_ptr, const TEntry<V>* T, int64_t nnz, int64_t m,
                         int32_t tau, int64_t ldas, int32_t nslots, double lam, const int32_t* hmap,
                         const int32_t* members, const int32_t* offs, int64_t nsel, double* AS,
                         double* G, int64_t ldg, const int32_t* done, hipStream_t s) {
  const size_t bytes = sizeof(double) * kWaves * (size_t)tau;
  hipError_t e = hipFuncSetAttribute((const void*)k_as_sparse_bucket<V, NCH>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_as_sparse_bucket<V, NCH>), dim3(tau, nslots), dim3(kWaves * 64), bytes, s,
                     zr_ptr, zr_col, zr_val, zt_ptr, T, nnz, m, tau, ldas, lam, hmap, members, offs,
                     nsel, AS, G, ldg, done);
  return hipGetLastError();
}

template <typename V>
hipError_t as_sparse(const int64_t* zr_ptr, const int32_t* zr_col, const V* zr_val,
                     const int64_t* zt_ptr, const int32_t* zt_col, const V* zt_val, int64_t nnz,
                     int64_t m, int32_t tau, int64_t ldas, int32_t nslots, int32_t kind, double lam,
                     const int32_t* hmap, const int32_t* members, const int32_t* offs, int64_t nsel,
                     void* tbuf, double* AS, double* G, int64_t ldg, const int32_t* done,
                     hipStream_t s) {
  const TEntry<V>* T = static_cast<const TEntry<V>*>(tbuf);
  hipError_t e = hipSuccess;
  if (tau <= 512)
    e = bucket_launch<V, 8>(zr_ptr, zr_col, zr_val, zt_ptr, T, nnz, m, tau, ldas, nslots, lam, hmap,
                            members, offs, nsel, AS, G, ldg, done, s);
  else if (tau <= 1024)
    e = bucket_launch<V, 16>(zr_ptr, zr_col, zr_val, zt_ptr, T, nnz, m, tau, ldas, nslots, lam, hmap,
                             members, offs, nsel, AS, G, ldg, done, s);
  else
    e = bucket_launch<V, 32>(zr_ptr, zr_col, zr_val, zt_ptr, T, nnz, m, tau, ldas, nslots, lam, hmap,
                             members, offs, nsel, AS, G, ldg, done, s);
  if (e != hipSuccess || kind != kSubcount) return e;
  const size_t rbytes = sizeof(double) * kWaves * (size_t)tau;
  e = hipFuncSetAttribute((const void*)k_as_sparse_rows<V>,
                          hipFuncAttributeMaxDynamicSharedMemorySize, (int)rbytes);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_as_sparse_rows<V>, dim3((unsigned)((m + kWaves - 1) / kWaves), nslots),
                     dim3(kWaves * 64), rbytes, s, zr_ptr, zr_col, zr_val, zt_ptr, T, nnz, m, tau,
                     ldas, lam, hmap, AS, done);
  return hipGetLastError();
}

template <typename V>
hipError_t transpose_impl(const int64_t* ptr, const int32_t* col, const V* val, int64_t rows,
                          int64_t cols, int64_t nnz, int64_t* tptr, int32_t* tcol, V* tval,
                          hipStream_t s) {
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
    hipLaunchKernelGGL(k_gather_transposed<V>, dim3((unsigned)((nnz + 255) / 256)), dim3(256), 0, s,
                       idx_out, row_of, val, nnz, tcol, tval);
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

}  // namespace

size_t sparse_t_bytes(int32_t vals_f32, int64_t nnz) {
  return (size_t)nnz * (vals_f32 ? sizeof(TEntry<float>) : sizeof(TEntry<double>));
}

hipError_t launch_build_t(const int32_t* zt_col, const void* zt_val, int32_t vals_f32, int64_t nnz,
                          const int32_t* hmap, int64_t m, int32_t nslots, void* tbuf,
                          const int32_t* done, hipStream_t s) {
  if (nnz == 0) return hipSuccess;
  const unsigned gx = (unsigned)std::min<int64_t>(4096, (nnz + 255) / 256);
  if (vals_f32)
    hipLaunchKernelGGL(k_build_t<float>, dim3(gx, nslots), dim3(256), 0, s, zt_col,
                       (const float*)zt_val, nnz, hmap, m, (TEntry<float>*)tbuf, done);
  else
    hipLaunchKernelGGL(k_build_t<double>, dim3(gx, nslots), dim3(256), 0, s, zt_col,
                       (const double*)zt_val, nnz, hmap, m, (TEntry<double>*)tbuf, done);
  return hipGetLastError();
}

hipError_t launch_as_sparse(const int64_t* zr_ptr, const int32_t* zr_col, const void* zr_val,
                            const int64_t* zt_ptr, const int32_t* zt_col, const void* zt_val,
                            int32_t vals_f32, int64_t nnz, int64_t m, int32_t tau, int64_t ldas,
                            int32_t nslots, int32_t kind, double lam, const int32_t* hmap,
                            const int32_t* members, const int32_t* offs, int64_t nsel, void* tbuf,
                            double* AS, double* G, int64_t ldg, const int32_t* done, hipStream_t s) {
  if (tau > 2048) return hipErrorInvalidValue;
  if (vals_f32)
    return as_sparse<float>(zr_ptr, zr_col, (const float*)zr_val, zt_ptr, zt_col, (const float*)zt_val,
                            nnz, m, tau, ldas, nslots, kind, lam, hmap, members, offs, nsel, tbuf, AS, G,
                            ldg, done, s);
  return as_sparse<double>(zr_ptr, zr_col, (const double*)zr_val, zt_ptr, zt_col,
                           (const double*)zt_val, nnz, m, tau, ldas, nslots, kind, lam, hmap, members,
                           offs, nsel, tbuf, AS, G, ldg, done, s);
}

hipError_t launch_spmv_csr(const int64_t* ptr, const int32_t* col, const void* val, int32_t vals_f32,
                           int64_t rows, const double* v, double* out, hipStream_t s) {
  if (rows == 0) return hipSuccess;
  if (vals_f32)
    hipLaunchKernelGGL(k_spmv_csr<float>, dim3((unsigned)((rows + 3) / 4)), dim3(256), 0, s, ptr,
                       col, (const float*)val, rows, v, out);
  else
    hipLaunchKernelGGL(k_spmv_csr<double>, dim3((unsigned)((rows + 3) / 4)), dim3(256), 0, s, ptr,
                       col, (const double*)val, rows, v, out);
  return hipGetLastError();
}

int64_t refresh_csr_partials(int64_t m) { return (m + kRefreshRows - 1) / kRefreshRows; }

hipError_t launch_refresh_csr(const int64_t* zr_ptr, const int32_t* zr_col, const void* zr_val,
                              const int64_t* zt_ptr, const int32_t* zt_col, const void* zt_val, int32_t vals_f32,
                              int64_t m, int64_t K, const double* x, const double* xp, const double* b, double lam,
                              double* r, double* rp, double* u, double* t, double* partials, DevFlags* flags,
                              double* hist, double* true_hist, int64_t k, double tol, hipStream_t s) {
  if (m <= 0 || K <= 0) return hipErrorInvalidValue;
  // u = Z^T [x, xp] (K rows of CSR(Z^T)), then t = Z u (m rows of CSR(Z))
  if (vals_f32) {
    hipLaunchKernelGGL(k_spmv_pair<float>, dim3((unsigned)((K + 3) / 4)), dim3(256), 0, s, zt_ptr, zt_col,
                       (const float*)zt_val, K, x, xp, u, u + K, flags);
    hipLaunchKernelGGL(k_spmv_pair<float>, dim3((unsigned)((m + 3) / 4)), dim3(256), 0, s, zr_ptr, zr_col,
                       (const float*)zr_val, m, u, u + K, t, t + m, flags);
  } else {
    hipLaunchKernelGGL(k_spmv_pair<double>, dim3((unsigned)((K + 3) / 4)), dim3(256), 0, s, zt_ptr, zt_col,
                       (const double*)zt_val, K, x, xp, u, u + K, flags);
    hipLaunchKernelGGL(k_spmv_pair<double>, dim3((unsigned)((m + 3) / 4)), dim3(256), 0, s, zr_ptr, zr_col,
                       (const double*)zr_val, m, u, u + K, t, t + m, flags);
  }
  const int64_t np = refresh_csr_partials(m);
  hipLaunchKernelGGL(k_resid_pair, dim3((unsigned)np), dim3(256), 0, s, t, t + m, x, xp, b, lam, m, r, rp, partials,
                     flags);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return launch_refresh_norm(partials, (int32_t)np, flags, hist, true_hist, k, tol, s);
}

hipError_t csr_transpose(const int64_t* ptr, const int32_t* col, const void* val, int32_t vals_f32,
                         int64_t rows, int64_t cols, int64_t nnz, int64_t* tptr, int32_t* tcol,
                         void* tval, hipStream_t s) {
  if (nnz == 0) return hipMemsetAsync(tptr, 0, sizeof(int64_t) * (cols + 1), s);
  if (vals_f32)
    return transpose_impl<float>(ptr, col, (const float*)val, rows, cols, nnz, tptr, tcol,
                                 (float*)tval, s);
  return transpose_impl<double>(ptr, col, (const double*)val, rows, cols, nnz, tptr, tcol,
                                (double*)tval, s);
}

hipError_t launch_sparse_tab(const SparseJob* jobs, int32_t njobs, const int32_t* items,
                             int32_t nitems, int32_t max_tau, int32_t grid, hipStream_t s) {
  if (njobs <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_build_t_tab, dim3(256, njobs), dim3(256), 0, s, jobs);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  grid = grid < 1 ? 1 : (grid > nitems ? nitems : grid);
  const size_t bytes = sizeof(double) * kWaves * (size_t)max_tau;
  if (max_tau <= 512) {
    e = hipFuncSetAttribute((const void*)k_as_sparse_bucket_tab<8>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_as_sparse_bucket_tab<8>, dim3(grid), dim3(kWaves * 64), bytes, s, jobs,
                       items, nitems);
  } else if (max_tau <= 1024) {
    e = hipFuncSetAttribute((const void*)k_as_sparse_bucket_tab<16>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_as_sparse_bucket_tab<16>, dim3(grid), dim3(kWaves * 64), bytes, s, jobs,
                       items, nitems);
  } else {
    return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

size_t sparse_entry_bytes_f64() { return sizeof(TEntry<double>); }

}  // namespace rs
