// Count / SubCount products through the rows of A0 = Z Z^T (Sec. 4.2: a count sketch
// costs O(nnz(A))).
//
// For a sparse Z, A0 is itself sparse and does not depend on the sketch, so it is
// formed once (a sparse product Z Z^T = sum_i z_i z_i^T over the rows z_i of Z^T,
// products in FP64) and every sketch then needs
//
//   AS[j, :] = sum_{j'} A0[j, j'] s_{j'} e_{h(j')} + lambda s_j e_{h(j)}
//
// -- a signed scatter-add of row j of A0 into tau bucket accumulators in LDS, through the
// bucket map of the sketch. One wavefront per sketch and a workgroup of several sketches
// per row: the row of A0 is read once for all of them, and the bucket maps of the
// workgroup's sketches (m ints each) stay in L2 while the rows stream. G = S^T AS then
// takes one bucket-major pass over the member rows of AS.
#include <hipcub/hipcub.hpp>

#include "dev_common.h"
#include "rs_internal.h"

namespace rs {
namespace {

constexpr int kGroups = 16;
constexpr int kLdsGroups = 8;
constexpr int kLdsRows = 64;  // rows of AS per workgroup in the LDS-map kernel

size_t arows_lds_bytes(int64_t m, int32_t tau) {
  return (size_t)((2 * m + 15) & ~15ll) + sizeof(double) * 8 * (size_t)tau;
}

// Packed bucket map for larger m: three 10-bit codes per 32-bit word (2 bucket + sign, 1023 = no
// entry; tau <= 511), beside the accumulators of kPackedWaves waves.
constexpr int kPackedWaves = 4;
constexpr uint32_t kNoCode = 1023;
size_t arows_packed_lds_bytes(int64_t m, int32_t tau) {
  return (size_t)(((m + 2) / 3 * 4 + 15) & ~15ll) + sizeof(double) * kPackedWaves * (size_t)tau;
}

// cnt[i] = (row length of Z^T)^2: the products row i contributes to Z Z^T.
__global__ void k_pair_counts(const int64_t* __restrict__ zt_ptr, int64_t K, int64_t* __restrict__ cnt) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= K) return;
  const int64_t L = zt_ptr[i + 1] - zt_ptr[i];
  cnt[i] = L * L;
}

// One wavefront per row i of Z^T: every ordered pair (a, b) of its entries gives key
// (col_a << 32 | col_b) and value z_a z_b (exact in FP64 for FP32 data).
template <typename V>
__global__ void k_pair_emit(const int64_t* __restrict__ zt_ptr, const int32_t* __restrict__ zt_col,
                            const V* __restrict__ zt_val, int64_t K, const int64_t* __restrict__ off,
                            uint64_t* __restrict__ keys, double* __restrict__ vals) {
  const int lane = threadIdx.x & 63;
  const int64_t i = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (i >= K) return;
  const int64_t q0 = zt_ptr[i];
  const int64_t L = zt_ptr[i + 1] - q0;
  const int64_t o = off[i];
  for (int64_t p = lane; p < L * L; p += 64) {
    const int64_t a = p / L, b = p - a * L;
    const uint64_t ja = (uint64_t)(uint32_t)zt_col[q0 + a], jb = (uint64_t)(uint32_t)zt_col[q0 + b];
    keys[o + p] = (ja << 32) | jb;
    vals[o + p] = (double)zt_val[q0 + a] * (double)zt_val[q0 + b];
  }
}

// a_ptr[r] = first unique key with row >= r; a_col from the low half of the keys.
__global__ void k_a_structure(const uint64_t* __restrict__ ukeys, int64_t nu, int64_t m,
                              int64_t* __restrict__ a_ptr, int32_t* __restrict__ a_col) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < nu) a_col[t] = (int32_t)(ukeys[t] & 0xffffffffull);
  if (t <= m) {
    const uint64_t target = (uint64_t)t << 32;
    int64_t lo = 0, hi = nu;
    while (lo < hi) {
      const int64_t mid = (lo + hi) >> 1;
      if (ukeys[mid] < target) lo = mid + 1; else hi = mid;
    }
    a_ptr[t] = lo;
  }
}

// Rows j0 .. j1 of AS for WAVES sketches (wave w: sketch blockIdx.y * WAVES + w). The bucket
// sums are FP64; OutT is the stored type of AS (FP64, or FP32 in mixed precision).
template <int WAVES, typename OutT>
__global__ __launch_bounds__(WAVES * 64) void k_as_arows(const int64_t* __restrict__ a_ptr,
                                                          const int32_t* __restrict__ a_col,
                                                          const double* __restrict__ a_val, int64_t m,
                                                          int32_t tau, int64_t ldas, int32_t nslots,
                                                          double lam, const int32_t* __restrict__ hmap_all,
                                                          OutT* __restrict__ AS, int32_t rows_per_block,
                                                          const int32_t* __restrict__ done) {
  extern __shared__ __align__(16) double lds[];  // [WAVES][tau]
  if (*done) return;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t slot = (int64_t)blockIdx.y * WAVES + wave;
  if (slot >= nslots) return;  // waves are independent: no workgroup barrier below
  const int32_t* hmap = hmap_all + slot * m;
  double* acc = lds + (int64_t)wave * tau;
  OutT* out_base = AS + slot * m * ldas;
  const int64_t j0 = (int64_t)blockIdx.x * rows_per_block;
  const int64_t j1 = min(m, j0 + rows_per_block);
  for (int64_t j = j0; j < j1; ++j) {
    for (int c = lane; c < tau; c += 64) acc[c] = 0.0;
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    const int64_t p0 = a_ptr[j], p1 = a_ptr[j + 1];
    // kGroups 64-entry groups per step: every load of a step (columns and values, then the
    // bucket codes they index) is issued before its atomics, so that a wave keeps
    // 64 kGroups gathers in flight
    for (int64_t pb = p0; pb < p1; pb += 64 * kGroups) {
      int32_t col[kGroups];
      double val[kGroups];
#pragma unroll
      for (int u = 0; u < kGroups; ++u) {
        const int64_t p = pb + u * 64 + lane;
        col[u] = p < p1 ? a_col[p] : -1;
        val[u] = p < p1 ? a_val[p] : 0.0;
      }
      int code[kGroups];
#pragma unroll
      for (int u = 0; u < kGroups; ++u) code[u] = col[u] >= 0 ? hmap[col[u]] : -1;
#pragma unroll
      for (int u = 0; u < kGroups; ++u)
        if (code[u] >= 0) atomicAdd(&acc[code[u] >> 1], (code[u] & 1) ? -val[u] : val[u]);
    }
    if (lane == 0) {
      const int cj = hmap[j];
      if (cj >= 0) atomicAdd(&acc[cj >> 1], (cj & 1) ? -lam : lam);
    }
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    OutT* out = out_base + j * ldas;
    for (int c = lane; c < tau; c += 64) out[c] = (OutT)acc[c];
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
  }
}

// Rows of AS for one sketch and one chunk of kLdsRows rows per workgroup, with the sketch's
// bucket map staged in LDS as 16-bit codes: the bucket lookups of the scatter-add become LDS
// reads instead of vector-memory gathers. Workgroups are dealt to the 8 XCDs in turn, so the
// block index is mapped so that each XCD takes whole row chunks, every sketch of a chunk
// before the next chunk: the chunk's rows of A0 are read into that XCD's L2 once and stay
// there while its sketches pass.
template <typename OutT>
__global__ __launch_bounds__(512) void k_as_arows_lds(const int64_t* __restrict__ a_ptr,
                                                      const int32_t* __restrict__ a_col,
                                                      const double* __restrict__ a_val, int64_t m,
                                                      int32_t tau, int64_t ldas, double lam,
                                                      const int32_t* __restrict__ hmap_all,
                                                      OutT* __restrict__ AS, int32_t nslots,
                                                      int64_t nchunks, const int32_t* __restrict__ done) {
  extern __shared__ __align__(16) unsigned char lds_raw[];
  int16_t* hm = reinterpret_cast<int16_t*>(lds_raw);                            // [m]
  double* acc_all = reinterpret_cast<double*>(lds_raw + ((2 * m + 15) & ~15ll));  // [8][tau]
  if (*done) return;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t xcd = blockIdx.x & 7, i = blockIdx.x >> 3;
  const int64_t chunk = 8 * (i / nslots) + xcd, slot = i % nslots;
  if (chunk >= nchunks) return;  // the last round of chunks does not cover every XCD
  const int32_t* hmap = hmap_all + slot * m;
  // 8 loads in flight per thread while the map is staged
  for (int64_t jb = tid; jb < m; jb += 512 * 8) {
    int32_t v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int64_t j = jb + u * 512;
      v[u] = j < m ? hmap[j] : 0;
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int64_t j = jb + u * 512;
      if (j < m) hm[j] = (int16_t)v[u];
    }
  }
  __syncthreads();
  double* acc = acc_all + (int64_t)wave * tau;
  OutT* out_base = AS + slot * m * ldas;
  const int64_t j0 = chunk * kLdsRows;
  const int64_t j1 = min(m, j0 + kLdsRows);
  for (int64_t j = j0 + wave; j < j1; j += 8) {
    for (int c = lane; c < tau; c += 64) acc[c] = 0.0;
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    const int64_t p0 = a_ptr[j], p1 = a_ptr[j + 1];
    for (int64_t pb = p0; pb < p1; pb += 64 * kLdsGroups) {
      int32_t col[kLdsGroups];
      double val[kLdsGroups];
#pragma unroll
      for (int u = 0; u < kLdsGroups; ++u) {
        const int64_t p = pb + u * 64 + lane;
        col[u] = p < p1 ? a_col[p] : -1;
        val[u] = p < p1 ? a_val[p] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < kLdsGroups; ++u) {
        const int code = col[u] >= 0 ? (int)hm[col[u]] : -1;
        if (code >= 0) atomicAdd(&acc[code >> 1], (code & 1) ? -val[u] : val[u]);
      }
    }
    if (lane == 0) {
      const int cj = hm[j];
      if (cj >= 0) atomicAdd(&acc[cj >> 1], (cj & 1) ? -lam : lam);
    }
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    OutT* out = out_base + j * ldas;
    for (int c = lane; c < tau; c += 64) out[c] = (OutT)acc[c];
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
  }
}

// As k_as_arows_lds for a bucket map too large for 16-bit codes in LDS: the codes are packed
// three to a 32-bit word, and 4 waves share a workgroup (one AS row each at a time).
template <typename OutT>
__global__ __launch_bounds__(64 * kPackedWaves) void k_as_arows_packed(const int64_t* __restrict__ a_ptr,
                                                                      const int32_t* __restrict__ a_col,
                                                                      const double* __restrict__ a_val, int64_t m,
                                                                      int32_t tau, int64_t ldas, double lam,
                                                                      const int32_t* __restrict__ hmap_all,
                                                                      OutT* __restrict__ AS, int32_t nslots,
                                                                      int64_t nchunks, const int32_t* __restrict__ done) {
  extern __shared__ __align__(16) unsigned char lds_raw[];
  const int64_t nwords = (m + 2) / 3;
  uint32_t* pm = reinterpret_cast<uint32_t*>(lds_raw);                                      // [nwords]
  double* acc_all = reinterpret_cast<double*>(lds_raw + ((nwords * 4 + 15) & ~15ll));     // [waves][tau]
  if (*done) return;
  constexpr int kT = 64 * kPackedWaves;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t xcd = blockIdx.x & 7, bi = blockIdx.x >> 3;
  const int64_t chunk = 8 * (bi / nslots) + xcd, slot = bi % nslots;
  if (chunk >= nchunks) return;
  const int32_t* hmap = hmap_all + slot * m;
  for (int64_t w = tid; w < nwords; w += kT) {
    uint32_t word = 0;
#pragma unroll
    for (int u = 0; u < 3; ++u) {
      const int64_t jj = 3 * w + u;
      const int32_t code = jj < m ? hmap[jj] : -1;
      word |= (code >= 0 ? (uint32_t)code : kNoCode) << (10 * u);
    }
    pm[w] = word;
  }
  __syncthreads();
  double* acc = acc_all + (int64_t)wave * tau;
  OutT* out_base = AS + slot * m * ldas;
  const int64_t j0 = chunk * kLdsRows;
  const int64_t j1 = min(m, j0 + kLdsRows);
  auto code_of = [&](int64_t col) -> int {
    const uint32_t q = (uint32_t)col / 3u, r = (uint32_t)col - 3u * q;
    const uint32_t c = (pm[q] >> (10u * r)) & kNoCode;
    return c == kNoCode ? -1 : (int)c;
  };
  for (int64_t j = j0 + wave; j < j1; j += kPackedWaves) {
    for (int c = lane; c < tau; c += 64) acc[c] = 0.0;
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    const int64_t p0 = a_ptr[j], p1 = a_ptr[j + 1];
    for (int64_t pb = p0; pb < p1; pb += 64 * kLdsGroups) {
      int32_t col[kLdsGroups];
      double val[kLdsGroups];
#pragma unroll
      for (int u = 0; u < kLdsGroups; ++u) {
        const int64_t p = pb + u * 64 + lane;
        col[u] = p < p1 ? a_col[p] : -1;
        val[u] = p < p1 ? a_val[p] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < kLdsGroups; ++u) {
        const int code = col[u] >= 0 ? code_of(col[u]) : -1;
        if (code >= 0) atomicAdd(&acc[code >> 1], (code & 1) ? -val[u] : val[u]);
      }
    }
    if (lane == 0) {
      const int cj = code_of(j);
      if (cj >= 0) atomicAdd(&acc[cj >> 1], (cj & 1) ? -lam : lam);
    }
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    OutT* out = out_base + j * ldas;
    for (int c = lane; c < tau; c += 64) out[c] = (OutT)acc[c];
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
  }
}

// G[slot][b][c] = sum over the members j of bucket b (in member order) of s_j AS[j][c], in FP64
// (AS stored as InT: FP64, or FP32 in mixed precision).
template <typename InT>
__global__ __launch_bounds__(256) void k_g_from_as(const InT* __restrict__ AS_all, int64_t m,
                                                   int32_t tau, int64_t ldas,
                                                   const int32_t* __restrict__ hmap_all,
                                                   const int32_t* __restrict__ members_all,
                                                   const int32_t* __restrict__ offs_all, int64_t nsel,
                                                   double* __restrict__ G_all, int64_t ldg,
                                                   const int32_t* __restrict__ done) {
  if (*done) return;
  const int b = blockIdx.x;
  const int64_t slot = blockIdx.y;
  const InT* AS = AS_all + slot * m * ldas;
  const int32_t* hmap = hmap_all + slot * m;
  const int32_t* members = members_all + slot * nsel;
  const int32_t* offs = offs_all + slot * (tau + 1);
  double* grow = G_all + (slot * ldg + b) * ldg;
  const int p0 = offs[b], p1 = offs[b + 1];
  for (int c = threadIdx.x; c < tau; c += blockDim.x) {
    double s = 0.0;
#pragma unroll 4
    for (int p = p0; p < p1; ++p) {
      const int64_t j = members[p];
      const double v = (double)AS[j * ldas + c];
      s += (hmap[j] & 1) ? -v : v;
    }
    grow[c] = s;
  }
}

template <typename V>
hipError_t zzt_impl(const int64_t* zt_ptr, const int32_t* zt_col, const V* zt_val, int64_t K, int64_t m,
                    int64_t npairs, int64_t** a_ptr, int32_t** a_col, double** a_val, int64_t* a_nnz,
                    hipStream_t s) {
  int64_t *cnt = nullptr, *off = nullptr, *d_runs = nullptr;
  uint64_t *kin = nullptr, *kout = nullptr, *ukeys = nullptr;
  double *vin = nullptr, *vout = nullptr, *agg = nullptr;
  void* tmp = nullptr;
  size_t tb = 0, tb2 = 0, tb3 = 0;
  const int n = (int)npairs;
  int end_bit = 33;
  while (end_bit < 64 && ((uint64_t)1 << (end_bit - 32)) <= (uint64_t)m) ++end_bit;
  hipError_t e = hipMalloc(&cnt, sizeof(int64_t) * (K + 1));
  if (e == hipSuccess) e = hipMalloc(&off, sizeof(int64_t) * (K + 1));
  if (e == hipSuccess) e = hipMalloc(&kin, sizeof(uint64_t) * npairs);
  if (e == hipSuccess) e = hipMalloc(&kout, sizeof(uint64_t) * npairs);
  if (e == hipSuccess) e = hipMalloc(&vin, sizeof(double) * npairs);
  if (e == hipSuccess) e = hipMalloc(&vout, sizeof(double) * npairs);
  if (e == hipSuccess) e = hipMalloc(&d_runs, sizeof(int64_t));
  if (e == hipSuccess) e = hipcub::DeviceScan::ExclusiveSum(nullptr, tb, cnt, off, (int)K, s);
  if (e == hipSuccess)
    e = hipcub::DeviceRadixSort::SortPairs(nullptr, tb2, kin, kout, vin, vout, n, 0, end_bit, s);
  if (e == hipSuccess)
    e = hipcub::DeviceReduce::ReduceByKey(nullptr, tb3, kout, kin, vout, vin, d_runs, hipcub::Sum(), n, s);
  if (e == hipSuccess) e = hipMalloc(&tmp, std::max(tb, std::max(tb2, tb3)));
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k_pair_counts, dim3((unsigned)((K + 255) / 256)), dim3(256), 0, s, zt_ptr, K, cnt);
    size_t t = tb;
    e = hipcub::DeviceScan::ExclusiveSum(tmp, t, cnt, off, (int)K, s);
  }
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k_pair_emit<V>, dim3((unsigned)((K + 3) / 4)), dim3(256), 0, s, zt_ptr, zt_col, zt_val,
                       K, off, kin, vin);
    size_t t = tb2;
    e = hipcub::DeviceRadixSort::SortPairs(tmp, t, kin, kout, vin, vout, n, 0, end_bit, s);
  }
  // unique keys into kin, their sums into vin (reusing the input buffers)
  if (e == hipSuccess) {
    size_t t = tb3;
    e = hipcub::DeviceReduce::ReduceByKey(tmp, t, kout, kin, vout, vin, d_runs, hipcub::Sum(), n, s);
  }
  int64_t nu = 0;
  if (e == hipSuccess) e = hipMemcpyAsync(&nu, d_runs, sizeof(int64_t), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e == hipSuccess) e = hipMalloc(a_ptr, sizeof(int64_t) * (m + 1));
  if (e == hipSuccess) e = hipMalloc(a_col, sizeof(int32_t) * std::max<int64_t>(1, nu));
  if (e == hipSuccess) e = hipMalloc(a_val, sizeof(double) * std::max<int64_t>(1, nu));
  if (e == hipSuccess) {
    const int64_t nt = std::max(nu, m + 1);
    hipLaunchKernelGGL(k_a_structure, dim3((unsigned)((nt + 255) / 256)), dim3(256), 0, s, kin, nu, m,
                       *a_ptr, *a_col);
    e = hipGetLastError();
  }
  if (e == hipSuccess && nu) e = hipMemcpyAsync(*a_val, vin, sizeof(double) * nu, hipMemcpyDeviceToDevice, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  *a_nnz = nu;
  for (void* p : {(void*)cnt, (void*)off, (void*)kin, (void*)kout, (void*)vin, (void*)vout, (void*)d_runs,
                  (void*)ukeys, (void*)agg, tmp})
    if (p) (void)hipFree(p);
  return e;
}

template <int W, typename OutT>
hipError_t arows_launch(const int64_t* a_ptr, const int32_t* a_col, const double* a_val, int64_t m,
                        int32_t tau, int64_t ldas, int32_t nslots, double lam, const int32_t* hmap,
                        OutT* AS, const int32_t* done, hipStream_t s) {
  const size_t bytes = sizeof(double) * W * (size_t)tau;
  hipError_t e = hipFuncSetAttribute((const void*)k_as_arows<W, OutT>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)bytes);
  if (e != hipSuccess) return e;
  const int rows = 16;
  const dim3 grid((unsigned)((m + rows - 1) / rows), (unsigned)((nslots + W - 1) / W));
  hipLaunchKernelGGL((k_as_arows<W, OutT>), grid, dim3(W * 64), bytes, s, a_ptr, a_col, a_val, m, tau, ldas,
                     nslots, lam, hmap, AS, rows, done);
  return hipGetLastError();
}

template <typename OutT>
hipError_t as_arows_impl(const int64_t* a_ptr, const int32_t* a_col, const double* a_val, int64_t m,
                         int32_t tau, int64_t ldas, int32_t nslots, double lam, const int32_t* hmap, OutT* AS,
                         const int32_t* done, hipStream_t s) {
  hipError_t e;
  const size_t lds = arows_lds_bytes(m, tau);
  if (tau < 16383 && lds <= 96 * 1024) {
    // bucket map in LDS (16-bit codes): one sketch per workgroup
    e = hipFuncSetAttribute((const void*)k_as_arows_lds<OutT>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)lds);
    if (e != hipSuccess) return e;
    const int64_t nchunks = (m + kLdsRows - 1) / kLdsRows;
    const int64_t nblocks = 8 * (int64_t)nslots * ((nchunks + 7) / 8);
    if (nblocks > (int64_t)INT32_MAX) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_as_arows_lds<OutT>, dim3((unsigned)nblocks), dim3(512), lds, s, a_ptr, a_col, a_val, m,
                       tau, ldas, lam, hmap, AS, nslots, nchunks, done);
    e = hipGetLastError();
  } else if (tau <= 511 && arows_packed_lds_bytes(m, tau) <= 156 * 1024) {
    // packed map in LDS: one workgroup of 4 waves per CU
    const size_t plds = arows_packed_lds_bytes(m, tau);
    e = hipFuncSetAttribute((const void*)k_as_arows_packed<OutT>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)plds);
    if (e != hipSuccess) return e;
    const int64_t nchunks = (m + kLdsRows - 1) / kLdsRows;
    const int64_t nblocks = 8 * (int64_t)nslots * ((nchunks + 7) / 8);
    if (nblocks > (int64_t)INT32_MAX) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_as_arows_packed<OutT>, dim3((unsigned)nblocks), dim3(64 * kPackedWaves), plds, s, a_ptr,
                       a_col, a_val, m, tau, ldas, lam, hmap, AS, nslots, nchunks, done);
    e = hipGetLastError();
  } else if (tau <= 1024)
    e = arows_launch<16, OutT>(a_ptr, a_col, a_val, m, tau, ldas, nslots, lam, hmap, AS, done, s);
  else if (tau <= 2048)
    e = arows_launch<8, OutT>(a_ptr, a_col, a_val, m, tau, ldas, nslots, lam, hmap, AS, done, s);
  else
    return hipErrorInvalidValue;
  return e;
}

}  // namespace

int64_t zzt_pairs(const int64_t* zt_ptr_host, int64_t K) {
  int64_t p = 0;
  for (int64_t i = 0; i < K; ++i) {
    const int64_t L = zt_ptr_host[i + 1] - zt_ptr_host[i];
    p += L * L;
  }
  return p;
}

hipError_t build_zzt(const int64_t* zt_ptr, const int32_t* zt_col, const void* zt_val, int32_t vals_f32,
                     int64_t K, int64_t m, int64_t npairs, int64_t** a_ptr, int32_t** a_col, double** a_val,
                     int64_t* a_nnz, hipStream_t s) {
  if (npairs <= 0 || npairs >= (int64_t)INT32_MAX) return hipErrorInvalidValue;
  if (vals_f32)
    return zzt_impl<float>(zt_ptr, zt_col, (const float*)zt_val, K, m, npairs, a_ptr, a_col, a_val, a_nnz, s);
  return zzt_impl<double>(zt_ptr, zt_col, (const double*)zt_val, K, m, npairs, a_ptr, a_col, a_val, a_nnz, s);
}

hipError_t launch_as_arows(const int64_t* a_ptr, const int32_t* a_col, const double* a_val, int64_t m,
                           int32_t tau, int64_t ldas, int32_t nslots, double lam, const int32_t* hmap, void* AS,
                           int32_t as_f32, const int32_t* done, hipStream_t s) {
  if (as_f32)
    return as_arows_impl<float>(a_ptr, a_col, a_val, m, tau, ldas, nslots, lam, hmap, (float*)AS, done, s);
  return as_arows_impl<double>(a_ptr, a_col, a_val, m, tau, ldas, nslots, lam, hmap, (double*)AS, done, s);
}

hipError_t launch_g_from_as(const void* AS, int32_t as_f32, int64_t m, int32_t tau, int64_t ldas, int32_t nslots,
                            const int32_t* hmap, const int32_t* members, const int32_t* offs, int64_t nsel,
                            double* G, int64_t ldg, const int32_t* done, hipStream_t s) {
  if (as_f32)
    hipLaunchKernelGGL(k_g_from_as<float>, dim3(tau, nslots), dim3(256), 0, s, (const float*)AS, m, tau, ldas, hmap,
                       members, offs, nsel, G, ldg, done);
  else
    hipLaunchKernelGGL(k_g_from_as<double>, dim3(tau, nslots), dim3(256), 0, s, (const double*)AS, m, tau, ldas,
                       hmap, members, offs, nsel, G, ldg, done);
  return hipGetLastError();
}

}  // namespace rs
