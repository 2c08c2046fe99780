// Sketch draws S_k ~ D on the device (Sec. 4): one workgroup per lookahead slot.
//
// Subsample (Def. 4.2): the tau coordinates with the smallest Philox words (W0_i, i)
//   form C; every tau-subset is equally likely (eq:subsample). Found by a radix select
//   over 12-bit digits of W0 followed by an LDS bitonic sort of the boundary digit.
// SubCount (Def. 4.3): the s = k tau smallest (W0_i, i) taken in ascending key order
//   (a uniformly random order); rank p goes to bucket floor(p / k) with the sign of
//   W1_i, so Sigma sums k contiguous rows (eq:Sigmacount).
// Count (Sec. 4.2): bucket h(i) = hi32(W0_i) * tau >> 32, sign from W1_i; the members
//   of each bucket are ordered by coordinate index with a deterministic counting sort.
#include "dev_common.h"
#include "rs_internal.h"

namespace rs {
namespace {

constexpr int kSelThreads = 1024;
constexpr int kBins = 4096;
constexpr int kCandCap = 4096;

struct SelHeader {
  int hist[kBins];
  int scan[32];
  int bin, before, ncand, pad;
};

__device__ __forceinline__ int next_pow2(int v) {
  int p = 1;
  while (p < v) p <<= 1;
  return p;
}

__device__ void bitonic_sort(uint64_t* key, uint32_t* idx, int n) {
  for (int k = 2; k <= n; k <<= 1) {
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int i = threadIdx.x; i < n; i += blockDim.x) {
        const int ixj = i ^ j;
        if (ixj > i) {
          const uint64_t ka = key[i], kb = key[ixj];
          const uint32_t ia = idx[i], ib = idx[ixj];
          const bool a_gt_b = (ka > kb) || (ka == kb && ia > ib);
          const bool ascending = (i & k) == 0;
          if (a_gt_b == ascending) {
            key[i] = kb;
            key[ixj] = ka;
            idx[i] = ib;
            idx[ixj] = ia;
          }
        }
      }
      __syncthreads();
    }
  }
}

// Bin holding the need-th smallest element (1-based) of a histogram of nbins <= 4096 bins.
__device__ void find_bin(SelHeader* H, int nbins, int need) {
  const int base = threadIdx.x * 4;
  int c[4], sum = 0;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    c[q] = (base + q < nbins) ? H->hist[base + q] : 0;
    sum += c[q];
  }
  int total;
  const int excl = block_exclusive_scan(sum, H->scan, &total);
  if (excl < need && need <= excl + sum) {
    int run = excl;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      if (run < need && need <= run + c[q]) {
        H->bin = base + q;
        H->before = run;
      }
      run += c[q];
    }
  }
  __syncthreads();
}

__device__ __forceinline__ void select_body(const SketchArgs& a, int slot, unsigned char* lds_raw) {
  SelHeader* H = reinterpret_cast<SelHeader*>(lds_raw);
  const int sort_cap = (a.kind == kSubcount) ? max(kCandCap, next_pow2((int)a.nsel)) : kCandCap;
  uint64_t* skey = reinterpret_cast<uint64_t*>(lds_raw + sizeof(SelHeader));
  uint32_t* sidx = reinterpret_cast<uint32_t*>(skey + sort_cap);

  if (*a.done) return;
  const int tid = threadIdx.x;
  const int64_t m = a.m;
  const uint64_t k = (uint64_t)((a.kdev ? *a.kdev : a.k0) + slot);
  const uint64_t tag = (a.kind == kSubcount) ? kTagSubcount : (a.kind == kSrht ? kTagSrht : kTagSubsample);
  const bool weighted = a.kind == kWeighted;
  const bool q_ok = weighted && a.q_ok && *a.q_ok != 0;
  uint64_t* keys = a.keys + (int64_t)slot * m;
  int32_t* hmap = a.hmap + (int64_t)slot * m;
  int32_t* members = a.members + (int64_t)slot * a.nsel;
  int32_t* offs = a.offs + (int64_t)slot * (a.tau + 1);
  const int want = (int)a.nsel;  // tau for subsample, k * tau for SubCount

  for (int i = tid; i < kBins; i += kSelThreads) H->hist[i] = 0;
  if (tid == 0) H->ncand = 0;
  __syncthreads();
  for (int64_t j = tid; j < m; j += kSelThreads) {
    uint64_t key;
    if (weighted) {
      // u_j in (0, 1), exact in FP64; key_j = u_j / q_j (IEEE division). A positive
      // double's bit pattern orders like its value, so the same 64-bit selection applies.
      // Without a usable proposal the keys are u_j themselves: a uniform tau-subset.
      const Philox4 r = philox4x64_10((uint64_t)j, k, kTagWeighted, 0, a.seed, a.pid);
      const double u = ((double)(r.v0 >> 12) + 0.5) * 0x1p-52;
      const double kv = q_ok ? u / (double)a.q[j] : u;
      key = (uint64_t)__double_as_longlong(kv);
    } else {
      key = philox4x64_10((uint64_t)j, k, tag, 0, a.seed, a.pid).v0;
    }
    keys[j] = key;
    hmap[j] = -1;
    atomicAdd(&H->hist[key >> 52], 1);
  }
  __syncthreads();

  // Radix select: narrow the digit containing the want-th smallest key. With few coordinates
  // another pass over the keys costs less than sorting a crowded digit (keys u_j / q_j of a
  // weighted draw share a binary exponent in large groups), so the narrowing goes on until at
  // most 64 candidates are left; with many, it stops at the sort's capacity.
  const int sort_max = m <= 16 * kSelThreads ? 64 : kCandCap;
  int need = want;
  uint64_t prefix = 0;  // value of (key >> shift) shared by the candidates
  int shift = 52, width = 12;
  for (;;) {
    find_bin(H, 1 << width, need);
    const int bin = H->bin;
    need -= H->before;
    prefix = (prefix << width) | (uint64_t)bin;
    const int binc = H->hist[bin];
    __syncthreads();
    if (binc <= sort_max || shift == 0) break;
    const int nshift = shift >= 12 ? shift - 12 : 0;
    width = shift - nshift;
    for (int i = tid; i < kBins; i += kSelThreads) H->hist[i] = 0;
    __syncthreads();
    const uint64_t mask = (1ull << width) - 1ull;
    for (int64_t j = tid; j < m; j += kSelThreads) {
      const uint64_t key = keys[j];
      if ((key >> shift) == prefix) atomicAdd(&H->hist[(key >> nshift) & mask], 1);
    }
    shift = nshift;
    __syncthreads();
  }

  // Gather the boundary digit and sort it on (key, index).
  for (int64_t j = tid; j < m; j += kSelThreads) {
    const uint64_t key = keys[j];
    if ((key >> shift) == prefix) {
      const int p = atomicAdd(&H->ncand, 1);
      if (p < kCandCap) {
        skey[p] = key;
        sidx[p] = (uint32_t)j;
      }
    }
  }
  __syncthreads();
  int ncand = H->ncand;
  if (ncand > kCandCap) {  // more than kCandCap equal 64-bit keys: not expected for Philox output
    if (tid == 0) atomicCAS(a.err, 0, 1);
    ncand = kCandCap;
  }
  const int nsort = next_pow2(ncand);
  for (int i = ncand + tid; i < nsort; i += kSelThreads) {
    skey[i] = ~0ull;
    sidx[i] = ~0u;
  }
  __syncthreads();
  bitonic_sort(skey, sidx, nsort);
  need = min(need, ncand);
  const uint64_t thr_key = skey[need - 1];
  const uint32_t thr_idx = sidx[need - 1];
  __syncthreads();

  if (a.kind != kSubcount) {
    // Subsample: compact the selected coordinates in ascending index order.
    const int64_t chunk = (m + kSelThreads - 1) / kSelThreads;
    const int64_t j0 = (int64_t)tid * chunk, j1 = min(m, j0 + chunk);
    int cnt = 0;
    for (int64_t j = j0; j < j1; ++j) {
      const uint64_t key = keys[j];
      cnt += (key < thr_key || (key == thr_key && (uint32_t)j <= thr_idx)) ? 1 : 0;
    }
    int total;
    int pos = block_exclusive_scan(cnt, H->scan, &total);
    if (tid == 0 && total != want) atomicCAS(a.err, 0, 2);
    for (int64_t j = j0; j < j1; ++j) {
      const uint64_t key = keys[j];
      if (key < thr_key || (key == thr_key && (uint32_t)j <= thr_idx)) {
        if (pos < want) {
          members[pos] = (int32_t)j;
          hmap[j] = 2 * pos;
        }
        ++pos;
      }
    }
    for (int c = tid; c <= a.tau; c += kSelThreads) offs[c] = c;
    return;
  }

  // SubCount: order the kept coordinates by (key, index); rank p -> bucket p / k.
  if (tid == 0) H->ncand = 0;
  __syncthreads();
  for (int64_t j = tid; j < m; j += kSelThreads) {
    const uint64_t key = keys[j];
    if (key < thr_key || (key == thr_key && (uint32_t)j <= thr_idx)) {
      const int p = atomicAdd(&H->ncand, 1);
      if (p < sort_cap) {
        skey[p] = key;
        sidx[p] = (uint32_t)j;
      }
    }
  }
  __syncthreads();
  const int nkept = min(H->ncand, sort_cap);
  if (tid == 0 && H->ncand != want) atomicCAS(a.err, 0, 3);
  const int nsort2 = next_pow2(nkept);
  for (int i = nkept + tid; i < nsort2; i += kSelThreads) {
    skey[i] = ~0ull;
    sidx[i] = ~0u;
  }
  __syncthreads();
  bitonic_sort(skey, sidx, nsort2);
  for (int p = tid; p < min(nkept, want); p += kSelThreads) {
    const uint32_t j = sidx[p];
    const Philox4 r = philox4x64_10((uint64_t)j, k, tag, 0, a.seed, a.pid);
    const int neg = (int)(r.v1 & 1ull);
    const int bucket = p / a.sub_k;
    members[p] = (int32_t)j;
    hmap[j] = 2 * bucket + neg;
  }
  for (int b = tid; b <= a.tau; b += kSelThreads) offs[b] = b * a.sub_k;
}

// Count sketch: 16 waves; wave w owns a contiguous coordinate segment. Placement is
// stable in the coordinate index, so the member order is deterministic.
__device__ __forceinline__ void count_body(const SketchArgs& a, int slot, int* cnt_lds) {
  int* cntw = cnt_lds;               // [16][tau]
  int* scan = cnt_lds + 16 * a.tau;  // 32 ints
  if (*a.done) return;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t m = a.m;
  const int tau = a.tau;
  const uint64_t k = (uint64_t)((a.kdev ? *a.kdev : a.k0) + slot);
  int32_t* hmap = a.hmap + (int64_t)slot * m;
  int32_t* members = a.members + (int64_t)slot * a.nsel;
  int32_t* offs = a.offs + (int64_t)slot * (tau + 1);
  const int64_t seg = (m + 15) / 16;
  const int64_t jb = min(m, (int64_t)wave * seg), je = min(m, jb + seg);

  for (int i = tid; i < 16 * tau; i += kSelThreads) cntw[i] = 0;
  __syncthreads();
  for (int64_t j = jb + lane; j < je; j += 64) {
    const Philox4 r = philox4x64_10((uint64_t)j, k, kTagCount, 0, a.seed, a.pid);
    const int h = (int)(((r.v0 >> 32) * (uint64_t)tau) >> 32);
    hmap[j] = 2 * h + (int)(r.v1 & 1ull);
    atomicAdd(&cntw[wave * tau + h], 1);
  }
  __syncthreads();

  // Bucket offsets, and per-wave starting cursors inside each bucket.
  const int per = (tau + kSelThreads - 1) / kSelThreads;
  const int b0 = min(tau, tid * per), b1 = min(tau, b0 + per);
  int local = 0;
  for (int b = b0; b < b1; ++b)
    for (int w = 0; w < 16; ++w) local += cntw[w * tau + b];
  int total;
  int run = block_exclusive_scan(local, scan, &total);
  for (int b = b0; b < b1; ++b) {
    offs[b] = run;
    for (int w = 0; w < 16; ++w) {
      const int c = cntw[w * tau + b];
      cntw[w * tau + b] = run;
      run += c;
    }
  }
  if (tid == 0) offs[tau] = (int)m;
  __syncthreads();

  // Stable placement: groups of 64 consecutive coordinates, peers found by ballot.
  const int64_t ngroups = (je - jb + 63) / 64;
  for (int64_t g = 0; g < ngroups; ++g) {
    const int64_t j = jb + g * 64 + lane;
    const bool valid = j < je;
    const int h = valid ? (hmap[j] >> 1) : -1;
    unsigned long long pending = __ballot(valid);
    unsigned long long peers = 0;
    while (pending) {
      const int leader = __ffsll((long long)pending) - 1;
      const int hl = __shfl(h, leader, 64);
      const unsigned long long eq = __ballot(valid && h == hl);
      if (valid && h == hl) peers = eq;
      pending &= ~eq;
    }
    int base = 0;
    if (valid) {
      const int rank = __popcll(peers & ((1ull << lane) - 1ull));
      base = cntw[wave * tau + h];
      members[base + rank] = (int32_t)j;
    }
    __builtin_amdgcn_wave_barrier();
    if (valid && lane == __ffsll((long long)peers) - 1) cntw[wave * tau + h] = base + __popcll(peers);
    __builtin_amdgcn_wave_barrier();
  }
}


__global__ __launch_bounds__(kSelThreads) void k_sketch_select(SketchArgs a) {
  extern __shared__ __align__(16) unsigned char lds_raw[];
  select_body(a, blockIdx.x, lds_raw);
}

__global__ __launch_bounds__(kSelThreads) void k_sketch_count(SketchArgs a) {
  extern __shared__ __align__(16) int cnt_lds[];
  count_body(a, blockIdx.x, cnt_lds);
}

// Grouped forms: blockIdx.y picks one problem's arguments from a device table.
__global__ __launch_bounds__(kSelThreads) void k_sketch_select_tab(const SketchArgs* __restrict__ tab) {
  extern __shared__ __align__(16) unsigned char lds_raw[];
  const SketchArgs a = tab[blockIdx.y];
  select_body(a, blockIdx.x, lds_raw);
}

__global__ __launch_bounds__(kSelThreads) void k_sketch_count_tab(const SketchArgs* __restrict__ tab) {
  extern __shared__ __align__(16) int cnt_lds[];
  const SketchArgs a = tab[blockIdx.y];
  count_body(a, blockIdx.x, cnt_lds);
}

}  // namespace

hipError_t launch_sketch(const SketchArgs& a, hipStream_t s) {
  if (a.nslots <= 0) return hipSuccess;
  if (a.kind == kCount) {
    const size_t bytes = sizeof(int) * (16 * (size_t)a.tau + 32);
    hipError_t e = hipFuncSetAttribute((const void*)k_sketch_count,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_sketch_count, dim3(a.nslots), dim3(kSelThreads), bytes, s, a);
    return hipGetLastError();
  }
  int cap = kCandCap;
  if (a.kind == kSubcount) {
    int p = 1;
    while (p < a.nsel) p <<= 1;
    cap = p > cap ? p : cap;
  }
  const size_t bytes = sizeof(SelHeader) + (size_t)cap * (sizeof(uint64_t) + sizeof(uint32_t));
  hipError_t e = hipFuncSetAttribute((const void*)k_sketch_select,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_sketch_select, dim3(a.nslots), dim3(kSelThreads), bytes, s, a);
  return hipGetLastError();
}

}  // namespace rs

namespace rs {

size_t sketch_lds_bytes(int32_t kind, int32_t tau, int64_t nsel) {
  if (kind == kCount) return sizeof(int) * (16 * (size_t)tau + 32);
  int cap = kCandCap;
  if (kind == kSubcount) {
    int p = 1;
    while (p < nsel) p <<= 1;
    cap = p > cap ? p : cap;
  }
  return sizeof(SelHeader) + (size_t)cap * (sizeof(uint64_t) + sizeof(uint32_t));
}

hipError_t launch_sketch_tab(const SketchArgs* tab, int32_t count, int32_t kind, size_t lds_bytes,
                             hipStream_t s) {
  if (count <= 0) return hipSuccess;
  const void* fn = kind == kCount ? (const void*)k_sketch_count_tab : (const void*)k_sketch_select_tab;
  hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_bytes);
  if (e != hipSuccess) return e;
  if (kind == kCount)
    hipLaunchKernelGGL(k_sketch_count_tab, dim3(1, count), dim3(kSelThreads), lds_bytes, s, tab);
  else
    hipLaunchKernelGGL(k_sketch_select_tab, dim3(1, count), dim3(kSelThreads), lds_bytes, s, tab);
  return hipGetLastError();
}

}  // namespace rs
