// Device helpers: Philox4x64-10 and wavefront / workgroup reductions (CDNA, wave64).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace rs {

// Philox4x64-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of
//   (c0, c1, c2, c3) <- (hi(M1 c2) ^ c1 ^ k0, lo(M1 c2), hi(M0 c0) ^ c3 ^ k1, lo(M0 c0))
// with the key advanced by the Weyl increments between rounds.
struct Philox4 {
  uint64_t v0, v1, v2, v3;
};

__device__ __forceinline__ Philox4 philox4x64_10(uint64_t c0, uint64_t c1, uint64_t c2, uint64_t c3,
                                                uint64_t k0, uint64_t k1) {
  constexpr uint64_t kMulA = 0xD2E7470EE14C6C93ull;
  constexpr uint64_t kMulB = 0xCA5A826395121157ull;
  constexpr uint64_t kWeylA = 0x9E3779B97F4A7C15ull;
  constexpr uint64_t kWeylB = 0xBB67AE8584CAA73Bull;
#pragma unroll
  for (int round = 0; round < 10; ++round) {
    if (round > 0) {
      k0 += kWeylA;
      k1 += kWeylB;
    }
    const uint64_t hiA = __umul64hi(kMulA, c0), loA = kMulA * c0;
    const uint64_t hiB = __umul64hi(kMulB, c2), loB = kMulB * c2;
    const uint64_t n0 = hiB ^ c1 ^ k0;
    const uint64_t n2 = hiA ^ c3 ^ k1;
    c0 = n0;
    c1 = loB;
    c2 = n2;
    c3 = loA;
  }
  return Philox4{c0, c1, c2, c3};
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

__device__ __forceinline__ int wave_sum_int(int v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Inclusive prefix sum across the 64 lanes of a wave.
__device__ __forceinline__ int wave_inclusive_scan(int v) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    int t = __shfl_up(v, off, 64);
    if (lane >= off) v += t;
  }
  return v;
}

// Exclusive prefix sum over all threads of a workgroup (blockDim.x a multiple of 64,
// at most 1024). `scratch` holds >= 17 ints of LDS. Returns the exclusive prefix and
// writes the total to *total (all threads).
__device__ __forceinline__ int block_exclusive_scan(int v, int* scratch, int* total) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nwaves = blockDim.x >> 6;
  int inc = wave_inclusive_scan(v);
  if (lane == 63) scratch[wave] = inc;
  __syncthreads();
  if (threadIdx.x == 0) {
    int run = 0;
    for (int w = 0; w < nwaves; ++w) {
      int t = scratch[w];
      scratch[w] = run;
      run += t;
    }
    scratch[16] = run;
  }
  __syncthreads();
  int excl = scratch[wave] + inc - v;
  *total = scratch[16];
  __syncthreads();
  return excl;
}

// Deterministic workgroup sum (fixed reduction tree). `scratch` holds >= 16 doubles.
__device__ __forceinline__ double block_sum(double v, double* scratch) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nwaves = blockDim.x >> 6;
  v = wave_sum(v);
  if (lane == 0) scratch[wave] = v;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0) {
    for (int w = 0; w < nwaves; ++w) t += scratch[w];
    scratch[0] = t;
  }
  __syncthreads();
  t = scratch[0];
  __syncthreads();
  return t;
}

}  // namespace rs
