// The weighted subsample draw (the sketch a coordinate proposal feeds, any distribution D
// of Sec. 3) into caller buffers with no allocation: the selection's working memory is a
// fixed device array of this file instead of buffers allocated per call.
//
// The array lives once per device for the life of the process. Host code never passes
// its name to a kernel (there it is only a host-side stand-in): the device address is
// looked up with hipGetSymbolAddress once per device and kept in g_scratch_ptr.
#include <hip/hip_runtime.h>

#include <cmath>
#include <mutex>

#include "rs_internal.h"

using namespace rs;

namespace {

constexpr int64_t kNoAllocMaxM = int64_t(1) << 20;  // largest m accepted
// Layout of the array (bytes): selection keys, coordinate map, bucket offsets, flags.
constexpr size_t kOffKeys = 0;                                        // uint64 [max m]
constexpr size_t kOffHmap = kOffKeys + sizeof(uint64_t) * kNoAllocMaxM;  // int32 [max m]
constexpr size_t kOffOffs = kOffHmap + sizeof(int32_t) * kNoAllocMaxM;   // int32 [max m + 1]
constexpr size_t kOffFlags =
    kOffOffs + ((sizeof(int32_t) * (kNoAllocMaxM + 1) + 255) / 256) * 256;  // int32 [4]
constexpr size_t kScratchBytes = kOffFlags + 256;
constexpr int kMaxDevices = 64;

}  // namespace

// Working memory of rs_draw_weighted_noalloc (about 16 MB per device).
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

std::mutex g_scratch_mu;
unsigned char* g_scratch_ptr[kMaxDevices] = {};

// Device address of this device's copy of the array (looked up once per device).
hipError_t scratch_address(unsigned char** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_scratch_ptr[dev] = static_cast<unsigned char*>(p);
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}

// flags[0] = done (1 skips the draw), flags[1] = error code (0 none, 1-3 selection limits,
// 4 invalid q), flags[2] = q usable. A proposal with an entry that is not positive and
// finite is rejected (no draw), as the host entry point rejects it.
__global__ __launch_bounds__(1024) void k_noalloc_begin(const float* __restrict__ q, int64_t m,
                                                        int32_t* __restrict__ flags) {
  __shared__ int bad;
  if (threadIdx.x == 0) bad = 0;
  __syncthreads();
  int b = 0;
  for (int64_t j = threadIdx.x; j < m; j += blockDim.x) {
    const float v = q[j];
    if (!(v > 0.0f) || !isfinite(v)) b = 1;
  }
  if (b) atomicOr(&bad, 1);
  __syncthreads();
  if (threadIdx.x == 0) {
    flags[0] = bad;
    flags[1] = bad ? 4 : 0;
    flags[2] = 1;
  }
}

// *status_out = the rs_status of the draw.
__global__ void k_noalloc_end(const int32_t* __restrict__ flags, int32_t* __restrict__ status_out) {
  if (threadIdx.x != 0) return;
  const int32_t e = flags[1];
  *status_out = e == 0 ? RS_OK : (e == 4 ? RS_EINVAL : RS_EDEVICE);
}

}  // namespace

extern "C" {

rs_status rs_draw_weighted_noalloc(const float* q, int64_t m, int32_t tau, uint64_t seed,
                                   uint64_t problem_id, int64_t k, int32_t* C_out,
                                   int32_t* status_out, void* stream) {
  if (!q || !C_out || !status_out || m < 1 || tau < 1 || tau > m || k < 0) return RS_EINVAL;
  if (m > kNoAllocMaxM) return RS_EINVAL;
  try {
    unsigned char* base = nullptr;
    if (scratch_address(&base) != hipSuccess) {
      (void)hipGetLastError();
      return RS_EDEVICE;
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    int32_t* flags = reinterpret_cast<int32_t*>(base + kOffFlags);
    hipLaunchKernelGGL(k_noalloc_begin, dim3(1), dim3(1024), 0, s, q, m, flags);
    if (hipGetLastError() != hipSuccess) return RS_EDEVICE;
    SketchArgs a{};
    a.kind = kWeighted;
    a.m = m;
    a.tau = tau;
    a.nsel = tau;
    a.seed = seed;
    a.pid = problem_id;
    a.k0 = k;
    a.nslots = 1;
    a.hmap = reinterpret_cast<int32_t*>(base + kOffHmap);
    a.members = C_out;
    a.offs = reinterpret_cast<int32_t*>(base + kOffOffs);
    a.keys = reinterpret_cast<uint64_t*>(base + kOffKeys);
    a.done = flags;
    a.err = flags + 1;
    a.q = q;
    a.q_ok = flags + 2;
    if (launch_sketch(a, s) != hipSuccess) {
      (void)hipGetLastError();
      return RS_EDEVICE;
    }
    hipLaunchKernelGGL(k_noalloc_end, dim3(1), dim3(64), 0, s, flags, status_out);
    if (hipGetLastError() != hipSuccess) return RS_EDEVICE;
    return RS_OK;
  } catch (...) {
    return RS_EDEVICE;
  }
}

}  // extern "C"
