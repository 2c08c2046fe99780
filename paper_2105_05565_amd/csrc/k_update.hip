// Per-iteration kernels of sketch-and-project with momentum (Alg. 2).
//
//   k_delta : ||r^k|| from the previous update's partial sums (fixed order), the stop
//             test ||r^k|| / ||r^0|| <= tol, rho = S_k^T r^k (bucket sums) and
//             delta_k = G_k^{-1} rho (rows of the precomputed inverse);
//   k_update: x^{k+1} = (1 + beta) x^k - beta x^{k-1} - gamma S_k delta and
//             r^{k+1} = (1 + beta) r^k - beta r^{k-1} - gamma AS_k delta
//             (eq:res_update_mom), written over the x^{k-1} / r^{k-1} buffers, plus
//             per-workgroup partial sums of ||r^{k+1}||^2.
// Once the stop test fires, a device flag turns every later kernel into a no-op, so
// the state stays at the iteration that met the tolerance.
#include "dev_common.h"
#include "rs_internal.h"

namespace rs {
namespace {

constexpr int kThreads = 256;
constexpr int kDeltaRows = 64;  // rows of G^{-1} per k_delta workgroup

__device__ __forceinline__ double reduce_partials(const double* __restrict__ partials, int npart,
                                                  double* scratch) {
  double s = 0.0;
  for (int i = threadIdx.x; i < npart; i += blockDim.x) s += partials[i];
  return block_sum(s, scratch);
}

__global__ __launch_bounds__(kThreads) void k_init_state(const double* __restrict__ b,
                                                         double* __restrict__ x0,
                                                         double* __restrict__ x1,
                                                         double* __restrict__ r0,
                                                         double* __restrict__ r1, int64_t m,
                                                         double* __restrict__ partials,
                                                         int32_t npart) {
  __shared__ double scratch[16];
  const int64_t per = (m + npart - 1) / npart;
  const int64_t j0 = min(m, (int64_t)blockIdx.x * per), j1 = min(m, j0 + per);
  double s = 0.0;
  for (int64_t j = j0 + threadIdx.x; j < j1; j += blockDim.x) {
    const double r = -b[j];
    x0[j] = 0.0;
    x1[j] = 0.0;
    r0[j] = r;
    r1[j] = r;
    s += r * r;
  }
  s = block_sum(s, scratch);
  if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

__global__ __launch_bounds__(kThreads) void k_norm0(const double* __restrict__ partials, int32_t npart,
                                                    DevFlags* __restrict__ flags,
                                                    double* __restrict__ hist) {
  __shared__ double scratch[16];
  const double s = reduce_partials(partials, npart, scratch);
  if (threadIdx.x == 0) {
    flags->r0norm = sqrt(s);
    flags->done = (s == 0.0) ? 1 : 0;
    flags->err = 0;
    flags->k_done = 0;
    hist[0] = 1.0;
  }
}

__global__ __launch_bounds__(kThreads) void k_delta(const double* __restrict__ r,
                                                    const int32_t* __restrict__ hmap,
                                                    const int32_t* __restrict__ members,
                                                    const int32_t* __restrict__ offs, int32_t tau,
                                                    const double* __restrict__ Ginv, int64_t ldg,
                                                    const double* __restrict__ partials,
                                                    int32_t npart, DevFlags* __restrict__ flags,
                                                    double* __restrict__ hist, int64_t k, double tol,
                                                    double* __restrict__ delta) {
  extern __shared__ __align__(16) double rho[];  // [tau]
  __shared__ double scratch[16];
  if (flags->done) return;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  double rel = 1.0;  // ||r^0|| / ||r^0||
  if (k > 0) {
    const double s = reduce_partials(partials, npart, scratch);
    rel = sqrt(s) / flags->r0norm;
    if (blockIdx.x == 0 && tid == 0) hist[k] = rel;
  }
  if (rel <= tol) {
    if (blockIdx.x == 0 && tid == 0) {
      flags->k_done = k;
      flags->done = 1;
    }
    return;
  }
  for (int bk = tid; bk < tau; bk += kThreads) {
    double s = 0.0;
    for (int p = offs[bk]; p < offs[bk + 1]; ++p) {
      const int j = members[p];
      const double v = r[j];
      s += (hmap[j] & 1) ? -v : v;
    }
    rho[bk] = s;
  }
  __syncthreads();
  const int row_end = min(tau, (int)(blockIdx.x + 1) * kDeltaRows);
  for (int c = blockIdx.x * kDeltaRows + wave; c < row_end; c += kThreads / 64) {
    const double* g = Ginv + (int64_t)c * ldg;
    double s = 0.0;
    for (int cc = lane; cc < tau; cc += 64) s += g[cc] * rho[cc];
    s = wave_sum(s);
    if (lane == 0) delta[c] = s;
  }
}

__global__ __launch_bounds__(kThreads) void k_update(const double* __restrict__ AS, int32_t tau,
                                                     const double* __restrict__ delta,
                                                     const int32_t* __restrict__ hmap, int64_t m,
                                                     const double* __restrict__ x,
                                                     double* __restrict__ x_prev_out,
                                                     const double* __restrict__ r,
                                                     double* __restrict__ r_prev_out, double gamma,
                                                     double beta, double* __restrict__ partials,
                                                     int32_t npart,
                                                     const DevFlags* __restrict__ flags) {
  extern __shared__ __align__(16) double dl[];  // [tau]
  __shared__ double scratch[16];
  if (flags->done) return;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  for (int c = tid; c < tau; c += kThreads) dl[c] = delta[c];
  __syncthreads();
  const int64_t per = (m + npart - 1) / npart;
  const int64_t j0 = min(m, (int64_t)blockIdx.x * per), j1 = min(m, j0 + per);
  const double onepb = 1.0 + beta;
  double ss = 0.0;
  for (int64_t j = j0 + wave; j < j1; j += kThreads / 64) {
    const double* row = AS + j * tau;
    double s = 0.0;
    for (int c = lane; c < tau; c += 64) s += row[c] * dl[c];
    s = wave_sum(s);
    if (lane == 0) {
      const int code = hmap[j];
      double sd = 0.0;
      if (code >= 0) sd = (code & 1) ? -dl[code >> 1] : dl[code >> 1];
      const double rn = onepb * r[j] - beta * r_prev_out[j] - gamma * s;
      const double xn = onepb * x[j] - beta * x_prev_out[j] - gamma * sd;
      r_prev_out[j] = rn;
      x_prev_out[j] = xn;
      ss += rn * rn;
    }
  }
  ss = block_sum(ss, scratch);
  if (tid == 0) partials[blockIdx.x] = ss;
}

__global__ __launch_bounds__(kThreads) void k_finalize(const double* __restrict__ partials,
                                                       int32_t npart, DevFlags* __restrict__ flags,
                                                       double* __restrict__ hist, int64_t k,
                                                       double tol) {
  __shared__ double scratch[16];
  if (flags->done) return;
  const double s = reduce_partials(partials, npart, scratch);
  if (threadIdx.x == 0) {
    const double rel = sqrt(s) / flags->r0norm;
    hist[k] = rel;
    if (rel <= tol) {
      flags->k_done = k;
      flags->done = 1;
    }
  }
}

}  // namespace

hipError_t launch_init_state(const double* b, double* x0, double* x1, double* r0, double* r1,
                             int64_t m, double* partials, int32_t npart, DevFlags* flags,
                             double* hist, hipStream_t s) {
  hipLaunchKernelGGL(k_init_state, dim3(npart), dim3(kThreads), 0, s, b, x0, x1, r0, r1, m,
                     partials, npart);
  hipLaunchKernelGGL(k_norm0, dim3(1), dim3(kThreads), 0, s, partials, npart, flags, hist);
  return hipGetLastError();
}

hipError_t launch_delta(const double* r, const int32_t* hmap, const int32_t* members,
                        const int32_t* offs, int32_t tau, const double* Ginv, int64_t ldg,
                        const double* partials, int32_t npart, DevFlags* flags, double* hist,
                        int64_t k, double tol, double* delta, hipStream_t s) {
  const unsigned grid = (unsigned)((tau + kDeltaRows - 1) / kDeltaRows);
  hipLaunchKernelGGL(k_delta, dim3(grid), dim3(kThreads), sizeof(double) * tau, s, r, hmap, members,
                     offs, tau, Ginv, ldg, partials, npart, flags, hist, k, tol, delta);
  return hipGetLastError();
}

hipError_t launch_update(const double* AS, int32_t tau, const double* delta, const int32_t* hmap,
                         int64_t m, const double* x, double* x_prev_out, const double* r,
                         double* r_prev_out, double gamma, double beta, double* partials,
                         int32_t npart, const DevFlags* flags, hipStream_t s) {
  hipLaunchKernelGGL(k_update, dim3(npart), dim3(kThreads), sizeof(double) * tau, s, AS, tau, delta,
                     hmap, m, x, x_prev_out, r, r_prev_out, gamma, beta, partials, npart, flags);
  return hipGetLastError();
}

hipError_t launch_finalize(const double* partials, int32_t npart, DevFlags* flags, double* hist,
                           int64_t k, double tol, hipStream_t s) {
  hipLaunchKernelGGL(k_finalize, dim3(1), dim3(kThreads), 0, s, partials, npart, flags, hist, k, tol);
  return hipGetLastError();
}

}  // namespace rs
