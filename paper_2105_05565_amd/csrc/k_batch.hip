// Per-iteration kernels of the batched solver: many problems, each with a grid of
// regularisers lambda_l and several right-hand sides, advanced in lock step.
//
// Problem p holds J = nlam * nrhs solves (slot j = l * nrhs + q) that share one sketch
// S_k per iteration, so that the lambda-free product B S = Z (Z^T S) is formed once and
// A(lambda) S delta = B S delta + lambda S delta (A(lambda) = Z Z^T + lambda I). The
// iterates of all slots are stored row-major, m x J, so a row of B S meets the J
// columns of Delta = [delta_0 .. delta_{J-1}] in one FP64 MFMA tile product and the
// update of eq:res_update_mom becomes
//   R^{k+1} = (1 + beta) R^k - beta R^{k-1} - gamma (B S Delta + (S Delta) diag(lambda_j)),
//   X^{k+1} = (1 + beta) X^k - beta X^{k-1} - gamma S Delta.
// A slot stops at the first iteration whose ||r^k|| / ||r^0|| <= tol and keeps that
// iterate (later updates copy it forward); a problem stops when every slot has stopped
// or its iteration cap is reached. The iteration counter lives in device memory, so
// the same captured sequence of launches can be replayed.
#include "chol_tiles.h"
#include "dev_common.h"
#include "rs_internal.h"

namespace rs {
namespace {

using chol::Acc;
using chol::LDT;
using chol::NB;

constexpr int kThreads = 256;

// ---------------------------------------------------------------------------
// Initial state: x^0 = x^{-1} = 0, r^0 = r^{-1} = -b_q for slot j = l nrhs + q,
// ||r^0|| per slot (fixed-order reduction), stop flags for b_q = 0.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kThreads) void k_binit(const BState* __restrict__ S) {
  __shared__ double scratch[16];
  const BState& st = S[blockIdx.x];
  const int tid = threadIdx.x;
  const int64_t m = st.m;
  const int J = st.J, nrhs = st.nrhs;
  for (int64_t e = tid; e < m * J; e += kThreads) {
    const int64_t i = e / J;
    const int j = (int)(e % J);
    const double r = -st.b[i * nrhs + (j % nrhs)];
    st.x[0][e] = 0.0;
    st.x[1][e] = 0.0;
    st.r[0][e] = r;
    st.r[1][e] = r;
  }
  for (int q = 0; q < nrhs; ++q) {
    double s = 0.0;
    for (int64_t i = tid; i < m; i += kThreads) {
      const double v = st.b[i * nrhs + q];
      s += v * v;
    }
    const double n0 = sqrt(block_sum(s, scratch));  // the total, in every thread
    for (int j = tid; j < J; j += kThreads)
      if (j % nrhs == q) {
        st.r0n[j] = n0;
        st.stop_k[j] = (n0 == 0.0) ? 0 : -1;
        st.rel[j] = (n0 == 0.0) ? 0.0 : 1.0;
      }
    __syncthreads();
  }
  if (tid == 0) {
    bool any = false;
    for (int j = 0; j < J; ++j) any |= st.stop_k[j] < 0;
    *st.inactive = (!any || st.cap <= 0) ? 1 : 0;
    *st.iters = 0;
  }
}

// ---------------------------------------------------------------------------
// rho_j = S^T r_j for every slot: one wavefront per (problem, bucket), lane j sums the
// bucket's members in order.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(64) void k_brho(const BState* __restrict__ S,
                                             const int32_t* __restrict__ items, int32_t nitems,
                                             const BGlobal* __restrict__ g) {
  const int j = threadIdx.x;
  const int64_t k = g->k;
  for (int32_t t = blockIdx.x; t < nitems; t += gridDim.x) {
    const BState& st = S[items[2 * t]];
    const int b = items[2 * t + 1];
    if (*st.inactive) continue;
    if (j >= st.J) continue;
    const double* r = st.r[k & 1];
    double s = 0.0;
    for (int p = st.offs[b]; p < st.offs[b + 1]; ++p) {
      const int64_t i = st.members[p];
      const double v = r[i * st.J + j];
      s += (st.hmap[i] & 1) ? -v : v;
    }
    st.rho[(int64_t)j * st.ldg + b] = s;
  }
}

// ---------------------------------------------------------------------------
// delta_j = G(lambda_l)^{-1} rho_j for the nrhs slots of lambda_l: one wavefront per
// row c of the inverse (lanes stride its columns), items = (problem, l, 4-row chunk).
// ---------------------------------------------------------------------------
constexpr int kMaxRhs = 8;

__global__ __launch_bounds__(kThreads) void k_bdelta(const BState* __restrict__ S,
                                                     const int32_t* __restrict__ items,
                                                     int32_t nitems) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int32_t t = blockIdx.x; t < nitems; t += gridDim.x) {
    const BState& st = S[items[3 * t]];
    if (*st.inactive) continue;
    const int l = items[3 * t + 1];
    const int c = items[3 * t + 2] * 4 + wave;
    if (c >= st.tau) continue;
    const int nrhs = st.nrhs;
    const int64_t ldg = st.ldg;
    const double* gi = st.Ginv + ((int64_t)l * ldg + c) * ldg;
    double acc[kMaxRhs];
#pragma unroll
    for (int q = 0; q < kMaxRhs; ++q) acc[q] = 0.0;
    for (int cc = lane; cc < st.tau; cc += 64) {
      const double gv = gi[cc];
#pragma unroll
      for (int q = 0; q < kMaxRhs; ++q)
        if (q < nrhs) acc[q] += gv * st.rho[(int64_t)(l * nrhs + q) * ldg + cc];
    }
#pragma unroll
    for (int q = 0; q < kMaxRhs; ++q) {
      if (q >= nrhs) break;
      const double s = wave_sum(acc[q]);
      const int j = l * nrhs + q;
      if (lane == 0) st.delta[(int64_t)j * ldg + c] = (st.stop_k[j] >= 0) ? 0.0 : s;
    }
  }
}

// ---------------------------------------------------------------------------
// Momentum update for a 64-row tile of one problem, all J slots at once. The product
// (B S)[rows, :] Delta runs on FP64 MFMA over 64-wide panels of the sketch dimension
// (B S and Delta are zero beyond tau). Per-tile sums of r_j^2 are reduced in a fixed
// order for the stop test.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kThreads) void k_bupdate(const BState* __restrict__ S,
                                                      const int32_t* __restrict__ items,
                                                      int32_t nitems, const BGlobal* __restrict__ g,
                                                      const double* __restrict__ betas,
                                                      const double* __restrict__ gammas) {
  extern __shared__ __align__(16) double lds[];
  double* ta = lds;             // B S panel [64 rows][64]
  double* tb = lds + NB * LDT;  // Delta^T panel [64 slots][64]
  const int tid = threadIdx.x;
  const int64_t k = g->k;
  if (g->done) return;
  const double beta = betas[k], gamma = gammas[k];
  const double onepb = 1.0 + beta;
  const int cur = (int)(k & 1), nxt = cur ^ 1;
  for (int32_t t = blockIdx.x; t < nitems; t += gridDim.x) {
    const BState& st = S[items[2 * t]];
    if (*st.inactive) continue;  // uniform across the workgroup
    const int tile = items[2 * t + 1];
    const int64_t r0 = (int64_t)tile * NB;
    const int64_t m = st.m, ldg = st.ldg, ldas = st.ldas;
    const int J = st.J;
    Acc c;
    chol::acc_zero(c);
    for (int64_t kc = 0; kc < ldg; kc += NB) {
      for (int e = tid; e < NB * NB; e += kThreads) {
        const int rr = e >> 6, cc = e & 63;
        const int64_t i = r0 + rr;
        ta[rr * LDT + cc] = (i < m) ? st.BS[i * ldas + kc + cc] : 0.0;
        tb[rr * LDT + cc] = (rr < J) ? st.delta[(int64_t)rr * ldg + kc + cc] : 0.0;
      }
      __syncthreads();
      chol::tile_mma(c, ta, tb);
      __syncthreads();
    }
    const double* x = st.x[cur];
    double* xo = st.x[nxt];
    const double* r = st.r[cur];
    double* ro = st.r[nxt];
    chol::acc_for_each(c, [&](int row, int j, double v) {
      const int64_t i = r0 + row;
      double sq = 0.0;
      if (i < m && j < J) {
        const int64_t idx = i * J + j;
        if (st.stop_k[j] >= 0) {  // stopped: carry the kept iterate forward
          ro[idx] = r[idx];
          xo[idx] = x[idx];
        } else {
          const int code = st.hmap[i];
          double sd = 0.0;
          if (code >= 0) {
            const double dv = st.delta[(int64_t)j * ldg + (code >> 1)];
            sd = (code & 1) ? -dv : dv;
          }
          const double asd = v + st.lam[j / st.nrhs] * sd;
          const double rn = onepb * r[idx] - beta * ro[idx] - gamma * asd;
          const double xn = onepb * x[idx] - beta * xo[idx] - gamma * sd;
          ro[idx] = rn;
          xo[idx] = xn;
          sq = rn * rn;
        }
      }
      ta[row * LDT + j] = sq;
    });
    __syncthreads();
    if (tid < J) {
      double s = 0.0;
      for (int rr = 0; rr < NB; ++rr) s += ta[rr * LDT + tid];
      st.partials[(int64_t)tile * J + tid] = s;
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Stop tests after the update of iteration k: one wavefront per problem.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(64) void k_bfinal(const BState* __restrict__ S,
                                               const BGlobal* __restrict__ g, double tol) {
  const BState& st = S[blockIdx.x];
  if (g->done || *st.inactive) return;
  const int64_t k = g->k;
  const int j = threadIdx.x;
  int running = 0;
  if (j < st.J && st.stop_k[j] < 0) {
    double s = 0.0;
    for (int t = 0; t < st.ntiles; ++t) s += st.partials[(int64_t)t * st.J + j];
    const double rel = sqrt(s) / st.r0n[j];
    st.rel[j] = rel;
    // mixed precision: only a refreshed (FP64) residual may stop a slot
    const bool may_stop = st.refresh == 0 || (k + 1) % st.refresh == 0;
    if (rel <= tol && may_stop) st.stop_k[j] = k + 1;
    else running = 1;
  }
  const int any = __syncthreads_or(running);
  if (j == 0 && (!any || k + 1 >= st.cap)) {
    *st.iters = k + 1;
    *st.inactive = 1;
  }
}

// ---------------------------------------------------------------------------
// FP64 refresh of a mixed-precision problem's residuals after the update of iteration k when
// (k + 1) is a multiple of its refresh interval: for the iterates X^{k+1} (h = 0) and X^k
// (h = 1), U_h = Z^T X_h (K x J), then R_h = Z U_h + X_h diag(lambda_j) - B. Both are FP64
// MFMA tile products over 64 x 64 tiles staged in LDS (contraction in ascending order); the
// squares of the refreshed R^{k+1} are summed per 64-row tile for the stop test. Slots that
// have stopped keep their carried residual.
// ---------------------------------------------------------------------------
__device__ __forceinline__ bool refresh_due(const BState& st, int64_t k) {
  return st.refresh > 0 && (k + 1) % st.refresh == 0;
}

__global__ __launch_bounds__(kThreads) void k_bref_u(const BState* __restrict__ S, const int32_t* __restrict__ items,
                                                     int32_t nitems, const BGlobal* __restrict__ g) {
  extern __shared__ __align__(16) double lds[];
  double* ta = lds;             // Z^T tile [64 columns of K][64 rows of Z]
  double* tb = lds + NB * LDT;  // X^T tile [64 slots][64 rows of Z]
  if (g->done) return;
  const int64_t k = g->k;
  const int tid = threadIdx.x;
  for (int32_t t = blockIdx.x; t < nitems; t += gridDim.x) {
    const BState& st = S[items[3 * t]];
    if (*st.inactive || !refresh_due(st, k)) continue;  // uniform across the workgroup
    const int64_t kk0 = (int64_t)items[3 * t + 1] * NB;
    const int h = items[3 * t + 2];
    const int nxt = (int)((k + 1) & 1);
    const double* X = st.x[h == 0 ? nxt : (nxt ^ 1)];
    const int64_t m = st.m, K = st.K, ldz = st.ldz;
    const int J = st.J;
    Acc c;
    chol::acc_zero(c);
    for (int64_t i0 = 0; i0 < m; i0 += NB) {
      for (int e = tid; e < NB * NB; e += kThreads) {
        const int ii = e >> 6, cc = e & 63;
        const int64_t i = i0 + ii;
        ta[cc * LDT + ii] = (i < m && kk0 + cc < K) ? st.Z[i * ldz + kk0 + cc] : 0.0;
        tb[cc * LDT + ii] = (i < m && cc < J) ? X[i * J + cc] : 0.0;
      }
      __syncthreads();
      chol::tile_mma(c, ta, tb);
      __syncthreads();
    }
    double* U = st.Uref + (int64_t)h * K * J;
    chol::acc_for_each(c, [&](int r, int j, double v) {
      if (kk0 + r < K && j < J) U[(kk0 + r) * J + j] = v;
    });
  }
}

__global__ __launch_bounds__(kThreads) void k_bref_r(const BState* __restrict__ S, const int32_t* __restrict__ items,
                                                     int32_t nitems, const BGlobal* __restrict__ g) {
  extern __shared__ __align__(16) double lds[];
  double* ta = lds;             // Z tile [64 rows][64 columns of K]
  double* tb = lds + NB * LDT;  // U^T tile [64 slots][64 columns of K]
  if (g->done) return;
  const int64_t k = g->k;
  const int tid = threadIdx.x;
  for (int32_t t = blockIdx.x; t < nitems; t += gridDim.x) {
    const BState& st = S[items[3 * t]];
    if (*st.inactive || !refresh_due(st, k)) continue;  // uniform across the workgroup
    const int tile = items[3 * t + 1];
    const int h = items[3 * t + 2];
    const int64_t i0 = (int64_t)tile * NB;
    const int nxt = (int)((k + 1) & 1);
    const int buf = h == 0 ? nxt : (nxt ^ 1);
    const double* X = st.x[buf];
    double* R = st.r[buf];
    const double* U = st.Uref + (int64_t)h * st.K * st.J;
    const int64_t m = st.m, K = st.K, ldz = st.ldz;
    const int J = st.J;
    Acc c;
    chol::acc_zero(c);
    for (int64_t kk0 = 0; kk0 < K; kk0 += NB) {
      for (int e = tid; e < NB * NB; e += kThreads) {
        const int rr = e >> 6, cc = e & 63;
        const int64_t i = i0 + rr;
        ta[rr * LDT + cc] = (i < m && kk0 + cc < K) ? st.Z[i * ldz + kk0 + cc] : 0.0;
        tb[cc * LDT + rr] = (kk0 + rr < K && cc < J) ? U[(kk0 + rr) * J + cc] : 0.0;
      }
      __syncthreads();
      chol::tile_mma(c, ta, tb);
      __syncthreads();
    }
    chol::acc_for_each(c, [&](int row, int j, double v) {
      const int64_t i = i0 + row;
      double sq = 0.0;
      if (i < m && j < J && st.stop_k[j] < 0) {
        const int64_t idx = i * J + j;
        const double rn = v + st.lam[j / st.nrhs] * X[idx] - st.b[i * st.nrhs + (j % st.nrhs)];
        R[idx] = rn;
        sq = rn * rn;
      }
      ta[row * LDT + j] = sq;
    });
    __syncthreads();
    if (h == 0 && tid < J) {
      double s = 0.0;
      for (int rr = 0; rr < NB; ++rr) s += ta[rr * LDT + tid];
      st.partials[(int64_t)tile * J + tid] = s;
    }
    __syncthreads();
  }
}

// Advance the shared iteration counter (unless every problem had already stopped) and
// record whether any problem is still running.
__global__ __launch_bounds__(kThreads) void k_badvance(const BState* __restrict__ S, int32_t nprob,
                                                       BGlobal* __restrict__ g, int32_t advance) {
  int all = 1;
  for (int p = threadIdx.x; p < nprob; p += kThreads) all &= (*S[p].inactive != 0) ? 1 : 0;
  all = __syncthreads_and(all);
  if (threadIdx.x == 0) {
    if (advance && !g->done) g->k += 1;
    g->done = all;
  }
}

// Strided column copy: dst[i * dst_ld + dst_col] = src[i * src_ld + src_col], i < m.
__global__ void k_bcol(const double* __restrict__ src, int64_t m, int64_t src_ld, int64_t src_col,
                       double* __restrict__ dst, int64_t dst_ld, int64_t dst_col) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < m) dst[i * dst_ld + dst_col] = src[i * src_ld + src_col];
}

}  // namespace

hipError_t launch_binit(const BState* S, int32_t nprob, BGlobal* g, hipStream_t s) {
  if (nprob <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_binit, dim3(nprob), dim3(kThreads), 0, s, S);
  hipLaunchKernelGGL(k_badvance, dim3(1), dim3(kThreads), 0, s, S, nprob, g, 0);
  return hipGetLastError();
}

hipError_t launch_brho(const BState* S, const int32_t* items, int32_t nitems, const BGlobal* g,
                       int32_t grid, hipStream_t s) {
  if (nitems <= 0) return hipSuccess;
  grid = grid < 1 ? 1 : (grid > nitems ? nitems : grid);
  hipLaunchKernelGGL(k_brho, dim3(grid), dim3(64), 0, s, S, items, nitems, g);
  return hipGetLastError();
}

hipError_t launch_bdelta(const BState* S, const int32_t* items, int32_t nitems, int32_t grid,
                         hipStream_t s) {
  if (nitems <= 0) return hipSuccess;
  grid = grid < 1 ? 1 : (grid > nitems ? nitems : grid);
  hipLaunchKernelGGL(k_bdelta, dim3(grid), dim3(kThreads), 0, s, S, items, nitems);
  return hipGetLastError();
}

hipError_t launch_bupdate(const BState* S, const int32_t* items, int32_t nitems, const BGlobal* g,
                          const double* betas, const double* gammas, int32_t grid, hipStream_t s) {
  if (nitems <= 0) return hipSuccess;
  grid = grid < 1 ? 1 : (grid > nitems ? nitems : grid);
  const size_t bytes = sizeof(double) * 2 * NB * LDT;
  hipError_t e = hipFuncSetAttribute((const void*)k_bupdate, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)bytes);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_bupdate, dim3(grid), dim3(kThreads), bytes, s, S, items, nitems, g, betas,
                     gammas);
  return hipGetLastError();
}

hipError_t launch_bfinal(const BState* S, int32_t nprob, BGlobal* g, double tol, hipStream_t s) {
  if (nprob <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_bfinal, dim3(nprob), dim3(64), 0, s, S, g, tol);
  hipLaunchKernelGGL(k_badvance, dim3(1), dim3(kThreads), 0, s, S, nprob, g, 1);
  return hipGetLastError();
}

hipError_t launch_brefresh(const BState* S, const int32_t* uitems, int32_t nu, const int32_t* ritems, int32_t nr,
                           const BGlobal* g, int32_t grid, hipStream_t s) {
  if (nu <= 0 || nr <= 0) return hipSuccess;
  const size_t bytes = sizeof(double) * 2 * NB * LDT;
  hipError_t e = hipFuncSetAttribute((const void*)k_bref_u, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
  if (e == hipSuccess)
    e = hipFuncSetAttribute((const void*)k_bref_r, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
  if (e != hipSuccess) return e;
  const int gu = grid < 1 ? 1 : (grid > nu ? nu : grid);
  const int gr = grid < 1 ? 1 : (grid > nr ? nr : grid);
  hipLaunchKernelGGL(k_bref_u, dim3(gu), dim3(kThreads), bytes, s, S, uitems, nu, g);
  hipLaunchKernelGGL(k_bref_r, dim3(gr), dim3(kThreads), bytes, s, S, ritems, nr, g);
  return hipGetLastError();
}

hipError_t launch_bcol(const double* src, int64_t m, int64_t src_ld, int64_t src_col, double* dst,
                       int64_t dst_ld, int64_t dst_col, hipStream_t s) {
  if (m <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_bcol, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, s, src, m, src_ld,
                     src_col, dst, dst_ld, dst_col);
  return hipGetLastError();
}

}  // namespace rs
