// Per-iteration kernels of sketch-and-project with momentum (Alg. 2).
//
//   k_delta : ||r^k|| from the previous update's partial sums (fixed order), the stop
//             test ||r^k|| / ||r^0|| <= tol, and delta_k = G_k^{-1} rho_k (rows of the
//             precomputed inverse; rho_k = S_k^T r^k was produced beforehand);
//   k_update: x^{k+1} = (1 + beta) x^k - beta x^{k-1} - gamma S_k delta and
//             r^{k+1} = (1 + beta) r^k - beta r^{k-1} - gamma AS_k delta
//             (eq:res_update_mom), written over the x^{k-1} / r^{k-1} buffers, plus
//             per-workgroup partial sums of ||r^{k+1}||^2. When the next sketch S_{k+1}
//             is already drawn, rows are visited bucket-major for S_{k+1} and the next
//             sketched residual rho_{k+1} = S_{k+1}^T r^{k+1} is summed on the way;
//   k_rho   : rho = S^T r on its own, with the same summation order, for iterations
//             whose predecessor did not produce it.
// The accelerated method (Alg. 3) uses the same kernels: k_update then also updates v and
// r_v in place and writes r_z = alpha r_v + (1 - alpha) r_w, which is what the next
// sketch is applied to, and the norm partials are those of r_v.
// Once the stop test fires, a device flag turns every later kernel into a no-op, so
// the state stays at the iteration that met the tolerance.
#include "dev_common.h"
#include "rs_internal.h"

namespace rs {
namespace {

constexpr int kThreads = 256;
constexpr int kDeltaRows = 4;       // rows of G^{-1} per k_delta workgroup (one per wave)
constexpr int kBucketWaves = 8;     // waves per bucket in the bucket-major update (and in k_rho)
constexpr int kUpdateThreads = 64 * kBucketWaves;
constexpr int kRowsPerWave = 4;     // rows per wave in the row-range update

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

// v = 0, r_v = r_z = r^0 (Alg. 3 starts from w = v = 0)
__global__ __launch_bounds__(kThreads) void k_init_accel(const double* __restrict__ r0, double* __restrict__ v,
                                                         double* __restrict__ rv, double* __restrict__ rz,
                                                         int64_t m) {
  const int64_t j = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (j < m) {
    v[j] = 0.0;
    rv[j] = r0[j];
    rz[j] = r0[j];
  }
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

// rho[b] = sum_{p in bucket b} s_{members[p]} r[members[p]]: wave w of the bucket's
// workgroup sums p = offs[b] + w, + kBucketWaves, ... in order; waves are combined in order
// (the bucket-major update uses the same order).
__global__ __launch_bounds__(kBucketWaves * 64) void k_rho(const double* __restrict__ r,
                                                           const int32_t* __restrict__ hmap,
                                                           const int32_t* __restrict__ members,
                                                           const int32_t* __restrict__ offs,
                                                           double* __restrict__ rho,
                                                           const DevFlags* __restrict__ flags) {
  __shared__ double part[kBucketWaves];
  if (flags->done) return;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int b = blockIdx.x;
  double s = 0.0;
  if (lane == 0) {
    for (int p = offs[b] + wave; p < offs[b + 1]; p += kBucketWaves) {
      const int j = members[p];
      const double v = r[j];
      s += (hmap[j] & 1) ? -v : v;
    }
    part[wave] = s;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < kBucketWaves; ++w) t += part[w];
    rho[b] = t;
  }
}

__global__ __launch_bounds__(kThreads) void k_delta(const double* __restrict__ rho_in, int32_t tau,
                                                    const double* __restrict__ Ginv, int64_t ldg,
                                                    const double* __restrict__ partials,
                                                    int32_t npart, DevFlags* __restrict__ flags,
                                                    double* __restrict__ hist, int64_t k, double tol,
                                                    double* __restrict__ delta) {
  extern __shared__ __align__(16) double rho[];  // [tau]
  __shared__ double scratch[16];
  if (flags->done) return;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  for (int c = tid; c < tau; c += kThreads) rho[c] = rho_in[c];
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
  __syncthreads();
  const int row_end = min(tau, (int)(blockIdx.x + 1) * kDeltaRows);
  for (int c = blockIdx.x * kDeltaRows + wave; c < row_end; c += kThreads / 64) {
    const double* g = Ginv + (int64_t)c * ldg;
    // four columns of the row per lane in flight together (clamped loads, selected terms:
    // the same terms in the same order as a column-by-column loop)
    double s = 0.0;
    for (int c0 = lane; c0 < tau; c0 += 256) {
      double v[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) v[q] = g[min(c0 + 64 * q, tau - 1)];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int cc = min(c0 + 64 * q, tau - 1);
        const double t = fma(v[q], rho[cc], s);
        s = c0 + 64 * q < tau ? t : s;
      }
    }
    s = wave_sum(s);
    if (lane == 0) delta[c] = s;
  }
}

// rows whose loads a wave issues before reducing any (FP64 rows: 2; FP32 rows: 1)
template <typename ASV>
struct RowsAtOnce {
  static constexpr int value = sizeof(ASV) == 8 ? 2 : 1;
};

// sum_c AS[j_u][c] dl[c] for R rows (j_u < 0: none, 0 returned), partial per lane, c ascending.
// A lane's chunks c0, c0 + 64, c0 + 128, c0 + 192 load together, unconditionally (past the row's
// end its last chunk is read again, and a missing row reads row 0; neither enters the sum), so a
// row costs one memory latency per four chunks instead of one per chunk.
template <int R>
__device__ __forceinline__ void rows_dot(const double* __restrict__ AS, const int64_t (&j)[R], int64_t ldas,
                                         const double* dl, int lane, double (&s)[R]) {
  const int half = (int)(ldas >> 1);
  const double2* row[R];
#pragma unroll
  for (int u = 0; u < R; ++u) {
    s[u] = 0.0;
    row[u] = reinterpret_cast<const double2*>(AS + (j[u] >= 0 ? j[u] : 0) * ldas);
  }
  for (int c0 = lane; c0 < half; c0 += 256) {
    double2 a[4][R];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int c = min(c0 + 64 * q, half - 1);
#pragma unroll
      for (int u = 0; u < R; ++u) a[q][u] = row[u][c];
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int c2 = min(c0 + 64 * q, half - 1);
      const bool in = c0 + 64 * q < half;
      const double d0 = dl[2 * c2], d1 = dl[2 * c2 + 1];
#pragma unroll
      for (int u = 0; u < R; ++u) {
        const double t = a[q][u].x * d0 + a[q][u].y * d1;
        s[u] += in ? t : 0.0;  // a select, not a branch: the loads stay ahead of every use
      }
    }
  }
#pragma unroll
  for (int u = 0; u < R; ++u)
    if (j[u] < 0) s[u] = 0.0;
}

template <int R>
__device__ __forceinline__ void rows_dot(const float* __restrict__ AS, const int64_t (&j)[R], int64_t ldas,
                                         const double* dl, int lane, double (&s)[R]) {
  const int quarter = (int)(ldas >> 2);
  const float4* row[R];
#pragma unroll
  for (int u = 0; u < R; ++u) {
    s[u] = 0.0;
    row[u] = reinterpret_cast<const float4*>(AS + (j[u] >= 0 ? j[u] : 0) * ldas);
  }
  for (int c0 = lane; c0 < quarter; c0 += 256) {
    float4 a[4][R];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int c = min(c0 + 64 * q, quarter - 1);
#pragma unroll
      for (int u = 0; u < R; ++u) a[q][u] = row[u][c];
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int c4 = min(c0 + 64 * q, quarter - 1);
      const bool in = c0 + 64 * q < quarter;
#pragma unroll
      for (int u = 0; u < R; ++u) {
        const double t = (double)a[q][u].x * dl[4 * c4] + (double)a[q][u].y * dl[4 * c4 + 1] +
                         (double)a[q][u].z * dl[4 * c4 + 2] + (double)a[q][u].w * dl[4 * c4 + 3];
        s[u] += in ? t : 0.0;  // a select, not a branch: the loads stay ahead of every use
      }
    }
  }
#pragma unroll
  for (int u = 0; u < R; ++u)
    if (j[u] < 0) s[u] = 0.0;
}

// Value of v in lane l (compile-time after unrolling), as a wave-uniform scalar.
__device__ __forceinline__ double lane_value(double v, int l) {
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), l);
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), l);
  return __hiloint2double(hi, lo);
}

// Accelerated method (Alg. 3): v and r_v (updated in place), r_z (written), constants.
struct AccelRows {
  double* v;
  double* rv;
  double* rz;
  double alpha, beta, gamma;
};

// Up to R rows of the update (j_u < 0: none), one wave: lane u loads and
// updates row u, all rows' loads in flight together. Returns in every lane the new
// residual entry whose norm is tracked (rn: r^{k+1}, or r_v^{k+1} for ACC) and the one
// the next sketch is applied to (rq: r^{k+1}, or r_z^{k+1}), 0 for none.
template <typename ASV, int R, bool ACC>
__device__ __forceinline__ void update_rows(const int64_t (&j)[R], const ASV* __restrict__ AS,
                                            int64_t ldas, const double* dl, const int32_t* __restrict__ hmap,
                                            const double* __restrict__ x, double* __restrict__ xo,
                                            const double* __restrict__ r, double* __restrict__ ro,
                                            double gamma, double beta, const AccelRows& ac, int lane,
                                            double (&rn)[R], double (&rq)[R]) {
  int64_t jl = -1;
#pragma unroll
  for (int u = 0; u < R; ++u)
    if (lane == u) jl = j[u];
  int code = -1;
  double rj = 0.0, roj = 0.0, xj = 0.0, xoj = 0.0;
  if (jl >= 0) {  // issued ahead of the products so their latency overlaps them
    code = hmap[jl];
    rj = r[jl];
    xj = x[jl];
    if constexpr (ACC) {
      roj = ac.rv[jl];  // r_v and v in place of r^{k-1} and x^{k-1}
      xoj = ac.v[jl];
    } else {
      roj = ro[jl];
      xoj = xo[jl];
    }
  }
  double s[R];
  rows_dot(AS, j, ldas, dl, lane, s);
  double sl = 0.0;
#pragma unroll
  for (int u = 0; u < R; ++u) {
    const double t = wave_sum(s[u]);
    if (lane == u) sl = t;
  }
  double rnl = 0.0, rql = 0.0;
  if (jl >= 0) {
    double sd = 0.0;
    if (code >= 0) sd = (code & 1) ? -dl[code >> 1] : dl[code >> 1];
    if constexpr (ACC) {
      // w = xj, v = xoj, r_w = rj, r_v = roj; g_j = sd, (A g)_j = sl
      const double z = ac.alpha * xoj + (1.0 - ac.alpha) * xj;
      const double rz = ac.alpha * roj + (1.0 - ac.alpha) * rj;
      const double wn = z - sd;
      const double vn = ac.beta * xoj + (1.0 - ac.beta) * z - ac.gamma * sd;
      const double rwn = rz - sl;
      const double rvn = ac.beta * roj + (1.0 - ac.beta) * rz - ac.gamma * sl;
      const double rzn = ac.alpha * rvn + (1.0 - ac.alpha) * rwn;
      xo[jl] = wn;
      ro[jl] = rwn;
      ac.v[jl] = vn;
      ac.rv[jl] = rvn;
      ac.rz[jl] = rzn;
      rnl = rvn;
      rql = rzn;
    } else {
      const double onepb = 1.0 + beta;
      rnl = onepb * rj - beta * roj - gamma * sl;
      const double xn = onepb * xj - beta * xoj - gamma * sd;
      ro[jl] = rnl;
      xo[jl] = xn;
      rql = rnl;
    }
  }
#pragma unroll
  for (int u = 0; u < R; ++u) {
    rn[u] = lane_value(rnl, u);
    if constexpr (ACC)
      rq[u] = lane_value(rql, u);
    else
      rq[u] = rn[u];
  }
}

template <typename ASV>
struct UpdateArgs {
  const ASV* AS;
  int64_t ldas;
  int32_t tau;
  const double* delta;
  const int32_t* hmap;
  int64_t m;
  const double* x;
  double* xo;
  const double* r;
  double* ro;
  double gamma, beta;
  double* partials;
  // next sketch (bucket-major visit and rho_{k+1}); hmap_n == nullptr: none
  const int32_t* hmap_n;
  const int32_t* members_n;
  const int32_t* offs_n;
  int32_t skip_all_rows;  // 1 when every coordinate is a member of the next sketch
  double* rho_n;
  int32_t nbucket_blocks;  // workgroups in the bucket-major part
  const DevFlags* flags;
  AccelRows acc;           // accelerated method only
};

template <typename ASV, bool ACC>
// at least 4 waves per SIMD (at most 128 VGPRs: the four chunks of a row's loads in flight)
__global__ __launch_bounds__(kUpdateThreads, 4) void k_update(UpdateArgs<ASV> a) {
  constexpr int R = RowsAtOnce<ASV>::value;
  extern __shared__ __align__(16) double dl[];  // [ldas]
  __shared__ double scratch[16];
  __shared__ double part[kBucketWaves];
  if (a.flags->done) return;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  for (int c = tid; c < (int)a.ldas; c += blockDim.x) dl[c] = (c < a.tau) ? a.delta[c] : 0.0;
  __syncthreads();
  double ss = 0.0;
  if ((int)blockIdx.x < a.nbucket_blocks) {
    // bucket b of the next sketch: 8 waves share its members, in a fixed order
    const int b = blockIdx.x;
    const int pe = a.offs_n[b + 1];
    double rs = 0.0;
    // members p = offs[b] + wave, + kBucketWaves, ... in order, R of them per pass
    for (int p0 = a.offs_n[b] + wave; p0 < pe; p0 += kBucketWaves * R) {
      int64_t j[R];
#pragma unroll
      for (int u = 0; u < R; ++u) {
        const int p = p0 + u * kBucketWaves;
        j[u] = p < pe ? (int64_t)a.members_n[p] : -1;
      }
      double rn[R], rq[R];
      update_rows<ASV, R, ACC>(j, a.AS, a.ldas, dl, a.hmap, a.x, a.xo, a.r, a.ro, a.gamma, a.beta, a.acc, lane,
                               rn, rq);
      if (lane == 0) {
#pragma unroll
        for (int u = 0; u < R; ++u)
          if (j[u] >= 0) {
            ss += rn[u] * rn[u];
            rs += (a.hmap_n[j[u]] & 1) ? -rq[u] : rq[u];
          }
      }
    }
    if (lane == 0) part[wave] = rs;
    __syncthreads();
    if (tid == 0) {
      double t = 0.0;
      for (int w = 0; w < kBucketWaves; ++w) t += part[w];
      a.rho_n[b] = t;
    }
  } else if (!a.skip_all_rows) {
    // rows outside the next sketch (all rows when there is none), in index order
    const int64_t blk = (int64_t)blockIdx.x - a.nbucket_blocks;
    const int64_t rows_per_block = (int64_t)(blockDim.x >> 6) * kRowsPerWave;
    const int64_t j0 = blk * rows_per_block, j1 = min(a.m, j0 + rows_per_block);
    const int nw = blockDim.x >> 6;
    for (int64_t jb = j0 + wave; jb < j1; jb += (int64_t)nw * R) {
      int64_t j[R];
#pragma unroll
      for (int u = 0; u < R; ++u) {
        const int64_t jj = jb + (int64_t)u * nw;
        j[u] = (jj < j1 && !(a.hmap_n && a.hmap_n[jj] >= 0)) ? jj : -1;
      }
      double rn[R], rq[R];
      update_rows<ASV, R, ACC>(j, a.AS, a.ldas, dl, a.hmap, a.x, a.xo, a.r, a.ro, a.gamma, a.beta, a.acc, lane,
                               rn, rq);
      if (lane == 0) {
#pragma unroll
        for (int u = 0; u < R; ++u) ss += rn[u] * rn[u];
      }
    }
  }
  ss = block_sum(ss, scratch);
  if (tid == 0) a.partials[blockIdx.x] = ss;
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

// One launch gathers the host's view of a finished batch (out: mapped host memory).
__global__ __launch_bounds__(256) void k_batch_report(const DevFlags* __restrict__ flags,
                                                      const int32_t* __restrict__ err,
                                                      const double* __restrict__ hist, int64_t k,
                                                      const int32_t* __restrict__ status, int32_t nb,
                                                      BatchReport* __restrict__ out) {
  for (int i = threadIdx.x; i < nb; i += blockDim.x) out->status[i] = status[i];
  if (threadIdx.x == 0) {
    out->flags = *flags;
    out->err = *err;
    out->nb = nb;
    out->rel = k > 0 ? hist[k - 1] : 1.0;
  }
}

}  // namespace

int32_t update_partials(int64_t m, int32_t tau) {
  const int64_t rows_per_block = (int64_t)(kUpdateThreads / 64) * kRowsPerWave;
  return (int32_t)(tau + (m + rows_per_block - 1) / rows_per_block);
}

hipError_t launch_init_state(const double* b, double* x0, double* x1, double* r0, double* r1,
                             int64_t m, double* partials, int32_t npart, DevFlags* flags,
                             double* hist, hipStream_t s) {
  hipLaunchKernelGGL(k_init_state, dim3(npart), dim3(kThreads), 0, s, b, x0, x1, r0, r1, m,
                     partials, npart);
  hipLaunchKernelGGL(k_norm0, dim3(1), dim3(kThreads), 0, s, partials, npart, flags, hist);
  return hipGetLastError();
}

hipError_t launch_init_accel(const double* r0, double* v, double* rv, double* rz, int64_t m, hipStream_t s) {
  if (m == 0) return hipSuccess;
  hipLaunchKernelGGL(k_init_accel, dim3((unsigned)((m + kThreads - 1) / kThreads)), dim3(kThreads), 0, s, r0, v,
                     rv, rz, m);
  return hipGetLastError();
}

hipError_t launch_rho(const double* r, const int32_t* hmap, const int32_t* members,
                      const int32_t* offs, int32_t tau, double* rho, const DevFlags* flags,
                      hipStream_t s) {
  hipLaunchKernelGGL(k_rho, dim3(tau), dim3(kBucketWaves * 64), 0, s, r, hmap, members, offs, rho,
                     flags);
  return hipGetLastError();
}

hipError_t launch_delta(const double* rho, int32_t tau, const double* Ginv, int64_t ldg,
                        const double* partials, int32_t npart, DevFlags* flags, double* hist,
                        int64_t k, double tol, double* delta, hipStream_t s) {
  const unsigned grid = (unsigned)((tau + kDeltaRows - 1) / kDeltaRows);
  hipLaunchKernelGGL(k_delta, dim3(grid), dim3(kThreads), sizeof(double) * tau, s, rho, tau, Ginv,
                     ldg, partials, npart, flags, hist, k, tol, delta);
  return hipGetLastError();
}

template <typename ASV>
hipError_t update_launch(const ASV* AS, int64_t ldas, int32_t tau, const double* delta,
                         const int32_t* hmap, int64_t m, const double* x, double* x_prev_out,
                         const double* r, double* r_prev_out, double gamma, double beta,
                         double* partials, int32_t npart, const int32_t* hmap_next,
                         const int32_t* members_next, const int32_t* offs_next,
                         int32_t next_covers_all, double* rho_next, const DevFlags* flags,
                         const AccelRows* acc, hipStream_t s) {
  UpdateArgs<ASV> a;
  a.AS = AS;
  a.ldas = ldas;
  a.tau = tau;
  a.delta = delta;
  a.hmap = hmap;
  a.m = m;
  a.x = x;
  a.xo = x_prev_out;
  a.r = r;
  a.ro = r_prev_out;
  a.gamma = gamma;
  a.beta = beta;
  a.partials = partials;
  a.hmap_n = hmap_next;
  a.members_n = members_next;
  a.offs_n = offs_next;
  a.skip_all_rows = (hmap_next && next_covers_all) ? 1 : 0;
  a.rho_n = rho_next;
  a.nbucket_blocks = hmap_next ? tau : 0;
  a.flags = flags;
  const int64_t rows_per_block = (int64_t)(kUpdateThreads / 64) * kRowsPerWave;
  const int32_t nrow_blocks = (int32_t)((m + rows_per_block - 1) / rows_per_block);
  const int32_t grid = tau + nrow_blocks;
  if (grid != npart) return hipErrorInvalidValue;
  a.acc = acc ? *acc : AccelRows{nullptr, nullptr, nullptr, 0.0, 0.0, 0.0};
  // without a next sketch the bucket part is empty: its partial slots are written as zero
  if (acc)
    hipLaunchKernelGGL((k_update<ASV, true>), dim3(grid), dim3(kUpdateThreads), sizeof(double) * ldas, s, a);
  else
    hipLaunchKernelGGL((k_update<ASV, false>), dim3(grid), dim3(kUpdateThreads), sizeof(double) * ldas, s, a);
  return hipGetLastError();
}

hipError_t launch_update(const void* AS, int32_t as_f32, int64_t ldas, int32_t tau, const double* delta,
                         const int32_t* hmap, int64_t m, const double* x, double* x_prev_out,
                         const double* r, double* r_prev_out, double gamma, double beta,
                         double* partials, int32_t npart, const int32_t* hmap_next,
                         const int32_t* members_next, const int32_t* offs_next,
                         int32_t next_covers_all, double* rho_next, const DevFlags* flags,
                         hipStream_t s) {
  if (as_f32)
    return update_launch<float>((const float*)AS, ldas, tau, delta, hmap, m, x, x_prev_out, r,
                                r_prev_out, gamma, beta, partials, npart, hmap_next, members_next,
                                offs_next, next_covers_all, rho_next, flags, nullptr, s);
  return update_launch<double>((const double*)AS, ldas, tau, delta, hmap, m, x, x_prev_out, r,
                               r_prev_out, gamma, beta, partials, npart, hmap_next, members_next,
                               offs_next, next_covers_all, rho_next, flags, nullptr, s);
}

hipError_t launch_update_accel(const double* AS, int64_t ldas, int32_t tau, const double* delta,
                               const int32_t* hmap, int64_t m, const double* w, double* w_out, const double* rw,
                               double* rw_out, double* v, double* rv, double* rz, double alpha, double beta,
                               double gamma, double* partials, int32_t npart, const int32_t* hmap_next,
                               const int32_t* members_next, const int32_t* offs_next, int32_t next_covers_all,
                               double* rho_next, const DevFlags* flags, hipStream_t s) {
  const AccelRows acc{v, rv, rz, alpha, beta, gamma};
  return update_launch<double>(AS, ldas, tau, delta, hmap, m, w, w_out, rw, rw_out, 0.0, 0.0, partials, npart,
                               hmap_next, members_next, offs_next, next_covers_all, rho_next, flags, &acc, s);
}

hipError_t launch_finalize(const double* partials, int32_t npart, DevFlags* flags, double* hist,
                           int64_t k, double tol, hipStream_t s) {
  hipLaunchKernelGGL(k_finalize, dim3(1), dim3(kThreads), 0, s, partials, npart, flags, hist, k, tol);
  return hipGetLastError();
}

hipError_t launch_batch_report(const DevFlags* flags, const int32_t* err, const double* hist, int64_t k,
                               const int32_t* status, int32_t nb, BatchReport* out, hipStream_t s) {
  hipLaunchKernelGGL(k_batch_report, dim3(1), dim3(256), 0, s, flags, err, hist, k, status, nb, out);
  return hipGetLastError();
}

}  // namespace rs
