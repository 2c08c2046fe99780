// Learned proposal for the subsample sketch (a distribution D other than uniform,
// Sec. 3; non-uniform coordinate probabilities, Sec. 7): per-coordinate features, a
// 6 -> 128 -> 128 -> 1 ReLU MLP (FP32) scoring the coordinates, the proposal
// q = (1 - eps) softmax(s) + eps / m, the trace of (features, credits) recorded from
// solves, and the network's training step (listwise loss, backward pass, Adam).
//
// Features of coordinate j at iteration k (r = r^k, rp = r^{k-1}, a_j = A_jj,
// last_j = latest iteration < k whose sketch held j, -1 if none), formed in FP64 and
// stored in FP32:
//   f0 = (log a_j - mean log a) / std log a,   f1 = clip(log|r_j| - log(a_j)/2 - log||r||
//   + log(sum a)/2, +-30),   f2 = log(1 + k - last_j),   f3 = clip(log|r_j - rp_j| - log||r||
//   + log(m)/2, +-30),   f4 = log(k + 1),   f5 = [last_j == k - 1].
// Credits of a recorded iteration: c_b = delta_b rho_b for the sketch's coordinates;
// they sum to delta^T G delta, the decrease of the squared A-norm error (eq:gradeqf).
//
// MLP parameters are one FP32 vector: W1 [6][128], b1, W2 [128][128], b2, w3, b3.
#include "dev_common.h"
#include "rs_internal.h"

namespace rs {
namespace {

constexpr int NF = kMlpFeatures;
constexpr int HID = kMlpHidden;
constexpr int OFF_W1 = 0, OFF_B1 = NF * HID, OFF_W2 = OFF_B1 + HID, OFF_B2 = OFF_W2 + HID * HID,
              OFF_W3 = OFF_B2 + HID, OFF_B3 = OFF_W3 + HID;
static_assert(OFF_B3 + 1 == kMlpParams, "parameter layout");
constexpr int kRows = 32;        // rows of the MLP per workgroup
constexpr int kW2Ld = HID + 1;   // padded LDS row of W2 (conflict-free by row and by column)
constexpr double kClip = 30.0;

// a_j = ||Z_j||^2 + lambda (FP64 accumulation), one wavefront per row.
template <typename T>
__global__ __launch_bounds__(256) void k_adiag(const T* __restrict__ Z, int64_t ldz, int64_t m,
                                               int64_t K, double lam, double* __restrict__ a) {
  const int lane = threadIdx.x & 63;
  const int64_t j = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (j >= m) return;
  const T* z = Z + j * ldz;
  double s = 0.0;
  for (int64_t c = lane; c < K; c += 64) {
    const double v = (double)z[c];
    s += v * v;
  }
  s = wave_sum(s);
  if (lane == 0) a[j] = s + lam;
}

// stats = {mean log a, std log a, sum a} (one workgroup, fixed reduction order).
__global__ __launch_bounds__(1024) void k_lstats(const double* __restrict__ a, int64_t m,
                                                 double* __restrict__ stats) {
  __shared__ double scratch[16];
  double s = 0.0, t = 0.0;
  for (int64_t j = threadIdx.x; j < m; j += blockDim.x) {
    s += log(a[j]);
    t += a[j];
  }
  const double mu = block_sum(s, scratch) / (double)m;
  const double tot = block_sum(t, scratch);
  double v = 0.0;
  for (int64_t j = threadIdx.x; j < m; j += blockDim.x) {
    const double d = log(a[j]) - mu;
    v += d * d;
  }
  const double var = block_sum(v, scratch) / (double)m;
  if (threadIdx.x == 0) {
    stats[0] = mu;
    stats[1] = sqrt(var);
    stats[2] = tot;
  }
}

__device__ __forceinline__ double clip30(double v) { return fmin(kClip, fmax(-kClip, v)); }

__device__ __forceinline__ void coord_features(int64_t j, const double* __restrict__ a,
                                               const double* __restrict__ stats,
                                               const double* __restrict__ r,
                                               const double* __restrict__ rp, int64_t lastj,
                                               int64_t k, double log_rn, double m, float* out) {
  const double la = log(a[j]);
  const double sd = stats[1];
  out[0] = (float)(sd > 0.0 ? (la - stats[0]) / sd : 0.0);
  out[1] = (float)clip30(log(fabs(r[j])) - 0.5 * la - log_rn + 0.5 * log(stats[2]));
  out[2] = (float)log(1.0 + (double)(k - lastj));
  out[3] = (float)clip30(log(fabs(r[j] - rp[j])) - log_rn + 0.5 * log(m));
  out[4] = (float)log((double)(k + 1));
  out[5] = (lastj == k - 1) ? 1.0f : 0.0f;
}

// ||r|| (one workgroup): written to *out as log ||r||.
__global__ __launch_bounds__(1024) void k_log_rnorm(const double* __restrict__ r, int64_t m,
                                                    double* __restrict__ out) {
  __shared__ double scratch[16];
  double s = 0.0;
  for (int64_t j = threadIdx.x; j < m; j += blockDim.x) s += r[j] * r[j];
  s = block_sum(s, scratch);
  if (threadIdx.x == 0) *out = 0.5 * log(s);
}

// Features of every coordinate (learned proposal at the start of a lookahead batch).
__global__ __launch_bounds__(256) void k_features(const double* __restrict__ a,
                                                  const double* __restrict__ stats,
                                                  const double* __restrict__ r,
                                                  const double* __restrict__ rp,
                                                  const int32_t* __restrict__ last, int64_t m,
                                                  int64_t k, const double* __restrict__ log_rn,
                                                  float* __restrict__ F,
                                                  const int32_t* __restrict__ done) {
  if (done && *done) return;
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= m) return;
  coord_features(j, a, stats, r, rp, last[j], k, *log_rn, (double)m, F + j * NF);
}

// Trace record of iteration k (one workgroup): features of the sketch's coordinates and
// their credits delta_b rho_b. last_j counts the sketches of earlier batches (`last`)
// and the earlier slots of the current batch (hmap of slots 0 .. slot - 1).
__global__ __launch_bounds__(1024) void k_trace(const TraceArgs t) {
  __shared__ double scratch[16];
  __shared__ int32_t rec;
  if (t.flags->done) return;
  double s = 0.0;
  for (int64_t j = threadIdx.x; j < t.m; j += blockDim.x) s += t.r[j] * t.r[j];
  s = block_sum(s, scratch);
  const double log_rn = 0.5 * log(s);
  if (threadIdx.x == 0) {
    rec = *t.count;
    *t.count = rec + 1;
  }
  __syncthreads();
  if (rec >= t.capacity) return;
  float* F = t.F + (int64_t)rec * t.tau * NF;
  float* c = t.credits + (int64_t)rec * t.tau;
  for (int b = threadIdx.x; b < t.tau; b += blockDim.x) {
    const int64_t j = t.members[b];
    int64_t lastj = t.last[j];
    for (int sl = t.slot - 1; sl >= 0; --sl)
      if (t.hmap_batch[(int64_t)sl * t.m + j] >= 0) {
        lastj = t.k0 + sl;
        break;
      }
    coord_features(j, t.a, t.stats, t.r, t.rp, lastj, t.k, log_rn, (double)t.m, F + (int64_t)b * NF);
    c[b] = (float)(t.delta[b] * t.rho[b]);
  }
}

// last_j <- the latest slot iteration holding j, for the slots of a finished batch.
__global__ void k_mark_last(const int32_t* __restrict__ members, int32_t tau, int32_t nslots,
                            int64_t k0, int32_t* __restrict__ last) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)tau * nslots) return;
  const int32_t slot = (int32_t)(e / tau);
  atomicMax(&last[members[e]], (int32_t)(k0 + slot));
}

// q = (1 - eps) softmax(s) + eps / m (one workgroup); *ok = 0 when q is not finite.
__global__ __launch_bounds__(1024) void k_proposal(const float* __restrict__ s, int64_t m, float eps,
                                                   float* __restrict__ q, int32_t* __restrict__ ok,
                                                   const int32_t* __restrict__ done) {
  __shared__ float red[1024];
  __shared__ double scratch[16];
  if (done && *done) return;
  float mx = -INFINITY;
  for (int64_t j = threadIdx.x; j < m; j += blockDim.x) mx = fmaxf(mx, s[j]);
  red[threadIdx.x] = mx;
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] = fmaxf(red[threadIdx.x], red[threadIdx.x + w]);
    __syncthreads();
  }
  mx = red[0];
  double z = 0.0;
  for (int64_t j = threadIdx.x; j < m; j += blockDim.x) z += (double)expf(s[j] - mx);
  z = block_sum(z, scratch);
  const float inv = (float)(1.0 / z);
  const float mix = 1.0f - eps, floor = eps / (float)m;
  int bad = !(mx < INFINITY && mx > -INFINITY) || !(z > 0.0 && z < INFINITY);
  for (int64_t j = threadIdx.x; j < m; j += blockDim.x) {
    const float v = mix * (expf(s[j] - mx) * inv) + floor;
    q[j] = v;
    bad |= !(v > 0.0f && v < INFINITY);
  }
  bad = __syncthreads_or(bad);
  if (threadIdx.x == 0) *ok = bad ? 0 : 1;
}

// q_j = a_j / sum a (the A_jj / Tr A proposal), FP32.
__global__ void k_diag_q(const double* __restrict__ a, const double* __restrict__ stats, int64_t m,
                         float* __restrict__ q) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j < m) q[j] = (float)(a[j] / stats[2]);
}

// Parameters from the counter RNG: weights uniform on +-1/sqrt(fan_in), biases 0.
__global__ void k_mlp_init(float* __restrict__ p, uint64_t seed) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= kMlpParams) return;
  double scale = 0.0;
  if (i < OFF_B1) scale = 1.0 / sqrt((double)NF);
  else if (i >= OFF_W2 && i < OFF_B2) scale = 1.0 / sqrt((double)HID);
  else if (i >= OFF_W3 && i < OFF_B3) scale = 1.0 / sqrt((double)HID);
  float v = 0.0f;
  if (scale > 0.0) {
    const Philox4 r = philox4x64_10((uint64_t)i, 0, kTagMlpInit, 0, seed, 0);
    const double u = ((double)(r.v0 >> 12) + 0.5) * 0x1p-52;
    v = (float)(scale * (2.0 * u - 1.0));
  }
  p[i] = v;
}

// ---------------------------------------------------------------------------
// MLP forward / backward on kRows rows per workgroup. Row r of the batch reads
// features F[row_index(r)]: rec == nullptr -> r itself; else record rec[r / tau],
// entry r % tau of a trace store with tau entries per record.
// ---------------------------------------------------------------------------
struct MlpLds {
  float W2[HID * kW2Ld];
  float W1[NF * HID];
  float b1[HID], b2[HID], w3[HID];
  float f[kRows * NF];
  float h1[kRows * HID];   // relu(z1); reused for the products of the output layer
  float d2[kRows * HID];   // dL/dz2 (backward)
  float ds[kRows];
};

__device__ __forceinline__ const float* feat_row(const float* F, const int32_t* rec, int32_t tau,
                                                 int64_t r) {
  if (!rec) return F + r * NF;
  return F + ((int64_t)rec[r / tau] * tau + (r % tau)) * NF;
}

// Loads the parameters and the block's rows, forms h1 in LDS and z2 for rows
// rg*16 .. rg*16+15 and unit u (returned in z2[16]).
__device__ __forceinline__ void mlp_front(MlpLds& L, const float* __restrict__ P,
                                          const float* __restrict__ F, const int32_t* rec,
                                          int32_t tau, int64_t r0, int64_t rows, float* z2) {
  const int tid = threadIdx.x;
  {
    // W2 as 16 float4 loads per thread, all issued before the first LDS store
    static_assert(HID * HID == 4 * 16 * 256 && OFF_W2 % 4 == 0, "W2 load layout");
    const float4* W2g = reinterpret_cast<const float4*>(P + OFF_W2);
    float4 v[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) v[q] = W2g[tid + 256 * q];
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int e = 4 * (tid + 256 * q);
      float* d = L.W2 + (e >> 7) * kW2Ld + (e & 127);
      d[0] = v[q].x;
      d[1] = v[q].y;
      d[2] = v[q].z;
      d[3] = v[q].w;
    }
  }
  for (int e = tid; e < NF * HID; e += 256) L.W1[e] = P[OFF_W1 + e];
  for (int e = tid; e < HID; e += 256) {
    L.b1[e] = P[OFF_B1 + e];
    L.b2[e] = P[OFF_B2 + e];
    L.w3[e] = P[OFF_W3 + e];
  }
  for (int e = tid; e < kRows * NF; e += 256) {
    const int64_t r = r0 + e / NF;
    L.f[e] = r < rows ? feat_row(F, rec, tau, r)[e % NF] : 0.0f;
  }
  __syncthreads();
  for (int e = tid; e < kRows * HID; e += 256) {
    const int rr = e >> 7, u = e & 127;
    float z = L.b1[u];
#pragma unroll
    for (int i = 0; i < NF; ++i) z += L.f[rr * NF + i] * L.W1[i * HID + u];
    L.h1[e] = fmaxf(z, 0.0f);
  }
  __syncthreads();
  const int u = tid & 127, rg = tid >> 7;
#pragma unroll
  for (int q = 0; q < 16; ++q) z2[q] = L.b2[u];
  for (int i = 0; i < HID; ++i) {
    const float w = L.W2[i * kW2Ld + u];
#pragma unroll
    for (int q = 0; q < 16; ++q) z2[q] += L.h1[(rg * 16 + q) * HID + i] * w;
  }
}

__global__ __launch_bounds__(256) void k_mlp_fwd(const float* __restrict__ P,
                                                 const float* __restrict__ F,
                                                 const int32_t* __restrict__ rec, int32_t tau,
                                                 int64_t rows, float* __restrict__ s,
                                                 const int32_t* __restrict__ done) {
  extern __shared__ __align__(16) unsigned char lds_raw[];
  MlpLds& L = *reinterpret_cast<MlpLds*>(lds_raw);
  if (done && *done) return;
  const int64_t r0 = (int64_t)blockIdx.x * kRows;
  float z2[16];
  mlp_front(L, P, F, rec, tau, r0, rows, z2);
  __syncthreads();  // h1 is overwritten below
  const int u = threadIdx.x & 127, rg = threadIdx.x >> 7;
#pragma unroll
  for (int q = 0; q < 16; ++q) L.h1[(rg * 16 + q) * HID + u] = fmaxf(z2[q], 0.0f) * L.w3[u];
  __syncthreads();
  if (threadIdx.x < kRows) {
    const int64_t r = r0 + threadIdx.x;
    float acc = P[OFF_B3];
    for (int i = 0; i < HID; ++i) acc += L.h1[threadIdx.x * HID + i];
    if (r < rows) s[r] = acc;
  }
}

// Listwise loss per record (one workgroup each): t = max(c, 0) / sum, p = softmax(s) over
// the record's tau entries, ds = (p - t) / nrec, loss[rec] = -sum t log p.
__global__ __launch_bounds__(256) void k_mlp_loss(const float* __restrict__ s,
                                                  const float* __restrict__ credits,
                                                  const int32_t* __restrict__ rec, int32_t tau,
                                                  int32_t nrec, float* __restrict__ ds,
                                                  double* __restrict__ loss) {
  __shared__ double scratch[16];
  __shared__ float red[256];
  const int i = blockIdx.x;
  const float* c = credits + (int64_t)rec[i] * tau;
  const float* si = s + (int64_t)i * tau;
  float* di = ds + (int64_t)i * tau;
  double cp = 0.0;
  float mx = -INFINITY;
  for (int b = threadIdx.x; b < tau; b += 256) {
    cp += (double)fmaxf(c[b], 0.0f);
    mx = fmaxf(mx, si[b]);
  }
  cp = block_sum(cp, scratch);
  red[threadIdx.x] = mx;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] = fmaxf(red[threadIdx.x], red[threadIdx.x + w]);
    __syncthreads();
  }
  mx = red[0];
  if (!(cp > 0.0)) {
    for (int b = threadIdx.x; b < tau; b += 256) di[b] = 0.0f;
    if (threadIdx.x == 0) loss[i] = 0.0;
    return;
  }
  double z = 0.0;
  for (int b = threadIdx.x; b < tau; b += 256) z += exp((double)(si[b] - mx));
  z = block_sum(z, scratch);
  const double lz = log(z);
  double l = 0.0;
  for (int b = threadIdx.x; b < tau; b += 256) {
    const double t = (double)fmaxf(c[b], 0.0f) / cp;
    const double logp = (double)(si[b] - mx) - lz;
    l -= t * logp;
    di[b] = (float)((exp(logp) - t) / (double)nrec);
  }
  l = block_sum(l, scratch);
  if (threadIdx.x == 0) loss[i] = l;
}

// Backward pass: per-workgroup partial gradients (kMlpParams floats) of sum_r ds_r s_r.
__global__ __launch_bounds__(256) void k_mlp_bwd(const float* __restrict__ P,
                                                 const float* __restrict__ F,
                                                 const int32_t* __restrict__ rec, int32_t tau,
                                                 int64_t rows, const float* __restrict__ ds,
                                                 float* __restrict__ partial) {
  extern __shared__ __align__(16) unsigned char lds_raw[];
  MlpLds& L = *reinterpret_cast<MlpLds*>(lds_raw);
  const int tid = threadIdx.x;
  const int64_t r0 = (int64_t)blockIdx.x * kRows;
  float* g = partial + (int64_t)blockIdx.x * kMlpParams;
  float z2[16];
  mlp_front(L, P, F, rec, tau, r0, rows, z2);
  for (int e = tid; e < kRows; e += 256) L.ds[e] = (r0 + e < rows) ? ds[r0 + e] : 0.0f;
  __syncthreads();
  const int u = tid & 127, rg = tid >> 7;
  // output layer: gw3_u = sum_r relu(z2) ds_r; dL/dz2 = ds_r w3_u [z2 > 0]
  float gw3 = 0.0f;
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const int rr = rg * 16 + q;
    const float h2 = fmaxf(z2[q], 0.0f);
    gw3 += h2 * L.ds[rr];
    L.d2[rr * HID + u] = z2[q] > 0.0f ? L.ds[rr] * L.w3[u] : 0.0f;
  }
  __shared__ float tmp[256];
  tmp[tid] = gw3;
  __syncthreads();
  if (tid < HID) g[OFF_W3 + tid] = tmp[tid] + tmp[tid + HID];
  if (tid == 0) {
    float sb = 0.0f;
    for (int rr = 0; rr < kRows; ++rr) sb += L.ds[rr];
    g[OFF_B3] = sb;
  }
  // gb2_u = sum_r d2; gW2[i][u] = sum_r h1[r][i] d2[r][u]
  if (tid < HID) {
    float sb = 0.0f;
    for (int rr = 0; rr < kRows; ++rr) sb += L.d2[rr * HID + tid];
    g[OFF_B2 + tid] = sb;
  }
  for (int ii = 0; ii < 64; ++ii) {
    const int i = rg * 64 + ii;
    float acc = 0.0f;
    for (int rr = 0; rr < kRows; ++rr) acc += L.h1[rr * HID + i] * L.d2[rr * HID + u];
    g[OFF_W2 + i * HID + u] = acc;
  }
  __syncthreads();
  // dL/dz1[r][i] = [h1 > 0] sum_u d2[r][u] W2[i][u]  (thread: unit i, rows rg*16 ..)
  const int i = tid & 127;
  float d1[16];
#pragma unroll
  for (int q = 0; q < 16; ++q) d1[q] = 0.0f;
  for (int uu = 0; uu < HID; ++uu) {
    const float w = L.W2[i * kW2Ld + uu];
#pragma unroll
    for (int q = 0; q < 16; ++q) d1[q] += L.d2[(rg * 16 + q) * HID + uu] * w;
  }
  __syncthreads();  // every read of d2 is done: reuse it for dL/dz1
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const int rr = rg * 16 + q;
    L.d2[rr * HID + i] = L.h1[rr * HID + i] > 0.0f ? d1[q] : 0.0f;
  }
  __syncthreads();
  if (tid < HID) {
    float sb = 0.0f;
    for (int rr = 0; rr < kRows; ++rr) sb += L.d2[rr * HID + tid];
    g[OFF_B1 + tid] = sb;
  }
  for (int e = tid; e < NF * HID; e += 256) {
    const int f = e / HID, ii = e % HID;
    float acc = 0.0f;
    for (int rr = 0; rr < kRows; ++rr) acc += L.f[rr * NF + f] * L.d2[rr * HID + ii];
    g[OFF_W1 + e] = acc;
  }
}

// grad[p] = sum over workgroups (in order, FP64) of the partial gradients.
__global__ void k_grad_reduce(const float* __restrict__ partial, int32_t nblocks,
                              float* __restrict__ grad) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= kMlpParams) return;
  double s = 0.0;
  for (int b = 0; b < nblocks; ++b) s += (double)partial[(int64_t)b * kMlpParams + p];
  grad[p] = (float)s;
}

// Adam with the scalar coefficients formed in FP64 and rounded once (1 - beta2 in FP32
// arithmetic would carry a relative error of order 1e-5).
__global__ void k_adam(float* __restrict__ P, float* __restrict__ m1, float* __restrict__ m2,
                       const float* __restrict__ g, int64_t t, double lr, double b1, double b2,
                       double eps) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= kMlpParams) return;
  const float fb1 = (float)b1, fc1 = (float)(1.0 - b1), fb2 = (float)b2, fc2 = (float)(1.0 - b2);
  const float inv_c1 = (float)(1.0 / (1.0 - pow(b1, (double)t)));
  const float inv_c2 = (float)(1.0 / (1.0 - pow(b2, (double)t)));
  const float gv = g[p];
  const float a = fb1 * m1[p] + fc1 * gv;
  const float v = fb2 * m2[p] + fc2 * gv * gv;
  m1[p] = a;
  m2[p] = v;
  P[p] -= (float)lr * (a * inv_c1) / (sqrtf(v * inv_c2) + (float)eps);
}

}  // namespace

size_t mlp_lds_bytes() { return sizeof(MlpLds); }

hipError_t launch_adiag(const void* Z, int32_t z_f32, int64_t ldz, int64_t m, int64_t K, double lam,
                        double* a, double* stats, hipStream_t s) {
  const unsigned g = (unsigned)((m + 3) / 4);
  if (z_f32)
    hipLaunchKernelGGL(k_adiag<float>, dim3(g), dim3(256), 0, s, (const float*)Z, ldz, m, K, lam, a);
  else
    hipLaunchKernelGGL(k_adiag<double>, dim3(g), dim3(256), 0, s, (const double*)Z, ldz, m, K, lam, a);
  hipLaunchKernelGGL(k_lstats, dim3(1), dim3(1024), 0, s, a, m, stats);
  return hipGetLastError();
}

hipError_t launch_lstats(const double* a, int64_t m, double* stats, hipStream_t s) {
  hipLaunchKernelGGL(k_lstats, dim3(1), dim3(1024), 0, s, a, m, stats);
  return hipGetLastError();
}

hipError_t launch_features(const double* a, const double* stats, const double* r, const double* rp,
                           const int32_t* last, int64_t m, int64_t k, double* log_rn, float* F,
                           const int32_t* done, hipStream_t s) {
  hipLaunchKernelGGL(k_log_rnorm, dim3(1), dim3(1024), 0, s, r, m, log_rn);
  hipLaunchKernelGGL(k_features, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, s, a, stats, r, rp,
                     last, m, k, log_rn, F, done);
  return hipGetLastError();
}

hipError_t launch_trace(const TraceArgs& t, hipStream_t s) {
  hipLaunchKernelGGL(k_trace, dim3(1), dim3(1024), 0, s, t);
  return hipGetLastError();
}

hipError_t launch_mark_last(const int32_t* members, int32_t tau, int32_t nslots, int64_t k0,
                            int32_t* last, hipStream_t s) {
  const int64_t n = (int64_t)tau * nslots;
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_mark_last, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, members, tau,
                     nslots, k0, last);
  return hipGetLastError();
}

hipError_t launch_proposal(const float* s_in, int64_t m, float eps, float* q, int32_t* ok,
                           const int32_t* done, hipStream_t s) {
  hipLaunchKernelGGL(k_proposal, dim3(1), dim3(1024), 0, s, s_in, m, eps, q, ok, done);
  return hipGetLastError();
}

hipError_t launch_diag_q(const double* a, const double* stats, int64_t m, float* q, hipStream_t s) {
  hipLaunchKernelGGL(k_diag_q, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, s, a, stats, m, q);
  return hipGetLastError();
}

hipError_t launch_mlp_init(float* p, uint64_t seed, hipStream_t s) {
  hipLaunchKernelGGL(k_mlp_init, dim3((kMlpParams + 255) / 256), dim3(256), 0, s, p, seed);
  return hipGetLastError();
}

hipError_t launch_mlp_fwd(const float* P, const float* F, const int32_t* rec, int32_t tau, int64_t rows,
                          float* out, const int32_t* done, hipStream_t s) {
  if (rows <= 0) return hipSuccess;
  const size_t bytes = sizeof(MlpLds);
  hipError_t e = hipFuncSetAttribute((const void*)k_mlp_fwd, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)bytes);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_mlp_fwd, dim3((unsigned)((rows + kRows - 1) / kRows)), dim3(256), bytes, s, P, F,
                     rec, tau, rows, out, done);
  return hipGetLastError();
}

int32_t mlp_bwd_blocks(int64_t rows) { return (int32_t)((rows + kRows - 1) / kRows); }

hipError_t launch_mlp_step(const float* P, const float* F, const float* credits, const int32_t* rec,
                           int32_t tau, int32_t nrec, float* s_buf, float* ds_buf, double* loss,
                           float* partial, float* grad, hipStream_t s) {
  const int64_t rows = (int64_t)nrec * tau;
  hipError_t e = launch_mlp_fwd(P, F, rec, tau, rows, s_buf, nullptr, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_mlp_loss, dim3(nrec), dim3(256), 0, s, s_buf, credits, rec, tau, nrec, ds_buf, loss);
  const size_t bytes = sizeof(MlpLds);
  e = hipFuncSetAttribute((const void*)k_mlp_bwd, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
  if (e != hipSuccess) return e;
  const int32_t nb = mlp_bwd_blocks(rows);
  hipLaunchKernelGGL(k_mlp_bwd, dim3(nb), dim3(256), bytes, s, P, F, rec, tau, rows, ds_buf, partial);
  hipLaunchKernelGGL(k_grad_reduce, dim3((kMlpParams + 255) / 256), dim3(256), 0, s, partial, nb, grad);
  return hipGetLastError();
}

hipError_t launch_adam(float* P, float* m1, float* m2, const float* g, int64_t t, double lr, double b1,
                       double b2, double eps, hipStream_t s) {
  hipLaunchKernelGGL(k_adam, dim3((kMlpParams + 255) / 256), dim3(256), 0, s, P, m1, m2, g, t, lr, b1, b2,
                     eps);
  return hipGetLastError();
}

}  // namespace rs
