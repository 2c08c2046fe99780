// FP64 Cholesky factorisation and inverse of the sketched matrix G = S^T A S.
//
// The least-norm solution of G delta = S^T r (eq:sketched_system) is computed as
// delta = G^{-1} rho with G^{-1} = L^{-T} L^{-1} from the Cholesky factor L of the
// lower triangle of G. The factorisation does not depend on the iterate, so it is
// computed ahead for a batch of sketches, one workgroup per sketch, and the
// per-iteration critical path keeps a single matrix-vector product.
//
// A column of S that is zero (an empty count bucket) makes the matching row and
// column of G zero and rho_b = 0; the diagonal entry is set to 1 so that delta_b = 0,
// which equals the pseudo-inverse solution. Padding to a multiple of 64 is the
// identity as well.
//
// Blocked algorithm on 64 x 64 tiles (4 waves, FP64 MFMA 16x16x4 for tile products,
// operands staged in LDS), with U = L^{-T} (upper triangular) kept instead of L^{-1}
// so that every tile product reads its operands row-major. Every phase is a sequence of
// chains sum_k A_k B_k^T accumulated in MFMA registers, one chain per output tile, written
// once; the operands of the next step load while the current step multiplies:
//   1. left-looking Cholesky: C_ij = G_ij - sum_{k<j} L_ik L_jk^T, the diagonal tile
//      factored and inverted in LDS (X_jj = L_jj^{-1}), panel L_ij = C_ij X_jj^T;
//   2. U_ji = -(sum_{k=j}^{i-1} U_jk L_ik^T) U_ii for i > j  (U = (L^{-1})^T);
//   3. G^{-1} = U U^T, tile (i, j) = sum_{k >= max(i,j)} U_ik U_jk^T, both triangles.
#include "chol_tiles.h"
#include "dev_common.h"
#include "rs_internal.h"

namespace rs {
namespace {

using namespace chol;

// One 64 x 64 tile held in registers between its global load and its LDS store:
// 16 doubles per thread as 8 double2 (element e = tid + 256 u: row e / 32, columns
// 2 (e % 32) and 2 (e % 32) + 1), so that a tile row is one 512-byte coalesced read.
struct TileRegs {
  double2 v[8];
};

__device__ __forceinline__ void tile_gload(TileRegs& t, const double* __restrict__ src, int64_t ld) {
#pragma unroll
  for (int u = 0; u < 8; ++u) {
    const int e = threadIdx.x + u * kThreads;
    t.v[u] = *reinterpret_cast<const double2*>(src + (int64_t)(e >> 5) * ld + 2 * (e & 31));
  }
}

__device__ __forceinline__ void tile_lstore(double* dst, const TileRegs& t) {
#pragma unroll
  for (int u = 0; u < 8; ++u) {
    const int e = threadIdx.x + u * kThreads;
    double* p = dst + (e >> 5) * LDT + 2 * (e & 31);
    p[0] = t.v[u].x;
    p[1] = t.v[u].y;
  }
}

__device__ __forceinline__ double* gtile(double* base, int64_t ld, int i, int j) {
  return base + (int64_t)i * NB * ld + (int64_t)j * NB;
}

// Chains of tile products C = sum_k A_k B_k^T, one chain per output tile, run back to
// back: while the MFMAs of step s read the operands in LDS (ta, tb), the operands of
// step s + 1 -- of the same chain or of the next one -- are already loading into
// registers. At the last step of a chain, epi(it, C) consumes the accumulator; it may use
// ta and tb as scratch and must end with a workgroup barrier. The operands of a chain's
// first step never depend on the epilogue of the chain before it (checked for each
// phase's order where the iterator is defined). Before a long epilogue (it.long_epi(),
// the diagonal factorisation) the next loads are issued after it instead: it is much
// longer than their latency, and the staging registers stay free for it.
template <class It, class Epi>
__device__ __forceinline__ void chain_pipeline(It it, int64_t ld, double* ta, double* tb, Epi epi) {
  if (!it.valid()) return;
  TileRegs ra, rb;
  tile_gload(ra, it.a(), ld);
  tile_gload(rb, it.b(), ld);
  tile_lstore(ta, ra);
  tile_lstore(tb, rb);
  __syncthreads();
  Acc c;
  acc_zero(c);
  while (true) {
    It nx = it;
    nx.advance();
    const bool more = nx.valid();
    const bool early = more && !(it.last() && it.long_epi());
    if (early) {
      tile_gload(ra, nx.a(), ld);
      tile_gload(rb, nx.b(), ld);
    }
    tile_mma(c, ta, tb);
    __syncthreads();
    if (it.last()) {
      epi(it, c);
      acc_zero(c);
    }
    if (!more) break;
    if (!early) {
      tile_gload(ra, nx.a(), ld);
      tile_gload(rb, nx.b(), ld);
    }
    tile_lstore(ta, ra);
    tile_lstore(tb, rb);
    __syncthreads();
    it = nx;
  }
}

// Phase 1, block columns j >= 1, left-looking: C_ij = sum_{k < j} L_ik L_jk^T for
// i = j .. nt-1 (the diagonal tile first). The first step of a chain reads block column 0.
struct ItChol {
  double* G;
  int64_t ld;
  int nt, j, i, k;
  __device__ bool valid() const { return j < nt; }
  __device__ const double* a() const { return gtile(G, ld, i, k); }
  __device__ const double* b() const { return gtile(G, ld, j, k); }
  __device__ bool last() const { return k == j - 1; }
  __device__ bool long_epi() const { return i == j; }
  __device__ void advance() {
    if (++k < j) return;
    k = 0;
    if (++i < nt) return;
    ++j;
    i = j;
  }
};

// Phase 2: S_ji = sum_{k = j}^{i-1} U_jk L_ik^T for i > j, rows j in order, columns i
// ascending. The chain of (j, i + 1) reads U_ji (the epilogue of (j, i)) only at its last
// step; its first step reads U_jj.
struct ItInv {
  double* U;
  double* G;
  int64_t ld;
  int nt, j, i, k;
  __device__ bool valid() const { return j < nt - 1; }
  __device__ const double* a() const { return gtile(U, ld, j, k); }
  __device__ const double* b() const { return gtile(G, ld, i, k); }
  __device__ bool last() const { return k == i - 1; }
  __device__ bool long_epi() const { return false; }
  __device__ void advance() {
    if (++k < i) return;
    if (++i == nt) {
      ++j;
      i = j + 1;
    }
    k = j;
  }
};

// Phase 3: (G^{-1})_ij = sum_{k >= i} U_ik U_jk^T for j <= i; reads U only.
struct ItLauum {
  double* U;
  int64_t ld;
  int nt, i, j, k;
  __device__ bool valid() const { return i < nt; }
  __device__ const double* a() const { return gtile(U, ld, i, k); }
  __device__ const double* b() const { return gtile(U, ld, j, k); }
  __device__ bool last() const { return k == nt - 1; }
  __device__ bool long_epi() const { return false; }
  __device__ void advance() {
    if (++k < nt) return;
    if (++j > i) {
      ++i;
      j = 0;
    }
    k = i;
  }
};

// Phases 1-3 on the assembled, padded ldg x ldg matrix G (lower triangle read):
// G <- G^{-1} (both triangles), U <- L^{-T} (upper block triangle; the tile below each
// diagonal tile, U_{i,i-1}, holds X_ii = L_ii^{-1} for phase 2).
// LDS: ta, tb, td, tx (64 x LDT each).
__device__ __forceinline__ void factor_invert(double* __restrict__ G, double* __restrict__ U,
                                              int64_t ldg, double* ta, double* tb, double* td,
                                              double* tx, int* bad_flag) {
  const int nt = (int)(ldg / NB);
  // td holds C_jj: factor it, keep X_jj = L_jj^{-1} in tx, store L_jj, U_jj = X_jj^T and
  // (j >= 1) the copy of X_jj read by phase 2
  auto diag = [&](int j) {
    factor_diag_tile(td, tx, bad_flag);
    double* Gjj = gtile(G, ldg, j, j);
    double* Ujj = gtile(U, ldg, j, j);
    double* Xjj = j > 0 ? gtile(U, ldg, j, j - 1) : nullptr;
    for (int e = threadIdx.x; e < NB * NB; e += kThreads) {
      const int r = e >> 6, c = e & 63;
      Gjj[(int64_t)r * ldg + c] = (c <= r) ? td[r * LDT + c] : 0.0;
      Ujj[(int64_t)r * ldg + c] = tx[c * LDT + r];
      if (Xjj) Xjj[(int64_t)r * ldg + c] = tx[r * LDT + c];
    }
    __syncthreads();
  };
  // ta holds C_ij (i > j): L_ij = C_ij L_jj^{-T} = C_ij X_jj^T
  auto panel = [&](int i, int j) {
    Acc o;
    acc_zero(o);
    tile_mma(o, ta, tx);
    double* Gij = gtile(G, ldg, i, j);
    acc_for_each(o, [&](int r, int c, double v) { Gij[(int64_t)r * ldg + c] = v; });
    __syncthreads();
  };

  // Phase 1, block column 0 (no updates)
  load_tile(td, G, ldg, false);
  __syncthreads();
  diag(0);
  for (int i = 1; i < nt; ++i) {
    load_tile(ta, gtile(G, ldg, i, 0), ldg, false);
    __syncthreads();
    panel(i, 0);
  }
  // Phase 1, block columns 1 .. nt-1
  chain_pipeline(ItChol{G, ldg, nt, 1, 1, 0}, ldg, ta, tb, [&](const ItChol& it, const Acc& c) {
    const double* Gij = gtile(G, ldg, it.i, it.j);
    double* dst = it.i == it.j ? td : ta;
    acc_for_each(c, [&](int r, int cc, double v) { dst[r * LDT + cc] = Gij[(int64_t)r * ldg + cc] - v; });
    __syncthreads();
    if (it.i == it.j) diag(it.j);
    else panel(it.i, it.j);
  });
  // Phase 2: U_ji = -S_ji U_ii = -S_ji X_ii^T
  chain_pipeline(ItInv{U, G, ldg, nt, 0, 1, 0}, ldg, ta, tb, [&](const ItInv& it, const Acc& c) {
    acc_for_each(c, [&](int r, int cc, double v) { ta[r * LDT + cc] = v; });
    load_tile(tb, gtile(U, ldg, it.i, it.i - 1), ldg, false);
    __syncthreads();
    Acc o;
    acc_zero(o);
    tile_mma(o, ta, tb);
    double* Uji = gtile(U, ldg, it.j, it.i);
    acc_for_each(o, [&](int r, int cc, double v) { Uji[(int64_t)r * ldg + cc] = -v; });
    __syncthreads();
  });
  // Phase 3: G^{-1} = U U^T, tile (i, j) and its transpose
  chain_pipeline(ItLauum{U, ldg, nt, 0, 0, 0}, ldg, ta, tb, [&](const ItLauum& it, const Acc& c) {
    double* Gij = gtile(G, ldg, it.i, it.j);
    double* Gji = gtile(G, ldg, it.j, it.i);
    const bool off = it.j != it.i;
    acc_for_each(c, [&](int r, int cc, double v) {
      Gij[(int64_t)r * ldg + cc] = v;
      if (off) Gji[(int64_t)cc * ldg + r] = v;
    });
    __syncthreads();
  });
}

template <typename ASV>
__global__ __launch_bounds__(kThreads) void k_chol_inverse(double* __restrict__ Gall,
                                                           double* __restrict__ Uall, int64_t ldg,
                                                           int32_t tau, int32_t kind,
                                                           const ASV* __restrict__ ASall,
                                                           int64_t ldas, int64_t m,
                                                           const int32_t* __restrict__ members_all,
                                                           const int32_t* __restrict__ offs_all,
                                                           int32_t* __restrict__ status,
                                                           const int32_t* __restrict__ done) {
  extern __shared__ __align__(16) double lds[];
  double* ta = lds;                  // [64][65]
  double* tb = lds + NB * LDT;       // [64][65]
  double* td = lds + 2 * NB * LDT;   // [64][65]
  double* tx = lds + 3 * NB * LDT;   // [64][65]
  __shared__ int bad;
  if (*done) return;
  const int tid = threadIdx.x;
  const int64_t slot = blockIdx.x;
  double* G = Gall + slot * ldg * ldg;
  double* U = Uall + slot * ldg * ldg;
  const int32_t* offs = offs_all + slot * (tau + 1);
  if (tid == 0) bad = 0;

  // Phase 0: assemble G (subsample: rows C of AS), padding and empty buckets.
  if (kind == kSubsample) {
    const int32_t* members = members_all + slot * tau;
    const ASV* AS = ASall + slot * m * ldas;
    for (int64_t e = tid; e < (int64_t)tau * tau; e += kThreads) {
      const int64_t c = e / tau, cc = e % tau;
      G[c * ldg + cc] = (double)AS[(int64_t)members[c] * ldas + cc];
    }
  }
  for (int64_t e = tid; e < ldg * ldg; e += kThreads) {
    const int64_t r = e / ldg, c = e % ldg;
    if (r >= tau || c >= tau) G[e] = (r == c) ? 1.0 : 0.0;
  }
  __syncthreads();
  if (kind != kSubsample) {
    for (int bkt = tid; bkt < tau; bkt += kThreads)
      if (offs[bkt + 1] == offs[bkt]) G[(int64_t)bkt * ldg + bkt] = 1.0;
  }
  __syncthreads();

  factor_invert(G, U, ldg, ta, tb, td, tx, &bad);
  if (tid == 0) status[slot] = bad;
}


// Grouped form (batched solves): job = one (problem, lambda) pair sharing the
// problem's product B S = Z (Z^T S) (no lambda term), so that
// S^T A(lambda) S = S^T B S + lambda S^T S. Subsample: rows C of B S plus lambda I;
// count: G0 = S^T B S plus lambda diag(bucket sizes) (S^T S for a count sketch), the
// diagonal of an empty bucket set to 1. Persistent grid striding over the jobs.
__global__ __launch_bounds__(kThreads) void k_chol_tab(const CholJob* __restrict__ jobs, int32_t njobs) {
  extern __shared__ __align__(16) double lds[];
  double* ta = lds;
  double* tb = lds + NB * LDT;
  double* td = lds + 2 * NB * LDT;
  double* tx = lds + 3 * NB * LDT;
  __shared__ int bad;
  const int tid = threadIdx.x;
  for (int32_t t = blockIdx.x; t < njobs; t += gridDim.x) {
    const CholJob& j = jobs[t];
    if (*j.done) continue;  // uniform across the workgroup
    double* G = j.G;
    const int64_t ldg = j.ldg;
    const int tau = j.tau;
    if (tid == 0) bad = 0;
    for (int64_t e = tid; e < ldg * ldg; e += kThreads) {
      const int64_t r = e / ldg, c = e % ldg;
      double v;
      if (r >= tau || c >= tau) {
        v = (r == c) ? 1.0 : 0.0;
      } else if (j.kind == kSubsample) {
        v = j.BS[(int64_t)j.members[r] * j.ldas + c];
        if (r == c) v += j.lam;
      } else {
        v = j.G0[r * ldg + c];
        if (r == c) {
          const int cnt = j.offs[r + 1] - j.offs[r];
          v = cnt == 0 ? 1.0 : v + j.lam * (double)cnt;
        }
      }
      G[e] = v;
    }
    __syncthreads();
    factor_invert(G, j.U, ldg, ta, tb, td, tx, &bad);
    if (tid == 0 && bad) *j.status = 1;  // sticky until the host clears it
    __syncthreads();
  }
}

template <typename ASV>
hipError_t chol_launch(double* G, double* W, int64_t ldg, int32_t tau, int32_t nslots, int32_t kind,
                       const ASV* AS, int64_t ldas, int64_t m, const int32_t* members,
                       const int32_t* offs, int32_t* status, const int32_t* done, hipStream_t s) {
  if (ldg % NB != 0) return hipErrorInvalidValue;
  const size_t bytes = sizeof(double) * 4 * NB * LDT;
  hipError_t e = hipFuncSetAttribute((const void*)k_chol_inverse<ASV>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_chol_inverse<ASV>, dim3(nslots), dim3(kThreads), bytes, s, G, W, ldg, tau,
                     kind, AS, ldas, m, members, offs, status, done);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_chol_inverse(double* G, double* W, int64_t ldg, int32_t tau, int32_t nslots,
                               int32_t kind, const void* AS, int32_t as_f32, int64_t ldas, int64_t m,
                               const int32_t* members, const int32_t* offs, int32_t* status,
                               const int32_t* done, hipStream_t s) {
  if (as_f32)
    return chol_launch<float>(G, W, ldg, tau, nslots, kind, (const float*)AS, ldas, m, members, offs,
                              status, done, s);
  return chol_launch<double>(G, W, ldg, tau, nslots, kind, (const double*)AS, ldas, m, members, offs,
                             status, done, s);
}

hipError_t launch_chol_tab(const CholJob* jobs, int32_t njobs, int32_t grid, hipStream_t s) {
  if (njobs <= 0) return hipSuccess;
  grid = grid < 1 ? 1 : (grid > njobs ? njobs : grid);
  const size_t bytes = sizeof(double) * 4 * NB * LDT;
  hipError_t e = hipFuncSetAttribute((const void*)k_chol_tab, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)bytes);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_chol_tab, dim3(grid), dim3(kThreads), bytes, s, jobs, njobs);
  return hipGetLastError();
}

}  // namespace rs
