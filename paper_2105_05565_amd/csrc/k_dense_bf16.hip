// Mixed-precision products for the subsample sketch (BF16 inputs, FP32 accumulation)
// and the FP64 residual refresh.
//
// AS = Z Z[C,:]^T + lambda I_C is formed from a BF16 copy of Z on MFMA
// (v_mfma_f32_32x32x16_bf16) with FP32 accumulation; several lookahead sketches share
// the first operand, so one launch contracts Z against the gathered rows of every
// slot (N = slots * tau columns). The tracked residual drifts with the BF16 rounding
// of AS; every R iterations it is recomputed in FP64 from an FP32 copy of Z
// (r = Z (Z^T x) + lambda x - b for x^k and x^{k-1}).
//
// GEMM tiling (gfx950): 256 x 256 output tile per workgroup, 8 waves each owning a
// 64 x 128 sub-tile (2 x 4 MFMA blocks of 32 x 32), K staged 64 at a time through two
// LDS stages filled by direct-to-LDS loads (XOR-swizzled 128-byte rows). Tiles are
// ordered so that the workgroups one XCD runs together share row strips of Z and
// gathered column strips (workgroups are dispatched to the 8 XCDs round-robin).
#include <algorithm>

#include "dev_common.h"
#include "rs_internal.h"

namespace rs {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr int kBN = 256;  // gathered columns (sketch coordinates) per output tile
constexpr int kXcds = 8;
constexpr int kGroupRows = 4;  // row tiles per tile group (XCD-local reuse of Z strips)

__device__ __forceinline__ uint16_t bf16_bits_rne(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));
  const uint32_t lsb = (u >> 16) & 1u;
  u += 0x7fffu + lsb;
  return (uint16_t)(u >> 16);
}

// dst (rows x ldd, BF16 bits, zero padded) and dst32 (FP32, ld ldd32) from src viewed
// row-major (rows_s x cols_s, ld lds); trans: dst[c][r] = src[r][c].
__global__ void k_cast_bf16(const void* __restrict__ src, int32_t is_f32, int64_t rows_s,
                            int64_t cols_s, int64_t lds, int32_t trans, uint16_t* __restrict__ dst,
                            int64_t ldd, float* __restrict__ dst32, int64_t ldd32) {
  __shared__ float tile[32][33];
  const int64_t r0 = (int64_t)blockIdx.y * 32, c0 = (int64_t)blockIdx.x * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  for (int yy = ty; yy < 32; yy += 8) {
    const int64_t r = r0 + yy, c = c0 + tx;
    float v = 0.0f;
    if (r < rows_s && c < cols_s)
      v = is_f32 ? ((const float*)src)[r * lds + c] : (float)((const double*)src)[r * lds + c];
    tile[yy][tx] = v;
  }
  __syncthreads();
  for (int yy = ty; yy < 32; yy += 8) {
    int64_t orow, ocol;
    float v;
    if (trans) {
      orow = c0 + yy;
      ocol = r0 + tx;
      v = tile[tx][yy];
    } else {
      orow = r0 + yy;
      ocol = c0 + tx;
      v = tile[yy][tx];
    }
    const int64_t out_rows = trans ? cols_s : rows_s;
    if (orow < out_rows && ocol < ldd) {
      dst[orow * ldd + ocol] = bf16_bits_rne(v);
      if (ocol < ldd32) dst32[orow * ldd32 + ocol] = v;
    }
  }
}

struct GemmArgs {
  const uint16_t* Z;   // m x ldz BF16 bits, zero padded to a multiple of 64
  int64_t ldz, m, kpad;
  const int32_t* members;  // [slots][tau]
  int32_t tau;
  int64_t ntot;  // slots * tau
  int64_t ldas;
  double lam;
  const double* Zk;    // kernel ridge (lam_kernel): the FP64 symmetric kernel matrix, row stride ldk
  int64_t ldk;
  int32_t lam_kernel;  // 1: the shift is lam K[C_c][row] (= lam K[row][C_c]) instead of lam I_C
  float* AS;  // [slot][m][ldas]
  int32_t n_row_tiles, n_col_tiles;
  const int32_t* done;
};

// Tile t of the grouped order: groups of kGroupRows row tiles, column by column within a
// group, so that a run of consecutive tiles covers a compact block of row and column strips.
__device__ __forceinline__ void tile_of_index(const GemmArgs& a, int t, int* rt, int* ct) {
  const int group = t / (kGroupRows * a.n_col_tiles);
  const int rows_in_group = min(kGroupRows, a.n_row_tiles - group * kGroupRows);
  const int idx = t - group * kGroupRows * a.n_col_tiles;
  *rt = group * kGroupRows + idx % rows_in_group;
  *ct = idx / rows_in_group;
}

// Workgroup bid (XCD bid % 8) -> its tile: each XCD takes a run of consecutive tiles.
__device__ __forceinline__ void tile_of_block(const GemmArgs& a, int bid, int* rt, int* ct) {
  const int ntiles = a.n_row_tiles * a.n_col_tiles;
  const int per = (ntiles + kXcds - 1) / kXcds;
  const int t = (bid % kXcds) * per + bid / kXcds;
  if (t >= ntiles) {
    *rt = -1;
    return;
  }
  tile_of_index(a, t, rt, ct);
}

// AS for a batch of subsample sketches: operand tiles move from global memory straight into
// LDS (global_load_lds_dwordx4, 16 bytes per lane, no register staging), 64 deep in K per
// stage, so that every row of a stage is one whole 128-byte line: the load path into a CU
// moves about a third more bytes per cycle with whole-line requests than with the half lines
// of 32-deep stages, and that rate, not the LDS reads, is what feeds the matrix cores. Two
// stages of 64 KB: one is multiplied while the next one loads.
constexpr int kDmaBK = 64;                    // K elements per stage
constexpr int kDmaRowBytes = kDmaBK * 2;      // 128

typedef __attribute__((address_space(3))) void lds_void_t;

// s_waitcnt immediate (gfx9 layout): vmcnt <= n, expcnt not waited on, lgkmcnt <= lgkm
constexpr int waitcnt_imm(int n, int lgkm) { return (n & 15) | ((n >> 4) << 14) | (7 << 4) | (lgkm << 8); }

// One BM x 256 output tile of Z Z[C, :]^T (BM = 32 WAVES) accumulated in FP32 by a workgroup
// of WAVES waves; each wave owns 64 x 128 as 2 x 4 MFMA blocks of 32 x 32, fed by
// v_mfma_f32_32x32x16_bf16. Output rows row0 .. row0 + BM - 1 of Z (rows >= m load row 0), output
// columns n0 .. n0 + 255 (column n takes row members[n] of Z; n >= ntot loads row 0). Operand rows
// are staged 64 deep in K through two LDS stages of ROWS x 128 bytes (dsm). A DMA instruction
// fills 1 KB: 8 rows of 128 bytes, lane L taking row L / 8 and 16-byte slot L % 8; the slot
// holding a row's logical 16-byte segment t is t ^ ((row / 2) % 8), which puts the 16 rows read
// by a quarter wave on distinct banks. The K steps are accumulated in ascending order, 16 at a
// time. Ends with every DMA of the workgroup landed and a barrier (dsm may be reused).
template <int WAVES>
__device__ __forceinline__ void bf16_tile(const uint16_t* __restrict__ Z, int64_t ldz, int64_t m, int64_t kpad,
                                          const int32_t* __restrict__ members, int64_t ntot, int64_t row0,
                                          int64_t n0, unsigned char* dsm, f32x16 (&acc)[2][4]) {
  constexpr int BM = 32 * WAVES, ROWS = BM + kBN;
  constexpr int NQ = ROWS / (8 * WAVES);             // DMA instructions per wave and stage
  constexpr int STAGE_BYTES = ROWS * kDmaRowBytes;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;

  // this lane's source rows for the wave's NQ DMA instructions of a stage
  const unsigned char* src[NQ];
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    const int r = (wave * NQ + q) * 8 + (lane >> 3);  // tile row 0 .. ROWS - 1
    int64_t g;
    if (r < BM) {
      g = row0 + r;
      if (g >= m) g = 0;
    } else {
      const int64_t n = n0 + r - BM;
      g = n < ntot ? (int64_t)members[n] : 0;
    }
    const int t = (lane & 7) ^ ((r >> 1) & 7);  // logical 16-byte segment stored in this slot
    src[q] = reinterpret_cast<const unsigned char*>(Z + g * ldz) + t * 16;
  }
  const int64_t nk = kpad / kDmaBK;
  auto stage = [&](int64_t kt) { return dsm + (size_t)(kt & 1) * STAGE_BYTES; };
  auto issue = [&](int64_t kt) {
    const int64_t ktl = kt < nk ? kt : nk - 1;  // past the end: reload the last stage
    unsigned char* dst = stage(kt);
#pragma unroll
    for (int q = 0; q < NQ; ++q)
      __builtin_amdgcn_global_load_lds((const void*)(src[q] + ktl * kDmaRowBytes),
                                       (lds_void_t*)(dst + (wave * NQ + q) * 1024), 16, 0, 0);
  };

  const int wr = (wave >> 1) * 64, wc = (wave & 1) * 128;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int v = 0; v < 16; ++v) acc[i][j][v] = 0.0f;
  const int l32 = lane & 31, khi = lane >> 5;

  // fragments of K step s (16 deep) of a stage: rows of the A strip (2) and of the gathered B
  // strip (4); lanes 0-31 take K 16 s .. 16 s + 7 of their row, lanes 32-63 the next eight
  auto read_frags = [&](const unsigned char* st, int s, bf16x8 (&av)[2], bf16x8 (&bv)[4]) {
    const int t = 2 * s + khi;
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      const int r = wr + i * 32 + l32;
      av[i] = *reinterpret_cast<const bf16x8*>(st + r * kDmaRowBytes + ((t ^ ((r >> 1) & 7)) << 4));
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int r = BM + wc + j * 32 + l32;
      bv[j] = *reinterpret_cast<const bf16x8*>(st + r * kDmaRowBytes + ((t ^ ((r >> 1) & 7)) << 4));
    }
  };
  auto mma = [&](const bf16x8 (&av)[2], const bf16x8 (&bv)[4]) {
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j)
        acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av[i], bv[j], acc[i][j], 0, 0, 0);
  };

  // The fragments of each step are read while the MFMAs of the step before run. Stage kt + 1
  // loads while stage kt is multiplied; the barrier that hands it over comes after this
  // wave's reads of stage kt have landed, so that the refill issued right after it (into
  // stage kt's buffer) cannot overtake them.
  issue(0);
  __builtin_amdgcn_s_waitcnt(waitcnt_imm(0, 15));  // stage 0 landed (own share), then every wave
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_sched_barrier(0);
  issue(1);
  bf16x8 a0[2], b0[4], a1[2], b1[4];
  read_frags(stage(0), 0, a0, b0);
  __builtin_amdgcn_s_waitcnt(waitcnt_imm(63, 0));
  __builtin_amdgcn_sched_barrier(0);
  // The body is the same on the last pass (its refill reloads the last stage and its reads of
  // stage nk go unused), so that no branch joins in-flight LDS reads of different ages.
  for (int64_t kt = 0; kt < nk; ++kt) {
    const unsigned char* st = stage(kt);
    read_frags(st, 1, a1, b1);
    __builtin_amdgcn_sched_barrier(0);
    mma(a0, b0);
    __builtin_amdgcn_sched_barrier(0);
    __builtin_amdgcn_s_waitcnt(waitcnt_imm(63, 0));
    read_frags(st, 2, a0, b0);
    __builtin_amdgcn_sched_barrier(0);
    mma(a1, b1);
    __builtin_amdgcn_sched_barrier(0);
    __builtin_amdgcn_s_waitcnt(waitcnt_imm(63, 0));
    read_frags(st, 3, a1, b1);
    __builtin_amdgcn_sched_barrier(0);
    mma(a0, b0);
    __builtin_amdgcn_sched_barrier(0);
    // step 3's fragments read and stage kt + 1 landed (own share), then every wave
    __builtin_amdgcn_s_waitcnt(waitcnt_imm(0, 0));
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_sched_barrier(0);
    issue(kt + 2);  // into stage kt's buffer, which no wave reads any more
    read_frags(stage(kt + 1), 0, a0, b0);
    __builtin_amdgcn_sched_barrier(0);
    mma(a1, b1);
    __builtin_amdgcn_sched_barrier(0);
    __builtin_amdgcn_s_waitcnt(waitcnt_imm(63, 0));
  }
  // no DMA may still be writing this workgroup's LDS when the tile ends
  __builtin_amdgcn_s_waitcnt(waitcnt_imm(0, 15));
  __builtin_amdgcn_s_barrier();
}

// Visit the tile's results: f(row in tile, column in tile, value), the 32x32x16 result layout
// (lane l, element v -> row 8 (v / 4) + 4 (l / 32) + v % 4, column l % 32) under the wave's block.
template <class F>
__device__ __forceinline__ void bf16_tile_for_each(const f32x16 (&acc)[2][4], F f) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wr = (wave >> 1) * 64, wc = (wave & 1) * 128;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int v = 0; v < 16; ++v)
        f(wr + i * 32 + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3), wc + j * 32 + (lane & 31), acc[i][j][v]);
}

// AS for a batch of subsample sketches: one BM x 256 output tile per workgroup (bf16_tile),
// AS[slot][row][c] = (Z Z[C_slot, :]^T)[row][c] + lam I_C (or lam K[row][C_c] for kernel ridge),
// stored in FP32.
template <int WAVES>
__global__ __launch_bounds__(WAVES * 64, 1) void k_as_dense_bf16(GemmArgs a) {
  constexpr int BM = 32 * WAVES;
  extern __shared__ __align__(16) unsigned char dsm[];  // [2][BM + 256][128 B]
  if (*a.done) return;
  int rt, ct;
  tile_of_block(a, blockIdx.x, &rt, &ct);
  if (rt < 0) return;
  const int64_t row0 = (int64_t)rt * BM, n0 = (int64_t)ct * kBN;
  f32x16 acc[2][4];
  bf16_tile<WAVES>(a.Z, a.ldz, a.m, a.kpad, a.members, a.ntot, row0, n0, dsm, acc);
  bf16_tile_for_each(acc, [&](int tr, int tc, float v) {
    const int64_t row = row0 + tr, n = n0 + tc;
    if (row < a.m && n < a.ntot) {
      const int64_t slot = n / a.tau, c = n % a.tau;
      const int64_t cj = a.members[n];
      float val = v;
      if (a.lam_kernel)
        val = (float)((double)val + a.lam * a.Zk[cj * a.ldk + row]);
      else if (row == cj)
        val = (float)((double)val + a.lam);
      a.AS[(slot * a.m + row) * a.ldas + c] = val;
    }
  });
}

// The shift of AS's entry (row, column n of the launch): lam I_C, or lam K[C_c][row] for kernel ridge.
__device__ __forceinline__ float shifted(const GemmArgs& a, int64_t row, int64_t n, float v) {
  const int64_t cj = a.members[n];
  if (a.lam_kernel) return (float)((double)v + a.lam * a.Zk[cj * a.ldk + row]);
  if (row == cj) return (float)((double)v + a.lam);
  return v;
}

// Split-K form for launches with fewer tiles than compute units: workgroup (s, tile) sums the
// K stages [s q, (s + 1) q) of its tile (q stages per split) into ws[s][slot][row][c] (FP32, no
// shift); k_splitk_reduce then adds the splits in order and the shift.
template <int WAVES>
__global__ __launch_bounds__(WAVES * 64, 1) void k_as_dense_bf16_split(GemmArgs a, int64_t stages_per_split,
                                                                       float* __restrict__ ws) {
  constexpr int BM = 32 * WAVES;
  extern __shared__ __align__(16) unsigned char dsm[];
  if (*a.done) return;
  // XCD x (= blockIdx.x % 8) takes a run of consecutive (split, tile) pairs in split-major
  // order: its workgroups share one K range and the strips of a compact block of tiles, so
  // each XCD's L2 fetches every operand strip it needs once (a K range's tiles spread over
  // all XCDs would have each XCD fetch every strip of that range for a few tiles)
  const int ntiles = a.n_row_tiles * a.n_col_tiles;
  const int64_t nk = a.kpad / kDmaBK;
  const int nsplit = (int)((nk + stages_per_split - 1) / stages_per_split);
  const int total = ntiles * nsplit, per = (total + kXcds - 1) / kXcds;
  const int pair = (blockIdx.x % kXcds) * per + blockIdx.x / kXcds;
  if (pair >= total) return;
  const int sp = pair / ntiles;
  int rt, ct;
  tile_of_index(a, pair % ntiles, &rt, &ct);
  const int64_t k0 = (int64_t)sp * stages_per_split, k1 = min(nk, k0 + stages_per_split);  // k1 > k0 (host)
  const int64_t row0 = (int64_t)rt * BM, n0 = (int64_t)ct * kBN;
  f32x16 acc[2][4];
  bf16_tile<WAVES>(a.Z + k0 * kDmaBK, a.ldz, a.m, (k1 - k0) * kDmaBK, a.members, a.ntot, row0, n0, dsm, acc);
  const int64_t nslots = a.ntot / a.tau;
  float* wsp = ws + (int64_t)sp * nslots * a.m * a.ldas;
  bf16_tile_for_each(acc, [&](int tr, int tc, float v) {
    const int64_t row = row0 + tr, n = n0 + tc;
    if (row < a.m && n < a.ntot) wsp[((n / a.tau) * a.m + row) * a.ldas + n % a.tau] = v;
  });
}

__global__ __launch_bounds__(256) void k_splitk_reduce(GemmArgs a, int32_t nsplit, const float* __restrict__ ws) {
  if (*a.done) return;
  const int64_t total = a.ntot * a.m;  // (slot, row, c) with c < tau
  const int64_t plane = a.ntot / a.tau * a.m * a.ldas;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < total; e += (int64_t)gridDim.x * 256) {
    const int64_t c = e % a.tau, sr = e / a.tau, row = sr % a.m, slot = sr / a.m;
    const int64_t idx = (slot * a.m + row) * a.ldas + c;
    float v = 0.0f;
    for (int sp = 0; sp < nsplit; ++sp) v += ws[sp * plane + idx];
    a.AS[idx] = shifted(a, row, slot * a.tau + c, v);
  }
}

// Grouped form for the batched solver: one workgroup per entry of a ragged table of (job,
// 256-row tile, 256-column tile) entries, ordered by decreasing contraction length so that the
// dispatcher hands the longest tiles out first; job p's lambda-free product BS = Z Z[C, :]^T
// (m x tau, row stride ldas) is stored in FP64 from the FP32 accumulators.
template <int WAVES>
__global__ __launch_bounds__(WAVES * 64, 1) void k_as_dense_bf16_tab(const DenseBf16Job* __restrict__ jobs,
                                                                     const DenseTile* __restrict__ tiles) {
  constexpr int BM = 32 * WAVES;
  extern __shared__ __align__(16) unsigned char dsm[];
  const DenseTile tl = tiles[blockIdx.x];
  const DenseBf16Job j = jobs[tl.job];
  if (*j.done) return;  // uniform across the workgroup
  const int64_t row0 = (int64_t)tl.tm * BM, n0 = (int64_t)tl.tn * kBN;
  f32x16 acc[2][4];
  bf16_tile<WAVES>(j.Z, j.ldz, j.m, j.kpad, j.members, j.tau, row0, n0, dsm, acc);
  const int64_t m = j.m, tau = j.tau, ldas = j.ldas;
  double* BS = j.BS;
  bf16_tile_for_each(acc, [&](int tr, int tc, float v) {
    const int64_t row = row0 + tr, c = n0 + tc;
    if (row < m && c < tau) BS[row * ldas + c] = (double)v;
  });
}

// Shape of the product launch: waves per workgroup (two LDS stages).
constexpr int kGemmWaves = 8;

constexpr int kRefreshSplit = 32;  // row ranges of Z summed separately in Z^T x

// V consecutive entries of a row of Z as FP64 (V = 4 FP32 or 2 FP64 entries: one 16-byte load;
// V = 1: one entry).
template <typename T, int V>
__device__ __forceinline__ void load_row_vec(const T* __restrict__ p, double (&out)[V]) {
  if constexpr (V == 1) {
    out[0] = (double)p[0];
  } else if constexpr (sizeof(T) == 4) {
    static_assert(V == 4, "FP32 rows load four entries");
    const float4 v = *reinterpret_cast<const float4*>(p);
    out[0] = v.x;
    out[1] = v.y;
    out[2] = v.z;
    out[3] = v.w;
  } else {
    static_assert(V == 2, "FP64 rows load two entries");
    const double2 v = *reinterpret_cast<const double2*>(p);
    out[0] = v.x;
    out[1] = v.y;
  }
}

// upart[js][k][0..1] = sum_{j in range js} Z[j][k] * (x[j], xp[j]) in FP64 (FP32 or FP64 data),
// rows in ascending order. Each thread owns V consecutive columns (ldz a multiple of V, so
// its loads stay inside the row) and keeps four rows of loads in flight.
template <typename T, int V>
__global__ __launch_bounds__(256) void k_gemv_t_pair(const T* __restrict__ Z, int64_t ldz, int64_t m, int64_t K,
                                                     const double* __restrict__ x, const double* __restrict__ xp,
                                                     double* __restrict__ upart, const int32_t* __restrict__ done) {
  if (*done) return;
  const int64_t k0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) * V;
  if (k0 >= K) return;
  const int64_t per = (m + kRefreshSplit - 1) / kRefreshSplit;
  const int64_t j0 = min(m, (int64_t)blockIdx.y * per), j1 = min(m, j0 + per);
  double s0[V], s1[V];
#pragma unroll
  for (int e = 0; e < V; ++e) s0[e] = s1[e] = 0.0;
  const T* zp = Z + k0;
  int64_t j = j0;
  for (; j + 4 <= j1; j += 4) {
    double z[4][V];
#pragma unroll
    for (int u = 0; u < 4; ++u) load_row_vec<T, V>(zp + (j + u) * ldz, z[u]);
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const double xj = x[j + u], xpj = xp[j + u];
#pragma unroll
      for (int e = 0; e < V; ++e) {
        s0[e] += z[u][e] * xj;
        s1[e] += z[u][e] * xpj;
      }
    }
  }
  for (; j < j1; ++j) {
    double z[V];
    load_row_vec<T, V>(zp + j * ldz, z);
    const double xj = x[j], xpj = xp[j];
#pragma unroll
    for (int e = 0; e < V; ++e) {
      s0[e] += z[e] * xj;
      s1[e] += z[e] * xpj;
    }
  }
#pragma unroll
  for (int e = 0; e < V; ++e)
    if (k0 + e < K) {
      double* out = upart + ((int64_t)blockIdx.y * K + k0 + e) * 2;
      out[0] = s0[e];
      out[1] = s1[e];
    }
}

// u[k] = sum over the row ranges in order.
__global__ void k_sum_upart(const double* __restrict__ upart, int64_t K, double* __restrict__ u,
                            const int32_t* __restrict__ done) {
  if (*done) return;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= 2 * K) return;
  double s = 0.0;
  for (int js = 0; js < kRefreshSplit; ++js) s += upart[(int64_t)js * 2 * K + i];
  u[i] = s;
}

// The product Z u of the refresh in column chunks: part[c][j][0..1] = sum over the columns k
// of chunk c of Z[j][k] (u[k][0], u[k][1]). A workgroup (8 waves, 8 rows each) stages the
// chunk of u in LDS once for its 64 rows; lane l takes columns l V, l V + 64 V, ... of the
// chunk (ldz a multiple of V; columns past K meet zeros of the staged u).
constexpr int kNChunk = 2048;          // columns per chunk
constexpr int kNRowsPerWave = 8;
constexpr int kNWaves = 8;
constexpr int kNRows = kNRowsPerWave * kNWaves;  // rows per workgroup

template <typename T, int V>
__global__ __launch_bounds__(kNWaves * 64) void k_gemv_n_pair_part(
    const T* __restrict__ Z, int64_t ldz, int64_t m, int64_t K, const double* __restrict__ u,
    double* __restrict__ part, const int32_t* __restrict__ done) {
  __shared__ double2 us[kNChunk];
  if (*done) return;
  const int64_t kc0 = (int64_t)blockIdx.y * kNChunk;
  const int kn = (int)min((int64_t)kNChunk, K - kc0);
  for (int i = threadIdx.x; i < kNChunk; i += kNWaves * 64)
    us[i] = i < kn ? reinterpret_cast<const double2*>(u)[kc0 + i] : make_double2(0.0, 0.0);
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t r0 = (int64_t)blockIdx.x * kNRows + wave * kNRowsPerWave;
  const T* zr[kNRowsPerWave];
#pragma unroll
  for (int r = 0; r < kNRowsPerWave; ++r) zr[r] = Z + min(r0 + r, m - 1) * ldz + kc0;  // rows past m: discarded
  double s0[kNRowsPerWave], s1[kNRowsPerWave];
#pragma unroll
  for (int r = 0; r < kNRowsPerWave; ++r) s0[r] = s1[r] = 0.0;
  for (int kk = lane * V; kk < kn; kk += 64 * V) {
    double u0[V], u1[V];
#pragma unroll
    for (int e = 0; e < V; ++e) {
      const double2 w = us[kk + e];
      u0[e] = w.x;
      u1[e] = w.y;
    }
#pragma unroll
    for (int r = 0; r < kNRowsPerWave; ++r) {
      double z[V];
      load_row_vec<T, V>(zr[r] + kk, z);
#pragma unroll
      for (int e = 0; e < V; ++e) {
        s0[r] += z[e] * u0[e];
        s1[r] += z[e] * u1[e];
      }
    }
  }
#pragma unroll
  for (int r = 0; r < kNRowsPerWave; ++r) {
    const double t0 = wave_sum(s0[r]), t1 = wave_sum(s1[r]);
    if (lane == 0 && r0 + r < m) {
      double* out = part + ((int64_t)blockIdx.y * m + r0 + r) * 2;
      out[0] = t0;
      out[1] = t1;
    }
  }
}

// r[j] = sum_c part[c][j][0] + lam x[j] - b[j] and rp[j] = sum_c part[c][j][1] + lam xp[j] - b[j]
// (chunks in order); kernel ridge (lam_u): the shift is lam u[j] = lam (K x)[j]. Partial sums
// of ||r||^2 per workgroup.
__global__ __launch_bounds__(256) void k_gemv_n_finish(const double* __restrict__ part, int32_t nchunk, int64_t m,
                                                       const double* __restrict__ u, const double* __restrict__ x,
                                                       const double* __restrict__ xp, const double* __restrict__ b,
                                                       double lam, int32_t lam_u, double* __restrict__ r,
                                                       double* __restrict__ rp, double* __restrict__ partials,
                                                       const int32_t* __restrict__ done) {
  __shared__ double scratch[16];
  if (*done) return;
  const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
  double ss = 0.0;
  if (j < m) {
    double s0 = 0.0, s1 = 0.0;
    for (int c = 0; c < nchunk; ++c) {
      const double2 w = reinterpret_cast<const double2*>(part)[(int64_t)c * m + j];
      s0 += w.x;
      s1 += w.y;
    }
    const double sx = lam_u ? u[2 * j] : x[j], sxp = lam_u ? u[2 * j + 1] : xp[j];
    const double rn = s0 + lam * sx - b[j];
    r[j] = rn;
    rp[j] = s1 + lam * sxp - b[j];
    ss = rn * rn;
  }
  ss = block_sum(ss, scratch);
  if (threadIdx.x == 0) partials[blockIdx.x] = ss;
}

__global__ void k_gemv_rows_f32(const float* __restrict__ Z, int64_t ldz, int64_t m, int64_t K,
                                const double* __restrict__ v, double* __restrict__ out) {
  const int lane = threadIdx.x & 63;
  const int64_t row = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (row >= m) return;
  double s = 0.0;
  for (int64_t k = lane; k < K; k += 64) s += (double)Z[row * ldz + k] * v[k];
  s = wave_sum(s);
  if (lane == 0) out[row] = s;
}

// out[k] = sum_j Z[j][k] v[j] in FP64 (FP32 data), one thread per column.
__global__ void k_gemv_cols_f32(const float* __restrict__ Z, int64_t ldz, int64_t m, int64_t K,
                                const double* __restrict__ v, double* __restrict__ out) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= K) return;
  double s = 0.0;
  for (int64_t j = 0; j < m; ++j) s += (double)Z[j * ldz + k] * v[j];
  out[k] = s;
}

// ||r||^2 from the refresh partials; records it and applies the stop test.
__global__ __launch_bounds__(256) void k_refresh_norm(const double* __restrict__ partials, int32_t n,
                                                      DevFlags* __restrict__ flags,
                                                      double* __restrict__ hist,
                                                      double* __restrict__ true_hist, int64_t k,
                                                      double tol) {
  __shared__ double scratch[16];
  if (flags->done) return;
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) s += partials[i];
  s = block_sum(s, scratch);
  if (threadIdx.x == 0) {
    const double rel = sqrt(s) / flags->r0norm;
    hist[k] = rel;
    true_hist[k] = rel;
    if (rel <= tol) {
      flags->k_done = k;
      flags->done = 1;
    }
  }
}

}  // namespace

hipError_t launch_cast_bf16(const void* src, int32_t src_is_f32, int64_t rows_s, int64_t cols_s,
                            int64_t lds, int32_t trans, uint16_t* dst, int64_t ldd, float* dst32,
                            int64_t ldd32, hipStream_t s) {
  const int64_t out_rows = trans ? cols_s : rows_s;
  // grid covers the padded output columns as well (zero fill)
  const int64_t gx = trans ? (out_rows + 31) / 32 : (ldd + 31) / 32;
  const int64_t gy = trans ? (ldd + 31) / 32 : (out_rows + 31) / 32;
  dim3 grid((unsigned)gx, (unsigned)gy);
  hipLaunchKernelGGL(k_cast_bf16, grid, dim3(256), 0, s, src, src_is_f32, rows_s, cols_s, lds, trans,
                     dst, ldd, dst32, ldd32);
  return hipGetLastError();
}

namespace {

int device_cus() {
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0) {
    (void)hipGetLastError();
    return 256;
  }
  return cus;
}

}  // namespace

int32_t bf16_split_factor(int64_t m, int64_t kpad, int32_t tau, int32_t nslots) {
  constexpr int BM = 32 * kGemmWaves;
  const int64_t ntiles = ((m + BM - 1) / BM) * (((int64_t)nslots * tau + kBN - 1) / kBN);
  const int64_t nk = kpad / kDmaBK;
  const int cus = device_cus();
  int32_t split = 1;
  // split while the tiles leave compute units idle and every split keeps >= 32 stages
  while (ntiles * split * 2 <= cus && nk >= (int64_t)split * 2 * 32) split *= 2;
  return split;
}

hipError_t launch_as_dense_bf16(const uint16_t* Zbf, int64_t ldz, int64_t m, int64_t kpad,
                                const int32_t* members, int32_t tau, int64_t ldas, int32_t nslots,
                                double lam, const double* Zk, int64_t ldk, int32_t lam_kernel, float* AS,
                                const int32_t* done, hipStream_t s, float* ws, int64_t ws_floats) {
  if (kpad % kDmaBK != 0 || ldz % 8 != 0) return hipErrorInvalidValue;
  if (lam_kernel && (!Zk || ldk < m)) return hipErrorInvalidValue;
  GemmArgs a;
  a.Z = Zbf;
  a.ldz = ldz;
  a.m = m;
  a.kpad = kpad;
  a.members = members;
  a.tau = tau;
  a.ntot = (int64_t)nslots * tau;
  a.ldas = ldas;
  a.lam = lam;
  a.Zk = Zk;
  a.ldk = ldk;
  a.lam_kernel = lam_kernel;
  a.AS = AS;
  constexpr int BM = 32 * kGemmWaves;
  a.n_row_tiles = (int32_t)((m + BM - 1) / BM);
  a.n_col_tiles = (int32_t)((a.ntot + kBN - 1) / kBN);
  a.done = done;
  const int ntiles = a.n_row_tiles * a.n_col_tiles;
  const int per = (ntiles + kXcds - 1) / kXcds;
  const size_t bytes = (size_t)2 * (BM + kBN) * kDmaRowBytes;
  const int32_t split = ws ? bf16_split_factor(m, kpad, tau, nslots) : 1;
  if (split > 1 && (int64_t)split * nslots * m * ldas <= ws_floats) {
    const int64_t nk = kpad / kDmaBK;
    const int64_t q = (nk + split - 1) / split;
    if ((split - 1) * q >= nk) return hipErrorInvalidValue;  // every split gets >= 1 stage
    auto kern = k_as_dense_bf16_split<kGemmWaves>;
    hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    if (e != hipSuccess) return e;
    const int64_t per_x = ((int64_t)ntiles * split + kXcds - 1) / kXcds;
    hipLaunchKernelGGL(kern, dim3((unsigned)(per_x * kXcds)), dim3(kGemmWaves * 64), bytes, s, a, q, ws);
    const int64_t total = a.ntot * m;
    const unsigned g = (unsigned)std::min<int64_t>((total + 255) / 256, 4096);
    hipLaunchKernelGGL(k_splitk_reduce, dim3(g), dim3(256), 0, s, a, split, ws);
    return hipGetLastError();
  }
  auto kern = k_as_dense_bf16<kGemmWaves>;
  hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(kern, dim3(per * kXcds), dim3(kGemmWaves * 64), bytes, s, a);
  return hipGetLastError();
}

namespace {

// The FP64 products of a refresh: u = Z^T (x, xp) (row ranges, then their sum in order), then
// r, rp = Z u + lam (x, xp) - b (lam_u: + lam u) with ||r||^2 partial sums. Returns the number
// of partial sums written.
hipError_t refresh_products(const void* Zr, int32_t z_f32, int64_t ldz, int64_t m, int64_t K, const double* x,
                            const double* xp, const double* b, double lam, int32_t lam_u, double* r, double* rp,
                            double* u, double* upart, double* partials, const int32_t* done, int32_t* nparts,
                            hipStream_t s) {
  if (lam_u && K != m) return hipErrorInvalidValue;
  const bool vec = z_f32 ? (ldz % 4 == 0) : (ldz % 2 == 0);
  const bool aligned = (reinterpret_cast<uintptr_t>(Zr) & 15) == 0;
  const int V = !(vec && aligned) ? 1 : (z_f32 ? 4 : 2);
  const dim3 gt((unsigned)((K + 256 * V - 1) / (256 * V)), kRefreshSplit);
  if (z_f32 && V == 4)
    hipLaunchKernelGGL((k_gemv_t_pair<float, 4>), gt, dim3(256), 0, s, (const float*)Zr, ldz, m, K, x, xp, upart, done);
  else if (z_f32)
    hipLaunchKernelGGL((k_gemv_t_pair<float, 1>), gt, dim3(256), 0, s, (const float*)Zr, ldz, m, K, x, xp, upart, done);
  else if (V == 2)
    hipLaunchKernelGGL((k_gemv_t_pair<double, 2>), gt, dim3(256), 0, s, (const double*)Zr, ldz, m, K, x, xp, upart,
                       done);
  else
    hipLaunchKernelGGL((k_gemv_t_pair<double, 1>), gt, dim3(256), 0, s, (const double*)Zr, ldz, m, K, x, xp, upart,
                       done);
  hipLaunchKernelGGL(k_sum_upart, dim3((unsigned)((2 * K + 255) / 256)), dim3(256), 0, s, upart, K, u, done);
  // the row ranges of upart have been summed into u: upart now holds the column-chunk partials
  const int64_t nchunk = (K + kNChunk - 1) / kNChunk;
  const dim3 gn((unsigned)((m + kNRows - 1) / kNRows), (unsigned)nchunk);
  if (z_f32 && V == 4)
    hipLaunchKernelGGL((k_gemv_n_pair_part<float, 4>), gn, dim3(kNWaves * 64), 0, s, (const float*)Zr, ldz, m, K, u,
                       upart, done);
  else if (z_f32)
    hipLaunchKernelGGL((k_gemv_n_pair_part<float, 1>), gn, dim3(kNWaves * 64), 0, s, (const float*)Zr, ldz, m, K, u,
                       upart, done);
  else if (V == 2)
    hipLaunchKernelGGL((k_gemv_n_pair_part<double, 2>), gn, dim3(kNWaves * 64), 0, s, (const double*)Zr, ldz, m, K,
                       u, upart, done);
  else
    hipLaunchKernelGGL((k_gemv_n_pair_part<double, 1>), gn, dim3(kNWaves * 64), 0, s, (const double*)Zr, ldz, m, K,
                       u, upart, done);
  const unsigned nb = (unsigned)((m + 255) / 256);
  hipLaunchKernelGGL(k_gemv_n_finish, dim3(nb), dim3(256), 0, s, upart, (int32_t)nchunk, m, u, x, xp, b, lam, lam_u,
                     r, rp, partials, done);
  *nparts = (int32_t)nb;
  return hipGetLastError();
}

}  // namespace

hipError_t launch_as_dense_bf16_tab(const DenseBf16Job* jobs, const DenseTile* tiles, int32_t ntiles,
                                    hipStream_t s) {
  if (ntiles <= 0) return hipSuccess;
  constexpr int BM = 32 * kGemmWaves;
  const size_t bytes = (size_t)2 * (BM + kBN) * kDmaRowBytes;
  auto kern = k_as_dense_bf16_tab<kGemmWaves>;
  hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(kern, dim3((unsigned)ntiles), dim3(kGemmWaves * 64), bytes, s, jobs, tiles);
  return hipGetLastError();
}

int32_t bf16_tile_rows() { return 32 * kGemmWaves; }
int32_t bf16_tile_cols() { return kBN; }

hipError_t launch_refresh(const void* Zr, int32_t z_f32, int64_t ldz, int64_t m, int64_t K, const double* x,
                          const double* xp, const double* b, double lam, int32_t lam_u, double* r, double* rp,
                          double* u, double* upart, double* partials, DevFlags* flags, double* hist,
                          double* true_hist, int64_t k, double tol, const int32_t* done,
                          hipStream_t s) {
  int32_t np = 0;
  hipError_t e = refresh_products(Zr, z_f32, ldz, m, K, x, xp, b, lam, lam_u, r, rp, u, upart, partials, done, &np, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_refresh_norm, dim3(1), dim3(256), 0, s, partials, np, flags, hist, true_hist, k, tol);
  return hipGetLastError();
}

hipError_t launch_refresh_norm(const double* partials, int32_t n, DevFlags* flags, double* hist, double* true_hist,
                               int64_t k, double tol, hipStream_t s) {
  hipLaunchKernelGGL(k_refresh_norm, dim3(1), dim3(256), 0, s, partials, n, flags, hist, true_hist, k, tol);
  return hipGetLastError();
}

hipError_t launch_true_residual(const void* Zr, int32_t z_f32, int64_t ldz, int64_t m, int64_t K, const double* x,
                                const double* b, double lam, int32_t lam_u, double* u, double* upart, double* r2,
                                double* partials, const int32_t* zero, hipStream_t s) {
  int32_t np = 0;
  return refresh_products(Zr, z_f32, ldz, m, K, x, x, b, lam, lam_u, r2, r2 + m, u, upart, partials, zero, &np, s);
}

// partial sums written by a refresh (at most)
int64_t refresh_partials(int64_t m) { return (m + 255) / 256; }

hipError_t launch_gemv_cols_f32(const float* Z, int64_t ldz, int64_t m, int64_t K, const double* v,
                                double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_gemv_cols_f32, dim3((unsigned)((K + 255) / 256)), dim3(256), 0, s, Z, ldz, m, K,
                     v, out);
  return hipGetLastError();
}

hipError_t launch_gemv_rows_f32(const float* Z, int64_t ldz, int64_t m, int64_t K, const double* v,
                                double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_gemv_rows_f32, dim3((unsigned)((m + 3) / 4)), dim3(256), 0, s, Z, ldz, m, K, v,
                     out);
  return hipGetLastError();
}
// the row-range partials of Z^T x, then the column-chunk partials of Z u, in one buffer
int64_t refresh_upart_doubles(int64_t m, int64_t K) {
  return std::max<int64_t>((int64_t)kRefreshSplit * 2 * K, 2 * m * ((K + kNChunk - 1) / kNChunk));
}

}  // namespace rs
