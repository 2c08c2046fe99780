// Internal declarations shared by the HIP translation units of librs.so.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>

#include "../../include/rs.h"

namespace rs {

// ---------------------------------------------------------------------------
// Sketch representation on the device (one per lookahead slot).
//
// Every sketch kind is stored bucket-major:
//   offs[tau + 1]   column (bucket) b of S holds members[offs[b] .. offs[b+1])
//   members[nsel]   coordinate indices carrying a nonzero of S
//   hmap[m]         per coordinate: -1 if its row of S is zero, else
//                   2 * bucket + (1 if the nonzero is -1)
// Subsample: bucket c holds exactly coordinate C[c] (C ascending), sign +1.
// Count: every coordinate is a member; members ordered by (bucket, index).
// SubCount: the s kept coordinates; bucket b holds ranks [b k, (b+1) k).
// ---------------------------------------------------------------------------
enum SketchKind : int32_t { kSubsample = 0, kCount = 1, kSubcount = 2, kWeighted = 3, kGaussian = 4, kSrht = 5 };
// kGaussian, kSrht: dense S (m x ldas per slot, row-major); for kSrht the selection of C runs
// as a subsample over m' = 2^ceil(log2 m) coordinates (its hmap and keys are m' long per slot).
// kWeighted: a subsample whose coordinates are the tau smallest (u_j / q_j, j) for a
// proposal q (u_j uniform from the tag-4 stream); stored exactly like a subsample.

// Philox4x64-10 stream tags (counter word 2).
constexpr uint64_t kTagSubsample = 1, kTagCount = 2, kTagSubcount = 3, kTagWeighted = 4, kTagGaussian = 6,
                   kTagSrht = 7;

struct SketchArgs {
  int32_t kind;
  int64_t m;
  int32_t tau;
  int32_t sub_k;       // SubCount sum size
  int64_t nsel;        // members per sketch: tau, m or k * tau
  uint64_t seed, pid;  // Philox key
  int64_t k0;          // iteration of slot 0
  int32_t nslots;      // sketches drawn by this launch
  int32_t* hmap;       // [nslots][m]
  int32_t* members;    // [nslots][nsel]
  int32_t* offs;       // [nslots][tau + 1]
  uint64_t* keys;      // [nslots][m] scratch
  int32_t* err;        // device error word (set nonzero on an internal limit)
  const int32_t* done; // skip all work when *done != 0
  const int64_t* kdev; // when set, slot 0 draws iteration *kdev (read on the device)
  const float* q;      // kWeighted: proposal q[m] (> 0)
  const int32_t* q_ok; // kWeighted: 0 -> q unusable, draw a uniform subset instead
};

// Device-side solve state shared by the per-iteration kernels.
struct DevFlags {
  int32_t done;      // 1 once ||r^k|| / ||r^0|| <= tol was seen
  int32_t err;       // first internal error code seen by a kernel
  int64_t k_done;    // iteration at which `done` was set
  double r0norm;     // ||r^0||
};

// What the host reads after a lookahead batch, gathered by one kernel into host memory:
// the flags, the error word, ||r^{k-1}|| / ||r^0|| of the tracked residual and the
// factorisation status of the batch's sketches (status[nb], allocated with the report).
struct BatchReport {
  DevFlags flags;
  int32_t err;
  int32_t nb;
  double rel;
  int32_t status[1];
};
inline size_t batch_report_bytes(int32_t nmax) { return sizeof(BatchReport) + sizeof(int32_t) * nmax; }
hipError_t launch_batch_report(const DevFlags* flags, const int32_t* err, const double* hist, int64_t k,
                               const int32_t* status, int32_t nb, BatchReport* out, hipStream_t s);

// ---------------------------------------------------------------------------
// Launchers (host functions defined in the .hip files).
// ---------------------------------------------------------------------------
hipError_t launch_sketch(const SketchArgs& a, hipStream_t s);
// Grouped draw: one sketch per entry of a device table of arguments (all of one kind;
// lds_bytes = the maximum of sketch_lds_bytes over the entries).
size_t sketch_lds_bytes(int32_t kind, int32_t tau, int64_t nsel);
hipError_t launch_sketch_tab(const SketchArgs* tab, int32_t count, int32_t kind, size_t lds_bytes,
                             hipStream_t s);

// AS[slot][j][c] (row stride ldas) = sum_k Z[j][k] * Z[C_slot[c]][k] + lam * [j == C_slot[c]],
// FP64 MFMA.
// Dense sketches and general FP64 products (k_dense_sketch.hip).
struct GemmF64Args {
  const double* A;   // A(i, k) = a_trans ? A[k lda + i] : A[i lda + k]
  int64_t lda, sA;   // row stride, slot stride
  const double* B;   // B(k, j) = B[k ldb + j]
  int64_t ldb, sB;
  double* C;         // C[i ldc + j] = sum_k A(i, k) B(k, j) (+ lam E[i lde + j] when E)
  int64_t ldc, sC;
  const double* E;
  int64_t lde, sE;
  double lam;
  int64_t M, N, Kd;
  const int32_t* done;  // skip all work when *done != 0 (may be null)
};
hipError_t launch_gemm_f64(const GemmF64Args& g, bool a_trans, int32_t nslots, hipStream_t s);
hipError_t launch_sketch_gauss(double* S, int64_t m, int32_t tau, int64_t ldas, uint64_t seed, uint64_t pid,
                               int64_t k0, int32_t nslots, int32_t* offs, const int32_t* done, hipStream_t s);
hipError_t launch_srht_fill(double* S, int64_t m, int32_t tau, int64_t ldas, const int32_t* members, uint64_t seed,
                            uint64_t pid, int64_t k0, int64_t mpad, int32_t nslots, const int32_t* done,
                            hipStream_t s);
// The SRHT by its fast transform, for m' = mpad <= srht_fast_max_mpad() (LDS-resident butterflies):
// OUT(j, c) = sum_{i < m} S_ic Y[i][j] for j < ncols, c < tau, where S_ic = d_i (-1)^popcount(i & C_c)
// / sqrt(tau m'), C = members[slot] (ascending in [0, m')) and the signs d_i are read back from the
// slot's explicit S (S[slot] m x lds, slot stride sS). Stored at OUT[j ldo + c] (trans_out 0) or
// OUT[c ldo + j]; Y and OUT have slot strides sY and sO.
int64_t srht_fast_max_mpad();
hipError_t launch_srht_apply(const double* Y, int64_t ldy, int64_t sY, int64_t m, int64_t ncols, int64_t mpad,
                             const double* S, int64_t lds, int64_t sS, const int32_t* members, int32_t tau,
                             double* OUT, int64_t ldo, int64_t sO, int32_t trans_out, int32_t nslots,
                             const int32_t* done, hipStream_t s);
// S[slot] (m x ldas) from a sparse sketch's bucket codes (hmap, m per slot).
hipError_t launch_sketch_densify(double* S, const int32_t* hmap, int64_t m, int64_t ldas, int32_t nslots,
                                 const int32_t* done, hipStream_t s);
int32_t rho_dense_blocks();
// rho = S^T r with part (rho_dense_blocks() x tau doubles) as scratch.
hipError_t launch_rho_dense(const double* S, int64_t ldas, int32_t tau, int64_t m, const double* r, double* part,
                            double* rho, const DevFlags* flags, hipStream_t s);
hipError_t launch_update_dense(const double* AS, const double* S, int64_t ldas, int32_t tau, const double* delta,
                               int64_t m, const double* x, double* x_prev_out, const double* r, double* r_prev_out,
                               double gamma, double beta, double* partials, int32_t npart, const DevFlags* flags,
                               hipStream_t s);

// lam_kernel != 0: Z is a symmetric kernel matrix (K == m) and the shift is lambda Z[:, C].
hipError_t launch_as_dense_f64(const double* Z, int64_t ldz, int64_t m, int64_t K,
                               const int32_t* members, int32_t tau, int64_t ldas, int32_t nslots,
                               double lam, int32_t lam_kernel, double* AS, const int32_t* done,
                               hipStream_t s);
// Gaussian kernel matrix of n points (P: n x d row-major FP64) into Kout (n x n, row stride ldk).
hipError_t launch_rbf_gram(const double* P, int64_t n, int64_t d, double sigma, double* Kout, int64_t ldk,
                           hipStream_t s);

// Grouped dense products (batched solves): job = one sketch of one problem,
// AS (m x tau, row stride ldas) = Z Z[C,:]^T + lam I_C; tiles = (job, row tile, column tile)
// of 64 x 64. tk = 16 or 32 (K panel depth); grid = workgroups striding over the tiles.
struct DenseJob {
  const double* Z;
  int64_t ldz, m, K;
  const int32_t* members;
  int32_t tau;
  int64_t ldas;
  double lam;
  double* AS;
  const int32_t* done;
};
struct DenseTile {
  int32_t job, tm, tn;
};
hipError_t launch_as_dense_f64_tab(const DenseJob* jobs, const DenseTile* tiles, int32_t ntiles,
                                   int32_t tk, int32_t grid, hipStream_t s);
// Batched mixed precision: BS = Z Z[C, :]^T from a BF16 copy of Z (m x kpad, row stride ldz,
// zero padded; kpad a multiple of 64), FP32 accumulation, stored in FP64 (m x tau, row stride
// ldas); tiles of bf16_tile_rows() x bf16_tile_cols().
struct DenseBf16Job {
  const uint16_t* Z;
  int64_t ldz, m, kpad;
  const int32_t* members;
  int32_t tau;
  int64_t ldas;
  double* BS;
  const int32_t* done;
};
hipError_t launch_as_dense_bf16_tab(const DenseBf16Job* jobs, const DenseTile* tiles, int32_t ntiles,
                                    hipStream_t s);
int32_t bf16_tile_rows();
int32_t bf16_tile_cols();

// Count / SubCount products from CSR(Z) (m rows) and CSR(Z^T) (nnz entries), values FP32 or
// FP64: AS[slot] (m x tau, row stride ldas) and, for member rows,
// G[slot][b][:] = sum_{j in b} sign_j AS[j][:]. tbuf holds nslots * sparse_t_bytes(...) bytes.
size_t sparse_t_bytes(int32_t vals_f32, int64_t nnz);
// T[slot][q] = (bucket of column zt_col[q], signed value) for every entry q of CSR(Z^T).
hipError_t launch_build_t(const int32_t* zt_col, const void* zt_val, int32_t vals_f32, int64_t nnz,
                          const int32_t* hmap, int64_t m, int32_t nslots, void* tbuf,
                          const int32_t* done, hipStream_t s);
hipError_t launch_as_sparse(const int64_t* zr_ptr, const int32_t* zr_col, const void* zr_val,
                            const int64_t* zt_ptr, const int32_t* zt_col, const void* zt_val,
                            int32_t vals_f32, int64_t nnz, int64_t m, int32_t tau, int64_t ldas,
                            int32_t nslots, int32_t kind, double lam, const int32_t* hmap,
                            const int32_t* members, const int32_t* offs, int64_t nsel, void* tbuf,
                            double* AS, double* G, int64_t ldg, const int32_t* done, hipStream_t s);

// Count / SubCount products through the rows of A0 = Z Z^T (formed once): pairs of the
// sparse product (host count from the row pointers of Z^T), A0 as CSR with FP64 values,
// then per batch of sketches AS (row-major, several sketches per workgroup) and G.
int64_t zzt_pairs(const int64_t* zt_ptr_host, int64_t K);
hipError_t build_zzt(const int64_t* zt_ptr, const int32_t* zt_col, const void* zt_val, int32_t vals_f32,
                     int64_t K, int64_t m, int64_t npairs, int64_t** a_ptr, int32_t** a_col, double** a_val,
                     int64_t* a_nnz, hipStream_t s);
// AS (m x ldas per slot) from the rows of A0 = Z Z^T; bucket sums in FP64, stored as FP64 or,
// when as_f32, rounded to FP32 (mixed precision).
hipError_t launch_as_arows(const int64_t* a_ptr, const int32_t* a_col, const double* a_val, int64_t m,
                           int32_t tau, int64_t ldas, int32_t nslots, double lam, const int32_t* hmap, void* AS,
                           int32_t as_f32, const int32_t* done, hipStream_t s);
// G = S^T AS from the member rows of AS (FP64 or FP32 when as_f32), summed in FP64.
hipError_t launch_g_from_as(const void* AS, int32_t as_f32, int64_t m, int32_t tau, int64_t ldas, int32_t nslots,
                            const int32_t* hmap, const int32_t* members, const int32_t* offs, int64_t nsel,
                            double* G, int64_t ldg, const int32_t* done, hipStream_t s);
// Mixed precision on CSR data: r = Z (Z^T x) + lambda x - b and rp from xp, in FP64 from CSR(Z)
// (m rows) and CSR(Z^T) (K rows); u holds 2 K doubles, t 2 m doubles, partials
// refresh_csr_partials(m) doubles; ||r|| / ||r^0|| is recorded at k in hist and true_hist and
// the stop test applied (flags->done).
int64_t refresh_csr_partials(int64_t m);
hipError_t launch_refresh_csr(const int64_t* zr_ptr, const int32_t* zr_col, const void* zr_val,
                              const int64_t* zt_ptr, const int32_t* zt_col, const void* zt_val, int32_t vals_f32,
                              int64_t m, int64_t K, const double* x, const double* xp, const double* b, double lam,
                              double* r, double* rp, double* u, double* t, double* partials, DevFlags* flags,
                              double* hist, double* true_hist, int64_t k, double tol, hipStream_t s);
// ||r|| / ||r^0|| from partial sums of squares (n of them, summed in order) into hist[k] and
// true_hist[k], with the stop test.
hipError_t launch_refresh_norm(const double* partials, int32_t n, DevFlags* flags, double* hist, double* true_hist,
                               int64_t k, double tol, hipStream_t s);

// Grouped count-sketch products (batched solves; CSR values held in FP64): per job,
// T = Z^T S into tbuf (nnz * sparse_entry_bytes_f64() bytes), then AS (m x tau) and
// G = S^T AS for the (job, bucket) pairs in items[2 * nitems].
struct SparseJob {
  const int64_t* zr_ptr;
  const int32_t* zr_col;
  const double* zr_val;
  const int64_t* zt_ptr;
  const int32_t* zt_col;
  const double* zt_val;
  int64_t nnz, m;
  int32_t tau;
  int64_t ldas;
  double lam;
  const int32_t* hmap;
  const int32_t* members;
  const int32_t* offs;
  int64_t nsel;
  void* tbuf;
  double* AS;
  double* G;
  int64_t ldg;
  const int32_t* done;
};
size_t sparse_entry_bytes_f64();
hipError_t launch_sparse_tab(const SparseJob* jobs, int32_t njobs, const int32_t* items,
                             int32_t nitems, int32_t max_tau, int32_t grid, hipStream_t s);

// Ginv[slot] = (S^T A S)^{-1} (padded ldg x ldg, identity on empty buckets and padding).
// AS is FP64, or FP32 when as_f32 (mixed precision).
hipError_t launch_chol_inverse(double* G, double* W, int64_t ldg, int32_t tau, int32_t nslots,
                               int32_t kind, const void* AS, int32_t as_f32, int64_t ldas, int64_t m,
                               const int32_t* members, const int32_t* offs, int32_t* status,
                               const int32_t* done, hipStream_t s);

// Grouped factorisation and inverse (batched solves): G (ldg x ldg) <- (S^T A(lam) S)^{-1}
// assembled from the lambda-free product B S (subsample: rows C of BS, row stride ldas)
// or from G0 = S^T B S (count), U: ldg x ldg scratch, *status <- 1 on a bad pivot.
struct CholJob {
  double* G;
  double* U;
  int64_t ldg;
  int32_t tau;
  int32_t kind;
  const double* BS;
  int64_t ldas;
  const int32_t* members;
  const int32_t* offs;
  const double* G0;
  double lam;
  int32_t* status;
  const int32_t* done;
};
hipError_t launch_chol_tab(const CholJob* jobs, int32_t njobs, int32_t grid, hipStream_t s);

// Same result computed by a sequence of launches in which every 64 x 64 tile of every
// sketch is a workgroup (for batches with few sketches or large tau). X holds
// nslots * chol_multi_x_bytes(ldg) bytes of scratch.
size_t chol_multi_x_bytes(int64_t ldg);
hipError_t launch_chol_multi(double* G, double* U, double* X, int64_t ldg, int32_t tau,
                             int32_t nslots, int32_t kind, const void* AS, int32_t as_f32,
                             int64_t ldas, int64_t m, const int32_t* members, const int32_t* offs,
                             int32_t* status, const int32_t* done, hipStream_t s);

// Mixed precision (dense subsample): BF16 copy of Z (ld multiple of 64, zero padded)
// and FP32 copy (ld = K), from src viewed row-major rows_s x cols_s (trans: Z = src^T).
hipError_t launch_cast_bf16(const void* src, int32_t src_is_f32, int64_t rows_s, int64_t cols_s,
                            int64_t lds, int32_t trans, uint16_t* dst, int64_t ldd, float* dst32,
                            int64_t ldd32, hipStream_t s);
// AS[slot] (FP32, row stride ldas) = Zbf Zbf[C_slot,:]^T + lambda I_C on BF16 MFMA.
// lam_kernel != 0: kernel ridge, the shift is lam Zk[C_c][row] (the FP64 symmetric kernel matrix)
// instead of lam I_C.
// ws (may be NULL): FP32 workspace of ws_floats; when the launch has fewer tiles than compute
// units it is split over K (bf16_split_factor(...) splits, each summed into ws, then added in
// order), which needs split * nslots * m * ldas floats.
hipError_t launch_as_dense_bf16(const uint16_t* Zbf, int64_t ldz, int64_t m, int64_t kpad,
                                const int32_t* members, int32_t tau, int64_t ldas, int32_t nslots,
                                double lam, const double* Zk, int64_t ldk, int32_t lam_kernel, float* AS,
                                const int32_t* done, hipStream_t s, float* ws = nullptr, int64_t ws_floats = 0);
int32_t bf16_split_factor(int64_t m, int64_t kpad, int32_t tau, int32_t nslots);
// FP64 recomputation r = Z (Z^T x) + lambda x - b (and rp from xp) from the FP32 copy;
// records ||r|| / ||r^0|| at k and applies the stop test.
int64_t refresh_partials(int64_t m);
int64_t refresh_upart_doubles(int64_t m, int64_t K);
// AS[slot][row][c] = A[row][members[slot][c]] from a formed A (m x m, row stride lda, FP32 when
// f32 else FP64; AS in the same type), members with row stride nsel.
hipError_t launch_gram_gather(const void* A, int32_t f32, int64_t lda, int64_t m, const int32_t* members,
                              int64_t nsel, int32_t tau, int64_t ldas, int32_t nslots, void* AS,
                              const int32_t* done, hipStream_t s);
// r = Z (Z^T x) + lambda x - b in FP64 from FP32 or FP64 data (lam_u: lambda Z^T x, kernel
// ridge with Z = K symmetric); r2 holds 2 m doubles (r twice), no state or flag is touched.
hipError_t launch_true_residual(const void* Zr, int32_t z_f32, int64_t ldz, int64_t m, int64_t K, const double* x,
                                const double* b, double lam, int32_t lam_u, double* u, double* upart, double* r2,
                                double* partials, const int32_t* zero, hipStream_t s);
// FP64 residuals r = Z (Z^T x) + lam x - b from the FP32 (z_f32) or FP64 copy of Z; lam_u != 0:
// kernel ridge, r = Z (Z^T x) + lam (Z^T x) - b.
hipError_t launch_refresh(const void* Zr, int32_t z_f32, int64_t ldz, int64_t m, int64_t K, const double* x,
                          const double* xp, const double* b, double lam, int32_t lam_u, double* r, double* rp,
                          double* u, double* upart, double* partials, DevFlags* flags, double* hist,
                          double* true_hist, int64_t k, double tol, const int32_t* done,
                          hipStream_t s);
hipError_t launch_gemv_rows_f32(const float* Z, int64_t ldz, int64_t m, int64_t K, const double* v,
                                double* out, hipStream_t s);  // out = Z v, FP64 accumulation
hipError_t launch_gemv_cols_f32(const float* Z, int64_t ldz, int64_t m, int64_t K, const double* v,
                                double* out, hipStream_t s);  // out = Z^T v, FP64 accumulation

// ---------------------------------------------------------------------------
// Batched solves: per-problem device state and the lock-step iteration kernels.
// ---------------------------------------------------------------------------
struct BState {
  int64_t m;
  int32_t J, nrhs, nlam, tau;
  int64_t ldg, ldas;
  const double* BS;       // m x ldas, lambda-free product Z (Z^T S), zero beyond tau
  const double* Ginv;     // nlam x ldg x ldg inverses of S^T A(lambda_l) S
  const int32_t* hmap;    // sketch (bucket-major, one slot)
  const int32_t* members;
  const int32_t* offs;
  const double* lam;      // [nlam]
  const double* b;        // m x nrhs row-major
  double* x[2];           // m x J row-major; buffer (k & 1) holds iterate k
  double* r[2];
  double* rho;            // J x ldg
  double* delta;          // J x ldg (zero beyond tau)
  double* partials;       // ntiles x J
  int32_t ntiles;         // 64-row tiles
  double* r0n;            // [J] ||r^0||
  int64_t* stop_k;        // [J] -1 while running, else the iteration whose iterate is kept
  double* rel;            // [J] last ||r^k|| / ||r^0||
  int32_t* inactive;      // problem finished (read as the `done` word of its launches)
  int64_t cap;            // iteration cap
  int64_t* iters;         // iterations performed when the problem finished
  // mixed precision (dense problems with BF16 products): after the update of iteration k with
  // (k + 1) % refresh == 0, R^{k+1} and R^k are recomputed in FP64 from Z (FP64, m x K, row
  // stride ldz) through Uref (2 x K x J), and a slot may stop only at such an iteration
  int32_t refresh;        // 0: FP64 products, tracked residuals only
  const double* Z;
  int64_t ldz, K;
  double* Uref;
};
struct BGlobal {
  int64_t k;     // shared iteration counter
  int32_t done;  // every problem finished
  int32_t pad;
};
hipError_t launch_binit(const BState* S, int32_t nprob, BGlobal* g, hipStream_t s);
hipError_t launch_brho(const BState* S, const int32_t* items, int32_t nitems, const BGlobal* g,
                       int32_t grid, hipStream_t s);
hipError_t launch_bdelta(const BState* S, const int32_t* items, int32_t nitems, int32_t grid,
                         hipStream_t s);
hipError_t launch_bupdate(const BState* S, const int32_t* items, int32_t nitems, const BGlobal* g,
                          const double* betas, const double* gammas, int32_t grid, hipStream_t s);
hipError_t launch_bfinal(const BState* S, int32_t nprob, BGlobal* g, double tol, hipStream_t s);
// FP64 refresh of the residuals of the mixed-precision problems (no-op at other iterations):
// uitems (p, 64-column tile of K, h) for U_h = Z^T X_h, ritems (p, 64-row tile, h) for
// R_h = Z U_h + X_h diag(lambda) - B, with h = 0 for X^{k+1} and 1 for X^k.
hipError_t launch_brefresh(const BState* S, const int32_t* uitems, int32_t nu, const int32_t* ritems, int32_t nr,
                           const BGlobal* g, int32_t grid, hipStream_t s);
hipError_t launch_bcol(const double* src, int64_t m, int64_t src_ld, int64_t src_col, double* dst,
                       int64_t dst_ld, int64_t dst_col, hipStream_t s);

// ---------------------------------------------------------------------------
// Learned proposal (features, MLP, proposal, traces, training).
// ---------------------------------------------------------------------------
constexpr int kMlpFeatures = 6;
constexpr int kMlpHidden = 128;
constexpr int kMlpParams = kMlpFeatures * kMlpHidden + kMlpHidden + kMlpHidden * kMlpHidden +
                           kMlpHidden + kMlpHidden + 1;
constexpr uint64_t kTagMlpInit = 5;

struct TraceArgs {
  int64_t m;
  int32_t tau;
  int64_t k, k0;               // iteration recorded; iteration of slot 0 of its batch
  int32_t slot;                // k - k0
  const int32_t* members;      // sketch of iteration k (subsample: bucket b = coordinate C_b)
  const int32_t* hmap_batch;   // [slots][m] sketches of the batch
  const int32_t* last;         // latest iteration < k0 holding each coordinate (-1: none)
  const double* a;             // A_jj
  const double* stats;         // mean log a, std log a, sum a
  const double* r;             // r^k
  const double* rp;            // r^{k-1}
  const double* delta;         // delta_k
  const double* rho;           // rho_k = S_k^T r^k
  float* F;                    // [capacity][tau][6]
  float* credits;              // [capacity][tau]
  int32_t* count;              // records written (may exceed capacity: extra ones dropped)
  int32_t capacity;
  const DevFlags* flags;
};

hipError_t launch_adiag(const void* Z, int32_t z_f32, int64_t ldz, int64_t m, int64_t K, double lam,
                        double* a, double* stats, hipStream_t s);
hipError_t launch_lstats(const double* a, int64_t m, double* stats, hipStream_t s);
hipError_t launch_features(const double* a, const double* stats, const double* r, const double* rp,
                           const int32_t* last, int64_t m, int64_t k, double* log_rn, float* F,
                           const int32_t* done, hipStream_t s);
hipError_t launch_trace(const TraceArgs& t, hipStream_t s);
hipError_t launch_mark_last(const int32_t* members, int32_t tau, int32_t nslots, int64_t k0,
                            int32_t* last, hipStream_t s);
hipError_t launch_proposal(const float* s_in, int64_t m, float eps, float* q, int32_t* ok,
                           const int32_t* done, hipStream_t s);
hipError_t launch_diag_q(const double* a, const double* stats, int64_t m, float* q, hipStream_t s);
hipError_t launch_mlp_init(float* p, uint64_t seed, hipStream_t s);
hipError_t launch_mlp_fwd(const float* P, const float* F, const int32_t* rec, int32_t tau, int64_t rows,
                          float* out, const int32_t* done, hipStream_t s);
int32_t mlp_bwd_blocks(int64_t rows);
// One training evaluation over nrec records (rows = nrec * tau): scores into s_buf, dL/ds
// into ds_buf, per-record losses into loss[nrec], gradient (mean over records) into grad.
// partial holds mlp_bwd_blocks(rows) * kMlpParams floats.
hipError_t launch_mlp_step(const float* P, const float* F, const float* credits, const int32_t* rec,
                           int32_t tau, int32_t nrec, float* s_buf, float* ds_buf, double* loss,
                           float* partial, float* grad, hipStream_t s);
hipError_t launch_adam(float* P, float* m1, float* m2, const float* g, int64_t t, double lr, double b1,
                       double b2, double eps, hipStream_t s);

// Solve-state kernels.
int32_t update_partials(int64_t m, int32_t tau);  // partial sums written by k_update
hipError_t launch_init_state(const double* b, double* x0, double* x1, double* r0, double* r1,
                             int64_t m, double* partials, int32_t npart, DevFlags* flags,
                             double* hist, hipStream_t s);
hipError_t launch_rho(const double* r, const int32_t* hmap, const int32_t* members,
                      const int32_t* offs, int32_t tau, double* rho, const DevFlags* flags,
                      hipStream_t s);
hipError_t launch_delta(const double* rho, int32_t tau, const double* Ginv, int64_t ldg,
                        const double* partials, int32_t npart, DevFlags* flags, double* hist,
                        int64_t k, double tol, double* delta, hipStream_t s);
hipError_t launch_update(const void* AS, int32_t as_f32, int64_t ldas, int32_t tau, const double* delta,
                         const int32_t* hmap, int64_t m, const double* x, double* x_prev_out,
                         const double* r, double* r_prev_out, double gamma, double beta,
                         double* partials, int32_t npart, const int32_t* hmap_next,
                         const int32_t* members_next, const int32_t* offs_next,
                         int32_t next_covers_all, double* rho_next, const DevFlags* flags,
                         hipStream_t s);
// Accelerated method (Alg. 3), FP64 AS: w' = z - S delta and r_w' = r_z - AS delta into
// w_out / rw_out; v, r_v updated in place; r_z = alpha r_v' + (1 - alpha) r_w' written;
// the norm partials are those of r_v' and rho_next is taken from r_z'.
hipError_t launch_update_accel(const double* AS, int64_t ldas, int32_t tau, const double* delta,
                               const int32_t* hmap, int64_t m, const double* w, double* w_out, const double* rw,
                               double* rw_out, double* v, double* rv, double* rz, double alpha, double beta,
                               double gamma, double* partials, int32_t npart, const int32_t* hmap_next,
                               const int32_t* members_next, const int32_t* offs_next, int32_t next_covers_all,
                               double* rho_next, const DevFlags* flags, hipStream_t s);
// v = 0, r_v = r_z = r0 (m entries).
hipError_t launch_init_accel(const double* r0, double* v, double* rv, double* rz, int64_t m, hipStream_t s);
hipError_t launch_finalize(const double* partials, int32_t npart, DevFlags* flags, double* hist,
                           int64_t k, double tol, hipStream_t s);

// Setup helpers.
hipError_t launch_transpose_to_f64(const void* src, int32_t src_is_f32, int64_t rows, int64_t cols,
                                   int64_t lds, double* dst, int64_t ldd, hipStream_t s);
hipError_t launch_copy_to_f64(const void* src, int32_t src_is_f32, int64_t rows, int64_t cols,
                              int64_t lds, double* dst, int64_t ldd, hipStream_t s);
hipError_t launch_gemv_rows(const double* Z, int64_t ldz, int64_t m, int64_t K, const double* v,
                            double* out, hipStream_t s);           // out = Z v
hipError_t launch_gemv_cols(const double* Z, int64_t ldz, int64_t m, int64_t K, const double* v,
                            double* out, hipStream_t s);           // out = Z^T v
hipError_t launch_spmv_csr(const int64_t* ptr, const int32_t* col, const void* val, int32_t vals_f32,
                           int64_t rows, const double* v, double* out, hipStream_t s);
hipError_t launch_vec_to_f64(const void* src, int32_t src_is_f32, int64_t n, double* dst,
                             hipStream_t s);
// CSR (rows x cols) -> CSR of the transpose, values kept in their precision. Stable:
// entries of each output row appear in increasing source-row order.
hipError_t csr_transpose(const int64_t* ptr, const int32_t* col, const void* val, int32_t vals_f32,
                         int64_t rows, int64_t cols, int64_t nnz, int64_t* tptr, int32_t* tcol,
                         void* tval, hipStream_t s);

}  // namespace rs
