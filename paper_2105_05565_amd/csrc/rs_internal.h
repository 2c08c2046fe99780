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
enum SketchKind : int32_t { kSubsample = 0, kCount = 1, kSubcount = 2 };

// Philox4x64-10 stream tags (counter word 2).
constexpr uint64_t kTagSubsample = 1, kTagCount = 2, kTagSubcount = 3, kTagWeighted = 4;

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
};

// Device-side solve state shared by the per-iteration kernels.
struct DevFlags {
  int32_t done;      // 1 once ||r^k|| / ||r^0|| <= tol was seen
  int32_t err;       // first internal error code seen by a kernel
  int64_t k_done;    // iteration at which `done` was set
  double r0norm;     // ||r^0||
};

// ---------------------------------------------------------------------------
// Launchers (host functions defined in the .hip files).
// ---------------------------------------------------------------------------
hipError_t launch_sketch(const SketchArgs& a, hipStream_t s);

// AS[slot][j][c] (row stride ldas) = sum_k Z[j][k] * Z[C_slot[c]][k] + lam * [j == C_slot[c]],
// FP64 MFMA.
hipError_t launch_as_dense_f64(const double* Z, int64_t ldz, int64_t m, int64_t K,
                               const int32_t* members, int32_t tau, int64_t ldas, int32_t nslots,
                               double lam, double* AS, const int32_t* done, hipStream_t s);

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

// Ginv[slot] = (S^T A S)^{-1} (padded ldg x ldg, identity on empty buckets and padding).
// AS is FP64, or FP32 when as_f32 (mixed precision).
hipError_t launch_chol_inverse(double* G, double* W, int64_t ldg, int32_t tau, int32_t nslots,
                               int32_t kind, const void* AS, int32_t as_f32, int64_t ldas, int64_t m,
                               const int32_t* members, const int32_t* offs, int32_t* status,
                               const int32_t* done, hipStream_t s);

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
hipError_t launch_as_dense_bf16(const uint16_t* Zbf, int64_t ldz, int64_t m, int64_t kpad,
                                const int32_t* members, int32_t tau, int64_t ldas, int32_t nslots,
                                double lam, float* AS, const int32_t* done, hipStream_t s);
// FP64 recomputation r = Z (Z^T x) + lambda x - b (and rp from xp) from the FP32 copy;
// records ||r|| / ||r^0|| at k and applies the stop test.
int64_t refresh_partials(int64_t m);
int64_t refresh_upart_doubles(int64_t K);
hipError_t launch_refresh(const float* Z32, int64_t ldz, int64_t m, int64_t K, const double* x,
                          const double* xp, const double* b, double lam, double* r, double* rp,
                          double* u, double* upart, double* partials, DevFlags* flags, double* hist,
                          double* true_hist, int64_t k, double tol, const int32_t* done,
                          hipStream_t s);
hipError_t launch_gemv_rows_f32(const float* Z, int64_t ldz, int64_t m, int64_t K, const double* v,
                                double* out, hipStream_t s);  // out = Z v, FP64 accumulation
hipError_t launch_gemv_cols_f32(const float* Z, int64_t ldz, int64_t m, int64_t K, const double* v,
                                double* out, hipStream_t s);  // out = Z^T v, FP64 accumulation

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
