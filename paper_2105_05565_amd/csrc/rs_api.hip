// Host runtime behind the C ABI declared in include/rs.h.
//
// Solve loop (Alg. 2, eq:res_update_mom). Sketches S_k, the products AS_k and the
// factorised inverses G_k^{-1} do not depend on the iterate (S_k is an independent
// draw, Sec. 3), so they are produced for a batch of `lookahead` iterations at a
// time, spreading the tau x tau factorisations over the compute units. The serial
// part per iteration is two launches: delta_k = G_k^{-1} S_k^T r^k and the fused
// momentum update. A device flag set by the stop test turns the remaining queued
// work into no-ops, so no host synchronisation is needed inside a batch.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "momentum.h"
#include "rs_internal.h"

using namespace rs;

struct rs_handle {
  rs_options opt{};
  int form = RS_FORM_PRIMAL;
  int64_t n = 0, d = 0, m = 0, K = 0;
  double lam = 0.0;
  int64_t mom_switch = 0;  // switch index of the theoretical momentum rule
  bool kern = false;        // kernel ridge: Z holds the symmetric kernel matrix (m = K = n)
  // dense sketches (Gaussian, SRHT): padded size m' of the SRHT, S of the iterating set,
  // scratch of S^T r
  bool dense_s = false;
  int64_t mpad = 0;
  double* S = nullptr;
  double* rho_part = nullptr;
  // accelerated method (Alg. 3): v, r_v, r_z and its constants
  bool accel = false;
  double* vbuf = nullptr;
  double* rvbuf = nullptr;
  double* rzbuf = nullptr;
  double acc_alpha = 0.0, acc_beta = 0.0, acc_gamma = 0.0;
  int64_t pdim = 0;         // kernel ridge: dimension of the points
  bool sparse = false;
  int kind = kSubsample;
  int tau = 0, sub_k = 0;
  int64_t nsel = 0;
  hipStream_t stream = nullptr;

  // Z (m x K): dense row-major, or CSR of Z and of Z^T.
  double* Z = nullptr;
  int64_t ldz = 0;
  // mixed precision: BF16 copy (ld kpad, a multiple of 64) and FP32 copy (ld K)
  bool mixed = false;
  uint16_t* Zbf = nullptr;
  int64_t kpad = 0;
  float* Z32 = nullptr;
  int64_t ld32 = 0;           // row stride of Z32: K rounded up to 4 (zero padding), for 16-byte loads
  float* splitk_ws = nullptr;  // BF16 products of small batches split over K: FP32 partial sums
  int64_t splitk_floats = 0;
  double* ref_u = nullptr;
  double* ref_upart = nullptr;
  double* ref_partials = nullptr;
  double* ref_t = nullptr;  // mixed precision on CSR data: Z (Z^T x) for x^k and x^{k-1} (2 m)
  // the FP64 residual of the returned iterate, recomputed from the data at the end of a solve
  double* tr_u = nullptr;
  double* tr_upart = nullptr;
  double* tr_r = nullptr;
  double* tr_part = nullptr;
  int32_t* tr_zero = nullptr;  // a 'done' word that stays 0, so those kernels always run
  // dense route 1: A = Z Z^T + lambda I formed once (m x ldgram, FP32 in mixed precision)
  void* gram = nullptr;
  int64_t ldgram = 0;
  double* true_hist = nullptr;
  int64_t* zr_ptr = nullptr;
  int32_t* zr_col = nullptr;
  void* zr_val = nullptr;
  int64_t* zt_ptr = nullptr;
  int32_t* zt_col = nullptr;
  void* zt_val = nullptr;
  int32_t vals_f32 = 0;  // CSR values kept in the input precision
  int64_t nnz = 0;
  void* tbuf = nullptr;  // per-sketch T = Z^T S entries (sparse path, scatter route)
  bool arows = false;    // sparse path through the rows of A0 = Z Z^T
  int64_t* a_ptr = nullptr;
  int32_t* a_col = nullptr;
  double* a_val = nullptr;
  int64_t a_nnz = 0;

  double* b = nullptr;
  double* xbuf[2] = {nullptr, nullptr};
  double* rbuf[2] = {nullptr, nullptr};

  // lookahead batch
  int B = 1;
  // Buffers a batch's preparation writes and its iterations read. With the pipeline on,
  // the next batch is prepared into the other set on prep_stream while the current one
  // iterates on `stream` (ev_ready[p]: set p prepared). hmap, members, offs, AS, G and
  // status below point at the set of the latest batch.
  struct BatchSet {
    int32_t* hmap = nullptr;
    int32_t* members = nullptr;
    int32_t* offs = nullptr;
    void* AS = nullptr;
    double* G = nullptr;
    int32_t* status = nullptr;
    double* S = nullptr;  // dense sketches: S (m x ldas per slot) and T = Z^T S (K x ldas per slot)
    double* T = nullptr;
  };
  BatchSet sets[2];
  int nsets = 1;
  int cur_set = 0;
  bool pipeline = false;
  hipStream_t prep_stream = nullptr;
  hipEvent_t ev_ready[2] = {nullptr, nullptr};
  hipEvent_t ev_start = nullptr;
  hipEvent_t ev_prep_done = nullptr;  // recorded on prep_stream before a batch report
  BatchReport* rep_host = nullptr;    // mapped pinned memory written by k_batch_report
  BatchReport* rep_dev = nullptr;     // its device address
  int64_t ldg = 0;
  int64_t ldas = 0;  // row stride of AS (tau rounded up to 8)
  double* rho = nullptr;
  int32_t* hmap = nullptr;
  int32_t* members = nullptr;
  int32_t* offs = nullptr;
  uint64_t* keys = nullptr;
  void* AS = nullptr;  // FP64, or FP32 in mixed precision
  double* G = nullptr;
  double* W = nullptr;
  double* Xd = nullptr;  // inverted diagonal tiles (tiled factorisation scratch)
  int32_t* status = nullptr;
  double* delta = nullptr;
  double* partials = nullptr;
  int npart = 0;
  double* hist = nullptr;
  int64_t hist_len = 0;
  DevFlags* flags = nullptr;
  int32_t* err = nullptr;

  // profiling (rs_options.profile)
  std::vector<hipEvent_t> ev;  // pool: 2 events per timed launch of one batch
  std::vector<int> ev_cls;     // kernel class of each pair
  std::vector<int> ev_slots;   // sketches processed by each pair
  std::vector<int64_t> ev_batch;  // first iteration of the batch a preparation pair belongs to (-1: none)
  int ev_used = 0;
  rs_profile prof{};

  // learned / diagonal proposal and traces (dense subsample only)
  int sampler = RS_SAMPLER_UNIFORM;
  int trace_every = 0;
  int trace_cap = 0;
  double* adiag = nullptr;   // A_jj
  double* lstats = nullptr;  // mean log a, std log a, sum a
  double* log_rn = nullptr;
  int32_t* last = nullptr;   // latest iteration before the current batch holding each coordinate
  float* feat = nullptr;     // m x 6
  float* score = nullptr;    // m
  float* q = nullptr;        // m
  int32_t* q_ok = nullptr;
  float* params = nullptr;   // MLP parameters
  bool params_set = false;
  float* tr_F = nullptr;
  float* tr_c = nullptr;
  int32_t* tr_count = nullptr;

  int64_t k = 0;          // iterations performed
  int64_t last_early = -1000000;  // iteration of the last refresh taken on the tracked estimate
  int64_t batch_k0 = -1;  // iteration of slot 0 of the most recent batch
  int batch_n = 0;
  bool done = false;
  std::string last_error;
  std::vector<void*> allocs;
};

namespace {

thread_local std::string g_create_error;

struct Fail {
  rs_status code;
  std::string msg;
};

void check_hip(hipError_t e, const char* what) {
  if (e != hipSuccess) throw Fail{RS_EDEVICE, std::string(what) + ": " + hipGetErrorString(e)};
}

template <class T>
T* dalloc(rs_handle* h, size_t count) {
  if (count == 0) count = 1;
  void* p = nullptr;
  hipError_t e = hipMalloc(&p, sizeof(T) * count);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    throw Fail{RS_ENOMEM, "hipMalloc of " + std::to_string(sizeof(T) * count) + " bytes failed"};
  }
  h->allocs.push_back(p);
  return static_cast<T*>(p);
}

void dfree_all(rs_handle* h) {
  for (void* p : h->allocs) (void)hipFree(p);
  h->allocs.clear();
  for (hipEvent_t e : h->ev) (void)hipEventDestroy(e);
  h->ev.clear();
  for (hipEvent_t* e : {&h->ev_ready[0], &h->ev_ready[1], &h->ev_start, &h->ev_prep_done})
    if (*e) {
      (void)hipEventDestroy(*e);
      *e = nullptr;
    }
  if (h->rep_host) {
    (void)hipHostFree(h->rep_host);
    h->rep_host = nullptr;
    h->rep_dev = nullptr;
  }
  if (h->prep_stream) {
    (void)hipStreamDestroy(h->prep_stream);
    h->prep_stream = nullptr;
  }
}

// Host arithmetic below in a fixed operation order (no contraction).
#pragma clang fp contract(off)
int subcount_rule(int64_t m, int tau) {
  if (10ll * tau <= m) return 10;
  return (int)(m / tau);
}

template <class T>
T* to_device(rs_handle* h, const void* src, size_t count, int mem) {
  T* d = dalloc<T>(h, count);
  if (count) check_hip(hipMemcpyAsync(d, src, sizeof(T) * count,
                                      mem == RS_DEVICE ? hipMemcpyDeviceToDevice
                                                       : hipMemcpyHostToDevice,
                                      h->stream),
                       "upload");
  return d;
}

// Event pair around one launch when profiling: returns the pair index or -1.
int prof_begin(rs_handle* h, int cls, int slots, int level = 1, hipStream_t s = nullptr, int64_t batch = -1) {
  if (h->opt.profile == 3) {
    if (cls != RS_PROF_AS) return -1;  // products only
  } else if (h->opt.profile < level) {
    return -1;
  }
  if (2 * (h->ev_used + 1) > (int)h->ev.size()) return -1;  // pool full: leave untimed
  const int i = h->ev_used++;
  h->ev_cls[i] = cls;
  h->ev_slots[i] = slots;
  h->ev_batch[i] = batch;
  check_hip(hipEventRecord(h->ev[2 * i], s ? s : h->stream), "event");
  return i;
}

void prof_end(rs_handle* h, int i, hipStream_t s = nullptr) {
  if (i >= 0) check_hip(hipEventRecord(h->ev[2 * i + 1], s ? s : h->stream), "event");
}

// After a synchronisation: fold the recorded pairs into h->prof. The preparation of a batch
// that starts at or after drop_from (prepared ahead past the stopping iteration, so its
// kernels returned at once) is left out.
void prof_collect(rs_handle* h, int64_t drop_from = INT64_MAX) {
  for (int i = 0; i < h->ev_used; ++i) {
    if (h->ev_batch[i] >= 0 && h->ev_batch[i] >= drop_from) continue;
    float ms = 0.0f;
    check_hip(hipEventElapsedTime(&ms, h->ev[2 * i], h->ev[2 * i + 1]), "elapsed");
    h->prof.ms[h->ev_cls[i]] += ms;
    h->prof.launches[h->ev_cls[i]] += 1;
    h->prof.slots[h->ev_cls[i]] += h->ev_slots[i];
  }
  h->ev_used = 0;
}

// Mixed precision: r^k and r^{k-1} recomputed in FP64 from x^k, x^{k-1}; stop test on it.
void refresh(rs_handle* h, int64_t k) {
  const int pe = prof_begin(h, RS_PROF_REFRESH, 1, 2);
  if (h->sparse) {
    // CSR: two sparse products over the data per vector (Z^T x, then Z (Z^T x)), FP64
    check_hip(launch_refresh_csr(h->zr_ptr, h->zr_col, h->zr_val, h->zt_ptr, h->zt_col, h->zt_val, h->vals_f32,
                                 h->m, h->K, h->xbuf[k & 1], h->xbuf[(k + 1) & 1], h->b, h->lam, h->rbuf[k & 1],
                                 h->rbuf[(k + 1) & 1], h->ref_u, h->ref_t, h->ref_partials, h->flags, h->hist,
                                 h->true_hist, k, h->opt.tol, h->stream),
              "refresh (CSR)");
    prof_end(h, pe);
    return;
  }
  // kernel ridge refreshes from the FP64 kernel matrix, dense ridge from the FP32 copy of X
  const void* Zr = h->kern ? (const void*)h->Z : (const void*)h->Z32;
  const int64_t ldr = h->kern ? h->ldz : h->ld32;
  check_hip(launch_refresh(Zr, h->kern ? 0 : 1, ldr, h->m, h->K, h->xbuf[k & 1], h->xbuf[(k + 1) & 1], h->b,
                           h->lam, h->kern ? 1 : 0, h->rbuf[k & 1], h->rbuf[(k + 1) & 1], h->ref_u, h->ref_upart,
                           h->ref_partials, h->flags, h->hist, h->true_hist, k, h->opt.tol,
                           &h->flags->done, h->stream),
            "refresh");
  prof_end(h, pe);
}

// ||A x^k - b|| / ||b|| with A x^k formed from the data in FP64 (dense: Z (Z^T x) + lambda x,
// from the FP32 copy for mixed precision; kernel ridge: K (K x) + lambda K x; CSR: two
// sparse products, the last two terms added on the host), not from the recursion.
double true_rel_res(rs_handle* h) {
  const int64_t m = h->m;
  const double* x = h->xbuf[h->k & 1];
  hipStream_t s = h->stream;
  std::vector<double> r(m);
  if (h->sparse) {
    check_hip(launch_spmv_csr(h->zt_ptr, h->zt_col, h->zt_val, h->vals_f32, h->K, x, h->tr_u, s), "Z^T x");
    check_hip(launch_spmv_csr(h->zr_ptr, h->zr_col, h->zr_val, h->vals_f32, m, h->tr_u, h->tr_r, s), "Z Z^T x");
    std::vector<double> hx(m), hb(m);
    check_hip(hipMemcpyAsync(r.data(), h->tr_r, sizeof(double) * m, hipMemcpyDeviceToHost, s), "copy");
    check_hip(hipMemcpyAsync(hx.data(), x, sizeof(double) * m, hipMemcpyDeviceToHost, s), "copy");
    check_hip(hipMemcpyAsync(hb.data(), h->b, sizeof(double) * m, hipMemcpyDeviceToHost, s), "copy");
    check_hip(hipStreamSynchronize(s), "sync");
    for (int64_t j = 0; j < m; ++j) r[j] = r[j] + h->lam * hx[j] - hb[j];
  } else {
    const bool f32 = h->mixed && !h->kern;
    const void* Zr = f32 ? (const void*)h->Z32 : (const void*)h->Z;
    const int64_t ldr = f32 ? h->ld32 : h->ldz;
    check_hip(launch_true_residual(Zr, f32 ? 1 : 0, ldr, m, h->K, x, h->b, h->lam, h->kern ? 1 : 0, h->tr_u,
                                   h->tr_upart, h->tr_r, h->tr_part, h->tr_zero, s),
              "true residual");
    check_hip(hipMemcpyAsync(r.data(), h->tr_r, sizeof(double) * m, hipMemcpyDeviceToHost, s), "copy");
    check_hip(hipStreamSynchronize(s), "sync");
  }
  double ss = 0.0;
  for (int64_t j = 0; j < m; ++j) ss += r[j] * r[j];
  DevFlags f{};
  check_hip(hipMemcpy(&f, h->flags, sizeof(DevFlags), hipMemcpyDeviceToHost), "flags");
  return f.r0norm > 0.0 ? std::sqrt(ss) / f.r0norm : 0.0;
}

// Sketches k0 .. k0 + nb - 1 of a batch, their products AS, G = S^T A S and its inverse,
// written into buffer set p on stream s. Only the learned proposal reads the iterate
// (and then s is the solver's stream).
void prep_batch(rs_handle* h, int p, int64_t k0, int nb, hipStream_t s) {
  rs_handle::BatchSet& bs = h->sets[p];
  const int32_t* done = &h->flags->done;
  SketchArgs a{};
  a.kind = h->kind;
  a.m = h->m;
  a.tau = h->tau;
  a.sub_k = h->sub_k;
  a.nsel = h->nsel;
  a.seed = h->opt.seed;
  a.pid = h->opt.problem_id;
  a.k0 = k0;
  a.nslots = nb;
  a.hmap = bs.hmap;
  a.members = bs.members;
  a.offs = bs.offs;
  a.keys = h->keys;
  a.err = h->err;
  a.done = done;
  int pe = prof_begin(h, RS_PROF_SKETCH, nb, 1, s, k0);
  if (h->sampler != RS_SAMPLER_UNIFORM) {
    // coordinates drawn from the proposal q (features of r^{k0}, r^{k0-1} for the
    // learned one): the tau smallest u_j / q_j per sketch
    if (h->sampler == RS_SAMPLER_LEARNED) {
      check_hip(launch_features(h->adiag, h->lstats, h->rbuf[k0 & 1], h->rbuf[(k0 + 1) & 1], h->last, h->m,
                                k0, h->log_rn, h->feat, done, s),
                "features");
      check_hip(launch_mlp_fwd(h->params, h->feat, nullptr, 0, h->m, h->score, done, s), "scores");
      check_hip(launch_proposal(h->score, h->m, 0.1f, h->q, h->q_ok, done, s), "proposal");
    }
    a.kind = kWeighted;
    a.q = h->q;
    a.q_ok = h->q_ok;
  }
  if (h->kind == kGaussian) {
    check_hip(launch_sketch_gauss(bs.S, h->m, h->tau, h->ldas, h->opt.seed, h->opt.problem_id, k0, nb, bs.offs,
                                  done, s),
              "sketch (Gaussian)");
  } else if (h->kind == kSrht) {
    a.m = h->mpad;  // C is drawn over the padded coordinates
    check_hip(launch_sketch(a, s), "sketch (SRHT subset)");
    check_hip(launch_srht_fill(bs.S, h->m, h->tau, h->ldas, bs.members, h->opt.seed, h->opt.problem_id, k0, h->mpad,
                               nb, done, s),
              "sketch (SRHT)");
  } else {
    check_hip(launch_sketch(a, s), "sketch");
    if (h->dense_s) check_hip(launch_sketch_densify(bs.S, bs.hmap, h->m, h->ldas, nb, done, s), "dense S");
  }
  if (h->sparse && !h->arows)
    check_hip(launch_build_t(h->zt_col, h->zt_val, h->vals_f32, h->nnz, bs.hmap, h->m, nb, h->tbuf,
                             done, s),
              "T map");
  prof_end(h, pe, s);
  pe = prof_begin(h, RS_PROF_AS, nb, 1, s, k0);
  if (h->dense_s) {
    // T = Z^T S, A S = Z T + lambda S (kernel ridge: + lambda T = lambda K S), G = S^T A S. The SRHT
    // forms T and G by its fast transform (Z and AS each read once) when m' fits the LDS butterflies.
    const bool fast = h->kind == kSrht && h->mpad <= srht_fast_max_mpad();
    if (fast) {
      check_hip(launch_srht_apply(h->Z, h->ldz, 0, h->m, h->K, h->mpad, bs.S, h->ldas, h->m * h->ldas, bs.members,
                                  h->tau, bs.T, h->ldas, h->K * h->ldas, 0, nb, done, s),
                "T = Z^T S (fast Walsh-Hadamard transform)");
    } else {
      GemmF64Args g{};
      g.A = h->Z; g.lda = h->ldz; g.sA = 0;
      g.B = bs.S; g.ldb = h->ldas; g.sB = h->m * h->ldas;
      g.C = bs.T; g.ldc = h->ldas; g.sC = h->K * h->ldas;
      g.M = h->K; g.N = h->tau; g.Kd = h->m; g.done = done;
      check_hip(launch_gemm_f64(g, true, nb, s), "T = Z^T S");
    }
    GemmF64Args g2{};
    g2.A = h->Z; g2.lda = h->ldz; g2.sA = 0;
    g2.B = bs.T; g2.ldb = h->ldas; g2.sB = h->K * h->ldas;
    g2.C = (double*)bs.AS; g2.ldc = h->ldas; g2.sC = h->m * h->ldas;
    g2.E = h->kern ? bs.T : bs.S; g2.lde = h->ldas; g2.sE = h->kern ? h->K * h->ldas : h->m * h->ldas;
    g2.lam = h->lam;
    g2.M = h->m; g2.N = h->tau; g2.Kd = h->K; g2.done = done;
    check_hip(launch_gemm_f64(g2, false, nb, s), "AS = Z T + lambda S");
    prof_end(h, pe, s);
    pe = prof_begin(h, RS_PROF_G, nb, 1, s, k0);
    if (fast) {
      check_hip(launch_srht_apply((const double*)bs.AS, h->ldas, h->m * h->ldas, h->m, h->tau, h->mpad, bs.S,
                                  h->ldas, h->m * h->ldas, bs.members, h->tau, bs.G, h->ldg, h->ldg * h->ldg, 1, nb,
                                  done, s),
                "G = S^T A S (fast Walsh-Hadamard transform)");
    } else {
      GemmF64Args g3{};
      g3.A = bs.S; g3.lda = h->ldas; g3.sA = h->m * h->ldas;
      g3.B = (const double*)bs.AS; g3.ldb = h->ldas; g3.sB = h->m * h->ldas;
      g3.C = bs.G; g3.ldc = h->ldg; g3.sC = h->ldg * h->ldg;
      g3.M = h->tau; g3.N = h->tau; g3.Kd = h->m; g3.done = done;
      check_hip(launch_gemm_f64(g3, true, nb, s), "G = S^T A S");
    }
  } else if (h->arows) {
    check_hip(launch_as_arows(h->a_ptr, h->a_col, h->a_val, h->m, h->tau, h->ldas, nb, h->lam, bs.hmap, bs.AS,
                              h->mixed ? 1 : 0, done, s),
              "AS (rows of Z Z^T)");
    prof_end(h, pe, s);
    pe = prof_begin(h, RS_PROF_G, nb, 1, s, k0);
    check_hip(launch_g_from_as(bs.AS, h->mixed ? 1 : 0, h->m, h->tau, h->ldas, nb, bs.hmap, bs.members, bs.offs,
                               h->nsel, bs.G, h->ldg, done, s),
              "G = S^T AS");
  } else if (h->sparse) {
    check_hip(launch_as_sparse(h->zr_ptr, h->zr_col, h->zr_val, h->zt_ptr, h->zt_col, h->zt_val,
                               h->vals_f32, h->nnz, h->m, h->tau, h->ldas, nb, h->kind, h->lam,
                               bs.hmap, bs.members, bs.offs, h->nsel, h->tbuf, (double*)bs.AS, bs.G,
                               h->ldg, done, s),
              "AS (sparse)");
  } else if (h->gram) {
    check_hip(launch_gram_gather(h->gram, h->mixed ? 1 : 0, h->ldgram, h->m, bs.members, h->nsel, h->tau, h->ldas,
                                 nb, bs.AS, done, s),
              "AS (columns of the formed A)");
  } else if (h->mixed) {
    check_hip(launch_as_dense_bf16(h->Zbf, h->kpad, h->m, h->kpad, bs.members, h->tau, h->ldas, nb,
                                   h->lam, h->Z, h->ldz, h->kern ? 1 : 0, (float*)bs.AS, done, s,
                                   h->splitk_ws, h->splitk_floats),
              "AS (dense, BF16)");
  } else {
    check_hip(launch_as_dense_f64(h->Z, h->ldz, h->m, h->K, bs.members, h->tau, h->ldas, nb, h->lam,
                                  h->kern ? 1 : 0, (double*)bs.AS, done, s),
              "AS (dense)");
  }
  prof_end(h, pe, s);
  pe = prof_begin(h, RS_PROF_CHOL, nb, 1, s, k0);
  // One workgroup per sketch when the batch fills the chip; otherwise one per tile.
  if (h->ldg >= 128 && nb < 128)
    check_hip(launch_chol_multi(bs.G, h->W, h->Xd, h->ldg, h->tau, nb, h->kind, bs.AS,
                                h->mixed ? 1 : 0, h->ldas, h->m, bs.members, bs.offs, bs.status, done,
                                s),
              "cholesky (tiled)");
  else
    check_hip(launch_chol_inverse(bs.G, h->W, h->ldg, h->tau, nb, h->kind, bs.AS, h->mixed ? 1 : 0,
                                  h->ldas, h->m, bs.members, bs.offs, bs.status, done, s),
              "cholesky");
  prof_end(h, pe, s);
}

// Point the solver at buffer set p (the batch about to iterate; the accessors read it).
void use_set(rs_handle* h, int p) {
  h->cur_set = p;
  h->hmap = h->sets[p].hmap;
  h->members = h->sets[p].members;
  h->offs = h->sets[p].offs;
  h->AS = h->sets[p].AS;
  h->G = h->sets[p].G;
  h->status = h->sets[p].status;
  h->S = h->sets[p].S;
}

// Iterations k0 .. k0 + nb - 1 on the solver's stream, from the batch prepared in set p.
void iterate_batch(rs_handle* h, int p, int64_t k0, int nb) {
  hipStream_t s = h->stream;
  use_set(h, p);
  int pe = -1;
  // rho_{k0} = S_{k0}^T r^{k0}; later iterations get rho from the preceding update
  // (accelerated method: the sketch is applied to r_z)
  if (h->dense_s)
    check_hip(launch_rho_dense(h->S, h->ldas, h->tau, h->m, h->rbuf[k0 & 1], h->rho_part, h->rho, h->flags, s),
              "rho (dense S)");
  else
    check_hip(launch_rho(h->accel ? h->rzbuf : h->rbuf[k0 & 1], h->hmap, h->members, h->offs, h->tau, h->rho,
                         h->flags, s),
              "rho");
  const int pe_iters = prof_begin(h, RS_PROF_ITERS, nb);
  for (int i = 0; i < nb; ++i) {
    const int64_t k = k0 + i;
    double gamma, beta;
    momentum_schedule(h->opt, h->mom_switch, k, &gamma, &beta);
    const int cur = (int)(k & 1), nxt = 1 - cur;
    const int32_t* hm = h->hmap + (int64_t)i * h->m;
    pe = prof_begin(h, RS_PROF_DELTA, 1, 2);
    // mixed precision: the tracked residual drifts, so only the refreshed one may stop
    check_hip(launch_delta(h->rho, h->tau, h->G + (int64_t)i * h->ldg * h->ldg, h->ldg, h->partials,
                           h->npart, h->flags, h->hist, k, h->mixed ? -1.0 : h->opt.tol, h->delta, s),
              "delta");
    prof_end(h, pe);
    if (h->trace_every > 0 && k % h->trace_every == 0) {
      TraceArgs t{};
      t.m = h->m;
      t.tau = h->tau;
      t.k = k;
      t.k0 = k0;
      t.slot = i;
      t.members = h->members + (int64_t)i * h->nsel;
      t.hmap_batch = h->hmap;
      t.last = h->last;
      t.a = h->adiag;
      t.stats = h->lstats;
      t.r = h->rbuf[cur];
      t.rp = h->rbuf[nxt];
      t.delta = h->delta;
      t.rho = h->rho;
      t.F = h->tr_F;
      t.credits = h->tr_c;
      t.count = h->tr_count;
      t.capacity = h->trace_cap;
      t.flags = h->flags;
      check_hip(launch_trace(t, s), "trace");
    }
    pe = prof_begin(h, RS_PROF_UPDATE, 1, 2);
    const bool has_next = i + 1 < nb;
    const size_t as_elt = h->mixed ? sizeof(float) : sizeof(double);
    const void* as_i = (const char*)h->AS + (size_t)i * h->m * h->ldas * as_elt;
    const int32_t* hm_n = has_next ? h->hmap + (int64_t)(i + 1) * h->m : nullptr;
    const int32_t* mem_n = has_next ? h->members + (int64_t)(i + 1) * h->nsel : nullptr;
    const int32_t* offs_n = has_next ? h->offs + (int64_t)(i + 1) * (h->tau + 1) : nullptr;
    if (h->dense_s) {
      const double* S_i = h->S + (size_t)i * h->m * h->ldas;
      check_hip(launch_update_dense((const double*)as_i, S_i, h->ldas, h->tau, h->delta, h->m, h->xbuf[cur],
                                    h->xbuf[nxt], h->rbuf[cur], h->rbuf[nxt], gamma, beta, h->partials, h->npart,
                                    h->flags, s),
                "update (dense S)");
      if (has_next)
        check_hip(launch_rho_dense(S_i + (size_t)h->m * h->ldas, h->ldas, h->tau, h->m, h->rbuf[nxt], h->rho_part,
                                   h->rho, h->flags, s),
                  "rho (dense S)");
    } else if (h->accel)
      check_hip(launch_update_accel((const double*)as_i, h->ldas, h->tau, h->delta, hm, h->m, h->xbuf[cur],
                                    h->xbuf[nxt], h->rbuf[cur], h->rbuf[nxt], h->vbuf, h->rvbuf, h->rzbuf,
                                    h->acc_alpha, h->acc_beta, h->acc_gamma, h->partials, h->npart, hm_n,
                                    mem_n, offs_n, h->kind == kCount ? 1 : 0, h->rho, h->flags, s),
                "update (accelerated)");
    else
      check_hip(launch_update(as_i, h->mixed ? 1 : 0, h->ldas, h->tau, h->delta, hm, h->m,
                              h->xbuf[cur], h->xbuf[nxt], h->rbuf[cur], h->rbuf[nxt], gamma, beta,
                              h->partials, h->npart, hm_n, mem_n, offs_n,
                              h->kind == kCount ? 1 : 0, h->rho, h->flags, s),
                "update");
    prof_end(h, pe);
    if (h->mixed && (k + 1) % h->opt.refresh_every == 0) {
      refresh(h, k + 1);
      if (has_next)
        check_hip(launch_rho(h->rbuf[(k + 1) & 1], h->hmap + (int64_t)(i + 1) * h->m,
                             h->members + (int64_t)(i + 1) * h->nsel,
                             h->offs + (int64_t)(i + 1) * (h->tau + 1), h->tau, h->rho, h->flags, s),
                  "rho");
    }
  }
  prof_end(h, pe_iters);
  if (h->last)
    check_hip(launch_mark_last(h->members, h->tau, nb, k0, h->last, s), "sketch history");
  h->batch_k0 = k0;
  h->batch_n = nb;
}

// Size of the batch starting at iteration k_from: the lookahead, or near the tolerance
// fewer, from the contraction observed between the last two known residual norms, so
// that few sketches are formed past the stopping iteration.
// Iterations still needed after k_from to reach the tolerance, extrapolated from the
// contraction between the last two known residual norms; +inf when unknown.
double predicted_need(const rs_handle* h, int64_t k_from, int64_t k_a, double rel_a, int64_t k_b, double rel_b) {
  if (k_a >= 0 && k_b > k_a && rel_b < rel_a && rel_b > 0.0 && h->opt.tol > 0.0) {
    const double rate = std::log(rel_b / rel_a) / (double)(k_b - k_a);
    return std::log(h->opt.tol / rel_b) / rate - (double)(k_from - k_b);
  }
  return INFINITY;
}

int batch_size(const rs_handle* h, int64_t left, int64_t k_from, int64_t k_a, double rel_a, int64_t k_b,
               double rel_b) {
  int nb = (int)std::min<int64_t>(h->B, left);
  const double need = predicted_need(h, k_from, k_a, rel_a, k_b, rel_b);
  // never above the lookahead buffers nor the iterations asked for
  if (need < nb) nb = (int)std::min<double>(nb, std::max<double>(std::min(16, nb), need * 1.1 + 8.0));
  return nb;
}

// Waits for the preparation stream when advance() leaves, also on an error.
struct PrepDrain {
  rs_handle* h;
  ~PrepDrain() {
    if (h->pipeline) (void)hipStreamSynchronize(h->prep_stream);
  }
};

// Advance up to `iters` iterations, one lookahead batch at a time. After each batch
// the stop flag, the factorisation status and the error word are read back.
//
// With the pipeline on, every batch is prepared on prep_stream (so preparations, which
// share scratch buffers, run in order) and batch t + 1 is queued there before the host
// waits for batch t: its sketches, products and factorisations run while batch t
// iterates, in the other buffer set. The host waits for both streams after each batch,
// so a set is never written while iterations read it.
void advance(rs_handle* h, int64_t iters) {
  if (h->sampler == RS_SAMPLER_LEARNED && !h->params_set)
    throw Fail{RS_EINVAL, "the learned sampler needs rs_set_sampler_params before iterating"};
  int64_t k_enq = h->k;
  int64_t left = std::min(iters, h->opt.max_iter - h->k);
  std::vector<int32_t> st(h->B);
  // last two known points (k, ||r^k|| / ||r^0||) of the residual history
  int64_t k_a = -1, k_b = -1;
  double rel_a = 0.0, rel_b = 0.0;
  const bool pipe = h->pipeline;
  PrepDrain drain{h};
  int p = h->cur_set;
  int nb = 0;
  bool prepared = false;  // set p holds the batch that starts at k_enq (nb sketches)
  // With the pipeline every preparation, also one that was not queued ahead, runs on
  // prep_stream: preparations share scratch buffers and must not overlap each other.
  hipStream_t ps = pipe ? h->prep_stream : h->stream;
  if (pipe && left > 0 && !h->done) {
    // the first preparation follows what the caller queued on the solver's stream
    check_hip(hipEventRecord(h->ev_start, h->stream), "event");
    check_hip(hipStreamWaitEvent(h->prep_stream, h->ev_start, 0), "wait");
  }
  while (left > 0 && !h->done) {
    if (!prepared) {
      nb = batch_size(h, left, k_enq, k_a, rel_a, k_b, rel_b);
      prep_batch(h, p, k_enq, nb, ps);
    }
    if (pipe) {
      check_hip(hipEventRecord(h->ev_ready[p], h->prep_stream), "event");
      check_hip(hipStreamWaitEvent(h->stream, h->ev_ready[p], 0), "wait");
    }
    iterate_batch(h, p, k_enq, nb);
    k_enq += nb;
    left -= nb;
    prepared = false;
    int nb_next = 0;
    // Not when the tolerance is predicted within the batch just queued or early in the
    // next: a batch prepared past the stopping iteration is only waited for, while a
    // batch prepared after the wait is a short one.
    if (pipe && left > 0 && predicted_need(h, k_enq, k_a, rel_a, k_b, rel_b) > 0.25 * nb) {
      nb_next = batch_size(h, left, k_enq, k_a, rel_a, k_b, rel_b);
      prep_batch(h, 1 - p, k_enq, nb_next, ps);
      prepared = true;
    }
    if (left == 0) {
      if (h->mixed) {
        if (k_enq % h->opt.refresh_every != 0) refresh(h, k_enq);
      } else {
        check_hip(launch_finalize(h->partials, h->npart, h->flags, h->hist, k_enq, h->opt.tol,
                                  h->stream),
                  "finalize");
      }
    }
    // One report kernel after the batch (and after the preparation queued ahead, so that
    // its errors are seen now) and one wait, instead of a round trip per value.
    if (pipe) {
      check_hip(hipEventRecord(h->ev_prep_done, h->prep_stream), "event");
      check_hip(hipStreamWaitEvent(h->stream, h->ev_prep_done, 0), "wait");
    }
    check_hip(launch_batch_report(h->flags, h->err, h->hist, k_enq, h->status, nb, h->rep_dev, h->stream),
              "report");
    check_hip(hipStreamSynchronize(h->stream), "sync");
    DevFlags f = h->rep_host->flags;
    const int32_t err = h->rep_host->err;
    for (int i = 0; i < nb; ++i) st[i] = h->rep_host->status[i];
    prof_collect(h, f.done ? f.k_done : INT64_MAX);
    if (err) throw Fail{RS_EDEVICE, "internal sketch limit hit (code " + std::to_string(err) + ")"};
    const int64_t k_end = f.done ? f.k_done : k_enq;
    for (int i = 0; i < nb; ++i)
      if (st[i] != 0 && h->batch_k0 + i < k_end)
        throw Fail{RS_ESINGULAR, "non-positive pivot in the Cholesky factorisation of S^T A S"};
    if (!f.done && left > 0 && k_end > 0) {
      const double rel = h->rep_host->rel;  // ||r^{k_end - 1}||, from the batch's last delta launch
      k_a = k_b;
      rel_a = rel_b;
      k_b = k_end - 1;
      rel_b = rel;
      // Mixed precision stops only on a refreshed residual. Besides every refresh_every
      // iterations, refresh at this batch boundary once the tracked estimate has reached
      // tol, so that a solve is not carried to the next multiple of refresh_every; a refresh
      // that does not meet tol resets the estimate to the FP64 residual, and the next such
      // refresh waits at least 4 iterations.
      if (h->mixed && h->opt.refresh_early && rel <= h->opt.tol && k_end % h->opt.refresh_every != 0 &&
          k_end - h->last_early >= 4) {
        h->last_early = k_end;
        refresh(h, k_end);
        check_hip(hipMemcpyAsync(&f, h->flags, sizeof(DevFlags), hipMemcpyDeviceToHost, h->stream), "flags");
        check_hip(hipStreamSynchronize(h->stream), "sync");
        prof_collect(h, f.done ? f.k_done : INT64_MAX);
      }
    }
    h->k = k_end;
    if (f.done) h->done = true;
    if (prepared) {
      p = 1 - p;
      nb = nb_next;
    }
  }
}

}  // namespace

extern "C" {

rs_status rs_options_default(rs_options* o) {
  if (!o) return RS_EINVAL;
  std::memset(o, 0, sizeof(*o));
  o->form = RS_FORM_AUTO;
  o->sketch = RS_SKETCH_SUBSAMPLE;
  o->tau = 0;
  o->subcount_k = 0;
  o->momentum = RS_MOMENTUM_HEURISTIC;
  o->precision = RS_PREC_FP64;
  o->gamma = 1.0;
  o->beta = 0.5;
  o->eta = 0.995;
  o->beta_max = 0.5;
  o->tol = 1e-6;
  o->max_iter = 100000;
  o->seed = 1;
  o->problem_id = 0;
  o->refresh_every = 20;
  o->refresh_early = 1;
  o->lookahead = 0;
  o->stream = nullptr;
  o->graph_iters = 0;
  o->autotune = 0;
  o->sampler = RS_SAMPLER_UNIFORM;
  o->trace_every = 0;
  o->trace_capacity = 0;
  o->sparse_route = RS_ROUTE_AUTO;
  o->pipeline = 1;
  o->accelerated = 0;
  o->accel_mu = 1.0;
  o->accel_nu = 1.0;
  return RS_OK;
}

rs_status rs_momentum_schedule(const rs_options* o, int64_t k, double* gamma, double* beta) {
  if (!o || !gamma || !beta || k < 0 || momentum_invalid(*o)) return RS_EINVAL;
  momentum_schedule(*o, momentum_switch(o->eta, o->beta_max), k, gamma, beta);
  return RS_OK;
}

const char* rs_status_string(rs_status s) {
  switch (s) {
    case RS_OK: return "ok";
    case RS_NOT_CONVERGED: return "not converged (max_iter reached)";
    case RS_EINVAL: return "invalid argument";
    case RS_ENOMEM: return "out of device memory";
    case RS_EDEVICE: return "device error";
    case RS_ESINGULAR: return "sketched system not positive definite";
    case RS_EUNSUPPORTED: return "unsupported option";
    default: return "unknown status";
  }
}

const char* rs_last_error(const rs_handle* h) {
  return h ? h->last_error.c_str() : g_create_error.c_str();
}

}  // extern "C"

namespace {

// Shared by rs_create and rs_create_kernel: sigma > 0 selects kernel ridge with X the points.
rs_status create_impl(const rs_matrix* X, const double* y, double lambda, double sigma, const rs_options* o,
                      rs_handle** out) {
  g_create_error.clear();
  if (!X || !y || !o || !out) {
    g_create_error = "null argument";
    return RS_EINVAL;
  }
  *out = nullptr;
  rs_handle* h = new rs_handle();
  try {
    const bool kern = sigma > 0.0;
    h->kern = kern;
    if (kern && X->layout == RS_CSR) throw Fail{RS_EINVAL, "kernel ridge takes dense points"};
    if (kern && (o->sampler != RS_SAMPLER_UNIFORM || o->trace_every != 0))
      throw Fail{RS_EUNSUPPORTED, "kernel ridge uses uniform sampling without traces"};
    h->opt = *o;
    h->stream = static_cast<hipStream_t>(o->stream);
    const int64_t n = X->n, d = X->d;
    if (n <= 0 || d <= 0) throw Fail{RS_EINVAL, "X must have n, d >= 1"};
    if (!(lambda > 0.0) || !std::isfinite(lambda)) throw Fail{RS_EINVAL, "lambda must be positive and finite"};
    if (X->dtype != RS_F64 && X->dtype != RS_F32) throw Fail{RS_EINVAL, "dtype must be RS_F64 or RS_F32"};
    if (X->mem != RS_HOST && X->mem != RS_DEVICE) throw Fail{RS_EINVAL, "mem must be RS_HOST or RS_DEVICE"};
    if (X->layout != RS_DENSE_ROWMAJOR && X->layout != RS_DENSE_COLMAJOR && X->layout != RS_CSR)
      throw Fail{RS_EINVAL, "unknown layout"};
    if (!X->vals) throw Fail{RS_EINVAL, "X.vals is null"};
    if (X->layout == RS_CSR && (!X->row_ptr || !X->col_idx || X->nnz < 0))
      throw Fail{RS_EINVAL, "CSR needs row_ptr, col_idx and nnz >= 0"};
    if (n > INT32_MAX || d > INT32_MAX) throw Fail{RS_EINVAL, "n and d must fit in int32"};
    if (o->precision != RS_PREC_FP64 && o->precision != RS_PREC_MIXED_BF16)
      throw Fail{RS_EINVAL, "unknown precision"};
    if (o->precision == RS_PREC_MIXED_BF16 && X->layout == RS_CSR &&
        (o->sketch != RS_SKETCH_COUNT && o->sketch != RS_SKETCH_SUBCOUNT))
      throw Fail{RS_EUNSUPPORTED, "mixed precision on CSR data is built for the count and SubCount sketches"};
    if (o->precision == RS_PREC_MIXED_BF16 && X->layout == RS_CSR &&
        (o->sparse_route == RS_ROUTE_SCATTER || o->accelerated != 0))
      throw Fail{RS_EUNSUPPORTED, "mixed precision on CSR data runs on the rows of Z Z^T (sparse_route AUTO or "
                                  "AROWS) with the momentum schedules"};
    if (o->precision == RS_PREC_MIXED_BF16 && o->refresh_every < 1)
      throw Fail{RS_EINVAL, "refresh_every must be >= 1"};
    if (o->refresh_early != 0 && o->refresh_early != 1) throw Fail{RS_EINVAL, "refresh_early is 0 or 1"};
    if (o->profile < 0 || o->profile > 3) throw Fail{RS_EINVAL, "profile is 0, 1, 2 or 3"};
    h->mixed = o->precision == RS_PREC_MIXED_BF16;
    if (o->sampler < RS_SAMPLER_UNIFORM || o->sampler > RS_SAMPLER_DIAG) throw Fail{RS_EINVAL, "unknown sampler"};
    if (o->sparse_route < RS_ROUTE_AUTO || o->sparse_route > RS_ROUTE_AROWS)
      throw Fail{RS_EINVAL, "unknown sparse route"};
    if (o->trace_every < 0 || o->trace_capacity < 0) throw Fail{RS_EINVAL, "trace settings must be >= 0"};
    if ((o->sampler != RS_SAMPLER_UNIFORM || o->trace_every > 0) &&
        (X->layout == RS_CSR || o->sketch != RS_SKETCH_SUBSAMPLE))
      throw Fail{RS_EUNSUPPORTED, "proposals and traces are built for the subsample sketch on dense data"};
    if (const char* why = momentum_invalid(*o)) throw Fail{RS_EINVAL, why};
    h->mom_switch = momentum_switch(o->eta, o->beta_max);
    if (o->accelerated != 0) {
      const double mu = o->accel_mu, nu = o->accel_nu;
      if (!(mu > 0.0 && mu <= 1.0) || !(nu >= 1.0 && nu <= 1.0 / mu))
        throw Fail{RS_EINVAL, "the accelerated method needs 0 < mu <= 1 and 1 <= nu <= 1 / mu"};
      if (o->precision != RS_PREC_FP64 || o->sampler != RS_SAMPLER_UNIFORM || o->trace_every != 0)
        throw Fail{RS_EUNSUPPORTED, "the accelerated method runs in FP64 with uniform sampling"};
      h->accel = true;
      accel_constants(mu, nu, &h->acc_alpha, &h->acc_beta, &h->acc_gamma);
    }
    if (!(o->tol >= 0.0)) throw Fail{RS_EINVAL, "tol must be >= 0"};
    if (o->max_iter < 0 || o->max_iter > 100000000) throw Fail{RS_EINVAL, "max_iter out of range"};
    h->form = o->form == RS_FORM_AUTO ? (d <= n ? RS_FORM_PRIMAL : RS_FORM_DUAL) : o->form;
    if (h->form != RS_FORM_PRIMAL && h->form != RS_FORM_DUAL) throw Fail{RS_EINVAL, "unknown form"};
    if (kern) h->form = RS_FORM_DUAL;  // n coefficients alpha; the weights are alpha itself
    h->n = n;
    h->d = kern ? n : d;
    h->pdim = kern ? d : 0;
    h->m = h->form == RS_FORM_PRIMAL ? d : n;
    h->K = h->form == RS_FORM_PRIMAL ? n : (kern ? n : d);
    h->lam = lambda;
    h->sparse = X->layout == RS_CSR;
    h->tau = o->tau;
    if (h->tau < 1 || h->tau > h->m) throw Fail{RS_EINVAL, "tau must satisfy 1 <= tau <= m"};
    switch (o->sketch) {
      case RS_SKETCH_SUBSAMPLE:
        h->kind = kSubsample;
        h->nsel = h->tau;
        break;
      case RS_SKETCH_COUNT:
        h->kind = kCount;
        h->nsel = h->m;
        if (h->tau > 2048) throw Fail{RS_EUNSUPPORTED, "count sketch supports tau <= 2048"};
        break;
      case RS_SKETCH_SUBCOUNT:
        h->kind = kSubcount;
        h->sub_k = o->subcount_k > 0 ? o->subcount_k : subcount_rule(h->m, h->tau);
        h->nsel = (int64_t)h->sub_k * h->tau;
        if (h->sub_k < 1 || h->nsel > h->m) throw Fail{RS_EINVAL, "SubCount needs 1 <= k and k * tau <= m"};
        if (h->nsel > 8192) throw Fail{RS_EUNSUPPORTED, "SubCount supports s = k * tau <= 8192"};
        if (h->tau > 2048) throw Fail{RS_EUNSUPPORTED, "SubCount supports tau <= 2048"};
        break;
      case RS_SKETCH_GAUSSIAN:
      case RS_SKETCH_SRHT:
        h->kind = o->sketch == RS_SKETCH_GAUSSIAN ? kGaussian : kSrht;
        h->nsel = h->tau;
        h->dense_s = true;
        h->mpad = 1;
        while (h->mpad < h->m) h->mpad <<= 1;
        if (h->sparse) throw Fail{RS_EUNSUPPORTED, "Gaussian and SRHT sketches are built for dense data"};
        if (h->mixed || o->sampler != RS_SAMPLER_UNIFORM || o->trace_every != 0 || o->accelerated != 0)
          throw Fail{RS_EUNSUPPORTED, "Gaussian and SRHT sketches run in FP64 with uniform sampling and momentum"};
        break;
      default:
        throw Fail{RS_EINVAL, "unknown sketch"};
    }
    if ((h->kind == kCount || h->kind == kSubcount) && !h->sparse) {
      // dense data: the drawn sketch is expanded to a dense S and takes the dense-S products
      if (h->mixed || o->sampler != RS_SAMPLER_UNIFORM || o->trace_every != 0 || o->accelerated != 0)
        throw Fail{RS_EUNSUPPORTED, "count and SubCount sketches on dense data run in FP64 with uniform sampling "
                                    "and momentum"};
      h->dense_s = true;
    }
    if (h->kind == kSubsample && h->sparse)
      throw Fail{RS_EUNSUPPORTED, "the subsample sketch needs dense data"};
    if (o->dense_route != 0 && o->dense_route != 1) throw Fail{RS_EINVAL, "dense_route is 0 or 1"};
    if (o->dense_route == 1 && (h->sparse || h->kind != kSubsample))
      throw Fail{RS_EUNSUPPORTED, "the formed-A route serves the subsample sketch on dense data or kernel ridge"};

    // y: validate on the host
    std::vector<double> yh(n);
    if (X->mem == RS_DEVICE)
      check_hip(hipMemcpy(yh.data(), y, sizeof(double) * n, hipMemcpyDeviceToHost), "y download");
    else
      std::memcpy(yh.data(), y, sizeof(double) * n);
    for (double v : yh)
      if (!std::isfinite(v)) throw Fail{RS_EINVAL, "y has a non-finite entry"};

    hipStream_t s = h->stream;
    const bool f32 = X->dtype == RS_F32;
    const size_t esz = f32 ? 4 : 8;
    double* yd = to_device<double>(h, yh.data(), n, RS_HOST);
    h->b = dalloc<double>(h, h->m);

    if (!h->sparse) {
      const size_t total = (size_t)n * d;
      void* xv = dalloc<char>(h, total * esz);
      check_hip(hipMemcpyAsync(xv, X->vals, total * esz,
                               X->mem == RS_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, s),
                "X upload");
      // Z = X^T (primal) or X (dual), row-major m x K
      const bool rowmajor = X->layout == RS_DENSE_ROWMAJOR;
      const bool need_transpose = (h->form == RS_FORM_PRIMAL) == rowmajor;
      if (kern) {
        // points as FP64 row-major n x d, then Z = K (n x n, eq:Gausskernel) and b = K y
        double* p64 = dalloc<double>(h, (size_t)n * d);
        if (rowmajor)
          check_hip(launch_copy_to_f64(xv, f32, n, d, d, p64, d, s), "points");
        else
          check_hip(launch_transpose_to_f64(xv, f32, d, n, n, p64, d, s), "points");
        h->ldz = n;
        h->Z = dalloc<double>(h, (size_t)n * h->ldz);
        check_hip(launch_rbf_gram(p64, n, d, sigma, h->Z, h->ldz, s), "kernel matrix");
        check_hip(launch_gemv_rows(h->Z, h->ldz, h->m, h->K, yd, h->b, s), "b = K y");
        std::vector<void*> tmp{(void*)p64, xv};
        if (h->mixed) {
          // BF16 copy for the products; K itself stays for the shift and the FP64 refresh (an
          // FP32 copy would make the refreshed residual that of a rounded kernel matrix)
          h->kpad = (h->K + 63) / 64 * 64;
          h->Zbf = dalloc<uint16_t>(h, (size_t)h->m * h->kpad);
          check_hip(launch_cast_bf16(h->Z, 0, n, n, n, 0, h->Zbf, h->kpad, nullptr, 0, s), "BF16 copy");
          h->ref_u = dalloc<double>(h, 2 * h->K);
          h->ref_upart = dalloc<double>(h, refresh_upart_doubles(h->m, h->K));
          h->ref_partials = dalloc<double>(h, refresh_partials(h->m));
        }
        check_hip(hipStreamSynchronize(s), "sync");
        for (void* p : tmp) {
          (void)hipFree(p);
          h->allocs.erase(std::find(h->allocs.begin(), h->allocs.end(), p));
        }
      } else if (h->mixed) {
        h->kpad = (h->K + 63) / 64 * 64;
        h->Zbf = dalloc<uint16_t>(h, (size_t)h->m * h->kpad);
        h->ld32 = (h->K + 3) / 4 * 4;
        h->Z32 = dalloc<float>(h, (size_t)h->m * h->ld32);
        const int64_t rows = rowmajor ? n : d, cols = rowmajor ? d : n;
        check_hip(launch_cast_bf16(xv, f32, rows, cols, cols, need_transpose ? 1 : 0, h->Zbf, h->kpad,
                                   h->Z32, h->ld32, s),
                  "BF16 copy");
        if (h->form == RS_FORM_PRIMAL)
          check_hip(launch_gemv_rows_f32(h->Z32, h->ld32, h->m, h->K, yd, h->b, s), "b = X^T y");
        else
          check_hip(hipMemcpyAsync(h->b, yd, sizeof(double) * n, hipMemcpyDeviceToDevice, s), "b = y");
        h->ref_u = dalloc<double>(h, 2 * h->K);
        h->ref_upart = dalloc<double>(h, refresh_upart_doubles(h->m, h->K));
        h->ref_partials = dalloc<double>(h, refresh_partials(h->m));
        check_hip(hipStreamSynchronize(s), "sync");
        (void)hipFree(xv);
        h->allocs.erase(std::find(h->allocs.begin(), h->allocs.end(), xv));
      } else {
      h->ldz = h->K;
      h->Z = dalloc<double>(h, (size_t)h->m * h->ldz);
      if (need_transpose) {
        // source viewed row-major: rowmajor -> n x d, colmajor -> d x n
        const int64_t rows = rowmajor ? n : d, cols = rowmajor ? d : n;
        check_hip(launch_transpose_to_f64(xv, f32, rows, cols, cols, h->Z, h->ldz, s), "transpose");
      } else {
        const int64_t rows = rowmajor ? n : d, cols = rowmajor ? d : n;
        check_hip(launch_copy_to_f64(xv, f32, rows, cols, cols, h->Z, h->ldz, s), "copy");
      }
      if (h->form == RS_FORM_PRIMAL)
        check_hip(launch_gemv_rows(h->Z, h->ldz, h->m, h->K, yd, h->b, s), "b = X^T y");
      else
        check_hip(hipMemcpyAsync(h->b, yd, sizeof(double) * n, hipMemcpyDeviceToDevice, s), "b = y");
      }
    } else {
      const int64_t nnz = X->nnz;
      if (nnz > INT32_MAX) throw Fail{RS_EINVAL, "nnz must fit in int32"};
      int64_t* xptr = to_device<int64_t>(h, X->row_ptr, n + 1, X->mem);
      int32_t* xcol = to_device<int32_t>(h, X->col_idx, nnz, X->mem);
      void* xval = dalloc<char>(h, (size_t)nnz * esz);
      if (nnz)
        check_hip(hipMemcpyAsync(xval, X->vals, nnz * esz,
                                 X->mem == RS_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, s),
                  "X upload");
      // host-side structural check of row_ptr
      std::vector<int64_t> ph(n + 1);
      check_hip(hipMemcpyAsync(ph.data(), xptr, sizeof(int64_t) * (n + 1), hipMemcpyDeviceToHost, s),
                "row_ptr");
      check_hip(hipStreamSynchronize(s), "sync");
      if (ph[0] != 0 || ph[n] != nnz) throw Fail{RS_EINVAL, "row_ptr must start at 0 and end at nnz"};
      for (int64_t i = 0; i < n; ++i)
        if (ph[i + 1] < ph[i]) throw Fail{RS_EINVAL, "row_ptr must be non-decreasing"};
      std::vector<int32_t> ch(nnz);
      if (nnz)
        check_hip(hipMemcpy(ch.data(), xcol, sizeof(int32_t) * nnz, hipMemcpyDeviceToHost), "col_idx");
      for (int64_t i = 0; i < n; ++i)
        for (int64_t p = ph[i]; p < ph[i + 1]; ++p)
          if (ch[p] < 0 || ch[p] >= d || (p > ph[i] && ch[p] <= ch[p - 1]))
            throw Fail{RS_EINVAL, "col_idx must be in [0, d) and strictly increasing within a row"};
      h->vals_f32 = f32 ? 1 : 0;
      h->nnz = nnz;
      int64_t* tptr = dalloc<int64_t>(h, d + 1);
      int32_t* tcol = dalloc<int32_t>(h, nnz);
      void* tval = dalloc<char>(h, (size_t)nnz * esz);
      check_hip(csr_transpose(xptr, xcol, xval, h->vals_f32, n, d, nnz, tptr, tcol, tval, s), "transpose");
      if (h->form == RS_FORM_PRIMAL) {
        h->zr_ptr = tptr; h->zr_col = tcol; h->zr_val = tval;  // Z = X^T
        h->zt_ptr = xptr; h->zt_col = xcol; h->zt_val = xval;
        check_hip(launch_spmv_csr(h->zr_ptr, h->zr_col, h->zr_val, h->vals_f32, h->m, yd, h->b, s),
                  "b = X^T y");
      } else {
        h->zr_ptr = xptr; h->zr_col = xcol; h->zr_val = xval;  // Z = X
        h->zt_ptr = tptr; h->zt_col = tcol; h->zt_val = tval;
        check_hip(hipMemcpyAsync(h->b, yd, sizeof(double) * n, hipMemcpyDeviceToDevice, s), "b = y");
      }
      if (h->mixed) {
        // FP64 refresh from the CSR data: Z^T [x, xp], Z (Z^T [x, xp]), partial norms
        h->ref_u = dalloc<double>(h, 2 * h->K);
        h->ref_t = dalloc<double>(h, 2 * h->m);
        h->ref_partials = dalloc<double>(h, refresh_csr_partials(h->m));
      }
    }

    if (h->sparse && (o->sparse_route == RS_ROUTE_AROWS || o->sparse_route == RS_ROUTE_AUTO)) {
      std::vector<int64_t> tp(h->K + 1);
      check_hip(hipMemcpy(tp.data(), h->zt_ptr, sizeof(int64_t) * (h->K + 1), hipMemcpyDeviceToHost),
                "row pointers");
      const int64_t pairs = zzt_pairs(tp.data(), h->K);
      size_t free_b = 0, total_b = 0;
      check_hip(hipMemGetInfo(&free_b, &total_b), "memory info");
      // sort and reduction buffers: 48 bytes per pair while A0 is formed
      const bool fits = pairs > 0 && pairs < (int64_t)INT32_MAX && (double)pairs * 48.0 < 0.25 * (double)free_b;
      if ((o->sparse_route == RS_ROUTE_AROWS || h->mixed) && !fits)
        throw Fail{RS_EUNSUPPORTED, "the product Z Z^T is too large for the rows-of-A route"};
      if (fits) {
        check_hip(build_zzt(h->zt_ptr, h->zt_col, h->zt_val, h->vals_f32, h->K, h->m, pairs, &h->a_ptr,
                            &h->a_col, &h->a_val, &h->a_nnz, s),
                  "Z Z^T");
        h->allocs.push_back(h->a_ptr);
        h->allocs.push_back(h->a_col);
        h->allocs.push_back(h->a_val);
        h->arows = true;
      }
    }

    // batch buffers
    h->ldg = ((int64_t)h->tau + 63) / 64 * 64;
    h->ldas = ((int64_t)h->tau + 7) / 8 * 8;
    // The learned proposal reads the iterate, so its batches cannot be prepared ahead.
    h->pipeline = o->pipeline != 0 && o->sampler != RS_SAMPLER_LEARNED;
    h->nsets = h->pipeline ? 2 : 1;
    const int64_t mkeys = h->kind == kSrht ? h->mpad : h->m;  // coordinates the selection keys span
    const size_t per_slot_set = (h->mixed ? sizeof(float) : sizeof(double)) * (size_t)h->m * h->ldas +
                                sizeof(double) * (size_t)h->ldg * h->ldg +
                                sizeof(int32_t) * ((size_t)mkeys + h->nsel + h->tau + 2) +
                                (h->dense_s ? sizeof(double) * (size_t)(h->m + h->K) * h->ldas : 0);
    const size_t per_slot = h->nsets * per_slot_set +
                            (h->sparse && !h->arows ? sparse_t_bytes(h->vals_f32, h->nnz) : 0) +
                            sizeof(double) * (size_t)h->ldg * h->ldg + sizeof(uint64_t) * (size_t)mkeys;
    // The formed A of dense_route = 1 (m x m) is held beside the batch buffers: it comes out of
    // the same budget, and a system whose A alone exceeds it is refused here, before any
    // device allocation.
    const size_t elt = h->mixed ? sizeof(float) : sizeof(double);
    const size_t gram_bytes = o->dense_route == 1 ? (size_t)h->m * (size_t)((h->m + 7) / 8 * 8) * elt : 0;
    const size_t budget_all = (size_t)48 << 30;
    if (gram_bytes + per_slot > budget_all)
      throw Fail{RS_ENOMEM, "dense_route = 1: the formed A (" + std::to_string(gram_bytes >> 20) +
                                " MiB) and one lookahead slot exceed the 48 GiB the solver budgets"};
    // Default lookahead: 256 sketches, fewer when one sketch's contraction is large (the
    // sketches formed past the stopping iteration are wasted work, and the first batch's
    // preparation is not overlapped). The formed-A route follows the same rule: its
    // factorisations of 32 sketches run device-wide (the 50000 x 8192, tau = 1024 mixed solve
    // with A formed: 0.075 s at 32 against 0.108 s at 256).
    int B = 256;
    if (!h->sparse && 2.0 * (double)h->m * (double)h->K * (double)h->tau > 1e11) B = 32;
    // the learned proposal is recomputed once per batch: short batches keep it fresh (the BF16
    // products of a short batch are split over K, so they still fill the chip)
    if (o->sampler == RS_SAMPLER_LEARNED) B = 2;
    if (o->lookahead > 0) B = o->lookahead;
    const size_t budget = budget_all - gram_bytes;
    while (B > 1 && (size_t)B * per_slot > budget) B >>= 1;
    h->B = B;
    if (h->mixed && !h->sparse && !h->dense_s && o->dense_route != 1) {
      // batches whose product tiles leave compute units idle are split over K: room for the
      // largest split any batch size up to B asks for
      int64_t need = 0;
      for (int nb = 1; nb <= B; ++nb) {
        const int32_t sp = bf16_split_factor(h->m, h->kpad, h->tau, nb);
        if (sp > 1) need = std::max<int64_t>(need, (int64_t)sp * nb * h->m * h->ldas);
      }
      if (need > 0) {
        h->splitk_ws = dalloc<float>(h, (size_t)need);
        h->splitk_floats = need;
      }
    }
    const size_t as_bytes = (h->mixed ? sizeof(float) : sizeof(double)) * (size_t)B * h->m * h->ldas;
    for (int p = 0; p < h->nsets; ++p) {
      rs_handle::BatchSet& bs = h->sets[p];
      bs.hmap = dalloc<int32_t>(h, (size_t)B * mkeys);
      bs.members = dalloc<int32_t>(h, (size_t)B * h->nsel);
      bs.offs = dalloc<int32_t>(h, (size_t)B * (h->tau + 1));
      bs.AS = dalloc<char>(h, as_bytes);
      // the padding columns of AS are read (times a zero delta) by the update: keep them zero
      check_hip(hipMemsetAsync(bs.AS, 0, as_bytes, s), "memset");
      bs.G = dalloc<double>(h, (size_t)B * h->ldg * h->ldg);
      bs.status = dalloc<int32_t>(h, B);
      check_hip(hipMemsetAsync(bs.status, 0, sizeof(int32_t) * B, s), "memset");
      if (h->dense_s) {
        bs.S = dalloc<double>(h, (size_t)B * h->m * h->ldas);
        bs.T = dalloc<double>(h, (size_t)B * h->K * h->ldas);
      }
    }
    use_set(h, 0);
    h->keys = dalloc<uint64_t>(h, (size_t)B * mkeys);
    if (h->dense_s) h->rho_part = dalloc<double>(h, (size_t)rho_dense_blocks() * h->tau);
    if (h->pipeline) {
      // default priority, like the solver's stream
      check_hip(hipStreamCreateWithFlags(&h->prep_stream, hipStreamNonBlocking), "stream create");
      for (hipEvent_t* e : {&h->ev_ready[0], &h->ev_ready[1], &h->ev_start, &h->ev_prep_done})
        check_hip(hipEventCreateWithFlags(e, hipEventDisableTiming), "event create");
    }
    check_hip(hipHostMalloc((void**)&h->rep_host, batch_report_bytes(B), hipHostMallocMapped | hipHostMallocCoherent),
              "host alloc");
    check_hip(hipHostGetDevicePointer((void**)&h->rep_dev, h->rep_host, 0), "host pointer");
    h->rho = dalloc<double>(h, h->ldg);
    if (h->sparse && !h->arows) h->tbuf = dalloc<char>(h, (size_t)B * sparse_t_bytes(h->vals_f32, h->nnz));
    h->W = dalloc<double>(h, (size_t)B * h->ldg * h->ldg);
    h->Xd = reinterpret_cast<double*>(dalloc<char>(h, (size_t)B * chol_multi_x_bytes(h->ldg)));
    h->delta = dalloc<double>(h, h->ldg);
    h->npart = update_partials(h->m, h->tau);
    h->partials = dalloc<double>(h, h->npart);
    h->tr_u = dalloc<double>(h, 2 * h->K);
    if (!h->sparse) h->tr_upart = dalloc<double>(h, refresh_upart_doubles(h->m, h->K));
    h->tr_r = dalloc<double>(h, 2 * h->m);
    h->tr_part = dalloc<double>(h, refresh_partials(h->m));
    h->tr_zero = dalloc<int32_t>(h, 1);
    check_hip(hipMemset(h->tr_zero, 0, sizeof(int32_t)), "memset");
    if (o->dense_route == 1) {
      // the sketches' AS become gathers of tau columns of A, formed here by the product
      // kernel itself with every coordinate as one sketch (C = 0 .. m-1)
      h->ldgram = (h->m + 7) / 8 * 8;
      h->gram = dalloc<char>(h, gram_bytes);
      std::vector<int32_t> all(h->m);
      for (int64_t j = 0; j < h->m; ++j) all[j] = (int32_t)j;
      int32_t* d_all = dalloc<int32_t>(h, h->m);
      check_hip(hipMemcpy(d_all, all.data(), sizeof(int32_t) * h->m, hipMemcpyHostToDevice), "coordinates");
      if (h->mixed)
        check_hip(launch_as_dense_bf16(h->Zbf, h->kpad, h->m, h->kpad, d_all, (int32_t)h->m, h->ldgram, 1, h->lam,
                                       h->Z, h->ldz, h->kern ? 1 : 0, (float*)h->gram, h->tr_zero, h->stream),
                  "A = Z Z^T + lambda I (BF16)");
      else
        check_hip(launch_as_dense_f64(h->Z, h->ldz, h->m, h->K, d_all, (int32_t)h->m, h->ldgram, 1, h->lam,
                                      h->kern ? 1 : 0, (double*)h->gram, h->tr_zero, h->stream),
                  "A = Z Z^T + lambda I");
      check_hip(hipStreamSynchronize(h->stream), "sync");
    }
    h->hist_len = h->opt.max_iter + 1;
    h->hist = dalloc<double>(h, h->hist_len);
    h->true_hist = dalloc<double>(h, h->hist_len);
    h->flags = dalloc<DevFlags>(h, 1);
    h->err = dalloc<int32_t>(h, 1);
    for (int i = 0; i < 2; ++i) {
      h->xbuf[i] = dalloc<double>(h, h->m);
      h->rbuf[i] = dalloc<double>(h, h->m);
    }
    if (h->accel) {
      h->vbuf = dalloc<double>(h, h->m);
      h->rvbuf = dalloc<double>(h, h->m);
      h->rzbuf = dalloc<double>(h, h->m);
    }
    h->sampler = o->sampler;
    h->trace_every = o->trace_every;
    if (h->sampler != RS_SAMPLER_UNIFORM || h->trace_every > 0) {
      h->adiag = dalloc<double>(h, h->m);
      h->lstats = dalloc<double>(h, 3);
      h->log_rn = dalloc<double>(h, 1);
      h->last = dalloc<int32_t>(h, h->m);
      h->q = dalloc<float>(h, h->m);
      h->q_ok = dalloc<int32_t>(h, 1);
      if (h->mixed)
        check_hip(launch_adiag(h->Z32, 1, h->ld32, h->m, h->K, h->lam, h->adiag, h->lstats, s), "A_jj");
      else
        check_hip(launch_adiag(h->Z, 0, h->ldz, h->m, h->K, h->lam, h->adiag, h->lstats, s), "A_jj");
      check_hip(hipMemsetAsync(h->last, 0xFF, sizeof(int32_t) * h->m, s), "memset");  // -1: never sampled
      if (h->sampler == RS_SAMPLER_DIAG) {
        check_hip(launch_diag_q(h->adiag, h->lstats, h->m, h->q, s), "A_jj / Tr A");
        const int32_t one = 1;
        check_hip(hipMemcpy(h->q_ok, &one, sizeof(int32_t), hipMemcpyHostToDevice), "flag");
      }
      if (h->sampler == RS_SAMPLER_LEARNED) {
        h->feat = dalloc<float>(h, (size_t)h->m * kMlpFeatures);
        h->score = dalloc<float>(h, h->m);
        h->params = dalloc<float>(h, kMlpParams);
      }
      if (h->trace_every > 0) {
        h->trace_cap = o->trace_capacity > 0 ? o->trace_capacity : 1024;
        h->tr_F = dalloc<float>(h, (size_t)h->trace_cap * h->tau * kMlpFeatures);
        h->tr_c = dalloc<float>(h, (size_t)h->trace_cap * h->tau);
        h->tr_count = dalloc<int32_t>(h, 1);
        check_hip(hipMemsetAsync(h->tr_count, 0, sizeof(int32_t), s), "memset");
      }
    }
    if (o->profile) {
      // sketch, AS, G, Cholesky of this batch and of the one prepared ahead, the iteration
      // sequence; delta, update and refresh per iteration
      const int pairs = 9 + 3 * B + 2;
      h->ev.resize(2 * pairs);
      h->ev_cls.resize(pairs);
      h->ev_slots.resize(pairs);
      h->ev_batch.resize(pairs);
      for (auto& e : h->ev) check_hip(hipEventCreate(&e), "event create");
    }
    check_hip(hipMemsetAsync(h->err, 0, sizeof(int32_t), s), "memset");
    check_hip(launch_init_state(h->b, h->xbuf[0], h->xbuf[1], h->rbuf[0], h->rbuf[1], h->m,
                                h->partials, h->npart, h->flags, h->hist, s),
              "init");
    if (h->accel) check_hip(launch_init_accel(h->rbuf[0], h->vbuf, h->rvbuf, h->rzbuf, h->m, s), "init");
    DevFlags f{};
    check_hip(hipMemcpyAsync(&f, h->flags, sizeof(DevFlags), hipMemcpyDeviceToHost, s), "flags");
    check_hip(hipStreamSynchronize(s), "sync");
    h->done = f.done != 0;
    *out = h;
    return RS_OK;
  } catch (const Fail& f) {
    g_create_error = f.msg;
    dfree_all(h);
    delete h;
    return f.code;
  } catch (const std::exception& e) {
    g_create_error = e.what();
    dfree_all(h);
    delete h;
    return RS_EDEVICE;
  }
}

}  // namespace

extern "C" {

rs_status rs_create(const rs_matrix* X, const double* y, double lambda, const rs_options* o,
                    rs_handle** out) {
  return create_impl(X, y, lambda, 0.0, o, out);
}

rs_status rs_create_kernel(const rs_matrix* P, const double* y, double sigma, double lambda,
                           const rs_options* o, rs_handle** out) {
  if (!(sigma > 0.0) || !std::isfinite(sigma)) {
    g_create_error = "sigma must be positive and finite";
    if (out) *out = nullptr;
    return RS_EINVAL;
  }
  return create_impl(P, y, lambda, sigma, o, out);
}

rs_status rs_step(rs_handle* h, int64_t iters, double* rel_res_out) {
  if (!h || iters < 0) return RS_EINVAL;
  try {
    if (iters > 0) advance(h, iters);
    if (rel_res_out) {
      double v = 1.0;
      // mixed precision reports the FP64-refreshed residual (the tracked one drifts)
      const double* src = (h->mixed && h->k > 0) ? h->true_hist : h->hist;
      check_hip(hipMemcpy(&v, src + h->k, sizeof(double), hipMemcpyDeviceToHost), "hist");
      *rel_res_out = v;
    }
    return RS_OK;
  } catch (const Fail& f) {
    h->last_error = f.msg;
    return f.code;
  } catch (const std::exception& e) {
    h->last_error = e.what();
    return RS_EDEVICE;
  }
}

rs_status rs_reset(rs_handle* h, uint64_t seed) {
  if (!h) return RS_EINVAL;
  try {
    h->opt.seed = seed;
    h->k = 0;
    h->last_early = -1000000;
    h->done = false;
    h->batch_k0 = -1;
    h->batch_n = 0;
    for (int p = 0; p < h->nsets; ++p)
      check_hip(hipMemsetAsync(h->sets[p].status, 0, sizeof(int32_t) * h->B, h->stream), "memset");
    check_hip(hipMemsetAsync(h->err, 0, sizeof(int32_t), h->stream), "memset");
    if (h->last) check_hip(hipMemsetAsync(h->last, 0xFF, sizeof(int32_t) * h->m, h->stream), "memset");
    check_hip(launch_init_state(h->b, h->xbuf[0], h->xbuf[1], h->rbuf[0], h->rbuf[1], h->m,
                                h->partials, h->npart, h->flags, h->hist, h->stream),
              "init");
    if (h->accel)
      check_hip(launch_init_accel(h->rbuf[0], h->vbuf, h->rvbuf, h->rzbuf, h->m, h->stream), "init");
    DevFlags f{};
    check_hip(hipMemcpyAsync(&f, h->flags, sizeof(DevFlags), hipMemcpyDeviceToHost, h->stream), "flags");
    check_hip(hipStreamSynchronize(h->stream), "sync");
    h->done = f.done != 0;
    return RS_OK;
  } catch (const Fail& f) {
    h->last_error = f.msg;
    return f.code;
  } catch (const std::exception& e) {
    h->last_error = e.what();
    return RS_EDEVICE;
  }
}

rs_status rs_get_profile(rs_handle* h, rs_profile* out, int32_t clear) {
  if (!h || !out) return RS_EINVAL;
  if (!h->opt.profile) {
    h->last_error = "profiling was not enabled in rs_options";
    return RS_EINVAL;
  }
  *out = h->prof;
  if (clear) h->prof = rs_profile{};
  return RS_OK;
}

int64_t rs_iteration(const rs_handle* h) { return h ? h->k : -1; }
int64_t rs_system_size(const rs_handle* h) { return h ? h->m : -1; }
int32_t rs_sketch_size(const rs_handle* h) { return h ? h->tau : -1; }

rs_status rs_get_route(const rs_handle* h, int32_t* route, int64_t* a_nnz) {
  if (!h) return RS_EINVAL;
  if (route) *route = !h->sparse ? 0 : (h->arows ? RS_ROUTE_AROWS : RS_ROUTE_SCATTER);
  if (a_nnz) *a_nnz = h->a_nnz;
  return RS_OK;
}

rs_status rs_get_weights(rs_handle* h, double* w_out) {
  if (!h || !w_out) return RS_EINVAL;
  try {
    const double* x = h->xbuf[h->k & 1];
    if (h->form == RS_FORM_PRIMAL || h->kern) {
      check_hip(hipMemcpyAsync(w_out, x, sizeof(double) * h->d, hipMemcpyDeviceToHost, h->stream), "w");
    } else {
      double* wd = nullptr;
      check_hip(hipMalloc(&wd, sizeof(double) * h->d), "alloc");
      hipError_t e = h->sparse ? launch_spmv_csr(h->zt_ptr, h->zt_col, h->zt_val, h->vals_f32, h->d, x, wd,
                                                 h->stream)
                     : h->mixed ? launch_gemv_cols_f32(h->Z32, h->ld32, h->m, h->K, x, wd, h->stream)
                                : launch_gemv_cols(h->Z, h->ldz, h->m, h->K, x, wd, h->stream);
      if (e == hipSuccess)
        e = hipMemcpyAsync(w_out, wd, sizeof(double) * h->d, hipMemcpyDeviceToHost, h->stream);
      if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
      (void)hipFree(wd);
      check_hip(e, "w = X^T alpha");
    }
    check_hip(hipStreamSynchronize(h->stream), "sync");
    return RS_OK;
  } catch (const Fail& f) {
    h->last_error = f.msg;
    return f.code;
  } catch (const std::exception& e) {
    h->last_error = e.what();
    return RS_EDEVICE;
  }
}

rs_status rs_solve(rs_handle* h, double* w_out, rs_report* rep) {
  if (!h) return RS_EINVAL;
  try {
    const auto t0 = std::chrono::steady_clock::now();
    advance(h, h->opt.max_iter - h->k);
    const auto t1 = std::chrono::steady_clock::now();
    double rel = 1.0;
    const double* src = (h->mixed && h->k > 0) ? h->true_hist : h->hist;
    check_hip(hipMemcpy(&rel, src + h->k, sizeof(double), hipMemcpyDeviceToHost), "hist");
    if (rep) {
      rep->iters = h->k;
      rep->rel_res = rel;
      rep->seconds = std::chrono::duration<double>(t1 - t0).count();
      rep->rel_res_true = true_rel_res(h);
    }
    if (w_out) {
      rs_status st = rs_get_weights(h, w_out);
      if (st != RS_OK) return st;
    }
    return h->done ? RS_OK : RS_NOT_CONVERGED;
  } catch (const Fail& f) {
    h->last_error = f.msg;
    return f.code;
  } catch (const std::exception& e) {
    h->last_error = e.what();
    return RS_EDEVICE;
  }
}

rs_status rs_get_state(const rs_handle* h, double* x, double* x_prev, double* r, double* r_prev) {
  if (!h) return RS_EINVAL;
  const int cur = (int)(h->k & 1), prv = 1 - cur;
  const double* src[4] = {h->xbuf[cur], h->accel ? h->vbuf : h->xbuf[prv], h->rbuf[cur],
                          h->accel ? h->rvbuf : h->rbuf[prv]};
  double* dst[4] = {x, x_prev, r, r_prev};
  for (int i = 0; i < 4; ++i)
    if (dst[i] && hipMemcpy(dst[i], src[i], sizeof(double) * h->m, hipMemcpyDeviceToHost) != hipSuccess)
      return RS_EDEVICE;
  return RS_OK;
}

rs_status rs_set_state(rs_handle* h, int64_t k, const double* x, const double* x_prev, const double* r,
                       const double* r_prev) {
  if (!h) return RS_EINVAL;
  if (!x || !x_prev || !r || !r_prev || k < 0 || k > h->opt.max_iter) {
    h->last_error = "rs_set_state: four host vectors and 0 <= k <= max_iter are required";
    return RS_EINVAL;
  }
  if (h->accel || h->sampler == RS_SAMPLER_LEARNED) {
    h->last_error = "rs_set_state: not available for the accelerated method or the learned sampler";
    return RS_EUNSUPPORTED;
  }
  const double* src[4] = {x, x_prev, r, r_prev};
  for (int i = 0; i < 4; ++i)
    for (int64_t j = 0; j < h->m; ++j)
      if (!std::isfinite(src[i][j])) {
        h->last_error = "rs_set_state: non-finite entry";
        return RS_EINVAL;
      }
  double ss = 0.0;
  for (int64_t j = 0; j < h->m; ++j) ss += r[j] * r[j];
  try {
    check_hip(hipStreamSynchronize(h->stream), "sync");
    if (h->pipeline) check_hip(hipStreamSynchronize(h->prep_stream), "sync");
    DevFlags f{};
    check_hip(hipMemcpy(&f, h->flags, sizeof(DevFlags), hipMemcpyDeviceToHost), "flags");
    // x^k and r^k sit in buffer k & 1; the update overwrites the other (x^{k-1}, r^{k-1})
    const int cur = (int)(k & 1), prv = 1 - cur;
    double* dst[4] = {h->xbuf[cur], h->xbuf[prv], h->rbuf[cur], h->rbuf[prv]};
    for (int i = 0; i < 4; ++i)
      check_hip(hipMemcpy(dst[i], src[i], sizeof(double) * h->m, hipMemcpyHostToDevice), "state");
    // the stop test at iteration k sums the partials: one slot holds ||r^k||^2
    std::vector<double> part(h->npart, 0.0);
    part[0] = ss;
    check_hip(hipMemcpy(h->partials, part.data(), sizeof(double) * h->npart, hipMemcpyHostToDevice), "partials");
    const double rel = f.r0norm > 0.0 ? std::sqrt(ss) / f.r0norm : 0.0;
    check_hip(hipMemcpy(h->hist + k, &rel, sizeof(double), hipMemcpyHostToDevice), "history");
    check_hip(hipMemcpy(h->true_hist + k, &rel, sizeof(double), hipMemcpyHostToDevice), "history");
    f.done = (f.r0norm == 0.0) ? 1 : 0;  // as at creation: b = 0 leaves nothing to solve
    f.err = 0;
    f.k_done = 0;
    check_hip(hipMemcpy(h->flags, &f, sizeof(DevFlags), hipMemcpyHostToDevice), "flags");
    check_hip(hipMemset(h->err, 0, sizeof(int32_t)), "error word");
    // sampling ages (trace features) restart: no coordinate sampled yet
    if (h->last) check_hip(hipMemset(h->last, 0xFF, sizeof(int32_t) * h->m), "sketch history");
    h->k = k;
    h->done = f.done != 0;
    h->batch_k0 = -1;
    h->batch_n = 0;
    return RS_OK;
  } catch (const Fail& f) {
    h->last_error = f.msg;
    return f.code;
  } catch (const std::exception& e) {
    h->last_error = e.what();
    return RS_EDEVICE;
  }
}

rs_status rs_get_last_sketch(const rs_handle* h, int32_t* rows, int32_t* cols, int8_t* signs,
                             int64_t* nnz_out) {
  if (!h || !rows || !cols || !signs || !nnz_out) return RS_EINVAL;
  if (h->kind == kGaussian || h->kind == kSrht) return RS_EUNSUPPORTED;
  const int64_t it = h->k - 1;
  if (it < 0 || h->batch_k0 < 0 || it < h->batch_k0 || it >= h->batch_k0 + h->batch_n) return RS_EINVAL;
  const int64_t slot = it - h->batch_k0;
  try {
    std::vector<int32_t> mem(h->nsel), off(h->tau + 1), hm(h->m);
    if (hipMemcpy(mem.data(), h->members + slot * h->nsel, sizeof(int32_t) * h->nsel, hipMemcpyDeviceToHost) != hipSuccess ||
        hipMemcpy(off.data(), h->offs + slot * (h->tau + 1), sizeof(int32_t) * (h->tau + 1), hipMemcpyDeviceToHost) != hipSuccess ||
        hipMemcpy(hm.data(), h->hmap + slot * h->m, sizeof(int32_t) * h->m, hipMemcpyDeviceToHost) != hipSuccess)
      return RS_EDEVICE;
    int64_t c = 0;
    for (int b = 0; b < h->tau; ++b)
      for (int p = off[b]; p < off[b + 1]; ++p) {
        const int32_t j = mem[p];
        rows[c] = j;
        cols[c] = b;
        signs[c] = (hm[j] & 1) ? -1 : 1;
        ++c;
      }
    *nnz_out = c;
    return RS_OK;
  } catch (const std::exception&) {
    return RS_ENOMEM;  // host buffers
  }
}

rs_status rs_get_products(const rs_handle* h, double* as_out, double* ginv_out) {
  if (!h) return RS_EINVAL;
  const int64_t it = h->k - 1;
  if (it < 0 || h->batch_k0 < 0 || it < h->batch_k0 || it >= h->batch_k0 + h->batch_n) return RS_EINVAL;
  const int64_t slot = it - h->batch_k0;
  try {
    if (as_out) {
      const size_t elt = h->mixed ? sizeof(float) : sizeof(double);
      std::vector<char> buf((size_t)h->m * h->ldas * elt);
      if (hipMemcpy(buf.data(), (const char*)h->AS + (size_t)slot * h->m * h->ldas * elt, buf.size(),
                    hipMemcpyDeviceToHost) != hipSuccess)
        return RS_EDEVICE;
      for (int64_t j = 0; j < h->m; ++j)
        for (int64_t c = 0; c < h->tau; ++c) {
          const size_t idx = (size_t)j * h->ldas + c;
          as_out[j * h->tau + c] = h->mixed ? (double)((const float*)buf.data())[idx]
                                            : ((const double*)buf.data())[idx];
        }
    }
    if (ginv_out) {
      std::vector<double> g((size_t)h->ldg * h->ldg);
      if (hipMemcpy(g.data(), h->G + (size_t)slot * h->ldg * h->ldg, sizeof(double) * g.size(),
                    hipMemcpyDeviceToHost) != hipSuccess)
        return RS_EDEVICE;
      for (int64_t r = 0; r < h->tau; ++r)
        for (int64_t c = 0; c < h->tau; ++c) ginv_out[r * h->tau + c] = g[(size_t)r * h->ldg + c];
    }
    return RS_OK;
  } catch (const std::exception&) {
    return RS_ENOMEM;  // host buffers
  }
}

rs_status rs_get_history(const rs_handle* h, double* out, int64_t count) {
  if (!h || !out || count < 0 || count > h->k + 1) return RS_EINVAL;
  if (count && hipMemcpy(out, h->hist, sizeof(double) * count, hipMemcpyDeviceToHost) != hipSuccess)
    return RS_EDEVICE;
  return RS_OK;
}

rs_status rs_set_sampler_params(rs_handle* h, const float* params) {
  if (!h || !params) return RS_EINVAL;
  if (h->sampler != RS_SAMPLER_LEARNED) {
    h->last_error = "the handle was not created with the learned sampler";
    return RS_EINVAL;
  }
  for (int i = 0; i < kMlpParams; ++i)
    if (!std::isfinite(params[i])) {
      h->last_error = "sampler parameters must be finite";
      return RS_EINVAL;
    }
  if (hipMemcpy(h->params, params, sizeof(float) * kMlpParams, hipMemcpyHostToDevice) != hipSuccess)
    return RS_EDEVICE;
  h->params_set = true;
  return RS_OK;
}

rs_status rs_trace_count(const rs_handle* h, int64_t* count) {
  if (!h || !count) return RS_EINVAL;
  if (!h->tr_count) {
    *count = 0;
    return RS_OK;
  }
  int32_t c = 0;
  if (hipMemcpy(&c, h->tr_count, sizeof(int32_t), hipMemcpyDeviceToHost) != hipSuccess) return RS_EDEVICE;
  *count = std::min<int64_t>(c, h->trace_cap);
  return RS_OK;
}

rs_status rs_get_trace(const rs_handle* h, float* F, float* credits, int64_t first, int64_t count) {
  int64_t n = 0;
  rs_status st = rs_trace_count(h, &n);
  if (st != RS_OK) return st;
  if (first < 0 || count < 0 || first + count > n) return RS_EINVAL;
  const size_t rf = (size_t)h->tau * kMlpFeatures, rc = (size_t)h->tau;
  if (F && count &&
      hipMemcpy(F, h->tr_F + first * rf, sizeof(float) * rf * count, hipMemcpyDeviceToHost) != hipSuccess)
    return RS_EDEVICE;
  if (credits && count &&
      hipMemcpy(credits, h->tr_c + first * rc, sizeof(float) * rc * count, hipMemcpyDeviceToHost) != hipSuccess)
    return RS_EDEVICE;
  return RS_OK;
}

rs_status rs_get_proposal(const rs_handle* h, float* q, int32_t* ok) {
  if (!h || !q || !h->q) return RS_EINVAL;
  if (hipMemcpy(q, h->q, sizeof(float) * h->m, hipMemcpyDeviceToHost) != hipSuccess) return RS_EDEVICE;
  if (ok && hipMemcpy(ok, h->q_ok, sizeof(int32_t), hipMemcpyDeviceToHost) != hipSuccess) return RS_EDEVICE;
  return RS_OK;
}

rs_status rs_destroy(rs_handle* h) {
  if (!h) return RS_EINVAL;
  if (h->stream) (void)hipStreamSynchronize(h->stream); else (void)hipDeviceSynchronize();
  dfree_all(h);
  delete h;
  return RS_OK;
}

}  // extern "C"
