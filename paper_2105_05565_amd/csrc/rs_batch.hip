// Host runtime of the batched solver (rs_batch_* in include/rs.h).
//
// Many ridge problems of different shapes, each with a grid of regularisers and
// several right-hand sides, advance in lock step. One iteration is a fixed sequence of
// device-wide launches over ragged work tables built here once:
//   sketch draw (one workgroup per problem) -> B S = Z (Z^T S) (dense: 64 x 64 FP64 MFMA
//   tiles of every problem; CSR: count-sketch scatter-add, one workgroup per bucket) ->
//   S^T A(lambda) S assembly, Cholesky and inverse (one workgroup per (problem, lambda)) ->
//   rho = S^T R -> Delta = G^{-1} rho -> momentum update of all slots -> stop tests.
// Every launch runs a fixed grid of workgroups that strides over its table (persistent
// launch), and each reads the iteration counter and the per-problem stop words from
// device memory, so the sequence is captured once into a HIP graph (several iterations
// per graph) and replayed until every problem has stopped. The first solve can time
// alternative launch shapes of the iterate-independent kernels on the real tables and
// keep the fastest (autotuner).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <functional>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "momentum.h"
#include "rs_internal.h"

using namespace rs;

namespace {

struct Fail {
  rs_status code;
  std::string msg;
};

void check_hip(hipError_t e, const char* what) {
  if (e != hipSuccess) throw Fail{RS_EDEVICE, std::string(what) + ": " + hipGetErrorString(e)};
}

// Host-side record of one problem.
struct BProb {
  int64_t n = 0, d = 0, m = 0, K = 0;
  int form = RS_FORM_PRIMAL;
  bool sparse = false;
  int kind = kSubsample;
  int tau = 0, nlam = 0, nrhs = 0, J = 0;
  int64_t ldg = 0, ldas = 0, cap = 0;
  int ntiles = 0;
  // device data
  double* Z = nullptr;  // dense m x K
  uint16_t* Zbf = nullptr;  // mixed precision: BF16 copy (m x kpad, zero padded)
  int64_t kpad = 0;
  int64_t* zr_ptr = nullptr;
  int32_t* zr_col = nullptr;
  double* zr_val = nullptr;
  int64_t* zt_ptr = nullptr;
  int32_t* zt_col = nullptr;
  double* zt_val = nullptr;
  int64_t nnz = 0;
  double* x[2] = {nullptr, nullptr};
  int64_t* stop_k = nullptr;
  double* rel = nullptr;
  int64_t* iters = nullptr;
};

// Launch shapes chosen by the tuner (workgroups = multiplier x compute units).
struct Tuning {
  int dense_tk = 16;
  int dense_mult = 4;
  int sparse_mult = 4;
  int chol_mult = 1;
  double dense_ms = -1.0, sparse_ms = -1.0, chol_ms = -1.0;
  int tuned = 0;
};

std::mutex g_tune_mu;
std::map<std::string, Tuning> g_tune_cache;  // shape signature -> tuned shapes (per process)

thread_local std::string g_batch_create_error;

}  // namespace

struct rs_batch {
  rs_options opt{};
  hipStream_t stream = nullptr;
  bool own_stream = false;
  int cus = 256;
  std::vector<BProb> P;
  std::vector<void*> allocs;
  std::string last_error;

  // device tables
  BState* S = nullptr;
  BGlobal* g = nullptr;
  double* betas = nullptr;
  double* gammas = nullptr;
  SketchArgs* sk_sub = nullptr;
  int n_sub = 0;
  size_t lds_sub = 0;
  SketchArgs* sk_cnt = nullptr;
  int n_cnt = 0;
  size_t lds_cnt = 0;
  DenseJob* djobs = nullptr;
  DenseTile* dtiles = nullptr;
  int n_dtiles = 0;
  bool mixed = false;          // BF16 products for the dense problems, FP64 refresh
  DenseBf16Job* bjobs = nullptr;
  DenseTile* btiles = nullptr;
  int n_btiles = 0;
  int32_t* ref_u = nullptr;    // refresh work items (p, K tile, h)
  int n_ref_u = 0;
  int32_t* ref_r = nullptr;    // (p, row tile, h)
  int n_ref_r = 0;
  SparseJob* sjobs = nullptr;
  int n_sjobs = 0;
  int32_t* sitems = nullptr;
  int n_sitems = 0;
  int max_sparse_tau = 0;
  CholJob* cjobs = nullptr;
  int n_cjobs = 0;
  int32_t* cstatus = nullptr;
  int32_t* rho_items = nullptr;
  int n_rho = 0;
  int32_t* delta_items = nullptr;
  int n_delta = 0;
  int32_t* upd_items = nullptr;
  int n_upd = 0;
  int32_t* err = nullptr;

  Tuning tune;
  std::string signature;
  int graph_iters = 8;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  int64_t k = 0;
  bool done = false;
};

namespace {

template <class T>
T* dalloc(rs_batch* b, size_t count) {
  if (count == 0) count = 1;
  void* p = nullptr;
  hipError_t e = hipMalloc(&p, sizeof(T) * count);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    throw Fail{RS_ENOMEM, "hipMalloc of " + std::to_string(sizeof(T) * count) + " bytes failed"};
  }
  b->allocs.push_back(p);
  return static_cast<T*>(p);
}

template <class T>
T* upload(rs_batch* b, const std::vector<T>& v) {
  T* d = dalloc<T>(b, v.size());
  if (!v.empty())
    check_hip(hipMemcpy(d, v.data(), sizeof(T) * v.size(), hipMemcpyHostToDevice), "table upload");
  return d;
}

void free_all(rs_batch* b) {
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  b->exec = nullptr;
  b->graph = nullptr;
  for (void* p : b->allocs) (void)hipFree(p);
  b->allocs.clear();
  if (b->own_stream && b->stream) (void)hipStreamDestroy(b->stream);
  b->stream = nullptr;
}

// Host arithmetic below in a fixed operation order (no contraction).
#pragma clang fp contract(off)

// Default sketch size of a batched problem: a multiple of 64 near m^{2/3}, in [64, 512].
int default_tau(int64_t m) {
  const double t = 64.0 * std::floor(std::pow((double)m, 2.0 / 3.0) / 64.0 + 0.5);
  int tau = (int)std::min(512.0, std::max(64.0, t));
  return (int)std::min<int64_t>(tau, m);
}

// Upload one problem's data into the device layouts (as a single solve does) and form b.
void setup_problem(rs_batch* B, int p, const rs_problem& pr, BProb& q, double* b_dev) {
  hipStream_t s = B->stream;
  const rs_matrix& X = pr.X;
  const bool f32 = X.dtype == RS_F32;
  const size_t esz = f32 ? 4 : 8;
  const auto kind_copy = X.mem == RS_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
  // right-hand sides: validate on the host, then one column at a time
  std::vector<double> yh((size_t)q.n * q.nrhs);
  if (X.mem == RS_DEVICE)
    check_hip(hipMemcpy(yh.data(), pr.y, sizeof(double) * yh.size(), hipMemcpyDeviceToHost), "y download");
  else
    std::memcpy(yh.data(), pr.y, sizeof(double) * yh.size());
  for (double v : yh)
    if (!std::isfinite(v)) throw Fail{RS_EINVAL, "problem " + std::to_string(p) + ": y has a non-finite entry"};
  double* yd = dalloc<double>(B, yh.size());
  check_hip(hipMemcpy(yd, yh.data(), sizeof(double) * yh.size(), hipMemcpyHostToDevice), "y upload");
  double* col = dalloc<double>(B, q.m);

  if (!q.sparse) {
    const size_t total = (size_t)q.n * q.d;
    void* xv = dalloc<char>(B, total * esz);
    check_hip(hipMemcpyAsync(xv, X.vals, total * esz, kind_copy, s), "X upload");
    const bool rowmajor = X.layout == RS_DENSE_ROWMAJOR;
    const bool need_transpose = (q.form == RS_FORM_PRIMAL) == rowmajor;
    q.Z = dalloc<double>(B, (size_t)q.m * q.K);
    const int64_t rows = rowmajor ? q.n : q.d, cols = rowmajor ? q.d : q.n;
    if (need_transpose)
      check_hip(launch_transpose_to_f64(xv, f32, rows, cols, cols, q.Z, q.K, s), "transpose");
    else
      check_hip(launch_copy_to_f64(xv, f32, rows, cols, cols, q.Z, q.K, s), "copy");
    for (int r = 0; r < q.nrhs; ++r) {
      const double* yr = yd + (size_t)r * q.n;
      if (q.form == RS_FORM_PRIMAL) {
        check_hip(launch_gemv_rows(q.Z, q.K, q.m, q.K, yr, col, s), "b = X^T y");
        check_hip(launch_bcol(col, q.m, 1, 0, b_dev, q.nrhs, r, s), "b");
      } else {
        check_hip(launch_bcol(yr, q.m, 1, 0, b_dev, q.nrhs, r, s), "b = y");
      }
    }
    check_hip(hipStreamSynchronize(s), "sync");
    (void)hipFree(xv);
    B->allocs.erase(std::find(B->allocs.begin(), B->allocs.end(), xv));
  } else {
    const int64_t n = q.n, d = q.d, nnz = X.nnz;
    if (nnz > INT32_MAX) throw Fail{RS_EINVAL, "nnz must fit in int32"};
    std::vector<int64_t> ph(n + 1);
    if (X.mem == RS_DEVICE)
      check_hip(hipMemcpy(ph.data(), X.row_ptr, sizeof(int64_t) * (n + 1), hipMemcpyDeviceToHost), "row_ptr");
    else
      std::memcpy(ph.data(), X.row_ptr, sizeof(int64_t) * (n + 1));
    if (ph[0] != 0 || ph[n] != nnz) throw Fail{RS_EINVAL, "row_ptr must start at 0 and end at nnz"};
    for (int64_t i = 0; i < n; ++i)
      if (ph[i + 1] < ph[i]) throw Fail{RS_EINVAL, "row_ptr must be non-decreasing"};
    std::vector<int32_t> ch(nnz);
    if (nnz) {
      if (X.mem == RS_DEVICE)
        check_hip(hipMemcpy(ch.data(), X.col_idx, sizeof(int32_t) * nnz, hipMemcpyDeviceToHost), "col_idx");
      else
        std::memcpy(ch.data(), X.col_idx, sizeof(int32_t) * nnz);
    }
    for (int64_t i = 0; i < n; ++i)
      for (int64_t e = ph[i]; e < ph[i + 1]; ++e)
        if (ch[e] < 0 || ch[e] >= d || (e > ph[i] && ch[e] <= ch[e - 1]))
          throw Fail{RS_EINVAL, "col_idx must be in [0, d) and strictly increasing within a row"};
    int64_t* xptr = dalloc<int64_t>(B, n + 1);
    int32_t* xcol = dalloc<int32_t>(B, nnz);
    double* xval = dalloc<double>(B, nnz);
    check_hip(hipMemcpy(xptr, ph.data(), sizeof(int64_t) * (n + 1), hipMemcpyHostToDevice), "upload");
    if (nnz) {
      check_hip(hipMemcpy(xcol, ch.data(), sizeof(int32_t) * nnz, hipMemcpyHostToDevice), "upload");
      void* raw = dalloc<char>(B, (size_t)nnz * esz);
      check_hip(hipMemcpyAsync(raw, X.vals, (size_t)nnz * esz, kind_copy, s), "X upload");
      check_hip(launch_vec_to_f64(raw, f32, nnz, xval, s), "values to FP64");
    }
    int64_t* tptr = dalloc<int64_t>(B, d + 1);
    int32_t* tcol = dalloc<int32_t>(B, nnz);
    double* tval = dalloc<double>(B, nnz);
    check_hip(csr_transpose(xptr, xcol, xval, 0, n, d, nnz, tptr, tcol, tval, s), "transpose");
    q.nnz = nnz;
    if (q.form == RS_FORM_PRIMAL) {
      q.zr_ptr = tptr; q.zr_col = tcol; q.zr_val = tval;  // Z = X^T
      q.zt_ptr = xptr; q.zt_col = xcol; q.zt_val = xval;
    } else {
      q.zr_ptr = xptr; q.zr_col = xcol; q.zr_val = xval;  // Z = X
      q.zt_ptr = tptr; q.zt_col = tcol; q.zt_val = tval;
    }
    for (int r = 0; r < q.nrhs; ++r) {
      const double* yr = yd + (size_t)r * n;
      if (q.form == RS_FORM_PRIMAL) {
        check_hip(launch_spmv_csr(q.zr_ptr, q.zr_col, q.zr_val, 0, q.m, yr, col, s), "b = X^T y");
        check_hip(launch_bcol(col, q.m, 1, 0, b_dev, q.nrhs, r, s), "b");
      } else {
        check_hip(launch_bcol(yr, q.m, 1, 0, b_dev, q.nrhs, r, s), "b = y");
      }
    }
  }
}

// One lock-step iteration: the fixed launch sequence (captured into the graph).
void enqueue_iteration(rs_batch* B) {
  hipStream_t s = B->stream;
  const Tuning& t = B->tune;
  check_hip(launch_sketch_tab(B->sk_sub, B->n_sub, kSubsample, B->lds_sub, s), "sketch (subsample)");
  check_hip(launch_sketch_tab(B->sk_cnt, B->n_cnt, kCount, B->lds_cnt, s), "sketch (count)");
  check_hip(launch_sparse_tab(B->sjobs, B->n_sjobs, B->sitems, B->n_sitems, B->max_sparse_tau,
                              t.sparse_mult * B->cus, s),
            "B S (count)");
  if (B->mixed)
    check_hip(launch_as_dense_bf16_tab(B->bjobs, B->btiles, B->n_btiles, s), "B S (dense, BF16)");
  else
    check_hip(launch_as_dense_f64_tab(B->djobs, B->dtiles, B->n_dtiles, t.dense_tk, t.dense_mult * B->cus, s),
              "B S (dense)");
  check_hip(launch_chol_tab(B->cjobs, B->n_cjobs, t.chol_mult * B->cus, s), "cholesky");
  check_hip(launch_brho(B->S, B->rho_items, B->n_rho, B->g, 8 * B->cus, s), "rho");
  check_hip(launch_bdelta(B->S, B->delta_items, B->n_delta, 8 * B->cus, s), "delta");
  check_hip(launch_bupdate(B->S, B->upd_items, B->n_upd, B->g, B->betas, B->gammas, 2 * B->cus, s),
            "update");
  if (B->mixed)
    check_hip(launch_brefresh(B->S, B->ref_u, B->n_ref_u, B->ref_r, B->n_ref_r, B->g, 4 * B->cus, s), "refresh");
  check_hip(launch_bfinal(B->S, (int)B->P.size(), B->g, B->opt.tol, s), "stop test");
}

// Read back the counter and the stop word after a synchronisation; raise on errors.
void sync_state(rs_batch* B) {
  BGlobal gh{};
  int32_t err = 0;
  std::vector<int32_t> st(B->n_cjobs);
  check_hip(hipMemcpyAsync(&gh, B->g, sizeof(BGlobal), hipMemcpyDeviceToHost, B->stream), "state");
  check_hip(hipMemcpyAsync(&err, B->err, sizeof(int32_t), hipMemcpyDeviceToHost, B->stream), "err");
  if (B->n_cjobs)
    check_hip(hipMemcpyAsync(st.data(), B->cstatus, sizeof(int32_t) * B->n_cjobs, hipMemcpyDeviceToHost,
                             B->stream),
              "status");
  check_hip(hipStreamSynchronize(B->stream), "sync");
  if (err) throw Fail{RS_EDEVICE, "internal sketch limit hit (code " + std::to_string(err) + ")"};
  for (int32_t v : st)
    if (v) throw Fail{RS_ESINGULAR, "non-positive pivot in the Cholesky factorisation of S^T A S"};
  B->k = gh.k;
  B->done = gh.done != 0;
}

void ensure_graph(rs_batch* B) {
  if (B->exec || B->graph_iters <= 0) return;
  check_hip(hipStreamBeginCapture(B->stream, hipStreamCaptureModeThreadLocal), "begin capture");
  try {
    for (int i = 0; i < B->graph_iters; ++i) enqueue_iteration(B);
  } catch (...) {
    hipGraph_t gr = nullptr;
    (void)hipStreamEndCapture(B->stream, &gr);
    if (gr) (void)hipGraphDestroy(gr);
    throw;
  }
  check_hip(hipStreamEndCapture(B->stream, &B->graph), "end capture");
  check_hip(hipGraphInstantiate(&B->exec, B->graph, nullptr, nullptr, 0), "graph instantiate");
}

// Time the iterate-independent launches (B S, factorisations) over candidate shapes on
// the batch's own tables and keep the fastest. The state is untouched: these kernels only
// rewrite products of the current sketch.
float time_launch(rs_batch* B, const std::function<void()>& f) {
  hipEvent_t e0, e1;
  check_hip(hipEventCreate(&e0), "event");
  check_hip(hipEventCreate(&e1), "event");
  f();  // warm
  float best = 1e30f;
  for (int rep = 0; rep < 2; ++rep) {
    check_hip(hipEventRecord(e0, B->stream), "event");
    f();
    check_hip(hipEventRecord(e1, B->stream), "event");
    check_hip(hipEventSynchronize(e1), "event");
    float ms = 0.0f;
    check_hip(hipEventElapsedTime(&ms, e0, e1), "elapsed");
    best = std::min(best, ms);
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return best;
}

void autotune(rs_batch* B) {
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tune_cache.find(B->signature);
    if (it != g_tune_cache.end()) {
      B->tune = it->second;
      return;
    }
  }
  hipStream_t s = B->stream;
  // sketches of the current iteration (the draw is a pure function of (seed, p, k))
  check_hip(launch_sketch_tab(B->sk_sub, B->n_sub, kSubsample, B->lds_sub, s), "sketch");
  check_hip(launch_sketch_tab(B->sk_cnt, B->n_cnt, kCount, B->lds_cnt, s), "sketch");
  Tuning t = B->tune;
  if (B->mixed && B->n_btiles) {
    // one workgroup per tile: nothing to choose, the launch is timed for the report
    t.dense_ms = time_launch(B, [&] {
      check_hip(launch_as_dense_bf16_tab(B->bjobs, B->btiles, B->n_btiles, s), "tune");
    });
  }
  if (B->n_dtiles && !B->mixed) {
    float best = 1e30f;
    for (int tk : {16})  // the product's K-panel depth (fixed)
      for (int mult : {1, 2, 4, 8}) {
        const float ms = time_launch(B, [&] {
          check_hip(launch_as_dense_f64_tab(B->djobs, B->dtiles, B->n_dtiles, tk, mult * B->cus, s), "tune");
        });
        if (ms < best) {
          best = ms;
          t.dense_tk = tk;
          t.dense_mult = mult;
        }
      }
    t.dense_ms = best;
  }
  if (B->n_sjobs) {
    float best = 1e30f;
    for (int mult : {1, 2, 4, 8}) {
      const float ms = time_launch(B, [&] {
        check_hip(launch_sparse_tab(B->sjobs, B->n_sjobs, B->sitems, B->n_sitems, B->max_sparse_tau,
                                    mult * B->cus, s),
                  "tune");
      });
      if (ms < best) {
        best = ms;
        t.sparse_mult = mult;
      }
    }
    t.sparse_ms = best;
  }
  if (B->n_cjobs) {
    float best = 1e30f;
    for (int mult : {1, 2}) {
      const float ms = time_launch(B, [&] {
        check_hip(launch_chol_tab(B->cjobs, B->n_cjobs, mult * B->cus, s), "tune");
      });
      if (ms < best) {
        best = ms;
        t.chol_mult = mult;
      }
    }
    t.chol_ms = best;
    // the factorisation status words are sticky: clear what the timing runs left
    check_hip(hipMemsetAsync(B->cstatus, 0, sizeof(int32_t) * B->n_cjobs, s), "memset");
  }
  t.tuned = 1;
  B->tune = t;
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tune_cache[B->signature] = t;
}

void init_state(rs_batch* B) {
  check_hip(hipMemsetAsync(B->cstatus, 0, sizeof(int32_t) * std::max(1, B->n_cjobs), B->stream), "memset");
  check_hip(hipMemsetAsync(B->err, 0, sizeof(int32_t), B->stream), "memset");
  check_hip(hipMemsetAsync(B->g, 0, sizeof(BGlobal), B->stream), "memset");
  check_hip(launch_binit(B->S, (int)B->P.size(), B->g, B->stream), "init");
  sync_state(B);
}

// Iteration whose iterate problem p's buffers hold: the problem's own count once it
// has stopped (later lock-step iterations skip it), else the shared counter.
int64_t problem_k(const rs_batch* B, int p) {
  const BState* dev = B->S + p;
  BState st{};
  int32_t inactive = 0;
  int64_t it = 0;
  check_hip(hipMemcpy(&st, dev, sizeof(BState), hipMemcpyDeviceToHost), "state");
  check_hip(hipMemcpy(&inactive, st.inactive, sizeof(int32_t), hipMemcpyDeviceToHost), "state");
  check_hip(hipMemcpy(&it, st.iters, sizeof(int64_t), hipMemcpyDeviceToHost), "state");
  return inactive ? it : B->k;
}

}  // namespace

extern "C" {

rs_status rs_batch_create(int32_t count, const rs_problem* problems, const rs_options* o,
                          rs_batch** out) {
  g_batch_create_error.clear();
  if (count <= 0 || !problems || !o || !out) {
    g_batch_create_error = "null argument or count <= 0";
    return RS_EINVAL;
  }
  *out = nullptr;
  rs_batch* B = new rs_batch();
  try {
    B->opt = *o;
    if (o->precision != RS_PREC_FP64 && o->precision != RS_PREC_MIXED_BF16)
      throw Fail{RS_EINVAL, "unknown precision"};
    B->mixed = o->precision == RS_PREC_MIXED_BF16;
    const int32_t refresh_every = o->refresh_every > 0 ? o->refresh_every : 20;
    if (o->dense_route != 0)
      throw Fail{RS_EUNSUPPORTED, "batched solves form B S per sketch (dense_route must be 0)"};
    if (const char* why = momentum_invalid(*o)) throw Fail{RS_EINVAL, why};
    if (!(o->tol >= 0.0)) throw Fail{RS_EINVAL, "tol must be >= 0"};
    if (o->max_iter < 0 || o->max_iter > 100000000) throw Fail{RS_EINVAL, "max_iter out of range"};
    B->graph_iters = o->graph_iters == 0 ? 8 : (o->graph_iters < 0 ? 0 : o->graph_iters);

    // validation and host-side plan (no device call before it)
    B->P.resize(count);
    int64_t max_cap = 0;
    for (int p = 0; p < count; ++p) {
      const rs_problem& pr = problems[p];
      BProb& q = B->P[p];
      const rs_matrix& X = pr.X;
      const std::string tag = "problem " + std::to_string(p) + ": ";
      if (X.n <= 0 || X.d <= 0 || X.n > INT32_MAX || X.d > INT32_MAX)
        throw Fail{RS_EINVAL, tag + "X must have 1 <= n, d < 2^31"};
      if (X.dtype != RS_F64 && X.dtype != RS_F32) throw Fail{RS_EINVAL, tag + "dtype must be RS_F64 or RS_F32"};
      if (X.mem != RS_HOST && X.mem != RS_DEVICE) throw Fail{RS_EINVAL, tag + "mem must be RS_HOST or RS_DEVICE"};
      if (X.layout != RS_DENSE_ROWMAJOR && X.layout != RS_DENSE_COLMAJOR && X.layout != RS_CSR)
        throw Fail{RS_EINVAL, tag + "unknown layout"};
      if (!X.vals || !pr.y || !pr.lambdas) throw Fail{RS_EINVAL, tag + "null X.vals, y or lambdas"};
      if (X.layout == RS_CSR && (!X.row_ptr || !X.col_idx || X.nnz < 0))
        throw Fail{RS_EINVAL, tag + "CSR needs row_ptr, col_idx and nnz >= 0"};
      if (pr.nrhs < 1 || pr.nrhs > 8) throw Fail{RS_EINVAL, tag + "nrhs must be in [1, 8]"};
      if (pr.nlambda < 1 || pr.nlambda * pr.nrhs > 64)
        throw Fail{RS_EINVAL, tag + "need nlambda >= 1 and nlambda * nrhs <= 64"};
      for (int l = 0; l < pr.nlambda; ++l)
        if (!(pr.lambdas[l] > 0.0) || !std::isfinite(pr.lambdas[l]))
          throw Fail{RS_EINVAL, tag + "every lambda must be positive and finite"};
      q.n = X.n;
      q.d = X.d;
      const int form = pr.form == RS_FORM_AUTO ? (q.d <= q.n ? RS_FORM_PRIMAL : RS_FORM_DUAL) : pr.form;
      if (form != RS_FORM_PRIMAL && form != RS_FORM_DUAL) throw Fail{RS_EINVAL, tag + "unknown form"};
      q.form = form;
      q.m = form == RS_FORM_PRIMAL ? q.d : q.n;
      q.K = form == RS_FORM_PRIMAL ? q.n : q.d;
      q.sparse = X.layout == RS_CSR;
      const int sketch = pr.sketch < 0 ? (q.sparse ? RS_SKETCH_COUNT : RS_SKETCH_SUBSAMPLE) : pr.sketch;
      if (sketch == RS_SKETCH_SUBSAMPLE && !q.sparse) q.kind = kSubsample;
      else if (sketch == RS_SKETCH_COUNT && q.sparse) q.kind = kCount;
      else throw Fail{RS_EUNSUPPORTED, tag + "batched solves use the subsample sketch for dense X and the count sketch for CSR X"};
      q.tau = pr.tau > 0 ? pr.tau : default_tau(q.m);
      if (q.tau > q.m || q.tau > 1024) throw Fail{RS_EINVAL, tag + "tau must satisfy 1 <= tau <= min(m, 1024)"};
      q.nlam = pr.nlambda;
      q.nrhs = pr.nrhs;
      q.J = q.nlam * q.nrhs;
      q.ldg = ((int64_t)q.tau + 63) / 64 * 64;
      q.ldas = q.ldg;
      q.cap = pr.max_iter > 0 ? std::min<int64_t>(pr.max_iter, o->max_iter) : o->max_iter;
      q.ntiles = (int)((q.m + 63) / 64);
      max_cap = std::max(max_cap, q.cap);
    }

    if (o->stream) {
      B->stream = static_cast<hipStream_t>(o->stream);
    } else {
      // graph capture needs a stream other than the legacy default stream
      check_hip(hipStreamCreateWithFlags(&B->stream, hipStreamNonBlocking), "stream");
      B->own_stream = true;
    }
    int dev = 0;
    check_hip(hipGetDevice(&dev), "device");
    check_hip(hipDeviceGetAttribute(&B->cus, hipDeviceAttributeMultiprocessorCount, dev), "attribute");
    hipStream_t s = B->stream;
    B->err = dalloc<int32_t>(B, 1);
    B->g = dalloc<BGlobal>(B, 1);
    std::vector<BState> hs(count);
    std::vector<SketchArgs> sub, cnt;
    std::vector<DenseJob> dj;
    std::vector<DenseTile> dt;
    std::vector<DenseBf16Job> bj;
    std::vector<DenseTile> bft;
    std::vector<int32_t> ru, rr;
    std::vector<SparseJob> sj;
    std::vector<int32_t> si, rho_it, del_it, upd_it;
    std::vector<CholJob> cj;
    std::string sig;
    int32_t* inactive = dalloc<int32_t>(B, count);
    int64_t* iters = dalloc<int64_t>(B, count);
    std::vector<std::pair<int64_t, CholJob>> chol_order;
    for (int p = 0; p < count; ++p) {
      const rs_problem& pr = problems[p];
      BProb& q = B->P[p];
      BState& st = hs[p];
      double* b_dev = dalloc<double>(B, (size_t)q.m * q.nrhs);
      setup_problem(B, p, pr, q, b_dev);
      const int64_t m = q.m, ldg = q.ldg;
      int32_t* hmap = dalloc<int32_t>(B, m);
      const int64_t nsel = q.kind == kCount ? m : q.tau;
      int32_t* members = dalloc<int32_t>(B, nsel);
      int32_t* offs = dalloc<int32_t>(B, q.tau + 1);
      uint64_t* keys = q.kind == kSubsample ? dalloc<uint64_t>(B, m) : nullptr;
      double* BS = dalloc<double>(B, (size_t)m * q.ldas);
      check_hip(hipMemsetAsync(BS, 0, sizeof(double) * m * q.ldas, s), "memset");  // padding stays 0
      double* G0 = q.kind == kCount ? dalloc<double>(B, (size_t)ldg * ldg) : nullptr;
      double* Ginv = dalloc<double>(B, (size_t)q.nlam * ldg * ldg);
      double* U = dalloc<double>(B, (size_t)q.nlam * ldg * ldg);
      double* lam = dalloc<double>(B, q.nlam);
      check_hip(hipMemcpy(lam, pr.lambdas, sizeof(double) * q.nlam, hipMemcpyHostToDevice), "lambdas");
      for (int i = 0; i < 2; ++i) {
        q.x[i] = dalloc<double>(B, (size_t)m * q.J);
        st.r[i] = dalloc<double>(B, (size_t)m * q.J);
        st.x[i] = q.x[i];
      }
      st.rho = dalloc<double>(B, (size_t)q.J * ldg);
      st.delta = dalloc<double>(B, (size_t)q.J * ldg);
      check_hip(hipMemsetAsync(st.delta, 0, sizeof(double) * q.J * ldg, s), "memset");
      check_hip(hipMemsetAsync(st.rho, 0, sizeof(double) * q.J * ldg, s), "memset");
      st.partials = dalloc<double>(B, (size_t)q.ntiles * q.J);
      st.r0n = dalloc<double>(B, q.J);
      q.stop_k = st.stop_k = dalloc<int64_t>(B, q.J);
      q.rel = st.rel = dalloc<double>(B, q.J);
      st.m = m;
      st.J = q.J;
      st.nrhs = q.nrhs;
      st.nlam = q.nlam;
      st.tau = q.tau;
      st.ldg = ldg;
      st.ldas = q.ldas;
      st.BS = BS;
      st.Ginv = Ginv;
      st.hmap = hmap;
      st.members = members;
      st.offs = offs;
      st.lam = lam;
      st.b = b_dev;
      st.ntiles = q.ntiles;
      st.inactive = inactive + p;
      st.cap = q.cap;
      q.iters = st.iters = iters + p;

      SketchArgs a{};
      a.kind = q.kind;
      a.m = m;
      a.tau = q.tau;
      a.nsel = nsel;
      a.seed = o->seed;
      a.pid = o->problem_id + (uint64_t)p;
      a.nslots = 1;
      a.hmap = hmap;
      a.members = members;
      a.offs = offs;
      a.keys = keys;
      a.err = B->err;
      a.done = st.inactive;
      a.kdev = &B->g->k;
      if (q.kind == kSubsample) {
        sub.push_back(a);
        B->lds_sub = std::max(B->lds_sub, sketch_lds_bytes(kSubsample, q.tau, nsel));
        if (B->mixed) {
          // BF16 copy for the products; the FP64 Z stays for the refresh
          q.kpad = (q.K + 63) / 64 * 64;
          q.Zbf = dalloc<uint16_t>(B, (size_t)m * q.kpad);
          check_hip(launch_cast_bf16(q.Z, 0, m, q.K, q.K, 0, q.Zbf, q.kpad, nullptr, 0, s), "BF16 copy");
          DenseBf16Job j{q.Zbf, q.kpad, m, q.kpad, members, q.tau, q.ldas, BS, st.inactive};
          const int jid = (int)bj.size();
          bj.push_back(j);
          const int tr = bf16_tile_rows(), tc = bf16_tile_cols();
          for (int tn = 0; tn < (q.tau + tc - 1) / tc; ++tn)
            for (int tm = 0; tm < (int)((m + tr - 1) / tr); ++tm) bft.push_back(DenseTile{jid, tm, tn});
          st.refresh = refresh_every;
          st.Z = q.Z;
          st.ldz = q.K;
          st.K = q.K;
          st.Uref = dalloc<double>(B, (size_t)2 * q.K * q.J);
          for (int h = 0; h < 2; ++h) {
            for (int kt = 0; kt < (int)((q.K + 63) / 64); ++kt) {
              ru.push_back(p);
              ru.push_back(kt);
              ru.push_back(h);
            }
            for (int rt = 0; rt < q.ntiles; ++rt) {
              rr.push_back(p);
              rr.push_back(rt);
              rr.push_back(h);
            }
          }
        } else {
          DenseJob j{q.Z, q.K, m, q.K, members, q.tau, q.ldas, 0.0, BS, st.inactive};
          const int jid = (int)dj.size();
          dj.push_back(j);
          // 128 x 128 product tiles (the kernel's unit)
          for (int tn = 0; tn < (q.tau + 127) / 128; ++tn)
            for (int tm = 0; tm < (int)((m + 127) / 128); ++tm) dt.push_back(DenseTile{jid, tm, tn});
        }
      } else {
        cnt.push_back(a);
        B->lds_cnt = std::max(B->lds_cnt, sketch_lds_bytes(kCount, q.tau, nsel));
        void* tbuf = dalloc<char>(B, (size_t)std::max<int64_t>(1, q.nnz) * sparse_entry_bytes_f64());
        SparseJob j{q.zr_ptr, q.zr_col, q.zr_val, q.zt_ptr, q.zt_col, q.zt_val, q.nnz, m, q.tau, q.ldas,
                    0.0, hmap, members, offs, nsel, tbuf, BS, G0, ldg, st.inactive};
        const int jid = (int)sj.size();
        sj.push_back(j);
        for (int bk = 0; bk < q.tau; ++bk) {
          si.push_back(jid);
          si.push_back(bk);
        }
        B->max_sparse_tau = std::max(B->max_sparse_tau, q.tau);
      }
      for (int l = 0; l < q.nlam; ++l) {
        CholJob c{Ginv + (size_t)l * ldg * ldg, U + (size_t)l * ldg * ldg, ldg, q.tau, q.kind, BS, q.ldas,
                  members, offs, G0, pr.lambdas[l], nullptr, st.inactive};
        chol_order.push_back({ldg, c});
      }
      for (int bk = 0; bk < q.tau; ++bk) {
        rho_it.push_back(p);
        rho_it.push_back(bk);
      }
      for (int l = 0; l < q.nlam; ++l)
        for (int ch = 0; ch < (q.tau + 3) / 4; ++ch) {
          del_it.push_back(p);
          del_it.push_back(l);
          del_it.push_back(ch);
        }
      for (int tl = 0; tl < q.ntiles; ++tl) {
        upd_it.push_back(p);
        upd_it.push_back(tl);
      }
      sig += (q.sparse ? "c" : (B->mixed ? "b" : "d")) + std::to_string(m) + "x" + std::to_string(q.K) + "t" +
             std::to_string(q.tau) + "l" + std::to_string(q.nlam) + ";";
    }
    // product tiles in decreasing contraction length (a tile costs ~K): with the
    // workgroups striding over the table this keeps the per-workgroup loads even
    std::stable_sort(dt.begin(), dt.end(), [&](const DenseTile& a, const DenseTile& b) {
      return dj[a.job].K > dj[b.job].K;
    });
    std::stable_sort(bft.begin(), bft.end(), [&](const DenseTile& a, const DenseTile& b) {
      return bj[a.job].kpad > bj[b.job].kpad;
    });
    // factorisations in decreasing size, so the largest start first
    std::stable_sort(chol_order.begin(), chol_order.end(),
                     [](const auto& a, const auto& b) { return a.first > b.first; });
    B->n_cjobs = (int)chol_order.size();
    B->cstatus = dalloc<int32_t>(B, std::max(1, B->n_cjobs));
    for (int i = 0; i < B->n_cjobs; ++i) {
      chol_order[i].second.status = B->cstatus + i;
      cj.push_back(chol_order[i].second);
    }
    // momentum schedule table, indexed by the device iteration counter
    std::vector<double> bt(max_cap + 1), gm(max_cap + 1);
    const int64_t sw = momentum_switch(o->eta, o->beta_max);
    for (int64_t kk = 0; kk <= max_cap; ++kk) momentum_schedule(*o, sw, kk, &gm[kk], &bt[kk]);

    B->S = upload(B, hs);
    B->betas = upload(B, bt);
    B->gammas = upload(B, gm);
    B->n_sub = (int)sub.size();
    B->n_cnt = (int)cnt.size();
    B->sk_sub = upload(B, sub);
    B->sk_cnt = upload(B, cnt);
    B->djobs = upload(B, dj);
    B->dtiles = upload(B, dt);
    B->n_dtiles = (int)dt.size();
    B->bjobs = upload(B, bj);
    B->btiles = upload(B, bft);
    B->n_btiles = (int)bft.size();
    B->ref_u = upload(B, ru);
    B->n_ref_u = (int)ru.size() / 3;
    B->ref_r = upload(B, rr);
    B->n_ref_r = (int)rr.size() / 3;
    B->sjobs = upload(B, sj);
    B->n_sjobs = (int)sj.size();
    B->sitems = upload(B, si);
    B->n_sitems = (int)si.size() / 2;
    B->cjobs = upload(B, cj);
    B->rho_items = upload(B, rho_it);
    B->n_rho = (int)rho_it.size() / 2;
    B->delta_items = upload(B, del_it);
    B->n_delta = (int)del_it.size() / 3;
    B->upd_items = upload(B, upd_it);
    B->n_upd = (int)upd_it.size() / 2;
    B->signature = sig;
    init_state(B);
    if (o->autotune) {
      autotune(B);
      init_state(B);
    }
    *out = B;
    return RS_OK;
  } catch (const Fail& f) {
    g_batch_create_error = f.msg;
    free_all(B);
    delete B;
    return f.code;
  } catch (const std::exception& e) {
    g_batch_create_error = e.what();
    free_all(B);
    delete B;
    return RS_EDEVICE;
  }
}

rs_status rs_batch_step(rs_batch* B, int64_t iters) {
  if (!B || iters < 0) return RS_EINVAL;
  try {
    int64_t left = iters;
    if (B->graph_iters > 0 && left >= B->graph_iters) {
      ensure_graph(B);
      while (left >= B->graph_iters && !B->done) {
        check_hip(hipGraphLaunch(B->exec, B->stream), "graph launch");
        left -= B->graph_iters;
        sync_state(B);
      }
    }
    while (left > 0 && !B->done) {
      enqueue_iteration(B);
      --left;
    }
    sync_state(B);
    return RS_OK;
  } catch (const Fail& f) {
    B->last_error = f.msg;
    return f.code;
  } catch (const std::exception& e) {
    B->last_error = e.what();
    return RS_EDEVICE;
  }
}

rs_status rs_batch_solve(rs_batch* B, rs_batch_report* rep) {
  if (!B) return RS_EINVAL;
  try {
    const auto t0 = std::chrono::steady_clock::now();
    if (B->graph_iters > 0) {
      ensure_graph(B);
      while (!B->done) {
        check_hip(hipGraphLaunch(B->exec, B->stream), "graph launch");
        sync_state(B);
      }
    } else {
      while (!B->done) {
        for (int i = 0; i < 8; ++i) enqueue_iteration(B);
        sync_state(B);
      }
    }
    const auto t1 = std::chrono::steady_clock::now();
    int solves = 0, converged = 0;
    for (const BProb& q : B->P) {
      std::vector<int64_t> sk(q.J);
      check_hip(hipMemcpy(sk.data(), q.stop_k, sizeof(int64_t) * q.J, hipMemcpyDeviceToHost), "stop");
      solves += q.J;
      for (int64_t v : sk) converged += v >= 0 ? 1 : 0;
    }
    if (rep) {
      rep->iters = B->k;
      rep->solves = solves;
      rep->converged = converged;
      rep->seconds = std::chrono::duration<double>(t1 - t0).count();
    }
    return converged == solves ? RS_OK : RS_NOT_CONVERGED;
  } catch (const Fail& f) {
    B->last_error = f.msg;
    return f.code;
  } catch (const std::exception& e) {
    B->last_error = e.what();
    return RS_EDEVICE;
  }
}

rs_status rs_batch_reset(rs_batch* B, uint64_t seed) {
  if (!B) return RS_EINVAL;
  try {
    if (seed != B->opt.seed) {
      // the sketch keys live in the captured argument tables: rewrite them
      B->opt.seed = seed;
      std::vector<SketchArgs> t(std::max(B->n_sub, B->n_cnt));
      for (auto [tab, n] : {std::make_pair(B->sk_sub, B->n_sub), std::make_pair(B->sk_cnt, B->n_cnt)}) {
        if (!n) continue;
        check_hip(hipMemcpy(t.data(), tab, sizeof(SketchArgs) * n, hipMemcpyDeviceToHost), "tables");
        for (int i = 0; i < n; ++i) t[i].seed = seed;
        check_hip(hipMemcpy(tab, t.data(), sizeof(SketchArgs) * n, hipMemcpyHostToDevice), "tables");
      }
    }
    B->k = 0;
    B->done = false;
    init_state(B);
    return RS_OK;
  } catch (const Fail& f) {
    B->last_error = f.msg;
    return f.code;
  } catch (const std::exception& e) {
    B->last_error = e.what();
    return RS_EDEVICE;
  }
}

int64_t rs_batch_iteration(const rs_batch* B) { return B ? B->k : -1; }

rs_status rs_batch_problem_info(const rs_batch* B, int32_t p, rs_batch_problem_info_t* info) {
  if (!B || !info || p < 0 || p >= (int)B->P.size()) return RS_EINVAL;
  const BProb& q = B->P[p];
  info->m = q.m;
  info->K = q.K;
  info->form = q.form;
  info->sketch = q.kind == kCount ? RS_SKETCH_COUNT : RS_SKETCH_SUBSAMPLE;
  info->tau = q.tau;
  info->slots = q.J;
  info->max_iter = q.cap;
  int64_t it = 0;
  if (hipMemcpy(&it, q.iters, sizeof(int64_t), hipMemcpyDeviceToHost) != hipSuccess) return RS_EDEVICE;
  info->iters = it;
  return RS_OK;
}

rs_status rs_batch_slot_report(const rs_batch* B, int32_t p, int64_t* stop_iter, double* rel_res) {
  if (!B || p < 0 || p >= (int)B->P.size()) return RS_EINVAL;
  const BProb& q = B->P[p];
  if (stop_iter && hipMemcpy(stop_iter, q.stop_k, sizeof(int64_t) * q.J, hipMemcpyDeviceToHost) != hipSuccess)
    return RS_EDEVICE;
  if (rel_res && hipMemcpy(rel_res, q.rel, sizeof(double) * q.J, hipMemcpyDeviceToHost) != hipSuccess)
    return RS_EDEVICE;
  return RS_OK;
}

rs_status rs_batch_get_state(const rs_batch* B, int32_t p, int32_t slot, double* x, double* x_prev,
                             double* r, double* r_prev) {
  if (!B || p < 0 || p >= (int)B->P.size()) return RS_EINVAL;
  const BProb& q = B->P[p];
  if (slot < 0 || slot >= q.J) return RS_EINVAL;
  const BState* dev = B->S + p;
  BState st{};
  if (hipMemcpy(&st, dev, sizeof(BState), hipMemcpyDeviceToHost) != hipSuccess) return RS_EDEVICE;
  int64_t kp = 0;
  try {
    kp = problem_k(B, p);
  } catch (const Fail& f) {
    return f.code;
  } catch (const std::exception&) {
    return RS_EDEVICE;
  }
  const int cur = (int)(kp & 1), prv = 1 - cur;
  const double* src[4] = {st.x[cur], st.x[prv], st.r[cur], st.r[prv]};
  double* dst[4] = {x, x_prev, r, r_prev};
  std::vector<double> buf((size_t)q.m * q.J);
  for (int i = 0; i < 4; ++i) {
    if (!dst[i]) continue;
    if (hipMemcpy(buf.data(), src[i], sizeof(double) * buf.size(), hipMemcpyDeviceToHost) != hipSuccess)
      return RS_EDEVICE;
    for (int64_t e = 0; e < q.m; ++e) dst[i][e] = buf[(size_t)e * q.J + slot];
  }
  return RS_OK;
}

rs_status rs_batch_get_weights(rs_batch* B, int32_t p, double* w_out) {
  if (!B || !w_out || p < 0 || p >= (int)B->P.size()) return RS_EINVAL;
  try {
    const BProb& q = B->P[p];
    hipStream_t s = B->stream;
    const double* x = q.x[problem_k(B, p) & 1];
    double* col = nullptr;
    double* w = nullptr;
    check_hip(hipMalloc(&col, sizeof(double) * q.m), "alloc");
    hipError_t e = hipMalloc(&w, sizeof(double) * q.d);
    for (int j = 0; j < q.J && e == hipSuccess; ++j) {
      e = launch_bcol(x, q.m, q.J, j, col, 1, 0, s);
      if (e != hipSuccess) break;
      if (q.form == RS_FORM_PRIMAL) {
        e = hipMemcpyAsync(w, col, sizeof(double) * q.d, hipMemcpyDeviceToDevice, s);
      } else if (q.sparse) {
        e = launch_spmv_csr(q.zt_ptr, q.zt_col, q.zt_val, 0, q.d, col, w, s);
      } else {
        e = launch_gemv_cols(q.Z, q.K, q.m, q.K, col, w, s);
      }
      if (e == hipSuccess)
        e = hipMemcpyAsync(w_out + (size_t)j * q.d, w, sizeof(double) * q.d, hipMemcpyDeviceToHost, s);
      if (e == hipSuccess) e = hipStreamSynchronize(s);
    }
    (void)hipFree(col);
    if (w) (void)hipFree(w);
    check_hip(e, "weights");
    return RS_OK;
  } catch (const Fail& f) {
    B->last_error = f.msg;
    return f.code;
  } catch (const std::exception& e) {
    B->last_error = e.what();
    return RS_EDEVICE;
  }
}

rs_status rs_batch_get_tuning(const rs_batch* B, rs_tuning* out) {
  if (!B || !out) return RS_EINVAL;
  out->tuned = B->tune.tuned;
  out->dense_tk = B->tune.dense_tk;
  out->dense_wg_per_cu = B->tune.dense_mult;
  out->sparse_wg_per_cu = B->tune.sparse_mult;
  out->chol_wg_per_cu = B->tune.chol_mult;
  out->dense_ms = B->tune.dense_ms;
  out->sparse_ms = B->tune.sparse_ms;
  out->chol_ms = B->tune.chol_ms;
  out->graph_iters = B->graph_iters;
  out->compute_units = B->cus;
  return RS_OK;
}

const char* rs_batch_last_error(const rs_batch* B) {
  return B ? B->last_error.c_str() : g_batch_create_error.c_str();
}

rs_status rs_batch_destroy(rs_batch* B) {
  if (!B) return RS_EINVAL;
  if (B->stream) (void)hipStreamSynchronize(B->stream);
  free_all(B);
  delete B;
  return RS_OK;
}

}  // extern "C"
