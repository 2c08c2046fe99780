// Host side of the learned proposal: the trainer (trace store, mini-batch Adam on the
// device) and entry points that run single kernels of the proposal on host arrays, so
// that each piece can be checked on its own (include/rs.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>
#include <random>
#include <string>
#include <vector>

#include "rs_internal.h"

using namespace rs;

struct rs_trainer {
  int32_t tau = 0;
  float* P = nullptr;   // parameters
  float* m1 = nullptr;  // Adam moments
  float* m2 = nullptr;
  float* grad = nullptr;
  int64_t t = 0;        // Adam steps taken
  // trace store
  float* F = nullptr;
  float* C = nullptr;
  int64_t n = 0, cap = 0;
  // step scratch
  int32_t batch_cap = 0;
  int32_t* rec = nullptr;
  float* s = nullptr;
  float* ds = nullptr;
  double* loss = nullptr;
  float* partial = nullptr;
  std::string last_error;
};

namespace {

struct Fail {
  rs_status code;
  std::string msg;
};

void ck(hipError_t e, const char* what) {
  if (e != hipSuccess) throw Fail{RS_EDEVICE, std::string(what) + ": " + hipGetErrorString(e)};
}

template <class T>
T* dmalloc(size_t count) {
  void* p = nullptr;
  if (hipMalloc(&p, sizeof(T) * std::max<size_t>(1, count)) != hipSuccess) {
    (void)hipGetLastError();
    throw Fail{RS_ENOMEM, "hipMalloc failed"};
  }
  return static_cast<T*>(p);
}

// Device buffers freed at scope exit (kernel-level entry points).
struct Scratch {
  std::vector<void*> p;
  template <class T>
  T* get(size_t count) {
    T* d = dmalloc<T>(count);
    p.push_back(d);
    return d;
  }
  template <class T>
  T* up(const T* src, size_t count) {
    T* d = get<T>(count);
    ck(hipMemcpy(d, src, sizeof(T) * count, hipMemcpyHostToDevice), "upload");
    return d;
  }
  ~Scratch() {
    for (void* q : p) (void)hipFree(q);
  }
};

void grow_store(rs_trainer* T, int64_t need) {
  if (need <= T->cap) return;
  int64_t cap = std::max<int64_t>(need, std::max<int64_t>(1024, 2 * T->cap));
  const size_t rf = (size_t)T->tau * kMlpFeatures, rc = (size_t)T->tau;
  float* F = dmalloc<float>(cap * rf);
  float* C = dmalloc<float>(cap * rc);
  if (T->n) {
    ck(hipMemcpy(F, T->F, sizeof(float) * rf * T->n, hipMemcpyDeviceToDevice), "copy");
    ck(hipMemcpy(C, T->C, sizeof(float) * rc * T->n, hipMemcpyDeviceToDevice), "copy");
  }
  (void)hipFree(T->F);
  (void)hipFree(T->C);
  T->F = F;
  T->C = C;
  T->cap = cap;
}

void ensure_batch(rs_trainer* T, int32_t nrec) {
  if (nrec <= T->batch_cap) return;
  for (void* q : {(void*)T->rec, (void*)T->s, (void*)T->ds, (void*)T->loss, (void*)T->partial})
    (void)hipFree(q);
  const int64_t rows = (int64_t)nrec * T->tau;
  T->rec = dmalloc<int32_t>(nrec);
  T->s = dmalloc<float>(rows);
  T->ds = dmalloc<float>(rows);
  T->loss = dmalloc<double>(nrec);
  T->partial = dmalloc<float>((size_t)mlp_bwd_blocks(rows) * kMlpParams);
  T->batch_cap = nrec;
}

}  // namespace

extern "C" {

rs_status rs_trainer_create(int32_t tau, uint64_t init_seed, rs_trainer** out) {
  if (!out || tau < 1) return RS_EINVAL;
  *out = nullptr;
  rs_trainer* T = new rs_trainer();
  try {
    T->tau = tau;
    T->P = dmalloc<float>(kMlpParams);
    T->m1 = dmalloc<float>(kMlpParams);
    T->m2 = dmalloc<float>(kMlpParams);
    T->grad = dmalloc<float>(kMlpParams);
    ck(launch_mlp_init(T->P, init_seed, nullptr), "init");
    ck(hipMemset(T->m1, 0, sizeof(float) * kMlpParams), "memset");
    ck(hipMemset(T->m2, 0, sizeof(float) * kMlpParams), "memset");
    ck(hipDeviceSynchronize(), "sync");
    *out = T;
    return RS_OK;
  } catch (const Fail& f) {
    rs_trainer_destroy(T);
    return f.code;
  } catch (const std::exception&) {
    rs_trainer_destroy(T);
    return RS_EDEVICE;
  }
}

rs_status rs_trainer_add_traces(rs_trainer* T, const rs_handle* h) {
  if (!T || !h) return RS_EINVAL;
  try {
    int64_t n = 0;
    rs_status st = rs_trace_count(h, &n);
    if (st != RS_OK) return st;
    if (n == 0) return RS_OK;
    if (rs_sketch_size(h) != T->tau) throw Fail{RS_EINVAL, "trace of a different sketch size"};
    std::vector<float> F((size_t)n * T->tau * kMlpFeatures), C((size_t)n * T->tau);
    st = rs_get_trace(h, F.data(), C.data(), 0, n);
    if (st != RS_OK) return st;
    return rs_trainer_add_records(T, F.data(), C.data(), n);
  } catch (const Fail& f) {
    T->last_error = f.msg;
    return f.code;
  } catch (const std::exception& e) {
    T->last_error = e.what();
    return RS_EDEVICE;
  }
}

rs_status rs_trainer_add_records(rs_trainer* T, const float* F, const float* credits, int64_t count) {
  if (!T || !F || !credits || count < 0) return RS_EINVAL;
  try {
    grow_store(T, T->n + count);
    const size_t rf = (size_t)T->tau * kMlpFeatures, rc = (size_t)T->tau;
    ck(hipMemcpy(T->F + T->n * rf, F, sizeof(float) * rf * count, hipMemcpyHostToDevice), "upload");
    ck(hipMemcpy(T->C + T->n * rc, credits, sizeof(float) * rc * count, hipMemcpyHostToDevice), "upload");
    T->n += count;
    return RS_OK;
  } catch (const Fail& f) {
    T->last_error = f.msg;
    return f.code;
  } catch (const std::exception& e) {
    T->last_error = e.what();
    return RS_EDEVICE;
  }
}

rs_status rs_trainer_records(const rs_trainer* T, int64_t* count) {
  if (!T || !count) return RS_EINVAL;
  *count = T->n;
  return RS_OK;
}

rs_status rs_trainer_fit(rs_trainer* T, int32_t epochs, int32_t batch, double lr, uint64_t shuffle_seed,
                         double* epoch_loss) {
  if (!T || epochs < 0 || batch < 1 || !(lr > 0.0)) return RS_EINVAL;
  if (T->n == 0) {
    T->last_error = "no trace records";
    return RS_EINVAL;
  }
  try {
    const int32_t nb = (int32_t)std::min<int64_t>(batch, T->n);
    ensure_batch(T, nb);
    std::vector<int32_t> order(T->n);
    std::vector<double> losses(nb);
    for (int e = 0; e < epochs; ++e) {
      std::iota(order.begin(), order.end(), 0);
      std::mt19937_64 gen(shuffle_seed + (uint64_t)e);
      std::shuffle(order.begin(), order.end(), gen);
      double tot = 0.0;
      int64_t seen = 0;
      for (int64_t off = 0; off + nb <= T->n; off += nb) {
        ck(hipMemcpy(T->rec, order.data() + off, sizeof(int32_t) * nb, hipMemcpyHostToDevice), "batch");
        ck(launch_mlp_step(T->P, T->F, T->C, T->rec, T->tau, nb, T->s, T->ds, T->loss, T->partial, T->grad,
                           nullptr),
           "gradient");
        T->t += 1;
        ck(launch_adam(T->P, T->m1, T->m2, T->grad, T->t, lr, 0.9, 0.999, 1e-8, nullptr), "adam");
        ck(hipMemcpy(losses.data(), T->loss, sizeof(double) * nb, hipMemcpyDeviceToHost), "loss");
        for (double l : losses) tot += l;
        seen += nb;
      }
      if (epoch_loss) epoch_loss[e] = seen ? tot / (double)seen : 0.0;
    }
    return RS_OK;
  } catch (const Fail& f) {
    T->last_error = f.msg;
    return f.code;
  } catch (const std::exception& e) {
    T->last_error = e.what();
    return RS_EDEVICE;
  }
}

rs_status rs_trainer_eval(rs_trainer* T, double* loss_out, double* floor_out) {
  if (!T || !loss_out) return RS_EINVAL;
  if (T->n == 0) {
    T->last_error = "no trace records";
    return RS_EINVAL;
  }
  try {
    // the mean loss over every record in index order, in batches of at most 256 (the gradient
    // the step kernels also form is scratch here)
    const int32_t nb = (int32_t)std::min<int64_t>(256, T->n);
    ensure_batch(T, nb);
    std::vector<int32_t> idx(nb);
    std::vector<double> losses(nb);
    double tot = 0.0;
    for (int64_t off = 0; off < T->n; off += nb) {
      const int32_t cnt = (int32_t)std::min<int64_t>(nb, T->n - off);
      for (int32_t i = 0; i < cnt; ++i) idx[i] = (int32_t)(off + i);
      ck(hipMemcpy(T->rec, idx.data(), sizeof(int32_t) * cnt, hipMemcpyHostToDevice), "records");
      ck(launch_mlp_step(T->P, T->F, T->C, T->rec, T->tau, cnt, T->s, T->ds, T->loss, T->partial, T->grad,
                         nullptr),
         "loss");
      ck(hipMemcpy(losses.data(), T->loss, sizeof(double) * cnt, hipMemcpyDeviceToHost), "loss");
      for (int32_t i = 0; i < cnt; ++i) tot += losses[i];
    }
    *loss_out = tot / (double)T->n;
    if (floor_out) {
      // the cross-entropy against t is at least the entropy of t, reached when softmax(s) = t
      std::vector<float> c((size_t)T->n * T->tau);
      ck(hipMemcpy(c.data(), T->C, sizeof(float) * c.size(), hipMemcpyDeviceToHost), "credits");
      double fl = 0.0;
      for (int64_t r = 0; r < T->n; ++r) {
        const float* cr = c.data() + (size_t)r * T->tau;
        double sum = 0.0;
        for (int32_t b = 0; b < T->tau; ++b) sum += std::max(0.0, (double)cr[b]);
        if (!(sum > 0.0)) continue;
        for (int32_t b = 0; b < T->tau; ++b) {
          const double t = std::max(0.0, (double)cr[b]) / sum;
          if (t > 0.0) fl -= t * std::log(t);
        }
      }
      *floor_out = fl / (double)T->n;
    }
    return RS_OK;
  } catch (const Fail& f) {
    T->last_error = f.msg;
    return f.code;
  } catch (const std::exception& e) {
    T->last_error = e.what();
    return RS_EDEVICE;
  }
}

rs_status rs_trainer_get_params(const rs_trainer* T, float* out) {
  if (!T || !out) return RS_EINVAL;
  return hipMemcpy(out, T->P, sizeof(float) * kMlpParams, hipMemcpyDeviceToHost) == hipSuccess ? RS_OK
                                                                                               : RS_EDEVICE;
}

rs_status rs_trainer_set_params(rs_trainer* T, const float* in) {
  if (!T || !in) return RS_EINVAL;
  return hipMemcpy(T->P, in, sizeof(float) * kMlpParams, hipMemcpyHostToDevice) == hipSuccess ? RS_OK
                                                                                              : RS_EDEVICE;
}

const char* rs_trainer_last_error(const rs_trainer* T) { return T ? T->last_error.c_str() : ""; }

rs_status rs_trainer_destroy(rs_trainer* T) {
  if (!T) return RS_EINVAL;
  for (void* q : {(void*)T->P, (void*)T->m1, (void*)T->m2, (void*)T->grad, (void*)T->F, (void*)T->C,
                  (void*)T->rec, (void*)T->s, (void*)T->ds, (void*)T->loss, (void*)T->partial})
    if (q) (void)hipFree(q);
  delete T;
  return RS_OK;
}

// ---------------------------------------------------------------- single kernels, host arrays
rs_status rs_mlp_init(uint64_t seed, float* params_out) {
  if (!params_out) return RS_EINVAL;
  try {
    Scratch S;
    float* P = S.get<float>(kMlpParams);
    ck(launch_mlp_init(P, seed, nullptr), "init");
    ck(hipMemcpy(params_out, P, sizeof(float) * kMlpParams, hipMemcpyDeviceToHost), "download");
    return RS_OK;
  } catch (const Fail& f) {
    return f.code;
  } catch (const std::exception&) {
    return RS_EDEVICE;
  }
}

rs_status rs_mlp_forward(const float* params, const float* F, int64_t rows, float* s_out) {
  if (!params || !F || !s_out || rows < 1) return RS_EINVAL;
  try {
    Scratch S;
    const float* P = S.up(params, kMlpParams);
    const float* Fd = S.up(F, (size_t)rows * kMlpFeatures);
    float* s = S.get<float>(rows);
    ck(launch_mlp_fwd(P, Fd, nullptr, 0, rows, s, nullptr, nullptr), "forward");
    ck(hipMemcpy(s_out, s, sizeof(float) * rows, hipMemcpyDeviceToHost), "download");
    return RS_OK;
  } catch (const Fail& f) {
    return f.code;
  } catch (const std::exception&) {
    return RS_EDEVICE;
  }
}

rs_status rs_mlp_gradient(const float* params, const float* F, const float* credits, int32_t nrec,
                          int32_t tau, float* grad_out, double* loss_out) {
  if (!params || !F || !credits || !grad_out || nrec < 1 || tau < 1) return RS_EINVAL;
  try {
    Scratch S;
    const int64_t rows = (int64_t)nrec * tau;
    const float* P = S.up(params, kMlpParams);
    const float* Fd = S.up(F, (size_t)rows * kMlpFeatures);
    const float* Cd = S.up(credits, (size_t)rows);
    std::vector<int32_t> idx(nrec);
    std::iota(idx.begin(), idx.end(), 0);
    const int32_t* rec = S.up(idx.data(), nrec);
    float* s = S.get<float>(rows);
    float* ds = S.get<float>(rows);
    double* loss = S.get<double>(nrec);
    float* partial = S.get<float>((size_t)mlp_bwd_blocks(rows) * kMlpParams);
    float* grad = S.get<float>(kMlpParams);
    ck(launch_mlp_step(P, Fd, Cd, rec, tau, nrec, s, ds, loss, partial, grad, nullptr), "gradient");
    ck(hipMemcpy(grad_out, grad, sizeof(float) * kMlpParams, hipMemcpyDeviceToHost), "download");
    if (loss_out) {
      std::vector<double> l(nrec);
      ck(hipMemcpy(l.data(), loss, sizeof(double) * nrec, hipMemcpyDeviceToHost), "download");
      *loss_out = std::accumulate(l.begin(), l.end(), 0.0) / (double)nrec;
    }
    return RS_OK;
  } catch (const Fail& f) {
    return f.code;
  } catch (const std::exception&) {
    return RS_EDEVICE;
  }
}

rs_status rs_adam_update(float* params, float* m1, float* m2, const float* grad, int64_t t, double lr,
                         double b1, double b2, double eps) {
  if (!params || !m1 || !m2 || !grad || t < 1) return RS_EINVAL;
  try {
    Scratch S;
    float* P = S.up(params, kMlpParams);
    float* a = S.up(m1, kMlpParams);
    float* v = S.up(m2, kMlpParams);
    const float* g = S.up(grad, kMlpParams);
    ck(launch_adam(P, a, v, g, t, lr, b1, b2, eps, nullptr), "adam");
    ck(hipMemcpy(params, P, sizeof(float) * kMlpParams, hipMemcpyDeviceToHost), "download");
    ck(hipMemcpy(m1, a, sizeof(float) * kMlpParams, hipMemcpyDeviceToHost), "download");
    ck(hipMemcpy(m2, v, sizeof(float) * kMlpParams, hipMemcpyDeviceToHost), "download");
    return RS_OK;
  } catch (const Fail& f) {
    return f.code;
  } catch (const std::exception&) {
    return RS_EDEVICE;
  }
}

rs_status rs_proposal(const float* s, int64_t m, double eps, float* q_out, int32_t* ok_out) {
  if (!s || !q_out || m < 1 || !(eps > 0.0 && eps <= 1.0)) return RS_EINVAL;
  try {
    Scratch S;
    const float* sd = S.up(s, m);
    float* q = S.get<float>(m);
    int32_t* ok = S.get<int32_t>(1);
    ck(launch_proposal(sd, m, (float)eps, q, ok, nullptr, nullptr), "proposal");
    ck(hipMemcpy(q_out, q, sizeof(float) * m, hipMemcpyDeviceToHost), "download");
    if (ok_out) ck(hipMemcpy(ok_out, ok, sizeof(int32_t), hipMemcpyDeviceToHost), "download");
    return RS_OK;
  } catch (const Fail& f) {
    return f.code;
  } catch (const std::exception&) {
    return RS_EDEVICE;
  }
}

rs_status rs_features(const double* a, const double* r, const double* rp, const int32_t* last, int64_t m,
                      int64_t k, float* F_out) {
  if (!a || !r || !rp || !last || !F_out || m < 1 || k < 0) return RS_EINVAL;
  for (int64_t j = 0; j < m; ++j)
    if (!(a[j] > 0.0) || last[j] >= k || last[j] < -1) return RS_EINVAL;
  try {
    Scratch S;
    const double* ad = S.up(a, m);
    const double* rd = S.up(r, m);
    const double* rpd = S.up(rp, m);
    const int32_t* ld = S.up(last, m);
    double* stats = S.get<double>(3);
    double* lrn = S.get<double>(1);
    float* F = S.get<float>((size_t)m * kMlpFeatures);
    ck(launch_lstats(ad, m, stats, nullptr), "statistics of A_jj");
    ck(launch_features(ad, stats, rd, rpd, ld, m, k, lrn, F, nullptr, nullptr), "features");
    ck(hipMemcpy(F_out, F, sizeof(float) * m * kMlpFeatures, hipMemcpyDeviceToHost), "download");
    return RS_OK;
  } catch (const Fail& f) {
    return f.code;
  } catch (const std::exception&) {
    return RS_EDEVICE;
  }
}

rs_status rs_draw_weighted(const float* q, int64_t m, int32_t tau, uint64_t seed, uint64_t problem_id,
                           int64_t k, int32_t* C_out) {
  if (!q || !C_out || m < 1 || tau < 1 || tau > m || k < 0 || m > INT32_MAX) return RS_EINVAL;
  for (int64_t j = 0; j < m; ++j)
    if (!(q[j] > 0.0f) || !std::isfinite(q[j])) return RS_EINVAL;
  try {
    Scratch S;
    const float* qd = S.up(q, m);
    int32_t* one = S.get<int32_t>(1);
    const int32_t v1 = 1;
    ck(hipMemcpy(one, &v1, sizeof(int32_t), hipMemcpyHostToDevice), "upload");
    int32_t* zero = S.get<int32_t>(2);  // [done = 0, err]
    ck(hipMemset(zero, 0, sizeof(int32_t) * 2), "memset");
    SketchArgs a{};
    a.kind = kWeighted;
    a.m = m;
    a.tau = tau;
    a.nsel = tau;
    a.seed = seed;
    a.pid = problem_id;
    a.k0 = k;
    a.nslots = 1;
    a.hmap = S.get<int32_t>(m);
    a.members = S.get<int32_t>(tau);
    a.offs = S.get<int32_t>(tau + 1);
    a.keys = S.get<uint64_t>(m);
    a.err = zero + 1;
    a.done = zero;
    a.q = qd;
    a.q_ok = one;
    ck(launch_sketch(a, nullptr), "sketch");
    ck(hipMemcpy(C_out, a.members, sizeof(int32_t) * tau, hipMemcpyDeviceToHost), "download");
    int32_t err = 0;
    ck(hipMemcpy(&err, zero + 1, sizeof(int32_t), hipMemcpyDeviceToHost), "download");
    return err ? RS_EDEVICE : RS_OK;
  } catch (const Fail& f) {
    return f.code;
  } catch (const std::exception&) {
    return RS_EDEVICE;
  }
}

}  // extern "C"
