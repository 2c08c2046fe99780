"""Python binding of librs.so (include/rs.h): argument marshalling only.

Every step of the solver runs inside the HIP library. This module converts
numpy arrays (host memory) or torch CUDA tensors (device memory) into the
plain pointers and sizes the C ABI takes, and raises ``RsError`` on a negative
status. It fails loudly when the library is missing: there is no fallback.
"""
import ctypes
import os

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "librs.so")

RS_OK, RS_NOT_CONVERGED = 0, 1
RS_EINVAL, RS_ENOMEM, RS_EDEVICE, RS_ESINGULAR, RS_EUNSUPPORTED = -1, -2, -3, -4, -5
RS_DENSE_ROWMAJOR, RS_DENSE_COLMAJOR, RS_CSR = 0, 1, 2
RS_F64, RS_F32 = 0, 1
RS_HOST, RS_DEVICE = 0, 1
RS_FORM_AUTO, RS_FORM_PRIMAL, RS_FORM_DUAL = 0, 1, 2
RS_SKETCH_SUBSAMPLE, RS_SKETCH_COUNT, RS_SKETCH_SUBCOUNT, RS_SKETCH_GAUSSIAN, RS_SKETCH_SRHT = 0, 1, 2, 3, 4
RS_MOMENTUM_NONE, RS_MOMENTUM_CONSTANT, RS_MOMENTUM_HEURISTIC, RS_MOMENTUM_THEORY = 0, 1, 2, 3
RS_PREC_FP64, RS_PREC_MIXED_BF16 = 0, 1

FORMS = {"auto": RS_FORM_AUTO, "primal": RS_FORM_PRIMAL, "dual": RS_FORM_DUAL}
SKETCHES = {"subsample": RS_SKETCH_SUBSAMPLE, "count": RS_SKETCH_COUNT, "subcount": RS_SKETCH_SUBCOUNT,
            "gaussian": RS_SKETCH_GAUSSIAN, "srht": RS_SKETCH_SRHT}
MOMENTA = {"none": RS_MOMENTUM_NONE, "constant": RS_MOMENTUM_CONSTANT, "heuristic": RS_MOMENTUM_HEURISTIC,
           "theory": RS_MOMENTUM_THEORY}
PRECISIONS = {"fp64": RS_PREC_FP64, "mixed": RS_PREC_MIXED_BF16}


class rs_matrix(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("d", ctypes.c_int64), ("layout", ctypes.c_int32),
                ("dtype", ctypes.c_int32), ("vals", ctypes.c_void_p), ("row_ptr", ctypes.c_void_p),
                ("col_idx", ctypes.c_void_p), ("nnz", ctypes.c_int64), ("mem", ctypes.c_int32)]


class rs_options(ctypes.Structure):
    _fields_ = [("form", ctypes.c_int32), ("sketch", ctypes.c_int32), ("tau", ctypes.c_int32),
                ("subcount_k", ctypes.c_int32), ("momentum", ctypes.c_int32),
                ("precision", ctypes.c_int32), ("gamma", ctypes.c_double), ("beta", ctypes.c_double),
                ("eta", ctypes.c_double), ("beta_max", ctypes.c_double), ("tol", ctypes.c_double),
                ("max_iter", ctypes.c_int64), ("seed", ctypes.c_uint64), ("problem_id", ctypes.c_uint64),
                ("refresh_every", ctypes.c_int32), ("lookahead", ctypes.c_int32),
                ("profile", ctypes.c_int32), ("stream", ctypes.c_void_p),
                ("graph_iters", ctypes.c_int32), ("autotune", ctypes.c_int32),
                ("sampler", ctypes.c_int32), ("trace_every", ctypes.c_int32),
                ("trace_capacity", ctypes.c_int32), ("sparse_route", ctypes.c_int32),
                ("pipeline", ctypes.c_int32), ("accelerated", ctypes.c_int32),
                ("accel_mu", ctypes.c_double), ("accel_nu", ctypes.c_double),
                ("dense_route", ctypes.c_int32), ("refresh_early", ctypes.c_int32)]


RS_SAMPLER_UNIFORM, RS_SAMPLER_LEARNED, RS_SAMPLER_DIAG = 0, 1, 2
SAMPLERS = {"uniform": RS_SAMPLER_UNIFORM, "learned": RS_SAMPLER_LEARNED, "diag": RS_SAMPLER_DIAG}
RS_MLP_FEATURES, RS_MLP_HIDDEN, RS_MLP_PARAMS = 6, 128, 17537
RS_ROUTE_AUTO, RS_ROUTE_SCATTER, RS_ROUTE_AROWS = 0, 1, 2
ROUTES = {"auto": RS_ROUTE_AUTO, "scatter": RS_ROUTE_SCATTER, "arows": RS_ROUTE_AROWS}


class rs_problem(ctypes.Structure):
    _fields_ = [("X", rs_matrix), ("y", ctypes.c_void_p), ("nrhs", ctypes.c_int32),
                ("lambdas", ctypes.c_void_p), ("nlambda", ctypes.c_int32), ("tau", ctypes.c_int32),
                ("sketch", ctypes.c_int32), ("form", ctypes.c_int32), ("max_iter", ctypes.c_int64)]


class rs_batch_report(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int64), ("solves", ctypes.c_int32), ("converged", ctypes.c_int32),
                ("seconds", ctypes.c_double)]


class rs_batch_problem_info_t(ctypes.Structure):
    _fields_ = [("m", ctypes.c_int64), ("K", ctypes.c_int64), ("form", ctypes.c_int32),
                ("sketch", ctypes.c_int32), ("tau", ctypes.c_int32), ("slots", ctypes.c_int32),
                ("max_iter", ctypes.c_int64), ("iters", ctypes.c_int64)]


class rs_tuning(ctypes.Structure):
    _fields_ = [("tuned", ctypes.c_int32), ("dense_tk", ctypes.c_int32),
                ("dense_wg_per_cu", ctypes.c_int32), ("sparse_wg_per_cu", ctypes.c_int32),
                ("chol_wg_per_cu", ctypes.c_int32), ("graph_iters", ctypes.c_int32),
                ("compute_units", ctypes.c_int32), ("dense_ms", ctypes.c_double),
                ("sparse_ms", ctypes.c_double), ("chol_ms", ctypes.c_double)]


RS_PROF_SKETCH, RS_PROF_AS, RS_PROF_CHOL, RS_PROF_DELTA, RS_PROF_UPDATE, RS_PROF_REFRESH, RS_PROF_ITERS, \
    RS_PROF_G = range(8)
RS_PROF_COUNT = 8
PROF_NAMES = ["sketch", "as", "chol", "delta", "update", "refresh", "iters", "g"]


class rs_profile(ctypes.Structure):
    _fields_ = [("ms", ctypes.c_double * RS_PROF_COUNT), ("launches", ctypes.c_int64 * RS_PROF_COUNT),
                ("slots", ctypes.c_int64 * RS_PROF_COUNT)]


class rs_report(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int64), ("rel_res", ctypes.c_double), ("seconds", ctypes.c_double),
                ("rel_res_true", ctypes.c_double)]


class RsError(RuntimeError):
    def __init__(self, status, where, detail=""):
        self.status = status
        super().__init__(f"{where}: status {status} ({status_string(status)}) {detail}".rstrip())


_lib = None
_P = ctypes.c_void_p
_D = ctypes.POINTER(ctypes.c_double)

# name -> (restype, argtypes): every entry point declared in include/rs.h
SIGNATURES = {
    "rs_options_default": (ctypes.c_int32, [ctypes.POINTER(rs_options)]),
    "rs_create": (ctypes.c_int32, [ctypes.POINTER(rs_matrix), _P, ctypes.c_double,
                                   ctypes.POINTER(rs_options), ctypes.POINTER(_P)]),
    "rs_create_kernel": (ctypes.c_int32, [ctypes.POINTER(rs_matrix), _P, ctypes.c_double, ctypes.c_double,
                                          ctypes.POINTER(rs_options), ctypes.POINTER(_P)]),
    "rs_step": (ctypes.c_int32, [_P, ctypes.c_int64, _D]),
    "rs_solve": (ctypes.c_int32, [_P, _P, ctypes.POINTER(rs_report)]),
    "rs_reset": (ctypes.c_int32, [_P, ctypes.c_uint64]),
    "rs_get_profile": (ctypes.c_int32, [_P, ctypes.POINTER(rs_profile), ctypes.c_int32]),
    "rs_iteration": (ctypes.c_int64, [_P]),
    "rs_system_size": (ctypes.c_int64, [_P]),
    "rs_get_state": (ctypes.c_int32, [_P, _P, _P, _P, _P]),
    "rs_set_state": (ctypes.c_int32, [_P, ctypes.c_int64, _P, _P, _P, _P]),
    "rs_get_weights": (ctypes.c_int32, [_P, _P]),
    "rs_get_last_sketch": (ctypes.c_int32, [_P, _P, _P, _P, ctypes.POINTER(ctypes.c_int64)]),
    "rs_get_history": (ctypes.c_int32, [_P, _P, ctypes.c_int64]),
    "rs_get_products": (ctypes.c_int32, [_P, _P, _P]),
    "rs_destroy": (ctypes.c_int32, [_P]),
    "rs_status_string": (ctypes.c_char_p, [ctypes.c_int32]),
    "rs_momentum_schedule": (ctypes.c_int32, [ctypes.POINTER(rs_options), ctypes.c_int64,
                                              ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]),
    "rs_last_error": (ctypes.c_char_p, [_P]),
    "rs_sketch_size": (ctypes.c_int32, [_P]),
    "rs_get_route": (ctypes.c_int32, [_P, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int64)]),
    "rs_set_sampler_params": (ctypes.c_int32, [_P, _P]),
    "rs_trace_count": (ctypes.c_int32, [_P, ctypes.POINTER(ctypes.c_int64)]),
    "rs_get_trace": (ctypes.c_int32, [_P, _P, _P, ctypes.c_int64, ctypes.c_int64]),
    "rs_get_proposal": (ctypes.c_int32, [_P, _P, _P]),
    "rs_trainer_create": (ctypes.c_int32, [ctypes.c_int32, ctypes.c_uint64, ctypes.POINTER(_P)]),
    "rs_trainer_add_traces": (ctypes.c_int32, [_P, _P]),
    "rs_trainer_add_records": (ctypes.c_int32, [_P, _P, _P, ctypes.c_int64]),
    "rs_trainer_records": (ctypes.c_int32, [_P, ctypes.POINTER(ctypes.c_int64)]),
    "rs_trainer_fit": (ctypes.c_int32, [_P, ctypes.c_int32, ctypes.c_int32, ctypes.c_double, ctypes.c_uint64,
                                        _P]),
    "rs_trainer_eval": (ctypes.c_int32, [_P, _P, _P]),
    "rs_trainer_get_params": (ctypes.c_int32, [_P, _P]),
    "rs_trainer_set_params": (ctypes.c_int32, [_P, _P]),
    "rs_trainer_last_error": (ctypes.c_char_p, [_P]),
    "rs_trainer_destroy": (ctypes.c_int32, [_P]),
    "rs_mlp_init": (ctypes.c_int32, [ctypes.c_uint64, _P]),
    "rs_mlp_forward": (ctypes.c_int32, [_P, _P, ctypes.c_int64, _P]),
    "rs_mlp_gradient": (ctypes.c_int32, [_P, _P, _P, ctypes.c_int32, ctypes.c_int32, _P, _D]),
    "rs_adam_update": (ctypes.c_int32, [_P, _P, _P, _P, ctypes.c_int64, ctypes.c_double, ctypes.c_double,
                                        ctypes.c_double, ctypes.c_double]),
    "rs_proposal": (ctypes.c_int32, [_P, ctypes.c_int64, ctypes.c_double, _P, _P]),
    "rs_features": (ctypes.c_int32, [_P, _P, _P, _P, ctypes.c_int64, ctypes.c_int64, _P]),
    "rs_draw_weighted": (ctypes.c_int32, [_P, ctypes.c_int64, ctypes.c_int32, ctypes.c_uint64,
                                          ctypes.c_uint64, ctypes.c_int64, _P]),
    "rs_draw_weighted_noalloc": (ctypes.c_int32, [_P, ctypes.c_int64, ctypes.c_int32, ctypes.c_uint64,
                                                  ctypes.c_uint64, ctypes.c_int64, _P, _P, _P]),
    "rs_batch_create": (ctypes.c_int32, [ctypes.c_int32, ctypes.POINTER(rs_problem),
                                         ctypes.POINTER(rs_options), ctypes.POINTER(_P)]),
    "rs_batch_step": (ctypes.c_int32, [_P, ctypes.c_int64]),
    "rs_batch_solve": (ctypes.c_int32, [_P, ctypes.POINTER(rs_batch_report)]),
    "rs_batch_reset": (ctypes.c_int32, [_P, ctypes.c_uint64]),
    "rs_batch_iteration": (ctypes.c_int64, [_P]),
    "rs_batch_problem_info": (ctypes.c_int32, [_P, ctypes.c_int32, ctypes.POINTER(rs_batch_problem_info_t)]),
    "rs_batch_slot_report": (ctypes.c_int32, [_P, ctypes.c_int32, _P, _P]),
    "rs_batch_get_state": (ctypes.c_int32, [_P, ctypes.c_int32, ctypes.c_int32, _P, _P, _P, _P]),
    "rs_batch_get_weights": (ctypes.c_int32, [_P, ctypes.c_int32, _P]),
    "rs_batch_get_tuning": (ctypes.c_int32, [_P, ctypes.POINTER(rs_tuning)]),
    "rs_batch_destroy": (ctypes.c_int32, [_P]),
    "rs_batch_last_error": (ctypes.c_char_p, [_P]),
}


def load(path=LIB_PATH):
    """Load librs.so; raises if it is not built. No CPU fallback exists.

    PyTorch wheels carry their own HIP runtime (same SONAME as the system one).
    torch is imported first when it is installed, so that librs.so binds to that
    runtime by SONAME and device pointers and streams from torch are valid for it:
    one process must hold a single HIP runtime.
    """
    global _lib
    if _lib is None:
        if not os.path.exists(path):
            raise RuntimeError(f"{path} is missing: build it with `python -m paper_2105_05565_amd.build`")
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        lib = ctypes.CDLL(path, mode=os.RTLD_NOW | os.RTLD_GLOBAL)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def status_string(s):
    return load().rs_status_string(int(s)).decode()


def last_error(h=None):
    return load().rs_last_error(h).decode()


def _check(status, where, h=None):
    if status < 0:
        raise RsError(status, where, last_error(h))
    return status


def _ptr(a):
    """Pointer of a numpy array (host) or torch tensor (device); keeps no reference."""
    if a is None:
        return None
    if isinstance(a, np.ndarray):
        return a.ctypes.data
    return a.data_ptr()


def _is_device(a):
    return not isinstance(a, np.ndarray) and getattr(a, "is_cuda", False)


# ---------------------------------------------------------------- thin wrappers (same names)
def rs_options_default():
    o = rs_options()
    _check(load().rs_options_default(ctypes.byref(o)), "rs_options_default")
    return o


def rs_momentum_schedule(opts, k):
    """(gamma_k, beta_k) of iteration k under opts' momentum settings, from the library."""
    g, b = ctypes.c_double(0.0), ctypes.c_double(0.0)
    _check(load().rs_momentum_schedule(ctypes.byref(opts), int(k), ctypes.byref(g), ctypes.byref(b)),
           "rs_momentum_schedule")
    return g.value, b.value


def rs_create(X, y, lam, opts):
    h = _P()
    _check(load().rs_create(ctypes.byref(X), _ptr(y), float(lam), ctypes.byref(opts), ctypes.byref(h)),
           "rs_create")
    return h


def rs_create_kernel(P, y, sigma, lam, opts):
    h = _P()
    _check(load().rs_create_kernel(ctypes.byref(P), _ptr(y), float(sigma), float(lam), ctypes.byref(opts),
                                   ctypes.byref(h)), "rs_create_kernel")
    return h


def rs_step(h, iters):
    rel = ctypes.c_double(0.0)
    _check(load().rs_step(h, int(iters), ctypes.byref(rel)), "rs_step", h)
    return rel.value


def rs_solve(h, w_out=None):
    rep = rs_report()
    st = _check(load().rs_solve(h, _ptr(w_out), ctypes.byref(rep)), "rs_solve", h)
    return st, rep


def rs_reset(h, seed):
    _check(load().rs_reset(h, int(seed)), "rs_reset", h)


def rs_get_profile(h, clear=False):
    p = rs_profile()
    _check(load().rs_get_profile(h, ctypes.byref(p), int(bool(clear))), "rs_get_profile", h)
    return {name: {"ms": p.ms[i], "launches": p.launches[i], "slots": p.slots[i]}
            for i, name in enumerate(PROF_NAMES)}


def rs_iteration(h):
    return load().rs_iteration(h)


def rs_system_size(h):
    return load().rs_system_size(h)


def rs_get_state(h, x=None, x_prev=None, r=None, r_prev=None):
    _check(load().rs_get_state(h, _ptr(x), _ptr(x_prev), _ptr(r), _ptr(r_prev)), "rs_get_state", h)


def rs_set_state(h, k, x, x_prev, r, r_prev):
    vs = [np.ascontiguousarray(v, dtype=np.float64) for v in (x, x_prev, r, r_prev)]
    _check(load().rs_set_state(h, int(k), *[_ptr(v) for v in vs]), "rs_set_state", h)


def rs_get_weights(h, w_out):
    _check(load().rs_get_weights(h, _ptr(w_out)), "rs_get_weights", h)


def rs_get_last_sketch(h, rows, cols, signs):
    nnz = ctypes.c_int64(0)
    _check(load().rs_get_last_sketch(h, _ptr(rows), _ptr(cols), _ptr(signs), ctypes.byref(nnz)),
           "rs_get_last_sketch", h)
    return nnz.value


def rs_get_products(h, as_out=None, ginv_out=None):
    _check(load().rs_get_products(h, _ptr(as_out), _ptr(ginv_out)), "rs_get_products", h)


def rs_get_history(h, out, count):
    _check(load().rs_get_history(h, _ptr(out), int(count)), "rs_get_history", h)


def rs_destroy(h):
    if h:
        load().rs_destroy(h)


def rs_sketch_size(h):
    return load().rs_sketch_size(h)


def rs_get_route(h):
    r = ctypes.c_int32(0)
    n = ctypes.c_int64(0)
    _check(load().rs_get_route(h, ctypes.byref(r), ctypes.byref(n)), "rs_get_route", h)
    return r.value, n.value


def rs_set_sampler_params(h, params):
    p = np.ascontiguousarray(params, dtype=np.float32)
    assert p.shape == (RS_MLP_PARAMS,)
    _check(load().rs_set_sampler_params(h, _ptr(p)), "rs_set_sampler_params", h)


def rs_trace_count(h):
    n = ctypes.c_int64(0)
    _check(load().rs_trace_count(h, ctypes.byref(n)), "rs_trace_count", h)
    return n.value


def rs_get_trace(h, F, credits, first, count):
    _check(load().rs_get_trace(h, _ptr(F), _ptr(credits), int(first), int(count)), "rs_get_trace", h)


def rs_get_proposal(h, q, ok=None):
    _check(load().rs_get_proposal(h, _ptr(q), _ptr(ok)), "rs_get_proposal", h)


def _f32(a):
    return np.ascontiguousarray(a, dtype=np.float32)


def rs_mlp_init(seed):
    out = np.zeros(RS_MLP_PARAMS, dtype=np.float32)
    _check(load().rs_mlp_init(int(seed), _ptr(out)), "rs_mlp_init")
    return out


def rs_mlp_forward(params, F):
    P, Fm = _f32(params), _f32(F)
    out = np.zeros(Fm.shape[0], dtype=np.float32)
    _check(load().rs_mlp_forward(_ptr(P), _ptr(Fm), Fm.shape[0], _ptr(out)), "rs_mlp_forward")
    return out


def rs_mlp_gradient(params, Fs, credits):
    P, Fm, C = _f32(params), _f32(Fs), _f32(credits)
    nrec, tau = C.shape
    g = np.zeros(RS_MLP_PARAMS, dtype=np.float32)
    loss = ctypes.c_double(0.0)
    _check(load().rs_mlp_gradient(_ptr(P), _ptr(Fm), _ptr(C), nrec, tau, _ptr(g), ctypes.byref(loss)),
           "rs_mlp_gradient")
    return loss.value, g


def rs_adam_update(params, m1, m2, grad, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    P, a, v, g = _f32(params).copy(), _f32(m1).copy(), _f32(m2).copy(), _f32(grad)
    _check(load().rs_adam_update(_ptr(P), _ptr(a), _ptr(v), _ptr(g), int(t), lr, b1, b2, eps), "rs_adam_update")
    return P, a, v


def rs_proposal(s, eps=0.1):
    sv = _f32(s)
    q = np.zeros(sv.shape[0], dtype=np.float32)
    ok = np.zeros(1, dtype=np.int32)
    _check(load().rs_proposal(_ptr(sv), sv.shape[0], eps, _ptr(q), _ptr(ok)), "rs_proposal")
    return q, bool(ok[0])


def rs_features(a, r, rp, last, k):
    a, r, rp = (np.ascontiguousarray(v, dtype=np.float64) for v in (a, r, rp))
    last = np.ascontiguousarray(last, dtype=np.int32)
    F = np.zeros((a.shape[0], RS_MLP_FEATURES), dtype=np.float32)
    _check(load().rs_features(_ptr(a), _ptr(r), _ptr(rp), _ptr(last), a.shape[0], int(k), _ptr(F)), "rs_features")
    return F


def rs_draw_weighted(q, tau, seed, problem_id, k):
    qv = _f32(q)
    C = np.zeros(int(tau), dtype=np.int32)
    _check(load().rs_draw_weighted(_ptr(qv), qv.shape[0], int(tau), int(seed), int(problem_id), int(k), _ptr(C)),
           "rs_draw_weighted")
    return C


def rs_draw_weighted_noalloc(q, tau, seed, problem_id, k, C_out, status_out, stream=None):
    """Enqueue the weighted draw on device tensors (q: m float32, C_out: >= tau int32,
    status_out: one int32); returns the entry point's status. Nothing is allocated."""
    for t, dt in ((q, "float32"), (C_out, "int32"), (status_out, "int32")):
        if not _is_device(t) or str(t.dtype) != f"torch.{dt}" or not t.is_contiguous():
            raise ValueError("q, C_out and status_out must be contiguous device tensors "
                             "(float32, int32, int32)")
    if C_out.numel() < int(tau) or status_out.numel() < 1:
        raise ValueError("C_out needs tau entries and status_out one")
    return load().rs_draw_weighted_noalloc(_ptr(q), q.numel(), int(tau), int(seed), int(problem_id), int(k),
                                           _ptr(C_out), _ptr(status_out), stream)


class Trainer:
    """Owns one rs_trainer (MLP parameters, Adam state and a store of trace records)."""

    def __init__(self, tau, init_seed=1):
        self.t = _P()
        _check(load().rs_trainer_create(int(tau), int(init_seed), ctypes.byref(self.t)), "rs_trainer_create")
        self.tau = int(tau)

    def _chk(self, st, where):
        if st < 0:
            raise RsError(st, where, load().rs_trainer_last_error(self.t).decode())

    def add_traces(self, solver):
        self._chk(load().rs_trainer_add_traces(self.t, solver.h), "rs_trainer_add_traces")

    def add_records(self, F, credits):
        Fm, C = _f32(F), _f32(credits)
        self._chk(load().rs_trainer_add_records(self.t, _ptr(Fm), _ptr(C), C.shape[0]), "rs_trainer_add_records")

    @property
    def records(self):
        n = ctypes.c_int64(0)
        self._chk(load().rs_trainer_records(self.t, ctypes.byref(n)), "rs_trainer_records")
        return n.value

    def fit(self, epochs, batch=16, lr=1e-3, shuffle_seed=1):
        out = np.zeros(max(1, epochs))
        self._chk(load().rs_trainer_fit(self.t, int(epochs), int(batch), float(lr), int(shuffle_seed), _ptr(out)),
                  "rs_trainer_fit")
        return out[:epochs]

    def evaluate(self):
        """(mean loss over the stored records, mean entropy of their targets: the loss floor)."""
        loss, floor = ctypes.c_double(0.0), ctypes.c_double(0.0)
        self._chk(load().rs_trainer_eval(self.t, ctypes.byref(loss), ctypes.byref(floor)), "rs_trainer_eval")
        return loss.value, floor.value

    def params(self):
        out = np.zeros(RS_MLP_PARAMS, dtype=np.float32)
        self._chk(load().rs_trainer_get_params(self.t, _ptr(out)), "rs_trainer_get_params")
        return out

    def set_params(self, p):
        pv = _f32(p)
        self._chk(load().rs_trainer_set_params(self.t, _ptr(pv)), "rs_trainer_set_params")

    def close(self):
        if self.t:
            load().rs_trainer_destroy(self.t)
            self.t = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def batch_last_error(b=None):
    return load().rs_batch_last_error(b).decode()


def _bcheck(status, where, b=None):
    if status < 0:
        raise RsError(status, where, batch_last_error(b))
    return status


def rs_batch_create(problems, opts):
    arr = (rs_problem * len(problems))(*problems)
    b = _P()
    _bcheck(load().rs_batch_create(len(problems), arr, ctypes.byref(opts), ctypes.byref(b)),
            "rs_batch_create")
    return b


def rs_batch_step(b, iters):
    _bcheck(load().rs_batch_step(b, int(iters)), "rs_batch_step", b)


def rs_batch_solve(b):
    rep = rs_batch_report()
    st = _bcheck(load().rs_batch_solve(b, ctypes.byref(rep)), "rs_batch_solve", b)
    return st, rep


def rs_batch_reset(b, seed):
    _bcheck(load().rs_batch_reset(b, int(seed)), "rs_batch_reset", b)


def rs_batch_iteration(b):
    return load().rs_batch_iteration(b)


def rs_batch_problem_info(b, p):
    info = rs_batch_problem_info_t()
    _bcheck(load().rs_batch_problem_info(b, int(p), ctypes.byref(info)), "rs_batch_problem_info", b)
    return info


def rs_batch_slot_report(b, p, stop_iter=None, rel_res=None):
    _bcheck(load().rs_batch_slot_report(b, int(p), _ptr(stop_iter), _ptr(rel_res)), "rs_batch_slot_report", b)


def rs_batch_get_state(b, p, slot, x=None, x_prev=None, r=None, r_prev=None):
    _bcheck(load().rs_batch_get_state(b, int(p), int(slot), _ptr(x), _ptr(x_prev), _ptr(r), _ptr(r_prev)),
            "rs_batch_get_state", b)


def rs_batch_get_weights(b, p, w_out):
    _bcheck(load().rs_batch_get_weights(b, int(p), _ptr(w_out)), "rs_batch_get_weights", b)


def rs_batch_get_tuning(b):
    t = rs_tuning()
    _bcheck(load().rs_batch_get_tuning(b, ctypes.byref(t)), "rs_batch_get_tuning", b)
    return {name: getattr(t, name) for name, _ in rs_tuning._fields_}


def rs_batch_destroy(b):
    if b:
        load().rs_batch_destroy(b)


# ---------------------------------------------------------------- convenience wrapper
def make_matrix(X):
    """rs_matrix for a numpy array, a scipy CSR matrix, or torch CUDA tensors.

    Returns (rs_matrix, keepalive) -- keep `keepalive` until rs_create returns.
    """
    import scipy.sparse as sp
    keep = []
    M = rs_matrix()
    if isinstance(X, tuple):  # (indptr, indices, data, shape) as torch CUDA tensors
        indptr, indices, data, shape = X
        M.n, M.d = shape
        M.layout = RS_CSR
        M.dtype = RS_F32 if str(data.dtype).endswith("float32") else RS_F64
        M.vals, M.row_ptr, M.col_idx = data.data_ptr(), indptr.data_ptr(), indices.data_ptr()
        M.nnz = int(data.numel())
        M.mem = RS_DEVICE
        keep += [indptr, indices, data]
        return M, keep
    if sp.issparse(X):
        X = sp.csr_matrix(X)
        X.sort_indices()
        indptr = np.ascontiguousarray(X.indptr, dtype=np.int64)
        indices = np.ascontiguousarray(X.indices, dtype=np.int32)
        data = np.ascontiguousarray(X.data)
        if data.dtype not in (np.float32, np.float64):
            data = data.astype(np.float64)
        M.n, M.d = X.shape
        M.layout = RS_CSR
        M.dtype = RS_F32 if data.dtype == np.float32 else RS_F64
        M.vals, M.row_ptr, M.col_idx = data.ctypes.data, indptr.ctypes.data, indices.ctypes.data
        M.nnz = int(data.shape[0])
        M.mem = RS_HOST
        keep += [indptr, indices, data]
        return M, keep
    if isinstance(X, np.ndarray):
        A = X if X.dtype in (np.float32, np.float64) else X.astype(np.float64)
        if A.flags.c_contiguous:
            M.layout = RS_DENSE_ROWMAJOR
        elif A.flags.f_contiguous:
            M.layout = RS_DENSE_COLMAJOR
        else:
            A = np.ascontiguousarray(A)
            M.layout = RS_DENSE_ROWMAJOR
        M.n, M.d = A.shape
        M.dtype = RS_F32 if A.dtype == np.float32 else RS_F64
        M.vals = A.ctypes.data
        M.mem = RS_HOST
        keep.append(A)
        return M, keep
    # torch tensor on the GPU, row-major contiguous
    A = X.contiguous()
    M.n, M.d = A.shape
    M.layout = RS_DENSE_ROWMAJOR
    M.dtype = RS_F32 if str(A.dtype).endswith("float32") else RS_F64
    M.vals = A.data_ptr()
    M.mem = RS_DEVICE if _is_device(A) else RS_HOST
    keep.append(A)
    return M, keep


class Solver:
    """Owns one rs_handle. `X` and `y` may live on the host (numpy) or the GPU (torch).
    With kernel_sigma set, X holds the points of a kernel ridge problem (rs_create_kernel)
    and the weights are its coefficients alpha."""

    def __init__(self, X, y, lam, *, tau, sketch="subsample", form="auto", momentum="heuristic",
                 precision="fp64", subcount_k=0, tol=1e-6, max_iter=100000, seed=1, problem_id=0,
                 eta=0.995, beta_max=0.5, gamma=1.0, beta=0.5, lookahead=0, refresh_every=20,
                 profile=False, stream=None, sampler="uniform", trace_every=0, trace_capacity=0,
                 sparse_route="auto", pipeline=True, kernel_sigma=None, accel=None, dense_route="products",
                 refresh_early=True):
        o = rs_options_default()
        o.dense_route = {"products": 0, "gram": 1}[dense_route]
        o.refresh_early = int(bool(refresh_early))
        if accel is not None:  # (mu, nu) of the accelerated method (Alg. 3)
            o.accelerated, o.accel_mu, o.accel_nu = 1, float(accel[0]), float(accel[1])
        o.form, o.sketch, o.tau = FORMS[form], SKETCHES[sketch], int(tau)
        o.subcount_k, o.momentum, o.precision = int(subcount_k), MOMENTA[momentum], PRECISIONS[precision]
        o.gamma, o.beta, o.eta, o.beta_max, o.tol = gamma, beta, eta, beta_max, tol
        o.max_iter, o.seed, o.problem_id = int(max_iter), int(seed), int(problem_id)
        o.refresh_every, o.lookahead, o.profile = int(refresh_every), int(lookahead), int(profile)
        o.stream = stream
        o.sampler, o.trace_every, o.trace_capacity = SAMPLERS[sampler], int(trace_every), int(trace_capacity)
        o.sparse_route = ROUTES[sparse_route]
        o.pipeline = int(bool(pipeline))
        M, keep = make_matrix(X)
        if M.mem == RS_DEVICE:
            yv = y.double().contiguous()
        else:
            yv = np.ascontiguousarray(np.asarray(y, dtype=np.float64))
        keep.append(yv)
        if kernel_sigma is None:
            self.h = rs_create(M, yv, lam, o)
            self.d = int(M.d)
        else:
            self.h = rs_create_kernel(M, yv, kernel_sigma, lam, o)
            self.d = int(M.n)  # the coefficients alpha
        self.m = rs_system_size(self.h)
        self.tau = int(tau)

    def reset(self, seed):
        rs_reset(self.h, seed)

    def profile(self, clear=False):
        return rs_get_profile(self.h, clear)

    def step(self, iters):
        return rs_step(self.h, iters)

    def solve(self):
        w = np.zeros(self.d)
        st, rep = rs_solve(self.h, w)
        return w, st, rep

    @property
    def k(self):
        return rs_iteration(self.h)

    def state(self):
        x, xp, r, rp = (np.zeros(self.m) for _ in range(4))
        rs_get_state(self.h, x, xp, r, rp)
        return x, xp, r, rp

    def set_state(self, k, x, x_prev, r, r_prev):
        """Resume at iteration k from a saved (x^k, x^{k-1}, r^k, r^{k-1})."""
        for v in (x, x_prev, r, r_prev):
            if np.shape(v) != (self.m,):
                raise ValueError(f"state vectors must have {self.m} entries")
        rs_set_state(self.h, k, x, x_prev, r, r_prev)

    def weights(self):
        w = np.zeros(self.d)
        rs_get_weights(self.h, w)
        return w

    def last_sketch(self):
        rows = np.zeros(self.m, dtype=np.int32)
        cols = np.zeros(self.m, dtype=np.int32)
        signs = np.zeros(self.m, dtype=np.int8)
        n = rs_get_last_sketch(self.h, rows, cols, signs)
        return rows[:n].astype(np.int64), cols[:n].astype(np.int64), signs[:n].astype(np.float64)

    def products(self):
        """(AS, G^{-1}) of the last iteration's sketch, as FP64 arrays."""
        tau = self.tau
        AS = np.zeros((self.m, tau))
        Gi = np.zeros((tau, tau))
        rs_get_products(self.h, AS, Gi)
        return AS, Gi

    def set_sampler_params(self, params):
        rs_set_sampler_params(self.h, params)

    def trace(self):
        n = rs_trace_count(self.h)
        F = np.zeros((n, self.tau, RS_MLP_FEATURES), dtype=np.float32)
        C = np.zeros((n, self.tau), dtype=np.float32)
        if n:
            rs_get_trace(self.h, F, C, 0, n)
        return F, C

    def proposal(self):
        q = np.zeros(self.m, dtype=np.float32)
        ok = np.zeros(1, dtype=np.int32)
        rs_get_proposal(self.h, q, ok)
        return q, bool(ok[0])

    def history(self):
        out = np.zeros(self.k + 1)
        rs_get_history(self.h, out, self.k + 1)
        return out

    def close(self):
        if self.h:
            rs_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Owns one rs_batch. `problems` is a list of dicts with keys X (numpy array or scipy
    CSR), y (n or n x nrhs), lambdas (sequence), and optionally tau, form, max_iter."""

    def __init__(self, problems, *, momentum="heuristic", tol=1e-6, max_iter=100000, seed=1,
                 problem_id=0, eta=0.995, beta_max=0.5, gamma=1.0, beta=0.5, graph_iters=0,
                 autotune=False, stream=None, precision="fp64", refresh_every=20):
        o = rs_options_default()
        o.precision = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
        o.refresh_every = int(refresh_every)
        o.momentum = MOMENTA[momentum] if isinstance(momentum, str) else int(momentum)
        o.tol, o.max_iter = tol, int(max_iter)
        o.seed, o.problem_id = int(seed), int(problem_id)
        o.eta, o.beta_max, o.gamma, o.beta = eta, beta_max, gamma, beta
        o.graph_iters, o.autotune, o.stream = int(graph_iters), int(bool(autotune)), stream
        self._keep = []
        structs = []
        self.shapes = []
        for pr in problems:
            M, keep = make_matrix(pr["X"])
            y = np.asarray(pr["y"], dtype=np.float64)
            if y.ndim == 1:
                y = y[:, None]
            yv = np.asfortranarray(y)
            lam = np.ascontiguousarray(np.asarray(pr["lambdas"], dtype=np.float64))
            keep += [yv, lam]
            self._keep.append(keep)
            P = rs_problem()
            P.X = M
            P.y = yv.ctypes.data
            P.nrhs = yv.shape[1]
            P.lambdas = lam.ctypes.data
            P.nlambda = lam.shape[0]
            P.tau = int(pr.get("tau", 0))
            P.sketch = -1
            P.form = FORMS[pr.get("form", "auto")]
            P.max_iter = int(pr.get("max_iter", 0))
            structs.append(P)
            self.shapes.append((int(M.n), int(M.d), yv.shape[1], lam.shape[0]))
        self.b = rs_batch_create(structs, o)
        self._keep = None  # the library copied X and y

    def info(self, p):
        return rs_batch_problem_info(self.b, p)

    def step(self, iters):
        rs_batch_step(self.b, iters)

    def solve(self):
        return rs_batch_solve(self.b)

    def reset(self, seed):
        rs_batch_reset(self.b, seed)

    @property
    def k(self):
        return rs_batch_iteration(self.b)

    def slots(self, p):
        J = self.info(p).slots
        stop = np.zeros(J, dtype=np.int64)
        rel = np.zeros(J)
        rs_batch_slot_report(self.b, p, stop, rel)
        return stop, rel

    def state(self, p, slot):
        m = self.info(p).m
        x, xp, r, rp = (np.zeros(m) for _ in range(4))
        rs_batch_get_state(self.b, p, slot, x, xp, r, rp)
        return x, xp, r, rp

    def weights(self, p):
        n, d, nrhs, nlam = self.shapes[p]
        w = np.zeros((nrhs * nlam, d))
        rs_batch_get_weights(self.b, p, w)
        return w  # row j = slot j = l * nrhs + q

    def tuning(self):
        return rs_batch_get_tuning(self.b)

    def close(self):
        if self.b:
            rs_batch_destroy(self.b)
            self.b = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
