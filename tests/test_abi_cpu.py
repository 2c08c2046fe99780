"""Host-side checks of the C ABI: the library loads, exports every declared entry
point, and rejects bad arguments before touching a device (no GPU needed)."""
import ctypes
import math
import os
import re

import numpy as np
import pytest

from paper_2105_05565_amd import rs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rs.h")

pytestmark = pytest.mark.skipif(not os.path.exists(rs.LIB_PATH), reason="librs.so not built")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(rs_[a-z_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ["rs_create", "rs_step", "rs_solve", "rs_destroy", "rs_get_state", "rs_status_string"]:
        assert must in names


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(rs.LIB_PATH)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing
    assert set(declared_functions()) == set(rs.SIGNATURES), "binding and header disagree"


def test_status_strings_and_defaults():
    assert rs.status_string(rs.RS_OK) == "ok"
    assert "invalid" in rs.status_string(rs.RS_EINVAL)
    o = rs.rs_options_default()
    assert o.tol == 1e-6 and o.eta == 0.995 and o.beta_max == 0.5 and o.momentum == rs.RS_MOMENTUM_HEURISTIC


def _create(X, y, lam, **kw):
    o = rs.rs_options_default()
    for k, v in kw.items():
        setattr(o, k, v)
    M, keep = rs.make_matrix(X)
    yv = np.ascontiguousarray(y, dtype=np.float64)
    h = rs.rs_create(M, yv, lam, o)
    rs.rs_destroy(h)


@pytest.mark.parametrize("kw,lam", [
    (dict(tau=0), 1.0),                      # tau < 1
    (dict(tau=9), 1.0),                      # tau > m = 8
    (dict(tau=3), 0.0),                      # lambda <= 0
    (dict(tau=3), -1.0),
    (dict(tau=3), math.inf),
    (dict(tau=3, max_iter=-1), 1.0),
    (dict(tau=3, tol=-1.0), 1.0),
    (dict(tau=3, momentum=7), 1.0),
    (dict(tau=3, form=9), 1.0),
    (dict(tau=3, sketch=9), 1.0),
    (dict(tau=3, profile=4), 1.0),           # profiling levels 0 .. 3
    (dict(tau=3, profile=-1), 1.0),
    (dict(tau=3, refresh_early=2), 1.0),     # 0 or 1
])
def test_rejects_bad_arguments_without_device(kw, lam):
    X = np.ones((20, 8))
    with pytest.raises(rs.RsError) as e:
        _create(X, np.ones(20), lam, **kw)
    assert e.value.status == rs.RS_EINVAL


def test_rejects_nonfinite_targets():
    y = np.ones(20)
    y[3] = np.nan
    with pytest.raises(rs.RsError) as e:
        _create(np.ones((20, 8)), y, 1.0, tau=3)
    assert e.value.status == rs.RS_EINVAL
    assert "non-finite" in rs.last_error()


def test_rejects_unsupported_combinations():
    import scipy.sparse as sp
    # count sketch on dense data: only FP64 (dense S products)
    with pytest.raises(rs.RsError) as e:
        _create(np.ones((20, 8)), np.ones(20), 1.0, tau=3, sketch=rs.RS_SKETCH_COUNT,
                precision=rs.RS_PREC_MIXED_BF16)
    assert e.value.status == rs.RS_EUNSUPPORTED
    for kind in (rs.RS_SKETCH_GAUSSIAN, rs.RS_SKETCH_SRHT):
        with pytest.raises(rs.RsError) as e:  # dense sketches need dense data
            _create(sp.random(20, 8, density=0.3, format="csr", random_state=0), np.ones(20), 1.0, tau=3,
                    sketch=kind)
        assert e.value.status == rs.RS_EUNSUPPORTED
        with pytest.raises(rs.RsError) as e:  # and not the accelerated method
            _create(np.ones((20, 8)), np.ones(20), 1.0, tau=3, sketch=kind, accelerated=1)
        assert e.value.status == rs.RS_EUNSUPPORTED
    X = sp.random(20, 8, density=0.3, format="csr", random_state=0)
    with pytest.raises(rs.RsError) as e:
        _create(X, np.ones(20), 1.0, tau=3, sketch=rs.RS_SKETCH_SUBCOUNT, subcount_k=3)  # 9 > m
    assert e.value.status == rs.RS_EINVAL


def test_binding_fails_loudly_without_library(tmp_path):
    saved = rs._lib
    try:
        rs._lib = None
        with pytest.raises(RuntimeError):
            rs.load(str(tmp_path / "nope.so"))
    finally:
        rs._lib = saved


def _batch_problem(n=30, d=10, nrhs=1, lams=(1.0,), csr=False, **kw):
    import scipy.sparse as sp
    rng = np.random.default_rng(0)
    X = rng.standard_normal((n, d))
    if csr:
        X = sp.csr_matrix(X * (rng.random((n, d)) < 0.3))
    pr = dict(X=X, y=rng.standard_normal((n, nrhs)), lambdas=list(lams))
    pr.update(kw)
    return pr


@pytest.mark.parametrize("pr,opt", [
    (dict(nrhs=9), {}),                                  # nrhs > 8
    (dict(nrhs=2, lams=[1.0] * 33), {}),                 # nlambda * nrhs > 64
    (dict(lams=(0.0,)), {}),                             # lambda <= 0
    (dict(lams=(math.nan,)), {}),
    (dict(tau=11), {}),                                  # tau > m = 10
    (dict(tau=-1 + 2000), {}),
    (dict(), dict(tol=-1.0)),
    (dict(), dict(momentum=9)),
])
def test_batch_rejects_bad_arguments_without_device(pr, opt):
    kw = {k: v for k, v in pr.items() if k in ("nrhs", "lams", "csr")}
    extra = {k: v for k, v in pr.items() if k not in kw}
    problem = _batch_problem(**kw, **extra)
    with pytest.raises(rs.RsError) as e:
        rs.Batch([problem], **opt)
    assert e.value.status == rs.RS_EINVAL, rs.batch_last_error()


def test_batch_rejects_unbuilt_pairs_without_device():
    o = rs.rs_options_default()
    o.precision = 7  # neither FP64 nor mixed
    M, keep = rs.make_matrix(np.ones((20, 8)))
    y = np.ones(20)
    lam = np.ones(1)
    P = rs.rs_problem()
    P.X, P.y, P.nrhs, P.lambdas, P.nlambda, P.sketch = M, y.ctypes.data, 1, lam.ctypes.data, 1, -1
    with pytest.raises(rs.RsError) as e:
        rs.rs_batch_create([P], o)
    assert e.value.status == rs.RS_EINVAL
    o.precision = rs.RS_PREC_FP64
    P.sketch = rs.RS_SKETCH_COUNT  # count sketch on dense data
    with pytest.raises(rs.RsError) as e:
        rs.rs_batch_create([P], o)
    assert e.value.status == rs.RS_EUNSUPPORTED


@pytest.mark.parametrize("name,kw", [
    ("none", {}), ("constant", dict(gamma=0.8, beta=0.4)), ("heuristic", {}),
    ("heuristic", dict(eta=0.9, beta_max=0.3)), ("theory", {}), ("theory", dict(eta=0.9, beta_max=0.3)),
    ("theory", dict(eta=0.5, beta_max=0.99)), ("theory", dict(eta=1.0)), ("theory", dict(beta_max=-0.5)),
    ("theory", dict(eta=0.999, beta_max=0.999)),
])
def test_momentum_schedule_matches_oracle_bit_exact(name, kw):
    from oracle.solver import Options, schedule

    o = rs.rs_options_default()
    o.momentum = rs.MOMENTA[name]
    for f, v in kw.items():
        setattr(o, f, v)
    opts = Options(momentum=name, **{("gamma_const" if f == "gamma" else "beta_const" if f == "beta" else f): v
                                     for f, v in kw.items()})
    for k in list(range(0, 420)) + [999, 10**6, 2 * 10**6 + 1, 10**8]:
        assert rs.rs_momentum_schedule(o, k) == schedule(opts, k), (name, kw, k)


@pytest.mark.parametrize("kw", [dict(momentum=4), dict(momentum=-1), dict(momentum=3, eta=0.0),
                                dict(momentum=3, eta=1.5), dict(momentum=3, eta=math.nan),
                                dict(momentum=3, beta_max=math.nan)])
def test_momentum_settings_rejected(kw):
    o = rs.rs_options_default()
    for f, v in kw.items():
        setattr(o, f, v)
    with pytest.raises(rs.RsError) as e:
        rs.rs_momentum_schedule(o, 0)
    assert e.value.status == rs.RS_EINVAL
    with pytest.raises(rs.RsError) as e:
        _create(np.ones((20, 8)), np.ones(20), 1.0, tau=3, **kw)
    assert e.value.status == rs.RS_EINVAL


@pytest.mark.parametrize("sigma,kw,status", [
    (0.0, {}, rs.RS_EINVAL), (-1.0, {}, rs.RS_EINVAL), (math.nan, {}, rs.RS_EINVAL), (math.inf, {}, rs.RS_EINVAL),
    (0.5, dict(sketch=rs.RS_SKETCH_COUNT, precision=rs.RS_PREC_MIXED_BF16), rs.RS_EUNSUPPORTED),
    (0.5, dict(sampler=rs.SAMPLERS["diag"]), rs.RS_EUNSUPPORTED),
])
def test_kernel_create_rejects_without_device(sigma, kw, status):
    o = rs.rs_options_default()
    o.tau = 3
    for f, v in kw.items():
        setattr(o, f, v)
    M, keep = rs.make_matrix(np.ones((20, 4)))
    with pytest.raises(rs.RsError) as e:
        rs.rs_create_kernel(M, np.ones(20), sigma, 1.0, o)
    assert e.value.status == status


def test_kernel_create_rejects_csr_points():
    import scipy.sparse as sp
    o = rs.rs_options_default()
    o.tau = 3
    M, keep = rs.make_matrix(sp.random(20, 4, density=0.5, format="csr", random_state=1))
    with pytest.raises(rs.RsError) as e:
        rs.rs_create_kernel(M, np.ones(20), 0.5, 1.0, o)
    assert e.value.status == rs.RS_EINVAL


@pytest.mark.parametrize("kw,status", [
    (dict(accelerated=1, accel_mu=0.0, accel_nu=1.0), rs.RS_EINVAL),
    (dict(accelerated=1, accel_mu=1.5, accel_nu=1.0), rs.RS_EINVAL),
    (dict(accelerated=1, accel_mu=0.5, accel_nu=0.9), rs.RS_EINVAL),
    (dict(accelerated=1, accel_mu=0.5, accel_nu=2.5), rs.RS_EINVAL),
    (dict(accelerated=1, accel_mu=math.nan, accel_nu=1.0), rs.RS_EINVAL),
    (dict(accelerated=1, precision=rs.RS_PREC_MIXED_BF16), rs.RS_EUNSUPPORTED),
])
def test_accelerated_settings_rejected_without_device(kw, status):
    with pytest.raises(rs.RsError) as e:
        _create(np.ones((20, 8)), np.ones(20), 1.0, tau=3, **kw)
    assert e.value.status == status


def test_accelerated_defaults():
    o = rs.rs_options_default()
    assert o.accelerated == 0 and o.accel_mu == 1.0 and o.accel_nu == 1.0


def test_state_entry_points_reject_null_handle_without_device():
    lib = rs.load()
    z = np.zeros(4)
    p = z.ctypes.data
    assert lib.rs_set_state(None, 0, p, p, p, p) == rs.RS_EINVAL
    assert lib.rs_get_state(None, p, p, p, p) == rs.RS_EINVAL


def test_trainer_eval_rejects_null_without_device():
    lib = rs.load()
    d = np.zeros(2)
    assert lib.rs_trainer_eval(None, d.ctypes.data, d.ctypes.data) == rs.RS_EINVAL
