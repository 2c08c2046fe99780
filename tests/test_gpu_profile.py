"""GPU: the HIP-event profiling levels report every kernel class they promise."""
import numpy as np
import pytest

from paper_2105_05565_amd import inputs, rs

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("level", [1, 2, 3])
def test_profile_levels(level):
    p = inputs.make_csr(400, 150, 0.04, 0.05, seed=3, dtype=np.float32)
    S = rs.Solver(p.X, p.y, p.lam, tau=23, sketch="count", tol=0.0, profile=level, lookahead=8)
    S.step(20)
    prof = S.profile(clear=True)
    assert prof["as"]["launches"] == 3 and prof["as"]["ms"] > 0, prof["as"]
    if level == 3:  # the products only
        for cls in ("sketch", "chol", "iters", "delta", "update"):
            assert prof[cls]["launches"] == 0, (cls, prof[cls])
        assert S.profile()["as"]["launches"] == 0  # cleared
        S.close()
        return
    for cls in ("sketch", "chol", "iters"):
        assert prof[cls]["launches"] == 3 and prof[cls]["ms"] > 0, (cls, prof[cls])
    assert prof["iters"]["slots"] == 20
    if level == 2:
        assert prof["delta"]["launches"] == 20 and prof["update"]["launches"] == 20
    else:
        assert prof["delta"]["launches"] == 0
    assert S.profile()["as"]["launches"] == 0  # cleared
    S.close()


def test_profile_level_out_of_range():
    p = inputs.make_csr(100, 40, 0.1, 0.1, seed=1, dtype=np.float32)
    for bad in (-1, 4):
        with pytest.raises(rs.RsError) as e:
            rs.Solver(p.X, p.y, p.lam, tau=5, sketch="count", profile=bad)
        assert e.value.status == rs.RS_EINVAL
