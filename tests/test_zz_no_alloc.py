"""GPU: rs_draw_weighted_noalloc (device buffers, no allocation) against rs_draw_weighted.

The draw is index work, so the bar is bit-exactness: two calls in a row (the second on a
smaller proposal) equal the allocating entry point's draws and the oracle's; a proposal
with a zero entry is reported through the status word without writing the output; sizes
beyond the fixed working array are rejected before anything is enqueued.
"""
import numpy as np
import pytest

from oracle import sketch as osk
from paper_2105_05565_amd import rs

pytestmark = pytest.mark.gpu


def _proposal(m, seed):
    rng = np.random.default_rng(seed)
    q = np.exp(3 * rng.standard_normal(m)).astype(np.float32)
    return q / q.sum()


def _draw_noalloc(torch, q, tau, seed, pid, k, fill=-7):
    qd = torch.from_numpy(q).cuda()
    C = torch.full((tau,), fill, dtype=torch.int32, device="cuda")
    st = torch.full((1,), 99, dtype=torch.int32, device="cuda")
    s = torch.cuda.current_stream()
    ret = rs.rs_draw_weighted_noalloc(qd, tau, seed, pid, k, C, st, stream=s.cuda_stream)
    s.synchronize()
    return ret, C.cpu().numpy(), int(st.cpu()[0])


def test_noalloc_draw_matches_allocating_entry_point():
    torch = pytest.importorskip("torch")
    torch.cuda.set_device(0)
    # the second call is smaller (m and tau) and must not see the first call's contents
    for m, tau, seed, pid, k in ((70000, 512, 9, 2, 13), (3001, 40, 4, 0, 0)):
        q = _proposal(m, m + tau)
        ret, got, status = _draw_noalloc(torch, q, tau, seed, pid, k)
        assert ret == 0 and status == 0, (ret, status)
        ref = rs.rs_draw_weighted(q, tau, seed=seed, problem_id=pid, k=k)
        assert np.array_equal(got, ref), (m, tau, got[:8], ref[:8])
        exp = osk.draw_weighted(seed, pid, k, q, tau)
        assert np.array_equal(got.astype(np.int64), exp.rows)


def test_noalloc_draw_rejects_bad_proposal_and_recovers():
    torch = pytest.importorskip("torch")
    torch.cuda.set_device(0)
    m, tau = 5000, 64
    q = _proposal(m, 3)
    bad = q.copy()
    bad[1234] = 0.0
    ret, got, status = _draw_noalloc(torch, bad, tau, 1, 0, 5)
    assert ret == 0 and status == rs.RS_EINVAL
    assert np.all(got == -7)  # not written
    # the next call starts from cleared flags
    ret, got, status = _draw_noalloc(torch, q, tau, 1, 0, 5)
    assert ret == 0 and status == 0
    assert np.array_equal(got, rs.rs_draw_weighted(q, tau, seed=1, problem_id=0, k=5))


def test_noalloc_draw_rejects_sizes_beyond_its_array():
    torch = pytest.importorskip("torch")
    torch.cuda.set_device(0)
    m = (1 << 20) + 1
    q = torch.full((m,), 1.0 / m, dtype=torch.float32, device="cuda")
    C = torch.zeros(8, dtype=torch.int32, device="cuda")
    st = torch.full((1,), 99, dtype=torch.int32, device="cuda")
    assert rs.rs_draw_weighted_noalloc(q, 8, 1, 0, 0, C, st) == rs.RS_EINVAL
    torch.cuda.synchronize()
    assert int(st.cpu()[0]) == 99  # nothing enqueued
