"""Scheduler of the serving loop with the host-only mock executor (no GPU):
admission in arrival order, the HBM budget, rejection of requests that can
never fit, and completion of every ticket."""
import numpy as np
import pytest

import mala_synth

pytest.importorskip("ctypes")


@pytest.fixture(scope="module")
def mala():
    import paper_2411_19617_amd as m
    try:
        m.lib()
    except ImportError:
        pytest.skip("libmala.so not built")
    return m


def _req(n_grid, T=298.0):
    L = np.array([8.1, 8.1, 8.1])
    pos = np.zeros((4, 3))
    return pos, L, np.array([n_grid] * 3), 4.67, 10, mala_synth.EGRID, T, 12.0


def test_fifo_and_all_done(mala):
    sv = mala.Server(max_inflight=2, hbm_budget=1 << 40, mock_ns_per_point=200.0)
    tickets = [sv.submit(*_req(n)) for n in (40, 10, 30, 20, 10, 50)]
    outs = [sv.wait(t, 30) for t in tickets]
    starts = [o["t_start"] for o in outs]
    assert starts == sorted(starts)                      # admitted in arrival order
    for t, o in zip(tickets, outs):
        assert o["dos"][0] == t and o["t_done"] >= o["t_start"] >= o["t_submit"]
    sv.close()


def test_budget_limits_concurrency(mala):
    # each request needs roughly the same bytes; a budget of ~1.5 requests
    # allows only one in flight although two slots exist
    probe = mala.Server(max_inflight=1, hbm_budget=1 << 40, mock_ns_per_point=0.0)
    t = probe.submit(*_req(40))
    probe.wait(t, 10)
    need = probe.stats()["peak_bytes"]
    probe.close()
    sv = mala.Server(max_inflight=2, hbm_budget=int(1.5 * need), mock_ns_per_point=300.0)
    tickets = [sv.submit(*_req(40)) for _ in range(4)]
    outs = [sv.wait(t, 30) for t in tickets]
    for a, b in zip(outs, outs[1:]):
        assert b["t_start"] >= a["t_done"] - 1e-3            # strictly one at a time
    assert sv.stats()["peak_bytes"] <= 1.5 * need
    sv.close()


def test_oversized_request_rejected(mala):
    sv = mala.Server(max_inflight=2, hbm_budget=1 << 20, mock_ns_per_point=0.0)
    with pytest.raises(mala.MalaError) as e:
        sv.submit(*_req(60))
    assert e.value.status == mala.MALA_E_OOM
    sv.close()


def test_poll_busy_then_done(mala):
    sv = mala.Server(max_inflight=1, hbm_budget=1 << 40, mock_ns_per_point=2000.0)
    t = sv.submit(*_req(40))                                 # 64000 points -> ~0.13 s
    assert sv.poll(t) is None
    o = sv.wait(t, 10)
    assert o["dos"][0] == t
    with pytest.raises(mala.MalaError):
        sv.poll(t)                                           # ticket already taken
    sv.close()


def test_invalid_requests(mala):
    sv = mala.Server(max_inflight=1, hbm_budget=1 << 40, mock_ns_per_point=0.0)
    pos, L, N, rc, tj, eg, T, ne = _req(10)
    with pytest.raises(mala.MalaError):
        sv.submit(pos, L, N, rc, 7, eg, T, ne)
    with pytest.raises(mala.MalaError):
        sv.submit(pos, L, N, rc, tj, eg, -5.0, ne)
    sv.close()
