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
    with pytest.raises(mala.MalaError):                     # every grid dimension must be >= 1
        sv.submit(pos, L, np.array([-1, -1, 5]), rc, tj, eg, T, ne)
    with pytest.raises(mala.MalaError):
        sv.reserve([(4, np.array([8.1] * 3), np.array([-2, -2, 40]), 4.67, 10, eg, 933.0)])
    sv.close()


def test_reserve_checks_budget_and_idleness(mala):
    shape = (4, np.array([8.1] * 3), np.array([40] * 3), 4.67, 10, mala_synth.EGRID, 933.0)
    sv = mala.Server(max_inflight=2, hbm_budget=1 << 40, mock_ns_per_point=0.0)
    sv.reserve([shape, shape])
    st = sv.stats()
    assert st["reserved_bytes_per_slot"] > 0 and st["allocations"] == 0
    sv.close()
    # two slots at the reserved size do not fit a budget of one
    probe = mala.Server(max_inflight=1, hbm_budget=1 << 40, mock_ns_per_point=0.0)
    probe.reserve([shape])
    per_slot = probe.stats()["reserved_bytes_per_slot"]
    probe.close()
    tight = mala.Server(max_inflight=2, hbm_budget=int(1.5 * per_slot), mock_ns_per_point=0.0)
    with pytest.raises(mala.MalaError) as e:
        tight.reserve([shape])
    assert e.value.status == mala.MALA_E_OOM
    tight.close()
    # a server with work in flight refuses to resize its slots
    busy = mala.Server(max_inflight=1, hbm_budget=1 << 40, mock_ns_per_point=1e4)
    t = busy.submit(*_req(40))
    with pytest.raises(mala.MalaError) as e:
        busy.reserve([shape])
    assert e.value.status == mala.MALA_E_BUSY
    busy.wait(t, 30)
    busy.close()


def test_allocation_counter_counts_slot_growth(mala):
    sv = mala.Server(max_inflight=1, hbm_budget=1 << 40, mock_ns_per_point=0.0)
    for n in (20, 10, 40, 30):
        sv.wait(sv.submit(*_req(n)), 30)
    # the slot grows for the first request and for the larger third one only
    assert sv.stats()["allocations"] == 2
    sv.close()


def test_inflight_points_cap_runs_large_requests_alone(mala):
    sv = mala.Server(max_inflight=3, hbm_budget=1 << 40, mock_ns_per_point=500.0)
    sv.set_inflight_points(40 ** 3)
    # 40^3 fills the cap alone; the two 20^3 requests may run together
    tickets = [sv.submit(*_req(n)) for n in (40, 20, 20, 40)]
    o = [sv.wait(t, 30) for t in tickets]
    sv.close()
    assert o[1]["t_start"] >= o[0]["t_done"]            # waits for the large one
    assert o[2]["t_start"] < o[1]["t_done"]             # small ones overlap
    assert o[3]["t_start"] >= max(o[1]["t_done"], o[2]["t_done"])
