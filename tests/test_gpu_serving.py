"""Serving loop on the GPU: each request's result is the same alone and in
the mix (bitwise: same kernels, same per-request work partition), and
equals the single-snapshot call."""
import sys

import numpy as np
import pytest

import mala_synth

pytestmark = pytest.mark.gpu
EG = mala_synth.EGRID


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def mala():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2411_19617_amd as m
    m.lib()
    return m


def small_requests(n, seed=21, pts_per_atom=600.0):
    rng = mala_synth.SplitMix64(seed)
    out = []
    for _ in range(n):
        r = mala_synth.serving_request(rng, pts_per_atom=pts_per_atom)
        out.append(r)
    return out


def run(sv, r):
    return sv.submit(r.positions, r.L, r.N, r.rcut, r.twojmax, EG, r.T, r.n_electrons)


def test_alone_equals_in_mix(mala):
    net = mala_synth.paper_net()
    reqs = small_requests(6)
    log("requests", [(r.name, r.n_points) for r in reqs])
    sv = mala.Server(mala_synth.net_to_blob(net), mala.PREC_FP32, hbm_budget=32 << 30, max_inflight=3)
    x = reqs[2]
    alone = sv.wait(run(sv, x), 120)
    tickets = [run(sv, r) for r in reqs]            # x runs again, among the others
    mixed = [sv.wait(t, 300) for t in tickets]
    sv.close()
    m = mixed[2]
    log("alone E_F", alone["e_fermi"], "mixed E_F", m["e_fermi"], "window", m["density_from_window"])
    assert alone["status"] == 0 and m["status"] == 0
    assert np.array_equal(alone["dos"], m["dos"])
    assert alone["e_fermi"] == m["e_fermi"] and alone["e_band"] == m["e_band"]
    assert alone["entropy"] == m["entropy"]
    assert np.array_equal(alone["density"], m["density"])
    # requests overlapped: some started before an earlier one finished
    overlaps = sum(1 for a, b in zip(mixed, mixed[1:]) if b["t_start"] < a["t_done"])
    log("overlapping starts", overlaps)
    assert overlaps >= 1


def test_server_equals_single_call(mala):
    import torch
    net = mala_synth.paper_net()
    r = small_requests(1, seed=33)[0]
    sv = mala.Server(mala_synth.net_to_blob(net), mala.PREC_FP32, hbm_budget=16 << 30, max_inflight=2)
    out = sv.wait(run(sv, r), 120)
    sv.close()
    ctx = mala.Context(0)
    w = ctx.weights(mala_synth.net_to_blob(net), mala.PREC_FP32)
    dos, dens, res = ctx.mala_predict(w, r.positions, r.L, r.N, r.rcut, r.twojmax, EG, r.T, r.n_electrons)
    rr = mala.read_result(res)
    assert np.array_equal(out["dos"], dos.cpu().numpy())
    assert out["e_fermi"] == rr["e_fermi"]
    assert np.array_equal(out["density"], dens.cpu().numpy())
    ctx.close()


def test_tiny_budget_serialises(mala):
    net = mala_synth.paper_net()
    reqs = small_requests(3, seed=44, pts_per_atom=300.0)
    sv = mala.Server(mala_synth.net_to_blob(net), mala.PREC_FP32, hbm_budget=4 << 30, max_inflight=3)
    outs = [sv.wait(t, 300) for t in [run(sv, r) for r in reqs]]
    st = sv.stats()
    sv.close()
    log("peak bytes", st["peak_bytes"], "budget", st["budget"])
    assert all(o["status"] == 0 for o in outs)
    assert st["peak_bytes"] <= st["budget"]


def test_reserved_slots_allocate_nothing_and_match(mala):
    """After mala_server_reserve for the mix and one warm-up round, a stream
    of requests makes no device or pinned allocation, the capacity flags come
    back clean, and results still equal the single-request ones."""
    net = mala_synth.paper_net()
    reqs = small_requests(8, seed=55)
    sv = mala.Server(mala_synth.net_to_blob(net), mala.PREC_FP32, hbm_budget=32 << 30, max_inflight=3)
    sv.reserve([(r.n_atoms, r.L, r.N, r.rcut, r.twojmax, EG, r.T) for r in reqs])
    warm = [sv.wait(t, 300) for t in [run(sv, r) for r in reqs[:3]]]
    st0 = sv.stats()
    outs = [sv.wait(t, 300) for t in [run(sv, r) for r in reqs]]
    st1 = sv.stats()
    sv.close()
    log("reserved GB per slot %.2f, allocations %d -> %d" % (st0["reserved_bytes_per_slot"] / 2 ** 30,
                                                               st0["allocations"], st1["allocations"]))
    assert st1["allocations"] == st0["allocations"]
    assert all(o["status"] == 0 for o in warm + outs)
    for a, b in zip(warm, outs[:3]):
        assert np.array_equal(a["dos"], b["dos"]) and a["e_fermi"] == b["e_fermi"]
        assert np.array_equal(a["density"], b["density"])
