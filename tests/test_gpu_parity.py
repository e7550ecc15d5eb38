"""GPU parity: the HIP path through the C ABI against the FP64 oracle.

Tolerances (plain FP32 form; derived from FP32 rounding of sums of a few
tens of neighbour terms and of 66k-term contractions):
  B        per point max|dB| / max|B_ref|            <= 1e-5
  LDOS     per point max|dd| / max|d_ref|            <= 1e-5 (network alone)
  DOS      max|dD| / max|D_ref|                      <= 1e-6
  E_F                                                <= 1e-4 eV
  E_band   per atom                                  <= 0.01 meV
  density  max|dn| / max|n_ref|                      <= 1e-5
  sum(n) dV vs N(E_F)                                <= 1e-9 relative
FP64-only stages fed identical inputs are held to 1e-10 or tighter.
"""
import json
import os
import sys

import numpy as np
import pytest

import mala_synth
import oracle

pytestmark = pytest.mark.gpu
GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
EG = mala_synth.EGRID


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch():
    import torch as t
    if not t.cuda.is_available():
        pytest.skip("no GPU")
    return t


@pytest.fixture(scope="module")
def mala(torch):
    import paper_2411_19617_amd as m
    m.lib()
    return m


@pytest.fixture(scope="module")
def ctx(mala):
    c = mala.Context(0)
    yield c
    c.close()


def rel_rows(a, b):
    """max over rows of max|a-b| / max|b| per row."""
    num = np.max(np.abs(a - b), axis=1)
    den = np.maximum(np.max(np.abs(b), axis=1), 1e-300)
    return float(np.max(num / den))


def golden(case, snap, net):
    """Stored oracle values of a whole grid, checked to belong to these inputs."""
    from tests.golden.make_golden import fingerprint
    path = os.path.join(GOLD, "full_%s.json" % case)
    g = json.load(open(path))
    assert g["fingerprint"] == fingerprint(snap, net), "golden %s does not match the current inputs" % case
    return g


# ------------------------------------------------------------------ descriptors

@pytest.fixture(scope="module")
def small_ref():
    s = mala_synth.small()
    return s, oracle.descriptors(s)


def test_descriptors_small_all_points(ctx, small_ref, torch):
    s, Bref = small_ref
    log("descriptors small", s.name)
    B = ctx.mala_descriptors(s.positions, s.L, s.N, s.rcut, s.twojmax)
    torch.cuda.synchronize()
    ctx.check_device_errors()
    err = rel_rows(B.cpu().double().numpy(), Bref)
    log("B rel err", err)
    assert err <= 1e-5


@pytest.mark.parametrize("rng_", [(37, 1000), (0, 1), (7999, 8000), (64, 128), (100, 100)])
def test_descriptors_ragged_ranges(ctx, small_ref, rng_, torch):
    s, Bref = small_ref
    b, e = rng_
    log("descriptors range", b, e)
    B = ctx.mala_descriptors(s.positions, s.L, s.N, s.rcut, s.twojmax, b, e)
    torch.cuda.synchronize()
    assert B.shape[0] == e - b
    if e > b:
        assert rel_rows(B.cpu().double().numpy(), Bref[b:e]) <= 1e-5


def test_descriptors_empty_cell_and_atom_on_point(ctx, torch):
    # no atoms: B = J+1 exactly; one atom on a grid point: that point gets 8(J+1)
    L, N = np.array([9.0, 9.0, 9.0]), np.array([4, 5, 6])
    trip = oracle.triples(8)
    B = ctx.mala_descriptors(np.zeros((0, 3)), L, N, 4.67, 8).cpu().double().numpy()
    assert np.max(np.abs(B - (trip[:, 2] + 1))) <= 1e-6 * 9
    pos = np.array([[0.0, 0.0, 0.0]])
    snap = mala_synth.Snapshot("one", pos, L, N, 4.67, 8, 298.0, 3.0)
    Bg = ctx.mala_descriptors(pos, L, N, 4.67, 8).cpu().double().numpy()
    Bo = oracle.descriptors(snap)
    assert np.max(np.abs(Bg[0] - 8 * (trip[:, 2] + 1))) <= 1e-5 * 72
    assert rel_rows(Bg, Bo) <= 1e-5


def test_descriptors_small_cell_many_images(ctx, torch):
    # cell edges below rcut: every atom appears through several images
    rng = mala_synth.SplitMix64(11)
    L = np.array([4.2, 5.1, 3.9])
    pos = rng.uniform(6).reshape(2, 3) * L
    snap = mala_synth.Snapshot("tiny", pos, L, np.array([3, 4, 5]), 4.67, 6, 298.0, 6.0)
    Bg = ctx.mala_descriptors(pos, snap.L, snap.N, 4.67, 6).cpu().double().numpy()
    ctx.check_device_errors()
    assert rel_rows(Bg, oracle.descriptors(snap)) <= 1e-5


@pytest.mark.parametrize("case", ["paper_solid", "paper_liquid"])
def test_descriptors_paper_scale_sampled(ctx, case, torch):
    s = getattr(mala_synth, case)()
    log("descriptors", s.name)
    B = ctx.mala_descriptors(s.positions, s.L, s.N, s.rcut, s.twojmax)
    torch.cuda.synchronize()
    ctx.check_device_errors()
    pts = mala_synth.sample_points(s.n_points, 192, 77)
    Bref = oracle.descriptors(s, pts)
    Bg = B[torch.as_tensor(pts, device=B.device)].cpu().double().numpy()
    err = rel_rows(Bg, Bref)
    log("B rel err", err)
    assert err <= 1e-5


# ------------------------------------------------------------------ network

@pytest.mark.parametrize("which", ["small", "paper"])
def test_ldos_infer_matches_oracle_network(ctx, mala, which, torch):
    net = mala_synth.small_net() if which == "small" else mala_synth.paper_net()
    snap = mala_synth.small()
    snap.twojmax = 8 if which == "small" else 10
    pts = mala_synth.sample_points(snap.n_points, 300, 5)
    Bref = oracle.descriptors(snap, pts).astype(np.float32)     # identical inputs to both sides
    w = ctx.weights(mala_synth.net_to_blob(net), mala.PREC_FP32)
    ld = ctx.mala_ldos_infer(w, torch.as_tensor(Bref, device="cuda"), net["widths"][-1])
    ref = oracle.mlp(Bref.astype(np.float64), net)
    err = rel_rows(ld.cpu().double().numpy(), ref)
    log("LDOS rel err", which, err)
    assert err <= 1e-5


def test_ldos_infer_bf16_error_reported(ctx, mala, torch):
    net = mala_synth.paper_net()
    snap = mala_synth.small()
    snap.twojmax = 10
    pts = mala_synth.sample_points(snap.n_points, 300, 6)
    Bref = oracle.descriptors(snap, pts).astype(np.float32)
    w = ctx.weights(mala_synth.net_to_blob(net), mala.PREC_BF16)
    ld = ctx.mala_ldos_infer(w, torch.as_tensor(Bref, device="cuda"), 250)
    err = rel_rows(ld.cpu().double().numpy(), oracle.mlp(Bref.astype(np.float64), net))
    log("BF16 LDOS rel err", err)
    assert err <= 3e-2


# ------------------------------------------------------------------ integration

def test_integrate_matches_oracle_on_identical_ldos(ctx, torch):
    rng = np.random.default_rng(3)
    e = EG[0] + EG[1] * np.arange(EG[2])
    n = 5000
    ld = (0.007 * np.sqrt(e + 5.5) * rng.uniform(0.8, 1.2, size=(n, EG[2]))).astype(np.float32)
    dV = 0.05
    D = oracle.dos(ld.astype(np.float64), dV)
    w_half = oracle.fermi_weights(EG, 6.0, 298.0)[0]
    ne = float(w_half @ D)
    for T in (298.0, 933.0):
        ref = oracle.fermi(D, EG, T, ne)
        dens_ref = oracle.density(ld.astype(np.float64), ref["weights"])
        dos, dens, res = ctx.mala_integrate(torch.as_tensor(ld, device="cuda"), dV, EG, T, ne)
        import paper_2411_19617_amd as m
        r = m.read_result(res)
        log("integrate", T, r, ref["e_fermi"], ref["e_band"])
        assert r["status"] == 0
        assert np.max(np.abs(dos.cpu().numpy() - D)) <= 1e-12 * np.max(D)
        assert abs(r["e_fermi"] - ref["e_fermi"]) <= 1e-9
        assert abs(r["e_band"] - ref["e_band"]) <= 1e-9 * abs(ref["e_band"])
        assert abs(r["n_found"] - ne) <= 1e-9 * ne
        assert np.max(np.abs(dens.cpu().numpy() - dens_ref)) <= 1e-12 * np.max(dens_ref)
        # entropy (Eq. electronicentropyDOS) of the same DOS at the oracle's E_F
        s_ref, mts_ref = oracle.entropy(D, EG, ref["e_fermi"], T)
        assert abs(r["entropy"] - s_ref) <= 1e-9 * s_ref
        assert abs(r["e_entropy"] - mts_ref) <= 1e-9 * abs(mts_ref)


def test_integrate_no_root(ctx, mala, torch):
    ld = torch.full((100, 250), 0.01, dtype=torch.float32, device="cuda")
    dos, dens, res = ctx.mala_integrate(ld, 0.1, EG, 298.0, 1e9)
    r = mala.read_result(res)
    assert r["status"] == mala.MALA_E_NO_ROOT and np.isnan(r["e_fermi"])
    assert np.isnan(r["entropy"]) and np.isnan(r["e_entropy"])


def test_invalid_arguments(ctx, mala, torch):
    with pytest.raises(mala.MalaError) as e:
        ctx.mala_descriptors(np.zeros((1, 3)), [8.1, 8.1, 8.1], [4, 4, 4], 4.67, 7)
    assert e.value.status == mala.MALA_E_UNSUPPORTED
    with pytest.raises(mala.MalaError) as e:
        ctx.mala_descriptors(np.array([[np.nan, 0, 0]]), [8.1, 8.1, 8.1], [4, 4, 4], 4.67, 8)
    assert e.value.status == mala.MALA_E_INVALID_ARG
    with pytest.raises(mala.MalaError) as e:
        ctx.mala_descriptors(np.zeros((1, 3)), [8.1, -1, 8.1], [4, 4, 4], 4.67, 8)
    assert e.value.status == mala.MALA_E_INVALID_ARG
    with pytest.raises(mala.MalaError) as e:
        ctx.mala_descriptors(np.zeros((1, 3)), [8.1, 8.1, 8.1], [4, 4, 4], 4.67, 8, 10, 5)
    assert e.value.status == mala.MALA_E_INVALID_ARG
    ld = torch.zeros((10, 250), dtype=torch.float32, device="cuda")
    with pytest.raises(mala.MalaError):
        ctx.mala_integrate(ld, 0.1, EG, -1.0, 3.0)
    with pytest.raises(mala.MalaError):
        ctx.mala_integrate(ld, 0.1, (-5.0, 0.1, 300), 298.0, 3.0)
    with pytest.raises(mala.MalaError):
        ctx.weights(b"not a blob at all", 0)


# ------------------------------------------------------------------ fused path

def _check_full(ctx, mala, torch, snap, net, gold, prec, tol_eb_mev, tol_dos, tol_ef):
    w = ctx.weights(mala_synth.net_to_blob(net), prec)
    dos, dens, res = ctx.mala_predict(w, snap.positions, snap.L, snap.N, snap.rcut, snap.twojmax, EG,
                                      snap.T, snap.n_electrons)
    r = mala.read_result(res)
    ctx.check_device_errors()
    D = dos.cpu().numpy()
    Dref = np.array(gold["dos"])
    err_dos = np.max(np.abs(D - Dref)) / np.max(np.abs(Dref))
    err_ef = abs(r["e_fermi"] - gold["e_fermi"])
    err_eb = abs(r["e_band"] - gold["e_band"]) / snap.n_atoms * 1000.0
    err_ts = abs(r["e_entropy"] - gold["minus_ts"]) / snap.n_atoms * 1000.0
    n = dens.cpu().numpy()
    log(snap.name, "prec", prec, "dos", err_dos, "E_F", err_ef, "E_b meV/atom", err_eb, "-TS meV/atom", err_ts,
        "iters", r["iterations"])
    assert r["status"] == 0
    assert err_dos <= tol_dos and err_ef <= tol_ef and err_eb <= tol_eb_mev and err_ts <= tol_eb_mev
    assert abs(r["e_entropy"] + 8.617333262e-5 * snap.T * r["entropy"]) <= 1e-12 * abs(r["e_entropy"])
    assert abs(n.sum() * snap.dV - r["n_found"]) <= 1e-9 * r["n_found"]
    assert abs(r["n_found"] - snap.n_electrons) <= 1e-10 * snap.n_electrons
    return n, r


def test_predict_small_full_grid(ctx, mala, torch):
    snap, net = mala_synth.small(), mala_synth.small_net()
    gold = golden("small", snap, net)
    n, r = _check_full(ctx, mala, torch, snap, net, gold, mala.PREC_FP32, 0.01, 1e-6, 1e-4)
    # density at every point against the oracle's density at its own E_F
    ref = oracle.predict(snap, net, EG)
    assert rel_rows(n[None, :], ref["density"][None, :]) <= 1e-5


@pytest.mark.parametrize("case", ["paper_solid", "paper_liquid"])
def test_predict_paper_scale(ctx, mala, case, torch):
    snap, net = getattr(mala_synth, case)(), mala_synth.paper_net()
    gold = golden(case, snap, net)
    n, r = _check_full(ctx, mala, torch, snap, net, gold, mala.PREC_FP32, 0.01, 1e-6, 1e-4)
    assert abs(n.sum() * snap.dV - gold["density_sum_dV"]) <= 1e-6 * gold["density_sum_dV"]
    # density at sampled points: oracle LDOS there, oracle weights at the oracle E_F
    pts = mala_synth.sample_points(snap.n_points, 64, 9)
    ld = oracle.mlp(oracle.descriptors(snap, pts), net)
    w, _ = oracle.fermi_weights(EG, gold["e_fermi"], snap.T)
    nref = oracle.density(ld, w)
    assert np.max(np.abs(n[pts] - nref)) <= 1e-5 * np.max(np.abs(nref))


@pytest.mark.parametrize("case", ["paper_solid", "paper_liquid"])
def test_predict_precision_form(ctx, mala, case, torch):
    snap, net = getattr(mala_synth, case)(), mala_synth.paper_net()
    gold = golden(case, snap, net)
    _check_full(ctx, mala, torch, snap, net, gold, mala.PREC_BF16, 1.0, 5e-2, 5e-2)


@pytest.mark.parametrize("case", ["small", "paper_liquid"])
def test_density_window_equals_recompute(ctx, mala, case, torch):
    snap = getattr(mala_synth, case)()
    net = mala_synth.small_net() if case == "small" else mala_synth.paper_net()
    w = ctx.weights(mala_synth.net_to_blob(net), mala.PREC_FP32)
    out = {}
    for mode in (mala.DENSITY_WINDOW, mala.DENSITY_RECOMPUTE):
        ctx.set_density_mode(mode)
        dos, dens, res = ctx.mala_predict(w, snap.positions, snap.L, snap.N, snap.rcut, snap.twojmax, EG,
                                          snap.T, snap.n_electrons)
        out[mode] = (dos.cpu().numpy(), dens.cpu().numpy(), mala.read_result(res))
    ctx.set_density_mode(mala.DENSITY_WINDOW)
    a, b = out[mala.DENSITY_WINDOW], out[mala.DENSITY_RECOMPUTE]
    log(case, "window path", a[2]["density_from_window"], "recompute path", b[2]["density_from_window"])
    assert a[2]["density_from_window"] == 1 and b[2]["density_from_window"] == 0
    assert np.array_equal(a[0], b[0]) and a[2]["e_fermi"] == b[2]["e_fermi"]
    assert np.max(np.abs(a[1] - b[1])) <= 1e-7 * np.max(np.abs(b[1]))


def test_predict_deterministic_and_matches_unfused(ctx, mala, torch):
    snap, net = mala_synth.small(), mala_synth.small_net()
    w = ctx.weights(mala_synth.net_to_blob(net), mala.PREC_FP32)
    a = ctx.mala_predict(w, snap.positions, snap.L, snap.N, snap.rcut, snap.twojmax, EG, snap.T,
                         snap.n_electrons)
    b = ctx.mala_predict(w, snap.positions, snap.L, snap.N, snap.rcut, snap.twojmax, EG, snap.T,
                         snap.n_electrons)
    assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1]) and torch.equal(a[2], b[2])
    B = ctx.mala_descriptors(snap.positions, snap.L, snap.N, snap.rcut, snap.twojmax)
    ld = ctx.mala_ldos_infer(w, B, 250)
    dos, dens, res = ctx.mala_integrate(ld, snap.dV, EG, snap.T, snap.n_electrons)
    ra, rb = mala.read_result(a[2]), mala.read_result(res)
    assert np.max(np.abs(dos.cpu().numpy() - a[0].cpu().numpy())) <= 1e-7 * a[0].abs().max().item()
    assert abs(ra["e_fermi"] - rb["e_fermi"]) <= 1e-6
    assert np.max(np.abs(dens.cpu().numpy() - a[1].cpu().numpy())) <= 1e-6 * a[1].abs().max().item()
