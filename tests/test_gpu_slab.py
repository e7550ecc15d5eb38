"""The 47,066,880-point fcc(111) slab (16,384 atoms, stacking fault, vacuum):
sampled outputs against the oracle, and properties that hold at any size for
the whole-grid quantities (the oracle would need ~27 core-hours for them)."""
import sys

import numpy as np
import pytest

import mala_synth
import oracle

pytestmark = pytest.mark.gpu
EG = mala_synth.EGRID


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def fermi(e, mu, kT):
    return 0.5 * (1.0 - np.tanh(0.5 * (e - mu) / kT))


def quad_weights(mu, T, n_gl=48):
    """Test-side Gauss-Legendre weights of f against the hat functions."""
    kT = 8.617333262e-5 * T
    e = EG[0] + EG[1] * np.arange(EG[2])
    x, wq = np.polynomial.legendre.leggauss(n_gl)
    w = np.zeros(EG[2])
    for i in range(EG[2] - 1):
        cuts = [e[i], e[i + 1]] if not (e[i] < mu < e[i + 1]) else [e[i], mu, e[i + 1]]
        for lo, hi in zip(cuts[:-1], cuts[1:]):
            t = 0.5 * (hi - lo) * x + 0.5 * (hi + lo)
            f = fermi(t, mu, kT) * 0.5 * (hi - lo) * wq
            w[i] += np.sum(f * (e[i + 1] - t) / EG[1])
            w[i + 1] += np.sum(f * (t - e[i]) / EG[1])
    return w


@pytest.fixture(scope="module")
def setup():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2411_19617_amd as mala
    mala.lib()
    ctx = mala.Context(0)
    snap, net = mala_synth.slab(), mala_synth.paper_net()
    yield mala, ctx, snap, net
    ctx.close()


def test_slab_descriptors_sampled(setup):
    mala, ctx, snap, net = setup
    pts = mala_synth.sample_points(snap.n_points, 48, 17)
    # include vacuum points and the fault plane region explicitly
    Nz = snap.N[2]
    extra = np.array([0, Nz // 2, (snap.N[1] // 2 * Nz) + Nz // 2], dtype=np.int64)
    pts = np.unique(np.concatenate([pts, extra]))
    Bref = oracle.descriptors(snap, pts)
    errs = []
    for p, ref in zip(pts, Bref):
        Bg = ctx.mala_descriptors(snap.positions, snap.L, snap.N, snap.rcut, snap.twojmax, int(p), int(p) + 1)
        g = Bg.cpu().double().numpy()[0]
        errs.append(np.max(np.abs(g - ref)) / np.max(np.abs(ref)))
    ctx.check_device_errors()
    log("slab B max rel err", max(errs))
    assert max(errs) <= 1e-5


@pytest.mark.parametrize("prec", [0, 1])
def test_slab_predict_properties(setup, prec):
    import torch
    mala, ctx, snap, net = setup
    w = ctx.weights(mala_synth.net_to_blob(net), prec)
    dos, dens, res = ctx.mala_predict(w, snap.positions, snap.L, snap.N, snap.rcut, snap.twojmax, EG, snap.T,
                                      snap.n_electrons)
    r = mala.read_result(res)
    ctx.check_device_errors()
    D = dos.cpu().numpy()
    log("slab prec", prec, r)
    assert r["status"] == 0 and EG[0] < r["e_fermi"] < EG[0] + EG[1] * (EG[2] - 1)
    # root property: N(E_F) from test-side quadrature of the GPU DOS
    wq = quad_weights(r["e_fermi"], snap.T)
    assert abs(wq @ D - snap.n_electrons) <= 1e-7 * snap.n_electrons
    # density integrates to the electron count
    tot = float(dens.sum().item()) * snap.dV
    assert abs(tot - snap.n_electrons) <= 1e-6 * snap.n_electrons
    # density on a sub-range equals the direct contraction of its LDOS
    b, e = 23_000_000, 23_000_000 + 4096
    B = ctx.mala_descriptors(snap.positions, snap.L, snap.N, snap.rcut, snap.twojmax, b, e)
    ld = ctx.mala_ldos_infer(w, B, 250).cpu().double().numpy()
    n_direct = ld @ wq
    n_gpu = dens[b:e].cpu().numpy()
    err = np.max(np.abs(n_gpu - n_direct)) / np.max(np.abs(n_direct))
    log("slab density vs direct contraction", err, "window", r["density_from_window"])
    assert err <= 1e-6


def test_slab_ldos_sampled_against_oracle(setup):
    import torch
    mala, ctx, snap, net = setup
    pts = mala_synth.sample_points(snap.n_points, 24, 23)
    Bref = oracle.descriptors(snap, pts)
    ld_ref = oracle.mlp(Bref, net)
    w = ctx.weights(mala_synth.net_to_blob(net), 0)
    rows = []
    for p in pts:
        Bg = ctx.mala_descriptors(snap.positions, snap.L, snap.N, snap.rcut, snap.twojmax, int(p), int(p) + 1)
        rows.append(ctx.mala_ldos_infer(w, Bg, 250).cpu().double().numpy()[0])
    g = np.array(rows)
    err = np.max(np.max(np.abs(g - ld_ref), axis=1) / np.max(np.abs(ld_ref), axis=1))
    log("slab LDOS rel err", err)
    assert err <= 2e-5
