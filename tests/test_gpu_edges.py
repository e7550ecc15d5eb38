"""GPU edge cases through the C ABI: every supported twojmax, a network shape
other than the two workloads' (generic padded path), the no-root and
mismatch paths of the fused call, and the neighbour-capacity flag."""
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


@pytest.fixture(scope="module")
def env():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2411_19617_amd as mala
    mala.lib()
    ctx = mala.Context(0)
    yield mala, ctx, torch
    ctx.close()


def rel_rows(a, b):
    return float(np.max(np.max(np.abs(a - b), axis=1) / np.maximum(np.max(np.abs(b), axis=1), 1e-300)))


@pytest.mark.parametrize("tj", [2, 4, 6, 8, 10])
def test_descriptors_every_twojmax(env, tj):
    mala, ctx, torch = env
    s = mala_synth.paper_liquid(grid=24)
    s.twojmax = tj
    pts = mala_synth.sample_points(s.n_points, 96, 100 + tj)
    B = ctx.mala_descriptors(s.positions, s.L, s.N, s.rcut, tj).cpu().double().numpy()
    ctx.check_device_errors()
    assert B.shape[1] == mala.n_descriptors(tj)
    err = rel_rows(B[pts], oracle.descriptors(s, pts))
    log("twojmax", tj, "B rel err", err)
    assert err <= 1e-5


@pytest.mark.parametrize("prec,tol", [(0, 1e-5), (1, 3e-2)])
def test_generic_network_shape(env, prec, tol):
    mala, ctx, torch = env
    net = mala_synth.make_net([55, 72, 96, 150], 7, 8, egrid=(-5.0, 0.1, 150))
    s = mala_synth.small()
    pts = mala_synth.sample_points(s.n_points, 200, 8)
    Bref = oracle.descriptors(s, pts).astype(np.float32)
    w = ctx.weights(mala_synth.net_to_blob(net), prec)
    ld = ctx.mala_ldos_infer(w, torch.as_tensor(Bref, device="cuda"), 150).cpu().double().numpy()
    err = rel_rows(ld, oracle.mlp(Bref.astype(np.float64), net))
    log("generic shape prec", prec, "LDOS rel err", err)
    assert err <= tol


@pytest.mark.parametrize("prec,tol", [(0, 1e-5), (1, 3e-2)])
def test_network_at_maximum_widths(env, prec, tol):
    """The widest network the build takes (128 inputs, hidden layers of 512,
    256 outputs): the FP32 network falls back to 32-point tiles there (its
    activations would not fit beside the epilogue at 64) and the BF16 one runs
    at its largest LDS footprint."""
    mala, ctx, torch = env
    eg = (-5.0, 0.1, 256)
    net = mala_synth.make_net([128, 512, 512, 256], 11, 8, egrid=eg, with_input_scaler=False)
    B, _ = mala_synth.network_inputs(net, 300, 12)
    w = ctx.weights(mala_synth.net_to_blob(net), prec)
    ld = ctx.mala_ldos_infer(w, torch.as_tensor(B, device="cuda"), 256).cpu().double().numpy()
    err = rel_rows(ld, oracle.mlp(B.astype(np.float64), net))
    log("maximum widths prec", prec, "LDOS rel err", err)
    assert err <= tol


@pytest.mark.parametrize("prec", [0, 1])
def test_predict_at_maximum_widths(env, prec):
    """The fused path (DOS, energy window, density) with hidden layers of 512
    and 256 energies, on the whole 8,000-point grid against the oracle."""
    mala, ctx, torch = env
    s = mala_synth.small()
    eg = (-5.0, 0.1, 256)
    net = mala_synth.make_net([55, 512, 512, 256], 13, 8, egrid=eg)
    ref = oracle.predict(s, net, eg)
    w = ctx.weights(mala_synth.net_to_blob(net), prec)
    dos, dens, res = ctx.mala_predict(w, s.positions, s.L, s.N, s.rcut, s.twojmax, eg, s.T, s.n_electrons)
    r = mala.read_result(res)
    assert r["status"] == 0
    d_err = float(np.max(np.abs(dos.cpu().numpy() - ref["dos"])) / np.max(np.abs(ref["dos"])))
    ef_err = abs(r["e_fermi"] - ref["e_fermi"])
    n = dens.cpu().numpy()
    n_err = float(np.max(np.abs(n - ref["density"])) / np.max(np.abs(ref["density"])))
    log("maximum widths predict prec", prec, "DOS %.2e E_F %.2e eV density %.2e" % (d_err, ef_err, n_err))
    if prec == 0:
        assert d_err <= 1e-5 and ef_err <= 1e-5 and n_err <= 1e-5
    else:
        assert d_err <= 5e-2 and ef_err <= 5e-2 and n_err <= 5e-2


def test_density_from_a_wide_window(env):
    """At 1,500 K the stored energy window holds 112 energies, more than the
    density kernel stages per point in LDS: its direct path, against the
    oracle's density at every point of the 8,000-point grid."""
    mala, ctx, torch = env
    s, net = mala_synth.small(), mala_synth.small_net()
    s.T = 1500.0
    ref = oracle.predict(s, net, EG)
    w = ctx.weights(mala_synth.net_to_blob(net), 0)
    dos, dens, res = ctx.mala_predict(w, s.positions, s.L, s.N, s.rcut, s.twojmax, EG, s.T, s.n_electrons)
    r = mala.read_result(res)
    assert r["status"] == 0 and r["density_from_window"] == 1
    n = dens.cpu().numpy()
    err = float(np.max(np.abs(n - ref["density"])) / np.max(np.abs(ref["density"])))
    log("wide window (1500 K): E_F %.2e eV, density %.2e" % (abs(r["e_fermi"] - ref["e_fermi"]), err))
    assert abs(r["e_fermi"] - ref["e_fermi"]) <= 1e-4 and err <= 1e-5


def test_predict_no_root_leaves_density(env):
    mala, ctx, torch = env
    s, net = mala_synth.small(), mala_synth.small_net()
    w = ctx.weights(mala_synth.net_to_blob(net), 0)
    dens = torch.full((s.n_points,), -7.0, dtype=torch.float64, device="cuda")
    dos, d2, res = ctx.mala_predict(w, s.positions, s.L, s.N, s.rcut, s.twojmax, EG, s.T, 1e9, dens=dens)
    r = mala.read_result(res)
    assert r["status"] == mala.MALA_E_NO_ROOT and np.isnan(r["e_fermi"])
    assert bool((dens == -7.0).all().item())


def test_predict_argument_mismatch(env):
    mala, ctx, torch = env
    s, net = mala_synth.small(), mala_synth.small_net()
    w = ctx.weights(mala_synth.net_to_blob(net), 0)
    with pytest.raises(mala.MalaError) as e:       # 55-input net with twojmax 10 (91 components)
        ctx.mala_predict(w, s.positions, s.L, s.N, s.rcut, 10, EG, s.T, s.n_electrons)
    assert e.value.status == mala.MALA_E_INVALID_ARG
    with pytest.raises(mala.MalaError) as e:       # 250 outputs vs 100-point energy grid
        ctx.mala_predict(w, s.positions, s.L, s.N, s.rcut, 8, (-5.0, 0.1, 100), s.T, s.n_electrons)
    assert e.value.status == mala.MALA_E_INVALID_ARG


def test_empty_cell_predict(env):
    mala, ctx, torch = env
    net = mala_synth.small_net()
    w = ctx.weights(mala_synth.net_to_blob(net), 0)
    L, N = [10.0, 10.0, 10.0], [8, 8, 8]
    dos, dens, res = ctx.mala_predict(w, np.zeros((0, 3)), L, N, 4.67, 8, EG, 298.0, 30.0)
    r = mala.read_result(res)
    assert r["status"] == 0
    d = dens.cpu().numpy()
    assert np.max(d) - np.min(d) <= 1e-12 * np.max(d)          # every point sees the same (empty) B
    assert abs(d.sum() * 1000.0 / 512 - 30.0) <= 1e-9 * 30.0


def test_neighbour_capacity_is_reported(env):
    mala, ctx, torch = env
    # 200 atoms packed within 1 A of the origin: more than 128 neighbours there
    rng = mala_synth.SplitMix64(5)
    pos = (rng.uniform(600).reshape(200, 3) - 0.5) * 1.0 + 5.0
    B = ctx.mala_descriptors(pos, [10.0, 10.0, 10.0], [4, 4, 4], 4.67, 4)
    with pytest.raises(mala.MalaError) as e:
        ctx.check_device_errors()
    assert e.value.status == mala.MALA_E_CAPACITY
    ctx.check_device_errors()                                   # flag cleared


def test_predict_status_reports_capacity(env):
    """The fused call carries the capacity flag into its result record."""
    mala, ctx, torch = env
    rng = mala_synth.SplitMix64(5)
    pos = (rng.uniform(600).reshape(200, 3) - 0.5) * 1.0 + 5.0
    w = ctx.weights(mala_synth.net_to_blob(mala_synth.small_net()), mala.PREC_FP32)
    dos, dens, res = ctx.mala_predict(w, pos, [10.0, 10.0, 10.0], [4, 4, 4], 4.67, 8, EG, 298.0, 600.0)
    r = mala.read_result(res)
    log("capacity in predict:", r["status"])
    assert r["status"] == mala.MALA_E_CAPACITY
    with pytest.raises(mala.MalaError):
        ctx.check_device_errors()
    ctx.check_device_errors()


@pytest.mark.parametrize("grid", [(60, 103, 121), (120, 200, 37)])
def test_tiles_crossing_rows_and_planes_of_a_large_cell(env, grid):
    """The 16,384-atom slab on grids whose planes (and, for 121, rows) hold a
    number of points that is not a multiple of 64: tiles cross z-rows and
    x-planes, and each keeps two compact boxes (one box would span the
    cell's 79 x 92 A cross-section: several thousand candidates)."""
    mala, ctx, torch = env
    s = mala_synth.with_grid(mala_synth.slab(), grid)
    plane = grid[1] * grid[2]
    assert plane % 64 != 0
    # a range over several plane boundaries, from a point that is not 64-aligned
    b = 7 * plane - 1000
    e = b + 4 * plane + 333
    B = ctx.mala_descriptors(s.positions, s.L, s.N, s.rcut, s.twojmax, b, e).cpu().double().numpy()
    ctx.check_device_errors()                          # no candidate overflow
    seam = [k * plane + d for k in range(8, 11) for d in (-2, -1, 0, 1, 2, 40)]
    rows = [k * plane + j * grid[2] + d for k in (8, 9) for j in (0, grid[1] // 2, grid[1] - 1) for d in (-1, 0, 1)]
    pts = np.unique(np.concatenate([np.array(seam + rows, dtype=np.int64),
                                    b + mala_synth.sample_points(e - b, 120, 61)]))
    pts = pts[(pts >= b) & (pts < e)]
    err = rel_rows(B[pts - b], oracle.descriptors(s, pts))
    log("grid", grid, "crossing tiles: B rel err %.3e over %d points" % (err, len(pts)))
    assert err <= 1e-5
