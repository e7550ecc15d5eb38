"""GPU parity of the descriptor vector-Jacobian product (the descriptor
factor of Eq. forcesmala) through the C ABI against the FP64 oracle's chain
rule, on whole small grids and point ranges of the 256-atom cell; at the
full 729,000-point grid the result is checked by properties that hold at
any size (linearity in the weights, additivity over point ranges)."""
import sys

import numpy as np
import pytest

import mala_synth
import oracle

pytestmark = pytest.mark.gpu

TOL = 2e-5        # max |d dL/dR| / max |dL/dR| (FP32 descriptors and recursion)


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


def weights(n, nb, seed):
    return np.random.default_rng(seed).standard_normal((n, nb)).astype(np.float32)


def gpu_vjp(env, s, gB, pt_begin, pt_end):
    mala, ctx, torch = env
    out = ctx.mala_descriptors_vjp(s.positions, s.L, s.N, s.rcut, s.twojmax, torch.as_tensor(gB, device="cuda"),
                                   pt_begin, pt_end)
    ctx.check_device_errors()
    return out.cpu().numpy()


def compare(env, s, pt_begin, pt_end, seed, tol=TOL):
    nb = oracle.lib().oracle_n_triples(s.twojmax)
    gB = weights(pt_end - pt_begin, nb, seed)
    log("adjoint", s.name, "twojmax", s.twojmax, "points", pt_begin, pt_end)
    g = gpu_vjp(env, s, gB, pt_begin, pt_end)
    ref = oracle.descriptors_vjp(s, gB.astype(np.float64), np.arange(pt_begin, pt_end, dtype=np.int64),
                                 nthreads=16)
    err = np.max(np.abs(g - ref)) / np.max(np.abs(ref))
    log("  dL/dR rel err %.3e (max |ref| %.3e)" % (err, np.max(np.abs(ref))))
    assert np.all(np.isfinite(g))
    assert err <= tol
    return g, ref


def test_adjoint_small_cell_whole_grid(env):
    compare(env, mala_synth.small(), 0, 8000, 1)


def test_adjoint_paper_cell_point_range(env):
    s = mala_synth.paper_solid()
    compare(env, s, 100000, 100000 + 4096 + 37, 2)


@pytest.mark.parametrize("tj", [2, 4, 6, 8, 10])
def test_adjoint_every_twojmax(env, tj):
    s = mala_synth.paper_liquid(grid=24)
    s.twojmax = tj
    compare(env, s, 3000, 3000 + 700, 10 + tj)


def test_adjoint_empty_range_writes_zeros(env):
    mala, ctx, torch = env
    s = mala_synth.small()
    out = torch.full((s.n_atoms, 3), 7.0, dtype=torch.float64, device="cuda")
    ctx.mala_descriptors_vjp(s.positions, s.L, s.N, s.rcut, s.twojmax,
                             torch.empty((0, 55), dtype=torch.float32, device="cuda"), 10, 10, out=out)
    assert float(out.abs().max()) == 0.0


def test_adjoint_full_grid_linear_and_additive(env):
    """729,000 points (the bench's launch configuration, two chunks of 2^19):
    F(g1) + F(g2) = F(g1 + g2) and F over [0, N) = F over [0, k) + F over [k, N).
    A split at a point that is not a multiple of 64 regroups the 64-point
    tiles, whose displacements are formed in FP32 relative to the tile
    origin, so both hold to FP32 rounding (as the oracle comparison)."""
    mala, ctx, torch = env
    s = mala_synth.paper_solid()
    n, nb = s.n_points, 91
    g1, g2 = weights(n, nb, 5), weights(n, nb, 6)
    f1, f2, f12 = (gpu_vjp(env, s, g, 0, n) for g in (g1, g2, g1 + g2))
    k = 300001
    fa, fb = gpu_vjp(env, s, g1[:k], 0, k), gpu_vjp(env, s, g1[k:], k, n)
    lin = np.max(np.abs(f1 + f2 - f12)) / np.max(np.abs(f12))
    add = np.max(np.abs(fa + fb - f1)) / np.max(np.abs(f1))
    log("full grid: linearity %.3e additivity %.3e" % (lin, add))
    assert lin <= 1e-5 and add <= 1e-5


def test_force_path_composition_matches_oracle(env):
    """The two factors chained as the force expression applies them: B from
    the GPU descriptors, g = (dd/dB)^T v from the network VJP, then
    dL/dR from the descriptor VJP; the oracle chains its own three steps.
    With slope 1 the network is affine (no kinks), so the comparison is
    element-wise for every point."""
    mala, ctx, torch = env
    s = mala_synth.small()
    net = mala_synth.make_net([55, 100, 100, 250], 104, 8, slope=1.0)
    n = s.n_points
    v = np.random.default_rng(77).standard_normal((n, 250)).astype(np.float32)
    w = ctx.weights(mala_synth.net_to_blob(net), mala.PREC_FP32)
    B = ctx.mala_descriptors(s.positions, s.L, s.N, s.rcut, s.twojmax)
    g = ctx.mala_ldos_vjp(w, B, torch.as_tensor(v, device="cuda"))
    F = ctx.mala_descriptors_vjp(s.positions, s.L, s.N, s.rcut, s.twojmax, g).cpu().numpy()
    ctx.check_device_errors()
    Bref = oracle.descriptors(s, nthreads=16)
    gref, _ = oracle.mlp_vjp(Bref, net, v.astype(np.float64), nthreads=16)
    Fref = oracle.descriptors_vjp(s, gref, nthreads=16)
    err = np.max(np.abs(F - Fref)) / np.max(np.abs(Fref))
    log("force path composition rel err %.3e (max |ref| %.3e)" % (err, np.max(np.abs(Fref))))
    assert err <= TOL


def test_adjoint_full_grid_launch_across_chunk_seam(env):
    """The full-grid launch (729,000 points, chunks of 2^19 from point 0) with
    weights that vanish outside a 4,096-point range straddling the chunk seam
    at 524,288: its dL/dR is the VJP of that range alone, which the oracle
    computes; the seam splits the range 2,048 / 2,048 between two launches."""
    mala, ctx, torch = env
    s = mala_synth.paper_solid()
    n, nb = s.n_points, 91
    b, e = (1 << 19) - 2048, (1 << 19) + 2048
    gB = np.zeros((n, nb), dtype=np.float32)
    gB[b:e] = weights(e - b, nb, 41)
    log("adjoint full grid, weights on", b, e)
    g = gpu_vjp(env, s, gB, 0, n)
    ref = oracle.descriptors_vjp(s, gB[b:e].astype(np.float64), np.arange(b, e, dtype=np.int64), nthreads=16)
    err = np.max(np.abs(g - ref)) / np.max(np.abs(ref))
    log("  dL/dR rel err %.3e (max |ref| %.3e)" % (err, np.max(np.abs(ref))))
    assert err <= TOL
