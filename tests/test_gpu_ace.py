"""GPU parity of the grid ACE descriptors (Sec. 3.2.3) through the C ABI
against the FP64 oracle, ranks 1-3 and rank 4: whole small grid, a range of
the 256-atom cell, several basis sizes, sampled rows of the full
729,000-point grid, and the empty / unsupported cases."""
import sys

import numpy as np
import pytest

import mala_synth
import oracle

pytestmark = pytest.mark.gpu

TOL = 1e-5        # per point max |dB| / max |B| (FP32 accumulation and products)


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


def compare(env, s, rcut, nmax, lmax, pt_begin, pt_end):
    mala, ctx, torch = env
    log("ace", s.name, "nmax", nmax, "lmax", lmax, "points", pt_begin, pt_end)
    g = ctx.mala_ace_descriptors(s.positions, s.L, s.N, rcut, nmax, lmax, pt_begin, pt_end).cpu().double().numpy()
    ctx.check_device_errors()
    ref = oracle.ace(s, rcut, nmax, lmax, np.arange(pt_begin, pt_end, dtype=np.int64), nthreads=16)
    assert g.shape == ref.shape
    err = rel_rows(g, ref)
    log("  rel err %.3e" % err)
    assert np.all(np.isfinite(g))
    assert err <= TOL


def test_ace_small_cell_whole_grid(env):
    s = mala_synth.small()
    compare(env, s, s.rcut, 4, 4, 0, s.n_points)


def test_ace_paper_cell_range(env):
    s = mala_synth.paper_liquid()
    compare(env, s, s.rcut, 4, 4, 200000, 200000 + 2048 + 29)


@pytest.mark.parametrize("nmax,lmax", [(1, 0), (2, 3), (3, 2), (4, 1)])
def test_ace_parameters(env, nmax, lmax):
    s = mala_synth.small()
    compare(env, s, s.rcut, nmax, lmax, 1000, 1000 + 333)


def test_ace_full_grid_sampled(env):
    """729,000 points in one launch; 256 seeded rows against the oracle."""
    mala, ctx, torch = env
    s = mala_synth.paper_solid()
    g = ctx.mala_ace_descriptors(s.positions, s.L, s.N, s.rcut, 4, 4)
    ctx.check_device_errors()
    rows = mala_synth.sample_points(s.n_points, 256, 41)
    gs = g[torch.as_tensor(rows, device="cuda")].cpu().double().numpy()
    err = rel_rows(gs, oracle.ace(s, s.rcut, 4, 4, rows, nthreads=16))
    log("ace full grid sampled rel err %.3e" % err)
    assert err <= TOL
    assert bool(torch.isfinite(g).all())


def test_ace_empty_and_unsupported(env):
    mala, ctx, torch = env
    s = mala_synth.small()
    out = ctx.mala_ace_descriptors(s.positions, s.L, s.N, s.rcut, 4, 4, 7, 7)
    assert out.shape == (0, 602)
    with pytest.raises(mala.MalaError):
        mala.ace_count(5, 4)
    e = torch.empty((4, 602), dtype=torch.float32, device="cuda")
    with pytest.raises(mala.MalaError):
        ctx.mala_ace_descriptors(s.positions, s.L, s.N, s.rcut, 4, 5, 0, 4, out=e)


# ---------------------------------------------------------------- rank 4

def compare4(env, s, rcut, nmax4, lmax4, pt_begin, pt_end):
    mala, ctx, torch = env
    log("ace4", s.name, "nmax4", nmax4, "lmax4", lmax4, "points", pt_begin, pt_end)
    g = ctx.mala_ace4_descriptors(s.positions, s.L, s.N, rcut, nmax4, lmax4, pt_begin, pt_end).cpu().double().numpy()
    ctx.check_device_errors()
    ref = oracle.ace4(s, rcut, nmax4, lmax4, np.arange(pt_begin, pt_end, dtype=np.int64), nthreads=16)
    assert g.shape == ref.shape
    err = rel_rows(g, ref)
    log("  rel err %.3e" % err)
    assert np.all(np.isfinite(g))
    assert err <= TOL


def test_ace4_small_cell_whole_grid(env):
    s = mala_synth.small()
    compare4(env, s, s.rcut, 3, 3, 0, s.n_points)


def test_ace4_paper_cell_range(env):
    s = mala_synth.paper_liquid()
    compare4(env, s, s.rcut, 3, 3, 310000, 310000 + 1024 + 77)


@pytest.mark.parametrize("nmax4,lmax4", [(1, 0), (1, 2), (2, 2), (3, 2), (2, 3)])
def test_ace4_parameters(env, nmax4, lmax4):
    s = mala_synth.small()
    compare4(env, s, s.rcut, nmax4, lmax4, 2000, 2000 + 257)


def test_ace4_full_grid_sampled(env):
    """729,000 points in one launch; 192 seeded rows against the oracle."""
    mala, ctx, torch = env
    s = mala_synth.paper_solid()
    g = ctx.mala_ace4_descriptors(s.positions, s.L, s.N, s.rcut, 3, 3)
    ctx.check_device_errors()
    rows = mala_synth.sample_points(s.n_points, 192, 43)
    gs = g[torch.as_tensor(rows, device="cuda")].cpu().double().numpy()
    err = rel_rows(gs, oracle.ace4(s, s.rcut, 3, 3, rows, nthreads=16))
    log("ace4 full grid sampled rel err %.3e" % err)
    assert err <= TOL
    assert bool(torch.isfinite(g).all())


def test_ace4_empty_and_unsupported(env):
    mala, ctx, torch = env
    s = mala_synth.small()
    n = mala.ace4_count(3, 3)
    out = ctx.mala_ace4_descriptors(s.positions, s.L, s.N, s.rcut, 3, 3, 7, 7)
    assert out.shape == (0, n)
    with pytest.raises(mala.MalaError):
        mala.ace4_count(4, 3)
    e = torch.empty((4, n), dtype=torch.float32, device="cuda")
    with pytest.raises(mala.MalaError):
        ctx.mala_ace4_descriptors(s.positions, s.L, s.N, s.rcut, 3, 4, 0, 4, out=e)


@pytest.mark.parametrize("rank", [3, 4])
def test_ace_descriptor_major_layout_is_the_transpose(env, rank):
    """The descriptor-major output is the transpose of the point-major one
    over a range that spans two 2^19-point chunks, and for rank 4 nine of
    the 65,536-point chunks its point-major staging runs in, the last one
    ragged."""
    mala, ctx, torch = env
    s = mala_synth.paper_solid()
    b, e = 100_000, 100_000 + (1 << 19) + 777
    f = ctx.mala_ace_descriptors if rank == 3 else ctx.mala_ace4_descriptors
    pm = f(s.positions, s.L, s.N, s.rcut, pt_begin=b, pt_end=e)
    dm = f(s.positions, s.L, s.N, s.rcut, pt_begin=b, pt_end=e, descriptor_major=True)
    ctx.check_device_errors()
    assert dm.shape == (pm.shape[1], pm.shape[0])
    err = rel_rows(dm.t().cpu().double().numpy(), pm.cpu().double().numpy())
    log("rank", rank, "layouts differ by %.3e" % err)
    assert err <= 1e-6
