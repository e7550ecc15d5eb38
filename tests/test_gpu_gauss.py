"""Gaussian descriptors (the Gaussian representation of the ionic positions
behind Eq. structurefactor_gaussian) through the C ABI against the oracle."""
import sys

import numpy as np
import pytest

import mala_synth
import oracle

pytestmark = pytest.mark.gpu


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
    yield mala, ctx
    ctx.close()


def rel(a, b):
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


@pytest.mark.parametrize("fac", [0.7, 1.0, 1.5])
def test_small_all_points(env, fac):
    mala, ctx = env
    s = mala_synth.small()
    sigma = fac * float(np.max(s.L / s.N))
    G = ctx.mala_gaussian_descriptors(s.positions, s.L, s.N, sigma, 8 * sigma).cpu().double().numpy()
    ctx.check_device_errors()
    ref = oracle.gaussian(s, sigma, 8 * sigma)
    err = rel(G, ref)
    log("gauss small sigma/h", fac, "max rel", err, "sum G dV / N - 1", G.sum() * s.dV / s.n_atoms - 1)
    assert err <= 1e-5
    assert abs(G.sum() - ref.sum()) <= 1e-5 * ref.sum()


@pytest.mark.parametrize("case", ["paper_solid", "paper_liquid"])
def test_paper_scale_sampled(env, case):
    mala, ctx = env
    s = getattr(mala_synth, case)()
    sigma = float(np.max(s.L / s.N))
    G = ctx.mala_gaussian_descriptors(s.positions, s.L, s.N, sigma, 8 * sigma).cpu().double().numpy()
    ctx.check_device_errors()
    pts = mala_synth.sample_points(s.n_points, 3000, 21)
    ref = oracle.gaussian(s, sigma, 8 * sigma, pts)
    err = rel(G[pts], ref)
    log(case, "gauss sampled max rel", err, "sum G dV / N - 1", G.sum() * s.dV / s.n_atoms - 1)
    assert err <= 1e-5
    assert abs(G.sum() * s.dV / s.n_atoms - 1.0) <= 1e-5


def test_ragged_ranges(env):
    # tiles start at pt_begin, so a range sees other tile origins and candidate
    # orders than the full grid: equal to FP32 rounding, and to the oracle
    mala, ctx = env
    s = mala_synth.small()
    sigma = 0.5
    full = ctx.mala_gaussian_descriptors(s.positions, s.L, s.N, sigma, 4.0).cpu().double().numpy()
    ref = oracle.gaussian(s, sigma, 4.0)
    for b, e in [(0, 1), (37, 1000), (7999, 8000), (64, 128), (100, 100)]:
        part = ctx.mala_gaussian_descriptors(s.positions, s.L, s.N, sigma, 4.0, b, e).cpu().double().numpy()
        assert part.shape[0] == e - b
        if e > b:
            assert np.max(np.abs(part - full[b:e])) <= 1e-6 * np.max(full)
            assert np.max(np.abs(part - ref[b:e])) <= 1e-5 * np.max(ref)


def test_empty_cell_and_many_images(env):
    mala, ctx = env
    L, N = np.array([9.0, 9.0, 9.0]), np.array([4, 5, 6])
    G = ctx.mala_gaussian_descriptors(np.zeros((0, 3)), L, N, 0.5, 4.0).cpu().numpy()
    assert np.all(G == 0.0)
    # cell edges below the cutoff: every atom is seen through many images
    rng = mala_synth.SplitMix64(11)
    L = np.array([4.2, 5.1, 3.9])
    pos = rng.uniform(6).reshape(2, 3) * L
    snap = mala_synth.Snapshot("tiny", pos, L, np.array([6, 7, 5]), 4.67, 8, 298.0, 6.0)
    G = ctx.mala_gaussian_descriptors(pos, L, snap.N, 1.2, 9.0).cpu().double().numpy()
    ctx.check_device_errors()
    assert rel(G, oracle.gaussian(snap, 1.2, 9.0)) <= 1e-5


def test_invalid_arguments(env):
    mala, ctx = env
    s = mala_synth.small()
    for sigma, cut in [(0.0, 4.0), (-1.0, 4.0), (0.5, 0.0), (float("nan"), 4.0)]:
        with pytest.raises(mala.MalaError) as e:
            ctx.mala_gaussian_descriptors(s.positions, s.L, s.N, sigma, cut)
        assert e.value.status == mala.MALA_E_INVALID_ARG
    with pytest.raises(mala.MalaError):
        ctx.mala_gaussian_descriptors(s.positions, s.L, s.N, 0.5, 4.0, 10, 5)
