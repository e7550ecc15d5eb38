"""GPU parity of the network vector-Jacobian product (the network factor of
Eq. forcesmala) through the C ABI against the FP64 oracle's backpropagation.

The network is piecewise linear, so g jumps where a hidden unit crosses its
kink: a point whose oracle kink margin (min |z| / (|b| + sum |W x|)) is at
FP32 rounding level has two defensible answers and is left out of the
element-wise comparison (its count is printed and bounded)."""
import sys

import numpy as np
import pytest

import mala_synth
import oracle

pytestmark = pytest.mark.gpu

TOL = 2e-5          # per point max |dg| / max |g|, FP32 network
MARGIN = 1e-5       # oracle kink margin below which a point has two answers (FP32
                    # rounding of z is ~1e-6 of its term magnitude at 400 terms)


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


def run(env, net, n, seed):
    mala, ctx, torch = env
    B, v = mala_synth.network_inputs(net, n, seed)
    w = ctx.weights(mala_synth.net_to_blob(net), mala.PREC_FP32)
    log("vjp widths", net["widths"], "out_act", net["output_activation"], "n", n, "seed", seed)
    g = ctx.mala_ldos_vjp(w, torch.as_tensor(B, device="cuda"), torch.as_tensor(v, device="cuda"))
    ctx.synchronize()
    g = g.cpu().double().numpy()
    ref, margin = oracle.mlp_vjp(B.astype(np.float64), net, v.astype(np.float64), nthreads=16)
    keep = margin > MARGIN
    err = np.max(np.abs(g - ref), axis=1) / np.maximum(np.max(np.abs(ref), axis=1), 1e-300)
    assert keep.any(), "every point within rounding of a kink: choose another seed"
    log("  rel err (kept %d of %d): max %.3e median %.3e; left out: max %.3e" % (
        keep.sum(), n, err[keep].max(), np.median(err[keep]), err[~keep].max() if (~keep).any() else 0.0))
    if n >= 100:
        assert keep.sum() >= 0.9 * n
    assert err[keep].max() <= TOL
    assert np.all(np.isfinite(g))
    return g, ref


@pytest.mark.parametrize("n", [1, 13, 32, 173])
def test_vjp_paper_network_small_counts(env, n):
    run(env, mala_synth.paper_net(), n, 40 + n)


def test_vjp_paper_network_several_tiles_per_block(env):
    # 256 blocks x 32 points x 2 tiles + a ragged tail: every block loops
    run(env, mala_synth.paper_net(), 256 * 32 * 2 + 5, 3)


@pytest.mark.parametrize("out_act", [1, 0])
def test_vjp_small_network(env, out_act):
    net = mala_synth.make_net([55, 100, 100, 250], 101, 8, output_activation=out_act)
    run(env, net, 4099, 5 + out_act)


def test_vjp_generic_shape(env):
    net = mala_synth.make_net([55, 72, 96, 150], 7, 8, egrid=(-5.0, 0.1, 150))
    run(env, net, 777, 9)


def test_vjp_is_linear_in_v(env):
    """g is linear in v for fixed B: g(v1) + g(v2) = g(v1 + v2) to rounding."""
    mala, ctx, torch = env
    net = mala_synth.paper_net()
    B, v1 = mala_synth.network_inputs(net, 300, 21)
    _, v2 = mala_synth.network_inputs(net, 300, 22)
    w = ctx.weights(mala_synth.net_to_blob(net), mala.PREC_FP32)
    tB = torch.as_tensor(B, device="cuda")
    g1, g2, g12 = (ctx.mala_ldos_vjp(w, tB, torch.as_tensor(v, device="cuda")).cpu().double().numpy()
                   for v in (v1, v2, v1 + v2))
    err = np.max(np.abs(g1 + g2 - g12)) / np.max(np.abs(g12))
    log("linearity err", err)
    assert err <= 1e-5


def test_vjp_empty_and_bf16_rejected(env):
    mala, ctx, torch = env
    net = mala_synth.paper_net()
    w = ctx.weights(mala_synth.net_to_blob(net), mala.PREC_FP32)
    e = torch.empty((0, 91), dtype=torch.float32, device="cuda")
    out = ctx.mala_ldos_vjp(w, e, torch.empty((0, 250), dtype=torch.float32, device="cuda"))
    assert out.shape == (0, 91)
    wb = ctx.weights(mala_synth.net_to_blob(net), mala.PREC_BF16)
    B, v = mala_synth.network_inputs(net, 4, 1)
    with pytest.raises(mala.MalaError):
        ctx.mala_ldos_vjp(wb, torch.as_tensor(B, device="cuda"), torch.as_tensor(v, device="cuda"))


def test_vjp_full_grid_sampled(env):
    """The 729,000-point grid of the 256-atom cell in the launch configuration
    the bench times (256 blocks looping over 32-point tiles); 512 seeded
    sample rows are compared with the oracle."""
    mala, ctx, torch = env
    net = mala_synth.paper_net()
    n = 90 ** 3
    B, v = mala_synth.network_inputs(net, n, 29)
    w = ctx.weights(mala_synth.net_to_blob(net), mala.PREC_FP32)
    log("vjp full grid n", n)
    g = ctx.mala_ldos_vjp(w, torch.as_tensor(B, device="cuda"), torch.as_tensor(v, device="cuda"))
    ctx.synchronize()
    rows = mala_synth.sample_points(n, 512, 31)
    gs = g[torch.as_tensor(rows, device="cuda")].cpu().double().numpy()
    ref, margin = oracle.mlp_vjp(B[rows].astype(np.float64), net, v[rows].astype(np.float64), nthreads=16)
    keep = margin > MARGIN
    err = np.max(np.abs(gs - ref), axis=1) / np.max(np.abs(ref), axis=1)
    log("  full grid sampled rel err (kept %d of 512): max %.3e" % (keep.sum(), err[keep].max()))
    assert keep.sum() >= 0.9 * 512
    assert err[keep].max() <= TOL
    assert bool(torch.isfinite(g).all())
