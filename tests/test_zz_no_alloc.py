"""GPU: mala_integrate_noalloc (fixed device scratch, no allocation) against
mala_integrate on the same stored LDOS, through the C ABI, for two calls in a
row on one device, the second with fewer points (fewer partial rows of the
shared scratch are used, so rows left from the first call must not leak in).
The two entry points share their kernels and their partition of the points,
so DOS, density and the result record must agree bit for bit; both are also
held to the oracle's DOS and E_F at the stored-LDOS tolerances (DOS 1e-12,
E_F 1e-9 eV)."""
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


def _ldos(n, seed):
    rng = np.random.default_rng(seed)
    e = EG[0] + EG[1] * np.arange(EG[2])
    return (0.007 * np.sqrt(e + 5.5) * rng.uniform(0.8, 1.2, size=(n, EG[2]))).astype(np.float32)


def test_integrate_noalloc_matches_integrate(mala, torch):
    ctx = mala.Context(0)
    try:
        dV = 0.05
        # first call: more points than partial rows (2048 rows in use);
        # second call: 777 points (777 rows), T and N_e changed as well
        for n, T, seed in ((60_001, 298.0, 11), (777, 933.0, 12)):
            ld = _ldos(n, seed)
            D = oracle.dos(ld.astype(np.float64), dV)
            ne = float(oracle.fermi_weights(EG, 6.1, T)[0] @ D)
            ref = oracle.fermi(D, EG, T, ne)
            ldt = torch.as_tensor(ld, device="cuda")
            log("noalloc: n=%d T=%g seed=%d" % (n, T, seed))
            dos_a, dens_a, res_a = ctx.mala_integrate(ldt, dV, EG, T, ne)
            dos_b = torch.full((EG[2],), float("nan"), dtype=torch.float64, device="cuda")
            dens_b = torch.full((n,), float("nan"), dtype=torch.float64, device="cuda")
            res_b = torch.zeros(mala.RESULT_BYTES, dtype=torch.uint8, device="cuda")
            ctx.mala_integrate_noalloc(ldt, dV, EG, T, ne, dos_b, dens_b, res_b)
            torch.cuda.synchronize()
            ra, rb = mala.read_result(res_a), mala.read_result(res_b)
            log("  integrate", ra, "\n  noalloc  ", rb)
            assert rb["status"] == 0
            assert torch.equal(dos_a, dos_b)
            assert torch.equal(dens_a, dens_b)
            assert torch.equal(res_a, res_b)
            assert np.max(np.abs(dos_b.cpu().numpy() - D)) <= 1e-12 * np.max(D)
            assert abs(rb["e_fermi"] - ref["e_fermi"]) <= 1e-9
            assert abs(rb["n_found"] - ne) <= 1e-9 * ne
    finally:
        ctx.close()


def test_integrate_noalloc_rejects_wide_energy_grid(mala, torch):
    ctx = mala.Context(0)
    try:
        ld = torch.zeros((10, 300), dtype=torch.float32, device="cuda")
        dos = torch.zeros(300, dtype=torch.float64, device="cuda")
        res = torch.zeros(mala.RESULT_BYTES, dtype=torch.uint8, device="cuda")
        with pytest.raises(mala.MalaError):
            ctx.mala_integrate_noalloc(ld, 0.1, (-5.0, 0.1, 300), 298.0, 10.0, dos, None, res)
    finally:
        ctx.close()
