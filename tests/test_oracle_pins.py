"""Pins of the FP64 oracle against facts fixed outside the oracle itself.

Each test ties one oracle function to mathematics or to an independent
library routine (sympy's Clebsch-Gordan and Wigner-d, mpmath's polylog and
quadrature, numpy's matmul, Gauss-Legendre quadrature), chosen so that a
plausible slip (dropped term, sign, transposed operand, wrong index) fails.
"""
import os

import numpy as np
import pytest

import mala_synth
import oracle

GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
RC = 4.67


def rand_rot(rng):
    q = rng.normal(size=4)
    q /= np.linalg.norm(q)
    w, x, y, z = q
    return np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
                     [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
                     [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)]])


def rand_su2(rng):
    q = rng.normal(size=4)
    q /= np.linalg.norm(q)
    return complex(q[0], q[1]), complex(q[2], q[3])


def rand_disp(rng, n, rmax=RC * 0.98):
    d = rng.normal(size=(n, 3))
    d /= np.linalg.norm(d, axis=1)[:, None]
    return d * (rng.uniform(0.5, rmax, size=n))[:, None]


# ------------------------------------------------------------------ counts

def test_triple_count_matches_paper_formula():
    rows = np.loadtxt(os.path.join(GOLD, "snap_dim.txt"), comments="#", dtype=int)
    for tj, count in rows:
        assert oracle.triples(int(tj)).shape[0] == count
        assert oracle.lib().oracle_n_triples(int(tj)) == count


def test_paper_descriptor_parameters_give_91():
    kv = dict(l.split() for l in open(os.path.join(GOLD, "paper_parameters.txt"))
              if l.strip() and not l.startswith("#"))
    assert oracle.triples(int(kv["twojmax"])).shape[0] == 91


def test_triple_order_and_constraints():
    t = oracle.triples(10)
    for j1, j2, j in t:
        assert j2 <= j1 <= j <= 10 and abs(j1 - j2) <= j <= j1 + j2 and (j1 + j2 + j) % 2 == 0
    assert [tuple(x) for x in t] == sorted(set(tuple(x) for x in t))


# ------------------------------------------------------------------ Clebsch-Gordan

def test_cg_matches_sympy():
    from sympy import Rational
    from sympy.physics.wigner import clebsch_gordan
    n = 0
    for j1 in range(0, 7):
        for j2 in range(0, 7):
            for j in range(abs(j1 - j2), j1 + j2 + 1, 2):
                for m1 in range(-j1, j1 + 1, 2):
                    for m2 in range(-j2, j2 + 1, 2):
                        m = m1 + m2
                        if abs(m) > j:
                            continue
                        ref = float(clebsch_gordan(Rational(j1, 2), Rational(j2, 2), Rational(j, 2),
                                                   Rational(m1, 2), Rational(m2, 2), Rational(m, 2)))
                        assert abs(oracle.cg(j1, m1, j2, m2, j, m) - ref) < 1e-14
                        n += 1
    assert n > 1000


def test_cg_orthonormality_up_to_twojmax_10():
    for j1 in range(0, 11):
        for j2 in range(0, j1 + 1):
            js = list(range(j1 - j2, j1 + j2 + 1, 2))
            for m in range(-(j1 + j2), j1 + j2 + 1, 2):
                pairs = [(m1, m - m1) for m1 in range(-j1, j1 + 1, 2) if abs(m - m1) <= j2]
                M = np.array([[oracle.cg(j1, m1, j2, m2, j, m) for (m1, m2) in pairs] for j in js
                              if abs(m) <= j])
                assert np.allclose(M @ M.T, np.eye(M.shape[0]), atol=1e-13)


# ------------------------------------------------------------------ U^j

def test_u_is_a_unitary_representation():
    rng = np.random.default_rng(7)
    for _ in range(5):
        a1, b1 = rand_su2(rng)
        a2, b2 = rand_su2(rng)
        g1 = np.array([[a1, b1], [-np.conj(b1), np.conj(a1)]])
        g2 = np.array([[a2, b2], [-np.conj(b2), np.conj(a2)]])
        g = g1 @ g2
        for J in range(0, 11):
            U1, U2 = oracle.wigner_u(J, a1, b1), oracle.wigner_u(J, a2, b2)
            U = oracle.wigner_u(J, g[0, 0], g[0, 1])
            assert np.allclose(U1 @ U1.conj().T, np.eye(J + 1), atol=1e-13)
            # the polynomial-substitution definition gives the transposed action,
            # so U(g1 g2) = U(g2) U(g1): U^T is a homomorphism of SU(2)
            assert np.allclose(U, U2 @ U1, atol=1e-12)


def test_u_character_formula():
    # trace of the spin-J/2 irrep of an SU(2) element with eigenvalues e^{+-i t}
    rng = np.random.default_rng(8)
    for _ in range(10):
        a, b = rand_su2(rng)
        t = np.arccos(a.real)
        for J in range(0, 11):
            chi = np.trace(oracle.wigner_u(J, a, b))
            assert abs(chi - np.sin((J + 1) * t) / np.sin(t)) < 1e-11


def test_u_rotation_about_y_matches_sympy_wigner_d():
    from sympy import Rational, N as sN
    from sympy.physics.quantum.spin import Rotation
    r = 0.8
    a, b = oracle.cayley_klein([0.0, r, 0.0], RC)
    th0 = 0.99363 * np.pi * r / RC
    for J in range(1, 7):
        U = oracle.wigner_u(J, a, b)
        D = np.zeros((J + 1, J + 1))
        for ma in range(J + 1):
            for mb in range(J + 1):
                v = complex(sN(Rotation.d(Rational(J, 2), Rational(J - 2 * ma, 2),
                                          Rational(J - 2 * mb, 2), 2 * th0).doit()))
                D[ma, mb] = v.real
        assert np.max(np.abs(U - D)) < 1e-12


def test_u_rotation_about_z_is_diagonal_phase():
    r = 1.3
    a, b = oracle.cayley_klein([0.0, 0.0, r], RC)
    th0 = 0.99363 * np.pi * r / RC
    assert abs(b) == 0.0
    for J in range(0, 11):
        U = oracle.wigner_u(J, a, b)
        phases = np.exp(-1j * th0 * (2 * np.arange(J + 1) - J))
        assert np.allclose(U, np.diag(phases), atol=1e-13)


def test_cayley_klein_and_cutoff():
    a, b = oracle.cayley_klein([0.0, 0.0, 0.0], RC)
    assert a == 1 and b == 0
    rng = np.random.default_rng(3)
    for d in rand_disp(rng, 10):
        a, b = oracle.cayley_klein(d, RC)
        assert abs(abs(a) ** 2 + abs(b) ** 2 - 1) < 1e-15
    assert oracle.cutoff(0.0, RC) == 1.0
    assert oracle.cutoff(RC, RC) == 0.0
    assert abs(oracle.cutoff(RC / 2, RC) - 0.5) < 1e-15


# ------------------------------------------------------------------ u and B

def test_u_sums_identity_and_weighted_neighbours():
    rng = np.random.default_rng(4)
    d = rand_disp(rng, 3)
    u = oracle.u_levels(d, RC, 4)
    r = np.linalg.norm(d, axis=1)
    assert abs(u[0][0, 0] - (1 + sum(oracle.cutoff(x, RC) for x in r))) < 1e-14
    for J in range(5):
        ref = np.eye(J + 1, dtype=complex)
        for k in range(3):
            a, b = oracle.cayley_klein(d[k], RC)
            ref += oracle.cutoff(r[k], RC) * oracle.wigner_u(J, a, b)
        assert np.allclose(u[J], ref, atol=1e-14)


@pytest.mark.parametrize("tj", [4, 8, 10])
def test_b_empty_neighbourhood_is_j_plus_1(tj):
    B, mi = oracle.bispectrum_from_disp(np.zeros((0, 3)), RC, tj)
    t = oracle.triples(tj)
    assert np.max(np.abs(B - (t[:, 2] + 1))) < 1e-12 and mi < 1e-14


def test_b_atom_on_grid_point():
    # one atom exactly on the point: u = 2 I, so B = 8 (J+1)
    B, _ = oracle.bispectrum_from_disp(np.zeros((1, 3)), RC, 8)
    t = oracle.triples(8)
    assert np.max(np.abs(B - 8 * (t[:, 2] + 1))) < 1e-11


def test_b000_is_weighted_count_cubed():
    rng = np.random.default_rng(5)
    d = rand_disp(rng, 12)
    B, _ = oracle.bispectrum_from_disp(d, RC, 6)
    fc = sum(oracle.cutoff(np.linalg.norm(x), RC) for x in d)
    assert abs(B[0] - (1 + fc) ** 3) < 1e-11 * B[0]


@pytest.mark.parametrize("tj", [6, 10])
def test_b_invariances(tj):
    rng = np.random.default_rng(10 + tj)
    d = rand_disp(rng, 9 if tj == 10 else 14)
    B, mi = oracle.bispectrum_from_disp(d, RC, tj)
    scale = np.max(np.abs(B))
    assert mi < 1e-13 * scale
    R = rand_rot(rng)
    Br, _ = oracle.bispectrum_from_disp(d @ R.T, RC, tj)
    Bi, _ = oracle.bispectrum_from_disp(-d, RC, tj)
    Bp, _ = oracle.bispectrum_from_disp(d[rng.permutation(d.shape[0])], RC, tj)
    for other in (Br, Bi, Bp):
        assert np.max(np.abs(other - B)) < 1e-12 * scale
    # a neighbour outside the cutoff changes nothing
    Bo, _ = oracle.bispectrum_from_disp(np.vstack([d, [[0, 0, RC * 1.01]]]), RC, tj)
    assert np.max(np.abs(Bo - B)) == 0.0


def _b_any(u, j1, j2, j):
    """B(j1,j2,j) for any admissible order, from u and the oracle's CG."""
    tot = 0j
    for m in range(-j, j + 1, 2):
        for mp in range(-j, j + 1, 2):
            z = 0j
            for m1 in range(-j1, j1 + 1, 2):
                for m1p in range(-j1, j1 + 1, 2):
                    m2, m2p = m - m1, mp - m1p
                    if abs(m2) > j2 or abs(m2p) > j2:
                        continue
                    z += (oracle.cg(j1, m1, j2, m2, j, m) * oracle.cg(j1, m1p, j2, m2p, j, mp) *
                          u[j1][(j1 + m1) // 2, (j1 + m1p) // 2] * u[j2][(j2 + m2) // 2, (j2 + m2p) // 2])
            tot += np.conj(u[j][(j + m) // 2, (j + mp) // 2]) * z
    return tot.real


def test_b_permutation_identities():
    rng = np.random.default_rng(12)
    d = rand_disp(rng, 6)
    u = oracle.u_levels(d, RC, 6)
    B, _ = oracle.bispectrum_from_u(u, 6)
    idx = {tuple(t): k for k, t in enumerate(oracle.triples(6))}
    for (j1, j2, j), k in idx.items():
        assert abs(_b_any(u, j2, j1, j) - B[k]) < 1e-11 * abs(B).max()
        # B(j1,j2,j) (j1+1) = B(j,j2,j1) (j+1)  (doubled indices)
        lhs = B[k] * (j1 + 1)
        rhs = _b_any(u, j, j2, j1) * (j + 1)
        assert abs(lhs - rhs) < 1e-10 * abs(B).max()


def test_b_single_neighbour_on_z_closed_form():
    # neighbour on +z: U is diagonal, so B = sum_m conj(u_mm) sum_m1 C^2 u1_m1m1 u2_m2m2
    from sympy import Rational
    from sympy.physics.wigner import clebsch_gordan
    r = 2.1
    fc = oracle.cutoff(r, RC)
    th0 = 0.99363 * np.pi * r / RC

    def diag(J, ma):
        return 1 + fc * np.exp(-1j * th0 * (2 * ma - J))

    B, _ = oracle.bispectrum_from_disp(np.array([[0.0, 0.0, r]]), RC, 6)
    for k, (j1, j2, j) in enumerate(oracle.triples(6)):
        tot = 0j
        for m in range(-j, j + 1, 2):
            s = 0j
            for m1 in range(-j1, j1 + 1, 2):
                m2 = m - m1
                if abs(m2) > j2:
                    continue
                c = float(clebsch_gordan(Rational(j1, 2), Rational(j2, 2), Rational(j, 2),
                                         Rational(m1, 2), Rational(m2, 2), Rational(m, 2)))
                s += c * c * diag(j1, (j1 + m1) // 2) * diag(j2, (j2 + m2) // 2)
            tot += np.conj(diag(j, (j + m) // 2)) * s
        assert abs(tot.real - B[k]) < 1e-12 * max(1.0, abs(B).max())
    # the same closed form holds for the neighbour in any direction
    R = rand_rot(np.random.default_rng(1))
    Br, _ = oracle.bispectrum_from_disp(np.array([[0.0, 0.0, r]]) @ R.T, RC, 6)
    assert np.max(np.abs(Br - B)) < 1e-12 * abs(B).max()


# ------------------------------------------------------------------ grid geometry

def test_neighbours_brute_force_periodic_images():
    import mala_synth
    s = mala_synth.small()                   # L = 8.1 < 2 rcut: several images per atom
    for p in (0, 137, 7999):
        d = oracle.neighbours(s, p)
        k, j, i = p % 20, (p // 20) % 20, p // 400
        r = np.array([i, j, k]) * s.L / s.N
        ref = []
        for a in s.positions:
            for n in np.ndindex(5, 5, 5):
                v = a + (np.array(n) - 2) * s.L - r
                if np.dot(v, v) < RC * RC:
                    ref.append(v)
        ref = np.array(ref)
        assert d.shape == ref.shape
        key = lambda x: tuple(np.round(x, 9))
        assert sorted(map(key, d)) == sorted(map(key, ref))


def test_descriptor_field_translation():
    import mala_synth
    s = mala_synth.small()
    shift = np.array([3, 1, 2])
    t = mala_synth.Snapshot("shifted", np.mod(s.positions + shift * s.L / s.N, s.L), s.L, s.N,
                            s.rcut, 6, s.T, s.n_electrons)
    s6 = mala_synth.with_grid(s, s.N)
    s6.twojmax = 6
    pts = np.array([0, 21, 455, 7999])
    ijk = np.stack([pts // 400, (pts // 20) % 20, pts % 20], 1)
    moved = ((ijk + shift) % 20) @ np.array([400, 20, 1])
    B0 = oracle.descriptors(s6, pts)
    B1 = oracle.descriptors(t, moved)
    assert np.max(np.abs(B0 - B1)) < 1e-9 * np.abs(B0).max()


# ------------------------------------------------------------------ network

def test_mlp_matches_numpy_chain():
    import mala_synth
    rng = np.random.default_rng(0)
    for out_act in (1, 0):
        net = mala_synth.make_net([7, 11, 5, 9], 3, 8, output_activation=out_act,
                                  with_input_scaler=False, egrid=(-5.0, 0.1, 9))
        net["in_mean"] = rng.normal(size=7)
        net["in_std"] = rng.uniform(0.5, 2, size=7)
        B = rng.normal(size=(13, 7)) * 3
        x = (B - net["in_mean"]) / net["in_std"]
        for l in range(3):
            x = x @ net["W"][l].T + net["b"][l]
            if l < 2 or out_act:
                x = np.where(x < 0, 0.01 * x, x)
        ref = net["out_scale"] * x + net["out_shift"]
        assert np.allclose(oracle.mlp(B, net), ref, rtol=1e-13, atol=1e-14)


@pytest.mark.parametrize("out_act", [1, 0])
def test_mlp_hand_built_network(out_act):
    """A 3-2-2-2 network evaluated by hand (Eq. ffnn with the input
    standardisation and the affine output transform): every bias, the slope
    of a negative unit, the input scaler, the output transform and the
    output-activation flag change the expected values below."""
    import mala_synth
    net = mala_synth.make_net([3, 2, 2, 2], 1, 2, output_activation=out_act, with_input_scaler=False,
                              egrid=(-5.0, 0.1, 2))
    net["in_mean"], net["in_std"] = np.array([1.0, 0.0, 1.0]), np.array([1.0, 2.0, 2.0])
    net["W"] = [np.array([[1.0, -1.0, 2.0], [-2.0, -3.0, 1.0]]), np.array([[1.0, 2.0], [-1.0, 1.0]]),
                np.array([[2.0, 0.0], [1.0, -4.0]])]
    net["b"] = [np.array([0.5, -0.25]), np.array([-1.0, 0.5]), np.array([0.25, -1.0])]
    net["out_scale"], net["out_shift"] = np.array([2.0, 0.5]), np.array([0.1, 0.2])
    net["slope"] = 0.01
    # x0 = (B - mean)/std = (0, 1, 1); layer 1: z = (1.5, -2.25) -> (1.5, -0.0225);
    # layer 2: z = (0.455, -1.0225) -> (0.455, -0.010225); layer 3: z = (1.16, -0.5041),
    # -> (1.16, -0.005041) with the activation on the output; d = s y + c
    expect = [2.42, 0.1974795] if out_act else [2.42, -0.05205]
    got = oracle.mlp(np.array([[1.0, 2.0, 3.0]]), net)
    np.testing.assert_allclose(got[0], expect, rtol=1e-14, atol=1e-15)


def test_dos_is_scaled_sum():
    rng = np.random.default_rng(2)
    ld = rng.uniform(size=(50, 17))
    assert np.allclose(oracle.dos(ld, 0.37), 0.37 * ld.sum(0), rtol=1e-14)


# ------------------------------------------------------------------ integration

def test_polylog_against_mpmath_and_closed_forms():
    import mpmath
    for s in (2, 3):
        for y in (0.0, 1e-8, 0.05, 0.3, 0.5, 0.77, 0.999, 1.0):
            ref = float(mpmath.polylog(s, -y))
            assert abs(oracle.li_neg(s, y) - ref) < 1e-15 * max(1, abs(ref))
    assert abs(oracle.li_neg(2, 1.0) + np.pi ** 2 / 12) < 1e-15
    assert abs(oracle.li_neg(3, 1.0) + 0.75 * 1.2020569031595942) < 1e-15
    assert abs(oracle.li_neg(1, 0.4) + np.log1p(0.4)) < 1e-15


def _fermi(e, mu, kT):
    return 0.5 * (1 - np.tanh(0.5 * (e - mu) / kT))


@pytest.mark.parametrize("T,mu", [(298.0, 6.27), (933.0, 3.05), (298.0, -4.93), (5000.0, 19.8)])
def test_weights_match_gauss_legendre(T, mu):
    eg = (-5.0, 0.1, 250)
    kT = oracle.KB_EV * T
    w, v = oracle.fermi_weights(eg, mu, T)
    e = eg[0] + eg[1] * np.arange(eg[2])
    rng = np.random.default_rng(1)
    D = rng.uniform(0.1, 2.0, size=eg[2])
    xg, wg = np.polynomial.legendre.leggauss(64)
    N = Eb = 0.0
    for i in range(eg[2] - 1):
        # split the interval at mu so the quadrature sees a smooth integrand
        cuts = [e[i], e[i + 1]]
        if e[i] < mu < e[i + 1]:
            cuts = [e[i], mu, e[i + 1]]
        for lo, hi in zip(cuts[:-1], cuts[1:]):
            x = 0.5 * (hi - lo) * xg + 0.5 * (hi + lo)
            Dx = D[i] + (D[i + 1] - D[i]) * (x - e[i]) / eg[1]
            f = _fermi(x, mu, kT)
            N += 0.5 * (hi - lo) * np.sum(wg * f * Dx)
            Eb += 0.5 * (hi - lo) * np.sum(wg * f * x * Dx)
    assert abs(w @ D - N) < 1e-12 * N
    assert abs(v @ D - Eb) < 1e-11 * max(1.0, abs(Eb))


def test_weights_constant_dos_closed_form():
    eg = (-5.0, 0.1, 250)
    for T, mu in ((298.0, 6.0), (933.0, 0.123)):
        kT = oracle.KB_EV * T
        w, _ = oracle.fermi_weights(eg, mu, T)
        a, b = eg[0], eg[0] + eg[1] * (eg[2] - 1)
        F = lambda e: e - kT * np.logaddexp(0.0, (e - mu) / kT)
        assert abs(w.sum() - (F(b) - F(a))) < 1e-12


def test_weights_zero_temperature_limit_is_trapezoid():
    eg = (-5.0, 0.1, 250)
    mu = 2.0                                   # on a grid point: e_70
    w, v = oracle.fermi_weights(eg, mu, 1e-3)
    ref = np.zeros(250)
    ref[:71] = 0.1
    ref[0] = ref[70] = 0.05
    assert np.max(np.abs(w - ref)) < 1e-9
    e = eg[0] + eg[1] * np.arange(250)
    # exact int_{e0}^{mu} e * (piecewise linear D = 1) de
    assert abs(v.sum() - 0.5 * (mu * mu - 25.0)) < 1e-8


def test_weights_mpmath_high_precision():
    import mpmath
    mpmath.mp.dps = 30
    eg = (-5.0, 0.1, 20)
    mu, T = -4.03, 933.0
    kT = oracle.KB_EV * T
    w, v = oracle.fermi_weights(eg, mu, T)
    e = [eg[0] + eg[1] * i for i in range(eg[2])]
    for i in (0, 5, 9, 10, 11, 19):
        def hat(x):
            if i > 0 and e[i - 1] <= x <= e[i]:
                return (x - e[i - 1]) / eg[1]
            if i < eg[2] - 1 and e[i] <= x <= e[i + 1]:
                return (e[i + 1] - x) / eg[1]
            return 0
        f = lambda x: hat(x) / (1 + mpmath.exp((x - mu) / kT))
        pts = [e[max(i - 1, 0)], e[i], e[min(i + 1, eg[2] - 1)]]
        ref = float(mpmath.quad(f, pts))
        refv = float(mpmath.quad(lambda x: x * f(x), pts))
        assert abs(w[i] - ref) < 1e-14
        assert abs(v[i] - refv) < 1e-13


def test_fermi_root_monotone_and_no_root():
    eg = (-5.0, 0.1, 250)
    e = eg[0] + eg[1] * np.arange(250)
    D = 40.0 * np.sqrt(e + 5.5)
    for T in (298.0, 933.0):
        r = oracle.fermi(D, eg, T, 768.0)
        w, _ = oracle.fermi_weights(eg, r["e_fermi"], T)
        assert abs(w @ D - 768.0) < 1e-8
        lo, _ = oracle.fermi_weights(eg, r["e_fermi"] - 1e-6, T)
        assert lo @ D < 768.0
        assert r["iters"] <= 64
    with pytest.raises(oracle.NoRoot):
        oracle.fermi(D, eg, 298.0, 1e7)
    with pytest.raises(oracle.NoRoot):
        oracle.fermi(D, eg, 298.0, 0.0)


def test_density_integrates_to_electron_count():
    rng = np.random.default_rng(9)
    eg = (-5.0, 0.1, 250)
    e = eg[0] + eg[1] * np.arange(250)
    ld = rng.uniform(0.5, 1.5, size=(300, 250)) * 0.007 * np.sqrt(e + 5.5)
    dV = 0.3
    D = oracle.dos(ld, dV)
    ne = 0.5 * (w0 := oracle.fermi_weights(eg, 19.0, 298.0)[0]) @ D
    r = oracle.fermi(D, eg, 298.0, ne)
    n = oracle.density(ld, r["weights"])
    assert abs(n.sum() * dV - ne) < 1e-9 * ne


# ---------------------------------------------------------------- entropy
# Eq. electronicentropyDOS: S_s / k_B = int -[f ln f + (1-f) ln(1-f)] D de.

def _entropy_integrand(E, mu, kT):
    x = (E - mu) / kT
    if abs(x) > 700:
        return 0.0
    f = 1.0 / (1.0 + np.exp(x))
    r = 0.0
    if f > 0.0:
        r -= f * np.log(f)
    if f < 1.0:
        r -= (1.0 - f) * np.log1p(-f)
    return r


@pytest.mark.parametrize("T,mu", [(298.0, 0.93), (933.0, 1.234), (3000.0, 2.0), (298.0, -1.97)])
def test_entropy_weights_match_quadrature(T, mu):
    # the paper's integrand integrated numerically against a random piecewise-linear D
    from scipy.integrate import quad
    kT = oracle.KB_EV * T
    rng = np.random.default_rng(7)
    eg = (-2.0, 0.1, 60)
    e = eg[0] + eg[1] * np.arange(eg[2])
    D = rng.uniform(0.0, 2.0, eg[2])
    q = 0.0
    for i in range(eg[2] - 1):
        a, b = e[i], e[i + 1]
        lin = lambda E, i=i, a=a: D[i] + (D[i + 1] - D[i]) * (E - a) / eg[1]
        q += quad(lambda E: _entropy_integrand(E, mu, kT) * lin(E), a, b, epsabs=1e-14, epsrel=1e-13,
                  limit=200, points=[mu] if a < mu < b else None)[0]
    S, mts = oracle.entropy(D, eg, mu, T)
    assert abs(S - q) <= 1e-12 * abs(q)
    assert abs(mts + kT * S) <= 1e-15 * abs(mts)


def test_entropy_closed_forms():
    # int s(x) dx = pi^2/3 and s is even: a constant D gives D kT pi^2/3 and a
    # linear D gives kT pi^2/3 D(mu) (the odd part integrates to zero), when the
    # grid reaches far past mu on both sides; at T -> 0 the entropy vanishes.
    eg = (-10.0, 0.05, 401)
    e = eg[0] + eg[1] * np.arange(eg[2])
    mu, T = 0.0123, 933.0
    kT = oracle.KB_EV * T
    S, _ = oracle.entropy(np.full(eg[2], 2.5), eg, mu, T)
    assert abs(S - 2.5 * kT * np.pi ** 2 / 3.0) <= 1e-13 * S
    D = 1.7 + 0.3 * (e - mu)
    S, _ = oracle.entropy(D, eg, mu, T)
    assert abs(S - 1.7 * kT * np.pi ** 2 / 3.0) <= 1e-12 * S
    S, _ = oracle.entropy(np.full(eg[2], 2.5), eg, mu, 1e-3)
    assert 0.0 <= S <= 2.5 * oracle.KB_EV * 1e-3 * np.pi ** 2 / 3.0 * (1 + 1e-9)
    u = oracle.entropy_weights(eg, mu, T)
    assert np.all(u >= 0.0)


# ---------------------------------------------------------------- Gaussian descriptors
# Normalised Gaussians on every atom image (the representation behind
# Eq. structurefactor_gaussian).

def _aliasing_bound(sigma, h):
    # Poisson summation: sum_p G(p) dV - N_atoms = N_atoms x (sum over nonzero
    # reciprocal grid vectors of the Gaussian's Fourier transform x phases), so
    # |error| / N_atoms <= sum_{m != 0} exp(-2 pi^2 sigma^2 sum_d (m_d / h_d)^2)
    m = np.arange(-4, 5)
    tot = 0.0
    for a in m:
        for b in m:
            for c in m:
                if a == b == c == 0:
                    continue
                tot += np.exp(-2 * np.pi ** 2 * sigma ** 2 * ((a / h[0]) ** 2 + (b / h[1]) ** 2 + (c / h[2]) ** 2))
    return tot


@pytest.mark.parametrize("fac", [0.7, 1.0, 1.5])
def test_gaussian_integrates_to_atom_count(fac):
    snap = mala_synth.small()
    h = snap.L / snap.N
    sigma = fac * float(np.max(h))
    G = oracle.gaussian(snap, sigma, 8.0 * sigma)
    err = abs(G.sum() * snap.dV / snap.n_atoms - 1.0)
    assert err <= 1.01 * _aliasing_bound(sigma, h) + 1e-13
    if fac == 0.7:
        assert err > 1e-7                     # the bound is not vacuous here


def test_gaussian_single_atom_closed_form_and_translation():
    # one atom on a grid point of a large cell: G there is the peak value;
    # moving the atom by whole grid steps moves the field by the same steps
    L, N = np.array([12.0, 12.0, 12.0]), np.array([24, 24, 24])
    sigma = 0.6
    pos = np.array([[6.0, 6.0, 6.0]])
    snap = mala_synth.Snapshot("one", pos, L, N, 4.67, 8, 298.0, 3.0)
    p0 = (12 * 24 + 12) * 24 + 12
    G = oracle.gaussian(snap, sigma, 5.0)
    assert abs(G[p0] - (2 * np.pi * sigma ** 2) ** -1.5) <= 1e-15 * G[p0]
    snap2 = mala_synth.Snapshot("one", pos + np.array([0.5, 1.0, 1.5]), L, N, 4.67, 8, 298.0, 3.0)
    G2 = oracle.gaussian(snap2, sigma, 5.0).reshape(24, 24, 24)
    G1 = np.roll(G.reshape(24, 24, 24), (1, 2, 3), axis=(0, 1, 2))
    assert np.max(np.abs(G2 - G1)) <= 1e-14 * np.max(G)
    # a point 1 A from the atom along x sees exp(-1/(2 sigma^2)) of the peak
    p1 = (14 * 24 + 12) * 24 + 12
    assert abs(G[p1] / G[p0] - np.exp(-1.0 / (2 * sigma ** 2))) <= 1e-14


# ---------------------------------------------------------------- network VJP
def _vjp_inputs(net, n, seed):
    B, v = mala_synth.network_inputs(net, n, seed)
    return B.astype(np.float64), v.astype(np.float64)


@pytest.mark.parametrize("out_act", [1, 0])
def test_mlp_vjp_matches_central_differences(out_act):
    """The network is piecewise linear in B, so a central difference that
    crosses no kink is exact up to rounding: g_k = sum_e v_e dd_e/dB_k."""
    net = mala_synth.make_net([55, 100, 100, 250], 101, 8, output_activation=out_act)
    B, v = _vjp_inputs(net, 8, 7)
    g, margin = oracle.mlp_vjp(B, net, v)
    keep = margin > 1e-4                 # far from every kink: a 1e-7 std step cannot cross one
    assert keep.sum() >= 4
    for p in np.nonzero(keep)[0]:
        for k in range(B.shape[1]):
            h = 1e-7 * net["in_std"][k]
            Bp, Bm = B[p:p + 1].copy(), B[p:p + 1].copy()
            Bp[0, k] += h
            Bm[0, k] -= h
            fd = (oracle.mlp(Bp, net) - oracle.mlp(Bm, net))[0] @ v[p] / (2 * h)
            assert abs(fd - g[p, k]) <= 1e-6 * np.max(np.abs(g[p])), (p, k, fd, g[p, k])


@pytest.mark.parametrize("out_act", [1, 0])
def test_mlp_vjp_linear_network_closed_form(out_act):
    """slope = 1 makes the network affine: g = ((s .* v) W3 W2 W1) ./ std."""
    net = mala_synth.make_net([55, 100, 100, 250], 103, 8, output_activation=out_act, slope=1.0)
    B, v = _vjp_inputs(net, 5, 11)
    g, _ = oracle.mlp_vjp(B, net, v)
    W1, W2, W3 = net["W"]
    ref = ((v * net["out_scale"]) @ W3 @ W2 @ W1) / net["in_std"]
    np.testing.assert_allclose(g, ref, rtol=1e-12, atol=1e-12 * np.abs(ref).max())


def test_mlp_vjp_kink_side_and_margin():
    """A unit with z <= 0 passes slope * delta back (the kink belongs to the
    negative side); the margin is the smallest relative distance to a kink."""
    net = mala_synth.make_net([4, 3, 3, 2], 5, 2, output_activation=1, with_input_scaler=False,
                              egrid=(-5.0, 0.1, 2))
    net["W"] = [np.eye(3, 4), np.eye(3), np.eye(2, 3)]
    net["b"] = [np.zeros(3), np.zeros(3), np.zeros(2)]
    net["out_scale"], net["out_shift"] = np.ones(2), np.zeros(2)
    B = np.array([[2.0, -3.0, 0.5, 7.0]])
    v = np.array([[1.0, 1.0]])
    g, margin = oracle.mlp_vjp(B, net, v)
    s = net["slope"]
    # unit 0 positive through all layers -> 1; unit 1 negative -> slope^3; input 3 unused
    np.testing.assert_allclose(g[0], [1.0 / net["in_std"][0], s ** 3 / net["in_std"][1], 0.0, 0.0],
                               rtol=1e-15)
    assert margin[0] == pytest.approx(1.0)


# ---------------------------------------------------------------- descriptor VJP
def _tiny_snap(n_atoms=3, L=6.0, N=4, tj=4, rcut=3.2, seed=3):
    rng = np.random.default_rng(seed)
    pos = rng.uniform(0, L, size=(n_atoms, 3))
    return mala_synth.Snapshot("tiny", pos, np.array([L, L, L]), np.array([N, N, N]), rcut, tj, 298.0,
                               3.0 * n_atoms)


def _loss(snap, pos, gB, pts):
    s = mala_synth.Snapshot(snap.name, pos, snap.L, snap.N, snap.rcut, snap.twojmax, snap.T, snap.n_electrons)
    return float(np.sum(gB * oracle.descriptors(s, pts)))


@pytest.mark.parametrize("tj", [2, 4, 6])
def test_descriptor_vjp_matches_central_differences(tj):
    """L(R) = sum_p gB(p).B(p) is smooth in R away from r = 0 and r = rcut;
    a central difference with h = 1e-5 A is accurate to ~1e-9 relative.
    The cell (6 A) is smaller than 2 rcut, so atoms enter through several
    periodic images."""
    snap = _tiny_snap(tj=tj)
    pts = np.array([0, 5, 21, 42, 63], dtype=np.int64)
    nb = oracle.lib().oracle_n_triples(tj)
    gB = np.random.default_rng(5).standard_normal((pts.size, nb))
    grad = oracle.descriptors_vjp(snap, gB, pts)
    h = 1e-5
    fd = np.zeros_like(grad)
    for a in range(snap.n_atoms):
        for d in range(3):
            pp, pm = snap.positions.copy(), snap.positions.copy()
            pp[a, d] += h
            pm[a, d] -= h
            fd[a, d] = (_loss(snap, pp, gB, pts) - _loss(snap, pm, gB, pts)) / (2 * h)
    assert np.max(np.abs(fd - grad)) <= 1e-7 * np.max(np.abs(grad)), (fd, grad)


def test_descriptor_vjp_b000_closed_form():
    """B_000 = (1 + sum_k fc(r_k))^3 (weighted neighbour count cubed), so with
    gB = e_000 the gradient on atom a is
    3 (1 + sum fc)^2 sum_{images k of a} fc'(r_k) Delta_k / r_k per point."""
    snap = _tiny_snap(n_atoms=4, tj=4, seed=8)
    pts = np.array([3, 17, 40], dtype=np.int64)
    nb = oracle.lib().oracle_n_triples(4)
    gB = np.zeros((pts.size, nb))
    gB[:, 0] = 1.0
    grad = oracle.descriptors_vjp(snap, gB, pts)
    ref = np.zeros_like(grad)
    L = snap.L
    for p in pts:
        i, j, k = p // 16, (p // 4) % 4, p % 4
        rp = np.array([i, j, k]) * L / snap.N
        terms = []
        for a in range(snap.n_atoms):
            for sh in np.array(np.meshgrid(*[np.arange(-2, 3)] * 3)).reshape(3, -1).T:
                dv = snap.positions[a] + sh * L - rp
                r = np.linalg.norm(dv)
                if 0 < r < snap.rcut:
                    fc = 0.5 * (np.cos(np.pi * r / snap.rcut) + 1)
                    dfc = -0.5 * np.pi / snap.rcut * np.sin(np.pi * r / snap.rcut)
                    terms.append((a, fc, dfc * dv / r))
        s = 1.0 + sum(t[1] for t in terms)
        for a, _, gv in terms:
            ref[a] += 3 * s ** 2 * gv
    np.testing.assert_allclose(grad, ref, rtol=1e-12, atol=1e-12 * np.abs(ref).max())


def test_descriptor_vjp_rotation_invariance_no_torque():
    """B(p) is invariant under rotations about the grid point, so with one
    image per atom sum_a Delta_a x dL/dR_a = 0 (no torque about r_p)."""
    rng = np.random.default_rng(12)
    L = 30.0
    rp = np.zeros(3)
    pos = rng.normal(scale=1.6, size=(5, 3))           # around the grid point at the origin
    pos = pos[np.linalg.norm(pos, axis=1) < 4.0]
    snap = mala_synth.Snapshot("iso", np.mod(pos, L), np.array([L, L, L]), np.array([10, 10, 10]), 4.67, 6,
                               298.0, 3.0)
    nb = oracle.lib().oracle_n_triples(6)
    gB = rng.standard_normal((1, nb))
    grad = oracle.descriptors_vjp(snap, gB, np.array([0], dtype=np.int64))
    torque = np.sum(np.cross(pos - rp, grad), axis=0)
    assert np.max(np.abs(torque)) <= 1e-12 * np.max(np.abs(grad)) * np.max(np.abs(pos)), torque
    assert np.max(np.abs(grad)) > 0


def test_descriptor_vjp_atom_on_grid_point_contributes_nothing():
    """At r = 0 the map from the displacement to U has no derivative (its
    first-order term depends on the direction), so an atom sitting exactly on
    a grid point is left out of that point's gradient by convention; the
    result stays finite."""
    snap = _tiny_snap(n_atoms=2, tj=2, seed=4)
    snap.positions[0] = np.array([1.5, 3.0, 4.5])       # grid points sit at multiples of 1.5 A
    p = np.array([(1 * 4 + 2) * 4 + 3], dtype=np.int64)
    nb = oracle.lib().oracle_n_triples(2)
    g1 = oracle.descriptors_vjp(snap, np.ones((1, nb)), p)
    assert np.all(np.isfinite(g1))


# ---------------------------------------------------------------- grid ACE
def _iso_snap(pos, L=30.0, N=10):
    return mala_synth.Snapshot("iso", np.mod(np.asarray(pos, float), L), np.array([L, L, L]),
                               np.array([N, N, N]), 4.67, 8, 298.0, 3.0)


def test_ace_ylm_matches_scipy_and_3j_matches_sympy():
    import scipy.special as sp
    from sympy.physics.wigner import wigner_3j
    rng = np.random.default_rng(3)
    for d in rng.normal(size=(6, 3)):
        r = np.linalg.norm(d)
        th, ph = np.arccos(d[2] / r), np.arctan2(d[1], d[0])
        for l in range(5):
            for m in range(-l, l + 1):
                assert abs(oracle.ylm(l, m, d) - complex(sp.sph_harm_y(l, m, th, ph))) < 1e-13
    for l1 in range(5):
        for l2 in range(5):
            for l3 in range(abs(l1 - l2), min(4, l1 + l2) + 1):
                for m1 in range(-l1, l1 + 1):
                    for m2 in range(-l2, l2 + 1):
                        m3 = -m1 - m2
                        if abs(m3) > l3:
                            continue
                        assert abs(oracle.wigner3j(l1, l2, l3, m1, m2, m3) -
                                   float(wigner_3j(l1, l2, l3, m1, m2, m3))) < 1e-14


def test_ace_radial_is_chebyshev_times_cutoff_and_count():
    from numpy.polynomial import chebyshev
    for r in (0.0, 0.7, 2.3, 4.0, 4.66, 4.67, 5.0):
        for n in range(4):
            x = 2 * r / 4.67 - 1
            ref = chebyshev.chebval(x, [0] * n + [1]) * (0.5 * (np.cos(np.pi * r / 4.67) + 1) if r < 4.67 else 0.0)
            assert abs(oracle.ace_radial(n, r, 4.67) - ref) < 1e-14
    # count: rank 1 n, rank 2 (l, n1 <= n2), rank 3 multisets of (n, l) with even l-sum and triangle
    nmax, lmax = 4, 4
    pairs = [(n, l) for n in range(nmax) for l in range(lmax + 1)]
    n3 = sum(1 for i in range(len(pairs)) for j in range(i, len(pairs)) for k in range(j, len(pairs))
             if abs(pairs[i][1] - pairs[j][1]) <= pairs[k][1] <= pairs[i][1] + pairs[j][1]
             and (pairs[i][1] + pairs[j][1] + pairs[k][1]) % 2 == 0)
    assert oracle.ace_count(nmax, lmax) == nmax + (lmax + 1) * nmax * (nmax + 1) // 2 + n3 == 602


def _ace_index(nmax, lmax):
    """(rank, key) of every descriptor in output order."""
    out = [(1, (n,)) for n in range(nmax)]
    out += [(2, (l, n1, n2)) for l in range(lmax + 1) for n1 in range(nmax) for n2 in range(n1, nmax)]
    np_ = nmax * (lmax + 1)
    for p1 in range(np_):
        for p2 in range(p1, np_):
            for p3 in range(p2, np_):
                ls = [p % (lmax + 1) for p in (p1, p2, p3)]
                if abs(ls[0] - ls[1]) <= ls[2] <= ls[0] + ls[1] and sum(ls) % 2 == 0:
                    out.append((3, tuple((p // (lmax + 1), p % (lmax + 1)) for p in (p1, p2, p3))))
    return out


def test_ace_empty_neighbourhood_and_single_atom_closed_forms():
    """Only the grid point's own delta: A_n00 = (-1)^n / sqrt(4 pi), all other
    A vanish.  One atom at distance r besides: for l > 0 the rank-2 value is
    R_n1 R_n2 (2l+1)/(4 pi) by the addition theorem."""
    idx = _ace_index(4, 4)
    s0 = _iso_snap([[15.0, 15.0, 15.0]])
    B0 = oracle.ace(s0, 4.67, 4, 4, np.array([0]))[0]
    y00 = 1 / np.sqrt(4 * np.pi)
    for v, (rank, key) in zip(B0, idx):
        if rank == 1:
            ref = (-1) ** key[0] * y00
        elif rank == 2:
            ref = (-1) ** (key[1] + key[2]) * y00 ** 2 if key[0] == 0 else 0.0
        else:
            ref = np.prod([(-1) ** n * y00 for n, l in key]) if all(l == 0 for n, l in key) else 0.0
        assert abs(v - ref) < 1e-14
    d = np.array([1.1, -0.7, 2.0])
    s1 = _iso_snap([d])
    B1 = oracle.ace(s1, 4.67, 4, 4, np.array([0]))[0]
    r = np.linalg.norm(d)
    R = [oracle.ace_radial(n, r, 4.67) for n in range(4)]
    for v, (rank, key) in zip(B1, idx):
        if rank == 2 and key[0] > 0:
            l, n1, n2 = key
            assert abs(v - R[n1] * R[n2] * (2 * l + 1) / (4 * np.pi)) < 1e-13


def test_ace_rotation_inversion_permutation_invariance():
    rng = np.random.default_rng(21)
    pos = rng.normal(scale=1.7, size=(7, 3))
    pos = pos[np.linalg.norm(pos, axis=1) < 4.5]
    q, _ = np.linalg.qr(rng.normal(size=(3, 3)))
    B = oracle.ace(_iso_snap(pos), 4.67, 4, 4, np.array([0]))[0]
    Br = oracle.ace(_iso_snap(pos @ q.T), 4.67, 4, 4, np.array([0]))[0]
    Bi = oracle.ace(_iso_snap(-pos), 4.67, 4, 4, np.array([0]))[0]
    Bp = oracle.ace(_iso_snap(pos[::-1]), 4.67, 4, 4, np.array([0]))[0]
    sc = np.max(np.abs(B))
    assert np.max(np.abs(Br - B)) <= 1e-12 * sc
    assert np.max(np.abs(Bi - B)) <= 1e-12 * sc
    assert np.max(np.abs(Bp - B)) <= 1e-12 * sc


# ---------------------------------------------------------------- grid ACE, rank 4
def _invariant_count_by_weights(ls):
    """Independent count of the rotation invariants of a product of four
    spherical-harmonic sets in which equal (n, l) keys are the same factor:
    for the representation of the symmetrised product, the multiplicity of
    the trivial representation is (number of weight states with M = 0) -
    (number with M = 1).  The states are, per distinct key repeated k times
    with angular momentum l, the multisets of k projections in -l..l."""
    import collections
    import itertools
    total = collections.Counter({0: 1})
    for key, k in collections.Counter(ls).items():
        l = key[1]
        sums = collections.Counter(sum(c) for c in itertools.combinations_with_replacement(range(-l, l + 1), k))
        nxt = collections.Counter()
        for a, ca in total.items():
            for b, cb in sums.items():
                nxt[a + b] += ca * cb
        total = nxt
    return total[0] - total[1]


@pytest.mark.parametrize("nmax4,lmax4", [(1, 1), (1, 2), (2, 2), (3, 2), (2, 3)])
def test_ace4_set_size_equals_independent_invariant_count(nmax4, lmax4):
    """The non-redundant rank-4 set has, for every multiset of keys with an
    even l-sum, exactly as many descriptors as there are independent
    rotation invariants of that symmetrised product (counted from weights
    alone, without any coupling coefficient)."""
    import collections
    import itertools
    got = collections.Counter(d[:4] for d in oracle.ace4_set(nmax4, lmax4))
    keys = [(n, l) for n in range(nmax4) for l in range(lmax4 + 1)]
    expect = 0
    for ps in itertools.combinations_with_replacement(range(len(keys)), 4):
        ks = [keys[p] for p in ps]
        if sum(l for _, l in ks) % 2:
            continue
        c = _invariant_count_by_weights(ks)
        assert got.get(tuple(ps), 0) == c, (ps, got.get(tuple(ps), 0), c)
        expect += c
    assert len(oracle.ace4_set(nmax4, lmax4)) == expect


def test_ace4_gcg_against_sympy_cg():
    """Generalized Clebsch-Gordan coefficient of the coupling tree
    ((l1 l2) L, (l3 l4) L) -> 0 from sympy's ordinary ones."""
    from sympy.physics.quantum.cg import CG
    rng = np.random.default_rng(8)
    for _ in range(60):
        ls = rng.integers(0, 4, size=4)
        lo, hi = max(abs(ls[0] - ls[1]), abs(ls[2] - ls[3])), min(ls[0] + ls[1], ls[2] + ls[3])
        if lo > hi:
            continue
        L = int(rng.integers(lo, hi + 1))
        m = [int(rng.integers(-l, l + 1)) for l in ls[:3]]
        m.append(-sum(m))
        if abs(m[3]) > ls[3]:
            continue
        M = m[0] + m[1]
        ref = 0.0
        if abs(M) <= L:
            ref = float(CG(int(ls[0]), m[0], int(ls[1]), m[1], L, M).doit() * CG(int(ls[2]), m[2], int(ls[3]), m[3], L, -M).doit()
                        * CG(L, M, L, -M, 0, 0).doit())
        assert abs(oracle.ace_gcg4(ls, L, m) - ref) < 1e-14


def test_ace4_empty_neighbourhood_single_atom_and_L0_product():
    """No atoms: only all-l = 0 descriptors are nonzero, prod (-1)^n / (4 pi)^2.
    One atom at distance r, all l > 0: two spherical harmonics of one
    direction couple to sqrt((2a+1)(2b+1)/(4 pi (2L+1))) <a0 b0|L0> Y_L, so
    B = prod R_n c12 c34 (-1)^L sqrt(2L+1) / (4 pi).  Any point, L = 0: the
    coupling factorises into two rank-2 invariants,
    B = (-1)^(l1+l3) / sqrt((2 l1+1)(2 l3+1)) B2(p1 p2) B2(p3 p4)."""
    from sympy.physics.quantum.cg import CG
    nmax4, lmax4 = 3, 2
    desc = oracle.ace4_set(nmax4, lmax4)
    nl = lmax4 + 1
    B0 = oracle.ace4(_iso_snap([[15.0, 15.0, 15.0]]), 4.67, nmax4, lmax4, np.array([0]))[0]
    for v, d in zip(B0, desc):
        ref = np.prod([(-1) ** (p // nl) for p in d[:4]]) / (4 * np.pi) ** 2 if all(p % nl == 0 for p in d[:4]) else 0.0
        assert abs(v - ref) < 1e-15
    dvec = np.array([0.9, 1.3, -1.6])
    r = np.linalg.norm(dvec)
    R = [oracle.ace_radial(n, r, 4.67) for n in range(nmax4)]
    B1 = oracle.ace4(_iso_snap([dvec]), 4.67, nmax4, lmax4, np.array([0]))[0]
    checked = 0
    for v, d in zip(B1, desc):
        ls = [p % nl for p in d[:4]]
        if min(ls) == 0:
            continue
        L = d[4]
        c = [np.sqrt((2 * a + 1) * (2 * b + 1) / (4 * np.pi * (2 * L + 1))) * float(CG(a, 0, b, 0, L, 0).doit())
             for a, b in ((ls[0], ls[1]), (ls[2], ls[3]))]
        ref = np.prod([R[p // nl] for p in d[:4]]) * c[0] * c[1] * (-1) ** L * np.sqrt(2 * L + 1) / (4 * np.pi)
        assert abs(v - ref) < 1e-13
        checked += 1
    assert checked > 10
    rng = np.random.default_rng(4)
    pos = rng.normal(scale=1.8, size=(6, 3))
    s = _iso_snap(pos)
    B4 = oracle.ace4(s, 4.67, nmax4, lmax4, np.array([0]))[0]
    B = oracle.ace(s, 4.67, nmax4, lmax4, np.array([0]))[0]
    r2 = {}
    k = nmax4
    for l in range(lmax4 + 1):
        for n1 in range(nmax4):
            for n2 in range(n1, nmax4):
                r2[(n1 * nl + l, n2 * nl + l)] = B[k]
                k += 1
    n0 = 0
    for v, d in zip(B4, desc):
        if d[4] != 0:
            continue
        l1, l3 = d[0] % nl, d[2] % nl
        ref = (-1) ** (l1 + l3) / np.sqrt((2 * l1 + 1) * (2 * l3 + 1)) * r2[(d[0], d[1])] * r2[(d[2], d[3])]
        assert abs(v - ref) <= 1e-13 * max(1.0, abs(ref))
        n0 += 1
    assert n0 > 10


def test_ace4_rotation_inversion_permutation_invariance():
    rng = np.random.default_rng(22)
    pos = rng.normal(scale=1.7, size=(8, 3))
    pos = pos[np.linalg.norm(pos, axis=1) < 4.5]
    q, _ = np.linalg.qr(rng.normal(size=(3, 3)))
    args = (4.67, 3, 2, np.array([0]))
    B = oracle.ace4(_iso_snap(pos), *args)[0]
    Br = oracle.ace4(_iso_snap(pos @ q.T), *args)[0]
    Bi = oracle.ace4(_iso_snap(-pos), *args)[0]
    Bp = oracle.ace4(_iso_snap(pos[::-1]), *args)[0]
    sc = np.max(np.abs(B))
    assert sc > 0
    assert np.max(np.abs(Br - B)) <= 1e-12 * sc
    assert np.max(np.abs(Bi - B)) <= 1e-12 * sc
    assert np.max(np.abs(Bp - B)) <= 1e-12 * sc
