"""FP64 CPU oracle -- TEST INFRASTRUCTURE ONLY.

Python side of the plain C oracle in ``mala_oracle.c``.  Only ``tests/``,
``__graft_entry__.smoke()`` and the CPU-baseline leg of ``bench.py`` may
import this package.  The GPU library never links, loads or calls it, and
the two share no code: only the seeded inputs of ``mala_synth`` serve both.

Each function cites the passage of arXiv:2411.19617 it follows; the C file
holds the arithmetic.
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "mala_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
KB_EV = 8.617333262e-5
BISECT_TOL = 1e-12

_lib = None
_lib_path = _LIB


def build(force=True):
    """Compile the oracle with gcc (plain -O2, OpenMP over grid points)."""
    if not force and os.path.exists(_LIB):
        return _LIB
    tmp = _LIB + ".tmp"
    cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", _SRC, "-o", tmp, "-lm"]
    subprocess.check_call(cmd)
    os.replace(tmp, _LIB)
    return _LIB


def build_native(out_dir):
    """Compile a copy of the oracle tuned for the host it runs on (-O3
    -march=native; ISO C, so no contraction into FMAs: the arithmetic is the
    same as the portable build's).  Used to time the CPU baseline on the
    machine that runs the benchmark; returns the library's path."""
    path = os.path.join(out_dir, "liboracle_native.so")
    cmd = ["gcc", "-O3", "-march=native", "-std=c11", "-fopenmp", "-fPIC", "-shared", _SRC, "-o", path, "-lm"]
    subprocess.check_call(cmd)
    return path


def use_library(path):
    """Load the oracle from another build of the same source (build_native)."""
    global _lib, _lib_path
    _lib, _lib_path = None, path


def lib():
    global _lib
    if _lib is None:
        if _lib_path == _LIB and not os.path.exists(_LIB):
            build()
        L = ctypes.CDLL(_lib_path)
        d, i, i64, p = ctypes.c_double, ctypes.c_int, ctypes.c_int64, ctypes.c_void_p
        L.oracle_cg.restype = d
        L.oracle_cg.argtypes = [i] * 6
        L.oracle_cayley_klein.argtypes = [d, d, d, d, p, p, p, p]
        L.oracle_cutoff.restype = d
        L.oracle_cutoff.argtypes = [d, d]
        L.oracle_wigner_u.argtypes = [i, d, d, d, d, p]
        L.oracle_u_size.restype = i
        L.oracle_u_size.argtypes = [i]
        L.oracle_ui.argtypes = [p, i, d, i, p]
        L.oracle_n_triples.restype = i
        L.oracle_n_triples.argtypes = [i]
        L.oracle_triples.argtypes = [i, p]
        L.oracle_bispectrum.argtypes = [p, i, p, p]
        L.oracle_neighbours.restype = i
        L.oracle_neighbours.argtypes = [p, i, p, p, d, i64, p, i]
        L.oracle_descriptors.restype = i
        L.oracle_descriptors.argtypes = [p, i, p, p, d, i, p, i64, p, p, i]
        L.oracle_mlp.argtypes = [p, i64, i, p, p, p, p, p, p, p, d, i, p, i]
        L.oracle_u_adjoint.argtypes = [p, i, p, p]
        L.oracle_wigner3j.restype = d
        L.oracle_wigner3j.argtypes = [i] * 6
        L.oracle_ace_radial.restype = d
        L.oracle_ace_radial.argtypes = [i, d, d]
        L.oracle_ace_count.restype = i
        L.oracle_ace_count.argtypes = [i, i]
        L.oracle_ace.restype = i
        L.oracle_ace.argtypes = [p, i, p, p, d, i, i, p, i64, p, i]
        L.oracle_ace_gcg4.restype = d
        L.oracle_ace_gcg4.argtypes = [i] * 9
        L.oracle_ace4.restype = i
        L.oracle_ace4.argtypes = [p, i, p, p, d, i, i, p, i, p, i64, p, i]
        L.oracle_dcayley_klein.argtypes = [d, d, d, d, p, p]
        L.oracle_dcutoff.restype = d
        L.oracle_dcutoff.argtypes = [d, d]
        L.oracle_dwigner_u.argtypes = [i, d, d, d, d, d, d, d, d, p]
        L.oracle_descriptors_vjp.restype = i
        L.oracle_descriptors_vjp.argtypes = [p, i, p, p, d, i, p, i64, p, p, i]
        L.oracle_mlp_vjp.argtypes = [p, i64, i, p, p, p, p, p, p, d, i, p, p, p, i]
        L.oracle_dos.argtypes = [p, i64, i, d, p]
        L.oracle_li_neg.restype = d
        L.oracle_li_neg.argtypes = [i, d]
        L.oracle_fermi_weights.argtypes = [d, d, i, d, d, p, p]
        L.oracle_entropy_weights.argtypes = [d, d, i, d, d, p]
        L.oracle_gaussian.argtypes = [p, i, p, p, d, d, p, i64, p, i]
        L.oracle_entropy.restype = d
        L.oracle_entropy.argtypes = [p, d, d, i, d, d, p]
        L.oracle_fermi.restype = i
        L.oracle_fermi.argtypes = [p, d, d, i, d, d, d, p, p]
        L.oracle_density.argtypes = [p, i64, i, p, p]
        _lib = L
    return _lib


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


# ------------------------------------------------------------------ pieces

def cg(j1, m1, j2, m2, j, m):
    """<j1 m1 j2 m2 | j m>, all arguments doubled (Racah closed form)."""
    return lib().oracle_cg(j1, m1, j2, m2, j, m)


def cayley_klein(d, rcut):
    """(a, b) of g = exp(-i theta0 n.sigma), theta0 = 0.99363 pi r / rcut."""
    out = [ctypes.c_double() for _ in range(4)]
    lib().oracle_cayley_klein(float(d[0]), float(d[1]), float(d[2]), float(rcut),
                              *[ctypes.byref(o) for o in out])
    return complex(out[0].value, out[1].value), complex(out[2].value, out[3].value)


def cutoff(r, rcut):
    return lib().oracle_cutoff(float(r), float(rcut))


def wigner_u(J, a, b):
    """(J+1)x(J+1) complex spin-J/2 representation of [[a, b], [-b*, a*]]."""
    out = np.zeros((J + 1) * (J + 1) * 2)
    lib().oracle_wigner_u(J, a.real, a.imag, b.real, b.imag, _ptr(out))
    return (out[0::2] + 1j * out[1::2]).reshape(J + 1, J + 1)


def u_levels(disp, rcut, twojmax):
    """List of u^J matrices (J = 0..twojmax) for one grid point (Eq. SNAPExpansion)."""
    disp = _f64(disp).reshape(-1, 3)
    size = lib().oracle_u_size(twojmax)
    u = np.zeros(2 * size)
    lib().oracle_ui(_ptr(disp), disp.shape[0], float(rcut), twojmax, _ptr(u))
    u = u[0::2] + 1j * u[1::2]
    out, o = [], 0
    for J in range(twojmax + 1):
        out.append(u[o:o + (J + 1) ** 2].reshape(J + 1, J + 1))
        o += (J + 1) ** 2
    return out


def triples(twojmax):
    n = lib().oracle_n_triples(twojmax)
    t = np.zeros(3 * n, dtype=np.int32)
    lib().oracle_triples(twojmax, _ptr(t))
    return t.reshape(n, 3)


def bispectrum_from_u(u_list, twojmax):
    """B(j1,j2,j) from a list of u^J matrices; returns (B, max |Im|)."""
    flat = np.concatenate([np.asarray(m, complex).reshape(-1) for m in u_list])
    buf = np.empty(2 * flat.size)
    buf[0::2], buf[1::2] = flat.real, flat.imag
    n = lib().oracle_n_triples(twojmax)
    B = np.zeros(n)
    mi = ctypes.c_double()
    lib().oracle_bispectrum(_ptr(buf), twojmax, _ptr(B), ctypes.byref(mi))
    return B, mi.value


def bispectrum_from_disp(disp, rcut, twojmax):
    """B for one grid point given its neighbour vectors (neighbour - point)."""
    return bispectrum_from_u(u_levels(disp, rcut, twojmax), twojmax)


def neighbours(snap, p, max_nbr=4096):
    pos = _f64(snap.positions)
    L = _f64(snap.L)
    N = np.ascontiguousarray(snap.N, dtype=np.int32)
    disp = np.zeros(3 * max_nbr)
    c = lib().oracle_neighbours(_ptr(pos), pos.shape[0], _ptr(L), _ptr(N), float(snap.rcut),
                                int(p), _ptr(disp), max_nbr)
    return disp[:3 * min(c, max_nbr)].reshape(-1, 3)


def descriptors(snap, points=None, nthreads=0, return_meta=False):
    """B[n_pts][n_B] (float64) at flat grid indices `points` (default: all)."""
    if points is None:
        points = np.arange(snap.n_points, dtype=np.int64)
    pts = np.ascontiguousarray(points, dtype=np.int64)
    pos = _f64(snap.positions)
    L = _f64(snap.L)
    N = np.ascontiguousarray(snap.N, dtype=np.int32)
    nt = lib().oracle_n_triples(snap.twojmax)
    B = np.zeros((pts.shape[0], nt))
    mi = ctypes.c_double()
    worst = lib().oracle_descriptors(_ptr(pos), pos.shape[0], _ptr(L), _ptr(N),
                                     float(snap.rcut), int(snap.twojmax), _ptr(pts),
                                     pts.shape[0], _ptr(B), ctypes.byref(mi), int(nthreads))
    if worst < 0:
        raise RuntimeError("oracle neighbour list overflow")
    if return_meta:
        return B, {"max_neighbours": worst, "max_imag": mi.value}
    return B


def descriptors_vjp(snap, gB, points=None, nthreads=0):
    """dL/dR [n_atoms][3] for L = sum_p sum_l gB[p][l] B_l(p) over the grid
    points `points` (default: all): the descriptor factor of the force
    expression (Eq. forcesmala) applied to gB [n_pts][n_B]."""
    if points is None:
        points = np.arange(snap.n_points, dtype=np.int64)
    pts = np.ascontiguousarray(points, dtype=np.int64)
    L = _f64(snap.L)
    pos = _f64(np.mod(snap.positions, L))
    N = np.ascontiguousarray(snap.N, dtype=np.int32)
    gB = _f64(gB)
    assert gB.shape == (pts.shape[0], lib().oracle_n_triples(snap.twojmax))
    out = np.zeros((pos.shape[0], 3))
    if lib().oracle_descriptors_vjp(_ptr(pos), pos.shape[0], _ptr(L), _ptr(N), float(snap.rcut),
                                    int(snap.twojmax), _ptr(pts), pts.shape[0], _ptr(gB), _ptr(out),
                                    int(nthreads)) < 0:
        raise RuntimeError("oracle neighbour list overflow")
    return out


class _Cplx(ctypes.Structure):
    _fields_ = [("re", ctypes.c_double), ("im", ctypes.c_double)]


def ylm(l, m, d):
    """Orthonormal complex spherical harmonic Y_l^m of the direction d (Condon-Shortley)."""
    f = lib().oracle_ylm
    f.restype = _Cplx
    f.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_double]
    v = f(int(l), int(m), float(d[0]), float(d[1]), float(d[2]))
    return complex(v.re, v.im)


def wigner3j(l1, l2, l3, m1, m2, m3):
    return lib().oracle_wigner3j(l1, l2, l3, m1, m2, m3)


def ace_radial(n, r, rcut):
    return lib().oracle_ace_radial(int(n), float(r), float(rcut))


def ace_count(nmax, lmax):
    return lib().oracle_ace_count(int(nmax), int(lmax))


def ace_gcg4(l, L, m):
    """Generalized Clebsch-Gordan coefficient of four angular momenta l with
    the intermediate coupling L ((l1 l2) L, (l3 l4) L -> 0) at projections m."""
    return lib().oracle_ace_gcg4(*[int(x) for x in l], int(L), *[int(x) for x in m])


def ace4_set(nmax4, lmax4, tol=1e-9):
    """Rank-4 grid ACE descriptors (Eq. ace_grid with four factors), one element:
    multisets of four keys p = n (lmax4+1) + l (n < nmax4, l <= lmax4),
    p1 <= p2 <= p3 <= p4, with l1+l2+l3+l4 even (real and parity-even), each
    coupled as ((p1 p2) L, (p3 p4) L) for every L allowed by both triangles.
    Where keys repeat, the A's of equal keys are the same numbers, so a
    coupling defines the invariant of its coefficients summed over the
    permutations that exchange equal keys; for each multiset the couplings are
    taken in increasing L and kept when that invariant is linearly independent
    of the ones kept before it (the paper requires the rank >= 4 set to be
    free of redundant descriptors).  Returns [(p1, p2, p3, p4, L), ...] in
    output order."""
    import itertools
    nk = nmax4 * (lmax4 + 1)
    out = []
    for ps in itertools.combinations_with_replacement(range(nk), 4):
        ls = [p % (lmax4 + 1) for p in ps]
        if sum(ls) % 2:
            continue
        perms = [q for q in itertools.permutations(range(4)) if all(ps[q[i]] == ps[i] for i in range(4))]
        kept = []
        for L in range(max(abs(ls[0] - ls[1]), abs(ls[2] - ls[3])), min(ls[0] + ls[1], ls[2] + ls[3]) + 1):
            T = np.zeros([2 * l + 1 for l in ls])
            for m1 in range(-ls[0], ls[0] + 1):
                for m2 in range(-ls[1], ls[1] + 1):
                    for m3 in range(-ls[2], ls[2] + 1):
                        m4 = -m1 - m2 - m3
                        if abs(m4) <= ls[3]:
                            T[m1 + ls[0], m2 + ls[1], m3 + ls[2], m4 + ls[3]] = ace_gcg4(ls, L, (m1, m2, m3, m4))
            v = sum(np.transpose(T, q) for q in perms).ravel() / len(perms)
            M = np.array(kept + [v])
            sv = np.linalg.svd(M, compute_uv=False)
            if np.sum(sv > tol * max(1.0, sv[0])) > len(kept):
                kept.append(v)
                out.append(tuple(ps) + (L,))
    return out


def ace4(snap, rcut, nmax4, lmax4, points=None, nthreads=0):
    """Rank-4 grid ACE descriptors [n_pts][len(ace4_set)] (one element)."""
    desc = np.ascontiguousarray(np.array(ace4_set(nmax4, lmax4), dtype=np.int32).reshape(-1, 5))
    if points is None:
        points = np.arange(snap.n_points, dtype=np.int64)
    pts = np.ascontiguousarray(points, dtype=np.int64)
    L = _f64(snap.L)
    pos = _f64(np.mod(snap.positions, L))
    N = np.ascontiguousarray(snap.N, dtype=np.int32)
    out = np.zeros((pts.shape[0], desc.shape[0]))
    if desc.shape[0] and lib().oracle_ace4(_ptr(pos), pos.shape[0], _ptr(L), _ptr(N), float(rcut), int(nmax4),
                                           int(lmax4), _ptr(desc), desc.shape[0], _ptr(pts), pts.shape[0],
                                           _ptr(out), int(nthreads)) < 0:
        raise RuntimeError("oracle neighbour list overflow")
    return out


def ace(snap, rcut, nmax, lmax, points=None, nthreads=0):
    """Grid ACE descriptors [n_pts][ace_count] (ranks 1-3, one element)."""
    if points is None:
        points = np.arange(snap.n_points, dtype=np.int64)
    pts = np.ascontiguousarray(points, dtype=np.int64)
    L = _f64(snap.L)
    pos = _f64(np.mod(snap.positions, L))
    N = np.ascontiguousarray(snap.N, dtype=np.int32)
    out = np.zeros((pts.shape[0], ace_count(nmax, lmax)))
    if lib().oracle_ace(_ptr(pos), pos.shape[0], _ptr(L), _ptr(N), float(rcut), int(nmax), int(lmax), _ptr(pts),
                        pts.shape[0], _ptr(out), int(nthreads)) < 0:
        raise RuntimeError("oracle neighbour list overflow")
    return out


def u_adjoint(u_full, twojmax, gB):
    """Y = dL/du (Y = dL/dRe u + i dL/dIm u) for L = sum_l gB_l B_l(u), all rows
    of every level, packed like u_levels' concatenation."""
    u = _f64(np.stack([np.real(u_full), np.imag(u_full)], -1))
    Y = np.zeros_like(u)
    lib().oracle_u_adjoint(_ptr(u), int(twojmax), _ptr(_f64(gB)), _ptr(Y))
    return Y[..., 0] + 1j * Y[..., 1]


def gaussian(snap, sigma, cutoff, points=None, nthreads=0):
    """Gaussian descriptors G(r) (normalised Gaussians on every atom image within
    the cutoff) at flat grid indices `points` (default: all)."""
    if points is None:
        points = np.arange(snap.n_points, dtype=np.int64)
    pts = np.ascontiguousarray(points, dtype=np.int64)
    pos = _f64(snap.positions)
    L = _f64(snap.L)
    N = np.ascontiguousarray(snap.N, dtype=np.int32)
    out = np.zeros(pts.shape[0])
    lib().oracle_gaussian(_ptr(pos), pos.shape[0], _ptr(L), _ptr(N), float(sigma), float(cutoff),
                          _ptr(pts), pts.shape[0], _ptr(out), int(nthreads))
    return out


def mlp(B, net, nthreads=0):
    """LDOS[n][n_e] = out_scale * net((B - mean)/std) + out_shift (Eq. ffnn)."""
    B = _f64(B)
    n = B.shape[0]
    widths = np.ascontiguousarray(net["widths"], dtype=np.int32)
    Wcat = np.concatenate([_f64(w).reshape(-1) for w in net["W"]])
    bcat = np.concatenate([_f64(b) for b in net["b"]])
    out = np.zeros((n, widths[-1]))
    lib().oracle_mlp(_ptr(B), n, len(widths) - 1, _ptr(widths), _ptr(Wcat), _ptr(bcat),
                     _ptr(_f64(net["in_mean"])), _ptr(_f64(net["in_std"])),
                     _ptr(_f64(net["out_scale"])), _ptr(_f64(net["out_shift"])),
                     float(net["slope"]), int(net["output_activation"]), _ptr(out), int(nthreads))
    return out


def mlp_vjp(B, net, v, nthreads=0):
    """g(p) = (dd(p)/dB(p))^T v(p): the network factor of the force expression
    (Eq. forcesmala) applied to v [n][n_e] by backpropagation in FP64.
    Returns (g [n][n_in], margin [n]); margin is each point's smallest
    |z| / (|b| + sum |W x|) over the units that pass through the activation
    (its distance from a kink of the piecewise-linear network)."""
    B = _f64(B)
    n = B.shape[0]
    widths = np.ascontiguousarray(net["widths"], dtype=np.int32)
    v = _f64(v)
    assert v.shape == (n, widths[-1])
    Wcat = np.concatenate([_f64(w).reshape(-1) for w in net["W"]])
    bcat = np.concatenate([_f64(b) for b in net["b"]])
    g = np.zeros((n, widths[0]))
    margin = np.zeros(n)
    lib().oracle_mlp_vjp(_ptr(B), n, len(widths) - 1, _ptr(widths), _ptr(Wcat), _ptr(bcat),
                         _ptr(_f64(net["in_mean"])), _ptr(_f64(net["in_std"])), _ptr(_f64(net["out_scale"])),
                         float(net["slope"]), int(net["output_activation"]), _ptr(v), _ptr(g), _ptr(margin),
                         int(nthreads))
    return g, margin


def dos(ldos, dV):
    """D_e = dV * sum_p d_e(p) (Eq. DOS.from.ldos)."""
    ldos = _f64(ldos)
    out = np.zeros(ldos.shape[1])
    lib().oracle_dos(_ptr(ldos), ldos.shape[0], ldos.shape[1], float(dV), _ptr(out))
    return out


def li_neg(s, y):
    """Li_s(-y), 0 <= y <= 1 (s >= 1)."""
    return lib().oracle_li_neg(int(s), float(y))


def fermi_weights(egrid, mu, T):
    """(w, v): int f D = w.D and int f e D = v.D for piecewise-linear D (Sec. 3.4)."""
    e0, de, n = egrid
    w, v = np.zeros(n), np.zeros(n)
    lib().oracle_fermi_weights(float(e0), float(de), int(n), float(mu), KB_EV * float(T),
                               _ptr(w), _ptr(v))
    return w, v


def entropy_weights(egrid, mu, T):
    """u with S_s / k_B = u.D for piecewise-linear D (Eq. electronicentropyDOS)."""
    e0, de, n = egrid
    u = np.zeros(n)
    lib().oracle_entropy_weights(float(e0), float(de), int(n), float(mu), KB_EV * float(T), _ptr(u))
    return u


def entropy(dos_, egrid, mu, T):
    """(S_s / k_B, -tau S_s in eV) at Fermi level mu (Eqs. electronicentropyDOS, KSfreeenergy)."""
    e0, de, n = egrid
    d = _f64(dos_)
    mts = ctypes.c_double()
    s = lib().oracle_entropy(_ptr(d), float(e0), float(de), int(n), float(T), float(mu), ctypes.byref(mts))
    return s, mts.value


class NoRoot(Exception):
    pass


def fermi(dos_, egrid, T, n_electrons, tol=BISECT_TOL):
    """E_F by bisection, band energy, N(E_F), iterations and final weights."""
    e0, de, n = egrid
    dos_ = _f64(dos_)
    res = np.zeros(4)
    w = np.zeros(n)
    st = lib().oracle_fermi(_ptr(dos_), float(e0), float(de), int(n), float(T),
                            float(n_electrons), float(tol), _ptr(res), _ptr(w))
    if st != 0:
        raise NoRoot("N_e outside the attainable range")
    return {"e_fermi": res[0], "e_band": res[1], "n_found": res[2], "iters": int(res[3]),
            "weights": w}


def density(ldos, w):
    """n(p) = sum_e w_e d_e(p) (Eq. density.from.ldos)."""
    ldos = _f64(ldos)
    out = np.zeros(ldos.shape[0])
    lib().oracle_density(_ptr(ldos), ldos.shape[0], ldos.shape[1], _ptr(_f64(w)), _ptr(out))
    return out


def predict(snap, net, egrid, points=None, nthreads=0):
    """Whole path on the listed points (all points by default): B, LDOS, DOS, E_F,
    E_band, the entropy term and density.  DOS/E_F/E_band are only meaningful over all points."""
    B = descriptors(snap, points, nthreads)
    ld = mlp(B, net, nthreads)
    D = dos(ld, snap.dV)
    fr = fermi(D, egrid, snap.T, snap.n_electrons)
    s_kb, mts = entropy(D, egrid, fr["e_fermi"], snap.T)
    return {"B": B, "ldos": ld, "dos": D, "e_fermi": fr["e_fermi"], "e_band": fr["e_band"],
            "n_found": fr["n_found"], "iters": fr["iters"], "weights": fr["weights"],
            "entropy": s_kb, "minus_ts": mts, "density": density(ld, fr["weights"])}
