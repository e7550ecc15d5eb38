"""Seeded synthetic inputs shared by the GPU path and the oracle.

This module only *generates inputs*: atomic snapshots (positions, periodic
cell, real-space grid, temperature, electron count), the energy grid and a
seeded random network with its input/output scalers.  It contains none of
the method's arithmetic (no descriptors, no network evaluation, no energy
integration).  Every draw comes from SplitMix64 with a fixed seed, so the two
sides see bit-identical inputs.

Workload shapes follow the paper's aluminium / beryllium experiments
(Sec. 5.2 and its tables: 256 atoms at a few thousand grid points per atom,
solid and liquid Al between 298 K and 933 K, a 16,384-atom entry and a
stacking-fault slab).  None of the paper's DFT data is reproduced; the
structures are generated here from crystallography (fcc Al, a = 4.05 A).
"""
from dataclasses import dataclass, field
import os
import struct

import numpy as np
from scipy.spatial import cKDTree

from .rng import SplitMix64

A_AL = 4.05                       # fcc Al lattice constant, Angstrom
E_PER_ATOM = 3                    # valence electrons per Al atom
RCUT = 4.67                       # descriptor cutoff radius, Angstrom
EGRID = (-5.0, 0.1, 250)          # energy grid: offset, spacing (eV), size
_DATA = os.path.join(os.path.dirname(os.path.abspath(__file__)), "data")


@dataclass
class Snapshot:
    name: str
    positions: np.ndarray         # [n_atoms, 3] float64, Angstrom, in [0, L)
    L: np.ndarray                 # [3] orthorhombic cell edges, Angstrom
    N: np.ndarray                 # [3] grid points per edge (int)
    rcut: float
    twojmax: int
    T: float                      # electronic temperature, K
    n_electrons: float
    meta: dict = field(default_factory=dict)

    @property
    def n_atoms(self):
        return int(self.positions.shape[0])

    @property
    def n_points(self):
        return int(np.prod(self.N))

    @property
    def dV(self):
        return float(np.prod(self.L) / np.prod(self.N))


# ----------------------------------------------------------------- structures

def fcc_cubic(n, a=A_AL):
    """n x n x n conventional fcc cells: 4 n^3 atoms in an n a cube."""
    basis = np.array([[0, 0, 0], [0.5, 0.5, 0], [0.5, 0, 0.5], [0, 0.5, 0.5]])
    cells = np.array([[i, j, k] for i in range(n) for j in range(n) for k in range(n)], float)
    pos = (cells[:, None, :] + basis[None, :, :]).reshape(-1, 3) * a
    return pos, np.array([n * a] * 3)


def jitter(pos, L, sigma, rng):
    """i.i.d. N(0, sigma^2) displacement per Cartesian coordinate, wrapped."""
    p = pos + sigma * rng.normal(pos.size).reshape(pos.shape)
    return np.mod(p, L)


def liquid_rsa(n_atoms, L, dmin, rng, max_tries=2_000_000, batch=256):
    """Random sequential packing with a periodic minimum-image distance >= dmin.

    Candidates are uniform points drawn in order; each is accepted if it is at
    least dmin from every atom accepted before it.  Candidates are drawn and
    screened in batches (vectorised against the atoms placed before the batch,
    then one by one against those accepted inside it), which gives the same
    decisions as testing them one at a time.
    """
    pos = np.empty((n_atoms, 3))
    k = 0
    tries = 0
    d2 = dmin * dmin
    while k < n_atoms:
        if tries >= max_tries:
            raise RuntimeError("random packing did not converge")
        m = min(batch, max_tries - tries)
        cand = rng.uniform(3 * m).reshape(m, 3) * L
        tries += m
        if k:
            # nearest placed atom (periodic) per candidate
            box = np.broadcast_to(np.asarray(L, float), (3,))
            tree = cKDTree(np.mod(pos[:k], box), boxsize=box)
            dist, _ = tree.query(np.mod(cand, box), k=1)
            ok = dist * dist >= d2
        else:
            ok = np.ones(m, bool)
        start = k
        for i in np.nonzero(ok)[0]:
            c = cand[i]
            if k > start:
                e = pos[start:k] - c
                e -= L * np.round(e / L)
                if np.min(np.einsum("ij,ij->i", e, e)) < d2:
                    continue
            pos[k] = c
            k += 1
            if k == n_atoms:
                break
    return pos


def slab_111_fault(nx=16, ny=16, n_layers=32, a=A_AL, vacuum=10.0, fault_at=16):
    """fcc(111) slab in a rectangular in-plane cell with an intrinsic fault.

    In-plane: 2 atoms per (d, sqrt(3) d) rectangle, d = a/sqrt(2).  Layers are
    a/sqrt(3) apart; layer i is stacked A,B,C by i mod 3 below `fault_at` and
    by (i+1) mod 3 from there on, which removes one layer from the ABC
    sequence (intrinsic stacking fault).  `vacuum` Angstrom on both sides.
    """
    d = a / np.sqrt(2.0)
    dz = a / np.sqrt(3.0)
    Lx, Ly = nx * d, ny * np.sqrt(3.0) * d
    thick = (n_layers - 1) * dz
    Lz = thick + 2.0 * vacuum
    base = []
    for i in range(nx):
        for j in range(ny):
            base.append((i * d, j * np.sqrt(3.0) * d))
            base.append((i * d + d / 2, j * np.sqrt(3.0) * d + np.sqrt(3.0) * d / 2))
    base = np.array(base)
    shift = [np.array([0.0, 0.0]), np.array([d / 2, d / (2 * np.sqrt(3.0))]),
             np.array([d, d / np.sqrt(3.0)])]
    layers = []
    for i in range(n_layers):
        s = i % 3 if i < fault_at else (i + 1) % 3
        xy = np.mod(base + shift[s], [Lx, Ly])
        z = np.full((xy.shape[0], 1), vacuum + i * dz)
        layers.append(np.hstack([xy, z]))
    return np.vstack(layers), np.array([Lx, Ly, Lz])


# ----------------------------------------------------------------- snapshots

def small(seed=1):
    """32-atom jittered fcc Al (2x2x2), 20^3 grid, twojmax 8, 298 K."""
    rng = SplitMix64(seed)
    pos, L = fcc_cubic(2)
    pos = jitter(pos, L, 0.1, rng)
    return Snapshot("al32_solid_298K_20c_tj8", pos, L, np.array([20, 20, 20]), RCUT, 8,
                    298.0, E_PER_ATOM * 32.0, {"seed": seed})


def paper_solid(seed=2, grid=90):
    """256-atom jittered fcc Al (4x4x4, 16.2 A cube), grid^3, twojmax 10, 298 K."""
    rng = SplitMix64(seed)
    pos, L = fcc_cubic(4)
    pos = jitter(pos, L, 0.1, rng)
    return Snapshot("al256_solid_298K_%dc_tj10" % grid, pos, L, np.array([grid] * 3), RCUT, 10,
                    298.0, E_PER_ATOM * 256.0, {"seed": seed})


def paper_liquid(seed=3, grid=90, n_atoms=256, density_gcc=2.4):
    """256-atom random packing (dmin 2.2 A) at 2.4 g/cc, grid^3, twojmax 10, 933 K."""
    rng = SplitMix64(seed)
    n_per_A3 = density_gcc / 26.9815385 * 6.02214076e23 * 1e-24
    L = (n_atoms / n_per_A3) ** (1.0 / 3.0)
    pos = liquid_rsa(n_atoms, L, 2.2, rng)
    return Snapshot("al256_liquid_933K_%dc_tj10" % grid, pos, np.array([L] * 3),
                    np.array([grid] * 3), RCUT, 10, 933.0, E_PER_ATOM * float(n_atoms),
                    {"seed": seed})


def slab(seed=4, grid=(238, 412, 480)):
    """16,384-atom fcc(111) slab with an intrinsic fault, 10 A vacuum per side."""
    rng = SplitMix64(seed)
    pos, L = slab_111_fault()
    pos = jitter(pos, L, 0.1, rng)
    return Snapshot("al16384_slab111_fault_298K_tj10", pos, L, np.array(grid), RCUT, 10,
                    298.0, E_PER_ATOM * float(pos.shape[0]), {"seed": seed})


def serving_request(rng, pts_per_atom=2800.0):
    """One request of the serving mix: fcc n^3*4 (n=2..8) or liquid N~U[32,2048]."""
    T = float(rng.uniform_range(1, 298.0, 933.0)[0])
    if rng.uniform(1)[0] < 0.5:
        n = 2 + int(rng.uniform(1)[0] * 7)
        pos, L = fcc_cubic(n)
        pos = jitter(pos, L, 0.1 * np.sqrt(T / 298.0), rng)
        kind = "fcc%d" % n
    else:
        n_at = 32 + int(rng.uniform(1)[0] * (2048 - 32 + 1))
        n_per_A3 = 2.4 / 26.9815385 * 6.02214076e23 * 1e-24
        Lc = (n_at / n_per_A3) ** (1.0 / 3.0)
        pos = liquid_rsa(n_at, Lc, 2.2, rng)
        L = np.array([Lc] * 3)
        kind = "liq%d" % n_at
    V = float(np.prod(L))
    h = (V / (pts_per_atom * pos.shape[0])) ** (1.0 / 3.0)
    N = np.maximum(np.round(L / h).astype(int), 4)
    return Snapshot("serve_%s_%.0fK" % (kind, T), pos, L, N, RCUT, 10, T,
                    E_PER_ATOM * float(pos.shape[0]), {})


def _mix_request(args):
    seed, i = args
    return serving_request(SplitMix64(seed * 1_000_003 + i))


def serving_mix(n_requests, seed=5, workers=16):
    """The serving mix: request i is drawn from its own SplitMix64 stream
    seeded with seed * 1,000,003 + i, so any request can be regenerated alone
    and the mix is generated in a pool of spawned worker processes."""
    jobs = [(seed, i) for i in range(n_requests)]
    if workers <= 1 or n_requests < 8:
        return [_mix_request(j) for j in jobs]
    import multiprocessing as mp
    with mp.get_context("spawn").Pool(min(workers, n_requests)) as pool:
        return pool.map(_mix_request, jobs, chunksize=4)


def with_grid(snap, N):
    """Same atoms on another grid (used for reduced-size parity cases)."""
    return Snapshot(snap.name + "_g%dx%dx%d" % tuple(N), snap.positions, snap.L,
                    np.array(N), snap.rcut, snap.twojmax, snap.T, snap.n_electrons,
                    dict(snap.meta))


# ----------------------------------------------------------------- network

def load_input_scaler(twojmax):
    """Per-component mean and std of B on the calibration snapshot."""
    path = os.path.join(_DATA, "input_scaler_tj%d.txt" % twojmax)
    a = np.loadtxt(path, comments="#", ndmin=2)
    return a[:, 0].copy(), a[:, 1].copy()


def output_scaler(egrid=EGRID, eb=-5.5, scale=0.1):
    """Affine LDOS output transform d = s*y + c, c = A sqrt(e - eb), s = scale*c.

    A makes c integrate to 3 electrons per 16.61 A^3 (fcc Al) at 6.2 eV.
    Units: LDOS in 1/(eV A^3).
    """
    e0, de, n = egrid
    e = e0 + de * np.arange(n)
    A = 3.0 / (16.61 * (2.0 / 3.0) * 11.7 ** 1.5)
    c = A * np.sqrt(e - eb)
    return scale * c, c


def make_net(widths, seed, twojmax, output_activation=1, slope=0.01, egrid=EGRID,
             with_input_scaler=True):
    """Seeded Xavier-uniform weights (rounded to fp32 values) and U(+-0.1) biases.

    Returns a dict: widths, W (list of [out][in] float64), b, in_mean, in_std,
    out_scale, out_shift, slope, output_activation, seed.
    """
    rng = SplitMix64(seed)
    W, b = [], []
    for l in range(len(widths) - 1):
        fin, fout = widths[l], widths[l + 1]
        lim = np.sqrt(6.0 / (fin + fout))
        w = rng.uniform_range(fin * fout, -lim, lim).reshape(fout, fin)
        W.append(w.astype(np.float32).astype(np.float64))
        b.append(rng.uniform_range(fout, -0.1, 0.1).astype(np.float32).astype(np.float64))
    if with_input_scaler:
        mu, sd = load_input_scaler(twojmax)
        assert mu.shape[0] == widths[0]
    else:
        mu, sd = np.zeros(widths[0]), np.ones(widths[0])
    s, c = output_scaler(egrid)
    assert s.shape[0] == widths[-1]
    return {"widths": list(widths), "W": W, "b": b, "in_mean": mu, "in_std": sd,
            "out_scale": s, "out_shift": c, "slope": float(slope),
            "output_activation": int(output_activation), "seed": int(seed)}


def small_net():
    return make_net([55, 100, 100, 250], 101, 8)


def paper_net():
    return make_net([91, 400, 400, 250], 102, 10)


def network_inputs(net, n, seed):
    """Seeded descriptor rows around the net's input scaler (x0 ~ N(0, 1)) and
    a vector over the energies ~ N(0, 1), both float32 [n][w0] and [n][wL]."""
    rng = np.random.default_rng(seed)
    w = net["widths"]
    B = (net["in_mean"] + net["in_std"] * rng.standard_normal((n, w[0]))).astype(np.float32)
    v = rng.standard_normal((n, w[-1])).astype(np.float32)
    return B, v


BLOB_MAGIC = b"MALANET1"


def net_to_blob(net):
    """Serialise a net dict into the little-endian weights blob of include/mala.h."""
    w = net["widths"]
    nl = len(w) - 1
    out = bytearray()
    out += BLOB_MAGIC
    out += struct.pack("<iiii", 1, nl, int(net["output_activation"]), 0)
    out += struct.pack("<d", float(net["slope"]))
    out += struct.pack("<%di" % (nl + 1), *w)
    if (nl + 1) % 2:
        out += struct.pack("<i", 0)
    out += np.asarray(net["in_mean"], "<f8").tobytes()
    out += np.asarray(net["in_std"], "<f8").tobytes()
    for l in range(nl):
        out += np.asarray(net["W"][l], "<f8").reshape(-1).tobytes()
        out += np.asarray(net["b"][l], "<f8").tobytes()
    out += np.asarray(net["out_scale"], "<f8").tobytes()
    out += np.asarray(net["out_shift"], "<f8").tobytes()
    out += struct.pack("<Q", int(net["seed"]))
    return bytes(out)


def strided_points(n_total, stride, offset=0):
    """Systematic sample of flat grid indices: offset, offset + stride, ..."""
    return np.arange(offset, n_total, stride, dtype=np.int64)


SLAB_SAMPLE = (719, 11)     # stride and offset of the slab's systematic sample (65,462 points)


def sample_points(n_total, n_sample, seed):
    """Seeded sorted sample of distinct flat grid indices."""
    rng = SplitMix64(seed)
    if n_sample >= n_total:
        return np.arange(n_total, dtype=np.int64)
    keys = rng.next_u64(n_total) if n_total <= 5_000_000 else None
    if keys is not None:
        return np.sort(np.argsort(keys)[:n_sample]).astype(np.int64)
    picked = set()
    while len(picked) < n_sample:
        for v in (rng.next_u64(n_sample) % np.uint64(n_total)):
            picked.add(int(v))
            if len(picked) == n_sample:
                break
    return np.array(sorted(picked), dtype=np.int64)
