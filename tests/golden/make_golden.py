"""Write full-grid expected values with the FP64 oracle (calls only oracle/).

Full-grid quantities (DOS, Fermi level, band energy, the integrated density)
need every grid point, which the oracle takes minutes to hours to compute,
so they are computed once here and stored as JSON next to this script.
Per-point quantities (B, LDOS, density at sampled points) are recomputed by
the tests directly, because the oracle finishes those in seconds.

The 47,066,880-point slab is too large for the oracle's whole grid; its file
(full_slab_sample.json) holds the oracle's path over a systematic sample of
every 719th point instead: the sample's DOS with the true volume element
dV (for parity with the GPU on the same points) and the whole-grid estimate
scaled by the stride, with the Fermi level, band energy and entropy of both.

Usage (from the repository root):
    python -m tests.golden.make_golden paper_solid paper_liquid small slab_sample [--threads N]
    python -m tests.golden.make_golden --derived paper_solid paper_liquid small

--derived recomputes only the quantities that follow from the stored oracle
DOS and Fermi level (the electronic entropy), without the descriptor pass.
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import mala_synth  # noqa: E402
import oracle  # noqa: E402

CASES = {
    "small": (mala_synth.small, mala_synth.small_net),
    "paper_solid": (mala_synth.paper_solid, mala_synth.paper_net),
    "paper_liquid": (mala_synth.paper_liquid, mala_synth.paper_net),
    "slab_sample": (mala_synth.slab, mala_synth.paper_net),
}


def fingerprint(snap, net):
    h = hashlib.sha256()
    h.update(np.ascontiguousarray(snap.positions).tobytes())
    h.update(np.asarray(snap.L, float).tobytes())
    h.update(np.asarray(snap.N, np.int64).tobytes())
    h.update(mala_synth.net_to_blob(net))
    return h.hexdigest()[:16]


def run(case, threads):
    snap, net = CASES[case][0](), CASES[case][1]()
    t0 = time.time()
    B = oracle.descriptors(snap, nthreads=threads)
    t1 = time.time()
    ld = oracle.mlp(B, net, nthreads=threads)
    del B
    D = oracle.dos(ld, snap.dV)
    fr = oracle.fermi(D, mala_synth.EGRID, snap.T, snap.n_electrons)
    dens = oracle.density(ld, fr["weights"])
    s_kb, minus_ts = oracle.entropy(D, mala_synth.EGRID, fr["e_fermi"], snap.T)
    out = {
        "case": case, "snapshot": snap.name, "fingerprint": fingerprint(snap, net),
        "n_points": snap.n_points, "n_atoms": snap.n_atoms, "dV": snap.dV,
        "T": snap.T, "n_electrons": snap.n_electrons, "egrid": list(mala_synth.EGRID),
        "dos": [float(x) for x in D], "e_fermi": fr["e_fermi"], "e_band": fr["e_band"],
        "n_found": fr["n_found"], "iters": fr["iters"],
        "entropy_kb": s_kb, "minus_ts": minus_ts,
        "density_sum_dV": float(dens.sum() * snap.dV),
        "density_min": float(dens.min()), "density_max": float(dens.max()),
        "oracle_seconds": time.time() - t0, "descriptor_seconds": t1 - t0, "threads": threads,
    }
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "full_%s.json" % case)
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print(case, "E_F", fr["e_fermi"], "E_b", fr["e_band"], "%.0fs" % (time.time() - t0), flush=True)


def run_slab_sample(threads):
    snap, net = mala_synth.slab(), mala_synth.paper_net()
    stride, offset = mala_synth.SLAB_SAMPLE
    pts = mala_synth.strided_points(snap.n_points, stride, offset)
    t0 = time.time()
    B, meta = oracle.descriptors(snap, pts, nthreads=threads, return_meta=True)
    nbr = [len(oracle.neighbours(snap, int(p))) for p in pts[::64]]
    ld = oracle.mlp(B, net, nthreads=threads)
    del B
    eg = mala_synth.EGRID
    frac = len(pts) / snap.n_points
    D_sample = oracle.dos(ld, snap.dV)                 # the sample's own DOS
    fr_s = oracle.fermi(D_sample, eg, snap.T, snap.n_electrons * frac)
    s_s, mts_s = oracle.entropy(D_sample, eg, fr_s["e_fermi"], snap.T)
    D_est = D_sample / frac                             # whole-grid estimate
    fr_e = oracle.fermi(D_est, eg, snap.T, snap.n_electrons)
    s_e, mts_e = oracle.entropy(D_est, eg, fr_e["e_fermi"], snap.T)
    out = {
        "case": "slab_sample", "snapshot": snap.name, "fingerprint": fingerprint(snap, net),
        "n_points": snap.n_points, "n_atoms": snap.n_atoms, "dV": snap.dV, "T": snap.T,
        "n_electrons": snap.n_electrons, "egrid": list(eg),
        "stride": stride, "offset": offset, "n_sample": int(len(pts)),
        "mean_neighbours_every_64th": float(np.mean(nbr)), "max_neighbours": int(meta["max_neighbours"]),
        "sample": {"n_electrons": snap.n_electrons * frac, "dos": [float(x) for x in D_sample],
                   "e_fermi": fr_s["e_fermi"], "e_band": fr_s["e_band"], "n_found": fr_s["n_found"],
                   "entropy_kb": s_s, "minus_ts": mts_s},
        "estimate": {"dos": [float(x) for x in D_est], "e_fermi": fr_e["e_fermi"], "e_band": fr_e["e_band"],
                     "entropy_kb": s_e, "minus_ts": mts_e},
        "oracle_seconds": time.time() - t0, "threads": threads,
    }
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "full_slab_sample.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print("slab_sample", len(pts), "points; E_F", fr_e["e_fermi"], "%.0fs" % (time.time() - t0), flush=True)


def derived(case):
    """Entropy from the stored oracle DOS and Fermi level (Eq. electronicentropyDOS)."""
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "full_%s.json" % case)
    g = json.load(open(path))
    s_kb, minus_ts = oracle.entropy(np.array(g["dos"]), tuple(g["egrid"]), g["e_fermi"], g["T"])
    g["entropy_kb"], g["minus_ts"] = s_kb, minus_ts
    with open(path, "w") as f:
        json.dump(g, f, indent=1)
    print(case, "S/k_B", s_kb, "-TS", minus_ts, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("cases", nargs="+", choices=sorted(CASES))
    ap.add_argument("--threads", type=int, default=0)
    ap.add_argument("--derived", action="store_true")
    a = ap.parse_args()
    for c in a.cases:
        if c == "slab_sample":
            run_slab_sample(a.threads)
        elif a.derived:
            derived(c)
        else:
            run(c, a.threads)


if __name__ == "__main__":
    main()
