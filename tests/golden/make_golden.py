"""Write full-grid expected values with the FP64 oracle (calls only oracle/).

Full-grid quantities (DOS, Fermi level, band energy, the integrated density)
need every grid point, which the oracle takes minutes to hours to compute,
so they are computed once here and stored as JSON next to this script.
Per-point quantities (B, LDOS, density at sampled points) are recomputed by
the tests directly, because the oracle finishes those in seconds.

Usage (from the repository root):
    python -m tests.golden.make_golden paper_solid paper_liquid small [--threads N]
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
        if a.derived:
            derived(c)
        else:
            run(c, a.threads)


if __name__ == "__main__":
    main()
