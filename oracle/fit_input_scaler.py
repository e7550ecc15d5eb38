"""Fit the network's input standardisation on a calibration snapshot.

The synthetic network stands in for a trained model, whose saved input
scaler would have been fit on training descriptors (the paper standardises
descriptors before the network, Sec. 3.5/3.6).  Here the calibration
snapshot is the 32-atom jittered fcc Al cell on a 20^3 grid (seed 1), and
the descriptors are the oracle's FP64 values at twojmax 8 and 10.  The
per-component mean and population standard deviation (1 where it is 0) are
written to ``mala_synth/data/input_scaler_tj<twojmax>.txt``, which both the
oracle and the GPU path then read as part of the model.

Run from the repository root:  python -m oracle.fit_input_scaler
"""
import os
import sys

import numpy as np

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))

import mala_synth  # noqa: E402
import oracle  # noqa: E402


def fit(twojmax):
    snap = mala_synth.small()
    snap.twojmax = twojmax
    B = oracle.descriptors(snap)
    mu = B.mean(axis=0)
    sd = B.std(axis=0)
    sd[sd == 0.0] = 1.0
    return mu, sd


def main():
    out_dir = os.path.join(os.path.dirname(mala_synth.__file__), "data")
    for tj in (8, 10):
        mu, sd = fit(tj)
        path = os.path.join(out_dir, "input_scaler_tj%d.txt" % tj)
        with open(path, "w") as f:
            f.write("# input standardisation for twojmax=%d: mean std per component\n" % tj)
            f.write("# fit by oracle/fit_input_scaler.py on the 32-atom fcc Al cell "
                    "(seed 1), 20^3 grid, rcut 4.67 A\n")
            for m, s in zip(mu, sd):
                f.write("%.17g %.17g\n" % (m, s))
        print(path, len(mu))


if __name__ == "__main__":
    main()
