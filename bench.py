"""Benchmark of the grid-inference path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload paper_solid]
                    [--precision fp32|bf16] [--no-cpu-baseline]

A step is one call of the fused path (mala_predict) on one synthetic
snapshot: atom binning, bispectrum descriptors of every grid point, an E_F
estimate on a point subsample, the network with the DOS and the energy
window reduced in its epilogue, Fermi level, band energy, and the density.  Inputs (positions are
host data by the ABI; the B cache and outputs are preallocated in HBM) are
in place before the timed region.  Prints one JSON line.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import mala_synth  # noqa: E402

METRIC = "grid points/s (bispectrum+MLP+LDOS reduce); p50/p99 snapshot latency"
PEAK_FP32_VALU_TFLOPS = 157.3     # 256 CU x 4 SIMD x 16 lanes x 2 (FMA) x 2 (packed) x 2.4 GHz
WORKLOADS = {
    "paper_solid": (mala_synth.paper_solid, mala_synth.paper_net),
    "paper_liquid": (mala_synth.paper_liquid, mala_synth.paper_net),
    "small": (mala_synth.small, mala_synth.small_net),
    "slab": (mala_synth.slab, mala_synth.paper_net),
}


def index_counts(tj):
    """Algorithmic term counts per grid point from the index sets."""
    n_half = sum((J // 2 + 1) * (J + 1) for J in range(tj + 1))
    z_terms = b_terms = 0
    for j1 in range(tj + 1):
        for j2 in range(j1 + 1):
            for j in range(j1 - j2, min(tj, j1 + j2) + 1, 2):
                if j < j1:
                    continue
                D, HR = (j1 + j2 - j) // 2, j // 2
                b_terms += (HR + 1) * (j + 1)
                for mb in range(j + 1):
                    for mb1 in range(max(0, mb + D - j2), min(j1, mb + D) + 1):
                        for ma in range(HR + 1):
                            for ma1 in range(j1 + 1):
                                if 0 <= ma - ma1 + D <= j2:
                                    z_terms += 1
    return n_half, z_terms, b_terms


def mean_neighbours(snap, n_sample=4096, seed=99):
    """Mean number of atom images within rcut over a seeded sample of points."""
    pts = mala_synth.sample_points(snap.n_points, n_sample, seed)
    N, L = snap.N, snap.L
    ijk = np.stack([pts // (N[1] * N[2]), (pts // N[2]) % N[1], pts % N[2]], 1)
    r = ijk * (L / N)
    if np.min(L) > 2.0 * snap.rcut:          # minimum image suffices: periodic KD-tree
        from scipy.spatial import cKDTree
        tree = cKDTree(np.mod(snap.positions, L), boxsize=L)
        return float(np.mean(tree.query_ball_point(np.mod(r, L), snap.rcut, return_length=True)))
    nmax = np.ceil(snap.rcut / L).astype(int) + 1
    shifts = np.array([[a, b, c] for a in range(-nmax[0], nmax[0] + 1)
                       for b in range(-nmax[1], nmax[1] + 1) for c in range(-nmax[2], nmax[2] + 1)]) * L
    tot = 0
    for k in range(0, len(pts), 256):
        d = snap.positions[None, :, None, :] + shifts[None, None, :, :] - r[k:k + 256, None, None, :]
        tot += int(np.sum(np.einsum("pasx,pasx->pas", d, d) < snap.rcut ** 2))
    return tot / len(pts)


def flops_per_point(snap, widths):
    n_half, z_terms, b_terms = index_counts(snap.twojmax)
    nb = mean_neighbours(snap)
    mlp = 2 * sum(widths[i] * widths[i + 1] for i in range(len(widths) - 1))
    return {"u": 22.0 * n_half * nb, "zb": 10.0 * z_terms + 4.0 * b_terms, "mlp": float(mlp),
            "mean_neighbours": nb, "z_terms": z_terms, "b_terms": b_terms, "n_half": n_half}


def cpu_baseline(snap, net, n_sample):
    import oracle
    threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or min(16, os.cpu_count() or 1)
    pts = mala_synth.sample_points(snap.n_points, n_sample, 1234)
    t0 = time.time()
    B = oracle.descriptors(snap, pts, nthreads=threads)
    ld = oracle.mlp(B, net, nthreads=threads)
    D = oracle.dos(ld, snap.dV) * (snap.n_points / n_sample)
    fr = oracle.fermi(D, mala_synth.EGRID, snap.T, snap.n_electrons)
    oracle.density(ld, fr["weights"])
    dt = time.time() - t0
    return {"value": n_sample / dt, "unit": "grid points/s", "cores": threads, "kind": "oracle",
            "sample": "%d seeded grid points of %s through the whole path (descriptors, network, DOS, "
                      "E_F, E_band, density), %.1f s" % (n_sample, snap.name, dt)}


TRAFFIC_FILES = {"paper_solid": "traffic_k_zb_al256_solid_90c_tj10.txt"}


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in ("paper_2411_19617_amd/csrc/bispectrum.hip", "paper_2411_19617_amd/csrc/mala_internal.h"):
        h.update(open(os.path.join(ROOT, f), "rb").read())
    return h.hexdigest()[:16]


def measured_traffic(workload):
    """HBM bytes per k_zb launch from the committed, calibrated rocprofv3 counters;
    None if there are none for this workload or the kernel source changed since."""
    name = TRAFFIC_FILES.get(workload)
    path = os.path.join(ROOT, "profiles", name) if name else None
    if not path or not os.path.exists(path):
        return None
    kv = dict(l.strip().split("=", 1) for l in open(path) if "=" in l and not l.startswith("#"))
    if kv.get("kernel_source_sha256_16") != kernel_source_hash():
        return None
    return float(kv["traffic_bytes_per_launch"])


def errors_vs_oracle(workload, snap, dos, r, dens):
    """Whole-grid errors against the oracle's stored full-grid values (if any)."""
    path = os.path.join(ROOT, "tests", "golden", "full_%s.json" % workload)
    if not os.path.exists(path):
        return None
    g = json.load(open(path))
    D = dos.cpu().numpy()
    Dref = np.array(g["dos"])
    return {"dos_max_rel": float(np.max(np.abs(D - Dref)) / np.max(np.abs(Dref))),
            "e_fermi_ev": abs(r["e_fermi"] - g["e_fermi"]),
            "e_band_mev_per_atom": abs(r["e_band"] - g["e_band"]) * 1000.0 / snap.n_atoms,
            "density_integral_rel": abs(float(dens.sum().item()) * snap.dV - g["density_sum_dV"]) / g["density_sum_dV"],
            "oracle": "tests/golden/full_%s.json (FP64 oracle, all %d points)" % (workload, g["n_points"])}


def serving_bench(mala, prec, n_requests, slots=4, budget_gb=64, seed=5):
    """Poisson stream of the serving mix through the library's request loop.

    The saturation request rate of the mix is measured first (all requests
    submitted at once); the stream then arrives at 0.7 x that rate.
    Latency = completion - arrival (server clock).
    """
    rng = mala_synth.SplitMix64(seed)
    reqs = [mala_synth.serving_request(rng) for _ in range(n_requests)]
    blob = mala_synth.net_to_blob(mala_synth.paper_net())
    sv = mala.Server(blob, prec, hbm_budget=budget_gb << 30, max_inflight=slots)

    def submit(r):
        return sv.submit(r.positions, r.L, r.N, r.rcut, r.twojmax, mala_synth.EGRID, r.T, r.n_electrons)

    for r in reqs[:slots]:                      # warm-up: slot buffers reach their sizes
        sv.wait(submit(r), 600)
    t0 = time.perf_counter()
    outs = [sv.wait(t, 600) for t in [submit(r) for r in reqs]]
    sat = time.perf_counter() - t0
    sat_rate = n_requests / sat
    lam = 0.7 * sat_rate
    gaps = -np.log(1.0 - rng.uniform(n_requests)) / lam
    arrivals = np.cumsum(gaps)
    tickets = []
    t0 = time.perf_counter()
    for r, ta in zip(reqs, arrivals):
        while time.perf_counter() - t0 < ta:
            time.sleep(0.0002)
        tickets.append(submit(r))
    outs = [sv.wait(t, 600) for t in tickets]
    span = time.perf_counter() - t0
    sv.close()
    lat = np.array([o["t_done"] - o["t_submit"] for o in outs]) * 1000.0
    pts = sum(r.n_points for r in reqs)
    bad = sum(1 for o in outs if o["status"] != 0)
    return {"requests": n_requests, "slots": slots, "hbm_budget_gb": budget_gb,
            "points_total": pts, "saturation_req_per_s": sat_rate,
            "saturation_points_per_s": pts / sat, "arrival_rate_req_per_s": lam,
            "p50_latency_ms": float(np.percentile(lat, 50)), "p99_latency_ms": float(np.percentile(lat, 99)),
            "stream_points_per_s": pts / span, "failed": bad,
            "mix": "fcc n^3*4 (n=2..8) or liquid N~U[32,2048], 298-933 K, ~2800 points/atom, seed %d" % seed}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="paper_solid", choices=sorted(WORKLOADS))
    ap.add_argument("--precision", default="fp32", choices=["fp32", "bf16"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=32768)
    ap.add_argument("--serve-requests", type=int, default=48, help="0 disables the serving stream")
    a = ap.parse_args()
    if a.gpus != 1:
        print("bench.py measures one GPU: the path shards by grid slabs with one 2 KB DOS all-reduce, "
              "but multi-GPU runs are not part of this build (use --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2411_19617_amd as mala

    mala.lib()
    snap, net = WORKLOADS[a.workload][0](), WORKLOADS[a.workload][1]()
    prec = mala.PREC_FP32 if a.precision == "fp32" else mala.PREC_BF16
    ctx = mala.Context(0)
    w = ctx.weights(mala_synth.net_to_blob(net), prec)
    dev = torch.device("cuda", 0)
    nB = mala.n_descriptors(snap.twojmax)
    Bc = torch.empty((snap.n_points, nB), dtype=torch.float32, device=dev)
    dos = torch.empty(mala_synth.EGRID[2], dtype=torch.float64, device=dev)
    dens = torch.empty(snap.n_points, dtype=torch.float64, device=dev)
    res = torch.zeros(mala.RESULT_BYTES, dtype=torch.uint8, device=dev)

    def step():
        ctx.mala_predict(w, snap.positions, snap.L, snap.N, snap.rcut, snap.twojmax, mala_synth.EGRID, snap.T,
                         snap.n_electrons, B_cache=Bc, dos=dos, dens=dens, res=res)

    for _ in range(a.warmup):
        step()
    torch.cuda.synchronize()
    ctx.check_device_errors()
    r = mala.read_result(res)
    if r["status"] != 0:
        raise RuntimeError("no Fermi level in warm-up: %s" % r)

    ctx.profile_enable(True)
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(a.steps + 1)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    evs[0].record()
    for k in range(a.steps):
        step()
        evs[k + 1].record()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = ctx.profile_read()
    ctx.profile_enable(False)
    ctx.check_device_errors()
    elapsed = t1 - t0
    lat = np.array([evs[k].elapsed_time(evs[k + 1]) for k in range(a.steps)])
    value = snap.n_points * a.steps / elapsed

    fl = flops_per_point(snap, net["widths"])
    zb_ms, zb_n, zb_pts = prof["zb"]
    zb_avg_ms = zb_ms / max(zb_n, 1)
    zb_flops_per_launch = fl["zb"] * zb_pts / max(zb_n, 1)
    achieved = zb_flops_per_launch / (zb_avg_ms * 1e-3) / 1e12
    stages = {k: {"ms_per_step": v[0] / a.steps, "launches_per_step": v[1] / a.steps}
              for k, v in prof.items() if v[1]}
    out = {
        "metric": METRIC, "value": value, "unit": "grid points/s", "n_gpus": 1, "steps": a.steps,
        "warmup": a.warmup, "ms_per_step": 1000.0 * elapsed / a.steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32" if prec == mala.PREC_FP32 else "bf16",
        "data": "synthetic",
        "config": {"workload": snap.name, "n_points": snap.n_points, "n_atoms": snap.n_atoms,
                   "twojmax": snap.twojmax, "network": "-".join(map(str, net["widths"])),
                   "network_precision": a.precision, "reductions": "f64", "T_K": snap.T,
                   "n_electrons": snap.n_electrons},
        "latency_ms": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99)),
                       "kind": "single snapshot, back-to-back"},
        "roofline": {"kernel": "k_zb (Z/B contraction)", "bound": "alu", "achieved": achieved,
                     "peak": PEAK_FP32_VALU_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP32_VALU_TFLOPS, "traffic": measured_traffic(a.workload),
                     "traffic_unit": "bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
                     "flops_per_point": fl["zb"], "points_per_launch": zb_pts / max(zb_n, 1),
                     "avg_launch_ms": zb_avg_ms},
        "stages": stages,
        "algorithmic_kflop_per_point": {"u": fl["u"] / 1e3, "zb": fl["zb"] / 1e3, "mlp": fl["mlp"] / 1e3,
                                        "mean_neighbours": fl["mean_neighbours"]},
        "result": {"e_fermi": r["e_fermi"], "e_band_mev_per_atom": 1000 * r["e_band"] / snap.n_atoms},
        "errors_vs_oracle": errors_vs_oracle(a.workload, snap, dos, mala.read_result(res), dens),
    }
    if a.serve_requests > 0:
        out["serving"] = serving_bench(mala, prec, a.serve_requests)
        out["latency_ms"]["serving_p50"] = out["serving"]["p50_latency_ms"]
        out["latency_ms"]["serving_p99"] = out["serving"]["p99_latency_ms"]
    if not a.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(snap, net, a.cpu_sample)
    print(json.dumps(out), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
