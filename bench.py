"""Benchmark of the grid-inference path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload slab]
                    [--no-cpu-baseline] [--serve-requests N] [--no-extras]

A step is one call of the fused path (mala_predict) on one synthetic
snapshot: atom binning, bispectrum descriptors of every grid point, an E_F
estimate on a point subsample, the network with the DOS and the energy
window reduced in its epilogue, Fermi level, band energy, and the density.
Inputs (positions are host data by the ABI; the B cache and outputs are
preallocated in HBM) are in place before the timed region.

The headline is the 47,066,880-point fcc(111) slab (16,384 atoms) with the
FP32 network; the same line carries the precision form (BF16 network, FP32
accumulation, FP64 reductions) on the slab, both forms on the 729,000-point
256-atom solid, the serving streams of both forms, lines outside the
metric (Gaussian descriptors, both VJPs, grid ACE) and the CPU oracle's
rate.  Prints one JSON line.
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
PEAK_MFMA_TFLOPS = {"fp32": 157.3, "bf16": 2500.0}   # dense matrix peaks
WORKLOADS = {
    "paper_solid": (mala_synth.paper_solid, mala_synth.paper_net),
    "paper_solid_200": (lambda: mala_synth.paper_solid(grid=200), mala_synth.paper_net),
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


def mean_neighbours(snap, n_sample=4096, seed=99, pts=None):
    """Mean number of atom images within rcut over a seeded sample of points
    (or over the given flat indices)."""
    if pts is None:
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


def path_ceiling(fl, precision):
    """Roofline rate of the whole path in grid points/s: the descriptor work
    (U and Z/B) at the FP32 vector peak plus the network at the matrix peak
    of its precision (the reductions are below 0.1% of the work)."""
    t = (fl["u"] + fl["zb"]) / (PEAK_FP32_VALU_TFLOPS * 1e12) + fl["mlp"] / (PEAK_MFMA_TFLOPS[precision] * 1e12)
    return 1.0 / t


def host_cpu():
    model = None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"nproc": os.cpu_count(), "affinity_cpus": len(os.sched_getaffinity(0)), "cpu_model": model}


def cpu_baseline(snap, net, n_sample):
    """The FP64 oracle (built -O3 -march=native for this host) on a seeded
    sample of the workload's grid points through the whole path; returns the
    record and the oracle's B and LDOS of the sample for the error check."""
    import tempfile

    import oracle
    threads = min(16, len(os.sched_getaffinity(0)))          # the host share of one GPU
    oracle.use_library(oracle.build_native(tempfile.mkdtemp(prefix="oracle_native_")))
    pts = mala_synth.sample_points(snap.n_points, n_sample, 1234)
    t0 = time.time()
    B = oracle.descriptors(snap, pts, nthreads=threads)
    ld = oracle.mlp(B, net, nthreads=threads)
    D = oracle.dos(ld, snap.dV) * (snap.n_points / n_sample)
    fr = oracle.fermi(D, mala_synth.EGRID, snap.T, snap.n_electrons)
    oracle.density(ld, fr["weights"])
    dt = time.time() - t0
    rec = {"value": n_sample / dt, "unit": "grid points/s", "cores": threads, "kind": "oracle",
           "sample": "%d seeded grid points of %s (mean %.1f neighbours) through the whole path (descriptors, "
                     "network, DOS, E_F, E_band, density), %.1f s; oracle built -O3 -march=native, OpenMP over "
                     "points" % (n_sample, snap.name, mean_neighbours(snap, pts=pts), dt),
           "host": host_cpu()}
    return rec, pts, B, ld


TRAFFIC_FILES = {"al16384_slab111_fault_298K_tj10": "traffic_k_zb_al16384_slab_tj10.txt"}


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in ("paper_2411_19617_amd/csrc/bispectrum.hip", "paper_2411_19617_amd/csrc/mala_internal.h"):
        h.update(open(os.path.join(ROOT, f), "rb").read())
    return h.hexdigest()[:16]


def measured_traffic(snapshot):
    """HBM bytes per k_zb point from the committed, calibrated rocprofv3 counters;
    None if there are none for this snapshot or the kernel source changed since."""
    name = TRAFFIC_FILES.get(snapshot)
    path = os.path.join(ROOT, "profiles", name) if name else None
    if not path or not os.path.exists(path):
        return None
    kv = dict(l.strip().split("=", 1) for l in open(path) if "=" in l and not l.startswith("#"))
    if kv.get("kernel_source_sha256_16") != kernel_source_hash():
        return None
    return float(kv["traffic_bytes_per_point"])


TRAFFIC_CMDS = """# commands (repository root = $REPO, output directory $OUT, after cd /tmp && export TMPDIR=/tmp):
#   rocprofv3 --pmc FETCH_SIZE --output-format csv -d $OUT/pmc_fetch -o run -- python $REPO/bench.py --workload %(w)s --headline-only --steps 1 --warmup 1 --no-cpu-baseline
#   rocprofv3 --pmc WRITE_SIZE --output-format csv -d $OUT/pmc_write -o run -- python $REPO/bench.py --workload %(w)s --headline-only --steps 1 --warmup 1 --no-cpu-baseline
#   rocprofv3 --pmc FETCH_SIZE --output-format csv -d $OUT/pmc_cfetch -o run -- python $REPO/bench.py --copy-calibration
#   rocprofv3 --pmc WRITE_SIZE --output-format csv -d $OUT/pmc_cwrite -o run -- python $REPO/bench.py --copy-calibration
#   python bench.py --workload %(w)s --traffic-summary $OUT/pmc_fetch $OUT/pmc_write $OUT/pmc_cfetch $OUT/pmc_cwrite
"""
COPY_GIB = 1


def copy_calibration():
    """Three plain device-to-device copies of 1 GiB: the reference for scaling
    FETCH_SIZE / WRITE_SIZE (KiB per dispatch) to bytes."""
    import torch
    a = torch.ones(COPY_GIB << 28, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print("copied 3 x %d GiB" % COPY_GIB, flush=True)


def _pmc_rows(d, counter, kernel_prefix):
    import csv
    import glob
    files = glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)
    if not files:
        raise SystemExit("no counter_collection.csv under %s" % d)
    out = []
    for f in files:
        for r in csv.DictReader(open(f)):
            if r["Counter_Name"] == counter and r["Kernel_Name"].startswith(kernel_prefix):
                out.append((int(r["Dispatch_Id"]), int(r["Grid_Size"]) // int(r["Workgroup_Size"]),
                            float(r["Counter_Value"])))
    return sorted(out)


def traffic_summary(fetch_dir, write_dir, cfetch_dir, cwrite_dir, workload="paper_solid"):
    """Write the calibrated HBM traffic of k_zb<10> into profiles/ from four
    rocprofv3 --pmc runs (kernel FETCH_SIZE, WRITE_SIZE; copy FETCH_SIZE, WRITE_SIZE)."""
    copy_kib = float(COPY_GIB << 20)
    cf = [v for _, _, v in _pmc_rows(cfetch_dir, "FETCH_SIZE", "__amd_rocclr_copyBuffer") if v > 0.5 * copy_kib / 4]
    cw = [v for _, _, v in _pmc_rows(cwrite_dir, "WRITE_SIZE", "__amd_rocclr_copyBuffer") if v > 0.5 * copy_kib / 4]
    fs, ws = copy_kib / float(np.mean(cf)), copy_kib / float(np.mean(cw))
    kz = "void mala::k_zb<10>"
    fr, wr = _pmc_rows(fetch_dir, "FETCH_SIZE", kz), _pmc_rows(write_dir, "WRITE_SIZE", kz)
    pts = [nb * 64 for _, nb, _ in fr]                  # one 64-point tile per workgroup
    fb = [v * 1024.0 * fs for _, _, v in fr]
    wb = [v * 1024.0 * ws for _, _, v in wr]
    snap = WORKLOADS[workload][0]()
    tj = snap.twojmax
    n_half = sum((J // 2 + 1) * (J + 1) for J in range(tj + 1))
    n_b = (tj + 2) * (tj + 3) * (tj + 4) // 24
    alg = n_half * 8 + n_b * 4
    per_launch = float(np.mean(fb) + np.mean(wb))
    per_point = (sum(fb) + sum(wb)) / float(sum(pts))
    name = TRAFFIC_FILES[snap.name]
    with open(os.path.join(ROOT, "profiles", name), "w") as f:
        f.write("# HBM traffic of k_zb<10> (Z/B contraction), %s\n" % snap.name)
        f.write(TRAFFIC_CMDS % {"w": workload})
        f.write("# calibration: the same two counters on a plain %d GiB device-to-device copy (torch copy_ ->\n"
                "# __amd_rocclr_copyBuffer), %d copies: FETCH_SIZE %.0f KiB, WRITE_SIZE %.0f KiB per copy of %.0f KiB\n"
                % (COPY_GIB, len(cf), np.mean(cf), np.mean(cw), copy_kib))
        f.write("# k_zb dispatches (points, tiles x 64): %s\n" % pts)
        f.write("# FETCH_SIZE KiB per dispatch: %s\n" % [round(v) for _, _, v in fr])
        f.write("# WRITE_SIZE KiB per dispatch: %s\n" % [round(v) for _, _, v in wr])
        f.write("# algorithmic bytes per point: read u %d x 8 = %d, write B %d x 4 = %d -> %d\n"
                % (n_half, n_half * 8, n_b, n_b * 4, alg))
        f.write("kernel_source_sha256_16=%s\n" % kernel_source_hash())
        f.write("fetch_scale=%.6f\nwrite_scale=%.6f\n" % (fs, ws))
        f.write("points_per_launch=%.1f\n" % float(np.mean(pts)))
        f.write("fetch_bytes_per_launch=%.0f\nwrite_bytes_per_launch=%.0f\n" % (np.mean(fb), np.mean(wb)))
        f.write("traffic_bytes_per_launch=%.0f\n" % per_launch)
        f.write("traffic_bytes_per_point=%.1f\n" % per_point)
    print("wrote profiles/%s: %.1f B/point (algorithmic %d)" % (name, per_point, alg))


def _short_kernel_name(n):
    n = n.replace("(anonymous namespace)", "(anon)")
    if n.startswith("void "):
        n = n[5:]
    depth, out = 0, []
    for ch in n:                       # drop the argument list, keep template arguments
        if ch == "(" and depth == 0 and out and out[-1] != ":":
            break
        depth += ch == "<"
        depth -= ch == ">"
        out.append(ch)
    return "".join(out)


def stats_summary(prof_dir, bench_json, out_name, command):
    """Markdown kernel table from a rocprofv3 --kernel-trace --stats run plus the
    bench line of the same build (for the live HIP-event launch time)."""
    import csv
    import glob
    f = glob.glob(os.path.join(prof_dir, "**", "*kernel_stats.csv"), recursive=True)
    if not f:
        raise SystemExit("no kernel_stats.csv under %s" % prof_dir)
    rows = list(csv.DictReader(open(f[0])))
    b = None
    for line in (open(bench_json).read().split("\n") if bench_json != "-" else []):  # the profiler may log after it
        if line.startswith("{"):
            try:
                b = json.loads(line)
            except ValueError:
                pass
    if b is None and bench_json != "-":
        raise SystemExit("no bench JSON line in %s" % bench_json)
    title = ("%s, %s network" % (b["config"]["workload"], b["config"]["network_precision"]) if b else
             "bench.py --probe-kernels (each kernel family once on the 729,000-point 256-atom solid)")
    lines = ["# rocprofv3 kernel stats: " + title, "",
             "Command (repository root = $REPO, output directory $OUT):", "", "```",
             "cd /tmp && export TMPDIR=/tmp && " + command, "```", "",
             "| kernel | calls | avg ms | min ms | max ms | total ms | share |", "|---|---|---|---|---|---|---|"]
    zb = None
    for r in rows:
        name = _short_kernel_name(r["Name"])
        lines.append("| `%s` | %s | %.4f | %.4f | %.4f | %.3f | %.1f%% |" % (
            name, r["Calls"], float(r["AverageNs"]) / 1e6, float(r["MinNs"]) / 1e6, float(r["MaxNs"]) / 1e6,
            float(r["TotalDurationNs"]) / 1e6, float(r["Percentage"])))
        if name.startswith("mala::k_zb<"):
            zb = float(r["AverageNs"]) / 1e6
    lines += ["", "The metric's step runs the cell list, `k_ui`, `k_zb`, `k_mlp` and `k_fermi` "
              "(and `k_density_window`); `k_gauss`, `k_mlp_vjp`, `k_yi`, `k_dedr`, `k_ace_proj`, `k_ace`, `k_ace4` and "
              "`k_planes_to_rows` come "
              "from the lines outside the metric (Gaussian descriptors, both VJPs, grid ACE) when they are run."]
    if b is None:
        with open(os.path.join(ROOT, "profiles", out_name), "w") as fo:
            fo.write("\n".join(lines) + "\n")
        print("wrote profiles/%s" % out_name)
        return
    rf = b["roofline"]
    lines += ["", "Dominant kernel `k_zb`: rocprof average %.4f ms per launch; bench.py (same build, "
              "HIP events on the library stream) %.4f ms per launch over %.0f points: achieved %.1f %s = "
              "%.3f of the %.1f %s peak (%.1f kflop/point)."
              % (zb or float("nan"), rf["avg_launch_ms"], rf["points_per_launch"], rf["achieved"], rf["unit"],
                 rf["frac"], rf["peak"], rf["unit"], rf["flops_per_point"] / 1e3), "",
              "Per-stage times of the bench step (ms): " + ", ".join(
                  "%s %.3f" % (k, v["ms_per_step"]) for k, v in b["stages"].items()), ""]
    with open(os.path.join(ROOT, "profiles", out_name), "w") as fo:
        fo.write("\n".join(lines))
    print("wrote profiles/%s" % out_name)


def probe_kernels():
    """Each kernel family once after one warm-up call, on the 729,000-point
    solid: the fused path in FP32 and BF16 (cell list, k_ui, k_zb, k_mlp,
    k_fermi), grid ACE (k_ace), the network VJP (k_mlp_vjp) and the
    descriptor VJP (k_yi, k_dedr).  A short program for counter runs."""
    import torch
    import paper_2411_19617_amd as mala
    mala.lib()
    ctx = mala.Context(0)
    snap, net = WORKLOADS["paper_solid"][0](), WORKLOADS["paper_solid"][1]()
    blob = mala_synth.net_to_blob(net)
    for prec in (mala.PREC_FP32, mala.PREC_BF16):
        w = ctx.weights(blob, prec)
        for _ in range(2):
            ctx.mala_predict(w, snap.positions, snap.L, snap.N, snap.rcut, snap.twojmax, mala_synth.EGRID, snap.T,
                             snap.n_electrons)
    for _ in range(2):
        ctx.mala_ace_descriptors(snap.positions, snap.L, snap.N, snap.rcut, 4, 4)
    for _ in range(2):
        ctx.mala_ace4_descriptors(snap.positions, snap.L, snap.N, snap.rcut, 3, 3)
    gen = torch.Generator(device="cuda")
    gen.manual_seed(3)
    B = ctx.mala_descriptors(snap.positions, snap.L, snap.N, snap.rcut, snap.twojmax)
    v = torch.randn((snap.n_points, 250), generator=gen, device="cuda", dtype=torch.float32)
    w = ctx.weights(blob, mala.PREC_FP32)
    for _ in range(2):
        g = ctx.mala_ldos_vjp(w, B, v)
    for _ in range(2):
        ctx.mala_descriptors_vjp(snap.positions, snap.L, snap.N, snap.rcut, snap.twojmax, g)
    torch.cuda.synchronize()
    ctx.check_device_errors()
    ctx.close()
    print("probe done", flush=True)


COUNTER_KERNELS = ["mala::k_ui<", "mala::k_zb<", "mala::k_mlp<0", "mala::k_mlp<1", "mala::k_ace4", "mala::k_ace",
                   "mala::k_planes_to_rows",
                   "mala::k_mlp_vjp", "mala::k_yi", "mala::k_dedr"]


def counter_summary(out_name, command, dirs):
    """Per-kernel sums of rocprofv3 --pmc counters (one or more runs, one
    counter set each) and the ratios derived from them: the GPU clock from
    GRBM_GUI_ACTIVE over the dispatch time, VALU issue use (a wave64 VALU
    instruction holds its SIMD for 4 cycles), MFMA busy, LDS bank
    conflicts, FMA share."""
    import csv
    import glob
    import re
    acc = {}
    pmc = {}                                            # counters of each run, in the order they appear
    for d in dirs:
        files = glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)
        if not files:
            raise SystemExit("no counter_collection.csv under %s" % d)
        for f in files:
            for r in csv.DictReader(open(f)):
                names = pmc.setdefault(d, [])
                if r["Counter_Name"] not in names:
                    names.append(r["Counter_Name"])
                name = _short_kernel_name(r["Kernel_Name"])
                key = next((k for k in COUNTER_KERNELS if name.startswith(k)), None)
                if key is None:
                    continue
                a = acc.setdefault(name, {"dispatch": {}, "counters": {}})
                dur = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) * 1e-9
                a["dispatch"][(d, r["Dispatch_Id"])] = dur
                c = a["counters"].setdefault(r["Counter_Name"], {})
                c[(d, r["Dispatch_Id"])] = c.get((d, r["Dispatch_Id"]), 0.0) + float(r["Counter_Value"])
    lines = ["# rocprofv3 counters per kernel", "", "Commands (repository root = $REPO, output directory $OUT, "
             "after `cd /tmp && export TMPDIR=/tmp`; one counter set per run):", "", "```"]
    lines += [command.replace("{DIR}", os.path.basename(os.path.normpath(d)).replace("pmc_", ""))
              .replace("{PMC}", " ".join(pmc.get(d, []))) for d in dirs]
    lines += ["```", "", "Counter sums over the kernel's dispatches of each run; derived ratios use the dispatch "
              "times of the same runs (counter collection serialises dispatches).  GRBM_GUI_ACTIVE is read as "
              "the sum over the 8 XCDs (its per-dispatch value divided by 8 x the dispatch time gives the clock).  "
              "VALU issue = SQ_INSTS_VALU x 4 cycles / (1,024 SIMDs x cycles); MFMA busy = "
              "SQ_VALU_MFMA_BUSY_CYCLES / (1,024 SIMDs x cycles); LDS conflict = SQ_LDS_BANK_CONFLICT / "
              "SQ_LDS_IDX_ACTIVE; wait share = SQ_WAIT_ANY / SQ_WAVE_CYCLES (wave cycles spent in a wait); "
              "L2 hit = TCC_HIT / (TCC_HIT + TCC_MISS).  SQ_INSTS_VALU includes the MFMA instructions "
              "(SQ_INSTS_MFMA), so for the network kernels the VALU issue figure counts their issue "
              "slots too.  Ratios of two counters use only the runs that collected both.", ""]
    names = sorted(acc)
    counters = sorted({c for n in names for c in acc[n]["counters"]})
    lines += ["| kernel | dispatches | " + " | ".join(counters) + " |", "|---|---|" + "---|" * len(counters)]
    derived = []
    for n in names:
        a = acc[n]
        row = ["`%s`" % n, str(max(len(v) for v in a["counters"].values()))]
        tot = {}
        for c in counters:
            v = a["counters"].get(c)
            tot[c] = sum(v.values()) if v else None
            row.append("%.4g" % tot[c] if v else "")
        lines.append("| " + " | ".join(row) + " |")
        # derived ratios per run that holds the needed counters
        def per(c, runs=None):
            v = a["counters"].get(c)
            if not v:
                return None
            keys = [k for k in v if runs is None or k[0] in runs]
            return sum(v[k] for k in keys), sum(a["dispatch"][k] for k in keys)

        def same_run(c1, c2):
            """Sums of two counters over the runs that collected both."""
            r1 = {k[0] for k in a["counters"].get(c1, {})}
            r2 = {k[0] for k in a["counters"].get(c2, {})}
            runs = r1 & r2
            return (per(c1, runs), per(c2, runs)) if runs else (None, None)
        g = per("GRBM_GUI_ACTIVE")
        d = {"kernel": n}
        if g and g[1] > 0:
            d["clock_GHz"] = g[0] / 8.0 / g[1] / 1e9
            d["ms_per_dispatch"] = 1e3 * g[1] / max(len(a["counters"]["GRBM_GUI_ACTIVE"]), 1)
        cyc_per_s = (d.get("clock_GHz") or 2.4) * 1e9
        for c, label, scale in (("SQ_INSTS_VALU", "valu_issue", 4.0), ("SQ_VALU_MFMA_BUSY_CYCLES", "mfma_busy", 1.0)):
            x = per(c)
            if x and x[1] > 0:
                d[label] = x[0] * scale / (1024.0 * cyc_per_s * x[1])
        for num, den, label in (("SQ_INSTS_VALU_FMA_F32", "SQ_INSTS_VALU", "fma_share_of_valu"),
                                ("SQ_LDS_BANK_CONFLICT", "SQ_LDS_IDX_ACTIVE", "lds_conflict_share"),
                                ("SQ_INSTS_LDS", "SQ_INSTS_VALU", "lds_per_valu"),
                                ("SQ_WAIT_ANY", "SQ_WAVE_CYCLES", "wait_share")):
            x, y = same_run(num, den)
            if x and y and y[0] > 0:
                d[label] = x[0] / y[0]
        x, y = same_run("TCC_HIT_sum", "TCC_MISS_sum")
        if x and y and x[0] + y[0] > 0:
            d["l2_hit"] = x[0] / (x[0] + y[0])
        # the two come from different runs of the same program: compare per dispatch
        x, y = a["counters"].get("SQ_INSTS_MFMA"), a["counters"].get("SQ_INSTS_VALU")
        if x and y and sum(y.values()) > 0:
            d["mfma_share_of_valu"] = (sum(x.values()) / len(x)) / (sum(y.values()) / len(y))
        derived.append(d)
    keys = ["clock_GHz", "ms_per_dispatch", "valu_issue", "mfma_share_of_valu", "fma_share_of_valu", "lds_per_valu",
            "mfma_busy", "lds_conflict_share", "wait_share", "l2_hit"]
    lines += ["", "| kernel | " + " | ".join(keys) + " |", "|---|" + "---|" * len(keys)]
    for d in derived:
        lines.append("| `%s` | " % d["kernel"] + " | ".join("%.3f" % d[k] if k in d else "" for k in keys) + " |")
    with open(os.path.join(ROOT, "profiles", out_name), "w") as fo:
        fo.write("\n".join(lines) + "\n")
    print("wrote profiles/%s" % out_name)


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
            "minus_ts_mev_per_atom": (abs(r["e_entropy"] - g["minus_ts"]) * 1000.0 / snap.n_atoms
                                      if "minus_ts" in g else None),
            "density_integral_rel": abs(float(dens.sum().item()) * snap.dV - g["density_sum_dV"]) / g["density_sum_dV"],
            "oracle": "tests/golden/full_%s.json (FP64 oracle, all %d points)" % (workload, g["n_points"])}


def slab_sample_errors(ctx, snap, w, Bc, dos, r, torch):
    """The slab against the oracle's path over its systematic sample (every
    719th point, tests/golden/full_slab_sample.json): the GPU network and
    integration on the same rows of the fused path's B cache, and the
    whole-grid DOS against the sample's estimate (a consistency figure)."""
    path = os.path.join(ROOT, "tests", "golden", "full_slab_sample.json")
    if not os.path.exists(path):
        return None
    g = json.load(open(path))
    pts = mala_synth.strided_points(snap.n_points, g["stride"], g["offset"])
    rows = Bc.index_select(0, torch.as_tensor(pts, device="cuda")).contiguous()
    ld = ctx.mala_ldos_infer(w, rows, mala_synth.EGRID[2])
    gs = g["sample"]
    D, _, res = ctx.mala_integrate(ld, snap.dV, mala_synth.EGRID, snap.T, gs["n_electrons"], density=False)
    import paper_2411_19617_amd as mala
    rs = mala.read_result(res)
    Dref = np.array(gs["dos"])
    atoms = snap.n_atoms * len(pts) / snap.n_points
    De = np.array(g["estimate"]["dos"])
    Dg = dos.cpu().numpy()
    return {"sample_points": len(pts),
            "sample_dos_max_rel": float(np.max(np.abs(D.cpu().numpy() - Dref)) / np.max(np.abs(Dref))),
            "sample_e_fermi_ev": abs(rs["e_fermi"] - gs["e_fermi"]),
            "sample_e_band_mev_per_atom": abs(rs["e_band"] - gs["e_band"]) * 1000.0 / atoms,
            "whole_grid_dos_vs_sample_estimate": float(np.max(np.abs(Dg - De)) / np.max(np.abs(De))),
            "whole_grid_e_fermi_vs_sample_estimate_ev": abs(r["e_fermi"] - g["estimate"]["e_fermi"]),
            "oracle": "tests/golden/full_slab_sample.json (FP64 oracle, every %dth point)" % g["stride"]}


def gaussian_bench(ctx, snap, torch, reps=5):
    """Gaussian descriptors of the whole grid (sigma = grid spacing, cutoff 8
    sigma), outside the metric's step: time per grid and the write rate (the
    kernel writes 4 B per point; its neighbour sums are short)."""
    sigma = float(np.max(snap.L / snap.N))
    G = torch.empty(snap.n_points, dtype=torch.float32, device="cuda")
    ctx.mala_gaussian_descriptors(snap.positions, snap.L, snap.N, sigma, 8 * sigma, out=G)
    ctx.profile_enable(True)
    for _ in range(reps):
        ctx.mala_gaussian_descriptors(snap.positions, snap.L, snap.N, sigma, 8 * sigma, out=G)
    ms = ctx.profile_read()["gauss"][0] / reps
    ctx.profile_enable(False)
    ctx.check_device_errors()
    return {"sigma": sigma, "cutoff": 8 * sigma, "ms_per_grid": ms,
            "points_per_s": snap.n_points / (ms * 1e-3),
            "write_GB_s": 4.0 * snap.n_points / (ms * 1e-3) / 1e9,
            "sum_G_dV_over_atoms": float(G.double().sum().item()) * snap.dV / snap.n_atoms}


def network_vjp_bench(ctx, mala, snap, net, torch, reps=5):
    """Network vector-Jacobian product (the network factor of the force
    expression) over the whole grid with FP32 weights, outside the metric's
    step: descriptor rows around the input scaler and a random vector over
    the energies (seeded, generated on the device).  Work per point: the
    forward pass again plus the three transposed layers, 4 sum(in x out)."""
    n, w0, wl = snap.n_points, net["widths"][0], net["widths"][-1]
    gen = torch.Generator(device="cuda")
    gen.manual_seed(17)
    x = torch.randn((n, w0), generator=gen, device="cuda", dtype=torch.float32)
    B = (x * torch.as_tensor(net["in_std"], dtype=torch.float32, device="cuda")
         + torch.as_tensor(net["in_mean"], dtype=torch.float32, device="cuda")).contiguous()
    del x
    v = torch.randn((n, wl), generator=gen, device="cuda", dtype=torch.float32)
    w = ctx.weights(mala_synth.net_to_blob(net), mala.PREC_FP32)
    g = ctx.mala_ldos_vjp(w, B, v)
    ctx.profile_enable(True)
    for _ in range(reps):
        ctx.mala_ldos_vjp(w, B, v, out=g)
    ms = ctx.profile_read()["mlp_vjp"][0] / reps
    ctx.profile_enable(False)
    ctx.check_device_errors()
    wd = net["widths"]
    flops = 4.0 * sum(wd[i] * wd[i + 1] for i in range(len(wd) - 1))
    tf = flops * n / (ms * 1e-3) / 1e12
    del B, v, g
    return {"ms_per_grid": ms, "points_per_s": n / (ms * 1e-3), "flops_per_point": flops,
            "tflops": tf, "peak": PEAK_MFMA_TFLOPS["fp32"], "frac": tf / PEAK_MFMA_TFLOPS["fp32"],
            "precision": "f32"}


def adjoint_z_terms(tj):
    """Z terms of the descriptor adjoint: for every coupled pair (A >= B) and
    output level C, the half rows ma <= C/2 of Z^C(A, B) over all columns,
    each a sum over (ma1, mb1) with both coupled indices in range."""
    tot = 0
    for C in range(tj + 1):
        for A in range(tj + 1):
            for B in range(A + 1):
                if not (A - B <= C <= A + B and (A + B + C) % 2 == 0):
                    continue
                D = (A + B - C) // 2
                rows = sum(1 for ma in range(C // 2 + 1) for ma1 in range(A + 1) if 0 <= ma - ma1 + D <= B)
                cols = sum(1 for mb in range(C + 1) for mb1 in range(A + 1) if 0 <= mb - mb1 + D <= B)
                tot += rows * cols
    return tot


def descriptor_adjoint_bench(ctx, snap, torch, reps=3):
    """Descriptor vector-Jacobian product (descriptor factor of the force
    expression) over the whole grid with seeded weights, outside the metric's
    step: time per grid, per stage (u again, dL/du, dL/dR), and the dL/du
    contraction's rate at 10 flop per Z term."""
    n, nb = snap.n_points, 91
    gen = torch.Generator(device="cuda")
    gen.manual_seed(23)
    gB = torch.randn((n, nb), generator=gen, device="cuda", dtype=torch.float32)
    out = ctx.mala_descriptors_vjp(snap.positions, snap.L, snap.N, snap.rcut, snap.twojmax, gB)
    ctx.profile_enable(True)
    for _ in range(reps):
        ctx.mala_descriptors_vjp(snap.positions, snap.L, snap.N, snap.rcut, snap.twojmax, gB, out=out)
    p = ctx.profile_read()
    ctx.profile_enable(False)
    ctx.check_device_errors()
    st = {k: p[k][0] / reps for k in ("bin", "ui", "adj_y", "adj_dedr")}
    ms = sum(st.values())
    zt = adjoint_z_terms(snap.twojmax)
    tf_y = 10.0 * zt * n / (st["adj_y"] * 1e-3) / 1e12
    del gB, out
    return {"ms_per_grid": ms, "points_per_s": n / (ms * 1e-3), "stages_ms": st,
            "adj_y": {"flops_per_point": 10.0 * zt, "tflops": tf_y, "peak": PEAK_FP32_VALU_TFLOPS,
                      "frac": tf_y / PEAK_FP32_VALU_TFLOPS}}


def ace_flops(nmax, lmax, mean_nbr):
    """Work of the grid ACE descriptors per point: 4 flop per (n, l, m >= 0)
    and neighbour for the projections, 4 per rank-2 term (n1 <= n2, all m),
    12 per nonzero rank-3 term (m1, m2, m3 = -m1-m2, 3j != 0)."""
    from sympy.physics.wigner import wigner_3j
    proj = 4.0 * nmax * (lmax + 1) * (lmax + 2) / 2 * mean_nbr
    r2 = 4.0 * sum((2 * l + 1) * nmax * (nmax + 1) / 2 for l in range(lmax + 1))
    keys = [(n, l) for n in range(nmax) for l in range(lmax + 1)]
    terms = 0
    for i in range(len(keys)):
        for j in range(i, len(keys)):
            for k in range(j, len(keys)):
                l1, l2, l3 = keys[i][1], keys[j][1], keys[k][1]
                if not (abs(l1 - l2) <= l3 <= l1 + l2 and (l1 + l2 + l3) % 2 == 0):
                    continue
                terms += sum(1 for m1 in range(-l1, l1 + 1) for m2 in range(-l2, l2 + 1)
                             if abs(m1 + m2) <= l3 and wigner_3j(l1, l2, l3, m1, m2, -m1 - m2) != 0)
    return proj + r2 + 12.0 * terms, terms


def ace_bench(ctx, mala, snap, mean_nbr, torch, reps=3, nmax=4, lmax=4):
    """Grid ACE descriptors (ranks 1-3, nmax = lmax = 4, 602 per point) over the
    whole grid, outside the metric's step."""
    out = ctx.mala_ace_descriptors(snap.positions, snap.L, snap.N, snap.rcut, nmax, lmax)
    ctx.profile_enable(True)
    for _ in range(reps):
        ctx.mala_ace_descriptors(snap.positions, snap.L, snap.N, snap.rcut, nmax, lmax, out=out)
    ms = ctx.profile_read()["ace"][0] / reps
    ctx.profile_enable(False)
    del out
    dm = ctx.mala_ace_descriptors(snap.positions, snap.L, snap.N, snap.rcut, nmax, lmax, descriptor_major=True)
    ctx.profile_enable(True)
    for _ in range(reps):
        ctx.mala_ace_descriptors(snap.positions, snap.L, snap.N, snap.rcut, nmax, lmax, out=dm, descriptor_major=True)
    ms_dm = ctx.profile_read()["ace"][0] / reps
    ctx.profile_enable(False)
    out = dm
    ctx.check_device_errors()
    fl, terms = ace_flops(nmax, lmax, mean_nbr)
    tf = fl * snap.n_points / (ms * 1e-3) / 1e12
    del out
    return {"nmax": nmax, "lmax": lmax, "descriptors": mala.ace_count(nmax, lmax), "rank3_terms": terms,
            "ms_per_grid": ms, "ms_per_grid_descriptor_major": ms_dm,
            "points_per_s": snap.n_points / (ms * 1e-3), "flops_per_point": fl,
            "tflops": tf, "peak": PEAK_FP32_VALU_TFLOPS, "frac": tf / PEAK_FP32_VALU_TFLOPS,
            "frac_descriptor_major": fl * snap.n_points / (ms_dm * 1e-3) / 1e12 / PEAK_FP32_VALU_TFLOPS}


def ace4_flops(mala, nmax4, lmax4, mean_nbr):
    """Work of the rank-4 grid ACE descriptors per point: the projection
    (4 flop per (n < 4, l <= 4, m >= 0) and neighbour), 10 flop per term of
    the coupled pairs P_a(M) = sum <l1 m1 l2 m2|L M> A A (M >= 0; terms where
    both m lie in range, the structural count) and 4 flop per M of every
    descriptor's inner product."""
    nl = lmax4 + 1
    pairs, desc = set(), 0.0
    for p1, p2, p3, p4, L in mala.ace4_list(nmax4, lmax4):
        pairs.add((p1, p2, L))
        pairs.add((p3, p4, L))
        desc += 4.0 * (L + 1)
    terms = 0
    for p1, p2, L in pairs:
        l1, l2 = p1 % nl, p2 % nl
        terms += sum(1 for M in range(L + 1) for m1 in range(-l1, l1 + 1) if abs(M - m1) <= l2)
    proj = 4.0 * 4 * 15 * mean_nbr
    return proj + 10.0 * terms + desc, terms


def ace4_bench(ctx, mala, snap, mean_nbr, torch, reps=3, nmax4=3, lmax4=3):
    """Rank-4 grid ACE descriptors (nmax4 = lmax4 = 3) over the whole grid,
    outside the metric's step."""
    out = ctx.mala_ace4_descriptors(snap.positions, snap.L, snap.N, snap.rcut, nmax4, lmax4)
    ctx.profile_enable(True)
    for _ in range(reps):
        ctx.mala_ace4_descriptors(snap.positions, snap.L, snap.N, snap.rcut, nmax4, lmax4, out=out)
    ms = ctx.profile_read()["ace4"][0] / reps
    ctx.profile_enable(False)
    del out
    out = ctx.mala_ace4_descriptors(snap.positions, snap.L, snap.N, snap.rcut, nmax4, lmax4, descriptor_major=True)
    ctx.profile_enable(True)
    for _ in range(reps):
        ctx.mala_ace4_descriptors(snap.positions, snap.L, snap.N, snap.rcut, nmax4, lmax4, out=out,
                                  descriptor_major=True)
    ms_dm = ctx.profile_read()["ace4"][0] / reps
    ctx.profile_enable(False)
    ctx.check_device_errors()
    fl, terms = ace4_flops(mala, nmax4, lmax4, mean_nbr)
    tf = fl * snap.n_points / (ms * 1e-3) / 1e12
    n4 = mala.ace4_count(nmax4, lmax4)
    del out
    return {"nmax4": nmax4, "lmax4": lmax4, "descriptors": n4, "pair_terms": terms, "ms_per_grid": ms,
            "ms_per_grid_descriptor_major": ms_dm,
            "points_per_s": snap.n_points / (ms * 1e-3), "flops_per_point": fl, "tflops": tf,
            "peak": PEAK_FP32_VALU_TFLOPS, "frac": tf / PEAK_FP32_VALU_TFLOPS,
            "write_GB_s": 4.0 * n4 * snap.n_points / (ms * 1e-3) / 1e9}


def serving_bench(mala, prec, reqs, n_main, n_side=200, slots=4, budget_gb=64, loads=(0.5, 0.7, 0.9), seed=5,
                  inflight_points=0):
    """Poisson streams of the serving mix through the library's request loop.

    At most `inflight_points` grid points run at once (a larger request runs
    alone), with up to `slots` requests.  Every slot is sized once for the
    largest request of the mix
    (mala_server_reserve) and warmed by the `slots` largest requests at once;
    the allocation counter of the slots must not move after that.  The
    saturation request rate comes from the first n_side requests submitted
    at once; the streams then arrive at 0.5, 0.7 and 0.9 x that rate, the
    0.7 x stream over n_main requests and the others over n_side.  Latency =
    completion - arrival (server clock).
    """
    rng = mala_synth.SplitMix64(seed + 1000)
    blob = mala_synth.net_to_blob(mala_synth.paper_net())
    sv = mala.Server(blob, prec, hbm_budget=budget_gb << 30, max_inflight=slots)
    sv.reserve([(r.n_atoms, r.L, r.N, r.rcut, r.twojmax, mala_synth.EGRID, r.T) for r in reqs])
    sv.set_inflight_points(inflight_points)

    def submit(r):
        return sv.submit(r.positions, r.L, r.N, r.rcut, r.twojmax, mala_synth.EGRID, r.T, r.n_electrons)

    big = sorted(reqs, key=lambda r: r.n_points)[-slots:]
    for t in [submit(r) for r in big]:            # every slot runs once, all at the same time
        sv.wait(t, 600)
    st0 = sv.stats()
    side = reqs[:n_side]
    t0 = time.perf_counter()
    outs = [sv.wait(t, 600) for t in [submit(r) for r in side]]
    sat = time.perf_counter() - t0
    sat_rate = len(side) / sat
    sat_pts = sum(r.n_points for r in side) / sat
    streams = []
    for load in loads:
        sub = reqs[:n_main] if abs(load - 0.7) < 1e-9 else side
        lam = load * sat_rate
        arrivals = np.cumsum(-np.log(1.0 - rng.uniform(len(sub))) / lam)
        tickets = []
        t0 = time.perf_counter()
        for r, ta in zip(sub, arrivals):
            while time.perf_counter() - t0 < ta:
                time.sleep(0.0002)
            tickets.append(submit(r))
        outs = [sv.wait(t, 600) for t in tickets]
        span = time.perf_counter() - t0
        lat = np.array([o["t_done"] - o["t_submit"] for o in outs]) * 1000.0
        streams.append({"load": load, "requests": len(sub), "arrival_rate_req_per_s": lam,
                        "p50_latency_ms": float(np.percentile(lat, 50)),
                        "p99_latency_ms": float(np.percentile(lat, 99)),
                        "stream_points_per_s": sum(r.n_points for r in sub) / span,
                        "failed": sum(1 for o in outs if o["status"] != 0)})
    st1 = sv.stats()
    sv.close()
    main_stream = min(streams, key=lambda x: abs(x["load"] - 0.7))
    return {"requests": main_stream["requests"], "slots": slots, "inflight_points_cap": inflight_points,
            "hbm_budget_gb": budget_gb,
            "reserved_gb_per_slot": st0["reserved_bytes_per_slot"] / 2 ** 30,
            "allocations_after_warmup": st1["allocations"] - st0["allocations"],
            "saturation_requests": len(side), "saturation_req_per_s": sat_rate, "saturation_points_per_s": sat_pts,
            "arrival_rate_req_per_s": main_stream["arrival_rate_req_per_s"],
            "p50_latency_ms": main_stream["p50_latency_ms"], "p99_latency_ms": main_stream["p99_latency_ms"],
            "stream_points_per_s": main_stream["stream_points_per_s"],
            "failed": sum(x["failed"] for x in streams), "streams": streams,
            "mix": "fcc n^3*4 (n=2..8) or liquid N~U[32,2048], 298-933 K, ~2800 points/atom, request i from "
                   "SplitMix64(%d * 1000003 + i)" % seed}


def measure(ctx, mala, torch, snap, net, precision, steps, warmup, Bc, fl):
    """Time `steps` fused-path calls after `warmup` untimed ones; stage times
    come from HIP events the library records on its own stream."""
    prec = mala.PREC_FP32 if precision == "fp32" else mala.PREC_BF16
    w = ctx.weights(mala_synth.net_to_blob(net), prec)
    dev = torch.device("cuda", 0)
    dos = torch.empty(mala_synth.EGRID[2], dtype=torch.float64, device=dev)
    dens = torch.empty(snap.n_points, dtype=torch.float64, device=dev)
    res = torch.zeros(mala.RESULT_BYTES, dtype=torch.uint8, device=dev)

    def step():
        ctx.mala_predict(w, snap.positions, snap.L, snap.N, snap.rcut, snap.twojmax, mala_synth.EGRID, snap.T,
                         snap.n_electrons, B_cache=Bc, dos=dos, dens=dens, res=res)

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    ctx.check_device_errors()
    r = mala.read_result(res)
    if r["status"] != 0:
        raise RuntimeError("no Fermi level in warm-up: %s" % r)
    ctx.profile_enable(True)
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    evs[0].record()
    for k in range(steps):
        step()
        evs[k + 1].record()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = ctx.profile_read()
    ctx.profile_enable(False)
    ctx.check_device_errors()
    r = mala.read_result(res)
    elapsed = t1 - t0
    lat = np.array([evs[k].elapsed_time(evs[k + 1]) for k in range(steps)])
    value = snap.n_points * steps / elapsed
    zb_ms, zb_n, zb_pts = prof["zb"]
    zb_avg_ms = zb_ms / max(zb_n, 1)
    achieved = fl["zb"] * zb_pts / max(zb_n, 1) / (zb_avg_ms * 1e-3) / 1e12
    stages = {k: {"ms_per_step": v[0] / steps, "launches_per_step": v[1] / steps} for k, v in prof.items() if v[1]}
    # per-stage algorithmic rate against the peak of the unit that bounds it
    for k, fk, peak in (("ui", "u", PEAK_FP32_VALU_TFLOPS), ("zb", "zb", PEAK_FP32_VALU_TFLOPS),
                        ("mlp_dos", "mlp", PEAK_MFMA_TFLOPS[precision])):
        if k in stages and prof[k][0] > 0:
            tf = fl[fk] * prof[k][2] / (prof[k][0] * 1e-3) / 1e12
            stages[k].update({"tflops": tf, "peak_tflops": peak, "frac": tf / peak})
    ceiling = path_ceiling(fl, precision)
    tpp = measured_traffic(snap.name)
    traffic = tpp * zb_pts / max(zb_n, 1) if tpp is not None else None
    return {
        "value": value, "ms_per_step": 1000.0 * elapsed / steps, "steps": steps, "warmup": warmup,
        "dtype": "f32" if precision == "fp32" else "bf16",
        "config": {"workload": snap.name, "n_points": snap.n_points, "n_atoms": snap.n_atoms,
                   "twojmax": snap.twojmax, "network": "-".join(map(str, net["widths"])),
                   "network_precision": precision, "reductions": "f64", "T_K": snap.T,
                   "n_electrons": snap.n_electrons},
        "latency_ms": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99)),
                       "kind": "single snapshot, back-to-back"},
        "roofline": {"kernel": "k_zb (Z/B contraction)", "bound": "alu", "achieved": achieved,
                     "peak": PEAK_FP32_VALU_TFLOPS, "unit": "TFLOP/s", "frac": achieved / PEAK_FP32_VALU_TFLOPS,
                     "traffic": traffic,
                     "traffic_unit": "bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated, "
                                     "per point x points per launch)",
                     "flops_per_point": fl["zb"], "points_per_launch": zb_pts / max(zb_n, 1),
                     "avg_launch_ms": zb_avg_ms},
        "path_roofline": {"ceiling_points_per_s": ceiling, "frac": value / ceiling,
                          "model": "(U + Z/B) at %.1f TFLOP/s FP32 vector + network at %.0f TFLOP/s %s matrix"
                                   % (PEAK_FP32_VALU_TFLOPS, PEAK_MFMA_TFLOPS[precision], precision)},
        "stages": stages,
        "algorithmic_kflop_per_point": {"u": fl["u"] / 1e3, "zb": fl["zb"] / 1e3, "mlp": fl["mlp"] / 1e3,
                                        "mean_neighbours": fl["mean_neighbours"]},
        "result": {"e_fermi": r["e_fermi"], "e_band_mev_per_atom": 1000 * r["e_band"] / snap.n_atoms,
                   "minus_ts_mev_per_atom": 1000 * r["e_entropy"] / snap.n_atoms, "entropy_kb": r["entropy"]},
        "_w": w, "_dos": dos, "_dens": dens, "_r": r,
    }


def public(rec):
    return {k: v for k, v in rec.items() if not k.startswith("_")}


def sampled_row_errors(ctx, Bc, pts, B_ref, ld_ref, w, torch):
    """Per-row max-norm relative errors of the fused path's cached B rows and
    of their LDOS (GPU network) against the oracle's at the CPU sample."""
    rows = Bc.index_select(0, torch.as_tensor(pts, device="cuda")).contiguous()
    Bg = rows.cpu().double().numpy()
    ld = ctx.mala_ldos_infer(w, rows, mala_synth.EGRID[2]).cpu().double().numpy()
    eb = np.max(np.abs(Bg - B_ref), axis=1) / np.max(np.abs(B_ref), axis=1)
    el = np.max(np.abs(ld - ld_ref), axis=1) / np.max(np.abs(ld_ref), axis=1)
    return {"points": int(len(pts)), "B_max_rel": float(np.max(eb)), "ldos_max_rel": float(np.max(el)),
            "ldos_median_rel": float(np.median(el))}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="slab", choices=sorted(WORKLOADS),
                    help="headline workload (default: the 47,066,880-point slab)")
    ap.add_argument("--precision", default="fp32", choices=["fp32", "bf16"], help="headline network precision")
    ap.add_argument("--headline-only", action="store_true",
                    help="time only the headline workload and precision (for profiler runs)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=32768)
    ap.add_argument("--serve-requests", type=int, default=1000,
                    help="requests of the 0.7x Poisson stream per precision (0 disables serving)")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the lines outside the metric (Gaussian descriptors, both VJPs, grid ACE)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run the plain device copies that calibrate the HBM byte counters")
    ap.add_argument("--traffic-summary", nargs=4, metavar="DIR",
                    help="write the calibrated k_zb traffic profile from four rocprofv3 --pmc output "
                         "directories (kernel FETCH_SIZE, WRITE_SIZE; copy FETCH_SIZE, WRITE_SIZE); no GPU")
    ap.add_argument("--probe-kernels", action="store_true",
                    help="run each kernel family once on the 256-atom solid (a short program for counter runs)")
    ap.add_argument("--counter-summary", nargs="+", metavar="ARG",
                    help="OUT_NAME COMMAND_TEMPLATE DIR...: write a profiles/ markdown table of rocprofv3 --pmc "
                         "counters per kernel from one or more output directories; no GPU")
    ap.add_argument("--stats-summary", nargs=4, metavar=("PROF_DIR", "BENCH_LOG", "OUT_NAME", "COMMAND"),
                    help="write a profiles/ markdown table from a rocprofv3 --kernel-trace --stats run; no GPU")
    a = ap.parse_args()
    if a.stats_summary:
        stats_summary(*a.stats_summary)
        return
    if a.traffic_summary:
        traffic_summary(*a.traffic_summary, workload=a.workload)
        return
    if a.counter_summary:
        counter_summary(a.counter_summary[0], a.counter_summary[1], a.counter_summary[2:])
        return
    if a.copy_calibration:
        copy_calibration()
        return
    if a.probe_kernels:
        probe_kernels()
        return
    if a.gpus != 1:
        print("bench.py measures one GPU: the path shards by grid slabs with one 2 KB DOS all-reduce, "
              "which this library does not implement (use --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2411_19617_amd as mala

    mala.lib()
    ctx = mala.Context(0)
    dev = torch.device("cuda", 0)
    snap, net = WORKLOADS[a.workload][0](), WORKLOADS[a.workload][1]()
    fl = flops_per_point(snap, net["widths"])
    Bc = torch.empty((snap.n_points, mala.n_descriptors(snap.twojmax)), dtype=torch.float32, device=dev)
    head = measure(ctx, mala, torch, snap, net, a.precision, a.steps, a.warmup, Bc, fl)
    print("headline %s %s: %.4g points/s" % (snap.name, a.precision, head["value"]), file=sys.stderr, flush=True)
    out = {"metric": METRIC, "value": head["value"], "unit": "grid points/s", "n_gpus": 1, "steps": a.steps,
           "warmup": a.warmup, "ms_per_step": head["ms_per_step"], "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": head["dtype"], "data": "synthetic"}
    out.update({k: v for k, v in public(head).items() if k not in out and k not in ("steps", "warmup")})
    if a.workload == "slab":
        out["errors_vs_oracle"] = slab_sample_errors(ctx, snap, head["_w"], Bc, head["_dos"], head["_r"], torch)
    else:
        out["errors_vs_oracle"] = errors_vs_oracle(a.workload, snap, head["_dos"], head["_r"], head["_dens"])
    cpu = None
    if not a.no_cpu_baseline:
        cpu, pts, B_ref, ld_ref = cpu_baseline(snap, net, a.cpu_sample)
        cpu["errors_on_sample"] = sampled_row_errors(ctx, Bc, pts, B_ref, ld_ref, head["_w"], torch)
        print("cpu baseline: %.4g points/s" % cpu["value"], file=sys.stderr, flush=True)
    if a.headline_only:
        if cpu:
            out["cpu_baseline"] = cpu
        print(json.dumps(out), flush=True)
        ctx.close()
        return
    other = "bf16" if a.precision == "fp32" else "fp32"
    pf = measure(ctx, mala, torch, snap, net, other, a.steps, a.warmup, Bc, fl)
    rec = public(pf)
    if a.workload == "slab":
        rec["errors_vs_oracle"] = slab_sample_errors(ctx, snap, pf["_w"], Bc, pf["_dos"], pf["_r"], torch)
    else:
        rec["errors_vs_oracle"] = errors_vs_oracle(a.workload, snap, pf["_dos"], pf["_r"], pf["_dens"])
    rec["e_band_vs_headline_mev_per_atom"] = abs(pf["_r"]["e_band"] - head["_r"]["e_band"]) * 1000.0 / snap.n_atoms
    if cpu:
        rec["errors_on_sample"] = sampled_row_errors(ctx, Bc, pts, B_ref, ld_ref, pf["_w"], torch)
    out["precision_form" if other == "bf16" else "plain_form"] = rec
    print("%s %s: %.4g points/s" % (snap.name, other, pf["value"]), file=sys.stderr, flush=True)
    del head, pf, Bc
    torch.cuda.empty_cache()

    # the 729,000-point 256-atom solid in both forms (the paper's per-GPU scale)
    if a.workload != "paper_solid":
        ps, pnet = WORKLOADS["paper_solid"][0](), WORKLOADS["paper_solid"][1]()
        pfl = flops_per_point(ps, pnet["widths"])
        pB = torch.empty((ps.n_points, mala.n_descriptors(ps.twojmax)), dtype=torch.float32, device=dev)
        solid = {}
        for prec in ("fp32", "bf16"):
            m = measure(ctx, mala, torch, ps, pnet, prec, max(a.steps, 20), max(a.warmup, 3), pB, pfl)
            rec = public(m)
            rec["errors_vs_oracle"] = errors_vs_oracle("paper_solid", ps, m["_dos"], m["_r"], m["_dens"])
            solid[prec] = rec
            print("paper_solid %s: %.4g points/s" % (prec, m["value"]), file=sys.stderr, flush=True)
        out["paper_solid"] = solid
        del pB
        torch.cuda.empty_cache()
    if not a.no_extras:
        es = WORKLOADS["paper_solid"][0]()
        efl = flops_per_point(es, WORKLOADS["paper_solid"][1]()["widths"])
        out["gaussian_descriptors"] = gaussian_bench(ctx, es, torch)
        out["network_vjp"] = network_vjp_bench(ctx, mala, es, WORKLOADS["paper_solid"][1](), torch)
        out["descriptor_vjp"] = descriptor_adjoint_bench(ctx, es, torch)
        out["ace_descriptors"] = ace_bench(ctx, mala, es, efl["mean_neighbours"], torch)
        out["ace4_descriptors"] = ace4_bench(ctx, mala, es, efl["mean_neighbours"], torch)
        print("extras done", file=sys.stderr, flush=True)
    if a.serve_requests > 0:
        sv = {}
        reqs = mala_synth.serving_mix(max(a.serve_requests, 200), 5, workers=min(16, len(os.sched_getaffinity(0))))
        print("serving mix generated", file=sys.stderr, flush=True)
        for prec in ("fp32", "bf16"):
            sv[prec] = serving_bench(mala, mala.PREC_FP32 if prec == "fp32" else mala.PREC_BF16,
                                     reqs, a.serve_requests, n_side=min(200, a.serve_requests))
            print("serving %s: p50 %.1f ms p99 %.1f ms" % (prec, sv[prec]["p50_latency_ms"],
                                                           sv[prec]["p99_latency_ms"]), file=sys.stderr, flush=True)
        out["serving"] = sv
        out["latency_ms"]["serving_p50"] = sv[a.precision]["p50_latency_ms"]
        out["latency_ms"]["serving_p99"] = sv[a.precision]["p99_latency_ms"]
    if cpu:
        out["cpu_baseline"] = cpu
    print(json.dumps(out), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
