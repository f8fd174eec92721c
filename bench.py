#!/usr/bin/env python3
"""Walker-steps/s of the k-point AFQMC block on one MI355X.

Workload (3x3x3 mesh, m = 26 bands per k, nocc = 4, nchol = 208 per Q, 64 walkers,
dt = 0.005): seeded synthetic inputs shaped like carbon in the diamond structure with
a GTH-DZVP basis.  One timed step is one block as the paper times it: 20 propagation
steps (force bias, HS potential, 6th-order Taylor propagation, new Green's function and
phaseless weights), one walker re-orthonormalisation, one local-energy evaluation.

Paths on the same inputs, named by the precision of the step contractions (force bias,
HS potential, Taylor products) and of the local energy: FP64 throughout, FP32
throughout, BF16X3 throughout, and BF16X3 steps with an FP64 or an FP32 energy
(overlap, inverse, QR and energy sums are FP64 in every path).  The reported value is
the walker-steps/s of the fastest path whose local energies, evaluated on the FP64
path's walkers after a block, differ from the FP64 energies by at most 1e-5 Ha/cell on
every walker that carries weight and in the weighted (mixed) estimate; the FP64 path
itself matches the FP64 CPU oracle to 1e-10 Ha/cell (GPU parity tests).  Every path
also reports how far its own trajectory ends from the FP64 one and the error of one
of its steps from the common state.

Prints one JSON line on stdout; progress goes to stderr.
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

METRIC = "walker-steps/s at Nk=27 M=26, mixed vs FP64 GPU, |ΔE_loc|≤1e-5 Ha/cell"
# dense MFMA TFLOP/s, MI355X; BF16-split counts its three BF16 passes per product
PEAK = {"fp64": 78.6, "fp32": 157.3, "bf16x3": 2500.0 / 3, "int8x5": 5000.0, "int8x4": 5000.0}
TOL = 1e-5  # Ha per cell
# the paths of the counter runs (every kernel class of the FP64, BF16X3 and int8 paths)
PMC_PATHS = "fp64,bf16x3,bf16x3+int8x4E,bf16x3+int8x5E"
# path -> (precision of the step contractions, precision of the local energy)
PATHS = {
    "fp64": ("fp64", "fp64"),
    "fp32": ("fp32", "fp32"),
    "bf16x3": ("bf16x3", "bf16x3"),
    "bf16x3+fp64E": ("bf16x3", "fp64"),
    "bf16x3+fp32E": ("bf16x3", "fp32"),
    "bf16x3+int8x5E": ("bf16x3", "int8x5"),
    "bf16x3+int8x4E": ("bf16x3", "int8x4"),
}
ENERGY_CLASSES = ("exchange", "energy_rest", "exchange_bwd")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_flops(name, c):
    """Algorithmic (executed) flops of one launch of a kernel class; 8 flops per complex MAC."""
    nk, m, nocc, C, W = c["nk"], c["m"], c["nocc"], c["nchol"], c["nwalk"]
    N, n = nk * m, nk * nocc
    if name == "taylor":
        return 8.0 * W * N * N * n
    if name == "vhs":
        return 8.0 * W * nk * nk * m * m * C
    if name == "vbias":
        return 8.0 * W * nk * nk * nocc * m * C
    if name == "exchange":
        # one T1 GEMM per (Q, k, k') triple: time-reversal pairs share the second GEMM
        return 8.0 * W * nk ** 3 * nocc * nocc * C * m
    return None


CSRC = os.path.join(os.path.dirname(os.path.abspath(__file__)), "paper_2003_09468_amd", "csrc")
COMMON = ["kcommon.h", "batch.h", "cgemm.h"]
# the sources each kernel class is built from (counter figures are kept while they match)
KERNEL_FILES = {
    "taylor": COMMON + ["propagate.hip"], "bhalf": COMMON + ["propagate.hip"],
    "vhs": COMMON + ["fields.hip"], "vbias": COMMON + ["fields.hip"],
    "exchange": COMMON + ["energy.hip"], "greens_solve": COMMON + ["greens.hip"],
    "greens_gj": COMMON + ["greens.hip"],
}
# kernel-name patterns of each class in a rocprofv3 trace
KERNEL_NAMES = {
    "taylor": "OpTaylor<{t}>", "vhs": "OpVhs<{t}>", "vbias": "OpVbias<{t}>",
    "exchange": "exchange_kernel<{t}", "greens_solve": "OpGreensSolve",
    "greens_gj": "gj_", "bhalf": "OpBhalf<{t}>",
}
# the BF16X3 kernels of the same classes
KERNEL_NAMES_BF16X3 = {
    "taylor": "taylor_bf16x3_kernel", "vhs": "vhs_bf16x3_kernel",
    "vbias": "vbias_bf16x3_kernel", "exchange": "exchange_bf16x3",
}


def kernel_source_hash(files=None):
    """Hash of HIP sources (all of them, or the given files)."""
    import hashlib
    names = sorted(f for f in os.listdir(CSRC) if f.endswith((".hip", ".h"))) \
        if files is None else sorted(set(files))
    h = hashlib.sha256()
    for f in names:
        h.update(f.encode())
        h.update(open(os.path.join(CSRC, f), "rb").read())
    return h.hexdigest()[:16]


def measured_traffic(kernel, prec):
    """HBM bytes per launch of a kernel class from the committed counter summary, if it was
    taken for the kernel's current sources (else None)."""
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "profiles",
                        "traffic_c1.json")
    try:
        rec = json.load(open(path))
    except (OSError, ValueError):
        return None
    ent = rec.get("kernels", {}).get(f"{kernel}_{prec}")
    if ent is None or kernel not in KERNEL_FILES:
        return None
    if ent.get("source_hash") != kernel_source_hash(KERNEL_FILES[kernel]):
        return None
    return ent.get("bytes_per_launch")


def _pmc_rows(path, counter):
    import csv
    out = []
    for r in csv.DictReader(open(path)):
        if r["Counter_Name"] == counter:
            out.append((r["Kernel_Name"], float(r["Counter_Value"])))
    return out


def reduce_pmc(fetch_csv, write_csv):
    """Per-launch HBM bytes of the c1 FP64 and BF16X3 kernels from two counter runs
    (FETCH_SIZE, then WRITE_SIZE, KiB per dispatch), each scaled by what it reads for the
    1 GiB copy; writes profiles/traffic_c1.json and profiles/traffic_c1.md."""
    from synth.kpt_inputs import config_shapes
    c = config_shapes("c1")
    W, nk, m, nocc, C = c["nwalk"], c["nk"], c["m"], c["nocc"], c["nchol"]
    N, n = nk * m, nk * nocc
    fetch, write = _pmc_rows(fetch_csv, "FETCH_SIZE"), _pmc_rows(write_csv, "WRITE_SIZE")

    def copy_kib(rows):
        v = [x for name, x in rows if "copyBuffer" in name]
        return max(v) if v else None
    gib = float(1 << 30)
    fs = gib / (copy_kib(fetch) * 1024.0)
    ws = gib / (copy_kib(write) * 1024.0)
    algo = {
        "taylor": (16.0 * W * (N * N + 2 * N * n), 16.0 * W * N * n * (1 + 5.0 / 6.0)),
        "vhs": (16.0 * (nk * nk * m * m * C + W * nk * C), 16.0 * W * N * N),
        "exchange": (16.0 * (nk * nk * nocc * m * C + W * n * N), 16.0 * nk ** 3 * W),
    }
    # BF16X3: planes are 8 bytes per complex entry (four bf16), complex64 8, complex128 16;
    # the Taylor launches are the six nested steps (five write planes, the last the FP64
    # result), L and Lh planes are padded to 32 along g and r
    KP, CP, KPm = 32 * ((N + 31) // 32), 32 * ((C + 31) // 32), 32 * ((m + 31) // 32)
    # the HS potential reads the half store of L (one slot per (Q, -Q) pair)
    from paper_2003_09468_amd.binding import ls_slots
    nq = ls_slots(c["mesh"])
    algo_bf = {
        "taylor": (8.0 * W * N * N + 8.0 * W * n * KP + (5 * 8.0 + 16.0) / 6 * W * N * n,
                   (5 * 8.0 * W * n * KP + 16.0 * W * N * n) / 6),
        "vhs": (8.0 * (nq * nk * m * m * CP + W * nk * CP), 8.0 * W * N * N),
        "exchange": (8.0 * nk * nk * C * nocc * KPm + 16.0 * W * n * N, 16.0 * nk ** 3 * W),
    }
    # the int8 exchanges read ND of the five stored digits per element of the [Re | Im] rows
    # (2m padded to 64) and the row exponents, and Gh
    KP8 = 64 * ((2 * m + 63) // 64)
    algo_i8 = {nd: {"exchange": (nk * nk * C * nocc * (nd * KP8 + 4.0) + 16.0 * W * n * N,
                                 16.0 * nk ** 3 * W)} for nd in (4, 5)}
    rec = {"workload": "c1: mesh 3x3x3, m=26, nocc=4, nchol=208, 64 walkers (FP64, BF16X3 "
                       "and int8-split energy paths)",
           "fetch_scale": fs, "write_scale": ws, "kernels": {}}
    for prec, names, alg in (("fp64", {k: v.format(t="double") for k, v in KERNEL_NAMES.items()},
                              algo),
                             ("bf16x3", KERNEL_NAMES_BF16X3, algo_bf),
                             ("int8x4", {"exchange": "exchange_int8_kernel<1, 4>"}, algo_i8[4]),
                             ("int8x5", {"exchange": "exchange_int8_kernel<1, 5>"}, algo_i8[5])):
        for k, pat in names.items():
            fv = [x for name, x in fetch if pat in name]
            wv = [x for name, x in write if pat in name]
            if not fv or not wv:
                continue
            fb = sum(fv) / len(fv) * 1024.0 * fs
            wb = sum(wv) / len(wv) * 1024.0 * ws
            e = {"launches": len(fv), "fetch_bytes_per_launch": fb,
                 "write_bytes_per_launch": wb, "bytes_per_launch": fb + wb,
                 "source_hash": kernel_source_hash(KERNEL_FILES[k])}
            if k in alg:
                e["algorithmic_read_bytes"], e["algorithmic_write_bytes"] = alg[k]
            rec["kernels"][f"{k}_{prec}"] = e
    base = os.path.join(os.path.dirname(os.path.abspath(__file__)), "profiles")
    json.dump(rec, open(os.path.join(base, "traffic_c1.json"), "w"), indent=1)
    lines = ["# HBM traffic per launch, c1 FP64, BF16X3 and int8-split energy paths "
             "(rocprofv3 counters)", "",
             "Commands (repository root, on the MI355X; each counter in its own run):", "",
             "```", "cd /tmp && export TMPDIR=/tmp && cd \"$GRAFT_REPO_ROOT\"",
             "timeout -s KILL 400 rocprofv3 --pmc FETCH_SIZE --output-format csv "
             "-d gpurun_out/pmc_fetch -o run -- \\",
             f"    python3 bench.py --steps 1 --warmup 0 --no-cpu-baseline --calib-copy "
             f"--prec {PMC_PATHS}",
             "timeout -s KILL 400 rocprofv3 --pmc WRITE_SIZE --output-format csv "
             "-d gpurun_out/pmc_write -o run -- \\",
             f"    python3 bench.py --steps 1 --warmup 0 --no-cpu-baseline --calib-copy "
             f"--prec {PMC_PATHS}",
             "python3 bench.py --reduce-pmc gpurun_out/pmc_fetch/run_counter_collection.csv "
             "gpurun_out/pmc_write/run_counter_collection.csv", "```", "",
             f"Scale: the plain 1 GiB device copy (`--calib-copy`) reads as FETCH_SIZE = "
             f"{gib / fs / 2**20:.1f} MiB and WRITE_SIZE = {gib / ws / 2**20:.1f} MiB, so "
             f"FETCH_SIZE is multiplied by {fs:.3f} and WRITE_SIZE by {ws:.3f}.", "",
             "Each row carries the hash of the kernel's own sources; bench.py reports the "
             "figure only while they hash the same.", "",
             "| kernel | launches | read MB/launch | write MB/launch | algorithmic read MB | "
             "algorithmic write MB | source hash |",
             "|:--|--:|--:|--:|--:|--:|:--|"]
    for k, e in rec["kernels"].items():
        ar = e.get("algorithmic_read_bytes")
        aw = e.get("algorithmic_write_bytes")
        lines.append(f"| {k} | {e['launches']} | {e['fetch_bytes_per_launch'] / 1e6:.1f} | "
                     f"{e['write_bytes_per_launch'] / 1e6:.1f} | "
                     f"{'' if ar is None else f'{ar / 1e6:.1f}'} | "
                     f"{'' if aw is None else f'{aw / 1e6:.1f}'} | {e['source_hash']} |")
    lines += ["", "Algorithmic bytes: a Taylor term reads vhs (W (nk m)^2), T_{j-1} and the FP64 "
              "accumulator and writes T_j (5 of 6 terms) and the accumulator; the HS potential "
              "reads L once and writes vhs; the exchange reads Lh and Gh once.  BF16X3 (8 bytes "
              "per split complex entry): a nested Taylor step reads the complex64 potential, "
              "the walker planes and T_0 (the last step the FP64 T_0) and writes the next "
              "planes (the last step the FP64 result); the HS potential reads the half store of "
              "the L planes and the combined-field planes and writes the complex64 potential; "
              "the exchange reads the Lh planes and Gh.  Int8 split: the exchange reads four "
              "(INT8X4) or five (INT8X5) int8 digits per element of the [Re | Im] rows of Lh "
              "(2m padded to 64) with their exponents, and Gh."]
    open(os.path.join(base, "traffic_c1.md"), "w").write("\n".join(lines) + "\n")
    print(json.dumps(rec["kernels"], indent=1))


def reduce_mfma(csv_path, out_md, title, command):
    """MFMA utilisation per kernel from one counter run (SQ_VALU_MFMA_BUSY_CYCLES,
    GRBM_GUI_ACTIVE, SQ_INSTS_VALU_MFMA_MOPS_*): busy cycles / (active cycles x 1024 SIMDs),
    and the MFMA flops counted by the hardware (MOPS x 512)."""
    import csv
    per, dur = {}, {}
    for r in csv.DictReader(open(csv_path)):
        key = (r["Kernel_Name"], r["Dispatch_Id"])
        per.setdefault(key, {})[r["Counter_Name"]] = float(r["Counter_Value"])
        dur[key] = float(r["End_Timestamp"]) - float(r["Start_Timestamp"])
    agg = {}
    for key, v in per.items():
        name = key[0]
        if "afqmc" not in name:
            continue
        short = name.replace("void ", "").replace("afqmc::", "").split("(")[0]
        a = agg.setdefault(short, {"n": 0, "busy": 0.0, "active": 0.0, "mops": 0.0, "ns": 0.0})
        a["n"] += 1
        a["busy"] += v.get("SQ_VALU_MFMA_BUSY_CYCLES", 0.0)
        # GRBM_GUI_ACTIVE arrives summed over the 8 XCDs (8x the dispatch's wall cycles)
        a["active"] += v.get("GRBM_GUI_ACTIVE", 0.0) / 8.0
        a["mops"] += sum(x for c, x in v.items() if c.startswith("SQ_INSTS_VALU_MFMA_MOPS"))
        a["ns"] += dur[key]
    rows = sorted(agg.items(), key=lambda kv: -kv[1]["active"])
    lines = [f"# MFMA utilisation: {title}", "", "Command (repository root, on the MI355X):", "",
             "```", "cd /tmp && export TMPDIR=/tmp && cd \"$GRAFT_REPO_ROOT\"", command,
             f"python3 bench.py --reduce-mfma <run_counter_collection.csv> {out_md}", "```", "",
             "MFMA busy = SQ_VALU_MFMA_BUSY_CYCLES / (active cycles x 1024 SIMDs), with the "
             "active cycles GRBM_GUI_ACTIVE / 8 (the counter arrives summed over the 8 XCDs: "
             "8x the dispatch's wall time in cycles); MFMA flops = SQ_INSTS_VALU_MFMA_MOPS_* "
             "x 512 (the hardware count, including zero padding and the three passes of the "
             "BF16 split), rate = flops / dispatch time (counter runs serialise dispatches).", "",
             "| kernel | dispatches | us/dispatch | MFMA busy % | MFMA Gflop/dispatch | "
             "MFMA TFLOP/s |", "|:--|--:|--:|--:|--:|--:|"]
    for k, a in rows[:24]:
        util = 100.0 * a["busy"] / (a["active"] * 1024.0) if a["active"] else 0.0
        gf = a["mops"] * 512 / a["n"] / 1e9
        us = a["ns"] / a["n"] / 1e3
        lines.append(f"| `{k}` | {a['n']} | {us:.1f} | {util:.1f} | {gf:.2f} | "
                     f"{gf / us * 1e3 if us else 0.0:.1f} |")
    open(out_md, "w").write("\n".join(lines) + "\n")
    print("\n".join(lines))


def run_block(p, xs, bufs, E):
    """One block: the steps (each Gh feeds only the next force bias, so reduced precisions
    form it by the FP32 product; the last step's re-orthonormalisation forms it in FP64),
    then the local energy."""
    nsteps = xs.shape[0]
    for s in range(nsteps):
        p.step(xs[s], ortho=(s == nsteps - 1), bufs=bufs, reduced_gh=True)
    return p.energy(out=E)


def make_problem(s, U0, prec, torch, tune=True):
    """Problem with its static data prepared and, once per shape, the tile autotuner run
    (setup, outside any timed region, like prepare)."""
    from paper_2003_09468_amd import KptProblem, KptBatch
    p = KptProblem(s.mesh, s.m, s.nocc, s.nchol, U0.shape[0], s.dt, torch.from_numpy(s.L),
                   torch.from_numpy(s.A), prec=prec)
    p.prepare(torch.from_numpy(s.H1))
    if tune:
        p.set_walkers(torch.from_numpy(U0))
        p.greens()
        KptBatch([p]).autotune()
    return p


def reset(p, U0d):
    p.set_walkers(U0d)
    p.weight.fill_(1.0)
    p.greens()


def bench_path(name, p, U0d, xs, args, torch, cfg):
    import paper_2003_09468_amd as lib
    W, N = p.nwalk, p.nk * p.m
    vdt = torch.complex64 if lib.step_prec(p.prec) != lib.PREC_FP64 else torch.complex128
    bufs = {
        "xbar": torch.empty((W, p.nk, p.nchol, 2), dtype=torch.complex128, device="cuda"),
        "X": torch.empty((W, p.nk, p.nchol), dtype=torch.complex128, device="cuda"),
        "vhs": torch.empty((W, N, N), dtype=vdt, device="cuda"),
    }
    E = torch.empty((W, 3), dtype=torch.complex128, device="cuda")
    reset(p, U0d)
    # first block from the common start: the path's own trajectory and its end state
    first = {"E": run_block(p, xs, bufs, E).clone()}
    for k in ("U", "Gh", "logdet", "weight", "status"):
        first[k] = getattr(p, k).clone()
    for _ in range(args.warmup):
        run_block(p, xs, bufs, E)
    torch.cuda.synchronize()
    # throughput: no per-kernel events in the timed blocks (two event records per launch
    # cost about 2 ms per block)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        run_block(p, xs, bufs, E)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    # per-kernel durations: the same blocks again, each launch bracketed by HIP events on
    # its stream
    lib.timing_enable(True, 1 << 16)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    for _ in range(args.steps):
        run_block(p, xs, bufs, E)
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    lib.timing_enable(False)
    kern = {}
    for kc in lib.KERNEL_CLASSES:
        ms, n = lib.timing_read(kc)
        if n:
            kern[kc] = {"ms_total": ms / args.steps, "launches": n // args.steps,
                        "ms_per_launch": ms / n}
    # comb population control, the step between blocks (not part of the timed block)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    p.population_control(0.5)
    ev[0].record()
    for r in range(5):
        p.population_control((r + 0.5) / 5)
    ev[1].record()
    torch.cuda.synchronize()
    pc_ms = ev[0].elapsed_time(ev[1]) / 5
    dt = (t1 - t0) / args.steps
    ws = W * xs.shape[0] / dt
    log(f"[{name}] block {dt * 1e3:.2f} ms  -> {ws:.1f} walker-steps/s "
        f"(with per-kernel events {(t3 - t2) / args.steps * 1e3:.2f} ms); "
        f"population control {pc_ms:.3f} ms")
    for k, v in sorted(kern.items(), key=lambda kv: -kv[1]["ms_total"]):
        log(f"    {k:13s} {v['ms_total']:9.3f} ms/block  {v['launches']:4d} launches  "
            f"{v['ms_per_launch']:.4f} ms/launch")
    return {"ms_per_block": dt * 1e3, "walker_steps_per_s": ws, "kernels": kern,
            "ms_per_block_with_kernel_events": (t3 - t2) / args.steps * 1e3,
            "population_control_ms": round(pc_ms, 4)}, first


def kernel_prec(path, kernel):
    """Precision a kernel class of a path runs in (the key of PEAK and of the traffic
    summary)."""
    sp, ep = PATHS[path]
    pk = ep if kernel in ENERGY_CLASSES else sp
    # in a BF16X3 stage the force bias, HS potential, Taylor terms and exchange run on the
    # BF16 split; the adjoint is FP32
    if pk == "bf16x3" and kernel not in ("vhs", "taylor", "exchange", "vbias"):
        pk = "fp32"
    # the int8 split replaces only the exchange contraction; the rest of that energy is FP64
    if pk in ("int8x5", "int8x4"):
        pk = pk if kernel == "exchange" else "fp64"
    return pk


def roofline(path_res, path, cfg, kernel=None):
    """Roofline of one kernel class of a path (default: the one with the most time per
    block)."""
    kern = path_res["kernels"]
    dom = kernel if kernel is not None else max(kern, key=lambda k: kern[k]["ms_total"])
    if dom not in kern:
        return None
    fl = kernel_flops(dom, cfg)
    if fl is None:
        return {"kernel": dom, "bound": "alu", "achieved": None, "peak": None, "unit": None,
                "frac": None, "traffic": None}
    ach = fl / (kern[dom]["ms_per_launch"] * 1e-3) / 1e12
    pk = kernel_prec(path, dom)
    return {"kernel": dom, "precision": pk, "bound": "mfma", "achieved": round(ach, 3),
            "peak": PEAK[pk], "unit": "TFLOP/s", "frac": round(ach / PEAK[pk], 4),
            "traffic": measured_traffic(dom, pk), "flops_per_launch": fl}


def exchange_roofline(path_res, path, cfg):
    """Roofline of the exchange; in the BF16X3 mode also the MFMA work the hardware executes
    (three BF16 passes, the contraction index r padded to a multiple of 32) against the
    dense BF16 peak."""
    r = roofline(path_res, path, cfg, "exchange")
    if r is not None and r["precision"] in ("int8x5", "int8x4"):
        # per complex T1 entry: two real products, 15 (10) digit pairs, K = 2m padded to 64
        kp8 = 64 * ((2 * cfg["m"] + 63) // 64)
        pairs = 15 if r["precision"] == "int8x5" else 10
        ex = r["flops_per_launch"] / (8.0 * cfg["m"]) * 2 * pairs * kp8 * 2
        ms = path_res["kernels"]["exchange"]["ms_per_launch"]
        r["executed_int8_ops_per_launch"] = ex
        r["executed_int8_tops"] = round(ex / (ms * 1e-3) / 1e12, 1)
        r["executed_frac_of_5000"] = round(ex / (ms * 1e-3) / 5.0e15, 4)
        r["fp64_equivalent_frac_of_78.6"] = round(r["achieved"] / 78.6, 4)
        return r
    if r is None or r["precision"] != "bf16x3":
        return r
    kp = 32 * ((cfg["m"] + 31) // 32)
    ex = 3.0 * r["flops_per_launch"] * kp / cfg["m"]
    ms = path_res["kernels"]["exchange"]["ms_per_launch"]
    r["executed_bf16_flops_per_launch"] = ex
    r["executed_bf16_tflops"] = round(ex / (ms * 1e-3) / 1e12, 1)
    r["executed_frac_of_2500"] = round(ex / (ms * 1e-3) / 2.5e15, 4)
    return r


def energy_evals(v, cfg):
    """Walker energy evaluations per second: walkers / time of the energy's launches (its
    Cholesky-vector traces X for the Coulomb term, which run as one more force-bias launch,
    the exchange, and the one-body/Coulomb/reduction kernels)."""
    k = v["kernels"]
    ms = sum(k[c]["ms_total"] for c in ("exchange", "energy_rest") if c in k)
    vb = k.get("vbias")
    if vb and vb["launches"] > cfg["nsteps"]:
        ms += vb["ms_per_launch"] * (vb["launches"] - cfg["nsteps"])
    return round(cfg["nwalk"] * 1e3 / ms, 2) if ms > 0 else None


DTYPE = {"fp64": "f64", "fp32": "f32+f64", "bf16x3": "bf16x3+f32+f64",
         "bf16x3+fp64E": "bf16x3+f64", "bf16x3+fp32E": "bf16x3+f32+f64",
         "bf16x3+int8x5E": "bf16x3+int8x5+f64", "bf16x3+int8x4E": "bf16x3+int8x4+f64"}


def step_from(p, st, x0):
    """One step of p from a saved walker state (U, Gh, logdet, weight, status); returns the
    new U, Gh and weights (device copies)."""
    for k in ("U", "Gh", "logdet", "weight", "status"):
        getattr(p, k).copy_(st[k])
    p.step(x0, reduced_gh=True)
    return {"U": p.U.clone(), "Gh": p.Gh.clone(), "weight": p.weight.clone()}


def overlap_cond(U, A):
    """2-norm condition number of each walker's overlap matrix A^H U (A block diagonal)."""
    import numpy as np
    nk, m, nocc = A.shape
    U = np.asarray(U).reshape(U.shape[0], nk, m, -1)
    O = np.einsum("kpa,wkpj->wkaj", A.conj(), U).reshape(U.shape[0], nk * nocc, -1)
    return np.linalg.cond(O)


def _stats(d, mask=None):
    import numpy as np
    d = np.asarray(d, dtype=float)
    out = {"max": float(d.max()), "median": float(np.median(d))}
    if mask is not None:
        out["live_walkers"] = int(mask.sum())
        out["live_max"] = float(d[mask].max()) if mask.any() else None
    return out


def accuracy_report(p64, first, st64, initial, s, cfg):
    """Errors of every path against the FP64 path, |dE_L| in Ha per cell.

    trajectory: each path propagated on its own from the same start for one block
      (measures the chaos of the walk as much as the precision: an FP64 run with 1e-13
      relative noise on the fields ends about 1e-6 away);
    energy_at_fp64_state: the path's local-energy stage on the FP64 path's walkers after
      that block (the tolerance applies here: on the walkers that carry weight and to the
      weighted mixed estimate);
    step_at_fp64_state: one step of the path from that state, its energies evaluated in
      FP64 (the error one step of its propagation adds);
    initial_walkers: the energy stage on the initial walkers.
    A walker is live when its weight is positive."""
    import numpy as np
    nk = cfg["nk"]

    def tot(E):
        return np.asarray(E).sum(1) / nk

    def mixed(e, w):
        return complex((w * e).sum() / w.sum()) if w.sum() > 0 else complex("nan")

    f64 = first["fp64"]
    e64 = tot(f64["E"].cpu().numpy())
    w64 = f64["weight"].cpu().numpy()
    live = w64 > 0
    cond = overlap_cond(f64["U"].cpu().numpy(), s.A)
    st = st64["step"]
    e64s = tot(p64.energy(Gh=st["Gh"]).cpu().numpy())
    w64s = st["weight"].cpu().numpy()
    acc = {"tolerance": TOL, "unit": "Ha/cell",
           "reading": "the tolerance applies to the local energy at a common walker state "
                      "(the FP64 path's walkers after one block): max |dE_L| over the live "
                      "walkers and |dE| of the weighted mixed estimate; the other figures "
                      "are reported beside it",
           "fp64_state": {"walkers": int(len(w64)), "live_walkers": int(live.sum()),
                          "mixed_energy_per_cell": [float(mixed(e64, w64).real),
                                                    float(mixed(e64, w64).imag)],
                          "cond_overlap": _stats(cond, live),
                          "cond_overlap_min": float(cond.min())}}
    for name in first:
        if name == "fp64":
            continue
        f = first[name]
        ent = {}
        e = tot(f["E"].cpu().numpy())
        w = f["weight"].cpu().numpy()
        both = live & (w > 0)
        ent["trajectory"] = _stats(np.abs(e - e64), both)
        ent["trajectory"]["mixed_abs_dE"] = abs(mixed(e, w) - mixed(e64, w64))
        o = st64["others"][name]
        e2 = tot(o["E"])
        ent["energy_at_fp64_state"] = _stats(np.abs(e2 - e64), live)
        ent["energy_at_fp64_state"]["mixed_abs_dE"] = abs(mixed(e2, w64) - mixed(e64, w64))
        so = o["step"]
        e3 = tot(p64.energy(Gh=so["Gh"]).cpu().numpy())
        w3 = so["weight"].cpu().numpy()
        both3 = (w3 > 0) & (w64s > 0)
        ent["step_at_fp64_state"] = _stats(np.abs(e3 - e64s), both3)
        dU = ((so["U"] - st["U"]).abs().pow(2).sum((1, 2)).sqrt() /
              st["U"].abs().pow(2).sum((1, 2)).sqrt()).cpu().numpy()
        ent["step_at_fp64_state"]["rel_dU"] = _stats(dU)
        ent["initial_walkers"] = _stats(np.abs(initial[name] - initial["fp64"]))
        es = ent["energy_at_fp64_state"]
        ent["meets_tolerance"] = bool(es["live_max"] is not None and es["live_max"] <= TOL
                                      and es["mixed_abs_dE"] <= TOL)
        acc[name] = ent
        log(f"accuracy {name}: energy at the FP64 state: live max {es['live_max']:.3e}, "
            f"mixed {es['mixed_abs_dE']:.3e}, all-walker max {es['max']:.3e} Ha/cell; "
            f"one step from it: live max {ent['step_at_fp64_state']['live_max']} Ha/cell; "
            f"own trajectory: live max {ent['trajectory']['live_max']}, mixed "
            f"{ent['trajectory']['mixed_abs_dE']:.3e}; initial walkers max "
            f"{ent['initial_walkers']['max']:.3e}")
    return acc


def _oracle_rate(kp, s, pre, U0, xs_host, nw, ne):
    """Oracle walker-steps/s from one step of nw walkers, QR + G of nw walkers and the
    local energy of ne walkers; returns (rate, description)."""
    import numpy as np
    U = U0[:nw]
    Gh, ld = kp.greens(U, s.A)
    t = time.perf_counter()
    out = kp.step(U, ld, np.ones(nw), xs_host[0][:nw], pre, s.A, s.L, s.mesh, s.dt)
    t_step = time.perf_counter() - t
    t = time.perf_counter()
    Q = kp.orthonormalize(out["U"])
    kp.greens(Q, s.A)
    t_qr = time.perf_counter() - t
    t = time.perf_counter()
    kp.local_energy(pre["Lh"], pre["h1h"], out["Gh"], s.mesh, walkers=list(range(ne)))
    t_e = time.perf_counter() - t
    nsteps = xs_host.shape[0]
    per_ws = t_step / nw + (t_qr / nw + t_e / ne) / nsteps
    return 1.0 / per_ws, (f"1 propagation step of {nw} walkers ({t_step:.2f} s), QR+G of "
                          f"{nw} walkers ({t_qr:.2f} s), local energy of {ne} walkers "
                          f"({t_e:.2f} s)")


def cpu_baseline(s, U0, xs_host):
    """The FP64 oracle on the host cores, on a bounded sample of the same block, with the
    BLAS threads of this process and with one thread."""
    from oracle import kpoint as kp
    try:
        from threadpoolctl import threadpool_info, threadpool_limits
        threads = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    except Exception:  # pragma: no cover
        threadpool_limits, threads = None, None
    cores = len(os.sched_getaffinity(0))
    pre = kp.prepare(s.L, s.H1, s.A, s.dt)
    rate, desc = _oracle_rate(kp, s, pre, U0, xs_host, 8, 2)
    out = {"value": round(rate, 3), "unit": "walker-steps/s",
           "cores": threads if threads else cores, "host_cores": cores, "kind": "oracle",
           "sample": (desc + "; walker-steps/s = 1/(t_step/nw + (t_QR/nw + t_E/ne)/"
                      f"{xs_host.shape[0]}) for the {xs_host.shape[0]}-step block")}
    if threadpool_limits is not None:
        with threadpool_limits(limits=1):
            r1, d1 = _oracle_rate(kp, s, pre, U0, xs_host, 2, 1)
        out["single_thread"] = {"value": round(r1, 3), "cores": 1, "sample": d1}
    return out


def gen_system(name, torch):
    from synth.kpt_inputs import config_shapes, make_system, make_walkers, make_fields
    cfg = config_shapes(name)
    s, rng = make_system(cfg["mesh"], cfg["m"], cfg["nocc"], cfg["nchol"], seed=cfg["seed"])
    U0 = make_walkers(s, cfg["nwalk"], rng)
    xs = make_fields(s, cfg["nwalk"], max(cfg["nsteps"], 1), rng)
    return cfg, s, U0, xs


def bench_batch(args, torch):
    """Uneven batch: systems A (2x2x2, m=26, 128 walkers), B (3x3x3, m=26, 64 walkers) and
    C (3x3x3, m=52, nchol=416, 32 walkers), FP64, one block = 10 steps + QR + energy.
    Modes: each system on its own (three calls per block), one batched call, the batched
    block captured in a HIP graph, and the graph recaptured after autotuning."""
    import numpy as np
    import paper_2003_09468_amd as lib
    names = ["c3A", "c3B", "c3C"]
    sysd = []
    for nm in names:
        t = time.perf_counter()
        cfg, s, U0, xs = gen_system(nm, torch)
        log(f"generated {nm} {cfg} in {time.perf_counter() - t:.1f} s")
        p = make_problem(s, U0, lib.PREC_FP64, torch, tune=False)
        sysd.append((cfg, s, torch.from_numpy(U0).cuda(), torch.from_numpy(xs), p))
        del s
    ps = [d[4] for d in sysd]
    walkers = sum(d[0]["nwalk"] for d in sysd)
    nsteps = sysd[0][0]["nsteps"]
    singles = [lib.KptBatch([p]) for p in ps]
    fsingle = [b.fields([d[3]]) for b, d in zip(singles, sysd)]
    allb = lib.KptBatch(ps)
    fall = allb.fields([d[3] for d in sysd])

    def reset_all():
        for d in sysd:
            reset(d[4], d[2])

    def run_separate():
        for b, f in zip(singles, fsingle):
            b.step(f, ortho=True, energy=True)

    def energies(batches):
        if batches is allb:
            return [allb.energy(i).cpu().numpy().copy() for i in range(len(ps))]
        return [b.energy(0).cpu().numpy().copy() for b in batches]

    graph = {"g": None}

    def run_batched():
        allb.step(fall, ortho=True, energy=True)

    def run_graph():
        graph["g"].launch()

    res, Es = {}, {}
    modes = [("separate", run_separate, singles), ("batched", run_batched, allb),
             ("graph", run_graph, allb), ("graph_autotuned", run_graph, allb)]
    for mode, fn, owner in modes:
        if mode == "graph":
            graph["g"] = allb.graph(fall, ortho=True, energy=True)
        if mode == "graph_autotuned":
            graph["g"].close()
            reset_all()
            allb.autotune()
            graph["g"] = allb.graph(fall, ortho=True, energy=True)
        reset_all()
        fn()
        torch.cuda.synchronize()
        Es[mode] = energies(owner)
        for _ in range(args.warmup):
            fn()
        torch.cuda.synchronize()
        lib.timing_enable(True, 1 << 16)
        t0 = time.perf_counter()
        for _ in range(args.steps):
            fn()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        lib.timing_enable(False)
        kern = {}
        for kc in lib.KERNEL_CLASSES:
            ms, n = lib.timing_read(kc)
            if n:
                kern[kc] = {"ms_per_block": round(ms / args.steps, 4),
                            "launches": n // args.steps}
        dt = (t1 - t0) / args.steps
        res[mode] = {"ms_per_block": round(dt * 1e3, 3),
                     "walker_steps_per_s": round(walkers * nsteps / dt, 2), "kernels": kern}
        log(f"[{mode}] block {dt * 1e3:.2f} ms -> {walkers * nsteps / dt:.1f} walker-steps/s")
    graph["g"].close()
    ref = Es["separate"]
    agree = max(float(np.abs(Es[m][i] - ref[i]).max()) for m in Es for i in range(len(ref)))
    best = max(res, key=lambda m: res[m]["walker_steps_per_s"])
    return {
        "metric": "walker-steps/s, uneven batch of three systems, 10-step block",
        "value": res[best]["walker_steps_per_s"],
        "unit": "walker-steps/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": res[best]["ms_per_block"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "c3: A mesh 2x2x2 m=26 nchol=208 W=128; B mesh 3x3x3 m=26 "
                               "nchol=208 W=64; C mesh 3x3x3 m=52 nchol=416 W=32; nocc=4; one "
                               "step = one block of 10 propagation steps + QR + local energy",
                   "path": best},
        "modes": res,
        "speedup_vs_separate": {m: round(res[m]["walker_steps_per_s"] /
                                         res["separate"]["walker_steps_per_s"], 3) for m in res},
        "max_abs_energy_difference_between_modes": agree,
        "kernel_source_hash": kernel_source_hash(),
    }


def bench_adjoint(args, torch):
    """Local energy and its adjoint dE/dGh at 3x3x3, m=26, 16 walkers, FP64 and FP32."""
    import numpy as np
    import paper_2003_09468_amd as lib
    cfg, s, U0, _ = gen_system("c4", torch)
    U0d = torch.from_numpy(U0).cuda()
    res, D = {}, {}
    for name, prec in (("fp64", lib.PREC_FP64), ("fp32", lib.PREC_FP32)):
        p = make_problem(s, U0, prec, torch)
        reset(p, U0d)
        gE = torch.ones(p.nwalk, dtype=torch.complex128, device="cuda")
        E = torch.empty((p.nwalk, 3), dtype=torch.complex128, device="cuda")
        G = torch.empty_like(p.Gh)
        p.energy(out=E)
        p.energy_backward(gE=gE, out=G)
        torch.cuda.synchronize()
        D[name] = (E.cpu().numpy().copy(), G.cpu().numpy().copy())
        for _ in range(args.warmup):
            p.energy(out=E)
            p.energy_backward(gE=gE, out=G)
        torch.cuda.synchronize()
        reps = max(args.steps, 1) * 5
        lib.timing_enable(True, 1 << 16)
        t0 = time.perf_counter()
        for _ in range(reps):
            p.energy(out=E)
            p.energy_backward(gE=gE, out=G)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        lib.timing_enable(False)
        kern = {}
        for kc in lib.KERNEL_CLASSES:
            ms, n = lib.timing_read(kc)
            if n:
                kern[kc] = {"ms_per_launch": round(ms / n, 5), "launches": n // reps}
        dt = (t1 - t0) / reps
        W = cfg["nwalk"]
        flb = 16.0 * W * cfg["nk"] ** 3 * cfg["nocc"] ** 2 * cfg["nchol"] * cfg["m"]
        ach = flb / (kern["exchange_bwd"]["ms_per_launch"] * 1e-3) / 1e12
        res[name] = {"ms_per_eval": round(dt * 1e3, 4),
                     "walker_evals_per_s": round(W / dt, 2), "kernels": kern,
                     "roofline": {"kernel": "exchange_bwd", "bound": "mfma",
                                  "achieved": round(ach, 3), "peak": PEAK[name],
                                  "unit": "TFLOP/s", "frac": round(ach / PEAK[name], 4),
                                  "traffic": None, "flops_per_launch": flb}}
        log(f"[{name}] energy+adjoint {dt * 1e3:.3f} ms -> {W / dt:.1f} walker evals/s; "
            f"adjoint kernel {kern['exchange_bwd']['ms_per_launch']:.3f} ms ({ach:.1f} TF)")
        del p
        torch.cuda.empty_cache()
    e64, g64 = D["fp64"]
    e32, g32 = D["fp32"]
    acc = {"max_abs_dE_per_cell": float(np.abs(e32.sum(1) - e64.sum(1)).max() / cfg["nk"]),
           "max_rel_dgrad": float(np.abs(g32 - g64).max() / np.abs(g64).max()),
           "compared": "FP32-contraction vs FP64 GPU path on the same walkers"}
    return {
        "metric": "walker energy+adjoint evaluations/s at Nk=27 M=26",
        "value": res["fp64"]["walker_evals_per_s"], "unit": "walker evals/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": res["fp64"]["ms_per_eval"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "c4: mesh 3x3x3, m=26, nocc=4, nchol=208, 16 walkers; one "
                               "step = local energy + its adjoint for all walkers",
                   "path": "fp64"},
        "roofline": res["fp64"]["roofline"], "paths": res, "accuracy": acc,
        "kernel_source_hash": kernel_source_hash(),
    }


def bench_dense(args, torch):
    """The k-point against the standard (dense) representation of the same system (the
    comparison of the paper's timing figure, at supercell sizes the dense kernels take:
    nk m <= 64): meshes 1x1x2, 2x2x1 and 2x2x2 with m = 8, nocc = 2, nchol = 24 per Q and 64
    walkers.  Both run FP64 blocks of 20 steps + QR + local energy on the same walkers, the
    dense system with the mapped fields, so both end on the same state."""
    import numpy as np
    from synth.kpt_inputs import make_system, make_walkers, make_fields
    import paper_2003_09468_amd as lib
    W, nsteps = 64, 20
    res = {}
    for mesh in ((1, 1, 2), (2, 2, 1), (2, 2, 2)):
        s, rng = make_system(mesh, 8, 2, 24, seed=0)
        U0 = make_walkers(s, W, rng)
        xs = torch.from_numpy(make_fields(s, W, nsteps, rng)).cuda()
        p = make_problem(s, U0, lib.PREC_FP64, torch)
        d = p.dense(torch.from_numpy(s.H1))
        xds = torch.stack([p.dense_fields(xs[t]) for t in range(nsteps)])
        U0d = torch.from_numpy(U0).cuda()
        times, E = {}, {}
        for name, q, fields in (("kpoint", p, xs), ("dense", d, xds)):
            Eo = torch.empty((W, 3), dtype=torch.complex128, device="cuda")
            reset(q, U0d)
            run_block(q, fields, {}, Eo)
            E[name] = Eo.sum(1).cpu().numpy() / s.nk
            for _ in range(args.warmup):
                reset(q, U0d)
                run_block(q, fields, {}, Eo)
            torch.cuda.synchronize()
            t = 0.0
            for _ in range(max(args.steps, 1)):
                reset(q, U0d)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                run_block(q, fields, {}, Eo)
                torch.cuda.synchronize()
                t += time.perf_counter() - t0
            times[name] = t / max(args.steps, 1) * 1e3
        key = "x".join(map(str, mesh))
        res[key] = {"nk": s.nk, "supercell_orbitals": s.nk * s.m,
                    "dense_cholesky_vectors": s.nk * s.nchol,
                    "kpoint_ms_per_block": round(times["kpoint"], 3),
                    "dense_ms_per_block": round(times["dense"], 3),
                    "dense_over_kpoint": round(times["dense"] / times["kpoint"], 3),
                    "max_abs_dE_per_cell": float(np.abs(E["dense"] - E["kpoint"]).max())}
        log(f"[{key}] k-point {times['kpoint']:.2f} ms, dense {times['dense']:.2f} ms per block; "
            f"energies after the block differ by {res[key]['max_abs_dE_per_cell']:.2e} Ha/cell")
        del p, d
        torch.cuda.empty_cache()
    last = res["2x2x2"]
    return {
        "metric": "block time, k-point vs standard (dense) representation, mesh 2x2x2, m=8",
        "value": last["dense_over_kpoint"], "unit": "dense/k-point time ratio", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": last["kpoint_ms_per_block"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "meshes 1x1x2, 2x2x1, 2x2x2; m=8, nocc=2, nchol=24 per Q, 64 "
                               "walkers; one step = one FP64 block of 20 steps + QR + energy "
                               "in each representation", "path": "fp64"},
        "paths": res, "kernel_source_hash": kernel_source_hash(),
    }


def time_batch_block(b, fields, args, torch, reset_fn):
    """Mean time of one block (afqmc_kpt_step over the packed fields with the last step's
    re-orthonormalisation and the local energy) after the warmup blocks."""
    for _ in range(args.warmup):
        reset_fn()
        b.step(fields, ortho=True, energy=True)
    torch.cuda.synchronize()
    t = 0.0
    for _ in range(max(args.steps, 1)):
        reset_fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        b.step(fields, ortho=True, energy=True)
        torch.cuda.synchronize()
        t += time.perf_counter() - t0
    return t / max(args.steps, 1) * 1e3


def bench_spin(args, torch):
    """Two-determinant (collinear) walkers at the c1 size: mesh 3x3x3, m=26, nchol=208, 64
    walkers, 4 up and 3 down electrons per k-point, against the closed-shell system with 4
    of each; one block = 20 steps + QR + local energy through afqmc_kpt_step, in FP64 and in
    the placed BF16X3-step / INT8X4-energy precision.  The energies of the initial walkers
    in the placed precision are compared with FP64."""
    import numpy as np
    from synth.kpt_inputs import (make_system, make_walkers, make_fields, make_spin_trial,
                                  spin_view)
    import paper_2003_09468_amd as lib
    W, nsteps, nu, nd = 64, 20, 4, 3
    s, rng = make_system((3, 3, 3), 26, nu, 208, seed=0)
    A_dn = make_spin_trial(s, nd, rng)
    U_up = torch.from_numpy(make_walkers(s, W, rng)).cuda()
    U_dn = torch.from_numpy(make_walkers(spin_view(s, A_dn), W, rng)).cuda()
    x = torch.from_numpy(make_fields(s, W, nsteps, rng)).cuda()
    L, A, Ad, H1 = (torch.from_numpy(v).cuda() for v in (s.L, s.A, A_dn, s.H1))
    res, E0 = {}, {}
    placed = lib.prec_place(lib.PREC_BF16X3, lib.PREC_INT8X4)
    for pname, prec in (("fp64", lib.PREC_FP64), ("bf16x3+int8x4E", placed)):
        pr = lib.KptSpinPair(s.mesh, s.m, nu, nd, s.nchol, W, s.dt, L, A, Ad, prec=prec)
        pr.prepare(H1)
        cs = lib.KptProblem(s.mesh, s.m, nu, s.nchol, W, s.dt, L, A, prec=prec)
        cs.prepare(H1)
        cb = lib.KptBatch([cs])

        def reset_pair():
            pr.set_walkers(U_up, U_dn)
            pr.greens()

        def reset_closed():
            cs.set_walkers(U_up)
            cs.greens()

        reset_pair()
        pr.autotune()
        reset_closed()
        cb.autotune()
        reset_pair()
        pr.local_energy()
        E0[pname] = pr.energy(0).sum(1).cpu().numpy() / s.nk
        fp = pr.step_fields(x)
        fc = cb.fields([x])
        tp = time_batch_block(pr, fp, args, torch, reset_pair)
        tc = time_batch_block(cb, fc, args, torch, reset_closed)
        res[pname] = {"pair_ms_per_block": round(tp, 3), "closed_ms_per_block": round(tc, 3),
                      "pair_walker_steps_per_s": round(W * nsteps / tp * 1e3, 1),
                      "closed_walker_steps_per_s": round(W * nsteps / tc * 1e3, 1),
                      "pair_over_closed": round(tp / tc, 3)}
        log(f"[{pname}] two-determinant block {tp:.2f} ms, closed shell {tc:.2f} ms "
            f"({tp / tc:.2f}x)")
        del pr, cs, cb
        torch.cuda.empty_cache()
    dE = float(np.abs(E0["bf16x3+int8x4E"] - E0["fp64"]).max())
    res["bf16x3+int8x4E"]["initial_energy_err_per_cell"] = dE
    log(f"initial-walker energy, placed vs FP64: {dE:.2e} Ha/cell")
    r = res["bf16x3+int8x4E"]
    return {
        "metric": "walker-steps/s, two-determinant walkers, Nk=27 M=26",
        "value": r["pair_walker_steps_per_s"], "unit": "walker-steps/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": r["pair_ms_per_block"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "bf16x3+int8x4+f64", "data": "synthetic",
        "config": {"workload": "mesh 3x3x3, m=26, nchol=208, 64 walkers, 4 up + 3 down "
                               "electrons per k-point; one step = one block of 20 steps + QR + "
                               "local energy", "path": "bf16x3+int8x4E"},
        "paths": res, "kernel_source_hash": kernel_source_hash(),
    }


def bench_bands(args, torch):
    """Non-uniform bands: a 3x3x3 system whose k-points hold 20 to 26 bands (drawn
    uniformly, seeded), 4 occupied, 208 Cholesky vectors per Q, 64 walkers, padded to 26
    bands on the device; FP64 blocks of 20 steps + QR + local energy, against the uniform
    26-band system of the same sizes.  Reports the padding entry's time and the padded
    block's throughput."""
    import numpy as np
    from synth.kpt_inputs import make_ragged_system, make_ragged_walkers, pack_ragged
    from synth.kpt_inputs import make_system, make_walkers
    import paper_2003_09468_amd as lib
    W, nsteps, m, nocc, C = 64, 20, 26, 4, 208
    rng0 = np.random.Generator(np.random.PCG64(5))
    mk = tuple(int(v) for v in rng0.integers(20, 27, size=27))
    rs, rng = make_ragged_system((3, 3, 3), mk, nocc, C, seed=5)
    Ur = make_ragged_walkers(rs, W, rng)
    x = torch.from_numpy(rng.standard_normal((nsteps, W, 27, C, 2))).cuda()
    Lr, Hr, Ar, Urp = (torch.from_numpy(np.ascontiguousarray(v)).cuda()
                       for v in pack_ragged(rs, Ur))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    L, H1, A, U = lib.pad_bands(rs.mesh, mk, m, nocc, C, Lr, Hr, Ar, Urp)
    torch.cuda.synchronize()
    tpad = (time.perf_counter() - t0) * 1e3
    del Lr
    res = {}
    us, rng2 = make_system((3, 3, 3), m, nocc, C, seed=5)
    Uu = torch.from_numpy(make_walkers(us, W, rng2)).cuda()
    for name, (LL, AA, HH, UU) in (("padded", (L, A, H1, U)),
                                   ("uniform", (torch.from_numpy(us.L).cuda(),
                                                torch.from_numpy(us.A).cuda(),
                                                torch.from_numpy(us.H1).cuda(), Uu))):
        p = lib.KptProblem((3, 3, 3), m, nocc, C, W, rs.dt, LL, AA)
        p.prepare(HH)
        b = lib.KptBatch([p])

        def reset_fn():
            p.set_walkers(UU)
            p.greens()

        reset_fn()
        b.autotune()
        t = time_batch_block(b, b.fields([x]), args, torch, reset_fn)
        res[name] = {"ms_per_block": round(t, 3),
                     "walker_steps_per_s": round(W * nsteps / t * 1e3, 1)}
        log(f"[{name}] block {t:.2f} ms")
        del p, b
        torch.cuda.empty_cache()
    res["padded"]["pad_entry_ms"] = round(tpad, 3)
    res["padded"]["mean_bands"] = float(np.mean(mk))
    log(f"padding entry {tpad:.2f} ms; mean bands {np.mean(mk):.2f} of {m}")
    r = res["padded"]
    return {
        "metric": "walker-steps/s, non-uniform bands (20-26 per k-point, padded to 26)",
        "value": r["walker_steps_per_s"], "unit": "walker-steps/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": r["ms_per_block"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"mesh 3x3x3, bands per k-point {list(mk)} padded to 26, "
                               "nocc=4, nchol=208, 64 walkers; one step = one FP64 block of 20 "
                               "steps + QR + local energy", "path": "fp64"},
        "paths": res, "kernel_source_hash": kernel_source_hash(),
    }


def bench_c2(args, torch):
    """4x4x4 mesh, m=52, nocc=4, nchol=400, 32 walkers (L: 70.9 GB complex128, streamed to
    the GPU block by block as it is drawn).  The local energy of the initial walkers with
    every contraction precision on the same Gh, each with its error against FP64, and 10
    FP64 propagation steps, the walkers re-orthonormalised after the last."""
    import numpy as np
    import paper_2003_09468_amd as lib
    from synth.kpt_inputs import config_shapes, make_system, make_walkers, make_fields
    cfg = config_shapes("c2")
    nk, m, C, W = cfg["nk"], cfg["m"], cfg["nchol"], cfg["nwalk"]
    Ld = torch.empty((nk, nk, m, m, C), dtype=torch.complex128, device="cuda")
    count = [0]
    t = time.perf_counter()

    def sink(Q, k, blk):
        Ld[Q, k].copy_(torch.from_numpy(blk))
        count[0] += 1
        if count[0] % (nk * nk // 8) == 0:
            log(f"  L blocks {count[0]}/{nk * nk} ({time.perf_counter() - t:.0f} s)")

    s, rng = make_system(cfg["mesh"], m, cfg["nocc"], C, seed=cfg["seed"], sink=sink)
    U0 = make_walkers(s, W, rng)
    xs = torch.from_numpy(make_fields(s, W, cfg["nsteps"], rng)).cuda()
    log(f"generated c2 in {time.perf_counter() - t:.1f} s")
    U0d = torch.from_numpy(U0).cuda()

    def problem(prec):
        p = lib.KptProblem(s.mesh, m, cfg["nocc"], C, W, s.dt, Ld, torch.from_numpy(s.A),
                           prec=prec)
        p.prepare(torch.from_numpy(s.H1))
        return p

    res = {}
    p64 = problem(lib.PREC_FP64)
    reset(p64, U0d)
    # the precisions are compared on the initial walkers (after 10 steps of this workload
    # the phaseless cut has removed every walker and the overlaps are ill-conditioned)
    G = p64.Gh.clone()
    bufs = {"xbar": torch.empty((W, nk, C, 2), dtype=torch.complex128, device="cuda"),
            "X": torch.empty((W, nk, C), dtype=torch.complex128, device="cuda"),
            "vhs": torch.empty((W, nk * m, nk * m), dtype=torch.complex128, device="cuda")}
    torch.cuda.synchronize()
    lib.timing_enable(True, 1 << 16)
    t0 = time.perf_counter()
    for st in range(cfg["nsteps"]):
        p64.step(xs[st], ortho=(st == cfg["nsteps"] - 1), bufs=bufs)
    torch.cuda.synchronize()
    dt_steps = time.perf_counter() - t0
    lib.timing_enable(False)
    kern = {}
    for kc in lib.KERNEL_CLASSES:
        ms, n = lib.timing_read(kc)
        if n:
            kern[kc] = {"ms_total": round(ms, 3), "launches": n}
    res["steps_fp64"] = {"walker_steps_per_s": round(W * cfg["nsteps"] / dt_steps, 2),
                         "ms_per_step": round(dt_steps * 1e3 / cfg["nsteps"], 3),
                         "kernels": kern}
    log(f"[fp64] {cfg['nsteps']} steps {dt_steps:.2f} s -> {W * cfg['nsteps'] / dt_steps:.1f} "
        f"walker-steps/s")
    del bufs
    alive = int((p64.status == 0).sum().item())
    E = {}
    paths = [("fp64", lib.PREC_FP64), ("fp32", lib.PREC_FP32), ("bf16x3", lib.PREC_BF16X3)]
    for name, prec in paths:
        p = p64 if prec == lib.PREC_FP64 else problem(prec)
        out = torch.empty((W, 3), dtype=torch.complex128, device="cuda")
        p.energy(out=out, Gh=G)
        torch.cuda.synchronize()
        E[name] = out.cpu().numpy().copy()
        reps = 3
        lib.timing_enable(True, 1 << 16)
        t0 = time.perf_counter()
        for _ in range(reps):
            p.energy(out=out, Gh=G)
        torch.cuda.synchronize()
        dte = (time.perf_counter() - t0) / reps
        lib.timing_enable(False)
        ms_x, n_x = lib.timing_read("exchange")
        fl = kernel_flops("exchange", cfg)
        ach = fl / (ms_x / n_x * 1e-3) / 1e12
        key = name
        res[name] = {"ms_per_energy": round(dte * 1e3, 3),
                     "walker_energy_evals_per_s": round(W / dte, 3),
                     "exchange_ms": round(ms_x / n_x, 3),
                     "roofline": {"kernel": "exchange", "bound": "mfma",
                                  "achieved": round(ach, 3), "peak": PEAK[key],
                                  "unit": "TFLOP/s", "frac": round(ach / PEAK[key], 4),
                                  "traffic": None, "flops_per_launch": fl}}
        log(f"[{name}] energy {dte * 1e3:.1f} ms (exchange {ms_x / n_x:.1f} ms, {ach:.1f} TF)")
        if p is not p64:
            del p
            torch.cuda.empty_cache()
    e64 = E["fp64"]
    for name in E:
        d = np.abs(E[name].sum(1) - e64.sum(1)) / nk
        res[name]["max_abs_dE_per_cell_vs_fp64"] = float(d.max())
        res[name]["median_abs_dE_per_cell_vs_fp64"] = float(np.median(d))
    return {
        "metric": "walker energy evaluations/s at Nk=64 M=52 (exchange-dominated)",
        "value": res["fp64"]["walker_energy_evals_per_s"], "unit": "walker evals/s",
        "n_gpus": 1, "steps": 3, "warmup": 1, "ms_per_step": res["fp64"]["ms_per_energy"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "c2: mesh 4x4x4, m=52, nocc=4, nchol=400, 32 walkers; local "
                               "energies of the initial walkers in FP64, FP32 and BF16x3, then 10 "
                               "FP64 propagation steps; one step = one local energy of all "
                               "walkers", "path": "fp64",
                   "walkers_alive_after_steps": alive},
        "roofline": res["fp64"]["roofline"], "paths": res,
        "kernel_source_hash": kernel_source_hash(),
    }


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3, help="timed blocks")
    ap.add_argument("--warmup", type=int, default=1, help="untimed blocks")
    ap.add_argument("--config", default="c1",
                    help="c1 (headline), c0, c2 (4x4x4 energy precisions), c3 (uneven batch modes), "
                         "c4 (energy adjoint), dense (k-point vs standard representation), "
                         "spin (two-determinant walkers) or bands (non-uniform bands)")
    ap.add_argument("--prec", default="all",
                    help="all, or a comma-separated list of paths: " + ", ".join(PATHS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--calib-copy", action="store_true",
                    help="also run one plain 1 GiB device copy (scale reference for HBM counters)")
    ap.add_argument("--reduce-pmc", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="write profiles/traffic_c1.{json,md} from two counter runs and exit")
    ap.add_argument("--reduce-mfma", nargs=2, metavar=("CSV", "OUT_MD"),
                    help="write an MFMA-utilisation summary from one counter run and exit")
    ap.add_argument("--title", default="", help="title of the --reduce-mfma summary")
    ap.add_argument("--command", default="", help="profiling command of the summary")
    args = ap.parse_args()
    if args.reduce_pmc:
        reduce_pmc(*args.reduce_pmc)
        return
    if args.reduce_mfma:
        reduce_mfma(args.reduce_mfma[0], args.reduce_mfma[1], args.title, args.command)
        return
    if args.gpus != 1:
        print(f"bench.py: the benchmark runs on one GPU; --gpus {args.gpus} is not supported "
              "(sharding walkers or Q blocks across GPUs is not built).",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from synth.kpt_inputs import config_shapes, make_system, make_walkers, make_fields
    import paper_2003_09468_amd as lib

    if not torch.cuda.is_available():
        print("bench.py: no GPU visible", file=sys.stderr)
        sys.exit(1)
    if args.config == "c3":
        print(json.dumps(bench_batch(args, torch)), flush=True)
        return
    if args.config == "c2":
        print(json.dumps(bench_c2(args, torch)), flush=True)
        return
    if args.config == "c4":
        print(json.dumps(bench_adjoint(args, torch)), flush=True)
        return
    if args.config == "dense":
        print(json.dumps(bench_dense(args, torch)), flush=True)
        return
    if args.config == "spin":
        print(json.dumps(bench_spin(args, torch)), flush=True)
        return
    if args.config == "bands":
        print(json.dumps(bench_bands(args, torch)), flush=True)
        return
    cfg = config_shapes(args.config)
    log(f"generating {args.config}: {cfg}")
    t = time.perf_counter()
    s, rng = make_system(cfg["mesh"], cfg["m"], cfg["nocc"], cfg["nchol"], seed=cfg["seed"])
    U0 = make_walkers(s, cfg["nwalk"], rng)
    xs_host = make_fields(s, cfg["nwalk"], cfg["nsteps"], rng)
    log(f"  inputs in {time.perf_counter() - t:.1f} s")
    U0d = torch.from_numpy(U0).cuda()
    xs = torch.from_numpy(xs_host).cuda()

    res, first, acc = {}, {}, None
    paths = list(PATHS) if args.prec == "all" else args.prec.split(",")
    for name in paths:
        if name not in PATHS:
            sys.exit(f"bench.py: unknown path {name!r} (known: {', '.join(PATHS)})")
    if "fp64" in paths:  # the reference path first: every other path is compared with it
        paths.remove("fp64")
        paths.insert(0, "fp64")
    code = {"fp64": lib.PREC_FP64, "fp32": lib.PREC_FP32, "bf16x3": lib.PREC_BF16X3,
            "int8x5": lib.PREC_INT8X5, "int8x4": lib.PREC_INT8X4}
    p64, initial, state64 = None, {}, {}
    for name in paths:
        sp, ep = PATHS[name]
        prec = code[sp] if sp == ep else lib.prec_place(code[sp], code[ep])
        p = make_problem(s, U0, prec, torch)
        res[name], first[name] = bench_path(name, p, U0d, xs, args, torch, cfg)
        # every path's energies on the initial walkers (the same Gh: FP64 greens)
        reset(p, U0d)
        initial[name] = p.energy().sum(1).cpu().numpy() / cfg["nk"]
        if name == "fp64":
            p64 = p
            state64 = first[name]
            # one FP64 step from the FP64 path's state after the block
            state64["step"] = step_from(p64, state64, xs[0])
            continue
        if p64 is not None:
            # the path's stages at the FP64 path's state after the block: its local energy
            # there, and one of its steps from there (evaluated with the FP64 energy)
            state64.setdefault("others", {})[name] = {
                "E": p.energy(Gh=state64["Gh"]).cpu().numpy(),
                "step": step_from(p, state64, xs[0]),
            }
        del p
        torch.cuda.empty_cache()

    if p64 is not None and len(res) > 1:
        acc = accuracy_report(p64, first, state64, initial, s, cfg)
        del p64
        torch.cuda.empty_cache()

    # the fastest path whose local energy meets the tolerance at the common state; FP64
    # otherwise
    use = "fp64" if "fp64" in res else paths[0]
    if acc is not None:
        for name in sorted(res, key=lambda k: -res[k]["walker_steps_per_s"]):
            if name == "fp64" or acc[name]["meets_tolerance"]:
                use = name
                break
    main_res = res[use]
    out = {
        "metric": METRIC,
        "value": round(main_res["walker_steps_per_s"], 2),
        "unit": "walker-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(main_res["ms_per_block"], 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": DTYPE[use],
        "data": "synthetic",
        "config": {"workload": f"{args.config}: mesh {'x'.join(map(str, cfg['mesh']))}, "
                               f"m={cfg['m']}, nocc={cfg['nocc']}, nchol={cfg['nchol']}, "
                               f"{cfg['nwalk']} walkers, dt={cfg['dt']}; one step = one block "
                               f"of {cfg['nsteps']} propagation steps + QR + local energy",
                   "nk": cfg["nk"], "m": cfg["m"], "nocc": cfg["nocc"], "nchol": cfg["nchol"],
                   "walkers": cfg["nwalk"], "steps_per_block": cfg["nsteps"],
                   "path": use},
        "roofline": roofline(main_res, use, cfg),
        "paths": {k: {"walker_steps_per_s": round(v["walker_steps_per_s"], 2),
                      "ms_per_block": round(v["ms_per_block"], 3),
                      "ms_per_block_with_kernel_events":
                          round(v["ms_per_block_with_kernel_events"], 3),
                      "energy_evals_per_s": energy_evals(v, cfg),
                      "population_control_ms": v.get("population_control_ms"),
                      "kernels": {kk: {"ms_per_block": round(vv["ms_total"], 4),
                                       "launches": vv["launches"],
                                       "ms_per_launch": round(vv["ms_per_launch"], 5)}
                                  for kk, vv in v["kernels"].items()},
                      "roofline_dominant": roofline(v, k, cfg),
                      "roofline_exchange": exchange_roofline(v, k, cfg)}
                  for k, v in res.items()},
        "accuracy": acc,
    }
    if "fp64" in res:
        out["speedup_vs_fp64"] = {k: round(v["walker_steps_per_s"] /
                                           res["fp64"]["walker_steps_per_s"], 3)
                                  for k, v in res.items() if k != "fp64"}
    if args.calib_copy:
        src = torch.empty(1 << 30, dtype=torch.uint8, device="cuda").fill_(1)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        out["calib_copy_bytes"] = 1 << 30
        del src, dst
    out["kernel_source_hash"] = kernel_source_hash()
    if not args.no_cpu_baseline:
        log("timing the CPU oracle on a bounded sample ...")
        out["cpu_baseline"] = cpu_baseline(s, U0, xs_host)
        log(f"  cpu baseline {out['cpu_baseline']}")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
