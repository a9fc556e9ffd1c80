#!/usr/bin/env python3
"""Throughput of the patch-dynamics hot path (Sec. 3.3 steps (i)-(vi)) on one GPU.

Default (--workload headline): the metric's pairing in one JSON line.  The plain batched
scheme in FP64 on the mixed batch of 512 seeded instances (tanh-stretched squares and
annuli, 17..129 macro nodes per side, 9..33 micro points per patch side), one persistent
launch per batch macro step replayed from a HIP graph, is the line's value (patch-point
updates/s, with macro steps/s and the k_batch roofline); the same batch with the learned
closure standing in for the bursts (1% spot checks, per-member fallback) reports its
macro steps/s, the speed-up over plain and its relative L2 error against the plain run,
also over a long horizon on held-out members.  The CPU baseline is the FP64 oracle on a
seeded sample of the batch, on all host cores and on one thread.

Other workloads (--workload): config1, config2 and config3 (the fused single-grid step
on the small square, the stretched square in FP64 or FP32, the annulus), config4 (the
batch alone), config5 (the closure line), full-domain (the explicit comparator on one fine
lattice), refresh (edge data refreshed between sub-bursts), adi (the ADI micro solver on
the Sec. 4.1.1 setup) and upwind (the 3- or 4-point upwind micro differences on the
config 2 problem).
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK = {"f64": 78.6e12, "f32": 157.3e12}  # MI355X vector ALU FLOP/s (dense, published)
KERNEL_NAME = {1: "k_burst", 2: "k_burst_x", 3: "k_burst_h"}  # by exchange: LDS, in-wave, hybrid


def workload(name):
    from paper_2405_08764_amd import workloads as W
    if name == "config1":
        return W.config1(), ("unit square, 11x11 macro nodes, 9x9 micro points per patch, "
                             "diag D, manufactured e^-t sin(pi x) sin(pi y), 10 macro steps")
    if name == "config3":
        return W.config3(), ("annulus r in [1,2], 64 radial x 256 angular macro nodes, 21x21 "
                             "micro points per patch, k = 1 + 0.5 cos(3 theta)(r - 1)")
    return W.config2(), ("tanh-stretched unit square (beta 2.5), 65x65 macro nodes, 17x17 "
                         "micro points per patch, eps 1e-3, 8 random Fourier modes for D and v, "
                         "source (1 + sin 4 pi t) g")


BURST_SOURCES = ["pd_burst.inc", "pd_internal.h"] + [
    f"pd_burst_{fam}_{prec}.hip" for fam in ("x", "lds", "h") for prec in ("f64", "f32")]


FD_SOURCES = ["pd_fd.hip", "pd_internal.h"]
HU_SOURCES = ["pd_upwind.hip", "pd_internal.h"]
ADI_SOURCES = ["pd_adi.hip", "pd_internal.h"]
ADU_SOURCES = ["pd_adi_upwind.hip", "pd_internal.h"]
SOLVE_SOURCES = ["pd_solve_x_f64.hip", "pd_burst.inc", "pd_internal.h"]
RESIDENT_STEPS = 16  # macro steps per graph replay, so per resident launch


def burst_source_hash(files=None):
    """SHA-256 over a kernel's sources (default: the burst kernels'): a traffic figure
    taken from counters is valid only for the code it was measured on."""
    import hashlib
    h = hashlib.sha256()
    for f in (BURST_SOURCES if files is None else files):
        with open(os.path.join(ROOT, "paper_2405_08764_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def traffic_file(kernel, workload, precision):
    return os.path.join(ROOT, "profiles", f"{kernel}_{workload}_{precision}_hbm_traffic.txt")


def read_traffic(kernel, workload, precision, shape, files=None):
    """HBM bytes per launch from the committed counter summary, or None when there is
    none for this kernel, workload and launch shape, or the kernel changed since."""
    path = traffic_file(kernel, workload, precision)
    if not os.path.exists(path):
        return None
    kv = {}
    with open(path) as fh:
        for line in fh:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
    if kv.get("source_sha256") != burst_source_hash(files) or kv.get("shape") != shape:
        return None
    return float(kv["hbm_bytes_per_launch"])


def pmc_summary(fetch_csv, write_csv, kernel_prefix, calib_mib, out, command, workload,
                precision, shape, files=None):
    """Per-launch HBM traffic of a kernel from two rocprofv3 --pmc runs (FETCH_SIZE, then
    WRITE_SIZE, both in KiB per dispatch), each scaled by what the same counter reads for
    the calibration kernel of known traffic (calib_mib MiB read and written)."""
    import csv

    def per_kernel(path, counter):
        vals, cal = [], []
        for r in csv.DictReader(open(path)):
            if r["Counter_Name"] != counter:
                continue
            name = r["Kernel_Name"]
            v = float(r["Counter_Value"]) * 1024.0
            if kernel_prefix in name:
                vals.append(v)
            elif "MulFunctor" in name or ("elementwise_kernel" in name and "Mul" in name):
                cal.append(v)
        if not vals or not cal:
            raise SystemExit(f"{path}: no {counter} rows for {kernel_prefix} or calibration")
        return sum(vals) / len(vals), max(cal), len(vals)

    known = calib_mib * float(1 << 20)
    f_raw, f_cal, nf = per_kernel(fetch_csv, "FETCH_SIZE")
    w_raw, w_cal, nw = per_kernel(write_csv, "WRITE_SIZE")
    ff, fw = known / f_cal, known / w_cal
    total = f_raw * ff + w_raw * fw
    with open(out, "w") as fh:
        fh.write(f"# HBM traffic of {kernel_prefix} ({workload}, {precision}) from rocprofv3 "
                 "counters\n")
        fh.write(f"# command (FETCH_SIZE pass; the WRITE_SIZE pass is the same with "
                 f"--pmc WRITE_SIZE):\n#   {command}\n")
        fh.write(f"# calibration: torch elementwise multiply reading and writing {calib_mib} "
                 "MiB; counter scale = known bytes / counted bytes\n")
        fh.write(f"kernel: {kernel_prefix}\nworkload: {workload}\nprecision: {precision}\n"
                 f"shape: {shape}\n")
        fh.write(f"dispatches: {nf} (fetch), {nw} (write)\n")
        fh.write(f"fetch_raw_bytes_per_launch: {f_raw:.6e}\nfetch_scale: {ff:.4f}\n")
        fh.write(f"write_raw_bytes_per_launch: {w_raw:.6e}\nwrite_scale: {fw:.4f}\n")
        fh.write(f"hbm_bytes_per_launch: {total:.6e}\n")
        fh.write(f"source_sha256: {burst_source_hash(files)}\n")
    print(open(out).read())


# rocprofv3 --pmc passes for the utilisation figures (each fits one pass: at most 8 SQ and
# 2 GRBM counters, derived metrics counted by their inputs).
COUNTER_PASSES = {
    "valu": ["SQ_INSTS_VALU", "SQ_INSTS_VALU_FMA_F64", "SQ_INSTS_VALU_ADD_F64",
             "SQ_INSTS_VALU_MUL_F64", "VALUBusy", "VALUUtilization"],
    "lds": ["SQ_INSTS_LDS", "SQ_WAIT_INST_LDS", "LdsUtil", "LdsBankConflict", "MfmaUtil",
            "SQ_INSTS_VALU_MFMA_MOPS_BF16", "SQ_INSTS_VALU_FMA_F32"],
}
CUS, CLOCK = 256, 2.4e9  # MI355X compute units and peak engine clock
# One wave64 VALU instruction occupies a 16-lane SIMD for 4 clocks and a CU has 4 SIMDs:
# the chip issues at most CUS * CLOCK wave instructions per second.
VALU_ISSUE_PEAK = CUS * CLOCK
PEAK_MFMA_BF16 = 2.5e15


def calibration_copy(mib):
    """A plain streaming kernel of known traffic for scaling HBM byte counters: torch's
    vectorized elementwise multiply by one reading MIB MiB and writing MIB MiB, twice."""
    import torch
    n = mib * (1 << 20) // 8
    src = torch.ones(n, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(2):
        torch.mul(src, 1.0, out=dst)
    torch.cuda.synchronize()
    del src, dst


def short_kernel_name(name):
    """A demangled kernel name without its namespace, return type and parameter list."""
    name = name.replace("pdk::(anonymous namespace)::", "")
    if name.startswith("void "):
        name = name[5:]
    return name.split("(")[0] if not name.startswith("(") else name


def stats_summary(csv_path, out, title, command, top=20, keep=""):
    """A rocprofv3 --stats kernel table (kernel_stats.csv) as a short text summary: the
    `top` kernels by total time, and every kernel whose name contains one of the
    '|'-separated names in `keep`."""
    import csv
    rows = list(csv.DictReader(open(csv_path)))
    rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
    for r in rows:
        r["Name"] = short_kernel_name(r["Name"])
    keys = [k for k in keep.split("|") if k]
    rows = [r for k, r in enumerate(rows) if k < top or any(x in r["Name"] for x in keys)]
    with open(out, "w") as fh:
        for line in title.strip().splitlines():
            fh.write(f"# {line}\n")
        fh.write(f"# command:\n#   {command}\n")
        fh.write(f"{'kernel':<66} {'calls':>6} {'avg_us':>12} {'min_us':>12} {'max_us':>12} "
                 f"{'total_ms':>12} {'pct':>7}\n")
        for r in rows:
            fh.write(f"{r['Name'][:66]:<66} {int(r['Calls']):>6} "
                     f"{float(r['AverageNs']) / 1e3:>12.2f} {float(r['MinNs']) / 1e3:>12.2f} "
                     f"{float(r['MaxNs']) / 1e3:>12.2f} {float(r['TotalDurationNs']) / 1e6:>12.3f} "
                     f"{float(r['Percentage']):>7.2f}\n")
    print(open(out).read())


def counter_file(kernel, workload, precision):
    return os.path.join(ROOT, "profiles", f"{kernel}_{workload}_{precision}_counters.txt")


def counter_summary(csvs, kernel_prefix, last, out, command, workload, precision, shape,
                    files=None):
    """Per-dispatch averages of rocprofv3 --pmc counters for one kernel (the last `last`
    dispatches of it in each file when last > 0), with the per-launch counts the bench
    lines turn into rates: VALU wave instructions, FP64 flops issued (64 lanes x (add + mul
    + 2 fma) instructions), bfloat16 MFMA flops (512 per MOPS unit), LDS instructions."""
    import csv
    vals, durs, counts = {}, [], {}
    for path in csvs:
        per = {}
        for r in csv.DictReader(open(path)):
            if kernel_prefix not in r["Kernel_Name"]:
                continue
            d = int(r["Dispatch_Id"])
            e = per.setdefault(d, {"dur": float(r["End_Timestamp"]) - float(r["Start_Timestamp"])})
            e[r["Counter_Name"]] = e.get(r["Counter_Name"], 0.0) + float(r["Counter_Value"])
        ids = sorted(per)
        if last > 0:
            ids = ids[-last:]
        if not ids:
            raise SystemExit(f"{path}: no dispatches of {kernel_prefix}")
        for d in ids:
            durs.append(per[d]["dur"])
            for k, v in per[d].items():
                if k != "dur":
                    vals.setdefault(k, []).append(v)
        counts[f"pass {len(counts) + 1}"] = len(ids)
    avg = {k: sum(v) / len(v) for k, v in vals.items()}
    g = lambda k: avg.get(k, 0.0)
    derived = {
        "valu_insts_per_launch": g("SQ_INSTS_VALU"),
        "fp64_flops_per_launch": 64.0 * (g("SQ_INSTS_VALU_ADD_F64") + g("SQ_INSTS_VALU_MUL_F64")
                                         + 2.0 * g("SQ_INSTS_VALU_FMA_F64")),
        "fp32_fma_insts_per_launch": g("SQ_INSTS_VALU_FMA_F32"),
        "mfma_bf16_flops_per_launch": 512.0 * g("SQ_INSTS_VALU_MFMA_MOPS_BF16"),
        "lds_insts_per_launch": g("SQ_INSTS_LDS"),
        "pmc_run_launch_us": sum(durs) / len(durs) / 1e3,
    }
    with open(out, "w") as fh:
        fh.write(f"# rocprofv3 counters of {kernel_prefix} ({workload}, {precision}), averaged per "
                 "dispatch" + (f" over the last {last} dispatches of each pass" if last else "")
                 + "\n")
        fh.write("# commands (one pass per counter set; <set> is each key of COUNTER_PASSES in "
                 f"bench.py):\n#   {command}\n")
        fh.write("# VALUBusy, VALUUtilization, LdsUtil, LdsBankConflict, MfmaUtil: rocprofv3's "
                 "derived metrics (percent; LdsBankConflict in conflicts per access)\n")
        fh.write(f"kernel: {kernel_prefix}\nworkload: {workload}\nprecision: {precision}\n"
                 f"shape: {shape}\n")
        fh.write("dispatches: " + ", ".join(f"{v} ({k})" for k, v in counts.items()) + "\n")
        for k in sorted(avg):
            fh.write(f"{k}: {avg[k]:.6e}\n")
        for k, v in derived.items():
            fh.write(f"{k}: {v:.6e}\n")
        fh.write(f"source_sha256: {burst_source_hash(files)}\n")
    print(open(out).read())


def read_counters(kernel, workload, precision, shape, kern_s, files=None):
    """Utilisation of one launch of `kern_s` seconds (the bench's own live timing) from the
    committed counter summary: VALU issue-slot fraction, FP64 and bfloat16 MFMA rates
    against their peaks, and rocprofv3's busy/utilisation metrics.  None when there is no
    summary for this kernel, workload and launch shape, or the kernel changed since."""
    path = counter_file(kernel, workload, precision)
    if not os.path.exists(path):
        return None
    kv = {}
    with open(path) as fh:
        for line in fh:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
    if kv.get("source_sha256") != burst_source_hash(files) or kv.get("shape") != shape:
        return None
    f = lambda k: float(kv[k]) if k in kv else None
    out = {"source": os.path.relpath(path, ROOT),
           "valu_insts_per_launch": f("valu_insts_per_launch"),
           "valu_issue_frac": f("valu_insts_per_launch") / kern_s / VALU_ISSUE_PEAK,
           "fp64_issued_tflops": f("fp64_flops_per_launch") / kern_s / 1e12,
           "fp64_issued_frac": f("fp64_flops_per_launch") / kern_s / PEAK["f64"],
           "lds_insts_per_launch": f("lds_insts_per_launch"),
           "pmc_run_launch_us": f("pmc_run_launch_us")}
    if f("mfma_bf16_flops_per_launch"):
        out["mfma_bf16_tflops"] = f("mfma_bf16_flops_per_launch") / kern_s / 1e12
        out["mfma_bf16_frac"] = f("mfma_bf16_flops_per_launch") / kern_s / PEAK_MFMA_BF16
    for k in ("VALUBusy", "VALUUtilization", "LdsUtil", "LdsBankConflict", "MfmaUtil"):
        if k in kv:
            out[k] = float(kv[k])
    return out


def cpu_baseline(prob, budget_s, steps_cap):
    """The FP64 CPU oracle on a bounded sample of the same workload: whole macro steps of
    the full grid on the host cores (OpenMP over patches)."""
    from oracle import pdo
    from paper_2405_08764_amd import workloads as W
    threads = max(1, min(16, os.cpu_count() or 1))
    o = pdo.Oracle(prob, threads=threads)
    _ = o.coef
    U = o.initial()
    t = prob["time"]
    done, el = 0, 0.0
    while done < steps_cap and (done == 0 or el < budget_s):
        s = time.perf_counter()
        U = o.step(U, t["t0"] + done * t["dt_macro"])
        el += time.perf_counter() - s
        done += 1
    ups = W.updates_per_step(prob) * done / el
    return {"value": ups, "unit": "patch-point updates/s", "cores": o.L.pdo_get_threads(),
            "kind": "oracle",
            "sample": f"{done} macro step(s) of the full grid ({o.P} patches x "
                      f"{o.mx}x{o.me} points x {t['n_t']} nano steps), {el:.1f} s",
            "macro_steps_per_s": done / el}


BATCH_SOURCES = ["pd_batch.hip", "pd_burst.inc", "pd_internal.h"]
CLOSURE_SOURCES = ["pd_closure.hip", "pd_internal.h"]


def host_info():
    """Host cores and CPU model of the machine the oracle runs on."""
    model = ""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"host_cpu_count": os.cpu_count(), "host_cpu_model": model,
            "omp_num_threads": os.environ.get("OMP_NUM_THREADS")}


def oracle_threads():
    """Threads for the all-cores leg: the host's cores, capped by OMP_NUM_THREADS (the
    CPU share a one-GPU job is given)."""
    n = os.cpu_count() or 1
    cap = os.environ.get("OMP_NUM_THREADS")
    if cap and cap.isdigit() and int(cap) > 0:
        n = min(n, int(cap))
    return n


def batch_cpu_baseline(probs, per_step_updates, budget_s, threads, patches=256, seed=1):
    """The FP64 oracle on a bounded sample of the mixed batch: seeded members in a seeded
    order, each advancing `patches` seeded patches (all of a smaller member) through one
    whole macro step (edge data, lift, burst, restriction, projection); coefficient
    planes of those patches are built before the clock starts.  Returns the rate and the
    batch macro steps/s it implies (the full batch's updates per step at that rate)."""
    import numpy as np
    from oracle import pdo
    rng = np.random.default_rng(seed)
    order = rng.permutation(len(probs))
    done_updates, el, used, members = 0, 0.0, 0, 0
    for i in order:
        if el >= budget_s:
            break
        p = probs[i]
        o = pdo.Oracle(p, threads=threads)
        k = min(patches, o.P)
        mask = np.zeros(o.P, dtype=np.uint8)
        mask[rng.choice(o.P, size=k, replace=False)] = 1
        o.coefficients_for(mask)
        U = o.initial()
        t = p["time"]
        s = time.perf_counter()
        o.step(U, t["t0"], mask=mask)
        el += time.perf_counter() - s
        done_updates += k * o.mx * o.me * t["n_t"]
        used = o.L.pdo_get_threads()
        members += 1
    rate = done_updates / el
    return {"value": rate, "unit": "patch-point updates/s", "cores": used, "kind": "oracle",
            "sample": f"{members} seeded members of the batch, up to {patches} seeded patches "
                      f"each, one whole macro step each: {done_updates:.3e} updates in "
                      f"{el:.1f} s",
            "batch_macro_steps_per_s_at_this_rate": rate / per_step_updates}


def make_batch(n_instances, n_steps, shapes_path=None, log=None):
    """The mixed batch (time parameters at 0.4 of each member's explicit bounds) with its
    launch shapes: read from shapes_path when that file exists, else autotuned (and
    written there).  Returns (probs, grids, batch, tuned_ms or None)."""
    from paper_2405_08764_amd import pd
    from paper_2405_08764_amd import workloads as W
    probs, grids = [], []
    for p in W.config4(n_instances):
        g = pd.Grid(p)
        info = g.query()
        g.prob = W.fit_time(p, info.dt_macro_limit, info.dt_micro_limit, n_steps)
        probs.append(g.prob)
        grids.append(g)
    B = pd.Batch(grids)
    tuned_ms = None
    if shapes_path and os.path.exists(shapes_path):
        with open(shapes_path) as fh:
            shapes = json.load(fh)
        assert len(shapes) == len(grids), "shape file is for another batch"
        for i, sh in enumerate(shapes):
            B.set_shape(i, int(sh))
        if log:
            log(f"launch shapes read from {shapes_path}")
    else:
        tuned_ms = B.autotune(reps=2)
        if shapes_path:
            with open(shapes_path, "w") as fh:
                json.dump([B.shape(i)[0] for i in range(len(grids))], fh)
    return probs, grids, B, tuned_ms


def reset_fields(grids, B):
    for g, U in zip(grids, B.U):
        g.initial(U=U)


def time_launches(stream, launch, reps):
    """Average seconds per call of `launch`: one untimed call, then `reps` calls back to
    back between one pair of HIP events recorded on the stream they run on.  (An event pair
    around every call adds the event packets' own processing to each launch: 10-50 us
    on a 40-200 us kernel, against rocprofv3's kernel trace.)"""
    import torch
    launch()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record(stream)
    for _ in range(reps):
        launch()
    b.record(stream)
    torch.cuda.synchronize()
    return a.elapsed_time(b) / reps / 1e3


def time_batch(B, grids, warmup, steps, stream, closure=False):
    """`warmup` untimed batch macro steps from the initial data, then the initial data
    again and `steps` timed steps (HIP events on the launch stream, and the host clock
    around synchronisations).  Returns (seconds, event seconds)."""
    import torch
    run = B.closure_solve if closure else B.solve
    reset_fields(grids, B)
    if warmup:
        run(warmup)
    torch.cuda.synchronize()
    reset_fields(grids, B)
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    s = time.perf_counter()
    a.record(stream)
    run(steps)
    b.record(stream)
    torch.cuda.synchronize()
    el = time.perf_counter() - s
    B.sync()
    return el, a.elapsed_time(b) / 1e3


def batch_line(grids, B, tuned_ms, el, ev_s, args, untuned_items=None):
    """The plain batch part of a JSON line: rates, shapes and the k_batch roofline."""
    from paper_2405_08764_amd import pd
    binfo = B.query()
    per_step = binfo.updates_per_step
    shapes = {}
    for i in range(len(grids)):
        sh, ppb = B.shape(i)
        shapes.setdefault(f"m={grids[i].mx}", set()).add(f"{pd.BATCH_MENU[sh]}x{ppb}")
    kern_s = ev_s / args.steps  # one k_batch launch per step (+ a table fill every 16)
    achieved = 20 * per_step / kern_s
    peak = PEAK["f64"]
    n_ts = [g.prob["time"]["n_t"] for g in grids]
    traffic = read_traffic("k_batch", "config4", "f64", "tuned", BATCH_SOURCES)
    cfg = {"patches": sum(g.P for g in grids),
           "micro_points": sum(g.P * g.mx * g.me for g in grids),
           "updates_per_step": per_step, "n_t_range": [min(n_ts), max(n_ts)],
           "items": binfo.n_items, "blocks": binfo.blocks, "lds_bytes": binfo.lds_bytes,
           "shapes": {k: sorted(v) for k, v in sorted(shapes.items())},
           "autotune_ms": tuned_ms}
    roof = {"bound": "alu", "achieved": achieved / 1e12, "peak": peak / 1e12,
            "unit": "TFLOP/s", "frac": achieved / peak, "traffic": traffic,
            "kernel": "k_batch (persistent, one batch macro step per launch)",
            "kernel_ms": kern_s * 1e3, "flops_per_update": 20,
            "issued_flops_per_update": 12,
            "issued_frac": 12 * per_step / kern_s / peak,
            "counters": read_counters("k_batch", "config4", "f64", "tuned", kern_s,
                                      BATCH_SOURCES)}
    return per_step, cfg, roof


def bench_batch(args):
    """The mixed batch alone: every instance advances one macro step per persistent
    launch."""
    import torch
    torch.cuda.set_device(0)
    stream = torch.cuda.Stream()
    log = lambda *a: print("[bench]", *a, file=sys.stderr, flush=True)
    with torch.cuda.stream(stream):
        t0 = time.perf_counter()
        probs, grids, B, tuned_ms = make_batch(args.instances, args.steps, args.batch_shapes,
                                               log)
        log(f"batch of {len(grids)} ready in {time.perf_counter() - t0:.1f} s")
        el, ev_s = time_batch(B, grids, args.warmup, args.steps, stream)
        if args.calibrate_copy:
            calibration_copy(args.calibrate_copy)
    per_step, cfg, roof = batch_line(grids, B, tuned_ms, el, ev_s, args)
    out = {
        "metric": "patch-point updates/s (and macro steps/s) of the batched plain scheme",
        "value": per_step * args.steps / el, "unit": "patch-point updates/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": el / args.steps * 1e3, "macro_steps_per_s": args.steps / el,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic (seeded analytic coefficients, no dataset)",
        "config": dict({"workload": f"config4: {len(grids)} mixed instances (tanh squares "
                                    "and annuli, N 17..129, m 9..33, Fourier D and v, eps "
                                    "1e-3..1e-2, reaction 0..2), one persistent launch per "
                                    "step"}, **cfg),
        "roofline": roof,
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = batch_cpu_baseline(probs, per_step, args.cpu_seconds,
                                                 oracle_threads())
        out["cpu_baseline"].update(host_info())
    print(json.dumps(out), flush=True)


def trace_avg_us(path, kernel):
    """Average duration (us) of `kernel` in a committed kernel-table summary, or None."""
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        for line in fh:
            if not line.startswith("#") and kernel in line:
                nums = line.split()[-6:]
                try:
                    return float(nums[1])
                except (ValueError, IndexError):
                    return None
    return None


def closure_kernel_roofline(n_patches):
    """k_closure_step against its two roofs: bfloat16 MFMA for the network (2 x (33 x 128 +
    128 x 128 + 128) flops per patch) and HBM (each patch's static table of 12 doubles,
    its macro value read and written, F_hat written: 120 bytes), with the duration from
    the committed rocprofv3 trace of the closure batch (the kernel runs inside the
    closure graph, so it is not timed apart here) and the counters taken with it."""
    stats = os.path.join(ROOT, "profiles", "k_closure_step_config5_kernel_stats.txt")
    us = trace_avg_us(stats, "k_closure_step")
    if us is None:
        return None
    flops = n_patches * 2.0 * (33 * 128 + 128 * 128 + 128)
    nbytes = n_patches * 120.0
    t = us * 1e-6
    return {"kernel": "k_closure_step (features, bf16 MFMA network, projective update; "
                      "one batch step)",
            "duration_us": us, "duration_source": os.path.relpath(stats, ROOT),
            "mfma": {"achieved_tflops": flops / t / 1e12, "peak_tflops": PEAK_MFMA_BF16 / 1e12,
                     "frac": flops / t / PEAK_MFMA_BF16, "flops_per_launch": flops},
            "hbm": {"achieved_gbs": nbytes / t / 1e9, "peak_gbs": 8000.0,
                    "frac": nbytes / t / 8e12, "algorithmic_bytes": nbytes,
                    "traffic": read_traffic("k_closure_step", "config5", "f64", "closure",
                                            CLOSURE_SOURCES)},
            "counters": read_counters("k_closure_step", "config5", "f64", "closure", t,
                                      CLOSURE_SOURCES)}


def closure_part(args, B, grids, stream, t_plain, ref, log):
    """Train the closure on plain-scheme pairs of disjoint instances and time the batch
    with it (spot checks on 1% of the work items per step, per-member fallback): rates,
    error against the plain batch over the same steps, and the baseline operator alone."""
    import numpy as np
    import torch

    from paper_2405_08764_amd import closure_train as T
    N = args.steps
    s = time.perf_counter()
    tg = T.instance_grids(args.train_instances, T.TRAIN_SEED, 40)
    X, y = T.generate(tg, steps=16, every=2, max_pairs=args.train_pairs)
    n_pairs = int(X.shape[0])
    torch.cuda.synchronize()
    t_gen = time.perf_counter() - s
    s = time.perf_counter()
    C, losses = T.train(X, y, epochs=args.epochs, batch=4096, lr=2e-3)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - s
    ym, ysd = C.target_scale()
    rms = float(np.sqrt(losses[-1])) * ysd  # residual RMS in units of s
    threshold = args.threshold_factor * rms
    log(f"pairs {n_pairs} generated in {t_gen:.1f} s, trained in {t_train:.1f} s, "
        f"loss {losses[0]:.4g} -> {losses[-1]:.4g}, threshold {threshold:.3g}")
    del tg, X, y
    B.attach_closure(C, stride=100, threshold=threshold)
    B.closure_stats(reset=True)
    t_cl, ev_cl = time_batch(B, grids, args.warmup, N, stream, closure=True)
    checked, fallbacks = B.closure_stats()
    # the warm-up steps are counted too: report the timed steps' share
    errs = np.array([T.rel_l2(a, b) for a, b in zip(B.U, ref)])
    Z = T.zero_closure(C)
    B.attach_closure(Z, stride=100, threshold=1e30)
    reset_fields(grids, B)
    B.closure_solve(N)
    torch.cuda.synchronize()
    errs0 = np.array([T.rel_l2(a, b) for a, b in zip(B.U, ref)])
    P = sum(g.P for g in grids)
    part = {
        "macro_steps_per_s": N / t_cl, "ms_per_step": t_cl / N * 1e3,
        "speedup_vs_plain": t_plain / t_cl,
        "rel_l2_vs_plain": {"steps": N, "max": float(errs.max()), "mean": float(errs.mean())},
        "rel_l2_baseline_operator_only": {"max": float(errs0.max()),
                                          "mean": float(errs0.mean())},
        "spot_checks": {"patches_checked": checked,
                        "fraction": checked / (P * (N + args.warmup)),
                        "member_fallbacks": fallbacks, "threshold": threshold},
        "training": {"pairs": n_pairs, "epochs": args.epochs,
                     "loss_first": float(losses[0]), "loss_last": float(losses[-1]),
                     "generate_s": t_gen, "train_s": t_train},
        "dtype": "bf16 MFMA (fp32 accumulate) closure, f64 plain fallback",
        "closure_kernel": closure_kernel_roofline(P),
    }
    return C, threshold, part


def closure_horizon(args, C, threshold, log):
    """The closure against the plain scheme over a long horizon on held-out members (the
    first members of the evaluation batch; training used other seeds)."""
    import numpy as np
    import torch

    from paper_2405_08764_amd import closure_train as T
    from paper_2405_08764_amd import pd
    from paper_2405_08764_amd import workloads as W
    n, H = args.horizon_members, args.horizon_steps
    grids = T.instance_grids(n, W.MASTER_SEED + 4000, H)
    U0 = [g.initial() for g in grids]
    B = pd.Batch(grids, [u.clone() for u in U0])
    B.autotune(reps=1)
    s = time.perf_counter()
    B.solve(H)
    torch.cuda.synchronize()
    t_plain = time.perf_counter() - s
    ref = [u.clone() for u in B.U]
    for u, u0 in zip(B.U, U0):
        u.copy_(u0)
    B.attach_closure(C, stride=100, threshold=threshold)
    B.closure_stats(reset=True)
    s = time.perf_counter()
    B.closure_solve(H)
    torch.cuda.synchronize()
    t_cl = time.perf_counter() - s
    checked, fallbacks = B.closure_stats()
    errs = np.array([T.rel_l2(a, b) for a, b in zip(B.U, ref)])
    log(f"horizon {H} steps on {n} members: max {errs.max():.3g}, mean {errs.mean():.3g}")
    return {"members": n, "steps": H, "max": float(errs.max()), "mean": float(errs.mean()),
            "member_fallbacks": fallbacks, "plain_s": t_plain, "closure_s": t_cl}


def bench_closure(args):
    """The mixed batch with the learned closure standing in for the micro-bursts, against
    the plain batched scheme on the same batch."""
    return bench_headline(args, workload_name="config5")


def bench_headline(args, workload_name="config4+config5"):
    """The metric's pairing on one GPU: the plain batched scheme (config 4, FP64) and the
    same batch with the learned closure (config 5), in one line."""
    import torch
    torch.cuda.set_device(0)
    stream = torch.cuda.Stream()
    log = lambda *a: print("[bench]", *a, file=sys.stderr, flush=True)
    with torch.cuda.stream(stream):
        t0 = time.perf_counter()
        probs, grids, B, tuned_ms = make_batch(args.instances, args.steps, args.batch_shapes,
                                               log)
        log(f"batch of {len(grids)} ready in {time.perf_counter() - t0:.1f} s")
        el, ev_s = time_batch(B, grids, args.warmup, args.steps, stream)
        ref = [u.clone() for u in B.U]
        log(f"plain: {args.steps / el:.3f} batch steps/s")
        C, threshold, surrogate = closure_part(args, B, grids, stream, el, ref, log)
        if args.horizon_steps > 0:
            surrogate["rel_l2_vs_plain_long_horizon"] = closure_horizon(args, C, threshold,
                                                                        log)
        if args.calibrate_copy:
            calibration_copy(args.calibrate_copy)
    per_step, cfg, roof = batch_line(grids, B, tuned_ms, el, ev_s, args)
    out = {
        "metric": "patch-point updates/s + macro steps/s at fixed L2 err; surrogate vs "
                  "plain GPU",
        "value": per_step * args.steps / el, "unit": "patch-point updates/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": el / args.steps * 1e3, "macro_steps_per_s": args.steps / el,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic (seeded analytic coefficients, no dataset)",
        "config": dict({"workload": f"{workload_name}: plain batched scheme (FP64) on "
                                    f"{len(grids)} mixed instances (tanh squares and annuli, "
                                    "N 17..129, m 9..33, Fourier D and v, eps 1e-3..1e-2, "
                                    "reaction 0..2), one persistent launch per step; and the "
                                    "same batch with the learned closure (bf16 MFMA MLP "
                                    "33-128-128-1, 1% spot checks, per-member fallback)"},
                       **cfg),
        "roofline": roof,
        "surrogate": surrogate,
    }
    if not args.no_cpu_baseline:
        cb = batch_cpu_baseline(probs, per_step, args.cpu_seconds, oracle_threads())
        one = batch_cpu_baseline(probs, per_step, args.cpu_seconds_one, 1, patches=32)
        cb["one_thread"] = {k: one[k] for k in ("value", "cores", "sample",
                                                "batch_macro_steps_per_s_at_this_rate")}
        cb.update(host_info())
        out["cpu_baseline"] = cb
    print(json.dumps(out), flush=True)


def fix_shape(pd, g, shape):
    """Fixes the burst's launch shape from "exchange,cols,rows,patches_per_block"."""
    xch, cols, rows, ppb = (int(v) for v in shape.split(","))
    g.set_option(pd.OPT_EXCHANGE, xch)
    g.set_option(pd.OPT_COLS_PER_LANE, cols)
    g.set_option(pd.OPT_ROWS_PER_LANE, rows)
    g.set_option(pd.OPT_PATCHES_PER_BLOCK, ppb)


def bench_refresh(args):
    """Config-2 macro steps with the edge data refreshed between sub-bursts
    (pd_macro_step_refresh), against the frozen-edge fused step of the same problem."""
    import torch

    from paper_2405_08764_amd import pd
    from paper_2405_08764_amd import workloads as W
    prob = W.config2()
    t = prob["time"]
    Q = args.refresh
    K = args.steps
    torch.cuda.set_device(0)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        g = pd.Grid(prob)
        U = g.initial()
        V = g.new_U()
        # the sub-bursts run on the grid's launch shape (split mode), tuned on the fused step
        tuned_ms = None
        if args.shape:
            fix_shape(pd, g, args.shape)
        elif not args.no_autotune:
            tuned_ms = g.autotune(U, reps=5)
        if args.no_resident:
            g.set_option(pd.OPT_RESIDENT_SOLVE, 0)
        for s in range(args.warmup):
            g.macro_step_refresh(U, t["t0"] + s * t["dt_macro"], Q, out=V)
            U, V = V, U
        g.sync()
        U = g.initial()
        torch.cuda.synchronize()
        s0 = time.perf_counter()
        for s in range(K):
            g.macro_step_refresh(U, t["t0"] + s * t["dt_macro"], Q, out=V)
            U, V = V, U
        torch.cuda.synchronize()
        el = time.perf_counter() - s0
        g.sync()
        info = g.query()
        resident = bool(info.resident_refresh)
        n_sub = t["n_t"] // Q
        if resident:
            # the dominant kernel: the resident refreshed step (k_refresh_x, one launch per
            # macro step with its three small set-up launches), timed with HIP events
            kern_s = time_launches(
                stream, lambda: g.macro_step_refresh(U, t["t0"], Q, out=V), args.kernel_reps)
        else:
            # the dominant kernel: one sub-burst (split-mode burst), timed with HIP events
            state, edge = g.lift_bc(U)
            kern_s = time_launches(
                stream, lambda: g.micro_burst(state, edge, t["t0"], t["dt_micro"], n_sub),
                args.kernel_reps)
        g.sync()
        if args.calibrate_copy:
            calibration_copy(args.calibrate_copy)
        # the frozen-edge fused step on the same problem (autotuned, graph replay)
        gf = pd.Grid(prob)
        Uf = gf.initial()
        gf.autotune(Uf, reps=5)
        gf.solve(Uf, n_steps=32)
        gf.sync()
        Uf = gf.initial()
        torch.cuda.synchronize()
        s0 = time.perf_counter()
        gf.solve(Uf, n_steps=K)
        torch.cuda.synchronize()
        t_fused = (time.perf_counter() - s0) / K
        gf.sync()
    per_step = W.updates_per_step(prob)
    shape = f"{info.exchange},{info.cols_per_lane},{info.rows_per_lane},{info.patches_per_block}"
    if resident:
        achieved = 20 * per_step / kern_s
        kname, kfiles = "k_refresh_x", SOLVE_SOURCES
        ktxt = "k_refresh_x (resident: the whole refreshed step, set-up launches included)"
    else:
        achieved = 20 * info.n_points * n_sub / kern_s
        kname, kfiles = KERNEL_NAME[info.exchange], None
        ktxt = KERNEL_NAME[info.exchange] + " (split mode: one sub-burst)"
    traffic = read_traffic(kname, "refresh", "f64", shape, kfiles)
    out = {
        "metric": "patch-point updates/s (and macro steps/s) with the edge data refreshed "
                  "during the burst",
        "value": per_step * K / el, "unit": "patch-point updates/s",
        "n_gpus": 1, "steps": K, "warmup": args.warmup, "ms_per_step": el / K * 1e3,
        "macro_steps_per_s": K / el,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic (seeded analytic coefficients, no dataset)",
        "config": {"workload": f"refresh: config-2 problem (65x65 macro nodes, 17x17 micro "
                               f"points per patch, n_t = {t['n_t']}) with the edge data "
                               f"refreshed {Q - 1} times per burst ({Q} sub-bursts)",
                   "n_refresh": Q, "updates_per_step": per_step,
                   "launch": {"exchange": {1: "lds", 2: "in-wave", 3: "hybrid"}[info.exchange],
                              "cols_per_lane": info.cols_per_lane,
                              "rows_per_lane": info.rows_per_lane,
                              "patches_per_block": info.patches_per_block,
                              "block_threads": info.block_threads, "tuned_ms": tuned_ms}},
        "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK["f64"] / 1e12,
                     "unit": "TFLOP/s", "frac": achieved / PEAK["f64"], "traffic": traffic,
                     "kernel": ktxt, "kernel_ms": kern_s * 1e3, "flops_per_update": 20,
                     "counters": read_counters(kname, "refresh", "f64", shape, kern_s,
                                               kfiles)},
        "frozen_edge_fused_ms_per_step": t_fused * 1e3,
    }
    if not args.no_cpu_baseline:
        from oracle import pdo
        threads = max(1, min(16, os.cpu_count() or 1))
        o = pdo.Oracle(prob, threads=threads)
        _ = o.coef
        Uo = o.initial()
        done, el_c = 0, 0.0
        while done < 200 and (done == 0 or el_c < args.cpu_seconds):
            s0 = time.perf_counter()
            Uo = o.step_refresh(Uo, t["t0"] + done * t["dt_macro"], Q)
            el_c += time.perf_counter() - s0
            done += 1
        out["cpu_baseline"] = {"value": per_step * done / el_c, "unit": "patch-point updates/s",
                               "cores": o.L.pdo_get_threads(), "kind": "oracle",
                               "sample": f"{done} refreshed macro step(s) of the full grid, "
                                         f"{el_c:.1f} s"}
    print(json.dumps(out), flush=True)


def bench_adi(args):
    """The ADI micro solver on a GPU-sized macro grid (sine map lambda = 0.1, f = 20,
    h = 1e-3, tau = 1e-6, 10 micro intervals, n_t = 2): lift and edge data, ADI burst,
    restriction, projective step.  adi: Sec. 4.1.1's setup (D = 1, v = (10x, 10y), 2-point
    upwind); adi-upwind: Sec. 4.1.2's (D = 1 + x, v = (1 + 10x, 10y)) with the 3- or
    4-point upwind first differences in the ADI solver."""
    import torch

    from paper_2405_08764_amd import pd
    from paper_2405_08764_amd import workloads as W
    n = args.adi_n
    hu = args.workload == "adi-upwind"
    points, r = args.upwind_points, args.upwind_r
    prob = W.paper_cdr(2 if hu else 1, lam=0.1, n=n, m=11)
    torch.cuda.set_device(0)
    stream = torch.cuda.Stream()
    K = args.steps
    with torch.cuda.stream(stream):
        g = pd.Grid(prob)
        info = g.query()
        dtm = 0.4 * info.dt_macro_limit
        t = prob["time"]
        dt, n_t = t["dt_micro"], t["n_t"]

        def burst(state, edge, tn):
            if hu:
                g.micro_burst_adi_upwind(state, edge, tn, dt, n_t, points, r)
            else:
                g.micro_burst_adi(state, edge, tn, dt, n_t)

        def step(U, tn):
            state, edge = g.lift_bc(U)
            burst(state, edge, tn)
            return g.macro_step(U, tn, dt_macro=dtm, dt_micro=dt, n_t=n_t,
                                Ubar=g.restrict(state))

        U = g.initial()
        for s in range(args.warmup):
            U = step(U, s * dtm)
        g.sync()
        U = g.initial()
        torch.cuda.synchronize()
        s0 = time.perf_counter()
        for s in range(K):
            U = step(U, s * dtm)
        torch.cuda.synchronize()
        el = time.perf_counter() - s0
        g.sync()
        state, edge = g.lift_bc(U)
        kern_s = time_launches(stream, lambda: burst(state, edge, 0.0), args.kernel_reps)
        if args.calibrate_copy:
            calibration_copy(args.calibrate_copy)
    pts = info.n_points
    n_src = len(prob["src"])
    if hu:
        # per point and nano step, each half: the explicit 5-point operator across the
        # line (10), the five band entries (10), the source (2 per term), the banded
        # elimination (about 16) and back substitution (4)
        flops_per_update = 2 * (10 + 10 + 2 * n_src + 16 + 4)
        kern, files, shape = "k_burst_adi_hu", ADU_SOURCES, f"p{points}"
        desc = (f"adi-upwind: Sec. 4.1.2 problem (sine map lambda 0.1, D = 1 + x, "
                f"v = (1 + 10x, 10y), f = 20, exact e^(x+y+t)) on {n}x{n} macro nodes, "
                f"11x11 micro points, h = 1e-3, tau = 1e-6, n_t = 2 ADI steps with the "
                f"{points}-point upwind first differences" + (f" (r = {r})" if points == 4
                                                               else "") +
                ", dt_macro at 0.4 of the macro bound")
        ktxt = "k_burst_adi_hu (banded ADI burst)"
    else:
        # per point and nano step: two tridiagonal rows (about 6 flops each), two explicit
        # half-operator evaluations (about 8 each), the source (2 per term each half), the
        # Thomas forward and backward passes (about 5 each)
        flops_per_update = 2 * (6 + 8 + 2 * n_src + 5)
        kern, files, shape = "k_burst_adi_r", ADI_SOURCES, "adi"
        desc = (f"adi: Sec. 4.1.1 problem (sine map lambda 0.1, D = 1, v = (10x, 10y), "
                f"f = 20, exact e^(x+y+t)) on {n}x{n} macro nodes, 11x11 micro points, "
                f"h = 1e-3, tau = 1e-6, n_t = 2 ADI steps, dt_macro at 0.4 of the macro bound")
        ktxt = "k_burst_adi_r (register-line ADI burst)"
    alg_bytes = pts * 8 * (2 + 5 + n_src) + info.n_patches * 4 * info.m_xi * 8
    out = {
        "metric": "patch-point updates/s of the ADI micro burst (Sec. 4.1.2 setup, higher-"
                  "order upwind)" if hu else
                  "patch-point updates/s of the ADI micro burst (Sec. 4.1.1 setup)",
        "value": pts * n_t * K / el, "unit": "patch-point updates/s",
        "n_gpus": 1, "steps": K, "warmup": args.warmup, "ms_per_step": el / K * 1e3,
        "macro_steps_per_s": K / el,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic (the paper's analytic coefficients, no dataset)",
        "config": {"workload": desc,
                   "patches": info.n_patches, "dt_macro": dtm,
                   "dt_micro_over_explicit_bound": dt / info.dt_micro_limit},
        "roofline": {"bound": "alu", "achieved": flops_per_update * pts * n_t / kern_s / 1e12,
                     "peak": PEAK["f64"] / 1e12, "unit": "TFLOP/s",
                     "frac": flops_per_update * pts * n_t / kern_s / PEAK["f64"],
                     "traffic": read_traffic(kern, args.workload, "f64", shape, files),
                     "algorithmic_bytes": alg_bytes,
                     "hbm_frac": alg_bytes / kern_s / 8e12,
                     "kernel": ktxt,
                     "kernel_ms": kern_s * 1e3, "flops_per_update": flops_per_update,
                     "counters": read_counters(kern, args.workload, "f64", shape, kern_s,
                                               files)},
    }
    if not args.no_cpu_baseline:
        # the oracle's ADI burst (numpy, dense line solves) on the first patches of the grid
        from oracle import adi, pdo
        o = pdo.Oracle(prob)
        Uo = o.initial()
        npat = 64
        u0, e = o.lift(Uo)[:npat], o.edge(Uo)[:npat]
        s0 = time.perf_counter()
        adi.adi_burst(prob["grid"], o.coef[:, :npat], u0, e, 0.0, dt, n_t,
                      adi.time_factors(prob), *((points, r) if hu else ()))
        el_c = time.perf_counter() - s0
        out["cpu_baseline"] = {"value": npat * info.m_xi * info.m_eta * n_t / el_c,
                               "unit": "patch-point updates/s", "cores": 1, "kind": "oracle",
                               "sample": f"one ADI burst ({n_t} steps) of {npat} patches, "
                                         f"{el_c:.1f} s"}
    print(json.dumps(out), flush=True)


def bench_upwind(args):
    """The config-2 problem with the 3- or 4-point upwind micro differences (the variant of
    Sec. 4.1.2) through the split path: lift and edge data, higher-order upwind burst,
    restriction, projective step.  Also times the burst kernel with each difference form,
    the cost comparison the paper reports."""
    import torch

    from paper_2405_08764_amd import pd
    from paper_2405_08764_amd import workloads as W
    points, r = args.upwind_points, args.upwind_r
    prob, desc = workload("config2")
    torch.cuda.set_device(0)
    stream = torch.cuda.Stream()
    K = args.steps
    t = prob["time"]
    dtm, dt, n_t = t["dt_macro"], t["dt_micro"], t["n_t"]
    with torch.cuda.stream(stream):
        g = pd.Grid(prob)
        info = g.query()

        def step(U, tn):
            state, edge = g.lift_bc(U)
            g.micro_burst_upwind(state, edge, tn, dt, n_t, points, r)
            return g.macro_step(U, tn, dt_macro=dtm, dt_micro=dt, n_t=n_t,
                                Ubar=g.restrict(state))

        U = g.initial()
        for s in range(args.warmup):
            U = step(U, s * dtm)
        g.sync()
        U = g.initial()
        torch.cuda.synchronize()
        s0 = time.perf_counter()
        for s in range(K):
            U = step(U, s * dtm)
        torch.cuda.synchronize()
        el = time.perf_counter() - s0
        g.sync()
        state, edge = g.lift_bc(U)
        kern = {}
        name = lambda p_, r_: f"{p_}-point" + (f" r={r_:g}" if p_ == 4 else "")
        for pts_, r_ in ((points, r), (2, 0.0), (3, 0.0), (4, 0.5)):
            if name(pts_, r_) in kern:
                continue
            kern[name(pts_, r_)] = time_launches(
                stream, lambda: g.micro_burst_upwind(state, edge, 0.0, dt, n_t, pts_, r_),
                args.kernel_reps)
        kern_s = kern[name(points, r)]
        g.sync()
        if args.calibrate_copy:
            # the streaming kernel of known traffic the counter summary is scaled by
            m = args.calibrate_copy * (1 << 20) // 8
            src = torch.ones(m, dtype=torch.float64, device="cuda")
            dst = torch.empty_like(src)
            for _ in range(2):
                torch.mul(src, 1.0, out=dst)
            torch.cuda.synchronize()
            del src, dst
    # config 2's 17 x 17 patches fit one wave: the in-wave kernel runs
    traffic = read_traffic("k_burst_hux", "upwind", "f64", "hux", HU_SOURCES)
    pts = info.n_points
    n_src = len(prob["src"])
    # per point and nano step: the folded 9-point cross on the increment (a multiply, eight
    # FMAs), the source (two FMAs over the time-dependent terms) scaled by dt onto the
    # lifted part (an FMA), the two adds forming the new increment
    flops_per_update = 1 + 2 * 8 + 2 * 2 + 2 + 1 + 1
    alg_bytes = pts * 8 * (2 + 5 + n_src) + info.n_patches * 4 * info.m_xi * 8
    form = f"{points}-point" + (f" (r = {r:g})" if points == 4 else "")
    out = {
        "metric": "patch-point updates/s of the higher-order upwind micro burst",
        "value": pts * n_t * K / el, "unit": "patch-point updates/s",
        "n_gpus": 1, "steps": K, "warmup": args.warmup, "ms_per_step": el / K * 1e3,
        "macro_steps_per_s": K / el,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic (seeded random Fourier coefficients, no dataset)",
        "config": {"workload": f"upwind: config2 ({desc}), {form} upwind micro "
                               f"differences, split path",
                   "patches": info.n_patches, "n_t": n_t, "dt_macro": dtm},
        "roofline": {"bound": "alu", "achieved": flops_per_update * pts * n_t / kern_s / 1e12,
                     "peak": PEAK["f64"] / 1e12, "unit": "TFLOP/s",
                     "frac": flops_per_update * pts * n_t / kern_s / PEAK["f64"],
                     "traffic": traffic, "algorithmic_bytes": alg_bytes,
                     "hbm_frac": alg_bytes / kern_s / 8e12,
                     "kernel": f"k_burst_hux (in-wave, one {form} burst)",
                     "kernel_ms": kern_s * 1e3,
                     "kernel_ms_by_form": {k: v * 1e3 for k, v in kern.items()},
                     "flops_per_update": flops_per_update,
                     "counters": read_counters("k_burst_hux", "upwind", "f64", "hux", kern_s,
                                               HU_SOURCES)},
    }
    if not args.no_cpu_baseline:
        # the oracle's burst (numpy) on the first patches of the grid
        from oracle import adi, pdo, upwind
        o = pdo.Oracle(prob)
        Uo = o.initial()
        npat = 64
        u0, e = o.lift(Uo)[:npat], o.edge(Uo)[:npat]
        s0 = time.perf_counter()
        upwind.burst(prob["grid"], o.coef[:, :npat], u0, e, 0.0, dt, n_t,
                     adi.time_factors(prob), points, r)
        el_c = time.perf_counter() - s0
        out["cpu_baseline"] = {"value": npat * info.m_xi * info.m_eta * n_t / el_c,
                               "unit": "patch-point updates/s", "cores": 1, "kind": "oracle",
                               "sample": f"one {form} burst ({n_t} steps) of {npat} "
                                         f"patches, {el_c:.1f} s"}
    print(json.dumps(out), flush=True)


def fd_cpu_baseline(prob, n, dt, steps):
    """The FP64 CPU oracle's lattice solver on the same lattice (OpenMP over rows): a few
    steps, the coefficient setup timed apart and excluded."""
    import numpy as np
    from oracle import pdo
    threads = max(1, min(16, os.cpu_count() or 1))
    o = pdo.Oracle(prob, threads=threads)
    U = np.zeros((n, n))
    s = time.perf_counter()
    o.full_domain(n, n, U, 0.0, dt, 0)
    t_setup = time.perf_counter() - s
    s = time.perf_counter()
    o.full_domain(n, n, U, 0.0, dt, steps)
    el = time.perf_counter() - s - t_setup
    interior = (n - 2) * (n - 2)
    return {"value": interior * steps / el, "unit": "lattice updates/s",
            "cores": o.L.pdo_get_threads(), "kind": "oracle",
            "sample": f"{steps} steps of the {n}x{n} lattice, {el:.1f} s (coefficient setup "
                      f"{t_setup:.1f} s excluded)"}


def bench_full_domain(args):
    """The full-domain explicit comparator (pd_fd_*): forward Euler with the bursts'
    differences on one lattice over the whole box, for the config-2 problem; and the time
    each method needs to reach the config-2 final time."""
    import torch

    from paper_2405_08764_amd import pd
    from paper_2405_08764_amd import workloads as W
    prob = W.config2()
    n = args.fd_n
    K = args.steps
    torch.cuda.set_device(0)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        g = pd.Grid(prob)
        f = pd.FullDomain(g, n, n, frac=0.5)
        info = f.query()
        dt = info.dt
        U = f.initial(0.0)
        f.solve(U, 0.0, args.warmup)
        f.sync()
        U = f.initial(0.0)
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        s = time.perf_counter()
        a.record(stream)
        f.solve(U, 0.0, K)
        b.record(stream)
        torch.cuda.synchronize()
        el = time.perf_counter() - s
        f.sync()
        kern_s = a.elapsed_time(b) / 1e3 / K  # step kernels (+ one table pass per 256)
        t_pd = None
        if not args.fd_no_pd:
            # patch dynamics on the same problem to the same final time, as the default
            # config-2 benchmark runs it
            gp = pd.Grid(prob)
            Up = gp.initial()
            gp.autotune(Up, reps=5)
            gp.solve(Up, n_steps=32)
            gp.sync()
            Up = gp.initial()
            torch.cuda.synchronize()
            s = time.perf_counter()
            gp.solve(Up, n_steps=prob["time"]["n_steps"])
            torch.cuda.synchronize()
            t_pd = time.perf_counter() - s
            gp.sync()
        if args.calibrate_copy:
            # the streaming kernel of known traffic the counter summary is scaled by
            m = args.calibrate_copy * (1 << 20) // 8
            src = torch.ones(m, dtype=torch.float64, device="cuda")
            dst = torch.empty_like(src)
            for _ in range(2):
                torch.mul(src, 1.0, out=dst)
            torch.cuda.synchronize()
            del src, dst
    ns = sum(1 for (tf, _, _) in prob["src"] if tf[0] != "const")
    has_k = any(tf[0] == "const" for (tf, _, _) in prob["src"])
    interior = (n - 2) * (n - 2)
    nb = 4 * n - 4
    planes = 5 + int(has_k) + ns
    bytes_per_node = 8 * planes + 16  # weight planes and the field read once, one write
    alg_bytes = interior * bytes_per_node + nb * 16
    achieved = alg_bytes / kern_s
    peak = 8.0e12
    T_end = prob["time"]["n_steps"] * prob["time"]["dt_macro"]
    fd_steps = math.ceil(T_end / dt)
    traffic = read_traffic("k_fd_step", "full-domain", "f64", "fd", FD_SOURCES)
    out = {
        "metric": "lattice-point updates/s of the full-domain explicit comparator",
        "value": interior * K / el,
        "unit": "lattice updates/s",
        "n_gpus": 1, "steps": K, "warmup": args.warmup, "ms_per_step": el / K * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic (seeded analytic coefficients, no dataset)",
        "config": {"workload": f"full-domain: config-2 problem (tanh-stretched square, "
                               f"beta 2.5, eps 1e-3, Fourier D and v, source (1 + sin 4 pi t) "
                               f"g) on a {n}x{n} lattice, forward Euler at half the "
                               f"explicit bound",
                   "n": n, "dt": dt, "dt_limit": info.dt_limit,
                   "spacing": info.spacing_x, "bytes_per_node_step": bytes_per_node},
        "roofline": {"bound": "hbm", "achieved": achieved / 1e9, "peak": peak / 1e9,
                     "unit": "GB/s", "frac": achieved / peak,
                     "traffic": traffic, "algorithmic_bytes": alg_bytes,
                     "kernel": "k_fd_step (one lattice step)", "kernel_ms": kern_s * 1e3,
                     "counters": read_counters("k_fd_step", "full-domain", "f64", "fd", kern_s,
                                               FD_SOURCES)},
        "vs_patch_dynamics": {
            "T": T_end, "fd_steps": fd_steps, "fd_time_s": fd_steps * el / K,
            "pd_macro_steps": prob["time"]["n_steps"], "pd_time_s": t_pd,
            "fd_over_pd_time": None if t_pd is None else fd_steps * el / K / t_pd,
            "pd_micro_spacing": prob["grid"]["h_xi"] / (prob["grid"]["m_xi"] - 1)},
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = fd_cpu_baseline(prob, n, dt, args.fd_cpu_steps)
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None,
                    help="timed macro steps (default 20 for the headline, config4 and "
                         "config5; 1000 for config1-3)")
    ap.add_argument("--warmup", type=int, default=None,
                    help="untimed macro steps run just before the timed ones (default 3 "
                         "for the batch workloads, 32 for config1-3, 4 otherwise)")
    ap.add_argument("--precision", default="f64", choices=["f64", "f32"])
    ap.add_argument("--workload", default="headline",
                    choices=["headline", "config1", "config2", "config3", "config4",
                             "config5", "full-domain", "refresh", "adi", "adi-upwind",
                             "upwind"])
    ap.add_argument("--batch-shapes", default=None, metavar="JSON",
                    help="config4/5 and headline: read the batch launch shapes from this "
                         "file if it exists (no autotuning), else autotune and write it")
    ap.add_argument("--horizon-steps", type=int, default=200,
                    help="headline/config5: closure error against plain over this many "
                         "steps on held-out members (0: skip)")
    ap.add_argument("--horizon-members", type=int, default=64,
                    help="headline/config5: members of that long-horizon comparison")
    ap.add_argument("--cpu-seconds-one", type=float, default=8.0,
                    help="headline: budget of the one-thread oracle leg")
    ap.add_argument("--adi-n", type=int, default=129,
                    help="adi: macro nodes per side")
    ap.add_argument("--upwind-points", type=int, default=3, choices=[2, 3, 4],
                    help="upwind, adi-upwind: the micro first difference (2-, 3- or "
                         "4-point)")
    ap.add_argument("--upwind-r", type=float, default=0.5,
                    help="upwind, adi-upwind: r of the 4-point difference")
    ap.add_argument("--refresh", type=int, default=5,
                    help="refresh: sub-bursts per macro step (edge data refreshed between)")
    ap.add_argument("--fd-n", type=int, default=4097,
                    help="full-domain: lattice nodes per side")
    ap.add_argument("--fd-cpu-steps", type=int, default=200,
                    help="full-domain: oracle steps of the CPU baseline")
    ap.add_argument("--fd-no-pd", action="store_true",
                    help="full-domain: skip the patch-dynamics run to the same final time")
    ap.add_argument("--train-instances", type=int, default=96,
                    help="config5: training instances (seeds disjoint from the batch)")
    ap.add_argument("--train-pairs", type=int, default=2_000_000,
                    help="config5: training pairs from plain steps")
    ap.add_argument("--epochs", type=int, default=25, help="config5: training epochs")
    ap.add_argument("--threshold-factor", type=float, default=10.0,
                    help="config5: fallback threshold in units of the training residual RMS")
    ap.add_argument("--instances", type=int, default=512,
                    help="config4: number of mixed instances in the batch")
    ap.add_argument("--kernel-reps", type=int, default=64)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep the heuristic launch shape instead of timing the candidates")
    ap.add_argument("--shape", default=None,
                    help="force the launch shape 'exchange,cols,rows,patches_per_block' "
                         "(exchange 1 = LDS, 2 = in-wave); implies --no-autotune")
    ap.add_argument("--no-resident", action="store_true",
                    help="config1-3 and refresh: one launch per macro step (or per sub-burst) "
                         "instead of the resident launches (PD_OPT_RESIDENT_SOLVE = 0)")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="also run a plain device copy of MIB MiB (twice), the reference "
                         "kernel for scaling HBM byte counters")
    ap.add_argument("--pmc-summary", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="write the HBM traffic summary of the burst kernel from two "
                         "rocprofv3 --pmc counter CSVs (no GPU needed) and exit")
    ap.add_argument("--counter-summary", nargs="+", metavar="CSV",
                    help="write the utilisation summary of one kernel (--counter-kernel) from "
                         "rocprofv3 --pmc counter CSVs of the COUNTER_PASSES sets (no GPU "
                         "needed) and exit")
    ap.add_argument("--stats-summary", nargs=2, metavar=("KERNEL_STATS_CSV", "OUT"),
                    help="write a rocprofv3 --stats kernel table as a text summary (with "
                         "--stats-title and --pmc-command) and exit")
    ap.add_argument("--stats-title", default="")
    ap.add_argument("--counter-kernel", default="",
                    help="kernel name as in profiles/ (k_burst_x, k_batch, k_closure_step, ...)")
    ap.add_argument("--counter-last", type=int, default=0,
                    help="summarise only the last N dispatches of the kernel in each CSV")
    ap.add_argument("--counter-match", default="",
                    help="kernel-name substring selecting the dispatches summarised (default: "
                         "the --counter-kernel name), e.g. one template instance")
    ap.add_argument("--pmc-shape", default="", help="launch shape the counters were taken at")
    ap.add_argument("--pmc-command", default="", help="command that produced the counters")
    args = ap.parse_args()
    if args.steps is None:
        args.steps = {"headline": 20, "config4": 20, "config5": 20, "full-domain": 400,
                      "refresh": 200, "adi": 200, "adi-upwind": 200,
                      "upwind": 200}.get(args.workload, 1000)
    if args.warmup is None:
        args.warmup = {"headline": 3, "config4": 3, "config5": 3, "config1": 32,
                       "config2": 32, "config3": 32}.get(args.workload, 4)
    if args.warmup < 0 or args.steps < 1:
        ap.error("--steps must be >= 1 and --warmup >= 0")
    if args.stats_summary:
        stats_summary(args.stats_summary[0], args.stats_summary[1], args.stats_title,
                      args.pmc_command, keep=args.counter_match)
        return
    if args.counter_summary:
        kern = args.counter_kernel
        files = {"k_batch": BATCH_SOURCES, "k_closure_step": CLOSURE_SOURCES,
                 "k_burst_hux": HU_SOURCES, "k_burst_adi_r": ADI_SOURCES,
                 "k_burst_adi_hu": ADU_SOURCES, "k_fd_step": FD_SOURCES,
                 "k_solve_x": SOLVE_SOURCES, "k_refresh_x": SOLVE_SOURCES}.get(kern)
        counter_summary(args.counter_summary, args.counter_match or
                        kern + ("<" if kern.startswith("k_burst") or kern == "k_batch" else ""),
                        args.counter_last, counter_file(kern, args.workload, args.precision),
                        args.pmc_command, args.workload, args.precision, args.pmc_shape, files)
        return
    if args.pmc_summary and args.counter_kernel:
        kern = args.counter_kernel
        files = {"k_batch": BATCH_SOURCES, "k_closure_step": CLOSURE_SOURCES,
                 "k_burst_hux": HU_SOURCES, "k_burst_adi_r": ADI_SOURCES,
                 "k_burst_adi_hu": ADU_SOURCES, "k_fd_step": FD_SOURCES,
                 "k_solve_x": SOLVE_SOURCES, "k_refresh_x": SOLVE_SOURCES}.get(kern)
        pmc_summary(args.pmc_summary[0], args.pmc_summary[1], args.counter_match or
                    kern + ("<" if kern.startswith("k_burst") or kern == "k_batch" else ""),
                    args.calibrate_copy or 256, traffic_file(kern, args.workload, args.precision),
                    args.pmc_command, args.workload, args.precision, args.pmc_shape, files)
        return
    if args.pmc_summary:
        if args.workload == "full-domain":
            pmc_summary(args.pmc_summary[0], args.pmc_summary[1], "k_fd_step",
                        args.calibrate_copy or 256,
                        traffic_file("k_fd_step", args.workload, "f64"), args.pmc_command,
                        args.workload, "f64", "fd", FD_SOURCES)
            return
        if args.workload == "upwind":
            pmc_summary(args.pmc_summary[0], args.pmc_summary[1], "k_burst_hux",
                        args.calibrate_copy or 256,
                        traffic_file("k_burst_hux", args.workload, "f64"), args.pmc_command,
                        args.workload, "f64", "hux", HU_SOURCES)
            return
        kernel = KERNEL_NAME[int(args.pmc_shape.split(",")[0])]
        pmc_summary(args.pmc_summary[0], args.pmc_summary[1], kernel + "<",
                    args.calibrate_copy or 256,
                    traffic_file(kernel, args.workload, args.precision), args.pmc_command,
                    args.workload, args.precision, args.pmc_shape)
        return
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py measures one GPU only (asked for {max(args.gpus, world)}); the "
              "multi-GPU sharding is a design note, not built.", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2405_08764_amd import pd
    from paper_2405_08764_amd import workloads as W

    if args.workload == "headline":
        return bench_headline(args)
    if args.workload == "config4":
        return bench_batch(args)
    if args.workload == "config5":
        return bench_closure(args)
    if args.workload == "full-domain":
        return bench_full_domain(args)
    if args.workload == "refresh":
        return bench_refresh(args)
    if args.workload in ("adi", "adi-upwind"):
        return bench_adi(args)
    if args.workload == "upwind":
        return bench_upwind(args)
    prob, desc = workload(args.workload)
    t = prob["time"]
    torch.cuda.set_device(0)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        g = pd.Grid(prob, precision=args.precision)
        U = g.initial()
        tuned_ms = None
        if args.shape:
            fix_shape(pd, g, args.shape)
        elif not args.no_autotune:
            tuned_ms = g.autotune(U, reps=5)
        if args.no_resident:
            g.set_option(pd.OPT_RESIDENT_SOLVE, 0)
        # set-up: one graph replay (16 steps) instantiates the solve graph on this field
        g.solve(U, n_steps=16)
        g.sync()
        g.initial(U=U)
        # exactly `warmup` untimed steps, then the timed steps continue from there
        g.solve(U, n_steps=args.warmup)
        g.sync()
        per_step = W.updates_per_step(prob)
        torch.cuda.synchronize()
        s = time.perf_counter()
        g.solve(U, n_steps=args.steps, t0=t["t0"] + args.warmup * t["dt_macro"])
        torch.cuda.synchronize()
        el = time.perf_counter() - s
        g.sync()
        info = g.query()
        resident = bool(info.resident_solve)
        if resident:
            # Dominant kernel: the resident solve, one launch per 16-step replay (with its
            # table fill), timed with HIP events on the stream it runs on, per macro step.
            kern_s = time_launches(stream, lambda: g.solve(U, n_steps=RESIDENT_STEPS),
                                   args.kernel_reps) / RESIDENT_STEPS
        else:
            # Dominant kernel: the fused burst (pd_patch_step launches exactly that kernel),
            # timed with HIP events on the stream it runs on.
            V = torch.empty_like(U)
            pair = [U, V]

            def step():
                g.patch_step(pair[0], t["t0"], out=pair[1])
                pair.reverse()
            kern_s = time_launches(stream, step, args.kernel_reps)
        g.sync()
        if args.calibrate_copy:
            # A plain streaming kernel of known traffic: read MIB MiB, write MIB MiB
            # (torch's vectorized elementwise multiply by one).
            n = args.calibrate_copy * (1 << 20) // 8
            src = torch.ones(n, dtype=torch.float64, device="cuda")
            dst = torch.empty_like(src)
            for _ in range(2):
                torch.mul(src, 1.0, out=dst)
            torch.cuda.synchronize()
            del src, dst

    ns = sum(1 for (tf, _, _) in prob["src"] if tf[0] != "const")
    # Algorithmic work of one nano update of the scheme with pre-scaled coefficients: two
    # neighbour sums, two -2u FMAs, two diffusion FMAs, two upwind differences, two
    # convection FMAs, the reaction FMA, the source add and the +u add (7 FMA + 6 ADD).
    flops_per_update = 20
    # What the kernel issues instead: the 5-point stencil with folded weights, the
    # constant forcing and one FMA per time-dependent source term.
    issued_flops_per_update = 2 * (5 + ns)
    achieved = flops_per_update * per_step / kern_s
    # Algorithmic HBM bytes of one fused launch: every coefficient plane once (alpha,
    # gamma, nu, omega, phi and the source terms' spatial parts), the macro field once,
    # one new value per patch node.
    n_src = len(prob["src"])
    alg_bytes = (5 + n_src) * info.n_points * 8 + info.n_xi * info.n_eta * 8 + info.n_patches * 8
    peak = PEAK[args.precision]
    value = per_step * args.steps / el
    shape = f"{info.exchange},{info.cols_per_lane},{info.rows_per_lane},{info.patches_per_block}"
    kname = "k_solve_x" if resident else KERNEL_NAME[info.exchange]
    kfiles = SOLVE_SOURCES if resident else None
    # per launch: the resident solve covers RESIDENT_STEPS macro steps; its coefficient
    # planes are read once per launch, dt phi (and constant sources) once per step
    per_launch = RESIDENT_STEPS if resident else 1
    if resident:
        n_const = sum(1 for (tf, _, _) in prob["src"] if tf[0] == "const")
        alg_bytes = ((5 + n_src) * info.n_points * 8 / per_launch
                     + (1 + (1 if n_const else 0)) * info.n_points * 8
                     + info.n_xi * info.n_eta * 8 + info.n_patches * 8)
    traffic = read_traffic(kname, args.workload, args.precision, shape, kfiles)
    if traffic is not None:
        traffic /= per_launch  # per macro step, like kernel_ms
    out = {
        "metric": "patch-point updates/s (and macro steps/s) of the plain GPU scheme",
        "value": value,
        "unit": "patch-point updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "setup_steps": 16,
        "ms_per_step": el / args.steps * 1e3,
        "macro_steps_per_s": args.steps / el,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.precision,
        "data": "synthetic (seeded analytic coefficients, no dataset)",
        "config": {"workload": f"{args.workload}: {desc}", "patches": info.n_patches,
                   "micro_points_per_patch": info.m_xi * info.m_eta, "n_t": t["n_t"],
                   "dt_macro": t["dt_macro"], "dt_micro": t["dt_micro"],
                   "updates_per_step": per_step,
                   "launch": {"rows_per_lane": info.rows_per_lane,
                              "cols_per_lane": info.cols_per_lane,
                              "patches_per_block": info.patches_per_block,
                              "block_threads": info.block_threads,
                              "exchange": {1: "lds", 2: "in-wave", 3: "hybrid"}[info.exchange],
                              "autotuned": bool(info.tuned), "tuned_ms": tuned_ms}},
        "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": peak / 1e12,
                     "unit": "TFLOP/s", "frac": achieved / peak, "traffic": traffic,
                     "algorithmic_bytes": alg_bytes,
                     "kernel": ("k_solve_x (resident fused solve, 16 macro steps per launch;"
                                " per macro step)") if resident else
                               KERNEL_NAME[info.exchange] + " (fused macro step)",
                     "kernel_ms": kern_s * 1e3,
                     "flops_per_update": flops_per_update,
                     "issued_flops_per_update": issued_flops_per_update,
                     "issued_frac": issued_flops_per_update * per_step / kern_s / peak,
                     "counters": read_counters(kname, args.workload, args.precision, shape,
                                               kern_s * per_launch, kfiles)},
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(prob, args.cpu_seconds, steps_cap=1000)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
