#!/usr/bin/env python3
"""Throughput of the fused patch-dynamics macro step (Sec. 3.3 steps (i)-(vi)) on one GPU.

A step is one macro step of the whole hot path over the full workload: edge data, lifting,
the forward-Euler burst in every patch, restriction and the projective update, plus the
Dirichlet boundary, replayed from a HIP graph.  Default workload: the stretched unit square
(tanh stretching, 65x65 macro nodes, 17x17 micro points per patch, random Fourier-mode
coefficients) in FP64.  Prints one JSON line.
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


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=32)
    ap.add_argument("--precision", default="f64", choices=["f64", "f32"])
    ap.add_argument("--workload", default="config2", choices=["config1", "config2", "config3"])
    ap.add_argument("--kernel-reps", type=int, default=64)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py measures one GPU only (asked for {max(args.gpus, world)}); the "
              "multi-GPU sharding is a design note, not built.", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2405_08764_amd import pd
    from paper_2405_08764_amd import workloads as W

    prob, desc = workload(args.workload)
    t = prob["time"]
    torch.cuda.set_device(0)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        g = pd.Grid(prob, precision=args.precision)
        U = g.initial()
        g.solve(U, n_steps=max(args.warmup, 16))
        g.sync()
        per_step = W.updates_per_step(prob)
        U = g.initial()
        torch.cuda.synchronize()
        s = time.perf_counter()
        g.solve(U, n_steps=args.steps)
        torch.cuda.synchronize()
        el = time.perf_counter() - s
        g.sync()
        # Dominant kernel: the fused burst (pd_patch_step launches exactly that kernel),
        # timed with HIP events on the stream it runs on.
        V = torch.empty_like(U)
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
               for _ in range(args.kernel_reps)]
        for k, (a, b) in enumerate(evs):
            a.record(stream)
            g.patch_step(U if k % 2 == 0 else V, t["t0"], out=V if k % 2 == 0 else U)
            b.record(stream)
        torch.cuda.synchronize()
        kern_s = sum(a.elapsed_time(b) for a, b in evs) / len(evs) / 1e3
        info = g.query()

    ns = sum(1 for (tf, _, _) in prob["src"] if tf[0] != "const")
    flops_per_update = 2 * (5 + ns)  # 5 stencil FMAs + one per time-dependent source term
    achieved = flops_per_update * per_step / kern_s
    peak = PEAK[args.precision]
    value = per_step * args.steps / el
    out = {
        "metric": "patch-point updates/s (and macro steps/s) of the plain GPU scheme",
        "value": value,
        "unit": "patch-point updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": max(args.warmup, 16),
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
                              "patches_per_block": info.patches_per_block,
                              "block_threads": info.block_threads}},
        "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": peak / 1e12,
                     "unit": "TFLOP/s", "frac": achieved / peak, "traffic": None,
                     "kernel": "k_burst (fused macro step)",
                     "kernel_ms": kern_s * 1e3,
                     "flops_per_update": flops_per_update},
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(prob, args.cpu_seconds, steps_cap=50)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
