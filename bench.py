"""Benchmark: batched RKC chemistry integration on one MI355X.

Workload (default): the 53-species / 634-reaction synthetic mechanism with
131072 cells, T ~ U(800, 2200) K, P = 1 atm, Y with five major species, one
global step dt = 1e-6 s, rtol 1e-6, atol 1e-10, integrated with RKC in FP64.
As in the paper's protocol (Sec. 3), K consecutive global steps are timed, each
restarting the integrator from the state the previous one produced; the state
is resident in HBM before the timed region starts.

Output: one JSON line with the metric (cell-ODEs integrated per second over
dt), the roofline of the integrator kernel (FP64 vector ALU bound) and the
serial FP64 oracle timed on a bounded sample of the same workload.

  python bench.py [--steps K] [--warmup W] [--config c3] [--no-cpu]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK_FP64_TFLOPS = 78.6        # MI355X FP64 vector: 256 CU x 128 flop/clk x 2.4 GHz
EXP_FLOPS = 27                 # FP64 arithmetic of one device exp: 13 FMA + 1 MUL
METRIC = "cell-ODEs integrated per sec over dt (53sp/634rx, FP64); p99 batch latency"


def rhs_flops(mech):
    """Algorithmic FP64 flops of one source-term evaluation.

    Per reaction: exponent argument 4, exp EXP_FLOPS, rate of progress m_j
    multiplies; per forward/reverse pair one subtraction; per nonzero
    (species, pair) coefficient of the net production sum 2; per species 28
    (mixture sums, concentration, NASA-7 Horner for Cp and H, species rate,
    energy sums); per evaluation 10 (density, 1/T, dT/dt)."""
    nS, nR = mech["n_species"], mech["n_reactions"]
    m = (np.asarray(mech["reac"]) >= 0).sum(1)
    f = int(nR * (4 + EXP_FLOPS) + m.sum())
    pairs = nR // 2
    f += pairs
    nnz = 0
    for p in range(pairs):
        d = {}
        for s in mech["reac"][2 * p]:
            if s >= 0:
                d[s] = d.get(s, 0) - 1
        for s in mech["prod"][2 * p]:
            if s >= 0:
                d[s] = d.get(s, 0) + 1
        nnz += sum(1 for v in d.values() if v != 0)
    f += 2 * nnz + 28 * nS + 10
    return f


def stage_flops(mech):
    """Flops of one RKC stage update (E:rkcj) per RHS evaluation: 1 mul + 4 FMA
    per state component."""
    return 9 * (mech["n_species"] + 1)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", default="c3")
    ap.add_argument("--lanes", type=int, default=0)
    ap.add_argument("--schedule", type=int, default=0)
    ap.add_argument("--params", type=int, default=0, help="0 auto, 1 registers, 2 LDS")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py: this build runs on one GPU only; the cells of a global step "
              "are independent and would shard by contiguous cell ranges (see DESIGN.md)",
              file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_1309_2710_amd import rkc, synth

    cfg = args.config
    c = synth.CONFIGS[cfg]
    mech = synth.config_mechanism(cfg)
    st = synth.config_states(cfg)
    n = st["T"].shape[0]
    dev = torch.device("cuda:0")
    gm = rkc.Mechanism(mech)
    T0 = torch.from_numpy(st["T"]).to(dev)
    P = torch.from_numpy(st["P"]).to(dev)
    Y0 = torch.from_numpy(st["Y"]).to(dev)
    T = T0.clone()
    Y = Y0.clone()
    kw = dict(lanes_per_cell=args.lanes, schedule=args.schedule, status=False,
              param_placement=args.params)

    # Warm-up and work census: the K timed steps are replayed once untimed with
    # statistics (results are bitwise deterministic, so the timed run performs
    # exactly this work).
    for _ in range(args.warmup):
        Tw, Yw = T0.clone(), Y0.clone()
        rkc.integrate(gm, Tw, P, Yw, c["dt"], c["rtol"], c["atol"], **kw)
    T.copy_(T0)
    Y.copy_(Y0)
    census = []
    for _ in range(args.steps):
        o = rkc.integrate(gm, T, P, Y, c["dt"], c["rtol"], c["atol"], stats=True, **kw)
        census.append(o["stats"])
    torch.cuda.synchronize()
    T.copy_(T0)
    Y.copy_(Y0)
    torch.cuda.synchronize()

    # Timed region: K consecutive global steps, device-resident state.
    stream = torch.cuda.current_stream(dev)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev[0].record(stream)
    for k in range(args.steps):
        rkc.integrate(gm, T, P, Y, c["dt"], c["rtol"], c["atol"], **kw)
        ev[k + 1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    step_ms = [ev[k].elapsed_time(ev[k + 1]) for k in range(args.steps)]
    ms_per_step = wall * 1e3 / args.steps

    f_rhs = rhs_flops(mech)
    f_stage = stage_flops(mech)
    tot_rhs = sum(s["n_rhs"] for s in census)
    flops_per_launch = (tot_rhs * (f_rhs + f_stage)) / args.steps
    launch_s = np.mean(step_ms) / 1e3
    achieved = flops_per_launch / launch_s / 1e12

    out = {
        "metric": METRIC,
        "value": n * args.steps / wall,
        "unit": "cell-ODEs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "%s: RKC, %s" % (cfg, c["label"]), "n_cells": n,
                   "n_species": mech["n_species"], "n_reactions": mech["n_reactions"],
                   "dt": c["dt"], "rtol": c["rtol"], "atol": c["atol"],
                   "lanes_per_cell": census[0]["lanes_per_cell"],
                   "schedule": ["auto", "plain", "persistent"][census[0]["schedule"]],
                   "parallelism": "single GPU"},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_FP64_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved / PEAK_FP64_TFLOPS, "traffic": None},
        "work": {"rhs_evals_per_step": tot_rhs / args.steps, "flops_per_rhs": f_rhs,
                 "flops_per_stage_update": f_stage,
                 "mean_rhs_per_cell": tot_rhs / args.steps / n,
                 "kernel_ms_per_step": step_ms,
                 "steps_per_cell": sum(s["n_steps"] for s in census) / args.steps / n,
                 "s_max_used": max(s["s_max_used"] for s in census)},
    }
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(mech, c, st, args.steps, args.cpu_seconds)
    print(json.dumps(out), flush=True)


def cpu_baseline(mech, c, st, steps, budget_s):
    """The serial FP64 oracle (unchanged; cells split over host threads) on a
    strided sample of the same workload, K consecutive global steps."""
    from oracle import oracle as O

    M = O.Model(mech)
    threads = min(os.cpu_count() or 1, 16)
    n = st["T"].shape[0]

    def run(idx):
        T, Y = st["T"][idx].copy(), st["Y"][idx].copy()
        P = st["P"][idx]
        t = time.perf_counter()
        for _ in range(steps):
            T, Y, _ = M.integrate(T, P, Y, c["dt"], c["rtol"], c["atol"], threads=threads)
        return time.perf_counter() - t

    probe = np.arange(0, n, max(1, n // (4 * threads)))[:4 * threads]
    t_probe = run(probe)
    per_cell = t_probe / len(probe)
    m = int(min(n, max(len(probe), budget_s / max(per_cell, 1e-9))))
    m = max(threads, (m // threads) * threads)
    idx = np.arange(0, n, max(1, n // m))[:m]
    t = run(idx)
    return {"value": len(idx) * steps / t, "unit": "cell-ODEs/s", "cores": threads,
            "kind": "oracle",
            "sample": "%d of %d cells (stride %d), %d consecutive global steps, %.1f s"
                      % (len(idx), n, max(1, n // m), steps, t)}


if __name__ == "__main__":
    main()
