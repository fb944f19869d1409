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
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK_FP64_TFLOPS = 78.6        # MI355X FP64 vector: 256 CU x 128 flop/clk x 2.4 GHz
EXP_FLOPS = 25                 # FP64 arithmetic of one device exponential (2^y): 3 ADD for
                               # y = n + f, 11 FMA for the polynomial
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
    return f + pdep_flops(mech)


LOG_FLOPS = EXP_FLOPS           # a logarithm counted like an exponential


def pdep_flops(mech):
    """Algorithmic flops of the pressure-dependent rates per evaluation
    (Chemkin forms, Sec. 2.2), per forward/reverse pair by kind, 0 for plain
    mechanisms.  Third-body concentration of each distinct efficiency set: 2
    per species.  Third body: [M] times both rate constants, 2.  Lindemann:
    both low-pressure constants (argument 4 + exp each), and per direction
    k0 [M], Pr = k0 [M] / kinf, 1 + Pr, Pr / (1 + Pr) and the product with kinf,
    5.  Troe adds the centre value (three exponentials with their arguments
    and the sum, 3 exp + 7), its log10 (log + 1), c and n (4), and per
    direction log10 Pr (log + 1), x, f = x / (n - 0.14 x), 1 + f^2, the
    quotient, the scaling to a base-2 exponent (8) and exp (exp + 1 for the
    product with the Lindemann rate)."""
    if mech.get("pdep") is None:
        return 0
    kind = np.asarray(mech["pdep"])[0::2]
    f = 0
    lind = 2 * (4 + EXP_FLOPS) + 2 * 5
    troe = lind + (3 * EXP_FLOPS + 7) + (LOG_FLOPS + 1) + 4 + 2 * (LOG_FLOPS + 1 + 8 + EXP_FLOPS + 1)
    f += 2 * int((kind == 1).sum()) + lind * int((kind == 2).sum()) + troe * int((kind == 3).sum())
    if mech.get("eff") is not None:
        eff = np.asarray(mech["eff"])[0::2][kind > 0]
        n_sets = len({tuple(r) for r in eff})
        f += 2 * mech["n_species"] * n_sets
    return f


def kernel_source_hash():
    """sha256 over the HIP sources of the library (host and device code) and
    the compiler flags and target it is built with."""
    from paper_1309_2710_amd import build as lib_build

    d = os.path.join(ROOT, "paper_1309_2710_amd", "csrc")
    h = hashlib.sha256()
    for f in sorted(os.listdir(d)):
        if f.endswith((".h", ".hip")):
            h.update(f.encode())
            h.update(open(os.path.join(d, f), "rb").read())
    # include directories are absolute paths of this checkout: left out
    flags = [f for f in lib_build.CFLAGS if not f.startswith("-I")]
    h.update(" ".join(flags + [lib_build.ARCH]).encode())
    return h.hexdigest()


def measured_traffic(workload):
    """HBM bytes per launch of the integrator from the committed counter
    summary (FETCH_SIZE and WRITE_SIZE passes, each scaled by the same counter
    on a copy kernel of known size), or None when no summary matches the
    current sources and workload."""
    path = os.path.join(ROOT, "profiles", "rkc_kernel_%s_traffic.txt" % workload)
    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip()
    if kv.get("source_sha256") != kernel_source_hash():
        return None
    try:
        return float(kv["bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def stage_flops(mech):
    """Flops of the state update per RHS evaluation, 9 per state component.
    RKC (E:rkcj): 1 mul + 4 FMA per stage.  RKCK (Table 1): per step and
    component, 15 FMAs for the inputs of stages 2-6, 4 for the fifth-order
    solution and 5 for the embedded error, about 53 flops with the error
    scale, over 6 evaluations: also about 9."""
    return 9 * (mech["n_species"] + 1)


def workload_tag(mech, n):
    return "%dsp%drx_%dcells" % (mech["n_species"], mech["n_reactions"], n)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", default="c3")
    ap.add_argument("--cells", type=int, default=None,
                    help="cells of the workload (default: the configuration's)")
    ap.add_argument("--method", choices=["rkc", "rkck"], default="rkc",
                    help="integrator: RKC (Sec. 2.4, default) or RKCK (Sec. 2.3)")
    ap.add_argument("--dt", type=float, default=None,
                    help="global step in s (default: the configuration's)")
    ap.add_argument("--rtol", type=float, default=None,
                    help="relative tolerance, epsilon for RKCK (default: the configuration's)")
    ap.add_argument("--lanes", type=int, default=0)
    ap.add_argument("--schedule", type=int, default=0)
    ap.add_argument("--params", type=int, default=0, help="0 auto, 1 registers, 2 LDS, 3 global memory")
    ap.add_argument("--layout", type=int, default=None,
                    help="memory order of Y: 0 cell-major Y[cell][species], 1 species-major "
                         "(cell-fastest) Y[species][cell]; default: species-major for one lane "
                         "per cell, else cell-major")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--autotune", action="store_true",
                    help="choose schedule and workgroup size with rkc_autotune on a strided "
                         "sample of 16384 cells before the census (results do not change)")
    ap.add_argument("--graph", action="store_true",
                    help="time replays of a recorded global step (rkc_graph_create) instead of "
                         "rkc_integrate calls")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--serve", action="store_true",
                    help="replay the served mixed-request trace (13/53 species, Poisson "
                         "arrivals) through the integration server and, as the baseline, "
                         "through sequential rkc_integrate calls; report latency")
    ap.add_argument("--study", choices=["divergence", "crossover"], default=None,
                    help="divergence study: states sampled along ignition trajectories, "
                         "timed in trajectory order (similar neighbours) and shuffled, with "
                         "the plain and the persistent schedule")
    ap.add_argument("--serve-requests", type=int, default=2000)
    ap.add_argument("--serve-rate", type=float, default=200.0)
    ap.add_argument("--serve-streams", type=int, default=4)
    ap.add_argument("--served-requests", type=int, default=120,
                    help="requests of the short served trace in the default line (0: none)")
    ap.add_argument("--served-util", type=float, default=0.7,
                    help="offered utilisation of that trace: arrival rate over measured capacity")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="run one device copy kernel of this many MiB (read + write) after the "
                         "timed region: the known-size reference for HBM byte counters")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py: measures one GPU only (--gpus 1); the cells of a global step "
              "are independent and would shard by contiguous cell ranges",
              file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_1309_2710_amd import build as lib_build
    from paper_1309_2710_amd import rkc, synth

    lib_build.ensure_built()   # load what is built; build only if nothing is
    if args.serve:
        serve(args)
        return
    if args.study == "divergence":
        study_divergence(args)
        return
    if args.study == "crossover":
        study_crossover(args)
        return

    cfg = args.config
    c = dict(synth.CONFIGS[cfg])
    if args.dt is not None:
        c["dt"] = args.dt
    if args.rtol is not None:
        c["rtol"] = args.rtol
    method = rkc.RKCK if args.method == "rkck" else rkc.RKC
    default_run = (args.method == "rkc" and args.dt is None and args.rtol is None and
                   args.cells is None)
    mech = synth.config_mechanism(cfg)
    st = synth.config_states(cfg, args.cells)
    n = st["T"].shape[0]
    dev = torch.device("cuda:0")
    gm = rkc.Mechanism(mech)
    layout = args.layout if args.layout is not None else (1 if args.lanes == 1 else 0)
    T0 = torch.from_numpy(st["T"]).to(dev)
    P = torch.from_numpy(st["P"]).to(dev)
    Y0 = torch.from_numpy(st["Y"] if layout == 0 else np.ascontiguousarray(st["Y"].T)).to(dev)
    T = T0.clone()
    Y = Y0.clone()
    kw = dict(lanes_per_cell=args.lanes, schedule=args.schedule, status=False,
              param_placement=args.params, layout=layout, method=method)
    tuned = None
    if args.autotune:
        idx = torch.arange(0, n, max(1, n // 16384), device=dev)[:16384]
        Ys = Y0[idx] if layout == 0 else Y0[:, idx].t()
        t_tune = time.perf_counter()
        tuned, tuned_ms = rkc.autotune(gm, T0[idx].contiguous(), P[idx].contiguous(),
                                       Ys.contiguous(), c["dt"], c["rtol"], c["atol"],
                                       method=method, lanes_per_cell=args.lanes,
                                       param_placement=args.params)
        tuned["tuning_s"] = time.perf_counter() - t_tune
        tuned["sample_cells"] = int(idx.shape[0])
        if tuned["lanes_per_cell"] != kw["lanes_per_cell"] and layout == 1 and \
                tuned["lanes_per_cell"] != 1:
            layout = 0   # lane groups read cell-major rows
            Y0 = torch.from_numpy(st["Y"]).to(dev)
            Y = Y0.clone()
            kw["layout"] = 0
        kw.update(schedule=tuned["schedule"], block_groups=tuned["block_groups"],
                  lanes_per_cell=tuned["lanes_per_cell"], param_placement=tuned["param_placement"])

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

    graph = None
    if args.graph:
        graph = rkc.Graph(gm, T, P, Y, c["dt"], c["rtol"], c["atol"], method=method,
                          lanes_per_cell=kw["lanes_per_cell"], schedule=kw["schedule"],
                          block_groups=kw.get("block_groups", 0),
                          param_placement=kw["param_placement"], layout=layout)

    # Timed region: K consecutive global steps, device-resident state.
    stream = torch.cuda.current_stream(dev)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev[0].record(stream)
    for k in range(args.steps):
        if graph is not None:
            graph.launch(stream)
        else:
            rkc.integrate(gm, T, P, Y, c["dt"], c["rtol"], c["atol"], **kw)
        ev[k + 1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    step_ms = [ev[k].elapsed_time(ev[k + 1]) for k in range(args.steps)]
    ms_per_step = wall * 1e3 / args.steps

    # One more global step from the final state with host arrays: the rate
    # including the PCIe copies (reported beside `value`, never as it).
    Th, Yh = T.cpu().numpy().copy(), Y.cpu().numpy().copy()
    Ph = P.cpu().numpy()
    Td, Yd = T.clone(), Y.clone()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    rkc.integrate(gm, Td, P, Yd, c["dt"], c["rtol"], c["atol"], **kw)
    e1.record(stream)
    torch.cuda.synchronize()
    dev_ms = e0.elapsed_time(e1)
    a = time.perf_counter()
    rkc.integrate(gm, Th, Ph, Yh, c["dt"], c["rtol"], c["atol"], **kw)
    host_ms = (time.perf_counter() - a) * 1e3
    pcie = {"step_ms_host_arrays": host_ms, "step_ms_device_arrays": dev_ms,
            "cells_per_s_host_arrays": n / host_ms * 1e3,
            "note": "one global step after the timed ones; host arrays add the H2D and D2H "
                    "copies of the state"}
    del Td, Yd

    if args.copy_mib > 0:
        src = torch.ones(args.copy_mib * (1 << 20) // 8, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        torch.neg(src, out=dst)
        torch.cuda.synchronize()
        del src, dst

    f_rhs = rhs_flops(mech)
    f_stage = stage_flops(mech)
    tot_rhs = sum(s["n_rhs"] for s in census)
    flops_per_launch = (tot_rhs * (f_rhs + f_stage)) / args.steps
    launch_s = np.mean(step_ms) / 1e3
    achieved = flops_per_launch / launch_s / 1e12

    out = {
        "metric": METRIC if args.config == "c3" else METRIC.replace(
            "53sp/634rx", "%dsp/%drx" % (mech["n_species"], mech["n_reactions"])),
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
        "config": {"workload": "%s, %s" % (args.method.upper(), c["label"] if
                                           default_run or (args.dt is None and args.cells is None)
                                           else "%dsp/%drx, %d cells, dt %g" % (
                                               mech["n_species"], mech["n_reactions"], n,
                                               c["dt"])),
                   "n_cells": n,
                   "n_species": mech["n_species"], "n_reactions": mech["n_reactions"],
                   "dt": c["dt"], "rtol": c["rtol"], "atol": c["atol"],
                   "lanes_per_cell": census[0]["lanes_per_cell"],
                   "layout": ["cell-major", "species-major"][layout],
                   "schedule": ["auto", "plain", "persistent"][census[0]["schedule"]],
                   "launch": "hip graph replay" if graph is not None else "rkc_integrate",
                   "autotuned": tuned,
                   "parallelism": "single GPU"},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_FP64_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved / PEAK_FP64_TFLOPS,
                     # the committed traffic summaries cover the default RKC runs
                     "traffic": measured_traffic(workload_tag(mech, n)) if default_run
                     else None},
        "pcie_inclusive": pcie,
        "fp64_probe": fp64_probe(),
        "work": {"rhs_evals_per_step": tot_rhs / args.steps, "flops_per_rhs": f_rhs,
                 "flops_per_stage_update": f_stage,
                 "mean_rhs_per_cell": tot_rhs / args.steps / n,
                 "kernel_ms_per_step": step_ms,
                 # per-launch batch latency of the timed global steps
                 "step_ms_p50": float(np.percentile(step_ms, 50)),
                 "step_ms_p99": float(np.percentile(step_ms, 99)),
                 "steps_per_cell": sum(s["n_steps"] for s in census) / args.steps / n,
                 "rhs_utilisation": tot_rhs / max(1, sum(s["n_rhs_slots"] for s in census)),
                 "s_max_used": max(s["s_max_used"] for s in census),
                 # cells that ended with a failure status (MAXSTEPS, UNDERFLOW,
                 # NONFINITE) over the timed steps; 0 for every default run
                 "failed_cells": int(sum(s["n_failed"] for s in census))},
    }
    if args.served_requests > 0 and args.config == "c3" and not args.graph and default_run:
        del T, Y, T0, Y0, P
        out["served"] = served_block(args.served_requests, args.served_util)
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(mech, c, st, args.steps, args.cpu_seconds,
                                           method=args.method)
    print(json.dumps(out), flush=True)


def fp64_probe():
    """Measured FP64 vector FMA throughput of the GPU (the probe library:
    independent FMA chains, 4 waves per SIMD), beside the published peak the
    roofline uses."""
    import ctypes as ct

    from paper_1309_2710_amd import build as lib_build

    L = ct.CDLL(lib_build.PROBE_LIB)
    L.rkc_probe_fp64_fma.argtypes = [ct.c_int, ct.c_int, ct.POINTER(ct.c_double),
                                     ct.POINTER(ct.c_float)]
    f, ms = ct.c_double(), ct.c_float()
    rc = L.rkc_probe_fp64_fma(4 * 256, 100000, ct.byref(f), ct.byref(ms))
    if rc != 0:
        return {"error": rc}
    return {"tflops": f.value / 1e12, "of_published_peak": f.value / 1e12 / PEAK_FP64_TFLOPS,
            "ms": ms.value, "kernel": "1024 workgroups x 256 lanes, 16 independent FMA chains "
                                      "per lane, 100000 steps"}


def trajectory_states(rkc, gm, c, synth, mech, n_traj, n_samp, seed):
    """States sampled along constant-pressure ignition trajectories (the
    paper's way of making initial conditions, Sec. 3): n_traj seeded starting
    compositions at 1600 K and 1 atm, each integrated over n_samp consecutive
    global steps of c["dt"] with rkc_integrate; sample k of trajectory j is the
    state after k steps.  Returned in trajectory order, so neighbouring cells
    hold similar conditions."""
    import torch
    st = synth.make_states(mech, n_traj, seed, T_dist=("uniform", 1600.0, 1600.0),
                           P_dist=("const", synth.ATM), Y_dist=c["Y"])
    dev = torch.device("cuda:0")
    T = torch.from_numpy(st["T"]).to(dev)
    P = torch.from_numpy(st["P"]).to(dev)
    Y = torch.from_numpy(st["Y"]).to(dev)
    Ts = torch.empty((n_traj, n_samp), dtype=torch.float64, device=dev)
    Ys = torch.empty((n_traj, n_samp, mech["n_species"]), dtype=torch.float64, device=dev)
    for k in range(n_samp):
        Ts[:, k] = T
        Ys[:, k] = Y
        rkc.integrate(gm, T, P, Y, c["dt"], c["rtol"], c["atol"], status=False)
    n = n_traj * n_samp
    return (Ts.reshape(n).contiguous(), torch.full((n,), synth.ATM, dtype=torch.float64,
                                                   device=dev),
            Ys.reshape(n, mech["n_species"]).contiguous())


def study_divergence(args):
    """Throughput and divergence D (Sec. 3.1) for ignition-sampled states in
    trajectory order and shuffled: the 13-species set with 16-lane groups
    (plain and persistent schedules) and with one lane per cell (persistent,
    species-major state), the 53-species set with 64-lane groups (plain and
    persistent).  D is reported for the paper's 32-thread warps and for the
    cells a wavefront holds at once (64 / lanes per cell), with histograms of
    D over ten equal bins of [0, 1] as in the paper's divergence figures."""
    import torch

    from paper_1309_2710_amd import rkc, synth

    dev = torch.device("cuda:0")
    rows = []
    bins = np.linspace(0.0, 1.0, 11)
    for cfg, n_traj, forms in (("c2", 1024, [(16, rkc.SCHED_PLAIN), (16, rkc.SCHED_PERSISTENT),
                                             (1, rkc.SCHED_PERSISTENT)]),
                               ("c3", 512, [(64, rkc.SCHED_PLAIN), (64, rkc.SCHED_PERSISTENT)])):
        c = synth.CONFIGS[cfg]
        mech = synth.config_mechanism(cfg)
        gm = rkc.Mechanism(mech)
        T0, P, Y0 = trajectory_states(rkc, gm, c, synth, mech, n_traj, 128, 4000)
        n = T0.shape[0]
        perm = torch.from_numpy(np.random.default_rng(4001).permutation(n)).to(dev)
        for order in ("trajectory", "shuffled"):
            Ti = T0 if order == "trajectory" else T0[perm].contiguous()
            Yi = Y0 if order == "trajectory" else Y0[perm].contiguous()
            for G, sched in forms:
                layout = 1 if G == 1 else 0
                Yl = Yi if layout == 0 else Yi.t().contiguous()
                T, Y = Ti.clone(), Yl.clone()
                o = rkc.integrate(gm, T, P, Y, c["dt"], c["rtol"], c["atol"], schedule=sched,
                                  lanes_per_cell=G, layout=layout, counters=True, stats=True)
                cn = o["counters"]
                D32 = rkc.divergence(cn, 32).cpu().numpy()
                Dw = rkc.divergence(cn, 64 // G).cpu().numpy()
                T, Y = Ti.clone(), Yl.clone()
                torch.cuda.synchronize()
                t = time.perf_counter()
                for _ in range(args.steps):
                    rkc.integrate(gm, T, P, Y, c["dt"], c["rtol"], c["atol"], schedule=sched,
                                  lanes_per_cell=G, layout=layout, status=False)
                torch.cuda.synchronize()
                wall = time.perf_counter() - t
                rows.append({"set": "%dsp/%drx" % (mech["n_species"], mech["n_reactions"]),
                             "cells": n, "order": order,
                             "schedule": "plain" if sched == rkc.SCHED_PLAIN else "persistent",
                             "lanes_per_cell": G, "cell_odes_per_s": n * args.steps / wall,
                             "mean_D32": float(D32.mean()), "mean_D_wave": float(Dw.mean()),
                             "hist_D32": np.histogram(D32, bins)[0].tolist(),
                             "hist_D_wave": np.histogram(Dw, bins)[0].tolist(),
                             "rhs_utilisation_step1": o["stats"]["n_rhs"] / max(1, o["stats"]["n_rhs_slots"])})
                print(json.dumps(rows[-1]), file=sys.stderr, flush=True)
    out = {"metric": "divergence study: ignition-sampled states, trajectory order vs shuffled",
           "unit": "cell-ODEs/s", "n_gpus": 1, "steps": args.steps, "dtype": "f64",
           "data": "synthetic", "hist_bins": bins.tolist(), "rows": rows}
    print(json.dumps(out), flush=True)


def study_crossover(args):
    """RKC against RKCK as stiffness and the global step grow (Sec. 3: RKCK
    suits nonstiff chemistry, RKC moderately stiff; the ethylene case of
    Sec. 3.4 runs dt = 1e-4 s).  Mechanisms of the 9- and 13-species shapes
    drawn with stiffness caps lambda_cap of 5, 30 and 100 stages over 1e-6 s;
    8192 cells of each set's states; one global step of dt = 1e-8 ... 1e-4 s
    with both methods at the same tolerance and at most 50000 steps per cell.
    Reports cell-ODEs/s, mean and largest evaluations per cell (a launch lasts
    as long as its most expensive cell) and which method is faster."""
    import torch

    from paper_1309_2710_amd import rkc, synth

    dev = torch.device("cuda:0")
    rows = []
    n = 8192
    for cfg in ("c1", "c2"):
        c = synth.CONFIGS[cfg]
        for s_cap in (5, 30, 100):
            mech = synth.make_mechanism(c["n_species"], c["n_reactions"], c["elements"],
                                        c["mech_seed"], ea_max=c["ea_max"], T_lo=c["T_range"][0],
                                        T_hi=c["T_range"][1], P_max=c["P_max"], dt=1e-6,
                                        s_target=s_cap, name="%s_cap%d" % (cfg, s_cap))
            gm = rkc.Mechanism(mech)
            st = synth.make_states(mech, n, c["state_seed"], T_dist=c["T"], P_dist=c["P"],
                                   Y_dist=c["Y"])
            T0 = torch.from_numpy(st["T"]).to(dev)
            P = torch.from_numpy(st["P"]).to(dev)
            Y0 = torch.from_numpy(st["Y"]).to(dev)
            for dt in (1e-8, 1e-7, 1e-6, 1e-5, 1e-4):
                res = {}
                for name, method in (("rkc", rkc.RKC), ("rkck", rkc.RKCK)):
                    T, Y = T0.clone(), Y0.clone()
                    torch.cuda.synchronize()
                    t = time.perf_counter()
                    o = rkc.integrate(gm, T, P, Y, dt, c["rtol"], c["atol"], method=method,
                                      stats=True, status=False, counters=True, max_steps=50000)
                    torch.cuda.synchronize()
                    wall = time.perf_counter() - t
                    res[name] = {"cell_odes_per_s": n / wall,
                                 "rhs_per_cell": o["stats"]["n_rhs"] / n,
                                 "rhs_max_cell": int(o["counters"][:, 0].max().item()),
                                 "failed": o["stats"]["n_failed"]}
                ok = [k for k in res if res[k]["failed"] == 0]
                row = {"set": "%dsp/%drx" % (mech["n_species"], mech["n_reactions"]),
                       "lambda_cap_stages": s_cap, "lambda_cap": mech["lambda_cap"], "dt": dt,
                       "cells": n, "rkc": res["rkc"], "rkck": res["rkck"],
                       "faster": max(ok, key=lambda k: res[k]["cell_odes_per_s"]) if ok else None}
                rows.append(row)
                print(json.dumps(row), file=sys.stderr, flush=True)
    out = {"metric": "RKC vs RKCK crossover in stiffness cap and global step", "unit": "cell-ODEs/s",
           "n_gpus": 1, "dtype": "f64", "data": "synthetic", "rows": rows}
    print(json.dumps(out), flush=True)


def served_block(n_requests, util):
    """Batch latency of the served workload at a stated offered utilisation.

    The mixed 13/53-species request stream (1024-65536 cells, dt 1e-6 or
    1e-5 s, fresh compositions) is first served back to back with
    rkc_integrate to measure the GPU's capacity for it (requests per second
    = requests / total service time); the same requests are then replayed with
    Poisson arrivals at util x capacity through the integration server, and
    through sequential rkc_integrate calls as the baseline.  Latency runs from
    arrival to completion, so at util < 1 p50/p99 measure service plus the
    queueing of a stable system."""
    import threading

    from paper_1309_2710_amd import rkc, synth

    trace = synth.c5_trace(n_requests=n_requests, rate=1.0)   # arrival times rescaled below
    keys = sorted({r["mech"] for r in trace})
    mechs = {k: synth.c5_mechanism(*k) for k in keys}
    gms = {k: rkc.Mechanism(m) for k, m in mechs.items()}
    cfg = {13: synth.CONFIGS["c2"], 53: synth.CONFIGS["c3"]}
    for k in keys:   # first-use tables outside the measurements
        c = cfg[k[0]]
        st = synth.make_states(mechs[k], 1, 1, T_dist=c["T"], P_dist=c["P"], Y_dist=c["Y"])
        rkc.integrate(gms[k], st["T"], st["P"], st["Y"], 1e-6)

    # capacity: the requests back to back
    inp = serve_inputs(trace, synth)
    busy = []
    for r, x in zip(trace, inp):
        c = cfg[r["mech"][0]]
        a = time.perf_counter()
        rkc.integrate(gms[r["mech"]], x["T"], x["P"], x["Y"], r["dt"], c["rtol"], c["atol"])
        busy.append(time.perf_counter() - a)
    capacity = len(trace) / sum(busy)
    rate = util * capacity
    scale = 1.0 / rate   # the trace was drawn at 1 request/s
    arrivals = [r["t_arrival"] * scale for r in trace]
    print("served: capacity %.2f req/s, replay at %.2f req/s" % (capacity, rate),
          file=sys.stderr, flush=True)

    def pct(v, q):
        v = sorted(v)
        return v[min(len(v), max(1, int(np.ceil(q * len(v))))) - 1]

    # sequential baseline at the same arrivals
    inp = serve_inputs(trace, synth)
    lat_b = []
    t0 = time.perf_counter()
    for r, x, ta in zip(trace, inp, arrivals):
        now = time.perf_counter() - t0
        if now < ta:
            time.sleep(ta - now)
        c = cfg[r["mech"][0]]
        rkc.integrate(gms[r["mech"]], x["T"], x["P"], x["Y"], r["dt"], c["rtol"], c["atol"])
        lat_b.append((time.perf_counter() - t0 - ta) * 1e3)

    # the server
    inp = serve_inputs(trace, synth)
    srv = rkc.Server(budget_bytes=4 << 30, n_streams=4)
    ids = {k: srv.register(m) for k, m in mechs.items()}
    rids = [None] * len(trace)

    def waiter():
        for i in range(len(trace)):
            while rids[i] is None:
                time.sleep(1e-4)
            srv.wait(rids[i])

    th = threading.Thread(target=waiter)
    srv.reset_stats()
    t0 = time.perf_counter()
    th.start()
    for i, (r, x, ta) in enumerate(zip(trace, inp, arrivals)):
        now = time.perf_counter() - t0
        if now < ta:
            time.sleep(ta - now)
        c = cfg[r["mech"][0]]
        rids[i] = srv.submit(ids[r["mech"]], x["T"], x["P"], x["Y"], r["dt"], c["rtol"], c["atol"])
    th.join()
    wall = time.perf_counter() - t0
    sst = srv.stats()
    srv.close()
    cells = sum(r["n_cells"] for r in trace)
    return {"p50_ms": sst["p50_ms"], "p99_ms": sst["p99_ms"], "mean_ms": sst["mean_ms"],
            "offered_utilisation": util, "capacity_req_per_s": capacity,
            "arrival_rate_req_per_s": rate, "requests": len(trace), "cells": cells,
            "served_cells_per_s": cells / wall, "failed_requests": sst["failed_requests"],
            "sequential_p50_ms": pct(lat_b, 0.5), "sequential_p99_ms": pct(lat_b, 0.99),
            "workload": "mixed 13/53-species requests (4 seeded mechanisms each), "
                        "2^U(10,16) cells, dt 1e-6 or 1e-5 s, fresh compositions, Poisson "
                        "arrivals at the stated fraction of the measured capacity"}


def serve_inputs(trace, synth):
    """Per-request input copies: each request takes a contiguous run of cells
    from a seeded pool of states of its mechanism (65536 cells, the largest
    request), starting at an offset drawn from its state seed."""
    pools = {}
    reqs = []
    for r in trace:
        key = r["mech"]
        if key not in pools:
            kind, i = key
            base = "c2" if kind == 13 else "c3"
            c = synth.CONFIGS[base]
            pools[key] = synth.make_states(synth.c5_mechanism(kind, i), 1 << 16,
                                           synth.C5_SEED * 10 + kind * 4 + i,
                                           T_dist=c["T"], P_dist=c["P"], Y_dist=c["Y"])
        pool = pools[key]
        n = r["n_cells"]
        o = r["state_seed"] % ((1 << 16) - n + 1)
        reqs.append({"T": pool["T"][o:o + n].copy(), "P": pool["P"][o:o + n].copy(),
                     "Y": pool["Y"][o:o + n].copy()})
    return reqs


def serve(args):
    """Served workload: the mixed-request trace replayed at its arrival times
    through the server (submission thread sleeping until each arrival), and
    the same trace served by sequential rkc_integrate calls as the baseline."""
    import threading

    from paper_1309_2710_amd import rkc, synth

    trace = synth.c5_trace(n_requests=args.serve_requests, rate=args.serve_rate)
    keys = sorted({r["mech"] for r in trace})
    mechs = {k: synth.c5_mechanism(*k) for k in keys}
    span = trace[-1]["t_arrival"]
    cells = sum(r["n_cells"] for r in trace)

    # baseline: one synchronous rkc_integrate per request in arrival order
    gms = {k: rkc.Mechanism(m) for k, m in mechs.items()}
    inp = serve_inputs(trace, synth)
    for r, x in zip(trace, inp):   # first-use table builds outside the timed replay
        if r["mech"] in keys:
            keys = [k for k in keys if k != r["mech"]]
            rkc.integrate(gms[r["mech"]], x["T"][:1].copy(), x["P"][:1].copy(),
                          x["Y"][:1].copy(), r["dt"])
    busy = 0.0
    lat_b = []
    base_status = np.zeros(5, np.int64)
    t0 = time.perf_counter()
    for r, x in zip(trace, inp):
        now = time.perf_counter() - t0
        if now < r["t_arrival"]:
            time.sleep(r["t_arrival"] - now)
        c = synth.CONFIGS["c2" if r["mech"][0] == 13 else "c3"]
        a = time.perf_counter()
        o = rkc.integrate(gms[r["mech"]], x["T"], x["P"], x["Y"], r["dt"], c["rtol"],
                          c["atol"])
        b = time.perf_counter()
        base_status += np.bincount(o["status"], minlength=5)[:5]
        if (len(lat_b) + 1) % 100 == 0:
            print("baseline: %d/%d requests, %.1f s" % (len(lat_b) + 1, len(trace),
                                                        time.perf_counter() - t0),
                  file=sys.stderr, flush=True)
        busy += b - a
        lat_b.append((b - t0 - r["t_arrival"]) * 1e3)
    base_wall = time.perf_counter() - t0
    del gms

    # served: the same trace through the server
    inp = serve_inputs(trace, synth)
    srv = rkc.Server(budget_bytes=4 << 30, n_streams=args.serve_streams)
    ids = {k: srv.register(m) for k, m in mechs.items()}
    rids = [None] * len(trace)
    done = threading.Event()

    def waiter():
        for i in range(len(trace)):
            while rids[i] is None:
                time.sleep(1e-4)
            srv.wait(rids[i])
            if (i + 1) % 100 == 0:
                print("served: %d/%d completed, %.1f s" % (i + 1, len(trace),
                                                           time.perf_counter() - t0),
                      file=sys.stderr, flush=True)
        done.set()

    th = threading.Thread(target=waiter)
    srv.reset_stats()
    t0 = time.perf_counter()
    th.start()
    for i, (r, x) in enumerate(zip(trace, inp)):
        now = time.perf_counter() - t0
        if now < r["t_arrival"]:
            time.sleep(r["t_arrival"] - now)
        c = synth.CONFIGS["c2" if r["mech"][0] == 13 else "c3"]
        x["S"] = np.empty(r["n_cells"], np.int32)
        rids[i] = srv.submit(ids[r["mech"]], x["T"], x["P"], x["Y"], r["dt"], c["rtol"],
                             c["atol"], status=x["S"])
        if (i + 1) % 200 == 0:
            print("served: %d/%d submitted, %.1f s" % (i + 1, len(trace), time.perf_counter() - t0),
                  file=sys.stderr, flush=True)
    th.join()
    wall = time.perf_counter() - t0
    st = srv.stats()
    srv.close()
    served_status = np.zeros(5, np.int64)
    failures = []
    for i, (r, x) in enumerate(zip(trace, inp)):
        h = np.bincount(x["S"], minlength=5)[:5]
        served_status += h
        if h[1:].sum() and len(failures) < 10:
            failures.append({"request": i, "mech": list(r["mech"]), "dt": r["dt"],
                             "n_cells": r["n_cells"], "status_counts": h.tolist(),
                             "first_failed_cell": int(np.nonzero(x["S"])[0][0])})

    def pct(v, q):
        v = sorted(v)
        return v[min(len(v), max(1, int(np.ceil(q * len(v))))) - 1]

    out = {
        "metric": "p99 request latency, served mixed 13/53-species trace (FP64)",
        "value": st["p99_ms"],
        "unit": "ms",
        "n_gpus": 1,
        "higher_is_better": False,
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "mixed 13/53-species requests: %d, Poisson %.0f req/s over %.2f s, 2^U(10,16) "
                               "cells, 13/53 species, dt 1e-6/1e-5" % (len(trace), args.serve_rate,
                                                                        span),
                   "cells": cells, "n_streams": args.serve_streams},
        "served": {"p50_ms": st["p50_ms"], "p99_ms": st["p99_ms"], "mean_ms": st["mean_ms"],
                   "max_ms": st["max_ms"], "wall_s": wall, "cells_per_s": cells / wall,
                   "launches": st["launches"], "peak_queue": st["peak_queue"],
                   "peak_bytes": st["peak_bytes"], "failed_requests": st["failed_requests"],
                   "cell_status_counts": served_status.tolist(), "failures": failures},
        "sequential_baseline": {"p50_ms": pct(lat_b, 0.5), "p99_ms": pct(lat_b, 0.99),
                                "wall_s": base_wall, "busy_s": busy,
                                "cell_status_counts": base_status.tolist(),
                                "cells_per_s": cells / busy},
        "offered_utilisation": busy / span,
    }
    print(json.dumps(out), flush=True)


def cpu_baseline(mech, c, st, steps, budget_s, method="rkc"):
    """The serial FP64 oracle (unchanged; cells split over host threads) on a
    strided sample of the same workload, K consecutive global steps."""
    from oracle import oracle as O

    M = O.Model(mech)
    om = O.RKCK if method == "rkck" else O.RKC
    # the host cores this process may use (affinity), within the 16-core
    # share the GPU host gives one GPU's job
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count() or 1
    threads = max(1, min(usable, 16))
    model = ""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    n = st["T"].shape[0]

    def run(idx):
        T, Y = st["T"][idx].copy(), st["Y"][idx].copy()
        P = st["P"][idx]
        t = time.perf_counter()
        for _ in range(steps):
            T, Y, _ = M.integrate(T, P, Y, c["dt"], c["rtol"], c["atol"], method=om,
                                  threads=threads)
        return time.perf_counter() - t

    # one host core on a small strided sample (the per-cell code is serial)
    one = np.arange(0, n, max(1, n // 64))[:64]
    T1, Y1 = st["T"][one].copy(), st["Y"][one].copy()
    t1 = time.perf_counter()
    for _ in range(steps):
        T1, Y1, _ = M.integrate(T1, st["P"][one], Y1, c["dt"], c["rtol"], c["atol"], method=om,
                                threads=1)
    one_core = len(one) * steps / (time.perf_counter() - t1)

    probe = np.arange(0, n, max(1, n // (4 * threads)))[:4 * threads]
    t_probe = run(probe)
    per_cell = t_probe / len(probe)
    m = int(min(n, max(len(probe), budget_s / max(per_cell, 1e-9))))
    m = max(threads, (m // threads) * threads)
    idx = np.arange(0, n, max(1, n // m))[:m]
    t = run(idx)
    return {"value": len(idx) * steps / t, "unit": "cell-ODEs/s", "cores": threads,
            "nproc": os.cpu_count(), "usable_cores": usable, "cpu_model": model,
            "kind": "oracle", "one_core_value": one_core,
            "sample": "%d of %d cells (stride %d), %d consecutive global steps, %.1f s"
                      % (len(idx), n, max(1, n // m), steps, t)}


if __name__ == "__main__":
    main()
