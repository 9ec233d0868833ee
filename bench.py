"""Benchmark of the coupled LB/MD hot path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload c3|c1|c0|c4]

A step is one full coupled step (trilinear gather, the 100-sub-step bead
cycle, deterministic spreading, and the fused stream + collide sweep over
every lattice node), replayed from the captured HIP graph of two steps: the
library's production path.  The default workload is the large single run:
512 x 256 x 256 nodes (33.5 M), wall normal to x at x = 256 with a 7 x 7
pore, one 8000-bead chain, FP32 deviation storage of the populations.
Inputs are synthetic (seeded self-avoiding coil, relaxed on the GPU before
timing) and resident in HBM before the timed region.  The sweep's tile
layout is the one the committed kernel trace of the coupled step was taken
in (profiles/coupled_step_<storage>_<workload>_kernels.json, the coupled
autotuner's choice when it was taken), so that the roofline line and the
trace describe the same launches; the autotuner's choice on the GPU at hand
is timed beside it (--sweep-layout auto times that instead).

Prints one JSON line: the metric (MLUPS of the whole coupled step), the
roofline of the dominant kernel (the LB sweep, timed with HIP events inside
the library on the stream it runs on, over the same number of eager steps),
the eager steps' rate, the FP64 path on the same workload, bead throughput, the
batched ensemble (64 uneven replicas in one context, graph replay, aggregate
MLUPS and translocation steps), the adjoint on the 64^3 gradient workload
(adjoint steps/s in FP64 and FP32, a finite-difference check), the same
workload with a fluctuating fluid (noise on the non-conserved modes drawn in
the sweep), the same lattice and chain with the paper's soft bead LJ under
the multiple-time-step cycle and under uniform sub-steps, FP32 deviation
storage against FP64 storage over time on the 128^3 system with 400 beads at
three frictions (errors of rho - 1, u and r, MLUPS of both), and the FP64 CPU
oracle timed on a bounded sample.  A line on stderr marks the end of each
leg.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0   # MI355X HBM3E peak, GB/s
Q = 19


def progress(msg):
    """One line on stderr when a leg of the benchmark has finished."""
    print(f"bench: {msg}", file=sys.stderr, flush=True)


def lb_bytes_per_update(elem_bytes):
    """Algorithmic bytes of one fluid-node update of the pull sweep: read 19
    populations, write 19 populations, read the 1-byte node flag."""
    return 2 * Q * elem_bytes + 1


def measured_traffic(workload, precision, layout, thermal=False):
    """HBM bytes per sweep launch from the committed rocprofv3 counter
    summary (of the athermal sweep, or with thermal of the sweep that draws
    the fluid noise), if it was taken on the current kernel source and holds
    the sweep layout in use; else None."""
    from paper_0711_2665_amd.build import kernel_source_hash
    tag = f"{precision}_thermal" if thermal else precision
    path = os.path.join(ROOT, "profiles", f"lb_sweep_{tag}_{workload}_counters.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        d = json.load(fh)
    if d.get("kernel_source_hash") != kernel_source_hash():
        return None
    for e in d.get("per_layout", []):
        if e["layout"] == layout:
            return e["bytes_per_launch"]
    return None


def profiled_launch(workload, precision, layout, mean_ms, alg_bytes):
    """The committed rocprofv3 kernel trace of the coupled step for this
    workload and storage: its file, the sweep layout and kernel source it was
    taken on, the sweep's mean launch over the trace's timed dispatches, and
    the roofline fraction that mean gives, beside this run's (None if there
    is no trace)."""
    from paper_0711_2665_amd.build import kernel_source_hash
    base = os.path.join("profiles", f"coupled_step_{precision}_{workload}_kernels")
    path = os.path.join(ROOT, base + ".json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        d = json.load(fh)
    prof_ms = d["mean_launch_ms"]
    return {"file": base + ".md", "layout": d.get("layout"), "same_layout": d.get("layout") == layout,
            "same_kernel_source": d.get("kernel_source_hash") == kernel_source_hash(),
            "dispatches": d["dispatches"], "mean_launch_ms": round(prof_ms, 5),
            "frac": round(alg_bytes / (prof_ms * 1e-3) / 1e9 / PEAK_HBM_GBS, 4),
            "vs_this_run": round(prof_ms / mean_ms - 1.0, 4)}


def sweep_alone(run, cells, elem):
    """Roofline of the sweep run alone over every fluid node in the layout
    the sweep-only autotuner picks (in the coupled step the layout is picked
    for the whole step, and the sweep shares the memory system with the bead
    phase)."""
    a = run["alone"]
    nbytes = run["nfluid"] * lb_bytes_per_update(elem) + (cells - run["nfluid"])
    gbs = nbytes / (a["ms"] * 1e-3) / 1e9
    return {"layout": {k: a[k] for k in ("tile_nodes", "order", "grid", "cap")}, "mean_launch_ms": round(a["ms"], 5),
            "bytes_per_launch": int(nbytes), "achieved": round(gbs, 1), "frac": round(gbs / PEAK_HBM_GBS, 4)}


def profile_layout(workload, precision):
    """The sweep layout of the committed kernel trace of the coupled step
    (profiles/coupled_step_<storage>_<workload>_kernels.json), or None."""
    path = os.path.join(ROOT, "profiles", f"coupled_step_{precision}_{workload}_kernels.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        lay = json.load(fh).get("layout")
    return tuple(lay[k] for k in ("tile_nodes", "order", "grid", "cap")) if lay else None


def run_gpu(cfg, precision_name, steps, warmup, layout=None, compare_autotuned=False):
    """Relax, time the sweep alone (autotuner, sweep-only mode), choose the
    sweep layout by timing whole coupled steps, then:
    `steps` coupled steps replayed from the captured two-step HIP graph (the
    timed region of the headline figure), and `steps` eager steps with the
    library's per-step HIP events around the sweep and the bead phase (the
    kernel durations of the roofline)."""
    import torch
    from paper_0711_2665_amd import lbmd
    from paper_0711_2665_amd.workloads import initial_chain

    prec = lbmd.LB_FP32_DEV if precision_name == "fp32dev" else lbmd.LB_FP64
    r, v = initial_chain(cfg)
    sim = lbmd.Simulation(cfg, r, v, precision=prec, device="cuda:0")
    sim.relax(cfg["relax_substeps"], cfg["gamma_relax"])
    # the sweep alone (every fluid node, nothing beside it), in the layout
    # that is fastest for it, timed by the autotuner with HIP events
    alone = sim.autotune(reps=10)
    auto = None
    if layout is None:
        tune = sim.autotune(reps=10, coupled=True)
    else:
        if compare_autotuned:
            # the coupled autotuner's choice on this GPU, timed like the
            # headline when it differs from the pinned layout
            at = sim.autotune(reps=10, coupled=True)
            alay = tuple(at[k] for k in ("tile_nodes", "order", "grid", "cap"))
            auto = {"layout": {k: at[k] for k in ("tile_nodes", "order", "grid", "cap")}}
            if alay != tuple(layout):
                sim.run(warmup + (warmup & 1), graph=True)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                sim.run(steps, graph=True)
                torch.cuda.synchronize()
                auto["ms_per_step"] = round(1e3 * (time.perf_counter() - t0) / steps, 4)
        sim.sweep_config(*layout)
        tune = dict(zip(("tile_nodes", "order", "grid", "cap"), layout))
    sim.run(warmup + (warmup & 1), graph=True)          # capture, warm replays
    torch.cuda.synchronize()
    sim.check()
    t0 = time.perf_counter()
    sim.run(steps, graph=True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    sim.check()
    out = dict(seconds=t1 - t0, tune=tune, alone=alone, autotuned=auto)
    diag0 = sim.diagnostics()
    sim.profile_start(steps)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.couple_step(steps)
    torch.cuda.synchronize()
    out["eager_seconds"] = time.perf_counter() - t0
    out["lb_ms"], out["bead_ms"], out["nrec"] = sim.profile_stop()
    sim.check()
    diag1 = sim.diagnostics()
    out["forced_per_step"] = (diag1["forced_total"] - diag0["forced_total"]) / steps
    out["rebuilds_per_step"] = (diag1["rebuilds"] - diag0["rebuilds"]) / steps
    out["cell_rebuilds_per_step"] = (diag1["cell_rebuilds"] - diag0["cell_rebuilds"]) / steps
    out["obs"] = sim.observables().cpu().numpy()
    out["nfluid"] = int(((sim.flags() & 1) == 0).sum().item())
    del sim
    torch.cuda.empty_cache()
    return out


def run_ensemble(steps, warmup, eager_steps):
    """The batched ensemble: 64 replicas, cubic edges from {48, 64, 80, 96},
    chains of {50, 100, 200, 500} beads, pore 3..5, pore force U(0.01, 0.04),
    own noise key each, FP32 deviation storage, one context; coupled steps
    replayed from a captured HIP graph."""
    import torch
    from paper_0711_2665_amd import lbmd
    from paper_0711_2665_amd.workloads import ensemble_configs, initial_chain

    cfgs = ensemble_configs(64)
    r0s = [initial_chain(c)[0] for c in cfgs]
    ens = lbmd.Ensemble(cfgs, r0s, precision=lbmd.LB_FP32_DEV, device="cuda:0")
    ens.relax(cfgs[0]["relax_substeps"], cfgs[0]["gamma_relax"])
    tune = ens.autotune(reps=10, coupled=True)
    ens.couple_step(warmup)
    torch.cuda.synchronize()
    ens.check()
    t0 = time.perf_counter()
    ens.couple_step(eager_steps)
    torch.cuda.synchronize()
    eager_s = time.perf_counter() - t0
    ens.run(2, graph=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ens.run(steps, graph=True)
    torch.cuda.synchronize()
    graph_s = time.perf_counter() - t0
    ens.check()
    tx = ens.translocation_steps()
    total_steps = ens.step_count()
    cells = sum(c["shape"][0] * c["shape"][1] * c["shape"][2] for c in cfgs)
    beads = sum(c["nb"] for c in cfgs)
    done = sorted(t for t in tx if t >= 0)
    by_len = {}
    for c, t in zip(cfgs, tx):
        by_len.setdefault(c["nb"], []).append(t)
    # the duration histogram of the replicas that translocated, with the
    # most probable time (Freedman-Diaconis bins)
    from paper_0711_2665_amd.translocation import most_probable_time
    mp, counts, edges = most_probable_time(done) if done else (None, None, None)
    res = {
        "replicas": len(cfgs), "cells": cells, "beads": beads, "steps": steps,
        "value": round(cells * steps / graph_s / 1e6, 1), "unit": "MLUPS (aggregate)",
        "ms_per_step": round(1e3 * graph_s / steps, 4),
        "eager_ms_per_step": round(1e3 * eager_s / eager_steps, 4),
        "bead_steps_per_s": round(beads * steps / graph_s, 1),
        "sweep_layout": {k: tune[k] for k in ("tile_nodes", "order", "grid", "cap")},
        "translocation": {"steps_run": total_steps, "translocated": len(done), "censored": len(tx) - len(done),
                          "steps": done,
                          "histogram": {"counts": counts.tolist() if counts is not None else [],
                                        "bin_edges": [round(float(e), 1) for e in edges] if edges is not None else [],
                                        "most_probable": mp},
                          "by_chain_length": {str(k): sorted(t for t in v if t >= 0) for k, v in sorted(by_len.items())}},
    }
    del ens
    torch.cuda.empty_cache()
    return res


VALIDATED_HORIZON = 200   # steps at which the FP64 adjoint of the benchmarked workload matches the oracle's
                          # forward-mode derivative to 1e-8 (tests/test_gpu_adjoint_horizon.py)


def run_adjoint(nsteps, K, horizons):
    """The gradient workload: 64^3, 100-bead chain, pore 3 x 3, loss = mean
    normal coordinate after the run, gradient w.r.t. gamma, F_drive and the
    initial positions by the library's adjoint with checkpoints every K
    steps.  Timed over nsteps coupled steps in FP64 and FP32 deviation
    storage, and again as one segment (the forward pass writes the whole
    horizon's tape into HBM, and the backward pass does not recompute it;
    the gradient is the same bit for bit).

    The bead dynamics is chaotic: the derivative of the discrete map grows
    roughly like exp(0.013 n), and the last-bit differences between two FP64
    evaluations of the same map (the GPU's and the host's log, sin, cos,
    atan2) are amplified as much.  The FP64 adjoint matches the oracle's
    forward-mode derivative to 1e-8 up to VALIDATED_HORIZON steps (the GPU
    test); the gradients reported there are the validated ones.  The values
    over the full nsteps are reported too, marked chaos-dominated, with the
    spread between FP32 and FP64 storage: they are the derivative of each
    run's own trajectory and do not agree between precisions.  Finite
    differences (h = 1e-6 in gamma, FP64) resolve the derivative only over
    short horizons, before trajectories cross interpolation kinks inside the
    difference interval; the scan shows where."""
    import numpy as np
    import torch
    from paper_0711_2665_amd import lbmd
    from paper_0711_2665_amd.workloads import C4, initial_chain

    cfg = C4
    r, v = initial_chain(cfg)
    out = {"workload": cfg["name"], "steps": nsteps, "checkpoint_every": K}
    dLdr = np.zeros((cfg["nb"], 3))
    dLdr[:, cfg["wall_axis"]] = 1.0 / cfg["nb"]
    sims = {}
    full = {}
    for name, prec in (("fp64", lbmd.LB_FP64), ("fp32dev", lbmd.LB_FP32_DEV)):
        sim = lbmd.Simulation(cfg, r, v, precision=prec, device="cuda:0")
        sim.relax(cfg["relax_substeps"], cfg["gamma_relax"])
        st = sim.get_state()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sim.adjoint_forward(nsteps, K)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        g = sim.adjoint_backward(dLdr).cpu().numpy()
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        sim.check()
        out[name] = {"adjoint_steps_per_s": round(nsteps / (t2 - t0), 2), "forward_s": round(t1 - t0, 3),
                     "reverse_s": round(t2 - t1, 3)}
        full[name] = {"dL_dgamma": float(g[0]), "dL_dF_drive": float(g[1])}
        # the same horizon as one segment: the forward pass writes the whole
        # tape (held in HBM) and the backward pass does not recompute it
        sim.set_state(st)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sim.adjoint_forward(nsteps, nsteps)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        g1 = sim.adjoint_backward(dLdr).cpu().numpy()
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        sim.check()
        out[name]["one_segment"] = {
            "adjoint_steps_per_s": round(nsteps / (t2 - t0), 2), "forward_s": round(t1 - t0, 3),
            "reverse_s": round(t2 - t1, 3), "workspace_GB": round(sim.adjoint_sizes(nsteps, nsteps) / 1e9, 2),
            "same_gradient_bits": bool(np.array_equal(g, g1))}
        sim._adj_ws = None
        torch.cuda.empty_cache()
        sims[name] = (sim, st)

    def grad(name, T):
        sim, st = sims[name]
        sim.set_state(st)
        sim.set_coupling(cfg["gamma"], cfg["f_drive"])
        sim.adjoint_forward(T, min(K, T))
        return sim.adjoint_backward(dLdr).cpu().numpy()

    def loss(T, gamma):
        sim, st = sims["fp64"]
        sim.set_state(st)
        sim.set_coupling(gamma, cfg["f_drive"])
        sim.couple_step(T)
        return float(sim.beads()["r"][:, cfg["wall_axis"]].mean())

    def spread(a, b):
        return abs(a - b) / max(abs(b), 1e-300)

    gv = {name: grad(name, VALIDATED_HORIZON) for name in sims}
    out["validated_horizon"] = {
        "steps": VALIDATED_HORIZON,
        "criterion": "FP64 adjoint within 1e-8 of the FP64 oracle's forward-mode derivative in dgamma, dF_drive "
                     "and a random direction of r(0) (the deterministic variant, kT = 0 and kappa = 0, "
                     "matches over the full horizon)",
        "fp64": {"dL_dgamma": float(gv["fp64"][0]), "dL_dF_drive": float(gv["fp64"][1])},
        "fp32dev": {"dL_dgamma": float(gv["fp32dev"][0]), "dL_dF_drive": float(gv["fp32dev"][1])},
        "fp32dev_rel_diff": {"dL_dgamma": spread(gv["fp32dev"][0], gv["fp64"][0]),
                             "dL_dF_drive": spread(gv["fp32dev"][1], gv["fp64"][1])}}
    out["full_horizon"] = {
        "steps": nsteps, "chaos_dominated": True,
        "note": "derivative of each run's own trajectory past the validated horizon; FP32 and FP64 storage, "
                "and two FP64 codes, disagree here",
        "fp64": full["fp64"], "fp32dev": full["fp32dev"],
        "fp32dev_rel_diff": {k: spread(full["fp32dev"][k], full["fp64"][k]) for k in ("dL_dgamma", "dL_dF_drive")}}
    h = 1e-6
    scan = []
    for T in horizons:
        g64 = grad("fp64", T)
        g32 = grad("fp32dev", T)
        fd = (loss(T, cfg["gamma"] + h) - loss(T, cfg["gamma"] - h)) / (2 * h)
        scan.append({"steps": T, "dL_dgamma_adjoint": float(g64[0]), "dL_dgamma_fd": fd,
                     "fd_rel_diff": spread(float(g64[0]), fd),
                     "fp32dev_rel_diff": spread(float(g32[0]), float(g64[0]))})
    out["fd_scan"] = scan
    for name in list(sims):
        del sims[name]
    torch.cuda.empty_cache()
    return out


def run_precision_study(steps):
    """The 128^3 system with 400 beads in both storages from the same relaxed
    chain, at each of its frictions: errors of rho - 1, u (relative to max |u|)
    and r against FP64 every 1/5 of the run, beside the envelope (the FP64
    run's distance from an FP64 run whose chain moved by one ulp), and the
    MLUPS of both storages."""
    from paper_0711_2665_amd.precision_study import run_gammas
    from paper_0711_2665_amd.workloads import C1
    n = C1["steps"] if steps is None else steps
    res = run_gammas(C1, n, max(1, n // 5))
    keys = ("step", "rho_err_max", "rho_err_rms", "rho_dev_max", "u_max", "u_err_max_rel", "u_err_rms_rel",
            "r_err_max", "r_err_rms", "env_rho_max", "env_u_max_rel", "env_r_max")
    return {"workload": C1["name"], "steps": n,
            "runs": [{"gamma": r["gamma"],
                      "mlups": {k: round(v, 1) for k, v in r["mlups"].items()},
                      "series": [{k: (row[k] if k == "step" else float(f"{row[k]:.3e}")) for k in keys}
                                 for row in r["series"]]} for r in res]}


def cpu_model():
    """Model name and logical CPU count of the host, from /proc/cpuinfo."""
    name, n = "unknown", 0
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    n += 1
                    name = line.split(":", 1)[1].strip()
    except OSError:
        pass
    return name, n or os.cpu_count()


def _time_oracle(cfg, steps, relax):
    """Seconds of `steps` coupled FP64 oracle steps of the whole workload
    (after `relax` oracle relaxation sub-steps and one untimed step)."""
    import oracle
    from paper_0711_2665_amd.workloads import initial_chain
    r, v = initial_chain(cfg)
    o = oracle.Oracle(cfg, r, v)
    o.relax(relax, cfg["gamma_relax"])
    o.couple_step(1)
    t0 = time.perf_counter()
    o.couple_step(steps)
    return time.perf_counter() - t0


def run_cpu_baseline(cfg, steps, full=True):
    """The FP64 oracle as it stands, timed on the host: the benchmarked
    workload on a bounded sample (`steps` coupled steps of the full lattice
    and chain after a short relaxation) on all host threads and on one; with
    `full`, also the 32^3 / 20-bead parity workload (200 steps) and the
    64^3 / 100-bead gradient workload (2000 steps) in full on all threads, a
    stated sample of each on one thread, and a sample of the 128^3 / 400-bead
    workload."""
    import oracle
    from paper_0711_2665_amd.workloads import C0, C1, C4

    def mlups(c, n, sec):
        return c["shape"][0] * c["shape"][1] * c["shape"][2] * n / sec / 1e6

    allthr = oracle.max_threads()
    runs = []

    def one(c, n, thr, relax, what):
        oracle.set_threads(thr)
        sec = _time_oracle(c, n, relax)
        runs.append({"workload": c["name"], "steps": n, "threads": thr, "seconds": round(sec, 2),
                     "MLUPS": round(mlups(c, n, sec), 3), "what": what})
        return sec

    try:
        sec = one(cfg, steps, allthr, 200, "sample")
        sec1 = one(cfg, 1, 1, 200, "sample")
        if full:
            one(C0, C0["steps"], allthr, C0["relax_substeps"], "full")
            one(C0, C0["steps"], 1, C0["relax_substeps"], "full")
            one(C4, C4["steps"], allthr, C4["relax_substeps"], "full")
            one(C4, 50, 1, C4["relax_substeps"], "sample")
            one(C1, 5, allthr, C1["relax_substeps"], "sample")
    finally:
        oracle.set_threads(allthr)
    model, logical = cpu_model()
    return dict(value=mlups(cfg, steps, sec), cores=allthr, seconds=sec,
                single_thread=mlups(cfg, 1, sec1), single_seconds=sec1, runs=runs,
                cpu_model=model, logical_cpus=logical)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="c3")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-steps", type=int, default=3)
    ap.add_argument("--cpu-quick", action="store_true", help="only the benchmarked workload's samples")
    ap.add_argument("--precision", default="fp32dev", choices=["fp32dev", "fp64"])
    ap.add_argument("--no-ensemble", action="store_true")
    ap.add_argument("--ensemble-steps", type=int, default=5000)
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--adjoint-steps", type=int, default=2000)
    ap.add_argument("--no-thermal", action="store_true")
    ap.add_argument("--no-mts", action="store_true")
    ap.add_argument("--no-precision-study", action="store_true")
    ap.add_argument("--c1-steps", type=int, default=None)
    ap.add_argument("--only", choices=["ensemble", "adjoint"], default=None,
                    help="run only this leg and print its object (profiling runs)")
    ap.add_argument("--sweep-layout", default="profiled",
                    help="the coupled step's sweep layout: tile_nodes,order,grid,cap; 'profiled' (the default) "
                         "takes the layout of the committed kernel trace, so that the roofline line and "
                         "profiles/ describe the same launches (the coupled autotuner's own choice is timed "
                         "beside it); 'auto' takes the coupled autotuner's choice")
    args = ap.parse_args()

    def layout_arg(prec):
        if args.sweep_layout == "auto":
            return None, "coupled autotuner"
        if args.sweep_layout == "profiled":
            lay = profile_layout(args.workload, prec)
            return (lay, "committed kernel trace") if lay else (None, "coupled autotuner (no kernel trace)")
        return tuple(int(x) for x in args.sweep_layout.split(",")), "argument"
    pinned, pinned_from = layout_arg(args.precision)
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU only (asked for {args.gpus}); "
              "the multi-GPU decomposition is a design, not an implementation", file=sys.stderr)
        sys.exit(2)

    if args.only:
        # one leg alone (for profiling runs): its object as the JSON line
        if args.only == "ensemble":
            res = run_ensemble(args.ensemble_steps, 20, 200)
        else:
            res = run_adjoint(args.adjoint_steps, 100, (5, 20, 50, 100))
        print(json.dumps({args.only: res}), flush=True)
        return

    from paper_0711_2665_amd.workloads import CONFIGS
    cfg = CONFIGS[args.workload]
    nx, ny, nz = cfg["shape"]
    cells = nx * ny * nz

    main_run = run_gpu(cfg, args.precision, args.steps, args.warmup, pinned,
                       compare_autotuned=args.sweep_layout == "profiled")
    progress(f"{cfg['name']} {args.precision}: {1e3 * main_run['seconds'] / args.steps:.4f} ms per step")
    ms_per_step = 1e3 * main_run["seconds"] / args.steps
    mlups = cells * args.steps / main_run["seconds"] / 1e6
    elem = 4 if args.precision == "fp32dev" else 8
    # the timed sweep skips the nodes carrying bead force (they are updated
    # after the spreading) and reads only their flag
    upd = main_run["nfluid"] - main_run["forced_per_step"]
    alg_bytes = int(round(upd * lb_bytes_per_update(elem) + (cells - upd)))
    achieved = alg_bytes / (main_run["lb_ms"] * 1e-3) / 1e9
    layout = {k: main_run["tune"][k] for k in ("tile_nodes", "order", "grid", "cap")}
    traffic = measured_traffic(args.workload, args.precision, layout)
    out = {
        "metric": "LB MLUPS of the coupled LB/MD step (and %HBM roofline of the LB sweep)",
        "value": round(mlups, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if args.precision == "fp32dev" else "f64",
        "data": "synthetic",
        "config": {"workload": cfg["name"], "lattice": [nx, ny, nz], "beads": cfg["nb"],
                   "n_sub": cfg["n_sub"], "storage": args.precision, "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": round(achieved / PEAK_HBM_GBS, 4), "traffic": traffic,
                     "kernel": "k_lb (fused stream+collide)", "bytes_per_launch": alg_bytes,
                     "mean_launch_ms": round(main_run["lb_ms"], 5),
                     "traffic_from": (f"profiles/lb_sweep_{args.precision}_{args.workload}_counters.md"
                                      if traffic is not None else None),
                     "profile": profiled_launch(args.workload, args.precision, layout, main_run["lb_ms"],
                                                alg_bytes)},
        "sweep_layout": layout,
        "sweep_layout_from": pinned_from,
        "autotuned": main_run["autotuned"],
        "sweep_alone": sweep_alone(main_run, cells, elem),
        "timing": "graph replay of the coupled step; roofline from the same kernels in eager steps",
        "eager": {"value": round(cells * args.steps / main_run["eager_seconds"] / 1e6, 1), "unit": "MLUPS",
                  "ms_per_step": round(1e3 * main_run["eager_seconds"] / args.steps, 4)},
        "lb_sweep_mlups": round(cells / (main_run["lb_ms"] * 1e-3) / 1e6, 1),
        "bead_phase_ms": round(main_run["bead_ms"], 4),
        "list_rebuilds_per_step": {"in_cycle": round(main_run["rebuilds_per_step"], 3),
                                   "from_cell_table": round(main_run["cell_rebuilds_per_step"], 3)},
        "bead_steps_per_s": round(cfg["nb"] * args.steps / main_run["seconds"], 1),
        "bead_substeps_per_s": round(cfg["nb"] * cfg["n_sub"] * args.steps / main_run["seconds"], 1),
    }
    if not args.no_fp64 and args.precision == "fp32dev":
        k64 = max(20, args.steps // 4)
        p64, p64_from = layout_arg("fp64")
        r64 = run_gpu(cfg, "fp64", k64, max(5, args.warmup // 4), p64)
        u64 = r64["nfluid"] - r64["forced_per_step"]
        alg64 = int(round(u64 * lb_bytes_per_update(8) + (cells - u64)))
        ach64 = alg64 / (r64["lb_ms"] * 1e-3) / 1e9
        lay64 = {k: r64["tune"][k] for k in ("tile_nodes", "order", "grid", "cap")}
        out["fp64"] = {"value": round(cells * k64 / r64["seconds"] / 1e6, 1), "unit": "MLUPS", "steps": k64,
                       "ms_per_step": round(1e3 * r64["seconds"] / k64, 4),
                       "eager_ms_per_step": round(1e3 * r64["eager_seconds"] / k64, 4),
                       "sweep_layout": lay64, "sweep_layout_from": p64_from,
                       "sweep_alone": sweep_alone(r64, cells, 8),
                       "lb_sweep_bytes_per_launch": alg64, "lb_sweep_mean_launch_ms": round(r64["lb_ms"], 5),
                       "lb_sweep_gbs": round(ach64, 1), "lb_sweep_frac": round(ach64 / PEAK_HBM_GBS, 4),
                       "lb_sweep_traffic": measured_traffic(args.workload, "fp64", lay64),
                       "profile": profiled_launch(args.workload, "fp64", lay64, r64["lb_ms"], alg64)}
        progress("fp64 done")
    if not args.no_thermal:
        # the same workload with a fluctuating fluid at the beads' temperature
        from paper_0711_2665_amd.workloads import scaled
        kth = max(20, args.steps // 2)
        rt = run_gpu(scaled(cfg, fluid_kT=cfg["kT"]), args.precision, kth, args.warmup)
        ut = rt["nfluid"] - rt["forced_per_step"]
        acht = (ut * lb_bytes_per_update(elem) + (cells - ut)) / (rt["lb_ms"] * 1e-3) / 1e9
        lay_t = {k: rt["tune"][k] for k in ("tile_nodes", "order", "grid", "cap")}
        out["thermal_fluid"] = {"value": round(cells * kth / rt["seconds"] / 1e6, 1), "unit": "MLUPS",
                                "steps": kth, "fluid_kT": cfg["kT"],
                                "ms_per_step": round(1e3 * rt["seconds"] / kth, 4),
                                "sweep_layout": lay_t,
                                "lb_sweep_traffic": measured_traffic(args.workload, args.precision, lay_t, True),
                                "sweep_alone": sweep_alone(rt, cells, elem),
                                "lb_sweep_gbs": round(acht, 1), "lb_sweep_frac": round(acht / PEAK_HBM_GBS, 4),
                                "lb_sweep_mean_launch_ms": round(rt["lb_ms"], 5)}
        progress("thermal fluid done")
    if not args.no_mts and args.workload == "c3":
        # the paper's bead LJ on the same lattice and chain, with the
        # multiple-time-step cycle (5 outer x 20 sub-steps) and, for
        # comparison, with 100 uniform sub-steps
        from paper_0711_2665_amd.workloads import C3M, scaled
        km = max(20, args.steps // 2)
        rm = run_gpu(C3M, args.precision, km, args.warmup)
        ru = run_gpu(scaled(C3M, mts_outer=0), args.precision, km, args.warmup)
        um = rm["nfluid"] - rm["forced_per_step"]
        achm = (um * lb_bytes_per_update(elem) + (cells - um)) / (rm["lb_ms"] * 1e-3) / 1e9
        out["paper_lj_mts"] = {
            "workload": C3M["name"], "value": round(cells * km / rm["seconds"] / 1e6, 1), "unit": "MLUPS",
            "steps": km, "ms_per_step": round(1e3 * rm["seconds"] / km, 4),
            "bead_phase_ms": round(rm["bead_ms"], 4), "lb_sweep_mean_launch_ms": round(rm["lb_ms"], 5),
            "lb_sweep_gbs": round(achm, 1), "lb_sweep_frac": round(achm / PEAK_HBM_GBS, 4),
            "sweep_layout": {k: rm["tune"][k] for k in ("tile_nodes", "order", "grid", "cap")},
            "uniform_100_substeps": {"value": round(cells * km / ru["seconds"] / 1e6, 1), "unit": "MLUPS",
                                     "ms_per_step": round(1e3 * ru["seconds"] / km, 4),
                                     "bead_phase_ms": round(ru["bead_ms"], 4)}}
        progress("multiple-time-step cycle done")
    if not args.no_ensemble and args.workload == "c3":
        out["ensemble"] = run_ensemble(args.ensemble_steps, 20, 200)
        progress("ensemble done")
    if not args.no_adjoint and args.workload == "c3":
        out["adjoint"] = run_adjoint(args.adjoint_steps, 100, (5, 20, 50, 100))
        progress("adjoint done")
    if not args.no_precision_study and args.workload == "c3":
        out["fp32_vs_fp64"] = run_precision_study(args.c1_steps)
        progress("FP32 against FP64 study done")
    if not args.no_cpu:
        cb = run_cpu_baseline(cfg, args.cpu_steps, full=not args.cpu_quick)
        out["cpu_baseline"] = {"value": round(cb["value"], 3), "unit": "MLUPS", "cores": cb["cores"],
                               "kind": "oracle",
                               "sample": f"{args.cpu_steps} coupled FP64 steps of the full {nx}x{ny}x{nz} lattice "
                                         f"with the {cfg['nb']}-bead chain ({cb['seconds']:.1f} s)",
                               "cpu_model": cb["cpu_model"], "logical_cpus": cb["logical_cpus"],
                               "single_thread": {"value": round(cb["single_thread"], 3), "unit": "MLUPS",
                                                 "sample": f"1 coupled FP64 step of the same lattice and chain "
                                                           f"({cb['single_seconds']:.1f} s)"},
                               "runs": cb["runs"],
                               "note": "the oracle as it stands (plain FP64 C++, OpenMP over nodes), a reported "
                                       "baseline and not a target"}
        progress("CPU baseline done")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
