"""FP32 deviation storage against FP64 storage on one system over time.

Two runs of the same system start from the same relaxed chain and the fluid
at rest, one storing f_i in FP64 and one storing f_i - w_i in FP32 (the bead
side is FP64 in both).  Every `sample_every` steps both fields are compared
on the fluid nodes:

- the density deviation rho - 1 (FP64: sum_i f_i - 1; FP32: sum_i (f_i - w_i),
  summed in FP64), max and RMS of the difference;
- the fluid velocity u = sum_i f_i c_i / rho, max and RMS of the difference
  divided by max |u| of the FP64 run;
- the bead positions, max and RMS of the absolute difference in lattice units.

The bead noise and the bead dynamics are the same in both runs, so the
position error starts at the FP32 rounding of the fluid and then grows with
the chain's own sensitivity to perturbations.  That sensitivity is measured
by a third run, FP64 from the same chain with every coordinate moved by one
ulp: its distance from the FP64 run (the envelope) is what any rounding
difference grows into, and the FP32 errors are reported beside it.  Each
run's stepping is timed
apart from the comparisons (graph replays of whole coupled steps), which
gives the MLUPS of both storages.

The comparisons read the populations through the binding's views and reduce
them with torch on the device; the stepping runs only in the library.
"""
import sys
import time

import numpy as np

from .workloads import initial_chain, scaled


def fluid_fields(sim, vel):
    """rho - 1 and u on the fluid nodes of replica 0, FP64 on the device."""
    from . import lbmd
    f = sim.pops().double().reshape(19, -1)
    fluid = ((sim.flags().reshape(-1) & 1) == 0)
    f = f[:, fluid]
    if sim.precision == lbmd.LB_FP32_DEV:      # deviations f - w
        drho = f.sum(0)
        rho = 1.0 + drho
    else:
        rho = f.sum(0)
        drho = rho - 1.0
    j = vel.t() @ f                              # [3, nfluid]; sum_i w_i c_i = 0
    return drho, j / rho


def _err(a, b, scale=1.0):
    d = (a - b).abs()
    return float(d.max().item()) / scale, float(d.pow(2).mean().sqrt().item()) / scale


def run(cfg, steps, sample_every, device="cuda:0", relax=None, envelope=True):
    """Both storages (and the perturbed FP64 run when `envelope`) over
    `steps` coupled steps; returns the error series and the MLUPS of each
    run."""
    import torch
    from . import lbmd
    vel = torch.tensor(lbmd.VELOCITIES, dtype=torch.float64, device=device)
    r, v = initial_chain(cfg)
    s64 = lbmd.Simulation(cfg, r, v, precision=lbmd.LB_FP64, device=device)
    s64.relax(cfg["relax_substeps"] if relax is None else relax, cfg["gamma_relax"])
    rr = s64.beads()["r"].cpu().numpy().copy()
    s64.close()
    sims = {"fp64": lbmd.Simulation(cfg, rr, np.zeros_like(rr), precision=lbmd.LB_FP64, device=device),
            "fp32dev": lbmd.Simulation(cfg, rr, np.zeros_like(rr), precision=lbmd.LB_FP32_DEV, device=device)}
    if envelope:
        rp = np.nextafter(rr, np.inf)
        sims["fp64_ulp"] = lbmd.Simulation(cfg, rp, np.zeros_like(rr), precision=lbmd.LB_FP64, device=device)
    seconds = {k: 0.0 for k in sims}
    series = []
    done = 0
    nx, ny, nz = cfg["shape"]
    while done < steps:
        n = min(sample_every, steps - done)
        for k, s in sims.items():
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            s.run(n, graph=True)
            torch.cuda.synchronize()
            seconds[k] += time.perf_counter() - t0
            s.check()
        done += n
        d64, u64 = fluid_fields(sims["fp64"], vel)
        d32, u32 = fluid_fields(sims["fp32dev"], vel)
        umax = float(u64.abs().max().item())
        r64, r32 = sims["fp64"].beads()["r"], sims["fp32dev"].beads()["r"]
        rho_max, rho_rms = _err(d32, d64)
        u_max, u_rms = _err(u32, u64, umax if umax > 0 else 1.0)
        r_max, r_rms = _err(r32, r64)
        row = dict(step=done, rho_err_max=rho_max, rho_err_rms=rho_rms,
                   rho_dev_max=float(d64.abs().max().item()), u_max=umax,
                   u_err_max_rel=u_max, u_err_rms_rel=u_rms, r_err_max=r_max, r_err_rms=r_rms)
        if envelope:
            de, ue = fluid_fields(sims["fp64_ulp"], vel)
            row["env_rho_max"] = _err(de, d64)[0]
            row["env_u_max_rel"] = _err(ue, u64, umax if umax > 0 else 1.0)[0]
            row["env_r_max"] = _err(sims["fp64_ulp"].beads()["r"], r64)[0]
        series.append(row)
    for s in sims.values():
        s.close()
    cells = nx * ny * nz
    return dict(steps=steps, series=series,
                mlups={k: cells * steps / t / 1e6 for k, t in seconds.items() if k != "fp64_ulp"})


def run_gammas(cfg, steps, sample_every, gammas=None, device="cuda:0"):
    """The study at every friction of the workload (cfg["gammas"])."""
    out = []
    for g in (cfg.get("gammas", (cfg["gamma"],)) if gammas is None else gammas):
        res = run(scaled(cfg, gamma=float(g)), steps, sample_every, device=device)
        res["gamma"] = float(g)
        out.append(res)
        print(f"precision study: gamma {g} done, MLUPS {res['mlups']}", file=sys.stderr, flush=True)
    return out


def main():
    import argparse
    import json
    from .workloads import CONFIGS
    ap = argparse.ArgumentParser(description="FP32 deviation storage against FP64 over time (GPU)")
    ap.add_argument("--workload", default="c1")
    ap.add_argument("--steps", type=int, default=None)
    ap.add_argument("--sample-every", type=int, default=1000)
    a = ap.parse_args()
    cfg = CONFIGS[a.workload]
    print(json.dumps(run_gammas(cfg, a.steps or cfg["steps"], a.sample_every)), flush=True)


if __name__ == "__main__":
    main()


__all__ = ["fluid_fields", "run", "run_gammas"]
