"""Workload driver for rocprofv3 counter runs of the LB sweep.

    python -m paper_0711_2665_amd.profile_run --workload c3 --precision fp32dev --steps 5 \
        --copy-mib 1024 --meta /tmp/lb_sweep_meta.json

Builds the workload's lattice without beads (with --fluid-kT, a fluctuating
fluid: the sweep variant that draws the fluid noise) and, for every sweep
layout the autotuner chooses from, runs `steps` fluid-only sweeps (the kernel the
coupled step launches for the nodes without bead force); then a plain
device-to-device copy of `copy_mib` MiB, whose counter readings calibrate
the HBM byte counters (FETCH_SIZE, WRITE_SIZE) against a known transfer.
Writes what the summary needs (layouts in launch order, kernel source hash,
node counts, algorithmic bytes, copy size) to --meta.
"""
import argparse
import json

import torch

from . import lbmd
from .build import kernel_source_hash
from .workloads import CONFIGS, scaled

# the autotuner's candidates (tile nodes, order, grid, cap)
LAYOUTS = [(t, o, 0, 0) for t in (256, 512, 1024, 2048) for o in (0, 1)] + \
    [(t, 0, g, 0) for t in (256, 512) for g in (256, 384, 512, 768, 1024, 2048)] + \
    [(t, 0, 0, k) for t in (256, 512, 1024) for k in (2, 3, 4)]


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="c3")
    ap.add_argument("--precision", default="fp32dev", choices=["fp32dev", "fp64"])
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--copy-mib", type=int, default=1024)
    ap.add_argument("--meta", default=None)
    ap.add_argument("--fluid-kT", type=float, default=0.0,
                    help="thermal energy of a fluctuating fluid (selects the sweep that draws its noise)")
    a = ap.parse_args()
    cfg = scaled(CONFIGS[a.workload], nb=0, fluid_kT=a.fluid_kT)
    prec = lbmd.LB_FP32_DEV if a.precision == "fp32dev" else lbmd.LB_FP64
    sim = lbmd.Simulation(cfg, precision=prec)
    for lay in LAYOUTS:
        sim.sweep_config(*lay)
        sim.lb_step(a.steps)
    torch.cuda.synchronize()
    sim.check()
    n = a.copy_mib * 2 ** 20 // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    nx, ny, nz = cfg["shape"]
    nfluid = int(((sim.flags() & 1) == 0).sum().item())
    es = 4 if a.precision == "fp32dev" else 8
    meta = dict(workload=a.workload, precision=a.precision, shape=[nx, ny, nz], nodes=nx * ny * nz, nfluid=nfluid,
                algorithmic_bytes_per_launch=nfluid * (2 * 19 * es + 1) + (nx * ny * nz - nfluid),
                layouts=[dict(tile_nodes=t, order=o, grid=g, cap=k) for t, o, g, k in LAYOUTS],
                kernel_source_hash=kernel_source_hash(), copy_bytes=n * 4, sweeps=a.steps, fluid_kT=a.fluid_kT)
    if a.meta:
        with open(a.meta, "w") as fh:
            json.dump(meta, fh)
    print(f"profile_run: {a.steps} sweeps of {cfg['shape']} ({a.precision}) in each of {len(LAYOUTS)} layouts, "
          f"copy of {a.copy_mib} MiB", flush=True)


if __name__ == "__main__":
    main()
