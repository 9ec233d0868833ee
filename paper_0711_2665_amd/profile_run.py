"""Workload driver for rocprofv3 runs of the LB sweep.

    python -m paper_0711_2665_amd.profile_run --workload c3 --precision fp32dev --steps 5 --copy-mib 1024

Runs `steps` fluid-only sweeps of the workload's lattice (the same kernel the
coupled step launches for the nodes without bead force) and then a plain
device-to-device copy of `copy_mib` MiB, whose counter readings calibrate the
HBM byte counters (FETCH_SIZE, WRITE_SIZE) against a known transfer.
"""
import argparse

import torch

from . import lbmd
from .workloads import CONFIGS, scaled


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="c3")
    ap.add_argument("--precision", default="fp32dev", choices=["fp32dev", "fp64"])
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--copy-mib", type=int, default=1024)
    a = ap.parse_args()
    cfg = scaled(CONFIGS[a.workload], nb=0)
    prec = lbmd.LB_FP32_DEV if a.precision == "fp32dev" else lbmd.LB_FP64
    sim = lbmd.Simulation(cfg, precision=prec)
    sim.lb_step(a.steps)
    torch.cuda.synchronize()
    sim.check()
    n = a.copy_mib * 2 ** 20 // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    print(f"profile_run: {a.steps} sweeps of {cfg['shape']} ({a.precision}), copy of {a.copy_mib} MiB", flush=True)


if __name__ == "__main__":
    main()
