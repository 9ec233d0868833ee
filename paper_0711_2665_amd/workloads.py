"""Seeded synthetic workloads: run descriptions and initial polymer coils.

This module generates inputs only.  It holds none of the method's arithmetic
(no lattice-Boltzmann update, no force law, no integrator), so both the GPU
path and the CPU oracle used by the tests can start from the same inputs.

Geometry and parameters follow the numerical set-up of Sec. 4 of the paper
(a box with one wall plane and a square pore at its centre, periodic on all
axes; a bead-spring chain that starts as a self-avoiding walk entirely on one
side of the wall with its first bead at the pore entrance), at the sizes of
the workloads this library is measured on.
"""
import math

import numpy as np

# Shared physical parameters (lattice units): tau = 1 (nu = 1/6), unit
# density, harmonic bonds k = 100, r0 = 1, bending kappa = 10, purely
# repulsive LJ eps = sigma = 1 cut at 2^(1/6), friction gamma = 0.1,
# kT = 1e-4, pore force 0.02, 100 MD sub-steps per LB step.
BASE = dict(
    tau=1.0, g=(0.0, 0.0, 0.0), mass=1.0, k_bond=100.0, r0=1.0, kappa=10.0,
    eps=1.0, sigma=1.0, rc=2.0 ** (1.0 / 6.0), gamma=0.1, kT=1e-4, f_drive=0.02,
    n_sub=100, seed=20071127, replica=0, relax_substeps=2000, gamma_relax=1.0,
)


def _cfg(**kw):
    c = dict(BASE)
    c.update(kw)
    return c


# Small parity case: 32^3, wall normal to z at z = 16 with a 3x3 pore, a
# 20-bead chain, 200 steps.
C0 = _cfg(name="parity_32cube_20beads", shape=(32, 32, 32), wall_axis=2, wall_pos=16,
          pore_h=3, nb=20, steps=200, init_seed=11)
# Single-run FP32 vs FP64 case: 128^3, wall at z = 64, 5x5 pore, 400 beads.
C1 = _cfg(name="single_128cube_400beads", shape=(128, 128, 128), wall_axis=2, wall_pos=64,
          pore_h=5, nb=400, steps=10000, init_seed=12, gammas=(0.05, 0.1, 0.2))
# Large single run: 512x256x256 (33.5M nodes), wall normal to x at x = 256
# with a 7x7 pore, 8000 beads, 2000 steps.
C3 = _cfg(name="large_512x256x256_8000beads", shape=(512, 256, 256), wall_axis=0, wall_pos=256,
          pore_h=7, nb=8000, steps=2000, init_seed=13)
# Gradient case: 64^3, wall at z = 32, 3x3 pore, 100 beads, 2000 steps.
C4 = _cfg(name="adjoint_64cube_100beads", shape=(64, 64, 64), wall_axis=2, wall_pos=32,
          pore_h=3, nb=100, steps=2000, init_seed=14, checkpoint_every=100)

# The paper's bead LJ (Sec. 2: sigma = 1.8, eps = 1e-4, cut-off 2^(1/6) sigma)
# with the bond rest length at the cut-off (the paper gives none), so the
# truncated LJ does not act along a bond at rest; and the multiple-time-step
# sub-cycle with M = 5 outer steps of 20 sub-steps (Sec. 2).
PAPER_LJ = dict(sigma=1.8, eps=1e-4, rc=2.0 ** (1.0 / 6.0) * 1.8, r0=2.0 ** (1.0 / 6.0) * 1.8)
C3M = _cfg(name="large_512x256x256_8000beads_paper_lj_mts5x20", shape=(512, 256, 256), wall_axis=0,
           wall_pos=256, pore_h=7, nb=8000, steps=2000, init_seed=13, mts_outer=5, **PAPER_LJ)

CONFIGS = {"c0": C0, "c1": C1, "c3": C3, "c4": C4, "c3m": C3M}


def ensemble_configs(n_replicas=64, seed=15, steps=5000):
    """Uneven ensemble: cubic edge from {48,64,80,96}, chain length from
    {50,100,200,500}, pore side from {3,4,5}, pore force ~ U(0.01, 0.04), one
    noise seed per replica; wall normal to z at the mid-plane."""
    rng = np.random.default_rng(seed)
    out = []
    for k in range(n_replicas):
        edge = int(rng.choice([48, 64, 80, 96]))
        nb = int(rng.choice([50, 100, 200, 500]))
        h = int(rng.choice([3, 4, 5]))
        fd = float(rng.uniform(0.01, 0.04))
        out.append(_cfg(name=f"replica{k}", shape=(edge, edge, edge), wall_axis=2, wall_pos=edge // 2,
                        pore_h=h, nb=nb, f_drive=fd, seed=int(rng.integers(1, 2**31)), replica=k,
                        steps=steps, init_seed=int(rng.integers(1, 2**31))))
    return out


def pore_bounds(cfg):
    """Inclusive pore block [lo, hi] on each transverse axis (centred)."""
    a = cfg["wall_axis"]
    tn = [t for t in range(3) if t != a]
    lo = [cfg["shape"][t] // 2 - cfg["pore_h"] // 2 for t in tn]
    return tn, lo, [l + cfg["pore_h"] - 1 for l in lo]


def initial_chain(cfg, seed=None, max_tries=60):
    """Seeded off-lattice self-avoiding walk (bond length r0, no two beads
    closer than sigma under the periodic minimum image) lying on the cis side
    of the wall (normal coordinate within [wall - L + 1.2, wall - 1.2]), with
    bead 0 one lattice spacing in front of the pore centre.  The walk is
    persistent (small turning angles) so that the coil stores little bending
    energy before the MD pre-relaxation.  Returns (r, v) as (nb, 3) float64
    arrays, v = 0."""
    nb = cfg["nb"]
    if nb == 0:
        return np.zeros((0, 3)), np.zeros((0, 3))
    rng = np.random.default_rng(cfg.get("init_seed", 0) if seed is None else seed)
    L = np.array(cfg["shape"], dtype=np.float64)
    a = cfg["wall_axis"]
    b0 = cfg["r0"]
    sig = cfg["sigma"]
    tn, lo, hi = pore_bounds(cfg)
    start = np.zeros(3)
    for k, t in enumerate(tn):
        start[t] = lo[k] + (cfg["pore_h"] - 1) / 2.0
    wall = float(cfg["wall_pos"])
    start[a] = wall - 1.0
    nmin, nmax = wall - L[a] + 1.2, wall - 1.2

    cell = {}

    def key(p):
        w = np.mod(p, L)
        return tuple(int(x) for x in np.floor(w))

    def too_close(p, upto):
        kx = key(p)
        for dx in (-1, 0, 1):
            for dy in (-1, 0, 1):
                for dz in (-1, 0, 1):
                    kk = ((kx[0] + dx) % int(L[0]), (kx[1] + dy) % int(L[1]), (kx[2] + dz) % int(L[2]))
                    for j in cell.get(kk, ()):
                        if j >= upto - 1:
                            continue
                        d = p - pos[j]
                        d -= L * np.floor(d / L + 0.5)
                        if d @ d < (sig * 0.999) ** 2:
                            return True
        return False

    pos = np.zeros((nb, 3))
    pos[0] = start
    cell.setdefault(key(start), []).append(0)
    direction = np.zeros(3)
    direction[a] = -1.0
    k = 1
    while k < nb:
        placed = False
        for attempt in range(max_tries):
            spread = 0.25 + 0.05 * attempt
            dnew = direction + spread * rng.standard_normal(3)
            dnew /= np.linalg.norm(dnew)
            p = pos[k - 1] + b0 * dnew
            if not (nmin <= p[a] <= nmax):
                continue
            if too_close(p, k):
                continue
            pos[k] = p
            cell.setdefault(key(p), []).append(k)
            direction = dnew
            placed = True
            break
        if placed:
            k += 1
            continue
        # dead end: step back a few beads and try again
        back = min(k - 1, 5)
        for j in range(k - back, k):
            cell[key(pos[j])].remove(j)
        k -= back
        if k > 1:
            d = pos[k - 1] - pos[k - 2]
            direction = d / np.linalg.norm(d)
        else:
            direction = np.zeros(3)
            direction[a] = -1.0
    return pos, np.zeros((nb, 3))


def scaled(cfg, **kw):
    """Copy of a workload with some fields replaced (smaller parity cases)."""
    c = dict(cfg)
    c.update(kw)
    return c


def geometry_summary(cfg):
    tn, lo, hi = pore_bounds(cfg)
    return dict(axis=cfg["wall_axis"], plane=cfg["wall_pos"], pore=[(l, h) for l, h in zip(lo, hi)])


def cells(cfg):
    nx, ny, nz = cfg["shape"]
    return nx * ny * nz


def mlups(cfg, seconds_per_step):
    return cells(cfg) / seconds_per_step / 1e6


__all__ = ["BASE", "C0", "C1", "C3", "C4", "C3M", "PAPER_LJ", "CONFIGS", "ensemble_configs", "initial_chain",
           "pore_bounds", "scaled", "cells", "mlups", "geometry_summary", "math"]
