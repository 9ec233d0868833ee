"""GPU: beads coupled to a fluctuating fluid at the same temperature come to
that temperature, and so does the fluid (Sec. 2: the fluid's stochastic
terms and the beads' noise are set by one kT, so that the bead and fluid
temperatures agree).  32 replicas of a periodic 16^3 box with a 20-bead
chain (no wall, no field) in one ensemble, FP64 storage: after equilibration
the bead kinetic temperature <v_a^2> m and the fluid's <j_a^2 / rho> over
the nodes both equal kT within 3%.  The measured values are printed beside
those of the same system with an athermal fluid."""
import numpy as np
import pytest

from paper_0711_2665_amd.workloads import C0, initial_chain, scaled

pytestmark = pytest.mark.gpu

KT = 1e-4


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _temperatures(fluid_kT, nrep=32, samples=300, every=10):
    torch = _torch()
    from paper_0711_2665_amd import lbmd
    cfgs, r0s = [], []
    for k in range(nrep):
        base = scaled(C0, name=f"t{k}", shape=(16, 16, 16), nb=20, wall_pos=8, init_seed=40 + k)
        r0s.append(initial_chain(base)[0])
        cfgs.append(scaled(base, wall_axis=-1, wall_pos=0, pore_h=0, kT=KT, fluid_kT=fluid_kT, kappa=1.0,
                           k_bond=10.0, seed=900 + k, replica=k))
    ens = lbmd.Ensemble(cfgs, r0s, precision=lbmd.LB_FP64)
    ens.relax(2000, 1.0)
    ens.run(600, graph=True)
    vel = torch.tensor(lbmd.VELOCITIES, dtype=torch.float64, device="cuda:0")
    vb = torch.zeros((), dtype=torch.float64, device="cuda:0")
    jf = torch.zeros((), dtype=torch.float64, device="cuda:0")
    for _ in range(samples):
        ens.run(every, graph=True)
        for k in range(nrep):
            v = ens.beads(k)["v"]
            vb += (v * v).mean()
            f = ens.pops(k).reshape(19, -1)
            rho = f.sum(0)
            j = vel.t() @ f
            jf += ((j * j).sum(0) / rho).mean() / 3.0
    torch.cuda.synchronize()
    ens.check()
    ens.close()
    n = samples * nrep
    return float(vb.item()) / n / KT, float(jf.item()) / n / KT


def test_beads_and_fluid_share_the_temperature():
    tb, tf = _temperatures(KT)
    tb0, tf0 = _temperatures(0.0)
    print(f"fluctuating fluid: bead T / kT = {tb:.4f}, fluid T / kT = {tf:.4f}; "
          f"athermal fluid: bead T / kT = {tb0:.4f}, fluid T / kT = {tf0:.4f}", flush=True)
    assert abs(tb - 1.0) < 0.03
    assert abs(tf - 1.0) < 0.03
    # an athermal fluid is heated only by the beads, far below kT
    assert tf0 < 0.5
