"""The adjoint on the 64^3 / 100-bead gradient workload at a horizon where
finite differences no longer resolve the derivative (the trajectories cross
trilinear-interpolation kinks inside the difference interval): the FP64
adjoint must still equal the oracle's forward-mode derivative of the same
discrete map."""
import numpy as np
import pytest

from paper_0711_2665_amd.workloads import C4, initial_chain

pytestmark = pytest.mark.gpu


def test_adjoint_c4_50_steps_matches_oracle_jvp(orc):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_0711_2665_amd import lbmd
    cfg, T = C4, 50
    r, v = initial_chain(cfg)
    o = orc.Oracle(cfg, r, v)
    o.relax(cfg["relax_substeps"], cfg["gamma_relax"])
    r0 = o.beads()["r"]
    v0 = np.zeros_like(r0)
    sim = lbmd.Simulation(cfg, r0)
    dLdr = np.zeros_like(r0)
    dLdr[:, cfg["wall_axis"]] = 1.0 / cfg["nb"]
    sim.adjoint_forward(T, 10)
    g = sim.adjoint_backward(dLdr).cpu().numpy()
    _, dg = orc.jvp(cfg, r0, v0, T, dgamma=1.0)
    d = np.random.default_rng(11).standard_normal(r0.shape)
    _, dd = orc.jvp(cfg, r0, v0, T, dr0=d)
    got = float((g[2:].reshape(-1, 3) * d).sum())
    print(f"c4 {T} steps: dL/dgamma adjoint {g[0]:.12e} oracle {dg:.12e}; "
          f"dL/dr0.dir adjoint {got:.12e} oracle {dd:.12e}", flush=True)
    assert abs(g[0] - dg) <= 1e-8 * abs(dg)
    assert abs(got - dd) <= 1e-8 * abs(dd)
