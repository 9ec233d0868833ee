"""torch.autograd interface to the library's hand-written adjoint.

`CoupledRun.apply(r0, gamma, f_drive, sim, start_state, nsteps, K)` runs
`nsteps` coupled steps of `sim` (a one-replica lbmd.Simulation) from
`start_state` (a buffer from sim.get_state()) with the bead positions
replaced by r0 (nb x 3, float64, on the device), friction gamma and pore
force f_drive (0-d float64 tensors), and returns the final positions.  Its
backward runs the library's reverse pass (checkpoints every K steps) and
returns dL/dr0, dL/dgamma, dL/dF_drive.  No derivative is formed by torch
itself: every forward and reverse step runs in the HIP kernels.
"""
import torch


class CoupledRun(torch.autograd.Function):
    @staticmethod
    def forward(ctx, r0, gamma, f_drive, sim, start_state, nsteps, K):
        sim.set_state(start_state)
        sim.beads()["r"].copy_(r0.detach().reshape(-1, 3))
        sim.set_coupling(float(gamma), float(f_drive))
        sim.adjoint_forward(int(nsteps), int(K))
        ctx.sim = sim
        return sim.beads()["r"].clone()

    @staticmethod
    def backward(ctx, grad_r):
        g = ctx.sim.adjoint_backward(grad_r.detach().contiguous())
        nb = grad_r.shape[0]
        return g[2:].view(nb, 3), g[0], g[1], None, None, None, None


def mean_normal_coordinate(sim, start_state, r0, gamma, f_drive, nsteps, K):
    """The translocation observable of the adjoint workload: the mean bead
    coordinate along the wall normal after nsteps coupled steps."""
    r = CoupledRun.apply(r0, gamma, f_drive, sim, start_state, nsteps, K)
    return r[:, sim.cfg["wall_axis"]].mean()
