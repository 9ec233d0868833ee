"""The hand-written adjoint (reverse pass through the coupled step, with
checkpointed recomputation) against the FP64 oracle's forward-mode
derivative of the same discrete map, against central finite differences of
GPU forward runs, and for internal consistency (checkpoint interval, the
autograd path, the state it leaves behind).  Loss: mean bead coordinate
along the wall normal after the run (the translocation observable)."""
import numpy as np
import pytest

from paper_0711_2665_amd.workloads import C4, initial_chain, scaled

pytestmark = pytest.mark.gpu

CFG = scaled(C4, shape=(20, 20, 20), wall_axis=2, wall_pos=10, pore_h=3, nb=12, n_sub=25)
NSTEPS = 12


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _start(orc, cfg):
    """Relaxed chain from the oracle, moved rigidly so that its bead nearest
    the wall sits inside the driven channel, 1.2 spacings in front of the
    wall plane and off the lattice planes (the trilinear weights have kinks
    on them, where the step map has no derivative).  Both sides start from
    these inputs."""
    r, v = initial_chain(cfg)
    o = orc.Oracle(cfg, r, v)
    o.relax(cfg["relax_substeps"], cfg["gamma_relax"])
    r = o.beads()["r"].copy()
    a = cfg["wall_axis"]
    top = int(np.argmax(r[:, a]))
    target = np.array([n / 2.0 for n in cfg["shape"]]) + np.array([0.3137, -0.2718, 0.1931])
    target[a] = cfg["wall_pos"] - 1.2
    return r + (target - r[top])


def _dLdr(cfg):
    g = np.zeros((cfg["nb"], 3))
    g[:, cfg["wall_axis"]] = 1.0 / cfg["nb"]
    return g


def _gpu_loss(sim, st, cfg, nsteps, gamma=None, fdrive=None, dr=None):
    sim.set_state(st)
    if dr is not None:
        sim.beads()["r"].add_(sim.torch.as_tensor(dr, device=sim.device))
    sim.set_coupling(cfg["gamma"] if gamma is None else gamma, cfg["f_drive"] if fdrive is None else fdrive)
    sim.couple_step(nsteps)
    return float(sim.beads()["r"][:, cfg["wall_axis"]].mean())


def _adjoint(sim, st, cfg, nsteps, K):
    sim.set_state(st)
    sim.set_coupling(cfg["gamma"], cfg["f_drive"])
    sim.adjoint_forward(nsteps, K)
    g = sim.adjoint_backward(_dLdr(cfg)).cpu().numpy()
    return g[0], g[1], g[2:].reshape(-1, 3)


# the paper's soft bead-bead and wall LJ (sigma = 1.8, eps = 1e-4): r_c =
# 2^(1/6) 1.8 > 2 reaches wall sites two nodes from the base node
CFG_SOFT = scaled(CFG, sigma=1.8, eps=1e-4, rc=2.0 ** (1.0 / 6.0) * 1.8)


@pytest.mark.parametrize("lj", ["wca", "paper_soft"])
def test_adjoint_fp64_matches_oracle_jvp(orc, lj):
    torch = _torch()
    from paper_0711_2665_amd import lbmd
    cfg = CFG if lj == "wca" else CFG_SOFT
    r0 = _start(orc, cfg)
    v0 = np.zeros_like(r0)
    sim = lbmd.Simulation(cfg, r0)
    st = sim.get_state()
    gg, gf, gr = _adjoint(sim, st, cfg, NSTEPS, 5)
    torch.cuda.synchronize()
    L_gpu = float(sim.beads()["r"][:, 2].mean())
    L, dg = orc.jvp(cfg, r0, v0, NSTEPS, dgamma=1.0)
    _, df = orc.jvp(cfg, r0, v0, NSTEPS, dfdrive=1.0)
    rng = np.random.default_rng(3)
    dirs = [rng.standard_normal(r0.shape) for _ in range(3)]
    dr = [orc.jvp(cfg, r0, v0, NSTEPS, dr0=d)[1] for d in dirs]
    print(f"L gpu {L_gpu:.15g} oracle {L:.15g}; dL/dgamma {gg:.12e} / {dg:.12e}; dL/dF {gf:.12e} / {df:.12e}",
          flush=True)
    assert abs(L_gpu - L) <= 1e-12 * abs(L)
    assert abs(gg - dg) <= 1e-8 * abs(dg), (gg, dg)
    assert abs(gf - df) <= 1e-8 * abs(df), (gf, df)
    assert df != 0.0
    for d, want in zip(dirs, dr):
        got = float((gr * d).sum())
        print(f"  dL/dr0 . dir: adjoint {got:.12e} oracle {want:.12e}", flush=True)
        assert abs(got - want) <= 1e-8 * max(abs(want), np.abs(gr).max()), (got, want)


def test_adjoint_matches_finite_differences_fp64(orc):
    """Central differences of GPU forward runs, h = 1e-6: agreement to 1e-4
    relative."""
    torch = _torch()
    from paper_0711_2665_amd import lbmd
    r0 = _start(orc, CFG)
    sim = lbmd.Simulation(CFG, r0)
    st = sim.get_state()
    gg, gf, gr = _adjoint(sim, st, CFG, NSTEPS, 4)
    h = 1e-6
    fd_g = (_gpu_loss(sim, st, CFG, NSTEPS, gamma=CFG["gamma"] + h) -
            _gpu_loss(sim, st, CFG, NSTEPS, gamma=CFG["gamma"] - h)) / (2 * h)
    fd_f = (_gpu_loss(sim, st, CFG, NSTEPS, fdrive=CFG["f_drive"] + h) -
            _gpu_loss(sim, st, CFG, NSTEPS, fdrive=CFG["f_drive"] - h)) / (2 * h)
    d = np.random.default_rng(4).standard_normal(r0.shape)
    fd_r = (_gpu_loss(sim, st, CFG, NSTEPS, dr=h * d) - _gpu_loss(sim, st, CFG, NSTEPS, dr=-h * d)) / (2 * h)
    got_r = float((gr * d).sum())
    torch.cuda.synchronize()
    print(f"FD vs adjoint: gamma {fd_g:.8e} / {gg:.8e}, F {fd_f:.8e} / {gf:.8e}, r.dir {fd_r:.8e} / {got_r:.8e}",
          flush=True)
    assert abs(gg - fd_g) <= 1e-4 * abs(fd_g)
    assert abs(gf - fd_f) <= 1e-4 * abs(fd_f)
    assert abs(got_r - fd_r) <= 1e-4 * abs(fd_r)


def test_adjoint_independent_of_checkpoint_interval(orc):
    _torch()
    from paper_0711_2665_amd import lbmd
    r0 = _start(orc, CFG)
    sim = lbmd.Simulation(CFG, r0)
    st = sim.get_state()
    a = _adjoint(sim, st, CFG, NSTEPS, 3)
    b = _adjoint(sim, st, CFG, NSTEPS, NSTEPS)
    c = _adjoint(sim, st, CFG, NSTEPS, 7)
    for x, y in ((a, b), (a, c)):
        assert x[0] == y[0] and x[1] == y[1] and np.array_equal(x[2], y[2])


def test_adjoint_leaves_the_forward_end_state(orc):
    torch = _torch()
    from paper_0711_2665_amd import lbmd
    r0 = _start(orc, CFG)
    sim = lbmd.Simulation(CFG, r0)
    st = sim.get_state()
    sim.couple_step(NSTEPS)
    torch.cuda.synchronize()
    want_p, want_r = sim.pops().clone(), sim.beads()["r"].clone()
    for K in (5, NSTEPS):   # recomputed segments; the tape written by the forward pass
        _adjoint(sim, st, CFG, NSTEPS, K)
        torch.cuda.synchronize()
        assert torch.equal(sim.pops(), want_p) and torch.equal(sim.beads()["r"], want_r)
        assert sim.step_count() == NSTEPS
    sim.check()


def test_fp32_deviation_adjoint_close_to_fp64(orc):
    _torch()
    from paper_0711_2665_amd import lbmd
    r0 = _start(orc, CFG)
    s64 = lbmd.Simulation(CFG, r0)
    s32 = lbmd.Simulation(CFG, r0, precision=lbmd.LB_FP32_DEV)
    g64 = _adjoint(s64, s64.get_state(), CFG, NSTEPS, 5)
    g32 = _adjoint(s32, s32.get_state(), CFG, NSTEPS, 5)
    eg = abs(g32[0] - g64[0]) / abs(g64[0])
    ef = abs(g32[1] - g64[1]) / abs(g64[1])
    er = np.abs(g32[2] - g64[2]).max() / np.abs(g64[2]).max()
    print(f"FP32-dev vs FP64 adjoint: gamma {eg:.2e}, F_drive {ef:.2e}, r0 {er:.2e}", flush=True)
    assert eg < 2e-8 and ef < 2e-8 and er < 2e-8   # measured 7.3e-10, 2.5e-11, 1.7e-9


def test_autograd_function_gives_the_adjoint(orc):
    torch = _torch()
    from paper_0711_2665_amd import lbmd
    from paper_0711_2665_amd.adjoint import mean_normal_coordinate
    r0 = _start(orc, CFG)
    sim = lbmd.Simulation(CFG, r0)
    st = sim.get_state()
    direct = _adjoint(sim, st, CFG, NSTEPS, 5)
    r = torch.tensor(r0, dtype=torch.float64, device=sim.device, requires_grad=True)
    g = torch.tensor(CFG["gamma"], dtype=torch.float64, device=sim.device, requires_grad=True)
    f = torch.tensor(CFG["f_drive"], dtype=torch.float64, device=sim.device, requires_grad=True)
    loss = mean_normal_coordinate(sim, st, r, g, f, NSTEPS, 5)
    dr, dg, df = torch.autograd.grad(loss, [r, g, f])
    assert float(dg) == direct[0] and float(df) == direct[1]
    assert np.array_equal(dr.cpu().numpy(), direct[2])


def _jvp_check(orc, cfg, r0, v0, nsteps, K, tag):
    from paper_0711_2665_amd import lbmd
    sim = lbmd.Simulation(cfg, r0, v0)
    st = sim.get_state()
    gg, gf, gr = _adjoint(sim, st, cfg, nsteps, K)
    L, dg = orc.jvp(cfg, r0, v0, nsteps, dgamma=1.0)
    _, df = orc.jvp(cfg, r0, v0, nsteps, dfdrive=1.0)
    d = np.random.default_rng(5).standard_normal(r0.shape)
    _, dr = orc.jvp(cfg, r0, v0, nsteps, dr0=d)
    got = float((gr * d).sum())
    print(f"{tag}: dL/dgamma {gg:.12e} / {dg:.12e}; dL/dF {gf:.12e} / {df:.12e}; dL/dr0.d {got:.12e} / {dr:.12e}",
          flush=True)
    assert abs(gg - dg) <= 1e-8 * abs(dg), (gg, dg)
    assert abs(gf - df) <= 1e-8 * abs(df), (gf, df)
    assert abs(got - dr) <= 1e-8 * max(abs(dr), np.abs(gr).max()), (got, dr)
    return sim


def test_adjoint_400_bead_chain_matches_oracle_jvp(orc):
    """A 400-bead chain (the chain length of the 128^3 workload) with noise
    and bending: the reversed sub-cycle runs over 25 workgroups with the
    neighbour lists built at every reversed step."""
    _torch()
    cfg = scaled(C4, shape=(48, 48, 48), wall_pos=24, nb=400, init_seed=21)
    r, v = initial_chain(cfg)
    o = orc.Oracle(cfg, r, v)
    o.relax(cfg["relax_substeps"], cfg["gamma_relax"])
    # the relaxed coil (bead 0 in front of the pore), moved off the lattice
    # planes, where the trilinear weights have kinks
    r0 = o.beads()["r"] + np.array([0.3137, -0.2718, 0.1931])
    _jvp_check(orc, cfg, r0, np.zeros_like(r0), NSTEPS, 5, "400 beads")


def test_adjoint_all_pairs_when_the_lists_do_not_hold(orc):
    """Beads drifting 1.5 spacings per step along the wall leave half the
    list skin inside every step, so the reversed sub-steps scan all pairs:
    the derivative still matches the oracle's."""
    _torch()
    r0 = _start(orc, CFG)
    v0 = np.zeros_like(r0)
    v0[:, 0] = 1.5
    from paper_0711_2665_amd import lbmd
    probe = lbmd.Simulation(CFG, r0, v0)
    probe.couple_step(1)
    moved = np.abs(probe.beads()["r"].cpu().numpy() - r0).max()
    assert moved > 0.6, moved                 # beyond half the skin within the first step
    _jvp_check(orc, CFG, r0, v0, NSTEPS, 5, "drifting chain")
