"""GPU parity at the full size of the large single-run workload (512 x 256 x
256 lattice, 33.5 M nodes, wall normal to x with a 7 x 7 pore, one
8000-bead chain) in the launch configuration the benchmark times: the sweep
layout chosen by the coupled-step autotuner and steps replayed from the
captured two-step graph.  The oracle runs the same two coupled steps on the
host (about 10 GB of FP64 populations); every population of every fluid node
and every bead field is compared.

- FP64 storage, no noise and no bending (no transcendental functions on the
  path): bit for bit.
- FP32 deviation storage, the workload as benchmarked (noise and bending
  on): |f - (f64 - w)| < 1e-8 and |r - r64| < 5e-11 (about ten times the
  measured 7.3e-10 and 4.9e-12).

The fluctuating-fluid leg (fluid kT = bead kT) in both storages, and both
checks above also for the same lattice and chain with the paper's bead LJ under the
multiple-time-step cycle (5 outer x 20 inner sub-steps), and for the
benchmarked ensemble (64 uneven replicas, 28.3 M nodes, 14050 beads, one
context) on a sample of replicas that includes the largest lattice and the
longest chains; there the oracle runs each sampled replica alone.
"""
import numpy as np
import pytest

from paper_0711_2665_amd.workloads import C3, C3M, ensemble_configs, initial_chain, scaled

pytestmark = pytest.mark.gpu

RELAX = 300


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _oracle_start(orc, cfg):
    """The oracle relaxes the seeded coil (MD only); both sides start from
    its positions with v = 0 and the fluid at rest."""
    r, v = initial_chain(cfg)
    o = orc.Oracle(cfg, r, v)
    o.relax(RELAX, cfg["gamma_relax"])
    rr = o.beads()["r"].copy()
    del o
    return orc.Oracle(cfg, rr, np.zeros_like(rr)), rr


def _gpu_two_steps(cfg, rr, precision):
    torch = _torch()
    from paper_0711_2665_amd import lbmd
    s = lbmd.Simulation(cfg, rr, None, precision=precision)
    tune = s.autotune(reps=2, coupled=True)         # restores the state it times
    s.run(2, graph=True)
    torch.cuda.synchronize()
    s.check()
    print(f"full size {cfg['name']}: layout {tune}", flush=True)
    return s


@pytest.mark.parametrize("base", [C3, C3M], ids=["uniform", "mts_paper_lj"])
def test_full_size_fp64_bitwise(orc, base):
    from paper_0711_2665_amd import lbmd
    cfg = scaled(base, kT=0.0, kappa=0.0)
    o, rr = _oracle_start(orc, cfg)
    s = _gpu_two_steps(cfg, rr, lbmd.LB_FP64)
    o.couple_step(2)
    fluid = (o.flags() == 0).reshape(-1)
    op = o.pops().reshape(19, -1)
    gp = s.pops().reshape(19, -1)
    ndiff = 0
    for i in range(19):
        ndiff += int((gp[i].cpu().numpy()[fluid] != op[i][fluid]).sum())
    sb = {k: t.cpu().numpy() for k, t in s.beads().items()}
    ob = o.beads()
    bdiff = {k: int((sb[k] != ob[k]).sum()) for k in ("r", "v", "up", "J")}
    print(f"full size FP64, 2 steps: populations differing {ndiff} of {19 * int(fluid.sum())}, beads {bdiff}",
          flush=True)
    assert ndiff == 0
    assert all(v == 0 for v in bdiff.values()), bdiff
    assert np.abs(ob["r"] - rr).max() > 1e-3                      # the chain moved
    s.close()


@pytest.mark.parametrize("cfg", [C3, C3M], ids=["uniform", "mts_paper_lj"])
def test_full_size_fp32_deviation_as_benchmarked(orc, cfg):
    from paper_0711_2665_amd import lbmd
    o, rr = _oracle_start(orc, cfg)
    s = _gpu_two_steps(cfg, rr, lbmd.LB_FP32_DEV)
    o.couple_step(2)
    _, w, _ = orc.tables()
    fluid = (o.flags() == 0).reshape(-1)
    op = o.pops().reshape(19, -1)
    gp = s.pops().reshape(19, -1)
    err = 0.0
    dev = 0.0
    for i in range(19):
        fo = op[i][fluid] - w[i]
        err = max(err, float(np.abs(gp[i].double().cpu().numpy()[fluid] - fo).max()))
        dev = max(dev, float(np.abs(fo).max()))
    rg, ro = s.beads()["r"].cpu().numpy(), o.beads()["r"]
    print(f"full size FP32 deviations, 2 steps: |f - f64|_max {err:.3e} (max |f - w| {dev:.3e}), "
          f"|r - r64|_max {np.abs(rg - ro).max():.3e}", flush=True)
    assert dev > 1e-4                                             # the chain forced the fluid
    assert err < 1e-8                      # measured 7.3e-10 (c3), 6.2e-10 (c3m)
    assert np.abs(rg - ro).max() < 5e-11   # measured 4.9e-12, 2.4e-12
    s.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32dev"])
def test_full_size_fluctuating_fluid(orc, precision):
    """The benchmark's fluctuating-fluid leg (fluid kT = bead kT): FP64
    within 1e-12 relative (the device's and the host's log and sin/cos may
    differ in the last bit).  FP32 deviation storage draws the fluid normals
    in FP32; the Box-Muller radius sqrt(-2 ln u) is then off by at most
    4e-7 (above u = 1 - 2^-6 it comes from the exact complement 1 - u; below,
    the FP32 u is within 2^-25 of the uniform and the radius at least
    sqrt(2 * 2^-6), plus the hardware log2's own error), and a radius error
    moves populations by at most that much times w_i sum_k |e_ki| a_k / b_k
    (a_k the mode's noise amplitude at the largest density): the bound of
    the FP32 test, plus 16 FP32 ulps of the largest deviation for the
    storage and the collision."""
    from paper_0711_2665_amd import lbmd
    cfg = scaled(C3, fluid_kT=C3["kT"])
    o, rr = _oracle_start(orc, cfg)
    s = _gpu_two_steps(cfg, rr, lbmd.LB_FP64 if precision == "fp64" else lbmd.LB_FP32_DEV)
    o.couple_step(2)
    _, w, _ = orc.tables()
    fluid = (o.flags() == 0).reshape(-1)
    op = o.pops().reshape(19, -1)
    gp = s.pops().reshape(19, -1)
    err = dev = fmax = 0.0
    rho = np.zeros(int(fluid.sum()))
    for i in range(19):
        rho += op[i][fluid]
        fo = op[i][fluid]
        fg = gp[i].double().cpu().numpy()[fluid]
        if precision == "fp32dev":
            fo = fo - w[i]
        err = max(err, float(np.abs(fg - fo).max()))
        dev = max(dev, float(np.abs(op[i][fluid] - w[i]).max()))
        fmax = max(fmax, float(np.abs(fo).max()))
    er = float(np.abs(s.beads()["r"].cpu().numpy() - o.beads()["r"]).max())
    print(f"full size fluctuating fluid {precision}, 2 steps: |f - f_oracle|_max {err:.3e} "
          f"(max |f - w| {dev:.3e}, max |f| {fmax:.3e}), |r - r_oracle|_max {er:.3e}", flush=True)
    assert dev > 1e-3                                            # the noise is on
    if precision == "fp64":
        assert err <= 1e-12 * fmax
        assert er <= 1e-12 * float(np.abs(rr).max())
    else:
        E = orc.mode_basis()
        b = (w[None, :] * E * E).sum(1)
        om = 1.0 / cfg["tau"]
        amp = np.sqrt(3.0 * rho.max() * cfg["fluid_kT"] * (1.0 - (1.0 - om) ** 2) * b[4:])
        tail = 4e-7 * (w * (np.abs(E[4:, :]) * (amp / b[4:])[:, None]).sum(0)).max()
        print(f"FP32 noise-tail bound {tail:.3e}", flush=True)
        assert err <= tail + 16 * 2.0 ** -24 * dev             # + 16 FP32 ulps of the largest deviation
        assert er < 1e-9                                         # measured 7.4e-11
    s.close()


def _sample(cfgs):
    """Replicas to compare: the largest lattice, the longest chain, the
    shortest chain and the first replica."""
    size = [c["shape"][0] * c["shape"][1] * c["shape"][2] for c in cfgs]
    pick = {0, int(np.argmax(size)), int(np.argmax([c["nb"] for c in cfgs])), int(np.argmin([c["nb"] for c in cfgs]))}
    return sorted(pick)


@pytest.mark.parametrize("precision", ["fp64_bitwise", "fp32dev_as_benchmarked"])
def test_full_size_ensemble_sampled_replicas(orc, precision):
    torch = _torch()
    from paper_0711_2665_amd import lbmd
    cfgs = ensemble_configs(64)
    if precision == "fp64_bitwise":
        cfgs = [scaled(c, kT=0.0, kappa=0.0) for c in cfgs]
    prec = lbmd.LB_FP64 if precision == "fp64_bitwise" else lbmd.LB_FP32_DEV
    rr = []
    for c in cfgs:                                   # the oracle relaxes every coil
        r, v = initial_chain(c)
        o = orc.Oracle(c, r, v)
        o.relax(RELAX, c["gamma_relax"])
        rr.append(o.beads()["r"].copy())
        del o
    ens = lbmd.Ensemble(cfgs, rr, precision=prec)
    tune = ens.autotune(reps=2, coupled=True)
    ens.run(2, graph=True)
    torch.cuda.synchronize()
    ens.check()
    print(f"full-size ensemble {precision}: layout {tune}", flush=True)
    _, w, _ = orc.tables()
    for k in _sample(cfgs):
        o = orc.Oracle(cfgs[k], rr[k], np.zeros_like(rr[k]))
        o.couple_step(2)
        fluid = (o.flags() == 0).reshape(-1)
        op = o.pops().reshape(19, -1)[:, fluid]
        gp = ens.pops(k).reshape(19, -1).double().cpu().numpy()[:, fluid]
        gb = {n: t.cpu().numpy() for n, t in ens.beads(k).items()}
        ob = o.beads()
        tag = f"replica {k} ({cfgs[k]['shape']}, {cfgs[k]['nb']} beads)"
        if precision == "fp64_bitwise":
            bd = {n: int((gb[n] != ob[n]).sum()) for n in ("r", "v", "up", "J")}
            print(f"{tag}: populations differing {int((gp != op).sum())}, beads {bd}", flush=True)
            assert np.array_equal(gp, op)
            assert all(v == 0 for v in bd.values()), (k, bd)
        else:
            err = float(np.abs(gp - (op - w[:, None])).max())
            er = float(np.abs(gb["r"] - ob["r"]).max())
            print(f"{tag}: |f - f64|_max {err:.3e}, |r - r64|_max {er:.3e}", flush=True)
            assert err < 1e-8 and er < 5e-11, (k, err, er)   # measured <= 5.6e-10, 3.9e-12
    ens.close()
