"""GPU parity of the nearest-grid-point bead/lattice transfer (the paper's
own coupling, Sec. 2): u_p from the node nearest to the bead, the impulse
back to that node alone.  Against the FP64 oracle through the C ABI: bitwise
without transcendental functions (also with the multiple-time-step cycle),
within 1e-12 or the chaos envelope with noise and bending, FP32 within its
bound, and replicas of either transfer in one ensemble equal to their runs
alone."""
import numpy as np
import pytest

from paper_0711_2665_amd.workloads import C0, PAPER_LJ, initial_chain, scaled

pytestmark = pytest.mark.gpu

TOL64 = 1e-12


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    den = np.abs(b).max()
    return float(np.abs(a - b).max() / (den if den > 0 else 1.0))


def _start(orc, cfg, precision=None):
    from paper_0711_2665_amd import lbmd
    r, v = initial_chain(cfg)
    o = orc.Oracle(cfg, r, v)
    o.relax(cfg["relax_substeps"], cfg["gamma_relax"])
    rr = o.beads()["r"]
    o = orc.Oracle(cfg, rr, np.zeros_like(rr))
    s = lbmd.Simulation(cfg, rr, None, precision=lbmd.LB_FP64 if precision is None else precision)
    return o, s


@pytest.mark.parametrize("extra", [{}, dict(mts_outer=5, **PAPER_LJ)], ids=["uniform", "mts_paper_lj"])
def test_ngp_coupled_steps_bitwise(orc, extra):
    torch = _torch()
    cfg = scaled(C0, kT=0.0, kappa=0.0, coupling=1, **extra)
    o, s = _start(orc, cfg)
    o.couple_step(6)
    s.couple_step(6)
    torch.cuda.synchronize()
    s.check()
    fluid = o.flags() == 0
    a, b = s.pops().cpu().numpy()[:, fluid], o.pops()[:, fluid]
    sb = {k: t.cpu().numpy() for k, t in s.beads().items()}
    ob = o.beads()
    print("ngp", extra, "6 steps: pops differing", int((a != b).sum()),
          {k: int((sb[k] != ob[k]).sum()) for k in ("r", "v", "up", "J")}, flush=True)
    assert np.array_equal(a, b)
    for k in ("r", "v", "up", "J"):
        assert np.array_equal(sb[k], ob[k]), k
    go, oo = s.observables().cpu().numpy(), o.observables()
    for k in list(range(16)) + [22]:
        assert abs(go[k] - oo[k]) <= TOL64 * max(1.0, abs(oo[k])), (k, go[k], oo[k])
    # at most one node per bead carries bead force
    assert s.diagnostics()["forced_total"] <= 6 * cfg["nb"]


def test_ngp_with_noise_and_bending_fp64(orc):
    torch = _torch()
    cfg = scaled(C0, coupling=1)
    o, s = _start(orc, cfg)
    r0 = o.beads()["r"]
    o2 = orc.Oracle(cfg, np.nextafter(r0, np.inf), np.zeros_like(r0))
    fluid = o.flags() == 0
    done = 0
    for target in (1, 10, 30):
        o.couple_step(target - done)
        o2.couple_step(target - done)
        s.couple_step(target - done)
        done = target
        torch.cuda.synchronize()
        ob, ob2 = o.beads(), o2.beads()
        sb = {k: t.cpu().numpy() for k, t in s.beads().items()}
        rows = {"pops": (_rel(s.pops().cpu().numpy()[:, fluid], o.pops()[:, fluid]),
                         _rel(o2.pops()[:, fluid], o.pops()[:, fluid]))}
        for k in ("r", "v", "up", "J"):
            rows[k] = (_rel(sb[k], ob[k]), _rel(ob2[k], ob[k]))
        print(f"ngp c0 step {target}: " + ", ".join(f"{k} gpu {g:.1e} / envelope {e:.1e}"
                                                   for k, (g, e) in rows.items()), flush=True)
        for k, (g, e) in rows.items():
            bound = TOL64 if target == 1 else max(TOL64, 100 * e)
            assert g <= bound, (target, k, g, e)
    s.check()


def test_ngp_fp32_deviation_error(orc):
    torch = _torch()
    from paper_0711_2665_amd import lbmd
    cfg = scaled(C0, coupling=1)
    o, s = _start(orc, cfg, precision=lbmd.LB_FP32_DEV)
    fluid = o.flags() == 0
    _, w, _ = orc.tables()
    o.couple_step(30)
    s.couple_step(30)
    torch.cuda.synchronize()
    fo = o.pops()[:, fluid] - w[:, None]
    fs = s.pops().double().cpu().numpy()[:, fluid]
    err_f = np.abs(fs - fo).max()
    rg, ro = s.beads()["r"].cpu().numpy(), o.beads()["r"]
    print(f"fp32-dev ngp c0 30 steps: |f - f64|_max {err_f:.3e}, |r - r64|_max {np.abs(rg - ro).max():.3e}",
          flush=True)
    assert err_f < 3e-9                    # measured 3.0e-10
    assert np.abs(rg - ro).max() < 3e-8     # measured 2.0e-9


def test_ngp_and_trilinear_replicas_in_one_ensemble():
    torch = _torch()
    from paper_0711_2665_amd import lbmd
    cfgs = [
        scaled(C0, name="n0", shape=(16, 12, 20), wall_axis=2, wall_pos=10, pore_h=3, nb=12, seed=11, replica=0,
               init_seed=5, coupling=1),
        scaled(C0, name="n1", shape=(20, 16, 16), wall_axis=0, wall_pos=10, pore_h=4, nb=20, seed=12, replica=1,
               init_seed=6),
        scaled(C0, name="n2", shape=(24, 24, 24), wall_axis=2, wall_pos=12, pore_h=3, nb=33, seed=13, replica=3,
               init_seed=7, coupling=1),
    ]
    r0s = [initial_chain(c)[0] for c in cfgs]
    ens = lbmd.Ensemble(cfgs, r0s, precision=lbmd.LB_FP32_DEV)
    ens.relax(300, 1.0)
    for n in (3, 4):
        ens.run(n, graph=True)
        ens.observables()
    torch.cuda.synchronize()
    ens.check()
    for k, cfg in enumerate(cfgs):
        s = lbmd.Simulation(cfg, r0s[k], precision=lbmd.LB_FP32_DEV)
        s.relax(300, 1.0)
        s.couple_step(7)
        torch.cuda.synchronize()
        nd = int((ens.pops(k) != s.pops()).sum())
        bd = {n: int((ens.beads(k)[n] != s.beads()[n]).sum()) for n in ("r", "v", "J")}
        print(f"ngp ensemble replica {k}: pops differing {nd}, beads {bd}", flush=True)
        assert nd == 0 and all(v == 0 for v in bd.values()), (k, nd, bd)
        s.close()


def test_adjoint_rejects_ngp():
    _torch()
    from paper_0711_2665_amd import lbmd
    cfg = scaled(C0, shape=(16, 16, 16), wall_pos=8, nb=8, coupling=1)
    r, _ = initial_chain(cfg)
    s = lbmd.Simulation(cfg, r)
    with pytest.raises(lbmd.LbError) as e:
        s.adjoint_sizes(4, 2)
    assert e.value.code == lbmd.LB_ERR_UNSUPPORTED
