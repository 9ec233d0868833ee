"""GPU parity of the fluctuating fluid (the stochastic term of the lattice
Boltzmann equation, Sec. 2, as noise on the 15 non-conserved D3Q19 modes):
the HIP path through the C ABI against the FP64 oracle on the same seeded
inputs, the ensemble and graph paths against single eager runs, and the
fluctuation-dissipation statistics of a periodic box."""
import numpy as np
import pytest

from paper_0711_2665_amd.workloads import BASE, C0, initial_chain, scaled

pytestmark = pytest.mark.gpu

TOL64 = 1e-12
# Norms b_k of the D3Q19 modes (textbook values, also pinned on the oracle)
B_LIT = np.array([1, 1 / 3, 1 / 3, 1 / 3, 2 / 3, 4 / 3, 4 / 9, 1 / 9, 1 / 9, 1 / 9,
                  2 / 3, 2 / 3, 2 / 3, 2 / 9, 2 / 9, 2 / 9, 2, 4 / 3, 4 / 9])


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _cfg(shape, **kw):
    c = dict(BASE)
    c.update(dict(shape=shape, wall_axis=-1, wall_pos=0, pore_h=0, nb=0))
    c.update(kw)
    return c


def _rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    den = np.abs(b).max()
    return float(np.abs(a - b).max() / (den if den > 0 else 1.0))


def _gpu_pops(sim):
    return sim.pops().double().cpu().numpy()


def _load_pops(sim, f):
    """Write populations (storage convention of the context) into a
    one-replica context through its state buffer, step counter 0."""
    torch = sim.torch
    st = sim.get_state()
    es = 8 if sim.dtype == torch.float64 else 4
    st[: 19 * sim.N * es].view(sim.dtype).copy_(torch.as_tensor(np.ascontiguousarray(f).reshape(-1)).to(sim.dtype))
    sim.set_state(st)


@pytest.mark.parametrize("shape,axis,pos,tau", [((12, 10, 16), 2, 8, 0.8), ((32, 16, 12), 0, 16, 1.3)])
def test_fluctuating_lb_only_fp64_matches_oracle(orc, shape, axis, pos, tau):
    """Nine fluid steps with walls, a pore, a body force and the fluid noise
    from a perturbed state: populations within 1e-12 of the oracle (the two
    sides' log, sin, cos may differ in the last bit)."""
    torch = _torch()
    from paper_0711_2665_amd import lbmd
    cfg = _cfg(shape, wall_axis=axis, wall_pos=pos, pore_h=3, g=(1e-5, 2e-5, -1e-5), tau=tau,
               fluid_kT=2e-4, seed=4242, replica=5)
    o = orc.Oracle(cfg)
    s = lbmd.Simulation(cfg)
    rng = np.random.default_rng(3)
    _, w, _ = orc.tables()
    nx, ny, nz = shape
    f0 = w[:, None, None, None] * (1 + 0.05 * rng.standard_normal((19, nz, ny, nx)))
    o.set_pops(f0)
    _load_pops(s, f0)
    fluid = o.flags() == 0
    quiet = orc.Oracle(scaled(cfg, fluid_kT=0.0))
    quiet.set_pops(f0)
    for k in range(3):
        o.lb_step(3)
        s.lb_step(3)
        quiet.lb_step(3)
        torch.cuda.synchronize()
        a, b = _gpu_pops(s)[:, fluid], o.pops()[:, fluid]
        noise = _rel(b, quiet.pops()[:, fluid])
        print(f"fluctuating lb-only {shape} step {3 * (k + 1)}: rel {_rel(a, b):.3e} "
              f"(noise moved the state by {noise:.2e})", flush=True)
        assert noise > 1e-3
        assert _rel(a, b) <= TOL64
    s.check()


def _c0_start(orc, cfg, precision):
    from paper_0711_2665_amd import lbmd
    r, v = initial_chain(cfg)
    o = orc.Oracle(cfg, r, v)
    o.relax(cfg["relax_substeps"], cfg["gamma_relax"])
    ob = o.beads()
    o = orc.Oracle(cfg, ob["r"], np.zeros_like(ob["r"]))
    s = lbmd.Simulation(cfg, ob["r"], None, precision=precision)
    return o, s


def test_fluctuating_coupled_fp64_matches_oracle(orc):
    """The 32^3 system with the 20-bead chain and a thermal fluid at the
    beads' temperature: the nodes carrying bead force take their noise in
    the fused spreading update, the others in the sweep.  After one step
    every field agrees to 1e-12; later, within 1e-12 or 100x the oracle's own
    divergence from a copy whose initial positions moved by one ulp."""
    torch = _torch()
    from paper_0711_2665_amd import lbmd
    cfg = scaled(C0, fluid_kT=C0["kT"])
    o, s = _c0_start(orc, cfg, lbmd.LB_FP64)
    r0 = o.beads()["r"]
    o2 = orc.Oracle(cfg, np.nextafter(r0, np.inf), np.zeros_like(r0))
    fluid = o.flags() == 0
    done = 0
    for target in (1, 5, 20):
        o.couple_step(target - done)
        o2.couple_step(target - done)
        s.couple_step(target - done)
        done = target
        torch.cuda.synchronize()
        ob, ob2 = o.beads(), o2.beads()
        sb = {k: t.cpu().numpy() for k, t in s.beads().items()}
        rows = {"pops": (_rel(_gpu_pops(s)[:, fluid], o.pops()[:, fluid]), _rel(o2.pops()[:, fluid],
                                                                              o.pops()[:, fluid]))}
        for k in ("r", "v", "up", "J"):
            rows[k] = (_rel(sb[k], ob[k]), _rel(ob2[k], ob[k]))
        print(f"thermal c0 step {target}: " + ", ".join(f"{k} gpu {g:.1e} / envelope {e:.1e}"
                                                       for k, (g, e) in rows.items()), flush=True)
        for k, (g, e) in rows.items():
            bound = TOL64 if target == 1 else max(TOL64, 100 * e)
            assert g <= bound, (target, k, g, e)
    s.check()


@pytest.mark.parametrize("shape,axis,pos", [((12, 10, 16), 2, 8), ((32, 16, 12), 0, 16)])
def test_fluctuating_lb_only_fp32_deviation_matches_oracle(orc, shape, axis, pos):
    """FP32 deviation storage with the hardware log2, sqrt and sine against
    the FP64 oracle over 20 fluid steps: deviations within 1e-5 of their
    largest size."""
    torch = _torch()
    from paper_0711_2665_amd import lbmd
    cfg = _cfg(shape, wall_axis=axis, wall_pos=pos, pore_h=3, g=(1e-5, 2e-5, -1e-5), tau=0.8,
               fluid_kT=2e-4, seed=99, replica=1)
    o = orc.Oracle(cfg)
    s = lbmd.Simulation(cfg, precision=lbmd.LB_FP32_DEV)
    rng = np.random.default_rng(4)
    _, w, _ = orc.tables()
    nx, ny, nz = shape
    dev = w[:, None, None, None] * 0.05 * rng.standard_normal((19, nz, ny, nx))
    o.set_pops(w[:, None, None, None] + dev)
    _load_pops(s, dev)
    o.lb_step(20)
    s.lb_step(20)
    torch.cuda.synchronize()
    fluid = o.flags() == 0
    a = _gpu_pops(s)[:, fluid]
    b = (o.pops() - w[:, None, None, None])[:, fluid]
    err = np.abs(a - b).max() / np.abs(b).max()
    print(f"fp32-dev fluctuating lb-only {shape}: rel err of deviations {err:.2e}", flush=True)
    assert err < 2e-6                       # measured 1.7e-7, 2.2e-7


def _ens_cfgs():
    return [
        scaled(C0, name="t0", shape=(16, 12, 20), wall_axis=2, wall_pos=10, pore_h=3, nb=12, seed=11, replica=0,
               init_seed=5, fluid_kT=1e-4),
        scaled(C0, name="t1", shape=(20, 16, 16), wall_axis=0, wall_pos=10, pore_h=4, nb=20, seed=12, replica=1,
               init_seed=6),
        scaled(C0, name="t2", shape=(12, 12, 13), wall_axis=-1, wall_pos=0, pore_h=0, nb=0, seed=13, replica=2,
               fluid_kT=3e-4),
    ]


@pytest.mark.parametrize("precision", ["fp64", "fp32dev"])
def test_fluctuating_ensemble_graph_equals_replicas_run_alone(precision):
    """An ensemble mixing thermal and athermal fluids, stepped by graph
    replays with eager work between them: every replica equals, bit for bit,
    the same system run alone with eager steps."""
    torch = _torch()
    from paper_0711_2665_amd import lbmd
    prec = lbmd.LB_FP64 if precision == "fp64" else lbmd.LB_FP32_DEV
    cfgs = _ens_cfgs()
    r0s = [initial_chain(c)[0] for c in cfgs]
    ens = lbmd.Ensemble(cfgs, r0s, precision=prec)
    ens.relax(300, 1.0)
    for n in (3, 4, 2):
        ens.run(n, graph=True)
        ens.observables()
    torch.cuda.synchronize()
    ens.check()
    for k, cfg in enumerate(cfgs):
        s = lbmd.Simulation(cfg, r0s[k] if cfg["nb"] else None, precision=prec)
        s.relax(300, 1.0)
        s.couple_step(9)
        torch.cuda.synchronize()
        nd = int((ens.pops(k) != s.pops()).sum())
        bd = {n: int((ens.beads(k)[n] != s.beads()[n]).sum()) for n in ("r", "v")} if cfg["nb"] else {}
        print(f"{precision} thermal ensemble replica {k}: pops differing {nd}, beads {bd}", flush=True)
        assert nd == 0 and all(v == 0 for v in bd.values()), (k, nd, bd)
        s.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32dev"])
def test_equipartition_on_gpu(orc, precision):
    """A periodic 16^3 box at rest with the fluid noise reaches equipartition:
    every mode k has variance 3 rho kT b_k (modes 0..3 reduced by the fixed
    totals, factor 1 - 1/N), over 400 sampled steps after 300 steps."""
    torch = _torch()
    from paper_0711_2665_amd import lbmd
    kT = 1e-4
    shape = (16, 16, 16)
    N = 16 ** 3
    cfg = _cfg(shape, tau=0.8, fluid_kT=kT, seed=7)
    prec = lbmd.LB_FP64 if precision == "fp64" else lbmd.LB_FP32_DEV
    s = lbmd.Simulation(cfg, precision=prec)
    E = torch.as_tensor(orc.mode_basis(), device=s.device)
    _, w, _ = orc.tables()
    shift = torch.as_tensor(w if precision == "fp64" else np.zeros(19), device=s.device)
    s.lb_step(300)
    acc = torch.zeros(19, dtype=torch.float64, device=s.device)
    nsamp = 400
    for _ in range(nsamp):
        s.lb_step(1)
        f = s.pops().double().reshape(19, -1) - shift[:, None]
        m = E @ f
        acc += (m * m).mean(dim=1)
    var = (acc / nsamp).cpu().numpy()
    want = 3 * kT * B_LIT
    want[:4] *= 1 - 1 / N
    rel = var / want - 1
    print(f"{precision} equipartition, relative deviation per mode: {np.round(rel, 4)}", flush=True)
    assert np.abs(rel).max() < 0.02
    s.check()


def test_adjoint_rejects_a_fluctuating_fluid():
    _torch()
    from paper_0711_2665_amd import lbmd
    cfg = scaled(C0, shape=(16, 16, 16), wall_pos=8, nb=8, fluid_kT=1e-4)
    r, _ = initial_chain(cfg)
    s = lbmd.Simulation(cfg, r)
    with pytest.raises(lbmd.LbError) as e:
        s.adjoint_sizes(4, 2)
        s.adjoint_forward(4, 2)
    assert e.value.code == lbmd.LB_ERR_UNSUPPORTED
