"""GPU parity: the HIP path (through the C ABI) against the FP64 CPU oracle on
the same seeded inputs.  FP64 storage must match to 1e-12 relative (the
kernels evaluate every expression in the oracle's order without
multiply-add contraction, so most fields agree bit for bit); FP32 deviation
storage is held to measured bounds."""
import math

import numpy as np
import pytest

from paper_0711_2665_amd.workloads import BASE, C0, initial_chain, scaled

pytestmark = pytest.mark.gpu

TOL64 = 1e-12


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


def _al(x):
    return (x + 255) // 256 * 256


def _state_tensor(sim, pops, r=None, v=None, step=0):
    """Pack a state buffer of a one-replica context in the layout
    lb_get_state writes: populations, r and v of every bead slot, the step
    counter, the translocation step (-1)."""
    torch = sim.torch
    st = torch.zeros(sim.sizes["state_bytes"], dtype=torch.uint8, device=sim.device)
    es = 8 if sim.dtype == torch.float64 else 4
    npop = 19 * sim.sizes["nodes"]
    st[: 19 * sim.N * es].view(sim.dtype).copy_(torch.as_tensor(np.ascontiguousarray(pops).reshape(-1)).to(sim.dtype))
    pr = _al(npop * es)
    nb3 = _al(3 * sim.slots * 8)
    if sim.nb > 0:
        st[pr: pr + 3 * sim.nb * 8].view(torch.float64).copy_(torch.as_tensor(np.ascontiguousarray(r).reshape(-1)))
        st[pr + nb3: pr + nb3 + 3 * sim.nb * 8].view(torch.float64).copy_(
            torch.as_tensor(np.ascontiguousarray(v).reshape(-1)))
    sb = pr + 2 * nb3
    st[sb: sb + 8].view(torch.int64)[0] = step
    st[sb + 256: sb + 264].view(torch.int64)[0] = -1
    return st


def _rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    den = np.abs(b).max()
    return float(np.abs(a - b).max() / (den if den > 0 else 1.0))


def _gpu_pops(sim):
    return sim.pops().double().cpu().numpy()


@pytest.mark.parametrize("shape,axis,pos", [((12, 10, 16), 2, 8), ((32, 16, 12), 0, 16), ((64, 8, 6), 1, 4)])
def test_lb_only_fp64_matches_oracle_bitwise(orc, shape, axis, pos):
    """Shapes cover the per-node sweep (12 x 10 x 16) and the vector sweep
    (rows of 32 and 64 nodes, walls normal to x and to y)."""
    torch = _torch()
    from paper_0711_2665_amd import lbmd
    cfg = _cfg(shape, wall_axis=axis, wall_pos=pos, pore_h=3, g=(1e-5, 2e-5, -1e-5), tau=0.8)
    o = orc.Oracle(cfg)
    s = lbmd.Simulation(cfg)
    rng = np.random.default_rng(1)
    _, w, _ = orc.tables()
    nx, ny, nz = shape
    f0 = w[:, None, None, None] * (1 + 0.05 * rng.standard_normal((19, nz, ny, nx)))
    o.set_pops(f0)
    s.set_state(_state_tensor(s, f0))
    fluid = o.flags() == 0
    assert np.array_equal(s.flags().cpu().numpy() & 1, o.flags())
    for k in range(3):
        o.lb_step(3)
        s.lb_step(3)
        torch.cuda.synchronize()
        a, b = _gpu_pops(s)[:, fluid], o.pops()[:, fluid]
        nbit = int((a != b).sum())
        print(f"lb-only step {3 * (k + 1)}: rel {_rel(a, b):.3e}, differing entries {nbit} of {a.size}", flush=True)
        assert _rel(a, b) <= TOL64
    assert nbit == 0
    s.check()


@pytest.mark.parametrize("precision", ["fp64", "fp32dev"])
def test_rest_start_on_unaligned_lattice_matches_oracle(orc, precision):
    """A lattice whose node count is not a multiple of 64 (11 x 9 x 13), run
    from the library's own rest initialisation under a body force: the
    populations must equal the oracle's (bitwise in FP64)."""
    torch = _torch()
    from paper_0711_2665_amd import lbmd
    cfg = _cfg((11, 9, 13), wall_axis=2, wall_pos=6, pore_h=3, g=(1e-5, -2e-5, 3e-5), tau=0.9)
    prec = lbmd.LB_FP64 if precision == "fp64" else lbmd.LB_FP32_DEV
    o = orc.Oracle(cfg)
    s = lbmd.Simulation(cfg, precision=prec)
    o.lb_step(10)
    s.lb_step(10)
    torch.cuda.synchronize()
    fluid = o.flags() == 0
    _, w, _ = orc.tables()
    a = _gpu_pops(s)[:, fluid]
    b = o.pops()[:, fluid] - (0.0 if precision == "fp64" else w[:, None])
    if precision == "fp64":
        assert np.array_equal(a, b)
    else:
        rel = np.abs(a - b).max() / np.abs(b).max()
        print(f"fp32-dev unaligned rest start, 10 steps: rel err of deviations {rel:.2e}", flush=True)
        assert rel <= 5e-6                 # the 20-step LB-only runs measure 4.5e-7


def test_poiseuille_on_gpu_matches_closed_form():
    _torch()
    from paper_0711_2665_amd import lbmd
    tau, g, L = 0.8, 1e-5, 32
    cfg = _cfg((4, 4, L), tau=tau, g=(g, 0.0, 0.0), wall_axis=2, wall_pos=0, pore_h=0)
    cfg["wall_pos"] = 2      # the library keeps the wall plane inside [2, n-3]
    s = lbmd.Simulation(cfg)
    nu = (tau - 0.5) / 3
    s.lb_step(int(40 * (L - 1) ** 2 / (nu * math.pi ** 2)))
    f = _gpu_pops(s)[:, :, 0, 0]
    c = np.array([[0, 0, 0], [1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0], [0, 0, 1], [0, 0, -1],
                  [1, 1, 0], [-1, -1, 0], [1, -1, 0], [-1, 1, 0], [1, 0, 1], [-1, 0, -1], [1, 0, -1],
                  [-1, 0, 1], [0, 1, 1], [0, -1, -1], [0, 1, -1], [0, -1, 1]], dtype=float)
    # pulled (post-stream) velocity at each fluid node z, bounce-back at z = 2
    u = []
    for z in range(L):
        if z == 2:
            continue
        fi = []
        for i in range(19):
            zs = (z - int(c[i, 2])) % L
            opp = i if i == 0 else (i + 1 if i % 2 else i - 1)
            fi.append(f[opp, z] if zs == 2 else f[i, zs])
        fi = np.array(fi)
        u.append((fi @ c[:, 0]) / fi.sum())
    u = np.array(u)
    zz = np.array([z for z in range(L) if z != 2], dtype=float)
    zz = np.where(zz < 2, zz + L, zz) - 2      # distance from the wall plane, 1..L-1
    lam = (tau - 0.5) ** 2
    want = g / (2 * nu) * (zz - 0.5) * (L - 0.5 - zz) + g * ((16 * lam - 3) / (24 * nu) - 0.5)
    assert _rel(u, want) < 1e-10


def _c0_relaxed_pair(orc, cfg, precision=None):
    from paper_0711_2665_amd import lbmd
    r, v = initial_chain(cfg)
    o = orc.Oracle(cfg, r, v)
    o.relax(cfg["relax_substeps"], cfg["gamma_relax"])
    s = lbmd.Simulation(cfg, r, v, precision=lbmd.LB_FP64 if precision is None else precision)
    s.relax(cfg["relax_substeps"], cfg["gamma_relax"])
    return o, s


def _compare_beads(o, s, tol, label):
    ob = o.beads()
    sb = {k: t.cpu().numpy() for k, t in s.beads().items()}
    errs = {k: _rel(sb[k], ob[k]) for k in ("r", "v", "up", "J")}
    print(label, {k: f"{e:.2e}" for k, e in errs.items()}, flush=True)
    for k, e in errs.items():
        assert e <= tol, (label, k, e)
    return errs


def test_relaxation_fp64_matches_oracle(orc):
    torch = _torch()
    o, s = _c0_relaxed_pair(orc, C0)
    torch.cuda.synchronize()
    rg = s.beads()["r"].cpu().numpy()
    ro = o.beads()["r"]
    print("relax rel", _rel(rg, ro), "bitwise", np.array_equal(rg, ro), flush=True)
    assert _rel(rg, ro) <= TOL64
    assert np.abs(s.beads()["v"].cpu().numpy()).max() == 0.0


def _c0_common_start(orc, cfg, precision=None):
    """Oracle relaxes the seeded coil; the GPU context is loaded with the
    oracle's relaxed state (rest populations, r, v = 0, step 0), so both sides
    start from identical inputs."""
    from paper_0711_2665_amd import lbmd
    r, v = initial_chain(cfg)
    o = orc.Oracle(cfg, r, v)
    o.relax(cfg["relax_substeps"], cfg["gamma_relax"])
    ob = o.beads()
    o = orc.Oracle(cfg, ob["r"], np.zeros_like(ob["r"]))
    s = lbmd.Simulation(cfg, ob["r"], None, precision=lbmd.LB_FP64 if precision is None else precision)
    return o, s


def test_coupled_c0_fp64_matches_oracle(orc):
    """c0 (32^3, 20 beads, 200 steps).  After one coupled step from identical
    inputs every field agrees to 1e-12 relative.  The bead dynamics is
    chaotic: the GPU's and the host's transcendental functions (noise and
    bending angle) differ in the last bit, and such differences grow
    exponentially.  From step 10 on, each field must therefore stay within
    1e-12 or within 100x the oracle's own divergence from a copy of itself
    whose initial positions were moved by one ulp (the intrinsic envelope);
    mass and momentum stay within 1e-12 throughout."""
    torch = _torch()
    cfg = C0
    o, s = _c0_common_start(orc, cfg)
    r0 = o.beads()["r"]
    o2 = orc.Oracle(cfg, np.nextafter(r0, np.inf), np.zeros_like(r0))
    fluid = o.flags() == 0
    # gross size of one step's bounce-back terms: 2 w_opp per wall link
    c, w, opp = orc.tables()
    solid = ~fluid
    gross_bb = sum(2.0 * w[opp[i]] * float((np.roll(solid, (c[i][2], c[i][1], c[i][0]), (0, 1, 2)) & fluid).sum())
                   for i in range(1, 19))
    done = 0
    for target in (1, 10, 50, 100, 200):
        o.couple_step(target - done)
        o2.couple_step(target - done)
        s.couple_step(target - done)
        done = target
        torch.cuda.synchronize()
        ob, ob2 = o.beads(), o2.beads()
        sb = {k: t.cpu().numpy() for k, t in s.beads().items()}
        a, b, b2 = _gpu_pops(s)[:, fluid], o.pops()[:, fluid], o2.pops()[:, fluid]
        rows = {"pops": (_rel(a, b), _rel(b2, b))}
        for k in ("r", "v", "up", "J"):
            rows[k] = (_rel(sb[k], ob[k]), _rel(ob2[k], ob[k]))
        print(f"c0 step {target}: " + ", ".join(f"{k} gpu {g:.1e} / 1-ulp envelope {e:.1e}"
                                                 for k, (g, e) in rows.items()), flush=True)
        for k, (g, e) in rows.items():
            bound = TOL64 if target == 1 else max(TOL64, 100 * e)
            assert g <= bound, (target, k, g, e)
        go = s.observables().cpu().numpy()
        oo = o.observables()
        oo2 = o2.observables()
        for k in list(range(16)) + [22, 23, 24]:
            scale = TOL64 * max(1.0, abs(oo[k]))
            bound = scale if k in (0, 22) or target == 1 else max(scale, 100 * abs(oo2[k] - oo[k]))
            assert abs(go[k] - oo[k]) <= bound, (target, k, go[k], oo[k], oo2[k])
        # the wall ledgers are running sums of cancelling terms (bounce-back
        # on both faces of the wall): relative to their gross size
        gross = (gross_bb * target, max(1e-300, float(np.abs(ob["J"]).sum()) * target))
        for k in range(16, 22):
            sc = TOL64 * gross[0 if k < 19 else 1]
            bound = sc if target == 1 else max(sc, 100 * abs(oo2[k] - oo[k]))
            assert abs(go[k] - oo[k]) <= bound, (target, k, go[k], oo[k], oo2[k])
    s.check()


def test_single_coupled_step_fp64_bitwise_up_to_libm(orc):
    """One coupled step with the noise and bending switched off (kT = 0,
    kappa = 0): no transcendental function is evaluated, so the GPU step must
    equal the oracle step bit for bit."""
    torch = _torch()
    cfg = scaled(C0, kT=0.0, kappa=0.0)
    o, s = _c0_common_start(orc, cfg)
    o.couple_step(3)
    s.couple_step(3)
    torch.cuda.synchronize()
    fluid = o.flags() == 0
    a, b = _gpu_pops(s)[:, fluid], o.pops()[:, fluid]
    sb = {k: t.cpu().numpy() for k, t in s.beads().items()}
    ob = o.beads()
    print("kT=0, kappa=0, 3 steps: pops differing", int((a != b).sum()),
          {k: int((sb[k] != ob[k]).sum()) for k in ("r", "v", "up", "J")}, flush=True)
    assert np.array_equal(a, b)
    for k in ("r", "v", "up", "J"):
        assert np.array_equal(sb[k], ob[k]), k


def test_long_chain_with_per_step_lists_bitwise(orc):
    """A chain of 1100 beads takes the long-chain path: neighbour lists from
    a hashed cell list at every coupled step (larger skin).  With kT = 0 and
    kappa = 0 three coupled steps must equal the oracle bit for bit."""
    torch = _torch()
    from paper_0711_2665_amd import lbmd
    cfg = scaled(C0, shape=(40, 40, 40), wall_pos=20, nb=1100, kT=0.0, kappa=0.0, init_seed=9)
    r, v = initial_chain(cfg)
    o = orc.Oracle(cfg, r, v)
    o.relax(300, 1.0)
    ob = o.beads()
    o = orc.Oracle(cfg, ob["r"], np.zeros_like(ob["r"]))
    s = lbmd.Simulation(cfg, ob["r"], None)
    o.couple_step(3)
    s.couple_step(3)
    torch.cuda.synchronize()
    s.check()
    fluid = o.flags() == 0
    a, b = _gpu_pops(s)[:, fluid], o.pops()[:, fluid]
    sb = {k: t.cpu().numpy() for k, t in s.beads().items()}
    ob = o.beads()
    print("1100 beads, 3 steps: pops differing", int((a != b).sum()),
          {k: int((sb[k] != ob[k]).sum()) for k in ("r", "v", "up", "J")}, s.diagnostics(), flush=True)
    assert np.array_equal(a, b)
    for k in ("r", "v", "up", "J"):
        assert np.array_equal(sb[k], ob[k]), k


def test_long_chain_rebuilds_inside_the_cycle_bitwise(orc):
    """The 1100-bead chain with a uniform drift of 1.5 per step parallel to
    the wall: beads pass half the skin inside a sub-cycle, so lists are
    rebuilt there -- from the cell table while every bead is within its
    margin of where it was binned, else by the full scan.  Three coupled
    steps (kT = 0, kappa = 0) must equal the oracle bit for bit, and both
    kinds of rebuild must have run."""
    torch = _torch()
    from paper_0711_2665_amd import lbmd
    cfg = scaled(C0, shape=(40, 40, 40), wall_pos=20, nb=1100, kT=0.0, kappa=0.0, init_seed=9)
    r, v = initial_chain(cfg)
    o = orc.Oracle(cfg, r, v)
    o.relax(300, 1.0)
    r0 = o.beads()["r"]
    v0 = np.zeros_like(r0)
    v0[:, 0] = 1.5
    o = orc.Oracle(cfg, r0, v0)
    s = lbmd.Simulation(cfg, r0, v0)
    o.couple_step(3)
    s.couple_step(3)
    torch.cuda.synchronize()
    s.check()
    diag = s.diagnostics()
    fluid = o.flags() == 0
    a, b = _gpu_pops(s)[:, fluid], o.pops()[:, fluid]
    sb = {k: t.cpu().numpy() for k, t in s.beads().items()}
    ob = o.beads()
    print("1100 beads drifting, 3 steps: pops differing", int((a != b).sum()),
          {k: int((sb[k] != ob[k]).sum()) for k in ("r", "v", "up", "J")}, diag, flush=True)
    assert np.array_equal(a, b)
    for k in ("r", "v", "up", "J"):
        assert np.array_equal(sb[k], ob[k]), k
    assert diag["cell_rebuilds"] >= 1 and diag["rebuilds"] > diag["cell_rebuilds"]


def test_long_chain_graph_replay_equals_eager_steps(orc):
    """The long-chain path builds the next step's lists on the sweep stream
    beside the spreading: steps replayed from the captured graph, with eager
    work between the replays, equal eager steps bit for bit."""
    torch = _torch()
    from paper_0711_2665_amd import lbmd
    cfg = scaled(C0, shape=(40, 40, 40), wall_pos=20, nb=1100, init_seed=9)
    r, _ = initial_chain(cfg)
    a = lbmd.Simulation(cfg, r)
    b = lbmd.Simulation(cfg, r)
    for e in (a, b):
        e.relax(300, 1.0)
    for n in (2, 3, 1, 4):
        a.couple_step(n)
        b.run(n, graph=True)
        b.observables()
        torch.cuda.synchronize()
        assert torch.equal(a.pops(), b.pops()), n
        for k in ("r", "v", "up", "J"):
            assert torch.equal(a.beads()[k], b.beads()[k]), (n, k)
    a.check()
    b.check()


def test_paper_soft_lj_coupled_steps_bitwise(orc):
    """The paper's bead LJ (sigma = 1.8, eps = 1e-4, r_c = 2^(1/6) 1.8 > 2,
    so wall sites two nodes from a bead's base node count), without noise and
    bending: five coupled steps equal the oracle bit for bit."""
    torch = _torch()
    cfg = scaled(C0, kT=0.0, kappa=0.0, sigma=1.8, eps=1e-4, rc=2.0 ** (1.0 / 6.0) * 1.8)
    o, s = _c0_common_start(orc, cfg)
    o.couple_step(5)
    s.couple_step(5)
    torch.cuda.synchronize()
    fluid = o.flags() == 0
    a, b = _gpu_pops(s)[:, fluid], o.pops()[:, fluid]
    sb = {k: t.cpu().numpy() for k, t in s.beads().items()}
    ob = o.beads()
    print("soft LJ, 5 steps: pops differing", int((a != b).sum()),
          {k: int((sb[k] != ob[k]).sum()) for k in ("r", "v", "up", "J")}, flush=True)
    assert np.array_equal(a, b)
    for k in ("r", "v", "up", "J"):
        assert np.array_equal(sb[k], ob[k]), k
    s.check()


@pytest.mark.parametrize("shape,axis,pos", [((12, 10, 16), 2, 8), ((32, 16, 12), 0, 16)])
def test_lb_only_fp32_deviation_matches_oracle(orc, shape, axis, pos):
    """FP32 deviation storage against the FP64 oracle over 20 fluid steps from
    a random perturbation: the deviations agree to a few FP32 ulps of their
    size (bound measured: well below 1e-6 of max |f - w|)."""
    torch = _torch()
    from paper_0711_2665_amd import lbmd
    cfg = _cfg(shape, wall_axis=axis, wall_pos=pos, pore_h=3, g=(1e-5, 2e-5, -1e-5), tau=0.8)
    o = orc.Oracle(cfg)
    s = lbmd.Simulation(cfg, precision=lbmd.LB_FP32_DEV)
    rng = np.random.default_rng(2)
    _, w, _ = orc.tables()
    nx, ny, nz = shape
    dev = w[:, None, None, None] * 0.05 * rng.standard_normal((19, nz, ny, nx))
    o.set_pops(w[:, None, None, None] + dev)
    s.set_state(_state_tensor(s, dev))
    o.lb_step(20)
    s.lb_step(20)
    torch.cuda.synchronize()
    fluid = o.flags() == 0
    a = _gpu_pops(s)[:, fluid]
    b = (o.pops() - w[:, None, None, None])[:, fluid]
    err = np.abs(a - b).max() / np.abs(b).max()
    print(f"fp32-dev lb-only {shape}: rel err of deviations {err:.2e}", flush=True)
    assert err < 5e-6                      # measured 4.5e-7


def test_fp32_deviation_rest_state_is_exact():
    torch = _torch()
    from paper_0711_2665_amd import lbmd
    cfg = _cfg((16, 12, 20), wall_axis=2, wall_pos=10, pore_h=3)
    s = lbmd.Simulation(cfg, precision=lbmd.LB_FP32_DEV)
    s.lb_step(7)
    torch.cuda.synchronize()
    assert float(s.pops().abs().max()) == 0.0


def test_fp32_deviation_coupled_c0_error(orc):
    torch = _torch()
    from paper_0711_2665_amd import lbmd
    o, s = _c0_common_start(orc, C0, precision=lbmd.LB_FP32_DEV)
    fluid = o.flags() == 0
    _, w, _ = orc.tables()
    o.couple_step(50)
    s.couple_step(50)
    torch.cuda.synchronize()
    fo = o.pops()[:, fluid] - w[:, None]
    fs = _gpu_pops(s)[:, fluid]
    err_f = np.abs(fs - fo).max()
    rg, ro = s.beads()["r"].cpu().numpy(), o.beads()["r"]
    print(f"fp32-dev c0 50 steps: |f - f64|_max {err_f:.3e} (max |f - w| {np.abs(fo).max():.3e}), "
          f"|r - r64|_max {np.abs(rg - ro).max():.3e}", flush=True)
    assert err_f < 3e-9                    # measured 2.4e-10
    assert np.abs(rg - ro).max() < 5e-8     # measured 4.9e-9


def test_watchdog_flags_nan_population(orc):
    _torch()
    from paper_0711_2665_amd import lbmd
    cfg = _cfg((8, 8, 8))
    s = lbmd.Simulation(cfg)
    _, w, _ = orc.tables()
    f = np.repeat(w[:, None], 512, axis=1).reshape(19, 8, 8, 8).copy()
    f[3, 4, 4, 4] = np.nan
    s.set_state(_state_tensor(s, f))
    s.lb_step(1)
    with pytest.raises(lbmd.LbError) as e:
        s.check()
    assert e.value.code == lbmd.LB_ERR_UNSTABLE


def test_runs_are_bitwise_reproducible_and_resumable(orc):
    torch = _torch()
    from paper_0711_2665_amd import lbmd
    cfg = scaled(C0, shape=(24, 24, 24), wall_pos=12, nb=16)
    r, v = initial_chain(cfg)
    a = lbmd.Simulation(cfg, r, v, precision=lbmd.LB_FP32_DEV)
    b = lbmd.Simulation(cfg, r, v, precision=lbmd.LB_FP32_DEV)
    for sim in (a, b):
        sim.relax(1000, 1.0)
        sim.couple_step(20)
    st = a.get_state()
    a.couple_step(15)
    b.couple_step(15)
    torch.cuda.synchronize()
    pa, pb = a.pops().clone(), b.pops().clone()
    ra = a.beads()["r"].clone()
    assert torch.equal(pa, pb) and torch.equal(ra, b.beads()["r"])
    a.set_state(st)
    assert a.step_count() == 20
    a.couple_step(15)
    torch.cuda.synchronize()
    assert torch.equal(a.pops(), pa) and torch.equal(a.beads()["r"], ra)
