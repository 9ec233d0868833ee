"""Wall momentum ledgers and the observable groups on the GPU, through the C
ABI, against the FP64 oracle.

The two wall terms of the bead-fluid momentum balance (Sec. 2,
Eq. (momentum_cons), with halfway bounce-back at the wall): the momentum the
wall takes from bounced populations, and the bead impulse the spreading
drops on solid nodes.  Both are running FP64 sums over steps; the GPU adds
each step's terms in another order than the oracle (block trees against
plane sums), so the comparison is relative to the gross size of the summed
terms, not to the (cancelling) net value.
"""
import numpy as np
import pytest

from paper_0711_2665_amd.workloads import C0, scaled

pytestmark = pytest.mark.gpu

TOL64 = 1e-12


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _gross_bb(o, steps):
    """Gross size of the bounce-back sum: steps x sum over wall links of
    2 |f_opp| with f at its rest value w (the flows here are slow)."""
    import oracle
    c, w, opp = oracle.tables()
    solid = o.flags().astype(bool)
    nz, ny, nx = solid.shape
    tot = 0.0
    for i in range(1, 19):
        up = np.roll(solid, shift=(c[i][2], c[i][1], c[i][0]), axis=(0, 1, 2))   # solid at x - c_i
        tot += 2.0 * w[opp[i]] * float((up & ~solid).sum())
    return steps * tot


def _wall_chain_cfg(**kw):
    # no bead LJ (so no wall force acts on the beads), no field: the only
    # momentum that leaves fluid + beads is what the two ledgers record
    c = scaled(C0, shape=(16, 16, 16), wall_pos=8, nb=6, n_sub=50, f_drive=0.0, kT=1e-3, eps=0.0)
    c.update(kw)
    return c


def _wall_chain():
    # beads straddling the solid part of the wall plane z = 8 (the pore is
    # x, y in 7..9): their stencils have solid corners
    return np.array([[2.3 + 0.9 * k, 3.4, 7.6 + 0.12 * k] for k in range(6)])


def test_ledgers_match_oracle_after_one_step(orc):
    """One coupled step from identical inputs: the bounce-back ledger within
    1e-12 of its gross size, the spread-on-solid ledger within 1e-12 of the
    sum of |W J| (both nonzero here)."""
    torch = _torch()
    from paper_0711_2665_amd import lbmd
    cfg = _wall_chain_cfg()
    r = _wall_chain()
    v = 0.02 * np.random.default_rng(4).standard_normal(r.shape)
    o = orc.Oracle(cfg, r, v)
    s = lbmd.Simulation(cfg, r, v, precision=lbmd.LB_FP64)
    o.couple_step(1)
    s.couple_step(1)
    torch.cuda.synchronize()
    s.check()
    go, oo = s.observables().cpu().numpy(), o.observables()
    gb = _gross_bb(o, 1)
    J = o.beads()["J"]
    gsp = float(np.abs(J).sum())
    print("bb gpu", go[16:19], "oracle", oo[16:19], "gross", gb, "| sp gpu", go[19:22], "oracle", oo[19:22],
          "gross", gsp, flush=True)
    assert np.abs(oo[19:22]).max() > 1e-3 * gsp > 0.0          # the spread did drop impulse on the wall
    assert np.abs(go[16:19] - oo[16:19]).max() <= TOL64 * gb
    assert np.abs(go[19:22] - oo[19:22]).max() <= TOL64 * gsp


@pytest.mark.parametrize("graph", [False, True])
def test_total_momentum_with_walls_is_conserved(orc, graph):
    """Pin P8 on the GPU: without bead LJ and field, fluid + bead momentum +
    both wall ledgers stay constant over 40 coupled steps (eager, and
    replayed from the captured graph), while the ledgers themselves grow."""
    torch = _torch()
    from paper_0711_2665_amd import lbmd
    cfg = _wall_chain_cfg()
    r = _wall_chain()
    v = 0.05 * np.random.default_rng(6).standard_normal(r.shape)
    s = lbmd.Simulation(cfg, r, v, precision=lbmd.LB_FP64)
    P0 = s.observables().cpu().numpy().copy()
    s.run(40, graph=graph)
    torch.cuda.synchronize()
    s.check()
    P1 = s.observables().cpu().numpy()

    def total(P):
        return P[1:4] + P[5:8] + P[16:19] + P[19:22]

    drift = np.abs(total(P1) - total(P0)).max()
    print(f"graph={graph}: ledgers bb {P1[16:19]}, sp {P1[19:22]}, total drift {drift:.2e}", flush=True)
    assert np.abs(P1[16:19]).max() > 1e-6 and np.abs(P1[19:22]).max() > 1e-6
    # running FP64 sums of ~1e5 terms of size ~0.03: the oracle's own pin
    # allows 5e-11 for the same system
    assert drift < 5e-11


def test_ledgers_follow_the_state_buffer(orc):
    """lb_get_state / lb_set_state carry the ledgers: a context restored from
    a checkpoint continues with the ledger it had there."""
    torch = _torch()
    from paper_0711_2665_amd import lbmd
    cfg = _wall_chain_cfg(kT=0.0)
    r = _wall_chain()
    s = lbmd.Simulation(cfg, r, None, precision=lbmd.LB_FP64)
    s.couple_step(5)
    st = s.get_state()
    a = s.observables().cpu().numpy()[16:22].copy()
    s.couple_step(5)
    b = s.observables().cpu().numpy()[16:22].copy()
    s.set_state(st)
    assert np.array_equal(s.observables().cpu().numpy()[16:22], a)
    s.couple_step(5)
    assert np.array_equal(s.observables().cpu().numpy()[16:22], b)


def test_observable_groups(orc):
    """Each group of the mask writes its own entries and leaves the others
    as they were; the groups together equal the full call; unknown bits are
    rejected."""
    torch = _torch()
    from paper_0711_2665_amd import lbmd
    cfg = _wall_chain_cfg()
    s = lbmd.Simulation(cfg, _wall_chain(), None, precision=lbmd.LB_FP64)
    s.couple_step(3)
    full = s.observables(lbmd.LB_OBS_ALL).cpu().numpy().copy()
    groups = {lbmd.LB_OBS_FLUID: [0, 1, 2, 3], lbmd.LB_OBS_BEADS: list(range(4, 16)) + [23, 24],
              lbmd.LB_OBS_LEDGERS: list(range(16, 22)), lbmd.LB_OBS_STEP: [22]}
    for m, idx in groups.items():
        got = s.observables(m).cpu().numpy()
        other = [k for k in range(lbmd.LB_NOBS) if k not in idx]
        assert np.array_equal(got[idx], full[idx]), m
        assert np.isnan(got[other]).all(), m
    with pytest.raises(lbmd.LbError):
        s.observables(16)
