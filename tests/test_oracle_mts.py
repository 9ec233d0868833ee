"""Pins of the oracle's multiple-time-step bead cycle (Sec. 2, the nested
cycle over the bonds with M outer steps; read as a RESPA split whose inner
steps are the SPV sub-steps with the bonded forces): with no slow forces it
is the uniform SPV cycle bit for bit; with no bonded forces and no friction
it is velocity Verlet of step 1/M on the slow forces; without friction it
conserves the energy; with friction and noise it reaches equipartition; a
coupled run conserves fluid + bead momentum.  CPU only."""
import math

import numpy as np
import pytest

from paper_0711_2665_amd.workloads import BASE, C0, initial_chain, scaled

pytestmark = pytest.mark.filterwarnings("ignore")

# the paper's bead LJ (sigma = 1.8, eps = 1e-4) with bonds at rest at the
# cut-off, so the truncated LJ does not act along a bond at rest
SOFT = dict(sigma=1.8, eps=1e-4, rc=2.0 ** (1.0 / 6.0) * 1.8, r0=2.0 ** (1.0 / 6.0) * 1.8)


def _cfg(shape, **kw):
    c = dict(BASE)
    c.update(dict(shape=shape, wall_axis=-1, wall_pos=0, pore_h=0, nb=0))
    c.update(kw)
    return c


@pytest.mark.parametrize("M", [1, 5, 20])
def test_mts_without_slow_forces_is_the_uniform_cycle_bitwise(orc, M):
    """eps = 0 and no wall: the slow kicks add exact zeros and the inner
    sub-steps are the uniform SPV sub-steps, noise index by index."""
    cfg = scaled(C0, shape=(16, 16, 16), wall_axis=-1, nb=12, n_sub=100, kT=1e-3, eps=0.0)
    r, _ = initial_chain(scaled(C0, shape=(16, 16, 16), wall_pos=8, nb=12))
    rng = np.random.default_rng(1)
    v0 = 0.02 * rng.standard_normal(r.shape)
    a = orc.Oracle(cfg, r, v0)
    b = orc.Oracle(scaled(cfg, mts_outer=M), r, v0)
    a.couple_step(4)
    b.couple_step(4)
    for k in ("r", "v", "up", "J"):
        assert np.array_equal(a.beads()[k], b.beads()[k]), k
    assert np.array_equal(a.pops(), b.pops())
    assert np.abs(a.beads()["r"] - r).max() > 1e-3


def _lj_textbook(r, ext, sigma, eps, rc):
    F = np.zeros_like(r)
    for p in range(len(r)):
        d = r[p] - r
        d -= ext * np.round(d / ext)
        r2 = (d * d).sum(1)
        r2[p] = np.inf
        near = r2 < rc * rc
        sr6 = (sigma ** 2 / r2[near]) ** 3
        F[p] = ((24 * eps * (2 * sr6 * sr6 - sr6) / r2[near])[:, None] * d[near]).sum(0)
    return F


def test_mts_without_bonded_forces_or_friction_is_velocity_verlet(orc):
    """k_bond = kappa = gamma = kT = 0: each outer step is v += dt/2 F/m,
    r += dt v (as 2 M_b half drifts), v += dt/2 F/m with dt = 1/M."""
    M, nsteps = 5, 10
    sig, eps = 1.8, 0.02
    rc = 2.0 ** (1.0 / 6.0) * sig
    r0 = np.array([[10.0, 10.0, 10.0], [11.9, 10.2, 10.1], [10.3, 11.8, 10.4], [11.5, 11.6, 11.9],
                   [9.2, 11.0, 11.6]])
    rng = np.random.default_rng(2)
    v0 = 0.05 * rng.standard_normal(r0.shape)
    cfg = _cfg((24, 24, 24), nb=len(r0), k_bond=0.0, kappa=0.0, gamma=0.0, kT=0.0, sigma=sig, eps=eps, rc=rc,
               n_sub=100, mts_outer=M)
    o = orc.Oracle(cfg, r0, v0)
    o.md_only(nsteps)
    ext = np.full(3, 24.0)
    r, v = r0.copy(), v0.copy()
    dt = 1.0 / M
    for _ in range(nsteps * M):
        v = v + 0.5 * dt * _lj_textbook(r, ext, sig, eps, rc)
        r = r + dt * v
        v = v + 0.5 * dt * _lj_textbook(r, ext, sig, eps, rc)
    b = o.beads()
    assert np.abs(b["r"] - r0).max() > 0.05             # the beads did interact and move
    assert np.abs(_lj_textbook(r0, ext, sig, eps, rc)).max() > 1e-3
    assert np.abs(b["r"] - r).max() < 1e-10, np.abs(b["r"] - r).max()
    assert np.abs(b["v"] - v).max() < 1e-10 * max(1.0, np.abs(v).max())


def test_mts_conserves_energy_without_friction(orc):
    """gamma = kT = 0, a relaxed 40-bead chain with bonds, bending and the
    paper's soft LJ, velocities of thermal size, M = 5 outer and 20 inner
    steps per LB step: over 1000 LB steps the total energy stays within a
    band far below the kinetic energy, with no drift (the split is
    time-reversible and symplectic); the uniform cycle gives a band of the
    same size."""
    cfg = _cfg((32, 32, 32), nb=40, gamma=0.0, kT=0.0, n_sub=100, mts_outer=5, **SOFT)
    r, _ = initial_chain(scaled(C0, shape=(32, 32, 32), wall_pos=16, nb=40, **SOFT))
    o = orc.Oracle(cfg, r)
    o.relax(20000, 1.0)
    rng = np.random.default_rng(3)
    o.set_beads(v=0.01 * rng.standard_normal(r.shape))

    def energy():
        v = o.beads()["v"]
        return 0.5 * (v * v).sum() + o.energy()

    ke0 = 0.5 * (o.beads()["v"] ** 2).sum()
    E = [energy()]
    for _ in range(50):
        o.md_only(20)
        E.append(energy())
    E = np.array(E) - E[0]
    band = np.abs(E).max()
    drift = abs(E[-10:].mean() - E[1:11].mean())
    print(f"energy band {band:.3e}, drift {drift:.3e}, kinetic energy {ke0:.3e}")
    assert band < 5e-3 * ke0
    assert drift < 2e-3 * ke0


def test_mts_equipartition(orc):
    """gamma = 0.5, kT = 1e-3: a relaxed 150-bead chain with bonds, bending
    and the soft LJ reaches <v_a^2> = kT/m within 4% (bonds k = 10 and
    bending kappa = 1 keep the integrator's own bias at h = 0.01 small)."""
    kT = 1e-3
    cfg = _cfg((40, 40, 40), nb=150, gamma=0.5, kT=kT, n_sub=100, mts_outer=5, k_bond=10.0, kappa=1.0, **SOFT)
    r, _ = initial_chain(scaled(C0, shape=(40, 40, 40), wall_pos=20, nb=150, **SOFT))
    o = orc.Oracle(cfg, r)
    o.relax(20000, 1.0)
    o.md_only(100)
    acc, n = 0.0, 0
    for _ in range(300):
        o.md_only(1)
        v = o.beads()["v"]
        acc += (v * v).mean()
        n += 1
    t = acc / n
    print(f"<v^2> / (kT/m) = {t / kT:.4f}")
    assert abs(t / kT - 1) < 0.04


def test_mts_coupled_run_conserves_momentum(orc):
    cfg = scaled(C0, shape=(16, 16, 16), wall_axis=-1, nb=10, n_sub=100, kT=1e-3, mts_outer=5, **SOFT)
    r, _ = initial_chain(scaled(C0, shape=(16, 16, 16), wall_pos=8, nb=10, **SOFT))
    rng = np.random.default_rng(5)
    o = orc.Oracle(cfg, r, 0.02 * rng.standard_normal(r.shape))
    P0 = o.observables()
    o.couple_step(20)
    P1 = o.observables()
    tot0 = P0[1:4] + P0[5:8]
    tot1 = P1[1:4] + P1[5:8]
    assert np.abs(P1[5:8] - P0[5:8]).max() > 1e-3
    assert np.abs(tot1 - tot0).max() < 1e-12, tot1 - tot0


def test_mts_rejects_an_uneven_split(orc):
    with pytest.raises(ValueError):
        orc.Oracle(_cfg((8, 8, 8), nb=0, n_sub=100, mts_outer=3))
