"""Pins of the oracle's rigid bonds (Sec. 2, Eq. (SPValgo) with its SHAKE and
RATTLE steps): the projections put every bond at r0 and remove every
relative velocity along a bond, by corrections along the bond vectors that
carry no momentum (the tridiagonal solver against a dense solve); a free rigid dimer keeps its kinetic energy; a
constrained chain without friction conserves its energy; with friction and
noise its kinetic temperature counts only the 3N - (N - 1) free degrees of
freedom; a coupled run conserves fluid + bead momentum.  CPU only."""
import numpy as np
import pytest

from paper_0711_2665_amd.workloads import BASE, C0, initial_chain, scaled

pytestmark = pytest.mark.filterwarnings("ignore")


def _cfg(shape, **kw):
    c = dict(BASE)
    c.update(dict(shape=shape, wall_axis=-1, wall_pos=0, pore_h=0, nb=0, constraints=1))
    c.update(kw)
    return c


def _bonds(x):
    return np.linalg.norm(np.diff(x, axis=0), axis=1)


def test_shake_puts_every_bond_at_r0_along_the_reference_bonds(orc):
    rng = np.random.default_rng(1)
    nb = 30
    steps = rng.standard_normal((nb - 1, 3))
    ref = np.vstack([np.zeros(3), np.cumsum(steps / np.linalg.norm(steps, axis=1)[:, None], axis=0)]) + 5.0
    o = orc.Oracle(_cfg((24, 24, 24), nb=nb), ref)
    x0 = ref + 0.03 * rng.standard_normal(ref.shape)
    x = o.shake(x0, ref)
    assert np.abs(_bonds(x) - 1.0).max() < 1e-12
    dx = x - x0
    assert np.abs(dx.sum(axis=0)).max() < 1e-14                   # no momentum
    # bead p moved along the reference bonds it belongs to: the correction
    # lies in the span of ref_{p} - ref_{p-1} and ref_{p+1} - ref_{p}
    b = np.diff(ref, axis=0)
    for p in range(nb):
        span = [b[k] for k in (p - 1, p) if 0 <= k < nb - 1]
        A = np.array(span).T
        coef, *_ = np.linalg.lstsq(A, dx[p], rcond=None)
        assert np.abs(A @ coef - dx[p]).max() < 1e-13
    assert not o.constraint_failed()


def test_rattle_removes_relative_velocity_along_bonds(orc):
    rng = np.random.default_rng(2)
    nb = 25
    steps = rng.standard_normal((nb - 1, 3))
    x = np.vstack([np.zeros(3), np.cumsum(steps / np.linalg.norm(steps, axis=1)[:, None], axis=0)]) + 4.0
    o = orc.Oracle(_cfg((24, 24, 24), nb=nb), x)
    v0 = 0.1 * rng.standard_normal(x.shape)
    v = o.rattle(v0, x)
    rel = (np.diff(x, axis=0) * np.diff(v, axis=0)).sum(axis=1)
    assert np.abs(rel).max() < 1e-12
    assert np.abs((v - v0).sum(axis=0)).max() < 1e-15
    # a velocity that already satisfies the constraints is left as it is
    assert np.abs(o.rattle(v, x) - v).max() < 1e-15


def test_tridiagonal_solver_matches_a_dense_solve(orc):
    # RATTLE's system for a random chain, built here from its definition and
    # solved densely: the oracle's projection must reach the same velocities
    rng = np.random.default_rng(6)
    nb = 12
    steps = rng.standard_normal((nb - 1, 3))
    x = np.vstack([np.zeros(3), np.cumsum(steps / np.linalg.norm(steps, axis=1)[:, None], axis=0)]) + 4.0
    o = orc.Oracle(_cfg((24, 24, 24), nb=nb), x)
    v0 = 0.1 * rng.standard_normal(x.shape)
    r = x[:-1] - x[1:]
    A = np.zeros((nb - 1, nb - 1))
    for k in range(nb - 1):
        A[k, k] = 2 * r[k] @ r[k]
        if k > 0:
            A[k, k - 1] = -r[k] @ r[k - 1]
        if k < nb - 2:
            A[k, k + 1] = -r[k] @ r[k + 1]
    mu = np.linalg.solve(A, -((v0[:-1] - v0[1:]) * r).sum(axis=1))
    want = v0.copy()
    want[:-1] += mu[:, None] * r
    want[1:] -= mu[:, None] * r
    assert np.abs(o.rattle(v0, x) - want).max() < 1e-14


def test_free_rigid_dimer_keeps_its_energy_and_length(orc):
    r0 = np.array([[10.0, 10.0, 10.0], [11.0, 10.0, 10.0]])
    v0 = np.array([[0.0, 0.02, 0.01], [0.0, -0.02, -0.01]])
    cfg = _cfg((24, 24, 24), nb=2, gamma=0.0, kT=0.0, eps=0.0, kappa=0.0, n_sub=20)
    o = orc.Oracle(cfg, r0, v0)
    ke0 = 0.5 * (v0 ** 2).sum()
    for _ in range(50):
        o.md_only(1)
        b = o.beads()
        assert abs(0.5 * (b["v"] ** 2).sum() - ke0) < 1e-9 * ke0
        # velocities stay perpendicular to the bond up to the second half
        # drift, which lengthens it by O(h^2 v^2)
        assert abs(_bonds(b["r"])[0] - 1.0) < 1e-5
    ang = np.arctan2(*(np.diff(o.beads()["r"], axis=0)[0][[1, 0]]))
    assert abs(ang) > 0.1                                          # it did rotate


def test_constrained_chain_conserves_energy(orc):
    cfg = _cfg((32, 32, 32), nb=40, gamma=0.0, kT=0.0, n_sub=100)
    r, _ = initial_chain(scaled(C0, shape=(32, 32, 32), wall_pos=16, nb=40))
    o = orc.Oracle(cfg, r)
    o.relax(5000, 1.0)
    rng = np.random.default_rng(3)
    v = o.rattle(0.01 * rng.standard_normal(r.shape), o.beads()["r"])
    o.set_beads(v=v)

    def energy():
        vv = o.beads()["v"]
        return 0.5 * (vv * vv).sum() + o.energy()

    ke0 = 0.5 * (v * v).sum()
    E = [energy()]
    for _ in range(40):
        o.md_only(5)
        E.append(energy())
    E = np.array(E) - E[0]
    print(f"constrained chain: energy band {np.abs(E).max():.3e}, kinetic {ke0:.3e}")
    assert np.abs(E).max() < 2e-2 * ke0
    assert not o.constraint_failed()


def test_constrained_chain_equipartition_counts_free_degrees(orc):
    kT, nb = 1e-3, 120
    cfg = _cfg((40, 40, 40), nb=nb, gamma=0.5, kT=kT, n_sub=100, kappa=1.0)
    r, _ = initial_chain(scaled(C0, shape=(40, 40, 40), wall_pos=20, nb=nb))
    o = orc.Oracle(cfg, r)
    o.relax(5000, 1.0)
    o.md_only(100)
    acc = 0.0
    for _ in range(200):
        o.md_only(1)
        v = o.beads()["v"]
        acc += (v * v).sum()
    ke = 0.5 * acc / 200
    want = 0.5 * kT * (3 * nb - (nb - 1))
    print(f"kinetic energy / (kT/2 (3N - (N-1))) = {ke / want:.4f}; / (kT/2 3N) = {ke / (1.5 * kT * nb):.4f}")
    assert abs(ke / want - 1) < 0.05
    assert not o.constraint_failed()


def test_constrained_coupled_run_conserves_momentum(orc):
    cfg = scaled(C0, shape=(16, 16, 16), wall_axis=-1, nb=10, n_sub=50, kT=1e-3, constraints=1)
    r, _ = initial_chain(scaled(C0, shape=(16, 16, 16), wall_pos=8, nb=10))
    rng = np.random.default_rng(5)
    o = orc.Oracle(cfg, r, 0.02 * rng.standard_normal(r.shape))
    P0 = o.observables()
    o.couple_step(20)
    P1 = o.observables()
    assert np.abs(P1[5:8] - P0[5:8]).max() > 1e-3
    # the constraint corrections are equal and opposite pairs along each bond,
    # kept apart from the positions, so the ledger closes to rounding
    assert np.abs((P1[1:4] + P1[5:8]) - (P0[1:4] + P0[5:8])).max() < 1e-12
    assert not o.constraint_failed()
