"""Pins of the oracle's bead part and of the bead <-> fluid coupling: closed
forms of the integrator, interpolation identities, force laws against their
energies, momentum ledgers, equipartition, the noise generator against an
independent implementation, and the forward-mode derivative against finite
differences.  CPU only."""
import math
import os
import shutil
import subprocess
import tempfile

import numpy as np
import pytest

from paper_0711_2665_amd.workloads import BASE, C0, initial_chain, scaled


def _cfg(shape, **kw):
    c = dict(BASE)
    c.update(dict(shape=shape, wall_axis=-1, wall_pos=0, pore_h=0, nb=0))
    c.update(kw)
    return c


# -- P9: Ornstein-Uhlenbeck kick with a frozen fluid velocity.  One free bead,
#    kT = 0, the fluid at the uniform equilibrium of velocity u0: after s
#    sub-steps v = u0 + (v0 - u0) e^s with e = exp(-gamma h), and the position
#    advances by h/2 (v_k + v_{k+1}) per sub-step (Eq. (SPValgo)).

def test_ou_closed_form(orc):
    u0 = np.array([0.01, -0.02, 0.005])
    v0 = np.array([0.1, 0.05, -0.03])
    cfg = _cfg((8, 8, 8), nb=1, kT=0.0, gamma=0.3, n_sub=37)
    o = orc.Oracle(cfg, np.array([[3.3, 4.1, 2.7]]), v0[None])
    f = np.stack([orc.feq(1.0, u0)] * 512, axis=1)
    o.set_pops(f)
    o.couple_step(1)
    b = o.beads()
    h = 1 / 37
    e = math.exp(-0.3 * h)
    vs = [u0 + (v0 - u0) * e ** k for k in range(38)]
    r = np.array([3.3, 4.1, 2.7]) + sum(h / 2 * (vs[k] + vs[k + 1]) for k in range(37))
    assert np.allclose(b["up"][0], u0, rtol=0, atol=1e-16)
    assert np.allclose(b["v"][0], vs[-1], rtol=1e-13, atol=0)
    assert np.allclose(b["r"][0], r, rtol=1e-14, atol=0)
    # the impulse handed to the fluid is minus the bead's momentum change
    assert np.allclose(b["J"][0], -(vs[-1] - v0), rtol=1e-12, atol=1e-18)


# -- P10: position Verlet on a harmonic dimer (gamma = 0, kT = 0, no LJ): the
#    stretch at full steps is x0 cos(n theta) with cos theta = 1 - (h w)^2 / 2,
#    w^2 = 2 k / m (the exact solution of the linear map)

def test_harmonic_dimer_position_verlet(orc):
    k, m, n_sub = 100.0, 1.0, 40
    x0 = 0.05
    cfg = _cfg((16, 16, 16), nb=2, k_bond=k, mass=m, eps=0.0, gamma=0.0, kT=0.0, n_sub=n_sub)
    r = np.array([[5.0, 7.0, 7.0], [6.0 + x0, 7.0, 7.0]])
    o = orc.Oracle(cfg, r, np.zeros((2, 3)))
    h = 1 / n_sub
    theta = math.acos(1 - (h * math.sqrt(2 * k / m)) ** 2 / 2)
    for n in range(1, 6):
        o.couple_step(1)
        b = o.beads()
        stretch = np.linalg.norm(b["r"][1] - b["r"][0]) - 1.0
        assert abs(stretch - x0 * math.cos(n * n_sub * theta)) < 1e-12
        assert np.abs(b["r"][:, 1:] - 7.0).max() == 0.0
        assert np.abs(b["J"]).max() == 0.0


# -- P11: trilinear stencil identities; gather is the transpose of spread

def test_trilinear_stencil_identities(orc):
    cfg = _cfg((6, 5, 7), nb=1)
    o = orc.Oracle(cfg, np.zeros((1, 3)))
    rng = np.random.default_rng(3)
    L = np.array([6, 5, 7])
    for _ in range(50):
        rp = rng.uniform(-20, 20, 3)
        nodes, W = o.stencil(rp)
        assert abs(W.sum() - 1) < 1e-15 and W.min() >= 0
        w = rp - L * np.floor(rp / L)
        b = np.floor(w)
        corners = np.array([[k & 1, (k >> 1) & 1, (k >> 2) & 1] for k in range(8)], dtype=float) + b
        assert np.allclose(W @ corners, w, rtol=0, atol=1e-13)
        a0, g = rng.standard_normal(), rng.standard_normal(3)
        assert abs(W @ (a0 + corners @ g) - (a0 + w @ g)) < 1e-12
        # node indices are the wrapped corners
        cw = corners.astype(int) % L
        assert np.array_equal(nodes, cw[:, 0] + 6 * (cw[:, 1] + 5 * cw[:, 2]))


def test_gather_is_transpose_of_spread(orc):
    cfg = scaled(C0, shape=(12, 10, 14), wall_pos=7, nb=9)
    r, _ = initial_chain(cfg)
    o = orc.Oracle(cfg, r)
    rng = np.random.default_rng(4)
    _, w, _ = orc.tables()
    f = w[:, None] * (1 + 0.05 * rng.standard_normal((19, o.N)))
    o.set_pops(f)
    U = o.node_velocity_field().reshape(3, -1)
    assert not np.any(U[:, o.flags().reshape(-1) == 1])
    up = o.gather()
    for p in range(cfg["nb"]):
        nodes, W = o.stencil(r[p])
        acc = np.zeros(3)
        for k in range(8):
            acc = acc + W[k] * U[:, nodes[k]]
        assert np.allclose(up[p], acc, rtol=0, atol=1e-16)
    J = rng.standard_normal((cfg["nb"], 3))
    F = o.spread(J).reshape(3, -1)
    lhs = math.fsum((up * J).ravel())
    rhs = math.fsum((U * F).ravel())
    assert abs(lhs - rhs) < 1e-14 * (abs(lhs) + 1e-3)


# -- nearest-grid-point transfer (Sec. 2, the particle/grid paragraph): u_p
#    is the fluid velocity at the node nearest to the bead (round half up,
#    periodic), and J goes back to that node alone; momentum is conserved

def _nearest_node(rp, L):
    w = rp - L * np.floor(rp / L)
    n = np.floor(w + 0.5).astype(int) % L
    return n[0] + L[0] * (n[1] + L[1] * n[2])


def test_ngp_gather_takes_the_nearest_node(orc):
    cfg = scaled(C0, shape=(12, 10, 14), wall_pos=7, nb=1, coupling=1)
    o = orc.Oracle(cfg, np.zeros((1, 3)))
    L = np.array([12, 10, 14])
    rng = np.random.default_rng(8)
    _, w, _ = orc.tables()
    o.set_pops(w[:, None] * (1 + 0.05 * rng.standard_normal((19, o.N))))
    U = o.node_velocity_field().reshape(3, -1)
    pts = [rng.uniform(-30, 30, 3) for _ in range(40)]
    pts += [np.array([3.5, 2.5, 6.5]), np.array([11.7, 9.6, 13.5]), np.array([-0.5, 4.49999, 7.0])]
    for rp in pts:
        o.set_beads(rp[None, :], np.zeros((1, 3)))
        up = o.gather()[0]
        assert np.array_equal(up, U[:, _nearest_node(rp, L)]), rp


def test_ngp_spread_is_the_transpose_and_conserves_momentum(orc):
    cfg = scaled(C0, shape=(12, 10, 14), wall_pos=7, nb=9, coupling=1)
    r, _ = initial_chain(cfg)
    o = orc.Oracle(cfg, r)
    rng = np.random.default_rng(9)
    J = rng.standard_normal((cfg["nb"], 3))
    F = o.spread(J).reshape(3, -1)
    want = np.zeros_like(F)
    L = np.array([12, 10, 14])
    solid = o.flags().reshape(-1) == 1
    for p in range(cfg["nb"]):
        n = _nearest_node(r[p], L)
        if not solid[n]:
            want[:, n] += J[p]
    assert np.allclose(F, want, rtol=0, atol=1e-15)
    # a coupled run in a periodic box conserves fluid + bead momentum
    cfg2 = scaled(C0, shape=(16, 16, 16), wall_axis=-1, nb=10, n_sub=50, kT=1e-3, coupling=1)
    r2, _ = initial_chain(scaled(C0, shape=(16, 16, 16), wall_pos=8, nb=10))
    o2 = orc.Oracle(cfg2, r2, 0.02 * rng.standard_normal(r2.shape))
    P0 = o2.observables()
    o2.couple_step(20)
    P1 = o2.observables()
    assert np.abs(P1[5:8] - P0[5:8]).max() > 1e-3
    assert np.abs((P1[1:4] + P1[5:8]) - (P0[1:4] + P0[5:8])).max() < 1e-12


# -- P12: force laws.  Cell list and all-pairs give the same LJ sums bitwise;
#    internal forces sum to zero; every force is minus the gradient of its
#    energy (central differences).

def _relaxed(cfg, nsub=400):
    r, v = initial_chain(cfg)
    from oracle import Oracle
    o = Oracle(cfg, r, v)
    o.relax(nsub, 1.0)
    return o


def test_lj_cell_list_equals_all_pairs_bitwise(orc):
    cfg = scaled(C0, shape=(40, 40, 40), wall_pos=20, nb=600)
    o = _relaxed(cfg, 200)
    a = o.lj_forces(cells=False)
    b = o.lj_forces(cells=True)
    assert np.array_equal(a, b)
    assert np.abs(a).max() > 1.0   # bonded neighbours overlap the LJ range


def test_internal_forces_sum_to_zero(orc):
    cfg = scaled(C0, shape=(40, 40, 40), wall_axis=-1, nb=200)
    r, _ = initial_chain(scaled(C0, shape=(40, 40, 40), wall_pos=20, nb=200))
    o = orc.Oracle(cfg, r + np.array([0.0, 0.0, 0.0]))
    F = o.forces(field_on=False)
    assert np.abs(F.sum(axis=0)).max() < 1e-12 * np.abs(F).max() * 200
    lj = o.lj_forces(cells=False)
    assert np.abs(lj.sum(axis=0)).max() < 1e-13 * np.abs(lj).max() * 200


@pytest.mark.parametrize("seed", [0, 1])
def test_forces_are_minus_energy_gradient(orc, seed):
    cfg = scaled(C0, shape=(16, 16, 16), wall_pos=8, nb=12, n_sub=50)
    r, _ = initial_chain(cfg)
    rng = np.random.default_rng(seed)
    r = r + 0.08 * rng.standard_normal(r.shape)
    r[0] = [8.0, 9.6, 7.05]  # next to the solid site (8, 10, 8) at the pore rim
    o = orc.Oracle(cfg, r)
    F = o.forces(field_on=False)
    d = 1e-6
    G = np.zeros_like(r)
    for p in range(cfg["nb"]):
        for a in range(3):
            rp = r.copy(); rp[p, a] += d
            rm = r.copy(); rm[p, a] -= d
            o.set_beads(rp); ep = o.energy()
            o.set_beads(rm); em = o.energy()
            G[p, a] = -(ep - em) / (2 * d)
    o.set_beads(r)
    assert np.abs(F - G).max() < 1e-6 * np.abs(F).max(), np.abs(F - G).max()
    # the wall force on bead 0 is present and pushes it away from the site
    o2 = orc.Oracle(scaled(cfg, wall_axis=-1), r)
    dF = o.forces(False)[0] - o2.forces(False)[0]
    assert dF[1] < -1.0 and dF[2] < -1.0 and abs(dF[0]) < 1e-12


def test_field_region_reading(orc):
    # the pore channel: [wall - 1.5, wall + 1.5) along the normal, the pore
    # opening [lo - 0.5, hi + 0.5) across (lo..hi = 15..17 for a 3-wide pore
    # centred in 32)
    cfg = scaled(C0, nb=1)
    o = orc.Oracle(cfg, np.zeros((1, 3)))
    inside = [(16, 16, 16), (14.5, 17.49, 14.5), (16, 16, 17.49), (16 + 32, 16 - 64, 16)]
    outside = [(16, 16, 14.49), (16, 16, 17.5), (14.49, 16, 16), (17.5, 16, 16), (16, 10, 16)]
    for p in inside:
        assert o.in_field(np.array(p, dtype=float)), p
    for p in outside:
        assert not o.in_field(np.array(p, dtype=float)), p


# -- wall repulsion: the truncated LJ of every solid site within r_c,
#    against a brute-force sum over all solid sites of the lattice (minimum
#    image), for cut-offs up to the largest the library accepts (r_c <= 3:
#    the paper's sigma = 1.8 gives r_c = 2^(1/6) 1.8 > 2)

@pytest.mark.parametrize("sigma", [1.0, 1.8, 2.6])
def test_wall_force_equals_brute_force_over_every_site(orc, sigma):
    rc = 2.0 ** (1.0 / 6.0) * sigma
    eps = 1e-4 if sigma > 1.0 else 1.0
    cfg = scaled(C0, shape=(24, 20, 22), wall_axis=1, wall_pos=10, pore_h=3, nb=1, sigma=sigma, rc=rc, eps=eps)
    o = orc.Oracle(cfg, np.zeros((1, 3)))
    solid = np.argwhere(o.flags() == 1)[:, ::-1].astype(float)      # (x, y, z) of every solid node
    ext = np.array([24.0, 20.0, 22.0])
    rng = np.random.default_rng(int(10 * sigma))
    pts = [np.array([12.3, 10 + dy, 11.7]) for dy in (-2.9, -2.2, -1.5, -0.6, 0.4, 1.1, 2.5, 3.3)]
    # beads inside the pore, near the wall plane: the nearest solid sites lie
    # two nodes below the base node along x or z, just inside r_c = 2.02
    pts += [np.array([12.005, 10.1, 11.0]), np.array([12.0, 9.9, 10.003])]
    pts += [np.array([10.6 + rng.random() * 3, 8.0 + rng.random() * 4, 9.6 + rng.random() * 3]) for _ in range(12)]
    for rp in pts:
        o.set_beads(rp[None, :], np.zeros((1, 3)))
        got = o.forces(field_on=False)[0]
        d = rp[None, :] - solid
        d -= ext * np.round(d / ext)
        r2 = (d * d).sum(1)
        near = r2 < rc * rc
        sr6 = (sigma ** 2 / r2[near]) ** 3
        want = ((24 * eps * (2 * sr6 * sr6 - sr6) / r2[near])[:, None] * d[near]).sum(0)
        scale = max(1.0, np.abs(want).max())
        assert np.abs(got - want).max() <= 1e-12 * scale, (rp, got, want, int(near.sum()))


# -- P8: momentum ledger.  In a periodic box without walls the fluid + bead
#    momentum is conserved; with walls (field off, beads away from them) the
#    bounce-back ledger closes the balance (halfway bounce-back hands the
#    wall 2 f c per reflected population).

def test_momentum_conserved_without_walls(orc):
    cfg = scaled(C0, shape=(16, 16, 16), wall_axis=-1, nb=10, n_sub=50, kT=1e-3)
    r, _ = initial_chain(scaled(C0, shape=(16, 16, 16), wall_pos=8, nb=10))
    rng = np.random.default_rng(5)
    o = orc.Oracle(cfg, r, 0.02 * rng.standard_normal(r.shape))
    P0 = o.observables()
    o.couple_step(20)
    P1 = o.observables()
    tot0 = P0[1:4] + P0[5:8]
    tot1 = P1[1:4] + P1[5:8]
    assert np.abs(P1[5:8] - P0[5:8]).max() > 1e-3      # momentum did move
    assert np.abs(tot1 - tot0).max() < 1e-12, tot1 - tot0


def test_momentum_ledger_with_walls(orc):
    cfg = scaled(C0, shape=(16, 16, 16), wall_pos=8, nb=6, n_sub=50, f_drive=0.0, kT=1e-3)
    r = np.array([[3.0 + k, 5.0, 3.5] for k in range(6)])   # far from the wall
    rng = np.random.default_rng(6)
    o = orc.Oracle(cfg, r, 0.05 * rng.standard_normal(r.shape))
    P0 = o.observables()
    o.couple_step(40)
    P1 = o.observables()

    def total(P):
        return P[1:4] + P[5:8] + P[16:19] + P[19:22]

    assert np.abs(P1[16:19]).max() > 1e-6                 # the wall took momentum
    # the ledger is a running FP64 sum of ~1e5 terms 2 f c (|f| ~ 0.03) with
    # partial sums up to ~1e2, so its own rounding is ~1e-11; a wrong
    # reflection index would break the balance at the 1e-3 level
    assert np.abs(total(P1) - total(P0)).max() < 5e-11


def test_momentum_ledger_with_beads_on_the_wall(orc):
    """The spread-on-solid term of the ledger: without bead LJ (so no wall
    force) and without field, beads straddling the solid part of the wall
    drop part of their impulse on solid nodes; fluid + beads + both wall
    ledgers still conserve momentum."""
    cfg = scaled(C0, shape=(16, 16, 16), wall_pos=8, nb=6, n_sub=50, f_drive=0.0, kT=1e-3, eps=0.0)
    r = np.array([[2.3 + 0.9 * k, 3.4, 7.6 + 0.12 * k] for k in range(6)])
    rng = np.random.default_rng(6)
    o = orc.Oracle(cfg, r, 0.05 * rng.standard_normal(r.shape))
    P0 = o.observables()
    o.couple_step(40)
    P1 = o.observables()

    def total(P):
        return P[1:4] + P[5:8] + P[16:19] + P[19:22]

    assert np.abs(P1[19:22]).max() > 1e-6                 # impulse fell on the wall
    assert np.abs(total(P1) - total(P0)).max() < 5e-11
    # without the spread-on-solid term the balance fails by that term
    part = P1[1:4] + P1[5:8] + P1[16:19] - (P0[1:4] + P0[5:8] + P0[16:19])
    assert np.abs(part).max() > 1e-7


# -- P13: equipartition of free beads under the OU kick: starting from rest,
#    <v_a^2> = kT/m (1 - exp(-2 gamma t)) exactly in expectation

def test_equipartition_free_beads(orc):
    nb = 2000
    g = np.stack(np.meshgrid(np.arange(20), np.arange(10), np.arange(10), indexing="ij"), -1).reshape(-1, 3)
    r = 2.0 * g[:nb] + 0.5
    cfg = _cfg((40, 40, 40), nb=nb, k_bond=0.0, kappa=0.0, eps=0.0, kT=2e-4, gamma=0.1, n_sub=20)
    o = orc.Oracle(cfg, r)
    nsteps = 10
    o.md_only(nsteps)
    v = o.beads()["v"]
    want = 2e-4 * (1 - math.exp(-2 * 0.1 * nsteps))
    m2 = (v ** 2).mean()
    sd = want * math.sqrt(2 / v.size)
    assert abs(m2 - want) < 3.5 * sd, (m2, want)
    assert abs(v.mean()) < 3.5 * math.sqrt(want / v.size)


# -- Philox4x32-10 against an independent implementation (rocRAND's engine,
#    compiled from its headers for the host) and the Gaussian transform's
#    distribution

_PHILOX_REF = r'''
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>
int main() {
  unsigned k0, k1, c0, c1, c2, c3;
  while (std::scanf("%u %u %u %u %u %u", &k0, &k1, &c0, &c1, &c2, &c3) == 6) {
    rocrand_state_philox4x32_10 st;
    unsigned long long seed = (unsigned long long)k0 | ((unsigned long long)k1 << 32);
    unsigned long long sub = (unsigned long long)c2 | ((unsigned long long)c3 << 32);
    unsigned long long blk = (unsigned long long)c0 | ((unsigned long long)c1 << 32);
    rocrand_init(seed, sub, 0ull, &st);
    // advance by blk blocks of four outputs without overflowing 64 bits
    for (int k = 0; k < 4; ++k) skipahead(blk, &st);
    uint4 r = rocrand4(&st);
    std::printf("%u %u %u %u\n", r.x, r.y, r.z, r.w);
  }
  return 0;
}
'''


def test_philox_matches_independent_implementation(orc):
    inc = "/opt/rocm/include"
    if not shutil.which("g++") or not os.path.exists(os.path.join(inc, "rocrand", "rocrand_philox4x32_10.h")):
        pytest.skip("no host compiler or rocRAND headers")
    rng = np.random.default_rng(7)
    cases = [(0, 0, 0, 0, 0, 0), (2**32 - 1,) * 6]
    cases += [tuple(int(x) for x in rng.integers(0, 2**32, 6, dtype=np.uint64)) for _ in range(300)]
    with tempfile.TemporaryDirectory() as d:
        src = os.path.join(d, "ref.cpp")
        exe = os.path.join(d, "ref")
        open(src, "w").write(_PHILOX_REF)
        subprocess.check_call(["g++", "-O1", "-std=c++17", "-D__HIP_PLATFORM_AMD__", "-I" + inc, src, "-o", exe])
        inp = "\n".join(" ".join(str(x) for x in c) for c in cases) + "\n"
        out = subprocess.run([exe], input=inp, capture_output=True, text=True, check=True).stdout.split("\n")
    for c, line in zip(cases, out):
        k0, k1, c0, c1, c2, c3 = c
        want = [int(x) for x in line.split()]
        assert orc.philox([c0, c1, c2, c3], [k0, k1]) == want, c


def test_gaussian_noise_distribution(orc):
    from scipy import stats
    xs = np.array([orc.gauss3(99, 3, n, s, p) for n in range(4) for s in range(25) for p in range(40)])
    assert xs.shape == (4000, 3)
    for a in range(3):
        assert abs(xs[:, a].mean()) < 4 / math.sqrt(4000)
        assert abs(xs[:, a].var() - 1) < 4 * math.sqrt(2 / 4000)
        assert stats.kstest(xs[:, a], "norm").pvalue > 1e-4
    # counter and key both matter
    assert not np.array_equal(orc.gauss3(99, 3, 0, 0, 0), orc.gauss3(99, 4, 0, 0, 0))
    assert not np.array_equal(orc.gauss3(99, 3, 0, 0, 0), orc.gauss3(99, 3, 1, 0, 0))


# -- forward-mode derivative of the loss (mean normal coordinate at the end)
#    against central finite differences of the plain FP64 run

def _loss(orc, cfg, r0, v0, nsteps, gamma=None, fdrive=None):
    c = dict(cfg)
    if gamma is not None:
        c["gamma"] = gamma
    if fdrive is not None:
        c["f_drive"] = fdrive
    o = orc.Oracle(c, r0, v0)
    o.couple_step(nsteps)
    return o.beads()["r"][:, c["wall_axis"]].mean()


def test_jvp_matches_finite_differences(orc):
    cfg = scaled(C0, shape=(16, 16, 16), wall_pos=8, nb=5, n_sub=50)
    r, v = initial_chain(cfg)
    o = orc.Oracle(cfg, r, v)
    o.relax(500, 1.0)
    r0 = o.beads()["r"]
    v0 = np.zeros_like(r0)
    nsteps = 4
    h = 1e-6
    L, dg = orc.jvp(cfg, r0, v0, nsteps, dgamma=1.0)
    assert abs(L - _loss(orc, cfg, r0, v0, nsteps)) < 1e-14
    fd = (_loss(orc, cfg, r0, v0, nsteps, gamma=cfg["gamma"] + h) -
          _loss(orc, cfg, r0, v0, nsteps, gamma=cfg["gamma"] - h)) / (2 * h)
    assert abs(dg - fd) < 1e-6 * abs(fd) + 1e-11, (dg, fd)
    _, dfd = orc.jvp(cfg, r0, v0, nsteps, dfdrive=1.0)
    fd = (_loss(orc, cfg, r0, v0, nsteps, fdrive=cfg["f_drive"] + h) -
          _loss(orc, cfg, r0, v0, nsteps, fdrive=cfg["f_drive"] - h)) / (2 * h)
    assert abs(dfd - fd) < 1e-6 * abs(fd) + 1e-11, (dfd, fd)
    rng = np.random.default_rng(8)
    dr = rng.standard_normal(r0.shape)
    _, dd = orc.jvp(cfg, r0, v0, nsteps, dr0=dr)
    fd = (_loss(orc, cfg, r0 + h * dr, v0, nsteps) - _loss(orc, cfg, r0 - h * dr, v0, nsteps)) / (2 * h)
    assert abs(dd - fd) < 1e-6 * abs(fd) + 1e-11, (dd, fd)
