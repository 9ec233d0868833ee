"""Pins of the oracle's fluctuating fluid (the stochastic term of the lattice
Boltzmann equation in Sec. 2, in the mode formulation of Adhikari et al. the
paper builds on) against what the mathematics fixes: the mode basis is
orthogonal under the lattice weights with the textbook norms, the noise
leaves mass and momentum of every node unchanged, each mode receives exactly
its fluctuation-dissipation amplitude, and a periodic box at rest reaches
equipartition, <delta f_i^2> = 3 rho kT w_i, with every mode at 3 rho kT b_k.
CPU only."""
import numpy as np
import pytest

pytestmark = pytest.mark.filterwarnings("ignore")

# Norms b_k = sum_i w_i e_ki^2 of the D3Q19 mode basis (Duenweg, Schiller and
# Ladd, Phys. Rev. E 76, 036704 (2007), Table I): mass, momentum, bulk and
# shear stress, the two ghost vectors, the three ghost scalars.
B_LIT = np.array([1, 1 / 3, 1 / 3, 1 / 3, 2 / 3, 4 / 3, 4 / 9, 1 / 9, 1 / 9, 1 / 9,
                  2 / 3, 2 / 3, 2 / 3, 2 / 9, 2 / 9, 2 / 9, 2, 4 / 3, 4 / 9])


def _box(shape, **kw):
    from paper_0711_2665_amd.workloads import BASE
    c = dict(BASE)
    c.update(dict(shape=shape, wall_axis=-1, wall_pos=0, pore_h=0, nb=0, g=(0.0, 0.0, 0.0)))
    c.update(kw)
    return c


def test_mode_basis_is_orthogonal_with_textbook_norms(orc):
    E = orc.mode_basis()
    c, w, _ = orc.tables()
    # modes 0..3 are the density and the momentum components
    assert np.array_equal(E[0], np.ones(19))
    assert np.array_equal(E[1:4], c.T.astype(float))
    G = E @ np.diag(w) @ E.T
    assert np.abs(G - np.diag(np.diag(G))).max() < 1e-15
    assert np.allclose(np.diag(G), B_LIT, rtol=0, atol=1e-15)
    # the basis spans the 19 populations: f = W E^T diag(1/b) E f
    F = np.diag(w) @ E.T @ np.diag(1.0 / B_LIT) @ E
    assert np.allclose(F, np.eye(19), rtol=0, atol=1e-14)
    # the moments of every non-conserved mode vanish at the rest equilibrium
    assert np.abs(E[4:] @ w).max() < 1e-16


def test_fluid_normals_counter_layout(orc):
    """Block k of the node's normals is Philox-4x32-10 of the counter
    (n, node, k, 1) under the key (seed, replica); uniforms (x + 1/2) 2^-32;
    Box-Muller with the cosine first.  Word 3 = 1 keeps the stream apart from
    the bead noise, which uses word 3 = 0."""
    seed, rep, n, node = 77, 3, 12, 4321
    r = orc.fluid_normals(seed, rep, n, node)
    for k in range(4):
        x = np.array(orc.philox([n, node, k, 1], [seed, rep]), dtype=np.float64)
        u = (x + 0.5) / 2.0 ** 32
        ra, rb = np.sqrt(-2 * np.log(u[0])), np.sqrt(-2 * np.log(u[2]))
        want = [ra * np.cos(2 * np.pi * u[1]), ra * np.sin(2 * np.pi * u[1]),
                rb * np.cos(2 * np.pi * u[3]), rb * np.sin(2 * np.pi * u[3])]
        assert np.allclose(r[4 * k:4 * k + 4], want, rtol=1e-14, atol=1e-15)
    # distinct from the bead noise drawn with the same first counter words
    assert not np.allclose(r[:3], orc.gauss3(seed, rep, n, node, 0))


def test_fluid_normals_are_independent_standard_normals(orc):
    R = np.array([orc.fluid_normals(5, 0, n, node) for n in range(4) for node in range(2500)])
    m = R.shape[0]
    assert np.abs(R.mean(axis=0)).max() < 5 / np.sqrt(m)
    assert np.abs(R.var(axis=0) - 1).max() < 6 * np.sqrt(2 / m)
    C = np.corrcoef(R.T)
    assert np.abs(C - np.eye(16)).max() < 5 / np.sqrt(m)
    kurt = ((R - R.mean(0)) ** 4).mean(0) / R.var(0) ** 2
    assert np.abs(kurt - 3).max() < 6 * np.sqrt(24 / m)


def _modes(E, f):
    """Modes of a population field f[19, ...] per node."""
    return np.tensordot(E, f, axes=(1, 0))


@pytest.mark.parametrize("tau", [0.8, 1.0, 1.6])
def test_noise_has_the_fluctuation_dissipation_amplitude_per_mode(orc, tau):
    """One step from the same perturbed state with and without the fluid
    noise: at every node the difference carries no mass and no momentum, and
    its mode k is sqrt(3 rho kT (1 - (1 - omega)^2) b_k) times the node's
    normal number k - 4, rho the node's density."""
    shape = (5, 4, 3)
    kT = 2.5e-4
    E = orc.mode_basis()
    rng = np.random.default_rng(11)
    c, w, _ = orc.tables()
    f0 = w[:, None, None, None] * (1 + 0.05 * rng.standard_normal((19,) + shape[::-1]))
    a = orc.Oracle(_box(shape, tau=tau))
    b = orc.Oracle(_box(shape, tau=tau, fluid_kT=kT, seed=99, replica=2))
    a.set_pops(f0)
    b.set_pops(f0)
    a.lb_step()
    b.lb_step()
    d = b.pops() - a.pops()
    md = _modes(E, d)
    assert np.abs(md[:4]).max() < 1e-16
    # density of the node after pulling: the post-step mass of the noiseless run
    rho = a.pops().sum(axis=0)
    g2 = (1 - 1 / tau) ** 2
    nx, ny, nz = shape
    for z in range(nz):
        for y in range(ny):
            for x in range(nx):
                node = x + nx * (y + ny * z)
                r = orc.fluid_normals(99, 2, 0, node)
                amp = np.sqrt(3 * rho[z, y, x] * kT * (1 - g2) * B_LIT[4:])
                assert np.allclose(md[4:, z, y, x], amp * r[:15], rtol=1e-12, atol=1e-17)


def test_fluctuating_run_conserves_mass_and_momentum(orc):
    shape = (6, 5, 4)
    o = orc.Oracle(_box(shape, tau=0.9, fluid_kT=1e-3, seed=3))
    f0 = o.pops()
    o.lb_step(40)
    f = o.pops()
    c, _, _ = orc.tables()
    assert abs(f.sum() - f0.sum()) < 1e-11
    j = np.tensordot(c.T.astype(float), f, axes=(1, 0)).reshape(3, -1).sum(axis=1)
    assert np.abs(j).max() < 1e-12
    assert f.std() > 0


@pytest.mark.parametrize("tau", [1.0, 0.7])
def test_equipartition_in_a_periodic_box(orc, tau):
    """A periodic 8^3 box at rest with fluid noise reaches the Gaussian
    equilibrium of the linearised fluctuating lattice Boltzmann equation:
    every mode k has variance mu b_k, mu = 3 rho kT, except for the fixed
    totals (mass and momentum sums), which remove one of the N degrees of
    freedom of modes 0..3.  Checked over 1200 sampled steps after 300 steps
    of equilibration."""
    shape = (8, 8, 8)
    N = 512
    kT = 1e-4
    E = orc.mode_basis()
    o = orc.Oracle(_box(shape, tau=tau, fluid_kT=kT, seed=21))
    o.lb_step(300)
    acc = np.zeros(19)
    nsamp = 1200
    for _ in range(nsamp):
        o.lb_step()
        m = _modes(E, o.pops()).reshape(19, -1)
        m[0] -= 1.0
        acc += (m ** 2).mean(axis=1)
    var = acc / nsamp
    want = 3 * kT * B_LIT
    want[:4] *= 1 - 1 / N
    rel = var / want - 1
    assert np.abs(rel).max() < 0.02, rel
    # the kinetic energy per node and axis is kT / 2 (equipartition)
    ke = 0.5 * var[1:4]
    assert np.allclose(ke, 0.5 * kT * (1 - 1 / N), rtol=0.02)
