"""Pins of the oracle's bead observables against their definitions, on
hand-built chains (CPU).

Each expected value is computed here from the paper's definition, not by
calling the oracle's arithmetic:
  - bead temperature m <v^2> / 3 over 3 N degrees of freedom (Sec. 2, the
    monitored bead temperature) and the bead momentum;
  - the mean unwrapped normal coordinate and the translocated fraction
    (a bead is translocated when its unwrapped normal coordinate exceeds the
    wall plane);
  - N_r, the beads resident in the pore channel (Sec. 4.2, the resident
    monomers; the channel is the field region [w - 1.5, w + 1.5) along the
    normal times [lo - 0.5, hi + 0.5) on each transverse axis, in wrapped
    coordinates);
  - R_U and R_T, the radii of gyration of the untranslocated and
    translocated parts about their own centroids in unwrapped coordinates,
    and R_eff = (R_T^nu + R_U^nu)^(1/nu) with nu = 0.6 (Sec. 4.2,
    Eq. (R_eff));
  - dW_H/dt = gamma sum_i v_i . u_i and dW_E/dt = sum_i F_drive,i . v_i
    (Sec. 4.3), the drive acting along the wall normal on the beads in the
    channel only;
  - the viscous drag along the normal on each part, sum m gamma (u_p - v).n
    (Sec. 4.2, the drag forces on the two parts).

The chains are chosen so that each of these plausible mistakes changes the
value it touches by far more than the tolerance: centroids of wrapped
instead of unwrapped coordinates, R_eff with nu and 1/nu exchanged, the drag
with the opposite sign, the drive counted on beads outside the channel,
3 (N - 1) instead of 3 N degrees of freedom, the wrapped coordinate in the
translocation test, and a closed instead of half-open channel edge.
"""
import numpy as np
import pytest

NU = 0.6
TOL = 1e-13


def _cfg(wall_axis, shape, wall_pos, nb, mass=2.0, gamma=0.3, f_drive=0.05):
    return dict(shape=shape, wall_axis=wall_axis, wall_pos=wall_pos, pore_h=3, nb=nb, mass=mass, gamma=gamma,
                kT=0.0, f_drive=f_drive, n_sub=10, kappa=0.0, eps=0.0, tau=1.0, seed=5, relax_substeps=0)


def _channel(cfg, rp):
    """Whether a bead at rp (unwrapped) lies in the pore channel (wrapped
    coordinates, half-open box)."""
    a = cfg["wall_axis"]
    shape = cfg["shape"]
    t = [k for k in range(3) if k != a]
    w = cfg["wall_pos"]
    wn = rp[a] % shape[a]
    if not (w - 1.5 <= wn < w + 1.5):
        return False
    for k in t:
        n = shape[k]
        lo = n // 2 - cfg["pore_h"] // 2
        hi = lo + cfg["pore_h"] - 1
        wt = rp[k] % n
        if not (lo - 0.5 <= wt < hi + 0.5):
            return False
    return True


def _expected(cfg, r, v, up):
    a = cfg["wall_axis"]
    m, g, fd = cfg["mass"], cfg["gamma"], cfg["f_drive"]
    nb = len(r)
    tr = r[:, a] > cfg["wall_pos"]
    out = {}
    out[4] = m * float((v * v).sum()) / (3.0 * nb)
    out[5], out[6], out[7] = (m * v.sum(axis=0)).tolist()
    out[8] = float(r[:, a].mean())
    out[9] = float(tr.sum()) / nb
    inch = np.array([_channel(cfg, rp) for rp in r])
    out[10] = float(inch.sum())

    def rg(part):
        if part.sum() == 0:
            return 0.0
        x = r[part]
        c = x.mean(axis=0)
        return float(np.sqrt(((x - c) ** 2).sum(axis=1).mean()))

    RU, RT = rg(~tr), rg(tr)
    out[11], out[12] = RU, RT
    out[13] = (RT ** NU + RU ** NU) ** (1.0 / NU)
    out[14] = g * float((v * up).sum())
    out[15] = float((fd * v[inch, a]).sum())
    drag = m * g * (up[:, a] - v[:, a])
    out[23] = float(drag[~tr].sum())
    out[24] = float(drag[tr].sum())
    return out


def _check(orc, cfg, r, v, up):
    o = orc.Oracle(cfg, r, v)
    o.set_up(up)
    got = o.observables()
    want = _expected(cfg, r, v, up)
    for k, w in want.items():
        scale = max(1.0, abs(w))
        assert abs(got[k] - w) <= TOL * scale, (k, got[k], w)
    return got, want


def _straddling_chain(cfg, rng):
    """Ten beads: five on the cis side, five past the wall, with unwrapped
    coordinates outside the box on the transverse axes and along the normal
    (so that wrapping would move the centroids and flip a translocation)."""
    a = cfg["wall_axis"]
    t0, t1 = [k for k in range(3) if k != a]
    n = cfg["shape"]
    w = cfg["wall_pos"]
    r = np.zeros((10, 3))
    # untranslocated: normal below the plane; one bead at exactly w (not
    # translocated), one unwrapped a period below (wrapped it would lie
    # above the plane)
    r[:5, a] = [w - 3.2, w - 1.0, w, w - 0.5, w - n[a] + 2.25]
    # translocated: above the plane, one a period above
    r[5:, a] = [w + 0.25, w + 1.0, w + 2.5, w + n[a] + 0.75, w + 4.0]
    # transverse: a spread that crosses the box edges
    r[:, t0] = [n[t0] - 0.6, n[t0] + 0.9, 1.2, -0.8, 3.0, n[t0] / 2.0, n[t0] / 2.0 - 0.3, -1.7, n[t0] + 2.1, 0.4]
    r[:, t1] = [2.0, -0.4, n[t1] + 1.1, 0.3, n[t1] - 1.2, n[t1] / 2.0 + 0.2, 1.9, n[t1] + 0.6, -2.2, 5.5]
    # two beads in the channel (one of them through an unwrapped period)
    r[3] = 0.0
    r[3, a] = w - 0.5
    r[3, t0] = n[t0] // 2 + 0.3
    r[3, t1] = n[t1] // 2 - 0.4 + n[t1]
    r[5, t0] = n[t0] // 2 - 0.2
    r[5, t1] = n[t1] // 2 + 1.3
    v = rng.normal(0.0, 0.05, size=(10, 3))
    up = rng.normal(0.0, 0.02, size=(10, 3))
    return r, v, up


@pytest.mark.parametrize("wall_axis,shape,wall_pos", [(2, (16, 14, 20), 10), (0, (24, 12, 16), 12),
                                                        (1, (10, 18, 14), 9)])
def test_observables_of_a_straddling_chain(orc, wall_axis, shape, wall_pos):
    cfg = _cfg(wall_axis, shape, wall_pos, nb=10)
    r, v, up = _straddling_chain(cfg, np.random.default_rng(11 + wall_axis))
    got, want = _check(orc, cfg, r, v, up)
    # the chain is built so that both parts, the channel and the drive are
    # populated, and the drags have opposite signs to their negations
    assert 0.0 < got[9] < 1.0 and got[10] == 2.0
    assert got[11] > 1.0 and got[12] > 1.0 and want[15] != 0.0
    assert want[23] != 0.0 and want[24] != 0.0


def test_plausible_mistakes_would_fail(orc):
    """The expected values of the straddling chain differ from what each
    listed mistake would give by far more than the tolerance (so that the
    pin above rejects an oracle that makes it)."""
    cfg = _cfg(2, (16, 14, 20), 10, nb=10)
    r, v, up = _straddling_chain(cfg, np.random.default_rng(13))
    want = _expected(cfg, r, v, up)
    a = cfg["wall_axis"]
    n = np.array(cfg["shape"], dtype=float)
    rw = np.mod(r, n)
    tr = r[:, a] > cfg["wall_pos"]

    def rg(x):
        c = x.mean(axis=0)
        return float(np.sqrt(((x - c) ** 2).sum(axis=1).mean()))

    wrong = {
        11: rg(rw[~tr]),                                              # wrapped centroid
        12: rg(rw[tr]),
        13: (want[12] ** (1 / NU) + want[11] ** (1 / NU)) ** NU,      # nu and 1/nu exchanged
        23: -want[23], 24: -want[24],                                  # drag sign
        15: float((cfg["f_drive"] * v[:, a]).sum()),                  # drive on every bead
        4: cfg["mass"] * float((v * v).sum()) / (3.0 * (len(r) - 1)),  # 3 (N - 1)
        9: float((rw[:, a] > cfg["wall_pos"]).sum()) / len(r),       # wrapped translocation test
    }
    for k, w in wrong.items():
        assert abs(w - want[k]) > 1e3 * TOL * max(1.0, abs(want[k])), k


def test_channel_edges_are_half_open(orc):
    """N_r and dW_E/dt at the exact edges of the channel: the lower edges
    belong to it, the upper ones do not, along the normal and both
    transverse axes, in wrapped coordinates."""
    cfg = _cfg(2, (16, 14, 20), 10, nb=8)
    w = 10
    lo0, hi0 = 16 // 2 - 1, 16 // 2 + 1
    lo1, hi1 = 14 // 2 - 1, 14 // 2 + 1
    cx, cy = 8.0, 7.0
    r = np.array([
        [cx, cy, w - 1.5],              # lower normal edge: in
        [cx, cy, w + 1.5],              # upper normal edge: out
        [lo0 - 0.5, cy, w],             # lower x edge: in
        [hi0 + 0.5, cy, w],             # upper x edge: out
        [cx, lo1 - 0.5, w + 1.0],       # lower y edge: in
        [cx, hi1 + 0.5, w + 1.0],       # upper y edge: out
        [cx + 16.0, cy - 14.0, w + 20.0],  # wrapped into the channel: in
        [cx, cy, w - 1.5 - 1e-9],       # just below the lower normal edge: out
    ])
    v = np.tile([0.0, 0.0, 0.1], (8, 1)) + np.arange(8)[:, None] * np.array([0.0, 0.0, 0.01])
    up = np.zeros((8, 3))
    got, want = _check(orc, cfg, r, v, up)
    assert got[10] == 4.0
    inside = [0, 2, 4, 6]
    assert abs(got[15] - cfg["f_drive"] * v[inside, 2].sum()) <= TOL


@pytest.mark.parametrize("side", ["cis", "trans"])
def test_one_part_empty(orc, side):
    """A chain entirely on one side: the radius of the empty part is 0, R_eff
    is the other radius, the drag of the empty part is 0."""
    cfg = _cfg(2, (16, 14, 20), 10, nb=6)
    rng = np.random.default_rng(3)
    r = rng.uniform(2.0, 12.0, size=(6, 3))
    r[:, 2] = rng.uniform(2.0, 8.0, size=6) + (0.0 if side == "cis" else 9.0)
    v = rng.normal(0, 0.03, size=(6, 3))
    up = rng.normal(0, 0.01, size=(6, 3))
    got, want = _check(orc, cfg, r, v, up)
    empty, full = (12, 11) if side == "cis" else (11, 12)
    assert got[empty] == 0.0
    assert abs(got[13] - got[full]) <= 1e-13 * got[full]
    assert got[24 if side == "cis" else 23] == 0.0
