"""P6: brute force on a 4^3 lattice.  One coupled step written a second time,
in a different form, straight from the definitions: streaming by whole-array
shifts (np.roll) instead of per-node pulls, moments by tensor contraction,
the bending force from the arccos form of the angle, the wall term by a
sweep over every solid site instead of a local window.  It must agree with
the oracle to rounding, on random populations, a wall with a pore, three
beads near the pore (field, wall and bead-bead terms all active) and noise.
CPU only."""
import itertools
import math

import numpy as np

from paper_0711_2665_amd.workloads import BASE

# textbook D3Q19: rest, 6 face neighbours (1/18), 12 edge neighbours (1/36)
VELS = [(0, 0, 0)] + [p for p in itertools.product((-1, 0, 1), repeat=3) if sum(map(abs, p)) == 1] \
    + [p for p in itertools.product((-1, 0, 1), repeat=3) if sum(map(abs, p)) == 2]
WTS = {0: 1 / 3, 1: 1 / 18, 2: 1 / 36}


def _tables_in_oracle_order(orc):
    c, _, _ = orc.tables()
    idx = [VELS.index(tuple(x)) for x in c]
    cv = np.array([VELS[k] for k in idx], dtype=float)
    w = np.array([WTS[int(np.abs(x).sum())] for x in cv])
    opp = np.array([[tuple(-x) for x in cv].index(tuple(y)) for y in cv])
    return cv, w, opp


def brute_step(cfg, f, solid, r, v, orc, step_index):
    """One coupled step: gather, MD sub-cycle, spread, stream+collide."""
    cv, w, opp = _tables_in_oracle_order(orc)
    nx, ny, nz = cfg["shape"]
    L = np.array([nx, ny, nz], dtype=float)
    nb = len(r)
    # --- pulled populations by whole-array shifts; arrays are [z, y, x]
    def shift(a, c):
        return np.roll(a, shift=(int(c[2]), int(c[1]), int(c[0])), axis=(0, 1, 2))

    pulled = np.empty_like(f)
    for i in range(19):
        from_solid = shift(solid, cv[i]).astype(bool)
        pulled[i] = np.where(from_solid, f[opp[i]], shift(f[i], cv[i]))
    rho = pulled.sum(axis=0)
    u = np.einsum("izyx,ia->azyx", pulled, cv) / rho
    u_nodes = np.where(solid[None].astype(bool), 0.0, u)

    # --- trilinear gather at r(n)
    def stencil(p):
        wpos = p - L * np.floor(p / L)
        b = np.floor(wpos).astype(int)
        d = wpos - b
        out = []
        for k in range(8):
            o = np.array([k & 1, (k >> 1) & 1, (k >> 2) & 1])
            node = (b + o) % np.array([nx, ny, nz])
            wt = np.prod(np.where(o == 1, d, 1 - d))
            out.append((node, wt))
        return out

    up = np.zeros((nb, 3))
    for p in range(nb):
        for node, wt in stencil(r[p]):
            up[p] += wt * u_nodes[:, node[2], node[1], node[0]]

    # --- forces
    sites = np.argwhere(solid.astype(bool))[:, ::-1].astype(float)  # (x, y, z)
    rc2 = cfg["rc"] ** 2

    def lj(dvec):
        r2 = dvec @ dvec
        if r2 >= rc2:
            return np.zeros(3)
        s6 = (cfg["sigma"] ** 2 / r2) ** 3
        return 24 * cfg["eps"] * (2 * s6 * s6 - s6) / r2 * dvec

    def angle_grad(a, b, c):
        # theta = arccos(b1.b2 / |b1||b2|), gradient w.r.t. a, b, c
        b1, b2 = b - a, c - b
        n1, n2 = np.linalg.norm(b1), np.linalg.norm(b2)
        cs = b1 @ b2 / (n1 * n2)
        th = math.acos(max(-1.0, min(1.0, cs)))
        dcs_db1 = b2 / (n1 * n2) - cs * b1 / n1 ** 2
        dcs_db2 = b1 / (n1 * n2) - cs * b2 / n2 ** 2
        k = -1.0 / math.sin(th)
        g1, g2 = k * dcs_db1, k * dcs_db2
        return th, -g1, g1 - g2, g2

    def force(pos, field_on=True):
        F = np.zeros((nb, 3))
        for p in range(nb - 1):
            d = pos[p + 1] - pos[p]
            dist = np.linalg.norm(d)
            fb = cfg["k_bond"] * (dist - cfg["r0"]) * d / dist
            F[p] += fb
            F[p + 1] -= fb
        for q in range(1, nb - 1):
            th, ga, gb, gc = angle_grad(pos[q - 1], pos[q], pos[q + 1])
            F[q - 1] -= cfg["kappa"] * th * ga
            F[q] -= cfg["kappa"] * th * gb
            F[q + 1] -= cfg["kappa"] * th * gc
        for p in range(nb):
            for j in range(nb):
                if j != p:
                    d = pos[p] - pos[j]
                    d -= L * np.floor(d / L + 0.5)
                    F[p] += lj(d)
            wpos = pos[p] - L * np.floor(pos[p] / L)
            for s in sites:
                d = wpos - s
                d -= L * np.floor(d / L + 0.5)
                F[p] += lj(d)
            a = cfg["wall_axis"]
            tn = [t for t in range(3) if t != a]
            lo = [cfg["shape"][t] // 2 - cfg["pore_h"] // 2 for t in tn]
            hi = [x + cfg["pore_h"] - 1 for x in lo]
            inside = cfg["wall_pos"] - 1.5 <= wpos[a] < cfg["wall_pos"] + 1.5 and all(
                lo[k] - 0.5 <= wpos[tn[k]] < hi[k] + 0.5 for k in range(2))
            if field_on and inside:
                F[p, a] += cfg["f_drive"]
        return F

    # --- MD sub-cycle with u_p frozen
    h = 1.0 / cfg["n_sub"]
    g, m, kT = cfg["gamma"], cfg["mass"], cfg["kT"]
    e = math.exp(-g * h)
    sig = math.sqrt(kT / m * (1 - e * e))
    rs = r.copy()
    J = np.zeros((nb, 3))
    r = r.copy()
    v = v.copy()
    for s in range(cfg["n_sub"]):
        r = r + h / 2 * v
        F = force(r)
        for p in range(nb):
            xi = orc.gauss3(cfg["seed"], cfg["replica"], step_index, s, p)
            vo = v[p].copy()
            v[p] = e * vo + (1 - e) / (m * g) * (F[p] + g * up[p]) + sig * xi
            J[p] -= m * ((1 - e) * (up[p] - vo) + sig * xi)
        r = r + h / 2 * v

    # --- spread at r(n)
    Fl = np.zeros((3, nz, ny, nx))
    for p in range(nb):
        for node, wt in stencil(rs[p]):
            if not solid[node[2], node[1], node[0]]:
                Fl[:, node[2], node[1], node[0]] += wt * J[p]

    # --- collide
    usq = (u ** 2).sum(axis=0)
    cu = np.einsum("ia,azyx->izyx", cv, u)
    feq = w[:, None, None, None] * rho * (1 + 3 * cu + 4.5 * cu ** 2 - 1.5 * usq)
    Ft = Fl + np.array(cfg["g"])[:, None, None, None]
    src = 3 * w[:, None, None, None] * np.einsum("ia,azyx->izyx", cv, Ft)
    post = pulled - (pulled - feq) / cfg["tau"] + src
    fnew = np.where(solid[None].astype(bool), f, post)
    return fnew, r, v, J, up


def test_bruteforce_4cube_coupled_step(orc):
    cfg = dict(BASE)
    cfg.update(shape=(4, 4, 4), wall_axis=2, wall_pos=2, pore_h=2, nb=3, n_sub=16, kT=1e-3,
               tau=0.9, g=(1e-4, -2e-4, 5e-5), kappa=0.5)
    # bonds of length 1.04 (inside the LJ range), beads 0 and 2 in the pore
    # channel (field on), bead 2 within r_c of the solid site (3, 2, 2)
    r = np.array([[1.37, 1.6, 1.53], [1.895, 1.285, 0.69], [2.311, 2.116, 1.158]])
    rng = np.random.default_rng(42)
    v = 0.01 * rng.standard_normal((3, 3))
    o = orc.Oracle(cfg, r, v)
    _, w, _ = orc.tables()
    f = w[:, None, None, None] * (1 + 0.1 * rng.standard_normal((19, 4, 4, 4)))
    o.set_pops(f)
    solid = o.flags()
    # the geometry is a plane at z = 2 with a 2x2 pore at x, y in {1, 2}
    want = np.zeros((4, 4, 4), dtype=np.uint8)
    want[2] = 1
    want[2, 1:3, 1:3] = 0
    assert np.array_equal(solid, want)
    for step in range(2):
        f_b, r_b, v_b, J_b, up_b = brute_step(cfg, o.pops().copy(), solid, o.beads()["r"], o.beads()["v"], orc, step)
        o.couple_step(1)
        b = o.beads()
        fo = o.pops()
        fl = solid == 0          # entries at solid nodes are never read
        assert np.abs(fo - f_b)[:, fl].max() < 1e-14, np.abs(fo - f_b)[:, fl].max()
        assert np.abs(b["up"] - up_b).max() < 1e-15
        assert np.abs(b["J"] - J_b).max() < 1e-12 * np.abs(J_b).max()
        assert np.abs(b["v"] - v_b).max() < 1e-12 * np.abs(v_b).max()
        assert np.abs(b["r"] - r_b).max() < 1e-13
        assert np.abs(v_b).max() < 2.0
    # the step did something on every channel
    assert np.abs(J_b).max() > 1e-4
