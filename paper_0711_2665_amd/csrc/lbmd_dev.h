// lbmd_dev.h -- device-side definitions shared by the kernels of liblbmd.
//
// D3Q19 tables, node flags, the argument blocks the host passes to the
// kernels, and the bead force laws.  Every floating-point expression that
// the FP64 path evaluates is written in a fixed evaluation order (the
// library is compiled without multiply-add contraction), so that a run is
// reproducible bit for bit.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lbmd {

constexpr int Q = 19;

// D3Q19 velocities: rest; +-x; +-y; +-z; xy, xz, yz diagonals, opposite
// pairs adjacent (Sec. 2 uses the standard 19-speed cubic lattice).
__host__ __device__ constexpr int cx(int i) {
  constexpr int t[Q] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
  return t[i];
}
__host__ __device__ constexpr int cy(int i) {
  constexpr int t[Q] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
  return t[i];
}
__host__ __device__ constexpr int cz(int i) {
  constexpr int t[Q] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};
  return t[i];
}
__host__ __device__ constexpr int opp(int i) { return i == 0 ? 0 : ((i & 1) ? i + 1 : i - 1); }
// weights 1/3, 1/18, 1/36 (rest, axis, diagonal)
__host__ __device__ constexpr double wgt(int i) { return i == 0 ? 1.0 / 3.0 : (i < 7 ? 1.0 / 18.0 : 1.0 / 36.0); }

// Modes of the fluctuating fluid: coefficient e_ki of population i in the
// non-conserved mode k = 4..18 (modes 0..3 are the density and the momentum,
// which take no noise).  Polynomials in the velocity c of population i,
// mutually orthogonal under the weights and orthogonal to 1 and c:
// k = 4 bulk stress c^2 - 1; 5, 6 normal-stress differences 3 c_x^2 - c^2,
// c_y^2 - c_z^2; 7..9 shear stresses c_x c_y, c_y c_z, c_z c_x; 10..12 the
// ghost vector (3 c^2 - 5) c; 13..15 the ghost vector (c_y^2 - c_z^2) c_x,
// (c_z^2 - c_x^2) c_y, (c_x^2 - c_y^2) c_z; 16 the ghost scalar
// 3 c^4 - 6 c^2 + 1; 17, 18 (2 c^2 - 3) times the modes 5 and 6.
__host__ __device__ constexpr int mode_coef(int k, int i) {
  const int x = cx(i), y = cy(i), z = cz(i);
  const int xx = x * x, yy = y * y, zz = z * z, q = xx + yy + zz;
  const int ax[3] = {x, y, z};
  if (k == 4) return q - 1;
  if (k == 5) return 3 * xx - q;
  if (k == 6) return yy - zz;
  if (k >= 7 && k <= 9) return ax[k - 7] * ax[(k - 6) % 3];
  if (k >= 10 && k <= 12) return (3 * q - 5) * ax[k - 10];
  if (k == 13) return (yy - zz) * x;
  if (k == 14) return (zz - xx) * y;
  if (k == 15) return (xx - yy) * z;
  if (k == 16) return 3 * q * q - 6 * q + 1;
  if (k == 17) return (2 * q - 3) * (3 * xx - q);
  return (2 * q - 3) * (yy - zz);
}
constexpr int NMODE_NOISE = 15;   // modes 4..18
// Parity of mode k under c -> -c: the ghost vectors 10..15 are odd, every
// other non-conserved mode is even.
__host__ __device__ constexpr bool mode_odd(int k) { return k >= 10 && k <= 15; }
__host__ __device__ constexpr bool mode_parity_holds() {
  for (int k = 4; k < Q; ++k)
    for (int i = 0; i < Q; ++i) {
      const int j = i == 0 ? 0 : ((i & 1) ? i + 1 : i - 1);   // the opposite velocity
      if (mode_coef(k, j) != (mode_odd(k) ? -1 : 1) * mode_coef(k, i)) return false;
    }
  return true;
}
static_assert(mode_parity_holds(), "mode parity table");

// node flags
constexpr uint8_t F_SOLID = 1;   // wall node: never updated; reflects links
constexpr uint8_t F_NEAR = 2;    // some upstream neighbour x - c_i is solid
constexpr uint8_t F_FORCED = 4;  // the bead force array holds this node's force

// watchdog bits
constexpr uint32_t E_DENSITY = 1u;   // density <= 0 or NaN in the LB update
constexpr uint32_t E_BEADS = 2u;     // non-finite bead state
constexpr uint32_t E_NBRLIST = 4u;   // neighbour list overflow
constexpr uint32_t E_SPREAD = 8u;    // too many beads share a node stencil

constexpr int MAXNBR = 48;        // neighbour-list capacity per bead
constexpr int MAXCONTRIB = 64;    // bead contributions gathered per node
// Neighbour-list skin.  The lists are built at every coupled step and stay
// valid while no bead moved more than SKIN_STEP / 2 from where they were
// built; 1.2 covers a step's motion of a driven chain (narrower skins
// forced a rebuild inside the sub-cycle in about one step of four at 0.8,
// every step at 0.6).  A sphere of r_c + 1.2 = 2.32 around a bead holds
// about 44 others at the density of a dense LJ liquid (0.85 per sigma^3),
// below MAXNBR; denser packing trips the list-overflow watchdog.
constexpr double SKIN_STEP = 1.2;
// Cells of the neighbour-search table are at least r_c + skin + CELL_MARGIN
// wide, so the table stays usable for a rebuild inside a sub-cycle while no
// bead has moved more than CELL_MARGIN from where it was binned.  It exceeds
// half the skin, so the first rebuild a cycle needs can use the table.
constexpr double CELL_MARGIN = 0.7;

// Control block at the head of the work buffer.
struct Ctrl {
  uint32_t err;
  uint32_t touched;          // nodes with the forced bit set this step
  uint64_t step;             // LB steps taken (Philox counter word 0)
  uint64_t rebuilds;         // neighbour-list rebuilds so far (diagnostic)
  uint64_t substeps;         // MD sub-steps so far (diagnostic)
  uint64_t forced_total;     // nodes carrying bead force, summed over steps (diagnostic)
  uint64_t cell_rebuilds;    // of the rebuilds, those that used the cell table (diagnostic)
  uint64_t fused_blocks;     // fused sub-step blocks completed (diagnostic)
  uint64_t fused_redos;      // replica sub-cycles redone from a failed block (diagnostic)
  // why fused blocks failed (diagnostic, per failing workgroup): lists not
  // valid or a bead too far from where they were built, too many close
  // partners, the set over its capacity, the closure not settled, a bead past
  // the displacement bound
  uint32_t fused_why[5];
  uint32_t nbr_max;          // longest neighbour list a per-step build found (diagnostic)
  uint32_t pad[42];
};
static_assert(sizeof(Ctrl) == 256, "control block is one 256-byte line");

// Geometry and lattice extents.
struct Geom {
  int nx, ny, nz;
  int nxy;
  long N;
  int wall_axis, wall_pos;
  int t0, t1;           // transverse axes
  int lo0, hi0, lo1, hi1;  // pore block
  int ngp;              // bead <-> lattice transfer at the nearest node (else trilinear)
};

__host__ __device__ inline int ext(const Geom& g, int a) { return a == 0 ? g.nx : (a == 1 ? g.ny : g.nz); }

// Is lattice site (sx, sy, sz) (any integers) solid?  One plane normal to
// wall_axis at wall_pos, minus the pore block (Sec. 4 geometry).
__host__ __device__ inline bool site_solid(const Geom& g, int sx, int sy, int sz) {
  if (g.wall_axis < 0) return false;
  int s[3] = {sx, sy, sz};
  int a = g.wall_axis;
  int n = ext(g, a);
  int sa = s[a] % n;
  if (sa < 0) sa += n;
  if (sa != g.wall_pos) return false;
  int n0 = ext(g, g.t0), n1 = ext(g, g.t1);
  int u = s[g.t0] % n0; if (u < 0) u += n0;
  int v = s[g.t1] % n1; if (v < 0) v += n1;
  bool pore = u >= g.lo0 && u <= g.hi0 && v >= g.lo1 && v <= g.hi1;
  return !pore;
}

// Wrap an unwrapped coordinate into [0, n): w = x - n floor(x / n), reduced
// once more if rounding lands on n.  For 0 <= x < n - 1 the quotient is
// certainly in [0, 1) so the result is x itself; that case skips the
// division and returns the same bits.
__device__ inline double wrapc(double x, int n) {
  double dn = (double)n;
  if (x >= 0.0 && x < dn - 1.0) return x;
  double q = floor(x / dn);
  double w = x - dn * q;
  if (w >= dn) w = w - dn;
  return w;
}

// Bead-side parameters.
struct MdParams {
  int nb;
  int n_sub;
  double hh;            // h / 2
  double m;
  double k_bond, r0, kappa, eps24, sig2, rc2;
  double gamma;         // friction rate used in the kick
  double e, omE, cf, sig;   // exp(-g h), 1 - e, (1-e)/(m g), noise sd
  double f_drive;
  int couple;           // 1: use u_p; 0: fluid decoupled (relaxation)
  int field_on;
  uint32_t seed, replica;
  double rlist2;        // (rc + skin)^2
  double halfskin2;     // (skin/2)^2
  double kick;          // multiple-time-step cycle: (dt/2)/m with dt = 1/M (0 without it)
  int wlo, whi;         // wall-site window offsets: 1 - ceil(rc) .. ceil(rc)
  int constrained;      // rigid bonds (SHAKE / RATTLE) instead of harmonic ones
};

// ---- Philox4x32-10 (Salmon et al., SC'11) and Box-Muller ------------------
__device__ inline void philox10(uint32_t& c0, uint32_t& c1, uint32_t& c2, uint32_t& c3, uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    // full 64-bit products: one v_mad_u64_u32 gives both halves
    const uint64_t p0 = (uint64_t)0xD2511F53u * c0, p1 = (uint64_t)0xCD9E8D57u * c2;
    // three-input XOR in one v_bitop3_b32 (truth table 0x96)
    const uint32_t n0 = __builtin_amdgcn_bitop3_b32((uint32_t)(p1 >> 32), c1, k0, 0x96);
    const uint32_t n2 = __builtin_amdgcn_bitop3_b32((uint32_t)(p0 >> 32), c3, k1, 0x96);
    c0 = n0; c1 = (uint32_t)p1; c2 = n2; c3 = (uint32_t)p0;
    k0 += 0x9E3779B9u; k1 += 0xBB67AE85u;
  }
}

// Three standard normals for (step n, sub-step s, bead p).
__device__ inline void gauss3(uint32_t seed, uint32_t rep, uint32_t n, uint32_t s, uint32_t p, double xi[3]) {
  uint32_t c0 = n, c1 = s, c2 = p, c3 = 0u;
  philox10(c0, c1, c2, c3, seed, rep);
  const double inv32 = 1.0 / 4294967296.0;
  double u0 = ((double)c0 + 0.5) * inv32;
  double u1 = ((double)c1 + 0.5) * inv32;
  double u2 = ((double)c2 + 0.5) * inv32;
  double u3 = ((double)c3 + 0.5) * inv32;
  const double two_pi = 6.283185307179586;
  double ra = sqrt(-2.0 * log(u0));
  double rb = sqrt(-2.0 * log(u2));
  xi[0] = ra * cos(two_pi * u1);
  xi[1] = ra * sin(two_pi * u1);
  xi[2] = rb * cos(two_pi * u3);
}

// ---- force laws (Sec. 2) ----------------------------------------------------
// Harmonic bond k/2 (|d| - r0)^2, d = r_p - r_q: adds the force on p.
__device__ inline void bond_add(const MdParams& P, const double* rp, const double* rq, double F[3]) {
  double d0 = rp[0] - rq[0], d1 = rp[1] - rq[1], d2 = rp[2] - rq[2];
  double dist = sqrt(d0 * d0 + d1 * d1 + d2 * d2);
  double coef = -(P.k_bond * (dist - P.r0)) / dist;
  F[0] += coef * d0; F[1] += coef * d1; F[2] += coef * d2;
}

// Bending kappa phi^2/2 at interior bead q (positions a = r_{q-1}, b = r_q,
// c = r_{q+1}); phi = atan2(|b1 x b2|, b1.b2).  which = 0: force on q-1,
// 1: on q, 2: on q+1; added to F.
__device__ inline void angle_add(const MdParams& P, const double* ra, const double* rb, const double* rc, int which,
                                 double F[3]) {
  double b1[3] = {rb[0] - ra[0], rb[1] - ra[1], rb[2] - ra[2]};
  double b2[3] = {rc[0] - rb[0], rc[1] - rb[1], rc[2] - rb[2]};
  double n[3] = {b1[1] * b2[2] - b1[2] * b2[1], b1[2] * b2[0] - b1[0] * b2[2], b1[0] * b2[1] - b1[1] * b2[0]};
  double s = sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
  double c = b1[0] * b2[0] + b1[1] * b2[1] + b1[2] * b2[2];
  if (s == 0.0) {
    // straight or folded: no unique gradient; the contribution is exactly 0
    F[0] += 0.0; F[1] += 0.0; F[2] += 0.0;
    return;
  }
  double phi = atan2(s, c);
  double den = s * s + c * c;
  double g1[3] = {b2[1] * n[2] - b2[2] * n[1], b2[2] * n[0] - b2[0] * n[2], b2[0] * n[1] - b2[1] * n[0]};
  double g2[3] = {n[1] * b1[2] - n[2] * b1[1], n[2] * b1[0] - n[0] * b1[2], n[0] * b1[1] - n[1] * b1[0]};
  double kp = P.kappa * phi;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    double d1 = (c * g1[a] / s - s * b2[a]) / den;
    double d2 = (c * g2[a] / s - s * b1[a]) / den;
    double f;
    if (which == 0) f = kp * d1;
    else if (which == 1) f = -(kp * (d1 - d2));
    else f = -(kp * d2);
    F[a] += f;
  }
}

// Truncated LJ (WCA): adds the pair force on the first bead for separation d.
__device__ inline void lj_add(const MdParams& P, double d0, double d1, double d2, double F[3]) {
  double r2 = d0 * d0 + d1 * d1 + d2 * d2;
  if (!(r2 < P.rc2)) return;
  double sr2 = P.sig2 / r2;
  double sr6 = sr2 * sr2 * sr2;
  double sr12 = sr6 * sr6;
  double coef = P.eps24 * (2.0 * sr12 - sr6) / r2;
  F[0] += coef * d0; F[1] += coef * d1; F[2] += coef * d2;
}

// Minimum image d - n floor(d / n + 1/2).  For |d| < n/4 the floor is 0 and
// the result is d itself; that case skips the division, same bits.
__device__ inline double min_image(double d, int n) {
  double dn = (double)n;
  if (fabs(d) < 0.25 * dn) return d;
  double k = floor(d / dn + 0.5);
  return d - dn * k;
}

// Pore channel: [wall - 1.5, wall + 1.5) along the normal times
// [lo - 0.5, hi + 0.5) on both transverse axes (wrapped coordinates).
__device__ inline bool in_field(const Geom& g, const double* rp) {
  if (g.wall_axis < 0) return false;
  int a = g.wall_axis;
  double wn = wrapc(rp[a], ext(g, a));
  if (!(wn >= g.wall_pos - 1.5 && wn < g.wall_pos + 1.5)) return false;
  double w0 = wrapc(rp[g.t0], ext(g, g.t0));
  if (!(w0 >= g.lo0 - 0.5 && w0 < g.hi0 + 0.5)) return false;
  double w1 = wrapc(rp[g.t1], ext(g, g.t1));
  if (!(w1 >= g.lo1 - 0.5 && w1 < g.hi1 + 0.5)) return false;
  return true;
}

// Trilinear stencil of a bead: base node index, fractions.
struct Stencil {
  int b[3];
  double d[3];
};
__device__ inline Stencil make_stencil(const Geom& g, const double* rp) {
  Stencil s;
  double w0 = wrapc(rp[0], g.nx), w1 = wrapc(rp[1], g.ny), w2 = wrapc(rp[2], g.nz);
  // a non-finite position (a blown-up run, reported by the watchdog) must
  // still index inside the lattice
  if (!(w0 >= 0.0 && w0 < (double)g.nx)) w0 = 0.0;
  if (!(w1 >= 0.0 && w1 < (double)g.ny)) w1 = 0.0;
  if (!(w2 >= 0.0 && w2 < (double)g.nz)) w2 = 0.0;
  s.b[0] = (int)floor(w0); s.b[1] = (int)floor(w1); s.b[2] = (int)floor(w2);
  s.d[0] = w0 - (double)s.b[0]; s.d[1] = w1 - (double)s.b[1]; s.d[2] = w2 - (double)s.b[2];
  if (g.ngp) {
    // nearest grid point: weight 1 at the nearest corner (the upper one
    // along an axis whose fraction is at least 1/2), 0 at the others
#pragma unroll
    for (int a = 0; a < 3; ++a) s.d[a] = s.d[a] >= 0.5 ? 1.0 : 0.0;
  }
  return s;
}
// corner k = (k&1, k>>1&1, k>>2&1): node index and weight
__device__ inline long corner_node(const Geom& g, const Stencil& s, int k) {
  int x = s.b[0] + (k & 1); if (x >= g.nx) x -= g.nx;
  int y = s.b[1] + ((k >> 1) & 1); if (y >= g.ny) y -= g.ny;
  int z = s.b[2] + ((k >> 2) & 1); if (z >= g.nz) z -= g.nz;
  return (long)x + (long)g.nx * ((long)y + (long)g.ny * (long)z);
}
__device__ inline double corner_weight(const Stencil& s, int k) {
  double wx = (k & 1) ? s.d[0] : 1.0 - s.d[0];
  double wy = ((k >> 1) & 1) ? s.d[1] : 1.0 - s.d[1];
  double wz = ((k >> 2) & 1) ? s.d[2] : 1.0 - s.d[2];
  return wx * wy * wz;
}
// Whether corner k takes part in the transfer: every corner of the
// trilinear stencil; only the nearest node with the nearest-grid-point one
// (the others carry no force, so they are neither marked nor updated by the
// spreading).
__device__ inline bool corner_used(const Geom& g, const Stencil& s, int k) {
  if (!g.ngp) return true;
  return (k & 1) == (int)s.d[0] && ((k >> 1) & 1) == (int)s.d[1] && ((k >> 2) & 1) == (int)s.d[2];
}

}  // namespace lbmd
