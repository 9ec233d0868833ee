// adj_kernels.hip -- reverse (adjoint) pass of the coupled step.
//
// The coupled step maps (A, r, v) -> (B, r', v') through four stages (gather,
// MD sub-cycle, spreading, LB sweep; Sec. 2).  Its transpose, applied to the
// adjoint (lam_B, lam_r', lam_v') of the step's output, gives the adjoint of
// its input and the contributions to dL/dgamma and dL/dF_drive:
//   LB^T      lam_f(x) = (dcoll/df)^T lam_B(x) [+ (du/df)^T lam_u(x) where a
//             bead stencil touches x], then lam_A = pull^T lam_f (each element
//             of A is pulled by exactly one (node, direction), so the
//             transpose is a scatter with one writer per element);
//   spread^T  lam_J_p = sum_k W_k lam_Fn(x_k), lam_Fn(x) = sum_i 3 w_i c_i
//             lam_B_i(x); d/dr of W_k gives a position term;
//   MD^T      the sub-steps in reverse; the force Jacobian enters as
//             (dF/dr)^T lam_F, which for conservative forces equals the
//             directional derivative of F along lam_F (evaluated with dual
//             numbers);
//   gather^T  lam_u(x_k) += W_k lam_up_p (summed per node like the forward
//             spreading), and d/dr of W_k gives a position term.
// The fields the reverse step needs (populations, r, v, u_p, J of the step)
// come from a tape written while the segment is recomputed from a checkpoint.
#include <type_traits>

#include "lbmd_kernels.h"
#include "lbmd_lattice.h"

namespace lbmd {

// ---------------------------------------------------------------------------
// Dual numbers: value and derivative along one direction.
// ---------------------------------------------------------------------------
struct Dd {
  double v, d;
};
__device__ inline Dd mkd(double v, double d = 0.0) { return Dd{v, d}; }
__device__ inline Dd operator+(Dd a, Dd b) { return Dd{a.v + b.v, a.d + b.d}; }
__device__ inline Dd operator-(Dd a, Dd b) { return Dd{a.v - b.v, a.d - b.d}; }
__device__ inline Dd operator-(Dd a) { return Dd{-a.v, -a.d}; }
__device__ inline Dd operator*(Dd a, Dd b) { return Dd{a.v * b.v, a.d * b.v + a.v * b.d}; }
__device__ inline Dd operator*(double s, Dd a) { return Dd{s * a.v, s * a.d}; }
__device__ inline Dd operator/(Dd a, Dd b) {
  double q = a.v / b.v;
  return Dd{q, (a.d - q * b.d) / b.v};
}
__device__ inline Dd dsqrt(Dd x) {
  double s = sqrt(x.v);
  return Dd{s, s > 0.0 ? x.d / (2.0 * s) : 0.0};
}
__device__ inline Dd datan2(Dd y, Dd x) {
  double den = x.v * x.v + y.v * y.v;
  return Dd{atan2(y.v, x.v), (x.v * y.d - y.v * x.d) / den};
}

// ---- force laws in dual arithmetic (the same expressions as the forward
// force laws; positions carry the direction in their derivative part) -----
__device__ inline void bond_dd(const MdParams& P, const Dd* rp, const Dd* rq, Dd F[3]) {
  Dd d0 = rp[0] - rq[0], d1 = rp[1] - rq[1], d2 = rp[2] - rq[2];
  Dd dist = dsqrt(d0 * d0 + d1 * d1 + d2 * d2);
  Dd coef = -(P.k_bond * (dist - mkd(P.r0))) / dist;
  F[0] = F[0] + coef * d0; F[1] = F[1] + coef * d1; F[2] = F[2] + coef * d2;
}

__device__ inline void angle_dd(const MdParams& P, const Dd* ra, const Dd* rb, const Dd* rc, int which, Dd F[3]) {
  Dd b1[3] = {rb[0] - ra[0], rb[1] - ra[1], rb[2] - ra[2]};
  Dd b2[3] = {rc[0] - rb[0], rc[1] - rb[1], rc[2] - rb[2]};
  Dd n[3] = {b1[1] * b2[2] - b1[2] * b2[1], b1[2] * b2[0] - b1[0] * b2[2], b1[0] * b2[1] - b1[1] * b2[0]};
  Dd s = dsqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
  Dd c = b1[0] * b2[0] + b1[1] * b2[1] + b1[2] * b2[2];
  if (s.v == 0.0) return;
  Dd phi = datan2(s, c);
  Dd den = s * s + c * c;
  Dd g1[3] = {b2[1] * n[2] - b2[2] * n[1], b2[2] * n[0] - b2[0] * n[2], b2[0] * n[1] - b2[1] * n[0]};
  Dd g2[3] = {n[1] * b1[2] - n[2] * b1[1], n[2] * b1[0] - n[0] * b1[2], n[0] * b1[1] - n[1] * b1[0]};
  Dd kp = P.kappa * phi;
  for (int a = 0; a < 3; ++a) {
    Dd d1 = (c * g1[a] / s - s * b2[a]) / den;
    Dd d2 = (c * g2[a] / s - s * b1[a]) / den;
    Dd f;
    if (which == 0) f = kp * d1;
    else if (which == 1) f = -(kp * (d1 - d2));
    else f = -(kp * d2);
    F[a] = F[a] + f;
  }
}

__device__ inline void lj_dd(const MdParams& P, Dd d0, Dd d1, Dd d2, Dd F[3]) {
  Dd r2 = d0 * d0 + d1 * d1 + d2 * d2;
  if (!(r2.v < P.rc2)) return;
  Dd sr2 = mkd(P.sig2) / r2;
  Dd sr6 = sr2 * sr2 * sr2;
  Dd sr12 = sr6 * sr6;
  Dd coef = P.eps24 * (2.0 * sr12 - sr6) / r2;
  F[0] = F[0] + coef * d0; F[1] = F[1] + coef * d1; F[2] = F[2] + coef * d2;
}

// Wall sites within r_c of the bead (r_c <= 3): the sites of the wall plane
// at offsets P.wlo..P.whi (1 - ceil(r_c)..ceil(r_c), within -2..3) around the
// base node, minus the pore block -- the rows outside hold no site within
// r_c, so the hit sites and their order are those of the full 6 x 6 window;
// the derivative of the wrapped position is that of r.
__device__ inline void wall_dd(const MdParams& P, const Geom& g, const Dd* rp, Dd F[3]) {
  if (g.wall_axis < 0) return;
  const double w[3] = {wrapc(rp[0].v, g.nx), wrapc(rp[1].v, g.ny), wrapc(rp[2].v, g.nz)};
  const int b[3] = {(int)floor(w[0]), (int)floor(w[1]), (int)floor(w[2])};
  const int n[3] = {g.nx, g.ny, g.nz};
  const int a = g.wall_axis, t0 = g.t0, t1 = g.t1;
  int off = g.wall_pos - b[a];               // offset along the normal reaching the plane
  if (off < -2) off += n[a];
  if (off > 3) off -= n[a];
  if (off < P.wlo || off > P.whi) return;
  int site[3];
  site[a] = b[a] + off;
  for (int o1 = P.wlo; o1 <= P.whi; ++o1) {
    const int u1 = b[t1] + o1;
    const int v1 = u1 < 0 ? u1 + n[t1] : (u1 >= n[t1] ? u1 - n[t1] : u1);
    const bool in1 = v1 >= g.lo1 && v1 <= g.hi1;
    for (int o0 = P.wlo; o0 <= P.whi; ++o0) {
      const int u0 = b[t0] + o0;
      const int v0 = u0 < 0 ? u0 + n[t0] : (u0 >= n[t0] ? u0 - n[t0] : u0);
      const bool in0 = v0 >= g.lo0 && v0 <= g.hi0;
      if (in0 && in1) continue;              // pore node: fluid
      site[t0] = u0;
      site[t1] = u1;
      const double e0 = w[0] - (double)site[0], e1 = w[1] - (double)site[1], e2 = w[2] - (double)site[2];
      if (!(e0 * e0 + e1 * e1 + e2 * e2 < P.rc2)) continue;
      lj_dd(P, Dd{e0, rp[0].d}, Dd{e1, rp[1].d}, Dd{e2, rp[2].d}, F);
    }
  }
}

// Bending forces of the angle centred at q (1 <= q <= nb - 2) at positions
// pos with direction dir, value and derivative, into LDS rows av[q], ad[q]:
// [0..2] force on q-1, [3..5] on q, [6..8] on q+1.
// The three vertex forces are independent: the caller gives vertex w to
// lane w of the bead.
__device__ inline void angle_to_lds(const MdParams& P, const double (*pos)[3], const double (*dir)[3], int q,
                                    int w, double (*av)[9], double (*ad)[9]) {
  Dd ra[3], rb[3], rc[3];
  for (int a = 0; a < 3; ++a) {
    ra[a] = Dd{pos[q - 1][a], dir[q - 1][a]};
    rb[a] = Dd{pos[q][a], dir[q][a]};
    rc[a] = Dd{pos[q + 1][a], dir[q + 1][a]};
  }
  Dd F[3] = {mkd(0.0), mkd(0.0), mkd(0.0)};
  angle_dd(P, ra, rb, rc, w, F);
  for (int a = 0; a < 3; ++a) { av[q][3 * w + a] = F[a].v; ad[q][3 * w + a] = F[a].d; }
}

// Conservative force on chain bead p at positions pos with direction dir
// (nb x 3, LDS), value and directional derivative, computed by the 4 lanes
// of the bead: lane l scans the pair partners j = l, l + 4, ... within r_c
// (distance screen in plain doubles, dual arithmetic only inside r_c); lane
// 0 adds the bonds, the angle forces from LDS (angles centred at p-1, p,
// p+1) and the wall sites.  The four partial sums are combined in a fixed
// order with cross-lane reads, so every lane of the bead ends with F, dF.
// The field is added by the caller (constant in r).
constexpr int ADJ_MAXHIT = 16;   // partners within r_c kept per lane (j = lane mod 4)

__device__ inline void bead_force_dd(const MdParams& P, const Geom& g, const double (*pos)[3],
                                     const double (*dir)[3], const double (*av)[9], const double (*ad)[9], int p,
                                     int lane, bool on, double F[3], double dF[3]) {
  const int nb = P.nb;
  Dd S[3] = {mkd(0.0), mkd(0.0), mkd(0.0)};
  if (on) {
    // the partners within r_c first, in ascending j, then their dual LJ
    // terms in that order: the lanes of a wave then evaluate the LJ terms
    // together instead of one scan iteration at a time (more than
    // ADJ_MAXHIT partners: the same sum in one pass)
    int hit[ADJ_MAXHIT];
    int nh = 0;
    for (int j = lane; j < nb; j += 4) {
      if (j == p) continue;
      const double e0 = min_image(pos[p][0] - pos[j][0], g.nx);
      const double e1 = min_image(pos[p][1] - pos[j][1], g.ny);
      const double e2 = min_image(pos[p][2] - pos[j][2], g.nz);
      if (!(e0 * e0 + e1 * e1 + e2 * e2 < P.rc2)) continue;
      if (nh < ADJ_MAXHIT) hit[nh] = j;
      ++nh;
    }
    if (nh <= ADJ_MAXHIT) {
      for (int k = 0; k < nh; ++k) {
        const int j = hit[k];
        const double e0 = min_image(pos[p][0] - pos[j][0], g.nx);
        const double e1 = min_image(pos[p][1] - pos[j][1], g.ny);
        const double e2 = min_image(pos[p][2] - pos[j][2], g.nz);
        lj_dd(P, Dd{e0, dir[p][0] - dir[j][0]}, Dd{e1, dir[p][1] - dir[j][1]}, Dd{e2, dir[p][2] - dir[j][2]}, S);
      }
    } else {
      for (int j = lane; j < nb; j += 4) {
        if (j == p) continue;
        const double e0 = min_image(pos[p][0] - pos[j][0], g.nx);
        const double e1 = min_image(pos[p][1] - pos[j][1], g.ny);
        const double e2 = min_image(pos[p][2] - pos[j][2], g.nz);
        if (!(e0 * e0 + e1 * e1 + e2 * e2 < P.rc2)) continue;
        lj_dd(P, Dd{e0, dir[p][0] - dir[j][0]}, Dd{e1, dir[p][1] - dir[j][1]}, Dd{e2, dir[p][2] - dir[j][2]}, S);
      }
    }
    if (lane == 0) {
      Dd rp[3] = {Dd{pos[p][0], dir[p][0]}, Dd{pos[p][1], dir[p][1]}, Dd{pos[p][2], dir[p][2]}};
      if (p > 0) {
        Dd rq[3] = {Dd{pos[p - 1][0], dir[p - 1][0]}, Dd{pos[p - 1][1], dir[p - 1][1]},
                    Dd{pos[p - 1][2], dir[p - 1][2]}};
        bond_dd(P, rp, rq, S);
      }
      if (p < nb - 1) {
        Dd rq[3] = {Dd{pos[p + 1][0], dir[p + 1][0]}, Dd{pos[p + 1][1], dir[p + 1][1]},
                    Dd{pos[p + 1][2], dir[p + 1][2]}};
        bond_dd(P, rp, rq, S);
      }
      if (p - 1 >= 1 && p - 1 <= nb - 2)
        for (int a = 0; a < 3; ++a) S[a] = S[a] + Dd{av[p - 1][6 + a], ad[p - 1][6 + a]};
      if (p >= 1 && p <= nb - 2)
        for (int a = 0; a < 3; ++a) S[a] = S[a] + Dd{av[p][3 + a], ad[p][3 + a]};
      if (p + 1 >= 1 && p + 1 <= nb - 2)
        for (int a = 0; a < 3; ++a) S[a] = S[a] + Dd{av[p + 1][a], ad[p + 1][a]};
      wall_dd(P, g, rp, S);
    }
  }
  // (lane0 + lane1) + (lane2 + lane3), the same on every lane of the bead
  const int base = (int)(threadIdx.x & 63u) & ~3;
  for (int a = 0; a < 3; ++a) {
    double v[4], d[4];
    for (int l = 0; l < 4; ++l) {
      v[l] = __shfl(S[a].v, base + l, 64);
      d[l] = __shfl(S[a].d, base + l, 64);
    }
    F[a] = (v[0] + v[1]) + (v[2] + v[3]);
    dF[a] = (d[0] + d[1]) + (d[2] + d[3]);
  }
}

// ---------------------------------------------------------------------------
// Initial adjoint: lam_r = dL/dr(final), lam_v = dL/dv(final) or 0, lam_A = 0,
// parameter accumulators 0.
// ---------------------------------------------------------------------------
__global__ void k_adj_init(const double* __restrict__ dLdr, const double* __restrict__ dLdv, AdjBufs a, int n3) {
  int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n3) {
    a.lr[k] = dLdr[k];
    a.lv[k] = dLdv ? dLdv[k] : 0.0;
  }
  if (k < 4) a.par[k] = 0.0;
}

// d W_k / d r_a of the trilinear weight of corner k.
__device__ inline double dweight(const Stencil& s, int k, int a) {
  double w[3], dw[3];
  for (int b = 0; b < 3; ++b) {
    bool hi = (k >> b) & 1;
    w[b] = hi ? s.d[b] : 1.0 - s.d[b];
    dw[b] = hi ? 1.0 : -1.0;
  }
  return a == 0 ? dw[0] * w[1] * w[2] : (a == 1 ? w[0] * dw[1] * w[2] : w[0] * w[1] * dw[2]);
}

// ---------------------------------------------------------------------------
// Spreading transpose, one thread per bead: lam_J and the position term of
// the spreading (J_p of the step from the tape).
// ---------------------------------------------------------------------------
template <typename T>
__global__ void k_adj_spread_t(const T* __restrict__ lamB, Dev d, AdjBufs a, const double* __restrict__ Jt, int nb) {
  int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= nb) return;
  const Rep& R = d.reps[0];
  const size_t N = (size_t)R.lp.N;
  double rp[3] = {d.rs[3 * p], d.rs[3 * p + 1], d.rs[3 * p + 2]};
  Stencil st = make_stencil(R.g, rp);
  double lJ[3] = {0.0, 0.0, 0.0}, lr[3] = {0.0, 0.0, 0.0};
  const double J[3] = {Jt[3 * p], Jt[3 * p + 1], Jt[3 * p + 2]};
  for (int k = 0; k < 8; ++k) {
    int n = (int)corner_node(R.g, st, k);
    if (d.flags[n] & F_SOLID) continue;
    double lf[Q];
    for (int i = 0; i < Q; ++i) lf[i] = (double)lamB[(size_t)i * N + n];
    double lF[3];
    lF[0] = 3.0 * (wgt(1) * (lf[1] - lf[2]) + wgt(7) * (lf[7] - lf[8] + lf[9] - lf[10] + lf[11] - lf[12] + lf[13] - lf[14]));
    lF[1] = 3.0 * (wgt(3) * (lf[3] - lf[4]) + wgt(7) * (lf[7] - lf[8] - lf[9] + lf[10] + lf[15] - lf[16] + lf[17] - lf[18]));
    lF[2] = 3.0 * (wgt(5) * (lf[5] - lf[6]) + wgt(11) * (lf[11] - lf[12] - lf[13] + lf[14] + lf[15] - lf[16] - lf[17] + lf[18]));
    double W = corner_weight(st, k);
    double JdotL = J[0] * lF[0] + J[1] * lF[1] + J[2] * lF[2];
    for (int b = 0; b < 3; ++b) {
      lJ[b] += W * lF[b];
      lr[b] += dweight(st, k, b) * JdotL;
    }
  }
  for (int b = 0; b < 3; ++b) {
    a.lJ[3 * p + b] = lJ[b];
    a.lrs[3 * p + b] = lr[b];
  }
}

// ---------------------------------------------------------------------------
// MD sub-cycle transpose of one chain, one workgroup, four lanes per bead.
// The force positions r_mid and the velocities at the start of every
// sub-step come from the tape the forward sub-cycle wrote while the segment
// was recomputed; the sub-steps are reversed.  On entry lr, lv hold
// the adjoint of r, v after the step and lJ that of the impulse J; on exit
// lr, lv hold the adjoint of r_n, v_n through the sub-cycle and lup that of
// u_p.  The parameter adjoints are added to par[0] (gamma) and par[1]
// (F_drive).
// ---------------------------------------------------------------------------
constexpr int ADJ_LANES = 4;
constexpr int ADJ_WG = ADJ_LANES * MAX_ADJ_BEADS;

// Forces on every bead at the positions in pos with direction dir: angles
// into LDS first (one thread per angle), then the per-bead sums.
__device__ inline void chain_forces(const MdParams& P, const Geom& g, const double (*pos)[3], const double (*dir)[3],
                                    double (*av)[9], double (*ad)[9], int p, int lane, bool on, double F[3],
                                    double dF[3]) {
  const int nb = P.nb;
  if (lane < 3 && p >= 1 && p <= nb - 2) angle_to_lds(P, pos, dir, p, lane, av, ad);
  __syncthreads();
  bead_force_dd(P, g, pos, dir, av, ad, p, lane, on, F, dF);
}

// The bead noise of every sub-step of the step being reversed, drawn in
// parallel before the serial reverse sub-cycle (the forward's draws: key
// (seed, replica), counter (step, s, p, 0)); one thread per (s, p).
__global__ void k_adj_noise(Dev d, double* __restrict__ xi, uint32_t step, int nb, int n_sub) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nb * n_sub) return;
  const MdParams& P = d.reps[0].mp;
  const int s = t / nb, p = t - s * nb;
  double x[3];
  gauss3(P.seed, P.replica, step, (uint32_t)s, (uint32_t)p, x);
  for (int c = 0; c < 3; ++c) xi[(size_t)t * 3 + c] = x[c];
}

__global__ __launch_bounds__(ADJ_WG) void k_adj_md(Dev d, AdjBufs a, const double* __restrict__ mdt,
                                                   const double* __restrict__ upt, uint32_t step, double kT) {
  extern __shared__ double lds[];
  const Rep& R = d.reps[0];
  const MdParams P = R.mp;
  const Geom g = R.g;
  const int nb = P.nb, n_sub = P.n_sub;
  double(*pos)[3] = (double(*)[3])lds;
  double(*dir)[3] = (double(*)[3])(lds + 3 * nb);
  double(*av)[9] = (double(*)[9])(lds + 6 * nb);
  double(*ad)[9] = (double(*)[9])(lds + 15 * nb);
  double* red = lds + 24 * nb;            // 2 x (ADJ_WG / ADJ_LANES) reduction scratch
  const int p = threadIdx.x / ADJ_LANES, lane = threadIdx.x % ADJ_LANES;
  const bool on = p < nb;
  const bool lead = on && lane == 0;
  double u[3];
  for (int c = 0; c < 3; ++c) u[c] = on ? upt[3 * p + c] : 0.0;
  // the forward sub-cycle recorded r_mid and v at the start of every
  // sub-step: mdt[s][p][0..2] and [3..5]
  // ---- reverse
  const double h = 2.0 * P.hh;
  const double gam = P.gamma;
  const double de = -h * P.e, domE = h * P.e;
  const double dcf = (h * P.e) / (P.m * gam) - P.omE / (P.m * gam * gam);
  const double dsig = P.sig > 0.0 ? ((kT / P.m) * (h * P.e * P.e)) / P.sig : 0.0;
  double lr[3], lv[3], lJ[3], lu[3];
  for (int c = 0; c < 3; ++c) {
    lr[c] = on ? a.lr[3 * p + c] : 0.0;
    lv[c] = on ? a.lv[3 * p + c] : 0.0;
    lJ[c] = on ? a.lJ[3 * p + c] : 0.0;
    lu[c] = 0.0;
  }
  double acc_g = 0.0, acc_f = 0.0;
  for (int s = n_sub - 1; s >= 0; --s) {
    double lvt[3], rm[3];
    for (int c = 0; c < 3; ++c) {
      lvt[c] = lv[c] + P.hh * lr[c];
      rm[c] = on ? mdt[((size_t)s * nb + p) * 6 + c] : 0.0;
    }
    if (lead)
      for (int c = 0; c < 3; ++c) { pos[p][c] = rm[c]; dir[p][c] = P.cf * lvt[c]; }
    __syncthreads();
    double f[3], df[3];
    chain_forces(P, g, pos, dir, av, ad, p, lane, on, f, df);
    if (on) {
      const bool field = P.field_on && in_field(g, rm);
      if (field) f[g.wall_axis] += P.f_drive;
      double xi[3] = {0.0, 0.0, 0.0};
      if (P.sig != 0.0 && lead)
        for (int c = 0; c < 3; ++c) xi[c] = a.xi[((size_t)s * nb + p) * 3 + c];
      for (int c = 0; c < 3; ++c) {
        const double vo = mdt[((size_t)s * nb + p) * 6 + 3 + c];
        if (lead) {
          acc_g += lvt[c] * (vo * de + (f[c] + gam * u[c]) * dcf + P.cf * u[c] + xi[c] * dsig);
          acc_g += lJ[c] * (-P.m) * ((u[c] - vo) * domE + xi[c] * dsig);
        }
        lu[c] += P.cf * gam * lvt[c] - P.m * P.omE * lJ[c];
        const double lrm = lr[c] + df[c];
        lr[c] = lrm;
        lv[c] = P.e * lvt[c] + P.m * P.omE * lJ[c] + P.hh * lrm;
      }
      if (lead && field) acc_f += P.cf * lvt[g.wall_axis];
    }
    __syncthreads();
  }
  if (lead) {
    for (int c = 0; c < 3; ++c) {
      a.lr[3 * p + c] = lr[c];
      a.lv[3 * p + c] = lv[c];
      a.lup[3 * p + c] = lu[c];
    }
  }
  // parameter adjoints: fixed-order tree over the beads (lane-0 values)
  constexpr int NB_ = ADJ_WG / ADJ_LANES;
  if (lane == 0) {
    red[p] = acc_g;
    red[NB_ + p] = acc_f;
  }
  __syncthreads();
  for (int w = NB_ / 2; w > 0; w >>= 1) {
    if (lane == 0 && p < w) { red[p] += red[p + w]; red[NB_ + p] += red[NB_ + p + w]; }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    a.par[0] += red[0];
    a.par[1] += red[NB_];
  }
}

// ---------------------------------------------------------------------------
// Gather transpose, position term, one thread per bead; adds the spreading
// and gathering position terms to lam_r.
// ---------------------------------------------------------------------------
template <typename T, bool DEV>
__global__ void k_adj_gather_t(const T* __restrict__ A, Dev d, AdjBufs a, int nb) {
  int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= nb) return;
  const Rep& R = d.reps[0];
  double rp[3] = {d.rs[3 * p], d.rs[3 * p + 1], d.rs[3 * p + 2]};
  Stencil st = make_stencil(R.g, rp);
  const double lu[3] = {a.lup[3 * p], a.lup[3 * p + 1], a.lup[3 * p + 2]};
  double lr[3] = {0.0, 0.0, 0.0};
  for (int k = 0; k < 8; ++k) {
    int n = (int)corner_node(R.g, st, k);
    double u[3];
    node_velocity<T, DEV>(A, d.flags, R.lp, n, u);
    double ul = u[0] * lu[0] + u[1] * lu[1] + u[2] * lu[2];
    for (int b = 0; b < 3; ++b) lr[b] += dweight(st, k, b) * ul;
  }
  for (int b = 0; b < 3; ++b) a.lr[3 * p + b] += a.lrs[3 * p + b] + lr[b];
}

// ---------------------------------------------------------------------------
// LB transpose over the sweep's tile table: for each fluid node x the
// adjoint of its post-streaming populations, lam_f = (1 - omega) lam_B +
// omega (G0 + c.G) with G0 = sum_i w_i lam_i (1 - 4.5 (c_i.u)^2 + 1.5 u.u),
// G = sum_i w_i lam_i (3 c_i + 9 (c_i.u) c_i - 3 u) (the transpose of the
// BGK Jacobian with the second-order equilibrium), plus (c.lam_u - u.lam_u)
// / rho where a bead stencil gathered u(x); then scattered to the element of
// A it was pulled from.
// ---------------------------------------------------------------------------
template <typename T, bool DEV>
__global__ __launch_bounds__(256) void k_adj_lb(const T* __restrict__ A, const T* __restrict__ lamB,
                                                T* __restrict__ lamA, Dev d, const T* __restrict__ lamu, int ntiles,
                                                int tile_nodes) {
  using R_ = typename std::conditional<DEV, float, double>::type;
  for (int tI = blockIdx.x; tI < ntiles; tI += gridDim.x) {
    const Tile tl = d.tiles[tI];
    const Rep& Rp = d.reps[tl.rep];
    const LbParams& p = Rp.lp;
    const size_t N = (size_t)p.N;
    const size_t no = (size_t)Rp.node_off;
    const T* Ar = A + Q * no;
    const T* lBr = lamB + Q * no;
    T* lAr = lamA + Q * no;
    const T* lur = lamu + 3 * no;
    const uint8_t* fr = d.flags + no;
    const int end = min(tl.start + tile_nodes, p.N);
    for (int c = tl.start + (int)threadIdx.x; c < end; c += blockDim.x) {
      const uint8_t fl = fr[c];
      if (fl & F_SOLID) continue;
      int x = c % p.nx, yz = c / p.nx, y = yz % p.ny, z = yz / p.ny;
      Nbr nb = make_nbr(p, x, y, z);
      T fT[Q];
      pull<T>(Ar, fr, p, c, fl, nb, fT);
      R_ f[Q], lb[Q];
      for (int i = 0; i < Q; ++i) { f[i] = (R_)fT[i]; lb[i] = (R_)lBr[(size_t)i * N + c]; }
      R_ rho = 0, jx, jy, jz;
      for (int i = 0; i < Q; ++i) rho += f[i];
      jx = f[1] - f[2] + f[7] - f[8] + f[9] - f[10] + f[11] - f[12] + f[13] - f[14];
      jy = f[3] - f[4] + f[7] - f[8] - f[9] + f[10] + f[15] - f[16] + f[17] - f[18];
      jz = f[5] - f[6] + f[11] - f[12] - f[13] + f[14] + f[15] - f[16] - f[17] + f[18];
      if (DEV) rho = (R_)1 + rho;
      const R_ ux = jx / rho, uy = jy / rho, uz = jz / rho;
      const R_ usq = ux * ux + uy * uy + uz * uz;
      R_ G0 = 0, A0 = 0, G1x = 0, G1y = 0, G1z = 0, G2x = 0, G2y = 0, G2z = 0;
      for (int i = 0; i < Q; ++i) {
        const R_ wl = (R_)wgt(i) * lb[i];
        const R_ cu = cdot<R_>(i, ux, uy, uz);
        G0 += wl * ((R_)1 - (R_)4.5 * cu * cu + (R_)1.5 * usq);
        A0 += wl;
        G1x += wl * (R_)cx(i); G1y += wl * (R_)cy(i); G1z += wl * (R_)cz(i);
        G2x += wl * cu * (R_)cx(i); G2y += wl * cu * (R_)cy(i); G2z += wl * cu * (R_)cz(i);
      }
      const R_ Gx = (R_)3 * G1x + (R_)9 * G2x - (R_)3 * ux * A0;
      const R_ Gy = (R_)3 * G1y + (R_)9 * G2y - (R_)3 * uy * A0;
      const R_ Gz = (R_)3 * G1z + (R_)9 * G2z - (R_)3 * uz * A0;
      const R_ om = (R_)p.omega;
      R_ Lx = 0, Ly = 0, Lz = 0, Lu = 0, irho = 0;
      const bool forced = (fl & F_FORCED) != 0;
      if (forced) {
        Lx = (R_)lur[c]; Ly = (R_)lur[N + c]; Lz = (R_)lur[2 * N + c];
        Lu = ux * Lx + uy * Ly + uz * Lz;
        irho = (R_)1 / rho;
      }
      for (int i = 0; i < Q; ++i) {
        R_ lf = ((R_)1 - om) * lb[i] + om * (G0 + cdot<R_>(i, Gx, Gy, Gz));
        if (forced) lf += (cdot<R_>(i, Lx, Ly, Lz) - Lu) * irho;
        // element of A this population was pulled from
        const int src = c + nb.off(-cx(i), -cy(i), -cz(i));
        size_t dst = (fr[src] & F_SOLID) ? (size_t)opp(i) * N + (size_t)c : (size_t)i * N + (size_t)src;
        lAr[dst] = (T)lf;
      }
    }
  }
}

// Clear the forced bits and node lists after a reverse step (the step
// counter is not advanced).
__global__ void k_adj_cleanup(Dev d, int nslots, int maxlist) {
  int k = blockIdx.x * blockDim.x + threadIdx.x;
  int nt = (int)d.ctrl->touched;
  if (k < nt && k < maxlist) {
    int2 e = d.touched[k];
    uint8_t* f = d.flags + d.reps[e.x].node_off + e.y;
    *f = *f & (uint8_t)~F_FORCED;
  }
  if (k < nslots) {
    const Rep& R = d.reps[d.slot_rep[k]];
    if (k - R.slot_off < R.mp.nb) d.head[R.node_off + d.base[k]] = -1;
  }
}
__global__ void k_adj_touched_reset(Ctrl* ctrl) { ctrl->touched = 0u; }

// grads = [dL/dgamma, dL/dF_drive, dL/dr_0 (nb x 3)]
__global__ void k_adj_finish(AdjBufs a, double* __restrict__ grads, int n3) {
  int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < 2) grads[k] = a.par[k];
  if (k < n3) grads[2 + k] = a.lr[k];
}

// ---------------------------------------------------------------------------
static inline unsigned nblk(long n, int bs) { return (unsigned)((n + bs - 1) / bs); }

void launch_adj_init(const double* dLdr, const double* dLdv, const AdjBufs& a, int nb, hipStream_t s) {
  long n = 3L * nb > 4 ? 3L * nb : 4;
  hipLaunchKernelGGL(k_adj_init, dim3(nblk(n, 256)), dim3(256), 0, s, dLdr, dLdv, a, 3 * nb);
}

template <typename T, bool DEV>
void launch_adj_reverse_step(const void* A, const void* lamB, void* lamA, const Dev& d, const Dev& dspread,
                             const AdjBufs& a, const double* mdt, const double* upt,
                             const double* Jt, uint32_t step, double kT, int ntiles, int tile_nodes, int nslots,
                             int nb, int n_sub, hipStream_t s) {
  launch_bead_prep(d, nslots, s);
  hipLaunchKernelGGL((k_adj_spread_t<T>), dim3(nblk(nb, 64)), dim3(64), 0, s, (const T*)lamB, d, a, Jt, nb);
  size_t lds = sizeof(double) * (24 * (size_t)nb + 2 * (ADJ_WG / ADJ_LANES));
  if (kT != 0.0) {   // sigma > 0 exactly when kT > 0 (gamma > 0 here)
    hipLaunchKernelGGL(k_adj_noise, dim3(nblk((long)nb * n_sub, 256)), dim3(256), 0, s, d, a.xi, step, nb, n_sub);
  }
  hipLaunchKernelGGL(k_adj_md, dim3(1), dim3(ADJ_WG), lds, s, d, a, mdt, upt, step, kT);
  hipLaunchKernelGGL((k_adj_gather_t<T, DEV>), dim3(nblk(nb, 64)), dim3(64), 0, s, (const T*)A, d, a, nb);
  launch_spread<T>(dspread, nslots, s);
  hipLaunchKernelGGL((k_adj_lb<T, DEV>), dim3((unsigned)ntiles), dim3(256), 0, s, (const T*)A, (const T*)lamB,
                     (T*)lamA, d, (const T*)a.lamu, ntiles, tile_nodes);
  int maxlist = 8 * nslots;
  int n = nslots > maxlist ? nslots : maxlist;
  hipLaunchKernelGGL(k_adj_cleanup, dim3(nblk(n, 256)), dim3(256), 0, s, d, nslots, maxlist);
  hipLaunchKernelGGL(k_adj_touched_reset, dim3(1), dim3(1), 0, s, d.ctrl);
}

void launch_adj_finish(const AdjBufs& a, double* grads, int nb, hipStream_t s) {
  long n = 3L * nb > 2 ? 3L * nb : 2;
  hipLaunchKernelGGL(k_adj_finish, dim3(nblk(n, 256)), dim3(256), 0, s, a, grads, 3 * nb);
}

template void launch_adj_reverse_step<double, false>(const void*, const void*, void*, const Dev&, const Dev&,
                                                     const AdjBufs&, const double*, const double*, const double*,
                                                     uint32_t, double, int, int, int, int, int, hipStream_t);
template void launch_adj_reverse_step<float, true>(const void*, const void*, void*, const Dev&, const Dev&,
                                                   const AdjBufs&, const double*, const double*, const double*,
                                                   uint32_t, double, int, int, int, int, int, hipStream_t);

}  // namespace lbmd
