// md_kernels.hip -- the bead sub-cycle: stochastic position Verlet sub-steps
// (Sec. 2, Eq. (SPValgo), no constraints) with the fluid velocity at each
// bead frozen for the whole cycle.  One launch per sub-step; the positions
// at which forces are evaluated are double buffered so that every bead reads
// a consistent snapshot.  Every replica of a context advances in the same
// launches; a workgroup never mixes replicas.
//
// Per sub-step s (h = 1/n_sub, e = exp(-gamma h)):
//   r_mid = r + h/2 v                      (written by the previous launch)
//   F     = bonds + bending + LJ + wall + field at r_mid
//   v'    = e v + (1-e)/(m gamma) (F + gamma u_p) + sig xi
//   J    -= m [(1-e)(u_p - v) + sig xi]    (friction + noise impulse)
//   r'    = r_mid + h/2 v'
// The next launch's r_mid = r' + h/2 v' is formed here as two separate
// additions, the same rounding as two half drifts.
//
// The LJ sum runs over a Verlet neighbour list (radius r_c + skin) kept in
// ascending bead order, so it adds exactly the terms of the all-pairs loop
// in the same order.  A list is rebuilt in the launch after any bead has
// moved more than skin/2 since the last build; the flag is carried between
// launches in three rotating words.
#include "lbmd_kernels.h"

namespace lbmd {

// Per replica r, rb[4 r + 0..2] are the three rotating rebuild flags and
// rb[4 r + 3] the "lists invalid" request from the host (initialisation,
// restored state).
__global__ void k_md_begin(uint32_t* rb, uint32_t* cst, int nrep, int* redo) {
  for (int r = threadIdx.x; r < nrep; r += blockDim.x) {
    if (redo) redo[r] = -1;
    uint32_t* w = rb + 4 * r;
    w[0] = w[3];
    w[1] = 0u;
    w[2] = 0u;
    w[3] = 0u;
    cst[4 * r] = 0u;
    cst[4 * r + 1] = 0u;
    cst[4 * r + 2] = 0u;
  }
}

__global__ void k_md_invalidate(uint32_t* rb, int nrep) {
  for (int r = threadIdx.x; r < nrep; r += blockDim.x) rb[4 * r + 3] = 1u;
}

// Coefficients of the sub-cycle for one replica: its own, or the
// relaxation's (no coupling, no field, no noise).
__device__ inline MdParams md_params(const Rep& R, const MdOverride& ov) {
  MdParams P = R.mp;
  if (ov.on) {
    P.gamma = ov.gamma; P.e = ov.e; P.omE = ov.omE;
    P.cf = ov.gamma == 0.0 ? (2.0 * P.hh) / P.m : ov.omE / (P.m * ov.gamma);
    P.sig = 0.0; P.couple = 0; P.field_on = 0;
  }
  return P;
}

// Neighbour-search cells: side >= r_c + skin + CELL_MARGIN per replica; each
// cell hashes to one bucket of a power-of-two table of fixed-capacity buckets
// (colliding cells share a bucket: their beads fail the distance test).
__device__ inline uint32_t cell_bucket(int rep, int cx, int cy, int cz, uint32_t mask) {
  uint32_t h = ((uint32_t)rep * 73856093u) ^ ((uint32_t)cx * 19349663u) ^ ((uint32_t)cy * 83492791u) ^
               ((uint32_t)cz * 2654435761u);
  return h & mask;
}

__device__ inline void bead_cell(const Rep& R, const double* rp, int c[3]) {
  const int n[3] = {R.g.nx, R.g.ny, R.g.nz};
  for (int a = 0; a < 3; ++a) {
    double w = wrapc(rp[a], n[a]);
    if (!(w >= 0.0 && w < (double)n[a])) w = 0.0;   // non-finite: still a valid cell
    int k = (int)(w * (double)R.ncell[a] / (double)n[a]);
    c[a] = k < R.ncell[a] ? k : R.ncell[a] - 1;
  }
}

// r_mid of sub-step 0 (with mts: r itself, where the first slow kick
// evaluates its forces) and the displacement check that decides whether the
// first launch rebuilds the lists.
__global__ void k_md_start(Dev d, int nslots, MdOverride ov, int mts) {
  int slot = blockIdx.x * blockDim.x + threadIdx.x;
  if (slot >= nslots) return;
  const int rep = d.slot_rep[slot];
  const Rep& R = d.reps[rep];
  if (slot - R.slot_off >= R.mp.nb) return;
  const double hh = R.mp.hh;
  double d2 = 0.0, b2 = 0.0;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    double x = mts ? d.r[3 * slot + a] : d.r[3 * slot + a] + hh * d.v[3 * slot + a];
    d.rmid0[3 * slot + a] = x;
    double dd = x - d.ref[3 * slot + a];
    d2 += dd * dd;
    double db = x - d.rbin[3 * slot + a];
    b2 += db * db;
  }
  if (d2 > R.mp.halfskin2) d.rb[4 * rep] = 1u;
  if (!(b2 <= CELL_MARGIN * CELL_MARGIN)) d.cst[4 * rep] = 1u;
}

// The noise of a whole sub-cycle at once: xi[(s nslots + slot) 3 + a] for
// every sub-step s and bead (the same counter-based values the sub-step would
// draw, keyed by the replica's seed and index and the bead's chain index), so
// the transcendental functions run in one wide launch instead of on the
// critical path of every sub-step.  The step counter word is the control
// block's step plus step_offset (1: the sub-cycle of the next step).
__global__ void k_md_noise(Dev d, int nslots, int n_sub, int step_offset) {
  long k = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= (long)n_sub * nslots) return;
  int sidx = (int)(k / nslots), slot = (int)(k - (long)sidx * nslots);
  const Rep& R = d.reps[d.slot_rep[slot]];
  const int p = slot - R.slot_off;
  if (p >= R.mp.nb || R.mp.sig == 0.0) return;
  double x[3];
  gauss3(R.mp.seed, R.mp.replica, (uint32_t)(d.ctrl->step + (uint64_t)step_offset), (uint32_t)sidx, (uint32_t)p, x);
  d.xi[3 * k] = x[0]; d.xi[3 * k + 1] = x[1]; d.xi[3 * k + 2] = x[2];
}

// The bending angle at (ra, rb, rc) and what its forces need: the bond
// vectors, their cross product n, |n| = s, b1.b2 = c, phi = atan2(s, c),
// s^2 + c^2 and kappa phi.  s = 0 (straight or folded) has no unique
// gradient: its forces are exactly 0.
struct AngleCore {
  double b1[3], b2[3], n[3];
  double s, c, den, kp;
};
__device__ inline bool angle_core(const MdParams& P, const double* ra, const double* rb, const double* rc,
                                  AngleCore& A) {
  for (int a = 0; a < 3; ++a) { A.b1[a] = rb[a] - ra[a]; A.b2[a] = rc[a] - rb[a]; }
  A.n[0] = A.b1[1] * A.b2[2] - A.b1[2] * A.b2[1];
  A.n[1] = A.b1[2] * A.b2[0] - A.b1[0] * A.b2[2];
  A.n[2] = A.b1[0] * A.b2[1] - A.b1[1] * A.b2[0];
  A.s = sqrt(A.n[0] * A.n[0] + A.n[1] * A.n[1] + A.n[2] * A.n[2]);
  A.c = A.b1[0] * A.b2[0] + A.b1[1] * A.b2[1] + A.b1[2] * A.b2[2];
  if (A.s == 0.0) return false;
  const double phi = atan2(A.s, A.c);
  A.den = A.s * A.s + A.c * A.c;
  A.kp = P.kappa * phi;
  return true;
}
// Component a of the angle's forces: out[0] on the first bead, out[1] on the
// centre, out[2] on the third -- the operations of angle_component (and of
// angle_add) for that component, evaluated from one AngleCore.
__device__ inline void angle_part(const AngleCore& A, int a, double out[3]) {
  const int a1 = (a + 1) % 3, a2 = (a + 2) % 3;
  double g1 = A.b2[a1] * A.n[a2] - A.b2[a2] * A.n[a1];
  double g2 = A.n[a1] * A.b1[a2] - A.n[a2] * A.b1[a1];
  double d1 = (A.c * g1 / A.s - A.s * A.b2[a]) / A.den;
  double d2 = (A.c * g2 / A.s - A.s * A.b1[a]) / A.den;
  out[0] = 0.0 + A.kp * d1;
  out[1] = 0.0 + -(A.kp * (d1 - d2));
  out[2] = 0.0 + -(A.kp * d2);
}
__device__ inline void angle_component(const MdParams& P, const double* ra, const double* rb, const double* rc,
                                       int a, double out[3]) {
  double b1[3] = {rb[0] - ra[0], rb[1] - ra[1], rb[2] - ra[2]};
  double b2[3] = {rc[0] - rb[0], rc[1] - rb[1], rc[2] - rb[2]};
  double n[3] = {b1[1] * b2[2] - b1[2] * b2[1], b1[2] * b2[0] - b1[0] * b2[2], b1[0] * b2[1] - b1[1] * b2[0]};
  double s = sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
  double c = b1[0] * b2[0] + b1[1] * b2[1] + b1[2] * b2[2];
  if (s == 0.0) {
    // straight or folded: the contribution is exactly 0 (as in angle_add)
    out[0] = 0.0; out[1] = 0.0; out[2] = 0.0;
    return;
  }
  double phi = atan2(s, c);
  double den = s * s + c * c;
  const int a1 = (a + 1) % 3, a2 = (a + 2) % 3;
  double g1 = b2[a1] * n[a2] - b2[a2] * n[a1];
  double g2 = n[a1] * b1[a2] - n[a2] * b1[a1];
  double kp = P.kappa * phi;
  double d1 = (c * g1 / s - s * b2[a]) / den;
  double d2 = (c * g2 / s - s * b1[a]) / den;
  out[0] = 0.0 + kp * d1;
  out[1] = 0.0 + -(kp * (d1 - d2));
  out[2] = 0.0 + -(kp * d2);
}

// ---------------------------------------------------------------------------
// Sub-step kernel.  A workgroup holds 16 consecutive bead slots of one
// replica in three waves that work side by side: in the first, 4 lanes per
// bead evaluate its LJ pair forces; the second evaluates the bending of the
// 18 angles that touch the 16 beads, one lane per angle and component; the
// third the wall sites, one lane per bead and window row, and the bonds.  All
// go to LDS.  One lane per bead of the third wave then adds every
// contribution in the fixed order of the definition (bonds to p-1 and p+1,
// the angles centred at p-1, p, p+1, LJ in ascending partner order, wall
// sites, field), so the sum is the same as a one-thread-per-bead loop, and
// moves the bead.  Spreading the work keeps each wave's registers few, so
// that the workgroups fit on CUs beside the lattice sweep.
// ---------------------------------------------------------------------------
constexpr int MD_LANES = 4;
constexpr int MD_WG = MD_LANES * MD_BPB;     // 64
constexpr int WLO = -2, WHI = 3;             // wall-site window: offsets -2..3 from the base node (r_c <= 3)
constexpr int WSPAN = WHI - WLO + 1;         // 6
constexpr int MAXWALL = WSPAN * WSPAN;       // the 6 x 6 window of wall sites in the wall plane
constexpr int NB_PER_LANE = MAXNBR / MD_LANES;

struct MdShared {
  double ang[MD_BPB + 2][9];                 // forces of the angles centred at p0-1 .. p0+16: [0..2] on
                                             // q-1, [3..5] on q, [6..8] on q+1
  double pairF[MD_BPB][MAXNBR][3];           // LJ pair force of list entry k
  uint32_t hit[MD_BPB][MD_LANES];            // lane l, bit m: entry l + 4m is within r_c
  uint32_t wmask[MD_BPB][WSPAN];             // row o1 - WLO: which sites o0 - WLO of the row are set
  int cnt[MD_BPB];
  int lst[MD_BPB][MAXNBR];                   // the neighbour list in use (partner slots)
  // the list rebuild's scratch is dead before the wall sites are written
  union {
    struct {
      double tile[MD_WG][3];                 // rebuild: positions of 64 candidates
      uint32_t tmask[MD_BPB][MD_LANES];      // rebuild: lane l, bit e: candidate 16 l + e is close
      uint32_t bk[MD_BPB][28];               // rebuild from the cell table: the 27 buckets around a bead
    };
    double wallF[MD_BPB][MAXWALL][3];        // wall site (o1 - WLO) * WSPAN + (o0 - WLO) of each bead
  };
  int over;
};
static_assert(2 * sizeof(MdShared) <= (size_t)LDS_KEEP, "two sub-step workgroups fit in the LDS a capped sweep leaves");

// Wall sites of the bead at rp, one row of the window at a time: the sites
// at offsets P.wlo..P.whi (within -2..3) from the base node along the lower
// transverse axis (o0), for offset o1 along the higher one; offsets outside
// 1 - ceil(r_c) .. ceil(r_c) cannot reach r_c, so the window shrinks to
// -1..2 for r_c <= 2.  Each is the truncated-LJ pair force of
// one solid site within r_c; the force of offset o0 goes to out[o0 - WLO] and
// the returned mask has bit o0 - WLO set.  r_c <= 3 makes the window cover
// every candidate.  Solid sites lie in the plane a = wall_pos (minus the
// pore), so at most one offset along the wall normal can match.  Rows
// o1 = -2..3, each in o0 order, visit the sites in the order of the
// definition's sum (higher transverse axis outer).  Wrapping uses compares
// only (the window is within one period: extents are at least 6).
__device__ inline uint32_t wall_row(const MdParams& P, const Geom& g, const double* rp, int o1,
                                    double out[WSPAN][3]) {
  if (g.wall_axis < 0) return 0u;
  const double w0 = wrapc(rp[0], g.nx), w1 = wrapc(rp[1], g.ny), w2 = wrapc(rp[2], g.nz);
  const int b0 = (int)floor(w0), b1 = (int)floor(w1), b2 = (int)floor(w2);
  const int a = g.wall_axis;
  // normal-axis base and extent; transverse axes t0 < t1
  const int ba = a == 0 ? b0 : (a == 1 ? b1 : b2);
  const int na = a == 0 ? g.nx : (a == 1 ? g.ny : g.nz);
  const int bt0 = a == 0 ? b1 : b0, n0 = a == 0 ? g.ny : g.nx;
  const int bt1 = a == 2 ? b1 : b2, n1 = a == 2 ? g.ny : g.nz;
  int off = g.wall_pos - ba;                // offset along the normal reaching the plane
  if (off < WLO) off += na;
  if (off > WHI) off -= na;
  if (off < P.wlo || off > P.whi) return 0u;
  const int sa = ba + off;
  const int u1 = bt1 + o1;
  const int v1 = u1 < 0 ? u1 + n1 : (u1 >= n1 ? u1 - n1 : u1);
  const bool in1 = v1 >= g.lo1 && v1 <= g.hi1;
  uint32_t mask = 0u;
  for (int o0 = P.wlo; o0 <= P.whi; ++o0) {
    const int u0 = bt0 + o0;
    const int v0 = u0 < 0 ? u0 + n0 : (u0 >= n0 ? u0 - n0 : u0);
    const bool in0 = v0 >= g.lo0 && v0 <= g.hi0;
    if (in0 && in1) continue;               // pore node: fluid
    const int sx = a == 0 ? sa : u0;
    const int sy = a == 1 ? sa : (a == 0 ? u0 : u1);
    const int sz = a == 2 ? sa : u1;
    const double d0 = w0 - (double)sx, d1 = w1 - (double)sy, d2 = w2 - (double)sz;
    if (!(d0 * d0 + d1 * d1 + d2 * d2 < P.rc2)) continue;
    double F[3] = {0.0, 0.0, 0.0};
    lj_add(P, d0, d1, d2, F);
    out[o0 - WLO][0] = F[0]; out[o0 - WLO][1] = F[1]; out[o0 - WLO][2] = F[2];
    mask |= 1u << (o0 - WLO);
  }
  return mask;
}

// SLOW: a kick of the multiple-time-step cycle instead of a sub-step.  The
// slow forces (bead LJ, wall sites, field) are evaluated at r, which does not
// change, and `last` half kicks v += kick F are applied one after the other
// (2 between two outer steps, 1 at the ends); s is the kick's index in the
// cycle (0..M), which selects the rotating rebuild words.
template <bool SLOW>
__global__ __launch_bounds__(3 * MD_WG) void k_md_substep(Dev d, MdOverride ov, int nslots, int s, int last) {
  __shared__ MdShared sh;
  const int t = threadIdx.x;
  // wave 0 holds the neighbour lists and LJ pairs (4 lanes per bead), wave 1
  // evaluates the angles, wave 2 the wall sites and bonds and then moves the
  // beads.  Every wave takes every barrier: the branches around barriers are
  // uniform in the workgroup.
  const int wave = __builtin_amdgcn_readfirstlane(t) / MD_WG;
  const int tb = t - wave * MD_WG;           // lane within the wave
  const int bslot = tb / MD_LANES, lane = tb % MD_LANES;
  const int slot0 = blockIdx.x * MD_BPB;
  const int slot = slot0 + bslot;            // the grid covers the nslots slots exactly
  const double* rabs = SLOW ? d.r : ((s & 1) ? d.rmid1 : d.rmid0);
  double* rout = (s & 1) ? d.rmid0 : d.rmid1;
  auto clampslot = [nslots](int q) { return q < 0 ? 0 : (q >= nslots ? nslots - 1 : q); };

  // ---- first-level loads, addressed by slot alone so that they are in
  // flight before the replica's parameters arrive.  Indices are clamped into
  // the slot range; a value from outside the chain is never used.
  double rp[3] = {0.0, 0.0, 0.0};
  int* nbr_row = d.nbr + (size_t)slot * MAXNBR;
  int ncnt_in = 0;
  int pre[NB_PER_LANE];                       // list entries lane, lane + 4, ... (past the length unused)
  double vo[3], Jo[3], ul[3], xl[3], rm[3], rq[3], rbl[3], rfl[3];
  double ra[3] = {0.0, 0.0, 0.0}, rb3[3] = {0.0, 0.0, 0.0}, rc[3] = {0.0, 0.0, 0.0};
  if (wave == 0) {
    rp[0] = rabs[3 * slot]; rp[1] = rabs[3 * slot + 1]; rp[2] = rabs[3 * slot + 2];
    ncnt_in = d.ncnt[slot];
#pragma unroll
    for (int m = 0; m < NB_PER_LANE; ++m) pre[m] = nbr_row[lane + MD_LANES * m];
  } else if (wave == 1) {
    if (!SLOW && tb < 3 * (MD_BPB + 2)) {
      // positions of the angle centred at slot slot0 - 1 + tb / 3
      const int c = slot0 - 1 + tb / 3;
      const int ia = clampslot(c - 1), ib = clampslot(c), ic = clampslot(c + 1);
#pragma unroll
      for (int a = 0; a < 3; ++a) { ra[a] = rabs[3 * ia + a]; rb3[a] = rabs[3 * ib + a]; rc[a] = rabs[3 * ic + a]; }
    }
  } else {
    rp[0] = rabs[3 * slot]; rp[1] = rabs[3 * slot + 1]; rp[2] = rabs[3 * slot + 2];
  }

  // ---- the replica
  const int rep = d.slot_rep[slot0];
  const Rep& R = d.reps[rep];
  const MdParams P = md_params(R, ov);
  const Geom g = R.g;
  const int so = R.slot_off;
  const int p0 = slot0 - so;                 // chain index of the first bead here
  const int p = p0 + bslot;
  const bool active = wave == 0 && p < P.nb;
  const double* rin = rabs + 3 * (size_t)so; // chain-relative
  uint32_t* rbr = d.rb + 4 * rep;
  const uint32_t rebuild = rbr[s % 3];
  const uint32_t table_stale = d.cst[4 * rep + s % 3];
  if (t == 0) {
    if (p0 == 0) {
      rbr[(s + 2) % 3] = 0u;
      d.cst[4 * rep + (s + 2) % 3] = 0u;
      if (rebuild) atomicAdd((unsigned long long*)&d.ctrl->rebuilds, 1ull);
      if (rebuild && !table_stale) atomicAdd((unsigned long long*)&d.ctrl->cell_rebuilds, 1ull);
    }
    if (!SLOW && blockIdx.x == 0) atomicAdd((unsigned long long*)&d.ctrl->substeps, 1ull);
    sh.over = 0;
  }
  // lane 0 of each bead in wave 2 adds the contributions and moves the bead
  const bool lead = wave == 2 && lane == 0 && p < P.nb;
  const int ncnt0 = active ? ncnt_in : 0;

  // ---- neighbour list: reuse (already in registers), or rebuild -- from
  // the cell table while every bead of the chain is within CELL_MARGIN of
  // where the table binned it, else by scanning the chain in tiles of 64
  int cnt = ncnt0;
  int jl[NB_PER_LANE];
  if (!rebuild) {
#pragma unroll
    for (int m = 0; m < NB_PER_LANE; ++m) jl[m] = (lane + MD_LANES * m < cnt) ? pre[m] : -1;
  } else {
    if (wave == 0 && lane == 0) sh.cnt[bslot] = 0;
    if (!table_stale) {
      // lane l scans the distinct buckets l, l + 4, ... of the 27 cells
      // around the bead (a candidate binned within CELL_MARGIN of its
      // position lies in one of them); the lead lane then sorts
      if (active) {
        int c[3];
        bead_cell(R, rp, c);
        for (int k = lane; k < 27; k += MD_LANES) {
          const int dx = k % 3 - 1, dy = (k / 3) % 3 - 1, dz = k / 9 - 1;
          sh.bk[bslot][k] = cell_bucket(rep, (c[0] + dx + R.ncell[0]) % R.ncell[0],
                                        (c[1] + dy + R.ncell[1]) % R.ncell[1], (c[2] + dz + R.ncell[2]) % R.ncell[2],
                                        d.cmask);
        }
      }
      __syncthreads();
      if (active) {
        for (int k = lane; k < 27; k += MD_LANES) {
          const uint32_t b = sh.bk[bslot][k];
          bool dup = false;
          for (int k2 = 0; k2 < k; ++k2) dup = dup || sh.bk[bslot][k2] == b;
          if (dup) continue;
          const int n = min(d.ccount[b], CELL_CAP);
          for (int e = 0; e < n; ++e) {
            const int q = d.cbuf[(size_t)b * CELL_CAP + e];
            if (d.slot_rep[q] != rep || q == slot) continue;
            double d0 = min_image(rp[0] - rabs[3 * q], g.nx);
            double d1 = min_image(rp[1] - rabs[3 * q + 1], g.ny);
            double d2 = min_image(rp[2] - rabs[3 * q + 2], g.nz);
            if (!(d0 * d0 + d1 * d1 + d2 * d2 < P.rlist2)) continue;
            const int at = atomicAdd(&sh.cnt[bslot], 1);
            if (at < MAXNBR) sh.lst[bslot][at] = q;
            else sh.over = 1;
          }
        }
      }
      __syncthreads();
      if (active && lane == 0) {
        const int c = min(sh.cnt[bslot], MAXNBR);
        int* L = sh.lst[bslot];
        for (int i = 1; i < c; ++i) {
          const int v = L[i];
          int m = i;
          while (m > 0 && L[m - 1] > v) { L[m] = L[m - 1]; --m; }
          L[m] = v;
        }
      }
    } else {
      for (int base = 0; base < P.nb; base += MD_WG) {
        __syncthreads();
        const int j = base + tb;
        if (wave == 0 && j < P.nb) {
          sh.tile[tb][0] = rin[3 * j]; sh.tile[tb][1] = rin[3 * j + 1]; sh.tile[tb][2] = rin[3 * j + 2];
        }
        __syncthreads();
        uint32_t m = 0;
        if (active) {
          for (int e = 0; e < 16; ++e) {
            int tt = 16 * lane + e;
            int jj = base + tt;
            if (jj >= P.nb || jj == p) continue;
            double d0 = min_image(rp[0] - sh.tile[tt][0], g.nx);
            double d1 = min_image(rp[1] - sh.tile[tt][1], g.ny);
            double d2 = min_image(rp[2] - sh.tile[tt][2], g.nz);
            if (d0 * d0 + d1 * d1 + d2 * d2 < P.rlist2) m |= 1u << e;
          }
        }
        if (wave == 0) sh.tmask[bslot][lane] = m;
        __syncthreads();
        if (active && lane == 0) {
          uint64_t mm = (uint64_t)sh.tmask[bslot][0] | ((uint64_t)sh.tmask[bslot][1] << 16) |
                        ((uint64_t)sh.tmask[bslot][2] << 32) | ((uint64_t)sh.tmask[bslot][3] << 48);
          int c = sh.cnt[bslot];
          while (mm) {
            int tt = __builtin_ctzll(mm);
            mm &= mm - 1;
            if (c < MAXNBR) sh.lst[bslot][c] = so + base + tt;
            else sh.over = 1;
            ++c;
          }
          sh.cnt[bslot] = c;
        }
      }
    }
    __syncthreads();
    if (active && lane == 0) {
      int c = sh.cnt[bslot];
      if (c > MAXNBR) { c = MAXNBR; sh.cnt[bslot] = c; }
      d.ncnt[slot] = c;
      d.ref[3 * slot] = rp[0]; d.ref[3 * slot + 1] = rp[1]; d.ref[3 * slot + 2] = rp[2];
    }
    __syncthreads();
    cnt = active ? sh.cnt[bslot] : 0;
    for (int k = lane; k < cnt; k += MD_LANES) nbr_row[k] = sh.lst[bslot][k];
    if (t == 0 && sh.over) atomicOr(&d.ctrl->err, E_NBRLIST);
#pragma unroll
    for (int m = 0; m < NB_PER_LANE; ++m) {
      int k = lane + MD_LANES * m;
      jl[m] = (k < cnt) ? sh.lst[bslot][k] : -1;
    }
  }

  double F[3] = {0.0, 0.0, 0.0};
  if (wave == 1) {
    // ---- the angles centred at p0 - 1 .. p0 + 16: lane 3 k + a takes
    // component a of angle k
    if (!SLOW && tb < 3 * (MD_BPB + 2)) {
      const int k = tb / 3, a = tb % 3;
      const int qc = p0 - 1 + k;
      if (qc >= 1 && qc <= P.nb - 2) {
        double f[3];
        angle_component(P, ra, rb3, rc, a, f);
        sh.ang[k][a] = f[0]; sh.ang[k][3 + a] = f[1]; sh.ang[k][6 + a] = f[2];
      }
    }
  } else if (wave == 2) {
    // the bead's own state, its chain neighbours and its list references
    // (every lane of the bead reads them; lane 0 uses them).  Loaded here,
    // not with the first loads, so that they hold no registers while the
    // other waves work; they are needed only at the end.
    if (SLOW) {
#pragma unroll
      for (int a = 0; a < 3; ++a) vo[a] = d.v[3 * slot + a];
    } else {
      const int sm = clampslot(slot - 1), sq = clampslot(slot + 1);
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        rbl[a] = d.rbin[3 * slot + a];
        rfl[a] = d.ref[3 * slot + a];
        vo[a] = d.v[3 * slot + a];
        Jo[a] = d.J[3 * slot + a];
        ul[a] = d.up[3 * slot + a];
        xl[a] = ov.on ? 0.0 : d.xi[(size_t)3 * ((size_t)s * nslots + slot) + a];
        rm[a] = rabs[3 * sm + a];
        rq[a] = rabs[3 * sq + a];
      }
    }
    // ---- wall sites: rows outside wlo..whi hold no site within r_c and
    // stay empty; lane l takes the rows o1 = wlo + l, wlo + l + 4, ... (for
    // r_c <= 2 one row per lane, all lanes at once).  The clearing stores
    // precede the row stores of the same wave.
    for (int row = lane; row < WSPAN; row += MD_LANES) sh.wmask[bslot][row] = 0u;
    for (int o1 = P.wlo + lane; o1 <= P.whi; o1 += MD_LANES)
      sh.wmask[bslot][o1 - WLO] = p < P.nb ? wall_row(P, g, rp, o1, &sh.wallF[bslot][WSPAN * (o1 - WLO)]) : 0u;
    // ---- lane 0: bonds now, the rest after the barrier
    if (!SLOW && lead && !P.constrained) {
      if (p > 0) bond_add(P, rp, rm, F);
      if (p < P.nb - 1) bond_add(P, rp, rq, F);
    }
  } else {
    // ---- LJ pair forces: lane l handles list entries l, l + 4, l + 8, ...
    double q[NB_PER_LANE][3];
#pragma unroll
    for (int m = 0; m < NB_PER_LANE; ++m) {
      const int j = jl[m] >= 0 ? jl[m] : slot0;   // an unused entry reads a valid slot
      q[m][0] = rabs[3 * j]; q[m][1] = rabs[3 * j + 1]; q[m][2] = rabs[3 * j + 2];
    }
    uint32_t hit = 0;
#pragma unroll
    for (int m = 0; m < NB_PER_LANE; ++m) {
      if (jl[m] < 0) continue;
      double d0 = min_image(rp[0] - q[m][0], g.nx);
      double d1 = min_image(rp[1] - q[m][1], g.ny);
      double d2 = min_image(rp[2] - q[m][2], g.nz);
      if (!(d0 * d0 + d1 * d1 + d2 * d2 < P.rc2)) continue;
      double Fp[3] = {0.0, 0.0, 0.0};
      lj_add(P, d0, d1, d2, Fp);
      int k = lane + MD_LANES * m;
      sh.pairF[bslot][k][0] = Fp[0]; sh.pairF[bslot][k][1] = Fp[1]; sh.pairF[bslot][k][2] = Fp[2];
      hit |= 1u << m;
    }
    sh.hit[bslot][lane] = hit;
    if (lane == 0) sh.cnt[bslot] = cnt;
  }
  __syncthreads();
  if (!lead) return;
  // every contribution in the fixed order
  const int cnt_b = sh.cnt[bslot];
  const int q0 = p0 - 1;
  const int nb = P.nb;
  if (!SLOW) {
    if (p - 1 >= 1 && p - 1 <= nb - 2) { const double* A = sh.ang[p - 1 - q0]; F[0] += A[6]; F[1] += A[7]; F[2] += A[8]; }
    if (p >= 1 && p <= nb - 2) { const double* A = sh.ang[p - q0]; F[0] += A[3]; F[1] += A[4]; F[2] += A[5]; }
    if (p + 1 >= 1 && p + 1 <= nb - 2) { const double* A = sh.ang[p + 1 - q0]; F[0] += A[0]; F[1] += A[1]; F[2] += A[2]; }
  }
  // the list entries with a pair force, in list order: entry k is bit
  // k / 4 of lane k % 4's word; interleaved into one mask so that only the
  // hits are visited (lists are much longer than the pairs within r_c)
  {
    uint32_t h[MD_LANES];
#pragma unroll
    for (int l = 0; l < MD_LANES; ++l) h[l] = sh.hit[bslot][l];
    uint64_t hm = 0;
#pragma unroll
    for (int e = 0; e < NB_PER_LANE; ++e)
#pragma unroll
      for (int l = 0; l < MD_LANES; ++l) hm |= (uint64_t)((h[l] >> e) & 1u) << (MD_LANES * e + l);
    (void)cnt_b;
    while (hm) {
      const int k = __builtin_ctzll(hm);
      hm &= hm - 1;
      F[0] += sh.pairF[bslot][k][0]; F[1] += sh.pairF[bslot][k][1]; F[2] += sh.pairF[bslot][k][2];
    }
  }
  // the wall sites within r_c, in ascending site order (set bits only: most
  // beads have none)
  uint64_t wm = 0;
#pragma unroll
  for (int row = 0; row < WSPAN; ++row) wm |= (uint64_t)sh.wmask[bslot][row] << (WSPAN * row);
  while (wm) {
    const int k = __builtin_ctzll(wm);
    wm &= wm - 1;
    F[0] += sh.wallF[bslot][k][0]; F[1] += sh.wallF[bslot][k][1]; F[2] += sh.wallF[bslot][k][2];
  }
  if (P.field_on && in_field(g, rp)) F[g.wall_axis] += P.f_drive;

  if (SLOW) {
    bool fin = true;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      double vn = vo[a] + P.kick * F[a];
      if (last == 2) vn = vn + P.kick * F[a];
      d.v[3 * slot + a] = vn;
      fin = fin && isfinite(vn);
    }
    if (!fin) atomicOr(&d.ctrl->err, E_BEADS);
    return;
  }

  double u[3], xi[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    u[a] = P.couple ? ul[a] : 0.0;
    xi[a] = P.sig != 0.0 ? xl[a] : 0.0;
  }
  double vn[3];
  bool finite = true;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    double sx = P.sig * xi[a];
    vn[a] = P.e * vo[a] + P.cf * (F[a] + P.gamma * u[a]) + sx;
    d.J[3 * slot + a] = Jo[a] - P.m * (P.omE * (u[a] - vo[a]) + sx);
    d.v[3 * slot + a] = vn[a];
    finite = finite && isfinite(vn[a]);
  }
  if (!finite) atomicOr(&d.ctrl->err, E_BEADS);
  // rigid bonds: RATTLE, the drift and the next SHAKE follow in
  // k_md_constraint, which also sets the rebuild words
  if (P.constrained) return;
  if (d.mdtape) {
    double* tp = d.mdtape + ((size_t)s * P.nb + p) * 6;
    tp[0] = rp[0]; tp[1] = rp[1]; tp[2] = rp[2];
    tp[3] = vo[0]; tp[4] = vo[1]; tp[5] = vo[2];
  }
  double re[3] = {rp[0] + P.hh * vn[0], rp[1] + P.hh * vn[1], rp[2] + P.hh * vn[2]};
  if (last) {
    d.r[3 * slot] = re[0]; d.r[3 * slot + 1] = re[1]; d.r[3 * slot + 2] = re[2];
  } else {
    double d2 = 0.0, b2 = 0.0;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      double x = re[a] + P.hh * vn[a];
      rout[3 * slot + a] = x;
      double dd = x - (rebuild ? rp[a] : rfl[a]);   // a rebuild this sub-step set ref = r_mid
      d2 += dd * dd;
      double db = x - rbl[a];
      b2 += db * db;
    }
    if (d2 > P.halfskin2) rbr[(s + 1) % 3] = 1u;
    if (!(b2 <= CELL_MARGIN * CELL_MARGIN)) d.cst[4 * rep + (s + 1) % 3] = 1u;
  }
}

__global__ void k_zero_v(double* v, int n) {
  int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) v[k] = 0.0;
}

// ---------------------------------------------------------------------------
// Inner cycle of outer step o of the multiple-time-step scheme: M_b SPV
// sub-steps with the bonded forces only (bonds, bending), the friction
// towards the frozen u_p and the noise of sub-step index o M_b + i, all in
// one launch.  The bonded force on a bead depends on the chain neighbours
// p-2 .. p+2 only, so a workgroup advances a segment of IN_WG consecutive
// slots through the whole inner cycle with its positions in LDS and one
// barrier per sub-step; the 2 M_b slots at each end are a halo computed again
// by the neighbouring workgroup (after i sub-steps the missing neighbours
// beyond the segment have corrupted at most 2 i slots at each end), so each
// workgroup stores only the IN_WG - 4 M_b slots in the middle.  Sums follow
// the definition's order: bonds to p-1 and p+1, then the angles centred at
// p-1, p, p+1.  The last lane state also gives the displacement checks of the
// slow kick that follows (index o + 1).
// ---------------------------------------------------------------------------
constexpr int IN_WG = 256;

__global__ __launch_bounds__(IN_WG) void k_md_inner(Dev d, int nslots, int o, int Mb) {
  __shared__ double pos[2][IN_WG][3];
  const int j = threadIdx.x;
  const int H = 2 * Mb, own = IN_WG - 2 * H;
  const int gslot = (int)blockIdx.x * own - H + j;
  const bool valid = gslot >= 0 && gslot < nslots;
  const int slot = valid ? gslot : 0;
  const int rep = d.slot_rep[slot];
  const Rep& R = d.reps[rep];
  const int p = slot - R.slot_off;
  const int nb = R.mp.nb;
  const bool active = valid && p < nb;
  const double hh = R.mp.hh, e = R.mp.e, cf = R.mp.cf, gam = R.mp.gamma, omE = R.mp.omE, sig = R.mp.sig;
  const double m = R.mp.m;
  double r[3] = {0.0, 0.0, 0.0}, v[3] = {0.0, 0.0, 0.0}, J[3] = {0.0, 0.0, 0.0}, u[3] = {0.0, 0.0, 0.0};
  if (active) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      r[a] = d.r[3 * slot + a];
      v[a] = d.v[3 * slot + a];
      J[a] = d.J[3 * slot + a];
      u[a] = R.mp.couple ? d.up[3 * slot + a] : 0.0;
    }
  }
  // chain neighbour p + k is in the chain and in this segment
  auto has = [&](int k) { return p + k >= 0 && p + k < nb && j + k >= 0 && j + k < IN_WG; };
  for (int i = 0; i < Mb; ++i) {
    const int sidx = o * Mb + i;
    double xi[3] = {0.0, 0.0, 0.0};
    if (active && sig != 0.0) {
#pragma unroll
      for (int a = 0; a < 3; ++a) xi[a] = d.xi[(size_t)3 * ((size_t)sidx * nslots + slot) + a];
    }
    double rh[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      rh[a] = r[a] + hh * v[a];
      pos[i & 1][j][a] = rh[a];
    }
    __syncthreads();
    if (active) {
      const double(*q)[3] = pos[i & 1];
      double F[3] = {0.0, 0.0, 0.0};
      if (p > 0 && has(-1)) bond_add(R.mp, rh, q[j - 1], F);
      if (p < nb - 1 && has(1)) bond_add(R.mp, rh, q[j + 1], F);
      if (p - 1 >= 1 && p - 1 <= nb - 2 && has(-2)) angle_add(R.mp, q[j - 2], q[j - 1], rh, 2, F);
      if (p >= 1 && p <= nb - 2 && has(-1) && has(1)) angle_add(R.mp, q[j - 1], rh, q[j + 1], 1, F);
      if (p + 1 >= 1 && p + 1 <= nb - 2 && has(2)) angle_add(R.mp, rh, q[j + 1], q[j + 2], 0, F);
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        const double sx = sig * xi[a];
        const double vn = e * v[a] + cf * (F[a] + gam * u[a]) + sx;
        J[a] = J[a] - m * (omE * (u[a] - v[a]) + sx);
        v[a] = vn;
        r[a] = rh[a] + hh * vn;
      }
    }
  }
  if (j == 0 && blockIdx.x == 0) atomicAdd((unsigned long long*)&d.ctrl->substeps, (unsigned long long)Mb);
  if (!active || j < H || j >= IN_WG - H) return;
  bool fin = true;
  double d2 = 0.0, b2 = 0.0;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    d.r[3 * slot + a] = r[a];
    d.v[3 * slot + a] = v[a];
    d.J[3 * slot + a] = J[a];
    fin = fin && isfinite(v[a]) && isfinite(r[a]);
    const double dd = r[a] - d.ref[3 * slot + a];
    d2 += dd * dd;
    const double db = r[a] - d.rbin[3 * slot + a];
    b2 += db * db;
  }
  if (!fin) atomicOr(&d.ctrl->err, E_BEADS);
  if (d2 > R.mp.halfskin2) d.rb[4 * rep + (o + 1) % 3] = 1u;
  if (!(b2 <= CELL_MARGIN * CELL_MARGIN)) d.cst[4 * rep + (o + 1) % 3] = 1u;
}

// ---------------------------------------------------------------------------
// Neighbour lists from the hashed cell table, once per coupled step.  Each
// bead is examined by 32 lanes, one per distinct bucket of its 27 neighbour
// cells; the lanes collect the other beads of its chain within r_c + skin,
// and one lane sorts their slots into ascending (chain) order -- the list the
// in-kernel scan would build.  A bucket that overflows leaves its replica's
// lists marked invalid (and the table unusable), so the first sub-step
// rebuilds them by the full scan: the same lists, found slower.
// ---------------------------------------------------------------------------
__global__ void k_cell_clear(int* __restrict__ ccount, int nbuckets, uint32_t* __restrict__ rb, int nrep) {
  int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < nbuckets) ccount[k] = 0;
  if (k < nrep) rb[4 * k + 3] = 0u;          // valid unless a bucket overflows below
}

__device__ inline void cell_insert_slot(const Dev& d, int slot) {
  const int rep = d.slot_rep[slot];
  const Rep& R = d.reps[rep];
  if (slot - R.slot_off >= R.mp.nb) return;
  int c[3];
  bead_cell(R, &d.r[3 * slot], c);
  const uint32_t b = cell_bucket(rep, c[0], c[1], c[2], d.cmask);
  const int pos = atomicAdd(&d.ccount[b], 1);
  if (pos < CELL_CAP) d.cbuf[(size_t)b * CELL_CAP + pos] = slot;
  // a bead left out of a full bucket is "far from its binned position", so
  // the table is not used inside the sub-cycle
#pragma unroll
  for (int a = 0; a < 3; ++a) d.rbin[3 * slot + a] = pos < CELL_CAP ? d.r[3 * slot + a] : 1e300;
}

__global__ void k_cell_insert(Dev d, int nslots) {
  int slot = blockIdx.x * blockDim.x + threadIdx.x;
  if (slot < nslots) cell_insert_slot(d, slot);
}

constexpr int LB_LANES = 32;                 // lanes per bead in the list build (27 cells)
constexpr int LB_BEADS = 2;                  // beads per 64-lane workgroup
constexpr int LB_CAND = 96;                  // candidates a bead may collect

__global__ __launch_bounds__(LB_LANES * LB_BEADS) void k_list_build(Dev d, int nslots) {
  __shared__ int cand[LB_BEADS][LB_CAND];
  __shared__ int ncand[LB_BEADS];
  __shared__ uint32_t bkt[LB_BEADS][LB_LANES];
  const int lb = threadIdx.x / LB_LANES, lane = threadIdx.x % LB_LANES;
  const int slot = blockIdx.x * LB_BEADS + lb;
  bool on = slot < nslots;
  int rep = 0, so = 0, p = 0;
  if (on) {
    rep = d.slot_rep[slot];
    so = d.reps[rep].slot_off;
    p = slot - so;
    on = p < d.reps[rep].mp.nb;
  }
  double rp[3] = {0.0, 0.0, 0.0};
  uint32_t b = 0xffffffffu;
  if (on) {
    rp[0] = d.r[3 * slot]; rp[1] = d.r[3 * slot + 1]; rp[2] = d.r[3 * slot + 2];
    if (lane < 27) {
      const Rep& R = d.reps[rep];
      int c[3];
      bead_cell(R, rp, c);
      const int dx = lane % 3 - 1, dy = (lane / 3) % 3 - 1, dz = lane / 9 - 1;
      b = cell_bucket(rep, (c[0] + dx + R.ncell[0]) % R.ncell[0], (c[1] + dy + R.ncell[1]) % R.ncell[1],
                      (c[2] + dz + R.ncell[2]) % R.ncell[2], d.cmask);
    }
  }
  bkt[lb][lane] = b;
  if (lane == 0) ncand[lb] = 0;
  __syncthreads();
  // a bucket reached from several neighbour cells (wrapped small cell counts,
  // hash collisions) is scanned by its lowest lane only: every candidate once
  bool scan = b != 0xffffffffu;
  for (int k = 0; k < lane && scan; ++k) scan = bkt[lb][k] != b;
  if (scan) {
    const Geom& g = d.reps[rep].g;
    const double rl2 = d.reps[rep].mp.rlist2;
    const int cnt = d.ccount[b];
    if (cnt > CELL_CAP) d.rb[4 * rep + 3] = 1u;   // incomplete bucket: rebuild in-kernel
    const int n = min(cnt, CELL_CAP);
    for (int k = 0; k < n; ++k) {
      const int q = d.cbuf[(size_t)b * CELL_CAP + k];
      if (d.slot_rep[q] != rep || q == slot) continue;
      double d0 = min_image(rp[0] - d.r[3 * q], g.nx);
      double d1 = min_image(rp[1] - d.r[3 * q + 1], g.ny);
      double d2 = min_image(rp[2] - d.r[3 * q + 2], g.nz);
      if (!(d0 * d0 + d1 * d1 + d2 * d2 < rl2)) continue;
      const int at = atomicAdd(&ncand[lb], 1);
      if (at < LB_CAND) cand[lb][at] = q;
    }
  }
  __syncthreads();
  if (!on || lane != 0) return;
  // ascending chain order, the MAXNBR smallest kept
  int nc = ncand[lb];
  if (nc > MAXNBR) atomicOr(&d.ctrl->err, E_NBRLIST);
  // read first: once the maximum is reached, most beads skip the atomic
  if ((uint32_t)nc > __hip_atomic_load(&d.ctrl->nbr_max, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
    atomicMax(&d.ctrl->nbr_max, (uint32_t)nc);
  if (nc > LB_CAND) nc = LB_CAND;
  int* c = cand[lb];
  for (int i = 1; i < nc; ++i) {
    const int v = c[i];
    int m = i;
    while (m > 0 && c[m - 1] > v) { c[m] = c[m - 1]; --m; }
    c[m] = v;
  }
  if (nc > MAXNBR) nc = MAXNBR;
  int* row = d.nbr + (size_t)slot * MAXNBR;
  for (int i = 0; i < nc; ++i) row[i] = c[i];
  d.ncnt[slot] = nc;
  d.ref[3 * slot] = rp[0]; d.ref[3 * slot + 1] = rp[1]; d.ref[3 * slot + 2] = rp[2];
}

// k_cell_clear with the spread-on-solid shares: k < nbuckets clears a bucket,
// k < nrep validates a replica's lists, k < nslots writes a slot's share.
__global__ void k_tail_clear(Dev d, int nbuckets, int nrep, int nslots, int ledger) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < nbuckets) d.ccount[k] = 0;
  if (k < nrep) d.rb[4 * k + 3] = 0u;
  if (ledger && k < nslots) ledger_sp_share(d, k);
}

// k_cell_insert in the first `nins` workgroups; after them one workgroup per
// replica adds its beads' shares (strided per thread, then a fixed tree)
// into its ledger.
constexpr int TAIL_WG = 1024;
__global__ __launch_bounds__(TAIL_WG) void k_tail_insert(Dev d, int nslots, int nins) {
  if ((int)blockIdx.x < nins) {                  // uniform in the workgroup
    const int slot = blockIdx.x * blockDim.x + threadIdx.x;
    if (slot < nslots) cell_insert_slot(d, slot);
    return;
  }
  __shared__ double sh[TAIL_WG];
  const int rep = blockIdx.x - nins;
  const Rep& R = d.reps[rep];
  double s[3] = {0.0, 0.0, 0.0};
  if (R.g.wall_axis >= 0)
    for (int p = threadIdx.x; p < R.mp.nb; p += TAIL_WG)
      for (int a = 0; a < 3; ++a) s[a] += d.lsp[3 * (size_t)(R.slot_off + p) + a];
  for (int a = 0; a < 3; ++a) {
    __syncthreads();
    sh[threadIdx.x] = s[a];
    __syncthreads();
    for (int w = TAIL_WG / 2; w > 0; w >>= 1) {
      if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
      __syncthreads();
    }
    if (threadIdx.x == 0) d.ledger[NLEDGER * rep + 3 + a] += sh[0];
  }
}

void launch_step_tail(const Dev& d, int nslots, int nrep, bool ledger, hipStream_t s) {
  if (nslots <= 0) return;
  const int nb = (int)d.cmask + 1;
  int n = nb > nrep ? nb : nrep;
  if (nslots > n) n = nslots;
  hipLaunchKernelGGL(k_tail_clear, dim3((n + 255) / 256), dim3(256), 0, s, d, nb, nrep, nslots, ledger ? 1 : 0);
  const int nins = (nslots + TAIL_WG - 1) / TAIL_WG;
  hipLaunchKernelGGL(k_tail_insert, dim3((unsigned)(nins + (ledger ? nrep : 0))), dim3(TAIL_WG), 0, s, d, nslots,
                     nins);
  hipLaunchKernelGGL(k_list_build, dim3((nslots + LB_BEADS - 1) / LB_BEADS), dim3(LB_LANES * LB_BEADS), 0, s, d,
                     nslots);
}

void launch_nbr_build(const Dev& d, int nslots, int nrep, hipStream_t s) {
  if (nslots <= 0) return;
  const int nb = (int)d.cmask + 1;
  const int nclr = nb > nrep ? nb : nrep;
  hipLaunchKernelGGL(k_cell_clear, dim3((nclr + 255) / 256), dim3(256), 0, s, d.ccount, nb, d.rb, nrep);
  hipLaunchKernelGGL(k_cell_insert, dim3((nslots + 255) / 256), dim3(256), 0, s, d, nslots);
  hipLaunchKernelGGL(k_list_build, dim3((nslots + LB_BEADS - 1) / LB_BEADS), dim3(LB_LANES * LB_BEADS), 0, s, d,
                     nslots);
}

void launch_md_invalidate(const Dev& d, int nrep, hipStream_t s) {
  hipLaunchKernelGGL(k_md_invalidate, dim3(1), dim3(256), 0, s, d.rb, nrep);
}

// ---------------------------------------------------------------------------
// Rigid bonds (Sec. 2, Eq. (SPValgo) with its SHAKE and RATTLE steps), one
// workgroup per chain (nb <= CON_WG).  Mode START opens the sub-cycle:
// ref = r, x = r + h/2 v (the gather's r_mid), SHAKE(x; ref), v += (x -
// x_drifted)/(h/2).  Mode STEP s follows the kick of sub-step s:
// RATTLE(v; x) at the sub-step's positions x, r = x + h/2 v, and unless it is
// the last sub-step the opening of the next: ref = r, x = r + h/2 v,
// SHAKE(x; ref), v += (x - x_drifted)/(h/2), x stored as the next r_mid.
// Both projections are tridiagonal systems in the bond multipliers: RATTLE's
// is solved once; SHAKE's linearised constraints by Newton iterations until
// the worst bond is within CON_TOL r0^2.  Each system is solved by parallel
// cyclic reduction in LDS (thread k owns bond k), or for chains of at most
// 32 beads by the Thomas algorithm on one lane; bead p adds the corrections
// of its bonds p (+) and p-1 (-) in that order.
// ---------------------------------------------------------------------------
constexpr int CON_WG = 1024;
constexpr double CON_TOL = 1e-13;
constexpr int CON_MAXIT = 50;

struct ConShared {
  double x[CON_WG][3];      // positions
  double e[CON_WG][3];      // bond vectors of the system's coefficients
  double w[CON_WG][3];      // velocities (RATTLE)
  double a[CON_WG], b[CON_WG], c[CON_WG], r[CON_WG];
  double red[CON_WG / 64];
};

// max over the workgroup (exact, any order)
__device__ inline double con_max(double x, ConShared& sh) {
  for (int o = 32; o > 0; o >>= 1) x = fmax(x, __shfl_xor(x, o, 64));
  const int wv = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) sh.red[wv] = x;
  __syncthreads();
  double m = 0.0;
  for (int k = 0; k < CON_WG / 64; ++k) m = fmax(m, sh.red[k]);
  return m;
}

// Solves a[k] y[k-1] + b[k] y[k] + c[k] y[k+1] = r[k], k < n, in place
// (parallel cyclic reduction; rows beyond the ends read as identity rows);
// returns thread k's y[k].
__device__ inline double con_pcr(ConShared& sh, int n) {
  const int k = threadIdx.x;
  for (int h = 1; h < n; h <<= 1) {
    double ai = 0.0, bi = 1.0, ci = 0.0, ri = 0.0;
    double am = 0.0, bm = 1.0, cm = 0.0, rm = 0.0, ap = 0.0, bp = 1.0, cp = 0.0, rp = 0.0;
    if (k < n) {
      ai = sh.a[k]; bi = sh.b[k]; ci = sh.c[k]; ri = sh.r[k];
      if (k - h >= 0) { am = sh.a[k - h]; bm = sh.b[k - h]; cm = sh.c[k - h]; rm = sh.r[k - h]; }
      if (k + h < n) { ap = sh.a[k + h]; bp = sh.b[k + h]; cp = sh.c[k + h]; rp = sh.r[k + h]; }
    }
    __syncthreads();
    if (k < n) {
      const double k1 = ai / bm, k2 = ci / bp;
      sh.a[k] = -(am * k1);
      sh.b[k] = bi - cm * k1 - ap * k2;
      sh.c[k] = -(cp * k2);
      sh.r[k] = ri - rm * k1 - rp * k2;
    }
    __syncthreads();
  }
  return k < n ? sh.r[k] / sh.b[k] : 0.0;
}

// The same system by the Thomas algorithm on one lane (forward elimination,
// then back substitution), for short chains: n - 1 dependent rows cost less
// than the reduction's barriers, and the result rounds as the textbook
// solve does.  Returns thread k's y[k].
constexpr int CON_THOMAS_MAX = 31;
__device__ inline double con_thomas(ConShared& sh, int n) {
  const int k = threadIdx.x;
  if (k == 0 && n > 0) {
    sh.c[0] = sh.c[0] / sh.b[0];
    sh.r[0] = sh.r[0] / sh.b[0];
    for (int i = 1; i < n; ++i) {
      const double den = sh.b[i] - sh.a[i] * sh.c[i - 1];
      sh.c[i] = sh.c[i] / den;
      sh.r[i] = (sh.r[i] - sh.a[i] * sh.r[i - 1]) / den;
    }
    for (int i = n - 2; i >= 0; --i) sh.r[i] = sh.r[i] - sh.c[i] * sh.r[i + 1];
  }
  __syncthreads();
  return k < n ? sh.r[k] : 0.0;
}
__device__ inline double con_solve(ConShared& sh, int n) {
  return n <= CON_THOMAS_MAX ? con_thomas(sh, n) : con_pcr(sh, n);   // uniform in the workgroup
}

__device__ inline double dot3v(const double* u, const double* v) { return u[0] * v[0] + u[1] * v[1] + u[2] * v[2]; }

// SHAKE of the drifted positions sh.x along the bonds held in sh.e (the
// reference bonds): the correction is accumulated in sh.w (x = x_drifted +
// dx, x itself left as drifted), so that the velocity impulse dx / (h/2)
// keeps its relative precision
__device__ inline void con_shake(ConShared& sh, int nb, double d2, uint32_t* err) {
  const int k = threadIdx.x, nbond = nb - 1;
  for (int it = 0;; ++it) {
    double sv[3] = {0.0, 0.0, 0.0}, sig = 0.0;
    if (k < nbond) {
#pragma unroll
      for (int a = 0; a < 3; ++a) sv[a] = (sh.x[k][a] + sh.w[k][a]) - (sh.x[k + 1][a] + sh.w[k + 1][a]);
      sig = dot3v(sv, sv) - d2;
    }
    const double worst = con_max(fabs(sig), sh);
    if (worst <= CON_TOL * d2) return;
    if (it == CON_MAXIT) {
      if (k == 0) atomicOr(err, E_BEADS);
      return;
    }
    if (k < nbond) {
      sh.b[k] = 4.0 * dot3v(sv, sh.e[k]);
      sh.a[k] = k > 0 ? -2.0 * dot3v(sv, sh.e[k - 1]) : 0.0;
      sh.c[k] = k < nbond - 1 ? -2.0 * dot3v(sv, sh.e[k + 1]) : 0.0;
      sh.r[k] = -sig;
    }
    __syncthreads();
    const double lam = con_solve(sh, nbond);
    // every thread has read what it needs; multipliers to sh.r, then apply
    sh.r[k] = lam;
    __syncthreads();
    if (k < nb) {
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        double y = sh.w[k][a];
        if (k < nbond) y = y + sh.r[k] * sh.e[k][a];
        if (k > 0) y = y - sh.r[k - 1] * sh.e[k - 1][a];
        sh.w[k][a] = y;                       // own entry only
      }
    }
    __syncthreads();
  }
}

__global__ __launch_bounds__(CON_WG) void k_md_constraint(Dev d, int nslots, int mode, int s, int last) {
  __shared__ ConShared sh;
  const int rep = blockIdx.x;
  const Rep& R = d.reps[rep];
  const int nb = R.mp.nb;
  if (nb < 2 || !R.mp.constrained) return;   // uniform in the workgroup
  const int k = threadIdx.x;
  const int slot = R.slot_off + k;
  const double hh = R.mp.hh, d2 = R.mp.r0 * R.mp.r0;
  const double* rin = (s & 1) ? d.rmid1 : d.rmid0;   // this sub-step's positions (STEP)
  double* rout = (s & 1) ? d.rmid0 : d.rmid1;        // the next sub-step's
  double v[3] = {0.0, 0.0, 0.0}, r[3] = {0.0, 0.0, 0.0};
  const bool own = k < nb;
  if (own) {
#pragma unroll
    for (int a = 0; a < 3; ++a) v[a] = d.v[3 * slot + a];
  }
  bool open_next = true;
  if (mode == 0) {
    // START: r is the step's start, the gather stored r_mid = r + h/2 v in rmid0
    if (own) {
#pragma unroll
      for (int a = 0; a < 3; ++a) r[a] = d.r[3 * slot + a];
    }
    rout = d.rmid0;
  } else {
    // RATTLE at the sub-step's positions
    if (own) {
#pragma unroll
      for (int a = 0; a < 3; ++a) { sh.x[k][a] = rin[3 * slot + a]; sh.w[k][a] = v[a]; }
    }
    __syncthreads();
    const int nbond = nb - 1;
    double rv[3] = {0.0, 0.0, 0.0};
    if (k < nbond) {
      double ww[3];
#pragma unroll
      for (int a = 0; a < 3; ++a) { rv[a] = sh.x[k][a] - sh.x[k + 1][a]; ww[a] = sh.w[k][a] - sh.w[k + 1][a]; }
      sh.b[k] = 2.0 * dot3v(rv, rv);
      sh.r[k] = -dot3v(rv, ww);
#pragma unroll
      for (int a = 0; a < 3; ++a) sh.e[k][a] = rv[a];
    }
    __syncthreads();
    if (k < nbond) {
      sh.a[k] = k > 0 ? -dot3v(rv, sh.e[k - 1]) : 0.0;
      sh.c[k] = k < nbond - 1 ? -dot3v(rv, sh.e[k + 1]) : 0.0;
    }
    __syncthreads();
    const double mu = con_solve(sh, nbond);
    sh.r[k] = mu;
    __syncthreads();
    if (own) {
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        if (k < nbond) v[a] = v[a] + sh.r[k] * sh.e[k][a];
        if (k > 0) v[a] = v[a] - sh.r[k - 1] * sh.e[k - 1][a];
        r[a] = sh.x[k][a] + hh * v[a];
      }
    }
    open_next = !last;
    if (last && own) {
#pragma unroll
      for (int a = 0; a < 3; ++a) { d.r[3 * slot + a] = r[a]; d.v[3 * slot + a] = v[a]; }
    }
    __syncthreads();
  }
  if (!open_next) return;
  // the opening of the next sub-step: ref = r, x = r + h/2 v, SHAKE
  double xd[3] = {0.0, 0.0, 0.0};
  if (own) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      xd[a] = r[a] + hh * v[a];
      sh.x[k][a] = xd[a];
      sh.w[k][a] = r[a];
    }
  }
  __syncthreads();
  if (k < nb - 1) {
#pragma unroll
    for (int a = 0; a < 3; ++a) sh.e[k][a] = sh.w[k][a] - sh.w[k + 1][a];
  }
  __syncthreads();
  if (own) {
#pragma unroll
    for (int a = 0; a < 3; ++a) sh.w[k][a] = 0.0;    // the SHAKE correction
  }
  __syncthreads();
  con_shake(sh, nb, d2, &d.ctrl->err);
  if (!own) return;
  double d2r = 0.0, b2 = 0.0;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const double dx = sh.w[k][a];
    const double x = xd[a] + dx;
    v[a] = v[a] + dx / hh;
    rout[3 * slot + a] = x;
    d.v[3 * slot + a] = v[a];
    const double dd = x - d.ref[3 * slot + a];
    d2r += dd * dd;
    const double db = x - d.rbin[3 * slot + a];
    b2 += db * db;
  }
  const int w = mode == 0 ? 0 : (s + 1) % 3;
  if (d2r > R.mp.halfskin2) d.rb[4 * rep + w] = 1u;
  if (!(b2 <= CELL_MARGIN * CELL_MARGIN)) d.cst[4 * rep + w] = 1u;
}

void launch_md_begin(const Dev& d, int nrep, hipStream_t s) {
  hipLaunchKernelGGL(k_md_begin, dim3(1), dim3(256), 0, s, d.rb, d.cst, nrep, d.redo);
}

void launch_md_cycle(const Dev& d, int nslots, int nrep, int n_sub, const MdOverride& ov, hipStream_t s,
                     bool prologue, bool constrained) {
  if (nslots <= 0 || n_sub <= 0) return;
  unsigned nblk = (unsigned)(nslots / MD_BPB);
  if (prologue) {
    hipLaunchKernelGGL(k_md_begin, dim3(1), dim3(256), 0, s, d.rb, d.cst, nrep, d.redo);
    hipLaunchKernelGGL(k_md_start, dim3((nslots + 255) / 256), dim3(256), 0, s, d, nslots, ov, 0);
  }
  if (constrained)
    hipLaunchKernelGGL(k_md_constraint, dim3((unsigned)nrep), dim3(CON_WG), 0, s, d, nslots, 0, 0, 0);
  for (int k = 0; k < n_sub; ++k) {
    hipLaunchKernelGGL(k_md_substep<false>, dim3(nblk), dim3(3 * MD_WG), 0, s, d, ov, nslots, k,
                       k == n_sub - 1 ? 1 : 0);
    if (constrained)
      hipLaunchKernelGGL(k_md_constraint, dim3((unsigned)nrep), dim3(CON_WG), 0, s, d, nslots, 1, k,
                         k == n_sub - 1 ? 1 : 0);
  }
}

void launch_md_cycle_mts(const Dev& d, int nslots, int nrep, int n_sub, int M, hipStream_t s, bool prologue) {
  if (nslots <= 0 || n_sub <= 0 || M <= 0) return;
  const int Mb = n_sub / M;
  const unsigned nblk = (unsigned)(nslots / MD_BPB);
  const int own = IN_WG - 4 * Mb;
  const unsigned nin = (unsigned)((nslots + own - 1) / own);
  MdOverride none{};
  if (prologue) {
    hipLaunchKernelGGL(k_md_begin, dim3(1), dim3(256), 0, s, d.rb, d.cst, nrep, d.redo);
    hipLaunchKernelGGL(k_md_start, dim3((nslots + 255) / 256), dim3(256), 0, s, d, nslots, none, 1);
  }
  for (int o = 0; o < M; ++o) {
    hipLaunchKernelGGL(k_md_substep<true>, dim3(nblk), dim3(3 * MD_WG), 0, s, d, none, nslots, o, o == 0 ? 1 : 2);
    hipLaunchKernelGGL(k_md_inner, dim3(nin), dim3(IN_WG), 0, s, d, nslots, o, Mb);
  }
  hipLaunchKernelGGL(k_md_substep<true>, dim3(nblk), dim3(3 * MD_WG), 0, s, d, none, nslots, M, 1);
}

// ---------------------------------------------------------------------------
// Fused sub-steps: one launch advances a block of K uniform sub-steps.
//
// Workgroup w owns the chain segment [a, b) of replica rep.  Over one
// sub-step a bead's new state depends on its own state and on the positions
// of its chain neighbours p-2 .. p+2 (bonds, and the angles centred at p-1,
// p, p+1) and of its pair partners within r_c.  Give every bead its level:
// its distance from [a, b) in that dependency graph.  A bead of level k must
// be exact for the first K - k sub-steps of the block, which needs its
// dependencies (level <= k + 1) exact for one sub-step less, so the set S of
// beads of level <= K, each advanced from the positions in S, leaves [a, b)
// exact after K sub-steps even though the beads at S's rim go wrong (the halo
// argument of overlapped tiling).  S is a union of chain spans: [a, b)
// widened by 2K (level 0 inside, +1 per two chain links), and for every
// close partner j of a bead of level k < K that is not yet in S with level
// <= k + 1, a span around j of level k + 1, widened by 2 (K - k - 1).
//
// Pair partners are the entries of the neighbour lists (built at the start
// of the LB step, radius r_c + skin) within close = r_c + 2 FUSED_DELTA at
// the block's start.  Partners farther than that stay beyond r_c for the
// whole block as long as no bead moves more than FUSED_DELTA within it, so
// they contribute nothing; and a list holds every bead within close of its
// bead as long as every bead is within skin/2 - FUSED_DELTA of where the
// lists were built.  Both conditions are checked, each workgroup on the
// beads it owns: if every workgroup of the replica finds them true, no bead
// of the replica violated them and the block equals the per-sub-step
// computation bit for bit (the same operations in the same order: bonds, the
// three angles, pair partners in ascending order, wall sites in ascending
// order, field, then the kick; only pairs within r_c ever add a term, so the
// list a partner came from does not matter).  Otherwise the replica's redo
// marker is set to the block's first sub-step, later blocks of the replica
// return at once, and k_md_redo redoes the replica from there in one
// workgroup.  A block reads its start state from one set of arrays (the
// canonical r_mid0, v, J, or the shadow ones) and writes the other, so that
// the start state of a block that fails is still there.
// ---------------------------------------------------------------------------
constexpr int FU_LANES = 4;        // lanes per bead in the sub-steps
constexpr int FU_CAP = 128;        // beads of S
constexpr int FU_WG = FU_LANES * FU_CAP;
constexpr int FU_NS = 16;          // spans of S (before merging)
constexpr int FU_NC = 16;          // close partners per bead
constexpr int FU_ROUNDS = 6;       // closure rounds
constexpr int FU_LD = 16;          // list entries loaded together

struct FuSpan {
  int blo, bhi;                    // base interval (level lv inside)
  int lv;
};

struct FuShared {
  double pos[2][FU_CAP][3];        // positions at the sub-step's start / the next one
  double ang[FU_CAP][9];           // forces of the angle centred at the bead (first, centre, third)
  double bnd[FU_CAP][6];           // the bead's bond forces towards its predecessor and successor
  int lst[FU_CAP][FU_NC];          // close partners: chain indices, then local indices; ascending
  unsigned char lcnt[FU_CAP];
  unsigned char lev[FU_CAP];       // level of the bead (K + 1: not needed)
  unsigned char angok[FU_CAP];     // the angle centred at the bead is evaluated
  FuSpan span[FU_NS];
  int nspan;
  int ilo[FU_NS], ihi[FU_NS], ioff[FU_NS + 1];   // S as sorted disjoint chain intervals
  int niv;
  int nreq;
  FuSpan req[FU_NS];
  int ctl;                         // set-up state, written by thread 0 only, between barriers:
                                   // 0 go on, 1 closure complete, 2 cannot certify, 3 an earlier block failed
  int ovf;                         // a request or a partner list did not fit
  int far;                         // a bead of the segment moved too far from where the lists were built
};

// chain index of local index li, and local index of chain index q (-1 if
// not in S); S is the concatenation of the sorted disjoint intervals
__device__ inline int fu_chain(const FuShared& sh, int li) {
  for (int k = 0; k < sh.niv; ++k)
    if (li < sh.ioff[k + 1]) return sh.ilo[k] + (li - sh.ioff[k]);
  return -1;
}
__device__ inline int fu_local(const FuShared& sh, int q) {
  for (int k = 0; k < sh.niv; ++k)
    if (q >= sh.ilo[k] && q < sh.ihi[k]) return sh.ioff[k] + (q - sh.ilo[k]);
  return -1;
}
// level of chain bead q: the least over the spans of lv + ceil(distance to
// the span's base / 2), K + 1 when above K (then not in S)
__device__ inline int fu_level(const FuShared& sh, int q, int K) {
  int best = K + 1;
  for (int k = 0; k < sh.nspan; ++k) {
    const FuSpan& p = sh.span[k];
    const int dist = q < p.blo ? p.blo - q : (q >= p.bhi ? q - p.bhi + 1 : 0);
    const int l = p.lv + (dist + 1) / 2;
    best = l < best ? l : best;
  }
  return best;
}
// S from the spans (one thread): every bead of level <= K, as sorted
// disjoint chain intervals.  False when S exceeds its capacity.
__device__ inline bool fu_build(FuShared& sh, int K, int nb) {
  int lo[FU_NS], hi[FU_NS];
  const int n = sh.nspan;
  for (int k = 0; k < n; ++k) {
    const int w = 2 * (K - sh.span[k].lv);
    lo[k] = max(0, sh.span[k].blo - w);
    hi[k] = min(nb, sh.span[k].bhi + w);
  }
  for (int i = 1; i < n; ++i) {
    const int l = lo[i], h = hi[i];
    int m = i;
    while (m > 0 && lo[m - 1] > l) { lo[m] = lo[m - 1]; hi[m] = hi[m - 1]; --m; }
    lo[m] = l; hi[m] = h;
  }
  int k = 0;
  for (int i = 1; i < n; ++i) {
    if (lo[i] <= hi[k]) { hi[k] = max(hi[k], hi[i]); continue; }
    ++k;
    lo[k] = lo[i]; hi[k] = hi[i];
  }
  const int niv = k + 1;
  int tot = 0;
  for (int i = 0; i < niv; ++i) tot += hi[i] - lo[i];
  if (tot > FU_CAP) return false;
  sh.niv = niv;
  sh.ioff[0] = 0;
  for (int i = 0; i < niv; ++i) { sh.ilo[i] = lo[i]; sh.ihi[i] = hi[i]; sh.ioff[i + 1] = sh.ioff[i] + hi[i] - lo[i]; }
  return true;
}

// The beads of the replica within sqrt(r2max) of position x (any bead but
// chain index self), from the neighbour-search cell table, in ascending
// chain order: at most cap of them into out (returns their number, cap + 1
// if more).  Every bead within range is found while every bead of the
// replica lies within CELL_MARGIN of the position the table binned it at
// and sqrt(r2max) + CELL_MARGIN does not exceed the cell side.
__device__ inline int cell_partners(const Dev& d, const Rep& R, int rep, const double* pos, int self,
                                    const double* x, double r2max, int* out, int cap) {
  const Geom& g = R.g;
  const int so = R.slot_off;
  int c[3];
  bead_cell(R, x, c);
  int n = 0;
  for (int k = 0; k < 27; ++k) {
    const int dx = k % 3 - 1, dy = (k / 3) % 3 - 1, dz = k / 9 - 1;
    const uint32_t b = cell_bucket(rep, (c[0] + dx + R.ncell[0]) % R.ncell[0], (c[1] + dy + R.ncell[1]) % R.ncell[1],
                                   (c[2] + dz + R.ncell[2]) % R.ncell[2], d.cmask);
    const int m = min(d.ccount[b], CELL_CAP);
    for (int e = 0; e < m; ++e) {
      const int sl = d.cbuf[(size_t)b * CELL_CAP + e];
      if (d.slot_rep[sl] != rep) continue;
      const int j = sl - so;
      if (j == self) continue;
      const double e0 = min_image(x[0] - pos[3 * sl], g.nx);
      const double e1 = min_image(x[1] - pos[3 * sl + 1], g.ny);
      const double e2 = min_image(x[2] - pos[3 * sl + 2], g.nz);
      if (!(e0 * e0 + e1 * e1 + e2 * e2 < r2max)) continue;
      // a bucket reached from two of the 27 cells (few cells per axis, or
      // hash collisions) gives its beads twice: keep each once
      int i = n;
      while (i > 0 && out[i - 1] > j) --i;
      if (i > 0 && out[i - 1] == j) continue;
      if (n == cap) return cap + 1;
      for (int m2 = n; m2 > i; --m2) out[m2] = out[m2 - 1];
      out[i] = j;
      ++n;
    }
  }
  return n;
}

// The wall sites' forces on a bead at rp, added to F in ascending site order
// (rows o1, then o0): the sites and operations of wall_row, summed as the
// sub-step kernel sums them.
__device__ inline void fu_wall(const MdParams& P, const Geom& g, const double* rp, double F[3]) {
  if (g.wall_axis < 0) return;
  const double w0 = wrapc(rp[0], g.nx), w1 = wrapc(rp[1], g.ny), w2 = wrapc(rp[2], g.nz);
  const int b0 = (int)floor(w0), b1 = (int)floor(w1), b2 = (int)floor(w2);
  const int a = g.wall_axis;
  const int ba = a == 0 ? b0 : (a == 1 ? b1 : b2);
  const int na = a == 0 ? g.nx : (a == 1 ? g.ny : g.nz);
  const int bt0 = a == 0 ? b1 : b0, n0 = a == 0 ? g.ny : g.nx;
  const int bt1 = a == 2 ? b1 : b2, n1 = a == 2 ? g.ny : g.nz;
  int off = g.wall_pos - ba;
  if (off < WLO) off += na;
  if (off > WHI) off -= na;
  if (off < P.wlo || off > P.whi) return;
  const int sa = ba + off;
  for (int o1 = P.wlo; o1 <= P.whi; ++o1) {
    const int u1 = bt1 + o1;
    const int v1 = u1 < 0 ? u1 + n1 : (u1 >= n1 ? u1 - n1 : u1);
    const bool in1 = v1 >= g.lo1 && v1 <= g.hi1;
    for (int o0 = P.wlo; o0 <= P.whi; ++o0) {
      const int u0 = bt0 + o0;
      const int v0 = u0 < 0 ? u0 + n0 : (u0 >= n0 ? u0 - n0 : u0);
      const bool in0 = v0 >= g.lo0 && v0 <= g.hi0;
      if (in0 && in1) continue;
      const int sx = a == 0 ? sa : u0;
      const int sy = a == 1 ? sa : (a == 0 ? u0 : u1);
      const int sz = a == 2 ? sa : u1;
      const double d0 = w0 - (double)sx, d1 = w1 - (double)sy, d2 = w2 - (double)sz;
      if (!(d0 * d0 + d1 * d1 + d2 * d2 < P.rc2)) continue;
      double Fs[3] = {0.0, 0.0, 0.0};
      lj_add(P, d0, d1, d2, Fs);
      F[0] += Fs[0]; F[1] += Fs[1]; F[2] += Fs[2];
    }
  }
}

// The force on chain bead q at rp in the order of the sub-step kernel: bonds
// to q-1 (at rm) and q+1 (at rq), the angles centred at q-1 (third-bead
// part a3), q (centre part ac) and q+1 (first-bead part a1) -- each NULL when
// not added --, the pair partners at base + 3 idx[0..np-1] in ascending
// chain order (terms within r_c only), the wall sites, the field.
__device__ inline void fu_force(const MdParams& P, const Geom& g, int q, const double* rp, const double* rm,
                                const double* rq, const double* a3, const double* ac, const double* a1,
                                const double* base, const int* idx, int np, double F[3]) {
  F[0] = 0.0; F[1] = 0.0; F[2] = 0.0;
  if (!P.constrained) {
    if (q > 0 && rm) bond_add(P, rp, rm, F);
    if (q < P.nb - 1 && rq) bond_add(P, rp, rq, F);
  }
  if (a3) { F[0] += a3[6]; F[1] += a3[7]; F[2] += a3[8]; }
  if (ac) { F[0] += ac[3]; F[1] += ac[4]; F[2] += ac[5]; }
  if (a1) { F[0] += a1[0]; F[1] += a1[1]; F[2] += a1[2]; }
  for (int k = 0; k < np; ++k) {
    const double* qp = base + 3 * (size_t)idx[k];
    const double e0 = min_image(rp[0] - qp[0], g.nx);
    const double e1 = min_image(rp[1] - qp[1], g.ny);
    const double e2 = min_image(rp[2] - qp[2], g.nz);
    if (!(e0 * e0 + e1 * e1 + e2 * e2 < P.rc2)) continue;
    double Fp[3] = {0.0, 0.0, 0.0};
    lj_add(P, e0, e1, e2, Fp);
    F[0] += Fp[0]; F[1] += Fp[1]; F[2] += Fp[2];
  }
  fu_wall(P, g, rp, F);
  if (P.field_on && in_field(g, rp)) F[g.wall_axis] += P.f_drive;
}

// All nine force components of the angle at (ra, rb, rc) into o (first,
// centre, third bead, each x, y, z), 0 for a straight or folded angle.
__device__ inline void fu_angle(const MdParams& P, const double* ra, const double* rb, const double* rc, double* o) {
  AngleCore A;
  if (angle_core(P, ra, rb, rc, A)) {
    for (int a = 0; a < 3; ++a) {
      double f[3];
      angle_part(A, a, f);
      o[a] = f[0]; o[3 + a] = f[1]; o[6 + a] = f[2];
    }
  } else {
    for (int k = 0; k < 9; ++k) o[k] = 0.0;
  }
}

// The SPV kick and drifts of one sub-step (as the sub-step kernel): v, J
// updated; returns r_mid of the next sub-step in x (or, when last, the end
// position).
__device__ inline bool fu_kick(const MdParams& P, const double F[3], const double* u, const double* xi, double* v,
                               double* J, const double* rp, bool last, double x[3]) {
  bool fin = true;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const double uu = P.couple ? u[a] : 0.0;
    const double xx = P.sig != 0.0 ? xi[a] : 0.0;
    const double sx = P.sig * xx;
    const double vn = P.e * v[a] + P.cf * (F[a] + P.gamma * uu) + sx;
    J[a] = J[a] - P.m * (P.omE * (uu - v[a]) + sx);
    v[a] = vn;
    fin = fin && isfinite(vn);
    const double re = rp[a] + P.hh * vn;
    x[a] = last ? re : re + P.hh * vn;
  }
  return fin;
}

__device__ inline void fu_fail(const Dev& d, const FusedBufs& fb, int rep, int s0) {
  if (atomicCAS(&fb.redo[rep], -1, s0) == -1) atomicAdd((unsigned long long*)&d.ctrl->fused_redos, 1ull);
}

// Block j = s0 / K of the sub-cycle.  iset: the set holding the block's start
// state (0: r_mid0, v, J; 1: the shadow arrays); the other receives the end
// state (the last block writes the final positions to r).
__global__ __launch_bounds__(FU_WG) void k_md_fused(Dev d, FusedBufs fb, int nslots, int s0, int K, int last,
                                                    int iset) {
  __shared__ FuShared sh;
  const FusedSeg seg = fb.seg[blockIdx.x];
  const int rep = seg.rep;
  const Rep& R = d.reps[rep];
  const MdParams P = R.mp;
  const Geom g = R.g;
  const int so = R.slot_off, nb = P.nb;
  const int t = threadIdx.x;
  const double* rin = iset ? fb.rmS : d.rmid0;
  const double* vin = iset ? fb.vS : d.v;
  const double* Jin = iset ? fb.JS : d.J;
  double* rout = iset ? d.rmid0 : fb.rmS;
  double* vout = iset ? d.v : fb.vS;
  double* Jout = iset ? d.J : fb.JS;
  const double close = sqrt(P.rc2) + 2.0 * FUSED_DELTA + 1e-9;
  const double close2 = close * close;
  if (t == 0) {
    // an earlier block of the replica failed (another workgroup may set the
    // marker during this launch: thread 0 reads it once for the workgroup)
    sh.ctl = fb.redo[rep] >= 0 ? 3 : (d.rb[4 * rep] != 0u ? 2 : 0);   // lists not valid at the cycle's start
    if (sh.ctl == 2) atomicAdd(&d.ctrl->fused_why[0], 1u);
    sh.ovf = 0;
    sh.far = 0;
    sh.nspan = 1;
    sh.span[0] = FuSpan{seg.a, seg.b, 0};
    sh.nreq = 0;
    if (!fu_build(sh, K, nb)) sh.ctl = 2;
  }
  __syncthreads();
  if (sh.ctl == 3) return;                        // uniform
  // the lists must hold every close partner: each workgroup checks its own beads
  const double keep = sqrt(P.halfskin2) - FUSED_DELTA;
  bool held = keep > 0.0;
  for (int q = seg.a + t; q < seg.b; q += FU_WG) {
    const int sl = so + q;
    double b2 = 0.0;
#pragma unroll
    for (int a = 0; a < 3; ++a) { const double db = rin[3 * sl + a] - d.ref[3 * sl + a]; b2 += db * db; }
    held = held && b2 <= keep * keep;
  }
  if (!held) sh.far = 1;
  // ---- closure.  Every thread reads sh.ctl right after a barrier; thread
  // 0 writes it only between the two barriers of a round.
  for (int round = 0;; ++round) {
    __syncthreads();
    if (sh.ctl != 0) break;
    const int n = sh.ioff[sh.niv];
    if (t < n) {
      const int q = fu_chain(sh, t);
      const int lv = fu_level(sh, q, K);
      sh.lev[t] = (unsigned char)lv;
      sh.lcnt[t] = 0;
      if (lv < K) {
        // the list and the positions of its first entries, loads issued
        // together; entries beyond FU_LD in a slower loop
        const int sl = so + q;
        const double x[3] = {rin[3 * sl], rin[3 * sl + 1], rin[3 * sl + 2]};
        const int cnt = d.ncnt[sl];
        const int* row = d.nbr + (size_t)sl * MAXNBR;
        int e[FU_LD];
#pragma unroll
        for (int k = 0; k < FU_LD; ++k) e[k] = row[k];
        double pj[FU_LD][3];
#pragma unroll
        for (int k = 0; k < FU_LD; ++k) {
          const int js = k < cnt ? e[k] : sl;    // list entries are slots
          pj[k][0] = rin[3 * js]; pj[k][1] = rin[3 * js + 1]; pj[k][2] = rin[3 * js + 2];
        }
        int c = 0;
        bool full = false;
        // one entry: keep it if close; request a span if it needs a lower level
        auto take = [&](int j, const double* y) {
          const double e0 = min_image(x[0] - y[0], g.nx);
          const double e1 = min_image(x[1] - y[1], g.ny);
          const double e2 = min_image(x[2] - y[2], g.nz);
          if (!(e0 * e0 + e1 * e1 + e2 * e2 < close2)) return;
          if (c == FU_NC) { full = true; return; }
          sh.lst[t][c++] = j;
          if (fu_level(sh, j, K) <= lv + 1) return;
          const int at = atomicAdd(&sh.nreq, 1);
          if (at < FU_NS) sh.req[at] = FuSpan{j, j + 1, lv + 1};
          else sh.ovf = 1;
        };
#pragma unroll
        for (int k = 0; k < FU_LD; ++k)
          if (k < cnt) take(e[k] - so, pj[k]);
        for (int k = FU_LD; k < cnt; ++k) {
          const int js = row[k];
          const double y[3] = {rin[3 * js], rin[3 * js + 1], rin[3 * js + 2]};
          take(js - so, y);
        }
        if (full) sh.ovf = 1;
        sh.lcnt[t] = (unsigned char)c;
      }
    }
    __syncthreads();
    if (t == 0) {
      int c = 0, why = -1;
      if (sh.far) { c = 2; why = 0; }
      else if (sh.ovf) { c = 2; why = 1; }
      else if (sh.nreq == 0) c = 1;
      else if (sh.nspan + sh.nreq > FU_NS) { c = 2; why = 2; }
      else {
        for (int k = 0; k < sh.nreq; ++k) sh.span[sh.nspan + k] = sh.req[k];
        sh.nspan += sh.nreq;
        if (!fu_build(sh, K, nb)) { c = 2; why = 2; }
        else if (round + 1 == FU_ROUNDS) { c = 2; why = 3; }   // the closure did not settle
      }
      if (why >= 0) atomicAdd(&d.ctrl->fused_why[why], 1u);
      sh.ctl = c;
      sh.nreq = 0;
    }
  }
  if (sh.ctl != 1) {                              // uniform: read after the barrier
    if (t == 0) fu_fail(d, fb, rep, s0);
    return;
  }
  const int n = sh.ioff[sh.niv];
  // ---- sub-steps: FU_LANES lanes per bead b of S.  Lanes 0-2 evaluate
  // component l of the angle centred at the bead, lane 3 its two bond forces;
  // lane 0 (the lead) then adds every contribution in the order of the
  // sub-step kernel, kicks and drifts the bead.
  const int b = t / FU_LANES, l = t % FU_LANES;
  const bool act = b < n;
  const bool lead = act && l == 0;
  const int q = act ? fu_chain(sh, b) : 0;
  const int slot = so + q;
  const bool own = lead && q >= seg.a && q < seg.b;
  const int lm1 = act && q > 0 ? fu_local(sh, q - 1) : -1;
  const int lp1 = act && q < nb - 1 ? fu_local(sh, q + 1) : -1;
  const bool angle_here = act && q >= 1 && q <= nb - 2 && lm1 >= 0 && lp1 >= 0;
  double rp[3] = {0.0, 0.0, 0.0}, rm0[3] = {0.0, 0.0, 0.0}, vo[3] = {0.0, 0.0, 0.0}, Jo[3] = {0.0, 0.0, 0.0};
  double ul[3] = {0.0, 0.0, 0.0};
  int lc = 0;
  if (lead) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      rp[a] = rin[3 * slot + a];
      rm0[a] = rp[a];
      vo[a] = vin[3 * slot + a];
      Jo[a] = Jin[3 * slot + a];
      ul[a] = P.couple ? d.up[3 * slot + a] : 0.0;
      sh.pos[0][b][a] = rp[a];
    }
    sh.angok[b] = angle_here ? 1 : 0;
    // partners to local indices (a bead of level < K has every close
    // partner in S by the closure; one that did not would be left out rather
    // than read outside S; a bead of level K needs none)
    const int c0 = sh.lev[b] < K ? sh.lcnt[b] : 0;
    for (int k = 0; k < c0; ++k) {
      const int lj = fu_local(sh, sh.lst[b][k]);
      if (lj >= 0) sh.lst[b][lc++] = lj;
    }
  }
  bool viol = false, fin = true;
  double rfin[3] = {0.0, 0.0, 0.0};
  double xn[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) xn[a] = lead && P.sig != 0.0 ? d.xi[(size_t)3 * ((size_t)s0 * nslots + slot) + a] : 0.0;
  __syncthreads();
  for (int s = s0; s < s0 + K; ++s) {
    const int cb = (s - s0) & 1;
    double xl[3] = {xn[0], xn[1], xn[2]};
    if (lead && P.sig != 0.0 && s + 1 < s0 + K) {
#pragma unroll
      for (int a = 0; a < 3; ++a) xn[a] = d.xi[(size_t)3 * ((size_t)(s + 1) * nslots + slot) + a];
    }
    // ---- phase 1: angle components, bonds
    if (act) {
      if (l < 3) {
        if (angle_here) {
          double f[3];
          angle_component(P, sh.pos[cb][lm1], sh.pos[cb][b], sh.pos[cb][lp1], l, f);
          sh.ang[b][l] = f[0]; sh.ang[b][3 + l] = f[1]; sh.ang[b][6 + l] = f[2];
        }
      } else {
        double F1[3] = {0.0, 0.0, 0.0}, F2[3] = {0.0, 0.0, 0.0};
        if (!P.constrained) {
          if (q > 0 && lm1 >= 0) bond_add(P, sh.pos[cb][b], sh.pos[cb][lm1], F1);
          if (q < nb - 1 && lp1 >= 0) bond_add(P, sh.pos[cb][b], sh.pos[cb][lp1], F2);
        }
        for (int a = 0; a < 3; ++a) { sh.bnd[b][a] = F1[a]; sh.bnd[b][3 + a] = F2[a]; }
      }
    }
    __syncthreads();
    // ---- phase 2: the lead adds, kicks and drifts
    if (lead) {
      double F[3] = {0.0, 0.0, 0.0};
      if (!P.constrained) {
        if (q > 0 && lm1 >= 0) { F[0] += sh.bnd[b][0]; F[1] += sh.bnd[b][1]; F[2] += sh.bnd[b][2]; }
        if (q < nb - 1 && lp1 >= 0) { F[0] += sh.bnd[b][3]; F[1] += sh.bnd[b][4]; F[2] += sh.bnd[b][5]; }
      }
      if (q - 1 >= 1 && q - 1 <= nb - 2 && lm1 >= 0 && sh.angok[lm1]) {
        const double* A = sh.ang[lm1]; F[0] += A[6]; F[1] += A[7]; F[2] += A[8];
      }
      if (angle_here) { const double* A = sh.ang[b]; F[0] += A[3]; F[1] += A[4]; F[2] += A[5]; }
      if (q + 1 >= 1 && q + 1 <= nb - 2 && lp1 >= 0 && sh.angok[lp1]) {
        const double* A = sh.ang[lp1]; F[0] += A[0]; F[1] += A[1]; F[2] += A[2];
      }
      for (int k = 0; k < lc; ++k) {
        const double* qp = sh.pos[cb][sh.lst[b][k]];
        const double e0 = min_image(rp[0] - qp[0], g.nx);
        const double e1 = min_image(rp[1] - qp[1], g.ny);
        const double e2 = min_image(rp[2] - qp[2], g.nz);
        if (!(e0 * e0 + e1 * e1 + e2 * e2 < P.rc2)) continue;
        double Fp[3] = {0.0, 0.0, 0.0};
        lj_add(P, e0, e1, e2, Fp);
        F[0] += Fp[0]; F[1] += Fp[1]; F[2] += Fp[2];
      }
      fu_wall(P, g, rp, F);
      if (P.field_on && in_field(g, rp)) F[g.wall_axis] += P.f_drive;
      const bool fl = last && s == s0 + K - 1;
      double x[3];
      fin = fu_kick(P, F, ul, xl, vo, Jo, rp, fl, x) && fin;
      if (fl) {
#pragma unroll
        for (int a = 0; a < 3; ++a) rfin[a] = x[a];
      } else {
        double dd2 = 0.0;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
          rp[a] = x[a];
          sh.pos[cb ^ 1][b][a] = x[a];
          const double dm = x[a] - rm0[a];
          dd2 += dm * dm;
        }
        // the positions of the block's next sub-steps stay within the bound
        if (own && s + 1 < s0 + K && !(dd2 <= FUSED_DELTA * FUSED_DELTA)) viol = true;
      }
    }
    __syncthreads();
  }
  if (own && !fin) atomicOr(&d.ctrl->err, E_BEADS);
  if (__syncthreads_or(viol ? 1 : 0)) {
    if (t == 0) {
      atomicAdd(&d.ctrl->fused_why[4], 1u);
      fu_fail(d, fb, rep, s0);
    }
    return;
  }
  if (blockIdx.x == 0 && t == 0) atomicAdd((unsigned long long*)&d.ctrl->fused_blocks, 1ull);
  if (!own) return;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    vout[3 * slot + a] = vo[a];
    Jout[3 * slot + a] = Jo[a];
    if (last) d.r[3 * slot + a] = rfin[a];
    else rout[3 * slot + a] = rp[a];
  }
}

// After the fused blocks, one workgroup per replica.  A replica whose block
// failed at sub-step sp is redone from that block's start state to the end
// of the cycle, sub-step by sub-step, with barriers: the angles of every
// centre, then every bead's force, kick and drifts; the positions alternate
// between r_mid0 and r_mid1.  A bead's pair partners within r_c, in
// ascending order, come from the step's neighbour lists while every bead
// lies within half the skin of where they were built, else from the cell
// table while every bead lies within CELL_MARGIN of where it was binned,
// else from all beads of the chain.  A replica whose last block wrote the
// shadow set gets v and J copied back.
constexpr int RD_WG = 1024;
constexpr int RD_NC = 32;          // pair partners within r_c of one bead

__global__ __launch_bounds__(RD_WG) void k_md_redo(Dev d, FusedBufs fb, double* ang, int nslots, int n_sub, int K) {
  __shared__ int any_far, any_off;
  const int rep = blockIdx.x;
  const Rep& R = d.reps[rep];
  const MdParams P = R.mp;
  const Geom g = R.g;
  const int so = R.slot_off, nb = P.nb;
  const int t = threadIdx.x;
  const int sp = fb.redo[rep];                    // constant during this launch
  const int M = n_sub / K;
  if (sp < 0) {
    if (M & 1)
      for (int q = t; q < nb; q += RD_WG)
        for (int a = 0; a < 3; ++a) {
          d.v[3 * (so + q) + a] = fb.vS[3 * (so + q) + a];
          d.J[3 * (so + q) + a] = fb.JS[3 * (so + q) + a];
        }
    return;
  }
  // the failed block's start state into r_mid0, v, J
  if ((sp / K) & 1)
    for (int q = t; q < nb; q += RD_WG)
      for (int a = 0; a < 3; ++a) {
        const int i = 3 * (so + q) + a;
        d.rmid0[i] = fb.rmS[i];
        d.v[i] = fb.vS[i];
        d.J[i] = fb.JS[i];
      }
  if (t == 0) atomicAdd((unsigned long long*)&d.ctrl->substeps, (unsigned long long)(n_sub - sp));
  bool fin = true, over = false;
  for (int s = sp; s < n_sub; ++s) {
    const double* cur = ((s - sp) & 1) ? d.rmid1 : d.rmid0;
    double* nxt = ((s - sp) & 1) ? d.rmid0 : d.rmid1;
    // every bead near the position the lists were built at, the position
    // the table binned it at?
    bool near = true, held = d.rb[4 * rep] == 0u;
    for (int q = t; q < nb; q += RD_WG) {
      double b2 = 0.0, f2 = 0.0;
      for (int a = 0; a < 3; ++a) {
        const double x = cur[3 * (so + q) + a];
        const double db = x - d.rbin[3 * (so + q) + a], df = x - d.ref[3 * (so + q) + a];
        b2 += db * db;
        f2 += df * df;
      }
      near = near && b2 <= CELL_MARGIN * CELL_MARGIN;
      held = held && f2 <= P.halfskin2;
    }
    if (t == 0) { any_far = 0; any_off = 0; }
    __syncthreads();                              // also orders the previous sub-step's writes
    if (!near) any_far = 1;
    if (!held) any_off = 1;
    for (int q = t; q < nb; q += RD_WG)
      if (q >= 1 && q <= nb - 2)
        fu_angle(P, &cur[3 * (so + q - 1)], &cur[3 * (so + q)], &cur[3 * (so + q + 1)], &ang[9 * (size_t)(so + q)]);
    __syncthreads();
    const bool lists = any_off == 0, table = any_far == 0;
    for (int q = t; q < nb; q += RD_WG) {
      const int sl = so + q;
      const double rp[3] = {cur[3 * sl], cur[3 * sl + 1], cur[3 * sl + 2]};
      int part[RD_NC];
      int np = 0;
      if (lists) {
        const int cnt = d.ncnt[sl];
        for (int k = 0; k < cnt && np <= RD_NC; ++k) {
          const int j = d.nbr[(size_t)sl * MAXNBR + k] - so;   // list entries are slots
          const double e0 = min_image(rp[0] - cur[3 * (so + j)], g.nx);
          const double e1 = min_image(rp[1] - cur[3 * (so + j) + 1], g.ny);
          const double e2 = min_image(rp[2] - cur[3 * (so + j) + 2], g.nz);
          if (!(e0 * e0 + e1 * e1 + e2 * e2 < P.rc2)) continue;
          if (np < RD_NC) part[np] = j;
          ++np;
        }
      } else if (table) {
        np = cell_partners(d, R, rep, cur, q, rp, P.rc2, part, RD_NC);
      } else {
        for (int j = 0; j < nb && np <= RD_NC; ++j) {
          if (j == q) continue;
          const double e0 = min_image(rp[0] - cur[3 * (so + j)], g.nx);
          const double e1 = min_image(rp[1] - cur[3 * (so + j) + 1], g.ny);
          const double e2 = min_image(rp[2] - cur[3 * (so + j) + 2], g.nz);
          if (!(e0 * e0 + e1 * e1 + e2 * e2 < P.rc2)) continue;
          if (np < RD_NC) part[np] = j;
          ++np;
        }
      }
      if (np > RD_NC) { over = true; np = RD_NC; }
      const double* a3 = (q - 1 >= 1 && q - 1 <= nb - 2) ? &ang[9 * (size_t)(sl - 1)] : nullptr;
      const double* ac = (q >= 1 && q <= nb - 2) ? &ang[9 * (size_t)sl] : nullptr;
      const double* a1 = (q + 1 >= 1 && q + 1 <= nb - 2) ? &ang[9 * (size_t)(sl + 1)] : nullptr;
      double F[3];
      fu_force(P, g, q, rp, q > 0 ? &cur[3 * (sl - 1)] : nullptr, q < nb - 1 ? &cur[3 * (sl + 1)] : nullptr, a3, ac,
               a1, cur + 3 * (size_t)so, part, np, F);
      double v[3] = {d.v[3 * sl], d.v[3 * sl + 1], d.v[3 * sl + 2]};
      double J[3] = {d.J[3 * sl], d.J[3 * sl + 1], d.J[3 * sl + 2]};
      double u[3] = {d.up[3 * sl], d.up[3 * sl + 1], d.up[3 * sl + 2]};
      double xi[3] = {0.0, 0.0, 0.0};
      if (P.sig != 0.0)
        for (int a = 0; a < 3; ++a) xi[a] = d.xi[(size_t)3 * ((size_t)s * nslots + sl) + a];
      const bool fl = s == n_sub - 1;
      double x[3];
      fin = fu_kick(P, F, u, xi, v, J, rp, fl, x) && fin;
      for (int a = 0; a < 3; ++a) {
        d.v[3 * sl + a] = v[a];
        d.J[3 * sl + a] = J[a];
        if (fl) d.r[3 * sl + a] = x[a];
        else nxt[3 * sl + a] = x[a];
      }
    }
    __syncthreads();                              // the angle buffer is rewritten next
  }
  if (!fin) atomicOr(&d.ctrl->err, E_BEADS);
  if (over) atomicOr(&d.ctrl->err, E_NBRLIST);
}

void launch_md_cycle_fused(const Dev& d, const FusedBufs& fb, int nseg, int nslots, int nrep, int n_sub, int K,
                           hipStream_t s) {
  if (nslots <= 0 || n_sub <= 0 || nseg <= 0) return;
  const int M = n_sub / K;
  for (int j = 0; j < M; ++j)
    hipLaunchKernelGGL(k_md_fused, dim3((unsigned)nseg), dim3(FU_WG), 0, s, d, fb, nslots, j * K, K,
                       j == M - 1 ? 1 : 0, j & 1);
  hipLaunchKernelGGL(k_md_redo, dim3((unsigned)nrep), dim3(RD_WG), 0, s, d, fb, fb.ang, nslots, n_sub, K);
}

void launch_md_noise(const Dev& d, int nslots, int n_sub, int step_offset, hipStream_t s) {
  long nk = (long)n_sub * nslots;
  if (nk > 0)
    hipLaunchKernelGGL(k_md_noise, dim3((unsigned)((nk + 255) / 256)), dim3(256), 0, s, d, nslots, n_sub,
                       step_offset);
}

void launch_zero_v(const Dev& d, int nslots, hipStream_t s) {
  if (nslots > 0) hipLaunchKernelGGL(k_zero_v, dim3((3 * nslots + 255) / 256), dim3(256), 0, s, d.v, 3 * nslots);
}

}  // namespace lbmd
