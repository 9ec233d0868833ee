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
__global__ void k_md_begin(uint32_t* rb, uint32_t* cst, int nrep) {
  for (int r = threadIdx.x; r < nrep; r += blockDim.x) {
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

// Component a of the bending forces of the angle at (ra, rb, rc): out[0] on
// the first bead, out[1] on the centre, out[2] on the third -- the operations
// of angle_add for that component, so the values a per-bead evaluation gives.
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
  int lst[MD_BPB][MAXNBR];                   // the neighbour list in use (chain indices)
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
            const int jj = q - so;
            double d0 = min_image(rp[0] - rin[3 * jj], g.nx);
            double d1 = min_image(rp[1] - rin[3 * jj + 1], g.ny);
            double d2 = min_image(rp[2] - rin[3 * jj + 2], g.nz);
            if (!(d0 * d0 + d1 * d1 + d2 * d2 < P.rlist2)) continue;
            const int at = atomicAdd(&sh.cnt[bslot], 1);
            if (at < MAXNBR) sh.lst[bslot][at] = jj;
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
            if (c < MAXNBR) sh.lst[bslot][c] = base + tt;
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
      const int j = jl[m] >= 0 ? jl[m] : p0;   // an unused entry reads a valid slot
      q[m][0] = rin[3 * j]; q[m][1] = rin[3 * j + 1]; q[m][2] = rin[3 * j + 2];
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
  for (int k = 0; k < cnt_b; ++k) {
    if (!((sh.hit[bslot][k % MD_LANES] >> (k / MD_LANES)) & 1u)) continue;
    F[0] += sh.pairF[bslot][k][0]; F[1] += sh.pairF[bslot][k][1]; F[2] += sh.pairF[bslot][k][2];
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
// and one lane sorts them into ascending chain order -- the list the
// in-kernel scan would build.  A bucket that overflows leaves its replica's
// lists marked invalid (and the table unusable), so the first sub-step
// rebuilds them by the full scan: the same lists, found slower.
// ---------------------------------------------------------------------------
__global__ void k_cell_clear(int* __restrict__ ccount, int nbuckets, uint32_t* __restrict__ rb, int nrep) {
  int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < nbuckets) ccount[k] = 0;
  if (k < nrep) rb[4 * k + 3] = 0u;          // valid unless a bucket overflows below
}

__global__ void k_cell_insert(Dev d, int nslots) {
  int slot = blockIdx.x * blockDim.x + threadIdx.x;
  if (slot >= nslots) return;
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
      if (at < LB_CAND) cand[lb][at] = q - so;
    }
  }
  __syncthreads();
  if (!on || lane != 0) return;
  // ascending chain order, the MAXNBR smallest kept
  int nc = ncand[lb];
  if (nc > MAXNBR) atomicOr(&d.ctrl->err, E_NBRLIST);
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
// cyclic reduction in LDS (thread k owns bond k); bead p adds the
// corrections of its bonds p (+) and p-1 (-) in that order.
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
    const double lam = con_pcr(sh, nbond);
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
    const double mu = con_pcr(sh, nbond);
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
  hipLaunchKernelGGL(k_md_begin, dim3(1), dim3(256), 0, s, d.rb, d.cst, nrep);
}

void launch_md_cycle(const Dev& d, int nslots, int nrep, int n_sub, const MdOverride& ov, hipStream_t s,
                     bool prologue, bool constrained) {
  if (nslots <= 0 || n_sub <= 0) return;
  unsigned nblk = (unsigned)(nslots / MD_BPB);
  if (prologue) {
    hipLaunchKernelGGL(k_md_begin, dim3(1), dim3(256), 0, s, d.rb, d.cst, nrep);
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
    hipLaunchKernelGGL(k_md_begin, dim3(1), dim3(256), 0, s, d.rb, d.cst, nrep);
    hipLaunchKernelGGL(k_md_start, dim3((nslots + 255) / 256), dim3(256), 0, s, d, nslots, none, 1);
  }
  for (int o = 0; o < M; ++o) {
    hipLaunchKernelGGL(k_md_substep<true>, dim3(nblk), dim3(3 * MD_WG), 0, s, d, none, nslots, o, o == 0 ? 1 : 2);
    hipLaunchKernelGGL(k_md_inner, dim3(nin), dim3(IN_WG), 0, s, d, nslots, o, Mb);
  }
  hipLaunchKernelGGL(k_md_substep<true>, dim3(nblk), dim3(3 * MD_WG), 0, s, d, none, nslots, M, 1);
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
