// lbmd_kernels.h -- data layout of a context and the host-side launchers.
//
// A context holds R replicas (R = 1 for a single system): independent
// lattices, each with its own chain, geometry and noise key, advanced in
// lockstep by the same launches.
//   - populations: replica r occupies Q * N_r elements at element offset
//     Q * node_off_r, laid out [Q][N_r] (structure of arrays);
//   - flags (1 byte / node) and the bead force density ([3][N_r]) follow the
//     same node offsets;
//   - beads live in slots; replica r owns slots [slot_off_r, slot_off_r +
//     nslot_r), nslot_r = nb_r rounded up to the MD workgroup size, so every
//     MD workgroup holds beads of one chain; chain index p = slot - slot_off_r;
//   - the sweep runs over a table of tiles (replica, first node), each of
//     tile_nodes consecutive nodes of one replica, in an order chosen by the
//     autotuner; the fluid reductions use a fixed table of OBS_TILE-node
//     tiles, contiguous per replica, so their summation order never changes.
#pragma once

#include "lbmd_dev.h"

namespace lbmd {

constexpr int MD_BPB = 16;                   // beads per MD workgroup (slot padding)
constexpr int NOBS = 25;                     // observables per replica
constexpr int MAX_REPLICAS = 1024;
constexpr int TILE_MIN = 256;                // smallest sweep tile (nodes)
constexpr int OBS_TILE = 4096;               // nodes per fluid-reduction tile
constexpr int CELL_CAP = 32;                 // beads per bucket of the neighbour-search table
// Sweep occupancy cap: a capped sweep workgroup reserves (LDS per CU - what
// two bead sub-step workgroups need) / cap bytes of LDS it does not use
constexpr int LDS_PER_CU = 160 * 1024;
constexpr int LDS_KEEP = 76 * 1024;
constexpr int SWEEP_CAP_MIN = 2, SWEEP_CAP_MAX = 8;

struct LbParams {
  int nx, ny, nz, nxy, N;
  double omega;     // 1 / tau
  double g[3];      // body-force density
  int has_g;
  // fluctuating fluid (fluct = 0: athermal): Philox key (fseed, frep); the
  // noise on mode k is sqrt(rho) famp[k-4] r, famp = sqrt(3 kT (1 - (1 -
  // omega)^2) / b_k), b_k the norm of mode k; famp32 the same in FP32
  int fluct;
  uint32_t fseed, frep;
  double famp[NMODE_NOISE];
  float famp32[NMODE_NOISE];
};

// One replica as the kernels see it.
struct Rep {
  Geom g;
  LbParams lp;
  MdParams mp;
  long node_off;    // first node in the packed node arrays
  int slot_off;     // first bead slot
  int nslot;        // bead slots (multiple of MD_BPB)
  int tile_begin;   // reduction tiles [tile_begin, tile_end)
  int tile_end;
  int wl_begin;     // bounce-back ledger blocks [wl_begin, wl_end) of the wall-link list
  int wl_end;
  double nfluid;    // fluid nodes (for the mass observable)
  int ncell[3];     // neighbour-search cells per axis (side >= r_c + skin)
};

struct Tile {
  int rep;
  int start;
};

// A fluid node with links to solid upstream nodes: bit i of mask is set when
// x - c_i is solid (the population f_i(x) is then bounced back).  Entries of
// one replica are contiguous and padded (mask 0) to a multiple of
// LEDGER_BLOCK, so that every reduction block holds one replica.
struct WallLink {
  int rep;
  int node;
  uint32_t mask;
  int pad;
};
constexpr int LEDGER_BLOCK = 256;
constexpr int NLEDGER = 6;                   // per replica: bounce-back [3], spread-on-solid [3]

// Every device array a kernel may touch.
struct Dev {
  const Rep* reps;
  const Tile* tiles;   // sweep tiles
  const Tile* otiles;  // reduction tiles
  uint8_t* flags;
  void* force;
  // beads, per slot [3] doubles
  double* r;
  double* v;
  double* up;
  double* J;
  double* rs;
  const int* slot_rep;
  // spreading: bead lists per base node, forced-node list
  int* head;        // per node, -1 when empty
  int* next;        // per slot
  int* base;        // per slot: base node (replica-local index)
  int2* touched;    // (replica, node) of the nodes carrying bead force
  // MD sub-cycle
  int* nbr;         // [slot][MAXNBR] slots of the partners, ascending
  int* ncnt;        // per slot
  double* ref;      // per slot [3]: positions at the last list build
  double* rmid0;    // per slot [3]: force-evaluation positions, double buffered
  double* rmid1;
  uint32_t* rb;     // [R][4]: rebuild flags (3 rotating) + list-invalid request
  double* xi;       // [n_sub][slots][3] noise of the current sub-cycle
  // reductions and per-replica bookkeeping
  double* part;     // [reduction tiles][4] fluid partial sums
  int64_t* tX;      // per replica: first step with the whole chain translocated, -1 before
  uint32_t* notdone;// per replica: some bead still on the cis side this step
  double* mdtape;   // when set: per sub-step s and bead p, r_mid and v at the start,
                    // [s][p][2][3] (recorded for the adjoint, one replica)
  int* ccount;      // neighbour search: beads per bucket of the hashed cell table
  int* cbuf;        // [buckets][CELL_CAP] bead slots of each bucket
  double* rbin;     // per slot: the position the table binned (1e300 before any build)
  uint32_t* cst;    // per replica, 3 rotating words: some bead is farther than CELL_MARGIN
                    // from its binned position at that sub-step (the table is not usable)
  uint32_t cmask;   // buckets - 1 (a power of two minus one)
  Ctrl* ctrl;
  int* redo;        // per replica: first sub-step the fused sub-cycle leaves to the per-sub-step
                    // launches (-1: none); reset at every cycle's opening
  // wall momentum ledgers (cumulative, FP64, per replica [NLEDGER]):
  // momentum the wall took by bounce-back, bead reaction that fell on solid
  // nodes; the wall-link list and one partial sum per list block
  const WallLink* wlinks;
  double* ledger;
  double* lpart;
  double* lsp;      // per slot [3]: the step's spread-on-solid share of the bead
};

// MD coefficients that replace the replicas' own during the pre-relaxation
// (friction gamma, e = exp(-gamma h), 1 - e; the force coefficient follows
// from each replica's mass).
struct MdOverride {
  int on;
  double gamma, e, omE, cf;
};

template <typename T, bool DEV> void launch_fill_rest(void* pops, long N, hipStream_t s);
void launch_fill_i32(int* p, long n, int v, hipStream_t s);
void launch_fill_f64(double* p, long n, double v, hipStream_t s);
// fluct: some replica has a fluctuating fluid (selects the sweep variant
// that draws the fluid noise; replicas without it skip the draw)
template <typename T, bool DEV>
void launch_lb(const void* A, void* B, const Dev& d, int ntiles, int tile_nodes, int grid, int cap, int skip_forced,
               bool fluct, hipStream_t s);
template <typename T, bool DEV>
void launch_lb_forced(const void* A, void* B, const Dev& d, int maxlist, hipStream_t s);
// start: 0, or also open the MD sub-cycle (what k_md_start does: 1 for
// uniform sub-steps, 2 for the multiple-time-step cycle) after launch_md_begin
template <typename T, bool DEV>
void launch_gather(const void* A, const Dev& d, int nslots, int start, hipStream_t s);
void launch_bead_prep(const Dev& d, int nslots, hipStream_t s);
template <typename T>
void launch_spread(const Dev& d, int nslots, hipStream_t s);
// Spreading fused with the update of the nodes it writes (forward step).
template <typename T, bool DEV>
void launch_spread_lb(const void* A, void* B, const Dev& d, int nslots, hipStream_t s);
void launch_step_end(const Dev& d, int nslots, int maxlist, int nrep, hipStream_t s);
// Observables into out[NOBS * r + k]; groups of the lb_observables mask
// (bit 0 fluid sums, 1 bead quantities, 2 wall ledgers, 3 step count); the
// entries of groups not asked for are left as they are.  part: the fluid
// partial sums (n_otiles x 4 doubles).
template <typename T, bool DEV>
void launch_observables(const void* A, const Dev& d, int n_otiles, int nrep, double* out, int mask, double* part,
                        hipStream_t s);
// Wall ledgers of one step: the bounce-back momentum of the links in the
// wall-link list (from the populations A the step reads; nblk list blocks),
// and the bead impulse of the step's spreading that falls on solid nodes.
template <typename T, bool DEV>
void launch_ledger_bb(const void* A, const Dev& d, int nblk, int nrep, hipStream_t s);
void launch_ledger_sp(const Dev& d, int nslots, int nrep, hipStream_t s);

// Adjoint pass (one replica, chains of at most MAX_ADJ_BEADS beads).
constexpr int MAX_ADJ_BEADS = 16384;
struct AdjBufs {
  double* lr;       // [slots][3] adjoint of r
  double* lv;       // [slots][3] adjoint of v
  double* lJ;       // [slots][3] adjoint of the impulse J
  double* lup;      // [slots][3] adjoint of u_p
  double* lrs;      // [slots][3] position term of the spreading transpose
  double* lr2;      // [slots][3] the other buffer of lr during the reversed sub-cycle
  double* lv2;      // [slots][3] the other buffer of lv
  double* gacc;     // [slots][3] per bead: dL/dgamma and dL/dF_drive terms of the reversed cycle
  double* dirA;     // [slots][3] the force derivative's direction cf (lv + hh lr) of each bead,
  double* dirB;     //   alternating between the reversed sub-steps
  int* lok;         // 0 while the reversed step's neighbour lists hold every close pair

  void* lamu;       // [3][N] (storage type) adjoint of the gathered node velocity
  double* par;      // [4]: dL/dgamma, dL/dF_drive accumulators
  double* xi;       // [n_sub][nb][3] the bead noise of the step being reversed
};
void launch_adj_init(const double* dLdr, const double* dLdv, const AdjBufs& a, int nb, hipStream_t s);
template <typename T, bool DEV>
void launch_adj_reverse_step(const void* A, const void* lamB, void* lamA, const Dev& d, const Dev& dspread,
                             const AdjBufs& a, const double* mdt, const double* upt,
                             const double* Jt, uint32_t step, double kT, int ntiles, int tile_nodes, int nslots,
                             int nb, int n_sub, hipStream_t s);
void launch_adj_finish(const AdjBufs& a, double* grads, int nb, hipStream_t s);

// MD sub-cycle of all replicas: n_sub launches, one per sub-step, reading
// the noise from d.xi (drawn beforehand by launch_md_noise; unused by
// replicas without noise and by the relaxation).
// prologue = false: the cycle's opening (launch_md_begin and the start of the
// sub-cycle) was done already, by launch_md_begin and launch_gather
// constrained: some replica has rigid bonds (a k_md_constraint launch after
// the opening and after every sub-step; chains without them skip it)
void launch_md_cycle(const Dev& d, int nslots, int nrep, int n_sub, const MdOverride& ov, hipStream_t s,
                     bool prologue = true, bool constrained = false);
void launch_md_begin(const Dev& d, int nrep, hipStream_t s);
// The multiple-time-step sub-cycle of a coupled step: M outer steps of
// n_sub / M SPV sub-steps with the bonded forces, between kicks of the slow
// forces (bead LJ, wall, field); noise from d.xi as in launch_md_cycle.
constexpr int MTS_MAX_INNER = 40;
constexpr int MAX_CONSTRAINED_BEADS = 1024;   // rigid bonds: one workgroup per chain   // inner sub-steps per outer step (the inner kernel's halo is 2 per sub-step)
void launch_md_cycle_mts(const Dev& d, int nslots, int nrep, int n_sub, int M, hipStream_t s, bool prologue = true);

// The uniform sub-cycle in blocks of K sub-steps, one launch per block:
// workgroup w advances the chain segment [a, b) of replica rep through the
// block, with the beads that can reach the segment within K sub-steps (its
// dependency cone: chain neighbours and close pair partners from the cell
// table) computed again alongside (see k_md_fused).  The state at a block's
// start is kept (the blocks alternate between the canonical arrays and the
// shadow ones); a block that cannot certify its result (a bead moved farther
// than FUSED_DELTA within it, or off its binned cell-table position by more
// than CELL_MARGIN, or a cone too large) leaves its replica to one
// workgroup that redoes the cycle from that block's start (k_md_redo).
// Results equal the per-sub-step cycle bit for bit.
struct FusedSeg {
  int rep, a, b, pad;
};
struct FusedBufs {
  const FusedSeg* seg;
  double* rmS;      // shadow [slots][3] r_mid, v, J
  double* vS;
  double* JS;
  double* ang;      // [slots][9] the redo's angle forces
  int* redo;        // per replica: first sub-step to redo, -1 when none
};
constexpr int FUSED_OWN = 48;                // chain beads a workgroup owns
constexpr int FUSED_K = 10;                  // sub-steps per block (the largest divisor of n_sub up to it)
constexpr double FUSED_DELTA = 0.1;          // displacement bound within a block
void launch_md_cycle_fused(const Dev& d, const FusedBufs& fb, int nseg, int nslots, int nrep, int n_sub, int K,
                           hipStream_t s);
// Noise of one sub-cycle into d.xi, for the step counter + step_offset.
void launch_md_noise(const Dev& d, int nslots, int n_sub, int step_offset, hipStream_t s);
void launch_md_invalidate(const Dev& d, int nrep, hipStream_t s);
// Verlet lists of every bead from a hashed cell list of the current
// positions (once per coupled step); marks the lists valid.
void launch_nbr_build(const Dev& d, int nslots, int nrep, hipStream_t s);
void launch_zero_v(const Dev& d, int nslots, hipStream_t s);

// Spread-on-solid ledger of one bead slot: the share W_k J_p of the step's
// impulse that the spreading drops because corner k of the bead's stencil
// (at the spread positions rs) is solid, corners in order, into lsp.  The
// wall is the only solid, so a stencil (base node and base + 1 along each
// axis) reaches it only from within one spacing below the plane.
__device__ inline void ledger_sp_share(const Dev& d, int slot) {
  const Rep& R = d.reps[d.slot_rep[slot]];
  const Geom& g = R.g;
  double s[3] = {0.0, 0.0, 0.0};
  const double rp[3] = {d.rs[3 * slot], d.rs[3 * slot + 1], d.rs[3 * slot + 2]};
  bool near = g.wall_axis >= 0 && slot - R.slot_off < R.mp.nb;
  if (near) {
    const double wn = wrapc(rp[g.wall_axis], ext(g, g.wall_axis));
    near = wn >= g.wall_pos - 1.0 && wn < g.wall_pos + 1.0;
  }
  if (near) {
    const uint8_t* fr = d.flags + R.node_off;
    const Stencil st = make_stencil(g, rp);
    uint8_t fl[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) fl[k] = fr[corner_node(g, st, k)];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      if (!corner_used(g, st, k) || !(fl[k] & F_SOLID)) continue;
      const double W = corner_weight(st, k);
      for (int a = 0; a < 3; ++a) s[a] += W * d.J[3 * slot + a];
    }
  }
  for (int a = 0; a < 3; ++a) d.lsp[3 * (size_t)slot + a] = s[a];
}

// The end of a coupled step on the sweep stream, once J is final: the
// spread-on-solid ledger (shares per slot, then each replica's beads added
// in a fixed order into its ledger) fused with the next step's neighbour
// lists (cell table cleared, beads binned, lists built): three launches.
void launch_step_tail(const Dev& d, int nslots, int nrep, bool ledger, hipStream_t s);

}  // namespace lbmd
