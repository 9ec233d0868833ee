/*
 * lbmd.h -- C ABI of the MI355X coupled lattice-Boltzmann / molecular-dynamics
 * library (liblbmd.so).
 *
 * The library advances the per-time-step hot path of the multiscale scheme of
 * Fyta, Sircar, Kaxiras, Melchionna, Bernaschi and Succi, "Parallel multiscale
 * modeling of biopolymer dynamics with hydrodynamic correlations":
 *   - a D3Q19 BGK solvent (Sec. 2, Eqs. (dens), (vel), (lbe2) and the
 *     equilibrium that follows it) with a force source term (the S_i of
 *     Sec. 2, Eq. (momentum_cons)) and halfway bounce-back at a wall plane
 *     with a square pore (Sec. 4);
 *   - a bead-spring polymer (Sec. 2, Eqs. (MD), (MDFORCES): truncated LJ,
 *     harmonic bonds, bending) advanced by the stochastic position Verlet
 *     scheme (Sec. 2, Eq. (SPValgo)) with the fluid velocity frozen during
 *     the MD sub-cycle;
 *   - the bead <-> fluid exchange: trilinear interpolation of u at each bead,
 *     friction gamma (u - v) plus Gaussian noise, and the reaction impulse
 *     spread back onto the 8 surrounding nodes.
 *
 * A context holds R >= 1 replicas (lb_ensemble_init; lb_init is R = 1):
 * independent systems, each with its own lattice, wall, chain and noise key,
 * advanced in lockstep by the same kernel launches.
 *
 * Conventions (all entry points):
 *   - Ownership: the caller allocates every device buffer (sizes from
 *     lb_buffer_sizes / lb_ensemble_sizes) and keeps it alive until
 *     lb_destroy; the library borrows the pointers and allocates no device
 *     memory (scratch areas such as the autotuner's state snapshot or the
 *     adjoint's checkpoints are buffers of the caller too).  It owns host
 *     objects only: two streams of its own, events, and the captured graph
 *     of lb_ensemble_run.
 *   - Streams: every call enqueues work on the stream given to lb_init and
 *     returns without synchronising, except where a call says that it
 *     synchronises.
 *   - Packing: replica r's nodes start at node offset node_off[r] (a
 *     multiple of 64) and its beads at slot offset slot_off[r] (a multiple
 *     of 16), both from lb_ensemble_layout; populations of replica r are
 *     [19][N_r] from element 19 node_off[r], flags and force ([3][N_r]) use
 *     the same node offsets, bead arrays the slot offsets.
 *   - Errors: each call returns LB_OK (0) or a negative LB_ERR_* code; the
 *     message of the last failure of the calling thread is returned by
 *     lb_last_error().  No C++ exception crosses this boundary.
 *   - Units: lattice units, lattice spacing = LB time step = 1.
 *   - Node index: c = x + nx * (y + ny * z).
 *   - Directions: population i moves along the D3Q19 velocity c_i (Sec. 2),
 *     in this order: 0 rest; 1, 2 = +x, -x; 3, 4 = +y, -y; 5, 6 = +z, -z;
 *     7, 8 = (1,1,0), (-1,-1,0); 9, 10 = (1,-1,0), (-1,1,0); 11, 12 =
 *     (1,0,1), (-1,0,-1); 13, 14 = (1,0,-1), (-1,0,1); 15, 16 = (0,1,1),
 *     (0,-1,-1); 17, 18 = (0,1,-1), (0,-1,1) (opposites adjacent); weights
 *     1/3, 1/18, 1/36 for rest, axis and diagonal directions.
 */
#ifndef LBMD_H
#define LBMD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  LB_OK = 0,
  LB_ERR_ARG = -1,         /* invalid description, size or pointer          */
  LB_ERR_DEVICE = -2,      /* a HIP call or kernel launch failed            */
  LB_ERR_UNSTABLE = -3,    /* watchdog: non-finite value or density <= 0    */
  LB_ERR_UNSUPPORTED = -4  /* valid request this build does not handle      */
};

/* Storage of the populations. */
enum {
  LB_FP64 = 0,     /* f_i in double                                           */
  LB_FP32_DEV = 1  /* f_i - w_i in float, collision in float, bead side FP64 */
};

/* Number of doubles lb_observables writes per replica. */
#define LB_NOBS 25

/* Groups of observables (the which_mask of lb_observables). */
enum {
  LB_OBS_FLUID = 1,     /* [0..3]: fluid mass and momentum (a pass over the lattice) */
  LB_OBS_BEADS = 2,     /* [4..15], [23], [24]: bead quantities                      */
  LB_OBS_LEDGERS = 4,   /* [16..21]: wall momentum ledgers                           */
  LB_OBS_STEP = 8,      /* [22]: step count                                          */
  LB_OBS_ALL = 15
};

/*
 * Run description.  The geometry follows Sec. 4: one wall plane normal to
 * wall_axis at lattice plane wall_pos, solid except a pore_h x pore_h block
 * centred on the two transverse axes (block [n/2 - pore_h/2, n/2 - pore_h/2 +
 * pore_h - 1] on each), periodic on all three axes.  wall_axis = -1 means no
 * wall (and no driving field).
 */
enum { LB_COUPLING_TRILINEAR = 0, LB_COUPLING_NGP = 1 };

typedef struct lb_desc {
  int32_t nx, ny, nz;
  int32_t precision;      /* LB_FP64 or LB_FP32_DEV                          */
  double tau;             /* BGK relaxation time (> 0.5); nu = (tau-1/2)/3   */
  double g[3];            /* uniform body-force density on every fluid node  */
  int32_t wall_axis;      /* -1, 0, 1, 2                                     */
  int32_t wall_pos;       /* 2 <= wall_pos <= n - 3 along wall_axis          */
  int32_t pore_h;         /* 0 <= pore_h <= transverse extent                */
  int32_t nb;             /* beads in the chain (0: fluid only)              */
  double mass;            /* bead mass; 1 whenever gamma > 0 (the exponential
                             kick of Sec. 2, Eq. (SPValgo), treats gamma as a
                             rate and its friction term as gamma u_p, which
                             gives the impulse m (1 - e)(u - v) that the fluid
                             takes only at unit mass)                        */
  double k_bond, r0;      /* harmonic bond constant and rest length          */
  double kappa;           /* bending constant, V = kappa phi^2 / 2           */
  double eps, sigma, rc;  /* truncated LJ (bead-bead and bead-wall site),
                             0 < rc <= 3                                     */
  double gamma, kT;       /* friction rate and thermal energy of the beads   */
  double f_drive;         /* force along +normal on beads in the pore channel */
  int32_t n_sub;          /* MD sub-steps per LB step                        */
  uint32_t seed, replica; /* Philox key of the bead and the fluid noise       */
  double fluid_kT;        /* thermal energy of the fluctuating fluid (Sec. 2,
                             the stochastic term F_i, read as noise on the 15
                             non-conserved D3Q19 modes with the amplitudes of
                             fluctuation-dissipation); 0: athermal BGK fluid.
                             Node c of a replica draws, at LB step n, Philox-
                             4x32-10 of counters (n, c, k, 1), k = 0..3       */
  int32_t mts_outer;      /* 0: the MD sub-cycle is n_sub uniform SPV sub-steps
                             with every force.  M > 0: the multiple-time-step
                             cycle (Sec. 2, the nested cycle over the bonds,
                             read as a RESPA split): M outer steps of 1/M, each
                             a half kick of the slow forces (bead LJ, wall,
                             field), n_sub / M SPV sub-steps with the bonds and
                             bending, friction and noise, and another half
                             kick.  n_sub / M must be a whole number <= 40; all
                             replicas share M; the pre-relaxation always uses
                             uniform sub-steps                               */
  int32_t coupling;       /* bead <-> lattice transfer of u_p and the impulse
                             (Sec. 2, the particle/grid paragraph):
                             LB_COUPLING_TRILINEAR (the 8 nodes around the
                             bead, trilinear weights) or LB_COUPLING_NGP (the
                             paper's: the nearest node, the upper one along an
                             axis where the fraction is 1/2)                 */
  int32_t constraints;    /* 0: harmonic bonds k_bond/2 (|d| - r0)^2.  1: rigid
                             bonds |r_{p+1} - r_p| = r0 (Sec. 2, Eq. (SPValgo)
                             with its SHAKE and RATTLE steps; k_bond unused):
                             per sub-step the drifted positions are projected
                             onto the bonds along the bonds at the sub-step's
                             start and the velocity takes the same impulse;
                             after the kick the relative velocities along the
                             bonds are removed.  Needs mts_outer = 0 and
                             nb <= 1024                                      */
} lb_desc;

/* Byte sizes of the caller-allocated device buffers (256-byte aligned), and
 * the packed node and bead-slot counts. */
typedef struct lb_sizes {
  size_t pops_bytes;   /* one population array, 19 per packed node, double or
                          float; two are needed (pops_a, pops_b)            */
  size_t flags_bytes;  /* uint8 per packed node                               */
  size_t force_bytes;  /* bead force density on the lattice, 3 per node       */
  size_t beads_bytes;  /* bead state, doubles: r, v, u_p, J, r_start, each
                          [bead_slots][3]                                     */
  size_t work_bytes;   /* private scratch: lists, counters, partial sums      */
  size_t state_bytes;  /* size of the buffer lb_get_state writes              */
  size_t nodes;        /* packed lattice nodes (all replicas, with padding)   */
  size_t bead_slots;   /* bead slots (all replicas, with padding)             */
  size_t snapshot_bytes; /* scratch lb_autotune_step needs: a copy of the
                            populations, force, beads and work buffers         */
} lb_sizes;

/* Device pointers (hipMalloc'ed or torch CUDA tensors), 256-byte aligned. */
typedef struct lb_buffers {
  void* pops_a;
  void* pops_b;
  void* flags;
  void* force;
  void* beads;
  void* work;
} lb_buffers;

typedef struct lb_ctx lb_ctx;

/* Validates *d and fills *out.  Host only: calls no HIP function.
 * LB_ERR_ARG: extents <= 0 or 19 N > 2^31 - 1, tau <= 0.5, a wall plane
 * outside [2, n-3], a pore wider than the face, nb < 0, n_sub < 1, negative
 * gamma, kT or fluid_kT, rc outside (0, 3], nb > 0 without a positive
 * mass, a mass other than 1 with gamma > 0, nb > 0 with a wall on a lattice
 * with an extent below 6, or an
 * mts_outer that is negative or does not divide n_sub into at most 40, an
 * unknown coupling, or rigid bonds with mts_outer > 0 or nb > 1024. */
int lb_buffer_sizes(const lb_desc* d, lb_sizes* out);

/* As lb_buffer_sizes for nrep replicas d[0..nrep-1] in one context.  All
 * replicas share precision, n_sub and mts_outer; extents, walls, chains, friction,
 * temperature, field and noise keys may differ.  LB_ERR_ARG also for nrep
 * outside [1, 1024] or mixed precision / n_sub / mts_outer. */
int lb_ensemble_sizes(const lb_desc* d, int nrep, lb_sizes* out);

/* Creates a context on the current HIP device, builds the solid flags of the
 * geometry on the host and uploads them, fills both population arrays with
 * the rest equilibrium f_i = w_i (zero in LB_FP32_DEV; Sec. 4: unit density,
 * zero velocity) and uploads the bead positions r0_host and velocities
 * v0_host ([nb][3] doubles, host memory; v0_host may be NULL for zero;
 * positions are unwrapped).  stream is a hipStream_t (NULL: the default
 * stream).  Synchronises the stream before returning.  LB_ERR_ARG: as
 * lb_buffer_sizes, a NULL or misaligned buffer, or non-finite bead state. */
int lb_init(const lb_desc* d, const lb_buffers* b, const double* r0_host, const double* v0_host,
            void* stream, lb_ctx** out);

/* As lb_init for nrep replicas (the batched ensemble): r0_host / v0_host
 * hold the chains one after the other, replica 0 first ([sum nb][3]). */
int lb_ensemble_init(const lb_desc* d, int nrep, const lb_buffers* b, const double* r0_host,
                     const double* v0_host, void* stream, lb_ctx** out);

/* Host only: writes the node offset and bead-slot offset of every replica
 * (arrays of nrep). */
int lb_ensemble_layout(lb_ctx* ctx, int64_t* node_off, int64_t* slot_off);

/* Releases the host-side context; the caller frees its buffers afterwards. */
void lb_destroy(lb_ctx* ctx);

/* nsteps fluid-only LB steps of every replica (Sec. 2, Eq. (lbe2)):
 * pull-stream with halfway bounce-back, BGK collision towards the
 * second-order equilibrium, source 3 w_i g.c_i of the uniform body force.
 * Beads are not moved. */
int lb_step(lb_ctx* ctx, int nsteps);

/* nsteps coupled steps of every replica.  Each step, at the bead positions
 * r(n):
 *   1. u_p = trilinear interpolation of the fluid velocity (from the pulled
 *      populations of the stored array; u = 0 at solid nodes) (Sec. 2, the
 *      particle-to-grid transfer, here trilinear instead of nearest point);
 *   2. n_sub SPV sub-steps of h = 1/n_sub with u_p frozen (Sec. 2,
 *      Eq. (SPValgo) without constraints): r += h/2 v;
 *      v = e v + (1-e)/(m gamma) (F(r) + gamma u_p) + sqrt(kT/m (1-e^2)) xi;
 *      r += h/2 v; e = exp(-gamma h); F = bonds + bending + bead LJ + wall LJ
 *      + field; xi from Philox4x32-10 keyed (seed, replica) with counter
 *      (step, sub-step, bead, 0) and Box-Muller;
 *   3. J_p = -(friction + noise impulse) is spread trilinearly at r(n) onto
 *      the 8 nodes, summed per node in ascending bead order (no atomics);
 *   4. one LB step with the source 3 w_i (F(x) + g).c_i (Sec. 2, S_i). */
int md_couple_step(lb_ctx* ctx, int nsteps);

/* As md_couple_step, for the batched ensemble: with use_graph != 0 the
 * launches of two coupled steps are captured once into a HIP graph
 * (re-captured after lb_sweep_config / lb_autotune) and the graph is
 * replayed; an odd step, or a step that brings the populations to the
 * graph's parity, runs eagerly.  Results are identical to md_couple_step.
 * While lb_profile_start is active the steps run eagerly. */
int lb_ensemble_run(lb_ctx* ctx, int nsteps, int use_graph);

/* Synchronises the stream and copies, per replica, the first step count at
 * which every bead's normal coordinate exceeded the wall plane (the chain
 * has translocated), or -1 (not yet, or no wall / no chain), to out_host
 * (nrep int64). */
int lb_ensemble_translocation(lb_ctx* ctx, int64_t* out_host);

/* The uniform MD sub-cycle (mts_outer = 0, harmonic bonds) can run in
 * blocks of K sub-steps, one launch per block (off by default: on the
 * workloads measured it is slower than one launch per sub-step): each
 * workgroup advances a chain segment and recomputes the beads that can reach
 * it within the block (chain neighbours, and pair partners closer than
 * r_c + 0.2 from the step's neighbour lists), then certifies the result (no
 * bead moved more than 0.1 within the block, and every bead was within half
 * the list skin less 0.1 of where the lists were built).  A replica whose
 * block cannot be certified is redone from that block's start by one
 * workgroup (a launch that returns at once when nothing is to be redone), so
 * results equal the per-sub-step cycle bit for bit.  lb_md_fused(ctx, 0)
 * switches back to one launch per sub-step.  Drops the captured graph.
 * LB_ERR_UNSUPPORTED: K > 0 and the context has no chain, or uses the
 * multiple-time-step cycle or rigid bonds; LB_ERR_ARG: K < 0, or K not
 * dividing n_sub, below 2 or above 10. */
int lb_md_fused(lb_ctx* ctx, int K);

/* Sweep layout: tile_nodes (a multiple of 256) consecutive nodes of one
 * replica per tile; order 0 lists tiles replica by replica, order 1 deals
 * them into 8 contiguous chunks interleaved so that neighbouring tiles run on
 * one XCD; grid 0 launches one workgroup per tile, grid > 0 that many
 * workgroups striding over the tiles.  A thread updates tile_nodes / 256
 * nodes of a tile (at most 4 per pass, their loads issued together).  cap 0
 * leaves the occupancy to the hardware; cap in [2, 8] lets at most cap sweep
 * workgroups share a CU (each reserves LDS it does not use), which leaves
 * the rest of the CU to the bead phase running beside the sweep.  Results do
 * not depend on the layout.  Synchronises the stream (uploads the tile
 * table).  LB_ERR_ARG: order not 0 or 1, grid < 0, cap outside {0, 2..8},
 * tile_nodes not a positive multiple of 256. */
int lb_sweep_config(lb_ctx* ctx, int tile_nodes, int order, int grid, int cap);

/* Autotuner of the sweep layout: times `reps` sweeps of every candidate
 * layout (tile sizes 256..2048 in both orders; persistent grids of 256,
 * 384, 512, 768, 1024 and 2048 workgroups over tiles of 256 and 512 nodes;
 * tiles of 256, 512 and 1024 nodes capped at 2, 3 or 4 workgroups per CU)
 * with HIP events, from the current populations into the other array (which
 * the next step overwrites, so the state is unchanged), keeps the first
 * candidate within
 * 1% of the fastest and caches it for the process by (replica extents,
 * walls and chain lengths, precision, athermal or fluctuating fluid).
 * Writes {tile_nodes, order, grid, cap} to out_cfg[4] and the mean sweep
 * time in ms to *out_ms (the time measured when the entry was cached).  With the
 * environment variable LBMD_AUTOTUNE_LOG set, every candidate's time is
 * printed to stderr.  Synchronises the stream.
 * LB_ERR_ARG: reps < 1; LB_ERR_DEVICE: a HIP call failed. */
int lb_autotune(lb_ctx* ctx, int reps, int* out_cfg, double* out_ms);

/* As lb_autotune, choosing the layout by the whole coupled step instead of
 * the sweep alone (the sweep shares the memory system with the bead phase
 * that runs beside it): per candidate, 2 ceil(reps / 2) coupled steps
 * replayed from the two-step graph are timed.  The complete device state
 * (current populations, beads, work area, force field) is first copied to
 * snap_dev, a device buffer of the caller of at least
 * lb_sizes.snapshot_bytes (256-byte aligned; unused when the layout is
 * already cached), and restored after every candidate, with the step count:
 * the state and every later result are unchanged.  *out_ms is the mean
 * coupled-step time (as measured when the entry was cached).  No device
 * memory is allocated.
 * Synchronises the stream.  LB_ERR_ARG: reps < 1, snap_dev NULL, too small
 * or misaligned (the layout not being cached); LB_ERR_DEVICE: a HIP call
 * failed (the state is restored from the snapshot). */
int lb_autotune_step(lb_ctx* ctx, int reps, void* snap_dev, size_t snap_bytes, int* out_cfg, double* out_ms);

/* Sets the friction rate gamma (>= 0) and the pore force F_drive of
 * replica rep and recomputes its SPV coefficients (e = exp(-gamma h), the
 * noise amplitude from the replica's kT).  Synchronises the stream.
 * LB_ERR_ARG: rep out of range, a negative or non-finite value, or gamma > 0
 * on a chain whose mass is not 1. */
int lb_set_coupling(lb_ctx* ctx, int rep, double gamma, double f_drive);

/*
 * Adjoint of nsteps coupled steps (reverse-mode derivative; the method's
 * gradient form).  For a loss L that depends on the bead positions (and
 * optionally velocities) after the steps, it returns dL/dgamma, dL/dF_drive
 * and dL/dr at the start, the derivative of the discrete step map itself
 * (fixed noise sequence: the Philox counters do not depend on the
 * parameters).  Each step is reversed stage by stage -- LB sweep (the
 * transposed BGK Jacobian and streaming), spreading, the MD sub-cycle
 * (sub-steps in reverse; force Jacobians as directional derivatives of the
 * conservative forces), gathering -- using the populations and bead state of
 * that step, recomputed segment by segment from checkpoints taken every K
 * steps of the forward pass.
 * Supported: one-replica contexts with 1 <= nb <= 16384, gamma > 0, an
 * athermal fluid (fluid_kT = 0), the uniform sub-cycle (mts_outer = 0),
 * harmonic bonds and the trilinear transfer (LB_ERR_UNSUPPORTED / LB_ERR_ARG
 * otherwise); either precision.
 *
 * lb_adjoint_sizes: workspace bytes for (nsteps, K): nsteps/K + 1
 *   checkpoints of lb_sizes.state_bytes, K population arrays and bead
 *   sub-cycle records of tape, the adjoint fields, and one step's bead noise
 *   (n_sub x nb x 3 doubles).  Host only.
 * lb_adjoint_forward: runs nsteps coupled steps from the current state (as
 *   md_couple_step does) and records the checkpoints in ws (device, at
 *   least the size above, 256-byte aligned, owned by the caller, kept until
 *   the backward call).  With K >= nsteps (one segment) it also writes the
 *   tape, and the backward pass does not recompute the horizon; the
 *   gradients are the same bit for bit as with any other K.
 * lb_adjoint_backward: dLdr_dev (and dLdv_dev, may be NULL for zero): [nb][3]
 *   doubles on the device, the loss gradient at the final state.  Writes
 *   grads_dev[0] = dL/dgamma, [1] = dL/dF_drive, [2 ..] = dL/dr_start
 *   ([nb][3]).  Leaves the context in the final state of the forward pass.
 * lb_adjoint_run: forward then backward with dLdv = 0.
 */
int lb_adjoint_sizes(lb_ctx* ctx, int nsteps, int K, size_t* bytes);
int lb_adjoint_forward(lb_ctx* ctx, int nsteps, int K, void* ws_dev, size_t ws_bytes);
int lb_adjoint_backward(lb_ctx* ctx, const double* dLdr_dev, const double* dLdv_dev, double* grads_dev);
int lb_adjoint_run(lb_ctx* ctx, int nsteps, int K, void* ws_dev, size_t ws_bytes, const double* dLdr_dev,
                   double* grads_dev);

/* Pre-relaxation of the chain (Sec. 4: the initial walk is relaxed by MD):
 * nsub_total SPV sub-steps with no fluid coupling, no field, no noise and
 * friction gamma_relax; the velocities are zeroed at the end. */
int md_relax(lb_ctx* ctx, int nsub_total, double gamma_relax);

/* Writes LB_NOBS doubles per replica to out_dev (device memory; replica r
 * at out_dev + LB_NOBS r), the groups of which_mask (LB_OBS_* bits; entries
 * of groups not asked for are left as they are; LB_ERR_ARG for unknown
 * bits): [0] fluid mass,
 * [1..3] fluid momentum (Sec. 3: global momentum reductions), [4] bead
 * temperature m<v^2>/3 (Sec. 2: the monitored bead temperature), [5..7] bead
 * momentum, [8] mean unwrapped normal coordinate, [9] translocated fraction,
 * [10] beads in the pore channel, [11] R_U, [12] R_T, [13] R_eff with
 * nu = 0.6 (Sec. 4, Eq. (R_eff)), [14] dW_H/dt = gamma sum v.u_p and
 * [15] dW_E/dt = sum F_drive.v (Sec. 4, translocation work), [16..18] the
 * momentum the wall has taken by bounce-back since lb_init, sum over steps
 * and links (x, i) with x - c_i solid of 2 f_opp(i)(x) c_opp(i), and
 * [19..21] the bead impulse the spreading dropped on solid nodes since
 * lb_init, sum of W_k J_p over solid corners (the two wall terms of the
 * bead-fluid momentum balance, Sec. 2, Eq. (momentum_cons)), [22] step
 * count, [23] and [24] the viscous drag along the wall normal, m gamma
 * (u_p - v) summed over the untranslocated and the translocated beads
 * (Sec. 4, the drag forces on the two parts).  Sums are FP64. */
int lb_observables(lb_ctx* ctx, double* out_dev, int which_mask);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): as
 * lb_observables, with the fluid reduction's partial sums in a static
 * device array the library holds on each GPU for the life of the process
 * (4 doubles per reduction tile of 4096 nodes, at most 16384 tiles, i.e.
 * packed lattices of up to 67,108,864 nodes; 512 KiB), instead of the
 * context's work buffer.  The caller still provides out_dev.  Allocates
 * nothing.  Every call on one GPU shares that array: calls that overlap on
 * one GPU (other streams, other threads) race and must be ordered by the
 * caller.  LB_ERR_ARG: as lb_observables, or LB_OBS_FLUID asked for on a
 * context whose packed lattice exceeds the limit. */
int lb_observables_static(lb_ctx* ctx, double* out_dev, int which_mask);

/* Checkpoint: copies the current populations (every replica, the storage
 * type), r and v of every bead slot, the step counter (uint64), the
 * translocation steps and the wall ledgers to dst_dev (device, lb_sizes.state_bytes) / restores
 * them from src_dev.  Device to device, enqueued on the stream;
 * lb_set_state synchronises it to read back the step counter. */
int lb_get_state(lb_ctx* ctx, void* dst_dev);
int lb_set_state(lb_ctx* ctx, const void* src_dev);

/* Device pointer of the populations that the next step reads. */
void* lb_current_pops(lb_ctx* ctx);

/* Synchronises the stream and reads the device watchdog word: LB_OK, or
 * LB_ERR_UNSTABLE (non-finite or non-positive density, non-finite bead
 * state, a neighbour list or node-contributor list overflow), with the
 * reason in lb_last_error(). */
int lb_check(lb_ctx* ctx);

/* Steps taken so far (host copy). */
int64_t lb_step_count(lb_ctx* ctx);

/* Kernel timing: from lb_profile_start on, HIP events are recorded around
 * every LB sweep (phase 0, on the stream the sweep runs on) and every bead
 * phase -- gather, MD sub-cycle, spreading and the update of the nodes that
 * carry bead force -- (phase 1) of lb_step / md_couple_step, for at most
 * max_steps steps.  lb_profile_stop synchronises the stream, writes the
 * mean duration in ms of each phase and the number of steps recorded, and
 * stops recording.  Events are host-side objects; no device memory is
 * allocated by the library.  LB_ERR_ARG: max_steps < 1 or recording already
 * active / not active. */
int lb_profile_start(lb_ctx* ctx, int max_steps);
int lb_profile_stop(lb_ctx* ctx, double* mean_lb_ms, double* mean_bead_ms, int* nsteps);

/* Diagnostics: synchronises the stream and writes fifteen int64: out[0] =
 * neighbour-list rebuilds inside sub-cycles (summed over replicas), out[1] =
 * MD sub-step launches that did work (with the fused sub-cycle: sub-steps
 * redone, per replica), out[2] = tiles of the sweep, out[3] = watchdog bits,
 * out[4] = LB steps taken, out[5] = nodes that carried bead force, summed
 * over steps, out[6] = the rebuilds of out[0] that searched the cell table
 * (the others scanned the whole chain), out[7] = fused sub-cycle blocks
 * completed, out[8] = replica sub-cycles redone from a fused block that
 * could not certify its result (see lb_md_fused), out[9..13] = why fused
 * blocks failed, counted per failing workgroup: the step's neighbour lists
 * not valid at the cycle's start, or a bead of its segment farther than half
 * the list skin less 0.1 from where they were built, more than 16 close
 * partners of a bead (or 16 new spans in one round), the dependency cone over
 * its capacity (128 beads in 16 spans), the cone not settled in 6 rounds, a
 * bead of the segment moved more than 0.1 within the block; out[14] = the
 * longest neighbour list a per-step build found so far (more than 48 trips
 * the watchdog, bit 4, which lb_check reports as LB_ERR_UNSTABLE). */
int lb_diagnostics(lb_ctx* ctx, int64_t* out);

/* Message of the last failed call on this thread (never NULL). */
const char* lb_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* LBMD_H */
