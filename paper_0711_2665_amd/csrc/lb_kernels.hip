// lb_kernels.hip -- lattice side of the coupled step: the fused
// stream + collide sweep, the bead gather (fluid velocity at the beads), the
// deterministic spreading of the bead reaction onto the lattice, and the
// fluid reductions.  All kernels serve every replica of a context.
#include "lbmd_kernels.h"
#include "lbmd_lattice.h"

namespace lbmd {

// ---------------------------------------------------------------------------
// Fills
// ---------------------------------------------------------------------------
template <typename T, bool DEV>
__global__ void k_fill_rest(T* __restrict__ pops, long N) {
  long c = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= N) return;
#pragma unroll
  for (int i = 0; i < Q; ++i) pops[(size_t)i * N + c] = DEV ? (T)0 : (T)wgt(i);
}

__global__ void k_fill_i32(int* __restrict__ p, long n, int v) {
  long k = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) p[k] = v;
}

__global__ void k_fill_f64(double* __restrict__ p, long n, double v) {
  long k = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) p[k] = v;
}

// ---------------------------------------------------------------------------
// K1: the sweep over a table of tiles (each tile_nodes consecutive nodes of
// one replica); workgroups stride over the table.  Solid nodes are skipped,
// and so are nodes carrying a bead force when skip_forced is set (they are
// updated by k_lb_forced once the force is known).
// ---------------------------------------------------------------------------
template <typename T, bool DEV, int U, bool FL>
__global__ __launch_bounds__(256) void k_lb(const T* __restrict__ A, T* __restrict__ B,
                                            const Tile* __restrict__ tiles, const Rep* __restrict__ reps,
                                            const uint8_t* __restrict__ flags, const T* __restrict__ force,
                                            Ctrl* __restrict__ ctrl, int ntiles, int tile_nodes, int skip_forced) {
  // The tile and replica tables are read-only arguments that alias nothing
  // the sweep writes, so their workgroup-uniform reads become scalar loads;
  // the next tile's record is requested before this tile's work.
  int t = blockIdx.x;
  if (t >= ntiles) return;
  const uint32_t n = FL ? (uint32_t)ctrl->step : 0u;   // LB step: counter word 0 of the fluid noise
  Tile tl = tiles[t];
  for (;;) {
    const int tn = t + (int)gridDim.x;
    const Tile next = tiles[tn < ntiles ? tn : t];
    const Rep& R = reps[tl.rep];
    const long no = R.node_off;
    const T* Ar = A + (size_t)Q * no;
    T* Br = B + (size_t)Q * no;
    const uint8_t* fr = flags + no;
    const T* Fr = force + (size_t)3 * no;
    const int end = min(tl.start + tile_nodes, R.lp.N);
    // U nodes per thread and pass, 256 apart, their loads issued together
    for (int c0 = tl.start + (int)threadIdx.x; c0 < end; c0 += U * 256) {
      int c[U];
      bool in[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int cu = c0 + u * 256;
        in[u] = cu < end;
        c[u] = in[u] ? cu : c0;             // past the tile: pull a valid node, store nothing
      }
      lb_nodes<T, DEV, U, FL>(Ar, Br, fr, Fr, R.lp, ctrl, c, in, skip_forced, n);
    }
    if (tn >= ntiles) break;
    t = tn;
    tl = next;
  }
}

// The nodes that carry a bead force this step (the list written by the
// spreading kernel).
template <typename T, bool DEV>
__global__ __launch_bounds__(64) void k_lb_forced(const T* __restrict__ A, T* __restrict__ B, Dev d, int maxlist) {
  int k = blockIdx.x * blockDim.x + threadIdx.x;
  int nt = (int)d.ctrl->touched;
  if (k >= nt || k >= maxlist) return;
  const int2 e = d.touched[k];
  const Rep& R = d.reps[e.x];
  const long no = R.node_off;
  const uint8_t* fr = d.flags + no;
  lb_node<T, DEV>(A + (size_t)Q * no, B + (size_t)Q * no, fr, (const T*)d.force + (size_t)3 * no, R.lp, d.ctrl, e.y,
                  fr[e.y]);
}

// ---------------------------------------------------------------------------
// Start of a coupled step: remember r(n), link every bead into the list of
// its base node, clear J, and mark the stencil nodes of r(n) as carrying bead
// force this step (solid ones are dropped by the spreading; every writer of
// a node stores the same byte).
// ---------------------------------------------------------------------------
__global__ void k_bead_prep(Dev d, int nslots) {
  int slot = blockIdx.x * blockDim.x + threadIdx.x;
  if (slot >= nslots) return;
  const Rep& R = d.reps[d.slot_rep[slot]];
  if (slot - R.slot_off >= R.mp.nb) return;
  double rp[3] = {d.r[3 * slot], d.r[3 * slot + 1], d.r[3 * slot + 2]};
  Stencil st = make_stencil(R.g, rp);
  int cell = st.b[0] + R.g.nx * (st.b[1] + R.g.ny * st.b[2]);
#pragma unroll
  for (int a = 0; a < 3; ++a) { d.rs[3 * slot + a] = rp[a]; d.J[3 * slot + a] = 0.0; }
  d.base[slot] = cell;
  d.next[slot] = atomicExch(&d.head[R.node_off + cell], slot);
  uint8_t* fr = d.flags + R.node_off;
  for (int k = 0; k < 8; ++k) {
    if (!corner_used(R.g, st, k)) continue;
    int n = (int)corner_node(R.g, st, k);
    uint8_t fl = fr[n];
    if (!(fl & F_SOLID)) fr[n] = fl | F_FORCED;
  }
}

// ---------------------------------------------------------------------------
// K2: u_p = sum_k W_k u(node_k) at r(n) (trilinear).  Eight consecutive
// lanes per bead, one corner each; the corner terms are added by the bead's
// first lane in corner order.
// ---------------------------------------------------------------------------
template <typename T, bool DEV>
__global__ void k_gather(const T* __restrict__ A, Dev d, int nslots, int start) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  const int slot = e >> 3, k = e & 7;
  bool on = slot < nslots;
  int rep = 0;
  if (on) {
    rep = d.slot_rep[slot];
    on = slot - d.reps[rep].slot_off < d.reps[rep].mp.nb;
  }
  double t[3] = {0.0, 0.0, 0.0};
  if (on) {
    const Rep& R = d.reps[rep];
    const T* Ar = A + (size_t)Q * R.node_off;
    const uint8_t* fr = d.flags + R.node_off;
    double rp[3] = {d.rs[3 * slot], d.rs[3 * slot + 1], d.rs[3 * slot + 2]};
    Stencil st = make_stencil(R.g, rp);
    int node = (int)corner_node(R.g, st, k);
    double W = corner_weight(st, k);
    double u[3];
    node_velocity<T, DEV>(Ar, fr, R.lp, node, u);
    t[0] = W * u[0]; t[1] = W * u[1]; t[2] = W * u[2];
  }
  const int base = (int)(threadIdx.x & 63u) & ~7;
  double acc[3] = {0.0, 0.0, 0.0};
  for (int c = 0; c < 8; ++c)
    for (int a = 0; a < 3; ++a) acc[a] += __shfl(t[a], base + c, 64);
  if (on && k == 0) {
    d.up[3 * slot] = acc[0]; d.up[3 * slot + 1] = acc[1]; d.up[3 * slot + 2] = acc[2];
    if (start) {
      // the opening of the MD sub-cycle: r_mid of sub-step 0 (start = 1;
      // with the multiple-time-step cycle, start = 2, r itself) and the
      // displacement checks that decide whether its first launch rebuilds
      // the neighbour lists
      const Rep& R = d.reps[rep];
      double d2 = 0.0, b2 = 0.0;
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        const double x = start == 2 ? d.r[3 * slot + a] : d.r[3 * slot + a] + R.mp.hh * d.v[3 * slot + a];
        d.rmid0[3 * slot + a] = x;
        const double dd = x - d.ref[3 * slot + a];
        d2 += dd * dd;
        const double db = x - d.rbin[3 * slot + a];
        b2 += db * db;
      }
      if (d2 > R.mp.halfskin2) d.rb[4 * rep] = 1u;
      if (!(b2 <= CELL_MARGIN * CELL_MARGIN)) d.cst[4 * rep] = 1u;
    }
  }
}

// ---------------------------------------------------------------------------
// K4: spreading.  One thread per (bead p, corner k).  The node n of that
// corner receives W_k'(q) J_q from every bead q whose base node is n - o_k';
// these contributions are collected from the per-node bead lists, sorted by
// (q, k') and summed in that order by the thread that holds the smallest
// (q, k') -- each node is written once, with no atomics, and the sum runs in
// ascending bead order.  Shares on solid nodes are dropped.
// ---------------------------------------------------------------------------
template <typename T>
__global__ void k_spread(Dev d, int nslots) {
  int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= 8 * nslots) return;
  int slot = e >> 3, k = e & 7;
  const int rep = d.slot_rep[slot];
  const Rep& R = d.reps[rep];
  const int p = slot - R.slot_off;
  if (p >= R.mp.nb) return;
  const Geom& g = R.g;
  const uint8_t* fr = d.flags + R.node_off;
  double rp[3] = {d.rs[3 * slot], d.rs[3 * slot + 1], d.rs[3 * slot + 2]};
  Stencil st = make_stencil(g, rp);
  if (!corner_used(g, st, k)) return;
  int n = (int)corner_node(g, st, k);
  if (fr[n] & F_SOLID) return;
  int nz_ = n / g.nxy, rem = n - nz_ * g.nxy, ny_ = rem / g.nx, nx_ = rem - ny_ * g.nx;
  // contributors as keys q*8 + k' (q the chain index)
  int keys[MAXCONTRIB];
  int cnt = 0;
  bool overflow = false;
  for (int k2 = 0; k2 < 8; ++k2) {
    int bx = nx_ - (k2 & 1); if (bx < 0) bx += g.nx;
    int by = ny_ - ((k2 >> 1) & 1); if (by < 0) by += g.ny;
    int bz = nz_ - ((k2 >> 2) & 1); if (bz < 0) bz += g.nz;
    int cell = bx + g.nx * (by + g.ny * bz);
    for (int q = d.head[R.node_off + cell]; q >= 0; q = d.next[q]) {
      if (g.ngp) {
        // with the nearest-grid-point transfer only q's nearest node counts
        const Stencil sq = make_stencil(g, &d.rs[3 * q]);
        if (!corner_used(g, sq, k2)) continue;
      }
      int key = (q - R.slot_off) * 8 + k2;
      if (cnt < MAXCONTRIB) {
        int j = cnt++;
        while (j > 0 && keys[j - 1] > key) { keys[j] = keys[j - 1]; --j; }
        keys[j] = key;
      } else {
        overflow = true;
      }
    }
  }
  if (overflow) { atomicOr(&d.ctrl->err, E_SPREAD); }
  if (keys[0] != p * 8 + k) return;   // not the owner of node n
  double F[3] = {0.0, 0.0, 0.0};
  for (int j = 0; j < cnt; ++j) {
    int qs = R.slot_off + (keys[j] >> 3), k2 = keys[j] & 7;
    double rq[3] = {d.rs[3 * qs], d.rs[3 * qs + 1], d.rs[3 * qs + 2]};
    Stencil sq = make_stencil(g, rq);
    double W = corner_weight(sq, k2);
    F[0] += W * d.J[3 * qs];
    F[1] += W * d.J[3 * qs + 1];
    F[2] += W * d.J[3 * qs + 2];
  }
  const size_t N = (size_t)g.N;
  T* Fr = (T*)d.force + (size_t)3 * R.node_off;
  Fr[n] = (T)F[0];
  Fr[N + n] = (T)F[1];
  Fr[2 * N + n] = (T)F[2];
  int s = atomicAdd(&d.ctrl->touched, 1u);
  d.touched[s] = make_int2(rep, n);
}

// Spreading fused with the LB update of the node it writes: the owner of a
// node (see k_spread) sums its force, stores it, and updates the node at
// once -- the same operations as k_spread followed by k_lb_forced.
template <typename T, bool DEV>
__global__ void k_spread_lb(const T* __restrict__ A, T* __restrict__ B, Dev d, int nslots) {
  int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= 8 * nslots) return;
  int slot = e >> 3, k = e & 7;
  const int rep = d.slot_rep[slot];
  const Rep& R = d.reps[rep];
  const int p = slot - R.slot_off;
  if (p >= R.mp.nb) return;
  const Geom& g = R.g;
  const uint8_t* fr = d.flags + R.node_off;
  double rp[3] = {d.rs[3 * slot], d.rs[3 * slot + 1], d.rs[3 * slot + 2]};
  Stencil st = make_stencil(g, rp);
  if (!corner_used(g, st, k)) return;
  int n = (int)corner_node(g, st, k);
  if (fr[n] & F_SOLID) return;
  int nz_ = n / g.nxy, rem = n - nz_ * g.nxy, ny_ = rem / g.nx, nx_ = rem - ny_ * g.nx;
  int keys[MAXCONTRIB];
  int cnt = 0;
  bool overflow = false;
  for (int k2 = 0; k2 < 8; ++k2) {
    int bx = nx_ - (k2 & 1); if (bx < 0) bx += g.nx;
    int by = ny_ - ((k2 >> 1) & 1); if (by < 0) by += g.ny;
    int bz = nz_ - ((k2 >> 2) & 1); if (bz < 0) bz += g.nz;
    int cell = bx + g.nx * (by + g.ny * bz);
    for (int q = d.head[R.node_off + cell]; q >= 0; q = d.next[q]) {
      if (g.ngp) {
        // with the nearest-grid-point transfer only q's nearest node counts
        const Stencil sq = make_stencil(g, &d.rs[3 * q]);
        if (!corner_used(g, sq, k2)) continue;
      }
      int key = (q - R.slot_off) * 8 + k2;
      if (cnt < MAXCONTRIB) {
        int j = cnt++;
        while (j > 0 && keys[j - 1] > key) { keys[j] = keys[j - 1]; --j; }
        keys[j] = key;
      } else {
        overflow = true;
      }
    }
  }
  if (overflow) { atomicOr(&d.ctrl->err, E_SPREAD); }
  if (keys[0] != p * 8 + k) return;   // not the owner of node n
  double F[3] = {0.0, 0.0, 0.0};
  for (int j = 0; j < cnt; ++j) {
    int qs = R.slot_off + (keys[j] >> 3), k2 = keys[j] & 7;
    double rq[3] = {d.rs[3 * qs], d.rs[3 * qs + 1], d.rs[3 * qs + 2]};
    Stencil sq = make_stencil(g, rq);
    double W = corner_weight(sq, k2);
    F[0] += W * d.J[3 * qs];
    F[1] += W * d.J[3 * qs + 1];
    F[2] += W * d.J[3 * qs + 2];
  }
  const size_t N = (size_t)g.N;
  T* Fr = (T*)d.force + (size_t)3 * R.node_off;
  Fr[n] = (T)F[0];
  Fr[N + n] = (T)F[1];
  Fr[2 * N + n] = (T)F[2];
  int s = atomicAdd(&d.ctrl->touched, 1u);
  d.touched[s] = make_int2(rep, n);
  const long no = R.node_off;
  lb_node<T, DEV>(A + (size_t)Q * no, B + (size_t)Q * no, fr, Fr, R.lp, d.ctrl, n, fr[n]);
}

// End of a coupled step: clear the forced bits, empty the node lists, note
// replicas with a bead still on the cis side of the wall.
__global__ void k_step_end(Dev d, int nslots, int maxlist) {
  int k = blockIdx.x * blockDim.x + threadIdx.x;
  int nt = (int)d.ctrl->touched;
  if (k < nt && k < maxlist) {
    int2 e = d.touched[k];
    uint8_t* f = d.flags + d.reps[e.x].node_off + e.y;
    *f = *f & (uint8_t)~F_FORCED;
  }
  if (k < nslots) {
    const int rep = d.slot_rep[k];
    const Rep& R = d.reps[rep];
    if (k - R.slot_off < R.mp.nb) {
      d.head[R.node_off + d.base[k]] = -1;
      if (R.g.wall_axis >= 0 && !(d.r[3 * k + R.g.wall_axis] > (double)R.g.wall_pos)) d.notdone[rep] = 1u;
    }
  }
}
// Advance the step counter; record the translocation step of replicas whose
// whole chain is past the wall plane for the first time.  One block.
__global__ void k_step_tick(Dev d, int nrep, int with_beads) {
  const uint64_t next = d.ctrl->step + 1u;
  for (int r = threadIdx.x; r < nrep && with_beads; r += blockDim.x) {
    const Rep& R = d.reps[r];
    if (R.g.wall_axis >= 0 && R.mp.nb > 0 && d.notdone[r] == 0u && d.tX[r] < 0) d.tX[r] = (int64_t)next;
    d.notdone[r] = 0u;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    d.ctrl->forced_total += d.ctrl->touched;
    d.ctrl->touched = 0u;
    d.ctrl->step = next;
  }
}

// ---------------------------------------------------------------------------
// Fluid reductions (mass deviation and momentum) in FP64: one partial per
// tile, then per replica the partials are summed in a fixed order.
// ---------------------------------------------------------------------------
template <typename T, bool DEV>
__global__ __launch_bounds__(256) void k_fluid_sums(const T* __restrict__ A, Dev d, double* __restrict__ part) {
  constexpr int tile_nodes = OBS_TILE;
  __shared__ double sh[4][256];
  const Tile tl = d.otiles[blockIdx.x];
  const Rep& R = d.reps[tl.rep];
  const size_t N = (size_t)R.lp.N;
  const T* Ar = A + (size_t)Q * R.node_off;
  const uint8_t* fr = d.flags + R.node_off;
  const int end = min(tl.start + tile_nodes, R.lp.N);
  double s[4] = {0.0, 0.0, 0.0, 0.0};
  for (int c = tl.start + (int)threadIdx.x; c < end; c += blockDim.x) {
    if (fr[c] & F_SOLID) continue;
    double f[Q];
#pragma unroll
    for (int i = 0; i < Q; ++i) f[i] = (double)Ar[(size_t)i * N + c] - (DEV ? 0.0 : wgt(i));
    double m = 0.0;
#pragma unroll
    for (int i = 0; i < Q; ++i) m += f[i];
    s[0] += m;
    s[1] += f[1] - f[2] + f[7] - f[8] + f[9] - f[10] + f[11] - f[12] + f[13] - f[14];
    s[2] += f[3] - f[4] + f[7] - f[8] - f[9] + f[10] + f[15] - f[16] + f[17] - f[18];
    s[3] += f[5] - f[6] + f[11] - f[12] - f[13] + f[14] + f[15] - f[16] - f[17] + f[18];
  }
  for (int a = 0; a < 4; ++a) sh[a][threadIdx.x] = s[a];
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w)
      for (int a = 0; a < 4; ++a) sh[a][threadIdx.x] += sh[a][threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x < 4) part[4 * (size_t)blockIdx.x + threadIdx.x] = sh[threadIdx.x][0];
}

// Block-wide sum of NT values (fixed tree order); every thread gets it.
template <int NT = 256>
__device__ inline double block_sum(double v, double* sh) {
  int t = threadIdx.x;
  __syncthreads();
  sh[t] = v;
  __syncthreads();
  for (int w = NT / 2; w > 0; w >>= 1) {
    if (t < w) sh[t] += sh[t + w];
    __syncthreads();
  }
  double r = sh[0];
  __syncthreads();
  return r;
}

// Observables of replica blockIdx.x (one block of 256 threads per replica),
// out[NOBS * r + k] in the order documented in lbmd.h, for the groups in
// mask (bit 0: fluid sums from part, 1: bead quantities, 2: wall ledgers,
// 3: step count); other entries are not written.
__global__ __launch_bounds__(256) void k_observables(Dev d, double* __restrict__ out, int mask,
                                                     const double* __restrict__ part) {
  __shared__ double sh[256];
  const int rep = blockIdx.x;
  const Rep& R = d.reps[rep];
  const Geom& g = R.g;
  const MdParams& P = R.mp;
  const int t = threadIdx.x;
  const int nb = P.nb;
  const int so = R.slot_off;
  double* o = out + (size_t)NOBS * rep;
  if (mask & 1) {
    double fl[4] = {0.0, 0.0, 0.0, 0.0};
    for (int k = R.tile_begin + t; k < R.tile_end; k += 256)
      for (int a = 0; a < 4; ++a) fl[a] += part[4 * (size_t)k + a];
    double tot[4];
    for (int a = 0; a < 4; ++a) tot[a] = block_sum(fl[a], sh);
    if (t == 0) {
      o[0] = R.nfluid + tot[0];
      o[1] = tot[1]; o[2] = tot[2]; o[3] = tot[3];
    }
  }
  if (t == 0) {
    if (mask & 4)
      for (int a = 0; a < NLEDGER; ++a) o[16 + a] = d.ledger[NLEDGER * rep + a];
    if (mask & 8) o[22] = (double)d.ctrl->step;
  }
  if (!(mask & 2)) return;   // uniform in the block
  const int an = g.wall_axis >= 0 ? g.wall_axis : 2;
  double acc[14];
  for (int a = 0; a < 14; ++a) acc[a] = 0.0;
  // 0 sum v^2, 1-3 momentum, 4 normal coordinate, 5 translocated, 6 in field,
  // 7 dW_E, 8 dW_H, 9-11 sum of r over translocated beads, 12-13 drag along
  // the normal on the untranslocated and translocated parts
  for (int p = t; p < nb; p += 256) {
    const int s = so + p;
    double v0 = d.v[3 * s], v1 = d.v[3 * s + 1], v2 = d.v[3 * s + 2];
    double rp[3] = {d.r[3 * s], d.r[3 * s + 1], d.r[3 * s + 2]};
    acc[0] += v0 * v0 + v1 * v1 + v2 * v2;
    acc[1] += P.m * v0; acc[2] += P.m * v1; acc[3] += P.m * v2;
    double zn = rp[an];
    acc[4] += zn;
    bool tr = g.wall_axis >= 0 && zn > (double)g.wall_pos;
    if (tr) { acc[5] += 1.0; acc[9] += rp[0]; acc[10] += rp[1]; acc[11] += rp[2]; }
    if (in_field(g, rp)) { acc[6] += 1.0; acc[7] += P.f_drive * d.v[3 * s + an]; }
    acc[8] += P.gamma * (v0 * d.up[3 * s] + v1 * d.up[3 * s + 1] + v2 * d.up[3 * s + 2]);
    acc[tr ? 13 : 12] += P.m * P.gamma * (d.up[3 * s + an] - d.v[3 * s + an]);
  }
  double res[14];
  for (int a = 0; a < 14; ++a) res[a] = block_sum(acc[a], sh);
  const double ntr = res[5], nun = (double)nb - ntr;
  double cu_s[3] = {0.0, 0.0, 0.0};
  for (int p = t; p < nb; p += 256) {
    const int s = so + p;
    bool tr = g.wall_axis >= 0 && d.r[3 * s + an] > (double)g.wall_pos;
    if (!tr) { cu_s[0] += d.r[3 * s]; cu_s[1] += d.r[3 * s + 1]; cu_s[2] += d.r[3 * s + 2]; }
  }
  double ct[3], cu[3];
  for (int a = 0; a < 3; ++a) {
    double su = block_sum(cu_s[a], sh);
    ct[a] = ntr > 0 ? res[9 + a] / ntr : 0.0;
    cu[a] = nun > 0 ? su / nun : 0.0;
  }
  double ru = 0.0, rt = 0.0;
  for (int p = t; p < nb; p += 256) {
    const int s = so + p;
    bool tr = g.wall_axis >= 0 && d.r[3 * s + an] > (double)g.wall_pos;
    double q = 0.0;
    for (int a = 0; a < 3; ++a) { double dd = d.r[3 * s + a] - (tr ? ct[a] : cu[a]); q += dd * dd; }
    if (tr) rt += q; else ru += q;
  }
  ru = block_sum(ru, sh);
  rt = block_sum(rt, sh);
  if (t == 0) {
    o[4] = nb > 0 ? P.m * res[0] / (3.0 * nb) : 0.0;
    o[5] = res[1]; o[6] = res[2]; o[7] = res[3];
    o[8] = nb > 0 ? res[4] / nb : 0.0;
    o[9] = nb > 0 ? ntr / nb : 0.0;
    o[10] = res[6];
    double RU = nun > 0 ? sqrt(ru / nun) : 0.0;
    double RT = ntr > 0 ? sqrt(rt / ntr) : 0.0;
    o[11] = RU; o[12] = RT;
    o[13] = pow(pow(RT, 0.6) + pow(RU, 0.6), 1.0 / 0.6);
    o[14] = res[8]; o[15] = res[7];
    o[23] = res[12]; o[24] = res[13];
  }
}

// ---------------------------------------------------------------------------
// Wall momentum ledgers (the momentum the wall takes, for the bead-fluid
// momentum balance of Sec. 2, Eq. (momentum_cons), with walls).
// Bounce-back: the population f_opp(i)(x) that leaves fluid node x towards a
// solid upstream node x - c_i returns as f_i(x), so the wall takes
// 2 f_opp(i)(x) c_opp(i); f from the post-collision array A the step pulls
// from (f = A + w_i in deviation storage).  Block b of the wall-link list
// sums its entries (fixed tree order) into lpart[3 b + a]; k_ledger_sum
// then adds each replica's blocks in a fixed order to its cumulative ledger.
// ---------------------------------------------------------------------------
template <typename T, bool DEV>
__global__ __launch_bounds__(LEDGER_BLOCK) void k_ledger_bb(const T* __restrict__ A, Dev d) {
  __shared__ double sh[LEDGER_BLOCK];
  const WallLink e = d.wlinks[(size_t)blockIdx.x * LEDGER_BLOCK + threadIdx.x];
  double s[3] = {0.0, 0.0, 0.0};
  if (e.mask) {
    const Rep& R = d.reps[e.rep];
    const size_t N = (size_t)R.lp.N;
    const T* Ar = A + (size_t)Q * R.node_off;
#pragma unroll
    for (int i = 1; i < Q; ++i) {
      if (!((e.mask >> i) & 1u)) continue;
      const int o = opp(i);
      double f = (double)Ar[(size_t)o * N + (size_t)e.node];
      if (DEV) f += wgt(o);
      const double f2 = 2.0 * f;
      s[0] += f2 * (double)cx(o);
      s[1] += f2 * (double)cy(o);
      s[2] += f2 * (double)cz(o);
    }
  }
  for (int a = 0; a < 3; ++a) {
    const double v = block_sum(s[a], sh);
    if (threadIdx.x == 0) d.lpart[3 * (size_t)blockIdx.x + a] = v;
  }
}

// One workgroup per replica: the step's bounce-back momentum, the replica's
// block sums added in a fixed order (strided per thread, then a tree), added
// to its ledger.
__global__ __launch_bounds__(256) void k_ledger_sum(Dev d) {
  __shared__ double sh[256];
  const Rep& R = d.reps[blockIdx.x];
  double s[3] = {0.0, 0.0, 0.0};
  for (int b = R.wl_begin + (int)threadIdx.x; b < R.wl_end; b += 256)
    for (int a = 0; a < 3; ++a) s[a] += d.lpart[3 * (size_t)b + a];
  for (int a = 0; a < 3; ++a) {
    const double v = block_sum(s[a], sh);
    if (threadIdx.x == 0) d.ledger[NLEDGER * blockIdx.x + a] += v;
  }
}

// Spread-on-solid: the share W_k J_p of the step's impulse that the
// spreading drops because corner k of bead p is solid.  One thread per bead
// slot writes its share (corners in order) to lsp; k_ledger_sp_sum then adds
// each replica's beads in a fixed order (strided per thread, then a tree).
__global__ void k_ledger_sp(Dev d, int nslots) {
  const int slot = blockIdx.x * blockDim.x + threadIdx.x;
  if (slot < nslots) ledger_sp_share(d, slot);
}

__global__ __launch_bounds__(1024) void k_ledger_sp_sum(Dev d) {
  __shared__ double sh[1024];
  const int rep = blockIdx.x;
  const Rep& R = d.reps[rep];
  double s[3] = {0.0, 0.0, 0.0};
  if (R.g.wall_axis >= 0)
    for (int p = threadIdx.x; p < R.mp.nb; p += 1024)
      for (int a = 0; a < 3; ++a) s[a] += d.lsp[3 * (size_t)(R.slot_off + p) + a];
  for (int a = 0; a < 3; ++a) {
    const double v = block_sum<1024>(s[a], sh);
    if (threadIdx.x == 0) d.ledger[NLEDGER * rep + 3 + a] += v;
  }
}

// ---------------------------------------------------------------------------
// Host launchers
// ---------------------------------------------------------------------------
static inline unsigned blocks_for(long n, int bs) { return (unsigned)((n + bs - 1) / bs); }

template <typename T, bool DEV>
void launch_fill_rest(void* pops, long N, hipStream_t s) {
  hipLaunchKernelGGL((k_fill_rest<T, DEV>), dim3(blocks_for(N, 256)), dim3(256), 0, s, (T*)pops, N);
}
void launch_fill_i32(int* p, long n, int v, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(k_fill_i32, dim3(blocks_for(n, 256)), dim3(256), 0, s, p, n, v);
}
void launch_fill_f64(double* p, long n, double v, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(k_fill_f64, dim3(blocks_for(n, 256)), dim3(256), 0, s, p, n, v);
}

template <typename T, bool DEV, bool FL>
static void launch_lb_u(const void* A, void* B, const Dev& d, int ntiles, int tile_nodes, int gsz, size_t lds,
                        int skip_forced, hipStream_t s) {
  const int per = tile_nodes / 256;         // nodes per thread and tile
  if (per >= 4)
    hipLaunchKernelGGL((k_lb<T, DEV, 4, FL>), dim3((unsigned)gsz), dim3(256), lds, s, (const T*)A, (T*)B, d.tiles,
                       d.reps, d.flags, (const T*)d.force, d.ctrl, ntiles, tile_nodes, skip_forced);
  else if (per >= 2)
    hipLaunchKernelGGL((k_lb<T, DEV, 2, FL>), dim3((unsigned)gsz), dim3(256), lds, s, (const T*)A, (T*)B, d.tiles,
                       d.reps, d.flags, (const T*)d.force, d.ctrl, ntiles, tile_nodes, skip_forced);
  else
    hipLaunchKernelGGL((k_lb<T, DEV, 1, FL>), dim3((unsigned)gsz), dim3(256), lds, s, (const T*)A, (T*)B, d.tiles,
                       d.reps, d.flags, (const T*)d.force, d.ctrl, ntiles, tile_nodes, skip_forced);
}

template <typename T, bool DEV>
void launch_lb(const void* A, void* B, const Dev& d, int ntiles, int tile_nodes, int grid, int cap, int skip_forced,
               bool fluct, hipStream_t s) {
  int gsz = (grid > 0 && grid < ntiles) ? grid : ntiles;
  // LDS the kernel does not use, reserved so that at most `cap` sweep
  // workgroups share a CU
  const size_t lds = cap > 0 ? (size_t)((LDS_PER_CU - LDS_KEEP) / cap) & ~(size_t)1023 : 0;
  if (fluct) launch_lb_u<T, DEV, true>(A, B, d, ntiles, tile_nodes, gsz, lds, skip_forced, s);
  else launch_lb_u<T, DEV, false>(A, B, d, ntiles, tile_nodes, gsz, lds, skip_forced, s);
}

template <typename T, bool DEV>
void launch_lb_forced(const void* A, void* B, const Dev& d, int maxlist, hipStream_t s) {
  if (maxlist > 0)
    hipLaunchKernelGGL((k_lb_forced<T, DEV>), dim3(blocks_for(maxlist, 64)), dim3(64), 0, s, (const T*)A, (T*)B, d,
                       maxlist);
}

template <typename T, bool DEV>
void launch_gather(const void* A, const Dev& d, int nslots, int start, hipStream_t s) {
  if (nslots > 0)
    hipLaunchKernelGGL((k_gather<T, DEV>), dim3(blocks_for(8L * nslots, 64)), dim3(64), 0, s, (const T*)A, d,
                       nslots, start);
}

void launch_bead_prep(const Dev& d, int nslots, hipStream_t s) {
  if (nslots > 0) hipLaunchKernelGGL(k_bead_prep, dim3(blocks_for(nslots, 64)), dim3(64), 0, s, d, nslots);
}

template <typename T>
void launch_spread(const Dev& d, int nslots, hipStream_t s) {
  if (nslots > 0) hipLaunchKernelGGL((k_spread<T>), dim3(blocks_for(8L * nslots, 64)), dim3(64), 0, s, d, nslots);
}

template <typename T, bool DEV>
void launch_spread_lb(const void* A, void* B, const Dev& d, int nslots, hipStream_t s) {
  if (nslots > 0)
    hipLaunchKernelGGL((k_spread_lb<T, DEV>), dim3(blocks_for(8L * nslots, 64)), dim3(64), 0, s, (const T*)A,
                       (T*)B, d, nslots);
}

void launch_step_end(const Dev& d, int nslots, int maxlist, int nrep, hipStream_t s) {
  long n = nslots > maxlist ? nslots : maxlist;
  if (n > 0) hipLaunchKernelGGL(k_step_end, dim3(blocks_for(n, 256)), dim3(256), 0, s, d, nslots, maxlist);
  hipLaunchKernelGGL(k_step_tick, dim3(1), dim3(256), 0, s, d, nrep, nslots > 0 ? 1 : 0);
}

template <typename T, bool DEV>
void launch_observables(const void* A, const Dev& d, int n_otiles, int nrep, double* out, int mask, double* part,
                        hipStream_t s) {
  if ((mask & 1) && n_otiles > 0)
    hipLaunchKernelGGL((k_fluid_sums<T, DEV>), dim3((unsigned)n_otiles), dim3(256), 0, s, (const T*)A, d, part);
  hipLaunchKernelGGL(k_observables, dim3((unsigned)nrep), dim3(256), 0, s, d, out, mask, (const double*)part);
}

template <typename T, bool DEV>
void launch_ledger_bb(const void* A, const Dev& d, int nblk, int nrep, hipStream_t s) {
  if (nblk <= 0) return;
  hipLaunchKernelGGL((k_ledger_bb<T, DEV>), dim3((unsigned)nblk), dim3(LEDGER_BLOCK), 0, s, (const T*)A, d);
  hipLaunchKernelGGL(k_ledger_sum, dim3((unsigned)nrep), dim3(256), 0, s, d);
}

void launch_ledger_sp(const Dev& d, int nslots, int nrep, hipStream_t s) {
  if (nslots <= 0) return;
  hipLaunchKernelGGL(k_ledger_sp, dim3(blocks_for(nslots, 64)), dim3(64), 0, s, d, nslots);
  hipLaunchKernelGGL(k_ledger_sp_sum, dim3((unsigned)nrep), dim3(1024), 0, s, d);
}

template void launch_fill_rest<double, false>(void*, long, hipStream_t);
template void launch_fill_rest<float, true>(void*, long, hipStream_t);
template void launch_lb<double, false>(const void*, void*, const Dev&, int, int, int, int, int, bool, hipStream_t);
template void launch_lb<float, true>(const void*, void*, const Dev&, int, int, int, int, int, bool, hipStream_t);
template void launch_lb_forced<double, false>(const void*, void*, const Dev&, int, hipStream_t);
template void launch_lb_forced<float, true>(const void*, void*, const Dev&, int, hipStream_t);
template void launch_gather<double, false>(const void*, const Dev&, int, int, hipStream_t);
template void launch_gather<float, true>(const void*, const Dev&, int, int, hipStream_t);
template void launch_spread<double>(const Dev&, int, hipStream_t);
template void launch_spread_lb<double, false>(const void*, void*, const Dev&, int, hipStream_t);
template void launch_spread_lb<float, true>(const void*, void*, const Dev&, int, hipStream_t);
template void launch_spread<float>(const Dev&, int, hipStream_t);
template void launch_observables<double, false>(const void*, const Dev&, int, int, double*, int, double*,
                                                hipStream_t);
template void launch_observables<float, true>(const void*, const Dev&, int, int, double*, int, double*, hipStream_t);
template void launch_ledger_bb<double, false>(const void*, const Dev&, int, int, hipStream_t);
template void launch_ledger_bb<float, true>(const void*, const Dev&, int, int, hipStream_t);

}  // namespace lbmd
