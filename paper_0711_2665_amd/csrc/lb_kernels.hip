// lb_kernels.hip -- lattice side of the coupled step: the fused
// stream + collide sweep, the bead gather (fluid velocity at the beads), the
// deterministic spreading of the bead reaction onto the lattice, and the
// fluid reductions.
#include "lbmd_kernels.h"

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
// Neighbour offsets of node c = (x, y, z) with periodic wrap.
// ---------------------------------------------------------------------------
struct Nbr {
  int xm, xp, ym, yp, zm, zp;   // index offsets to x-1, x+1, y-1, ...
  __device__ inline int off(int dx, int dy, int dz) const {
    return (dx < 0 ? xm : (dx > 0 ? xp : 0)) + (dy < 0 ? ym : (dy > 0 ? yp : 0)) + (dz < 0 ? zm : (dz > 0 ? zp : 0));
  }
};
__device__ inline Nbr make_nbr(const LbParams& p, int x, int y, int z) {
  Nbr n;
  n.xm = (x > 0) ? -1 : p.nx - 1;
  n.xp = (x < p.nx - 1) ? 1 : -(p.nx - 1);
  n.ym = (y > 0) ? -p.nx : p.nx * (p.ny - 1);
  n.yp = (y < p.ny - 1) ? p.nx : -p.nx * (p.ny - 1);
  n.zm = (z > 0) ? -p.nxy : p.nxy * (p.nz - 1);
  n.zp = (z < p.nz - 1) ? p.nxy : -p.nxy * (p.nz - 1);
  return n;
}

// Population store of the sweep: written once per step and read only in the
// next step, so it bypasses the caches (non-temporal).
template <typename T>
__device__ inline void store_pop(T* ptr, T v) {
  __builtin_nontemporal_store(v, ptr);
}

// Post-streaming populations at node c: f_i(x) = A_i(x - c_i), or
// A_opp(i)(x) when x - c_i is solid (halfway bounce-back).  Nodes away from
// walls take a straight run of 19 independent loads; next to a wall the 19
// upstream flags are loaded first and the addresses selected without
// branches, so the population loads are again issued together.
template <typename T>
__device__ inline void pull(const T* __restrict__ A, const uint8_t* __restrict__ flags, const LbParams& p, int c,
                            uint8_t fl, const Nbr& nb, T f[Q]) {
  const size_t N = (size_t)p.N;
  if (!(fl & F_NEAR)) {
#pragma unroll
    for (int i = 0; i < Q; ++i) f[i] = A[(size_t)i * N + (size_t)(c + nb.off(-cx(i), -cy(i), -cz(i)))];
  } else {
    uint8_t sf[Q];
#pragma unroll
    for (int i = 0; i < Q; ++i) sf[i] = flags[c + nb.off(-cx(i), -cy(i), -cz(i))];
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      size_t src = (size_t)i * N + (size_t)(c + nb.off(-cx(i), -cy(i), -cz(i)));
      size_t ref = (size_t)opp(i) * N + (size_t)c;
      f[i] = A[(sf[i] & F_SOLID) ? ref : src];
    }
  }
}

// FP64 moments in the order of the definition: rho = sum_i f_i,
// j_a = sum_i f_i c_ia (terms with c_ia = 0 add exact zeros and are omitted).
__device__ inline void moments64(const double f[Q], double& rho, double& ux, double& uy, double& uz) {
  rho = 0.0;
#pragma unroll
  for (int i = 0; i < Q; ++i) rho += f[i];
  double jx = f[1] - f[2] + f[7] - f[8] + f[9] - f[10] + f[11] - f[12] + f[13] - f[14];
  double jy = f[3] - f[4] + f[7] - f[8] - f[9] + f[10] + f[15] - f[16] + f[17] - f[18];
  double jz = f[5] - f[6] + f[11] - f[12] - f[13] + f[14] + f[15] - f[16] - f[17] + f[18];
  ux = jx / rho; uy = jy / rho; uz = jz / rho;
}

// c_i . v with the zero components omitted, in x, y, z order.
template <typename R>
__device__ inline R cdot(int i, R vx, R vy, R vz) {
  switch (i) {
    case 0: return (R)0;
    case 1: return vx;
    case 2: return -vx;
    case 3: return vy;
    case 4: return -vy;
    case 5: return vz;
    case 6: return -vz;
    case 7: return vx + vy;
    case 8: return -vx - vy;
    case 9: return vx - vy;
    case 10: return -vx + vy;
    case 11: return vx + vz;
    case 12: return -vx - vz;
    case 13: return vx - vz;
    case 14: return -vx + vz;
    case 15: return vy + vz;
    case 16: return -vy - vz;
    case 17: return vy - vz;
    default: return -vy + vz;
  }
}

// ---------------------------------------------------------------------------
// K1: fused stream + collide (Sec. 2, Eq. (lbe2) as a BGK relaxation with the
// source S_i = 3 w_i F.c_i) of one fluid node c.
// ---------------------------------------------------------------------------
// BGK collision with the source term of one fluid node (index c, flags fl)
// from its post-streaming populations f; writes f* to out.
template <typename T, bool DEV>
__device__ inline void collide_node(const T f[Q], T out[Q], const T* __restrict__ force, const LbParams& p,
                                    Ctrl* __restrict__ ctrl, int c, uint8_t fl) {
  const size_t N = (size_t)p.N;
  if constexpr (!DEV) {
    // FP64: f* = f - omega (f - f^eq) + 3 w_i (F + g).c_i, f^eq =
    // w_i rho (1 + 3 cu + 4.5 cu^2 - 1.5 u.u)
    double rho, ux, uy, uz;
    moments64(f, rho, ux, uy, uz);
    if (!(rho > 0.0)) atomicOr(&ctrl->err, E_DENSITY);
    double usq = ux * ux + uy * uy + uz * uz;
    double Fx = p.g[0], Fy = p.g[1], Fz = p.g[2];
    if (fl & F_FORCED) {
      Fx = (double)force[c] + p.g[0];
      Fy = (double)force[N + c] + p.g[1];
      Fz = (double)force[2 * N + c] + p.g[2];
    }
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      double cu = cdot<double>(i, ux, uy, uz);
      double fe = wgt(i) * rho * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * usq);
      double src = (3.0 * wgt(i)) * cdot<double>(i, Fx, Fy, Fz);
      out[i] = (T)(f[i] - p.omega * (f[i] - fe) + src);
    }
  } else {
    // FP32 deviation storage: g_i = f_i - w_i; drho = sum g, j = sum g c;
    // g^eq = w_i (drho + rho (3 cu + 4.5 cu^2 - 1.5 u.u)).
    float drho = 0.f;
#pragma unroll
    for (int i = 0; i < Q; ++i) drho += (float)f[i];
    float jx = (float)(f[1] - f[2] + f[7] - f[8] + f[9] - f[10] + f[11] - f[12] + f[13] - f[14]);
    float jy = (float)(f[3] - f[4] + f[7] - f[8] - f[9] + f[10] + f[15] - f[16] + f[17] - f[18]);
    float jz = (float)(f[5] - f[6] + f[11] - f[12] - f[13] + f[14] + f[15] - f[16] - f[17] + f[18]);
    float rho = 1.f + drho;
    if (!(rho > 0.f)) atomicOr(&ctrl->err, E_DENSITY);
    float ir = 1.f / rho;
    float ux = jx * ir, uy = jy * ir, uz = jz * ir;
    float usq = ux * ux + uy * uy + uz * uz;
    float om = (float)p.omega;
    bool forced = (fl & F_FORCED) != 0;
    float Fx = (float)p.g[0], Fy = (float)p.g[1], Fz = (float)p.g[2];
    if (forced) {
      Fx += (float)force[c];
      Fy += (float)force[N + c];
      Fz += (float)force[2 * N + c];
    }
    bool src_on = forced || p.has_g;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      float cu = cdot<float>(i, ux, uy, uz);
      float w = (float)wgt(i);
      float ge = w * (drho + rho * (3.f * cu + 4.5f * cu * cu - 1.5f * usq));
      float o = (float)f[i] - om * ((float)f[i] - ge);
      if (src_on) o += (3.f * w) * cdot<float>(i, Fx, Fy, Fz);
      out[i] = (T)o;
    }
  }
}

// Stream + collide one fluid node at (x, y, z), index c.
template <typename T, bool DEV>
__device__ inline void lb_node_xyz(const T* __restrict__ A, T* __restrict__ B, const uint8_t* __restrict__ flags,
                                   const T* __restrict__ force, const LbParams& p, Ctrl* __restrict__ ctrl, int c,
                                   uint8_t fl, int x, int y, int z) {
  Nbr nb = make_nbr(p, x, y, z);
  T f[Q];
  pull<T>(A, flags, p, c, fl, nb, f);
  collide_node<T, DEV>(f, f, force, p, ctrl, c, fl);
  const size_t N = (size_t)p.N;
#pragma unroll
  for (int i = 0; i < Q; ++i) store_pop(&B[(size_t)i * N + c], f[i]);
}

template <typename T, bool DEV>
__device__ inline void lb_node(const T* __restrict__ A, T* __restrict__ B, const uint8_t* __restrict__ flags,
                               const T* __restrict__ force, const LbParams& p, Ctrl* __restrict__ ctrl, int c,
                               uint8_t fl) {
  int x = c % p.nx;
  int yz = c / p.nx;
  int y = yz % p.ny;
  int z = yz / p.ny;
  lb_node_xyz<T, DEV>(A, B, flags, force, p, ctrl, c, fl, x, y, z);
}

// Sweep over all nodes; solid nodes are skipped, and so are nodes carrying a
// bead force when skip_forced is set (those are updated by k_lb_forced once
// the force is known).
template <typename T, bool DEV>
__global__ __launch_bounds__(256) void k_lb(const T* __restrict__ A, T* __restrict__ B,
                                            const uint8_t* __restrict__ flags, const T* __restrict__ force,
                                            LbParams p, Ctrl* __restrict__ ctrl, int skip_forced) {
  int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= p.N) return;
  uint8_t fl = flags[c];
  if (fl & F_SOLID) return;
  if (skip_forced && (fl & F_FORCED)) return;
  lb_node<T, DEV>(A, B, flags, force, p, ctrl, c, fl);
}

// The nodes that carry a bead force this step (the list written by the
// spreading kernel).
template <typename T, bool DEV>
__global__ __launch_bounds__(64) void k_lb_forced(const T* __restrict__ A, T* __restrict__ B,
                                                  const uint8_t* __restrict__ flags, const T* __restrict__ force,
                                                  LbParams p, Ctrl* __restrict__ ctrl,
                                                  const int* __restrict__ touched, int maxlist) {
  int k = blockIdx.x * blockDim.x + threadIdx.x;
  int nt = (int)ctrl->touched;
  if (k >= nt || k >= maxlist) return;
  int c = touched[k];
  uint8_t fl = flags[c];
  lb_node<T, DEV>(A, B, flags, force, p, ctrl, c, fl);
}

// ---------------------------------------------------------------------------
// Fluid velocity at node c from the pulled populations (zero at solid nodes),
// accumulated in FP64.
// ---------------------------------------------------------------------------
template <typename T, bool DEV>
__device__ inline void node_velocity(const T* __restrict__ A, const uint8_t* __restrict__ flags, const LbParams& p,
                                     int c, double u[3]) {
  uint8_t fl = flags[c];
  if (fl & F_SOLID) { u[0] = u[1] = u[2] = 0.0; return; }
  int x = c % p.nx, yz = c / p.nx, y = yz % p.ny, z = yz / p.ny;
  Nbr nb = make_nbr(p, x, y, z);
  T ft[Q];
  pull<T>(A, flags, p, c, fl, nb, ft);
  double f[Q];
#pragma unroll
  for (int i = 0; i < Q; ++i) f[i] = (double)ft[i];
  if constexpr (!DEV) {
    double rho;
    moments64(f, rho, u[0], u[1], u[2]);
  } else {
    double drho = 0.0;
#pragma unroll
    for (int i = 0; i < Q; ++i) drho += f[i];
    double jx = f[1] - f[2] + f[7] - f[8] + f[9] - f[10] + f[11] - f[12] + f[13] - f[14];
    double jy = f[3] - f[4] + f[7] - f[8] - f[9] + f[10] + f[15] - f[16] + f[17] - f[18];
    double jz = f[5] - f[6] + f[11] - f[12] - f[13] + f[14] + f[15] - f[16] - f[17] + f[18];
    double rho = 1.0 + drho;
    u[0] = jx / rho; u[1] = jy / rho; u[2] = jz / rho;
  }
}

// ---------------------------------------------------------------------------
// Start of a coupled step: remember r(n), link every bead into the list of
// its base node, clear J.
// ---------------------------------------------------------------------------
__global__ void k_bead_prep(BeadPtrs b, Geom g, int nb, int* __restrict__ head, int* __restrict__ next,
                            int* __restrict__ base, uint8_t* __restrict__ flags) {
  int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= nb) return;
  double rp[3] = {b.r[3 * p], b.r[3 * p + 1], b.r[3 * p + 2]};
  Stencil st = make_stencil(g, rp);
  int cell = st.b[0] + g.nx * (st.b[1] + g.ny * st.b[2]);
#pragma unroll
  for (int a = 0; a < 3; ++a) { b.rs[3 * p + a] = rp[a]; b.J[3 * p + a] = 0.0; }
  base[p] = cell;
  next[p] = atomicExch(&head[cell], p);
  // the 8 stencil nodes of r(n) receive bead force this step (solid ones are
  // dropped by the spreading); every writer of a node stores the same byte
  for (int k = 0; k < 8; ++k) {
    int n = (int)corner_node(g, st, k);
    uint8_t fl = flags[n];
    if (!(fl & F_SOLID)) flags[n] = fl | F_FORCED;
  }
}

// ---------------------------------------------------------------------------
// K2: u_p = sum_k W_k u(node_k) at r(n) (trilinear).
// ---------------------------------------------------------------------------
template <typename T, bool DEV>
__global__ void k_gather(const T* __restrict__ A, const uint8_t* __restrict__ flags, LbParams p, Geom g, BeadPtrs b,
                         int nb) {
  int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= nb) return;
  double rp[3] = {b.rs[3 * q], b.rs[3 * q + 1], b.rs[3 * q + 2]};
  Stencil st = make_stencil(g, rp);
  double acc[3] = {0.0, 0.0, 0.0};
  for (int k = 0; k < 8; ++k) {
    int node = (int)corner_node(g, st, k);
    double W = corner_weight(st, k);
    double u[3];
    node_velocity<T, DEV>(A, flags, p, node, u);
    acc[0] += W * u[0]; acc[1] += W * u[1]; acc[2] += W * u[2];
  }
  b.up[3 * q] = acc[0]; b.up[3 * q + 1] = acc[1]; b.up[3 * q + 2] = acc[2];
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
__global__ void k_spread(BeadPtrs b, Geom g, int nb, const int* __restrict__ head, const int* __restrict__ next,
                         uint8_t* __restrict__ flags, T* __restrict__ force, int* __restrict__ touched,
                         Ctrl* __restrict__ ctrl) {
  int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= 8 * nb) return;
  int p = e >> 3, k = e & 7;
  double rp[3] = {b.rs[3 * p], b.rs[3 * p + 1], b.rs[3 * p + 2]};
  Stencil st = make_stencil(g, rp);
  int n = (int)corner_node(g, st, k);
  if (flags[n] & F_SOLID) return;
  int nz_ = n / g.nxy, rem = n - nz_ * g.nxy, ny_ = rem / g.nx, nx_ = rem - ny_ * g.nx;
  // contributors as keys q*8 + k'
  int keys[MAXCONTRIB];
  int cnt = 0;
  bool overflow = false;
  for (int k2 = 0; k2 < 8; ++k2) {
    int bx = nx_ - (k2 & 1); if (bx < 0) bx += g.nx;
    int by = ny_ - ((k2 >> 1) & 1); if (by < 0) by += g.ny;
    int bz = nz_ - ((k2 >> 2) & 1); if (bz < 0) bz += g.nz;
    int cell = bx + g.nx * (by + g.ny * bz);
    for (int q = head[cell]; q >= 0; q = next[q]) {
      int key = q * 8 + k2;
      if (cnt < MAXCONTRIB) {
        int j = cnt++;
        while (j > 0 && keys[j - 1] > key) { keys[j] = keys[j - 1]; --j; }
        keys[j] = key;
      } else {
        overflow = true;
      }
    }
  }
  if (overflow) { atomicOr(&ctrl->err, E_SPREAD); }
  if (keys[0] != p * 8 + k) return;   // not the owner of node n
  double F[3] = {0.0, 0.0, 0.0};
  for (int j = 0; j < cnt; ++j) {
    int q = keys[j] >> 3, k2 = keys[j] & 7;
    double rq[3] = {b.rs[3 * q], b.rs[3 * q + 1], b.rs[3 * q + 2]};
    Stencil sq = make_stencil(g, rq);
    double W = corner_weight(sq, k2);
    F[0] += W * b.J[3 * q];
    F[1] += W * b.J[3 * q + 1];
    F[2] += W * b.J[3 * q + 2];
  }
  const size_t N = (size_t)g.N;
  force[n] = (T)F[0];
  force[N + n] = (T)F[1];
  force[2 * N + n] = (T)F[2];
  int slot = atomicAdd(&ctrl->touched, 1u);
  touched[slot] = n;
}

// End of a coupled step: clear the forced bits, empty the node lists,
// advance the step counter.
__global__ void k_step_end(int nb, const int* __restrict__ base, int* __restrict__ head,
                           const int* __restrict__ touched, uint8_t* __restrict__ flags, Ctrl* __restrict__ ctrl,
                           int advance) {
  int k = blockIdx.x * blockDim.x + threadIdx.x;
  int nt = (int)ctrl->touched;
  if (k < nt) { int n = touched[k]; flags[n] = flags[n] & (uint8_t)~F_FORCED; }
  if (k < nb) head[base[k]] = -1;
}
__global__ void k_step_tick(Ctrl* __restrict__ ctrl, int advance) {
  ctrl->touched = 0u;
  ctrl->step += (uint64_t)advance;
}

// ---------------------------------------------------------------------------
// Fluid reductions (mass deviation and momentum) in FP64: block partials,
// then one block sums the partials in a fixed order.
// ---------------------------------------------------------------------------
template <typename T, bool DEV>
__global__ __launch_bounds__(256) void k_fluid_sums(const T* __restrict__ A, const uint8_t* __restrict__ flags,
                                                    long N, double* __restrict__ part) {
  __shared__ double sh[4][256];
  double s[4] = {0.0, 0.0, 0.0, 0.0};
  for (long c = (long)blockIdx.x * blockDim.x + threadIdx.x; c < N; c += (long)gridDim.x * blockDim.x) {
    if (flags[c] & F_SOLID) continue;
    double f[Q];
#pragma unroll
    for (int i = 0; i < Q; ++i) f[i] = (double)A[(size_t)i * N + c] - (DEV ? 0.0 : wgt(i));
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
  if (threadIdx.x < 4) part[4 * blockIdx.x + threadIdx.x] = sh[threadIdx.x][0];
}

// Bead observables + final fluid sums (one block of 256 threads).
__global__ __launch_bounds__(256) void k_observables(const double* __restrict__ part, int nparts, double nfluid,
                                                     BeadPtrs b, int nb, Geom g, MdParams P,
                                                     const Ctrl* __restrict__ ctrl, double* __restrict__ out) {
  __shared__ double sh[16][256];
  int t = threadIdx.x;
  double acc[16];
  for (int a = 0; a < 16; ++a) acc[a] = 0.0;
  for (int k = t; k < nparts; k += 256)
    for (int a = 0; a < 4; ++a) acc[a] += part[4 * k + a];
  int an = g.wall_axis >= 0 ? g.wall_axis : 2;
  // pass 1: kinetic, momentum, normal coordinate, counts, work rates, centres
  for (int p = t; p < nb; p += 256) {
    double v0 = b.v[3 * p], v1 = b.v[3 * p + 1], v2 = b.v[3 * p + 2];
    double rp[3] = {b.r[3 * p], b.r[3 * p + 1], b.r[3 * p + 2]};
    acc[4] += v0 * v0 + v1 * v1 + v2 * v2;
    acc[5] += P.m * v0; acc[6] += P.m * v1; acc[7] += P.m * v2;
    double zn = rp[an];
    acc[8] += zn;
    bool tr = g.wall_axis >= 0 && zn > (double)g.wall_pos;
    acc[9] += tr ? 1.0 : 0.0;
    bool res = in_field(g, rp);
    if (res) { acc[10] += 1.0; acc[15] += P.f_drive * b.v[3 * p + an]; }
    acc[14] += P.gamma * (v0 * b.up[3 * p] + v1 * b.up[3 * p + 1] + v2 * b.up[3 * p + 2]);
    if (tr) { acc[11] += rp[0]; acc[12] += rp[1]; acc[13] += rp[2]; }
  }
  for (int a = 0; a < 16; ++a) sh[a][t] = acc[a];
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (t < w) for (int a = 0; a < 16; ++a) sh[a][t] += sh[a][t + w];
    __syncthreads();
  }
  __shared__ double res[16];
  if (t < 16) res[t] = sh[t][0];
  __syncthreads();
  // centres of the translocated (T) and untranslocated (U) parts
  double ntr = res[9];
  double nun = (double)nb - ntr;
  double ct[3] = {0, 0, 0}, cu[3] = {0, 0, 0};
  double acc2[3] = {0, 0, 0};
  for (int p = t; p < nb; p += 256) {
    bool tr = g.wall_axis >= 0 && b.r[3 * p + an] > (double)g.wall_pos;
    if (!tr) { acc2[0] += b.r[3 * p]; acc2[1] += b.r[3 * p + 1]; acc2[2] += b.r[3 * p + 2]; }
  }
  __syncthreads();
  for (int a = 0; a < 3; ++a) sh[a][t] = acc2[a];
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (t < w) for (int a = 0; a < 3; ++a) sh[a][t] += sh[a][t + w];
    __syncthreads();
  }
  for (int a = 0; a < 3; ++a) {
    ct[a] = ntr > 0 ? res[11 + a] / ntr : 0.0;
    cu[a] = nun > 0 ? sh[a][0] / nun : 0.0;
  }
  __syncthreads();
  double ru = 0.0, rt = 0.0;
  for (int p = t; p < nb; p += 256) {
    bool tr = g.wall_axis >= 0 && b.r[3 * p + an] > (double)g.wall_pos;
    double s = 0.0;
    for (int a = 0; a < 3; ++a) { double d = b.r[3 * p + a] - (tr ? ct[a] : cu[a]); s += d * d; }
    if (tr) rt += s; else ru += s;
  }
  sh[0][t] = ru; sh[1][t] = rt;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (t < w) { sh[0][t] += sh[0][t + w]; sh[1][t] += sh[1][t + w]; }
    __syncthreads();
  }
  if (t == 0) {
    out[0] = nfluid + res[0];
    out[1] = res[1]; out[2] = res[2]; out[3] = res[3];
    out[4] = nb > 0 ? P.m * res[4] / (3.0 * nb) : 0.0;
    out[5] = res[5]; out[6] = res[6]; out[7] = res[7];
    out[8] = nb > 0 ? res[8] / nb : 0.0;
    out[9] = nb > 0 ? ntr / nb : 0.0;
    out[10] = res[10];
    double RU = nun > 0 ? sqrt(sh[0][0] / nun) : 0.0;
    double RT = ntr > 0 ? sqrt(sh[1][0] / ntr) : 0.0;
    out[11] = RU; out[12] = RT;
    out[13] = pow(pow(RT, 0.6) + pow(RU, 0.6), 1.0 / 0.6);
    out[14] = res[14]; out[15] = res[15];
    for (int a = 16; a < 22; ++a) out[a] = __builtin_nan("");
    out[22] = (double)ctrl->step;
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

template <typename T, bool DEV>
void launch_lb(const void* A, void* B, const uint8_t* flags, const void* force, const LbParams& p, Ctrl* ctrl,
               int skip_forced, hipStream_t s) {
  hipLaunchKernelGGL((k_lb<T, DEV>), dim3(blocks_for(p.N, 256)), dim3(256), 0, s, (const T*)A, (T*)B, flags,
                     (const T*)force, p, ctrl, skip_forced);
}

template <typename T, bool DEV>
void launch_lb_forced(const void* A, void* B, const uint8_t* flags, const void* force, const LbParams& p, Ctrl* ctrl,
                      const int* touched, int maxlist, hipStream_t s) {
  if (maxlist > 0)
    hipLaunchKernelGGL((k_lb_forced<T, DEV>), dim3(blocks_for(maxlist, 64)), dim3(64), 0, s, (const T*)A, (T*)B,
                       flags, (const T*)force, p, ctrl, touched, maxlist);
}

template <typename T, bool DEV>
void launch_gather(const void* A, const uint8_t* flags, const LbParams& p, const Geom& g, const BeadPtrs& b, int nb,
                   hipStream_t s) {
  if (nb > 0)
    hipLaunchKernelGGL((k_gather<T, DEV>), dim3(blocks_for(nb, 64)), dim3(64), 0, s, (const T*)A, flags, p, g, b, nb);
}

void launch_bead_prep(const BeadPtrs& b, const Geom& g, int nb, int* head, int* next, int* base, uint8_t* flags,
                      hipStream_t s) {
  if (nb > 0)
    hipLaunchKernelGGL(k_bead_prep, dim3(blocks_for(nb, 64)), dim3(64), 0, s, b, g, nb, head, next, base, flags);
}

template <typename T>
void launch_spread(const BeadPtrs& b, const Geom& g, int nb, const int* head, const int* next, uint8_t* flags,
                   void* force, int* touched, Ctrl* ctrl, hipStream_t s) {
  if (nb > 0)
    hipLaunchKernelGGL((k_spread<T>), dim3(blocks_for(8L * nb, 64)), dim3(64), 0, s, b, g, nb, head, next, flags,
                       (T*)force, touched, ctrl);
}

void launch_step_end(int nb, const int* base, int* head, const int* touched, uint8_t* flags, Ctrl* ctrl, int advance,
                     hipStream_t s) {
  if (nb > 0)
    hipLaunchKernelGGL(k_step_end, dim3(blocks_for(8L * nb, 256)), dim3(256), 0, s, nb, base, head, touched, flags,
                       ctrl, advance);
  hipLaunchKernelGGL(k_step_tick, dim3(1), dim3(1), 0, s, ctrl, advance);
}

template <typename T, bool DEV>
void launch_observables(const void* A, const uint8_t* flags, long N, double nfluid, double* part, int nparts,
                        const BeadPtrs& b, int nb, const Geom& g, const MdParams& P, const Ctrl* ctrl, double* out,
                        hipStream_t s) {
  hipLaunchKernelGGL((k_fluid_sums<T, DEV>), dim3(nparts), dim3(256), 0, s, (const T*)A, flags, N, part);
  hipLaunchKernelGGL(k_observables, dim3(1), dim3(256), 0, s, part, nparts, nfluid, b, nb, g, P, ctrl, out);
}

template void launch_fill_rest<double, false>(void*, long, hipStream_t);
template void launch_fill_rest<float, true>(void*, long, hipStream_t);
template void launch_lb<double, false>(const void*, void*, const uint8_t*, const void*, const LbParams&, Ctrl*,
                                       int, hipStream_t);
template void launch_lb<float, true>(const void*, void*, const uint8_t*, const void*, const LbParams&, Ctrl*, int,
                                     hipStream_t);
template void launch_lb_forced<double, false>(const void*, void*, const uint8_t*, const void*, const LbParams&,
                                              Ctrl*, const int*, int, hipStream_t);
template void launch_lb_forced<float, true>(const void*, void*, const uint8_t*, const void*, const LbParams&, Ctrl*,
                                            const int*, int, hipStream_t);
template void launch_gather<double, false>(const void*, const uint8_t*, const LbParams&, const Geom&, const BeadPtrs&,
                                           int, hipStream_t);
template void launch_gather<float, true>(const void*, const uint8_t*, const LbParams&, const Geom&, const BeadPtrs&,
                                         int, hipStream_t);
template void launch_spread<double>(const BeadPtrs&, const Geom&, int, const int*, const int*, uint8_t*, void*, int*,
                                    Ctrl*, hipStream_t);
template void launch_spread<float>(const BeadPtrs&, const Geom&, int, const int*, const int*, uint8_t*, void*, int*,
                                   Ctrl*, hipStream_t);
template void launch_observables<double, false>(const void*, const uint8_t*, long, double, double*, int,
                                                const BeadPtrs&, int, const Geom&, const MdParams&, const Ctrl*,
                                                double*, hipStream_t);
template void launch_observables<float, true>(const void*, const uint8_t*, long, double, double*, int,
                                              const BeadPtrs&, int, const Geom&, const MdParams&, const Ctrl*,
                                              double*, hipStream_t);

}  // namespace lbmd
