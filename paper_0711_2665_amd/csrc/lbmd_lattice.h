// lbmd_lattice.h -- device functions of the lattice update shared by the
// forward sweep and its adjoint: neighbour offsets with periodic wrap, the
// pull of post-streaming populations with halfway bounce-back, moments, the
// BGK collision with source, and the fluid velocity at a node.
#pragma once

#include "lbmd_kernels.h"

namespace lbmd {

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
// BGK collision with the source term (Sec. 2, Eq. (lbe2) read as a relaxation
// with S_i = 3 w_i F.c_i) of one fluid node (index c, flags fl) from its
// post-streaming populations f; writes f* to out (may alias f) and returns
// the node's density.
// ---------------------------------------------------------------------------
template <typename T, bool DEV>
__device__ inline auto collide_node(const T f[Q], T out[Q], const T* __restrict__ force, const LbParams& p,
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
    return rho;
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
    return rho;
  }
}

// ---------------------------------------------------------------------------
// Stochastic term of the fluctuating fluid (Sec. 2, F_i; read in the mode
// formulation of Adhikari et al.): after the collision of node c at LB step
// n, every non-conserved mode k = 4..18 receives sqrt(rho) famp[k-4] r_k and
// the populations f_i += w_i sum_k e_ki (that noise), so mass and momentum
// stay as they are.  The 15 normals r_k come from four Philox-4x32-10 blocks
// with key (fseed, frep) and counters (n, c, b, 1), b = 0..3: uniforms
// (x + 1/2) 2^-32, Box-Muller on the pairs (u0, u1) and (u2, u3), cosine then
// sine.  FP64: double log, sincos and sqrt.  FP32 deviation storage: the
// hardware log2 (through the complement near 1), sqrt and sin/cos of a
// fraction of a turn.
// ---------------------------------------------------------------------------
// -2 ln u in FP32 for the uniform u = (x + 1/2) 2^-32.  Near 1 the FP32 u
// itself is off by up to 2^-25 (it rounds to 1 for the top 2^7 values of x),
// so above 1 - 2^-6 the complement t = 1 - u = (~x + 1/2) 2^-32, which FP32
// holds to its own precision, gives -ln(1 - t) = t + t^2/2 + t^3/3 + t^4/4
// (the next term is below 2^-24 of the sum); below, the hardware log2.
__device__ inline float neg2_log_uniform(uint32_t x) {
  const float s32 = 2.3283064365386963e-10f;     // 2^-32
  const float u = fmaf((float)x, s32, 0.5f * s32);
  const float t = fmaf((float)(~x), s32, 0.5f * s32);
  const float series = 2.0f * (t * fmaf(t, fmaf(t, fmaf(t, 0.25f, 0.33333334f), 0.5f), 1.0f));
  const float m2ln2 = -1.3862943611198906f;       // -2 ln 2: -2 ln u = -2 ln 2 log2 u
  const float hw = m2ln2 * __builtin_amdgcn_logf(u);
  return t <= 0.015625f ? series : hw;
}

template <typename T, bool DEV, typename R>
__device__ inline void fluid_noise(const LbParams& p, uint32_t n, int c, R rho, T f[Q]) {
  // s[k-4] = famp[k-4] r_k
  R s[NMODE_NOISE];
#pragma unroll
  for (int b = 0; b < 4; ++b) {
    uint32_t x0 = n, x1 = (uint32_t)c, x2 = (uint32_t)b, x3 = 1u;
    philox10(x0, x1, x2, x3, p.fseed, p.frep);
    R r[4];
    if constexpr (DEV) {
      const float s32 = 2.3283064365386963e-10f;   // 2^-32
      const float u1 = fmaf((float)x1, s32, 0.5f * s32), u3 = fmaf((float)x3, s32, 0.5f * s32);
      const float ra = __builtin_amdgcn_sqrtf(neg2_log_uniform(x0));
      const float rb = __builtin_amdgcn_sqrtf(neg2_log_uniform(x2));
      r[0] = ra * __builtin_amdgcn_cosf(u1);
      r[1] = ra * __builtin_amdgcn_sinf(u1);
      r[2] = rb * __builtin_amdgcn_cosf(u3);
      r[3] = rb * __builtin_amdgcn_sinf(u3);
    } else {
      const double inv32 = 1.0 / 4294967296.0;
      const double two_pi = 6.283185307179586;
      const double ra = sqrt(-2.0 * log(((double)x0 + 0.5) * inv32));
      const double rb = sqrt(-2.0 * log(((double)x2 + 0.5) * inv32));
      double sa, ca, sb, cb;
      sincos(two_pi * (((double)x1 + 0.5) * inv32), &sa, &ca);
      sincos(two_pi * (((double)x3 + 0.5) * inv32), &sb, &cb);
      r[0] = ra * ca; r[1] = ra * sa; r[2] = rb * cb; r[3] = rb * sb;
    }
#pragma unroll
    for (int j = 0; j < 4; ++j)
      if (4 * b + j < NMODE_NOISE) {
        if constexpr (DEV) s[4 * b + j] = p.famp32[4 * b + j] * r[j];
        else s[4 * b + j] = p.famp[4 * b + j] * r[j];
      }
  }
  // back to populations, f_i += sqrt(rho) w_i sum_k e_ki s_k, a velocity and
  // its opposite together: the even modes add to both, the odd ones with
  // opposite signs
  R sr;
  if constexpr (DEV) sr = __builtin_amdgcn_sqrtf(rho);
  else sr = sqrt(rho);
  const R a0 = sr * (R)wgt(0), a1 = sr * (R)wgt(1), a2 = sr * (R)wgt(7);
  // h = 0: the rest population; h = 1..9: the pair (2h - 1, 2h)
#pragma unroll
  for (int h = 0; h < 10; ++h) {
    const int i = h == 0 ? 0 : 2 * h - 1;
    R ev = (R)0, od = (R)0;
#pragma unroll
    for (int k = 0; k < NMODE_NOISE; ++k) {
      const int e = mode_coef(k + 4, i);
      R& acc = mode_odd(k + 4) ? od : ev;
      if (e == 1) acc += s[k];
      else if (e == -1) acc -= s[k];
      else if (e != 0) {
        if constexpr (DEV) acc = fmaf((float)e, s[k], acc);
        else acc += (R)e * s[k];
      }
    }
    if (h == 0) {
      f[0] = (T)((R)f[0] + a0 * ev);
    } else {
      const R a = i < 7 ? a1 : a2;
      f[i] = (T)((R)f[i] + a * (ev + od));
      f[i + 1] = (T)((R)f[i + 1] + a * (ev - od));
    }
  }
}

// Stream + collide one fluid node c of a replica (pointers already offset to
// the replica).
template <typename T, bool DEV>
__device__ inline void lb_node(const T* __restrict__ A, T* __restrict__ B, const uint8_t* __restrict__ flags,
                               const T* __restrict__ force, const LbParams& p, Ctrl* __restrict__ ctrl, int c,
                               uint8_t fl) {
  int x = c % p.nx;
  int yz = c / p.nx;
  int y = yz % p.ny;
  int z = yz / p.ny;
  Nbr nb = make_nbr(p, x, y, z);
  T f[Q];
  pull<T>(A, flags, p, c, fl, nb, f);
  const auto rho = collide_node<T, DEV>(f, f, force, p, ctrl, c, fl);
  if (p.fluct) fluid_noise<T, DEV>(p, (uint32_t)ctrl->step, c, rho, f);
  const size_t N = (size_t)p.N;
#pragma unroll
  for (int i = 0; i < Q; ++i) store_pop(&B[(size_t)i * N + c], f[i]);
}

// Halfway bounce-back at a node next to a wall, after a straight pull: the
// populations pulled from solid upstream nodes are replaced by the node's own
// opposite populations -- the values pull gives.  The replacements arrive
// before it returns, so no load of it is outstanding in the caller.
template <typename T>
__device__ inline void bounce_back(const T* __restrict__ A, const uint8_t* __restrict__ flags, const LbParams& p,
                                   int c, T f[Q]) {
  const size_t N = (size_t)p.N;
  int x = c % p.nx;
  int yz = c / p.nx;
  const Nbr nb = make_nbr(p, x, yz % p.ny, yz / p.ny);
  uint8_t sf[Q];
#pragma unroll
  for (int i = 0; i < Q; ++i) sf[i] = flags[c + nb.off(-cx(i), -cy(i), -cz(i))];
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    const T r = A[(size_t)opp(i) * N + (size_t)c];
    f[i] = (sf[i] & F_SOLID) ? r : f[i];
  }
#pragma unroll
  for (int i = 0; i < Q; ++i) asm volatile("" ::"v"(f[i]));
}

// Stream + collide U nodes c[u] of one replica (c[u] must be a valid node
// also where in[u] is false).  The flags and the straight pulls f_i =
// A_i(x - c_i) of all U nodes are issued together (a straight pull is a valid
// read at any node); a node next to a wall then replaces what came from solid
// nodes.  Flags and pulls are non-temporal loads: the streamed lattice then
// does not push the bead phase's working set out of the caches while the two
// run side by side.  Nodes with in[u] false, solid nodes and, with skip_forced, nodes
// carrying bead force are neither collided nor stored.  FL: replicas with a
// fluctuating fluid add its noise for LB step n.
template <typename T, bool DEV, int U, bool FL>
__device__ inline void lb_nodes(const T* __restrict__ A, T* __restrict__ B, const uint8_t* __restrict__ flags,
                                const T* __restrict__ force, const LbParams& p, Ctrl* __restrict__ ctrl,
                                const int c[U], const bool in[U], int skip_forced, uint32_t n) {
  const size_t N = (size_t)p.N;
  uint8_t fl[U];
  T f[U][Q];
#pragma unroll
  for (int u = 0; u < U; ++u) {
    fl[u] = __builtin_nontemporal_load(&flags[c[u]]);
    int x = c[u] % p.nx;
    int yz = c[u] / p.nx;
    const Nbr nb = make_nbr(p, x, yz % p.ny, yz / p.ny);
#pragma unroll
    for (int i = 0; i < Q; ++i)
      f[u][i] = __builtin_nontemporal_load(&A[(size_t)i * N + (size_t)(c[u] + nb.off(-cx(i), -cy(i), -cz(i)))]);
  }
  // every pull is taken here, so none is deferred behind the flag tests
#pragma unroll
  for (int u = 0; u < U; ++u)
#pragma unroll
    for (int i = 0; i < Q; ++i) asm volatile("" ::"v"(f[u][i]));
#pragma unroll
  for (int u = 0; u < U; ++u)
    if (fl[u] & F_NEAR) bounce_back<T>(A, flags, p, c[u], f[u]);
#pragma unroll
  for (int u = 0; u < U; ++u) {
    if (!in[u] || (fl[u] & F_SOLID) || (skip_forced && (fl[u] & F_FORCED))) continue;
    const auto rho = collide_node<T, DEV>(f[u], f[u], force, p, ctrl, c[u], fl[u]);
    if constexpr (FL)
      if (p.fluct) fluid_noise<T, DEV>(p, n, c[u], rho, f[u]);
#pragma unroll
    for (int i = 0; i < Q; ++i) store_pop(&B[(size_t)i * N + c[u]], f[u][i]);
  }
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

}  // namespace lbmd
