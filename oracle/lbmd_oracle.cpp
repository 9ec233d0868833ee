// lbmd_oracle.cpp -- TEST INFRASTRUCTURE, not product code.
//
// A plain, slow, FP64 CPU implementation of the coupled lattice-Boltzmann /
// molecular-dynamics time step described in Fyta, Sircar, Kaxiras,
// Melchionna, Bernaschi and Succi, "Parallel multiscale modeling of
// biopolymer dynamics with hydrodynamic correlations" (Sec. 2, numerical
// set-up in Sec. 4).  It exists only to check the GPU library: the test
// suite, the smoke check and the CPU-baseline leg of the benchmark load it
// through ctypes.  It shares no code, header or table with the GPU library.
//
// Everything is written in the most direct form of the paper's equations,
// loop by loop, with no blocking or fusion.  Where the paper is garbled or
// silent the reading used here is stated at the point of use (the same
// readings are listed in the design notes).
//
// The simulation is templated on the real type so that the same code runs in
// double and in forward-mode dual numbers (value + one tangent), which gives
// exact directional derivatives of a loss for checking the hand-written
// adjoint of the GPU library.

#include <algorithm>
#include <type_traits>
#include <unordered_map>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <vector>

#ifdef _OPENMP
#include <omp.h>
#endif

namespace orc {

// ---------------------------------------------------------------------------
// Dual numbers (value, derivative along one direction).
// ---------------------------------------------------------------------------
struct Dual {
  double v, d;
  Dual() : v(0.0), d(0.0) {}
  Dual(double x) : v(x), d(0.0) {}
  Dual(double x, double dx) : v(x), d(dx) {}
};
inline Dual operator+(Dual a, Dual b) { return Dual(a.v + b.v, a.d + b.d); }
inline Dual operator-(Dual a, Dual b) { return Dual(a.v - b.v, a.d - b.d); }
inline Dual operator-(Dual a) { return Dual(-a.v, -a.d); }
inline Dual operator*(Dual a, Dual b) { return Dual(a.v * b.v, a.d * b.v + a.v * b.d); }
inline Dual operator/(Dual a, Dual b) {
  double q = a.v / b.v;
  return Dual(q, (a.d - q * b.d) / b.v);
}
inline Dual& operator+=(Dual& a, Dual b) { a = a + b; return a; }
inline Dual& operator-=(Dual& a, Dual b) { a = a - b; return a; }
inline bool operator<(Dual a, Dual b) { return a.v < b.v; }
inline bool operator>(Dual a, Dual b) { return a.v > b.v; }
inline bool operator<=(Dual a, Dual b) { return a.v <= b.v; }
inline bool operator>=(Dual a, Dual b) { return a.v >= b.v; }
inline bool operator==(Dual a, Dual b) { return a.v == b.v; }

inline double val(double x) { return x; }
inline double val(Dual x) { return x.v; }
inline double dsqrt(double x) { return std::sqrt(x); }
inline Dual dsqrt(Dual x) {
  double s = std::sqrt(x.v);
  return Dual(s, s > 0.0 ? x.d / (2.0 * s) : 0.0);
}
inline double dexp(double x) { return std::exp(x); }
inline Dual dexp(Dual x) { double e = std::exp(x.v); return Dual(e, e * x.d); }
inline double datan2(double y, double x) { return std::atan2(y, x); }
inline Dual datan2(Dual y, Dual x) {
  double den = x.v * x.v + y.v * y.v;
  return Dual(std::atan2(y.v, x.v), (x.v * y.d - y.v * x.d) / den);
}

// ---------------------------------------------------------------------------
// D3Q19 lattice (Sec. 2: the standard three-dimensional 19-speed lattice).
// Velocity order: rest; +-x; +-y; +-z; the xy, xz and yz diagonals, each
// opposite pair adjacent.  Weights: 1/3 (rest), 1/18 (axis), 1/36 (diagonal).
// The paper prints neither table; these are the standard D3Q19 values of the
// lattice it cites.
// ---------------------------------------------------------------------------
constexpr int Q = 19;
const int CV[Q][3] = {
    {0, 0, 0},
    {1, 0, 0},   {-1, 0, 0},  {0, 1, 0},   {0, -1, 0},  {0, 0, 1},   {0, 0, -1},
    {1, 1, 0},   {-1, -1, 0}, {1, -1, 0},  {-1, 1, 0},
    {1, 0, 1},   {-1, 0, -1}, {1, 0, -1},  {-1, 0, 1},
    {0, 1, 1},   {0, -1, -1}, {0, 1, -1},  {0, -1, 1}};
const int OPP[Q] = {0, 2, 1, 4, 3, 6, 5, 8, 7, 10, 9, 12, 11, 14, 13, 16, 15, 18, 17};
inline double weight(int i) { return i == 0 ? 1.0 / 3.0 : (i < 7 ? 1.0 / 18.0 : 1.0 / 36.0); }

inline int wrapi(int a, int n) { a %= n; return a < 0 ? a + n : a; }

// ---------------------------------------------------------------------------
// Counter-based noise: Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11),
// written from its published definition: ten rounds of two 32x32->64-bit
// multiplies with multipliers 0xD2511F53 and 0xCD9E8D57, the key bumped by
// the Weyl constants 0x9E3779B9 and 0xBB67AE85 between rounds.
// ---------------------------------------------------------------------------
void philox4x32_10(const uint32_t in[4], const uint32_t key[2], uint32_t out[4]) {
  uint32_t c0 = in[0], c1 = in[1], c2 = in[2], c3 = in[3];
  uint32_t k0 = key[0], k1 = key[1];
  for (int round = 0; round < 10; ++round) {
    if (round > 0) { k0 += 0x9E3779B9u; k1 += 0xBB67AE85u; }
    uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
    uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
    uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
    uint32_t n1 = (uint32_t)p1;
    uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
    uint32_t n3 = (uint32_t)p0;
    c0 = n0; c1 = n1; c2 = n2; c3 = n3;
  }
  out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

// Three standard normals for bead p at LB step n, MD sub-step s: one Philox
// block with key (seed, replica) and counter (n, s, p, 0); uniforms
// (x + 1/2) 2^-32 in (0,1); Box-Muller (1958) on (u0,u1) and (u2,u3).
void gauss3(uint32_t seed, uint32_t rep, uint32_t n, uint32_t s, uint32_t p, double xi[3]) {
  uint32_t ctr[4] = {n, s, p, 0u};
  uint32_t key[2] = {seed, rep};
  uint32_t x[4];
  philox4x32_10(ctr, key, x);
  const double two32inv = 1.0 / 4294967296.0;
  double u0 = ((double)x[0] + 0.5) * two32inv;
  double u1 = ((double)x[1] + 0.5) * two32inv;
  double u2 = ((double)x[2] + 0.5) * two32inv;
  double u3 = ((double)x[3] + 0.5) * two32inv;
  const double two_pi = 6.283185307179586;
  double ra = std::sqrt(-2.0 * std::log(u0));
  double rb = std::sqrt(-2.0 * std::log(u2));
  xi[0] = ra * std::cos(two_pi * u1);
  xi[1] = ra * std::sin(two_pi * u1);
  xi[2] = rb * std::cos(two_pi * u3);
}

// ---------------------------------------------------------------------------
// Fluctuating lattice Boltzmann (Sec. 2, the stochastic term F_i: a noisy
// stress on the five shear/bulk stress modes plus noise on the ghost modes,
// in the mode formulation of Adhikari et al. the paper refers to).  Reading:
// the 19 populations are mapped to 19 moments m_k = sum_i e_ki f_i of a basis
// orthogonal under the weights, sum_i w_i e_ki e_li = b_k delta_kl; the BGK
// collision relaxes every non-conserved mode by the same factor 1 - omega;
// fluctuation-dissipation then fixes the noise on each non-conserved mode k
// as sqrt(mu b_k (1 - (1 - omega)^2)) r_k with mu = rho kT / c_s^2 and r_k
// standard normal, mapped back by f_i += w_i sum_k e_ki noise_k / b_k.
// The basis, in powers of the lattice velocity c:
//   k = 0: 1;  1..3: c_x, c_y, c_z;  4: c^2 - 1;  5: 3 c_x^2 - c^2;
//   6: c_y^2 - c_z^2;  7..9: c_x c_y, c_y c_z, c_z c_x;
//   10..12: (3 c^2 - 5) c_x, (3 c^2 - 5) c_y, (3 c^2 - 5) c_z;
//   13..15: (c_y^2 - c_z^2) c_x, (c_z^2 - c_x^2) c_y, (c_x^2 - c_y^2) c_z;
//   16: 3 c^4 - 6 c^2 + 1;  17: (2 c^2 - 3)(3 c_x^2 - c^2);
//   18: (2 c^2 - 3)(c_y^2 - c_z^2).
// Modes 0..3 (mass, momentum) are conserved and get no noise.
// ---------------------------------------------------------------------------
inline double mode_poly(int k, int i) {
  const double x = CV[i][0], y = CV[i][1], z = CV[i][2];
  const double c2 = x * x + y * y + z * z;
  switch (k) {
    case 0: return 1.0;
    case 1: return x;
    case 2: return y;
    case 3: return z;
    case 4: return c2 - 1.0;
    case 5: return 3.0 * x * x - c2;
    case 6: return y * y - z * z;
    case 7: return x * y;
    case 8: return y * z;
    case 9: return z * x;
    case 10: return (3.0 * c2 - 5.0) * x;
    case 11: return (3.0 * c2 - 5.0) * y;
    case 12: return (3.0 * c2 - 5.0) * z;
    case 13: return (y * y - z * z) * x;
    case 14: return (z * z - x * x) * y;
    case 15: return (x * x - y * y) * z;
    case 16: return 3.0 * c2 * c2 - 6.0 * c2 + 1.0;
    case 17: return (2.0 * c2 - 3.0) * (3.0 * x * x - c2);
    default: return (2.0 * c2 - 3.0) * (y * y - z * z);
  }
}

// Norm b_k = sum_i w_i e_ki^2 of a basis vector.
inline double mode_norm(int k) {
  double b = 0.0;
  for (int i = 0; i < Q; ++i) b += weight(i) * mode_poly(k, i) * mode_poly(k, i);
  return b;
}

// Sixteen standard normals for fluid node `node` of replica `rep` at LB step
// n: four Philox blocks with key (seed, replica) and counter (n, node, k, 1),
// k = 0..3 (the bead noise uses counter word 3 = 0), uniforms (x + 1/2) 2^-32,
// Box-Muller on (u0,u1) and (u2,u3) of each block, cosine then sine.
void fluid_normals(uint32_t seed, uint32_t rep, uint32_t n, uint32_t node, double r[16]) {
  const double two32inv = 1.0 / 4294967296.0;
  const double two_pi = 6.283185307179586;
  uint32_t key[2] = {seed, rep};
  for (uint32_t k = 0; k < 4; ++k) {
    uint32_t ctr[4] = {n, node, k, 1u};
    uint32_t x[4];
    philox4x32_10(ctr, key, x);
    double u[4];
    for (int j = 0; j < 4; ++j) u[j] = ((double)x[j] + 0.5) * two32inv;
    double ra = std::sqrt(-2.0 * std::log(u[0]));
    double rb = std::sqrt(-2.0 * std::log(u[2]));
    r[4 * k + 0] = ra * std::cos(two_pi * u[1]);
    r[4 * k + 1] = ra * std::sin(two_pi * u[1]);
    r[4 * k + 2] = rb * std::cos(two_pi * u[3]);
    r[4 * k + 3] = rb * std::sin(two_pi * u[3]);
  }
}

}  // namespace orc

// ---------------------------------------------------------------------------
// Run description shared with the Python side through ctypes.
// ---------------------------------------------------------------------------
extern "C" {
typedef struct {
  int nx, ny, nz;
  double tau;          // BGK relaxation time, omega = 1/tau
  double g[3];         // uniform body-force density on every fluid node
  int wall_axis;       // -1: no wall; 0,1,2: the wall is normal to x,y,z
  int wall_pos;        // lattice plane of the wall along wall_axis
  int pore_h;          // side of the square pore (lattice nodes)
  int nb;              // number of beads (0: fluid only)
  double mass, k_bond, r0, kappa, eps, sigma, rc;
  double gamma, kT, f_drive;
  int n_sub;           // MD sub-steps per LB step
  uint32_t seed, replica;
  double fluid_kT;     // thermal energy of the fluid noise (0: athermal BGK fluid)
  int mts_outer;       // 0: n_sub uniform sub-steps; M > 0: the multiple-time-step cycle with M outer steps
  int coupling;        // bead <-> lattice transfer: 0 trilinear, 1 nearest grid point
  int constraints;     // 0: harmonic bonds; 1: rigid bonds |r_{p+1} - r_p| = r0 (SHAKE / RATTLE)
} or_desc;
}

namespace orc {

template <class R>
struct Sim {
  or_desc d;
  int nx, ny, nz;
  long N;
  int nb;
  double omega, h, hh, m;
  R gamma, fdrive;
  R e, omE, cf, sig;   // SPV coefficients exp(-g h), 1-exp(-g h), (1-exp(-g h))/(m g), noise sd
  std::vector<uint8_t> solid;
  std::vector<R> A, B;         // post-collision populations, layout [Q][N]
  std::vector<R> F;            // bead force density on the lattice, [3][N]
  std::vector<R> r, v, up, J;  // bead arrays, [nb][3]
  std::vector<R> rstart;
  long long step;
  R ledger_bb[3];      // momentum given to solid nodes by bounce-back (cumulative)
  R ledger_sp[3];      // bead reaction force that fell on solid nodes (cumulative)
  int tn[2];           // transverse axes of the wall
  int lo[2], hi[2];    // pore block bounds on the transverse axes
  bool use_cells;

  long idx(int x, int y, int z) const { return (long)x + (long)nx * ((long)y + (long)ny * (long)z); }
  int ext(int a) const { return a == 0 ? nx : (a == 1 ? ny : nz); }

  // -- geometry (Sec. 4): one wall plane normal to wall_axis at wall_pos,
  // solid except an h x h pore block centred on the two transverse axes.
  void build_geometry() {
    solid.assign(N, 0);
    if (d.wall_axis < 0) return;
    int a = d.wall_axis;
    tn[0] = (a == 0) ? 1 : 0;
    tn[1] = (a == 2) ? 1 : 2;
    for (int k = 0; k < 2; ++k) {
      lo[k] = ext(tn[k]) / 2 - d.pore_h / 2;
      hi[k] = lo[k] + d.pore_h - 1;
    }
    for (int z = 0; z < nz; ++z)
      for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
          int c[3] = {x, y, z};
          if (c[a] != d.wall_pos) continue;
          bool in_pore = c[tn[0]] >= lo[0] && c[tn[0]] <= hi[0] && c[tn[1]] >= lo[1] && c[tn[1]] <= hi[1];
          if (!in_pore) solid[idx(x, y, z)] = 1;
        }
  }

  void init(const or_desc& desc, const double* r0in, const double* v0in) {
    d = desc;
    nx = d.nx; ny = d.ny; nz = d.nz;
    N = (long)nx * ny * nz;
    nb = d.nb;
    omega = 1.0 / d.tau;
    h = 1.0 / (double)d.n_sub;
    hh = 0.5 * h;
    m = d.mass;
    gamma = R(d.gamma);
    fdrive = R(d.f_drive);
    build_geometry();
    // Sec. 4: the solvent starts at the equilibrium of unit density and zero
    // velocity, i.e. f_i = w_i.
    A.assign((size_t)Q * N, R(0.0));
    for (int i = 0; i < Q; ++i)
      for (long c = 0; c < N; ++c) A[(size_t)i * N + c] = R(weight(i));
    B = A;
    F.assign((size_t)3 * N, R(0.0));
    r.assign((size_t)3 * nb, R(0.0));
    v.assign((size_t)3 * nb, R(0.0));
    up.assign((size_t)3 * nb, R(0.0));
    J.assign((size_t)3 * nb, R(0.0));
    rstart.assign((size_t)3 * nb, R(0.0));
    for (int k = 0; k < 3 * nb; ++k) {
      r[k] = R(r0in ? r0in[k] : 0.0);
      v[k] = R(v0in ? v0in[k] : 0.0);
    }
    step = 0;
    for (int a = 0; a < 3; ++a) { ledger_bb[a] = R(0.0); ledger_sp[a] = R(0.0); }
    use_cells = false;
    if (nb > 256) {
      use_cells = true;
      for (int a = 0; a < 3; ++a)
        if ((int)std::floor((double)ext(a) / d.rc) < 3) use_cells = false;
    }
    set_spv_coefficients(gamma, d.kT);
  }

  // Sec. 2, Eq. (SPValgo): exponential factors of the stochastic position
  // Verlet kick, computed once.  gamma = 0 is the deterministic limit.
  void set_spv_coefficients(R g, double kT) {
    if (val(g) == 0.0) {
      e = R(1.0); omE = R(0.0); cf = R(h / m); sig = R(0.0);
      return;
    }
    e = dexp(-(g * R(h)));
    omE = R(1.0) - e;
    cf = omE / (R(m) * g);
    R var = R(kT / m) * (R(1.0) - e * e);
    sig = (kT > 0.0) ? dsqrt(var) : R(0.0);
  }

  // ---- lattice-Boltzmann ---------------------------------------------------
  // Post-streaming population i at node (x,y,z): pulled from the upstream
  // node x - c_i of the stored post-collision array S; if that node is solid
  // the population leaving (x,y,z) towards it returns reversed (halfway
  // bounce-back at the wall, Sec. 3 lists walls as a boundary type).
  R pulled(const std::vector<R>& S, int x, int y, int z, int i) const {
    int sx = wrapi(x - CV[i][0], nx), sy = wrapi(y - CV[i][1], ny), sz = wrapi(z - CV[i][2], nz);
    long src = idx(sx, sy, sz);
    if (solid[src]) return S[(size_t)OPP[i] * N + idx(x, y, z)];
    return S[(size_t)i * N + src];
  }

  // Moments, Eqs. (dens) and (vel): rho = sum f_i, rho u = sum f_i c_i.
  static void moments(const R f[Q], R& rho, R u[3]) {
    rho = R(0.0);
    for (int i = 0; i < Q; ++i) rho += f[i];
    R j[3] = {R(0.0), R(0.0), R(0.0)};
    for (int i = 0; i < Q; ++i)
      for (int a = 0; a < 3; ++a) j[a] += f[i] * R((double)CV[i][a]);
    for (int a = 0; a < 3; ++a) u[a] = j[a] / rho;
  }

  // Local equilibrium: second-order expansion of the Maxwellian,
  // f_i^eq = w_i rho [1 + 3 c.u + 9/2 (c.u)^2 - 3/2 u.u].  The printed form
  // lost the leading rho and the "1 +"; beta = 1/c_s^2 = 3 in lattice units.
  static R feq(int i, R rho, const R u[3]) {
    R cu = R((double)CV[i][0]) * u[0] + R((double)CV[i][1]) * u[1] + R((double)CV[i][2]) * u[2];
    R usq = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    return R(weight(i)) * rho * (R(1.0) + R(3.0) * cu + R(4.5) * cu * cu - R(1.5) * usq);
  }

  // One BGK collision with source, Eq. (lbe2) read as a relaxation,
  // f* = f - omega (f - f^eq) + S, with the first-order source
  // S_i = 3 w_i F.c_i (the S_i of Sec. 2 with beta = 3; F is the force density
  // the beads exert on the fluid plus any uniform body force).
  void collide(const R f[Q], const R Fx[3], R out[Q]) const {
    R rho, u[3];
    moments(f, rho, u);
    for (int i = 0; i < Q; ++i) {
      R fe = feq(i, rho, u);
      R dot = Fx[0] * R((double)CV[i][0]) + Fx[1] * R((double)CV[i][1]) + Fx[2] * R((double)CV[i][2]);
      R src = R(3.0 * weight(i)) * dot;
      out[i] = f[i] - R(omega) * (f[i] - fe) + src;
    }
  }

  // The stochastic term of the fluctuating fluid at node c (see
  // fluid_normals and mode_poly): with rho from the pulled populations f,
  // noise_k = sqrt(3 rho kT (1 - (1 - omega)^2) / b_k) r_{k-4} on modes
  // k = 4..18, added as out_i += w_i sum_k e_ki noise_k in ascending k.
  void fluctuate(long c, const R f[Q], R out[Q]) const {
    double r[16];
    fluid_normals(d.seed, d.replica, (uint32_t)step, (uint32_t)c, r);
    R rho = R(0.0);
    for (int i = 0; i < Q; ++i) rho += f[i];
    const double g2 = (1.0 - omega) * (1.0 - omega);
    R noise[Q];
    for (int k = 4; k < Q; ++k)
      noise[k] = dsqrt(R(3.0 * d.fluid_kT * (1.0 - g2) / mode_norm(k)) * rho) * R(r[k - 4]);
    for (int i = 0; i < Q; ++i) {
      R s = R(0.0);
      for (int k = 4; k < Q; ++k) s += R(mode_poly(k, i)) * noise[k];
      out[i] = out[i] + R(weight(i)) * s;
    }
  }

  // One LB time step: stream (pull) + collide every fluid node, A -> B, then
  // swap.  Solid nodes are never written.  The bounce-back momentum given to
  // the wall is recorded in ledger_bb.
  void lb_sweep() {
    // Ledger: every link (x, i) whose upstream node x - c_i is solid carried
    // A_opp(i)(x) into the wall and came back as f_i(x): the wall took
    // 2 A_opp(i)(x) c_opp(i).  Summed per z plane, then over planes in order.
    std::vector<R> plane_ledger((size_t)3 * nz, R(0.0));
#pragma omp parallel for schedule(static)
    for (int z = 0; z < nz; ++z) {
      R f[Q], out[Q], Fx[3];
      for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
          long c = idx(x, y, z);
          if (solid[c]) continue;
          for (int i = 0; i < Q; ++i) f[i] = pulled(A, x, y, z, i);
          for (int a = 0; a < 3; ++a) Fx[a] = F[(size_t)a * N + c] + R(d.g[a]);
          collide(f, Fx, out);
          if (d.fluid_kT > 0.0) fluctuate(c, f, out);
          for (int i = 0; i < Q; ++i) B[(size_t)i * N + c] = out[i];
          for (int i = 1; i < Q; ++i) {
            long src = idx(wrapi(x - CV[i][0], nx), wrapi(y - CV[i][1], ny), wrapi(z - CV[i][2], nz));
            if (!solid[src]) continue;
            R fo = A[(size_t)OPP[i] * N + c];
            for (int a = 0; a < 3; ++a) plane_ledger[3 * (size_t)z + a] += R(2.0) * fo * R((double)CV[OPP[i]][a]);
          }
        }
    }
    for (int z = 0; z < nz; ++z)
      for (int a = 0; a < 3; ++a) ledger_bb[a] += plane_ledger[3 * (size_t)z + a];
    std::swap(A, B);
  }

  // Fluid velocity at a node from the pulled (post-streaming) populations of
  // the stored array; zero at solid nodes.
  void node_velocity(int x, int y, int z, R u[3]) const {
    if (solid[idx(x, y, z)]) { u[0] = u[1] = u[2] = R(0.0); return; }
    R f[Q], rho;
    for (int i = 0; i < Q; ++i) f[i] = pulled(A, x, y, z, i);
    moments(f, rho, u);
  }

  // ---- bead <-> lattice interpolation --------------------------------------
  // Periodic wrap of an unwrapped coordinate into [0, n).
  R wrapc(R x, int n) const {
    double q = std::floor(val(x) / (double)n);
    R w = x - R((double)n * q);
    if (val(w) >= (double)n) w = w - R((double)n);
    return w;
  }
  // Stencil of bead p at position rp: base node b, the 8 corner nodes
  // (corner k has offsets (k&1, k>>1&1, k>>2&1)) and their weights --
  // trilinear, or with the nearest-grid-point transfer (Sec. 2, the
  // particle/grid paragraph: the fluid velocity is taken at the nearest node
  // and the forces go back to it) weight 1 at the nearest corner, which is
  // the upper one along an axis where the fraction is at least 1/2, and 0 at
  // the others.
  void stencil(const R* rp, long node[8], R W[8]) const {
    int b[3];
    R del[3];
    for (int a = 0; a < 3; ++a) {
      R w = wrapc(rp[a], ext(a));
      b[a] = (int)std::floor(val(w));
      del[a] = w - R((double)b[a]);
      if (d.coupling == 1) del[a] = val(del[a]) >= 0.5 ? R(1.0) : R(0.0);
    }
    for (int k = 0; k < 8; ++k) {
      int o[3] = {k & 1, (k >> 1) & 1, (k >> 2) & 1};
      node[k] = idx(wrapi(b[0] + o[0], nx), wrapi(b[1] + o[1], ny), wrapi(b[2] + o[2], nz));
      R wx = o[0] ? del[0] : R(1.0) - del[0];
      R wy = o[1] ? del[1] : R(1.0) - del[1];
      R wz = o[2] ? del[2] : R(1.0) - del[2];
      W[k] = wx * wy * wz;
    }
  }
  // u_p = sum_k W_k u(node_k)  (the paper uses the nearest grid point; the
  // trilinear stencil is the finer interpolation it compares against).
  void gather(const std::vector<R>& pos, std::vector<R>& out) const {
    for (int p = 0; p < nb; ++p) {
      long node[8];
      R W[8];
      stencil(&pos[3 * p], node, W);
      R acc[3] = {R(0.0), R(0.0), R(0.0)};
      for (int k = 0; k < 8; ++k) {
        long c = node[k];
        int x = (int)(c % nx), y = (int)((c / nx) % ny), z = (int)(c / ((long)nx * ny));
        R u[3];
        node_velocity(x, y, z, u);
        for (int a = 0; a < 3; ++a) acc[a] += W[k] * u[a];
      }
      for (int a = 0; a < 3; ++a) out[3 * p + a] = acc[a];
    }
  }
  // Force density on the lattice: F(x) = sum_p W(x - r_p) J_p, beads in
  // ascending order; shares landing on solid nodes go to ledger_sp.
  void spread(const std::vector<R>& pos, const std::vector<R>& Jin) {
    std::fill(F.begin(), F.end(), R(0.0));
    for (int p = 0; p < nb; ++p) {
      long node[8];
      R W[8];
      stencil(&pos[3 * p], node, W);
      for (int k = 0; k < 8; ++k) {
        for (int a = 0; a < 3; ++a) {
          R add = W[k] * Jin[3 * p + a];
          if (solid[node[k]]) ledger_sp[a] += add;
          else F[(size_t)a * N + node[k]] += add;
        }
      }
    }
  }

  // ---- bead forces (Sec. 2, Eq. (MDFORCES) and the potentials after it) ----
  void min_image(R dd[3]) const {
    for (int a = 0; a < 3; ++a) {
      double n = (double)ext(a);
      double k = std::floor(val(dd[a]) / n + 0.5);
      dd[a] = dd[a] - R(n * k);
    }
  }
  // Harmonic bond V = k_r/2 (|r_p - r_q| - r0)^2: force on p.
  void bond_force(const std::vector<R>& pos, int p, int q, R Fp[3]) const {
    R dd[3];
    for (int a = 0; a < 3; ++a) dd[a] = pos[3 * p + a] - pos[3 * q + a];
    R dist = dsqrt(dd[0] * dd[0] + dd[1] * dd[1] + dd[2] * dd[2]);
    R coef = -(R(d.k_bond) * (dist - R(d.r0))) / dist;
    for (int a = 0; a < 3; ++a) Fp[a] += coef * dd[a];
  }
  // Bending V = kappa phi^2 / 2 at interior bead q, phi the angle between
  // bonds b1 = r_q - r_{q-1} and b2 = r_{q+1} - r_q, phi = atan2(|b1 x b2|, b1.b2).
  // Returns the forces on q-1, q, q+1.
  void angle_forces(const std::vector<R>& pos, int q, R Fm[3], R F0[3], R Fp[3]) const {
    R b1[3], b2[3];
    for (int a = 0; a < 3; ++a) {
      b1[a] = pos[3 * q + a] - pos[3 * (q - 1) + a];
      b2[a] = pos[3 * (q + 1) + a] - pos[3 * q + a];
    }
    R n[3] = {b1[1] * b2[2] - b1[2] * b2[1], b1[2] * b2[0] - b1[0] * b2[2], b1[0] * b2[1] - b1[1] * b2[0]};
    R s = dsqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
    R c = b1[0] * b2[0] + b1[1] * b2[1] + b1[2] * b2[2];
    for (int a = 0; a < 3; ++a) { Fm[a] = R(0.0); F0[a] = R(0.0); Fp[a] = R(0.0); }
    if (val(s) == 0.0) return;   // straight (or folded) chain: no unique gradient
    R phi = datan2(s, c);
    R den = s * s + c * c;
    R g1[3] = {b2[1] * n[2] - b2[2] * n[1], b2[2] * n[0] - b2[0] * n[2], b2[0] * n[1] - b2[1] * n[0]};
    R g2[3] = {n[1] * b1[2] - n[2] * b1[1], n[2] * b1[0] - n[0] * b1[2], n[0] * b1[1] - n[1] * b1[0]};
    R kp = R(d.kappa) * phi;
    for (int a = 0; a < 3; ++a) {
      R d1 = (c * g1[a] / s - s * b2[a]) / den;   // d phi / d b1
      R d2 = (c * g2[a] / s - s * b1[a]) / den;   // d phi / d b2
      Fm[a] = kp * d1;
      F0[a] = -(kp * (d1 - d2));
      Fp[a] = -(kp * d2);
    }
  }
  // Lennard-Jones 6-12 truncated at r_c = 2^(1/6) sigma (purely repulsive):
  // adds the pair force on the first bead of a pair with separation dd.
  void lj_pair(const R dd[3], R Fp[3]) const {
    R r2 = dd[0] * dd[0] + dd[1] * dd[1] + dd[2] * dd[2];
    if (!(val(r2) < d.rc * d.rc)) return;
    R sr2 = R(d.sigma * d.sigma) / r2;
    R sr6 = sr2 * sr2 * sr2;
    R sr12 = sr6 * sr6;
    R coef = R(24.0 * d.eps) * (R(2.0) * sr12 - sr6) / r2;
    for (int a = 0; a < 3; ++a) Fp[a] += coef * dd[a];
  }
  // Bead-bead LJ on bead p, summed over all other beads j in ascending order
  // (every pair, bonded or not; minimum image in the periodic box).
  void lj_on_bead(const std::vector<R>& pos, int p, const std::vector<int>* cand, R Fp[3]) const {
    if (cand) {
      for (int j : *cand) {
        R dd[3];
        for (int a = 0; a < 3; ++a) dd[a] = pos[3 * p + a] - pos[3 * j + a];
        min_image(dd);
        lj_pair(dd, Fp);
      }
      return;
    }
    for (int j = 0; j < nb; ++j) {
      if (j == p) continue;
      R dd[3];
      for (int a = 0; a < 3; ++a) dd[a] = pos[3 * p + a] - pos[3 * j + a];
      min_image(dd);
      lj_pair(dd, Fp);
    }
  }
  // Wall repulsion: the same truncated LJ between a bead and every solid node
  // site within r_c.  r_c <= 3, so the sites at offsets -2..3 from the bead's
  // base node on each axis cover every candidate (z outer, x inner).
  void wall_on_bead(const std::vector<R>& pos, int p, R Fp[3]) const {
    if (d.wall_axis < 0) return;
    R w[3];
    int b[3];
    for (int a = 0; a < 3; ++a) {
      w[a] = wrapc(pos[3 * p + a], ext(a));
      b[a] = (int)std::floor(val(w[a]));
    }
    for (int oz = -2; oz <= 3; ++oz)
      for (int oy = -2; oy <= 3; ++oy)
        for (int ox = -2; ox <= 3; ++ox) {
          int sx = b[0] + ox, sy = b[1] + oy, sz = b[2] + oz;
          if (!solid[idx(wrapi(sx, nx), wrapi(sy, ny), wrapi(sz, nz))]) continue;
          R dd[3] = {w[0] - R((double)sx), w[1] - R((double)sy), w[2] - R((double)sz)};
          lj_pair(dd, Fp);
        }
  }
  // Driving field: F_drive along +normal on beads inside the pore channel,
  // the box [wall-1.5, wall+1.5) along the normal times the pore opening
  // [lo-0.5, hi+0.5) on each transverse axis (wrapped coordinates).
  bool in_field(const R* rp) const {
    if (d.wall_axis < 0) return false;
    int a = d.wall_axis;
    double wn = val(wrapc(rp[a], ext(a)));
    if (!(wn >= d.wall_pos - 1.5 && wn < d.wall_pos + 1.5)) return false;
    for (int k = 0; k < 2; ++k) {
      double wt = val(wrapc(rp[tn[k]], ext(tn[k])));
      if (!(wt >= lo[k] - 0.5 && wt < hi[k] + 0.5)) return false;
    }
    return true;
  }

  // Cell list for the LJ sum (cells of side >= r_c); the candidates of each
  // bead are sorted, so the sum runs in the same ascending order as the
  // all-pairs loop.
  void build_candidates(const std::vector<R>& pos, std::vector<std::vector<int>>& cand) const {
    int mc[3];
    double side[3];
    for (int a = 0; a < 3; ++a) {
      mc[a] = (int)std::floor((double)ext(a) / d.rc);
      side[a] = (double)ext(a) / (double)mc[a];
    }
    // occupied cells only (most cells of a large box are empty)
    std::unordered_map<long, std::vector<int>> cells;
    auto cell_of = [&](int x, int y, int z) { return (long)x + (long)mc[0] * ((long)y + (long)mc[1] * (long)z); };
    std::vector<int> cid(nb * 3);
    for (int p = 0; p < nb; ++p) {
      for (int a = 0; a < 3; ++a) {
        double w = val(wrapc(pos[3 * p + a], ext(a)));
        int c = (int)std::floor(w / side[a]);
        if (c >= mc[a]) c = mc[a] - 1;
        cid[3 * p + a] = c;
      }
      cells[cell_of(cid[3 * p], cid[3 * p + 1], cid[3 * p + 2])].push_back(p);
    }
    cand.assign(nb, {});
    for (int p = 0; p < nb; ++p) {
      for (int oz = -1; oz <= 1; ++oz)
        for (int oy = -1; oy <= 1; ++oy)
          for (int ox = -1; ox <= 1; ++ox) {
            int cx = wrapi(cid[3 * p] + ox, mc[0]), cy = wrapi(cid[3 * p + 1] + oy, mc[1]),
                cz = wrapi(cid[3 * p + 2] + oz, mc[2]);
            auto it = cells.find(cell_of(cx, cy, cz));
            if (it == cells.end()) continue;
            for (int j : it->second)
              if (j != p) cand[p].push_back(j);
          }
      std::sort(cand[p].begin(), cand[p].end());
    }
  }

  // Total conservative force on every bead, in a fixed order per bead:
  // bonds (p-1, p+1), bending angles centred at p-1, p, p+1, bead LJ
  // (ascending partner), wall LJ, driving field.
  void forces(const std::vector<R>& pos, std::vector<R>& Fc, bool field_on) const {
    std::vector<std::vector<int>> cand;
    if (use_cells) build_candidates(pos, cand);
    for (int p = 0; p < nb; ++p) {
      R Fp[3] = {R(0.0), R(0.0), R(0.0)};
      if (!d.constraints) {
        if (p > 0) bond_force(pos, p, p - 1, Fp);
        if (p < nb - 1) bond_force(pos, p, p + 1, Fp);
      }
      for (int q = p - 1; q <= p + 1; ++q) {
        if (q < 1 || q > nb - 2) continue;
        R Fm[3], F0[3], Fq[3];
        angle_forces(pos, q, Fm, F0, Fq);
        const R* mine = (q == p + 1) ? Fm : (q == p ? F0 : Fq);
        for (int a = 0; a < 3; ++a) Fp[a] += mine[a];
      }
      lj_on_bead(pos, p, use_cells ? &cand[p] : nullptr, Fp);
      wall_on_bead(pos, p, Fp);
      if (field_on && in_field(&pos[3 * p])) Fp[d.wall_axis] += fdrive;
      for (int a = 0; a < 3; ++a) Fc[3 * p + a] = Fp[a];
    }
  }

  // The two force groups of the multiple-time-step cycle, each summed in the
  // order of forces(): the bonded forces (bonds to p-1 and p+1, the angles
  // centred at p-1, p, p+1) and the slow forces (bead LJ in ascending
  // partner order, wall sites, field).
  void fast_forces(const std::vector<R>& pos, std::vector<R>& Fb) const {
    for (int p = 0; p < nb; ++p) {
      R Fp[3] = {R(0.0), R(0.0), R(0.0)};
      if (p > 0) bond_force(pos, p, p - 1, Fp);
      if (p < nb - 1) bond_force(pos, p, p + 1, Fp);
      for (int q = p - 1; q <= p + 1; ++q) {
        if (q < 1 || q > nb - 2) continue;
        R Fm[3], F0[3], Fq[3];
        angle_forces(pos, q, Fm, F0, Fq);
        const R* mine = (q == p + 1) ? Fm : (q == p ? F0 : Fq);
        for (int a = 0; a < 3; ++a) Fp[a] += mine[a];
      }
      for (int a = 0; a < 3; ++a) Fb[3 * p + a] = Fp[a];
    }
  }
  void slow_forces(const std::vector<R>& pos, std::vector<R>& Fs, bool field_on) const {
    std::vector<std::vector<int>> cand;
    if (use_cells) build_candidates(pos, cand);
    for (int p = 0; p < nb; ++p) {
      R Fp[3] = {R(0.0), R(0.0), R(0.0)};
      lj_on_bead(pos, p, use_cells ? &cand[p] : nullptr, Fp);
      wall_on_bead(pos, p, Fp);
      if (field_on && in_field(&pos[3 * p])) Fp[d.wall_axis] += fdrive;
      for (int a = 0; a < 3; ++a) Fs[3 * p + a] = Fp[a];
    }
  }

  // Potential energy of the conservative forces except the field (the field
  // is a step in space and has no potential): used by finite-difference pins.
  double energy(const std::vector<R>& pos) const {
    double E = 0.0;
    auto P = [&](int p, int a) { return val(pos[3 * p + a]); };
    for (int p = 0; p + 1 < nb && !d.constraints; ++p) {
      double dd[3], s = 0.0;
      for (int a = 0; a < 3; ++a) { dd[a] = P(p + 1, a) - P(p, a); s += dd[a] * dd[a]; }
      double dl = std::sqrt(s) - d.r0;
      E += 0.5 * d.k_bond * dl * dl;
    }
    for (int q = 1; q + 1 < nb; ++q) {
      double b1[3], b2[3];
      for (int a = 0; a < 3; ++a) { b1[a] = P(q, a) - P(q - 1, a); b2[a] = P(q + 1, a) - P(q, a); }
      double n0 = b1[1] * b2[2] - b1[2] * b2[1], n1 = b1[2] * b2[0] - b1[0] * b2[2], n2 = b1[0] * b2[1] - b1[1] * b2[0];
      double phi = std::atan2(std::sqrt(n0 * n0 + n1 * n1 + n2 * n2), b1[0] * b2[0] + b1[1] * b2[1] + b1[2] * b2[2]);
      E += 0.5 * d.kappa * phi * phi;
    }
    auto lj = [&](double r2) {
      if (!(r2 < d.rc * d.rc)) return 0.0;
      double sr6 = std::pow(d.sigma * d.sigma / r2, 3);
      return 4.0 * d.eps * (sr6 * sr6 - sr6) + d.eps;
    };
    for (int p = 0; p < nb; ++p)
      for (int j = p + 1; j < nb; ++j) {
        R dd[3];
        for (int a = 0; a < 3; ++a) dd[a] = pos[3 * p + a] - pos[3 * j + a];
        min_image(dd);
        E += lj(val(dd[0]) * val(dd[0]) + val(dd[1]) * val(dd[1]) + val(dd[2]) * val(dd[2]));
      }
    if (d.wall_axis >= 0) {
      for (int p = 0; p < nb; ++p) {
        double w[3];
        int b[3];
        for (int a = 0; a < 3; ++a) { w[a] = val(wrapc(pos[3 * p + a], ext(a))); b[a] = (int)std::floor(w[a]); }
        for (int oz = -2; oz <= 3; ++oz)
          for (int oy = -2; oy <= 3; ++oy)
            for (int ox = -2; ox <= 3; ++ox) {
              int sx = b[0] + ox, sy = b[1] + oy, sz = b[2] + oz;
              if (!solid[idx(wrapi(sx, nx), wrapi(sy, ny), wrapi(sz, nz))]) continue;
              double dx = w[0] - sx, dy = w[1] - sy, dz = w[2] - sz;
              E += lj(dx * dx + dy * dy + dz * dz);
            }
      }
    }
    return E;
  }

  // ---- MD sub-cycle (Sec. 2, Eq. (SPValgo) without constraints) ------------
  // n_sub sub-steps of h = 1/n_sub with the fluid velocity at each bead
  // frozen at its start-of-step value u_p:
  //   r += h/2 v;  v = e v + (1-e)/(m gamma) (F^c(r) + gamma u_p) + sig xi;  r += h/2 v
  // F^c includes the field.  The noise enters only through sig xi.  The
  // friction + noise impulse m[(1-e)(u_p - v_old) + sig xi] is the momentum
  // the bead takes from the fluid; J collects minus its sum.
  void md_subcycle(bool couple, bool field_on, uint32_t n_counter, bool allow_mts = true) {
    if (allow_mts && d.mts_outer > 0) {
      md_subcycle_mts(couple, field_on, n_counter);
      return;
    }
    if (d.constraints) {
      md_subcycle_constrained(couple, field_on, n_counter);
      return;
    }
    std::vector<R> Fc((size_t)3 * nb);
    for (int s = 0; s < d.n_sub; ++s) {
      for (int k = 0; k < 3 * nb; ++k) r[k] = r[k] + R(hh) * v[k];
      forces(r, Fc, field_on);
      for (int p = 0; p < nb; ++p) {
        double xi[3] = {0.0, 0.0, 0.0};
        if (val(sig) != 0.0) gauss3(d.seed, d.replica, n_counter, (uint32_t)s, (uint32_t)p, xi);
        for (int a = 0; a < 3; ++a) {
          R u = couple ? up[3 * p + a] : R(0.0);
          R vold = v[3 * p + a];
          R sx = sig * R(xi[a]);
          v[3 * p + a] = e * vold + cf * (Fc[3 * p + a] + gamma * u) + sx;
          J[3 * p + a] = J[3 * p + a] - R(m) * (omE * (u - vold) + sx);
        }
      }
      for (int k = 0; k < 3 * nb; ++k) r[k] = r[k] + R(hh) * v[k];
    }
  }

  // ---- rigid bonds (Sec. 2, Eq. (SPValgo) with its SHAKE and RATTLE steps) ---
  // Constraints sigma_k = |s_k|^2 - r0^2 = 0, s_k = r_k - r_{k+1}, replace the
  // harmonic bonds (equal masses).  For a linear chain both projections are
  // tridiagonal systems in the bond multipliers, solved directly (Thomas
  // algorithm): RATTLE's is linear and needs one solve; SHAKE's is solved by
  // Newton iterations, each a tridiagonal solve of the linearised
  // constraints, until the worst bond is within SHAKE_TOL r0^2 (at most
  // CONSTRAINT_MAXIT iterations, else the run is flagged).  Bead p takes the
  // corrections of its bonds p (+) and p-1 (-) in that order.
  static constexpr double SHAKE_TOL = 1e-13;
  static constexpr int CONSTRAINT_MAXIT = 50;
  bool constraint_failed = false;
  // x solves a[k] x[k-1] + b[k] x[k] + c[k] x[k+1] = d[k], k = 0..n-1
  static void tridiag(int n, const std::vector<R>& a, const std::vector<R>& b, const std::vector<R>& c,
                      const std::vector<R>& d, std::vector<R>& x) {
    std::vector<R> cp((size_t)n), dp((size_t)n);
    cp[0] = c[0] / b[0];
    dp[0] = d[0] / b[0];
    for (int k = 1; k < n; ++k) {
      const R den = b[k] - a[k] * cp[k - 1];
      cp[k] = c[k] / den;
      dp[k] = (d[k] - a[k] * dp[k - 1]) / den;
    }
    x.assign((size_t)n, R(0.0));
    x[n - 1] = dp[n - 1];
    for (int k = n - 2; k >= 0; --k) x[k] = dp[k] - cp[k] * x[k + 1];
  }
  static R dot3(const R* u, const R* w) { return u[0] * w[0] + u[1] * w[1] + u[2] * w[2]; }
  // bead p += lam[p] e[p] - lam[p-1] e[p-1]  (e[k]: the vector of bond k)
  void apply_bonds(std::vector<R>& y, const std::vector<R>& lam, const std::vector<R>& e) const {
    for (int p = 0; p < nb; ++p)
      for (int a = 0; a < 3; ++a) {
        if (p < nb - 1) y[3 * p + a] = y[3 * p + a] + lam[p] * e[3 * p + a];
        if (p > 0) y[3 * p + a] = y[3 * p + a] - lam[p - 1] * e[3 * (p - 1) + a];
      }
  }
  // SHAKE: moves x (the drifted positions) along the bond vectors of ref
  // (the positions before the drift) until every bond has length r0.  The
  // correction dx is accumulated apart from x (x = x_drifted + dx), so that
  // the velocity impulse dx / (h/2) keeps its relative precision; dx is
  // returned in *dx_out when given.
  void shake(std::vector<R>& x, const std::vector<R>& ref, std::vector<R>* dx_out = nullptr) {
    const int nbond = nb - 1;
    std::vector<R> dx((size_t)3 * nb, R(0.0));
    if (nbond < 1) {
      if (dx_out) *dx_out = dx;
      return;
    }
    const double d2 = d.r0 * d.r0;
    const std::vector<R> x0 = x;
    std::vector<R> rv((size_t)3 * nbond), sv((size_t)3 * nbond), a(nbond), b(nbond), c(nbond), rhs(nbond), dl;
    for (int k = 0; k < nbond; ++k)
      for (int q = 0; q < 3; ++q) rv[3 * k + q] = ref[3 * k + q] - ref[3 * (k + 1) + q];
    auto finish = [&]() {
      for (int k = 0; k < 3 * nb; ++k) x[k] = x0[k] + dx[k];
      if (dx_out) *dx_out = dx;
    };
    for (int it = 0;; ++it) {
      double worst = 0.0;
      for (int k = 0; k < nbond; ++k) {
        for (int q = 0; q < 3; ++q)
          sv[3 * k + q] = (x0[3 * k + q] + dx[3 * k + q]) - (x0[3 * (k + 1) + q] + dx[3 * (k + 1) + q]);
        const R sig = dot3(&sv[3 * k], &sv[3 * k]) - R(d2);
        rhs[k] = -sig;
        worst = std::max(worst, std::fabs(val(sig)));
      }
      if (worst <= SHAKE_TOL * d2) { finish(); return; }
      if (it == CONSTRAINT_MAXIT) { constraint_failed = true; finish(); return; }
      for (int k = 0; k < nbond; ++k) {
        b[k] = R(4.0) * dot3(&sv[3 * k], &rv[3 * k]);
        a[k] = k > 0 ? R(-2.0) * dot3(&sv[3 * k], &rv[3 * (k - 1)]) : R(0.0);
        c[k] = k < nbond - 1 ? R(-2.0) * dot3(&sv[3 * k], &rv[3 * (k + 1)]) : R(0.0);
      }
      tridiag(nbond, a, b, c, rhs, dl);
      apply_bonds(dx, dl, rv);
    }
  }
  // RATTLE: removes from vel the relative velocity along every bond of x.
  void rattle(std::vector<R>& vel, const std::vector<R>& x) {
    const int nbond = nb - 1;
    if (nbond < 1) return;
    std::vector<R> rv((size_t)3 * nbond), a(nbond), b(nbond), c(nbond), rhs(nbond), mu;
    for (int k = 0; k < nbond; ++k)
      for (int q = 0; q < 3; ++q) rv[3 * k + q] = x[3 * k + q] - x[3 * (k + 1) + q];
    for (int k = 0; k < nbond; ++k) {
      R w[3];
      for (int q = 0; q < 3; ++q) w[q] = vel[3 * k + q] - vel[3 * (k + 1) + q];
      rhs[k] = -dot3(&rv[3 * k], w);
      b[k] = R(2.0) * dot3(&rv[3 * k], &rv[3 * k]);
      a[k] = k > 0 ? -dot3(&rv[3 * k], &rv[3 * (k - 1)]) : R(0.0);
      c[k] = k < nbond - 1 ? -dot3(&rv[3 * k], &rv[3 * (k + 1)]) : R(0.0);
    }
    tridiag(nbond, a, b, c, rhs, mu);
    apply_bonds(vel, mu, rv);
  }
  // The uniform sub-cycle with rigid bonds: per sub-step
  //   ref = r;  r += h/2 v;  SHAKE(r; ref), and v takes the same constraint
  //   impulse, v += dx / (h/2) with dx the SHAKE correction;
  //   v = e v + (1-e)/(m gamma) (F(r) + gamma u_p) + sig xi   (F without bonds);
  //   RATTLE(v; r);  r += h/2 v
  // Reading: the printed scheme moves the positions onto the constraints
  // without the velocity; the constraint force acts during the drift, so the
  // velocity takes its impulse too (else every RATTLE removes the velocity
  // the bond's rotation turned along it, and a free rigid rotor loses energy
  // step after step).  J collects the friction + noise impulse as in the
  // unconstrained cycle (the constraint corrections are internal and carry
  // no momentum).
  void md_subcycle_constrained(bool couple, bool field_on, uint32_t n_counter) {
    std::vector<R> Fc((size_t)3 * nb), ref, dx;
    for (int s = 0; s < d.n_sub; ++s) {
      ref = r;
      for (int k = 0; k < 3 * nb; ++k) r[k] = r[k] + R(hh) * v[k];
      shake(r, ref, &dx);
      for (int k = 0; k < 3 * nb; ++k) v[k] = v[k] + dx[k] / R(hh);
      forces(r, Fc, field_on);
      for (int p = 0; p < nb; ++p) {
        double xi[3] = {0.0, 0.0, 0.0};
        if (val(sig) != 0.0) gauss3(d.seed, d.replica, n_counter, (uint32_t)s, (uint32_t)p, xi);
        for (int a = 0; a < 3; ++a) {
          R u = couple ? up[3 * p + a] : R(0.0);
          R vold = v[3 * p + a];
          R sx = sig * R(xi[a]);
          v[3 * p + a] = e * vold + cf * (Fc[3 * p + a] + gamma * u) + sx;
          J[3 * p + a] = J[3 * p + a] - R(m) * (omE * (u - vold) + sx);
        }
      }
      rattle(v, r);
      for (int k = 0; k < 3 * nb; ++k) r[k] = r[k] + R(hh) * v[k];
    }
  }

  // ---- multiple-time-step sub-cycle (Sec. 2, the nested cycle over the
  // bonds; read as a RESPA split, the printed inner loop moving no position):
  // M outer steps of dt = 1/M.  Each opens and closes with a half kick of the
  // slow forces, v += (dt/2)/m F_s(r), around M_b = n_sub/M SPV sub-steps of
  // h = 1/n_sub with the bonded forces only:
  //   r += h/2 v;  v = e v + (1-e)/(m gamma) (F_b(r) + gamma u_p) + sig xi;  r += h/2 v
  // Sub-step i of outer step o draws the noise of sub-step index o M_b + i;
  // J collects the friction + noise impulse of every sub-step as in the
  // uniform cycle.
  void md_subcycle_mts(bool couple, bool field_on, uint32_t n_counter) {
    const int M = d.mts_outer, Mb = d.n_sub / M;
    const R kick = R(0.5 * (1.0 / (double)M) / m);
    std::vector<R> Fs((size_t)3 * nb), Fb((size_t)3 * nb);
    for (int o = 0; o < M; ++o) {
      slow_forces(r, Fs, field_on);
      for (int k = 0; k < 3 * nb; ++k) v[k] = v[k] + kick * Fs[k];
      for (int i = 0; i < Mb; ++i) {
        const int s = o * Mb + i;
        for (int k = 0; k < 3 * nb; ++k) r[k] = r[k] + R(hh) * v[k];
        fast_forces(r, Fb);
        for (int p = 0; p < nb; ++p) {
          double xi[3] = {0.0, 0.0, 0.0};
          if (val(sig) != 0.0) gauss3(d.seed, d.replica, n_counter, (uint32_t)s, (uint32_t)p, xi);
          for (int a = 0; a < 3; ++a) {
            R u = couple ? up[3 * p + a] : R(0.0);
            R vold = v[3 * p + a];
            R sx = sig * R(xi[a]);
            v[3 * p + a] = e * vold + cf * (Fb[3 * p + a] + gamma * u) + sx;
            J[3 * p + a] = J[3 * p + a] - R(m) * (omE * (u - vold) + sx);
          }
        }
        for (int k = 0; k < 3 * nb; ++k) r[k] = r[k] + R(hh) * v[k];
      }
      slow_forces(r, Fs, field_on);
      for (int k = 0; k < 3 * nb; ++k) v[k] = v[k] + kick * Fs[k];
    }
  }

  // One coupled step: gather u_p at r(n) from the stored populations, the MD
  // sub-cycle, spreading of J at the same r(n), one LB step.
  void couple_step() {
    rstart = r;
    gather(rstart, up);
    std::fill(J.begin(), J.end(), R(0.0));
    md_subcycle(true, true, (uint32_t)step);
    spread(rstart, J);
    lb_sweep();
    ++step;
  }
  // Fluid-only LB step (body force only).
  void lb_step() {
    std::fill(F.begin(), F.end(), R(0.0));
    lb_sweep();
    ++step;
  }
  // Pre-relaxation of the chain (Sec. 4: the initial walk is relaxed by MD):
  // the same SPV sub-steps with no fluid, no field, no noise and friction
  // gamma_relax; velocities are zeroed at the end.
  void md_relax(int nsub_total, double gamma_relax) {
    R g_save = gamma;
    R e_s = e, omE_s = omE, cf_s = cf, sig_s = sig;
    gamma = R(gamma_relax);
    set_spv_coefficients(gamma, 0.0);
    std::vector<R> Jsave = J;
    int save_nsub = d.n_sub;
    int left = nsub_total;
    while (left > 0) {
      d.n_sub = std::min(left, save_nsub);
      md_subcycle(false, false, 0u, false);
      left -= d.n_sub;
    }
    d.n_sub = save_nsub;
    J = Jsave;
    for (auto& x : v) x = R(0.0);
    gamma = g_save;
    e = e_s; omE = omE_s; cf = cf_s; sig = sig_s;
  }

  // ---- observables -----------------------------------------------------------
  // out: [0] fluid mass, [1..3] fluid momentum (fluid nodes only), [4] bead kinetic temperature
  // m<v^2>/3, [5..7] bead momentum, [8] mean normal coordinate (unwrapped),
  // [9] translocated fraction, [10] beads in the field region, [11] R_U,
  // [12] R_T, [13] R_eff (nu = 0.6, Eq. (R_eff)), [14] dW_H/dt = gamma sum v.u_p,
  // [15] dW_E/dt = sum F_drive.v, [16..18] bounce-back wall ledger,
  // [19..21] spread-on-solid ledger, [22] step, [23] drag on the
  // untranslocated part, [24] drag on the translocated part.
  void observables(double* out) const {
    for (int k = 0; k < 25; ++k) out[k] = 0.0;
    // Mass and momentum are accumulated as deviations from the rest state
    // (f_i - w_i), which keeps the FP64 sums accurate; the fluid node count is
    // added at the end (sum_i w_i c_i = 0).
    long nfluid = 0;
    for (long c = 0; c < N; ++c) {
      if (solid[c]) continue;
      ++nfluid;
      for (int i = 0; i < Q; ++i) {
        double f = val(A[(size_t)i * N + c]) - weight(i);
        out[0] += f;
        for (int a = 0; a < 3; ++a) out[1 + a] += f * CV[i][a];
      }
    }
    out[0] += (double)nfluid;
    if (nb > 0) {
      int an = d.wall_axis >= 0 ? d.wall_axis : 2;
      double ke = 0.0, zsum = 0.0;
      int ntr = 0, nres = 0;
      double cu[3] = {0, 0, 0}, ct[3] = {0, 0, 0};
      int nu = 0, nt = 0;
      for (int p = 0; p < nb; ++p) {
        for (int a = 0; a < 3; ++a) {
          double vv = val(v[3 * p + a]);
          ke += vv * vv;
          out[5 + a] += m * vv;
        }
        double zn = val(r[3 * p + an]);
        zsum += zn;
        bool tr = d.wall_axis >= 0 && zn > (double)d.wall_pos;
        if (tr) { ++ntr; ++nt; for (int a = 0; a < 3; ++a) ct[a] += val(r[3 * p + a]); }
        else { ++nu; for (int a = 0; a < 3; ++a) cu[a] += val(r[3 * p + a]); }
        bool res = in_field(&r[3 * p]);
        if (res) {
          ++nres;
          out[15] += val(fdrive) * val(v[3 * p + an]);
        }
        for (int a = 0; a < 3; ++a) out[14] += val(gamma) * val(v[3 * p + a]) * val(up[3 * p + a]);
        // viscous drag along the wall normal, m gamma (u_p - v), on the
        // untranslocated [23] and translocated [24] parts (Sec. 4)
        const double drag = m * val(gamma) * (val(up[3 * p + an]) - val(v[3 * p + an]));
        out[tr ? 24 : 23] += drag;
      }
      out[4] = m * ke / (3.0 * nb);
      out[8] = zsum / nb;
      out[9] = (double)ntr / nb;
      out[10] = (double)nres;
      for (int a = 0; a < 3; ++a) { if (nu) cu[a] /= nu; if (nt) ct[a] /= nt; }
      double ru = 0.0, rt = 0.0;
      for (int p = 0; p < nb; ++p) {
        double zn = val(r[3 * p + an]);
        bool tr = d.wall_axis >= 0 && zn > (double)d.wall_pos;
        double s = 0.0;
        for (int a = 0; a < 3; ++a) {
          double dd = val(r[3 * p + a]) - (tr ? ct[a] : cu[a]);
          s += dd * dd;
        }
        if (tr) rt += s; else ru += s;
      }
      out[11] = nu ? std::sqrt(ru / nu) : 0.0;
      out[12] = nt ? std::sqrt(rt / nt) : 0.0;
      out[13] = std::pow(std::pow(out[12], 0.6) + std::pow(out[11], 0.6), 1.0 / 0.6);
    }
    for (int a = 0; a < 3; ++a) { out[16 + a] = val(ledger_bb[a]); out[19 + a] = val(ledger_sp[a]); }
    out[22] = (double)step;
  }
};

}  // namespace orc

using orc::Dual;
using orc::Sim;

extern "C" {

typedef Sim<double> SimD;

void* or_create(const or_desc* d, const double* r0, const double* v0) {
  if (!d || d->nx <= 0 || d->ny <= 0 || d->nz <= 0 || !(d->tau > 0.5) || d->n_sub <= 0) return nullptr;
  if (d->mts_outer < 0 || (d->mts_outer > 0 && d->n_sub % d->mts_outer != 0)) return nullptr;
  if (d->coupling != 0 && d->coupling != 1) return nullptr;
  if (d->constraints != 0 && (d->constraints != 1 || d->mts_outer > 0)) return nullptr;
  SimD* s = new SimD();
  s->init(*d, r0, v0);
  return s;
}
void or_destroy(void* h) { delete (SimD*)h; }
long long or_num_cells(void* h) { return ((SimD*)h)->N; }
void or_set_threads(int n) {
#ifdef _OPENMP
  omp_set_num_threads(n);
#else
  (void)n;
#endif
}
int or_max_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}
void or_lb_step(void* h, int nsteps) { for (int k = 0; k < nsteps; ++k) ((SimD*)h)->lb_step(); }
void or_couple_step(void* h, int nsteps) { for (int k = 0; k < nsteps; ++k) ((SimD*)h)->couple_step(); }
void or_md_relax(void* h, int nsub_total, double gamma_relax) { ((SimD*)h)->md_relax(nsub_total, gamma_relax); }
void or_get_pops(void* h, double* out) { auto* s = (SimD*)h; std::memcpy(out, s->A.data(), sizeof(double) * s->A.size()); }
void or_set_pops(void* h, const double* in) { auto* s = (SimD*)h; std::memcpy(s->A.data(), in, sizeof(double) * s->A.size()); }
void or_get_flags(void* h, uint8_t* out) { auto* s = (SimD*)h; std::memcpy(out, s->solid.data(), s->N); }
void or_get_beads(void* h, double* r, double* v, double* up, double* J) {
  auto* s = (SimD*)h;
  size_t n = (size_t)3 * s->nb;
  if (r) std::memcpy(r, s->r.data(), n * sizeof(double));
  if (v) std::memcpy(v, s->v.data(), n * sizeof(double));
  if (up) std::memcpy(up, s->up.data(), n * sizeof(double));
  if (J) std::memcpy(J, s->J.data(), n * sizeof(double));
}
void or_set_beads(void* h, const double* r, const double* v) {
  auto* s = (SimD*)h;
  size_t n = (size_t)3 * s->nb;
  if (r) std::memcpy(s->r.data(), r, n * sizeof(double));
  if (v) std::memcpy(s->v.data(), v, n * sizeof(double));
}
// Sets the fluid velocity at the beads, u_p (the value the next observables
// read; a coupled step overwrites it with its gather).
void or_set_up(void* h, const double* up) {
  auto* s = (SimD*)h;
  std::memcpy(s->up.data(), up, (size_t)3 * s->nb * sizeof(double));
}
void or_get_force(void* h, double* out) { auto* s = (SimD*)h; std::memcpy(out, s->F.data(), sizeof(double) * s->F.size()); }
void or_observables(void* h, double* out) { ((SimD*)h)->observables(out); }
long long or_step_count(void* h) { return ((SimD*)h)->step; }

// Pieces exposed for the pins.
void or_tables(int* c, double* w, int* opp) {
  for (int i = 0; i < orc::Q; ++i) {
    for (int a = 0; a < 3; ++a) c[3 * i + a] = orc::CV[i][a];
    w[i] = orc::weight(i);
    opp[i] = orc::OPP[i];
  }
}
void or_feq(double rho, const double* u, double* out) {
  for (int i = 0; i < orc::Q; ++i) out[i] = SimD::feq(i, rho, u);
}
void or_collide(void* h, const double* f, const double* F, double* out) { ((SimD*)h)->collide(f, F, out); }
void or_philox4x32_10(const uint32_t* ctr, const uint32_t* key, uint32_t* out) { orc::philox4x32_10(ctr, key, out); }
double or_mode_poly(int k, int i) { return orc::mode_poly(k, i); }
void or_fluid_normals(uint32_t seed, uint32_t rep, uint32_t n, uint32_t node, double* out) {
  orc::fluid_normals(seed, rep, n, node, out);
}
void or_gauss3(uint32_t seed, uint32_t rep, uint32_t n, uint32_t s, uint32_t p, double* out) {
  orc::gauss3(seed, rep, n, s, p, out);
}
void or_stencil(void* h, const double* rp, long long* nodes, double* W) {
  long nd[8];
  ((SimD*)h)->stencil(rp, nd, W);
  for (int k = 0; k < 8; ++k) nodes[k] = nd[k];
}
// u_p at the current bead positions from the current populations.
void or_gather(void* h, double* out) {
  auto* s = (SimD*)h;
  std::vector<double> tmp((size_t)3 * s->nb);
  s->gather(s->r, tmp);
  std::memcpy(out, tmp.data(), tmp.size() * sizeof(double));
}
// Force density from spreading J (nb x 3) at the current positions; [3][N].
void or_spread(void* h, const double* J, double* Fout) {
  auto* s = (SimD*)h;
  std::vector<double> Jv(J, J + 3 * s->nb);
  s->spread(s->r, Jv);
  std::memcpy(Fout, s->F.data(), sizeof(double) * s->F.size());
}
void or_forces(void* h, int field_on, double* out) {
  auto* s = (SimD*)h;
  std::vector<double> Fc((size_t)3 * s->nb);
  s->forces(s->r, Fc, field_on != 0);
  std::memcpy(out, Fc.data(), Fc.size() * sizeof(double));
}
// LJ force only, by all pairs (cells=0) or through the cell list (cells=1).
int or_lj_forces(void* h, int cells, double* out) {
  auto* s = (SimD*)h;
  std::vector<std::vector<int>> cand;
  if (cells) {
    for (int a = 0; a < 3; ++a)
      if ((int)std::floor((double)s->ext(a) / s->d.rc) < 3) return -1;
    s->build_candidates(s->r, cand);
  }
  for (int p = 0; p < s->nb; ++p) {
    double Fp[3] = {0, 0, 0};
    s->lj_on_bead(s->r, p, cells ? &cand[p] : nullptr, Fp);
    for (int a = 0; a < 3; ++a) out[3 * p + a] = Fp[a];
  }
  return 0;
}
// Velocity of every node from the pulled populations (zero at solid nodes), [3][N].
void or_node_velocity_field(void* h, double* out) {
  auto* s = (SimD*)h;
  for (int z = 0; z < s->nz; ++z)
    for (int y = 0; y < s->ny; ++y)
      for (int x = 0; x < s->nx; ++x) {
        double u[3];
        s->node_velocity(x, y, z, u);
        long c = s->idx(x, y, z);
        for (int a = 0; a < 3; ++a) out[(size_t)a * s->N + c] = u[a];
      }
}
// MD sub-cycles alone (fluid decoupled: u_p = 0, J discarded), noise on,
// field as requested; the step counter advances as in a coupled step.
void or_md_only(void* h, int nsteps, int field_on) {
  auto* s = (SimD*)h;
  for (int k = 0; k < nsteps; ++k) {
    s->md_subcycle(false, field_on != 0, (uint32_t)s->step);
    ++s->step;
  }
}
double or_energy(void* h) { auto* s = (SimD*)h; return s->energy(s->r); }
// The constraint projections alone, on caller arrays [nb][3]; returns 1 if a
// projection ran out of sweeps at any point of the run so far.
void or_shake(void* h, double* x, const double* ref) {
  auto* s = (SimD*)h;
  std::vector<double> xv(x, x + 3 * s->nb), rv(ref, ref + 3 * s->nb);
  s->shake(xv, rv);
  std::memcpy(x, xv.data(), xv.size() * sizeof(double));
}
void or_rattle(void* h, double* vel, const double* x) {
  auto* s = (SimD*)h;
  std::vector<double> vv(vel, vel + 3 * s->nb), xv(x, x + 3 * s->nb);
  s->rattle(vv, xv);
  std::memcpy(vel, vv.data(), vv.size() * sizeof(double));
}
int or_constraint_failed(void* h) { return ((SimD*)h)->constraint_failed ? 1 : 0; }
int or_in_field(void* h, const double* rp) { return ((SimD*)h)->in_field(rp) ? 1 : 0; }
void or_set_use_cells(void* h, int on) { ((SimD*)h)->use_cells = on != 0; }
int or_get_use_cells(void* h) { return ((SimD*)h)->use_cells ? 1 : 0; }

// Forward-mode derivative of the loss L = mean_p (normal coordinate of r_p)
// after nsteps coupled steps, along the direction (dr0, dgamma, dfdrive),
// starting from positions r0 and velocities v0.  out[0] = L, out[1] = dL.
int or_jvp(const or_desc* d, const double* r0, const double* v0, int nsteps, const double* dr0,
           double dgamma, double dfdrive, double* out) {
  if (!d || d->nb <= 0 || d->wall_axis < 0) return -1;
  Sim<Dual> s;
  s.init(*d, r0, v0);
  for (int k = 0; k < 3 * d->nb; ++k) s.r[k] = Dual(r0[k], dr0 ? dr0[k] : 0.0);
  s.gamma = Dual(d->gamma, dgamma);
  s.fdrive = Dual(d->f_drive, dfdrive);
  s.set_spv_coefficients(s.gamma, d->kT);
  for (int k = 0; k < nsteps; ++k) s.couple_step();
  Dual L(0.0, 0.0);
  for (int p = 0; p < d->nb; ++p) L += s.r[3 * p + d->wall_axis];
  L = L / Dual((double)d->nb);
  out[0] = L.v;
  out[1] = L.d;
  return 0;
}

// As or_jvp, recording L and its derivative after every step: out[2 k],
// out[2 k + 1] after step k + 1 (k < nsteps).
int or_jvp_series(const or_desc* d, const double* r0, const double* v0, int nsteps, const double* dr0,
                  double dgamma, double dfdrive, double* out) {
  if (!d || d->nb <= 0 || d->wall_axis < 0) return -1;
  Sim<Dual> s;
  s.init(*d, r0, v0);
  for (int k = 0; k < 3 * d->nb; ++k) s.r[k] = Dual(r0[k], dr0 ? dr0[k] : 0.0);
  s.gamma = Dual(d->gamma, dgamma);
  s.fdrive = Dual(d->f_drive, dfdrive);
  s.set_spv_coefficients(s.gamma, d->kT);
  for (int k = 0; k < nsteps; ++k) {
    s.couple_step();
    Dual L(0.0, 0.0);
    for (int p = 0; p < d->nb; ++p) L += s.r[3 * p + d->wall_axis];
    L = L / Dual((double)d->nb);
    out[2 * k] = L.v;
    out[2 * k + 1] = L.d;
  }
  return 0;
}

}  // extern "C"
