// md_kernels.hip -- the bead sub-cycle: stochastic position Verlet sub-steps
// (Sec. 2, Eq. (SPValgo), no constraints) with the fluid velocity at each
// bead frozen for the whole cycle.  One launch per sub-step, one thread per
// bead; the positions at which forces are evaluated are double buffered so
// that every bead reads a consistent snapshot.
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
// in the same order.  A list is rebuilt (by a scan over all beads) in the
// launch after any bead has moved more than skin/2 since the last build; the
// flag is carried between launches in three rotating words.
#include "lbmd_kernels.h"

namespace lbmd {

// Reset the rebuild flags; word 3 is the "lists invalid" request from the
// host (initialisation, restored state).
__global__ void k_md_begin(uint32_t* rb) {
  rb[0] = rb[3];
  rb[1] = 0u;
  rb[2] = 0u;
  rb[3] = 0u;
}

__global__ void k_md_invalidate(uint32_t* rb) { rb[3] = 1u; }

// r_mid of sub-step 0 and the displacement check that decides whether the
// first launch rebuilds the lists.
__global__ void k_md_start(BeadPtrs b, MdWork w, MdParams P) {
  int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= P.nb) return;
  double d2 = 0.0;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    double x = b.r[3 * p + a] + P.hh * b.v[3 * p + a];
    w.rmid0[3 * p + a] = x;
    double d = x - w.ref[3 * p + a];
    d2 += d * d;
  }
  if (d2 > P.halfskin2) w.rb[0] = 1u;
}

__device__ inline void rebuild_list(const double* __restrict__ rin, const MdParams& P, const Geom& g, int p,
                                    const double rp[3], int* __restrict__ nbr, int* __restrict__ ncnt,
                                    Ctrl* __restrict__ ctrl) {
  int cnt = 0;
  for (int j = 0; j < P.nb; ++j) {
    if (j == p) continue;
    double d0 = min_image(rp[0] - rin[3 * j], g.nx);
    double d1 = min_image(rp[1] - rin[3 * j + 1], g.ny);
    double d2 = min_image(rp[2] - rin[3 * j + 2], g.nz);
    if (d0 * d0 + d1 * d1 + d2 * d2 < P.rlist2) {
      if (cnt < MAXNBR) nbr[(size_t)p * MAXNBR + cnt] = j;
      ++cnt;
    }
  }
  if (cnt > MAXNBR) { atomicOr(&ctrl->err, E_NBRLIST); cnt = MAXNBR; }
  ncnt[p] = cnt;
}

// Conservative force on bead p at positions rin, in a fixed order: bonds to
// p-1 and p+1, bending angles centred at p-1, p, p+1, LJ over the neighbour
// list, wall sites, field.
__device__ inline void bead_force(const double* __restrict__ rin, const MdParams& P, const Geom& g, int p,
                                  const double rp[3], const int* __restrict__ nbr, int cnt, double F[3]) {
  F[0] = 0.0; F[1] = 0.0; F[2] = 0.0;
  const int nb = P.nb;
  if (p > 0) bond_add(P, rp, &rin[3 * (p - 1)], F);
  if (p < nb - 1) bond_add(P, rp, &rin[3 * (p + 1)], F);
  if (p - 1 >= 1 && p - 1 <= nb - 2) angle_add(P, &rin[3 * (p - 2)], &rin[3 * (p - 1)], rp, 2, F);
  if (p >= 1 && p <= nb - 2) angle_add(P, &rin[3 * (p - 1)], rp, &rin[3 * (p + 1)], 1, F);
  if (p + 1 >= 1 && p + 1 <= nb - 2) angle_add(P, rp, &rin[3 * (p + 1)], &rin[3 * (p + 2)], 0, F);
  for (int k = 0; k < cnt; ++k) {
    int j = nbr[(size_t)p * MAXNBR + k];
    double d0 = min_image(rp[0] - rin[3 * j], g.nx);
    double d1 = min_image(rp[1] - rin[3 * j + 1], g.ny);
    double d2 = min_image(rp[2] - rin[3 * j + 2], g.nz);
    lj_add(P, d0, d1, d2, F);
  }
  wall_add(P, g, rp, F);
  if (P.field_on && in_field(g, rp)) F[g.wall_axis] += P.f_drive;
}

__global__ __launch_bounds__(256) void k_md_substep(BeadPtrs b, MdWork w, MdParams P, Geom g,
                                                    Ctrl* __restrict__ ctrl, int s, int last) {
  int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p == 0) w.rb[(s + 2) % 3] = 0u;
  if (p >= P.nb) return;
  const double* rin = (s & 1) ? w.rmid1 : w.rmid0;
  double* rout = (s & 1) ? w.rmid0 : w.rmid1;
  double rp[3] = {rin[3 * p], rin[3 * p + 1], rin[3 * p + 2]};
  if (w.rb[s % 3]) {
    rebuild_list(rin, P, g, p, rp, w.nbr, w.ncnt, ctrl);
    w.ref[3 * p] = rp[0]; w.ref[3 * p + 1] = rp[1]; w.ref[3 * p + 2] = rp[2];
  }
  double F[3];
  bead_force(rin, P, g, p, rp, w.nbr, w.ncnt[p], F);
  double xi[3] = {0.0, 0.0, 0.0};
  if (P.sig != 0.0) gauss3(P.seed, P.replica, (uint32_t)ctrl->step, (uint32_t)s, (uint32_t)p, xi);
  double vn[3];
  bool finite = true;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    double u = P.couple ? b.up[3 * p + a] : 0.0;
    double vold = b.v[3 * p + a];
    double sx = P.sig * xi[a];
    vn[a] = P.e * vold + P.cf * (F[a] + P.gamma * u) + sx;
    b.J[3 * p + a] = b.J[3 * p + a] - P.m * (P.omE * (u - vold) + sx);
    b.v[3 * p + a] = vn[a];
    finite = finite && isfinite(vn[a]);
  }
  if (!finite) atomicOr(&ctrl->err, E_BEADS);
  double re[3] = {rp[0] + P.hh * vn[0], rp[1] + P.hh * vn[1], rp[2] + P.hh * vn[2]};
  if (last) {
    b.r[3 * p] = re[0]; b.r[3 * p + 1] = re[1]; b.r[3 * p + 2] = re[2];
  } else {
    double d2 = 0.0;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      double x = re[a] + P.hh * vn[a];
      rout[3 * p + a] = x;
      double d = x - w.ref[3 * p + a];
      d2 += d * d;
    }
    if (d2 > P.halfskin2) w.rb[(s + 1) % 3] = 1u;
  }
}

__global__ void k_zero_v(double* v, int n) {
  int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) v[k] = 0.0;
}

void launch_md_invalidate(const MdWork& w, hipStream_t s) {
  hipLaunchKernelGGL(k_md_invalidate, dim3(1), dim3(1), 0, s, w.rb);
}

void launch_md_cycle(const BeadPtrs& b, const MdWork& w, const MdParams& P, const Geom& g, Ctrl* ctrl, int n_sub,
                     hipStream_t s) {
  if (P.nb <= 0 || n_sub <= 0) return;
  unsigned nblk = (unsigned)((P.nb + 255) / 256);
  hipLaunchKernelGGL(k_md_begin, dim3(1), dim3(1), 0, s, w.rb);
  hipLaunchKernelGGL(k_md_start, dim3(nblk), dim3(256), 0, s, b, w, P);
  for (int k = 0; k < n_sub; ++k)
    hipLaunchKernelGGL(k_md_substep, dim3(nblk), dim3(256), 0, s, b, w, P, g, ctrl, k, k == n_sub - 1 ? 1 : 0);
}

void launch_zero_v(double* v, int nb, hipStream_t s) {
  if (nb > 0) hipLaunchKernelGGL(k_zero_v, dim3((3 * nb + 255) / 256), dim3(256), 0, s, v, 3 * nb);
}

}  // namespace lbmd
