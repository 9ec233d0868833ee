// lbmd_kernels.h -- kernel argument blocks and host-side launchers.
#pragma once

#include "lbmd_dev.h"

namespace lbmd {

struct LbParams {
  int nx, ny, nz, nxy, N;
  double omega;     // 1 / tau
  double g[3];      // body-force density
  int has_g;
};

struct BeadPtrs {
  double* r;    // [nb][3] unwrapped positions
  double* v;    // [nb][3]
  double* up;   // [nb][3] fluid velocity at the bead (frozen for the sub-cycle)
  double* J;    // [nb][3] momentum handed to the fluid this step
  double* rs;   // [nb][3] positions at the start of the step
};

struct MdWork {
  double* rmid0;  // [nb][3] positions at the force evaluation, double buffered
  double* rmid1;
  double* ref;    // [nb][3] positions at the last neighbour-list build
  int* nbr;       // [nb][MAXNBR]
  int* ncnt;      // [nb]
  uint32_t* rb;   // [4] rebuild flags (3-phase) + list-invalid flag
  double* xi;     // [n_sub][nb][3] noise of the current sub-cycle
};

template <typename T, bool DEV> void launch_fill_rest(void* pops, long N, hipStream_t s);
void launch_fill_i32(int* p, long n, int v, hipStream_t s);
void launch_fill_f64(double* p, long n, double v, hipStream_t s);
template <typename T, bool DEV>
void launch_lb(const void* A, void* B, const uint8_t* flags, const void* force, const LbParams& p, Ctrl* ctrl,
               int skip_forced, hipStream_t s);
template <typename T, bool DEV>
void launch_lb_forced(const void* A, void* B, const uint8_t* flags, const void* force, const LbParams& p, Ctrl* ctrl,
                      const int* touched, int maxlist, hipStream_t s);
template <typename T, bool DEV>
void launch_gather(const void* A, const uint8_t* flags, const LbParams& p, const Geom& g, const BeadPtrs& b, int nb,
                   hipStream_t s);
void launch_bead_prep(const BeadPtrs& b, const Geom& g, int nb, int* head, int* next, int* base, uint8_t* flags,
                      hipStream_t s);
template <typename T>
void launch_spread(const BeadPtrs& b, const Geom& g, int nb, const int* head, const int* next, uint8_t* flags,
                   void* force, int* touched, Ctrl* ctrl, hipStream_t s);
void launch_step_end(int nb, const int* base, int* head, const int* touched, uint8_t* flags, Ctrl* ctrl, int advance,
                     hipStream_t s);
template <typename T, bool DEV>
void launch_observables(const void* A, const uint8_t* flags, long N, double nfluid, double* part, int nparts,
                        const BeadPtrs& b, int nb, const Geom& g, const MdParams& P, const Ctrl* ctrl, double* out,
                        hipStream_t s);

// MD sub-cycle: n_sub launches, one per sub-step.
void launch_md_cycle(const BeadPtrs& b, const MdWork& w, const MdParams& P, const Geom& g, Ctrl* ctrl, int n_sub,
                     hipStream_t s);
void launch_md_invalidate(const MdWork& w, hipStream_t s);
void launch_zero_v(double* v, int nb, hipStream_t s);

}  // namespace lbmd
