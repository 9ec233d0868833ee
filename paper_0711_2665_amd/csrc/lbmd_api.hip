// lbmd_api.hip -- host side of liblbmd: argument checking, geometry, buffer
// layout and the sequence of kernel launches of each entry point declared in
// include/lbmd.h.
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "lbmd.h"
#include "lbmd_kernels.h"

using namespace lbmd;

namespace {

thread_local std::string g_last_error = "no error";

int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return code;
}

int take_acc(const char* where);
int check_hip(const char* where) {
  int rc = take_acc(where);
  if (rc) return rc;
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(LB_ERR_DEVICE, "%s: %s", where, hipGetErrorString(e));
  return LB_OK;
}

// First failure among a sequence of asynchronous HIP calls.
thread_local hipError_t g_acc = hipSuccess;
inline void acc(hipError_t e) {
  if (e != hipSuccess && g_acc == hipSuccess) g_acc = e;
}
int take_acc(const char* where) {
  hipError_t e = g_acc;
  g_acc = hipSuccess;
  if (e != hipSuccess) return fail(LB_ERR_DEVICE, "%s: %s", where, hipGetErrorString(e));
  return LB_OK;
}

inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

constexpr int NPARTS = 1024;

struct WorkLayout {
  size_t ctrl, head, next, base, touched, nbr, ncnt, rb, rmid0, rmid1, ref, part, xi;
  size_t total;
};

WorkLayout work_layout(const lb_desc* d) {
  long N = (long)d->nx * d->ny * d->nz;
  int nb = d->nb;
  WorkLayout w;
  size_t o = 0;
  auto take = [&](size_t bytes) { size_t at = o; o += align256(bytes); return at; };
  size_t nbs = (size_t)(nb > 0 ? nb : 1);
  w.ctrl = take(sizeof(Ctrl));
  w.head = take(sizeof(int) * (size_t)N);
  w.next = take(sizeof(int) * nbs);
  w.base = take(sizeof(int) * nbs);
  w.touched = take(sizeof(int) * 8 * nbs);
  w.nbr = take(sizeof(int) * MAXNBR * nbs);
  w.ncnt = take(sizeof(int) * nbs);
  w.rb = take(sizeof(uint32_t) * 4);
  w.rmid0 = take(sizeof(double) * 3 * nbs);
  w.rmid1 = take(sizeof(double) * 3 * nbs);
  w.ref = take(sizeof(double) * 3 * nbs);
  w.part = take(sizeof(double) * 4 * NPARTS);
  w.xi = take(sizeof(double) * 3 * nbs * (size_t)(d->n_sub > 0 ? d->n_sub : 1));
  w.total = o;
  return w;
}

int validate(const lb_desc* d) {
  if (!d) return fail(LB_ERR_ARG, "null description");
  if (d->nx <= 0 || d->ny <= 0 || d->nz <= 0) return fail(LB_ERR_ARG, "extents must be positive");
  long N = (long)d->nx * d->ny * d->nz;
  if (N * (long)Q > 2147483647L) return fail(LB_ERR_ARG, "lattice too large: 19 N must fit in 31 bits");
  if (d->precision != LB_FP64 && d->precision != LB_FP32_DEV) return fail(LB_ERR_ARG, "unknown precision %d", d->precision);
  if (!(d->tau > 0.5)) return fail(LB_ERR_ARG, "tau must exceed 1/2 (got %g)", d->tau);
  for (int a = 0; a < 3; ++a)
    if (!std::isfinite(d->g[a])) return fail(LB_ERR_ARG, "body force must be finite");
  if (d->wall_axis < -1 || d->wall_axis > 2) return fail(LB_ERR_ARG, "wall_axis must be -1, 0, 1 or 2");
  if (d->wall_axis >= 0) {
    int n = d->wall_axis == 0 ? d->nx : (d->wall_axis == 1 ? d->ny : d->nz);
    if (d->wall_pos < 2 || d->wall_pos > n - 3) return fail(LB_ERR_ARG, "wall plane must lie in [2, n-3]");
    int t0 = d->wall_axis == 0 ? d->ny : d->nx;
    int t1 = d->wall_axis == 2 ? d->ny : d->nz;
    if (d->pore_h < 0 || d->pore_h > t0 || d->pore_h > t1) return fail(LB_ERR_ARG, "pore wider than the wall");
  }
  if (d->nb < 0) return fail(LB_ERR_ARG, "negative bead count");
  if (d->n_sub < 1) return fail(LB_ERR_ARG, "n_sub must be >= 1");
  if (d->nb > 0) {
    if (!(d->mass > 0.0)) return fail(LB_ERR_ARG, "bead mass must be positive");
    if (!(d->gamma >= 0.0) || !(d->kT >= 0.0)) return fail(LB_ERR_ARG, "gamma and kT must be >= 0");
    if (!(d->rc > 0.0) || d->rc > 2.0) return fail(LB_ERR_ARG, "rc must lie in (0, 2]");
    if (!(d->sigma > 0.0)) return fail(LB_ERR_ARG, "sigma must be positive");
    if ((long)d->nb * 8 > 2147483647L / 8) return fail(LB_ERR_ARG, "too many beads");
  }
  return LB_OK;
}

Geom make_geom(const lb_desc* d) {
  Geom g;
  g.nx = d->nx; g.ny = d->ny; g.nz = d->nz;
  g.nxy = d->nx * d->ny;
  g.N = (long)d->nx * d->ny * d->nz;
  g.wall_axis = d->wall_axis;
  g.wall_pos = d->wall_pos;
  g.t0 = d->wall_axis == 0 ? 1 : 0;
  g.t1 = d->wall_axis == 2 ? 1 : 2;
  if (d->wall_axis < 0) { g.t0 = 0; g.t1 = 1; }
  int n0 = ext(g, g.t0), n1 = ext(g, g.t1);
  g.lo0 = n0 / 2 - d->pore_h / 2; g.hi0 = g.lo0 + d->pore_h - 1;
  g.lo1 = n1 / 2 - d->pore_h / 2; g.hi1 = g.lo1 + d->pore_h - 1;
  return g;
}

// SPV coefficients for friction rate gamma and thermal energy kT.
void spv_coefficients(MdParams& P, double gamma, double kT, double h) {
  P.gamma = gamma;
  if (gamma == 0.0) {
    P.e = 1.0; P.omE = 0.0; P.cf = h / P.m; P.sig = 0.0;
    return;
  }
  P.e = std::exp(-(gamma * h));
  P.omE = 1.0 - P.e;
  P.cf = P.omE / (P.m * gamma);
  double var = (kT / P.m) * (1.0 - P.e * P.e);
  P.sig = kT > 0.0 ? std::sqrt(var) : 0.0;
}

}  // namespace

struct lb_ctx {
  lb_desc d;
  lb_buffers b;
  hipStream_t s;
  int cur;          // 0: pops_a holds the current populations
  Geom g;
  LbParams lp;
  MdParams mp;
  BeadPtrs bp;
  MdWork mw;
  WorkLayout wl;
  Ctrl* ctrl;
  int* head;
  int* next;
  int* base;
  int* touched;
  double* part;
  double nfluid;
  int64_t steps;
  int64_t last_touched = 0;
  bool dev;
  // second stream for the sweep over the nodes without bead force, which
  // runs concurrently with the bead phase; fork/join events
  hipStream_t s2 = nullptr;
  hipEvent_t fork = nullptr, join = nullptr;
  // kernel timing (lb_profile_start / lb_profile_stop)
  std::vector<hipEvent_t> ev;   // 4 per recorded step: bead start/end, LB start/end
  int prof_max = 0;
  int prof_n = 0;
  bool prof_on = false;
};

namespace {

void* cur_pops(lb_ctx* c) { return c->cur == 0 ? c->b.pops_a : c->b.pops_b; }
void* other_pops(lb_ctx* c) { return c->cur == 0 ? c->b.pops_b : c->b.pops_a; }

// Event slot k of the current recorded step (0, 1: bead phase; 2, 3: sweep),
// recorded on stream st.
void prof_mark(lb_ctx* c, int k, hipStream_t st) {
  if (!c->prof_on || c->prof_n >= c->prof_max) return;
  acc(hipEventRecord(c->ev[4 * (size_t)c->prof_n + k], st));
}
void prof_next(lb_ctx* c) {
  if (c->prof_on && c->prof_n < c->prof_max) ++c->prof_n;
}

void launch_lb_any(lb_ctx* c, int skip_forced, hipStream_t st) {
  if (c->dev)
    launch_lb<float, true>(cur_pops(c), other_pops(c), (const uint8_t*)c->b.flags, c->b.force, c->lp, c->ctrl,
                           skip_forced, st);
  else
    launch_lb<double, false>(cur_pops(c), other_pops(c), (const uint8_t*)c->b.flags, c->b.force, c->lp, c->ctrl,
                             skip_forced, st);
}

void launch_lb_forced_any(lb_ctx* c, hipStream_t st) {
  int maxlist = 8 * c->d.nb;
  if (c->dev)
    launch_lb_forced<float, true>(cur_pops(c), other_pops(c), (const uint8_t*)c->b.flags, c->b.force, c->lp,
                                  c->ctrl, c->touched, maxlist, st);
  else
    launch_lb_forced<double, false>(cur_pops(c), other_pops(c), (const uint8_t*)c->b.flags, c->b.force, c->lp,
                                    c->ctrl, c->touched, maxlist, st);
}

}  // namespace

extern "C" {

const char* lb_last_error(void) { return g_last_error.c_str(); }
void lb_destroy(lb_ctx* ctx);

int lb_buffer_sizes(const lb_desc* d, lb_sizes* out) {
  int rc = validate(d);
  if (rc) return rc;
  if (!out) return fail(LB_ERR_ARG, "null output");
  long N = (long)d->nx * d->ny * d->nz;
  size_t es = d->precision == LB_FP64 ? sizeof(double) : sizeof(float);
  size_t nbs = (size_t)(d->nb > 0 ? d->nb : 1);
  out->pops_bytes = align256(es * Q * (size_t)N);
  out->flags_bytes = align256((size_t)N);
  out->force_bytes = align256(es * 3 * (size_t)N);
  out->beads_bytes = align256(sizeof(double) * 15 * nbs);
  out->work_bytes = work_layout(d).total;
  out->state_bytes = align256(es * Q * (size_t)N) + align256(sizeof(double) * 6 * nbs) + 256;
  return LB_OK;
}

int lb_init(const lb_desc* d, const lb_buffers* b, const double* r0_host, const double* v0_host, void* stream,
            lb_ctx** out) {
  int rc = validate(d);
  if (rc) return rc;
  if (!b || !out) return fail(LB_ERR_ARG, "null buffers or output");
  const void* ptrs[6] = {b->pops_a, b->pops_b, b->flags, b->force, b->beads, b->work};
  for (int k = 0; k < 6; ++k) {
    if (!ptrs[k]) return fail(LB_ERR_ARG, "buffer %d is NULL", k);
    if (((uintptr_t)ptrs[k]) & 255) return fail(LB_ERR_ARG, "buffer %d is not 256-byte aligned", k);
  }
  if (d->nb > 0 && !r0_host) return fail(LB_ERR_ARG, "bead positions required");
  for (long k = 0; k < 3L * d->nb; ++k) {
    if (!std::isfinite(r0_host[k]) || (v0_host && !std::isfinite(v0_host[k])))
      return fail(LB_ERR_ARG, "non-finite bead state");
  }
  lb_ctx* c = new lb_ctx();
  c->d = *d;
  c->b = *b;
  c->s = (hipStream_t)stream;
  {
    hipError_t e1 = hipStreamCreateWithFlags(&c->s2, hipStreamNonBlocking);
    hipError_t e2 = hipEventCreateWithFlags(&c->fork, hipEventDisableTiming);
    hipError_t e3 = hipEventCreateWithFlags(&c->join, hipEventDisableTiming);
    if (e1 != hipSuccess || e2 != hipSuccess || e3 != hipSuccess) {
      lb_destroy(c);
      return fail(LB_ERR_DEVICE, "stream/event creation failed");
    }
  }
  c->cur = 0;
  c->dev = d->precision == LB_FP32_DEV;
  c->g = make_geom(d);
  long N = c->g.N;
  c->lp.nx = d->nx; c->lp.ny = d->ny; c->lp.nz = d->nz; c->lp.nxy = d->nx * d->ny; c->lp.N = (int)N;
  c->lp.omega = 1.0 / d->tau;
  for (int a = 0; a < 3; ++a) c->lp.g[a] = d->g[a];
  c->lp.has_g = (d->g[0] != 0.0 || d->g[1] != 0.0 || d->g[2] != 0.0) ? 1 : 0;

  MdParams& P = c->mp;
  std::memset(&P, 0, sizeof(P));
  P.nb = d->nb;
  P.n_sub = d->n_sub;
  double h = 1.0 / (double)d->n_sub;
  P.hh = 0.5 * h;
  P.m = d->nb > 0 ? d->mass : 1.0;
  P.k_bond = d->k_bond; P.r0 = d->r0; P.kappa = d->kappa;
  P.eps24 = 24.0 * d->eps; P.sig2 = d->sigma * d->sigma; P.rc2 = d->rc * d->rc;
  P.f_drive = d->f_drive;
  P.couple = 1; P.field_on = 1;
  P.seed = d->seed; P.replica = d->replica;
  P.rlist2 = (d->rc + SKIN) * (d->rc + SKIN);
  P.halfskin2 = (0.5 * SKIN) * (0.5 * SKIN);
  spv_coefficients(P, d->gamma, d->kT, h);

  size_t nbs = (size_t)(d->nb > 0 ? d->nb : 1);
  double* beads = (double*)b->beads;
  c->bp.r = beads; c->bp.v = beads + 3 * nbs; c->bp.up = beads + 6 * nbs; c->bp.J = beads + 9 * nbs;
  c->bp.rs = beads + 12 * nbs;
  c->wl = work_layout(d);
  char* w = (char*)b->work;
  c->ctrl = (Ctrl*)(w + c->wl.ctrl);
  c->head = (int*)(w + c->wl.head);
  c->next = (int*)(w + c->wl.next);
  c->base = (int*)(w + c->wl.base);
  c->touched = (int*)(w + c->wl.touched);
  c->part = (double*)(w + c->wl.part);
  c->mw.rmid0 = (double*)(w + c->wl.rmid0);
  c->mw.rmid1 = (double*)(w + c->wl.rmid1);
  c->mw.ref = (double*)(w + c->wl.ref);
  c->mw.nbr = (int*)(w + c->wl.nbr);
  c->mw.ncnt = (int*)(w + c->wl.ncnt);
  c->mw.rb = (uint32_t*)(w + c->wl.rb);
  c->mw.xi = (double*)(w + c->wl.xi);
  c->steps = 0;

  // geometry flags on the host (Sec. 4: wall plane with a square pore)
  std::vector<uint8_t> fl((size_t)N, 0);
  const Geom& g = c->g;
  long nfluid = 0;
  for (int z = 0; z < g.nz; ++z)
    for (int y = 0; y < g.ny; ++y)
      for (int x = 0; x < g.nx; ++x)
        if (site_solid(g, x, y, z)) fl[(size_t)x + (size_t)g.nx * ((size_t)y + (size_t)g.ny * z)] = F_SOLID;
  for (int z = 0; z < g.nz; ++z)
    for (int y = 0; y < g.ny; ++y)
      for (int x = 0; x < g.nx; ++x) {
        size_t cidx = (size_t)x + (size_t)g.nx * ((size_t)y + (size_t)g.ny * z);
        if (fl[cidx] & F_SOLID) continue;
        ++nfluid;
        for (int i = 1; i < Q; ++i)
          if (site_solid(g, x - cx(i), y - cy(i), z - cz(i))) { fl[cidx] |= F_NEAR; break; }
      }
  c->nfluid = (double)nfluid;

  hipError_t e = hipMemcpyAsync(b->flags, fl.data(), (size_t)N, hipMemcpyHostToDevice, c->s);
  if (e != hipSuccess) { lb_destroy(c); return fail(LB_ERR_DEVICE, "flag upload: %s", hipGetErrorString(e)); }
  if (c->dev) {
    launch_fill_rest<float, true>(b->pops_a, N, c->s);
    launch_fill_rest<float, true>(b->pops_b, N, c->s);
  } else {
    launch_fill_rest<double, false>(b->pops_a, N, c->s);
    launch_fill_rest<double, false>(b->pops_b, N, c->s);
  }
  acc(hipMemsetAsync(b->force, 0, (c->dev ? sizeof(float) : sizeof(double)) * 3 * (size_t)N, c->s));
  acc(hipMemsetAsync(b->beads, 0, sizeof(double) * 15 * nbs, c->s));
  acc(hipMemsetAsync(c->ctrl, 0, sizeof(Ctrl), c->s));
  launch_fill_i32(c->head, N, -1, c->s);
  launch_fill_f64(c->mw.ref, 3L * (long)nbs, 1e300, c->s);
  acc(hipMemsetAsync(c->mw.ncnt, 0, sizeof(int) * nbs, c->s));
  acc(hipMemsetAsync(c->mw.rb, 0, 16, c->s));
  launch_md_invalidate(c->mw, c->s);
  if (d->nb > 0) {
    acc(hipMemcpyAsync(c->bp.r, r0_host, sizeof(double) * 3 * d->nb, hipMemcpyHostToDevice, c->s));
    if (v0_host) acc(hipMemcpyAsync(c->bp.v, v0_host, sizeof(double) * 3 * d->nb, hipMemcpyHostToDevice, c->s));
  }
  e = hipStreamSynchronize(c->s);
  if (e != hipSuccess) { lb_destroy(c); return fail(LB_ERR_DEVICE, "init: %s", hipGetErrorString(e)); }
  rc = check_hip("init");
  if (rc) { lb_destroy(c); return rc; }
  *out = c;
  return LB_OK;
}

void lb_destroy(lb_ctx* ctx) {
  if (!ctx) return;
  if (ctx->s2) (void)hipStreamSynchronize(ctx->s2);
  for (hipEvent_t e : ctx->ev) (void)hipEventDestroy(e);
  if (ctx->fork) (void)hipEventDestroy(ctx->fork);
  if (ctx->join) (void)hipEventDestroy(ctx->join);
  if (ctx->s2) (void)hipStreamDestroy(ctx->s2);
  delete ctx;
}

int lb_profile_start(lb_ctx* c, int max_steps) {
  if (!c || max_steps < 1) return fail(LB_ERR_ARG, "bad arguments");
  if (c->prof_on) return fail(LB_ERR_ARG, "profiling already active");
  size_t need = 4 * (size_t)max_steps;
  while (c->ev.size() < need) {
    hipEvent_t e;
    hipError_t r = hipEventCreate(&e);
    if (r != hipSuccess) return fail(LB_ERR_DEVICE, "hipEventCreate: %s", hipGetErrorString(r));
    c->ev.push_back(e);
  }
  c->prof_max = max_steps;
  c->prof_n = 0;
  c->prof_on = true;
  return LB_OK;
}

int lb_profile_stop(lb_ctx* c, double* mean_lb_ms, double* mean_bead_ms, int* nsteps) {
  if (!c) return fail(LB_ERR_ARG, "null context");
  if (!c->prof_on) return fail(LB_ERR_ARG, "profiling not active");
  c->prof_on = false;
  hipError_t r = hipStreamSynchronize(c->s);
  if (r == hipSuccess) r = hipStreamSynchronize(c->s2);
  if (r != hipSuccess) return fail(LB_ERR_DEVICE, "stream: %s", hipGetErrorString(r));
  double tl = 0.0, tb = 0.0;
  for (int k = 0; k < c->prof_n; ++k) {
    float a = 0.f, b = 0.f;
    r = hipEventElapsedTime(&b, c->ev[4 * (size_t)k], c->ev[4 * (size_t)k + 1]);
    if (r != hipSuccess) return fail(LB_ERR_DEVICE, "event time: %s", hipGetErrorString(r));
    r = hipEventElapsedTime(&a, c->ev[4 * (size_t)k + 2], c->ev[4 * (size_t)k + 3]);
    if (r != hipSuccess) return fail(LB_ERR_DEVICE, "event time: %s", hipGetErrorString(r));
    tl += a;
    tb += b;
  }
  int n = c->prof_n;
  if (mean_lb_ms) *mean_lb_ms = n ? tl / n : 0.0;
  if (mean_bead_ms) *mean_bead_ms = n ? tb / n : 0.0;
  if (nsteps) *nsteps = n;
  return take_acc("lb_profile_stop");
}

int lb_step(lb_ctx* c, int nsteps) {
  if (!c || nsteps < 0) return fail(LB_ERR_ARG, "bad arguments");
  for (int k = 0; k < nsteps; ++k) {
    prof_mark(c, 0, c->s);
    prof_mark(c, 1, c->s);
    prof_mark(c, 2, c->s);
    launch_lb_any(c, 0, c->s);
    prof_mark(c, 3, c->s);
    launch_step_end(0, c->base, c->head, c->touched, (uint8_t*)c->b.flags, c->ctrl, 1, c->s);
    c->cur ^= 1;
    prof_next(c);
  }
  c->steps += nsteps;
  return check_hip("lb_step");
}

int md_couple_step(lb_ctx* c, int nsteps) {
  if (!c || nsteps < 0) return fail(LB_ERR_ARG, "bad arguments");
  const int nb = c->d.nb;
  uint8_t* flags = (uint8_t*)c->b.flags;
  for (int k = 0; k < nsteps; ++k) {
    if (nb == 0) {
      prof_mark(c, 0, c->s);
      prof_mark(c, 1, c->s);
      prof_mark(c, 2, c->s);
      launch_lb_any(c, 0, c->s);
      prof_mark(c, 3, c->s);
    } else {
      // the stencil nodes of r(n) are marked first; the sweep over all other
      // nodes then runs on the second stream while the beads move
      prof_mark(c, 0, c->s);
      launch_bead_prep(c->bp, c->g, nb, c->head, c->next, c->base, flags, c->s);
      acc(hipEventRecord(c->fork, c->s));
      acc(hipStreamWaitEvent(c->s2, c->fork, 0));
      prof_mark(c, 2, c->s2);
      launch_lb_any(c, 1, c->s2);
      prof_mark(c, 3, c->s2);
      acc(hipEventRecord(c->join, c->s2));
      if (c->dev) launch_gather<float, true>(cur_pops(c), flags, c->lp, c->g, c->bp, nb, c->s);
      else launch_gather<double, false>(cur_pops(c), flags, c->lp, c->g, c->bp, nb, c->s);
      launch_md_cycle(c->bp, c->mw, c->mp, c->g, c->ctrl, c->d.n_sub, c->s);
      if (c->dev) launch_spread<float>(c->bp, c->g, nb, c->head, c->next, flags, c->b.force, c->touched, c->ctrl, c->s);
      else launch_spread<double>(c->bp, c->g, nb, c->head, c->next, flags, c->b.force, c->touched, c->ctrl, c->s);
      launch_lb_forced_any(c, c->s);
      prof_mark(c, 1, c->s);
      acc(hipStreamWaitEvent(c->s, c->join, 0));
    }
    launch_step_end(nb, c->base, c->head, c->touched, flags, c->ctrl, 1, c->s);
    c->cur ^= 1;
    prof_next(c);
  }
  c->steps += nsteps;
  return check_hip("md_couple_step");
}

int md_relax(lb_ctx* c, int nsub_total, double gamma_relax) {
  if (!c || nsub_total < 0 || !(gamma_relax >= 0.0)) return fail(LB_ERR_ARG, "bad arguments");
  if (c->d.nb == 0) return LB_OK;
  MdParams P = c->mp;
  P.couple = 0;
  P.field_on = 0;
  spv_coefficients(P, gamma_relax, 0.0, 1.0 / (double)c->d.n_sub);
  int left = nsub_total;
  while (left > 0) {
    int n = left < c->d.n_sub ? left : c->d.n_sub;
    launch_md_cycle(c->bp, c->mw, P, c->g, c->ctrl, n, c->s);
    left -= n;
  }
  launch_zero_v(c->bp.v, c->d.nb, c->s);
  return check_hip("md_relax");
}

int lb_observables(lb_ctx* c, double* out_dev) {
  if (!c || !out_dev) return fail(LB_ERR_ARG, "bad arguments");
  if (c->dev)
    launch_observables<float, true>(cur_pops(c), (const uint8_t*)c->b.flags, c->g.N, c->nfluid, c->part, NPARTS,
                                    c->bp, c->d.nb, c->g, c->mp, c->ctrl, out_dev, c->s);
  else
    launch_observables<double, false>(cur_pops(c), (const uint8_t*)c->b.flags, c->g.N, c->nfluid, c->part, NPARTS,
                                      c->bp, c->d.nb, c->g, c->mp, c->ctrl, out_dev, c->s);
  return check_hip("lb_observables");
}

static size_t pops_state_bytes(const lb_ctx* c) {
  size_t es = c->dev ? sizeof(float) : sizeof(double);
  return align256(es * Q * (size_t)c->g.N);
}

int lb_get_state(lb_ctx* c, void* dst) {
  if (!c || !dst) return fail(LB_ERR_ARG, "bad arguments");
  size_t es = c->dev ? sizeof(float) : sizeof(double);
  size_t nbs = (size_t)(c->d.nb > 0 ? c->d.nb : 1);
  char* o = (char*)dst;
  acc(hipMemcpyAsync(o, cur_pops(c), es * Q * (size_t)c->g.N, hipMemcpyDeviceToDevice, c->s));
  o += pops_state_bytes(c);
  if (c->d.nb > 0) {
    acc(hipMemcpyAsync(o, c->bp.r, sizeof(double) * 3 * c->d.nb, hipMemcpyDeviceToDevice, c->s));
    acc(hipMemcpyAsync(o + sizeof(double) * 3 * nbs, c->bp.v, sizeof(double) * 3 * c->d.nb, hipMemcpyDeviceToDevice, c->s));
  }
  o += align256(sizeof(double) * 6 * nbs);
  acc(hipMemcpyAsync(o, &c->ctrl->step, sizeof(uint64_t), hipMemcpyDeviceToDevice, c->s));
  return check_hip("lb_get_state");
}

int lb_set_state(lb_ctx* c, const void* src) {
  if (!c || !src) return fail(LB_ERR_ARG, "bad arguments");
  size_t es = c->dev ? sizeof(float) : sizeof(double);
  size_t nbs = (size_t)(c->d.nb > 0 ? c->d.nb : 1);
  const char* o = (const char*)src;
  acc(hipMemcpyAsync(cur_pops(c), o, es * Q * (size_t)c->g.N, hipMemcpyDeviceToDevice, c->s));
  o += pops_state_bytes(c);
  if (c->d.nb > 0) {
    acc(hipMemcpyAsync(c->bp.r, o, sizeof(double) * 3 * c->d.nb, hipMemcpyDeviceToDevice, c->s));
    acc(hipMemcpyAsync(c->bp.v, o + sizeof(double) * 3 * nbs, sizeof(double) * 3 * c->d.nb, hipMemcpyDeviceToDevice, c->s));
  }
  o += align256(sizeof(double) * 6 * nbs);
  acc(hipMemcpyAsync(&c->ctrl->step, o, sizeof(uint64_t), hipMemcpyDeviceToDevice, c->s));
  launch_md_invalidate(c->mw, c->s);
  uint64_t st = 0;
  acc(hipMemcpyAsync(&st, o, sizeof(uint64_t), hipMemcpyDeviceToHost, c->s));
  hipError_t e = hipStreamSynchronize(c->s);
  if (e != hipSuccess) return fail(LB_ERR_DEVICE, "lb_set_state: %s", hipGetErrorString(e));
  c->steps = (int64_t)st;
  return check_hip("lb_set_state");
}

void* lb_current_pops(lb_ctx* c) { return c ? cur_pops(c) : nullptr; }

int lb_check(lb_ctx* c) {
  if (!c) return fail(LB_ERR_ARG, "null context");
  hipError_t e = hipStreamSynchronize(c->s);
  if (e == hipSuccess) e = hipStreamSynchronize(c->s2);
  if (e != hipSuccess) return fail(LB_ERR_DEVICE, "stream: %s", hipGetErrorString(e));
  uint32_t err = 0;
  e = hipMemcpy(&err, &c->ctrl->err, sizeof(err), hipMemcpyDeviceToHost);
  if (e != hipSuccess) return fail(LB_ERR_DEVICE, "watchdog read: %s", hipGetErrorString(e));
  if (err) {
    std::string why;
    if (err & E_DENSITY) why += "non-positive or non-finite density; ";
    if (err & E_BEADS) why += "non-finite bead velocity; ";
    if (err & E_NBRLIST) why += "neighbour list overflow; ";
    if (err & E_SPREAD) why += "too many beads on one node stencil; ";
    return fail(LB_ERR_UNSTABLE, "watchdog: %s", why.c_str());
  }
  return LB_OK;
}

int64_t lb_step_count(lb_ctx* c) { return c ? c->steps : -1; }

int lb_diagnostics(lb_ctx* c, int64_t* out) {
  if (!c || !out) return fail(LB_ERR_ARG, "bad arguments");
  hipError_t e = hipStreamSynchronize(c->s);
  if (e != hipSuccess) return fail(LB_ERR_DEVICE, "stream: %s", hipGetErrorString(e));
  Ctrl h;
  e = hipMemcpy(&h, c->ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost);
  if (e != hipSuccess) return fail(LB_ERR_DEVICE, "diagnostics read: %s", hipGetErrorString(e));
  out[0] = (int64_t)h.rebuilds;
  out[1] = (int64_t)h.substeps;
  out[2] = (int64_t)c->last_touched;
  out[3] = (int64_t)h.err;
  out[4] = (int64_t)h.step;
  return LB_OK;
}

}  // extern "C"
