"""Python binding of liblbmd.so (the C ABI in include/lbmd.h).

Argument marshalling only: every step of the coupled LB/MD method runs in the
library's HIP kernels.  PyTorch provides the device memory (uint8 tensors
sized by lb_buffer_sizes / lb_ensemble_sizes) and the stream (the current
torch stream).  The binding refuses to run when the library is missing: there
is no CPU path.
"""
import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblbmd.so")

LB_OK, LB_ERR_ARG, LB_ERR_DEVICE, LB_ERR_UNSTABLE, LB_ERR_UNSUPPORTED = 0, -1, -2, -3, -4
LB_FP64, LB_FP32_DEV = 0, 1
LB_NOBS = 25
# groups of lb_observables' mask
LB_OBS_FLUID, LB_OBS_BEADS, LB_OBS_LEDGERS, LB_OBS_STEP = 1, 2, 4, 8
LB_OBS_ALL = 15
Q = 19
# The population order of the library's storage (documented in the header):
# rest, +-x, +-y, +-z, then the xy, xz and yz diagonals, opposites adjacent.
VELOCITIES = ((0, 0, 0), (1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1),
              (1, 1, 0), (-1, -1, 0), (1, -1, 0), (-1, 1, 0), (1, 0, 1), (-1, 0, -1), (1, 0, -1), (-1, 0, 1),
              (0, 1, 1), (0, -1, -1), (0, 1, -1), (0, -1, 1))
WEIGHTS = (1.0 / 3.0,) + (1.0 / 18.0,) * 6 + (1.0 / 36.0,) * 12

OBS_NAMES = ["mass", "px", "py", "pz", "T_beads", "bpx", "bpy", "bpz", "mean_normal", "translocated",
             "N_r", "R_U", "R_T", "R_eff", "dWH_dt", "dWE_dt", "wall_bb_x", "wall_bb_y", "wall_bb_z",
             "wall_sp_x", "wall_sp_y", "wall_sp_z", "step", "drag_U", "drag_T"]


class LbDesc(C.Structure):
    _fields_ = [
        ("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32), ("precision", C.c_int32),
        ("tau", C.c_double), ("g", C.c_double * 3),
        ("wall_axis", C.c_int32), ("wall_pos", C.c_int32), ("pore_h", C.c_int32), ("nb", C.c_int32),
        ("mass", C.c_double), ("k_bond", C.c_double), ("r0", C.c_double), ("kappa", C.c_double),
        ("eps", C.c_double), ("sigma", C.c_double), ("rc", C.c_double),
        ("gamma", C.c_double), ("kT", C.c_double), ("f_drive", C.c_double),
        ("n_sub", C.c_int32), ("seed", C.c_uint32), ("replica", C.c_uint32),
        ("fluid_kT", C.c_double), ("mts_outer", C.c_int32), ("coupling", C.c_int32), ("constraints", C.c_int32),
    ]


class LbSizes(C.Structure):
    _fields_ = [(n, C.c_size_t) for n in ("pops_bytes", "flags_bytes", "force_bytes", "beads_bytes",
                                          "work_bytes", "state_bytes", "nodes", "bead_slots", "snapshot_bytes")]


class LbBuffers(C.Structure):
    _fields_ = [(n, C.c_void_p) for n in ("pops_a", "pops_b", "flags", "force", "beads", "work")]


class LbError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"liblbmd error {code}: {msg}")
        self.code = code


_lib = None


def lib():
    """Load liblbmd.so (built in-tree by paper_0711_2665_amd.build)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_0711_2665_amd.build`")
        L = C.CDLL(LIB_PATH)
        _declare(L)
        _lib = L
    return _lib


def _declare(L):
    P = C.c_void_p
    D = C.POINTER(LbDesc)
    L.lb_last_error.restype = C.c_char_p
    L.lb_buffer_sizes.argtypes = [D, C.POINTER(LbSizes)]
    L.lb_ensemble_sizes.argtypes = [D, C.c_int, C.POINTER(LbSizes)]
    L.lb_init.argtypes = [D, C.POINTER(LbBuffers), P, P, P, C.POINTER(P)]
    L.lb_ensemble_init.argtypes = [D, C.c_int, C.POINTER(LbBuffers), P, P, P, C.POINTER(P)]
    L.lb_ensemble_layout.argtypes = [P, C.POINTER(C.c_int64), C.POINTER(C.c_int64)]
    L.lb_destroy.argtypes = [P]
    L.lb_destroy.restype = None
    L.lb_step.argtypes = [P, C.c_int]
    L.md_couple_step.argtypes = [P, C.c_int]
    L.lb_ensemble_run.argtypes = [P, C.c_int, C.c_int]
    L.lb_ensemble_translocation.argtypes = [P, C.POINTER(C.c_int64)]
    L.lb_sweep_config.argtypes = [P, C.c_int, C.c_int, C.c_int, C.c_int]
    L.lb_md_fused.argtypes = [P, C.c_int]
    L.lb_autotune.argtypes = [P, C.c_int, C.POINTER(C.c_int), C.POINTER(C.c_double)]
    L.lb_autotune_step.argtypes = [P, C.c_int, P, C.c_size_t, C.POINTER(C.c_int), C.POINTER(C.c_double)]
    L.md_relax.argtypes = [P, C.c_int, C.c_double]
    L.lb_set_coupling.argtypes = [P, C.c_int, C.c_double, C.c_double]
    L.lb_adjoint_sizes.argtypes = [P, C.c_int, C.c_int, C.POINTER(C.c_size_t)]
    L.lb_adjoint_forward.argtypes = [P, C.c_int, C.c_int, P, C.c_size_t]
    L.lb_adjoint_backward.argtypes = [P, P, P, P]
    L.lb_adjoint_run.argtypes = [P, C.c_int, C.c_int, P, C.c_size_t, P, P]
    L.lb_observables.argtypes = [P, P, C.c_int]
    L.lb_observables_static.argtypes = [P, P, C.c_int]
    L.lb_get_state.argtypes = [P, P]
    L.lb_set_state.argtypes = [P, P]
    L.lb_current_pops.argtypes = [P]
    L.lb_current_pops.restype = P
    L.lb_check.argtypes = [P]
    L.lb_step_count.argtypes = [P]
    L.lb_step_count.restype = C.c_int64
    L.lb_diagnostics.argtypes = [P, C.POINTER(C.c_int64)]
    L.lb_profile_start.argtypes = [P, C.c_int]
    L.lb_profile_stop.argtypes = [P, C.POINTER(C.c_double), C.POINTER(C.c_double), C.POINTER(C.c_int)]


def _raise(code):
    if code != LB_OK:
        raise LbError(code, lib().lb_last_error().decode())


def make_desc(cfg, precision=LB_FP64):
    d = LbDesc()
    _fill_desc(d, cfg, precision)
    return d


def _fill_desc(d, cfg, precision):
    d.nx, d.ny, d.nz = cfg["shape"]
    d.precision = precision
    d.tau = cfg.get("tau", 1.0)
    g = cfg.get("g", (0.0, 0.0, 0.0))
    for a in range(3):
        d.g[a] = g[a]
    d.wall_axis = cfg.get("wall_axis", -1)
    d.wall_pos = cfg.get("wall_pos", 0)
    d.pore_h = cfg.get("pore_h", 0)
    d.nb = cfg.get("nb", 0)
    d.mass = cfg.get("mass", 1.0)
    d.k_bond = cfg.get("k_bond", 100.0)
    d.r0 = cfg.get("r0", 1.0)
    d.kappa = cfg.get("kappa", 10.0)
    d.eps = cfg.get("eps", 1.0)
    d.sigma = cfg.get("sigma", 1.0)
    d.rc = cfg.get("rc", 2.0 ** (1.0 / 6.0) * d.sigma)
    d.gamma = cfg.get("gamma", 0.1)
    d.kT = cfg.get("kT", 1e-4)
    d.f_drive = cfg.get("f_drive", 0.02)
    d.n_sub = cfg.get("n_sub", 100)
    d.seed = cfg.get("seed", 1234) & 0xFFFFFFFF
    d.replica = cfg.get("replica", 0) & 0xFFFFFFFF
    d.fluid_kT = cfg.get("fluid_kT", 0.0)
    d.mts_outer = cfg.get("mts_outer", 0)
    d.coupling = cfg.get("coupling", 0)
    d.constraints = cfg.get("constraints", 0)


def make_descs(cfgs, precision=LB_FP64):
    arr = (LbDesc * len(cfgs))()
    for k, cfg in enumerate(cfgs):
        _fill_desc(arr[k], cfg, precision)
    return arr


def _sizes_dict(s):
    return {n: getattr(s, n) for n, _ in LbSizes._fields_}


def buffer_sizes(cfg, precision=LB_FP64):
    d = make_desc(cfg, precision)
    s = LbSizes()
    _raise(lib().lb_buffer_sizes(C.byref(d), C.byref(s)))
    return _sizes_dict(s)


def ensemble_sizes(cfgs, precision=LB_FP64):
    arr = make_descs(cfgs, precision)
    s = LbSizes()
    _raise(lib().lb_ensemble_sizes(arr, len(cfgs), C.byref(s)))
    return _sizes_dict(s)


class Context:
    """R >= 1 coupled LB/MD systems on one GPU, advanced in lockstep (one
    context of liblbmd).  Replica r has its own lattice, wall, chain and
    noise key; r0s[r] / v0s[r] are its chain's positions / velocities."""

    def __init__(self, cfgs, r0s=None, v0s=None, precision=LB_FP64, device="cuda:0"):
        import torch
        self.torch = torch
        self.cfgs = [dict(c) for c in cfgs]
        self.nrep = len(self.cfgs)
        self.precision = precision
        self.device = torch.device(device)
        self.descs = make_descs(self.cfgs, precision)
        self.nbs = [int(c.get("nb", 0)) for c in self.cfgs]
        self.shapes = [tuple(c["shape"]) for c in self.cfgs]
        self.Ns = [nx * ny * nz for nx, ny, nz in self.shapes]
        self.sizes = ensemble_sizes(self.cfgs, precision)
        alloc = lambda n: torch.empty(int(n), dtype=torch.uint8, device=self.device)
        self._bufs = {
            "pops_a": alloc(self.sizes["pops_bytes"]), "pops_b": alloc(self.sizes["pops_bytes"]),
            "flags": alloc(self.sizes["flags_bytes"]), "force": alloc(self.sizes["force_bytes"]),
            "beads": alloc(self.sizes["beads_bytes"]), "work": alloc(self.sizes["work_bytes"]),
        }
        b = LbBuffers(*[self._bufs[k].data_ptr() for k, _ in LbBuffers._fields_])
        nbt = sum(self.nbs)
        rp = vp = None
        if nbt > 0:
            if r0s is None:
                raise ValueError("bead positions required")
            r0 = np.ascontiguousarray(np.concatenate([np.asarray(r, dtype=np.float64).reshape(-1, 3)
                                                      for r, n in zip(r0s, self.nbs) if n > 0]))
            assert r0.shape == (nbt, 3)
            rp = r0.ctypes.data_as(C.c_void_p)
            if v0s is not None:
                v0 = np.ascontiguousarray(np.concatenate([np.asarray(v, dtype=np.float64).reshape(-1, 3)
                                                          for v, n in zip(v0s, self.nbs) if n > 0]))
                assert v0.shape == (nbt, 3)
                vp = v0.ctypes.data_as(C.c_void_p)
        with torch.cuda.device(self.device):
            self.stream = torch.cuda.current_stream(self.device)
            ctx = C.c_void_p()
            _raise(lib().lb_ensemble_init(self.descs, self.nrep, C.byref(b), rp, vp,
                                          C.c_void_p(self.stream.cuda_stream), C.byref(ctx)))
        self.ctx = ctx
        self._destroy = lib().lb_destroy      # kept for teardown at interpreter exit
        no = (C.c_int64 * self.nrep)()
        so = (C.c_int64 * self.nrep)()
        _raise(lib().lb_ensemble_layout(self.ctx, no, so))
        self.node_off = list(no)
        self.slot_off = list(so)
        self.slots = int(self.sizes["bead_slots"])
        self._obs = torch.empty(LB_NOBS * self.nrep, dtype=torch.float64, device=self.device)

    def close(self):
        """Synchronise and release the library context (the buffers are freed
        with this object)."""
        ctx = getattr(self, "ctx", None)
        if ctx is not None and ctx.value:
            try:
                self.stream.synchronize()
            except Exception:
                pass
            self._destroy(ctx)
            self.ctx = None

    def __del__(self):
        self.close()

    # -- stepping ------------------------------------------------------------
    def lb_step(self, n=1):
        _raise(lib().lb_step(self.ctx, int(n)))

    def couple_step(self, n=1):
        _raise(lib().md_couple_step(self.ctx, int(n)))

    def run(self, n, graph=True):
        """n coupled steps, replayed from a captured HIP graph when graph."""
        _raise(lib().lb_ensemble_run(self.ctx, int(n), 1 if graph else 0))

    def relax(self, nsub_total, gamma_relax):
        _raise(lib().md_relax(self.ctx, int(nsub_total), float(gamma_relax)))

    def check(self):
        _raise(lib().lb_check(self.ctx))

    def set_coupling(self, gamma, f_drive, rep=0):
        _raise(lib().lb_set_coupling(self.ctx, int(rep), float(gamma), float(f_drive)))
        self.cfgs[rep]["gamma"] = float(gamma)
        self.cfgs[rep]["f_drive"] = float(f_drive)

    # -- adjoint -------------------------------------------------------------
    def adjoint_sizes(self, nsteps, K):
        n = C.c_size_t()
        _raise(lib().lb_adjoint_sizes(self.ctx, int(nsteps), int(K), C.byref(n)))
        return n.value

    def adjoint_forward(self, nsteps, K):
        """nsteps coupled steps with checkpoints every K steps kept in a
        workspace tensor for adjoint_backward."""
        n = self.adjoint_sizes(nsteps, K)
        self._adj_ws = self.torch.empty(n, dtype=self.torch.uint8, device=self.device)
        _raise(lib().lb_adjoint_forward(self.ctx, int(nsteps), int(K), C.c_void_p(self._adj_ws.data_ptr()), n))

    def adjoint_backward(self, dLdr, dLdv=None):
        """Gradient [dL/dgamma, dL/dF_drive, dL/dr_start (nb x 3)] (float64,
        device) of a loss whose gradient at the final bead state is dLdr
        (and dLdv)."""
        torch = self.torch
        nb = self.nbs[0]
        gr = torch.as_tensor(dLdr, dtype=torch.float64, device=self.device).reshape(nb, 3).contiguous()
        gv = None
        if dLdv is not None:
            gv = torch.as_tensor(dLdv, dtype=torch.float64, device=self.device).reshape(nb, 3).contiguous()
        out = torch.empty(2 + 3 * nb, dtype=torch.float64, device=self.device)
        _raise(lib().lb_adjoint_backward(self.ctx, C.c_void_p(gr.data_ptr()),
                                         C.c_void_p(gv.data_ptr()) if gv is not None else None,
                                         C.c_void_p(out.data_ptr())))
        return out

    def md_fused(self, K):
        """Sub-steps per fused launch of the uniform MD sub-cycle (0: one
        launch per sub-step); see lb_md_fused."""
        _raise(lib().lb_md_fused(self.ctx, int(K)))

    def sweep_config(self, tile_nodes, order=0, grid=0, cap=0):
        _raise(lib().lb_sweep_config(self.ctx, int(tile_nodes), int(order), int(grid), int(cap)))

    def autotune(self, reps=5, coupled=False):
        """Chooses the sweep layout by timing the sweep alone, or with
        coupled=True the whole coupled step (graph-replayed, from a snapshot
        of the state that is restored afterwards)."""
        cfg = (C.c_int * 4)()
        ms = C.c_double()
        if coupled:
            # the snapshot buffer the library fills and restores from
            n = int(self.sizes["snapshot_bytes"])
            snap = self.torch.empty(n, dtype=self.torch.uint8, device=self.device)
            _raise(lib().lb_autotune_step(self.ctx, int(reps), C.c_void_p(snap.data_ptr()), n, cfg, C.byref(ms)))
            del snap
        else:
            _raise(lib().lb_autotune(self.ctx, int(reps), cfg, C.byref(ms)))
        return dict(tile_nodes=cfg[0], order=cfg[1], grid=cfg[2], cap=cfg[3], ms=ms.value)

    def translocation_steps(self):
        out = (C.c_int64 * self.nrep)()
        _raise(lib().lb_ensemble_translocation(self.ctx, out))
        return list(out)

    def profile_start(self, max_steps):
        _raise(lib().lb_profile_start(self.ctx, int(max_steps)))

    def profile_stop(self):
        """Mean LB-sweep and bead-phase durations (ms) of the recorded steps."""
        a, b, n = C.c_double(), C.c_double(), C.c_int()
        _raise(lib().lb_profile_stop(self.ctx, C.byref(a), C.byref(b), C.byref(n)))
        return a.value, b.value, n.value

    def diagnostics(self):
        out = (C.c_int64 * 15)()
        _raise(lib().lb_diagnostics(self.ctx, out))
        return dict(zip(("rebuilds", "substeps", "sweep_tiles", "watchdog", "steps", "forced_total",
                         "cell_rebuilds", "fused_blocks", "fused_redos", "why_moved", "why_partners",
                         "why_capacity", "why_unsettled", "why_displacement", "nbr_max"), list(out)))

    def step_count(self):
        return int(lib().lb_step_count(self.ctx))

    # -- state ---------------------------------------------------------------
    @property
    def dtype(self):
        return self.torch.float64 if self.precision == LB_FP64 else self.torch.float32

    def _cur(self):
        ptr = lib().lb_current_pops(self.ctx)
        return self._bufs["pops_a"] if ptr == self._bufs["pops_a"].data_ptr() else self._bufs["pops_b"]

    def pops(self, r=0):
        """View of replica r's current populations as [19, nz, ny, nx] (f_i
        in FP64 storage, f_i - w_i in FP32 deviation storage)."""
        nx, ny, nz = self.shapes[r]
        flat = self._cur().view(self.dtype)
        o = Q * self.node_off[r]
        return flat[o: o + Q * self.Ns[r]].view(Q, nz, ny, nx)

    def flags(self, r=0):
        nx, ny, nz = self.shapes[r]
        o = self.node_off[r]
        return self._bufs["flags"][o: o + self.Ns[r]].view(nz, ny, nx)

    def beads(self, r=0):
        """Views of replica r's bead arrays: r, v, up, J, rs, each (nb, 3)
        float64."""
        ns = self.slots
        b = self._bufs["beads"][: 15 * ns * 8].view(self.torch.float64)
        o, nb = self.slot_off[r], self.nbs[r]
        out = {}
        for k, name in enumerate(("r", "v", "up", "J", "rs")):
            out[name] = b[3 * ns * k + 3 * o: 3 * ns * k + 3 * (o + nb)].view(nb, 3)
        return out

    def observables(self, mask=LB_OBS_ALL):
        """[nrep, LB_NOBS] float64 on the device (see lb_observables); the
        groups outside mask are NaN."""
        self._obs.fill_(float("nan"))
        _raise(lib().lb_observables(self.ctx, C.c_void_p(self._obs.data_ptr()), int(mask)))
        return self._obs.view(self.nrep, LB_NOBS)

    def observables_static(self, out, mask=LB_OBS_ALL):
        """lb_observables_static into the caller's float64 device tensor out
        (at least nrep * LB_NOBS elements): no allocation on any side."""
        assert out.dtype == self.torch.float64 and out.is_cuda and out.numel() >= LB_NOBS * self.nrep
        _raise(lib().lb_observables_static(self.ctx, C.c_void_p(out.data_ptr()), int(mask)))
        return out

    def get_state(self):
        st = self.torch.empty(self.sizes["state_bytes"], dtype=self.torch.uint8, device=self.device)
        _raise(lib().lb_get_state(self.ctx, C.c_void_p(st.data_ptr())))
        return st

    def set_state(self, st):
        _raise(lib().lb_set_state(self.ctx, C.c_void_p(st.data_ptr())))


class Simulation(Context):
    """One coupled LB/MD system (a context with one replica)."""

    def __init__(self, cfg, r0=None, v0=None, precision=LB_FP64, device="cuda:0"):
        super().__init__([cfg], [r0] if r0 is not None else None, [v0] if v0 is not None else None,
                         precision=precision, device=device)
        self.cfg = self.cfgs[0]
        self.nb = self.nbs[0]
        self.shape = self.shapes[0]
        self.N = self.Ns[0]

    def observables(self, mask=LB_OBS_ALL):
        return super().observables(mask)[0]


class Ensemble(Context):
    """The batched ensemble: replicas of uneven lattices and chain lengths in
    one context."""
