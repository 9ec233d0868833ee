"""Python binding of liblbmd.so (the C ABI in include/lbmd.h).

Argument marshalling only: every step of the coupled LB/MD method runs in the
library's HIP kernels.  PyTorch provides the device memory (uint8 tensors
sized by lb_buffer_sizes) and the stream (the current torch stream).  The
binding refuses to run when the library is missing: there is no CPU path.
"""
import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblbmd.so")

LB_OK, LB_ERR_ARG, LB_ERR_DEVICE, LB_ERR_UNSTABLE, LB_ERR_UNSUPPORTED = 0, -1, -2, -3, -4
LB_FP64, LB_FP32_DEV = 0, 1
LB_NOBS = 23
Q = 19

OBS_NAMES = ["mass", "px", "py", "pz", "T_beads", "bpx", "bpy", "bpz", "mean_normal", "translocated",
             "N_r", "R_U", "R_T", "R_eff", "dWH_dt", "dWE_dt", "wall_bb_x", "wall_bb_y", "wall_bb_z",
             "wall_sp_x", "wall_sp_y", "wall_sp_z", "step"]


class LbDesc(C.Structure):
    _fields_ = [
        ("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32), ("precision", C.c_int32),
        ("tau", C.c_double), ("g", C.c_double * 3),
        ("wall_axis", C.c_int32), ("wall_pos", C.c_int32), ("pore_h", C.c_int32), ("nb", C.c_int32),
        ("mass", C.c_double), ("k_bond", C.c_double), ("r0", C.c_double), ("kappa", C.c_double),
        ("eps", C.c_double), ("sigma", C.c_double), ("rc", C.c_double),
        ("gamma", C.c_double), ("kT", C.c_double), ("f_drive", C.c_double),
        ("n_sub", C.c_int32), ("seed", C.c_uint32), ("replica", C.c_uint32),
    ]


class LbSizes(C.Structure):
    _fields_ = [(n, C.c_size_t) for n in ("pops_bytes", "flags_bytes", "force_bytes", "beads_bytes",
                                          "work_bytes", "state_bytes")]


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
    L.lb_last_error.restype = C.c_char_p
    L.lb_buffer_sizes.argtypes = [C.POINTER(LbDesc), C.POINTER(LbSizes)]
    L.lb_init.argtypes = [C.POINTER(LbDesc), C.POINTER(LbBuffers), P, P, P, C.POINTER(P)]
    L.lb_destroy.argtypes = [P]
    L.lb_destroy.restype = None
    L.lb_step.argtypes = [P, C.c_int]
    L.md_couple_step.argtypes = [P, C.c_int]
    L.md_relax.argtypes = [P, C.c_int, C.c_double]
    L.lb_observables.argtypes = [P, P]
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
    return d


def buffer_sizes(cfg, precision=LB_FP64):
    d = make_desc(cfg, precision)
    s = LbSizes()
    _raise(lib().lb_buffer_sizes(C.byref(d), C.byref(s)))
    return {n: getattr(s, n) for n, _ in LbSizes._fields_}


class Simulation:
    """One coupled LB/MD system on one GPU (a context of liblbmd)."""

    def __init__(self, cfg, r0=None, v0=None, precision=LB_FP64, device="cuda:0"):
        import torch
        self.torch = torch
        self.cfg = dict(cfg)
        self.precision = precision
        self.device = torch.device(device)
        self.desc = make_desc(cfg, precision)
        self.nb = self.desc.nb
        self.shape = tuple(cfg["shape"])
        nx, ny, nz = self.shape
        self.N = nx * ny * nz
        self.sizes = buffer_sizes(cfg, precision)
        alloc = lambda n: torch.empty(int(n), dtype=torch.uint8, device=self.device)
        self._bufs = {
            "pops_a": alloc(self.sizes["pops_bytes"]), "pops_b": alloc(self.sizes["pops_bytes"]),
            "flags": alloc(self.sizes["flags_bytes"]), "force": alloc(self.sizes["force_bytes"]),
            "beads": alloc(self.sizes["beads_bytes"]), "work": alloc(self.sizes["work_bytes"]),
        }
        b = LbBuffers(*[self._bufs[k].data_ptr() for k, _ in LbBuffers._fields_])
        if self.nb > 0:
            if r0 is None:
                raise ValueError("bead positions required")
            r0 = np.ascontiguousarray(r0, dtype=np.float64).reshape(-1)
            assert r0.size == 3 * self.nb
        rp = r0.ctypes.data_as(C.c_void_p) if self.nb > 0 else None
        if v0 is not None:
            v0 = np.ascontiguousarray(v0, dtype=np.float64).reshape(-1)
            assert v0.size == 3 * self.nb
        vp = v0.ctypes.data_as(C.c_void_p) if v0 is not None and self.nb > 0 else None
        with torch.cuda.device(self.device):
            self.stream = torch.cuda.current_stream(self.device)
            ctx = C.c_void_p()
            _raise(lib().lb_init(C.byref(self.desc), C.byref(b), rp, vp, C.c_void_p(self.stream.cuda_stream),
                                 C.byref(ctx)))
        self.ctx = ctx
        self._destroy = lib().lb_destroy      # kept for teardown at interpreter exit
        self._obs = torch.empty(LB_NOBS, dtype=torch.float64, device=self.device)

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

    def relax(self, nsub_total, gamma_relax):
        _raise(lib().md_relax(self.ctx, int(nsub_total), float(gamma_relax)))

    def check(self):
        _raise(lib().lb_check(self.ctx))

    def profile_start(self, max_steps):
        _raise(lib().lb_profile_start(self.ctx, int(max_steps)))

    def profile_stop(self):
        """Mean LB-sweep and bead-phase durations (ms) of the recorded steps."""
        a, b, n = C.c_double(), C.c_double(), C.c_int()
        _raise(lib().lb_profile_stop(self.ctx, C.byref(a), C.byref(b), C.byref(n)))
        return a.value, b.value, n.value

    def diagnostics(self):
        out = (C.c_int64 * 5)()
        _raise(lib().lb_diagnostics(self.ctx, out))
        return dict(zip(("rebuilds", "substeps", "forced_nodes", "watchdog", "steps"), list(out)))

    def step_count(self):
        return int(lib().lb_step_count(self.ctx))

    # -- state ---------------------------------------------------------------
    @property
    def dtype(self):
        return self.torch.float64 if self.precision == LB_FP64 else self.torch.float32

    def pops(self):
        """View of the current populations as [19, nz, ny, nx] (f_i in FP64
        storage, f_i - w_i in FP32 deviation storage)."""
        ptr = lib().lb_current_pops(self.ctx)
        t = self._bufs["pops_a"] if ptr == self._bufs["pops_a"].data_ptr() else self._bufs["pops_b"]
        nx, ny, nz = self.shape
        es = 8 if self.precision == LB_FP64 else 4
        return t[: Q * self.N * es].view(self.dtype).view(Q, nz, ny, nx)

    def flags(self):
        nx, ny, nz = self.shape
        return self._bufs["flags"][: self.N].view(nz, ny, nx)

    def beads(self):
        """Views of the bead arrays: r, v, up, J, rs, each (nb, 3) float64."""
        nbs = max(self.nb, 1)
        b = self._bufs["beads"][: 15 * nbs * 8].view(self.torch.float64)
        out = {}
        for k, name in enumerate(("r", "v", "up", "J", "rs")):
            out[name] = b[3 * nbs * k: 3 * nbs * k + 3 * self.nb].view(self.nb, 3)
        return out

    def observables(self):
        _raise(lib().lb_observables(self.ctx, C.c_void_p(self._obs.data_ptr())))
        return self._obs

    def get_state(self):
        st = self.torch.empty(self.sizes["state_bytes"], dtype=self.torch.uint8, device=self.device)
        _raise(lib().lb_get_state(self.ctx, C.c_void_p(st.data_ptr())))
        return st

    def set_state(self, st):
        _raise(lib().lb_set_state(self.ctx, C.c_void_p(st.data_ptr())))
