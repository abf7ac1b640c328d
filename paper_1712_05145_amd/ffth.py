"""Thin ctypes binding of libffth (include/ffth.h).

Argument marshalling only: every step of the solve runs in the HIP kernels of
libffth.so.  PyTorch provides device memory and streams.  The module fails
loudly (FFTHError / OSError) when the library is missing or a call fails;
there is no CPU fallback.

Functions keep the C names (ffth_solve_order0, ...).  ``Solver`` is a small
convenience wrapper that allocates the workspace and output tensors with
torch and owns one plan.
"""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIBPATH = os.path.join(HERE, "libffth.so")

FFTH_OK, FFTH_ERR_INVALID, FFTH_ERR_OOM, FFTH_ERR_NOT_CONVERGED, FFTH_ERR_DIVERGED, \
    FFTH_ERR_DEVICE, FFTH_ERR_BUSY, FFTH_ERR_CANCELLED = range(8)
FFTH_BASIC, FFTH_CG, FFTH_BICGSTAB = 0, 1, 2
FFTH_FP64, FFTH_FP32, FFTH_MIXED = 0, 1, 2

FFTH_CG3 = 3
SCHEMES = {"basic": FFTH_BASIC, "cg": FFTH_CG, "bicgstab": FFTH_BICGSTAB, "cg3": FFTH_CG3}
PRECISIONS = {"fp64": FFTH_FP64, "fp32": FFTH_FP32, "mixed": FFTH_MIXED}


class FFTHError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(msg)
        self.status = status


class ffth_problem(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32 * 3), ("nphases", ctypes.c_int32), ("phase", ctypes.c_void_p),
                ("lame", ctypes.POINTER(ctypes.c_double)), ("stiffness", ctypes.POINTER(ctypes.c_double)),
                ("lambda0", ctypes.c_double), ("mu0", ctypes.c_double)]


class ffth_opts(ctypes.Structure):
    _fields_ = [("scheme", ctypes.c_int32), ("precision", ctypes.c_int32), ("tol", ctypes.c_double),
                ("max_iter", ctypes.c_int32), ("inner_tol", ctypes.c_double), ("max_outer", ctypes.c_int32),
                ("check_every", ctypes.c_int32), ("autotune", ctypes.c_int32), ("spectrum16", ctypes.c_int32)]


class ffth_result(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("iters", ctypes.c_int32), ("outer_iters", ctypes.c_int32),
                ("fp64_applications", ctypes.c_int32), ("projections", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("residual", ctypes.c_double),
                ("mean_stress", ctypes.c_double * 6), ("g_mean", ctypes.c_double * 3),
                ("seconds", ctypes.c_double)]

    def as_dict(self):
        return {"status": self.status, "iters": self.iters, "outer_iters": self.outer_iters,
                "fp64_applications": self.fp64_applications, "projections": self.projections,
                "residual": self.residual,
                "mean_stress": list(self.mean_stress), "g_mean": list(self.g_mean), "seconds": self.seconds}


_lib = None

# (name, restype, argtypes) of every entry point declared in include/ffth.h
SIGNATURES = [
    ("ffth_default_opts", None, [ctypes.POINTER(ffth_opts)]),
    ("ffth_size_supported", ctypes.c_int32, [ctypes.c_int32]),
    ("ffth_stiffness_contrast", ctypes.c_double,
     [ctypes.c_int32, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]),
    ("ffth_workspace_bytes", ctypes.c_size_t,
     [ctypes.POINTER(ctypes.c_int32), ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(ffth_opts)]),
    ("ffth_plan_create", ctypes.c_int,
     [ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(ffth_problem), ctypes.POINTER(ffth_opts), ctypes.c_int32,
      ctypes.c_int32, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p]),
    ("ffth_plan_destroy", ctypes.c_int, [ctypes.c_void_p]),
    ("ffth_solve_order0", ctypes.c_int,
     [ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(ctypes.c_double), ctypes.c_void_p,
      ctypes.POINTER(ffth_result)]),
    ("ffth_solve_order1", ctypes.c_int,
     [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(ctypes.c_double), ctypes.c_void_p,
      ctypes.POINTER(ffth_result)]),
    ("ffth_green_apply", ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32]),
    ("ffth_displacement", ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    ("ffth_order1_rhs", ctypes.c_int,
     [ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER(ctypes.c_double), ctypes.c_void_p,
      ctypes.POINTER(ctypes.c_double)]),
    ("ffth_solve_order2", ctypes.c_int,
     [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(ctypes.c_double),
      ctypes.c_void_p, ctypes.POINTER(ffth_result)]),
    ("ffth_order2_rhs", ctypes.c_int,
     [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER(ctypes.c_double), ctypes.c_void_p,
      ctypes.POINTER(ctypes.c_double)]),
    ("ffth_profile_enable", ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32]),
    ("ffth_profile_read", ctypes.c_int,
     [ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64),
      ctypes.POINTER(ctypes.c_double)]),
    ("ffth_profile_name", ctypes.c_char_p, [ctypes.c_int32]),
    ("ffth_tile_variants", ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int32)]),
    ("ffth_set_tile_variants", ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int32)]),
    ("ffth_launch_loads", ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int32)]),
    ("ffth_set_launch_loads", ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int32)]),
    ("ffth_request_bytes", ctypes.c_size_t,
     [ctypes.POINTER(ctypes.c_int32), ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(ffth_opts)]),
    ("ffth_server_create", ctypes.c_int,
     [ctypes.POINTER(ctypes.c_void_p), ctypes.c_void_p, ctypes.c_size_t, ctypes.POINTER(ffth_opts), ctypes.c_int32,
      ctypes.c_void_p]),
    ("ffth_submit", ctypes.c_int,
     [ctypes.c_void_p, ctypes.POINTER(ffth_problem), ctypes.c_int32, ctypes.POINTER(ctypes.c_double),
      ctypes.POINTER(ctypes.c_uint64)]),
    ("ffth_server_step", ctypes.c_int,
     [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32)]),
    ("ffth_poll", ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint64, ctypes.POINTER(ffth_result)]),
    ("ffth_cancel", ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint64]),
    ("ffth_server_destroy", ctypes.c_int, [ctypes.c_void_p]),
    ("ffth_server_stats", ctypes.c_int,
     [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int32)]),
    ("ffth_green_apply_noalloc", ctypes.c_int,
     [ctypes.POINTER(ctypes.c_int32), ctypes.c_double, ctypes.c_double, ctypes.c_void_p, ctypes.c_void_p,
      ctypes.c_int32, ctypes.c_void_p]),
    ("ffth_status_string", ctypes.c_char_p, [ctypes.c_int]),
    ("ffth_last_error", ctypes.c_char_p, []),
]


def load(path=LIBPATH):
    """Load libffth.so (raises OSError if it is not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(path):
            raise OSError(f"{path} not built: run python -m paper_1712_05145_amd.build")
        lib = ctypes.CDLL(path)
        for name, res, args in SIGNATURES:
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def _check(status, what):
    if status != FFTH_OK:
        lib = load()
        raise FFTHError(status, f"{what}: {lib.ffth_status_string(status).decode()} "
                                f"({lib.ffth_last_error().decode()})")


def _dptr(t):
    return ctypes.c_void_p(t.data_ptr())


def check_field(t, device, shape, what):
    """Raise FFTHError(FFTH_ERR_INVALID) unless t is a contiguous float64
    tensor of exactly `shape` on `device`.  The library takes device fields as
    bare pointers: a tensor on another device, of another type or of fewer
    elements would make the kernels read or write outside it."""
    import torch
    if not isinstance(t, torch.Tensor):
        raise FFTHError(FFTH_ERR_INVALID, f"{what}: expected a torch tensor, got {type(t).__name__}")
    if t.device != torch.device(device):
        raise FFTHError(FFTH_ERR_INVALID, f"{what}: tensor on {t.device}, the plan runs on {device}")
    if t.dtype != torch.float64:
        raise FFTHError(FFTH_ERR_INVALID, f"{what}: dtype {t.dtype}, expected torch.float64")
    if tuple(t.shape) != tuple(shape):
        raise FFTHError(FFTH_ERR_INVALID, f"{what}: shape {tuple(t.shape)}, expected {tuple(shape)}")
    if not t.is_contiguous():
        raise FFTHError(FFTH_ERR_INVALID, f"{what}: tensor is not contiguous")
    return t


def _darr(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a, a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def make_opts(scheme="cg", precision="mixed", tol=1e-8, max_iter=20000, inner_tol=1e-3, max_outer=30,
              check_every=8, autotune=True, spectrum16=True):
    o = ffth_opts()
    load().ffth_default_opts(ctypes.byref(o))
    o.scheme = SCHEMES[scheme] if isinstance(scheme, str) else scheme
    o.precision = PRECISIONS[precision] if isinstance(precision, str) else precision
    o.tol, o.max_iter, o.inner_tol = tol, max_iter, inner_tol
    o.max_outer, o.check_every = max_outer, check_every
    o.autotune = 1 if autotune else 0
    # True / False: binary16 where the grid size and stiffness contrast allow it / never;
    # "force": on grids of any size (the contrast limit still applies)
    o.spectrum16 = 2 if spectrum16 == "force" else 1 if spectrum16 else 0
    return o


# compiled candidates per pass: tile shapes 0-3, radix plans 1 and 2 on the
# default tile (4, 5)
TILE_VARIANTS = 6


def ffth_tile_variants(plan):
    out = (ctypes.c_int32 * 8)()
    _check(load().ffth_tile_variants(plan, out), "ffth_tile_variants")
    return list(out)


def ffth_set_tile_variants(plan, variants):
    arr = (ctypes.c_int32 * 8)(*[int(v) for v in variants])
    _check(load().ffth_set_tile_variants(plan, arr), "ffth_set_tile_variants")


def ffth_launch_loads(plan):
    out = (ctypes.c_int32 * 2)()
    _check(load().ffth_launch_loads(plan, out), "ffth_launch_loads")
    return list(out)


def ffth_set_launch_loads(plan, widths):
    arr = (ctypes.c_int32 * 2)(*[int(v) for v in widths])
    _check(load().ffth_set_launch_loads(plan, arr), "ffth_set_launch_loads")


def ffth_size_supported(n):
    return bool(load().ffth_size_supported(int(n)))


SPECTRUM16_MAX_CONTRAST = 128.0   # FFTH_SPECTRUM16_MAX_CONTRAST
SPECTRUM16_MIN_VOXELS = 128 ** 3   # FFTH_SPECTRUM16_MIN_VOXELS


def ffth_stiffness_contrast(lame=None, voigt21=None):
    """Largest over smallest eigen-modulus (Mandel form) across the phases;
    inf when a phase is not positive definite."""
    if lame is not None:
        a, ptr = _darr(np.asarray(lame, dtype=np.float64).reshape(-1, 2))
        return float(load().ffth_stiffness_contrast(a.shape[0], ptr, None))
    a, ptr = _darr(np.asarray(voigt21, dtype=np.float64).reshape(-1, 21))
    return float(load().ffth_stiffness_contrast(a.shape[0], None, ptr))


def ffth_workspace_bytes(n, nphases, nloads, order, opts):
    arr = (ctypes.c_int32 * 3)(*n)
    return int(load().ffth_workspace_bytes(arr, nphases, nloads, order, ctypes.byref(opts)))


def ffth_plan_create(problem, opts, nloads, order, workspace_ptr, nbytes, stream_ptr=None):
    plan = ctypes.c_void_p()
    st = load().ffth_plan_create(ctypes.byref(plan), ctypes.byref(problem), ctypes.byref(opts), nloads, order,
                                 workspace_ptr, nbytes, stream_ptr)
    _check(st, "ffth_plan_create")
    return plan


def ffth_plan_destroy(plan):
    _check(load().ffth_plan_destroy(plan), "ffth_plan_destroy")


def ffth_solve_order0(plan, E, eps_ptr, nloads):
    e, ep = _darr(E)
    res = (ffth_result * nloads)()
    st = load().ffth_solve_order0(plan, nloads, ep, eps_ptr, res)
    return st, [r.as_dict() for r in res]


def ffth_solve_order1(plan, eps0_ptr, G, eps_ptr, nloads):
    g, gp = _darr(G)
    res = (ffth_result * nloads)()
    st = load().ffth_solve_order1(plan, eps0_ptr, nloads, gp, eps_ptr, res)
    return st, [r.as_dict() for r in res]


def ffth_green_apply(plan, tau_ptr, eta_ptr, precision=FFTH_FP64):
    _check(load().ffth_green_apply(plan, tau_ptr, eta_ptr, precision), "ffth_green_apply")


NOALLOC_MAX_VOXELS = 262144   # FFTH_NOALLOC_MAX_VOXELS


def ffth_green_apply_noalloc(n, lambda0, mu0, tau_ptr, eta_ptr, precision=FFTH_FP64, stream_ptr=None):
    """eta = -Gamma0 * tau without a plan or workspace (the library's fixed
    per-GPU array); queued on the stream, returns without waiting."""
    arr = (ctypes.c_int32 * 3)(*n)
    _check(load().ffth_green_apply_noalloc(arr, lambda0, mu0, tau_ptr, eta_ptr, precision, stream_ptr),
           "ffth_green_apply_noalloc")


def ffth_displacement(plan, eps_ptr, u_ptr):
    _check(load().ffth_displacement(plan, eps_ptr, u_ptr), "ffth_displacement")


def ffth_order1_rhs(plan, eps0_ptr, G, p_ptr):
    g, gp = _darr(G)
    gm = (ctypes.c_double * 3)()
    _check(load().ffth_order1_rhs(plan, eps0_ptr, gp, p_ptr, gm), "ffth_order1_rhs")
    return list(gm)


def ffth_solve_order2(plan, eps0_ptr, eps1_ptr, H, eps_ptr, nloads):
    h, hp = _darr(H)
    res = (ffth_result * nloads)()
    st = load().ffth_solve_order2(plan, eps0_ptr, eps1_ptr, nloads, hp, eps_ptr, res)
    return st, [r.as_dict() for r in res]


def ffth_order2_rhs(plan, eps0_ptr, eps1_ptr, H, p_ptr):
    h, hp = _darr(H)
    gm = (ctypes.c_double * 3)()
    _check(load().ffth_order2_rhs(plan, eps0_ptr, eps1_ptr, hp, p_ptr, gm), "ffth_order2_rhs")
    return list(gm)


def ffth_profile_enable(plan, on=True):
    _check(load().ffth_profile_enable(plan, 1 if on else 0), "ffth_profile_enable")


PROFILE_CATEGORIES = 14


def ffth_profile_read(plan):
    """{category name: (launches, total ms, loads processed)} for every kernel category."""
    lib = load()
    out = {}
    for c in range(PROFILE_CATEGORIES):
        n = ctypes.c_int64()
        u = ctypes.c_int64()
        ms = ctypes.c_double()
        _check(lib.ffth_profile_read(plan, c, ctypes.byref(n), ctypes.byref(u), ctypes.byref(ms)),
               "ffth_profile_read")
        out[lib.ffth_profile_name(c).decode()] = (int(n.value), float(ms.value), int(u.value))
    return out


class Solver:
    """One plan over a phase field on cuda:0 (or the given device).

    phase: numpy/torch uint16 array (n0, n1, n2); lame: (nphases, 2) or
    voigt21: (nphases, 21); lam0, mu0: reference medium.  spectrum16 (mixed
    CG): True keeps the inner solve's forward spectrum in binary16 where the
    grid size and stiffness contrast allow it, "force" on grids of any size
    (within the contrast limit), False never (options of include/ffth.h).
    """

    def __init__(self, phase, lam0, mu0, lame=None, voigt21=None, nloads=1, order=0, scheme="cg",
                 precision="mixed", tol=1e-8, max_iter=20000, inner_tol=1e-3, max_outer=30, check_every=8,
                 autotune=True, spectrum16=True, device="cuda:0", stream=None):
        import torch
        self.torch = torch
        self.device = torch.device(device)
        if self.device.type == "cuda" and self.device.index is None:
            self.device = torch.device("cuda", torch.cuda.current_device())
        if isinstance(phase, np.ndarray):
            ph = torch.from_numpy(np.ascontiguousarray(phase.astype(np.int16, copy=False).view(np.int16)))
        else:
            ph = phase.to(torch.int16)
        self.phase = ph.contiguous().to(self.device)
        self.n = tuple(int(v) for v in self.phase.shape)
        self.nvox = int(np.prod(self.n))
        self.nloads = nloads
        self.order = order
        self.opts = make_opts(scheme, precision, tol, max_iter, inner_tol, max_outer, check_every, autotune,
                              spectrum16)
        self._lame = None if lame is None else _darr(lame)
        self._v21 = None if voigt21 is None else _darr(voigt21)
        nph = (len(np.asarray(lame).reshape(-1, 2)) if lame is not None
               else len(np.asarray(voigt21).reshape(-1, 21)))
        self.problem = ffth_problem()
        self.problem.n = (ctypes.c_int32 * 3)(*self.n)
        self.problem.nphases = nph
        self.problem.phase = self.phase.data_ptr()
        self.problem.lame = self._lame[1] if self._lame else None
        self.problem.stiffness = self._v21[1] if self._v21 else None
        self.problem.lambda0 = lam0
        self.problem.mu0 = mu0
        nbytes = ffth_workspace_bytes(self.n, nph, nloads, order, self.opts)
        if nbytes == 0:
            raise FFTHError(FFTH_ERR_INVALID, f"unsupported configuration n={self.n}")
        self.ws = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.plan = ffth_plan_create(self.problem, self.opts, nloads, order, _dptr(self.ws), nbytes,
                                     ctypes.c_void_p(self.stream.cuda_stream))

    def close(self):
        if getattr(self, "plan", None) is not None:
            ffth_plan_destroy(self.plan)
            self.plan = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def tile_variants(self):
        """Tile variant per pass: [xf32, xf64, y32, y64, z32, z64, xi32, xi64]."""
        return ffth_tile_variants(self.plan)

    @tile_variants.setter
    def tile_variants(self, v):
        ffth_set_tile_variants(self.plan, v)

    @property
    def launch_loads(self):
        """Loads per launch of the iteration passes [FP32, FP64] (0: all at once)."""
        return ffth_launch_loads(self.plan)

    @launch_loads.setter
    def launch_loads(self, v):
        ffth_set_launch_loads(self.plan, v)

    def _out(self, out, nl):
        if out is None:
            return self.field(6, nl)
        return check_field(out, self.device, (nl, 6) + self.n, "out")

    def field(self, comps=6, nloads=1):
        return self.torch.empty((nloads, comps) + self.n, dtype=self.torch.float64, device=self.device)

    def solve_order0(self, E, out=None, check=True):
        E = np.asarray(E, dtype=np.float64).reshape(-1, 6)
        nl = E.shape[0]
        if nl > self.nloads:
            raise FFTHError(FFTH_ERR_INVALID, f"{nl} load cases, the plan holds {self.nloads}")
        eps = self._out(out, nl)
        st, res = ffth_solve_order0(self.plan, E, _dptr(eps), nl)
        if check:
            _check(st, "ffth_solve_order0")
        return eps, res

    def solve_order1(self, eps0_six, G, out=None, check=True):
        G = np.asarray(G, dtype=np.float64).reshape(-1, 18)
        nl = G.shape[0]
        if nl > self.nloads:
            raise FFTHError(FFTH_ERR_INVALID, f"{nl} load cases, the plan holds {self.nloads}")
        eps = self._out(out, nl)
        e0 = check_field(eps0_six, self.device, (6, 6) + self.n, "eps0_six")
        st, res = ffth_solve_order1(self.plan, _dptr(e0), G, _dptr(eps), nl)
        if check:
            _check(st, "ffth_solve_order1")
        return eps, res

    def green_apply(self, tau, precision="fp64"):
        tau = check_field(tau, self.device, (6,) + self.n, "tau")
        eta = self.torch.empty_like(tau)
        ffth_green_apply(self.plan, _dptr(tau), _dptr(eta), PRECISIONS[precision])
        return eta

    def displacement(self, eps):
        eps = check_field(eps, self.device, (6,) + self.n, "eps")
        u = self.torch.empty((3,) + self.n, dtype=self.torch.float64, device=self.device)
        ffth_displacement(self.plan, _dptr(eps), _dptr(u))
        return u

    def solve_order2(self, eps0_six, eps1_18, H, out=None, check=True):
        H = np.asarray(H, dtype=np.float64).reshape(-1, 54)
        nl = H.shape[0]
        if nl > self.nloads:
            raise FFTHError(FFTH_ERR_INVALID, f"{nl} load cases, the plan holds {self.nloads}")
        eps = self._out(out, nl)
        e0 = check_field(eps0_six, self.device, (6, 6) + self.n, "eps0_six")
        e1 = check_field(eps1_18, self.device, (18, 6) + self.n, "eps1_18")
        st, res = ffth_solve_order2(self.plan, _dptr(e0), _dptr(e1), H, _dptr(eps), nl)
        if check:
            _check(st, "ffth_solve_order2")
        return eps, res

    def order2_rhs(self, eps0_six, eps1_18, H):
        p = self.torch.empty((6,) + self.n, dtype=self.torch.float64, device=self.device)
        eps0_six = check_field(eps0_six, self.device, (6, 6) + self.n, "eps0_six")
        eps1_18 = check_field(eps1_18, self.device, (18, 6) + self.n, "eps1_18")
        gm = ffth_order2_rhs(self.plan, _dptr(eps0_six), _dptr(eps1_18),
                             np.asarray(H, np.float64).reshape(54), _dptr(p))
        return p, gm

    def order1_rhs(self, eps0_six, G):
        p = self.torch.empty((6,) + self.n, dtype=self.torch.float64, device=self.device)
        eps0_six = check_field(eps0_six, self.device, (6, 6) + self.n, "eps0_six")
        gm = ffth_order1_rhs(self.plan, _dptr(eps0_six), np.asarray(G, np.float64).reshape(18),
                             _dptr(p))
        return p, gm


def ffth_request_bytes(n, nphases, nloads, opts):
    arr = (ctypes.c_int32 * 3)(*n)
    return int(load().ffth_request_bytes(arr, nphases, nloads, ctypes.byref(opts)))


def ffth_server_create(arena_ptr, nbytes, opts, max_running, stream_ptr=None):
    srv = ctypes.c_void_p()
    _check(load().ffth_server_create(ctypes.byref(srv), arena_ptr, nbytes, ctypes.byref(opts), max_running,
                                     stream_ptr), "ffth_server_create")
    return srv


def ffth_submit(srv, problem, E):
    e, ep = _darr(E)
    rid = ctypes.c_uint64()
    _check(load().ffth_submit(srv, ctypes.byref(problem), e.shape[0], ep, ctypes.byref(rid)), "ffth_submit")
    return int(rid.value)


def ffth_server_step(srv):
    run, wait = ctypes.c_int32(), ctypes.c_int32()
    _check(load().ffth_server_step(srv, ctypes.byref(run), ctypes.byref(wait)), "ffth_server_step")
    return run.value, wait.value


def ffth_poll(srv, rid, nloads):
    """(status, results): status FFTH_ERR_BUSY while running."""
    res = (ffth_result * nloads)()
    st = load().ffth_poll(srv, rid, res)
    return st, ([r.as_dict() for r in res] if st != FFTH_ERR_BUSY else None)


def ffth_cancel(srv, rid):
    _check(load().ffth_cancel(srv, rid), "ffth_cancel")


def ffth_server_stats(srv):
    it = ctypes.c_int64()
    grids = ctypes.c_int32()
    _check(load().ffth_server_stats(srv, ctypes.byref(it), ctypes.byref(grids)), "ffth_server_stats")
    return {"multi_iterations": it.value, "multi_max_grids": grids.value}


def ffth_server_destroy(srv):
    _check(load().ffth_server_destroy(srv), "ffth_server_destroy")

