"""MI355X implicit grey flux-limited-diffusion (FLD) radiation step.

Thin ctypes binding over ``libfld.so`` (C-ABI declared in ``include/fld.h``).
Every step of the solve runs in the library's HIP kernels; this module only
marshals arguments.  PyTorch supplies device memory (workspaces, fields) and
the HIP stream.  There is no CPU fallback: importing raises if the library is
missing.

Low-level functions carry the C names (``fld_create``, ``fld_assemble``,
``fld_solve``, ``fld_step`` ...); ``Solver``, ``Batch`` and ``Server`` wrap a
handle for convenience.
"""
from __future__ import annotations

import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfld.so")

FLD_OK, FLD_EINVAL, FLD_ENOMEM, FLD_ENOCONV = 0, -1, -2, -3
FLD_ENONFINITE, FLD_EDEVICE, FLD_EBUSY = -4, -5, -6
FLD_PREC_FP64, FLD_PREC_MIXED = 0, 1
FLD_SMOOTH_RBGS, FLD_SMOOTH_JACOBI = 0, 1

EXPORTS = (
    "fld_default_params", "fld_strerror", "fld_workspace_bytes", "fld_create",
    "fld_assemble", "fld_solve", "fld_step", "fld_destroy", "fld_get_system",
    "fld_apply", "fld_precondition", "fld_batch_workspace_bytes",
    "fld_batch_create", "fld_batch_step", "fld_batch_destroy",
    "fld_server_create", "fld_server_submit", "fld_server_poll",
    "fld_server_drain", "fld_server_destroy",
    "fld_profile_num_kernels", "fld_profile_kernel_name", "fld_profile_select",
    "fld_profile_read", "fld_static_scratch_bytes", "fld_step_static",
    "fld_advance", "fld_batch_advance",
    "fld_chem_default_params", "fld_chem_h_update", "fld_chem_ionized_sum",
)


class Grid(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
                ("nz", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("dx", ctypes.c_double), ("dy", ctypes.c_double),
                ("dz", ctypes.c_double)]


class Params(ctypes.Structure):
    _fields_ = [("c", ctypes.c_double), ("theta", ctypes.c_double),
                ("d_max", ctypes.c_double), ("r_min", ctypes.c_double),
                ("rtol", ctypes.c_double), ("tau_tol", ctypes.c_double),
                ("e_floor", ctypes.c_double), ("coarse_scale", ctypes.c_double),
                ("max_iter", ctypes.c_int32), ("mg_levels", ctypes.c_int32),
                ("nu_pre", ctypes.c_int32), ("nu_post", ctypes.c_int32),
                ("precision", ctypes.c_int32), ("max_dt_cuts", ctypes.c_int32),
                ("tile_z", ctypes.c_int32), ("check_every", ctypes.c_int32),
                ("use_graph", ctypes.c_int32), ("fused_tile_z", ctypes.c_int32),
                ("cycle_switch", ctypes.c_int32), ("prolongation", ctypes.c_int32),
                ("warm_start", ctypes.c_int32), ("tail_cells", ctypes.c_int32),
                ("smoother", ctypes.c_int32), ("fused_levels", ctypes.c_int32),
                ("coarse_op", ctypes.c_int32), ("direction_fp64", ctypes.c_int32),
                ("local_sweeps", ctypes.c_int32), ("local_coupling", ctypes.c_double)]


class Stats(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("iters", ctypes.c_int32),
                ("subcycles", ctypes.c_int32), ("dt_cuts", ctypes.c_int32),
                ("levels", ctypes.c_int32), ("restarts", ctypes.c_int32),
                ("cycle_nu", ctypes.c_int32), ("trilinear", ctypes.c_int32),
                ("rel_resid", ctypes.c_double), ("err_bound", ctypes.c_double),
                ("rel_change_rms", ctypes.c_double), ("dt_next", ctypes.c_double),
                ("bnorm", ctypes.c_double), ("dEnorm", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class Request(ctypes.Structure):
    _fields_ = [("grid", Grid), ("n_steps", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("dt", ctypes.c_double),
                ("a", ctypes.c_double), ("adot", ctypes.c_double),
                ("E", ctypes.c_void_p), ("kappa", ctypes.c_void_p),
                ("eta", ctypes.c_void_p), ("E_out", ctypes.c_void_p)]


class Result(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("steps_done", ctypes.c_int32),
                ("iters", ctypes.c_int32), ("dt_cuts", ctypes.c_int32),
                ("queue_s", ctypes.c_double), ("latency_s", ctypes.c_double),
                ("rel_resid", ctypes.c_double), ("err_bound", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class ChemParams(ctypes.Structure):
    _fields_ = [("c", ctypes.c_double), ("sigma", ctypes.c_double),
                ("hnu", ctypes.c_double), ("alpha_b", ctypes.c_double),
                ("substeps", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class FLDError(RuntimeError):
    def __init__(self, status, what=""):
        self.status = status
        super().__init__(f"{what}: {fld_strerror(status)} ({status})")


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(
            f"{LIB_PATH} is missing: build it with "
            "`python paper_1306_0645_amd/build.py` (hipcc, gfx950)")
    lib = ctypes.CDLL(LIB_PATH)
    P, vp, i32, u64 = ctypes.POINTER, ctypes.c_void_p, ctypes.c_int32, ctypes.c_uint64
    d, sz = ctypes.c_double, ctypes.c_size_t
    sig = {
        "fld_default_params": (None, [P(Params), d, d]),
        "fld_strerror": (ctypes.c_char_p, [i32]),
        "fld_workspace_bytes": (sz, [P(Grid), P(Params)]),
        "fld_create": (i32, [P(Grid), P(Params), vp, vp, sz, P(vp)]),
        "fld_assemble": (i32, [vp, vp, vp, vp, d, d, d]),
        "fld_solve": (i32, [vp, vp, P(Stats)]),
        "fld_step": (i32, [vp, vp, vp, vp, d, d, d, P(Stats)]),
        "fld_destroy": (i32, [vp]),
        "fld_advance": (i32, [vp, vp, vp, vp, i32, d, d, d, d, i32, P(Stats),
                              P(i32)]),
        "fld_batch_advance": (i32, [vp, P(vp), P(vp), P(vp), i32, P(d), d, P(d),
                                    P(d), i32, P(Stats), P(i32)]),
        "fld_static_scratch_bytes": (sz, []),
        "fld_step_static": (i32, [P(Grid), P(Params), vp, vp, vp, vp, d, d, d,
                                  P(Stats)]),
        "fld_get_system": (i32, [vp, vp, vp, vp, vp, vp]),
        "fld_apply": (i32, [vp, vp, vp]),
        "fld_precondition": (i32, [vp, vp, vp]),
        "fld_batch_workspace_bytes": (sz, [i32, P(Grid), P(Params)]),
        "fld_batch_create": (i32, [i32, P(Grid), P(Params), vp, vp, sz, P(vp)]),
        "fld_batch_step": (i32, [vp, P(vp), P(vp), P(vp), P(d), P(d), P(d),
                                 P(Stats)]),
        "fld_batch_destroy": (i32, [vp]),
        "fld_server_create": (i32, [P(Params), vp, sz, vp, P(vp)]),
        "fld_server_submit": (i32, [vp, P(Request), P(u64)]),
        "fld_server_poll": (i32, [vp, u64, P(Result)]),
        "fld_server_drain": (i32, [vp]),
        "fld_server_destroy": (i32, [vp]),
        "fld_profile_num_kernels": (i32, []),
        "fld_profile_kernel_name": (ctypes.c_char_p, [i32]),
        "fld_profile_select": (i32, [i32]),
        "fld_profile_read": (i32, [i32, P(d), P(ctypes.c_int64)]),
        "fld_chem_default_params": (None, [P(ChemParams)]),
        "fld_chem_h_update": (i32, [P(Grid), P(ChemParams), vp, vp, vp, vp, vp,
                                    d, d]),
        "fld_chem_ionized_sum": (i32, [P(Grid), vp, vp, vp]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    return lib


_lib = _load()


def fld_strerror(status: int) -> str:
    return _lib.fld_strerror(int(status)).decode()


def _check(status, what):
    if status != FLD_OK:
        raise FLDError(status, what)


def _stream_ptr(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _dptr(t, n=None, name="field"):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != torch.float64 or not t.is_contiguous():
        raise TypeError(f"{name} must be contiguous float64")
    if n is not None and t.numel() != n:
        raise ValueError(f"{name} has {t.numel()} cells, expected {n}")
    return ctypes.c_void_p(t.data_ptr())


def _workspace(nbytes, device):
    # torch's caching allocator returns >= 512-byte aligned blocks
    ws = torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device=device)
    if ws.data_ptr() % 256:
        raise RuntimeError("workspace is not 256-byte aligned")
    return ws


def fld_default_params(c_light: float, L_unit: float, /, **overrides) -> Params:
    """Paper defaults for light speed c_light and length unit L_unit, with
    any Params field overridden by keyword."""
    p = Params()
    _lib.fld_default_params(ctypes.byref(p), float(c_light), float(L_unit))
    for k, v in overrides.items():
        if not hasattr(p, k):
            raise KeyError(k)
        setattr(p, k, v)
    return p


def make_grid(shape, h) -> Grid:
    """Grid for a field of shape (nz, ny, nx) and cell sizes (dx, dy, dz)."""
    nz, ny, nx = (int(s) for s in shape)
    return Grid(nx, ny, nz, 0, float(h[0]), float(h[1]), float(h[2]))


def fld_workspace_bytes(grid: Grid, params: Params) -> int:
    return int(_lib.fld_workspace_bytes(ctypes.byref(grid), ctypes.byref(params)))


def profile_kernels():
    """Names of the kernels the timing hook can select, by id."""
    return [_lib.fld_profile_kernel_name(k).decode()
            for k in range(_lib.fld_profile_num_kernels())]


def fld_profile_select(k: int):
    """Time every launch of kernel id k with hipEvents (-1 none, -2 all)."""
    if _lib.fld_profile_select(int(k)) != 0:
        raise ValueError(k)


def fld_profile_read(k: int):
    """(total milliseconds, launches) timed for kernel id k."""
    ms, n = ctypes.c_double(), ctypes.c_int64()
    if _lib.fld_profile_read(int(k), ctypes.byref(ms), ctypes.byref(n)) != 0:
        raise RuntimeError("fld_profile_read failed")
    return ms.value, n.value


class Solver:
    """One fld_handle: assemble / solve / step on one periodic grid."""

    def __init__(self, shape, h, params: Params, device="cuda", stream=None):
        self.grid = make_grid(shape, h)
        self.params = params
        self.shape = tuple(int(s) for s in shape)
        self.n = self.shape[0] * self.shape[1] * self.shape[2]
        nbytes = fld_workspace_bytes(self.grid, params)
        if nbytes == 0:
            raise FLDError(FLD_EINVAL, "fld_workspace_bytes")
        self.device = torch.device(device)
        self.workspace = _workspace(nbytes, self.device)
        self.stream = stream
        self.handle = ctypes.c_void_p()
        _check(_lib.fld_create(ctypes.byref(self.grid), ctypes.byref(params),
                               _stream_ptr(stream),
                               ctypes.c_void_p(self.workspace.data_ptr()),
                               nbytes, ctypes.byref(self.handle)), "fld_create")
        self._keep = ()

    def close(self):
        if self.handle:
            _lib.fld_destroy(self.handle)
            self.handle = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def fld_assemble(self, E, kappa, eta, dt, a=1.0, adot=0.0):
        args = [_dptr(E, self.n, "E"), _dptr(kappa, self.n, "kappa"),
                _dptr(eta, self.n, "eta")]
        self._keep = (E, kappa, eta)
        _check(_lib.fld_assemble(self.handle, *args, float(dt), float(a),
                                 float(adot)), "fld_assemble")

    def fld_solve(self, dE=None, check=True):
        if dE is None:
            dE = torch.empty(self.shape, dtype=torch.float64, device=self.device)
        st = Stats()
        s = _lib.fld_solve(self.handle, _dptr(dE, self.n, "dE"), ctypes.byref(st))
        if check:
            _check(s, "fld_solve")
        return dE, st.as_dict()

    def fld_step(self, E, kappa, eta, dt, a=1.0, adot=0.0, check=True):
        st = Stats()
        s = _lib.fld_step(self.handle, _dptr(E, self.n, "E"),
                          _dptr(kappa, self.n, "kappa"), _dptr(eta, self.n, "eta"),
                          float(dt), float(a), float(adot), ctypes.byref(st))
        if check:
            _check(s, "fld_step")
        return st.as_dict()

    def fld_advance(self, E, kappa, eta, dt, n_steps=1, t_end=0.0, a=1.0,
                    adot=0.0, units=0, check=True):
        """Steps with the substep control on the device: n_steps steps of dt
        (n_steps = 0: steps of the controller's dt_next from dt until t_end).
        Returns the stats dict with 'steps' (steps completed) added."""
        st = Stats()
        done = ctypes.c_int32(0)
        s = _lib.fld_advance(self.handle, _dptr(E, self.n, "E"),
                             _dptr(kappa, self.n, "kappa"), _dptr(eta, self.n, "eta"),
                             int(n_steps), float(dt), float(t_end), float(a),
                             float(adot), int(units), ctypes.byref(st),
                             ctypes.byref(done))
        if check:
            _check(s, "fld_advance")
        out = st.as_dict()
        out["steps"] = done.value
        out["returned"] = s
        return out

    def fld_get_system(self):
        out = {k: torch.empty(self.shape, dtype=torch.float64, device=self.device)
               for k in ("diag", "Tx", "Ty", "Tz", "b")}
        _check(_lib.fld_get_system(self.handle, *[_dptr(out[k]) for k in
                                                  ("diag", "Tx", "Ty", "Tz", "b")]),
               "fld_get_system")
        return out

    def fld_apply(self, u):
        out = torch.empty(self.shape, dtype=torch.float64, device=self.device)
        _check(_lib.fld_apply(self.handle, _dptr(u, self.n, "u"), _dptr(out)),
               "fld_apply")
        return out

    def fld_precondition(self, r):
        z = torch.empty(self.shape, dtype=torch.float64, device=self.device)
        _check(_lib.fld_precondition(self.handle, _dptr(r, self.n, "r"), _dptr(z)),
               "fld_precondition")
        return z

    # short aliases
    assemble, solve, step, advance = fld_assemble, fld_solve, fld_step, fld_advance


def fld_static_scratch_bytes() -> int:
    """Size of the library's own device workspace used by fld_step_static."""
    return int(_lib.fld_static_scratch_bytes())


def fld_step_static(shape, h, params: Params, E, kappa, eta, dt, a=1.0, adot=0.0,
                    stream=None, check=True):
    """One radiation step on the library's own device workspace (no caller
    workspace and no device allocation): E is updated in place."""
    grid = make_grid(shape, h)
    n = grid.nx * grid.ny * grid.nz
    st = Stats()
    s = _lib.fld_step_static(ctypes.byref(grid), ctypes.byref(params),
                             _stream_ptr(stream), _dptr(E, n, "E"),
                             _dptr(kappa, n, "kappa"), _dptr(eta, n, "eta"),
                             float(dt), float(a), float(adot), ctypes.byref(st))
    if check:
        _check(s, "fld_step_static")
    return s, st.as_dict()


class Batch:
    """One fld_batch: a step for many independent problems of uneven sizes."""

    def __init__(self, shapes, hs, params: Params, device="cuda", stream=None):
        self.n = len(shapes)
        grids = (Grid * self.n)(*[make_grid(s, h) for s, h in zip(shapes, hs)])
        self.grids = grids
        self.shapes = [tuple(int(v) for v in s) for s in shapes]
        nbytes = int(_lib.fld_batch_workspace_bytes(self.n, grids,
                                                    ctypes.byref(params)))
        if nbytes == 0:
            raise FLDError(FLD_EINVAL, "fld_batch_workspace_bytes")
        self.workspace_bytes = nbytes
        self.workspace = _workspace(nbytes, torch.device(device))
        self.handle = ctypes.c_void_p()
        _check(_lib.fld_batch_create(self.n, grids, ctypes.byref(params),
                                     _stream_ptr(stream),
                                     ctypes.c_void_p(self.workspace.data_ptr()),
                                     nbytes, ctypes.byref(self.handle)),
               "fld_batch_create")

    def close(self):
        if self.handle:
            _lib.fld_batch_destroy(self.handle)
            self.handle = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def fld_batch_step(self, Es, kappas, etas, dts, a=None, adot=None,
                       check=True):
        n = self.n
        cells = [s[0] * s[1] * s[2] for s in self.shapes]
        VP = ctypes.c_void_p * n
        E = VP(*[_dptr(t, c, "E") for t, c in zip(Es, cells)])
        K = VP(*[_dptr(t, c, "kappa") for t, c in zip(kappas, cells)])
        H = VP(*[_dptr(t, c, "eta") for t, c in zip(etas, cells)])
        D = (ctypes.c_double * n)(*[float(v) for v in dts])
        A = (ctypes.c_double * n)(*([1.0] * n if a is None else [float(v) for v in a]))
        AD = (ctypes.c_double * n)(*([0.0] * n if adot is None else
                                     [float(v) for v in adot]))
        stats = (Stats * n)()
        s = _lib.fld_batch_step(self.handle, E, K, H, D, A, AD, stats)
        if check:
            _check(s, "fld_batch_step")
        return [st.as_dict() for st in stats]

    def fld_batch_advance(self, Es, kappas, etas, dts, n_steps=1, t_end=0.0,
                          a=None, adot=None, units=0, check=True):
        """fld_advance for every problem of the batch at once."""
        n = self.n
        cells = [s[0] * s[1] * s[2] for s in self.shapes]
        VP = ctypes.c_void_p * n
        E = VP(*[_dptr(t, c, "E") for t, c in zip(Es, cells)])
        K = VP(*[_dptr(t, c, "kappa") for t, c in zip(kappas, cells)])
        H = VP(*[_dptr(t, c, "eta") for t, c in zip(etas, cells)])
        D = (ctypes.c_double * n)(*[float(v) for v in dts])
        A = (ctypes.c_double * n)(*([1.0] * n if a is None else [float(v) for v in a]))
        AD = (ctypes.c_double * n)(*([0.0] * n if adot is None else
                                     [float(v) for v in adot]))
        stats = (Stats * n)()
        done = (ctypes.c_int32 * n)()
        s = _lib.fld_batch_advance(self.handle, E, K, H, int(n_steps), D,
                                   float(t_end), A, AD, int(units), stats, done)
        if check:
            _check(s, "fld_batch_advance")
        out = [st.as_dict() for st in stats]
        for o, d in zip(out, done):
            o["steps"] = int(d)
        return out

    step = fld_batch_step
    advance = fld_batch_advance


class Server:
    """One fld_server: continuous batching of step requests in an HBM arena."""

    def __init__(self, params: Params, arena_bytes: int, device="cuda",
                 stream=None):
        self.arena = _workspace(arena_bytes, torch.device(device))
        self.handle = ctypes.c_void_p()
        self._live = {}
        _check(_lib.fld_server_create(ctypes.byref(params),
                                      ctypes.c_void_p(self.arena.data_ptr()),
                                      int(arena_bytes), _stream_ptr(stream),
                                      ctypes.byref(self.handle)),
               "fld_server_create")

    def fld_server_submit(self, shape, h, E, kappa, eta, E_out, dt, n_steps=1,
                          a=1.0, adot=0.0):
        g = make_grid(shape, h)
        n = g.nx * g.ny * g.nz
        r = Request(g, int(n_steps), 0, float(dt), float(a), float(adot),
                    _dptr(E, n, "E"), _dptr(kappa, n, "kappa"),
                    _dptr(eta, n, "eta"), _dptr(E_out, n, "E_out"))
        t = ctypes.c_uint64()
        _check(_lib.fld_server_submit(self.handle, ctypes.byref(r), ctypes.byref(t)),
               "fld_server_submit")
        self._live[t.value] = (E, kappa, eta, E_out)
        return t.value

    def fld_server_poll(self, ticket):
        res = Result()
        s = _lib.fld_server_poll(self.handle, ctypes.c_uint64(ticket),
                                 ctypes.byref(res))
        if s == FLD_EBUSY:
            return None
        _check(s, "fld_server_poll")
        self._live.pop(ticket, None)
        return res.as_dict()

    def fld_server_drain(self):
        _check(_lib.fld_server_drain(self.handle), "fld_server_drain")

    def close(self):
        if self.handle:
            _lib.fld_server_destroy(self.handle)
            self.handle = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    submit, poll, drain = fld_server_submit, fld_server_poll, fld_server_drain


# ---------------------------------------------------------------------------
# Isothermal hydrogen chemistry (include/fld_chem.h)
# ---------------------------------------------------------------------------

def fld_chem_default_params(**overrides) -> ChemParams:
    """Test-1 chemistry constants (CGS), with any field overridden."""
    p = ChemParams()
    _lib.fld_chem_default_params(ctypes.byref(p))
    for k, v in overrides.items():
        if not hasattr(p, k):
            raise KeyError(k)
        setattr(p, k, v)
    return p


def fld_chem_h_update(grid: Grid, params: ChemParams, E, n_h, x, kappa, dt,
                      a=1.0, stream=None):
    """x and kappa updated in place over dt at expansion factor a (see
    include/fld_chem.h)."""
    n = grid.nx * grid.ny * grid.nz
    _check(_lib.fld_chem_h_update(ctypes.byref(grid), ctypes.byref(params),
                                  _stream_ptr(stream), _dptr(E, n, "E"),
                                  _dptr(n_h, n, "n_h"), _dptr(x, n, "x"),
                                  _dptr(kappa, n, "kappa"), float(dt),
                                  float(a)),
           "fld_chem_h_update")


def fld_chem_ionized_sum(grid: Grid, x, out=None, stream=None):
    """Device scalar (1-element float64 tensor) holding sum(x)."""
    n = grid.nx * grid.ny * grid.nz
    if out is None:
        out = torch.empty(1, dtype=torch.float64, device=x.device)
    _check(_lib.fld_chem_ionized_sum(ctypes.byref(grid), _stream_ptr(stream),
                                     _dptr(x, n, "x"), _dptr(out, 1, "out")),
           "fld_chem_ionized_sum")
    return out
