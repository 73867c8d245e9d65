"""FP64 CPU oracle for the implicit grey FLD radiation step.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  The product
library (``paper_1306_0645_amd``) never imports it and shares no code with it.

The arithmetic lives in ``fld_oracle.c`` (plain C, FP64, no fast-math), built
with gcc into ``liboracle.so`` beside this file.  This module only marshals
numpy arrays.  Every routine follows the paper (Norman et al. 2014,
arXiv:1306.0645):

* ``face_limiter`` / ``faces`` -- the limiter D and its face means (Sec. 2).
* ``apply_L`` -- the finite-volume form of the right-hand side of eq. "fld"
  without eta (Sec. 3.3).
* ``system`` / ``apply_A`` / ``solve`` -- the theta-method linear system in
  residual-correction form, (I - theta dt L) dE = dt (L E^n + eta), solved
  with Jacobi-PCG (Sec. 3.3).
* ``residual_at`` -- b - A x at chosen cells, each computed on its own.
* ``step`` -- one radiation step with the 10x cut-and-subcycle rule
  (Sec. 3.4); its dt estimator is a reading of ours and is PARITY UNPINNED.
* ``chem_h`` -- the loosely coupled chemistry update (Sec. 3.3) for isothermal
  pure hydrogen, the gas of Test 1 (Sec. 4.1.1).
* ``hii_run`` -- radiation then chemistry per step in the order of Sec. 3.4,
  pinned by the Stromgren-sphere growth law of Test 1.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "fld_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
# the same source with OpenMP over its cell loops: only for timing the oracle
# on all host cores (its reductions sum in another order)
_LIB_OMP = os.path.join(_HERE, "liboracle_omp.so")

OK, NOCONV, NONFINITE, BADARG = 0, 1, 2, 3

# Paper limiter constants (Sec. 2): D_max = 0.006 c L_unit, R_min = 1e-20 / L_unit
DMAX_FACTOR = 0.006
RMIN_FACTOR = 1e-20


def _compile(out, extra):
    tmp = out + ".tmp"
    subprocess.check_call(
        ["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-fno-fast-math", *extra,
         "-o", tmp, _SRC, "-lm"])
    os.replace(tmp, out)


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain -O2, no fast-math), serially and
    with OpenMP."""
    if force or not os.path.exists(_LIB):
        _compile(_LIB, [])
    if force or not os.path.exists(_LIB_OMP):
        _compile(_LIB_OMP, ["-fopenmp"])
    return _LIB


_libs = {}


def _load(parallel: bool = False):
    """The serial library (every parity check) or, with parallel, the OpenMP
    build (timing only)."""
    lib = _libs.get(parallel)
    if lib is None:
        path = _LIB_OMP if parallel else _LIB
        if not os.path.exists(path):
            build(force=True)
        lib = ctypes.CDLL(path)
        d, i, p = ctypes.c_double, ctypes.c_int, ctypes.c_void_p
        i64 = ctypes.c_int64
        lib.oracle_threads.restype = i
        lib.oracle_threads.argtypes = [i]
        lib.oracle_face_limiter.restype = d
        lib.oracle_face_limiter.argtypes = [d] * 8
        lib.oracle_faces.restype = None
        lib.oracle_faces.argtypes = [i, i, i, d, d, d, p, p, d, d, d, p, p, p]
        lib.oracle_apply_L.restype = None
        lib.oracle_apply_L.argtypes = [i, i, i, d, d, d, p, p, p, p, d, d, p, p]
        lib.oracle_system.restype = None
        lib.oracle_system.argtypes = [i, i, i, d, d, d, p, p, p, d, d, d, d, d,
                                      d, d, p, p, p, p, p]
        lib.oracle_apply_A.restype = None
        lib.oracle_apply_A.argtypes = [i, i, i, d, d, d, p, p, d, d, d, d, d, d,
                                       d, p, p]
        lib.oracle_solve.restype = i
        lib.oracle_solve.argtypes = [i, i, i, d, d, d, p, p, p, d, d, d, d, d,
                                     d, d, d, i, p, ctypes.POINTER(i),
                                     ctypes.POINTER(d)]
        lib.oracle_residual_at.restype = None
        lib.oracle_residual_at.argtypes = [i, i, i, d, d, d, p, p, p, d, d, d,
                                           d, d, d, d, p, p, i64, p, p]
        lib.oracle_step.restype = i
        lib.oracle_step.argtypes = [i, i, i, d, d, d, p, p, p, d, d, d, d, d,
                                    d, d, d, i, d, d, i, p]
        lib.oracle_chem_h.restype = None
        lib.oracle_chem_h.argtypes = [i64, p, p, p, p, d, i, d, d, d, d, d]
        _libs[parallel] = lib
    return lib


def threads(n: int = 0) -> int:
    """Threads of the OpenMP build (n > 0 sets them); the serial build uses 1."""
    return int(_load(True).oracle_threads(int(n)))


def _arr(x, shape=None):
    a = np.ascontiguousarray(x, dtype=np.float64)
    if shape is not None and a.shape != tuple(shape):
        raise ValueError(f"expected shape {shape}, got {a.shape}")
    return a


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def limits(c: float, L_unit: float):
    """(D_max, R_min) from the paper's definitions (Sec. 2)."""
    return DMAX_FACTOR * c * L_unit, RMIN_FACTOR / L_unit


def face_limiter(E1, E2, k1, k2, dxd, c, d_max, r_min) -> float:
    return _load().oracle_face_limiter(E1, E2, k1, k2, dxd, c, d_max, r_min)


def faces(E, kappa, h, c, d_max, r_min):
    """Face limiters (Dx, Dy, Dz) on the +faces of every cell; fields are [nz,ny,nx]."""
    E = _arr(E)
    kappa = _arr(kappa, E.shape)
    nz, ny, nx = E.shape
    out = [np.empty_like(E) for _ in range(3)]
    _load().oracle_faces(nx, ny, nz, h[0], h[1], h[2], _ptr(E), _ptr(kappa), c,
                         d_max, r_min, *[_ptr(o) for o in out])
    return tuple(out)


def apply_L(Dx, Dy, Dz, kappa, u, h, c, adot_over_a):
    u = _arr(u)
    nz, ny, nx = u.shape
    Dx, Dy, Dz, kappa = (_arr(v, u.shape) for v in (Dx, Dy, Dz, kappa))
    out = np.empty_like(u)
    _load().oracle_apply_L(nx, ny, nz, h[0], h[1], h[2], _ptr(Dx), _ptr(Dy),
                           _ptr(Dz), _ptr(kappa), c, adot_over_a, _ptr(u),
                           _ptr(out))
    return out


class Problem:
    """One step's frozen data: E^n, kappa, eta, dt, a, adot and the constants."""

    def __init__(self, E, kappa, eta, h, c, d_max, r_min, dt, theta=1.0, a=1.0,
                 adot=0.0, parallel=False):
        # parallel: run on the OpenMP build (timing only; parity uses the
        # serial build)
        self._lib = _load(parallel)
        self.E = _arr(E)
        self.kappa = _arr(kappa, self.E.shape)
        self.eta = _arr(eta, self.E.shape)
        self.h = tuple(float(v) for v in h)
        self.c, self.d_max, self.r_min = float(c), float(d_max), float(r_min)
        self.dt, self.theta = float(dt), float(theta)
        self.a, self.adot = float(a), float(adot)

    @property
    def shape(self):
        return self.E.shape

    def _common(self):
        nz, ny, nx = self.E.shape
        return (nx, ny, nz, self.h[0], self.h[1], self.h[2])

    def system(self):
        """(diag, Ax, Ay, Az, b): A_pp, -A_{p,p+e_d}, and the right-hand side."""
        outs = [np.empty_like(self.E) for _ in range(5)]
        self._lib.oracle_system(*self._common(), _ptr(self.E), _ptr(self.kappa),
                              _ptr(self.eta), self.c, self.d_max, self.r_min,
                              self.theta, self.dt, self.a, self.adot,
                              *[_ptr(o) for o in outs])
        return tuple(outs)

    def apply_A(self, u):
        u = _arr(u, self.E.shape)
        out = np.empty_like(u)
        self._lib.oracle_apply_A(*self._common(), _ptr(self.E), _ptr(self.kappa),
                               self.c, self.d_max, self.r_min, self.theta,
                               self.dt, self.a, self.adot, _ptr(u), _ptr(out))
        return out

    def solve(self, tol=1e-13, max_iter=100000):
        """dE solving A dE = b by Jacobi-PCG; returns (dE, status, iters, relres)."""
        dE = np.empty_like(self.E)
        it = ctypes.c_int(0)
        rr = ctypes.c_double(0.0)
        st = self._lib.oracle_solve(*self._common(), _ptr(self.E), _ptr(self.kappa),
                                  _ptr(self.eta), self.c, self.d_max,
                                  self.r_min, self.theta, self.dt, self.a,
                                  self.adot, tol, max_iter, _ptr(dE),
                                  ctypes.byref(it), ctypes.byref(rr))
        return dE, st, it.value, rr.value

    def residual_at(self, x, cells):
        """(b - A x, b) at the given linear cell indices, each computed alone."""
        x = _arr(x, self.E.shape)
        cells = np.ascontiguousarray(cells, dtype=np.int64)
        res = np.empty(cells.shape, dtype=np.float64)
        rhs = np.empty(cells.shape, dtype=np.float64)
        self._lib.oracle_residual_at(*self._common(), _ptr(self.E),
                                   _ptr(self.kappa), _ptr(self.eta), self.c,
                                   self.d_max, self.r_min, self.theta, self.dt,
                                   self.a, self.adot, _ptr(x), _ptr(cells),
                                   cells.size, _ptr(res), _ptr(rhs))
        return res, rhs


def step(E, kappa, eta, h, c, d_max, r_min, dt, theta=1.0, a=1.0, adot=0.0,
         tol=1e-13, max_iter=100000, tau_tol=1e-4, e_floor=0.0, max_cuts=8):
    """One radiation step with cut-and-subcycle; returns (E_new, status, stats)."""
    E = _arr(E).copy()
    kappa = _arr(kappa, E.shape)
    eta = _arr(eta, E.shape)
    nz, ny, nx = E.shape
    stats = np.zeros(6)
    st = _load().oracle_step(nx, ny, nz, h[0], h[1], h[2], _ptr(E), _ptr(kappa),
                             _ptr(eta), c, d_max, r_min, theta, dt, a, adot,
                             tol, max_iter, tau_tol, e_floor, max_cuts,
                             _ptr(stats))
    keys = ("substeps", "cuts", "iters", "relres", "rho", "dt_next")
    return E, st, dict(zip(keys, stats.tolist()))


# ---------------------------------------------------------------------------
# Isothermal hydrogen chemistry and the operator-split Test-1 driver
# ---------------------------------------------------------------------------

def chem_h(E, n_h, x, dt, c, sigma, hnu, alpha_b, substeps=1, a=1.0):
    """Loosely coupled chemistry update of the ionized fraction (Sec. 3.3) for
    pure hydrogen at fixed temperature; returns (x_new, kappa_new) with
    kappa = sigma n_HI (proper).  E and n_h are comoving densities at
    expansion factor a.  See ``oracle_chem_h`` for the update."""
    E = _arr(E)
    n_h = _arr(n_h, E.shape)
    xo = _arr(x, E.shape).copy()
    kappa = np.empty_like(E)
    _load().oracle_chem_h(E.size, _ptr(E), _ptr(n_h), _ptr(xo), _ptr(kappa),
                          float(dt), int(substeps), float(c), float(sigma),
                          float(hnu), float(alpha_b), float(a))
    return xo, kappa


def ionized_radius(x, cell_volume):
    """Radius of the sphere whose volume is the ionized volume sum(x) V_cell."""
    return (3.0 * float(np.sum(x)) * cell_volume / (4.0 * math.pi)) ** (1.0 / 3.0)


def eds_expansion(t, H0):
    """Expansion factor and its rate in an Einstein-de Sitter universe (the
    Friedmann solution for Omega_m = 1): a = (3 H0 t / 2)^(2/3) with a = 1 at
    the present, adot = (2 / (3 t)) a."""
    a = (1.5 * H0 * t) ** (2.0 / 3.0)
    return a, a * 2.0 / (3.0 * t)


def hii_run(E, x, n_h, eta, h, c, d_max, r_min, sigma, hnu, alpha_b, outputs,
            dt0, tau_tol, e_floor, chem_substeps=1, tol=1e-13, max_cuts=8,
            dts=None, max_steps=10 ** 7, t0=0.0, H0=None, theta=1.0,
            spacing="comoving"):
    """Radiation + chemistry in the operator-split order of Sec. 3.4.

    Each step t -> t + dt: the radiation step (with its 10x cut-and-subcycle
    rule) evolves E with kappa held at the current ionization state; the new E
    then drives the chemistry over the same dt, which gives the opacity of
    the next step.  With static gas the radiation estimate alone sets the
    next dt (Sec. 3.4 takes the minimum over the processes), clipped so that
    steps land on the output times (absolute times, the run starts at t0).
    ``dts`` replays a given sequence of step sizes instead.  With H0 the
    fields are comoving in an Einstein-de Sitter background: each step uses
    a and adot at its midpoint.  spacing: "comoving" (the reading the solver
    takes) poses eq. "fld" as printed, every spatial derivative with respect
    to the comoving position (Sec. 2); "proper" instead poses the diffusion
    operator on the proper separation a h of the comoving cells (the step is
    given a h), for comparing the two readings.
    Returns the final fields, the ionized radius (comoving) at every output
    time and the step sizes taken."""
    E = _arr(E).copy()
    x = _arr(x, E.shape).copy()
    n_h = _arr(n_h, E.shape)
    eta = _arr(eta, E.shape)
    vcell = h[0] * h[1] * h[2]
    a0 = eds_expansion(t0, H0)[0] if H0 else 1.0
    kappa = sigma * (n_h / a0 ** 3) * (1.0 - x)
    outputs = [float(o) for o in outputs]
    t, dt, k, i = float(t0), float(dt0), 0, 0
    radii, taken, iters = [], [], 0
    while k < len(outputs) and i < max_steps:
        target = outputs[k]
        step_dt = float(dts[i]) if dts is not None else min(dt, target - t)
        a, adot = eds_expansion(t + 0.5 * step_dt, H0) if H0 else (1.0, 0.0)
        hs = h if spacing == "comoving" else tuple(v * a for v in h)
        E, st, s = step(E, kappa, eta, hs, c, d_max, r_min, step_dt,
                        theta=theta, a=a, adot=adot, tol=tol,
                        tau_tol=tau_tol, e_floor=e_floor, max_cuts=max_cuts)
        if st != OK:
            raise RuntimeError(f"oracle radiation step failed with status {st}")
        x, kappa = chem_h(E, n_h, x, step_dt, c, sigma, hnu, alpha_b,
                          chem_substeps, a)
        iters += int(s["iters"])
        taken.append(step_dt)
        t += step_dt
        dt = s["dt_next"]
        i += 1
        if t >= target * (1.0 - 1e-12):
            t = target
            radii.append(ionized_radius(x, vcell))
            k += 1
    return {"E": E, "x": x, "kappa": kappa, "times": outputs[:len(radii)],
            "radii": radii, "dts": taken, "iters": iters}
