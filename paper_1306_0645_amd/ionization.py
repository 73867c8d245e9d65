"""Operator-split radiation + isothermal hydrogen chemistry on the GPU.

Each step t -> t + dt follows the order of Sec. 3.4 for the loosely coupled
chemistry solver: the implicit FLD radiation step (``fld_step``, with its 10x
cut-and-subcycle rule) evolves E with the opacity of the current ionization
state; the new E then drives the chemistry (``fld_chem_h_update``) over the
same dt, which also writes the opacity of the next step.  With static gas
the radiation estimate alone sets the next dt (Sec. 3.4 takes the minimum
over the physical processes); steps are clipped to land on the output times,
where the ionized volume is reduced on the device (``fld_chem_ionized_sum``).

This is the driver of Test 1 (Sec. 4.1.1), the growth of an HII region
around a point source towards its Stromgren radius, and of Test 2
(Sec. 4.1.2), the same in an expanding Einstein-de Sitter universe: there the
fields are comoving, and each step passes the expansion factor a and its rate
at the step's midpoint to the radiation step (the operator on the proper
cell separation a dx, the ionizing-photon redshift term adot/a) and to the
chemistry (proper densities = comoving / a^3).  All field arithmetic runs in
the library's kernels; this module sequences calls and keeps time.
"""
from __future__ import annotations

import math
import time

import torch

from . import (ChemParams, Params, Solver, fld_chem_h_update,
               fld_chem_ionized_sum, make_grid)


def eds_expansion(H0):
    """a(t) and da/dt of an Einstein-de Sitter background (the Friedmann
    solution for Omega_m = 1, a = 1 at the present): a = (3 H0 t / 2)^(2/3),
    adot = 2 a / (3 t)."""
    def f(t):
        a = (1.5 * H0 * t) ** (2.0 / 3.0)
        return a, a * 2.0 / (3.0 * t)
    return f


class IsothermalHII:
    """Radiation + chemistry driver on one periodic grid; ``expansion`` maps
    cosmic time to (a, adot) for a comoving run (None: static, a = 1).

    On the slowly drifting fronts of Tests 1 and 2 the extrapolated warm start
    (``params.warm_start = 1``) takes fewer PCG iterations per step than the
    Galerkin default (7.7 against 9.4 on the 32^3 octant), so callers of these
    sweeps set it."""

    def __init__(self, shape, h, params: Params, chem: ChemParams,
                 device="cuda", expansion=None):
        self.shape = tuple(int(v) for v in shape)
        self.h = tuple(float(v) for v in h)
        self.params = params
        self.chem = chem
        self.device = torch.device(device)
        self.grid = make_grid(self.shape, self.h)
        self.solver = Solver(self.shape, self.h, params, device=self.device)
        self.cell_volume = self.h[0] * self.h[1] * self.h[2]
        self.expansion = expansion
        self._sum = torch.empty(1, dtype=torch.float64, device=self.device)

    def close(self):
        self.solver.close()

    def ionized_radius(self, x) -> float:
        """Radius of the sphere whose volume is the ionized volume."""
        fld_chem_ionized_sum(self.grid, x, out=self._sum)
        s = float(self._sum.item())
        return (3.0 * s * self.cell_volume / (4.0 * math.pi)) ** (1.0 / 3.0)

    def _a(self, t):
        return self.expansion(t) if self.expansion is not None else (1.0, 0.0)

    def run(self, E, x, n_h, eta, outputs, dt0, dts=None, max_steps=10 ** 7,
            on_output=None, wall_cap_s=None, t0=0.0):
        """Advance E and x (device tensors, updated in place) through the
        output times.  ``dts`` replays a given sequence of step sizes.  With
        ``wall_cap_s`` the run stops at the first output time reached after
        that much wall-clock time.  Returns the ionized radius at each output
        reached, the steps taken and the solver totals.  Output times are
        absolute; the run starts at t0."""
        kappa = torch.empty_like(E)
        fld_chem_h_update(self.grid, self.chem, E, n_h, x, kappa, 0.0,
                          self._a(t0)[0])
        outputs = [float(o) for o in outputs]
        t, dt, k, i = float(t0), float(dt0), 0, 0
        radii, taken = [], []
        capped = False
        iters = subcycles = cuts = 0
        torch.cuda.synchronize(self.device)
        t0 = time.perf_counter()
        while k < len(outputs) and i < max_steps:
            target = outputs[k]
            step_dt = float(dts[i]) if dts is not None else min(dt, target - t)
            a, adot = self._a(t + 0.5 * step_dt)
            st = self.solver.step(E, kappa, eta, step_dt, a, adot)
            fld_chem_h_update(self.grid, self.chem, E, n_h, x, kappa, step_dt, a)
            iters += st["iters"]
            subcycles += st["subcycles"]
            cuts += st["dt_cuts"]
            taken.append(step_dt)
            t += step_dt
            dt = st["dt_next"]
            i += 1
            if t >= target * (1.0 - 1e-12):
                t = target
                radii.append(self.ionized_radius(x))
                if on_output is not None:
                    on_output(t, radii[-1], i)
                k += 1
                if (wall_cap_s is not None and k < len(outputs)
                        and time.perf_counter() - t0 > wall_cap_s):
                    capped = True
                    break
        torch.cuda.synchronize(self.device)
        wall = time.perf_counter() - t0
        return {"times": outputs[:len(radii)], "radii": radii, "dts": taken,
                "steps": i, "iters": iters, "subcycles": subcycles,
                "dt_cuts": cuts, "wall_s": wall, "kappa": kappa,
                "dt_next": dt, "capped": capped}
