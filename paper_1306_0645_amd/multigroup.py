"""Multigroup FLD: one implicit FLD step per frequency group.

A multigroup discretisation of the radiation field (the extension Sec. 6
names for harder spectra) evolves one energy density E_g per group with its
own opacity kappa_g and emissivity eta_g.  Without inter-group coupling the
groups' steps are independent systems on the same mesh, so the cost grows
linearly with the number of groups.  Here all G systems advance together in
the batched engine: one launch per kernel and level covers every group's
tiles, and each group keeps its own PCG state and convergence test, so a
group's result is bit-identical to solving it alone.

Fields are packed (G, nz, ny, nx) float64 device tensors; this module only
hands per-group views to ``fld_batch_step``.
"""
from __future__ import annotations

import torch

from . import Batch, Params


class MultigroupFLD:
    """G groups on one periodic grid, stepped together."""

    def __init__(self, shape, h, groups: int, params: Params, device="cuda",
                 stream=None):
        if groups < 1:
            raise ValueError("groups must be >= 1")
        self.shape = tuple(int(v) for v in shape)
        self.groups = int(groups)
        self.batch = Batch([self.shape] * self.groups, [tuple(h)] * self.groups,
                           params, device=device, stream=stream)

    def close(self):
        self.batch.close()

    def _views(self, t, name):
        if t.dim() != 4 or tuple(t.shape) != (self.groups,) + self.shape:
            raise ValueError(f"{name} must have shape {(self.groups,) + self.shape}")
        if not t.is_contiguous():
            raise TypeError(f"{name} must be contiguous")
        return [t[g] for g in range(self.groups)]

    def step(self, E, kappa, eta, dt, a=1.0, adot=0.0):
        """Advance every group's E_g (in place) over dt; returns the
        per-group stats."""
        Es = self._views(E, "E")
        Ks = self._views(kappa, "kappa")
        Hs = self._views(eta, "eta")
        n = self.groups
        return self.batch.step(Es, Ks, Hs, [float(dt)] * n, [float(a)] * n,
                               [float(adot)] * n)
