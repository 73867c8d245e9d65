"""Seeded synthetic inputs for the implicit grey FLD step.

This module only builds input fields (opacity, emissivity, initial radiation
energy) and step parameters.  It holds none of the solver's arithmetic: it
neither evaluates the limiter nor assembles or solves anything.  Both the
oracle-side tests and the GPU-side tests and benchmark draw their inputs here.

Inputs stand in for the paper's cosmological fields (Norman et al. 2014,
Sec. 5), which are not available: a smoothed lognormal neutral-hydrogen
density, opacity kappa = sigma_HI n_HI for monochromatic 13.6 eV radiation
(Sec. 4.1.1 sets the source at the HI ionization threshold), and point sources
of Ndot ionizing photons per second deposited as eta = sum Ndot h nu / V_cell
in the cell that holds them (Sec. 3.2 accumulates emissivity per cell).

All lengths are cm, times s, energies erg (CGS).  Randomness comes from numpy
PCG64 with base seed 1306 + workload index; problem i of a workload uses
SeedSequence([base, i]).
"""
from __future__ import annotations

import math

import numpy as np

C_LIGHT = 2.99792458e10          # cm / s
KPC = 3.0857e21                  # cm
MYR = 3.156e13                   # s
EV = 1.602176634e-12             # erg
HNU_HI = 13.6 * EV               # erg, HI ionization threshold
SIGMA_HI = 6.3e-18               # cm^2, HI cross-section at 13.6 eV
ALPHA_B = 2.59e-13               # cm^3 / s, case-B recombination at 1e4 K
DX_TEST1 = 6.6 * KPC / 32        # 206 pc: the 6.6 kpc Test-1 box on 32 cells

BASE_SEED = 1306


def rng_for(workload: int, problem: int = 0) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(
        np.random.SeedSequence([BASE_SEED + workload, problem])))


def smooth_gaussian(shape, sigma_cells: float, rng) -> np.ndarray:
    """White Gaussian noise smoothed by a periodic Gaussian kernel of
    ``sigma_cells``, renormalised to zero mean and unit variance."""
    g = rng.standard_normal(shape)
    if sigma_cells > 0:
        G = np.fft.rfftn(g, axes=(0, 1, 2))
        kz = np.fft.fftfreq(shape[0])[:, None, None]
        ky = np.fft.fftfreq(shape[1])[None, :, None]
        kx = np.fft.rfftfreq(shape[2])[None, None, :]
        k2 = (2 * np.pi) ** 2 * (kx * kx + ky * ky + kz * kz)
        G *= np.exp(-0.5 * sigma_cells ** 2 * k2)
        g = np.fft.irfftn(G, s=shape, axes=(0, 1, 2))
        del G
    g -= g.mean()
    sd = g.std()
    if sd > 0:
        g /= sd
    return g


def lognormal(shape, mean_density: float, sigma_ln: float, rng,
              smooth_cells: float = 1.5) -> np.ndarray:
    """n = exp(ln(mean_density) + sigma_ln * g), g smoothed Gaussian noise."""
    g = smooth_gaussian(shape, smooth_cells, rng)
    return np.exp(math.log(mean_density) + sigma_ln * g)


def point_sources(shape, n_src: int, lum_lo: float, lum_hi: float, rng):
    """(linear cell indices, Ndot) for sources at uniform random cells with
    log-uniform photon rates in [lum_lo, lum_hi]."""
    n = int(np.prod(shape))
    cells = rng.integers(0, n, size=n_src, dtype=np.int64)
    ndot = np.exp(rng.uniform(math.log(lum_lo), math.log(lum_hi), size=n_src))
    return cells, ndot


def emissivity(shape, cells, ndot, cell_volume: float) -> np.ndarray:
    """eta [erg cm^-3 s^-1]: photon rate times h nu per cell volume, summed
    over all sources that share a cell."""
    eta = np.zeros(int(np.prod(shape)))
    np.add.at(eta, np.asarray(cells, dtype=np.int64),
              np.asarray(ndot) * HNU_HI / cell_volume)
    return eta.reshape(shape)


def _problem(shape, dx, kappa, eta, E, L_unit, dt, name, theta=1.0):
    return {
        "name": name, "shape": tuple(shape), "h": (dx, dx, dx),
        "E": np.ascontiguousarray(E, dtype=np.float64),
        "kappa": np.ascontiguousarray(kappa, dtype=np.float64),
        "eta": np.ascontiguousarray(eta, dtype=np.float64),
        "c": C_LIGHT, "L_unit": L_unit, "dt": dt, "theta": theta,
        "a": 1.0, "adot": 0.0,
    }


def smooth_radiation(shape, eta, dt, rng, sigma_cells=8.0):
    """E^n = E0 exp(g), g smoothed at 8 cells, E0 = mean(eta) dt."""
    g = smooth_gaussian(shape, sigma_cells, rng)
    return float(np.mean(eta)) * dt * np.exp(g)


def single_source(n: int = 32, sigma_ln: float = 1.0, seed_problem: int = 0):
    """Workload 1: one FP64 step on n^3 (default 32^3) with a lognormal HI
    field (mean 1e-3 cm^-3), E^n = 0 and one 5e48 photon/s source in the
    centre cell; dt = 1e-3 light-crossing times of the box."""
    rng = rng_for(1, seed_problem)
    shape = (n, n, n)
    dx = DX_TEST1
    L = n * dx
    nH = lognormal(shape, 1e-3, sigma_ln, rng)
    kappa = SIGMA_HI * nH
    centre = (n // 2 * n + n // 2) * n + n // 2
    eta = emissivity(shape, [centre], [5e48], dx ** 3)
    dt = 1e-3 * L / C_LIGHT
    return _problem(shape, dx, kappa, eta, np.zeros(shape), L, dt,
                    f"single_source_{n}")


def many_sources(n: int = 256, sigma_ln: float = 1.5, n_src: int = 64,
                 seed_problem: int = 0):
    """Workload 2: n^3 (default 256^3), lognormal HI (sigma_ln 1.5), n_src
    sources with Ndot log-uniform in [1e47, 1e50] at random cells, smooth
    random E^n; dt = 1e-3 light-crossing times of the box."""
    rng = rng_for(2, seed_problem)
    shape = (n, n, n)
    dx = DX_TEST1
    L = n * dx
    nH = lognormal(shape, 1e-3, sigma_ln, rng)
    kappa = SIGMA_HI * nH
    del nH
    cells, ndot = point_sources(shape, n_src, 1e47, 1e50, rng)
    eta = emissivity(shape, cells, ndot, dx ** 3)
    dt = 1e-3 * L / C_LIGHT
    E = smooth_radiation(shape, eta, dt, rng)
    return _problem(shape, dx, kappa, eta, E, L, dt, f"many_sources_{n}")


def stromgren_radius(ndot, n_h, alpha_b=ALPHA_B):
    """r_s = (3 Ndot / (4 pi alpha_B n_H^2))^(1/3)  (Sec. 4.1.1)."""
    return (3.0 * np.asarray(ndot) / (4.0 * math.pi * alpha_b * n_h * n_h)) ** (1.0 / 3.0)


def reionization_share(n: int = 640, n_src: int = 10000, sigma_ln: float = 2.0,
                       seed_problem: int = 0, L_cells: int = 3200):
    """Workload 3: one 640^3 share of a 3200^3 reionization box at z = 8
    (proper dx = 2.78 kpc), lognormal HI (mean 1.43e-4 cm^-3, sigma_ln 2.0),
    n_src sources with Ndot log-uniform in [1e46, 1e49], ionized bubbles of
    the Stromgren radius of each source (x_HI = 1e-4 inside), E^n = 1e-45,
    L_unit = 3200 dx, dt = 1e-3 L_unit / c."""
    rng = rng_for(3, seed_problem)
    shape = (n, n, n)
    dx = 25.0 * KPC / 9.0
    nbar = 1.43e-4
    nH = lognormal(shape, nbar, sigma_ln, rng)
    cells, ndot = point_sources(shape, n_src, 1e46, 1e49, rng)
    # carve bubbles: x_HI = 1e-4 within r_s of each source (periodic)
    rs_cells = stromgren_radius(ndot, nbar) / dx
    xhi = np.ones(shape, dtype=np.float64)
    cz, rem = np.divmod(cells, n * n)
    cy, cx = np.divmod(rem, n)
    for x0, y0, z0, r in zip(cx, cy, cz, rs_cells):
        ri = int(math.ceil(r))
        if ri < 1:
            continue
        o = np.arange(-ri, ri + 1)
        d2 = (o[:, None, None] ** 2 + o[None, :, None] ** 2
              + o[None, None, :] ** 2)
        mask = d2 <= r * r
        iz = (z0 + o) % n
        iy = (y0 + o) % n
        ix = (x0 + o) % n
        sub = xhi[np.ix_(iz, iy, ix)]
        sub[mask] = 1e-4
        xhi[np.ix_(iz, iy, ix)] = sub
    kappa = SIGMA_HI * nH * xhi
    del nH, xhi
    eta = emissivity(shape, cells, ndot, dx ** 3)
    L = L_cells * dx
    dt = 1e-3 * L / C_LIGHT
    E = np.full(shape, 1e-45)
    return _problem(shape, dx, kappa, eta, E, L, dt, f"reionization_{n}")


def hii_test1(n_oct: int = 16, t_end_myr: float = 500.0, n_out: int = 50):
    """Test 1 (Sec. 4.1.1): a 5e48 photon/s source in static uniform hydrogen
    (n_H = 1e-3 cm^-3, T = 1e4 K), E = 1e-45 erg cm^-3 and x = n_HII/n_H =
    0.0012 at t = 0, over [0, t_end] with n_out evenly spaced outputs.

    The paper runs the octant [0, 6.6 kpc]^3 on n_oct^3 cells with the
    source at the origin and reflecting faces there.  The periodic solver
    runs the mirror image: (2 n_oct)^3 cells of the same width on a 13.2 kpc
    box, the source split evenly over the 8 cells that meet at the centre.
    The I-front stays inside 6.6 kpc of the source (r_s = 5.39 kpc), so the
    periodic images do not interact.  L_unit is the octant side (6.6 kpc).
    The relative-change floor of the step estimator is 1e-3 of the
    optically thin energy density at the Stromgren radius,
    Ndot h nu / (4 pi r_s^2 c)."""
    n = 2 * n_oct
    shape = (n, n, n)
    L = 6.6 * KPC
    dx = L / n_oct
    ndot, n_h, x0 = 5e48, 1e-3, 0.0012
    c0 = n_oct
    cells = [((c0 - 1 + k) * n + (c0 - 1 + j)) * n + (c0 - 1 + i)
             for k in (0, 1) for j in (0, 1) for i in (0, 1)]
    eta = emissivity(shape, cells, [ndot / 8.0] * 8, dx ** 3)
    rs = float(stromgren_radius(ndot, n_h))
    t_end = t_end_myr * MYR
    return {
        "name": f"hii_test1_{n_oct}", "shape": shape, "h": (dx, dx, dx),
        "E": np.full(shape, 1e-45), "x": np.full(shape, x0),
        "n_h": np.full(shape, n_h), "eta": eta, "L_unit": L, "ndot": ndot,
        "n_h_mean": n_h, "r_s": rs, "t_rec": 1.0 / (ALPHA_B * n_h),
        "dt0": 1e-3 * L / C_LIGHT,
        "e_floor": 1e-3 * ndot * HNU_HI / (4.0 * math.pi * rs * rs * C_LIGHT),
        "outputs": [t_end * (k + 1) / n_out for k in range(n_out)],
        "sigma": SIGMA_HI, "hnu": HNU_HI, "alpha_b": ALPHA_B,
        "cell_volume": dx ** 3,
    }


BATCH_SIZES = (32, 48, 64, 96, 128)


def batch_problem(i: int, sizes=BATCH_SIZES, max_src: int = 32,
                  workload: int = 4):
    """Problem i of the batched workload: n uniform over ``sizes``, sigma_ln
    uniform in [0.5, 2], 1..max_src sources, smooth random E^n."""
    rng = rng_for(workload, i)
    n = int(rng.choice(sizes))
    sigma_ln = float(rng.uniform(0.5, 2.0))
    n_src = int(rng.integers(1, max_src + 1))
    shape = (n, n, n)
    dx = DX_TEST1
    L = n * dx
    kappa = SIGMA_HI * lognormal(shape, 1e-3, sigma_ln, rng)
    cells, ndot = point_sources(shape, n_src, 1e47, 1e50, rng)
    eta = emissivity(shape, cells, ndot, dx ** 3)
    dt = 1e-3 * L / C_LIGHT
    E = smooth_radiation(shape, eta, dt, rng)
    return _problem(shape, dx, kappa, eta, E, L, dt, f"batch_{i}_{n}")


def serve_request_shape(i: int, lo: int = 64, hi: int = 384, multiple: int = 16):
    """Grid size, step count and source count of request i of the served
    stream: n log-uniform in [lo, hi] rounded to a multiple of 16, 1-5 steps,
    1-1000 sources."""
    rng = rng_for(5, i)
    n = int(round(math.exp(rng.uniform(math.log(lo), math.log(hi))) / multiple)) * multiple
    n = max(lo, min(hi, n))
    steps = int(rng.integers(1, 6))
    n_src = int(rng.integers(1, 1001))
    sigma_ln = float(rng.uniform(0.5, 2.0))
    return n, steps, n_src, sigma_ln


def serve_request(i: int, lo: int = 64, hi: int = 384, n_override=None):
    n, steps, n_src, sigma_ln = serve_request_shape(i, lo, hi)
    if n_override is not None:
        n = n_override
    rng = rng_for(5, 100000 + i)
    shape = (n, n, n)
    dx = DX_TEST1
    L = n * dx
    kappa = SIGMA_HI * lognormal(shape, 1e-3, sigma_ln, rng)
    cells, ndot = point_sources(shape, n_src, 1e47, 1e50, rng)
    eta = emissivity(shape, cells, ndot, dx ** 3)
    dt = 1e-3 * L / C_LIGHT
    E = smooth_radiation(shape, eta, dt, rng)
    p = _problem(shape, dx, kappa, eta, E, L, dt, f"request_{i}_{n}")
    p["steps"] = steps
    return p


def random_problem(shape, seed: int, sigma_ln: float = 1.0, n_src: int = 4,
                   E_mode: str = "smooth", dx=DX_TEST1, dt_factor=1e-3,
                   L_unit=None, theta=1.0, iid=False):
    """General small test problem on an arbitrary (nz, ny, nx) shape.
    ``dt_factor`` scales dt in light-crossing times of L_unit (default: the
    largest box side); ``iid`` draws an unsmoothed per-cell lognormal."""
    rng = rng_for(10, seed)
    shape = tuple(int(s) for s in shape)
    L = (L_unit if L_unit is not None else max(shape) * dx)
    nH = (np.exp(math.log(1e-3) + sigma_ln * rng.standard_normal(shape)) if iid
          else lognormal(shape, 1e-3, sigma_ln, rng))
    kappa = SIGMA_HI * nH
    cells, ndot = point_sources(shape, n_src, 1e47, 1e50, rng)
    eta = emissivity(shape, cells, ndot, dx ** 3)
    dt = dt_factor * L / C_LIGHT
    if E_mode == "zero":
        E = np.zeros(shape)
    elif E_mode == "smooth":
        E = smooth_radiation(shape, eta, dt, rng, sigma_cells=2.0)
    else:
        raise ValueError(E_mode)
    return _problem(shape, dx, kappa, eta, E, L, dt, f"random_{shape}_{seed}",
                    theta=theta)


# ---------------------------------------------------------------------------
# Device-side generators for large workloads (same recipe, drawn with torch's
# seeded generator on the GPU so 640^3 fields and hundreds of requests can be
# made in seconds).  They return torch float64 tensors on `device`.
# ---------------------------------------------------------------------------

def t_smooth_gaussian(shape, sigma_cells, gen, device):
    import torch
    g = torch.randn(shape, generator=gen, device=device, dtype=torch.float64)
    if sigma_cells > 0:
        G = torch.fft.rfftn(g)
        kz = torch.fft.fftfreq(shape[0], device=device, dtype=torch.float64)[:, None, None]
        ky = torch.fft.fftfreq(shape[1], device=device, dtype=torch.float64)[None, :, None]
        kx = torch.fft.rfftfreq(shape[2], device=device, dtype=torch.float64)[None, None, :]
        k2 = (2 * math.pi) ** 2 * (kx * kx + ky * ky + kz * kz)
        G *= torch.exp(-0.5 * sigma_cells ** 2 * k2)
        del k2
        g = torch.fft.irfftn(G, s=shape)
        del G
    g -= g.mean()
    sd = g.std()
    if sd > 0:
        g /= sd
    return g


def t_generator(workload, problem, device):
    import torch
    seed = int(np.random.SeedSequence([BASE_SEED + workload, problem]).generate_state(1)[0])
    gen = torch.Generator(device=device)
    gen.manual_seed(seed)
    return gen


def t_emissivity(shape, cells, ndot, cell_volume, device):
    import torch
    eta = torch.zeros(int(np.prod(shape)), dtype=torch.float64, device=device)
    eta.index_add_(0, torch.as_tensor(np.asarray(cells, dtype=np.int64), device=device),
                   torch.as_tensor(np.asarray(ndot) * HNU_HI / cell_volume,
                                   dtype=torch.float64, device=device))
    return eta.reshape(shape)


def t_problem(shape, sigma_ln, n_src, lum, workload, problem, device, dx=DX_TEST1,
              mean_density=1e-3, E_mode="smooth", L_cells=None):
    """One problem of the lognormal / point-source recipe on the device:
    kappa = sigma_HI n_HI, n_HI lognormal (1.5-cell smoothing), n_src sources
    with Ndot log-uniform in lum at random cells, E^n smooth (8-cell) around
    mean(eta) dt, dt = 1e-3 light-crossing times of L_unit."""
    import torch
    gen = t_generator(workload, problem, device)
    rng = rng_for(workload, 200000 + problem)
    shape = tuple(int(s) for s in shape)
    g = t_smooth_gaussian(shape, 1.5, gen, device)
    kappa = SIGMA_HI * torch.exp(math.log(mean_density) + sigma_ln * g)
    del g
    cells, ndot = point_sources(shape, n_src, lum[0], lum[1], rng)
    eta = t_emissivity(shape, cells, ndot, dx ** 3, device)
    L = (L_cells if L_cells is not None else max(shape)) * dx
    dt = 1e-3 * L / C_LIGHT
    if E_mode == "smooth":
        E = float(eta.mean()) * dt * torch.exp(t_smooth_gaussian(shape, 8.0, gen, device))
    else:
        E = torch.full(shape, float(E_mode), dtype=torch.float64, device=device)
    return {"name": f"t_{workload}_{problem}_{shape[0]}", "shape": shape,
            "h": (dx, dx, dx), "E": E, "kappa": kappa, "eta": eta,
            "c": C_LIGHT, "L_unit": L, "dt": dt, "theta": 1.0, "a": 1.0,
            "adot": 0.0, "cells": cells, "ndot": ndot}


def t_reionization_share(n=640, n_src=10000, sigma_ln=2.0, device="cuda",
                         L_cells=3200):
    """Workload 3 on the device (see reionization_share)."""
    import torch
    shape = (n, n, n)
    dx = 25.0 * KPC / 9.0
    nbar = 1.43e-4
    gen = t_generator(3, 0, device)
    rng = rng_for(3, 0)
    g = t_smooth_gaussian(shape, 1.5, gen, device)
    nH = torch.exp(math.log(nbar) + sigma_ln * g)
    del g
    cells, ndot = point_sources(shape, n_src, 1e46, 1e49, rng)
    rs = stromgren_radius(ndot, nbar) / dx
    cz, rem = np.divmod(cells, n * n)
    cy, cx = np.divmod(rem, n)
    # the cells within r of each source (periodic), listed on the host and
    # marked on the device in one scatter
    idx = []
    for x0, y0, z0, r in zip(cx, cy, cz, rs):
        ri = int(math.ceil(r))
        if ri < 1:
            continue
        o = np.arange(-ri, ri + 1)
        d2 = o[:, None, None] ** 2 + o[None, :, None] ** 2 + o[None, None, :] ** 2
        kz, ky, kx = np.nonzero(d2 <= r * r)
        idx.append((((int(z0) + o[kz]) % n) * n + (int(y0) + o[ky]) % n) * n
                   + (int(x0) + o[kx]) % n)
    ionized = torch.zeros(n * n * n, dtype=torch.bool, device=device)
    if idx:
        ionized[torch.as_tensor(np.concatenate(idx), device=device)] = True
    ionized = ionized.reshape(shape)
    # x_HI = 1e-4 inside the bubbles
    kappa = SIGMA_HI * nH * torch.where(ionized, 1e-4, 1.0)
    ion_frac = float(ionized.double().mean())
    del nH, ionized
    eta = t_emissivity(shape, cells, ndot, dx ** 3, device)
    L = L_cells * dx
    dt = 1e-3 * L / C_LIGHT
    E = torch.full(shape, 1e-45, dtype=torch.float64, device=device)
    return {"name": f"reionization_{n}", "shape": shape, "h": (dx, dx, dx),
            "E": E, "kappa": kappa, "eta": eta, "c": C_LIGHT, "L_unit": L,
            "dt": dt, "theta": 1.0, "a": 1.0, "adot": 0.0,
            "ionized_fraction": ion_frac}


def group_structure(G: int, e_lo_ev: float = 13.6, e_hi_ev: float = 13.6 * 8.0,
                    T_source: float = 1e5):
    """G frequency groups log-spaced in photon energy over [e_lo, e_hi] eV:
    (mean photon energy per group [erg], HI cross-section per group [cm^2],
    fraction of a T_source blackbody's ionizing photons in each group).
    The cross-section follows the hydrogenic nu^-3 fall-off from 6.3e-18 cm^2
    at the threshold; photons above e_hi are dropped."""
    kT = 8.617333262e-5 * T_source  # eV
    edges = np.geomspace(e_lo_ev, e_hi_ev, G + 1)
    e_mid = np.sqrt(edges[:-1] * edges[1:])
    fine = np.geomspace(e_lo_ev, 40.0 * e_hi_ev, 20001)
    planck = fine ** 2 / np.expm1(fine / kT)  # photon number per unit energy
    total = np.trapezoid(planck, fine)
    frac = np.empty(G)
    for g in range(G):
        m = (fine >= edges[g]) & (fine <= edges[g + 1])
        frac[g] = np.trapezoid(planck[m], fine[m]) / total
    sigma = SIGMA_HI * (e_mid / e_lo_ev) ** -3
    return e_mid * EV, sigma, frac


def t_multigroup(n: int, G: int, n_src: int = 64, sigma_ln: float = 1.5,
                 device="cuda", problem: int = 0):
    """Multigroup stand-in: one lognormal HI field (mean 1e-3 cm^-3) on n^3
    cells of 206 pc, n_src sources with Ndot log-uniform in [1e47, 1e50] and a
    1e5 K blackbody spectrum split over G groups; per group
    kappa_g = sigma_g n_HI, eta_g = sum Ndot f_g h nu_g / V_cell and a smooth
    E_g^n; dt = 1e-3 light-crossing times.  Fields are (G, n, n, n)."""
    import torch
    shape = (n, n, n)
    gen = t_generator(6, problem, device)
    rng = rng_for(6, 100000 + problem)
    dx = DX_TEST1
    g = t_smooth_gaussian(shape, 1.5, gen, device)
    nH = torch.exp(math.log(1e-3) + sigma_ln * g)
    del g
    hnu, sig, frac = group_structure(G)
    cells, ndot = point_sources(shape, n_src, 1e47, 1e50, rng)
    L = n * dx
    dt = 1e-3 * L / C_LIGHT
    kappa = torch.empty((G,) + shape, dtype=torch.float64, device=device)
    eta = torch.empty_like(kappa)
    E = torch.empty_like(kappa)
    for k in range(G):
        kappa[k] = sig[k] * nH
        e1 = t_emissivity(shape, cells, ndot * frac[k], dx ** 3, device)
        eta[k] = e1 * (hnu[k] / HNU_HI)
        E[k] = float(eta[k].mean()) * dt * torch.exp(
            t_smooth_gaussian(shape, 8.0, gen, device))
    return {"name": f"multigroup_{n}_G{G}", "shape": shape, "groups": G,
            "h": (dx, dx, dx), "E": E, "kappa": kappa, "eta": eta,
            "c": C_LIGHT, "L_unit": L, "dt": dt, "theta": 1.0, "a": 1.0,
            "adot": 0.0, "hnu": hnu, "sigma": sig, "frac": frac}


GYR = 1e3 * MYR


def cosmo_test2(n_oct: int = 16, ndot: float = 5e46, z_end: float = 0.0,
                n_out: int = 50, z0: float = 4.0):
    """Test 2 (Sec. 4.1.2): a point source in uniform hydrogen in an
    Einstein-de Sitter universe (Omega_m = 1, q0 = 1/2, H0 = 50 km/s/Mpc,
    Omega_b = 0.2), from z0 = 4 to z_end; proper density 1.175e-28 g cm^-3 at
    z0 (pure hydrogen), T = 1e4 K, E = 1e-45 erg cm^-3, x = 0.0012 (as in
    Test 1).  The comoving domain [0, 80 kpc]^3 (comoving lengths in units of
    the present, a = 1/(1+z)) is run as its periodic mirror image: (2 n_oct)^3
    cells with the source split over the 8 central cells.  Fields are
    comoving (proper x a^3); outputs are evenly spaced in cosmic time."""
    n = 2 * n_oct
    shape = (n, n, n)
    L = 80.0 * KPC
    dx = L / n_oct
    H0 = 50.0 * 1e5 / (1e3 * KPC)          # s^-1
    t_of_z = lambda z: (2.0 / (3.0 * H0)) * (1.0 + z) ** -1.5
    a0 = 1.0 / (1.0 + z0)
    m_h = 1.6726e-24
    n_h0 = 1.175e-28 / m_h                  # proper, at z0
    n_h_com = n_h0 * a0 ** 3
    c0 = n_oct
    cells = [((c0 - 1 + k) * n + (c0 - 1 + j)) * n + (c0 - 1 + i)
             for k in (0, 1) for j in (0, 1) for i in (0, 1)]
    eta = emissivity(shape, cells, [ndot / 8.0] * 8, dx ** 3)  # comoving
    t0, t1 = t_of_z(z0), t_of_z(z_end)
    rs0 = float(stromgren_radius(ndot, n_h0))                   # proper, z0
    e_floor = 1e-3 * ndot * HNU_HI / (4.0 * math.pi * rs0 * rs0 * C_LIGHT) * a0 ** 3
    return {
        "name": f"cosmo_test2_{n_oct}", "shape": shape, "h": (dx, dx, dx),
        "E": np.full(shape, 1e-45), "x": np.full(shape, 0.0012),
        "n_h": np.full(shape, n_h_com), "eta": eta, "L_unit": L, "ndot": ndot,
        "z0": z0, "H0": H0, "t0": t0, "t1": t1, "n_h0": n_h0, "r_s0": rs0,
        "lambda": ALPHA_B * n_h0 / H0 / (1.0 + z0), "q0": 0.5,
        "dt0": 1e-3 * a0 * L / C_LIGHT, "e_floor": e_floor,
        "outputs": [t0 + (t1 - t0) * (k + 1) / n_out for k in range(n_out)],
        "sigma": SIGMA_HI, "hnu": HNU_HI, "alpha_b": ALPHA_B,
        "cell_volume": dx ** 3,
    }



def thin_uniform_problem(n: int, nu: float, seed: int = 0, kappa_scale: float = 1e-12):
    """An optically thin periodic n^3 box (the lognormal HI opacity scaled by
    kappa_scale) with a smooth positive emissivity (a smoothed lognormal of
    sigma 0.5 around 1e-25 erg cm^-3 s^-1) and a uniform E^n = 1e-20, over a
    step long enough that the diffusion number dt D_max / dx^2 is nu
    (D_max = 0.006 c L_unit with L_unit the box side)."""
    rng = rng_for(11, seed)
    shape = (int(n),) * 3
    dx = DX_TEST1
    L = n * dx
    kappa = kappa_scale * SIGMA_HI * lognormal(shape, 1e-3, 1.0, rng)
    eta = 1e-25 * np.exp(0.5 * smooth_gaussian(shape, 3.0, rng))
    dt = nu * dx * dx / (0.006 * C_LIGHT * L)
    E = np.full(shape, 1e-20)
    return _problem(shape, dx, kappa, eta, E, L, dt, f"thin_{n}_{nu:g}_{seed}")
