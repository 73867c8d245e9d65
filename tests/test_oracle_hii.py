"""Pins of the oracle's isothermal hydrogen chemistry and of its
operator-split radiation + chemistry driver (Test 1, Sec. 4.1.1).

The chemistry update (Sec. 3.3, the loosely coupled solver) is fixed by three
closed forms that do not come from the oracle: pure recombination, where the
linearly implicit step happens to be exact; pure photo-ionization, whose
discrete solution is a geometric sequence tending to an exponential; and the
photo-ionization equilibrium, a root of a quadratic that every step size must
leave unchanged.  The driver is pinned by the Stromgren-sphere growth law
r(t) = r_s (1 - exp(-t / t_rec))^(1/3) of Test 1.
"""
import math

import numpy as np
import pytest

import synth
from conftest import read_golden

C = synth.C_LIGHT
SIGMA, HNU = synth.SIGMA_HI, synth.HNU_HI


def _fields(n, seed):
    rng = np.random.default_rng(seed)
    shape = (n,)
    x0 = rng.uniform(1e-4, 1.0, shape)
    n_h = np.exp(rng.normal(math.log(1e-3), 1.0, shape))
    return rng, x0, n_h


def _gamma(E):
    return C * SIGMA * E / HNU


@pytest.mark.parametrize("a", [1.0, 0.2])
@pytest.mark.parametrize("substeps", [1, 3, 7])
def test_chem_pure_recombination_is_exact(oracle_mod, substeps, a):
    # E = 0: dx/dt = -alpha n x^2 has x(t) = x0 / (1 + alpha n x0 t), and
    # 1/x grows linearly, which the linearly implicit step reproduces exactly;
    # n is the proper density, the comoving n_h over a^3
    alpha = 2.59e-13
    _, x0, n_h = _fields(4096, 1)
    n_p = n_h / a ** 3
    E = np.zeros_like(x0)
    x = x0.copy()
    t = 0.0
    for dt in (1e12, 3e13, 2e15):
        x, kappa = oracle_mod.chem_h(E, n_h, x, dt, C, SIGMA, HNU, alpha,
                                     substeps, a)
        t += dt
        exact = x0 / (1.0 + alpha * n_p * x0 * t)
        np.testing.assert_allclose(x, exact, rtol=1e-13)
        np.testing.assert_allclose(kappa, SIGMA * n_p * (1.0 - exact),
                                   rtol=1e-12)


def test_chem_pure_photoionization(oracle_mod):
    # alpha = 0: dx/dt = Gamma (1 - x).  Backward Euler over m equal pieces
    # gives 1 - x = (1 - x0) / (1 + h Gamma)^m, which tends to
    # (1 - x0) exp(-Gamma t) as m grows.
    rng, x0, n_h = _fields(2048, 2)
    E = np.exp(rng.uniform(math.log(1e-20), math.log(1e-16), x0.shape))
    g = _gamma(E)
    # comoving E = a^3 x the proper E that sets the rate (a = 0.5)
    x, _ = oracle_mod.chem_h(0.125 * E, n_h, x0, 5e10, C, SIGMA, HNU, 0.0, 4, 0.5)
    exact = 1.0 - (1.0 - x0) / (1.0 + (5e10 / 4) * g) ** 4
    np.testing.assert_allclose(1.0 - x, 1.0 - exact, rtol=1e-10)
    for dt, m in ((1e9, 1), (5e10, 4), (3e11, 9)):
        x, _ = oracle_mod.chem_h(E, n_h, x0, dt, C, SIGMA, HNU, 0.0, m)
        exact = 1.0 - (1.0 - x0) / (1.0 + (dt / m) * g) ** m
        # 1 - x near x = 1 magnifies the rounding of x
        np.testing.assert_allclose(1.0 - x, 1.0 - exact, rtol=1e-10)
    # the continuous limit, with Gamma t up to 5
    dt = 5.0 / g.max()
    x, _ = oracle_mod.chem_h(E, n_h, x0, dt, C, SIGMA, HNU, 0.0, 20000)
    limit = (1.0 - x0) * np.exp(-g * dt)
    np.testing.assert_allclose(1.0 - x, limit, rtol=2e-3)


def test_chem_equilibrium_is_a_fixed_point(oracle_mod):
    # Gamma (1 - x) = alpha n x^2  <=>  alpha n x^2 + Gamma x - Gamma = 0
    alpha = 2.59e-13
    rng, _, n_h = _fields(64, 3)
    E = np.exp(rng.uniform(math.log(1e-24), math.log(1e-16), n_h.shape))
    g = _gamma(E)
    xs = np.empty_like(g)
    for p in range(g.size):
        roots = np.roots([alpha * n_h[p], g[p], -g[p]])
        xs[p] = max(r.real for r in roots)
    assert np.all((xs > 0) & (xs < 1))
    for dt in (1e8, 1e13, 1e18):
        x, _ = oracle_mod.chem_h(E, n_h, xs, dt, C, SIGMA, HNU, alpha, 1)
        np.testing.assert_allclose(x, xs, rtol=1e-12)
    # large steps from the neutral state settle on the same root
    x = np.full_like(g, 0.0012)
    for _ in range(5000):  # contraction factor 1 - x*, slow for small x*
        x, _ = oracle_mod.chem_h(E, n_h, x, 1e20, C, SIGMA, HNU, alpha, 1)
    np.testing.assert_allclose(x, xs, rtol=1e-10)


def test_chem_bounds(oracle_mod):
    rng, x0, n_h = _fields(8192, 4)
    x0[:16] = 0.0
    x0[16:32] = 1.0
    E = np.exp(rng.uniform(math.log(1e-45), math.log(1e-8), x0.shape))
    for dt in (1e3, 1e12, 1e20):
        x, kappa = oracle_mod.chem_h(E, n_h, x0, dt, C, SIGMA, HNU, 2.59e-13, 2)
        assert np.all((x >= 0.0) & (x <= 1.0))
        assert np.all(kappa >= 0.0)


def test_stromgren_sphere_growth(oracle_mod):
    """Test 1 on the 16^3 octant (32^3 mirrored), tau_tol = 1e-2, over the
    first 20 Myr: the ionized radius follows r_s (1 - exp(-t/t_rec))^(1/3).
    The paper's own error curves survive only as figures; the gate is the
    error norm eq. "i1_error" <= 0.02 of r_s."""
    g = read_golden("test1_parameters.txt")
    ndot = float(g["ndot_photons_per_s"])
    n_h = float(g["n_h_cm3"])
    alpha = float(g["alpha_b_cm3_s"])
    r_s = (3.0 * ndot / (4.0 * math.pi * alpha * n_h * n_h)) ** (1.0 / 3.0)
    t_rec = 1.0 / (alpha * n_h)
    assert r_s / synth.KPC == pytest.approx(5.39, abs=0.01)
    assert t_rec / synth.MYR == pytest.approx(122.3, abs=0.1)

    d = synth.hii_test1(16, t_end_myr=20.0, n_out=10)
    d_max, r_min = oracle_mod.limits(C, d["L_unit"])
    run = oracle_mod.hii_run(d["E"], d["x"], d["n_h"], d["eta"], d["h"], C,
                             d_max, r_min, SIGMA, HNU, alpha, d["outputs"],
                             d["dt0"], 1e-2, d["e_floor"])
    assert len(run["radii"]) == 10
    t = np.array(run["times"])
    r = np.array(run["radii"])
    r_true = r_s * (1.0 - np.exp(-t / t_rec)) ** (1.0 / 3.0)
    err = math.sqrt(np.mean(((r - r_true) / r_s) ** 2))
    assert err <= 0.02, (err, r / synth.KPC, r_true / synth.KPC)
    assert np.all(np.diff(r) > 0)
    assert np.all((run["x"] >= 0) & (run["x"] <= 1))
    # the mirrored source keeps the octant symmetry of the paper's setup
    x = run["x"]
    np.testing.assert_allclose(x, x[::-1, :, :], rtol=1e-6, atol=1e-12)
    np.testing.assert_allclose(x, np.transpose(x, (2, 1, 0)), rtol=1e-6,
                               atol=1e-12)


def _shapiro_giroux(t, H0, z0, lam, q0, r_s0):
    """Comoving I-front radius (present-day units) of eq. "radius_cosmo":
    r = r_s0 (lam e^-tau(a) int_1^a e^tau(b) (1 - 2q0 + 2q0 (1+z0)/b)^-1/2 db)^1/3
    with tau from eq. "tau" and F from eq. "Fa", a the expansion factor
    normalised to 1 at z0 (the paper's integrand prints (1 - z0); F's (1 + z0)
    is the consistent reading), and r_s0 the proper Stromgren radius at z0,
    which is comoving in units of z0; times (1 + z0) for present-day units."""
    from scipy.integrate import quad
    F = lambda a: ((2 - 4 * q0 - 2 * q0 / a * (1 + z0))
                   * (1 - 2 * q0 + 2 * q0 / a * (1 + z0)) ** 0.5)
    tau = lambda a: lam * (F(a) - F(1.0)) / (6 * q0 ** 2 * (1 + z0) ** 2)
    a_abs = (1.5 * H0 * t) ** (2.0 / 3.0)   # Einstein-de Sitter, a = 1 today
    an = a_abs * (1 + z0)
    integral = quad(lambda b: math.exp(tau(b))
                    * (1 - 2 * q0 + 2 * q0 / b * (1 + z0)) ** -0.5, 1.0, an)[0]
    y = lam * math.exp(-tau(an)) * integral
    return r_s0 * y ** (1.0 / 3.0) * (1 + z0)


@pytest.mark.parametrize("theta", [1.0, 0.5])
def test_cosmological_front(oracle_mod, theta):
    """Test 2 on the 8^3 octant (16^3 mirrored), tau_tol = 1e-2, z = 4 -> 2:
    the comoving ionized radius follows the Shapiro-Giroux solution with the
    error norm of eq. "i1_error" (relative to the comoving r_s at z0) <= 0.05
    for backward Euler and the trapezoidal rule."""
    g = read_golden("test2_parameters.txt")
    h = float(g["hubble_h"])
    H0 = 100.0 * h * 1e5 / (1e3 * synth.KPC)
    z0, q0 = float(g["z_start"]), float(g["q0"])
    n_h0 = float(g["rho_g_cm3"]) / 1.6726e-24
    alpha = float(g["alpha_b_cm3_s"])
    ndot = float(g["ndot_photons_per_s"])
    lam = alpha * n_h0 / H0 / (1 + z0)
    r_s0 = (3 * ndot / (4 * math.pi * alpha * n_h0 ** 2)) ** (1.0 / 3.0)
    # the printed density is the proper baryon density at z0 for h = 0.5,
    # Omega_b = 0.2: Omega_b rho_crit (1 + z0)^3
    rho_crit = 3 * H0 ** 2 / (8 * math.pi * 6.674e-8)
    assert float(g["rho_g_cm3"]) == pytest.approx(
        float(g["omega_b"]) * rho_crit * (1 + z0) ** 3, rel=2e-3)

    d = synth.cosmo_test2(8, ndot=ndot, z_end=2.0, n_out=10)
    assert d["H0"] == pytest.approx(H0, rel=1e-12)
    d_max, r_min = oracle_mod.limits(C, d["L_unit"])
    run = oracle_mod.hii_run(d["E"], d["x"], d["n_h"], d["eta"], d["h"], C,
                             d_max, r_min, SIGMA, HNU, alpha, d["outputs"],
                             d["dt0"], 1e-2, d["e_floor"], t0=d["t0"], H0=H0,
                             theta=theta)
    t = np.array(run["times"])
    r = np.array(run["radii"])
    r_true = np.array([_shapiro_giroux(tt, H0, z0, lam, q0, r_s0) for tt in t])
    err = math.sqrt(np.mean(((r - r_true) / (r_s0 * (1 + z0))) ** 2))
    assert err <= 0.05, (err, r / synth.KPC, r_true / synth.KPC)
    assert np.all(np.diff(r) > 0)
    # the front first approaches the Stromgren radius r_s(t) and then falls
    # behind it as expansion drives r_s outward (comoving r_s grows as a)
    a = (1.5 * H0 * t) ** (2.0 / 3.0)
    frac = r / (r_s0 * (1 + z0) * (1 + z0) * a)
    assert frac[1] > frac[0] and frac[-1] < frac[-2]
