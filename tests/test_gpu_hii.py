"""GPU parity of the isothermal hydrogen chemistry and of the operator-split
radiation + chemistry driver (Test 1, Sec. 4.1.1) against the FP64 oracle.

Gates: the chemistry kernel evaluates the same closed-form update as the
oracle, so its results agree to a few ulps (relative 1e-13).  The coupled run
replays the oracle's own step sizes, so the two differ only by the radiation
solves' tolerance: each GPU step is within rtol ||b|| of the exact step, and
over a run these differences stay below 1e-6 relative on E and x.  The
adaptive run is checked against the Stromgren growth law.
"""
import math

import numpy as np
import pytest

import synth
from gpu_util import dev, host, log_case, rel_l2

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def fld():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    import paper_1306_0645_amd as m
    return m


CHEM_SHAPES = [(1, 1, 1), (7, 11, 1299), (64, 64, 64), (3, 5, 333337)]


@pytest.mark.parametrize("shape,a", [(s, 1.0) for s in CHEM_SHAPES]
                         + [((6, 10, 14), 0.25)])
@pytest.mark.parametrize("substeps", [1, 4])
def test_chem_update_matches_oracle(fld, oracle_mod, shape, a, substeps):
    log_case("chem_update", shape=shape, substeps=substeps, a=a)
    rng = np.random.default_rng(7 + substeps)
    E = np.exp(rng.uniform(math.log(1e-45), math.log(1e-14), shape))
    n_h = np.exp(rng.normal(math.log(1e-3), 1.0, shape))
    x0 = rng.uniform(0.0, 1.0, shape)
    x0.flat[0] = 0.0
    if x0.size > 1:
        x0.flat[-1] = 1.0
    p = fld.fld_chem_default_params(substeps=substeps)
    grid = fld.make_grid(shape, (1.0, 1.0, 1.0))
    x, kappa = dev(x0), dev(np.zeros(shape))
    Ed, nd = dev(E), dev(n_h)
    xr = x0
    for dt in (0.0, 3e9, 2e12, 5e14):
        fld.fld_chem_h_update(grid, p, Ed, nd, x, kappa, dt, a)
        xr, kr = oracle_mod.chem_h(E, n_h, xr, dt, p.c, p.sigma, p.hnu,
                                   p.alpha_b, substeps, a)
        np.testing.assert_allclose(host(x), xr, rtol=1e-13, atol=1e-300)
        # kappa = sigma n_H (1 - x) carries the absolute rounding of 1 - x,
        # which is large relative to 1 - x where x is close to 1
        scale = p.sigma * n_h / a ** 3
        assert np.all(np.abs(host(kappa) - kr) <= 1e-13 * scale + 1e-13 * kr)
    s = fld.fld_chem_ionized_sum(grid, x)
    assert float(s.item()) == pytest.approx(float(np.sum(xr)), rel=1e-12)


def _test1_setup(fld, n_oct, t_end_myr, n_out, tau, prec, chem_substeps=1):
    d = synth.hii_test1(n_oct, t_end_myr=t_end_myr, n_out=n_out)
    prm = fld.fld_default_params(synth.C_LIGHT, d["L_unit"], precision=prec,
                                 tau_tol=tau, e_floor=d["e_floor"])
    chem = fld.fld_chem_default_params(substeps=chem_substeps)
    return d, prm, chem


@pytest.mark.parametrize("n_oct,t_end,n_out,chem_sub", [(16, 2.0, 4, 1),
                                                      (8, 20.0, 4, 3)])
@pytest.mark.parametrize("prec", [0, 1])
def test_hii_replay_matches_oracle(fld, oracle_mod, n_oct, t_end, n_out,
                                   chem_sub, prec):
    """Same step sizes on both sides (the oracle's adaptive sequence)."""
    from paper_1306_0645_amd.ionization import IsothermalHII
    log_case("hii_replay", n_oct=n_oct, t_end_myr=t_end, prec=prec,
             chem_substeps=chem_sub)
    d, prm, chem = _test1_setup(fld, n_oct, t_end, n_out, 1e-2, prec, chem_sub)
    ref = oracle_mod.hii_run(d["E"], d["x"], d["n_h"], d["eta"], d["h"],
                             synth.C_LIGHT, prm.d_max, prm.r_min, chem.sigma,
                             chem.hnu, chem.alpha_b, d["outputs"], d["dt0"],
                             1e-2, d["e_floor"], chem_substeps=chem_sub)
    drv = IsothermalHII(d["shape"], d["h"], prm, chem)
    E, x = dev(d["E"]), dev(d["x"])
    out = drv.run(E, x, dev(d["n_h"]), dev(d["eta"]), d["outputs"], d["dt0"],
                  dts=ref["dts"])
    drv.close()
    assert out["steps"] == len(ref["dts"])
    assert out["times"] == ref["times"]
    eE = rel_l2(host(E), ref["E"])
    ex = float(np.max(np.abs(host(x) - ref["x"])))
    er = max(abs(a - b) / b for a, b in zip(out["radii"], ref["radii"]))
    print(f"[hii_replay] steps={out['steps']} relL2(E)={eE:.2e} "
          f"max|dx|={ex:.2e} max rel dr={er:.2e}", flush=True)
    assert eE <= 1e-6
    assert ex <= 1e-6
    assert er <= 1e-7
    np.testing.assert_allclose(host(out["kappa"]), ref["kappa"], rtol=1e-5,
                               atol=1e-6 * float(np.max(ref["kappa"])))


@pytest.mark.parametrize("prec", [0, 1])
def test_hii_stromgren_growth(fld, prec):
    """Adaptive run on the 32^3 octant over the first 100 Myr: the error norm
    of eq. "i1_error" against r_s (1 - exp(-t/t_rec))^(1/3) stays <= 0.02."""
    from paper_1306_0645_amd.ionization import IsothermalHII
    log_case("hii_adaptive", n_oct=32, prec=prec)
    d, prm, chem = _test1_setup(fld, 32, 100.0, 20, 1e-2, prec)
    drv = IsothermalHII(d["shape"], d["h"], prm, chem)
    E, x = dev(d["E"]), dev(d["x"])
    out = drv.run(E, x, dev(d["n_h"]), dev(d["eta"]), d["outputs"], d["dt0"])
    drv.close()
    t = np.array(out["times"])
    r = np.array(out["radii"])
    r_true = d["r_s"] * (1.0 - np.exp(-t / d["t_rec"])) ** (1.0 / 3.0)
    err = math.sqrt(np.mean(((r - r_true) / d["r_s"]) ** 2))
    print(f"[hii_adaptive] prec={prec} steps={out['steps']} "
          f"iters={out['iters']} err={err:.4f} wall={out['wall_s']:.2f}s",
          flush=True)
    assert len(r) == 20
    assert err <= 0.02
    assert np.all(np.diff(r) > 0)
    xs = host(x)
    assert np.all((xs >= 0) & (xs <= 1))


# ---------------------------------------------------------------------------
# Test 2: comoving fields in an Einstein-de Sitter background (Sec. 4.1.2)
# ---------------------------------------------------------------------------

def _test2_setup(fld, n_oct, z_end, n_out, tau, prec, theta):
    d = synth.cosmo_test2(n_oct, z_end=z_end, n_out=n_out)
    prm = fld.fld_default_params(synth.C_LIGHT, d["L_unit"], precision=prec,
                                 tau_tol=tau, e_floor=d["e_floor"], theta=theta)
    chem = fld.fld_chem_default_params()
    return d, prm, chem


@pytest.mark.parametrize("theta", [1.0, 0.5])
@pytest.mark.parametrize("prec", [0, 1])
def test_cosmo_replay_matches_oracle(fld, oracle_mod, theta, prec):
    """Test 2 on the 8^3 octant, z = 4 -> 3, the oracle's step sizes
    replayed: same gates as Test 1."""
    from paper_1306_0645_amd.ionization import IsothermalHII, eds_expansion
    log_case("cosmo_replay", prec=prec, theta=theta)
    d, prm, chem = _test2_setup(fld, 8, 3.0, 4, 1e-2, prec, theta)
    ref = oracle_mod.hii_run(d["E"], d["x"], d["n_h"], d["eta"], d["h"],
                             synth.C_LIGHT, prm.d_max, prm.r_min, chem.sigma,
                             chem.hnu, chem.alpha_b, d["outputs"], d["dt0"],
                             1e-2, d["e_floor"], t0=d["t0"], H0=d["H0"],
                             theta=theta)
    drv = IsothermalHII(d["shape"], d["h"], prm, chem,
                        expansion=eds_expansion(d["H0"]))
    E, x = dev(d["E"]), dev(d["x"])
    out = drv.run(E, x, dev(d["n_h"]), dev(d["eta"]), d["outputs"], d["dt0"],
                  dts=ref["dts"], t0=d["t0"])
    drv.close()
    assert out["steps"] == len(ref["dts"])
    eE = rel_l2(host(E), ref["E"])
    ex = float(np.max(np.abs(host(x) - ref["x"])))
    er = max(abs(a - b) / b for a, b in zip(out["radii"], ref["radii"]))
    print(f"[cosmo_replay] steps={out['steps']} relL2(E)={eE:.2e} "
          f"max|dx|={ex:.2e} max rel dr={er:.2e}", flush=True)
    assert eE <= 1e-6
    assert ex <= 1e-6
    assert er <= 1e-7


@pytest.mark.parametrize("prec", [0, 1])
def test_cosmo_front_follows_shapiro_giroux(fld, prec):
    """Adaptive Test 2 on the 16^3 octant from z = 4 to 1: the comoving
    ionized radius against the Shapiro-Giroux solution, error norm <= 0.03."""
    from paper_1306_0645_amd.ionization import IsothermalHII, eds_expansion
    from test_oracle_hii import _shapiro_giroux
    log_case("cosmo_adaptive", n_oct=16, prec=prec)
    d, prm, chem = _test2_setup(fld, 16, 1.0, 20, 1e-2, prec, 1.0)
    drv = IsothermalHII(d["shape"], d["h"], prm, chem,
                        expansion=eds_expansion(d["H0"]))
    E, x = dev(d["E"]), dev(d["x"])
    out = drv.run(E, x, dev(d["n_h"]), dev(d["eta"]), d["outputs"], d["dt0"],
                  t0=d["t0"])
    drv.close()
    r = np.array(out["radii"])
    r_true = np.array([_shapiro_giroux(t, d["H0"], d["z0"], d["lambda"],
                                       d["q0"], d["r_s0"]) for t in out["times"]])
    err = math.sqrt(np.mean(((r - r_true) / (d["r_s0"] * (1 + d["z0"]))) ** 2))
    print(f"[cosmo_adaptive] prec={prec} steps={out['steps']} "
          f"iters={out['iters']} err={err:.4f} wall={out['wall_s']:.2f}s",
          flush=True)
    assert len(r) == 20
    assert err <= 0.03
