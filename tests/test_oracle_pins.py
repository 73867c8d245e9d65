"""Pins of the FP64 oracle against facts that do not come from the oracle.

Each test fixes a value by hand arithmetic, a closed form, an invariant of the
discrete operator, brute force or a LAPACK solve, so that a plausible mistake
in the oracle (a dropped term, a wrong sign, a wrong face index, dx and dy
swapped, the wrong mean) fails at least one of them.  Passages followed:
eq. "fld" (Sec. 3.3), the limiter and its face means (Sec. 2), the
theta-method with lagged D in residual-correction form (Sec. 3.3), the
cut-and-subcycle rule (Sec. 3.4).
"""
import math

import numpy as np
import pytest

from conftest import read_golden

C = 1.0  # unit light speed for the hand-value pins


# --------------------------------------------------------------------------
# Limiter and face means (Sec. 2), hand values
# --------------------------------------------------------------------------

def test_limiter_hand_values(oracle_mod):
    lim = oracle_mod.face_limiter
    big = 1e30
    # harmonic mean of kappa = (1, 3) is 2*1*3/4 = 1.5; flat E -> R = R_min
    assert lim(1.0, 1.0, 1.0, 3.0, 1.0, C, big, 1e-20) == pytest.approx(
        1.0 / 4.5, rel=1e-15)
    # E = (1, 3), dx = 1: Ebar = 2, R = |3-1|/(1*2) = 1; kbar = 1.5
    #   D = 1 / sqrt(9*2.25 + 1) = 1 / sqrt(21.25)
    assert lim(1.0, 3.0, 1.0, 3.0, 1.0, C, big, 1e-20) == pytest.approx(
        1.0 / math.sqrt(21.25), rel=1e-15)
    # same with dx = 0.5: R = 2 -> 1/sqrt(20.25 + 4)
    assert lim(1.0, 3.0, 1.0, 3.0, 0.5, C, big, 1e-20) == pytest.approx(
        1.0 / math.sqrt(24.25), rel=1e-15)
    # c scales D linearly
    assert lim(1.0, 3.0, 1.0, 3.0, 1.0, 7.0, big, 1e-20) == pytest.approx(
        7.0 / math.sqrt(21.25), rel=1e-15)
    # symmetric in the two cells
    assert lim(3.0, 1.0, 3.0, 1.0, 1.0, C, big, 1e-20) == lim(
        1.0, 3.0, 1.0, 3.0, 1.0, C, big, 1e-20)


def test_limiter_limits(oracle_mod):
    lim = oracle_mod.face_limiter
    # optically thick: kbar >> R -> D -> c / (3 kbar)
    assert lim(1.0, 1.0001, 2e6, 2e6, 1.0, C, 1e30, 1e-20) == pytest.approx(
        1.0 / 6e6, rel=1e-12)
    # kbar = 0 (either cell transparent) -> min(c/R, D_max)
    assert lim(1.0, 3.0, 0.0, 5.0, 1.0, C, 1e30, 1e-20) == pytest.approx(1.0)
    assert lim(1.0, 3.0, 0.0, 5.0, 1.0, C, 0.25, 1e-20) == 0.25
    # kappa = 0 on both sides (0/0 in the harmonic mean) -> kbar = 0
    assert lim(1.0, 3.0, 0.0, 0.0, 1.0, C, 1e30, 1e-20) == pytest.approx(1.0)
    # Ebar = 0 -> R = R_min; kbar = 0 -> c / R_min capped at D_max
    assert lim(0.0, 0.0, 0.0, 0.0, 1.0, C, 1e30, 1e-20) == pytest.approx(1e20)
    assert lim(0.0, 0.0, 0.0, 0.0, 1.0, C, 0.006, 1e-20) == 0.006
    # negative face mean (undershoot) also takes R_min
    assert lim(-1.0, -1.0, 1.0, 1.0, 1.0, C, 1e30, 0.5) == pytest.approx(
        1.0 / math.sqrt(9.0 + 0.25), rel=1e-15)
    # R below R_min is raised to R_min
    assert lim(1.0, 1.0, 0.0, 0.0, 1.0, C, 1e30, 0.5) == pytest.approx(2.0)


def test_paper_constants(oracle_mod):
    g = read_golden("limiter_constants.txt")
    L, c = 3.0e24, 2.99792458e10
    dmax, rmin = oracle_mod.limits(c, L)
    assert dmax == pytest.approx(float(g["dmax_factor"]) * c * L, rel=1e-15)
    assert rmin == pytest.approx(float(g["rmin_factor"]) / L, rel=1e-15)


def test_faces_use_the_right_neighbour(oracle_mod):
    """Brute force over every cell: the +d face of cell p pairs p with
    p + e_d (periodic), on a ragged anisotropic grid."""
    rng = np.random.default_rng(0)
    nz, ny, nx = 3, 4, 5
    E = rng.uniform(0.5, 2.0, (nz, ny, nx))
    kap = rng.uniform(0.1, 3.0, (nz, ny, nx))
    h = (0.7, 1.3, 2.1)
    Dx, Dy, Dz = oracle_mod.faces(E, kap, h, C, 1e30, 1e-20)
    lim = oracle_mod.face_limiter
    for k in range(nz):
        for j in range(ny):
            for i in range(nx):
                q = (k, j, (i + 1) % nx)
                assert Dx[k, j, i] == lim(E[k, j, i], E[q], kap[k, j, i],
                                          kap[q], h[0], C, 1e30, 1e-20)
                q = (k, (j + 1) % ny, i)
                assert Dy[k, j, i] == lim(E[k, j, i], E[q], kap[k, j, i],
                                          kap[q], h[1], C, 1e30, 1e-20)
                q = ((k + 1) % nz, j, i)
                assert Dz[k, j, i] == lim(E[k, j, i], E[q], kap[k, j, i],
                                          kap[q], h[2], C, 1e30, 1e-20)


# --------------------------------------------------------------------------
# Closed forms of one theta-step (Sec. 3.3)
# --------------------------------------------------------------------------

def _prob(oracle_mod, E, kap, eta, h, dt, theta=1.0, a=1.0, adot=0.0,
          d_max=1e30, r_min=1e-20, c=C):
    return oracle_mod.Problem(E, kap, eta, h, c, d_max, r_min, dt, theta, a,
                              adot)


@pytest.mark.parametrize("theta", [1.0, 0.5])
def test_no_diffusion_is_cellwise(oracle_mod, theta):
    """D_max = 0 makes A diagonal: dE_p = dt (eta_p - mu_p E_p) / (1 + theta
    dt mu_p), mu_p = adot/a + c kappa_p, for arbitrary lognormal kappa."""
    rng = np.random.default_rng(1)
    shape = (4, 6, 8)
    E = rng.uniform(0.0, 2.0, shape)
    kap = np.exp(rng.normal(0.0, 1.5, shape))
    eta = rng.uniform(0.0, 3.0, shape)
    dt, a, adot = 0.37, 1.3, 0.2
    P = _prob(oracle_mod, E, kap, eta, (1.0, 0.5, 2.0), dt, theta, a, adot,
              d_max=0.0)
    dE, st, it, rr = P.solve()
    assert st == oracle_mod.OK
    mu = adot / a + C * kap
    want = dt * (eta - mu * E) / (1.0 + theta * dt * mu)
    np.testing.assert_allclose(dE, want, rtol=1e-12, atol=0)


@pytest.mark.parametrize("theta", [1.0, 0.5])
def test_uniform_state(oracle_mod, theta):
    E0, k0, eta0, dt = 0.8, 2.5, 1.7, 0.11
    shape = (4, 4, 6)
    P = _prob(oracle_mod, np.full(shape, E0), np.full(shape, k0),
              np.full(shape, eta0), (1.0, 1.0, 1.0), dt, theta, c=3.0)
    dE, st, _, _ = P.solve()
    mu = 3.0 * k0
    np.testing.assert_allclose(dE, dt * (eta0 - mu * E0) / (1 + theta * dt * mu),
                               rtol=1e-13)


@pytest.mark.parametrize("theta", [1.0, 0.5])
def test_expansion_term(oracle_mod, theta):
    """kappa = 0, eta = 0, uniform E: only adot/a acts.
    E^{n+1} = E^n (1 - (1-theta) dt adot/a) / (1 + theta dt adot/a)."""
    shape = (4, 4, 4)
    E0, dt, a, adot = 2.0, 0.3, 0.5, 0.4
    P = _prob(oracle_mod, np.full(shape, E0), np.zeros(shape), np.zeros(shape),
              (1.0, 1.0, 1.0), dt, theta, a, adot)
    dE, st, _, _ = P.solve()
    h = adot / a
    np.testing.assert_allclose(
        E0 + dE, E0 * (1 - (1 - theta) * dt * h) / (1 + theta * dt * h),
        rtol=1e-13)


@pytest.mark.parametrize("a", [1.0, 0.4])
@pytest.mark.parametrize("theta", [1.0, 0.5])
def test_fourier_mode_decay(oracle_mod, theta, a):
    """Constant kappa, D pinned at D_max, E = E0 (1 + eps cos(k.x)) on a
    ragged anisotropic grid: A is circulant, so the mean and the mode evolve
    separately with growth factors (1 - (1-theta) dt mu)/(1 + theta dt mu),
    mu_k = adot/a + c kappa + D_max sum_d 4 sin^2(k_d h_d / 2) / h_d^2, where
    h_d = dx_d is the comoving cell size: every spatial derivative is with
    respect to the comoving position (Sec. 2), so a enters only as adot/a."""
    nz, ny, nx = 8, 12, 10
    hc = (0.9, 1.4, 0.6)
    h = hc  # comoving spacing
    m = (2, 1, 3)  # mode numbers along x, y, z
    k0, E0, eps, c = 0.05, 1.0, 0.1, 2.0
    adot, dt = 0.03 * a, 0.7
    x = np.arange(nx)[None, None, :]
    y = np.arange(ny)[None, :, None]
    z = np.arange(nz)[:, None, None]
    phase = 2 * np.pi * (m[0] * x / nx + m[1] * y / ny + m[2] * z / nz)
    mode = np.cos(phase)
    # R <= 2 eps / ((1 - eps) min dx); D_max well below c/sqrt(9k^2 + R^2)
    Rb = 2 * eps / ((1 - eps) * min(h))
    d_max = 0.5 * c / math.sqrt(9 * k0 ** 2 + Rb ** 2)
    kd = [2 * np.pi * m[0] / (nx * h[0]), 2 * np.pi * m[1] / (ny * h[1]),
          2 * np.pi * m[2] / (nz * h[2])]
    mu0 = adot / a + c * k0
    muk = mu0 + d_max * sum(4 * math.sin(kd[d] * h[d] / 2) ** 2 / h[d] ** 2
                            for d in range(3))
    g0 = (1 - (1 - theta) * dt * mu0) / (1 + theta * dt * mu0)
    gk = (1 - (1 - theta) * dt * muk) / (1 + theta * dt * muk)
    E = E0 * (1 + eps * mode)
    kap = np.full(E.shape, k0)
    zero = np.zeros(E.shape)
    mean, amp = E0, E0 * eps
    for n in range(5):
        P = _prob(oracle_mod, E, kap, zero, hc, dt, theta, a, adot, d_max=d_max,
                  c=c)
        Dx, Dy, Dz = oracle_mod.faces(E, kap, h, c, d_max, 1e-20)
        assert np.all(Dx == d_max) and np.all(Dy == d_max) and np.all(Dz == d_max)
        dE, st, _, _ = P.solve()
        assert st == oracle_mod.OK
        E = E + dE
        mean, amp = mean * g0, amp * gk
        np.testing.assert_allclose(E, mean + amp * mode, rtol=0, atol=1e-12)


@pytest.mark.parametrize("a", [1.0, 0.25])
def test_nyquist_mode_limiter_active(oracle_mod, a):
    """E = E0 (1 + eps (-1)^i) with D_max out of reach: every x face has
    Ebar = E0 and |dE| = 2 eps E0, so with the comoving spacing hx = dx
    (whatever a is), R = 2 eps / hx and D_x = c / sqrt(9 k0^2 + 4 eps^2 /
    hx^2).  The x-Nyquist mode then has mu_N = c k0 + 4 D_x / hx^2 and the
    mean mu_0 = c k0 (adot = 0)."""
    nz, ny, nx = 4, 6, 8
    h = (0.5, 1.0, 1.5)
    hx = h[0]
    k0, E0, eps, c, dt, theta = 0.4, 3.0, 0.2, 1.5, 0.25, 1.0
    s = (-1.0) ** np.arange(nx)[None, None, :] * np.ones((nz, ny, 1))
    E = E0 * (1 + eps * s)
    kap = np.full(E.shape, k0)
    P = _prob(oracle_mod, E, kap, np.zeros(E.shape), h, dt, theta, a, 0.0, c=c)
    dE, st, _, _ = P.solve()
    Dx = c / math.sqrt(9 * k0 ** 2 + 4 * eps ** 2 / hx ** 2)
    mu0 = c * k0
    muN = mu0 + 4 * Dx / hx ** 2
    want = (dt * (-mu0 * E0) / (1 + theta * dt * mu0)
            + dt * (-muN * E0 * eps) * s / (1 + theta * dt * muN))
    np.testing.assert_allclose(dE, want, rtol=1e-12)


def test_alternating_opacity_harmonic_face(oracle_mod):
    """Uniform E and kappa alternating kappa1/kappa2 along x: every x face
    has kbar = 2 k1 k2 / (k1 + k2) (harmonic, not arithmetic) and
    D_x = c / (3 kbar).  The step maps span{1, s = (-1)^i} into itself; dE =
    alpha + beta s solves a 2x2 system written out here by hand."""
    nz, ny, nx = 4, 4, 6
    h = (0.8, 1.0, 1.0)
    k1, k2, E0, c, dt, theta = 0.5, 4.0, 2.0, 1.0, 0.6, 1.0
    s = (-1.0) ** np.arange(nx)[None, None, :] * np.ones((nz, ny, 1))
    kap = np.where(s > 0, k1, k2)
    E = np.full(kap.shape, E0)
    P = _prob(oracle_mod, E, kap, np.zeros(E.shape), h, dt, theta, c=c)
    dE, st, _, _ = P.solve()
    kbar = 2 * k1 * k2 / (k1 + k2)
    Dx = c / (3 * kbar)
    ka, kd = (k1 + k2) / 2, (k1 - k2) / 2
    # L(alpha + beta s) = -4 Dx beta s / dx^2 - c (ka + kd s)(alpha + beta s)
    #   = [-c (ka alpha + kd beta)] + [-4 Dx beta / dx^2 - c (ka beta + kd alpha)] s
    # A u = u - theta dt L u ; b = dt L E (E = E0 const)
    w = 4 * Dx / h[0] ** 2
    tdt = theta * dt
    M = np.array([[1 + tdt * c * ka, tdt * c * kd],
                  [tdt * c * kd, 1 + tdt * (w + c * ka)]])
    rhs = np.array([-dt * c * ka * E0, -dt * c * kd * E0])
    alpha, beta = np.linalg.solve(M, rhs)
    np.testing.assert_allclose(dE, alpha + beta * s, rtol=1e-12)


def test_conservation_without_sinks(oracle_mod):
    """kappa = 0, eta = 0, adot = 0: the fluxes telescope, so
    sum(E^{n+1}) - sum(E^n) = sum(dE) = -sum(residual) which is bounded by
    sqrt(N) * tol * ||b||_2."""
    rng = np.random.default_rng(3)
    shape = (8, 6, 10)
    E = np.exp(rng.normal(0.0, 1.0, shape))
    zero = np.zeros(shape)
    P = _prob(oracle_mod, E, zero, zero, (1.0, 0.7, 1.3), 0.9, 1.0,
              d_max=0.8, r_min=1e-3)
    diag, Ax, Ay, Az, b = P.system()
    assert abs(b.sum()) <= 1e-13 * np.abs(b).sum()
    dE, st, _, rel = P.solve(tol=1e-13)
    bound = math.sqrt(E.size) * 1e-13 * np.linalg.norm(b)
    assert abs(dE.sum()) <= bound + 1e-14 * np.abs(dE).sum()
    assert np.linalg.norm(dE) > 1e-3 * np.linalg.norm(E)  # nontrivial step


# --------------------------------------------------------------------------
# Structure of A, brute force, LAPACK
# --------------------------------------------------------------------------

def _dense_by_columns(P):
    n = P.E.size
    M = np.empty((n, n))
    for j in range(n):
        e = np.zeros(n)
        e[j] = 1.0
        M[:, j] = P.apply_A(e.reshape(P.shape)).ravel()
    return M


@pytest.mark.parametrize("a", [1.0, 0.5])
def test_matrix_structure(oracle_mod, a):
    """Brute-force columns A e_j against the exported system, on a static and
    on a comoving mesh (a != 1: only adot/a carries it)."""
    rng = np.random.default_rng(4)
    shape = (4, 6, 8)
    E = np.exp(rng.normal(0.0, 1.0, shape))
    kap = np.exp(rng.normal(-1.0, 1.5, shape))
    h = (0.9, 1.1, 1.6)
    dt, theta, adot, c, d_max = 0.8, 1.0, 0.05 * a, 1.0, 0.4
    P = _prob(oracle_mod, E, kap, np.zeros(shape), h, dt, theta, a, adot,
              d_max=d_max, c=c)
    M = _dense_by_columns(P)
    np.testing.assert_allclose(M, M.T, rtol=0, atol=1e-15 * np.abs(M).max())
    diag, Ax, Ay, Az, b = P.system()
    np.testing.assert_allclose(np.diag(M), diag.ravel(), rtol=1e-14)
    nz, ny, nx = shape
    idx = np.arange(M.shape[0]).reshape(shape)
    xp = np.roll(idx, -1, axis=2)
    yp = np.roll(idx, -1, axis=1)
    zp = np.roll(idx, -1, axis=0)
    r = idx.ravel()
    np.testing.assert_allclose(-M[r, xp.ravel()], Ax.ravel(), rtol=1e-14)
    np.testing.assert_allclose(-M[r, yp.ravel()], Ay.ravel(), rtol=1e-14)
    np.testing.assert_allclose(-M[r, zp.ravel()], Az.ravel(), rtol=1e-14)
    # exactly 7 nonzeros per row (periodic, all extents >= 3)
    assert np.all((np.abs(M) > 0).sum(axis=1) == 7)
    lam = np.linalg.eigvalsh(0.5 * (M + M.T))
    assert lam.min() >= 1.0 - 1e-12  # adot >= 0 -> lambda_min(A) >= 1
    gersh = 1 + theta * dt * (c * kap.max() + adot / a
                              + 4 * d_max * sum(1 / hh ** 2 for hh in h))
    assert lam.max() <= gersh * (1 + 1e-12)


def test_dense_solve_8cubed(oracle_mod):
    """8^3 = 512 unknowns: the oracle's CG solution equals a LAPACK solve of
    the brute-force matrix, and b matches dt (L E + eta) built from columns."""
    import synth
    p = synth.random_problem((8, 8, 8), seed=5, sigma_ln=1.5, n_src=3,
                             dt_factor=2e-2)
    dmax, rmin = oracle_mod.limits(p["c"], p["L_unit"])
    P = oracle_mod.Problem(p["E"], p["kappa"], p["eta"], p["h"], p["c"], dmax,
                           rmin, p["dt"], p["theta"], p["a"], p["adot"])
    M = _dense_by_columns(P)
    diag, Ax, Ay, Az, b = P.system()
    # b = dt (L E + eta) and L u = (u - A u) / (theta dt)
    LE = (p["E"].ravel() - M @ p["E"].ravel()) / (p["theta"] * p["dt"])
    np.testing.assert_allclose(b.ravel(), p["dt"] * (LE + p["eta"].ravel()),
                               rtol=1e-9, atol=1e-12 * np.abs(b).max())
    x_lapack = np.linalg.solve(M, b.ravel())
    dE, st, it, rel = P.solve(tol=1e-13)
    assert st == oracle_mod.OK and rel <= 1e-13
    err = np.linalg.norm(dE.ravel() - x_lapack) / np.linalg.norm(x_lapack)
    assert err <= 1e-12
    # ||A^{-1}||_2 <= 1 -> error bounded by the residual
    r = b.ravel() - M @ dE.ravel()
    assert np.linalg.norm(dE.ravel() - x_lapack) <= np.linalg.norm(r) * (1 + 1e-6) + 1e-30


@pytest.mark.parametrize("a", [1.0, 0.3])
def test_residual_at_matches_assembled(oracle_mod, a):
    """The cell-by-cell residual used for spot checks on large grids agrees
    with b - A x from the assembled system (also on a comoving mesh)."""
    import synth
    p = synth.random_problem((6, 8, 10), seed=6, sigma_ln=1.0, n_src=2,
                             dt_factor=5e-2)
    dmax, rmin = oracle_mod.limits(p["c"], p["L_unit"])
    P = oracle_mod.Problem(p["E"], p["kappa"], p["eta"], p["h"], p["c"], dmax,
                           rmin, p["dt"], 1.0, a, 0.2 / p["dt"])
    rng = np.random.default_rng(7)
    x = rng.normal(size=p["E"].shape) * np.abs(p["E"]).max()
    diag, Ax, Ay, Az, b = P.system()
    full = b - P.apply_A(x)
    cells = np.arange(x.size)
    res, rhs = P.residual_at(x, cells)
    np.testing.assert_allclose(res, full.ravel(), rtol=1e-9,
                               atol=1e-12 * np.abs(full).max())
    np.testing.assert_allclose(rhs, b.ravel(), rtol=1e-12,
                               atol=1e-14 * np.abs(b).max())


# --------------------------------------------------------------------------
# Subcycling mechanism (Sec. 3.4); the dt estimator itself is unpinned
# --------------------------------------------------------------------------

def test_step_failure_leaves_E_untouched(oracle_mod):
    import synth
    p = synth.random_problem((8, 8, 8), seed=8, dt_factor=0.5)
    dmax, rmin = oracle_mod.limits(p["c"], p["L_unit"])
    E1, st, stats = oracle_mod.step(p["E"], p["kappa"], p["eta"], p["h"],
                                    p["c"], dmax, rmin, p["dt"], tol=1e-8,
                                    max_iter=1, max_cuts=0)
    assert st == oracle_mod.NOCONV
    assert np.array_equal(E1, p["E"])
    assert stats["cuts"] == 0


def test_step_cuts_and_subcycles(oracle_mod):
    """A step whose full-length solve fails is cut by 10x and subcycled to
    the requested time; the subcycled result equals successive single solves
    of the substep lengths, within the solve tolerance."""
    import synth
    p = synth.random_problem((8, 8, 8), seed=9, dt_factor=2.0, sigma_ln=0.5)
    dmax, rmin = oracle_mod.limits(p["c"], p["L_unit"])
    args = (p["kappa"], p["eta"], p["h"], p["c"], dmax, rmin)
    # max_iter small enough that the full step fails but 0.1 dt converges
    full = oracle_mod.Problem(p["E"], *args[:2], p["h"], p["c"], dmax, rmin,
                              p["dt"])
    _, st_full, it_full, _ = full.solve(tol=1e-6, max_iter=10 ** 6)
    small = oracle_mod.Problem(p["E"], *args[:2], p["h"], p["c"], dmax, rmin,
                               0.1 * p["dt"])
    _, _, it_small, _ = small.solve(tol=1e-6, max_iter=10 ** 6)
    assert it_small < it_full
    cap = it_small
    E1, st, stats = oracle_mod.step(p["E"], *args, p["dt"], tol=1e-6,
                                    max_iter=cap, max_cuts=60, tau_tol=10.0)
    assert st == oracle_mod.OK
    assert stats["cuts"] >= 1 and stats["substeps"] >= 2
    assert np.all(np.isfinite(E1))
    # the same substeps taken by hand: tau_tol = 10 lets the step double
    # after each success, each substep clipped to the time left.
    E = p["E"].copy()
    t, hstep, cuts = 0.0, p["dt"], 0
    while p["dt"] - t > 1e-12 * p["dt"]:
        hstep = min(hstep, p["dt"] - t)
        P = oracle_mod.Problem(E, *args[:2], p["h"], p["c"], dmax, rmin, hstep)
        dE, s2, _, _ = P.solve(tol=1e-6, max_iter=cap)
        if s2 != oracle_mod.OK:
            hstep *= 0.1
            cuts += 1
            continue
        E = E + dE
        t += hstep
        w = np.abs(E)
        rho = math.sqrt(np.mean(np.where(w > 0, dE / np.where(w > 0, w, 1), 0) ** 2))
        hstep *= min(max(10.0 / rho, 0.1), 2.0) if rho > 0 else 2.0
    assert cuts == stats["cuts"]
    np.testing.assert_allclose(E1, E, rtol=1e-14, atol=0)
