"""GPU parity: the HIP path (through the C-ABI) against the FP64 oracle.

Gates (from the method's required accuracy): relative L2 error of dE (or
E^{n+1}) at most 1e-6 in FP64 and 1e-5 in mixed precision, the true FP64
residual of the GPU result (computed by the oracle's own operator) at most the
1e-8 PCG tolerance, and the a-posteriori bound ||dE - dE*|| <= ||b - A dE||
(since ||A^-1||_2 <= 1 for adot >= 0) holding.  Inputs are seeded synthetic
fields of the paper's kind (lognormal opacity, point-source emissivity).
"""
import math

import numpy as np
import pytest

import synth
from gpu_util import dev, full_residual, host, log_case, oracle_problem, params, rel_l2

pytestmark = pytest.mark.gpu

GATE = {0: 1e-6, 1: 1e-5}


@pytest.fixture(scope="module")
def fld():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    import paper_1306_0645_amd as m
    return m


def _problem(shape, seed, theta=1.0, aniso=True, adot_frac=0.0, dt_factor=0.05,
             E_mode="smooth", sigma_ln=1.5):
    p = synth.random_problem(shape, seed, sigma_ln=sigma_ln, n_src=3,
                             dt_factor=dt_factor, E_mode=E_mode, theta=theta)
    if aniso:
        dx = p["h"][0]
        p["h"] = (dx, 1.25 * dx, 0.8 * dx)
    p["adot"] = adot_frac / p["dt"]
    return p


def _solver(fld, p, **kw):
    prm = params(fld, p, **kw)
    return fld.Solver(p["shape"], p["h"], prm), prm


def _assemble(S, p):
    S.assemble(dev(p["E"]), dev(p["kappa"]), dev(p["eta"]), p["dt"], p["a"],
               p["adot"])


ASM_CASES = [((8, 8, 8), 1.0), ((12, 16, 20), 0.5), ((48, 48, 48), 1.0),
             ((40, 64, 96), 1.0)]


@pytest.mark.parametrize("shape,theta", ASM_CASES)
@pytest.mark.parametrize("prec", [0, 1])
def test_assembly_matches_oracle(fld, oracle_mod, shape, theta, prec):
    log_case("assembly", shape=shape, theta=theta, prec=prec)
    p = _problem(shape, 11, theta=theta, adot_frac=0.05)
    S, prm = _solver(fld, p, precision=prec)
    _assemble(S, p)
    got = {k: host(v) for k, v in S.fld_get_system().items()}
    diag, Ax, Ay, Az, b = oracle_problem(oracle_mod, p, prm).system()
    np.testing.assert_allclose(got["diag"], diag, rtol=1e-13)
    for g, w in ((got["Tx"], Ax), (got["Ty"], Ay), (got["Tz"], Az)):
        np.testing.assert_allclose(g, w, rtol=1e-13, atol=1e-16 * np.abs(w).max())
    np.testing.assert_allclose(got["b"], b, rtol=0, atol=1e-12 * np.abs(b).max())


@pytest.mark.parametrize("shape", [(8, 8, 8), (12, 16, 20), (40, 64, 96)])
def test_spmv_matches_oracle(fld, oracle_mod, shape):
    log_case("spmv", shape=shape)
    p = _problem(shape, 12, dt_factor=0.5)
    S, prm = _solver(fld, p)
    _assemble(S, p)
    u = np.random.default_rng(3).normal(size=shape)
    got = host(S.fld_apply(dev(u)))
    want = oracle_problem(oracle_mod, p, prm).apply_A(u)
    np.testing.assert_allclose(got, want, rtol=0, atol=1e-13 * np.abs(want).max())


SOLVE_CASES = [
    ((8, 8, 8), 1.0, 0.05, "zero"),
    ((12, 16, 20), 0.5, 0.2, "smooth"),
    ((32, 32, 32), 1.0, 0.05, "zero"),
    ((48, 48, 48), 1.0, 1.0, "smooth"),
    ((40, 64, 96), 1.0, 2.0, "smooth"),
    ((64, 64, 64), 0.5, 4.0, "smooth"),
]


def _check_solution(oracle_mod, p, prm, dE, st, prec, tag):
    O = oracle_problem(oracle_mod, p, prm)
    dEo, sto, it, rel = O.solve(tol=1e-13)
    assert sto == oracle_mod.OK
    err = rel_l2(dE, dEo)
    diag, Ax, Ay, Az, b = O.system()
    r = b - O.apply_A(dE)
    true_rel = np.linalg.norm(r) / np.linalg.norm(b)
    print(f"[{tag}] iters={st['iters']} levels={st['levels']} err={err:.3e} "
          f"bound={st['err_bound']:.3e} true_rel={true_rel:.3e}", flush=True)
    assert st["status"] == 0
    assert true_rel <= prm.rtol * (1 + 1e-6)
    assert abs(st["rel_resid"] - true_rel) <= 1e-3 * prm.rtol + 1e-6 * true_rel
    assert err <= GATE[prec]
    # a-posteriori bound: ||dE - dE*|| <= ||r||  (||A^-1|| <= 1)
    assert np.linalg.norm(dE - dEo) <= np.linalg.norm(r) * (1 + 1e-6) + 1e-13 * np.linalg.norm(dEo)
    return err


@pytest.mark.parametrize("shape,theta,dtf,emode", SOLVE_CASES)
@pytest.mark.parametrize("prec,d64", [(0, 1), (1, 1), (1, 0)])
def test_solve_matches_oracle(fld, oracle_mod, shape, theta, dtf, emode, prec, d64):
    """d64: the mixed form's search direction in FP64 (the default) or FP32."""
    log_case("solve", shape=shape, theta=theta, dtf=dtf, prec=prec, d64=d64)
    p = _problem(shape, 13, theta=theta, dt_factor=dtf, E_mode=emode)
    S, prm = _solver(fld, p, precision=prec, direction_fp64=d64)
    _assemble(S, p)
    dE, st = S.solve()
    _check_solution(oracle_mod, p, prm, host(dE), st, prec, f"solve{shape}")


@pytest.mark.parametrize("prec", [0, 1])
def test_step_matches_oracle(fld, oracle_mod, prec):
    log_case("step", prec=prec)
    p = _problem((32, 24, 16), 14, dt_factor=0.5)
    S, prm = _solver(fld, p, precision=prec)
    E = dev(p["E"])
    st = S.step(E, dev(p["kappa"]), dev(p["eta"]), p["dt"], p["a"], p["adot"])
    assert st["status"] == 0 and st["subcycles"] == 1 and st["dt_cuts"] == 0
    dEo, sto, _, _ = oracle_problem(oracle_mod, p, prm).solve(tol=1e-13)
    assert rel_l2(host(E), p["E"] + dEo) <= GATE[prec]
    # the step controller's relative change, from its definition
    En = p["E"] + dEo
    rho = math.sqrt(np.mean((dEo / np.abs(En)) ** 2))
    assert st["rel_change_rms"] == pytest.approx(rho, rel=1e-4)
    f = min(2.0, max(0.1, prm.tau_tol / rho))
    assert st["dt_next"] == pytest.approx(p["dt"] * f, rel=1e-4)


def test_single_source_workload(fld, oracle_mod):
    """The 32^3 single-source step in FP64 with a 4-level V(2,2) cycle."""
    log_case("single_source_32")
    p = synth.single_source(32)
    S, prm = _solver(fld, p, mg_levels=4, nu_pre=2, nu_post=2)
    _assemble(S, p)
    dE, st = S.solve()
    assert st["levels"] == 4
    _check_solution(oracle_mod, p, prm, host(dE), st, 0, "c1")


def test_fp64_preconditioner_is_symmetric_positive(fld):
    log_case("vcycle_symmetry")
    p = _problem((32, 32, 48), 15, dt_factor=2.0)
    S, prm = _solver(fld, p)
    rng = np.random.default_rng(5)
    u = rng.normal(size=p["shape"])
    v = rng.normal(size=p["shape"])
    _assemble(S, p)
    Bu = host(S.fld_precondition(dev(u)))
    _assemble(S, p)
    Bv = host(S.fld_precondition(dev(v)))
    a, b = np.vdot(u, Bv), np.vdot(v, Bu)
    assert abs(a - b) <= 1e-12 * abs(a)
    assert np.vdot(u, Bu) > 0 and np.vdot(v, Bv) > 0
    # and it is a contraction in the A-norm: ||(I - B A) e||_A < ||e||_A
    _assemble(S, p)
    Ae = host(S.fld_apply(dev(u)))
    _assemble(S, p)
    BAe = host(S.fld_precondition(dev(Ae)))
    e2 = u - BAe
    _assemble(S, p)
    Ae2 = host(S.fld_apply(dev(e2)))
    ratio = math.sqrt(np.vdot(e2, Ae2) / np.vdot(u, Ae))
    print(f"[vcycle] A-norm contraction {ratio:.3f}", flush=True)
    assert ratio < 0.5


def test_graph_replay_is_bit_identical(fld):
    log_case("graph")
    p = _problem((48, 48, 48), 16, dt_factor=1.0)
    out = []
    for g in (0, 1):
        S, prm = _solver(fld, p, precision=1, use_graph=g, check_every=2)
        _assemble(S, p)
        dE, st = S.solve()
        out.append((host(dE), st["iters"]))
        # a second solve on the same handle replays the captured graph again
        _assemble(S, p)
        dE2, st2 = S.solve()
        assert np.array_equal(host(dE2), out[-1][0])
    assert out[0][1] == out[1][1]
    assert np.array_equal(out[0][0], out[1][0])


def test_failure_paths(fld):
    import torch
    log_case("failures")
    p = _problem((16, 16, 16), 17, dt_factor=1.0)
    # NaN opacity -> non-finite residual, E untouched
    S, prm = _solver(fld, p, max_dt_cuts=0)
    kap = p["kappa"].copy()
    kap[3, 4, 5] = np.nan
    E = dev(p["E"])
    st = S.step(E, dev(kap), dev(p["eta"]), p["dt"], check=False)
    assert st["status"] == fld.FLD_ENONFINITE
    assert np.array_equal(host(E), p["E"])
    # iteration cap with no cuts allowed -> ENOCONV, E untouched
    S, prm = _solver(fld, p, max_iter=1, rtol=1e-14, max_dt_cuts=0)
    E = dev(p["E"])
    st = S.step(E, dev(p["kappa"]), dev(p["eta"]), p["dt"], check=False)
    assert st["status"] == fld.FLD_ENOCONV
    assert np.array_equal(host(E), p["E"])
    # invalid arguments are rejected before any launch
    with pytest.raises(fld.FLDError) as ei:
        S.step(E, dev(p["kappa"]), dev(p["eta"]), -1.0)
    assert ei.value.status == fld.FLD_EINVAL
    S2, _ = _solver(fld, p)
    with pytest.raises(fld.FLDError):
        S2.solve()  # nothing assembled on this handle yet
    torch.cuda.synchronize()


def test_subcycling_matches_oracle_substeps(fld, oracle_mod):
    """A step whose full-length solve fails is cut 10x and subcycled; the
    result equals oracle solves over the same substeps.  The iteration cap is
    the count a 0.1 dt solve needs (so dt fails and 0.1 dt succeeds); the
    substep sequence is replayed with single GPU solves under the same cap
    (tau_tol is huge, so the step doubles after every success).  A one-level
    cycle (symmetric Gauss-Seidel) is used because its iteration count grows
    with dt, unlike multigrid's."""
    log_case("subcycle")
    p = _problem((32, 32, 32), 18, dt_factor=2.0, E_mode="smooth")
    kap, eta = dev(p["kappa"]), dev(p["eta"])
    U, _ = _solver(fld, p, mg_levels=1, cycle_switch=0)
    its = []
    for h in (p["dt"], 0.1 * p["dt"]):
        U.assemble(dev(p["E"]), kap, eta, h)
        its.append(U.solve()[1]["iters"])
    print(f"[subcycle] iterations at dt, 0.1 dt: {its}", flush=True)
    assert its[1] < its[0]
    # cold starts on both sides: the replay below solves each substep from 0
    cap = dict(max_iter=its[1], tau_tol=1e30, max_dt_cuts=60, mg_levels=1,
               cycle_switch=0, warm_start=0)
    S, prm = _solver(fld, p, **cap)
    E = dev(p["E"])
    st = S.step(E, kap, eta, p["dt"])
    assert st["dt_cuts"] >= 1 and st["subcycles"] >= 2, st
    R, _ = _solver(fld, p, **cap)
    t, h, seq, cuts, Ecur = 0.0, p["dt"], [], 0, dev(p["E"])
    while p["dt"] - t > 1e-12 * p["dt"]:
        h = min(h, p["dt"] - t)
        R.assemble(Ecur, kap, eta, h)
        dE, s = R.solve(check=False)
        if s["status"] != 0:
            h *= 0.1
            cuts += 1
            continue
        Ecur = Ecur + dE
        seq.append(h)
        t += h
        h *= 2.0
    assert len(seq) == st["subcycles"] and cuts == st["dt_cuts"]
    assert np.array_equal(host(Ecur), host(E))
    En = p["E"].copy()
    for hh in seq:
        q = dict(p)
        q["E"], q["dt"] = En, hh
        dEo, sto, _, _ = oracle_problem(oracle_mod, q, prm).solve(tol=1e-13)
        En = En + dEo
    assert rel_l2(host(E), En) <= 1e-6


@pytest.mark.parametrize("d64", [1, 0])
def test_fused_tile_spmv_ragged(fld, oracle_mod, d64):
    """The fused iteration's SpMV on the fused tiles (4 rows per thread): a
    ragged 96 x 194 x 320 grid (a 32-wide x tile, a 2-row y tile) with
    4-plane fused tiles gives 2080 of them, enough for that SpMV; with
    32-plane tiles (260) the same solve takes the 64 x 4 tiles.  Both meet the
    gates against the oracle's residual at every cell, and the two solutions
    differ by no more than their residual norms allow."""
    log_case("fused_tile_spmv", d64=d64)
    p = _problem((320, 194, 96), 29, dt_factor=0.05)
    cells = np.arange(320 * 194 * 96, dtype=np.int64)
    sols, rnorm = [], []
    for ftz in (4, 32):
        S, prm = _solver(fld, p, precision=1, direction_fp64=d64, fused_tile_z=ftz)
        _assemble(S, p)
        dE, st = S.solve()
        dEh = host(dE)
        O = oracle_problem(oracle_mod, p, prm)
        res, rhs = O.residual_at(dEh, cells)
        true_rel = np.linalg.norm(res) / np.linalg.norm(rhs)
        bound = np.linalg.norm(res) / np.linalg.norm(dEh)
        print(f"[fused_tile_spmv ftz={ftz} d64={d64}] iters={st['iters']} "
              f"true_rel={true_rel:.3e} err_bound={bound:.3e}", flush=True)
        assert st["status"] == 0
        assert true_rel <= prm.rtol * (1 + 1e-6)
        assert bound <= GATE[1]
        sols.append(dEh)
        rnorm.append(np.linalg.norm(res))
    # each within ||r|| of the exact solution (||A^-1|| <= 1)
    assert np.linalg.norm(sols[0] - sols[1]) <= (rnorm[0] + rnorm[1]) * (1 + 1e-6)


@pytest.mark.parametrize("prec", [0, 1])
def test_full_size_many_sources_residual(fld, oracle_mod, prec):
    """256^3, 64 sources (the benchmark workload), two successive steps in the
    benchmark's launch configuration: the oracle evaluates b - A dE at every
    cell, one cell at a time, from its own limiter and operator."""
    import torch
    log_case("many_sources_256", prec=prec)
    p = synth.many_sources(256)
    S, prm = _solver(fld, p, precision=prec)
    E = dev(p["E"])
    kap, eta = dev(p["kappa"]), dev(p["eta"])
    cells = np.arange(E.numel(), dtype=np.int64)
    En = p["E"]
    for step in range(2):
        S.assemble(E, kap, eta, p["dt"])
        dE, st = S.solve()
        q = dict(p)
        q["E"] = En
        O = oracle_problem(oracle_mod, q, prm)
        dEh = host(dE)
        res, rhs = O.residual_at(dEh, cells)
        true_rel = np.linalg.norm(res) / np.linalg.norm(rhs)
        bound = np.linalg.norm(res) / np.linalg.norm(dEh)
        print(f"[c2 step {step} prec {prec}] iters={st['iters']} "
              f"true_rel={true_rel:.3e} err_bound={bound:.3e}", flush=True)
        assert st["status"] == 0
        assert true_rel <= prm.rtol * (1 + 1e-6)
        assert bound <= GATE[prec]
        E += dE
        torch.cuda.synchronize()
        En = En + dEh


@pytest.mark.parametrize("prec", [0, 1])
def test_full_size_reionization_share_residual(fld, oracle_mod, prec):
    """640^3 reionization share (10^4 sources, ionized bubbles), 6 levels,
    in the benchmark's launch configuration: two successive fld_step calls
    from E^0, the first with the configured V(1,1) cycle and the second with
    the cycle it switches to (mixed: trilinear V(1,1) with the interpolated
    finest correction).  The oracle evaluates b - A dE at every cell of both
    steps: the relative residual meets the tolerance and the error bound
    ||b - A dE|| / ||dE|| the gate."""
    import torch
    log_case("reionization_640", prec=prec)
    q = synth.t_reionization_share(n=640, device="cuda")
    prm = fld.fld_default_params(q["c"], q["L_unit"], precision=prec, mg_levels=6)
    S = fld.Solver(q["shape"], q["h"], prm)
    E, kap, eta = q["E"], q["kappa"], q["eta"]
    for step in range(2):
        Eb = E.clone()
        st = S.step(E, kap, eta, q["dt"])
        dE = E - Eb
        torch.cuda.synchronize()
        true_rel, bound = full_residual(oracle_mod, q, prm, Eb, dE)
        print(f"[c3 step {step} prec {prec}] iters={st['iters']} nu={st['cycle_nu']} "
              f"tri={st['trilinear']} solver_rel={st['rel_resid']:.3e} "
              f"true_rel={true_rel:.3e} err_bound={bound:.3e}", flush=True)
        assert st["status"] == 0 and st["rel_resid"] <= prm.rtol
        assert true_rel <= prm.rtol * (1 + 1e-6)
        assert bound <= GATE[prec]
        if prec == 1 and step == 1:
            assert st["trilinear"] == 1 and st["cycle_nu"] == 1
        del Eb, dE
    S.close()


@pytest.mark.parametrize("prec", [0, 1])
def test_adaptive_cycle_switch(fld, oracle_mod, prec):
    """A high-contrast problem (ionized bubbles, nu ~ 61) needs more than 12
    V(1,1) iterations, so the handle's next steps switch cycle: at 64^3
    (below the 2^23 cells from which mixed precision keeps V(1,1) with the
    trilinear correction) to V(2,2), with the trilinear correction in mixed
    precision.  Every step still meets the tolerance and matches the
    oracle."""
    log_case("cycle_switch", prec=prec)
    q = synth.t_reionization_share(n=64, n_src=12, device="cpu")
    p = {k: (v.numpy() if hasattr(v, "numpy") else v) for k, v in q.items()}
    S, prm = _solver(fld, p, precision=prec)
    E = dev(p["E"])
    kap, eta = dev(p["kappa"]), dev(p["eta"])
    En = p["E"].copy()
    seen = []
    for k in range(3):
        st = S.step(E, kap, eta, p["dt"])
        seen.append((st["cycle_nu"], st["trilinear"], st["iters"]))
        qq = dict(p)
        qq["E"] = En
        dEo, _, _, _ = oracle_problem(oracle_mod, qq, prm).solve(tol=1e-13)
        En = En + dEo
        assert st["status"] == 0
        assert rel_l2(host(E), En) <= GATE[prec]
    print(f"[cycle_switch] (nu, trilinear, iters) per step: {seen}", flush=True)
    assert seen[0][:2] == (1, 0)
    if seen[0][2] > 12:
        assert seen[1][:2] == ((2, 1) if prec == 1 else (2, 0))


@pytest.mark.parametrize("theta", [1.0, 0.5])
@pytest.mark.parametrize("prec", [0, 1])
def test_comoving_step_matches_oracle(fld, oracle_mod, theta, prec):
    """a != 1: the operator on the comoving cell sizes plus adot/a;
    assembly and the solve against the oracle."""
    log_case("comoving", theta=theta, prec=prec)
    p = _problem((24, 32, 40), 23, theta=theta, dt_factor=0.1)
    p["a"] = 0.3
    p["adot"] = 0.3 * 0.05 / p["dt"]
    S, prm = _solver(fld, p, precision=prec)
    _assemble(S, p)
    got = {k: host(v) for k, v in S.fld_get_system().items()}
    O = oracle_problem(oracle_mod, p, prm)
    diag, Ax, Ay, Az, b = O.system()
    np.testing.assert_allclose(got["diag"], diag, rtol=1e-13)
    for g, w in ((got["Tx"], Ax), (got["Ty"], Ay), (got["Tz"], Az)):
        np.testing.assert_allclose(g, w, rtol=1e-13, atol=1e-16 * np.abs(w).max())
    np.testing.assert_allclose(got["b"], b, rtol=0, atol=1e-12 * np.abs(b).max())
    dE, st = S.solve()
    dEo, _, _, _ = O.solve(tol=1e-13)
    err = rel_l2(host(dE), dEo)
    print(f"[comoving] iters={st['iters']} err={err:.2e}", flush=True)
    assert st["status"] == 0
    assert err <= GATE[prec]


@pytest.mark.parametrize("warm", [1, 2])
@pytest.mark.parametrize("prec", [0, 1])
def test_warm_start_steps_match_oracle(fld, oracle_mod, prec, warm):
    """fld_step seeds each step's PCG with a guess from the previous steps'
    dE (warm = 1: extrapolated by the step ratios; warm = 2: the Galerkin
    combination of the last two in the new operator), or starts from 0 when
    that guess does not reduce the residual.  Three successive steps
    (the last at half the step size) must match the oracle's cold solves to
    the gates (the seed changes iteration counts, not the stopping rule); a
    following step with b = 0 (E = eta = 0) must return exactly E = 0, not
    the seed."""
    import torch
    log_case("warm_start", prec=prec, warm=warm)
    p = _problem((48, 40, 32), 31, dt_factor=0.2)
    kap, eta = dev(p["kappa"]), dev(p["eta"])
    W, prm = _solver(fld, p, precision=prec, warm_start=warm)
    C, _ = _solver(fld, p, precision=prec, warm_start=0)
    Ew, Ec = dev(p["E"]), dev(p["E"])
    En = p["E"].copy()
    its_w = its_c = 0
    for k, f in enumerate((1.0, 1.0, 0.5)):
        dt = f * p["dt"]
        sw = W.step(Ew, kap, eta, dt)
        sc = C.step(Ec, kap, eta, dt)
        q = dict(p)
        q["E"], q["dt"] = En, dt
        dEo, _, _, _ = oracle_problem(oracle_mod, q, prm).solve(tol=1e-13)
        En = En + dEo
        err = rel_l2(host(Ew), En)
        print(f"[warm] step {k}: iters warm {sw['iters']} cold {sc['iters']} "
              f"err {err:.2e}", flush=True)
        assert sw["status"] == 0 and sw["rel_resid"] <= prm.rtol
        assert err <= GATE[prec]
        its_w += sw["iters"]
        its_c += sc["iters"]
    print(f"[warm] iterations in all: warm {its_w}, cold {its_c}", flush=True)
    zero, no_eta = torch.zeros_like(Ew), torch.zeros_like(Ew)
    st = W.step(zero, kap, no_eta, p["dt"])
    assert st["status"] == 0
    assert torch.count_nonzero(zero).item() == 0


@pytest.mark.parametrize("prec", [0, 1])
def test_galerkin_guess_recovers_a_combination(fld, oracle_mod, prec):
    """With E^n, kappa and dt fixed, dE is affine in eta: for eta3 = 0.3 eta1
    + 0.7 eta2 the solution is 0.3 dE(eta1) + 0.7 dE(eta2), a point of the
    span of the two previous steps' dE.  The Galerkin guess (warm_start = 2)
    is that point to the previous solves' tolerance, so the third step takes
    at most 2 PCG iterations; the extrapolation (2 dE(n) - dE(n-1), warm_start
    = 1) is not, and takes more.  Both results match the oracle's solve."""
    import torch
    log_case("galerkin_combination", prec=prec)
    p = _problem((48, 40, 32), 35, dt_factor=0.2)
    rng = np.random.default_rng(35)
    eta1 = p["eta"]
    eta2 = np.roll(p["eta"], (5, 7, 3), axis=(0, 1, 2)) * rng.uniform(0.5, 1.5)
    eta3 = 0.3 * eta1 + 0.7 * eta2
    kap = dev(p["kappa"])
    its = {}
    for warm in (1, 2):
        S, prm = _solver(fld, p, precision=prec, warm_start=warm)
        for k, eta in enumerate((eta1, eta2, eta3)):
            E = dev(p["E"])
            st = S.step(E, kap, dev(eta), p["dt"])
            assert st["status"] == 0
        its[warm] = st["iters"]
        q = dict(p)
        q["eta"] = eta3
        dEo, _, _, _ = oracle_problem(oracle_mod, q, prm).solve(tol=1e-13)
        assert rel_l2(host(E), p["E"] + dEo) <= GATE[prec]
        S.close()
    print(f"[galerkin] third-step iterations: extrapolated {its[1]}, "
          f"Galerkin {its[2]}", flush=True)
    assert its[2] <= 2 < its[1]


@pytest.mark.parametrize("nu", [1, 2])
@pytest.mark.parametrize("prec", [0, 1])
def test_single_workgroup_tail_matches_oracle(fld, oracle_mod, prec, nu):
    """tail_cells > 0 moves the small coarse levels (here 16^3 and 8^3 of a
    64^3 grid) into the single-workgroup coarse-solve kernel: the solve still
    matches the oracle, and the FP64 preconditioner stays symmetric."""
    import torch
    log_case("tail", prec=prec, nu=nu)
    p = _problem((64, 64, 64), 41, dt_factor=0.5)
    S, prm = _solver(fld, p, precision=prec, tail_cells=4096, nu_pre=nu,
                     nu_post=nu, cycle_switch=0)
    _assemble(S, p)
    dE, st = S.solve()
    dEo, _, _, _ = oracle_problem(oracle_mod, p, prm).solve(tol=1e-13)
    err = rel_l2(host(dE), dEo)
    print(f"[tail] iters={st['iters']} err={err:.2e}", flush=True)
    assert st["status"] == 0 and err <= GATE[prec]
    if prec == 0:
        g = torch.Generator(device="cuda").manual_seed(5)
        u = torch.randn(p["shape"], dtype=torch.float64, device="cuda", generator=g)
        v = torch.randn(p["shape"], dtype=torch.float64, device="cuda", generator=g)
        _assemble(S, p)
        Mu = S.fld_precondition(u)
        _assemble(S, p)
        Mv = S.fld_precondition(v)
        a, b = float((v * Mu).sum()), float((u * Mv).sum())
        assert abs(a - b) <= 1e-12 * max(abs(a), abs(b))


def test_largest_grid_1024(fld, oracle_mod):
    """1024^3 = 2^30 cells (the C-ABI takes up to 2^31 - 1; a 132 GiB mixed
    workspace), one mixed step of the many-source recipe: the solver's
    residual meets the tolerance, and the oracle's residual at every cell
    meets it too, with the error bound within the gate."""
    import torch
    log_case("grid_1024", prec=1)
    n = 1024
    q = synth.t_problem((n, n, n), 1.5, 64, (1e47, 1e50), 7, 0, "cuda")
    prm = fld.fld_default_params(q["c"], q["L_unit"], precision=1)
    S = fld.Solver(q["shape"], q["h"], prm)
    S.assemble(q["E"], q["kappa"], q["eta"], q["dt"])
    dE, st = S.solve()
    torch.cuda.synchronize()
    S.close()
    del S
    torch.cuda.empty_cache()
    print(f"[grid_1024] iters={st['iters']} rel={st['rel_resid']:.2e}", flush=True)
    assert st["status"] == 0 and st["rel_resid"] <= prm.rtol
    true_rel, bound = full_residual(oracle_mod, q, prm, q["E"], dE)
    print(f"[grid_1024] true_rel={true_rel:.3e} err_bound={bound:.3e}", flush=True)
    assert true_rel <= prm.rtol * (1 + 1e-6)
    assert bound <= GATE[1]


RESTART_CASES = [(1e5, 1e-10), (1e7, 1e-8)]


@pytest.mark.parametrize("nu,rtol", RESTART_CASES)
@pytest.mark.parametrize("prec,d64", [(0, 1), (1, 1), (1, 0)])
def test_refinement_restart(fld, oracle_mod, prec, d64, nu, rtol):
    """An optically thin box over a long step (diffusion number nu = dt D /
    dx^2 of 1e5 and 1e7) with a smooth emissivity and a uniform E^n: the
    step's solution is dominated by its mean, which the diffusion term leaves
    alone, so the SpMV's rounding (of order eps nu relative) enters the
    recursive residual every iteration and drifts it away from the true one.
    The recursive residual meets the tolerance first; the true FP64 residual
    does not, so the solve restarts from it (iterative refinement) and then
    meets the tolerance on the true residual: status OK, at least one
    restart, the oracle's own residual of the result within the tolerance,
    and the result within the gate of the oracle's solution."""
    log_case("restart", prec=prec, d64=d64, nu=nu, rtol=rtol)
    p = synth.thin_uniform_problem(32, nu, seed=3)
    S, prm = _solver(fld, p, precision=prec, direction_fp64=d64, rtol=rtol,
                     max_iter=200, cycle_switch=0, warm_start=0)
    _assemble(S, p)
    dE, st = S.solve()
    dEh = host(dE)
    true_rel, bound = full_residual(oracle_mod, p, prm, p["E"], dEh)
    dEo, ost, _, _ = oracle_problem(oracle_mod, p, prm).solve(tol=1e-13, max_iter=20000)
    err = rel_l2(dEh, dEo)
    print(f"[restart] iters={st['iters']} restarts={st['restarts']} "
          f"solver_rel={st['rel_resid']:.2e} oracle_rel={true_rel:.2e} err={err:.2e}",
          flush=True)
    assert st["status"] == 0 and st["restarts"] >= 1
    assert st["rel_resid"] <= rtol
    assert true_rel <= rtol * (1 + 1e-6)
    assert ost == 0 and err <= GATE[prec]


@pytest.mark.parametrize("nu", [1, 2])
@pytest.mark.parametrize("prec", [0, 1])
def test_jacobi_smoother_solve_matches_oracle(fld, oracle_mod, prec, nu):
    """The weighted-Jacobi smoother (the alternative to red/black sweeps) on
    an anisotropic ragged grid: the PCG solve meets the same gates."""
    log_case("jacobi_solve", prec=prec, nu=nu)
    p = _problem((40, 64, 96), 43, dt_factor=0.5)
    S, prm = _solver(fld, p, precision=prec, smoother=fld.FLD_SMOOTH_JACOBI,
                     nu_pre=nu, nu_post=nu, cycle_switch=0)
    _assemble(S, p)
    dE, st = S.solve()
    _check_solution(oracle_mod, p, prm, host(dE), st, prec, f"jacobi nu={nu}")


@pytest.mark.parametrize("nu", [1, 2, 3])
def test_jacobi_one_level_cycle_is_the_sweeps(fld, oracle_mod, nu):
    """On one level the cycle is nu_pre sweeps from x = 0, then nu_post
    sweeps, each x <- x + w D^-1 (f - A x) with w = 6/7: computed here with
    the oracle's operator and diagonal."""
    log_case("jacobi_one_level", nu=nu)
    p = _problem((16, 12, 20), 44, dt_factor=0.5)
    S, prm = _solver(fld, p, smoother=fld.FLD_SMOOTH_JACOBI, mg_levels=1,
                     nu_pre=nu, nu_post=nu, cycle_switch=0)
    O = oracle_problem(oracle_mod, p, prm)
    diag = O.system()[0]
    f = np.random.default_rng(6).normal(size=p["shape"])
    w = 6.0 / 7.0
    x = np.zeros_like(f)
    for _ in range(2 * nu):
        x = x + w * (f - O.apply_A(x)) / diag
    _assemble(S, p)
    z = host(S.fld_precondition(dev(f)))
    assert rel_l2(z, x) <= 1e-13


def test_jacobi_fp64_preconditioner_is_symmetric_positive(fld):
    log_case("jacobi_symmetry")
    p = _problem((32, 32, 48), 15, dt_factor=2.0)
    S, prm = _solver(fld, p, smoother=fld.FLD_SMOOTH_JACOBI)
    rng = np.random.default_rng(5)
    u = rng.normal(size=p["shape"])
    v = rng.normal(size=p["shape"])
    _assemble(S, p)
    Bu = host(S.fld_precondition(dev(u)))
    _assemble(S, p)
    Bv = host(S.fld_precondition(dev(v)))
    a, b = np.vdot(u, Bv), np.vdot(v, Bu)
    assert abs(a - b) <= 1e-12 * abs(a)
    assert np.vdot(u, Bu) > 0 and np.vdot(v, Bv) > 0
    _assemble(S, p)
    Ae = host(S.fld_apply(dev(u)))
    _assemble(S, p)
    e2 = u - host(S.fld_precondition(dev(Ae)))
    _assemble(S, p)
    Ae2 = host(S.fld_apply(dev(e2)))
    ratio = math.sqrt(np.vdot(e2, Ae2) / np.vdot(u, Ae))
    print(f"[jacobi vcycle] A-norm contraction {ratio:.3f}", flush=True)
    assert ratio < 0.7


@pytest.mark.parametrize("prec", [0, 1])
def test_fused_coarse_levels_match_oracle(fld, oracle_mod, prec):
    """Every level above the coarsest of a 128 x 96 x 64 grid in the fused
    passes (fused_levels = 4; the automatic rule fuses a coarse level only
    from 2^20 cells): the solve meets the gates."""
    log_case("fused_coarse", prec=prec)
    p = _problem((64, 96, 128), 45, dt_factor=0.5)
    S, prm = _solver(fld, p, precision=prec, fused_levels=4, cycle_switch=0)
    _assemble(S, p)
    dE, st = S.solve()
    _check_solution(oracle_mod, p, prm, host(dE), st, prec, "fused_coarse")


@pytest.mark.parametrize("prolongation", [0, 1])
def test_v11_prolongation_matches_oracle(fld, oracle_mod, prolongation):
    """Mixed V(1,1) with piecewise-constant (0) and trilinear (1) correction
    through the fused finest passes, the per-half-sweep coarse kernels and
    the single-workgroup tail: the solve meets the gates."""
    log_case("v11_prolongation", prolongation=prolongation)
    p = _problem((64, 64, 64), 46, dt_factor=0.5)
    S, prm = _solver(fld, p, precision=1, prolongation=prolongation,
                     cycle_switch=0)
    _assemble(S, p)
    dE, st = S.solve()
    _check_solution(oracle_mod, p, prm, host(dE), st, 1, f"prolong{prolongation}")
