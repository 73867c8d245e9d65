"""GPU: device-side step control (fld_advance, fld_batch_advance; Sec. 3.4,
the radiation subcycling loop run on the device).  Each run must equal the
same steps taken through the host-driven fld_step / fld_batch_step, bit for
bit (the controller repeats the host's arithmetic), with the same iteration,
substep and cut counts; the steps themselves are checked against the oracle."""
import numpy as np
import pytest

import synth
from gpu_util import dev, host, log_case, oracle_problem, params, rel_l2

pytestmark = pytest.mark.gpu

GATE = {0: 1e-6, 1: 1e-5}


@pytest.fixture(scope="module")
def fld():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    import paper_1306_0645_amd as m
    return m


def _problem(shape, seed, dtf=0.5):
    p = synth.random_problem(shape, seed, sigma_ln=1.5, n_src=3, dt_factor=dtf,
                             E_mode="smooth")
    dx = p["h"][0]
    p["h"] = (dx, 1.25 * dx, 0.8 * dx)
    return p


@pytest.mark.parametrize("warm", [0, 1, 2])
@pytest.mark.parametrize("prec", [0, 1])
def test_advance_equals_host_steps(fld, oracle_mod, prec, warm):
    """Six fixed steps: device control against six fld_step calls."""
    log_case("advance_fixed", prec=prec, warm=warm)
    p = _problem((32, 40, 48), 81)
    prm = params(fld, p, precision=prec, warm_start=warm, cycle_switch=0)
    kap, eta = dev(p["kappa"]), dev(p["eta"])
    H = fld.Solver(p["shape"], p["h"], prm)
    Eh = dev(p["E"])
    its = subs = 0
    for _ in range(6):
        st = H.step(Eh, kap, eta, p["dt"])
        its += st["iters"]
        subs += st["subcycles"]
    H.close()
    D = fld.Solver(p["shape"], p["h"], prm)
    Ed = dev(p["E"])
    sd = D.advance(Ed, kap, eta, p["dt"], n_steps=6, units=5)
    D.close()
    print(f"[advance] prec={prec} warm={warm} iters host={its} device={sd['iters']} "
          f"substeps {subs}/{sd['subcycles']}", flush=True)
    assert sd["status"] == 0 and sd["steps"] == 6
    assert sd["iters"] == its and sd["subcycles"] == subs
    assert np.array_equal(host(Ed), host(Eh))
    # and the six steps are the oracle's six steps
    En = p["E"].copy()
    for _ in range(6):
        q = dict(p)
        q["E"] = En
        dEo, ost, _, _ = oracle_problem(oracle_mod, q, prm).solve(tol=1e-13)
        assert ost == 0
        En = En + dEo
    assert rel_l2(host(Ed), En) <= GATE[prec]


def test_advance_on_the_fused_tile_spmv(fld):
    """Device control on a grid whose fused iteration runs the fused-tile SpMV
    (ragged 96 x 194 x 320, 4-plane fused tiles: 2080 of them), with the
    cycle switch and the local sweeps on: three steps equal three fld_step
    calls bit for bit."""
    log_case("advance_spmv_f")
    p = _problem((320, 194, 96), 84, dtf=0.05)
    prm = params(fld, p, precision=1, fused_tile_z=4)
    kap, eta = dev(p["kappa"]), dev(p["eta"])
    H = fld.Solver(p["shape"], p["h"], prm)
    Eh = dev(p["E"])
    its = 0
    for _ in range(3):
        st = H.step(Eh, kap, eta, p["dt"])
        assert st["status"] == 0
        its += st["iters"]
    H.close()
    D = fld.Solver(p["shape"], p["h"], prm)
    Ed = dev(p["E"])
    sd = D.advance(Ed, kap, eta, p["dt"], n_steps=3, units=5)
    D.close()
    print(f"[advance spmv_f] iters host={its} device={sd['iters']}", flush=True)
    assert sd["status"] == 0 and sd["steps"] == 3
    assert sd["iters"] == its
    assert np.array_equal(host(Ed), host(Eh))


@pytest.mark.parametrize("prec", [0, 1])
def test_advance_subcycles_like_the_host(fld, prec):
    """Solves capped at a few iterations fail at the full step: both drivers
    cut the substep by 10x and subcycle back up to dt, step after step."""
    log_case("advance_cuts", prec=prec)
    p = _problem((24, 32, 32), 82, dtf=2.0)
    kap, eta = dev(p["kappa"]), dev(p["eta"])
    # one level (symmetric Gauss-Seidel PCG): its iteration count grows with
    # dt, so a cap at the count of dt / 10 fails the full step
    U = fld.Solver(p["shape"], p["h"], params(fld, p, precision=prec, mg_levels=1,
                                              cycle_switch=0))
    its = []
    for h in (p["dt"], 0.1 * p["dt"]):
        U.assemble(dev(p["E"]), kap, eta, h)
        its.append(U.solve()[1]["iters"])
    U.close()
    assert its[1] < its[0]
    # (each failure of a grown substep costs a cut: allow plenty)
    prm = params(fld, p, precision=prec, mg_levels=1, max_iter=its[1], max_dt_cuts=60,
                 tau_tol=1e30, cycle_switch=0, warm_start=1)
    H = fld.Solver(p["shape"], p["h"], prm)
    Eh = dev(p["E"])
    tot = {"iters": 0, "subcycles": 0, "dt_cuts": 0}
    for _ in range(2):
        st = H.step(Eh, kap, eta, p["dt"])
        assert st["status"] == 0
        for k in tot:
            tot[k] += st[k]
    H.close()
    D = fld.Solver(p["shape"], p["h"], prm)
    Ed = dev(p["E"])
    sd = D.advance(Ed, kap, eta, p["dt"], n_steps=2, units=4)
    D.close()
    print(f"[advance cuts] host {tot} device iters={sd['iters']} "
          f"substeps={sd['subcycles']} cuts={sd['dt_cuts']}", flush=True)
    assert tot["dt_cuts"] >= 1 and tot["subcycles"] > 2
    assert sd["status"] == 0 and sd["steps"] == 2
    assert (sd["iters"], sd["subcycles"], sd["dt_cuts"]) == \
        (tot["iters"], tot["subcycles"], tot["dt_cuts"])
    assert np.array_equal(host(Ed), host(Eh))


@pytest.mark.parametrize("prec", [0, 1])
def test_adaptive_advance_equals_host_loop(fld, prec):
    """Steps of the controller's dt_next until t_end (the host loop a caller
    would write: dt = min(dt_next, t_end - t))."""
    log_case("advance_adaptive", prec=prec)
    p = _problem((32, 32, 32), 83, dtf=0.05)
    prm = params(fld, p, precision=prec, tau_tol=0.05, cycle_switch=0)
    kap, eta = dev(p["kappa"]), dev(p["eta"])
    t_end = 20 * p["dt"]
    H = fld.Solver(p["shape"], p["h"], prm)
    Eh = dev(p["E"])
    t, dt, n, its = 0.0, p["dt"], 0, 0
    while not (t_end - t <= 1e-12 * t_end):
        h = min(dt, t_end - t)
        st = H.step(Eh, kap, eta, h)
        assert st["status"] == 0
        its += st["iters"]
        t += h
        dt = st["dt_next"]
        n += 1
    H.close()
    D = fld.Solver(p["shape"], p["h"], prm)
    Ed = dev(p["E"])
    sd = D.advance(Ed, kap, eta, p["dt"], n_steps=0, t_end=t_end, units=3)
    D.close()
    print(f"[advance adaptive] steps host={n} device={sd['steps']} "
          f"iters {its}/{sd['iters']}", flush=True)
    assert n > 3 and sd["status"] == 0
    assert sd["steps"] == n and sd["iters"] == its
    assert np.array_equal(host(Ed), host(Eh))


def test_batch_advance_equals_host_batch_steps(fld):
    """Three uneven problems in one batch: device-controlled steps equal
    host-driven batched steps and each problem's own device run."""
    log_case("batch_advance")
    shapes = [(16, 24, 32), (32, 32, 32), (24, 16, 40)]
    ps = [_problem(s, 90 + i) for i, s in enumerate(shapes)]
    ref = max(ps, key=lambda q: q["L_unit"])
    prm = fld.fld_default_params(ref["c"], ref["L_unit"], precision=1, cycle_switch=0)
    K = [dev(q["kappa"]) for q in ps]
    Hs = [dev(q["eta"]) for q in ps]
    dts = [q["dt"] for q in ps]
    B = fld.Batch([q["shape"] for q in ps], [q["h"] for q in ps], prm)
    Eh = [dev(q["E"]) for q in ps]
    for _ in range(4):
        B.step(Eh, K, Hs, dts)
    B.close()
    B = fld.Batch([q["shape"] for q in ps], [q["h"] for q in ps], prm)
    Ed = [dev(q["E"]) for q in ps]
    sts = B.advance(Ed, K, Hs, dts, n_steps=4, units=6)
    B.close()
    assert all(s["status"] == 0 and s["steps"] == 4 for s in sts)
    for a, b in zip(Ed, Eh):
        assert np.array_equal(host(a), host(b))
    for i, q in enumerate(ps):
        S = fld.Solver(q["shape"], q["h"], prm)
        Es = dev(q["E"])
        S.advance(Es, K[i], Hs[i], dts[i], n_steps=4, units=6)
        S.close()
        assert np.array_equal(host(Es), host(Ed[i]))


def test_advance_rejects_bad_arguments(fld):
    p = _problem((16, 16, 16), 84)
    prm = params(fld, p)
    S = fld.Solver(p["shape"], p["h"], prm)
    E = dev(p["E"])
    before = E.clone()
    for kw in (dict(n_steps=-1), dict(n_steps=0, t_end=0.0), dict(units=-2),
               dict(n_steps=0, t_end=float("nan"))):
        st = S.advance(E, dev(p["kappa"]), dev(p["eta"]), p["dt"], check=False, **kw)
        assert st["returned"] == fld.FLD_EINVAL, kw
    st = S.advance(E, dev(p["kappa"]), dev(p["eta"]), -p["dt"], check=False)
    assert st["returned"] == fld.FLD_EINVAL
    import torch
    assert torch.equal(E, before)
    S.close()
