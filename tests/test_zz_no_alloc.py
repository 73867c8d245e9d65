"""fld_step_static, the step entry point that allocates nothing (its
workspace is a device array of the library): on two calls in a row, the
second on a smaller grid, its result equals the same step through
fld_create + fld_step with a caller workspace, bit for bit, and meets the
oracle's gates."""
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


@pytest.mark.parametrize("prec", [0, 1])
def test_static_step_equals_workspace_step(fld, oracle_mod, prec):
    import torch
    log_case("no_alloc", prec=prec)
    # the larger grid first, then a smaller one: the second call must not
    # see anything of the first
    for shape, seed in (((48, 40, 56), 71), ((16, 24, 20), 72)):
        p = synth.random_problem(shape, seed, sigma_ln=1.5, n_src=3, dt_factor=0.5,
                                 E_mode="smooth")
        prm = params(fld, p, precision=prec, use_graph=0)
        assert fld.fld_workspace_bytes(fld.make_grid(shape, p["h"]), prm) <= \
            fld.fld_static_scratch_bytes()
        kap, eta = dev(p["kappa"]), dev(p["eta"])
        E_ref = dev(p["E"])
        S = fld.Solver(shape, p["h"], prm)
        st_ref = S.step(E_ref, kap, eta, p["dt"])
        S.close()
        E = dev(p["E"])
        status, st = fld.fld_step_static(shape, p["h"], prm, E, kap, eta, p["dt"])
        torch.cuda.synchronize()
        print(f"[no_alloc] shape={shape} prec={prec} status={status} "
              f"iters={st['iters']} ref_iters={st_ref['iters']}", flush=True)
        assert status == 0 and st["iters"] == st_ref["iters"]
        assert np.array_equal(host(E), host(E_ref))
        dEo, ost, _, _ = oracle_problem(oracle_mod, p, prm).solve(tol=1e-13)
        assert ost == 0
        assert rel_l2(host(E), p["E"] + dEo) <= GATE[prec]


def test_static_step_rejects_a_grid_beyond_its_array(fld):
    import torch
    p = synth.random_problem((128, 128, 128), 73, n_src=2, dt_factor=0.5)
    prm = params(fld, p, precision=1)
    need = fld.fld_workspace_bytes(fld.make_grid(p["shape"], p["h"]), prm)
    assert need > fld.fld_static_scratch_bytes()
    E = dev(p["E"])
    before = E.clone()
    status, _ = fld.fld_step_static(p["shape"], p["h"], prm, E, dev(p["kappa"]),
                                    dev(p["eta"]), p["dt"], check=False)
    torch.cuda.synchronize()
    assert status == fld.FLD_ENOMEM
    assert torch.equal(E, before)
