"""Multigroup FLD on the GPU: G independent group systems stepped together in
the batched engine.  Each group's E^{n+1} must match the oracle's step of that
group alone (the gates of the single-problem solves), and be bit-identical to
the same group stepped by a single-problem handle."""
import numpy as np
import pytest

import synth
from gpu_util import host, log_case, rel_l2

pytestmark = pytest.mark.gpu

GATE = {0: 1e-6, 1: 1e-5}


@pytest.fixture(scope="module")
def fld():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    import paper_1306_0645_amd as m
    return m


@pytest.mark.parametrize("n,G", [(32, 3), (48, 5)])
@pytest.mark.parametrize("prec", [0, 1])
def test_multigroup_matches_oracle_and_solo(fld, oracle_mod, n, G, prec):
    import torch
    from paper_1306_0645_amd.multigroup import MultigroupFLD
    log_case("multigroup", n=n, G=G, prec=prec)
    q = synth.t_multigroup(n, G, n_src=8, device="cpu", problem=n)
    E0, K, H = (q[k].to("cuda") for k in ("E", "kappa", "eta"))
    prm = fld.fld_default_params(q["c"], q["L_unit"], precision=prec)
    mg = MultigroupFLD(q["shape"], q["h"], G, prm)
    E = E0.clone()
    sts = mg.step(E, K, H, q["dt"])
    mg.close()
    assert all(s["status"] == 0 for s in sts)
    for g in range(G):
        S = fld.Solver(q["shape"], q["h"], prm)
        Eg = E0[g].clone()
        S.step(Eg, K[g].contiguous(), H[g].contiguous(), q["dt"])
        S.close()
        assert torch.equal(Eg, E[g]), f"group {g} differs from its solo step"
        O = oracle_mod.Problem(q["E"][g].numpy(), q["kappa"][g].numpy(),
                               q["eta"][g].numpy(), q["h"], q["c"], prm.d_max,
                               prm.r_min, q["dt"])
        dEo, _, _, _ = O.solve(tol=1e-13)
        err = rel_l2(host(E[g]), q["E"][g].numpy() + dEo)
        print(f"[multigroup] g={g} iters={sts[g]['iters']} err={err:.2e}",
              flush=True)
        assert err <= GATE[prec]
