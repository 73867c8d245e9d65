"""Helpers shared by the GPU tests: move synthetic problems to the device,
build the paper-default parameters, and run the oracle on the same inputs."""
import numpy as np


def dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to("cuda")


def host(t):
    return t.detach().cpu().numpy()


def params(fld, p, **kw):
    kw.setdefault("theta", p["theta"])
    return fld.fld_default_params(p["c"], p["L_unit"], **kw)


def oracle_problem(oracle, p, prm):
    """The oracle's view of problem p with the same d_max / r_min as prm."""
    return oracle.Problem(p["E"], p["kappa"], p["eta"], p["h"], p["c"],
                          prm.d_max, prm.r_min, p["dt"], p["theta"], p["a"],
                          p["adot"])


def rel_l2(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / nb if nb > 0 else np.linalg.norm(a)


def log_case(name, **kw):
    print(f"[case] {name} " + " ".join(f"{k}={v}" for k, v in kw.items()),
          flush=True)
