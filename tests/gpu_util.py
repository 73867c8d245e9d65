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


def full_residual(oracle, p, prm, E_before, dE, chunk=1 << 24):
    """The oracle's b - A dE at every cell, each cell computed on its own from
    the oracle's limiter and operator (the OpenMP build evaluates every cell
    with the same arithmetic as the serial one), in chunks of cells.
    Returns (||b - A dE|| / ||b||, ||b - A dE|| / ||dE||); the second bounds
    the relative error against the exact step since ||A^-1||_2 <= 1."""
    En = np.ascontiguousarray(E_before if isinstance(E_before, np.ndarray) else host(E_before))
    dEh = np.ascontiguousarray(dE if isinstance(dE, np.ndarray) else host(dE))
    K = p["kappa"] if isinstance(p["kappa"], np.ndarray) else host(p["kappa"])
    H = p["eta"] if isinstance(p["eta"], np.ndarray) else host(p["eta"])
    O = oracle.Problem(En, K, H, p["h"], p["c"], prm.d_max, prm.r_min, p["dt"],
                       p.get("theta", 1.0), p.get("a", 1.0), p.get("adot", 0.0),
                       parallel=True)
    rr = bb = 0.0
    for a in range(0, En.size, chunk):
        cells = np.arange(a, min(En.size, a + chunk), dtype=np.int64)
        res, rhs = O.residual_at(dEh, cells)
        rr += float(np.dot(res, res))
        bb += float(np.dot(rhs, rhs))
    dd = float(np.dot(dEh.ravel(), dEh.ravel()))
    return (rr / bb) ** 0.5 if bb > 0 else 0.0, (rr / dd) ** 0.5 if dd > 0 else 0.0
