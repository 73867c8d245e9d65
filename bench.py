#!/usr/bin/env python3
"""Benchmark of the implicit grey FLD step on one MI355X.

Default workload: one GPU's share of a large reionization box (Sec. 5: the
3200^3 run on 125 GPU shares of 640^3 cells each), the 640^3 share with
periodic self-wrapped halos, lognormal HI (sigma_ln 2.0) with ionized bubbles
(x_HI = 1e-4) around 10^4 Poisson-placed sources (Ndot log-uniform
1e46-1e49), E^0 = 1e-45 erg cm^-3, dt = 1e-3 light-crossing times of the
3200-cell box, 6-level multigrid, PCG to a 1e-8 relative residual, 20
successive steps from E^0 (the limiter recomputed from the new E each step).
A "step" is one full timestep: assembly of the limiter system and every
multigrid level, the preconditioned CG solve, and E += dE.

Prints ONE JSON line: Mcell-updates/s of the mixed-precision form (the plain
FP64 form is reported beside it), per-step latency quantiles, the roofline of
the dominant kernel timed live with hipEvents, each form's residual and
error bound evaluated by the oracle at every cell, and the oracle's CPU
throughput on a bounded sample of the same step.  The 256^3 many-source
workload and the 32^3 single-source latency run follow in "secondary".
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E

# Algorithmic (compulsory) bytes per finest-level cell of one launch of each
# finest-level kernel: every input array read once, every output written
# once; neighbours and 1/8-size coarse arrays included where they are read.
# (FP64 V-cycle, FP32 V-cycle)
BYTES_PER_CELL = {
    # assembly with a warm start: E, kappa, eta and the two dE history
    # buffers in; the system, b, the guess x and its residual r = b - A x out
    "assemble": (96.0, 112.0),
    # mixed form: z and p are FP32 (z in, p_old in, p_new out: 4 B each)
    "spmv_p": (64.0, 52.0),
    # fused iteration's SpMV: also x += alpha p_old (x read and written)
    "spmv_px": (80.0, 68.0),
    # the deferred x += alpha p when a solve stops iterating
    "xfix": (24.0, 20.0),
    # Galerkin warm guess: x0 and r = b - A x0 from the operator, b and the
    # two dE (72 B), less the x and r the assembly then leaves to it (16 B)
    "warm_x": (56.0, 56.0),
    "update": (48.0, 44.0),
    "pre0_fine": (48.0, 28.0),
    "half_fine": (56.0, 32.0),
    # mixed: reads the old FP32 z (flexible PCG) and writes the new one
    "half_out": (56.0, 36.0),
    "resid_restrict_fine": (49.0, 28.5),
    "prolong_black_fine": (57.0, 32.5),
    "true_resid": (56.0, 56.0),
    "update_E": (24.0, 24.0),
    # fused down pass; in the mixed form it also reads q and writes the
    # updated residual r - alpha q (the first iteration of a solve skips both)
    "vdown_fine": (41.0, 40.5),
    "vup_fine": (49.0, 32.5),
    # weighted-Jacobi smoother: first sweep from zero (diag, f, x out), a
    # sweep (4 coefficient arrays, x in, f, x out), the last finest sweep
    # (writes z; the mixed form also reads the old z, both FP32), x + P e (x,
    # e at 1/8, out)
    "jacobi0_fine": (24.0, 16.0),
    "jacobi_fine": (56.0, 32.0),
    "jacobi_out": (56.0, 36.0),
    "prolong_add_fine": (17.0, 8.5),
}

# The mixed form with an FP64 search direction (direction_fp64) reads and
# writes p in 8 bytes instead of 4: p_old in and p_new out of the SpMV, p in
# the update and the deferred x update.
DIR64_EXTRA = {"spmv_p": 8.0, "spmv_px": 8.0, "xfix": 4.0, "update": 4.0}


def bpc(name, prec_idx, dir64=False):
    """Algorithmic bytes per finest cell of one launch of kernel `name`."""
    v = BYTES_PER_CELL[name][prec_idx]
    if prec_idx and dir64:
        v += DIR64_EXTRA.get(name, 0.0)
    return v


# Coarse levels (every level below the finest).  One V-cycle's generic
# kernels there (red+black pre-sweep from zero, residual and restriction,
# prolongation with the black post-sweep, the red post-sweep) move these bytes
# per coarse cell (FP64 cycle, FP32 cycle).  Building level l from level l-1
# reads 4 FP64 arrays of level l-1 and writes 4 of level l (plus 4 FP32 copies
# in mixed mode).
COARSE_CYCLE_BYTES = (48.0 + 49.0 + 57.0 + 56.0, 28.0 + 28.5 + 32.5 + 32.0)
# the same under the weighted-Jacobi smoother: first sweep, residual and
# restriction, x + P e, one sweep
COARSE_CYCLE_BYTES_JACOBI = (24.0 + 49.0 + 17.0 + 56.0, 12.0 + 28.5 + 8.5 + 28.0)


def coarse_fraction(levels):
    """Cells of all coarse levels per finest cell (full 2x coarsening)."""
    return sum(8.0 ** -l for l in range(1, levels))


STEP_KERNELS = ("assemble", "true_resid", "update_E", "xfix", "warm_x")
# the old FP32 z that the mixed form's finest up pass reads for flexible PCG
OLD_Z_BYTES = 4.0


def step_bytes(counts, cells, prec_idx, levels, dir64=False):
    """Algorithmic bytes of one step from the launches counted in a survey
    step, split into (per step, per PCG iteration x iterations): finest-level
    kernels exactly, coarse levels from their share of cells."""
    fixed = it = 0.0
    for name, count in counts.items():
        if name in BYTES_PER_CELL:
            v = count * bpc(name, prec_idx, dir64) * cells
            if name in STEP_KERNELS:
                fixed += v
            else:
                it += v
    cf = coarse_fraction(levels)
    cycles = counts.get("vdown_fine", 0) or counts.get("pre0_fine", 0)
    it += cycles * cf * COARSE_CYCLE_BYTES[prec_idx] * cells
    it += counts.get("jacobi0_fine", 0) * cf * COARSE_CYCLE_BYTES_JACOBI[prec_idx] * cells
    coarsen = 32.0 * (1.0 + cf - 8.0 ** -(levels - 1)) + (48.0 if prec_idx else 32.0) * cf
    fixed += counts.get("assemble", 0) * coarsen * cells
    if prec_idx:
        # the first cycle of each solve reads no old z (beta = 0 there)
        fixed -= counts.get("assemble", 0) * OLD_Z_BYTES * cells
    return fixed, it


def model_step_bytes(cells, iters, nu, prec_idx, levels, steps=1, warm=False,
                     dir64=False):
    # warm: 0/False cold, 1 extrapolated guess, 2 or True Galerkin guess (the
    # library default)
    """Algorithmic bytes of `steps` steps of one problem taking `iters` PCG
    iterations in all, from the cycle structure:
    assembly and coarse operators, the true-residual check and E += dE once,
    then per PCG iteration one V(nu,nu) cycle (fused finest-level passes for
    nu = 1), the SpMV and the vector update."""
    B = {k: bpc(k, prec_idx, dir64) for k in BYTES_PER_CELL}
    cf = coarse_fraction(levels)
    coarse = (COARSE_CYCLE_BYTES[prec_idx]
              + (4 * (nu - 1)) * (56.0, 32.0)[prec_idx])
    if nu == 1 and prec_idx == 1:
        # fused mixed iteration: the residual update rides in the down pass
        # and the x update in the SpMV
        per_iter = B["vdown_fine"] + B["vup_fine"] + cf * coarse + B["spmv_px"]
    elif nu == 1:
        per_iter = (B["vdown_fine"] + B["vup_fine"] + cf * coarse + B["spmv_p"]
                    + B["update"])
    else:
        fine = (B["pre0_fine"] + B["resid_restrict_fine"] + B["prolong_black_fine"]
                + B["half_out"] + (4 * (nu - 1)) * B["half_fine"])
        per_iter = fine + cf * coarse + B["spmv_p"] + B["update"]
    coarsen = 32.0 * (1.0 + cf - 8.0 ** -(levels - 1)) + (48.0 if prec_idx else 32.0) * cf
    fixed = B["assemble"] + coarsen + B["true_resid"] + B["update_E"]
    if nu == 1 and prec_idx == 1:
        fixed += B["xfix"]
    if prec_idx == 1:
        fixed -= OLD_Z_BYTES  # no old z in the first cycle of the solve
    warm = 2 if warm is True else int(warm)
    if not warm:  # a cold assembly reads no history
        fixed -= 16.0
    elif warm >= 2:
        fixed += B["warm_x"]
    return cells * (steps * fixed + iters * per_iter)


def auto_levels(n):
    """Levels of the automatic hierarchy of an n^3 grid: halve while the
    extent is even and the coarse extent stays >= 4."""
    lv = 1
    while n % 2 == 0 and n // 2 >= 4:
        n //= 2
        lv += 1
    return lv


def measured_traffic(kernel, form, workload=None, root=ROOT):
    """HBM bytes per launch of `kernel` from the rocprofv3 byte-counter
    records under root/profiles/ (for that workload, when one is named), or
    None when there is no record or any source the record names (relative to
    root) has changed since the counters were taken."""
    import glob
    import hashlib
    for path in sorted(glob.glob(os.path.join(root, "profiles", "*.md"))):
        with open(path) as f:
            for line in f:
                if not line.startswith("traffic-record:"):
                    continue
                kv = dict(t.split("=", 1) for t in line.split()[1:])
                if kv.get("kernel") != kernel or kv.get("form") != form:
                    continue
                if workload is not None and kv.get("workload") != workload:
                    continue
                for item in kv.get("sources", "").split(","):
                    rel, want = item.rsplit(":", 1)
                    try:
                        with open(os.path.join(root, rel), "rb") as src:
                            have = hashlib.sha256(src.read()).hexdigest()
                    except OSError:
                        return None
                    if have != want:
                        return None
                return float(kv["bytes_per_launch"])
    return None


# rocprofv3 kernel names of the finest-level kernels, by (bench name, form)
PMC_KERNELS = {
    # the fused iteration's SpMV: on the fused tiles where a grid gives 2048
    # of them, else on the 64 x 4 tiles (the first name that ran is taken)
    ("spmv_px", "mixed_dir64"): ("fld::k_spmv_f<true, 2>", "fld::k_spmv_p<true, 2>"),
    ("spmv_px", "mixed"): ("fld::k_spmv_f<true, 1>", "fld::k_spmv_p<true, 1>"),
    ("spmv_p", "fp64"): "fld::k_spmv_p<false, 0>",
    ("vup_fine", "mixed"): "fld::k_vup<float, true, false>",
    ("vup_fine", "mixed_tri"): "fld::k_vup<float, true, true>",
    ("vup_fine", "fp64"): "fld::k_vup<double, true, false>",
    ("vdown_fine", "mixed"): "fld::k_vdown<float, true>",
    ("vdown_fine", "fp64"): "fld::k_vdown<double, true>",
    ("update", "fp64"): "fld::k_update<0>",
    ("true_resid", "any"): "fld::k_true_resid",
    ("assemble", "any"): "fld::k_assemble",
    ("local", "mixed"): "fld::k_local",
    ("lmask", "mixed"): "fld::k_lmask",
}
PMC_SOURCES = {
    "fld_kernels.hip": ("spmv_px", "spmv_p", "update", "true_resid", "assemble", "local",
                        "lmask"),
    "fld_fused.hip": ("vup_fine", "vdown_fine"),
}


def traffic_records(pmc_dir, workload, root=ROOT):
    """Traffic records (the lines measured_traffic reads) from two rocprofv3
    counter runs in pmc_dir (FETCH_SIZE_counter_collection.csv and
    WRITE_SIZE_counter_collection.csv, KiB per dispatch), each scaled by what
    its counter reads for the copy probe of --copy-probe (2 GiB read, 2 GiB
    written): HBM bytes per launch, averaged over the kernel's dispatches."""
    import csv
    import hashlib
    per = {}
    for cn in ("FETCH_SIZE", "WRITE_SIZE"):
        acc = {}
        with open(os.path.join(pmc_dir, f"{cn}_counter_collection.csv")) as f:
            for row in csv.DictReader(f):
                acc.setdefault((row["Kernel_Name"], int(row["Grid_Size"])), []).append(
                    float(row["Counter_Value"]))
        per[cn] = acc
    probe = [k for k in per["FETCH_SIZE"]
             if "CUDAFunctorOnSelf_add" in k[0] and k[1] == 1 << 26]
    if not probe:
        raise RuntimeError("no copy-probe dispatch in the counter runs")
    scale = {cn: 2.0 * (1 << 20) / per[cn][probe[0]][0] for cn in per}

    def avg(cn, name):
        v = [x for (k, _), xs in per[cn].items() if k.split("(")[0].replace("void ", "") == name
             for x in xs]
        return sum(v) / len(v) if v else None

    def digest(rel):
        with open(os.path.join(root, rel), "rb") as f:
            return hashlib.sha256(f.read()).hexdigest()

    lines = []
    for (kernel, form), names in PMC_KERNELS.items():
        for name in (names if isinstance(names, tuple) else (names,)):
            fa, wa = avg("FETCH_SIZE", name), avg("WRITE_SIZE", name)
            if fa is not None and wa is not None:
                break
        if fa is None or wa is None:
            continue
        src = next(f for f, ks in PMC_SOURCES.items() if kernel in ks)
        rels = [f"paper_1306_0645_amd/csrc/{src}", "paper_1306_0645_amd/csrc/fld_device.h",
                "paper_1306_0645_amd/csrc/fld_internal.h"]
        nbytes = 1024.0 * (fa * scale["FETCH_SIZE"] + wa * scale["WRITE_SIZE"])
        lines.append(f"traffic-record: kernel={kernel} form={form} workload={workload} "
                     f"bytes_per_launch={nbytes:.0f} sources="
                     + ",".join(f"{r}:{digest(r)}" for r in rels))
    return scale, lines


def copy_bandwidth(torch, n=1 << 27, reps=5):
    """Measured HBM bandwidth of a plain streaming kernel (y = x + 0 over n
    doubles: n*8 bytes read and written), best of reps, for context beside
    the vendor peak."""
    x = torch.ones(n, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    best = float("inf")
    for _ in range(reps + 1):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        torch.add(x, 0.0, out=y)
        b.record()
        b.synchronize()
        best = min(best, a.elapsed_time(b) * 1e-3)
    del x, y
    return 2 * n * 8 / best / 1e9


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None,
                    help="timed steps (default: 20 for the reionization share, "
                         "10 for the other step workloads)")
    ap.add_argument("--warmup", type=int, default=2,
                    help="untimed steps on a separate handle before the timed run")
    ap.add_argument("--n", type=int, default=None, help="grid extent")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-secondary", action="store_true",
                    help="reionization: skip the 256^3 and 32^3 secondary runs")
    ap.add_argument("--no-parity", action="store_true",
                    help="reionization: skip the oracle's residual of each form")
    ap.add_argument("--forms", default="mixed,mixed_dir32,fp64")
    ap.add_argument("--direction-fp64", type=int, default=1,
                    help="mixed form: 1 keeps the PCG search direction in FP64, "
                         "0 rounds it to FP32 at a per-problem scale")
    ap.add_argument("--tile-z", type=int, default=0)
    ap.add_argument("--graph", type=int, default=1)
    ap.add_argument("--fused-tile-z", type=int, default=0)
    ap.add_argument("--warm-start", type=int, default=None,
                    help="start each step's PCG from the previous dEs: 0 off, "
                         "1 extrapolated, 2 Galerkin projection (default: 2, "
                         "or 1 for the batch and the Strömgren sweeps)")
    ap.add_argument("--check-every", type=int, default=0,
                    help="PCG iterations between host convergence reads "
                         "(0: automatic)")
    ap.add_argument("--tail-cells", type=int, default=512,
                    help="coarse levels of at most this many cells run in "
                         "one workgroup per V-cycle")
    ap.add_argument("--fused-levels", type=int, default=0,
                    help="levels run by the fused V(1,1) passes (0: automatic)")
    ap.add_argument("--smoother", type=int, default=0,
                    help="multigrid smoother: 0 red/black Gauss-Seidel, "
                         "1 weighted Jacobi")
    ap.add_argument("--cycle-switch", type=int, default=12,
                    help="iterations above which a V(1,1) handle switches cycle")
    ap.add_argument("--prolongation", type=int, default=2,
                    help="mixed cycle: 0 constant, 1 trilinear, 2 automatic")
    ap.add_argument("--coarse-op", type=int, default=0,
                    help="coarse faces: 0 sum of the fine faces, 1 rows in series")
    ap.add_argument("--local-sweeps", type=int, default=None,
                    help="mixed fused cycle: extra sweeps over the strongly "
                         "coupled finest cells (default: the library's)")
    ap.add_argument("--local-coupling", type=float, default=None,
                    help="threshold of the local-sweep mask (default: the library's)")
    ap.add_argument("--workload", default="reionization",
                    choices=["reionization", "many_sources", "single_source",
                             "batch", "served", "hii_test1", "multigroup",
                             "cosmo_test2"])
    ap.add_argument("--reps", type=int, default=300,
                    help="single_source: timed solves for the latency quantiles")
    ap.add_argument("--batch", type=int, default=96, help="batch: problems")
    ap.add_argument("--autotune", type=int, default=1)
    ap.add_argument("--requests", type=int, default=500, help="served: requests")
    ap.add_argument("--load", type=float, default=0.7,
                    help="served: arrival rate as a fraction of saturation")
    ap.add_argument("--groups", type=int, default=4, help="multigroup: groups")
    ap.add_argument("--hii-meshes", default="16,32,64",
                    help="hii_test1: octant meshes")
    ap.add_argument("--hii-taus", default="1e-2,1e-3,1e-4",
                    help="hii_test1: step tolerances")
    ap.add_argument("--hii-t-end", type=float, default=500.0,
                    help="hii_test1: end time [Myr]")
    ap.add_argument("--hii-cap-s", type=float, default=60.0,
                    help="hii_test1: wall-clock cap per run [s]")
    ap.add_argument("--hii-precision", default="mixed")
    ap.add_argument("--traffic-records", default=None, metavar="PMC_DIR",
                    help="print the traffic records of two rocprofv3 counter "
                         "runs (FETCH_SIZE, WRITE_SIZE) in PMC_DIR for the "
                         "workload named by --record-workload, and exit")
    ap.add_argument("--record-workload", default="reionization_share_640")
    ap.add_argument("--copy-probe", action="store_true",
                    help="first run a plain copy kernel of 2 GiB read + 2 GiB "
                         "written, to calibrate the HBM byte counters")
    return ap.parse_args()


def form_params(fld, p, prec, args, **kw):
    """Library parameters of a form: the paper's defaults with the bench's
    switches."""
    base = dict(precision=prec, tile_z=args.tile_z, use_graph=args.graph,
                fused_tile_z=args.fused_tile_z, warm_start=args.warm_start,
                prolongation=args.prolongation, tail_cells=args.tail_cells,
                smoother=args.smoother, fused_levels=args.fused_levels,
                check_every=args.check_every, cycle_switch=args.cycle_switch,
                coarse_op=args.coarse_op,
                direction_fp64=args.direction_fp64 if prec else 0)
    if args.local_sweeps is not None:
        base["local_sweeps"] = args.local_sweeps
    if args.local_coupling is not None:
        base["local_coupling"] = args.local_coupling
    base.update(kw)
    return fld.fld_default_params(p["c"], p["L_unit"], **base)


def host_cpu():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def time_steps(fld, torch, p, prm, steps, warmup):
    """`warmup` untimed steps on a handle of their own from E^0, then a
    fresh handle times `steps` successive steps from E^0 (the limiter
    recomputed each step).  Returns the handle (still open), E after the
    timed steps, and the per-step records."""
    E0 = p["E"]
    K, H = p["kappa"], p["eta"]
    if warmup > 0:
        W = fld.Solver(p["shape"], p["h"], prm)
        Ew = E0.clone()
        for _ in range(warmup):
            W.step(Ew, K, H, p["dt"])
        W.close()
        del W, Ew
        torch.cuda.empty_cache()
    S = fld.Solver(p["shape"], p["h"], prm)
    E = E0.clone()
    torch.cuda.synchronize()
    lat, recs = [], []
    t0 = time.perf_counter()
    for k in range(steps):
        ta = time.perf_counter()
        st = S.step(E, K, H, p["dt"])  # returns once the step is decided
        lat.append(time.perf_counter() - ta)
        recs.append(st)
    torch.cuda.synchronize()
    sec = time.perf_counter() - t0
    return S, E, recs, lat, sec


def kernel_pass(fld, torch, p, prm, E, steps, prec_idx, dir64):
    """Per-kernel timing on a handle without graph replay (a replayed graph
    hides its kernels from the timing hook), reading the convergence state
    after every iteration so that no launch of a converged problem enters
    the averages: survey one step with every kernel timed, then time the
    dominant kernel's launches over `steps` steps with hipEvents on the
    handle's stream."""
    names = fld.profile_kernels()
    P = fld.Solver(p["shape"], p["h"], prm)
    Ek = E.clone()
    P.step(Ek, p["kappa"], p["eta"], p["dt"])
    fld.fld_profile_select(-2)
    st_survey = P.step(Ek, p["kappa"], p["eta"], p["dt"])
    torch.cuda.synchronize()
    reads = {n: fld.fld_profile_read(k) for k, n in enumerate(names)}
    totals = {n: r[0] for n, r in reads.items()}
    counts = {n: r[1] for n, r in reads.items()}
    dom = max((n for n in totals if n in BYTES_PER_CELL), key=lambda n: totals[n])
    dom_id = names.index(dom)
    fld.fld_profile_select(dom_id)
    torch.cuda.synchronize()
    for _ in range(steps):
        P.step(Ek, p["kappa"], p["eta"], p["dt"])
    torch.cuda.synchronize()
    ms_total, launches = fld.fld_profile_read(dom_id)
    fld.fld_profile_select(-1)
    P.close()
    del Ek
    cells = int(E.numel())
    avg_ms = ms_total / max(launches, 1)
    b = bpc(dom, prec_idx, dir64)
    fixed_b, iter_b = step_bytes(counts, cells, prec_idx, st_survey["levels"], dir64)
    return {"dominant": dom, "dominant_avg_ms": avg_ms, "dominant_launches": launches,
            "dominant_bytes_per_cell": b,
            "dominant_GBps": b * cells / (avg_ms * 1e-3) / 1e9,
            "survey_ms": {k: round(v, 4) for k, v in sorted(
                totals.items(), key=lambda kv: -kv[1]) if v > 0},
            "survey_iters": st_survey["iters"], "_fixed_b": fixed_b, "_iter_b": iter_b}


def oracle_residual(p, E_before, dE, parallel=True, chunk=1 << 24):
    """The oracle's residual b - A dE at every cell, each computed on its own
    from the oracle's limiter and operator, in chunks: returns the relative
    residual ||b - A dE|| / ||b|| and the error bound ||b - A dE|| / ||dE||
    (||A^-1||_2 <= 1 when adot >= 0, so this bounds the relative error
    against the exact step).  The parallel build evaluates each cell with the
    same arithmetic as the serial one."""
    import numpy as np

    import oracle
    En = E_before.detach().cpu().numpy()
    Kh = p["kappa"].detach().cpu().numpy()
    Hh = p["eta"].detach().cpu().numpy()
    dEh = dE.detach().cpu().numpy()
    dmax, rmin = oracle.limits(p["c"], p["L_unit"])
    O = oracle.Problem(En, Kh, Hh, p["h"], p["c"], dmax, rmin, p["dt"], parallel=parallel)
    n = En.size
    rr = bb = 0.0
    for a in range(0, n, chunk):
        cells = np.arange(a, min(n, a + chunk), dtype=np.int64)
        res, rhs = O.residual_at(dEh, cells)
        rr += float(np.dot(res, res))
        bb += float(np.dot(rhs, rhs))
    dd = float(np.dot(dEh.ravel(), dEh.ravel()))
    return {"true_rel_resid": math.sqrt(rr / bb) if bb > 0 else 0.0,
            "err_bound": math.sqrt(rr / dd) if dd > 0 else 0.0,
            "cells_checked": int(n)}


def run_form_headline(fld, torch, p, name, args, steps, levels=6):
    prec = fld.FLD_PREC_MIXED if name.startswith("mixed") else fld.FLD_PREC_FP64
    dir64 = bool(args.direction_fp64) if prec else False
    if name == "mixed_dir32":
        dir64 = False
    elif name == "mixed_dir64":
        dir64 = True
    prm = form_params(fld, p, prec, args, mg_levels=levels,
                      direction_fp64=int(dir64) if prec else 0)
    log(f"[bench] form {name}: {args.warmup} warm-up + {steps} timed steps from E^0")
    S, E, recs, lat, sec = time_steps(fld, torch, p, prm, steps, args.warmup)
    for k in range(0, steps, 5):
        log(f"[bench]   step {k + 1}: {recs[k]['iters']} iterations, "
            f"{1e3 * lat[k]:.1f} ms")
    import numpy as np
    cells = int(E.numel())
    iters = [r["iters"] for r in recs]
    rels = [r["rel_resid"] for r in recs]
    assert all(r["status"] == 0 for r in recs), [r["status"] for r in recs]
    out = {"mcell_updates_per_s": cells * steps / sec / 1e6,
           "ms_per_step": 1e3 * sec / steps,
           "latency_ms": {"p50": float(np.percentile(np.array(lat) * 1e3, 50)),
                          "p99": float(np.percentile(np.array(lat) * 1e3, 99)),
                          "mean": float(np.mean(lat) * 1e3),
                          "max": float(np.max(lat) * 1e3)},
           "iters_per_step": float(np.mean(iters)), "iters": iters,
           "max_rel_resid": float(max(rels)),
           "max_err_bound": float(max(r["err_bound"] for r in recs)),
           "restarts": int(sum(r["restarts"] for r in recs)),
           "final_cycle": {"nu": recs[-1]["cycle_nu"], "trilinear": recs[-1]["trilinear"]},
           "direction": "fp64" if (dir64 or not prec) else "fp32"}
    if not args.no_parity:
        # one more step of the same handle (its warm start and cycle), checked
        # by the oracle at every cell
        Eb = E.clone()
        st = S.step(E, p["kappa"], p["eta"], p["dt"])
        dE = E - Eb
        torch.cuda.synchronize()
        log(f"[bench]   oracle residual of step {steps + 1} at every cell")
        par = oracle_residual(p, Eb, dE)
        par["solver_rel_resid"] = st["rel_resid"]
        par["step"] = steps + 1
        out["parity"] = par
        del Eb, dE
    S.close()
    del S
    torch.cuda.empty_cache()
    nu, tri = recs[-1]["cycle_nu"], recs[-1]["trilinear"]
    kprm = form_params(fld, p, prec, args, mg_levels=levels, use_graph=0, check_every=1,
                       cycle_switch=0, nu_pre=nu, nu_post=nu, prolongation=tri,
                       direction_fp64=int(dir64) if prec else 0)
    prec_idx = 1 if prec else 0
    kp = kernel_pass(fld, torch, p, kprm, E, 2, prec_idx, dir64)
    it_mean = out["iters_per_step"]
    sb = kp.pop("_fixed_b") + kp.pop("_iter_b") / max(kp["survey_iters"], 1) * it_mean
    out.update(kp)
    out["step_bytes_per_cell"] = sb / cells
    out["step_GBps"] = sb * steps / sec / 1e9
    del E
    torch.cuda.empty_cache()
    return out


def _oracle_problem(p, parallel):
    import oracle
    En = p["E"].detach().cpu().numpy()
    Kh = p["kappa"].detach().cpu().numpy()
    Hh = p["eta"].detach().cpu().numpy()
    dmax, rmin = oracle.limits(p["c"], p["L_unit"])
    return oracle.Problem(En, Kh, Hh, p["h"], p["c"], dmax, rmin, p["dt"],
                          parallel=parallel)


def recorded_oracle_iterations(n):
    path = os.path.join(ROOT, "oracle", f"reionization_{n}_iterations.txt")
    try:
        with open(path) as f:
            for line in f:
                if line.startswith("step1_iterations"):
                    return int(line.split("=", 1)[1])
    except OSError:
        pass
    return None


def cpu_baselines(p, args):
    """The oracle on the host cores, on step 1 of the workload (its E^0).
    All cores (the host share of one GPU, 16 threads, through the OpenMP
    build of the same source): the whole step, limiter assembly and
    Jacobi-PCG to the same 1e-8 rule.  One core (the serial build): the
    assembly and the first one and two iterations are timed, and the step is
    extrapolated to the iteration count of the all-cores solve (or, without
    it, to the count recorded by oracle/record_iterations.py)."""
    import oracle
    n = p["shape"][0]
    cells = int(p["E"].numel())
    cpu = host_cpu()
    out = {}
    thr = min(16, os.cpu_count() or 1)
    used = oracle.threads(thr)
    log(f"[bench] the oracle's step 1 on {used} threads, to 1e-8")
    O = _oracle_problem(p, True)
    t0 = time.perf_counter()
    _, st, it_all, rel = O.solve(tol=1e-8, max_iter=100000)
    sec = time.perf_counter() - t0
    del O
    out["all"] = {"value": round(cells / sec / 1e6, 4), "unit": "Mcell-updates/s",
                  "cores": used, "kind": "oracle", "host_cpu": cpu,
                  "sample": (f"step 1 of the {n}^3 share (E^0): the oracle's limiter "
                             f"assembly and Jacobi-PCG to 1e-8 ({it_all} iterations, "
                             f"relative residual {rel:.2e}) in {sec:.1f} s on {used} "
                             "threads (OpenMP build of the oracle)"),
                  "status": int(st), "seconds": round(sec, 2), "iterations": int(it_all)}
    need = it_all if st == oracle.OK else recorded_oracle_iterations(n)
    log("[bench] the oracle's step 1 on one thread: assembly + 1 and 3 iterations")
    O = _oracle_problem(p, False)
    t0 = time.perf_counter()
    O.solve(tol=1e-8, max_iter=1)
    t1 = time.perf_counter() - t0
    t0 = time.perf_counter()
    O.solve(tol=1e-8, max_iter=3)
    t3 = time.perf_counter() - t0
    del O
    t_it = max(t3 - t1, 0.0) / 2.0
    t_asm = max(t1 - t_it, 0.0)
    rec = {"unit": "Mcell-updates/s", "cores": 1, "kind": "oracle", "host_cpu": cpu,
           "assembly_s": round(t_asm, 3), "s_per_iteration": round(t_it, 4)}
    if need:
        t_step = t_asm + need * t_it
        rec["value"] = round(cells / t_step / 1e6, 4)
        rec["sample"] = (f"step 1 of the {n}^3 share on one thread (serial build): "
                         f"the assembly ({t_asm:.1f} s) and the per-iteration time "
                         f"({t_it:.2f} s, from runs of 1 and 3 Jacobi-PCG "
                         f"iterations) timed, the step extrapolated to the {need} "
                         f"iterations of its 1e-8 solve: {t_step:.0f} s")
        rec["extrapolated"] = True
    else:
        rec["value"] = None
        rec["sample"] = "no oracle iteration count for this grid"
    out["single"] = rec
    return out


def secondary(fld, torch, synth, args):
    """The 256^3 many-source workload (10 steps from its initial state, both
    forms) and the 32^3 single-source latency (FP64 V(2,2), >= 200 reps)."""
    import numpy as np
    res = {}
    p = synth.many_sources(256)
    q = dict(p)
    for k in ("E", "kappa", "eta"):
        q[k] = torch.from_numpy(p[k]).cuda()
    c2 = {}
    for name, prec in (("mixed", fld.FLD_PREC_MIXED), ("fp64", fld.FLD_PREC_FP64)):
        prm = form_params(fld, q, prec, args)
        S, E, recs, lat, sec = time_steps(fld, torch, q, prm, 10, args.warmup)
        S.close()
        c2[name] = {"mcell_updates_per_s": round(256 ** 3 * 10 / sec / 1e6, 2),
                    "ms_per_step": round(1e3 * sec / 10, 3),
                    "latency_ms": {"p50": round(float(np.percentile(np.array(lat) * 1e3, 50)), 3),
                                   "p99": round(float(np.percentile(np.array(lat) * 1e3, 99)), 3)},
                    "iters_per_step": float(np.mean([r["iters"] for r in recs])),
                    "max_rel_resid": float(max(r["rel_resid"] for r in recs))}
        log(f"[bench] secondary many_sources_256^3 {name}: {c2[name]}")
        del S, E
    res["many_sources_256^3"] = c2
    del q
    torch.cuda.empty_cache()
    p = synth.single_source(32)
    prm = fld.fld_default_params(p["c"], p["L_unit"], mg_levels=4, nu_pre=2, nu_post=2,
                                 use_graph=args.graph, warm_start=1)
    S = fld.Solver(p["shape"], p["h"], prm)
    E0 = torch.from_numpy(p["E"]).cuda()
    K = torch.from_numpy(p["kappa"]).cuda()
    H = torch.from_numpy(p["eta"]).cuda()
    E = E0.clone()
    lat, rel = [], []
    for r in range(args.warmup + max(args.reps, 200)):
        E.copy_(E0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st = S.step(E, K, H, p["dt"])
        t1 = time.perf_counter()
        if r >= args.warmup:
            lat.append(t1 - t0)
            rel.append(st["rel_resid"])
    S.close()
    lat_ms = np.array(lat) * 1e3
    res["single_source_32^3"] = {
        "precision": "fp64", "cycle": "V(2,2)", "levels": 4, "reps": len(lat),
        "latency_ms": {"p50": round(float(np.percentile(lat_ms, 50)), 4),
                       "p99": round(float(np.percentile(lat_ms, 99)), 4)},
        "mcell_updates_per_s": round(32 ** 3 / float(np.mean(lat)) / 1e6, 2),
        "max_rel_resid": float(max(rel))}
    log(f"[bench] secondary single_source_32^3: {res['single_source_32^3']}")
    return res


def copy_probe(torch):
    """Calibration kernel of the byte-counter runs: y = x + 0 over 2^28
    doubles, one kernel reading 2 GiB and writing 2 GiB."""
    x = torch.ones(1 << 28, dtype=torch.float64, device="cuda")
    y = x.add(0.0)
    torch.cuda.synchronize()
    del x, y


def headline(args, fld, torch, synth):
    n = args.n or 640
    steps = args.steps or 20
    if args.copy_probe:
        copy_probe(torch)
    log(f"[bench] generating the {n}^3 reionization share on the GPU")
    t0 = time.perf_counter()
    p = synth.t_reionization_share(n=n, n_src=int(round(10000 * (n / 640) ** 3)),
                                   device="cuda")
    torch.cuda.synchronize()
    log(f"[bench]   generated in {time.perf_counter() - t0:.1f} s; ionized "
        f"(x_HI = 1e-4) volume {p['ionized_fraction']:.4f}")
    cpu = None
    if not args.no_cpu_baseline and not args.copy_probe:
        cpu = cpu_baselines(p, args)
    forms = {}
    for name in args.forms.split(","):
        forms[name] = run_form_headline(fld, torch, p, name, args, steps)
        log(f"[bench] {name}: " + json.dumps(
            {k: v for k, v in forms[name].items() if k not in ("survey_ms",)}))
    head = forms.get("mixed") or forms[list(forms)[0]]
    head_name = "mixed" if "mixed" in forms else list(forms)[0]
    copy_bw = copy_bandwidth(torch)
    log(f"[bench] streaming copy: {copy_bw:.0f} GB/s")
    wl = f"reionization_share_{n}"
    tform = "fp64" if head_name == "fp64" else (
        "mixed_dir64" if head["direction"] == "fp64" else "mixed")
    roof = {
        "bound": "hbm",
        "kernel": head["dominant"],
        "achieved": round(head["dominant_GBps"], 1),
        "peak": HBM_PEAK_GBS,
        "unit": "GB/s",
        "frac": round(head["dominant_GBps"] / HBM_PEAK_GBS, 4),
        "traffic": measured_traffic(head["dominant"], tform, wl),
        "bytes_per_cell": head["dominant_bytes_per_cell"],
        "avg_launch_ms": round(head["dominant_avg_ms"], 4),
    }
    sec = None if args.no_secondary else secondary(fld, torch, synth, args)
    fp64 = forms.get("fp64")
    out = {
        "metric": "FLD solve Mcell-updates/s + % HBM roofline at 1e-8 residual; "
                  "p50/p99 solve latency",
        "value": round(head["mcell_updates_per_s"], 2),
        "unit": "Mcell-updates/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": args.warmup,
        "ms_per_step": round(head["ms_per_step"], 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64+f32" if head_name.startswith("mixed") else "f64",
        "data": "synthetic",
        "config": {"workload": f"reionization_share_{n}^3", "grid": [n] * 3,
                   "sources": int(round(10000 * (n / 640) ** 3)), "sigma_ln": 2.0,
                   "levels": 6, "rtol": 1e-8, "precision": head_name,
                   "direction": head["direction"],
                   "start": "E^0 = 1e-45 erg/cm^3, all steps timed",
                   "warm_start": ("off", "extrapolated", "galerkin")[args.warm_start],
                   "steps_per_run": steps},
        "latency_ms": {k: round(v, 3) for k, v in head["latency_ms"].items()},
        "roofline": roof,
        "step_roofline": {
            "bytes_per_cell": round(head["step_bytes_per_cell"], 1),
            "achieved": round(head["step_GBps"], 1), "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": round(head["step_GBps"] / HBM_PEAK_GBS, 4)},
        "hbm_copy_GBps": round(copy_bw, 1),
        "cpu_baseline": cpu["all"] if cpu else None,
        "cpu_baseline_single_core": cpu["single"] if cpu else None,
        "speedup_vs_fp64": (round(head["mcell_updates_per_s"] / fp64["mcell_updates_per_s"], 3)
                            if fp64 and head is not fp64 else None),
        "forms": {k: {kk: (round(vv, 4) if isinstance(vv, float) and "resid" not in kk
                           and "bound" not in kk else vv)
                      for kk, vv in v.items()} for k, v in forms.items()},
        "secondary": sec,
    }
    return out


def main():
    args = parse()
    if args.traffic_records:
        scale, lines = traffic_records(args.traffic_records, args.record_workload)
        print(f"# scales: FETCH_SIZE x {scale['FETCH_SIZE']:.3f}, "
              f"WRITE_SIZE x {scale['WRITE_SIZE']:.3f}")
        print("\n".join(lines))
        return
    if args.warm_start is None:
        # the Galerkin guess (the library default) where it measured faster;
        # the extrapolation for the single source and the batch (1 and about
        # 1.45 iterations a step leave no room for the guess's extra pass)
        # and for the Stromgren sweeps (slowly drifting fronts, where it took
        # fewer iterations)
        args.warm_start = 1 if args.workload in ("single_source", "batch",
                                                 "hii_test1", "cosmo_test2") else 2
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); this build "
              "has no multi-GPU path", file=sys.stderr)
        sys.exit(2)
    import torch

    import paper_1306_0645_amd as fld
    import synth

    if args.workload == "reionization":
        out = headline(args, fld, torch, synth)
    else:
        import bench_workloads
        if args.steps is None:
            args.steps = 10
        if args.n is None:
            args.n = 256
        out = getattr(bench_workloads, args.workload)(args, fld, torch, synth, log)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
