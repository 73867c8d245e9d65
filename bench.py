#!/usr/bin/env python3
"""Benchmark of the implicit grey FLD step on one MI355X.

Default workload: 256^3 periodic grid, lognormal HI opacity (sigma_ln 1.5),
64 point sources (Ndot log-uniform 1e47-1e50), smooth random E^n, dt = 1e-3
light-crossing times, successive timesteps with the limiter recomputed from
the new E each step, PCG + geometric multigrid to a 1e-8 relative residual.
A "step" is one full timestep: assembly of the limiter system and every
multigrid level, the preconditioned CG solve, and E += dE.

Prints ONE JSON line: Mcell-updates/s of the mixed-precision form (the FP64
form is reported beside it), the roofline of the dominant kernel timed live
with hipEvents, and the oracle's CPU throughput on a bounded sample.
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
    # trilinear mixed cycle: level 1's correction interpolated to every finest
    # cell (coarse values at 1/8, FP32 out); the up pass then reads it at the
    # red cells (2 B/cell, not counted in vup_fine's 32.5)
    "tri_fine": (0.0, 4.5),
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


def step_bytes(counts, cells, prec_idx, levels):
    """Algorithmic bytes of one step from the launches counted in a survey
    step, split into (per step, per PCG iteration x iterations): finest-level
    kernels exactly, coarse levels from their share of cells."""
    fixed = it = 0.0
    for name, count in counts.items():
        if name in BYTES_PER_CELL:
            v = count * BYTES_PER_CELL[name][prec_idx] * cells
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


def model_step_bytes(cells, iters, nu, prec_idx, levels, steps=1, warm=False):
    # warm: 0/False cold, 1 extrapolated guess, 2 or True Galerkin guess (the
    # library default)
    """Algorithmic bytes of `steps` steps of one problem taking `iters` PCG
    iterations in all, from the cycle structure:
    assembly and coarse operators, the true-residual check and E += dE once,
    then per PCG iteration one V(nu,nu) cycle (fused finest-level passes for
    nu = 1), the SpMV and the vector update."""
    B = {k: v[prec_idx] for k, v in BYTES_PER_CELL.items()}
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


def measured_traffic(kernel, form, root=ROOT):
    """HBM bytes per launch of `kernel` from the rocprofv3 byte-counter
    records under root/profiles/, or None when there is no record or any
    source the record names (relative to root) has changed since the
    counters were taken."""
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
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=256, help="grid extent")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--forms", default="fp64,mixed")
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
    ap.add_argument("--workload", default="many_sources",
                    choices=["many_sources", "single_source", "reionization",
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
    ap.add_argument("--copy-probe", action="store_true",
                    help="first run a plain copy kernel of 2 GiB read + 2 GiB "
                         "written, to calibrate the HBM byte counters")
    return ap.parse_args()


def run_form(fld, torch, p, prec, steps, warmup, args):
    """Timed steps with graph replay (the throughput), then the same number of
    steps with per-kernel launches so hipEvents can time the dominant kernel
    on its stream (a graph replay hides its kernels from the timing hook)."""
    E = torch.from_numpy(p["E"]).cuda()
    kap = torch.from_numpy(p["kappa"]).cuda()
    eta = torch.from_numpy(p["eta"]).cuda()
    names = fld.profile_kernels()

    def solver(graph):
        # the kernel-timing pass reads the convergence state after every
        # iteration, so no launch of a converged problem (which returns at
        # once) enters the per-launch average
        prm = fld.fld_default_params(p["c"], p["L_unit"], precision=prec,
                                     tile_z=args.tile_z, use_graph=graph,
                                     fused_tile_z=args.fused_tile_z,
                                     warm_start=args.warm_start,
                                     prolongation=args.prolongation,
                                     tail_cells=args.tail_cells,
                                     smoother=args.smoother,
                                     fused_levels=args.fused_levels,
                                     check_every=args.check_every if graph else 1)
        return fld.Solver(p["shape"], p["h"], prm)

    S = solver(args.graph)
    for w in range(max(1, warmup)):
        S.step(E, kap, eta, p["dt"])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    iters, rels = [], []
    for _ in range(steps):
        st = S.step(E, kap, eta, p["dt"])
        iters.append(st["iters"])
        rels.append(st["rel_resid"])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    S.close()
    # kernel timing pass: survey one step, then time the dominant kernel
    P = solver(0)
    P.step(E, kap, eta, p["dt"])
    fld.fld_profile_select(-2)
    st_survey = P.step(E, kap, eta, p["dt"])
    torch.cuda.synchronize()
    reads = {n: fld.fld_profile_read(k) for k, n in enumerate(names)}
    totals = {n: r[0] for n, r in reads.items()}
    counts = {n: r[1] for n, r in reads.items()}
    dom = max((n for n in totals if n in BYTES_PER_CELL), key=lambda n: totals[n])
    dom_id = names.index(dom)
    fld.fld_profile_select(dom_id)
    torch.cuda.synchronize()
    tp0 = time.perf_counter()
    for _ in range(steps):
        P.step(E, kap, eta, p["dt"])
    torch.cuda.synchronize()
    tp1 = time.perf_counter()
    ms_total, launches = fld.fld_profile_read(dom_id)
    fld.fld_profile_select(-1)
    P.close()
    cells = p["E"].size
    sec = t1 - t0
    avg_ms = ms_total / max(launches, 1)
    bpc = BYTES_PER_CELL[dom][1 if prec == fld.FLD_PREC_MIXED else 0]
    achieved = bpc * cells / (avg_ms * 1e-3) / 1e9
    prec_idx = 1 if prec == fld.FLD_PREC_MIXED else 0
    # whole-step algorithmic bytes, scaled from the survey step's iteration
    # count to the timed steps' mean
    fixed_b, iter_b = step_bytes(counts, cells, prec_idx, st_survey["levels"])
    it_mean = sum(iters) / len(iters)
    sb = fixed_b + iter_b / max(st_survey["iters"], 1) * it_mean
    return {
        "mcell_updates_per_s": cells * steps / sec / 1e6,
        "ms_per_step": 1e3 * sec / steps,
        "ms_per_step_unfused_launches": 1e3 * (tp1 - tp0) / steps,
        "iters_per_step": sum(iters) / len(iters),
        "max_rel_resid": max(rels),
        "survey_ms": {k: round(v, 4) for k, v in sorted(
            totals.items(), key=lambda kv: -kv[1]) if v > 0},
        "dominant": dom,
        "dominant_avg_ms": avg_ms,
        "dominant_launches": launches,
        "dominant_GBps": achieved,
        "dominant_bytes_per_cell": bpc,
        "step_bytes_per_cell": sb / cells,
        "step_GBps": sb * steps / sec / 1e9,
    }


def cpu_baseline(p):
    import oracle
    dmax, rmin = oracle.limits(p["c"], p["L_unit"])
    O = oracle.Problem(p["E"], p["kappa"], p["eta"], p["h"], p["c"], dmax, rmin,
                       p["dt"], p["theta"], p["a"], p["adot"])
    t0 = time.perf_counter()
    _, st, it, rel = O.solve(tol=1e-8, max_iter=1000)
    sec = time.perf_counter() - t0
    cpu = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    cpu = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"value": p["E"].size / sec / 1e6, "unit": "Mcell-updates/s",
            "cores": 1, "kind": "oracle",
            "sample": f"one {p['shape'][0]}^3 step (limiter assembly + Jacobi-PCG "
                      f"to 1e-8, {it} iterations, {sec:.1f} s), single thread",
            "host_cpu": cpu, "host_threads": os.cpu_count()}


_CPU_PROBLEM = None


def _oracle_step_seconds(_):
    import oracle
    p = _CPU_PROBLEM
    dmax, rmin = oracle.limits(p["c"], p["L_unit"])
    O = oracle.Problem(p["E"], p["kappa"], p["eta"], p["h"], p["c"], dmax, rmin,
                       p["dt"], p["theta"], p["a"], p["adot"])
    t0 = time.perf_counter()
    O.solve(tol=1e-8, max_iter=1000)
    return time.perf_counter() - t0


def cpu_baseline_all_cores(p, procs):
    """The same oracle step solved by `procs` single-threaded processes at
    once, one per host core (the oracle itself is serial); forked before the
    GPU is touched.  Throughput = procs x cells / the slowest process."""
    import multiprocessing as mp
    global _CPU_PROBLEM
    _CPU_PROBLEM = p
    with mp.get_context("fork").Pool(procs) as pool:
        secs = pool.map(_oracle_step_seconds, range(procs))
    _CPU_PROBLEM = None
    return {"value": procs * p["E"].size / max(secs) / 1e6,
            "unit": "Mcell-updates/s", "cores": procs, "kind": "oracle",
            "sample": f"{procs} concurrent single-threaded solves of the same "
                      f"{p['shape'][0]}^3 step to 1e-8 ({max(secs):.1f} s for "
                      f"the slowest)"}


def main():
    args = parse()
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

    if args.workload != "many_sources":
        import bench_workloads
        out = getattr(bench_workloads, args.workload)(args, fld, torch, synth, log)
        print(json.dumps(out), flush=True)
        return

    if args.copy_probe:
        # y = x + 0 over 2^28 doubles: one kernel reading 2 GiB and writing 2 GiB
        x = torch.ones(1 << 28, dtype=torch.float64, device="cuda")
        y = x.add(0.0)
        torch.cuda.synchronize()
        del x, y
    log(f"[bench] generating the {args.n}^3 many-source workload")
    p = synth.many_sources(args.n)
    cpu_all = None
    if not args.no_cpu_baseline and not args.copy_probe:
        # the host share of one GPU is 16 cores, whatever os.cpu_count() says
        procs = max(1, min(16, os.cpu_count() or 1))
        log(f"[bench] timing the oracle on {procs} cores (before the GPU starts)")
        cpu_all = cpu_baseline_all_cores(p, procs)
    forms = {}
    for name in args.forms.split(","):
        prec = fld.FLD_PREC_MIXED if name == "mixed" else fld.FLD_PREC_FP64
        log(f"[bench] form {name}: {args.warmup} warmup + {args.steps} timed steps")
        forms[name] = run_form(fld, torch, p, prec, args.steps, args.warmup, args)
        log(f"[bench] {name}: {json.dumps(forms[name])}")
    head = forms.get("mixed") or forms[list(forms)[0]]
    copy_bw = copy_bandwidth(torch)
    log(f"[bench] streaming copy: {copy_bw:.0f} GB/s")
    cpu = None
    if not args.no_cpu_baseline:
        log("[bench] timing the oracle on one step")
        cpu = cpu_baseline(p)
    roof = {
        "bound": "hbm",
        "kernel": head["dominant"],
        "achieved": round(head["dominant_GBps"], 1),
        "peak": HBM_PEAK_GBS,
        "unit": "GB/s",
        "frac": round(head["dominant_GBps"] / HBM_PEAK_GBS, 4),
        "traffic": measured_traffic(head["dominant"],
                                    "mixed" if "mixed" in forms else "fp64"),
    }
    out = {
        "metric": "FLD solve Mcell-updates/s + % HBM roofline at 1e-8 residual; "
                  "p50/p99 solve latency",
        "value": round(head["mcell_updates_per_s"], 2),
        "unit": "Mcell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(head["ms_per_step"], 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64+f32" if "mixed" in forms else "f64",
        "data": "synthetic",
        "config": {"workload": f"many_sources_{args.n}^3", "grid": [args.n] * 3,
                   "sources": 64, "sigma_ln": 1.5, "rtol": 1e-8,
                   "precision": "mixed" if "mixed" in forms else "fp64",
                   "smoother": ("red/black Gauss-Seidel", "weighted Jacobi")[args.smoother],
                   "warm_start": ("off", "extrapolated",
                                  "galerkin")[args.warm_start],
                   "steps_per_run": args.steps},
        "roofline": roof,
        "step_roofline": {
            "bytes_per_cell": round(head["step_bytes_per_cell"], 1),
            "achieved": round(head["step_GBps"], 1), "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": round(head["step_GBps"] / HBM_PEAK_GBS, 4)},
        "hbm_copy_GBps": round(copy_bw, 1),
        "cpu_baseline": cpu,
        "cpu_baseline_all_cores": cpu_all,
        "forms": {k: {kk: (round(vv, 4) if isinstance(vv, float) else vv)
                      for kk, vv in v.items()} for k, v in forms.items()},
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
