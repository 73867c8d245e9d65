"""Workloads of bench.py beyond the default 640^3 reionization share.

many_sources   256^3, 64 sources, both forms, successive steps from the
               initial state, each form checked by the oracle at every cell
single_source  32^3, one source, FP64 V(2,2) 4 levels: latency p50/p99 of
               one step over many repetitions (fields cache-resident)
batch          96 independent problems of 32..128^3 in one batched step,
               autotuned, against the same problems solved one by one
served         Poisson stream of 64..384^3 requests of 1-5 steps through the
               continuous-batching server: p50/p99 latency and throughput
hii_test1      Test 1 end to end (radiation + hydrogen chemistry): I-front
               error, average step and run time over a tau_tol sweep
multigroup     G frequency groups on one 256^3 mesh stepped together,
               against the same groups one by one
cosmo_test2    Test 2 end to end (comoving, Einstein-de Sitter): error
               against the Shapiro-Giroux front over a tau_tol sweep

Each function returns the JSON object bench.py prints.
"""
import json
import math
import time

import numpy as np

HBM_PEAK_GBS = 8000.0


def _base(metric_note, value, ms, steps, warmup, dtype, config, roofline=None,
          extra=None):
    out = {
        "metric": "FLD solve Mcell-updates/s + % HBM roofline at 1e-8 residual; "
                  "p50/p99 solve latency",
        "value": round(value, 2),
        "unit": "Mcell-updates/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": warmup,
        "ms_per_step": round(ms, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": dtype,
        "data": "synthetic",
        "config": config,
        "roofline": roofline,
        "cpu_baseline": None,
        "note": metric_note,
    }
    if extra:
        out.update(extra)
    return out


def _dominant(fld, names, totals, cells, bytes_table, prec_idx):
    cand = [n for n in totals if n in bytes_table and totals[n] > 0]
    if not cand:
        return None
    return max(cand, key=lambda n: totals[n])


def _survey(fld, fn):
    """Run fn() once with every kernel timed; return {kernel: total ms}."""
    names = fld.profile_kernels()
    fld.fld_profile_select(-2)
    fn()
    import torch
    torch.cuda.synchronize()
    totals = {n: fld.fld_profile_read(k)[0] for k, n in enumerate(names)}
    fld.fld_profile_select(-1)
    return names, totals


def single_source(args, fld, torch, synth, log):
    from bench import BYTES_PER_CELL
    p = synth.single_source(32)
    prm = fld.fld_default_params(p["c"], p["L_unit"], mg_levels=4, nu_pre=2,
                                 nu_post=2, use_graph=args.graph,
                                 warm_start=args.warm_start)
    S = fld.Solver(p["shape"], p["h"], prm)
    E0 = torch.from_numpy(p["E"]).cuda()
    K = torch.from_numpy(p["kappa"]).cuda()
    H = torch.from_numpy(p["eta"]).cuda()
    E = E0.clone()
    lat, iters, rel = [], [], []
    reps = max(args.reps, 200)
    log(f"[bench] single_source 32^3: {args.warmup} warmup + {reps} timed steps")
    for r in range(args.warmup + reps):
        E.copy_(E0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st = S.step(E, K, H, p["dt"])
        t1 = time.perf_counter()
        if r >= args.warmup:
            lat.append(t1 - t0)
            iters.append(st["iters"])
            rel.append(st["rel_resid"])
    names, totals = _survey(fld, lambda: (E.copy_(E0), S.step(E, K, H, p["dt"])))
    dom = _dominant(fld, names, totals, E.numel(), BYTES_PER_CELL, 0)
    lat_ms = np.array(lat) * 1e3
    p50, p99 = np.percentile(lat_ms, [50, 99])
    mean_s = float(np.mean(lat))
    cells = E.numel()
    return _base(
        "32^3 fields are cache-resident; the HBM roofline does not apply",
        cells / mean_s / 1e6, mean_s * 1e3, reps, args.warmup, "f64",
        {"workload": "single_source_32^3", "grid": [32, 32, 32], "sources": 1,
         "precision": "fp64", "levels": 4, "cycle": "V(2,2)", "rtol": 1e-8},
        None,
        {"latency_ms": {"p50": round(float(p50), 4), "p99": round(float(p99), 4),
                        "mean": round(float(lat_ms.mean()), 4)},
         "iters_per_step": float(np.mean(iters)), "max_rel_resid": max(rel),
         "survey_ms": {k: round(v, 4) for k, v in sorted(
             totals.items(), key=lambda kv: -kv[1]) if v > 0},
         "dominant": dom})


def many_sources(args, fld, torch, synth, log):
    """The 256^3 many-source workload: 64 sources, sigma_ln 1.5, smooth E^n,
    `steps` successive steps from the initial state in both forms, each
    form's extra step checked by the oracle at every cell."""
    import bench
    n = args.n
    if args.copy_probe:
        bench.copy_probe(torch)
    log(f"[bench] generating the {n}^3 many-source workload")
    p = synth.many_sources(n)
    q = dict(p)
    for k in ("E", "kappa", "eta"):
        q[k] = torch.from_numpy(p[k]).cuda()
    forms = {}
    for name in args.forms.split(","):
        forms[name] = bench.run_form_headline(fld, torch, q, name, args, args.steps,
                                              levels=0)
        log(f"[bench] {name}: " + json.dumps(
            {k: v for k, v in forms[name].items() if k != "survey_ms"}))
    head_name = "mixed" if "mixed" in forms else list(forms)[0]
    head = forms[head_name]
    tform = "fp64" if head_name == "fp64" else (
        "mixed_dir64" if head["direction"] == "fp64" else "mixed")
    return _base(
        "256^3 many-source workload; inputs resident in HBM",
        head["mcell_updates_per_s"], head["ms_per_step"], args.steps, args.warmup,
        "f64+f32" if head_name.startswith("mixed") else "f64",
        {"workload": f"many_sources_{n}^3", "grid": [n] * 3, "sources": 64,
         "sigma_ln": 1.5, "rtol": 1e-8, "precision": head_name,
         "direction": head["direction"], "steps_per_run": args.steps},
        {"bound": "hbm", "kernel": head["dominant"],
         "achieved": round(head["dominant_GBps"], 1), "peak": HBM_PEAK_GBS,
         "unit": "GB/s", "frac": round(head["dominant_GBps"] / HBM_PEAK_GBS, 4),
         "traffic": bench.measured_traffic(head["dominant"], tform, f"many_sources_{n}")},
        {"latency_ms": head["latency_ms"], "forms": forms})


def _batch_problems(synth, torch, nprob):
    probs = []
    for i in range(nprob):
        rng = synth.rng_for(4, i)
        n = int(rng.choice(synth.BATCH_SIZES))
        sigma = float(rng.uniform(0.5, 2.0))
        nsrc = int(rng.integers(1, 33))
        probs.append(synth.t_problem((n, n, n), sigma, nsrc, (1e47, 1e50), 4, i,
                                     "cuda"))
    torch.cuda.synchronize()
    return probs


def batch(args, fld, torch, synth, log):
    """96 independent problems of 32..128^3, one step each to 1e-8, in one
    batched step (one launch per kernel and level for all problems, the PCG
    iterations replayed from captured graphs), with the tile depth and sweep
    counts the autotuner picks, timed as it is tuned: each timed step starts
    cold from the problems' initial fields.  Beside it: the same cold step
    problem by problem (mixed and plain FP64), and warm successive steps."""
    from paper_1306_0645_amd import autotune
    from bench import model_step_bytes
    log(f"[bench] generating {args.batch} batch problems on the GPU")
    probs = _batch_problems(synth, torch, args.batch)
    shapes = [p["shape"] for p in probs]
    hs = [p["h"] for p in probs]
    cells = sum(int(np.prod(s)) for s in shapes)
    E0 = [p["E"] for p in probs]
    K = [p["kappa"] for p in probs]
    H = [p["eta"] for p in probs]
    dts = [p["dt"] for p in probs]
    # one length unit for the batch parameters (limits from the largest box)
    ref = max(probs, key=lambda p: p["L_unit"])
    base = fld.fld_default_params(ref["c"], ref["L_unit"],
                                  precision=fld.FLD_PREC_MIXED, use_graph=args.graph,
                                  warm_start=0)
    report = None
    if args.autotune:
        log("[bench] autotuning tile depth and sweep counts (cold steps)")
        base, report = autotune.tune_batch(shapes, hs, base, (E0, K, H), dts, log=log)

    def cold_steps(B, reps):
        """reps timed single steps, each from the initial fields (the handle
        keeps no warm-start history: warm_start = 0)"""
        times, iters, nbytes = [], [], 0.0
        for r in range(reps + 1):
            Es = [e.clone() for e in E0]
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            sts = B.step(Es, K, H, dts)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            assert all(s["status"] == 0 for s in sts)
            if r == 0:
                continue  # captures the graphs
            times.append(dt)
            iters += [s["iters"] for s in sts]
            nbytes += sum(model_step_bytes(int(np.prod(shp)), s["iters"], s["cycle_nu"],
                                           1, s["levels"], warm=0)
                          for shp, s in zip(shapes, sts))
        return times, iters, nbytes

    reps = max(3, args.steps)
    B = fld.Batch(shapes, hs, base)
    times, iters, nbytes = cold_steps(B, reps)
    B.close()
    sec = float(np.median(times))
    batched = cells / sec / 1e6
    step_gbps = nbytes / sum(times) / 1e9

    def one_by_one(prec):
        q = fld.fld_default_params(ref["c"], ref["L_unit"], precision=prec,
                                   use_graph=args.graph, warm_start=0,
                                   tile_z=base.tile_z if prec else 0)
        solvers = [fld.Solver(p["shape"], p["h"], q) for p in probs]
        best = float("inf")
        for r in range(3):
            Es1 = [e.clone() for e in E0]
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for S, E, k, h, dt in zip(solvers, Es1, K, H, dts):
                S.step(E, k, h, dt)
            torch.cuda.synchronize()
            if r:
                best = min(best, time.perf_counter() - t0)
        for S in solvers:
            S.close()
        return cells / best / 1e6

    log("[bench] the same cold step problem by problem (mixed, then FP64)")
    single_mixed = one_by_one(fld.FLD_PREC_MIXED)
    single_fp64 = one_by_one(fld.FLD_PREC_FP64)
    # warm successive steps (each problem's PCG starts from its previous dEs)
    wprm = fld.Params()
    autotune.ctypes_copy(wprm, base)
    wprm.warm_start = 1
    B = fld.Batch(shapes, hs, wprm)
    Es = [e.clone() for e in E0]
    B.step(Es, K, H, dts)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    witers = []
    for _ in range(args.steps):
        witers += [s["iters"] for s in B.step(Es, K, H, dts)]
    torch.cuda.synchronize()
    wsec = time.perf_counter() - t0
    B.close()
    warm = cells * args.steps / wsec / 1e6
    return _base(
        "aggregate over the batch, one cold step per problem (median of "
        f"{reps}); per-problem working sets up to 128^3",
        batched, 1e3 * sec, 1, 0, "f64+f32",
        {"workload": f"batch_{args.batch}x{{32..128}}^3", "problems": args.batch,
         "cells": cells, "precision": "mixed", "rtol": 1e-8, "start": "cold",
         "tuned": {"tile_z": base.tile_z, "nu_pre": base.nu_pre,
                   "nu_post": base.nu_post}},
        None,
        {"step_roofline": {"bytes_per_cell": round(nbytes / (cells * reps), 1),
                           "achieved": round(step_gbps, 1), "peak": HBM_PEAK_GBS,
                           "unit": "GB/s", "frac": round(step_gbps / HBM_PEAK_GBS, 4),
                           "model": "algorithmic bytes of each problem's step "
                                    "from its iterations and cycle"},
         "latency_ms": {"p50": round(1e3 * float(np.percentile(times, 50)), 3),
                        "p99": round(1e3 * float(np.percentile(times, 99)), 3)},
         "forms": {"batched_mixed_cold": round(batched, 2),
                   "one_by_one_mixed_cold": round(single_mixed, 2),
                   "one_by_one_fp64_cold": round(single_fp64, 2),
                   "batched_mixed_warm_successive": round(warm, 2)},
         "iters_per_problem": float(np.mean(iters)),
         "iters_per_problem_warm": float(np.mean(witers)),
         "autotune": report})


def _oracle_request_error(req, prm, E0, K, H, E_out, steps):
    """The oracle's steps of one served request (its fields copied to the
    host, the server's limiter constants), each solved to 1e-13 from the
    previous one's result: relative L2 error of the served E against the
    oracle's (OpenMP build of the oracle, which evaluates every cell as the
    serial one does; its reductions sum in another order)."""
    import oracle
    dmax, rmin = prm.d_max, prm.r_min
    En = E0.detach().cpu().numpy()
    Kh, Hh = K.detach().cpu().numpy(), H.detach().cpu().numpy()
    for _ in range(steps):
        O = oracle.Problem(En, Kh, Hh, req["h"], req["c"], dmax, rmin, req["dt"],
                           parallel=True)
        dE, st, _, _ = O.solve(tol=1e-13, max_iter=100000)
        if st != oracle.OK:
            return float("nan")
        En = En + dE
    got = E_out.detach().cpu().numpy()
    return float(np.linalg.norm(got - En) / np.linalg.norm(En))


def served(args, fld, torch, synth, log):
    """Poisson stream of requests of 64..384^3 (log-uniform, multiples of 16)
    with 1-5 steps each through the continuous-batching server: every request
    has its own seeded opacity and sources (up to 1000); E^0 is one smooth
    field per grid size.  The arena is 80 % of the free HBM once the request
    fields are resident.  Reports p50/p99 latency (submit -> result) and
    aggregate Mcell-updates/s, an oracle check of a sample of the results,
    and the same requests through plain FP64 handles one after another."""
    nreq = args.requests
    shapes = [synth.serve_request_shape(i) for i in range(nreq)]
    sizes = sorted({s[0] for s in shapes})
    log(f"[bench] served: {nreq} requests over {len(sizes)} grid sizes; "
        "generating each request's fields on the GPU")
    t0 = time.perf_counter()
    reqs, e0 = [], {}
    for i, (n, steps, n_src, sigma) in enumerate(shapes):
        q = synth.t_problem((n, n, n), sigma, n_src, (1e47, 1e50), 5, i, "cuda")
        if n not in e0:
            e0[n] = q["E"]
        else:
            del q["E"]
        q["E"] = e0[n]
        q["out"] = torch.empty_like(e0[n])
        reqs.append(q)
        if i % 100 == 99:
            log(f"[bench]   generated {i + 1}/{nreq}")
    torch.cuda.synchronize()
    log(f"[bench]   fields generated in {time.perf_counter() - t0:.1f} s")
    ref = max(reqs, key=lambda q: q["L_unit"])
    prm = fld.fld_default_params(ref["c"], ref["L_unit"],
                                 precision=fld.FLD_PREC_MIXED,
                                 prolongation=args.prolongation,
                                 warm_start=args.warm_start)
    free, total = torch.cuda.mem_get_info()
    arena = int(0.8 * free) // 256 * 256
    stream = torch.cuda.Stream()
    srv = fld.Server(prm, arena, stream=stream)
    log(f"[bench]   arena {arena / 2**30:.1f} GiB (80 % of {free / 2**30:.1f} GiB free)")

    def submit(i):
        q = reqs[i]
        return srv.submit(q["shape"], q["h"], q["E"], q["kappa"], q["eta"], q["out"],
                          q["dt"], n_steps=shapes[i][1])

    def work(idx):
        return sum(shapes[i][0] ** 3 * shapes[i][1] for i in idx)

    # closed loop: everything at once -> saturation throughput
    nsat = min(64, nreq)
    t0 = time.perf_counter()
    ts = [submit(i) for i in range(nsat)]
    srv.drain()
    sat_s = time.perf_counter() - t0
    for t in ts:
        r = srv.poll(t)
        assert r is not None and r["status"] == 0, r
    sat_rate = nsat / sat_s
    sat_mcells = work(range(nsat)) / sat_s / 1e6
    log(f"[bench]   saturation: {sat_rate:.1f} req/s, {sat_mcells:.0f} Mcell-updates/s")
    # open loop: Poisson arrivals at load x saturation
    lam = args.load * sat_rate
    rng = np.random.default_rng(1311)
    arrivals = np.cumsum(rng.exponential(1.0 / lam, size=nreq))
    tickets = []
    t0 = time.perf_counter()
    for i in range(nreq):
        now = time.perf_counter() - t0
        if arrivals[i] > now:
            time.sleep(arrivals[i] - now)
        tickets.append(submit(i))
        if i % 100 == 99:
            log(f"[bench]   submitted {i + 1}/{nreq}")
    srv.drain()
    wall = time.perf_counter() - t0
    res = [srv.poll(t) for t in tickets]
    srv.close()
    del srv
    torch.cuda.empty_cache()
    assert all(r is not None and r["status"] == 0 for r in res)
    from bench import auto_levels, model_step_bytes
    sbytes = sum(model_step_bytes(shapes[i][0] ** 3, r["iters"], 1, 1,
                                  auto_levels(shapes[i][0]), steps=shapes[i][1])
                 for i, r in enumerate(res))
    sgbps = sbytes / wall / 1e9
    lat = np.array([r["latency_s"] for r in res]) * 1e3
    que = np.array([r["queue_s"] for r in res]) * 1e3
    thr = work(range(nreq)) / wall / 1e6
    p50, p99 = np.percentile(lat, [50, 99])
    # oracle check of a sample: 20 requests drawn (seeded) among those of at
    # most 96^3, where the oracle's steps take about a second each
    small = [i for i in range(nreq) if shapes[i][0] <= 96]
    pick = sorted(np.random.default_rng(1312).choice(small, size=min(20, len(small)),
                                                     replace=False).tolist())
    log(f"[bench]   oracle check of {len(pick)} requests")
    import oracle
    oracle.threads(16)
    errs = [_oracle_request_error(reqs[i], prm, reqs[i]["E"], reqs[i]["kappa"],
                                  reqs[i]["eta"], reqs[i]["out"], shapes[i][1])
            for i in pick]
    # the same requests through plain FP64 handles, one after another (a
    # handle per request: its workspace, its steps)
    log("[bench]   the same requests through plain FP64 handles")
    p64 = fld.fld_default_params(ref["c"], ref["L_unit"], precision=fld.FLD_PREC_FP64,
                                 warm_start=args.warm_start)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i, q in enumerate(reqs):
        S = fld.Solver(q["shape"], q["h"], p64)
        E = q["E"].clone()
        for _ in range(shapes[i][1]):
            S.step(E, q["kappa"], q["eta"], q["dt"])
        S.close()
        del S, E
    torch.cuda.synchronize()
    fp64_wall = time.perf_counter() - t0
    fp64_thr = work(range(nreq)) / fp64_wall / 1e6
    return _base(
        "open-loop Poisson arrivals; latency = submit -> result",
        thr, 1e3 * wall / nreq, nreq, 0, "f64+f32",
        {"workload": f"served_{nreq}_requests_64..384^3", "requests": nreq,
         "load": args.load, "arrival_rate_per_s": round(lam, 2),
         "precision": "mixed", "rtol": 1e-8, "arena_GiB": round(arena / 2**30, 1),
         "fields": "per request (seeded opacity and sources); E^0 per grid size"},
        None,
        {"latency_ms": {"p50": round(float(p50), 3), "p99": round(float(p99), 3),
                        "mean": round(float(lat.mean()), 3)},
         "queue_ms": {"p50": round(float(np.percentile(que, 50)), 3),
                      "p99": round(float(np.percentile(que, 99)), 3)},
         "saturation": {"req_per_s": round(sat_rate, 2),
                        "mcell_updates_per_s": round(sat_mcells, 1)},
         "max_rel_resid": max(r["rel_resid"] for r in res),
         "iters_mean": float(np.mean([r["iters"] for r in res])),
         "oracle_sample": {"requests": pick, "max_rel_l2": max(errs),
                           "gate": 1e-5},
         "forms": {"served_mixed_open_loop": round(thr, 2),
                   "served_mixed_saturation": round(sat_mcells, 2),
                   "plain_fp64_one_by_one": round(fp64_thr, 2),
                   "note": "the open-loop rate is set by the offered load "
                           f"({args.load} x saturation); capacity is the "
                           "saturation rate, against the same requests "
                           "through plain FP64 handles back to back"},
         "step_roofline": {"bytes_per_cell": round(sbytes / work(range(nreq)), 1),
                           "achieved": round(sgbps, 1), "peak": HBM_PEAK_GBS,
                           "unit": "GB/s", "frac": round(sgbps / HBM_PEAK_GBS, 4),
                           "model": "algorithmic bytes of each request from its "
                                    "iterations, V(1,1)"}})


def hii_test1(args, fld, torch, synth, log):
    """Test 1 (Sec. 4.1.1) end to end: radiation + isothermal hydrogen
    chemistry, operator split, over [0, t_end] on the paper's octant meshes
    (mirrored periodic boxes of twice the extent), for each step tolerance
    tau_tol.  Reports the I-front error norm of eq. "i1_error", the average
    step, and the run time per configuration (the paper's Fig. "i1_stats"),
    with a wall-clock cap per run (a capped run reports the time reached)."""
    from paper_1306_0645_amd.ionization import IsothermalHII
    meshes = [int(v) for v in args.hii_meshes.split(",")]
    taus = [float(v) for v in args.hii_taus.split(",")]
    prec = fld.FLD_PREC_MIXED if args.hii_precision == "mixed" else fld.FLD_PREC_FP64
    rows, cells_steps, wall_total = [], 0.0, 0.0
    for n_oct in meshes:
        for tau in taus:
            d = synth.hii_test1(n_oct, t_end_myr=args.hii_t_end, n_out=50)
            prm = fld.fld_default_params(synth.C_LIGHT, d["L_unit"],
                                         precision=prec, tau_tol=tau,
                                         e_floor=d["e_floor"],
                                         tail_cells=args.tail_cells,
                                         warm_start=args.warm_start)
            chem = fld.fld_chem_default_params()
            drv = IsothermalHII(d["shape"], d["h"], prm, chem)
            E, x = (torch.from_numpy(d[k]).cuda() for k in ("E", "x"))
            nh, eta = (torch.from_numpy(d[k]).cuda() for k in ("n_h", "eta"))
            t_start = time.perf_counter()

            def on_output(t, r, i, n_oct=n_oct, tau=tau, t_start=t_start):
                if i and round(t / d["outputs"][0]) % 10 == 0:
                    log(f"[hii] n={n_oct} tau={tau:g} t={t / synth.MYR:.0f} Myr "
                        f"steps={i} r={r / synth.KPC:.3f} kpc "
                        f"wall={time.perf_counter() - t_start:.1f}s")

            res = drv.run(E, x, nh, eta, d["outputs"], d["dt0"],
                          on_output=on_output, wall_cap_s=args.hii_cap_s)
            drv.close()
            t = np.array(res["times"])
            rr = np.array(res["radii"])
            r_true = d["r_s"] * (1.0 - np.exp(-t / d["t_rec"])) ** (1.0 / 3.0)
            err = float(math.sqrt(np.mean(((rr - r_true) / d["r_s"]) ** 2))) if len(t) else None
            cells = int(np.prod(d["shape"]))
            cells_steps += cells * res["steps"]
            wall_total += res["wall_s"]
            row = {"octant": n_oct, "cells": list(d["shape"]), "tau_tol": tau,
                   "t_reached_myr": round(float(t[-1]) / synth.MYR, 2) if len(t) else 0.0,
                   "capped": res["capped"], "steps": res["steps"],
                   "dt_avg_myr": (float(t[-1]) / res["steps"] / synth.MYR) if res["steps"] else None,
                   "iters_per_step": res["iters"] / max(res["steps"], 1),
                   "error_rms": err, "wall_s": round(res["wall_s"], 3),
                   "ms_per_step": 1e3 * res["wall_s"] / max(res["steps"], 1)}
            log(f"[hii] {json.dumps(row)}")
            rows.append(row)
    value = cells_steps / wall_total / 1e6 if wall_total > 0 else 0.0
    total_steps = sum(r["steps"] for r in rows)
    return _base(
        "operator-split radiation + chemistry; small grids are launch-latency "
        "bound, so no HBM roofline is reported for this workload",
        value, 1e3 * wall_total / max(total_steps, 1), total_steps, 0,
        "f64+f32" if prec else "f64",
        {"workload": "hii_test1", "octant_meshes": meshes, "tau_tol": taus,
         "t_end_myr": args.hii_t_end, "precision": args.hii_precision,
         "rtol": 1e-8},
        None, {"sweep": rows})


def multigroup(args, fld, torch, synth, log):
    """Multigroup FLD: G group systems on one 256^3 mesh stepped together in
    the batched engine, against the same groups stepped one by one."""
    from bench import model_step_bytes
    from paper_1306_0645_amd.multigroup import MultigroupFLD
    n = args.n
    G = args.groups
    log(f"[bench] multigroup {n}^3 x {G} groups: generating on the GPU")
    q = synth.t_multigroup(n, G, device="cuda")
    prm = fld.fld_default_params(q["c"], q["L_unit"], precision=fld.FLD_PREC_MIXED,
                                 use_graph=args.graph, warm_start=args.warm_start)
    mg = MultigroupFLD(q["shape"], q["h"], G, prm)
    E = q["E"].clone()
    for _ in range(args.warmup):
        mg.step(E, q["kappa"], q["eta"], q["dt"])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sbytes, iters = 0.0, []
    for k in range(args.steps):
        sts = mg.step(E, q["kappa"], q["eta"], q["dt"])
        assert all(s["status"] == 0 for s in sts)
        iters += [s["iters"] for s in sts]
        sbytes += sum(model_step_bytes(n ** 3, s["iters"], s["cycle_nu"], 1,
                                       s["levels"], warm=args.warm_start) for s in sts)
    torch.cuda.synchronize()
    sec = time.perf_counter() - t0
    mg.close()
    cells = G * n ** 3
    value = cells * args.steps / sec / 1e6
    # the same groups one after another on single-problem handles
    solvers = [fld.Solver(q["shape"], q["h"], prm) for _ in range(G)]
    E1 = q["E"].clone()
    Ks = [q["kappa"][g] for g in range(G)]
    Hs = [q["eta"][g] for g in range(G)]
    for g in range(G):
        solvers[g].step(E1[g], Ks[g], Hs[g], q["dt"])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for _ in range(args.steps):
        for g in range(G):
            solvers[g].step(E1[g], Ks[g], Hs[g], q["dt"])
    torch.cuda.synchronize()
    seq = cells * args.steps / (time.perf_counter() - t1) / 1e6
    for S in solvers:
        S.close()
    gbps = sbytes / sec / 1e9
    return _base(
        "Mcell-updates/s counts every group's cells (G x n^3 per step)",
        value, 1e3 * sec / args.steps, args.steps, args.warmup, "f64+f32",
        {"workload": f"multigroup_{n}^3_x{G}", "grid": [n] * 3, "groups": G,
         "sources": 64, "sigma_ln": 1.5, "precision": "mixed", "rtol": 1e-8},
        None,
        {"step_roofline": {"bytes_per_cell": round(sbytes / (cells * args.steps), 1),
                           "achieved": round(gbps, 1), "peak": HBM_PEAK_GBS,
                           "unit": "GB/s", "frac": round(gbps / HBM_PEAK_GBS, 4),
                           "model": "algorithmic bytes of each group's step "
                                    "from its iterations and cycle"},
         "forms": {"groups_batched": round(value, 2),
                   "groups_one_by_one": round(seq, 2)},
         "iters_per_group_step": float(np.mean(iters))})


def _shapiro_giroux(t, H0, z0, lam, q0, r_s0):
    """Comoving (present-day units) I-front radius of the Shapiro-Giroux
    solution, eq. "radius_cosmo", in an Einstein-de Sitter background."""
    from scipy.integrate import quad
    F = lambda a: ((2 - 4 * q0 - 2 * q0 / a * (1 + z0))
                   * (1 - 2 * q0 + 2 * q0 / a * (1 + z0)) ** 0.5)
    tau = lambda a: lam * (F(a) - F(1.0)) / (6 * q0 ** 2 * (1 + z0) ** 2)
    an = (1.5 * H0 * t) ** (2.0 / 3.0) * (1 + z0)
    integral = quad(lambda b: math.exp(tau(b))
                    * (1 - 2 * q0 + 2 * q0 / b * (1 + z0)) ** -0.5, 1.0, an)[0]
    return r_s0 * (lam * math.exp(-tau(an)) * integral) ** (1.0 / 3.0) * (1 + z0)


def cosmo_test2(args, fld, torch, synth, log):
    """Test 2 (Sec. 4.1.2) end to end: comoving radiation + hydrogen
    chemistry in an Einstein-de Sitter background from z = 4 to 0, on the
    octant meshes for each tau_tol; the error norm against the Shapiro-Giroux
    front, the average step and the run time (the paper's Fig. "sg_stats"),
    with a wall-clock cap per run."""
    from paper_1306_0645_amd.ionization import IsothermalHII, eds_expansion
    meshes = [int(v) for v in args.hii_meshes.split(",")]
    taus = [float(v) for v in args.hii_taus.split(",")]
    prec = fld.FLD_PREC_MIXED if args.hii_precision == "mixed" else fld.FLD_PREC_FP64
    rows, cells_steps, wall_total = [], 0.0, 0.0
    for n_oct in meshes:
        for tau in taus:
            d = synth.cosmo_test2(n_oct, z_end=0.0, n_out=50)
            prm = fld.fld_default_params(synth.C_LIGHT, d["L_unit"],
                                         precision=prec, tau_tol=tau,
                                         e_floor=d["e_floor"],
                                         tail_cells=args.tail_cells,
                                         warm_start=args.warm_start)
            drv = IsothermalHII(d["shape"], d["h"], prm,
                                fld.fld_chem_default_params(),
                                expansion=eds_expansion(d["H0"]))
            E, x = (torch.from_numpy(d[k]).cuda() for k in ("E", "x"))
            nh, eta = (torch.from_numpy(d[k]).cuda() for k in ("n_h", "eta"))
            t_start = time.perf_counter()

            def on_output(t, r, i, n_oct=n_oct, tau=tau, t_start=t_start, d=d):
                k = round((t - d["t0"]) / (d["outputs"][0] - d["t0"]))
                if k % 10 == 0:
                    z = 1.0 / (1.5 * d["H0"] * t) ** (2.0 / 3.0) - 1.0
                    log(f"[cosmo] n={n_oct} tau={tau:g} z={z:.2f} steps={i} "
                        f"r={r / synth.KPC:.2f} kpc(comoving) "
                        f"wall={time.perf_counter() - t_start:.1f}s")

            res = drv.run(E, x, nh, eta, d["outputs"], d["dt0"], t0=d["t0"],
                          on_output=on_output, wall_cap_s=args.hii_cap_s)
            drv.close()
            t = np.array(res["times"])
            rr = np.array(res["radii"])
            r_true = np.array([_shapiro_giroux(tt, d["H0"], d["z0"], d["lambda"],
                                               d["q0"], d["r_s0"]) for tt in t])
            norm = d["r_s0"] * (1 + d["z0"])
            err = float(math.sqrt(np.mean(((rr - r_true) / norm) ** 2))) if len(t) else None
            cells = int(np.prod(d["shape"]))
            cells_steps += cells * res["steps"]
            wall_total += res["wall_s"]
            z_reached = (1.0 / (1.5 * d["H0"] * t[-1]) ** (2.0 / 3.0) - 1.0) if len(t) else 4.0
            row = {"octant": n_oct, "cells": list(d["shape"]), "tau_tol": tau,
                   "z_reached": round(float(z_reached), 3), "capped": res["capped"],
                   "steps": res["steps"],
                   "dt_avg_myr": (float(t[-1] - d["t0"]) / res["steps"] / synth.MYR)
                   if res["steps"] else None,
                   "iters_per_step": res["iters"] / max(res["steps"], 1),
                   "error_rms": err, "wall_s": round(res["wall_s"], 3),
                   "ms_per_step": 1e3 * res["wall_s"] / max(res["steps"], 1)}
            log(f"[cosmo] {json.dumps(row)}")
            rows.append(row)
    value = cells_steps / wall_total / 1e6 if wall_total > 0 else 0.0
    total_steps = sum(r["steps"] for r in rows)
    return _base(
        "comoving radiation + chemistry, Einstein-de Sitter; small grids are "
        "launch-latency bound, so no HBM roofline is reported",
        value, 1e3 * wall_total / max(total_steps, 1), total_steps, 0,
        "f64+f32" if prec else "f64",
        {"workload": "cosmo_test2", "octant_meshes": meshes, "tau_tol": taus,
         "z": [4.0, 0.0], "ndot": 5e46, "precision": args.hii_precision,
         "rtol": 1e-8},
        None, {"sweep": rows})
