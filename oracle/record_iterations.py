"""Record how many Jacobi-PCG iterations the oracle needs for the first step
of the 640^3 reionization share (one of the 125 GPU shares of the 3200^3 run,
Sec. 5) to reach ||b - A dE||_2 <= 1e-8 ||b||_2, the stopping rule of Table 1.

The benchmark times the oracle on a bounded sample of that step (its assembly
and a few iterations) and extrapolates to this count, since the full solve
takes minutes on the host.  This script calls only the oracle and the seeded
input generator (drawn on the GPU, as the benchmark draws it, then copied to
the host) and writes the count to reionization_640_iterations.txt beside it:

    python oracle/record_iterations.py [--threads 16] [--out PATH]
"""
import argparse
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--threads", type=int, default=16)
    ap.add_argument("--n", type=int, default=640)
    ap.add_argument("--device", default="cuda")
    ap.add_argument("--out", default=os.path.join(HERE, "reionization_640_iterations.txt"))
    args = ap.parse_args()
    import torch

    import oracle
    import synth
    oracle.build(force=False)
    q = synth.t_reionization_share(n=args.n, device=args.device)
    E, K, H = (q[k].cpu().numpy() for k in ("E", "kappa", "eta"))
    del q["E"], q["kappa"], q["eta"]
    if args.device != "cpu":
        torch.cuda.empty_cache()
    threads = oracle.threads(args.threads)
    dmax, rmin = oracle.limits(q["c"], q["L_unit"])
    O = oracle.Problem(E, K, H, q["h"], q["c"], dmax, rmin, q["dt"], parallel=True)
    t0 = time.perf_counter()
    _, st, it, rel = O.solve(tol=1e-8, max_iter=100000)
    sec = time.perf_counter() - t0
    print(f"status {st} iterations {it} relres {rel:.3e} in {sec:.1f} s on {threads} threads",
          flush=True)
    if st != oracle.OK:
        sys.exit(1)
    with open(args.out, "w") as f:
        f.write("# Jacobi-PCG iterations of the oracle to ||b - A dE||_2 <= 1e-8 ||b||_2 on\n"
                f"# step 1 of the {args.n}^3 reionization share (E^0 = 1e-45 erg/cm^3,\n"
                f"# fields of synth.t_reionization_share drawn on {args.device}); "
                f"{sec:.0f} s on {threads} host threads\n"
                "# written by: python oracle/record_iterations.py\n"
                f"n = {args.n}\nstep1_iterations = {it}\nstep1_relres = {rel:.6e}\n")


if __name__ == "__main__":
    main()
