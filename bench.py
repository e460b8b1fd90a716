#!/usr/bin/env python3
"""Benchmark: dofs solved per second by one Newton step of the solid problem.

Workload (default): the 48^3 Kuhn cube (117,649 nodes, 470,596 dofs),
Mooney-Rivlin c10=0.5 c01=0.1 kappa=1e4, clamped at x=0, dead traction
(0,0,0.05) on x=1.  The state is first driven through load increments
0.2..0.8 (untimed); every timed step then performs one full Newton step at
load 1.0 from that converged state: assembly of R and K, AMG set-up on A,
FGMRES with the block preconditioner to ||b-Kx|| <= 1e-8 ||b||, update and
mass norm.  All arithmetic runs in the HIP library; inputs are resident in
device memory before the timed region.

value = dofs * steps / elapsed for the mixed-precision path (fp32 V-cycle
inside fp64 FGMRES, classical interpolation); the plain fp64 path is timed
the same way and reported beside it.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "dofs solved/s to 1e-8 rel. residual: learned-AMG FP32 vs plain FP64 AMG"
HBM_PEAK_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--N", type=int, default=48, help="hexahedra per cube edge")
    ap.add_argument("--kappa", type=float, default=1e4)
    ap.add_argument("--smoother", type=int, default=1, help="0 l1-Jacobi, 1 Chebyshev")
    ap.add_argument("--restart", type=int, default=50)
    ap.add_argument("--max-iter", type=int, default=3000)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-fp64", action="store_true", help="skip the plain fp64 comparison")
    ap.add_argument("--roofline-reps", type=int, default=50)
    return ap.parse_args()


def run_steps(ctx, v0, v, prm, steps, torch):
    infos = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        v.copy_(v0)
        info, code = ctx.newton_step(v, 1.0, prm)
        if code != 0:
            raise RuntimeError("Newton step did not converge its linear solve")
        infos.append(info)
    torch.cuda.synchronize()
    return time.perf_counter() - t0, infos


def summarize(infos):
    keys = ("krylov_iterations", "t_assemble", "t_setup", "t_solve", "t_total", "rel_residual", "amg_levels")
    out = {k: float(np.median([getattr(i, k) for i in infos])) for k in keys}
    out["krylov_iterations"] = int(out["krylov_iterations"])
    out["amg_levels"] = int(out["amg_levels"])
    return out


def cpu_baseline(N_sample=16, kappa=1e4):
    """The oracle, untuned, on one Newton step of the same cube physics at
    N_sample^3 hexahedra, single-threaded."""
    import synth
    from oracle import fe, newton
    try:
        from threadpoolctl import threadpool_limits
    except ImportError:  # pragma: no cover
        threadpool_limits = None
    prob = synth.cube_problem(N_sample, kappa=kappa)
    d = fe.Discretization(prob)
    prm = newton.NewtonParams()
    v = np.zeros(4 * prob.n_nodes)
    v, _, _ = newton.solve_increment(d, v, 0.8, newton.NewtonParams(eps2=1e-6))

    def one():
        t = time.perf_counter()
        newton.newton_step(d, v, 1.0, prm)
        return time.perf_counter() - t

    if threadpool_limits is not None:
        with threadpool_limits(limits=1):
            dt = one()
    else:
        dt = one()
    return {"value": prob.n_dofs / dt, "unit": "dofs/s", "cores": 1, "kind": "oracle",
            "sample": f"one full Newton step (assembly, AMG set-up, FGMRES to 1e-8) of the same cube physics at "
                      f"{N_sample}^3 hexahedra ({prob.n_dofs} dofs), numpy/scipy fp64 single thread, {dt:.2f} s"}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported (the multi-GPU "
              f"partitioning is a design in DESIGN.md, not built)", file=sys.stderr)
        sys.exit(2)
    import torch
    import synth
    from paper_1312_5561_amd import hfsi

    prob = synth.cube_problem(args.N, kappa=args.kappa)
    ndofs = prob.n_dofs
    ctx = hfsi.Context(0)
    ctx.set_problem(prob)
    v = torch.zeros(ndofs, dtype=torch.float64, device="cuda")
    amg32 = hfsi.amg_params(precision=1, smoother=args.smoother)
    amg64 = hfsi.amg_params(precision=0, smoother=args.smoother)
    sp = hfsi.solve_params(tol=1e-8, restart=args.restart, max_iter=args.max_iter)
    p32 = hfsi.newton_params(amg=amg32, solve=sp)
    p64 = hfsi.newton_params(amg=amg64, solve=sp)
    # untimed: converge the load increments 0.2 .. 0.8
    for k in range(1, int(round(0.8 * 5)) + 1):
        n0 = None
        for _ in range(25):
            info, _ = ctx.newton_step(v, k / 5.0, p32)
            n0 = info.dv_mass_norm if n0 is None else n0
            if info.dv_mass_norm <= 1e-10 * n0:
                break
    v0 = v.clone()
    print(f"[bench] prepared state: {ndofs} dofs", file=sys.stderr, flush=True)

    # mixed precision (value)
    run_steps(ctx, v0, v, p32, args.warmup, torch)
    dt32, inf32 = run_steps(ctx, v0, v, p32, args.steps, torch)
    v32 = v.clone()
    print(f"[bench] fp32 V-cycle: {dt32 / args.steps * 1e3:.1f} ms/step", file=sys.stderr, flush=True)
    res = {}
    if not args.no_fp64:
        run_steps(ctx, v0, v, p64, max(1, args.warmup // 2), torch)
        dt64, inf64 = run_steps(ctx, v0, v, p64, args.steps, torch)
        v64 = v.clone()
        d32 = (v32 - v0).double()
        d64 = (v64 - v0).double()
        err = float(torch.linalg.norm(d32 - d64) / torch.linalg.norm(d64))
        res["fp64_plain"] = {"value": ndofs * args.steps / dt64, "unit": "dofs/s",
                             "ms_per_step": dt64 / args.steps * 1e3, **summarize(inf64)}
        res["fp32_vs_fp64_update_rel_err"] = err
        print(f"[bench] fp64: {dt64 / args.steps * 1e3:.1f} ms/step, update rel diff {err:.2e}", file=sys.stderr,
              flush=True)
        # leave the mixed-precision hierarchy in place for the roofline timing
        v.copy_(v0)
        ctx.newton_step(v, 1.0, p32)

    # roofline of the dominant kernel: the level-0 smoother sweep (fp32)
    ms, nbytes = ctx.time_kernel(0, args.roofline_reps)
    achieved = nbytes / (ms * 1e-3) / 1e9
    sweep = "l1-Jacobi sweep (OP_JACOBI)" if args.smoother == 0 else "Chebyshev step (OP_CHEB)"
    roof = {"kernel": f"level-0 {sweep}, fp32 CSR, k_csr<float,16,...>", "bound": "hbm",
            "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
            "traffic": None, "avg_us": ms * 1e3, "bytes_per_launch": nbytes}
    extra = {}
    for kid, name in ((1, "level-0 residual fp32"), (2, "tangent SpMV fp64 4x4 blocks"), (3, "element assembly")):
        kms, kb = ctx.time_kernel(kid, 20 if kid != 3 else 3)
        extra[name] = {"avg_us": kms * 1e3, "GB/s": kb / (kms * 1e-3) / 1e9}
    cms, cb = ctx.time_kernel(9, 20, 256 << 20)
    extra["copy 256 MiB"] = {"avg_us": cms * 1e3, "GB/s": cb / (cms * 1e-3) / 1e9}

    out = {
        "metric": METRIC,
        "value": ndofs * args.steps / dt32,
        "unit": "dofs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt32 / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64 (fp32 V-cycle)",
        "data": "synthetic",
        "config": {"workload": f"cube{args.N} Mooney-Rivlin kappa={args.kappa:g}: one Newton step at load 1.0 from "
                               f"the converged load-0.8 state, FGMRES to 1e-8", "dofs": ndofs,
                   "interp": "classical", "precision": "fp32 V-cycle in fp64 FGMRES",
                   "smoother": "l1-Jacobi" if args.smoother == 0 else "Chebyshev"},
        "breakdown": summarize(inf32),
        **res,
        "roofline": roof,
        "kernels": extra,
    }
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(kappa=args.kappa)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
