"""Train the learned-interpolation network on AMG set-ups the method itself
generates (GPU: set-ups, targets, forward, backward and Adam all run in the
HIP library).

Set-up k (seed 1000 + k): jittered Kuhn cube (interior nodes moved by
U(-0.1h, 0.1h)^3), kappa = 10^U(3,6), c10 and c01 scaled by U(0.7, 1.3), the
tangent taken after `newton_per_inc` Newton steps of each load increment up to
a random increment 1..5 (of 5).  Samples: every level-0 F point with a strong
C neighbour; target: the local ideal interpolation.  The default recipe is
1800 set-ups of the 8^3 cube (all samples) and 200 of the 48^3 cube (set-ups
1800..1999, a seeded 3.5% of their samples, hfsi_mlp_collect_sampled): about
4M samples, 8 epochs.

    python -m paper_1312_5561_amd.train_mlp --out gpurun_out/mlp_cube.npz
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

FORMAT_VERSION = 1
DEFAULT_WEIGHTS = os.path.join(os.path.dirname(os.path.abspath(__file__)), "weights", "mlp_cube.npz")
# the same weights as the raw file hfsi_mlp_load reads (C callers)
DEFAULT_RAW_WEIGHTS = os.path.join(os.path.dirname(os.path.abspath(__file__)), "weights", "mlp_cube.hfsimlp")
RAW_MAGIC = b"HFSIMLP\0"
RAW_VERSION = 1


def _fnv1a64(data: bytes) -> int:
    h = 14695981039346656037
    for byte in data:
        h = ((h ^ byte) * 1099511628211) & 0xFFFFFFFFFFFFFFFF
    return h


def write_raw(path, w):
    """The raw weight file of hfsi_mlp_load: magic, int32 version, int32
    count, fp32 parameters, uint64 FNV-1a hash of the parameter bytes."""
    w = np.ascontiguousarray(w, "<f4")
    payload = w.tobytes()
    with open(path, "wb") as f:
        f.write(RAW_MAGIC)
        f.write(np.array([RAW_VERSION, w.size], "<i4").tobytes())
        f.write(payload)
        f.write(np.array([_fnv1a64(payload)], "<u8").tobytes())


def init_weights(seed=0):
    """He-normal hidden layers, zero last layer (starts as classical)."""
    r = np.random.default_rng(seed)
    w1 = r.normal(0, np.sqrt(2.0 / 64), (64, 64))
    w2 = r.normal(0, np.sqrt(2.0 / 64), (64, 64))
    parts = [w1, np.zeros(64), w2, np.zeros(64), np.zeros((64, 32)), np.zeros(32)]
    return np.concatenate([p.ravel() for p in parts]).astype(np.float32)


def setup_problem(k, N):
    import synth
    r = np.random.default_rng(1000 + k)
    kappa = 10.0 ** r.uniform(3, 6)
    c10 = 0.5 * r.uniform(0.7, 1.3)
    c01 = 0.1 * r.uniform(0.7, 1.3)
    prob = synth.cube_problem(N, kappa=kappa, c10=c10, c01=c01, jitter=0.1, seed=1000 + k)
    inc = int(r.integers(1, 6))
    return prob, inc


def collect(ctx_factory, n_setups, N, newton_per_inc=2, first=0, log=print, ctx=None, fraction=1.0):
    """Append the samples of set-ups first .. first + n_setups - 1 to the
    training set of `ctx` (a fresh context from ctx_factory when None); with
    fraction < 1 a seeded subset of each set-up's samples (seed 1000 + k)."""
    import torch
    from paper_1312_5561_amd import hfsi
    ctx = ctx_factory() if ctx is None else ctx
    total, failed = 0, 0
    prm = hfsi.newton_params(amg=hfsi.amg_params(smoother=1, precision=1, max_coarse=100),
                             solve=hfsi.solve_params(max_iter=2000))
    for k in range(first, first + n_setups):
        prob, inc = setup_problem(k, N)
        ctx.set_problem(prob)
        v = torch.zeros(prob.n_dofs, dtype=torch.float64, device="cuda")
        for q in range(1, inc + 1):
            for _ in range(newton_per_inc):
                ctx.newton_step(v, q / 5.0, prm)
        R = torch.zeros_like(v)
        ctx.assemble_residual_tangent(v, inc / 5.0, R)
        ctx.amg_setup(hfsi.amg_params(smoother=1, precision=1, max_coarse=100))
        a, f = ctx.mlp_collect() if fraction >= 1.0 else ctx.mlp_collect_sampled(fraction, 1000 + k)
        total += a
        failed += f
        if (k - first) % 25 == 0:
            log(f"[train] set-up {k}: {a} samples (total {total}, failed targets {failed})")
    return ctx, total, failed


def train(ctx, epochs, batch=1024, lr=1e-3, seed=7, weights=None, log=print):
    from paper_1312_5561_amd import hfsi
    ns = ctx.mlp_samples()[0].shape[0]
    ctx.mlp_set_weights(init_weights(seed) if weights is None else weights)
    r = np.random.default_rng(seed)
    order = np.concatenate([r.permutation(ns) for _ in range(epochs)]).astype(np.int32)
    info = ctx.mlp_train(order, hfsi.train_params(batch=batch, lr=lr))
    log(f"[train] {info.steps} Adam steps on {ns} samples: loss {info.loss_first:.3e} -> {info.loss_last:.3e} "
        f"in {info.seconds:.1f} s")
    return info


def save(path, ctx, meta):
    w = ctx.mlp_get_weights()
    m, v, step = ctx.mlp_adam_state()
    os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
    np.savez(path, weights=w, adam_m=m, adam_v=v, step=np.int64(step), version=np.int64(FORMAT_VERSION),
             meta=np.frombuffer(json.dumps(meta).encode(), dtype=np.uint8))
    write_raw(os.path.splitext(path)[0] + ".hfsimlp", w)


def load(path):
    """(weights, meta) from a checkpoint written by save()."""
    with np.load(path, allow_pickle=False) as z:
        if int(z["version"]) != FORMAT_VERSION:
            raise ValueError(f"unsupported checkpoint version {int(z['version'])}")
        return z["weights"].astype(np.float32), json.loads(bytes(z["meta"]).decode())


HELD_OUT = ((8, 9001, None), (8, 9002, None), (16, 9003, None), (24, 9004, None), (48, 9005, None),
            (96, 9101, 1e3), (96, 9102, 1e4), (96, 9103, 1e5), (96, 9104, 1e6))


def evaluate(path, cases=HELD_OUT, log=print):
    """Held-out comparison of learned and classical level-0 interpolation:
    jittered cube (seed s, kappa = 10^U(3,6) unless given), two Newton steps
    per increment 0.2..0.8, tangent at load 1.0, set-up with the judge
    disabled, FGMRES(50) to 1e-8 from zero; time = set-up + solve."""
    import torch
    import synth
    from paper_1312_5561_amd import hfsi
    w, meta = load(path)
    rows = []
    for N, seed, kap in cases:
        r = np.random.default_rng(seed)
        kappa = 10 ** r.uniform(3, 6) if kap is None else kap
        prob = synth.cube_problem(N, kappa=kappa, jitter=0.1, seed=seed)
        ctx = hfsi.Context(0)
        ctx.set_problem(prob)
        ctx.mlp_set_weights(w)
        v = torch.zeros(prob.n_dofs, dtype=torch.float64, device="cuda")
        p = hfsi.newton_params(amg=hfsi.amg_params(smoother=1, precision=1), solve=hfsi.solve_params(max_iter=3000))
        for q in range(1, 5):
            for _ in range(2):
                ctx.newton_step(v, q / 5.0, p)
        R = torch.zeros_like(v)
        ctx.assemble_residual_tangent(v, 1.0, R)
        b = -R
        res = {}
        for interp in (0, 1):
            torch.cuda.synchronize()
            t = time.time()
            info = ctx.amg_setup(hfsi.amg_params(smoother=1, precision=1, interp=interp, fallback_rho=1.0,
                                                    judge_classical=0))
            x = torch.zeros_like(b)
            si, _ = ctx.krylov_amg_solve(b, x, hfsi.solve_params(max_iter=3000))
            torch.cuda.synchronize()
            ms = (time.time() - t) * 1e3
            rho = ctx.amg_convergence_factor(10, 777)
            res[interp] = dict(rho=rho, its=si.iterations, ms=ms, opc=info.op_complexity)
        line = (f"N={N} kappa={kappa:.2e} classical rho={res[0]['rho']:.3f} its={res[0]['its']} "
                f"t={res[0]['ms']:.0f}ms opc={res[0]['opc']:.2f} | learned rho={res[1]['rho']:.3f} "
                f"its={res[1]['its']} t={res[1]['ms']:.0f}ms opc={res[1]['opc']:.2f}")
        log(line)
        rows.append((N, kappa, res))
    return rows


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--evaluate", default=None, help="checkpoint to compare against classical interpolation")
    ap.add_argument("--setups", type=int, default=1800)
    ap.add_argument("--N", type=int, default=8)
    ap.add_argument("--setups-large", type=int, default=200)
    ap.add_argument("--N-large", type=int, default=48)
    ap.add_argument("--fraction-large", type=float, default=0.035,
                    help="share of each large set-up's samples kept")
    ap.add_argument("--epochs", type=int, default=8)
    ap.add_argument("--batch", type=int, default=1024)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--out", default="gpurun_out/mlp_cube.npz")
    args = ap.parse_args()
    from paper_1312_5561_amd import hfsi
    if args.evaluate:
        evaluate(args.evaluate, log=lambda s: print(s, flush=True))
        return
    t0 = time.time()
    log = lambda s: print(s, flush=True)  # noqa: E731
    ctx, total, failed = collect(lambda: hfsi.Context(0), args.setups, args.N, log=log)
    total_l = failed_l = 0
    if args.setups_large > 0:
        ctx, total_l, failed_l = collect(None, args.setups_large, args.N_large, first=args.setups, log=log, ctx=ctx,
                                         fraction=args.fraction_large)
    print(f"[train] collected {total} + {total_l} samples ({failed + failed_l} failed targets) in "
          f"{time.time() - t0:.1f} s", flush=True)
    info = train(ctx, args.epochs, args.batch, args.lr, log=log)
    meta = dict(setups=args.setups, N=args.N, setups_large=args.setups_large, N_large=args.N_large,
                fraction_large=args.fraction_large, strength_theta=hfsi.amg_params().strength_theta,
                epochs=args.epochs, batch=args.batch, lr=args.lr, samples=total + total_l,
                samples_large=total_l, failed_targets=failed + failed_l, loss_first=info.loss_first,
                loss_last=info.loss_last, steps=info.steps)
    save(args.out, ctx, meta)
    print(json.dumps(meta), flush=True)


if __name__ == "__main__":
    main()
