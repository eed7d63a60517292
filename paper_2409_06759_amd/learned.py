"""Learned initial amplitudes: data, training and the guess with MP2 fallback.

Training data are the converged CCSD doubles of generated systems, solved
on the GPU in batches (dressed-denominator Jacobi to ||R|| < tol); the
network (``include/cc.h``, cc_mlp_*) is trained with the library's own
forward/backward kernels and Adam.  For a new system the guess is the
network's t2 (t1 = 0) unless its residual norm exceeds that of the MP2
amplitudes t2 = <ab||ij> / D_ij^ab, which are then used instead.

    python -m paper_2409_06759_amd.learned train --systems 200 --out mlp.npz
    python -m paper_2409_06759_amd.learned eval --params mlp.npz --o 32 --v 160
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np
import torch

from ccinputs.synth import BASE_SEED, batch_shapes, make_system

from . import engine as E

TRAIN_SEED = BASE_SEED + 10000


def training_shapes(n, seed=TRAIN_SEED, o_range=(8, 24), v_range=(40, 120)):
    return batch_shapes(n, seed=seed, o_range=o_range, v_range=v_range)


def generate(ctx, shapes, tol=1e-8, group=16, max_iter=400, log=None):
    """(raw features, targets) of the converged amplitudes of `shapes`."""
    raws, ys = [], []
    for g0 in range(0, len(shapes), group):
        chunk = shapes[g0:g0 + group]
        ds = [E.DeviceSystem(make_system(o, v, seed), drop_host=True) for o, v, seed in chunk]
        with E.Batch(ctx, ds, E.CCSD) as B:
            out = B.iterate(tol=tol, max_iter=max_iter, dressed=True)
            for d, (t1, t2), rec in zip(ds, B.amps, out["systems"]):
                if not rec["converged"]:
                    continue
                raws.append(E.MLP.raw_features(ctx, d))
                ys.append(E.MLP.targets(ctx, d.o, d.v, t2))
        if log:
            log(f"[learned] solved {min(g0 + group, len(shapes))}/{len(shapes)} systems "
                f"({out['n_converged']}/{len(chunk)} converged in this group)")
        del ds
        torch.cuda.empty_cache()
    return torch.cat(raws), torch.cat(ys)


def train(ctx, raw, y, epochs=4, batch=65536, lr=1e-3, seed=0, prec=E.F32, log=None):
    stats = E.MLP.fit_stats(ctx, raw, y)
    mlp = E.MLP(ctx, E.MLP.init_params(seed, raw.device), stats, prec)
    z, ys = mlp.standardise(raw, y)
    order = torch.from_numpy(np.random.default_rng(seed).permutation(z.shape[0])).to(raw.device)
    t0 = time.perf_counter()
    hist = mlp.train(z, ys, epochs=epochs, batch=batch, lr=lr, order=order)
    torch.cuda.synchronize()
    if log:
        log(f"[learned] trained {epochs} epochs on {z.shape[0]} samples in {time.perf_counter() - t0:.1f}s; "
            f"loss per epoch {[round(h, 5) for h in hist]}")
    return mlp, hist


def mp2_guess(plan, dsys):
    """t2 = <ab||ij> / D (one Jacobi step from t = 0), t1 = 0."""
    t1, t2 = E.zeros_amps(dsys, plan.method)
    plan.step(t1, t2, 0.0, False)
    if t1 is not None:
        t1.zero_()
    return t1, t2


def guess_with_fallback(ctx, plan, dsys, mlp):
    """(t1, t2, source, ||R(mlp)||, ||R(mp2)||, inference seconds)."""
    t1, t2 = E.zeros_amps(dsys, plan.method)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    mlp.guess(dsys, t1, t2)
    torch.cuda.synchronize()
    t_inf = time.perf_counter() - t0
    _, _, rn_mlp = plan.residual(t1, t2, want_r=False)
    m1, m2 = mp2_guess(plan, dsys)
    _, _, rn_mp2 = plan.residual(m1, m2, want_r=False)
    if rn_mlp <= rn_mp2:
        return t1, t2, "mlp", rn_mlp, rn_mp2, t_inf
    return m1, m2, "mp2", rn_mlp, rn_mp2, t_inf


def evaluate(ctx, mlp, o=32, v=160, seed=BASE_SEED, tol=1e-8, max_iter=1000, precs=("f64",), log=None):
    """Iterations and time to ||R|| < tol from the network's guess and from
    MP2, for each contraction precision in `precs` (reduced ones finish in
    FP64).  Times include the guess (network inference, or the MP2 step)."""
    s = make_system(o, v, seed)
    d = E.DeviceSystem(s, drop_host=True)
    res = {"o": o, "v": v}
    with E.Plan(ctx, d, E.CCSD) as plan:
        t1, t2, src, rn_mlp, rn_mp2, t_inf = guess_with_fallback(ctx, plan, d, mlp)
        del t1, t2
        for pname in precs:
            for name in ("mlp", "mp2"):
                a1, a2 = E.zeros_amps(d, E.CCSD)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                if name == "mlp":
                    mlp.guess(d, a1, a2)
                else:
                    plan.step(a1, a2, 0.0, False)
                    a1.zero_()
                torch.cuda.synchronize()
                t_guess = time.perf_counter() - t0
                out = E.iterate(ctx, d, E.CCSD, a1, a2, tol=tol, max_iter=max_iter, dressed=True,
                                prec=E.PRECS[pname], autotune=True)
                res.setdefault(pname, {})[name] = {
                    "iterations": out["iters"], "reduced_precision_iterations": out["lowp_iters"],
                    "seconds": out["seconds"] + t_guess, "guess_seconds": t_guess, "energy": out["energy"],
                    "converged": out["converged"]}
                if log:
                    log(f"[learned] o={o} v={v} {pname} from {name} guess: {out['iters']} it, "
                        f"{out['seconds'] + t_guess:.2f}s (guess {t_guess * 1e3:.1f} ms), E={out['energy']:.10f}")
    res["inference_seconds"] = t_inf
    res["rnorm_guess"] = {"mlp": rn_mlp, "mp2": rn_mp2}
    res["chosen"] = src
    base = res[precs[0]]
    res["mlp"], res["mp2"] = base["mlp"], base["mp2"]
    res["iterations_saved"] = base["mp2"]["iterations"] - base["mlp"]["iterations"]
    res["speedup_vs_mp2"] = base["mp2"]["seconds"] / base["mlp"]["seconds"]
    if log:
        log(f"[learned] ||R|| of the guess: mlp {rn_mlp:.3e}, mp2 {rn_mp2:.3e}; inference {t_inf * 1e3:.1f} ms")
    return res


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    tr = sub.add_parser("train")
    tr.add_argument("--systems", type=int, default=2000)
    tr.add_argument("--epochs", type=int, default=4)
    tr.add_argument("--batch", type=int, default=65536)
    tr.add_argument("--lr", type=float, default=1e-3)
    tr.add_argument("--group", type=int, default=64, help="systems solved together in one batch")
    tr.add_argument("--tol", type=float, default=1e-8, help="residual norm of the training solutions")
    tr.add_argument("--out", required=True)
    tr.add_argument("--eval", action="store_true", help="evaluate on o=32 v=160 after training")
    tr.add_argument("--precs", default="f64", help="contraction precisions of the evaluation")
    ev = sub.add_parser("eval")
    ev.add_argument("--params", required=True)
    ev.add_argument("--o", type=int, default=32)
    ev.add_argument("--v", type=int, default=160)
    ev.add_argument("--precs", default="f64")
    args = ap.parse_args(argv)
    log = lambda *a: print(*a, file=sys.stderr, flush=True)  # noqa: E731
    ctx = E.Context(0)
    if args.cmd == "train":
        t0 = time.perf_counter()
        raw, y = generate(ctx, training_shapes(args.systems), tol=args.tol, group=args.group, log=log)
        t_gen = time.perf_counter() - t0
        mlp, hist = train(ctx, raw, y, epochs=args.epochs, batch=args.batch, lr=args.lr, log=log)
        mlp.save(args.out)
        summary = {"systems": args.systems, "samples": int(raw.shape[0]), "data_seconds": t_gen,
                   "loss_per_epoch": hist, "stats": mlp.stats}
        if args.eval:
            summary["eval"] = evaluate(ctx, mlp, precs=tuple(args.precs.split(",")), log=log)
        print(json.dumps(summary))
    else:
        mlp = E.MLP.load(ctx, args.params)
        print(json.dumps(evaluate(ctx, mlp, o=args.o, v=args.v, precs=tuple(args.precs.split(",")), log=log)))


if __name__ == "__main__":
    main()
