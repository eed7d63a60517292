"""Learned initial amplitudes: data, training and the guess with MP2 fallback.

Training data are the converged CCSD doubles of generated systems, solved
on the GPU in batches (dressed-denominator Jacobi to ||R|| < tol); the
network (``include/cc.h``, cc_mlp_*) is trained with the library's own
forward/backward kernels and Adam.  For a new system cc_iterate's MLP guess
takes the network's t2 (t1 = 0) unless its residual norm exceeds that of the
MP2 amplitudes t2 = <ab||ij> / D_ij^ab, which are then used instead.

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
    raw, y = torch.cat(raws), torch.cat(ys)
    if log:
        log(f"[learned] data: {raw.shape[0]} samples")
    return raw, y


def train(ctx, raw, y, epochs=4, batch=65536, lr=1e-3, seed=0, prec=E.F32, log=None, mlp=None):
    """Adam on (raw, y); a fresh network with statistics fitted to this data,
    or `mlp` (parameters, statistics and Adam state kept) trained further."""
    t0 = time.perf_counter()
    if mlp is None:
        stats = E.MLP.fit_stats(ctx, raw, y)
        mlp = E.MLP(ctx, E.MLP.init_params(seed, raw.device), stats, prec)
    z, ys = mlp.standardise(raw, y)
    n = z.shape[0]
    if log:
        log(f"[learned] standardised {n} samples ({time.perf_counter() - t0:.1f}s)")
    gen = torch.Generator(device=raw.device)
    gen.manual_seed(seed)
    order = torch.randperm(n, generator=gen, device=raw.device)
    # the rows are gathered into the shuffled order once: minibatches that
    # gather single rows from all over a table of 1e8+ rows run several times
    # slower than contiguous ones
    z, ys = z[order], ys[order]
    del order
    torch.cuda.synchronize()
    if log:
        log(f"[learned] shuffled ({time.perf_counter() - t0:.1f}s)")
    t0 = time.perf_counter()
    # every epoch visits the rows in the same shuffled order, in pieces of
    # whole minibatches so that progress can be reported
    piece = max(batch, (n // 8) // batch * batch)
    hist = []
    for ep in range(epochs):
        losses, counts = [], []
        for a in range(0, n, piece):
            b = min(a + piece, n)
            losses.append(mlp.train(z[a:b], ys[a:b], epochs=1, batch=batch, lr=lr)[0])
            counts.append((b - a + batch - 1) // batch)
            if log:
                log(f"[learned] epoch {ep}: {min(a + piece, n)}/{n} samples, loss {losses[-1]:.5f}")
        hist.append(float(np.dot(losses, counts) / sum(counts)))
    torch.cuda.synchronize()
    if log:
        log(f"[learned] trained {epochs} epochs on {z.shape[0]} samples in {time.perf_counter() - t0:.1f}s; "
            f"loss per epoch {[round(h, 5) for h in hist]}")
    return mlp, hist


def evaluate(ctx, mlp, o=32, v=160, seed=BASE_SEED, tol=1e-8, max_iter=1000, precs=("f64",), log=None):
    """Iterations and time to ||R|| < tol from the network's start (cc_iterate's
    MLP guess with its MP2 fallback), from the MP2 start and from t = 0, for
    each contraction precision in `precs` (reduced ones finish in FP64).
    Times include forming the start."""
    d = E.DeviceSystem(make_system(o, v, seed), drop_host=True)
    res = {"o": o, "v": v}
    for pname in precs:
        for start in ("mlp", "mp2", "given"):
            a1, a2 = E.zeros_amps(d, E.CCSD)
            out = E.iterate(ctx, d, E.CCSD, a1, a2, tol=tol, max_iter=max_iter, dressed=True, prec=E.PRECS[pname],
                            autotune=True, guess=start, mlp=mlp if start == "mlp" else None)
            name = "zero" if start == "given" else start
            res.setdefault(pname, {})[name] = {
                "iterations": out["iters"], "reduced_precision_iterations": out["lowp_iters"],
                "seconds": out["seconds"], "guess_seconds": out["guess_seconds"], "guess_used": out["guess_used"],
                "energy": out["energy"], "converged": out["converged"]}
            if start == "mlp":
                res["rnorm_guess"] = out["guess_rnorm"]
            if log:
                log(f"[learned] o={o} v={v} {pname} from {name}: {out['iters']} it, {out['seconds']:.2f}s "
                    f"(guess {out['guess_seconds'] * 1e3:.1f} ms, used {out['guess_used']}), E={out['energy']:.10f}")
    base = res[precs[0]]
    res["mlp"], res["mp2"] = base["mlp"], base["mp2"]
    res["iterations_saved"] = base["mp2"]["iterations"] - base["mlp"]["iterations"]
    res["speedup_vs_mp2"] = base["mp2"]["seconds"] / base["mlp"]["seconds"]
    res["speedup_vs_zero"] = base["zero"]["seconds"] / base["mlp"]["seconds"]
    if log:
        log(f"[learned] ||R|| of the starts: {res['rnorm_guess']}")
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
    tr.add_argument("--shard", default="0/1", help="k/n: train on systems k, k+n, k+2n, ... of the list")
    tr.add_argument("--resume", help="network (with Adam state) to train further")
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
        k, n = (int(x) for x in args.shard.split("/"))
        shapes = training_shapes(args.systems)[k::n]
        raw, y = generate(ctx, shapes, tol=args.tol, group=args.group, log=log)
        t_gen = time.perf_counter() - t0
        prev = E.MLP.load(ctx, args.resume) if args.resume else None
        mlp, hist = train(ctx, raw, y, epochs=args.epochs, batch=args.batch, lr=args.lr, log=log, mlp=prev)
        mlp.save(args.out, with_state=True)
        summary = {"systems": args.systems, "shard": args.shard, "shard_systems": len(shapes),
                   "samples": int(raw.shape[0]), "data_seconds": t_gen, "loss_per_epoch": hist, "stats": mlp.stats,
                   "adam_steps": mlp.t.value}
        if args.eval:
            summary["eval"] = evaluate(ctx, mlp, precs=tuple(args.precs.split(",")), log=log)
        print(json.dumps(summary))
    else:
        mlp = E.MLP.load(ctx, args.params)
        print(json.dumps(evaluate(ctx, mlp, o=args.o, v=args.v, precs=tuple(args.precs.split(",")), log=log)))


if __name__ == "__main__":
    main()
