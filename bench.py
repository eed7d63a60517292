"""Benchmark of the CCSD residual path on one MI355X.

One step = one Jacobi iteration of spin-orbital CCSD: tau formation and the
energy, every binary contraction of the residual (ladder, ring, hh ladder,
Z, intermediates, singles), the antisymmetrising assembly, the denominator
update and the residual norm.  Workload: o = 32 occupied, v = 160 virtual
spin orbitals, FP64, seeded random antisymmetrised integrals (sigma = 0.01),
diagonal Fock with occupied energies in [-2, -0.5] and virtual in [0.5, 3].

Prints one JSON line.  `value` is the algorithmic dense FLOP rate of a step
(inputs resident in HBM); `roofline` is the ladder GEMM's rate measured with
HIP events on the library stream during the timed steps; `cpu_baseline` is
the FP64 NumPy oracle timed on the host for one residual evaluation.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import pathlib
import sys
import time

ROOT = pathlib.Path(__file__).resolve().parent
sys.path.insert(0, str(ROOT))

PEAK_FP64_TFLOPS = 78.6  # MI355X dense FP64 matrix peak (published)
# Peaks per contraction precision, in algorithmic TFLOP/s: FP32 matrix 157.3;
# split-bf16 issues three bf16 MFMA products per algorithmic product, so its
# roofline is the dense bf16 peak (2.5 PFLOP/s) divided by three.
PEAKS = {"f64": 78.6, "f32": 157.3, "bf16x3": 2500.0 / 3.0}
CONFIGS = {
    "c2": dict(o=32, v=160, method="ccsd"),
    "c1": dict(o=8, v=24, method="ccd"),
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def source_hash() -> str:
    h = hashlib.sha256()
    for f in ("gemm_f64.hip", "common.hpp"):
        h.update((ROOT / "paper_2409_06759_amd" / "csrc" / f).read_bytes())
    return h.hexdigest()[:16]


def read_traffic(config: str):
    """HBM bytes per ladder launch from the committed counter summary, if it
    was taken from the current GEMM source."""
    f = ROOT / "profiles" / f"ladder_{config}_traffic.json"
    if not f.exists():
        return None
    try:
        d = json.loads(f.read_text())
    except Exception:
        return None
    if d.get("gemm_source_hash") != source_hash():
        return None
    return d.get("bytes_per_launch")


def cpu_baseline(sysm, method, flops_per_step):
    import numpy as np
    from oracle.cc import Fock, residual
    from oracle.integrals import Integrals
    try:
        from threadpoolctl import threadpool_info
        cores = max((d.get("num_threads", 1) for d in threadpool_info()), default=os.cpu_count())
    except Exception:
        cores = os.cpu_count()
    F, V = Fock.from_system(sysm), Integrals.from_system(sysm)
    o, v = sysm.o, sysm.v
    rng = np.random.default_rng(1)
    t2 = rng.normal(size=(o, o, v, v)) * 1e-3
    t2 = t2 - t2.transpose(1, 0, 2, 3)
    t2 = t2 - t2.transpose(0, 1, 3, 2)
    t1 = rng.normal(size=(o, v)) * 1e-3 if method == "ccsd" else None
    t0 = time.perf_counter()
    residual(F, V, t1, t2)
    el = time.perf_counter() - t0
    return {"value": flops_per_step / el / 1e12, "unit": "TFLOP/s", "cores": int(cores), "kind": "oracle",
            "sample": f"one {method.upper()} residual evaluation (unfactorised einsum oracle, FP64) at "
                      f"o={o} v={v}: {el:.1f} s", "seconds": el}


def bench_batched(ctx, E, torch, steps, warmup):
    """64 uneven systems (o in [4,16], v in [20,60]), one grouped launch per
    step of the contraction list, FP64, FP32 and split-bf16 contractions;
    then all 64 iterated to ||R|| < 1e-8 in FP64."""
    from ccinputs.synth import batch_shapes, make_system
    shapes = batch_shapes(64)
    ds = [E.DeviceSystem(make_system(o, v, seed), drop_host=True) for o, v, seed in shapes]
    out = {"systems": len(ds), "o_range": [min(s[0] for s in shapes), max(s[0] for s in shapes)],
           "v_range": [min(s[1] for s in shapes), max(s[1] for s in shapes)],
           "pairs": "packed (ladder, hole-hole ladder and Z over i<j, a<b, e<f); flops_per_step counts those"}
    for pname in ("f64", "f32", "bf16x3"):
        with E.Batch(ctx, ds, E.CCSD, prec=E.PRECS[pname]) as B:
            B.step(0.0, True)
            torch.cuda.synchronize()
            B.autotune(2)
            for _ in range(warmup):
                B.step(0.0, True)
            torch.cuda.synchronize()
            ts = time.perf_counter()
            for _ in range(steps):
                B.step(0.0, True)
            torch.cuda.synchronize()
            el = (time.perf_counter() - ts) / steps
            fl = B.flops()
            out[pname] = {"ms_per_step": round(el * 1e3, 3), "tflops": round(fl / el / 1e12, 3),
                          "flops_per_step": fl}
        log(f"[bench] batched {pname}: {el * 1e3:.3f} ms/step, {fl / el / 1e12:.2f} TFLOP/s")
    with E.Batch(ctx, ds, E.CCSD) as B:
        r = B.iterate(tol=1e-8, max_iter=300, dressed=True)
        out["time_to_1e-8"] = {"n_converged": r["n_converged"],
                               "seconds": round(max(x["seconds"] for x in r["systems"]), 3),
                               "max_iterations": max(x["iters"] for x in r["systems"])}
    log(f"[bench] batched time to 1e-8: {out['time_to_1e-8']}")
    return out


def bench_shard_share(ctx, E, torch, o=32, v=160, gpus=8):
    """The ladder GEMM one GPU would run if vvvv's (ab) rows were split over
    `gpus` devices: M = o^2, N = v^2 / gpus, K = v^2; best FP64 tile."""
    M, N, K = o * o, v * v // gpus, v * v
    A = torch.randn(M, K, dtype=torch.float64, device="cuda") * 0.01
    B = torch.randn(N, K, dtype=torch.float64, device="cuda") * 0.01
    Cm = torch.zeros(M, N, dtype=torch.float64, device="cuda")
    best = None
    old = os.environ.get("CC_GEMM_TILE")
    try:
        for t in range(E.gemm_tile_count(ctx)):
            os.environ["CC_GEMM_TILE"] = str(t)
            E.gemm(ctx, A, B, Cm, 0.5, 0.0)
            ts = time.perf_counter()
            for _ in range(3):
                E.gemm(ctx, A, B, Cm, 0.5, 0.0)
            el = (time.perf_counter() - ts) / 3
            if best is None or el < best[0]:
                best = (el, t)
    finally:
        if old is None:
            os.environ.pop("CC_GEMM_TILE", None)
        else:
            os.environ["CC_GEMM_TILE"] = old
    el = best[0]
    res = {"M": M, "N": N, "K": K, "ms": round(el * 1e3, 3), "tflops": round(2 * M * N * K / el / 1e12, 2),
           "frac_fp64_peak": round(2 * M * N * K / el / 1e12 / PEAK_FP64_TFLOPS, 4)}
    log(f"[bench] ladder share at {gpus} GPUs: {res}")
    return res


def bench_generated(ctx, E, torch, dsys, builtin_plan, reps=3):
    """The CCSD residual evaluated from the diagram generator's contraction
    list (derived equations, binary ops, cc_plan_create_ops) against the
    built-in factorised table, at the same amplitudes."""
    from paper_2409_06759_amd.codegen.emit import op_list
    t0 = time.perf_counter()
    text = op_list("ccsd", dsys.o, dsys.v)
    t_gen = time.perf_counter() - t0
    t1, t2 = E.zeros_amps(dsys, E.CCSD)
    builtin_plan.step(t1, t2, 0.0, True)
    builtin_plan.step(t1, t2, 0.0, True)
    rb1, rb2, rnb = builtin_plan.residual(t1, t2)
    with E.Plan(ctx, dsys, E.CCSD, ops=text) as p:
        p.autotune(t1, t2, 1)
        r1, r2, rn = p.residual(t1, t2)
        diff = max((r2 - rb2).abs().max().item(), (r1 - rb1).abs().max().item())
        torch.cuda.synchronize()
        ts = time.perf_counter()
        for _ in range(reps):
            p.residual(t1, t2, want_r=False)
        torch.cuda.synchronize()
        el = (time.perf_counter() - ts) / reps
        res = {"ops": text.count("\nop "), "derive_and_emit_seconds": round(t_gen, 3),
               "ms_per_residual": round(el * 1e3, 2), "flops": p.flops(), "tflops": round(p.flops() / el / 1e12, 2),
               "max_abs_diff_vs_builtin": diff, "workspace_gb": round(p.workspace_bytes() / 1e9, 1)}
    log(f"[bench] generated contraction list: {res}")
    return res


def bench_packed(ctx, E, torch, dsys, f64_seconds, steps=10):
    """The same CCSD workload with the ladder over packed pairs (i<j, a<b,
    e<f): step time (TFLOP/s of the packed count) and time to ||R|| < 1e-8
    in FP64 and with split-bf16 contractions plus FP64 refinement."""
    out = {}
    with E.Plan(ctx, dsys, E.CCSD, packed=True) as p:
        t1, t2 = E.zeros_amps(dsys, E.CCSD)
        p.step(t1, t2, 0.0, True)
        p.autotune(t1, t2, 2)
        p.step(t1, t2, 0.0, True)
        p.profile(True)
        torch.cuda.synchronize()
        ts = time.perf_counter()
        for _ in range(steps):
            p.step(t1, t2, 0.0, True)
        torch.cuda.synchronize()
        el = (time.perf_counter() - ts) / steps
        rows = p.profile_table()
        lad = [r for r in rows if r[1] == "GEMM" and r[2].startswith("ladder@")]
        out["ms_per_step"] = round(el * 1e3, 3)
        out["flops_per_step"] = p.flops()
        out["tflops"] = round(p.flops() / el / 1e12, 2)
        if lad:
            lf = p.flops(ladder_only=True)
            out["ladder_ms"] = round(lad[0][5], 3)
            out["ladder_tflops"] = round(lf / (lad[0][5] / 1e3) / 1e12, 2)
    for pname in ("f64", "bf16x3"):
        u1, u2 = E.zeros_amps(dsys, E.CCSD)
        r = E.iterate(ctx, dsys, E.CCSD, u1, u2, tol=1e-8, max_iter=1500, dressed=True, autotune=True,
                      prec=E.PRECS[pname], packed=True)
        out[f"time_to_1e-8_{pname}"] = {"converged": r["converged"], "iterations": r["iters"],
                                        "seconds": round(r["seconds"], 3), "energy": r["energy"],
                                        "speedup_vs_dense_f64": round(f64_seconds / r["seconds"], 3)
                                        if f64_seconds else None}
    log(f"[bench] packed ladder: {out}")
    return out


def bench_ccsdt(ctx, E, torch, o=10, v=40, steps=3):
    """CCSDT iterations from the generated contraction list (t3 stored
    dense, o^3 v^3 elements), bare-denominator Jacobi from t = 0."""
    from ccinputs.synth import make_system
    from paper_2409_06759_amd.codegen.emit import op_list
    d = E.DeviceSystem(make_system(o, v), drop_host=True)
    t1, t2 = E.zeros_amps(d, E.CCSD)
    t3 = torch.zeros((o,) * 3 + (v,) * 3, dtype=torch.float64, device="cuda")
    with E.Plan(ctx, d, E.CCSD, ops=op_list("ccsdt", o, v)) as p:
        p.set_triples(t3)
        p.step(t1, t2, 0.0, False)
        p.autotune(t1, t2, 1)
        torch.cuda.synchronize()
        ts = time.perf_counter()
        for _ in range(steps):
            p.step(t1, t2, 0.0, False)
        torch.cuda.synchronize()
        el = (time.perf_counter() - ts) / steps
        rn, e, _ = p.scalars()
        res = {"o": o, "v": v, "ms_per_iteration": round(el * 1e3, 2), "flops": p.flops(),
               "tflops": round(p.flops() / el / 1e12, 2), "t3_elements": o ** 3 * v ** 3,
               "energy_after": e, "rnorm_after": rn, "iterations": steps + 1}
    log(f"[bench] CCSDT (generated) {res}")
    return res


def bench_complex(ctx, E, torch, steps, warmup, o=40, v=200, precs=("f64", "f32", "bf16x3")):
    """Complex128 Hermitian system: step time and ladder rate per contraction
    precision (FP64: complex MFMA GEMMs; FP32 / split bf16: real GEMMs of
    M x 2N x 2K on realified operands)."""
    from ccinputs.synth import make_system
    t0 = time.time()
    d = E.DeviceSystem(make_system(o, v, is_complex=True), drop_host=True)
    log(f"[bench] complex o={o} v={v} resident ({time.time() - t0:.1f}s)")
    res = {"o": o, "v": v}
    for pname in precs:
        with E.Plan(ctx, d, E.CCSD, prec=E.PRECS[pname]) as plan:
            t1, t2 = E.zeros_amps(d, E.CCSD)
            plan.step(t1, t2, 0.0, True)
            torch.cuda.synchronize()
            plan.autotune(t1, t2, 1)
            for _ in range(warmup):
                plan.step(t1, t2, 0.0, True)
            plan.profile(True)
            torch.cuda.synchronize()
            ts = time.perf_counter()
            for _ in range(steps):
                plan.step(t1, t2, 0.0, True)
            torch.cuda.synchronize()
            el = (time.perf_counter() - ts) / steps
            rows = plan.profile_table()
            plan.profile(False)
            lad = [r for r in rows if r[1] == "GEMM" and r[2].startswith("ladder@")]
            lad_ms = lad[0][5]
            lf = plan.flops(ladder_only=True)
            rn, e, _ = plan.scalars()
            r = {"ms_per_step": round(el * 1e3, 2), "tflops": round(plan.flops() / el / 1e12, 3),
                 "flops_per_step": plan.flops(), "ladder_ms": round(lad_ms, 3),
                 "ladder_tflops": round(lf / (lad_ms / 1e3) / 1e12, 3),
                 "ladder_frac_peak": round(lf / (lad_ms / 1e3) / 1e12 / PEAKS[pname], 4), "steps": steps,
                 "rnorm_last": rn}
            if pname == "f64":
                res.update(r)
                res["ladder_frac_fp64_peak"] = r["ladder_frac_peak"]
            else:
                res[pname] = r
        log(f"[bench] complex {pname}: {r}")
    return res


def bench_complex_converge(ctx, E, torch, o=40, v=200, precs=("f64", "bf16x3", "f32")):
    """Complex o=40 v=200 to ||R|| < 1e-8 (dressed Jacobi from t = 0): FP64,
    and reduced-precision contractions with FP64 refinement (minutes)."""
    from ccinputs.synth import make_system
    d = E.DeviceSystem(make_system(o, v, is_complex=True), drop_host=True)
    out = {"o": o, "v": v}
    os.environ.setdefault("CC_ITERATE_PROGRESS", "50")
    for pname in precs:
        t1, t2 = E.zeros_amps(d, E.CCSD)
        r = E.iterate(ctx, d, E.CCSD, t1, t2, tol=1e-8, max_iter=1500, dressed=True, autotune=True,
                      prec=E.PRECS[pname])
        rec = {"converged": r["converged"], "iterations": r["iters"], "reduced_precision_iterations": r["lowp_iters"],
               "seconds": round(r["seconds"], 3), "setup_seconds": round(r["setup_seconds"], 3),
               "energy_re": r["energy"].real, "energy_im": r["energy"].imag, "rnorm": r["rnorm"]}
        if "f64" in out:
            rec["abs_err_vs_f64"] = abs(r["energy"] - complex(out["f64"]["energy_re"], out["f64"]["energy_im"]))
            rec["speedup_vs_f64"] = round(out["f64"]["seconds"] / r["seconds"], 3)
        out[pname] = rec
        log(f"[bench] complex {pname} to 1e-8: {rec}")
    return out


def bench_learned(ctx, E, torch, dsys, f64_seconds, precs=("f64", "bf16x3")):
    """Time to ||R|| < 1e-8 from the network's start (cc_iterate's MLP guess:
    inference and the MP2 fallback check included) and from the MP2 start,
    against the FP64 run from t = 0."""
    f = ROOT / "paper_2409_06759_amd" / "data" / "mlp_guess.npz"
    if not f.exists():
        return None
    mlp = E.MLP.load(ctx, str(f))
    out = {"params": str(f.relative_to(ROOT))}
    for pname in precs:
        rec = {}
        for start in ("mlp", "mp2"):
            a1, a2 = E.zeros_amps(dsys, E.CCSD)
            r = E.iterate(ctx, dsys, E.CCSD, a1, a2, tol=1e-8, max_iter=1500, dressed=True, autotune=True,
                          prec=E.PRECS[pname], guess=start, mlp=mlp if start == "mlp" else None)
            rec[start] = {"converged": r["converged"], "iterations": r["iters"], "seconds": round(r["seconds"], 3),
                          "guess_seconds": round(r["guess_seconds"], 4), "guess_used": r["guess_used"],
                          "energy": r["energy"],
                          "speedup_vs_f64_from_zero": round(f64_seconds / r["seconds"], 3) if f64_seconds else None}
            if start == "mlp":
                rec["guess_rnorm"] = r["guess_rnorm"]
            log(f"[bench] {start} start + {pname}: {r['iters']} iterations, {r['seconds']:.2f}s "
                f"(guess {r['guess_seconds'] * 1e3:.1f} ms, used {r['guess_used']})")
        rec["speedup_mlp_vs_mp2"] = round(rec["mp2"]["seconds"] / rec["mlp"]["seconds"], 3)
        out[pname] = rec
    out["network"] = bench_network(ctx, E, torch, dsys, mlp)
    return out


# Network flops per sample: two branches (z and z with the integral negated)
# of Linear 3 -> 128, 128 -> 128, 128 -> 1.  Forward: 2 x 2 x 16,896 MACs.
# Training adds per branch the gradients of W3, W2, W1 and the layer-2 input
# (128 + 16,384 + 384 + 16,384 MACs).
NET_FWD_FLOP = 2 * 2 * (3 * 128 + 128 * 128 + 128)
NET_TRAIN_FLOP = NET_FWD_FLOP + 2 * 2 * (128 + 128 * 128 + 3 * 128 + 128 * 128)
FP32_MFMA_PEAK = 157.3e12


def bench_network(ctx, E, torch, dsys, mlp, reps=5):
    """Throughput of the network's kernels on the features of the evaluation
    system: the fused FP32 forward (inference) and one Adam epoch (minibatches
    of 65,536) on a copy of the network."""
    raw = E.MLP.raw_features(ctx, dsys)
    z, _ = mlp.standardise(raw)
    n = z.shape[0]
    mlp.forward(z)
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(reps):
        y = mlp.forward(z)
    torch.cuda.synchronize()
    fwd = (time.perf_counter() - t) / reps
    net = E.MLP(ctx, mlp.params.clone(), mlp.stats, mlp.prec)
    net.train(z, y, epochs=1)
    torch.cuda.synchronize()
    t = time.perf_counter()
    net.train(z, y, epochs=1)
    torch.cuda.synchronize()
    tr = time.perf_counter() - t
    rec = {"samples": n, "forward_ms": round(fwd * 1e3, 3),
           "forward_tflops": round(n * NET_FWD_FLOP / fwd / 1e12, 2),
           "forward_frac_fp32_mfma_peak": round(n * NET_FWD_FLOP / fwd / FP32_MFMA_PEAK, 3),
           "train_epoch_ms": round(tr * 1e3, 2), "train_msamples_per_s": round(n / tr / 1e6, 2),
           "train_tflops": round(n * NET_TRAIN_FLOP / tr / 1e12, 2)}
    log(f"[bench] network: {rec}")
    return rec


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--config", default="c2", choices=sorted(CONFIGS))
    ap.add_argument("--shift", type=float, default=0.0, help="level shift of the Jacobi update")
    ap.add_argument("--bare", action="store_true", help="bare Fock denominators instead of dressed")
    ap.add_argument("--no-converge", action="store_true", help="skip the time-to-1e-8 run")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--max-iter", type=int, default=1500)
    ap.add_argument("--prec", default="f64", choices=["f64", "f32", "bf16x3"],
                    help="contraction precision of the timed steps")
    ap.add_argument("--converge-precs", default="f64,f32,bf16x3",
                    help="precisions whose time to ||R||<1e-8 is reported (reduced ones refine in FP64)")
    ap.add_argument("--extras", default="packed,batched,learned,share,generated,ccsdt,complex",
                    help="comma list of extra workloads reported in the same line: packed (the ladder "
                         "over i<j, a<b, e<f), batched (64 uneven "
                         "systems), learned (time to 1e-8 from the trained network's guess), share (the "
                         "one-GPU share of an 8-GPU ladder), generated (the residual from the diagram "
                         "generator's contraction list), ccsdt (CCSDT o=10 v=40 from the generated list), complex "
                         "(complex128 o=40 v=200 steps per precision), complex_converge (the same system to "
                         "1e-8 per precision; minutes, not in the default list); 'none' for no extras")
    ap.add_argument("--packed", action="store_true",
                    help="time the plan whose ladder, hole-hole ladder and Z run over packed pairs (profiling; "
                         "the flop counts are then the packed ones)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run one plain 1 GiB copy (for HBM counter scaling)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the residual path has no "
              "multi-GPU mode.", file=sys.stderr)
        sys.exit(2)

    import torch
    from ccinputs.synth import make_system
    from paper_2409_06759_amd import engine as E

    cfg = CONFIGS[args.config]
    o, v, method = cfg["o"], cfg["v"], cfg["method"]
    m = E.METHODS[method]
    t0 = time.time()
    sysm = make_system(o, v)
    dsys = E.DeviceSystem(sysm, drop_host=args.no_cpu_baseline)
    log(f"[bench] system o={o} v={v} {method} generated and resident in HBM ({time.time() - t0:.1f}s)")
    ctx = E.Context(0)
    torch.cuda.synchronize()
    t_setup = time.perf_counter()
    # created in the timed precision, as cc_iterate creates its plans (the
    # hole-hole ladder's operand layout follows the creation precision)
    plan = E.Plan(ctx, dsys, m, prec=E.PRECS[args.prec], packed=args.packed)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t_setup
    flops = plan.flops()
    ladder_flops = plan.flops(ladder_only=True)
    t1, t2 = E.zeros_amps(dsys, m)
    dressed = not args.bare
    plan.set_precision(E.PRECS[args.prec])
    plan.step(t1, t2, args.shift, dressed)
    torch.cuda.synchronize()
    t_tune = time.perf_counter()
    plan.autotune(t1, t2, 2)
    torch.cuda.synchronize()
    tune_s = time.perf_counter() - t_tune
    log(f"[bench] plan setup {setup_s:.2f}s, autotune {tune_s:.2f}s")
    for _ in range(args.warmup):
        plan.step(t1, t2, args.shift, dressed)
    torch.cuda.synchronize()
    log(f"[bench] warmup done ({args.warmup} steps)")

    plan.profile(True)
    torch.cuda.synchronize()
    ts = time.perf_counter()
    for _ in range(args.steps):
        plan.step(t1, t2, args.shift, dressed)
    torch.cuda.synchronize()
    el = time.perf_counter() - ts
    rows = plan.profile_table()
    plan.profile(False)
    ms_per_step = el / args.steps * 1e3
    value = flops / (el / args.steps) / 1e12
    lad = [r for r in rows if r[1] == "GEMM" and r[2].startswith("ladder@")]
    lad_ms = lad[0][5] if lad else float("nan")
    achieved = ladder_flops / (lad_ms / 1e3) / 1e12 if lad else None
    log(f"[bench] {args.steps} steps: {ms_per_step:.2f} ms/step, {value:.2f} TFLOP/s; ladder {lad_ms:.3f} ms "
        f"({achieved:.2f} TFLOP/s)")
    top = sorted(rows, key=lambda r: -r[4])[:8]
    for r in top:
        log(f"[bench]   {r[1]:8s} {r[2]:44s} {r[5]:8.3f} ms")

    if args.copy_calibration:
        n = 1 << 27  # 1 GiB of doubles, copied by the library's flat permute kernel
        src = torch.ones(n, dtype=torch.float64, device="cuda")
        E.permute(ctx, src, (0,))
        torch.cuda.synchronize()
        log("[bench] copy calibration: 1 GiB read + 1 GiB write")

    conv = {}
    if not args.no_converge:
        gold = ROOT / "tests" / "golden" / f"{args.config}_{method}_energy.json"
        g = json.loads(gold.read_text()) if gold.exists() else None
        for pname in [x for x in args.converge_precs.split(",") if x]:
            u1, u2 = E.zeros_amps(dsys, m)
            out = E.iterate(ctx, dsys, m, u1, u2, tol=1e-8, max_iter=args.max_iter, level_shift=args.shift,
                            dressed=dressed, use_graph=True, prec=E.PRECS[pname], autotune=True)
            rec = {"converged": out["converged"], "iterations": out["iters"],
                   "reduced_precision_iterations": out["lowp_iters"], "seconds": round(out["seconds"], 3),
                   "setup_seconds": round(out["setup_seconds"], 3), "energy": out["energy"], "rnorm": out["rnorm"]}
            if g is not None:
                rec["oracle_energy"] = g["energy"]
                rec["abs_err_vs_oracle"] = abs(out["energy"] - g["energy"])
            if "f64" in conv:
                rec["abs_err_vs_f64"] = abs(out["energy"] - conv["f64"]["energy"])
                rec["speedup_vs_f64"] = round(conv["f64"]["seconds"] / out["seconds"], 3)
            conv[pname] = rec
            log(f"[bench] {pname}: time to ||R||<1e-8 {out['seconds']:.2f}s, {out['iters']} iterations "
                f"({out['lowp_iters']} reduced), E={out['energy']:.10f}")

    extras = {}
    plan_closed = False
    for name in [x for x in args.extras.split(",") if x and x != "none"]:
        if name == "batched":
            extras["batched"] = bench_batched(ctx, E, torch, max(args.steps, 5), args.warmup)
        elif name == "learned":
            if args.config == "c2":
                f64s = conv.get("f64", {}).get("seconds")
                extras["learned"] = bench_learned(ctx, E, torch, dsys, f64s)
        elif name == "generated":
            if method == "ccsd" and not plan_closed:
                extras["generated"] = bench_generated(ctx, E, torch, dsys, plan)
        elif name == "share":
            extras["ladder_share_g8"] = bench_shard_share(ctx, E, torch, o, v)
        elif name == "packed":
            if args.config == "c2":
                extras["packed_ladder"] = bench_packed(ctx, E, torch, dsys, conv.get("f64", {}).get("seconds"))
        elif name == "ccsdt":
            extras["ccsdt"] = bench_ccsdt(ctx, E, torch)
        elif name == "complex":
            plan.close()
            plan_closed = True
            extras["complex"] = bench_complex(ctx, E, torch, 3, 1)
        elif name == "complex_converge":
            plan.close()
            plan_closed = True
            extras["complex_converge"] = bench_complex_converge(ctx, E, torch)
        else:
            raise SystemExit(f"unknown extra workload {name}")

    cpu = None
    if not args.no_cpu_baseline:
        log("[bench] timing the CPU oracle (one residual evaluation)...")
        cpu = cpu_baseline(sysm, method, flops)
        log(f"[bench] oracle: {cpu['seconds']:.1f}s per residual -> {cpu['value']:.4f} TFLOP/s")
        f64c = conv.get("f64")
        if f64c:
            # the oracle's Jacobi loop is one residual per iteration (plus the
            # dressed diagonals, a few o^2 v^2 einsums): its time to 1e-8 on the
            # same host threads is about iterations x one residual
            cpu["time_to_1e-8_extrapolated_s"] = round(cpu["seconds"] * f64c["iterations"], 1)

    line = {
        "metric": "CCSD residual TFLOP/s & time-to-1e-8 convergence, FP64 vs mixed/learned",
        "value": round(value, 3), "unit": "TFLOP/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3), "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": args.prec, "data": "synthetic",
        "config": {"workload": f"{method} o={o} v={v} fp64 real, seeded antisymmetrised <pq||rs>~N(0,0.01^2), "
                               f"diagonal Fock", "o": o, "v": v, "method": method,
                   "update": ("dressed" if dressed else "bare") + f" Jacobi, shift {args.shift}",
                   "pairs": "packed" if args.packed else "dense",
                   "flops_per_step": flops},
        "roofline": {"bound": "mfma", "achieved": round(achieved, 3) if achieved else None,
                     "peak": round(PEAKS[args.prec], 1), "unit": "TFLOP/s",
                     "frac": round(achieved / PEAKS[args.prec], 4) if achieved else None,
                     "traffic": read_traffic(args.config) if args.prec == "f64" else None,
                     "kernel": f"ladder GEMM ({args.prec} MFMA)",
                     "avg_ms": round(lad_ms, 4), "flops_per_launch": ladder_flops},
        "cpu_baseline": ({k: cpu[k] for k in ("value", "unit", "cores", "kind", "sample", "time_to_1e-8_extrapolated_s")
                          if k in cpu} if cpu else None),
        "time_to_1e-8": conv or None,
        "setup": {"plan_seconds": round(setup_s, 3), "autotune_seconds": round(tune_s, 3),
                  "note": "outside the timed steps and outside every time_to_1e-8 'seconds' (each run's own plan "
                          "creation and autotuning are its 'setup_seconds')"},
    }
    line.update(extras)
    print(json.dumps(line), flush=True)
    plan.close()
    ctx.close()


if __name__ == "__main__":
    main()
