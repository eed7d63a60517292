"""Write reference energies computed by the CPU oracle (and nothing else).

    python tests/golden/make_reference.py c1     # CCD o=8 v=24, 10 Jacobi iterations
    python tests/golden/make_reference.py c2     # CCSD o=32 v=160 to ||R|| < 1e-8 (hours)
    python tests/golden/make_reference.py c3     # complex CCSD o=40 v=200: sampled residual

The C2 run uses the dressed-denominator Jacobi update without level shift,
starting from t = 0, and records E(t_n) and ||R(t_n)|| for every iteration
plus the energy at the first iterate with ||R|| < 1e-8, and then continues
to ||R|| < 1e-10 for a tighter value of the converged energy.
"""
import json
import os
import pathlib
import sys
import time

HERE = pathlib.Path(__file__).resolve().parent
sys.path.insert(0, str(HERE.parents[1]))

import numpy as np  # noqa: E402

from ccinputs.synth import make_system, random_amplitudes  # noqa: E402
from oracle.cc import Fock, energy, jacobi, residual, residual_norm  # noqa: E402
from oracle.integrals import Integrals  # noqa: E402


def complex_sample(o=40, v=200, amp_seed=7, n2=2048, n1=256):
    """Residual and energy of complex CCSD at seeded random amplitudes; the
    norm, the energy, max |R2| and a seeded sample of R1 and R2 elements."""
    t0 = time.time()
    s = make_system(o, v, is_complex=True)
    F, V = Fock.from_system(s), Integrals.from_system(s)
    t1, t2 = random_amplitudes(o, v, amp_seed, is_complex=True)
    print(f"inputs {time.time() - t0:.0f}s", flush=True)
    e = energy(F, V, t1, t2)
    r1, r2 = residual(F, V, t1, t2)
    print(f"residual {time.time() - t0:.0f}s", flush=True)
    rng = np.random.Generator(np.random.PCG64(amp_seed + 1))
    i2 = np.sort(rng.choice(r2.size, size=n2, replace=False))
    i1 = np.sort(rng.choice(r1.size, size=n1, replace=False))
    pair = lambda z: [[float(x.real), float(x.imag)] for x in z]  # noqa: E731
    out = {"config": f"complex CCSD o={o} v={v}, seeded integrals (base seed), amplitudes "
                     f"random_amplitudes(o, v, seed={amp_seed}, scale=0.01, is_complex=True)",
           "o": o, "v": v, "amp_seed": amp_seed, "amp_scale": 0.01,
           "fingerprint": {"t2_sum_abs": float(np.abs(t2).sum()), "vvvv_0123": pair([V.get("vvvv")[0, 1, 2, 3]])[0]},
           "energy": [float(e.real), float(e.imag)], "rnorm": residual_norm(r1, r2),
           "r2_max_abs": float(np.abs(r2).max()), "r1_max_abs": float(np.abs(r1).max()),
           "r2_index": i2.tolist(), "r2": pair(r2.ravel()[i2]), "r1_index": i1.tolist(), "r1": pair(r1.ravel()[i1]),
           "oracle_seconds": round(time.time() - t0, 1)}
    (HERE / f"c3_complex_o{o}_v{v}_sample.json").write_text(json.dumps(out))


def main(which):
    if which == "c3":
        complex_sample(*[int(x) for x in sys.argv[2:4]])
        return
    if which == "c1":
        s = make_system(8, 24)
        r = jacobi(Fock.from_system(s), Integrals.from_system(s), "ccd", tol=0.0, max_iter=10)
        out = {"config": "CCD o=8 v=24 fp64, t=0 start, bare Jacobi", "hist_e": r["hist_e"],
               "hist_rnorm": r["hist_r"]}
        (HERE / "c1_ccd_trajectory.json").write_text(json.dumps(out, indent=1))
        return
    s = make_system(32, 160)
    F, V = Fock.from_system(s), Integrals.from_system(s)
    t0 = time.time()
    log = open(HERE / "c2_progress.log", "w") if os.environ.get("CC_GOLDEN_LOG") else None

    def cb(it, e, rn):
        msg = f"{it} {rn:.6e} {e:.13f} {time.time() - t0:.0f}s"
        print(msg, flush=True)
        if log:
            log.write(msg + "\n")
            log.flush()

    r = jacobi(F, V, "ccsd", tol=1e-8, max_iter=400, dressed=True, callback=cb)
    out = {"config": "CCSD o=32 v=160 fp64, t=0 start, dressed-denominator Jacobi, shift 0",
           "energy": r["energy"], "iterations": r["iters"], "rnorm": r["rnorm"], "converged": r["converged"],
           "hist_e": r["hist_e"], "hist_rnorm": r["hist_r"]}
    (HERE / "c2_ccsd_energy.json").write_text(json.dumps(out, indent=1))
    r2 = jacobi(F, V, "ccsd", tol=1e-10, max_iter=200, dressed=True, t1=r["t1"], t2=r["t2"], callback=cb)
    out["energy_tight"] = r2["energy"]
    out["rnorm_tight"] = r2["rnorm"]
    (HERE / "c2_ccsd_energy.json").write_text(json.dumps(out, indent=1))


if __name__ == "__main__":
    main(sys.argv[1] if len(sys.argv) > 1 else "c1")
