"""Write reference energies computed by the CPU oracle (and nothing else).

    python tests/golden/make_reference.py c1     # CCD o=8 v=24, 10 Jacobi iterations
    python tests/golden/make_reference.py c2     # CCSD o=32 v=160 to ||R|| < 1e-8 (hours)

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

from ccinputs.synth import make_system  # noqa: E402
from oracle.cc import Fock, jacobi  # noqa: E402
from oracle.integrals import Integrals  # noqa: E402


def main(which):
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
