"""NumPy interpreter of the planner's step listing (cc_plan_describe_dry /
cc_plan_describe_ops_dry) for CPU checks of a plan's semantics."""
import re

import numpy as np
from numpy.lib.stride_tricks import as_strided

from ccinputs.synth import make_system
from oracle.cc import Fock, residual
from oracle.integrals import Integrals


def _parse(txt):
    sec, steps, slots, alias = None, {"setup": [], "iteration": []}, {}, {}
    for line in txt.splitlines():
        if line.startswith("# "):
            sec = line[2:]
            continue
        if sec in steps:
            steps[sec].append(line)
        elif sec == "slots":
            name, rest = line.split(" ", 1)
            slots[name] = [int(x) for x in re.search(r"dims=([\d,]+)", rest).group(1).split(",")]
        elif sec == "aliases":
            a, b = line.split(" -> ")
            alias[a] = b
    return steps, slots, alias


def _kv(line):
    return dict(re.findall(r"(\w+)=([^ ]+)", line))


def _ints(s):
    return [int(x) for x in s.split(",")]


def execute(listing, inputs, o, v, cplx, method):
    """Run the setup and iteration steps of a listing on NumPy buffers.
    `inputs` maps stored tensor names (foo, fov, fvv, the six integral
    blocks, t1, t2, t3) to arrays; returns a getter name -> flat array."""
    steps, slots, alias = _parse(listing)
    dt = np.complex128 if cplx else np.float64
    mem = {k: np.full(int(np.prod(d)), np.nan, dtype=dt) for k, d in slots.items()}
    for k, a in inputs.items():
        if a is not None and k in mem:
            mem[k] = np.ascontiguousarray(a, dtype=dt).ravel().copy()
    it = np.dtype(dt).itemsize
    get = lambda name: mem[alias.get(name, name)]  # noqa: E731
    for line in steps["setup"] + steps["iteration"]:
        kind, p = line.split(" ")[0], _kv(line)
        if kind == "PERMUTE":
            od = _ints(p["out_dims"])
            x = as_strided(get(p["src"]), od, [q * it for q in _ints(p["in_strides"])])
            if int(p["conj"]):
                x = np.conj(x)
            y = as_strided(get(p["dst"]), od, [q * it for q in _ints(p["out_strides"])])
            y[...] = float(p["alpha"]) * x + (float(p["beta"]) * y if float(p["beta"]) else 0)
        elif kind == "GEMM":
            M, N, K = int(p["M"]), int(p["N"]), int(p["K"])
            a = as_strided(get(p["A"]), (M, K), (int(p["sam"]) * it, int(p["sak"]) * it))
            b = as_strided(get(p["B"]), (N, K), (int(p["sbn"]) * it, int(p["sbk"]) * it))
            c = as_strided(get(p["C"]), (M, N), (int(p["ldc"]) * it, it))
            c[...] = float(p["alpha"]) * (a @ b.T) + (float(p["beta"]) * c if float(p["beta"]) else 0)
        elif kind == "OUTER":
            d = _ints(p["dims"])
            a = as_strided(get(p["A"]), d, [q * it for q in _ints(p["sa"])])
            b = as_strided(get(p["B"]), d, [q * it for q in _ints(p["sb"])])
            get(p["C"]).reshape(d)[...] += float(p["alpha"]) * a * b
        elif kind == "FILL":
            get(line.split(" ")[1])[:] = 0
        elif kind == "SPECIAL" and line.split(" ")[1] == "tau_energy" and method == 1:
            T1, T2 = get("t1").reshape(o, v), get("t2").reshape(o, o, v, v)
            x = np.einsum("ia,jb->ijab", T1, T1)
            x = x - x.transpose(0, 1, 3, 2)
            get("tau")[:] = (T2 + x).ravel()
            get("taut")[:] = (T2 + 0.5 * x).ravel()
    return get


def doubles(get, o, v):
    """R2 from the four accumulators, as the assembly kernel forms it."""
    XP, Xij, Xab, Xr = [get(k).reshape(o, o, v, v) for k in ("XP", "Xij", "Xab", "Xr")]
    R2 = XP + (Xij - Xij.transpose(1, 0, 2, 3)) + (Xab - Xab.transpose(0, 1, 3, 2))
    Q = Xr - Xr.transpose(1, 0, 2, 3)
    return R2 + Q - Q.transpose(0, 1, 3, 2)


def triples(get, o, v):
    """R3 = full antisymmetriser of Y3, as the triples kernel forms it."""
    import itertools
    Y = get("Y3").reshape((o,) * 3 + (v,) * 3)
    R = np.zeros_like(Y)
    for ph in itertools.permutations(range(3)):
        for pp in itertools.permutations(range(3)):
            sg = round(np.linalg.det(np.eye(3)[list(ph)]) * np.linalg.det(np.eye(3)[list(pp)]))
            R = R + sg * np.transpose(Y, list(ph) + [3 + q for q in pp])
    return R


def run_listing(listing, o, v, method, cplx, seed=3):
    """Execute the listing on a random system and amplitudes; return
    (R1 or None, R2, oracle R1, oracle R2)."""
    steps, slots, alias = _parse(listing)
    dt = np.complex128 if cplx else np.float64
    s = make_system(o, v, seed, is_complex=cplx, sigma=0.1)
    rng = np.random.default_rng(7)
    n = o + v
    F = s.fock()
    X = rng.normal(size=(n, n)) * 0.1 + (1j * rng.normal(size=(n, n)) * 0.1 if cplx else 0)
    F = F + X + X.conj().T
    Fk = Fock(F[:o, :o], F[:o, o:], F[o:, o:])
    V = Integrals.from_system(s)
    t1 = rng.normal(size=(o, v)) * 0.1 + (1j * rng.normal(size=(o, v)) * 0.1 if cplx else 0)
    t2 = rng.normal(size=(o, o, v, v)) * 0.1 + (1j * rng.normal(size=(o, o, v, v)) * 0.1 if cplx else 0)
    t2 = t2 - t2.transpose(1, 0, 2, 3)
    t2 = t2 - t2.transpose(0, 1, 3, 2)
    if method == 0:
        t1 = None
    mem = {k: np.full(int(np.prod(d)), np.nan, dtype=dt) for k, d in slots.items()}
    init = {"foo": Fk.oo, "fov": Fk.ov, "fvv": Fk.vv, "t2": t2}
    if t1 is not None:
        init["t1"] = t1
    for b in ("oooo", "ooov", "oovv", "ovvo", "ovvv", "vvvv"):
        init[b] = V.get(b)
    for k, a in init.items():
        mem[k] = np.ascontiguousarray(a, dtype=dt).ravel().copy()
    it = np.dtype(dt).itemsize
    get = lambda name: mem[alias.get(name, name)]  # noqa: E731
    for line in steps["setup"] + steps["iteration"]:
        kind, p = line.split(" ")[0], _kv(line)
        if kind == "PERMUTE":
            od = _ints(p["out_dims"])
            x = as_strided(get(p["src"]), od, [q * it for q in _ints(p["in_strides"])])
            if int(p["conj"]):
                x = np.conj(x)
            y = as_strided(get(p["dst"]), od, [q * it for q in _ints(p["out_strides"])])
            y[...] = float(p["alpha"]) * x + (float(p["beta"]) * y if float(p["beta"]) else 0)
        elif kind == "GEMM":
            M, N, K = int(p["M"]), int(p["N"]), int(p["K"])
            a = as_strided(get(p["A"]), (M, K), (int(p["sam"]) * it, int(p["sak"]) * it))
            b = as_strided(get(p["B"]), (N, K), (int(p["sbn"]) * it, int(p["sbk"]) * it))
            c = as_strided(get(p["C"]), (M, N), (int(p["ldc"]) * it, it))
            c[...] = float(p["alpha"]) * (a @ b.T) + (float(p["beta"]) * c if float(p["beta"]) else 0)
        elif kind == "OUTER":
            d = _ints(p["dims"])
            a = as_strided(get(p["A"]), d, [q * it for q in _ints(p["sa"])])
            b = as_strided(get(p["B"]), d, [q * it for q in _ints(p["sb"])])
            get(p["C"]).reshape(d)[...] += float(p["alpha"]) * a * b
        elif kind == "FILL":
            get(line.split(" ")[1])[:] = 0
        elif kind == "SPECIAL" and line.split(" ")[1] == "tau_energy" and method == 1:
            T1, T2 = get("t1").reshape(o, v), get("t2").reshape(o, o, v, v)
            x = np.einsum("ia,jb->ijab", T1, T1)
            x = x - x.transpose(0, 1, 3, 2)
            get("tau")[:] = (T2 + x).ravel()
            get("taut")[:] = (T2 + 0.5 * x).ravel()
    XP, Xij, Xab, Xr = [get(k).reshape(o, o, v, v) for k in ("XP", "Xij", "Xab", "Xr")]
    R2 = XP + (Xij - Xij.transpose(1, 0, 2, 3)) + (Xab - Xab.transpose(0, 1, 3, 2))
    Q = Xr - Xr.transpose(1, 0, 2, 3)
    R2 = R2 + Q - Q.transpose(0, 1, 3, 2)
    r1_ref, r2_ref = residual(Fk, V, t1, t2)
    R1 = get("R1").reshape(o, v) if method == 1 else None
    return R1, R2, r1_ref, r2_ref
