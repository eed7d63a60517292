"""Host-side checks that need no GPU: the C ABI library loads and exports
every declared symbol, error paths that need no device, and the planner's
step listing (executed here by a small NumPy interpreter of the listing)
reproduces the oracle residual."""
import re
import pathlib
import ctypes as C

import numpy as np
import pytest
from numpy.lib.stride_tricks import as_strided

from ccinputs.synth import make_system
from oracle.cc import Fock, residual
from oracle.integrals import Integrals

ROOT = pathlib.Path(__file__).resolve().parents[1]


def _lib():
    from paper_2409_06759_amd import _lib as L
    return L, L.load()


def _has_gpu():
    try:
        import torch
        return torch.cuda.device_count() > 0
    except Exception:
        return False


def test_header_symbols_exported():
    L, lib = _lib()
    hdr = (ROOT / "include" / "cc.h").read_text()
    declared = set(re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\s*\*?\s*(cc_[a-z0-9_]+)\s*\(", hdr, re.M))
    assert declared, "no declarations parsed"
    assert declared == set(L.EXPORTS), declared ^ set(L.EXPORTS)
    for name in declared:
        assert hasattr(lib, name), name


def test_status_strings():
    L, lib = _lib()
    assert lib.cc_status_string(0) == b"ok"
    assert lib.cc_status_string(L.CC_EDIVERGED) == b"diverged"
    assert lib.cc_status_string(12345) == b"unknown status"


@pytest.mark.skipif(_has_gpu(), reason="checks the no-device path")
def test_create_without_device_reports_edevice():
    L, lib = _lib()
    h = C.c_void_p()
    assert lib.cc_create(C.byref(h), 0, None) == L.CC_EDEVICE
    assert not h.value
    assert b"device" in lib.cc_last_error(None)


def test_null_arguments_rejected():
    L, lib = _lib()
    assert lib.cc_create(None, 0, None) == L.CC_EINVAL
    assert lib.cc_plan_residual(None, None, None, None) == L.CC_EINVAL
    assert lib.cc_iterate(None, None, 0, None, None, None) == L.CC_EINVAL
    assert lib.cc_destroy(None) == 0


def test_dry_plan_rejects_bad_sizes():
    _, lib = _lib()
    assert lib.cc_plan_describe_dry(0, 5, 1, 0).startswith(b"error")
    assert lib.cc_plan_describe_dry(3, 5, 7, 0).startswith(b"error")


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


def test_ladder_is_one_direct_gemm():
    _, lib = _lib()
    o, v = 6, 20
    steps, slots, _ = _parse(lib.cc_plan_describe_dry(o, v, 1, 0).decode())
    lad = [s for s in steps["iteration"] if s.startswith("GEMM ladder ")]
    assert len(lad) == 1
    p = _kv(lad[0])
    assert (int(p["M"]), int(p["N"]), int(p["K"])) == (o * o, v * v, v * v)
    assert p["A"] == "tau" and p["B"] == "vvvv" and p["C"] == "XP" and float(p["alpha"]) == 0.5
    assert int(p["sak"]) == 1 and int(p["sbk"]) == 1  # both operands K-contiguous
    # the four-virtual block is never copied or permuted
    assert not any("src=vvvv" in s for s in steps["setup"] + steps["iteration"])


@pytest.mark.parametrize("method", [0, 1])
@pytest.mark.parametrize("cplx", [False, True])
@pytest.mark.parametrize("ov", [(4, 7), (1, 4), (2, 1), (1, 1), (3, 2)])
def test_plan_listing_reproduces_oracle(method, cplx, ov):
    """Interpret the planner's steps with NumPy; compare with the oracle
    (including the degenerate sizes with no i<j or no a<b pair)."""
    _, lib = _lib()
    o, v = ov
    steps, slots, alias = _parse(lib.cc_plan_describe_dry(o, v, method, 1 if cplx else 0).decode())
    dt = np.complex128 if cplx else np.float64
    s = make_system(o, v, 3, is_complex=cplx, sigma=0.1)
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
    assert np.abs(R2 - r2_ref).max() < 1e-13
    if method == 1:
        assert np.abs(get("R1").reshape(o, v) - r1_ref).max() < 1e-13
