"""Host-side checks that need no GPU: the C ABI library loads and exports
every declared symbol, error paths that need no device, and the planner's
step listing (executed here by a small NumPy interpreter of the listing)
reproduces the oracle residual."""
import re
import pathlib
import ctypes as C

import numpy as np
import pytest


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


def test_tile_counts():
    """Configuration counts for the forced-tile sweeps (no device needed)."""
    L, lib = _lib()
    for prec in (L.CC_PREC_F64, L.CC_PREC_F32, L.CC_PREC_BF16X3):
        assert lib.cc_gemm_tile_count(prec) > 1
    assert lib.cc_gemm_tile_count(7) == -1
    assert lib.cc_gemm_tile_count_c128() > 1


def test_dry_plan_rejects_bad_sizes():
    _, lib = _lib()
    assert lib.cc_plan_describe_dry(0, 5, 1, 0).startswith(b"error")
    assert lib.cc_plan_describe_dry(3, 5, 7, 0).startswith(b"error")


from plan_interp import _kv, _parse, run_listing  # noqa: E402


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
    R1, R2, r1_ref, r2_ref = run_listing(lib.cc_plan_describe_dry(o, v, method, 1 if cplx else 0).decode(), o, v,
                                         method, cplx)
    assert np.abs(R2 - r2_ref).max() < 1e-13
    if method == 1:
        assert np.abs(R1 - r1_ref).max() < 1e-13


def test_m0_check_flags_violations():
    """The build-time check of the LDS-direct loads accepts the inline
    sequence and rejects a stray M0 write, an implicit M0 reader and a load
    without its M0 write."""
    from paper_2409_06759_amd.check_m0 import check_text
    good = ("0000000000001000 <k>:\n  s_mov_b32 m0, s4 // x\n  s_nop 0\n  global_load_lds_dwordx4 v[0:1], off\n"
            "  v_mfma_f64_16x16x4_f64 v[2:9], v[10:11], v[12:13], v[2:9]\n")
    assert check_text(good) == (1, [])
    for extra in ("  s_mov_b32 m0, -1\n", "  s_movrels_b32 s0, s1\n", "  global_load_lds_dwordx4 v[0:1], off\n",
                  "  s_sendmsg sendmsg(MSG_INTERRUPT)\n"):
        n, bad = check_text(good + extra)
        assert n == 1 and len(bad) == 1, extra
    # kernels without LDS-direct loads are not constrained
    assert check_text("0000000000002000 <j>:\n  s_mov_b32 m0, -1\n  ds_read_b64 v[0:1], v2\n") == (0, [])
