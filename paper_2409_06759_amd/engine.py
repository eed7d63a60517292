"""Python front end of the engine: device tensors from PyTorch, every
computation in the HIP library behind ``include/cc.h``."""
from __future__ import annotations

import ctypes as C
from typing import Optional

import numpy as np
import torch

from . import _lib as L

CCD, CCSD = L.CC_CCD, L.CC_CCSD
F64, F32, BF16X3 = L.CC_PREC_F64, L.CC_PREC_F32, L.CC_PREC_BF16X3
METHODS = {"ccd": CCD, "ccsd": CCSD}
PRECS = {"f64": F64, "f32": F32, "bf16x3": BF16X3}


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else C.c_void_p(t.data_ptr())


class Context:
    """A library context bound to one device and one stream (torch's
    current stream of that device unless given)."""

    def __init__(self, device: int = 0, stream: Optional["torch.cuda.Stream"] = None):
        self.lib = L.load()
        self.device = device
        # A stream of its own (default priority) so that one iteration can be
        # captured as a graph; every call is ordered against torch's current
        # stream on entry and exit.
        self.stream = stream if stream is not None else torch.cuda.Stream(device=device)
        self.h = C.c_void_p()
        rc = self.lib.cc_create(C.byref(self.h), device, C.c_void_p(self.stream.cuda_stream))
        if rc != 0:
            raise L.CCError(rc, self.lib.cc_last_error(None).decode())

    def check(self, rc: int, ok=(0,)):
        cur = torch.cuda.current_stream(self.device)
        cur.wait_stream(self.stream)
        if rc not in ok:
            raise L.CCError(rc, self.lib.cc_last_error(self.h).decode())
        return rc

    def enter(self):
        """Order the library stream after the work queued so far by torch."""
        self.stream.wait_stream(torch.cuda.current_stream(self.device))

    def close(self):
        if self.h:
            self.lib.cc_destroy(self.h)
            self.h = C.c_void_p()

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


class DeviceSystem:
    """Fock and integral blocks of one system resident in device memory."""

    NAMES = ("f_oo", "f_ov", "f_vv", "oooo", "ooov", "oovv", "ovvo", "ovvv", "vvvv")

    def __init__(self, sysm, device: str = "cuda", drop_host: bool = False):
        self.o, self.v = sysm.o, sysm.v
        self.is_complex = sysm.is_complex
        self.dtype = torch.complex128 if sysm.is_complex else torch.float64
        self.t = {}
        for n in self.NAMES:
            if n.startswith("f_"):
                arr = getattr(sysm, n)
            else:
                arr = sysm.block(n)
            self.t[n] = torch.from_numpy(np.ascontiguousarray(arr)).to(device)
            if drop_host and not n.startswith("f_"):
                sysm.drop(n)
        self.struct = L.CCSystemStruct(self.o, self.v, L.CC_C128 if self.is_complex else L.CC_R64,
                                       *[self.t[n].data_ptr() for n in self.NAMES])

    @classmethod
    def from_tensors(cls, o, v, tensors: dict):
        self = cls.__new__(cls)
        self.o, self.v = o, v
        self.dtype = tensors["oovv"].dtype
        self.is_complex = self.dtype == torch.complex128
        self.t = {n: tensors[n].contiguous() for n in cls.NAMES}
        self.struct = L.CCSystemStruct(o, v, L.CC_C128 if self.is_complex else L.CC_R64,
                                       *[self.t[n].data_ptr() for n in cls.NAMES])
        return self


def zeros_amps(dsys: DeviceSystem, method: int):
    o, v = dsys.o, dsys.v
    dev = dsys.t["oovv"].device
    t2 = torch.zeros((o, o, v, v), dtype=dsys.dtype, device=dev)
    t1 = torch.zeros((o, v), dtype=dsys.dtype, device=dev) if method == CCSD else None
    return t1, t2


def _amps(t1, t2):
    return L.CCAmps(None if t1 is None else t1.data_ptr(), t2.data_ptr())


class Plan:
    """A planned residual (cc_plan_create), or, with `ops`, one built from a
    contraction list such as `codegen.emit.op_list` (cc_plan_create_ops)."""

    def __init__(self, ctx: Context, dsys: DeviceSystem, method: int = CCSD, prec: int = F64,
                 ops: Optional[str] = None, packed: bool = False, lowp_all: bool = False):
        self.ctx, self.dsys, self.method = ctx, dsys, method
        self.h = C.c_void_p()
        ctx.enter()
        if ops is None:
            flags = (1 if packed else 0) | (2 if lowp_all else 0)
            ctx.check(ctx.lib.cc_plan_create2(ctx.h, C.byref(dsys.struct), method, prec, flags, C.byref(self.h)))
        else:
            ctx.check(ctx.lib.cc_plan_create_ops(ctx.h, C.byref(dsys.struct), method, prec, ops.encode(),
                                                 C.byref(self.h)))

    def residual(self, t1, t2, want_r=True):
        r1 = r2 = None
        if want_r:
            r2 = torch.empty_like(t2)
            r1 = torch.empty_like(t1) if t1 is not None else None
        rn = C.c_double()
        ra = _amps(r1, r2) if want_r else None
        self.ctx.enter()
        self.ctx.check(self.ctx.lib.cc_plan_residual(self.h, C.byref(_amps(t1, t2)),
                                                     C.byref(ra) if ra is not None else None,
                                                     C.byref(rn)))
        return r1, r2, rn.value

    def step(self, t1, t2, shift: float = 0.0, dressed: bool = False):
        self.ctx.enter()
        self.ctx.check(self.ctx.lib.cc_plan_step(self.h, C.byref(_amps(t1, t2)), shift,
                                                 1 if dressed else 0))

    def scalars(self):
        rn, er, ei = C.c_double(), C.c_double(), C.c_double()
        self.ctx.check(self.ctx.lib.cc_plan_scalars(self.h, C.byref(rn), C.byref(er), C.byref(ei)))
        return rn.value, er.value, ei.value

    def describe(self) -> str:
        return self.ctx.lib.cc_plan_describe(self.h).decode()

    def flops(self, ladder_only=False) -> float:
        return self.ctx.lib.cc_plan_flops(self.h, 1 if ladder_only else 0)

    def autotune(self, t1, t2, reps: int = 2):
        self.ctx.enter()
        self.ctx.check(self.ctx.lib.cc_plan_autotune(self.h, C.byref(_amps(t1, t2)), reps))

    def set_triples(self, t3, r3=None):
        """Bind t3 (and optionally an R3 output) for a plan whose op list has
        triples (cc_plan_set_triples)."""
        self._triples = (t3, r3)
        self.ctx.check(self.ctx.lib.cc_plan_set_triples(self.h, _ptr(t3), _ptr(r3)))

    def set_precision(self, prec: int):
        self.ctx.check(self.ctx.lib.cc_plan_set_precision(self.h, prec))

    def set_correction(self, mode: int, prec: int = F32):
        """1: the next FP64 step takes a reference, later ones add a
        reduced-precision correction to it (cc_plan_set_correction)."""
        self.ctx.check(self.ctx.lib.cc_plan_set_correction(self.h, mode, prec))

    def profile(self, enable: bool = True):
        self.ctx.check(self.ctx.lib.cc_plan_profile(self.h, 1 if enable else 0))

    def profile_table(self):
        """[(index, kind, tag, calls, total_ms, avg_ms, flops_per_call)]"""
        rows = []
        for line in self.ctx.lib.cc_plan_profile_table(self.h).decode().splitlines():
            if line.startswith("#") or not line.strip():
                continue
            i, kind, tag, calls, tot, avg, fl = line.split()
            rows.append((int(i), kind, tag, int(calls), float(tot), float(avg), float(fl)))
        return rows

    def workspace_bytes(self) -> int:
        return self.ctx.lib.cc_plan_workspace_bytes(self.h)

    def close(self):
        if self.h:
            self.ctx.lib.cc_plan_destroy(self.h)
            self.h = C.c_void_p()

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


def residual(ctx, dsys, method, t1, t2, prec=F64):
    r2 = torch.empty_like(t2)
    r1 = torch.empty_like(t1) if t1 is not None else None
    rn = C.c_double()
    ctx.enter()
    ctx.check(ctx.lib.cc_residual(ctx.h, C.byref(dsys.struct), method, prec, C.byref(_amps(t1, t2)),
                                  C.byref(_amps(r1, r2)), C.byref(rn)))
    return r1, r2, rn.value


def energy(ctx, dsys, method, t1, t2):
    er, ei = C.c_double(), C.c_double()
    ctx.enter()
    ctx.check(ctx.lib.cc_energy(ctx.h, C.byref(dsys.struct), method, C.byref(_amps(t1, t2)),
                                C.byref(er), C.byref(ei)))
    return complex(er.value, ei.value) if dsys.is_complex else er.value


GUESSES = {"given": L.CC_GUESS_GIVEN, "mp2": L.CC_GUESS_MP2, "mlp": L.CC_GUESS_MLP}


def iterate(ctx, dsys, method, t1, t2, tol=1e-8, max_iter=100, level_shift=0.0, prec=F64,
            use_graph=True, refine_tol=0.0, diverge_window=0, hist_cap=None, dressed=False,
            autotune=False, correction=True, packed=False, check_every=1, guess="given", mlp=None):
    """Jacobi iteration (cc_iterate).  Reduced `prec` runs its contractions in
    that precision until the norm stagnates, then finishes with FP64 steps
    (with `correction`, in reference + reduced-precision-correction form for
    the contractions linear in the amplitudes).  `guess` selects the start:
    the amplitudes given, "mp2", or "mlp" (the network `mlp`, with the MP2
    amplitudes as fallback), formed inside the library and timed with it."""
    cap = hist_cap or max_iter
    hr = (C.c_double * cap)()
    he = (C.c_double * cap)()
    stats = mlp._st() if mlp is not None else None
    opts = L.CCIterOpts(tol, max_iter, prec, level_shift, refine_tol, 1 if use_graph else 0, check_every,
                        diverge_window, 1 if dressed else 0, 1 if autotune else 0, 1 if correction else 0,
                        1 if packed else 0, GUESSES[guess], mlp.prec if mlp is not None else F64,
                        _ptr(mlp.params) if mlp is not None else None,
                        C.cast(C.pointer(stats), C.c_void_p) if stats is not None else None)
    rep = L.CCIterReport(0, 0, 0.0, 0.0, 0.0, 0.0, 0.0, 0, 0, C.cast(hr, C.POINTER(C.c_double)),
                         C.cast(he, C.POINTER(C.c_double)), cap, 0, 0.0, 0.0, 0.0)
    ctx.enter()
    rc = ctx.lib.cc_iterate(ctx.h, C.byref(dsys.struct), method, C.byref(opts), C.byref(_amps(t1, t2)),
                            C.byref(rep))
    ctx.check(rc, ok=(L.CC_OK, L.CC_ENOTCONV, L.CC_EDIVERGED))
    n = min(rep.iters, cap)
    return {"status": rc, "iters": rep.iters, "converged": bool(rep.converged), "rnorm": rep.rnorm,
            "energy": complex(rep.e_re, rep.e_im) if dsys.is_complex else rep.e_re,
            "seconds": rep.seconds, "setup_seconds": rep.setup_seconds, "lowp_iters": rep.lowp_iters,
            "corr_iters": rep.corr_iters, "guess_used": {v: k for k, v in GUESSES.items()}[rep.guess_used],
            "guess_rnorm": {"mlp": rep.guess_rnorm_mlp, "mp2": rep.guess_rnorm_mp2},
            "guess_seconds": rep.guess_seconds,
            "hist_rnorm": list(hr[:n]), "hist_e": list(he[:n])}


def gemm(ctx, A, B, Cm, alpha=1.0, beta=0.0, a_kcontig=True, b_kcontig=True, prec=F64):
    """C = alpha * A' B'^T + beta * C with A' (M x K), B' (N x K).  A is stored
    [M][K] if a_kcontig else [K][M]; B is [N][K] if b_kcontig else [K][N]."""
    M, N = Cm.shape
    K = A.shape[1] if a_kcontig else A.shape[0]
    sam, sak = (K, 1) if a_kcontig else (1, M)
    sbn, sbk = (K, 1) if b_kcontig else (1, N)
    scalar = L.CC_C128 if Cm.dtype == torch.complex128 else L.CC_R64
    ctx.enter()
    ctx.check(ctx.lib.cc_gemm(ctx.h, prec, scalar, M, N, K, alpha, _ptr(A), sam, sak, _ptr(B), sbn, sbk,
                              beta, _ptr(Cm), N))


def gemm_noalloc(ctx, A, B, Cm, alpha=1.0, beta=0.0, a_kcontig=True, b_kcontig=True):
    """gemm() in FP64 through the entry point that allocates nothing (split-K
    partial sums in the library's static device buffer); enqueued only."""
    M, N = Cm.shape
    K = A.shape[1] if a_kcontig else A.shape[0]
    sam, sak = (K, 1) if a_kcontig else (1, M)
    sbn, sbk = (K, 1) if b_kcontig else (1, N)
    scalar = L.CC_C128 if Cm.dtype == torch.complex128 else L.CC_R64
    ctx.enter()
    ctx.check(ctx.lib.cc_gemm_noalloc(ctx.h, scalar, M, N, K, alpha, _ptr(A), sam, sak, _ptr(B), sbn, sbk,
                                      beta, _ptr(Cm), N))


def gemm_tile_count(ctx, prec=F64, cplx=False) -> int:
    """Number of GEMM tile configurations of a precision, or of the complex
    GEMM (for forced-tile sweeps through the CC_GEMM_TILE environment variable)."""
    return ctx.lib.cc_gemm_tile_count_c128() if cplx else ctx.lib.cc_gemm_tile_count(prec)


def permute(ctx, x, perm, out=None, alpha=1.0, beta=0.0):
    """out = alpha * x.permute(perm) + beta * out (dense result)."""
    shape = [x.shape[p] for p in perm]
    if out is None:
        out = torch.empty(shape, dtype=x.dtype, device=x.device)
    dims = (C.c_int64 * x.dim())(*x.shape)
    pr = (C.c_int32 * x.dim())(*perm)
    scalar = L.CC_C128 if x.dtype == torch.complex128 else L.CC_R64
    ctx.enter()
    ctx.check(ctx.lib.cc_permute(ctx.h, scalar, x.dim(), dims, pr, alpha, _ptr(x), beta, _ptr(out)))
    return out


class Batch:
    """Many independent systems iterated together (one grouped launch per
    step of the contraction list, the iteration replayed as one graph)."""

    def __init__(self, ctx: Context, dsystems, method: int = CCSD, prec: int = F64, amps=None):
        self.ctx, self.dsystems, self.method, self.n = ctx, list(dsystems), method, len(dsystems)
        self.amps = amps if amps is not None else [zeros_amps(d, method) for d in self.dsystems]
        arr_s = (L.CCSystemStruct * self.n)(*[d.struct for d in self.dsystems])
        arr_a = (L.CCAmps * self.n)(*[_amps(t1, t2) for t1, t2 in self.amps])
        self._keep = (arr_s, arr_a)
        self.h = C.c_void_p()
        ctx.enter()
        ctx.check(ctx.lib.cc_batch_create(ctx.h, self.n, arr_s, method, prec, arr_a, C.byref(self.h)))

    def step(self, shift: float = 0.0, dressed: bool = False):
        self.ctx.enter()
        self.ctx.check(self.ctx.lib.cc_batch_step(self.h, shift, 1 if dressed else 0))

    def scalars(self):
        rn, er, ei = (C.c_double * self.n)(), (C.c_double * self.n)(), (C.c_double * self.n)()
        self.ctx.check(self.ctx.lib.cc_batch_scalars(self.h, rn, er, ei))
        return list(rn), list(er), list(ei)

    def autotune(self, reps: int = 2):
        self.ctx.enter()
        self.ctx.check(self.ctx.lib.cc_batch_autotune(self.h, reps))

    def iterate(self, tol=1e-8, max_iter=200, level_shift=0.0, dressed=False, prec=F64, use_graph=True):
        opts = L.CCIterOpts(tol, max_iter, prec, level_shift, 0.0, 1 if use_graph else 0, 1, 0,
                            1 if dressed else 0, 0, 0, 0)
        reps = (L.CCIterReport * self.n)()
        nconv = C.c_int32()
        self.ctx.enter()
        rc = self.ctx.lib.cc_batch_iterate(self.h, C.byref(opts), reps, C.byref(nconv))
        self.ctx.check(rc, ok=(L.CC_OK, L.CC_ENOTCONV, L.CC_EDIVERGED))
        return {"status": rc, "n_converged": nconv.value,
                "systems": [{"iters": r.iters, "converged": bool(r.converged), "rnorm": r.rnorm,
                             "energy": r.e_re, "seconds": r.seconds} for r in reps]}

    def profile(self, enable: bool = True):
        self.ctx.check(self.ctx.lib.cc_batch_profile(self.h, 1 if enable else 0))

    def profile_table(self):
        rows = []
        for line in self.ctx.lib.cc_batch_profile_table(self.h).decode().splitlines():
            if line.startswith("#") or not line.strip():
                continue
            i, kind, tag, calls, tot, avg, fl = line.split()
            rows.append((int(i), kind, tag, int(calls), float(tot), float(avg), float(fl)))
        return rows

    def flops(self) -> float:
        return self.ctx.lib.cc_batch_flops(self.h)

    def close(self):
        if self.h:
            self.ctx.lib.cc_batch_destroy(self.h)
            self.h = C.c_void_p()

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


class MLP:
    """Amplitude-guess network (parameters on the device, FP64 storage)."""

    def __init__(self, ctx: Context, params: torch.Tensor, stats: dict, prec: int = F32):
        self.ctx, self.params, self.stats, self.prec = ctx, params.contiguous(), dict(stats), prec
        n = ctx.lib.cc_mlp_num_params()
        assert self.params.numel() == n and self.params.dtype == torch.float64
        self.m = torch.zeros_like(self.params)
        self.v = torch.zeros_like(self.params)
        self.t = C.c_int64(0)

    @staticmethod
    def init_params(seed: int = 0, device="cuda") -> torch.Tensor:
        """He-normal weights, zero biases (seeded; drawn on the host)."""
        rng = np.random.default_rng(seed)
        h = 128
        parts = [rng.normal(size=(h, 3)) * np.sqrt(2 / 3), np.zeros(h), rng.normal(size=(h, h)) * np.sqrt(2 / h),
                 np.zeros(h), rng.normal(size=(1, h)) * np.sqrt(2 / h), np.zeros(1)]
        return torch.from_numpy(np.concatenate([p.ravel() for p in parts])).to(device)

    def _st(self):
        return L.CCMlpStats(*[self.stats[k] for k in ("sx", "mD", "sD", "me", "se", "st")])

    @staticmethod
    def raw_features(ctx: Context, dsys: DeviceSystem) -> torch.Tensor:
        n = ctx.lib.cc_mlp_num_samples(dsys.o, dsys.v)
        z = torch.empty((n, 3), dtype=torch.float64, device=dsys.t["oovv"].device)
        ctx.enter()
        ctx.check(ctx.lib.cc_mlp_features(ctx.h, C.byref(dsys.struct), None, _ptr(z)))
        return z

    @staticmethod
    def targets(ctx: Context, o: int, v: int, t2: torch.Tensor, scale: float = 1.0) -> torch.Tensor:
        n = ctx.lib.cc_mlp_num_samples(o, v)
        y = torch.empty(n, dtype=torch.float64, device=t2.device)
        ctx.enter()
        ctx.check(ctx.lib.cc_mlp_targets(ctx.h, o, v, _ptr(t2), scale, _ptr(y)))
        return y

    @staticmethod
    def fit_stats(ctx: Context, raw: torch.Tensor, y: torch.Tensor) -> dict:
        out = (C.c_double * 7)()
        ctx.enter()
        ctx.check(ctx.lib.cc_mlp_moments(ctx.h, _ptr(raw), _ptr(y), raw.shape[0], out))
        sx2, sD, sD2, se, se2, sy2, n = list(out)
        mD, me = sD / n, se / n
        return {"sx": (sx2 / n) ** 0.5, "mD": mD, "sD": max(sD2 / n - mD * mD, 1e-300) ** 0.5, "me": me,
                "se": max(se2 / n - me * me, 1e-300) ** 0.5, "st": (sy2 / n) ** 0.5}

    def standardise(self, raw: torch.Tensor, y: Optional[torch.Tensor] = None):
        z = torch.empty_like(raw)
        ys = torch.empty_like(y) if y is not None else None
        st = self._st()
        self.ctx.enter()
        self.ctx.check(self.ctx.lib.cc_mlp_standardise(self.ctx.h, _ptr(raw), _ptr(y), raw.shape[0], C.byref(st),
                                                       _ptr(z), _ptr(ys)))
        return z, ys

    def forward(self, z: torch.Tensor) -> torch.Tensor:
        f = torch.empty(z.shape[0], dtype=torch.float64, device=z.device)
        self.ctx.enter()
        self.ctx.check(self.ctx.lib.cc_mlp_forward(self.ctx.h, self.prec, _ptr(self.params), _ptr(z), z.shape[0],
                                                   _ptr(f)))
        return f

    def loss_grad(self, z: torch.Tensor, y: torch.Tensor):
        g = torch.empty_like(self.params)
        loss = C.c_double()
        self.ctx.enter()
        self.ctx.check(self.ctx.lib.cc_mlp_loss_grad(self.ctx.h, self.prec, _ptr(self.params), _ptr(z), _ptr(y),
                                                     z.shape[0], C.byref(loss), _ptr(g)))
        return loss.value, g

    def train(self, z: torch.Tensor, y: torch.Tensor, epochs: int = 1, batch: int = 65536, lr: float = 1e-3,
              order: Optional[torch.Tensor] = None):
        """Adam over the rows of z, y in the order given (all rows when None;
        else the rows `order` lists, which may be a subset)."""
        n = z.shape[0] if order is None else order.shape[0]
        if order is not None:
            assert order.dtype == torch.int64 and order.is_contiguous() and n <= z.shape[0]
        hist = (C.c_double * epochs)()
        self.ctx.enter()
        self.ctx.check(self.ctx.lib.cc_mlp_train(self.ctx.h, self.prec, _ptr(self.params), _ptr(self.m),
                                                 _ptr(self.v), _ptr(z), _ptr(y), n, _ptr(order), batch,
                                                 epochs, lr, C.byref(self.t), hist, epochs))
        return list(hist)

    def guess(self, dsys: DeviceSystem, t1, t2):
        st = self._st()
        self.ctx.enter()
        self.ctx.check(self.ctx.lib.cc_guess_mlp(self.ctx.h, C.byref(dsys.struct), self.prec, _ptr(self.params),
                                                 C.byref(st), C.byref(_amps(t1, t2))))

    def save(self, path, with_state: bool = False):
        """Parameters and standardisation; with_state also Adam's moments and
        step count (to continue training on more data)."""
        extra = {}
        if with_state:
            extra = dict(adam_m=self.m.cpu().numpy(), adam_v=self.v.cpu().numpy(), adam_t=np.array([self.t.value]))
        np.savez(path, params=self.params.cpu().numpy(),
                 stats=np.array([self.stats[k] for k in ("sx", "mD", "sD", "me", "se", "st")]), **extra)

    @classmethod
    def load(cls, ctx: Context, path, prec: int = F32, device="cuda"):
        d = np.load(path, allow_pickle=False)
        keys = ("sx", "mD", "sD", "me", "se", "st")
        net = cls(ctx, torch.from_numpy(d["params"]).to(device), dict(zip(keys, d["stats"].tolist())), prec)
        if "adam_m" in d:
            net.m = torch.from_numpy(d["adam_m"]).to(device)
            net.v = torch.from_numpy(d["adam_v"]).to(device)
            net.t = C.c_int64(int(d["adam_t"][0]))
        return net
