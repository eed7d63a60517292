"""Kernel-level parity on the GPU: the MFMA GEMM against numpy.matmul in
FP64 and the LDS-tiled permutation against numpy transposes (exact)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def ctx():
    from paper_2409_06759_amd import engine as E
    c = E.Context(0)
    yield c
    c.close()


SHAPES = [(1, 1, 1), (16, 16, 16), (17, 33, 65), (64, 576, 576), (100, 129, 37), (257, 300, 49),
          (1024, 160, 96)]


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("akc", [True, False])
@pytest.mark.parametrize("bkc", [True, False])
def test_gemm_f64_matches_numpy(ctx, shape, akc, bkc):
    from paper_2409_06759_amd import engine as E
    M, N, K = shape
    print(f"gemm M={M} N={N} K={K} akc={akc} bkc={bkc}", flush=True)
    rng = np.random.default_rng(M * 7 + N * 3 + K)
    A = rng.normal(size=(M, K))
    B = rng.normal(size=(N, K))
    C0 = rng.normal(size=(M, N))
    alpha, beta = 0.5, -1.25
    ref = alpha * (A @ B.T) + beta * C0
    Ad = torch.from_numpy(A if akc else np.ascontiguousarray(A.T)).cuda()
    Bd = torch.from_numpy(B if bkc else np.ascontiguousarray(B.T)).cuda()
    Cd = torch.from_numpy(C0).cuda()
    E.gemm(ctx, Ad, Bd, Cd, alpha, beta, a_kcontig=akc, b_kcontig=bkc)
    got = Cd.cpu().numpy()
    bound = 2 * K * np.finfo(np.float64).eps * (abs(alpha) * (np.abs(A) @ np.abs(B).T) + abs(beta) * np.abs(C0))
    assert np.all(np.abs(got - ref) <= bound + 1e-300), np.abs(got - ref).max()


def test_gemm_beta_zero_ignores_nan(ctx):
    from paper_2409_06759_amd import engine as E
    A = torch.ones((33, 20), dtype=torch.float64, device="cuda")
    B = torch.ones((45, 20), dtype=torch.float64, device="cuda")
    Cd = torch.full((33, 45), float("nan"), dtype=torch.float64, device="cuda")
    E.gemm(ctx, A, B, Cd, 1.0, 0.0)
    assert torch.all(Cd == 20.0)


@pytest.mark.parametrize("dims,perm", [((5, 7), (1, 0)), ((3, 40, 33, 5), (0, 2, 1, 3)),
                                       ((6, 6, 35, 35), (2, 0, 3, 1)), ((4, 5, 6, 7), (3, 2, 1, 0)),
                                       ((3, 4, 5, 6, 7), (4, 0, 3, 1, 2)),
                                       ((2, 3, 4, 5, 6, 7), (5, 4, 3, 2, 1, 0)),
                                       # short fast dims (4..256-long tiles): output, input, both
                                       ((4, 4, 20, 20), (0, 2, 3, 1)), ((7, 23, 23, 7), (0, 3, 1, 2)),
                                       ((5, 300, 2, 3), (3, 1, 0, 2)), ((3, 5, 1, 6), (3, 2, 0, 1))])
def test_permute_exact(ctx, dims, perm):
    from paper_2409_06759_amd import engine as E
    rng = np.random.default_rng(len(dims))
    x = rng.normal(size=dims)
    got = E.permute(ctx, torch.from_numpy(x).cuda(), perm).cpu().numpy()
    assert np.array_equal(got, np.ascontiguousarray(x.transpose(perm)))


def test_permute_accumulate(ctx):
    from paper_2409_06759_amd import engine as E
    rng = np.random.default_rng(5)
    x = rng.normal(size=(9, 37, 8, 41))
    y = rng.normal(size=(9, 8, 41, 37))
    out = torch.from_numpy(y).cuda()
    E.permute(ctx, torch.from_numpy(x).cuda(), (0, 2, 3, 1), out=out, alpha=2.0, beta=-1.0)
    ref = 2.0 * x.transpose(0, 2, 3, 1) - y
    assert np.abs(out.cpu().numpy() - ref).max() < 1e-14


@pytest.mark.parametrize("prec", ["f32", "bf16x3"])
@pytest.mark.parametrize("shape", [(16, 16, 16), (17, 33, 65), (64, 576, 576), (100, 129, 37), (257, 300, 49)])
@pytest.mark.parametrize("akc,bkc", [(True, True), (False, False), (True, False)])
def test_gemm_lowp_error_bound(ctx, prec, shape, akc, bkc):
    """Reduced precision: |C - C_ref| <= 2 eps_eff (|alpha| |A||B|^T) + FP64 rounding of beta C.
    eps_eff = (K + 2) 2^-24 (FP32 inputs, FP32 accumulation) plus 3 * 2^-17 for
    the split-bf16 product (hi*hi + hi*lo + lo*hi; lo*lo and the second split's
    remainder dropped)."""
    from paper_2409_06759_amd import engine as E
    M, N, K = shape
    print(f"gemm {prec} M={M} N={N} K={K} akc={akc} bkc={bkc}", flush=True)
    rng = np.random.default_rng(M + 3 * N + 7 * K)
    A = rng.normal(size=(M, K))
    B = rng.normal(size=(N, K))
    C0 = rng.normal(size=(M, N))
    alpha, beta = 0.5, -1.25
    ref = alpha * (A @ B.T) + beta * C0
    Ad = torch.from_numpy(A if akc else np.ascontiguousarray(A.T)).cuda()
    Bd = torch.from_numpy(B if bkc else np.ascontiguousarray(B.T)).cuda()
    Cd = torch.from_numpy(C0).cuda()
    E.gemm(ctx, Ad, Bd, Cd, alpha, beta, a_kcontig=akc, b_kcontig=bkc, prec=E.PRECS[prec])
    eps = (K + 2) * 2.0 ** -24 + (3 * 2.0 ** -17 if prec == "bf16x3" else 0.0)
    bound = 2 * eps * abs(alpha) * (np.abs(A) @ np.abs(B).T) + 4 * np.finfo(float).eps * np.abs(beta * C0)
    err = np.abs(Cd.cpu().numpy() - ref)
    assert np.all(err <= bound), (err / bound).max()


@pytest.mark.parametrize("prec", ["f32", "bf16x3"])
@pytest.mark.parametrize("shape", [(17, 33, 65), (100, 129, 37), (257, 300, 100), (64, 576, 576)])
@pytest.mark.parametrize("akc,bkc", [(True, True), (False, False), (True, False), (False, True)])
def test_gemm_lowp_converted_operands_match_inline(ctx, monkeypatch, prec, shape, akc, bkc):
    """Operands converted once into 4-byte copies and read with vector loads
    give bit-identical results to rounding/splitting FP64 operands while
    staging (same LDS contents, same accumulation order).  Odd leading
    dimensions take the scalar-load fallback."""
    from paper_2409_06759_amd import engine as E
    M, N, K = shape
    print(f"gemm staging {prec} M={M} N={N} K={K} akc={akc} bkc={bkc}", flush=True)
    rng = np.random.default_rng(M + N + K)
    A = rng.normal(size=(M, K))
    B = rng.normal(size=(N, K))
    C0 = rng.normal(size=(M, N))
    Ad = torch.from_numpy(A if akc else np.ascontiguousarray(A.T)).cuda()
    Bd = torch.from_numpy(B if bkc else np.ascontiguousarray(B.T)).cuda()
    out = []
    for lpin in ("1", "0"):
        monkeypatch.setenv("CC_GEMM_LPIN", lpin)
        Cd = torch.from_numpy(C0).cuda()
        E.gemm(ctx, Ad, Bd, Cd, 0.5, -1.25, a_kcontig=akc, b_kcontig=bkc, prec=E.PRECS[prec])
        out.append(Cd.cpu().numpy())
    assert np.array_equal(out[0], out[1])



@pytest.mark.parametrize("shape", [(1, 1, 1), (17, 33, 65), (64, 100, 300), (130, 70, 33)])
@pytest.mark.parametrize("akc,bkc", [(True, True), (False, False), (False, True)])
def test_gemm_c128_matches_numpy(ctx, shape, akc, bkc):
    from paper_2409_06759_amd import engine as E
    M, N, K = shape
    rng = np.random.default_rng(M * 5 + N + K)
    A = rng.normal(size=(M, K)) + 1j * rng.normal(size=(M, K))
    B = rng.normal(size=(N, K)) + 1j * rng.normal(size=(N, K))
    C0 = rng.normal(size=(M, N)) + 1j * rng.normal(size=(M, N))
    alpha, beta = 0.5, -1.25
    ref = alpha * (A @ B.T) + beta * C0
    Ad = torch.from_numpy(A if akc else np.ascontiguousarray(A.T)).cuda()
    Bd = torch.from_numpy(B if bkc else np.ascontiguousarray(B.T)).cuda()
    Cd = torch.from_numpy(C0).cuda()
    E.gemm(ctx, Ad, Bd, Cd, alpha, beta, a_kcontig=akc, b_kcontig=bkc)
    bound = 4 * (K + 2) * np.finfo(float).eps * (abs(alpha) * (np.abs(A) @ np.abs(B).T) + abs(beta) * np.abs(C0))
    assert np.all(np.abs(Cd.cpu().numpy() - ref) <= bound)


@pytest.mark.parametrize("prec", ["f32", "bf16x3"])
@pytest.mark.parametrize("shape", [(1, 1, 1), (17, 33, 65), (64, 100, 300), (130, 70, 33), (70, 200, 512)])
@pytest.mark.parametrize("akc,bkc", [(True, True), (False, False), (False, True)])
def test_gemm_c128_lowp_error_bound(ctx, prec, shape, akc, bkc):
    """Complex reduced precision as the real GEMM of M x 2N x 2K on realified
    operands: the real and imaginary parts each carry the real bound with
    K' = 2K terms of |Re a| + |Im a| times |Re b| + |Im b| per k."""
    from paper_2409_06759_amd import engine as E
    M, N, K = shape
    print(f"gemm c128 {prec} M={M} N={N} K={K} akc={akc} bkc={bkc}", flush=True)
    rng = np.random.default_rng(M * 3 + N + 11 * K)
    A = rng.normal(size=(M, K)) + 1j * rng.normal(size=(M, K))
    B = rng.normal(size=(N, K)) + 1j * rng.normal(size=(N, K))
    C0 = rng.normal(size=(M, N)) + 1j * rng.normal(size=(M, N))
    alpha, beta = 0.5, -1.25
    ref = alpha * (A @ B.T) + beta * C0
    Ad = torch.from_numpy(A if akc else np.ascontiguousarray(A.T)).cuda()
    Bd = torch.from_numpy(B if bkc else np.ascontiguousarray(B.T)).cuda()
    Cd = torch.from_numpy(C0).cuda()
    E.gemm(ctx, Ad, Bd, Cd, alpha, beta, a_kcontig=akc, b_kcontig=bkc, prec=E.PRECS[prec])
    got = Cd.cpu().numpy()
    eps = (2 * K + 2) * 2.0 ** -24 + (3 * 2.0 ** -17 if prec == "bf16x3" else 0.0)
    mag = (np.abs(A.real) + np.abs(A.imag)) @ (np.abs(B.real) + np.abs(B.imag)).T
    bound = 2 * eps * abs(alpha) * mag + 4 * np.finfo(float).eps * np.abs(beta * C0)
    for part in (np.real, np.imag):
        err = np.abs(part(got) - part(ref))
        assert np.all(err <= bound), (err / bound).max()


@pytest.mark.parametrize("prec,cplx", [("f64", False), ("f32", False), ("bf16x3", False), ("f64", True),
                                       ("f32", True)])
def test_gemm_with_empty_contraction_scales_c(ctx, prec, cplx):
    """K = 0: C = beta C (no products)."""
    from paper_2409_06759_amd import engine as E
    dt = torch.complex128 if cplx else torch.float64
    C0 = torch.randn(37, 53, dtype=dt)
    Cd = C0.cuda()
    A = torch.zeros((37, 0), dtype=dt, device="cuda")
    B = torch.zeros((53, 0), dtype=dt, device="cuda")
    E.gemm(ctx, A, B, Cd, 0.5, -1.5, prec=E.PRECS[prec])
    assert torch.equal(Cd.cpu(), -1.5 * C0)


# Forced tile configurations whose launches end in an almost empty round of
# workgroups: 544 tiles = 2 x 256 + 32 (one workgroup per CU) or 512 + 32 (two).
TAIL_CASES = [
    ("f64", 4, 1024, 136 * 128, 2048, True, True, 1),     # 256x128 tiles, column panels cut
    ("f64", 4, 1024, 136 * 128, 2048, False, False, 1),
    ("f64", 4, 136 * 256, 512, 2048, True, True, 2),      # row panels cut
    ("bf16x3", 7, 1024, 136 * 128, 2048, True, True, 1),  # 256x128x32
    ("f32", 7, 1024, 68 * 128, 2048, True, True, 1),      # 128x128x32
]


@pytest.mark.parametrize("prec,tile,M,N,K,akc,bkc,axis", TAIL_CASES)
def test_gemm_tail_cut(ctx, monkeypatch, prec, tile, M, N, K, akc, bkc, axis):
    """A GEMM whose last round of workgroups would be nearly empty runs as whole
    rounds plus a K-split tail: the result meets the same error bound as one
    launch, the main panels are bitwise those of one launch, and exactly a
    trailing block of whole panels differs (summed over K in another order)."""
    from paper_2409_06759_amd import engine as E
    print(f"tail cut {prec} tile {tile} M={M} N={N} K={K} akc={akc} bkc={bkc}", flush=True)
    rng = np.random.default_rng(M + 3 * N + K)
    A = rng.normal(size=(M, K))
    B = rng.normal(size=(N, K))
    C0 = rng.normal(size=(M, N))
    alpha, beta = 0.75, -0.5
    Ad = torch.from_numpy(A if akc else np.ascontiguousarray(A.T)).cuda()
    Bd = torch.from_numpy(B if bkc else np.ascontiguousarray(B.T)).cuda()
    monkeypatch.setenv("CC_GEMM_TILE", str(tile))
    out = {}
    for cut in ("0", "1"):
        monkeypatch.setenv("CC_GEMM_TAIL", cut)
        Cd = torch.from_numpy(C0).cuda()
        E.gemm(ctx, Ad, Bd, Cd, alpha, beta, a_kcontig=akc, b_kcontig=bkc, prec=E.PRECS[prec])
        out[cut] = Cd.cpu().numpy()
    ref = alpha * (A @ B.T) + beta * C0
    u = 2.0 ** -53 if prec == "f64" else 2.0 ** -24
    eps = (K + 16) * u + (3 * 2.0 ** -17 if prec == "bf16x3" else 0.0)
    bound = 2 * eps * abs(alpha) * (np.abs(A) @ np.abs(B).T) + 4 * np.finfo(float).eps * np.abs(beta * C0)
    for cut in ("0", "1"):
        err = np.abs(out[cut] - ref)
        assert np.all(err <= bound), (cut, (err / bound).max())
    diff = out["0"] != out["1"]
    lines = np.nonzero(diff.any(axis=0 if axis == 1 else 1))[0]
    assert lines.size > 0, "no tail cut happened"
    first = int(lines[0])
    panel = 128 if axis == 1 else 256
    extent = N if axis == 1 else M
    print(f"tail from {first} of {extent}", flush=True)
    assert first % panel == 0 and first >= extent // 2
    assert np.array_equal(lines, np.arange(first, extent))
    main = out["0"][:, :first] if axis == 1 else out["0"][:first]
    main1 = out["1"][:, :first] if axis == 1 else out["1"][:first]
    assert np.array_equal(main, main1)


# (precision, one-chunk-prefetch configuration, two-chunk configuration of the same tile)
PF_PAIRS = [("f32", 7, 8), ("bf16x3", 6, 8)]


@pytest.mark.parametrize("prec,t1,t2", PF_PAIRS)
@pytest.mark.parametrize("K", [5, 32, 64, 133, 160, 1000])
@pytest.mark.parametrize("akc,bkc", [(True, True), (False, False), (True, False), (False, True)])
def test_gemm_lowp_two_chunk_prefetch_is_bitwise_one_chunk(ctx, monkeypatch, prec, t1, t2, K, akc, bkc):
    """Keeping two K chunks in flight changes when operands arrive, not what
    is multiplied or in which order: results are bit-identical for one, two,
    odd and even chunk counts and every operand layout."""
    from paper_2409_06759_amd import engine as E
    M, N = 300, 270
    print(f"prefetch {prec} tiles {t1}/{t2} K={K} akc={akc} bkc={bkc}", flush=True)
    rng = np.random.default_rng(K + 17)
    A = rng.normal(size=(M, K))
    B = rng.normal(size=(N, K))
    C0 = rng.normal(size=(M, N))
    Ad = torch.from_numpy(A if akc else np.ascontiguousarray(A.T)).cuda()
    Bd = torch.from_numpy(B if bkc else np.ascontiguousarray(B.T)).cuda()
    out = []
    for t in (t1, t2):
        monkeypatch.setenv("CC_GEMM_TILE", str(t))
        Cd = torch.from_numpy(C0).cuda()
        E.gemm(ctx, Ad, Bd, Cd, 0.5, -1.25, a_kcontig=akc, b_kcontig=bkc, prec=E.PRECS[prec])
        out.append(Cd.cpu().numpy())
    assert np.array_equal(out[0], out[1])
    ref = 0.5 * (A @ B.T) - 1.25 * C0
    tol = 1e-4 if prec == "f32" else 1e-3
    assert np.abs(out[1] - ref).max() <= tol * max(1.0, np.sqrt(K))


@pytest.mark.parametrize("M,N,K", [
    (256, 128, 32), (512, 256, 96), (300, 270, 160), (496, 1000, 96), (37, 300, 64), (1, 17, 32),
    (1024, 136 * 128, 2048)])  # cut: whole rounds + a K-split tail
@pytest.mark.parametrize("tile", [9, 10, 11])
def test_gemm_bf16x3_blocked_copies_are_bitwise_row_major(ctx, monkeypatch, tile, M, N, K):
    """Split-bf16 operand copies in 16-row x 32-k blocks (rows padded to a
    multiple of 16) put the same values in the same LDS slots as the
    row-major copies: every LDS-direct configuration gives bit-identical
    results with either, on ragged M and N, padded rows and the K-split tail."""
    from paper_2409_06759_amd import engine as E
    print(f"blocked tile {tile} M={M} N={N} K={K}", flush=True)
    rng = np.random.default_rng(M + 7 * N + K)
    A = rng.normal(size=(M, K))
    B = rng.normal(size=(N, K))
    C0 = rng.normal(size=(M, N))
    Ad, Bd = torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda()
    monkeypatch.setenv("CC_GEMM_TILE", str(tile))
    out = []
    for blocked in ("0", "1"):
        monkeypatch.setenv("CC_GEMM_BLOCKED", blocked)
        Cd = torch.from_numpy(C0).cuda()
        E.gemm(ctx, Ad, Bd, Cd, 0.5, -1.25, prec=E.PRECS["bf16x3"])
        out.append(Cd.cpu().numpy())
    assert np.array_equal(out[0], out[1])
    ref = 0.5 * (A @ B.T) - 1.25 * C0
    assert np.abs(out[1] - ref).max() <= 1e-3 * max(1.0, np.sqrt(K))


@pytest.mark.parametrize("M,N,K,akc,bkc", [
    (256, 128, 32, True, True), (256, 128, 64, True, True), (512, 256, 96, True, True),
    (256, 384, 160, True, True), (768, 256, 1024, True, True),
    (1024, 136 * 128, 2048, True, True),   # cut: whole rounds + a K-split tail, both on this kernel
    (300, 270, 160, True, True), (496, 1000, 96, True, True),   # ragged M and N: rows clamped
    (300, 270, 133, True, True), (256, 128, 64, False, True)])  # shapes it hands to the staged kernel
@pytest.mark.parametrize("prec,staged,direct", [("bf16x3", 7, 9), ("bf16x3", 7, 10), ("bf16x3", 7, 11),
                                                ("f32", 9, 10)])
def test_gemm_lowp_lds_direct_is_bitwise_staged(ctx, monkeypatch, prec, staged, direct, M, N, K, akc, bkc):
    """The reduced-precision configurations with LDS-direct loads (256x128,
    and split bf16 at 256x256) multiply the same fragments in the same order
    as the register-staged 256x128 kernel: bit-identical results (and they
    fall back to that kernel on shapes they do not take).  The 256x256 tile
    cuts its last round differently (another K-split tail), so it is compared
    without the cut."""
    from paper_2409_06759_amd import engine as E
    print(f"lds-direct {prec} {direct} M={M} N={N} K={K} akc={akc} bkc={bkc}", flush=True)
    if direct == 11:
        monkeypatch.setenv("CC_GEMM_TAIL", "0")
    rng = np.random.default_rng(M + N + K)
    A = rng.normal(size=(M, K))
    B = rng.normal(size=(N, K))
    C0 = rng.normal(size=(M, N))
    Ad = torch.from_numpy(A if akc else np.ascontiguousarray(A.T)).cuda()
    Bd = torch.from_numpy(B if bkc else np.ascontiguousarray(B.T)).cuda()
    out = []
    for t in (staged, direct):
        monkeypatch.setenv("CC_GEMM_TILE", str(t))
        Cd = torch.from_numpy(C0).cuda()
        E.gemm(ctx, Ad, Bd, Cd, 0.5, -1.25, a_kcontig=akc, b_kcontig=bkc, prec=E.PRECS[prec])
        out.append(Cd.cpu().numpy())
    assert np.array_equal(out[0], out[1])
    ref = 0.5 * (A @ B.T) - 1.25 * C0
    assert np.abs(out[1] - ref).max() <= 1e-3 * max(1.0, np.sqrt(K))


@pytest.mark.parametrize("M,N,K,akc,bkc", [
    (256, 128, 16, True, True), (256, 128, 32, True, True), (512, 256, 48, True, True),
    (256, 384, 80, True, True), (768, 256, 1024, True, True),
    (1024, 136 * 128, 2048, True, True),   # cut: whole rounds + a K-split tail, both on this kernel
    (300, 270, 160, True, True), (496, 1000, 96, True, True),   # ragged M and N: rows clamped
    (300, 270, 133, True, True), (256, 128, 64, True, False)])  # shapes it hands to the staged kernel
def test_gemm_f64_lds_direct_is_bitwise_staged(ctx, monkeypatch, M, N, K, akc, bkc):
    """The 256x128x16 FP64 configuration with LDS-direct loads feeds every
    MFMA the operands of the register-staged kernel of that tile in the same
    order: bit-identical results; shapes it does not take fall back."""
    from paper_2409_06759_amd import engine as E
    staged, direct = 4, 16
    print(f"f64 lds-direct M={M} N={N} K={K} akc={akc} bkc={bkc}", flush=True)
    rng = np.random.default_rng(M + 2 * N + K)
    A = rng.normal(size=(M, K))
    B = rng.normal(size=(N, K))
    C0 = rng.normal(size=(M, N))
    Ad = torch.from_numpy(A if akc else np.ascontiguousarray(A.T)).cuda()
    Bd = torch.from_numpy(B if bkc else np.ascontiguousarray(B.T)).cuda()
    out = []
    for t in (staged, direct):
        monkeypatch.setenv("CC_GEMM_TILE", str(t))
        Cd = torch.from_numpy(C0).cuda()
        E.gemm(ctx, Ad, Bd, Cd, 0.5, -1.25, a_kcontig=akc, b_kcontig=bkc)
        out.append(Cd.cpu().numpy())
    assert np.array_equal(out[0], out[1])
    ref = 0.5 * (A @ B.T) - 1.25 * C0
    bound = (K + 16) * 2.0 ** -52 * 0.5 * (np.abs(A) @ np.abs(B).T) + 4 * np.finfo(float).eps * np.abs(1.25 * C0)
    assert np.all(np.abs(out[1] - ref) <= bound)


@pytest.mark.parametrize("M,N,K,akc,bkc", [
    (64, 128, 16, True, True), (128, 256, 48, True, True), (100, 70, 48, True, True),   # ragged M and N
    (130, 260, 160, True, True), (64, 128, 16, False, True), (64, 128, 24, True, True)])  # fallbacks
def test_gemm_c128_lds_direct_is_bitwise_staged(ctx, monkeypatch, M, N, K, akc, bkc):
    """The complex 64x128x16 configuration with LDS-direct loads feeds every
    MFMA the staged kernel's operands in the same order: bit-identical
    complex results, also with rows past M or N clamped, and fallbacks for
    layouts and K it does not take."""
    from paper_2409_06759_amd import engine as E
    staged, direct = 3, 4
    print(f"c128 lds-direct M={M} N={N} K={K} akc={akc} bkc={bkc}", flush=True)
    rng = np.random.default_rng(M + 5 * N + K)
    A = rng.normal(size=(M, K)) + 1j * rng.normal(size=(M, K))
    B = rng.normal(size=(N, K)) + 1j * rng.normal(size=(N, K))
    C0 = rng.normal(size=(M, N)) + 1j * rng.normal(size=(M, N))
    Ad = torch.from_numpy(A if akc else np.ascontiguousarray(A.T)).cuda()
    Bd = torch.from_numpy(B if bkc else np.ascontiguousarray(B.T)).cuda()
    out = []
    for t in (staged, direct):
        monkeypatch.setenv("CC_GEMM_TILE", str(t))
        Cd = torch.from_numpy(C0).cuda()
        E.gemm(ctx, Ad, Bd, Cd, 0.5, -1.25, a_kcontig=akc, b_kcontig=bkc)
        out.append(Cd.cpu().numpy())
    assert np.array_equal(out[0], out[1])
    ref = 0.5 * (A @ B.T) - 1.25 * C0
    assert np.abs(out[1] - ref).max() <= 1e-12 * max(1.0, K)


# Every tile configuration, forced through CC_GEMM_TILE, on a ragged shape
# (staged loads, partial tiles on every side) and on one whose K and row
# strides admit the LDS-direct and vector-load paths.
EVERY_TILE_SHAPES = [(100, 129, 37), (257, 300, 64)]


@pytest.mark.parametrize("prec", ["f64", "f32", "bf16x3", "c128"])
def test_gemm_every_tile_meets_bound(ctx, monkeypatch, prec):
    from paper_2409_06759_amd import engine as E
    cplx = prec == "c128"
    p = E.PRECS["f64" if cplx else prec]
    ntiles = E.gemm_tile_count(ctx, p, cplx=cplx)
    assert ntiles > 0
    u = {"f64": 2.0 ** -53, "c128": 2.0 ** -53, "f32": 2.0 ** -24, "bf16x3": 2.0 ** -24}[prec]
    for M, N, K in EVERY_TILE_SHAPES:
        rng = np.random.default_rng(M + N + K)
        A = rng.normal(size=(M, K))
        B = rng.normal(size=(N, K))
        C0 = rng.normal(size=(M, N))
        if cplx:
            A = A + 1j * rng.normal(size=(M, K))
            B = B + 1j * rng.normal(size=(N, K))
            C0 = C0 + 1j * rng.normal(size=(M, N))
        alpha, beta = 0.5, -1.25
        ref = alpha * (A @ B.T) + beta * C0
        eps = (4 if cplx else 2) * (K + 2) * u + (3 * 2.0 ** -17 if prec == "bf16x3" else 0.0)
        bound = eps * abs(alpha) * (np.abs(A) @ np.abs(B).T) + 4 * (K + 2) * np.finfo(float).eps * np.abs(beta * C0)
        for akc in (True, False):
            for bkc in (True, False):
                Ad = torch.from_numpy(A if akc else np.ascontiguousarray(A.T)).cuda()
                Bd = torch.from_numpy(B if bkc else np.ascontiguousarray(B.T)).cuda()
                for t in range(ntiles):
                    print(f"every tile {prec} tile {t} M={M} N={N} K={K} akc={akc} bkc={bkc}", flush=True)
                    monkeypatch.setenv("CC_GEMM_TILE", str(t))
                    Cd = torch.from_numpy(C0).cuda()
                    E.gemm(ctx, Ad, Bd, Cd, alpha, beta, a_kcontig=akc, b_kcontig=bkc, prec=p)
                    err = np.abs(Cd.cpu().numpy() - ref)
                    assert np.all(err <= bound), (t, akc, bkc, (err / bound).max())


def test_permute_pairs_accumulate(ctx):
    """Shared even unit-stride dimension (16-byte pair path) with alpha/beta
    accumulation; exact against numpy (alpha, beta powers of two)."""
    from paper_2409_06759_amd import engine as E
    rng = np.random.default_rng(11)
    x = rng.normal(size=(6, 10, 4, 8))
    y = rng.normal(size=(10, 6, 4, 8))
    yd = torch.from_numpy(y).cuda()
    E.permute(ctx, torch.from_numpy(x).cuda(), (1, 0, 2, 3), out=yd, alpha=0.5, beta=-2.0)
    assert np.array_equal(yd.cpu().numpy(), 0.5 * x.transpose(1, 0, 2, 3) + (-2.0) * y)


@pytest.mark.parametrize("ldc", [4, 5, 7])
def test_gemm_empty_contraction_strided_c(ctx, ldc):
    """K = 0 scales C in place, row stride ldc (odd ldc: rows start at odd
    element offsets, so elements cannot move in aligned pairs); the columns
    past N are left alone."""
    import ctypes as C
    from paper_2409_06759_amd import _lib as L
    M, N = 3, 4
    rng = np.random.default_rng(ldc)
    c0 = rng.normal(size=(M, ldc))
    Cd = torch.from_numpy(c0).cuda()
    A = torch.zeros(16, dtype=torch.float64, device="cuda")
    ctx.enter()
    ctx.check(ctx.lib.cc_gemm(ctx.h, L.CC_PREC_F64, L.CC_R64, M, N, 0, 1.0, C.c_void_p(A.data_ptr()), 1, 1,
                              C.c_void_p(A.data_ptr()), 1, 1, -0.5, C.c_void_p(Cd.data_ptr()), ldc))
    want = c0.copy()
    want[:, :N] *= -0.5
    assert np.array_equal(Cd.cpu().numpy(), want)
