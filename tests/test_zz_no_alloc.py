"""The GEMM entry point that allocates nothing (cc_gemm_noalloc) against
cc_gemm: the same results to the FP64 error bound, on two calls in a row
whose second is smaller (the static scratch keeps the first call's partial
sums), real shapes split along K and a complex one."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _bound(A, B, C0, alpha, beta):
    K = A.shape[1]
    eps = np.finfo(np.float64).eps
    return 4 * (K + 2) * eps * (abs(alpha) * (np.abs(A) @ np.abs(B).T) + abs(beta) * np.abs(C0))


def _case(E, ctx, M, N, K, seed, akc=True, bkc=True, cplx=False):
    rng = np.random.default_rng(seed)
    if cplx:
        A = rng.normal(size=(M, K)) + 1j * rng.normal(size=(M, K))
        B = rng.normal(size=(N, K)) + 1j * rng.normal(size=(N, K))
        C0 = rng.normal(size=(M, N)) + 1j * rng.normal(size=(M, N))
    else:
        A, B, C0 = rng.normal(size=(M, K)), rng.normal(size=(N, K)), rng.normal(size=(M, N))
    alpha, beta = 0.75, -0.5
    ref = alpha * (A @ B.T) + beta * C0
    Ad = torch.from_numpy(A if akc else np.ascontiguousarray(A.T)).cuda()
    Bd = torch.from_numpy(B if bkc else np.ascontiguousarray(B.T)).cuda()
    c_alloc = torch.from_numpy(C0).cuda()
    c_static = torch.from_numpy(C0).cuda()
    E.gemm(ctx, Ad, Bd, c_alloc, alpha, beta, a_kcontig=akc, b_kcontig=bkc)
    E.gemm_noalloc(ctx, Ad, Bd, c_static, alpha, beta, a_kcontig=akc, b_kcontig=bkc)
    torch.cuda.synchronize()
    got, want = c_static.cpu().numpy(), c_alloc.cpu().numpy()
    bound = _bound(np.abs(A), np.abs(B), np.abs(C0), alpha, beta) + 1e-300
    assert np.all(np.abs(got - ref) <= bound), np.abs(got - ref).max()
    assert np.all(np.abs(got - want) <= 2 * bound), np.abs(got - want).max()
    return got


@pytest.fixture(scope="module")
def ctx():
    from paper_2409_06759_amd import engine as E
    c = E.Context(0)
    yield c
    c.close()


def test_noalloc_gemm_two_calls_second_smaller(ctx):
    from paper_2409_06759_amd import engine as E
    from paper_2409_06759_amd import _lib as L
    lib = L.load()
    # split along K (few output tiles, long K): partial sums in the static scratch
    for M, N, K, seed in ((96, 200, 20000, 1), (33, 17, 4099, 2)):
        print(f"noalloc gemm M={M} N={N} K={K}", flush=True)
        _case(E, ctx, M, N, K, seed)
    # K-strided operands, then a complex GEMM (no scratch), then a plain real one again
    _case(E, ctx, 130, 70, 3000, 3, akc=False, bkc=False)
    _case(E, ctx, 40, 24, 900, 4, cplx=True)
    _case(E, ctx, 17, 9, 513, 5)
    assert lib.cc_gemm_tile_count(0) > 0


def test_noalloc_gemm_rejects_bad_arguments(ctx):
    from paper_2409_06759_amd import _lib as L
    lib = L.load()
    x = torch.zeros(16, dtype=torch.float64, device="cuda")
    p = x.data_ptr()
    # neither operand stride is one
    assert lib.cc_gemm_noalloc(ctx.h, 0, 2, 2, 2, 1.0, p, 2, 2, p, 1, 2, 0.0, p, 2) == L.CC_EINVAL
    # ldc < N
    assert lib.cc_gemm_noalloc(ctx.h, 0, 2, 4, 2, 1.0, p, 2, 1, p, 2, 1, 0.0, p, 2) == L.CC_EINVAL
    assert b"ldc" in lib.cc_last_error(ctx.h)
    # unknown scalar type
    assert lib.cc_gemm_noalloc(ctx.h, 7, 2, 2, 2, 1.0, p, 2, 1, p, 2, 1, 0.0, p, 2) == L.CC_EINVAL
