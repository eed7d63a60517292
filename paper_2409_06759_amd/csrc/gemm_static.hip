// cc_gemm_noalloc: the kernel-level GEMM for callers that cannot allocate
// device memory.  Its only scratch memory -- the split-K partial sums and the
// partial sums of the K-split tail of a launch whose last round would be
// mostly empty -- lives in a file-scope device array of fixed size instead of
// a buffer the context grows with hipMalloc.
//
// Each device the library runs on holds its own copy of the array until the
// process ends.  Host code never passes the array's name to a kernel (on the
// host that name is only a stand-in for the symbol): the device address is
// looked up once per device with hipGetSymbolAddress, with that device
// current, and kept in a per-device table.
#include <mutex>
#include <string>

#include "plan.hpp"

namespace {

// 128 MiB of FP64 partial sums per device.
constexpr int64_t kScratchElems = int64_t(1) << 24;
constexpr int kMaxDevices = 64;

static __device__ __align__(256) double scratch[kScratchElems];

std::mutex g_mu;
void *g_scratch_ptr[kMaxDevices] = {nullptr};

thread_local std::string g_err;

int fail(cc_ctx *ctx, int status, const std::string &msg) {
  if (ctx) ctx->last_error = msg;
  g_err = msg;
  return status;
}

}  // namespace

namespace ccmi {

// Device address of this device's copy of the scratch array; the current
// device must be `device`.  Looked up on first use and cached.
void *static_scratch(int device) {
  CC_REQUIRE(device >= 0 && device < kMaxDevices, CC_EINVAL, "device index beyond the scratch table");
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_scratch_ptr[device]) {
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || p == nullptr) {
      (void)hipGetLastError();
      throw CCError(CC_EDEVICE, std::string("hipGetSymbolAddress(scratch) failed: ") + hipGetErrorString(e));
    }
    g_scratch_ptr[device] = p;
  }
  return g_scratch_ptr[device];
}

int64_t static_scratch_elems() { return kScratchElems; }

}  // namespace ccmi

extern "C" int cc_gemm_noalloc(cc_ctx *ctx, int scalar, int64_t M, int64_t N, int64_t K, double alpha,
                               const void *A, int64_t sam, int64_t sak, const void *B, int64_t sbn,
                               int64_t sbk, double beta, void *C, int64_t ldc) {
  if (!ctx) return fail(nullptr, CC_EINVAL, "ctx is NULL");
  try {
    if (scalar != CC_R64 && scalar != CC_C128) throw ccmi::CCError(CC_EINVAL, "unknown scalar type");
    if (M < 0 || N < 0 || K < 0) throw ccmi::CCError(CC_EINVAL, "negative GEMM size");
    if (M == 0 || N == 0) return CC_OK;
    auto check = [](const void *p, const char *what) {
      if (!p) throw ccmi::CCError(CC_EINVAL, std::string(what) + " is NULL");
      if (reinterpret_cast<uintptr_t>(p) & 15u) throw ccmi::CCError(CC_EINVAL, std::string(what) + " is not 16-byte aligned");
    };
    check(C, "C");
    if (K > 0) {
      check(A, "A");
      check(B, "B");
    }
    if (!(sam == 1 || sak == 1) || !(sbn == 1 || sbk == 1))
      throw ccmi::CCError(CC_EINVAL, "each operand needs one unit stride");
    if (ldc < N) throw ccmi::CCError(CC_EINVAL, "ldc < N");
    CC_HIP_CHECK(hipSetDevice(ctx->device));
    ccmi::GemmDesc d{M, N, K, A, sam, sak, B, sbn, sbk, C, ldc, alpha, beta};
    if (scalar == CC_C128) {
      // the complex GEMM runs as one launch and uses no scratch memory
      ccmi::gemm_c128(d, ctx->stream, -1);
      return CC_OK;
    }
    if (K > 0) {
      // split along K as cc_gemm does; the partial sums must fit the array
      const int split = ccmi::gemm_split_pick(M, N, K, -1);
      if (split > 1 && int64_t(split) * M * N > kScratchElems)
        throw ccmi::CCError(CC_EINVAL, "GEMM of " + std::to_string(M) + " x " + std::to_string(N) + " split " +
                                           std::to_string(split) + " ways along K needs " +
                                           std::to_string(int64_t(split) * M * N * 8) +
                                           " bytes of partial sums; the static scratch holds " +
                                           std::to_string(kScratchElems * 8));
      d.split = split;
      d.ws = ccmi::static_scratch(ctx->device);
      d.ws_elems = kScratchElems;
    }
    ccmi::gemm_f64(d, ctx->stream, -1);
    return CC_OK;
  } catch (const ccmi::CCError &e) {
    return fail(ctx, e.status, e.what());
  } catch (const std::exception &e) {
    return fail(ctx, CC_EINTERNAL, e.what());
  }
}
