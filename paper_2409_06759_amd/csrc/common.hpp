// Shared host/device definitions of the coupled-cluster engine (gfx950).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <stdexcept>
#include <string>

namespace ccmi {

// Error raised inside the library; converted to a cc_status at the ABI.
struct CCError : public std::runtime_error {
  int status;
  CCError(int s, const std::string &m) : std::runtime_error(m), status(s) {}
};

#define CC_HIP_CHECK(expr)                                                                  \
  do {                                                                                      \
    hipError_t _e = (expr);                                                                 \
    if (_e != hipSuccess)                                                                   \
      throw ::ccmi::CCError(-3, std::string(#expr) + ": " + hipGetErrorString(_e));         \
  } while (0)

#define CC_REQUIRE(cond, status, msg)                                                       \
  do {                                                                                      \
    if (!(cond)) throw ::ccmi::CCError((status), (msg));                                    \
  } while (0)

constexpr int kWave = 64;
constexpr int kNumXcd = 8;   // MI355X: 8 accelerator complex dies, round-robin dispatch

// Workgroup-id remap so that consecutive logical tiles land on the same XCD
// (workgroups are dispatched round-robin over the XCDs; each has its own L2).
__device__ __forceinline__ int64_t xcd_remap(int64_t bid, int64_t total) {
  const int64_t per = total / kNumXcd, rem = total % kNumXcd;
  const int64_t x = bid % kNumXcd, l = bid / kNumXcd;
  return (x < rem) ? x * (per + 1) + l : rem * (per + 1) + (x - rem) * per + l;
}

// ---- LDS-direct loads ----
// 16 bytes per lane from src (global) into LDS at lds_base + 16 * lane, with
// lds_base a wave-uniform byte offset in the shared aperture.  Issued from
// inline assembly so that the compiler inserts no waits for it: the caller
// waits with s_waitcnt vmcnt (vector memory operations of a wave complete in
// issue order).  One wait state separates the M0 write from the load; the
// kernels that use it use M0 for nothing else.
#pragma clang diagnostic push
#pragma clang diagnostic ignored "-Winline-asm"  // m0 is a reserved register
__device__ __forceinline__ void lds_load16(const void *src, uint32_t lds_base) {
  asm volatile("s_mov_b32 m0, %1\n\ts_nop 0\n\tglobal_load_lds_dwordx4 %0, off" ::"v"(src), "s"(lds_base)
               : "memory", "m0");
}
#pragma clang diagnostic pop

// ---- GEMM descriptor: C[m][n] = alpha * sum_k A(m,k) B(n,k) + beta * C ----
struct GemmDesc {
  int64_t M, N, K;
  const void *A;
  int64_t sam, sak;  // A(m,k) = A[m*sam + k*sak]
  const void *B;
  int64_t sbn, sbk;  // B(n,k) = B[n*sbn + k*sbk]
  void *C;
  int64_t ldc;       // C[m*ldc + n]
  double alpha, beta;
  int conj_a = 0, conj_b = 0;  // complex only
  int ladder = 0;              // 1: the ladder's own kernel symbol (profiling); 2: its cut tail
  int split = 1;               // split-K factor; > 1 needs ws of split*M*N elements
  void *ws = nullptr;
  int64_t ws_elems = 0;        // capacity of ws in elements (the tail cut checks it)
  // reduced precision with converted operands ("shadows"): A and B point to
  // FP32 (F32) or to bf16 hi planes whose lo planes follow at +a_plane /
  // +b_plane elements (BF16X3), indexed exactly like the FP64 tensors
  // (lp_in 1), or, split bf16 only, in the 16 x 32 blocks of
  // convert_blocked (lp_in 2: K-contiguous rows of K, K a multiple of 32;
  // only the LDS-direct configurations read them).
  int lp_in = 0;
  int64_t a_plane = 0, b_plane = 0;
};

// FP64 tensor -> reduced-precision shadow with the same element indexing.
void convert_shadow(int prec, const double *src, int64_t n, void *dst, hipStream_t s);
// Row-major R x K FP64 operand (minus ref, if not NULL) -> split-bf16 copy
// in 16-row x 32-k blocks (rows padded to a multiple of 16); each plane
// holds blocked_plane(R, K) elements, lo after hi.
int64_t blocked_plane(int64_t R, int64_t K);
void convert_blocked(const double *src, const double *ref, int64_t R, int64_t K, void *dst, hipStream_t s);
bool gemm_lowp_tile_blocked(int prec, int tile_id);  // its LDS-direct kernel reads blocked copies
// dst = reduced-precision (a - ref), same layout as convert_shadow.
void convert_delta(int prec, const double *a, const double *ref, int64_t n, void *dst, hipStream_t s);
void copy_f64(double *dst, const double *src, int64_t n, hipStream_t s);
// Complex operands of a reduced-precision complex GEMM as real ones: side 0
// writes A' = [Re A(r,k), Im A(r,k)] (R x 2K), side 1 writes B' (2R x 2K)
// with rows [Re B, -Im B] and [Im B, Re B], from the complex tensor src
// (element (r,k) at r*sr + k*sk) minus ref (or NULL) at the same indexing;
// dense rows of 2K, FP32 or a bf16 hi plane followed by a lo plane.
void realify_complex(int prec, int side, const double *src, const double *ref, int64_t R, int64_t K, int64_t sr,
                     int64_t sk, void *dst, hipStream_t s);
// The same split-bf16 copies of dense rows (sr = K, sk = 1) in the 16 x 32
// blocks of convert_blocked (rows of 2K, K a multiple of 16): planes of
// blocked_plane(R, 2K) (side 0) or blocked_plane(2R, 2K) (side 1) elements;
// rows past the copy's are left as they are.
void realify_complex_blocked(int side, const double *src, int64_t R, int64_t K, void *dst, hipStream_t s);
// The real reduced-precision GEMM (M x 2N x 2K) on realified operands that
// computes the complex GEMM d in its interleaved output layout.
GemmDesc realified_desc(const GemmDesc &d, const void *a_form, const void *b_form);
// C = beta C + P with P dense M x N and C of leading dimension ldc.
void add_product(double *C, int64_t ldc, double beta, const double *P, int64_t M, int64_t N, hipStream_t s);

enum Prec { PREC_F64 = 0, PREC_F32 = 1, PREC_BF16X3 = 2 };

// Grouped launches: entry b of a group describes system b's share; the
// workgroup range of system b is [off[b], off[b+1]).
struct GemmGroupEntry {
  GemmDesc d;
  int64_t tilesM, tilesN;
};

__device__ __forceinline__ int group_find(const int64_t *off, int n, int64_t bid) {
  int lo = 0, hi = n - 1;  // largest b with off[b] <= bid
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (off[mid] <= bid) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// Tile configuration chosen by the tuner for one GEMM shape.
struct GemmTile {
  int id;  // index into the instantiated configuration table
};

void gemm_f64(const GemmDesc &d, hipStream_t s, int tile_id = -1);
void gemm_f64_grouped_launch(const GemmGroupEntry *dev_entries, const int64_t *dev_off, int n,
                             int64_t blocks, bool akc, bool bkc, int tile_id, hipStream_t s);
void gemm_f64_tile_shape(int tile_id, int *bm, int *bn);
void gemm_lowp(const GemmDesc &d, int prec, hipStream_t s, int tile_id = -1);
void gemm_c128(const GemmDesc &d, hipStream_t s, int tile_id = -1);
int gemm_c128_num_tiles();
const char *gemm_c128_tile_name(int id);
int gemm_f64_num_tiles();
const char *gemm_f64_tile_name(int id);
int gemm_f64_pick(int64_t M, int64_t N, int64_t K, bool a_kc, bool b_kc);
int gemm_split_pick(int64_t M, int64_t N, int64_t K, int tile_id);
int gemm_lowp_pick(int prec, int64_t M, int64_t N);
void gemm_lowp_tile_shape(int prec, int tile_id, int *bm, int *bn);
bool gemm_lowp_tile_grouped(int prec, int tile_id);  // has a grouped launch
void gemm_lowp_grouped_launch(const GemmGroupEntry *dev_entries, const int64_t *dev_off, int n, int64_t blocks,
                              bool akc, bool bkc, int prec, int tile_id, hipStream_t s);
int gemm_lowp_num_tiles(int prec);
const char *gemm_lowp_tile_name(int prec, int id);
void splitk_reduce(bool cplx, const void *ws, int split, int64_t M, int64_t N, void *C, int64_t ldc,
                   double alpha, double beta, hipStream_t s);

// ---- tail rounds ----
// T workgroups on S resident slots (workgroups per CU x CUs) run in
// ceil(T / S) rounds.  When the last round is at most half full, the GEMM is
// cut into a main part of whole row or column panels that fills the full
// rounds, and a tail sub-GEMM split along K whose split * tiles workgroups
// fill one short round (partial sums in ws, reduced in a fixed order).
struct TailCut {
  int axis = 0;          // 0: no cut; 1: columns [0, main) are the main part; 2: rows [0, main)
  int64_t main = 0;
  int split = 1;
  int64_t ws_elems = 0;  // split x tail rows x tail columns
};
TailCut gemm_tail_cut(int64_t M, int64_t N, int64_t K, int BM, int BN, int BK, int64_t slots);
// Split-K factor for a launch the plan split along K (split > 1): the factor
// in [1, 16] that minimises rounds per unit of K for this tile's resident
// slots (within ws_elems, at least 8 chunks per split); the plan's factor
// unless another is better.  Large GEMMs only, as for the tail cut.
int gemm_split_refine(int64_t M, int64_t N, int64_t K, int BM, int BN, int BK, int64_t slots, int split,
                      int64_t ws_elems);
// Workspace that covers the tail cut of every tile configuration (0 when
// the GEMM is too small for any cut); no device query needed.
int64_t gemm_tail_ws_bound(int64_t M, int64_t N, int64_t K);
// Exact workspace the tail cut of one launch needs (0: no cut).
int64_t gemm_f64_tail_ws(const GemmDesc &d, int tile_id);
int64_t gemm_lowp_tail_ws(const GemmDesc &d, int prec, int tile_id);
int gpu_cu_count();

// Runs `launch(desc)` on the main part and then on the K-split tail.  `esa`,
// `esb` are the element sizes of A and B (pointer offsets of the panels).
template <class Launch>
void gemm_run_cut(const GemmDesc &d, const TailCut &tc, size_t esa, size_t esb, Launch &&launch) {
  GemmDesc mainp = d, tail = d;
  if (tc.axis == 1) {
    mainp.N = tc.main;
    tail.N = d.N - tc.main;
    tail.B = static_cast<const char *>(d.B) + size_t(tc.main * d.sbn) * esb;
    tail.C = static_cast<double *>(d.C) + tc.main;
  } else {
    mainp.M = tc.main;
    tail.M = d.M - tc.main;
    tail.A = static_cast<const char *>(d.A) + size_t(tc.main * d.sam) * esa;
    tail.C = static_cast<double *>(d.C) + tc.main * d.ldc;
  }
  mainp.split = 1;
  tail.split = tc.split;
  if (tail.ladder) tail.ladder = 2;  // its own kernel symbol
  launch(mainp);
  launch(tail);
}

// ---- dense rank<=6 tensor views for permutation kernels ----
constexpr int kMaxRank = 6;
struct PermDesc {
  int rank;
  int64_t out_dims[kMaxRank];   // output dims
  int64_t in_strides[kMaxRank]; // stride in the input for each OUTPUT dim
  int64_t out_strides[kMaxRank];// output strides (dense row-major normally)
  double alpha, beta;
  int conj;
};
void permute_f64(const PermDesc &d, const void *in, void *out, hipStream_t s);
void permute_c128(const PermDesc &d, const void *in, void *out, hipStream_t s);

}  // namespace ccmi
