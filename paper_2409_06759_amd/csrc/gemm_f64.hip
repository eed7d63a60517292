// FP64 MFMA GEMM for gfx950:  C[m][n] = alpha * sum_k A(m,k) B(n,k) + beta * C[m][n].
//
// This is the GEMM step of the transpose-transpose-GEMM-transpose evaluation
// of a binary tensor contraction (paper, Sec. "Tensor contractions"); the
// particle-particle ladder R_ij^ab += 1/2 sum_ef tau_ij^ef <ab||ef> is one call
// with A = tau[(ij)][(ef)] and B = vvvv[(ab)][(ef)], both K-contiguous.
//
// Design (CDNA4):
// * v_mfma_f64_16x16x4_f64: each lane holds one A and one B value and four
//   accumulators.  Lane l covers row (l & 15) of A / column (l & 15) of B and
//   k-slot (l >> 4); accumulator t of lane l is C[(l >> 4) + 4t][l & 15].
//   Four consecutive MFMAs consume 16 k values: in MFMA s lane group
//   q = l >> 4 supplies logical k = 4q + s, identically for A and B, so each
//   lane reads 4 consecutive k of its row when the operand is K-contiguous.
// * Staged configurations: block tile BM x BN, K chunk BK, staged through LDS
//   with two buffers; the next chunk's global loads are in flight (in
//   registers) while the current one is multiplied.  Operands may be
//   K-contiguous or M/N-contiguous; the LDS layout follows the global one so
//   both the HBM reads and the LDS fragment reads stay unit-stride.
// * The LDS-direct configuration (256x128x16) takes K-contiguous operands
//   with global_load_lds_dwordx4 into three LDS stages (see its kernel).
// * Workgroup ids are remapped so that the M tiles sharing one N tile are
//   dispatched to the same XCD (shared L2 for the B panel).
// * A launch whose last round of resident workgroups would be at most half
//   full runs as whole rounds plus a K-split tail (gemm_tail_cut), and the
//   split-K factor of a plan is re-chosen for the tile's resident workgroups
//   (gemm_split_refine).
#include "common.hpp"

#include <algorithm>
#include <atomic>
#include <mutex>

#include <cmath>

namespace ccmi {
namespace {

typedef double d4 __attribute__((ext_vector_type(4)));

template <int BM, int BN, int BK, int WM, int WN, bool AKC, bool BKC>
struct Cfg {
  static constexpr int NT = WM * WN * kWave;
  static constexpr int WTM = BM / WM, WTN = BN / WN;
  static constexpr int FM = WTM / 16, FN = WTN / 16;
  static constexpr int PAD = 2;
  // LDS panel shapes (rows x row-stride) per operand
  static constexpr int A_ROWS = AKC ? BM : BK, A_LD = AKC ? BK + PAD : BM + PAD;
  static constexpr int B_ROWS = BKC ? BN : BK, B_LD = BKC ? BK + PAD : BN + PAD;
  static constexpr int A_ELEMS = A_ROWS * A_LD, B_ELEMS = B_ROWS * B_LD;
  static constexpr int LA = BM * BK / NT, LB = BN * BK / NT;  // global loads per thread
  static_assert(BM % (16 * WM) == 0 && BN % (16 * WN) == 0, "tile/wave mismatch");
  static_assert(BK % 16 == 0, "BK must be a multiple of 16");
  static_assert((BM * BK) % NT == 0 && (BN * BK) % NT == 0, "load split");
};

// One workgroup's share of a GEMM: logical tile L0 in [0, tiles * split).
template <int BM, int BN, int BK, int WM, int WN, bool AKC, bool BKC>
__device__ __forceinline__ void gemm_f64_body(const GemmDesc &d, int64_t tilesM, int64_t tilesN,
                                              int64_t L0) {
  using C = Cfg<BM, BN, BK, WM, WN, AKC, BKC>;
  __shared__ __attribute__((aligned(16))) double smem[2 * (C::A_ELEMS + C::B_ELEMS)];
  // buffer b of A at smem + b*A_ELEMS, of B at smem + 2*A_ELEMS + b*B_ELEMS

  const int64_t tiles = tilesM * tilesN;
  const int64_t ks = L0 / tiles, L = L0 % tiles;
  const int64_t m0 = (L % tilesM) * BM, n0 = (L / tilesM) * BN;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm0 = (wave / WN) * C::WTM, wn0 = (wave % WN) * C::WTN;
  const int q = lane >> 4, r = lane & 15;

  const double *__restrict__ A = static_cast<const double *>(d.A);
  const double *__restrict__ B = static_cast<const double *>(d.B);
  const int64_t M = d.M, N = d.N;
  // split-K: this workgroup covers k in [kb, kb + K) of the full range
  const int64_t kchunk = ((d.K + d.split - 1) / d.split + BK - 1) / BK * BK;
  const int64_t kb = ks * kchunk;
  const int64_t K = std::max<int64_t>(0, std::min<int64_t>(d.K - kb, kchunk));
  A += kb * d.sak;
  B += kb * d.sbk;

  // Global -> register staging in 16-byte vectors (two doubles along the
  // unit-stride dimension) when the strides and base allow it; otherwise the
  // same vectors are assembled element by element.  Out-of-range elements are 0.
  constexpr int AR = AKC ? BM : BK, AC = AKC ? BK : BM, BR = BKC ? BN : BK, BC = BKC ? BK : BN;
  constexpr int ANV = AR * AC / 2, BNV = BR * BC / 2;
  constexpr int AVT = (ANV + C::NT - 1) / C::NT, BVT = (BNV + C::NT - 1) / C::NT;
  typedef double d2 __attribute__((ext_vector_type(2)));
  d2 ra[AVT], rb[BVT];
  const bool vec_a = ((AKC ? d.sam : d.sak) % 2 == 0) && ((reinterpret_cast<uintptr_t>(A) & 15) == 0);
  const bool vec_b = ((BKC ? d.sbn : d.sbk) % 2 == 0) && ((reinterpret_cast<uintptr_t>(B) & 15) == 0);

  auto vload = [&](const double *base, int64_t rstride, int64_t r_lim, int64_t c_lim, int64_t r0, int64_t c0,
                   bool vec_ok, int v, int ncolv) -> d2 {
    const int rr = v / ncolv, cc = (v % ncolv) * 2;
    const int64_t gr = r0 + rr, gc = c0 + cc;
    const double *src = base + gr * rstride + gc;
    if (vec_ok && gr < r_lim && gc + 2 <= c_lim) return *reinterpret_cast<const d2 *>(src);
    d2 t;
    t.x = (gr < r_lim && gc < c_lim) ? src[0] : 0.0;
    t.y = (gr < r_lim && gc + 1 < c_lim) ? src[1] : 0.0;
    return t;
  };
  auto gload = [&](int64_t k0) {
#pragma unroll
    for (int i = 0; i < AVT; ++i) {
      const int v = tid + i * C::NT;
      if (ANV % C::NT == 0 || v < ANV)
        ra[i] = AKC ? vload(A, d.sam, M, K, m0, k0, vec_a, v, AC / 2) : vload(A, d.sak, K, M, k0, m0, vec_a, v, AC / 2);
    }
#pragma unroll
    for (int i = 0; i < BVT; ++i) {
      const int v = tid + i * C::NT;
      if (BNV % C::NT == 0 || v < BNV)
        rb[i] = BKC ? vload(B, d.sbn, N, K, n0, k0, vec_b, v, BC / 2) : vload(B, d.sbk, K, N, k0, n0, vec_b, v, BC / 2);
    }
  };
  auto sstore = [&](int buf) {
#pragma unroll
    for (int i = 0; i < AVT; ++i) {
      const int v = tid + i * C::NT;
      if (ANV % C::NT == 0 || v < ANV) {
        const int rr = v / (AC / 2), cc = (v % (AC / 2)) * 2;
        *reinterpret_cast<d2 *>(smem + buf * C::A_ELEMS + rr * C::A_LD + cc) = ra[i];
      }
    }
#pragma unroll
    for (int i = 0; i < BVT; ++i) {
      const int v = tid + i * C::NT;
      if (BNV % C::NT == 0 || v < BNV) {
        const int rr = v / (BC / 2), cc = (v % (BC / 2)) * 2;
        *reinterpret_cast<d2 *>(smem + 2 * C::A_ELEMS + buf * C::B_ELEMS + rr * C::B_LD + cc) = rb[i];
      }
    }
  };

  d4 acc[C::FM][C::FN];
#pragma unroll
  for (int i = 0; i < C::FM; ++i)
#pragma unroll
    for (int j = 0; j < C::FN; ++j) acc[i][j] = d4{0.0, 0.0, 0.0, 0.0};

  const int64_t nk = (K + BK - 1) / BK;
  gload(0);
  sstore(0);
  __syncthreads();
  for (int64_t kt = 0; kt < nk; ++kt) {
    const int buf = kt & 1;
    if (kt + 1 < nk) gload((kt + 1) * BK);
    const double *as = smem + buf * C::A_ELEMS, *bs = smem + 2 * C::A_ELEMS + buf * C::B_ELEMS;
#pragma unroll
    for (int kc = 0; kc < BK; kc += 16) {
      double fa[C::FM][4], fb[C::FN][4];
#pragma unroll
      for (int i = 0; i < C::FM; ++i) {
        const int mm = wm0 + i * 16 + r;
#pragma unroll
        for (int s = 0; s < 4; ++s)
          fa[i][s] = AKC ? as[mm * C::A_LD + kc + 4 * q + s] : as[(kc + 4 * q + s) * C::A_LD + mm];
      }
#pragma unroll
      for (int j = 0; j < C::FN; ++j) {
        const int nn = wn0 + j * 16 + r;
#pragma unroll
        for (int s = 0; s < 4; ++s)
          fb[j][s] = BKC ? bs[nn * C::B_LD + kc + 4 * q + s] : bs[(kc + 4 * q + s) * C::B_LD + nn];
      }
#pragma unroll
      for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int i = 0; i < C::FM; ++i)
#pragma unroll
          for (int j = 0; j < C::FN; ++j)
            acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(fa[i][s], fb[j][s], acc[i][j], 0, 0, 0);
    }
    if (kt + 1 < nk) sstore(buf ^ 1);
    __syncthreads();
  }

  // epilogue: accumulator t of lane l holds row (l >> 4) + 4t, column l & 15
  // of its 16x16 block (f64 MFMA output layout, checked on the device)
  double *__restrict__ Cp = static_cast<double *>(d.C);
  double alpha = d.alpha, beta = d.beta;
  int64_t ldc = d.ldc;
  if (d.split > 1) {  // raw partial sums; splitk_reduce applies alpha and beta
    Cp = static_cast<double *>(d.ws) + ks * M * N;
    alpha = 1.0;
    beta = 0.0;
    ldc = N;
  }
#pragma unroll
  for (int i = 0; i < C::FM; ++i)
#pragma unroll
    for (int j = 0; j < C::FN; ++j) {
      const int64_t gn = n0 + wn0 + j * 16 + r;
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int64_t gm = m0 + wm0 + i * 16 + q + 4 * t;
        if (gm < M && gn < N) {
          double *p = Cp + gm * ldc + gn;
          const double v = alpha * acc[i][j][t];
          *p = (beta == 0.0) ? v : v + beta * *p;
        }
      }
    }
}

template <int BM, int BN, int BK, int WM, int WN, bool AKC, bool BKC, int TAG>
__global__ __launch_bounds__(WM *WN *kWave) void gemm_f64_kernel(GemmDesc d, int64_t tilesM,
                                                                  int64_t tilesN) {
  const int64_t total = tilesM * tilesN * d.split;
  gemm_f64_body<BM, BN, BK, WM, WN, AKC, BKC>(d, tilesM, tilesN, xcd_remap(blockIdx.x, total));
}

// Grouped launch: one workgroup range per system; system b owns logical
// tiles [g.off[b], g.off[b+1]).  Same arithmetic as the single launch.
template <int BM, int BN, int BK, int WM, int WN, bool AKC, bool BKC>
__global__ __launch_bounds__(WM *WN *kWave) void gemm_f64_grouped(const GemmGroupEntry *__restrict__ e,
                                                                   const int64_t *__restrict__ off, int n) {
  const int b = group_find(off, n, blockIdx.x);
  const GemmGroupEntry &g = e[b];
  gemm_f64_body<BM, BN, BK, WM, WN, AKC, BKC>(g.d, g.tilesM, g.tilesN, int64_t(blockIdx.x) - off[b]);
}

// ---- 256x128x16 with LDS-direct loads ---------------------------------------
// K a multiple of 16, both operands K-contiguous with 16-byte aligned rows
// (the particle-particle ladder's layout); rows past M or N load the last
// valid row instead, which only reaches outputs that are never stored.  Each lane's 16
// bytes go straight from HBM/L2 into LDS (global_load_lds_dwordx4): no
// staging registers, three LDS stages, two chunks of K in flight.  A 16-row
// block of a stage is two halves of 64 slots of 16 bytes; slot L of half h
// holds row (L & 15), k = 4 (L >> 4) + 2h + {0, 1}, so lane L reads the four
// k values it feeds the f64 MFMA (k = 4q + s, as in the staged kernel) as
// two 16-byte reads, each contiguous across the wave (no bank conflicts).  The
// products and their order are those of the staged kernel of the same tile,
// so results are bitwise the same.  Waits: "vmcnt <= 6" after the six loads
// of chunk kt+1 means chunk kt has landed (in-order completion), the barrier
// behind it makes that so for every wave, and "lgkmcnt == 0" before it
// means every wave has finished reading the stage the next loads overwrite.
namespace dma64 {
constexpr int BM = 256, BN = 128, BK = 16, WM = 4, WN = 2, NT = WM * WN * kWave;
constexpr int FM = BM / WM / 16, FN = BN / WN / 16;
constexpr int A_EL = BM * BK, B_EL = BN * BK, STAGE = A_EL + B_EL;  // doubles
constexpr int NSTAGE = 3;
constexpr int LOADS = (2 * (BM / 16) + 2 * (BN / 16)) / (WM * WN);  // per wave and chunk
static_assert(LOADS == 6, "the explicit waits count six loads per chunk");
}  // namespace dma64

__device__ __forceinline__ void gemm_f64_dma_body(const GemmDesc &d, int64_t tilesM, int64_t tilesN, int64_t L0) {
  using namespace dma64;
  __shared__ __attribute__((aligned(16))) double S[NSTAGE * STAGE];

  const int64_t tiles = tilesM * tilesN;
  const int64_t ks = L0 / tiles, L = L0 % tiles;
  const int64_t m0 = (L % tilesM) * BM, n0 = (L / tilesM) * BN;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm0 = (wave / WN) * (BM / WM), wn0 = (wave % WN) * (BN / WN);
  const int q = lane >> 4, r = lane & 15;
  const int64_t M = d.M, N = d.N;
  const int64_t kchunk = ((d.K + d.split - 1) / d.split + BK - 1) / BK * BK;
  const int64_t kb = ks * kchunk;
  const int64_t K = std::max<int64_t>(0, std::min<int64_t>(d.K - kb, kchunk));
  const int64_t nk = K / BK;

  // this wave's loads: A blocks 2w and 2w+1, B block w, each as two halves;
  // lane l of half h loads row (l & 15), k = 4 (l >> 4) + 2h + {0, 1}
  const uint32_t lds0 = static_cast<uint32_t>(reinterpret_cast<uintptr_t>(S));
  const double *src[LOADS];
  uint32_t dst[LOADS];
  const double *Ag = static_cast<const double *>(d.A) + kb;
  const double *Bg = static_cast<const double *>(d.B) + kb;
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int blk = 2 * wave + (u >> 1), h = u & 1;
    src[u] = Ag + std::min<int64_t>(m0 + blk * 16 + r, M - 1) * d.sam + 4 * q + 2 * h;
    dst[u] = __builtin_amdgcn_readfirstlane(lds0 + 8u * uint32_t(blk * 256 + h * 128));
  }
#pragma unroll
  for (int u = 0; u < 2; ++u) {
    src[4 + u] = Bg + std::min<int64_t>(n0 + wave * 16 + r, N - 1) * d.sbn + 4 * q + 2 * u;
    dst[4 + u] = __builtin_amdgcn_readfirstlane(lds0 + 8u * uint32_t(A_EL + wave * 256 + u * 128));
  }
  auto issue = [&](int stage, int64_t k0) {
#pragma unroll
    for (int u = 0; u < LOADS; ++u) lds_load16(src[u] + k0, dst[u] + uint32_t(stage) * uint32_t(8 * STAGE));
  };

  d4 acc[FM][FN];
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j) acc[i][j] = d4{0.0, 0.0, 0.0, 0.0};

  if (nk > 0) issue(0, 0);
  if (nk > 1) issue(1, BK);
  int cur = 0, nxt = 2;
  for (int64_t kt = 0; kt < nk; ++kt) {
    if (kt + 1 < nk) asm volatile("s_waitcnt vmcnt(6) lgkmcnt(0)\n\ts_barrier" ::: "memory");
    else asm volatile("s_waitcnt vmcnt(0) lgkmcnt(0)\n\ts_barrier" ::: "memory");
    if (kt + 2 < nk) issue(nxt, (kt + 2) * BK);
    const double *St = S + cur * STAGE;
    // the k pair of steps 0-1 of every fragment is read first; the pair of
    // steps 2-3 is read behind the MFMAs of step 0, so it overlaps them (at
    // most eight LDS reads in flight, within what lgkmcnt can count)
    typedef double d2 __attribute__((ext_vector_type(2)));
    d2 fa[2][FM], fb[2][FN];
    auto read_pair = [&](int h) {
#pragma unroll
      for (int i = 0; i < FM; ++i)
        fa[h][i] = *reinterpret_cast<const d2 *>(St + ((wm0 >> 4) + i) * 256 + h * 128 + lane * 2);
#pragma unroll
      for (int j = 0; j < FN; ++j)
        fb[h][j] = *reinterpret_cast<const d2 *>(St + A_EL + ((wn0 >> 4) + j) * 256 + h * 128 + lane * 2);
    };
    auto mfma_step = [&](int s) {
#pragma unroll
      for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(fa[s >> 1][i][s & 1], fb[s >> 1][j][s & 1], acc[i][j],
                                                           0, 0, 0);
    };
    read_pair(0);
    __builtin_amdgcn_sched_barrier(0);
    mfma_step(0);
    __builtin_amdgcn_sched_barrier(0);
    read_pair(1);
    __builtin_amdgcn_sched_barrier(0);
    mfma_step(1);
    mfma_step(2);
    mfma_step(3);
    cur = cur == NSTAGE - 1 ? 0 : cur + 1;
    nxt = nxt == NSTAGE - 1 ? 0 : nxt + 1;
  }

  // epilogue (as the staged kernel): accumulator t of lane l holds row
  // (l >> 4) + 4t, column l & 15 of its 16x16 block
  double *__restrict__ Cp = static_cast<double *>(d.C);
  double alpha = d.alpha, beta = d.beta;
  int64_t ldc = d.ldc;
  if (d.split > 1) {
    Cp = static_cast<double *>(d.ws) + ks * M * N;
    alpha = 1.0;
    beta = 0.0;
    ldc = N;
  }
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j) {
      const int64_t gn = n0 + wn0 + j * 16 + r;
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int64_t gm = m0 + wm0 + i * 16 + q + 4 * t;
        if (gm < M && gn < N) {
          double *p = Cp + gm * ldc + gn;
          const double v = alpha * acc[i][j][t];
          *p = (beta == 0.0) ? v : v + beta * *p;
        }
      }
    }
}

template <int TAG>
__global__ __launch_bounds__(dma64::NT) void gemm_f64_dma_kernel(GemmDesc d, int64_t tilesM, int64_t tilesN) {
  gemm_f64_dma_body(d, tilesM, tilesN, xcd_remap(blockIdx.x, tilesM * tilesN * d.split));
}

// the shapes and layouts the LDS-direct kernel handles
bool f64_dma_ok(const GemmDesc &d) {
  return d.sak == 1 && d.sbk == 1 && d.K % dma64::BK == 0 &&
         d.sam % 2 == 0 && d.sbn % 2 == 0 && (reinterpret_cast<uintptr_t>(d.A) & 15) == 0 &&
         (reinterpret_cast<uintptr_t>(d.B) & 15) == 0;
}

struct TileInfo {
  const char *name;
  int BM, BN, BK, threads;
  void (*launch[4])(const GemmDesc &, int64_t, int64_t, hipStream_t);  // [akc*2 + bkc]
  void (*launch_ladder)(const GemmDesc &, int64_t, int64_t, hipStream_t);  // both K-contiguous
  void (*launch_ladder_tail)(const GemmDesc &, int64_t, int64_t, hipStream_t);
  void (*launch_grouped[4])(const GemmGroupEntry *, const int64_t *, int, int64_t, hipStream_t);
  int (*occupancy[4])();  // resident workgroups per CU, [akc*2 + bkc]
};

// Workgroups of one configuration that fit on a CU at once (registers, LDS,
// waves), as the runtime computes it for the compiled kernel; 0 if unknown.
template <int BM, int BN, int BK, int WM, int WN, bool AKC, bool BKC>
int occupancy_cfg() {
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, gemm_f64_kernel<BM, BN, BK, WM, WN, AKC, BKC, 0>,
                                                   WM * WN * kWave, 0) != hipSuccess) {
    (void)hipGetLastError();
    return 0;
  }
  return nb;
}

template <int BM, int BN, int BK, int WM, int WN, bool AKC, bool BKC>
void launch_grp(const GemmGroupEntry *e, const int64_t *off, int n, int64_t blocks, hipStream_t s) {
  hipLaunchKernelGGL((gemm_f64_grouped<BM, BN, BK, WM, WN, AKC, BKC>), dim3(blocks), dim3(WM * WN * kWave),
                     0, s, e, off, n);
}

// TAG only changes the kernel's symbol name: TAG 1 is the particle-particle
// ladder and TAG 2 the K-split tail of a cut ladder launch, so that profilers
// report them on lines of their own.
template <int BM, int BN, int BK, int WM, int WN, bool AKC, bool BKC, int TAG = 0>
void launch_cfg(const GemmDesc &d, int64_t tm, int64_t tn, hipStream_t s) {
  hipLaunchKernelGGL((gemm_f64_kernel<BM, BN, BK, WM, WN, AKC, BKC, TAG>), dim3(tm * tn * d.split),
                     dim3(WM * WN * kWave), 0, s, d, tm, tn);
}

#define CC_TILE(BM, BN, BK, WM, WN)                                                          \
  TileInfo {                                                                                 \
    #BM "x" #BN "x" #BK "_w" #WM "x" #WN, BM, BN, BK, WM *WN * kWave, {                      \
      &launch_cfg<BM, BN, BK, WM, WN, false, false>, &launch_cfg<BM, BN, BK, WM, WN, false, true>, \
          &launch_cfg<BM, BN, BK, WM, WN, true, false>, &launch_cfg<BM, BN, BK, WM, WN, true, true> \
    }, &launch_cfg<BM, BN, BK, WM, WN, true, true, 1>, &launch_cfg<BM, BN, BK, WM, WN, true, true, 2>, \
    {&launch_grp<BM, BN, BK, WM, WN, false, false>, &launch_grp<BM, BN, BK, WM, WN, false, true>, \
     &launch_grp<BM, BN, BK, WM, WN, true, false>, &launch_grp<BM, BN, BK, WM, WN, true, true>},  \
    {&occupancy_cfg<BM, BN, BK, WM, WN, false, false>, &occupancy_cfg<BM, BN, BK, WM, WN, false, true>, \
     &occupancy_cfg<BM, BN, BK, WM, WN, true, false>, &occupancy_cfg<BM, BN, BK, WM, WN, true, true>} \
  }

template <int TAG>
void launch_f64_dma(const GemmDesc &d, int64_t tm, int64_t tn, hipStream_t s) {
  if (f64_dma_ok(d))
    hipLaunchKernelGGL((gemm_f64_dma_kernel<TAG>), dim3(tm * tn * d.split), dim3(dma64::NT), 0, s, d, tm, tn);
  else
    launch_cfg<256, 128, 16, 4, 2, true, true, TAG>(d, tm, tn, s);
}
int occ_f64_dma() {
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, gemm_f64_dma_kernel<0>, dma64::NT, 0) != hipSuccess) {
    (void)hipGetLastError();
    return 0;
  }
  return nb;
}

const TileInfo kTiles[] = {
    CC_TILE(128, 128, 16, 2, 2),
    CC_TILE(128, 160, 16, 2, 2),
    CC_TILE(64, 64, 16, 2, 2),
    CC_TILE(32, 32, 16, 2, 2),
    CC_TILE(256, 128, 16, 4, 2),
    CC_TILE(128, 64, 16, 2, 2),
    CC_TILE(64, 128, 16, 2, 2),
    CC_TILE(128, 128, 32, 2, 2),
    CC_TILE(64, 64, 32, 2, 2),
    CC_TILE(128, 64, 32, 2, 2),
    CC_TILE(64, 128, 32, 2, 2),
    CC_TILE(128, 128, 16, 4, 2),
    CC_TILE(128, 64, 16, 4, 2),
    CC_TILE(64, 128, 16, 2, 4),
    CC_TILE(128, 128, 16, 4, 4),
    CC_TILE(256, 64, 16, 8, 2),
    // 256x128x16 with LDS-direct loads where the shape allows, else staged
    TileInfo{"256x128x16_w4x2_lds",
             256,
             128,
             16,
             4 * 2 * kWave,
             {&launch_cfg<256, 128, 16, 4, 2, false, false>, &launch_cfg<256, 128, 16, 4, 2, false, true>,
              &launch_cfg<256, 128, 16, 4, 2, true, false>, &launch_f64_dma<0>},
             &launch_f64_dma<1>,
             &launch_f64_dma<2>,
             {&launch_grp<256, 128, 16, 4, 2, false, false>, &launch_grp<256, 128, 16, 4, 2, false, true>,
              &launch_grp<256, 128, 16, 4, 2, true, false>, &launch_grp<256, 128, 16, 4, 2, true, true>},
             {&occupancy_cfg<256, 128, 16, 4, 2, false, false>, &occupancy_cfg<256, 128, 16, 4, 2, false, true>,
              &occupancy_cfg<256, 128, 16, 4, 2, true, false>, &occ_f64_dma}},
};
constexpr int kNumTiles = sizeof(kTiles) / sizeof(kTiles[0]);

// resident slots of a configuration on the whole device (cached per process,
// which assumes every device it uses is the same GPU model; -1 = not yet asked)
std::atomic<int64_t> g_slots[kNumTiles][4];
std::once_flag g_slots_once;

int64_t tile_slots(int tile_id, int variant) {
  std::call_once(g_slots_once, [] {
    for (auto &row : g_slots)
      for (auto &x : row) x.store(-1);
  });
  int64_t v = g_slots[tile_id][variant].load();
  if (v < 0) {
    v = int64_t(kTiles[tile_id].occupancy[variant]()) * gpu_cu_count();
    g_slots[tile_id][variant].store(v);
  }
  return v;
}

TailCut f64_cut(const GemmDesc &d, int tile_id) {
  const bool akc = (d.sak == 1), bkc = (d.sbk == 1);
  const TileInfo &ti = kTiles[tile_id];
  if (d.split != 1 || d.K <= 0) return TailCut{};
  return gemm_tail_cut(d.M, d.N, d.K, ti.BM, ti.BN, ti.BK, tile_slots(tile_id, (akc ? 2 : 0) + (bkc ? 1 : 0)));
}

}  // namespace

int gpu_cu_count() {
  static std::atomic<int> cus{0};
  int c = cus.load();
  if (c == 0) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&c, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || c <= 0) {
      (void)hipGetLastError();
      c = 256;
    }
    cus.store(c);
  }
  return c;
}

// A round must carry enough work to pay for the two extra launches (the tail
// and its reduction), about 0.2 ms at the FP64 rate.
constexpr double kTailMinRoundFlops = 1.2e10;

TailCut gemm_tail_cut(int64_t M, int64_t N, int64_t K, int BM, int BN, int BK, int64_t slots) {
  TailCut best;
  if (slots <= 0 || M <= 0 || N <= 0 || K <= 0) return best;
  const int64_t tm = (M + BM - 1) / BM, tn = (N + BN - 1) / BN, tiles = tm * tn;
  if (tiles <= slots || 2.0 * double(slots) * BM * BN * double(K) < kTailMinRoundFlops) return best;
  const int64_t full = tiles / slots, rem = tiles - full * slots;
  if (rem == 0 || 2 * rem > slots) return best;  // the last round is full enough
  double best_rounds = double(full + 1);
  for (int axis = 1; axis <= 2; ++axis) {
    const int64_t per = axis == 1 ? tm : tn;  // tiles per panel
    const int64_t np = axis == 1 ? tn : tm;   // panels
    const int64_t mainp = (full * slots) / per;
    if (mainp <= 0 || mainp >= np) continue;
    const int64_t tail_tiles = (np - mainp) * per;
    int64_t split = std::min<int64_t>({slots / tail_tiles, 16, K / (8 * int64_t(BK))});
    if (split < 2) continue;
    const double rounds = std::ceil(double(mainp * per) / double(slots)) + 1.0 / double(split);
    if (rounds < best_rounds) {
      best_rounds = rounds;
      best.axis = axis;
      best.main = mainp * (axis == 1 ? BN : BM);
      best.split = int(split);
      const int64_t tr = axis == 1 ? M : M - best.main, tc = axis == 1 ? N - best.main : N;
      best.ws_elems = split * tr * tc;
    }
  }
  return best;
}

int gemm_split_refine(int64_t M, int64_t N, int64_t K, int BM, int BN, int BK, int64_t slots, int split,
                      int64_t ws_elems) {
  if (split <= 1 || slots <= 0 || M <= 0 || N <= 0 || K <= 0) return split;
  const int64_t tiles = ((M + BM - 1) / BM) * ((N + BN - 1) / BN);
  if (2.0 * double(std::min(tiles, slots)) * BM * BN * double(K) < kTailMinRoundFlops) return split;
  const int64_t smax = std::min<int64_t>({16, std::max<int64_t>(1, K / (8 * int64_t(BK))), ws_elems / (M * N)});
  // full-K rounds the launch takes with s splits, plus a small charge per
  // split for its partial sums (written once, read once by the reduction)
  auto cost = [&](int64_t s) { return std::ceil(double(tiles * s) / double(slots)) / double(s) + 0.02 * double(s); };
  int best = split <= smax ? split : 1;
  double best_cost = cost(best);
  for (int64_t s = 1; s <= smax; ++s)
    if (cost(s) < best_cost - 1e-9) {
      best_cost = cost(s);
      best = int(s);
    }
  return best;
}

int64_t gemm_tail_ws_bound(int64_t M, int64_t N, int64_t K) {
  if (M <= 0 || N <= 0 || K <= 0 || 2.0 * double(M) * double(N) * double(K) < kTailMinRoundFlops) return 0;
  // split x tail elements <= slots x BM x BN = every resident workgroup's
  // accumulators, bounded by the register file (256 CUs x 512 KiB of 4-byte
  // accumulators); the launch checks the exact figure against ws_elems
  return std::min<int64_t>(16 * M * N, int64_t(1) << 25);
}

int64_t gemm_f64_tail_ws(const GemmDesc &d, int tile_id) {
  if (d.M <= 0 || d.N <= 0 || d.K <= 0) return 0;
  if (tile_id < 0 || tile_id >= kNumTiles) tile_id = gemm_f64_pick(d.M, d.N, d.K, d.sak == 1, d.sbk == 1);
  return f64_cut(d, tile_id).ws_elems;
}

int gemm_f64_num_tiles() { return kNumTiles; }
const char *gemm_f64_tile_name(int id) { return (id >= 0 && id < kNumTiles) ? kTiles[id].name : "?"; }

// Static choice: the tile that minimises (rounds of resident workgroups) x
// (tile work), counting padding; the autotuner refines this by timing.
int gemm_f64_pick(int64_t M, int64_t N, int64_t K, bool, bool) {
  (void)K;
  const double cus = 256.0;
  int best = 0;
  double best_cost = 1e300;
  for (int t = 0; t < kNumTiles; ++t) {
    const TileInfo &ti = kTiles[t];
    if (ti.BK != 16) continue;
    const double tiles = double((M + ti.BM - 1) / ti.BM) * double((N + ti.BN - 1) / ti.BN);
    const double rounds = std::ceil(tiles / cus);
    // a tile's time ~ its MFMA work; small tiles pay a fixed per-tile overhead
    const double cost = rounds * (double(ti.BM) * ti.BN + 4096.0);
    if (cost < best_cost) { best_cost = cost; best = t; }
  }
  return best;
}

// Split-K factor: about 1024 workgroups (four per CU) when the output has
// few tiles and the contraction is long (e.g. M = N = o, K = o v^2), each
// split covering at least 256 of K.
// Independent of the tile so that the autotuner can change tiles freely.
int gemm_split_pick(int64_t M, int64_t N, int64_t K, int) {
  const int64_t tiles = ((M + 63) / 64) * ((N + 63) / 64);
  if (tiles >= 2048) return 1;  // eight 64x64 tiles per CU or more
  int64_t split = (2048 + tiles - 1) / tiles;
  split = std::min<int64_t>(split, std::max<int64_t>(1, K / 256));
  return int(std::max<int64_t>(1, std::min<int64_t>(split, 1024)));
}

void gemm_f64_grouped_launch(const GemmGroupEntry *dev_entries, const int64_t *dev_off, int n,
                             int64_t blocks, bool akc, bool bkc, int tile_id, hipStream_t s) {
  if (blocks <= 0) return;
  CC_REQUIRE(tile_id >= 0 && tile_id < kNumTiles, -7, "grouped gemm: tile");
  CC_REQUIRE(blocks < (int64_t(1) << 31), -1, "grouped gemm: too many tiles");
  kTiles[tile_id].launch_grouped[(akc ? 2 : 0) + (bkc ? 1 : 0)](dev_entries, dev_off, n, blocks, s);
  CC_HIP_CHECK(hipGetLastError());
}

void gemm_f64_tile_shape(int tile_id, int *bm, int *bn) {
  *bm = kTiles[tile_id].BM;
  *bn = kTiles[tile_id].BN;
}

void gemm_f64(const GemmDesc &d, hipStream_t s, int tile_id) {
  if (d.M <= 0 || d.N <= 0) return;
  const bool akc = (d.sak == 1), bkc = (d.sbk == 1);
  CC_REQUIRE(akc || d.sam == 1, -1, "gemm: A needs a unit stride in m or k");
  CC_REQUIRE(bkc || d.sbn == 1, -1, "gemm: B needs a unit stride in n or k");
  if (d.K <= 0) {
    // C = beta * C: a GEMM with an empty contraction still scales C (an
    // in-place, element-by-element identity permutation with alpha = beta)
    PermDesc p{};
    p.rank = 2;
    p.out_dims[0] = d.M; p.out_dims[1] = d.N;
    p.out_strides[0] = d.ldc; p.out_strides[1] = 1;
    p.in_strides[0] = d.ldc; p.in_strides[1] = 1;
    p.alpha = d.beta; p.beta = 0.0; p.conj = 0;
    permute_f64(p, d.C, d.C, s);
    return;
  }
  if (tile_id < 0 || tile_id >= kNumTiles) tile_id = gemm_f64_pick(d.M, d.N, d.K, akc, bkc);
  const TileInfo &ti = kTiles[tile_id];
  const int64_t tm = (d.M + ti.BM - 1) / ti.BM, tn = (d.N + ti.BN - 1) / ti.BN;
  CC_REQUIRE(d.split >= 1, -1, "gemm: split must be >= 1");
  CC_REQUIRE(d.split == 1 || d.ws != nullptr, -1, "gemm: split-K needs a workspace");
  CC_REQUIRE(d.split == 1 || d.ws_elems == 0 || d.ws_elems >= d.split * d.M * d.N, -1,
             "gemm: split-K workspace too small");
  CC_REQUIRE(tm * tn * d.split < (int64_t(1) << 31), -1, "gemm: too many tiles");
  auto one = [&](const GemmDesc &g) {
    const int64_t gm = (g.M + ti.BM - 1) / ti.BM, gn = (g.N + ti.BN - 1) / ti.BN;
    if (g.ladder == 2 && akc && bkc) ti.launch_ladder_tail(g, gm, gn, s);
    else if (g.ladder && akc && bkc) ti.launch_ladder(g, gm, gn, s);
    else ti.launch[(akc ? 2 : 0) + (bkc ? 1 : 0)](g, gm, gn, s);
    CC_HIP_CHECK(hipGetLastError());
    if (g.split > 1) splitk_reduce(false, g.ws, g.split, g.M, g.N, g.C, g.ldc, g.alpha, g.beta, s);
  };
  if (d.ws && d.split == 1) {
    const TailCut tc = f64_cut(d, tile_id);
    if (tc.axis && tc.ws_elems <= d.ws_elems) {
      gemm_run_cut(d, tc, sizeof(double), sizeof(double), one);
      return;
    }
  }
  if (d.ws && d.split > 1 && d.ws_elems > 0) {
    GemmDesc g = d;
    g.split = gemm_split_refine(d.M, d.N, d.K, ti.BM, ti.BN, ti.BK,
                                tile_slots(tile_id, (akc ? 2 : 0) + (bkc ? 1 : 0)), d.split, d.ws_elems);
    one(g);
    return;
  }
  one(d);
}

}  // namespace ccmi
