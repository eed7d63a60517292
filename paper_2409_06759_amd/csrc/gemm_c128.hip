// Complex128 GEMM on FP64 MFMA:  C = alpha * sum_k A(m,k) B(n,k) + beta * C,
// interleaved (re, im) storage, real alpha and beta.
//
// Each complex product is four real products on v_mfma_f64_16x16x4_f64:
//   re += ar*br - ai*bi,  im += ar*bi + ai*br
// with separate real and imaginary accumulators (8 real flop per complex
// multiply-add, the algorithmic count of the complex residual).  Tiles are
// staged into planar real/imaginary LDS panels, double buffered; split-K and
// the XCD-aware tile order follow the real FP64 kernel.  The 64x128x16
// LDS-direct configuration loads K-contiguous operands straight into three
// interleaved (re, im) LDS stages.  Conjugated operands
// never reach this kernel: the contraction planner materialises them as
// conjugated views.
#include "common.hpp"

#include <algorithm>
#include <cmath>

namespace ccmi {
namespace {

typedef double d4 __attribute__((ext_vector_type(4)));

template <int BM, int BN, int BK, int WM, int WN, bool AKC, bool BKC>
struct ZCfg {
  static constexpr int NT = WM * WN * kWave;
  static constexpr int WTM = BM / WM, WTN = BN / WN;
  static constexpr int FM = WTM / 16, FN = WTN / 16;
  static constexpr int PAD = 2;
  static constexpr int A_ROWS = AKC ? BM : BK, A_LD = AKC ? BK + PAD : BM + PAD;
  static constexpr int B_ROWS = BKC ? BN : BK, B_LD = BKC ? BK + PAD : BN + PAD;
  static constexpr int A_ELEMS = A_ROWS * A_LD, B_ELEMS = B_ROWS * B_LD;
  static constexpr int LA = BM * BK / NT, LB = BN * BK / NT;
  static_assert(BM % (16 * WM) == 0 && BN % (16 * WN) == 0, "tile/wave mismatch");
  static_assert(BK % 16 == 0 && (BM * BK) % NT == 0 && (BN * BK) % NT == 0, "tile");
};

template <int BM, int BN, int BK, int WM, int WN, bool AKC, bool BKC>
__global__ __launch_bounds__(WM *WN *kWave) void gemm_c128_kernel(GemmDesc d, int64_t tilesM,
                                                                   int64_t tilesN) {
  using C = ZCfg<BM, BN, BK, WM, WN, AKC, BKC>;
  // per buffer: A re, A im, B re, B im
  constexpr int BUF = 2 * C::A_ELEMS + 2 * C::B_ELEMS;
  __shared__ double smem[2 * BUF];

  const int64_t tiles = tilesM * tilesN, total = tiles * d.split;
  const int64_t L0 = xcd_remap(blockIdx.x, total);
  const int64_t ks = L0 / tiles, L = L0 % tiles;
  const int64_t m0 = (L % tilesM) * BM, n0 = (L / tilesM) * BN;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm0 = (wave / WN) * C::WTM, wn0 = (wave % WN) * C::WTN;
  const int q = lane >> 4, r = lane & 15;

  const double2 *__restrict__ A = static_cast<const double2 *>(d.A);
  const double2 *__restrict__ B = static_cast<const double2 *>(d.B);
  const int64_t M = d.M, N = d.N;
  const int64_t kchunk = ((d.K + d.split - 1) / d.split + BK - 1) / BK * BK;
  const int64_t kb = ks * kchunk;
  const int64_t K = std::max<int64_t>(0, std::min<int64_t>(d.K - kb, kchunk));
  A += kb * d.sak;
  B += kb * d.sbk;

  double2 ra[C::LA], rb[C::LB];
  auto gload = [&](int64_t k0) {
#pragma unroll
    for (int i = 0; i < C::LA; ++i) {
      const int e = tid + i * C::NT;
      int mm, kk;
      if (AKC) { mm = e / BK; kk = e % BK; } else { kk = e / BM; mm = e % BM; }
      const int64_t gm = m0 + mm, gk = k0 + kk;
      ra[i] = (gm < M && gk < K) ? A[gm * d.sam + gk * d.sak] : make_double2(0.0, 0.0);
    }
#pragma unroll
    for (int i = 0; i < C::LB; ++i) {
      const int e = tid + i * C::NT;
      int nn, kk;
      if (BKC) { nn = e / BK; kk = e % BK; } else { kk = e / BN; nn = e % BN; }
      const int64_t gn = n0 + nn, gk = k0 + kk;
      rb[i] = (gn < N && gk < K) ? B[gn * d.sbn + gk * d.sbk] : make_double2(0.0, 0.0);
    }
  };
  auto sstore = [&](int buf) {
    double *ar = smem + buf * BUF, *ai = ar + C::A_ELEMS;
    double *br = ai + C::A_ELEMS, *bi = br + C::B_ELEMS;
#pragma unroll
    for (int i = 0; i < C::LA; ++i) {
      const int e = tid + i * C::NT;
      const int idx = AKC ? (e / BK) * C::A_LD + (e % BK) : (e / BM) * C::A_LD + (e % BM);
      ar[idx] = ra[i].x;
      ai[idx] = ra[i].y;
    }
#pragma unroll
    for (int i = 0; i < C::LB; ++i) {
      const int e = tid + i * C::NT;
      const int idx = BKC ? (e / BK) * C::B_LD + (e % BK) : (e / BN) * C::B_LD + (e % BN);
      br[idx] = rb[i].x;
      bi[idx] = rb[i].y;
    }
  };

  d4 acr[C::FM][C::FN], aci[C::FM][C::FN];
#pragma unroll
  for (int i = 0; i < C::FM; ++i)
#pragma unroll
    for (int j = 0; j < C::FN; ++j) {
      acr[i][j] = d4{0.0, 0.0, 0.0, 0.0};
      aci[i][j] = d4{0.0, 0.0, 0.0, 0.0};
    }

  const int64_t nk = (K + BK - 1) / BK;
  gload(0);
  sstore(0);
  __syncthreads();
  for (int64_t kt = 0; kt < nk; ++kt) {
    const int buf = kt & 1;
    if (kt + 1 < nk) gload((kt + 1) * BK);
    const double *ar = smem + buf * BUF, *ai = ar + C::A_ELEMS;
    const double *br = ai + C::A_ELEMS, *bi = br + C::B_ELEMS;
#pragma unroll
    for (int kc = 0; kc < BK; kc += 16) {
      double far_[C::FM][4], fai[C::FM][4], fbr[C::FN][4], fbi[C::FN][4];
#pragma unroll
      for (int i = 0; i < C::FM; ++i) {
        const int mm = wm0 + i * 16 + r;
#pragma unroll
        for (int s = 0; s < 4; ++s) {
          const int idx = AKC ? mm * C::A_LD + kc + 4 * q + s : (kc + 4 * q + s) * C::A_LD + mm;
          far_[i][s] = ar[idx];
          fai[i][s] = ai[idx];
        }
      }
#pragma unroll
      for (int j = 0; j < C::FN; ++j) {
        const int nn = wn0 + j * 16 + r;
#pragma unroll
        for (int s = 0; s < 4; ++s) {
          const int idx = BKC ? nn * C::B_LD + kc + 4 * q + s : (kc + 4 * q + s) * C::B_LD + nn;
          fbr[j][s] = br[idx];
          fbi[j][s] = bi[idx];
        }
      }
#pragma unroll
      for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int i = 0; i < C::FM; ++i)
#pragma unroll
          for (int j = 0; j < C::FN; ++j) {
            acr[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(far_[i][s], fbr[j][s], acr[i][j], 0, 0, 0);
            acr[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(-fai[i][s], fbi[j][s], acr[i][j], 0, 0, 0);
            aci[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(far_[i][s], fbi[j][s], aci[i][j], 0, 0, 0);
            aci[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(fai[i][s], fbr[j][s], aci[i][j], 0, 0, 0);
          }
    }
    if (kt + 1 < nk) sstore(buf ^ 1);
    __syncthreads();
  }

  // accumulator t of lane l is row (l >> 4) + 4t, column l & 15 (f64 MFMA layout)
  double2 *__restrict__ Cp = static_cast<double2 *>(d.C);
  double alpha = d.alpha, beta = d.beta;
  int64_t ldc = d.ldc;
  if (d.split > 1) {
    Cp = static_cast<double2 *>(d.ws) + ks * M * N;
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
          double2 *p = Cp + gm * ldc + gn;
          double2 v = make_double2(alpha * acr[i][j][t], alpha * aci[i][j][t]);
          if (beta != 0.0) {
            const double2 o = *p;
            v.x += beta * o.x;
            v.y += beta * o.y;
          }
          *p = v;
        }
      }
    }
}

// ---- 64x128x16 with LDS-direct loads ----------------------------------------
// Both operands K-contiguous, K a multiple of 16 (the complex ladder's
// layout).  Each lane's 16 bytes (one complex element) go straight into LDS
// with global_load_lds_dwordx4: three 48 KiB stages, two chunks of K in
// flight, no staging registers.  A 16-row block of a stage is four quarters
// of 64 slots; slot L of quarter s holds element (row L & 15, k = 4 (L >> 4)
// + s), the value lane L feeds the f64 MFMAs at step s (as in the staged
// kernel), so each quarter is read contiguously across the wave.  Rows past
// M or N load the last valid row instead: they only reach outputs that are
// never stored.  The products and their order are those of the staged
// 64x128 kernel, so results are bitwise the same.  Waits as in the real
// LDS-direct kernel: "vmcnt <= 6" after the next chunk's six loads, a
// barrier, and "lgkmcnt == 0" before it for the stage being overwritten.
namespace zdma {
constexpr int BM = 64, BN = 128, BK = 16, WM = 2, WN = 4, NT = WM * WN * kWave;
constexpr int FM = BM / WM / 16, FN = BN / WN / 16;      // 2 x 2 blocks of 16x16 per wave
constexpr int A_EL = BM * BK, B_EL = BN * BK, STAGE = A_EL + B_EL;  // complex elements
constexpr int NSTAGE = 3;
constexpr int LOADS = (4 * (BM / 16) + 4 * (BN / 16)) / (WM * WN);
static_assert(LOADS == 6, "the explicit waits count six loads per chunk");
}  // namespace zdma

__global__ __launch_bounds__(zdma::NT) void gemm_c128_dma_kernel(GemmDesc d, int64_t tilesM, int64_t tilesN) {
  using namespace zdma;
  __shared__ __attribute__((aligned(16))) double2 S[NSTAGE * STAGE];

  const int64_t tiles = tilesM * tilesN, total = tiles * d.split;
  const int64_t L0 = xcd_remap(blockIdx.x, total);
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

  // load j of this wave (j = 6 wave + u): A (block j >> 2, quarter j & 3) for
  // j < 16, else B (block (j - 16) >> 2, quarter j & 3); a block-quarter of A
  // sits at elements (blk * 4 + quarter) * 64 of the stage, of B at A_EL + ...
  const uint32_t lds0 = static_cast<uint32_t>(reinterpret_cast<uintptr_t>(S));
  const double2 *src[LOADS];
  uint32_t dst[LOADS];
  const double2 *Ag = static_cast<const double2 *>(d.A) + kb;
  const double2 *Bg = static_cast<const double2 *>(d.B) + kb;
  const int wv = __builtin_amdgcn_readfirstlane(wave);  // wave-uniform, so the choice below is too
#pragma unroll
  for (int u = 0; u < LOADS; ++u) {
    const int j = LOADS * wv + u;
    const bool isa = j < 4 * (BM / 16);
    const int jj = isa ? j : j - 4 * (BM / 16), blk = jj >> 2, qt = jj & 3;
    const int64_t lim = isa ? M : N, want = (isa ? m0 : n0) + blk * 16 + r;
    const int64_t row = want < lim ? want : lim - 1;
    src[u] = (isa ? Ag + row * d.sam : Bg + row * d.sbn) + 4 * q + qt;
    dst[u] = __builtin_amdgcn_readfirstlane(lds0 + 16u * uint32_t((isa ? 0 : A_EL) + (blk * 4 + qt) * 64));
  }
  auto issue = [&](int stage, int64_t k0) {
#pragma unroll
    for (int u = 0; u < LOADS; ++u) lds_load16(src[u] + k0, dst[u] + uint32_t(stage) * uint32_t(16 * STAGE));
  };

  d4 acr[FM][FN], aci[FM][FN];
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j) {
      acr[i][j] = d4{0.0, 0.0, 0.0, 0.0};
      aci[i][j] = d4{0.0, 0.0, 0.0, 0.0};
    }

  if (nk > 0) issue(0, 0);
  if (nk > 1) issue(1, BK);
  int cur = 0, nxt = 2;
  for (int64_t kt = 0; kt < nk; ++kt) {
    if (kt + 1 < nk) asm volatile("s_waitcnt vmcnt(6) lgkmcnt(0)\n\ts_barrier" ::: "memory");
    else asm volatile("s_waitcnt vmcnt(0) lgkmcnt(0)\n\ts_barrier" ::: "memory");
    if (kt + 2 < nk) issue(nxt, (kt + 2) * BK);
    const double2 *St = S + cur * STAGE;
    // steps 0-1 are read first and steps 2-3 behind the MFMAs of step 0, so
    // those reads overlap them (at most eight LDS reads in flight)
    double2 fa[FM][4], fb[FN][4];
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      if (s == 0 || s == 2) {
        // the fragments of steps s and s + 1
#pragma unroll
        for (int t = s; t < s + 2; ++t) {
#pragma unroll
          for (int i = 0; i < FM; ++i) fa[i][t] = St[(((wm0 >> 4) + i) * 4 + t) * 64 + lane];
#pragma unroll
          for (int j = 0; j < FN; ++j) fb[j][t] = St[A_EL + (((wn0 >> 4) + j) * 4 + t) * 64 + lane];
        }
      }
      if (s <= 1) __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j) {
          acr[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(fa[i][s].x, fb[j][s].x, acr[i][j], 0, 0, 0);
          acr[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(-fa[i][s].y, fb[j][s].y, acr[i][j], 0, 0, 0);
          aci[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(fa[i][s].x, fb[j][s].y, aci[i][j], 0, 0, 0);
          aci[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(fa[i][s].y, fb[j][s].x, aci[i][j], 0, 0, 0);
        }
      if (s == 0) __builtin_amdgcn_sched_barrier(0);
    }
    cur = cur == NSTAGE - 1 ? 0 : cur + 1;
    nxt = nxt == NSTAGE - 1 ? 0 : nxt + 1;
  }

  // epilogue (as the staged kernel): accumulator t of lane l is row (l >> 4) + 4t, column l & 15
  double2 *__restrict__ Cp = static_cast<double2 *>(d.C);
  double alpha = d.alpha, beta = d.beta;
  int64_t ldc = d.ldc;
  if (d.split > 1) {
    Cp = static_cast<double2 *>(d.ws) + ks * M * N;
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
          double2 *p = Cp + gm * ldc + gn;
          double2 v = make_double2(alpha * acr[i][j][t], alpha * aci[i][j][t]);
          if (beta != 0.0) {
            const double2 o = *p;
            v.x += beta * o.x;
            v.y += beta * o.y;
          }
          *p = v;
        }
      }
    }
}

bool c128_dma_ok(const GemmDesc &d) {
  return d.sak == 1 && d.sbk == 1 && d.K % zdma::BK == 0 && (reinterpret_cast<uintptr_t>(d.A) & 15) == 0 &&
         (reinterpret_cast<uintptr_t>(d.B) & 15) == 0;
}

struct ZTile {
  const char *name;
  int BM, BN, BK;
  void (*launch[4])(const GemmDesc &, int64_t, int64_t, hipStream_t);
};

template <int BM, int BN, int BK, int WM, int WN, bool AKC, bool BKC>
void launch_z(const GemmDesc &d, int64_t tm, int64_t tn, hipStream_t s) {
  hipLaunchKernelGGL((gemm_c128_kernel<BM, BN, BK, WM, WN, AKC, BKC>), dim3(tm * tn * d.split),
                     dim3(WM * WN * kWave), 0, s, d, tm, tn);
}

#define CC_ZTILE(BM, BN, BK, WM, WN)                                                              \
  ZTile {                                                                                         \
    #BM "x" #BN "x" #BK "_w" #WM "x" #WN, BM, BN, BK,                                             \
        {&launch_z<BM, BN, BK, WM, WN, false, false>, &launch_z<BM, BN, BK, WM, WN, false, true>, \
         &launch_z<BM, BN, BK, WM, WN, true, false>, &launch_z<BM, BN, BK, WM, WN, true, true>}   \
  }

void launch_z_dma(const GemmDesc &d, int64_t tm, int64_t tn, hipStream_t s) {
  if (c128_dma_ok(d))
    hipLaunchKernelGGL(gemm_c128_dma_kernel, dim3(tm * tn * d.split), dim3(zdma::NT), 0, s, d, tm, tn);
  else
    launch_z<64, 128, 16, 2, 2, true, true>(d, tm, tn, s);
}

const ZTile kZTiles[] = {CC_ZTILE(64, 64, 16, 2, 2), CC_ZTILE(32, 32, 16, 2, 2), CC_ZTILE(128, 64, 16, 2, 2),
                         CC_ZTILE(64, 128, 16, 2, 2),
                         // 64x128x16 with LDS-direct loads where the layout allows, else staged
                         ZTile{"64x128x16_w2x4_lds",
                               64,
                               128,
                               16,
                               {&launch_z<64, 128, 16, 2, 2, false, false>, &launch_z<64, 128, 16, 2, 2, false, true>,
                                &launch_z<64, 128, 16, 2, 2, true, false>, &launch_z_dma}}};
constexpr int kNumZ = sizeof(kZTiles) / sizeof(kZTiles[0]);

}  // namespace

int gemm_c128_num_tiles() { return kNumZ; }
const char *gemm_c128_tile_name(int id) { return (id >= 0 && id < kNumZ) ? kZTiles[id].name : "?"; }

void gemm_c128(const GemmDesc &d, hipStream_t s, int tile_id) {
  if (d.M <= 0 || d.N <= 0) return;
  const bool akc = (d.sak == 1), bkc = (d.sbk == 1);
  CC_REQUIRE(akc || d.sam == 1, -1, "gemm: A needs a unit stride in m or k");
  CC_REQUIRE(bkc || d.sbn == 1, -1, "gemm: B needs a unit stride in n or k");
  CC_REQUIRE(d.conj_a == 0 && d.conj_b == 0, -7, "gemm_c128: conjugated operands are planned as views");
  if (d.K <= 0) {
    PermDesc p{};
    p.rank = 2;
    p.out_dims[0] = d.M;
    p.out_dims[1] = d.N;
    p.out_strides[0] = d.ldc;
    p.out_strides[1] = 1;
    p.in_strides[0] = d.ldc;
    p.in_strides[1] = 1;
    p.alpha = d.beta;
    permute_c128(p, d.C, d.C, s);
    return;
  }
  if (tile_id < 0 || tile_id >= kNumZ) {
    // fewest rounds of resident workgroups, then the larger tile
    double best_cost = 1e300;
    for (int t = 0; t < kNumZ; ++t) {
      const double n = double((d.M + kZTiles[t].BM - 1) / kZTiles[t].BM) *
                       double((d.N + kZTiles[t].BN - 1) / kZTiles[t].BN);
      const double cost = std::ceil(n * d.split / 512.0) * (double(kZTiles[t].BM) * kZTiles[t].BN + 2048.0);
      if (cost < best_cost) {
        best_cost = cost;
        tile_id = t;
      }
    }
  }
  const ZTile &ti = kZTiles[tile_id];
  const int64_t tm = (d.M + ti.BM - 1) / ti.BM, tn = (d.N + ti.BN - 1) / ti.BN;
  CC_REQUIRE(d.split >= 1 && (d.split == 1 || d.ws != nullptr), -1, "gemm: split-K workspace");
  CC_REQUIRE(tm * tn * d.split < (int64_t(1) << 31), -1, "gemm: too many tiles");
  ti.launch[(akc ? 2 : 0) + (bkc ? 1 : 0)](d, tm, tn, s);
  CC_HIP_CHECK(hipGetLastError());
  if (d.split > 1) splitk_reduce(true, d.ws, d.split, d.M, d.N, d.C, d.ldc, d.alpha, d.beta, s);
}

}  // namespace ccmi
