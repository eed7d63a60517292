// Complex128 GEMM on FP64 MFMA:  C = alpha * sum_k A(m,k) B(n,k) + beta * C,
// interleaved (re, im) storage, real alpha and beta.
//
// Each complex product is four real products on v_mfma_f64_16x16x4_f64:
//   re += ar*br - ai*bi,  im += ar*bi + ai*br
// with separate real and imaginary accumulators (8 real flop per complex
// multiply-add, the algorithmic count of the complex residual).  Tiles are
// staged into planar real/imaginary LDS panels, double buffered; split-K and
// the XCD-aware tile order follow the real FP64 kernel.  Conjugated operands
// never reach this kernel: the contraction planner materialises them as
// conjugated views.
#include "common.hpp"

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

const ZTile kZTiles[] = {CC_ZTILE(64, 64, 16, 2, 2), CC_ZTILE(32, 32, 16, 2, 2), CC_ZTILE(128, 64, 16, 2, 2),
                         CC_ZTILE(64, 128, 16, 2, 2)};
constexpr int kNumZ = 4;

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
