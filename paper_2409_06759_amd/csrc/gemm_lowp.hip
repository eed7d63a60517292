// Reduced-precision GEMMs on FP64 tensors:
//   C[m][n] = alpha * sum_k A(m,k) B(n,k) + beta * C[m][n]   (C in FP64)
// * F32:    operands rounded to FP32, v_mfma_f32_16x16x4_f32, FP32 accumulate.
// * BF16X3: operands rounded to FP32 and split x = hi + lo with hi = bf16(x),
//           lo = bf16(x - hi); the product keeps hi*hi + hi*lo + lo*hi
//           (v_mfma_f32_16x16x32_bf16, FP32 accumulate), dropping lo*lo
//           (split-bfloat16 products: Henry, Tang & Heinecke, ARITH 2019).
// Two ways to get the operands in:
// * FP64 tensors, rounded/split while a tile is staged into LDS;
// * converted copies made once by convert_shadow (FP32, or a bf16 hi plane
//   followed by a bf16 lo plane, same element indexing as the FP64 tensor),
//   read with 16-byte vector loads and stored to LDS unchanged.  The LDS
//   contents, hence the results, are identical for both.
// Everything outside the contractions (permutations, assembly, norms,
// denominators, energy) stays FP64.  Tiling, double buffering, split-K, the
// tail cut and the XCD-aware tile order follow the FP64 kernel; the 128x128
// 8-wave configurations also come with two chunks in flight (a second
// register set), and the 256x128 configurations with LDS-direct loads into
// three stages for K-contiguous converted operands.
#include "common.hpp"
#include "kernels.hpp"

#include <atomic>
#include <cmath>
#include <mutex>
#include <type_traits>

namespace ccmi {
namespace {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));

// round-to-nearest-even FP32 -> BF16 bits (finite inputs)
__device__ __forceinline__ unsigned short bf16_bits(float x) {
  unsigned u = __float_as_uint(x);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return static_cast<unsigned short>(u >> 16);
}
__device__ __forceinline__ float bf16_to_float(unsigned short h) {
  return __uint_as_float(static_cast<unsigned>(h) << 16);
}

template <int MODE, int BM, int BN, int BK, int WM, int WN, bool AKC, bool BKC>
struct LCfg {
  static constexpr int NT = WM * WN * kWave;
  static constexpr int WTM = BM / WM, WTN = BN / WN;
  static constexpr int FM = WTM / 16, FN = WTN / 16;
  static constexpr int PAD = (MODE == PREC_F32) ? 4 : 8;  // elements
  static constexpr int A_ROWS = AKC ? BM : BK, A_LD = AKC ? BK + PAD : BM + PAD;
  static constexpr int B_ROWS = BKC ? BN : BK, B_LD = BKC ? BK + PAD : BN + PAD;
  static constexpr int A_ELEMS = A_ROWS * A_LD, B_ELEMS = B_ROWS * B_LD;
  static constexpr int LA = BM * BK / NT, LB = BN * BK / NT;
  static constexpr int KSTEP = (MODE == PREC_F32) ? 16 : 32;  // k consumed per fragment load
  static_assert(BM % (16 * WM) == 0 && BN % (16 * WN) == 0, "tile/wave mismatch");
  static_assert(BK % KSTEP == 0, "BK");
  static_assert((BM * BK) % NT == 0 && (BN * BK) % NT == 0, "load split");
};

template <int MODE, int BM, int BN, int BK, int WM, int WN, bool AKC, bool BKC, bool LPIN, int PF = 1>
__device__ __forceinline__ void gemm_lowp_body(const GemmDesc &d, int64_t tilesM, int64_t tilesN, int64_t L0) {
  using C = LCfg<MODE, BM, BN, BK, WM, WN, AKC, BKC>;
  // F32: one float array per operand and buffer.  BF16X3: hi and lo arrays
  // (16-bit) per operand and buffer, laid out as [hi | lo].
  constexpr int ESZ = (MODE == PREC_F32) ? 4 : 2;
  constexpr int NPART = (MODE == PREC_F32) ? 1 : 2;
  constexpr int A_BYTES = C::A_ELEMS * ESZ * NPART, B_BYTES = C::B_ELEMS * ESZ * NPART;
  __shared__ __attribute__((aligned(16))) unsigned char smem[2 * (A_BYTES + B_BYTES)];

  const int64_t tiles = tilesM * tilesN;
  const int64_t ks = L0 / tiles, L = L0 % tiles;
  const int64_t m0 = (L % tilesM) * BM, n0 = (L / tilesM) * BN;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm0 = (wave / WN) * C::WTM, wn0 = (wave % WN) * C::WTN;
  const int q = lane >> 4, r = lane & 15;

  const int64_t M = d.M, N = d.N;
  const int64_t kchunk = ((d.K + d.split - 1) / d.split + BK - 1) / BK * BK;
  const int64_t kb = ks * kchunk;
  const int64_t K = std::max<int64_t>(0, std::min<int64_t>(d.K - kb, kchunk));
  auto a_base = [&](int buf) { return smem + buf * A_BYTES; };
  auto b_base = [&](int buf) { return smem + 2 * A_BYTES + buf * B_BYTES; };

  // ---- path 1: FP64 operands, rounded/split while staging --------------------
  const double *__restrict__ A = static_cast<const double *>(d.A) + kb * d.sak;
  const double *__restrict__ B = static_cast<const double *>(d.B) + kb * d.sbk;
  constexpr int LA1 = LPIN ? 1 : C::LA, LB1 = LPIN ? 1 : C::LB;
  float ra[LA1], rb[LB1];
  // ---- path 2: converted operands, 16-byte vectors straight into LDS --------
  typedef typename std::conditional<MODE == PREC_F32, float, unsigned short>::type EL;
  constexpr int VEC = 16 / int(sizeof(EL));
  constexpr int AR = AKC ? BM : BK, AC = AKC ? BK : BM, BR = BKC ? BN : BK, BC = BKC ? BK : BN;
  constexpr int ANV = AR * AC / VEC, BNV = BR * BC / VEC;
  constexpr int AVT = LPIN ? (ANV + C::NT - 1) / C::NT : 1, BVT = LPIN ? (BNV + C::NT - 1) / C::NT : 1;
  uint4 va[AVT][NPART], vb[BVT][NPART];
  const EL *__restrict__ Al = static_cast<const EL *>(d.A) + kb * d.sak;
  const EL *__restrict__ Bl = static_cast<const EL *>(d.B) + kb * d.sbk;
  const bool vec_a = ((AKC ? d.sam : d.sak) % VEC == 0) && ((reinterpret_cast<uintptr_t>(Al) & 15) == 0) &&
                     (d.a_plane % VEC == 0);
  const bool vec_b = ((BKC ? d.sbn : d.sbk) % VEC == 0) && ((reinterpret_cast<uintptr_t>(Bl) & 15) == 0) &&
                     (d.b_plane % VEC == 0);

  // one operand's vector loads: rows along the strided dim, VEC columns along
  // the unit-stride dim; out-of-range elements read as zero
  auto vload = [&](const EL *base, int64_t plane, int64_t rstride, int64_t r_lim, int64_t c_lim, int64_t r0,
                   int64_t c0, bool vec_ok, int v, int ncolv, uint4 *out) {
    const int r = v / ncolv, c = (v % ncolv) * VEC;
    const int64_t gr = r0 + r, gc = c0 + c;
    for (int pl = 0; pl < NPART; ++pl) {
      const EL *src = base + pl * plane + gr * rstride + gc;
      if (vec_ok && gr < r_lim && gc + VEC <= c_lim) {
        out[pl] = *reinterpret_cast<const uint4 *>(src);
      } else {
        union {
          uint4 u;
          EL e[VEC];
        } tmp;
#pragma unroll
        for (int q = 0; q < VEC; ++q) tmp.e[q] = (gr < r_lim && gc + q < c_lim) ? src[q] : EL(0);
        out[pl] = tmp.u;
      }
    }
  };

  // converted operands: one register set of a chunk's vectors
  auto gload_into = [&](int64_t k0, uint4 (&xa)[AVT][NPART], uint4 (&xb)[BVT][NPART]) {
#pragma unroll
    for (int i = 0; i < AVT; ++i) {
      const int v = tid + i * C::NT;
      if (v < ANV) {
        if (AKC) vload(Al, d.a_plane, d.sam, M, K, m0, k0, vec_a, v, AC / VEC, xa[i]);
        else vload(Al, d.a_plane, d.sak, K, M, k0, m0, vec_a, v, AC / VEC, xa[i]);
      }
    }
#pragma unroll
    for (int i = 0; i < BVT; ++i) {
      const int v = tid + i * C::NT;
      if (v < BNV) {
        if (BKC) vload(Bl, d.b_plane, d.sbn, N, K, n0, k0, vec_b, v, BC / VEC, xb[i]);
        else vload(Bl, d.b_plane, d.sbk, K, N, k0, n0, vec_b, v, BC / VEC, xb[i]);
      }
    }
  };
  auto sstore_from = [&](int buf, const uint4 (&xa)[AVT][NPART], const uint4 (&xb)[BVT][NPART]) {
#pragma unroll
    for (int i = 0; i < AVT; ++i) {
      const int v = tid + i * C::NT;
      if (v < ANV) {
        const int r = v / (AC / VEC), c = (v % (AC / VEC)) * VEC;
        EL *dst = reinterpret_cast<EL *>(a_base(buf));
#pragma unroll
        for (int pl = 0; pl < NPART; ++pl)
          *reinterpret_cast<uint4 *>(dst + pl * C::A_ELEMS + r * C::A_LD + c) = xa[i][pl];
      }
    }
#pragma unroll
    for (int i = 0; i < BVT; ++i) {
      const int v = tid + i * C::NT;
      if (v < BNV) {
        const int r = v / (BC / VEC), c = (v % (BC / VEC)) * VEC;
        EL *dst = reinterpret_cast<EL *>(b_base(buf));
#pragma unroll
        for (int pl = 0; pl < NPART; ++pl)
          *reinterpret_cast<uint4 *>(dst + pl * C::B_ELEMS + r * C::B_LD + c) = xb[i][pl];
      }
    }
  };

  auto gload = [&](int64_t k0) {
    if constexpr (LPIN) {
      gload_into(k0, va, vb);
    } else {
#pragma unroll
      for (int i = 0; i < C::LA; ++i) {
        const int e = tid + i * C::NT;
        int mm, kk;
        if (AKC) { mm = e / BK; kk = e % BK; } else { kk = e / BM; mm = e % BM; }
        const int64_t gm = m0 + mm, gk = k0 + kk;
        ra[i] = (gm < M && gk < K) ? static_cast<float>(A[gm * d.sam + gk * d.sak]) : 0.0f;
      }
#pragma unroll
      for (int i = 0; i < C::LB; ++i) {
        const int e = tid + i * C::NT;
        int nn, kk;
        if (BKC) { nn = e / BK; kk = e % BK; } else { kk = e / BN; nn = e % BN; }
        const int64_t gn = n0 + nn, gk = k0 + kk;
        rb[i] = (gn < N && gk < K) ? static_cast<float>(B[gn * d.sbn + gk * d.sbk]) : 0.0f;
      }
    }
  };
  auto sstore = [&](int buf) {
    if constexpr (LPIN) {
      sstore_from(buf, va, vb);
    } else {
#pragma unroll
      for (int i = 0; i < C::LA; ++i) {
        const int e = tid + i * C::NT;
        const int idx = AKC ? (e / BK) * C::A_LD + (e % BK) : (e / BM) * C::A_LD + (e % BM);
        if (MODE == PREC_F32) {
          reinterpret_cast<float *>(a_base(buf))[idx] = ra[i];
        } else {
          const unsigned short h = bf16_bits(ra[i]);
          unsigned short *p = reinterpret_cast<unsigned short *>(a_base(buf));
          p[idx] = h;
          p[C::A_ELEMS + idx] = bf16_bits(ra[i] - bf16_to_float(h));
        }
      }
#pragma unroll
      for (int i = 0; i < C::LB; ++i) {
        const int e = tid + i * C::NT;
        const int idx = BKC ? (e / BK) * C::B_LD + (e % BK) : (e / BN) * C::B_LD + (e % BN);
        if (MODE == PREC_F32) {
          reinterpret_cast<float *>(b_base(buf))[idx] = rb[i];
        } else {
          const unsigned short h = bf16_bits(rb[i]);
          unsigned short *p = reinterpret_cast<unsigned short *>(b_base(buf));
          p[idx] = h;
          p[C::B_ELEMS + idx] = bf16_bits(rb[i] - bf16_to_float(h));
        }
      }
    }
  };

  f4 acc[C::FM][C::FN];
#pragma unroll
  for (int i = 0; i < C::FM; ++i)
#pragma unroll
    for (int j = 0; j < C::FN; ++j) acc[i][j] = f4{0.f, 0.f, 0.f, 0.f};

  const int64_t nk = (K + BK - 1) / BK;
  // MFMAs over the chunk staged in LDS buffer buf
  auto mma = [&](int buf) {
    if constexpr (MODE == PREC_F32) {
      const float *as = reinterpret_cast<const float *>(a_base(buf));
      const float *bs = reinterpret_cast<const float *>(b_base(buf));
#pragma unroll
      for (int kc = 0; kc < BK; kc += 16) {
        float fa[C::FM][4], fb[C::FN][4];
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
              acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(fa[i][s], fb[j][s], acc[i][j], 0, 0, 0);
      }
    } else {
      const unsigned short *ah = reinterpret_cast<const unsigned short *>(a_base(buf));
      const unsigned short *bh = reinterpret_cast<const unsigned short *>(b_base(buf));
      const unsigned short *al = ah + C::A_ELEMS, *bl = bh + C::B_ELEMS;
#pragma unroll
      for (int kc = 0; kc < BK; kc += 32) {
        bf8 fah[C::FM], fal[C::FM], fbh[C::FN], fbl[C::FN];
        // lane group q supplies logical k = kc + 8q .. kc + 8q + 7 for A and B alike
#pragma unroll
        for (int i = 0; i < C::FM; ++i) {
          const int mm = wm0 + i * 16 + r;
#pragma unroll
          for (int s = 0; s < 8; ++s) {
            const int idx = AKC ? mm * C::A_LD + kc + 8 * q + s : (kc + 8 * q + s) * C::A_LD + mm;
            fah[i][s] = __builtin_bit_cast(__bf16, ah[idx]);
            fal[i][s] = __builtin_bit_cast(__bf16, al[idx]);
          }
        }
#pragma unroll
        for (int j = 0; j < C::FN; ++j) {
          const int nn = wn0 + j * 16 + r;
#pragma unroll
          for (int s = 0; s < 8; ++s) {
            const int idx = BKC ? nn * C::B_LD + kc + 8 * q + s : (kc + 8 * q + s) * C::B_LD + nn;
            fbh[j][s] = __builtin_bit_cast(__bf16, bh[idx]);
            fbl[j][s] = __builtin_bit_cast(__bf16, bl[idx]);
          }
        }
#pragma unroll
        for (int i = 0; i < C::FM; ++i)
#pragma unroll
          for (int j = 0; j < C::FN; ++j) {
            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fal[i], fbh[j], acc[i][j], 0, 0, 0);
            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fah[i], fbl[j], acc[i][j], 0, 0, 0);
            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fah[i], fbh[j], acc[i][j], 0, 0, 0);
          }
      }
    }
  };

  if constexpr (LPIN && PF == 2) {
    // Two chunks in flight: while chunk kt is multiplied out of one LDS
    // buffer, chunk kt+1 sits in registers (stored to the other buffer after
    // the MFMAs) and chunk kt+2 is being loaded into the second register set.
    // Unrolled by two so that each register set is named statically.
    uint4 wa[AVT][NPART], wb[BVT][NPART];
    gload_into(0, va, vb);
    if (nk > 1) gload_into(BK, wa, wb);
    sstore_from(0, va, vb);
    __syncthreads();
    for (int64_t kt = 0; kt < nk; kt += 2) {
      if (kt + 2 < nk) gload_into((kt + 2) * BK, va, vb);
      mma(0);
      if (kt + 1 < nk) sstore_from(1, wa, wb);
      __syncthreads();
      if (kt + 1 >= nk) break;
      if (kt + 3 < nk) gload_into((kt + 3) * BK, wa, wb);
      mma(1);
      if (kt + 2 < nk) sstore_from(0, va, vb);
      __syncthreads();
    }
  } else {
    gload(0);
    sstore(0);
    __syncthreads();
    for (int64_t kt = 0; kt < nk; ++kt) {
      const int buf = kt & 1;
      if (kt + 1 < nk) gload((kt + 1) * BK);
      mma(buf);
      if (kt + 1 < nk) sstore(buf ^ 1);
      __syncthreads();
    }
  }

  // epilogue: accumulator t of lane l is C[4 (l >> 4) + t][l & 15] of its block
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
  for (int i = 0; i < C::FM; ++i)
#pragma unroll
    for (int j = 0; j < C::FN; ++j) {
      const int64_t gn = n0 + wn0 + j * 16 + r;
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int64_t gm = m0 + wm0 + i * 16 + 4 * q + t;
        if (gm < M && gn < N) {
          double *p = Cp + gm * ldc + gn;
          const double v = alpha * static_cast<double>(acc[i][j][t]);
          *p = (beta == 0.0) ? v : v + beta * *p;
        }
      }
    }
}

template <int MODE, int BM, int BN, int BK, int WM, int WN, bool AKC, bool BKC, int TAG, bool LPIN, int PF>
__global__ __launch_bounds__(WM *WN *kWave) void gemm_lowp_kernel(GemmDesc d, int64_t tilesM,
                                                                   int64_t tilesN) {
  gemm_lowp_body<MODE, BM, BN, BK, WM, WN, AKC, BKC, LPIN, PF>(d, tilesM, tilesN,
                                                           xcd_remap(blockIdx.x, tilesM * tilesN * d.split));
}

// ---- split bf16 with LDS-direct loads --------------------------------------
// 256x128 tiles, K a multiple of 32, both operands K-contiguous converted
// copies (bf16 hi plane + lo plane) with 16-byte aligned rows.  Rows past M
// or N load the last valid row instead: they only reach outputs that are
// never stored.
// global_load_lds_dwordx4 writes each lane's 16 bytes straight into LDS, so
// no registers stage the operands, and three LDS stages keep two chunks of K
// in flight while the third is multiplied.  A 16-row block of a stage is 64
// slots of 16 bytes: slot s holds row (s & 15), k-group (s >> 4), which is the
// MFMA operand layout of lane s, so a fragment is one contiguous 1 KiB
// ds_read_b128 per wave.  Products, their order and the epilogue are those of
// the staged kernel of the same tile, so results are bitwise the same.
//
// The loads are issued from inline assembly, so the compiler neither knows
// of them nor inserts waits for them; the waits are explicit.  Vector memory
// operations of a wave complete in issue order, so "vmcnt <= 6" after the
// six loads of chunk kt+1 means chunk kt has landed (more operations issued
// in between only make that wait longer), and a barrier behind it makes the
// chunk visible to every wave.  The same barrier, behind "lgkmcnt == 0",
// guarantees that every wave has finished reading the stage the next loads
// overwrite.  Nothing else in the kernel uses M0.
namespace dma {
constexpr int BM = 256, BN = 128, BK = 32, WM = 4, WN = 2, NT = WM * WN * kWave;
constexpr int FM = BM / WM / 16, FN = BN / WN / 16;
constexpr int A_EL = BM * BK, B_EL = BN * BK;  // bf16 elements per plane and stage
constexpr int STAGE = 2 * A_EL + 2 * B_EL;     // [A hi | A lo | B hi | B lo]
constexpr int NSTAGE = 3;
constexpr int LOADS = (2 * (BM / 16) + 2 * (BN / 16)) / (WM * WN);  // per wave and chunk
static_assert(LOADS == 6, "the explicit waits count six loads per chunk");
}  // namespace dma

__device__ __forceinline__ void gemm_b3_dma_body(const GemmDesc &d, int64_t tilesM, int64_t tilesN, int64_t L0) {
  using namespace dma;
  __shared__ __attribute__((aligned(16))) unsigned short S[NSTAGE * STAGE];

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

  // this wave's loads: A blocks 2w and 2w+1, B block w, hi and lo planes of
  // each; LDS addresses are byte offsets in the shared aperture (its low 32
  // bits), made wave-uniform for M0
  const uint32_t lds0 = static_cast<uint32_t>(reinterpret_cast<uintptr_t>(S));
  const unsigned short *src[LOADS];
  uint32_t dst[LOADS];
  // lp_in == 2: operands in 16-row x 32-k blocks of 1 KiB (convert_blocked),
  // a chunk of a 16-row block one contiguous wave load; 16 elements of a
  // block per element of k
  const int64_t kx = d.lp_in == 2 ? 16 : 1;
  const unsigned short *Ag = static_cast<const unsigned short *>(d.A) + kb * kx;
  const unsigned short *Bg = static_cast<const unsigned short *>(d.B) + kb * kx;
  auto row_src = [&](const unsigned short *g, int64_t r0, int64_t lim, int64_t stride) {
    return kx == 16 ? g + std::min<int64_t>(r0 >> 4, (lim - 1) >> 4) * (d.K * 16) + lane * 8
                    : g + std::min<int64_t>(r0 + r, lim - 1) * stride + q * 8;
  };
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int blk = 2 * wave + (u >> 1), pl = u & 1;
    src[u] = row_src(Ag + pl * d.a_plane, m0 + blk * 16, M, d.sam);
    dst[u] = __builtin_amdgcn_readfirstlane(lds0 + 2u * uint32_t(pl * A_EL + blk * 512));
  }
#pragma unroll
  for (int u = 0; u < 2; ++u) {
    src[4 + u] = row_src(Bg + u * d.b_plane, n0 + wave * 16, N, d.sbn);
    dst[4 + u] = __builtin_amdgcn_readfirstlane(lds0 + 2u * uint32_t(2 * A_EL + u * B_EL + wave * 512));
  }
  auto issue = [&](int stage, int64_t k0) {
#pragma unroll
    for (int u = 0; u < LOADS; ++u) lds_load16(src[u] + k0 * kx, dst[u] + uint32_t(stage) * uint32_t(2 * STAGE));
  };

  f4 acc[FM][FN];
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j) acc[i][j] = f4{0.f, 0.f, 0.f, 0.f};

  if (nk > 0) issue(0, 0);
  if (nk > 1) issue(1, BK);
  int cur = 0, nxt = 2;
  for (int64_t kt = 0; kt < nk; ++kt) {
    if (kt + 1 < nk) asm volatile("s_waitcnt vmcnt(6) lgkmcnt(0)\n\ts_barrier" ::: "memory");
    else asm volatile("s_waitcnt vmcnt(0) lgkmcnt(0)\n\ts_barrier" ::: "memory");
    if (kt + 2 < nk) issue(nxt, (kt + 2) * BK);
    const unsigned short *St = S + cur * STAGE;
    bf8 fah[FM], fal[FM], fbh[FN], fbl[FN];
#pragma unroll
    for (int i = 0; i < FM; ++i) {
      const int blk = (wm0 >> 4) + i;
      fah[i] = *reinterpret_cast<const bf8 *>(St + blk * 512 + lane * 8);
      fal[i] = *reinterpret_cast<const bf8 *>(St + A_EL + blk * 512 + lane * 8);
    }
#pragma unroll
    for (int j = 0; j < FN; ++j) {
      const int blk = (wn0 >> 4) + j;
      fbh[j] = *reinterpret_cast<const bf8 *>(St + 2 * A_EL + blk * 512 + lane * 8);
      fbl[j] = *reinterpret_cast<const bf8 *>(St + 2 * A_EL + B_EL + blk * 512 + lane * 8);
    }
    // the products at raised wave priority, so that the SIMD's other wave
    // issues its loads and fragment reads around them rather than between
    __builtin_amdgcn_s_setprio(1);
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
      for (int j = 0; j < FN; ++j) {
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fal[i], fbh[j], acc[i][j], 0, 0, 0);
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fah[i], fbl[j], acc[i][j], 0, 0, 0);
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fah[i], fbh[j], acc[i][j], 0, 0, 0);
      }
    __builtin_amdgcn_s_setprio(0);
    cur = cur == NSTAGE - 1 ? 0 : cur + 1;
    nxt = nxt == NSTAGE - 1 ? 0 : nxt + 1;
  }

  // epilogue (as the staged kernel): accumulator t of lane l is C[4 (l >> 4) + t][l & 15]
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
        const int64_t gm = m0 + wm0 + i * 16 + 4 * q + t;
        if (gm < M && gn < N) {
          double *p = Cp + gm * ldc + gn;
          const double v = alpha * static_cast<double>(acc[i][j][t]);
          *p = (beta == 0.0) ? v : v + beta * *p;
        }
      }
    }
}

// The same tile with the fragments of the next chunk read from LDS into a
// second register set while the current chunk's MFMAs run, so that the
// waves do not all read their fragments at once behind each barrier.  A
// stage is free for new loads once every wave holds its fragments, so the
// loads of chunk kt+3 go to the stage of chunk kt right after the barrier
// that ends its reads; chunks still land two iterations ahead of their
// reads.  The products and their order are those of gemm_b3_dma_body.
template <bool HAVE_NEXT>
__device__ __forceinline__ void b3_read(const unsigned short *St, int wm0, int wn0, int lane, bf8 (&ah)[dma::FM],
                                        bf8 (&al)[dma::FM], bf8 (&bh)[dma::FN], bf8 (&bl)[dma::FN]) {
  using namespace dma;
#pragma unroll
  for (int i = 0; i < FM; ++i) {
    const int blk = (wm0 >> 4) + i;
    ah[i] = *reinterpret_cast<const bf8 *>(St + blk * 512 + lane * 8);
    al[i] = *reinterpret_cast<const bf8 *>(St + A_EL + blk * 512 + lane * 8);
  }
#pragma unroll
  for (int j = 0; j < FN; ++j) {
    const int blk = (wn0 >> 4) + j;
    bh[j] = *reinterpret_cast<const bf8 *>(St + 2 * A_EL + blk * 512 + lane * 8);
    bl[j] = *reinterpret_cast<const bf8 *>(St + 2 * A_EL + B_EL + blk * 512 + lane * 8);
  }
}

// the three products of output block (i, j), in the staged kernel's order
__device__ __forceinline__ void b3_block(f4 &acc, const bf8 &ah, const bf8 &al, const bf8 &bh, const bf8 &bl) {
  acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh, acc, 0, 0, 0);
  acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl, acc, 0, 0, 0);
  acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh, acc, 0, 0, 0);
}

__device__ __forceinline__ void gemm_b3_dmap_body(const GemmDesc &d, int64_t tilesM, int64_t tilesN, int64_t L0) {
  using namespace dma;
  __shared__ __attribute__((aligned(16))) unsigned short S[NSTAGE * STAGE];

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

  const uint32_t lds0 = static_cast<uint32_t>(reinterpret_cast<uintptr_t>(S));
  const unsigned short *src[LOADS];
  uint32_t dst[LOADS];
  // lp_in == 2: operands in 16-row x 32-k blocks of 1 KiB (convert_blocked),
  // a chunk of a 16-row block one contiguous wave load; 16 elements of a
  // block per element of k
  const int64_t kx = d.lp_in == 2 ? 16 : 1;
  const unsigned short *Ag = static_cast<const unsigned short *>(d.A) + kb * kx;
  const unsigned short *Bg = static_cast<const unsigned short *>(d.B) + kb * kx;
  auto row_src = [&](const unsigned short *g, int64_t r0, int64_t lim, int64_t stride) {
    return kx == 16 ? g + std::min<int64_t>(r0 >> 4, (lim - 1) >> 4) * (d.K * 16) + lane * 8
                    : g + std::min<int64_t>(r0 + r, lim - 1) * stride + q * 8;
  };
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int blk = 2 * wave + (u >> 1), pl = u & 1;
    src[u] = row_src(Ag + pl * d.a_plane, m0 + blk * 16, M, d.sam);
    dst[u] = __builtin_amdgcn_readfirstlane(lds0 + 2u * uint32_t(pl * A_EL + blk * 512));
  }
#pragma unroll
  for (int u = 0; u < 2; ++u) {
    src[4 + u] = row_src(Bg + u * d.b_plane, n0 + wave * 16, N, d.sbn);
    dst[4 + u] = __builtin_amdgcn_readfirstlane(lds0 + 2u * uint32_t(2 * A_EL + u * B_EL + wave * 512));
  }
  auto issue = [&](int stage, int64_t k0) {
#pragma unroll
    for (int u = 0; u < LOADS; ++u) lds_load16(src[u] + k0 * kx, dst[u] + uint32_t(stage) * uint32_t(2 * STAGE));
  };

  f4 acc[FM][FN];
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j) acc[i][j] = f4{0.f, 0.f, 0.f, 0.f};

  bf8 ah0[FM], al0[FM], bh0[FN], bl0[FN], ah1[FM], al1[FM], bh1[FN], bl1[FN];
  if (nk > 0) {
    issue(0, 0);
    if (nk > 1) issue(1, BK);
    if (nk > 2) issue(2, 2 * BK);
    // chunk 0 landed: the loads of chunks 1 and 2 may still be in flight
    if (nk > 2) asm volatile("s_waitcnt vmcnt(12)\n\ts_barrier" ::: "memory");
    else if (nk > 1) asm volatile("s_waitcnt vmcnt(6)\n\ts_barrier" ::: "memory");
    else asm volatile("s_waitcnt vmcnt(0)\n\ts_barrier" ::: "memory");
    b3_read<true>(S, wm0, wn0, lane, ah0, al0, bh0, bl0);
  }
  // one step: wait for chunk kt+1 to land and for this wave's reads of chunk
  // kt; the barrier then frees chunk kt's stage for the loads of chunk kt+3
  auto step = [&](int64_t kt, bf8 (&ah)[FM], bf8 (&al)[FM], bf8 (&bh)[FN], bf8 (&bl)[FN], bf8 (&nah)[FM],
                  bf8 (&nal)[FM], bf8 (&nbh)[FN], bf8 (&nbl)[FN]) {
    if (kt + 2 < nk) asm volatile("s_waitcnt vmcnt(6) lgkmcnt(0)\n\ts_barrier" ::: "memory");
    else if (kt + 1 < nk) asm volatile("s_waitcnt vmcnt(0) lgkmcnt(0)\n\ts_barrier" ::: "memory");
    else asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
    if (kt + 3 < nk) issue(int(kt % NSTAGE), (kt + 3) * BK);
    // the first block's products wait for this chunk's fragments; the next
    // chunk's reads go out behind them, so the compiler, which cannot count
    // sixteen reads in flight, does not make the remaining products wait
    // for those reads too
    b3_block(acc[0][0], ah[0], al[0], bh[0], bl[0]);
    __builtin_amdgcn_sched_barrier(0);
    if (kt + 1 < nk) b3_read<true>(S + int((kt + 1) % NSTAGE) * STAGE, wm0, wn0, lane, nah, nal, nbh, nbl);
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
      for (int j = 0; j < FN; ++j)
        if (i + j > 0) b3_block(acc[i][j], ah[i], al[i], bh[j], bl[j]);
  };
  for (int64_t kt = 0; kt < nk; kt += 2) {
    step(kt, ah0, al0, bh0, bl0, ah1, al1, bh1, bl1);
    if (kt + 1 < nk) step(kt + 1, ah1, al1, bh1, bl1, ah0, al0, bh0, bl0);
  }

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
        const int64_t gm = m0 + wm0 + i * 16 + 4 * q + t;
        if (gm < M && gn < N) {
          double *p = Cp + gm * ldc + gn;
          const double v = alpha * static_cast<double>(acc[i][j][t]);
          *p = (beta == 0.0) ? v : v + beta * *p;
        }
      }
    }
}

template <int TAG>
__global__ __launch_bounds__(dma::NT) void gemm_b3_dma_kernel(GemmDesc d, int64_t tilesM, int64_t tilesN) {
  gemm_b3_dma_body(d, tilesM, tilesN, xcd_remap(blockIdx.x, tilesM * tilesN * d.split));
}

template <int TAG>
__global__ __launch_bounds__(dma::NT) void gemm_b3_dmap_kernel(GemmDesc d, int64_t tilesM, int64_t tilesN) {
  gemm_b3_dmap_body(d, tilesM, tilesN, xcd_remap(blockIdx.x, tilesM * tilesN * d.split));
}

// ---- split bf16, 256x256 tiles with LDS-direct loads -----------------------
// Eight waves of 128x64 outputs: each fragment read from LDS feeds twice the
// products it feeds in a 64x64 wave tile along one axis, so LDS reads per
// product fall by a quarter, and the operand bytes a tile fetches per product
// fall by a third.  A 32-deep stage is 64 KiB, so two stages fit: chunk kt+1
// loads while chunk kt is multiplied.  Slot layout, the products of a block
// and their order, and the epilogue are those of the 256x128 kernel: results
// are bitwise the same.
namespace dmw {
constexpr int BM = 256, BN = 256, BK = 32, WM = 2, WN = 4, NT = WM * WN * kWave;
constexpr int FM = BM / WM / 16, FN = BN / WN / 16;
constexpr int A_EL = BM * BK, B_EL = BN * BK;
constexpr int STAGE = 2 * A_EL + 2 * B_EL;  // [A hi | A lo | B hi | B lo]
constexpr int NSTAGE = 2;
constexpr int LOADS = (2 * (BM / 16) + 2 * (BN / 16)) / (WM * WN);  // per wave and chunk
static_assert(LOADS == 8 && FM == 8 && FN == 4, "wave tiling");
}  // namespace dmw

__device__ __forceinline__ void gemm_b3_dmw_body(const GemmDesc &d, int64_t tilesM, int64_t tilesN, int64_t L0) {
  using namespace dmw;
  __shared__ __attribute__((aligned(16))) unsigned short S[NSTAGE * STAGE];

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

  // this wave's loads: blocks 2w and 2w+1 of A and of B, hi and lo planes
  const uint32_t lds0 = static_cast<uint32_t>(reinterpret_cast<uintptr_t>(S));
  const unsigned short *src[LOADS];
  uint32_t dst[LOADS];
  // lp_in == 2: operands in 16-row x 32-k blocks of 1 KiB (convert_blocked),
  // a chunk of a 16-row block one contiguous wave load; 16 elements of a
  // block per element of k
  const int64_t kx = d.lp_in == 2 ? 16 : 1;
  const unsigned short *Ag = static_cast<const unsigned short *>(d.A) + kb * kx;
  const unsigned short *Bg = static_cast<const unsigned short *>(d.B) + kb * kx;
  auto row_src = [&](const unsigned short *g, int64_t r0, int64_t lim, int64_t stride) {
    return kx == 16 ? g + std::min<int64_t>(r0 >> 4, (lim - 1) >> 4) * (d.K * 16) + lane * 8
                    : g + std::min<int64_t>(r0 + r, lim - 1) * stride + q * 8;
  };
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int blk = 2 * wave + (u >> 1), pl = u & 1;
    src[u] = row_src(Ag + pl * d.a_plane, m0 + blk * 16, M, d.sam);
    dst[u] = __builtin_amdgcn_readfirstlane(lds0 + 2u * uint32_t(pl * A_EL + blk * 512));
    src[4 + u] = row_src(Bg + pl * d.b_plane, n0 + blk * 16, N, d.sbn);
    dst[4 + u] = __builtin_amdgcn_readfirstlane(lds0 + 2u * uint32_t(2 * A_EL + pl * B_EL + blk * 512));
  }
  auto issue = [&](int stage, int64_t k0) {
#pragma unroll
    for (int u = 0; u < LOADS; ++u) lds_load16(src[u] + k0 * kx, dst[u] + uint32_t(stage) * uint32_t(2 * STAGE));
  };

  f4 acc[FM][FN];
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j) acc[i][j] = f4{0.f, 0.f, 0.f, 0.f};

  if (nk > 0) issue(0, 0);
  for (int64_t kt = 0; kt < nk; ++kt) {
    // chunk kt has landed (the only loads in flight) and this wave has read
    // chunk kt-1; after the barrier every wave has, so its stage takes kt+1
    asm volatile("s_waitcnt vmcnt(0) lgkmcnt(0)\n\ts_barrier" ::: "memory");
    if (kt + 1 < nk) issue(int((kt + 1) & 1), (kt + 1) * BK);
    const unsigned short *St = S + int(kt & 1) * STAGE;
    bf8 bh[FN], bl[FN];
#pragma unroll
    for (int j = 0; j < FN; ++j) {
      const int blk = (wn0 >> 4) + j;
      bh[j] = *reinterpret_cast<const bf8 *>(St + 2 * A_EL + blk * 512 + lane * 8);
      bl[j] = *reinterpret_cast<const bf8 *>(St + 2 * A_EL + B_EL + blk * 512 + lane * 8);
    }
#pragma unroll
    for (int i = 0; i < FM; ++i) {
      const int blk = (wm0 >> 4) + i;
      const bf8 ah = *reinterpret_cast<const bf8 *>(St + blk * 512 + lane * 8);
      const bf8 al = *reinterpret_cast<const bf8 *>(St + A_EL + blk * 512 + lane * 8);
#pragma unroll
      for (int j = 0; j < FN; ++j) b3_block(acc[i][j], ah, al, bh[j], bl[j]);
    }
  }

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
        const int64_t gm = m0 + wm0 + i * 16 + 4 * q + t;
        if (gm < M && gn < N) {
          double *p = Cp + gm * ldc + gn;
          const double v = alpha * static_cast<double>(acc[i][j][t]);
          *p = (beta == 0.0) ? v : v + beta * *p;
        }
      }
    }
}

template <int TAG>
__global__ __launch_bounds__(dmw::NT) void gemm_b3_dmw_kernel(GemmDesc d, int64_t tilesM, int64_t tilesN) {
  gemm_b3_dmw_body(d, tilesM, tilesN, xcd_remap(blockIdx.x, tilesM * tilesN * d.split));
}

// FP32 variant of the LDS-direct kernel (same tile, stages and waits): the
// f32 MFMA takes one k per lane and step, lane group q feeding k = 4q + s at
// step s of each 16-wide k half, so a 16-row block of a k half is 64 slots
// of 16 bytes, slot L = row (L & 15), k = 4 (L >> 4) .. +3.  A chunk of 32 k
// is two such halves: 16 + 16 A loads and 8 + 8 B loads, six per wave.
__device__ __forceinline__ void gemm_f32_dma_body(const GemmDesc &d, int64_t tilesM, int64_t tilesN, int64_t L0) {
  using namespace dma;
  constexpr int FA_EL = BM * BK, FB_EL = BN * BK, FSTAGE = FA_EL + FB_EL;  // floats: [A | B]
  static_assert(FSTAGE * 4 == STAGE * 2, "same stage size as the split-bf16 kernel");
  __shared__ __attribute__((aligned(16))) float S[NSTAGE * FSTAGE];

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

  // loads: (block, k half) pairs; A: blocks 2w, 2w+1 x halves 0, 1; B: block w x halves 0, 1.
  // A block b, half h sits at floats (h * (BM / 16) + b) * 256 of the stage.
  const uint32_t lds0 = static_cast<uint32_t>(reinterpret_cast<uintptr_t>(S));
  const float *src[LOADS];
  uint32_t dst[LOADS];
  const float *Ag = static_cast<const float *>(d.A) + kb;
  const float *Bg = static_cast<const float *>(d.B) + kb;
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int blk = 2 * wave + (u >> 1), h = u & 1;
    src[u] = Ag + std::min<int64_t>(m0 + blk * 16 + r, M - 1) * d.sam + 16 * h + 4 * q;
    dst[u] = __builtin_amdgcn_readfirstlane(lds0 + 4u * uint32_t((h * (BM / 16) + blk) * 256));
  }
#pragma unroll
  for (int u = 0; u < 2; ++u) {
    src[4 + u] = Bg + std::min<int64_t>(n0 + wave * 16 + r, N - 1) * d.sbn + 16 * u + 4 * q;
    dst[4 + u] = __builtin_amdgcn_readfirstlane(lds0 + 4u * uint32_t(FA_EL + (u * (BN / 16) + wave) * 256));
  }
  auto issue = [&](int stage, int64_t k0) {
#pragma unroll
    for (int u = 0; u < LOADS; ++u) lds_load16(src[u] + k0, dst[u] + uint32_t(stage) * uint32_t(4 * FSTAGE));
  };

  f4 acc[FM][FN];
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j) acc[i][j] = f4{0.f, 0.f, 0.f, 0.f};

  if (nk > 0) issue(0, 0);
  if (nk > 1) issue(1, BK);
  int cur = 0, nxt = 2;
  for (int64_t kt = 0; kt < nk; ++kt) {
    if (kt + 1 < nk) asm volatile("s_waitcnt vmcnt(6) lgkmcnt(0)\n\ts_barrier" ::: "memory");
    else asm volatile("s_waitcnt vmcnt(0) lgkmcnt(0)\n\ts_barrier" ::: "memory");
    if (kt + 2 < nk) issue(nxt, (kt + 2) * BK);
    const float *St = S + cur * FSTAGE;
    // the second k half is read behind the first half's first MFMA step
    f4 fa[2][FM], fb[2][FN];
    auto read_half = [&](int h) {
#pragma unroll
      for (int i = 0; i < FM; ++i)
        fa[h][i] = *reinterpret_cast<const f4 *>(St + (h * (BM / 16) + (wm0 >> 4) + i) * 256 + lane * 4);
#pragma unroll
      for (int j = 0; j < FN; ++j)
        fb[h][j] = *reinterpret_cast<const f4 *>(St + FA_EL + (h * (BN / 16) + (wn0 >> 4) + j) * 256 + lane * 4);
    };
    auto mfma_step = [&](int h, int s) {
#pragma unroll
      for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(fa[h][i][s], fb[h][j][s], acc[i][j], 0, 0, 0);
    };
    read_half(0);
    __builtin_amdgcn_sched_barrier(0);
    mfma_step(0, 0);
    __builtin_amdgcn_sched_barrier(0);
    read_half(1);
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int s = 1; s < 4; ++s) mfma_step(0, s);
#pragma unroll
    for (int s = 0; s < 4; ++s) mfma_step(1, s);
    cur = cur == NSTAGE - 1 ? 0 : cur + 1;
    nxt = nxt == NSTAGE - 1 ? 0 : nxt + 1;
  }

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
        const int64_t gm = m0 + wm0 + i * 16 + 4 * q + t;
        if (gm < M && gn < N) {
          double *p = Cp + gm * ldc + gn;
          const double v = alpha * static_cast<double>(acc[i][j][t]);
          *p = (beta == 0.0) ? v : v + beta * *p;
        }
      }
    }
}

template <int TAG>
__global__ __launch_bounds__(dma::NT) void gemm_f32_dma_kernel(GemmDesc d, int64_t tilesM, int64_t tilesN) {
  gemm_f32_dma_body(d, tilesM, tilesN, xcd_remap(blockIdx.x, tilesM * tilesN * d.split));
}

bool f32_dma_ok(const GemmDesc &d) {
  return d.lp_in && d.sak == 1 && d.sbk == 1 && d.K % dma::BK == 0 &&
         d.sam % 4 == 0 && d.sbn % 4 == 0 && (reinterpret_cast<uintptr_t>(d.A) & 15) == 0 &&
         (reinterpret_cast<uintptr_t>(d.B) & 15) == 0;
}

// the shapes and layouts the LDS-direct kernel handles
bool b3_dma_ok(const GemmDesc &d) {
  return d.lp_in && d.sak == 1 && d.sbk == 1 && d.K % dma::BK == 0 &&
         d.sam % 8 == 0 && d.sbn % 8 == 0 && d.a_plane % 8 == 0 && d.b_plane % 8 == 0 &&
         (reinterpret_cast<uintptr_t>(d.A) & 15) == 0 && (reinterpret_cast<uintptr_t>(d.B) & 15) == 0;
}

// Grouped launch over many systems: system b owns logical tiles
// [off[b], off[b+1]).  FP64 operands converted while staging, or (LPIN)
// operand copies converted beforehand.
template <int MODE, int BM, int BN, int BK, int WM, int WN, bool AKC, bool BKC, bool LPIN>
__global__ __launch_bounds__(WM *WN *kWave) void gemm_lowp_grouped(const GemmGroupEntry *__restrict__ e,
                                                                    const int64_t *__restrict__ off, int n) {
  const int b = group_find(off, n, blockIdx.x);
  const GemmGroupEntry &g = e[b];
  gemm_lowp_body<MODE, BM, BN, BK, WM, WN, AKC, BKC, LPIN>(g.d, g.tilesM, g.tilesN,
                                                           int64_t(blockIdx.x) - off[b]);
}

template <int MODE, int BM, int BN, int BK, int WM, int WN, bool AKC, bool BKC, bool LPIN = false>
void launch_lg(const GemmGroupEntry *e, const int64_t *off, int n, int64_t blocks, hipStream_t s) {
  hipLaunchKernelGGL((gemm_lowp_grouped<MODE, BM, BN, BK, WM, WN, AKC, BKC, LPIN>), dim3(blocks),
                     dim3(WM * WN * kWave), 0, s, e, off, n);
}

// PF: chunks of K in flight (1 or 2); only the converted-operand variant has
// a deeper pipeline, the staging variant is shared by both.
template <int MODE, int BM, int BN, int BK, int WM, int WN, bool AKC, bool BKC, int PF, int TAG = 0>
void launch_l(const GemmDesc &d, int64_t tm, int64_t tn, hipStream_t s) {
  CC_REQUIRE(d.lp_in != 2, -1, "gemm: blocked operand copies need an LDS-direct configuration and shape");
  if (d.lp_in)
    hipLaunchKernelGGL((gemm_lowp_kernel<MODE, BM, BN, BK, WM, WN, AKC, BKC, TAG, true, PF>),
                       dim3(tm * tn * d.split), dim3(WM * WN * kWave), 0, s, d, tm, tn);
  else
    hipLaunchKernelGGL((gemm_lowp_kernel<MODE, BM, BN, BK, WM, WN, AKC, BKC, TAG, false, 1>),
                       dim3(tm * tn * d.split), dim3(WM * WN * kWave), 0, s, d, tm, tn);
}

struct LTile {
  const char *name;
  int BM, BN, BK;
  void (*launch[4])(const GemmDesc &, int64_t, int64_t, hipStream_t);
  void (*launch_ladder)(const GemmDesc &, int64_t, int64_t, hipStream_t);
  void (*launch_ladder_tail)(const GemmDesc &, int64_t, int64_t, hipStream_t);
  void (*launch_grouped[4])(const GemmGroupEntry *, const int64_t *, int, int64_t, hipStream_t);
  int (*occupancy[8])();  // resident workgroups per CU, [lp_in*4 + akc*2 + bkc]
  bool blocked = false;   // its LDS-direct kernel also reads blocked copies (lp_in == 2)
  // grouped launch on converted copies of K-contiguous operands (lp_in == 1)
  void (*launch_grouped_lp)(const GemmGroupEntry *, const int64_t *, int, int64_t, hipStream_t) = nullptr;
};

// workgroups of one configuration resident on a CU (0 if unknown)
template <int MODE, int BM, int BN, int BK, int WM, int WN, bool AKC, bool BKC, bool LPIN, int PF>
int occ_l() {
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
          &nb, gemm_lowp_kernel<MODE, BM, BN, BK, WM, WN, AKC, BKC, 0, LPIN, LPIN ? PF : 1>, WM * WN * kWave, 0) !=
      hipSuccess) {
    (void)hipGetLastError();
    return 0;
  }
  return nb;
}
#define CC_LOCC(MODE, BM, BN, BK, WM, WN, LPIN, PF)                                                            \
  &occ_l<MODE, BM, BN, BK, WM, WN, false, false, LPIN, PF>, &occ_l<MODE, BM, BN, BK, WM, WN, false, true, LPIN, PF>, \
      &occ_l<MODE, BM, BN, BK, WM, WN, true, false, LPIN, PF>, &occ_l<MODE, BM, BN, BK, WM, WN, true, true, LPIN, PF>
#define CC_LTILE(MODE, BM, BN, BK, WM, WN, PF)                                                                   \
  LTile {                                                                                                        \
    #BM "x" #BN "x" #BK "_w" #WM "x" #WN "_p" #PF, BM, BN, BK,                                                   \
        {&launch_l<MODE, BM, BN, BK, WM, WN, false, false, PF>, &launch_l<MODE, BM, BN, BK, WM, WN, false, true, PF>, \
         &launch_l<MODE, BM, BN, BK, WM, WN, true, false, PF>, &launch_l<MODE, BM, BN, BK, WM, WN, true, true, PF>},  \
        &launch_l<MODE, BM, BN, BK, WM, WN, true, true, PF, 1>, &launch_l<MODE, BM, BN, BK, WM, WN, true, true, PF, 2>, \
        {&launch_lg<MODE, BM, BN, BK, WM, WN, false, false>, &launch_lg<MODE, BM, BN, BK, WM, WN, false, true>,     \
         &launch_lg<MODE, BM, BN, BK, WM, WN, true, false>, &launch_lg<MODE, BM, BN, BK, WM, WN, true, true>},      \
        {CC_LOCC(MODE, BM, BN, BK, WM, WN, false, PF), CC_LOCC(MODE, BM, BN, BK, WM, WN, true, PF)},             \
        false, &launch_lg<MODE, BM, BN, BK, WM, WN, true, true, true>                                           \
  }
template <int TAG>
void launch_b3_dma(const GemmDesc &d, int64_t tm, int64_t tn, hipStream_t s) {
  if (b3_dma_ok(d))
    hipLaunchKernelGGL((gemm_b3_dma_kernel<TAG>), dim3(tm * tn * d.split), dim3(dma::NT), 0, s, d, tm, tn);
  else
    launch_l<PREC_BF16X3, 256, 128, 32, 4, 2, true, true, 1, TAG>(d, tm, tn, s);
}
template <int TAG>
void launch_f32_dma(const GemmDesc &d, int64_t tm, int64_t tn, hipStream_t s) {
  if (f32_dma_ok(d))
    hipLaunchKernelGGL((gemm_f32_dma_kernel<TAG>), dim3(tm * tn * d.split), dim3(dma::NT), 0, s, d, tm, tn);
  else
    launch_l<PREC_F32, 256, 128, 32, 4, 2, true, true, 1, TAG>(d, tm, tn, s);
}
int occ_f32_dma() {
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, gemm_f32_dma_kernel<0>, dma::NT, 0) != hipSuccess) {
    (void)hipGetLastError();
    return 0;
  }
  return nb;
}
template <int TAG>
void launch_b3_dmap(const GemmDesc &d, int64_t tm, int64_t tn, hipStream_t s) {
  if (b3_dma_ok(d))
    hipLaunchKernelGGL((gemm_b3_dmap_kernel<TAG>), dim3(tm * tn * d.split), dim3(dma::NT), 0, s, d, tm, tn);
  else
    launch_l<PREC_BF16X3, 256, 128, 32, 4, 2, true, true, 1, TAG>(d, tm, tn, s);
}
int occ_b3_dmap() {
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, gemm_b3_dmap_kernel<0>, dma::NT, 0) != hipSuccess) {
    (void)hipGetLastError();
    return 0;
  }
  return nb;
}
int occ_b3_dma() {
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, gemm_b3_dma_kernel<0>, dma::NT, 0) != hipSuccess) {
    (void)hipGetLastError();
    return 0;
  }
  return nb;
}
template <int TAG>
void launch_b3_dmw(const GemmDesc &d, int64_t tm, int64_t tn, hipStream_t s) {
  if (b3_dma_ok(d))
    hipLaunchKernelGGL((gemm_b3_dmw_kernel<TAG>), dim3(tm * tn * d.split), dim3(dmw::NT), 0, s, d, tm, tn);
  else  // shapes it does not take: the staged 256x128 kernel over its own tiles
    launch_l<PREC_BF16X3, 256, 128, 32, 4, 2, true, true, 1, TAG>(d, (d.M + 255) / 256, (d.N + 127) / 128, s);
}
template <bool AKC, bool BKC>
void launch_b3_w_staged(const GemmDesc &d, int64_t, int64_t, hipStream_t s) {
  launch_l<PREC_BF16X3, 256, 128, 32, 4, 2, AKC, BKC, 1>(d, (d.M + 255) / 256, (d.N + 127) / 128, s);
}
int occ_b3_dmw() {
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, gemm_b3_dmw_kernel<0>, dmw::NT, 0) != hipSuccess) {
    (void)hipGetLastError();
    return 0;
  }
  return nb;
}
const LTile kF32Tiles[] = {
    CC_LTILE(PREC_F32, 128, 128, 16, 2, 2, 1), CC_LTILE(PREC_F32, 64, 64, 16, 2, 2, 1),
    CC_LTILE(PREC_F32, 32, 32, 16, 2, 2, 1),   CC_LTILE(PREC_F32, 128, 64, 16, 2, 2, 1),
    CC_LTILE(PREC_F32, 64, 128, 16, 2, 2, 1),  CC_LTILE(PREC_F32, 128, 128, 32, 2, 2, 1),
    CC_LTILE(PREC_F32, 128, 128, 16, 4, 2, 1), CC_LTILE(PREC_F32, 128, 128, 32, 4, 2, 1),
    CC_LTILE(PREC_F32, 128, 128, 32, 4, 2, 2), CC_LTILE(PREC_F32, 256, 128, 32, 4, 2, 1),
    // 256x128x32 with LDS-direct loads where the shape allows, else staged
    LTile{"256x128x32_w4x2_lds",
          256,
          128,
          32,
          {&launch_l<PREC_F32, 256, 128, 32, 4, 2, false, false, 1>, &launch_l<PREC_F32, 256, 128, 32, 4, 2, false, true, 1>,
           &launch_l<PREC_F32, 256, 128, 32, 4, 2, true, false, 1>, &launch_f32_dma<0>},
          &launch_f32_dma<1>,
          &launch_f32_dma<2>,
          {&launch_lg<PREC_F32, 256, 128, 32, 4, 2, false, false>, &launch_lg<PREC_F32, 256, 128, 32, 4, 2, false, true>,
           &launch_lg<PREC_F32, 256, 128, 32, 4, 2, true, false>, &launch_lg<PREC_F32, 256, 128, 32, 4, 2, true, true>},
          {CC_LOCC(PREC_F32, 256, 128, 32, 4, 2, false, 1), &occ_l<PREC_F32, 256, 128, 32, 4, 2, false, false, true, 1>,
           &occ_l<PREC_F32, 256, 128, 32, 4, 2, false, true, true, 1>,
           &occ_l<PREC_F32, 256, 128, 32, 4, 2, true, false, true, 1>, &occ_f32_dma},
          false,
          &launch_lg<PREC_F32, 256, 128, 32, 4, 2, true, true, true>},
};
const LTile kB3Tiles[] = {
    CC_LTILE(PREC_BF16X3, 128, 128, 32, 2, 2, 1), CC_LTILE(PREC_BF16X3, 64, 64, 32, 2, 2, 1),
    CC_LTILE(PREC_BF16X3, 32, 32, 32, 2, 2, 1),   CC_LTILE(PREC_BF16X3, 128, 64, 32, 2, 2, 1),
    CC_LTILE(PREC_BF16X3, 64, 128, 32, 2, 2, 1),  CC_LTILE(PREC_BF16X3, 128, 128, 64, 2, 2, 1),
    CC_LTILE(PREC_BF16X3, 128, 128, 32, 4, 2, 1), CC_LTILE(PREC_BF16X3, 256, 128, 32, 4, 2, 1),
    CC_LTILE(PREC_BF16X3, 128, 128, 32, 4, 2, 2),
    // 256x128x32 with LDS-direct loads where the shape allows, else staged
    LTile{"256x128x32_w4x2_lds",
          256,
          128,
          32,
          {&launch_l<PREC_BF16X3, 256, 128, 32, 4, 2, false, false, 1>,
           &launch_l<PREC_BF16X3, 256, 128, 32, 4, 2, false, true, 1>,
           &launch_l<PREC_BF16X3, 256, 128, 32, 4, 2, true, false, 1>, &launch_b3_dma<0>},
          &launch_b3_dma<1>,
          &launch_b3_dma<2>,
          {&launch_lg<PREC_BF16X3, 256, 128, 32, 4, 2, false, false>,
           &launch_lg<PREC_BF16X3, 256, 128, 32, 4, 2, false, true>,
           &launch_lg<PREC_BF16X3, 256, 128, 32, 4, 2, true, false>,
           &launch_lg<PREC_BF16X3, 256, 128, 32, 4, 2, true, true>},
          {CC_LOCC(PREC_BF16X3, 256, 128, 32, 4, 2, false, 1), &occ_l<PREC_BF16X3, 256, 128, 32, 4, 2, false, false, true, 1>,
           &occ_l<PREC_BF16X3, 256, 128, 32, 4, 2, false, true, true, 1>,
           &occ_l<PREC_BF16X3, 256, 128, 32, 4, 2, true, false, true, 1>, &occ_b3_dma},
          true,
          &launch_lg<PREC_BF16X3, 256, 128, 32, 4, 2, true, true, true>},
    // the same with the next chunk's fragments read behind the current MFMAs
    LTile{"256x128x32_w4x2_ldsp",
          256,
          128,
          32,
          {&launch_l<PREC_BF16X3, 256, 128, 32, 4, 2, false, false, 1>,
           &launch_l<PREC_BF16X3, 256, 128, 32, 4, 2, false, true, 1>,
           &launch_l<PREC_BF16X3, 256, 128, 32, 4, 2, true, false, 1>, &launch_b3_dmap<0>},
          &launch_b3_dmap<1>,
          &launch_b3_dmap<2>,
          {&launch_lg<PREC_BF16X3, 256, 128, 32, 4, 2, false, false>,
           &launch_lg<PREC_BF16X3, 256, 128, 32, 4, 2, false, true>,
           &launch_lg<PREC_BF16X3, 256, 128, 32, 4, 2, true, false>,
           &launch_lg<PREC_BF16X3, 256, 128, 32, 4, 2, true, true>},
          {CC_LOCC(PREC_BF16X3, 256, 128, 32, 4, 2, false, 1), &occ_l<PREC_BF16X3, 256, 128, 32, 4, 2, false, false, true, 1>,
           &occ_l<PREC_BF16X3, 256, 128, 32, 4, 2, false, true, true, 1>,
           &occ_l<PREC_BF16X3, 256, 128, 32, 4, 2, true, false, true, 1>, &occ_b3_dmap},
          true,
          &launch_lg<PREC_BF16X3, 256, 128, 32, 4, 2, true, true, true>},
    // 256x256 with LDS-direct loads where the shape allows, else the staged
    // 256x128 kernel over its own tiles; no grouped launches (batches use
    // per-system tile tables of one tile shape)
    LTile{"256x256x32_w2x4_lds",
          256,
          256,
          32,
          {&launch_b3_w_staged<false, false>, &launch_b3_w_staged<false, true>, &launch_b3_w_staged<true, false>,
           &launch_b3_dmw<0>},
          &launch_b3_dmw<1>,
          &launch_b3_dmw<2>,
          {nullptr, nullptr, nullptr, nullptr},
          {CC_LOCC(PREC_BF16X3, 256, 128, 32, 4, 2, false, 1), &occ_l<PREC_BF16X3, 256, 128, 32, 4, 2, false, false, true, 1>,
           &occ_l<PREC_BF16X3, 256, 128, 32, 4, 2, false, true, true, 1>,
           &occ_l<PREC_BF16X3, 256, 128, 32, 4, 2, true, false, true, 1>, &occ_b3_dmw},
          true},
};
constexpr int kNumF32 = sizeof(kF32Tiles) / sizeof(kF32Tiles[0]);
constexpr int kNumB3 = sizeof(kB3Tiles) / sizeof(kB3Tiles[0]);
constexpr int kNumL = kNumF32 > kNumB3 ? kNumF32 : kNumB3;  // slot cache extent
int num_l(int prec) { return prec == PREC_F32 ? kNumF32 : kNumB3; }

// resident slots per (precision, configuration, variant) on the device; -1 = not yet asked
std::atomic<int64_t> g_lslots[2][kNumL][8];
std::once_flag g_lslots_once;

int64_t lowp_slots(const GemmDesc &d, int prec, int tile_id) {
  std::call_once(g_lslots_once, [] {
    for (auto &a : g_lslots)
      for (auto &b : a)
        for (auto &x : b) x.store(-1);
  });
  const LTile &ti = (prec == PREC_F32 ? kF32Tiles : kB3Tiles)[tile_id];
  const int var = (d.lp_in ? 4 : 0) + (d.sak == 1 ? 2 : 0) + (d.sbk == 1 ? 1 : 0);
  std::atomic<int64_t> &cell = g_lslots[prec == PREC_F32 ? 0 : 1][tile_id][var];
  int64_t slots = cell.load();
  if (slots < 0) {
    slots = int64_t(ti.occupancy[var]()) * gpu_cu_count();
    cell.store(slots);
  }
  return slots;
}

TailCut lowp_cut(const GemmDesc &d, int prec, int tile_id) {
  if (d.split != 1 || d.K <= 0) return TailCut{};
  const LTile &ti = (prec == PREC_F32 ? kF32Tiles : kB3Tiles)[tile_id];
  return gemm_tail_cut(d.M, d.N, d.K, ti.BM, ti.BN, ti.BK, lowp_slots(d, prec, tile_id));
}

int pick_l(const LTile *tiles, int64_t M, int64_t N) {
  const int count = tiles == kF32Tiles ? kNumF32 : kNumB3;
  int best = 0;
  double best_cost = 1e300;
  for (int t = 0; t < count; ++t) {
    if (!tiles[t].launch_grouped[0]) continue;  // chosen by timing only
    const double n = double((M + tiles[t].BM - 1) / tiles[t].BM) * double((N + tiles[t].BN - 1) / tiles[t].BN);
    const double cost = std::ceil(n / 256.0) * (double(tiles[t].BM) * tiles[t].BN + 4096.0);
    if (cost < best_cost) {
      best_cost = cost;
      best = t;
    }
  }
  return best;
}

__global__ __launch_bounds__(256) void to_f32_kernel(const double *__restrict__ src, int64_t n,
                                                     float *__restrict__ dst) {
  for (int64_t e = blockIdx.x * int64_t(256) + threadIdx.x; e < n; e += int64_t(gridDim.x) * 256)
    dst[e] = static_cast<float>(src[e]);
}

__global__ __launch_bounds__(256) void to_bf16x2_kernel(const double *__restrict__ src, int64_t n,
                                                        unsigned short *__restrict__ hi) {
  unsigned short *__restrict__ lo = hi + n;
  for (int64_t e = blockIdx.x * int64_t(256) + threadIdx.x; e < n; e += int64_t(gridDim.x) * 256) {
    const float x = static_cast<float>(src[e]);
    const unsigned short h = bf16_bits(x);
    hi[e] = h;
    lo[e] = bf16_bits(x - bf16_to_float(h));
  }
}

// Grouped conversion: entry b's n values, kConvChunk per workgroup, rounded
// and split exactly as to_f32_kernel / to_bf16x2_kernel do.
constexpr int64_t kConvChunk = 2048;

template <int MODE>
__global__ __launch_bounds__(256) void g_convert_kernel(const ConvEntry *__restrict__ es,
                                                        const int64_t *__restrict__ off, int n) {
  const int b = group_find(off, n, blockIdx.x);
  const double *__restrict__ src = es[b].src;
  const int64_t m = es[b].n;
  const int64_t base = (int64_t(blockIdx.x) - off[b]) * kConvChunk, end = std::min(m, base + kConvChunk);
  for (int64_t e = base + threadIdx.x; e < end; e += 256) {
    const float x = static_cast<float>(src[e]);
    if (MODE == PREC_F32) {
      static_cast<float *>(es[b].dst)[e] = x;
    } else {
      unsigned short *__restrict__ hi = static_cast<unsigned short *>(es[b].dst);
      const unsigned short h = bf16_bits(x);
      hi[e] = h;
      hi[m + e] = bf16_bits(x - bf16_to_float(h));
    }
  }
}

// The same split of a row-major R x K operand (K a multiple of 32) into
// 16-row x 32-k blocks of 512 elements: block (rb, kb) at (rb K/32 + kb) 512,
// slot s = (row & 15) + 16 ((k & 31) >> 3) holding k & 7 = 0..7 at 8 s (the
// LDS slot order of the LDS-direct kernels), rows padded with zeros to a
// multiple of 16; hi plane, then the lo plane `plane` elements further.
// One thread per slot: eight elements, one 16-byte store per plane.
// With ref, the copy is of src - ref (the correction form's varying operand).
__global__ __launch_bounds__(256) void to_bf16x2_blocked_kernel(const double *__restrict__ src,
                                                                const double *__restrict__ ref, int64_t R, int64_t K,
                                                                int64_t nslot, int64_t plane,
                                                                unsigned short *__restrict__ hi) {
  const int64_t kblocks = K >> 5;
  for (int64_t t = blockIdx.x * int64_t(256) + threadIdx.x; t < nslot; t += int64_t(gridDim.x) * 256) {
    const int64_t blk = t >> 6;
    const int sl = int(t & 63);
    const int64_t row = (blk / kblocks) * 16 + (sl & 15), k = (blk % kblocks) * 32 + (sl >> 4) * 8;
    union {
      uint4 u;
      unsigned short e[8];
    } h, l;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int64_t at = row * K + k + e;
      const float x = row < R ? static_cast<float>(ref ? src[at] - ref[at] : src[at]) : 0.f;
      h.e[e] = bf16_bits(x);
      l.e[e] = bf16_bits(x - bf16_to_float(h.e[e]));
    }
    *reinterpret_cast<uint4 *>(hi + 8 * t) = h.u;
    *reinterpret_cast<uint4 *>(hi + plane + 8 * t) = l.u;
  }
}

// The same copy with one wave per block (src and ref 16-byte aligned): load
// i of lane L takes the two doubles k = 2 (L & 15), +1 of block row
// 4 i + (L >> 4), so each load covers four whole 256-byte row segments; the
// pair goes to slot row + 16 ((L & 15) >> 2), elements 2 (L & 3), +1.
__global__ __launch_bounds__(256) void to_bf16x2_blocked_rows_kernel(const double *__restrict__ src,
                                                                     const double *__restrict__ ref, int64_t R,
                                                                     int64_t K, int64_t nblk, int64_t plane,
                                                                     unsigned short *__restrict__ hi) {
  const int64_t kblocks = K >> 5;
  const int lane = threadIdx.x & 63, p = lane & 15;
  for (int64_t blk = (blockIdx.x * int64_t(256) + threadIdx.x) >> 6; blk < nblk; blk += int64_t(gridDim.x) * 4) {
    const int64_t r0 = (blk / kblocks) * 16, k = (blk % kblocks) * 32 + 2 * p;
    unsigned short *__restrict__ hb = hi + blk * 512;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int rr = 4 * i + (lane >> 4);
      const int64_t row = r0 + rr;
      double x0 = 0.0, x1 = 0.0;
      if (row < R) {
        const double2 a = *reinterpret_cast<const double2 *>(src + row * K + k);
        x0 = a.x;
        x1 = a.y;
        if (ref) {
          const double2 b = *reinterpret_cast<const double2 *>(ref + row * K + k);
          x0 = x0 - b.x;
          x1 = x1 - b.y;
        }
      }
      const float f0 = static_cast<float>(x0), f1 = static_cast<float>(x1);
      const unsigned short h0 = bf16_bits(f0), h1 = bf16_bits(f1);
      const unsigned short l0 = bf16_bits(f0 - bf16_to_float(h0)), l1 = bf16_bits(f1 - bf16_to_float(h1));
      const int at = (rr + 16 * (p >> 2)) * 8 + 2 * (p & 3);
      *reinterpret_cast<uint32_t *>(hb + at) = uint32_t(h0) | (uint32_t(h1) << 16);
      *reinterpret_cast<uint32_t *>(hb + plane + at) = uint32_t(l0) | (uint32_t(l1) << 16);
    }
  }
}

__global__ __launch_bounds__(256) void delta_f32_kernel(const double *__restrict__ a, const double *__restrict__ ref,
                                                        int64_t n, float *__restrict__ dst) {
  for (int64_t e = blockIdx.x * int64_t(256) + threadIdx.x; e < n; e += int64_t(gridDim.x) * 256)
    dst[e] = static_cast<float>(a[e] - ref[e]);
}

__global__ __launch_bounds__(256) void delta_bf16x2_kernel(const double *__restrict__ a,
                                                           const double *__restrict__ ref, int64_t n,
                                                           unsigned short *__restrict__ hi) {
  unsigned short *__restrict__ lo = hi + n;
  for (int64_t e = blockIdx.x * int64_t(256) + threadIdx.x; e < n; e += int64_t(gridDim.x) * 256) {
    const float x = static_cast<float>(a[e] - ref[e]);
    const unsigned short h = bf16_bits(x);
    hi[e] = h;
    lo[e] = bf16_bits(x - bf16_to_float(h));
  }
}

__global__ __launch_bounds__(256) void copy_f64_kernel(const double *__restrict__ src, int64_t n,
                                                       double *__restrict__ dst) {
  for (int64_t e = blockIdx.x * int64_t(256) + threadIdx.x; e < n; e += int64_t(gridDim.x) * 256) dst[e] = src[e];
}

// C[m][n] = beta C[m][n] + P[m][n]   (P dense M x N; C not read when beta = 0)
__global__ __launch_bounds__(256) void add_product_kernel(double *__restrict__ C, int64_t ldc, double beta,
                                                          const double *__restrict__ P, int64_t M, int64_t N) {
  const int64_t total = M * N;
  for (int64_t e = blockIdx.x * int64_t(256) + threadIdx.x; e < total; e += int64_t(gridDim.x) * 256) {
    const int64_t m = e / N, c = e % N;
    double *q = C + m * ldc + c;
    *q = (beta == 0.0) ? P[e] : beta * *q + P[e];
  }
}

int64_t ew_blocks(int64_t n) { return std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 65536)); }

// ---- complex operands as real ones -----------------------------------------
// A complex product C(m,n) = sum_k A(m,k) B(n,k) is the real product of
//   A' (M x 2K):  A'[m][2k] = Re A(m,k),   A'[m][2k+1] = Im A(m,k)
//   B' (2N x 2K): B'[2n][2k]   = Re B(n,k), B'[2n][2k+1]   = -Im B(n,k)
//                 B'[2n+1][2k] = Im B(n,k), B'[2n+1][2k+1] =  Re B(n,k)
// since sum_k' A'(m,k') B'(2n+c,k') is the real (c = 0) or imaginary (c = 1)
// part of C(m,n): exactly the interleaved layout of complex C, read as a real
// M x 2N matrix.  The reduced-precision copies hold A', B' dense (rows of
// 2K), rounded as convert_shadow rounds, optionally of X - X_ref.
// Each value goes to dst (FP32) or to the bf16 hi plane at dst and the lo
// plane `plane` elements further.
template <int MODE>
__device__ __forceinline__ void put_lp(void *dst, int64_t plane, int64_t i, double x) {
  const float f = static_cast<float>(x);
  if constexpr (MODE == PREC_F32) {
    static_cast<float *>(dst)[i] = f;
  } else {
    unsigned short *hi = static_cast<unsigned short *>(dst);
    const unsigned short h = bf16_bits(f);
    hi[i] = h;
    hi[plane + i] = bf16_bits(f - bf16_to_float(h));
  }
}

// element (row, k) of a real operand with rows of Kr (a multiple of 32) in
// the 16 x 32 blocks of convert_blocked
__device__ __forceinline__ int64_t blocked_at(int64_t row, int64_t k, int64_t Kr) {
  return ((row >> 4) * (Kr >> 5) + (k >> 5)) * 512 + ((row & 15) + 16 * ((k & 31) >> 3)) * 8 + (k & 7);
}

// one thread per complex element (r, k), k fastest; SIDE 0 writes A', 1 B';
// BLK: in 16 x 32 blocks (split bf16; rows of 2K, planes padded to 16 rows)
template <int MODE, int SIDE, bool REF, bool BLK>
__global__ __launch_bounds__(256) void realify_kernel(const double2 *__restrict__ src, const double2 *__restrict__ ref,
                                                      int64_t R, int64_t K, int64_t sr, int64_t sk, void *dst) {
  const int64_t total = R * K;
  const int64_t plane = BLK ? (((SIDE == 0 ? R : 2 * R) + 15) / 16 * 16) * 2 * K : (SIDE == 0 ? 2 : 4) * total;
  auto at = [K](int64_t row, int64_t kk) { return BLK ? blocked_at(row, kk, 2 * K) : row * 2 * K + kk; };
  for (int64_t e = blockIdx.x * int64_t(256) + threadIdx.x; e < total; e += int64_t(gridDim.x) * 256) {
    const int64_t r = e / K, k = e - r * K;
    const int64_t q = r * sr + k * sk;
    double re = src[q].x, im = src[q].y;
    if constexpr (REF) {
      re -= ref[q].x;
      im -= ref[q].y;
    }
    if constexpr (SIDE == 0) {
      put_lp<MODE>(dst, plane, at(r, 2 * k), re);
      put_lp<MODE>(dst, plane, at(r, 2 * k + 1), im);
    } else {
      put_lp<MODE>(dst, plane, at(2 * r, 2 * k), re);
      put_lp<MODE>(dst, plane, at(2 * r, 2 * k + 1), -im);
      put_lp<MODE>(dst, plane, at(2 * r + 1, 2 * k), im);
      put_lp<MODE>(dst, plane, at(2 * r + 1, 2 * k + 1), re);
    }
  }
}

template <int MODE, int SIDE>
void realify_launch(const double *src, const double *ref, int64_t R, int64_t K, int64_t sr, int64_t sk, void *dst,
                    hipStream_t s) {
  const auto *a = reinterpret_cast<const double2 *>(src);
  const auto *b = reinterpret_cast<const double2 *>(ref);
  if (ref)
    hipLaunchKernelGGL((realify_kernel<MODE, SIDE, true, false>), dim3(ew_blocks(R * K)), dim3(256), 0, s, a, b, R, K,
                       sr, sk, dst);
  else
    hipLaunchKernelGGL((realify_kernel<MODE, SIDE, false, false>), dim3(ew_blocks(R * K)), dim3(256), 0, s, a, b, R,
                       K, sr, sk, dst);
}

}  // namespace

void realify_complex(int prec, int side, const double *src, const double *ref, int64_t R, int64_t K, int64_t sr,
                     int64_t sk, void *dst, hipStream_t s) {
  if (R <= 0 || K <= 0) return;
  CC_REQUIRE(prec == PREC_F32 || prec == PREC_BF16X3, -1, "realify: precision");
  if (prec == PREC_F32) {
    if (side == 0) realify_launch<PREC_F32, 0>(src, ref, R, K, sr, sk, dst, s);
    else realify_launch<PREC_F32, 1>(src, ref, R, K, sr, sk, dst, s);
  } else {
    if (side == 0) realify_launch<PREC_BF16X3, 0>(src, ref, R, K, sr, sk, dst, s);
    else realify_launch<PREC_BF16X3, 1>(src, ref, R, K, sr, sk, dst, s);
  }
  CC_HIP_CHECK(hipGetLastError());
}

void realify_complex_blocked(int side, const double *src, int64_t R, int64_t K, void *dst, hipStream_t s) {
  if (R <= 0 || K <= 0) return;
  CC_REQUIRE(K % 16 == 0, -1, "blocked realified copy: K must be a multiple of 16");
  CC_REQUIRE((reinterpret_cast<uintptr_t>(dst) & 15) == 0, -1, "blocked realified copy: alignment");
  const auto *a = reinterpret_cast<const double2 *>(src);
  if (side == 0)
    hipLaunchKernelGGL((realify_kernel<PREC_BF16X3, 0, false, true>), dim3(ew_blocks(R * K)), dim3(256), 0, s, a,
                       nullptr, R, K, K, int64_t(1), dst);
  else
    hipLaunchKernelGGL((realify_kernel<PREC_BF16X3, 1, false, true>), dim3(ew_blocks(R * K)), dim3(256), 0, s, a,
                       nullptr, R, K, K, int64_t(1), dst);
  CC_HIP_CHECK(hipGetLastError());
}

GemmDesc realified_desc(const GemmDesc &d, const void *a_form, const void *b_form) {
  GemmDesc g = d;
  g.N = 2 * d.N;
  g.K = 2 * d.K;
  g.A = a_form;
  g.sam = 2 * d.K;
  g.sak = 1;
  g.B = b_form;
  g.sbn = 2 * d.K;
  g.sbk = 1;
  g.ldc = 2 * d.ldc;
  g.a_plane = 2 * d.M * d.K;
  g.b_plane = 4 * d.N * d.K;
  g.lp_in = 1;
  g.ws_elems = 2 * d.ws_elems;  // complex elements of the workspace, as doubles
  return g;
}

void convert_delta(int prec, const double *a, const double *ref, int64_t n, void *dst, hipStream_t s) {
  if (n <= 0) return;
  if (prec == PREC_F32)
    hipLaunchKernelGGL(delta_f32_kernel, dim3(ew_blocks(n)), dim3(256), 0, s, a, ref, n, static_cast<float *>(dst));
  else
    hipLaunchKernelGGL(delta_bf16x2_kernel, dim3(ew_blocks(n)), dim3(256), 0, s, a, ref, n,
                       static_cast<unsigned short *>(dst));
  CC_HIP_CHECK(hipGetLastError());
}

void copy_f64(double *dst, const double *src, int64_t n, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(copy_f64_kernel, dim3(ew_blocks(n)), dim3(256), 0, s, src, n, dst);
  CC_HIP_CHECK(hipGetLastError());
}

void add_product(double *C, int64_t ldc, double beta, const double *P, int64_t M, int64_t N, hipStream_t s) {
  if (M <= 0 || N <= 0) return;
  hipLaunchKernelGGL(add_product_kernel, dim3(ew_blocks(M * N)), dim3(256), 0, s, C, ldc, beta, P, M, N);
  CC_HIP_CHECK(hipGetLastError());
}

void convert_shadow(int prec, const double *src, int64_t n, void *dst, hipStream_t s) {
  if (n <= 0) return;
  const int64_t blocks = std::min<int64_t>((n + 255) / 256, 65536);
  if (prec == PREC_F32)
    hipLaunchKernelGGL(to_f32_kernel, dim3(blocks), dim3(256), 0, s, src, n, static_cast<float *>(dst));
  else
    hipLaunchKernelGGL(to_bf16x2_kernel, dim3(blocks), dim3(256), 0, s, src, n, static_cast<unsigned short *>(dst));
  CC_HIP_CHECK(hipGetLastError());
}

int64_t blocked_plane(int64_t R, int64_t K) { return (R + 15) / 16 * 16 * K; }

ConvEntry make_conv_entry(const double *src, int64_t n, void *dst) {
  return ConvEntry{src, dst, n, n > 0 ? (n + kConvChunk - 1) / kConvChunk : 0};
}

void convert_shadow_grouped(int prec, const ConvEntry *e, const int64_t *off, int n, int64_t blocks,
                            hipStream_t s) {
  if (blocks <= 0) return;
  CC_REQUIRE(blocks < (int64_t(1) << 31), -1, "grouped conversion: grid too large");
  if (prec == PREC_F32) hipLaunchKernelGGL(g_convert_kernel<PREC_F32>, dim3(blocks), dim3(256), 0, s, e, off, n);
  else hipLaunchKernelGGL(g_convert_kernel<PREC_BF16X3>, dim3(blocks), dim3(256), 0, s, e, off, n);
  CC_HIP_CHECK(hipGetLastError());
}

void convert_blocked(const double *src, const double *ref, int64_t R, int64_t K, void *dst, hipStream_t s) {
  CC_REQUIRE(R > 0 && K > 0 && K % 32 == 0, -1, "blocked split-bf16 copy: K must be a multiple of 32");
  CC_REQUIRE((reinterpret_cast<uintptr_t>(dst) & 15) == 0, -1, "blocked split-bf16 copy: alignment");
  const int64_t plane = blocked_plane(R, K), nslot = plane / 8;
  if (((reinterpret_cast<uintptr_t>(src) | reinterpret_cast<uintptr_t>(ref)) & 15) == 0) {
    const int64_t nblk = plane / 512;
    hipLaunchKernelGGL(to_bf16x2_blocked_rows_kernel, dim3(std::min<int64_t>((nblk + 3) / 4, 65536)), dim3(256), 0,
                       s, src, ref, R, K, nblk, plane, static_cast<unsigned short *>(dst));
  } else {
    const int64_t blocks = std::min<int64_t>((nslot + 255) / 256, 65536);
    hipLaunchKernelGGL(to_bf16x2_blocked_kernel, dim3(blocks), dim3(256), 0, s, src, ref, R, K, nslot, plane,
                       static_cast<unsigned short *>(dst));
  }
  CC_HIP_CHECK(hipGetLastError());
}

bool gemm_lowp_tile_blocked(int prec, int tile_id) {
  return prec == PREC_BF16X3 && tile_id >= 0 && tile_id < num_l(prec) && kB3Tiles[tile_id].blocked;
}

int gemm_lowp_num_tiles(int prec) { return num_l(prec); }

int gemm_lowp_pick(int prec, int64_t M, int64_t N) { return pick_l(prec == PREC_F32 ? kF32Tiles : kB3Tiles, M, N); }

bool gemm_lowp_tile_grouped(int prec, int tile_id) {
  return tile_id >= 0 && tile_id < num_l(prec) &&
         (prec == PREC_F32 ? kF32Tiles : kB3Tiles)[tile_id].launch_grouped[0] != nullptr &&
         (prec == PREC_F32 ? kF32Tiles : kB3Tiles)[tile_id].launch_grouped_lp != nullptr;
}

void gemm_lowp_tile_shape(int prec, int tile_id, int *bm, int *bn) {
  const LTile &t = (prec == PREC_F32 ? kF32Tiles : kB3Tiles)[tile_id];
  *bm = t.BM;
  *bn = t.BN;
}

void gemm_lowp_grouped_launch(const GemmGroupEntry *dev_entries, const int64_t *dev_off, int n, int64_t blocks,
                              bool akc, bool bkc, int prec, int tile_id, hipStream_t s) {
  if (blocks <= 0) return;
  CC_REQUIRE(prec == PREC_F32 || prec == PREC_BF16X3, -1, "grouped gemm: precision");
  CC_REQUIRE(tile_id >= 0 && tile_id < num_l(prec), -7, "grouped gemm: tile");
  CC_REQUIRE(blocks < (int64_t(1) << 31), -1, "grouped gemm: too many tiles");
  CC_REQUIRE(gemm_lowp_tile_grouped(prec, tile_id), -7, "grouped gemm: tile has no grouped launch");
  (prec == PREC_F32 ? kF32Tiles : kB3Tiles)[tile_id].launch_grouped[(akc ? 2 : 0) + (bkc ? 1 : 0)](
      dev_entries, dev_off, n, blocks, s);
  CC_HIP_CHECK(hipGetLastError());
}
void gemm_lowp_grouped_launch_lp(const GemmGroupEntry *dev_entries, const int64_t *dev_off, int n,
                                 int64_t blocks, int prec, int tile_id, hipStream_t s) {
  if (blocks <= 0) return;
  CC_REQUIRE(prec == PREC_F32 || prec == PREC_BF16X3, -1, "grouped gemm: precision");
  CC_REQUIRE(gemm_lowp_tile_grouped(prec, tile_id), -7, "grouped gemm: tile has no grouped launch");
  CC_REQUIRE(blocks < (int64_t(1) << 31), -1, "grouped gemm: too many tiles");
  (prec == PREC_F32 ? kF32Tiles : kB3Tiles)[tile_id].launch_grouped_lp(dev_entries, dev_off, n, blocks, s);
  CC_HIP_CHECK(hipGetLastError());
}

const char *gemm_lowp_tile_name(int prec, int id) {
  if (id < 0 || id >= num_l(prec)) return "?";
  return prec == PREC_F32 ? kF32Tiles[id].name : kB3Tiles[id].name;
}

void gemm_lowp(const GemmDesc &d, int prec, hipStream_t s, int tile_id) {
  if (d.M <= 0 || d.N <= 0) return;
  CC_REQUIRE(prec == PREC_F32 || prec == PREC_BF16X3, -1, "gemm_lowp: precision");
  const bool akc = (d.sak == 1), bkc = (d.sbk == 1);
  CC_REQUIRE(akc || d.sam == 1, -1, "gemm: A needs a unit stride in m or k");
  CC_REQUIRE(bkc || d.sbn == 1, -1, "gemm: B needs a unit stride in n or k");
  if (d.K <= 0) {
    gemm_f64(d, s, -1);  // pure scaling of C: no products involved
    return;
  }
  const LTile *tiles = prec == PREC_F32 ? kF32Tiles : kB3Tiles;
  if (tile_id < 0 || tile_id >= num_l(prec)) tile_id = pick_l(tiles, d.M, d.N);
  const LTile &ti = tiles[tile_id];
  const int64_t tm = (d.M + ti.BM - 1) / ti.BM, tn = (d.N + ti.BN - 1) / ti.BN;
  CC_REQUIRE(d.split >= 1 && (d.split == 1 || d.ws != nullptr), -1, "gemm: split-K workspace");
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
    const TailCut tc = lowp_cut(d, prec, tile_id);
    if (tc.axis && tc.ws_elems <= d.ws_elems) {
      // operand element size: converted copies (4-byte FP32, 2-byte bf16
      // planes) or the FP64 tensors themselves
      const size_t es = d.lp_in ? (prec == PREC_F32 ? 4 : 2) : sizeof(double);
      gemm_run_cut(d, tc, es, es, one);
      return;
    }
  }
  if (d.ws && d.split > 1 && d.ws_elems > 0) {
    GemmDesc g = d;
    g.split = gemm_split_refine(d.M, d.N, d.K, ti.BM, ti.BN, ti.BK, lowp_slots(d, prec, tile_id), d.split,
                                d.ws_elems);
    one(g);
    return;
  }
  one(d);
}

int64_t gemm_lowp_tail_ws(const GemmDesc &d, int prec, int tile_id) {
  if (d.M <= 0 || d.N <= 0 || d.K <= 0 || (prec != PREC_F32 && prec != PREC_BF16X3)) return 0;
  if (tile_id < 0 || tile_id >= num_l(prec)) tile_id = pick_l(prec == PREC_F32 ? kF32Tiles : kB3Tiles, d.M, d.N);
  return lowp_cut(d, prec, tile_id).ws_elems;
}

}  // namespace ccmi
