// Data-movement and elementwise kernels of the residual path (HBM bound):
//  * LDS-tiled index permutation with scale/accumulate (the two transposes of
//    the transpose-transpose-GEMM-transpose scheme, paper Sec. "Tensor
//    contractions");
//  * outer-product accumulation (tau formation, the t1 t1 pieces);
//  * tau / tau~ formation fused with the energy reduction (Eq. eq:amp, first
//    line: E = sum f_ia t_i^a + 1/4 sum <ij||ab> tau_ij^ab);
//  * the doubles-residual assembly that applies P(ij), P(ab) and P(ij)P(ab)
//    (the permutation operators of the contraction list) fused with the
//    Jacobi update t <- t + R/(D - s) and the residual norm;
//  * deterministic two-stage reductions (fixed order: bitwise reproducible).
#include "kernels.hpp"

namespace ccmi {
namespace {

// ---------------------------------------------------------------- scalars --
__device__ __forceinline__ double cj(double x) { return x; }
__device__ __forceinline__ double2 cj(double2 x) { return make_double2(x.x, -x.y); }
__device__ __forceinline__ double sc(double a, double x) { return a * x; }
__device__ __forceinline__ double2 sc(double a, double2 x) { return make_double2(a * x.x, a * x.y); }
__device__ __forceinline__ double add(double a, double b) { return a + b; }
__device__ __forceinline__ double2 add(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double sub(double a, double b) { return a - b; }
__device__ __forceinline__ double2 sub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ double mul(double a, double b) { return a * b; }
__device__ __forceinline__ double2 mul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double abs2(double a) { return a * a; }
__device__ __forceinline__ double abs2(double2 a) { return a.x * a.x + a.y * a.y; }
template <class T> __device__ __forceinline__ T zero();
template <> __device__ __forceinline__ double zero<double>() { return 0.0; }
template <> __device__ __forceinline__ double2 zero<double2>() { return make_double2(0.0, 0.0); }
__device__ __forceinline__ double re(double a) { return a; }
__device__ __forceinline__ double re(double2 a) { return a.x; }
__device__ __forceinline__ double im(double) { return 0.0; }
__device__ __forceinline__ double im(double2 a) { return a.y; }

constexpr int RED_THREADS = 256;

// Block-wide sum in a fixed order (tree over LDS); result in every thread.
__device__ __forceinline__ double block_sum(double v, double *sh) {
  const int t = threadIdx.x;
  sh[t] = v;
  __syncthreads();
  for (int w = RED_THREADS / 2; w > 0; w >>= 1) {
    if (t < w) sh[t] += sh[t + w];
    __syncthreads();
  }
  const double r = sh[0];
  __syncthreads();
  return r;
}


constexpr int64_t CH = 1024;      // elements per workgroup, flat kernels
constexpr int64_t CH_TAU = 2048;  // elements per workgroup, tau + energy

// ------------------------------------------------------------- permutation --
// Flat path: input and output share their unit-stride dimension.
template <class T>
__device__ __forceinline__ void perm_flat_body(const PermEntry &E, int64_t bid) {
  const PermArgs &p = E.p;
  const T *__restrict__ in = static_cast<const T *>(E.in);
  T *__restrict__ out = static_cast<T *>(E.out);
  const int64_t e1 = std::min<int64_t>(p.total, (bid + 1) * CH);
  // Real tensors whose shared unit-stride dimension is even, whose other
  // strides are even and whose bases are 16-byte aligned move pairs of
  // elements with 16-byte accesses (every pair starts at an even offset and
  // never straddles a row, so one offset computation serves both).
  if constexpr (sizeof(T) == 8) {
    const int r1 = p.rank - 1;
    bool even = true;
    for (int d = 0; d < r1; ++d) even = even && (p.istr[d] % 2 == 0) && (p.ostr[d] % 2 == 0);
    if (p.rank >= 1 && even && p.dims[r1] % 2 == 0 && p.istr[r1] == 1 && p.ostr[r1] == 1 &&
        p.total < (int64_t(1) << 31) && (reinterpret_cast<uintptr_t>(in) & 15) == 0 &&
        (reinterpret_cast<uintptr_t>(out) & 15) == 0 && !p.conj) {
      typedef double d2v __attribute__((ext_vector_type(2)));
      for (int64_t e = bid * CH + 2 * threadIdx.x; e < e1; e += 512) {
        uint32_t rem = uint32_t(e);
        int64_t io = 0, oo = 0;
        for (int d = r1; d >= 0; --d) {
          const uint32_t n = uint32_t(p.dims[d]), x = rem % n;
          rem /= n;
          io += int64_t(x) * p.istr[d];
          oo += int64_t(x) * p.ostr[d];
        }
        d2v v = *reinterpret_cast<const d2v *>(in + io);
        v = d2v{p.alpha * v.x, p.alpha * v.y};
        d2v *o = reinterpret_cast<d2v *>(out + oo);
        if (p.beta != 0.0) {
          const d2v w = *o;
          v = d2v{v.x + p.beta * w.x, v.y + p.beta * w.y};
        }
        *o = v;
      }
      return;
    }
  }
  // element index -> (input, output) offsets; 32-bit division when the
  // whole tensor indexes in 32 bits (several times cheaper than 64-bit)
  const bool narrow = p.total < (int64_t(1) << 31);
  for (int64_t e = bid * CH + threadIdx.x; e < e1; e += 256) {
    int64_t io = 0, oo = 0;
    if (narrow) {
      uint32_t rem = uint32_t(e);
      for (int d = p.rank - 1; d >= 0; --d) {
        const uint32_t n = uint32_t(p.dims[d]), x = rem % n;
        rem /= n;
        io += int64_t(x) * p.istr[d];
        oo += int64_t(x) * p.ostr[d];
      }
    } else {
      int64_t rem = e;
      for (int d = p.rank - 1; d >= 0; --d) {
        const int64_t x = rem % p.dims[d];
        rem /= p.dims[d];
        io += x * p.istr[d];
        oo += x * p.ostr[d];
      }
    }
    T v = in[io];
    if (p.conj) v = cj(v);
    v = sc(p.alpha, v);
    if (p.beta != 0.0) v = add(v, sc(p.beta, out[oo]));
    out[oo] = v;
  }
}

// Tiled path: a TI x TO tile (TI TO = 1,024; 32 x 32 unless one of the two
// dims is shorter) over (input unit-stride dim, output unit-stride dim),
// read coalesced along the input's fast dim, written coalesced along the
// output's fast dim through a padded LDS tile.
template <class T>
__device__ __forceinline__ void perm_tiled_body(const PermEntry &E, int64_t bid) {
  const PermArgs &p = E.p;
  const T *__restrict__ in = static_cast<const T *>(E.in);
  T *__restrict__ out = static_cast<T *>(E.out);
  __shared__ T tile[1280];  // TO rows of TI + 1 (TO <= 256)
  int64_t b = bid;
  const int64_t ti = b % p.tiles_i; b /= p.tiles_i;
  const int64_t to = b % p.tiles_o; b /= p.tiles_o;
  int64_t ib = 0, ob = 0;
  for (int d = p.nrest - 1; d >= 0; --d) {
    const int64_t x = b % p.rest_dims[d];
    b /= p.rest_dims[d];
    ib += x * p.rest_istr[d];
    ob += x * p.rest_ostr[d];
  }
  const int lti = p.lti, lto = 10 - lti, TI = 1 << lti, TO = 1 << lto;
  const int64_t Do = p.dims[p.d_o], Di = p.dims[p.d_i];
  const int64_t i0 = ti * TI, o0 = to * TO;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int t = threadIdx.x + 256 * k, ri = t & (TI - 1), ro = t >> lti;
    const int64_t xi = i0 + ri, xo = o0 + ro;
    if (xi < Di && xo < Do) tile[ro * (TI + 1) + ri] = in[ib + xi * p.istr[p.d_i] + xo * p.istr[p.d_o]];
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int t = threadIdx.x + 256 * k, ro = t & (TO - 1), ri = t >> lto;
    const int64_t xo = o0 + ro, xi = i0 + ri;
    if (xi < Di && xo < Do) {
      T v = tile[ro * (TI + 1) + ri];
      if (p.conj) v = cj(v);
      v = sc(p.alpha, v);
      T *o = out + ob + xo * p.ostr[p.d_o] + xi * p.ostr[p.d_i];
      if (p.beta != 0.0) v = add(v, sc(p.beta, *o));
      *o = v;
    }
  }
}

// ------------------------------------------------------------ outer product --
// C[I] += alpha * A[sum_d I_d sa_d] * B[sum_d I_d sb_d]  (rank <= 4)
template <class T>
__device__ __forceinline__ void outer_body(const OuterEntry &E, int64_t bid) {
  const OuterArgs &p = E.a;
  const T *__restrict__ A = static_cast<const T *>(E.A);
  const T *__restrict__ B = static_cast<const T *>(E.B);
  T *__restrict__ C = static_cast<T *>(E.C);
  const int64_t e1 = std::min<int64_t>(E.total, (bid + 1) * CH);
  for (int64_t e = bid * CH + threadIdx.x; e < e1; e += 256) {
    int64_t rem = e, ia = 0, ibb = 0;
    for (int d = p.rank - 1; d >= 0; --d) {
      const int64_t x = rem % p.dims[d];
      rem /= p.dims[d];
      ia += x * p.sa[d];
      ibb += x * p.sb[d];
    }
    T a = A[ia], bb = B[ibb];
    if (p.conj_a) a = cj(a);
    if (p.conj_b) bb = cj(bb);
    C[e] = add(C[e], sc(p.alpha, mul(a, bb)));
  }
}

// ------------------------------------------------------------------- fill --
template <class T>
__device__ __forceinline__ void fill_body(const FillEntry &E, int64_t bid) {
  T *__restrict__ p = static_cast<T *>(E.p);
  const int64_t e1 = std::min<int64_t>(E.n, (bid + 1) * CH);
  for (int64_t e = bid * CH + threadIdx.x; e < e1; e += 256) p[e] = zero<T>();
}

// ---------------------------------------------------------- split-K sum --
// C = alpha * sum_s W[s] + beta * C.  A workgroup covers 256 / lanes
// outputs; lane l of an output sums the partials s = l, l + lanes, ... in
// increasing order, then lane 0 adds the lanes' sums in lane order.  The
// order depends only on (split, lanes), never on timing.
template <class T>
__device__ __forceinline__ void splitk_body(const SplitkEntry &E, int64_t bid) {
  __shared__ T part[256];
  const T *__restrict__ W = static_cast<const T *>(E.ws);
  T *__restrict__ C = static_cast<T *>(E.C);
  const int64_t total = E.M * E.N;
  const int L = E.lanes, nout = 256 / L;
  const int oi = threadIdx.x % nout, lane = threadIdx.x / nout;
  const int64_t e = bid * nout + oi;
  T acc = zero<T>();
  if (e < total)
    for (int k = lane; k < E.split; k += L) acc = add(acc, W[int64_t(k) * total + e]);
  part[threadIdx.x] = acc;
  __syncthreads();
  if (lane == 0 && e < total) {
    T sum = part[oi];
    for (int l = 1; l < L; ++l) sum = add(sum, part[l * nout + oi]);
    const int64_t m = e / E.N, n = e % E.N;
    T v = sc(E.alpha, sum);
    if (E.beta != 0.0) v = add(v, sc(E.beta, C[m * E.ldc + n]));
    C[m * E.ldc + n] = v;
  }
}

// --------------------------------------------------- tau + energy partials --
// tau = t2 + (t_i^a t_j^b - t_i^b t_j^a), taut = t2 + 1/2 (...),
// energy partial: 1/4 sum <ij||ab> tau_ij^ab  (+ sum f_ia t_i^a by unit 0).
template <class T>
__device__ __forceinline__ void tau_body(const TauEntry &E, int64_t bid) {
  __shared__ double sh[RED_THREADS];
  const T *__restrict__ t1 = static_cast<const T *>(E.t1);
  const T *__restrict__ t2 = static_cast<const T *>(E.t2);
  const T *__restrict__ oovv = static_cast<const T *>(E.oovv);
  const T *__restrict__ fov = static_cast<const T *>(E.fov);
  T *__restrict__ tau = static_cast<T *>(E.tau);
  T *__restrict__ taut = static_cast<T *>(E.taut);
  const int o = E.o, v = E.v;
  const int64_t vv = int64_t(v) * v, total = int64_t(o) * o * vv;
  double er = 0.0, ei = 0.0;
  const int64_t e1 = std::min<int64_t>(total, (bid + 1) * CH_TAU);
  for (int64_t e = bid * CH_TAU + threadIdx.x; e < e1; e += RED_THREADS) {
    T x = t2[e];
    if (t1 != nullptr) {
      const int b = e % v, a = (e / v) % v;
      const int64_t ij = e / vv;
      const int j = ij % o, i = ij / o;
      const T p = sub(mul(t1[i * v + a], t1[j * v + b]), mul(t1[i * v + b], t1[j * v + a]));
      const T full = add(x, p), half = add(x, sc(0.5, p));
      tau[e] = full;
      taut[e] = half;
      x = full;
    }
    const T w = mul(oovv[e], x);
    er += re(w);
    ei += im(w);
  }
  er = 0.25 * er;
  ei = 0.25 * ei;
  if (bid == 0 && t1 != nullptr) {
    for (int e = threadIdx.x; e < o * v; e += RED_THREADS) {
      const T w = mul(fov[e], t1[e]);
      er += re(w);
      ei += im(w);
    }
  }
  const double sr = block_sum(er, sh);
  const double si = block_sum(ei, sh);
  if (threadIdx.x == 0) {
    E.partials[2 * bid] = sr;
    E.partials[2 * bid + 1] = si;
  }
}

// ------------------------------------------- doubles residual + Jacobi ------
// R_ijab = XP + (Xij_ijab - Xij_jiab) + (Xab_ijab - Xab_ijba)
//        + ((Xr_ijab - Xr_jiab) - (Xr_ijba - Xr_jiba))
// evaluated once per canonical element (i < j, a < b) and written to its
// four images R_ijab = -R_jiab = -R_ijba = R_jiba; the diagonals i == j and
// a == b are exact zeros.  The amplitudes are updated the same way, so the
// result is bitwise antisymmetric whatever the rounding of the intermediates.
// One workgroup per (i <= j, 32-tile A <= 32-tile B); the (b,a)-ordered
// operands are read coalesced into padded LDS tiles, and the (b,a)-ordered
// images are written coalesced through an LDS tile.
__device__ __forceinline__ void tri_decode(int64_t k, int n, int &i, int &j) {
  int r = 0;
  while (k >= n - r) {
    k -= n - r;
    ++r;
  }
  i = r;
  j = r + int(k);
}

template <class T>
__device__ __forceinline__ void asm_body(const AsmEntry &E, int64_t bid) {
  const R2Args &p = E.a;
  const T *__restrict__ XP = static_cast<const T *>(E.XP);
  const T *__restrict__ Xij = static_cast<const T *>(E.Xij);
  const T *__restrict__ Xab = static_cast<const T *>(E.Xab);
  const T *__restrict__ Xr = static_cast<const T *>(E.Xr);
  T *__restrict__ R = static_cast<T *>(E.R);
  T *__restrict__ t2 = static_cast<T *>(E.t2);
  double *partials = E.partials;
  __shared__ T sab[32][33], sr_ij[32][33], sr_ji[32][33], sv[32][33], st[32][33];
  __shared__ double sh[RED_THREADS];
  const int o = p.o, v = p.v;
  const int tiles = (v + 31) / 32;
  const int64_t ntp = int64_t(tiles) * (tiles + 1) / 2;
  int ta, tb, i, j;
  tri_decode(bid % ntp, tiles, ta, tb);
  tri_decode(bid / ntp, o, i, j);
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  const int64_t vv = int64_t(v) * v;
  const int64_t base_ij = (int64_t(i) * o + j) * vv, base_ji = (int64_t(j) * o + i) * vv;
  const int a0 = ta * 32, b0 = tb * 32;
  const bool diag_tile = (ta == tb);
  double nrm = 0.0;
  if (i == j) {
    // the whole (i,i) block is zero: write both tile orientations
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int aa = a0 + ty + 8 * k, bb = b0 + tx;
      if (aa < v && bb < v) {
        if (R != nullptr) {
          R[base_ij + int64_t(aa) * v + bb] = zero<T>();
          R[base_ij + int64_t(bb) * v + aa] = zero<T>();
        }
      }
    }
  } else {
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int bb = b0 + ty + 8 * k, aa = a0 + tx;
      if (bb < v && aa < v) {
        const int64_t off = int64_t(bb) * v + aa;
        sab[ty + 8 * k][tx] = Xab[base_ij + off];
        sr_ij[ty + 8 * k][tx] = Xr[base_ij + off];
        sr_ji[ty + 8 * k][tx] = Xr[base_ji + off];
      }
    }
    __syncthreads();
    const double *d_oo = p.fdiag_o, *d_vv = p.fdiag_v;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int la = ty + 8 * k, lb = tx;
      const int aa = a0 + la, bb = b0 + lb;
      const bool canon = aa < v && bb < v && (!diag_tile || aa < bb);
      T r = zero<T>(), tn = zero<T>();
      if (canon) {
        const int64_t e = base_ij + int64_t(aa) * v + bb, e_ji = base_ji + int64_t(aa) * v + bb;
        const T g_ij = sub(Xij[e], Xij[e_ji]);
        const T g_ab = sub(Xab[e], sab[lb][la]);
        const T g_r = sub(sub(Xr[e], Xr[e_ji]), sub(sr_ij[lb][la], sr_ji[lb][la]));
        r = add(add(add(XP[e], g_ij), g_ab), g_r);
        nrm += 4.0 * abs2(r);
        if (R != nullptr) {
          R[e] = r;
          R[e_ji] = sc(-1.0, r);
        }
        if (t2 != nullptr) {
          double D;
          if (p.dressed) {
            const T *Fo = static_cast<const T *>(p.Fo), *Fv = static_cast<const T *>(p.Fv);
            D = (re(Fo[int64_t(i) * o + i]) + re(Fo[int64_t(j) * o + j])) -
                (re(Fv[int64_t(aa) * v + aa]) + re(Fv[int64_t(bb) * v + bb]));
          } else {
            D = (d_oo[i] + d_oo[j]) - (d_vv[aa] + d_vv[bb]);
          }
          tn = add(t2[e], sc(1.0 / (D - p.shift), r));
          t2[e] = tn;
          t2[e_ji] = sc(-1.0, tn);
        }
      } else if (diag_tile && aa == bb && aa < v) {
        const int64_t e = base_ij + int64_t(aa) * v + bb, e_ji = base_ji + int64_t(aa) * v + bb;
        if (R != nullptr) {
          R[e] = zero<T>();
          R[e_ji] = zero<T>();
        }
      }
      sv[la][lb] = r;
      st[la][lb] = tn;
    }
    __syncthreads();
    // images with (b, a) order: rows b, columns a (coalesced along a)
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int lb = ty + 8 * k, la = tx;
      const int aa = a0 + la, bb = b0 + lb;
      if (aa < v && bb < v && (!diag_tile || aa < bb)) {
        const int64_t e = base_ij + int64_t(bb) * v + aa, e_ji = base_ji + int64_t(bb) * v + aa;
        if (R != nullptr) {
          R[e] = sc(-1.0, sv[la][lb]);
          R[e_ji] = sv[la][lb];
        }
        if (t2 != nullptr) {
          t2[e] = sc(-1.0, st[la][lb]);
          t2[e_ji] = st[la][lb];
        }
      }
    }
  }
  const double s = block_sum(nrm, sh);
  if (threadIdx.x == 0) partials[bid] = s;
}


// ----------------------------------------------------------------- singles --
// R1 already assembled: norm partial and optional update.
template <class T>
__device__ __forceinline__ void r1_body(const R1Entry &E) {
  __shared__ double sh[RED_THREADS];
  const T *__restrict__ R1 = static_cast<const T *>(E.R1);
  T *__restrict__ t1 = static_cast<T *>(E.t1);
  const T *Fo = static_cast<const T *>(E.Fo), *Fv = static_cast<const T *>(E.Fv);
  const int o = E.o, v = E.v;
  double nrm = 0.0;
  for (int e = threadIdx.x; e < o * v; e += RED_THREADS) {
    const int i = e / v, a = e % v;
    const T r = R1[e];
    nrm += abs2(r);
    const double D = E.dressed ? re(Fo[int64_t(i) * o + i]) - re(Fv[int64_t(a) * v + a])
                               : E.d_oo[i] - E.d_vv[a];
    if (t1 != nullptr) t1[e] = add(t1[e], sc(1.0 / (D - E.shift), r));
  }
  const double s = block_sum(nrm, sh);
  if (threadIdx.x == 0) E.partial[0] = s;
}

// scalars[0] = ||R||, scalars[1..2] = E (re, im); fixed summation order.
template <class T>
__device__ __forceinline__ void pair_body(const PairEntry &E, int64_t bid) {
  const T *__restrict__ src = static_cast<const T *>(E.src);
  T *__restrict__ dst = static_cast<T *>(E.dst);
  const int64_t total = E.nP * E.nQ;
  const int64_t e1 = std::min<int64_t>(total, (bid + 1) * CH);
  for (int64_t e = bid * CH + threadIdx.x; e < e1; e += 256) {
    const int64_t P = e / E.nQ, Q = e % E.nQ;
    const int r0 = E.rows[2 * P], r1 = E.rows[2 * P + 1], c0 = E.cols[2 * Q], c1 = E.cols[2 * Q + 1];
    const int64_t q = ((int64_t(r0) * E.n1 + r1) * E.n2 + c0) * E.n3 + c1;
    const int64_t pe = P * E.ldq + Q;  // packed side
    if (E.mode == 0) dst[pe] = src[q];
    else if (E.mode == 1) dst[q] = add(dst[q], src[pe]);
    else dst[q] = src[pe];
  }
}

constexpr int64_t CH_T3 = 1024;

// Triples: R3 = sum over permutations (s of ijk, r of abc) of
// sign(s) sign(r) Y3[s(ijk)][r(abc)].
template <class T>
__device__ __forceinline__ void t3_body(const T3Entry &E, int64_t bid) {
  __shared__ double sh[RED_THREADS];
  const int o = E.o, v = E.v;
  const int64_t oo = int64_t(o) * o, vvv = int64_t(v) * v * v, total = oo * o * vvv;
  const T *__restrict__ Y = static_cast<const T *>(E.Y3);
  T *__restrict__ R = static_cast<T *>(E.R3);
  T *__restrict__ t3 = static_cast<T *>(E.t3);
  // the six permutations of three slots and their signs
  const int P[6][3] = {{0, 1, 2}, {1, 2, 0}, {2, 0, 1}, {1, 0, 2}, {0, 2, 1}, {2, 1, 0}};
  const double S[6] = {1, 1, 1, -1, -1, -1};
  double nrm = 0.0;
  const int64_t e1 = std::min<int64_t>(total, (bid + 1) * CH_T3);
  for (int64_t e = bid * CH_T3 + threadIdx.x; e < e1; e += RED_THREADS) {
    int64_t r = e;
    const int c = int(r % v); r /= v;
    const int b = int(r % v); r /= v;
    const int a = int(r % v); r /= v;
    const int k = int(r % o); r /= o;
    const int j = int(r % o); r /= o;
    const int i = int(r);
    T val = zero<T>();
    if (i != j && j != k && i != k && a != b && b != c && a != c) {
      const int h[3] = {i, j, k}, q[3] = {a, b, c};
      for (int s1 = 0; s1 < 6; ++s1) {
        const int64_t hb = ((int64_t(h[P[s1][0]]) * o + h[P[s1][1]]) * o + h[P[s1][2]]) * vvv;
        for (int s2 = 0; s2 < 6; ++s2) {
          const int64_t idx = hb + (int64_t(q[P[s2][0]]) * v + q[P[s2][1]]) * v + q[P[s2][2]];
          val = add(val, sc(S[s1] * S[s2], Y[idx]));
        }
      }
      nrm += abs2(val);
      if (t3 != nullptr) {
        const double D = E.d_oo[i] + E.d_oo[j] + E.d_oo[k] - E.d_vv[a] - E.d_vv[b] - E.d_vv[c] - E.shift;
        t3[e] = add(t3[e], sc(1.0 / D, val));
      }
    } else if (t3 != nullptr) {
      t3[e] = zero<T>();
    }
    if (R != nullptr) R[e] = val;
  }
  const double tot = block_sum(nrm, sh);
  if (threadIdx.x == 0) E.partials[bid] = tot;
}

__device__ __forceinline__ void fin_body(const FinEntry &E) {
  __shared__ double sh[RED_THREADS];
  double a = 0.0, b = 0.0, c = 0.0;
  for (int k = threadIdx.x; k < E.ne; k += RED_THREADS) {
    a += E.epart[2 * k];
    b += E.epart[2 * k + 1];
  }
  for (int k = threadIdx.x; k < E.nn; k += RED_THREADS) c += E.n2part[k];
  for (int k = threadIdx.x; k < E.nn3; k += RED_THREADS) c += E.n3part[k];
  const double sa = block_sum(a, sh), sb = block_sum(b, sh), scn = block_sum(c, sh);
  if (threadIdx.x == 0) {
    const double n2 = scn + (E.n1part ? E.n1part[0] : 0.0);
    E.scalars[0] = sqrt(n2);
    E.scalars[1] = sa;
    E.scalars[2] = sb;
  }
}

// Fock diagonals (real parts) into contiguous arrays.
template <class T>
__global__ void fock_diag_kernel(int o, int v, const T *foo, const T *fvv, double *d_oo, double *d_vv) {
  for (int e = threadIdx.x + blockIdx.x * blockDim.x; e < o + v; e += blockDim.x * gridDim.x) {
    if (e < o) d_oo[e] = re(foo[int64_t(e) * o + e]);
    else d_vv[e - o] = re(fvv[int64_t(e - o) * v + (e - o)]);
  }
}

// ------------------------------------------------------- kernels (both forms)
#define CC_EW_KERNELS(NAME, ENTRY, BODY)                                                          \
  template <class T>                                                                              \
  __global__ __launch_bounds__(256) void k_##NAME(ENTRY e) {                                     \
    BODY<T>(e, blockIdx.x);                                                                       \
  }                                                                                               \
  template <class T>                                                                              \
  __global__ __launch_bounds__(256) void g_##NAME(const ENTRY *__restrict__ es,                  \
                                                  const int64_t *__restrict__ off, int n) {      \
    const int b = group_find(off, n, blockIdx.x);                                                 \
    BODY<T>(es[b], int64_t(blockIdx.x) - off[b]);                                                 \
  }

CC_EW_KERNELS(perm_flat, PermEntry, perm_flat_body)
CC_EW_KERNELS(perm_tiled, PermEntry, perm_tiled_body)
CC_EW_KERNELS(outer, OuterEntry, outer_body)
CC_EW_KERNELS(fill, FillEntry, fill_body)
CC_EW_KERNELS(splitk, SplitkEntry, splitk_body)
CC_EW_KERNELS(tau, TauEntry, tau_body)
CC_EW_KERNELS(asm, AsmEntry, asm_body)
CC_EW_KERNELS(t3, T3Entry, t3_body)
CC_EW_KERNELS(pair, PairEntry, pair_body)

template <class T>
__global__ __launch_bounds__(RED_THREADS) void k_r1(R1Entry e) { r1_body<T>(e); }
template <class T>
__global__ __launch_bounds__(RED_THREADS) void g_r1(const R1Entry *__restrict__ es) { r1_body<T>(es[blockIdx.x]); }
__global__ __launch_bounds__(RED_THREADS) void k_fin(FinEntry e) { fin_body(e); }
__global__ __launch_bounds__(RED_THREADS) void g_fin(const FinEntry *__restrict__ es) { fin_body(es[blockIdx.x]); }

int64_t chunks(int64_t n, int64_t ch) { return std::max<int64_t>(1, (n + ch - 1) / ch); }

}  // namespace

// ============================================================ host: entries ==
PermEntry make_perm_entry(const PermDesc &d, const void *in, void *out) {
  PermEntry e{};
  PermArgs &p = e.p;
  // Drop dims of extent 1 and merge each dim into the one outside it when it
  // continues that one in both tensors (outer stride = inner stride x inner
  // extent): the same element map over fewer, longer dims.
  int64_t total = 1;
  p.rank = 0;
  for (int i = 0; i < d.rank; ++i) {
    const int64_t n = d.out_dims[i];
    total *= n;
    if (n == 1) continue;
    const int r = p.rank;
    if (r > 0 && p.istr[r - 1] == d.in_strides[i] * n && p.ostr[r - 1] == d.out_strides[i] * n) {
      p.dims[r - 1] *= n;
      p.istr[r - 1] = d.in_strides[i];
      p.ostr[r - 1] = d.out_strides[i];
    } else {
      p.dims[r] = n;
      p.istr[r] = d.in_strides[i];
      p.ostr[r] = d.out_strides[i];
      p.rank = r + 1;
    }
  }
  if (p.rank == 0) {  // one element
    p.rank = 1;
    p.dims[0] = 1;
    p.istr[0] = p.ostr[0] = 0;
  }
  p.total = total;
  p.alpha = d.alpha;
  p.beta = d.beta;
  p.conj = d.conj;
  int d_o = -1, d_i = -1;
  for (int i = 0; i < p.rank; ++i) {
    if (p.ostr[i] == 1 && p.dims[i] > 1) d_o = i;
    if (p.istr[i] == 1 && p.dims[i] > 1) d_i = i;
  }
  e.in = in;
  e.out = out;
  if (total == 0) {
    e.units = 0;
    return e;
  }
  if (d_o < 0 || d_i < 0 || d_o == d_i) {
    e.tiled = 0;
    e.units = chunks(total, CH);
  } else {
    e.tiled = 1;
    p.d_o = d_o;
    p.d_i = d_i;
    p.nrest = 0;
    p.n_rest_total = 1;
    for (int i = 0; i < p.rank; ++i) {
      if (i == d_o || i == d_i) continue;
      p.rest_dims[p.nrest] = p.dims[i];
      p.rest_istr[p.nrest] = p.istr[i];
      p.rest_ostr[p.nrest] = p.ostr[i];
      p.n_rest_total *= p.dims[i];
      ++p.nrest;
    }
    // 32 x 32, or a narrow, long tile when one of the two fast dims is short
    // (the occupied index of small systems) instead of a mostly empty one
    auto lg = [](int64_t n) {  // log2 of the smallest power of two >= n, in [2, 8]
      int l = 2;
      while (l < 8 && (int64_t(1) << l) < n) ++l;
      return l;
    };
    const int li = lg(p.dims[d_i]), lo = lg(p.dims[d_o]);
    p.lti = li < 5 ? li : (lo < 5 ? 10 - lo : 5);
    p.tiles_i = (p.dims[d_i] + (1 << p.lti) - 1) >> p.lti;
    p.tiles_o = (p.dims[d_o] + (1 << (10 - p.lti)) - 1) >> (10 - p.lti);
    e.units = p.n_rest_total * p.tiles_o * p.tiles_i;
  }
  return e;
}

OuterEntry make_outer_entry(const OuterArgs &a, const void *A, const void *B, void *C) {
  OuterEntry e{};
  e.a = a;
  e.A = A;
  e.B = B;
  e.C = C;
  e.total = 1;
  for (int i = 0; i < a.rank; ++i) e.total *= a.dims[i];
  e.units = e.total ? chunks(e.total, CH) : 0;
  return e;
}

FillEntry make_fill_entry(void *p, int64_t n) { return FillEntry{p, n, n > 0 ? chunks(n, CH) : 0}; }

SplitkEntry make_splitk_entry(const void *ws, int split, int64_t M, int64_t N, void *C, int64_t ldc, double alpha,
                              double beta) {
  int lanes = 1;
  while (lanes < 16 && 2 * lanes <= split) lanes *= 2;
  return SplitkEntry{ws, split, lanes, M, N, C, ldc, alpha, beta, M * N > 0 ? chunks(M * N, 256 / lanes) : 0};
}

int64_t tau_units(int o, int v) { return chunks(int64_t(o) * o * v * v, CH_TAU); }

TauEntry make_tau_entry(int o, int v, const void *t1, const void *t2, const void *oovv, const void *fov,
                        void *tau, void *taut, double *partials) {
  return TauEntry{o, v, t1, t2, oovv, fov, tau, taut, partials, tau_units(o, v)};
}

int64_t t3_units(int o, int v) { return chunks(int64_t(o) * o * o * v * v * v, CH_T3); }

PairEntry make_pair_entry(const void *src, void *dst, const int *rows, const int *cols, int64_t nP, int64_t nQ,
                          int64_t ldq, int64_t n1, int64_t n2, int64_t n3, int mode) {
  CC_REQUIRE(ldq >= nQ, -1, "pair: row stride below the row length");
  return PairEntry{src, dst, rows, cols, nP, nQ, ldq, n1, n2, n3, mode, nP * nQ > 0 ? chunks(nP * nQ, CH) : 0};
}

int64_t asm_units(int o, int v) {
  const int64_t tiles = (v + 31) / 32;
  return (int64_t(o) * (o + 1) / 2) * (tiles * (tiles + 1) / 2);
}

AsmEntry make_asm_entry(const R2Args &a, const void *XP, const void *Xij, const void *Xab, const void *Xr, void *R,
                        void *t2, double *partials) {
  return AsmEntry{a, XP, Xij, Xab, Xr, R, t2, partials, asm_units(a.o, a.v)};
}

// ========================================================= host: launches ==
#define CC_LAUNCH1(KER, E, UNITS, CPLX, S)                                                          \
  do {                                                                                            \
    if ((UNITS) <= 0) return;                                                                     \
    CC_REQUIRE((UNITS) < (int64_t(1) << 31), -1, "grid too large");                               \
    if (CPLX) hipLaunchKernelGGL(KER<double2>, dim3(UNITS), dim3(256), 0, S, E);                  \
    else hipLaunchKernelGGL(KER<double>, dim3(UNITS), dim3(256), 0, S, E);                        \
    CC_HIP_CHECK(hipGetLastError());                                                              \
  } while (0)

#define CC_LAUNCHG(KER, E, OFF, N, BLOCKS, CPLX, S)                                                 \
  do {                                                                                            \
    if ((BLOCKS) <= 0) return;                                                                    \
    CC_REQUIRE((BLOCKS) < (int64_t(1) << 31), -1, "grid too large");                              \
    if (CPLX) hipLaunchKernelGGL(KER<double2>, dim3(BLOCKS), dim3(256), 0, S, E, OFF, N);         \
    else hipLaunchKernelGGL(KER<double>, dim3(BLOCKS), dim3(256), 0, S, E, OFF, N);               \
    CC_HIP_CHECK(hipGetLastError());                                                              \
  } while (0)

void launch_perm(const PermEntry &e, bool cplx, hipStream_t s) {
  if (e.tiled) CC_LAUNCH1(k_perm_tiled, e, e.units, cplx, s);
  else CC_LAUNCH1(k_perm_flat, e, e.units, cplx, s);
}
void launch_outer(const OuterEntry &e, bool cplx, hipStream_t s) { CC_LAUNCH1(k_outer, e, e.units, cplx, s); }
void launch_fill(const FillEntry &e, bool cplx, hipStream_t s) { CC_LAUNCH1(k_fill, e, e.units, cplx, s); }
void launch_splitk(const SplitkEntry &e, bool cplx, hipStream_t s) { CC_LAUNCH1(k_splitk, e, e.units, cplx, s); }
void launch_tau(const TauEntry &e, bool cplx, hipStream_t s) { CC_LAUNCH1(k_tau, e, e.units, cplx, s); }
void launch_asm(const AsmEntry &e, bool cplx, hipStream_t s) { CC_LAUNCH1(k_asm, e, e.units, cplx, s); }
void launch_t3(const T3Entry &e, bool cplx, hipStream_t s) { CC_LAUNCH1(k_t3, e, e.units, cplx, s); }
void launch_pair(const PairEntry &e, bool cplx, hipStream_t s) { CC_LAUNCH1(k_pair, e, e.units, cplx, s); }
void launch_r1(const R1Entry &e, bool cplx, hipStream_t s) {
  if (cplx) hipLaunchKernelGGL(k_r1<double2>, dim3(1), dim3(RED_THREADS), 0, s, e);
  else hipLaunchKernelGGL(k_r1<double>, dim3(1), dim3(RED_THREADS), 0, s, e);
  CC_HIP_CHECK(hipGetLastError());
}
void launch_fin(const FinEntry &e, hipStream_t s) {
  hipLaunchKernelGGL(k_fin, dim3(1), dim3(RED_THREADS), 0, s, e);
  CC_HIP_CHECK(hipGetLastError());
}

void launch_perm_grouped(const PermEntry *e, const int64_t *off, int n, int64_t blocks, bool tiled, bool cplx,
                         hipStream_t s) {
  if (tiled) CC_LAUNCHG(g_perm_tiled, e, off, n, blocks, cplx, s);
  else CC_LAUNCHG(g_perm_flat, e, off, n, blocks, cplx, s);
}
void launch_outer_grouped(const OuterEntry *e, const int64_t *off, int n, int64_t blocks, bool cplx, hipStream_t s) {
  CC_LAUNCHG(g_outer, e, off, n, blocks, cplx, s);
}
void launch_pair_grouped(const PairEntry *e, const int64_t *off, int n, int64_t blocks, bool cplx, hipStream_t s) {
  CC_LAUNCHG(g_pair, e, off, n, blocks, cplx, s);
}
void launch_fill_grouped(const FillEntry *e, const int64_t *off, int n, int64_t blocks, bool cplx, hipStream_t s) {
  CC_LAUNCHG(g_fill, e, off, n, blocks, cplx, s);
}
void launch_splitk_grouped(const SplitkEntry *e, const int64_t *off, int n, int64_t blocks, bool cplx,
                           hipStream_t s) {
  CC_LAUNCHG(g_splitk, e, off, n, blocks, cplx, s);
}
void launch_tau_grouped(const TauEntry *e, const int64_t *off, int n, int64_t blocks, bool cplx, hipStream_t s) {
  CC_LAUNCHG(g_tau, e, off, n, blocks, cplx, s);
}
void launch_asm_grouped(const AsmEntry *e, const int64_t *off, int n, int64_t blocks, bool cplx, hipStream_t s) {
  CC_LAUNCHG(g_asm, e, off, n, blocks, cplx, s);
}
void launch_r1_grouped(const R1Entry *e, int n, bool cplx, hipStream_t s) {
  if (n <= 0) return;
  if (cplx) hipLaunchKernelGGL(g_r1<double2>, dim3(n), dim3(RED_THREADS), 0, s, e);
  else hipLaunchKernelGGL(g_r1<double>, dim3(n), dim3(RED_THREADS), 0, s, e);
  CC_HIP_CHECK(hipGetLastError());
}
void launch_fin_grouped(const FinEntry *e, int n, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(g_fin, dim3(n), dim3(RED_THREADS), 0, s, e);
  CC_HIP_CHECK(hipGetLastError());
}

// ====================================================== host: conveniences ==
void permute_f64(const PermDesc &d, const void *in, void *out, hipStream_t s) {
  launch_perm(make_perm_entry(d, in, out), false, s);
}
void permute_c128(const PermDesc &d, const void *in, void *out, hipStream_t s) {
  launch_perm(make_perm_entry(d, in, out), true, s);
}
void outer_acc(const OuterArgs &a, bool cplx, const void *A, const void *B, void *C, hipStream_t s) {
  launch_outer(make_outer_entry(a, A, B, C), cplx, s);
}
void fill_zero(void *p, int64_t n_elems, bool cplx, hipStream_t s) {
  launch_fill(make_fill_entry(p, n_elems), cplx, s);
}
void splitk_reduce(bool cplx, const void *ws, int split, int64_t M, int64_t N, void *C, int64_t ldc,
                   double alpha, double beta, hipStream_t s) {
  launch_splitk(make_splitk_entry(ws, split, M, N, C, ldc, alpha, beta), cplx, s);
}
void fock_diag(bool cplx, int o, int v, const void *foo, const void *fvv, double *d_oo, double *d_vv,
               hipStream_t s) {
  if (cplx)
    hipLaunchKernelGGL(fock_diag_kernel<double2>, dim3(1), dim3(256), 0, s, o, v, (const double2 *)foo,
                       (const double2 *)fvv, d_oo, d_vv);
  else
    hipLaunchKernelGGL(fock_diag_kernel<double>, dim3(1), dim3(256), 0, s, o, v, (const double *)foo,
                       (const double *)fvv, d_oo, d_vv);
  CC_HIP_CHECK(hipGetLastError());
}

}  // namespace ccmi
