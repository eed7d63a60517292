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

// Block-wide sum in a fixed order (tree over LDS); result in thread 0.
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

// ------------------------------------------------------------- permutation --
struct PermArgs {
  int rank;
  int64_t dims[kMaxRank];
  int64_t istr[kMaxRank];
  int64_t ostr[kMaxRank];
  double alpha, beta;
  int conj;
  int d_o, d_i;          // tiled dims: output unit-stride dim and input unit-stride dim
  int64_t rest_dims[kMaxRank];  // dims other than d_o, d_i (rank-2 entries used)
  int64_t rest_istr[kMaxRank], rest_ostr[kMaxRank];
  int nrest;
  int64_t n_rest_total, tiles_o, tiles_i;
};

// Plain path: input and output share their unit-stride dimension.
template <class T>
__global__ __launch_bounds__(256) void permute_flat_kernel(PermArgs p, const T *__restrict__ in,
                                                           T *__restrict__ out, int64_t total) {
  for (int64_t e = blockIdx.x * int64_t(256) + threadIdx.x; e < total;
       e += int64_t(gridDim.x) * 256) {
    int64_t rem = e, io = 0, oo = 0;
    for (int d = p.rank - 1; d >= 0; --d) {
      const int64_t x = rem % p.dims[d];
      rem /= p.dims[d];
      io += x * p.istr[d];
      oo += x * p.ostr[d];
    }
    T v = in[io];
    if (p.conj) v = cj(v);
    v = sc(p.alpha, v);
    if (p.beta != 0.0) v = add(v, sc(p.beta, out[oo]));
    out[oo] = v;
  }
}

// Tiled path: 32x32 tile over (output unit-stride dim, input unit-stride dim),
// read coalesced along the input's fast dim, written coalesced along the
// output's fast dim through a padded LDS tile.
template <class T>
__global__ __launch_bounds__(256) void permute_tiled_kernel(PermArgs p, const T *__restrict__ in,
                                                            T *__restrict__ out) {
  __shared__ T tile[32][33];
  int64_t b = blockIdx.x;
  const int64_t ti = b % p.tiles_i; b /= p.tiles_i;
  const int64_t to = b % p.tiles_o; b /= p.tiles_o;
  int64_t ib = 0, ob = 0;
  for (int d = p.nrest - 1; d >= 0; --d) {
    const int64_t x = b % p.rest_dims[d];
    b /= p.rest_dims[d];
    ib += x * p.rest_istr[d];
    ob += x * p.rest_ostr[d];
  }
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  const int64_t Do = p.dims[p.d_o], Di = p.dims[p.d_i];
  const int64_t i0 = ti * 32, o0 = to * 32;
  // load: x runs along the input's unit-stride dim
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int64_t xi = i0 + tx, xo = o0 + ty + 8 * k;
    if (xi < Di && xo < Do) tile[ty + 8 * k][tx] = in[ib + xi * p.istr[p.d_i] + xo * p.istr[p.d_o]];
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int64_t xo = o0 + tx, xi = i0 + ty + 8 * k;
    if (xi < Di && xo < Do) {
      T v = tile[tx][ty + 8 * k];
      if (p.conj) v = cj(v);
      v = sc(p.alpha, v);
      T *o = out + ob + xo * p.ostr[p.d_o] + xi * p.ostr[p.d_i];
      if (p.beta != 0.0) v = add(v, sc(p.beta, *o));
      *o = v;
    }
  }
}

template <class T>
void permute_impl(const PermDesc &d, const void *in, void *out, hipStream_t s) {
  PermArgs p{};
  p.rank = d.rank;
  int64_t total = 1;
  for (int i = 0; i < d.rank; ++i) {
    p.dims[i] = d.out_dims[i];
    p.istr[i] = d.in_strides[i];
    p.ostr[i] = d.out_strides[i];
    total *= d.out_dims[i];
  }
  if (total == 0) return;
  p.alpha = d.alpha;
  p.beta = d.beta;
  p.conj = d.conj;
  int d_o = -1, d_i = -1;
  for (int i = 0; i < d.rank; ++i) {
    if (p.ostr[i] == 1 && p.dims[i] > 1) d_o = i;
    if (p.istr[i] == 1 && p.dims[i] > 1) d_i = i;
  }
  const T *ip = static_cast<const T *>(in);
  T *op = static_cast<T *>(out);
  if (d_o < 0 || d_i < 0 || d_o == d_i) {
    const int64_t blocks = std::min<int64_t>((total + 255) / 256, 65536);
    hipLaunchKernelGGL(permute_flat_kernel<T>, dim3(blocks), dim3(256), 0, s, p, ip, op, total);
  } else {
    p.d_o = d_o;
    p.d_i = d_i;
    p.nrest = 0;
    p.n_rest_total = 1;
    for (int i = 0; i < d.rank; ++i) {
      if (i == d_o || i == d_i) continue;
      p.rest_dims[p.nrest] = p.dims[i];
      p.rest_istr[p.nrest] = p.istr[i];
      p.rest_ostr[p.nrest] = p.ostr[i];
      p.n_rest_total *= p.dims[i];
      ++p.nrest;
    }
    p.tiles_o = (p.dims[d_o] + 31) / 32;
    p.tiles_i = (p.dims[d_i] + 31) / 32;
    const int64_t blocks = p.n_rest_total * p.tiles_o * p.tiles_i;
    CC_REQUIRE(blocks < (int64_t(1) << 31), -1, "permute: grid too large");
    hipLaunchKernelGGL(permute_tiled_kernel<T>, dim3(blocks), dim3(256), 0, s, p, ip, op);
  }
  CC_HIP_CHECK(hipGetLastError());
}

// ------------------------------------------------------------ outer product --
// C[I] += alpha * A[sum_d I_d sa_d] * B[sum_d I_d sb_d]  (rank <= 4)
template <class T>
__global__ __launch_bounds__(256) void outer_kernel(OuterArgs p, const T *__restrict__ A,
                                                    const T *__restrict__ B, T *__restrict__ C,
                                                    int64_t total) {
  for (int64_t e = blockIdx.x * int64_t(256) + threadIdx.x; e < total;
       e += int64_t(gridDim.x) * 256) {
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

// ---------------------------------------------------------- split-K sum --
// C = alpha * sum_s W[s] + beta * C, s in increasing order (deterministic).
template <class T>
__global__ __launch_bounds__(256) void splitk_kernel(const T *__restrict__ W, int split, int64_t M,
                                                     int64_t N, T *__restrict__ C, int64_t ldc,
                                                     double alpha, double beta) {
  const int64_t total = M * N;
  for (int64_t e = blockIdx.x * int64_t(256) + threadIdx.x; e < total;
       e += int64_t(gridDim.x) * 256) {
    T acc = W[e];
    for (int k = 1; k < split; ++k) acc = add(acc, W[int64_t(k) * total + e]);
    const int64_t m = e / N, n = e % N;
    T v = sc(alpha, acc);
    if (beta != 0.0) v = add(v, sc(beta, C[m * ldc + n]));
    C[m * ldc + n] = v;
  }
}

// ------------------------------------------------------------------- fill --
template <class T>
__global__ __launch_bounds__(256) void fill_kernel(T *__restrict__ p, T val, int64_t n) {
  for (int64_t e = blockIdx.x * int64_t(256) + threadIdx.x; e < n; e += int64_t(gridDim.x) * 256)
    p[e] = val;
}

// --------------------------------------------------- tau + energy partials --
// tau = t2 + (t_i^a t_j^b - t_i^b t_j^a), taut = t2 + 1/2 (...),
// energy partial: 1/4 sum <ij||ab> tau_ij^ab  (+ sum f_ia t_i^a by block 0).
template <class T>
__global__ __launch_bounds__(RED_THREADS) void tau_energy_kernel(
    int o, int v, const T *__restrict__ t1, const T *__restrict__ t2, const T *__restrict__ oovv,
    const T *__restrict__ fov, T *__restrict__ tau, T *__restrict__ taut, double *partials) {
  __shared__ double sh[RED_THREADS];
  const int64_t vv = int64_t(v) * v, total = int64_t(o) * o * vv;
  double er = 0.0, ei = 0.0;
  for (int64_t e = blockIdx.x * int64_t(RED_THREADS) + threadIdx.x; e < total;
       e += int64_t(gridDim.x) * RED_THREADS) {
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
  if (blockIdx.x == 0 && t1 != nullptr) {
    for (int e = threadIdx.x; e < o * v; e += RED_THREADS) {
      const T w = mul(fov[e], t1[e]);
      er += re(w);
      ei += im(w);
    }
  }
  const double sr = block_sum(er, sh);
  const double si = block_sum(ei, sh);
  if (threadIdx.x == 0) {
    partials[2 * blockIdx.x] = sr;
    partials[2 * blockIdx.x + 1] = si;
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
__global__ __launch_bounds__(256) void r2_assemble_kernel(R2Args p, const T *__restrict__ XP,
                                                          const T *__restrict__ Xij,
                                                          const T *__restrict__ Xab,
                                                          const T *__restrict__ Xr,
                                                          T *__restrict__ R, T *__restrict__ t2,
                                                          double *partials) {
  __shared__ T sab[32][33], sr_ij[32][33], sr_ji[32][33], sv[32][33], st[32][33];
  __shared__ double sh[RED_THREADS];
  const int o = p.o, v = p.v;
  const int tiles = (v + 31) / 32;
  const int64_t ntp = int64_t(tiles) * (tiles + 1) / 2;
  int ta, tb, i, j;
  tri_decode(blockIdx.x % ntp, tiles, ta, tb);
  tri_decode(blockIdx.x / ntp, o, i, j);
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
  if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

// singles: R1 already assembled; norm partial and optional update
template <class T>
__global__ __launch_bounds__(RED_THREADS) void r1_update_kernel(int o, int v, const T *__restrict__ R1,
                                                                T *__restrict__ t1, const double *d_oo,
                                                                const double *d_vv, double shift,
                                                                int dressed, const T *Fo, const T *Fv,
                                                                double *partial) {
  __shared__ double sh[RED_THREADS];
  double nrm = 0.0;
  for (int e = threadIdx.x; e < o * v; e += RED_THREADS) {
    const int i = e / v, a = e % v;
    const T r = R1[e];
    nrm += abs2(r);
    const double D = dressed ? re(Fo[int64_t(i) * o + i]) - re(Fv[int64_t(a) * v + a]) : d_oo[i] - d_vv[a];
    if (t1 != nullptr) t1[e] = add(t1[e], sc(1.0 / (D - shift), r));
  }
  const double s = block_sum(nrm, sh);
  if (threadIdx.x == 0) partial[0] = s;
}

// Fock diagonals (real parts) into contiguous arrays.
template <class T>
__global__ void fock_diag_kernel(int o, int v, const T *foo, const T *fvv, double *d_oo, double *d_vv) {
  for (int e = threadIdx.x + blockIdx.x * blockDim.x; e < o + v; e += blockDim.x * gridDim.x) {
    if (e < o) d_oo[e] = re(foo[int64_t(e) * o + e]);
    else d_vv[e - o] = re(fvv[int64_t(e - o) * v + (e - o)]);
  }
}

// scalars[0] = ||R||, scalars[1..2] = E (re, im); fixed summation order.
__global__ __launch_bounds__(RED_THREADS) void finalize_kernel(const double *epart, int ne,
                                                               const double *n2part, int nn,
                                                               const double *n1part,
                                                               double *scalars) {
  __shared__ double sh[RED_THREADS];
  double a = 0.0, b = 0.0, c = 0.0;
  for (int k = threadIdx.x; k < ne; k += RED_THREADS) {
    a += epart[2 * k];
    b += epart[2 * k + 1];
  }
  for (int k = threadIdx.x; k < nn; k += RED_THREADS) c += n2part[k];
  const double sa = block_sum(a, sh), sb = block_sum(b, sh), scn = block_sum(c, sh);
  if (threadIdx.x == 0) {
    const double n2 = scn + (n1part ? n1part[0] : 0.0);
    scalars[0] = sqrt(n2);
    scalars[1] = sa;
    scalars[2] = sb;
  }
}

}  // namespace

// ================================================================ launchers ==
void permute_f64(const PermDesc &d, const void *in, void *out, hipStream_t s) {
  permute_impl<double>(d, in, out, s);
}
void permute_c128(const PermDesc &d, const void *in, void *out, hipStream_t s) {
  permute_impl<double2>(d, in, out, s);
}

void outer_acc(const OuterArgs &a, bool cplx, const void *A, const void *B, void *C, hipStream_t s) {
  int64_t total = 1;
  for (int i = 0; i < a.rank; ++i) total *= a.dims[i];
  if (total == 0) return;
  const int64_t blocks = std::min<int64_t>((total + 255) / 256, 65536);
  if (cplx)
    hipLaunchKernelGGL(outer_kernel<double2>, dim3(blocks), dim3(256), 0, s, a,
                       static_cast<const double2 *>(A), static_cast<const double2 *>(B),
                       static_cast<double2 *>(C), total);
  else
    hipLaunchKernelGGL(outer_kernel<double>, dim3(blocks), dim3(256), 0, s, a,
                       static_cast<const double *>(A), static_cast<const double *>(B),
                       static_cast<double *>(C), total);
  CC_HIP_CHECK(hipGetLastError());
}

void splitk_reduce(bool cplx, const void *ws, int split, int64_t M, int64_t N, void *C, int64_t ldc,
                   double alpha, double beta, hipStream_t s) {
  const int64_t total = M * N;
  if (total == 0) return;
  const int64_t blocks = std::min<int64_t>((total + 255) / 256, 65536);
  if (cplx)
    hipLaunchKernelGGL(splitk_kernel<double2>, dim3(blocks), dim3(256), 0, s,
                       static_cast<const double2 *>(ws), split, M, N, static_cast<double2 *>(C), ldc,
                       alpha, beta);
  else
    hipLaunchKernelGGL(splitk_kernel<double>, dim3(blocks), dim3(256), 0, s,
                       static_cast<const double *>(ws), split, M, N, static_cast<double *>(C), ldc,
                       alpha, beta);
  CC_HIP_CHECK(hipGetLastError());
}

void fill_zero(void *p, int64_t n_elems, bool cplx, hipStream_t s) {
  if (n_elems <= 0) return;
  const int64_t blocks = std::min<int64_t>((n_elems + 255) / 256, 65536);
  if (cplx)
    hipLaunchKernelGGL(fill_kernel<double2>, dim3(blocks), dim3(256), 0, s,
                       static_cast<double2 *>(p), make_double2(0.0, 0.0), n_elems);
  else
    hipLaunchKernelGGL(fill_kernel<double>, dim3(blocks), dim3(256), 0, s, static_cast<double *>(p),
                       0.0, n_elems);
  CC_HIP_CHECK(hipGetLastError());
}

int tau_energy_blocks(int o, int v) {
  const int64_t total = int64_t(o) * o * v * v;
  return int(std::max<int64_t>(1, std::min<int64_t>((total + RED_THREADS - 1) / RED_THREADS, 2048)));
}

void tau_energy(bool cplx, int o, int v, const void *t1, const void *t2, const void *oovv,
                const void *fov, void *tau, void *taut, double *partials, hipStream_t s) {
  const int blocks = tau_energy_blocks(o, v);
  if (cplx)
    hipLaunchKernelGGL(tau_energy_kernel<double2>, dim3(blocks), dim3(RED_THREADS), 0, s, o, v,
                       (const double2 *)t1, (const double2 *)t2, (const double2 *)oovv,
                       (const double2 *)fov, (double2 *)tau, (double2 *)taut, partials);
  else
    hipLaunchKernelGGL(tau_energy_kernel<double>, dim3(blocks), dim3(RED_THREADS), 0, s, o, v,
                       (const double *)t1, (const double *)t2, (const double *)oovv,
                       (const double *)fov, (double *)tau, (double *)taut, partials);
  CC_HIP_CHECK(hipGetLastError());
}

int64_t r2_assemble_blocks(int o, int v) {
  const int64_t tiles = (v + 31) / 32;
  return (int64_t(o) * (o + 1) / 2) * (tiles * (tiles + 1) / 2);
}

void r2_assemble(bool cplx, const R2Args &a, const void *XP, const void *Xij, const void *Xab,
                 const void *Xr, void *R, void *t2, double *partials, hipStream_t s) {
  const int64_t blocks = r2_assemble_blocks(a.o, a.v);
  CC_REQUIRE(blocks < (int64_t(1) << 31), -1, "r2_assemble: grid too large");
  if (cplx)
    hipLaunchKernelGGL(r2_assemble_kernel<double2>, dim3(blocks), dim3(256), 0, s, a,
                       (const double2 *)XP, (const double2 *)Xij, (const double2 *)Xab,
                       (const double2 *)Xr, (double2 *)R, (double2 *)t2, partials);
  else
    hipLaunchKernelGGL(r2_assemble_kernel<double>, dim3(blocks), dim3(256), 0, s, a,
                       (const double *)XP, (const double *)Xij, (const double *)Xab,
                       (const double *)Xr, (double *)R, (double *)t2, partials);
  CC_HIP_CHECK(hipGetLastError());
}

void r1_update(bool cplx, int o, int v, const void *R1, void *t1, const double *d_oo,
               const double *d_vv, double shift, int dressed, const void *Fo, const void *Fv,
               double *partial, hipStream_t s) {
  if (cplx)
    hipLaunchKernelGGL(r1_update_kernel<double2>, dim3(1), dim3(RED_THREADS), 0, s, o, v,
                       (const double2 *)R1, (double2 *)t1, d_oo, d_vv, shift, dressed,
                       (const double2 *)Fo, (const double2 *)Fv, partial);
  else
    hipLaunchKernelGGL(r1_update_kernel<double>, dim3(1), dim3(RED_THREADS), 0, s, o, v,
                       (const double *)R1, (double *)t1, d_oo, d_vv, shift, dressed,
                       (const double *)Fo, (const double *)Fv, partial);
  CC_HIP_CHECK(hipGetLastError());
}

void fock_diag(bool cplx, int o, int v, const void *foo, const void *fvv, double *d_oo,
               double *d_vv, hipStream_t s) {
  if (cplx)
    hipLaunchKernelGGL(fock_diag_kernel<double2>, dim3(1), dim3(256), 0, s, o, v,
                       (const double2 *)foo, (const double2 *)fvv, d_oo, d_vv);
  else
    hipLaunchKernelGGL(fock_diag_kernel<double>, dim3(1), dim3(256), 0, s, o, v,
                       (const double *)foo, (const double *)fvv, d_oo, d_vv);
  CC_HIP_CHECK(hipGetLastError());
}

void finalize_scalars(const double *epart, int ne, const double *n2part, int nn,
                      const double *n1part, double *scalars, hipStream_t s) {
  hipLaunchKernelGGL(finalize_kernel, dim3(1), dim3(RED_THREADS), 0, s, epart, ne, n2part, nn,
                     n1part, scalars);
  CC_HIP_CHECK(hipGetLastError());
}

}  // namespace ccmi
