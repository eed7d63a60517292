// Learned initial amplitudes: features, forward, backward, Adam, guess.
//
// Network (parameters FP64 in device memory, 17153 values in this order):
//   W1[128][3], b1[128], W2[128][128], b2[128], W3[1][128], b3[1]
//   g(z) = W3 relu(W2 relu(W1 z + b1) + b2) + b3,   f(z) = (g(z) - g(z~)) / 2
// where z~ is z with its first component (the scaled integral <ij||ab>)
// negated, so f is odd in <ij||ab> and the predicted t2 is antisymmetric.
// A batch of c samples is evaluated as 2c rows (the + and - branches).  The
// three dense layers are MFMA GEMMs (FP64, or FP32 MFMA with FP32
// accumulation); the elementwise parts below are FP64.
#include <cmath>
#include <string>
#include <vector>

#include "plan.hpp"

namespace ccmi {
namespace {

constexpr int HID = 128;
constexpr int64_t NPAR = HID * 3 + HID + HID * HID + HID + HID + 1;  // 17153
constexpr int64_t OFF_W1 = 0, OFF_B1 = HID * 3, OFF_W2 = OFF_B1 + HID, OFF_B2 = OFF_W2 + HID * HID,
                  OFF_W3 = OFF_B2 + HID, OFF_B3 = OFF_W3 + HID;

__device__ __forceinline__ void tri(int64_t k, int n, int &i, int &j) {
  int r = 0;
  while (k >= n - 1 - r) {
    k -= n - 1 - r;
    ++r;
  }
  i = r;
  j = r + 1 + int(k);
}

// e_ij = sum_{a<b} <ij||ab>^2 / D_ij^ab for every i < j (one workgroup each).
__global__ __launch_bounds__(256) void pair_energy_kernel(int o, int v, const double *__restrict__ oovv,
                                                          const double *__restrict__ d_oo,
                                                          const double *__restrict__ d_vv,
                                                          double *__restrict__ epair) {
  __shared__ double sh[256];
  int i, j;
  tri(blockIdx.x, o, i, j);
  const int64_t base = (int64_t(i) * o + j) * v * v;
  double s = 0.0;
  const int64_t nab = int64_t(v) * (v - 1) / 2;
  for (int64_t u = threadIdx.x; u < nab; u += 256) {
    int a, b;
    tri(u, v, a, b);
    const double x = oovv[base + int64_t(a) * v + b];
    const double D = (d_oo[i] + d_oo[j]) - (d_vv[a] + d_vv[b]);
    s += x * x / D;
  }
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) epair[blockIdx.x] = sh[0];
}

// Raw (x, D, e) or standardised features of unique amplitudes, (ij, ab) order.
__global__ __launch_bounds__(256) void features_kernel(int o, int v, const double *__restrict__ oovv,
                                                       const double *__restrict__ d_oo,
                                                       const double *__restrict__ d_vv,
                                                       const double *__restrict__ epair, cc_mlp_stats st,
                                                       int standardise, double *__restrict__ z) {
  const int64_t nab = int64_t(v) * (v - 1) / 2, n = nab * (int64_t(o) * (o - 1) / 2);
  for (int64_t u = blockIdx.x * int64_t(256) + threadIdx.x; u < n; u += int64_t(gridDim.x) * 256) {
    int i, j, a, b;
    tri(u / nab, o, i, j);
    tri(u % nab, v, a, b);
    const double x = oovv[(int64_t(i) * o + j) * v * v + int64_t(a) * v + b];
    const double D = (d_oo[i] + d_oo[j]) - (d_vv[a] + d_vv[b]);
    const double e = epair[u / nab];
    if (standardise) {
      z[3 * u] = x / st.sx;
      z[3 * u + 1] = (D - st.mD) / st.sD;
      z[3 * u + 2] = (e - st.me) / st.se;
    } else {
      z[3 * u] = x;
      z[3 * u + 1] = D;
      z[3 * u + 2] = e;
    }
  }
}

__global__ __launch_bounds__(256) void standardise_kernel(const double *__restrict__ raw, const double *__restrict__ y,
                                                          int64_t n, cc_mlp_stats st, double *__restrict__ z,
                                                          double *__restrict__ ys) {
  for (int64_t r = blockIdx.x * int64_t(256) + threadIdx.x; r < n; r += int64_t(gridDim.x) * 256) {
    z[3 * r] = raw[3 * r] / st.sx;
    z[3 * r + 1] = (raw[3 * r + 1] - st.mD) / st.sD;
    z[3 * r + 2] = (raw[3 * r + 2] - st.me) / st.se;
    if (y) ys[r] = y[r] / st.st;
  }
}

// unique amplitudes of t2 (scaled by 1/st) -> y
__global__ __launch_bounds__(256) void gather_targets_kernel(int o, int v, const double *__restrict__ t2,
                                                             double inv_st, double *__restrict__ y) {
  const int64_t nab = int64_t(v) * (v - 1) / 2, n = nab * (int64_t(o) * (o - 1) / 2);
  for (int64_t u = blockIdx.x * int64_t(256) + threadIdx.x; u < n; u += int64_t(gridDim.x) * 256) {
    int i, j, a, b;
    tri(u / nab, o, i, j);
    tri(u % nab, v, a, b);
    y[u] = t2[(int64_t(i) * o + j) * v * v + int64_t(a) * v + b] * inv_st;
  }
}

// predictions f (scaled by st) -> antisymmetric t2 (four images, zero diagonals)
__global__ __launch_bounds__(256) void scatter_t2_kernel(int o, int v, const double *__restrict__ f, double st,
                                                         double *__restrict__ t2) {
  const int64_t total = int64_t(o) * o * v * v;
  for (int64_t e = blockIdx.x * int64_t(256) + threadIdx.x; e < total; e += int64_t(gridDim.x) * 256) {
    const int b = e % v, a = (e / v) % v;
    const int64_t ij = e / (int64_t(v) * v);
    const int j = ij % o, i = ij / o;
    double val = 0.0;
    if (i != j && a != b) {
      const int ii = i < j ? i : j, jj = i < j ? j : i, aa = a < b ? a : b, bb = a < b ? b : a;
      const double sgn = ((i < j) == (a < b)) ? 1.0 : -1.0;
      const int64_t pij = int64_t(ii) * (2 * o - ii - 1) / 2 + (jj - ii - 1);
      const int64_t pab = int64_t(aa) * (2 * v - aa - 1) / 2 + (bb - aa - 1);
      val = sgn * st * f[pij * (int64_t(v) * (v - 1) / 2) + pab];
    }
    t2[e] = val;
  }
}

// rows [0,c): z[order[r]], rows [c,2c): same with the first component negated
__global__ __launch_bounds__(256) void build_z2_kernel(const double *__restrict__ z, const int64_t *__restrict__ order,
                                                       int64_t r0, int64_t c, double *__restrict__ z2) {
  for (int64_t r = blockIdx.x * int64_t(256) + threadIdx.x; r < c; r += int64_t(gridDim.x) * 256) {
    const int64_t src = order ? order[r0 + r] : r0 + r;
    const double a = z[3 * src], b = z[3 * src + 1], d = z[3 * src + 2];
    z2[3 * r] = a;
    z2[3 * r + 1] = b;
    z2[3 * r + 2] = d;
    z2[3 * (c + r)] = -a;
    z2[3 * (c + r) + 1] = b;
    z2[3 * (c + r) + 2] = d;
  }
}

__global__ __launch_bounds__(256) void bias_relu_kernel(double *__restrict__ A, const double *__restrict__ b,
                                                        int64_t rows) {
  const int64_t n = rows * HID;
  for (int64_t e = blockIdx.x * int64_t(256) + threadIdx.x; e < n; e += int64_t(gridDim.x) * 256) {
    const double x = A[e] + b[e % HID];
    A[e] = x > 0.0 ? x : 0.0;
  }
}

// f = (g+ - g-)/2 (g includes b3, which cancels); optional loss terms.
__global__ __launch_bounds__(256) void head_kernel(const double *__restrict__ g, int64_t c,
                                                   const double *__restrict__ y, const int64_t *__restrict__ order,
                                                   int64_t r0, double *__restrict__ f, double *__restrict__ dg,
                                                   double *__restrict__ lpart) {
  __shared__ double sh[256];
  double s = 0.0;
  for (int64_t r = blockIdx.x * int64_t(256) + threadIdx.x; r < c; r += int64_t(gridDim.x) * 256) {
    const double fv = 0.5 * (g[r] - g[c + r]);
    if (f) f[r0 + r] = fv;
    if (y) {
      const double res = fv - y[order ? order[r0 + r] : r0 + r];
      s += res * res;
      // d loss / d f = 2 res / c ; d f / d g+- = +-1/2
      dg[r] = res / double(c);
      dg[c + r] = -res / double(c);
    }
  }
  if (lpart) {
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
      if (threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
      __syncthreads();
    }
    if (threadIdx.x == 0) lpart[blockIdx.x] = sh[0];
  }
}

// dA2[r][j] = dg[r] W3[j] (H2[r][j] > 0)
__global__ __launch_bounds__(256) void da2_kernel(const double *__restrict__ dg, const double *__restrict__ W3,
                                                  const double *__restrict__ H2, int64_t rows,
                                                  double *__restrict__ dA2) {
  const int64_t n = rows * HID;
  for (int64_t e = blockIdx.x * int64_t(256) + threadIdx.x; e < n; e += int64_t(gridDim.x) * 256)
    dA2[e] = H2[e] > 0.0 ? dg[e / HID] * W3[e % HID] : 0.0;
}

__global__ __launch_bounds__(256) void relu_mask_kernel(double *__restrict__ d, const double *__restrict__ H,
                                                        int64_t n) {
  for (int64_t e = blockIdx.x * int64_t(256) + threadIdx.x; e < n; e += int64_t(gridDim.x) * 256)
    if (!(H[e] > 0.0)) d[e] = 0.0;
}

__global__ __launch_bounds__(256) void fill_kernel(double *p, double v, int64_t n) {
  for (int64_t e = blockIdx.x * int64_t(256) + threadIdx.x; e < n; e += int64_t(gridDim.x) * 256) p[e] = v;
}

// loss = sum of partials / c, written to out[idx] (fixed order)
__global__ void loss_sum_kernel(const double *lpart, int nb, int64_t c, double *out, int64_t idx) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    double s = 0.0;
    for (int k = 0; k < nb; ++k) s += lpart[k];
    out[idx] = s / double(c);
  }
}

__global__ __launch_bounds__(256) void adam_kernel(double *__restrict__ p, const double *__restrict__ g,
                                                   double *__restrict__ m, double *__restrict__ vv, int64_t n,
                                                   double lr, double b1, double b2, double eps, double c1,
                                                   double c2) {
  for (int64_t e = blockIdx.x * int64_t(256) + threadIdx.x; e < n; e += int64_t(gridDim.x) * 256) {
    const double gi = g[e];
    const double mi = b1 * m[e] + (1.0 - b1) * gi;
    const double vi = b2 * vv[e] + (1.0 - b2) * gi * gi;
    m[e] = mi;
    vv[e] = vi;
    p[e] -= lr * (mi / c1) / (sqrt(vi / c2) + eps);
  }
}

// column moments of raw features: [sum x^2, sum D, sum D^2, sum e, sum e^2] partials
__global__ __launch_bounds__(256) void moments_kernel(const double *__restrict__ raw, const double *__restrict__ y,
                                                      int64_t n, double *__restrict__ part) {
  __shared__ double sh[256];
  double acc[7] = {0, 0, 0, 0, 0, 0, 0};
  for (int64_t r = blockIdx.x * int64_t(256) + threadIdx.x; r < n; r += int64_t(gridDim.x) * 256) {
    const double x = raw[3 * r], D = raw[3 * r + 1], e = raw[3 * r + 2];
    acc[0] += x * x;
    acc[1] += D;
    acc[2] += D * D;
    acc[3] += e;
    acc[4] += e * e;
    if (y) acc[5] += y[r] * y[r];
    acc[6] += 1.0;
  }
  for (int q = 0; q < 7; ++q) {
    sh[threadIdx.x] = acc[q];
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
      if (threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
      __syncthreads();
    }
    if (threadIdx.x == 0) part[7 * blockIdx.x + q] = sh[0];
    __syncthreads();
  }
}

int64_t grid_of(int64_t n) { return std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 4096)); }

// ---- fused FP32 forward (inference) ----------------------------------------
// f[u] = (g(z_u) - g(z~_u)) / 2 without writing activations anywhere: one
// wave takes 16 samples at a time as two 16-row blocks (the + branch and the
// branch with z0 negated) against all 128 hidden units.  Layer 1 is formed in
// registers directly in the MFMA operand layout, layer 2 runs on
// v_mfma_f32_16x16x4_f32 with W2 (rounded to FP32) staged once per workgroup
// in LDS, and bias, ReLU and the 128 -> 1 layer are applied to the
// accumulators, summed over the 16 lanes that share output rows.
//   MFMA 16x16x4 operands: lane l = 16 q + r supplies A[row r][k q] and
//   B[k q][col r] and holds D[4 q + t][r], t = 0..3.  Step s of chunk c uses
//   hidden unit k = 16 c + 4 q + s for lane group q (a permutation of the
//   128 units, the same on both operands).
typedef float f4v __attribute__((ext_vector_type(4)));
constexpr int FW_WAVES = 4;
constexpr int W2_LD = HID + 4;  // padded LDS row: the 16 lanes of a read phase hit distinct banks

__global__ __launch_bounds__(FW_WAVES * 64) void mlp_forward_fused_kernel(const double *__restrict__ P,
                                                                          const double *__restrict__ z, int64_t n,
                                                                          double *__restrict__ f) {
  __shared__ __attribute__((aligned(16))) float sW2[HID * W2_LD];
  __shared__ __attribute__((aligned(16))) float sW1[HID * 4];  // (w1 x, w1 y, w1 z, b1) per hidden unit
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  for (int e = tid; e < HID * HID; e += FW_WAVES * 64) sW2[(e / HID) * W2_LD + e % HID] = float(P[OFF_W2 + e]);
  for (int k = tid; k < HID; k += FW_WAVES * 64) {
    sW1[4 * k] = float(P[OFF_W1 + 3 * k]);
    sW1[4 * k + 1] = float(P[OFF_W1 + 3 * k + 1]);
    sW1[4 * k + 2] = float(P[OFF_W1 + 3 * k + 2]);
    sW1[4 * k + 3] = float(P[OFF_B1 + k]);
  }
  __syncthreads();
  const int r = lane & 15, q = lane >> 4;
  float b2r[8], w3r[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    b2r[j] = float(P[OFF_B2 + 16 * j + r]);
    w3r[j] = float(P[OFF_W3 + 16 * j + r]);
  }
  const int64_t nblk = (n + 15) / 16;
  for (int64_t blk = int64_t(blockIdx.x) * FW_WAVES + wave; blk < nblk; blk += int64_t(gridDim.x) * FW_WAVES) {
    const int64_t u = std::min<int64_t>(blk * 16 + r, n - 1);
    const float z0 = float(z[3 * u]), z1 = float(z[3 * u + 1]), z2 = float(z[3 * u + 2]);
    f4v acc[2][8];
#pragma unroll
    for (int j = 0; j < 8; ++j) acc[0][j] = acc[1][j] = f4v{0.f, 0.f, 0.f, 0.f};
#pragma unroll 2
    for (int c = 0; c < 8; ++c) {
      float a0[4], a1[4];
#pragma unroll
      for (int st = 0; st < 4; ++st) {
        const f4v w = *reinterpret_cast<const f4v *>(&sW1[4 * (16 * c + 4 * q + st)]);
        const float common = w[1] * z1 + w[2] * z2 + w[3];
        const float hp = common + w[0] * z0, hm = common - w[0] * z0;
        a0[st] = hp > 0.f ? hp : 0.f;
        a1[st] = hm > 0.f ? hm : 0.f;
      }
      f4v bf[8];
#pragma unroll
      for (int j = 0; j < 8; ++j) bf[j] = *reinterpret_cast<const f4v *>(&sW2[(16 * j + r) * W2_LD + 16 * c + 4 * q]);
#pragma unroll
      for (int st = 0; st < 4; ++st)
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          acc[0][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a0[st], bf[j][st], acc[0][j], 0, 0, 0);
          acc[1][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a1[st], bf[j][st], acc[1][j], 0, 0, 0);
        }
    }
    // g (without b3, which cancels in f) for rows 4 q + t of both branches
    float g[2][4];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        float sum = 0.f;
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          const float h = acc[i][j][t] + b2r[j];
          sum += (h > 0.f ? h : 0.f) * w3r[j];
        }
        g[i][t] = sum;
      }
#pragma unroll
    for (int off = 1; off < 16; off <<= 1)
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int t = 0; t < 4; ++t) g[i][t] += __shfl_xor(g[i][t], off, 64);
    if (r == 0) {
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int64_t uu = blk * 16 + 4 * q + t;
        if (uu < n) f[uu] = 0.5 * (double(g[0][t]) - double(g[1][t]));
      }
    }
  }
}

void forward_fused(const double *P, const double *z, int64_t n, double *f, hipStream_t s) {
  if (n <= 0) return;
  const int64_t blocks = std::max<int64_t>(1, std::min<int64_t>((n + 16 * FW_WAVES - 1) / (16 * FW_WAVES), 512));
  hipLaunchKernelGGL(mlp_forward_fused_kernel, dim3(blocks), dim3(FW_WAVES * 64), 0, s, P, z, n, f);
  CC_HIP_CHECK(hipGetLastError());
}

// Dense layer helper: C[M][N] = alpha * A' B'^T + beta C (GemmDesc conventions)
void dense(int prec, int64_t M, int64_t N, int64_t K, const double *A, int64_t sam, int64_t sak, const double *B,
           int64_t sbn, int64_t sbk, double *C, double beta, double *ws, int64_t ws_elems, hipStream_t s) {
  GemmDesc d{M, N, K, A, sam, sak, B, sbn, sbk, C, N, 1.0, beta};
  // the split-K factor the library picks, down to what the workspace holds
  // (the weight gradients, K = rows of a minibatch, run on a handful of
  // output tiles and need the split)
  int64_t split = gemm_split_pick(M, N, K, -1);
  if (ws) split = std::min<int64_t>(split, ws_elems / (M * N));
  if (split > 1 && ws) {
    d.split = int(split);
    d.ws = ws;
  }
  if (prec == PREC_F64) gemm_f64(d, s, -1);
  else gemm_lowp(d, prec, s, -1);
}

struct MlpWork {
  int64_t cap = 0;  // rows per chunk (samples)
  double *z2 = nullptr, *H1 = nullptr, *H2 = nullptr, *dH = nullptr, *g = nullptr, *dg = nullptr,
         *grad = nullptr, *ones = nullptr, *lpart = nullptr, *ws = nullptr;
  int64_t ws_elems = 0;
  void alloc(int64_t c) {
    cap = c;
    auto A = [](double **p, int64_t n) {
      if (hipMalloc(p, sizeof(double) * std::max<int64_t>(n, 1)) != hipSuccess) {
        (void)hipGetLastError();
        throw CCError(CC_ENOMEM, "MLP workspace allocation failed");
      }
    };
    A(&z2, 2 * c * 3);
    A(&H1, 2 * c * HID);
    A(&H2, 2 * c * HID);
    A(&dH, 2 * c * HID);
    A(&g, 2 * c);
    A(&dg, 2 * c);
    A(&grad, NPAR);
    A(&ones, 2 * c);
    A(&lpart, 4096);
    ws_elems = 256 * int64_t(HID) * HID;
    A(&ws, ws_elems);
  }
  ~MlpWork() {
    for (double *p : {z2, H1, H2, dH, g, dg, grad, ones, lpart, ws})
      if (p) (void)hipFree(p);
  }
};

// Forward of rows [r0, r0+c): leaves H1, H2, g in the workspace.
void forward_chunk(int prec, const double *P, const double *z, const int64_t *order, int64_t r0, int64_t c,
                   MlpWork &w, hipStream_t s) {
  const int64_t R = 2 * c;
  hipLaunchKernelGGL(build_z2_kernel, dim3(grid_of(c)), dim3(256), 0, s, z, order, r0, c, w.z2);
  dense(prec, R, HID, 3, w.z2, 3, 1, P + OFF_W1, 3, 1, w.H1, 0.0, nullptr, 0, s);
  hipLaunchKernelGGL(bias_relu_kernel, dim3(grid_of(R * HID)), dim3(256), 0, s, w.H1, P + OFF_B1, R);
  dense(prec, R, HID, HID, w.H1, HID, 1, P + OFF_W2, HID, 1, w.H2, 0.0, nullptr, 0, s);
  hipLaunchKernelGGL(bias_relu_kernel, dim3(grid_of(R * HID)), dim3(256), 0, s, w.H2, P + OFF_B2, R);
  dense(prec, R, 1, HID, w.H2, HID, 1, P + OFF_W3, HID, 1, w.g, 0.0, nullptr, 0, s);
  CC_HIP_CHECK(hipGetLastError());
}

// Gradient of the chunk's mean squared error into w.grad (overwritten).
void backward_chunk(int prec, const double *P, const double *z, const double *y, const int64_t *order, int64_t r0,
                    int64_t c, MlpWork &w, double *loss_out, int64_t loss_idx, hipStream_t s) {
  const int64_t R = 2 * c;
  forward_chunk(prec, P, z, order, r0, c, w, s);
  const int nb = int(grid_of(c));
  hipLaunchKernelGGL(head_kernel, dim3(nb), dim3(256), 0, s, w.g, c, y, order, r0, (double *)nullptr, w.dg,
                     w.lpart);
  if (loss_out) hipLaunchKernelGGL(loss_sum_kernel, dim3(1), dim3(64), 0, s, w.lpart, nb, c, loss_out, loss_idx);
  double *G = w.grad;
  // W3 (1 x 128) = dg^T H2 ; b3 = sum dg
  dense(prec, 1, HID, R, w.dg, R, 1, w.H2, 1, HID, G + OFF_W3, 0.0, w.ws, w.ws_elems, s);
  dense(prec, 1, 1, R, w.dg, R, 1, w.ones, R, 1, G + OFF_B3, 0.0, w.ws, w.ws_elems, s);
  // dA2 in place of H2 (H2 is needed for the mask first)
  hipLaunchKernelGGL(da2_kernel, dim3(grid_of(R * HID)), dim3(256), 0, s, w.dg, P + OFF_W3, w.H2, R, w.H2);
  dense(prec, HID, HID, R, w.H2, 1, HID, w.H1, 1, HID, G + OFF_W2, 0.0, w.ws, w.ws_elems, s);
  dense(prec, 1, HID, R, w.ones, R, 1, w.H2, 1, HID, G + OFF_B2, 0.0, w.ws, w.ws_elems, s);
  // dA1 = (dA2 W2) * (H1 > 0)
  dense(prec, R, HID, HID, w.H2, HID, 1, P + OFF_W2, 1, HID, w.dH, 0.0, nullptr, 0, s);
  hipLaunchKernelGGL(relu_mask_kernel, dim3(grid_of(R * HID)), dim3(256), 0, s, w.dH, w.H1, R * HID);
  dense(prec, HID, 3, R, w.dH, 1, HID, w.z2, 1, 3, G + OFF_W1, 0.0, w.ws, w.ws_elems, s);
  dense(prec, 1, HID, R, w.ones, R, 1, w.dH, 1, HID, G + OFF_B1, 0.0, w.ws, w.ws_elems, s);
  CC_HIP_CHECK(hipGetLastError());
}

void device_diag(cc_ctx *ctx, const cc_system *sys, double **d_oo, double **d_vv) {
  CC_HIP_CHECK(hipMalloc(d_oo, sizeof(double) * sys->o));
  CC_HIP_CHECK(hipMalloc(d_vv, sizeof(double) * sys->v));
  fock_diag(false, sys->o, sys->v, sys->f_oo, sys->f_vv, *d_oo, *d_vv, ctx->stream);
}

}  // namespace
}  // namespace ccmi

// ================================================================ C ABI ====
using ccmi::CCError;
namespace {
int mfail(cc_ctx *ctx, int st, const std::string &m) {
  if (ctx) ctx->last_error = m;
  return st;
}
template <class F>
int mguard(cc_ctx *ctx, F &&f) {
  try {
    return f();
  } catch (const CCError &e) {
    return mfail(ctx, e.status, e.what());
  } catch (const std::exception &e) {
    return mfail(ctx, CC_EINTERNAL, e.what());
  }
}
void check_sys_real(const cc_system *sys) {
  if (!sys || sys->o < 2 || sys->v < 2) throw CCError(CC_EINVAL, "MLP features need o >= 2 and v >= 2");
  if (sys->scalar != CC_R64) throw CCError(CC_EUNSUPPORTED, "the amplitude-guess network is real-valued");
  if (!sys->oovv || !sys->f_oo || !sys->f_vv) throw CCError(CC_EINVAL, "system pointers are NULL");
}
void check_prec(int prec) {
  if (prec != CC_PREC_F64 && prec != CC_PREC_F32) throw CCError(CC_EINVAL, "MLP precision must be F64 or F32");
}
}  // namespace

extern "C" {

int64_t cc_mlp_num_params(void) { return ccmi::NPAR; }

int64_t cc_mlp_num_samples(int o, int v) {
  if (o < 2 || v < 2) return 0;
  return (int64_t(o) * (o - 1) / 2) * (int64_t(v) * (v - 1) / 2);
}

int cc_mlp_features(cc_ctx *ctx, const cc_system *sys, const cc_mlp_stats *stats, double *z_out) {
  if (!ctx) return mfail(nullptr, CC_EINVAL, "ctx is NULL");
  return mguard(ctx, [&] {
    check_sys_real(sys);
    if (!z_out) throw CCError(CC_EINVAL, "z_out is NULL");
    CC_HIP_CHECK(hipSetDevice(ctx->device));
    hipStream_t s = ctx->stream;
    const int o = sys->o, v = sys->v;
    const int64_t npair = int64_t(o) * (o - 1) / 2, n = cc_mlp_num_samples(o, v);
    double *d_oo = nullptr, *d_vv = nullptr, *ep = nullptr;
    ccmi::device_diag(ctx, sys, &d_oo, &d_vv);
    CC_HIP_CHECK(hipMalloc(&ep, sizeof(double) * npair));
    cc_mlp_stats st = stats ? *stats : cc_mlp_stats{1, 0, 1, 0, 1, 1};
    hipLaunchKernelGGL(ccmi::pair_energy_kernel, dim3(npair), dim3(256), 0, s, o, v,
                       static_cast<const double *>(sys->oovv), d_oo, d_vv, ep);
    hipLaunchKernelGGL(ccmi::features_kernel, dim3(ccmi::grid_of(n)), dim3(256), 0, s, o, v,
                       static_cast<const double *>(sys->oovv), d_oo, d_vv, ep, st, stats ? 1 : 0, z_out);
    CC_HIP_CHECK(hipGetLastError());
    CC_HIP_CHECK(hipStreamSynchronize(s));
    (void)hipFree(d_oo);
    (void)hipFree(d_vv);
    (void)hipFree(ep);
    return CC_OK;
  });
}

int cc_mlp_targets(cc_ctx *ctx, int o, int v, const double *t2, double scale, double *y_out) {
  if (!ctx) return mfail(nullptr, CC_EINVAL, "ctx is NULL");
  return mguard(ctx, [&] {
    if (!t2 || !y_out || o < 2 || v < 2 || !(scale != 0.0)) throw CCError(CC_EINVAL, "bad arguments");
    const int64_t n = cc_mlp_num_samples(o, v);
    hipLaunchKernelGGL(ccmi::gather_targets_kernel, dim3(ccmi::grid_of(n)), dim3(256), 0, ctx->stream, o, v, t2,
                       1.0 / scale, y_out);
    CC_HIP_CHECK(hipGetLastError());
    CC_HIP_CHECK(hipStreamSynchronize(ctx->stream));
    return CC_OK;
  });
}

int cc_mlp_standardise(cc_ctx *ctx, const double *raw, const double *y, int64_t n, const cc_mlp_stats *stats,
                       double *z_out, double *y_out) {
  if (!ctx) return mfail(nullptr, CC_EINVAL, "ctx is NULL");
  return mguard(ctx, [&] {
    if (!raw || !stats || !z_out || n < 1 || (y && !y_out)) throw CCError(CC_EINVAL, "bad arguments");
    hipLaunchKernelGGL(ccmi::standardise_kernel, dim3(ccmi::grid_of(n)), dim3(256), 0, ctx->stream, raw, y, n,
                       *stats, z_out, y_out);
    CC_HIP_CHECK(hipGetLastError());
    CC_HIP_CHECK(hipStreamSynchronize(ctx->stream));
    return CC_OK;
  });
}

int cc_mlp_moments(cc_ctx *ctx, const double *raw, const double *y, int64_t n, double *out7) {
  if (!ctx) return mfail(nullptr, CC_EINVAL, "ctx is NULL");
  return mguard(ctx, [&] {
    if (!raw || n < 1 || !out7) throw CCError(CC_EINVAL, "bad arguments");
    const int nb = int(ccmi::grid_of(n));
    double *part = nullptr;
    CC_HIP_CHECK(hipMalloc(&part, sizeof(double) * 7 * nb));
    hipLaunchKernelGGL(ccmi::moments_kernel, dim3(nb), dim3(256), 0, ctx->stream, raw, y, n, part);
    std::vector<double> h(7 * nb);
    CC_HIP_CHECK(hipMemcpyAsync(h.data(), part, sizeof(double) * 7 * nb, hipMemcpyDeviceToHost, ctx->stream));
    CC_HIP_CHECK(hipStreamSynchronize(ctx->stream));
    (void)hipFree(part);
    for (int q = 0; q < 7; ++q) {
      double s = 0.0;
      for (int b = 0; b < nb; ++b) s += h[7 * b + q];
      out7[q] = s;
    }
    return CC_OK;
  });
}

int cc_mlp_forward(cc_ctx *ctx, int prec, const double *params, const double *z, int64_t n, double *f_out) {
  if (!ctx) return mfail(nullptr, CC_EINVAL, "ctx is NULL");
  return mguard(ctx, [&] {
    check_prec(prec);
    if (!params || !z || !f_out || n < 1) throw CCError(CC_EINVAL, "bad arguments");
    CC_HIP_CHECK(hipSetDevice(ctx->device));
    if (prec == CC_PREC_F32) {  // inference in one fused launch
      ccmi::forward_fused(params, z, n, f_out, ctx->stream);
      CC_HIP_CHECK(hipStreamSynchronize(ctx->stream));
      return CC_OK;
    }
    ccmi::MlpWork w;
    const int64_t cap = std::min<int64_t>(n, 1 << 18);
    w.alloc(cap);
    for (int64_t r0 = 0; r0 < n; r0 += cap) {
      const int64_t c = std::min(cap, n - r0);
      ccmi::forward_chunk(prec, params, z, nullptr, r0, c, w, ctx->stream);
      hipLaunchKernelGGL(ccmi::head_kernel, dim3(ccmi::grid_of(c)), dim3(256), 0, ctx->stream, w.g, c,
                         (const double *)nullptr, (const int64_t *)nullptr, r0, f_out, (double *)nullptr,
                         (double *)nullptr);
    }
    CC_HIP_CHECK(hipStreamSynchronize(ctx->stream));
    return CC_OK;
  });
}

int cc_mlp_loss_grad(cc_ctx *ctx, int prec, const double *params, const double *z, const double *y, int64_t n,
                     double *loss, double *grad_out) {
  if (!ctx) return mfail(nullptr, CC_EINVAL, "ctx is NULL");
  return mguard(ctx, [&] {
    check_prec(prec);
    if (!params || !z || !y || !grad_out || n < 1) throw CCError(CC_EINVAL, "bad arguments");
    CC_HIP_CHECK(hipSetDevice(ctx->device));
    ccmi::MlpWork w;
    w.alloc(n);
    hipStream_t s = ctx->stream;
    hipLaunchKernelGGL(ccmi::fill_kernel, dim3(ccmi::grid_of(2 * n)), dim3(256), 0, s, w.ones, 1.0, 2 * n);
    double *dl = nullptr;
    CC_HIP_CHECK(hipMalloc(&dl, sizeof(double)));
    ccmi::backward_chunk(prec, params, z, y, nullptr, 0, n, w, dl, 0, s);
    CC_HIP_CHECK(hipMemcpyAsync(grad_out, w.grad, sizeof(double) * ccmi::NPAR, hipMemcpyDeviceToDevice, s));
    double hl = 0.0;
    CC_HIP_CHECK(hipMemcpyAsync(&hl, dl, sizeof(double), hipMemcpyDeviceToHost, s));
    CC_HIP_CHECK(hipStreamSynchronize(s));
    (void)hipFree(dl);
    if (loss) *loss = hl;
    return CC_OK;
  });
}

int cc_mlp_train(cc_ctx *ctx, int prec, double *params, double *adam_m, double *adam_v, const double *z,
                 const double *y, int64_t n, const int64_t *order, int64_t batch, int32_t epochs, double lr,
                 int64_t *adam_t, double *loss_hist, int32_t hist_cap) {
  if (!ctx) return mfail(nullptr, CC_EINVAL, "ctx is NULL");
  return mguard(ctx, [&] {
    check_prec(prec);
    if (!params || !adam_m || !adam_v || !z || !y || !adam_t || n < 1 || batch < 1 || epochs < 1 || !(lr > 0))
      throw CCError(CC_EINVAL, "bad arguments");
    CC_HIP_CHECK(hipSetDevice(ctx->device));
    hipStream_t s = ctx->stream;
    const int64_t c = std::min(batch, n);
    ccmi::MlpWork w;
    w.alloc(c);
    hipLaunchKernelGGL(ccmi::fill_kernel, dim3(ccmi::grid_of(2 * c)), dim3(256), 0, s, w.ones, 1.0, 2 * c);
    const int64_t steps_per_epoch = (n + c - 1) / c;
    double *dl = nullptr;
    CC_HIP_CHECK(hipMalloc(&dl, sizeof(double) * steps_per_epoch));
    const double b1 = 0.9, b2 = 0.999, eps = 1e-8;
    for (int ep = 0; ep < epochs; ++ep) {
      for (int64_t st = 0; st < steps_per_epoch; ++st) {
        const int64_t r0 = st * c, cc = std::min(c, n - r0);
        ccmi::backward_chunk(prec, params, z, y, order, r0, cc, w, dl, st, s);
        const int64_t t = ++(*adam_t);
        hipLaunchKernelGGL(ccmi::adam_kernel, dim3(ccmi::grid_of(ccmi::NPAR)), dim3(256), 0, s, params, w.grad,
                           adam_m, adam_v, ccmi::NPAR, lr, b1, b2, eps, 1.0 - std::pow(b1, double(t)),
                           1.0 - std::pow(b2, double(t)));
      }
      std::vector<double> h(steps_per_epoch);
      CC_HIP_CHECK(hipMemcpyAsync(h.data(), dl, sizeof(double) * steps_per_epoch, hipMemcpyDeviceToHost, s));
      CC_HIP_CHECK(hipStreamSynchronize(s));
      double mean = 0.0;
      for (double x : h) mean += x;
      mean /= double(steps_per_epoch);
      if (loss_hist && ep < hist_cap) loss_hist[ep] = mean;
    }
    (void)hipFree(dl);
    return CC_OK;
  });
}

int cc_guess_mlp(cc_ctx *ctx, const cc_system *sys, int prec, const double *params, const cc_mlp_stats *stats,
                 cc_amps *t_out) {
  if (!ctx) return mfail(nullptr, CC_EINVAL, "ctx is NULL");
  return mguard(ctx, [&] {
    check_sys_real(sys);
    check_prec(prec);
    if (!params || !stats || !t_out || !t_out->t2) throw CCError(CC_EINVAL, "bad arguments");
    const int o = sys->o, v = sys->v;
    const int64_t n = cc_mlp_num_samples(o, v);
    double *z = nullptr, *f = nullptr;
    CC_HIP_CHECK(hipMalloc(&z, sizeof(double) * 3 * n));
    CC_HIP_CHECK(hipMalloc(&f, sizeof(double) * n));
    int st = cc_mlp_features(ctx, sys, stats, z);
    if (st == CC_OK) st = cc_mlp_forward(ctx, prec, params, z, n, f);
    if (st == CC_OK) {
      hipLaunchKernelGGL(ccmi::scatter_t2_kernel, dim3(ccmi::grid_of(int64_t(o) * o * v * v)), dim3(256), 0,
                         ctx->stream, o, v, f, stats->st, static_cast<double *>(t_out->t2));
      if (t_out->t1)
        hipLaunchKernelGGL(ccmi::fill_kernel, dim3(ccmi::grid_of(int64_t(o) * v)), dim3(256), 0, ctx->stream,
                           static_cast<double *>(t_out->t1), 0.0, int64_t(o) * v);
      CC_HIP_CHECK(hipGetLastError());
      CC_HIP_CHECK(hipStreamSynchronize(ctx->stream));
    }
    (void)hipFree(z);
    (void)hipFree(f);
    return st;
  });
}

}  // extern "C"
