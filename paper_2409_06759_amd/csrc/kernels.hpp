// Launchers of the device kernels (declarations shared by the host code).
//
// Every data-movement / elementwise kernel is described by an "entry" struct
// that holds one system's arguments and device pointers.  A single launch
// takes one entry by value; a grouped launch takes a device array of entries
// (one per system of a batch) and an offset table: system b owns workgroups
// [off[b], off[b+1]).  Both launch forms run the same device body, so a
// batched result equals the single-system one bit for bit.
#pragma once

#include "common.hpp"

#include <algorithm>

namespace ccmi {

struct PermArgs {
  int rank;
  int64_t dims[kMaxRank];
  int64_t istr[kMaxRank];
  int64_t ostr[kMaxRank];
  double alpha, beta;
  int conj;
  int d_o, d_i;  // tiled dims: output unit-stride dim and input unit-stride dim
  int lti;       // tiled: log2 of the tile's extent along d_i (4..256; 1,024 elements per tile)
  int64_t rest_dims[kMaxRank], rest_istr[kMaxRank], rest_ostr[kMaxRank];
  int nrest;
  int64_t n_rest_total, tiles_o, tiles_i;
  int64_t total;
};

struct PermEntry {
  PermArgs p;
  const void *in;
  void *out;
  int tiled;
  int64_t units;
};

struct OuterArgs {
  int rank;
  int64_t dims[4];
  int64_t sa[4], sb[4];  // strides of A and B for each C dimension (0 = not indexed)
  double alpha;
  int conj_a, conj_b;
};

struct OuterEntry {
  OuterArgs a;
  const void *A, *B;
  void *C;
  int64_t total, units;
};

struct FillEntry {
  void *p;
  int64_t n, units;
};

struct SplitkEntry {
  const void *ws;
  int split;
  int lanes;  // threads summing one output (power of two <= 16); 256 / lanes outputs per workgroup
  int64_t M, N;
  void *C;
  int64_t ldc;
  double alpha, beta;
  int64_t units;
};

struct TauEntry {
  int o, v;
  const void *t1, *t2, *oovv, *fov;  // t1 == nullptr: CCD (tau = t2, not written)
  void *tau, *taut;
  double *partials;  // 2 per unit (re, im)
  int64_t units;
};

struct R2Args {
  int o, v;
  const double *fdiag_o, *fdiag_v;  // bare Fock diagonals
  double shift;
  int dressed;                      // 1: denominators from the dressed one-body diagonals
  const void *Fo, *Fv;              // dressed [o][o] and [v][v] one-body intermediates
};

struct AsmEntry {
  R2Args a;
  const void *XP, *Xij, *Xab, *Xr;
  void *R, *t2;  // either may be nullptr
  double *partials;
  int64_t units;
};

struct R1Entry {
  int o, v;
  const void *R1;
  void *t1;  // nullptr: no update
  const double *d_oo, *d_vv;
  double shift;
  int dressed;
  const void *Fo, *Fv;
  double *partial;
};

struct FinEntry {
  const double *epart;
  int ne;
  const double *n2part;
  int nn;
  const double *n1part;  // may be nullptr
  double *scalars;       // [0] = ||R||, [1] = Re E, [2] = Im E
  const double *n3part = nullptr;  // triples norm partials (may be nullptr)
  int nn3 = 0;
};

// Packed index pairs: for a rank-4 tensor X[n0][n1][n2][n3] and index-pair
// tables rows (P -> (x0, x1)) and cols (Q -> (x2, x3)):
// mode 0 gathers dst[P][Q] = X[x0][x1][x2][x3] (X = src), mode 1 scatters
// X[..] += src[P][Q] and mode 2 sets X[..] = src[P][Q] (X = dst).
struct PairEntry {
  const void *src;
  void *dst;
  const int *rows, *cols;  // rows[2P], rows[2P+1]; cols[2Q], cols[2Q+1]
  int64_t nP, nQ;
  int64_t ldq;             // row stride of the packed side (>= nQ; padding columns untouched)
  int64_t n1, n2, n3;      // dims 1..3 of X (dim 0 is implied)
  int mode;
  int64_t units;
};

// R3 = full antisymmetriser of the accumulated triples contributions Y3
// (sum over the 36 signed permutations of (ijk) and (abc)), exact zeros for
// repeated indices, optional Jacobi update t3 += R3 / (D - shift) with bare
// denominators, and per-workgroup partial sums of |R3|^2.
struct T3Entry {
  int o, v;
  const void *Y3;
  void *R3;   // nullptr: not stored
  void *t3;   // nullptr: no update
  const double *d_oo, *d_vv;
  double shift;
  double *partials;
  int64_t units;
};

// ---- entry construction (host) ---------------------------------------------
PermEntry make_perm_entry(const PermDesc &d, const void *in, void *out);
OuterEntry make_outer_entry(const OuterArgs &a, const void *A, const void *B, void *C);
FillEntry make_fill_entry(void *p, int64_t n);
SplitkEntry make_splitk_entry(const void *ws, int split, int64_t M, int64_t N, void *C, int64_t ldc,
                              double alpha, double beta);
TauEntry make_tau_entry(int o, int v, const void *t1, const void *t2, const void *oovv, const void *fov,
                        void *tau, void *taut, double *partials);
AsmEntry make_asm_entry(const R2Args &a, const void *XP, const void *Xij, const void *Xab, const void *Xr,
                        void *R, void *t2, double *partials);
int64_t tau_units(int o, int v);
int64_t asm_units(int o, int v);
int64_t t3_units(int o, int v);
PairEntry make_pair_entry(const void *src, void *dst, const int *rows, const int *cols, int64_t nP, int64_t nQ,
                          int64_t ldq, int64_t n1, int64_t n2, int64_t n3, int mode);

// ---- single launches ---------------------------------------------------------
void launch_perm(const PermEntry &e, bool cplx, hipStream_t s);
void launch_outer(const OuterEntry &e, bool cplx, hipStream_t s);
void launch_fill(const FillEntry &e, bool cplx, hipStream_t s);
void launch_splitk(const SplitkEntry &e, bool cplx, hipStream_t s);
void launch_tau(const TauEntry &e, bool cplx, hipStream_t s);
void launch_asm(const AsmEntry &e, bool cplx, hipStream_t s);
void launch_t3(const T3Entry &e, bool cplx, hipStream_t s);
void launch_pair(const PairEntry &e, bool cplx, hipStream_t s);
void launch_r1(const R1Entry &e, bool cplx, hipStream_t s);
void launch_fin(const FinEntry &e, hipStream_t s);

// ---- grouped launches (entries and offsets in device memory) -----------------
void launch_perm_grouped(const PermEntry *e, const int64_t *off, int n, int64_t blocks, bool tiled, bool cplx,
                         hipStream_t s);
void launch_outer_grouped(const OuterEntry *e, const int64_t *off, int n, int64_t blocks, bool cplx, hipStream_t s);
void launch_fill_grouped(const FillEntry *e, const int64_t *off, int n, int64_t blocks, bool cplx, hipStream_t s);
void launch_pair_grouped(const PairEntry *e, const int64_t *off, int n, int64_t blocks, bool cplx, hipStream_t s);
void launch_splitk_grouped(const SplitkEntry *e, const int64_t *off, int n, int64_t blocks, bool cplx,
                           hipStream_t s);
void launch_tau_grouped(const TauEntry *e, const int64_t *off, int n, int64_t blocks, bool cplx, hipStream_t s);
void launch_asm_grouped(const AsmEntry *e, const int64_t *off, int n, int64_t blocks, bool cplx, hipStream_t s);
void launch_r1_grouped(const R1Entry *e, int n, bool cplx, hipStream_t s);
void launch_fin_grouped(const FinEntry *e, int n, hipStream_t s);

// One system's reduced-precision operand copy: n FP64 values to FP32, or to a
// bf16 hi plane followed by the lo plane n elements further (the rounding and
// split of the single-system copies).
struct ConvEntry {
  const double *src;
  void *dst;
  int64_t n;
  int64_t units;  // workgroups
};
ConvEntry make_conv_entry(const double *src, int64_t n, void *dst);
void convert_shadow_grouped(int prec, const ConvEntry *e, const int64_t *off, int n, int64_t blocks,
                            hipStream_t s);
// grouped reduced-precision GEMM reading such copies (lp_in = 1) of
// K-contiguous operands
void gemm_lowp_grouped_launch_lp(const GemmGroupEntry *dev_entries, const int64_t *dev_off, int n,
                                 int64_t blocks, int prec, int tile_id, hipStream_t s);

// ---- conveniences used by the single-system planner --------------------------
void outer_acc(const OuterArgs &a, bool cplx, const void *A, const void *B, void *C, hipStream_t s);
void fill_zero(void *p, int64_t n_elems, bool cplx, hipStream_t s);
void fock_diag(bool cplx, int o, int v, const void *foo, const void *fvv, double *d_oo, double *d_vv,
               hipStream_t s);

}  // namespace ccmi
