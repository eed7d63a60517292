// Launchers of the device kernels (declarations shared by the host code).
#pragma once

#include "common.hpp"

#include <algorithm>

namespace ccmi {

struct OuterArgs {
  int rank;
  int64_t dims[4];
  int64_t sa[4], sb[4];  // strides of A and B for each C dimension (0 = not indexed)
  double alpha;
  int conj_a, conj_b;
};

struct R2Args {
  int o, v;
  const double *fdiag_o, *fdiag_v;  // bare Fock diagonals
  double shift;
  int dressed;                      // 1: denominators from the dressed one-body diagonals
  const void *Fo, *Fv;              // dressed [o][o] and [v][v] one-body intermediates
};

void outer_acc(const OuterArgs &a, bool cplx, const void *A, const void *B, void *C, hipStream_t s);
void fill_zero(void *p, int64_t n_elems, bool cplx, hipStream_t s);

int tau_energy_blocks(int o, int v);
void tau_energy(bool cplx, int o, int v, const void *t1, const void *t2, const void *oovv,
                const void *fov, void *tau, void *taut, double *partials, hipStream_t s);

int64_t r2_assemble_blocks(int o, int v);
void r2_assemble(bool cplx, const R2Args &a, const void *XP, const void *Xij, const void *Xab,
                 const void *Xr, void *R, void *t2, double *partials, hipStream_t s);
void r1_update(bool cplx, int o, int v, const void *R1, void *t1, const double *d_oo,
               const double *d_vv, double shift, int dressed, const void *Fo, const void *Fv,
               double *partial, hipStream_t s);
void fock_diag(bool cplx, int o, int v, const void *foo, const void *fvv, double *d_oo,
               double *d_vv, hipStream_t s);
void finalize_scalars(const double *epart, int ne, const double *n2part, int nn,
                      const double *n1part, double *scalars, hipStream_t s);

}  // namespace ccmi
