/*
 * cc.h -- C ABI of the MI355X coupled-cluster residual engine.
 *
 * The library evaluates the spin-orbital CCD / CCSD energy and amplitude
 * equations
 *
 *     E - E_HF = <Phi_0| exp(-T) H_N exp(T) |Phi_0>
 *     R_l      = <Phi_l| exp(-T) H_N exp(T) |Phi_0>      (paper, Eq. eq:amp)
 *
 * with T = T1 + T2 (paper, Sec. "Coupled cluster amplitude equations") and
 * H_N the normal-ordered Hamiltonian of Eq. ham2q, as a list of binary tensor
 * contractions (the transpose-transpose-GEMM-transpose scheme of Sec.
 * "Tensor contractions"), led by the particle-particle ladder
 * 1/2 sum_cd <ab||cd> tau_ij^cd.  A Jacobi denominator update and the
 * correlation-energy reduction complete one iteration.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Every tensor pointer is DEVICE memory on the context's device, dense and
 *   row-major, 16-byte aligned, and owned by the caller.  The library never
 *   frees caller memory.  Scalars of type CC_R64 are double; CC_C128 are
 *   interleaved (re, im) double pairs.
 * - o = number of occupied spin orbitals, v = number of virtual ones.
 *   Index letters i,j,k,l,m,n run over occupied and a,b,c,d,e,f over virtual
 *   orbitals.  Integral blocks hold <pq||rs> (antisymmetrised, Eq. ham2q):
 *     oooo[i][j][k][l] = <ij||kl>      ooov[i][j][k][a] = <ij||ka>
 *     oovv[i][j][a][b] = <ij||ab>      ovvo[i][a][b][j] = <ia||bj>
 *     ovvv[i][a][b][c] = <ia||bc>      vvvv[a][b][c][d] = <ab||cd>
 *   Every other block follows from antisymmetry and <rs||pq> = conj(<pq||rs>).
 *   Fock blocks: f_oo[i][j], f_ov[i][a], f_vv[a][b] (f_vo = f_ov^H).
 * - Amplitudes: t1[i][a] (o*v), t2[i][j][a][b] (o*o*v*v), antisymmetric in
 *   (i,j) and in (a,b); T2 = 1/4 sum t_ij^ab a+_a a+_b a_j a_i.
 * - Work is enqueued on the context's HIP stream.  Calls that return host
 *   scalars synchronise that stream before returning.
 * - One context per host thread.  No C++ exception crosses this ABI.  Every
 *   call returns CC_OK (0) or a negative cc_status; cc_last_error() gives
 *   a human-readable reason for the last failure on that context.
 */
#ifndef CC_H_
#define CC_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  CC_OK = 0,
  CC_EINVAL = -1,       /* bad argument: null/misaligned pointer, o<1, v<1, t1 vs method */
  CC_ENOMEM = -2,       /* device workspace allocation failed */
  CC_EDEVICE = -3,      /* no usable HIP device, or a HIP runtime error */
  CC_ENOTCONV = -4,     /* cc_iterate reached max_iter above tolerance */
  CC_EDIVERGED = -5,    /* non-finite or growing residual norm */
  CC_EUNSUPPORTED = -6, /* unsupported combination (e.g. precision x scalar) */
  CC_EINTERNAL = -7
} cc_status;

typedef enum { CC_CCD = 0, CC_CCSD = 1 } cc_method;
typedef enum { CC_R64 = 0, CC_C128 = 1 } cc_scalar;
/* Arithmetic of the contractions.  Norms, denominators, the update and the
 * energy are always FP64. */
typedef enum { CC_PREC_F64 = 0, CC_PREC_F32 = 1, CC_PREC_BF16X3 = 2 } cc_prec;

typedef struct cc_ctx cc_ctx;
typedef struct cc_plan cc_plan;
typedef struct cc_batch cc_batch;

/* One system: sizes plus device pointers to the Fock and integral blocks
 * (layouts above).  f_ov may be all zeros but must be a valid pointer. */
typedef struct {
  int32_t o, v;
  int32_t scalar; /* cc_scalar */
  const void *f_oo, *f_ov, *f_vv;
  const void *oooo, *ooov, *oovv, *ovvo, *ovvv, *vvvv;
} cc_system;

/* Amplitudes or residuals.  t1 must be NULL for CC_CCD, non-NULL for CC_CCSD. */
typedef struct {
  void *t1;
  void *t2;
} cc_amps;

/* Standardisation of the amplitude-guess network's features (see the
 * learned initial amplitudes below). */
typedef struct {
  double sx, mD, sD, me, se, st;
} cc_mlp_stats;

/* Starting amplitudes of cc_iterate. */
typedef enum {
  CC_GUESS_GIVEN = 0, /* the amplitudes in t_inout */
  CC_GUESS_MP2 = 1,   /* one bare-denominator Jacobi step from t = 0: t2 = <ab||ij> / D_ij^ab, t1 = f_ai / D_i^a */
  CC_GUESS_MLP = 2    /* the network's t2 (t1 = 0), or the MP2 amplitudes when their residual norm is smaller */
} cc_guess;

typedef struct {
  double tol;          /* stop when ||R(t_n)|| < tol (Frobenius norm over all stored R1, R2) */
  int32_t max_iter;    /* at most this many residual evaluations */
  int32_t prec;        /* cc_prec of the contractions */
  double level_shift;  /* s >= 0: update t <- t + R / (D - s); s = 0 is plain Jacobi */
  double refine_tol;   /* reduced prec: switch to FP64 steps once ||R|| < refine_tol, or when the
                          norm fell by less than 10% over 5 steps (refinement phase) */
  int32_t use_graph;   /* 1: capture one iteration as a HIP graph and replay it */
  int32_t check_every; /* k >= 1: launch k steps, then read their norms and energies back at
                          once (0 counts as 1); decisions on step n act from the next batch on,
                          so up to k - 1 further updates may already be in t_inout when the
                          report (iters, norm, energy of step n) says converged */
  int32_t diverge_window; /* EDIVERGED if the norm grew for this many checks in a row (0 = off) */
  int32_t dressed;     /* 0: D from the bare Fock diagonal; 1: from the diagonals of the
                          T-dressed one-body intermediates of the current iterate */
  int32_t autotune;    /* 1: run the GEMM tile autotuner before iterating (counted as setup) */
  int32_t correction;  /* reduced prec only, 1: in the FP64 phase, evaluate each contraction with
                          >= 1% of the work that is linear in the amplitudes (one constant operand)
                          as a stored FP64 product at reference amplitudes plus a reduced-precision
                          product of the change since the reference (defect correction), and for
                          real systems in split bf16 each product A B of two varying operands as
                          A_ref B_ref + (A - A_ref) B + A_ref (B - B_ref), the last two products
                          in split bf16; a new
                          reference is taken whenever ||R|| fell 1000-fold since the last one,
                          and convergence is confirmed by one plain FP64 step */
  int32_t packed;      /* 1: particle-particle ladder over packed pairs (see CC_PLAN_PACKED_LADDER) */
  int32_t guess;       /* cc_guess: where the iteration starts (0 = t_inout as given); the guess is
                          written to t_inout and its time is part of `seconds` */
  int32_t mlp_prec;    /* CC_GUESS_MLP: CC_PREC_F64 or CC_PREC_F32 network layers */
  const double *mlp_params;      /* CC_GUESS_MLP: device, cc_mlp_num_params() doubles */
  const cc_mlp_stats *mlp_stats; /* CC_GUESS_MLP: host; real systems only (EUNSUPPORTED otherwise) */
} cc_iter_opts;

typedef struct {
  int32_t iters;       /* residual evaluations performed */
  int32_t converged;   /* 1 if ||R|| < tol was reached */
  double rnorm;        /* ||R(t_final)|| */
  double e_re, e_im;   /* E(t_final) - E_HF */
  double seconds;      /* wall time of the loop (setup excluded) */
  double setup_seconds;/* plan creation: derived integral views, workspace */
  int32_t lowp_iters;  /* iterations done in reduced precision before the FP64 phase */
  int32_t corr_iters;  /* FP64-phase iterations that used the reference + correction form */
  double *hist_rnorm;  /* host arrays of capacity hist_cap, or NULL */
  double *hist_e;      /* E per iteration (real part) */
  int32_t hist_cap;
  int32_t guess_used;  /* cc_guess of the start actually used (CC_GUESS_MLP may fall back to MP2) */
  double guess_rnorm_mlp, guess_rnorm_mp2; /* CC_GUESS_MLP: ||R|| of the two candidate starts (FP64) */
  double guess_seconds;/* time spent forming the start (included in seconds) */
} cc_iter_report;

/* ---- context ------------------------------------------------------------ */
/* Binds device `device` and `hip_stream` (a hipStream_t, NULL = a stream the
 * library creates and owns).  Returns CC_EDEVICE when no HIP device exists. */
int cc_create(cc_ctx **ctx, int device, void *hip_stream);
int cc_destroy(cc_ctx *ctx);
const char *cc_last_error(const cc_ctx *ctx);
/* Static error text for a status code. */
const char *cc_status_string(int status);

/* ---- plans: setup once, evaluate many times ------------------------------
 * A plan binds one system (the pointers in *sys are retained, not copied:
 * they must stay valid and unchanged until cc_plan_destroy), a method and a
 * contraction precision.  Creation derives the permuted / conjugated integral
 * views the contraction list needs and allocates the workspace. */
int cc_plan_create(cc_ctx *ctx, const cc_system *sys, int method, int prec, cc_plan **plan);
int cc_plan_destroy(cc_plan *plan);
/* Plan options for cc_plan_create2. */
enum {
  /* Contractions over canonical index pairs only (summands symmetric under
   * the summed pair swap, R antisymmetric): the particle-particle ladder
   * 1/2 sum_ef tau_ij^ef <ab||ef> as one GEMM of o(o-1)/2 x v(v-1)/2 x
   * v(v-1)/2 (eight times fewer operations), the hole-hole ladder
   * 1/2 sum_mn W_mnij tau_mn^ab over m<n, i<j, a<b, and Z_ij^am over e<f,
   * i<j.  Packed copies of vvvv and ovvv are made at plan creation.  Flop
   * counts of such a plan count the packed operations. */
  CC_PLAN_PACKED_LADDER = 1,
  /* Reduced-precision plans run the contractions under 1% of an iteration's
   * flops in FP64 (they are bandwidth- or latency-bound, and FP64 is faster
   * for them as well as exact).  With this flag every contraction runs in
   * the plan's precision, as the batched launches do. */
  CC_PLAN_LOWP_ALL = 2
};
/* cc_plan_create with option flags (0 = cc_plan_create). */
int cc_plan_create2(cc_ctx *ctx, const cc_system *sys, int method, int prec, int flags, cc_plan **plan);
/* A plan whose residual contractions come from the text `ops` instead of the
 * built-in factorised table: the list emitted by the diagram generator
 * (paper, Sec. "Coupled cluster amplitude equations": the equations are
 * derived, then evaluated as binary contractions).  Lines (host memory,
 * copied): "work NAME SPACES" declares an intermediate (SPACES over o/v);
 * "op TAG C cl ALPHA A al B bl [conjA] [conjB] [swap=xy]" accumulates
 * C[cl] += ALPHA * A[al] * B[bl] (summing labels absent from cl; B bl "-"
 * for C[cl] += ALPHA * A[al]); '#' starts a comment.  Index labels i..n run
 * over occupied orbitals, the others over virtual ones.  Tensors: foo, fov,
 * fvv, oooo, ooov, oovv, ovvo, ovvv, vvvv (inputs), t1, t2 (amplitudes),
 * the declared intermediates, and the residual accumulators XP (R2 as is),
 * Xij (R2 += X - X(i<->j)), Xab (R2 += X - X(a<->b)), Xr (both
 * antisymmetrisers) and R1, all labelled ijab / ia; with triples also t3
 * (ijkabc) and Y3 (R3 = full antisymmetriser of Y3, see
 * cc_plan_set_triples).  conjA/conjB conjugate
 * an operand (complex systems).  The energy and norms are computed as for
 * cc_plan_create; dressed denominators are not available (EUNSUPPORTED in
 * cc_plan_step).  A malformed list gives CC_EINVAL with the line number. */
int cc_plan_create_ops(cc_ctx *ctx, const cc_system *sys, int method, int prec, const char *ops,
                       cc_plan **plan);
/* Triples for a CCSD op-list plan that reads t3 or accumulates Y3 (the
 * CCSDT equations of the diagram generator): t3[i][j][k][a][b][c] (device,
 * antisymmetric, o^3 v^3 elements) is read by every residual and updated by
 * cc_plan_step (t3 += R3 / (D_ijk^abc - shift), bare denominators); r3 (or
 * NULL) receives R3 = the full (ijk)x(abc) antisymmetriser of Y3 on every
 * cc_plan_residual.  The residual norm includes R3.  Pointers are kept by
 * the plan until the next call.  CC_EINVAL if the plan has no triples. */
int cc_plan_set_triples(cc_plan *plan, void *t3, void *r3);
/* Workspace bytes held by the plan (derived views + intermediates). */
size_t cc_plan_workspace_bytes(const cc_plan *plan);

/* Residual R(t) (Eq. eq:amp, singles and doubles projections).  r may be
 * NULL (only the norm is produced); r->t1 is ignored for CC_CCD.
 * rnorm_out (host, may be NULL) receives ||R||. */
int cc_plan_residual(cc_plan *plan, const cc_amps *t, cc_amps *r, double *rnorm_out);
/* One Jacobi step: evaluates E(t) and R(t), then t <- t + R/(D - s) in
 * place (D bare, or dressed when dressed != 0: D_ij^ab = F~_ii + F~_jj -
 * F~_aa - F~_bb with F~ the one-body intermediates that multiply t2 in the
 * doubles residual, and D_i^a = F~_ii - F~_aa for the singles).  The scalars
 * are left in device memory; cc_plan_scalars reads them. */
int cc_plan_step(cc_plan *plan, cc_amps *t, double level_shift, int dressed);
/* ||R|| and E (re, im) of the last cc_plan_step / cc_plan_residual (syncs). */
int cc_plan_scalars(cc_plan *plan, double *rnorm, double *e_re, double *e_im);

/* ---- one-shot conveniences ---------------------------------------------- */
/* Residual of the amplitude equations (Eq. eq:amp: the singles and doubles
 * projections of the similarity-transformed normal-ordered Hamiltonian,
 * with T and H_N as in Sec. "Coupled cluster amplitude equations") at the
 * amplitudes t (device, layouts as in cc_amps).  r (device, caller-owned,
 * same layout) receives R1/R2 and may be NULL; rnorm_out (host, may be NULL)
 * receives the Frobenius norm over every stored element of R1 and R2.  A
 * temporary plan is built and freed inside the call.  Errors: CC_EINVAL
 * for bad sizes or method, CC_ENOMEM, CC_EHIP. */
int cc_residual(cc_ctx *ctx, const cc_system *sys, int method, int prec, const cc_amps *t,
                cc_amps *r, double *rnorm_out);
/* E - E_HF = sum f_ia t_i^a + 1/4 sum <ij||ab> tau_ij^ab (first line of Eq. eq:amp). */
int cc_energy(cc_ctx *ctx, const cc_system *sys, int method, const cc_amps *t, double *e_re,
              double *e_im);
/* Solves the amplitude equations of Eq. eq:amp by Jacobi iteration until
 * the residual norm is below opts->tol, the convergence test of Sec.
 * "Correctness: H2O and LiH" (energies compared at a residual-norm
 * threshold).  Starts from the amplitudes in t_inout (device, caller-owned;
 * zeros = the reference, whose first step yields the MP2 amplitudes), or
 * from the guess opts->guess selects (MP2, or the network's t2 with the
 * MP2 amplitudes as fallback: whichever has the smaller FP64 residual norm).  Returns CC_OK, CC_ENOTCONV or
 * CC_EDIVERGED; t_inout holds the last finite iterate, report (host, may be
 * NULL) the per-iteration history. */
int cc_iterate(cc_ctx *ctx, const cc_system *sys, int method, const cc_iter_opts *opts,
               cc_amps *t_inout, cc_iter_report *report);

/* ---- kernel-level entry points (used by the kernel tests) ----------------
 * C[m][n] = alpha * sum_k A(m,k) B(n,k) + beta * C[m][n], row-major C with
 * leading dimension ldc.  A(m,k) = A[m*sam + k*sak] with sam == 1 or sak == 1;
 * B(n,k) = B[n*sbn + k*sbk] with sbn == 1 or sbk == 1.  prec selects the
 * MFMA path (F64: FP64 MFMA; F32: FP32 MFMA on FP64 data rounded to FP32;
 * BF16X3: split-bf16 MFMA), scalar CC_C128 the complex path (F64: complex
 * FP64 MFMA GEMM; F32 / BF16X3: the real GEMM of M x 2N x 2K on the realified
 * operands A' = [Re A, Im A] and B' with rows [Re B, -Im B], [Im B, Re B],
 * whose output is the interleaved complex C).  Accumulation is FP64 for F64,
 * FP32 otherwise.
 * A real GEMM is split along K as a plan would split it (few output tiles,
 * long K; the factor refined for the tile's resident workgroups), and one
 * whose workgroups would end in a mostly empty last round runs as a main part
 * of whole rounds plus the remaining row or column panels split along K into
 * one short round.  Partial sums sit in a device buffer the context keeps
 * (grown on demand, freed by cc_destroy) and are reduced in a fixed order;
 * split parts sum K in a different order than one launch would.
 * CC_GEMM_TAIL=0 in the environment runs every GEMM as one launch.
 * Reduced precision converts A and B once into temporary 4-byte copies; a
 * split-bf16 GEMM on dense K-contiguous rows (sam = sbn = K, K a multiple of
 * 32) whose configuration is LDS-direct takes copies in 16-row x 32-k blocks
 * instead, with identical results (CC_GEMM_BLOCKED=0: row-major copies). */
int cc_gemm(cc_ctx *ctx, int prec, int scalar, int64_t M, int64_t N, int64_t K, double alpha,
            const void *A, int64_t sam, int64_t sak, const void *B, int64_t sbn, int64_t sbk,
            double beta, void *C, int64_t ldc);
/* Number of tile configurations of the real GEMM of precision prec (cc_prec);
 * cc_gemm uses configuration i when the environment variable CC_GEMM_TILE=i
 * is set (tuning sweeps; for complex operands i indexes the complex GEMM's
 * own configurations), its own choice otherwise.  -1 for an unknown prec. */
int cc_gemm_tile_count(int prec);
/* Number of tile configurations of the complex (CC_C128) FP64 GEMM;
 * CC_GEMM_TILE=i selects configuration i of that set (reduced-precision
 * complex GEMMs use the real configurations of their precision). */
int cc_gemm_tile_count_c128(void);
/* cc_gemm with FP64 arithmetic (real, or complex for scalar CC_C128) that
 * allocates nothing, for callers that cannot allocate device memory: code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc.  Arguments, layouts and results are those of cc_gemm with
 * prec CC_PREC_F64 (the default tile choice; CC_GEMM_TILE and CC_GEMM_TAIL
 * are not read).  Scratch: a real GEMM keeps its split-K partial sums (and
 * those of the K-split tail of a launch whose last round would be mostly
 * empty) in a static device buffer of 128 MiB (2^24 doubles) that the
 * library holds on every device it runs on until the process ends; the
 * complex GEMM runs as one launch and uses none.  The split-K factor is
 * cc_gemm's (about 2048 workgroups of 64 x 64 outputs when the output has
 * fewer tiles), so split x M x N stays below 4096 x 4096 < 2^24 doubles;
 * a GEMM whose partial sums would still exceed the buffer is refused with
 * CC_EINVAL and a message giving both sizes, and a tail cut whose partial
 * sums would not fit is skipped (the GEMM then runs as one launch).  The work is only enqueued on the context's stream (no
 * host synchronisation; launch errors are returned, faults surface at the
 * caller's next synchronisation).  Every call on one device shares that
 * device's buffer: calls that overlap in time on one GPU (other streams,
 * contexts or threads) race, calls ordered on one stream do not. */
int cc_gemm_noalloc(cc_ctx *ctx, int scalar, int64_t M, int64_t N, int64_t K, double alpha, const void *A,
                    int64_t sam, int64_t sak, const void *B, int64_t sbn, int64_t sbk, double beta, void *C,
                    int64_t ldc);
/* out[I] = alpha * in[perm(I)] + beta * out[I] for a dense rank-r tensor
 * (r <= 6): out has dims out_dims[0..r-1]; out index d reads input dim
 * perm[d]; in is dense row-major with dims in_dims. */
int cc_permute(cc_ctx *ctx, int scalar, int rank, const int64_t *in_dims, const int32_t *perm,
               double alpha, const void *in, double beta, void *out);

/* ---- batches of independent systems --------------------------------------
 * n systems (each its own o, v and integral blocks; all real or all complex)
 * iterated together.  Each iteration step of the contraction list is ONE
 * grouped launch over all systems; the whole iteration is replayed as one
 * HIP graph.  The amplitude buffers amps[b] are bound at creation (they are
 * updated in place by every step) and must stay valid until destruction.
 * The contraction precision is fixed at creation; batches of complex
 * systems take CC_PREC_F64 only (CC_EUNSUPPORTED otherwise).  Split-K
 * factors follow the tiles of all systems together (fewer K-slices than a
 * system alone would take); with the environment variable
 * CC_BATCH_OWN_SPLITS set at creation each system keeps its own plan's
 * factors, and its results then equal its single-system solve bit for bit.
 * Real systems run the ladder, the hole-hole ladder and Z over packed pairs
 * (i<j, a<b, e<f), as plans created with the packed flag of cc_plan_create2;
 * CC_BATCH_DENSE set at creation keeps them dense. */
int cc_batch_create(cc_ctx *ctx, int n, const cc_system *systems, int method, int prec, cc_amps *amps,
                    cc_batch **batch);
int cc_batch_destroy(cc_batch *batch);
/* One Jacobi step of every system (see cc_plan_step); no host sync. */
int cc_batch_step(cc_batch *batch, double level_shift, int dressed);
/* Per-system ||R||, Re E, Im E of the last step (arrays of n; syncs). */
int cc_batch_scalars(cc_batch *batch, double *rnorm, double *e_re, double *e_im);
/* Choose one GEMM tile configuration per contraction class by timing the
 * grouped launches (FP64 real batches). */
int cc_batch_autotune(cc_batch *batch, int reps);
/* Iterate until every system has ||R|| < tol (converged systems keep being
 * updated, which leaves them converged).  reports: array of n (host); each
 * records the iteration at which its system first met the tolerance and the
 * scalars there.  n_converged (may be NULL) receives the count.  Returns
 * CC_OK, CC_ENOTCONV or CC_EDIVERGED. */
int cc_batch_iterate(cc_batch *batch, const cc_iter_opts *opts, cc_iter_report *reports,
                     int32_t *n_converged);
/* Per-step timing of the grouped launches (see cc_plan_profile). */
int cc_batch_profile(cc_batch *batch, int enable);
const char *cc_batch_profile_table(const cc_batch *batch);
/* Algorithmic flops of one batch iteration (sum over systems). */
double cc_batch_flops(const cc_batch *batch);

/* ---- learned initial amplitudes -------------------------------------------
 * A 3 -> 128 -> 128 -> 1 ReLU network maps the MP2 features of each unique
 * doubles amplitude (i<j, a<b) -- the integral <ij||ab>, the denominator
 * D_ij^ab and the pair energy e_ij = sum_{a<b} <ij||ab>^2 / D_ij^ab -- to
 * t_ij^ab.  With z the standardised features (z0 = x/sx, z1 = (D-mD)/sD,
 * z2 = (e-me)/se) the output is t = st * (g(z) - g(-z0, z1, z2)) / 2, odd in
 * <ij||ab>, so the guess is antisymmetric.  Real systems only.
 * Parameters: cc_mlp_num_params() doubles in device memory, in the order
 * W1[128][3], b1[128], W2[128][128], b2[128], W3[1][128], b3[1].
 * prec: CC_PREC_F64 or CC_PREC_F32 (the dense layers on FP32 MFMA). */
int64_t cc_mlp_num_params(void);
/* number of unique amplitudes, C(o,2) * C(v,2) */
int64_t cc_mlp_num_samples(int o, int v);
/* Features of every unique amplitude in (ij, ab) order into z_out (device,
 * 3 per sample): raw (x, D, e) when stats is NULL, standardised otherwise. */
int cc_mlp_features(cc_ctx *ctx, const cc_system *sys, const cc_mlp_stats *stats, double *z_out);
/* y_out[u] = t2 at unique amplitude u, divided by scale (device). */
int cc_mlp_targets(cc_ctx *ctx, int o, int v, const double *t2, double scale, double *y_out);
/* Column sums over n raw feature rows: out7 = (sum x^2, sum D, sum D^2,
 * sum e, sum e^2, sum y^2 (0 if y is NULL), n) (host). */
int cc_mlp_moments(cc_ctx *ctx, const double *raw, const double *y, int64_t n, double *out7);
/* z_out = standardised raw rows; y_out = y / st when y is non-NULL (device). */
int cc_mlp_standardise(cc_ctx *ctx, const double *raw, const double *y, int64_t n, const cc_mlp_stats *stats,
                       double *z_out, double *y_out);
/* f_out[u] = (g(z_u) - g(z~_u)) / 2 for n standardised rows (device). */
int cc_mlp_forward(cc_ctx *ctx, int prec, const double *params, const double *z, int64_t n, double *f_out);
/* Mean squared error of f against y over n rows and its gradient
 * (device, cc_mlp_num_params() values); loss to host. */
int cc_mlp_loss_grad(cc_ctx *ctx, int prec, const double *params, const double *z, const double *y, int64_t n,
                     double *loss, double *grad_out);
/* Adam training (beta1 0.9, beta2 0.999, eps 1e-8) on minibatches of
 * `batch` consecutive rows of the order permutation (device int64 array of
 * n, or NULL for 0..n-1), for `epochs` passes.  params, adam_m, adam_v are
 * device arrays updated in place; *adam_t counts steps across calls.
 * loss_hist (host, may be NULL) receives the mean minibatch loss per epoch. */
int cc_mlp_train(cc_ctx *ctx, int prec, double *params, double *adam_m, double *adam_v, const double *z,
                 const double *y, int64_t n, const int64_t *order, int64_t batch, int32_t epochs, double lr,
                 int64_t *adam_t, double *loss_hist, int32_t hist_cap);
/* Initial amplitudes from the network: t_out->t2 (all o*o*v*v elements,
 * antisymmetric, zero diagonals) and t_out->t1 = 0 when non-NULL. */
int cc_guess_mlp(cc_ctx *ctx, const cc_system *sys, int prec, const double *params, const cc_mlp_stats *stats,
                 cc_amps *t_out);

/* ---- introspection ------------------------------------------------------ */
/* Text listing of the plan's setup and per-iteration steps (permutes, GEMMs
 * with shapes and tiles, elementwise kernels).  Valid until the next call on
 * the same host thread. */
const char *cc_plan_describe(const cc_plan *plan);
/* The same listing for a plan of the given sizes, built without a device
 * (no allocation, no kernel launch). */
const char *cc_plan_describe_dry(int o, int v, int method, int scalar);
/* Listing of a plan built from a caller-supplied op list (see
 * cc_plan_create_ops), without a device; "error: ..." on a bad list. */
const char *cc_plan_describe_ops_dry(int o, int v, int method, int scalar, const char *ops);
/* Precision of the contractions of the following steps (cc_prec); the
 * plan's creation precision is the initial value. */
int cc_plan_set_precision(cc_plan *plan, int prec);
/* Reference + correction form of the linear (and, real systems with split-bf16
 * corrections, bilinear) contractions for the following FP64 steps (see cc_iter_opts.correction):
 * mode 0 off; mode 1 takes a
 * reference at the next step's amplitudes and uses it from then on; prec
 * (CC_PREC_F32 or CC_PREC_BF16X3) is the precision of the correction
 * products (complex systems: realified products as in cc_gemm). */
int cc_plan_set_correction(cc_plan *plan, int mode, int prec);
/* Autotuner: times every instantiated GEMM tile configuration (of the
 * plan's current precision) for each distinct GEMM shape of the plan (reps launches each, on the plan's own
 * buffers, with t as the amplitude operand) and keeps the fastest.  Choices
 * are cached per shape for the life of the process; if the environment
 * variable CC_AUTOTUNE_CACHE names a file, choices are also read from it at
 * the process's first autotune and new ones appended to it (lines
 * "key tile"), so that separate processes take the same choices.  Workspace
 * contents are clobbered; the next step recomputes them.  t is only read. */
int cc_plan_autotune(cc_plan *plan, const cc_amps *t, int reps);
/* Per-step timing: with enable != 0 every later cc_plan_step /
 * cc_plan_residual records a HIP event after each of its steps on the
 * context stream and waits for the last one; durations accumulate per step.
 * Enabling (again) clears the accumulators. */
int cc_plan_profile(cc_plan *plan, int enable);
/* Table "index kind tag calls total_ms avg_ms flops_per_call", one line per
 * step.  Valid until the next call on the same host thread. */
const char *cc_plan_profile_table(const cc_plan *plan);
/* Algorithmic (dense) flops of one iteration (which = 0) or of the
 * particle-particle ladder alone (which = 1). */
double cc_plan_flops(const cc_plan *plan, int which);

#ifdef __cplusplus
}
#endif
#endif /* CC_H_ */
