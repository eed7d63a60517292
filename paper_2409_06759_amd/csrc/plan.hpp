// Contraction table, planner and executor of the residual path.
#pragma once

#include <map>
#include <memory>
#include <string>
#include <vector>

#include "../../include/cc.h"
#include "kernels.hpp"

struct cc_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  std::string last_error;
  double *pinned = nullptr;  // small pinned host buffer for scalar read-back
  void *gemm_ws = nullptr;   // cc_gemm's tail workspace (grown on demand, freed by cc_destroy)
  int64_t gemm_ws_elems = 0;
};

namespace ccmi {

// One binary (or unary / outer-product) tensor operation of the contraction
// list:  C[cl] += alpha * op(A)[al] * op(B)[bl], optionally followed by the
// antisymmetriser P(xy) over two labels of C (swap = "xy").
struct OpSpec {
  const char *C, *cl;
  double alpha;
  const char *A, *al;
  const char *B, *bl;  // B == nullptr: unary accumulate
  bool conjA, conjB;
  const char *swap;    // nullptr or two labels of C
  bool needs_t1;       // skipped for CCD
  const char *tag;     // short name for profiling
  bool kc = false;     // reduced-precision plans: both GEMM operands K-contiguous (permuted if need be)
};

// Realified copy of a complex slot read as the B operand of reduced-precision
// GEMMs with rows of K complex elements (the layout depends on K).
struct BForm {
  int kind = 0;   // 0: complex realified B' copy; 1: real split-bf16 copy in 16 x 32 blocks (A or B side);
                  // 2, 3: complex realified A', B' split-bf16 copies in 16 x 32 blocks
  int slot = -1;
  int64_t K = 0;
  void *ptr = nullptr;
  int prec = -1;  // precision held (constant slots)
  char ok = 0;    // matches the slot in the current run
};

struct Slot {
  std::string name, spaces;
  std::vector<int64_t> dims;
  int64_t elems = 0;
  void *ptr = nullptr;
  bool constant = false;  // integrals / Fock: unchanged for the plan's lifetime
  bool owned = false;     // allocated by the plan
  bool external = false;  // amplitudes / residual supplied per call
};

struct Step {
  enum Kind { PERMUTE, GEMM, OUTER, FILL, TAU_E, ASSEMBLE, R1UPD, FINALIZE, TRIPLES, PAIR } kind;
  int a = -1, b = -1, c = -1, b2 = -1;  // b2: split-K workspace of a GEMM
  PermDesc perm{};
  GemmDesc gemm{};
  OuterArgs outer{};
  int tile = -1;        // FP64 tile
  int tile_lp[3] = {-1, -1, -1};  // per reduced precision (index = cc_prec)
  int tile_z = -1;      // complex128 tile
  int delta = -1;       // index into cc_plan::deltas (GEMM linear in the amplitudes)
  int bform = -1;       // complex reduced precision: index into cc_plan::bforms of the B operand
  int blk_a = -1, blk_b = -1;  // real split bf16: blocked copies (cc_plan::bforms) of A and B, or -1
  int blk_use = -1;            // autotuner: 1 blocked copies, 0 row-major copies, -1 blocked if the tile reads them
  bool lowp_ok = true;  // runs in the plan's reduced precision (else FP64: under 1% of the work)
  // PAIR: slot a -> slot c through index-pair tables (PairEntry): mode 0
  // gathers packed rows/columns, 1 scatter-adds, 2 scatter-sets; tables:
  // 0 occupied i<j, 1 virtual a<b, 2 (m,a) all, 3 (a,m) all (same order as 2)
  int64_t pair_np = 0, pair_nq = 0, pair_ldq = 0, pair_n[3] = {0, 0, 0};
  int pair_rows = 0, pair_cols = 0, pair_mode = 0;
  int64_t nelem = 0;
  double flops = 0.0;
  std::string tag;
};

// A contraction with one constant operand, evaluated as a stored FP64
// product at reference amplitudes plus a reduced-precision product of the
// change since the reference: C = beta C + alpha X_ref Y + alpha (X - X_ref) Y.
struct DeltaRef {
  int step = -1;
  int var = 0;                    // 0: A varies, 1: B varies, 2: both vary (real systems)
  int64_t n_op = 0;               // elements of the varying operand's slot (var 2: A's)
  double *ref_op = nullptr;       // FP64 copy of the varying operand at the reference (var 2: A_ref)
  double *ref_out = nullptr;      // alpha * X_ref Y, dense M x N (var 2: alpha * A_ref B_ref)
  void *dshadow = nullptr;        // reduced-precision (X - X_ref) (var 2: A - A_ref)
  void *dblk = nullptr;           // split bf16 (X - X_ref) in 16 x 32 blocks (steps with blocked copies)
  // var 2: A B = A_ref B_ref + (A - A_ref) B + A_ref (B - B_ref)
  int64_t n_b = 0;                // elements of B's slot
  double *ref_b = nullptr;        // FP64 B_ref
  void *ref_a_lp = nullptr;       // reduced-precision A_ref (made at the reference)
  void *cur_b_lp = nullptr;       // reduced-precision B
  void *dshadow_b = nullptr;      // reduced-precision (B - B_ref)
};

// A caller-supplied contraction list (e.g. emitted by the diagram
// generator): intermediates to allocate and binary / unary ops in the
// format of the built-in table, with owned strings.
struct OpText {
  std::string C, cl, A, al, B, bl, swap, tag;
  double alpha = 1.0;
  bool conjA = false, conjB = false;
};
struct OpList {
  std::vector<std::pair<std::string, std::string>> work;  // name, spaces
  std::vector<OpText> ops;
};
// Parses "work NAME SPACES" and "op TAG C cl ALPHA A al B bl [conjA] [conjB]
// [swap=xy]" lines (B and bl "-" for a unary accumulate; '#' comments).
OpList parse_op_list(const char *text);

}  // namespace ccmi

struct cc_plan {
  cc_ctx *ctx = nullptr;
  int o = 0, v = 0, method = 0, prec = 0;
  int cur_prec = 0;  // precision of the contractions in the next run
  bool cplx = false;
  size_t esize = 8;
  std::shared_ptr<ccmi::OpList> custom;  // null: the built-in contraction table
  // particle-particle ladder over packed pairs (i<j, e<f, a<b)
  bool packed = false;
  bool lowp_all = false;  // every contraction in the reduced precision (else small ones in FP64)
  // every GEMM gets its own output scratch and split-K workspace (batched
  // plans, whose steps may run concurrently), instead of one shared buffer each
  bool private_work = false;
  int *pair_tab[4] = {nullptr, nullptr, nullptr, nullptr};  // device index-pair tables
  // triples (op lists that read t3 or accumulate Y3): bound per plan
  bool triples = false;
  void *t3 = nullptr, *r3_out = nullptr;
  double *n3part = nullptr;
  int n_n3part = 0;
  std::vector<ccmi::Slot> slots;
  std::map<std::string, int> index;
  std::vector<ccmi::Step> setup, iter;
  std::map<std::string, int> view_cache;  // (tensor, labels, conj, version) -> slot
  std::map<int, int> version;             // writes seen so far while planning
  std::map<int, bool> touched;            // first write of an iteration uses beta = 0
  size_t workspace = 0;
  // scalar machinery (device)
  double *d_oo = nullptr, *d_vv = nullptr;
  double *epart = nullptr, *n2part = nullptr, *n1part = nullptr, *scalars = nullptr;
  int n_epart = 0, n_n2part = 0;
  // per-call state
  void *t1 = nullptr, *t2 = nullptr, *r1_out = nullptr, *r2_out = nullptr;
  bool update = false;
  double shift = 0.0;
  int dressed = 0;
  // graph replay
  hipGraphExec_t graph = nullptr;
  void *graph_key[4] = {nullptr, nullptr, nullptr, nullptr};
  double graph_shift = 0.0;
  bool graph_update = false;
  int graph_dressed = 0;
  int graph_prec = -1;
  double flops_per_iter = 0.0, ladder_flops = 0.0;
  std::vector<ccmi::Step *> gemm_steps;
  // per-step timing (HIP events around every step of an iteration)
  bool profiling = false;
  std::vector<hipEvent_t> events;
  std::vector<double> step_ms;   // accumulated per iteration step
  std::vector<int64_t> step_calls;
  // reduced-precision operand copies (4 bytes per real element), per slot:
  // the slot's elements in their own order (complex: re, im interleaved,
  // which is also the realified A' of a dense K-contiguous complex operand)
  std::vector<void *> shadow;
  std::vector<int> shadow_prec;   // precision held by a constant slot's copy
  std::vector<char> shadow_ok;    // copy matches the slot in the current run
  // complex slots read as the B operand of a reduced-precision GEMM: the
  // realified B' (rows [Re, -Im] and [Im, Re]), one copy per (slot, K)
  std::vector<ccmi::BForm> bforms;
  // reference + correction mode of the FP64 contractions (0 off, 1 use the
  // stored reference, 2 take a new reference in the next run)
  int delta_mode = 0;
  int delta_prec = 1;             // precision of the correction products
  std::vector<ccmi::DeltaRef> deltas;
  int graph_delta = -1;
};

namespace ccmi {
void plan_layout(cc_plan *p, const cc_system *sys);  // planning only, no device work
void plan_build(cc_plan *p, const cc_system *sys);
void plan_free(cc_plan *p);
void plan_run(cc_plan *p);           // enqueue one residual (+ update) on the stream
void plan_prepare(cc_plan *p);       // allocate / refresh operand copies; never under capture
void plan_run_energy(cc_plan *p);    // tau + energy only
std::string plan_describe(const cc_plan *p);
void plan_autotune(cc_plan *p, int reps);
std::string plan_profile_table(const cc_plan *p);
TauEntry tau_entry(cc_plan *p);
T3Entry t3_entry(cc_plan *p);
AsmEntry asm_entry(cc_plan *p);
R1Entry r1_entry(cc_plan *p);
FinEntry fin_entry(cc_plan *p);
void *ptr_of(cc_plan *p, int slot);
cc_plan *make_plan_checked(cc_ctx *ctx, const cc_system *sys, int method, int prec, bool lowp_all = false,
                           bool private_work = false, bool packed = false);
void check_amps(const cc_amps *t, int method);
}  // namespace ccmi
