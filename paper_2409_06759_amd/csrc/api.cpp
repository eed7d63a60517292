// C ABI of the engine: validation, error mapping and the Jacobi driver.
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <string>
#include <vector>

#include "plan.hpp"

using ccmi::CCError;

namespace {

thread_local std::string g_last_error;

int fail(cc_ctx *ctx, int status, const std::string &msg) {
  if (ctx) ctx->last_error = msg;
  g_last_error = msg;
  return status;
}

template <class F>
int guarded(cc_ctx *ctx, F &&f) {
  try {
    return f();
  } catch (const CCError &e) {
    return fail(ctx, e.status, e.what());
  } catch (const std::bad_alloc &) {
    return fail(ctx, CC_ENOMEM, "host allocation failed");
  } catch (const std::exception &e) {
    return fail(ctx, CC_EINTERNAL, e.what());
  }
}

bool aligned(const void *p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

void check_ptr(const void *p, const char *what) {
  if (p == nullptr) throw CCError(CC_EINVAL, std::string(what) + " is NULL");
  if (!aligned(p)) throw CCError(CC_EINVAL, std::string(what) + " is not 16-byte aligned");
}

void validate_system(const cc_system *s) {
  if (!s) throw CCError(CC_EINVAL, "system is NULL");
  if (s->o < 1 || s->v < 1) throw CCError(CC_EINVAL, "o and v must be >= 1");
  if (int64_t(s->o) * s->o * s->v * s->v > (int64_t(1) << 40))
    throw CCError(CC_EINVAL, "system too large");
  if (s->scalar != CC_R64 && s->scalar != CC_C128) throw CCError(CC_EINVAL, "unknown scalar type");
  check_ptr(s->f_oo, "f_oo");
  check_ptr(s->f_ov, "f_ov");
  check_ptr(s->f_vv, "f_vv");
  check_ptr(s->oooo, "oooo");
  check_ptr(s->ooov, "ooov");
  check_ptr(s->oovv, "oovv");
  check_ptr(s->ovvo, "ovvo");
  check_ptr(s->ovvv, "ovvv");
  check_ptr(s->vvvv, "vvvv");
}

void validate_method(int method, int prec, int scalar) {
  if (method != CC_CCD && method != CC_CCSD) throw CCError(CC_EINVAL, "unknown method");
  if (prec != CC_PREC_F64 && prec != CC_PREC_F32 && prec != CC_PREC_BF16X3)
    throw CCError(CC_EINVAL, "unknown precision");
}

void validate_amps(const cc_amps *t, int method, const char *what) {
  if (!t) throw CCError(CC_EINVAL, std::string(what) + " is NULL");
  check_ptr(t->t2, (std::string(what) + ".t2").c_str());
  if (method == CC_CCSD) check_ptr(t->t1, (std::string(what) + ".t1").c_str());
  if (method == CC_CCD && t->t1 != nullptr)
    throw CCError(CC_EINVAL, std::string(what) + ".t1 must be NULL for CCD");
}

void set_device(cc_ctx *ctx) { CC_HIP_CHECK(hipSetDevice(ctx->device)); }

void read_scalars(cc_plan *p, double *rn, double *er, double *ei) {
  cc_ctx *ctx = p->ctx;
  CC_HIP_CHECK(hipMemcpyAsync(ctx->pinned, p->scalars, 3 * sizeof(double), hipMemcpyDeviceToHost,
                              ctx->stream));
  CC_HIP_CHECK(hipStreamSynchronize(ctx->stream));
  if (rn) *rn = ctx->pinned[0];
  if (er) *er = ctx->pinned[1];
  if (ei) *ei = ctx->pinned[2];
}

// One update step; replays a captured graph when asked and when the
// amplitude pointers and shift match the capture.
void run_step(cc_plan *p, bool use_graph) {
  ccmi::plan_prepare(p);
  if (!use_graph || p->delta_mode == 2) {  // a reference run is never captured
    ccmi::plan_run(p);
    return;
  }
  const bool same = p->graph && p->graph_key[0] == p->t1 && p->graph_key[1] == p->t2 &&
                    p->graph_key[2] == p->r1_out && p->graph_key[3] == p->r2_out &&
                    p->graph_shift == p->shift && p->graph_update == p->update &&
                    p->graph_dressed == p->dressed && p->graph_prec == p->cur_prec &&
                    p->graph_delta == p->delta_mode;
  if (!same) {
    if (p->graph) (void)hipGraphExecDestroy(p->graph);
    p->graph = nullptr;
    hipGraph_t g;
    CC_HIP_CHECK(hipStreamBeginCapture(p->ctx->stream, hipStreamCaptureModeThreadLocal));
    try {
      ccmi::plan_run(p);
    } catch (...) {
      hipGraph_t dummy;
      (void)hipStreamEndCapture(p->ctx->stream, &dummy);
      throw;
    }
    CC_HIP_CHECK(hipStreamEndCapture(p->ctx->stream, &g));
    CC_HIP_CHECK(hipGraphInstantiate(&p->graph, g, nullptr, nullptr, 0));
    (void)hipGraphDestroy(g);
    p->graph_key[0] = p->t1;
    p->graph_key[1] = p->t2;
    p->graph_key[2] = p->r1_out;
    p->graph_key[3] = p->r2_out;
    p->graph_shift = p->shift;
    p->graph_update = p->update;
    p->graph_dressed = p->dressed;
    p->graph_prec = p->cur_prec;
    p->graph_delta = p->delta_mode;
  }
  CC_HIP_CHECK(hipGraphLaunch(p->graph, p->ctx->stream));
}

// Eager evaluation of the plan at (t1, t2) in FP64: a bare Jacobi update in
// place (update) or only R and the scalars; the plan's per-call state is
// restored afterwards.  Returns ||R(t)||.
double eval_fp64(cc_plan *p, void *t1, void *t2, bool update) {
  void *o1 = p->t1, *o2 = p->t2, *r1 = p->r1_out, *r2 = p->r2_out;
  const bool ou = p->update;
  const int od = p->dressed, op = p->cur_prec, om = p->delta_mode;
  const double os = p->shift;
  p->t1 = t1;
  p->t2 = t2;
  p->r1_out = p->r2_out = nullptr;
  p->update = update;
  p->dressed = 0;
  p->shift = 0.0;
  p->cur_prec = CC_PREC_F64;
  p->delta_mode = 0;
  double rn = NAN, er = NAN, ei = NAN;
  try {
    ccmi::plan_run(p);
    read_scalars(p, &rn, &er, &ei);
  } catch (...) {
    p->t1 = o1; p->t2 = o2; p->r1_out = r1; p->r2_out = r2; p->update = ou;
    p->dressed = od; p->shift = os; p->cur_prec = op; p->delta_mode = om;
    throw;
  }
  p->t1 = o1; p->t2 = o2; p->r1_out = r1; p->r2_out = r2; p->update = ou;
  p->dressed = od; p->shift = os; p->cur_prec = op; p->delta_mode = om;
  return rn;
}

// The MP2 amplitudes: one bare-denominator Jacobi step from t = 0.
void mp2_start(cc_plan *p, void *t1, void *t2) {
  hipStream_t s = p->ctx->stream;
  const size_t n1 = size_t(p->o) * p->v * p->esize, n2 = n1 * size_t(p->o) * p->v;
  CC_HIP_CHECK(hipMemsetAsync(t2, 0, n2, s));
  if (t1) CC_HIP_CHECK(hipMemsetAsync(t1, 0, n1, s));
  (void)eval_fp64(p, t1, t2, true);
}

// Writes the start opts->guess selects into t; returns the cc_guess used.
int form_guess(cc_ctx *ctx, const cc_system *sys, cc_plan *p, const cc_iter_opts *opts, cc_amps *t,
               double *rn_mlp, double *rn_mp2) {
  if (opts->guess == CC_GUESS_MP2) {
    mp2_start(p, t->t1, t->t2);
    return CC_GUESS_MP2;
  }
  cc_amps g{t->t1, t->t2};
  const int st = cc_guess_mlp(ctx, sys, opts->mlp_prec, opts->mlp_params, opts->mlp_stats, &g);
  if (st != CC_OK) throw CCError(st, ctx->last_error);
  *rn_mlp = eval_fp64(p, t->t1, t->t2, false);
  const size_t n1 = size_t(p->o) * p->v * p->esize, n2 = n1 * size_t(p->o) * p->v;
  void *m1 = nullptr, *m2 = nullptr;
  CC_HIP_CHECK(hipMalloc(&m2, n2));
  if (t->t1 && hipMalloc(&m1, n1) != hipSuccess) {
    (void)hipFree(m2);
    throw CCError(CC_ENOMEM, "guess buffers");
  }
  int used = CC_GUESS_MLP;
  try {
    mp2_start(p, m1, m2);
    *rn_mp2 = eval_fp64(p, m1, m2, false);
    if (*rn_mp2 < *rn_mlp) {
      CC_HIP_CHECK(hipMemcpyAsync(t->t2, m2, n2, hipMemcpyDeviceToDevice, p->ctx->stream));
      if (t->t1) CC_HIP_CHECK(hipMemcpyAsync(t->t1, m1, n1, hipMemcpyDeviceToDevice, p->ctx->stream));
      used = CC_GUESS_MP2;
    }
    CC_HIP_CHECK(hipStreamSynchronize(p->ctx->stream));
  } catch (...) {
    (void)hipStreamSynchronize(p->ctx->stream);
    (void)hipFree(m2);
    if (m1) (void)hipFree(m1);
    throw;
  }
  (void)hipFree(m2);
  if (m1) (void)hipFree(m1);
  return used;
}

cc_plan *make_plan(cc_ctx *ctx, const cc_system *sys, int method, int prec,
                   std::shared_ptr<ccmi::OpList> custom = nullptr, bool packed = false, bool lowp_all = false,
                   bool private_work = false) {
  validate_system(sys);
  validate_method(method, prec, sys->scalar);
  set_device(ctx);
  cc_plan *p = new cc_plan();
  p->custom = std::move(custom);
  p->packed = packed;
  p->lowp_all = lowp_all;
  p->private_work = private_work;
  p->ctx = ctx;
  p->o = sys->o;
  p->v = sys->v;
  p->method = method;
  p->prec = prec;
  p->cur_prec = prec;
  p->cplx = sys->scalar == CC_C128;
  p->esize = p->cplx ? 16 : 8;
  try {
    ccmi::plan_build(p, sys);
  } catch (...) {
    ccmi::plan_free(p);
    delete p;
    throw;
  }
  return p;
}

}  // namespace

namespace ccmi {
cc_plan *make_plan_checked(cc_ctx *ctx, const cc_system *sys, int method, int prec, bool lowp_all,
                           bool private_work, bool packed) {
  return make_plan(ctx, sys, method, prec, nullptr, packed, lowp_all, private_work);
}
void check_amps(const cc_amps *t, int method) { validate_amps(t, method, "t"); }
}  // namespace ccmi

extern "C" {

const char *cc_status_string(int s) {
  switch (s) {
    case CC_OK: return "ok";
    case CC_EINVAL: return "invalid argument";
    case CC_ENOMEM: return "out of device memory";
    case CC_EDEVICE: return "device error";
    case CC_ENOTCONV: return "not converged";
    case CC_EDIVERGED: return "diverged";
    case CC_EUNSUPPORTED: return "unsupported";
    case CC_EINTERNAL: return "internal error";
    default: return "unknown status";
  }
}

const char *cc_last_error(const cc_ctx *ctx) {
  return ctx ? ctx->last_error.c_str() : g_last_error.c_str();
}

int cc_create(cc_ctx **out, int device, void *stream) {
  if (!out) return fail(nullptr, CC_EINVAL, "ctx pointer is NULL");
  *out = nullptr;
  return guarded(nullptr, [&] {
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || n == 0) {
      (void)hipGetLastError();
      throw CCError(CC_EDEVICE, "no HIP device available");
    }
    if (device < 0 || device >= n) throw CCError(CC_EINVAL, "device index out of range");
    CC_HIP_CHECK(hipSetDevice(device));
    cc_ctx *c = new cc_ctx();
    c->device = device;
    if (stream) {
      c->stream = static_cast<hipStream_t>(stream);
    } else {
      if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess) {
        delete c;
        throw CCError(CC_EDEVICE, "stream creation failed");
      }
      c->own_stream = true;
    }
    if (hipHostMalloc(reinterpret_cast<void **>(&c->pinned), 64, hipHostMallocDefault) != hipSuccess) {
      if (c->own_stream) (void)hipStreamDestroy(c->stream);
      delete c;
      throw CCError(CC_EDEVICE, "pinned host allocation failed");
    }
    *out = c;
    return CC_OK;
  });
}

int cc_destroy(cc_ctx *ctx) {
  if (!ctx) return CC_OK;
  (void)hipSetDevice(ctx->device);
  if (ctx->pinned) (void)hipHostFree(ctx->pinned);
  if (ctx->gemm_ws) {
    (void)hipStreamSynchronize(ctx->stream);
    (void)hipFree(ctx->gemm_ws);
  }
  if (ctx->own_stream) (void)hipStreamDestroy(ctx->stream);
  delete ctx;
  return CC_OK;
}

int cc_plan_create(cc_ctx *ctx, const cc_system *sys, int method, int prec, cc_plan **plan) {
  if (!ctx) return fail(nullptr, CC_EINVAL, "ctx is NULL");
  if (!plan) return fail(ctx, CC_EINVAL, "plan pointer is NULL");
  *plan = nullptr;
  return guarded(ctx, [&] {
    *plan = make_plan(ctx, sys, method, prec);
    return CC_OK;
  });
}

int cc_plan_create2(cc_ctx *ctx, const cc_system *sys, int method, int prec, int flags, cc_plan **plan) {
  if (!ctx) return fail(nullptr, CC_EINVAL, "ctx is NULL");
  if (!plan) return fail(ctx, CC_EINVAL, "plan pointer is NULL");
  *plan = nullptr;
  return guarded(ctx, [&] {
    if (flags & ~int(CC_PLAN_PACKED_LADDER | CC_PLAN_LOWP_ALL)) throw CCError(CC_EINVAL, "unknown plan flags");
    *plan = make_plan(ctx, sys, method, prec, nullptr, (flags & CC_PLAN_PACKED_LADDER) != 0,
                      (flags & CC_PLAN_LOWP_ALL) != 0);
    return CC_OK;
  });
}

int cc_plan_create_ops(cc_ctx *ctx, const cc_system *sys, int method, int prec, const char *ops,
                       cc_plan **plan) {
  if (!ctx) return fail(nullptr, CC_EINVAL, "ctx is NULL");
  if (!plan) return fail(ctx, CC_EINVAL, "plan pointer is NULL");
  *plan = nullptr;
  return guarded(ctx, [&] {
    auto list = std::make_shared<ccmi::OpList>(ccmi::parse_op_list(ops));
    *plan = make_plan(ctx, sys, method, prec, list);
    return CC_OK;
  });
}

int cc_plan_set_triples(cc_plan *p, void *t3, void *r3) {
  if (!p) return fail(nullptr, CC_EINVAL, "plan is NULL");
  return guarded(p->ctx, [&] {
    if (!p->triples) throw CCError(CC_EINVAL, "the plan's contraction list has no triples");
    check_ptr(t3, "t3");
    if (r3) check_ptr(r3, "r3");
    p->t3 = t3;
    p->r3_out = r3;
    return CC_OK;
  });
}

int cc_plan_destroy(cc_plan *p) {
  if (!p) return CC_OK;
  (void)hipSetDevice(p->ctx->device);
  (void)hipStreamSynchronize(p->ctx->stream);
  ccmi::plan_free(p);
  delete p;
  return CC_OK;
}

size_t cc_plan_workspace_bytes(const cc_plan *p) { return p ? p->workspace : 0; }

int cc_plan_residual(cc_plan *p, const cc_amps *t, cc_amps *r, double *rnorm_out) {
  if (!p) return fail(nullptr, CC_EINVAL, "plan is NULL");
  return guarded(p->ctx, [&] {
    validate_amps(t, p->method, "t");
    if (r) validate_amps(r, p->method, "r");
    set_device(p->ctx);
    p->t1 = t->t1;
    p->t2 = t->t2;
    p->r1_out = r ? r->t1 : nullptr;
    p->r2_out = r ? r->t2 : nullptr;
    p->update = false;
    p->shift = 0.0;
    ccmi::plan_run(p);
    if (rnorm_out) read_scalars(p, rnorm_out, nullptr, nullptr);
    else CC_HIP_CHECK(hipStreamSynchronize(p->ctx->stream));
    return CC_OK;
  });
}

int cc_plan_step(cc_plan *p, cc_amps *t, double level_shift, int dressed) {
  if (!p) return fail(nullptr, CC_EINVAL, "plan is NULL");
  return guarded(p->ctx, [&] {
    validate_amps(t, p->method, "t");
    if (!(level_shift >= 0.0) || !std::isfinite(level_shift))
      throw CCError(CC_EINVAL, "level_shift must be finite and >= 0");
    set_device(p->ctx);
    p->t1 = t->t1;
    p->t2 = t->t2;
    p->r1_out = nullptr;
    p->r2_out = nullptr;
    p->update = true;
    if (dressed && p->custom)
      throw CCError(CC_EUNSUPPORTED, "dressed denominators need the built-in contraction table");
    p->shift = level_shift;
    p->dressed = dressed ? 1 : 0;
    ccmi::plan_run(p);
    CC_HIP_CHECK(hipGetLastError());
    return CC_OK;
  });
}

int cc_plan_scalars(cc_plan *p, double *rn, double *er, double *ei) {
  if (!p) return fail(nullptr, CC_EINVAL, "plan is NULL");
  return guarded(p->ctx, [&] {
    set_device(p->ctx);
    read_scalars(p, rn, er, ei);
    return CC_OK;
  });
}

int cc_residual(cc_ctx *ctx, const cc_system *sys, int method, int prec, const cc_amps *t,
                cc_amps *r, double *rnorm_out) {
  if (!ctx) return fail(nullptr, CC_EINVAL, "ctx is NULL");
  return guarded(ctx, [&] {
    validate_amps(t, method, "t");
    if (r) validate_amps(r, method, "r");
    cc_plan *p = make_plan(ctx, sys, method, prec);
    int st = cc_plan_residual(p, t, r, rnorm_out);
    cc_plan_destroy(p);
    return st;
  });
}

int cc_energy(cc_ctx *ctx, const cc_system *sys, int method, const cc_amps *t, double *e_re,
              double *e_im) {
  if (!ctx) return fail(nullptr, CC_EINVAL, "ctx is NULL");
  return guarded(ctx, [&] {
    validate_amps(t, method, "t");
    cc_plan *p = make_plan(ctx, sys, method, CC_PREC_F64);
    try {
      p->t1 = t->t1;
      p->t2 = t->t2;
      ccmi::plan_run_energy(p);
      read_scalars(p, nullptr, e_re, e_im);
    } catch (...) {
      cc_plan_destroy(p);
      throw;
    }
    cc_plan_destroy(p);
    return CC_OK;
  });
}

int cc_iterate(cc_ctx *ctx, const cc_system *sys, int method, const cc_iter_opts *opts,
               cc_amps *t, cc_iter_report *rep) {
  if (!ctx) return fail(nullptr, CC_EINVAL, "ctx is NULL");
  return guarded(ctx, [&] {
    if (!opts) throw CCError(CC_EINVAL, "opts is NULL");
    if (opts->max_iter < 1) throw CCError(CC_EINVAL, "max_iter must be >= 1");
    if (!(opts->tol > 0.0)) throw CCError(CC_EINVAL, "tol must be > 0");
    if (!(opts->level_shift >= 0.0)) throw CCError(CC_EINVAL, "level_shift must be >= 0");
    if (opts->guess < CC_GUESS_GIVEN || opts->guess > CC_GUESS_MLP) throw CCError(CC_EINVAL, "unknown guess");
    if (opts->guess == CC_GUESS_MLP) {
      if (!opts->mlp_params || !opts->mlp_stats) throw CCError(CC_EINVAL, "MLP guess needs parameters and stats");
      if (sys && sys->scalar != CC_R64) throw CCError(CC_EUNSUPPORTED, "the amplitude-guess network is real-valued");
    }
    validate_amps(t, method, "t");
    const auto t0 = std::chrono::steady_clock::now();
    cc_plan *p = make_plan(ctx, sys, method, opts->prec, nullptr, opts->packed != 0);
    int status = CC_ENOTCONV;
    int iters = 0;
    double rn = NAN, er = NAN, ei = NAN, best = INFINITY;
    int grew = 0;
    std::vector<double> seen;  // norms seen in the current precision
    int switched_at = -1;
    int corr_iters = 0;
    double ref_rn = INFINITY;   // norm at the last reference (correction form)
    bool confirming = false;    // the next step is the plain FP64 confirmation
    const bool use_corr = opts->correction != 0 && opts->prec != CC_PREC_F64 && !p->deltas.empty();
    if (use_corr) p->delta_prec = opts->prec;
    std::chrono::steady_clock::time_point t1c;
    int guess_used = CC_GUESS_GIVEN;
    double g_mlp = NAN, g_mp2 = NAN, guess_s = 0.0;
    // CC_ITERATE_PROGRESS=n: one line on stderr every n iterations (long runs)
    const char *pv = std::getenv("CC_ITERATE_PROGRESS");
    const int progress = pv ? std::atoi(pv) : 0;
    try {
      p->t1 = t->t1;
      p->t2 = t->t2;
      p->r1_out = p->r2_out = nullptr;
      p->update = true;
      p->shift = opts->level_shift;
      p->dressed = opts->dressed ? 1 : 0;
      if (opts->autotune) {
        for (int pr : {opts->prec, int(CC_PREC_F64)}) {
          p->cur_prec = pr;
          ccmi::plan_autotune(p, 1);
        }
        p->cur_prec = opts->prec;
      }
      ccmi::plan_prepare(p);
      CC_HIP_CHECK(hipStreamSynchronize(p->ctx->stream));
      t1c = std::chrono::steady_clock::now();
      if (opts->guess != CC_GUESS_GIVEN) {
        guess_used = form_guess(ctx, sys, p, opts, t, &g_mlp, &g_mp2);
        guess_s = std::chrono::duration<double>(std::chrono::steady_clock::now() - t1c).count();
      }
      // Steps are launched in batches of check_every; each step's three
      // scalars are copied to pinned memory asynchronously and the batch is
      // examined after one synchronisation.  Decisions taken while examining
      // step n (convergence, precision switch, new reference) apply from the
      // next batch on, so up to check_every - 1 further steps may already
      // have updated t; the report describes step n.
      const int k = std::max(1, opts->check_every);
      double *hbuf = nullptr;
      if (hipHostMalloc(reinterpret_cast<void **>(&hbuf), sizeof(double) * 3 * k, hipHostMallocDefault) !=
          hipSuccess) {
        (void)hipGetLastError();
        throw CCError(CC_ENOMEM, "pinned host allocation failed");
      }
      std::vector<int> modes(k), precs(k);
      bool done = false;
      int it = 0;
      try {
        while (it < opts->max_iter && !done) {
          const int nb = std::min(k, opts->max_iter - it);
          for (int q = 0; q < nb; ++q) {
            modes[q] = p->delta_mode;
            precs[q] = p->cur_prec;
            run_step(p, opts->use_graph != 0);
            CC_HIP_CHECK(hipMemcpyAsync(hbuf + 3 * q, p->scalars, 3 * sizeof(double), hipMemcpyDeviceToHost,
                                        p->ctx->stream));
          }
          CC_HIP_CHECK(hipStreamSynchronize(p->ctx->stream));
          for (int q = 0; q < nb && !done; ++q, ++it) {
            const int mode_now = modes[q], prec_now = precs[q];
            ++iters;
            if (mode_now != 0) ++corr_iters;
            rn = hbuf[3 * q];
            er = hbuf[3 * q + 1];
            ei = hbuf[3 * q + 2];
            if (mode_now == 2) {
              ref_rn = rn;
            } else if (mode_now == 1 && rn < 1e-3 * ref_rn && p->delta_mode == 1) {
              p->delta_mode = 2;  // refresh the reference at the next step
            }
            if (progress > 0 && iters % progress == 0)
              std::fprintf(stderr, "cc_iterate: iteration %d ||R|| %.6e E %.12f%s\n", iters, rn, er,
                           prec_now != CC_PREC_F64 ? " (reduced precision)" : mode_now ? " (corrected)" : "");
            if (rep && rep->hist_rnorm && it < rep->hist_cap) rep->hist_rnorm[it] = rn;
            if (rep && rep->hist_e && it < rep->hist_cap) rep->hist_e[it] = er;
            if (!std::isfinite(rn) || !std::isfinite(er)) {
              status = CC_EDIVERGED;
              done = true;
              break;
            }
            if (rn < opts->tol && prec_now == CC_PREC_F64) {
              if (mode_now != 1) {  // plain or reference step: an FP64 evaluation
                status = CC_OK;
                done = true;
                break;
              }
              // correction form reached tol: confirm with a plain FP64 step
              p->delta_mode = 0;
              confirming = true;
            } else if (confirming && std::isfinite(rn)) {
              confirming = false;  // not confirmed: stay with plain FP64 steps
            }
            if (prec_now != CC_PREC_F64 && p->cur_prec != CC_PREC_F64) {
              // refinement: leave reduced precision once the norm is below
              // refine_tol or has stopped falling (less than 10% over 5 steps);
              // the following FP64 steps correct the reduced-precision iterate.
              seen.push_back(rn);
              const size_t n = seen.size();
              const bool stagnant = n > 5 && seen[n - 1] > 0.9 * seen[n - 6];
              if (rn < std::max(opts->refine_tol, opts->tol) || stagnant) {
                p->cur_prec = CC_PREC_F64;
                switched_at = it + 1;
                best = INFINITY;
                grew = 0;
                if (use_corr) {
                  p->delta_mode = 2;
                  ccmi::plan_prepare(p);  // reference buffers, outside any capture
                }
              }
            }
            if (rn < best) {
              best = rn;
              grew = 0;
            } else if (opts->diverge_window > 0 && ++grew >= opts->diverge_window) {
              status = CC_EDIVERGED;
              done = true;
              break;
            }
          }
        }
      } catch (...) {
        (void)hipHostFree(hbuf);
        throw;
      }
      (void)hipHostFree(hbuf);
    } catch (...) {
      cc_plan_destroy(p);
      throw;
    }
    const auto t2c = std::chrono::steady_clock::now();
    if (rep) {
      rep->iters = iters;
      rep->converged = status == CC_OK;
      rep->rnorm = rn;
      rep->e_re = er;
      rep->e_im = ei;
      rep->seconds = std::chrono::duration<double>(t2c - t1c).count();
      rep->lowp_iters = switched_at < 0 ? (opts->prec == CC_PREC_F64 ? 0 : iters) : switched_at;
      rep->corr_iters = corr_iters;
      rep->setup_seconds = std::chrono::duration<double>(t1c - t0).count();
      rep->guess_used = guess_used;
      rep->guess_rnorm_mlp = g_mlp;
      rep->guess_rnorm_mp2 = g_mp2;
      rep->guess_seconds = guess_s;
    }
    cc_plan_destroy(p);
    if (status == CC_ENOTCONV) ctx->last_error = "max_iter reached before tolerance";
    if (status == CC_EDIVERGED) ctx->last_error = "residual norm diverged";
    return status;
  });
}

// ---- kernel-level entry points -------------------------------------------
int cc_gemm(cc_ctx *ctx, int prec, int scalar, int64_t M, int64_t N, int64_t K, double alpha,
            const void *A, int64_t sam, int64_t sak, const void *B, int64_t sbn, int64_t sbk,
            double beta, void *C, int64_t ldc) {
  if (!ctx) return fail(nullptr, CC_EINVAL, "ctx is NULL");
  return guarded(ctx, [&] {
    if (M < 0 || N < 0 || K < 0) throw CCError(CC_EINVAL, "negative GEMM size");
    if (M == 0 || N == 0) return CC_OK;
    check_ptr(C, "C");
    if (K > 0) {
      check_ptr(A, "A");
      check_ptr(B, "B");
    }
    if (!(sam == 1 || sak == 1) || !(sbn == 1 || sbk == 1))
      throw CCError(CC_EINVAL, "each operand needs one unit stride");
    if (ldc < N) throw CCError(CC_EINVAL, "ldc < N");
    if (prec != CC_PREC_F64 && prec != CC_PREC_F32 && prec != CC_PREC_BF16X3)
      throw CCError(CC_EINVAL, "unknown precision");
    set_device(ctx);
    ccmi::GemmDesc d{M, N, K, A, sam, sak, B, sbn, sbk, C, ldc, alpha, beta};
    const char *tv = std::getenv("CC_GEMM_TILE");  // tuning sweeps: force one tile configuration
    const int tile = tv ? std::atoi(tv) : -1;
    // Partial sums of split-K (as a plan would split this shape, the factor
    // then refined for the tile) or of the K-split tail of a launch whose last
    // round would be mostly empty, in a buffer the context keeps.  Without it
    // (or with CC_GEMM_TAIL=0) the GEMM runs as one launch.
    const char *cv = std::getenv("CC_GEMM_TAIL");
    const bool ws_ok = !(cv && cv[0] == '0');
    auto with_ws = [&](int64_t need) -> bool {
      if (need <= 0 || !ws_ok) return false;
      if (need > ctx->gemm_ws_elems) {
        CC_HIP_CHECK(hipStreamSynchronize(ctx->stream));
        if (ctx->gemm_ws) (void)hipFree(ctx->gemm_ws);
        ctx->gemm_ws = nullptr;
        ctx->gemm_ws_elems = 0;
        if (hipMalloc(&ctx->gemm_ws, size_t(need) * sizeof(double)) != hipSuccess) {
          (void)hipGetLastError();
          ctx->gemm_ws = nullptr;
          return false;
        }
        ctx->gemm_ws_elems = need;
      }
      d.ws = ctx->gemm_ws;
      d.ws_elems = ctx->gemm_ws_elems;
      return true;
    };
    auto plan_ws = [&](int64_t tail_need) {
      d.split = ws_ok ? ccmi::gemm_split_pick(M, N, K, -1) : 1;
      if (d.split > 1) {
        if (!with_ws(std::max<int64_t>(int64_t(d.split) * M * N, ccmi::gemm_tail_ws_bound(M, N, K)))) d.split = 1;
      } else {
        with_ws(tail_need);
      }
    };
    if (scalar == CC_C128 && prec != CC_PREC_F64) {
      // the real reduced-precision GEMM of M x 2N x 2K on realified copies
      // of the operands (A' M x 2K, B' 2N x 2K; 4 bytes per real element)
      if (K == 0) {
        ccmi::gemm_c128(d, ctx->stream, tile);
        CC_HIP_CHECK(hipStreamSynchronize(ctx->stream));
        return CC_OK;
      }
      void *sa = nullptr, *sb = nullptr;
      CC_HIP_CHECK(hipMalloc(&sa, size_t(2 * M * K) * 4));
      if (hipMalloc(&sb, size_t(4 * N * K) * 4) != hipSuccess) {
        (void)hipFree(sa);
        throw CCError(CC_ENOMEM, "GEMM operand copy allocation failed");
      }
      ccmi::realify_complex(prec, 0, static_cast<const double *>(A), nullptr, M, K, sam, sak, sa, ctx->stream);
      ccmi::realify_complex(prec, 1, static_cast<const double *>(B), nullptr, N, K, sbn, sbk, sb, ctx->stream);
      ccmi::GemmDesc g = ccmi::realified_desc(d, sa, sb);
      g.ws_elems = 0;
      g.split = ws_ok ? ccmi::gemm_split_pick(g.M, g.N, g.K, -1) : 1;
      if (g.split > 1) {
        if (with_ws(std::max<int64_t>(int64_t(g.split) * g.M * g.N, ccmi::gemm_tail_ws_bound(g.M, g.N, g.K)))) {
          g.ws = d.ws;
          g.ws_elems = d.ws_elems;
        } else {
          g.split = 1;
        }
      } else if (with_ws(ccmi::gemm_lowp_tail_ws(g, prec, tile))) {
        g.ws = d.ws;
        g.ws_elems = d.ws_elems;
      }
      ccmi::gemm_lowp(g, prec, ctx->stream, tile);
      const hipError_t e = hipStreamSynchronize(ctx->stream);
      (void)hipFree(sa);
      (void)hipFree(sb);
      CC_HIP_CHECK(e);
      return CC_OK;
    }
    if (scalar == CC_C128) ccmi::gemm_c128(d, ctx->stream, tile);
    else if (prec == CC_PREC_F64) {
      plan_ws(ccmi::gemm_f64_tail_ws(d, tile));
      ccmi::gemm_f64(d, ctx->stream, tile);
    }
    else {
      // operands converted once into temporary 4-byte copies (CC_GEMM_LPIN=0:
      // convert while staging instead); split bf16 on dense K-contiguous rows
      // with an LDS-direct configuration: copies in 16 x 32 blocks, which
      // those kernels load whole (CC_GEMM_BLOCKED=0: row-major copies)
      const char *lv = std::getenv("CC_GEMM_LPIN");
      const char *bv = std::getenv("CC_GEMM_BLOCKED");
      void *sa = nullptr, *sb = nullptr;
      const bool blocked = K > 0 && !(lv && lv[0] == '0') && !(bv && bv[0] == '0') && prec == CC_PREC_BF16X3 &&
                           K % 32 == 0 && sak == 1 && sbk == 1 && sam == K && sbn == K &&
                           ccmi::gemm_lowp_tile_blocked(prec, tile >= 0 ? tile : ccmi::gemm_lowp_pick(prec, M, N));
      if (blocked) {
        const int64_t pa = ccmi::blocked_plane(M, K), pb = ccmi::blocked_plane(N, K);
        CC_HIP_CHECK(hipMalloc(&sa, size_t(pa) * 4));
        if (hipMalloc(&sb, size_t(pb) * 4) != hipSuccess) {
          (void)hipFree(sa);
          throw CCError(CC_ENOMEM, "GEMM operand copy allocation failed");
        }
        ccmi::convert_blocked(static_cast<const double *>(A), nullptr, M, K, sa, ctx->stream);
        ccmi::convert_blocked(static_cast<const double *>(B), nullptr, N, K, sb, ctx->stream);
        d.A = sa;
        d.B = sb;
        d.a_plane = pa;
        d.b_plane = pb;
        d.lp_in = 2;
      } else if (K > 0 && !(lv && lv[0] == '0')) {
        const int64_t na = (M - 1) * sam + (K - 1) * sak + 1, nb = (N - 1) * sbn + (K - 1) * sbk + 1;
        CC_HIP_CHECK(hipMalloc(&sa, size_t(na) * 4));
        if (hipMalloc(&sb, size_t(nb) * 4) != hipSuccess) {
          (void)hipFree(sa);
          throw CCError(CC_ENOMEM, "GEMM operand copy allocation failed");
        }
        ccmi::convert_shadow(prec, static_cast<const double *>(A), na, sa, ctx->stream);
        ccmi::convert_shadow(prec, static_cast<const double *>(B), nb, sb, ctx->stream);
        d.A = sa;
        d.B = sb;
        d.a_plane = na;
        d.b_plane = nb;
        d.lp_in = 1;
      }
      plan_ws(ccmi::gemm_lowp_tail_ws(d, prec, tile));
      ccmi::gemm_lowp(d, prec, ctx->stream, tile);
      const hipError_t e = hipStreamSynchronize(ctx->stream);
      if (sa) (void)hipFree(sa);
      if (sb) (void)hipFree(sb);
      CC_HIP_CHECK(e);
      return CC_OK;
    }
    CC_HIP_CHECK(hipStreamSynchronize(ctx->stream));
    return CC_OK;
  });
}

int cc_gemm_tile_count(int prec) {
  if (prec == CC_PREC_F64) return ccmi::gemm_f64_num_tiles();
  if (prec == CC_PREC_F32 || prec == CC_PREC_BF16X3) return ccmi::gemm_lowp_num_tiles(prec);
  return -1;
}

int cc_gemm_tile_count_c128(void) { return ccmi::gemm_c128_num_tiles(); }

int cc_permute(cc_ctx *ctx, int scalar, int rank, const int64_t *in_dims, const int32_t *perm,
               double alpha, const void *in, double beta, void *out) {
  if (!ctx) return fail(nullptr, CC_EINVAL, "ctx is NULL");
  return guarded(ctx, [&] {
    if (rank < 1 || rank > ccmi::kMaxRank) throw CCError(CC_EINVAL, "rank must be 1..6");
    if (!in_dims || !perm) throw CCError(CC_EINVAL, "dims/perm NULL");
    check_ptr(in, "in");
    check_ptr(out, "out");
    int64_t istr[ccmi::kMaxRank];
    istr[rank - 1] = 1;
    for (int d = rank - 2; d >= 0; --d) istr[d] = istr[d + 1] * in_dims[d + 1];
    bool seen[ccmi::kMaxRank] = {false};
    ccmi::PermDesc pd{};
    pd.rank = rank;
    for (int d = 0; d < rank; ++d) {
      if (perm[d] < 0 || perm[d] >= rank || seen[perm[d]]) throw CCError(CC_EINVAL, "bad permutation");
      if (in_dims[d] < 0) throw CCError(CC_EINVAL, "negative dim");
      seen[perm[d]] = true;
      pd.out_dims[d] = in_dims[perm[d]];
      pd.in_strides[d] = istr[perm[d]];
    }
    pd.out_strides[rank - 1] = 1;
    for (int d = rank - 2; d >= 0; --d) pd.out_strides[d] = pd.out_strides[d + 1] * pd.out_dims[d + 1];
    pd.alpha = alpha;
    pd.beta = beta;
    pd.conj = 0;
    set_device(ctx);
    if (scalar == CC_C128) ccmi::permute_c128(pd, in, out, ctx->stream);
    else ccmi::permute_f64(pd, in, out, ctx->stream);
    CC_HIP_CHECK(hipStreamSynchronize(ctx->stream));
    return CC_OK;
  });
}

// Text dump of a plan's steps (debugging aid; the string stays valid until
// the next call on the same thread).
const char *cc_plan_describe(const cc_plan *p) {
  static thread_local std::string s;
  s = p ? ccmi::plan_describe(p) : std::string();
  return s.c_str();
}

const char *cc_plan_describe_ops_dry(int o, int v, int method, int scalar, const char *ops) {
  static thread_local std::string s;
  try {
    if (o < 1 || v < 1) throw CCError(CC_EINVAL, "o and v must be >= 1");
    validate_method(method, CC_PREC_F64, scalar);
    cc_plan p;
    if (ops) p.custom = std::make_shared<ccmi::OpList>(ccmi::parse_op_list(ops));
    p.o = o;
    p.v = v;
    p.method = method;
    p.cplx = scalar == CC_C128;
    p.esize = p.cplx ? 16 : 8;
    cc_system sys{};
    sys.o = o;
    sys.v = v;
    sys.scalar = scalar;
    ccmi::plan_layout(&p, &sys);
    s = ccmi::plan_describe(&p);
  } catch (const std::exception &e) {
    s = std::string("error: ") + e.what();
  }
  return s.c_str();
}

const char *cc_plan_describe_dry(int o, int v, int method, int scalar) {
  static thread_local std::string s;
  try {
    if (o < 1 || v < 1) throw CCError(CC_EINVAL, "o and v must be >= 1");
    validate_method(method, CC_PREC_F64, scalar);
    cc_plan p;
    p.o = o;
    p.v = v;
    p.method = method;
    p.cplx = scalar == CC_C128;
    p.esize = p.cplx ? 16 : 8;
    cc_system sys{};
    sys.o = o;
    sys.v = v;
    sys.scalar = scalar;
    ccmi::plan_layout(&p, &sys);
    s = ccmi::plan_describe(&p);
  } catch (const std::exception &e) {
    s = std::string("error: ") + e.what();
  }
  return s.c_str();
}

int cc_plan_set_precision(cc_plan *p, int prec) {
  if (!p) return fail(nullptr, CC_EINVAL, "plan is NULL");
  return guarded(p->ctx, [&] {
    validate_method(p->method, prec, p->cplx ? CC_C128 : CC_R64);
    p->cur_prec = prec;
    return CC_OK;
  });
}

int cc_plan_set_correction(cc_plan *p, int mode, int prec) {
  if (!p) return fail(nullptr, CC_EINVAL, "plan is NULL");
  return guarded(p->ctx, [&] {
    if (mode != 0 && mode != 1) throw CCError(CC_EINVAL, "mode must be 0 or 1");
    if (prec != CC_PREC_F32 && prec != CC_PREC_BF16X3)
      throw CCError(CC_EINVAL, "correction precision must be F32 or BF16X3");
    p->delta_prec = prec;
    p->delta_mode = mode ? 2 : 0;
    return CC_OK;
  });
}

int cc_plan_autotune(cc_plan *p, const cc_amps *t, int reps) {
  if (!p) return fail(nullptr, CC_EINVAL, "plan is NULL");
  return guarded(p->ctx, [&] {
    validate_amps(t, p->method, "t");
    if (reps < 1) throw CCError(CC_EINVAL, "reps must be >= 1");
    set_device(p->ctx);
    p->t1 = t->t1;
    p->t2 = t->t2;
    ccmi::plan_autotune(p, reps);
    return CC_OK;
  });
}

int cc_plan_profile(cc_plan *p, int enable) {
  if (!p) return fail(nullptr, CC_EINVAL, "plan is NULL");
  return guarded(p->ctx, [&] {
    p->profiling = enable != 0;
    p->step_ms.assign(p->iter.size(), 0.0);
    p->step_calls.assign(p->iter.size(), 0);
    return CC_OK;
  });
}

const char *cc_plan_profile_table(const cc_plan *p) {
  static thread_local std::string s;
  s = p ? ccmi::plan_profile_table(p) : std::string();
  return s.c_str();
}

double cc_plan_flops(const cc_plan *p, int which) {
  if (!p) return 0.0;
  return which == 1 ? p->ladder_flops : p->flops_per_iter;
}

}  // extern "C"
