// Batched evaluation of many independent, uneven CC systems.
//
// Every system gets its own plan (same contraction list, its own shapes and
// workspace).  The plans' iteration steps are then fused index by index: step
// k of all systems becomes ONE grouped launch whose workgroup range is the
// concatenation of the systems' ranges (system b owns [off[b], off[b+1])).
// A grouped GEMM uses one tile configuration for the whole contraction class
// (chosen by timing the grouped launch), each system keeps its own split-K
// factor.  One iteration of the whole batch is therefore ~60 launches,
// independent of the number of systems, and is replayed as one HIP graph.
// Steps whose launch form differs between systems (possible only for
// degenerate dimensions) fall back to per-system launches inside the graph.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <map>
#include <string>

#include "plan.hpp"


namespace ccmi {
namespace {

struct GStep {
  Step::Kind kind;
  std::string tag;
  bool grouped = true;
  bool tiled = false;     // permutations
  bool akc = true, bkc = true;
  int tile = 0;           // grouped GEMM tile configuration
  int64_t blocks = 0;     // total workgroups of the grouped launch
  size_t entry_off = 0;   // byte offset of the entries in the device arena
  size_t off_off = 0;     // byte offset of the n+1 block offsets
  // split-K reduction that follows a grouped GEMM
  int64_t sk_blocks = 0;
  size_t sk_entry_off = 0, sk_off_off = 0;
  double flops = 0.0;
  // reduced precision: the GEMM reads operand copies (lp), made by the
  // grouped conversions listed here for the slots written since their last one
  bool lp = false;
  struct Conv {
    size_t entry_off, off_off;
    int64_t blocks;
  };
  std::vector<Conv> conv;
};

}  // namespace
}  // namespace ccmi

struct cc_batch {
  cc_ctx *ctx = nullptr;
  int n = 0, method = 0, prec = 0;
  bool cplx = false;
  std::vector<cc_plan *> plans;
  std::vector<ccmi::GStep> gsteps;
  std::vector<unsigned char> host_arena;
  void *dev_arena = nullptr;
  size_t arena_bytes = 0;
  double *scalars = nullptr;  // 4 per system
  double shift = 0.0;
  int dressed = 0;
  bool built_for_update = false;
  hipGraphExec_t graph = nullptr;
  bool profiling = false;
  std::vector<hipEvent_t> events;
  std::vector<double> step_ms;
  int64_t prof_calls = 0;
  double flops = 0.0;
  std::vector<std::vector<int>> own_split;  // per step and system: the plan's own split-K factor
};

namespace ccmi {
namespace {

template <class E>
size_t push_entries(cc_batch *B, const std::vector<E> &v) {
  size_t off = (B->host_arena.size() + 255) & ~size_t(255);
  B->host_arena.resize(off + sizeof(E) * v.size());
  std::memcpy(B->host_arena.data() + off, v.data(), sizeof(E) * v.size());
  return off;
}

size_t push_offsets(cc_batch *B, const std::vector<int64_t> &units, int64_t *total) {
  std::vector<int64_t> off(units.size() + 1, 0);
  for (size_t i = 0; i < units.size(); ++i) off[i + 1] = off[i] + units[i];
  *total = off.back();
  return push_entries(B, off);
}

int64_t batch_slot_elems(const cc_plan *p, int s) {
  const Slot &sl = p->slots[s];
  if (!sl.external) return sl.elems;
  return sl.name == "t1" ? int64_t(p->o) * p->v : int64_t(p->o) * p->o * p->v * p->v;
}

// (Re)build the device tables of every grouped step from the plans' current
// per-call state (amplitude pointers, shift, denominator mode).
void build_tables(cc_batch *B) {
  B->host_arena.clear();
  B->gsteps.clear();
  const size_t nsteps = B->plans[0]->iter.size();
  for (cc_plan *p : B->plans)
    CC_REQUIRE(p->iter.size() == nsteps, CC_EINTERNAL, "batch: plans differ in step count");
  // Reduced precision (real systems): the grouped GEMMs on K-contiguous
  // operands read 4-byte copies made by grouped conversions, each slot
  // converted once after every write (constant slots once, here).
  const bool lowp = B->prec != PREC_F64 && !B->cplx;
  if (lowp)
    for (cc_plan *p : B->plans) {
      p->cur_prec = B->prec;
      plan_prepare(p);
    }
  // per plan and slot: the copy matches the slot at this point of the step list
  std::vector<std::vector<char>> fresh;
  for (cc_plan *p : B->plans) fresh.emplace_back(p->slots.size(), 0);
  auto written = [&](size_t k) {
    for (size_t b = 0; b < B->plans.size(); ++b) {
      const Step &st = B->plans[b]->iter[k];
      switch (st.kind) {
        case Step::PERMUTE:
        case Step::GEMM:
        case Step::OUTER:
        case Step::FILL:
        case Step::PAIR:
          if (st.c >= 0) fresh[b][st.c] = 0;
          break;
        default:  // tau, the assembly, the updates: conservatively every slot
          std::fill(fresh[b].begin(), fresh[b].end(), 0);
      }
    }
  };
  for (size_t k = 0; k < nsteps; ++k) {
    GStep g;
    const Step &s0 = B->plans[0]->iter[k];
    g.kind = s0.kind;
    g.tag = s0.tag;
    for (cc_plan *p : B->plans) {
      CC_REQUIRE(p->iter[k].kind == s0.kind, CC_EINTERNAL, "batch: plans differ in step kinds");
      g.flops += p->iter[k].flops;
    }
    std::vector<int64_t> units;
    switch (g.kind) {
      case Step::PERMUTE: {
        std::vector<PermEntry> es;
        for (cc_plan *p : B->plans) {
          const Step &st = p->iter[k];
          es.push_back(make_perm_entry(st.perm, ptr_of(p, st.a), ptr_of(p, st.c)));
          units.push_back(es.back().units);
        }
        g.tiled = es[0].tiled;
        for (auto &e : es)
          if (e.tiled != g.tiled && e.units > 0) g.grouped = false;
        g.entry_off = push_entries(B, es);
        g.off_off = push_offsets(B, units, &g.blocks);
        break;
      }
      case Step::GEMM: {
        std::vector<GemmGroupEntry> es;
        std::vector<SplitkEntry> sk;
        std::vector<int64_t> skunits;
        const Step &st0 = B->plans[0]->iter[k];
        g.akc = st0.gemm.sak == 1;
        g.bkc = st0.gemm.sbk == 1;
        // tile: the plans' choice for the largest system (the tuner may refine it)
        int64_t best = -1;
        for (cc_plan *p : B->plans) {
          const Step &st = p->iter[k];
          if ((st.gemm.sak == 1) != g.akc || (st.gemm.sbk == 1) != g.bkc) g.grouped = false;
          const int64_t work = st.gemm.M * st.gemm.N * st.gemm.K;
          if (work > best) {
            best = work;
            if (B->prec == PREC_F64)
              g.tile = st.tile >= 0 ? st.tile : gemm_f64_pick(st.gemm.M, st.gemm.N, st.gemm.K, g.akc, g.bkc);
            else
              g.tile = st.tile_lp[B->prec] >= 0 && gemm_lowp_tile_grouped(B->prec, st.tile_lp[B->prec])
                           ? st.tile_lp[B->prec]
                           : gemm_lowp_pick(B->prec, st.gemm.M, st.gemm.N);
          }
        }
        int bm, bn;
        if (B->prec == PREC_F64) gemm_f64_tile_shape(g.tile, &bm, &bn);
        else gemm_lowp_tile_shape(B->prec, g.tile, &bm, &bn);
        for (cc_plan *p : B->plans) {
          const Step &st = p->iter[k];
          GemmGroupEntry e{};
          e.d = st.gemm;
          e.d.A = ptr_of(p, st.a);
          e.d.B = ptr_of(p, st.b);
          e.d.C = ptr_of(p, st.c);
          e.d.ws = st.b2 >= 0 ? ptr_of(p, st.b2) : nullptr;
          e.tilesM = (e.d.M + bm - 1) / bm;
          e.tilesN = (e.d.N + bn - 1) / bn;
          const bool empty = e.d.M <= 0 || e.d.N <= 0 || e.d.K <= 0;
          if (empty) g.grouped = false;
          units.push_back(empty ? 0 : e.tilesM * e.tilesN * e.d.split);
          es.push_back(e);
          if (e.d.split > 1) {
            sk.push_back(make_splitk_entry(e.d.ws, e.d.split, e.d.M, e.d.N, e.d.C, e.d.ldc, e.d.alpha, e.d.beta));
          } else {
            sk.push_back(SplitkEntry{});
          }
          skunits.push_back(e.d.split > 1 ? sk.back().units : 0);
        }
        if (lowp && g.grouped && g.akc && g.bkc) {
          g.lp = true;
          for (cc_plan *p : B->plans) {
            const Step &st = p->iter[k];
            if (p->shadow.size() != p->slots.size() || !p->shadow[st.a] || !p->shadow[st.b]) g.lp = false;
          }
        }
        if (g.lp) {
          for (size_t b = 0; b < es.size(); ++b) {
            cc_plan *p = B->plans[b];
            const Step &st = p->iter[k];
            es[b].d.A = p->shadow[st.a];
            es[b].d.B = p->shadow[st.b];
            es[b].d.a_plane = batch_slot_elems(p, st.a);
            es[b].d.b_plane = batch_slot_elems(p, st.b);
            es[b].d.lp_in = 1;
          }
          // one grouped conversion per operand side, over the systems whose
          // slot was written since its last conversion (the others: no work)
          for (int side = 0; side < 2; ++side) {
            std::vector<ConvEntry> ce;
            std::vector<int64_t> cu;
            bool any = false;
            for (size_t b = 0; b < B->plans.size(); ++b) {
              cc_plan *p = B->plans[b];
              const Step &st = p->iter[k];
              const int sl = side ? st.b : st.a;
              const bool need = !fresh[b][sl] && !p->slots[sl].constant;
              ce.push_back(need ? make_conv_entry(static_cast<const double *>(ptr_of(p, sl)),
                                                  batch_slot_elems(p, sl), p->shadow[sl])
                                : make_conv_entry(nullptr, 0, nullptr));
              cu.push_back(ce.back().units);
              fresh[b][sl] = 1;
              any = any || need;
            }
            if (!any) continue;
            GStep::Conv c{};
            c.entry_off = push_entries(B, ce);
            c.off_off = push_offsets(B, cu, &c.blocks);
            g.conv.push_back(c);
          }
        }
        // systems in the launch in order of K per workgroup, longest first,
        // so that the longest workgroups start in the first round instead of
        // finishing last (the entries carry their own pointers: any order)
        {
          std::vector<size_t> ord(es.size());
          for (size_t b = 0; b < ord.size(); ++b) ord[b] = b;
          auto klen = [&](size_t b) { return (es[b].d.K + es[b].d.split - 1) / es[b].d.split; };
          std::stable_sort(ord.begin(), ord.end(), [&](size_t x, size_t y) { return klen(x) > klen(y); });
          std::vector<GemmGroupEntry> es2;
          std::vector<int64_t> u2;
          for (size_t b : ord) {
            es2.push_back(es[b]);
            u2.push_back(units[b]);
          }
          es.swap(es2);
          units.swap(u2);
        }
        g.entry_off = push_entries(B, es);
        g.off_off = push_offsets(B, units, &g.blocks);
        g.sk_entry_off = push_entries(B, sk);
        g.sk_off_off = push_offsets(B, skunits, &g.sk_blocks);
        break;
      }
      case Step::PAIR: {
        std::vector<PairEntry> es;
        for (cc_plan *p : B->plans) {
          const Step &st = p->iter[k];
          es.push_back(make_pair_entry(ptr_of(p, st.a), ptr_of(p, st.c), p->pair_tab[st.pair_rows],
                                       p->pair_tab[st.pair_cols], st.pair_np, st.pair_nq, st.pair_ldq, st.pair_n[0],
                                       st.pair_n[1], st.pair_n[2], st.pair_mode));
          units.push_back(es.back().units);
        }
        g.entry_off = push_entries(B, es);
        g.off_off = push_offsets(B, units, &g.blocks);
        break;
      }
      case Step::OUTER: {
        std::vector<OuterEntry> es;
        for (cc_plan *p : B->plans) {
          const Step &st = p->iter[k];
          es.push_back(make_outer_entry(st.outer, ptr_of(p, st.a), ptr_of(p, st.b), ptr_of(p, st.c)));
          units.push_back(es.back().units);
        }
        g.entry_off = push_entries(B, es);
        g.off_off = push_offsets(B, units, &g.blocks);
        break;
      }
      case Step::FILL: {
        std::vector<FillEntry> es;
        for (cc_plan *p : B->plans) {
          const Step &st = p->iter[k];
          es.push_back(make_fill_entry(ptr_of(p, st.c), st.nelem));
          units.push_back(es.back().units);
        }
        g.entry_off = push_entries(B, es);
        g.off_off = push_offsets(B, units, &g.blocks);
        break;
      }
      case Step::TAU_E: {
        std::vector<TauEntry> es;
        for (cc_plan *p : B->plans) {
          es.push_back(tau_entry(p));
          units.push_back(es.back().units);
        }
        g.entry_off = push_entries(B, es);
        g.off_off = push_offsets(B, units, &g.blocks);
        break;
      }
      case Step::ASSEMBLE: {
        std::vector<AsmEntry> es;
        for (cc_plan *p : B->plans) {
          es.push_back(asm_entry(p));
          units.push_back(es.back().units);
        }
        g.entry_off = push_entries(B, es);
        g.off_off = push_offsets(B, units, &g.blocks);
        break;
      }
      case Step::R1UPD: {
        std::vector<R1Entry> es;
        for (cc_plan *p : B->plans) es.push_back(r1_entry(p));
        g.entry_off = push_entries(B, es);
        g.blocks = B->n;
        break;
      }
      case Step::FINALIZE: {
        std::vector<FinEntry> es;
        for (int b = 0; b < B->n; ++b) {
          FinEntry e = fin_entry(B->plans[b]);
          e.scalars = B->scalars + 4 * b;
          es.push_back(e);
        }
        g.entry_off = push_entries(B, es);
        g.blocks = B->n;
        break;
      }
    }
    written(k);
    B->gsteps.push_back(g);
  }
  const size_t bytes = std::max<size_t>(B->host_arena.size(), 256);
  if (bytes > B->arena_bytes) {
    if (B->dev_arena) (void)hipFree(B->dev_arena);
    B->dev_arena = nullptr;
    CC_HIP_CHECK(hipMalloc(&B->dev_arena, bytes));
    B->arena_bytes = bytes;
  }
  CC_HIP_CHECK(hipMemcpyAsync(B->dev_arena, B->host_arena.data(), B->host_arena.size(), hipMemcpyHostToDevice,
                              B->ctx->stream));
  CC_HIP_CHECK(hipStreamSynchronize(B->ctx->stream));
  if (B->graph) (void)hipGraphExecDestroy(B->graph);
  B->graph = nullptr;
}

template <class E>
const E *dev_at(cc_batch *B, size_t off) {
  return reinterpret_cast<const E *>(static_cast<unsigned char *>(B->dev_arena) + off);
}

void run_gstep(cc_batch *B, size_t k, hipStream_t s) {
  const GStep &g = B->gsteps[k];
  const bool cplx = B->cplx;
  const int n = B->n;
  if (!g.grouped || (g.kind == Step::GEMM && cplx)) {
    // per-system launches (complex GEMMs, degenerate shapes)
    for (cc_plan *p : B->plans) {
      Step &st = p->iter[k];
      if (st.kind == Step::GEMM) {
        GemmDesc d = st.gemm;
        d.A = ptr_of(p, st.a);
        d.B = ptr_of(p, st.b);
        d.C = ptr_of(p, st.c);
        d.ws = st.b2 >= 0 ? ptr_of(p, st.b2) : nullptr;
        if (cplx) gemm_c128(d, s, st.tile_z);
        else if (B->prec == PREC_F64) gemm_f64(d, s, st.tile);
        else gemm_lowp(d, B->prec, s, st.tile_lp[B->prec]);
      } else if (st.kind == Step::PERMUTE) {
        launch_perm(make_perm_entry(st.perm, ptr_of(p, st.a), ptr_of(p, st.c)), cplx, s);
      } else {
        throw CCError(CC_EINTERNAL, "batch: unexpected ungrouped step");
      }
    }
    return;
  }
  const int64_t *off = dev_at<int64_t>(B, g.off_off);
  switch (g.kind) {
    case Step::PERMUTE:
      launch_perm_grouped(dev_at<PermEntry>(B, g.entry_off), off, n, g.blocks, g.tiled, cplx, s);
      break;
    case Step::GEMM:
      for (const GStep::Conv &c : g.conv)
        convert_shadow_grouped(B->prec, dev_at<ConvEntry>(B, c.entry_off), dev_at<int64_t>(B, c.off_off), n,
                               c.blocks, s);
      if (B->prec == PREC_F64)
        gemm_f64_grouped_launch(dev_at<GemmGroupEntry>(B, g.entry_off), off, n, g.blocks, g.akc, g.bkc, g.tile, s);
      else if (g.lp)
        gemm_lowp_grouped_launch_lp(dev_at<GemmGroupEntry>(B, g.entry_off), off, n, g.blocks, B->prec, g.tile, s);
      else
        gemm_lowp_grouped_launch(dev_at<GemmGroupEntry>(B, g.entry_off), off, n, g.blocks, g.akc, g.bkc, B->prec,
                                 g.tile, s);
      if (g.sk_blocks > 0)
        launch_splitk_grouped(dev_at<SplitkEntry>(B, g.sk_entry_off), dev_at<int64_t>(B, g.sk_off_off), n,
                              g.sk_blocks, cplx, s);
      break;
    case Step::OUTER:
      launch_outer_grouped(dev_at<OuterEntry>(B, g.entry_off), off, n, g.blocks, cplx, s);
      break;
    case Step::PAIR:
      launch_pair_grouped(dev_at<PairEntry>(B, g.entry_off), off, n, g.blocks, cplx, s);
      break;
    case Step::FILL:
      launch_fill_grouped(dev_at<FillEntry>(B, g.entry_off), off, n, g.blocks, cplx, s);
      break;
    case Step::TAU_E:
      launch_tau_grouped(dev_at<TauEntry>(B, g.entry_off), off, n, g.blocks, cplx, s);
      break;
    case Step::ASSEMBLE:
      launch_asm_grouped(dev_at<AsmEntry>(B, g.entry_off), off, n, g.blocks, cplx, s);
      break;
    case Step::R1UPD:
      launch_r1_grouped(dev_at<R1Entry>(B, g.entry_off), n, cplx, s);
      break;
    case Step::FINALIZE:
      launch_fin_grouped(dev_at<FinEntry>(B, g.entry_off), n, s);
      break;
  }
}

}  // namespace

// Split-K factors for the batch as a whole.  Each plan chose its factors to
// fill the GPU with its own GEMMs alone (up to 16 K-slices for a small
// system); in a batch the systems' tiles fill it together, so a step's
// factor follows the tiles of all systems: slices only while they number
// under 2,048 of 64 x 64, and never K-slices shorter than 256.  The plans'
// workspaces were sized for their own, larger factors.
void batch_group_splits(cc_batch *B) {
  B->own_split.assign(B->plans[0]->iter.size(), {});
  for (size_t k = 0; k < B->plans[0]->iter.size(); ++k) {
    if (B->plans[0]->iter[k].kind != Step::GEMM) continue;
    for (cc_plan *p : B->plans) B->own_split[k].push_back(p->iter[k].gemm.split);
    int64_t tiles = 0;
    for (cc_plan *p : B->plans) {
      const GemmDesc &d = p->iter[k].gemm;
      tiles += ((d.M + 63) / 64) * ((d.N + 63) / 64);
    }
    const int64_t split = tiles >= 2048 ? 1 : (2048 + tiles - 1) / std::max<int64_t>(tiles, 1);
    for (cc_plan *p : B->plans) {
      GemmDesc &d = p->iter[k].gemm;
      d.split = int(std::max<int64_t>(1, std::min<int64_t>({split, int64_t(d.split), std::max<int64_t>(1, d.K / 256)})));
    }
  }
}

void batch_run(cc_batch *B) {
  hipStream_t s = B->ctx->stream;
  if (!B->profiling) {
    for (size_t k = 0; k < B->gsteps.size(); ++k) run_gstep(B, k, s);
    return;
  }
  const size_t n = B->gsteps.size();
  if (B->events.size() != n + 1) {
    for (hipEvent_t e : B->events) (void)hipEventDestroy(e);
    B->events.assign(n + 1, nullptr);
    for (auto &e : B->events) CC_HIP_CHECK(hipEventCreate(&e));
    B->step_ms.assign(n, 0.0);
  }
  CC_HIP_CHECK(hipEventRecord(B->events[0], s));
  for (size_t k = 0; k < n; ++k) {
    run_gstep(B, k, s);
    CC_HIP_CHECK(hipEventRecord(B->events[k + 1], s));
  }
  CC_HIP_CHECK(hipEventSynchronize(B->events[n]));
  for (size_t k = 0; k < n; ++k) {
    float ms = 0.f;
    CC_HIP_CHECK(hipEventElapsedTime(&ms, B->events[k], B->events[k + 1]));
    B->step_ms[k] += ms;
  }
  ++B->prof_calls;
}

// Time every tile configuration of each grouped GEMM (a contraction class
// across the batch) and keep the fastest; then the plans' own split-K
// factors against the batch's.
void batch_autotune(cc_batch *B, int reps) {
  if (B->cplx) return;
  const int prec = B->prec;
  const int ntiles = prec == PREC_F64 ? gemm_f64_num_tiles() : gemm_lowp_num_tiles(prec);
  auto tile_of = [prec](Step &st) -> int & { return prec == PREC_F64 ? st.tile : st.tile_lp[prec]; };
  hipStream_t s = B->ctx->stream;
  hipEvent_t e0, e1;
  CC_HIP_CHECK(hipEventCreate(&e0));
  CC_HIP_CHECK(hipEventCreate(&e1));
  try {
    for (size_t k = 0; k < B->gsteps.size(); ++k) {
      if (B->gsteps[k].kind != Step::GEMM || !B->gsteps[k].grouped) continue;
      int best = B->gsteps[k].tile;
      float best_ms = 1e30f;
      for (int t = 0; t < ntiles; ++t) {
        if (prec != PREC_F64 && !gemm_lowp_tile_grouped(prec, t)) continue;
        for (cc_plan *p : B->plans) tile_of(p->iter[k]) = t;
        build_tables(B);
        run_gstep(B, k, s);
        CC_HIP_CHECK(hipEventRecord(e0, s));
        for (int r = 0; r < reps; ++r) run_gstep(B, k, s);
        CC_HIP_CHECK(hipEventRecord(e1, s));
        CC_HIP_CHECK(hipEventSynchronize(e1));
        float ms = 0.f;
        CC_HIP_CHECK(hipEventElapsedTime(&ms, e0, e1));
        if (ms < best_ms) {
          best_ms = ms;
          best = t;
        }
      }
      for (cc_plan *p : B->plans) tile_of(p->iter[k]) = best;
      // then the plans' own split-K factors instead of the batch's, where
      // faster (GEMMs with a tiny M x N and a long K want many K-slices)
      if (B->own_split.size() == B->gsteps.size() && B->own_split[k].size() == B->plans.size()) {
        std::vector<int> cur;
        bool differs = false;
        for (size_t b = 0; b < B->plans.size(); ++b) {
          cur.push_back(B->plans[b]->iter[k].gemm.split);
          differs = differs || cur[b] != B->own_split[k][b];
        }
        if (differs) {
          for (size_t b = 0; b < B->plans.size(); ++b) B->plans[b]->iter[k].gemm.split = B->own_split[k][b];
          build_tables(B);
          run_gstep(B, k, s);
          CC_HIP_CHECK(hipEventRecord(e0, s));
          for (int r = 0; r < reps; ++r) run_gstep(B, k, s);
          CC_HIP_CHECK(hipEventRecord(e1, s));
          CC_HIP_CHECK(hipEventSynchronize(e1));
          float ms = 0.f;
          CC_HIP_CHECK(hipEventElapsedTime(&ms, e0, e1));
          if (ms >= best_ms)
            for (size_t b = 0; b < B->plans.size(); ++b) B->plans[b]->iter[k].gemm.split = cur[b];
        }
      }
    }
  } catch (...) {
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    throw;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  build_tables(B);
}

}  // namespace ccmi

// ============================================================== C ABI =====
namespace {
int bfail(cc_ctx *ctx, int status, const std::string &msg) {
  if (ctx) ctx->last_error = msg;
  return status;
}

template <class F>
int bguard(cc_ctx *ctx, F &&f) {
  try {
    return f();
  } catch (const ccmi::CCError &e) {
    return bfail(ctx, e.status, e.what());
  } catch (const std::exception &e) {
    return bfail(ctx, CC_EINTERNAL, e.what());
  }
}

void batch_free(cc_batch *B) {
  if (B->graph) (void)hipGraphExecDestroy(B->graph);
  for (hipEvent_t e : B->events) (void)hipEventDestroy(e);
  for (cc_plan *p : B->plans) {
    ccmi::plan_free(p);
    delete p;
  }
  if (B->dev_arena) (void)hipFree(B->dev_arena);
  if (B->scalars) (void)hipFree(B->scalars);
}

void batch_prepare(cc_batch *B, double shift, int dressed) {
  if (!B->built_for_update || B->shift != shift || B->dressed != dressed) {
    for (cc_plan *p : B->plans) {
      p->update = true;
      p->shift = shift;
      p->dressed = dressed;
      p->r1_out = p->r2_out = nullptr;
      p->cur_prec = B->prec;
    }
    B->shift = shift;
    B->dressed = dressed;
    B->built_for_update = true;
    ccmi::build_tables(B);
  }
}

void batch_launch(cc_batch *B, bool use_graph) {
  if (!use_graph || B->profiling) {
    ccmi::batch_run(B);
    return;
  }
  if (!B->graph) {
    hipGraph_t g;
    CC_HIP_CHECK(hipStreamBeginCapture(B->ctx->stream, hipStreamCaptureModeThreadLocal));
    try {
      ccmi::batch_run(B);
    } catch (...) {
      hipGraph_t dummy;
      (void)hipStreamEndCapture(B->ctx->stream, &dummy);
      throw;
    }
    CC_HIP_CHECK(hipStreamEndCapture(B->ctx->stream, &g));
    CC_HIP_CHECK(hipGraphInstantiate(&B->graph, g, nullptr, nullptr, 0));
    (void)hipGraphDestroy(g);
  }
  CC_HIP_CHECK(hipGraphLaunch(B->graph, B->ctx->stream));
}
}  // namespace

extern "C" {

int cc_batch_create(cc_ctx *ctx, int n, const cc_system *systems, int method, int prec, cc_amps *amps,
                    cc_batch **out) {
  if (!ctx) return bfail(nullptr, CC_EINVAL, "ctx is NULL");
  if (!out) return bfail(ctx, CC_EINVAL, "batch pointer is NULL");
  *out = nullptr;
  return bguard(ctx, [&] {
    if (n < 1 || !systems || !amps) throw ccmi::CCError(CC_EINVAL, "n >= 1 systems and amplitudes required");
    cc_batch *B = new cc_batch();
    B->ctx = ctx;
    B->n = n;
    B->method = method;
    B->prec = prec;
    try {
      for (int b = 0; b < n; ++b) {
        // every contraction in the batch's precision: one grouped launch per step
        // real systems: the ladder, the hole-hole ladder and Z over packed
        // pairs (i<j, a<b, e<f) unless CC_BATCH_DENSE is set
        cc_plan *p = ccmi::make_plan_checked(ctx, &systems[b], method, prec, true, true,
                                             !std::getenv("CC_BATCH_DENSE") && systems[b].scalar != CC_C128);
        ccmi::check_amps(&amps[b], method);
        p->t1 = amps[b].t1;
        p->t2 = amps[b].t2;
        B->plans.push_back(p);
        B->flops += p->flops_per_iter;
      }
      B->cplx = B->plans[0]->cplx;
      if (B->cplx && prec != CC_PREC_F64)
        throw ccmi::CCError(CC_EUNSUPPORTED, "batches of complex systems run FP64 contractions only");
      for (cc_plan *p : B->plans)
        if (p->cplx != B->cplx) throw ccmi::CCError(CC_EINVAL, "batch mixes real and complex systems");
      if (!std::getenv("CC_BATCH_OWN_SPLITS")) ccmi::batch_group_splits(B);
      CC_HIP_CHECK(hipMalloc(reinterpret_cast<void **>(&B->scalars), sizeof(double) * 4 * n));
      batch_prepare(B, 0.0, 0);
    } catch (...) {
      batch_free(B);
      delete B;
      throw;
    }
    *out = B;
    return CC_OK;
  });
}

int cc_batch_destroy(cc_batch *B) {
  if (!B) return CC_OK;
  (void)hipSetDevice(B->ctx->device);
  (void)hipStreamSynchronize(B->ctx->stream);
  batch_free(B);
  delete B;
  return CC_OK;
}

int cc_batch_step(cc_batch *B, double level_shift, int dressed) {
  if (!B) return bfail(nullptr, CC_EINVAL, "batch is NULL");
  return bguard(B->ctx, [&] {
    if (!(level_shift >= 0.0)) throw ccmi::CCError(CC_EINVAL, "level_shift must be >= 0");
    CC_HIP_CHECK(hipSetDevice(B->ctx->device));
    batch_prepare(B, level_shift, dressed ? 1 : 0);
    batch_launch(B, true);
    return CC_OK;
  });
}

int cc_batch_scalars(cc_batch *B, double *rnorm, double *e_re, double *e_im) {
  if (!B) return bfail(nullptr, CC_EINVAL, "batch is NULL");
  return bguard(B->ctx, [&] {
    std::vector<double> h(4 * B->n);
    CC_HIP_CHECK(hipMemcpyAsync(h.data(), B->scalars, sizeof(double) * 4 * B->n, hipMemcpyDeviceToHost,
                                B->ctx->stream));
    CC_HIP_CHECK(hipStreamSynchronize(B->ctx->stream));
    for (int b = 0; b < B->n; ++b) {
      if (rnorm) rnorm[b] = h[4 * b];
      if (e_re) e_re[b] = h[4 * b + 1];
      if (e_im) e_im[b] = h[4 * b + 2];
    }
    return CC_OK;
  });
}

int cc_batch_autotune(cc_batch *B, int reps) {
  if (!B) return bfail(nullptr, CC_EINVAL, "batch is NULL");
  return bguard(B->ctx, [&] {
    if (reps < 1) throw ccmi::CCError(CC_EINVAL, "reps must be >= 1");
    batch_prepare(B, B->shift, B->dressed);
    ccmi::batch_autotune(B, reps);
    return CC_OK;
  });
}

int cc_batch_iterate(cc_batch *B, const cc_iter_opts *opts, cc_iter_report *reports, int32_t *n_converged) {
  if (!B) return bfail(nullptr, CC_EINVAL, "batch is NULL");
  return bguard(B->ctx, [&] {
    if (!opts || opts->max_iter < 1 || !(opts->tol > 0.0)) throw ccmi::CCError(CC_EINVAL, "bad options");
    if (opts->prec != B->prec) throw ccmi::CCError(CC_EINVAL, "batch precision is fixed at creation");
    batch_prepare(B, opts->level_shift, opts->dressed ? 1 : 0);
    const int n = B->n;
    std::vector<double> h(4 * n);
    std::vector<int> done(n, 0);
    int ndone = 0, it = 0;
    const auto t0 = std::chrono::steady_clock::now();
    bool bad = false;
    for (; it < opts->max_iter && ndone < n; ++it) {
      batch_launch(B, opts->use_graph != 0);
      CC_HIP_CHECK(hipMemcpyAsync(h.data(), B->scalars, sizeof(double) * 4 * n, hipMemcpyDeviceToHost,
                                  B->ctx->stream));
      CC_HIP_CHECK(hipStreamSynchronize(B->ctx->stream));
      const double el = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
      for (int b = 0; b < n; ++b) {
        if (done[b]) continue;
        const double rn = h[4 * b];
        if (reports) {
          cc_iter_report &r = reports[b];
          if (r.hist_rnorm && it < r.hist_cap) r.hist_rnorm[it] = rn;
          if (r.hist_e && it < r.hist_cap) r.hist_e[it] = h[4 * b + 1];
          r.iters = it + 1;
          r.rnorm = rn;
          r.e_re = h[4 * b + 1];
          r.e_im = h[4 * b + 2];
          r.seconds = el;
          r.lowp_iters = 0;
        }
        if (!std::isfinite(rn)) bad = true;
        if (rn < opts->tol) {
          done[b] = 1;
          ++ndone;
          if (reports) reports[b].converged = 1;
        }
      }
      if (bad) break;
    }
    if (n_converged) *n_converged = ndone;
    if (bad) return int(CC_EDIVERGED);
    return ndone == n ? int(CC_OK) : int(CC_ENOTCONV);
  });
}

int cc_batch_profile(cc_batch *B, int enable) {
  if (!B) return bfail(nullptr, CC_EINVAL, "batch is NULL");
  B->profiling = enable != 0;
  B->step_ms.assign(B->gsteps.size(), 0.0);
  B->prof_calls = 0;
  return CC_OK;
}

const char *cc_batch_profile_table(const cc_batch *B) {
  static thread_local std::string s;
  s.clear();
  if (!B) return s.c_str();
  static const char *kinds[] = {"PERMUTE", "GEMM", "OUTER", "FILL", "TAU_E", "ASSEMBLE", "R1UPD", "FINALIZE", "TRIPLES", "PAIR"};
  s = "# step kind tag calls total_ms avg_ms flops_per_call\n";
  for (size_t k = 0; k < B->gsteps.size() && k < B->step_ms.size(); ++k) {
    const auto &g = B->gsteps[k];
    std::string tag = g.tag.empty() ? "-" : g.tag;
    for (auto &c : tag)
      if (c == ' ') c = '_';
    if (g.kind == ccmi::Step::GEMM)
      tag += std::string("@") + (B->prec == ccmi::PREC_F64 ? ccmi::gemm_f64_tile_name(g.tile)
                                                           : ccmi::gemm_lowp_tile_name(B->prec, g.tile)) +
             (g.lp ? "/copies" : "");
    const double avg = B->prof_calls ? B->step_ms[k] / double(B->prof_calls) : 0.0;
    s += std::to_string(k) + " " + kinds[g.kind] + " " + tag + " " + std::to_string(B->prof_calls) + " " +
         std::to_string(B->step_ms[k]) + " " + std::to_string(avg) + " " + std::to_string(g.flops) + "\n";
  }
  return s.c_str();
}

double cc_batch_flops(const cc_batch *B) { return B ? B->flops : 0.0; }

}  // extern "C"
