// Contraction list of the spin-orbital CCD/CCSD residual, the planner that
// turns each binary contraction into permute -> MFMA GEMM -> permute-accumulate
// steps (paper, Sec. "Tensor contractions": transpose-transpose-GEMM-transpose),
// and the executor that enqueues those steps on one HIP stream.
//
// The list follows the usual factorisation of the spin-orbital CCSD
// equations into one- and two-body intermediates (F_ae, F_mi, F_me, W_mnij,
// W_mbej), with two changes that keep every operation binary and bound the
// memory (paper, Sec. "Secondary optimization": intermediates that are too
// large are not formed): the four-virtual intermediate W_abef is never built
// -- its <ab||ef> part is the particle-particle ladder contracted directly
// with the stored vvvv block, its t1 part goes through Z_ij^am, and its
// tau<mn||ef>tau part is folded into W_mnij with a factor 1/2.
//
// Every integral is used in the orientation <pq||rs> where p, q are creation
// indices of H_N (external virtual or summed occupied indices) and r, s are
// annihilation indices; with complex Hermitian integrals the blocks not stored
// are conjugates of stored ones (driver <ab||ij> = conj <ij||ab>).
#include "plan.hpp"

#include <algorithm>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <mutex>
#include <set>
#include <sstream>

namespace ccmi {
namespace {

// clang-format off
// C, labels, alpha, A, labels, B, labels, conjA, conjB, P(xy), needs_t1, tag
const OpSpec kOps[] = {
  // F_me = f_me + t_n^f <mn||ef>
  {"Fme", "me", 1.0, "fov", "me", nullptr, nullptr, false, false, nullptr, true, "Fme_f"},
  {"Fme", "me", 1.0, "oovv", "mnef", "t1", "nf", false, false, nullptr, true, "Fme_t1"},
  // F_ae = f_ae - 1/2 t_m^a f_me + t_m^f <ma||fe> - 1/2 taut_mn^af <mn||ef>
  {"Fae", "ae", 1.0, "fvv", "ae", nullptr, nullptr, false, false, nullptr, false, "Fae_f"},
  {"Fae", "ae", -0.5, "t1", "ma", "fov", "me", false, false, nullptr, true, "Fae_ft1"},
  {"Fae", "ae", 1.0, "ovvv", "mafe", "t1", "mf", false, false, nullptr, true, "Fae_t1"},
  {"Fae", "ae", -0.5, "taut", "mnaf", "oovv", "mnef", false, false, nullptr, false, "Fae_t2"},
  // F_mi = f_mi + 1/2 t_i^e f_me + t_n^e <mn||ie> + 1/2 taut_in^ef <mn||ef>
  {"Fmi", "mi", 1.0, "foo", "mi", nullptr, nullptr, false, false, nullptr, false, "Fmi_f"},
  {"Fmi", "mi", 0.5, "fov", "me", "t1", "ie", false, false, nullptr, true, "Fmi_ft1"},
  {"Fmi", "mi", 1.0, "ooov", "mnie", "t1", "ne", false, false, nullptr, true, "Fmi_t1"},
  {"Fmi", "mi", 0.5, "oovv", "mnef", "taut", "inef", false, false, nullptr, false, "Fmi_t2"},
  // W_mnij = <mn||ij> + P(ij) t_j^e <mn||ie> + 1/2 tau_ij^ef <mn||ef>
  {"Wmnij", "mnij", 1.0, "oooo", "mnij", nullptr, nullptr, false, false, nullptr, false, "Wmnij_v"},
  {"Wmnij", "mnij", 1.0, "ooov", "mnie", "t1", "je", false, false, "ij", true, "Wmnij_t1"},
  {"Wmnij", "mnij", 0.5, "oovv", "mnef", "tau", "ijef", false, false, nullptr, false, "Wmnij_tau"},
  // W_mbej (stored [j][b][m][e]) = <mb||ej> + t_j^f <mb||ef> - t_n^b <mn||ej>
  //                               - (1/2 t_jn^fb + t_j^f t_n^b) <mn||ef>
  {"Wjbme", "jbme", 1.0, "ovvo", "mbej", nullptr, nullptr, false, false, nullptr, false, "Wmbej_v"},
  {"Wjbme", "jbme", 1.0, "ovvv", "mbef", "t1", "jf", false, false, nullptr, true, "Wmbej_ovvv"},
  {"Wjbme", "jbme", 1.0, "ooov", "mnje", "t1", "nb", false, false, nullptr, true, "Wmbej_ooov"},
  {"Y", "jbnf", 0.5, "t2", "jnfb", nullptr, nullptr, false, false, nullptr, false, "Y_t2"},
  {"Y", "jbnf", 1.0, "t1", "jf", "t1", "nb", false, false, nullptr, true, "Y_t1t1"},
  {"Wjbme", "jbme", -1.0, "Y", "jbnf", "oovv", "mnef", false, false, nullptr, false, "Wmbej_ring"},
  // doubles: driver <ab||ij>
  {"XP", "ijab", 1.0, "oovv", "ijab", nullptr, nullptr, true, false, nullptr, false, "driver"},
  // P(ij)P(ab) ( t_im^ae W_mbej - t_i^e t_m^a <mb||ej> )
  {"Xr", "ijab", 1.0, "t2", "imae", "Wjbme", "jbme", false, false, nullptr, false, "ring"},
  {"Q", "imbj", 1.0, "t1", "ie", "ovvo", "mbej", false, false, nullptr, true, "Q"},
  {"Xr", "ijab", -1.0, "Q", "imbj", "t1", "ma", false, false, nullptr, true, "ring_t1t1"},
  // P(ij) t_i^e <ab||ej>,  <ab||ej> = -conj <je||ab>
  {"Xij", "ijab", -1.0, "t1", "ie", "ovvv", "jeab", false, true, nullptr, true, "abej_t1"},
  // -P(ab) t_m^a <mb||ij>,  <mb||ij> = conj <ij||mb>
  {"Xab", "ijab", -1.0, "t1", "ma", "ooov", "ijmb", false, true, nullptr, true, "mbij_t1"},
  // P(ab) t_ij^ae (F_be - 1/2 t_m^b F_me)
  {"FF", "be", 1.0, "Fae", "be", nullptr, nullptr, false, false, nullptr, false, "FF"},
  {"FF", "be", -0.5, "t1", "mb", "Fme", "me", false, false, nullptr, true, "FF_t1"},
  {"Xab", "ijab", 1.0, "t2", "ijae", "FF", "be", false, false, nullptr, false, "Fvv_t2"},
  // -P(ij) t_im^ab (F_mj + 1/2 t_j^e F_me)
  {"GG", "mj", 1.0, "Fmi", "mj", nullptr, nullptr, false, false, nullptr, false, "GG"},
  {"GG", "mj", 0.5, "Fme", "me", "t1", "je", false, false, nullptr, true, "GG_t1"},
  {"Xij", "ijab", -1.0, "t2", "imab", "GG", "mj", false, false, nullptr, false, "Foo_t2"},
  // 1/2 tau_mn^ab W_mnij
  // (plans made for a reduced precision permute tau to [ab][mn] so that the
  // LDS-direct kernels serve it: 0.66 -> 0.40 + 0.09 ms in split bf16; in FP64
  // the staged kernel on the stored layout is the faster, 0.93 against 0.99 ms)
  {"XP", "ijab", 0.5, "Wmnij", "mnij", "tau", "mnab", false, false, nullptr, false, "hh_ladder", true},
  // 1/2 <ab||ef> tau_ij^ef : the particle-particle ladder
  {"XP", "ijab", 0.5, "tau", "ijef", "vvvv", "abef", false, false, nullptr, false, "ladder"},
  // -1/2 P(ab) t_m^b Z_ij^am with Z_ij^am = <am||ef> tau_ij^ef = -Zs[ij][am]
  {"Zs", "ijam", 1.0, "tau", "ijef", "ovvv", "maef", false, false, nullptr, true, "Z"},
  {"Xab", "ijab", 0.5, "Zs", "ijam", "t1", "mb", false, false, nullptr, true, "Z_t1"},
  // singles
  {"R1", "ia", 1.0, "fov", "ia", nullptr, nullptr, true, false, nullptr, true, "R1_f"},
  {"R1", "ia", 1.0, "t1", "ie", "Fae", "ae", false, false, nullptr, true, "R1_Fae"},
  {"R1", "ia", -1.0, "Fmi", "mi", "t1", "ma", false, false, nullptr, true, "R1_Fmi"},
  {"R1", "ia", 1.0, "t2", "imae", "Fme", "me", false, false, nullptr, true, "R1_Fme"},
  {"R1", "ia", 1.0, "ovvo", "nafi", "t1", "nf", false, false, nullptr, true, "R1_ovvo"},
  {"R1", "ia", -0.5, "t2", "imef", "ovvv", "maef", false, false, nullptr, true, "R1_ovvv"},
  {"R1", "ia", -0.5, "t2", "mnae", "ooov", "mnie", false, false, nullptr, true, "R1_ooov"},
};
// clang-format on

int64_t dim_of(char c, int o, int v) {
  if (c >= 'i' && c <= 'n') return o;
  if (c >= 'a' && c <= 'h') return v;
  throw CCError(CC_EINTERNAL, std::string("bad index label ") + c);
}
char space_of(char c) { return (c >= 'i' && c <= 'n') ? 'o' : 'v'; }

std::vector<int64_t> dense_strides(const std::vector<int64_t> &dims) {
  std::vector<int64_t> s(dims.size(), 1);
  for (int i = int(dims.size()) - 2; i >= 0; --i) s[i] = s[i + 1] * dims[i + 1];
  return s;
}

void *dev_alloc(size_t bytes) {
  const char *f = std::getenv("CC_FAULT_INJECT");
  if (f && std::strcmp(f, "alloc") == 0) throw CCError(CC_ENOMEM, "allocation failure injected (CC_FAULT_INJECT=alloc)");
  void *ptr = nullptr;
  if (bytes == 0) bytes = 16;
  if (hipMalloc(&ptr, bytes) != hipSuccess) {
    (void)hipGetLastError();
    throw CCError(CC_ENOMEM, "hipMalloc of " + std::to_string(bytes) + " bytes failed");
  }
  return ptr;
}

struct Planner {
  cc_plan *p;
  int scratch = -1;        // shared buffer for GEMM outputs that need a permute
  int64_t scratch_elems = 0;
  int splitws = -1;        // split-K partial sums
  int64_t splitws_elems = 0;

  // Split-K partial sums, or room for the K-split tail of a launch whose last
  // round of workgroups would be mostly empty (real GEMMs only).
  void reserve_ws(Step &g, int64_t M, int64_t N, int64_t K) {
    const int64_t split = g.gemm.split > 1 ? int64_t(g.gemm.split) * M * N : 0;
    // complex: room for the tail of the realified M x 2N x 2K reduced-precision
    // GEMM, in complex elements
    const int64_t tail = p->cplx ? (gemm_tail_ws_bound(M, 2 * N, 2 * K) + 1) / 2 : gemm_tail_ws_bound(M, N, K);
    if (split > 0 || tail > 0) {
      if (p->private_work) {
        g.b2 = add_work("splitk_ws_" + std::to_string(p->slots.size()), {std::max(split, tail)});
        return;
      }
      splitws_elems = std::max<int64_t>(splitws_elems, std::max(split, tail));
      g.b2 = splitws;
    }
  }

  int slot(const std::string &name) {
    auto it = p->index.find(name);
    if (it == p->index.end()) throw CCError(CC_EINTERNAL, "unknown tensor " + name);
    return it->second;
  }

  int add_slot(const std::string &name, const std::string &spaces, bool constant, bool external,
               bool owned) {
    Slot s;
    s.name = name;
    s.spaces = spaces;
    s.elems = 1;
    for (char c : spaces) {
      const int64_t d = (c == 'o') ? p->o : p->v;
      s.dims.push_back(d);
      s.elems *= d;
    }
    s.constant = constant;
    s.external = external;
    s.owned = owned;
    p->slots.push_back(s);
    const int id = int(p->slots.size()) - 1;
    p->index[name] = id;
    return id;
  }

  int add_work(const std::string &name, const std::vector<int64_t> &dims) {
    Slot s;
    s.name = name;
    s.dims = dims;
    s.elems = 1;
    for (auto d : dims) s.elems *= d;
    s.owned = true;
    p->slots.push_back(s);
    const int id = int(p->slots.size()) - 1;
    p->index[name] = id;
    return id;
  }

  std::vector<int64_t> label_dims(const std::string &l) {
    std::vector<int64_t> d;
    for (char c : l) d.push_back(dim_of(c, p->o, p->v));
    return d;
  }

  void check_labels(int s, const std::string &l) {
    const Slot &sl = p->slots[s];
    if (sl.dims.size() != l.size()) throw CCError(CC_EINTERNAL, "rank mismatch for " + sl.name + "[" + l + "]");
    if (!sl.spaces.empty())
      for (size_t i = 0; i < l.size(); ++i)
        if (space_of(l[i]) != sl.spaces[i])
          throw CCError(CC_EINTERNAL, "space mismatch for " + sl.name + "[" + l + "]");
  }

  bool is_const(int s) { return p->slots[s].constant; }

  std::vector<Step> &stream_for(int src) { return is_const(src) ? p->setup : p->iter; }

  // dst[dl] (+)= alpha * conj?(src[sl]); beta decided by first touch.
  void accumulate(int src, const std::string &sl, bool conj, int dst, const std::string &dl,
                  double alpha, const char *swap, std::vector<Step> &out, bool force_first,
                  const std::vector<int64_t> *src_dims = nullptr) {
    const auto sst = dense_strides(src_dims ? *src_dims : p->slots[src].dims);
    const auto dst_dims = p->slots[dst].dims;
    const auto dstr = dense_strides(dst_dims);
    auto make = [&](const std::string &lab, double a, double b) {
      Step st;
      st.kind = Step::PERMUTE;
      st.a = src;
      st.c = dst;
      st.perm.rank = int(dl.size());
      for (size_t d = 0; d < dl.size(); ++d) {
        st.perm.out_dims[d] = dst_dims[d];
        st.perm.out_strides[d] = dstr[d];
        const size_t pos = sl.find(lab[d]);
        if (pos == std::string::npos) throw CCError(CC_EINTERNAL, "label missing in accumulate");
        st.perm.in_strides[d] = sst[pos];
      }
      st.perm.alpha = a;
      st.perm.beta = b;
      st.perm.conj = conj ? 1 : 0;
      st.nelem = p->slots[dst].elems;
      st.tag = p->slots[src].name + "[" + sl + "]->" + p->slots[dst].name + "[" + lab + "]";
      out.push_back(st);
    };
    const bool first = force_first || !p->touched[dst];
    make(dl, alpha, first ? 0.0 : 1.0);
    if (swap) {
      std::string sw = dl;
      for (auto &c : sw) {
        if (c == swap[0]) c = swap[1];
        else if (c == swap[1]) c = swap[0];
      }
      make(sw, -alpha, 1.0);
    }
    p->touched[dst] = true;
    p->version[dst]++;
  }

  // A view of tensor s with its labels rearranged to `target` (cached).
  int view(int s, const std::string &sl, const std::string &target, bool conj) {
    if (sl == target && !(conj && p->cplx)) return s;
    const bool cj = conj && p->cplx;
    std::string key = p->slots[s].name + "|" + target + "|" + (cj ? "c" : "n") + "|" +
                      std::to_string(p->version[s]) + "|" + sl;
    auto it = p->view_cache.find(key);
    if (it != p->view_cache.end()) return it->second;
    const int v = add_work(p->slots[s].name + "_" + target + (cj ? "_conj" : ""), label_dims(target));
    p->slots[v].constant = is_const(s);
    std::vector<Step> &out = stream_for(s);
    // a fresh buffer: write with beta = 0
    const bool saved = p->touched[v];
    accumulate(s, sl, cj, v, target, 1.0, nullptr, out, true);
    p->touched[v] = saved;
    p->view_cache[key] = v;
    return v;
  }

  static std::string order_in(const std::string &lab, const std::set<char> &set) {
    std::string r;
    for (char c : lab)
      if (set.count(c)) r += c;
    return r;
  }

  void contract(const OpSpec &op) {
    const int c = slot(op.C), a = slot(op.A), b = slot(op.B);
    const std::string cl = op.cl, al = op.al, bl = op.bl;
    check_labels(c, cl);
    check_labels(a, al);
    check_labels(b, bl);
    std::set<char> sA(al.begin(), al.end()), sB(bl.begin(), bl.end()), sC(cl.begin(), cl.end());
    std::set<char> K;
    for (char x : sA)
      if (sB.count(x)) K.insert(x);
    for (char x : sC)
      if (!(sA.count(x) ^ sB.count(x))) throw CCError(CC_EINTERNAL, std::string("label ") + x + " of " + op.tag);
    for (char x : K)
      if (sC.count(x)) throw CCError(CC_EINTERNAL, "hadamard label");
    if (K.empty()) return outer(op, c, a, b);

    struct Cand {
      bool swap;
      std::string rows, cols, k;
      bool xm, ym, cm, xkc, ykc;
      double cost;
    } best{};
    best.cost = 1e300;
    for (int sw = 0; sw < 2; ++sw) {
      const int X = sw ? b : a, Y = sw ? a : b;
      const std::string xl = sw ? bl : al, yl = sw ? al : bl;
      std::set<char> rs, cs;
      for (char x : xl)
        if (sC.count(x)) rs.insert(x);
      for (char x : yl)
        if (sC.count(x)) cs.insert(x);
      const std::string rowOpt[2] = {order_in(cl, rs), order_in(xl, rs)};
      const std::string colOpt[2] = {order_in(cl, cs), order_in(yl, cs)};
      const std::string kOpt[2] = {order_in(xl, K), order_in(yl, K)};
      for (int ri = 0; ri < 2; ++ri)
        for (int ci = 0; ci < 2; ++ci)
          for (int ki = 0; ki < 2; ++ki) {
            Cand cd;
            cd.swap = sw;
            cd.rows = rowOpt[ri];
            cd.cols = colOpt[ci];
            cd.k = kOpt[ki];
            cd.xm = (xl == cd.rows + cd.k) || (xl == cd.k + cd.rows);
            cd.xkc = (xl == cd.rows + cd.k);
            cd.ym = (yl == cd.cols + cd.k) || (yl == cd.k + cd.cols);
            cd.ykc = (yl == cd.cols + cd.k);
            cd.cm = (cl == cd.rows + cd.cols) && op.swap == nullptr;
            const bool cjx = (sw ? op.conjB : op.conjA) && p->cplx;
            const bool cjy = (sw ? op.conjA : op.conjB) && p->cplx;
            if (cjx) cd.xm = false;  // conjugation is applied while permuting
            if (cjy) cd.ym = false;
            if (op.kc && p->prec != PREC_F64) {  // only the K-contiguous order counts as matched
              cd.xm = cd.xm && cd.xkc;
              cd.ym = cd.ym && cd.ykc;
            }
            double cost = 0.0;
            auto opcost = [&](int s, bool matched) {
              if (matched) return 0.0;
              return (is_const(s) ? 0.01 : 2.0) * double(p->slots[s].elems);
            };
            cost += opcost(X, cd.xm) + opcost(Y, cd.ym);
            if (!cd.cm) cost += 3.0 * double(p->slots[c].elems);
            if (!(cd.xm ? cd.xkc : true)) cost += 1e-3;  // prefer K-contiguous panels
            if (!(cd.ym ? cd.ykc : true)) cost += 1e-3;
            cost += sw * 1e-6;
            cd.cost = cost;
            if (cd.cost < best.cost) best = cd;
          }
    }
    const int X = best.swap ? b : a, Y = best.swap ? a : b;
    const std::string xl = best.swap ? bl : al, yl = best.swap ? al : bl;
    const bool cjx = (best.swap ? op.conjB : op.conjA), cjy = (best.swap ? op.conjA : op.conjB);
    int xs = X, ys = Y;
    bool xkc = best.xkc, ykc = best.ykc;
    if (!best.xm) {
      xs = view(X, xl, best.rows + best.k, cjx);
      xkc = true;
    }
    if (!best.ym) {
      ys = view(Y, yl, best.cols + best.k, cjy);
      ykc = true;
    }
    int64_t M = 1, N = 1, Kd = 1;
    for (char x : best.rows) M *= dim_of(x, p->o, p->v);
    for (char x : best.cols) N *= dim_of(x, p->o, p->v);
    for (char x : best.k) Kd *= dim_of(x, p->o, p->v);
    Step g;
    g.kind = Step::GEMM;
    g.a = xs;
    g.b = ys;
    g.gemm.M = M;
    g.gemm.N = N;
    g.gemm.K = Kd;
    g.gemm.sam = xkc ? Kd : 1;
    g.gemm.sak = xkc ? 1 : M;
    g.gemm.sbn = ykc ? Kd : 1;
    g.gemm.sbk = ykc ? 1 : N;
    g.gemm.ldc = N;
    g.gemm.conj_a = 0;
    g.gemm.conj_b = 0;
    g.flops = (p->cplx ? 8.0 : 2.0) * double(M) * double(N) * double(Kd);
    g.tag = op.tag;
    g.gemm.ladder = std::string(op.tag) == "ladder" ? 1 : 0;
    g.gemm.split = gemm_split_pick(M, N, Kd, -1);
    reserve_ws(g, M, N, Kd);
    g.tile = p->cplx ? -1 : gemm_f64_pick(M, N, Kd, xkc, ykc);
    if (best.cm) {
      g.c = c;
      g.gemm.alpha = op.alpha;
      g.gemm.beta = p->touched[c] ? 1.0 : 0.0;
      p->touched[c] = true;
      p->version[c]++;
      p->iter.push_back(g);
    } else {
      const int64_t need = M * N;
      int sc = scratch;
      if (p->private_work) sc = add_work("scratch_" + std::to_string(p->slots.size()), {need});
      else if (need > scratch_elems) scratch_elems = need;
      g.c = sc;
      g.gemm.alpha = op.alpha;
      g.gemm.beta = 0.0;
      p->iter.push_back(g);
      const auto tdims = label_dims(best.rows + best.cols);
      accumulate(sc, best.rows + best.cols, false, c, cl, 1.0, op.swap, p->iter, false, &tdims);
    }
    p->flops_per_iter += g.flops;
    if (std::string(op.tag) == "ladder") p->ladder_flops += g.flops;
  }

  void outer(const OpSpec &op, int c, int a, int b) {
    if (op.swap) throw CCError(CC_EINTERNAL, "antisymmetrised outer product");
    const std::string cl = op.cl, al = op.al, bl = op.bl;
    if (!p->touched[c]) {
      Step f;
      f.kind = Step::FILL;
      f.c = c;
      f.nelem = p->slots[c].elems;
      f.tag = "zero " + p->slots[c].name;
      p->iter.push_back(f);
      p->touched[c] = true;
    }
    Step st;
    st.kind = Step::OUTER;
    st.a = a;
    st.b = b;
    st.c = c;
    st.outer.rank = int(cl.size());
    const auto sa = dense_strides(p->slots[a].dims), sb = dense_strides(p->slots[b].dims);
    for (size_t d = 0; d < cl.size(); ++d) {
      st.outer.dims[d] = p->slots[c].dims[d];
      const size_t pa = al.find(cl[d]), pb = bl.find(cl[d]);
      st.outer.sa[d] = pa == std::string::npos ? 0 : sa[pa];
      st.outer.sb[d] = pb == std::string::npos ? 0 : sb[pb];
    }
    st.outer.alpha = op.alpha;
    st.outer.conj_a = op.conjA && p->cplx;
    st.outer.conj_b = op.conjB && p->cplx;
    st.nelem = p->slots[c].elems;
    st.tag = op.tag;
    p->iter.push_back(st);
    p->version[c]++;
  }

  // ---- packed index pairs (i<j, m<n, a<b, e<f) ----------------------------
  int tau_packed_version = -1;

  // Row length of a packed e<f dimension that a GEMM sums over: padded with
  // zero columns to a multiple of 32, so that every GEMM configuration takes
  // whole K chunks (the padding adds zero products).
  static int64_t packed_ld(int64_t n) { return std::max<int64_t>(32, (n + 31) / 32 * 32); }

  // ldq: row stride of the packed side (0: dense, nq)
  Step pair_step(int a, int c, int64_t np, int64_t nq, int64_t n1, int64_t n2, int64_t n3, int rows, int cols,
                 int mode, const char *tag, int64_t ldq = 0) {
    Step st;
    st.kind = Step::PAIR;
    st.a = a;
    st.c = c;
    st.pair_np = np;
    st.pair_nq = nq;
    st.pair_ldq = ldq > 0 ? ldq : nq;
    st.pair_n[0] = n1;
    st.pair_n[1] = n2;
    st.pair_n[2] = n3;
    st.pair_rows = rows;
    st.pair_cols = cols;
    st.pair_mode = mode;
    st.tag = tag;
    return st;
  }

  // tau packed over i<j (rows) and e<f (columns), gathered once per version of tau
  int ensure_taup() {
    const int tau = slot("tau"), tp = slot("taup");
    if (tau_packed_version != p->version[tau]) {
      const int64_t no = int64_t(p->o) * (p->o - 1) / 2, nv = int64_t(p->v) * (p->v - 1) / 2;
      p->iter.push_back(pair_step(tau, tp, no, nv, p->o, p->v, p->v, 0, 1, 0, "pack_tau", packed_ld(nv)));
      p->version[tp]++;
      tau_packed_version = p->version[tau];
    }
    return tp;
  }

  // lda, ldb: row strides of the stored operands ([M][K] or [K][M], ...);
  // K may include zero padding columns, Kalg is the summed pair count
  Step packed_gemm(int a, int b, int c, int64_t M, int64_t N, int64_t K, bool akc, bool bkc, double alpha,
                   const char *tag, int64_t lda, int64_t ldb, int64_t Kalg) {
    Step g;
    g.kind = Step::GEMM;
    g.a = a;
    g.b = b;
    g.c = c;
    g.gemm.M = M;
    g.gemm.N = N;
    g.gemm.K = K;
    g.gemm.sam = akc ? lda : 1;
    g.gemm.sak = akc ? 1 : lda;
    g.gemm.sbn = bkc ? ldb : 1;
    g.gemm.sbk = bkc ? 1 : ldb;
    g.gemm.ldc = N;
    g.gemm.alpha = alpha;
    g.gemm.beta = 0.0;
    g.gemm.ladder = std::string(tag) == "ladder" ? 1 : 0;
    g.flops = (p->cplx ? 8.0 : 2.0) * double(M) * double(N) * double(Kalg);
    g.tag = tag;
    g.gemm.split = gemm_split_pick(M, N, K, -1);
    reserve_ws(g, M, N, K);
    g.tile = p->cplx ? -1 : gemm_f64_pick(M, N, K, akc, bkc);
    p->flops_per_iter += g.flops;
    if (g.gemm.ladder) p->ladder_flops += g.flops;
    return g;
  }

  // Contractions whose summed index pair (e<f or m<n) and output pairs
  // (i<j, a<b) can run over canonical pairs only: the summand is symmetric
  // under the summed swap (factor 2 on a sum over half of it), and only the
  // canonical i<j (a<b) elements of the target are read later.
  //   ladder:    XP(ij,ab)  += 1/2 sum_ef tau(ij,ef) <ab||ef>
  //   hh_ladder: XP(ij,ab)  += 1/2 sum_mn W(mn,ij) tau(mn,ab)
  //   Z:         Zs(ij,am)   =     sum_ef tau(ij,ef) <ma||ef>
  bool packed_op(const OpSpec &op) {
    const std::string tag = op.tag;
    if (tag != "ladder" && tag != "hh_ladder" && tag != "Z") return false;
    const int64_t no = int64_t(p->o) * (p->o - 1) / 2, nv = int64_t(p->v) * (p->v - 1) / 2;
    const int c = slot(op.C);
    if (no == 0 || nv == 0) {  // no canonical pair: the term contributes nothing that is read
      if (tag == "Z") {
        if (!p->touched[c]) {
          Step f;
          f.kind = Step::FILL;
          f.c = c;
          f.nelem = p->slots[c].elems;
          f.tag = "zero Zs";
          p->iter.push_back(f);
          p->touched[c] = true;
          p->version[c]++;
        }
      }
      return true;
    }
    const int tp = ensure_taup();
    const int xp = slot("XPp");
    const int64_t nvp = packed_ld(nv);  // e<f columns of taup, vvvvp, ovvvp (zero padded)
    if (tag == "ladder") {
      p->iter.push_back(
          packed_gemm(tp, slot("vvvvp"), xp, no, nv, nvp, true, true, 2.0 * op.alpha, "ladder", nvp, nvp, nv));
      p->iter.push_back(pair_step(xp, c, no, nv, p->o, p->v, p->v, 0, 1, 1, "unpack_ladder"));
    } else if (tag == "hh_ladder") {
      const int wg = slot("Wp");
      p->iter.push_back(pair_step(slot("Wmnij"), wg, no, no, p->o, p->o, p->o, 0, 0, 0, "pack_Wmnij"));
      p->version[wg]++;
      // C(ij, ab) = sum_{m<n} Wp[mn][ij] taup[mn][ab]: both operands stored [K][...]
      p->iter.push_back(packed_gemm(wg, tp, xp, no, nv, no, false, false, 2.0 * op.alpha, "hh_ladder", no, nvp, no));
      p->iter.push_back(pair_step(xp, c, no, nv, p->o, p->v, p->v, 0, 1, 1, "unpack_hh_ladder"));
    } else {
      const int zp = slot("Zp");
      const int64_t nov = int64_t(p->o) * p->v;
      p->iter.push_back(packed_gemm(tp, slot("ovvvp"), zp, no, nov, nvp, true, true, 2.0 * op.alpha, "Z", nvp, nvp, nv));
      // Zs[i][j][a][m] (i<j) <- Zp[ij][m a]; rows i>j stay as set up (zero)
      p->iter.push_back(pair_step(zp, c, no, nov, p->o, p->v, p->o, 0, 3, 2, "unpack_Z"));
    }
    if (!p->touched[c] && tag != "Z") throw CCError(CC_EINTERNAL, "packed op before the first write of its target");
    p->touched[c] = true;
    p->version[c]++;
    return true;
  }

  void unary(const OpSpec &op) {
    const int c = slot(op.C), a = slot(op.A);
    check_labels(c, op.cl);
    check_labels(a, op.al);
    accumulate(a, op.al, op.conjA && p->cplx, c, op.cl, op.alpha, op.swap, p->iter, false);
    p->iter.back().tag = op.tag;
  }

  void build(const cc_system *sys) {
    const bool ccsd = p->method == CC_CCSD;
    const char *inputs[] = {"foo", "fov", "fvv", "oooo", "ooov", "oovv", "ovvo", "ovvv", "vvvv"};
    const char *spaces[] = {"oo", "ov", "vv", "oooo", "ooov", "oovv", "ovvo", "ovvv", "vvvv"};
    const void *ptrs[] = {sys->f_oo, sys->f_ov, sys->f_vv, sys->oooo, sys->ooov,
                          sys->oovv, sys->ovvo, sys->ovvv, sys->vvvv};
    for (int i = 0; i < 9; ++i) {
      const int s = add_slot(inputs[i], spaces[i], true, false, false);
      p->slots[s].ptr = const_cast<void *>(ptrs[i]);
    }
    add_slot("t1", "ov", false, true, false);
    add_slot("t2", "oovv", false, true, false);
    if (ccsd) {
      add_slot("tau", "oovv", false, false, true);
      add_slot("taut", "oovv", false, false, true);
    } else {
      p->index["tau"] = p->index["t2"];
      p->index["taut"] = p->index["t2"];
    }
    const char *work[][2] = {{"Fme", "ov"},  {"Fae", "vv"},   {"Fmi", "oo"}, {"Wmnij", "oooo"},
                             {"Wjbme", "ovov"}, {"Y", "ovov"}, {"XP", "oovv"}, {"Xij", "oovv"},
                             {"Xab", "oovv"}, {"Xr", "oovv"},  {"R1", "ov"},   {"Zs", "oovo"},
                             {"FF", "vv"},   {"GG", "oo"},    {"Q", "oovo"}};
    for (auto &w : work) add_slot(w[0], w[1], false, false, true);
    std::vector<OpSpec> custom_ops;
    if (p->custom) {
      for (const OpText &o : p->custom->ops)
        if (o.A == "t3" || o.B == "t3" || o.C == "Y3") p->triples = true;
      if (p->triples) {
        if (!ccsd) throw CCError(CC_EINVAL, "op list: triples need the CCSD method (singles and doubles)");
        add_slot("t3", "ooovvv", false, true, false);
        add_slot("Y3", "ooovvv", false, false, true);
      }
      for (const auto &w : p->custom->work) {
        if (p->index.count(w.first)) throw CCError(CC_EINVAL, "op list: tensor " + w.first + " already exists");
        for (char c : w.second)
          if (c != 'o' && c != 'v') throw CCError(CC_EINVAL, "op list: spaces of " + w.first + " must be o/v");
        add_slot(w.first, w.second, false, false, true);
      }
      for (const OpText &o : p->custom->ops) {
        const bool un = o.B.empty();
        custom_ops.push_back(OpSpec{o.C.c_str(), o.cl.c_str(), o.alpha, o.A.c_str(), o.al.c_str(),
                                    un ? nullptr : o.B.c_str(), un ? nullptr : o.bl.c_str(), o.conjA, o.conjB,
                                    o.swap.empty() ? nullptr : o.swap.c_str(),
                                    o.A == "t1" || (!un && o.B == "t1"), o.tag.c_str()});
      }
    }
    scratch = add_work("scratch", {1});
    splitws = add_work("splitk_ws", {1});
    if (p->packed) {
      if (p->custom) throw CCError(CC_EINVAL, "packed pairs apply to the built-in table");
      const int64_t no0 = int64_t(p->o) * (p->o - 1) / 2, nv0 = int64_t(p->v) * (p->v - 1) / 2;
      const int64_t no = std::max<int64_t>(1, no0), nv = std::max<int64_t>(1, nv0);
      const int64_t nov = int64_t(p->o) * p->v;
      const int64_t nvp = packed_ld(nv);
      const int tpk = add_work("taup", {no, nvp});
      add_work("XPp", {no, nv});
      add_work("Wp", {no, no});
      add_work("Zp", {no, nov});
      const int vp = add_work("vvvvp", {nv, nvp});
      const int op_ = add_work("ovvvp", {nov, nvp});
      p->slots[vp].constant = true;
      p->slots[op_].constant = true;
      // padding columns start at zero and are never written afterwards
      for (int z : {tpk, vp, op_}) {
        Step f;
        f.kind = Step::FILL;
        f.c = z;
        f.nelem = p->slots[z].elems;
        f.tag = "zero packed padding";
        p->setup.push_back(f);
      }
      if (nv0 > 0) {
        p->setup.push_back(pair_step(slot("vvvv"), vp, nv, nv, p->v, p->v, p->v, 1, 1, 0, "pack_vvvv", nvp));
        p->setup.push_back(pair_step(slot("ovvv"), op_, nov, nv, p->v, p->v, p->v, 2, 1, 0, "pack_ovvv", nvp));
      }
      // rows i > j of Zs are never written by the packed Z: keep them zero
      Step f;
      f.kind = Step::FILL;
      f.c = slot("Zs");
      f.nelem = p->slots[f.c].elems;
      f.tag = "zero Zs";
      p->setup.push_back(f);
    }

    Step te;
    te.kind = Step::TAU_E;
    te.tag = "tau_energy";
    p->iter.push_back(te);
    auto run_ops = [&](const OpSpec *ops, size_t n) {
      for (size_t q = 0; q < n; ++q) {
        const OpSpec &op = ops[q];
        if (op.needs_t1 && !ccsd) {
          if (p->custom) throw CCError(CC_EINVAL, std::string("op list: ") + op.tag + " reads t1 in a CCD plan");
          continue;
        }
        if (op.B == nullptr) unary(op);
        else if (p->packed && packed_op(op)) continue;
        else contract(op);
      }
    };
    if (p->custom) {
      try {
        run_ops(custom_ops.data(), custom_ops.size());
      } catch (const CCError &e) {
        if (e.status != CC_EINTERNAL) throw;
        throw CCError(CC_EINVAL, std::string("op list: ") + e.what());
      }
    } else {
      run_ops(kOps, sizeof(kOps) / sizeof(kOps[0]));
    }
    for (const char *x : {"XP", "Xij", "Xab", "Xr"}) {
      const int s = slot(x);
      if (!p->touched[s]) {
        Step f;
        f.kind = Step::FILL;
        f.c = s;
        f.nelem = p->slots[s].elems;
        f.tag = std::string("zero ") + x;
        p->iter.push_back(f);
      }
    }
    if (p->triples) {
      const int y = slot("Y3");
      if (!p->touched[y]) {
        Step f;
        f.kind = Step::FILL;
        f.c = y;
        f.nelem = p->slots[y].elems;
        f.tag = "zero Y3";
        p->iter.push_back(f);
      }
    }
    Step as;
    as.kind = Step::ASSEMBLE;
    as.tag = "r2_assemble_update";
    p->iter.push_back(as);
    if (p->triples) {
      Step t3s;
      t3s.kind = Step::TRIPLES;
      t3s.tag = "r3_antisymmetrise_update";
      p->iter.push_back(t3s);
    }
    if (ccsd) {
      Step r1;
      r1.kind = Step::R1UPD;
      r1.tag = "r1_update";
      p->iter.push_back(r1);
    }
    Step fin;
    fin.kind = Step::FINALIZE;
    fin.tag = "finalize";
    p->iter.push_back(fin);
    p->slots[scratch].dims = {std::max<int64_t>(scratch_elems, 1)};
    p->slots[scratch].elems = std::max<int64_t>(scratch_elems, 1);
    p->slots[splitws].dims = {std::max<int64_t>(splitws_elems, 1)};
    p->slots[splitws].elems = std::max<int64_t>(splitws_elems, 1);
  }
};

}  // namespace

void *ptr_of(cc_plan *p, int s) {
  const Slot &sl = p->slots[s];
  if (sl.external) return sl.name == "t1" ? p->t1 : (sl.name == "t3" ? p->t3 : p->t2);
  return sl.ptr;
}

namespace {

int64_t slot_elems(const cc_plan *p, int s) {
  const Slot &sl = p->slots[s];
  if (sl.external) {
    if (sl.name == "t1") return int64_t(p->o) * p->v;
    if (sl.name == "t3") return int64_t(p->o) * p->o * p->o * p->v * p->v * p->v;
    return int64_t(p->o) * p->o * p->v * p->v;
  }
  return sl.elems;
}

// Point a reduced-precision GEMM at the converted copies of its operands,
// converting a copy first when its slot was written since the last
// conversion in this run.
void use_shadows(cc_plan *p, GemmDesc &d, const Step &st, hipStream_t s, bool convert) {
  for (int which = 0; which < 2; ++which) {
    const int sl = which ? st.b : st.a;
    void *sh = p->shadow[sl];
    if (!sh) return;
    if (convert && !p->shadow_ok[sl]) {
      convert_shadow(p->cur_prec, static_cast<const double *>(ptr_of(p, sl)), slot_elems(p, sl), sh, s);
      p->shadow_ok[sl] = 1;
    }
  }
  d.A = p->shadow[st.a];
  d.B = p->shadow[st.b];
  d.a_plane = slot_elems(p, st.a);
  d.b_plane = slot_elems(p, st.b);
  d.lp_in = 1;
}

// The realified B' copy of a complex slot for rows of K complex elements.
void convert_b_form(cc_plan *p, BForm &bf, int prec, hipStream_t s) {
  const int64_t n = slot_elems(p, bf.slot);
  CC_REQUIRE(bf.ptr && bf.K > 0 && n % bf.K == 0, CC_EINTERNAL, "complex B operand rows");
  realify_complex(prec, 1, static_cast<const double *>(ptr_of(p, bf.slot)), nullptr, n / bf.K, bf.K, bf.K, 1, bf.ptr,
                  s);
}

// Complex reduced precision: the realified real GEMM (M x 2N x 2K) on the
// interleaved copy of A and the realified copy of B, converting a copy first
// when its slot was written since the last conversion in this run.
void use_shadows_c(cc_plan *p, GemmDesc &d, const Step &st, hipStream_t s, bool convert) {
  const int prec = p->cur_prec;
  const int64_t na = slot_elems(p, st.a), nb = slot_elems(p, st.b);
  CC_REQUIRE(st.bform >= 0 && p->shadow[st.a] && p->bforms[st.bform].ptr, CC_EINTERNAL,
             "complex operand copies not prepared");
  BForm &bf = p->bforms[st.bform];
  if (convert && !p->shadow_ok[st.a]) {
    convert_shadow(prec, static_cast<const double *>(ptr_of(p, st.a)), 2 * na, p->shadow[st.a], s);
    p->shadow_ok[st.a] = 1;
  }
  if (convert && !bf.ok) {
    convert_b_form(p, bf, prec, s);
    bf.ok = 1;
  }
  d = realified_desc(d, p->shadow[st.a], bf.ptr);
  d.a_plane = 2 * na;
  d.b_plane = 4 * nb;
}

// The blocked split-bf16 copies serve a contraction when the plan runs in
// split bf16 and the configuration (the autotuner's, else the default)
// is an LDS-direct one that reads them, unless the autotuner timed that
// configuration faster on the row-major copies.
bool blocked_for(const cc_plan *p, const Step &st, int tile) {
  if (p->cur_prec != PREC_BF16X3 || st.blk_a < 0 || st.blk_b < 0 || st.blk_use == 0) return false;
  if (!p->bforms[st.blk_a].ptr || !p->bforms[st.blk_b].ptr) return false;
  if (tile < 0) tile = gemm_lowp_pick(PREC_BF16X3, st.gemm.M, p->cplx ? 2 * st.gemm.N : st.gemm.N);
  return gemm_lowp_tile_blocked(PREC_BF16X3, tile);
}

// rows of a blocked copy: the slot's rows of K (twice that for a realified B')
int64_t blocked_rows(const cc_plan *p, const BForm &bf) {
  return slot_elems(p, bf.slot) / bf.K * (bf.kind == 3 ? 2 : 1);
}

int64_t blocked_bytes(const cc_plan *p, const BForm &bf) {
  return blocked_plane(blocked_rows(p, bf), bf.kind >= 2 ? 2 * bf.K : bf.K) * 2 * int64_t(sizeof(uint16_t));
}

void convert_blocked_form(cc_plan *p, BForm &bf, hipStream_t s) {
  const double *src = static_cast<const double *>(ptr_of(p, bf.slot));
  if (bf.kind == 1) convert_blocked(src, nullptr, blocked_rows(p, bf), bf.K, bf.ptr, s);
  else realify_complex_blocked(bf.kind == 2 ? 0 : 1, src, slot_elems(p, bf.slot) / bf.K, bf.K, bf.ptr, s);
}

// Point a split-bf16 GEMM at the blocked copies of its operands, converting
// a copy first when its slot was written since the last conversion.
void use_blocked(cc_plan *p, GemmDesc &d, const Step &st, hipStream_t s, bool convert) {
  BForm &fa = p->bforms[st.blk_a], &fb = p->bforms[st.blk_b];
  for (BForm *f : {&fa, &fb})
    if (convert && !f->ok) {
      convert_blocked_form(p, *f, s);
      f->ok = 1;
    }
  if (p->cplx) {
    d = realified_desc(d, fa.ptr, fb.ptr);
    d.a_plane = blocked_plane(blocked_rows(p, fa), 2 * fa.K);
    d.b_plane = blocked_plane(blocked_rows(p, fb), 2 * fb.K);
  } else {
    d.A = fa.ptr;
    d.B = fb.ptr;
    d.a_plane = blocked_plane(blocked_rows(p, fa), fa.K);
    d.b_plane = blocked_plane(blocked_rows(p, fb), fb.K);
  }
  d.lp_in = 2;
}

void run_gemm(cc_plan *p, GemmDesc &d, const Step &st, hipStream_t s) {
  if (p->cplx && (p->cur_prec == PREC_F64 || !st.lowp_ok)) gemm_c128(d, s, st.tile_z);
  else if (p->cplx) {
    const int tile = st.tile_lp[p->cur_prec];
    if (blocked_for(p, st, tile)) use_blocked(p, d, st, s, true);
    else use_shadows_c(p, d, st, s, true);
    gemm_lowp(d, p->cur_prec, s, tile);
  } else if (p->cur_prec == PREC_F64 || !st.lowp_ok) gemm_f64(d, s, st.tile);
  else {
    const int tile = st.tile_lp[p->cur_prec];
    if (blocked_for(p, st, tile)) use_blocked(p, d, st, s, true);
    else use_shadows(p, d, st, s, true);
    gemm_lowp(d, p->cur_prec, s, tile);
  }
}

void invalidate(cc_plan *p, int sl) {
  if (sl >= 0 && !p->shadow_ok.empty()) p->shadow_ok[sl] = 0;
  for (BForm &bf : p->bforms)
    if (bf.slot == sl) bf.ok = 0;
}

// Mode 2: store X_ref and alpha X_ref Y (FP64), then C = beta C + that.
// Mode 1: C = beta C + alpha X_ref Y + alpha (X - X_ref) Y, the last product
// in reduced precision; its rounding error scales with |X - X_ref|.
void run_delta_gemm(cc_plan *p, GemmDesc &d, const Step &st, hipStream_t s) {
  DeltaRef &r = p->deltas[st.delta];
  // products of two varying operands are corrected in split bf16 only: two
  // FP32 products take as long as the FP64 one
  if (r.var == 2 && p->delta_prec != PREC_BF16X3) {
    gemm_f64(d, s, st.tile);
    return;
  }
  CC_REQUIRE(r.ref_op && r.ref_out && r.dshadow, CC_EINTERNAL, "reference buffers not prepared");
  const int var_slot = r.var ? st.b : st.a, con_slot = r.var ? st.a : st.b;
  const double *X = static_cast<const double *>(ptr_of(p, var_slot));
  double *C = static_cast<double *>(d.C);
  const int64_t w = p->cplx ? 2 : 1;  // doubles per element
  if (r.var == 2) {
    // A B = A_ref B_ref (FP64, stored) + (A - A_ref) B + A_ref (B - B_ref),
    // the two corrections in reduced precision: their error scales with the
    // change since the reference
    const double *A = static_cast<const double *>(ptr_of(p, st.a));
    const double *Bv = static_cast<const double *>(ptr_of(p, st.b));
    if (p->delta_mode == 2) {
      copy_f64(r.ref_op, A, r.n_op, s);
      copy_f64(r.ref_b, Bv, r.n_b, s);
      convert_shadow(p->delta_prec, A, r.n_op, r.ref_a_lp, s);
      GemmDesc g = d;
      g.C = r.ref_out;
      g.ldc = d.N;
      g.beta = 0.0;
      gemm_f64(g, s, st.tile);
      add_product(C, d.ldc, d.beta, r.ref_out, d.M, d.N, s);
      return;
    }
    add_product(C, d.ldc, d.beta, r.ref_out, d.M, d.N, s);
    convert_delta(p->delta_prec, A, r.ref_op, r.n_op, r.dshadow, s);
    convert_shadow(p->delta_prec, Bv, r.n_b, r.cur_b_lp, s);
    convert_delta(p->delta_prec, Bv, r.ref_b, r.n_b, r.dshadow_b, s);
    GemmDesc g = d;
    g.lp_in = 1;
    g.beta = 1.0;
    g.A = r.dshadow;
    g.a_plane = r.n_op;
    g.B = r.cur_b_lp;
    g.b_plane = r.n_b;
    gemm_lowp(g, p->delta_prec, s, st.tile_lp[p->delta_prec]);
    g.A = r.ref_a_lp;
    g.B = r.dshadow_b;
    gemm_lowp(g, p->delta_prec, s, st.tile_lp[p->delta_prec]);
    return;
  }
  if (p->delta_mode == 2) {
    copy_f64(r.ref_op, X, w * r.n_op, s);
    GemmDesc g = d;
    g.C = r.ref_out;
    g.ldc = d.N;
    g.beta = 0.0;
    if (p->cplx) gemm_c128(g, s, st.tile_z);
    else gemm_f64(g, s, st.tile);
    add_product(C, w * d.ldc, d.beta, r.ref_out, d.M, w * d.N, s);
    return;
  }
  if (p->cplx) {
    // (X - X_ref) as the realified operand of its side; the constant operand's
    // copy of the other side was made by plan_prepare
    CC_REQUIRE(r.var ? (p->shadow[con_slot] && p->shadow_prec[con_slot] == p->delta_prec)
                     : (st.bform >= 0 && p->bforms[st.bform].ptr && p->bforms[st.bform].prec == p->delta_prec),
               CC_EINTERNAL, "constant operand copy not prepared");
    if (r.var) realify_complex(p->delta_prec, 1, X, r.ref_op, r.n_op / d.K, d.K, d.K, 1, r.dshadow, s);
    else convert_delta(p->delta_prec, X, r.ref_op, 2 * r.n_op, r.dshadow, s);
    add_product(C, 2 * d.ldc, d.beta, r.ref_out, d.M, 2 * d.N, s);
    GemmDesc g = realified_desc(d, r.var ? p->shadow[con_slot] : r.dshadow,
                                r.var ? r.dshadow : p->bforms[st.bform].ptr);
    g.a_plane = 2 * slot_elems(p, st.a);
    g.b_plane = 4 * slot_elems(p, st.b);
    g.beta = 1.0;
    gemm_lowp(g, p->delta_prec, s, st.tile_lp[p->delta_prec]);
    return;
  }
  // split bf16 with blocked copies (prepared by an earlier split-bf16 run)
  // and an LDS-direct configuration: (X - X_ref) blocked as well
  const int con_blk = r.var ? st.blk_a : st.blk_b;
  const int tile = st.tile_lp[p->delta_prec];
  if (p->delta_prec == PREC_BF16X3 && r.dblk && con_blk >= 0 && st.blk_use != 0 && p->bforms[con_blk].ptr &&
      p->bforms[con_blk].prec == PREC_BF16X3 &&
      gemm_lowp_tile_blocked(PREC_BF16X3, tile >= 0 ? tile : gemm_lowp_pick(PREC_BF16X3, d.M, d.N))) {
    const BForm &cf = p->bforms[con_blk];
    const int64_t rows = r.n_op / d.K;
    convert_blocked(X, r.ref_op, rows, d.K, r.dblk, s);
    add_product(C, d.ldc, d.beta, r.ref_out, d.M, d.N, s);
    GemmDesc g = d;
    const int64_t vplane = blocked_plane(rows, d.K), cplane = blocked_plane(slot_elems(p, cf.slot) / cf.K, cf.K);
    if (r.var) {
      g.A = cf.ptr;
      g.a_plane = cplane;
      g.B = r.dblk;
      g.b_plane = vplane;
    } else {
      g.A = r.dblk;
      g.a_plane = vplane;
      g.B = cf.ptr;
      g.b_plane = cplane;
    }
    g.lp_in = 2;
    g.beta = 1.0;
    gemm_lowp(g, PREC_BF16X3, s, tile);
    return;
  }
  CC_REQUIRE(p->shadow.size() == p->slots.size() && p->shadow[con_slot] &&
                 p->shadow_prec[con_slot] == p->delta_prec,
             CC_EINTERNAL, "constant operand copy not prepared");
  convert_delta(p->delta_prec, X, r.ref_op, r.n_op, r.dshadow, s);
  add_product(C, d.ldc, d.beta, r.ref_out, d.M, d.N, s);
  GemmDesc g = d;
  if (r.var) {
    g.B = r.dshadow;
    g.b_plane = r.n_op;
    g.A = p->shadow[con_slot];
    g.a_plane = slot_elems(p, con_slot);
  } else {
    g.A = r.dshadow;
    g.a_plane = r.n_op;
    g.B = p->shadow[con_slot];
    g.b_plane = slot_elems(p, con_slot);
  }
  g.lp_in = 1;
  g.beta = 1.0;
  gemm_lowp(g, p->delta_prec, s, st.tile_lp[p->delta_prec]);
}

}  // namespace

// Reduced-precision runs read each GEMM operand from a 4-byte-per-element
// copy (FP32, or bf16 hi plane followed by bf16 lo plane) made by one
// conversion pass: constant operands once per precision, the others once per
// write.  Allocation and the constant conversions happen here, outside any
// graph capture.
// Complex slots: the interleaved copy (2 reals per element) serves the A
// side; the B side reads the realified copy (4 reals per element).
void plan_prepare(cc_plan *p) {
  const bool lowp = p->cur_prec != PREC_F64;
  const bool delta = !lowp && p->delta_mode != 0 && !p->deltas.empty();
  if (!lowp && !delta) return;
  const int prec = lowp ? p->cur_prec : p->delta_prec;
  const size_t n = p->slots.size();
  const int64_t w = p->cplx ? 2 : 1;  // reals per element
  if (p->shadow.size() != n) {
    p->shadow.assign(n, nullptr);
    p->shadow_prec.assign(n, -1);
    p->shadow_ok.assign(n, 0);
  }
  hipStream_t s = p->ctx->stream;
  for (const Step &st : p->iter) {
    if (st.kind != Step::GEMM || (!lowp && st.delta < 0) || (lowp && !st.lowp_ok)) continue;
    for (int side = 0; side < 2; ++side) {
      const int sl = side ? st.b : st.a;
      if (!lowp && !p->slots[sl].constant) continue;  // the correction reads its own copy
      if (lowp && prec == PREC_BF16X3 && (side ? st.blk_b : st.blk_a) >= 0) {
        BForm &bf = p->bforms[side ? st.blk_b : st.blk_a];
        if (!bf.ptr) {
          // the padding rows are never written: zero once (outside any capture)
          const size_t bytes = size_t(blocked_bytes(p, bf));
          CC_HIP_CHECK(hipMalloc(&bf.ptr, bytes));
          CC_HIP_CHECK(hipMemsetAsync(bf.ptr, 0, bytes, s));
          bf.prec = -1;
        }
        if (p->slots[sl].constant && bf.prec != prec) {
          convert_blocked_form(p, bf, s);
          bf.prec = prec;
        }
      }
      if (p->cplx && side == 1) {
        CC_REQUIRE(st.bform >= 0, CC_EINTERNAL, "complex B operand copy not planned");
        BForm &bf = p->bforms[st.bform];
        if (!bf.ptr) {
          CC_HIP_CHECK(hipMalloc(&bf.ptr, size_t(slot_elems(p, sl)) * 16));
          bf.prec = -1;
        }
        if (p->slots[sl].constant && bf.prec != prec) {
          convert_b_form(p, bf, prec, s);
          bf.prec = prec;
        }
        continue;
      }
      if (!p->shadow[sl]) {
        CC_HIP_CHECK(hipMalloc(&p->shadow[sl], size_t(slot_elems(p, sl)) * w * 4));
        p->shadow_prec[sl] = -1;
      }
      if (p->slots[sl].constant && p->shadow_prec[sl] != prec) {
        convert_shadow(prec, static_cast<const double *>(ptr_of(p, sl)), w * slot_elems(p, sl), p->shadow[sl], s);
        p->shadow_prec[sl] = prec;
      }
    }
  }
  if (delta) {
    for (DeltaRef &d : p->deltas) {
      if (d.var == 2 && prec != PREC_BF16X3) continue;  // such products stay plain FP64
      const GemmDesc &g = p->iter[d.step].gemm;
      const int64_t wd = p->cplx ? (d.var ? 4 : 2) : 1;  // reals per element of the varying operand's copy
      if (!d.ref_op) CC_HIP_CHECK(hipMalloc(reinterpret_cast<void **>(&d.ref_op), size_t(d.n_op) * w * 8));
      if (!d.ref_out) CC_HIP_CHECK(hipMalloc(reinterpret_cast<void **>(&d.ref_out), size_t(g.M) * g.N * w * 8));
      if (!d.dshadow) CC_HIP_CHECK(hipMalloc(&d.dshadow, size_t(d.n_op) * wd * 4));
      const Step &ds = p->iter[d.step];
      if (d.var == 2) {
        if (!d.ref_b) CC_HIP_CHECK(hipMalloc(reinterpret_cast<void **>(&d.ref_b), size_t(d.n_b) * 8));
        if (!d.ref_a_lp) CC_HIP_CHECK(hipMalloc(&d.ref_a_lp, size_t(d.n_op) * 4));
        if (!d.cur_b_lp) CC_HIP_CHECK(hipMalloc(&d.cur_b_lp, size_t(d.n_b) * 4));
        if (!d.dshadow_b) CC_HIP_CHECK(hipMalloc(&d.dshadow_b, size_t(d.n_b) * 4));
        continue;
      }
      if (!p->cplx && prec == PREC_BF16X3 && ds.blk_a >= 0 && ds.blk_b >= 0 && !d.dblk)
        CC_HIP_CHECK(hipMalloc(&d.dblk, size_t(blocked_plane(d.n_op / g.K, g.K)) * 4));
    }
  }
}

TauEntry tau_entry(cc_plan *p) {
  const bool ccsd = p->method == CC_CCSD;
  return make_tau_entry(p->o, p->v, ccsd ? p->t1 : nullptr, p->t2, p->slots[p->index["oovv"]].ptr,
                        p->slots[p->index["fov"]].ptr, ccsd ? p->slots[p->index["tau"]].ptr : nullptr,
                        ccsd ? p->slots[p->index["taut"]].ptr : nullptr, p->epart);
}

AsmEntry asm_entry(cc_plan *p) {
  R2Args a{p->o, p->v, p->d_oo, p->d_vv, p->shift, p->dressed, p->slots[p->index["GG"]].ptr,
           p->slots[p->index["FF"]].ptr};
  return make_asm_entry(a, p->slots[p->index["XP"]].ptr, p->slots[p->index["Xij"]].ptr,
                        p->slots[p->index["Xab"]].ptr, p->slots[p->index["Xr"]].ptr, p->r2_out,
                        p->update ? p->t2 : nullptr, p->n2part);
}

R1Entry r1_entry(cc_plan *p) {
  return R1Entry{p->o, p->v, p->slots[p->index["R1"]].ptr, p->update ? p->t1 : nullptr, p->d_oo, p->d_vv,
                 p->shift, p->dressed, p->slots[p->index["Fmi"]].ptr, p->slots[p->index["Fae"]].ptr,
                 p->n1part};
}

FinEntry fin_entry(cc_plan *p) {
  FinEntry f{p->epart, p->n_epart, p->n2part, p->n_n2part,
             p->method == CC_CCSD ? p->n1part : nullptr, p->scalars};
  if (p->triples) {
    f.n3part = p->n3part;
    f.nn3 = p->n_n3part;
  }
  return f;
}

T3Entry t3_entry(cc_plan *p) {
  return T3Entry{p->o, p->v, p->slots[p->index["Y3"]].ptr, p->r3_out, p->update ? p->t3 : nullptr,
                 p->d_oo, p->d_vv, p->shift, p->n3part, t3_units(p->o, p->v)};
}

namespace {

void exec(cc_plan *p, Step &st, hipStream_t s) {
  const bool cplx = p->cplx;
  invalidate(p, st.c);
  if (st.kind == Step::TAU_E && p->method == CC_CCSD) {
    invalidate(p, p->index["tau"]);
    invalidate(p, p->index["taut"]);
  }
  switch (st.kind) {
    case Step::PERMUTE:
      if (cplx) permute_c128(st.perm, ptr_of(p, st.a), ptr_of(p, st.c), s);
      else permute_f64(st.perm, ptr_of(p, st.a), ptr_of(p, st.c), s);
      break;
    case Step::GEMM: {
      GemmDesc d = st.gemm;
      d.A = ptr_of(p, st.a);
      d.B = ptr_of(p, st.b);
      d.C = ptr_of(p, st.c);
      d.ws = st.b2 >= 0 ? ptr_of(p, st.b2) : nullptr;
      d.ws_elems = st.b2 >= 0 ? p->slots[st.b2].elems : 0;
      if (st.delta >= 0 && p->delta_mode != 0 && p->cur_prec == PREC_F64) run_delta_gemm(p, d, st, s);
      else run_gemm(p, d, st, s);
      break;
    }
    case Step::OUTER:
      outer_acc(st.outer, cplx, ptr_of(p, st.a), ptr_of(p, st.b), ptr_of(p, st.c), s);
      break;
    case Step::FILL:
      fill_zero(ptr_of(p, st.c), st.nelem, cplx, s);
      break;
    case Step::TAU_E:
      launch_tau(tau_entry(p), cplx, s);
      break;
    case Step::ASSEMBLE:
      launch_asm(asm_entry(p), cplx, s);
      break;
    case Step::R1UPD: {
      void *R1 = p->slots[p->index["R1"]].ptr;
      if (p->r1_out)
        CC_HIP_CHECK(hipMemcpyAsync(p->r1_out, R1, size_t(p->o) * p->v * p->esize,
                                    hipMemcpyDeviceToDevice, s));
      launch_r1(r1_entry(p), cplx, s);
      break;
    }
    case Step::FINALIZE:
      launch_fin(fin_entry(p), s);
      break;
    case Step::PAIR:
      launch_pair(make_pair_entry(ptr_of(p, st.a), ptr_of(p, st.c), p->pair_tab[st.pair_rows],
                                  p->pair_tab[st.pair_cols], st.pair_np, st.pair_nq, st.pair_ldq, st.pair_n[0],
                                  st.pair_n[1], st.pair_n[2], st.pair_mode),
                  cplx, s);
      break;
    case Step::TRIPLES:
      CC_REQUIRE(p->t3 != nullptr, CC_EINVAL, "triples amplitudes not bound (cc_plan_set_triples)");
      launch_t3(t3_entry(p), cplx, s);
      break;
  }
}

}  // namespace

OpList parse_op_list(const char *text) {
  if (!text) throw CCError(CC_EINVAL, "op list is NULL");
  OpList out;
  std::istringstream in(text);
  std::string line;
  int lineno = 0;
  auto bad = [&](const std::string &why) {
    throw CCError(CC_EINVAL, "op list line " + std::to_string(lineno) + ": " + why);
  };
  while (std::getline(in, line)) {
    ++lineno;
    const size_t hash = line.find('#');
    if (hash != std::string::npos) line.resize(hash);
    std::istringstream ls(line);
    std::vector<std::string> tok;
    for (std::string t; ls >> t;) tok.push_back(t);
    if (tok.empty()) continue;
    if (tok[0] == "work") {
      if (tok.size() != 3) bad("expected: work NAME SPACES");
      out.work.emplace_back(tok[1], tok[2]);
    } else if (tok[0] == "op") {
      if (tok.size() < 9) bad("expected: op TAG C cl ALPHA A al B bl [flags]");
      OpText o;
      o.tag = tok[1];
      o.C = tok[2];
      o.cl = tok[3];
      char *end = nullptr;
      o.alpha = std::strtod(tok[4].c_str(), &end);
      if (!end || *end != '\0') bad("bad coefficient " + tok[4]);
      o.A = tok[5];
      o.al = tok[6];
      if (tok[7] != "-") {
        o.B = tok[7];
        o.bl = tok[8];
      }
      for (size_t q = 9; q < tok.size(); ++q) {
        if (tok[q] == "conjA") o.conjA = true;
        else if (tok[q] == "conjB") o.conjB = true;
        else if (tok[q].rfind("swap=", 0) == 0 && tok[q].size() == 7) o.swap = tok[q].substr(5);
        else if (tok[q] != "-") bad("unknown flag " + tok[q]);
      }
      out.ops.push_back(o);
    } else {
      bad("unknown keyword " + tok[0]);
    }
  }
  if (out.ops.empty()) throw CCError(CC_EINVAL, "op list has no ops");
  return out;
}

void plan_layout(cc_plan *p, const cc_system *sys) {
  Planner pl{p};
  pl.build(sys);
}

void plan_build(cc_plan *p, const cc_system *sys) {
  plan_layout(p, sys);
  // allocate owned slots
  for (Slot &s : p->slots) {
    if (!s.owned) continue;
    const size_t bytes = size_t(std::max<int64_t>(s.elems, 1)) * p->esize;
    s.ptr = dev_alloc(bytes);
    p->workspace += bytes;
  }
  p->n_epart = int(tau_units(p->o, p->v));
  p->n_n2part = int(asm_units(p->o, p->v));
  p->d_oo = static_cast<double *>(dev_alloc(sizeof(double) * p->o));
  p->d_vv = static_cast<double *>(dev_alloc(sizeof(double) * p->v));
  p->epart = static_cast<double *>(dev_alloc(sizeof(double) * 2 * p->n_epart));
  p->n2part = static_cast<double *>(dev_alloc(sizeof(double) * p->n_n2part));
  p->n1part = static_cast<double *>(dev_alloc(sizeof(double) * 2));
  if (p->triples) {
    p->n_n3part = int(t3_units(p->o, p->v));
    p->n3part = static_cast<double *>(dev_alloc(sizeof(double) * p->n_n3part));
  }
  p->scalars = static_cast<double *>(dev_alloc(sizeof(double) * 4));
  hipStream_t s = p->ctx->stream;
  fock_diag(p->cplx, p->o, p->v, sys->f_oo, sys->f_vv, p->d_oo, p->d_vv, s);
  fill_zero(p->n1part, 2, false, s);
  if (p->packed) {
    auto upload = [&](std::vector<int> h, int **dst) {
      if (h.empty()) h.assign(2, 0);
      *dst = static_cast<int *>(dev_alloc(sizeof(int) * h.size()));
      CC_HIP_CHECK(hipMemcpyAsync(*dst, h.data(), sizeof(int) * h.size(), hipMemcpyHostToDevice, s));
      CC_HIP_CHECK(hipStreamSynchronize(s));
    };
    auto pairs = [](int n) {
      std::vector<int> h;
      for (int x = 0; x < n; ++x)
        for (int y = x + 1; y < n; ++y) {
          h.push_back(x);
          h.push_back(y);
        }
      return h;
    };
    std::vector<int> ma, am;
    for (int m = 0; m < p->o; ++m)
      for (int a = 0; a < p->v; ++a) {
        ma.push_back(m);
        ma.push_back(a);
        am.push_back(a);
        am.push_back(m);
      }
    upload(pairs(p->o), &p->pair_tab[0]);
    upload(pairs(p->v), &p->pair_tab[1]);
    upload(ma, &p->pair_tab[2]);
    upload(am, &p->pair_tab[3]);
  }
  for (Step &st : p->setup) exec(p, st, s);
  CC_HIP_CHECK(hipStreamSynchronize(s));
  for (Step &st : p->iter)
    if (st.kind == Step::GEMM) p->gemm_steps.push_back(&st);
  // Reduced precision pays for the contractions that carry the work; the
  // ones under 1% of the iteration's flops are bandwidth- or latency-bound
  // and run in FP64 (measured faster, and exact), unless the plan asks for
  // every contraction in its precision (CC_PLAN_LOWP_ALL, batched plans).
  // Complex contractions run in reduced precision as real GEMMs on realified
  // operands, which needs both operands in dense K-contiguous rows.
  auto shape_ok = [p](const Step &st) {
    const GemmDesc &g = st.gemm;
    return !p->cplx || (g.K > 0 && g.sak == 1 && g.sbk == 1 && g.sam == g.K && g.sbn == g.K &&
                        slot_elems(p, st.b) % g.K == 0);
  };
  for (Step &st : p->iter)
    if (st.kind == Step::GEMM) st.lowp_ok = (p->lowp_all || st.flops >= 0.01 * p->flops_per_iter) && shape_ok(st);
  // contractions worth a reference + correction evaluation (at least 1% of
  // the iteration's work): linear in the amplitudes (one constant operand),
  // and, for real systems, products of two varying operands, corrected as
  // A B = A_ref B_ref + (A - A_ref) B + A_ref (B - B_ref)
  {
    for (size_t k = 0; k < p->iter.size(); ++k) {
      Step &st = p->iter[k];
      if (st.kind != Step::GEMM || st.flops < 0.01 * p->flops_per_iter || !shape_ok(st)) continue;
      const bool ca = p->slots[st.a].constant, cb = p->slots[st.b].constant;
      if (ca && cb) continue;
      if (!ca && !cb && p->cplx) continue;
      DeltaRef d;
      d.step = int(k);
      d.var = (!ca && !cb) ? 2 : ca ? 1 : 0;
      d.n_op = slot_elems(p, ca ? st.b : st.a);
      if (d.var == 2) d.n_b = slot_elems(p, st.b);
      st.delta = int(p->deltas.size());
      p->deltas.push_back(d);
    }
  }
  // complex: one realified copy per (B slot, row length K) of those GEMMs
  if (p->cplx)
    for (Step &st : p->iter) {
      if (st.kind != Step::GEMM || (!st.lowp_ok && st.delta < 0)) continue;
      int idx = -1;
      for (size_t i = 0; i < p->bforms.size(); ++i)
        if (p->bforms[i].kind == 0 && p->bforms[i].slot == st.b && p->bforms[i].K == st.gemm.K) idx = int(i);
      if (idx < 0) {
        BForm bf;
        bf.slot = st.b;
        bf.K = st.gemm.K;
        p->bforms.push_back(bf);
        idx = int(p->bforms.size()) - 1;
      }
      st.bform = idx;
    }
  // real split bf16: the large contractions on dense K-contiguous rows (K a
  // multiple of 32) also get copies of both operands in the 16 x 32 blocks
  // the LDS-direct kernels load whole (one per slot and row length K);
  // batched plans run grouped launches on FP64 operands instead
  // (complex: of the realified A' and B', rows of 2K, so K a multiple of 16)
  if (!p->lowp_all)
    for (Step &st : p->iter) {
      const GemmDesc &g = st.gemm;
      const int64_t rk = p->cplx ? 2 * g.K : g.K, rn = p->cplx ? 2 * g.N : g.N;
      if (st.kind != Step::GEMM || !st.lowp_ok || g.K <= 0 || rk % 32 != 0 || g.sak != 1 || g.sbk != 1 ||
          g.sam != g.K || g.sbn != g.K || g.M < 256 || rn < 128 || slot_elems(p, st.a) % g.K != 0 ||
          slot_elems(p, st.b) % g.K != 0)
        continue;
      auto form = [p](int kind, int slot, int64_t K) {
        for (size_t i = 0; i < p->bforms.size(); ++i)
          if (p->bforms[i].kind == kind && p->bforms[i].slot == slot && p->bforms[i].K == K) return int(i);
        BForm bf;
        bf.kind = kind;
        bf.slot = slot;
        bf.K = K;
        p->bforms.push_back(bf);
        return int(p->bforms.size()) - 1;
      };
      st.blk_a = form(p->cplx ? 2 : 1, st.a, g.K);
      st.blk_b = form(p->cplx ? 3 : 1, st.b, g.K);
    }
}

void plan_free(cc_plan *p) {
  for (hipEvent_t e : p->events) (void)hipEventDestroy(e);
  p->events.clear();
  if (p->graph) (void)hipGraphExecDestroy(p->graph);
  p->graph = nullptr;
  for (Slot &s : p->slots)
    if (s.owned && s.ptr) (void)hipFree(s.ptr);
  for (void *q : p->shadow)
    if (q) (void)hipFree(q);
  p->shadow.clear();
  for (BForm &bf : p->bforms)
    if (bf.ptr) (void)hipFree(bf.ptr);
  p->bforms.clear();
  for (DeltaRef &d : p->deltas) {
    for (void *q : {static_cast<void *>(d.ref_op), static_cast<void *>(d.ref_out), d.dshadow, d.dblk,
                    static_cast<void *>(d.ref_b), d.ref_a_lp, d.cur_b_lp, d.dshadow_b})
      if (q) (void)hipFree(q);
    d.ref_op = d.ref_out = d.ref_b = nullptr;
    d.dshadow = d.dblk = d.ref_a_lp = d.cur_b_lp = d.dshadow_b = nullptr;
  }
  for (double *q : {p->d_oo, p->d_vv, p->epart, p->n2part, p->n1part, p->scalars, p->n3part})
    if (q) (void)hipFree(q);
  for (int *q : p->pair_tab)
    if (q) (void)hipFree(q);
}

void plan_run(cc_plan *p) {
  hipStream_t s = p->ctx->stream;
  {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    CC_HIP_CHECK(hipStreamIsCapturing(s, &cs));
    if (cs == hipStreamCaptureStatusNone) plan_prepare(p);
  }
  if (p->cur_prec != PREC_F64) {
    CC_REQUIRE(p->shadow.size() == p->slots.size(), CC_EINTERNAL, "operand copies not prepared");
    for (size_t i = 0; i < p->slots.size(); ++i)
      p->shadow_ok[i] = p->slots[i].constant && p->shadow_prec[i] == p->cur_prec;
    for (BForm &bf : p->bforms) bf.ok = p->slots[bf.slot].constant && bf.prec == p->cur_prec;
  }
  if (p->delta_mode == 2 && p->cur_prec == PREC_F64 && !p->deltas.empty()) {
    // this run stores the reference; the following ones correct it
    for (Step &st : p->iter) exec(p, st, s);
    p->delta_mode = 1;
    return;
  }
  if (!p->profiling) {
    for (Step &st : p->iter) exec(p, st, s);
    return;
  }
  const size_t n = p->iter.size();
  if (p->events.size() != n + 1) {
    for (hipEvent_t e : p->events) (void)hipEventDestroy(e);
    p->events.assign(n + 1, nullptr);
    for (auto &e : p->events) CC_HIP_CHECK(hipEventCreate(&e));
    p->step_ms.assign(n, 0.0);
    p->step_calls.assign(n, 0);
  }
  CC_HIP_CHECK(hipEventRecord(p->events[0], s));
  for (size_t i = 0; i < n; ++i) {
    exec(p, p->iter[i], s);
    CC_HIP_CHECK(hipEventRecord(p->events[i + 1], s));
  }
  CC_HIP_CHECK(hipEventSynchronize(p->events[n]));
  for (size_t i = 0; i < n; ++i) {
    float ms = 0.f;
    CC_HIP_CHECK(hipEventElapsedTime(&ms, p->events[i], p->events[i + 1]));
    p->step_ms[i] += ms;
    p->step_calls[i] += 1;
  }
}

// Time every tile configuration for each distinct GEMM shape of the
// iteration (on the plan's own buffers) and keep the fastest.  Results are
// cached per (M, N, K, layouts) for the life of the process; with
// CC_AUTOTUNE_CACHE naming a file they are also read from it (lines "key
// tile", at the first autotune of the process) and appended to it, so that
// another process (a profiler pass, say) takes the same choices.
void plan_autotune(cc_plan *p, int reps) {
  // shared by every context of the process (contexts may live on different
  // host threads): lookups and inserts are serialised
  static std::map<std::string, int> cache;
  static std::mutex cache_mutex;
  static bool file_read = false;
  const char *cache_file = std::getenv("CC_AUTOTUNE_CACHE");
  if (cache_file && *cache_file) {
    std::lock_guard<std::mutex> lk(cache_mutex);
    if (!file_read) {
      file_read = true;
      std::ifstream in(cache_file);
      std::string k;
      int t;
      while (in >> k >> t) cache.emplace(k, t);
    }
  }
  const int prec_plan = p->cplx ? 9 : p->cur_prec;  // 9: complex128 tiles
  plan_prepare(p);
  hipStream_t s = p->ctx->stream;
  hipEvent_t e0, e1;
  CC_HIP_CHECK(hipEventCreate(&e0));
  CC_HIP_CHECK(hipEventCreate(&e1));
  try {
    for (Step *st : p->gemm_steps) {
      GemmDesc d = st->gemm;
      const bool akc = d.sak == 1, bkc = d.sbk == 1;
      // this step's precision: contractions under 1% of the work run in FP64;
      // complex ones in reduced precision are real GEMMs of M x 2N x 2K
      const bool lowp = p->cur_prec != PREC_F64 && st->lowp_ok;
      const int prec = lowp ? p->cur_prec : prec_plan == 9 ? 9 : PREC_F64;
      const bool cz = prec == 9;
      const int ntiles = cz ? gemm_c128_num_tiles()
                            : (prec == PREC_F64 ? gemm_f64_num_tiles() : gemm_lowp_num_tiles(prec));
      const int64_t rN = (p->cplx && lowp) ? 2 * d.N : d.N, rK = (p->cplx && lowp) ? 2 * d.K : d.K;
      // blocked split-bf16 copies available: the LDS-direct configurations
      // are timed on them (a choice of its own in the cache)
      const bool blk = lowp && prec == PREC_BF16X3 && st->blk_a >= 0 && st->blk_b >= 0 &&
                       p->bforms[st->blk_a].ptr && p->bforms[st->blk_b].ptr;
      const std::string key = std::to_string(prec) + ":" + std::to_string(d.M) + "x" +
                              std::to_string(rN) + "x" + std::to_string(rK) + (akc ? "k" : "m") +
                              (bkc ? "k" : "n") + (blk ? "b" : "");
      int &slot = cz ? st->tile_z : (prec == PREC_F64 ? st->tile : st->tile_lp[prec]);
      std::unique_lock<std::mutex> lk(cache_mutex);
      auto it = cache.find(key);
      // cached value: the tile, plus kBlockedChoice when it runs on the blocked copies
      constexpr int kBlockedChoice = 1000;
      if (it != cache.end()) {
        slot = it->second % kBlockedChoice;
        if (blk) st->blk_use = it->second >= kBlockedChoice ? 1 : 0;
        continue;
      }
      lk.unlock();
      d.A = ptr_of(p, st->a);
      d.B = ptr_of(p, st->b);
      d.C = ptr_of(p, st->c);
      d.ws = st->b2 >= 0 ? ptr_of(p, st->b2) : nullptr;
      d.ws_elems = st->b2 >= 0 ? p->slots[st->b2].elems : 0;
      GemmDesc db = d;
      if (lowp && p->cplx) use_shadows_c(p, d, *st, s, false);
      else if (lowp) use_shadows(p, d, *st, s, false);
      if (blk) use_blocked(p, db, *st, s, false);
      int best = slot, best_blk = 0;
      float best_ms = 1e30f;
      auto launch = [&](int t, int b) {
        if (cz) gemm_c128(d, s, t);
        else if (prec == PREC_F64) gemm_f64(d, s, t);
        else gemm_lowp(b ? db : d, prec, s, t);
      };
      // every configuration on the row-major copies, and the LDS-direct
      // ones also on the blocked copies
      for (int t = 0; t < ntiles; ++t)
        for (int b = 0; b < ((blk && gemm_lowp_tile_blocked(prec, t)) ? 2 : 1); ++b) {
          launch(t, b);
          CC_HIP_CHECK(hipEventRecord(e0, s));
          for (int r = 0; r < reps; ++r) launch(t, b);
          CC_HIP_CHECK(hipEventRecord(e1, s));
          CC_HIP_CHECK(hipEventSynchronize(e1));
          float ms = 0.f;
          CC_HIP_CHECK(hipEventElapsedTime(&ms, e0, e1));
          if (ms < best_ms) {
            best_ms = ms;
            best = t;
            best_blk = b;
          }
        }
      slot = best;
      if (blk) st->blk_use = best_blk;
      const int value = best + (best_blk ? kBlockedChoice : 0);
      lk.lock();
      cache[key] = value;
      if (cache_file && *cache_file) {
        std::ofstream out(cache_file, std::ios::app);
        out << key << " " << value << "\n";
      }
    }
  } catch (...) {
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    throw;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (p->graph) (void)hipGraphExecDestroy(p->graph);
  p->graph = nullptr;
}

std::string plan_profile_table(const cc_plan *p) {
  std::ostringstream os;
  os << "# step kind tag calls total_ms avg_ms flops_per_call\n";
  for (size_t i = 0; i < p->step_ms.size() && i < p->iter.size(); ++i) {
    const Step &st = p->iter[i];
    static const char *kinds[] = {"PERMUTE", "GEMM", "OUTER", "FILL", "TAU_E", "ASSEMBLE", "R1UPD", "FINALIZE", "TRIPLES", "PAIR"};
    std::string tag = st.tag.empty() ? "-" : st.tag;
    for (auto &c : tag)
      if (c == ' ') c = '_';
    if (st.kind == Step::GEMM) {
      tag += "@" + std::string((p->cur_prec != PREC_F64 && st.lowp_ok) ? gemm_lowp_tile_name(p->cur_prec, st.tile_lp[p->cur_prec])
                               : p->cplx                                  ? gemm_c128_tile_name(st.tile_z)
                                                                          : gemm_f64_tile_name(st.tile));
      if (st.lowp_ok && blocked_for(p, st, st.tile_lp[PREC_BF16X3])) tag += "/blk";  // blocked copies
    }
    os << i << " " << kinds[st.kind] << " " << tag << " " << p->step_calls[i]
       << " " << p->step_ms[i] << " " << (p->step_calls[i] ? p->step_ms[i] / p->step_calls[i] : 0.0)
       << " " << st.flops << "\n";
  }
  return os.str();
}

void plan_run_energy(cc_plan *p) {
  hipStream_t s = p->ctx->stream;
  for (Step &st : p->iter)
    if (st.kind == Step::TAU_E) exec(p, st, s);
  launch_fin(FinEntry{p->epart, p->n_epart, p->n2part, 0, nullptr, p->scalars}, s);
}

std::string plan_describe(const cc_plan *p) {
  std::ostringstream os;
  os.precision(17);  // coefficients round-trip exactly
  auto nm = [&](int s) { return s >= 0 ? p->slots[s].name : std::string("-"); };
  auto dump = [&](const char *title, const std::vector<Step> &v) {
    os << title << "\n";
    for (const Step &st : v) {
      switch (st.kind) {
        case Step::PERMUTE:
          os << "PERMUTE " << st.tag << " alpha=" << st.perm.alpha << " beta=" << st.perm.beta
             << " conj=" << st.perm.conj << " in_strides=";
          for (int d = 0; d < st.perm.rank; ++d) os << st.perm.in_strides[d] << (d + 1 < st.perm.rank ? "," : "");
          os << " out_dims=";
          for (int d = 0; d < st.perm.rank; ++d) os << st.perm.out_dims[d] << (d + 1 < st.perm.rank ? "," : "");
          os << " out_strides=";
          for (int d = 0; d < st.perm.rank; ++d) os << st.perm.out_strides[d] << (d + 1 < st.perm.rank ? "," : "");
          os << " src=" << nm(st.a) << " dst=" << nm(st.c) << "\n";
          break;
        case Step::GEMM:
          os << "GEMM " << st.tag << " A=" << nm(st.a) << " B=" << nm(st.b) << " C=" << nm(st.c)
             << " M=" << st.gemm.M << " N=" << st.gemm.N << " K=" << st.gemm.K << " sam=" << st.gemm.sam
             << " sak=" << st.gemm.sak << " sbn=" << st.gemm.sbn << " sbk=" << st.gemm.sbk
             << " ldc=" << st.gemm.ldc << " alpha=" << st.gemm.alpha << " beta=" << st.gemm.beta
             << " split=" << st.gemm.split
             << " tile=" << (st.tile >= 0 ? gemm_f64_tile_name(st.tile) : "auto") << "\n";
          break;
        case Step::OUTER:
          os << "OUTER " << st.tag << " A=" << nm(st.a) << " B=" << nm(st.b) << " C=" << nm(st.c)
             << " alpha=" << st.outer.alpha << " sa=";
          for (int d = 0; d < st.outer.rank; ++d) os << st.outer.sa[d] << (d + 1 < st.outer.rank ? "," : "");
          os << " sb=";
          for (int d = 0; d < st.outer.rank; ++d) os << st.outer.sb[d] << (d + 1 < st.outer.rank ? "," : "");
          os << " dims=";
          for (int d = 0; d < st.outer.rank; ++d) os << st.outer.dims[d] << (d + 1 < st.outer.rank ? "," : "");
          os << " conj=" << st.outer.conj_a << st.outer.conj_b << "\n";
          break;
        case Step::FILL: os << "FILL " << nm(st.c) << "\n"; break;
        default: os << "SPECIAL " << st.tag << "\n"; break;
      }
    }
  };
  dump("# setup", p->setup);
  dump("# iteration", p->iter);
  os << "# aliases\n";
  for (const auto &kv : p->index)
    if (p->slots[kv.second].name != kv.first) os << kv.first << " -> " << p->slots[kv.second].name << "\n";
  os << "# slots\n";
  for (const Slot &s : p->slots) {
    os << s.name << " dims=";
    for (size_t i = 0; i < s.dims.size(); ++i) os << s.dims[i] << (i + 1 < s.dims.size() ? "," : "");
    os << (s.constant ? " const" : "") << (s.external ? " external" : "") << "\n";
  }
  return os.str();
}

}  // namespace ccmi
