// planner.cpp - structural plan and device program of the density-matrix contraction.
//
// For every partition of a maximally unbalanced path (section 4.2 of the paper,
// partitioned_contract on a linear path) the planner
//   1. orders the new leaves and embeds the union of the old boundary MPS and the
//      partition's tensors into the positions of an MPS tree (the appendix on
//      embedding trees, MPS tree definition), inserting identity matrices where a
//      leaf's owner sits elsewhere (section 6.2),
//   2. emits the memoised right environments R_k (Eq. dm_cache), then the forward
//      sweep of Algorithm density_matrix_alg: L = C R_k C^T, kept eigenvectors U,
//      C <- U^T C merged with the next group, with power-of-two rescaling.
// Every pairwise contraction becomes one GEMM over two-level index tables, so any
// mode permutation is folded into the operand gathers. Workspace buffers are
// assigned by a liveness scan over the op list.
#include "planner.hpp"

#include <algorithm>
#include <cmath>
#include <limits>
#include <map>
#include <queue>
#include <sstream>
#include <unordered_map>
#include <unordered_set>

namespace tn {

std::string build_graph(const int64_t *const *dims, const int32_t *orders, int32_t nt,
                        const int32_t *e4, int32_t ne, Graph &g) {
  if (nt < 1) return "network has no tensors";
  if (ne < 0) return "negative edge count";
  g = Graph();
  g.nt = nt;
  g.dims.resize(nt);
  g.const_off.resize(nt);
  int64_t off = 0;
  for (int32_t t = 0; t < nt; ++t) {
    if (orders[t] < 0 || orders[t] > 24) return "tensor order out of range [0, 24]";
    int64_t size = 1;
    for (int32_t m = 0; m < orders[t]; ++m) {
      int64_t d = dims[t][m];
      if (d < 1) return "tensor dimension < 1";
      if (d > (int64_t(1) << 30) || size > (int64_t(1) << 40) / d) return "tensor too large";
      g.dims[t].push_back(d);
      size *= d;
    }
    g.const_off[t] = off;
    off += (size + 3) & ~int64_t(3);
  }
  g.const_size = off;
  std::vector<std::vector<int32_t>> used(nt);
  for (int32_t t = 0; t < nt; ++t) used[t].assign(orders[t], -1);
  g.e_t0.resize(ne); g.e_m0.resize(ne); g.e_t1.resize(ne); g.e_m1.resize(ne);
  for (int32_t e = 0; e < ne; ++e) {
    int32_t t0 = e4[4 * e], m0 = e4[4 * e + 1], t1 = e4[4 * e + 2], m1 = e4[4 * e + 3];
    if (t0 < 0 || t0 >= nt || t1 < 0 || t1 >= nt) return "edge references a missing tensor";
    if (t0 == t1) return "self-loop edge";
    if (m0 < 0 || m0 >= orders[t0] || m1 < 0 || m1 >= orders[t1]) return "edge references a missing mode";
    if (used[t0][m0] >= 0 || used[t1][m1] >= 0) return "mode referenced twice";
    if (g.dims[t0][m0] != g.dims[t1][m1]) return "dimensions disagree across an edge";
    used[t0][m0] = e;
    used[t1][m1] = e;
    g.e_t0[e] = t0; g.e_m0[e] = m0; g.e_t1[e] = t1; g.e_m1[e] = m1;
  }
  for (int32_t t = 0; t < nt; ++t)
    for (int32_t m = 0; m < orders[t]; ++m)
      if (used[t][m] < 0) return "dangling mode (only closed networks are supported)";
  g.inc.assign(nt, {});
  for (int32_t e = 0; e < ne; ++e) {
    g.inc[g.e_t0[e]].push_back({e, g.e_m0[e], g.e_t1[e]});
    g.inc[g.e_t1[e]].push_back({e, g.e_m1[e], g.e_t0[e]});
  }
  return "";
}

namespace {

constexpr int64_t kInf = std::numeric_limits<int64_t>::max() / 4;
constexpr int64_t kAlign = 32;        // doubles (256 bytes)
constexpr int64_t kLoMax = 4096;      // inner part of a two-level index map

struct Sym {                  // a tensor known by its labelled modes
  std::vector<int64_t> lab, dim;
  int32_t buf = -1;           // virtual workspace buffer; -1 = constant area
  int64_t cst = 0;            // constant-area offset when buf < 0
  // storage as a [rows][cols] matrix with runtime extents (set for GEMM outputs)
  Box rows{0, 1, {0}, {0}}, cols{0, 1, {0}, {0}};
  int64_t ncols = 1;
  int64_t size() const {
    int64_t s = 1;
    for (int64_t d : dim) s *= d;
    return s;
  }
  int find(int64_t l) const {
    for (size_t i = 0; i < lab.size(); ++i)
      if (lab[i] == l) return int(i);
    return -1;
  }
};

enum UnitKind { U_MPS = 0, U_SITE = 1, U_ID = 2 };

struct Unit {
  Sym t;
  int kind;
  int64_t ref;     // mps: own old position; site: vertex; id: position
  int64_t order;   // tie-break order within a group
  int64_t sweep[3];  // closing-sweep key: (old position or anchor, kind, path index)
};

struct MpsTensor {
  Sym t;
  int64_t own;     // position of its own leaf (1-based)
};

class Builder {
 public:
  Builder(const Graph &g, Plan &p, int32_t chi) : g_(g), p_(p), chi_(chi) {
    next_label_ = int64_t(g.e_t0.size());
  }

  int64_t fresh() { return next_label_++; }

  // MPS bonds have a runtime extent (the kept rank) held in a per-network slot.
  int32_t new_dyn(int64_t label) {
    int32_t d = n_dyn_++;
    dynl_[label] = d;
    return d;
  }
  void share_dyn(int64_t label, int64_t copy) {
    auto it = dynl_.find(label);
    if (it != dynl_.end()) dynl_[copy] = it->second;
  }
  int32_t dyn_of(int64_t label) const {
    auto it = dynl_.find(label);
    return it == dynl_.end() ? -1 : it->second;
  }
  int32_t n_dyn() const { return n_dyn_; }
  std::string err;
  int32_t gemm_flags = 0;     // flags given to every GEMM emitted (F_ENV while environments
                              // and density matrices are built)

  struct Group {
    std::vector<int64_t> lab, dim, sa, sb;   // labels, static dims, strides in A (and B)
    std::vector<int32_t> dyn;
  };
  // bond modes first (stable), so the valid region of the group is a Box
  static void dyn_first(Group &g) {
    std::vector<size_t> idx(g.lab.size());
    for (size_t i = 0; i < idx.size(); ++i) idx[i] = i;
    std::stable_sort(idx.begin(), idx.end(), [&](size_t x, size_t y) { return (g.dyn[x] >= 0) > (g.dyn[y] >= 0); });
    Group o;
    for (size_t i : idx) {
      o.lab.push_back(g.lab[i]); o.dim.push_back(g.dim[i]); o.dyn.push_back(g.dyn[i]);
      if (!g.sa.empty()) o.sa.push_back(g.sa[i]);
      if (!g.sb.empty()) o.sb.push_back(g.sb[i]);
    }
    g = o;
  }
  Box box_of(const Group &g) {
    Box b{};
    int64_t rest = 1;
    for (size_t i = 0; i < g.lab.size(); ++i) {
      if (g.dyn[i] >= 0) {
        if (b.nd >= kMaxDyn) { err = "more than 8 bond modes in one index group"; continue; }
        b.id[b.nd] = g.dyn[i];
        b.cap[b.nd] = int32_t(g.dim[i]);
        b.nd++;
      } else rest *= g.dim[i];
    }
    b.rest = int32_t(rest);
    p_.max_dyn_modes = std::max<int32_t>(p_.max_dyn_modes, b.nd);
    return b;
  }

  int32_t new_buf(int64_t size) {
    vb_.push_back({size, -1, -1});
    return int32_t(vb_.size() - 1);
  }

  // ---------------------------------------------------------------- tables
  int32_t table(const std::vector<int64_t> &dims, const std::vector<int64_t> &strides) {
    std::vector<int32_t> t(1, 0);
    for (size_t i = 0; i < dims.size(); ++i) {
      std::vector<int32_t> nx;
      nx.reserve(t.size() * dims[i]);
      for (int32_t base : t)
        for (int64_t j = 0; j < dims[i]; ++j) nx.push_back(int32_t(base + j * strides[i]));
      t.swap(nx);
    }
    auto it = cache_.find(t);
    if (it != cache_.end()) return it->second;
    int32_t off = int32_t(p_.tables.size());
    p_.tables.insert(p_.tables.end(), t.begin(), t.end());
    cache_.emplace(std::move(t), off);
    return off;
  }

  IdxMap make_map(const std::vector<int64_t> &dims, const std::vector<int64_t> &strides) {
    IdxMap m{};
    size_t r = dims.size();
    size_t split = r;          // modes [split, r) form the inner part
    int64_t inner = 1;
    while (split > 0 && inner * dims[split - 1] <= kLoMax) {
      inner *= dims[split - 1];
      --split;
    }
    if (split == r && r > 0) {  // last mode alone exceeds kLoMax
      split = r - 1;
      inner = dims[r - 1];
    }
    std::vector<int64_t> od(dims.begin(), dims.begin() + split), os(strides.begin(), strides.begin() + split);
    std::vector<int64_t> id(dims.begin() + split, dims.end()), is(strides.begin() + split, strides.end());
    m.hi = table(od, os);
    m.lo = table(id, is);
    m.lo_n = int32_t(inner);
    int64_t n = 1;
    for (int64_t d : dims) n *= d;
    m.n = int32_t(n);
    return m;
  }

  static std::vector<int64_t> strides_of(const Sym &s) {
    std::vector<int64_t> st(s.dim.size(), 1);
    for (int i = int(s.dim.size()) - 2; i >= 0; --i) st[i] = st[i + 1] * s.dim[i + 1];
    return st;
  }

  // ---------------------------------------------------------------- ops
  void bind(int32_t op, int field, const Sym &s) {
    if (s.buf >= 0) {
      refs_.push_back({op, field, s.buf});
      vb_[s.buf].last = std::max(vb_[s.buf].last, op);
      if (vb_[s.buf].def < 0) vb_[s.buf].def = op;
    } else {
      Op &o = p_.ops[op];
      if (field == 1) { o.a = s.cst; o.flags |= F_A_CONST; }
      else if (field == 2) { o.b = s.cst; o.flags |= F_B_CONST; }
    }
  }
  void def(int32_t op, int32_t buf) {
    refs_.push_back({op, 0, buf});
    if (vb_[buf].def < 0) vb_[buf].def = op;
    vb_[buf].last = std::max(vb_[buf].last, op);
  }
  int32_t emit(const Op &o) {
    p_.ops.push_back(o);
    return int32_t(p_.ops.size() - 1);
  }

  // Element count of a shape, saturated at k32 (no int64 overflow for long shapes).
  static constexpr int64_t k32 = int64_t(1) << 31;
  static int64_t sat_size(const std::vector<int64_t> &dim) {
    int64_t s = 1;
    for (int64_t d : dim) {
      if (s >= k32 / d + 1) return k32;
      s *= d;
    }
    return s;
  }

  // Pairwise contraction over all shared labels; A's free modes come first. Within
  // each index group (A-free, shared, B-free) bond modes are placed first.
  // Index maps, table entries and an op's row, column and contraction extents are
  // int32 on the device, so a contraction whose operands, result or contraction
  // extent reach 2^31 elements is refused (the plan fails as unsupported).
  Sym contract_ab(const Sym &A, const Sym &B) {
    {
      std::vector<int64_t> od, kd;
      for (size_t i = 0; i < A.lab.size(); ++i) (B.find(A.lab[i]) >= 0 ? kd : od).push_back(A.dim[i]);
      for (size_t i = 0; i < B.lab.size(); ++i)
        if (A.find(B.lab[i]) < 0) od.push_back(B.dim[i]);
      if (sat_size(A.dim) >= k32 || sat_size(B.dim) >= k32 || sat_size(od) >= k32 || sat_size(kd) >= k32) {
        if (err.empty()) err = "a contraction operand or result reaches 2^31 elements";
        Sym out;                 // a placeholder with the result's labels; no op is emitted
        for (size_t i = 0; i < A.lab.size(); ++i)
          if (B.find(A.lab[i]) < 0) { out.lab.push_back(A.lab[i]); out.dim.push_back(1); }
        for (size_t i = 0; i < B.lab.size(); ++i)
          if (A.find(B.lab[i]) < 0) { out.lab.push_back(B.lab[i]); out.dim.push_back(1); }
        out.buf = new_buf(1);
        return out;
      }
    }
    Group ga, gk, gb;
    auto sa = strides_of(A), sb = strides_of(B);
    for (size_t i = 0; i < A.lab.size(); ++i) {
      int j = B.find(A.lab[i]);
      if (j >= 0) {
        gk.lab.push_back(A.lab[i]); gk.dim.push_back(A.dim[i]); gk.sa.push_back(sa[i]); gk.sb.push_back(sb[j]);
        gk.dyn.push_back(dyn_of(A.lab[i]));
      } else {
        ga.lab.push_back(A.lab[i]); ga.dim.push_back(A.dim[i]); ga.sa.push_back(sa[i]); ga.dyn.push_back(dyn_of(A.lab[i]));
      }
    }
    for (size_t i = 0; i < B.lab.size(); ++i)
      if (A.find(B.lab[i]) < 0) {
        gb.lab.push_back(B.lab[i]); gb.dim.push_back(B.dim[i]); gb.sa.push_back(sb[i]); gb.dyn.push_back(dyn_of(B.lab[i]));
      }
    dyn_first(ga);
    dyn_first(gk);
    dyn_first(gb);
    Sym out;
    out.lab = ga.lab; out.lab.insert(out.lab.end(), gb.lab.begin(), gb.lab.end());
    out.dim = ga.dim; out.dim.insert(out.dim.end(), gb.dim.begin(), gb.dim.end());
    out.buf = new_buf(out.size());
    Op o{};
    o.kind = OP_GEMM;
    o.flags = gemm_flags;
    o.am = make_map(ga.dim, ga.sa);
    o.bn = make_map(gb.dim, gb.sa);
    int64_t K = 1;
    for (int64_t d : gk.dim) K *= d;
    o.K = int32_t(K);
    o.ak = table(gk.dim, gk.sa);
    o.bk = table(gk.dim, gk.sb);
    o.bm = box_of(ga);
    o.bnb = box_of(gb);
    o.bk_ = box_of(gk);
    if (!gk.sa.empty() && gk.sa.back() == 1) o.flags |= F_A_KFAST;
    if (gb.sa.empty() || gb.sa.back() == 1) o.flags |= F_B_NFAST;
    out.rows = o.bm;
    out.cols = o.bnb;
    out.ncols = o.bn.n;
    int32_t id = emit(o);
    bind(id, 1, A);
    bind(id, 2, B);
    def(id, out.buf);
    p_.flops += 2 * int64_t(o.am.n) * int64_t(o.bn.n) * K;
    return out;
  }

  // Smaller operand as A so the larger one is read along its free (row-major) modes.
  Sym contract(const Sym &x, const Sym &y) {
    if (y.size() < x.size()) return contract_ab(y, x);
    return contract_ab(x, y);
  }

  static double log_result(const Sym &a, const Sym &b) {
    double s = 0;
    for (size_t i = 0; i < a.lab.size(); ++i)
      if (b.find(a.lab[i]) < 0) s += std::log(double(a.dim[i]));
    for (size_t i = 0; i < b.lab.size(); ++i)
      if (a.find(b.lab[i]) < 0) s += std::log(double(b.dim[i]));
    return s;
  }

  // Running-intermediate contraction: always absorb the tensor giving the smallest result.
  Sym absorb(const Sym *start, std::vector<Sym> units) {
    Sym cur;
    size_t first = 0;
    if (start) cur = *start;
    else { cur = units[0]; first = 1; }
    std::vector<bool> done(units.size(), false);
    for (size_t i = 0; i < first; ++i) done[i] = true;
    for (size_t step = first; step < units.size(); ++step) {
      size_t best = SIZE_MAX;
      double bv = 0;
      for (size_t i = 0; i < units.size(); ++i) {
        if (done[i]) continue;
        double v = log_result(cur, units[i]);
        if (best == SIZE_MAX || v < bv - 1e-9) { best = i; bv = v; }
      }
      done[best] = true;
      cur = contract(cur, units[best]);
    }
    if (start == nullptr && units.size() == 1 && cur.buf < 0) {
      // a lone constant tensor: copy it into the workspace through a 1x1 identity GEMM
      Sym one;
      one.buf = new_buf(1);
      Op o{};
      o.kind = OP_IDENT;
      o.count = 1;
      int32_t id = emit(o);
      def(id, one.buf);
      cur = contract_ab(one, cur);
    }
    return cur;
  }

  void rescale(const Sym &s, bool accum) {
    Op o{};
    o.kind = OP_RESCALE;
    o.count = s.ncols;
    o.bm = s.rows;
    o.bnb = s.cols;
    if (accum) o.flags |= F_ACCUM;
    int32_t id = emit(o);
    refs_.push_back({id, 0, s.buf});
    vb_[s.buf].last = std::max(vb_[s.buf].last, id);
  }

  Sym ident(int64_t d, int64_t l0, int64_t l1) {
    if (d >= 46341 && err.empty()) err = "an identity of more than 2^31 elements";
    Sym s;
    s.lab = {l0, l1};
    s.dim = {d, d};
    s.buf = new_buf(d * d);
    s.rows.rest = int32_t(d * d);
    Op o{};
    o.kind = OP_IDENT;
    o.count = d;
    int32_t id = emit(o);
    def(id, s.buf);
    return s;
  }

  // Kept leading eigenvectors of L (rows = its first nrow modes, bond modes first).
  // U is stored [bond][rows] so that the new bond is the outermost mode.
  Sym eig(const Sym &L, size_t nrow, int64_t ucols, int64_t bond, int32_t flags = 0) {
    int64_t n = 1;
    for (size_t i = 0; i < nrow; ++i) n *= L.dim[i];
    Sym U;
    U.lab.push_back(bond);
    U.dim.push_back(ucols);
    for (size_t i = 0; i < nrow; ++i) { U.lab.push_back(L.lab[i]); U.dim.push_back(L.dim[i]); }
    U.buf = new_buf(n * ucols);
    int32_t slot = new_dyn(bond);
    Op o{};
    o.kind = OP_EIG;
    o.count = n;
    o.K = int32_t(ucols);
    o.bm = L.rows;
    o.out_dyn = slot;
    U.rows = Box{1, 1, {slot}, {int32_t(ucols)}};
    U.cols = L.rows;
    U.ncols = n;
    // scratch: reflectors (n^2 + n), then the matrix and Z of a solve too large for LDS, or the
    // second eigenvector buffer and the merge matrices of a divide-and-conquer solve
    o.flags |= F_V_GLOBAL | flags;
    int32_t scratch = new_buf(3 * (n * n + n));
    int32_t id = emit(o);
    refs_.push_back({id, 1, L.buf});
    vb_[L.buf].last = std::max(vb_[L.buf].last, id);
    if (scratch >= 0) { refs_.push_back({id, 2, scratch}); vb_[scratch].def = id; vb_[scratch].last = id; }
    def(id, U.buf);
    p_.n_eig += 1;
    p_.eig_flops += 9 * n * n * n;
    p_.max_eig_dim = std::max<int32_t>(p_.max_eig_dim, int32_t(n));
    return U;
  }

  // QR factorisation of C viewed as a matrix with the modes `row_labels` as rows and the
  // others as columns (the QR-SVD branch of Algorithm density_matrix_alg): Q with labels
  // (q, rows) stored [q][rows], R with labels (q, cols) stored [q][cols]; q is a new bond
  // whose runtime extent min(rows, cols) the op writes to its slot.
  std::pair<Sym, Sym> qr(const Sym &C, const std::vector<int64_t> &row_labels, int64_t q) {
    Group gr, gc;
    auto sc = strides_of(C);
    for (size_t i = 0; i < C.lab.size(); ++i) {
      Group &g = std::find(row_labels.begin(), row_labels.end(), C.lab[i]) != row_labels.end() ? gr : gc;
      g.lab.push_back(C.lab[i]); g.dim.push_back(C.dim[i]); g.sa.push_back(sc[i]); g.dyn.push_back(dyn_of(C.lab[i]));
    }
    dyn_first(gr);
    dyn_first(gc);
    int64_t nr = 1, nc = 1;
    for (int64_t d : gr.dim) nr *= d;
    for (int64_t d : gc.dim) nc *= d;
    const int64_t cap = std::min(nr, nc);
    const int32_t slot = new_dyn(q);
    Op o{};
    o.kind = OP_QR;
    o.am = make_map(gr.dim, gr.sa);
    o.bn = make_map(gc.dim, gc.sa);
    o.bm = box_of(gr);
    o.bnb = box_of(gc);
    o.K = int32_t(cap);
    o.count = nr;
    o.out_dyn = slot;
    Sym Q, R;
    Q.lab.push_back(q); Q.dim.push_back(cap);
    Q.lab.insert(Q.lab.end(), gr.lab.begin(), gr.lab.end()); Q.dim.insert(Q.dim.end(), gr.dim.begin(), gr.dim.end());
    R.lab.push_back(q); R.dim.push_back(cap);
    R.lab.insert(R.lab.end(), gc.lab.begin(), gc.lab.end()); R.dim.insert(R.dim.end(), gc.dim.begin(), gc.dim.end());
    Q.buf = new_buf(cap * nr);
    R.buf = new_buf(cap * nc);
    Q.rows = R.rows = Box{1, 1, {slot}, {int32_t(cap)}};
    Q.cols = o.bm;
    R.cols = o.bnb;
    Q.ncols = nr;
    R.ncols = nc;
    const int32_t id = emit(o);
    bind(id, 1, C);
    def(id, Q.buf);
    refs_.push_back({id, 2, R.buf});
    if (vb_[R.buf].def < 0) vb_[R.buf].def = id;
    vb_[R.buf].last = std::max(vb_[R.buf].last, id);
    p_.eig_flops += 4 * nr * nc * cap;
    p_.n_qr += 1;
    return {Q, R};
  }

  // ---------------------------------------------------------------- memory
  void allocate() {
    std::vector<int32_t> order(vb_.size());
    for (size_t i = 0; i < order.size(); ++i) order[i] = int32_t(i);
    for (auto &b : vb_) {
      if (b.def < 0) b.def = 0;
      if (b.last < b.def) b.last = b.def;
    }
    std::stable_sort(order.begin(), order.end(), [&](int32_t x, int32_t y) { return vb_[x].def < vb_[y].def; });
    std::map<int64_t, int64_t> freel;   // offset -> size
    using Act = std::pair<int32_t, int32_t>;  // (last use, buffer)
    std::priority_queue<Act, std::vector<Act>, std::greater<Act>> active;
    std::vector<int64_t> off(vb_.size(), 0);
    const int64_t dyn_doubles = ((int64_t(n_dyn_) + 1) / 2 + kAlign - 1) / kAlign * kAlign;
    p_.dyn_off = 0;
    p_.n_dyn = n_dyn_;
    int64_t top = dyn_doubles;
    auto release = [&](int32_t b) {
      int64_t o = off[b], s = (vb_[b].size + kAlign - 1) / kAlign * kAlign;
      auto it = freel.emplace(o, s).first;
      auto nx = std::next(it);
      if (nx != freel.end() && it->first + it->second == nx->first) { it->second += nx->second; freel.erase(nx); }
      if (it != freel.begin()) {
        auto pv = std::prev(it);
        if (pv->first + pv->second == it->first) { pv->second += it->second; freel.erase(it); }
      }
    };
    for (int32_t b : order) {
      while (!active.empty() && active.top().first < vb_[b].def) { release(active.top().second); active.pop(); }
      int64_t need = (vb_[b].size + kAlign - 1) / kAlign * kAlign;
      auto best = freel.end();
      for (auto it = freel.begin(); it != freel.end(); ++it)
        if (it->second >= need) { best = it; break; }
      if (best != freel.end()) {
        off[b] = best->first;
        int64_t o = best->first, s = best->second;
        freel.erase(best);
        if (s > need) freel.emplace(o + need, s - need);
      } else {
        // grow: merge with a free block that ends at top
        if (!freel.empty()) {
          auto last = std::prev(freel.end());
          if (last->first + last->second == top) { top = last->first; freel.erase(last); }
        }
        off[b] = top;
        top += need;
      }
      active.push({vb_[b].last, b});
    }
    p_.ws_size = top;
    for (const Ref &r : refs_) {
      Op &o = p_.ops[r.op];
      if (r.field == 0) o.c = off[r.buf];
      else if (r.field == 1) o.a = off[r.buf];
      else o.b = off[r.buf];
    }
  }

  static constexpr int64_t kLdsDoubles = 20000;

  const Graph &g_;
  Plan &p_;
  int32_t chi_;
  int64_t next_label_;

 private:
  struct VB { int64_t size; int32_t def, last; };
  struct Ref { int32_t op; int field; int32_t buf; };
  std::vector<VB> vb_;
  std::vector<Ref> refs_;
  std::map<std::vector<int32_t>, int32_t> cache_;
  std::unordered_map<int64_t, int32_t> dynl_;
  int32_t n_dyn_ = 0;
};

struct Key {            // sort key of a new leaf
  int64_t anchor, kind, pt, po, e;
  bool operator<(const Key &o) const {
    if (anchor != o.anchor) return anchor < o.anchor;
    if (kind != o.kind) return kind < o.kind;
    if (pt != o.pt) return pt < o.pt;
    if (po != o.po) return po < o.po;
    return e < o.e;
  }
};

// Everything of a partition step contracted at once, in a sweep along the old leaf
// positions; a greedy order could leave a whole row of bonds open at the same time.
Sym absorb_closing(Builder &B, const std::vector<Unit> &units) {
  std::vector<size_t> idx(units.size());
  for (size_t i = 0; i < idx.size(); ++i) idx[i] = i;
  std::stable_sort(idx.begin(), idx.end(), [&](size_t x, size_t y) {
    const int64_t *a = units[x].sweep, *b = units[y].sweep;
    if (a[0] != b[0]) return a[0] < b[0];
    if (a[1] != b[1]) return a[1] < b[1];
    return a[2] < b[2];
  });
  if (idx.size() == 1) return B.absorb(nullptr, {units[idx[0]].t});
  Sym cur = units[idx[0]].t;
  for (size_t i = 1; i < idx.size(); ++i) cur = B.contract(cur, units[idx[i]].t);
  return cur;
}

}  // namespace

std::string make_plan(const Graph &g, const PlanArgs &a, Plan &out, bool *unsupported) {
  *unsupported = false;
  out = Plan();
  if (a.chi < 1) return "max_rank must be >= 1";
  if (a.env < 1) return "env_size must be >= 1";
  const int32_t nt = g.nt;
  std::vector<int64_t> pidx(nt, -1);
  int64_t cnt = 0;
  for (const auto &s : a.slices)
    for (int32_t v : s) {
      if (v < 0 || v >= nt) return "path references a missing tensor";
      if (pidx[v] >= 0) return "path lists a tensor twice";
      pidx[v] = cnt++;
    }
  if (cnt != nt) return "path does not cover every tensor";

  Builder B(g, out, a.chi);
  std::vector<char> absorbed(nt, 0);
  std::vector<MpsTensor> mps;
  std::vector<int32_t> leaves;          // old leaf edges in order
  std::ostringstream js;
  js << "{\"partitions\":[";
  size_t nslices = a.slices.size();
  int jpart = 0;
  for (size_t s0 = 0; s0 < nslices; s0 += a.env, ++jpart) {
    std::vector<int32_t> part;
    for (size_t s = s0; s < std::min(nslices, s0 + a.env); ++s)
      part.insert(part.end(), a.slices[s].begin(), a.slices[s].end());
    std::vector<char> inP(nt, 0);
    for (int32_t v : part) inP[v] = 1;
    std::vector<int32_t> order_p = part;
    std::sort(order_p.begin(), order_p.end(), [&](int32_t x, int32_t y) { return pidx[x] < pidx[y]; });

    auto far_end = [&](int32_t e) { return absorbed[g.e_t0[e]] ? g.e_t1[e] : g.e_t0[e]; };

    // old leaves: contracted into P or surviving
    std::vector<std::pair<int64_t, int32_t>> contracted, surviving;   // (position, edge)
    for (size_t p = 0; p < leaves.size(); ++p) {
      if (inP[far_end(leaves[p])]) contracted.push_back({int64_t(p + 1), leaves[p]});
      else surviving.push_back({int64_t(p + 1), leaves[p]});
    }
    // anchors
    std::unordered_map<int32_t, int64_t> anchor, direct;
    for (int32_t t : order_p) {
      int64_t best = -1;
      for (auto &ce : contracted)
        if (far_end(ce.second) == t && (best < 0 || ce.first < best)) best = ce.first;
      anchor[t] = best;
      direct[t] = best;
    }
    for (int32_t t : order_p) {
      if (anchor[t] >= 0) continue;
      int32_t bu = -1;
      for (auto &ic : g.inc[t]) {
        int32_t u = ic.other;
        if (!inP[u] || anchor[u] < 0) continue;
        if (bu < 0 || pidx[u] < pidx[bu]) bu = u;
      }
      if (bu >= 0) anchor[t] = anchor[bu];
    }
    for (int32_t t : order_p)
      if (anchor[t] < 0) anchor[t] = kInf;

    // new leaves, sorted by key
    std::vector<std::pair<Key, int32_t>> keyed;
    for (auto &se : surviving) keyed.push_back({Key{se.first, 0, 0, 0, 0}, se.second});
    for (int32_t t : order_p)
      for (auto &ic : g.inc[t])
        if (!absorbed[ic.other] && !inP[ic.other])
          keyed.push_back({Key{anchor[t], 1, pidx[t], pidx[ic.other], ic.e}, ic.e});
    std::sort(keyed.begin(), keyed.end(), [](const auto &x, const auto &y) { return x.first < y.first; });
    const int64_t n = int64_t(keyed.size());
    std::vector<int32_t> leaf(n);
    std::unordered_map<int32_t, int64_t> pos_of_edge;
    for (int64_t i = 0; i < n; ++i) { leaf[i] = keyed[i].second; pos_of_edge[leaf[i]] = i + 1; }
    auto first_pos_at_or_after = [&](int64_t av) -> int64_t {
      for (int64_t i = 0; i < n; ++i)
        if (keyed[i].first.anchor >= av) return i + 1;
      return n;
    };

    // union network
    std::vector<Unit> units;
    for (auto &m : mps) units.push_back({m.t, U_MPS, m.own, 0, {m.own, 0, 0}});
    std::unordered_map<int32_t, size_t> site_unit;
    for (int32_t t : order_p) {
      Sym s;
      s.lab.assign(g.dims[t].size(), -1);
      s.dim = g.dims[t];
      for (auto &ic : g.inc[t]) s.lab[ic.m] = ic.e;
      s.buf = -1;
      s.cst = g.const_off[t];
      site_unit[t] = units.size();
      units.push_back({s, U_SITE, t, 1 + pidx[t], {anchor[t], 1, pidx[t]}});
    }

    js << (jpart ? "," : "") << "{\"leaves\":[";
    for (int64_t i = 0; i < n; ++i) js << (i ? "," : "") << leaf[i];
    js << "],\"placement\":[";

    static const char *kname[3] = {"mps", "site", "id"};
    if (n == 0) {
      for (size_t i = 0; i < units.size(); ++i)
        js << (i ? "," : "") << "[\"" << kname[units[i].kind] << "\"," << units[i].ref << ",0]";
      js << "]}";
      {
        Sym z = absorb_closing(B, units);
        Op o{};
        o.kind = OP_SCALAR;
        int32_t id = B.emit(o);
        B.bind(id, 1, z);   // records the use; offset patched into .a
      }
      mps.clear();
      leaves.clear();
      for (int32_t v : part) absorbed[v] = 1;
      continue;
    }

    // embedding
    std::vector<int64_t> pos(units.size(), -1);
    for (size_t i = 0; i < units.size(); ++i) {
      Unit &u = units[i];
      if (u.kind == U_MPS) {
        int32_t own_edge = leaves[u.ref - 1];
        auto it = pos_of_edge.find(own_edge);
        pos[i] = it != pos_of_edge.end() ? it->second : first_pos_at_or_after(u.ref);
      } else {
        int64_t best = -1;
        for (int64_t l : u.t.lab) {
          auto it = pos_of_edge.find(int32_t(l));
          if (l < int64_t(g.e_t0.size()) && it != pos_of_edge.end() && (best < 0 || it->second < best)) best = it->second;
        }
        if (best >= 0) pos[i] = best;
        else if (direct[int32_t(u.ref)] >= 0) pos[i] = first_pos_at_or_after(direct[int32_t(u.ref)]);
      }
    }
    while (true) {   // leafless, anchorless tensors follow a neighbour placed in an earlier pass
      std::vector<int64_t> prev = pos;
      for (int32_t t : order_p) {
        size_t i = site_unit[t];
        if (prev[i] >= 0) continue;
        int32_t bu = -1;
        for (auto &ic : g.inc[t]) {
          int32_t u = ic.other;
          if (!inP[u] || prev[site_unit[u]] < 0) continue;
          if (bu < 0 || pidx[u] < pidx[bu]) bu = u;
        }
        if (bu >= 0) pos[i] = prev[site_unit[bu]];
      }
      if (pos == prev) break;
    }
    for (auto &p : pos)
      if (p < 0) p = n;

    // identity insertion: the leaf of position k must live in group k
    for (int64_t k = 1; k <= n; ++k) {
      int64_t l = leaf[k - 1];
      size_t owner = SIZE_MAX;
      for (size_t i = 0; i < units.size() && owner == SIZE_MAX; ++i)
        if (units[i].t.find(l) >= 0) owner = i;
      if (pos[owner] != k) {
        int64_t s = B.fresh();
        Sym &ot = units[owner].t;
        int64_t d = ot.dim[ot.find(l)];
        ot.lab[ot.find(l)] = s;
        Sym id = B.ident(d, s, l);
        units.push_back({id, U_ID, k, (int64_t(1) << 40) + k, {kInf, 2, k}});
        pos.push_back(k);
      }
    }
    for (size_t i = 0; i < units.size(); ++i)
      js << (i ? "," : "") << "[\"" << kname[units[i].kind] << "\"," << units[i].ref << "," << pos[i] << "]";
    js << "]}";

    std::vector<std::vector<size_t>> groups(n + 1);
    for (size_t i = 0; i < units.size(); ++i) groups[pos[i]].push_back(i);
    for (auto &gp : groups)
      std::stable_sort(gp.begin(), gp.end(), [&](size_t x, size_t y) { return units[x].order < units[y].order; });
    auto gsyms = [&](int64_t k) {
      std::vector<Sym> v;
      for (size_t i : groups[k]) v.push_back(units[i].t);
      return v;
    };

    if (n <= 2) {
      Sym root = absorb_closing(B, units);
      B.rescale(root, true);
      mps.clear();
      mps.push_back({root, 1});
      leaves = leaf;
      for (int32_t v : part) absorbed[v] = 1;
      continue;
    }

    // crossing sets X_k
    std::unordered_map<int64_t, std::pair<int64_t, int64_t>> span;   // label -> (min pos, max pos)
    std::unordered_map<int64_t, int> seen;
    std::unordered_map<int64_t, int64_t> ldim;
    for (size_t i = 0; i < units.size(); ++i)
      for (size_t m = 0; m < units[i].t.lab.size(); ++m) {
        int64_t l = units[i].t.lab[m];
        ldim[l] = units[i].t.dim[m];
        auto it = span.find(l);
        if (it == span.end()) span[l] = {pos[i], pos[i]};
        else { it->second.first = std::min(it->second.first, pos[i]); it->second.second = std::max(it->second.second, pos[i]); }
        seen[l] += 1;
      }
    std::vector<std::vector<int64_t>> X(n + 1);
    std::vector<int64_t> labs_sorted;
    for (auto &kv : seen)
      if (kv.second == 2) labs_sorted.push_back(kv.first);
    std::sort(labs_sorted.begin(), labs_sorted.end());
    for (int64_t l : labs_sorted)
      for (int64_t k = span[l].first; k < span[l].second; ++k) X[k].push_back(l);
    auto xdim = [&](int64_t k) {
      int64_t d = 1;
      for (int64_t l : X[k]) d *= ldim[l];
      return d;
    };

    std::unordered_map<int64_t, int64_t> bra;
    auto bra_of = [&](int64_t l) {
      auto it = bra.find(l);
      if (it != bra.end()) return it->second;
      int64_t b = B.fresh();
      bra[l] = b;
      B.share_dyn(l, b);
      return b;
    };
    auto check_labels = [&](const Sym &s, std::vector<int64_t> want) -> bool {
      std::vector<int64_t> have = s.lab;
      std::sort(have.begin(), have.end());
      std::sort(want.begin(), want.end());
      return have == want;
    };

    // right environments R_k, k = n-1 .. 2
    std::vector<Sym> R(n + 1);
    B.gemm_flags = F_ENV;
    for (int64_t k = n - 1; k >= 2; --k) {
      int64_t lf = leaf[k];          // leaf of position k+1
      std::vector<Sym> ket = gsyms(k + 1), all = ket;
      for (const Sym &s : ket) {
        Sym b = s;
        for (auto &l : b.lab)
          if (l != lf) l = bra_of(l);
        all.push_back(b);
      }
      Sym r = B.absorb(k + 1 <= n - 1 ? &R[k + 1] : nullptr, all);
      std::vector<int64_t> want = X[k];
      for (int64_t l : X[k]) want.push_back(bra_of(l));
      if (!check_labels(r, want)) return "internal planner error: right environment modes";
      B.rescale(r, false);
      R[k] = r;
    }
    B.gemm_flags = 0;

    // forward sweep
    std::vector<Sym> g12 = gsyms(1), g2 = gsyms(2);
    g12.insert(g12.end(), g2.begin(), g2.end());
    Sym C = B.absorb(nullptr, g12);
    {
      std::vector<int64_t> want = X[2];
      want.push_back(leaf[0]);
      want.push_back(leaf[1]);
      if (!check_labels(C, want)) return "internal planner error: first block modes";
    }
    B.rescale(C, true);
    std::vector<int64_t> rows = {leaf[0], leaf[1]};
    std::vector<MpsTensor> next;
    for (int64_t k = 2; k <= n - 1; ++k) {
      int64_t nr = 1;
      for (size_t i = 0; i < C.lab.size(); ++i)
        if (std::find(rows.begin(), rows.end(), C.lab[i]) != rows.end()) nr *= C.dim[i];
      if (nr > kMaxEigDim) {
        *unsupported = true;
        return "density matrix of dimension " + std::to_string(nr) + " exceeds the supported " +
               std::to_string(kMaxEigDim);
      }
      int64_t ucols = std::min<int64_t>({int64_t(a.chi), nr, xdim(k)});
      int64_t bond = B.fresh();
      Sym U;
      if (nr > xdim(k) && nr <= kQrMaxRows && xdim(k) <= kQrMaxCols) {
        // QR-SVD branch (the open size exceeds the crossing size): C = Q Rc, the
        // leading eigenvectors of Rc R_k Rc^T, mapped back through Q
        const int64_t q = B.fresh(), qb = B.fresh();
        auto qr = B.qr(C, rows, q);
        B.share_dyn(q, qb);
        B.gemm_flags = F_ENV;
        Sym T = B.contract_ab(qr.second, R[k]);  // q x bra(X_k)
        Sym Rb = qr.second;
        for (auto &l : Rb.lab) l = (l == q) ? qb : bra_of(l);
        Sym M = B.contract_ab(T, Rb);            // q x qb
        B.gemm_flags = 0;
        Sym Uh = B.eig(M, 1, ucols, bond, F_NO_WARM);
        U = B.contract_ab(Uh, qr.first);         // bond x rows
      } else {
        B.gemm_flags = F_ENV;
        Sym T = B.contract_ab(C, R[k]);          // rows x bra(X_k)
        Sym Cb = C;
        for (auto &l : Cb.lab) l = bra_of(l);    // C with every mode primed
        Sym L = B.contract_ab(T, Cb);            // rows x bra(rows)
        B.gemm_flags = 0;
        U = B.eig(L, rows.size(), ucols, bond);
      }
      Sym Cn = B.contract_ab(U, C);              // bond x X_k
      Cn = B.absorb(&Cn, gsyms(k + 1));
      std::vector<int64_t> want = k + 1 <= n - 1 ? X[k + 1] : std::vector<int64_t>();
      want.push_back(bond);
      want.push_back(leaf[k]);
      if (!check_labels(Cn, want)) return "internal planner error: carried block modes";
      B.rescale(Cn, true);
      next.push_back({U, k == 2 ? 1 : k});
      C = Cn;
      rows = {bond, leaf[k]};
    }
    next.push_back({C, n});
    mps = next;
    leaves = leaf;
    for (int32_t v : part) absorbed[v] = 1;
  }
  js << "],\"max_dyn_modes\":" << out.max_dyn_modes << ",\"n_eig\":" << out.n_eig << "}";
  out.plan_json = js.str();
  if (!B.err.empty()) { *unsupported = true; return B.err; }
  B.allocate();
  return "";
}

}  // namespace tn
