// FIND plan construction (host only).
//
// Trees and sets follow the paper's Sec. 2.1-2.2: the mesh is split by
// alternating bisection into basic clusters; each basic cluster C has a
// boundary set B_C (nodes of C adjacent to the outside) and each complement
// cluster C-bar = M \ C has the boundary set B_{C-bar} (nodes outside C
// adjacent to C).  Adjacency is the sparsity pattern of A: the 5- or 9-point
// stencil plus the dense contact blocks on the first and last columns (the
// pattern of Sigma< is contained in it).
//
// Every elimination is recorded as an ordered node list [S ; B] with, for
// each entry, where its rows/columns of the assembled matrix come from:
//   * upward merge of children i, j  (procedure updateBoundaryNodes):
//       list B_i ++ B_j, blocks (B_i,B_i) = U_i, (B_j,B_j) = U_j, cross blocks
//       from the original A; S = (B_i u B_j) \ B_k, B = B_k;
//   * upward leaf: A(C,C) from the original matrix, S = C \ B_C, B = B_C;
//   * downward step for C with parent D, sibling D1 (procedure
//       updateAdjacentNodes): list B_{D-bar} ++ B_{D1} (just B_{D1} when D is
//       the root), S = list \ B_{C-bar}, B = B_{C-bar};
//   * leaf extraction: list B_{C-bar} ++ C; the kept set is C (plus, when bond
//       entries are wanted, the second nodes N of the bonds the leaf owns that
//       lie outside C); eliminating the rest leaves the Schur complement on
//       C u N, whose inverse is G(C u N, C u N) (eq. (cd1)); its Sigma block
//       gives G< on the same set by eq. (gless-nn);
//   * final leaf block: the inverse and G Sigma G^dagger of that block, run
//       as one more elimination of the bordered matrix [[U, I], [I, 0]].
// The same rules apply to Sigma with R in place of U (the Sigma_g block
// assembly of Sec. 3.1 and its leaf case).
#include "plan.hpp"

#include <algorithm>
#include <array>
#include <cstdio>
#include <cstdlib>
#include <map>
#include <numeric>

namespace findmi {

int count_bonds(int Nx, int Ny, int stencil) {
  int n = (Nx - 1) * Ny + Nx * (Ny - 1);
  if (stencil == 9) n += 2 * (Nx - 1) * (Ny - 1);
  return n;
}

double elim_flops(const Elim& e, int sym) {
  double s = e.s, b = e.b, q = e.ssig;
  // final leaf block of size s: the inverse (s^3) and T = R_K G^dagger over the
  // q rows and columns where R_K may be non-zero (q^2 s)
  if (e.kind == K_FINAL) return 8.0 * (s * s * s + q * q * s);
  // complex multiply-adds: LU s^3/3 + s^2 b / 2, L s^2 b / 2, U = A(B,B) - L A(S,B)
  // s b^2.  Sigma_g is supported on the q eliminated nodes that carry Sigma< (and
  // the kept ones): W_q = Sigma(B,S_q) - L_q Sigma(S_q,S_q) costs b q^2 and
  // R = Sigma(B,B) - [L_q | W_q] [Sigma(S_q,B) ; L_q^dagger] costs 2 q b^2 (q b^2
  // when no kept node carries Sigma<, so that Sigma(S_q,B) = 0).  With U complex
  // symmetric (sym bit 0) only its lower half is formed, and with R
  // anti-Hermitian (sym bit 1) only R's lower half.  With R = 0 (no Sigma< in
  // the front) W and R are not formed.
  // Kept nodes not coupled to S (b - bact of them) take no part in any of it.
  b = e.bact;
  const double hu = (sym & 1) ? 0.5 : 1.0, hr = (sym & 2) ? 0.5 : 1.0;
  const double base = s * s * s / 3.0 + s * s * b + hu * s * b * b;
  if (e.rzero) return 8.0 * base;
  const double q0 = e.bsig ? q : 0.0;
  return 8.0 * (base + b * q * q + hr * b * b * (q0 + q));
}

namespace {

struct Builder {
  Plan& P;
  int Nx, Ny, stencil;
  std::vector<int> mark;   // scratch marker over all nodes
  int stamp = 0;
  explicit Builder(Plan& p) : P(p), Nx(p.Nx), Ny(p.Ny), stencil(p.stencil), mark(size_t(p.Nx) * p.Ny, 0) {}
  // pool elements of one cluster's U and R for b kept nodes
  int64_t slot(int64_t b) const { return block_elems(b, P.pack & 1) + block_elems(b, P.pack & 2); }
  std::vector<std::pair<int64_t, int64_t>> slot_size;   // (provisional offset, elements) per slot

  // Split stages whose fronts differ widely in size.  At the tree levels that
  // touch a contact column, the dense contact coupling puts the whole column
  // into the boundary sets of the clusters next to it, so a few large fronts
  // share a stage with many small interior ones; a stage's launch
  // configuration is sized for its largest front.  The eliminations of a stage
  // are independent, so the stage becomes consecutive sub-stages by front
  // size class (at most 128, 256, 512, ... nodes), a class of fewer than
  // kMinSplit fronts joining the next larger one.  Final leaf blocks are not
  // split.
  void split_stages() {
    constexpr int kMinSplit = 16, kClasses = 6;
    auto cls = [](int n) { int c = 0; while (c < kClasses - 1 && n > (128 << c)) ++c; return c; };
    std::vector<Stage> out;
    for (const Stage& st : P.stages) {
      if (st.phase == PH_FINAL || st.count < 2 * kMinSplit) { out.push_back(st); continue; }
      int count[kClasses] = {0}, group_of[kClasses], groups = 0, acc = 0;
      for (int k = st.first; k < st.first + st.count; ++k) ++count[cls(P.elims[k].n)];
      for (int c = 0; c < kClasses; ++c) {
        group_of[c] = groups;
        acc += count[c];
        if (acc >= kMinSplit) { ++groups; acc = 0; }
      }
      if (acc > 0) {   // a small trailing group joins the one before it
        if (groups > 0)
          for (int c = 0; c < kClasses; ++c)
            if (group_of[c] == groups) group_of[c] = groups - 1;
        if (groups == 0) groups = 1;
      }
      if (groups <= 1) { out.push_back(st); continue; }
      std::vector<Elim> part;
      for (int g = 0; g < groups; ++g) {
        const int first = st.first + int(part.size());
        for (int k = st.first; k < st.first + st.count; ++k)
          if (group_of[cls(P.elims[k].n)] == g) part.push_back(P.elims[k]);
        const int cnt = st.first + int(part.size()) - first;
        if (cnt > 0) out.push_back({first, cnt, st.phase, st.variant});
      }
      std::copy(part.begin(), part.end(), P.elims.begin() + st.first);
    }
    P.stages = out;
  }

  // Place the slots in the energy pool by lifetime.  A slot lives from the
  // stage that writes it to the last stage that reads it (stages in plan
  // order; a solve runs a subset of them, in the same order), and two slots
  // share memory only if their lifetimes are disjoint: the upward results of a
  // level die once the downward pass has read them, the downward results of a
  // level once the next level (or the leaf extraction) has, so the pool holds
  // about the upward results plus two downward levels instead of every slot.
  // The node diagonal (read by every stage) comes first; slots start on
  // 16-element boundaries.  First fit over a free list, in stage order.
  void assign_pool() {
    const int ns = int(P.stages.size());
    std::map<int64_t, int> id;   // provisional offset -> slot
    for (size_t k = 0; k < slot_size.size(); ++k) id[slot_size[k].first] = int(k);
    const int n = int(slot_size.size());
    std::vector<int> birth(n, ns), death(n, -1);
    for (int t = 0; t < ns; ++t)
      for (int k = P.stages[t].first; k < P.stages[t].first + P.stages[t].count; ++k) {
        const Elim& e = P.elims[k];
        const int d = id.at(e.dst);
        birth[d] = std::min(birth[d], t);
        death[d] = std::max(death[d], t);
        for (int j = 0; j < 2; ++j)
          if (e.src_off[j] >= 0) death[id.at(e.src_off[j])] = std::max(death[id.at(e.src_off[j])], t);
      }
    auto up16 = [](int64_t x) { return (x + 15) & ~int64_t(15); };
    P.onsite_off = 0;
    const int64_t base = up16(2 * int64_t(Nx) * Ny);
    std::vector<int64_t> place(n, -1);
    std::map<int64_t, int64_t> free_ = {{base, INT64_MAX / 4}};   // offset -> length
    auto release = [&](int64_t o, int64_t len) {
      auto it = free_.emplace(o, len).first;
      auto nx = std::next(it);
      if (nx != free_.end() && it->first + it->second == nx->first) { it->second += nx->second; free_.erase(nx); }
      if (it != free_.begin()) {
        auto pv = std::prev(it);
        if (pv->first + pv->second == it->first) { pv->second += it->second; free_.erase(it); }
      }
    };
    int64_t high = base;
    for (int t = 0; t < ns; ++t) {
      for (int k = 0; k < n; ++k)   // free the slots last read before stage t
        if (place[k] >= 0 && death[k] < t && death[k] >= 0 && birth[k] <= death[k]) {
          release(place[k], up16(slot_size[k].second));
          death[k] = -2;   // released
        }
      for (int k = 0; k < n; ++k) {
        if (birth[k] != t) continue;
        const int64_t len = up16(slot_size[k].second);
        auto it = free_.begin();
        while (it->second < len) ++it;
        place[k] = it->first;
        const int64_t rest = it->second - len, at = it->first + len;
        free_.erase(it);
        if (rest > 0) free_.emplace(at, rest);
        high = std::max(high, place[k] + len);
      }
    }
    auto remap = [&](int64_t o) { return o < 0 ? o : place[id.at(o)]; };
    for (Elim& e : P.elims) {
      e.dst = remap(e.dst);
      for (int j = 0; j < 2; ++j) e.src_off[j] = remap(e.src_off[j]);
    }
    for (Cluster& c : P.cl) { c.up_off = remap(c.up_off); c.dn_off = remap(c.dn_off); }
    P.pool_per_energy = high;
  }

  bool inside(const Rect& r, int x, int y) const {
    return x >= r.x0 && x < r.x0 + r.w && y >= r.y0 && y < r.y0 + r.h;
  }

  void build_tree() {
    P.cl.clear();
    Cluster root;
    root.r = {0, 0, Nx, Ny};
    P.cl.push_back(root);
    for (size_t q = 0; q < P.cl.size(); ++q) {  // breadth-first
      Rect r = P.cl[q].r;
      if (r.w <= P.leaf && r.h <= P.leaf) continue;
      Rect a = r, b = r;
      if (r.h >= r.w) { a.h = r.h / 2; b.y0 = r.y0 + a.h; b.h = r.h - a.h; }
      else            { a.w = r.w / 2; b.x0 = r.x0 + a.w; b.w = r.w - a.w; }
      for (int k = 0; k < 2; ++k) {
        Cluster c;
        c.r = k ? b : a;
        c.parent = int(q);
        c.depth = P.cl[q].depth + 1;
        P.cl[q].child[k] = int(P.cl.size());
        P.cl.push_back(c);
      }
      P.cl[P.cl[q].child[0]].sibling = P.cl[q].child[1];
      P.cl[P.cl[q].child[1]].sibling = P.cl[q].child[0];
    }
    P.depth = 0; P.n_leaves = 0;
    for (int q = int(P.cl.size()) - 1; q >= 0; --q) {
      Cluster& c = P.cl[q];
      P.depth = std::max(P.depth, c.depth);
      if (c.leaf()) { c.height = 0; ++P.n_leaves; }
      else c.height = 1 + std::max(P.cl[c.child[0]].height, P.cl[c.child[1]].height);
    }
  }

  // Stencil neighbours of (x, y) inside the mesh.
  template <class F> void stencil_nbrs(int x, int y, F&& f) const {
    static const int d5[4][2] = {{1, 0}, {-1, 0}, {0, 1}, {0, -1}};
    static const int d9[4][2] = {{1, 1}, {-1, -1}, {1, -1}, {-1, 1}};
    for (auto& d : d5) { int u = x + d[0], v = y + d[1]; if (u >= 0 && u < Nx && v >= 0 && v < Ny) f(u, v); }
    if (stencil == 9)
      for (auto& d : d9) { int u = x + d[0], v = y + d[1]; if (u >= 0 && u < Nx && v >= 0 && v < Ny) f(u, v); }
  }

  void build_sets() {
    for (auto& c : P.cl) {
      const Rect r = c.r;
      ++stamp;  // stamp marks nodes already placed in Bc
      std::vector<int> B, Bc;
      for (int y = r.y0; y < r.y0 + r.h; ++y)
        for (int x = r.x0; x < r.x0 + r.w; ++x) {
          bool bnd = false;
          stencil_nbrs(x, y, [&](int u, int v) {
            if (!inside(r, u, v)) {
              bnd = true;
              int j = v * Nx + u;
              if (mark[j] != stamp) { mark[j] = stamp; Bc.push_back(j); }
            }
          });
          // dense contact blocks couple every pair of nodes on a contact column
          bool full_col = (r.x0 == 0 && r.w == Nx);
          if (P.contacts && (y == 0 || y == Ny - 1) && !full_col) bnd = true;
          if (bnd) B.push_back(y * Nx + x);
        }
      for (int cy : {0, Ny - 1}) {
        if (!P.contacts) break;
        if (cy < r.y0 || cy >= r.y0 + r.h) continue;  // C does not touch this contact column
        for (int x = 0; x < Nx; ++x) {
          if (x >= r.x0 && x < r.x0 + r.w) continue;
          int j = cy * Nx + x;
          if (mark[j] != stamp) { mark[j] = stamp; Bc.push_back(j); }
        }
      }
      std::sort(B.begin(), B.end());
      std::sort(Bc.begin(), Bc.end());
      c.B = std::move(B);
      c.Bc = std::move(Bc);
    }
  }

  // Position of each node of `list` in `keep` (-1 if absent); requires keep sorted.
  static int find_sorted(const std::vector<int>& v, int x) {
    auto it = std::lower_bound(v.begin(), v.end(), x);
    return (it != v.end() && *it == x) ? int(it - v.begin()) : -1;
  }

  // R_C = 0 for an upward-pass cluster away from both contact columns: Sigma<
  // is supported on the contact columns y = 0 and y = Ny - 1 only, so
  // Sigma<(C, C) = 0, and so R = 0 for it and (recursively) for all its
  // descendants
  // (with diagonal scattering self-energies every node carries Sigma<, and no R vanishes)
  bool up_rzero(const Cluster& c) const {
    return !P.scattering && (!P.contacts || (c.r.y0 > 0 && c.r.y0 + c.r.h < Ny));
  }

  // Emit an elimination whose assembled node list is `list` (with per-entry
  // source and source position) and whose kept set is `keep` (in this order).
  // sig_src[k][p]: the row of source k's stored R at position p may be
  // non-zero (null: source k has none).  An entry carries Sigma< (its row and
  // column of Sigma_g may be non-zero) if its source row does, or if it comes
  // from the original matrix and lies on a contact column; the eliminated
  // entries that carry it are placed first in S.  out_sig receives, per kept
  // node, whether its row of the resulting R may be non-zero: every row when
  // an eliminated node carries Sigma< (the L Sigma(S,S) L^dagger terms fill
  // R), else the rows of the kept nodes that carry it (R = Sigma_g(B,B)).
  // With keep_out, the kept nodes coupled to S (a common source, a stencil
  // bond, or one contact column) are moved ahead of the others, then the
  // uncoupled ones that carry Sigma<, and the resulting kept order is stored
  // there; *rsup_out receives the number of kept nodes whose rows of R may be
  // non-zero (coupled or carrying: R vanishes on the rest).  Otherwise `keep`
  // is used as given.
  std::string emit(const std::vector<int>& list, const std::vector<int>& src,
                   const std::vector<int>& pos, const std::vector<int>& keep_in, Elim e,
                   const std::vector<char>* const sig_src[2], std::vector<char>* out_sig = nullptr,
                   std::vector<int>* keep_out = nullptr, int* rsup_out = nullptr) {
    std::vector<int> keep = keep_in;
    std::vector<int> keep_sorted = keep;
    std::sort(keep_sorted.begin(), keep_sorted.end());
    std::vector<int> S_idx, in_list(keep.size(), -1);
    for (size_t k = 0; k < list.size(); ++k)
      if (find_sorted(keep_sorted, list[k]) < 0) S_idx.push_back(int(k));
    auto carries = [&](int k) -> bool {
      if (src[k] == SRC0 || src[k] == SRC1) return sig_src[src[k]] && (*sig_src[src[k]])[pos[k]];
      const int y = list[k] / Nx;
      return P.scattering || (P.contacts && (y == 0 || y == Ny - 1));
    };
    const auto mid = std::stable_partition(S_idx.begin(), S_idx.end(), carries);
    e.ssig = e.rzero ? 0 : int(mid - S_idx.begin());
    e.bsig = 0;
    // kept nodes in `keep` order, located in the list
    std::vector<int> listpos_sorted(list.size());
    std::iota(listpos_sorted.begin(), listpos_sorted.end(), 0);
    std::sort(listpos_sorted.begin(), listpos_sorted.end(), [&](int a, int b) { return list[a] < list[b]; });
    for (size_t q = 0; q < keep.size(); ++q) {
      auto it = std::lower_bound(listpos_sorted.begin(), listpos_sorted.end(), keep[q],
                                 [&](int a, int val) { return list[a] < val; });
      if (it == listpos_sorted.end() || list[*it] != keep[q]) {
        char buf[160];
        snprintf(buf, sizeof buf, "plan: kept node %d missing from assembled list (phase %d cluster %d)",
                 keep[q], e.phase, e.cluster);
        return buf;
      }
      in_list[q] = *it;
      if (!e.rzero && carries(*it)) e.bsig = 1;
    }
    e.bact = int(keep.size());
    if (keep_out) {
      auto coupled = [&](int kb) {
        const int xb = list[kb] % Nx, yb = list[kb] / Nx;
        for (int ks : S_idx) {
          if (src[ks] == src[kb] && src[kb] != SRC_ORIG) return true;
          const int xs = list[ks] % Nx, ys = list[ks] / Nx;
          const int dx = std::abs(xs - xb), dy = std::abs(ys - yb);
          if (dx <= 1 && dy <= 1 && (dx + dy == 1 || (stencil == 9 && dx + dy == 2))) return true;
          if (P.contacts && ys == yb && (ys == 0 || ys == Ny - 1)) return true;
        }
        return false;
      };
      std::vector<int> order(keep.size());
      std::iota(order.begin(), order.end(), 0);
      const auto mid = std::stable_partition(order.begin(), order.end(), [&](int q) { return coupled(in_list[q]); });
      e.bact = int(mid - order.begin());
      const auto mid2 = std::stable_partition(mid, order.end(), [&](int q) { return !e.rzero && carries(in_list[q]); });
      if (rsup_out) *rsup_out = e.rzero ? 0 : int(mid2 - order.begin());
      std::vector<int> k2, l2;
      for (int q : order) { k2.push_back(keep[q]); l2.push_back(in_list[q]); }
      keep.swap(k2); in_list.swap(l2);
      *keep_out = keep;
      // Sigma(S, B) vanishes on the uncoupled kept nodes: only coupled ones count
      e.bsig = 0;
      for (int q = 0; q < e.bact; ++q)
        if (!e.rzero && carries(in_list[q])) e.bsig = 1;
    }
    if (out_sig) {
      out_sig->assign(keep.size(), 0);
      if (!e.rzero)
        for (size_t q = 0; q < keep.size(); ++q) (*out_sig)[q] = (e.ssig > 0 || carries(in_list[q])) ? 1 : 0;
    }
    e.s = int(S_idx.size());
    e.b = int(keep.size());
    e.n = e.s + e.b;
    e.map = int(P.map_node.size());
    for (int k : S_idx) { P.map_node.push_back(list[k]); P.map_src.push_back(src[k]); P.map_pos.push_back(pos[k]); }
    for (int k : in_list) { P.map_node.push_back(list[k]); P.map_src.push_back(src[k]); P.map_pos.push_back(pos[k]); }
    P.elims.push_back(e);
    return "";
  }

  std::vector<int> cluster_nodes(const Rect& r) const {
    std::vector<int> v;
    for (int y = r.y0; y < r.y0 + r.h; ++y)
      for (int x = r.x0; x < r.x0 + r.w; ++x) v.push_back(y * Nx + x);
    return v;
  }

  // Second nodes of the bonds owned by the leaf (first node in C), and the
  // owned bonds themselves: (bond id, first node, second node, k, hflat).
  void leaf_bonds(const Rect& r, std::vector<std::array<int, 5>>& owned) const {
    const int nx1 = Nx - 1;
    const int off1 = nx1 * Ny, off2 = off1 + Nx * (Ny - 1), off3 = off2 + nx1 * (Ny - 1);
    for (int y = r.y0; y < r.y0 + r.h; ++y)
      for (int x = r.x0; x < r.x0 + r.w; ++x) {
        int i = y * Nx + x;
        if (x + 1 < Nx) owned.push_back({y * nx1 + x, i, i + 1, 1, y * Nx + x});
        if (y + 1 < Ny) owned.push_back({off1 + y * Nx + x, i, i + Nx, 2, y * Nx + x});
        if (stencil == 9 && x + 1 < Nx && y + 1 < Ny)
          owned.push_back({off2 + y * nx1 + x, i, i + Nx + 1, 3, y * Nx + x});
        if (stencil == 9 && x >= 1 && y + 1 < Ny)  // d- bond with first node (x, y) = ((x-1)+1, y)
          owned.push_back({off3 + y * nx1 + (x - 1), i, (y + 1) * Nx + (x - 1), 4, y * Nx + (x - 1)});
      }
  }

  std::string build() {
    build_tree();
    build_sets();
    const int nc = int(P.cl.size());
    // pool slots (provisional offsets, one per slot; assign_pool places them by
    // lifetime at the end): upward (U_C, R_C) and downward (U_{C-bar},
    // R_{C-bar}) for non-root clusters
    int64_t off = 0;
    auto new_slot = [&](int64_t size) { const int64_t o = off; slot_size.push_back({o, size}); off += size; return o; };
    for (int q = 1; q < nc; ++q) {
      Cluster& c = P.cl[q];
      c.up_off = new_slot(slot(c.B.size()));
      c.dn_off = new_slot(slot(c.Bc.size()));
    }
    std::string err;
    // ---- upward pass: stages by height (leaves first); the root is not eliminated
    int max_h = P.cl[0].height;
    for (int h = 0; h < max_h; ++h) {
      int first = int(P.elims.size());
      for (int q = 1; q < nc; ++q) {
        Cluster& c = P.cl[q];
        if (c.height != h) continue;
        Elim e; e.phase = PH_UP; e.cluster = q; e.level = c.depth; e.dst = c.up_off;
        e.rzero = up_rzero(c) ? 1 : 0;
        const std::vector<char>* sig_src[2] = {nullptr, nullptr};
        std::vector<int> list, src, pos;
        if (c.leaf()) {
          list = cluster_nodes(c.r);
          src.assign(list.size(), SRC_ORIG); pos.assign(list.size(), -1);
        } else {
          for (int k = 0; k < 2; ++k) {
            const Cluster& ch = P.cl[c.child[k]];
            for (size_t p = 0; p < ch.B.size(); ++p) { list.push_back(ch.B[p]); src.push_back(k); pos.push_back(int(p)); }
            e.src_off[k] = ch.up_off; e.src_ld[k] = int(ch.B.size());
            sig_src[k] = &ch.up_sig;
          }
        }
        if (!(err = emit(list, src, pos, c.B, e, sig_src, &c.up_sig)).empty()) return err;
      }
      if (int(P.elims.size()) > first) P.stages.push_back({first, int(P.elims.size()) - first, PH_UP, -1});
    }
    // ---- downward pass: stages by depth
    for (int d = 1; d <= P.depth; ++d) {
      int first = int(P.elims.size());
      for (int q = 1; q < nc; ++q) {
        Cluster& c = P.cl[q];
        if (c.depth != d) continue;
        const Cluster& D = P.cl[c.parent];
        const Cluster& D1 = P.cl[c.sibling];
        Elim e; e.phase = PH_DOWN; e.cluster = q; e.level = d; e.dst = c.dn_off;
        std::vector<int> list, src, pos;
        if (c.parent != 0) {
          for (size_t p = 0; p < D.Bc.size(); ++p) { list.push_back(D.Bc[p]); src.push_back(SRC0); pos.push_back(int(p)); }
          e.src_off[0] = D.dn_off; e.src_ld[0] = int(D.Bc.size());
        }
        for (size_t p = 0; p < D1.B.size(); ++p) { list.push_back(D1.B[p]); src.push_back(SRC1); pos.push_back(int(p)); }
        e.src_off[1] = D1.up_off; e.src_ld[1] = int(D1.B.size());
        const std::vector<char>* sig_src[2] = {c.parent != 0 ? &D.dn_sig : nullptr, &D1.up_sig};
        if (!(err = emit(list, src, pos, c.Bc, e, sig_src, &c.dn_sig)).empty()) return err;
      }
      if (int(P.elims.size()) > first) P.stages.push_back({first, int(P.elims.size()) - first, PH_DOWN, -1});
    }
    // ---- leaf extraction, two variants (0: diagonal only, 1: with bond entries)
    P.n_bonds = count_bonds(Nx, Ny, stencil);
    std::vector<int> leaves;
    for (int q = 0; q < nc; ++q) if (P.cl[q].leaf()) leaves.push_back(q);
    // Which leaves run the extraction, and what each keeps and outputs.  By
    // default every leaf outputs its own nodes and the bonds whose first node
    // it holds (keeping the bonds' other ends).  With half_leaves (the current
    // density scheme of Sec. 4.3: chosen leaves also output the diagonal and
    // bond entries of the ring of nodes around them, so the other leaves need
    // no extraction at all) a checkerboard of leaves is chosen, topped up
    // greedily until every node and bond lies in the kept set C u ring of a
    // chosen leaf, and every output is owned by one chosen leaf.
    const int nl = int(leaves.size());
    std::vector<int> leaf_of(size_t(Nx) * Ny, -1);
    for (int l = 0; l < nl; ++l)
      for (int i : cluster_nodes(P.cl[leaves[l]].r)) leaf_of[i] = l;
    std::vector<std::vector<std::array<int, 5>>> all_bonds(nl);   // bonds by the leaf of their first node
    for (int l = 0; l < nl; ++l) leaf_bonds(P.cl[leaves[l]].r, all_bonds[l]);
    std::vector<char> chosen(nl, 1);
    std::vector<std::vector<int>> own_nodes(nl), extra(nl * 2);   // extra[2 l + v]: kept nodes outside C
    std::vector<std::vector<std::array<int, 5>>> owned(nl);
    // leaves whose kept set C u ring(l) holds node i: its own leaf and the leaves of its neighbours
    auto leaves_at = [&](int i) {
      std::vector<int> ls{leaf_of[i]};
      stencil_nbrs(i % Nx, i / Nx, [&](int u, int v) { ls.push_back(leaf_of[v * Nx + u]); });
      std::sort(ls.begin(), ls.end());
      ls.erase(std::unique(ls.begin(), ls.end()), ls.end());
      return ls;
    };
    if (!P.half_leaves) {
      for (int l = 0; l < nl; ++l) {
        own_nodes[l] = cluster_nodes(P.cl[leaves[l]].r);
        owned[l] = all_bonds[l];
      }
    } else {
      for (int l = 0; l < nl; ++l) {
        const Rect& r = P.cl[leaves[l]].r;
        chosen[l] = ((r.x0 / 2 + r.y0 / 2) & 1) == 0;
      }
      // greedy top-up: a node or bond no chosen leaf holds chooses the leaf of its first node
      auto holder = [&](int i, int j) {   // a chosen leaf whose kept set holds i and j, else -1
        const std::vector<int> a = leaves_at(i), b = leaves_at(j);
        for (int l : a)
          if (chosen[l] && std::binary_search(b.begin(), b.end(), l)) return l;
        return -1;
      };
      for (int i = 0; i < Nx * Ny; ++i)
        if (holder(i, i) < 0) chosen[leaf_of[i]] = 1;
      for (int l = 0; l < nl; ++l)
        for (auto& ob : all_bonds[l])
          if (holder(ob[1], ob[2]) < 0) chosen[leaf_of[ob[1]]] = 1;
      // owners: the node's (bond's first node's) own leaf if chosen, else the
      // lowest chosen leaf holding it
      auto owner = [&](int i, int j) {
        if (chosen[leaf_of[i]]) {
          const std::vector<int> b = leaves_at(j);
          if (std::binary_search(b.begin(), b.end(), leaf_of[i])) return leaf_of[i];
        }
        return holder(i, j);
      };
      for (int i = 0; i < Nx * Ny; ++i) {
        const int l = owner(i, i);
        if (l < 0) return "plan: half-leaf extraction left a node uncovered";
        own_nodes[l].push_back(i);
        if (leaf_of[i] != l) { extra[2 * l].push_back(i); extra[2 * l + 1].push_back(i); }
      }
      for (int l0 = 0; l0 < nl; ++l0)
        for (auto& ob : all_bonds[l0]) {
          const int l = owner(ob[1], ob[2]);
          if (l < 0) return "plan: half-leaf extraction left a bond uncovered";
          owned[l].push_back(ob);
        }
    }
    for (int l = 0; l < nl; ++l) {
      if (!chosen[l]) continue;
      const Rect& r = P.cl[leaves[l]].r;
      for (auto& ob : owned[l])
        for (int end : {ob[1], ob[2]})
          if (!inside(r, end % Nx, end / Nx)) extra[2 * l + 1].push_back(end);
      for (int v = 0; v < 2; ++v) {
        std::vector<int>& x = extra[2 * l + v];
        std::sort(x.begin(), x.end());
        x.erase(std::unique(x.begin(), x.end()), x.end());
      }
    }
    // pool slots for leaf blocks: sized for the larger variant, shared by both
    std::vector<int64_t> leaf1_off(nl, -1), fin_off(nl, -1);
    std::vector<int> rsup(nl, 0);
    for (int l = 0; l < nl; ++l) {
      if (!chosen[l]) continue;
      const Cluster& c = P.cl[leaves[l]];
      const int64_t bp = int64_t(c.r.w) * c.r.h + int64_t(extra[2 * l + 1].size());
      leaf1_off[l] = new_slot(slot(bp));
      fin_off[l] = new_slot(bp * bp);   // G(K,K) of the final block (LU form), whole
    }
    for (int v = 0; v < 2; ++v) {
      int first = int(P.elims.size());
      std::vector<std::vector<int>> keeps(leaves.size());
      std::vector<int> ext_leaf;      // the leaves that run the extraction, in stage order
      for (int l = 0; l < nl; ++l) {
        if (!chosen[l]) continue;
        ext_leaf.push_back(l);
        const Cluster& c = P.cl[leaves[l]];
        std::vector<int> Cn = cluster_nodes(c.r);
        const std::vector<int>& N = extra[2 * l + v];
        std::vector<int> list, src, pos;
        Elim e; e.phase = PH_LEAF; e.cluster = leaves[l]; e.level = c.depth; e.dst = leaf1_off[l];
        if (leaves[l] != 0) {
          for (size_t p = 0; p < c.Bc.size(); ++p) { list.push_back(c.Bc[p]); src.push_back(SRC0); pos.push_back(int(p)); }
          e.src_off[0] = c.dn_off; e.src_ld[0] = int(c.Bc.size());
        }
        for (int i : Cn) { list.push_back(i); src.push_back(SRC_ORIG); pos.push_back(-1); }
        std::vector<int> keep = Cn;
        keep.insert(keep.end(), N.begin(), N.end());
        const std::vector<char>* sig_src[2] = {leaves[l] != 0 ? &c.dn_sig : nullptr, nullptr};
        if (!(err = emit(list, src, pos, keep, e, sig_src, nullptr, &keeps[l], &rsup[l])).empty()) return err;
      }
      P.stages.push_back({first, int(P.elims.size()) - first, PH_LEAF, v});
      first = int(P.elims.size());
      for (size_t t = 0; t < ext_leaf.size(); ++t) {
        const int l = ext_leaf[t];
        const Elim& le = P.elims[P.stages.back().first + t];
        Elim e; e.kind = K_FINAL; e.phase = PH_FINAL; e.cluster = leaves[l]; e.level = le.level;
        e.s = le.b; e.b = le.b; e.n = 2 * le.b;
        // R_K is supported on its first rsup rows and columns (the Sigma<-carrying
        // prefix of the final block); bact = b as every node is coupled
        e.ssig = rsup[l]; e.bact = le.b;
        e.src_off[0] = le.dst; e.src_ld[0] = le.b; e.dst = fin_off[l];
        e.map = int(P.map_node.size());
        for (int r = 0; r < 2 * le.b; ++r) {
          P.map_node.push_back(keeps[l][r % le.b]);
          P.map_src.push_back(r < le.b ? SRC0 : SRC1);
          P.map_pos.push_back(r % le.b);
        }
        P.elims.push_back(e);
        // output records: the nodes the leaf owns at their positions in the kept order
        LeafOut lo;
        lo.elim = int(P.elims.size()) - 1; lo.variant = v;
        lo.n_nodes = 0; lo.node_first = int(P.outnode_node.size());
        {
          std::vector<int> own = own_nodes[l];
          std::sort(own.begin(), own.end());
          for (int q2 = 0; q2 < int(keeps[l].size()); ++q2) {
            const int nd = keeps[l][q2];
            if (!std::binary_search(own.begin(), own.end(), nd)) continue;
            P.outnode_node.push_back(nd); P.outnode_local.push_back(q2);
            ++lo.n_nodes;
          }
          if (lo.n_nodes != int(own.size())) return "plan: owned node missing from leaf block";
        }
        lo.bond_first = int(P.outbonds.size()); lo.n_bonds = 0;
        if (v == 1) {
          std::vector<int> ks = keeps[l];
          std::vector<int> idx(ks.size());
          std::iota(idx.begin(), idx.end(), 0);
          std::sort(idx.begin(), idx.end(), [&](int a, int b) { return ks[a] < ks[b]; });
          auto local = [&](int node) {
            auto it = std::lower_bound(idx.begin(), idx.end(), node, [&](int a, int val) { return ks[a] < val; });
            return (it != idx.end() && ks[*it] == node) ? *it : -1;
          };
          for (auto& ob : owned[l]) {
            int li = local(ob[1]), lj = local(ob[2]);
            if (li < 0 || lj < 0) return "plan: bond endpoint missing from leaf block";
            P.outbonds.push_back({ob[0], li, lj, ob[3], ob[4]});
            ++lo.n_bonds;
          }
        }
        P.leafout.push_back(lo);
      }
      P.stages.push_back({first, int(P.elims.size()) - first, PH_FINAL, v});
    }
    split_stages();
    assign_pool();
    // size limits and flop model
    for (auto& st : P.stages)
      for (int k = st.first; k < st.first + st.count; ++k) {
        const Elim& e = P.elims[k];
        P.max_n = std::max(P.max_n, e.n); P.max_s = std::max(P.max_s, e.s); P.max_b = std::max(P.max_b, e.b);
        for (int mode : {0, 1, 3}) {
          const double f = elim_flops(e, mode);   // 0: general, 1: U halved, 3: U and R halved
          if (st.variant < 0) { P.flops[mode][0] += f; P.flops[mode][1] += f; }
          else P.flops[mode][st.variant] += f;
        }
      }
    return "";
  }
};

}  // namespace

std::string build_plan(int Nx, int Ny, int stencil, int leaf, Plan& P, bool scattering, bool half_leaves,
                       bool contacts, int pack) {
  P = Plan();
  P.pack = pack;
  P.Nx = Nx; P.Ny = Ny; P.stencil = stencil; P.leaf = leaf; P.scattering = scattering;
  P.half_leaves = half_leaves;
  P.contacts = contacts;
  Builder b(P);
  return b.build();
}

}  // namespace findmi
