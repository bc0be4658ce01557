// Expansion of formatted H-matrix products and of the recursive H-inverse
// into per-target piece lists (see hprog.h).
//
// Product C(t,s) += alpha A(t,r) B(r,s) on the common block tree follows
// Hackbusch's recursion: while A(t,r) and B(r,s) are both subdivided the
// recursion descends into the 2x2x2 children; if C(t,s) is a leaf at that
// point the children become sub-windows of that leaf.  When A(t,r) or B(r,s)
// is a leaf the product is emitted:
//   A low rank  (U V^T): U (B^T V)^T        -> piece LRX, list = B-region
//   B low rank  (U V^T): (A U) V^T          -> piece LRY, list = A-region
//   dense x dense                           -> piece DD
//   dense x region / region x dense: split over the region's leaves
//   (low-rank leaves give LRY / LRX pieces, dense leaves DD pieces).
// Each emitted product is restricted to every target leaf it overlaps.
//
// H-inverse of a diagonal block (tau,tau) with children tau1, tau2 (the
// 2x2 Schur-complement formula):
//   X11 = inv(M11);  T12 = X11 M12;  T21 = M21 X11;  M22 <- M22 - M21 T12;
//   X22 = inv(M22);  X12 = -T12 X22; X21 = -X22 T21; X11 <- X11 - X12 T21,
// dense diagonal leaves inverted by LU-type elimination with partial
// pivoting.  Every step is batched over all instances of role 0.
#include "program.h"

#include <algorithm>
#include <functional>
#include <stdexcept>

namespace acr {

namespace {
inline int lo_of(const Geometry& G, int c) { return G.cl[c].lo; }
inline int hi_of(const Geometry& G, int c) { return G.cl[c].hi; }
}  // namespace

void StepBuilder::mul(int arole, int brole, int crole, int t, int r, int s, double alpha) {
  rec(arole, brole, crole, t, r, s, -1, alpha);
}

void StepBuilder::rec(int arole, int brole, int crole, int t, int r, int s, int vleaf, double alpha) {
  const int na = G.node(t, r), nb = G.node(r, s);
  if (na < 0 || nb < 0) throw std::runtime_error("block tree: missing operand block");
  const int nc = vleaf < 0 ? G.node(t, s) : -1;
  if (vleaf < 0 && nc < 0) throw std::runtime_error("block tree: missing target block");
  const BNode &A = G.bn[na], &B = G.bn[nb];
  if (A.kind == BK_H && B.kind == BK_H) {
    int v = vleaf;
    if (v < 0 && G.bn[nc].kind != BK_H) v = G.bn[nc].leaf;  // continue inside the target leaf
    const Cluster &ct = G.cl[t], &cr = G.cl[r], &cs = G.cl[s];
    const int tc[2] = {ct.c0, ct.c1}, rc[2] = {cr.c0, cr.c1}, sc[2] = {cs.c0, cs.c1};
    for (int i = 0; i < 2; ++i)
      for (int j = 0; j < 2; ++j)
        for (int l = 0; l < 2; ++l) rec(arole, brole, crole, tc[i], rc[l], sc[j], v, alpha);
    return;
  }
  emit(arole, brole, crole, t, r, s, na, nb, nc, vleaf, alpha);
}

void StepBuilder::add_piece_for_targets(const std::vector<int>& tg, Piece pc, int pr0, int pr1, int pc0, int pc1,
                                        const std::vector<int>* list, int list_is_rows, int crole) {
  for (int c : tg) {
    const Leaf& L = G.lf[c];
    int wr0 = std::max(pr0, L.r0), wr1 = std::min(pr1, L.r0 + L.m);
    int wc0 = std::max(pc0, L.c0), wc1 = std::min(pc1, L.c0 + L.n);
    if (wr0 >= wr1 || wc0 >= wc1) continue;
    Piece q = pc;
    q.wr0 = wr0;
    q.wr1 = wr1;
    q.wc0 = wc0;
    q.wc1 = wc1;
    std::vector<int32_t> fl;
    if (list) {
      for (int l : *list) {
        const Leaf& M = G.lf[l];
        if (list_is_rows) {
          if (std::max(M.r0, wr0) < std::min(M.r0 + M.m, wr1)) fl.push_back(l);
        } else {
          if (std::max(M.c0, wc0) < std::min(M.c0 + M.n, wc1)) fl.push_back(l);
        }
      }
      if (fl.empty()) continue;
    }
    acc_[{crole, c}].emplace_back(q, std::move(fl));
  }
}

void StepBuilder::emit(int arole, int brole, int crole, int t, int r, int s, int na, int nb, int nc, int vleaf,
                       double alpha) {
  std::vector<int> tg;
  if (vleaf >= 0)
    tg.push_back(vleaf);
  else
    G.leaves_under(nc, tg);
  const BNode &A = G.bn[na], &B = G.bn[nb];
  const int ar0 = lo_of(G, t), ar1 = hi_of(G, t), bc0 = lo_of(G, s), bc1 = hi_of(G, s);
  Piece base{};
  base.alpha = alpha;
  base.rv = base.cv = -1;
  base.l0 = base.l1 = 0;
  const bool a_leaf = A.kind != BK_H, b_leaf = B.kind != BK_H;
  const bool a_lr = a_leaf && G.lf[A.leaf].fmt == LF_LR;
  const bool b_lr = b_leaf && G.lf[B.leaf].fmt == LF_LR;
  if (a_lr) {
    std::vector<int> list;
    G.leaves_under(nb, list);
    Piece pc = base;
    pc.kind = PK_LRX;
    pc.xrole = arole;
    pc.xleaf = A.leaf;
    pc.yrole = brole;
    pc.yleaf = -1;
    add_piece_for_targets(tg, pc, ar0, ar1, bc0, bc1, &list, 0, crole);
    return;
  }
  if (b_lr) {
    std::vector<int> list;
    G.leaves_under(na, list);
    Piece pc = base;
    pc.kind = PK_LRY;
    pc.xrole = arole;
    pc.xleaf = -1;
    pc.yrole = brole;
    pc.yleaf = B.leaf;
    add_piece_for_targets(tg, pc, ar0, ar1, bc0, bc1, &list, 1, crole);
    return;
  }
  // both operands dense leaves or dense x region
  if (a_leaf && b_leaf) {
    Piece pc = base;
    pc.kind = PK_DD;
    pc.xrole = arole;
    pc.xleaf = A.leaf;
    pc.yrole = brole;
    pc.yleaf = B.leaf;
    add_piece_for_targets(tg, pc, ar0, ar1, bc0, bc1, nullptr, 0, crole);
    return;
  }
  if (a_leaf) {  // dense A-leaf times the B-region: split over B's leaves
    std::vector<int> list;
    G.leaves_under(nb, list);
    for (int l : list) {
      const Leaf& M = G.lf[l];
      Piece pc = base;
      if (M.fmt == LF_LR) {
        pc.kind = PK_LRY;
        pc.xrole = arole;
        pc.xleaf = -1;
        pc.yrole = brole;
        pc.yleaf = l;
        std::vector<int> one{A.leaf};
        add_piece_for_targets(tg, pc, ar0, ar1, M.c0, M.c0 + M.n, &one, 1, crole);
      } else {
        pc.kind = PK_DD;
        pc.xrole = arole;
        pc.xleaf = A.leaf;
        pc.yrole = brole;
        pc.yleaf = l;
        add_piece_for_targets(tg, pc, ar0, ar1, M.c0, M.c0 + M.n, nullptr, 0, crole);
      }
    }
    return;
  }
  // A-region times dense B-leaf: split over A's leaves
  std::vector<int> list;
  G.leaves_under(na, list);
  for (int l : list) {
    const Leaf& M = G.lf[l];
    Piece pc = base;
    if (M.fmt == LF_LR) {
      pc.kind = PK_LRX;
      pc.xrole = arole;
      pc.xleaf = l;
      pc.yrole = brole;
      pc.yleaf = -1;
      std::vector<int> one{B.leaf};
      add_piece_for_targets(tg, pc, M.r0, M.r0 + M.m, bc0, bc1, &one, 0, crole);
    } else {
      pc.kind = PK_DD;
      pc.xrole = arole;
      pc.xleaf = l;
      pc.yrole = brole;
      pc.yleaf = B.leaf;
      add_piece_for_targets(tg, pc, M.r0, M.r0 + M.m, bc0, bc1, nullptr, 0, crole);
    }
  }
}

void StepBuilder::copy(int srole, int crole, int node, double alpha, int rv, int cv) {
  std::vector<int> tg;
  G.leaves_under(node, tg);
  for (int c : tg) {
    const Leaf& L = G.lf[c];
    Piece pc{};
    pc.kind = PK_COPY;
    pc.alpha = alpha;
    pc.xrole = srole;
    pc.xleaf = c;
    pc.yrole = -1;
    pc.yleaf = -1;
    pc.wr0 = L.r0;
    pc.wr1 = L.r0 + L.m;
    pc.wc0 = L.c0;
    pc.wc1 = L.c0 + L.n;
    pc.rv = rv;
    pc.cv = cv;
    acc_[{crole, c}].emplace_back(pc, std::vector<int32_t>{});
  }
}

void StepBuilder::targets(int crole, int node, int beta) {
  if (step_t0_ < 0) step_t0_ = (int)P.targets.size();
  std::vector<int> tg;
  G.leaves_under(node, tg);
  for (int c : tg) {
    Target T{};
    T.crole = crole;
    T.cleaf = c;
    T.beta = beta;
    T.p0 = (int)P.pieces.size();
    auto it = acc_.find({crole, c});
    int ncopy = 0, nother = 0;
    if (it != acc_.end()) {
      for (auto& pr : it->second) {
        Piece pc = pr.first;
        if (!pr.second.empty()) {
          pc.l0 = (int)P.lists.size();
          P.lists.insert(P.lists.end(), pr.second.begin(), pr.second.end());
          pc.l1 = (int)P.lists.size();
        }
        (pc.kind == PK_COPY ? ncopy : nother)++;
        P.pieces.push_back(pc);
      }
      acc_.erase(it);
    }
    T.p1 = (int)P.pieces.size();
    T.direct = (beta == 0 && ncopy == 1 && nother == 0 && G.lf[c].fmt == LF_LR) ? 1 : 0;
    P.targets.push_back(T);
  }
}

void StepBuilder::finish_step() {
  if (!acc_.empty()) throw std::runtime_error("step builder: pieces without targets");
  Step st{};
  st.type = 0;
  st.t0 = step_t0_ < 0 ? (int)P.targets.size() : step_t0_;
  st.nt = (int)P.targets.size() - st.t0;
  st.leaf = -1;
  st.max_m = st.max_n = 0;
  for (int i = st.t0; i < st.t0 + st.nt; ++i) {
    st.max_m = std::max(st.max_m, G.lf[P.targets[i].cleaf].m);
    st.max_n = std::max(st.max_n, G.lf[P.targets[i].cleaf].n);
  }
  P.max_m = std::max(P.max_m, st.max_m);
  P.max_n = std::max(P.max_n, st.max_n);
  // Longest targets first: the blocks of a launch take targets in order, so
  // a long one (a large low-rank leaf fed by long leaf lists) that came last
  // would run alone at the end of the step.  The estimate is the target's
  // border (m + n) times its pieces and their list leaves; targets are
  // independent, so the order changes no result.
  auto cost = [&](const Target& T) {
    const Leaf& L = G.lf[T.cleaf];
    int64_t w = 0;
    for (int p = T.p0; p < T.p1; ++p) w += 1 + (P.pieces[p].l1 - P.pieces[p].l0);
    return (int64_t)(L.m + L.n) * w;
  };
  std::stable_sort(P.targets.begin() + st.t0, P.targets.begin() + st.t0 + st.nt,
                   [&](const Target& a, const Target& b) { return cost(a) > cost(b); });
  if (st.nt > 0) P.steps.push_back(st);
  step_t0_ = -1;
}

Program build_inverse_program(const Geometry& G) {
  Program P;
  StepBuilder sb(G, P);
  const int M = 0, T = 1;
  std::function<void(int)> inv = [&](int tau) {
    const int nd = G.node(tau, tau);
    const BNode& b = G.bn[nd];
    if (b.kind != BK_H) {
      const Leaf& L = G.lf[b.leaf];
      if (L.fmt != LF_DENSE || L.m != L.n) throw std::runtime_error("H-inverse: diagonal leaf is not dense square");
      Step st{};
      st.type = 1;
      st.leaf = b.leaf;
      st.max_m = L.m;
      st.max_n = L.n;
      P.steps.push_back(st);
      return;
    }
    const int t1 = G.cl[tau].c0, t2 = G.cl[tau].c1;
    const int n12 = G.node(t1, t2), n21 = G.node(t2, t1), n22 = G.node(t2, t2), n11 = G.node(t1, t1);
    inv(t1);
    // T12 = X11 M12 ; T21 = M21 X11
    sb.mul(M, M, T, t1, t1, t2, 1.0);
    sb.mul(M, M, T, t2, t1, t1, 1.0);
    sb.targets(T, n12, 0);
    sb.targets(T, n21, 0);
    sb.finish_step();
    // S = M22 - M21 T12
    sb.mul(M, T, M, t2, t1, t2, -1.0);
    sb.targets(M, n22, 1);
    sb.finish_step();
    inv(t2);
    // X12 = -T12 X22 ; X21 = -X22 T21
    sb.mul(T, M, M, t1, t2, t2, -1.0);
    sb.mul(M, T, M, t2, t2, t1, -1.0);
    sb.targets(M, n12, 0);
    sb.targets(M, n21, 0);
    sb.finish_step();
    // X11 <- X11 - X12 T21
    sb.mul(M, T, M, t1, t2, t1, -1.0);
    sb.targets(M, n11, 1);
    sb.finish_step();
  };
  inv(0);
  return P;
}

}  // namespace acr
