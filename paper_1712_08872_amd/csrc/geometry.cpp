// Plane geometry: bisection cluster tree, admissibility-driven block tree
// and the storage layout of an H-matrix instance.
#include "geometry.h"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <functional>

namespace acr {

namespace {

int64_t diam2(const Cluster& c) {
  int64_t dx = c.x1 - 1 - c.x0, dy = c.y1 - 1 - c.y0;
  return dx * dx + dy * dy;
}

int64_t dist2(const Cluster& a, const Cluster& b) {
  int64_t dx = std::max<int64_t>({0, (int64_t)b.x0 - (a.x1 - 1), (int64_t)a.x0 - (b.x1 - 1)});
  int64_t dy = std::max<int64_t>({0, (int64_t)b.y0 - (a.y1 - 1), (int64_t)a.y0 - (b.y1 - 1)});
  return dx * dx + dy * dy;
}

}  // namespace

Geometry build_geometry(int nx, int ny, int leaf_size, double eta, int dense_work, bool diag9) {
  Geometry g;
  g.nx = nx;
  g.ny = ny;
  g.leaf_size = leaf_size;
  g.eta = eta;
  g.dense_work = dense_work;

  // ---- cluster tree by recursive bisection of the longer side
  std::function<int(int, int, int, int, int)> rec = [&](int x0, int x1, int y0, int y1, int d) {
    int id = (int)g.cl.size();
    Cluster c{(int)g.perm.size(), 0, x0, x1, y0, y1, -1, -1, d};
    g.cl.push_back(c);
    int sx = x1 - x0, sy = y1 - y0;
    if (sx * sy <= leaf_size) {
      for (int y = y0; y < y1; ++y)
        for (int x = x0; x < x1; ++x) g.perm.push_back(x + nx * y);
      g.leaf_clusters.push_back(id);
    } else if (sx >= sy) {
      int m = x0 + sx / 2;
      int a = rec(x0, m, y0, y1, d + 1);
      int b = rec(m, x1, y0, y1, d + 1);
      g.cl[id].c0 = a;
      g.cl[id].c1 = b;
    } else {
      int m = y0 + sy / 2;
      int a = rec(x0, x1, y0, m, d + 1);
      int b = rec(x0, x1, m, y1, d + 1);
      g.cl[id].c0 = a;
      g.cl[id].c1 = b;
    }
    g.cl[id].hi = (int)g.perm.size();
    return id;
  };
  rec(0, nx, 0, ny, 0);

  // ---- block tree under the admissibility condition
  const double eta2 = eta * eta;
  const int64_t ncl = (int64_t)g.cl.size();
  std::function<int(int, int)> brec = [&](int t, int s) {
    int id = (int)g.bn.size();
    g.bn.push_back(BNode{t, s, BK_H, {-1, -1, -1, -1}, -1});
    g.bmap[(int64_t)t * ncl + s] = id;
    const Cluster &ct = g.cl[t], &cs = g.cl[s];
    int64_t d2 = dist2(ct, cs);
    if (d2 > 0 && (double)std::min(diam2(ct), diam2(cs)) <= eta2 * (double)d2) {
      g.bn[id].kind = BK_LR;
    } else if (ct.leaf() || cs.leaf()) {
      g.bn[id].kind = BK_DENSE;
    } else {
      int tc[2] = {ct.c0, ct.c1}, sc[2] = {cs.c0, cs.c1};
      for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j) {
          int c = brec(tc[i], sc[j]);
          g.bn[id].ch[2 * i + j] = c;
        }
    }
    return id;
  };
  brec(0, 0);

  // ---- leaves, formats and (capacity-independent) fields
  for (int id = 0; id < (int)g.bn.size(); ++id) {
    BNode& b = g.bn[id];
    if (b.kind == BK_H) continue;
    Leaf L;
    L.node = id;
    L.t = b.t;
    L.s = b.s;
    L.m = g.cl[b.t].size();
    L.n = g.cl[b.s].size();
    L.r0 = g.cl[b.t].lo;
    L.c0 = g.cl[b.s].lo;
    L.adm = b.kind == BK_LR;
    L.fmt = (b.kind == BK_LR && std::min(L.m, L.n) > dense_work) ? LF_LR : LF_DENSE;
    L.cap = 0;
    L.off = 0;
    b.leaf = (int)g.lf.size();
    g.lf.push_back(L);
  }

  // In-plane couplings (5-point, or 9-point with diag9) inside an admissible
  // low-rank leaf (possible only for large eta) would not be representable
  // exactly at level 0: such leaves are kept dense.
  {
    std::vector<int> pos(nx * ny);
    for (int i = 0; i < nx * ny; ++i) pos[g.perm[i]] = i;
    std::vector<int> leaf_of_pos(nx * ny);
    for (int lc : g.leaf_clusters)
      for (int i = g.cl[lc].lo; i < g.cl[lc].hi; ++i) leaf_of_pos[i] = lc;
    auto find_leaf = [&](int i, int j) {
      // descend the block tree from the root
      int nd = 0;
      while (g.bn[nd].kind == BK_H) {
        const BNode& b = g.bn[nd];
        int tc0 = g.cl[b.t].c0, sc0 = g.cl[b.s].c0;
        int ii = i < g.cl[tc0].hi ? 0 : 1;
        int jj = j < g.cl[sc0].hi ? 0 : 1;
        nd = b.ch[2 * ii + jj];
      }
      return g.bn[nd].leaf;
    };
    for (int y = 0; y < ny; ++y)
      for (int x = 0; x < nx; ++x) {
        int i = pos[x + nx * y];
        const int dxs[8] = {-1, 1, 0, 0, -1, 1, -1, 1}, dys[8] = {0, 0, -1, 1, -1, -1, 1, 1};
        for (int d = 0; d < (diag9 ? 8 : 4); ++d) {
          int xx = x + dxs[d], yy = y + dys[d];
          if (xx < 0 || xx >= nx || yy < 0 || yy >= ny) continue;
          int j = pos[xx + nx * yy];
          int l = find_leaf(i, j);
          if (g.lf[l].fmt == LF_LR) g.lf[l].fmt = LF_DENSE;
        }
      }
  }

  // ---- segment lists for the H-matvec: leaves covering each leaf cluster
  std::vector<int> seg_of_cluster(g.cl.size(), -1);
  for (int k = 0; k < (int)g.leaf_clusters.size(); ++k) seg_of_cluster[g.leaf_clusters[k]] = k;
  g.rows_of_seg.assign(g.leaf_clusters.size(), {});
  g.cols_of_seg.assign(g.leaf_clusters.size(), {});
  for (int l = 0; l < (int)g.lf.size(); ++l) {
    const Leaf& L = g.lf[l];
    for (int k = 0; k < (int)g.leaf_clusters.size(); ++k) {
      const Cluster& c = g.cl[g.leaf_clusters[k]];
      if (c.lo >= L.r0 && c.hi <= L.r0 + L.m) g.rows_of_seg[k].push_back(l);
      if (c.lo >= L.c0 && c.hi <= L.c0 + L.n) g.cols_of_seg[k].push_back(l);
    }
  }
  for (const Leaf& L : g.lf) ++(L.fmt == LF_LR ? g.nlr : g.ndense);
  return g;
}

void Geometry::leaves_under(int nd, std::vector<int>& out) const {
  const BNode& b = bn[nd];
  if (b.kind != BK_H) {
    out.push_back(b.leaf);
    return;
  }
  for (int q = 0; q < 4; ++q) leaves_under(b.ch[q], out);
}

int Geometry::max_depth() const {
  int d = 0;
  for (const auto& c : cl) d = std::max(d, c.depth);
  return d;
}

void Geometry::assign_caps(const std::vector<int>& cap_by_depth) {
  inst_elems = 0;
  nlr = ndense = 0;
  max_dense_rows = max_dense_cols = max_lr_dim = max_cap = 0;
  // dense leaves first, then low-rank leaves: the apply streams the dense
  // part contiguously
  for (auto& L : lf) {
    if (L.fmt != LF_DENSE) continue;
    L.cap = 0;
    L.off = inst_elems;
    inst_elems += (int64_t)L.m * L.n;
    ++ndense;
    max_dense_rows = std::max(max_dense_rows, L.m);
    max_dense_cols = std::max(max_dense_cols, L.n);
  }
  dense_elems = inst_elems;
  for (auto& L : lf) {
    if (L.fmt != LF_LR) continue;
    int d = cl[L.t].depth;
    int c = cap_by_depth[std::min<int>(d, (int)cap_by_depth.size() - 1)];
    L.cap = std::max(1, std::min({L.m, L.n, c}));
    L.off = inst_elems;
    inst_elems += (int64_t)(L.m + L.n) * L.cap;
    ++nlr;
    max_lr_dim = std::max({max_lr_dim, L.m, L.n});
    max_cap = std::max(max_cap, L.cap);
  }
}

std::string Geometry::summary() const {
  char buf[256];
  snprintf(buf, sizeof(buf), "plane %dx%d leaf %d eta %.3g: %zu clusters, %d dense + %d LR leaves, %lld elems",
           nx, ny, leaf_size, eta, cl.size(), ndense, nlr, (long long)inst_elems);
  return buf;
}

}  // namespace acr
