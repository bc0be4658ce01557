// Plane geometry of the H-matrices: cluster tree, block cluster tree and
// the fixed storage layout of one H-matrix instance.
//
// Cluster tree (Sec. 3.1.2 with the planar bisection of Sec. 4.2): the
// root is the nx x ny index box of a plane; boxes with at most n_min points
// are leaves; otherwise the longer side is split (ties split x) into
// floor(s/2) and the rest, lower coordinates first.  Depth-first leaf
// order is the H-order of the plane's unknowns.
//
// Block cluster tree (Sec. 3.1.3-3.1.4, eq. admis): (t,s) is admissible iff
// dist > 0 and min(diam t, diam s) <= eta dist (bounding boxes in grid
// units, Euclidean); admissible -> low-rank leaf, inadmissible with a leaf
// cluster -> dense leaf, otherwise 2 x 2 children.  One tree serves every
// H-matrix of a plane shape.
#pragma once
#include <cstdint>
#include <string>
#include <unordered_map>
#include <vector>

namespace acr {

struct Cluster {
  int lo, hi;          // H-order index range [lo, hi)
  int x0, x1, y0, y1;  // bounding box, half-open, grid units
  int c0, c1;          // children (-1 for leaves)
  int depth;
  int size() const { return hi - lo; }
  bool leaf() const { return c0 < 0; }
};

enum BKind : int8_t { BK_H = 0, BK_DENSE = 1, BK_LR = 2 };

struct BNode {
  int t, s;
  BKind kind;          // geometric kind
  int ch[4];           // children (t_i, s_j) at ch[2*i+j]; -1 for leaves
  int leaf;            // leaf index for leaves, -1 otherwise
};

// Working/storage format of a leaf.  Inadmissible leaves are dense;
// admissible leaves are low rank unless their smaller dimension is at most
// `dense_work`, in which case they are held dense (exactly) during setup.
enum LFmt : int32_t { LF_DENSE = 0, LF_LR = 1 };

struct Leaf {
  int node;
  int t, s;            // clusters
  int m, n;            // |t|, |s|
  int r0, c0;          // H-order offsets of the block (rows t.lo, cols s.lo)
  int fmt;             // LFmt
  int adm;             // 1 if geometrically admissible
  int cap;             // rank capacity (LR) or 0
  int64_t off;         // element offset inside an instance
};

struct Geometry {
  int nx = 0, ny = 0, leaf_size = 32, dense_work = 0;
  double eta = 2.0;
  std::vector<Cluster> cl;
  std::vector<int> perm;                 // H-order position -> natural in-plane index
  std::vector<int> leaf_clusters;        // leaf clusters in H-order
  std::vector<BNode> bn;                 // block tree nodes, root = 0
  std::unordered_map<int64_t, int> bmap; // (t,s) -> node
  std::vector<Leaf> lf;                  // leaves (dense and low rank)
  int64_t inst_elems = 0;                // elements of one instance (dense + LR at capacity)
  int64_t dense_elems = 0;
  int nlr = 0, ndense = 0;
  int max_dense_rows = 0, max_dense_cols = 0, max_lr_dim = 0, max_cap = 0;
  // per leaf cluster: leaves whose row (resp. column) range contains it
  std::vector<std::vector<int>> rows_of_seg, cols_of_seg;

  int B() const { return nx * ny; }
  int node(int t, int s) const {
    auto it = bmap.find((int64_t)t * (int64_t)cl.size() + s);
    return it == bmap.end() ? -1 : it->second;
  }
  void leaves_under(int node, std::vector<int>& out) const;
  // rank capacities: cap(leaf) = min(m, n, cap_for_depth(depth))
  void assign_caps(const std::vector<int>& cap_by_depth);
  int max_depth() const;
  std::string summary() const;
};

// Build the geometry of a plane shape.  Capacities are set separately by
// assign_caps.
// diag9: the plane blocks also couple diagonal in-plane neighbours (the
// 27-point operator), which level 0 must hold exactly as well.
Geometry build_geometry(int nx, int ny, int leaf_size, double eta, int dense_work, bool diag9 = false);

}  // namespace acr
