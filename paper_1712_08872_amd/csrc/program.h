// Host-side expansion of H-arithmetic into batched device steps.
#pragma once
#include <map>
#include <string>
#include <utility>
#include <vector>

#include "geometry.h"
#include "hprog.h"

namespace acr {

struct Step {
  int type;      // 0: accumulate (targets [t0, t0+nt)), 1: dense leaf inverse of `leaf`
  int t0, nt;
  int leaf;
  int max_m, max_n;  // largest target dimensions (scratch sizing)
  int64_t dstride = 0;  // elements of dense accumulators per batch item
};

struct Program {
  std::vector<Piece> pieces;
  std::vector<Target> targets;
  std::vector<int32_t> lists;
  std::vector<Step> steps;
  // device copies (owned by the handle that uploaded them)
  Piece* d_pieces = nullptr;
  Target* d_targets = nullptr;
  int32_t* d_lists = nullptr;
  // per target: offset of its dense accumulator within its step's per-item
  // region (small low-rank targets that may be summed densely), else -1
  std::vector<int64_t> doff;
  int64_t* d_doff = nullptr;
  int max_m = 0, max_n = 0;
  std::string name;
};

// Collects the pieces of one device step: any number of formatted products
// and scaled copies into leaves of target roles, then turns them into
// Target records.
class StepBuilder {
 public:
  StepBuilder(const Geometry& g, Program& p) : G(g), P(p) {}
  // C(t,s) <- ... + alpha A(t,r) B(r,s)  (roles; t, r, s are clusters)
  void mul(int arole, int brole, int crole, int t, int r, int s, double alpha);
  // C <- ... + alpha diag(v_rv) S diag(v_cv) leaf by leaf under `node`
  void copy(int srole, int crole, int node, double alpha, int rv, int cv);
  // emit targets for every leaf under `node` in role `crole` and close the step
  void targets(int crole, int node, int beta);
  void finish_step();

 private:
  void rec(int arole, int brole, int crole, int t, int r, int s, int vleaf, double alpha);
  void emit(int arole, int brole, int crole, int t, int r, int s, int na, int nb, int nc, int vleaf, double alpha);
  void add_piece_for_targets(const std::vector<int>& tg, Piece pc, int prow0, int prow1, int pcol0, int pcol1,
                             const std::vector<int>* list, int list_is_rows, int crole);
  const Geometry& G;
  Program& P;
  std::map<std::pair<int, int>, std::vector<std::pair<Piece, std::vector<int32_t>>>> acc_;
  int step_t0_ = -1;
};

// Program of the recursive 2x2 H-inverse of the root block, in place in
// role 0 with scratch role 1.
Program build_inverse_program(const Geometry& g);

}  // namespace acr
