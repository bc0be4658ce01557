// Import of a factorisation given on the host (acr_import_factors): the
// cyclic-reduction structure of Sec. 4.1 (plane lists, eliminated and kept
// planes per level) is rebuilt from nz, and every stored factor is taken
// from the caller instead of being computed, so the apply kernels run on
// exactly the given H-matrices.
#include <hip/hip_runtime.h>

#include <map>
#include <tuple>

#include "runtime.h"

namespace acr {

namespace {
// The plane lists P_0 = (0..nz-1), P_{r+1} = entries at odd 0-based
// positions of P_r, down to one plane.
std::vector<std::vector<int>> plane_lists(int nz) {
  std::vector<std::vector<int>> Pl{{}};
  for (int k = 0; k < nz; ++k) Pl[0].push_back(k);
  while (Pl.back().size() > 1) {
    std::vector<int> K;
    for (size_t q = 1; q < Pl.back().size(); q += 2) K.push_back(Pl.back()[q]);
    Pl.push_back(K);
  }
  return Pl;
}
}  // namespace

// Host-side check of a factor blob against the cyclic-reduction structure
// of nz planes and the plane geometry of (nx, ny, options); throws
// ACR_E_INVALID.  Needs no device.
void check_factor_blob(const acr_problem* p, const acr_options* o, const acr_factor_blob* blob) {
  if (o->precision == ACR_MIXED_BF16) throw AcrError(ACR_E_INVALID, "import supports FP64 and FP32 factors");
  const auto Pl = plane_lists(p->nz);
  const int top = (int)Pl.size() - 1;
  const Geometry G = build_geometry(p->nx, p->ny, o->leaf_size, o->eta, o->dense_work,
                                    p->kind == ACR_HELMHOLTZ_FEM27);
  std::map<std::tuple<int, int, int>, int> seen;
  for (int f = 0; f < blob->count; ++f) {
    const acr_factor& F = blob->factors[f];
    const std::string where = "factor " + std::to_string(f);
    if (F.level < 0 || F.level > top) throw AcrError(ACR_E_INVALID, where + ": level out of range");
    if (F.role < ACR_FACTOR_DINV || F.role > ACR_FACTOR_C) throw AcrError(ACR_E_INVALID, where + ": unknown role");
    const auto& P = Pl[F.level];
    int pos = -1;
    for (size_t q = 0; q < P.size(); ++q)
      if (P[q] == F.plane) pos = (int)q;
    if (pos < 0) throw AcrError(ACR_E_INVALID, where + ": plane is not in the level's plane list");
    if (F.role == ACR_FACTOR_DINV && pos % 2 != 0) throw AcrError(ACR_E_INVALID, where + ": plane is not eliminated");
    if (F.level == top && F.role != ACR_FACTOR_DINV)
      throw AcrError(ACR_E_INVALID, where + ": the last level holds the top inverse only");
    if (F.role == ACR_FACTOR_DINV && F.diag) throw AcrError(ACR_E_INVALID, where + ": an inverse is an H-matrix");
    if (!F.data || (!F.diag && !F.ranks)) throw AcrError(ACR_E_INVALID, where + ": missing data");
    if (!seen.emplace(std::make_tuple(F.level, F.role, F.plane), f).second)
      throw AcrError(ACR_E_INVALID, where + ": duplicated");
    if (!F.diag)
      for (size_t l = 0; l < G.lf.size(); ++l) {
        const Leaf& L = G.lf[l];
        if (L.fmt == LF_LR && (F.ranks[l] < 0 || F.ranks[l] > std::min(L.m, L.n)))
          throw AcrError(ACR_E_INVALID, where + ": rank out of range in leaf " + std::to_string(l));
      }
  }
  for (int r = 0; r <= top; ++r)
    for (size_t q = 0; q < Pl[r].size(); q += 2)
      if (!seen.count(std::make_tuple(r, (int)ACR_FACTOR_DINV, Pl[r][q])))
        throw AcrError(ACR_E_INVALID, "missing inverse of plane " + std::to_string(Pl[r][q]) + " at level " +
                                          std::to_string(r));
}

// The blob has passed check_factor_blob.
void Handle::import_factors(const acr_problem* p, const acr_factor_blob* blob, hipStream_t s) {
  const auto t_start = std::chrono::steady_clock::now();
  prepare(p, 1, s);
  const auto Pl = plane_lists(nz);
  const int top = (int)Pl.size() - 1;
  std::map<std::tuple<int, int, int>, const acr_factor*> fac;
  for (int f = 0; f < blob->count; ++f) {
    const acr_factor& F = blob->factors[f];
    fac[std::make_tuple(F.level, F.role, F.plane)] = &F;
  }
  // coefficient slots sized by the largest given rank of each leaf
  const size_t nl = G.lf.size();
  for (size_t l = 0; l < nl; ++l) {
    Leaf& L = G.lf[l];
    L.cap = 0;
    if (L.fmt != LF_LR) continue;
    L.cap = 1;
    for (const auto& kv : fac)
      if (!kv.second->diag) L.cap = std::max(L.cap, (int)kv.second->ranks[l]);
  }
  upload_leaf_tables();
  Prob& P = probs[0];
  P.plane_inst.assign(nz, -1);
  auto load = [&](int r, int role, int plane) -> Coupling {
    auto it = fac.find(std::make_tuple(r, role, plane));
    if (it == fac.end()) return Coupling{};
    const acr_factor& F = *it->second;
    if (F.diag) {
      double* d = dnew<double>(B);
      HIPCHK(hipMemcpy(d, F.data, (size_t)B * sizeof(double), hipMemcpyHostToDevice));
      return Coupling{1, -1, d};
    }
    std::vector<int32_t> rk(nl, 0);
    for (size_t l = 0; l < nl; ++l)
      if (G.lf[l].fmt == LF_LR) rk[l] = F.ranks[l];
    return Coupling{2, new_packed_instance(rk, F.data, s), nullptr};
  };
  for (int r = 0; r < top; ++r) {
    Level L;
    L.P = Pl[r];
    for (size_t q = 0; q < L.P.size(); ++q) (q % 2 == 0 ? L.E : L.K).push_back(L.P[q]);
    for (int i : L.E) L.dinv[i] = P.plane_inst[i] = load(r, ACR_FACTOR_DINV, i).inst;
    for (int pl : L.P) {
      L.A[pl] = load(r, ACR_FACTOR_A, pl);
      L.C[pl] = load(r, ACR_FACTOR_C, pl);
    }
    P.levels.push_back(L);
  }
  P.top_plane = Pl[top][0];
  P.top_inst = P.plane_inst[P.top_plane] = load(top, ACR_FACTOR_DINV, P.top_plane).inst;
  level_secs.clear();
  finish(s, t_start);
}

}  // namespace acr
