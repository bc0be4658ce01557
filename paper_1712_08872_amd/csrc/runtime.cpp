// ACR runtime: assembly, level-by-level cyclic reduction with H-matrix
// plane blocks (Sec. 4.1-4.2), preconditioner sweeps and statistics.
//
// Cyclic reduction (Sec. 4.1), level r on the ordered plane list P_r: the
// planes at 1-based odd positions are eliminated (E_r), the others kept
// (K_r).  For i in E_r: Dinv_i = H-inv(D_i) (batched over E_r).  For kept j
// with neighbours j-1, j+1: X = A_j Dinv_{j-1}, Y = C_j Dinv_{j+1},
// D_j <- D_j - X C_{j-1} - Y A_{j+1}, A_j <- -X A_{j-1}, C_j <- -Y C_{j+1}
// (formatted products with truncation, batched over K_r).  At level 0 the
// couplings are the diagonal z-couplings, so X C_{j-1} is a row/column
// scaling of Dinv_{j-1}.  The level-r couplings are stored before they are
// updated; the recursion ends with the H-inverse of the last plane.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>

#include "runtime.h"

namespace acr {

// ------------------------------------------------------------ memory
void* Handle::dmalloc(size_t bytes) {
  if (bytes == 0) bytes = 8;
  void* p = nullptr;
  if (opt.alloc) {
    p = opt.alloc(bytes, opt.alloc_ctx);
    if (!p) throw AcrError(ACR_E_NOMEM, "allocator callback returned NULL");
  } else {
    hipError_t e = hipMalloc(&p, bytes);
    if (e != hipSuccess || !p) {
      (void)hipGetLastError();
      throw AcrError(ACR_E_NOMEM, "hipMalloc of " + std::to_string(bytes) + " bytes failed");
    }
  }
  owned.emplace_back(p, bytes);
  bytes_alloc += bytes;
  return p;
}

void Handle::dfree(void* p) {
  if (!p) return;
  for (size_t i = 0; i < owned.size(); ++i)
    if (owned[i].first == p) {
      bytes_alloc -= owned[i].second;
      owned[i] = owned.back();
      owned.pop_back();
      break;
    }
  if (opt.free)
    opt.free(p, opt.alloc_ctx);
  else
    (void)hipFree(p);
}

Handle::~Handle() {
  if (hres) (void)hipHostFree(hres);
  for (hipEvent_t e : ev_pool) (void)hipEventDestroy(e);
  for (auto& o : owned) {
    if (opt.free)
      opt.free(o.first, opt.alloc_ctx);
    else
      (void)hipFree(o.first);
  }
}

// ------------------------------------------------------------ instances
int Handle::new_instance(hipStream_t s) {
  const size_t esz = fp32 ? 4 : 8;
  const size_t data = (size_t)G.inst_elems * esz;
  const size_t bytes = ((data + 255) / 256) * 256 + G.lf.size() * sizeof(int32_t);
  int id;
  if (!free_inst.empty()) {
    id = free_inst.back();
    free_inst.pop_back();
  } else {
    id = (int)inst.size();
    inst.emplace_back();
    Instance& I = inst[id];
    I.base = dmalloc(bytes);
    I.rank = (int32_t*)((char*)I.base + ((data + 255) / 256) * 256);
    table_dirty = true;
  }
  Instance& I = inst[id];
  I.live = true;
  HIPCHK(hipMemsetAsync(I.base, 0, bytes, s));
  return id;
}

void Handle::release_instance(int id) {
  if (id < 0) return;
  inst[id].live = false;
  free_inst.push_back(id);
}

void Handle::sync_tables() {
  if (!table_dirty) return;
  if ((int)inst.size() > inst_table_cap) {
    if (d_inst_base) dfree(d_inst_base);
    if (d_inst_rank) dfree(d_inst_rank);
    inst_table_cap = std::max<int>(256, (int)inst.size() * 2);
    d_inst_base = dnew<void*>(inst_table_cap);
    d_inst_rank = dnew<int32_t*>(inst_table_cap);
  }
  std::vector<void*> b(inst.size());
  std::vector<int32_t*> r(inst.size());
  for (size_t i = 0; i < inst.size(); ++i) {
    b[i] = inst[i].base;
    r[i] = inst[i].rank;
  }
  HIPCHK(hipMemcpy(d_inst_base, b.data(), b.size() * sizeof(void*), hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(d_inst_rank, r.data(), r.size() * sizeof(int32_t*), hipMemcpyHostToDevice));
  table_dirty = false;
}

// ------------------------------------------------------------ programs
void Handle::upload_program(Program& p) {
  p.d_pieces = upload(p.pieces);
  p.d_targets = upload(p.targets);
  p.d_lists = upload(p.lists);
}

Program& Handle::get_program(const std::string& key) {
  auto it = prog.find(key);
  if (it != prog.end()) return it->second;
  Program P;
  if (key == "inv") {
    P = build_inverse_program(G);
  } else {
    StepBuilder sb(G, P);
    const int root = 0;
    if (key == "copy_schur") {          // D_j -= a_j Dinv_{j-1} c_{j-1} + c_j Dinv_{j+1} a_{j+1}
      sb.copy(1, 0, root, -1.0, 0, 1);
      sb.copy(2, 0, root, -1.0, 2, 3);
      sb.targets(0, root, 1);
    } else if (key == "copy_direct") {  // new coupling = -diag Dinv diag
      sb.copy(1, 0, root, -1.0, 0, 1);
      sb.targets(0, root, 0);
    } else if (key == "mul_new") {      // C = A B
      sb.mul(1, 2, 0, 0, 0, 0, 1.0);
      sb.targets(0, root, 0);
    } else if (key == "mul_neg") {      // C = -A B
      sb.mul(1, 2, 0, 0, 0, 0, -1.0);
      sb.targets(0, root, 0);
    } else if (key == "schur2") {       // D -= X Cp + Y An
      sb.mul(1, 2, 0, 0, 0, 0, -1.0);
      sb.mul(3, 4, 0, 0, 0, 0, -1.0);
      sb.targets(0, root, 1);
    } else {
      throw AcrError(ACR_E_INVALID, "unknown program " + key);
    }
    sb.finish_step();
  }
  upload_program(P);
  auto res = prog.emplace(key, std::move(P));
  return res.first->second;
}

void Handle::run_program(Program& P, int nbatch, int nroles, const std::vector<int32_t>& roles, int nvroles,
                         const std::vector<const double*>& vecs, hipStream_t s) {
  if (nbatch <= 0) return;
  sync_tables();
  // role and vector tables of this run (synchronous copies: the host
  // vectors are rewritten by the next call)
  if ((int)roles.size() > roles_cap) {
    if (d_roles) dfree(d_roles);
    roles_cap = std::max<int>(1024, (int)roles.size() * 2);
    d_roles = dnew<int32_t>(roles_cap);
  }
  HIPCHK(hipStreamSynchronize(s));
  HIPCHK(hipMemcpy(d_roles, roles.data(), roles.size() * sizeof(int32_t), hipMemcpyHostToDevice));
  if (!vecs.empty()) {
    if ((int)vecs.size() > vecs_cap) {
      if (d_vecs) dfree((void*)d_vecs);
      vecs_cap = std::max<int>(1024, (int)vecs.size() * 2);
      d_vecs = dnew<const double*>(vecs_cap);
    }
    HIPCHK(hipMemcpy((void*)d_vecs, vecs.data(), vecs.size() * sizeof(double*), hipMemcpyHostToDevice));
  }
  for (const Step& st : P.steps) {
    if (st.type == 1) {
      const Leaf& L = G.lf[st.leaf];
      if (fp32)
        launch_leaf_inverse<float>((float* const*)d_inst_base, d_roles, nroles, nbatch, L.off, L.m, d_flags, s);
      else
        launch_leaf_inverse<double>((double* const*)d_inst_base, d_roles, nroles, nbatch, L.off, L.m, d_flags, s);
      continue;
    }
    int64_t items = (int64_t)nbatch * st.nt;
    int grid = (int)std::min<int64_t>(items, scratch_slots);
    if (fp32) {
      AccumArgs<float> a{};
      a.leaves = d_leaves;
      a.pieces = P.d_pieces;
      a.targets = P.d_targets;
      a.lists = P.d_lists;
      a.t0 = st.t0;
      a.nt = st.nt;
      a.nbatch = nbatch;
      a.nroles = nroles;
      a.nvroles = nvroles;
      a.role_inst = d_roles;
      a.vec_ptr = d_vecs;
      a.inst_base = (float* const*)d_inst_base;
      a.inst_rank = d_inst_rank;
      a.scratch = (float*)scratch;
      a.scratch_stride = scratch_stride;
      a.eps = opt.eps;
      a.flags = d_flags;
      a.prof = d_prof;
      a.flops = d_flops;
      if (timing) {
        while (ev_pool.size() < ev_used + 2) {
          hipEvent_t e;
          HIPCHK(hipEventCreate(&e));
          ev_pool.push_back(e);
        }
        HIPCHK(hipEventRecord(ev_pool[ev_used], s));
      }
      if (kc == 38)
        kc38::launch_accum<float>(a, grid, s);
      else
        kc64::launch_accum<float>(a, grid, s);
      if (timing) {
        HIPCHK(hipEventRecord(ev_pool[ev_used + 1], s));
        ev_used += 2;
      }
      ++accum_launches;
    } else {
      AccumArgs<double> a{};
      a.leaves = d_leaves;
      a.pieces = P.d_pieces;
      a.targets = P.d_targets;
      a.lists = P.d_lists;
      a.t0 = st.t0;
      a.nt = st.nt;
      a.nbatch = nbatch;
      a.nroles = nroles;
      a.nvroles = nvroles;
      a.role_inst = d_roles;
      a.vec_ptr = d_vecs;
      a.inst_base = (double* const*)d_inst_base;
      a.inst_rank = d_inst_rank;
      a.scratch = (double*)scratch;
      a.scratch_stride = scratch_stride;
      a.eps = opt.eps;
      a.flags = d_flags;
      a.prof = d_prof;
      a.flops = d_flops;
      if (timing) {
        while (ev_pool.size() < ev_used + 2) {
          hipEvent_t e;
          HIPCHK(hipEventCreate(&e));
          ev_pool.push_back(e);
        }
        HIPCHK(hipEventRecord(ev_pool[ev_used], s));
      }
      if (kc == 38)
        kc38::launch_accum<double>(a, grid, s);
      else
        kc64::launch_accum<double>(a, grid, s);
      if (timing) {
        HIPCHK(hipEventRecord(ev_pool[ev_used + 1], s));
        ev_used += 2;
      }
      ++accum_launches;
    }
  }
  HIPCHK(hipGetLastError());
}

// ------------------------------------------------------------ setup
static std::vector<int> initial_caps(const acr_options& o, int depth) {
  int c = o.max_rank;
  if (c <= 0) c = (int)std::lround(6.0 + 6.0 * std::log10(1.0 / o.eps));
  c = std::max(8, std::min(KC_MAX - 8, c));
  return std::vector<int>(depth + 1, c);
}

void Handle::setup(const acr_problem* p, hipStream_t s) {
  auto t_start = std::chrono::steady_clock::now();
  nx = p->nx;
  ny = p->ny;
  nz = p->nz;
  kind = p->kind;
  B = nx * ny;
  N = (int64_t)B * nz;
  beta_amp = p->beta_amp;
  beta_phase = p->beta_phase;
  omega = p->omega;
  fp32 = opt.precision == ACR_MIXED_FP32;
  const int64_t M = (int64_t)(nx + 2) * (ny + 2) * (nz + 2);
  d_flags = dnew<int32_t>(FL_COUNT);
  HIPCHK(hipMemsetAsync(d_flags, 0, FL_COUNT * sizeof(int32_t), s));
  if (const char* e = getenv("ACR_KERNEL_TIMING"); e && e[0] == '1') {
    timing = true;
    d_flops = dnew<double>(1);
    HIPCHK(hipMemsetAsync(d_flops, 0, sizeof(double), s));
  }
  if (const char* e = getenv("ACR_PROFILE"); e && e[0] == '1') {
    d_prof = dnew<unsigned long long>(PS_COUNT);
    HIPCHK(hipMemsetAsync(d_prof, 0, PS_COUNT * sizeof(unsigned long long), s));
  }
  // ---- operator
  S = dnew<double>(7 * N);
  if (kind == ACR_STENCIL7_RAW) {
    HIPCHK(hipMemcpyAsync(S, p->stencil7, 7 * N * sizeof(double), hipMemcpyDeviceToDevice, s));
    launch_check(S, 7 * N, 0, d_flags + FL_NONFINITE, s);
  } else {
    if (p->kappa) {
      kappa = dnew<double>(M);
      HIPCHK(hipMemcpyAsync(kappa, p->kappa, M * sizeof(double), hipMemcpyDeviceToDevice, s));
      launch_check(kappa, M, 1, d_flags + FL_NONFINITE, s);
    }
    if (kind == ACR_HELMHOLTZ) launch_check(p->c, M, 1, d_flags + FL_NONFINITE, s);
    launch_assemble(kind == ACR_CONVDIFF_UPWIND ? 1 : (kind == ACR_HELMHOLTZ ? 2 : 0), nx, ny, nz, kappa, beta_amp,
                    beta_phase, p->c, omega, S, s);
    launch_check(S, 7 * N, 0, d_flags + FL_NONFINITE, s);
  }
  HIPCHK(hipGetLastError());
  int32_t hflags[FL_COUNT];
  HIPCHK(hipMemcpyAsync(hflags, d_flags, sizeof(hflags), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  if (hflags[FL_NONFINITE]) throw AcrError(ACR_E_NUMERIC, "non-finite or non-positive coefficient");

  // ---- geometry and its device tables
  G = build_geometry(nx, ny, opt.leaf_size, opt.eta, opt.dense_work);
  d_perm = upload(G.perm);
  {
    std::vector<int32_t> seg_lo, rp{0}, ri, cp{0}, ci;
    for (int lc : G.leaf_clusters) seg_lo.push_back(G.cl[lc].lo);
    seg_lo.push_back(B);
    for (size_t k = 0; k < G.leaf_clusters.size(); ++k) {
      for (int l : G.rows_of_seg[k]) ri.push_back(l);
      rp.push_back((int32_t)ri.size());
      for (int l : G.cols_of_seg[k]) ci.push_back(l);
      cp.push_back((int32_t)ci.size());
    }
    d_seg_lo = upload(seg_lo);
    d_rows_ptr = upload(rp);
    d_rows_idx = upload(ri);
    d_cols_ptr = upload(cp);
    d_cols_idx = upload(ci);
  }
  zA = dnew<double>(N);
  zC = dnew<double>(N);
  launch_zcoupling(S, N, B, nz, d_perm, zA, zC, s);

  std::vector<int> caps = initial_caps(opt, G.max_depth());
  for (int attempt = 0;; ++attempt) {
    build_factors(s, caps);
    HIPCHK(hipMemcpyAsync(hflags, d_flags, sizeof(hflags), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (hflags[FL_SINGULAR]) throw AcrError(ACR_E_SINGULAR, "exactly singular dense leaf in an H-inverse");
    if (hflags[FL_NONFINITE]) throw AcrError(ACR_E_NUMERIC, "non-finite value during setup");
    int cmax = *std::max_element(caps.begin(), caps.end());
    if (!hflags[FL_RANK_OVERFLOW] || cmax >= KC_MAX - 8 || attempt >= 3) {
      st.max_rank_all = hflags[FL_MAXRANK];
      st.retries = attempt;
      if (hflags[FL_RANK_OVERFLOW]) st.rank_overflow = 1;
      break;
    }
    // rank capacity exhausted: redo with larger capacities
    free_factors();
    if (d_flops) HIPCHK(hipMemsetAsync(d_flops, 0, sizeof(double), s));
    accum_launches = 0;
    ev_used = 0;
    for (auto& c : caps) c = std::min(KC_MAX - 8, std::max(c + 8, (int)(c * 1.5)));
    HIPCHK(hipMemsetAsync(d_flags, 0, FL_COUNT * sizeof(int32_t), s));
  }
  build_apply_jobs();
  HIPCHK(hipStreamSynchronize(s));
  st.setup_seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count();
  compute_stats();
  st.accum_launches = accum_launches;
  if (timing) {
    double ms = 0.0;
    for (size_t i = 0; i + 1 < ev_used; i += 2) {
      float t = 0.f;
      HIPCHK(hipEventElapsedTime(&t, ev_pool[i], ev_pool[i + 1]));
      ms += t;
    }
    st.accum_seconds = ms * 1e-3;
    HIPCHK(hipMemcpy(&st.accum_flops, d_flops, sizeof(double), hipMemcpyDeviceToHost));
    st.setup_flops = st.accum_flops;
  }
  if (d_prof) {
    unsigned long long pc[PS_COUNT];
    HIPCHK(hipMemcpy(pc, d_prof, sizeof(pc), hipMemcpyDeviceToHost));
    const char* names[] = {"pieces_lr", "gram", "eig1", "eig2", "rebuild", "dense", "items", "trunc", "sweeps",
                           "npieces", "ksum"};
    fprintf(stderr, "[acr profile]");
    for (int i = 0; i <= PS_KSUM; ++i) fprintf(stderr, " %s=%.4g", names[i], (double)pc[i]);
    fprintf(stderr, "\n");
  }
}

void Handle::free_factors() {
  levels.clear();
  top_inst = top_plane = -1;
  for (size_t i = 0; i < inst.size(); ++i)
    if (inst[i].live) release_instance((int)i);
}

void Handle::build_factors(hipStream_t s, const std::vector<int>& caps) {
  G.assign_caps(caps);
  // device leaf table (offsets depend on the capacities)
  {
    std::vector<DLeaf> dl(G.lf.size());
    for (size_t i = 0; i < G.lf.size(); ++i) {
      const Leaf& L = G.lf[i];
      dl[i] = DLeaf{L.m, L.n, L.r0, L.c0, L.fmt, L.cap, L.off};
    }
    if (d_leaves) dfree(d_leaves);
    d_leaves = upload(dl);
    std::vector<int32_t> lrl;
    std::vector<int64_t> soff(G.lf.size(), 0);
    int64_t acc = 0;
    for (size_t i = 0; i < G.lf.size(); ++i)
      if (G.lf[i].fmt == LF_LR) {
        lrl.push_back((int32_t)i);
        soff[i] = acc;
        acc += G.lf[i].cap;
      }
    sstride = std::max<int64_t>(acc, 1);
    if (d_lr_leaves) dfree(d_lr_leaves);
    if (d_soff) dfree(d_soff);
    d_lr_leaves = upload(lrl);
    d_soff = upload(soff);
    // level-0 scatter map: in-plane couplings -> dense leaf entries
    std::vector<int64_t> map(5 * (size_t)B, -1);
    std::vector<int> pos(B);
    for (int i = 0; i < B; ++i) pos[G.perm[i]] = i;
    auto find_leaf = [&](int i, int j) {
      int nd = 0;
      while (G.bn[nd].kind == BK_H) {
        const BNode& b = G.bn[nd];
        int ii = i < G.cl[G.cl[b.t].c0].hi ? 0 : 1;
        int jj = j < G.cl[G.cl[b.s].c0].hi ? 0 : 1;
        nd = b.ch[2 * ii + jj];
      }
      return G.bn[nd].leaf;
    };
    const int dxs[5] = {0, -1, 1, 0, 0}, dys[5] = {0, 0, 0, -1, 1};
    for (int y = 0; y < ny; ++y)
      for (int x = 0; x < nx; ++x) {
        int i = pos[x + nx * y];
        for (int d = 0; d < 5; ++d) {
          int xx = x + dxs[d], yy = y + dys[d];
          if (xx < 0 || xx >= nx || yy < 0 || yy >= ny) continue;
          int j = pos[xx + nx * yy];
          int l = find_leaf(i, j);
          const Leaf& L = G.lf[l];
          if (L.fmt != LF_DENSE) throw AcrError(ACR_E_INVALID, "level-0 coupling in a low-rank leaf");
          map[(size_t)d * B + i] = L.off + (i - L.r0) + (int64_t)(j - L.c0) * L.m;
        }
      }
    if (d_l0map) dfree(d_l0map);
    d_l0map = upload(map);
  }
  // programs depend on the leaf formats only; cache across retries
  Program& inv = get_program("inv");
  // accumulation scratch: one slot per resident block
  {
    int mm = std::max(G.max_dense_rows, G.max_lr_dim), nn = std::max(G.max_dense_cols, G.max_lr_dim);
    // narrow rounds (more resident blocks per CU) when every capacity fits
    kc = (*std::max_element(caps.begin(), caps.end()) <= 30) ? 38 : 64;
    int64_t stride = (int64_t)(mm + nn) * kc;
    stride = ((stride + 63) / 64) * 64;
    if (stride > scratch_stride || !scratch) {
      if (scratch) dfree(scratch);
      scratch_slots = 2048;
      scratch_stride = stride;
      scratch = dmalloc((size_t)scratch_slots * stride * (fp32 ? 4 : 8));
    }
  }
  (void)inv;

  // ---- level 0: the plane operators D_k as H-matrices
  plane_inst.assign(nz, -1);
  for (int k = 0; k < nz; ++k) plane_inst[k] = new_instance(s);
  sync_tables();
  {
    int32_t* d_pi = upload(plane_inst);
    if (fp32)
      launch_level0<float>((float* const*)d_inst_base, d_pi, nz, 0, S, N, B, d_perm, d_l0map, s);
    else
      launch_level0<double>((double* const*)d_inst_base, d_pi, nz, 0, S, N, B, d_perm, d_l0map, s);
    HIPCHK(hipStreamSynchronize(s));
    dfree(d_pi);
  }
  std::vector<Coupling> Acur(nz), Ccur(nz);
  for (int k = 0; k < nz; ++k) {
    if (k > 0) Acur[k] = Coupling{1, -1, zA + (int64_t)k * B};
    if (k < nz - 1) Ccur[k] = Coupling{1, -1, zC + (int64_t)k * B};
  }
  // scratch instances of the H-inverse
  std::vector<int> tpool;
  auto inverse_batch = [&](const std::vector<int>& planes) {
    while (tpool.size() < planes.size()) tpool.push_back(new_instance(s));
    std::vector<int32_t> roles;
    for (size_t b = 0; b < planes.size(); ++b) {
      roles.push_back(plane_inst[planes[b]]);
      roles.push_back(tpool[b]);
    }
    run_program(get_program("inv"), (int)planes.size(), 2, roles, 0, {}, s);
  };

  std::vector<int> P(nz);
  for (int k = 0; k < nz; ++k) P[k] = k;
  levels.clear();
  while (true) {
    if (P.size() == 1) {
      inverse_batch(P);
      top_plane = P[0];
      top_inst = plane_inst[P[0]];
      break;
    }
    Level L;
    L.P = P;
    for (size_t q = 0; q < P.size(); ++q) (q % 2 == 0 ? L.E : L.K).push_back(P[q]);
    inverse_batch(L.E);
    for (int i : L.E) L.dinv[i] = plane_inst[i];
    for (int p : P) {
      L.A[p] = Acur[p];
      L.C[p] = Ccur[p];
    }
    const bool diag = levels.empty();
    std::vector<Coupling> An(nz), Cn(nz);
    if (diag) {
      // D_j <- D_j - diag(a_j) Dinv_{j-1} diag(c_{j-1}) - diag(c_j) Dinv_{j+1} diag(a_{j+1})
      std::vector<int32_t> roles;
      std::vector<const double*> vecs;
      std::vector<int32_t> roles2;
      std::vector<const double*> vecs2;
      std::vector<std::pair<int, int>> newc;  // (plane, 0 = A / 1 = C)
      for (size_t m = 0; m < L.K.size(); ++m) {
        const int pos = 2 * (int)m + 1;
        const int j = P[pos], im = P[pos - 1];
        const int ip = pos + 1 < (int)P.size() ? P[pos + 1] : -1;
        roles.push_back(plane_inst[j]);
        roles.push_back(plane_inst[im]);
        roles.push_back(ip >= 0 ? plane_inst[ip] : -1);
        vecs.push_back(Acur[j].diag);
        vecs.push_back(Ccur[im].diag);
        vecs.push_back(ip >= 0 ? Ccur[j].diag : nullptr);
        vecs.push_back(ip >= 0 ? Acur[ip].diag : nullptr);
        if (Acur[im].kind) {  // A_j <- -diag(a_j) Dinv_{j-1} diag(a_{j-1})
          int id = new_instance(s);
          An[j] = Coupling{2, id, nullptr};
          roles2.push_back(id);
          roles2.push_back(plane_inst[im]);
          vecs2.push_back(Acur[j].diag);
          vecs2.push_back(Acur[im].diag);
        }
        if (ip >= 0 && Ccur[ip].kind) {  // C_j <- -diag(c_j) Dinv_{j+1} diag(c_{j+1})
          int id = new_instance(s);
          Cn[j] = Coupling{2, id, nullptr};
          roles2.push_back(id);
          roles2.push_back(plane_inst[ip]);
          vecs2.push_back(Ccur[j].diag);
          vecs2.push_back(Ccur[ip].diag);
        }
      }
      run_program(get_program("copy_schur"), (int)L.K.size(), 3, roles, 4, vecs, s);
      run_program(get_program("copy_direct"), (int)roles2.size() / 2, 2, roles2, 2, vecs2, s);
    } else {
      std::vector<int32_t> rXY, rS, rN;
      std::vector<int> tmp;
      for (size_t m = 0; m < L.K.size(); ++m) {
        const int pos = 2 * (int)m + 1;
        const int j = P[pos], im = P[pos - 1];
        const int ip = pos + 1 < (int)P.size() ? P[pos + 1] : -1;
        const int X = new_instance(s);
        tmp.push_back(X);
        rXY.insert(rXY.end(), {X, Acur[j].inst, plane_inst[im]});
        int Y = -1;
        if (ip >= 0) {
          Y = new_instance(s);
          tmp.push_back(Y);
          rXY.insert(rXY.end(), {Y, Ccur[j].inst, plane_inst[ip]});
        }
        rS.insert(rS.end(), {plane_inst[j], X, Ccur[im].inst, Y, ip >= 0 ? Acur[ip].inst : -1});
        if (Acur[im].kind) {
          int id = new_instance(s);
          An[j] = Coupling{2, id, nullptr};
          rN.insert(rN.end(), {id, X, Acur[im].inst});
        }
        if (ip >= 0 && Ccur[ip].kind) {
          int id = new_instance(s);
          Cn[j] = Coupling{2, id, nullptr};
          rN.insert(rN.end(), {id, Y, Ccur[ip].inst});
        }
      }
      run_program(get_program("mul_new"), (int)rXY.size() / 3, 3, rXY, 0, {}, s);
      run_program(get_program("schur2"), (int)L.K.size(), 5, rS, 0, {}, s);
      run_program(get_program("mul_neg"), (int)rN.size() / 3, 3, rN, 0, {}, s);
      HIPCHK(hipStreamSynchronize(s));
      for (int t : tmp) release_instance(t);
    }
    for (int j : L.K) {
      Acur[j] = An[j];
      Ccur[j] = Cn[j];
    }
    levels.push_back(L);
    P = L.K;
  }
  HIPCHK(hipStreamSynchronize(s));
  for (int t : tpool) release_instance(t);
}

// ------------------------------------------------------------ apply
static MvTerm term_of(const Coupling& c, const double* x, double alpha, int trans) {
  MvTerm t{};
  t.alpha = alpha;
  t.trans = trans;
  t.x = x;
  t.inst = -1;
  t.dvec = nullptr;
  if (c.kind == 1) t.dvec = c.diag;
  if (c.kind == 2) t.inst = c.inst;
  return t;
}

void Handle::build_apply_jobs() {
  for (auto* ph : {&ph_apply, &ph_applyT}) {
    for (auto& p : *ph)
      if (p.d) dfree(p.d);
    ph->clear();
  }
  if (!g) {
    g = dnew<double>(N);
    w = dnew<double>(N);
    z = dnew<double>(N);
  }
  auto V = [&](double* base, int plane) { return base + (int64_t)plane * B; };
  auto push = [&](std::vector<PhaseJobs>& ph, const std::vector<MvJob>& jobs) {
    if (jobs.empty()) return;
    PhaseJobs pj;
    pj.d = upload(jobs);
    pj.n = (int)jobs.size();
    max_jobs = std::max(max_jobs, pj.n);
    ph.push_back(pj);
  };
  const MvTerm none{-1, 0, 0.0, nullptr, nullptr};
  for (int tr = 0; tr < 2; ++tr) {
    std::vector<PhaseJobs>& ph = tr ? ph_applyT : ph_apply;
    // forward elimination
    for (const Level& L : levels) {
      const auto& P = L.P;
      std::vector<MvJob> j1, j2;
      for (int i : L.E) {
        MvJob J{};
        J.y = V(w, i);
        J.base = nullptr;
        J.t[0] = MvTerm{L.dinv.at(i), tr, 1.0, V(g, i), nullptr};
        J.t[1] = none;
        j1.push_back(J);
      }
      for (size_t m = 0; m < L.K.size(); ++m) {
        const int pos = 2 * (int)m + 1;
        const int j = P[pos], im = P[pos - 1];
        const int ip = pos + 1 < (int)P.size() ? P[pos + 1] : -1;
        MvJob J{};
        J.y = V(g, j);
        J.base = V(g, j);
        if (!tr) {
          J.t[0] = term_of(L.A.at(j), V(w, im), -1.0, 0);
          J.t[1] = ip >= 0 ? term_of(L.C.at(j), V(w, ip), -1.0, 0) : none;
        } else {
          J.t[0] = term_of(L.C.at(im), V(w, im), -1.0, 1);
          J.t[1] = ip >= 0 ? term_of(L.A.at(ip), V(w, ip), -1.0, 1) : none;
        }
        j2.push_back(J);
      }
      push(ph, j1);
      push(ph, j2);
    }
    {
      MvJob J{};
      J.y = V(z, top_plane);
      J.base = nullptr;
      J.t[0] = MvTerm{top_inst, tr, 1.0, V(g, top_plane), nullptr};
      J.t[1] = none;
      push(ph, {J});
    }
    // back substitution
    for (auto it = levels.rbegin(); it != levels.rend(); ++it) {
      const Level& L = *it;
      const auto& P = L.P;
      std::vector<MvJob> j3, j4;
      for (size_t m = 0; m < L.E.size(); ++m) {
        const int pos = 2 * (int)m;
        const int i = P[pos];
        const int im = pos > 0 ? P[pos - 1] : -1;
        const int ip = pos + 1 < (int)P.size() ? P[pos + 1] : -1;
        MvJob J{};
        J.y = V(w, i);
        J.base = V(g, i);
        if (!tr) {
          J.t[0] = im >= 0 ? term_of(L.A.at(i), V(z, im), -1.0, 0) : none;
          J.t[1] = ip >= 0 ? term_of(L.C.at(i), V(z, ip), -1.0, 0) : none;
        } else {
          J.t[0] = im >= 0 ? term_of(L.C.at(im), V(z, im), -1.0, 1) : none;
          J.t[1] = ip >= 0 ? term_of(L.A.at(ip), V(z, ip), -1.0, 1) : none;
        }
        j3.push_back(J);
        MvJob K{};
        K.y = V(z, i);
        K.base = nullptr;
        K.t[0] = MvTerm{L.dinv.at(i), tr, 1.0, V(w, i), nullptr};
        K.t[1] = none;
        j4.push_back(K);
      }
      push(ph, j3);
      push(ph, j4);
    }
  }
  if (coef) dfree(coef);
  coef = dnew<double>((size_t)std::max(max_jobs, 1) * 2 * sstride);
}

void Handle::apply(const double* r, double* out, bool transpose, hipStream_t s) {
  sync_tables();
  launch_to_horder(r, g, d_perm, B, N, s);
  const auto& ph = transpose ? ph_applyT : ph_apply;
  for (const PhaseJobs& pj : ph) {
    if (fp32) {
      MvArgs<float> a{};
      a.leaves = d_leaves;
      a.lr_leaves = d_lr_leaves;
      a.soff = d_soff;
      a.nlr = G.nlr;
      a.sstride = sstride;
      a.jobs = pj.d;
      a.njobs = pj.n;
      a.inst_base = (float* const*)d_inst_base;
      a.inst_rank = d_inst_rank;
      a.coef = coef;
      a.seg_lo = d_seg_lo;
      a.rows_ptr = d_rows_ptr;
      a.rows_idx = d_rows_idx;
      a.cols_ptr = d_cols_ptr;
      a.cols_idx = d_cols_idx;
      a.nseg = (int)G.leaf_clusters.size();
      launch_mv<float>(a, s);
    } else {
      MvArgs<double> a{};
      a.leaves = d_leaves;
      a.lr_leaves = d_lr_leaves;
      a.soff = d_soff;
      a.nlr = G.nlr;
      a.sstride = sstride;
      a.jobs = pj.d;
      a.njobs = pj.n;
      a.inst_base = (double* const*)d_inst_base;
      a.inst_rank = d_inst_rank;
      a.coef = coef;
      a.seg_lo = d_seg_lo;
      a.rows_ptr = d_rows_ptr;
      a.rows_idx = d_rows_idx;
      a.cols_ptr = d_cols_ptr;
      a.cols_idx = d_cols_idx;
      a.nseg = (int)G.leaf_clusters.size();
      launch_mv<double>(a, s);
    }
  }
  launch_from_horder(z, out, d_perm, B, N, s);
  HIPCHK(hipGetLastError());
}

void Handle::matvec(const double* x, double* y, bool transpose, hipStream_t s) {
  launch_stencil_mv(S, nx, ny, nz, transpose ? 1 : 0, x, y, s);
  HIPCHK(hipGetLastError());
}

// ------------------------------------------------------------ statistics
double Handle::instance_bytes(int id, const std::vector<int32_t>& rk) const {
  (void)id;
  const double esz = fp32 ? 4.0 : 8.0;
  double b = 0.0;
  for (size_t l = 0; l < G.lf.size(); ++l) {
    const Leaf& L = G.lf[l];
    if (L.fmt == LF_DENSE)
      b += (double)L.m * L.n * esz;
    else
      b += (double)(L.m + L.n) * rk[l] * esz;
  }
  return b;
}

void Handle::compute_stats() {
  acr_stats_t s{};
  s.levels = (int)levels.size() + 1;
  s.nplanes = nz;
  s.plane_points = B;
  s.clusters = (int)G.cl.size();
  s.dense_leaves = G.ndense;
  s.lr_leaves = G.nlr;
  s.precision = opt.precision;
  s.retries = st.retries;
  s.max_rank_all = st.max_rank_all;
  s.rank_overflow = st.rank_overflow;
  s.setup_seconds = st.setup_seconds;
  std::map<int, std::vector<int32_t>> ranks;
  auto get = [&](int id) -> const std::vector<int32_t>& {
    auto it = ranks.find(id);
    if (it != ranks.end()) return it->second;
    std::vector<int32_t> r(G.lf.size());
    HIPCHK(hipMemcpy(r.data(), inst[id].rank, r.size() * sizeof(int32_t), hipMemcpyDeviceToHost));
    return ranks.emplace(id, std::move(r)).first->second;
  };
  double total = 0.0, apply_bytes = 0.0;
  double rank_cnt[ACR_MAX_LEVELS] = {0};
  int nf = 0;
  auto level_of = [&](int r, int id, double weight) {
    const auto& rk = get(id);
    double b = instance_bytes(id, rk);
    total += b;
    apply_bytes += weight * b;
    ++nf;
    int mx = 0;
    double sum = 0;
    int cnt = 0;
    for (size_t l = 0; l < G.lf.size(); ++l)
      if (G.lf[l].fmt == LF_LR) {
        mx = std::max(mx, (int)rk[l]);
        sum += rk[l];
        ++cnt;
      }
    if (r < ACR_MAX_LEVELS) {
      s.max_rank[r] = std::max(s.max_rank[r], mx);
      s.mean_rank[r] += sum;
      rank_cnt[r] += cnt;
    }
  };
  for (size_t r = 0; r < levels.size(); ++r) {
    const Level& L = levels[r];
    for (auto& kv : L.dinv) level_of((int)r, kv.second, 2.0);
    for (int p : L.P) {
      for (const Coupling* c : {&L.A.at(p), &L.C.at(p)}) {
        if (c->kind == 2) level_of((int)r, c->inst, 1.0);
        if (c->kind == 1) apply_bytes += (double)B * 8.0;
      }
    }
  }
  level_of((int)levels.size(), top_inst, 1.0);
  for (int r = 0; r < ACR_MAX_LEVELS; ++r)
    if (rank_cnt[r] > 0) s.mean_rank[r] /= rank_cnt[r];
  // vectors: every job reads its inputs and writes its output plane
  apply_bytes += 2.0 * (double)N * 8.0 * 2.0 * (double)levels.size() + 2.0 * (double)N * 8.0;
  s.factors = nf;
  s.bytes_factors = total;
  s.bytes_allocated = (double)bytes_alloc;
  s.bytes_per_apply = apply_bytes;
  st = s;
}

}  // namespace acr
