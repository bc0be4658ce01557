// Cyclic reduction with H-matrix plane blocks (Sec. 4.1-4.2): setup of one
// group of problems, the preconditioner sweeps and statistics.
//
// Level r on the ordered plane list P_r: the planes at 1-based odd positions
// are eliminated (E_r), the others kept (K_r).  For i in E_r:
// Dinv_i = H-inv(D_i).  For kept j with neighbours j-1, j+1:
// X = A_j Dinv_{j-1}, Y = C_j Dinv_{j+1}, D_j <- D_j - X C_{j-1} - Y A_{j+1},
// A_j <- -X A_{j-1}, C_j <- -Y C_{j+1} (formatted products with truncation).
// At level 0 the couplings are the diagonal z-couplings, so X C_{j-1} is a
// row/column scaling of Dinv_{j-1}.  The level-r couplings are stored before
// they are updated; the recursion ends with the H-inverse of the last plane.
//
// All problems of a group have the same plane shape and plane count, so
// their levels coincide and every step is one batched launch over all
// planes of all problems.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>

#include "runtime.h"

namespace acr {

static std::vector<int> initial_caps(const acr_options& o, int depth) {
  // a caller-given max_rank is the cap itself; the automatic capacity is
  // 6 + 6 log10(1/eps), at least 8
  int c = o.max_rank;
  if (c <= 0) c = std::max(8, (int)std::lround(6.0 + 6.0 * std::log10(1.0 / o.eps)));
  c = std::max(1, std::min(KC_MAX - 8, c));
  return std::vector<int>(depth + 1, c);
}

void Handle::setup(const acr_problem* ps, int count, hipStream_t s) {
  auto t_start = std::chrono::steady_clock::now();
  prepare(ps, count, s);
  int32_t hflags[FL_COUNT];
  std::vector<int> caps = initial_caps(opt, G.max_depth());
  for (int attempt = 0;; ++attempt) {
    build_factors(s, caps);
    HIPCHK(hipMemcpyAsync(hflags, d_flags, sizeof(hflags), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (hflags[FL_SINGULAR]) throw AcrError(ACR_E_SINGULAR, "exactly singular dense leaf in an H-inverse");
    if (hflags[FL_NONFINITE]) throw AcrError(ACR_E_NUMERIC, "non-finite value during setup");
    if (hflags[FL_LAYOUT]) throw AcrError(ACR_E_DEVICE, "internal: packed instance used as a target");
    int cmax = *std::max_element(caps.begin(), caps.end());
    // a caller-given max_rank is a fixed cap: ranks are clamped to it and
    // the overflow is reported, not retried
    if (!hflags[FL_RANK_OVERFLOW] || opt.max_rank > 0 || cmax >= KC_MAX - 8 || attempt >= 3) {
      st.max_rank_all = hflags[FL_MAXRANK];
      st.retries = attempt;
      if (hflags[FL_RANK_OVERFLOW]) st.rank_overflow = 1;
      break;
    }
    // rank capacity exhausted: redo with larger capacities (the pooled
    // capacity buffers have the old layout)
    free_factors();
    HIPCHK(hipStreamSynchronize(s));
    for (void* b : cap_pool) dfree(b);
    cap_pool.clear();
    if (d_flops) HIPCHK(hipMemsetAsync(d_flops, 0, 2 * (FC_COUNT + 1) * sizeof(double), s));
    leaf_inverse_flops = 0.0;
    accum_launches = dense_launches = 0;
    ev_used = 0;
    ev_tag.clear();
    for (auto& c : caps) c = std::min(KC_MAX - 8, std::max(c + 8, (int)(c * 1.5)));
    HIPCHK(hipMemsetAsync(d_flags, 0, FL_COUNT * sizeof(int32_t), s));
  }
  finish(s, t_start);
}

// Operators of every problem (assembly and checks), the plane geometry with
// its segment tables, and the level-0 z-couplings.
void Handle::prepare(const acr_problem* ps, int count, hipStream_t s) {
  nx = ps[0].nx;
  ny = ps[0].ny;
  nz = ps[0].nz;
  B = nx * ny;
  N = (int64_t)B * nz;
  fp32 = opt.precision == ACR_MIXED_FP32 || opt.precision == ACR_MIXED_BF16;
  bf16 = opt.precision == ACR_MIXED_BF16;
  fem27 = ps[0].kind == ACR_HELMHOLTZ_FEM27;
  const int64_t M = (int64_t)(nx + 2) * (ny + 2) * (nz + 2);
  d_flags = dnew<int32_t>(FL_COUNT);
  HIPCHK(hipMemsetAsync(d_flags, 0, FL_COUNT * sizeof(int32_t), s));
  if (const char* e = getenv("ACR_KERNEL_TIMING"); e && e[0] == '1') {
    timing = true;
    d_flops = dnew<double>(2 * (FC_COUNT + 1));
    HIPCHK(hipMemsetAsync(d_flops, 0, 2 * (FC_COUNT + 1) * sizeof(double), s));
  }
  if (const char* e = getenv("ACR_PROFILE"); e && e[0] == '1') {
    d_prof = dnew<unsigned long long>(PS_COUNT);
    HIPCHK(hipMemsetAsync(d_prof, 0, PS_COUNT * sizeof(unsigned long long), s));
  }
  // ---- operators
  probs.assign(count, Prob{});
  for (int q = 0; q < count; ++q) {
    const acr_problem* p = ps + q;
    Prob& P = probs[q];
    P.kind = p->kind;
    P.beta_amp = p->beta_amp;
    P.beta_phase = p->beta_phase;
    P.omega = p->omega;
    P.S = dnew<double>((size_t)nst() * N);
    if (P.kind == ACR_STENCIL7_RAW) {
      HIPCHK(hipMemcpyAsync(P.S, p->stencil7, 7 * N * sizeof(double), hipMemcpyDeviceToDevice, s));
      launch_check(P.S, 7 * N, 0, d_flags + FL_NONFINITE, s);
    } else if (P.kind == ACR_HELMHOLTZ_FEM27) {
      launch_check(p->c, M, 1, d_flags + FL_NONFINITE, s);
      launch_assemble27(nx, ny, nz, p->c, P.omega, P.S, s);
      launch_check(P.S, 27 * N, 0, d_flags + FL_NONFINITE, s);
    } else {
      if (p->kappa) {
        P.kappa = dnew<double>(M);
        HIPCHK(hipMemcpyAsync(P.kappa, p->kappa, M * sizeof(double), hipMemcpyDeviceToDevice, s));
        launch_check(P.kappa, M, 1, d_flags + FL_NONFINITE, s);
      }
      if (P.kind == ACR_HELMHOLTZ) launch_check(p->c, M, 1, d_flags + FL_NONFINITE, s);
      launch_assemble(P.kind == ACR_CONVDIFF_UPWIND ? 1 : P.kind == ACR_HELMHOLTZ ? 2 : P.kind == ACR_CONVDIFF_RECIRC ? 3 : 0,
                      nx, ny, nz, P.kappa,
                      P.beta_amp, P.beta_phase, p->c, P.omega, P.S, s);
      launch_check(P.S, 7 * N, 0, d_flags + FL_NONFINITE, s);
    }
  }
  HIPCHK(hipGetLastError());
  int32_t hflags[FL_COUNT];
  HIPCHK(hipMemcpyAsync(hflags, d_flags, sizeof(hflags), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  if (hflags[FL_NONFINITE]) throw AcrError(ACR_E_NUMERIC, "non-finite or non-positive coefficient");

  // ---- geometry and its device tables
  G = build_geometry(nx, ny, opt.leaf_size, opt.eta, opt.dense_work, fem27);
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
  if (!fem27)
    for (Prob& P : probs) {
      P.zA = dnew<double>(N);
      P.zC = dnew<double>(N);
      launch_zcoupling(P.S, N, B, nz, d_perm, P.zA, P.zC, s);
    }
}

// After the factors exist: release the setup's working memory, build and
// tune the apply phases, and gather statistics.
void Handle::finish(hipStream_t s, std::chrono::steady_clock::time_point t_start) {
  // working memory of the setup: recycled capacity buffers and the
  // accumulation scratch
  HIPCHK(hipStreamSynchronize(s));
  for (void* b : cap_pool) dfree(b);
  cap_pool.clear();
  for (Lane& ln : lanes) {
    if (ln.scratch) dfree(ln.scratch);
    if (ln.dbuf) dfree(ln.dbuf);
    ln.scratch = ln.dbuf = nullptr;
    ln.dbuf_bytes = 0;
  }
  scratch_stride = 0;
  const bool log = [] {
    const char* e = getenv("ACR_LOG");
    return e && e[0] == '1';
  }();
  auto t_mark = std::chrono::steady_clock::now();
  auto mark = [&](const char* what) {
    if (!log) return;
    HIPCHK(hipStreamSynchronize(s));
    const auto now = std::chrono::steady_clock::now();
    fprintf(stderr, "[acr] %s: %.3f s\n", what, std::chrono::duration<double>(now - t_mark).count());
    fflush(stderr);
    t_mark = now;
  };
  build_apply_jobs();
  mark("apply jobs");
  build_apply_image(s);
  mark("apply images");
  tune_apply(s);
  HIPCHK(hipStreamSynchronize(s));
  mark("apply tuning");
  const int retries = st.retries, overflow = st.rank_overflow, maxr = st.max_rank_all;
  compute_stats();
  mark("statistics");
  st.retries = retries;
  st.rank_overflow = overflow;
  st.max_rank_all = std::max(st.max_rank_all, maxr);  // the largest rank produced, stored or not
  st.setup_seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count();
  st.accum_launches = accum_launches;
  st.dense_launches = dense_launches;
  st.leaf_inverse_flops = leaf_inverse_flops;
  for (size_t r = 0; r < level_secs.size() && r < (size_t)ACR_MAX_LEVELS; ++r) st.level_seconds[r] = level_secs[r];
  if (timing) {
    double ms = 0.0, msd = 0.0;
    for (size_t i = 0; i + 1 < ev_used; i += 2) {
      float t = 0.f;
      HIPCHK(hipEventElapsedTime(&t, ev_pool[i], ev_pool[i + 1]));
      const bool dense = i / 2 < ev_tag.size() && ev_tag[i / 2].kernel[0] != '\0';
      (dense ? msd : ms) += t;
    }
    st.accum_seconds = ms * 1e-3;
    st.dense_seconds = msd * 1e-3;
    if (const char* path = getenv("ACR_TIMING_LOG"); path && path[0]) {
      // one line per accumulation launch: program, CR level, step, batch, targets, widest target, ms
      if (FILE* f = fopen(path, "w")) {
        fprintf(f, "prog,kernel,level,step,nbatch,nt,max_m,ms\n");
        for (size_t i = 0; i + 1 < ev_used && i / 2 < ev_tag.size(); i += 2) {
          float t = 0.f;
          HIPCHK(hipEventElapsedTime(&t, ev_pool[i], ev_pool[i + 1]));
          const LaunchTag& g = ev_tag[i / 2];
          fprintf(f, "%s,%s,%d,%d,%d,%d,%d,%.4f\n", g.prog, g.kernel, g.level, g.step, g.nbatch, g.nt, g.max_m, t);
        }
        fclose(f);
      }
    }
    // [kernel][flops by class, bytes]: the truncating kernel, then the accumulate-only one
    constexpr int W = FC_COUNT + 1;
    double fl[2 * W] = {0.0};
    HIPCHK(hipMemcpy(fl, d_flops, sizeof(fl), hipMemcpyDeviceToHost));
    st.accum_flops = st.dense_flops = 0.0;
    for (int c = 0; c < FC_COUNT; ++c) {
      st.accum_flops += fl[c];
      st.dense_flops += fl[W + c];
      st.setup_flops_class[c] = fl[c] + fl[W + c];
    }
    st.accum_bytes = fl[FC_COUNT];
    st.dense_bytes = fl[W + FC_COUNT];
    st.setup_flops = st.accum_flops + st.dense_flops + leaf_inverse_flops;
  }
  if (d_prof) {
    unsigned long long pc[PS_COUNT];
    HIPCHK(hipMemcpy(pc, d_prof, sizeof(pc), hipMemcpyDeviceToHost));
    const char* names[] = {"pieces_lr", "gram", "eig1", "eig2", "rebuild", "dense", "items", "trunc", "sweeps",
                           "npieces", "ksum", "dacc", "lrx", "lry", "dd", "outer", "tn", "nn"};
    fprintf(stderr, "[acr profile]");
    for (int i = 0; i < PS_COUNT; ++i) fprintf(stderr, " %s=%.4g", names[i], (double)pc[i]);
    fprintf(stderr, "\n");
  }
}

void Handle::free_factors() {
  for (Prob& P : probs) {
    P.levels.clear();
    P.top_inst = P.top_plane = -1;
    P.plane_inst.clear();
  }
  for (size_t i = 0; i < inst.size(); ++i)
    if (inst[i].live) release_instance((int)i);
}

// Device leaf table, coefficient slots and the coefficient kernel's leaf
// classes, from the leaves' current capacities.
void Handle::upload_leaf_tables() {
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
  if (d_soff) dfree(d_soff);
  d_soff = upload(soff);
  // coefficient kernel order: low-rank leaves by the lane-group class of
  // the factor length it reduces over (n for V^T x, m for U^T x)
  auto by_class = [&](bool use_m, int32_t*& dst, int32_t* cls, int32_t (*cw)[6], int32_t& w4) {
    // elements per lane of the coefficient kernel: 4 (FP64 factors) or 8 (FP32)
    const int e = fp32 ? 8 : 4;
    auto cl = [e](int len) {
      return len <= 4 * e ? 0 : len <= 8 * e ? 1 : len <= 16 * e ? 2 : len <= 32 * e ? 3 : 4;
    };
    std::vector<int32_t> v(lrl);
    std::stable_sort(v.begin(), v.end(), [&](int a, int b) {
      return cl(use_m ? G.lf[a].m : G.lf[a].n) < cl(use_m ? G.lf[b].m : G.lf[b].n);
    });
    int cnt[5] = {0, 0, 0, 0, 0};
    int cap4 = 1;
    for (int l : v) {
      const int c = cl(use_m ? G.lf[l].m : G.lf[l].n);
      cnt[c]++;
      if (c == 4) cap4 = std::max(cap4, G.lf[l].cap);
    }
    // the longest leaves: one wavefront per 4 columns of a leaf
    w4 = (cap4 + 3) / 4;
    cls[0] = 0;
    cw[0][0] = cw[1][0] = 0;
    for (int c = 0; c < 5; ++c) {
      cls[c + 1] = cls[c] + cnt[c];
      for (int ri = 0; ri < 2; ++ri) {
        const int per_wave = (ri ? 4 : 1) * (64 >> (c + 2));  // rounds of 64 / G leaves
        cw[ri][c + 1] = cw[ri][c] + (c < 4 ? (cnt[c] + per_wave - 1) / per_wave : cnt[c] * w4);
      }
    }
    if (dst) dfree(dst);
    dst = upload(v);
  };
  by_class(false, d_lr_n, cls_n, cw_n, w4_n);
  by_class(true, d_lr_t, cls_t, cw_t, w4_t);
}

void Handle::build_factors(hipStream_t s, const std::vector<int>& caps) {
  G.assign_caps(caps);
  upload_leaf_tables();
  {
    // level-0 scatter map: in-plane couplings -> dense leaf entries
    std::vector<int64_t> map;
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
    // in-plane offsets of the scatter map: the 5-point star (centre, x-1,
    // x+1, y-1, y+1: stencil rows 0..4) or all 9 offsets d = (dx+1) + 3 (dy+1)
    // of the 27-point operator
    const int nd = fem27 ? 9 : 5;
    int dxs[9], dys[9];
    for (int d = 0; d < nd; ++d) {
      const int sx5[5] = {0, -1, 1, 0, 0}, sy5[5] = {0, 0, 0, -1, 1};
      dxs[d] = fem27 ? d % 3 - 1 : sx5[d];
      dys[d] = fem27 ? d / 3 - 1 : sy5[d];
    }
    map.assign((size_t)nd * B, -1);
    for (int y = 0; y < ny; ++y)
      for (int x = 0; x < nx; ++x) {
        int i = pos[x + nx * y];
        for (int d = 0; d < nd; ++d) {
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
  get_program("inv");
  // accumulation scratch: one slot per resident block
  {
    int mm = std::max(G.max_dense_rows, G.max_lr_dim), nn = std::max(G.max_dense_cols, G.max_lr_dim);
    // narrow rounds (more resident blocks per CU) when every capacity fits
    kc = (*std::max_element(caps.begin(), caps.end()) <= 30) ? 38 : 64;
    int64_t stride = (int64_t)(mm + nn) * kc + DACC_ELEMS;  // + dense accumulator of small low-rank targets
    stride = ((stride + 63) / 64) * 64;
    if (stride > scratch_stride) {
      for (Lane& ln : lanes)
        if (ln.scratch) {
          dfree(ln.scratch);
          ln.scratch = nullptr;
        }
      scratch_slots = 2048;
      scratch_stride = stride;
    }
    // two regions per lane: its main stream's and its second stream's launches
    ensure_lane(lanes[0], s);
  }

  // ---- level 0: the plane operators D_k as H-matrices
  const int np = (int)probs.size();
  for (Prob& P : probs) {
    P.plane_inst.assign(nz, -1);
    for (int k = 0; k < nz; ++k) P.plane_inst[k] = new_instance(s);
  }
  sync_tables();
  // stencil rows of the in-plane entries of the scatter map: D (dz = 0), and
  // for the 27-point operator also A (dz = -1) and C (dz = +1)
  auto l0rows = [&](int dz) {
    L0Rows r{};
    r.nd = fem27 ? 9 : 5;
    for (int d = 0; d < r.nd; ++d) r.row[d] = fem27 ? d + 9 * (dz + 1) : d;
    return r;
  };
  auto fill = [&](const Prob& P, const std::vector<int>& ids, int plane0, int dz) {
    int32_t* d_ids = upload(std::vector<int32_t>(ids.begin(), ids.end()));
    sync_tables();
    if (fp32)
      launch_level0<float>((float* const*)d_inst_base, d_ids, (int)ids.size(), plane0, P.S, N, B, d_perm, d_l0map,
                           l0rows(dz), s);
    else
      launch_level0<double>((double* const*)d_inst_base, d_ids, (int)ids.size(), plane0, P.S, N, B, d_perm,
                            d_l0map, l0rows(dz), s);
    HIPCHK(hipStreamSynchronize(s));
    dfree(d_ids);
  };
  for (Prob& P : probs) fill(P, P.plane_inst, 0, 0);
  std::vector<std::vector<Coupling>> Acur(np, std::vector<Coupling>(nz)), Ccur(np, std::vector<Coupling>(nz));
  if (!fem27) {
    for (int q = 0; q < np; ++q)
      for (int k = 0; k < nz; ++k) {
        if (k > 0) Acur[q][k] = Coupling{1, -1, probs[q].zA + (int64_t)k * B};
        if (k < nz - 1) Ccur[q][k] = Coupling{1, -1, probs[q].zC + (int64_t)k * B};
      }
  } else {
    // the 9-point z-coupling planes as H-matrices (exact: their entries lie in
    // dense leaves), final at once: built and packed a chunk at a time so that
    // only a few capacity buffers are live
    constexpr int kChunk = 16;
    for (int q = 0; q < np; ++q)
      for (int dz : {-1, 1}) {
        const int k0 = dz < 0 ? 1 : 0, k1 = dz < 0 ? nz : nz - 1;
        for (int c0 = k0; c0 < k1; c0 += kChunk) {
          std::vector<int> ids;
          for (int k = c0; k < std::min(k1, c0 + kChunk); ++k) ids.push_back(new_instance(s));
          fill(probs[q], ids, c0, dz);
          pack_instances(ids, s);
          for (size_t t = 0; t < ids.size(); ++t)
            (dz < 0 ? Acur : Ccur)[q][c0 + (int)t] = Coupling{2, ids[t], nullptr};
        }
      }
  }
  // H-inverse of the given planes of every problem, in place, with scratch
  // instances released right after; the inverses are final and get packed
  auto inverse_batch = [&](const std::vector<int>& planes) {
    const size_t nb = planes.size() * np;
    std::vector<int> tpool;
    while (tpool.size() < nb) tpool.push_back(new_instance(s));
    std::vector<int32_t> roles;
    std::vector<int> done;
    size_t b = 0;
    for (int q = 0; q < np; ++q)
      for (int pl : planes) {
        roles.push_back(probs[q].plane_inst[pl]);
        roles.push_back(tpool[b++]);
        done.push_back(probs[q].plane_inst[pl]);
      }
    run_program(get_program("inv"), (int)nb, 2, roles, 0, {}, lanes[0]);
    for (int t : tpool) release_instance(t);
    pack_instances(done, s);
  };
  // couplings created by this level are final once written
  auto pack_new_couplings = [&](const std::vector<std::vector<Coupling>>& An,
                                const std::vector<std::vector<Coupling>>& Cn) {
    std::vector<int> ids;
    for (int q = 0; q < np; ++q)
      for (int k = 0; k < nz; ++k) {
        if (An[q][k].kind == 2) ids.push_back(An[q][k].inst);
        if (Cn[q][k].kind == 2) ids.push_back(Cn[q][k].inst);
      }
    pack_instances(ids, s);
  };

  // the previous level's new couplings still being formed on lane 1
  struct Pending {
    bool on = false;
    std::vector<int> tmp;
    std::vector<std::vector<Coupling>> An, Cn;
  } pend;
  auto join_pending = [&] {
    if (!pend.on) return;
    HIPCHK(hipStreamSynchronize(lanes[1].s));
    for (int t : pend.tmp) release_instance(t);
    pack_new_couplings(pend.An, pend.Cn);
    pend = Pending{};
  };
  if (!ev_products) HIPCHK(hipEventCreateWithFlags(&ev_products, hipEventDisableTiming));

  std::vector<int> P(nz);
  for (int k = 0; k < nz; ++k) P[k] = k;
  int lev = 0;
  const bool log = [] {
    const char* e = getenv("ACR_LOG");
    return e && e[0] == '1';
  }();
  const auto t_lev0 = std::chrono::steady_clock::now();
  level_secs.clear();
  auto t_mark = t_lev0;
  auto mark_level = [&] {
    HIPCHK(hipStreamSynchronize(s));
    const auto now = std::chrono::steady_clock::now();
    level_secs.push_back(std::chrono::duration<double>(now - t_mark).count());
    t_mark = now;
  };
  while (true) {
    cur_level = lev;
    if (lev > 0) mark_level();
    if (log) {
      HIPCHK(hipStreamSynchronize(s));
      fprintf(stderr, "[acr] level %d: %zu planes, %.2f s, %.2f GB held (peak %.2f GB)\n", lev, P.size(),
              std::chrono::duration<double>(std::chrono::steady_clock::now() - t_lev0).count(), bytes_alloc * 1e-9,
              bytes_peak * 1e-9);
      fflush(stderr);
    }
    if (P.size() == 1) {
      inverse_batch(P);
      for (Prob& pr : probs) {
        pr.top_plane = P[0];
        pr.top_inst = pr.plane_inst[P[0]];
      }
      mark_level();
      break;
    }
    Level L;
    L.P = P;
    for (size_t q = 0; q < P.size(); ++q) (q % 2 == 0 ? L.E : L.K).push_back(P[q]);
    inverse_batch(L.E);
    std::vector<std::vector<Coupling>> An(np, std::vector<Coupling>(nz)), Cn(np, std::vector<Coupling>(nz));
    for (int q = 0; q < np; ++q) {
      Level Lq = L;
      for (int i : L.E) Lq.dinv[i] = probs[q].plane_inst[i];
      for (int p : P) {
        Lq.A[p] = Acur[q][p];
        Lq.C[p] = Ccur[q][p];
      }
      probs[q].levels.push_back(Lq);
    }
    if (lev == 0 && !fem27) {
      // D_j <- D_j - diag(a_j) Dinv_{j-1} diag(c_{j-1}) - diag(c_j) Dinv_{j+1} diag(a_{j+1})
      std::vector<int32_t> roles, roles2;
      std::vector<const double*> vecs, vecs2;
      for (int q = 0; q < np; ++q) {
        const auto& pi = probs[q].plane_inst;
        for (size_t m = 0; m < L.K.size(); ++m) {
          const int pos = 2 * (int)m + 1;
          const int j = P[pos], im = P[pos - 1];
          const int ip = pos + 1 < (int)P.size() ? P[pos + 1] : -1;
          roles.push_back(pi[j]);
          roles.push_back(pi[im]);
          roles.push_back(ip >= 0 ? pi[ip] : -1);
          vecs.push_back(Acur[q][j].diag);
          vecs.push_back(Ccur[q][im].diag);
          vecs.push_back(ip >= 0 ? Ccur[q][j].diag : nullptr);
          vecs.push_back(ip >= 0 ? Acur[q][ip].diag : nullptr);
          if (Acur[q][im].kind) {  // A_j <- -diag(a_j) Dinv_{j-1} diag(a_{j-1})
            int id = new_instance(s);
            An[q][j] = Coupling{2, id, nullptr};
            roles2.push_back(id);
            roles2.push_back(pi[im]);
            vecs2.push_back(Acur[q][j].diag);
            vecs2.push_back(Acur[q][im].diag);
          }
          if (ip >= 0 && Ccur[q][ip].kind) {  // C_j <- -diag(c_j) Dinv_{j+1} diag(c_{j+1})
            int id = new_instance(s);
            Cn[q][j] = Coupling{2, id, nullptr};
            roles2.push_back(id);
            roles2.push_back(pi[ip]);
            vecs2.push_back(Ccur[q][j].diag);
            vecs2.push_back(Ccur[q][ip].diag);
          }
        }
      }
      run_program(get_program("copy_schur"), (int)roles.size() / 3, 3, roles, 4, vecs, lanes[0]);
      run_program(get_program("copy_direct"), (int)roles2.size() / 2, 2, roles2, 2, vecs2, lanes[0]);
      pack_new_couplings(An, Cn);
    } else {
      join_pending();  // this level's products read the couplings made by the previous one
      std::vector<int32_t> rXY, rS, rN;
      std::vector<int> tmp;
      for (int q = 0; q < np; ++q) {
        const auto& pi = probs[q].plane_inst;
        for (size_t m = 0; m < L.K.size(); ++m) {
          const int pos = 2 * (int)m + 1;
          const int j = P[pos], im = P[pos - 1];
          const int ip = pos + 1 < (int)P.size() ? P[pos + 1] : -1;
          const int X = new_instance(s);
          tmp.push_back(X);
          rXY.insert(rXY.end(), {X, Acur[q][j].inst, pi[im]});
          int Y = -1;
          if (ip >= 0) {
            Y = new_instance(s);
            tmp.push_back(Y);
            rXY.insert(rXY.end(), {Y, Ccur[q][j].inst, pi[ip]});
          }
          rS.insert(rS.end(), {pi[j], X, Ccur[q][im].inst, Y, ip >= 0 ? Acur[q][ip].inst : -1});
          if (Acur[q][im].kind) {
            int id = new_instance(s);
            An[q][j] = Coupling{2, id, nullptr};
            rN.insert(rN.end(), {id, X, Acur[q][im].inst});
          }
          if (ip >= 0 && Ccur[q][ip].kind) {
            int id = new_instance(s);
            Cn[q][j] = Coupling{2, id, nullptr};
            rN.insert(rN.end(), {id, Y, Ccur[q][ip].inst});
          }
        }
      }
      run_program(get_program("mul_new"), (int)rXY.size() / 3, 3, rXY, 0, {}, lanes[0]);
      HIPCHK(hipEventRecord(ev_products, s));
      run_program(get_program("schur2"), (int)rS.size() / 5, 5, rS, 0, {}, lanes[0]);
      // the new couplings are needed only by the next level's products: they
      // run on lane 1 while lane 0 goes on with the Schur updates and the
      // next level's inverses; X and Y are released and the couplings packed
      // when the next level joins them
      ensure_lane(lanes[1], s);
      HIPCHK(hipStreamWaitEvent(lanes[1].s, ev_products, 0));
      run_program(get_program("mul_neg"), (int)rN.size() / 3, 3, rN, 0, {}, lanes[1]);
      pend.on = true;
      pend.tmp = tmp;
      pend.An = An;
      pend.Cn = Cn;
    }
    for (int q = 0; q < np; ++q)
      for (int j : L.K) {
        Acur[q][j] = An[q][j];
        Ccur[q][j] = Cn[q][j];
      }
    P = L.K;
    ++lev;
  }
  join_pending();
  HIPCHK(hipStreamSynchronize(s));
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
  auto clear = [&](std::vector<PhaseJobs>& ph) {
    for (auto& p : ph) {
      if (p.d) dfree(p.d);
      if (p.terms) dfree(p.terms);
    }
    ph.clear();
  };
  clear(ph_apply);
  clear(ph_applyT);
  for (Prob& P : probs) {
    clear(P.ph_apply);
    clear(P.ph_applyT);
  }
  const int np = (int)probs.size();
  if (!g) {
    g = dnew<double>((size_t)N * np);
    w = dnew<double>((size_t)N * np);
    z = dnew<double>((size_t)N * np);
  }
  auto V = [&](double* base, int q, int plane) { return base + (int64_t)q * N + (int64_t)plane * B; };
  const MvTerm none{-1, 0, 0.0, nullptr, nullptr};
  max_jobs = 0;
  // phases of problem q (q < 0: all problems concatenated per phase)
  auto build = [&](int qsel, int tr, std::vector<PhaseJobs>& out) {
    std::vector<std::vector<MvJob>> phases;
    const Prob& P0 = probs[0];
    const int nlev = (int)P0.levels.size();
    auto add = [&](size_t ph, const MvJob& J) {
      if (phases.size() <= ph) phases.resize(ph + 1);
      phases[ph].push_back(J);
    };
    for (int q = 0; q < np; ++q) {
      if (qsel >= 0 && q != qsel) continue;
      const Prob& pr = probs[q];
      size_t ph = 0;
      for (int r = 0; r < nlev; ++r, ph += 2) {  // forward elimination
        const Level& L = pr.levels[r];
        const auto& Pl = L.P;
        for (int i : L.E) {
          MvJob J{};
          J.y = V(w, q, i);
          J.base = nullptr;
          J.t[0] = MvTerm{L.dinv.at(i), tr, 1.0, V(g, q, i), nullptr};
          J.t[1] = none;
          add(ph, J);
        }
        for (size_t m = 0; m < L.K.size(); ++m) {
          const int pos = 2 * (int)m + 1;
          const int j = Pl[pos], im = Pl[pos - 1];
          const int ip = pos + 1 < (int)Pl.size() ? Pl[pos + 1] : -1;
          MvJob J{};
          J.y = V(g, q, j);
          J.base = V(g, q, j);
          if (!tr) {
            J.t[0] = term_of(L.A.at(j), V(w, q, im), -1.0, 0);
            J.t[1] = ip >= 0 ? term_of(L.C.at(j), V(w, q, ip), -1.0, 0) : none;
          } else {
            J.t[0] = term_of(L.C.at(im), V(w, q, im), -1.0, 1);
            J.t[1] = ip >= 0 ? term_of(L.A.at(ip), V(w, q, ip), -1.0, 1) : none;
          }
          add(ph + 1, J);
        }
      }
      {  // top plane
        MvJob J{};
        J.y = V(z, q, pr.top_plane);
        J.base = nullptr;
        J.t[0] = MvTerm{pr.top_inst, tr, 1.0, V(g, q, pr.top_plane), nullptr};
        J.t[1] = none;
        add(ph, J);
        ph += 1;
      }
      for (int r = nlev - 1; r >= 0; --r, ph += 2) {  // back substitution
        const Level& L = pr.levels[r];
        const auto& Pl = L.P;
        for (size_t m = 0; m < L.E.size(); ++m) {
          const int pos = 2 * (int)m;
          const int i = Pl[pos];
          const int im = pos > 0 ? Pl[pos - 1] : -1;
          const int ip = pos + 1 < (int)Pl.size() ? Pl[pos + 1] : -1;
          MvJob J{};
          J.y = V(w, q, i);
          J.base = V(g, q, i);
          if (!tr) {
            J.t[0] = im >= 0 ? term_of(L.A.at(i), V(z, q, im), -1.0, 0) : none;
            J.t[1] = ip >= 0 ? term_of(L.C.at(i), V(z, q, ip), -1.0, 0) : none;
          } else {
            J.t[0] = im >= 0 ? term_of(L.C.at(im), V(z, q, im), -1.0, 1) : none;
            J.t[1] = ip >= 0 ? term_of(L.A.at(ip), V(z, q, ip), -1.0, 1) : none;
          }
          add(ph, J);
          MvJob K{};
          K.y = V(z, q, i);
          K.base = nullptr;
          K.t[0] = MvTerm{L.dinv.at(i), tr, 1.0, V(w, q, i), nullptr};
          K.t[1] = none;
          add(ph + 1, K);
        }
      }
    }
    for (auto& jobs : phases) {
      if (jobs.empty()) continue;
      PhaseJobs pj;
      pj.d = upload(jobs);
      pj.h = jobs;
      pj.n = (int)jobs.size();
      std::vector<int32_t> terms;
      for (size_t jj = 0; jj < jobs.size(); ++jj)
        for (int tt = 0; tt < 2; ++tt)
          if (jobs[jj].t[tt].inst >= 0) terms.push_back((int32_t)(2 * jj + tt));
      pj.terms = upload(terms);
      pj.nterms = (int)terms.size();
      pj.trans = tr;
      max_jobs = std::max(max_jobs, pj.n);
      out.push_back(pj);
    }
  };
  build(-1, 0, ph_apply);
  build(-1, 1, ph_applyT);
  if (np > 1)
    for (int q = 0; q < np; ++q) {
      build(q, 0, probs[q].ph_apply);
      build(q, 1, probs[q].ph_applyT);
    }
  if (coef) dfree(coef);
  coef = dnew<double>((size_t)std::max(max_jobs, 1) * 2 * sstride);
}

// Apply images (see SegImg): every H-matrix that an apply phase multiplies
// gets, per row segment, its rows of the dense leaves and of the U factors
// as one contiguous run of columns (the row image, for H x), and per column
// segment the transposed dense leaves and the rows of the V factors (the
// column image, for H^T x), so the segment kernel streams a segment with
// 16-byte loads and no per-leaf descriptors.  Sized on the host from each
// instance's ranks, filled on the device.
void Handle::build_apply_image(hipStream_t s) {
  for (void* p : {(void*)img_data, (void*)img_widx, (void*)d_img_seg, (void*)d_img_of_inst}) dfree(p);
  img_data = nullptr;
  img_widx = nullptr;
  d_img_seg = nullptr;
  d_img_of_inst = nullptr;
  img_tab_half = 0;
  img_bytes = 0.0;
  std::vector<int32_t> img_of(inst.size(), -1), ids;
  for (const std::vector<PhaseJobs>* phv : {&ph_apply, &ph_applyT})
    for (const PhaseJobs& pj : *phv)
      for (const MvJob& J : pj.h)
        for (const MvTerm& t : J.t)
          if (t.inst >= 0 && img_of[t.inst] < 0) {
            img_of[t.inst] = (int32_t)ids.size();
            ids.push_back(t.inst);
          }
  if (ids.empty()) return;
  const int nseg = (int)G.leaf_clusters.size();
  const int64_t half = (int64_t)ids.size() * nseg;
  // dense columns per segment (geometry only): n of each dense leaf in the
  // row image, m in the column image
  std::vector<int> nd_row(nseg, 0), nd_col(nseg, 0), seg_ld(nseg);
  for (int sg = 0; sg < nseg; ++sg) {
    const Cluster& c = G.cl[G.leaf_clusters[sg]];
    seg_ld[sg] = ((c.hi - c.lo) + 3) & ~3;
    for (int l : G.rows_of_seg[sg])
      if (G.lf[l].fmt != LF_LR) nd_row[sg] += G.lf[l].n;
    for (int l : G.cols_of_seg[sg])
      if (G.lf[l].fmt != LF_LR) nd_col[sg] += G.lf[l].m;
  }
  std::vector<SegImg> tab(2 * half);
  std::vector<int32_t> rk(G.lf.size());
  int64_t doff = 0, woff = 0;
  for (size_t i = 0; i < ids.size(); ++i) {
    HIPCHK(hipMemcpy(rk.data(), inst[ids[i]].rank, rk.size() * sizeof(int32_t), hipMemcpyDeviceToHost));
    for (int tr = 0; tr < 2; ++tr)
      for (int sg = 0; sg < nseg; ++sg) {
        int nu = 0;
        for (int l : (tr ? G.cols_of_seg[sg] : G.rows_of_seg[sg]))
          if (G.lf[l].fmt == LF_LR) nu += rk[l];
        SegImg& e = tab[tr * half + (int64_t)i * nseg + sg];
        e.data_off = doff;
        e.widx_off = woff;
        e.nd = tr ? nd_col[sg] : nd_row[sg];
        e.nu = nu;
        doff += (int64_t)(e.nd + nu) * seg_ld[sg];
        woff += e.nd + nu;
      }
  }
  const size_t esz = fp32 ? 4 : 8;
  img_data = dmalloc((size_t)doff * esz);
  img_widx = dnew<int32_t>((size_t)woff);
  d_img_seg = upload(tab);
  d_img_of_inst = upload(img_of);
  img_tab_half = half;
  int32_t* d_ids = upload(ids);
  sync_tables();
  for (int tr = 0; tr < 2; ++tr) {
    const int32_t* lp = tr ? d_cols_ptr : d_rows_ptr;
    const int32_t* li = tr ? d_cols_idx : d_rows_idx;
    if (fp32)
      launch_img_build<float>((float* const*)d_inst_base, d_inst_rank, d_inst_off, d_leaves, d_soff, d_seg_lo, lp, li,
                              nseg, tr, d_ids, d_img_seg + tr * half, (int)ids.size(), (float*)img_data, img_widx, s);
    else
      launch_img_build<double>((double* const*)d_inst_base, d_inst_rank, d_inst_off, d_leaves, d_soff, d_seg_lo, lp,
                               li, nseg, tr, d_ids, d_img_seg + tr * half, (int)ids.size(), (double*)img_data,
                               img_widx, s);
  }
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(s));
  dfree(d_ids);
  img_bytes = (double)doff * esz + (double)woff * 4 + (double)tab.size() * sizeof(SegImg);
}

void Handle::apply(const std::vector<const double*>& r, const std::vector<double*>& out, bool transpose, int prob,
                   hipStream_t s) {
  sync_tables();
  const int np = (int)probs.size();
  for (int q = 0; q < np; ++q)
    if (prob < 0 || q == prob) launch_to_horder(r[q], g + (int64_t)q * N, d_perm, B, N, s);
  const std::vector<PhaseJobs>* ph;
  if (prob < 0 || np == 1)
    ph = transpose ? &ph_applyT : &ph_apply;
  else
    ph = transpose ? &probs[prob].ph_applyT : &probs[prob].ph_apply;
  for (const PhaseJobs& pj : *ph) launch_phase(pj, pj.ri, s);
  for (int q = 0; q < np; ++q)
    if (prob < 0 || q == prob) launch_from_horder(z + (int64_t)q * N, out[q], d_perm, B, N, s);
  HIPCHK(hipGetLastError());
}

// One apply phase: the coefficient kernel and the segment kernel of its
// jobs.  ri selects the coefficient kernel's schedule (0: one leaf round
// per lane group, 1: four); -1 takes it from the phase size.  The schedule
// changes which wavefront handles a leaf, not the arithmetic of any leaf,
// so results do not depend on it.
void Handle::launch_phase(const PhaseJobs& pj, int ri, hipStream_t s) {
  auto run = [&](auto tag) {
    using T = decltype(tag);
    MvArgs<T> a{};
    a.leaves = d_leaves;
    a.soff = d_soff;
    a.sstride = sstride;
    a.jobs = pj.d;
    a.njobs = pj.n;
    a.terms = pj.terms;
    a.nterms = pj.nterms;
    a.trans = pj.trans;
    a.lr_sorted = pj.trans ? d_lr_t : d_lr_n;
    const int32_t(*cw)[6] = pj.trans ? cw_t : cw_n;
    // by size: four leaves per lane group when the phase fills the chip anyway
    const int r = ri >= 0 ? ri : ((int64_t)pj.nterms * cw[1][5] >= 8192 ? 1 : 0);
    a.rounds = r ? 4 : 1;
    a.w4 = pj.trans ? w4_t : w4_n;
    for (int c = 0; c < 6; ++c) {
      a.cls[c] = pj.trans ? cls_t[c] : cls_n[c];
      a.cw[c] = cw[r][c];
    }
    a.inst_base = (T* const*)d_inst_base;
    a.inst_rank = d_inst_rank;
    a.inst_off = d_inst_off;
    a.coef = coef;
    a.seg_lo = d_seg_lo;
    a.nseg = (int)G.leaf_clusters.size();
    a.img_data = (const T*)img_data;
    a.img_widx = img_widx;
    a.img_seg = d_img_seg + (pj.trans ? img_tab_half : 0);
    a.img_of_inst = d_img_of_inst;
    launch_mv<T>(a, s);
  };
  if (fp32)
    run(float{});
  else
    run(double{});
}

// Schedule autotuning of the apply: every phase of apply and apply_T is
// timed (HIP events, three launches after a warm-up) with each coefficient
// kernel schedule on the handle's own factors, and keeps the faster.  The
// work vectors are cleared first (their values do not affect the time).
// ACR_AUTOTUNE=0 keeps the size rule.
void Handle::tune_apply(hipStream_t s) {
  tuned_phases = 0;
  if (const char* e = getenv("ACR_AUTOTUNE"); e && e[0] == '0') return;
  sync_tables();
  const size_t np = probs.size();
  HIPCHK(hipMemsetAsync(g, 0, (size_t)N * np * sizeof(double), s));
  HIPCHK(hipMemsetAsync(w, 0, (size_t)N * np * sizeof(double), s));
  HIPCHK(hipMemsetAsync(z, 0, (size_t)N * np * sizeof(double), s));
  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  for (std::vector<PhaseJobs>* phv : {&ph_apply, &ph_applyT})
    for (PhaseJobs& pj : *phv) {
      if (pj.nterms == 0) continue;  // no coefficient work: nothing to choose
      float best = 0.f;
      int pick = -1;
      for (int r = 0; r < 2; ++r) {
        launch_phase(pj, r, s);
        HIPCHK(hipEventRecord(e0, s));
        for (int rep = 0; rep < 3; ++rep) launch_phase(pj, r, s);
        HIPCHK(hipEventRecord(e1, s));
        HIPCHK(hipEventSynchronize(e1));
        float t = 0.f;
        HIPCHK(hipEventElapsedTime(&t, e0, e1));
        if (pick < 0 || t < best) {
          best = t;
          pick = r;
        }
      }
      pj.ri = pick;
      ++tuned_phases;
    }
  HIPCHK(hipEventDestroy(e0));
  HIPCHK(hipEventDestroy(e1));
  HIPCHK(hipGetLastError());
}

void Handle::matvec(int prob, const double* x, double* y, bool transpose, hipStream_t s) {
  if (fem27)
    launch_stencil27_mv(probs[prob].S, nx, ny, nz, transpose ? 1 : 0, x, y, s);
  else
    launch_stencil_mv(probs[prob].S, nx, ny, nz, transpose ? 1 : 0, x, y, s);
  HIPCHK(hipGetLastError());
}

// ------------------------------------------------------------ statistics
double Handle::instance_bytes(const std::vector<int32_t>& rk) const {
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

// Statistics.  bytes_per_apply counts the algorithmic traffic of one
// acr_apply from its job list: every job reads each term's stored factor
// (H-matrix at its actual ranks and storage precision, or a diagonal
// coupling in FP64), each term's input plane vector and the base vector if
// any, and writes its output plane vector (plane vectors FP64).  So each
// Dinv below the top counts twice (forward and back substitution).
void Handle::compute_stats() {
  acr_stats_t s{};
  s.levels = (int)probs[0].levels.size() + 1;
  s.nplanes = nz;
  s.plane_points = B;
  s.clusters = (int)G.cl.size();
  s.dense_leaves = G.ndense;
  s.lr_leaves = G.nlr;
  s.precision = opt.precision;
  double total = 0.0;
  double rank_cnt[ACR_MAX_LEVELS] = {0};
  int nf = 0;
  std::map<int, double> ibytes;
  std::vector<int32_t> rk(G.lf.size());
  auto level_of = [&](int r, int id) {
    HIPCHK(hipMemcpy(rk.data(), inst[id].rank, rk.size() * sizeof(int32_t), hipMemcpyDeviceToHost));
    const double b = instance_bytes(rk);
    ibytes[id] = b;
    total += b;
    if (r < ACR_MAX_LEVELS) s.bytes_level[r] += b;
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
  for (const Prob& P : probs) {
    for (size_t r = 0; r < P.levels.size(); ++r) {
      const Level& L = P.levels[r];
      for (auto& kv : L.dinv) level_of((int)r, kv.second);
      for (int p : L.P)
        for (const Coupling* c : {&L.A.at(p), &L.C.at(p)})
          if (c->kind == 2) level_of((int)r, c->inst);
    }
    level_of((int)P.levels.size(), P.top_inst);
  }
  const double vec = 8.0 * B;
  double apply_bytes = 0.0;
  for (const PhaseJobs& pj : ph_apply)
    for (const MvJob& J : pj.h) {
      apply_bytes += vec * (1 + (J.base ? 1 : 0));  // output, base
      for (const MvTerm& t : J.t) {
        if (t.inst >= 0)
          apply_bytes += vec + ibytes.at(t.inst);
        else if (t.dvec)
          apply_bytes += vec + vec;
      }
    }
  for (int r = 0; r < ACR_MAX_LEVELS; ++r)
    if (rank_cnt[r] > 0) s.mean_rank[r] /= rank_cnt[r];
  for (int r = 0; r < ACR_MAX_LEVELS; ++r) s.max_rank_all = std::max(s.max_rank_all, s.max_rank[r]);
  s.factors = nf;
  s.bytes_factors = total;
  s.bytes_allocated = (double)bytes_alloc;
  s.bytes_per_apply = apply_bytes;
  s.bytes_apply_image = img_bytes;
  st = s;
}

}  // namespace acr
