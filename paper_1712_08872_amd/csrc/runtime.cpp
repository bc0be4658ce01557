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
  bytes_peak = std::max(bytes_peak, bytes_alloc);
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
  for (int l = 0; l < 2; ++l) {
    Lane& ln = lanes[l];
    if (ln.s2) {
      (void)hipStreamSynchronize(ln.s2);
      (void)hipStreamDestroy(ln.s2);
    }
    if (l == 1 && ln.s) {  // lane 0's main stream is the caller's
      (void)hipStreamSynchronize(ln.s);
      (void)hipStreamDestroy(ln.s);
    }
    if (ln.fork) (void)hipEventDestroy(ln.fork);
    if (ln.join) (void)hipEventDestroy(ln.join);
  }
  if (kbuf.hres) (void)hipHostFree(kbuf.hres);
  if (ev_products) (void)hipEventDestroy(ev_products);
  for (hipEvent_t e : ev_pool) (void)hipEventDestroy(e);
  for (auto& o : owned) {
    if (opt.free)
      opt.free(o.first, opt.alloc_ctx);
    else
      (void)hipFree(o.first);
  }
}

// ------------------------------------------------------------ instances
static size_t round_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

int Handle::new_instance(hipStream_t s) {
  const size_t esz = fp32 ? 4 : 8;
  const size_t data = round_up((size_t)G.inst_elems * esz, 256);
  const size_t bytes = data + G.lf.size() * sizeof(int32_t);
  int id;
  if (!free_inst.empty()) {
    id = free_inst.back();
    free_inst.pop_back();
  } else {
    id = (int)inst.size();
    inst.emplace_back();
  }
  Instance& I = inst[id];
  if (!cap_pool.empty()) {
    I.buf = cap_pool.back();
    cap_pool.pop_back();
  } else {
    I.buf = dmalloc(bytes);
  }
  I.base = I.buf;
  I.rank = (int32_t*)((char*)I.buf + data);
  I.off = nullptr;
  I.live = true;
  I.packed = false;
  I.packed_bytes = 0;
  table_dirty = true;
  // zero the dense leaves (level 0 scatters a sparse pattern into them) and
  // the ranks; low-rank columns are only ever read below their rank, so the
  // capacity beyond it (most of the buffer) is left as it is
  HIPCHK(hipMemsetAsync(I.buf, 0, (size_t)G.dense_elems * esz, s));
  HIPCHK(hipMemsetAsync(I.rank, 0, G.lf.size() * sizeof(int32_t), s));
  return id;
}

void Handle::release_instance(int id) {
  if (id < 0 || !inst[id].live) return;
  Instance& I = inst[id];
  if (I.packed)
    dfree(I.buf);
  else
    cap_pool.push_back(I.buf);
  I = Instance{};
  free_inst.push_back(id);
  table_dirty = true;
}

// Storage order of the leaves in packed instances: by first row, then first
// column, so that the leaves a row segment of the matrix-vector product
// reads lie together.
void Handle::ensure_pack_order() {
  const size_t nl = G.lf.size();
  if (pack_order.size() == nl) return;
  pack_order.resize(nl);
  for (size_t l = 0; l < nl; ++l) pack_order[l] = (int)l;
  std::stable_sort(pack_order.begin(), pack_order.end(), [&](int a, int b) {
    const Leaf &A = G.lf[a], &B = G.lf[b];
    return A.r0 != B.r0 ? A.r0 < B.r0 : A.c0 < B.c0;
  });
}

// A packed instance from host data given leaf by leaf in leaf order: dense
// leaves m x n column-major, low-rank leaves U (m x k) then V (n x k), both
// column-major, k = rank[l].  Stored in the packed layout at the handle's
// factor precision.
int Handle::new_packed_instance(const std::vector<int32_t>& rank, const double* data, hipStream_t s) {
  ensure_pack_order();
  const size_t nl = G.lf.size();
  const size_t esz = fp32 ? 4 : 8;
  std::vector<int64_t> off(nl), src(nl);
  int64_t acc = 0, sacc = 0;
  for (size_t l = 0; l < nl; ++l) {
    const Leaf& L = G.lf[l];
    src[l] = sacc;
    sacc += L.fmt == LF_DENSE ? (int64_t)L.m * L.n : (int64_t)(L.m + L.n) * rank[l];
  }
  for (int l : pack_order) {
    const Leaf& L = G.lf[l];
    off[l] = acc;
    const int64_t ldm = (L.m + 3) & ~3, ldn = (L.n + 3) & ~3;
    acc += L.fmt == LF_DENSE ? ldm * L.n : (ldm + ldn) * rank[l];
  }
  std::vector<double> host((size_t)acc, 0.0);
  for (size_t l = 0; l < nl; ++l) {
    const Leaf& L = G.lf[l];
    const int64_t ldm = (L.m + 3) & ~3, ldn = (L.n + 3) & ~3;
    const double* d = data + src[l];
    double* o = host.data() + off[l];
    const int cols = L.fmt == LF_DENSE ? L.n : rank[l];
    for (int c = 0; c < cols; ++c)
      for (int i = 0; i < L.m; ++i) o[i + ldm * c] = d[i + (int64_t)L.m * c];
    if (L.fmt == LF_LR) {
      const double* dv = d + (int64_t)L.m * rank[l];
      double* ov = o + ldm * rank[l];
      for (int c = 0; c < rank[l]; ++c)
        for (int i = 0; i < L.n; ++i) ov[i + ldn * c] = dv[i + (int64_t)L.n * c];
    }
  }
  const size_t bytes = round_up((size_t)acc * esz, 256);
  const size_t rbytes = round_up(nl * sizeof(int32_t), 256);
  char* nb = (char*)dmalloc(bytes + rbytes + nl * sizeof(int64_t));
  if (fp32) {
    std::vector<float> hf(host.begin(), host.end());
    HIPCHK(hipMemcpy(nb, hf.data(), hf.size() * 4, hipMemcpyHostToDevice));
  } else {
    HIPCHK(hipMemcpy(nb, host.data(), host.size() * 8, hipMemcpyHostToDevice));
  }
  HIPCHK(hipMemcpy(nb + bytes, rank.data(), nl * sizeof(int32_t), hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(nb + bytes + rbytes, off.data(), nl * sizeof(int64_t), hipMemcpyHostToDevice));
  int id;
  if (!free_inst.empty()) {
    id = free_inst.back();
    free_inst.pop_back();
  } else {
    id = (int)inst.size();
    inst.emplace_back();
  }
  Instance& I = inst[id];
  I.buf = nb;
  I.base = nb;
  I.rank = (int32_t*)(nb + bytes);
  I.off = (int64_t*)(nb + bytes + rbytes);
  I.live = true;
  I.packed = true;
  I.packed_bytes = (double)acc * esz;
  table_dirty = true;
  (void)s;
  return id;
}

// Pack final instances: exact ranks, leading dimensions padded to 4
// elements, per-leaf offsets; their capacity buffers return to the pool.
void Handle::pack_instances(const std::vector<int>& ids, hipStream_t s) {
  if (ids.empty()) return;
  HIPCHK(hipStreamSynchronize(s));
  const size_t esz = fp32 ? 4 : 8;
  const size_t nl = G.lf.size();
  std::vector<int32_t> rk(nl);
  std::vector<int64_t> off(nl);
  for (int id : ids) {
    Instance& I = inst[id];
    if (!I.live || I.packed) continue;
    HIPCHK(hipMemcpy(rk.data(), I.rank, nl * sizeof(int32_t), hipMemcpyDeviceToHost));
    ensure_pack_order();
    int64_t acc = 0;
    for (int l : pack_order) {
      const Leaf& L = G.lf[l];
      off[l] = acc;
      const int64_t ldm = (L.m + 3) & ~3, ldn = (L.n + 3) & ~3;
      acc += L.fmt == LF_DENSE ? ldm * L.n : (ldm + ldn) * rk[l];
    }
    const size_t data = round_up((size_t)acc * esz, 256);
    const size_t rbytes = round_up(nl * sizeof(int32_t), 256);
    char* nb = (char*)dmalloc(data + rbytes + nl * sizeof(int64_t));
    int32_t* nrank = (int32_t*)(nb + data);
    int64_t* noff = (int64_t*)(nb + data + rbytes);
    HIPCHK(hipMemcpy(noff, off.data(), nl * sizeof(int64_t), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpyAsync(nrank, I.rank, nl * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
    if (fp32)
      launch_pack<float>((const float*)I.base, I.rank, d_leaves, (int)nl, (float*)nb, noff, s);
    else
      launch_pack<double>((const double*)I.base, I.rank, d_leaves, (int)nl, (double*)nb, noff, s);
    cap_pool.push_back(I.buf);  // later users are ordered after the pack on the stream
    I.buf = nb;
    I.base = nb;
    I.rank = nrank;
    I.off = noff;
    I.packed = true;
    I.packed_bytes = (double)acc * esz;
  }
  HIPCHK(hipGetLastError());
  table_dirty = true;
}

void Handle::sync_tables() {
  if (!table_dirty) return;
  if ((int)inst.size() > inst_table_cap) {
    if (lanes[1].s) HIPCHK(hipStreamSynchronize(lanes[1].s));  // it may read the old tables
    if (lanes[1].s2) HIPCHK(hipStreamSynchronize(lanes[1].s2));
    if (d_inst_base) dfree(d_inst_base);
    if (d_inst_rank) dfree(d_inst_rank);
    if (d_inst_off) dfree(d_inst_off);
    inst_table_cap = std::max<int>(256, (int)inst.size() * 2);
    d_inst_base = dnew<void*>(inst_table_cap);
    d_inst_rank = dnew<int32_t*>(inst_table_cap);
    d_inst_off = dnew<int64_t*>(inst_table_cap);
  }
  std::vector<void*> b(inst.size());
  std::vector<int32_t*> r(inst.size());
  std::vector<int64_t*> o(inst.size());
  for (size_t i = 0; i < inst.size(); ++i) {
    b[i] = inst[i].base;
    r[i] = inst[i].rank;
    o[i] = inst[i].off;
  }
  HIPCHK(hipMemcpy(d_inst_base, b.data(), b.size() * sizeof(void*), hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(d_inst_rank, r.data(), r.size() * sizeof(int32_t*), hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(d_inst_off, o.data(), o.size() * sizeof(int64_t*), hipMemcpyHostToDevice));
  table_dirty = false;
}

// ------------------------------------------------------------ programs
void Handle::upload_program(Program& p) {
  // dense accumulators of the small low-rank targets, per step and batch item
  p.doff.assign(p.targets.size(), -1);
  for (Step& st : p.steps) {
    if (st.type != 0) continue;
    int64_t acc = 0;
    for (int t = st.t0; t < st.t0 + st.nt; ++t) {
      const Target& T = p.targets[t];
      const Leaf& L = G.lf[T.cleaf];
      if (L.fmt == LF_LR && (int64_t)L.m * L.n <= DACC_ELEMS && !T.direct && T.p1 > T.p0) {
        p.doff[t] = acc;
        acc += ((int64_t)L.m * L.n + 63) / 64 * 64;
      }
    }
    st.dstride = acc;
  }
  p.d_pieces = upload(p.pieces);
  p.d_targets = upload(p.targets);
  p.d_lists = upload(p.lists);
  p.d_doff = upload(p.doff);
}

// Streams, events and accumulation scratch of a lane (created on first use;
// every stream of the library has the default priority).
void Handle::ensure_lane(Lane& ln, hipStream_t main) {
  if (&ln == &lanes[0]) {
    ln.s = main;
  } else if (!ln.s) {
    HIPCHK(hipStreamCreateWithFlags(&ln.s, hipStreamNonBlocking));
  }
  if (!ln.s2) {
    HIPCHK(hipStreamCreateWithFlags(&ln.s2, hipStreamNonBlocking));
    HIPCHK(hipEventCreateWithFlags(&ln.fork, hipEventDisableTiming));
    HIPCHK(hipEventCreateWithFlags(&ln.join, hipEventDisableTiming));
  }
  if (!ln.scratch) ln.scratch = dmalloc((size_t)2 * scratch_slots * scratch_stride * (fp32 ? 4 : 8));
}

template <typename T>
void Handle::run_accum_step(Program& P, const Step& st, int nbatch, int nroles, int nvroles, Lane& ln) {
  const hipStream_t s = ln.s, s2 = ln.s2;
  // batch chunks whose dense accumulators fit the buffer limit
  constexpr size_t kDbufMax = size_t(4) << 30;
  int chunk = nbatch;
  if (st.dstride > 0) {
    const size_t per = (size_t)st.dstride * sizeof(T);
    chunk = (int)std::max<int64_t>(1, std::min<int64_t>(nbatch, (int64_t)(kDbufMax / per)));
    const size_t need = per * (size_t)chunk;
    if (need > ln.dbuf_bytes) {
      HIPCHK(hipStreamSynchronize(s));  // the lane's previous steps are done with the buffer
      if (ln.dbuf) dfree(ln.dbuf);
      ln.dbuf = dmalloc(need);
      ln.dbuf_bytes = need;
    }
  }
  for (int b0 = 0; b0 < nbatch; b0 += chunk) {
    const int nb = std::min(chunk, nbatch - b0);
    AccumArgs<T> a{};
    a.leaves = d_leaves;
    a.pieces = P.d_pieces;
    a.targets = P.d_targets;
    a.lists = P.d_lists;
    a.t0 = st.t0;
    a.nt = st.nt;
    a.nbatch = nb;
    a.nroles = nroles;
    a.nvroles = nvroles;
    a.role_inst = ln.d_roles + (size_t)b0 * nroles;
    a.vec_ptr = nvroles > 0 ? ln.d_vecs + (size_t)b0 * nvroles : nullptr;
    a.inst_base = (T* const*)d_inst_base;
    a.inst_rank = d_inst_rank;
    a.inst_off = d_inst_off;
    a.scratch = (T*)ln.scratch;
    a.scratch_stride = scratch_stride;
    a.eps = opt.eps;
    a.flags = d_flags;
    a.dbuf = (T*)ln.dbuf;
    a.doff = P.d_doff;
    a.dstride = st.dstride;
    a.prof = d_prof;
    a.flops = d_flops;
    a.bf16_products = bf16 ? 1 : 0;
    const int64_t items = (int64_t)nb * st.nt;
    const int grid = (int)std::min<int64_t>(items, scratch_slots);
    auto timed = [&](hipStream_t q, auto&& launch, const char* tag_suffix) {
      if (timing) {
        while (ev_pool.size() < ev_used + 2) {
          hipEvent_t e;
          HIPCHK(hipEventCreate(&e));
          ev_pool.push_back(e);
        }
        HIPCHK(hipEventRecord(ev_pool[ev_used], q));
        ev_tag.push_back({P.name.c_str(), cur_level, (int)(&st - P.steps.data()), nb, st.nt, st.max_m,
                          tag_suffix});
      }
      launch();
      if (timing) {
        HIPCHK(hipEventRecord(ev_pool[ev_used + 1], q));
        ev_used += 2;
      }
    };
    // The low-rank targets that do not need the first phase run on the
    // second stream (own scratch slots) while the first phase and then the
    // compression of its dense sums run on the main stream; joined before
    // the next step.
    AccumArgs<T> a1 = a;
    a1.mode = 1;
    a1.scratch = (T*)ln.scratch + (int64_t)scratch_slots * scratch_stride;
    HIPCHK(hipEventRecord(ln.fork, s));
    HIPCHK(hipStreamWaitEvent(s2, ln.fork, 0));
    timed(s2, [&] {
      if (kc == 38)
        kc38::launch_accum<T>(a1, grid, s2);
      else
        kc64::launch_accum<T>(a1, grid, s2);
    }, "");
    AccumArgs<T> ad = a;
    ad.flops = d_flops ? d_flops + FC_COUNT + 1 : nullptr;
    timed(s, [&] {
      if (kc == 38)
        kc38::launch_accum_dense<T>(ad, grid, s);
      else
        kc64::launch_accum_dense<T>(ad, grid, s);
    }, "dense");
    ++dense_launches;
    if (st.dstride > 0) {
      AccumArgs<T> a2 = a;
      a2.mode = 2;
      timed(s, [&] {
        if (kc == 38)
          kc38::launch_accum<T>(a2, grid, s);
        else
          kc64::launch_accum<T>(a2, grid, s);
      }, "");
      ++accum_launches;
    }
    ++accum_launches;
    HIPCHK(hipEventRecord(ln.join, s2));
    HIPCHK(hipStreamWaitEvent(s, ln.join, 0));
  }
}
template void Handle::run_accum_step<float>(Program&, const Step&, int, int, int, Lane&);
template void Handle::run_accum_step<double>(Program&, const Step&, int, int, int, Lane&);

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
  P.name = key;
  upload_program(P);
  auto res = prog.emplace(key, std::move(P));
  return res.first->second;
}

void Handle::run_program(Program& P, int nbatch, int nroles, const std::vector<int32_t>& roles, int nvroles,
                         const std::vector<const double*>& vecs, Lane& ln) {
  if (nbatch <= 0) return;
  const hipStream_t s = ln.s;
  sync_tables();
  // role and vector tables of this run (synchronous copies after the lane's
  // previous work: the host vectors are rewritten by the next call)
  HIPCHK(hipStreamSynchronize(s));
  if ((int)roles.size() > ln.roles_cap) {
    if (ln.d_roles) dfree(ln.d_roles);
    ln.roles_cap = std::max<int>(1024, (int)roles.size() * 2);
    ln.d_roles = dnew<int32_t>(ln.roles_cap);
  }
  HIPCHK(hipMemcpy(ln.d_roles, roles.data(), roles.size() * sizeof(int32_t), hipMemcpyHostToDevice));
  if (!vecs.empty()) {
    if ((int)vecs.size() > ln.vecs_cap) {
      if (ln.d_vecs) dfree((void*)ln.d_vecs);
      ln.vecs_cap = std::max<int>(1024, (int)vecs.size() * 2);
      ln.d_vecs = dnew<const double*>(ln.vecs_cap);
    }
    HIPCHK(hipMemcpy((void*)ln.d_vecs, vecs.data(), vecs.size() * sizeof(double*), hipMemcpyHostToDevice));
  }
  for (size_t si = 0; si < P.steps.size(); ++si) {
    const Step& st = P.steps[si];
    if (st.type == 1) {
      const Leaf& L = G.lf[st.leaf];
      leaf_inverse_flops += 2.0 * L.m * L.m * L.m * nbatch;  // LU and inverse of an m x m leaf
      if (fp32)
        launch_leaf_inverse<float>((float* const*)d_inst_base, ln.d_roles, nroles, nbatch, L.off, L.m, d_flags, s);
      else
        launch_leaf_inverse<double>((double* const*)d_inst_base, ln.d_roles, nroles, nbatch, L.off, L.m, d_flags,
                                    s);
      continue;
    }
    if (fp32)
      run_accum_step<float>(P, st, nbatch, nroles, nvroles, ln);
    else
      run_accum_step<double>(P, st, nbatch, nroles, nvroles, ln);
  }
  HIPCHK(hipGetLastError());
}

}  // namespace acr
