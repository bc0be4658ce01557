// C ABI of libacr (declared in include/acr.h): argument validation on the
// host before any device work, error codes and thread-local messages, and
// the handle lifecycle.  A handle holds one or more groups of problems
// (problems of a group share the plane shape and run every setup and apply
// step in the same launches).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <map>
#include <exception>
#include <string>
#include <thread>
#include <tuple>

#include "runtime.h"

namespace acr {
acr_status krylov_cg(Handle& h, KrylovBuffers* wb, int prob, bool flexible, bool tr, double rtol, int maxit,
                     const double* b, double* x, acr_solve_info* info, hipStream_t s);
acr_status krylov_gmres(Handle& h, KrylovBuffers* wb, int prob, int m, bool tr, double rtol, int maxit,
                        const double* b, double* x, acr_solve_info* info, hipStream_t s);
}  // namespace acr

namespace {
thread_local std::string g_last_error;

acr_status fail(acr_status s, const std::string& msg) {
  g_last_error = msg;
  return s;
}

acr_status device_check() {
  int n = 0;
  hipError_t e = hipGetDeviceCount(&n);
  if (e != hipSuccess || n == 0) {
    (void)hipGetLastError();
    return fail(ACR_E_DEVICE, "no HIP device available");
  }
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return fail(ACR_E_DEVICE, "hipGetDevice failed");
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return fail(ACR_E_DEVICE, "hipGetDeviceProperties failed");
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
    return fail(ACR_E_DEVICE, std::string("libacr is built for gfx950, device is ") + prop.gcnArchName);
  return ACR_OK;
}

template <typename F>
acr_status guard(F&& f) {
  try {
    return f();
  } catch (const acr::AcrError& e) {
    return fail(e.st, e.what());
  } catch (const std::bad_alloc&) {
    return fail(ACR_E_NOMEM, "host allocation failed");
  } catch (const std::exception& e) {
    return fail(ACR_E_DEVICE, e.what());
  }
}

bool finite_pos(double v) { return std::isfinite(v) && v > 0.0; }

acr_status check_problem(const acr_problem* p) {
  if (p->nx < 1 || p->ny < 1 || p->nz < 1) return fail(ACR_E_INVALID, "grid sizes must be >= 1");
  if ((int64_t)p->nx * p->ny > (1 << 26) || (int64_t)p->nx * p->ny * p->nz > ((int64_t)1 << 34))
    return fail(ACR_E_INVALID, "grid too large");
  if (p->kind < ACR_POISSON_HARMONIC || p->kind > ACR_HELMHOLTZ_FEM27) return fail(ACR_E_INVALID, "unknown problem kind");
  if (p->kind == ACR_STENCIL7_RAW && !p->stencil7) return fail(ACR_E_INVALID, "RAW problem needs stencil7");
  if ((p->kind == ACR_HELMHOLTZ || p->kind == ACR_HELMHOLTZ_FEM27) && (!p->c || !std::isfinite(p->omega)))
    return fail(ACR_E_INVALID, "Helmholtz problem needs c and a finite omega");
  if ((p->kind == ACR_CONVDIFF_UPWIND || p->kind == ACR_CONVDIFF_RECIRC) &&
      (!std::isfinite(p->beta_amp) || !std::isfinite(p->beta_phase)))
    return fail(ACR_E_INVALID, "convection parameters must be finite");
  return ACR_OK;
}

acr_status check_options(const acr_options* o) {
  // the truncation forms FP64 Gram matrices of the factors, whose
  // eigenvalues resolve singular values down to about 1e-8 of the largest:
  // a smaller eps could not be honoured
  if (!(o->eps >= ACR_EPS_MIN && o->eps < 1.0))
    return fail(ACR_E_INVALID, "eps must lie in [1e-7, 1): the truncation resolves singular values only down "
                               "to about 1e-8 of the largest");
  if (!finite_pos(o->eta)) return fail(ACR_E_INVALID, "eta must be positive");
  if (o->leaf_size < 4 || o->leaf_size > 64) return fail(ACR_E_INVALID, "leaf_size must lie in [4, 64]");
  if (o->precision != ACR_FP64 && o->precision != ACR_MIXED_FP32 && o->precision != ACR_MIXED_BF16)
    return fail(ACR_E_INVALID, "unknown precision");
  if (o->precision == ACR_MIXED_BF16 && !(o->eps >= 1e-2))
    return fail(ACR_E_INVALID, "BF16 factors need eps >= 1e-2");
  if (o->max_rank < 0 || o->max_rank > acr::KC_MAX - 8) return fail(ACR_E_INVALID, "max_rank must lie in [0, 56]");
  if (o->dense_work < 0 || o->dense_work > 64) return fail(ACR_E_INVALID, "dense_work must lie in [0, 64]");
  if ((o->alloc == nullptr) != (o->free == nullptr)) return fail(ACR_E_INVALID, "alloc and free come together");
  if (o->flags != 0) return fail(ACR_E_INVALID, "flags must be 0");
  return ACR_OK;
}

// Set up `count` problems: group them by (nx, ny, nz), one group per shape,
// in order of first appearance.
acr_status setup_many(const acr_problem* ps, int count, const acr_options* o, void* stream, acr_handle** out) {
  acr_handle* h = nullptr;
  acr_status st = guard([&]() {
    h = new acr_handle();
    std::map<std::tuple<int, int, int, int>, int> gid;
    std::vector<std::vector<int>> members;
    for (int i = 0; i < count; ++i) {
      // a group shares the plane shape and the stencil (7- or 27-point)
      auto key = std::make_tuple(ps[i].nx, ps[i].ny, ps[i].nz, ps[i].kind == ACR_HELMHOLTZ_FEM27 ? 27 : 7);
      auto it = gid.find(key);
      int g;
      if (it == gid.end()) {
        g = (int)members.size();
        gid[key] = g;
        members.emplace_back();
      } else {
        g = it->second;
      }
      h->where.emplace_back(g, (int)members[g].size());
      members[g].push_back(i);
    }
    for (int i = 0; i < count; ++i) {
      h->off.push_back(h->total);
      h->grid_off.push_back(h->grid_total);
      h->total += (int64_t)ps[i].nx * ps[i].ny * ps[i].nz;
      h->grid_total += (int64_t)(ps[i].nx + 2) * (ps[i].ny + 2) * (ps[i].nz + 2);
    }
    const int G = (int)members.size();
    std::vector<std::vector<acr_problem>> gp(G);
    for (int g = 0; g < G; ++g) {
      for (int i : members[g]) gp[g].push_back(ps[i]);
      h->groups.push_back(std::make_unique<acr::Handle>());
      h->groups.back()->opt = *o;
    }
    if (G == 1) {
      h->groups[0]->setup(gp[0].data(), (int)gp[0].size(), (hipStream_t)stream);
      return ACR_OK;
    }
    // several plane shapes: each group on its own stream (forked from the
    // caller's, so the inputs are ready) and host thread, concurrently when
    // their estimated setup footprints fit the free device memory together
    // (about 400 bytes per unknown and unit of rank capacity and per byte of
    // factor precision, the measured peak of the 127^3 setups with margin)
    HIPCHK(hipEventCreateWithFlags(&h->fork, hipEventDisableTiming));
    HIPCHK(hipEventRecord(h->fork, (hipStream_t)stream));
    for (int g = 0; g < G; ++g) {
      hipStream_t gs;
      hipEvent_t ge;
      HIPCHK(hipStreamCreateWithFlags(&gs, hipStreamNonBlocking));
      h->gstream.push_back(gs);
      HIPCHK(hipEventCreateWithFlags(&ge, hipEventDisableTiming));
      h->gdone.push_back(ge);
      HIPCHK(hipStreamWaitEvent(gs, h->fork, 0));
    }
    const double cap = o->max_rank > 0 ? o->max_rank : std::max(8.0, 6.0 + 6.0 * std::log10(1.0 / o->eps));
    const double esz = o->precision == ACR_FP64 ? 8.0 : 4.0;
    double est = 0.0;
    for (int g = 0; g < G; ++g)
      est += 400.0 * cap * esz * (double)gp[g][0].nx * gp[g][0].ny * gp[g][0].nz * (double)gp[g].size();
    size_t free_b = 0, total_b = 0;
    HIPCHK(hipMemGetInfo(&free_b, &total_b));
    const bool serial = est > 0.7 * (double)free_b || [] {
      const char* e = getenv("ACR_SERIAL_GROUPS");
      return e && e[0] == '1';
    }();
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    std::vector<std::exception_ptr> err(G);
    auto run = [&](int g) {
      try {
        HIPCHK(hipSetDevice(dev));
        h->groups[g]->setup(gp[g].data(), (int)gp[g].size(), h->gstream[g]);
      } catch (...) {
        err[g] = std::current_exception();
      }
    };
    if (serial) {
      for (int g = 0; g < G; ++g) run(g);
    } else {
      std::vector<std::thread> th;
      for (int g = 0; g < G; ++g) th.emplace_back(run, g);
      for (auto& t : th) t.join();
    }
    for (int g = 0; g < G; ++g)
      if (err[g]) std::rethrow_exception(err[g]);
    return ACR_OK;
  });
  if (st != ACR_OK) {
    delete h;
    return st;
  }
  *out = h;
  return ACR_OK;
}

// Run f(group, per-problem input pointers, per-problem output pointers) for
// every group, slicing concatenated vectors at the problem offsets.
template <typename F>
void for_groups(acr_handle* h, const double* r, double* z, F&& f) {
  for (size_t g = 0; g < h->groups.size(); ++g) {
    acr::Handle& grp = *h->groups[g];
    std::vector<const double*> in(grp.probs.size());
    std::vector<double*> outp(grp.probs.size());
    for (size_t i = 0; i < h->where.size(); ++i)
      if (h->where[i].first == (int)g) {
        in[h->where[i].second] = r + h->off[i];
        outp[h->where[i].second] = z + h->off[i];
      }
    f(grp, in, outp);
  }
}
// z = M^{-1} r or M^{-T} r for every problem: one group on the caller's
// stream; several groups each on its own stream, forked from and joined to
// the caller's (stream-ordered for the caller, concurrent between groups).
acr_status apply_all(acr_handle* h, const double* r, double* z, int32_t nrhs, void* stream, bool tr) {
  if (!h || !r || !z) return fail(ACR_E_INVALID, "null argument");
  if (nrhs < 1) return fail(ACR_E_INVALID, "nrhs must be >= 1");
  if (r == z) return fail(ACR_E_INVALID, "z must not alias r");
  return guard([&]() {
    const bool fork = !h->gstream.empty();
    if (fork) {
      HIPCHK(hipEventRecord(h->fork, (hipStream_t)stream));
      for (hipStream_t gs : h->gstream) HIPCHK(hipStreamWaitEvent(gs, h->fork, 0));
    }
    size_t gi = 0;
    for (int k = 0; k < nrhs; ++k) {
      gi = 0;
      for_groups(h, r + (int64_t)k * h->total, z + (int64_t)k * h->total,
                 [&](acr::Handle& g, const std::vector<const double*>& in, const std::vector<double*>& outp) {
                   g.apply(in, outp, tr, -1, fork ? h->gstream[gi] : (hipStream_t)stream);
                   ++gi;
                 });
    }
    if (fork)
      for (size_t g = 0; g < h->gstream.size(); ++g) {
        HIPCHK(hipEventRecord(h->gdone[g], h->gstream[g]));
        HIPCHK(hipStreamWaitEvent((hipStream_t)stream, h->gdone[g], 0));
      }
    return ACR_OK;
  });
}

}  // namespace

namespace acr {

acr_status set_last_error(acr_status s, const std::string& msg) { return fail(s, msg); }

int krylov_vectors(int32_t method, int32_t restart) { return method == ACR_GMRES ? 2 * restart + 3 : 5; }

acr_status check_solve_args(const acr_handle* h, int32_t method, int32_t restart, double rtol, int32_t maxit,
                            const double* b, const double* x, const acr_solve_info* info) {
  if (!h || !b || !x || !info) return fail(ACR_E_INVALID, "null argument");
  if (b == x) return fail(ACR_E_INVALID, "x must not alias b");
  if (method < ACR_CG || method > ACR_GMRES) return fail(ACR_E_INVALID, "unknown method");
  if (!(rtol > 0.0 && rtol < 1.0)) return fail(ACR_E_INVALID, "rtol must lie in (0, 1)");
  if (maxit < 1) return fail(ACR_E_INVALID, "maxit must be >= 1");
  if (method == ACR_GMRES && (restart < 1 || restart > 60)) return fail(ACR_E_INVALID, "restart must lie in [1, 60]");
  return ACR_OK;
}

// krylov_solve: validation, then every problem solved to its own tolerance;
// the info reports the largest iteration count and residual and the first
// failure.  wb = nullptr: the handle's own buffers (allocated at the first
// solve), else the given fixed buffers.
acr_status solve_problems(acr_handle* h, int32_t method, int32_t restart, int32_t transpose, double rtol,
                          int32_t maxit, const double* b, double* x, acr_solve_info* info, void* stream,
                          KrylovBuffers* wb) {
  acr_status v = check_solve_args(h, method, restart, rtol, maxit, b, x, info);
  if (v != ACR_OK) return v;
  std::memset(info, 0, sizeof(*info));
  acr_status result = ACR_OK;
  acr_status st = guard([&]() {
    for (size_t i = 0; i < h->where.size(); ++i) {
      Handle& g = *h->groups[h->where[i].first];
      const int q = h->where[i].second;
      acr_solve_info one{};
      acr_status r;
      if (method == ACR_GMRES)
        r = krylov_gmres(g, wb, q, restart, transpose != 0, rtol, maxit, b + h->off[i], x + h->off[i], &one,
                         (hipStream_t)stream);
      else
        r = krylov_cg(g, wb, q, method == ACR_FCG, transpose != 0, rtol, maxit, b + h->off[i], x + h->off[i], &one,
                      (hipStream_t)stream);
      info->iters = std::max(info->iters, one.iters);
      info->relres_true = std::max(info->relres_true, one.relres_true);
      if (one.variant == ACR_FCG || i == 0) info->variant = one.variant;
      if (r != ACR_OK && result == ACR_OK) result = r;
    }
    info->status = result;
    return ACR_OK;
  });
  if (st != ACR_OK) return st;
  if (result != ACR_OK) return fail(result, std::string("krylov_solve: ") + acr_status_string(result));
  return ACR_OK;
}

}  // namespace acr

extern "C" {

void acr_default_options(acr_options* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->eps = 1e-4;
  o->eta = 2.0;
  o->leaf_size = 32;
  o->precision = ACR_FP64;
  o->max_rank = 0;
  o->dense_work = 0;
}

const char* acr_status_string(acr_status s) {
  switch (s) {
    case ACR_OK: return "ok";
    case ACR_E_INVALID: return "invalid argument";
    case ACR_E_NUMERIC: return "non-finite or non-positive coefficient";
    case ACR_E_NOMEM: return "out of device memory";
    case ACR_E_SINGULAR: return "singular leaf block";
    case ACR_E_BREAKDOWN: return "Krylov breakdown";
    case ACR_E_NOTCONV: return "not converged";
    case ACR_E_DEVICE: return "device or runtime error";
    case ACR_E_RANK: return "rank capacity exhausted";
  }
  return "unknown status";
}

const char* acr_last_error(void) { return g_last_error.c_str(); }

acr_status acr_setup(const acr_problem* p, const acr_options* o, void* stream, acr_handle** out) {
  if (out) *out = nullptr;
  if (!p || !o || !out) return fail(ACR_E_INVALID, "null argument");
  acr_status s = check_problem(p);
  if (s != ACR_OK) return s;
  s = check_options(o);
  if (s != ACR_OK) return s;
  s = device_check();
  if (s != ACR_OK) return s;
  return setup_many(p, 1, o, stream, out);
}

acr_status acr_setup_batched(const acr_problem* ps, int32_t count, const acr_options* o, void* stream,
                             acr_handle** out) {
  if (out) *out = nullptr;
  if (!ps || !o || !out) return fail(ACR_E_INVALID, "null argument");
  if (count < 1 || count > 4096) return fail(ACR_E_INVALID, "count must lie in [1, 4096]");
  for (int i = 0; i < count; ++i) {
    acr_status s = check_problem(ps + i);
    if (s != ACR_OK) return fail(s, "problem " + std::to_string(i) + ": " + g_last_error);
  }
  acr_status s = check_options(o);
  if (s != ACR_OK) return s;
  s = device_check();
  if (s != ACR_OK) return s;
  return setup_many(ps, count, o, stream, out);
}

acr_status acr_import_factors(const acr_problem* p, const acr_options* o, const acr_factor_blob* blob, void* stream,
                              acr_handle** out) {
  if (out) *out = nullptr;
  if (!p || !o || !blob || !out || (blob->count > 0 && !blob->factors)) return fail(ACR_E_INVALID, "null argument");
  if (blob->count < 1) return fail(ACR_E_INVALID, "no factors");
  acr_status s = check_problem(p);
  if (s != ACR_OK) return s;
  s = check_options(o);
  if (s != ACR_OK) return s;
  s = guard([&]() {
    acr::check_factor_blob(p, o, blob);
    return ACR_OK;
  });
  if (s != ACR_OK) return s;
  s = device_check();
  if (s != ACR_OK) return s;
  acr_handle* h = nullptr;
  s = guard([&]() {
    h = new acr_handle();
    h->where.emplace_back(0, 0);
    h->off.push_back(0);
    h->grid_off.push_back(0);
    h->total = (int64_t)p->nx * p->ny * p->nz;
    h->grid_total = (int64_t)(p->nx + 2) * (p->ny + 2) * (p->nz + 2);
    auto grp = std::make_unique<acr::Handle>();
    grp->opt = *o;
    grp->import_factors(p, blob, (hipStream_t)stream);
    h->groups.push_back(std::move(grp));
    return ACR_OK;
  });
  if (s != ACR_OK) {
    delete h;
    return s;
  }
  *out = h;
  return ACR_OK;
}

acr_status acr_problem_offset(const acr_handle* h, int32_t i, int64_t* off, int64_t* n, int64_t* grid_off,
                              int64_t* grid_n) {
  if (!h) return fail(ACR_E_INVALID, "null handle");
  if (i < 0 || i >= (int)h->where.size()) return fail(ACR_E_INVALID, "problem index out of range");
  const acr::Handle& g = *h->groups[h->where[i].first];
  if (off) *off = h->off[i];
  if (n) *n = g.N;
  if (grid_off) *grid_off = h->grid_off[i];
  if (grid_n) *grid_n = (int64_t)(g.nx + 2) * (g.ny + 2) * (g.nz + 2);
  return ACR_OK;
}

acr_status acr_apply(acr_handle* h, const double* r, double* z, int32_t nrhs, void* stream) {
  return apply_all(h, r, z, nrhs, stream, false);
}

acr_status acr_apply_T(acr_handle* h, const double* r, double* z, int32_t nrhs, void* stream) {
  return apply_all(h, r, z, nrhs, stream, true);
}

acr_status acr_matvec(acr_handle* h, int32_t transpose, const double* x, double* y, void* stream) {
  if (!h || !x || !y) return fail(ACR_E_INVALID, "null argument");
  if (x == y) return fail(ACR_E_INVALID, "y must not alias x");
  return guard([&]() {
    for (size_t i = 0; i < h->where.size(); ++i)
      h->groups[h->where[i].first]->matvec(h->where[i].second, x + h->off[i], y + h->off[i], transpose != 0,
                                           (hipStream_t)stream);
    return ACR_OK;
  });
}

acr_status acr_get_stencil(acr_handle* h, double* out, void* stream) {
  if (!h || !out) return fail(ACR_E_INVALID, "null argument");
  return guard([&]() {
    int64_t o = 0;
    for (size_t i = 0; i < h->where.size(); ++i) {
      const acr::Handle& g = *h->groups[h->where[i].first];
      HIPCHK(hipMemcpyAsync(out + o, g.probs[h->where[i].second].S, g.nst() * g.N * sizeof(double),
                            hipMemcpyDeviceToDevice, (hipStream_t)stream));
      o += g.nst() * g.N;
    }
    return ACR_OK;
  });
}

acr_status krylov_solve(acr_handle* h, int32_t method, int32_t restart, int32_t transpose, double rtol, int32_t maxit,
                        const double* b, double* x, acr_solve_info* info, void* stream) {
  return acr::solve_problems(h, method, restart, transpose, rtol, maxit, b, x, info, stream, nullptr);
}

acr_status acr_grad_kappa(acr_handle* h, const double* u, const double* lam, double* dkappa, void* stream) {
  if (!h || !u || !lam || !dkappa) return fail(ACR_E_INVALID, "null argument");
  for (size_t i = 0; i < h->where.size(); ++i) {
    const acr::Prob& P = h->groups[h->where[i].first]->probs[h->where[i].second];
    if (P.kind != ACR_POISSON_HARMONIC) return fail(ACR_E_INVALID, "gradient needs harmonic-average Poisson problems");
    if (!P.kappa) return fail(ACR_E_INVALID, "gradient needs the problem's kappa");
  }
  return guard([&]() {
    for (size_t i = 0; i < h->where.size(); ++i) {
      const acr::Handle& g = *h->groups[h->where[i].first];
      const acr::Prob& P = g.probs[h->where[i].second];
      acr::launch_grad_kappa(g.nx, g.ny, g.nz, P.kappa, u + h->off[i], lam + h->off[i], dkappa + h->grid_off[i],
                             (hipStream_t)stream);
    }
    HIPCHK(hipGetLastError());
    return ACR_OK;
  });
}

acr_status acr_plane_geometry(int32_t nx, int32_t ny, const acr_options* o, acr_geometry_info* info,
                              int32_t* perm, int32_t* leaves, int32_t leaves_cap) {
  if (!o || !info) return fail(ACR_E_INVALID, "null argument");
  if (nx < 1 || ny < 1 || (int64_t)nx * ny > (1 << 26)) return fail(ACR_E_INVALID, "plane sizes out of range");
  acr_status s = check_options(o);
  if (s != ACR_OK) return s;
  return guard([&]() {
    const acr::Geometry G = acr::build_geometry(nx, ny, o->leaf_size, o->eta, o->dense_work);
    acr_geometry_info g{};
    g.clusters = (int32_t)G.cl.size();
    g.leaf_clusters = (int32_t)G.leaf_clusters.size();
    g.depth = G.max_depth();
    g.block_nodes = (int32_t)G.bn.size();
    g.leaves = (int32_t)G.lf.size();
    for (const acr::Leaf& L : G.lf) {
      g.admissible += L.adm;
      (L.fmt == acr::LF_LR ? g.lr_leaves : g.dense_leaves)++;
    }
    *info = g;
    if (leaves && leaves_cap < g.leaves)
      throw acr::AcrError(ACR_E_INVALID, "leaves_cap is smaller than the number of leaves");
    if (perm)
      for (int i = 0; i < nx * ny; ++i) perm[i] = G.perm[i];
    if (leaves)
      for (int l = 0; l < g.leaves; ++l) {
        const acr::Leaf& L = G.lf[l];
        int32_t* o6 = leaves + 6 * (int64_t)l;
        o6[0] = L.r0;
        o6[1] = L.c0;
        o6[2] = L.m;
        o6[3] = L.n;
        o6[4] = L.adm;
        o6[5] = L.fmt == acr::LF_LR ? 1 : 0;
      }
    return ACR_OK;
  });
}

acr_status acr_stats(const acr_handle* h, acr_stats_t* st) {
  if (!h || !st) return fail(ACR_E_INVALID, "null argument");
  // one group: its statistics; several groups: sums and maxima
  *st = h->groups[0]->st;
  st->bytes_allocated = (double)h->groups[0]->bytes_alloc;
  st->bytes_peak = (double)h->groups[0]->bytes_peak;
  for (size_t g = 1; g < h->groups.size(); ++g) {
    const acr_stats_t& o = h->groups[g]->st;
    st->factors += o.factors;
    st->retries = std::max(st->retries, o.retries);
    st->rank_overflow |= o.rank_overflow;
    for (int r = 0; r < ACR_MAX_LEVELS; ++r) st->max_rank[r] = std::max(st->max_rank[r], o.max_rank[r]);
    st->max_rank_all = std::max(st->max_rank_all, o.max_rank_all);
    st->bytes_factors += o.bytes_factors;
    st->bytes_allocated += (double)h->groups[g]->bytes_alloc;
    st->bytes_peak += (double)h->groups[g]->bytes_peak;
    st->bytes_per_apply += o.bytes_per_apply;
    st->setup_seconds += o.setup_seconds;
    st->setup_flops += o.setup_flops;
    st->accum_launches += o.accum_launches;
    st->accum_seconds += o.accum_seconds;
    st->accum_flops += o.accum_flops;
    st->dense_launches += o.dense_launches;
    st->dense_seconds += o.dense_seconds;
    st->dense_flops += o.dense_flops;
    for (int c = 0; c < 4; ++c) st->setup_flops_class[c] += o.setup_flops_class[c];
    st->leaf_inverse_flops += o.leaf_inverse_flops;
    st->bytes_apply_image += o.bytes_apply_image;
    st->accum_bytes += o.accum_bytes;
    st->dense_bytes += o.dense_bytes;
    st->levels = std::max(st->levels, o.levels);
    for (int r = 0; r < ACR_MAX_LEVELS; ++r) {
      st->bytes_level[r] += o.bytes_level[r];
      st->level_seconds[r] += o.level_seconds[r];
    }
  }
  return ACR_OK;
}

int32_t acr_num_problems(const acr_handle* h) { return h ? (int32_t)h->where.size() : 0; }

void acr_destroy(acr_handle* h) {
  if (!h) return;
  (void)hipDeviceSynchronize();
  delete h;
}

}  // extern "C"
