// C ABI of libacr (declared in include/acr.h): argument validation on the
// host before any device work, error codes and thread-local messages, and
// the handle lifecycle.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <string>

#include "runtime.h"

namespace acr {
acr_status krylov_cg(Handle& h, bool flexible, bool tr, double rtol, int maxit, const double* b, double* x,
                     acr_solve_info* info, hipStream_t s);
acr_status krylov_gmres(Handle& h, int m, bool tr, double rtol, int maxit, const double* b, double* x,
                        acr_solve_info* info, hipStream_t s);
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
}  // namespace

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
  if (p->nx < 1 || p->ny < 1 || p->nz < 1) return fail(ACR_E_INVALID, "grid sizes must be >= 1");
  if ((int64_t)p->nx * p->ny > (1 << 26) || (int64_t)p->nx * p->ny * p->nz > ((int64_t)1 << 34))
    return fail(ACR_E_INVALID, "grid too large");
  if (p->kind < ACR_POISSON_HARMONIC || p->kind > ACR_STENCIL7_RAW) return fail(ACR_E_INVALID, "unknown problem kind");
  if (p->kind == ACR_STENCIL7_RAW && !p->stencil7) return fail(ACR_E_INVALID, "RAW problem needs stencil7");
  if (p->kind == ACR_HELMHOLTZ && (!p->c || !std::isfinite(p->omega)))
    return fail(ACR_E_INVALID, "Helmholtz problem needs c and a finite omega");
  if (p->kind == ACR_CONVDIFF_UPWIND && (!std::isfinite(p->beta_amp) || !std::isfinite(p->beta_phase)))
    return fail(ACR_E_INVALID, "convection parameters must be finite");
  if (!(o->eps > 0.0 && o->eps < 1.0)) return fail(ACR_E_INVALID, "eps must lie in (0, 1)");
  if (!finite_pos(o->eta)) return fail(ACR_E_INVALID, "eta must be positive");
  if (o->leaf_size < 4 || o->leaf_size > 64) return fail(ACR_E_INVALID, "leaf_size must lie in [4, 64]");
  if (o->precision != ACR_FP64 && o->precision != ACR_MIXED_FP32) return fail(ACR_E_INVALID, "unknown precision");
  if (o->max_rank < 0 || o->max_rank > acr::KC_MAX - 8) return fail(ACR_E_INVALID, "max_rank must lie in [0, 56]");
  if (o->dense_work < 0 || o->dense_work > 64) return fail(ACR_E_INVALID, "dense_work must lie in [0, 64]");
  if ((o->alloc == nullptr) != (o->free == nullptr)) return fail(ACR_E_INVALID, "alloc and free come together");
  if (o->flags != 0) return fail(ACR_E_INVALID, "flags must be 0");
  acr_status ds = device_check();
  if (ds != ACR_OK) return ds;
  acr_handle* h = nullptr;
  acr_status st = guard([&]() {
    h = new acr_handle();
    h->h.opt = *o;
    h->h.setup(p, (hipStream_t)stream);
    return ACR_OK;
  });
  if (st != ACR_OK) {
    delete h;
    return st;
  }
  *out = h;
  return ACR_OK;
}

acr_status acr_apply(acr_handle* h, const double* r, double* z, int32_t nrhs, void* stream) {
  if (!h || !r || !z) return fail(ACR_E_INVALID, "null argument");
  if (nrhs < 1) return fail(ACR_E_INVALID, "nrhs must be >= 1");
  if (r == z) return fail(ACR_E_INVALID, "z must not alias r");
  return guard([&]() {
    for (int k = 0; k < nrhs; ++k) h->h.apply(r + (int64_t)k * h->h.N, z + (int64_t)k * h->h.N, false, (hipStream_t)stream);
    return ACR_OK;
  });
}

acr_status acr_apply_T(acr_handle* h, const double* r, double* z, int32_t nrhs, void* stream) {
  if (!h || !r || !z) return fail(ACR_E_INVALID, "null argument");
  if (nrhs < 1) return fail(ACR_E_INVALID, "nrhs must be >= 1");
  if (r == z) return fail(ACR_E_INVALID, "z must not alias r");
  return guard([&]() {
    for (int k = 0; k < nrhs; ++k) h->h.apply(r + (int64_t)k * h->h.N, z + (int64_t)k * h->h.N, true, (hipStream_t)stream);
    return ACR_OK;
  });
}

acr_status acr_matvec(acr_handle* h, int32_t transpose, const double* x, double* y, void* stream) {
  if (!h || !x || !y) return fail(ACR_E_INVALID, "null argument");
  if (x == y) return fail(ACR_E_INVALID, "y must not alias x");
  return guard([&]() {
    h->h.matvec(x, y, transpose != 0, (hipStream_t)stream);
    return ACR_OK;
  });
}

acr_status acr_get_stencil(acr_handle* h, double* out, void* stream) {
  if (!h || !out) return fail(ACR_E_INVALID, "null argument");
  return guard([&]() {
    HIPCHK(hipMemcpyAsync(out, h->h.S, 7 * h->h.N * sizeof(double), hipMemcpyDeviceToDevice, (hipStream_t)stream));
    return ACR_OK;
  });
}

acr_status krylov_solve(acr_handle* h, int32_t method, int32_t restart, int32_t transpose, double rtol, int32_t maxit,
                        const double* b, double* x, acr_solve_info* info, void* stream) {
  if (!h || !b || !x || !info) return fail(ACR_E_INVALID, "null argument");
  if (b == x) return fail(ACR_E_INVALID, "x must not alias b");
  if (method < ACR_CG || method > ACR_GMRES) return fail(ACR_E_INVALID, "unknown method");
  if (!(rtol > 0.0 && rtol < 1.0)) return fail(ACR_E_INVALID, "rtol must lie in (0, 1)");
  if (maxit < 1) return fail(ACR_E_INVALID, "maxit must be >= 1");
  if (method == ACR_GMRES && (restart < 1 || restart > 60)) return fail(ACR_E_INVALID, "restart must lie in [1, 60]");
  std::memset(info, 0, sizeof(*info));
  acr_status result = ACR_OK;
  acr_status st = guard([&]() {
    if (method == ACR_GMRES)
      result = acr::krylov_gmres(h->h, restart, transpose != 0, rtol, maxit, b, x, info, (hipStream_t)stream);
    else
      result = acr::krylov_cg(h->h, method == ACR_FCG, transpose != 0, rtol, maxit, b, x, info, (hipStream_t)stream);
    return ACR_OK;
  });
  if (st != ACR_OK) return st;
  if (result != ACR_OK) return fail(result, std::string("krylov_solve: ") + acr_status_string(result));
  return ACR_OK;
}

acr_status acr_grad_kappa(acr_handle* h, const double* u, const double* lam, double* dkappa, void* stream) {
  if (!h || !u || !lam || !dkappa) return fail(ACR_E_INVALID, "null argument");
  if (h->h.kind != ACR_POISSON_HARMONIC) return fail(ACR_E_INVALID, "gradient needs a harmonic-average Poisson problem");
  if (!h->h.kappa) return fail(ACR_E_INVALID, "gradient needs the problem's kappa");
  return guard([&]() {
    acr::launch_grad_kappa(h->h.nx, h->h.ny, h->h.nz, h->h.kappa, u, lam, dkappa, (hipStream_t)stream);
    HIPCHK(hipGetLastError());
    return ACR_OK;
  });
}

acr_status acr_stats(const acr_handle* h, acr_stats_t* st) {
  if (!h || !st) return fail(ACR_E_INVALID, "null argument");
  *st = h->h.st;
  st->bytes_allocated = (double)h->h.bytes_alloc;
  return ACR_OK;
}

void acr_destroy(acr_handle* h) {
  if (!h) return;
  (void)hipDeviceSynchronize();
  delete h;
}

}  // extern "C"
