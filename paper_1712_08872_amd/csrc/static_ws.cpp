// krylov_solve_static: krylov_solve with its work vectors, dot-product
// partials and result slots in a fixed device array instead of memory the
// library allocates, for callers that cannot allocate device memory.
//
// The array lives in this file's code object; each GPU the library runs on
// holds its own copy until the process ends.  Its device address is looked
// up once per device (hipGetSymbolAddress, with that device current) and
// only that address is used from the host: kernel arguments and copies.
// Every call on a GPU shares that GPU's array, so calls that overlap on one
// GPU (several host threads or streams at once) race.  No part of the array
// has to start at zero: every entry a solve reads it has written before.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>

#include "runtime.h"

namespace {

constexpr size_t kScratchDoubles = (size_t)ACR_STATIC_WORKSPACE_BYTES / sizeof(double);
static __device__ __align__(256) double scratch[kScratchDoubles];

constexpr int kMaxDevices = 64;
std::mutex g_mutex;
double* g_scratch[kMaxDevices] = {nullptr};

// Layout in doubles: dot partials, result slots, two tables of 8 vector
// pointers, then the work vectors from a 256-byte boundary.
constexpr size_t kPartOff = 0;
constexpr size_t kResOff = kPartOff + acr::KRYLOV_PART;
constexpr size_t kTabOff = kResOff + acr::KRYLOV_RES;
constexpr size_t kVecOff = (kTabOff + 16 + 31) / 32 * 32;
constexpr size_t kVecDoubles = kScratchDoubles - kVecOff;

// The array's device address on the current device (looked up once).
acr_status device_scratch(double** out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices)
    return acr::set_last_error(ACR_E_DEVICE, "krylov_solve_static: no usable current device");
  std::lock_guard<std::mutex> lock(g_mutex);
  if (!g_scratch[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      (void)hipGetLastError();
      return acr::set_last_error(ACR_E_DEVICE, std::string("krylov_solve_static: hipGetSymbolAddress failed: ") +
                                                   hipGetErrorString(e));
    }
    g_scratch[dev] = (double*)p;
  }
  *out = g_scratch[dev];
  return ACR_OK;
}

}  // namespace

extern "C" acr_status krylov_solve_static(acr_handle* h, int32_t method, int32_t restart, int32_t transpose,
                                          double rtol, int32_t maxit, const double* b, double* x,
                                          acr_solve_info* info, void* stream) {
  acr_status v = acr::check_solve_args(h, method, restart, rtol, maxit, b, x, info);
  if (v != ACR_OK) return v;
  int64_t nmax = 0;
  for (const auto& g : h->groups) nmax = std::max<int64_t>(nmax, g->N);
  const int nvec = acr::krylov_vectors(method, restart);
  if ((double)nvec * (double)nmax > (double)kVecDoubles)
    return acr::set_last_error(
        ACR_E_INVALID, "krylov_solve_static: " + std::to_string(nvec) + " work vectors of " + std::to_string(nmax) +
                           " doubles exceed the fixed workspace of " + std::to_string(kVecDoubles) +
                           " doubles (ACR_STATIC_WORKSPACE_BYTES); use krylov_solve");
  double* base = nullptr;
  v = device_scratch(&base);
  if (v != ACR_OK) return v;
  double hres[acr::KRYLOV_RES];  // host landing slots of the results (pageable)
  acr::KrylovBuffers wb;
  wb.part = base + kPartOff;
  wb.dres = base + kResOff;
  wb.dots_a = (const double**)(base + kTabOff);
  wb.dots_b = (const double**)(base + kTabOff + 8);
  wb.kv = base + kVecOff;
  wb.kv_len = (size_t)(kVecDoubles / (size_t)nmax);
  wb.hres = hres;
  return acr::solve_problems(h, method, restart, transpose, rtol, maxit, b, x, info, stream, &wb);
}
