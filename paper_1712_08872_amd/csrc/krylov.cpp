// FP64 Krylov solvers preconditioned by ACR (Sec. 5.3: CG to a 1e-8
// relative residual in the 2-norm; Sec. 7-8: GMRES for the nonsymmetric
// and indefinite problems).
//
//   CG  : Hestenes-Stiefel recurrences, Fletcher-Reeves beta; switches to
//         the flexible Polak-Ribiere beta (FCG) when the residual has not
//         decreased for 5 iterations (an H-truncated preconditioner is only
//         approximately symmetric).
//   GMRES(m): right preconditioning (monitored residual = true residual),
//         classical Gram-Schmidt applied twice, Givens rotations on the host.
// Vectors live on the device; every iteration reads back a few scalars.
#include <hip/hip_runtime.h>

#include <cmath>
#include <vector>

#include "runtime.h"

namespace acr {

namespace {

struct KWork {
  Handle& h;
  KrylovBuffers& wb;
  const bool fixed;  // caller-given buffers of fixed size: never allocate
  hipStream_t s;
  int64_t N;
  int prob;
  KWork(Handle& hh, KrylovBuffers* ext, hipStream_t ss, int p)
      : h(hh), wb(ext ? *ext : hh.kbuf), fixed(ext != nullptr), s(ss), N(hh.N), prob(p) {}

  void ensure(size_t nvec) {
    if (wb.kv_len >= nvec) return;
    if (fixed)
      throw AcrError(ACR_E_INVALID, "the Krylov method needs " + std::to_string(nvec) + " work vectors of " +
                                        std::to_string(N) + " doubles, more than the fixed workspace holds");
    if (wb.kv) h.dfree(wb.kv);
    wb.kv = h.dnew<double>(nvec * (size_t)N);
    wb.kv_len = nvec;
    if (!wb.part) {
      wb.part = h.dnew<double>(KRYLOV_PART);
      wb.dres = h.dnew<double>(KRYLOV_RES);
      wb.dots_a = h.dnew<const double*>(8);
      wb.dots_b = h.dnew<const double*>(8);
      HIPCHK(hipHostMalloc((void**)&wb.hres, KRYLOV_RES * sizeof(double), hipHostMallocDefault));
    }
  }
  double* vec(int i) { return wb.kv + (size_t)i * N; }

  // nd dot products (a[d], b[d]) -> host
  void dots(const std::vector<const double*>& a, const std::vector<const double*>& b, double* out) {
    int nd = (int)a.size();
    HIPCHK(hipMemcpyAsync((void*)wb.dots_a, a.data(), nd * sizeof(double*), hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync((void*)wb.dots_b, b.data(), nd * sizeof(double*), hipMemcpyHostToDevice, s));
    launch_dots(wb.dots_a, wb.dots_b, nd, N, wb.part, wb.dres, s);
    HIPCHK(hipMemcpyAsync(wb.hres, wb.dres, nd * sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    for (int d = 0; d < nd; ++d) out[d] = wb.hres[d];
  }
  void A(const double* x, double* y, bool tr) { h.matvec(prob, x, y, tr, s); }
  void M(const double* x, double* y, bool tr) {
    std::vector<const double*> in(h.probs.size(), nullptr);
    std::vector<double*> out(h.probs.size(), nullptr);
    in[prob] = x;
    out[prob] = y;
    h.apply(in, out, tr, prob, s);
  }
};

}  // namespace

acr_status krylov_cg(Handle& h, KrylovBuffers* wb, int prob, bool flexible, bool tr, double rtol, int maxit,
                     const double* b, double* x, acr_solve_info* info, hipStream_t s) {
  KWork k(h, wb, s, prob);
  k.ensure(5);
  double *r = k.vec(0), *zz = k.vec(1), *p = k.vec(2), *Ap = k.vec(3), *zold = k.vec(4);
  const int64_t N = h.N;
  double d[4];
  k.dots({b}, {b}, d);
  const double nb = std::sqrt(d[0]);
  info->variant = flexible ? ACR_FCG : ACR_CG;
  if (nb == 0.0) {
    HIPCHK(hipMemsetAsync(x, 0, N * sizeof(double), s));
    info->iters = 0;
    info->relres_true = 0.0;
    info->status = ACR_OK;
    return ACR_OK;
  }
  // r = b - A x
  k.A(x, r, tr);
  launch_axpby(N, 1.0, b, -1.0, r, s);
  k.dots({r}, {r}, d);
  double relres = std::sqrt(d[0]) / nb;
  int it = 0;
  if (relres <= rtol) {
    info->iters = 0;
    info->relres_true = relres;
    info->status = ACR_OK;
    return ACR_OK;
  }
  k.M(r, zz, tr);
  HIPCHK(hipMemcpyAsync(p, zz, N * sizeof(double), hipMemcpyDeviceToDevice, s));
  k.dots({r}, {zz}, d);
  double rz = d[0];
  double best = relres;
  int stall = 0;
  acr_status stt = ACR_E_NOTCONV;
  while (it < maxit) {
    ++it;
    k.A(p, Ap, tr);
    k.dots({p}, {Ap}, d);
    const double pAp = d[0];
    if (!(pAp > 0.0) || !std::isfinite(pAp)) {
      stt = ACR_E_BREAKDOWN;
      break;
    }
    const double alpha = rz / pAp;
    launch_axpby(N, alpha, p, 1.0, x, s);
    launch_axpby(N, -alpha, Ap, 1.0, r, s);
    k.dots({r}, {r}, d);
    relres = std::sqrt(d[0]) / nb;
    if (relres <= rtol) {
      // confirm with the true residual
      k.A(x, r, tr);
      launch_axpby(N, 1.0, b, -1.0, r, s);
      k.dots({r}, {r}, d);
      relres = std::sqrt(d[0]) / nb;
      if (relres <= rtol) {
        stt = ACR_OK;
        break;
      }
    }
    if (relres < 0.99 * best) {
      best = relres;
      stall = 0;
    } else if (++stall >= 5 && !flexible) {
      flexible = true;
      info->variant = ACR_FCG;
    }
    if (flexible) HIPCHK(hipMemcpyAsync(zold, zz, N * sizeof(double), hipMemcpyDeviceToDevice, s));
    k.M(r, zz, tr);
    double beta;
    if (flexible) {
      k.dots({r, r}, {zz, zold}, d);
      beta = (d[0] - d[1]) / rz;
      rz = d[0];
    } else {
      k.dots({r}, {zz}, d);
      beta = d[0] / rz;
      rz = d[0];
    }
    launch_axpby(N, 1.0, zz, beta, p, s);
  }
  // true residual at exit
  k.A(x, r, tr);
  launch_axpby(N, 1.0, b, -1.0, r, s);
  k.dots({r}, {r}, d);
  info->iters = it;
  info->relres_true = std::sqrt(d[0]) / nb;
  info->status = stt;
  return stt;
}

acr_status krylov_gmres(Handle& h, KrylovBuffers* wb, int prob, int m, bool tr, double rtol, int maxit,
                        const double* b, double* x, acr_solve_info* info, hipStream_t s) {
  KWork k(h, wb, s, prob);
  // layout: V[0..m] (m+1 vectors), Z[0..m-1] (m vectors), r, w
  k.ensure(2 * (size_t)m + 3);
  const int64_t N = h.N;
  double* V = k.vec(0);
  double* Z = k.vec(m + 1);
  double* r = k.vec(2 * m + 1);
  double* w = k.vec(2 * m + 2);
  info->variant = ACR_GMRES;
  double d[4];
  k.dots({b}, {b}, d);
  const double nb = std::sqrt(d[0]);
  if (nb == 0.0) {
    HIPCHK(hipMemsetAsync(x, 0, N * sizeof(double), s));
    info->iters = 0;
    info->relres_true = 0.0;
    info->status = ACR_OK;
    return ACR_OK;
  }
  std::vector<double> H((size_t)(m + 1) * m), cs(m), sn(m), gv(m + 1), hcol(m + 1), h2(m + 1);
  // device coefficient vector (m + 1 <= 61 entries of the KRYLOV_RES = 64)
  double* dcoef = k.wb.dres;
  int it = 0;
  acr_status stt = ACR_E_NOTCONV;
  double relres = 1.0;
  while (true) {
    k.A(x, r, tr);
    launch_axpby(N, 1.0, b, -1.0, r, s);
    k.dots({r}, {r}, d);
    const double beta = std::sqrt(d[0]);
    relres = beta / nb;
    if (relres <= rtol) {
      stt = ACR_OK;
      break;
    }
    if (it >= maxit) break;
    launch_axpby(N, 1.0 / beta, r, 0.0, V, s);
    std::fill(gv.begin(), gv.end(), 0.0);
    gv[0] = beta;
    int kk = 0;
    bool done = false;
    while (kk < m && it < maxit) {
      double* vk = V + (size_t)kk * N;
      double* zk = Z + (size_t)kk * N;
      k.M(vk, zk, tr);
      k.A(zk, w, tr);
      // classical Gram-Schmidt, twice
      for (int pass = 0; pass < 2; ++pass) {
        launch_multi_dot(N, kk + 1, V, N, w, k.wb.part, dcoef, s);
        HIPCHK(hipMemcpyAsync(k.wb.hres, dcoef, (kk + 1) * sizeof(double), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        for (int i = 0; i <= kk; ++i) (pass ? h2 : hcol)[i] = k.wb.hres[i];
        launch_multi_axpy(N, kk + 1, V, N, dcoef, w, -1.0, s);
      }
      for (int i = 0; i <= kk; ++i) hcol[i] += h2[i];
      k.dots({w}, {w}, d);
      const double hn = std::sqrt(d[0]);
      if (hn > 0.0) launch_axpby(N, 1.0 / hn, w, 0.0, V + (size_t)(kk + 1) * N, s);
      // apply previous rotations and form the new one
      for (int i = 0; i < kk; ++i) {
        double a = hcol[i], c = hcol[i + 1];
        hcol[i] = cs[i] * a + sn[i] * c;
        hcol[i + 1] = -sn[i] * a + cs[i] * c;
      }
      double den = std::hypot(hcol[kk], hn);
      if (den > 0.0) {
        cs[kk] = hcol[kk] / den;
        sn[kk] = hn / den;
      } else {
        cs[kk] = 1.0;
        sn[kk] = 0.0;
      }
      hcol[kk] = den;
      for (int i = 0; i <= kk; ++i) H[(size_t)i * m + kk] = hcol[i];
      gv[kk + 1] = -sn[kk] * gv[kk];
      gv[kk] = cs[kk] * gv[kk];
      ++kk;
      ++it;
      if (std::fabs(gv[kk]) / nb <= rtol || hn == 0.0) {
        done = true;
        break;
      }
    }
    // y = R^{-1} g ; x += Z y
    std::vector<double> y(kk);
    for (int i = kk - 1; i >= 0; --i) {
      double acc = gv[i];
      for (int j = i + 1; j < kk; ++j) acc -= H[(size_t)i * m + j] * y[j];
      y[i] = H[(size_t)i * m + i] != 0.0 ? acc / H[(size_t)i * m + i] : 0.0;
    }
    HIPCHK(hipMemcpyAsync(dcoef, y.data(), kk * sizeof(double), hipMemcpyHostToDevice, s));
    launch_lincomb(N, kk, Z, N, dcoef, 1.0, x, s);
    HIPCHK(hipStreamSynchronize(s));
    (void)done;
  }
  info->iters = it;
  info->relres_true = relres;
  info->status = stt;
  return stt;
}

}  // namespace acr
