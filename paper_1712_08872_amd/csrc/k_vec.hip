// Grid kernels: 7-point assembly (Sec. 6 harmonic-average Poisson, Sec. 7
// upwind convection-diffusion, Sec. 8 Helmholtz shift), stencil
// matrix-vector products, the adjoint gradient stencil, plane permutations
// and FP64 reductions for the Krylov solvers.  All memory-bound; one
// thread per grid node, x fastest so that loads coalesce.
#include <hip/hip_runtime.h>

#include <cstdint>

namespace acr {

__device__ __forceinline__ double harm(double a, double b) { return 2.0 * a * b / (a + b); }

// S rows: 0 centre, 1 x-1, 2 x+1, 3 y-1, 4 y+1, 5 z-1, 6 z+1
__global__ void assemble_kernel(int kind, int nx, int ny, int nz, const double* kappa, double beta_amp,
                                double beta_phase, const double* c, double omega, double* S) {
  const int64_t N = (int64_t)nx * ny * nz;
  const double hx = 1.0 / (nx + 1), hy = 1.0 / (ny + 1), hz = 1.0 / (nz + 1);
  const int sx = nx + 2, sy = ny + 2;
  for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < N; p += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(p % nx), j = (int)((p / nx) % ny), k = (int)(p / ((int64_t)nx * ny));
    const int64_t q = (int64_t)(i + 1) + sx * ((int64_t)(j + 1) + (int64_t)sy * (k + 1));
    const double kc = kappa ? kappa[q] : 1.0;
    const int64_t nb[6] = {q - 1, q + 1, q - sx, q + sx, q - (int64_t)sx * sy, q + (int64_t)sx * sy};
    const bool in[6] = {i > 0, i < nx - 1, j > 0, j < ny - 1, k > 0, k < nz - 1};
    const double h2[3] = {hx * hx, hy * hy, hz * hz};
    double diag = 0.0, off[6];
    for (int d = 0; d < 6; ++d) {
      const double kn = kappa ? kappa[nb[d]] : 1.0;
      const double w = harm(kc, kn) / h2[d >> 1];
      diag += w;
      off[d] = in[d] ? -w : 0.0;
    }
    if (kind == 1) {  // upwind convection, beta_d(x) identical in d = x, y, z
      const double x = (i + 1) * hx;
      const double b = beta_amp * (1.0 + 0.5 * sin(2.0 * M_PI * x + beta_phase));
      const double bp = b > 0.0 ? b : 0.0, bm = b < 0.0 ? b : 0.0;
      const double hh[3] = {hx, hy, hz};
      for (int a = 0; a < 3; ++a) {
        diag += (bp - bm) / hh[a];
        if (in[2 * a]) off[2 * a] += -bp / hh[a];
        if (in[2 * a + 1]) off[2 * a + 1] += bm / hh[a];
      }
    } else if (kind == 2) {
      const double cc = c[q];
      diag -= omega * omega / (cc * cc);
    } else if (kind == 3) {  // alpha b(x).grad u, b the recirculating flow of wavenumber a = beta_phase
      const double w2 = 2.0 * M_PI * beta_phase;
      const double x = (i + 1) * hx, y = (j + 1) * hy, z = (k + 1) * hz;
      const double sx0 = sin(w2 * x), cx0 = cos(w2 * x);
      const double sy8 = sin(w2 * (0.125 + y)), cy8 = cos(w2 * (0.125 + y));
      const double sz8 = sin(w2 * (0.125 + z)), cz8 = cos(w2 * (0.125 + z));
      const double sz0 = sin(w2 * z), cz0 = cos(w2 * z);
      const double bv[3] = {beta_amp * (sx0 * sy8 + sz8 * sx0), beta_amp * (cx0 * cy8 + cy8 * cz0),
                            beta_amp * (cx0 * cz8 + sy8 * sz0)};
      const double hh[3] = {hx, hy, hz};
      for (int a = 0; a < 3; ++a) {
        const double bp = bv[a] > 0.0 ? bv[a] : 0.0, bm = bv[a] < 0.0 ? bv[a] : 0.0;
        diag += (bp - bm) / hh[a];
        if (in[2 * a]) off[2 * a] += -bp / hh[a];
        if (in[2 * a + 1]) off[2 * a + 1] += bm / hh[a];
      }
    }
    S[p] = diag;
    for (int d = 0; d < 6; ++d) S[(int64_t)(d + 1) * N + p] = off[d];
  }
}

// y = A x (transpose = 0) or A^T x (transpose = 1)
__global__ void stencil_mv_kernel(const double* __restrict__ S, int nx, int ny, int nz, int transpose,
                                  const double* __restrict__ x, double* __restrict__ y) {
  const int64_t N = (int64_t)nx * ny * nz;
  const int64_t P = (int64_t)nx * ny;
  for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < N; p += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(p % nx), j = (int)((p / nx) % ny), k = (int)(p / P);
    double s = S[p] * x[p];
    if (!transpose) {
      if (i > 0) s += S[N + p] * x[p - 1];
      if (i < nx - 1) s += S[2 * N + p] * x[p + 1];
      if (j > 0) s += S[3 * N + p] * x[p - nx];
      if (j < ny - 1) s += S[4 * N + p] * x[p + nx];
      if (k > 0) s += S[5 * N + p] * x[p - P];
      if (k < nz - 1) s += S[6 * N + p] * x[p + P];
    } else {  // (A^T x)_p = sum_q A_qp x_q: neighbour q's coupling towards p
      if (i > 0) s += S[2 * N + p - 1] * x[p - 1];
      if (i < nx - 1) s += S[N + p + 1] * x[p + 1];
      if (j > 0) s += S[4 * N + p - nx] * x[p - nx];
      if (j < ny - 1) s += S[3 * N + p + nx] * x[p + nx];
      if (k > 0) s += S[6 * N + p - P] * x[p - P];
      if (k < nz - 1) s += S[5 * N + p + P] * x[p + P];
    }
    y[p] = s;
  }
}

// ---------------------------------------------------------------- 27-point
// Trilinear (Q1) finite elements for -Lap u - omega^2 / c^2 u (Sec. 8, eq.
// HelmVarVel; the 27-point scheme on hexahedra).  Row p is the sum over the
// 8 elements around node p of K_e - M_e: the Q1 stiffness of -Lap, products
// of the 1D element matrices k = [[1, -1], [-1, 1]] / h and
// m = [[2, 1], [1, 2]] h / 6, minus the mass weighted by omega^2 / c^2 with
// the 2 x 2 x 2 Gauss rule, c interpolated trilinearly from the element's
// node values.  S row m = (dx+1) + 3 (dy+1) + 9 (dz+1) holds the coupling to
// the neighbour at offset (dx, dy, dz); couplings to boundary nodes are 0.
__global__ void assemble27_kernel(int nx, int ny, int nz, const double* c, double omega, double* S) {
  const int64_t N = (int64_t)nx * ny * nz;
  const double hx = 1.0 / (nx + 1), hy = 1.0 / (ny + 1), hz = 1.0 / (nz + 1);
  const double hh[3] = {hx, hy, hz};
  const int sx = nx + 2, sy = ny + 2;
  const double gp[2] = {0.5 - 0.5 / sqrt(3.0), 0.5 + 0.5 / sqrt(3.0)};
  const double wq = hx * hy * hz / 8.0;
  for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < N; p += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(p % nx), j = (int)((p / nx) % ny), k = (int)(p / ((int64_t)nx * ny));
    const int I = i + 1, J = j + 1, K = k + 1;  // node-grid coordinates
    double acc[27];
#pragma unroll
    for (int m = 0; m < 27; ++m) acc[m] = 0.0;
    for (int e = 0; e < 8; ++e) {
      // element with first node (ex, ey, ez); p is its local node a
      const int ax = e & 1, ay = (e >> 1) & 1, az = e >> 2;
      const int ex = I - ax, ey = J - ay, ez = K - az;
      const int a = ax + 2 * ay + 4 * az;
      double ce[8], mab[8];
#pragma unroll
      for (int b = 0; b < 8; ++b) {
        ce[b] = c[(ex + (b & 1)) + (int64_t)sx * ((ey + ((b >> 1) & 1)) + (int64_t)sy * (ez + (b >> 2)))];
        mab[b] = 0.0;
      }
      for (int qz = 0; qz < 2; ++qz)
        for (int qy = 0; qy < 2; ++qy)
          for (int qx = 0; qx < 2; ++qx) {
            const double xi[3] = {gp[qx], gp[qy], gp[qz]};
            double phi[8], cq = 0.0;
#pragma unroll
            for (int b = 0; b < 8; ++b) {
              const double fx = (b & 1) ? xi[0] : 1.0 - xi[0];
              const double fy = ((b >> 1) & 1) ? xi[1] : 1.0 - xi[1];
              const double fz = (b >> 2) ? xi[2] : 1.0 - xi[2];
              phi[b] = fx * fy * fz;
            }
#pragma unroll
            for (int b = 0; b < 8; ++b) cq += phi[b] * ce[b];
            const double kq = omega * omega / (cq * cq) * wq;
#pragma unroll
            for (int b = 0; b < 8; ++b) mab[b] += kq * (phi[a] * phi[b]);
          }
#pragma unroll
      for (int b = 0; b < 8; ++b) {
        const int bx = b & 1, by = (b >> 1) & 1, bz = b >> 2;
        const int dx = bx - ax, dy = by - ay, dz = bz - az;
        const int ii = i + dx, jj = j + dy, kk = k + dz;
        if (ii < 0 || ii >= nx || jj < 0 || jj >= ny || kk < 0 || kk >= nz) continue;
        const int aa[3] = {ax, ay, az}, bb[3] = {bx, by, bz};
        double kd[3], md[3];
        for (int d = 0; d < 3; ++d) {
          kd[d] = (aa[d] == bb[d] ? 1.0 : -1.0) / hh[d];
          md[d] = (aa[d] == bb[d] ? 2.0 : 1.0) * hh[d] / 6.0;
        }
        const double kab = kd[0] * md[1] * md[2] + md[0] * kd[1] * md[2] + md[0] * md[1] * kd[2];
        acc[(dx + 1) + 3 * (dy + 1) + 9 * (dz + 1)] += kab - mab[b];
      }
    }
#pragma unroll
    for (int m = 0; m < 27; ++m) S[(int64_t)m * N + p] = acc[m];
  }
}

// y = A x (transpose = 0) or A^T x (transpose = 1) with a 27-point stencil
// (row m = (dx+1) + 3 (dy+1) + 9 (dz+1)); the transpose reads the
// neighbour's coupling of the opposite offset, row 26 - m.
__global__ void stencil27_mv_kernel(const double* __restrict__ S, int nx, int ny, int nz, int transpose,
                                    const double* __restrict__ x, double* __restrict__ y) {
  const int64_t N = (int64_t)nx * ny * nz;
  for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < N; p += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(p % nx), j = (int)((p / nx) % ny), k = (int)(p / ((int64_t)nx * ny));
    double s = 0.0;
    for (int m = 0; m < 27; ++m) {
      const int dx = m % 3 - 1, dy = (m / 3) % 3 - 1, dz = m / 9 - 1;
      if (i + dx < 0 || i + dx >= nx || j + dy < 0 || j + dy >= ny || k + dz < 0 || k + dz >= nz) continue;
      const int64_t q = p + dx + (int64_t)nx * (dy + (int64_t)ny * dz);
      s += (transpose ? S[(int64_t)(26 - m) * N + q] : S[(int64_t)m * N + p]) * x[q];
    }
    y[p] = s;
  }
}

// dJ/dkappa_m = -sum over faces (m,o) of dkf/dkm / h^2 *
//   ( [m interior] lam_m (u_m - u_o) + [o interior] lam_o (u_o - u_m) ),
// u = lam = 0 on the boundary; dkf/dkm = 2 kappa_o^2 / (kappa_m + kappa_o)^2.
__global__ void grad_kappa_kernel(int nx, int ny, int nz, const double* kappa, const double* u, const double* lam,
                                  double* g) {
  const int sx = nx + 2, sy = ny + 2, sz = nz + 2;
  const int64_t M = (int64_t)sx * sy * sz;
  // 1/h^2 per axis
  const double h2[3] = {(nx + 1.0) * (nx + 1.0), (ny + 1.0) * (ny + 1.0), (nz + 1.0) * (nz + 1.0)};
  for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < M; q += (int64_t)gridDim.x * blockDim.x) {
    const int I = (int)(q % sx), J = (int)((q / sx) % sy), K = (int)(q / ((int64_t)sx * sy));
    const bool min_ = I >= 1 && I <= nx && J >= 1 && J <= ny && K >= 1 && K <= nz;
    const double km = kappa[q];
    double um = 0.0, lm = 0.0;
    if (min_) {
      const int64_t p = (I - 1) + (int64_t)nx * ((J - 1) + (int64_t)ny * (K - 1));
      um = u[p];
      lm = lam[p];
    }
    double acc = 0.0;
    const int dI[6] = {-1, 1, 0, 0, 0, 0}, dJ[6] = {0, 0, -1, 1, 0, 0}, dK[6] = {0, 0, 0, 0, -1, 1};
    for (int d = 0; d < 6; ++d) {
      const int I2 = I + dI[d], J2 = J + dJ[d], K2 = K + dK[d];
      if (I2 < 0 || I2 >= sx || J2 < 0 || J2 >= sy || K2 < 0 || K2 >= sz) continue;
      const bool oin = I2 >= 1 && I2 <= nx && J2 >= 1 && J2 <= ny && K2 >= 1 && K2 <= nz;
      // a coupling of A joins an interior node to one of its six
      // neighbours, so at least one end of the face must be interior
      if (!min_ && !oin) continue;
      const int64_t q2 = I2 + (int64_t)sx * (J2 + (int64_t)sy * K2);
      const double ko = kappa[q2];
      double uo = 0.0, lo = 0.0;
      if (oin) {
        const int64_t p2 = (I2 - 1) + (int64_t)nx * ((J2 - 1) + (int64_t)ny * (K2 - 1));
        uo = u[p2];
        lo = lam[p2];
      }
      const double dk = 2.0 * ko * ko / ((km + ko) * (km + ko));
      double t = 0.0;
      if (min_) t += lm * (um - uo);
      if (oin) t += lo * (uo - um);
      acc -= dk * h2[d >> 1] * t;
    }
    g[q] = acc;
  }
}

// H-order plane vectors <-> natural ordering: h[k*B + i] = n[k*B + perm[i]]
__global__ void to_horder_kernel(const double* n, double* h, const int32_t* perm, int B, int64_t N) {
  for (int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g < N; g += (int64_t)gridDim.x * blockDim.x) {
    const int64_t k = g / B;
    const int i = (int)(g - k * B);
    h[g] = n[k * B + perm[i]];
  }
}
__global__ void from_horder_kernel(const double* h, double* n, const int32_t* perm, int B, int64_t N) {
  for (int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g < N; g += (int64_t)gridDim.x * blockDim.x) {
    const int64_t k = g / B;
    const int i = (int)(g - k * B);
    n[k * B + perm[i]] = h[g];
  }
}

// ---------------------------------------------------------------- BLAS-1
// Deterministic dot products: fixed grid, per-block partials, second pass
// in one block.  `nd` dot products of pairs (a[d], b[d]) at once.
constexpr int DOT_BLOCKS = 1024;

__global__ __launch_bounds__(256) void dot_partial_kernel(const double* const* a, const double* const* b, int nd,
                                                          int64_t n, double* part) {
  __shared__ double red[256];
  for (int d = 0; d < nd; ++d) {
    const double* x = a[d];
    const double* y = b[d];
    double s = 0.0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
      s += x[i] * y[i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
      if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
      __syncthreads();
    }
    if (threadIdx.x == 0) part[(int64_t)d * gridDim.x + blockIdx.x] = red[0];
    __syncthreads();
  }
}

__global__ __launch_bounds__(256) void dot_final_kernel(const double* part, int nparts, int nd, double* out) {
  __shared__ double red[256];
  for (int d = 0; d < nd; ++d) {
    double s = 0.0;
    for (int i = threadIdx.x; i < nparts; i += blockDim.x) s += part[(int64_t)d * nparts + i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
      if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
      __syncthreads();
    }
    if (threadIdx.x == 0) out[d] = red[0];
    __syncthreads();
  }
}

// y = a*x + b*y; with b = 0, y is not read (y = a*x), so a work vector
// whose memory still holds a non-finite value from earlier use is simply
// overwritten (0 * Inf would be NaN)
__global__ void axpby_kernel(int64_t n, double a, const double* x, double b, double* y) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    y[i] = b == 0.0 ? a * x[i] : a * x[i] + b * y[i];
}

// w = x - sum_j h[j] V[j]  (GMRES orthogonalisation update; V rows of length n)
__global__ void multi_axpy_kernel(int64_t n, int nv, const double* V, int64_t ldv, const double* h, double* w,
                                  double sign) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    double s = 0.0;
    for (int j = 0; j < nv; ++j) s += h[j] * V[(int64_t)j * ldv + i];
    w[i] += sign * s;
  }
}

// h[j] = V[j] . w for j < nv (partials per block; final pass by dot_final)
__global__ __launch_bounds__(256) void multi_dot_partial_kernel(int64_t n, int nv, const double* V, int64_t ldv,
                                                                const double* w, double* part) {
  __shared__ double red[256];
  for (int j = 0; j < nv; ++j) {
    double s = 0.0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
      s += V[(int64_t)j * ldv + i] * w[i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
      if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
      __syncthreads();
    }
    if (threadIdx.x == 0) part[(int64_t)j * gridDim.x + blockIdx.x] = red[0];
    __syncthreads();
  }
}

// y = sum_j c[j] V[j] + beta*y
__global__ void lincomb_kernel(int64_t n, int nv, const double* V, int64_t ldv, const double* c, double beta,
                               double* y) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    double s = 0.0;
    for (int j = 0; j < nv; ++j) s += c[j] * V[(int64_t)j * ldv + i];
    y[i] = beta == 0.0 ? s : s + beta * y[i];
  }
}

__global__ void check_finite_positive_kernel(const double* x, int64_t n, int positive, int32_t* flag) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    double v = x[i];
    if (!isfinite(v) || (positive && !(v > 0.0))) atomicOr(flag, 1);
  }
}

// ---------------------------------------------------------------- launchers
static inline int grid_for(int64_t n, int bs = 256) {
  int64_t g = (n + bs - 1) / bs;
  if (g > 16384) g = 16384;
  if (g < 1) g = 1;
  return (int)g;
}

void launch_assemble(int kind, int nx, int ny, int nz, const double* kappa, double ba, double bph, const double* c,
                     double omega, double* S, hipStream_t s) {
  int64_t N = (int64_t)nx * ny * nz;
  hipLaunchKernelGGL(assemble_kernel, dim3(grid_for(N)), dim3(256), 0, s, kind, nx, ny, nz, kappa, ba, bph, c, omega,
                     S);
}
void launch_stencil_mv(const double* S, int nx, int ny, int nz, int tr, const double* x, double* y, hipStream_t s) {
  int64_t N = (int64_t)nx * ny * nz;
  hipLaunchKernelGGL(stencil_mv_kernel, dim3(grid_for(N)), dim3(256), 0, s, S, nx, ny, nz, tr, x, y);
}
void launch_assemble27(int nx, int ny, int nz, const double* c, double omega, double* S, hipStream_t s) {
  const int64_t N = (int64_t)nx * ny * nz;
  hipLaunchKernelGGL(assemble27_kernel, dim3(grid_for(N)), dim3(256), 0, s, nx, ny, nz, c, omega, S);
}
void launch_stencil27_mv(const double* S, int nx, int ny, int nz, int tr, const double* x, double* y, hipStream_t s) {
  const int64_t N = (int64_t)nx * ny * nz;
  hipLaunchKernelGGL(stencil27_mv_kernel, dim3(grid_for(N)), dim3(256), 0, s, S, nx, ny, nz, tr, x, y);
}
void launch_grad_kappa(int nx, int ny, int nz, const double* kappa, const double* u, const double* lam, double* g,
                       hipStream_t s) {
  int64_t M = (int64_t)(nx + 2) * (ny + 2) * (nz + 2);
  hipLaunchKernelGGL(grad_kappa_kernel, dim3(grid_for(M)), dim3(256), 0, s, nx, ny, nz, kappa, u, lam, g);
}
void launch_to_horder(const double* n, double* h, const int32_t* perm, int B, int64_t N, hipStream_t s) {
  hipLaunchKernelGGL(to_horder_kernel, dim3(grid_for(N)), dim3(256), 0, s, n, h, perm, B, N);
}
void launch_from_horder(const double* h, double* n, const int32_t* perm, int B, int64_t N, hipStream_t s) {
  hipLaunchKernelGGL(from_horder_kernel, dim3(grid_for(N)), dim3(256), 0, s, h, n, perm, B, N);
}
void launch_dots(const double* const* a, const double* const* b, int nd, int64_t n, double* part, double* out,
                 hipStream_t s) {
  hipLaunchKernelGGL(dot_partial_kernel, dim3(DOT_BLOCKS), dim3(256), 0, s, a, b, nd, n, part);
  hipLaunchKernelGGL(dot_final_kernel, dim3(1), dim3(256), 0, s, part, DOT_BLOCKS, nd, out);
}
void launch_axpby(int64_t n, double a, const double* x, double b, double* y, hipStream_t s) {
  hipLaunchKernelGGL(axpby_kernel, dim3(grid_for(n)), dim3(256), 0, s, n, a, x, b, y);
}
void launch_multi_dot(int64_t n, int nv, const double* V, int64_t ldv, const double* w, double* part, double* out,
                      hipStream_t s) {
  hipLaunchKernelGGL(multi_dot_partial_kernel, dim3(DOT_BLOCKS), dim3(256), 0, s, n, nv, V, ldv, w, part);
  hipLaunchKernelGGL(dot_final_kernel, dim3(1), dim3(256), 0, s, part, DOT_BLOCKS, nv, out);
}
void launch_multi_axpy(int64_t n, int nv, const double* V, int64_t ldv, const double* h, double* w, double sign,
                       hipStream_t s) {
  hipLaunchKernelGGL(multi_axpy_kernel, dim3(grid_for(n)), dim3(256), 0, s, n, nv, V, ldv, h, w, sign);
}
void launch_lincomb(int64_t n, int nv, const double* V, int64_t ldv, const double* c, double beta, double* y,
                    hipStream_t s) {
  hipLaunchKernelGGL(lincomb_kernel, dim3(grid_for(n)), dim3(256), 0, s, n, nv, V, ldv, c, beta, y);
}
void launch_check(const double* x, int64_t n, int positive, int32_t* flag, hipStream_t s) {
  hipLaunchKernelGGL(check_finite_positive_kernel, dim3(grid_for(n)), dim3(256), 0, s, x, n, positive, flag);
}

}  // namespace acr
