// H-arithmetic kernels for gfx950: batched accumulation of formatted
// products into H-matrix leaves with truncation, dense leaf inversion and
// the level-0 conversion of the plane operators.
//
// A step of formatted H-arithmetic (a product or a stage of the recursive
// inverse, expanded on the host into targets and pieces) runs as two
// launches over (batch item x target): accum_dense_kernel sums every dense
// target and, exactly, every small low-rank target that receives more
// columns than its smaller dimension; accum_kernel then compresses those
// dense sums and builds the other low-rank targets by appending piece
// columns and recompressing every ROUND columns.
//
// Truncation T_eps (Sec. 3.1.5, Sec. 4.3 of the paper: block-wise relative
// accuracy, singular values sigma_i > eps sigma_1 kept) of a block given as
// U V^T with K columns (the block's current factors concatenated with the
// incoming contributions): the column pairs are norm-balanced, the Gram
// matrices G_U = U^T U and G_V = V^T V are formed in FP64 (on the FP64
// matrix cores, like the final product with the factors), each is factored
// by Cholesky with symmetric pivoting, stopped at its numerical rank
// (G = P R^T R P^T, so U = Q_U R_U P^T with Q_U = U_piv R_U11^-1); the
// small core C = R_U P_U^T P_V R_V^T is reduced by Cholesky with symmetric
// pivoting of C^T C at (0.01 eps)^2 of its largest diagonal, the rest
// diagonalised by one-sided (Hestenes) Jacobi, and U' = Q_U W_k S_k,
// V' = Q_V Z_k are formed by triangular solves and one product with the
// concatenated factors.  This is the truncated SVD of U V^T; through the
// Gram matrices it resolves singular values down to about 1e-8 sigma_1.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

#include "hprog.h"

// The accumulation kernel is compiled once per round width KCV (the widest
// low-rank concatenation held in LDS): a narrow round keeps the LDS
// footprint small enough for several resident blocks per CU.
#ifndef KCV
#define KCV 64
#endif
#define ACR_CAT2(a, b) a##b
#define ACR_CAT(a, b) ACR_CAT2(a, b)
#define KCNS ACR_CAT(kc, KCV)

namespace acr {
namespace KCNS {
constexpr int KC = KCV;

// ------------------------------------------------------------ utilities
template <typename T>
__device__ __forceinline__ int inst_of(const AccumArgs<T>& A, int b, int role) {
  return role < 0 ? -1 : A.role_inst[b * A.nroles + role];
}

template <typename T>
__device__ __forceinline__ T* leaf_base(const AccumArgs<T>& A, int inst, int leaf) {
  return A.inst_base[inst] + A.leaves[leaf].off;
}

template <typename T>
__device__ __forceinline__ int rank_of(const AccumArgs<T>& A, int inst, int leaf) {
  return A.inst_rank[inst][leaf];
}

// Operand view of a stored leaf: dense data or the U / V factors with their
// leading dimensions, in either the capacity layout (V after cap columns of
// U) or the packed layout (exact rank, leading dimensions padded to 4).
template <typename T>
struct LeafRef {
  const T* U;
  const T* V;
  int ldu, ldv;
};

template <typename T>
__device__ __forceinline__ LeafRef<T> leaf_ref(const AccumArgs<T>& A, int inst, int leaf, const DLeaf& L) {
  LeafRef<T> r;
  const int64_t* po = A.inst_off[inst];
  if (po) {
    r.ldu = (L.m + 3) & ~3;
    r.ldv = (L.n + 3) & ~3;
    r.U = A.inst_base[inst] + po[leaf];
    r.V = r.U + (int64_t)r.ldu * (L.fmt ? A.inst_rank[inst][leaf] : 0);
  } else {
    r.ldu = L.m;
    r.ldv = L.n;
    r.U = A.inst_base[inst] + L.off;
    r.V = r.U + (int64_t)L.m * L.cap;
  }
  return r;
}

// Arithmetic type of the staged piece products: FP32 for FP32 factors
// (products accumulated in FP32), FP64 otherwise.
template <typename T>
struct CompT {
  using type = double;
};
template <>
struct CompT<float> {
  using type = float;
};

__device__ __forceinline__ int imax(int a, int b) { return a > b ? a : b; }
__device__ __forceinline__ int imin(int a, int b) { return a < b ? a : b; }

// Round-robin (tournament) pairing of K' = K + (K odd) indices: round r,
// pair i.  Every unordered pair appears exactly once in K'-1 rounds.
__device__ __forceinline__ void rr_pair(int Kp, int r, int i, int& p, int& q) {
  int M = Kp - 1;
  p = (i == 0) ? 0 : ((i - 1 + r) % M) + 1;
  q = ((Kp - 2 - i + r) % M) + 1;
}

#ifndef ACR_ROUND
#define ACR_ROUND 32
#endif
constexpr int ROUND = ACR_ROUND;  // columns appended between recompressions
constexpr int DACC_MAX = DACC_ELEMS;  // largest m*n of a low-rank target accumulated densely
constexpr int LDM = KC + 1;  // padded leading dimension of the K x K matrices (no LDS bank conflicts)

struct Lds {
  double S0[KC * LDM];
  double S1[KC * LDM];
  double S2[KC * LDM];
  double S3[KC * LDM];
  double v0[KC], v1[KC];
  int permU[KC], permV[KC], posU[KC], posV[KC], order[KC], permC[KC], posC[KC];
  int ival[8];
  double dval[4];
  double flops[FC_COUNT];  // algorithmic flops of the block's items by class (thread 0)
  double bytes;            // algorithmic operand and target bytes of the block's items (thread 0)
};

// LDS of the accumulate-only kernel: the staging tiles of the piece
// products only (no truncation workspace).
template <typename CT>
struct LdsPiece {
  CT S0[KC * LDM];
  CT S1[KC * LDM];
  CT S2[KC * LDM];
  double flops[FC_COUNT];
  double bytes;
};

#define FLOP(L_, c_, x_)                    \
  do {                                      \
    if (threadIdx.x == 0) (L_).flops[c_] += (double)(x_); \
  } while (0)
// algorithmic bytes, counted only when the counters are on
#define BYTES(A_, L_, x_)                                     \
  do {                                                        \
    if ((A_).flops && threadIdx.x == 0) (L_).bytes += (double)(x_); \
  } while (0)

// The tall products of a truncation on the FP64 matrix cores
// (v_mfma_f64_16x16x4: lane l supplies A[l % 16][l / 16] and B[l / 16][l % 16],
// accumulator element r of lane l is row l / 16 + 4 r, column l % 16), the
// operands read straight from the scratch, no LDS staging and no barrier
// inside.  Both factors of the block at once, so that all four wavefronts
// have work.
typedef double f64x4 __attribute__((ext_vector_type(4)));

// G_U = U^T U and G_V = V^T V of the first K columns (U: m rows, V: n rows,
// row-major ld KC) into GU, GV (LDS, ld LDM): 16 x 16 tiles of the upper
// triangles over the wavefronts, 4 rows per step, mirrored below the
// diagonal tiles.
template <typename T>
__device__ void gram2(const T* U, int m, const T* V, int n, int K, double* GU, double* GV) {
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int l16 = lane & 15, g = lane >> 4;
  const int nt = (K + 15) >> 4, nu = nt * (nt + 1) / 2;
  for (int u = w; u < 2 * nu; u += TPB / 64) {
    const bool second = u >= nu;
    const T* X = second ? V : U;
    const int rows = second ? n : m;
    double* G = second ? GV : GU;
    int ti = 0, rem = second ? u - nu : u;
    while (rem >= nt - ti) {
      rem -= nt - ti;
      ++ti;
    }
    const int tj = ti + rem;
    const int ci = ti * 16 + l16, cj = tj * 16 + l16;
    const bool ai = ci < K, bj = cj < K;
    f64x4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll 4
    for (int r0 = 0; r0 < rows; r0 += 4) {
      const int row = r0 + g;
      const bool in = row < rows;
      const double a = (ai && in) ? (double)X[(int64_t)row * KC + ci] : 0.0;
      const double b = (bj && in) ? (double)X[(int64_t)row * KC + cj] : 0.0;
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int i = ti * 16 + g + 4 * r, j = cj;
      if (i < K && j < K) {
        G[i * LDM + j] = acc[r];
        if (ti != tj) G[j * LDM + i] = acc[r];  // a diagonal tile holds both halves itself
      }
    }
  }
  __syncthreads();
}

// In place U[:, 0:k] = U[:, 0:K] RU and V[:, 0:k] = V[:, 0:K] RV (RU, RV:
// K x k in LDS, ld LDM): a wavefront owns 16 rows and forms all their k
// columns (at most four 16-column tiles) before it writes any of them.
template <typename T>
__device__ void rebuild2(T* U, int m, T* V, int n, int K, int k, const double* RU, const double* RV) {
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int l16 = lane & 15, g = lane >> 4;
  const int nct = (k + 15) >> 4;
  const int nbu = (m + 15) >> 4, nb = nbu + ((n + 15) >> 4);
  for (int u = w; u < nb; u += TPB / 64) {
    const bool second = u >= nbu;
    T* X = second ? V : U;
    const int rows = second ? n : m;
    const double* R = second ? RV : RU;
    const int rb = (second ? u - nbu : u) * 16;
    const int row = rb + l16;
    const bool rin = row < rows;
    f64x4 acc[4];
#pragma unroll
    for (int ct = 0; ct < 4; ++ct) acc[ct] = f64x4{0.0, 0.0, 0.0, 0.0};
    for (int a0 = 0; a0 < K; a0 += 4) {
      const int a = a0 + g;
      const bool kin = a < K;
      const double av = (rin && kin) ? (double)X[(int64_t)row * KC + a] : 0.0;
#pragma unroll
      for (int ct = 0; ct < 4; ++ct) {
        if (ct < nct) {
          const int c = ct * 16 + l16;
          const double bv = (kin && c < k) ? R[a * LDM + c] : 0.0;
          acc[ct] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc[ct], 0, 0, 0);
        }
      }
    }
#pragma unroll
    for (int ct = 0; ct < 4; ++ct) {
      if (ct < nct) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int i = rb + g + 4 * r, c = ct * 16 + l16;
          if (i < rows && c < k) X[(int64_t)i * KC + c] = (T)acc[ct][r];
        }
      }
    }
  }
  __syncthreads();
}

// Ordering point inside one wavefront: the LDS accesses of a wavefront are
// executed in program order, the fences keep the compiler from moving them
// across this point.
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Cholesky factorisation with symmetric pivoting of the K x K (K <= 64)
// symmetric positive semi-definite G (LDS, ld KC), in place, by ONE
// wavefront (lane j owns column j): on exit the rows a < r of the upper
// trapezoid hold R (pivot order), perm[a] is the original index of pivot a,
// pos[] its inverse.  Stops when the largest remaining diagonal entry is <=
// rel_tol times the largest initial one; returns r (the same in all lanes).
__device__ int wave_pivoted_cholesky(double* G, int K, int* perm, int* pos, double rel_tol) {
  const int lane = threadIdx.x & 63;
  if (lane < K) perm[lane] = lane;
  double dm = lane < K ? G[lane * LDM + lane] : 0.0;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) dm = fmax(dm, __shfl_xor(dm, o));
  const double tol = rel_tol * dm;
  wave_sync();
  int r = 0;
  for (int a = 0; a < K; ++a) {
    double v = (lane >= a && lane < K) ? G[lane * LDM + lane] : -1.0;
    int idx = lane;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      const double v2 = __shfl_xor(v, o);
      const int i2 = __shfl_xor(idx, o);
      if (v2 > v || (v2 == v && i2 < idx)) {
        v = v2;
        idx = i2;
      }
    }
    if (!(v > tol && v > 0.0)) break;
    const int p = idx;
    if (p != a) {
      if (lane < K) {
        const double t = G[a * LDM + lane];
        G[a * LDM + lane] = G[p * LDM + lane];
        G[p * LDM + lane] = t;
      }
      wave_sync();
      if (lane < K) {
        const double t = G[lane * LDM + a];
        G[lane * LDM + a] = G[lane * LDM + p];
        G[lane * LDM + p] = t;
      }
      if (lane == 0) {
        const int t = perm[a];
        perm[a] = perm[p];
        perm[p] = t;
      }
      wave_sync();
    }
    const double rd = sqrt(G[a * LDM + a]);
    wave_sync();
    if (lane >= a && lane < K) G[a * LDM + lane] = (lane == a) ? rd : G[a * LDM + lane] / rd;
    wave_sync();
    if (lane > a && lane < K) {
      const double rj = G[a * LDM + lane];
      for (int i = a + 1; i < K; ++i) G[i * LDM + lane] -= G[a * LDM + i] * rj;
    }
    wave_sync();
    r = a + 1;
  }
  if (lane < K) pos[perm[lane]] = lane;
  wave_sync();
  return r;
}

// One-sided Jacobi (Hestenes) on the columns of C (rows x cols, LDS ld KC):
// C <- C Z with orthogonal columns, Z accumulated (initialised by the
// caller; Z may be null).  Column pairs in tournament order, one pair per group of 8 lanes
// (up to 32 pairs per round across the block), dot products reduced with
// lane shuffles, one barrier per round.  Pairs whose inner product is below
// 1e-15 of the geometric mean of their norms, or below 1e-18 ||C||_F^2,
// count as orthogonal.  Returns the number of sweeps.
__device__ int onesided_jacobi(double* C, double* Z, int rows, int cols, int* sflag, double* dval) {
  const int tid = threadIdx.x;
  if (cols <= 1) return 0;
  if (tid < 64) {
    double f = 0.0;
    for (int e = tid; e < rows * cols; e += 64) {
      const double x = C[(e / cols) * LDM + (e % cols)];
      f += x * x;
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) f += __shfl_xor(f, o);
    if (tid == 0) dval[1] = 1e-18 * f;
  }
  __syncthreads();
  const double cabs = dval[1];
  const int Kp = cols + (cols & 1), np = Kp / 2;
  const int g = tid >> 3, l = tid & 7;
  int sweep = 0;
  for (; sweep < 30; ++sweep) {
    if (tid == 0) *sflag = 0;
    __syncthreads();
    for (int r = 0; r < Kp - 1; ++r) {
      if (g < np) {
        int p, q;
        rr_pair(Kp, r, g, p, q);
        if (p > q) {
          const int t = p;
          p = q;
          q = t;
        }
        if (q < cols) {
          double a = 0.0, b = 0.0, c = 0.0;
          for (int i = l; i < rows; i += 8) {
            const double x = C[i * LDM + p], y = C[i * LDM + q];
            a += x * x;
            b += y * y;
            c += x * y;
          }
#pragma unroll
          for (int o = 1; o < 8; o <<= 1) {
            a += __shfl_xor(a, o);
            b += __shfl_xor(b, o);
            c += __shfl_xor(c, o);
          }
          if (fabs(c) > 1e-15 * sqrt(a * b) && fabs(c) > cabs) {
            const double zeta = (b - a) / (2.0 * c);
            const double t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
            const double cs = 1.0 / sqrt(1.0 + t * t), sn = cs * t;
            for (int i = l; i < rows; i += 8) {
              const double x = C[i * LDM + p], y = C[i * LDM + q];
              C[i * LDM + p] = cs * x - sn * y;
              C[i * LDM + q] = sn * x + cs * y;
            }
            if (Z)
              for (int i = l; i < cols; i += 8) {
                const double x = Z[i * LDM + p], y = Z[i * LDM + q];
                Z[i * LDM + p] = cs * x - sn * y;
                Z[i * LDM + q] = sn * x + cs * y;
              }
            if (l == 0) *sflag = 1;
          }
        }
      }
      __syncthreads();
    }
    const int f = *sflag;
    __syncthreads();
    if (!f) break;
  }
  return sweep + 1;
}

// T_eps of Us Vs^T (m x K and n x K row-major scratch); on exit the first k
// columns hold the truncated factors (singular values folded into U).
// Returns k.
#define PROF_ADD(slot, v) \
  do {                     \
    if (prof && threadIdx.x == 0) atomicAdd(&prof[slot], (unsigned long long)(v)); \
  } while (0)

template <typename T, bool BF = false>
__device__ int truncate_block(T* Us, T* Vs, int m, int n, int K, double eps, Lds& L, int32_t* flags,
                              unsigned long long* prof = nullptr) {
  const int tid = threadIdx.x;
  if (K == 0) return 0;
  long long t0 = clock64();
  PROF_ADD(PS_TRUNC, 1);
  PROF_ADD(PS_KSUM, K);
  gram2(Us, m, Vs, n, K, L.S2, L.S0);
  FLOP(L, FC_GRAM, (double)(m + n) * K * (K + 1));
  long long t1 = clock64();
  PROF_ADD(PS_GRAM, t1 - t0);
  // norm balancing of the column pairs: d_j = sqrt(|v_j| / |u_j|)
  if (tid < K) {
    const double nu = L.S2[tid * LDM + tid], nv = L.S0[tid * LDM + tid];
    const double d = (nu > 0.0 && nv > 0.0 && isfinite(nu) && isfinite(nv)) ? sqrt(sqrt(nv / nu)) : 0.0;
    L.v0[tid] = d;
    if (!isfinite(nu) || !isfinite(nv)) atomicOr(&flags[FL_NONFINITE], 1);
  }
  __syncthreads();
  for (int idx = tid; idx < K * K; idx += TPB) {
    const int i = idx / K, j = idx - i * K;
    const double di = L.v0[i], dj = L.v0[j];
    L.S2[i * LDM + j] *= di * dj;
    L.S0[i * LDM + j] = (di > 0.0 && dj > 0.0) ? L.S0[i * LDM + j] / (di * dj) : 0.0;
  }
  __syncthreads();
  // the two factorisations run concurrently on waves 0 and 1
  if (tid < 64) {
    const int r = wave_pivoted_cholesky(L.S2, K, L.permU, L.posU, 1e-16);
    if (tid == 0) L.ival[0] = r;
  } else if (tid < 128) {
    const int r = wave_pivoted_cholesky(L.S0, K, L.permV, L.posV, 1e-16);
    if (tid == 64) L.ival[1] = r;
  }
  __syncthreads();
  const int rU = L.ival[0], rV = L.ival[1];
  FLOP(L, FC_CORE, (double)K * K * (rU + rV));
  long long t2 = clock64();
  PROF_ADD(PS_EIG1, t2 - t1);
  if (rU == 0 || rV == 0) return 0;
  // core C = R_U P_U^T P_V R_V^T (rU x rV) -> S1
  for (int idx = tid; idx < rU * rV; idx += TPB) {
    const int a = idx / rV, c = idx - a * rV;
    double s = 0.0;
    for (int j = 0; j < K; ++j) {
      const int pu = L.posU[j], pv = L.posV[j];
      if (pu >= a && pv >= c) s += L.S2[a * LDM + pu] * L.S0[c * LDM + pv];
    }
    L.S1[a * LDM + c] = s;
  }
  __syncthreads();
  FLOP(L, FC_CORE, 2.0 * rU * rV * K);
  // Rank pre-reduction of the core: Cholesky with symmetric pivoting of
  // H = C^T C, stopped once every remaining diagonal entry is below
  // (0.01 eps)^2 max diag(H).  The dropped part E of C then has
  // ||E||_F <= sqrt(rV) 0.01 eps sigma_1, far below the truncation level,
  // and C ~ Q M with M = R_C P_C^T (r' x rV).  The rotations act on the
  // r' columns of M^T only: M^T W = Z S gives the right singular vectors
  // Z and the singular values S, and C Z the left ones (times S).
  constexpr int PER = (KC * KC + TPB - 1) / TPB;
  const double ptol = 1e-4 * eps * eps;
  int rr = rV;
  bool reduced = false;
  if (rV > 8 && ptol > 1e-15) {
    for (int idx = tid; idx < rV * rV; idx += TPB) {
      const int a = idx / rV, c = idx - a * rV;
      double s = 0.0;
      for (int i = 0; i < rU; ++i) s += L.S1[i * LDM + a] * L.S1[i * LDM + c];
      L.S3[a * LDM + c] = s;
    }
    __syncthreads();
    if (tid < 64) {
      const int r = wave_pivoted_cholesky(L.S3, rV, L.permC, L.posC, ptol);
      if (tid == 0) L.ival[6] = r;
    }
    __syncthreads();
    const int rp = L.ival[6];
    FLOP(L, FC_CORE, (double)rU * rV * rV + (double)rV * rV * rp);
    if (rp > 0 && rp + 3 <= rV) {
      // M^T (rV x r'): row i is column pos_C(i) of the pivot-ordered R_C
      double tmp[PER];
#pragma unroll
      for (int e = 0; e < PER; ++e) {
        const int idx = tid + e * TPB;
        tmp[e] = 0.0;
        if (idx < rV * rp) {
          const int i = idx / rp, a = idx - i * rp, pc = L.posC[i];
          tmp[e] = pc >= a ? L.S3[a * LDM + pc] : 0.0;
        }
      }
      __syncthreads();
#pragma unroll
      for (int e = 0; e < PER; ++e) {
        const int idx = tid + e * TPB;
        if (idx < rV * rp) {
          const int i = idx / rp, a = idx - i * rp;
          L.S3[i * LDM + a] = tmp[e];
        }
      }
      __syncthreads();
      reduced = true;
      rr = rp;
    }
  }
  if (!reduced) {  // Z = I -> S3
    for (int idx = tid; idx < rV * rV; idx += TPB) {
      const int a = idx / rV, c = idx - a * rV;
      L.S3[a * LDM + c] = (a == c) ? 1.0 : 0.0;
    }
    __syncthreads();
  }
  const int sweeps = reduced ? onesided_jacobi(L.S3, nullptr, rV, rr, &L.ival[4], L.dval)
                             : onesided_jacobi(L.S1, L.S3, rU, rV, &L.ival[4], L.dval);
  PROF_ADD(PS_SWEEPS, sweeps);
  const int jrows = reduced ? rV : rU;
  FLOP(L, FC_CORE, (double)sweeps * (rr / 2) * (rr - 1 + (rr & 1)) * (12.0 * jrows + (reduced ? 0.0 : 6.0 * rV)));
  // singular values = column norms of the rotated matrix; order, rank
  const double* Rot = reduced ? L.S3 : L.S1;
  if (tid < rr) {
    double s = 0.0;
    for (int i = 0; i < jrows; ++i) s += Rot[i * LDM + tid] * Rot[i * LDM + tid];
    L.v1[tid] = sqrt(s);
  }
  __syncthreads();
  if (tid < rr) {
    const double sa = L.v1[tid];
    int rnk = 0;
    for (int b2 = 0; b2 < rr; ++b2) {
      const double sb = L.v1[b2];
      if (sb > sa || (sb == sa && b2 < tid)) ++rnk;
    }
    L.order[rnk] = tid;
  }
  __syncthreads();
  if (tid == 0) {
    const double s1 = L.v1[L.order[0]];
    int k = 0;
    if (s1 > 0.0 && isfinite(s1))
      while (k < rr && L.v1[L.order[k]] > eps * s1) ++k;
    if (!isfinite(s1)) atomicOr(&flags[FL_NONFINITE], 1);
    L.ival[2] = k;
  }
  __syncthreads();
  if (reduced) {
    // right singular vectors: rotated columns / sigma (S3, rV rows); left
    // ones times sigma: C Z -> the same columns of S1 (rU rows)
    const int kk = L.ival[2];
    for (int idx = tid; idx < rV * rr; idx += TPB) {
      const int i = idx / rr, a = idx - i * rr;
      const double sg = L.v1[a];
      L.S3[i * LDM + a] = sg > 0.0 ? L.S3[i * LDM + a] / sg : 0.0;
    }
    __syncthreads();
    double tmp[PER];
#pragma unroll
    for (int e = 0; e < PER; ++e) {
      const int idx = tid + e * TPB;
      tmp[e] = 0.0;
      if (idx < rU * kk) {
        const int i = idx / kk, a = L.order[idx - i * kk];
        double s = 0.0;
        for (int j = 0; j < rV; ++j) s += L.S1[i * LDM + j] * L.S3[j * LDM + a];
        tmp[e] = s;
      }
    }
    __syncthreads();
#pragma unroll
    for (int e = 0; e < PER; ++e) {
      const int idx = tid + e * TPB;
      if (idx < rU * kk) {
        const int i = idx / kk, a = L.order[idx - i * kk];
        L.S1[i * LDM + a] = tmp[e];
      }
    }
    __syncthreads();
    FLOP(L, FC_CORE, 2.0 * rU * rV * kk);
  }
  const int k = L.ival[2];
  if (k == 0) return 0;
  // back substitution R_U11 y = C[:, order[c]] and R_V11 y = Z[:, order[c]],
  // in place, one thread per column
  if (tid < k) {
    const int c = L.order[tid];
    for (int a = rU - 1; a >= 0; --a) {
      double s = L.S1[a * LDM + c];
      for (int b2 = a + 1; b2 < rU; ++b2) s -= L.S2[a * LDM + b2] * L.S1[b2 * LDM + c];
      L.S1[a * LDM + c] = s / L.S2[a * LDM + a];
    }
  } else if (tid >= 64 && tid < 64 + k) {
    const int c = L.order[tid - 64];
    for (int a = rV - 1; a >= 0; --a) {
      double s = L.S3[a * LDM + c];
      for (int b2 = a + 1; b2 < rV; ++b2) s -= L.S0[a * LDM + b2] * L.S3[b2 * LDM + c];
      L.S3[a * LDM + c] = s / L.S0[a * LDM + a];
    }
  }
  __syncthreads();
  // coefficient matrices in the original column order (balancing included):
  // X_U -> S2, X_V -> S0
  for (int idx = tid; idx < K * k; idx += TPB) {
    const int j = idx / k, c = idx - j * k;
    const int pu = L.posU[j], pv = L.posV[j];
    const double d = L.v0[j];
    const int oc = L.order[c];
    L.S2[j * LDM + c] = (pu < rU) ? d * L.S1[pu * LDM + oc] : 0.0;
    L.S0[j * LDM + c] = (pv < rV && d > 0.0) ? L.S3[pv * LDM + oc] / d : 0.0;
  }
  __syncthreads();
  long long t3 = clock64();
  PROF_ADD(PS_EIG2, t3 - t2);
  rebuild2(Us, m, Vs, n, K, k, L.S2, L.S0);
  FLOP(L, FC_REBUILD, (double)k * (rU * rU + rV * rV) + 2.0 * (m + n) * K * k);
  PROF_ADD(PS_REBUILD, clock64() - t3);
  return k;
}

// ------------------------------------------------------------ pieces
// Number of columns a piece contributes to a low-rank target.
template <typename T>
__device__ int piece_width(const AccumArgs<T>& A, int b, const Piece& P) {
  switch (P.kind) {
    case PK_LRX: {
      int xi = inst_of(A, b, P.xrole), yi = inst_of(A, b, P.yrole);
      return (xi < 0 || yi < 0) ? 0 : rank_of(A, xi, P.xleaf);
    }
    case PK_LRY: {
      int xi = inst_of(A, b, P.xrole), yi = inst_of(A, b, P.yrole);
      return (xi < 0 || yi < 0) ? 0 : rank_of(A, yi, P.yleaf);
    }
    case PK_DD: {
      int xi = inst_of(A, b, P.xrole), yi = inst_of(A, b, P.yrole);
      return (xi < 0 || yi < 0) ? 0 : (P.wc1 - P.wc0);
    }
    case PK_COPY: {
      int si = inst_of(A, b, P.xrole);
      if (si < 0) return 0;
      return A.leaves[P.xleaf].fmt == 1 ? rank_of(A, si, P.xleaf) : A.leaves[P.xleaf].n;
    }
  }
  return 0;
}

// One 16 x 16 x 4 matrix-core step in the compute type: lane l supplies
// A[l % 16][l / 16] and B[l / 16][l % 16]; element r of the lane's
// accumulator is row row(l / 16, r), column l % 16 of the 16 x 16 tile
// (4 (l / 16) + r for FP32, l / 16 + 4 r for FP64, as measured on gfx950).
template <typename CT>
struct Mfma16;
template <>
struct Mfma16<float> {
  typedef float v4 __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ v4 step(float a, float b, v4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int g, int r) { return 4 * g + r; }
};
template <>
struct Mfma16<double> {
  typedef double v4 __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ v4 step(double a, double b, v4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int g, int r) { return g + 4 * r; }
};

// BF16 operands of the 16 x 16 x 16 matrix-core step (FP32 accumulation):
// lane l supplies A[l % 16][4 (l / 16) + e] and B[4 (l / 16) + e][l % 16],
// e < 4; the accumulator layout is that of the FP32 16 x 16 x 4 step (row
// 4 (l / 16) + r, column l % 16), as measured on gfx950.
typedef short bf16x4_t __attribute__((ext_vector_type(4)));
__device__ __forceinline__ short bf16_rne(float f) {  // round to nearest even (finite inputs)
  uint32_t u = __float_as_uint(f);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (short)(u >> 16);
}

// One 16 x 16 tile of Us Vs^T over `take` columns with BF16 operands, lane
// layout as above.  Not inlined: inside the accumulate-only kernel its
// conversions push the register allocation into heavy spilling.
__device__ __attribute__((noinline)) Mfma16<float>::v4 bf16_outer_tile(const float* ui, const float* vj, bool ai,
                                                                      bool bj, int take, int g) {
  Mfma16<float>::v4 acc = {0, 0, 0, 0};
  for (int k0 = 0; k0 < take; k0 += 16) {
    bf16x4_t a4, b4;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int k = k0 + 4 * g + e;
      const bool in = k < take;
      a4[e] = bf16_rne((ai && in) ? ui[k] : 0.0f);
      b4[e] = bf16_rne((bj && in) ? vj[k] : 0.0f);
    }
    acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a4, b4, acc, 0, 0, 0);
  }
  return acc;
}

// Out[i][j] = sum_q P[q + i*ldp] * R[q + j*ldr] for i < mo, j < no (both
// operands contiguous along q) on the matrix cores: 16 x 16 output tiles,
// the operands read straight from memory (a lane takes 4 consecutive q of
// one column, consumed by 4 steps), 16 q per chunk.  With fewer than four
// tiles the chunks of a tile are split over the wavefronts and the partial
// tiles added in a fixed order in LDS (`bP`, >= 4 x 256 elements).  Out is
// LDS with leading dimension KC; mo, no <= KC.
template <typename T, bool BF = false>
__device__ void tn_product(const T* P, int64_t ldp, const T* R, int64_t ldr, int nq, int mo, int no,
                           typename CompT<T>::type* Out, typename CompT<T>::type* bP,
                           typename CompT<T>::type* bR, unsigned long long* prof) {
  using CT = typename CompT<T>::type;
  using MF = Mfma16<CT>;
  using V = typename MF::v4;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int l16 = lane & 15, g = lane >> 4;
  const long long tp0 = clock64();
  const int ntn = (no + 15) >> 4, nt = ((mo + 15) >> 4) * ntn;
  const int nparts = nt >= 4 ? 1 : 4 / nt;
  const int nchunk = (nq + 15) >> 4;
  __syncthreads();  // the caller's last reads of Out / bP are done
  for (int u = w; u < nt * nparts; u += TPB / 64) {
    const int t = u % nt, part = u / nt;
    const int ti = t / ntn, tj = t - ti * ntn;
    const int i = ti * 16 + l16, j = tj * 16 + l16;
    const bool ai = i < mo, bj = j < no;
    const T* pa = P + (int64_t)i * ldp;
    const T* pb = R + (int64_t)j * ldr;
    V acc = {0, 0, 0, 0};
    bool done = false;
    if constexpr (sizeof(CT) == 4 && BF) {
      {  // BF16 operands, one 16 x 16 x 16 step per chunk
#pragma unroll 1
        for (int c = part; c < nchunk; c += nparts) {
          const int q = c * 16 + 4 * g;
          bf16x4_t a4, b4;
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const bool in = q + e < nq;
            a4[e] = bf16_rne((ai && in) ? (float)pa[q + e] : 0.0f);
            b4[e] = bf16_rne((bj && in) ? (float)pb[q + e] : 0.0f);
          }
          acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a4, b4, acc, 0, 0, 0);
        }
        done = true;
      }
    }
    if (!done) {
#pragma unroll 1
      for (int c = part; c < nchunk; c += nparts) {
        const int q = c * 16 + 4 * g;
        CT av[4], bv[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const bool in = q + e < nq;
          av[e] = (ai && in) ? (CT)pa[q + e] : (CT)0;
          bv[e] = (bj && in) ? (CT)pb[q + e] : (CT)0;
        }
#pragma unroll
        for (int e = 0; e < 4; ++e) acc = MF::step(av[e], bv[e], acc);
      }
    }
    if (nparts == 1) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int ii = ti * 16 + MF::row(g, r), jj = tj * 16 + l16;
        if (ii < mo && jj < no) Out[ii * KC + jj] = acc[r];
      }
    } else {
#pragma unroll
      for (int r = 0; r < 4; ++r) bP[u * 256 + MF::row(g, r) * 16 + l16] = acc[r];
    }
  }
  if (nparts > 1) {
    __syncthreads();
    // tile t's partials are units t, t + nt, ...
    for (int idx = tid; idx < nt * 256; idx += TPB) {
      const int t = idx >> 8, e = idx & 255;
      const int ti = t / ntn, tj = t - ti * ntn;
      const int ii = ti * 16 + (e >> 4), jj = tj * 16 + (e & 15);
      if (ii < mo && jj < no) {
        CT sum = 0;
        for (int p = 0; p < nparts; ++p) sum += bP[(t + p * nt) * 256 + e];
        Out[ii * KC + jj] = sum;
      }
    }
  }
  __syncthreads();
  PROF_ADD(PS_TN, clock64() - tp0);
}

// dst[i*drs + j*dcs] += alpha * sum_a M[i + a*ldm] * Z[a*KC + j] for i < mi,
// a < na (<= KC), j < no (<= KC); M contiguous along i, Z in LDS.  `bM` is
// an LDS staging buffer of KC x KC doubles.
template <typename T>
__device__ void nn_acc(const T* M, int64_t ldm, int mi, int na, const typename CompT<T>::type* Z, int no, T* dst,
                       int64_t drs, int64_t dcs, double alpha, typename CompT<T>::type* bM,
                       unsigned long long* prof) {
  using CT = typename CompT<T>::type;
  const int tid = threadIdx.x;
  const long long tp0 = clock64();
  for (int i0 = 0; i0 < mi; i0 += KC) {
    const int ni = imin(KC, mi - i0);
    for (int idx = tid; idx < ni * na; idx += TPB) {
      const int ii = idx % ni, a = idx / ni;
      bM[a * KC + ii] = (CT)M[(i0 + ii) + (int64_t)a * ldm];
    }
    __syncthreads();
    for (int idx = tid; idx < ni * no; idx += TPB) {
      const int j = idx % no, ii = idx / no;
      CT s = 0;
      for (int a = 0; a < na; ++a) s += bM[a * KC + ii] * Z[a * KC + j];
      T* d = dst + (int64_t)(i0 + ii) * drs + (int64_t)j * dcs;
      *d = (T)((double)*d + alpha * s);
    }
    __syncthreads();
  }
  PROF_ADD(PS_NN, clock64() - tp0);
}

// One-leaf list whose overlap with the piece fits one staging tile: the
// product is formed in one LDS round and its rows are written directly.
//   LRX: U part = alpha U_x (window rows); V part on the window columns =
//        lam^T V_x, i.e. V_l (U_l^T V_x) for a low-rank lam.
//   LRY: V part = V_y (window columns); U part on the window rows =
//        alpha lam U_y, i.e. alpha U_l (V_l^T U_y) for a low-rank lam.
// Returns false when the piece does not qualify (the general path runs).
template <typename T, typename LT>
__device__ bool lrx_single(const AccumArgs<T>& A, const Piece& P, const DLeaf& tc, const DLeaf& x,
                           const LeafRef<T>& xr, int yi, int j0, int take, T* Us, T* Vs, int K, LT& L) {
  using CT = typename CompT<T>::type;
  CT* S0c = reinterpret_cast<CT*>(L.S0);
  CT* S1c = reinterpret_cast<CT*>(L.S1);
  CT* S2c = reinterpret_cast<CT*>(L.S2);
  if (P.l1 - P.l0 != 1) return false;
  const int l = A.lists[P.l0];
  const DLeaf lam = A.leaves[l];
  const int cA = imax(lam.c0, P.wc0), cB = imin(lam.c0 + lam.n, P.wc1);
  const int q0 = imax(lam.r0, x.c0), q1 = imin(lam.r0 + lam.m, x.c0 + x.n);
  const int nq = q1 - q0, nc = cB - cA;
  const int kl = lam.fmt ? rank_of(A, yi, l) : 0;
  if (nq <= 0 || nq > KC || nc <= 0 || (lam.fmt ? kl > KC : nc > KC)) return false;
  const int tid = threadIdx.x;
  const int m = tc.m, n = tc.n;
  const double alpha = P.alpha;
  const LeafRef<T> lr = leaf_ref(A, yi, l, lam);
  const T* vx = xr.V + (q0 - x.c0) + (int64_t)j0 * xr.ldv;
  for (int idx = tid; idx < m * take; idx += TPB) {
    const int i = idx / take, jj = idx - i * take;
    const int gi = tc.r0 + i;
    const double v =
        (gi >= P.wr0 && gi < P.wr1) ? alpha * (CT)xr.U[(gi - x.r0) + (int64_t)(j0 + jj) * xr.ldu] : 0.0;
    Us[(int64_t)i * KC + K + jj] = (T)v;
  }
  for (int idx = tid; idx < n * take; idx += TPB) {
    const int c = idx / take, jj = idx - c * take;
    const int gc = tc.c0 + c;
    if (gc < cA || gc >= cB) Vs[(int64_t)c * KC + K + jj] = (T)0;
  }
  for (int idx = tid; idx < nq * take; idx += TPB) {
    const int q = idx % nq, jj = idx / nq;
    S2c[q * KC + jj] = (CT)vx[q + (int64_t)jj * xr.ldv];
  }
  if (lam.fmt) {
    for (int idx = tid; idx < nq * kl; idx += TPB) {
      const int q = idx % nq, a = idx / nq;
      S1c[q * KC + a] = (CT)lr.U[(q0 - lam.r0) + q + (int64_t)a * lr.ldu];
    }
  } else {
    for (int idx = tid; idx < nq * nc; idx += TPB) {
      const int q = idx % nq, cc = idx / nq;
      S1c[q * KC + cc] = (CT)lr.U[(q0 - lam.r0) + q + (int64_t)(cA - lam.c0 + cc) * lr.ldu];
    }
  }
  __syncthreads();
  if (lam.fmt) {
    for (int idx = tid; idx < kl * take; idx += TPB) {
      const int a = idx / take, jj = idx - a * take;
      CT s = 0;
      for (int q = 0; q < nq; ++q) s += S1c[q * KC + a] * S2c[q * KC + jj];
      S0c[a * KC + jj] = s;
    }
    __syncthreads();
    for (int idx = tid; idx < nc * take; idx += TPB) {
      const int cc = idx / take, jj = idx - cc * take;
      CT s = 0;
      for (int a = 0; a < kl; ++a) s += (CT)lr.V[(cA - lam.c0 + cc) + (int64_t)a * lr.ldv] * S0c[a * KC + jj];
      Vs[(int64_t)(cA - tc.c0 + cc) * KC + K + jj] = (T)s;
    }
    FLOP(L, FC_PRODUCT, 2.0 * kl * take * (nq + nc));
    BYTES(A, L, (double)kl * (nq + nc) * sizeof(T));
  } else {
    for (int idx = tid; idx < nc * take; idx += TPB) {
      const int cc = idx / take, jj = idx - cc * take;
      CT s = 0;
      for (int q = 0; q < nq; ++q) s += S1c[q * KC + cc] * S2c[q * KC + jj];
      Vs[(int64_t)(cA - tc.c0 + cc) * KC + K + jj] = (T)s;
    }
    FLOP(L, FC_PRODUCT, 2.0 * nq * nc * take);
    BYTES(A, L, (double)nq * nc * sizeof(T));
  }
  return true;
}

template <typename T, typename LT>
__device__ bool lry_single(const AccumArgs<T>& A, const Piece& P, const DLeaf& tc, const DLeaf& y,
                           const LeafRef<T>& yr, int xi, int j0, int take, T* Us, T* Vs, int K, LT& L) {
  using CT = typename CompT<T>::type;
  CT* S0c = reinterpret_cast<CT*>(L.S0);
  CT* S1c = reinterpret_cast<CT*>(L.S1);
  CT* S2c = reinterpret_cast<CT*>(L.S2);
  if (P.l1 - P.l0 != 1) return false;
  const int l = A.lists[P.l0];
  const DLeaf lam = A.leaves[l];
  const int rA = imax(lam.r0, P.wr0), rB = imin(lam.r0 + lam.m, P.wr1);
  const int q0 = imax(lam.c0, y.r0), q1 = imin(lam.c0 + lam.n, y.r0 + y.m);
  const int nq = q1 - q0, nr = rB - rA;
  const int kl = lam.fmt ? rank_of(A, xi, l) : 0;
  if (nq <= 0 || nq > KC || nr <= 0 || (lam.fmt ? kl > KC : nr > KC)) return false;
  const int tid = threadIdx.x;
  const int m = tc.m, n = tc.n;
  const double alpha = P.alpha;
  const LeafRef<T> lr = leaf_ref(A, xi, l, lam);
  const T* uy = yr.U + (q0 - y.r0) + (int64_t)j0 * yr.ldu;
  for (int idx = tid; idx < n * take; idx += TPB) {
    const int c = idx / take, jj = idx - c * take;
    const int gc = tc.c0 + c;
    const double v = (gc >= P.wc0 && gc < P.wc1) ? (CT)yr.V[(gc - y.c0) + (int64_t)(j0 + jj) * yr.ldv] : 0.0;
    Vs[(int64_t)c * KC + K + jj] = (T)v;
  }
  for (int idx = tid; idx < m * take; idx += TPB) {
    const int i = idx / take, jj = idx - i * take;
    const int gi = tc.r0 + i;
    if (gi < rA || gi >= rB) Us[(int64_t)i * KC + K + jj] = (T)0;
  }
  for (int idx = tid; idx < nq * take; idx += TPB) {
    const int q = idx % nq, jj = idx / nq;
    S2c[q * KC + jj] = (CT)uy[q + (int64_t)jj * yr.ldu];
  }
  if (lam.fmt) {
    for (int idx = tid; idx < nq * kl; idx += TPB) {
      const int q = idx % nq, a = idx / nq;
      S1c[q * KC + a] = (CT)lr.V[(q0 - lam.c0) + q + (int64_t)a * lr.ldv];
    }
  } else {
    for (int idx = tid; idx < nq * nr; idx += TPB) {
      const int r = idx % nr, q = idx / nr;
      S1c[q * KC + r] = (CT)lr.U[(rA - lam.r0) + r + (int64_t)(q0 - lam.c0 + q) * lr.ldu];
    }
  }
  __syncthreads();
  if (lam.fmt) {
    for (int idx = tid; idx < kl * take; idx += TPB) {
      const int a = idx / take, jj = idx - a * take;
      CT s = 0;
      for (int q = 0; q < nq; ++q) s += S1c[q * KC + a] * S2c[q * KC + jj];
      S0c[a * KC + jj] = s;
    }
    __syncthreads();
    for (int idx = tid; idx < nr * take; idx += TPB) {
      const int r = idx / take, jj = idx - r * take;
      CT s = 0;
      for (int a = 0; a < kl; ++a) s += (CT)lr.U[(rA - lam.r0) + r + (int64_t)a * lr.ldu] * S0c[a * KC + jj];
      Us[(int64_t)(rA - tc.r0 + r) * KC + K + jj] = (T)(alpha * s);
    }
    FLOP(L, FC_PRODUCT, 2.0 * kl * take * (nq + nr));
    BYTES(A, L, (double)kl * (nq + nr) * sizeof(T));
  } else {
    for (int idx = tid; idx < nr * take; idx += TPB) {
      const int r = idx / take, jj = idx - r * take;
      CT s = 0;
      for (int q = 0; q < nq; ++q) s += S1c[q * KC + r] * S2c[q * KC + jj];
      Us[(int64_t)(rA - tc.r0 + r) * KC + K + jj] = (T)(alpha * s);
    }
    FLOP(L, FC_PRODUCT, 2.0 * nq * nr * take);
    BYTES(A, L, (double)nq * nr * sizeof(T));
  }
  return true;
}

// Write columns [j0, j0+take) of a piece into scratch columns [K, K+take)
// of Us (target rows) and Vs (target columns), row-major ld KC.  The alpha
// of the piece is folded into Us.  LDS buffers S0 (products), S1, S2
// (staging) are used.
template <bool BF, typename T, typename LT>
__device__ void piece_columns(const AccumArgs<T>& A, int b, const Piece& P, const DLeaf& tc, int j0, int take,
                              T* Us, T* Vs, int K, LT& L) {
  using CT = typename CompT<T>::type;
  CT* S0c = reinterpret_cast<CT*>(L.S0);
  CT* S1c = reinterpret_cast<CT*>(L.S1);
  CT* S2c = reinterpret_cast<CT*>(L.S2);
  const int tid = threadIdx.x;
  const int m = tc.m, n = tc.n;
  const double alpha = P.alpha;
  unsigned long long* prof = A.prof;
  const long long tpc = clock64();
  if (P.kind == PK_LRX) {
    const int xi = inst_of(A, b, P.xrole), yi = inst_of(A, b, P.yrole);
    const DLeaf x = A.leaves[P.xleaf];
    const LeafRef<T> xr = leaf_ref(A, xi, P.xleaf, x);
    const T* Ux = xr.U;
    const T* Vx = xr.V;
    BYTES(A, L, (double)take * ((P.wr1 - P.wr0) + x.n) * sizeof(T));  // U_x window rows, V_x
    if (lrx_single(A, P, tc, x, xr, yi, j0, take, Us, Vs, K, L)) {
      __syncthreads();
      PROF_ADD(PS_LRX, clock64() - tpc);
      return;
    }
    for (int idx = tid; idx < m * take; idx += TPB) {
      const int i = idx / take, jj = idx - i * take;
      const int gi = tc.r0 + i;
      const double v =
          (gi >= P.wr0 && gi < P.wr1) ? alpha * (CT)Ux[(gi - x.r0) + (int64_t)(j0 + jj) * xr.ldu] : 0.0;
      Us[(int64_t)i * KC + K + jj] = (T)v;
    }
    for (int idx = tid; idx < n * take; idx += TPB) {
      const int c = idx / take, jj = idx - c * take;
      Vs[(int64_t)c * KC + K + jj] = (T)0;
    }
    __syncthreads();
    for (int li = P.l0; li < P.l1; ++li) {
      const int l = A.lists[li];
      const DLeaf lam = A.leaves[l];
      const int cA = imax(lam.c0, P.wc0), cB = imin(lam.c0 + lam.n, P.wc1);
      const int q0 = imax(lam.r0, x.c0), q1 = imin(lam.r0 + lam.m, x.c0 + x.n);
      if (cA >= cB || q0 >= q1) continue;
      const int nq = q1 - q0;
      const LeafRef<T> lr = leaf_ref(A, yi, l, lam);
      const T* lp = lr.U;
      const T* vx = Vx + (q0 - x.c0) + (int64_t)j0 * xr.ldv;
      if (lam.fmt == 0) {
        for (int c0 = cA; c0 < cB; c0 += KC) {
          const int nc = imin(KC, cB - c0);
          tn_product<T, BF>(lp + (q0 - lam.r0) + (int64_t)(c0 - lam.c0) * lr.ldu, lr.ldu, vx, xr.ldv, nq, nc, take,
                            S0c, S1c, S2c, A.prof);
          FLOP(L, FC_PRODUCT, 2.0 * nq * nc * take);
          BYTES(A, L, (double)nq * nc * sizeof(T));
          for (int idx = tid; idx < nc * take; idx += TPB) {
            const int cc = idx / take, jj = idx - cc * take;
            T* d = &Vs[(int64_t)(c0 + cc - tc.c0) * KC + K + jj];
            *d = (T)((CT)*d + S0c[cc * KC + jj]);
          }
          __syncthreads();
        }
      } else {
        const int kl = rank_of(A, yi, l);
        if (kl == 0) continue;
        const T* Ul = lp;
        const T* Vl = lr.V;
        tn_product<T, BF>(Ul + (q0 - lam.r0), lr.ldu, vx, xr.ldv, nq, kl, take, S0c, S1c, S2c, A.prof);
        nn_acc(Vl + (cA - lam.c0), lr.ldv, cB - cA, kl, S0c, take, Vs + (int64_t)(cA - tc.c0) * KC + K, KC, 1, 1.0,
               S1c, A.prof);
        FLOP(L, FC_PRODUCT, 2.0 * kl * take * (nq + (cB - cA)));
        BYTES(A, L, (double)kl * (nq + (cB - cA)) * sizeof(T));
      }
    }
  } else if (P.kind == PK_LRY) {
    const int xi = inst_of(A, b, P.xrole), yi = inst_of(A, b, P.yrole);
    const DLeaf y = A.leaves[P.yleaf];
    const LeafRef<T> yr = leaf_ref(A, yi, P.yleaf, y);
    const T* Uy = yr.U;
    const T* Vy = yr.V;
    BYTES(A, L, (double)take * ((P.wc1 - P.wc0) + y.m) * sizeof(T));  // V_y window columns, U_y
    if (lry_single(A, P, tc, y, yr, xi, j0, take, Us, Vs, K, L)) {
      __syncthreads();
      PROF_ADD(PS_LRY, clock64() - tpc);
      return;
    }
    for (int idx = tid; idx < n * take; idx += TPB) {
      const int c = idx / take, jj = idx - c * take;
      const int gc = tc.c0 + c;
      const double v = (gc >= P.wc0 && gc < P.wc1) ? (CT)Vy[(gc - y.c0) + (int64_t)(j0 + jj) * yr.ldv] : 0.0;
      Vs[(int64_t)c * KC + K + jj] = (T)v;
    }
    for (int idx = tid; idx < m * take; idx += TPB) {
      const int i = idx / take, jj = idx - i * take;
      Us[(int64_t)i * KC + K + jj] = (T)0;
    }
    __syncthreads();
    for (int li = P.l0; li < P.l1; ++li) {
      const int l = A.lists[li];
      const DLeaf lam = A.leaves[l];
      const int rA = imax(lam.r0, P.wr0), rB = imin(lam.r0 + lam.m, P.wr1);
      const int q0 = imax(lam.c0, y.r0), q1 = imin(lam.c0 + lam.n, y.r0 + y.m);
      if (rA >= rB || q0 >= q1) continue;
      const int nq = q1 - q0;
      const LeafRef<T> lr = leaf_ref(A, xi, l, lam);
      const T* lp = lr.U;
      const T* uy = Uy + (q0 - y.r0) + (int64_t)j0 * yr.ldu;
      if (lam.fmt == 0) {
        for (int qc = 0; qc < nq; qc += KC) {
          const int nqc = imin(KC, nq - qc);
          for (int idx = tid; idx < nqc * take; idx += TPB) {
            const int q = idx % nqc, jj = idx / nqc;
            S0c[q * KC + jj] = (CT)uy[qc + q + (int64_t)jj * yr.ldu];
          }
          __syncthreads();
          nn_acc(lp + (rA - lam.r0) + (int64_t)(q0 + qc - lam.c0) * lr.ldu, lr.ldu, rB - rA, nqc, S0c, take,
                 Us + (int64_t)(rA - tc.r0) * KC + K, KC, 1, alpha, S1c, A.prof);
          FLOP(L, FC_PRODUCT, 2.0 * (rB - rA) * nqc * take);
          BYTES(A, L, (double)(rB - rA) * nqc * sizeof(T));
        }
      } else {
        const int kl = rank_of(A, xi, l);
        if (kl == 0) continue;
        const T* Ul = lp;
        const T* Vl = lr.V;
        tn_product<T, BF>(Vl + (q0 - lam.c0), lr.ldv, uy, yr.ldu, nq, kl, take, S0c, S1c, S2c, A.prof);
        nn_acc(Ul + (rA - lam.r0), lr.ldu, rB - rA, kl, S0c, take, Us + (int64_t)(rA - tc.r0) * KC + K, KC, 1, alpha,
               S1c, A.prof);
        FLOP(L, FC_PRODUCT, 2.0 * kl * take * (nq + (rB - rA)));
        BYTES(A, L, (double)kl * (nq + (rB - rA)) * sizeof(T));
      }
    }
  } else if (P.kind == PK_DD) {
    // dense product into a low-rank target: U-part = alpha P[:, cols], V-part = selector
    const int xi = inst_of(A, b, P.xrole), yi = inst_of(A, b, P.yrole);
    const DLeaf x = A.leaves[P.xleaf], y = A.leaves[P.yleaf];
    const LeafRef<T> xr = leaf_ref(A, xi, P.xleaf, x), yr = leaf_ref(A, yi, P.yleaf, y);
    const T* xp = xr.U;
    const T* yp = yr.U;
    const int M0 = imax(x.c0, y.r0), M1 = imin(x.c0 + x.n, y.r0 + y.m);
    for (int idx = tid; idx < m * take; idx += TPB) {
      const int i = idx / take, jj = idx - i * take;
      Us[(int64_t)i * KC + K + jj] = (T)0;
    }
    for (int idx = tid; idx < n * take; idx += TPB) {
      const int c = idx / take, jj = idx - c * take;
      Vs[(int64_t)c * KC + K + jj] = (T)((tc.c0 + c == P.wc0 + j0 + jj) ? 1.0 : 0.0);
    }
    __syncthreads();
    for (int qc = M0; qc < M1; qc += KC) {
      const int nqc = imin(KC, M1 - qc);
      for (int idx = tid; idx < nqc * take; idx += TPB) {
        const int q = idx % nqc, jj = idx / nqc;
        S0c[q * KC + jj] = (CT)yp[(qc + q - y.r0) + (int64_t)(P.wc0 + j0 + jj - y.c0) * yr.ldu];
      }
      __syncthreads();
      nn_acc(xp + (P.wr0 - x.r0) + (int64_t)(qc - x.c0) * xr.ldu, xr.ldu, P.wr1 - P.wr0, nqc, S0c, take,
             Us + (int64_t)(P.wr0 - tc.r0) * KC + K, KC, 1, alpha, S1c, A.prof);
      FLOP(L, FC_PRODUCT, 2.0 * (P.wr1 - P.wr0) * nqc * take);
      BYTES(A, L, (double)((P.wr1 - P.wr0) + take) * nqc * sizeof(T));  // x block, y columns
    }
  } else {  // PK_COPY of a low-rank leaf
    BYTES(A, L, (double)take * (m + n) * sizeof(T));
    const int si = inst_of(A, b, P.xrole);
    const DLeaf s = A.leaves[P.xleaf];
    const LeafRef<T> sr = leaf_ref(A, si, P.xleaf, s);
    const T* Usrc = sr.U;
    const T* Vsrc = sr.V;
    const double* rho = P.rv >= 0 ? A.vec_ptr[b * A.nvroles + P.rv] : nullptr;
    const double* gam = P.cv >= 0 ? A.vec_ptr[b * A.nvroles + P.cv] : nullptr;
    for (int idx = tid; idx < m * take; idx += TPB) {
      const int i = idx / take, jj = idx - i * take;
      double v = alpha * (CT)Usrc[i + (int64_t)(j0 + jj) * sr.ldu];
      if (rho) v *= rho[tc.r0 + i];
      Us[(int64_t)i * KC + K + jj] = (T)v;
    }
    for (int idx = tid; idx < n * take; idx += TPB) {
      const int c = idx / take, jj = idx - c * take;
      double v = (CT)Vsrc[c + (int64_t)(j0 + jj) * sr.ldv];
      if (gam) v *= gam[tc.c0 + c];
      Vs[(int64_t)c * KC + K + jj] = (T)v;
    }
  }
  __syncthreads();
  if (P.kind == PK_LRX) PROF_ADD(PS_LRX, clock64() - tpc);
  if (P.kind == PK_LRY) PROF_ADD(PS_LRY, clock64() - tpc);
}

// Dense target: C += Us Vs^T for `take` columns (C column-major m x n;
// Us, Vs row-major with leading dimension KC): 16 x 16 tiles of C over the
// wavefronts on the matrix cores.
template <bool BF, typename T, typename LT>
__device__ void dense_add_outer(T* C, const DLeaf& tc, const T* Us, const T* Vs, int take, LT& L) {
  using CT = typename CompT<T>::type;
  using MF = Mfma16<CT>;
  using V = typename MF::v4;
  (void)L;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int l16 = lane & 15, g = lane >> 4;
  const int m = tc.m, n = tc.n;
  const int ntn = (n + 15) >> 4, nt = ((m + 15) >> 4) * ntn;
  const int nk = (take + 3) >> 2;
  for (int t = w; t < nt; t += TPB / 64) {
    const int ti = t / ntn, tj = t - ti * ntn;
    const int i = ti * 16 + l16, j = tj * 16 + l16;
    const bool ai = i < m, bj = j < n;
    V acc = {0, 0, 0, 0};
    bool done = false;
    if constexpr (sizeof(CT) == 4 && BF) {
      acc = bf16_outer_tile(Us + (int64_t)i * KC, Vs + (int64_t)j * KC, ai, bj, take, g);
      done = true;
    }
    if (!done) {
#pragma unroll 4
      for (int kk = 0; kk < nk; ++kk) {
        const int k = 4 * kk + g;
        const bool in = k < take;
        const CT av = (ai && in) ? (CT)Us[(int64_t)i * KC + k] : (CT)0;
        const CT bv = (bj && in) ? (CT)Vs[(int64_t)j * KC + k] : (CT)0;
        acc = MF::step(av, bv, acc);
      }
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int ii = ti * 16 + MF::row(g, r), jj = tj * 16 + l16;
      if (ii < m && jj < n) {
        T* d = &C[ii + (int64_t)jj * m];
        *d = (T)((CT)*d + acc[r]);
      }
    }
  }
  __syncthreads();
}

// Dense accumulation C += sum of the target's pieces (C column-major,
// leading dimension tc.m).  The columns of consecutive low-rank pieces are
// staged side by side in Us / Vs and added as one outer product whenever
// the KC staging columns are full (and at the end): one read-modify-write
// of C per KC columns rather than per piece.
template <bool BF, typename T, typename LT>
__device__ void dense_pieces(const AccumArgs<T>& A, int b, const Target& tg, const DLeaf& tc, T* C, T* Us, T* Vs,
                             LT& L) {
  using CT = typename CompT<T>::type;
  CT* S0c = reinterpret_cast<CT*>(L.S0);
  CT* S1c = reinterpret_cast<CT*>(L.S1);
  CT* S2c = reinterpret_cast<CT*>(L.S2);
  const int tid = threadIdx.x;
  unsigned long long* prof = A.prof;
  // Columns of low-rank pieces are staged at [K, K + take) of Us / Vs; the
  // outer product has one call site (inlined twice, the kernel spills).
  int K = 0, j0 = 0;
  for (int p = tg.p0; p < tg.p1 || K > 0;) {
    if (p == tg.p1 || K == KC) {
      const long long to = clock64();
      dense_add_outer<BF>(C, tc, Us, Vs, K, L);
      PROF_ADD(PS_OUTER, clock64() - to);
      FLOP(L, FC_PRODUCT, 2.0 * tc.m * tc.n * K);
      K = 0;
      continue;
    }
    const Piece P = A.pieces[p];
    const long long tpd = clock64();
    if (P.kind == PK_DD) {
      ++p;
      const int xi = inst_of(A, b, P.xrole), yi = inst_of(A, b, P.yrole);
      if (xi < 0 || yi < 0) continue;
      const DLeaf x = A.leaves[P.xleaf], y = A.leaves[P.yleaf];
      const LeafRef<T> xr = leaf_ref(A, xi, P.xleaf, x), yr = leaf_ref(A, yi, P.yleaf, y);
      const T* xp = xr.U;
      const T* yp = yr.U;
      const int M0 = imax(x.c0, y.r0), M1 = imin(x.c0 + x.n, y.r0 + y.m);
      BYTES(A, L, (double)imax(M1 - M0, 0) * ((P.wr1 - P.wr0) + (P.wc1 - P.wc0)) * sizeof(T));  // the two blocks
      for (int cc0 = P.wc0; cc0 < P.wc1; cc0 += KC) {
        const int nc = imin(KC, P.wc1 - cc0);
        for (int qc = M0; qc < M1; qc += KC) {
          const int nqc = imin(KC, M1 - qc);
          for (int idx = tid; idx < nqc * nc; idx += TPB) {
            const int q = idx % nqc, jj = idx / nqc;
            S0c[q * KC + jj] = (CT)yp[(qc + q - y.r0) + (int64_t)(cc0 + jj - y.c0) * yr.ldu];
          }
          __syncthreads();
          nn_acc(xp + (P.wr0 - x.r0) + (int64_t)(qc - x.c0) * xr.ldu, xr.ldu, P.wr1 - P.wr0, nqc, S0c, nc,
                 C + (P.wr0 - tc.r0) + (int64_t)(cc0 - tc.c0) * tc.m, 1, tc.m, P.alpha, S1c, A.prof);
          FLOP(L, FC_PRODUCT, 2.0 * (P.wr1 - P.wr0) * nqc * nc);
        }
      }
      PROF_ADD(PS_DDP, clock64() - tpd);
    } else if (P.kind == PK_COPY && A.leaves[P.xleaf].fmt == 0) {
      ++p;
      const int si = inst_of(A, b, P.xrole);
      if (si < 0) continue;
      BYTES(A, L, (double)tc.m * tc.n * sizeof(T));  // the source leaf
      const LeafRef<T> sr = leaf_ref(A, si, P.xleaf, A.leaves[P.xleaf]);
      const T* src = sr.U;
      const double* rho = P.rv >= 0 ? A.vec_ptr[b * A.nvroles + P.rv] : nullptr;
      const double* gam = P.cv >= 0 ? A.vec_ptr[b * A.nvroles + P.cv] : nullptr;
      for (int idx = tid; idx < tc.m * tc.n; idx += TPB) {
        int i = idx % tc.m, c = idx / tc.m;
        double v = P.alpha * (CT)src[i + (int64_t)c * sr.ldu];
        if (rho) v *= rho[tc.r0 + i];
        if (gam) v *= gam[tc.c0 + c];
        C[idx] = (T)((CT)C[idx] + v);
      }
      __syncthreads();
    } else {
      // a low-rank piece, `take` of its columns per pass
      const int w = piece_width(A, b, P);
      const int take = imin(KC - K, w - j0);
      if (take > 0) piece_columns<BF>(A, b, P, tc, j0, take, Us, Vs, K, L);
      K += imax(take, 0);
      j0 += imax(take, 0);
      if (j0 >= w) {
        j0 = 0;
        ++p;
      }
    }
  }
}

// ------------------------------------------------------------ main kernel
// Narrow rounds leave LDS for three resident blocks per CU: hold the
// register budget to that occupancy.
#if KCV <= 40
#define ACCUM_OCCUPANCY __attribute__((amdgpu_waves_per_eu(3, 3)))
#else
// one block per CU (LDS): the whole register file, AGPRs included, is free
#define ACCUM_OCCUPANCY __attribute__((amdgpu_waves_per_eu(1, 1)))
#endif
template <typename T, bool BF>
__global__ __launch_bounds__(TPB) ACCUM_OCCUPANCY void accum_kernel(AccumArgs<T> A) {
  __shared__ Lds L;
  const int tid = threadIdx.x;
  const int total = A.nbatch * A.nt;
  T* Us = A.scratch + (int64_t)blockIdx.x * A.scratch_stride;
  unsigned long long* prof = A.prof;
  if (tid == 0) {
    for (int c = 0; c < FC_COUNT; ++c) L.flops[c] = 0.0;
    L.bytes = 0.0;
  }
  for (int item = blockIdx.x; item < total; item += gridDim.x) {
    const int b = item / A.nt;
    const int t = A.t0 + item % A.nt;
    const Target tg = A.targets[t];
    const int ci = inst_of(A, b, tg.crole);
    if (ci < 0) continue;
    const DLeaf tc = A.leaves[tg.cleaf];
    if (tc.fmt == 0) continue;  // dense targets: the accumulate-only kernel
    if (A.inst_off[ci]) {  // targets are working instances (capacity layout)
      if (tid == 0) atomicOr(&A.flags[FL_LAYOUT], 1);
      continue;
    }
    T* C = leaf_base(A, ci, tg.cleaf);
    T* Vs = Us + (int64_t)tc.m * KC;
    PROF_ADD(PS_ITEMS, 1);
    PROF_ADD(PS_NPIECES, tg.p1 - tg.p0);
    int32_t* rk = &A.inst_rank[ci][tg.cleaf];
    T* Uc = C;
    T* Vc = C + (int64_t)tc.m * tc.cap;
    if (tg.direct) {  // exact scaled copy of a low-rank leaf
      if (A.mode == 2) continue;
      const Piece P = A.pieces[tg.p0];
      const int si = inst_of(A, b, P.xrole);
      const int ks = si < 0 ? 0 : rank_of(A, si, P.xleaf);
      LeafRef<T> sr{nullptr, nullptr, tc.m, tc.n};
      if (si >= 0) sr = leaf_ref(A, si, P.xleaf, tc);
      const double* rho = P.rv >= 0 ? A.vec_ptr[b * A.nvroles + P.rv] : nullptr;
      const double* gam = P.cv >= 0 ? A.vec_ptr[b * A.nvroles + P.cv] : nullptr;
      for (int idx = tid; idx < tc.m * ks; idx += TPB) {
        int i = idx % tc.m, j = idx / tc.m;
        double v = P.alpha * (double)sr.U[i + (int64_t)j * sr.ldu];
        if (rho) v *= rho[tc.r0 + i];
        Uc[idx] = (T)v;
      }
      for (int idx = tid; idx < tc.n * ks; idx += TPB) {
        int c = idx % tc.n, j = idx / tc.n;
        double v = (double)sr.V[c + (int64_t)j * sr.ldv];
        if (gam) v *= gam[tc.c0 + c];
        Vc[idx] = (T)v;
      }
      if (tid == 0) *rk = ks;
      BYTES(A, L, 2.0 * (tc.m + tc.n) * ks * sizeof(T));
      __syncthreads();
      continue;
    }
    const int k0 = tg.beta ? *rk : 0;
    // Small low-rank targets that receive more columns than their smaller
    // dimension were summed exactly as a dense m x n block by the
    // accumulate-only kernel (the same decision); here they are compressed.
    if (tid == 0) L.ival[5] = 0;
    __syncthreads();
    if (A.doff[t] >= 0)
      for (int p = tg.p0 + tid; p < tg.p1; p += TPB) atomicAdd(&L.ival[5], piece_width(A, b, A.pieces[p]));
    __syncthreads();
    const bool dacc = A.doff[t] >= 0 && L.ival[5] > imin(tc.m, tc.n);
    if ((A.mode == 1 && dacc) || (A.mode == 2 && !dacc)) continue;
    const T* D = dacc ? A.dbuf + (int64_t)b * A.dstride + A.doff[t] : nullptr;
    // ---------------- low-rank target: columns appended in rounds of ROUND
    // beyond the current rank, recompressed in between (the cost of a
    // recompression grows with the cube of its width).  The columns come
    // from the pieces, or from the dense accumulator along its smaller
    // dimension (rows when m <= n: U = identity columns, V = rows of D).
    int K = 0;
    int kbase = 0;  // rank after the last recompression
    if (!dacc && tg.beta) {
      for (int idx = tid; idx < tc.m * k0; idx += TPB) {
        int i = idx % tc.m, j = idx / tc.m;
        Us[(int64_t)i * KC + j] = Uc[idx];
      }
      for (int idx = tid; idx < tc.n * k0; idx += TPB) {
        int c = idx % tc.n, j = idx / tc.n;
        Vs[(int64_t)c * KC + j] = Vc[idx];
      }
      K = k0;
      kbase = k0;
      __syncthreads();
    }
    const bool by_rows = tc.m <= tc.n;
    const int pend = dacc ? tg.p0 + 1 : tg.p1;
    for (int p = tg.p0; p < pend; ++p) {
      Piece P{};
      int w;
      if (dacc) {
        w = by_rows ? tc.m : tc.n;
      } else {
        P = A.pieces[p];
        w = piece_width(A, b, P);
      }
      int j0 = 0;
      while (j0 < w) {
        const int klim = imin(KC, kbase + ROUND);
        if (K >= klim) {
          K = truncate_block<T, BF>(Us, Vs, tc.m, tc.n, K, A.eps, L, A.flags, A.prof);
          if (K > KC - 8) {
            if (tid == 0) atomicOr(&A.flags[FL_RANK_OVERFLOW], 1);
            K = KC - 8;
          }
          kbase = K;
        }
        const int take = imin(w - j0, imin(KC, kbase + ROUND) - K);
        const long long tp0 = clock64();
        if (dacc) {
          for (int idx = tid; idx < tc.m * take; idx += TPB) {
            const int i = idx / take, jj = idx - i * take;
            Us[(int64_t)i * KC + K + jj] = by_rows ? (T)(i == j0 + jj ? 1.0 : 0.0) : D[i + (int64_t)(j0 + jj) * tc.m];
          }
          for (int idx = tid; idx < tc.n * take; idx += TPB) {
            const int c = idx / take, jj = idx - c * take;
            Vs[(int64_t)c * KC + K + jj] = by_rows ? D[(j0 + jj) + (int64_t)c * tc.m] : (T)(c == j0 + jj ? 1.0 : 0.0);
          }
          __syncthreads();
        } else {
          piece_columns<BF>(A, b, P, tc, j0, take, Us, Vs, K, L);
        }
        PROF_ADD(PS_PIECES_LR, clock64() - tp0);
        K += take;
        j0 += take;
      }
    }
    if (dacc || tg.p1 > tg.p0 || !tg.beta) {
      int k = truncate_block<T, BF>(Us, Vs, tc.m, tc.n, K, A.eps, L, A.flags, A.prof);
      int kw = imin(k, tc.cap);
      // the dense sum or the old factors read, the truncated factors written
      BYTES(A, L, ((double)(tc.m + tc.n) * kw +
                   (dacc ? (double)tc.m * tc.n : (tg.beta ? (double)(tc.m + tc.n) * k0 : 0.0))) * sizeof(T));
      if (tid == 0) {
        if (k > tc.cap) atomicOr(&A.flags[FL_RANK_OVERFLOW], 1);
        atomicMax(&A.flags[FL_MAXRANK], k);
        *rk = kw;
      }
      for (int idx = tid; idx < tc.m * kw; idx += TPB) {
        int i = idx % tc.m, j = idx / tc.m;
        Uc[idx] = Us[(int64_t)i * KC + j];
      }
      for (int idx = tid; idx < tc.n * kw; idx += TPB) {
        int c = idx % tc.n, j = idx / tc.n;
        Vc[idx] = Vs[(int64_t)c * KC + j];
      }
    }
    __syncthreads();
  }
  if (tid == 0 && A.flops) {
    for (int c = 0; c < FC_COUNT; ++c) atomicAdd(A.flops + c, L.flops[c]);
    atomicAdd(A.flops + FC_COUNT, L.bytes);
  }
}

// The accumulate-only kernel needs only the staging tiles (FP32 tiles for
// FP32 factors): with narrow rounds, four resident wavefronts per SIMD
// (128 VGPRs, no spilling with FP32 factors; measured best among 4, 5, 6
// once the staged piece columns are batched: 6 spills 300 B per lane).
#if KCV <= 40
#ifndef DENSE_WPE
#define DENSE_WPE 4
#endif
#define DENSE_OCCUPANCY __attribute__((amdgpu_waves_per_eu(DENSE_WPE, DENSE_WPE)))
#else
#define DENSE_OCCUPANCY
#endif
// Accumulate-only first phase of a step: every dense target, and the dense
// sum of every small low-rank target that is summed densely (same decision
// as the truncating kernel, which then compresses it).  No truncation
// workspace: a small LDS footprint, more resident blocks.
template <typename T, bool BF>
__global__ __launch_bounds__(TPB) DENSE_OCCUPANCY void accum_dense_kernel(AccumArgs<T> A) {
  __shared__ LdsPiece<typename CompT<T>::type> L;
  __shared__ int wsum;
  const int tid = threadIdx.x;
  const int total = A.nbatch * A.nt;
  T* Us = A.scratch + (int64_t)blockIdx.x * A.scratch_stride;
  if (tid == 0) {
    for (int c = 0; c < FC_COUNT; ++c) L.flops[c] = 0.0;
    L.bytes = 0.0;
  }
  for (int item = blockIdx.x; item < total; item += gridDim.x) {
    const int b = item / A.nt;
    const int t = A.t0 + item % A.nt;
    const Target tg = A.targets[t];
    const int ci = inst_of(A, b, tg.crole);
    if (ci < 0) continue;
    const DLeaf tc = A.leaves[tg.cleaf];
    if (tc.fmt != 0 && (tg.direct || A.doff[t] < 0)) continue;
    if (A.inst_off[ci]) {
      if (tid == 0) atomicOr(&A.flags[FL_LAYOUT], 1);
      continue;
    }
    T* C = leaf_base(A, ci, tg.cleaf);
    T* Vs = Us + (int64_t)tc.m * KC;
    unsigned long long* prof = A.prof;
    const long long t_item = clock64();
    T* dst = C;  // the dense leaf itself, or the dense sum of a low-rank leaf
    if (tc.fmt == 0) {
      if (!tg.beta)
        for (int idx = tid; idx < tc.m * tc.n; idx += TPB) C[idx] = (T)0;
      BYTES(A, L, (tg.beta ? 2.0 : 1.0) * tc.m * tc.n * sizeof(T));  // the leaf read (accumulated into), written
    } else {
      if (tid == 0) wsum = 0;
      __syncthreads();
      for (int p = tg.p0 + tid; p < tg.p1; p += TPB) atomicAdd(&wsum, piece_width(A, b, A.pieces[p]));
      __syncthreads();
      if (!(wsum > imin(tc.m, tc.n))) continue;
      dst = A.dbuf + (int64_t)b * A.dstride + A.doff[t];
      const int k0 = tg.beta ? A.inst_rank[ci][tg.cleaf] : 0;
      const T* Uc = C;
      const T* Vc = C + (int64_t)tc.m * tc.cap;
      for (int idx = tid; idx < tc.m * tc.n; idx += TPB) {
        const int i = idx % tc.m, c = idx / tc.m;
        double v = 0.0;
        for (int j = 0; j < k0; ++j) v += (double)Uc[i + (int64_t)j * tc.m] * (double)Vc[c + (int64_t)j * tc.n];
        dst[idx] = (T)v;
      }
      FLOP(L, FC_PRODUCT, 2.0 * tc.m * tc.n * k0);
      BYTES(A, L, ((double)(tc.m + tc.n) * k0 + (double)tc.m * tc.n) * sizeof(T));  // old factors read, sum written
    }
    __syncthreads();
    // one call site, so that the product code is inlined once
    dense_pieces<BF>(A, b, tg, tc, dst, Us, Vs, L);
    PROF_ADD(tc.fmt == 0 ? PS_DENSE : PS_DACC, clock64() - t_item);
  }
  if (tid == 0 && A.flops) {
    for (int c = 0; c < FC_COUNT; ++c) atomicAdd(A.flops + c, L.flops[c]);
    atomicAdd(A.flops + FC_COUNT, L.bytes);
  }
}

// ------------------------------------------------------------ launchers
// BF16 piece products are a separate build of the FP32 kernels, so that the
// FP32 build keeps its registers (the BF16 branches would make it spill).
template <typename T>
void launch_accum(const AccumArgs<T>& a, int grid, hipStream_t s) {
  if constexpr (std::is_same<T, float>::value) {
    if (a.bf16_products) {
      hipLaunchKernelGGL((accum_kernel<T, true>), dim3(grid), dim3(TPB), 0, s, a);
      return;
    }
  }
  hipLaunchKernelGGL((accum_kernel<T, false>), dim3(grid), dim3(TPB), 0, s, a);
}
template <typename T>
void launch_accum_dense(const AccumArgs<T>& a, int grid, hipStream_t s) {
  if constexpr (std::is_same<T, float>::value) {
    if (a.bf16_products) {
      hipLaunchKernelGGL((accum_dense_kernel<T, true>), dim3(grid), dim3(TPB), 0, s, a);
      return;
    }
  }
  hipLaunchKernelGGL((accum_dense_kernel<T, false>), dim3(grid), dim3(TPB), 0, s, a);
}
template void launch_accum_dense<double>(const AccumArgs<double>&, int, hipStream_t);
template void launch_accum_dense<float>(const AccumArgs<float>&, int, hipStream_t);
template void launch_accum<double>(const AccumArgs<double>&, int, hipStream_t);
template void launch_accum<float>(const AccumArgs<float>&, int, hipStream_t);

}  // namespace KCNS

#if KCV == 64
// ------------------------------------------------------------ leaf inverse
// In-place inverse of dense diagonal leaves by Gauss-Jordan elimination with
// partial pivoting in FP64 (one block per instance).
template <typename T>
__global__ __launch_bounds__(TPB) void leaf_inverse_kernel(T* const* inst_base, const int32_t* insts, int stride,
                                                          int ninst, int64_t off, int m, int32_t* flags) {
  __shared__ double W[64 * 129];
  __shared__ double red[TPB];
  __shared__ int redi[TPB];
  __shared__ int piv_s;
  const int tid = threadIdx.x;
  const int ld = 2 * m + 1;
  for (int it = blockIdx.x; it < ninst; it += gridDim.x) {
    T* a = inst_base[insts[it * stride]] + off;
    for (int idx = tid; idx < m * 2 * m; idx += TPB) {
      int i = idx / (2 * m), j = idx - i * 2 * m;
      W[i * ld + j] = (j < m) ? (double)a[i + (int64_t)j * m] : (j - m == i ? 1.0 : 0.0);
    }
    __syncthreads();
    for (int k = 0; k < m; ++k) {
      double best = -1.0;
      int bi = k;
      for (int i = k + tid; i < m; i += TPB) {
        double v = fabs(W[i * ld + k]);
        if (v > best) { best = v; bi = i; }
      }
      red[tid] = best;
      redi[tid] = bi;
      __syncthreads();
      for (int s = TPB / 2; s > 0; s >>= 1) {
        if (tid < s) {
          if (red[tid + s] > red[tid] || (red[tid + s] == red[tid] && redi[tid + s] < redi[tid])) {
            red[tid] = red[tid + s];
            redi[tid] = redi[tid + s];
          }
        }
        __syncthreads();
      }
      if (tid == 0) {
        piv_s = redi[0];
        if (!(red[0] > 0.0)) atomicOr(&flags[FL_SINGULAR], 1);
      }
      __syncthreads();
      const int p = piv_s;
      if (p != k)
        for (int j = tid; j < 2 * m; j += TPB) {
          double t = W[k * ld + j];
          W[k * ld + j] = W[p * ld + j];
          W[p * ld + j] = t;
        }
      __syncthreads();
      const double pv = W[k * ld + k];
      const double inv = pv != 0.0 ? 1.0 / pv : 0.0;
      __syncthreads();
      for (int j = tid; j < 2 * m; j += TPB) W[k * ld + j] *= inv;
      __syncthreads();
      for (int idx = tid; idx < m * 2 * m; idx += TPB) {
        int i = idx / (2 * m), j = idx - i * 2 * m;
        if (i == k || j == k) continue;
        W[i * ld + j] -= W[i * ld + k] * W[k * ld + j];
      }
      __syncthreads();
      for (int i = tid; i < m; i += TPB)
        if (i != k) W[i * ld + k] = 0.0;
      __syncthreads();
    }
    for (int idx = tid; idx < m * m; idx += TPB) {
      int i = idx % m, j = idx / m;
      a[idx] = (T)W[i * ld + m + j];
    }
    __syncthreads();
  }
}

// ------------------------------------------------------------ level 0
// D_k^(0): write the in-plane 5-point couplings of every plane into the
// dense leaves of its H-matrix instance (the low-rank leaves start empty).
// map[d * B + i] = element offset inside the instance of the entry
// (row i, column of neighbour d) or -1; d = centre, x-1, x+1, y-1, y+1.
template <typename T>
__global__ void level0_kernel(T* const* inst_base, const int32_t* insts, int nplanes, int plane0, const double* S,
                              int64_t N, int B, const int32_t* perm, const int64_t* map, L0Rows rows) {
  const int64_t total = (int64_t)nplanes * B;
  for (int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g < total; g += (int64_t)gridDim.x * blockDim.x) {
    int k = (int)(g / B), i = (int)(g - (int64_t)k * B);
    int64_t p = (int64_t)(plane0 + k) * B + perm[i];
    T* base = inst_base[insts[k]];
    for (int d = 0; d < rows.nd; ++d) {
      int64_t o = map[(int64_t)d * B + i];
      if (o >= 0) base[o] = (T)S[(int64_t)rows.row[d] * N + p];
    }
  }
}

// H-ordered z-couplings of every plane: out[k*B + i] = S[row][k*B + perm[i]].
__global__ void zcoupling_kernel(const double* S, int64_t N, int B, int nz, const int32_t* perm, double* outA,
                                 double* outC) {
  const int64_t total = (int64_t)nz * B;
  for (int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g < total; g += (int64_t)gridDim.x * blockDim.x) {
    int k = (int)(g / B), i = (int)(g - (int64_t)k * B);
    int64_t p = (int64_t)k * B + perm[i];
    outA[g] = S[5 * N + p];
    outC[g] = S[6 * N + p];
  }
}

template <typename T>
void launch_leaf_inverse(T* const* base, const int32_t* insts, int stride, int ninst, int64_t off, int m,
                         int32_t* flags, hipStream_t s) {
  int grid = ninst < 1024 ? ninst : 1024;
  hipLaunchKernelGGL(leaf_inverse_kernel<T>, dim3(grid), dim3(TPB), 0, s, base, insts, stride, ninst, off, m, flags);
}
template <typename T>
void launch_level0(T* const* base, const int32_t* insts, int nplanes, int plane0, const double* S, int64_t N, int B,
                   const int32_t* perm, const int64_t* map, const L0Rows& rows, hipStream_t s) {
  int64_t total = (int64_t)nplanes * B;
  int grid = (int)((total + 255) / 256);
  if (grid > 65535) grid = 65535;
  hipLaunchKernelGGL(level0_kernel<T>, dim3(grid), dim3(256), 0, s, base, insts, nplanes, plane0, S, N, B, perm, map,
                     rows);
}
void launch_zcoupling(const double* S, int64_t N, int B, int nz, const int32_t* perm, double* outA, double* outC,
                      hipStream_t s) {
  int64_t total = (int64_t)nz * B;
  int grid = (int)((total + 255) / 256);
  if (grid > 65535) grid = 65535;
  hipLaunchKernelGGL(zcoupling_kernel, dim3(grid), dim3(256), 0, s, S, N, B, nz, perm, outA, outC);
}
template void launch_leaf_inverse<double>(double* const*, const int32_t*, int, int, int64_t, int, int32_t*,
                                          hipStream_t);
template void launch_leaf_inverse<float>(float* const*, const int32_t*, int, int, int64_t, int, int32_t*, hipStream_t);
template void launch_level0<double>(double* const*, const int32_t*, int, int, const double*, int64_t, int,
                                    const int32_t*, const int64_t*, const L0Rows&, hipStream_t);
template void launch_level0<float>(float* const*, const int32_t*, int, int, const double*, int64_t, int,
                                   const int32_t*, const int64_t*, const L0Rows&, hipStream_t);
#endif

}  // namespace acr
