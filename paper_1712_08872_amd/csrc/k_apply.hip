// Batched H-matrix-vector products for the preconditioner sweeps.
//
// The apply phase of ACR consists of H-matrix-vector products only
// (Sec. 5.3.1): each step of the forward/backward
// substitution multiplies every plane of a cyclic-reduction level by a
// stored H-matrix (Dinv_i or a coupling).  A *job* computes
//     y = base + sum_t alpha_t op_t(H_t) x_t
// for one plane, with up to two terms (op = identity or transpose; a term
// may also be a diagonal vector, the level-0 z-couplings).  Every stored
// H-matrix is packed (exact ranks, leading dimensions padded to a multiple
// of 4 elements, leaves 4-element aligned), so columns stream with 16-byte
// loads.  Three wavefront-level kernels, no block barriers:
//   mv_coef_kernel : s = V^T x (or U^T x) per (job term, low-rank leaf);
//                    a power-of-two group of lanes per column;
//   mv_rows_kernel : y = sum D x + sum U s per (job, row segment);
//   mv_cols_kernel : y = sum D^T x + sum V s per (job, column segment).
// Sums are formed in a fixed order (deterministic results).  Arithmetic is
// FP64; the factor loads are FP32 in mixed precision.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

#include "hprog.h"

namespace acr {

__device__ __forceinline__ int pad4(int x) { return (x + 3) & ~3; }
__device__ __forceinline__ int imin_(int a, int b) { return a < b ? a : b; }

// Four consecutive elements (16-byte aligned for float, 32 for double).
__device__ __forceinline__ void load4(const float* p, double* o) {
  const float4 v = *reinterpret_cast<const float4*>(p);
  o[0] = v.x;
  o[1] = v.y;
  o[2] = v.z;
  o[3] = v.w;
}
__device__ __forceinline__ void load4(const double* p, double* o) {
  const double2 a = *reinterpret_cast<const double2*>(p);
  const double2 b = *reinterpret_cast<const double2*>(p + 2);
  o[0] = a.x;
  o[1] = a.y;
  o[2] = b.x;
  o[3] = b.y;
}

// Four consecutive elements in the factor's own precision (16-byte loads).
template <typename T>
__device__ __forceinline__ void load4raw(const T* p, T* o);
template <>
__device__ __forceinline__ void load4raw<float>(const float* p, float* o) {
  const float4 v = *reinterpret_cast<const float4*>(p);
  o[0] = v.x;
  o[1] = v.y;
  o[2] = v.z;
  o[3] = v.w;
}
template <>
__device__ __forceinline__ void load4raw<double>(const double* p, double* o) {
  const double2 a = *reinterpret_cast<const double2*>(p);
  const double2 b = *reinterpret_cast<const double2*>(p + 2);
  o[0] = a.x;
  o[1] = a.y;
  o[2] = b.x;
  o[3] = b.y;
}

// lanes per column: the power of two covering ceil(len / 4) quads, <= 64
__device__ __forceinline__ int lanes_per_col(int len) {
  int g = 1;
  while (g * 4 < len && g < 64) g <<= 1;
  return g;
}

// Uniform copies of lane i's value (the descriptors of a chunk of leaves
// are fetched lane-parallel, then walked one leaf at a time).
__device__ __forceinline__ int bcast(int v, int i) { return __builtin_amdgcn_readlane(v, i); }
__device__ __forceinline__ int64_t bcast64(int64_t v, int i) {
  const int lo = __builtin_amdgcn_readlane((int)(uint32_t)(uint64_t)v, i);
  const int hi = __builtin_amdgcn_readlane((int)(uint32_t)((uint64_t)v >> 32), i);
  return (int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint64_t)(uint32_t)lo);
}

// Elements of a factor column per lane in the coefficient kernel: 4 for
// FP64 factors, 8 for FP32 ones.
template <typename T>
struct Epl {
  static constexpr int value = sizeof(T) == 8 ? 4 : 8;
};

// Columns of a leaf whose loads a lane issues together in the coefficient
// kernel (NB x E factor values held at once).
#ifndef ACR_COEF_NB32
#define ACR_COEF_NB32 2
#endif
#ifndef ACR_COEF_NB64
#define ACR_COEF_NB64 2
#endif
template <typename T>
struct CoefCols {
  static constexpr int value = sizeof(T) == 8 ? ACR_COEF_NB64 : ACR_COEF_NB32;
};

// s = V^T x (or U^T x) for every low-rank leaf of a job term.  The leaves
// are ordered by the class of the length len they reduce over; a leaf of
// class c gets a group of G = 4 << c lanes (E = 4 consecutive elements of
// each column per lane for FP64 factors, 8 for FP32), so a wavefront works
// on 64 / G leaves at once (1 or 4 rounds); a lane issues the loads of NB
// columns together (x read once for them), and each column is reduced
// within its lane group.
template <typename T>
__global__ __launch_bounds__(256) void mv_coef_kernel(MvArgs<T> A) {
  constexpr int E = Epl<T>::value;
  constexpr int NB = CoefCols<T>::value;
  const int lane = threadIdx.x & 63;
  const int W = A.cw[5];
  const int64_t nitems = (int64_t)A.nterms * W;
  for (int64_t item = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); item < nitems; item += (int64_t)gridDim.x * 4) {
    const int ti = (int)(item / W);
    const int wv = (int)(item - (int64_t)ti * W);
    int c = 0;
    while (c < 4 && wv >= A.cw[c + 1]) ++c;
    const int G = 4 << c, groups = 64 / G;
    const int gi = lane / G, q = lane & (G - 1);
    const int jt = A.terms[ti];
    const MvTerm& tm = A.jobs[jt >> 1].t[jt & 1];
    const T* base = A.inst_base[tm.inst];
    double* coef = A.coef + (int64_t)jt * A.sstride;
    if (c == 4) {  // longest leaves: this wavefront takes 4 columns of one leaf
      const int rel = wv - A.cw[4];
      const int l = A.lr_sorted[A.cls[4] + rel / A.w4];
      const int a0 = 4 * (rel % A.w4);
      const DLeaf L = A.leaves[l];
      const int k = A.inst_rank[tm.inst][l];
      if (a0 >= k) continue;
      const int ldu = pad4(L.m), ldv = pad4(L.n);
      const T* F = base + A.inst_off[tm.inst][l] + (A.trans ? 0 : (int64_t)ldu * k);
      const int len = A.trans ? L.m : L.n, ld = A.trans ? ldu : ldv;
      const double* x = tm.x + (A.trans ? L.r0 : L.c0);
      double* out = coef + A.soff[l];
      const int a1 = imin_(k, a0 + 4);
      // NB columns side by side: their loads are in flight together and
      // share the lane's slice of x
      for (int ab = a0; ab < a1; ab += NB) {
        const int nb = imin_(a1 - ab, NB);
        const T* f = F + (int64_t)ab * ld;
        double s[NB];
#pragma unroll
        for (int u = 0; u < NB; ++u) s[u] = 0.0;
        for (int r0 = E * lane; r0 < len; r0 += 64 * E) {
          double xv[E];
#pragma unroll
          for (int e = 0; e < E; ++e) xv[e] = (r0 + e < len) ? x[r0 + e] : 0.0;
          const bool second = E == 8 && r0 + 4 < len;
          T v[NB][E];
#pragma unroll
          for (int u = 0; u < NB; ++u) {
            if (u < nb) {
              load4raw(f + (int64_t)u * ld + r0, v[u]);
              if (E == 8) {
                if (second) {
                  load4raw(f + (int64_t)u * ld + r0 + 4, v[u] + 4);
                } else {
#pragma unroll
                  for (int e = 4; e < E; ++e) v[u][e] = T{};
                }
              }
            }
          }
#pragma unroll
          for (int u = 0; u < NB; ++u) {
            if (u < nb) {
              double t = 0.0;
#pragma unroll
              for (int e = 0; e < E; ++e)
                if (r0 + e < len) t += (double)v[u][e] * xv[e];
              s[u] += t;
            }
          }
        }
#pragma unroll
        for (int u = 0; u < NB; ++u)
          for (int o = 32; o > 0; o >>= 1) s[u] += __shfl_xor(s[u], o);
        if (lane == 0)
#pragma unroll
          for (int u = 0; u < NB; ++u)
            if (u < nb) out[ab + u] = s[u];
      }
      continue;
    }
    const int lb = A.cls[c] + (wv - A.cw[c]) * A.rounds * groups, cend = A.cls[c + 1];
    for (int r = 0; r < A.rounds; ++r) {
      const int li = lb + r * groups + gi;
      if (li >= cend) continue;  // a whole lane group at a time
      const int l = A.lr_sorted[li];
      const DLeaf L = A.leaves[l];
      const int k = A.inst_rank[tm.inst][l];
      const int ldu = pad4(L.m), ldv = pad4(L.n);
      const T* F = base + A.inst_off[tm.inst][l] + (A.trans ? 0 : (int64_t)ldu * k);
      const int len = A.trans ? L.m : L.n, ld = A.trans ? ldu : ldv;
      const double* x = tm.x + (A.trans ? L.r0 : L.c0);
      double* out = coef + A.soff[l];
      // the host bins a leaf into class c only if len <= E * G: one lane
      // segment per column, x read once, NB columns' loads together
      const int r0 = E * q;
      double xv[E];
#pragma unroll
      for (int e = 0; e < E; ++e) xv[e] = (r0 + e < len) ? x[r0 + e] : 0.0;
      const bool act = r0 < len, act2 = E == 8 && r0 + 4 < len;
      for (int a0 = 0; a0 < k; a0 += NB) {
        T v[NB][E];
#pragma unroll
        for (int u = 0; u < NB; ++u) {
          if (act && a0 + u < k) {
            load4raw(F + (int64_t)(a0 + u) * ld + r0, v[u]);
            if (E == 8) {
              if (act2) {
                load4raw(F + (int64_t)(a0 + u) * ld + r0 + 4, v[u] + 4);
              } else {
#pragma unroll
                for (int e = 4; e < E; ++e) v[u][e] = T{};
              }
            }
          } else {
#pragma unroll
            for (int e = 0; e < E; ++e) v[u][e] = T{};
          }
        }
        double s[NB];
#pragma unroll
        for (int u = 0; u < NB; ++u) {
          s[u] = 0.0;
#pragma unroll
          for (int e = 0; e < E; ++e) s[u] += (double)v[u][e] * xv[e];
        }
#pragma unroll
        for (int u = 0; u < NB; ++u)
          for (int o = G >> 1; o > 0; o >>= 1) s[u] += __shfl_xor(s[u], o);
        if (q == 0)
#pragma unroll
          for (int u = 0; u < NB; ++u)
            if (a0 + u < k) out[a0 + u] = s[u];
      }
    }
  }
}

// Lane-parallel descriptors of up to 64 leaves of a segment list.
struct SegDesc {
  int m, n, r0, c0, fmt, k;
  int64_t off, so;
};

template <typename T>
__device__ __forceinline__ SegDesc seg_desc(const MvArgs<T>& A, const int32_t* idx, int e, int inst) {
  SegDesc d;
  const int l = idx[e];
  const DLeaf L = A.leaves[l];
  d.m = L.m;
  d.n = L.n;
  d.r0 = L.r0;
  d.c0 = L.c0;
  d.fmt = L.fmt;
  d.k = L.fmt ? A.inst_rank[inst][l] : 0;
  d.off = A.inst_off[inst][l];
  d.so = L.fmt ? A.soff[l] : 0;
  return d;
}

// Columns per unit of the row kernel: two for FP32 factors (32 bytes per
// lane per unit, as one column of FP64 factors).
template <typename T>
struct RowCols {
  static constexpr int value = sizeof(T) == 8 ? 1 : 2;
};

// One (leaf, pass) unit of the row kernel for this lane: rows 4q..4q+3 of
// the segment in columns c + s cpp (s < NC) of a dense leaf or of a U
// factor (raw factor values), and the weights of those columns (x for a
// dense leaf, the coefficients s = V^T x for U).
template <typename T>
struct RowUnit {
  static constexpr int NC = RowCols<T>::value;
  T v[NC][4];
  double w[NC];
};

template <typename T>
__device__ __forceinline__ void row_unit_load(const T* P, int ldm, int ro, int c, int cpp, int ncols,
                                              const double* wp, int q, int R, bool act, RowUnit<T>& u) {
#pragma unroll
  for (int s = 0; s < RowUnit<T>::NC; ++s) {
    const int cs = c + s * cpp;
    if (act && cs < ncols) {
      const T* col = P + (int64_t)cs * ldm + ro + 4 * q;
      if ((ro & 3) == 0) {
        load4raw(col, u.v[s]);
      } else {
#pragma unroll
        for (int r = 0; r < 4; ++r) u.v[s][r] = (4 * q + r < R) ? col[r] : T{};
      }
      u.w[s] = wp[cs];
    } else {
      u.v[s][0] = u.v[s][1] = u.v[s][2] = u.v[s][3] = T{};
      u.w[s] = 0.0;
    }
  }
}

// Units in flight per wavefront in the row kernel (a ring: the loads of the
// next RING-1 units are issued before a unit is accumulated).
#ifndef ACR_RING32
#define ACR_RING32 2
#endif
#ifndef ACR_RING64
#define ACR_RING64 3
#endif
template <typename T>
struct RowRing {
  static constexpr int value = sizeof(T) == 8 ? ACR_RING64 : ACR_RING32;
};

// y[lo:hi] (+)= sum_t alpha_t (H_t x_t)[lo:hi], one block per (job, row
// segment); wavefront w takes every 4th leaf of the segment's list and the
// four partial sums are added in wave order (deterministic).  A dense leaf
// contributes its columns weighted by x, a low-rank leaf the columns of U
// weighted by its coefficients s = V^T x; lanes map to (row quad, column)
// with 16-byte loads when the segment starts 4-aligned inside the leaf.
// The (leaf, column pass) units are walked through a ring, so the loads of
// several units are in flight while one is accumulated.
template <typename T>
__global__ __launch_bounds__(256) void mv_rows_kernel(MvArgs<T> A) {
  constexpr int D = RowRing<T>::value;
  // the walker preloads D - 1 units before the loop; with D = 1 nothing
  // would be issued and every contribution dropped
  static_assert(D >= 2, "the row kernel's ring needs at least two slots");
  __shared__ double red[4][256];
  __shared__ double part[4][64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  double* rw = red[w];
  const int64_t nitems = (int64_t)A.njobs * A.nseg;
  for (int64_t item = blockIdx.x; item < nitems; item += gridDim.x) {
    const int j = (int)(item / A.nseg);
    const int sg = (int)(item - (int64_t)j * A.nseg);
    const MvJob& J = A.jobs[j];
    const int lo = A.seg_lo[sg], R = A.seg_lo[sg + 1] - lo;  // R <= 64
    const int ldR = pad4(R), g = ldR / 4, cpp = 64 / g;       // quad layout: g lanes per column
    const int q = lane % g, co = lane / g;
    const bool qact = co < cpp;
    const int e0 = A.rows_ptr[sg], ne = A.rows_ptr[sg + 1] - e0;
    double accq[4] = {0.0, 0.0, 0.0, 0.0};  // rows 4q..4q+3, column group co
    double accr = 0.0;                      // row `lane` (diagonal terms)
    for (int tt = 0; tt < 2; ++tt) {
      const MvTerm& tm = J.t[tt];
      if (tm.inst < 0) {
        if (tm.dvec && w == 0 && lane < R) accr += tm.alpha * tm.dvec[lo + lane] * tm.x[lo + lane];
        continue;
      }
      const T* base = A.inst_base[tm.inst];
      const double* coef = A.coef + (int64_t)(2 * j + tt) * A.sstride;
      const double al = tm.alpha;
      for (int eb = w; eb < ne; eb += 256) {
        const int cnt = imin_(64, (ne - eb + 3) / 4);  // this wave's leaves eb, eb+4, ...
        if (cnt <= 0) continue;
        SegDesc d{};
        if (lane < cnt) d = seg_desc(A, A.rows_idx, e0 + eb + 4 * lane, tm.inst);
        // the walker: the next unit to load is column pass c0 of leaf i
        int i = 0, c0 = 0;
        bool more = true;
        const T* P = nullptr;
        const double* wp = nullptr;
        int ldm = 0, ro = 0, ncols = 0;
        auto leaf = [&](int ii) {
          const int fmt = bcast(d.fmt, ii);
          P = base + bcast64(d.off, ii);
          ldm = pad4(bcast(d.m, ii));
          ro = lo - bcast(d.r0, ii);
          ncols = fmt ? bcast(d.k, ii) : bcast(d.n, ii);
          wp = fmt ? coef + bcast64(d.so, ii) : tm.x + bcast(d.c0, ii);
        };
        int issued = 0;  // real units loaded so far (uniform)
        auto issue = [&](RowUnit<T>& u) {
          if (!more) {
#pragma unroll
            for (int sc = 0; sc < RowUnit<T>::NC; ++sc) {
              u.v[sc][0] = u.v[sc][1] = u.v[sc][2] = u.v[sc][3] = T{};
              u.w[sc] = 0.0;
            }
            return;
          }
          row_unit_load(P, ldm, ro, c0 + co, cpp, ncols, wp, q, R, qact, u);
          ++issued;
          c0 += RowUnit<T>::NC * cpp;
          if (c0 >= ncols) {
            c0 = 0;
            if (++i < cnt)
              leaf(i);
            else
              more = false;
          }
        };
        leaf(0);
        RowUnit<T> u[D];
#pragma unroll
        for (int s = 0; s < D - 1; ++s) issue(u[s]);
        for (int done = 0; done < issued; ++done) {
          issue(u[D - 1]);
#pragma unroll
          for (int sc = 0; sc < RowUnit<T>::NC; ++sc) {
            const double wc = al * u[0].w[sc];
#pragma unroll
            for (int r = 0; r < 4; ++r) accq[r] += (double)u[0].v[sc][r] * wc;
          }
#pragma unroll
          for (int s = 0; s < D - 1; ++s) u[s] = u[s + 1];
        }
      }
    }
    // this wave's rows: its column groups in a fixed order
    if (qact)
#pragma unroll
      for (int r = 0; r < 4; ++r) rw[co * ldR + 4 * q + r] = accq[r];
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    if (lane < R) {
      double sum = accr;
      for (int c = 0; c < cpp; ++c) sum += rw[c * ldR + lane];
      part[w][lane] = sum;
    }
    __syncthreads();
    if (w == 0 && lane < R) {
      double sum = part[0][lane] + part[1][lane] + part[2][lane] + part[3][lane];
      if (J.base) sum += J.base[lo + lane];
      J.y[lo + lane] = sum;
    }
    __syncthreads();
  }
}

// y[lo:hi] (+)= sum_t alpha_t (H_t^T x_t)[lo:hi], one block per (job,
// column segment), leaves split over the four wavefronts as above.  Dense
// leaves: one aligned column dot product per lane group (16-byte loads);
// low-rank leaves: lane = row of V (= output column).
template <typename T>
__global__ __launch_bounds__(256) void mv_cols_kernel(MvArgs<T> A) {
  __shared__ double yacc[4][64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  double* yw = yacc[w];
  const int64_t nitems = (int64_t)A.njobs * A.nseg;
  for (int64_t item = blockIdx.x; item < nitems; item += gridDim.x) {
    const int j = (int)(item / A.nseg);
    const int sg = (int)(item - (int64_t)j * A.nseg);
    const MvJob& J = A.jobs[j];
    const int lo = A.seg_lo[sg], R = A.seg_lo[sg + 1] - lo;
    const int e0 = A.cols_ptr[sg], ne = A.cols_ptr[sg + 1] - e0;
    yw[lane] = 0.0;
    double accr = 0.0;
    for (int tt = 0; tt < 2; ++tt) {
      const MvTerm& tm = J.t[tt];
      if (tm.inst < 0) {
        if (tm.dvec && w == 0 && lane < R) accr += tm.alpha * tm.dvec[lo + lane] * tm.x[lo + lane];
        continue;
      }
      const T* base = A.inst_base[tm.inst];
      const double* coef = A.coef + (int64_t)(2 * j + tt) * A.sstride;
      const double al = tm.alpha;
      for (int eb = w; eb < ne; eb += 256) {
        const int cnt = imin_(64, (ne - eb + 3) / 4);
        SegDesc d{};
        if (lane < cnt) d = seg_desc(A, A.cols_idx, e0 + eb + 4 * lane, tm.inst);
        for (int i = 0; i < cnt; ++i) {
          const int m = bcast(d.m, i), n = bcast(d.n, i), fmt = bcast(d.fmt, i);
          const T* P = base + bcast64(d.off, i);
          const int co0 = lo - bcast(d.c0, i), ldm = pad4(m);
          if (fmt == 0) {
            const double* x = tm.x + bcast(d.r0, i);
            const int g = lanes_per_col(m), cpp = 64 / g;
            const int q = lane & (g - 1), cg = lane / g;
            for (int c0 = 0; c0 < R; c0 += cpp) {
              const int c = c0 + cg;
              double s = 0.0;
              if (c < R) {
                const T* col = P + (int64_t)(co0 + c) * ldm;
#pragma unroll 4
                for (int r = 4 * q; r < m; r += 4 * g) {
                  double v[4];
                  load4(col + r, v);
#pragma unroll
                  for (int e = 0; e < 4; ++e)
                    if (r + e < m) s += v[e] * x[r + e];
                }
              }
              for (int o = g >> 1; o > 0; o >>= 1) s += __shfl_xor(s, o);
              if (q == 0 && c < R) yw[c] += al * s;
            }
          } else {
            const int k = bcast(d.k, i);
            const double* s = coef + bcast64(d.so, i);
            const T* V = P + (int64_t)ldm * k;
            const int ldn = pad4(n);
            if (lane < R) {
#pragma unroll 8
              for (int a = 0; a < k; ++a) accr += (double)V[co0 + lane + (int64_t)a * ldn] * (al * s[a]);
            }
          }
        }
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    yw[lane] += accr;
    __syncthreads();
    if (w == 0 && lane < R) {
      double sum = yacc[0][lane] + yacc[1][lane] + yacc[2][lane] + yacc[3][lane];
      if (J.base) sum += J.base[lo + lane];
      J.y[lo + lane] = sum;
    }
    __syncthreads();
  }
}

// Packed copy of one instance: one block per leaf; dense leaves and the
// U / V factors get leading dimensions padded to 4 (padding rows zero), low-
// rank leaves keep their `rank` columns only.
template <typename T>
__global__ __launch_bounds__(256) void pack_kernel(const T* src, const int32_t* rank, const DLeaf* leaves, int nleaf,
                                                   T* dst, const int64_t* off) {
  for (int l = blockIdx.x; l < nleaf; l += gridDim.x) {
    const DLeaf L = leaves[l];
    const T* s = src + L.off;
    T* d = dst + off[l];
    const int ldm = (L.m + 3) & ~3;
    if (L.fmt == 0) {
      for (int idx = threadIdx.x; idx < ldm * L.n; idx += blockDim.x) {
        const int i = idx % ldm, c = idx / ldm;
        d[idx] = i < L.m ? s[i + (int64_t)c * L.m] : T{};
      }
    } else {
      const int k = rank[l], ldn = (L.n + 3) & ~3;
      for (int idx = threadIdx.x; idx < ldm * k; idx += blockDim.x) {
        const int i = idx % ldm, a = idx / ldm;
        d[idx] = i < L.m ? s[i + (int64_t)a * L.m] : T{};
      }
      const T* sv = s + (int64_t)L.m * L.cap;
      T* dv = d + (int64_t)ldm * k;
      for (int idx = threadIdx.x; idx < ldn * k; idx += blockDim.x) {
        const int c = idx % ldn, a = idx / ldn;
        dv[idx] = c < L.n ? sv[c + (int64_t)a * L.n] : T{};
      }
    }
  }
}

template <typename T>
void launch_pack(const T* src, const int32_t* rank, const DLeaf* leaves, int nleaf, T* dst, const int64_t* off,
                 hipStream_t s) {
  const int grid = nleaf < 4096 ? nleaf : 4096;
  if (grid > 0) hipLaunchKernelGGL(pack_kernel<T>, dim3(grid), dim3(256), 0, s, src, rank, leaves, nleaf, dst, off);
}
template void launch_pack<double>(const double*, const int32_t*, const DLeaf*, int, double*, const int64_t*,
                                  hipStream_t);
template void launch_pack<float>(const float*, const int32_t*, const DLeaf*, int, float*, const int64_t*,
                                 hipStream_t);

template <typename T>
void launch_mv(const MvArgs<T>& a, hipStream_t s) {
  const int64_t n1 = ((int64_t)a.nterms * a.cw[5] + 3) / 4;
  const int g1 = (int)(n1 < 16384 ? n1 : 16384);
  if (g1 > 0) hipLaunchKernelGGL(mv_coef_kernel<T>, dim3(g1), dim3(256), 0, s, a);
  const int64_t n2 = (int64_t)a.njobs * a.nseg;
  const int g2 = (int)(n2 < 16384 ? n2 : 16384);
  if (g2 > 0) {
    if (a.trans)
      hipLaunchKernelGGL(mv_cols_kernel<T>, dim3(g2), dim3(256), 0, s, a);
    else
      hipLaunchKernelGGL(mv_rows_kernel<T>, dim3(g2), dim3(256), 0, s, a);
  }
}

template void launch_mv<double>(const MvArgs<double>&, hipStream_t);
template void launch_mv<float>(const MvArgs<float>&, hipStream_t);

}  // namespace acr
