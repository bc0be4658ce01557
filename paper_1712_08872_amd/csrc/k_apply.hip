// Batched H-matrix-vector products for the preconditioner sweeps.
//
// The apply phase of ACR is "solely based on H matrix-vector
// multiplications" (Sec. 5.3.1): each step of the forward/backward
// substitution multiplies every plane of a cyclic-reduction level by a
// stored H-matrix (Dinv_i or a coupling).  A *job* computes
//     y = base + sum_t alpha_t op_t(H_t) x_t
// for one plane, with up to two terms (op = identity or transpose; a term
// may also be a diagonal vector, the level-0 z-couplings).  Two kernels:
//   mv_lr_kernel   : s = V^T x_s (or U^T x_t) for every low-rank leaf, one
//                    wavefront per rank column, coalesced over the leaf rows;
//   mv_seg_kernel  : one block per (job, leaf cluster of the output): streams
//                    the dense leaves and the U (or V) rows covering that
//                    cluster once, reduces in registers + LDS.
// Everything is FP64 except the factor loads (T = float in mixed mode).
#include <hip/hip_runtime.h>

#include <cstdint>

#include "hprog.h"

namespace acr {

template <typename T>
__global__ __launch_bounds__(256) void mv_lr_kernel(MvArgs<T> A) {
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int64_t total = (int64_t)A.njobs * 2 * A.nlr;
  for (int64_t item = blockIdx.x; item < total; item += gridDim.x) {
    const int jt = (int)(item / A.nlr);
    const int li = (int)(item - (int64_t)jt * A.nlr);
    const MvJob& J = A.jobs[jt >> 1];
    const MvTerm& tm = J.t[jt & 1];
    if (tm.inst < 0) continue;
    const int l = A.lr_leaves[li];
    const DLeaf L = A.leaves[l];
    const int k = A.inst_rank[tm.inst][l];
    const int ldu = (L.m + 3) & ~3, ldv = (L.n + 3) & ~3;
    const T* U = A.inst_base[tm.inst] + A.inst_off[tm.inst][l];
    const T* V = U + (int64_t)ldu * k;
    double* out = A.coef + (int64_t)jt * A.sstride + A.soff[l];
    // transposed: s = U^T x[t]; otherwise s = V^T x[s]
    const T* F = tm.trans ? U : V;
    const int len = tm.trans ? L.m : L.n;
    const int ld = tm.trans ? ldu : ldv;
    const double* x = tm.x + (tm.trans ? L.r0 : L.c0);
    for (int a = wave; a < k; a += 4) {
      const T* f = F + (int64_t)a * ld;
      double s = 0.0;
      for (int i = lane; i < len; i += 64) s += (double)f[i] * x[i];
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
      if (lane == 0) out[a] = s;
    }
  }
}

template <typename T>
__global__ __launch_bounds__(256) void mv_seg_kernel(MvArgs<T> A) {
  __shared__ double red[256];
  const int tid = threadIdx.x;
  const int64_t total = (int64_t)A.njobs * A.nseg;
  for (int64_t item = blockIdx.x; item < total; item += gridDim.x) {
    const int j = (int)(item / A.nseg);
    const int sg = (int)(item - (int64_t)j * A.nseg);
    const MvJob& J = A.jobs[j];
    const int lo = A.seg_lo[sg], hi = A.seg_lo[sg + 1];
    const int R = hi - lo;                 // rows of this segment (<= 64)
    const int G = 256 / 64;                // column groups
    const int r = tid & 63, g = tid >> 6;
    double acc = 0.0;
    for (int tt = 0; tt < 2; ++tt) {
      const MvTerm& tm = J.t[tt];
      if (tm.inst < 0) {
        if (tm.dvec && g == 0 && r < R) acc += tm.alpha * tm.dvec[lo + r] * tm.x[lo + r];
        continue;
      }
      const T* base = A.inst_base[tm.inst];
      const int32_t* rk = A.inst_rank[tm.inst];
      const int64_t* po = A.inst_off[tm.inst];
      const double* coef = A.coef + (int64_t)(2 * j + tt) * A.sstride;
      double part = 0.0;
      if (!tm.trans) {
        for (int e = A.rows_ptr[sg]; e < A.rows_ptr[sg + 1]; ++e) {
          const int l = A.rows_idx[e];
          const DLeaf L = A.leaves[l];
          const T* P = base + po[l];
          const int ldm = (L.m + 3) & ~3;
          if (r >= R) continue;
          const int i = lo - L.r0 + r;
          if (L.fmt == 0) {
            const double* x = tm.x + L.c0;
            for (int c = g; c < L.n; c += G) part += (double)P[i + (int64_t)c * ldm] * x[c];
          } else {
            const int k = rk[l];
            const double* s = coef + A.soff[l];
            for (int a = g; a < k; a += G) part += (double)P[i + (int64_t)a * ldm] * s[a];
          }
        }
      } else {
        for (int e = A.cols_ptr[sg]; e < A.cols_ptr[sg + 1]; ++e) {
          const int l = A.cols_idx[e];
          const DLeaf L = A.leaves[l];
          const T* P = base + po[l];
          const int ldm = (L.m + 3) & ~3, ldn = (L.n + 3) & ~3;
          if (r >= R) continue;
          const int c = lo - L.c0 + r;
          if (L.fmt == 0) {
            const double* x = tm.x + L.r0;
            const T* col = P + (int64_t)c * ldm;
            for (int i = g; i < L.m; i += G) part += (double)col[i] * x[i];
          } else {
            const int k = rk[l];
            const double* s = coef + A.soff[l];
            const T* V = P + (int64_t)ldm * k;
            for (int a = g; a < k; a += G) part += (double)V[c + (int64_t)a * ldn] * s[a];
          }
        }
      }
      acc += tm.alpha * part;
    }
    red[tid] = acc;
    __syncthreads();
    if (g == 0 && r < R) {
      double s = red[r] + red[r + 64] + red[r + 128] + red[r + 192];
      if (J.base) s += J.base[lo + r];
      J.y[lo + r] = s;
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
        d[idx] = i < L.m ? s[i + (int64_t)c * L.m] : (T)0;
      }
    } else {
      const int k = rank[l], ldn = (L.n + 3) & ~3;
      for (int idx = threadIdx.x; idx < ldm * k; idx += blockDim.x) {
        const int i = idx % ldm, a = idx / ldm;
        d[idx] = i < L.m ? s[i + (int64_t)a * L.m] : (T)0;
      }
      const T* sv = s + (int64_t)L.m * L.cap;
      T* dv = d + (int64_t)ldm * k;
      for (int idx = threadIdx.x; idx < ldn * k; idx += blockDim.x) {
        const int c = idx % ldn, a = idx / ldn;
        dv[idx] = c < L.n ? sv[c + (int64_t)a * L.n] : (T)0;
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
  int64_t n1 = (int64_t)a.njobs * 2 * a.nlr;
  int g1 = (int)(n1 < 8192 ? n1 : 8192);
  if (g1 > 0) hipLaunchKernelGGL(mv_lr_kernel<T>, dim3(g1), dim3(256), 0, s, a);
  int64_t n2 = (int64_t)a.njobs * a.nseg;
  int g2 = (int)(n2 < 8192 ? n2 : 8192);
  if (g2 > 0) hipLaunchKernelGGL(mv_seg_kernel<T>, dim3(g2), dim3(256), 0, s, a);
}

template void launch_mv<double>(const MvArgs<double>&, hipStream_t);
template void launch_mv<float>(const MvArgs<float>&, hipStream_t);

}  // namespace acr
