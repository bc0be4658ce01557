// Batched H-matrix-vector products for the preconditioner sweeps.
//
// The apply phase of ACR consists of H-matrix-vector products only
// (Sec. 5.3.1): each step of the forward/backward substitution multiplies
// every plane of a cyclic-reduction level by a stored H-matrix (Dinv_i or a
// coupling).  A *job* computes
//     y = base + sum_t alpha_t op_t(H_t) x_t
// for one plane, with up to two terms (op = identity or transpose; a term
// may also be a diagonal vector, the level-0 z-couplings).  Two kernels per
// phase, no atomics:
//   mv_coef_kernel : s = V^T x (or U^T x) per (job term, low-rank leaf) on
//                    the packed factors (exact ranks, leading dimensions
//                    padded to 4, 16-byte column loads), whose V (U)
//                    columns are contiguous; a power-of-two group of lanes
//                    per column;
//   mv_seg_kernel  : y = sum D x + sum U s per (job, row segment), or
//                    y = sum D^T x + sum V s per (job, column segment), from
//                    the apply images: per segment and H-matrix, every
//                    column the segment needs stored contiguously with the
//                    index of its weight (see SegImg), built once at the end
//                    of the setup by img_build_kernel.
// Sums are formed in a fixed order (deterministic results).  Arithmetic is
// FP64; the factor loads are FP32 in mixed precision.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

#include "hprog.h"

namespace acr {

__device__ __forceinline__ int pad4(int x) { return (x + 3) & ~3; }
__device__ __forceinline__ int imin_(int a, int b) { return a < b ? a : b; }

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

// ------------------------------------------------------------ apply images
// Image of (image i, segment s), one block each.  Row image (trans = 0):
// rows [lo, lo + R) of the segment's dense leaves, then of the U factors of
// its low-rank leaves, as columns of ldR = pad4(R) elements (padding rows
// zero); the weight index of dense column c is c0 + c (the term's input
// vector), of U column a it is soff + a (the term's coefficients V^T x).
// Column image (trans = 1), for H^T: the segment's columns [lo, lo + R) of
// the dense leaves covering them, transposed (row r of the leaf becomes a
// column, weight index r0 + r), then the rows [lo, lo + R) of the V factors
// (weight index soff + a: the coefficients U^T x).  Leaves in the order of
// the segment's leaf list; the host sized every segment from the same ranks.
template <typename T>
__global__ __launch_bounds__(256) void img_build_kernel(T* const* inst_base, int32_t* const* inst_rank,
                                                        const int64_t* const* inst_off, const DLeaf* leaves,
                                                        const int64_t* soff, const int32_t* seg_lo,
                                                        const int32_t* list_ptr, const int32_t* list_idx, int nseg,
                                                        int trans, const int32_t* img_inst, const SegImg* img_seg,
                                                        int nimg, T* img_data, int32_t* img_widx) {
  __shared__ int s_cnt[2][256];  // running column counts: dense leaves, low-rank leaves
  __shared__ int s_cur[256];     // first image column of each leaf of the chunk
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  for (int64_t b = blockIdx.x; b < (int64_t)nimg * nseg; b += gridDim.x) {
    const int im = (int)(b / nseg), sg = (int)(b - (int64_t)im * nseg);
    const int X = img_inst[im];
    const SegImg si = img_seg[b];
    const int lo = seg_lo[sg], R = seg_lo[sg + 1] - lo, ldR = pad4(R);
    T* out = img_data + si.data_off;
    int32_t* wi = img_widx + si.widx_off;
    const T* base = inst_base[X];
    const int e0 = list_ptr[sg], ne = list_ptr[sg + 1] - e0;
    int carry0 = 0, carry1 = 0;  // columns of the chunks before (uniform)
    for (int ec = 0; ec < ne; ec += 256) {
      // each thread sizes one leaf; prefix sums place dense leaves first,
      // then the low-rank factors, each group in list order
      int fmt = 0, nc = 0;
      if (ec + tid < ne) {
        const int l = list_idx[e0 + ec + tid];
        const DLeaf L = leaves[l];
        fmt = L.fmt;
        nc = fmt ? inst_rank[X][l] : (trans ? L.m : L.n);
      }
      s_cnt[0][tid] = fmt ? 0 : nc;
      s_cnt[1][tid] = fmt ? nc : 0;
      __syncthreads();
      for (int o = 1; o < 256; o <<= 1) {
        const int a0 = tid >= o ? s_cnt[0][tid - o] : 0, a1 = tid >= o ? s_cnt[1][tid - o] : 0;
        __syncthreads();
        s_cnt[0][tid] += a0;
        s_cnt[1][tid] += a1;
        __syncthreads();
      }
      s_cur[tid] = fmt ? si.nd + carry1 + s_cnt[1][tid] - nc : carry0 + s_cnt[0][tid] - nc;
      const int tot0 = s_cnt[0][255], tot1 = s_cnt[1][255];
      __syncthreads();
      // wavefront w copies leaves w, w + 4, ... of the chunk
      const int nchunk = ne - ec < 256 ? ne - ec : 256;
      for (int t = w; t < nchunk; t += 4) {
        const int l = list_idx[e0 + ec + t];
        const DLeaf L = leaves[l];
        const int k = L.fmt ? inst_rank[X][l] : 0;
        const int ldm = pad4(L.m), ldn = pad4(L.n), cur = s_cur[t];
        const T* src = base + inst_off[X][l];
        int ncl;
        int64_t off0, cstride, rstride;
        if (!trans) {  // dense columns or U columns, rows lo - r0 ...
          ncl = L.fmt ? k : L.n;
          off0 = lo - L.r0;
          cstride = ldm;
          rstride = 1;
        } else if (L.fmt) {  // V columns, rows lo - c0 ...
          ncl = k;
          src += (int64_t)ldm * k;
          off0 = lo - L.c0;
          cstride = ldn;
          rstride = 1;
        } else {  // rows of the dense leaf, columns lo - c0 ...
          ncl = L.m;
          off0 = (int64_t)(lo - L.c0) * ldm;
          cstride = 1;
          rstride = ldm;
        }
        for (int idx = lane; idx < ncl * ldR; idx += 64) {
          const int c = idx / ldR, r = idx - c * ldR;
          out[(int64_t)(cur + c) * ldR + r] = r < R ? src[off0 + (int64_t)c * cstride + (int64_t)r * rstride] : T{};
          if (r == 0) wi[cur + c] = L.fmt ? (int32_t)(soff[l] + c) : (trans ? L.r0 : L.c0) + c;
        }
      }
      carry0 += tot0;
      carry1 += tot1;
      __syncthreads();  // the chunk's LDS is read before the next one overwrites it
    }
  }
}

template <typename T>
void launch_img_build(T* const* inst_base, int32_t* const* inst_rank, const int64_t* const* inst_off,
                      const DLeaf* leaves, const int64_t* soff, const int32_t* seg_lo, const int32_t* list_ptr,
                      const int32_t* list_idx, int nseg, int trans, const int32_t* img_inst, const SegImg* img_seg,
                      int nimg, T* img_data, int32_t* img_widx, hipStream_t s) {
  const int64_t n = (int64_t)nimg * nseg;
  const int grid = (int)(n < 16384 ? n : 16384);
  if (grid > 0)
    hipLaunchKernelGGL(img_build_kernel<T>, dim3(grid), dim3(256), 0, s, inst_base, inst_rank, inst_off, leaves, soff,
                       seg_lo, list_ptr, list_idx, nseg, trans, img_inst, img_seg, nimg, img_data, img_widx);
}
template void launch_img_build<double>(double* const*, int32_t* const*, const int64_t* const*, const DLeaf*,
                                       const int64_t*, const int32_t*, const int32_t*, const int32_t*, int, int,
                                       const int32_t*, const SegImg*, int, double*, int32_t*, hipStream_t);
template void launch_img_build<float>(float* const*, int32_t* const*, const int64_t* const*, const DLeaf*,
                                      const int64_t*, const int32_t*, const int32_t*, const int32_t*, int, int,
                                      const int32_t*, const SegImg*, int, float*, int32_t*, hipStream_t);

// y[lo:hi] (+)= sum_t alpha_t (H_t x_t)[lo:hi] (row images) or
// sum_t alpha_t (H_t^T x_t)[lo:hi] (column images), one block per (job,
// segment).  The segment's image columns of a term are contiguous, so they
// stream with 16-byte loads: thread = (column group cg, row quad q) with
// g = ldR / 4 threads per column, cpb = 256 / g columns per block step and U
// columns in flight per thread; each column is weighted by the input-vector
// or coefficient entry its index names.  The column groups' partial rows
// are added in a fixed order (deterministic).
template <typename T>
__global__ __launch_bounds__(256) void mv_seg_kernel(MvArgs<T> A) {
  constexpr int U = 4;  // columns in flight per thread
  __shared__ double red[1024];
  const int tid = threadIdx.x;
  const int64_t nitems = (int64_t)A.njobs * A.nseg;
  for (int64_t item = blockIdx.x; item < nitems; item += gridDim.x) {
    const int j = (int)(item / A.nseg);
    const int sg = (int)(item - (int64_t)j * A.nseg);
    const MvJob& J = A.jobs[j];
    const int lo = A.seg_lo[sg], R = A.seg_lo[sg + 1] - lo;  // R <= 64
    const int ldR = pad4(R), g = ldR >> 2, cpb = 256 / g;
    const int q = tid % g, cg = tid / g;
    const bool act = cg < cpb;
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    double accr = 0.0;
    for (int tt = 0; tt < 2; ++tt) {
      const MvTerm& tm = J.t[tt];
      if (tm.inst < 0) {
        if (tm.dvec && tid < R) accr += tm.alpha * tm.dvec[lo + tid] * tm.x[lo + tid];
        continue;
      }
      const SegImg si = A.img_seg[(int64_t)A.img_of_inst[tm.inst] * A.nseg + sg];
      const T* d = A.img_data + si.data_off + 4 * q;
      const int32_t* wi = A.img_widx + si.widx_off;
      const double* xw = tm.x;
      const double* cw = A.coef + (int64_t)(2 * j + tt) * A.sstride;
      const double al = tm.alpha;
      const int nc = act ? si.nd + si.nu : 0, nd = si.nd;
      int c = cg;
      for (; c + (U - 1) * cpb < nc; c += U * cpb) {
        T v[U][4];
        int k[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
          load4raw(d + (int64_t)(c + u * cpb) * ldR, v[u]);
          k[u] = wi[c + u * cpb];
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const double wt = al * (c + u * cpb < nd ? xw[k[u]] : cw[k[u]]);
#pragma unroll
          for (int r = 0; r < 4; ++r) acc[r] += (double)v[u][r] * wt;
        }
      }
      for (; c < nc; c += cpb) {
        T v[4];
        load4raw(d + (int64_t)c * ldR, v);
        const int k = wi[c];
        const double wt = al * (c < nd ? xw[k] : cw[k]);
#pragma unroll
        for (int r = 0; r < 4; ++r) acc[r] += (double)v[r] * wt;
      }
    }
    if (act)
#pragma unroll
      for (int r = 0; r < 4; ++r) red[cg * ldR + 4 * q + r] = acc[r];
    __syncthreads();
    if (tid < R) {
      double sum = accr;
      for (int k = 0; k < cpb; ++k) sum += red[k * ldR + tid];
      if (J.base) sum += J.base[lo + tid];
      J.y[lo + tid] = sum;
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

// A phase without H-matrix terms (the level-0 updates with diagonal
// couplings): y = base + sum_t alpha_t d_t .* x_t elementwise over the
// jobs' planes, in the order the segment kernel adds them.
template <typename T>
__global__ __launch_bounds__(256) void mv_diag_kernel(MvArgs<T> A) {
  const int64_t B = A.seg_lo[A.nseg];
  const int64_t n = (int64_t)A.njobs * B;
  for (int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g < n; g += (int64_t)gridDim.x * blockDim.x) {
    const int j = (int)(g / B);
    const int64_t i = g - (int64_t)j * B;
    const MvJob& J = A.jobs[j];
    double sum = 0.0;
    for (int tt = 0; tt < 2; ++tt)
      if (J.t[tt].dvec) sum += J.t[tt].alpha * J.t[tt].dvec[i] * J.t[tt].x[i];
    if (J.base) sum += J.base[i];
    J.y[i] = sum;
  }
}

// One apply phase: the coefficient kernel and the segment kernel, or the
// elementwise kernel when the phase has no H-matrix terms.
template <typename T>
void launch_mv(const MvArgs<T>& a, hipStream_t s) {
  const int64_t n1 = ((int64_t)a.nterms * a.cw[5] + 3) / 4;
  const int g1 = (int)(n1 < 16384 ? n1 : 16384);
  if (g1 > 0) hipLaunchKernelGGL(mv_coef_kernel<T>, dim3(g1), dim3(256), 0, s, a);
  if (a.nterms == 0) {  // diagonal terms only
    if (a.njobs > 0) hipLaunchKernelGGL(mv_diag_kernel<T>, dim3(4096), dim3(256), 0, s, a);
    return;
  }
  const int64_t n2 = (int64_t)a.njobs * a.nseg;
  const int g2 = (int)(n2 < 16384 ? n2 : 16384);
  if (g2 > 0) hipLaunchKernelGGL(mv_seg_kernel<T>, dim3(g2), dim3(256), 0, s, a);
}

template void launch_mv<double>(const MvArgs<double>&, hipStream_t);
template void launch_mv<float>(const MvArgs<float>&, hipStream_t);

}  // namespace acr
