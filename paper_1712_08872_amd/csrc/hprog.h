// Device-visible records that describe one batched H-arithmetic step.
//
// A formatted H-product C <- beta C + alpha A B (Hackbusch's recursion on the
// common block tree, Sec. 3-4 of the paper) is expanded once per plane
// shape, on the host, into a list of *targets* (the leaves of C that the
// step writes) and, per target, a list of *pieces*: the contributions of
// the recursion that land on that leaf, each a product of stored leaves
// restricted to a window of the target.  A kernel launch then processes
// (batch item x target) pairs; a batch item maps the abstract roles used
// in the pieces (e.g. "the matrix being inverted", "its scratch") to
// concrete H-matrix instances, which is how all planes of a cyclic
// reduction level share one launch.
#pragma once
#include <cstdint>

namespace acr {

constexpr int KC_MAX = 64;     // widest low-rank accumulation round the kernels support
constexpr int TPB = 256;       // threads per block of the H-arithmetic kernels
#ifndef ACR_DACC_ELEMS
#define ACR_DACC_ELEMS 16384
#endif
constexpr int DACC_ELEMS = ACR_DACC_ELEMS;  // low-rank targets with m*n up to this may be accumulated densely

enum PieceKind : int32_t {
  PK_LRX = 0,   // x low-rank A-leaf times a B-region (list): rank k_x
  PK_LRY = 1,   // A-region (list) times y low-rank B-leaf: rank k_y
  PK_DD = 2,    // dense A-leaf times dense B-leaf
  PK_COPY = 3,  // diag(rho) * (same leaf of another instance) * diag(gamma)
};

struct DLeaf {           // device copy of the leaf table
  int32_t m, n, r0, c0;
  int32_t fmt, cap;
  int64_t off;
};

struct Piece {
  int32_t kind;
  int32_t xrole, xleaf;  // LRX: low-rank A-leaf; DD: dense A-leaf; LRY: role of the A-list; COPY: source role/leaf
  int32_t yrole, yleaf;  // LRY: low-rank B-leaf; DD: dense B-leaf; LRX: role of the B-list
  int32_t l0, l1;        // list range into `lists` (leaf ids)
  int32_t wr0, wr1;      // window rows   (H-order plane indices)
  int32_t wc0, wc1;      // window columns
  int32_t rv, cv;        // COPY: vector roles for row / column scaling (-1 = none)
  double alpha;
};

struct Target {
  int32_t crole, cleaf;
  int32_t beta;          // 0: overwrite, 1: accumulate into the current value
  int32_t p0, p1;        // piece range
  int32_t direct;        // 1: beta = 0 and a single COPY piece -> exact copy
};

// flags written by kernels (device int array)
enum Flag : int32_t {
  FL_RANK_OVERFLOW = 0,  // a truncated rank exceeded the block's capacity
  FL_SINGULAR = 1,       // zero pivot in a dense leaf inverse
  FL_NONFINITE = 2,      // NaN/Inf met in a truncation
  FL_MAXRANK = 3,        // largest rank produced (atomicMax)
  FL_LAYOUT = 4,         // a packed (read-only) instance was addressed as a target
  FL_COUNT = 5
};

template <typename T>
struct AccumArgs {
  const DLeaf* leaves;
  const Piece* pieces;
  const Target* targets;
  const int32_t* lists;
  int32_t t0, nt;              // target range of this launch
  int32_t nbatch, nroles, nvroles;
  const int32_t* role_inst;    // [nbatch * nroles] instance ids (-1 = absent)
  const double* const* vec_ptr;  // [nbatch * nvroles] H-order plane vectors
  T* const* inst_base;         // [ninst]
  int32_t* const* inst_rank;   // [ninst] rank arrays (one entry per leaf)
  const int64_t* const* inst_off;  // [ninst] packed per-leaf offsets (null: capacity layout)
  T* scratch;                  // per block slot: (max_m + max_n) * round width
  int64_t scratch_stride;
  double eps;
  int32_t* flags;
  // two-phase steps: dense accumulators of small low-rank targets, filled
  // by the accumulate-only kernel and compressed by the truncating one
  T* dbuf;
  const int64_t* doff;         // per target (-1: none)
  int64_t dstride;             // per batch item
  int32_t mode;                // truncating kernel: 0 every low-rank target, 1 all but the dense
                               // sums, 2 the dense sums only
  unsigned long long* prof;    // optional cycle counters (null = off)
  double* flops;               // optional counters (null = off): flops by FlopClass, then algorithmic bytes
  int32_t bf16_products;       // 1: the matrix-core piece products take BF16 operands (rounded to
                               // nearest even) with FP32 accumulation (FP32 factors, eps >= 1e-2)
};

// Level-0 conversion of a plane block: entry d < nd of the scatter map
// (in-plane neighbour offset d of every row) takes stencil row row[d].
struct L0Rows {
  int32_t nd;
  int32_t row[9];
};

// classes of the algorithmic flop counters of the accumulation kernels
enum FlopClass : int32_t {
  FC_PRODUCT = 0,  // piece products and dense sums (GEMM-shaped)
  FC_GRAM = 1,     // Gram matrices of the factors
  FC_CORE = 2,     // pivoted Cholesky, core products, Jacobi rotations, triangular solves
  FC_REBUILD = 3,  // products forming the truncated factors
  FC_COUNT = 4
};

// cycle-counter slots of the accumulation kernel
enum ProfSlot : int32_t {
  PS_PIECES_LR = 0, PS_GRAM = 1, PS_EIG1 = 2, PS_EIG2 = 3, PS_REBUILD = 4, PS_DENSE = 5, PS_ITEMS = 6,
  PS_TRUNC = 7, PS_SWEEPS = 8, PS_NPIECES = 9, PS_KSUM = 10, PS_DACC = 11, PS_LRX = 12, PS_LRY = 13,
  PS_DDP = 14, PS_OUTER = 15, PS_TN = 16, PS_NN = 17, PS_COUNT = 18
};

struct MvTerm {
  int32_t inst;        // H-matrix instance (-1: none or diagonal)
  int32_t trans;
  double alpha;
  const double* x;     // H-order plane vector
  const double* dvec;  // diagonal term (if inst < 0 and dvec != null)
};

struct MvJob {
  double* y;
  const double* base;  // optional
  MvTerm t[2];
};

// Apply image of one H-matrix for one segment (leaf cluster) of R indices,
// as columns of ldR = pad4(R) elements (zero padding), contiguous from
// data_off.  Row image (H x): the segment's rows of every leaf covering
// them, first the nd columns of the dense leaves (weights from the term's
// input vector), then the nu columns of the U factors (weights from the
// term's coefficients V^T x).  Column image (H^T x): the segment's columns
// of the dense leaves covering them, transposed (weights from the input),
// then the segment's rows of the V factors (weights from U^T x).
// widx[widx_off + c] is the weight index of column c.
struct SegImg {
  int64_t data_off;
  int64_t widx_off;
  int32_t nd, nu;
};

template <typename T>
struct MvArgs {
  const DLeaf* leaves;
  const int64_t* soff;        // per leaf: offset of its coefficient slot (sum of caps)
  int64_t sstride;            // per (job, term) coefficient stride
  const MvJob* jobs;
  int32_t njobs;
  const int32_t* terms;       // non-empty H-matrix terms of the phase: 2 * job + term
  int32_t nterms;
  int32_t trans;              // 1: every term of the phase is transposed
  int32_t rounds;             // leaves per lane group and wavefront in the coefficient kernel (1 or 4)
  int32_t w4;                 // wavefronts per leaf of the longest class (4 columns each)
  // low-rank leaves ordered by the lane-group class of their column length
  // (4, 8, 16, 32, 64 lanes); cls[c] = first leaf of class c in lr_sorted,
  // cw[c] = first wavefront of class c within one job term (for `rounds`)
  const int32_t* lr_sorted;
  int32_t cls[6];
  int32_t cw[6];
  T* const* inst_base;
  int32_t* const* inst_rank;
  const int64_t* const* inst_off;  // packed per-leaf offsets (every factor is packed)
  double* coef;               // [njobs * 2 * sstride]
  const int32_t* seg_lo;      // [nseg + 1] H-order bounds of the leaf clusters (segments)
  int32_t nseg;
  // apply images of the phase's direction (row images for H x, column
  // images for H^T x): instance i's entry for a segment is
  // img_seg[img_of_inst[i] * nseg + segment]
  const T* img_data;
  const int32_t* img_widx;
  const SegImg* img_seg;
  const int32_t* img_of_inst;
};

}  // namespace acr
