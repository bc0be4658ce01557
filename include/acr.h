/*
 * acr.h -- C ABI of the accelerated cyclic reduction (ACR) library for
 * AMD MI355X (gfx950).
 *
 * Method (Chavez, Turkiyyah, Zampini, Keyes, "Parallel accelerated cyclic
 * reduction preconditioner for three-dimensional elliptic PDEs with
 * variable coefficients"):
 *   - Sec. 4.1: block cyclic reduction (red/black ordering of the grid
 *     planes, block Gaussian elimination without pivoting, recursive
 *     halving, forward/backward substitution);
 *   - Sec. 4.2: every plane block held as an H-matrix built on a planar
 *     bisection cluster tree (Sec. 3.1) with standard admissibility
 *     (eq. admis) and leaf size n_min;
 *   - Sec. 4.3: tuning parameters eps (block-wise relative accuracy of
 *     the low-rank blocks and of the H-arithmetic), eta, n_min;
 *   - Sec. 5.3, 7, 8: use as a preconditioner of CG / GMRES to a 1e-8
 *     relative residual.
 *
 * Conventions shared by every call
 *   - Grid: nx, ny, nz interior nodes on the unit cube, h_d = 1/(n_d+1),
 *     Dirichlet zero boundary.  Unknown p = i + nx*(j + ny*k), x fastest;
 *     a plane is a fixed k.  N = nx*ny*nz.
 *   - Node-grid fields (kappa, c, gradients) have (nz+2)*(ny+2)*(nx+2)
 *     entries, x fastest, boundary layer included.
 *   - All vector/field pointers are DEVICE pointers (hipMalloc'd or torch
 *     CUDA tensors) of doubles unless stated otherwise; the caller owns
 *     them.  The handle owns everything it allocates.
 *   - Work is ordered on the given stream (0 = the default stream).  Only
 *     acr_setup and krylov_solve block the host.  Handles are not
 *     thread-safe.
 *   - Every call returns an acr_status; no C++ exception crosses the ABI.
 *     Arguments are validated on the host before any device work; on
 *     failure *out handles are set to NULL and partial allocations are
 *     released.  acr_last_error() gives a thread-local message.
 */
#ifndef ACR_H
#define ACR_H

#include <stdint.h>
#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    ACR_OK = 0,
    ACR_E_INVALID = 1,   /* bad argument (null pointer, size, eps <= 0, ...) */
    ACR_E_NUMERIC = 2,   /* NaN/Inf or non-positive kappa detected */
    ACR_E_NOMEM = 3,     /* device allocation failed */
    ACR_E_SINGULAR = 4,  /* exactly singular dense leaf during H-inversion */
    ACR_E_BREAKDOWN = 5, /* Krylov breakdown (e.g. p'Ap <= 0 in CG) */
    ACR_E_NOTCONV = 6,   /* Krylov did not reach rtol within maxit */
    ACR_E_DEVICE = 7,    /* HIP runtime error or no usable gfx950 device */
    ACR_E_RANK = 8       /* rank capacity exhausted after all retries */
} acr_status;

typedef enum {
    ACR_POISSON_HARMONIC = 0, /* -div(kappa grad u), harmonic face averages (Sec. 6) */
    ACR_CONVDIFF_UPWIND = 1,  /* -div(kappa grad u) + beta.grad u, first-order upwind (Sec. 7) */
    ACR_HELMHOLTZ = 2,        /* -Lap u - (omega/c)^2 u, 7-point (Sec. 8, FD variant) */
    ACR_STENCIL7_RAW = 3,     /* caller-provided 7-point stencil */
    ACR_CONVDIFF_RECIRC = 4,  /* -div(kappa grad u) + alpha b(x).grad u with the divergence-free
                                 recirculating flow b of Sec. 7 (eq. codi), wavenumber a:
                                 beta_amp = alpha, beta_phase = a; first-order upwind per
                                 direction at the node */
    ACR_HELMHOLTZ_FEM27 = 5   /* -Lap u - (omega/c)^2 u discretised by continuous trilinear finite
                                 elements on the hexahedral grid (Sec. 8, eq. HelmVarVel: the
                                 27-point scheme): Q1 stiffness minus the mass weighted by
                                 omega^2/c^2, integrated by the 2x2x2 Gauss rule with c (node
                                 grid) interpolated trilinearly; the plane couplings are 9-point
                                 in-plane matrices, held as H-matrices from level 0 on */
} acr_kind;

typedef enum {
    ACR_FP64 = 0,       /* factors stored and multiplied in FP64 */
    ACR_MIXED_FP32 = 1, /* factors stored and multiplied in FP32; leaf
                           inversion, Gram matrices, core eigen/SVD and
                           Krylov in FP64 */
    ACR_MIXED_BF16 = 2  /* as ACR_MIXED_FP32, with the piece products of the
                           setup's H-arithmetic on the BF16 matrix cores:
                           their operands are rounded to BF16 (8-bit
                           mantissa, nearest even) and accumulated in FP32;
                           factors stored in FP32.  Only for eps >= 1e-2
                           (ACR_E_INVALID otherwise): the rounding, about
                           4e-3 relative per operand, must stay below the
                           truncation accuracy */
} acr_precision;

typedef enum { ACR_CG = 0, ACR_FCG = 1, ACR_GMRES = 2 } acr_method;

typedef struct {
    int32_t nx, ny, nz;
    int32_t kind;              /* acr_kind */
    const double* kappa;       /* device, node grid; POISSON/CONVDIFF; NULL -> kappa = 1 */
    double beta_amp;           /* CONVDIFF: beta_d(x) = beta_amp (1 + 0.5 sin(2 pi x + beta_phase)), d = x,y,z */
    double beta_phase;
    const double* c;           /* device, node grid; HELMHOLTZ wave speed */
    double omega;              /* HELMHOLTZ angular frequency */
    const double* stencil7;    /* device, 7*N; RAW: rows centre, x-1, x+1, y-1, y+1, z-1, z+1 */
} acr_problem;

typedef void* (*acr_alloc_fn)(size_t bytes, void* ctx);
typedef void (*acr_free_fn)(void* ptr, void* ctx);

/* Smallest accepted eps.  The truncation T_eps (Sec. 3.1.5, Sec. 4.3) keeps
 * the singular values sigma_i > eps sigma_1 of a block; it finds them from
 * FP64 Gram matrices of the factors, whose eigenvalues resolve singular
 * values down to about 1e-8 sigma_1, so a smaller eps is rejected with
 * ACR_E_INVALID instead of being silently met only to about 1e-8. */
#define ACR_EPS_MIN 1e-7

typedef struct {
    double eps;                /* block-wise relative truncation accuracy, in [ACR_EPS_MIN, 1) */
    double eta;                /* admissibility parameter, > 0 */
    int32_t leaf_size;         /* n_min: cluster leaves have <= leaf_size points (8..64) */
    int32_t precision;         /* acr_precision */
    int32_t max_rank;          /* rank cap of the low-rank blocks (<= 56).  0 = automatic: the
                                  capacity starts at 6 + 6 log10(1/eps) and the setup is redone
                                  with larger capacities when a rank overflows.  > 0: a fixed
                                  cap; ranks are clamped to it and acr_stats reports
                                  rank_overflow = 1 (the factors are then less accurate than
                                  eps, a Krylov solve still converges) */
    int32_t dense_work;        /* admissible blocks with min dimension <= dense_work are kept
                                  dense (exact) during setup; 0 = paper's format everywhere */
    acr_alloc_fn alloc;        /* optional device allocator (NULL -> hipMalloc) */
    acr_free_fn free;
    void* alloc_ctx;
    uint64_t flags;            /* reserved, must be 0 */
} acr_options;

typedef struct {
    int32_t iters;
    double relres_true;        /* ||b - A x||_2 / ||b||_2 recomputed at exit */
    int32_t status;            /* acr_status of the solve */
    int32_t variant;           /* method actually used (CG may switch to FCG) */
} acr_solve_info;

#define ACR_MAX_LEVELS 32

typedef struct {
    int32_t levels;                        /* CR levels (eliminations incl. top) */
    int32_t nplanes;                       /* nz */
    int32_t plane_points;                  /* nx*ny */
    int32_t clusters, dense_leaves, lr_leaves;
    int32_t factors;                       /* stored H-matrices */
    int32_t retries;                       /* setups redone after rank overflow */
    int32_t rank_overflow;                 /* 1 if a rank was clamped to the capacity limit */
    int32_t max_rank[ACR_MAX_LEVELS];      /* per CR level */
    double mean_rank[ACR_MAX_LEVELS];
    int32_t max_rank_all;
    double bytes_factors;                  /* stored factor bytes (actual ranks) */
    double bytes_allocated;                /* device bytes held by the handle */
    double bytes_per_apply;                /* algorithmic bytes streamed by one acr_apply */
    double setup_seconds;
    double setup_flops;                    /* algorithmic flops counted in setup */
    int32_t precision;
    /* with the environment variable ACR_KERNEL_TIMING=1 at setup time: the
       H-arithmetic truncating kernel's launch count, summed launch
       durations (HIP events on the launch stream) and algorithmic flops */
    int32_t accum_launches;
    double accum_seconds;
    double accum_flops;
    /* the accumulate-only first phase of every H-arithmetic step (dense
       targets and dense sums of small low-rank targets), timed like the
       accumulation kernel above, which then covers the truncating phase */
    int32_t dense_launches;
    double dense_seconds;
    double dense_flops;
    double bytes_peak;                     /* largest device footprint reached during setup (a
                                              batched handle with several shape groups: the sum
                                              of the groups' peaks, an upper bound) */
    double bytes_level[ACR_MAX_LEVELS];    /* stored factor bytes per CR level (Dinv and the
                                              couplings of the level; the top inverse is the
                                              last level) */
    double level_seconds[ACR_MAX_LEVELS];  /* setup wall time per CR level (host clock, the
                                              stream synchronised at level boundaries) */
    /* algorithmic setup flops by class (Sec. 6.4's operation count, counted in the kernels
       from the operand sizes of every operation, with ACR_KERNEL_TIMING=1): [0] piece
       products and dense sums (GEMM-shaped), [1] Gram matrices of the factors, [2] core
       factorisations (pivoted Cholesky, core products, Jacobi rotations, triangular
       solves), [3] the products forming the truncated factors */
    double setup_flops_class[4];
    double leaf_inverse_flops;             /* 2 m^3 per m x m dense diagonal leaf inverted
                                              (LU with partial pivoting and inverse), always
                                              counted; setup_flops = the classes + this */
    double bytes_apply_image;              /* device bytes of the apply images: every H-matrix
                                              that acr_apply multiplies, stored a second time
                                              row segment by row segment (its dense leaves and U
                                              factors) for the row kernel; part of
                                              bytes_allocated, not of bytes_factors */
    /* algorithmic bytes of the two H-arithmetic kernels (with ACR_KERNEL_TIMING=1), summed
       over their launches: every operand entry a piece product reads (factor rows, leaf
       blocks; once per product), each target's old value or dense sum read and its result
       written, at storage precision; scratch traffic is not counted */
    double accum_bytes;
    double dense_bytes;
} acr_stats_t;

typedef struct acr_handle acr_handle;

/* Build the ACR factorisation of the problem (Sec. 4.1-4.2).  Blocks the
 * host until the factors are complete.  *out receives a new handle. */
acr_status acr_setup(const acr_problem* p, const acr_options* o, void* stream,
                     acr_handle** out);

/* Set up `count` independent problems (1 <= count <= 4096) in one handle.
 * Problems with the same (nx, ny, nz) form a group whose cyclic-reduction
 * levels run in lockstep: every H-arithmetic step and every apply phase is
 * one batched launch over all planes of all problems of the group.  Every
 * vector argument of a batched handle (apply, apply_T, matvec, Krylov,
 * gradient) is the concatenation of the problems' vectors in the order
 * given; acr_problem_offset gives the slices.  Problem i's factors equal
 * those of acr_setup on problem i alone (same arithmetic, same order). */
acr_status acr_setup_batched(const acr_problem* ps, int32_t count, const acr_options* o, void* stream,
                             acr_handle** out);

/* Offset and length of problem i's unknowns and of its node grid inside
 * the concatenated vectors of a (batched) handle.  Any output may be NULL. */
acr_status acr_problem_offset(const acr_handle* h, int32_t i, int64_t* off, int64_t* n, int64_t* grid_off,
                              int64_t* grid_n);

/* Number of problems held by a handle (0 for NULL). */
int32_t acr_num_problems(const acr_handle* h);

/* z = M^{-1} r, forward elimination / top solve / back substitution
 * (Sec. 4.1) with H-matrix-vector products (Sec. 5.3).  r, z: device,
 * N*nrhs doubles, natural ordering, column-major by right-hand side; z
 * must not alias r. */
acr_status acr_apply(acr_handle* h, const double* r, double* z, int32_t nrhs, void* stream);

/* z = M^{-T} r, the exact transpose of the linear map of acr_apply: the
 * substitution sweeps of Sec. 4.1 in reverse order with every stored
 * H-matrix transposed (the adjoint solves of the gradient and of A^T x = b).
 * Arguments, layout and errors as acr_apply. */
acr_status acr_apply_T(acr_handle* h, const double* r, double* z, int32_t nrhs, void* stream);

/* y = A x (transpose = 0) or A^T x (transpose = 1) with the assembled
 * operator (the 7-point discretisations of Sec. 6 eq. poissonEquation, Sec.
 * 7 eq. codi and Sec. 8, or the 27-point FEM of Sec. 8 eq. HelmVarVel), the
 * operator the Krylov methods of Sec. 5.3 iterate on; x, y device, N
 * doubles (a batched handle: all problems concatenated), natural ordering,
 * y must not alias x.  ACR_E_INVALID for null pointers. */
acr_status acr_matvec(acr_handle* h, int32_t transpose, const double* x, double* y, void* stream);

/* Copy the assembled stencil to the device buffer out: 7*N doubles in the
 * layout of acr_problem.stencil7, or for ACR_HELMHOLTZ_FEM27 27*N doubles,
 * row m = (dx+1) + 3 (dy+1) + 9 (dz+1) holding the coupling to the
 * neighbour at offset (dx, dy, dz) (row 13 the centre).  A batched handle
 * writes its problems one after another, each with its own row count. */
acr_status acr_get_stencil(acr_handle* h, double* out, void* stream);

/* Preconditioned Krylov solve of A x = b (or A^T x = b when transpose=1,
 * then preconditioned by acr_apply_T) from the initial guess in x,
 * stopping at ||b - A x||/||b|| <= rtol (Sec. 5.3: CG, 2-norm, 1e-8;
 * Sec. 7-8: GMRES).  CG: Fletcher-Reeves; FCG: Polak-Ribiere; CG switches
 * to FCG if the residual stagnates for 5 iterations.  GMRES: right
 * preconditioning, restart m = restart, classical Gram-Schmidt with
 * reorthogonalisation.  Dots and norms in FP64.  Blocks the host. */
acr_status krylov_solve(acr_handle* h, int32_t method, int32_t restart, int32_t transpose,
                        double rtol, int32_t maxit, const double* b, double* x,
                        acr_solve_info* info, void* stream);

/* krylov_solve without allocating: for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid allocation).  Same arguments, semantics and results as
 * krylov_solve, but the Krylov work vectors, the dot-product partials and
 * the result slots live in a fixed array of ACR_STATIC_WORKSPACE_BYTES in
 * the library's device code object (one per GPU, held until the process
 * ends) instead of memory the handle allocates at its first solve; the call
 * allocates no device or pinned host memory.  The handle itself is made by
 * acr_setup, which allocates.  CG/FCG need 5 vectors of the largest
 * problem's N doubles, GMRES(m) 2m + 3; ACR_E_INVALID if they do not fit
 * (CG fits up to about 3.3 million unknowns per problem, GMRES(30) up to
 * about 266 thousand).  Every call on a GPU shares that GPU's array: calls
 * that overlap on one GPU (concurrent host threads or streams) race. */
#define ACR_STATIC_WORKSPACE_BYTES (128u << 20)

acr_status krylov_solve_static(acr_handle* h, int32_t method, int32_t restart, int32_t transpose, double rtol,
                               int32_t maxit, const double* b, double* x, acr_solve_info* info, void* stream);

/* Adjoint gradient for ACR_POISSON_HARMONIC (the operator of Sec. 6 eq.
 * poissonEquation with the harmonic face average): dkappa = -lam^T
 * (dA/dkappa) u, the derivative of A u with respect to every node value of
 * kappa contracted with the adjoint state lam (computed by the caller with
 * acr_apply_T / krylov_solve(transpose = 1)).  u, lam: device, N doubles;
 * dkappa: device, the node grid ((nz+2)(ny+2)(nx+2) doubles, overwritten).
 * ACR_E_INVALID for other problem kinds or null pointers. */
acr_status acr_grad_kappa(acr_handle* h, const double* u, const double* lam, double* dkappa,
                          void* stream);

/* Plane geometry (Sec. 3.1.2-3.1.4 with the planar bisection of Sec. 4.2;
 * eq. admis): the cluster tree of an nx x ny plane (a box with at most
 * o->leaf_size points is a leaf; otherwise its longer side is split, ties
 * splitting x, into floor(s/2) and the rest, lower coordinates first),
 * the block tree under the admissibility test dist > 0 and
 * min(diam t, diam s) <= o->eta dist (bounding boxes in grid units,
 * Euclidean), and the H-order of the plane's unknowns (depth-first leaf
 * order).  This is the geometry acr_setup builds for every plane of that
 * shape with the same options.  Host only: needs no device.
 *   info   : counts (required);
 *   perm   : host, nx*ny int32 or NULL: perm[i] = natural in-plane index
 *            x + nx*y of H-order position i;
 *   leaves : host, 6*leaves_cap int32 or NULL: per leaf of the block tree,
 *            in the library's leaf order, (r0, c0, m, n, admissible,
 *            low_rank): the block's first row and column in H-order, its
 *            size, 1 if eq. admis holds, 1 if it is stored low rank (an
 *            admissible leaf is stored dense when its smaller dimension is
 *            at most o->dense_work, or when it holds an in-plane coupling
 *            of the 5-point operator, possible only for large eta);
 *            ACR_E_INVALID if leaves_cap < info->leaves. */
typedef struct {
    int32_t clusters;          /* nodes of the cluster tree */
    int32_t leaf_clusters;
    int32_t depth;             /* largest cluster depth (root 0) */
    int32_t block_nodes;       /* nodes of the block tree */
    int32_t leaves;            /* leaves of the block tree */
    int32_t admissible;        /* leaves for which eq. admis holds */
    int32_t dense_leaves;      /* leaves stored dense */
    int32_t lr_leaves;         /* leaves stored low rank */
} acr_geometry_info;

acr_status acr_plane_geometry(int32_t nx, int32_t ny, const acr_options* o, acr_geometry_info* info,
                              int32_t* perm, int32_t* leaves, int32_t leaves_cap);
/* (The geometry is that of the 7-point operators; with ACR_HELMHOLTZ_FEM27
 * an admissible leaf holding a diagonal in-plane coupling is also stored
 * dense, which happens only for eta above about 5.) */

/* ---- Test hook: factors built elsewhere (e.g. by a CPU reference) ----
 *
 * The stored factors of the cyclic reduction (Sec. 4.1, with every plane
 * block an H-matrix as in Sec. 4.2): per level r of the plane lists
 * P_0 = (0..nz-1), P_{r+1} = planes at the 1-based even positions of P_r,
 * the inverse Dinv_i of every eliminated plane i (1-based odd positions of
 * P_r) and the couplings A_p (to the previous plane of P_r) and C_p (to the
 * next) of every plane p of P_r, as they are before level r updates them;
 * the last level holds the single remaining plane's inverse only.  A
 * coupling that is not given is absent (zero).  acr_import_factors loads
 * such a factorisation instead of computing it, so that acr_apply,
 * acr_apply_T and krylov_solve run on exactly the given factors.
 *
 * Each factor's data is on the HOST, read during the call only (the caller
 * keeps ownership).  An H-matrix factor lists its leaves in the order of
 * acr_plane_geometry (same nx, ny and options): a dense leaf as m x n
 * column-major, a low-rank leaf as U (m x k, column-major) followed by
 * V (n x k, column-major) with the block U V^T and k = ranks[l]
 * (0 <= k <= min(m, n); entries of dense leaves are ignored).  Rows and
 * columns are in H-order.  A diagonal factor (diag = 1, the level-0
 * z-couplings) holds nx*ny doubles in H-order. */
typedef enum { ACR_FACTOR_DINV = 0, ACR_FACTOR_A = 1, ACR_FACTOR_C = 2 } acr_factor_role;

typedef struct {
    int32_t level;             /* cyclic-reduction level r (the top inverse: the last level) */
    int32_t role;              /* acr_factor_role */
    int32_t plane;             /* 0-based plane index k */
    int32_t diag;              /* 1: diagonal coupling (nx*ny doubles), 0: H-matrix */
    const int32_t* ranks;      /* host, one per leaf (H-matrix factors) */
    const double* data;        /* host, the leaves in order (or the diagonal) */
} acr_factor;

typedef struct {
    int32_t count;
    const acr_factor* factors; /* host array of count factors */
} acr_factor_blob;

/* A handle for problem p (its operator is assembled as in acr_setup, for
 * acr_matvec and krylov_solve) whose preconditioner is the given
 * factorisation.  o->precision ACR_FP64 stores the factors as given,
 * ACR_MIXED_FP32 rounds them to FP32 (ACR_MIXED_BF16 is refused); the
 * geometry follows o->leaf_size, o->eta and o->dense_work.  ACR_E_INVALID
 * if a factor is out of range or duplicated, a rank is out of range, a
 * required inverse is missing or an H-matrix factor has no data.  Used by
 * the tests that pin the apply kernels to a reference factorisation. */
acr_status acr_import_factors(const acr_problem* p, const acr_options* o, const acr_factor_blob* blob, void* stream,
                              acr_handle** out);

/* Statistics of a handle: ranks and bytes per level (the memory footprint
 * of Sec. 6.4 and Sec. 8.3: the sum of the stored H-matrices at their
 * actual ranks), algorithmic bytes per application, setup flops by class
 * (the operation count of Sec. 6.4), timings.  st: host, filled on
 * success; ACR_E_INVALID for null pointers. */
acr_status acr_stats(const acr_handle* h, acr_stats_t* st);

/* Release a handle and all device memory it owns (NULL is ignored). */
void acr_destroy(acr_handle* h);

const char* acr_status_string(acr_status s);
const char* acr_last_error(void);

/* Default options: eps 1e-4, eta 2, leaf 32, FP64, automatic capacity,
 * dense_work 0. */
void acr_default_options(acr_options* o);

#ifdef __cplusplus
}
#endif
#endif /* ACR_H */
