// Handle state and internal interfaces of the ACR runtime.
#pragma once
#include <hip/hip_runtime.h>

#include <chrono>
#include <map>
#include <memory>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/acr.h"
#include "geometry.h"
#include "hprog.h"
#include "program.h"

namespace acr {

struct AcrError : std::runtime_error {
  acr_status st;
  AcrError(acr_status s, const std::string& m) : std::runtime_error(m), st(s) {}
};

#define HIPCHK(expr)                                                                                 \
  do {                                                                                               \
    hipError_t e_ = (expr);                                                                          \
    if (e_ != hipSuccess)                                                                            \
      throw ::acr::AcrError(e_ == hipErrorOutOfMemory ? ACR_E_NOMEM : ACR_E_DEVICE,                  \
                            std::string(#expr) + ": " + hipGetErrorString(e_));                      \
  } while (0)

// kernel launchers (the accumulation kernel exists for round widths 38 and 64)
namespace kc38 {
template <typename T> void launch_accum(const AccumArgs<T>&, int grid, hipStream_t);
template <typename T> void launch_accum_dense(const AccumArgs<T>&, int grid, hipStream_t);
}
namespace kc64 {
template <typename T> void launch_accum(const AccumArgs<T>&, int grid, hipStream_t);
template <typename T> void launch_accum_dense(const AccumArgs<T>&, int grid, hipStream_t);
}
template <typename T>
void launch_leaf_inverse(T* const*, const int32_t*, int stride, int ninst, int64_t off, int m, int32_t* flags,
                         hipStream_t);
template <typename T>
void launch_level0(T* const*, const int32_t*, int nplanes, int plane0, const double* S, int64_t N, int B,
                   const int32_t* perm, const int64_t* map, const L0Rows& rows, hipStream_t);
void launch_zcoupling(const double* S, int64_t N, int B, int nz, const int32_t* perm, double* outA, double* outC,
                      hipStream_t);
template <typename T> void launch_mv(const MvArgs<T>&, hipStream_t);
template <typename T>
void launch_img_build(T* const* inst_base, int32_t* const* inst_rank, const int64_t* const* inst_off,
                      const DLeaf* leaves, const int64_t* soff, const int32_t* seg_lo, const int32_t* list_ptr,
                      const int32_t* list_idx, int nseg, int trans, const int32_t* img_inst, const SegImg* img_seg,
                      int nimg, T* img_data, int32_t* img_widx, hipStream_t s);
template <typename T>
void launch_pack(const T* src, const int32_t* rank, const DLeaf* leaves, int nleaf, T* dst, const int64_t* off,
                 hipStream_t);
void launch_assemble(int kind, int nx, int ny, int nz, const double* kappa, double ba, double bph, const double* c,
                     double omega, double* S, hipStream_t);
void launch_stencil_mv(const double* S, int nx, int ny, int nz, int tr, const double* x, double* y, hipStream_t);
void launch_assemble27(int nx, int ny, int nz, const double* c, double omega, double* S, hipStream_t);
void launch_stencil27_mv(const double* S, int nx, int ny, int nz, int tr, const double* x, double* y, hipStream_t);
void launch_grad_kappa(int nx, int ny, int nz, const double* kappa, const double* u, const double* lam, double* g,
                       hipStream_t);
void launch_to_horder(const double* n, double* h, const int32_t* perm, int B, int64_t N, hipStream_t);
void launch_from_horder(const double* h, double* n, const int32_t* perm, int B, int64_t N, hipStream_t);
void launch_dots(const double* const* a, const double* const* b, int nd, int64_t n, double* part, double* out,
                 hipStream_t);
void launch_axpby(int64_t n, double a, const double* x, double b, double* y, hipStream_t);
void launch_multi_dot(int64_t n, int nv, const double* V, int64_t ldv, const double* w, double* part, double* out,
                      hipStream_t);
void launch_multi_axpy(int64_t n, int nv, const double* V, int64_t ldv, const double* h, double* w, double sign,
                       hipStream_t);
void launch_lincomb(int64_t n, int nv, const double* V, int64_t ldv, const double* c, double beta, double* y,
                    hipStream_t);
void launch_check(const double* x, int64_t n, int positive, int32_t* flag, hipStream_t);

// One stored or working H-matrix of a plane.  A working instance has the
// capacity layout (every low-rank leaf holds `cap` columns at the leaf's
// fixed offset); once it is final it is packed: exact ranks, leading
// dimensions padded to a multiple of 4 elements, per-leaf offsets in a
// device table.  Capacity buffers are recycled through a pool.
struct Instance {
  void* base = nullptr;      // leaf data (capacity or packed layout)
  int32_t* rank = nullptr;   // device: one rank per leaf
  int64_t* off = nullptr;    // device: per-leaf element offsets (packed); null = capacity layout
  void* buf = nullptr;       // allocation holding data, ranks (and offsets)
  bool live = false;
  bool packed = false;
  double packed_bytes = 0;   // packed leaf data in bytes
};

// Work buffers of a Krylov solve: kv_len vectors of N doubles, dot-product
// partials, result slots, two device tables of vector pointers and a host
// landing buffer for the results.
constexpr int KRYLOV_PART = 64 * 1024;  // dot partials (>= 61 dots x 1024 blocks)
constexpr int KRYLOV_RES = 64;          // result slots (>= GMRES(60)'s 61 coefficients)
struct KrylovBuffers {
  double* kv = nullptr;
  size_t kv_len = 0;
  double* part = nullptr;
  double* dres = nullptr;
  const double** dots_a = nullptr;
  const double** dots_b = nullptr;
  double* hres = nullptr;
};

struct Coupling {            // coupling of a plane to its previous (A) or next (C) plane
  int kind = 0;              // 0 absent, 1 diagonal (level 0), 2 H-matrix instance
  int inst = -1;
  const double* diag = nullptr;  // H-order plane vector
};

struct Level {
  std::vector<int> P, E, K;
  std::map<int, int> dinv;   // eliminated plane -> instance
  std::map<int, Coupling> A, C;
};

struct PhaseJobs {           // device job array of one apply phase
  MvJob* d = nullptr;
  std::vector<MvJob> h;      // host copy (algorithmic byte count)
  int n = 0;
  int32_t* terms = nullptr;  // non-empty H-matrix terms (2 * job + term)
  int nterms = 0;
  int trans = 0;
  int ri = -1;               // coefficient-kernel schedule: 0 one leaf round per lane
                             // group, 1 four; -1 by the phase size (set by tune_apply)
};

// One problem of a handle.  All problems of a handle share the plane shape
// (nx, ny) and the number of planes nz, hence the geometry, the programs and
// the cyclic-reduction structure: their levels run in lockstep and every
// batched launch covers all of them.
struct Prob {
  int kind = 0;
  double beta_amp = 0, beta_phase = 0, omega = 0;
  double* S = nullptr;       // nst() * N assembled stencil
  double* kappa = nullptr;   // node-grid copy (Poisson / convection-diffusion)
  double *zA = nullptr, *zC = nullptr;  // H-ordered level-0 z-couplings
  std::vector<Level> levels;
  int top_plane = -1, top_inst = -1;
  std::vector<int> plane_inst;          // current D / Dinv instance of each plane
  std::vector<PhaseJobs> ph_apply, ph_applyT;  // this problem alone (Krylov)
};

struct Handle {
  // shape shared by the problems
  int nx = 0, ny = 0, nz = 0, B = 0;
  int64_t N = 0;               // unknowns of one problem
  acr_options opt{};
  bool fp32 = false;  // FP32 factors during setup (ACR_MIXED_FP32 and ACR_MIXED_BF16)
  bool fem27 = false; // 27-point operator: 9-point plane couplings held as H-matrices from level 0
  int nst() const { return fem27 ? 27 : 7; }  // stencil rows per unknown
  bool bf16 = false;  // ACR_MIXED_BF16: piece products on BF16 matrix cores (FP32 factors)
  std::vector<double> level_secs;  // setup wall time per CR level (last build)
  std::vector<Prob> probs;
  // allocator
  std::vector<std::pair<void*, size_t>> owned;
  size_t bytes_alloc = 0;
  void* dmalloc(size_t bytes);
  void dfree(void* p);
  template <typename X> X* dnew(size_t n) { return (X*)dmalloc(n * sizeof(X)); }
  template <typename X> X* upload(const std::vector<X>& v) {
    if (v.empty()) return nullptr;
    X* p = dnew<X>(v.size());
    HIPCHK(hipMemcpy(p, v.data(), v.size() * sizeof(X), hipMemcpyHostToDevice));
    return p;
  }
  // geometry and device tables
  Geometry G;
  DLeaf* d_leaves = nullptr;
  int32_t* d_perm = nullptr;
  int64_t* d_l0map = nullptr;
  int32_t *d_seg_lo = nullptr, *d_rows_ptr = nullptr, *d_rows_idx = nullptr, *d_cols_ptr = nullptr,
          *d_cols_idx = nullptr;
  int64_t* d_soff = nullptr;
  int32_t *d_lr_n = nullptr, *d_lr_t = nullptr;  // low-rank leaves by lane class of n (of m)
  int32_t cls_n[6] = {0}, cls_t[6] = {0};
  int32_t cw_n[2][6] = {{0}}, cw_t[2][6] = {{0}};  // wavefront offsets for 1 and 4 rounds
  int32_t w4_n = 1, w4_t = 1;                       // wavefronts per leaf of the longest class
  int64_t sstride = 0;
  // instances
  std::vector<Instance> inst;
  void** d_inst_base = nullptr;
  int32_t** d_inst_rank = nullptr;
  int64_t** d_inst_off = nullptr;
  std::vector<void*> cap_pool;          // free capacity-layout buffers
  std::vector<int> pack_order;          // storage order of the leaves in packed instances
  size_t bytes_peak = 0;
  int inst_table_cap = 0;
  bool table_dirty = true;
  std::vector<int> free_inst;
  int new_instance(hipStream_t s);
  void release_instance(int id);
  void pack_instances(const std::vector<int>& ids, hipStream_t s);
  void sync_tables();
  // programs
  std::map<std::string, Program> prog;
  Program& get_program(const std::string& key);
  void upload_program(Program& p);
  // A lane runs one H-arithmetic program at a time: a main stream (lane 0:
  // the caller's), a second stream for the targets of a step that do not
  // need its first phase, the accumulation scratch (one region of
  // scratch_slots slots per stream), the dense accumulators of two-phase
  // steps and the role tables.  Lane 1 runs a level's new couplings while
  // lane 0 goes on with the Schur updates and the next level's inverses.
  struct Lane {
    hipStream_t s = nullptr, s2 = nullptr;
    hipEvent_t fork = nullptr, join = nullptr;
    void* scratch = nullptr;
    void* dbuf = nullptr;      // dense accumulators (a chunk of batch items)
    size_t dbuf_bytes = 0;
    int32_t* d_roles = nullptr;
    int roles_cap = 0;
    const double** d_vecs = nullptr;
    int vecs_cap = 0;
  };
  Lane lanes[2];
  int64_t scratch_stride = 0;
  int scratch_slots = 0;
  int kc = 64;                 // round width of the accumulation kernel in use
  void ensure_lane(Lane& ln, hipStream_t main);
  hipEvent_t ev_products = nullptr;  // a level's first products done (lane 1 may start)
  int32_t* d_flags = nullptr;
  unsigned long long* d_prof = nullptr;  // optional kernel cycle counters (ACR_PROFILE=1)
  double* d_flops = nullptr;             // optional algorithmic flop counters (ACR_KERNEL_TIMING=1):
                                         // [kernel][FlopClass], the truncating kernel first
  double leaf_inverse_flops = 0.0;       // 2 m^3 per inverted dense diagonal leaf (host count)
  bool timing = false;
  std::vector<hipEvent_t> ev_pool;
  size_t ev_used = 0;
  struct LaunchTag {
    const char* prog;
    int level, step, nbatch, nt, max_m;
    const char* kernel;  // "dense": accumulate-only kernel, "": truncating kernel
  };
  std::vector<LaunchTag> ev_tag;  // one per timed launch (ACR_KERNEL_TIMING=1)
  int cur_level = -1;
  int accum_launches = 0, dense_launches = 0;
  // apply workspace (all problems, plane vectors concatenated by problem)
  double *g = nullptr, *w = nullptr, *z = nullptr, *coef = nullptr;
  int max_jobs = 0;
  std::vector<PhaseJobs> ph_apply, ph_applyT;  // all problems at once
  // apply images of the H-matrices the apply phases use (the segment
  // kernel's input): data and weight-index arenas, per-(image, segment)
  // tables (the row images of all images, then their column images for the
  // transposed phases), image of each instance id (-1: none)
  void* img_data = nullptr;
  int32_t* img_widx = nullptr;
  SegImg* d_img_seg = nullptr;
  int32_t* d_img_of_inst = nullptr;
  int64_t img_tab_half = 0;  // entries of the row-image tables
  double img_bytes = 0.0;
  void build_apply_image(hipStream_t s);
  // krylov workspace (allocated at the first solve; hres is pinned host memory)
  KrylovBuffers kbuf;
  // statistics
  acr_stats_t st{};

  ~Handle();
  void setup(const acr_problem* ps, int count, hipStream_t s);
  // operators, geometry and segment tables, level-0 z-couplings
  void prepare(const acr_problem* ps, int count, hipStream_t s);
  // release setup memory, apply jobs and their tuning, statistics
  void finish(hipStream_t s, std::chrono::steady_clock::time_point t_start);
  void upload_leaf_tables();
  // factors given on the host (acr_import_factors) instead of the setup
  void import_factors(const acr_problem* p, const acr_factor_blob* blob, hipStream_t s);
  int new_packed_instance(const std::vector<int32_t>& rank, const double* data, hipStream_t s);
  void ensure_pack_order();
  void build_factors(hipStream_t s, const std::vector<int>& caps);
  void free_factors();
  void run_program(Program& P, int nbatch, int nroles, const std::vector<int32_t>& roles, int nvroles,
                   const std::vector<const double*>& vecs, Lane& ln);
  template <typename T>
  void run_accum_step(Program& P, const Step& st, int nbatch, int nroles, int nvroles, Lane& ln);
  void build_apply_jobs();
  void launch_phase(const PhaseJobs& pj, int ri, hipStream_t s);
  void tune_apply(hipStream_t s);
  int tuned_phases = 0;
  // z_p = M_p^{-1} r_p (or M_p^{-T}) for every problem (prob < 0) or one
  void apply(const std::vector<const double*>& r, const std::vector<double*>& z, bool transpose, int prob,
             hipStream_t s);
  void matvec(int prob, const double* x, double* y, bool transpose, hipStream_t s);
  void compute_stats();
  double instance_bytes(const std::vector<int32_t>& ranks) const;
};

}  // namespace acr
struct acr_handle;
namespace acr {
// krylov_solve over every problem of a handle (wb = nullptr: the handle's
// own buffers), argument checks, the work-vector count of a method, and the
// thread-local error text of the ABI
acr_status solve_problems(acr_handle* h, int32_t method, int32_t restart, int32_t transpose, double rtol,
                          int32_t maxit, const double* b, double* x, acr_solve_info* info, void* stream,
                          KrylovBuffers* wb);
acr_status check_solve_args(const acr_handle* h, int32_t method, int32_t restart, double rtol, int32_t maxit,
                            const double* b, const double* x, const acr_solve_info* info);
int krylov_vectors(int32_t method, int32_t restart);
acr_status set_last_error(acr_status s, const std::string& msg);

// host-side validation of acr_import_factors' blob (throws ACR_E_INVALID)
void check_factor_blob(const acr_problem* p, const acr_options* o, const acr_factor_blob* blob);

}  // namespace acr

// A handle holds one or more groups of problems; the problems of a group
// share a plane shape.  Vectors passed through the ABI concatenate the
// problems in the order they were given.
struct acr_handle {
  std::vector<std::unique_ptr<acr::Handle>> groups;
  std::vector<std::pair<int, int>> where;  // problem -> (group, index in group)
  std::vector<int64_t> off, grid_off;      // vector / node-grid offsets per problem
  int64_t total = 0, grid_total = 0;
  // several groups: one stream per group (default priority), so that the
  // groups' setups and applies run concurrently, and the events that fork
  // from and join to the caller's stream
  std::vector<hipStream_t> gstream;
  std::vector<hipEvent_t> gdone;
  hipEvent_t fork = nullptr;
  ~acr_handle() {
    groups.clear();  // the groups' memory first (their work is complete)
    for (hipStream_t s : gstream) (void)hipStreamDestroy(s);
    for (hipEvent_t e : gdone) (void)hipEventDestroy(e);
    if (fork) (void)hipEventDestroy(fork);
  }
};
