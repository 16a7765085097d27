// Internal declarations of the bie2d HIP library (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <functional>
#include <string>
#include <vector>

#include "bie2d.h"

namespace bie {

constexpr double kPi = 3.14159265358979323846;
constexpr int kBlock = 256;  // threads per workgroup for every kernel (4 wave64)
constexpr int kSub = 4;                // workgroups per chunk in the segmented update kernels
constexpr int kChunk = kSub * kBlock;  // entries per chunk of a segmented vector

void set_error(const std::string &msg);
// Makes `dev` the current device for the lifetime of the guard (restoring the previous one).
struct DeviceGuard {
  int prev = -1;
  explicit DeviceGuard(int dev) {
    int cur = -1;
    if (hipGetDevice(&cur) == hipSuccess && cur != dev && hipSetDevice(dev) == hipSuccess)
      prev = cur;
  }
  ~DeviceGuard() {
    if (prev >= 0) (void)hipSetDevice(prev);
  }
};

int check_opts(const bie_opts &o);       // BIE_EINVAL (message set) for invalid options
int effective_order(const bie_opts &o, int kind);  // FMM order from fmm_eps or fmm_order

#define BIE_HIP_CHECK(call)                                                              \
  do {                                                                                   \
    hipError_t e_ = (call);                                                              \
    if (e_ != hipSuccess) {                                                              \
      ::bie::set_error(std::string(#call) + ": " + hipGetErrorString(e_));               \
      return BIE_EDEVICE;                                                                \
    }                                                                                    \
  } while (0)

#define BIE_TRY(call)                 \
  do {                                \
    int rc_ = (call);                 \
    if (rc_ != BIE_OK) return rc_;    \
  } while (0)

// Device buffer owned by a geometry (hipMalloc'd, grown on demand, freed on destroy).
struct DevBuf {
  void *ptr = nullptr;
  size_t bytes = 0;
  int reserve(size_t need);
  void release();
  template <class T>
  T *as() const { return static_cast<T *>(ptr); }
};

struct FmmPlan;  // far-field FMM state (fmm.hip)

// Independent systems stored back to back in flat vectors; chunks never straddle two systems.
struct Segments {
  int S = 0, C = 0;
  long long Ntot = 0;
  std::vector<long long> h_off;  // [S+1] host offsets
  DevBuf buf;
  long long *c0 = nullptr, *c1 = nullptr;  // [C] flat chunk ranges
  int *csys = nullptr, *sys_chunk = nullptr;  // [C] system of chunk, [S+1] chunks of a system
  // systems back to back, or at the given start offsets (gaps between systems are never read
  // by the segmented kernels)
  int build(const std::vector<long long> &lens, hipStream_t s,
            const std::vector<long long> *starts = nullptr);
};

// Number of device buffer (re)allocations so far: a cached HIP graph whose kernels point into
// library buffers is valid only while this has not changed since its capture.
unsigned long long buffer_epoch();

// Whether solves replay captured HIP graphs of their Arnoldi steps (bie_set_graphs).
bool graphs_enabled();

// Instantiated graphs of the Arnoldi steps j = 0, 1, ... of one solver configuration: each
// replays step j's operator apply and Gram-Schmidt kernels with the same buffers.
struct StepGraphs {
  std::string key;
  unsigned long long epoch = 0;
  std::vector<hipGraphExec_t> exec;
  void clear();
};

// Krylov workspace and pinned staging of a solver owner (a geometry or a batch).
struct SolverMem {
  DevBuf big, small;
  double *pinned = nullptr;      // mapped, coherent host memory
  double *pinned_dev = nullptr;  // its device address (kernels write Hessenberg columns there)
  size_t pinned_bytes = 0;
  unsigned long long seq = 0;  // last Arnoldi step number handed out (column flags)
  StepGraphs graphs[2];        // by apply precision (BIE_FP64, BIE_MIXED)
  hipStream_t cap = nullptr;   // private stream the steps are captured on (capture is not
                               // possible on the legacy null stream); replays use the caller's
  long long graph_replays = 0, graph_captures = 0;
  int ensure_pinned(size_t bytes);
  void release();
};

// A set of systems with one batched apply: out = A in (flat layout of seg).
// BIE_AUTO: the FMM for geometries with more than this many nodes, else direct summation.
constexpr long long kAutoFmmNodes = 32768;
inline bool method_is_fmm(int method, long long M) {
  return method == BIE_FMM || (method == BIE_AUTO && M > kAutoFmmNodes);
}
// Relative error (2-norm) that the relaxed mixed strategy assumes for a BIE_MIXED apply.
double mixed_apply_error(const bie_geom *g, int kind, int method, int order);

// Apply precision value meaning "per group": group g's systems use float32 where
// SysSet::group_f32[g] is set, float64 elsewhere.
constexpr int kPrecPerGroup = -1;
// Most groups (batch items) whose applies can take per-group precisions; a set with more groups
// is treated as one group.
constexpr int kMaxPrecGroups = 1024;

struct SysSet {
  Segments *seg = nullptr;
  SolverMem *mem = nullptr;
  long long pairs_per_apply = 0;
  std::vector<char> active;  // per system; set by the solver before each apply (empty = all)
  // groups of systems whose applies are independent of each other's (batch items: system
  // ranges group_ptr[g] .. group_ptr[g+1]-1); empty = all systems form one group. A relaxed
  // mixed solve chooses each step's precision per group, so a group's iterates do not depend on
  // the other groups.
  std::vector<int> group_ptr;
  std::vector<char> group_f32;  // per group, read by apply(kPrecPerGroup, ...)
  // per group (or one value for all), the relative error of its BIE_MIXED apply (empty: 1e-6)
  std::vector<double> group_eta;
  std::function<int(int precision, const double *in, double *out, hipStream_t s)> apply;
  // identity of the apply's arguments for graph capture (empty: the steps are never captured,
  // e.g. batches, whose applies depend on the active flags)
  std::string graph_key;
};

// Resolution warning thresholds: a node closer than kResolveGap node spacings of another body
// (trapezoidal error about exp(-2 pi kResolveGap) ~ 6e-9 there), or a trapezoidal turning
// number off 2 pi by more than kResolveTurn (relative).
constexpr double kResolveGap = 3.0;
constexpr double kResolveTurn = 1e-8;

// Checks of curve samples (host [6][M]: x, y, x', y', x'', y'') and optional read-off points
// (host [N][2]) before a geometry is built (checks.cpp): BIE_EINVAL (msg set) for non-finite
// samples, a clockwise body or a read-off point outside its body's node polygon; else
// BIE_ERESOLVE (msg set) for a turning number off 2 pi by more than kResolveTurn or a node
// closer than kResolveGap node spacings of another body; else BIE_OK.
int check_curves(int N, const int32_t *nodes_per_body, const double *curve,
                 const double *interior, std::string &msg);

}  // namespace bie

struct bie_ctx;

struct bie_geom {
  bie_ctx *ctx = nullptr;  // owning context (NULL: created by bie_geom_create)
  int N = 0, M = 0, device = 0;
  // process-unique id given at creation: caches keyed on a geometry (batched-apply plans) use
  // it, never the address, which a later geometry may reuse
  unsigned long long gen = 0;
  std::vector<int> h_body_ptr;  // host copy [N+1]
  int max_nb = 0;               // nodes of the largest body
  int max_nodes = 0;            // largest n_b
  // device arrays (one arena)
  bie::DevBuf arena;
  int *body_ptr = nullptr, *body_of = nullptr;                  // [N+1], [M]
  double *x = nullptr, *y = nullptr, *nx = nullptr, *ny = nullptr;  // [M]
  double *w = nullptr, *kappa = nullptr, *px = nullptr, *py = nullptr;
  double *len = nullptr, *xc = nullptr, *yc = nullptr, *W = nullptr;  // [N]
  double *pint = nullptr;   // [N][2] interior read-off points
  double *area = nullptr;   // [N] signed area (validation)
  double *dl_scale = nullptr;  // [1] length scale R of the completed double layers
  double2 *xy = nullptr;    // [M] float64 source coordinates
  float2 *xr = nullptr;     // [M] float32 coordinates relative to the body centroid
  // source-body splits of the far-field sweep
  int nsplit = 1;
  int *split_body = nullptr;  // [nsplit+1] device
  std::vector<int> h_split_body;
  long long far_pairs = 0;    // pairs with distinct bodies: M^2 - sum n_b^2
  // workspaces
  bie::DevBuf ws_apply;   // strengths + far-field partials
  bie::SolverMem sm;      // Krylov basis, vectors, reductions, pinned staging
  hipEvent_t in_ev = nullptr;  // a solve's input has reached the pinned staging area
  bie::Segments seg;      // chunk list of the current nrhs systems
  int seg_nrhs = -1;
  long long seg_len = -1;
  bie::DevBuf ws_out;     // solver outputs (densities, rhs) for solve entry points
  bie::DevBuf ws_read;    // read-off partial sums [split][rhs][body][comp]
  bie::DevBuf ws_scale;   // L2-scaled solves: scaled rhs and the unscaled apply input
  bie::FmmPlan *fmm = nullptr;
  int fmm_order = 40;  // expansion order of the float64 FMM apply (set from bie_opts)
  int fmm_leaf = 64;   // maximum nodes per leaf box
  int fmm_leaf_mixed = 0;  // leaf size of the mixed-precision applies (0: fmm_leaf)
  // block preconditioner per kind (precond.hip): inverted coarse blocks [N][BJ][BJ] (float32,
  // column-major, inv); per body the coarse node count (meta)
  struct Precond {
    bie::DevBuf inv, meta;
    bool ready = false;
    int BJ = 0;
    int *ncoarse = nullptr;
    long long macs = 0;  // multiply-adds per apply and right-hand side
    size_t lds = 0;      // dynamic LDS of the apply
  } pc[2];
};

namespace bie {

// ---- kernels.hip: operator pieces -------------------------------------------------------
// kind: 0 = Laplace (len = M per rhs), 1 = Stokes (len = 2M per rhs); 2 and 3 are the
// completed double layers of the capacitance and resistance problems (Laplace, Stokes)
int apply_operator(bie_geom *g, int kind, int precision, int method, int with_L, double alpha,
                   int nrhs, const double *mu, double *out, hipStream_t s);
// the same with a caller-provided workspace of ws_bytes >= apply_workspace_bytes(...) bytes
// (kinds 0 and 1; method BIE_DIRECT or BIE_FMM)
int apply_operator_ws(bie_geom *g, int kind, int precision, int method, int with_L,
                      double alpha, int nrhs, const double *mu, double *out, void *ws,
                      size_t ws_bytes, hipStream_t s);
size_t apply_workspace_bytes(const bie_geom *g, int kind, int method, int nrhs);
int incident_density(bie_geom *g, int kind, int nrhs, const double *data, double *dens,
                     hipStream_t s);
// out = D in, or D^-1 in with inverse, D = diag(sqrt(w)) per node and component ([nrhs][M comps])
int scale_sqrtw(bie_geom *g, int comps, int nrhs, int inverse, const double *in, double *out,
                hipStream_t s);
// method BIE_FMM (or BIE_AUTO above 32768 nodes): treecode over the float64 FMM tree of the
// geometry's order and leaf size; else the direct sum over all nodes
int read_off(bie_geom *g, int kind, int nrhs, const double *dens, double *res, hipStream_t s,
             int method = BIE_DIRECT);
int eval_points(bie_geom *g, int kind, int nrhs, const double *dens, int npts, const double *pts,
                bool rigid, double *res, hipStream_t st, int method = BIE_DIRECT);
int geometry_build(bie_geom *g, const double *curve, const double *interior, hipStream_t s);

// ---- dirichlet.hip: capacitance and resistance problems (completed double layers) --------
// kind 2 (Laplace) and 3 (Stokes) of apply_operator / solve_system
int dl_apply(bie_geom *g, int stokes, int with_C, double alpha, int nrhs, const double *mu,
             double *out, hipStream_t s);
int dl_solve(bie_geom *g, int stokes, int nrhs, const double *data, double *res, double *u_inf,
             double *mu_out, const bie_opts &opts, bie_info *info, hipStream_t s);

// ---- blas.hip: segmented float64 vector kernels used by GMRES -------------------------------
int seg_dots(const Segments &sg, int nvec, const double *V, long long vstride, const double *w,
             double *h, long long hs, double *scratch, hipStream_t s);
int seg_combination(const Segments &sg, int nvec, const double *V, long long vstride,
                    const double *h, long long hs, double *w, double sign, hipStream_t s);
int seg_nrm2(const Segments &sg, const double *w, double *out, double *scratch, hipStream_t s);
int seg_scale_to(const Segments &sg, const double *w, const double *den, double *v, hipStream_t s);
// w -= V h2 (nvec vectors), then nrm = ||w|| per system, vnext = w / ||w||,
// h2[s][0..nvec-1] += h1[s][...] and h2[s][nvec] = nrm[s] (the new Hessenberg column, also written to
// col_out [S][hs] when not NULL, and then seq to flag[s] when flag is not NULL: both in mapped
// host memory); scratch holds C * 4 partials
int seg_combination_column(const Segments &sg, int nvec, const double *V, long long vstride,
                           const double *h1, double *h2, long long hs, double *w, double *nrm,
                           double *vnext, double *col_out, unsigned long long *flag,
                           const unsigned long long *seq_base, unsigned long long seq_off,
                           double *scratch, hipStream_t s);
// the value stored in a column's flag word for step number seq (a NaN bit pattern with seq in
// its payload, which the doubles staged through the same pinned buffer never take)
__host__ __device__ inline unsigned long long column_tag(unsigned long long seq) {
  return 0x7FF5A00000000000ULL | (seq & 0x00000FFFFFFFFFFFULL);
}
int vec_axpby(long long total, double a, const double *x, double b, double *y, hipStream_t s);
// DCGS2 Arnoldi step pieces (blas.hip): raw[s][0 .. 2nv+1] = (V_l.U, V_l.Z)_l, U.U, U.Z (Z may be
// NULL); the per-system column and coefficients; the update writing V_j and the next candidate
int dcgs_dots(const Segments &sg, int nv, const double *V, long long vstride, const double *U,
              const double *Z, double *raw, long long rstride, double *scratch, hipStream_t s);
int dcgs_small(int S, int j, bool finalize, const double *raw, long long rstride, double *G,
               double *Hd, long long ldh, long long hstride, double *sc, double *cc, double *inu,
               long long hs, double *col_out, unsigned long long *flag,
               const unsigned long long *seq_base, unsigned long long seq_off, hipStream_t s);
int dcgs_update(const Segments &sg, int j, const double *V, long long vstride, const double *sc,
                const double *cc, const double *inu, long long hs, double *U, const double *Z,
                double *Vj, hipStream_t s);
int seg_add_h(int S, const double *h1, double *h2, int cnt, long long hs, hipStream_t s);

// ---- gmres.cpp ----------------------------------------------------------------------------
int solve_system(bie_geom *g, int kind, const bie_opts &o, int nrhs, const double *f,
                 double *x, bie_info *info, hipStream_t s);
int solve_systems(SysSet &ss, const bie_opts &o, const double *f, double *x,
                  std::vector<double> &relres, bie_info *info, hipStream_t s);
int gmres_cycle(SysSet &ss, int precision, const double *r, double *d,
                const std::vector<double> &tol, int m, int &iters, int &applies, hipStream_t s);

// ---- fmm.hip ------------------------------------------------------------------------------
// mu [nrhs][len] in; s64 [nrhs][len] out (the strengths w mu, for the epilogue)
// The per-node terms a Laplace FMM apply can add in its evaluation kernel instead of a separate
// epilogue: out = alpha (1/2 mu - s kappa / (4 pi) [+ with_L: the sum of s over the node's body]
// + near + far), [R][M] in node order.
struct FmmFinish {
  const double *mu = nullptr;
  double *out = nullptr;
  double alpha = 1.0;
  int with_L = 0;
};
int fmm_far_field(bie_geom *g, int kind, int precision, int nrhs, const double *mu, double *s64,
                  double *partial, hipStream_t s, int order, int leaf,
                  const FmmFinish *finish = nullptr);
void fmm_destroy(FmmPlan *p);
// single-layer potentials at points by the treecode over the float64 FMM tree (see kernels.hip
// eval_points for the layouts)
int fmm_eval_points(bie_geom *g, int kind, int nrhs, const double *dens, int npts,
                    const double *pts, bool rigid, double *res, hipStream_t s);
// device bytes of g's FMM state (tree and work area) for one solve kind, precision, order and
// leaf size: the actual size where the tree exists, else an upper estimate
long long fmm_state_bytes(const bie_geom *g, int kind, int precision, int order, int leaf);
// frees g's tree for this precision, order and leaf size (if any)
void fmm_drop_tree(bie_geom *g, int precision, int order, int leaf);

// ---- autotune.cpp: FMM leaf size per shape class ------------------------------------------
// Sets g->fmm_leaf / g->fmm_leaf_mixed for a solve of `kind` at `precision` with nrhs right-hand
// sides: from the cache of g's context (or the process cache) for g's shape class, else by
// timing applies on g over the candidate leaf sizes and storing the fastest.
int autotune_leaf(bie_geom *g, int kind, int precision, int nrhs, hipStream_t s);
// Sets g's FMM leaf sizes for a solve with opts o: o.fmm_leaf > 0 for both precisions; 0 = the
// autotuner's (tune true) or 64 (tune false: callers that must not pause to time applies).
int resolve_leaf(bie_geom *g, int kind, const bie_opts &o, int nrhs, bool tune, hipStream_t s);
// ---- precond.hip: block right preconditioner of the Laplace and Stokes operators ------------
// Block preconditioner of kind 0 (Laplace) or 1 (Stokes): built once per geometry and kind
// (BIE_EINVAL for a body it cannot coarsen); apply out = P in, [nrhs][M] resp. [nrhs][2M].
int pc_build(bie_geom *g, int kind, hipStream_t s);
int pc_apply(bie_geom *g, int kind, int nrhs, const double *in, double *out, hipStream_t s);
// Batched apply over geometries whose preconditioners are built: per item its geometry's data,
// the item's offset in the flat vector and its first workgroup (prefix of N nrhs).
struct PcBatchItem {
  const int *body_ptr, *ncoarse;
  const float *inv;
  long long off;
  int BJ, N, M, kind, nrhs, block0;
};
int pc_batch_items(const std::vector<bie_geom *> &geoms, const std::vector<int> &kinds,
                   const std::vector<int> &nrhs, const std::vector<long long> &offs,
                   std::vector<PcBatchItem> &items, size_t &lds, long long &blocks,
                   long long &macs);
int pc_apply_batch(int nitems, const PcBatchItem *d_items, size_t lds, long long blocks,
                   long long macs, const double *in, double *out, hipStream_t s);

// Expansion length (terms, a multiple of 8) the FMM apply of `precision` uses for an order.
int fmm_length(int order, int precision);

// ---- multi.hip: one apply for many geometries ------------------------------------------------
struct MultiItem {
  bie_geom *g;
  int kind, nrhs;
  long long io;  // start of the item's rhs block in the flat vectors (64-byte aligned)
  bool fmm;      // applied by the single-geometry FMM path
  int fmm_order = 40, fmm_leaf = 64;  // its expansion order and leaf population (FMM items)
};
struct MultiPlan;
// item_f32 (nullptr: every item uses precision): per item, 1 = float32 far field (BIE_MIXED),
// 0 = float64; at most kMaxPrecGroups items.
int multi_apply(MultiPlan *&plan, const std::vector<MultiItem> &items,
                const std::vector<char> &active, int precision, const double *in, double *out,
                long long Ntot, hipStream_t s, const std::vector<char> *item_f32 = nullptr);
void multi_destroy(MultiPlan *p);
inline long long align8(long long v) { return (v + 7) / 8 * 8; }

// ---- profile.cpp: optional per-class launch timing ------------------------------------------
// While a ProfSuspend lives, this thread records no profiling events (no event is created).
struct ProfSuspend {
  ProfSuspend();
  ~ProfSuspend();
};
struct ProfScope {
  int kclass;
  hipStream_t s;
  long long pairs;
  bool on;
  ProfScope(int kclass, hipStream_t s, long long pairs);
  ~ProfScope();
};

}  // namespace bie
