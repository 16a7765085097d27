// Internal declarations of the bie2d HIP library (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "bie2d.h"

namespace bie {

constexpr double kPi = 3.14159265358979323846;
constexpr int kBlock = 256;  // threads per workgroup for every kernel (4 wave64)

void set_error(const std::string &msg);

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

}  // namespace bie

struct bie_geom {
  int N = 0, M = 0, device = 0;
  std::vector<int> h_body_ptr;  // host copy [N+1]
  int max_nodes = 0;            // largest n_b
  // device arrays (one arena)
  bie::DevBuf arena;
  int *body_ptr = nullptr, *body_of = nullptr;                  // [N+1], [M]
  double *x = nullptr, *y = nullptr, *nx = nullptr, *ny = nullptr;  // [M]
  double *w = nullptr, *kappa = nullptr, *px = nullptr, *py = nullptr;
  double *len = nullptr, *xc = nullptr, *yc = nullptr, *W = nullptr;  // [N]
  double *pint = nullptr;   // [N][2] interior read-off points
  double *area = nullptr;   // [N] signed area (validation)
  double2 *xy = nullptr;    // [M] float64 source coordinates
  float2 *xr = nullptr;     // [M] float32 coordinates relative to the body centroid
  // source-body splits of the far-field sweep
  int nsplit = 1;
  int *split_body = nullptr;  // [nsplit+1] device
  std::vector<int> h_split_body;
  long long far_pairs = 0;    // pairs with distinct bodies: M^2 - sum n_b^2
  // workspaces
  bie::DevBuf ws_apply;   // strengths + far-field partials
  bie::DevBuf ws_solve;   // Krylov basis and vectors
  bie::DevBuf ws_small;   // reductions, Hessenberg columns
  bie::DevBuf ws_out;     // solver outputs (densities, rhs) for solve entry points
  double *h_pinned = nullptr;  // pinned host staging for small reads
  size_t h_pinned_bytes = 0;
  bie::FmmPlan *fmm = nullptr;
  int fmm_order = 40;  // expansion order of the float64 FMM apply (set from bie_opts)
  int fmm_leaf = 64;   // maximum nodes per leaf box
};

namespace bie {

// ---- kernels.hip: operator pieces -------------------------------------------------------
// kind: 0 = Laplace (len = M per rhs), 1 = Stokes (len = 2M per rhs)
int apply_operator(bie_geom *g, int kind, int precision, int method, int with_L, double alpha,
                   int nrhs, const double *mu, double *out, hipStream_t s);
int incident_density(bie_geom *g, int kind, int nrhs, const double *data, double *dens,
                     hipStream_t s);
int read_off(bie_geom *g, int kind, int nrhs, const double *dens, double *res, hipStream_t s);
int geometry_build(bie_geom *g, const double *curve, const double *interior, hipStream_t s);

// ---- blas.hip: float64 vector kernels used by GMRES ------------------------------------------
// Batched over nrhs vectors of length n with the given strides (in doubles).
int vec_dots(int nrhs, int n, int nvec, const double *V, long long vstride_rhs, long long vstride_vec,
             const double *w, long long wstride, double *h, long long hstride, double *scratch,
             hipStream_t s);
int vec_sub_combination(int nrhs, int n, int nvec, const double *V, long long vstride_rhs,
                        long long vstride_vec, const double *h, long long hstride, double *w,
                        long long wstride, double sign, hipStream_t s);
int vec_nrm2(int nrhs, int n, const double *w, long long wstride, double *out, double *scratch,
             hipStream_t s);
int vec_scale_to(int nrhs, int n, const double *w, long long wstride, const double *den,
                 double *v, long long vstride, hipStream_t s);
int vec_axpby(int nrhs, int n, double a, const double *x, double b, double *y, hipStream_t s);
int vec_add_h(int nrhs, int n, const double *h1, double *h2, int cnt, long long hstride,
              hipStream_t s);

// ---- gmres.cpp ----------------------------------------------------------------------------
int solve_system(bie_geom *g, int kind, const bie_opts &o, int nrhs, const double *f,
                 double *x, bie_info *info, hipStream_t s);

// ---- fmm.hip ------------------------------------------------------------------------------
int fmm_far_field(bie_geom *g, int kind, int precision, int nrhs, const double *s64,
                  double *partial, hipStream_t s, int order, int leaf);
void fmm_destroy(FmmPlan *p);
int fmm_current_order();

int ensure_pinned(bie_geom *g, size_t bytes);

// ---- profile.cpp: optional per-class launch timing ------------------------------------------
struct ProfScope {
  int kclass;
  hipStream_t s;
  long long pairs;
  bool on;
  ProfScope(int kclass, hipStream_t s, long long pairs);
  ~ProfScope();
};

}  // namespace bie
