// C ABI entry points of libbie2d (declared in include/bie2d.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "internal.h"

namespace bie {

static thread_local std::string g_last_error = "no error";

void set_error(const std::string &msg) { g_last_error = msg; }

int DevBuf::reserve(size_t need) {
  if (need <= bytes) return BIE_OK;
  if (ptr) {
    hipError_t e = hipDeviceSynchronize();
    (void)e;
    hipFree(ptr);
    ptr = nullptr;
    bytes = 0;
  }
  size_t want = need + need / 8 + 4096;
  if (hipMalloc(&ptr, want) != hipSuccess) {
    ptr = nullptr;
    set_error("device allocation of " + std::to_string(want) + " bytes failed");
    return BIE_ENOMEM;
  }
  bytes = want;
  return BIE_OK;
}

void DevBuf::release() {
  if (ptr) hipFree(ptr);
  ptr = nullptr;
  bytes = 0;
}

// Source-body ranges of the far-field sweep: contiguous groups of bodies with about equal node
// counts, enough of them that the grid holds >= ~32k wavefronts (256 CUs x 4 SIMDs x several).
static void plan_splits(bie_geom *g) {
  const long long target_waves = 32768;
  const long long tblocks = (g->M + kBlock - 1) / kBlock;
  long long want = (target_waves + 4 * tblocks - 1) / (4 * tblocks);
  want = std::max(1LL, std::min<long long>(want, std::min(g->N, 64)));
  const int S = (int)want;
  g->h_split_body.assign(1, 0);
  const long long M = g->M;
  for (int s = 1; s < S; ++s) {
    const long long cut = M * s / S;
    int b = g->h_split_body.back();
    while (b < g->N && g->h_body_ptr[b + 1] <= cut) ++b;
    if (b > g->h_split_body.back() && b < g->N) g->h_split_body.push_back(b);
  }
  g->h_split_body.push_back(g->N);
  g->nsplit = (int)g->h_split_body.size() - 1;
}

static hipStream_t as_stream(void *s) { return reinterpret_cast<hipStream_t>(s); }

static int check_geom(const bie_geom *g) {
  if (!g) {
    set_error("NULL geometry");
    return BIE_EINVAL;
  }
  return BIE_OK;
}

static void fill_defaults(bie_opts *o) {
  o->precision = BIE_FP64;
  o->method = BIE_DIRECT;
  o->tol = 1e-12;
  o->restart = 100;
  o->max_iter = 500;
  o->inner_tol = 1e-6;
  o->max_refine = 10;
  o->fmm_order = 40;
  o->fmm_leaf = 64;
}

static int check_opts(const bie_opts &o) {
  if ((o.precision != BIE_FP64 && o.precision != BIE_MIXED) ||
      (o.method != BIE_DIRECT && o.method != BIE_FMM && o.method != BIE_AUTO) ||
      !(o.tol > 0.0) || o.restart < 1 ||
      o.max_iter < 1 || !(o.inner_tol > 0.0) || o.max_refine < 0 || o.fmm_order < 4 ||
      o.fmm_order > 64 || o.fmm_leaf < 1) {
    set_error("invalid bie_opts");
    return BIE_EINVAL;
  }
  return BIE_OK;
}

}  // namespace bie

using namespace bie;

extern "C" {

const char *bie_last_error(void) { return g_last_error.c_str(); }

int bie_default_opts(bie_opts *o) {
  if (!o) {
    set_error("NULL opts");
    return BIE_EINVAL;
  }
  fill_defaults(o);
  return BIE_OK;
}

int bie_geom_create(int nbodies, const int32_t *nodes_per_body, const double *curve,
                    const double *interior, void *stream, bie_geom **out) {
  if (!out || !nodes_per_body || !curve || nbodies < 1) {
    set_error("bie_geom_create: need nbodies >= 1 and non-NULL nodes_per_body, curve, out");
    return BIE_EINVAL;
  }
  *out = nullptr;
  long long M = 0;
  int maxn = 0;
  for (int b = 0; b < nbodies; ++b) {
    if (nodes_per_body[b] < 3) {
      set_error("bie_geom_create: body " + std::to_string(b) + " has fewer than 3 nodes");
      return BIE_EINVAL;
    }
    M += nodes_per_body[b];
    maxn = std::max(maxn, (int)nodes_per_body[b]);
  }
  if (M > (1LL << 28)) {
    set_error("bie_geom_create: more than 2^28 nodes");
    return BIE_EINVAL;
  }
  bie_geom *g = new (std::nothrow) bie_geom();
  if (!g) {
    set_error("host allocation failed");
    return BIE_ENOMEM;
  }
  g->N = nbodies;
  g->M = (int)M;
  g->max_nodes = maxn;
  hipGetDevice(&g->device);
  g->h_body_ptr.resize(nbodies + 1);
  g->h_body_ptr[0] = 0;
  for (int b = 0; b < nbodies; ++b) {
    g->h_body_ptr[b + 1] = g->h_body_ptr[b] + nodes_per_body[b];
    g->max_nb = std::max(g->max_nb, nodes_per_body[b]);
  }
  plan_splits(g);
  g->far_pairs = (long long)M * M;
  for (int b = 0; b < nbodies; ++b) g->far_pairs -= (long long)nodes_per_body[b] * nodes_per_body[b];
  const size_t Md = (size_t)M, Nd = (size_t)nbodies;
  // arena: doubles first (8 node arrays, xy (2M), 4 body arrays, pint (2N), area, the
  // double-layer length scale), then floats, ints
  const size_t nd = 8 * Md + 2 * Md + 4 * Nd + 2 * Nd + Nd + 1;
  const size_t bytes = nd * 8 + Md * 8 /*xr*/ + (Nd + 1 + Md + g->h_split_body.size()) * 4 + 256;
  int rc = g->arena.reserve(bytes);
  if (rc != BIE_OK) {
    delete g;
    return rc;
  }
  double *p = g->arena.as<double>();
  auto take = [&](size_t cnt) {
    double *q = p;
    p += cnt;
    return q;
  };
  g->x = take(Md);
  g->y = take(Md);
  g->nx = take(Md);
  g->ny = take(Md);
  g->w = take(Md);
  g->kappa = take(Md);
  g->px = take(Md);
  g->py = take(Md);
  g->xy = reinterpret_cast<double2 *>(take(2 * Md));
  g->len = take(Nd);
  g->xc = take(Nd);
  g->yc = take(Nd);
  g->W = take(Nd);
  g->pint = take(2 * Nd);
  g->area = take(Nd);
  g->dl_scale = take(1);
  g->xr = reinterpret_cast<float2 *>(p);
  int *ip = reinterpret_cast<int *>(g->xr + Md);
  g->body_ptr = ip;
  ip += Nd + 1;
  g->body_of = ip;
  ip += Md;
  g->split_body = ip;
  hipStream_t s = as_stream(stream);
  auto fail = [&](int code) {
    bie_geom_destroy(g);
    return code;
  };
  if (hipMemcpyAsync(g->body_ptr, g->h_body_ptr.data(), (Nd + 1) * 4, hipMemcpyHostToDevice, s) !=
          hipSuccess ||
      hipMemcpyAsync(g->split_body, g->h_split_body.data(), g->h_split_body.size() * 4,
                     hipMemcpyHostToDevice, s) != hipSuccess) {
    set_error("bie_geom_create: host to device copy failed");
    return fail(BIE_EDEVICE);
  }
  rc = geometry_build(g, curve, interior, s);
  if (rc != BIE_OK) return fail(rc);
  std::vector<double> area(Nd), len(Nd);
  if (hipMemcpyAsync(area.data(), g->area, Nd * 8, hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipMemcpyAsync(len.data(), g->len, Nd * 8, hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess) {
    set_error("bie_geom_create: device to host copy failed");
    return fail(BIE_EDEVICE);
  }
  for (int b = 0; b < nbodies; ++b) {
    if (!std::isfinite(area[b]) || !std::isfinite(len[b])) {
      set_error("bie_geom_create: non-finite curve samples on body " + std::to_string(b));
      return fail(BIE_EINVAL);
    }
    if (!(area[b] > 0.0)) {
      set_error("bie_geom_create: body " + std::to_string(b) +
                " is not positively oriented (signed area <= 0)");
      return fail(BIE_EINVAL);
    }
  }
  *out = g;
  return BIE_OK;
}

int bie_geom_destroy(bie_geom *g) {
  if (!g) return BIE_OK;
  hipDeviceSynchronize();
  g->arena.release();
  g->ws_apply.release();
  g->sm.release();
  g->seg.buf.release();
  g->ws_out.release();
  g->ws_read.release();
  if (g->fmm) fmm_destroy(g->fmm);
  delete g;
  return BIE_OK;
}

int bie_geom_sizes(const bie_geom *g, int *nbodies, int *M) {
  BIE_TRY(check_geom(g));
  if (nbodies) *nbodies = g->N;
  if (M) *M = g->M;
  return BIE_OK;
}

long long bie_geom_device_bytes(const bie_geom *g) {
  if (!g) return 0;
  return (long long)(g->arena.bytes + g->ws_apply.bytes + g->sm.big.bytes + g->sm.small.bytes +
                     g->ws_out.bytes + g->ws_read.bytes);
}

int bie_geom_set_fmm(bie_geom *g, int order, int leaf) {
  BIE_TRY(check_geom(g));
  if (order < 4 || order > 64 || leaf < 1) {
    set_error("bie_geom_set_fmm: order must lie in [4, 64] and leaf >= 1");
    return BIE_EINVAL;
  }
  g->fmm_order = order;
  g->fmm_leaf = leaf;
  return BIE_OK;
}

int bie_geom_export(const bie_geom *g, double *out, double *out_body, void *stream) {
  BIE_TRY(check_geom(g));
  hipStream_t s = as_stream(stream);
  const size_t Md = g->M, Nd = g->N;
  const double *src[8] = {g->x, g->y, g->nx, g->ny, g->w, g->kappa, g->px, g->py};
  if (out)
    for (int a = 0; a < 8; ++a)
      BIE_HIP_CHECK(hipMemcpyAsync(out + a * Md, src[a], Md * 8, hipMemcpyDeviceToDevice, s));
  const double *bsrc[4] = {g->len, g->xc, g->yc, g->W};
  if (out_body)
    for (int a = 0; a < 4; ++a)
      BIE_HIP_CHECK(hipMemcpyAsync(out_body + a * Nd, bsrc[a], Nd * 8, hipMemcpyDeviceToDevice, s));
  return BIE_OK;
}

static int apply_entry(bie_geom *g, int kind, int precision, int method, int with_L, int nrhs,
                       const double *mu, double *out, void *stream) {
  BIE_TRY(check_geom(g));
  if (mu == out) {
    set_error("apply: mu and out must not alias");
    return BIE_EINVAL;
  }
  return apply_operator(g, kind, precision, method, with_L ? 1 : 0, 1.0, nrhs, mu, out,
                        as_stream(stream));
}

int bie_laplace_apply(bie_geom *g, int precision, int method, int with_L, int nrhs,
                      const double *mu, double *out, void *stream) {
  return apply_entry(g, 0, precision, method, with_L, nrhs, mu, out, stream);
}

int bie_stokes_apply(bie_geom *g, int precision, int method, int with_L, int nrhs,
                     const double *mu, double *out, void *stream) {
  return apply_entry(g, 1, precision, method, with_L, nrhs, mu, out, stream);
}

// dens = incident density; f = -(1/2 I + K) dens (float64, same method as the solve)
static int rhs_entry(bie_geom *g, int kind, int method, int nrhs, const double *data,
                     double *dens, double *f, void *stream) {
  BIE_TRY(check_geom(g));
  if (nrhs < 1 || !data) {
    set_error("rhs: nrhs >= 1 and non-NULL input required");
    return BIE_EINVAL;
  }
  hipStream_t s = as_stream(stream);
  const size_t len = (size_t)g->M * (kind == 0 ? 1 : 2);
  double *tmp = dens;
  if (!tmp) {
    BIE_TRY(g->ws_out.reserve(len * nrhs * 8));
    tmp = g->ws_out.as<double>();
  }
  BIE_TRY(incident_density(g, kind, nrhs, data, tmp, s));
  if (f) BIE_TRY(apply_operator(g, kind, BIE_FP64, method, 0, -1.0, nrhs, tmp, f, s));
  return BIE_OK;
}

int bie_elastance_rhs(bie_geom *g, int nrhs, const double *q, double *sigma, double *f,
                      void *stream) {
  return rhs_entry(g, 0, BIE_DIRECT, nrhs, q, sigma, f, stream);
}

int bie_mobility_rhs(bie_geom *g, int nrhs, const double *FT, double *rho, double *f,
                     void *stream) {
  return rhs_entry(g, 1, BIE_DIRECT, nrhs, FT, rho, f, stream);
}

// Off-surface evaluation: total density = mu + incident density of `in`, then its layer
// potential at the given points.
static int field_entry(bie_geom *g, int kind, int nrhs, const double *in, const double *mu,
                       int npts, const double *pts, double *u, void *stream) {
  BIE_TRY(check_geom(g));
  if (nrhs < 1 || npts < 0 || !in || !mu || (npts > 0 && (!pts || !u))) {
    set_error("field: nrhs >= 1, npts >= 0 and non-NULL buffers required");
    return BIE_EINVAL;
  }
  if (npts == 0) return BIE_OK;
  hipStream_t s = as_stream(stream);
  const long long len = kind == 0 ? g->M : 2LL * g->M;
  BIE_TRY(g->ws_out.reserve((size_t)len * nrhs * 8));
  double *dens = g->ws_out.as<double>();
  BIE_TRY(incident_density(g, kind, nrhs, in, dens, s));
  BIE_TRY(vec_axpby(len * nrhs, 1.0, mu, 1.0, dens, s));
  return eval_points(g, kind, nrhs, dens, npts, pts, false, u, s);
}

int bie_laplace_potential(bie_geom *g, int nrhs, const double *dens, double *phi, void *stream) {
  BIE_TRY(check_geom(g));
  if (nrhs < 1 || !dens || !phi) {
    set_error("potential: nrhs >= 1 and non-NULL buffers required");
    return BIE_EINVAL;
  }
  return read_off(g, 0, nrhs, dens, phi, as_stream(stream));
}

int bie_elastance_field(bie_geom *g, int nrhs, const double *q, const double *mu, int npts,
                        const double *pts, double *u, void *stream) {
  return field_entry(g, 0, nrhs, q, mu, npts, pts, u, stream);
}

int bie_mobility_field(bie_geom *g, int nrhs, const double *FT, const double *mu, int npts,
                       const double *pts, double *u, void *stream) {
  return field_entry(g, 1, nrhs, FT, mu, npts, pts, u, stream);
}

int bie_stokes_rigid_motion(bie_geom *g, int nrhs, const double *dens, double *VW, void *stream) {
  BIE_TRY(check_geom(g));
  if (nrhs < 1 || !dens || !VW) {
    set_error("rigid motion: nrhs >= 1 and non-NULL buffers required");
    return BIE_EINVAL;
  }
  return read_off(g, 1, nrhs, dens, VW, as_stream(stream));
}

// The whole path: incident density, rhs, GMRES, read-off.
static int solve_entry(bie_geom *g, int kind, int nrhs, const double *data, double *res,
                       double *mu_out, const bie_opts *opts, bie_info *info, void *stream) {
  auto t0 = std::chrono::steady_clock::now();
  BIE_TRY(check_geom(g));
  if (nrhs < 1 || !data || !res) {
    set_error("solve: nrhs >= 1 and non-NULL input/output required");
    return BIE_EINVAL;
  }
  bie_opts o;
  if (opts) o = *opts; else fill_defaults(&o);
  BIE_TRY(check_opts(o));
  hipStream_t s = as_stream(stream);
  const size_t len = (size_t)g->M * (kind == 0 ? 1 : 2);
  g->fmm_order = o.fmm_order;
  g->fmm_leaf = o.fmm_leaf;
  // ws_out: dens [nrhs][len], f [nrhs][len], mu [nrhs][len]
  BIE_TRY(g->ws_out.reserve(3 * len * nrhs * 8));
  double *dens = g->ws_out.as<double>();
  double *f = dens + len * nrhs;
  double *mu = mu_out ? mu_out : f + len * nrhs;
  BIE_TRY(incident_density(g, kind, nrhs, data, dens, s));
  BIE_TRY(apply_operator(g, kind, BIE_FP64, o.method, 0, -1.0, nrhs, dens, f, s));
  int rc = solve_system(g, kind, o, nrhs, f, mu, info, s);
  if (rc != BIE_OK && rc != BIE_ENOCONV) return rc;
  BIE_TRY(vec_axpby((long long)nrhs * len, 1.0, mu, 1.0, dens, s));  // dens = mu + incident
  BIE_TRY(read_off(g, kind, nrhs, dens, res, s));
  BIE_HIP_CHECK(hipStreamSynchronize(s));
  if (info) {
    info->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (rc == BIE_OK && !(info->rel_residual <= o.tol)) rc = BIE_ENOCONV;
  }
  return rc;
}

int bie_elastance_solve(bie_geom *g, int nrhs, const double *q, double *phi, double *mu_out,
                        const bie_opts *opts, bie_info *info, void *stream) {
  return solve_entry(g, 0, nrhs, q, phi, mu_out, opts, info, stream);
}

int bie_mobility_solve(bie_geom *g, int nrhs, const double *FT, double *VW, double *mu_out,
                       const bie_opts *opts, bie_info *info, void *stream) {
  return solve_entry(g, 1, nrhs, FT, VW, mu_out, opts, info, stream);
}

// Capacitance and resistance: completed double layers, bounded solution (dirichlet.hip).
static int dl_apply_entry(bie_geom *g, int stokes, int with_C, int nrhs, const double *mu,
                          double *out, void *stream) {
  BIE_TRY(check_geom(g));
  if (nrhs < 1 || !mu || !out || mu == out) {
    set_error("double-layer apply: nrhs >= 1, non-NULL and distinct mu, out required");
    return BIE_EINVAL;
  }
  return dl_apply(g, stokes, with_C ? 1 : 0, 1.0, nrhs, mu, out, as_stream(stream));
}

int bie_laplace_dl_apply(bie_geom *g, int with_completion, int nrhs, const double *mu, double *out,
                         void *stream) {
  return dl_apply_entry(g, 0, with_completion, nrhs, mu, out, stream);
}

int bie_stokes_dl_apply(bie_geom *g, int with_completion, int nrhs, const double *mu, double *out,
                        void *stream) {
  return dl_apply_entry(g, 1, with_completion, nrhs, mu, out, stream);
}

static int dl_solve_entry(bie_geom *g, int stokes, int nrhs, const double *data, double *res,
                          double *u_inf, double *mu_out, const bie_opts *opts, bie_info *info,
                          void *stream) {
  auto t0 = std::chrono::steady_clock::now();
  BIE_TRY(check_geom(g));
  if (nrhs < 1 || !data || !res || !u_inf) {
    set_error("capacitance/resistance solve: nrhs >= 1 and non-NULL input and outputs required");
    return BIE_EINVAL;
  }
  bie_opts o;
  if (opts) o = *opts; else fill_defaults(&o);
  BIE_TRY(check_opts(o));
  hipStream_t s = as_stream(stream);
  int rc = dl_solve(g, stokes, nrhs, data, res, u_inf, mu_out, o, info, s);
  if (rc != BIE_OK && rc != BIE_ENOCONV) return rc;
  BIE_HIP_CHECK(hipStreamSynchronize(s));
  if (info) {
    info->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (rc == BIE_OK && !(info->rel_residual <= o.tol)) rc = BIE_ENOCONV;
  }
  return rc;
}

int bie_capacitance_solve(bie_geom *g, int nrhs, const double *phi, double *q, double *u_inf,
                          double *mu_out, const bie_opts *opts, bie_info *info, void *stream) {
  return dl_solve_entry(g, 0, nrhs, phi, q, u_inf, mu_out, opts, info, stream);
}

int bie_resistance_solve(bie_geom *g, int nrhs, const double *VW, double *FT, double *u_inf,
                         double *mu_out, const bie_opts *opts, bie_info *info, void *stream) {
  return dl_solve_entry(g, 1, nrhs, VW, FT, u_inf, mu_out, opts, info, stream);
}

// Identity right-hand-side block, solved in passes of <= max_rhs columns; column j of the
// result is written to out + j * ncols (column-major, ncols = N or 3N).
static int matrix_entry(bie_geom *g, int kind, double *out, int max_rhs, const bie_opts *opts,
                        bie_info *info, void *stream) {
  auto t0 = std::chrono::steady_clock::now();
  BIE_TRY(check_geom(g));
  if (!out) {
    set_error("matrix: NULL output");
    return BIE_EINVAL;
  }
  hipStream_t s = as_stream(stream);
  const int ncols = kind == 0 ? g->N : 3 * g->N;
  if (max_rhs <= 0) max_rhs = kind == 0 ? 32 : 24;
  max_rhs = std::min(max_rhs, ncols);
  // identity columns built on the host (ncols x ncols would be large; only one pass at a time)
  bie::DevBuf idbuf;
  BIE_TRY(idbuf.reserve((size_t)max_rhs * ncols * 8));
  std::vector<double> host((size_t)max_rhs * ncols);
  bie_info acc{};
  int rc_all = BIE_OK;
  for (int c0 = 0; c0 < ncols; c0 += max_rhs) {
    const int nr = std::min(max_rhs, ncols - c0);
    std::fill(host.begin(), host.end(), 0.0);
    for (int r = 0; r < nr; ++r) host[(size_t)r * ncols + c0 + r] = 1.0;
    if (hipMemcpyAsync(idbuf.ptr, host.data(), (size_t)nr * ncols * 8, hipMemcpyHostToDevice, s) !=
        hipSuccess) {
      idbuf.release();
      set_error("matrix: host to device copy failed");
      return BIE_EDEVICE;
    }
    bie_info one{};
    int rc = solve_entry(g, kind, nr, idbuf.as<double>(), out + (size_t)c0 * ncols, nullptr,
                         opts, &one, stream);
    if (rc != BIE_OK && rc != BIE_ENOCONV) {
      idbuf.release();
      return rc;
    }
    if (rc == BIE_ENOCONV) rc_all = rc;
    acc.iters = std::max(acc.iters, one.iters);
    acc.refinements = std::max(acc.refinements, one.refinements);
    acc.applies_fp64 += one.applies_fp64;
    acc.applies_fp32 += one.applies_fp32;
    acc.rel_residual = std::max(acc.rel_residual, one.rel_residual);
    acc.pairs += one.pairs;
  }
  hipStreamSynchronize(s);
  idbuf.release();
  acc.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  if (info) *info = acc;
  return rc_all;
}

int bie_elastance_matrix(bie_geom *g, double *P, int max_rhs_per_pass, const bie_opts *opts,
                         bie_info *info, void *stream) {
  return matrix_entry(g, 0, P, max_rhs_per_pass, opts, info, stream);
}

int bie_mobility_matrix(bie_geom *g, double *Mmat, int max_rhs_per_pass, const bie_opts *opts,
                        bie_info *info, void *stream) {
  return matrix_entry(g, 1, Mmat, max_rhs_per_pass, opts, info, stream);
}

}  // extern "C"
