// C ABI entry points of libbie2d (declared in include/bie2d.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstring>
#include <mutex>
#include <new>
#include <set>
#include <string>
#include <vector>

#include "internal.h"

namespace bie {

static thread_local std::string g_last_error = "no error";

void set_error(const std::string &msg) { g_last_error = msg; }

static std::atomic<unsigned long long> g_epoch{0};
unsigned long long buffer_epoch() { return g_epoch.load(); }

// off by default: on ROCm 7.2 a replayed step measured slower than its stream launches (about
// 6 us more per Arnoldi step of the 1000-starfish solve)
static std::atomic<int> g_graphs{0};
bool graphs_enabled() { return g_graphs.load() != 0; }

int DevBuf::reserve(size_t need) {
  if (need <= bytes) return BIE_OK;
  g_epoch.fetch_add(1);
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
  if (ptr) g_epoch.fetch_add(1);
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
  o->mixed_strategy = BIE_MIXED_RELAXED;
  o->precond = BIE_PRECOND_NONE;
  o->viscosity = 1.0;
  o->fmm_eps = 0.0;
  o->l2_scaling = 0;
}

int check_opts(const bie_opts &o) {
  if ((o.precision != BIE_FP64 && o.precision != BIE_MIXED) ||
      (o.method != BIE_DIRECT && o.method != BIE_FMM && o.method != BIE_AUTO) ||
      !(o.tol > 0.0) || o.restart < 1 ||
      o.max_iter < 1 || !(o.inner_tol > 0.0) || o.max_refine < 0 || o.fmm_order < 4 ||
      o.fmm_order > 64 || o.fmm_leaf < 0 || !(o.viscosity > 0.0) || !std::isfinite(o.viscosity) ||
      !(o.fmm_eps >= 0.0) || !(o.fmm_eps < 1.0) || (o.l2_scaling != 0 && o.l2_scaling != 1) ||
      (o.mixed_strategy != BIE_MIXED_RELAXED && o.mixed_strategy != BIE_MIXED_REFINE) ||
      (o.precond != BIE_PRECOND_NONE && o.precond != BIE_PRECOND_BLOCK) ||
      (o.precond == BIE_PRECOND_BLOCK && o.l2_scaling)) {
    set_error("invalid bie_opts");
    return BIE_EINVAL;
  }
  return BIE_OK;
}

// The expansion order the options ask for: from fmm_eps when it is set, else fmm_order.
// The float64 FMM apply's relative error (2-norm against direct summation, measured on the
// 1000-starfish and 200-ellipse geometries at orders 16, 24, 32) falls as about 0.45^p from
// 2.1e-3 (Laplace) and 4.3e-2 (Stokes); fmm_eps takes the smallest order that this model puts
// below it.
int effective_order(const bie_opts &o, int kind) {
  if (!(o.fmm_eps > 0.0)) return o.fmm_order;
  const double k0 = (kind & 1) ? 4.3e-2 : 2.1e-3;
  const int p = (int)std::ceil(std::log(o.fmm_eps / k0) / std::log(0.45));
  return std::max(8, std::min(64, p));
}


}  // namespace bie

struct bie_tune_cache;

struct bie_ctx {
  int device = 0;
  bie_opts defaults{};
  std::mutex mu;
  std::set<bie_geom *> geoms;  // owned until bie_geom_destroy
  bie_tune_cache *tune = nullptr;  // autotuned FMM leaf sizes of this context's shape classes
};

namespace bie {
bie_tune_cache *new_tune_cache();
void delete_tune_cache(bie_tune_cache *c);
bie_tune_cache *process_tune_cache();
int tune_cache_stats(bie_tune_cache *c, long long *tunings, long long *hits);
bie_tune_cache *tune_cache_of(bie_geom *g) { return g && g->ctx ? g->ctx->tune : nullptr; }
// Options of a call: the caller's, else its context's defaults, else the process defaults.
static bie_opts opts_for(const bie_geom *g, const bie_opts *opts) {
  bie_opts o;
  if (opts) o = *opts;
  else if (g && g->ctx) o = g->ctx->defaults;
  else fill_defaults(&o);
  return o;
}
}  // namespace bie

using namespace bie;

static int geom_create(int nbodies, const int32_t *nodes_per_body, const double *curve,
                       const double *interior, void *stream, bie_geom **out);

extern "C" {

int bie_create(bie_ctx **out, int device, const bie_opts *defaults) {
  if (!out) {
    set_error("bie_create: NULL out");
    return BIE_EINVAL;
  }
  *out = nullptr;
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || count < 1) {
    set_error("bie_create: no HIP device");
    return BIE_EDEVICE;
  }
  if (device < 0 || device >= count) {
    set_error("bie_create: device ordinal " + std::to_string(device) + " out of range [0, " +
              std::to_string(count) + ")");
    return BIE_EINVAL;
  }
  bie_opts o;
  if (defaults) o = *defaults; else fill_defaults(&o);
  BIE_TRY(check_opts(o));
  bie_ctx *c = new (std::nothrow) bie_ctx();
  if (!c) {
    set_error("host allocation failed");
    return BIE_ENOMEM;
  }
  c->device = device;
  c->defaults = o;
  c->tune = new_tune_cache();
  *out = c;
  return BIE_OK;
}

int bie_destroy(bie_ctx *ctx) {
  if (!ctx) return BIE_OK;
  std::set<bie_geom *> left;
  {
    std::lock_guard<std::mutex> lk(ctx->mu);
    left.swap(ctx->geoms);
  }
  for (bie_geom *g : left) {
    g->ctx = nullptr;
    bie_geom_destroy(g);
  }
  delete_tune_cache(ctx->tune);
  delete ctx;
  return BIE_OK;
}

int bie_ctx_defaults(const bie_ctx *ctx, bie_opts *out) {
  if (!ctx || !out) {
    set_error("bie_ctx_defaults: NULL argument");
    return BIE_EINVAL;
  }
  *out = ctx->defaults;
  return BIE_OK;
}

int bie_ctx_geom_create(bie_ctx *ctx, int nbodies, const int32_t *nodes_per_body,
                        const double *curve, const double *interior, void *stream,
                        bie_geom **out) {
  if (!ctx) {
    set_error("bie_ctx_geom_create: NULL context");
    return BIE_EINVAL;
  }
  DeviceGuard dg(ctx->device);
  const int rc = geom_create(nbodies, nodes_per_body, curve, interior, stream, out);
  if ((rc == BIE_OK || rc == BIE_ERESOLVE) && out && *out) {
    (*out)->ctx = ctx;
    std::lock_guard<std::mutex> lk(ctx->mu);
    ctx->geoms.insert(*out);
  }
  return rc;
}

const char *bie_last_error(void) { return g_last_error.c_str(); }

int bie_set_graphs(int on) {
  g_graphs.store(on ? 1 : 0);
  return BIE_OK;
}

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
  return geom_create(nbodies, nodes_per_body, curve, interior, stream, out);
}

int bie_curves_check(int nbodies, const int32_t *nodes_per_body, const double *curve,
                     const double *interior) {
  if (!nodes_per_body || !curve || nbodies < 1) {
    set_error("bie_curves_check: need nbodies >= 1 and non-NULL nodes_per_body, curve");
    return BIE_EINVAL;
  }
  for (int b = 0; b < nbodies; ++b)
    if (nodes_per_body[b] < 3) {
      set_error("bie_curves_check: body " + std::to_string(b) + " has fewer than 3 nodes");
      return BIE_EINVAL;
    }
  std::string msg;
  const int rc = check_curves(nbodies, nodes_per_body, curve, interior, msg);
  if (rc != BIE_OK) set_error("bie_curves_check: " + msg);
  return rc;
}

}  // extern "C"

static int geom_create(int nbodies, const int32_t *nodes_per_body, const double *curve,
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
  // the caller's samples (device memory) are checked on the host before anything is built
  int warn = BIE_OK;
  std::string warn_msg;
  {
    hipStream_t s0 = as_stream(stream);
    std::vector<double> hc(6 * (size_t)M), hi(interior ? 2 * (size_t)nbodies : 0);
    if (hipMemcpyAsync(hc.data(), curve, hc.size() * 8, hipMemcpyDeviceToHost, s0) != hipSuccess ||
        (interior && hipMemcpyAsync(hi.data(), interior, hi.size() * 8, hipMemcpyDeviceToHost,
                                    s0) != hipSuccess) ||
        hipStreamSynchronize(s0) != hipSuccess) {
      set_error("bie_geom_create: device to host copy of the curve samples failed");
      return BIE_EDEVICE;
    }
    warn = check_curves(nbodies, nodes_per_body, hc.data(), interior ? hi.data() : nullptr,
                        warn_msg);
    if (warn == BIE_EINVAL) {
      set_error("bie_geom_create: " + warn_msg);
      return BIE_EINVAL;
    }
  }
  bie_geom *g = new (std::nothrow) bie_geom();
  if (!g) {
    set_error("host allocation failed");
    return BIE_ENOMEM;
  }
  static std::atomic<unsigned long long> next_gen{1};
  g->gen = next_gen.fetch_add(1);
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
  if (hipStreamSynchronize(s) != hipSuccess) {  // the geometry is ready on any stream
    set_error("bie_geom_create: geometry build failed on the device");
    return fail(BIE_EDEVICE);
  }
  *out = g;
  if (warn != BIE_OK) set_error("bie_geom_create (warning, geometry created): " + warn_msg);
  return warn;
}

extern "C" {

int bie_geom_destroy(bie_geom *g) {
  if (!g) return BIE_OK;
  if (g->ctx) {
    std::lock_guard<std::mutex> lk(g->ctx->mu);
    g->ctx->geoms.erase(g);
  }
  DeviceGuard dg(g->device);
  (void)hipDeviceSynchronize();
  g->arena.release();
  g->ws_apply.release();
  g->sm.release();
  g->seg.buf.release();
  g->ws_out.release();
  g->ws_read.release();
  g->ws_scale.release();
  for (auto &pc : g->pc) {
    pc.inv.release();
    pc.meta.release();
  }
  if (g->in_ev) (void)hipEventDestroy(g->in_ev);
  if (g->fmm) fmm_destroy(g->fmm);
  delete g;
  return BIE_OK;
}

int bie_autotune(bie_geom *g, int kind, int precision, int nrhs, int *leaf_fp64,
                 int *leaf_mixed, void *stream) {
  BIE_TRY(check_geom(g));
  DeviceGuard dg(g->device);
  if ((kind != 0 && kind != 1) || (precision != BIE_FP64 && precision != BIE_MIXED) || nrhs < 1) {
    set_error("bie_autotune: kind 0 or 1, precision BIE_FP64 or BIE_MIXED, nrhs >= 1");
    return BIE_EINVAL;
  }
  BIE_TRY(autotune_leaf(g, kind, precision, nrhs, as_stream(stream)));
  if (leaf_fp64) *leaf_fp64 = g->fmm_leaf;
  if (leaf_mixed) *leaf_mixed = g->fmm_leaf_mixed > 0 ? g->fmm_leaf_mixed : g->fmm_leaf;
  return BIE_OK;
}

int bie_fmm_terms(const bie_opts *opts, int kind, int precision, int *terms) {
  if (!opts || (kind != 0 && kind != 1) || (precision != BIE_FP64 && precision != BIE_MIXED) ||
      !terms) {
    set_error("bie_fmm_terms: need opts, kind 0 or 1, precision BIE_FP64 or BIE_MIXED, terms");
    return BIE_EINVAL;
  }
  BIE_TRY(check_opts(*opts));
  *terms = fmm_length(effective_order(*opts, kind), precision);
  return BIE_OK;
}

int bie_autotune_stats(const bie_ctx *ctx, long long *tunings, long long *hits) {
  return tune_cache_stats(ctx ? ctx->tune : process_tune_cache(), tunings, hits);
}

int bie_geom_graph_stats(const bie_geom *g, long long *captured, long long *replayed) {
  BIE_TRY(check_geom(g));
  if (captured) *captured = g->sm.graph_captures;
  if (replayed) *replayed = g->sm.graph_replays;
  return BIE_OK;
}

int bie_geom_sizes(const bie_geom *g, int *nbodies, int *M) {
  BIE_TRY(check_geom(g));
  DeviceGuard dg(g->device);
  if (nbodies) *nbodies = g->N;
  if (M) *M = g->M;
  return BIE_OK;
}

long long bie_geom_device_bytes(const bie_geom *g) {
  if (!g) return 0;
  return (long long)(g->arena.bytes + g->ws_apply.bytes + g->sm.big.bytes + g->sm.small.bytes +
                     g->ws_out.bytes + g->ws_read.bytes + g->ws_scale.bytes);
}

int bie_geom_set_fmm(bie_geom *g, int order, int leaf) {
  BIE_TRY(check_geom(g));
  DeviceGuard dg(g->device);
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
  DeviceGuard dg(g->device);
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
  DeviceGuard dg(g->device);
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
  DeviceGuard dg(g->device);
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
  DeviceGuard dg(g->device);
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
  return eval_points(g, kind, nrhs, dens, npts, pts, false, u, s, BIE_AUTO);
}

int bie_laplace_potential(bie_geom *g, int nrhs, const double *dens, double *phi, void *stream) {
  BIE_TRY(check_geom(g));
  DeviceGuard dg(g->device);
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
  DeviceGuard dg(g->device);
  if (nrhs < 1 || !dens || !VW) {
    set_error("rigid motion: nrhs >= 1 and non-NULL buffers required");
    return BIE_EINVAL;
  }
  return read_off(g, 1, nrhs, dens, VW, as_stream(stream));
}

// Checks a solve's input ([nrhs][N] charges, or [nrhs][3N] (F, T)) once it is on the host (h):
// rejects non-finite entries, and returns the net charge (sum q) or net force (sum F) of the
// right-hand side with the largest magnitude.
static int input_check(int kind, int N, int nrhs, const double *h, double net[2]) {
  const size_t width = kind == 0 ? (size_t)N : 3 * (size_t)N;
  net[0] = net[1] = 0.0;
  double best = -1.0;
  for (int r = 0; r < nrhs; ++r) {
    const double *v = h + (size_t)r * width;
    double a = 0.0, b = 0.0;
    for (size_t j = 0; j < width; ++j)
      if (!std::isfinite(v[j])) {
        set_error(std::string("solve: non-finite ") + (kind == 0 ? "charge" : "force or torque") +
                  " in right-hand side " + std::to_string(r));
        return BIE_EINVAL;
      }
    if (kind == 0) {
      for (int j = 0; j < N; ++j) a += v[j];
    } else {
      for (int j = 0; j < N; ++j) {
        a += v[3 * j];
        b += v[3 * j + 1];
      }
    }
    if (std::hypot(a, b) > best) {
      best = std::hypot(a, b);
      net[0] = a;
      net[1] = b;
    }
  }
  return BIE_OK;
}

// The whole path: incident density, rhs, GMRES, read-off.
static int solve_entry(bie_geom *g, int kind, int nrhs, const double *data, double *res,
                       double *mu_out, const bie_opts *opts, bie_info *info, void *stream) {
  auto t0 = std::chrono::steady_clock::now();
  BIE_TRY(check_geom(g));
  DeviceGuard dg(g->device);
  if (nrhs < 1 || !data || !res) {
    set_error("solve: nrhs >= 1 and non-NULL input/output required");
    return BIE_EINVAL;
  }
  const bie_opts o = opts_for(g, opts);
  BIE_TRY(check_opts(o));
  hipStream_t s = as_stream(stream);
  // the input goes to pinned host memory ahead of the right-hand side's work, and is checked
  // while that work runs (a rejected input leaves only scratch written)
  const size_t in_bytes = (size_t)nrhs * (kind == 0 ? g->N : 3 * (size_t)g->N) * sizeof(double);
  BIE_TRY(g->sm.ensure_pinned(in_bytes));
  if (!g->in_ev) BIE_HIP_CHECK(hipEventCreateWithFlags(&g->in_ev, hipEventDisableTiming));
  BIE_HIP_CHECK(hipMemcpyAsync(g->sm.pinned, data, in_bytes, hipMemcpyDeviceToHost, s));
  BIE_HIP_CHECK(hipEventRecord(g->in_ev, s));
  const size_t len = (size_t)g->M * (kind == 0 ? 1 : 2);
  g->fmm_order = effective_order(o, kind);
  const int meth = o.method == BIE_AUTO ? (method_is_fmm(o.method, g->M) ? BIE_FMM : BIE_DIRECT) : o.method;
  // leaf sizes (fmm_leaf 0: from the tuner, cached per shape class)
  BIE_TRY(resolve_leaf(g, kind, o, nrhs, meth == BIE_FMM, s));
  // ws_out: dens [nrhs][len], f [nrhs][len], mu [nrhs][len]
  BIE_TRY(g->ws_out.reserve(3 * len * nrhs * 8));
  double *dens = g->ws_out.as<double>();
  double *f = dens + len * nrhs;
  double *mu = mu_out ? mu_out : f + len * nrhs;
  BIE_TRY(incident_density(g, kind, nrhs, data, dens, s));
  BIE_TRY(apply_operator(g, kind, BIE_FP64, o.method, 0, -1.0, nrhs, dens, f, s));
  double net[2];
  BIE_HIP_CHECK(hipEventSynchronize(g->in_ev));
  {
    const int rc = input_check(kind, g->N, nrhs, g->sm.pinned, net);
    if (rc != BIE_OK) {
      (void)hipStreamSynchronize(s);
      return rc;
    }
  }
  int rc = solve_system(g, kind, o, nrhs, f, mu, info, s);
  if (rc != BIE_OK && rc != BIE_ENOCONV) return rc;
  BIE_TRY(vec_axpby((long long)nrhs * len, 1.0, mu, 1.0, dens, s));  // dens = mu + incident
  BIE_TRY(read_off(g, kind, nrhs, dens, res, s, o.method));
  if (kind == 1 && o.viscosity != 1.0)  // velocities of the viscosity-1 problem, rescaled
    BIE_TRY(vec_axpby((long long)nrhs * 3 * g->N, 0.0, res, 1.0 / o.viscosity, res, s));
  BIE_HIP_CHECK(hipStreamSynchronize(s));
  if (info) {
    info->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    info->net_charge_or_force[0] = net[0];
    info->net_charge_or_force[1] = net[1];
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
  DeviceGuard dg(g->device);
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
  DeviceGuard dg(g->device);
  if (nrhs < 1 || !data || !res || !u_inf) {
    set_error("capacitance/resistance solve: nrhs >= 1 and non-NULL input and outputs required");
    return BIE_EINVAL;
  }
  const bie_opts o = opts_for(g, opts);
  BIE_TRY(check_opts(o));
  hipStream_t s = as_stream(stream);
  int rc = dl_solve(g, stokes, nrhs, data, res, u_inf, mu_out, o, info, s);
  if (rc != BIE_OK && rc != BIE_ENOCONV) return rc;
  if (stokes && o.viscosity != 1.0)  // forces and torques of the viscosity-1 problem, rescaled
    BIE_TRY(vec_axpby((long long)nrhs * 3 * g->N, 0.0, res, o.viscosity, res, s));
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
  DeviceGuard dg(g->device);
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
    if (std::hypot(one.net_charge_or_force[0], one.net_charge_or_force[1]) >
        std::hypot(acc.net_charge_or_force[0], acc.net_charge_or_force[1])) {
      acc.net_charge_or_force[0] = one.net_charge_or_force[0];
      acc.net_charge_or_force[1] = one.net_charge_or_force[1];
    }
  }
  const hipError_t se = hipStreamSynchronize(s);
  idbuf.release();
  if (se != hipSuccess) {
    set_error(std::string("matrix: stream synchronisation failed: ") + hipGetErrorString(se));
    return BIE_EDEVICE;
  }
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
