// Serving loop: continuous batching of elastance and mobility requests at GMRES-cycle
// granularity, with admission by device-memory footprint (declared in include/bie2d.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "internal.h"

namespace bie {
namespace {

using Clock = std::chrono::steady_clock;

struct Request {
  long long id = 0;
  bie_geom *g = nullptr;
  int kind = 0, nrhs = 0;
  long long n = 0;                 // unknowns per rhs
  std::vector<double> in;          // host copy of the input
  double *out = nullptr;           // caller's host buffer
  DevBuf dev;                      // inc, f, x, result  [nrhs][n] x 3 + [nrhs][width]
  double *inc = nullptr, *f = nullptr, *x = nullptr, *res = nullptr;
  std::vector<double> relres;      // per rhs, from the last residual
  long long bytes = 0;             // admission footprint
  int cycles = 0;
  Clock::time_point t_submit, t_admit;
  bie_request_info info{};
  bool done = false;
};

}  // namespace
}  // namespace bie

struct bie_server {
  bie_server_config cfg;
  int device = 0;
  hipStream_t stream = nullptr;  // the worker's stream (created with the server)
  std::thread worker;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<std::shared_ptr<bie::Request>> queue;
  std::map<long long, std::shared_ptr<bie::Request>> all;  // until waited for
  long long next_id = 1;
  bool stopping = false;
  // per (geometry id, kind) in flight: requests using it and the bytes charged once for its
  // apply state (FMM tree and work area, apply workspace)
  std::map<unsigned long long, std::pair<int, long long>> geom_use;
  int inject_fail = 0;  // cycles still to fail on purpose (tests of the error path)
  // worker-side state
  std::vector<std::shared_ptr<bie::Request>> active;
  long long bytes_in_flight = 0, peak_bytes = 0;
  long long n_requests = 0, n_solves = 0, n_cycles = 0;
  bie::Segments seg;
  bie::SolverMem sm;
  bie::DevBuf flat;  // F, X, R, D [Ntot] each
  bie::DevBuf pcitems;  // the block preconditioner's item descriptors of a cycle
  bie::MultiPlan *plan = nullptr;
  void run();
  int cycle();
  void complete(bie::Request &r, int status);
  void fail_active(int status);
};

namespace bie {
namespace {

bool uses_fmm(const bie_opts &o, const bie_geom *g) {
  return method_is_fmm(o.method, g->M);
}

// Device bytes of one request's solver state: its buffers (incident density, rhs, iterate,
// result), its share of the flat vectors (F, X, R, D), of the Krylov basis (restart + 1
// vectors) and of the apply workspace (float64 and float32 strengths).
long long footprint(const bie_server_config &c, bie_geom *g, int kind, int nrhs) {
  const long long n = kind == 0 ? g->M : 2LL * g->M;
  const int width = kind == 0 ? g->N : 3 * g->N;
  return 8LL * nrhs * (3 * n + width) + 8LL * nrhs * n * (c.opts.restart + 1 + 4 + 3) +
         12LL * nrhs * n;
}

// Device bytes charged once per geometry (and kind) while any of its requests is in flight:
// the FMM tree and work area of the orders the solve uses, and the far-field partial sums of
// the geometry's own apply workspace.
long long geom_footprint(const bie_server_config &c, const bie_geom *g, int kind) {
  // the block preconditioner's coarse inverses (float32, padded to 64 x 64 Laplace, 128 x 128
  // Stokes, per body) and node counts
  const long long pc = c.opts.precond == BIE_PRECOND_BLOCK
                           ? (long long)g->N * ((kind == 0 ? 64LL * 64 : 128LL * 128) * 4 + 4)
                           : 0;
  if (!uses_fmm(c.opts, g)) return pc;
  const long long len = kind == 0 ? g->M : 2LL * g->M;
  return pc + fmm_state_bytes(g, kind, c.opts.precision, effective_order(c.opts, kind),
                              c.opts.fmm_leaf) +
         8LL * (kind == 0 ? 8 : 4) * len;
}

unsigned long long geom_key(const Request &r) { return r.g->gen * 2 + (unsigned)r.kind; }

int prepare(Request &r, const bie_opts &o, hipStream_t s) {
  const int width = r.kind == 0 ? r.g->N : 3 * r.g->N;
  const size_t cnt = (size_t)r.nrhs * (3 * r.n + width);
  BIE_TRY(r.dev.reserve(cnt * sizeof(double)));
  r.inc = r.dev.as<double>();
  r.f = r.inc + (size_t)r.nrhs * r.n;
  r.x = r.f + (size_t)r.nrhs * r.n;
  r.res = r.x + (size_t)r.nrhs * r.n;
  r.g->fmm_order = effective_order(o, r.kind);
  // fmm_leaf 0 serves with 64 nodes per leaf: timing leaf sizes would pause the other requests
  BIE_TRY(resolve_leaf(r.g, r.kind, o, r.nrhs, false, s));
  if (o.precond == BIE_PRECOND_BLOCK) BIE_TRY(pc_build(r.g, r.kind, s));  // once per geometry
  // stage the input in the result buffer, then incident density and rhs f = -(1/2 I + K) inc
  BIE_HIP_CHECK(hipMemcpyAsync(r.res, r.in.data(), r.in.size() * sizeof(double),
                               hipMemcpyHostToDevice, s));
  BIE_TRY(incident_density(r.g, r.kind, r.nrhs, r.res, r.inc, s));
  BIE_TRY(apply_operator(r.g, r.kind, BIE_FP64, o.method, 0, -1.0, r.nrhs, r.inc, r.f, s));
  BIE_HIP_CHECK(hipMemsetAsync(r.x, 0, sizeof(double) * r.nrhs * r.n, s));
  r.relres.assign(r.nrhs, 1.0);
  return BIE_OK;
}

int finish(Request &r, const bie_opts &o, hipStream_t s) {
  const int width = r.kind == 0 ? r.g->N : 3 * r.g->N;
  BIE_TRY(vec_axpby((long long)r.nrhs * r.n, 1.0, r.x, 1.0, r.inc, s));  // inc = mu + incident
  BIE_TRY(read_off(r.g, r.kind, r.nrhs, r.inc, r.res, s, uses_fmm(o, r.g) ? BIE_FMM : BIE_DIRECT));
  if (r.kind == 1 && o.viscosity != 1.0)  // velocities for the configured viscosity
    BIE_TRY(vec_axpby((long long)r.nrhs * width, 0.0, r.res, 1.0 / o.viscosity, r.res, s));
  BIE_HIP_CHECK(hipMemcpyAsync(r.out, r.res, sizeof(double) * r.nrhs * width,
                               hipMemcpyDeviceToHost, s));
  BIE_HIP_CHECK(hipStreamSynchronize(s));
  return BIE_OK;
}

// Flat layout of the active requests: requests of one geometry and kind are adjacent (the
// active list is kept sorted that way) and packed back to back, so each such group is one item
// of the multi-geometry apply; groups start at 64-byte boundaries. off[i] is the start of
// request i; items[k] covers requests first[k] .. first[k+1]-1.
struct Layout {
  std::vector<long long> off;
  std::vector<MultiItem> items;
  std::vector<size_t> first;
  long long total = 0;
};

Layout layout(const std::vector<std::shared_ptr<Request>> &reqs, const bie_opts &o) {
  Layout L;
  L.off.assign(reqs.size() + 1, 0);
  long long cur = 0;
  for (size_t i = 0; i < reqs.size(); ++i) {
    const Request &r = *reqs[i];
    const bool new_group = i == 0 || reqs[i - 1]->g != r.g || reqs[i - 1]->kind != r.kind;
    if (new_group) {
      cur = align8(cur);
      L.first.push_back(i);
      L.items.push_back({r.g, r.kind, 0, cur, uses_fmm(o, r.g), effective_order(o, r.kind),
                         r.g->fmm_leaf});
    }
    L.off[i] = cur;
    L.items.back().nrhs += r.nrhs;
    cur += (long long)r.nrhs * r.n;
  }
  L.first.push_back(reqs.size());
  L.total = align8(cur);
  L.off[reqs.size()] = L.total;
  return L;
}

}  // namespace
}  // namespace bie

using namespace bie;

// Marks r done with the given status and returns its bytes (and, with its geometry's last
// request, the geometry's charge) to the budget. Takes the lock.
void bie_server::complete(Request &r, int status) {
  r.info.status = status;
  r.info.cycles = r.cycles;
  r.info.latency_s = std::chrono::duration<double>(Clock::now() - r.t_submit).count();
  r.dev.release();
  std::lock_guard<std::mutex> lk(mu);
  bytes_in_flight -= r.bytes;
  auto it = geom_use.find(geom_key(r));
  if (it != geom_use.end() && --it->second.first == 0) {
    bytes_in_flight -= it->second.second;
    geom_use.erase(it);
  }
  if (status == BIE_OK || status == BIE_ENOCONV) {
    n_requests += 1;
    n_solves += r.nrhs;
  }
  r.done = true;
  cv_done.notify_all();
}

// After a failed cycle: every request of the cycle fails with `status`; the worker drains its
// stream, drops the batched-apply plan (its workspace may be half written) and goes on with
// the requests that arrive later.
void bie_server::fail_active(int status) {
  (void)hipStreamSynchronize(stream);
  for (auto &r : active) complete(*r, status);
  active.clear();
  multi_destroy(plan);
  plan = nullptr;
}

// One cycle over the active requests: float64 residuals, retirement of converged requests,
// one Arnoldi cycle for the rest. A non-OK return fails the requests still active.
int bie_server::cycle() {
  hipStream_t s = stream;
  const bie_opts &o = cfg.opts;
  const int m = std::max(1, o.restart);
  {
    std::lock_guard<std::mutex> lk(mu);
    if (inject_fail > 0) {
      --inject_fail;
      set_error("server cycle: injected failure");
      return BIE_EDEVICE;
    }
  }
  // ---- flat layout of the active systems ------------------------------------------------------
  const Layout L1 = layout(active, o);
  const std::vector<long long> &off = L1.off;
  std::vector<long long> lens, starts;
  for (size_t i = 0; i < active.size(); ++i)
    for (int k = 0; k < active[i]->nrhs; ++k) {
      lens.push_back(active[i]->n);
      starts.push_back(off[i] + k * active[i]->n);
    }
  const long long N = L1.total;
  BIE_TRY(seg.build(lens, s, &starts));
  BIE_TRY(flat.reserve(4 * (size_t)N * sizeof(double)));
  double *F = flat.as<double>(), *X = F + N, *R = X + N, *D = R + N;
  for (size_t i = 0; i < active.size(); ++i) {
    const size_t bytes = sizeof(double) * active[i]->nrhs * active[i]->n;
    BIE_HIP_CHECK(hipMemcpyAsync(F + off[i], active[i]->f, bytes, hipMemcpyDeviceToDevice, s));
    BIE_HIP_CHECK(hipMemcpyAsync(X + off[i], active[i]->x, bytes, hipMemcpyDeviceToDevice, s));
  }
  SysSet ss;
  ss.seg = &seg;
  ss.mem = &sm;
  MultiPlan **planp = &plan;
  {
    const std::vector<MultiItem> mi = L1.items;
    ss.apply = [mi, planp, N](int precision, const double *in, double *out, hipStream_t st) {
      return multi_apply(*planp, mi, std::vector<char>(mi.size(), 1), precision, in, out, N, st);
    };
  }
  // ---- true residual with the float64 operator; retire converged requests -------------------
  BIE_TRY(ss.apply(BIE_FP64, X, R, s));
  BIE_TRY(vec_axpby(N, 1.0, F, -1.0, R, s));
  std::vector<double> rn, fn;
  {
    BIE_TRY(sm.small.reserve((size_t)(2 * seg.S + seg.C) * sizeof(double) + 64));
    double *tmp = sm.small.as<double>();
    BIE_TRY(seg_nrm2(seg, R, tmp, tmp + 2 * seg.S, s));
    BIE_TRY(seg_nrm2(seg, F, tmp + seg.S, tmp + 2 * seg.S, s));
    BIE_TRY(sm.ensure_pinned(2 * seg.S * sizeof(double)));
    BIE_HIP_CHECK(hipMemcpyAsync(sm.pinned, tmp, 2 * seg.S * sizeof(double),
                                 hipMemcpyDeviceToHost, s));
    BIE_HIP_CHECK(hipStreamSynchronize(s));
    rn.assign(sm.pinned, sm.pinned + seg.S);
    fn.assign(sm.pinned + seg.S, sm.pinned + 2 * seg.S);
  }
  std::vector<double> itol_all(seg.S, 1.0);
  std::vector<char> retire(active.size(), 0);
  size_t k = 0;
  for (size_t i = 0; i < active.size(); ++i) {
    Request &r = *active[i];
    bool all = true;
    for (int j = 0; j < r.nrhs; ++j, ++k) {
      r.relres[j] = fn[k] > 0.0 ? rn[k] / fn[k] : 0.0;
      const bool c = r.relres[j] <= o.tol;
      all = all && c;
      // each cycle only has to bring the residual to what the outer tolerance needs
      // (margin 3); with float32 far fields never tighter than inner_tol
      itol_all[k] = c ? 1.0 : std::max(o.precision == BIE_MIXED ? o.inner_tol : 0.0,
                                       o.tol / (3.0 * r.relres[j]));
      if (c) BIE_HIP_CHECK(hipMemsetAsync(R + seg.h_off[k], 0, sizeof(double) * r.n, s));
    }
    if (all || r.cycles >= cfg.max_cycles) retire[i] = 1;
  }
  // ---- retire: results of converged requests go out before the next cycle --------------------
  std::vector<std::shared_ptr<Request>> keep;
  std::vector<long long> keep_old_off;
  std::vector<double> itol;
  k = 0;
  for (size_t i = 0; i < active.size(); ++i) {
    auto &r = active[i];
    if (!retire[i]) {
      keep.push_back(r);
      keep_old_off.push_back(off[i]);
      for (int j = 0; j < r->nrhs; ++j) itol.push_back(itol_all[k + j]);
      k += r->nrhs;
      continue;
    }
    k += r->nrhs;
    const int st = finish(*r, o, s);  // a failed read-off fails this request only
    double worst = 0.0;
    for (double v : r->relres) worst = std::max(worst, v);
    r->info.rel_residual = worst;
    complete(*r, st != BIE_OK ? st : (worst <= o.tol ? BIE_OK : BIE_ENOCONV));
  }
  active.swap(keep);
  if (active.empty()) return BIE_OK;
  // ---- one Arnoldi cycle on the residual of every remaining system ---------------------------
  const Layout L2 = layout(active, o);
  const std::vector<long long> &off2 = L2.off;
  std::vector<long long> lens2, starts2;
  for (size_t i = 0; i < active.size(); ++i)
    for (int j = 0; j < active[i]->nrhs; ++j) {
      lens2.push_back(active[i]->n);
      starts2.push_back(off2[i] + j * active[i]->n);
    }
  double *T = X;  // X is no longer needed this cycle: it holds the re-laid-out residual
  for (size_t i = 0; i < active.size(); ++i)
    BIE_HIP_CHECK(hipMemcpyAsync(T + off2[i], R + keep_old_off[i],
                                 sizeof(double) * active[i]->nrhs * active[i]->n,
                                 hipMemcpyDeviceToDevice, s));
  BIE_TRY(seg.build(lens2, s, &starts2));
  // right preconditioning of the cycle: GMRES on (A P) u = r, then d = P u (R, no longer read
  // this cycle, holds P u); one launch applies every item's blocks
  const PcBatchItem *pc_items = nullptr;
  size_t pc_lds = 0;
  long long pc_blocks = 0, pc_macs = 0;
  const int pc_n = (int)L2.items.size();
  if (o.precond == BIE_PRECOND_BLOCK) {
    std::vector<bie_geom *> gs;
    std::vector<int> kinds, nr;
    std::vector<long long> offs;
    for (const MultiItem &it : L2.items) {
      gs.push_back(it.g);
      kinds.push_back(it.kind);
      nr.push_back(it.nrhs);
      offs.push_back(it.io);
    }
    std::vector<PcBatchItem> pit;
    BIE_TRY(pc_batch_items(gs, kinds, nr, offs, pit, pc_lds, pc_blocks, pc_macs));
    BIE_TRY(pcitems.reserve(pit.size() * sizeof(PcBatchItem)));
    BIE_HIP_CHECK(hipMemcpyAsync(pcitems.ptr, pit.data(), pit.size() * sizeof(PcBatchItem),
                                 hipMemcpyHostToDevice, s));
    BIE_HIP_CHECK(hipStreamSynchronize(s));  // the host descriptors go out of scope
    pc_items = reinterpret_cast<const PcBatchItem *>(pcitems.ptr);
  }
  {
    const std::vector<MultiItem> mi = L2.items;
    // systems of item k: those of requests L2.first[k] .. L2.first[k+1]-1
    std::vector<int> sys0(active.size() + 1, 0);
    for (size_t i = 0; i < active.size(); ++i) sys0[i + 1] = sys0[i] + active[i]->nrhs;
    std::vector<int> first(mi.size() + 1, 0);
    for (size_t q = 0; q <= mi.size(); ++q) first[q] = sys0[L2.first[q]];
    SysSet *ssp = &ss;
    const long long N2 = L2.total;
    double *pu = R;
    ss.apply = [mi, planp, N2, first, ssp, pc_items, pc_n, pc_lds, pc_blocks, pc_macs, pu](
                   int precision, const double *in, double *out, hipStream_t st) {
      if (pc_items) {
        BIE_TRY(pc_apply_batch(pc_n, pc_items, pc_lds, pc_blocks, pc_macs, in, pu, st));
        in = pu;
      }
      std::vector<char> act(mi.size(), 1);
      if (!ssp->active.empty())
        for (size_t i = 0; i < mi.size(); ++i) {
          char a = 0;
          for (int q = first[i]; q < first[i + 1]; ++q) a |= ssp->active[q];
          act[i] = a;
        }
      return multi_apply(*planp, mi, act, precision, in, out, N2, st);
    };
  }
  int iters = 0, applies = 0;
  BIE_TRY(gmres_cycle(ss, o.precision, T, D, itol, m, iters, applies, s));
  if (pc_items)  // d = P u, in place (each body is staged before it is written)
    BIE_TRY(pc_apply_batch(pc_n, pc_items, pc_lds, pc_blocks, pc_macs, D, D, s));
  for (size_t i = 0; i < active.size(); ++i) {
    BIE_TRY(vec_axpby((long long)active[i]->nrhs * active[i]->n, 1.0, D + off2[i], 1.0,
                      active[i]->x, s));
    active[i]->cycles += 1;
  }
  std::lock_guard<std::mutex> lk(mu);
  ++n_cycles;
  return BIE_OK;
}

void bie_server::run() {
  (void)hipSetDevice(device);
  for (;;) {
    // ---- admission (arrival order, HBM footprint, system cap) ---------------------------------
    std::vector<std::shared_ptr<Request>> admitted;
    {
      std::unique_lock<std::mutex> lk(mu);
      cv_work.wait(lk, [&] { return stopping || !queue.empty() || !active.empty(); });
      if (stopping && queue.empty() && active.empty()) break;
      long long systems = 0;
      for (auto &r : active) systems += r->nrhs;
      while (!queue.empty()) {
        auto &r = queue.front();
        auto gu = geom_use.find(geom_key(*r));
        const long long gbytes = gu == geom_use.end() ? geom_footprint(cfg, r->g, r->kind) : 0;
        const bool alone = active.empty() && admitted.empty();
        const bool fits_mem = cfg.hbm_budget_bytes <= 0 ||
                              bytes_in_flight + r->bytes + gbytes <= cfg.hbm_budget_bytes || alone;
        const bool fits_sys = cfg.max_systems <= 0 || systems + r->nrhs <= cfg.max_systems || alone;
        if (!fits_mem || !fits_sys) break;
        bytes_in_flight += r->bytes + gbytes;
        auto &use = geom_use[geom_key(*r)];
        use.first += 1;
        use.second += gbytes;
        r->info.footprint_bytes = r->bytes + use.second;
        systems += r->nrhs;
        r->t_admit = Clock::now();
        admitted.push_back(r);
        queue.pop_front();
      }
      for (auto &r : admitted)
        r->info.inflight = (int)(active.size() + admitted.size());
      peak_bytes = std::max(peak_bytes, bytes_in_flight);
    }
    for (auto &r : admitted) {
      r->info.queue_s = std::chrono::duration<double>(r->t_admit - r->t_submit).count();
      const int rc = prepare(*r, cfg.opts, stream);
      if (rc != BIE_OK) {
        complete(*r, rc);
        continue;
      }
      active.push_back(r);
    }
    if (active.empty()) continue;
    std::stable_sort(active.begin(), active.end(),
                     [](const std::shared_ptr<Request> &a, const std::shared_ptr<Request> &b) {
                       return a->g != b->g ? a->g->gen < b->g->gen : a->kind < b->kind;
                     });
    const int rc = cycle();
    if (rc != BIE_OK) fail_active(rc);
  }
}

extern "C" {

int bie_server_create(const bie_server_config *cfg, bie_server **out) {
  if (!cfg || !out) {
    set_error("bie_server_create: NULL argument");
    return BIE_EINVAL;
  }
  if (cfg->max_cycles < 1 || check_opts(cfg->opts) != BIE_OK) {
    set_error("bie_server_create: invalid configuration");
    return BIE_EINVAL;
  }
  if (cfg->opts.l2_scaling) {
    set_error("bie_server_create: l2_scaling is supported by the single-geometry solves only");
    return BIE_EINVAL;
  }
  bie_server *srv = new (std::nothrow) bie_server();
  if (!srv) {
    set_error("host allocation failed");
    return BIE_ENOMEM;
  }
  srv->cfg = *cfg;
  // the worker's stream is made here, on the caller's current device: a server that cannot
  // use the device fails now instead of leaving later waits without a worker
  if (hipGetDevice(&srv->device) != hipSuccess || hipStreamCreate(&srv->stream) != hipSuccess) {
    set_error("bie_server_create: no usable HIP device (stream creation failed)");
    delete srv;
    return BIE_EDEVICE;
  }
  srv->worker = std::thread([srv] { srv->run(); });
  *out = srv;
  return BIE_OK;
}

int bie_server_submit(bie_server *srv, bie_geom *g, int kind, int nrhs, const double *in,
                      double *out, long long *ticket) {
  if (!srv || !g || (kind != 0 && kind != 1) || nrhs < 1 || !in || !out || !ticket) {
    set_error("bie_server_submit: invalid argument");
    return BIE_EINVAL;
  }
  auto r = std::make_shared<Request>();
  r->g = g;
  r->kind = kind;
  r->nrhs = nrhs;
  r->n = kind == 0 ? g->M : 2LL * g->M;
  const int width = kind == 0 ? g->N : 3 * g->N;
  r->in.assign(in, in + (size_t)nrhs * width);
  for (double v : r->in)
    if (!std::isfinite(v)) {
      set_error("bie_server_submit: non-finite charge, force or torque");
      return BIE_EINVAL;
    }
  r->out = out;
  r->bytes = footprint(srv->cfg, g, kind, nrhs);
  r->t_submit = Clock::now();
  {
    std::lock_guard<std::mutex> lk(srv->mu);
    if (srv->stopping) {
      set_error("bie_server_submit: server is stopping");
      return BIE_EINVAL;
    }
    r->id = srv->next_id++;
    srv->queue.push_back(r);
    srv->all[r->id] = r;
  }
  srv->cv_work.notify_one();
  *ticket = r->id;
  return BIE_OK;
}

int bie_server_wait(bie_server *srv, long long ticket, double timeout_s, bie_request_info *info) {
  if (!srv) {
    set_error("bie_server_wait: NULL server");
    return BIE_EINVAL;
  }
  std::unique_lock<std::mutex> lk(srv->mu);
  auto it = srv->all.find(ticket);
  if (it == srv->all.end()) {
    set_error("bie_server_wait: unknown ticket");
    return BIE_EINVAL;
  }
  auto r = it->second;
  auto pred = [&] { return r->done; };
  if (timeout_s < 0) {
    srv->cv_done.wait(lk, pred);
  } else if (!srv->cv_done.wait_for(lk, std::chrono::duration<double>(timeout_s), pred)) {
    set_error("bie_server_wait: timed out");
    return BIE_EINVAL;
  }
  if (info) *info = r->info;
  srv->all.erase(it);
  return r->info.status == BIE_ENOCONV ? BIE_OK : r->info.status;
}

int bie_server_stats(bie_server *srv, long long *requests, long long *solves, long long *cycles,
                     long long *peak_bytes) {
  if (!srv) {
    set_error("bie_server_stats: NULL server");
    return BIE_EINVAL;
  }
  std::lock_guard<std::mutex> lk(srv->mu);
  if (requests) *requests = srv->n_requests;
  if (solves) *solves = srv->n_solves;
  if (cycles) *cycles = srv->n_cycles;
  if (peak_bytes) *peak_bytes = srv->peak_bytes;
  return BIE_OK;
}

int bie_server_inject_failure(bie_server *srv, int cycles) {
  if (!srv || cycles < 0) {
    set_error("bie_server_inject_failure: NULL server or negative count");
    return BIE_EINVAL;
  }
  std::lock_guard<std::mutex> lk(srv->mu);
  srv->inject_fail = cycles;
  return BIE_OK;
}

int bie_server_destroy(bie_server *srv) {
  if (!srv) return BIE_OK;
  {
    std::lock_guard<std::mutex> lk(srv->mu);
    srv->stopping = true;
  }
  srv->cv_work.notify_all();
  if (srv->worker.joinable()) srv->worker.join();
  if (srv->stream) (void)hipStreamDestroy(srv->stream);
  srv->seg.buf.release();
  srv->sm.release();
  srv->flat.release();
  srv->pcitems.release();
  bie::multi_destroy(srv->plan);
  delete srv;
  return BIE_OK;
}

}  // extern "C"
