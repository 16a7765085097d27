// Restarted GMRES in float64 (classical Gram-Schmidt applied twice) over a set of independent
// systems that advance in lock step and share one batched operator apply per Arnoldi step, and
// float64 iterative refinement around a float32 far-field apply (BIE_MIXED).
//
// Device: Krylov basis V [m+1][Ntot] (all systems back to back), applies, dot products, updates.
// Host: one (m+1) x m Hessenberg matrix per system (its new column is read back once per step,
// while the next step already runs on the device), Givens rotations, triangular solves. The true residual ||f - A x|| / ||f|| with the float64
// operator decides convergence at the end of every cycle. The paper iterates GMRES to a
// relative residual of 1e-6 with unstated restart details; x0 = 0 and CGS2 are choices made here.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "internal.h"

namespace bie {
namespace {

// BIE_VERBOSE=1: one line per GMRES cycle and refinement step; =2: also every Arnoldi step.
int verbosity() {
  static int v = [] {
    const char *e = std::getenv("BIE_VERBOSE");
    return e ? std::atoi(e) : 0;
  }();
  return v;
}

struct Stats {
  int iters = 0, applies64 = 0, applies32 = 0;
  long long pairs = 0;
};

int apply(SysSet &ss, int precision, const double *in, double *out, Stats &st, hipStream_t s) {
  BIE_TRY(ss.apply(precision, in, out, s));
  if (precision != BIE_FP64) st.applies32 += 1; else st.applies64 += 1;  // (per group: some f32)
  st.pairs += ss.pairs_per_apply;
  return BIE_OK;
}

int read_host(SolverMem &mem, const double *dev, size_t count, std::vector<double> &dst,
              hipStream_t s) {
  BIE_TRY(mem.ensure_pinned(count * sizeof(double)));
  BIE_HIP_CHECK(hipMemcpyAsync(mem.pinned, dev, count * sizeof(double), hipMemcpyDeviceToHost, s));
  BIE_HIP_CHECK(hipStreamSynchronize(s));
  dst.assign(mem.pinned, mem.pinned + count);
  return BIE_OK;
}

int write_dev(SolverMem &mem, double *dev, const std::vector<double> &src, hipStream_t s) {
  BIE_TRY(mem.ensure_pinned(src.size() * sizeof(double)));
  BIE_HIP_CHECK(hipStreamSynchronize(s));  // the pinned buffer may still feed an earlier copy
  std::memcpy(mem.pinned, src.data(), src.size() * sizeof(double));
  BIE_HIP_CHECK(hipMemcpyAsync(dev, mem.pinned, src.size() * sizeof(double), hipMemcpyHostToDevice, s));
  BIE_HIP_CHECK(hipStreamSynchronize(s));
  return BIE_OK;
}

// Waits until the kernel of an Arnoldi step has stored `tag` in all S flag words (mapped host
// memory, written after the column). After every 2 ms without them the stream is queried (a
// step normally takes far less): an error is returned as such, and a stream that is idle while
// a flag is still missing is an error too.
int wait_column(const double *flags, int S, unsigned long long tag, hipStream_t s) {
  const volatile unsigned long long *f = reinterpret_cast<const volatile unsigned long long *>(flags);
  auto ready = [&]() {
    for (int r = 0; r < S; ++r)
      if (f[r] != tag) return false;
    return true;
  };
  using clk = std::chrono::steady_clock;
  auto last = clk::now();
  for (unsigned spin = 1;; ++spin) {
    if (ready()) break;
    if ((spin & 1023) == 0 && clk::now() - last > std::chrono::milliseconds(2)) {
      last = clk::now();
      const hipError_t e = hipStreamQuery(s);
      if (e == hipSuccess) {
        if (ready()) break;
        set_error("Arnoldi step finished without its Hessenberg column");
        return BIE_EDEVICE;
      }
      if (e != hipErrorNotReady) BIE_HIP_CHECK(e);
    }
  }
  std::atomic_thread_fence(std::memory_order_acquire);
  return BIE_OK;
}

struct Work {
  double *V, *w, *r, *U;      // V [(m+1)][Ntot]; w (= A U), r, U (the next candidate) [Ntot]
  double *y, *nrm;            // [S][m+2], [S]
  double *h1, *zero;          // one-pass steps: coefficients, and zeros (the absent second pass)
  double *G, *sc, *cc, *inu;  // DCGS2 coefficients: [S][m+2] x3, [S]
  double *raw;                // per-system reductions [S][2m+4]
  double *Hd;                 // device copy of the Hessenberg matrices [S][(m+2)(m+1)]
  double *scratch;            // partial sums [2m+4][C]
  long long hs = 0, rstride = 0, ldh = 0, hstride = 0;
};

// Arnoldi steps: DCGS2 (two passes over the basis, the column finished one step late) for the
// float64 operator; one classical Gram-Schmidt pass for the float32-apply inner solves of the
// mixed mode, which only reach about 1e-6 and whose result the float64 refinement residual
// checks (the late column of DCGS2 would cost them one more apply per cycle).
bool one_pass(int precision) { return precision == BIE_MIXED; }

int make_work(SysSet &ss, int m, Work &wk, int extra_vectors, double **extra, hipStream_t st) {
  const size_t N = (size_t)ss.seg->Ntot;
  const int S = ss.seg->S;
  BIE_TRY(ss.mem->big.reserve(((size_t)(m + 1) + 3 + extra_vectors) * N * sizeof(double) + 64));
  double *p = ss.mem->big.as<double>();
  wk.V = p;
  p += (size_t)(m + 1) * N;
  wk.w = p;
  p += N;
  wk.r = p;
  p += N;
  wk.U = p;
  p += N;
  for (int e = 0; e < extra_vectors; ++e) {
    extra[e] = p;
    p += N;
  }
  wk.hs = m + 2;
  wk.rstride = 2 * (long long)m + 4;
  wk.ldh = m + 2;
  wk.hstride = wk.ldh * (m + 1);
  const size_t hs = (size_t)wk.hs;
  const size_t np = (size_t)wk.rstride * (size_t)ss.seg->C;
  const size_t small = (6 * hs + 2) * S + (size_t)wk.rstride * S + (size_t)wk.hstride * S + np;
  BIE_TRY(ss.mem->small.reserve(small * sizeof(double) + 64));
  double *q = ss.mem->small.as<double>();
  auto take = [&](size_t n) {
    double *r = q;
    q += n;
    return r;
  };
  wk.y = take(hs * S);
  wk.G = take(hs * S);
  wk.sc = take(hs * S);
  wk.cc = take(hs * S);
  wk.nrm = take(S);
  wk.inu = take(S);
  wk.raw = take((size_t)wk.rstride * S);
  wk.Hd = take((size_t)wk.hstride * S);
  wk.h1 = take(hs * S);
  wk.zero = take(hs * S);
  wk.scratch = take(np);
  // written once here, never by a step (kernels only read it)
  BIE_HIP_CHECK(hipMemsetAsync(wk.zero, 0, hs * S * sizeof(double), st));
  return BIE_OK;
}

// GMRES(m) on A x = f for every system. x holds the iterate on exit (x0 = 0 if x_is_zero).
// With relaxed (and precision BIE_MIXED): float64 GMRES whose Arnoldi steps apply the float32
// operator once every active system's estimated relative residual is below tol / eta, eta the
// relative error of that apply (the apply error a step may carry grows as the residual it
// reduces falls, Simoncini & Szyld 2003); earlier steps and every cycle's true residual use
// float64. Per group of systems (ss.group_ptr), with the group's eta (ss.group_eta).
constexpr double kF32ApplyError = 1e-6;  // eta where the set gives none


int gmres(SysSet &ss, int precision, const double *f, double *x, bool x_is_zero,
          const std::vector<double> &tol, int m, int max_iter, Work &wk, Stats &st,
          std::vector<double> &relres, std::vector<int> &conv, hipStream_t s,
          int max_cycles = 1 << 30, bool relaxed = false) {
  const Segments &sg = *ss.seg;
  SolverMem &mem = *ss.mem;
  const int S = sg.S;
  const long long N = sg.Ntot;
  const long long hs = m + 2;
  std::vector<double> fnorm, beta;
  if (x_is_zero) BIE_HIP_CHECK(hipMemsetAsync(x, 0, sizeof(double) * N, s));
  BIE_TRY(seg_nrm2(sg, f, wk.nrm, wk.scratch, s));
  // pinned host memory of a cycle: two column slots (the S columns, then one flag word per
  // system), the tag base, (from x = 0) the norms of f, and the staging of the coefficients y
  const size_t slot = (size_t)S * hs + S, fn_at = 2 * slot + 1, y_at = fn_at + S;
  BIE_TRY(mem.ensure_pinned((y_at + (size_t)S * hs) * sizeof(double)));
  // From x = 0 the first cycle starts from r = f without a host round trip: its Givens
  // recurrence runs on f / ||f|| (beta 1, relative residuals directly), and the norms, copied to
  // pinned memory behind the norm kernel, are read once the cycle's steps are complete, to scale
  // its coefficients y. Every system then starts active (a zero f gives V_0 = 0 and a zero
  // correction); with a tolerance of 1 or more a system would start converged, and its device
  // norm would have to be cleared from the host: those calls read the norms first.
  bool defer = x_is_zero;
  for (int r = 0; r < S; ++r) defer = defer && tol[r] < 1.0;
  bool fn_pending = false;
  if (defer) {
    BIE_HIP_CHECK(hipMemcpyAsync(mem.pinned + fn_at, wk.nrm, S * sizeof(double),
                                 hipMemcpyDeviceToHost, s));
    fnorm.assign(S, 1.0);
    fn_pending = true;
  } else {
    BIE_TRY(read_host(mem, wk.nrm, S, fnorm, s));
  }
  relres.assign(S, 0.0);
  conv.assign(S, 0);
  std::vector<char> done(S, 0);  // converged systems stay converged (their x no longer changes)
  bool first = true;
  int cycles = 0;
  std::vector<double> H((size_t)S * (m + 1) * m), cs((size_t)S * m), sn((size_t)S * m),
      gv((size_t)S * (m + 1));
  const int ngroups = relaxed && ss.group_ptr.size() >= 2 &&
                              (int)ss.group_ptr.size() - 1 <= kMaxPrecGroups
                          ? (int)ss.group_ptr.size() - 1
                          : 1;
  std::vector<int> group_of(S, 0);
  if (ngroups > 1)
    for (int q = 0; q < ngroups; ++q)
      for (int r = ss.group_ptr[q]; r < ss.group_ptr[q + 1]; ++r) group_of[r] = q;
  std::vector<char> gf32(ngroups, 0);
  std::vector<double> geta(ngroups, kF32ApplyError);
  for (int q = 0; q < ngroups; ++q)
    if (!ss.group_eta.empty())
      geta[q] = ngroups == 1 ? *std::max_element(ss.group_eta.begin(), ss.group_eta.end())
                             : ss.group_eta[q];
  while (cycles < max_cycles) {
    ++cycles;
    // the first cycle from x = 0 starts from r = f, whose norms wk.nrm already holds
    const bool from_f = first && x_is_zero;
    if (from_f) {
      beta = fnorm;
    } else {
      BIE_TRY(apply(ss, relaxed ? BIE_FP64 : precision, x, wk.r, st, s));
      BIE_TRY(vec_axpby(N, 1.0, f, -1.0, wk.r, s));
      BIE_TRY(seg_nrm2(sg, wk.r, wk.nrm, wk.scratch, s));
      BIE_TRY(read_host(mem, wk.nrm, S, beta, s));
    }
    first = false;
    std::vector<int> active(S, 0);
    int nact = 0;
    for (int r = 0; r < S; ++r) {
      if (!done[r]) relres[r] = fnorm[r] > 0.0 ? beta[r] / fnorm[r] : 0.0;
      conv[r] = done[r] || relres[r] <= tol[r];
      done[r] = conv[r];
      active[r] = !conv[r];
      nact += active[r];
    }
    ss.active.assign(active.begin(), active.end());  // later applies skip converged systems
    if (verbosity() >= 1)
      std::fprintf(stderr, "[bie] gmres prec=%d cycle start: iters=%d active=%d true rel res[0]=%.3e\n",
                   precision, st.iters, nact, relres[0]);
    if (nact == 0 || st.iters >= max_iter) break;
    bool zeroed = false;  // the device norms change only where a converged system had one
    for (int r = 0; r < S; ++r)
      if (!active[r]) {
        zeroed = zeroed || beta[r] != 0.0;
        beta[r] = 0.0;
      }
    if (zeroed) BIE_TRY(write_dev(mem, wk.nrm, beta, s));
    BIE_TRY(seg_scale_to(sg, from_f ? f : wk.r, wk.nrm, wk.V, s));
    std::fill(gv.begin(), gv.end(), 0.0);
    for (int r = 0; r < S; ++r) gv[(size_t)r * (m + 1)] = beta[r];
    std::vector<int> jdone(S, -1);
    int jend = -1;
    // Arnoldi step j: apply, CGS2 against V_0..V_j, V_{j+1} = w / ||w||, and the new Hessenberg
    // column, written by the last kernel into pinned slot j % 2. Steps run one ahead of the
    // host: step j+1 is queued before the host waits for step j's column (a cycle that stops at
    // step j leaves step j+1's work unused).
    // pinned: the two column slots, then the tag base of this cycle (step j stores the tag of
    // base + j + 1; its kernels read the base when they run). The base is written before the
    // cycle's first step, when no earlier step is in flight: a later cycle starts after the
    // host read of its true residual (a stream synchronisation), and every caller synchronises
    // the stream between two calls of this function (a solve ends with one; the serving loop
    // and the refinement read a residual norm in between). The norms of f behind the base, if
    // pending, stay untouched.
    BIE_TRY(mem.ensure_pinned((2 * slot + 1) * sizeof(double)));
    volatile unsigned long long *base_h =
        reinterpret_cast<volatile unsigned long long *>(mem.pinned + 2 * slot);
    const unsigned long long *base_d =
        reinterpret_cast<const unsigned long long *>(mem.pinned_dev + 2 * slot);
    const unsigned long long base = mem.seq;
    *base_h = base;
    std::atomic_thread_fence(std::memory_order_seq_cst);
    mem.seq += (unsigned long long)m + 1;
    unsigned long long seqv[2] = {0, 0};
    // The launches of Arnoldi step j (DCGS2; their arguments depend only on j and the solver's
    // buffers). Step 0: U = A V_0 - (V_0.A V_0) V_0 (the first projection of the first
    // candidate). Step j in 1..m-1: Z = A U; the reductions; column j - 1 finished and written
    // to pinned slot (j - 1) % 2 with its flag; V_j and the next candidate U. Step m (the end of
    // a full cycle) only finishes column m - 1 (no apply).
    // One-pass steps: step j (0..m-1) applies A to V_j, projects once and writes V_{j+1} and
    // column j. Either way column c goes to pinned slot c % 2 with the tag of base + c + 1.
    const bool onep = one_pass(precision) && !relaxed;
    // relaxed: per group of systems (batch items; else all systems), the largest estimated
    // relative residual over tolerance of its systems still iterating (after the last column
    // the host has seen) decides the precision of the group's apply when a step is queued
    std::vector<double> gworst(ngroups, 0.0);
    for (int r = 0; r < S; ++r)
      if (active[r]) gworst[group_of[r]] = std::max(gworst[group_of[r]], relres[r] / tol[r]);
    const int lag = onep ? 0 : 1;       // column c comes from step c + lag
    const int last_step = onep ? m - 1 : m;
    auto step_body = [&](int j, Stats &sts, hipStream_t s, int sp) -> int {
      if (onep) {
        BIE_TRY(apply(ss, sp, wk.V + (size_t)j * N, wk.w, sts, s));
        BIE_TRY(seg_dots(sg, j + 1, wk.V, N, wk.w, wk.h1, hs, wk.scratch, s));
        double *col = mem.pinned_dev + (j & 1) * slot;
        auto *flag = reinterpret_cast<unsigned long long *>(col + (size_t)S * hs);
        return seg_combination_column(sg, j + 1, wk.V, N, wk.zero, wk.h1, hs, wk.w, wk.nrm,
                                      wk.V + (size_t)(j + 1) * N, col, flag, base_d,
                                      (unsigned long long)j + 1, wk.scratch, s);
      }
      if (j == 0) {
        BIE_TRY(apply(ss, sp, wk.V, wk.U, sts, s));
        BIE_TRY(seg_dots(sg, 1, wk.V, N, wk.U, wk.G, hs, wk.scratch, s));
        BIE_TRY(seg_combination(sg, 1, wk.V, N, wk.G, hs, wk.U, -1.0, s));
        return BIE_OK;
      }
      const bool fin = j == m;
      if (!fin) BIE_TRY(apply(ss, sp, wk.U, wk.w, sts, s));
      BIE_TRY(dcgs_dots(sg, j, wk.V, N, wk.U, fin ? nullptr : wk.w, wk.raw, wk.rstride,
                        wk.scratch, s));
      double *col = mem.pinned_dev + ((j - 1) & 1) * slot;
      auto *flag = reinterpret_cast<unsigned long long *>(col + (size_t)S * hs);
      BIE_TRY(dcgs_small(S, j, fin, wk.raw, wk.rstride, wk.G, wk.Hd, wk.ldh, wk.hstride, wk.sc,
                         wk.cc, wk.inu, hs, col, flag, base_d, (unsigned long long)j, s));
      if (!fin)
        BIE_TRY(dcgs_update(sg, j, wk.V, N, wk.sc, wk.cc, wk.inu, hs, wk.U, wk.w,
                            wk.V + (size_t)j * N, s));
      return BIE_OK;
    };
    // With graphs: step j is captured (after running it once eagerly, which sizes every buffer)
    // and replayed in later cycles and solves of the same configuration; a change of the
    // configuration or any buffer reallocation drops the captured steps.
    const bool use_graphs = graphs_enabled() && !ss.graph_key.empty();
    std::string gkey;
    if (use_graphs) {
      char buf[256];
      std::snprintf(buf, sizeof buf, "|m%d|o%d|S%d|N%lld|%p|%p|%p|%p|%p|%p|%p|%p", m, (int)onep, S, N,
                    (void *)wk.V, (void *)wk.w, (void *)wk.U, (void *)wk.G, (void *)wk.Hd,
                    (void *)wk.scratch, (void *)mem.pinned_dev, (void *)sg.c0);
      gkey = ss.graph_key + buf;
    }
    auto step = [&](int j) -> int {
      const int c = j - lag;  // the column this step finishes (none for the first DCGS2 step)
      if (c >= 0) seqv[c & 1] = column_tag(base + (unsigned long long)c + 1);
      int sp = precision;
      if (relaxed) {
        int nf = 0;
        for (int q = 0; q < ngroups; ++q) nf += gf32[q] = gworst[q] * geta[q] < 1.0;
        sp = nf == ngroups ? BIE_MIXED : nf == 0 ? BIE_FP64 : kPrecPerGroup;
        if (sp == kPrecPerGroup) ss.group_f32 = gf32;
      }
      if (!use_graphs || sp == kPrecPerGroup || (!onep && j == m)) return step_body(j, st, s, sp);
      StepGraphs &gr = mem.graphs[sp == BIE_MIXED ? 1 : 0];
      if (gr.key != gkey || gr.epoch != buffer_epoch()) {
        gr.clear();
        gr.key = gkey;
        gr.epoch = buffer_epoch();
      }
      if (j < (int)gr.exec.size() && gr.exec[j]) {
        BIE_HIP_CHECK(hipGraphLaunch(gr.exec[j], s));
        if (sp == BIE_MIXED) st.applies32 += 1; else st.applies64 += 1;  // (j < m)
        st.pairs += ss.pairs_per_apply;
        ++mem.graph_replays;
        return BIE_OK;
      }
      BIE_TRY(step_body(j, st, s, sp));
      if (gr.epoch != buffer_epoch()) {  // the eager step allocated: earlier captures are stale
        gr.clear();
        gr.key = gkey;
        gr.epoch = buffer_epoch();
      }
      if (!mem.cap) BIE_HIP_CHECK(hipStreamCreateWithFlags(&mem.cap, hipStreamNonBlocking));
      hipGraph_t graph = nullptr;
      BIE_HIP_CHECK(hipStreamBeginCapture(mem.cap, hipStreamCaptureModeThreadLocal));
      Stats dummy;
      int rc;
      {
        ProfSuspend quiet;  // no profiling events inside a captured step
        rc = step_body(j, dummy, mem.cap, sp);
      }
      const hipError_t e = hipStreamEndCapture(mem.cap, &graph);
      if (rc != BIE_OK || e != hipSuccess || !graph) {
        if (graph) (void)hipGraphDestroy(graph);
        if (rc == BIE_OK) set_error(std::string("graph capture of an Arnoldi step failed: ") +
                                    hipGetErrorString(e));
        return rc != BIE_OK ? rc : BIE_EDEVICE;
      }
      hipGraphExec_t exec = nullptr;
      const hipError_t ei = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
      (void)hipGraphDestroy(graph);
      if (ei != hipSuccess) {
        set_error(std::string("graph instantiation of an Arnoldi step failed: ") +
                  hipGetErrorString(ei));
        return BIE_EDEVICE;
      }
      if ((int)gr.exec.size() <= j) gr.exec.resize(j + 1, nullptr);
      gr.exec[j] = exec;
      ++mem.graph_captures;
      return BIE_OK;
    };
    // Column j comes from step j + lag; step j + lag + 1 is queued before the host waits for it,
    // unless column j is expected to end the cycle: the largest estimated residual over
    // tolerance, extrapolated from the last two columns at their rate of decrease (no faster
    // than the last step), is at most kHoldRatio. Then the step is queued only once column j
    // shows it is needed (the device idles for the host's round trip, a few tens of
    // microseconds), and a step whose work the converged cycle would discard is not run.
    constexpr double kHoldRatio = 2.0;
    double wlast = -1.0, wlast2 = -1.0;  // that ratio for the last two columns
    for (int k = 0; k <= lag; ++k) BIE_TRY(step(k));
    for (int j = 0; j < m; ++j) {
      st.iters += 1;
      const bool more = j + lag + 1 <= last_step && st.iters < max_iter;
      const bool hold = more && wlast > 0.0 && wlast2 > 0.0 &&
                        wlast * std::min(1.0, wlast / wlast2) <= kHoldRatio;
      if (more && !hold) BIE_TRY(step(j + lag + 1));
      BIE_TRY(wait_column(mem.pinned + (j & 1) * slot + (size_t)S * hs, S, seqv[j & 1], s));
      const double *hh2 = mem.pinned + (j & 1) * slot;
      bool all_done = true;
      std::fill(gworst.begin(), gworst.end(), 0.0);
      for (int r = 0; r < S; ++r) {
        if (!active[r] || jdone[r] >= 0) continue;
        double *Hc = &H[((size_t)r * (m + 1)) * m];  // column-major (m+1) x m
        double *col = Hc + (size_t)j * (m + 1);
        for (int i = 0; i <= j + 1; ++i) col[i] = hh2[(size_t)r * hs + i];
        const double hn = col[j + 1];
        double *c = &cs[(size_t)r * m], *sv = &sn[(size_t)r * m], *gg = &gv[(size_t)r * (m + 1)];
        for (int i = 0; i < j; ++i) {
          const double a = col[i], b = col[i + 1];
          col[i] = c[i] * a + sv[i] * b;
          col[i + 1] = -sv[i] * a + c[i] * b;
        }
        const double a = col[j], b = col[j + 1];
        const double den = std::hypot(a, b);
        c[j] = den > 0.0 ? a / den : 1.0;
        sv[j] = den > 0.0 ? b / den : 0.0;
        col[j] = den;
        col[j + 1] = 0.0;
        gg[j + 1] = -sv[j] * gg[j];
        gg[j] = c[j] * gg[j];
        const double res = std::fabs(gg[j + 1]) / fnorm[r];
        gworst[group_of[r]] = std::max(gworst[group_of[r]], res / tol[r]);
        if (verbosity() >= 2 && r == 0)
          std::fprintf(stderr, "[bie]   j=%d est rel res=%.3e hn=%.3e\n", j, res, hn);
        if (res <= tol[r] || hn == 0.0) jdone[r] = j;
        else all_done = false;
      }
      jend = j;
      if (all_done || st.iters >= max_iter) break;
      if (hold) BIE_TRY(step(j + lag + 1));
      wlast2 = wlast;
      wlast = *std::max_element(gworst.begin(), gworst.end());
    }
    // No stream synchronisation here: the last column's flag shows that every step whose basis
    // vectors y combines has run (a step queued ahead writes only the next column slot, the
    // next basis vector and candidate), and that the copy of the norms of f, queued before the
    // first step, is complete.
    // the first cycle from f ran on f / ||f||: its coefficients scale by ||f||
    std::vector<double> yscale(S, 1.0);
    if (fn_pending) {
      for (int r = 0; r < S; ++r) fnorm[r] = yscale[r] = mem.pinned[fn_at + r];
      fn_pending = false;
    }
    // y = H^{-1} g (upper triangular), x += V y
    const int nv = jend + 1;
    std::vector<double> yv((size_t)S * hs, 0.0);
    for (int r = 0; r < S; ++r) {
      if (!active[r]) continue;
      const int k = (jdone[r] >= 0 ? jdone[r] : jend) + 1;
      const double *Hc = &H[((size_t)r * (m + 1)) * m];
      const double *gg = &gv[(size_t)r * (m + 1)];
      double *yr = &yv[(size_t)r * hs];
      for (int i = k - 1; i >= 0; --i) {
        double acc = gg[i];
        for (int l = i + 1; l < k; ++l) acc -= Hc[(size_t)l * (m + 1) + i] * yr[l];
        const double d = Hc[(size_t)i * (m + 1) + i];
        yr[i] = d != 0.0 ? acc / d : 0.0;
      }
      for (int i = 0; i < k; ++i) yr[i] *= yscale[r];
    }
    // y to the device through its own pinned area: the previous copy from it is complete, as it
    // was queued on this stream before this cycle's steps, whose columns the host has seen
    std::memcpy(mem.pinned + y_at, yv.data(), yv.size() * sizeof(double));
    BIE_HIP_CHECK(hipMemcpyAsync(wk.y, mem.pinned + y_at, yv.size() * sizeof(double),
                                 hipMemcpyHostToDevice, s));
    BIE_TRY(seg_combination(sg, nv, wk.V, N, wk.y, hs, x, 1.0, s));
  }
  return BIE_OK;
}

}  // namespace

// The BIE_MIXED apply's relative error (2-norm, random densities, against the float64 direct
// apply), from measurements on the 1000-starfish and 200-ellipse geometries: direct float32 far
// field 2.4e-8 .. 4.4e-8 (taken as 1e-7); FMM Laplace with float32 expansions and near field
// 2.6e-7 .. 3.1e-7 at 24 terms, set by the float32 rounding (taken as 5e-7: on the preconditioned
// 1000-starfish solve one more of the 12 steps runs in float32 than with 1e-6, same accuracy);
// FMM Stokes with float64 expansions and the float32 near field (4.3e-7 on the 200 ellipses):
// the larger of the same rounding level and ten
// times the fitted truncation error 4.3e-2 * 0.45^terms (which alone measured 1.4e-10 .. 2.0e-10
// at 24 terms, 0.8e-7 .. 1.2e-7 at 16). A value set too large only delays the switch; one too
// small can cost a further restart cycle, never accuracy (the solve stops on float64 true
// residuals).
double mixed_apply_error(const bie_geom *g, int kind, int method, int order) {
  if (!method_is_fmm(method, g->M)) return 1e-7;
  const int terms = fmm_length(order, BIE_MIXED);
  const double trunc = ((kind & 1) ? 4.3e-2 : 2.1e-3) * std::pow(0.45, terms);
  return std::max(5e-7, 10.0 * trunc);
}

// One Arnoldi cycle (at most m steps, x0 = 0) on A d = r for every system, each system stopping
// at its own relative tolerance; d receives the correction. Used by the serving loop.
int gmres_cycle(SysSet &ss, int precision, const double *r, double *d,
                const std::vector<double> &tol, int m, int &iters, int &applies, hipStream_t s) {
  Work wk;
  BIE_TRY(make_work(ss, m, wk, 0, nullptr, s));
  Stats st;
  std::vector<double> relres;
  std::vector<int> conv;
  BIE_TRY(gmres(ss, precision, r, d, true, tol, m, 1 << 30, wk, st, relres, conv, s, 1));
  iters += st.iters;
  applies += st.applies32 + st.applies64;
  return BIE_OK;
}

int SolverMem::ensure_pinned(size_t bytes) {
  if (pinned_bytes >= bytes) return BIE_OK;
  if (pinned) {
    BIE_HIP_CHECK(hipDeviceSynchronize());  // no kernel or copy may still use the old buffer
    BIE_HIP_CHECK(hipHostFree(pinned));
    pinned = nullptr;
    pinned_dev = nullptr;
    pinned_bytes = 0;
  }
  size_t want = std::max<size_t>(bytes, 1 << 16);
  // mapped and coherent: kernels write Hessenberg columns into it directly, each followed by a
  // flag word that tells the host the column is complete
  if (hipHostMalloc((void **)&pinned, want, hipHostMallocMapped | hipHostMallocCoherent) !=
      hipSuccess) {
    set_error("pinned host allocation failed");
    return BIE_ENOMEM;
  }
  BIE_HIP_CHECK(hipHostGetDevicePointer((void **)&pinned_dev, pinned, 0));
  pinned_bytes = want;
  return BIE_OK;
}

void StepGraphs::clear() {
  for (hipGraphExec_t e : exec)
    if (e) (void)hipGraphExecDestroy(e);
  exec.clear();
  key.clear();
}

void SolverMem::release() {
  graphs[0].clear();
  graphs[1].clear();
  if (cap) (void)hipStreamDestroy(cap);
  cap = nullptr;
  big.release();
  small.release();
  if (pinned) (void)hipHostFree(pinned);
  pinned = nullptr;
  pinned_dev = nullptr;
  pinned_bytes = 0;
}

// Solves every system of ss to o.tol (relative, float64 operator). relres_out gets the final true
// relative residual per system.
int solve_systems(SysSet &ss, const bie_opts &o, const double *f, double *x,
                  std::vector<double> &relres_out, bie_info *info, hipStream_t s) {
  const int m = std::max(1, std::min(o.restart, 1000));
  const int S = ss.seg->S;
  const long long N = ss.seg->Ntot;
  Stats st;
  std::vector<double> relres;
  std::vector<int> conv;
  Work wk;
  double *extra[2] = {nullptr, nullptr};
  const bool mixed = o.precision == BIE_MIXED;
  BIE_TRY(make_work(ss, m, wk, mixed ? 2 : 0, extra, s));
  int refinements = 0;
  if (!mixed || o.mixed_strategy == BIE_MIXED_RELAXED) {
    BIE_TRY(gmres(ss, mixed ? BIE_MIXED : BIE_FP64, f, x, true, std::vector<double>(S, o.tol), m,
                  o.max_iter, wk, st, relres, conv, s, 1 << 30, mixed));
  } else {
    // x = 0, r = f; repeat: solve A32 d = r to what the outer tolerance needs; x += d; r = f - A64 x
    double *rr = extra[0], *d = extra[1];
    std::vector<double> fnorm, rn;
    BIE_HIP_CHECK(hipMemsetAsync(x, 0, sizeof(double) * N, s));
    BIE_TRY(seg_nrm2(*ss.seg, f, wk.nrm, wk.scratch, s));
    BIE_TRY(read_host(*ss.mem, wk.nrm, S, fnorm, s));
    BIE_HIP_CHECK(hipMemcpyAsync(rr, f, sizeof(double) * N, hipMemcpyDeviceToDevice, s));
    relres.assign(S, 1.0);
    conv.assign(S, 0);
    ss.active.assign(S, 1);
    for (int it = 0;; ++it) {
      BIE_TRY(seg_nrm2(*ss.seg, rr, wk.nrm, wk.scratch, s));
      BIE_TRY(read_host(*ss.mem, wk.nrm, S, rn, s));
      bool all = true;
      double worst = 0.0;
      for (int r = 0; r < S; ++r) {
        if (!conv[r]) relres[r] = fnorm[r] > 0.0 ? rn[r] / fnorm[r] : 0.0;
        conv[r] = conv[r] || relres[r] <= o.tol;
        all = all && conv[r];
        if (!conv[r]) worst = std::max(worst, relres[r]);
      }
      if (verbosity() >= 1)
        std::fprintf(stderr, "[bie] refinement %d: worst true rel res=%.3e iters=%d\n", it, worst,
                     st.iters);
      if (all || it >= o.max_refine || st.iters >= o.max_iter) break;
      // converged systems get a zero residual so the inner solve leaves them untouched
      for (int r = 0; r < S; ++r)
        if (conv[r])
          BIE_HIP_CHECK(hipMemsetAsync(rr + ss.seg->h_off[r], 0,
                                       sizeof(double) * (ss.seg->h_off[r + 1] - ss.seg->h_off[r]), s));
      // each inner solve only has to bring its residual to what the outer tolerance needs
      // (with a margin of 3), never tighter than inner_tol; per system, so that a system's
      // iterates do not depend on the rest of the batch
      std::vector<double> itol(S);
      for (int r = 0; r < S; ++r)
        itol[r] = conv[r] ? 1.0 : std::max(o.inner_tol, o.tol / (3.0 * relres[r]));
      std::vector<double> irel;
      std::vector<int> iconv;
      BIE_TRY(gmres(ss, BIE_MIXED, rr, d, true, itol, m, o.max_iter, wk, st, irel, iconv, s));
      BIE_TRY(vec_axpby(N, 1.0, d, 1.0, x, s));
      ss.active.resize(S);
      for (int r = 0; r < S; ++r) ss.active[r] = !conv[r];
      BIE_TRY(apply(ss, BIE_FP64, x, rr, st, s));
      BIE_TRY(vec_axpby(N, 1.0, f, -1.0, rr, s));
      ++refinements;
    }
  }
  bool ok = true;
  double worst = 0.0;
  for (int r = 0; r < S; ++r) {
    ok = ok && conv[r];
    worst = std::max(worst, relres[r]);
  }
  relres_out = relres;
  if (info) {
    info->iters = st.iters;
    info->refinements = refinements;
    info->applies_fp64 = st.applies64;
    info->applies_fp32 = st.applies32;
    info->rel_residual = worst;
    info->pairs = st.pairs;
  }
  if (!ok) {
    set_error("GMRES did not reach the tolerance within max_iter / max_refine");
    return BIE_ENOCONV;
  }
  return BIE_OK;
}

// One geometry, nrhs systems of length n = M (kinds 0, 2) or 2M (kinds 1, 3).
int solve_system(bie_geom *g, int kind, const bie_opts &o, int nrhs, const double *f, double *x,
                 bie_info *info, hipStream_t s) {
  const long long n = (kind & 1) ? 2LL * g->M : g->M;
  if (g->seg_nrhs != nrhs || g->seg_len != n) {
    BIE_TRY(g->seg.build(std::vector<long long>(nrhs, n), s));
    g->seg_nrhs = nrhs;
    g->seg_len = n;
  }
  SysSet ss;
  ss.seg = &g->seg;
  ss.mem = &g->sm;
  ss.pairs_per_apply = (long long)nrhs * g->M * (long long)g->M;
  const int method = o.method;
  {
    char key[160];
    std::snprintf(key, sizeof key, "g%llu|k%d|m%d|r%d|o%d|l%d|s%d|p%d|%p|%p", g->gen, kind,
                  method, nrhs, g->fmm_order, g->fmm_leaf, o.l2_scaling, o.precond,
                  (void *)g->ws_apply.ptr, (void *)g->ws_scale.ptr);
    ss.graph_key = key;
  }
  ss.group_eta.assign(1, mixed_apply_error(g, kind, method, g->fmm_order));
  std::vector<double> rel;
  if (o.precond == BIE_PRECOND_BLOCK) {
    // right preconditioning: GMRES on (A P) u = f, then x = P u
    if (kind > 1) {
      set_error("the block preconditioner is for the elastance and mobility solves");
      return BIE_EINVAL;
    }
    BIE_TRY(pc_build(g, kind, s));
    BIE_TRY(g->ws_scale.reserve((size_t)nrhs * n * sizeof(double)));
    double *tmp = g->ws_scale.as<double>();
    ss.apply = [g, kind, method, nrhs, tmp](int precision, const double *in, double *out,
                                            hipStream_t st) {
      BIE_TRY(pc_apply(g, kind, nrhs, in, tmp, st));
      return apply_operator(g, kind, precision, method, 1, 1.0, nrhs, tmp, out, st);
    };
    const int rc = solve_systems(ss, o, f, x, rel, info, s);
    if (rc != BIE_OK && rc != BIE_ENOCONV) return rc;
    BIE_TRY(pc_apply(g, kind, nrhs, x, x, s));  // in place: each body is staged before written
    return rc;
  }
  if (!o.l2_scaling) {
    ss.apply = [g, kind, method, nrhs](int precision, const double *in, double *out,
                                       hipStream_t st) {
      return apply_operator(g, kind, precision, method, 1, 1.0, nrhs, in, out, st);
    };
    return solve_systems(ss, o, f, x, rel, info, s);
  }
  // L2 rescaling: GMRES on (D A D^-1)(D x) = D f with D = diag(sqrt(w)), the trapezoidal
  // discretisation of the L2 inner product on the curves; then x = D^-1 (D x)
  const int comps = (kind & 1) ? 2 : 1;
  BIE_TRY(g->ws_scale.reserve(2 * (size_t)nrhs * n * sizeof(double)));
  double *fs = g->ws_scale.as<double>(), *tmp = fs + (size_t)nrhs * n;
  BIE_TRY(scale_sqrtw(g, comps, nrhs, 0, f, fs, s));
  ss.apply = [g, kind, method, nrhs, comps, tmp](int precision, const double *in, double *out,
                                                 hipStream_t st) {
    BIE_TRY(scale_sqrtw(g, comps, nrhs, 1, in, tmp, st));
    BIE_TRY(apply_operator(g, kind, precision, method, 1, 1.0, nrhs, tmp, out, st));
    return scale_sqrtw(g, comps, nrhs, 0, out, out, st);
  };
  const int rc = solve_systems(ss, o, fs, x, rel, info, s);
  if (rc != BIE_OK && rc != BIE_ENOCONV) return rc;
  BIE_TRY(scale_sqrtw(g, comps, nrhs, 1, x, x, s));
  return rc;
}

}  // namespace bie
