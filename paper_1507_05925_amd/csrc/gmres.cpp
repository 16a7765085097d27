// Restarted GMRES in float64 (classical Gram-Schmidt applied twice), batched over nrhs
// independent right-hand sides that share one operator apply per Arnoldi step, and float64
// iterative refinement around a float32 far-field apply (BIE_MIXED).
//
// Device: Krylov basis V [m+1][nrhs][n], operator applies, dot products, updates. Host: the
// (m+1) x m Hessenberg columns (read back once per step), Givens rotations, the triangular
// solve; the true residual ||f - A x|| / ||f|| with the float64 operator decides convergence
// at the end of every cycle. The paper iterates GMRES to a relative residual of 1e-6 with
// unstated restart details; x0 = 0 and CGS2 here are this library's choices.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "internal.h"

namespace bie {
namespace {

struct Op {
  int kind, precision, method;
};

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

int apply(bie_geom *g, const Op &op, int nrhs, const double *in, double *out, Stats &st,
          hipStream_t s) {
  BIE_TRY(apply_operator(g, op.kind, op.precision, op.method, 1, 1.0, nrhs, in, out, s));
  if (op.precision == BIE_MIXED) st.applies32 += 1; else st.applies64 += 1;
  st.pairs += (long long)nrhs * g->M * (long long)g->M;
  return BIE_OK;
}

// Host read of `count` doubles from device (stream-ordered).
int read_host(bie_geom *g, const double *dev, size_t count, std::vector<double> &dst, hipStream_t s) {
  BIE_TRY(ensure_pinned(g, count * sizeof(double)));
  BIE_HIP_CHECK(hipMemcpyAsync(g->h_pinned, dev, count * sizeof(double), hipMemcpyDeviceToHost, s));
  BIE_HIP_CHECK(hipStreamSynchronize(s));
  dst.assign(g->h_pinned, g->h_pinned + count);
  return BIE_OK;
}

int write_dev(bie_geom *g, double *dev, const std::vector<double> &src, hipStream_t s) {
  BIE_TRY(ensure_pinned(g, src.size() * sizeof(double)));
  BIE_HIP_CHECK(hipStreamSynchronize(s));  // pinned buffer may still feed an earlier copy
  std::memcpy(g->h_pinned, src.data(), src.size() * sizeof(double));
  BIE_HIP_CHECK(hipMemcpyAsync(dev, g->h_pinned, src.size() * sizeof(double), hipMemcpyHostToDevice, s));
  BIE_HIP_CHECK(hipStreamSynchronize(s));
  return BIE_OK;
}

// Workspace carved from g->ws_solve / g->ws_small.
struct Work {
  double *V, *w, *r, *t;       // V [(m+1)][nrhs][n]; w, r, t [nrhs][n]
  double *h1, *h2, *nrm, *y;   // [nrhs][m+2], [nrhs][m+2], [nrhs], [nrhs][m+1]
  double *scratch;             // dot partials [nrhs][m+2][128]
};

int make_work(bie_geom *g, int nrhs, int n, int m, Work &wk, int extra_vectors, double **extra) {
  const size_t nv = (size_t)nrhs * n;
  const size_t big = ((size_t)(m + 1) + 3 + extra_vectors) * nv * sizeof(double);
  BIE_TRY(g->ws_solve.reserve(big));
  double *p = g->ws_solve.as<double>();
  wk.V = p;
  p += (size_t)(m + 1) * nv;
  wk.w = p;
  p += nv;
  wk.r = p;
  p += nv;
  wk.t = p;
  p += nv;
  for (int e = 0; e < extra_vectors; ++e) {
    extra[e] = p;
    p += nv;
  }
  const size_t hs = (size_t)m + 2;
  const size_t small = (3 * hs * nrhs + nrhs + (size_t)nrhs * (m + 2) * 128) * sizeof(double);
  BIE_TRY(g->ws_small.reserve(small));
  double *q = g->ws_small.as<double>();
  wk.h1 = q;
  q += hs * nrhs;
  wk.h2 = q;
  q += hs * nrhs;
  wk.y = q;
  q += hs * nrhs;
  wk.nrm = q;
  q += nrhs;
  wk.scratch = q;
  return BIE_OK;
}

// GMRES(m) on A x = f for nrhs systems. x [nrhs][n] holds the initial guess on entry (x0 = 0 if
// x_is_zero) and the iterate on exit. conv[r] reports whether rhs r reached tol.
int gmres(bie_geom *g, const Op &op, int nrhs, int n, const double *f, double *x, bool x_is_zero,
          double tol, int m, int max_iter, Work &wk, Stats &st, std::vector<double> &relres,
          std::vector<int> &conv, hipStream_t s) {
  const long long vs_v = (long long)nrhs * n;  // stride between Krylov vectors
  const long long vs_r = n;                    // stride between rhs inside one Krylov vector
  const long long hs = m + 2;
  std::vector<double> fnorm, beta, hh1, hh2, hn;
  if (x_is_zero) BIE_HIP_CHECK(hipMemsetAsync(x, 0, sizeof(double) * nrhs * n, s));
  BIE_TRY(vec_nrm2(nrhs, n, f, n, wk.nrm, wk.scratch, s));
  BIE_TRY(read_host(g, wk.nrm, nrhs, fnorm, s));
  relres.assign(nrhs, 0.0);
  conv.assign(nrhs, 0);
  bool first = true;
  std::vector<double> H((size_t)nrhs * (m + 1) * m), cs((size_t)nrhs * m), sn((size_t)nrhs * m),
      gv((size_t)nrhs * (m + 1));
  while (true) {
    // r = f - A x
    if (first && x_is_zero) {
      BIE_HIP_CHECK(hipMemcpyAsync(wk.r, f, sizeof(double) * nrhs * n, hipMemcpyDeviceToDevice, s));
    } else {
      BIE_TRY(apply(g, op, nrhs, x, wk.r, st, s));
      BIE_TRY(vec_axpby(nrhs, n, 1.0, f, -1.0, wk.r, s));
    }
    first = false;
    BIE_TRY(vec_nrm2(nrhs, n, wk.r, n, wk.nrm, wk.scratch, s));
    BIE_TRY(read_host(g, wk.nrm, nrhs, beta, s));
    std::vector<int> active(nrhs, 0);
    int nact = 0;
    for (int r = 0; r < nrhs; ++r) {
      relres[r] = fnorm[r] > 0.0 ? beta[r] / fnorm[r] : 0.0;
      conv[r] = relres[r] <= tol;
      active[r] = !conv[r];
      nact += active[r];
    }
    if (verbosity() >= 1)
      std::fprintf(stderr, "[bie] gmres prec=%d cycle start: iters=%d true rel res[0]=%.3e\n",
                   op.precision, st.iters, relres[0]);
    if (nact == 0 || st.iters >= max_iter) break;
    // V_0 = r / beta (inactive rhs: zero vector)
    for (int r = 0; r < nrhs; ++r)
      if (!active[r]) beta[r] = 0.0;
    BIE_TRY(write_dev(g, wk.nrm, beta, s));
    BIE_TRY(vec_scale_to(nrhs, n, wk.r, n, wk.nrm, wk.V, n, s));
    std::fill(gv.begin(), gv.end(), 0.0);
    for (int r = 0; r < nrhs; ++r) gv[(size_t)r * (m + 1)] = beta[r];
    std::vector<int> jdone(nrhs, -1);
    int jend = -1;
    for (int j = 0; j < m; ++j) {
      double *Vj = wk.V + (size_t)j * vs_v;
      double *Vj1 = wk.V + (size_t)(j + 1) * vs_v;
      BIE_TRY(apply(g, op, nrhs, Vj, wk.w, st, s));
      st.iters += 1;
      BIE_TRY(vec_dots(nrhs, n, j + 1, wk.V, vs_r, vs_v, wk.w, n, wk.h1, hs, wk.scratch, s));
      BIE_TRY(vec_sub_combination(nrhs, n, j + 1, wk.V, vs_r, vs_v, wk.h1, hs, wk.w, n, -1.0, s));
      BIE_TRY(vec_dots(nrhs, n, j + 1, wk.V, vs_r, vs_v, wk.w, n, wk.h2, hs, wk.scratch, s));
      BIE_TRY(vec_sub_combination(nrhs, n, j + 1, wk.V, vs_r, vs_v, wk.h2, hs, wk.w, n, -1.0, s));
      BIE_TRY(vec_nrm2(nrhs, n, wk.w, n, wk.nrm, wk.scratch, s));
      BIE_TRY(vec_scale_to(nrhs, n, wk.w, n, wk.nrm, Vj1, n, s));
      BIE_TRY(vec_add_h(nrhs, n, wk.h1, wk.h2, j + 1, hs, s));
      BIE_TRY(read_host(g, wk.h2, (size_t)nrhs * hs, hh2, s));
      BIE_TRY(read_host(g, wk.nrm, nrhs, hn, s));
      bool all_done = true;
      for (int r = 0; r < nrhs; ++r) {
        if (!active[r] || jdone[r] >= 0) continue;
        double *Hc = &H[((size_t)r * (m + 1)) * m];  // column-major (m+1) x m
        double *col = Hc + (size_t)j * (m + 1);
        for (int i = 0; i <= j; ++i) col[i] = hh2[(size_t)r * hs + i];
        col[j + 1] = hn[r];
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
        if (verbosity() >= 2 && r == 0)
          std::fprintf(stderr, "[bie]   j=%d est rel res=%.3e hn=%.3e\n", j, res, hn[r]);
        if (res <= tol || hn[r] == 0.0) jdone[r] = j;
        else all_done = false;
      }
      jend = j;
      if (all_done || st.iters >= max_iter) break;
    }
    // y = H^{-1} g (upper triangular), x += V y
    const int nv = jend + 1;
    std::vector<double> yv((size_t)nrhs * hs, 0.0);
    for (int r = 0; r < nrhs; ++r) {
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
    }
    BIE_TRY(write_dev(g, wk.y, yv, s));
    BIE_TRY(vec_sub_combination(nrhs, n, nv, wk.V, vs_r, vs_v, wk.y, hs, x, n, 1.0, s));
  }
  return BIE_OK;
}

}  // namespace

int ensure_pinned(bie_geom *g, size_t bytes) {
  if (g->h_pinned_bytes >= bytes) return BIE_OK;
  if (g->h_pinned) {
    BIE_HIP_CHECK(hipHostFree(g->h_pinned));
    g->h_pinned = nullptr;
    g->h_pinned_bytes = 0;
  }
  size_t want = std::max<size_t>(bytes, 1 << 16);
  if (hipHostMalloc((void **)&g->h_pinned, want, hipHostMallocDefault) != hipSuccess) {
    set_error("pinned host allocation failed");
    return BIE_ENOMEM;
  }
  g->h_pinned_bytes = want;
  return BIE_OK;
}

// Solves (1/2 I + K + L) x = f (kind 0, n = M) or the Stokes system (kind 1, n = 2M).
int solve_system(bie_geom *g, int kind, const bie_opts &o, int nrhs, const double *f, double *x,
                 bie_info *info, hipStream_t s) {
  const int n = kind == 0 ? g->M : 2 * g->M;
  const int m = std::max(1, std::min(o.restart, 1000));
  Stats st;
  std::vector<double> relres;
  std::vector<int> conv;
  Work wk;
  double *extra[3] = {nullptr, nullptr, nullptr};
  const bool mixed = o.precision == BIE_MIXED;
  BIE_TRY(make_work(g, nrhs, n, m, wk, mixed ? 3 : 0, extra));
  BIE_HIP_CHECK(hipMemsetAsync(x, 0, sizeof(double) * nrhs * n, s));
  const Op op64{kind, BIE_FP64, o.method};
  int refinements = 0;
  if (!mixed) {
    BIE_TRY(gmres(g, op64, nrhs, n, f, x, true, o.tol, m, o.max_iter, wk, st, relres, conv, s));
  } else {
    // x = 0, r = f; repeat: solve A32 d = r to inner_tol; x += d; r = f - A64 x
    const Op op32{kind, BIE_MIXED, o.method};
    double *rr = extra[0], *d = extra[1];
    std::vector<double> fnorm, rn;
    BIE_TRY(vec_nrm2(nrhs, n, f, n, wk.nrm, wk.scratch, s));
    BIE_TRY(read_host(g, wk.nrm, nrhs, fnorm, s));
    BIE_HIP_CHECK(hipMemcpyAsync(rr, f, sizeof(double) * nrhs * n, hipMemcpyDeviceToDevice, s));
    relres.assign(nrhs, 1.0);
    conv.assign(nrhs, 0);
    for (int it = 0;; ++it) {
      BIE_TRY(vec_nrm2(nrhs, n, rr, n, wk.nrm, wk.scratch, s));
      BIE_TRY(read_host(g, wk.nrm, nrhs, rn, s));
      bool all = true;
      for (int r = 0; r < nrhs; ++r) {
        relres[r] = fnorm[r] > 0.0 ? rn[r] / fnorm[r] : 0.0;
        conv[r] = relres[r] <= o.tol;
        all = all && conv[r];
      }
      if (verbosity() >= 1)
        std::fprintf(stderr, "[bie] refinement %d: true rel res[0]=%.3e iters=%d\n", it,
                     relres[0], st.iters);
      if (all || it >= o.max_refine || st.iters >= o.max_iter) break;
      // converged rhs get a zero residual so the inner solve leaves them untouched
      double worst = 0.0;
      for (int r = 0; r < nrhs; ++r) {
        if (conv[r])
          BIE_HIP_CHECK(hipMemsetAsync(rr + (size_t)r * n, 0, sizeof(double) * n, s));
        else
          worst = std::max(worst, relres[r]);
      }
      // the inner solve only has to bring the residual to what the outer tolerance needs
      // (with a margin of 3), never tighter than inner_tol
      const double itol = std::max(o.inner_tol, o.tol / (3.0 * worst));
      std::vector<double> irel;
      std::vector<int> iconv;
      BIE_TRY(gmres(g, op32, nrhs, n, rr, d, true, itol, m, o.max_iter, wk, st, irel, iconv, s));
      BIE_TRY(vec_axpby(nrhs, n, 1.0, d, 1.0, x, s));
      BIE_TRY(apply(g, op64, nrhs, x, rr, st, s));
      BIE_TRY(vec_axpby(nrhs, n, 1.0, f, -1.0, rr, s));
      ++refinements;
    }
  }
  bool ok = true;
  double worst = 0.0;
  for (int r = 0; r < nrhs; ++r) {
    ok = ok && conv[r];
    worst = std::max(worst, relres[r]);
  }
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

}  // namespace bie
