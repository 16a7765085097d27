// Autotuning of the FMM leaf size: the population of a leaf box trades the near-field pair work
// (which grows with it) against the expansion work (which shrinks with it), and the balance
// depends on the kernel, the precision (the mixed apply's expansions are half as long and in
// float32 for Laplace) and the node density. Candidates are timed on the geometry itself, each
// with its own tree, and the fastest is kept per shape class.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "internal.h"

struct bie_tune_cache {
  std::mutex mu;
  std::map<std::tuple<int, int, int, int, int>, int> leaf;  // shape class -> leaf size
  long long tunings = 0, hits = 0;
};

namespace bie {
namespace {

constexpr int kCandidates[] = {24, 32, 48, 64, 96, 128};

bie_tune_cache g_process_cache;

// shape class: kind, precision, rhs per pass (1, 2-4, more), log2 M, log2 of nodes per body
std::tuple<int, int, int, int, int> shape_class(const bie_geom *g, int kind, int precision,
                                                 int nrhs) {
  const int rb = nrhs <= 1 ? 0 : (nrhs <= 4 ? 1 : 2);
  const int lm = (int)std::floor(std::log2((double)g->M));
  const int lb = (int)std::floor(std::log2((double)g->M / g->N));
  return std::make_tuple(kind, precision, rb, lm, lb);
}

// Average time of `reps` applies of the precision's operator with leaf size `leaf` (ms), after
// one untimed apply (which builds the tree the first time).
int time_leaf(bie_geom *g, int kind, int precision, int R, int leaf, const double *mu,
              double *out, hipStream_t s, double &ms) {
  const int keep = g->fmm_leaf, keepm = g->fmm_leaf_mixed;
  if (precision == BIE_MIXED) g->fmm_leaf_mixed = leaf; else g->fmm_leaf = leaf;
  int rc = apply_operator(g, kind, precision, BIE_FMM, 1, 1.0, R, mu, out, s);
  hipEvent_t a = nullptr, b = nullptr;
  constexpr int reps = 3;
  if (rc == BIE_OK && (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess)) {
    set_error("autotune: event creation failed");
    rc = BIE_EDEVICE;
  }
  if (rc == BIE_OK && hipEventRecord(a, s) != hipSuccess) rc = BIE_EDEVICE;
  for (int i = 0; i < reps && rc == BIE_OK; ++i)
    rc = apply_operator(g, kind, precision, BIE_FMM, 1, 1.0, R, mu, out, s);
  if (rc == BIE_OK && (hipEventRecord(b, s) != hipSuccess || hipEventSynchronize(b) != hipSuccess))
    rc = BIE_EDEVICE;
  float t = 0.f;
  if (rc == BIE_OK && hipEventElapsedTime(&t, a, b) != hipSuccess) rc = BIE_EDEVICE;
  if (a) (void)hipEventDestroy(a);
  if (b) (void)hipEventDestroy(b);
  ms = t / reps;
  g->fmm_leaf = keep;
  g->fmm_leaf_mixed = keepm;
  return rc;
}

int tune_one(bie_geom *g, int kind, int precision, int nrhs, hipStream_t s, int &best) {
  const int R = std::min(nrhs, kind == 0 ? 8 : 4);
  const size_t len = (size_t)g->M * (kind == 0 ? 1 : 2);
  DevBuf io;
  BIE_TRY(io.reserve(2 * len * R * sizeof(double)));
  double *mu = io.as<double>(), *out = mu + len * R;
  // a smooth non-trivial density: the timing does not depend on its values
  std::vector<double> h(len * R);
  for (size_t i = 0; i < h.size(); ++i) h[i] = std::sin(0.37 * (double)i) + 0.5;
  int rc = hipMemcpyAsync(mu, h.data(), h.size() * 8, hipMemcpyHostToDevice, s) == hipSuccess &&
                   hipStreamSynchronize(s) == hipSuccess
               ? BIE_OK
               : BIE_EDEVICE;
  best = 64;
  const int current = precision == BIE_MIXED && g->fmm_leaf_mixed > 0 ? g->fmm_leaf_mixed
                                                                       : g->fmm_leaf;
  // kRounds passes over the candidates, each candidate keeping its fastest pass: neighbouring
  // candidates often differ by a few percent, less than the spread of a single timing
  constexpr int kRounds = 3;
  constexpr int nc = sizeof(kCandidates) / sizeof(kCandidates[0]);
  double cand_ms[nc];
  for (int i = 0; i < nc; ++i) cand_ms[i] = 1e300;
  for (int round = 0; round < kRounds && rc == BIE_OK; ++round)
    for (int i = 0; i < nc; ++i) {
      const int leaf = kCandidates[i];
      if (leaf * 4 > g->M) continue;  // a tree of a handful of leaves: not a candidate
      double ms = 0.0;
      rc = time_leaf(g, kind, precision, R, leaf, mu, out, s, ms);
      if (rc != BIE_OK) break;
      cand_ms[i] = std::min(cand_ms[i], ms);
    }
  double best_ms = 1e300;
  for (int i = 0; i < nc; ++i)
    if (cand_ms[i] < best_ms) {
      best_ms = cand_ms[i];
      best = kCandidates[i];
    }
  // the losers' trees are freed (each holds its own work area)
  for (int leaf : kCandidates)
    if (leaf != best && leaf != current) fmm_drop_tree(g, precision, g->fmm_order, leaf);
  (void)hipStreamSynchronize(s);
  io.release();
  return rc;
}

}  // namespace

bie_tune_cache *tune_cache_of(bie_geom *g);

int autotune_leaf(bie_geom *g, int kind, int precision, int nrhs, hipStream_t s) {
  bie_tune_cache *cache = tune_cache_of(g);
  if (!cache) cache = &g_process_cache;
  // the float64 applies (all of a float64 solve; the residuals of a mixed one) and, for a mixed
  // solve, the float32 inner applies each get their own leaf size
  const int precs[2] = {BIE_FP64, BIE_MIXED};
  for (int k = 0; k < (precision == BIE_MIXED ? 2 : 1); ++k) {
    const auto key = shape_class(g, kind, precs[k], nrhs);
    int leaf = 0;
    {
      std::lock_guard<std::mutex> lk(cache->mu);
      auto it = cache->leaf.find(key);
      if (it != cache->leaf.end()) {
        leaf = it->second;
        cache->hits += 1;
      }
    }
    if (leaf == 0) {
      BIE_TRY(tune_one(g, kind, precs[k], nrhs, s, leaf));
      std::lock_guard<std::mutex> lk(cache->mu);
      cache->leaf[key] = leaf;
      cache->tunings += 1;
    }
    if (precs[k] == BIE_MIXED) g->fmm_leaf_mixed = leaf; else g->fmm_leaf = leaf;
  }
  return BIE_OK;
}

bie_tune_cache *process_tune_cache() { return &g_process_cache; }
bie_tune_cache *new_tune_cache() { return new bie_tune_cache(); }
void delete_tune_cache(bie_tune_cache *c) { delete c; }
int tune_cache_stats(bie_tune_cache *c, long long *tunings, long long *hits) {
  std::lock_guard<std::mutex> lk(c->mu);
  if (tunings) *tunings = c->tunings;
  if (hits) *hits = c->hits;
  return BIE_OK;
}

int resolve_leaf(bie_geom *g, int kind, const bie_opts &o, int nrhs, bool tune, hipStream_t s) {
  if (o.fmm_leaf == 0 && tune) return autotune_leaf(g, kind, o.precision, nrhs, s);
  g->fmm_leaf = o.fmm_leaf > 0 ? o.fmm_leaf : 64;
  g->fmm_leaf_mixed = 0;
  return BIE_OK;
}

}  // namespace bie
