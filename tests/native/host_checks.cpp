// Host-side paths of the C ABI, built with AddressSanitizer and UndefinedBehaviorSanitizer on the
// host code (the device code is built as usual) and run without a GPU: option validation, the
// curve checks bie_geom_create applies (finite samples, orientation, read-off points inside their
// bodies, the resolution warning), the expansion-length helper, profiling state and the no-device
// errors of the context and the server. Exits non-zero on the first unexpected result; the
// sanitizers abort on any invalid memory access or undefined behaviour in the host code.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <vector>

#include "bie2d.h"

namespace {

int failures = 0;

void expect(bool ok, const char *what) {
  if (!ok) {
    std::fprintf(stderr, "FAIL: %s (last error: %s)\n", what, bie_last_error());
    ++failures;
  }
}

// Circles of radius r centred at (cx_b, 0), n nodes each, counter-clockwise unless cw: the
// curve samples [6][M] as bie_curves_check takes them.
std::vector<double> circles(const std::vector<double> &cx, double r, int n, bool cw = false) {
  const int N = (int)cx.size(), M = N * n;
  std::vector<double> c(6 * (size_t)M);
  for (int b = 0; b < N; ++b)
    for (int k = 0; k < n; ++k) {
      const double t = 2.0 * M_PI * k / n, s = cw ? -1.0 : 1.0;
      const int i = b * n + k;
      c[0 * (size_t)M + i] = cx[b] + r * std::cos(t);
      c[1 * (size_t)M + i] = s * r * std::sin(t);
      c[2 * (size_t)M + i] = -r * std::sin(t);
      c[3 * (size_t)M + i] = s * r * std::cos(t);
      c[4 * (size_t)M + i] = -r * std::cos(t);
      c[5 * (size_t)M + i] = -s * r * std::sin(t);
    }
  return c;
}

void curve_checks() {
  std::vector<int32_t> npb(2, 256);
  std::vector<double> good = circles({-1.25, 1.25}, 1.0, 256);
  expect(bie_curves_check(2, npb.data(), good.data(), nullptr) == BIE_OK, "two discs pass");
  std::vector<double> in = {-1.25, 0.1, 1.25, -0.3};
  expect(bie_curves_check(2, npb.data(), good.data(), in.data()) == BIE_OK, "points inside");
  std::vector<double> out = {-1.25, 0.1, 3.0, 0.0};
  expect(bie_curves_check(2, npb.data(), good.data(), out.data()) == BIE_EINVAL,
         "point outside its body");
  expect(std::strstr(bie_last_error(), "not inside") != nullptr, "outside message");
  std::vector<double> cw = circles({-1.25, 1.25}, 1.0, 256, true);
  expect(bie_curves_check(2, npb.data(), cw.data(), nullptr) == BIE_EINVAL, "clockwise");
  std::vector<double> bad = good;
  bad[5 * 512 + 300] = NAN;
  expect(bie_curves_check(2, npb.data(), bad.data(), nullptr) == BIE_EINVAL, "non-finite");
  // a gap of 0.005 between unit discs: 2048 nodes give 1.6 node spacings (warning)
  std::vector<int32_t> npb2(2, 2048);
  std::vector<double> close = circles({-1.0025, 1.0025}, 1.0, 2048);
  expect(bie_curves_check(2, npb2.data(), close.data(), nullptr) == BIE_ERESOLVE, "gap warning");
  // a body of 3 nodes: under-resolved (turning number of a triangle's samples)
  std::vector<int32_t> npb3 = {3, 256};
  std::vector<double> tri(6 * 259);
  std::vector<double> d1 = circles({-1.25}, 1.0, 3), d2 = circles({1.25}, 1.0, 256);
  for (int r = 0; r < 6; ++r) {
    for (int k = 0; k < 3; ++k) tri[r * 259 + k] = d1[r * 3 + k];
    for (int k = 0; k < 256; ++k) tri[r * 259 + 3 + k] = d2[r * 256 + k];
  }
  const int rc = bie_curves_check(2, npb3.data(), tri.data(), nullptr);
  expect(rc == BIE_ERESOLVE || rc == BIE_EINVAL, "three-node body flagged");
  expect(bie_curves_check(0, npb.data(), good.data(), nullptr) == BIE_EINVAL, "no bodies");
  expect(bie_curves_check(2, npb.data(), nullptr, nullptr) == BIE_EINVAL, "null curve");
}

void option_checks() {
  bie_opts o;
  expect(bie_default_opts(&o) == BIE_OK, "defaults");
  expect(o.precision == BIE_FP64 && o.fmm_leaf == 64 && o.viscosity == 1.0 &&
             o.mixed_strategy == BIE_MIXED_RELAXED && o.l2_scaling == 0,
         "default values");
  bie_batch *b = nullptr;
  expect(bie_batch_create(&b) == BIE_OK && b, "batch create");
  bie_batch_item item{};
  bie_info info{};
  const struct {
    const char *what;
    void (*set)(bie_opts &);
  } bad[] = {
      {"viscosity 0", [](bie_opts &x) { x.viscosity = 0.0; }},
      {"viscosity nan", [](bie_opts &x) { x.viscosity = NAN; }},
      {"fmm_eps < 0", [](bie_opts &x) { x.fmm_eps = -1e-3; }},
      {"l2_scaling 2", [](bie_opts &x) { x.l2_scaling = 2; }},
      {"mixed_strategy 2", [](bie_opts &x) { x.mixed_strategy = 2; }},
      {"fmm_order 100", [](bie_opts &x) { x.fmm_order = 100; }},
      {"fmm_leaf < 0", [](bie_opts &x) { x.fmm_leaf = -1; }},
      {"tol 0", [](bie_opts &x) { x.tol = 0.0; }},
  };
  for (const auto &c : bad) {
    bie_opts x = o;
    c.set(x);
    expect(bie_batch_solve(b, 1, &item, &x, &info, nullptr, nullptr) == BIE_EINVAL, c.what);
  }
  expect(bie_batch_destroy(b) == BIE_OK, "batch destroy");
  // expansion lengths: fixed order and accuracy targets
  int t64 = 0, t32 = 0;
  expect(bie_fmm_terms(&o, 0, BIE_FP64, &t64) == BIE_OK && t64 == 40, "order 40 -> 40 terms");
  expect(bie_fmm_terms(&o, 0, BIE_MIXED, &t32) == BIE_OK && t32 == 24, "mixed 24 terms");
  bie_opts e = o;
  e.fmm_eps = 1e-10;
  expect(bie_fmm_terms(&e, 0, BIE_FP64, &t64) == BIE_OK && t64 == 24, "Laplace 1e-10 -> 24");
  expect(bie_fmm_terms(&e, 1, BIE_FP64, &t64) == BIE_OK && t64 == 32, "Stokes 1e-10 -> 32");
  expect(bie_fmm_terms(&e, 2, BIE_FP64, &t64) == BIE_EINVAL, "bad kind");
}

void profile_checks() {
  expect(bie_profile_select(0xffffffffu) == BIE_OK, "profile select");
  expect(bie_profile_sample(1) == BIE_OK, "profile sample");
  long long launches = -1, pairs = -1;
  double ms = -1.0;
  expect(bie_profile_read(BIE_K_FMM, &launches, &ms, &pairs) == BIE_OK && launches == 0,
         "profile read");
  expect(bie_profile_read(BIE_K_COUNT, &launches, &ms, &pairs) == BIE_EINVAL, "bad class");
}

void device_less_checks() {
  expect(bie_create(nullptr, 0, nullptr) == BIE_EINVAL, "context needs out");
  bie_ctx *ctx = nullptr;
  expect(bie_create(&ctx, 0, nullptr) == BIE_EDEVICE && ctx == nullptr, "no device: context");
  bie_server_config cfg{};
  cfg.max_cycles = 10;
  bie_default_opts(&cfg.opts);
  bie_server *srv = nullptr;
  expect(bie_server_create(&cfg, &srv) == BIE_EDEVICE && srv == nullptr, "no device: server");
  cfg.opts.l2_scaling = 1;
  expect(bie_server_create(&cfg, &srv) == BIE_EINVAL, "server rejects l2_scaling");
}

}  // namespace

int main() {
  curve_checks();
  option_checks();
  profile_checks();
  device_less_checks();
  if (failures) {
    std::fprintf(stderr, "%d host check(s) failed\n", failures);
    return 1;
  }
  std::printf("host checks passed\n");
  return 0;
}
