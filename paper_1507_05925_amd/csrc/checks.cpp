// Host-side checks of curve samples before a geometry is built: finite samples, positive
// orientation, read-off points inside their bodies, and the resolution warning (curves
// resolved by their nodes; no node closer than a few node spacings to another body).
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <string>
#include <unordered_map>
#include <vector>

#include "internal.h"

namespace bie {
namespace {

// Winding number of the closed polygon (x[k], y[k]), k = 0..n-1, around (px, py); 0 outside.
int winding(const double *x, const double *y, int n, double px, double py) {
  int wn = 0;
  for (int k = 0; k < n; ++k) {
    const int k1 = k + 1 == n ? 0 : k + 1;
    const double ax = x[k] - px, ay = y[k] - py, bx = x[k1] - px, by = y[k1] - py;
    const double cr = ax * by - ay * bx;  // > 0: p left of the edge
    if (ay <= 0.0) {
      if (by > 0.0 && cr > 0.0) ++wn;
    } else if (by <= 0.0 && cr < 0.0) {
      --wn;
    }
  }
  return wn;
}

// Smallest |x_i - x_k| / w_k over nodes i, k of different bodies, if below gap_factor (else
// gap_factor, with wi = wk = -1). Uniform grid of cells of size gap_factor * max w: only the
// 3 x 3 cells around a node can hold such a pair.
double min_gap_ratio(const std::vector<double> &x, const std::vector<double> &y,
                     const std::vector<double> &w, const std::vector<int> &body_of,
                     double gap_factor, int &wi, int &wk) {
  const int M = (int)x.size();
  wi = wk = -1;
  double wmax = 0.0, x0 = x[0], y0 = y[0];
  for (int k = 0; k < M; ++k) {
    wmax = std::max(wmax, w[k]);
    x0 = std::min(x0, x[k]);
    y0 = std::min(y0, y[k]);
  }
  const double cell = gap_factor * wmax;
  if (!(cell > 0.0)) return gap_factor;
  // cell indices >= 0, neighbours down to -1: hashed as unsigned (no shift of a negative value)
  auto key = [](long long ix, long long iy) {
    return ((unsigned long long)ix << 32) ^ ((unsigned long long)iy & 0xffffffffULL);
  };
  std::vector<long long> kx(M), ky(M);
  std::unordered_map<unsigned long long, std::vector<int>> grid;
  grid.reserve((size_t)M / 4 + 16);
  for (int k = 0; k < M; ++k) {
    kx[k] = (long long)std::floor((x[k] - x0) / cell);
    ky[k] = (long long)std::floor((y[k] - y0) / cell);
    grid[key(kx[k], ky[k])].push_back(k);
  }
  double worst = gap_factor;
  for (int i = 0; i < M; ++i) {
    for (long long dx = -1; dx <= 1; ++dx)
      for (long long dy = -1; dy <= 1; ++dy) {
        auto it = grid.find(key(kx[i] + dx, ky[i] + dy));
        if (it == grid.end()) continue;
        for (int k : it->second) {
          if (body_of[k] == body_of[i]) continue;
          const double d = std::hypot(x[i] - x[k], y[i] - y[k]) / w[k];
          if (d < worst) {
            worst = d;
            wi = i;
            wk = k;
          }
        }
      }
  }
  return worst;
}

}  // namespace

int check_curves(int N, const int32_t *npb, const double *curve, const double *interior,
                 std::string &msg) {
  long long M = 0;
  for (int b = 0; b < N; ++b) M += npb[b];
  const double *X = curve, *Y = curve + M, *DX = curve + 2 * M, *DY = curve + 3 * M,
               *DDX = curve + 4 * M, *DDY = curve + 5 * M;
  std::vector<double> x(X, X + M), y(Y, Y + M), w(M);
  std::vector<int> body_of(M);
  int resolve = BIE_OK;
  std::string resolve_msg;
  for (int b = 0, k0 = 0; b < N; k0 += npb[b], ++b) {
    const int n = npb[b];
    const double h = 2.0 * kPi / n;
    double area = 0.0, len = 0.0, cx = 0.0, cy = 0.0, turn = 0.0;
    for (int k = k0; k < k0 + n; ++k) {
      for (int a = 0; a < 6; ++a)
        if (!std::isfinite(curve[a * M + k])) {
          msg = "non-finite curve samples on body " + std::to_string(b);
          return BIE_EINVAL;
        }
      const double sp = std::hypot(DX[k], DY[k]);
      w[k] = h * sp;
      body_of[k] = b;
      area += 0.5 * h * (X[k] * DY[k] - Y[k] * DX[k]);
      len += w[k];
      cx += w[k] * X[k];
      cy += w[k] * Y[k];
      // curvature times arc length: (x' y'' - y' x'') / |x'|^2 dt
      if (sp > 0.0) turn += h * (DX[k] * DDY[k] - DY[k] * DDX[k]) / (sp * sp);
    }
    if (!(area > 0.0)) {
      msg = "body " + std::to_string(b) + " is not positively oriented (signed area <= 0)";
      return BIE_EINVAL;
    }
    // the read-off point: the caller's, else the arc-length centroid
    const double px = interior ? interior[2 * b] : cx / len;
    const double py = interior ? interior[2 * b + 1] : cy / len;
    if (!std::isfinite(px) || !std::isfinite(py) || winding(X + k0, Y + k0, n, px, py) != 1) {
      msg = "read-off point (" + std::to_string(px) + ", " + std::to_string(py) + ") of body " +
            std::to_string(b) +
            " is not inside its curve (the default is the arc-length centroid; pass interior "
            "points for bodies whose centroid lies outside)";
      return BIE_EINVAL;
    }
    // the trapezoidal sum of the curvature against arc length is the turning number 2 pi of a
    // simple closed curve, up to the aliasing error of the samples
    const double err = std::fabs(turn - 2.0 * kPi) / (2.0 * kPi);
    if (resolve == BIE_OK && !(err <= kResolveTurn)) {
      resolve = BIE_ERESOLVE;
      resolve_msg = "body " + std::to_string(b) +
                    " is under-resolved: its trapezoidal turning number misses 2 pi by " +
                    std::to_string(err) + " (relative); use more nodes";
    }
  }
  if (resolve == BIE_OK && N > 1) {
    int wi, wk;
    const double r = min_gap_ratio(x, y, w, body_of, kResolveGap, wi, wk);
    if (wi >= 0) {
      resolve = BIE_ERESOLVE;
      resolve_msg = "bodies " + std::to_string(body_of[wi]) + " and " +
                    std::to_string(body_of[wk]) + " are closer than " +
                    std::to_string(kResolveGap) + " node spacings (" + std::to_string(r) +
                    " spacings of body " + std::to_string(body_of[wk]) +
                    "); use more nodes on the closer bodies";
    }
  }
  msg = resolve_msg;
  return resolve;
}

}  // namespace bie
