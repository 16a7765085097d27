// Operator kernels of the bie2d library for gfx950.
//
// The apply of (1/2 I + K + L) (elastance, eq. ModRep2) and (1/2 I + Kcal + L) (mobility,
// eq. ModRep2Stokes) is split into
//   (1) a far-field sweep over all (target, source) pairs whose bodies differ, and
//   (2) a per-body epilogue: the self-body block in float64 with the smooth diagonal limit, the
//       identity, the completion L (per-body charge / force and torque reductions), and the sum
//       of the far-field partials in a fixed order.
// The far-field sweep maps one target node to one lane and streams source nodes through scalar
// registers: the source loop index is wave-uniform, so each source record is fetched once per
// wave by a scalar load and enters the vector instructions as an SGPR operand (no LDS traffic,
// no bank conflicts, 64 pairs per vector instruction). Sources are swept body by body; a body's
// float32 partial sum is added into float64 accumulators before the next body (compensation of
// the float32 roundoff at body granularity) and the body of the target itself is skipped.
// The source range is cut into `nsplit` contiguous groups of bodies (grid.y); each group writes
// its own partial, so the result is deterministic and independent of scheduling.
#include <hip/hip_runtime.h>

#include <cmath>
#include <mutex>
#include <string>

#include "internal.h"

namespace bie {

namespace {

__device__ inline double block_sum(double v, double *sh) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) sh[wid] = v;
  __syncthreads();
  const double t = (sh[0] + sh[1]) + (sh[2] + sh[3]);
  __syncthreads();
  return t;
}

// float64 reciprocal: the hardware estimate (relative error below 5e-8 on gfx950, measured)
// refined by one Newton step, which squares the error (about 2e-15, measured).
__device__ inline double rcp64(double a) {
  const double y = __builtin_amdgcn_rcp(a);
  const double e = fma(-a, y, 1.0);
  return fma(y, e, y);
}

// ------------------------------------------------------------------------------------------
// a1: geometry. One workgroup per body. Non-finite samples poison area[b] (checked on host).
// ------------------------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_geometry(
    int M, const int *__restrict__ body_ptr, const double *__restrict__ curve,
    const double *__restrict__ interior, double *__restrict__ x, double *__restrict__ y,
    double *__restrict__ nx, double *__restrict__ ny, double *__restrict__ w,
    double *__restrict__ kappa, double *__restrict__ px, double *__restrict__ py,
    double *__restrict__ len, double *__restrict__ xc, double *__restrict__ yc,
    double *__restrict__ W, double *__restrict__ pint, double *__restrict__ area,
    double2 *__restrict__ xy, float2 *__restrict__ xr, int *__restrict__ body_of) {
  __shared__ double sh[4];
  const int b = blockIdx.x;
  const int k0 = body_ptr[b], k1 = body_ptr[b + 1];
  const double h = 2.0 * kPi / (double)(k1 - k0);
  double sl = 0.0, sx = 0.0, sy = 0.0, sa = 0.0;
  for (int k = k0 + threadIdx.x; k < k1; k += kBlock) {
    const double X = curve[k], Y = curve[M + k];
    const double dX = curve[2 * M + k], dY = curve[3 * M + k];
    const double ddX = curve[4 * M + k], ddY = curve[5 * M + k];
    const double sp = sqrt(dX * dX + dY * dY);
    const double tx = dX / sp, ty = dY / sp;
    const double kap = (dX * ddY - dY * ddX) / (sp * sp * sp);
    const double wk = h * sp;
    x[k] = X;
    y[k] = Y;
    nx[k] = ty;
    ny[k] = -tx;
    kappa[k] = kap;
    w[k] = wk;
    xy[k] = make_double2(X, Y);
    body_of[k] = b;
    sl += wk;
    sx += wk * X;
    sy += wk * Y;
    sa += (X * dY - Y * dX) + 0.0 * (kap + wk);  // 0 * non-finite -> NaN marks the body
  }
  const double L = block_sum(sl, sh);
  const double cx = block_sum(sx, sh) / L;
  const double cy = block_sum(sy, sh) / L;
  const double A = 0.5 * h * block_sum(sa, sh);
  double sw = 0.0;
  for (int k = k0 + threadIdx.x; k < k1; k += kBlock) {
    const double rx = x[k] - cx, ry = y[k] - cy;
    px[k] = -ry;
    py[k] = rx;
    xr[k] = make_float2((float)rx, (float)ry);
    sw += w[k] * (rx * rx + ry * ry);
  }
  const double Wb = block_sum(sw, sh);
  if (threadIdx.x == 0) {
    len[b] = L;
    xc[b] = cx;
    yc[b] = cy;
    W[b] = Wb;
    area[b] = A;
    pint[2 * b] = interior ? interior[2 * b] : cx;
    pint[2 * b + 1] = interior ? interior[2 * b + 1] : cy;
  }
}

// Length scale R of the completed double layers (capacitance and resistance problems): twice the
// diagonal of the nodes' bounding box, which exceeds the logarithmic capacity of the curves.
// One workgroup.
__global__ __launch_bounds__(kBlock) void k_scale_length(int M, const double *__restrict__ x,
                                                         const double *__restrict__ y,
                                                         double *__restrict__ R) {
  __shared__ double sh[4][4];
  double v[4] = {x[0], -x[0], y[0], -y[0]};  // min x, -max x, min y, -max y
  for (int k = threadIdx.x; k < M; k += kBlock) {
    v[0] = fmin(v[0], x[k]);
    v[1] = fmin(v[1], -x[k]);
    v[2] = fmin(v[2], y[k]);
    v[3] = fmin(v[3], -y[k]);
  }
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v[a] = fmin(v[a], __shfl_down(v[a], off, 64));
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0)
#pragma unroll
    for (int a = 0; a < 4; ++a) sh[wid][a] = v[a];
  __syncthreads();
  if (threadIdx.x == 0) {
    double m[4];
#pragma unroll
    for (int a = 0; a < 4; ++a) m[a] = fmin(fmin(sh[0][a], sh[1][a]), fmin(sh[2][a], sh[3][a]));
    const double dx = -m[1] - m[0], dy = -m[3] - m[2];
    R[0] = 2.0 * sqrt(dx * dx + dy * dy);
  }
}

// ------------------------------------------------------------------------------------------
// Source strengths s = w * mu (float64 and float32 copies); len = M (Laplace) or 2M (Stokes).
// ------------------------------------------------------------------------------------------
__global__ void k_pack(long long total, int M, int comps, const double *__restrict__ w,
                       const double *__restrict__ mu, double *__restrict__ s64,
                       float *__restrict__ s32) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= total) return;
  const int node = (int)((t % ((long long)M * comps)) / comps);
  const double v = w[node] * mu[t];
  s64[t] = v;
  if (s32) s32[t] = (float)v;
}

// ------------------------------------------------------------------------------------------
// a3: far-field sweeps. Lane = target i; loop over source bodies c of this split, c != body(i).
// ------------------------------------------------------------------------------------------
constexpr float kFar32 = 1.0e18f;   // parking coordinate for lanes whose own body is swept
constexpr double kFar64 = 1.0e100;  // (their sum is discarded; it only has to stay finite)

template <int R>
__global__ __launch_bounds__(kBlock) void k_lap_far_f32(
    int M, const int *__restrict__ body_ptr, const int *__restrict__ body_of,
    const double *__restrict__ xc, const double *__restrict__ yc, const float2 *__restrict__ xr,
    const float *__restrict__ s32, const double *__restrict__ nx, const double *__restrict__ ny,
    const int *__restrict__ split_body, double *__restrict__ partial) {
  const int split = blockIdx.y;
  const int i = blockIdx.x * kBlock + threadIdx.x;
  const bool valid = i < M;
  const int ii = valid ? i : M - 1;
  const int bi = body_of[ii];
  const double cxi = xc[bi], cyi = yc[bi];
  const float2 pr = xr[ii];
  double Gx[R], Gy[R];
#pragma unroll
  for (int r = 0; r < R; ++r) Gx[r] = Gy[r] = 0.0;
  const int c0 = split_body[split], c1 = split_body[split + 1];
  for (int c = c0; c < c1; ++c) {
    const bool self = (c == bi);
    if (__all(self)) continue;
    // target in the frame of source body c: float64 offset of the centroids, then float32
    float tx = (float)((cxi - xc[c]) + (double)pr.x);
    float ty = (float)((cyi - yc[c]) + (double)pr.y);
    tx = self ? kFar32 : tx;
    ty = self ? kFar32 : ty;
    float gx[R], gy[R];
#pragma unroll
    for (int r = 0; r < R; ++r) gx[r] = gy[r] = 0.0f;
    const int k0 = body_ptr[c], k1 = body_ptr[c + 1];
#pragma unroll 4
    for (int k = k0; k < k1; ++k) {
      const float2 q = xr[k];
      const float dx = tx - q.x, dy = ty - q.y;
      const float inv = __builtin_amdgcn_rcpf(fmaf(dx, dx, dy * dy));
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const float t = s32[(size_t)r * M + k] * inv;
        gx[r] = fmaf(dx, t, gx[r]);
        gy[r] = fmaf(dy, t, gy[r]);
      }
    }
    if (!self) {
#pragma unroll
      for (int r = 0; r < R; ++r) {
        Gx[r] += (double)gx[r];
        Gy[r] += (double)gy[r];
      }
    }
  }
  if (valid) {
    const double a = nx[i], b = ny[i];
#pragma unroll
    for (int r = 0; r < R; ++r)
      partial[((size_t)split * R + r) * M + i] = -(a * Gx[r] + b * Gy[r]) / (2.0 * kPi);
  }
}

template <int R>
__global__ __launch_bounds__(kBlock) void k_lap_far_f64(
    int M, const int *__restrict__ body_ptr, const int *__restrict__ body_of,
    const double2 *__restrict__ xy, const double *__restrict__ s64, const double *__restrict__ nx,
    const double *__restrict__ ny, const int *__restrict__ split_body, double *__restrict__ partial) {
  const int split = blockIdx.y;
  const int i = blockIdx.x * kBlock + threadIdx.x;
  const bool valid = i < M;
  const int ii = valid ? i : M - 1;
  const int bi = body_of[ii];
  const double2 p = xy[ii];
  double Gx[R], Gy[R];
#pragma unroll
  for (int r = 0; r < R; ++r) Gx[r] = Gy[r] = 0.0;
  const int c0 = split_body[split], c1 = split_body[split + 1];
  for (int c = c0; c < c1; ++c) {
    const bool self = (c == bi);
    if (__all(self)) continue;
    const double tx = self ? kFar64 : p.x;
    const double ty = self ? kFar64 : p.y;
    double gx[R], gy[R];
#pragma unroll
    for (int r = 0; r < R; ++r) gx[r] = gy[r] = 0.0;
    const int k0 = body_ptr[c], k1 = body_ptr[c + 1];
#pragma unroll 2
    for (int k = k0; k < k1; ++k) {
      const double2 q = xy[k];
      const double dx = tx - q.x, dy = ty - q.y;
      const double inv = rcp64(fma(dx, dx, dy * dy));
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const double t = s64[(size_t)r * M + k] * inv;
        gx[r] = fma(dx, t, gx[r]);
        gy[r] = fma(dy, t, gy[r]);
      }
    }
    if (!self) {
#pragma unroll
      for (int r = 0; r < R; ++r) {
        Gx[r] += gx[r];
        Gy[r] += gy[r];
      }
    }
  }
  if (valid) {
    const double a = nx[i], b = ny[i];
#pragma unroll
    for (int r = 0; r < R; ++r)
      partial[((size_t)split * R + r) * M + i] = -(a * Gx[r] + b * Gy[r]) / (2.0 * kPi);
  }
}

// Stokes: sum_k -(1/pi) (r.n_i)(r.s_k) r / |r|^4, s_k = w_k mu_k (vector), r = x_i - x_k.
template <int R>
__global__ __launch_bounds__(kBlock) void k_stk_far_f32(
    int M, const int *__restrict__ body_ptr, const int *__restrict__ body_of,
    const double *__restrict__ xc, const double *__restrict__ yc, const float2 *__restrict__ xr,
    const float2 *__restrict__ s32, const double *__restrict__ nx, const double *__restrict__ ny,
    const int *__restrict__ split_body, double *__restrict__ partial) {
  const int split = blockIdx.y;
  const int i = blockIdx.x * kBlock + threadIdx.x;
  const bool valid = i < M;
  const int ii = valid ? i : M - 1;
  const int bi = body_of[ii];
  const double cxi = xc[bi], cyi = yc[bi];
  const float2 pr = xr[ii];
  const float nxi = (float)nx[ii], nyi = (float)ny[ii];
  double Gx[R], Gy[R];
#pragma unroll
  for (int r = 0; r < R; ++r) Gx[r] = Gy[r] = 0.0;
  const int c0 = split_body[split], c1 = split_body[split + 1];
  for (int c = c0; c < c1; ++c) {
    const bool self = (c == bi);
    if (__all(self)) continue;
    float tx = (float)((cxi - xc[c]) + (double)pr.x);
    float ty = (float)((cyi - yc[c]) + (double)pr.y);
    tx = self ? kFar32 : tx;
    ty = self ? kFar32 : ty;
    float gx[R], gy[R];
#pragma unroll
    for (int r = 0; r < R; ++r) gx[r] = gy[r] = 0.0f;
    const int k0 = body_ptr[c], k1 = body_ptr[c + 1];
#pragma unroll 2
    for (int k = k0; k < k1; ++k) {
      const float2 q = xr[k];
      const float dx = tx - q.x, dy = ty - q.y;
      const float inv = __builtin_amdgcn_rcpf(fmaf(dx, dx, dy * dy));
      const float a = fmaf(dx, nxi, dy * nyi) * (inv * inv);
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const float2 sv = s32[(size_t)r * M + k];
        const float cc = fmaf(dx, sv.x, dy * sv.y) * a;
        gx[r] = fmaf(cc, dx, gx[r]);
        gy[r] = fmaf(cc, dy, gy[r]);
      }
    }
    if (!self) {
#pragma unroll
      for (int r = 0; r < R; ++r) {
        Gx[r] += (double)gx[r];
        Gy[r] += (double)gy[r];
      }
    }
  }
  if (valid) {
#pragma unroll
    for (int r = 0; r < R; ++r) {
      double *o = partial + ((size_t)split * R + r) * 2 * M;
      o[2 * i] = -Gx[r] / kPi;
      o[2 * i + 1] = -Gy[r] / kPi;
    }
  }
}

template <int R>
__global__ __launch_bounds__(kBlock) void k_stk_far_f64(
    int M, const int *__restrict__ body_ptr, const int *__restrict__ body_of,
    const double2 *__restrict__ xy, const double2 *__restrict__ s64, const double *__restrict__ nx,
    const double *__restrict__ ny, const int *__restrict__ split_body, double *__restrict__ partial) {
  const int split = blockIdx.y;
  const int i = blockIdx.x * kBlock + threadIdx.x;
  const bool valid = i < M;
  const int ii = valid ? i : M - 1;
  const int bi = body_of[ii];
  const double2 p = xy[ii];
  const double nxi = nx[ii], nyi = ny[ii];
  double Gx[R], Gy[R];
#pragma unroll
  for (int r = 0; r < R; ++r) Gx[r] = Gy[r] = 0.0;
  const int c0 = split_body[split], c1 = split_body[split + 1];
  for (int c = c0; c < c1; ++c) {
    const bool self = (c == bi);
    if (__all(self)) continue;
    const double tx = self ? kFar64 : p.x;
    const double ty = self ? kFar64 : p.y;
    double gx[R], gy[R];
#pragma unroll
    for (int r = 0; r < R; ++r) gx[r] = gy[r] = 0.0;
    const int k0 = body_ptr[c], k1 = body_ptr[c + 1];
#pragma unroll 2
    for (int k = k0; k < k1; ++k) {
      const double2 q = xy[k];
      const double dx = tx - q.x, dy = ty - q.y;
      const double inv = rcp64(fma(dx, dx, dy * dy));
      const double a = fma(dx, nxi, dy * nyi) * (inv * inv);
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const double2 sv = s64[(size_t)r * M + k];
        const double cc = fma(dx, sv.x, dy * sv.y) * a;
        gx[r] = fma(cc, dx, gx[r]);
        gy[r] = fma(cc, dy, gy[r]);
      }
    }
    if (!self) {
#pragma unroll
      for (int r = 0; r < R; ++r) {
        Gx[r] += gx[r];
        Gy[r] += gy[r];
      }
    }
  }
  if (valid) {
#pragma unroll
    for (int r = 0; r < R; ++r) {
      double *o = partial + ((size_t)split * R + r) * 2 * M;
      o[2 * i] = -Gx[r] / kPi;
      o[2 * i + 1] = -Gy[r] / kPi;
    }
  }
}

// ------------------------------------------------------------------------------------------
// a4: per-body epilogue, float64. grid = (N bodies, nrhs). Adds the self-body block (pairs
// k != i of body b), the smooth diagonal limit, 1/2 mu, the completion L (with_L), and the
// far-field partials (nsplit of them, summed in split order); out = alpha * total.
// ------------------------------------------------------------------------------------------
// Epilogues: grid (body x target tile, rhs), tiles of kBlock targets (ntile per body, the
// largest body's count; tiles past a body's end exit at once). Each workgroup forms its body's
// completion sums itself, then the self-body block (sources read four per step), the diagonal
// limit, the identity and the far-field partials for its targets.
__global__ __launch_bounds__(kBlock) void k_lap_epilogue(
    int M, int nsplit, int R, int ntile, const int *__restrict__ body_ptr,
    const double *__restrict__ x, const double *__restrict__ y, const double *__restrict__ nx,
    const double *__restrict__ ny, const double *__restrict__ w, const double *__restrict__ kappa,
    const double *__restrict__ mu, const double *__restrict__ s64, const double *__restrict__ partial,
    int with_L, int self_block, double alpha, double *__restrict__ out) {
  __shared__ double sh[4];
  const int b = blockIdx.x / ntile, tile = blockIdx.x % ntile, r = blockIdx.y;
  const int k0 = body_ptr[b], k1 = body_ptr[b + 1];
  if (k0 + tile * kBlock >= k1) return;  // whole workgroup
  const int kend = self_block ? k1 : k0;  // the FMM far field already holds same-body pairs
  const double *s = s64 + (size_t)r * M;
  const double *m = mu + (size_t)r * M;
  double part = 0.0;
  for (int k = k0 + threadIdx.x; k < k1; k += kBlock) part += s[k];
  const double charge = block_sum(part, sh);  // int_{Gamma_b} mu ds
  const int i = k0 + tile * kBlock + threadIdx.x;
  const bool valid = i < k1;
  const int ii = valid ? i : k0;
  const double xi = x[ii], yi = y[ii], a = nx[ii], bb = ny[ii];
  double gx = 0.0, gy = 0.0;
  int k = k0;
  for (; k + 4 <= kend; k += 4) {
    double xs[4], ys[4], ss[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      xs[u] = x[k + u];
      ys[u] = y[k + u];
      ss[u] = s[k + u];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const double dx = xi - xs[u], dy = yi - ys[u];
      const bool same = (k + u == ii);
      const double inv = rcp64(same ? 1.0 : fma(dx, dx, dy * dy));
      const double t = same ? 0.0 : ss[u] * inv;
      gx = fma(dx, t, gx);
      gy = fma(dy, t, gy);
    }
  }
  for (; k < kend; ++k) {
    const double dx = xi - x[k], dy = yi - y[k];
    const bool same = (k == ii);
    const double inv = rcp64(same ? 1.0 : fma(dx, dx, dy * dy));
    const double t = same ? 0.0 : s[k] * inv;
    gx = fma(dx, t, gx);
    gy = fma(dy, t, gy);
  }
  double v = 0.5 * m[ii] - (a * gx + bb * gy) / (2.0 * kPi) - s[ii] * kappa[ii] / (4.0 * kPi);
  if (with_L) v += charge;
  for (int sp = 0; sp < nsplit; ++sp) v += partial[((size_t)sp * R + r) * M + ii];
  if (valid) out[(size_t)r * M + i] = alpha * v;
}

__global__ __launch_bounds__(kBlock) void k_stk_epilogue(
    int M, int nsplit, int R, int ntile, const int *__restrict__ body_ptr,
    const double *__restrict__ x, const double *__restrict__ y, const double *__restrict__ nx,
    const double *__restrict__ ny, const double *__restrict__ kappa, const double *__restrict__ px,
    const double *__restrict__ py, const double *__restrict__ mu, const double *__restrict__ s64,
    const double *__restrict__ partial, int with_L, int self_block, double alpha,
    double *__restrict__ out) {
  __shared__ double sh[4];
  const int b = blockIdx.x / ntile, tile = blockIdx.x % ntile, r = blockIdx.y;
  const int k0 = body_ptr[b], k1 = body_ptr[b + 1];
  if (k0 + tile * kBlock >= k1) return;  // whole workgroup
  const int kend = self_block ? k1 : k0;
  const double *s = s64 + (size_t)r * 2 * M;
  const double *m = mu + (size_t)r * 2 * M;
  double f1 = 0.0, f2 = 0.0, tq = 0.0;
  for (int k = k0 + threadIdx.x; k < k1; k += kBlock) {
    f1 += s[2 * k];
    f2 += s[2 * k + 1];
    tq += px[k] * s[2 * k] + py[k] * s[2 * k + 1];
  }
  const double F1 = block_sum(f1, sh), F2 = block_sum(f2, sh), TQ = block_sum(tq, sh);
  const int i = k0 + tile * kBlock + threadIdx.x;
  const bool valid = i < k1;
  const int ii = valid ? i : k0;
  const double xi = x[ii], yi = y[ii], a = nx[ii], bb = ny[ii];
  double gx = 0.0, gy = 0.0;
  int k = k0;
  for (; k + 4 <= kend; k += 4) {
    double xs[4], ys[4], s1[4], s2[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      xs[u] = x[k + u];
      ys[u] = y[k + u];
      s1[u] = s[2 * (k + u)];
      s2[u] = s[2 * (k + u) + 1];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const double dx = xi - xs[u], dy = yi - ys[u];
      const bool same = (k + u == ii);
      const double inv = rcp64(same ? 1.0 : fma(dx, dx, dy * dy));
      const double rn = fma(dx, a, dy * bb);
      const double cc = same ? 0.0 : fma(dx, s1[u], dy * s2[u]) * rn * (inv * inv);
      gx = fma(cc, dx, gx);
      gy = fma(cc, dy, gy);
    }
  }
  for (; k < kend; ++k) {
    const double dx = xi - x[k], dy = yi - y[k];
    const bool same = (k == ii);
    const double inv = rcp64(same ? 1.0 : fma(dx, dx, dy * dy));
    const double rn = fma(dx, a, dy * bb);
    const double cc = same ? 0.0 : fma(dx, s[2 * k], dy * s[2 * k + 1]) * rn * (inv * inv);
    gx = fma(cc, dx, gx);
    gy = fma(cc, dy, gy);
  }
  // tangent tau = (-n_y, n_x); diagonal -(kappa/2pi) w tau (tau . mu)
  const double t1 = -bb, t2 = a;
  const double ts = t1 * s[2 * ii] + t2 * s[2 * ii + 1];
  const double d = -kappa[ii] / (2.0 * kPi);
  double v1 = 0.5 * m[2 * ii] - gx / kPi + d * t1 * ts;
  double v2 = 0.5 * m[2 * ii + 1] - gy / kPi + d * t2 * ts;
  if (with_L) {
    v1 += F1 + px[ii] * TQ;
    v2 += F2 + py[ii] * TQ;
  }
  for (int sp = 0; sp < nsplit; ++sp) {
    const double *o = partial + ((size_t)sp * R + r) * 2 * M;
    v1 += o[2 * ii];
    v2 += o[2 * ii + 1];
  }
  if (valid) {
    out[(size_t)r * 2 * M + 2 * i] = alpha * v1;
    out[(size_t)r * 2 * M + 2 * i + 1] = alpha * v2;
  }
}

// ------------------------------------------------------------------------------------------
// a2: incident densities sigma = q/|Gamma| (eq. sigma), rho = F/|Gamma| + T p / W (eq. rho)
// ------------------------------------------------------------------------------------------
__global__ void k_sigma(int M, int N, int R, const int *__restrict__ body_of,
                        const double *__restrict__ len, const double *__restrict__ q,
                        double *__restrict__ sigma) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long long)R * M) return;
  const int r = (int)(t / M), k = (int)(t % M);
  const int b = body_of[k];
  sigma[t] = q[(size_t)r * N + b] / len[b];
}

__global__ void k_rho(int M, int N, int R, const int *__restrict__ body_of,
                      const double *__restrict__ len, const double *__restrict__ W,
                      const double *__restrict__ px, const double *__restrict__ py,
                      const double *__restrict__ FT, double *__restrict__ rho) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long long)R * M) return;
  const int r = (int)(t / M), k = (int)(t % M);
  const int b = body_of[k];
  const double *f = FT + (size_t)r * 3 * N + 3 * b;
  rho[(size_t)r * 2 * M + 2 * k] = f[0] / len[b] + f[2] * px[k] / W[b];
  rho[(size_t)r * 2 * M + 2 * k + 1] = f[1] / len[b] + f[2] * py[k] / W[b];
}

// ------------------------------------------------------------------------------------------
// a7: read-off inside the bodies. grid = (N targets, nrhs); block sums over all M sources.
// ------------------------------------------------------------------------------------------
// Read-off kernels: a workgroup takes kTJ interior points (targets) against one range of
// sources (grid: target groups x rhs x source splits), so each source record is loaded once per
// kTJ targets. Raw sums go to part[split][rhs][target][comp]; a second kernel adds the splits in
// order and applies the constants.
constexpr int kTJ = 8;

// Sums v[0..n) over the workgroup; the totals land in every thread's v.
template <int n>
__device__ inline void block_sums(double *v, double (*sh)[n]) {
#pragma unroll
  for (int t = 0; t < n; ++t)
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v[t] += __shfl_down(v[t], off, 64);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0)
#pragma unroll
    for (int t = 0; t < n; ++t) sh[wid][t] = v[t];
  __syncthreads();
#pragma unroll
  for (int t = 0; t < n; ++t) v[t] = (sh[0][t] + sh[1][t]) + (sh[2][t] + sh[3][t]);
}

// sum_k w_k d_k log |p_j - x_k|^2 over the split's sources
__global__ __launch_bounds__(kBlock) void k_potential(int M, int N, int nrhs,
                                                     const double2 *__restrict__ xy,
                                                     const double *__restrict__ w,
                                                     const double *__restrict__ pint,
                                                     const double *__restrict__ dens,
                                                     double *__restrict__ part) {
  __shared__ double sh[4][kTJ];
  const int j0 = blockIdx.x * kTJ, r = blockIdx.y, sp = blockIdx.z, S = gridDim.z;
  double p1[kTJ], p2[kTJ], acc[kTJ];
#pragma unroll
  for (int t = 0; t < kTJ; ++t) {
    const int j = min(j0 + t, N - 1);
    p1[t] = pint[2 * j];
    p2[t] = pint[2 * j + 1];
    acc[t] = 0.0;
  }
  const double *d = dens + (size_t)r * M;
  const int k0 = (int)((long long)M * sp / S), k1 = (int)((long long)M * (sp + 1) / S);
  for (int k = k0 + threadIdx.x; k < k1; k += kBlock) {
    const double2 q = xy[k];
    const double c = w[k] * d[k];
#pragma unroll
    for (int t = 0; t < kTJ; ++t) {
      const double dx = p1[t] - q.x, dy = p2[t] - q.y;
      acc[t] = fma(c, log(fma(dx, dx, dy * dy)), acc[t]);
    }
  }
  block_sums<kTJ>(acc, sh);
  if (threadIdx.x < kTJ && j0 + (int)threadIdx.x < N) {
    double v = acc[0];
#pragma unroll
    for (int t = 1; t < kTJ; ++t) v = (int)threadIdx.x == t ? acc[t] : v;
    part[((size_t)sp * nrhs + r) * N + j0 + threadIdx.x] = v;
  }
}

// phi_j = -(1/4 pi) sum (log |r|^2 = 2 log |r|, so S mu = -(1/2 pi) sum w mu log |r|)
__global__ void k_potential_fin(int N, int nrhs, int S, const double *__restrict__ part,
                                double *__restrict__ phi) {
  const long long i = (long long)blockIdx.x * kBlock + threadIdx.x;
  if (i >= (long long)N * nrhs) return;
  double v = 0.0;
  for (int sp = 0; sp < S; ++sp) v += part[(size_t)sp * N * nrhs + i];
  phi[i] = -v / (4.0 * kPi);
}

// Stokeslet velocity and the vorticity sum over the split's sources (raw sums u1, u2, om)
__global__ __launch_bounds__(kBlock) void k_rigid(int M, int N, int nrhs,
                                                 const double2 *__restrict__ xy,
                                                 const double *__restrict__ w,
                                                 const double *__restrict__ pint,
                                                 const double *__restrict__ dens,
                                                 double *__restrict__ part) {
  __shared__ double sh[4][3 * kTJ];
  const int j0 = blockIdx.x * kTJ, r = blockIdx.y, sp = blockIdx.z, S = gridDim.z;
  double p1[kTJ], p2[kTJ], acc[3 * kTJ];
#pragma unroll
  for (int t = 0; t < kTJ; ++t) {
    const int j = min(j0 + t, N - 1);
    p1[t] = pint[2 * j];
    p2[t] = pint[2 * j + 1];
    acc[3 * t] = acc[3 * t + 1] = acc[3 * t + 2] = 0.0;
  }
  const double *d = dens + (size_t)r * 2 * M;
  const int k0 = (int)((long long)M * sp / S), k1 = (int)((long long)M * (sp + 1) / S);
  for (int k = k0 + threadIdx.x; k < k1; k += kBlock) {
    const double2 q = xy[k];
    const double t1 = w[k] * d[2 * k], t2 = w[k] * d[2 * k + 1];
#pragma unroll
    for (int t = 0; t < kTJ; ++t) {
      const double dx = p1[t] - q.x, dy = p2[t] - q.y;
      const double rr = fma(dx, dx, dy * dy);
      const double lg = 0.5 * log(rr);
      const double inv = 1.0 / rr;
      const double rt = fma(dx, t1, dy * t2) * inv;
      acc[3 * t] += -lg * t1 + dx * rt;
      acc[3 * t + 1] += -lg * t2 + dy * rt;
      acc[3 * t + 2] += (dx * t2 - dy * t1) * inv;
    }
  }
  block_sums<3 * kTJ>(acc, sh);
  if (threadIdx.x < kTJ && j0 + (int)threadIdx.x < N) {
    const int t0 = threadIdx.x;
    double U1 = acc[0], U2 = acc[1], OM = acc[2];
#pragma unroll
    for (int t = 1; t < kTJ; ++t) {
      U1 = t0 == t ? acc[3 * t] : U1;
      U2 = t0 == t ? acc[3 * t + 1] : U2;
      OM = t0 == t ? acc[3 * t + 2] : OM;
    }
    double *o = part + (((size_t)sp * nrhs + r) * N + j0 + t0) * 3;
    o[0] = U1;
    o[1] = U2;
    o[2] = OM;
  }
}

// u = (1/4 pi) sums, omega = -(1/4 pi) om; v = u(p) - omega (p - x^c)^perp, a^perp = (-a2, a1)
__global__ void k_rigid_fin(int N, int nrhs, int S, const double *__restrict__ pint,
                            const double *__restrict__ xc, const double *__restrict__ yc,
                            const double *__restrict__ part, double *__restrict__ VW) {
  const long long i = (long long)blockIdx.x * kBlock + threadIdx.x;
  if (i >= (long long)N * nrhs) return;
  const int j = (int)(i % N);
  double U1 = 0.0, U2 = 0.0, OM = 0.0;
  for (int sp = 0; sp < S; ++sp) {
    const double *o = part + ((size_t)sp * N * nrhs + i) * 3;
    U1 += o[0];
    U2 += o[1];
    OM += o[2];
  }
  U1 /= 4.0 * kPi;
  U2 /= 4.0 * kPi;
  OM = -OM / (4.0 * kPi);
  const double e1 = pint[2 * j] - xc[j], e2 = pint[2 * j + 1] - yc[j];
  double *o = VW + 3 * i;
  o[0] = U1 + OM * e2;
  o[1] = U2 - OM * e1;
  o[2] = OM;
}

inline unsigned nblocks(long long n, int bs = kBlock) { return (unsigned)((n + bs - 1) / bs); }

template <int R>
void launch_far(bie_geom *g, int kind, int precision, const double *s64, const float *s32,
                double *partial, hipStream_t st, size_t off) {
  dim3 grid(nblocks(g->M), g->nsplit), block(kBlock);
  const int kc = kind == 0 ? (precision == BIE_MIXED ? BIE_K_FAR_LAPLACE_F32 : BIE_K_FAR_LAPLACE_F64)
                           : (precision == BIE_MIXED ? BIE_K_FAR_STOKES_F32 : BIE_K_FAR_STOKES_F64);
  ProfScope prof(kc, st, g->far_pairs * R);
  if (kind == 0) {
    if (precision == BIE_MIXED)
      hipLaunchKernelGGL(k_lap_far_f32<R>, grid, block, 0, st, g->M, g->body_ptr, g->body_of, g->xc,
                         g->yc, g->xr, s32 + off, g->nx, g->ny, g->split_body, partial);
    else
      hipLaunchKernelGGL(k_lap_far_f64<R>, grid, block, 0, st, g->M, g->body_ptr, g->body_of, g->xy,
                         s64 + off, g->nx, g->ny, g->split_body, partial);
  } else {
    if (precision == BIE_MIXED)
      hipLaunchKernelGGL(k_stk_far_f32<R>, grid, block, 0, st, g->M, g->body_ptr, g->body_of, g->xc,
                         g->yc, g->xr, reinterpret_cast<const float2 *>(s32 + off), g->nx, g->ny,
                         g->split_body, partial);
    else
      hipLaunchKernelGGL(k_stk_far_f64<R>, grid, block, 0, st, g->M, g->body_ptr, g->body_of, g->xy,
                         reinterpret_cast<const double2 *>(s64 + off), g->nx, g->ny,
                         g->split_body, partial);
  }
}

}  // namespace

int geometry_build(bie_geom *g, const double *curve, const double *interior, hipStream_t st) {
  hipLaunchKernelGGL(k_geometry, dim3(g->N), dim3(kBlock), 0, st, g->M, g->body_ptr, curve,
                     interior, g->x, g->y, g->nx, g->ny, g->w, g->kappa, g->px, g->py, g->len,
                     g->xc, g->yc, g->W, g->pint, g->area, g->xy, g->xr, g->body_of);
  hipLaunchKernelGGL(k_scale_length, dim3(1), dim3(kBlock), 0, st, g->M, g->x, g->y, g->dl_scale);
  BIE_HIP_CHECK(hipGetLastError());
  return BIE_OK;
}

// Workspace bytes of one apply: strengths s64 [nrhs][len], s32 [nrhs][len], then (64-byte
// aligned) the far-field partials [nsplit][maxR][len].
size_t apply_workspace_bytes(const bie_geom *g, int kind, int method, int nrhs) {
  const long long len = (long long)g->M * (kind == 0 ? 1 : 2);
  const int maxR = kind == 0 ? 8 : 4;
  const int nsplit = method == BIE_FMM ? 1 : g->nsplit;
  return (size_t)nrhs * len * (sizeof(double) + sizeof(float)) + 64 +
         (size_t)nsplit * maxR * len * sizeof(double);
}

// Far-field partials per rhs chunk and the epilogue. Chunks of <= 8 (Laplace) / 4 (Stokes) rhs
// share each pair's geometry work.
int apply_operator(bie_geom *g, int kind, int precision, int method, int with_L, double alpha,
                   int nrhs, const double *mu, double *out, hipStream_t st) {
  if (kind == 2 || kind == 3) return dl_apply(g, kind - 2, with_L, alpha, nrhs, mu, out, st);
  if (method == BIE_AUTO) method = method_is_fmm(method, g->M) ? BIE_FMM : BIE_DIRECT;
  if (nrhs < 1) {
    set_error("apply: nrhs >= 1 required");
    return BIE_EINVAL;
  }
  BIE_TRY(g->ws_apply.reserve(apply_workspace_bytes(g, kind, method, nrhs)));
  return apply_operator_ws(g, kind, precision, method, with_L, alpha, nrhs, mu, out,
                           g->ws_apply.ptr, g->ws_apply.bytes, st);
}

int apply_operator_ws(bie_geom *g, int kind, int precision, int method, int with_L,
                      double alpha, int nrhs, const double *mu, double *out, void *ws,
                      size_t ws_bytes, hipStream_t st) {
  if (precision != BIE_FP64 && precision != BIE_MIXED) {
    set_error("precision must be BIE_FP64 or BIE_MIXED");
    return BIE_EINVAL;
  }
  if (method == BIE_AUTO) method = method_is_fmm(method, g->M) ? BIE_FMM : BIE_DIRECT;
  if (method != BIE_DIRECT && method != BIE_FMM) {
    set_error("method must be BIE_DIRECT, BIE_FMM or BIE_AUTO");
    return BIE_EINVAL;
  }
  if (nrhs < 1 || !mu || !out) {
    set_error("apply: nrhs >= 1 and non-NULL mu, out required");
    return BIE_EINVAL;
  }
  const int comps = kind == 0 ? 1 : 2;
  const long long len = (long long)g->M * comps;
  const int maxR = kind == 0 ? 8 : 4;
  const int nsplit = method == BIE_FMM ? 1 : g->nsplit;
  if (!ws || ws_bytes < apply_workspace_bytes(g, kind, method, nrhs)) {
    set_error("apply: workspace too small");
    return BIE_EINVAL;
  }
  double *s64 = static_cast<double *>(ws);
  float *s32 = reinterpret_cast<float *>(s64 + (size_t)nrhs * len);
  double *partial = reinterpret_cast<double *>(
      (reinterpret_cast<uintptr_t>(s32 + (size_t)nrhs * len) + 63) & ~uintptr_t(63));
  const long long tot = (long long)nrhs * len;
  if (method != BIE_FMM) {  // the FMM gather forms the strengths itself
    hipLaunchKernelGGL(k_pack, dim3(nblocks(tot)), dim3(kBlock), 0, st, tot, g->M, comps, g->w, mu,
                       s64, precision == BIE_MIXED ? s32 : nullptr);
    BIE_HIP_CHECK(hipGetLastError());
  }
  for (int r0 = 0; r0 < nrhs;) {
    const int left = nrhs - r0;
    const int R = left >= maxR ? maxR : (left >= 4 ? 4 : (left >= 2 ? 2 : 1));
    const size_t off = (size_t)r0 * len;
    if (method == BIE_FMM) {
      const int leaf = precision == BIE_MIXED && g->fmm_leaf_mixed > 0 ? g->fmm_leaf_mixed
                                                                        : g->fmm_leaf;
      if (kind == 0) {  // the Laplace evaluation finishes the apply itself (no epilogue launch)
        FmmFinish fin;
        fin.mu = mu + off;
        fin.out = out + off;
        fin.alpha = alpha;
        fin.with_L = with_L;
        BIE_TRY(fmm_far_field(g, kind, precision, R, mu + off, s64 + off, partial, st,
                              g->fmm_order, leaf, &fin));
        r0 += R;
        continue;
      }
      BIE_TRY(fmm_far_field(g, kind, precision, R, mu + off, s64 + off, partial, st, g->fmm_order,
                            leaf));
    } else {
      switch (R) {
        case 8: launch_far<8>(g, kind, precision, s64, s32, partial, st, off); break;
        case 4: launch_far<4>(g, kind, precision, s64, s32, partial, st, off); break;
        case 2: launch_far<2>(g, kind, precision, s64, s32, partial, st, off); break;
        default: launch_far<1>(g, kind, precision, s64, s32, partial, st, off); break;
      }
      BIE_HIP_CHECK(hipGetLastError());
    }
    const int ntile = std::max(1, (g->max_nb + kBlock - 1) / kBlock);
    dim3 eg(g->N * ntile, R);
    ProfScope prof(BIE_K_EPILOGUE, st, 0);
    if (kind == 0)
      hipLaunchKernelGGL(k_lap_epilogue, eg, dim3(kBlock), 0, st, g->M, nsplit, R, ntile,
                         g->body_ptr, g->x, g->y, g->nx, g->ny, g->w, g->kappa, mu + off,
                         s64 + off, partial, with_L, method == BIE_FMM ? 0 : 1, alpha, out + off);
    else
      hipLaunchKernelGGL(k_stk_epilogue, eg, dim3(kBlock), 0, st, g->M, nsplit, R, ntile,
                         g->body_ptr, g->x, g->y, g->nx, g->ny, g->kappa, g->px, g->py, mu + off,
                         s64 + off, partial, with_L, method == BIE_FMM ? 0 : 1, alpha, out + off);
    BIE_HIP_CHECK(hipGetLastError());
    r0 += R;
  }
  return BIE_OK;
}

// out = D in (inverse: D^-1 in), D = diag(sqrt(w)) on every component of every node.
__global__ void k_scale_sqrtw(long long total, int M, int comps, const double *__restrict__ w,
                              int inverse, const double *__restrict__ in,
                              double *__restrict__ out) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= total) return;
  const int node = (int)((t % ((long long)M * comps)) / comps);
  const double d = sqrt(w[node]);
  out[t] = inverse ? in[t] / d : in[t] * d;
}

int scale_sqrtw(bie_geom *g, int comps, int nrhs, int inverse, const double *in, double *out,
                hipStream_t st) {
  const long long tot = (long long)nrhs * g->M * comps;
  hipLaunchKernelGGL(k_scale_sqrtw, dim3(nblocks(tot)), dim3(kBlock), 0, st, tot, g->M, comps,
                     g->w, inverse, in, out);
  BIE_HIP_CHECK(hipGetLastError());
  return BIE_OK;
}

int incident_density(bie_geom *g, int kind, int nrhs, const double *data, double *dens,
                     hipStream_t st) {
  const long long tot = (long long)nrhs * g->M;
  if (kind == 0)
    hipLaunchKernelGGL(k_sigma, dim3(nblocks(tot)), dim3(kBlock), 0, st, g->M, g->N, nrhs,
                       g->body_of, g->len, data, dens);
  else
    hipLaunchKernelGGL(k_rho, dim3(nblocks(tot)), dim3(kBlock), 0, st, g->M, g->N, nrhs,
                       g->body_of, g->len, g->W, g->px, g->py, data, dens);
  BIE_HIP_CHECK(hipGetLastError());
  return BIE_OK;
}

// Layer potentials of a total density at arbitrary points: Laplace u = S[dens], one value per
// point; Stokes the velocity of the Stokeslet sum (two values per point) or, with rigid (the
// interior read-off at the geometry's interior points), (v, omega) per body.
__global__ void k_velocity_fin(int N, int nrhs, int S, const double *__restrict__ part,
                               double *__restrict__ U) {
  const long long i = (long long)blockIdx.x * kBlock + threadIdx.x;
  if (i >= (long long)N * nrhs) return;
  double U1 = 0.0, U2 = 0.0;
  for (int sp = 0; sp < S; ++sp) {
    const double *o = part + ((size_t)sp * N * nrhs + i) * 3;
    U1 += o[0];
    U2 += o[1];
  }
  U[2 * i] = U1 / (4.0 * kPi);
  U[2 * i + 1] = U2 / (4.0 * kPi);
}

int eval_points(bie_geom *g, int kind, int nrhs, const double *dens, int npts, const double *pts,
                bool rigid, double *res, hipStream_t st, int method) {
  if (nrhs <= 0 || npts <= 0) return BIE_OK;
  if (method == BIE_AUTO) method = method_is_fmm(method, g->M) ? BIE_FMM : BIE_DIRECT;
  if (method == BIE_FMM) return fmm_eval_points(g, kind, nrhs, dens, npts, pts, rigid, res, st);
  // source splits: about 2048 workgroups in all, at most 32 splits, at least 2048 sources each
  const long long groups = (long long)((npts + kTJ - 1) / kTJ) * nrhs;
  int S = (int)std::max<long long>(1, std::min<long long>(32, (2048 + groups - 1) / groups));
  S = std::max(1, std::min(S, g->M / 2048));
  const int comps = kind == 0 ? 1 : 3;
  BIE_TRY(g->ws_read.reserve((size_t)S * nrhs * npts * comps * 8));
  double *part = g->ws_read.as<double>();
  dim3 grid((npts + kTJ - 1) / kTJ, nrhs, S);
  const unsigned fin = nblocks((long long)npts * nrhs);
  if (kind == 0) {
    hipLaunchKernelGGL(k_potential, grid, dim3(kBlock), 0, st, g->M, npts, nrhs, g->xy, g->w, pts,
                       dens, part);
    hipLaunchKernelGGL(k_potential_fin, dim3(fin), dim3(kBlock), 0, st, npts, nrhs, S, part, res);
  } else {
    hipLaunchKernelGGL(k_rigid, grid, dim3(kBlock), 0, st, g->M, npts, nrhs, g->xy, g->w, pts,
                       dens, part);
    if (rigid)
      hipLaunchKernelGGL(k_rigid_fin, dim3(fin), dim3(kBlock), 0, st, npts, nrhs, S, pts, g->xc,
                         g->yc, part, res);
    else
      hipLaunchKernelGGL(k_velocity_fin, dim3(fin), dim3(kBlock), 0, st, npts, nrhs, S, part, res);
  }
  BIE_HIP_CHECK(hipGetLastError());
  return BIE_OK;
}

int read_off(bie_geom *g, int kind, int nrhs, const double *dens, double *res, hipStream_t st,
             int method) {
  return eval_points(g, kind, nrhs, dens, g->N, g->pint, true, res, st, method);
}

}  // namespace bie

// ---- the apply without allocation ---------------------------------------------------------
// The direct apply's workspace (strengths and far-field partials) lives in this file-scope
// device array instead of memory the library allocates. Each device holds its own copy for the
// life of the process; host code uses only the device address that hipGetSymbolAddress returns
// for it (the array's name is a host-side stand-in, not a device address).
namespace bie {
namespace {

constexpr size_t kScratchBytes = (size_t)64 << 20;
constexpr int kMaxDevices = 64;
static __device__ __align__(256) char scratch[kScratchBytes];

std::mutex g_scratch_mu;
char *g_scratch_ptr[kMaxDevices] = {};

// The scratch address on the current device (looked up once per device, with it current).
int scratch_on_current_device(char **out) {
  int dev = -1;
  BIE_HIP_CHECK(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) {
    set_error("bie_apply_noalloc: device ordinal out of range");
    return BIE_EINVAL;
  }
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *p = nullptr;
    BIE_HIP_CHECK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    g_scratch_ptr[dev] = static_cast<char *>(p);
  }
  *out = g_scratch_ptr[dev];
  return BIE_OK;
}

}  // namespace
}  // namespace bie

extern "C" int bie_apply_noalloc(bie_geom *g, int kind, int precision, int with_L, int nrhs,
                                 const double *mu, double *out, void *stream) {
  using namespace bie;
  if (!g || (kind != 0 && kind != 1) || nrhs < 1 || !mu || !out || mu == out) {
    set_error("bie_apply_noalloc: need a geometry, kind 0 or 1, nrhs >= 1 and distinct "
              "non-NULL mu, out");
    return BIE_EINVAL;
  }
  if (precision != BIE_FP64 && precision != BIE_MIXED) {
    set_error("bie_apply_noalloc: precision must be BIE_FP64 or BIE_MIXED");
    return BIE_EINVAL;
  }
  const size_t need = apply_workspace_bytes(g, kind, BIE_DIRECT, nrhs);
  if (need > kScratchBytes) {
    set_error("bie_apply_noalloc: this apply needs " + std::to_string(need) +
              " bytes of scratch, more than its fixed " + std::to_string(kScratchBytes) +
              " (use fewer right-hand sides per call or bie_laplace_apply / bie_stokes_apply)");
    return BIE_EINVAL;
  }
  DeviceGuard dg(g->device);
  char *ws = nullptr;
  BIE_TRY(scratch_on_current_device(&ws));
  ProfSuspend quiet;  // profiling events would be created (allocated) on first use
  return apply_operator_ws(g, kind, precision, BIE_DIRECT, with_L ? 1 : 0, 1.0, nrhs, mu, out,
                           ws, kScratchBytes, reinterpret_cast<hipStream_t>(stream));
}
