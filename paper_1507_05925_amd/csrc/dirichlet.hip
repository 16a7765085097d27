// Capacitance and resistance problems: the inverse problems that the paper's numerical section
// solves to test the elastance and mobility solvers (prescribed potentials -> charges; prescribed
// rigid motions -> forces and torques). The paper leaves their equations to the literature; these
// are the classical completed double layers.
//
// Laplace: u = D[mu] + sum_j G_R(x, z_j) int_{Gamma_j} mu, with D[mu](x) = int dG/dn_y mu ds_y,
//   G = -(1/2pi) log|x - y|, G_R(x, z) = -(1/2pi) log(|x - z| / R); exterior boundary values give
//   (1/2 I + D + C) mu = f.
// Stokes: u = Dcal[mu] + sum_j [Gcal_R(x, z_j) a_j + t_j (x - z_j)^perp / (4 pi |x - z_j|^2)],
//   Dcal[mu](x) = (1/pi) int (r.n_y)(r.mu) r / |r|^4 ds_y (r = x - y), the Stokeslet
//   Gcal_R = (1/4pi)(-log(|d|/R) I + d d^T / |d|^2), a_j = int_{Gamma_j} mu,
//   t_j = int_{Gamma_j} ((y - z_j)^perp, mu).
// z_j are the geometry's interior points and R twice the diagonal of the nodes' bounding box.
// The equations hold any boundary data; the bounded solution of the physical problem (u tends to
// a constant, net charge / force zero) is a combination of the data solve with the solves for
// f = 1 (Laplace), resp. f = e_x and e_y (Stokes).
//
// The double-layer sweep is float64 over all pairs (the self pair masked without a branch; its
// smooth diagonal limit is added in the epilogue): lane = target, sources streamed through scalar
// registers, source range split over grid.y with one partial per split, summed in a fixed order.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>

#include "internal.h"

namespace bie {

namespace {

// float64 reciprocal: hardware estimate refined by one Newton step (about 2e-15 relative).
__device__ inline double rcp_nr(double a) {
  const double y = __builtin_amdgcn_rcp(a);
  const double e = fma(-a, y, 1.0);
  return fma(y, e, y);
}

__device__ inline double wg_sum(double v, double *sh) {
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

// Double-layer pair sums over the sources of split blockIdx.y, R densities at a time.
// Laplace: (1/2pi) sum_k w_k mu_k (r.n_k) / |r|^2; Stokes: (1/pi) sum_k (r.n_k)(r.w_k mu_k) r / |r|^4.
template <bool STOKES, int R>
__global__ __launch_bounds__(kBlock) void k_dl_sweep(int M, int S, const double2 *__restrict__ xy,
                                                     const double *__restrict__ nx,
                                                     const double *__restrict__ ny,
                                                     const double *__restrict__ w,
                                                     const double *__restrict__ mu, long long len,
                                                     double *__restrict__ partial) {
  const int sp = blockIdx.y;
  const int i = blockIdx.x * kBlock + threadIdx.x;
  const bool valid = i < M;
  const int ii = valid ? i : M - 1;
  const double2 p = xy[ii];
  const int k0 = (int)((long long)M * sp / S), k1 = (int)((long long)M * (sp + 1) / S);
  double g1[R], g2[R];
#pragma unroll
  for (int r = 0; r < R; ++r) g1[r] = g2[r] = 0.0;
#pragma unroll 2
  for (int k = k0; k < k1; ++k) {
    const double2 q = xy[k];
    const double dx = p.x - q.x, dy = p.y - q.y;
    const double rr = fma(dx, dx, dy * dy);
    const double inv = k == ii ? 0.0 : rcp_nr(rr);  // self pair: r = 0, contributes nothing
    const double rn = fma(dx, nx[k], dy * ny[k]) * inv * w[k];
    if (!STOKES) {
#pragma unroll
      for (int r = 0; r < R; ++r) g1[r] = fma(rn, mu[(size_t)r * len + k], g1[r]);
    } else {
      const double a = rn * inv;
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const double m1 = mu[(size_t)r * len + 2 * k], m2 = mu[(size_t)r * len + 2 * k + 1];
        const double c = fma(dx, m1, dy * m2) * a;
        g1[r] = fma(c, dx, g1[r]);
        g2[r] = fma(c, dy, g2[r]);
      }
    }
  }
  if (!valid) return;
#pragma unroll
  for (int r = 0; r < R; ++r) {
    double *o = partial + ((size_t)sp * R + r) * len;
    if (!STOKES) {
      o[i] = g1[r] / (2.0 * kPi);
    } else {
      o[2 * i] = g1[r] / kPi;
      o[2 * i + 1] = g2[r] / kPi;
    }
  }
}

// Per (body, density): Laplace int mu (one value); Stokes a = int mu (two) and
// t = int ((y - z)^perp, mu) about the body's interior point z.
template <bool STOKES>
__global__ __launch_bounds__(kBlock) void k_dl_moments(int N, const int *__restrict__ body_ptr,
                                                       const double *__restrict__ x,
                                                       const double *__restrict__ y,
                                                       const double *__restrict__ w,
                                                       const double *__restrict__ pint,
                                                       const double *__restrict__ mu,
                                                       long long len, double *__restrict__ mom) {
  __shared__ double sh[4];
  const int b = blockIdx.x, r = blockIdx.y;
  const int k0 = body_ptr[b], k1 = body_ptr[b + 1];
  const double *m = mu + (size_t)r * len;
  const double zx = pint[2 * b], zy = pint[2 * b + 1];
  double a1 = 0.0, a2 = 0.0, t = 0.0;
  for (int k = k0 + threadIdx.x; k < k1; k += kBlock) {
    if (!STOKES) {
      a1 += w[k] * m[k];
    } else {
      const double m1 = w[k] * m[2 * k], m2 = w[k] * m[2 * k + 1];
      a1 += m1;
      a2 += m2;
      t += (x[k] - zx) * m2 - (y[k] - zy) * m1;
    }
  }
  a1 = wg_sum(a1, sh);
  if (STOKES) {
    a2 = wg_sum(a2, sh);
    t = wg_sum(t, sh);
  }
  if (threadIdx.x == 0) {
    if (!STOKES) {
      mom[(size_t)r * N + b] = a1;
    } else {
      double *o = mom + ((size_t)r * N + b) * 3;
      o[0] = a1;
      o[1] = a2;
      o[2] = t;
    }
  }
}

// out = alpha (1/2 mu + diagonal limit + sum of the split partials + completion), one lane per
// node, grid.y = density. The completion loops over all bodies (wave-uniform).
template <bool STOKES>
__global__ __launch_bounds__(kBlock) void k_dl_epilogue(
    int M, int N, int S, int R, const double2 *__restrict__ xy, const double *__restrict__ nx,
    const double *__restrict__ ny, const double *__restrict__ w, const double *__restrict__ kappa,
    const double *__restrict__ pint, const double *__restrict__ scale, const double *__restrict__ mu,
    long long len, const double *__restrict__ partial, const double *__restrict__ mom,
    int with_C, double alpha, double *__restrict__ out) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  const int r = blockIdx.y;
  if (i >= M) return;
  const double2 p = xy[i];
  const double logR = log(scale[0]);
  const double *m = mu + (size_t)r * len;
  if (!STOKES) {
    double c = 0.0, tot = 0.0;
    if (with_C) {
      const double *A = mom + (size_t)r * N;
      for (int b = 0; b < N; ++b) {
        const double dx = p.x - pint[2 * b], dy = p.y - pint[2 * b + 1];
        c = fma(A[b], log(fma(dx, dx, dy * dy)), c);
        tot += A[b];
      }
    }
    const double comp = -(0.5 * c - logR * tot) / (2.0 * kPi);
    double far = 0.0;
    for (int sp = 0; sp < S; ++sp) far += partial[((size_t)sp * R + r) * len + i];
    const double mi = m[i];
    const double dg = -kappa[i] * w[i] / (4.0 * kPi) * mi;
    out[(size_t)r * len + i] = alpha * (0.5 * mi + dg + far + comp);
  } else {
    double u1 = 0.0, u2 = 0.0;
    if (with_C) {
      const double *A = mom + (size_t)r * N * 3;
      for (int b = 0; b < N; ++b) {
        const double dx = p.x - pint[2 * b], dy = p.y - pint[2 * b + 1];
        const double dd = fma(dx, dx, dy * dy);
        const double inv = 1.0 / dd;
        const double lg = 0.5 * log(dd) - logR;
        const double a1 = A[3 * b], a2 = A[3 * b + 1], t = A[3 * b + 2];
        const double da = fma(dx, a1, dy * a2) * inv;
        u1 += -lg * a1 + dx * da - t * dy * inv;
        u2 += -lg * a2 + dy * da + t * dx * inv;
      }
    }
    double f1 = 0.0, f2 = 0.0;
    for (int sp = 0; sp < S; ++sp) {
      const double *o = partial + ((size_t)sp * R + r) * len;
      f1 += o[2 * i];
      f2 += o[2 * i + 1];
    }
    const double m1 = m[2 * i], m2 = m[2 * i + 1];
    const double tx = -ny[i], ty = nx[i];  // unit tangent (n = (tau_2, -tau_1))
    const double d = -kappa[i] * w[i] / (2.0 * kPi) * fma(tx, m1, ty * m2);
    double *o = out + (size_t)r * len;
    o[2 * i] = alpha * (0.5 * m1 + d * tx + f1 + u1 / (4.0 * kPi));
    o[2 * i + 1] = alpha * (0.5 * m2 + d * ty + f2 + u2 / (4.0 * kPi));
  }
}

// Boundary data of the capacitance systems: rows r < nrhs hold phi_{body(i)}, the last row 1.
__global__ void k_cap_rhs(int M, int N, int nrhs, const int *__restrict__ body_of,
                          const double *__restrict__ phi, double *__restrict__ f) {
  const long long t = (long long)blockIdx.x * kBlock + threadIdx.x;
  if (t >= (long long)(nrhs + 1) * M) return;
  const int r = (int)(t / M), i = (int)(t % M);
  f[t] = r < nrhs ? phi[(size_t)r * N + body_of[i]] : 1.0;
}

// Resistance systems: rows r < nrhs hold v_j + omega_j (x - x^c_j)^perp, then e_x and e_y.
__global__ void k_res_rhs(int M, int N, int nrhs, const int *__restrict__ body_of,
                          const double *__restrict__ px, const double *__restrict__ py,
                          const double *__restrict__ VW, double *__restrict__ f) {
  const long long t = (long long)blockIdx.x * kBlock + threadIdx.x;
  if (t >= (long long)(nrhs + 2) * M) return;
  const int r = (int)(t / M), i = (int)(t % M);
  double u1, u2;
  if (r < nrhs) {
    const double *v = VW + ((size_t)r * N + body_of[i]) * 3;
    u1 = v[0] + v[2] * px[i];
    u2 = v[1] + v[2] * py[i];
  } else {
    u1 = r == nrhs ? 1.0 : 0.0;
    u2 = r == nrhs ? 0.0 : 1.0;
  }
  f[(size_t)r * 2 * M + 2 * i] = u1;
  f[(size_t)r * 2 * M + 2 * i + 1] = u2;
}

// Bounded capacitance solution of density r (one workgroup each): beta = sum q~[r] / sum q~[1],
// q = q~[r] - beta q~[1], u_inf = beta.
__global__ __launch_bounds__(kBlock) void k_cap_combine(int N, int nrhs,
                                                        const double *__restrict__ mom,
                                                        double *__restrict__ q,
                                                        double *__restrict__ u_inf,
                                                        double *__restrict__ beta) {
  __shared__ double sh[4];
  const int r = blockIdx.x;
  const double *A = mom + (size_t)r * N, *A1 = mom + (size_t)nrhs * N;
  double s = 0.0, s1 = 0.0;
  for (int b = threadIdx.x; b < N; b += kBlock) {
    s += A[b];
    s1 += A1[b];
  }
  s = wg_sum(s, sh);
  s1 = wg_sum(s1, sh);
  const double be = s / s1;
  for (int b = threadIdx.x; b < N; b += kBlock) q[(size_t)r * N + b] = A[b] - be * A1[b];
  if (threadIdx.x == 0) {
    u_inf[r] = be;
    beta[2 * r] = be;
    beta[2 * r + 1] = 0.0;
  }
}

// Bounded resistance solution of density r: beta solves [sum a[e_x], sum a[e_y]] beta = sum a[r];
// F = a[r] - beta_1 a[e_x] - beta_2 a[e_y] (likewise t); torque about the centroid
// T = t + (z - x^c) x F; u_inf = beta.
__global__ __launch_bounds__(kBlock) void k_res_combine(int N, int nrhs,
                                                        const double *__restrict__ mom,
                                                        const double *__restrict__ pint,
                                                        const double *__restrict__ xc,
                                                        const double *__restrict__ yc,
                                                        double *__restrict__ FT,
                                                        double *__restrict__ u_inf,
                                                        double *__restrict__ beta) {
  __shared__ double sh[4];
  const int r = blockIdx.x;
  const double *A = mom + (size_t)r * N * 3, *X = mom + (size_t)nrhs * N * 3,
               *Y = mom + (size_t)(nrhs + 1) * N * 3;
  double s1 = 0.0, s2 = 0.0, x1 = 0.0, x2 = 0.0, y1 = 0.0, y2 = 0.0;
  for (int b = threadIdx.x; b < N; b += kBlock) {
    s1 += A[3 * b];
    s2 += A[3 * b + 1];
    x1 += X[3 * b];
    x2 += X[3 * b + 1];
    y1 += Y[3 * b];
    y2 += Y[3 * b + 1];
  }
  s1 = wg_sum(s1, sh);
  s2 = wg_sum(s2, sh);
  x1 = wg_sum(x1, sh);
  x2 = wg_sum(x2, sh);
  y1 = wg_sum(y1, sh);
  y2 = wg_sum(y2, sh);
  const double det = x1 * y2 - y1 * x2;
  const double b1 = (s1 * y2 - y1 * s2) / det, b2 = (x1 * s2 - s1 * x2) / det;
  for (int b = threadIdx.x; b < N; b += kBlock) {
    const double F1 = A[3 * b] - b1 * X[3 * b] - b2 * Y[3 * b];
    const double F2 = A[3 * b + 1] - b1 * X[3 * b + 1] - b2 * Y[3 * b + 1];
    const double t = A[3 * b + 2] - b1 * X[3 * b + 2] - b2 * Y[3 * b + 2];
    const double e1 = pint[2 * b] - xc[b], e2 = pint[2 * b + 1] - yc[b];
    double *o = FT + ((size_t)r * N + b) * 3;
    o[0] = F1;
    o[1] = F2;
    o[2] = t + e1 * F2 - e2 * F1;
  }
  if (threadIdx.x == 0) {
    u_inf[2 * r] = b1;
    u_inf[2 * r + 1] = b2;
    beta[2 * r] = b1;
    beta[2 * r + 1] = b2;
  }
}

// Density of the bounded solution: mu[r] - beta_1 mu[nrhs] (- beta_2 mu[nrhs + 1] for Stokes).
__global__ void k_dl_density(long long len, int nrhs, int extra, const double *__restrict__ beta,
                             const double *__restrict__ mu, double *__restrict__ out) {
  const long long t = (long long)blockIdx.x * kBlock + threadIdx.x;
  if (t >= (long long)nrhs * len) return;
  const int r = (int)(t / len);
  const long long j = t % len;
  double v = mu[t] - beta[2 * r] * mu[(size_t)nrhs * len + j];
  if (extra == 2) v -= beta[2 * r + 1] * mu[(size_t)(nrhs + 1) * len + j];
  out[t] = v;
}

inline unsigned nb(long long n) { return (unsigned)((n + kBlock - 1) / kBlock); }

// source splits: about 1024 workgroups, each split at least 256 sources
int dl_splits(int M) {
  const int tb = (M + kBlock - 1) / kBlock;
  int S = std::max(1, std::min(32, (1024 + tb - 1) / tb));
  return std::max(1, std::min(S, M / 256));
}

template <bool STOKES, int R>
void launch_sweep(bie_geom *g, int S, const double *mu, long long len, double *partial,
                  hipStream_t st) {
  hipLaunchKernelGGL((k_dl_sweep<STOKES, R>), dim3(nb(g->M), S), dim3(kBlock), 0, st, g->M, S,
                     g->xy, g->nx, g->ny, g->w, mu, len, partial);
}

template <bool STOKES>
void sweep_chunk(bie_geom *g, int S, int R, const double *mu, long long len, double *partial,
                 hipStream_t st) {
  switch (R) {
    case 8: launch_sweep<STOKES, 8>(g, S, mu, len, partial, st); break;
    case 4: launch_sweep<STOKES, 4>(g, S, mu, len, partial, st); break;
    case 2: launch_sweep<STOKES, 2>(g, S, mu, len, partial, st); break;
    default: launch_sweep<STOKES, 1>(g, S, mu, len, partial, st); break;
  }
}

int dl_moments(bie_geom *g, int stokes, int nrhs, const double *mu, double *mom, hipStream_t st) {
  const long long len = stokes ? 2LL * g->M : g->M;
  if (stokes)
    hipLaunchKernelGGL(k_dl_moments<true>, dim3(g->N, nrhs), dim3(kBlock), 0, st, g->N,
                       g->body_ptr, g->x, g->y, g->w, g->pint, mu, len, mom);
  else
    hipLaunchKernelGGL(k_dl_moments<false>, dim3(g->N, nrhs), dim3(kBlock), 0, st, g->N,
                       g->body_ptr, g->x, g->y, g->w, g->pint, mu, len, mom);
  BIE_HIP_CHECK(hipGetLastError());
  return BIE_OK;
}

}  // namespace

int dl_apply(bie_geom *g, int stokes, int with_C, double alpha, int nrhs, const double *mu,
             double *out, hipStream_t st) {
  if (nrhs < 1 || !mu || !out) {
    set_error("double-layer apply: nrhs >= 1 and non-NULL mu, out required");
    return BIE_EINVAL;
  }
  const int comps = stokes ? 2 : 1, C = stokes ? 3 : 1;
  const long long len = (long long)g->M * comps;
  const int maxR = stokes ? 4 : 8;
  const int S = dl_splits(g->M);
  // workspace: partial [S][maxR][len], moments [nrhs][N][C]
  const size_t need = ((size_t)S * maxR * len + (size_t)nrhs * g->N * C) * sizeof(double);
  BIE_TRY(g->ws_apply.reserve(need));
  double *partial = g->ws_apply.as<double>();
  double *mom = partial + (size_t)S * maxR * len;
  ProfScope prof(BIE_K_DOUBLE_LAYER, st, (long long)nrhs * g->M * (long long)g->M);
  if (with_C) BIE_TRY(dl_moments(g, stokes, nrhs, mu, mom, st));
  for (int r0 = 0; r0 < nrhs;) {
    const int left = nrhs - r0;
    const int R = left >= maxR ? maxR : (left >= 4 ? 4 : (left >= 2 ? 2 : 1));
    const size_t off = (size_t)r0 * len;
    if (stokes)
      sweep_chunk<true>(g, S, R, mu + off, len, partial, st);
    else
      sweep_chunk<false>(g, S, R, mu + off, len, partial, st);
    BIE_HIP_CHECK(hipGetLastError());
    const double *mo = mom + (size_t)r0 * g->N * C;
    if (stokes)
      hipLaunchKernelGGL(k_dl_epilogue<true>, dim3(nb(g->M), R), dim3(kBlock), 0, st, g->M, g->N,
                         S, R, g->xy, g->nx, g->ny, g->w, g->kappa, g->pint, g->dl_scale,
                         mu + off, len, partial, mo, with_C, alpha, out + off);
    else
      hipLaunchKernelGGL(k_dl_epilogue<false>, dim3(nb(g->M), R), dim3(kBlock), 0, st, g->M,
                         g->N, S, R, g->xy, g->nx, g->ny, g->w, g->kappa, g->pint, g->dl_scale,
                         mu + off, len, partial, mo, with_C, alpha, out + off);
    BIE_HIP_CHECK(hipGetLastError());
    r0 += R;
  }
  return BIE_OK;
}

int dl_solve(bie_geom *g, int stokes, int nrhs, const double *data, double *res, double *u_inf,
             double *mu_out, const bie_opts &opts, bie_info *info, hipStream_t s) {
  const int extra = stokes ? 2 : 1, C = stokes ? 3 : 1;
  const int nsys = nrhs + extra;
  const long long len = stokes ? 2LL * g->M : g->M;
  bie_opts o = opts;
  o.precision = BIE_FP64;  // the double-layer apply is float64 only
  o.method = BIE_DIRECT;
  // ws_out: f [nsys][len], mu [nsys][len]; ws_read: moments [nsys][N][C], beta [nrhs][2]
  BIE_TRY(g->ws_out.reserve(2 * (size_t)nsys * len * 8));
  double *f = g->ws_out.as<double>();
  double *mu = f + (size_t)nsys * len;
  BIE_TRY(g->ws_read.reserve(((size_t)nsys * g->N * C + 2 * (size_t)nrhs) * 8));
  double *mom = g->ws_read.as<double>();
  double *beta = mom + (size_t)nsys * g->N * C;
  if (stokes)
    hipLaunchKernelGGL(k_res_rhs, dim3(nb((long long)nsys * g->M)), dim3(kBlock), 0, s, g->M,
                       g->N, nrhs, g->body_of, g->px, g->py, data, f);
  else
    hipLaunchKernelGGL(k_cap_rhs, dim3(nb((long long)nsys * g->M)), dim3(kBlock), 0, s, g->M,
                       g->N, nrhs, g->body_of, data, f);
  BIE_HIP_CHECK(hipGetLastError());
  int rc = solve_system(g, stokes ? 3 : 2, o, nsys, f, mu, info, s);
  if (rc != BIE_OK && rc != BIE_ENOCONV) return rc;
  BIE_TRY(dl_moments(g, stokes, nsys, mu, mom, s));
  if (stokes)
    hipLaunchKernelGGL(k_res_combine, dim3(nrhs), dim3(kBlock), 0, s, g->N, nrhs, mom, g->pint,
                       g->xc, g->yc, res, u_inf, beta);
  else
    hipLaunchKernelGGL(k_cap_combine, dim3(nrhs), dim3(kBlock), 0, s, g->N, nrhs, mom, res, u_inf,
                       beta);
  BIE_HIP_CHECK(hipGetLastError());
  if (mu_out) {
    hipLaunchKernelGGL(k_dl_density, dim3(nb((long long)nrhs * len)), dim3(kBlock), 0, s, len,
                       nrhs, extra, beta, mu, mu_out);
    BIE_HIP_CHECK(hipGetLastError());
  }
  return rc;
}

}  // namespace bie
