// Block right preconditioner of the second-kind operators A = 1/2 I + K + L (Laplace, eq.
// ModRep2; Stokes, eq. ModRep2Stokes): GMRES solves (A P) u = f and x = P u, with P an
// approximation of the inverse of A's block diagonal (each body's interactions with itself:
// the identity, the smooth diagonal limit, the same-body double-layer pairs and the body's
// completion). The preconditioner changes the GMRES iterates, not the solution: every stopping
// test is on the true float64 residual of A x = f.
//
// Two-grid blocks. The inverse of a body's block is 2 I plus a smooth part (K and L have smooth
// kernels on a smooth closed curve), so the smooth part is formed on a coarse grid of the same
// curve: nc of the body's n nodes (every s-th, s = n / nc, with s-fold trapezoidal weights).
// With R the restriction of a fine density to the coarse nodes by trigonometric truncation (the
// modes |m| <= (nc - 1) / 2) and E the trigonometric interpolation back,
//   P_b = 2 I + E (B_b^-1 - 2 I) R,   B_b the coarse block,
// and P_b = B_b^-1 exactly when nc = n (bodies of at most kPcNodes nodes). When every body has at
// most kPcExact unknowns (C n, C = 1 Laplace, 2 Stokes) the blocks are not coarsened at all:
// the exact inverses are stored as int8 less the exact 2 I, with a float64 scale per row (an
// HBM-bound apply, faster there than the two-grid one). Both transfers are
// sampled Dirichlet kernels, R[j][k] = rho((j s - k) mod n) / n and E[i][j] = rho((i - j s) mod
// n) / nc with rho(d) = 1 + 2 sum_{m=1}^{(nc-1)/2} cos(2 pi m d / n), one table per (n, nc).
// The coarse blocks are inverted on the device in float32 (Gauss-Jordan without pivoting: the
// leading minors of 1/2 I + K + L stay near those of 1/2 I + L, which are positive) and stored
// in float32; the apply is float64 arithmetic on these fixed entries, so P is a fixed linear map.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <map>
#include <utility>

#include "internal.h"

namespace bie {
namespace {

constexpr int kPcNodes = 64;        // most coarse nodes per body
constexpr int kPcMinNodes = 16;     // fewest coarse nodes of a coarsened body
constexpr int kPcMaxFine = 2048;    // most nodes per body (the apply stages a body in LDS)
constexpr int kPcRows = 64;         // rows per thread in the inversion
constexpr int kPcExact = 256;       // most unknowns per body of the exact (uncoarsened) blocks

// Coarse blocks, column-major and padded to BJ x BJ (identity past the body's U = C nc unknowns;
// C = 1 Laplace, 2 Stokes, node-major components). Grid N, BJ threads: thread c forms column c.
// Coarse node j is fine node off + j s, with weight s w.
template <int BJ>
__global__ __launch_bounds__(BJ) void k_pc_blocks(
    int kind, const int *__restrict__ body_ptr, const int *__restrict__ ncoarse,
    const double *__restrict__ x, const double *__restrict__ y, const double *__restrict__ nx,
    const double *__restrict__ ny, const double *__restrict__ w, const double *__restrict__ kappa,
    const double *__restrict__ px, const double *__restrict__ py, float *__restrict__ inv) {
  const int b = blockIdx.x, c = threadIdx.x;
  const int off = body_ptr[b], n = body_ptr[b + 1] - off, nc = ncoarse[b], s = n / nc;
  const int C = kind == 0 ? 1 : 2, U = C * nc;
  float *col = inv + ((size_t)b * BJ + c) * BJ;
  const bool cin = c < U;
  const int k = c / C, cb = c % C, fk = off + k * s;
  const double xk = cin ? x[fk] : 0.0, yk = cin ? y[fk] : 0.0, wk = cin ? s * w[fk] : 0.0;
  const double pk = cin ? (cb == 0 ? px[fk] : py[fk]) : 0.0;
  for (int i = 0; i < BJ; ++i) {
    double v = i == c ? 1.0 : 0.0;
    if (cin && i < U) {
      const int j = i / C, a = i % C, fj = off + j * s;
      if (kind == 0) {
        if (j == k) {
          v = 0.5 - wk * kappa[fj] / (4.0 * kPi) + wk;
        } else {
          const double dx = x[fj] - xk, dy = y[fj] - yk;
          v = -wk * (nx[fj] * dx + ny[fj] * dy) / (2.0 * kPi * (dx * dx + dy * dy)) + wk;
        }
      } else {
        const double pa = a == 0 ? px[fj] : py[fj];
        double kab;
        if (j == k) {  // the smooth limit -(kappa / 2 pi) w tau_a tau_b, tau = (-n_y, n_x)
          const double ta = a == 0 ? -ny[fj] : nx[fj], tb = cb == 0 ? -ny[fj] : nx[fj];
          kab = -(kappa[fj] / (2.0 * kPi)) * wk * ta * tb;
        } else {
          const double dx = x[fj] - xk, dy = y[fj] - yk, rr = dx * dx + dy * dy;
          const double rn = dx * nx[fj] + dy * ny[fj];
          kab = -(1.0 / kPi) * rn / (rr * rr) * wk * (a == 0 ? dx : dy) * (cb == 0 ? dx : dy);
        }
        v = (i == c ? 0.5 : 0.0) + kab + wk * ((a == cb ? 1.0 : 0.0) + pa * pk);
      }
    }
    col[i] = (float)v;
  }
}

// In-place inversion of each padded block by Gauss-Jordan elimination without pivoting, one
// workgroup of BJ (BJ / 64) threads per body: thread t holds column t % BJ, rows
// 64 (t / BJ) .. 64 (t / BJ) + 63, in registers; the pivot row and column of each step are
// exchanged through LDS. Rows and columns past the body's U unknowns hold the identity and are
// never eliminated.
template <int BJ>
__global__ __launch_bounds__(BJ *(BJ / kPcRows)) void k_pc_invert(int kind,
                                                                 const int *__restrict__ ncoarse,
                                                                 float *__restrict__ inv) {
  __shared__ float rowk[BJ], colk[BJ];
  const int b = blockIdx.x;
  const int U = (kind == 0 ? 1 : 2) * ncoarse[b];
  const int c = threadIdx.x % BJ, rg = threadIdx.x / BJ, r0 = rg * kPcRows;
  float *o = inv + ((size_t)b * BJ + c) * BJ + r0;
  float a[kPcRows];
#pragma unroll
  for (int e = 0; e < kPcRows; e += 4) {
    const float4 q = *reinterpret_cast<const float4 *>(o + e);
    a[e] = q.x;
    a[e + 1] = q.y;
    a[e + 2] = q.z;
    a[e + 3] = q.w;
  }
  for (int k = 0; k < U; ++k) {
    if (c == k) {
#pragma unroll
      for (int e = 0; e < kPcRows; ++e) colk[r0 + e] = a[e];
    }
    if (rg == k / kPcRows) {
      const int ek = k % kPcRows;
#pragma unroll
      for (int e = 0; e < kPcRows; ++e)
        if (e == ek) rowk[c] = a[e];
    }
    __syncthreads();
    const float ip = 1.0f / rowk[k];
    const float rkj = rowk[c] * ip;  // the pivot row entry of this column, scaled
#pragma unroll
    for (int e = 0; e < kPcRows; ++e) {
      const int i = r0 + e;
      const float aik = colk[i];
      if (c == k)
        a[e] = i == k ? ip : -aik * ip;
      else
        a[e] = i == k ? rkj : fmaf(-aik, rkj, a[e]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int e = 0; e < kPcRows; e += 4)
    *reinterpret_cast<float4 *>(o + e) = make_float4(a[e], a[e + 1], a[e + 2], a[e + 3]);
}

// out = P in for one body and right-hand side per workgroup (grid (N, nrhs), NT threads). The
// body's fine values are staged in LDS as [component][k mod s][k / s], so that the
// restriction's reads at (j s - d) mod n are consecutive over j. Three products, each cut into
// `parts` ranges of its sum whose partial sums are added in range order: w = R v, y = B^-1 w,
// and out = 2 v + E (y - 2 w); with s = 1, out = B^-1 v. Dynamic LDS: (C + 1) n doubles.
template <int BJ, int NT>
__global__ __launch_bounds__(NT) void k_pc_apply(
    int kind, int M, const int *__restrict__ body_ptr, const int *__restrict__ ncoarse,
    const int *__restrict__ rho_off, const double *__restrict__ rho_tab,
    const float *__restrict__ inv, const double *__restrict__ in, double *__restrict__ out) {
  extern __shared__ double sm[];
  __shared__ double wv[2 * kPcNodes], yv[2 * kPcNodes], part[NT];
  const int b = blockIdx.x, r = blockIdx.y, t = threadIdx.x;
  const int off = body_ptr[b], n = body_ptr[b + 1] - off, nc = ncoarse[b], s = n / nc;
  const int C = kind == 0 ? 1 : 2, U = C * nc;
  const double *vin = in + (size_t)r * C * M + (size_t)C * off;
  double *vout = out + (size_t)r * C * M + (size_t)C * off;
  double *vs = sm, *rho = sm + (size_t)C * n;
  for (int e = t; e < C * n; e += NT) {
    const int k = e / C, a = e % C;
    vs[(a * s + k % s) * nc + k / s] = vin[e];
  }
  if (s > 1)
    for (int d = t; d < n; d += NT) rho[d] = rho_tab[rho_off[b] + d];
  __syncthreads();
  const int parts = NT / U;  // U <= 128: at least two
  // w = R v, in the block's node-major order (unknown C j + a)
  if (s == 1) {
    if (t < U) wv[t] = vs[(t % C) * nc + t / C];
  } else {
    double acc = 0.0;
    if (t < parts * U) {
      const int o = t % U, p = t / U, a = o / nc, j = o % nc;
      const int d0 = p * n / parts, d1 = (p + 1) * n / parts;
      int q = d0 / s, e = d0 % s;  // d = q s + e, so j s - d = (j - q) s - e
      for (int d = d0; d < d1; ++d) {
        const int km = e == 0 ? 0 : s - e;
        int kd = j - q - (e == 0 ? 0 : 1);
        kd += kd < 0 ? nc : 0;
        acc = fma(rho[d], vs[(a * s + km) * nc + kd], acc);
        if (++e == s) {
          e = 0;
          ++q;
        }
      }
    }
    part[t] = acc;
    __syncthreads();
    if (t < U) {
      double sum = 0.0;
      for (int p = 0; p < parts; ++p) sum += part[p * U + t];
      const int a = t / nc, j = t % nc;
      wv[C * j + a] = sum / (double)n;
    }
  }
  __syncthreads();
  // y = B^-1 w (column k of the stored inverse at inv[(b BJ + k) BJ + .])
  {
    double acc = 0.0;
    if (t < parts * U) {
      const int o = t % U, p = t / U;
      const int k0 = p * U / parts, k1 = (p + 1) * U / parts;
      const float *ib = inv + (size_t)b * BJ * BJ + o;
      for (int k = k0; k < k1; ++k) acc = fma((double)ib[(size_t)k * BJ], wv[k], acc);
    }
    part[t] = acc;
    __syncthreads();
    if (t < U) {
      double sum = 0.0;
      for (int p = 0; p < parts; ++p) sum += part[p * U + t];
      yv[t] = s == 1 ? sum : sum - 2.0 * wv[t];
    }
    __syncthreads();
  }
  if (s == 1) {
    if (t < U) vout[t] = yv[t];
    return;
  }
  // out = 2 v + E (y - 2 w): the sum over j cut into fparts ranges when the body has fewer
  // fine unknowns than threads
  const int F = C * n, fparts = F >= NT ? 1 : NT / F;
  const double inc = 1.0 / (double)nc;
  for (int e0 = 0; e0 < F; e0 += NT / fparts) {
    const int e = e0 + t % (NT / fparts), p = t / (NT / fparts);
    double acc = 0.0;
    if (e < F && p < fparts) {
      const int i = e / C, a = e % C;
      const int j0 = p * nc / fparts, j1 = (p + 1) * nc / fparts;
      int d = i - j0 * s;  // (i - j s) mod n
      d += d < 0 ? n : 0;
      for (int j = j0; j < j1; ++j) {
        acc = fma(rho[d], yv[C * j + a], acc);
        d -= s;
        d += d < 0 ? n : 0;
      }
    }
    if (fparts > 1) {
      __syncthreads();  // the previous pass has read part
      part[t] = acc;
      __syncthreads();
      if (t < NT / fparts && e < F) {
        double sum = 0.0;
        for (int q = 0; q < fparts; ++q) sum += part[q * (NT / fparts) + t];
        acc = sum;
      }
    }
    if (p == 0 && e < F) {
      const int i = e / C, a = e % C;
      vout[e] = fma(acc, inc, 2.0 * vs[(a * s + i % s) * nc + i / s]);
    }
  }
}

// The exact inverses as the int8 apply reads them: D_b = Inv_b - 2 I, each row scaled to its
// largest magnitude, s_i = max_k |D_b[i][k]| / 127, and rounded, q_ik = rint(D_b[i][k] / s_i);
// four consecutive entries of a row in one 32-bit word: word ((b BJ / 4 + k / 4) BJ + i) holds
// q_i,k .. q_i,k+3 (byte k % 4). Grid N, BJ threads: thread i forms row i. Scales [N][BJ].
template <int BJ>
__global__ __launch_bounds__(BJ) void k_pc_store_i8(int kind, const int *__restrict__ body_ptr,
                                                   const float *__restrict__ in,
                                                   unsigned *__restrict__ words,
                                                   double *__restrict__ scale) {
  const int b = blockIdx.x, i = threadIdx.x;
  const int U = (kind == 0 ? 1 : 2) * (body_ptr[b + 1] - body_ptr[b]);
  const float *col = in + (size_t)b * BJ * BJ + i;  // entry (i, k) at col[k BJ]
  float mx = 0.0f;
  if (i < U)
    for (int k = 0; k < U; ++k) mx = fmaxf(mx, fabsf(col[(size_t)k * BJ] - (k == i ? 2.0f : 0.0f)));
  const double sc = mx > 0.0f ? (double)mx / 127.0 : 1.0;
  scale[(size_t)b * BJ + i] = sc;
  const double isc = 1.0 / sc;
  unsigned *o = words + (size_t)b * (BJ / 4) * BJ + i;
  for (int k4 = 0; k4 < BJ; k4 += 4) {
    unsigned w = 0;
    for (int e = 0; e < 4; ++e) {
      const int k = k4 + e;
      int q = 0;
      if (i < U && k < U) {
        const double d = (double)col[(size_t)k * BJ] - (k == i ? 2.0 : 0.0);
        q = (int)rint(d * isc);
        q = q > 127 ? 127 : (q < -127 ? -127 : q);
      }
      w |= (unsigned)(q & 0xff) << (8 * e);
    }
    o[(size_t)(k4 / 4) * BJ] = w;
  }
}

// out = P in with the exact int8 inverses: out_b[i] = 2 in_b[i] + s_i sum_k q_ik in_b[k] (k
// ascending, float64 accumulation of the exact integer entries) over the body's U unknowns.
// Grid (N, ceil(nrhs / R)), BJ threads: thread i = row i reads its row's words, eight per batch
// of loads; R right-hand sides share each entry.
template <int BJ, int R>
__global__ __launch_bounds__(BJ) void k_pc_apply_i8(int kind, int M, int nrhs,
                                                   const int *__restrict__ body_ptr,
                                                   const unsigned *__restrict__ words,
                                                   const double *__restrict__ scale,
                                                   const double *__restrict__ in,
                                                   double *__restrict__ out) {
  __shared__ double v[R][BJ];
  const int C = kind == 0 ? 1 : 2;
  const int b = blockIdx.x, r0 = blockIdx.y * R, i = threadIdx.x;
  const int k0 = C * body_ptr[b], U = C * body_ptr[b + 1] - k0;
  const int nr = min(R, nrhs - r0);
  const size_t ld = (size_t)C * M;
#pragma unroll
  for (int r = 0; r < R; ++r) v[r][i] = (r < nr && i < U) ? in[(r0 + r) * ld + k0 + i] : 0.0;
  __syncthreads();
  if (i >= U) return;
  const unsigned *row = words + (size_t)b * (BJ / 4) * BJ + i;  // word p at row[p BJ]
  double acc[R];
#pragma unroll
  for (int r = 0; r < R; ++r) acc[r] = 0.0;
  const int nw = (U + 3) / 4;  // words; missing entries of the last one are zero
  int p = 0;
  for (; p + 8 <= nw; p += 8) {
    unsigned h[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) h[u] = row[(size_t)(p + u) * BJ];
#pragma unroll
    for (int u = 0; u < 8; ++u)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const double q = (double)(int)(signed char)(h[u] >> (8 * e));
#pragma unroll
        for (int r = 0; r < R; ++r) acc[r] = fma(q, v[r][4 * (p + u) + e], acc[r]);
      }
  }
  for (; p < nw; ++p) {
    const unsigned h = row[(size_t)p * BJ];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const double q = (double)(int)(signed char)(h >> (8 * e));
#pragma unroll
      for (int r = 0; r < R; ++r) acc[r] = fma(q, v[r][4 * p + e], acc[r]);
    }
  }
  const double sc = scale[(size_t)b * BJ + i];
#pragma unroll
  for (int r = 0; r < R; ++r)
    if (r < nr) out[(r0 + r) * ld + k0 + i] = fma(sc, acc[r], 2.0 * v[r][i]);
}

// Coarse node count of a body of n nodes: n itself up to kPcNodes, else the largest divisor of
// n not above kPcNodes; 0 when that is below kPcMinNodes or n exceeds kPcMaxFine.
int coarse_nodes(int n) {
  if (n <= kPcNodes) return n;
  if (n > kPcMaxFine) return 0;
  for (int nc = kPcNodes; nc >= kPcMinNodes; --nc)
    if (n % nc == 0) return nc;
  return 0;
}

}  // namespace

namespace {

template <int BJ>
int launch_blocks(bie_geom *g, int kind, const int *d_nc, float *inv, hipStream_t s) {
  hipLaunchKernelGGL(k_pc_blocks<BJ>, dim3(g->N), dim3(BJ), 0, s, kind, g->body_ptr, d_nc, g->x,
                     g->y, g->nx, g->ny, g->w, g->kappa, g->px, g->py, inv);
  hipLaunchKernelGGL(k_pc_invert<BJ>, dim3(g->N), dim3(BJ * (BJ / kPcRows)), 0, s, kind, d_nc,
                     inv);
  BIE_HIP_CHECK(hipGetLastError());
  return BIE_OK;
}

}  // namespace

int pc_build(bie_geom *g, int kind, hipStream_t s) {
  bie_geom::Precond &pc = g->pc[kind & 1];
  if (pc.ready) return BIE_OK;
  DeviceGuard dg(g->device);
  const int N = g->N, C = kind == 0 ? 1 : 2;
  int nmax = 1;
  for (int b = 0; b < N; ++b) nmax = std::max(nmax, g->h_body_ptr[b + 1] - g->h_body_ptr[b]);
  const bool exact = C * nmax <= kPcExact;
  std::vector<int> nc(N), roff(N, 0);
  std::map<std::pair<int, int>, int> tables;  // (n, nc) -> offset in rho_tab
  std::vector<double> rho_tab;
  int umax = 1;
  long long macs = 0;
  for (int b = 0; b < N; ++b) {
    const int n = g->h_body_ptr[b + 1] - g->h_body_ptr[b];
    nc[b] = exact ? n : coarse_nodes(n);
    if (nc[b] == 0) {
      set_error("block preconditioner: body " + std::to_string(b) + " has " + std::to_string(n) +
                " nodes; bodies of more than " + std::to_string(kPcNodes) +
                " nodes need a node count of at most " + std::to_string(kPcMaxFine) +
                " with a divisor in [" + std::to_string(kPcMinNodes) + ", " +
                std::to_string(kPcNodes) + "]");
      return BIE_EINVAL;
    }
    umax = std::max(umax, C * nc[b]);
    const long long U = (long long)C * nc[b];
    macs += U * U + (nc[b] < n ? 2LL * C * n * nc[b] : 0);
    if (nc[b] < n) {
      auto it = tables.find({n, nc[b]});
      if (it == tables.end()) {
        it = tables.emplace(std::make_pair(n, nc[b]), (int)rho_tab.size()).first;
        const int h = (nc[b] - 1) / 2;
        for (int d = 0; d < n; ++d) {
          double v = 1.0;
          for (int m = 1; m <= h; ++m)
            v += 2.0 * std::cos(2.0 * kPi * (double)((long long)m * d % n) / n);
          rho_tab.push_back(v);
        }
      }
      roff[b] = it->second;
    }
  }
  const int BJ = umax <= 64 ? 64 : umax <= 128 ? 128 : 256;
  const size_t fbytes = (size_t)N * BJ * BJ * sizeof(float);
  const size_t meta_bytes = 2 * (size_t)N * sizeof(int) + 256 + rho_tab.size() * sizeof(double) + 8;
  BIE_TRY(pc.inv.reserve(fbytes));
  BIE_TRY(pc.meta.reserve(meta_bytes));
  int *d_nc = pc.meta.as<int>(), *d_roff = d_nc + N;
  double *d_rho = reinterpret_cast<double *>(
      (reinterpret_cast<uintptr_t>(d_roff + N) + 255) & ~uintptr_t(255));
  BIE_HIP_CHECK(hipMemcpyAsync(d_nc, nc.data(), N * sizeof(int), hipMemcpyHostToDevice, s));
  BIE_HIP_CHECK(hipMemcpyAsync(d_roff, roff.data(), N * sizeof(int), hipMemcpyHostToDevice, s));
  if (!rho_tab.empty())
    BIE_HIP_CHECK(hipMemcpyAsync(d_rho, rho_tab.data(), rho_tab.size() * sizeof(double),
                                 hipMemcpyHostToDevice, s));
  float *inv = pc.inv.as<float>();
  if (BJ == 64) BIE_TRY(launch_blocks<64>(g, kind, d_nc, inv, s));
  else if (BJ == 128) BIE_TRY(launch_blocks<128>(g, kind, d_nc, inv, s));
  else BIE_TRY(launch_blocks<256>(g, kind, d_nc, inv, s));
  if (exact) {  // int8 words [N][BJ / 4][BJ], then the row scales [N][BJ]
    const size_t wbytes = (size_t)N * BJ * BJ;
    BIE_TRY(pc.q.reserve(wbytes + (size_t)N * BJ * sizeof(double)));
    unsigned *words = pc.q.as<unsigned>();
    double *scale = reinterpret_cast<double *>(pc.q.as<char>() + wbytes);
    if (BJ == 64)
      hipLaunchKernelGGL(k_pc_store_i8<64>, dim3(N), dim3(64), 0, s, kind, g->body_ptr, inv, words, scale);
    else if (BJ == 128)
      hipLaunchKernelGGL(k_pc_store_i8<128>, dim3(N), dim3(128), 0, s, kind, g->body_ptr, inv, words, scale);
    else
      hipLaunchKernelGGL(k_pc_store_i8<256>, dim3(N), dim3(256), 0, s, kind, g->body_ptr, inv, words, scale);
    BIE_HIP_CHECK(hipGetLastError());
  }
  BIE_HIP_CHECK(hipStreamSynchronize(s));  // the host tables go out of scope
  if (exact) pc.inv.release();             // only the int8 copy stays resident
  pc.exact = exact;
  pc.BJ = BJ;
  pc.ncoarse = d_nc;
  pc.rho_off = d_roff;
  pc.rho = d_rho;
  pc.macs = macs;
  pc.lds = (size_t)(C + 1) * nmax * sizeof(double);
  pc.ready = true;
  return BIE_OK;
}

namespace {

template <int BJ>
void launch_exact(const bie_geom *g, const bie_geom::Precond &pc, int kind, int nrhs,
                  const double *in, double *out, hipStream_t s) {
  constexpr int R = 4;
  const unsigned *words = pc.q.as<unsigned>();
  const double *scale =
      reinterpret_cast<const double *>(pc.q.as<char>() + (size_t)g->N * BJ * BJ);
  if (nrhs == 1)
    hipLaunchKernelGGL((k_pc_apply_i8<BJ, 1>), dim3(g->N, 1), dim3(BJ), 0, s, kind, g->M, nrhs,
                       g->body_ptr, words, scale, in, out);
  else
    hipLaunchKernelGGL((k_pc_apply_i8<BJ, R>), dim3(g->N, (nrhs + R - 1) / R), dim3(BJ), 0, s,
                       kind, g->M, nrhs, g->body_ptr, words, scale, in, out);
}

template <int BJ>
void launch_two_grid(const bie_geom *g, const bie_geom::Precond &pc, int kind, int nrhs,
                     const double *in, double *out, hipStream_t s) {
  // few bodies: 1024 threads per body shorten each one's sums; many: 256 threads, more
  // workgroups per compute unit
  if (g->N < 512)
    hipLaunchKernelGGL((k_pc_apply<BJ, 1024>), dim3(g->N, nrhs), dim3(1024), pc.lds, s, kind,
                       g->M, g->body_ptr, pc.ncoarse, pc.rho_off, pc.rho, pc.inv.as<float>(), in,
                       out);
  else
    hipLaunchKernelGGL((k_pc_apply<BJ, 256>), dim3(g->N, nrhs), dim3(256), pc.lds, s, kind, g->M,
                       g->body_ptr, pc.ncoarse, pc.rho_off, pc.rho, pc.inv.as<float>(), in, out);
}

}  // namespace

int pc_apply(bie_geom *g, int kind, int nrhs, const double *in, double *out, hipStream_t s) {
  const bie_geom::Precond &pc = g->pc[kind & 1];
  if (!pc.ready) {
    set_error("block preconditioner not built");
    return BIE_EINVAL;
  }
  // units: multiply-adds (exact blocks: one per stored entry; two-grid: restriction, coarse
  // product and interpolation) per right-hand side
  ProfScope prof(BIE_K_PRECOND, s, pc.macs * nrhs);
  if (pc.exact) {
    if (pc.BJ == 64) launch_exact<64>(g, pc, kind, nrhs, in, out, s);
    else if (pc.BJ == 128) launch_exact<128>(g, pc, kind, nrhs, in, out, s);
    else launch_exact<256>(g, pc, kind, nrhs, in, out, s);
  } else {
    if (pc.BJ == 64) launch_two_grid<64>(g, pc, kind, nrhs, in, out, s);
    else launch_two_grid<128>(g, pc, kind, nrhs, in, out, s);
  }
  BIE_HIP_CHECK(hipGetLastError());
  return BIE_OK;
}

}  // namespace bie
