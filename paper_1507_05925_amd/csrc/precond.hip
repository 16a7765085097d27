// Block right preconditioner of the second-kind operators A = 1/2 I + K + L (Laplace, eq.
// ModRep2; Stokes, eq. ModRep2Stokes): GMRES solves (A P) u = f and x = P u, with P an
// approximation of the inverse of A's block diagonal (each body's interactions with itself:
// the identity, the smooth diagonal limit, the same-body double-layer pairs and the body's
// completion). The preconditioner changes the GMRES iterates, not the solution: every stopping
// test is on the true float64 residual of A x = f.
//
// Two-grid blocks. The inverse of a body's block is 2 I plus a smooth part (K and L have smooth
// kernels on a smooth closed curve), so the smooth part is formed on a coarse grid of the same
// curve: nc of the body's n nodes (every s-th, s = n / nc, with s-fold trapezoidal weights;
// nc = n for bodies of at most kPcNodes nodes). With R the full-weighting restriction to the
// coarse nodes and E the linear interpolation back (the standard multigrid pair),
//   P_b = 2 I + E (B_b^-1 - 2 I) R,   B_b the coarse block,
// and P_b = B_b^-1 exactly when nc = n. The coarse blocks are inverted on the device in float32
// (Gauss-Jordan without pivoting: the leading minors of 1/2 I + K + L stay near those of
// 1/2 I + L, which are positive) and stored in float32; the apply is float64 arithmetic on these
// fixed entries and fixed weights, so P is a fixed linear map.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "internal.h"

namespace bie {
namespace {

constexpr int kPcNodes = 64;        // most coarse nodes per body
constexpr int kPcMinNodes = 16;     // fewest coarse nodes of a coarsened body
constexpr int kPcMaxFine = 2048;    // most nodes per body (the apply stages a body in LDS)
constexpr int kPcRows = 64;         // rows per thread in the inversion

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

// bad[b] = 1 when body b's inverted coarse block holds a non-finite entry (a vanishing pivot of
// the elimination without pivoting), else 0. Grid N, BJ threads: thread c checks column c.
template <int BJ>
__global__ __launch_bounds__(BJ) void k_pc_check(int kind, const int *__restrict__ ncoarse,
                                                const float *__restrict__ inv,
                                                int *__restrict__ bad) {
  __shared__ int any;
  const int b = blockIdx.x, c = threadIdx.x;
  const int U = (kind == 0 ? 1 : 2) * ncoarse[b];
  if (c == 0) any = 0;
  __syncthreads();
  if (c < U) {
    const float *col = inv + ((size_t)b * BJ + c) * BJ;
    bool ok = true;
    for (int i = 0; i < U; ++i) ok = ok && isfinite(col[i]);
    if (!ok) any = 1;  // a benign race: every writer stores 1
  }
  __syncthreads();
  if (c == 0) bad[b] = any;
}

// out = P in for body b of one geometry and right-hand side r (in and out point at the
// geometry's [nrhs][C M] block), by one workgroup of NT threads, the body's values staged in LDS
// (vs, C n doubles) in their node-major order. Coarse node j is fine node j s; the restriction is
// full weighting, w_j = sum_{|d| < s} (1 - |d| / s) v_{j s + d} / s (indices mod n), the
// interpolation linear, (E y)_i = (1 - t) y_{i / s} + t y_{i / s + 1} with t = (i mod s) / s;
// then y = B^-1 w (the sum over k cut into `parts` ranges whose partial sums are added in range
// order) and out = 2 v + E (y - 2 w); with s = 1, out = B^-1 v.
template <int NT>
__device__ void pc_body(int kind, int M, int b, int r, const int *__restrict__ body_ptr,
                        const int *__restrict__ ncoarse, const float *__restrict__ inv, int BJ,
                        const double *in, double *out, double *vs, double *wv, double *yv,
                        double *part) {  // in == out allowed: the body is staged first
  const int t = threadIdx.x;
  const int off = body_ptr[b], n = body_ptr[b + 1] - off, nc = ncoarse[b], s = n / nc;
  const int C = kind == 0 ? 1 : 2, U = C * nc, F = C * n;
  const double *vin = in + (size_t)r * C * M + (size_t)C * off;
  double *vout = out + (size_t)r * C * M + (size_t)C * off;
  for (int e = t; e < F; e += NT) vs[e] = vin[e];
  __syncthreads();
  // w = R v, node-major (unknown C j + a)
  if (t < U) {
    const int j = t / C, a = t % C, c = j * s;
    double acc = 0.0;
    if (s == 1) {
      acc = vs[t];
    } else {
      const double is = 1.0 / (double)s;
      for (int d = 1 - s; d < s; ++d) {
        int k = c + d;
        k += k < 0 ? n : 0;
        k -= k >= n ? n : 0;
        acc = fma((1.0 - (double)abs(d) * is) * is, vs[C * k + a], acc);
      }
    }
    wv[t] = acc;
  }
  __syncthreads();
  // y = B^-1 w (column k of the stored inverse at inv[(b BJ + k) BJ + .])
  const int parts = NT / U;  // U <= 128: at least two
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
  if (s == 1) {
    if (t < U) vout[t] = yv[t];
    return;
  }
  const double is = 1.0 / (double)s;
  for (int e = t; e < F; e += NT) {
    const int i = e / C, a = e % C, j0 = i / s, j1 = j0 + 1 == nc ? 0 : j0 + 1;
    const double tt = (double)(i - j0 * s) * is;
    vout[e] = fma(tt, yv[C * j1 + a], fma(1.0 - tt, yv[C * j0 + a], 2.0 * vs[e]));
  }
}

// One geometry: grid (N, nrhs). Dynamic LDS: C n_max doubles.
template <int NT>
__global__ __launch_bounds__(NT) void k_pc_apply(int kind, int M, int BJ,
                                                 const int *__restrict__ body_ptr,
                                                 const int *__restrict__ ncoarse,
                                                 const float *__restrict__ inv,
                                                 const double *in,
                                                 double *out) {  // in == out allowed
  extern __shared__ double vs[];
  __shared__ double wv[2 * kPcNodes], yv[2 * kPcNodes], part[NT];
  pc_body<NT>(kind, M, blockIdx.x, blockIdx.y, body_ptr, ncoarse, inv, BJ, in, out, vs, wv, yv,
              part);
}

// A batch of geometries in one launch: workgroup w belongs to the item i with
// items[i].block0 <= w < items[i + 1].block0 (binary search), and takes its body
// (w - block0) mod N and right-hand side (w - block0) / N. Dynamic LDS: C n_max doubles over the
// items.
template <int NT>
__global__ __launch_bounds__(NT) void k_pc_apply_batch(int nitems,
                                                       const PcBatchItem *__restrict__ items,
                                                       const double *in,
                                                       double *out) {  // in == out allowed
  extern __shared__ double vs[];
  __shared__ double wv[2 * kPcNodes], yv[2 * kPcNodes], part[NT];
  const int w = blockIdx.x;
  int lo = 0, hi = nitems - 1;  // the last item whose block0 <= w
  while (lo < hi) {
    const int mid = (lo + hi + 1) / 2;
    if (items[mid].block0 <= w) lo = mid; else hi = mid - 1;
  }
  const PcBatchItem it = items[lo];
  const int local = w - it.block0;
  pc_body<NT>(it.kind, it.M, local % it.N, local / it.N, it.body_ptr, it.ncoarse, it.inv, it.BJ,
              in + it.off, out + it.off, vs, wv, yv, part);
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
int launch_blocks(bie_geom *g, int kind, const int *d_nc, float *inv, int *bad, hipStream_t s) {
  hipLaunchKernelGGL(k_pc_blocks<BJ>, dim3(g->N), dim3(BJ), 0, s, kind, g->body_ptr, d_nc, g->x,
                     g->y, g->nx, g->ny, g->w, g->kappa, g->px, g->py, inv);
  hipLaunchKernelGGL(k_pc_invert<BJ>, dim3(g->N), dim3(BJ * (BJ / kPcRows)), 0, s, kind, d_nc,
                     inv);
  hipLaunchKernelGGL(k_pc_check<BJ>, dim3(g->N), dim3(BJ), 0, s, kind, d_nc, inv, bad);
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
  std::vector<int> nc(N);
  int umax = 1;
  long long macs = 0;
  for (int b = 0; b < N; ++b) {
    const int n = g->h_body_ptr[b + 1] - g->h_body_ptr[b];
    nc[b] = coarse_nodes(n);
    if (nc[b] == 0) {
      set_error("block preconditioner: body " + std::to_string(b) + " has " + std::to_string(n) +
                " nodes; bodies of more than " + std::to_string(kPcNodes) +
                " nodes need a node count of at most " + std::to_string(kPcMaxFine) +
                " with a divisor in [" + std::to_string(kPcMinNodes) + ", " +
                std::to_string(kPcNodes) + "]");
      return BIE_EINVAL;
    }
    umax = std::max(umax, C * nc[b]);
    const long long U = (long long)C * nc[b], s = n / nc[b];
    macs += U * U + (s > 1 ? U * (2 * s - 1) + 2LL * C * n : 0);
  }
  const int BJ = umax <= 64 ? 64 : 128;
  BIE_TRY(pc.inv.reserve((size_t)N * BJ * BJ * sizeof(float)));
  BIE_TRY(pc.meta.reserve(2 * (size_t)N * sizeof(int)));
  int *d_nc = pc.meta.as<int>(), *d_bad = d_nc + N;
  BIE_HIP_CHECK(hipMemcpyAsync(d_nc, nc.data(), N * sizeof(int), hipMemcpyHostToDevice, s));
  float *inv = pc.inv.as<float>();
  if (BJ == 64) BIE_TRY(launch_blocks<64>(g, kind, d_nc, inv, d_bad, s));
  else BIE_TRY(launch_blocks<128>(g, kind, d_nc, inv, d_bad, s));
  std::vector<int> bad(N);
  BIE_HIP_CHECK(hipMemcpyAsync(bad.data(), d_bad, N * sizeof(int), hipMemcpyDeviceToHost, s));
  BIE_HIP_CHECK(hipStreamSynchronize(s));  // the host tables go out of scope
  for (int b = 0; b < N; ++b)
    if (bad[b]) {
      set_error("block preconditioner: the coarse block of body " + std::to_string(b) +
                " could not be inverted without pivoting");
      return BIE_EINVAL;
    }
  pc.BJ = BJ;
  pc.ncoarse = d_nc;
  pc.macs = macs;
  pc.lds = (size_t)C * nmax * sizeof(double);
  pc.ready = true;
  return BIE_OK;
}

int pc_apply(bie_geom *g, int kind, int nrhs, const double *in, double *out, hipStream_t s) {
  const bie_geom::Precond &pc = g->pc[kind & 1];
  if (!pc.ready) {
    set_error("block preconditioner not built");
    return BIE_EINVAL;
  }
  // units: multiply-adds (restriction, coarse product and interpolation) per right-hand side
  ProfScope prof(BIE_K_PRECOND, s, pc.macs * nrhs);
  // few bodies: 1024 threads per body shorten each one's sums; many: 512 threads, more
  // workgroups per compute unit (1000 starfish: 10.4 us per apply against 11.8 with 256 and
  // 14.3 with 1024)
  if (g->N < 512)
    hipLaunchKernelGGL(k_pc_apply<1024>, dim3(g->N, nrhs), dim3(1024), pc.lds, s, kind, g->M,
                       pc.BJ, g->body_ptr, pc.ncoarse, pc.inv.as<float>(), in, out);
  else
    hipLaunchKernelGGL(k_pc_apply<512>, dim3(g->N, nrhs), dim3(512), pc.lds, s, kind, g->M,
                       pc.BJ, g->body_ptr, pc.ncoarse, pc.inv.as<float>(), in, out);
  BIE_HIP_CHECK(hipGetLastError());
  return BIE_OK;
}

int pc_batch_items(const std::vector<bie_geom *> &geoms, const std::vector<int> &kinds,
                   const std::vector<int> &nrhs, const std::vector<long long> &offs,
                   std::vector<PcBatchItem> &items, size_t &lds, long long &blocks,
                   long long &macs) {
  items.clear();
  lds = 0;
  blocks = 0;
  macs = 0;
  for (size_t i = 0; i < geoms.size(); ++i) {
    const bie_geom::Precond &pc = geoms[i]->pc[kinds[i] & 1];
    if (!pc.ready) {
      set_error("block preconditioner not built");
      return BIE_EINVAL;
    }
    if (blocks + (long long)geoms[i]->N * nrhs[i] > (1LL << 31) - 1) {
      set_error("batched preconditioner: more than 2^31 - 1 (body, right-hand side) pairs");
      return BIE_EINVAL;
    }
    items.push_back(PcBatchItem{geoms[i]->body_ptr, pc.ncoarse, pc.inv.as<float>(), offs[i],
                                pc.BJ, geoms[i]->N, geoms[i]->M, kinds[i], nrhs[i], (int)blocks});
    blocks += (long long)geoms[i]->N * nrhs[i];
    lds = std::max(lds, pc.lds);
    macs += pc.macs * nrhs[i];
  }
  return BIE_OK;
}

int pc_apply_batch(int nitems, const PcBatchItem *d_items, size_t lds, long long blocks,
                   long long macs, const double *in, double *out, hipStream_t s) {
  ProfScope prof(BIE_K_PRECOND, s, macs);
  if (blocks > 0)
    hipLaunchKernelGGL(k_pc_apply_batch<256>, dim3((unsigned)blocks), dim3(256), lds, s, nitems,
                       d_items, in, out);
  BIE_HIP_CHECK(hipGetLastError());
  return BIE_OK;
}

}  // namespace bie
