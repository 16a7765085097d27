// Block-Jacobi right preconditioner of the Laplace operator (1/2 I + K + L): P = blockdiag of
// the inverses of the bodies' self blocks, GMRES solving (A P) u = f and x = P u. A body's self
// block holds the interactions of its own nodes: the identity, the smooth diagonal limit, the
// same-body double-layer pairs and its completion,
//   A_bb[i][k] = delta_ik (1/2 - w_i kappa_i / (4 pi))
//              - (1 - delta_ik) (1/2pi) w_k n_i . (x_i - x_k) / |x_i - x_k|^2 + w_k,
// the discrete operator of eq. ModRep2 restricted to body b (the same terms as the apply). The
// preconditioner changes the GMRES iterates, not the solution: every stopping test is on the
// true residual of A x = f. Bodies of at most 256 nodes; the inverses are formed in float32
// ([N][256][256] column-major, zero-padded) and kept in float16 for the apply (a preconditioner
// need not be exact, only fixed).
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "internal.h"

namespace bie {
namespace {

constexpr int kBj = 256;              // largest body the preconditioner takes
constexpr int kBjRows = 64;           // rows per thread in the inversion
constexpr int kBjThreads = kBj * (kBj / kBjRows);  // 1024
constexpr double kPi = 3.14159265358979323846;

// The self blocks, column-major and zero-padded to 256 x 256 (identity past n), float32 from
// float64 entries. Grid N, 256 threads: thread c forms column c.
__global__ __launch_bounds__(kBj) void k_bj_blocks(
    const int *__restrict__ body_ptr, const double *__restrict__ x, const double *__restrict__ y,
    const double *__restrict__ nx, const double *__restrict__ ny, const double *__restrict__ w,
    const double *__restrict__ kappa, float *__restrict__ inv) {
  const int b = blockIdx.x, c = threadIdx.x;
  const int k0 = body_ptr[b], n = body_ptr[b + 1] - k0;
  float *col = inv + (size_t)b * kBj * kBj + (size_t)c * kBj;
  const bool cin = c < n;
  const double xk = cin ? x[k0 + c] : 0.0, yk = cin ? y[k0 + c] : 0.0;
  const double wk = cin ? w[k0 + c] : 0.0;
  for (int i = 0; i < kBj; ++i) {
    double v = i == c ? 1.0 : 0.0;
    if (cin && i < n) {
      if (i == c) {
        v = 0.5 - w[k0 + i] * kappa[k0 + i] / (4.0 * kPi) + wk;
      } else {
        const double dx = x[k0 + i] - xk, dy = y[k0 + i] - yk;
        const double dot = nx[k0 + i] * dx + ny[k0 + i] * dy;
        v = -wk * dot / (2.0 * kPi * (dx * dx + dy * dy)) + wk;
      }
    }
    col[i] = (float)v;
  }
}

// One workgroup of 1024 threads per body inverts its block in place: thread t holds column
// c = t % 256, rows 64 (t / 256) .. 64 (t / 256) + 63, in registers, and the workgroup runs
// Gauss-Jordan elimination without pivoting (the leading minors of 1/2 I + 1 w^T + K stay near
// those of 1/2 I + 1 w^T, all positive). Rows and columns past the body's n nodes hold the
// identity and are never eliminated.
__global__ __launch_bounds__(kBjThreads) void k_bj_invert(const int *__restrict__ body_ptr,
                                                         float *__restrict__ inv) {
  __shared__ float rowk[kBj], colk[kBj];
  const int b = blockIdx.x;
  const int n = body_ptr[b + 1] - body_ptr[b];
  const int c = threadIdx.x % kBj, rg = threadIdx.x / kBj, r0 = rg * kBjRows;
  float *o = inv + (size_t)b * kBj * kBj + (size_t)c * kBj + r0;
  float a[kBjRows];
#pragma unroll
  for (int e = 0; e < kBjRows; e += 4) {
    const float4 q = *reinterpret_cast<const float4 *>(o + e);
    a[e] = q.x;
    a[e + 1] = q.y;
    a[e + 2] = q.z;
    a[e + 3] = q.w;
  }
  for (int k = 0; k < n; ++k) {
    // the pivot row and column before this step
    if (c == k) {
#pragma unroll
      for (int e = 0; e < kBjRows; ++e) colk[r0 + e] = a[e];
    }
    if (rg == k / kBjRows) {
      const int ek = k % kBjRows;
#pragma unroll
      for (int e = 0; e < kBjRows; ++e)
        if (e == ek) rowk[c] = a[e];
    }
    __syncthreads();
    const float ip = 1.0f / rowk[k];
    const float rkj = rowk[c] * ip;  // the pivot row entry of this column, scaled
#pragma unroll
    for (int e = 0; e < kBjRows; ++e) {
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
  for (int e = 0; e < kBjRows; e += 4)
    *reinterpret_cast<float4 *>(o + e) = make_float4(a[e], a[e + 1], a[e + 2], a[e + 3]);
}

// The inverses as the apply reads them: float16 (a preconditioner need not be exact; the
// iteration counts are those of the float32 inverses), entries k, k + 1 of row i side by side:
// out[((b * 128 + k / 2) * 256 + i) * 2 + k % 2] = Inv_b[i][k].
__global__ void k_bj_store(long long total, const float *__restrict__ in, __half *__restrict__ out) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;  // (b, k, i) in order
  if (t >= total) return;
  const long long bk = t / kBj;
  const int i = (int)(t % kBj), k = (int)(bk % kBj);
  const long long b = bk / kBj;
  out[((b * (kBj / 2) + k / 2) * kBj + i) * 2 + (k & 1)] = __float2half(in[t]);
}

// out = P in for every rhs: per body b, out_b[i] = sum_k Inv_b[i][k] in_b[k] (k ascending, float64
// accumulation). Grid (N, ceil(nrhs / R)); thread i = row i reads the pairs (k, k + 1) of its row,
// sixteen entries per batch of loads; the block's input entries are staged in LDS.
template <int R>
__global__ __launch_bounds__(kBj) void k_bj_apply(int M, int nrhs, const int *__restrict__ body_ptr,
                                                  const __half2 *__restrict__ inv,
                                                  const double *__restrict__ in,
                                                  double *__restrict__ out) {
  __shared__ double v[R][kBj];
  const int b = blockIdx.x, r0 = blockIdx.y * R;
  const int k0 = body_ptr[b], n = body_ptr[b + 1] - k0, i = threadIdx.x;
  const int nr = min(R, nrhs - r0);
#pragma unroll
  for (int r = 0; r < R; ++r) v[r][i] = (r < nr && i < n) ? in[(size_t)(r0 + r) * M + k0 + i] : 0.0;
  __syncthreads();
  if (i >= n) return;
  const __half2 *row = inv + (size_t)b * (kBj / 2) * kBj + i;  // pair p at row[p * kBj]
  double acc[R];
#pragma unroll
  for (int r = 0; r < R; ++r) acc[r] = 0.0;
  const int np = (n + 1) / 2;  // pairs; a missing last column is zero
  int p = 0;
  for (; p + 8 <= np; p += 8) {
    __half2 h[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) h[u] = row[(size_t)(p + u) * kBj];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const float2 e = __half22float2(h[u]);
#pragma unroll
      for (int r = 0; r < R; ++r) {
        acc[r] = fma((double)e.x, v[r][2 * (p + u)], acc[r]);
        acc[r] = fma((double)e.y, v[r][2 * (p + u) + 1], acc[r]);
      }
    }
  }
  for (; p < np; ++p) {
    const float2 e = __half22float2(row[(size_t)p * kBj]);
#pragma unroll
    for (int r = 0; r < R; ++r) {
      acc[r] = fma((double)e.x, v[r][2 * p], acc[r]);
      acc[r] = fma((double)e.y, v[r][2 * p + 1], acc[r]);
    }
  }
#pragma unroll
  for (int r = 0; r < R; ++r)
    if (r < nr) out[(size_t)(r0 + r) * M + k0 + i] = acc[r];
}

}  // namespace

int bj_build(bie_geom *g, hipStream_t s) {
  if (g->bj_ready) return BIE_OK;
  if (g->max_nb > kBj) {
    set_error("block-Jacobi preconditioner: bodies of at most 256 nodes (the largest has " +
              std::to_string(g->max_nb) + ")");
    return BIE_EINVAL;
  }
  DeviceGuard dg(g->device);
  BIE_TRY(g->bj.reserve((size_t)g->N * kBj * kBj * sizeof(float)));
  hipLaunchKernelGGL(k_bj_blocks, dim3(g->N), dim3(kBj), 0, s, g->body_ptr, g->x, g->y, g->nx,
                     g->ny, g->w, g->kappa, g->bj.as<float>());
  hipLaunchKernelGGL(k_bj_invert, dim3(g->N), dim3(kBjThreads), 0, s, g->body_ptr,
                     g->bj.as<float>());
  BIE_HIP_CHECK(hipGetLastError());
  const long long total = (long long)g->N * kBj * kBj;
  BIE_TRY(g->bj_store.reserve((size_t)total * sizeof(__half)));
  hipLaunchKernelGGL(k_bj_store, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, total,
                     g->bj.as<float>(), g->bj_store.as<__half>());
  BIE_HIP_CHECK(hipGetLastError());
  BIE_HIP_CHECK(hipStreamSynchronize(s));
  g->bj.release();  // only the float16 copy stays resident
  g->bj_entries = 0;
  for (int b = 0; b < g->N; ++b) {
    const long long n = g->h_body_ptr[b + 1] - g->h_body_ptr[b];
    g->bj_entries += n * n;
  }
  g->bj_ready = true;
  return BIE_OK;
}

int bj_apply(bie_geom *g, int nrhs, const double *in, double *out, hipStream_t s) {
  if (!g->bj_ready) {
    set_error("block-Jacobi preconditioner not built");
    return BIE_EINVAL;
  }
  constexpr int R = 4;
  // units: block entries read, sum over bodies of n_b^2 once per chunk of R right-hand sides
  ProfScope prof(BIE_K_PRECOND, s, g->bj_entries * ((nrhs + R - 1) / R));
  hipLaunchKernelGGL(k_bj_apply<R>, dim3(g->N, (nrhs + R - 1) / R), dim3(kBj), 0, s, g->M, nrhs,
                     g->body_ptr, g->bj_store.as<__half2>(), in, out);
  BIE_HIP_CHECK(hipGetLastError());
  return BIE_OK;
}

}  // namespace bie
