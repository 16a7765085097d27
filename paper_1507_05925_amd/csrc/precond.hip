// Block-Jacobi right preconditioner of the Laplace operator (1/2 I + K + L): P = blockdiag of
// the inverses of the bodies' self blocks, GMRES solving (A P) u = f and x = P u. A body's self
// block holds the interactions of its own nodes: the identity, the smooth diagonal limit, the
// same-body double-layer pairs and its completion,
//   A_bb[i][k] = delta_ik (1/2 - w_i kappa_i / (4 pi))
//              - (1 - delta_ik) (1/2pi) w_k n_i . (x_i - x_k) / |x_i - x_k|^2 + w_k,
// the discrete operator of eq. ModRep2 restricted to body b (the same terms as the apply). The
// preconditioner changes the GMRES iterates, not the solution: every stopping test is on the
// true residual of A x = f. Bodies of at most 256 nodes; the inverses are formed in float32
// ([N][256][256] column-major, zero-padded) and kept as int8 with a float64 scale per row, less
// the exact 2 I (a preconditioner need not be exact, only fixed: the apply is exact arithmetic
// on the stored entries, in float64).
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

// The inverses as the int8 apply reads them: D_b = Inv_b - 2 I (the identity's exact part
// taken out), each row scaled to its largest magnitude, s_i = max_k |D_b[i][k]| / 127, and
// rounded, q_ik = rint(D_b[i][k] / s_i); four consecutive entries of a row in one 32-bit word:
// word ((b * 64 + k / 4) * 256 + i) holds q_i,k .. q_i,k+3 (byte k % 4). Grid N, 256 threads:
// thread i forms row i. Scales [N][256] after the words.
__global__ __launch_bounds__(kBj) void k_bj_store_i8(const int *__restrict__ body_ptr,
                                                    const float *__restrict__ in,
                                                    unsigned *__restrict__ words,
                                                    double *__restrict__ scale) {
  const int b = blockIdx.x, i = threadIdx.x;
  const int n = body_ptr[b + 1] - body_ptr[b];
  const float *col = in + (size_t)b * kBj * kBj + i;  // entry (i, k) at col[k * 256]
  float mx = 0.0f;
  if (i < n)
    for (int k = 0; k < n; ++k) mx = fmaxf(mx, fabsf(col[(size_t)k * kBj] - (k == i ? 2.0f : 0.0f)));
  const double sc = mx > 0.0f ? (double)mx / 127.0 : 1.0;
  scale[(size_t)b * kBj + i] = sc;
  const double isc = 1.0 / sc;
  unsigned *o = words + (size_t)b * (kBj / 4) * kBj + i;
  for (int k4 = 0; k4 < kBj; k4 += 4) {
    unsigned w = 0;
    for (int e = 0; e < 4; ++e) {
      const int k = k4 + e;
      int q = 0;
      if (i < n && k < n) {
        const double d = (double)col[(size_t)k * kBj] - (k == i ? 2.0 : 0.0);
        q = (int)rint(d * isc);
        q = q > 127 ? 127 : (q < -127 ? -127 : q);
      }
      w |= (unsigned)(q & 0xff) << (8 * e);
    }
    o[(size_t)(k4 / 4) * kBj] = w;
  }
}

// out = P in with the int8 inverses: out_b[i] = 2 in_b[i] + s_i sum_k q_ik in_b[k] (k
// ascending, float64 accumulation of the exact integer entries). Grid (N, ceil(nrhs / R)), thread
// i = row i reads its row's words, eight per batch of loads.
template <int R>
__global__ __launch_bounds__(kBj) void k_bj_apply_i8(int M, int nrhs, const int *__restrict__ body_ptr,
                                                     const unsigned *__restrict__ words,
                                                     const double *__restrict__ scale,
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
  const unsigned *row = words + (size_t)b * (kBj / 4) * kBj + i;  // word p at row[p * kBj]
  double acc[R];
#pragma unroll
  for (int r = 0; r < R; ++r) acc[r] = 0.0;
  const int nw = (n + 3) / 4;  // words; missing entries of the last one are zero
  int p = 0;
  for (; p + 8 <= nw; p += 8) {
    unsigned h[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) h[u] = row[(size_t)(p + u) * kBj];
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
    const unsigned h = row[(size_t)p * kBj];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const double q = (double)(int)(signed char)(h >> (8 * e));
#pragma unroll
      for (int r = 0; r < R; ++r) acc[r] = fma(q, v[r][4 * p + e], acc[r]);
    }
  }
  const double sc = scale[(size_t)b * kBj + i];
#pragma unroll
  for (int r = 0; r < R; ++r)
    if (r < nr) out[(size_t)(r0 + r) * M + k0 + i] = fma(sc, acc[r], 2.0 * v[r][i]);
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
  const size_t total = (size_t)g->N * kBj * kBj;  // int8 entries, then the row scales
  BIE_TRY(g->bj_store.reserve(total + (size_t)g->N * kBj * sizeof(double)));
  hipLaunchKernelGGL(k_bj_store_i8, dim3(g->N), dim3(kBj), 0, s, g->body_ptr, g->bj.as<float>(),
                     g->bj_store.as<unsigned>(),
                     reinterpret_cast<double *>(g->bj_store.as<char>() + total));
  BIE_HIP_CHECK(hipGetLastError());
  BIE_HIP_CHECK(hipStreamSynchronize(s));
  g->bj.release();  // only the int8 copy stays resident
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
  const size_t total = (size_t)g->N * kBj * kBj;
  const unsigned *words = g->bj_store.as<unsigned>();
  const double *scale = reinterpret_cast<const double *>(g->bj_store.as<char>() + total);
  if (nrhs == 1)
    hipLaunchKernelGGL(k_bj_apply_i8<1>, dim3(g->N, 1), dim3(kBj), 0, s, g->M, nrhs, g->body_ptr,
                       words, scale, in, out);
  else
    hipLaunchKernelGGL(k_bj_apply_i8<R>, dim3(g->N, (nrhs + R - 1) / R), dim3(kBj), 0, s, g->M,
                       nrhs, g->body_ptr, words, scale, in, out);
  BIE_HIP_CHECK(hipGetLastError());
  return BIE_OK;
}

}  // namespace bie
