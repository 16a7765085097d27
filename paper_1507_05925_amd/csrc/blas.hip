// float64 vector kernels for the Arnoldi process (classical Gram-Schmidt, twice).
// All reductions are two-stage with a fixed summation order, so results are bitwise
// reproducible run to run. Batched over nrhs independent vectors.
#include <hip/hip_runtime.h>

#include "internal.h"

namespace bie {
namespace {

constexpr int kDotBlocks = 128;  // first-stage blocks per rhs (upper bound)

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

// scratch[(r * nvec + l) * nblk + blk] = partial of <V_l, w> over this block's range
__global__ __launch_bounds__(kBlock) void k_dots_stage1(int n, int nvec, int nblk,
                                                       const double *__restrict__ V,
                                                       long long vs_r, long long vs_v,
                                                       const double *__restrict__ w, long long ws,
                                                       double *__restrict__ scratch) {
  __shared__ double sh[4];
  const int blk = blockIdx.x, r = blockIdx.y;
  const long long chunk = ((long long)n + nblk - 1) / nblk;
  const long long i0 = blk * chunk;
  const long long i1 = i0 + chunk < n ? i0 + chunk : n;
  const double *wr = w + r * ws;
  for (int l = 0; l < nvec; ++l) {
    const double *v = V + r * vs_r + l * vs_v;
    double acc = 0.0;
    for (long long i = i0 + threadIdx.x; i < i1; i += kBlock) acc = fma(v[i], wr[i], acc);
    const double t = block_sum(acc, sh);
    if (threadIdx.x == 0) scratch[((long long)r * nvec + l) * nblk + blk] = t;
  }
}

__global__ __launch_bounds__(64) void k_dots_stage2(int nvec, int nblk,
                                                   const double *__restrict__ scratch,
                                                   double *__restrict__ h, long long hs,
                                                   int do_sqrt) {
  const int l = blockIdx.x, r = blockIdx.y;
  const double *p = scratch + ((long long)r * nvec + l) * nblk;
  double acc = 0.0;
  for (int b = threadIdx.x; b < nblk; b += 64) acc += p[b];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
  if (threadIdx.x == 0) h[r * hs + l] = do_sqrt ? sqrt(acc) : acc;
}

// w_r += sign * sum_l V_{r,l} h_{r,l}
__global__ __launch_bounds__(kBlock) void k_combination(int n, int nvec,
                                                       const double *__restrict__ V,
                                                       long long vs_r, long long vs_v,
                                                       const double *__restrict__ h, long long hs,
                                                       double *__restrict__ w, long long ws,
                                                       double sign) {
  const int r = blockIdx.y;
  const long long i = (long long)blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  const double *hr = h + r * hs;
  const double *v = V + r * vs_r + i;
  double acc = 0.0;
  for (int l = 0; l < nvec; ++l) acc = fma(v[l * vs_v], hr[l], acc);
  w[r * ws + i] += sign * acc;
}

__global__ void k_scale_to(int n, const double *__restrict__ w, long long ws,
                           const double *__restrict__ den, double *__restrict__ v, long long vs) {
  const int r = blockIdx.y;
  const long long i = (long long)blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  const double d = den[r];
  v[r * vs + i] = d > 0.0 ? w[r * ws + i] / d : 0.0;
}

__global__ void k_axpby(long long total, double a, const double *__restrict__ x, double b,
                        double *__restrict__ y) {
  const long long i = (long long)blockIdx.x * kBlock + threadIdx.x;
  if (i < total) y[i] = a * x[i] + b * y[i];
}

__global__ void k_add_h(int cnt, long long hs, const double *__restrict__ h1, double *__restrict__ h2) {
  const int r = blockIdx.x;
  for (int l = threadIdx.x; l < cnt; l += blockDim.x) h2[r * hs + l] += h1[r * hs + l];
}

int dot_blocks(int n) {
  int b = (n + 4 * kBlock - 1) / (4 * kBlock);
  return b < 1 ? 1 : (b > kDotBlocks ? kDotBlocks : b);
}

}  // namespace

int vec_dots(int nrhs, int n, int nvec, const double *V, long long vs_r, long long vs_v,
             const double *w, long long ws, double *h, long long hs, double *scratch,
             hipStream_t s) {
  const int nblk = dot_blocks(n);
  hipLaunchKernelGGL(k_dots_stage1, dim3(nblk, nrhs), dim3(kBlock), 0, s, n, nvec, nblk, V, vs_r,
                     vs_v, w, ws, scratch);
  hipLaunchKernelGGL(k_dots_stage2, dim3(nvec, nrhs), dim3(64), 0, s, nvec, nblk, scratch, h, hs, 0);
  BIE_HIP_CHECK(hipGetLastError());
  return BIE_OK;
}

int vec_sub_combination(int nrhs, int n, int nvec, const double *V, long long vs_r, long long vs_v,
                        const double *h, long long hs, double *w, long long ws, double sign,
                        hipStream_t s) {
  hipLaunchKernelGGL(k_combination, dim3((n + kBlock - 1) / kBlock, nrhs), dim3(kBlock), 0, s, n,
                     nvec, V, vs_r, vs_v, h, hs, w, ws, sign);
  BIE_HIP_CHECK(hipGetLastError());
  return BIE_OK;
}

int vec_nrm2(int nrhs, int n, const double *w, long long ws, double *out, double *scratch,
             hipStream_t s) {
  const int nblk = dot_blocks(n);
  hipLaunchKernelGGL(k_dots_stage1, dim3(nblk, nrhs), dim3(kBlock), 0, s, n, 1, nblk, w, ws, 0LL,
                     w, ws, scratch);
  hipLaunchKernelGGL(k_dots_stage2, dim3(1, nrhs), dim3(64), 0, s, 1, nblk, scratch, out, 1LL, 1);
  BIE_HIP_CHECK(hipGetLastError());
  return BIE_OK;
}

int vec_scale_to(int nrhs, int n, const double *w, long long ws, const double *den, double *v,
                 long long vs, hipStream_t s) {
  hipLaunchKernelGGL(k_scale_to, dim3((n + kBlock - 1) / kBlock, nrhs), dim3(kBlock), 0, s, n, w,
                     ws, den, v, vs);
  BIE_HIP_CHECK(hipGetLastError());
  return BIE_OK;
}

int vec_axpby(int nrhs, int n, double a, const double *x, double b, double *y, hipStream_t s) {
  const long long tot = (long long)nrhs * n;
  hipLaunchKernelGGL(k_axpby, dim3((unsigned)((tot + kBlock - 1) / kBlock)), dim3(kBlock), 0, s,
                     tot, a, x, b, y);
  BIE_HIP_CHECK(hipGetLastError());
  return BIE_OK;
}

int vec_add_h(int nrhs, int n, const double *h1, double *h2, int cnt, long long hs, hipStream_t s) {
  (void)n;
  hipLaunchKernelGGL(k_add_h, dim3(nrhs), dim3(64), 0, s, cnt, hs, h1, h2);
  BIE_HIP_CHECK(hipGetLastError());
  return BIE_OK;
}

}  // namespace bie
