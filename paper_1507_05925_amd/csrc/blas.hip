// float64 vector kernels for the Arnoldi process over a set of independent systems ("segments")
// of possibly different lengths, stored back to back in flat vectors of Ntot entries. Work is
// cut into chunks that never straddle two systems; reductions are two-stage (per chunk, then per
// system in chunk order), so every result is bitwise reproducible run to run and independent of
// which other systems share the batch.
#include <hip/hip_runtime.h>

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

// partial[l * C + c] = <V_l, w> over chunk c; grid (C, nvec), one workgroup per (chunk, vector)
__global__ __launch_bounds__(kBlock) void k_dots_stage1(int C, const long long *__restrict__ c0,
                                                       const long long *__restrict__ c1,
                                                       const double *__restrict__ V, long long vstride,
                                                       const double *__restrict__ w,
                                                       double *__restrict__ partial) {
  __shared__ double sh[4];
  const int c = blockIdx.x, l = blockIdx.y;
  const long long i0 = c0[c], i1 = c1[c];
  const double *v = V + l * vstride;
  double acc = 0.0;
  for (long long i = i0 + threadIdx.x; i < i1; i += kBlock) acc = fma(v[i], w[i], acc);
  const double t = block_sum(acc, sh);
  if (threadIdx.x == 0) partial[(long long)l * C + c] = t;
}

// h[s * hs + l] = sum over the chunks of system s (in order); sqrt for norms
__global__ __launch_bounds__(64) void k_dots_stage2(int C, const int *__restrict__ sys_chunk,
                                                   const double *__restrict__ partial,
                                                   double *__restrict__ h, long long hs, int do_sqrt) {
  const int l = blockIdx.x, s = blockIdx.y;
  const int a = sys_chunk[s], b = sys_chunk[s + 1];
  double acc = 0.0;
  for (int c = a + threadIdx.x; c < b; c += 64) acc += partial[(long long)l * C + c];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
  if (threadIdx.x == 0) h[s * hs + l] = do_sqrt ? sqrt(acc) : acc;
}

// w += sign * sum_l V_l h[s][l] on each chunk (s = system of the chunk); grid (C, kSub), each
// workgroup takes every kSub-th block of 256 entries of its chunk
__global__ __launch_bounds__(kBlock) void k_combination(int nvec, const int *__restrict__ csys,
                                                       const long long *__restrict__ c0,
                                                       const long long *__restrict__ c1,
                                                       const double *__restrict__ V, long long vstride,
                                                       const double *__restrict__ h, long long hs,
                                                       double *__restrict__ w, double sign) {
  const int c = blockIdx.x;
  const int s = csys[c];
  const double *hr = h + s * hs;
  for (long long i = c0[c] + blockIdx.y * kBlock + threadIdx.x; i < c1[c]; i += kSub * kBlock) {
    double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
    int l = 0;
    for (; l + 4 <= nvec; l += 4) {
      a0 = fma(V[l * vstride + i], hr[l], a0);
      a1 = fma(V[(l + 1) * vstride + i], hr[l + 1], a1);
      a2 = fma(V[(l + 2) * vstride + i], hr[l + 2], a2);
      a3 = fma(V[(l + 3) * vstride + i], hr[l + 3], a3);
    }
    // term l always goes to accumulator l mod 4, so trailing zero coefficients (a system frozen
    // inside a longer batch cycle) leave every sum unchanged
    if (l < nvec) a0 = fma(V[l * vstride + i], hr[l], a0);
    if (l + 1 < nvec) a1 = fma(V[(l + 1) * vstride + i], hr[l + 1], a1);
    if (l + 2 < nvec) a2 = fma(V[(l + 2) * vstride + i], hr[l + 2], a2);
    w[i] += sign * ((a0 + a1) + (a2 + a3));
  }
}

// The second Gram-Schmidt update fused with the norm of its result: as k_combination, and each
// workgroup (chunk c, part sub) writes the sum of squares of the entries it wrote to
// partial[c * kSub + sub].
__global__ __launch_bounds__(kBlock) void k_combination_nrm(
    int nvec, const int *__restrict__ csys, const long long *__restrict__ c0,
    const long long *__restrict__ c1, const double *__restrict__ V, long long vstride,
    const double *__restrict__ h, long long hs, double *__restrict__ w, double sign,
    double *__restrict__ partial) {
  __shared__ double sh[4];
  const int c = blockIdx.x;
  const int s = csys[c];
  const double *hr = h + s * hs;
  double sq = 0.0;
  for (long long i = c0[c] + blockIdx.y * kBlock + threadIdx.x; i < c1[c]; i += kSub * kBlock) {
    double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
    int l = 0;
    for (; l + 4 <= nvec; l += 4) {
      a0 = fma(V[l * vstride + i], hr[l], a0);
      a1 = fma(V[(l + 1) * vstride + i], hr[l + 1], a1);
      a2 = fma(V[(l + 2) * vstride + i], hr[l + 2], a2);
      a3 = fma(V[(l + 3) * vstride + i], hr[l + 3], a3);
    }
    if (l < nvec) a0 = fma(V[l * vstride + i], hr[l], a0);
    if (l + 1 < nvec) a1 = fma(V[(l + 1) * vstride + i], hr[l + 1], a1);
    if (l + 2 < nvec) a2 = fma(V[(l + 2) * vstride + i], hr[l + 2], a2);
    const double v = w[i] + sign * ((a0 + a1) + (a2 + a3));
    w[i] = v;
    sq = fma(v, v, sq);
  }
  const double t = block_sum(sq, sh);
  if (threadIdx.x == 0) partial[(long long)c * kSub + blockIdx.y] = t;
}

// Normalisation of the new Krylov vector, one workgroup per chunk c (system s): every workgroup
// of s sums s's partials in the same fixed order, so all of them form the same ||w||, and writes
// v = w / ||w|| over its chunk; the first workgroup of s also completes the Hessenberg column,
// h2[s][0..cnt-1] += h1[s][...] and h2[s][cnt] = ||w||, stores ||w|| in nrm[s] and, when col_out
// is given (mapped host memory), writes the column there too, then (when flag is given) stores
// the tag of step *seq_base + seq_off in flag[s] once the column is visible to the host (the
// base is read when the kernel runs, so a captured graph of the step stays valid across
// cycles).
__global__ __launch_bounds__(kBlock) void k_normalize_column(
    int cnt, const int *__restrict__ csys, const int *__restrict__ sys_chunk,
    const long long *__restrict__ c0, const long long *__restrict__ c1,
    const double *__restrict__ partial, const double *__restrict__ w, double *__restrict__ v,
    const double *__restrict__ h1, double *__restrict__ h2, long long hs,
    double *__restrict__ nrm, double *__restrict__ col_out, unsigned long long *flag,
    const unsigned long long *seq_base, unsigned long long seq_off) {
  __shared__ double sh[4];
  const int c = blockIdx.x, s = csys[c];
  const int a = sys_chunk[s] * kSub, b = sys_chunk[s + 1] * kSub;
  double acc = 0.0;
  for (int e = a + threadIdx.x; e < b; e += kBlock) acc += partial[e];
  const double n = sqrt(block_sum(acc, sh));
  for (long long i = c0[c] + threadIdx.x; i < c1[c]; i += kBlock) v[i] = n > 0.0 ? w[i] / n : 0.0;
  if (c == sys_chunk[s]) {
    for (int l = threadIdx.x; l < cnt; l += kBlock) {
      const double hv = h2[s * hs + l] + h1[s * hs + l];
      h2[s * hs + l] = hv;
      if (col_out) col_out[s * hs + l] = hv;
    }
    if (threadIdx.x == 0) {
      nrm[s] = n;
      h2[s * hs + cnt] = n;
      if (col_out) col_out[s * hs + cnt] = n;
    }
    if (flag) {  // (uniform over the workgroup)
      __threadfence_system();  // this thread's column entries reach host memory first
      __syncthreads();
      if (threadIdx.x == 0) {
        const unsigned long long seq = column_tag(*seq_base + seq_off);
        __hip_atomic_store(flag + s, seq, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
      }
    }
  }
}

__global__ __launch_bounds__(kBlock) void k_scale_to(const int *__restrict__ csys,
                                                    const long long *__restrict__ c0,
                                                    const long long *__restrict__ c1,
                                                    const double *__restrict__ w,
                                                    const double *__restrict__ den,
                                                    double *__restrict__ v) {
  const int c = blockIdx.x;
  const double d = den[csys[c]];
  for (long long i = c0[c] + threadIdx.x; i < c1[c]; i += kBlock) v[i] = d > 0.0 ? w[i] / d : 0.0;
}

// ---- DCGS2 Arnoldi (classical Gram-Schmidt with delayed reorthogonalisation) ---------------
// Step j >= 1 works on U, the candidate for basis vector V_j after one projection, and
// Z = A U. One pass over V_0..V_{j-1} gives s = V^T U, t = V^T Z, U.U and U.Z (one reduction);
// from them a small per-system kernel finishes column j - 1 of the Hessenberg matrix (the first
// projection's coefficients plus s, and nu = sqrt(U.U - s.s) below the diagonal) and forms the
// coefficients of the next projection without another pass, using the Arnoldi relation
// A V_i = sum_k H[k][i] V_k: with V_j = (U - V s) / nu, A V_j = (Z - V (H s)) / nu, so
// V_k . A V_j = (t_k - (H s)_k) / nu (k < j) and ((U.Z - s.t) / nu - (H s)_j) / nu (k = j).
// A second pass writes V_j and the next candidate U' = A V_j - sum_{k<=j} g'_k V_k
// = Z / nu - sum_{k<=j} c_k V_k with c_k = (H s)_k / nu + g'_k.

// partial rows over chunk c: 2l = V_l . U and 2l + 1 = V_l . Z (l < nv); 2 nv = U . U and
// 2 nv + 1 = U . Z. Z NULL: the odd rows are zero. Grid (C, ceil((nv + 1) / kDotsVecs)): a
// workgroup holds its chunk of U and Z in registers (entries i0 + t + 256 k, k < kSub) and takes
// kDotsVecs of the vectors, so U and Z are read once per kDotsVecs vectors instead of once per
// vector. Each row's sum has the order of a one-vector reduction: per thread in entry order, the
// wave's shuffle tree, then the four waves as (w0 + w1) + (w2 + w3).
constexpr int kDotsVecs = 8;

__global__ __launch_bounds__(kBlock) void k_dots_uz(int C, const long long *__restrict__ c0,
                                                   const long long *__restrict__ c1, int nv,
                                                   const double *__restrict__ V, long long vstride,
                                                   const double *__restrict__ U,
                                                   const double *__restrict__ Z,
                                                   double *__restrict__ partial) {
  __shared__ double sh[4][2 * kDotsVecs];
  const int c = blockIdx.x, l0 = blockIdx.y * kDotsVecs;
  const int nl = min(kDotsVecs, nv + 1 - l0);
  const long long i0 = c0[c], i1 = c1[c];
  double u[kSub], z[kSub];
#pragma unroll
  for (int k = 0; k < kSub; ++k) {
    const long long i = i0 + threadIdx.x + (long long)k * kBlock;
    u[k] = i < i1 ? U[i] : 0.0;
    z[k] = (Z && i < i1) ? Z[i] : 0.0;
  }
  double su[kDotsVecs], sz[kDotsVecs];
#pragma unroll
  for (int q = 0; q < kDotsVecs; ++q) {
    su[q] = sz[q] = 0.0;
    if (q < nl) {
      const int l = l0 + q;
      const double *a = l < nv ? V + l * vstride : U;
#pragma unroll
      for (int k = 0; k < kSub; ++k) {
        const long long i = i0 + threadIdx.x + (long long)k * kBlock;
        if (i < i1) {
          const double x = a[i];
          su[q] = fma(x, u[k], su[q]);
          sz[q] = fma(x, z[k], sz[q]);
        }
      }
    }
  }
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int q = 0; q < kDotsVecs; ++q) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      su[q] += __shfl_down(su[q], off, 64);
      sz[q] += __shfl_down(sz[q], off, 64);
    }
    if (lane == 0) {
      sh[wid][2 * q] = su[q];
      sh[wid][2 * q + 1] = sz[q];
    }
  }
  __syncthreads();
  if (threadIdx.x < 2 * nl) {
    const int x = threadIdx.x;
    const double t = (sh[0][x] + sh[1][x]) + (sh[2][x] + sh[3][x]);
    partial[(long long)(2 * l0 + x) * C + c] = t;
  }
}

// Per system s (one workgroup): raw[s][2i], raw[s][2i + 1] = s_i, t_i (i < j), raw[s][2j],
// raw[s][2j + 1] = U.U, U.Z. Finishes column j - 1 (H[i][j-1] = G[i] + s_i, H[j][j-1] = nu) in
// the device copy Hd (column-major, leading dimension ldh) and in mapped host memory col_out,
// then stores the tag of step *seq_base + seq_off in flag[s]. Unless finalize: the coefficients
// of the update, sc = s (k < j), cc = c (k <= j), inu = 1/nu, and G = g' (the first projection's
// coefficients of the next column). nu = 0 (breakdown) gives zero coefficients. Dynamic LDS:
// 3 (j + 1) doubles.
__global__ __launch_bounds__(kBlock) void k_dcgs_small(
    int j, int finalize, const double *__restrict__ raw, long long rstride,
    double *__restrict__ G, double *__restrict__ Hd, long long ldh, long long hstride,
    double *__restrict__ sc, double *__restrict__ cc, double *__restrict__ inu, long long hs,
    double *__restrict__ col_out, unsigned long long *flag,
    const unsigned long long *seq_base, unsigned long long seq_off) {
  extern __shared__ double sm[];
  double *sv = sm, *tv = sm + (j + 1), *hv = sm + 2 * (j + 1);
  __shared__ double red[2];
  const int s = blockIdx.x;
  const double *rw = raw + s * rstride;
  double *H = Hd + s * hstride;
  for (int i = threadIdx.x; i < j; i += kBlock) {
    sv[i] = rw[2 * i];
    tv[i] = rw[2 * i + 1];
  }
  __syncthreads();
  // s.s and s.t in a fixed order (first wave: lanes stride, then the shuffle tree)
  if (threadIdx.x < 64) {
    double a = 0.0, b = 0.0;
    for (int i = threadIdx.x; i < j; i += 64) {
      a = fma(sv[i], sv[i], a);
      b = fma(sv[i], tv[i], b);
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      a += __shfl_down(a, off, 64);
      b += __shfl_down(b, off, 64);
    }
    if (threadIdx.x == 0) {
      red[0] = a;
      red[1] = b;
    }
  }
  __syncthreads();
  const double nu2 = rw[2 * j] - red[0];
  const double nu = nu2 > 0.0 ? sqrt(nu2) : 0.0;
  // column j - 1, final
  for (int i = threadIdx.x; i <= j; i += kBlock) {
    const double v = i < j ? G[s * hs + i] + sv[i] : nu;
    H[(long long)(j - 1) * ldh + i] = v;
    if (col_out) col_out[s * hs + i] = v;
  }
  if (flag) {
    __threadfence_system();  // the column reaches host memory before its flag
    __syncthreads();
    if (threadIdx.x == 0) {
      const unsigned long long tag = column_tag(*seq_base + seq_off);
      __hip_atomic_store(flag + s, tag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    }
  }
  if (finalize) return;
  __syncthreads();  // column j - 1 of H is written (and G read)
  // (H s)_k = sum_{i < j} H[k][i] s_i, k = 0..j (H[k][i] = 0 for k > i + 1)
  // (eight loads in flight per step; the sum keeps the order of i)
  for (int k = threadIdx.x; k <= j; k += kBlock) {
    double a = 0.0;
    int i = k > 0 ? k - 1 : 0;
    for (; i + 8 <= j; i += 8) {
      double h[8];
#pragma unroll
      for (int e = 0; e < 8; ++e) h[e] = H[(long long)(i + e) * ldh + k];
#pragma unroll
      for (int e = 0; e < 8; ++e) a = fma(h[e], sv[i + e], a);
    }
    for (; i < j; ++i) a = fma(H[(long long)i * ldh + k], sv[i], a);
    hv[k] = a;
  }
  __syncthreads();
  const double iv = nu > 0.0 ? 1.0 / nu : 0.0;
  for (int k = threadIdx.x; k <= j; k += kBlock) {
    const double g = k < j ? (tv[k] - hv[k]) * iv : ((rw[2 * j + 1] - red[1]) * iv - hv[k]) * iv;
    cc[s * hs + k] = nu > 0.0 ? hv[k] * iv + g : 0.0;
    G[s * hs + k] = nu > 0.0 ? g : 0.0;
    if (k < j) sc[s * hs + k] = sv[k];
  }
  if (threadIdx.x == 0) inu[s] = iv;
}

// V_j = (U - sum_{k<j} sc_k V_k) / nu and U = Z / nu - sum_{k<j} cc_k V_k - cc_j V_j, entry by
// entry (one pass over V_0..V_{j-1}); grid (C, kSub) as k_combination.
__global__ __launch_bounds__(kBlock) void k_dcgs_update(
    int j, const int *__restrict__ csys, const long long *__restrict__ c0,
    const long long *__restrict__ c1, const double *__restrict__ V, long long vstride,
    const double *__restrict__ sc, const double *__restrict__ cc, const double *__restrict__ inu,
    long long hs, double *__restrict__ U, const double *__restrict__ Z, double *__restrict__ Vj) {
  const int c = blockIdx.x, s = csys[c];
  const double *sr = sc + s * hs, *cr = cc + s * hs;
  const double iv = inu[s], cj = cr[j];
  for (long long i = c0[c] + blockIdx.y * kBlock + threadIdx.x; i < c1[c]; i += kSub * kBlock) {
    double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0, b0 = 0.0, b1 = 0.0, b2 = 0.0, b3 = 0.0;
    int l = 0;
    for (; l + 4 <= j; l += 4) {
      const double v0 = V[l * vstride + i], v1 = V[(l + 1) * vstride + i];
      const double v2 = V[(l + 2) * vstride + i], v3 = V[(l + 3) * vstride + i];
      a0 = fma(v0, sr[l], a0);
      a1 = fma(v1, sr[l + 1], a1);
      a2 = fma(v2, sr[l + 2], a2);
      a3 = fma(v3, sr[l + 3], a3);
      b0 = fma(v0, cr[l], b0);
      b1 = fma(v1, cr[l + 1], b1);
      b2 = fma(v2, cr[l + 2], b2);
      b3 = fma(v3, cr[l + 3], b3);
    }
    for (int r = 0; l + r < j; ++r) {
      const double v = V[(l + r) * vstride + i];
      if (r == 0) { a0 = fma(v, sr[l], a0); b0 = fma(v, cr[l], b0); }
      if (r == 1) { a1 = fma(v, sr[l + 1], a1); b1 = fma(v, cr[l + 1], b1); }
      if (r == 2) { a2 = fma(v, sr[l + 2], a2); b2 = fma(v, cr[l + 2], b2); }
    }
    const double vj = (U[i] - ((a0 + a1) + (a2 + a3))) * iv;
    Vj[i] = vj;
    U[i] = Z[i] * iv - ((b0 + b1) + (b2 + b3)) - cj * vj;
  }
}

__global__ void k_axpby(long long total, double a, const double *__restrict__ x, double b,
                        double *__restrict__ y) {
  const long long i = (long long)blockIdx.x * kBlock + threadIdx.x;
  if (i < total) y[i] = a * x[i] + b * y[i];
}

__global__ void k_add_h(int cnt, long long hs, const double *__restrict__ h1, double *__restrict__ h2) {
  const int s = blockIdx.x;
  for (int l = threadIdx.x; l < cnt; l += blockDim.x) h2[s * hs + l] += h1[s * hs + l];
}

}  // namespace

int seg_dots(const Segments &sg, int nvec, const double *V, long long vstride, const double *w,
             double *h, long long hs, double *scratch, hipStream_t s) {
  if (nvec <= 0) return BIE_OK;
  hipLaunchKernelGGL(k_dots_stage1, dim3(sg.C, nvec), dim3(kBlock), 0, s, sg.C, sg.c0, sg.c1, V,
                     vstride, w, scratch);
  hipLaunchKernelGGL(k_dots_stage2, dim3(nvec, sg.S), dim3(64), 0, s, sg.C, sg.sys_chunk, scratch,
                     h, hs, 0);
  BIE_HIP_CHECK(hipGetLastError());
  return BIE_OK;
}

int seg_combination(const Segments &sg, int nvec, const double *V, long long vstride,
                    const double *h, long long hs, double *w, double sign, hipStream_t s) {
  if (nvec <= 0) return BIE_OK;
  hipLaunchKernelGGL(k_combination, dim3(sg.C, kSub), dim3(kBlock), 0, s, nvec, sg.csys, sg.c0,
                     sg.c1, V, vstride, h, hs, w, sign);
  BIE_HIP_CHECK(hipGetLastError());
  return BIE_OK;
}

int seg_nrm2(const Segments &sg, const double *w, double *out, double *scratch, hipStream_t s) {
  hipLaunchKernelGGL(k_dots_stage1, dim3(sg.C, 1), dim3(kBlock), 0, s, sg.C, sg.c0, sg.c1, w, 0LL,
                     w, scratch);
  hipLaunchKernelGGL(k_dots_stage2, dim3(1, sg.S), dim3(64), 0, s, sg.C, sg.sys_chunk, scratch, out,
                     1LL, 1);
  BIE_HIP_CHECK(hipGetLastError());
  return BIE_OK;
}

int seg_combination_column(const Segments &sg, int nvec, const double *V, long long vstride,
                           const double *h1, double *h2, long long hs, double *w, double *nrm,
                           double *vnext, double *col_out, unsigned long long *flag,
                           const unsigned long long *seq_base, unsigned long long seq_off,
                           double *scratch, hipStream_t s) {
  if (nvec <= 0) return BIE_OK;
  hipLaunchKernelGGL(k_combination_nrm, dim3(sg.C, kSub), dim3(kBlock), 0, s, nvec, sg.csys, sg.c0,
                     sg.c1, V, vstride, h2, hs, w, -1.0, scratch);
  hipLaunchKernelGGL(k_normalize_column, dim3(sg.C), dim3(kBlock), 0, s, nvec, sg.csys,
                     sg.sys_chunk, sg.c0, sg.c1, scratch, w, vnext, h1, h2, hs, nrm, col_out, flag,
                     seq_base, seq_off);
  BIE_HIP_CHECK(hipGetLastError());
  return BIE_OK;
}

int dcgs_dots(const Segments &sg, int nv, const double *V, long long vstride, const double *U,
              const double *Z, double *raw, long long rstride, double *scratch, hipStream_t s) {
  hipLaunchKernelGGL(k_dots_uz, dim3(sg.C, (nv + kDotsVecs) / kDotsVecs), dim3(kBlock), 0, s,
                     sg.C, sg.c0, sg.c1, nv, V, vstride, U, Z, scratch);
  hipLaunchKernelGGL(k_dots_stage2, dim3(2 * nv + 2, sg.S), dim3(64), 0, s, sg.C, sg.sys_chunk,
                     scratch, raw, rstride, 0);
  BIE_HIP_CHECK(hipGetLastError());
  return BIE_OK;
}

int dcgs_small(int S, int j, bool finalize, const double *raw, long long rstride, double *G,
               double *Hd, long long ldh, long long hstride, double *sc, double *cc, double *inu,
               long long hs, double *col_out, unsigned long long *flag,
               const unsigned long long *seq_base, unsigned long long seq_off, hipStream_t s) {
  hipLaunchKernelGGL(k_dcgs_small, dim3(S), dim3(kBlock), (size_t)3 * (j + 1) * sizeof(double), s,
                     j, finalize ? 1 : 0, raw, rstride, G, Hd, ldh, hstride, sc, cc, inu, hs,
                     col_out, flag, seq_base, seq_off);
  BIE_HIP_CHECK(hipGetLastError());
  return BIE_OK;
}

int dcgs_update(const Segments &sg, int j, const double *V, long long vstride, const double *sc,
                const double *cc, const double *inu, long long hs, double *U, const double *Z,
                double *Vj, hipStream_t s) {
  hipLaunchKernelGGL(k_dcgs_update, dim3(sg.C, kSub), dim3(kBlock), 0, s, j, sg.csys, sg.c0, sg.c1,
                     V, vstride, sc, cc, inu, hs, U, Z, Vj);
  BIE_HIP_CHECK(hipGetLastError());
  return BIE_OK;
}

int seg_scale_to(const Segments &sg, const double *w, const double *den, double *v, hipStream_t s) {
  hipLaunchKernelGGL(k_scale_to, dim3(sg.C), dim3(kBlock), 0, s, sg.csys, sg.c0, sg.c1, w, den, v);
  BIE_HIP_CHECK(hipGetLastError());
  return BIE_OK;
}

int vec_axpby(long long total, double a, const double *x, double b, double *y, hipStream_t s) {
  hipLaunchKernelGGL(k_axpby, dim3((unsigned)((total + kBlock - 1) / kBlock)), dim3(kBlock), 0, s,
                     total, a, x, b, y);
  BIE_HIP_CHECK(hipGetLastError());
  return BIE_OK;
}

int seg_add_h(int S, const double *h1, double *h2, int cnt, long long hs, hipStream_t s) {
  hipLaunchKernelGGL(k_add_h, dim3(S), dim3(64), 0, s, cnt, hs, h1, h2);
  BIE_HIP_CHECK(hipGetLastError());
  return BIE_OK;
}

// Chunk list of systems with the given lengths (flat, back to back).
int Segments::build(const std::vector<long long> &lens, hipStream_t s,
                    const std::vector<long long> *starts) {
  S = (int)lens.size();
  std::vector<long long> a, b;
  std::vector<int> cs, sc(1, 0);
  long long off = 0;
  h_off.assign(S + 1, 0);
  for (int k = 0; k < S; ++k) {
    const long long n = lens[k];
    if (starts) off = (*starts)[k];
    h_off[k] = off;
    const long long per = kChunk;  // chunk length
    for (long long i = 0; i < n; i += per) {
      a.push_back(off + i);
      b.push_back(off + std::min(n, i + per));
      cs.push_back(k);
    }
    if (n == 0) {  // keep one empty chunk so stage 2 sees the system
      a.push_back(off);
      b.push_back(off);
      cs.push_back(k);
    }
    sc.push_back((int)cs.size());
    off += n;
    h_off[k + 1] = off;
  }
  // h_off[k] is the start of system k; h_off[S] the end of the last one
  C = (int)cs.size();
  Ntot = off;
  const size_t bytes = (size_t)C * (8 + 8 + 4) + (S + 1) * 4 + 256;
  BIE_TRY(buf.reserve(bytes));
  char *q = buf.as<char>();
  c0 = (long long *)q;
  c1 = c0 + C;
  csys = (int *)(c1 + C);
  sys_chunk = csys + C;
  BIE_HIP_CHECK(hipMemcpyAsync(c0, a.data(), C * 8, hipMemcpyHostToDevice, s));
  BIE_HIP_CHECK(hipMemcpyAsync(c1, b.data(), C * 8, hipMemcpyHostToDevice, s));
  BIE_HIP_CHECK(hipMemcpyAsync(csys, cs.data(), C * 4, hipMemcpyHostToDevice, s));
  BIE_HIP_CHECK(hipMemcpyAsync(sys_chunk, sc.data(), (S + 1) * 4, hipMemcpyHostToDevice, s));
  BIE_HIP_CHECK(hipStreamSynchronize(s));
  return BIE_OK;
}

}  // namespace bie
