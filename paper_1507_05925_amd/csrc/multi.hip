// One operator apply for many geometries at once (batched solves and the server): the far-field
// sweeps, the per-body epilogues and the strength packing of every item run as three launches
// per kernel class instead of three per geometry. Work is described by task lists built on the
// host whenever the set of active items changes:
//   far task      = (item, rhs chunk of R, 256-target tile, source-body split)
//   epilogue task = (item, body, rhs)
//   pack task     = (item, rhs)
// The arithmetic per target is the single-geometry sweep's (kernels.hip): float32 body-relative
// or float64 coordinates, float64 accumulation per source body, own body skipped, then self
// block, diagonal limit, identity and completion in float64 with the partials summed in split
// order. Items above the FMM threshold are applied by the single-geometry path.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "internal.h"

namespace bie {

struct ItemDesc {
  int M, N, kind, nrhs, R, nchunk, ntile, nsplit;
  long long io;    // offset of the item's rhs block in the flat in/out vectors (doubles)
  long long slot;  // first partial slot of the item
  const int *body_ptr, *body_of, *split_body;
  const double *x, *y, *nx, *ny, *w, *kappa, *px, *py, *xc, *yc;
  const double2 *xy;
  const float2 *xr;
};

constexpr int kFmmStreams = 4;

struct MultiPlan {
  DevBuf desc_buf, task_buf, ws;
  // items applied by the FMM run on a small pool of streams (one per geometry, by first
  // appearance), forked from and joined back to the caller's stream
  hipStream_t pool[kFmmStreams] = {};
  hipEvent_t fork = nullptr, join[kFmmStreams] = {};
  std::vector<int> split_host;
  int nfar[2] = {0, 0}, nepi[2] = {0, 0}, npack = 0;
  int *far_task[2] = {nullptr, nullptr}, *epi_task[2] = {nullptr, nullptr}, *pack_task = nullptr;
  ItemDesc *desc = nullptr;
  long long nslots[2] = {0, 0};
  // the plan is reused while every item matches: geometry id, kind, rhs count, method and
  // offset of its block, and the active flags
  std::vector<unsigned long long> key_gen;
  std::vector<int> key_kind, key_nrhs;
  std::vector<char> key_fmm;
  std::vector<long long> key_io;
  std::vector<char> key_active;
  bool valid = false;
};

void multi_destroy(MultiPlan *p) {
  if (!p) return;
  for (int i = 0; i < kFmmStreams; ++i) {
    if (p->pool[i]) {
      (void)hipStreamSynchronize(p->pool[i]);
      (void)hipStreamDestroy(p->pool[i]);
    }
    if (p->join[i]) (void)hipEventDestroy(p->join[i]);
  }
  if (p->fork) (void)hipEventDestroy(p->fork);
  p->desc_buf.release();
  p->task_buf.release();
  p->ws.release();
  delete p;
}

namespace {

constexpr int kT = 256;  // targets per far tile (= kBlock)
constexpr float kFar32 = 1.0e18f;
constexpr double kFar64 = 1.0e100;

// The descriptor's pointers are generic; a load through a generic pointer may reach per-lane
// private memory, so the compiler treats its result as divergent even at a uniform address.
// Casting to the global address space lets wave-uniform reads (source nodes, strengths, body
// ranges) become scalar loads.
template <class T>
using gptr = const T __attribute__((address_space(1))) *;
template <class T>
__device__ __forceinline__ gptr<T> G(const T *p) {
  return (gptr<T>)p;
}

__device__ __forceinline__ float2 ldf2(const float2 *p, long long i) {
  const gptr<float> q = G(reinterpret_cast<const float *>(__builtin_assume_aligned(p, 8)));
  return make_float2(q[2 * i], q[2 * i + 1]);
}
__device__ __forceinline__ double2 ldd2(const double2 *p, long long i) {
  const gptr<double> q = G(reinterpret_cast<const double *>(__builtin_assume_aligned(p, 16)));
  return make_double2(q[2 * i], q[2 * i + 1]);
}

__device__ inline double rcp64(double a) {
  const double y = __builtin_amdgcn_rcp(a);
  const double e = fma(-a, y, 1.0);
  return fma(y, e, y);
}

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

// task encoding: 4 ints per far task (item, chunk, tile, split); 3 per epilogue (item, body, rhs);
// 2 per pack task (item, rhs)

// Far-field precision of an item: MODE 0 float64, 1 float32, 2 bit `it` of the mask (per-item
// precisions of a relaxed mixed batch; the branch is uniform over the workgroup).
struct ItemMask {
  unsigned long long w[kMaxPrecGroups / 64];
};
__device__ __forceinline__ bool item_f32(int mode, const ItemMask &m, int it) {
  return mode == 1 || (mode == 2 && ((m.w[it >> 6] >> (it & 63)) & 1ull));
}

__global__ __launch_bounds__(kBlock) void k_multi_pack(const int *__restrict__ tasks,
                                                      const ItemDesc *__restrict__ D,
                                                      const double *__restrict__ mu,
                                                      double *__restrict__ s64,
                                                      float *__restrict__ s32) {
  const int it = tasks[2 * blockIdx.x], r = tasks[2 * blockIdx.x + 1];
  const ItemDesc &d = D[it];
  const int comps = d.kind == 0 ? 1 : 2;
  const long long len = (long long)d.M * comps;
  const long long base = d.io + r * len;
  for (long long t = threadIdx.x; t < len; t += kBlock) {
    const double v = G(d.w)[t / comps] * mu[base + t];
    s64[base + t] = v;
    if (s32) s32[base + t] = (float)v;
  }
}

template <int R, int MODE>
__global__ __launch_bounds__(kBlock) void k_multi_far_lap(const int *__restrict__ tasks,
                                                         const ItemDesc *__restrict__ D,
                                                         const double *__restrict__ s64,
                                                         const float *__restrict__ s32,
                                                         double *__restrict__ partial,
                                                         const ItemMask f32mask) {
  const int *tk = tasks + 4 * blockIdx.x;
  const int it = tk[0], ch = tk[1], tile = tk[2], sp = tk[3];
  const bool F32 = item_f32(MODE, f32mask, it);
  const ItemDesc &d = D[it];
  const int M = d.M;
  const int i = tile * kT + threadIdx.x;
  const bool valid = i < M;
  const int ii = valid ? i : M - 1;
  const int bi = G(d.body_of)[ii];
  const int r0 = ch * R;  // rhs r0..r0+R-1; those past nrhs read padding or the next item and
                          // only fill partial entries that the epilogue never reads
  const long long sb = d.io + (long long)r0 * M;
  double Gx[R], Gy[R];
#pragma unroll
  for (int r = 0; r < R; ++r) Gx[r] = Gy[r] = 0.0;
  const int c0 = G(d.split_body)[sp], c1 = G(d.split_body)[sp + 1];
  const double cxi = G(d.xc)[bi], cyi = G(d.yc)[bi];
  const float2 pr = ldf2(d.xr, ii);
  const double2 p64 = ldd2(d.xy, ii);
  for (int c = c0; c < c1; ++c) {
    const bool self = (c == bi);
    if (__all(self)) continue;
    const int k0 = G(d.body_ptr)[c], k1 = G(d.body_ptr)[c + 1];
    if (F32) {
      float tx = (float)((cxi - G(d.xc)[c]) + (double)pr.x);
      float ty = (float)((cyi - G(d.yc)[c]) + (double)pr.y);
      tx = self ? kFar32 : tx;
      ty = self ? kFar32 : ty;
      float gx[R], gy[R];
#pragma unroll
      for (int r = 0; r < R; ++r) gx[r] = gy[r] = 0.0f;
#pragma unroll 4
      for (int k = k0; k < k1; ++k) {
        const float2 q = ldf2(d.xr, k);
        const float dx = tx - q.x, dy = ty - q.y;
        const float inv = __builtin_amdgcn_rcpf(fmaf(dx, dx, dy * dy));
#pragma unroll
        for (int r = 0; r < R; ++r) {
          const float sv = s32[sb + (long long)r * M + k];
          const float t = sv * inv;
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
    } else {
      const double tx = self ? kFar64 : p64.x, ty = self ? kFar64 : p64.y;
      double gx[R], gy[R];
#pragma unroll
      for (int r = 0; r < R; ++r) gx[r] = gy[r] = 0.0;
#pragma unroll 2
      for (int k = k0; k < k1; ++k) {
        const double2 q = ldd2(d.xy, k);
        const double dx = tx - q.x, dy = ty - q.y;
        const double inv = rcp64(fma(dx, dx, dy * dy));
#pragma unroll
        for (int r = 0; r < R; ++r) {
          const double sv = s64[sb + (long long)r * M + k];
          const double t = sv * inv;
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
  }
  const long long slot = d.slot + ((long long)ch * d.ntile + tile) * d.nsplit + sp;
  double *o = partial + slot * (R * kT);
  const double a = G(d.nx)[ii], b = G(d.ny)[ii];
#pragma unroll
  for (int r = 0; r < R; ++r) o[r * kT + threadIdx.x] = -(a * Gx[r] + b * Gy[r]) / (2.0 * kPi);
}

template <int R, int MODE>
__global__ __launch_bounds__(kBlock) void k_multi_far_stk(const int *__restrict__ tasks,
                                                         const ItemDesc *__restrict__ D,
                                                         const double *__restrict__ s64,
                                                         const float *__restrict__ s32,
                                                         double *__restrict__ partial,
                                                         const ItemMask f32mask) {
  const int *tk = tasks + 4 * blockIdx.x;
  const int it = tk[0], ch = tk[1], tile = tk[2], sp = tk[3];
  const bool F32 = item_f32(MODE, f32mask, it);
  const ItemDesc &d = D[it];
  const int M = d.M;
  const int i = tile * kT + threadIdx.x;
  const bool valid = i < M;
  const int ii = valid ? i : M - 1;
  const int bi = G(d.body_of)[ii];
  const int r0 = ch * R;
  const long long sb = d.io + (long long)r0 * 2 * M;
  double Gx[R], Gy[R];
#pragma unroll
  for (int r = 0; r < R; ++r) Gx[r] = Gy[r] = 0.0;
  const int c0 = G(d.split_body)[sp], c1 = G(d.split_body)[sp + 1];
  const double cxi = G(d.xc)[bi], cyi = G(d.yc)[bi];
  const float2 pr = ldf2(d.xr, ii);
  const double2 p64 = ldd2(d.xy, ii);
  const double nxi = G(d.nx)[ii], nyi = G(d.ny)[ii];
  for (int c = c0; c < c1; ++c) {
    const bool self = (c == bi);
    if (__all(self)) continue;
    const int k0 = G(d.body_ptr)[c], k1 = G(d.body_ptr)[c + 1];
    if (F32) {
      float tx = (float)((cxi - G(d.xc)[c]) + (double)pr.x);
      float ty = (float)((cyi - G(d.yc)[c]) + (double)pr.y);
      tx = self ? kFar32 : tx;
      ty = self ? kFar32 : ty;
      const float fnx = (float)nxi, fny = (float)nyi;
      float gx[R], gy[R];
#pragma unroll
      for (int r = 0; r < R; ++r) gx[r] = gy[r] = 0.0f;
#pragma unroll 2
      for (int k = k0; k < k1; ++k) {
        const float2 q = ldf2(d.xr, k);
        const float dx = tx - q.x, dy = ty - q.y;
        const float inv = __builtin_amdgcn_rcpf(fmaf(dx, dx, dy * dy));
        const float a = fmaf(dx, fnx, dy * fny) * (inv * inv);
#pragma unroll
        for (int r = 0; r < R; ++r) {
          const float2 sv = ldf2(reinterpret_cast<const float2 *>(s32 + sb + (long long)r * 2 * M), k);
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
    } else {
      const double tx = self ? kFar64 : p64.x, ty = self ? kFar64 : p64.y;
      double gx[R], gy[R];
#pragma unroll
      for (int r = 0; r < R; ++r) gx[r] = gy[r] = 0.0;
#pragma unroll 2
      for (int k = k0; k < k1; ++k) {
        const double2 q = ldd2(d.xy, k);
        const double dx = tx - q.x, dy = ty - q.y;
        const double inv = rcp64(fma(dx, dx, dy * dy));
        const double a = fma(dx, nxi, dy * nyi) * (inv * inv);
#pragma unroll
        for (int r = 0; r < R; ++r) {
          const double2 sv = ldd2(reinterpret_cast<const double2 *>(s64 + sb + (long long)r * 2 * M), k);
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
  }
  const long long slot = d.slot + ((long long)ch * d.ntile + tile) * d.nsplit + sp;
  double *o = partial + slot * (R * kT * 2);
#pragma unroll
  for (int r = 0; r < R; ++r) {
    o[(r * kT + threadIdx.x) * 2] = -Gx[r] / kPi;
    o[(r * kT + threadIdx.x) * 2 + 1] = -Gy[r] / kPi;
  }
}

// Epilogue: self block, diagonal, identity, completion, far partials (in split order).
template <int R>
__global__ __launch_bounds__(kBlock) void k_multi_epi_lap(const int *__restrict__ tasks,
                                                         const ItemDesc *__restrict__ D,
                                                         const double *__restrict__ mu,
                                                         const double *__restrict__ s64,
                                                         const double *__restrict__ partial,
                                                         double *__restrict__ out) {
  __shared__ double sh[4];
  const int it = tasks[3 * blockIdx.x], b = tasks[3 * blockIdx.x + 1], r = tasks[3 * blockIdx.x + 2];
  const ItemDesc &d = D[it];
  const int M = d.M;
  const int k0 = G(d.body_ptr)[b], k1 = G(d.body_ptr)[b + 1];
  const double *s = s64 + d.io + (long long)r * M;
  const double *m = mu + d.io + (long long)r * M;
  double part = 0.0;
  for (int k = k0 + threadIdx.x; k < k1; k += kBlock) part += s[k];
  const double charge = block_sum(part, sh);
  const int ch = r / R, j = r % R;
  for (int base = k0; base < k1; base += kBlock) {
    const int i = base + threadIdx.x;
    const bool valid = i < k1;
    const int ii = valid ? i : k0;
    const double xi = G(d.x)[ii], yi = G(d.y)[ii], a = G(d.nx)[ii], bb = G(d.ny)[ii];
    double gx = 0.0, gy = 0.0;
    for (int k = k0; k < k1; ++k) {
      const double dx = xi - G(d.x)[k], dy = yi - G(d.y)[k];
      const bool same = (k == ii);
      const double inv = rcp64(same ? 1.0 : fma(dx, dx, dy * dy));
      const double t = same ? 0.0 : s[k] * inv;
      gx = fma(dx, t, gx);
      gy = fma(dy, t, gy);
    }
    double v = 0.5 * m[ii] - (a * gx + bb * gy) / (2.0 * kPi) - s[ii] * G(d.kappa)[ii] / (4.0 * kPi) + charge;
    const int tile = ii / kT;
    for (int sp = 0; sp < d.nsplit; ++sp) {
      const long long slot = d.slot + ((long long)ch * d.ntile + tile) * d.nsplit + sp;
      v += partial[slot * (R * kT) + j * kT + (ii - tile * kT)];
    }
    if (valid) out[d.io + (long long)r * M + i] = v;
  }
}

template <int R>
__global__ __launch_bounds__(kBlock) void k_multi_epi_stk(const int *__restrict__ tasks,
                                                         const ItemDesc *__restrict__ D,
                                                         const double *__restrict__ mu,
                                                         const double *__restrict__ s64,
                                                         const double *__restrict__ partial,
                                                         double *__restrict__ out) {
  __shared__ double sh[4];
  const int it = tasks[3 * blockIdx.x], b = tasks[3 * blockIdx.x + 1], r = tasks[3 * blockIdx.x + 2];
  const ItemDesc &d = D[it];
  const int M = d.M;
  const int k0 = G(d.body_ptr)[b], k1 = G(d.body_ptr)[b + 1];
  const double *s = s64 + d.io + (long long)r * 2 * M;
  const double *m = mu + d.io + (long long)r * 2 * M;
  double f1 = 0.0, f2 = 0.0, tq = 0.0;
  for (int k = k0 + threadIdx.x; k < k1; k += kBlock) {
    f1 += s[2 * k];
    f2 += s[2 * k + 1];
    tq += G(d.px)[k] * s[2 * k] + G(d.py)[k] * s[2 * k + 1];
  }
  const double F1 = block_sum(f1, sh), F2 = block_sum(f2, sh), TQ = block_sum(tq, sh);
  const int ch = r / R, j = r % R;
  for (int base = k0; base < k1; base += kBlock) {
    const int i = base + threadIdx.x;
    const bool valid = i < k1;
    const int ii = valid ? i : k0;
    const double xi = G(d.x)[ii], yi = G(d.y)[ii], a = G(d.nx)[ii], bb = G(d.ny)[ii];
    double gx = 0.0, gy = 0.0;
    for (int k = k0; k < k1; ++k) {
      const double dx = xi - G(d.x)[k], dy = yi - G(d.y)[k];
      const bool same = (k == ii);
      const double inv = rcp64(same ? 1.0 : fma(dx, dx, dy * dy));
      const double rn = fma(dx, a, dy * bb);
      const double cc = same ? 0.0 : fma(dx, s[2 * k], dy * s[2 * k + 1]) * rn * (inv * inv);
      gx = fma(cc, dx, gx);
      gy = fma(cc, dy, gy);
    }
    const double t1 = -bb, t2 = a;
    const double ts = t1 * s[2 * ii] + t2 * s[2 * ii + 1];
    const double dg = -G(d.kappa)[ii] / (2.0 * kPi);
    double v1 = 0.5 * m[2 * ii] - gx / kPi + dg * t1 * ts + F1 + G(d.px)[ii] * TQ;
    double v2 = 0.5 * m[2 * ii + 1] - gy / kPi + dg * t2 * ts + F2 + G(d.py)[ii] * TQ;
    const int tile = ii / kT;
    for (int sp = 0; sp < d.nsplit; ++sp) {
      const long long slot = d.slot + ((long long)ch * d.ntile + tile) * d.nsplit + sp;
      const double *o = partial + slot * (R * kT * 2) + (j * kT + (ii - tile * kT)) * 2;
      v1 += o[0];
      v2 += o[1];
    }
    if (valid) {
      out[d.io + (long long)r * 2 * M + 2 * i] = v1;
      out[d.io + (long long)r * 2 * M + 2 * i + 1] = v2;
    }
  }
}

constexpr int kRLap = 8, kRStk = 4;

// Source-body split ranges with about equal node counts.
void split_bodies(const bie_geom *g, int S, std::vector<int> &out) {
  out.clear();
  out.push_back(0);
  for (int s = 1; s < S; ++s) {
    const long long cut = (long long)g->M * s / S;
    int b = out.back();
    while (b < g->N && g->h_body_ptr[b + 1] <= cut) ++b;
    if (b > out.back() && b < g->N) out.push_back(b);
  }
  out.push_back(g->N);
}

int build_plan(MultiPlan &P, const std::vector<MultiItem> &items, const std::vector<char> &active,
               hipStream_t s) {
  const int n = (int)items.size();
  std::vector<ItemDesc> desc(n);
  std::vector<int> far[2], epi[2], pack, splits;
  long long slots[2] = {0, 0};
  std::vector<std::vector<int>> item_splits(n);
  for (int i = 0; i < n; ++i) {
    const MultiItem &m = items[i];
    bie_geom *g = m.g;
    ItemDesc &d = desc[i];
    d.M = g->M;
    d.N = g->N;
    d.kind = m.kind;
    d.nrhs = m.nrhs;
    d.R = m.kind == 0 ? kRLap : kRStk;
    d.nchunk = (m.nrhs + d.R - 1) / d.R;
    d.ntile = (g->M + kT - 1) / kT;
    d.io = m.io;
    d.body_ptr = g->body_ptr;
    d.body_of = g->body_of;
    d.x = g->x; d.y = g->y; d.nx = g->nx; d.ny = g->ny; d.w = g->w; d.kappa = g->kappa;
    d.px = g->px; d.py = g->py; d.xc = g->xc; d.yc = g->yc; d.xy = g->xy; d.xr = g->xr;
    // source splits from the geometry alone (about 4k workgroups for one rhs chunk, at most 16
    // splits, which bounds the partial sums of items with many rhs), so a system's summation
    // order depends neither on the rest of the batch nor on how many rhs share its item
    const long long base = d.ntile;
    const long long want = std::min<long long>(16, (4096 + base - 1) / base);
    split_bodies(g, (int)std::min<long long>(want, std::min(g->N, 64)), item_splits[i]);
    d.nsplit = (int)item_splits[i].size() - 1;
    d.slot = slots[m.kind];
    if (!active[i] || m.fmm) continue;
    slots[m.kind] += (long long)d.nchunk * d.ntile * d.nsplit;
    for (int c = 0; c < d.nchunk; ++c)
      for (int t = 0; t < d.ntile; ++t)
        for (int sp = 0; sp < d.nsplit; ++sp) {
          far[m.kind].push_back(i);
          far[m.kind].push_back(c);
          far[m.kind].push_back(t);
          far[m.kind].push_back(sp);
        }
    for (int b = 0; b < g->N; ++b)
      for (int r = 0; r < m.nrhs; ++r) {
        epi[m.kind].push_back(i);
        epi[m.kind].push_back(b);
        epi[m.kind].push_back(r);
      }
    for (int r = 0; r < m.nrhs; ++r) {
      pack.push_back(i);
      pack.push_back(r);
    }
  }
  // split arrays live in the task buffer; patch pointers after upload
  std::vector<int> split_off(n + 1, 0);
  for (int i = 0; i < n; ++i) split_off[i + 1] = split_off[i] + (int)item_splits[i].size();
  const size_t nint = far[0].size() + far[1].size() + epi[0].size() + epi[1].size() + pack.size() +
                      split_off[n] + 64;
  BIE_TRY(P.task_buf.reserve(nint * 4 + 1024));
  BIE_TRY(P.desc_buf.reserve(n * sizeof(ItemDesc) + 256));
  int *q = P.task_buf.as<int>();
  auto put = [&](const std::vector<int> &v) -> int * {
    int *dst = q;
    if (!v.empty())
      (void)hipMemcpyAsync(dst, v.data(), v.size() * 4, hipMemcpyHostToDevice, s);
    q += v.size();
    return dst;
  };
  P.far_task[0] = put(far[0]);
  P.far_task[1] = put(far[1]);
  P.epi_task[0] = put(epi[0]);
  P.epi_task[1] = put(epi[1]);
  P.pack_task = put(pack);
  for (int i = 0; i < n; ++i) desc[i].split_body = put(item_splits[i]);
  P.desc = P.desc_buf.as<ItemDesc>();
  BIE_HIP_CHECK(hipMemcpyAsync(P.desc, desc.data(), n * sizeof(ItemDesc), hipMemcpyHostToDevice, s));
  BIE_HIP_CHECK(hipStreamSynchronize(s));  // host vectors go out of scope
  P.nfar[0] = (int)far[0].size() / 4;
  P.nfar[1] = (int)far[1].size() / 4;
  P.nepi[0] = (int)epi[0].size() / 3;
  P.nepi[1] = (int)epi[1].size() / 3;
  P.npack = (int)pack.size() / 2;
  P.nslots[0] = slots[0];
  P.nslots[1] = slots[1];
  return BIE_OK;
}

}  // namespace

// out = (1/2 I + K + L) in for every active item (rhs blocks at items[i].io in flat vectors);
// inactive items get out = 0.
int multi_apply(MultiPlan *&P, const std::vector<MultiItem> &items, const std::vector<char> &active,
                int precision, const double *in, double *out, long long Ntot, hipStream_t s,
                const std::vector<char> *item_f32) {
  if (!P) P = new MultiPlan();
  const int n = (int)items.size();
  if (item_f32 && ((int)item_f32->size() != n || n > kMaxPrecGroups)) {
    set_error("multi_apply: per-item precisions need one flag per item and at most 1024 items");
    return BIE_EINVAL;
  }
  // far-field mode: 0 float64, 1 float32, 2 per item (mask)
  ItemMask mask{};
  int mode = precision == BIE_MIXED ? 1 : 0;
  if (item_f32) {
    int nf = 0;
    for (int i = 0; i < n; ++i)
      if ((*item_f32)[i]) {
        mask.w[i >> 6] |= 1ull << (i & 63);
        ++nf;
      }
    mode = nf == 0 ? 0 : nf == n ? 1 : 2;
  }
  auto f32_of = [&](int i) { return mode == 2 ? (*item_f32)[i] != 0 : mode == 1; };
  bool same = P->valid && (int)P->key_gen.size() == n && P->key_active == active;
  for (int i = 0; same && i < n; ++i)
    same = P->key_gen[i] == items[i].g->gen && P->key_kind[i] == items[i].kind &&
           P->key_nrhs[i] == items[i].nrhs && P->key_fmm[i] == (char)items[i].fmm &&
           P->key_io[i] == items[i].io;
  if (!same) {
    P->valid = false;
    BIE_TRY(build_plan(*P, items, active, s));
    P->key_gen.resize(n);
    P->key_kind.resize(n);
    P->key_nrhs.resize(n);
    P->key_fmm.resize(n);
    P->key_io.resize(n);
    for (int i = 0; i < n; ++i) {
      P->key_gen[i] = items[i].g->gen;
      P->key_kind[i] = items[i].kind;
      P->key_nrhs[i] = items[i].nrhs;
      P->key_fmm[i] = (char)items[i].fmm;
      P->key_io[i] = items[i].io;
    }
    P->key_active = active;
    P->valid = true;
  }
  const bool f32 = mode != 0;  // some item needs the float32 strengths
  // workspace: s64 [Np], s32 [Np], partial (Laplace slots, then Stokes slots); Np pads Ntot by
  // R rhs of the longest item so that a far task's last rhs chunk can read past its item
  long long maxlen = 0;
  for (const auto &it : items) maxlen = std::max<long long>(maxlen, (long long)it.g->M * 2);
  const long long Np = align8(Ntot + (long long)kRLap * maxlen);
  const size_t plap = (size_t)P->nslots[0] * kRLap * kT, pstk = (size_t)P->nslots[1] * kRStk * kT * 2;
  const bool grow = P->ws.bytes < (size_t)Np * 12 + (plap + pstk) * 8 + 512;
  BIE_TRY(P->ws.reserve((size_t)Np * 12 + (plap + pstk) * 8 + 512));
  double *s64 = P->ws.as<double>();
  float *s32 = reinterpret_cast<float *>(s64 + Np);
  if (grow) BIE_HIP_CHECK(hipMemsetAsync(P->ws.ptr, 0, P->ws.bytes, s));  // padding stays finite
  double *part = reinterpret_cast<double *>(
      (reinterpret_cast<uintptr_t>(s32 + Np) + 63) & ~uintptr_t(63));
  double *part_lap = part, *part_stk = part + plap;
  // inactive items (and FMM items, filled below) start from zero
  for (int i = 0; i < n; ++i)
    if (!active[i]) {
      const long long len = (long long)items[i].nrhs * items[i].g->M * (items[i].kind == 0 ? 1 : 2);
      BIE_HIP_CHECK(hipMemsetAsync(out + items[i].io, 0, len * sizeof(double), s));
    }
  if (P->npack > 0)
    hipLaunchKernelGGL(k_multi_pack, dim3(P->npack), dim3(kBlock), 0, s, P->pack_task, P->desc, in,
                       s64, f32 ? s32 : nullptr);
  if (P->nfar[0] > 0) {
    ProfScope prof(f32 ? BIE_K_FAR_LAPLACE_F32 : BIE_K_FAR_LAPLACE_F64, s, 0);
    if (mode == 2)
      hipLaunchKernelGGL((k_multi_far_lap<kRLap, 2>), dim3(P->nfar[0]), dim3(kBlock), 0, s,
                         P->far_task[0], P->desc, s64, s32, part_lap, mask);
    else if (mode == 1)
      hipLaunchKernelGGL((k_multi_far_lap<kRLap, 1>), dim3(P->nfar[0]), dim3(kBlock), 0, s,
                         P->far_task[0], P->desc, s64, s32, part_lap, mask);
    else
      hipLaunchKernelGGL((k_multi_far_lap<kRLap, 0>), dim3(P->nfar[0]), dim3(kBlock), 0, s,
                         P->far_task[0], P->desc, s64, s32, part_lap, mask);
  }
  if (P->nfar[1] > 0) {
    ProfScope prof(f32 ? BIE_K_FAR_STOKES_F32 : BIE_K_FAR_STOKES_F64, s, 0);
    if (mode == 2)
      hipLaunchKernelGGL((k_multi_far_stk<kRStk, 2>), dim3(P->nfar[1]), dim3(kBlock), 0, s,
                         P->far_task[1], P->desc, s64, s32, part_stk, mask);
    else if (mode == 1)
      hipLaunchKernelGGL((k_multi_far_stk<kRStk, 1>), dim3(P->nfar[1]), dim3(kBlock), 0, s,
                         P->far_task[1], P->desc, s64, s32, part_stk, mask);
    else
      hipLaunchKernelGGL((k_multi_far_stk<kRStk, 0>), dim3(P->nfar[1]), dim3(kBlock), 0, s,
                         P->far_task[1], P->desc, s64, s32, part_stk, mask);
  }
  {
    ProfScope prof(BIE_K_EPILOGUE, s, 0);
    if (P->nepi[0] > 0)
      hipLaunchKernelGGL(k_multi_epi_lap<kRLap>, dim3(P->nepi[0]), dim3(kBlock), 0, s,
                         P->epi_task[0], P->desc, in, s64, part_lap, out);
    if (P->nepi[1] > 0)
      hipLaunchKernelGGL(k_multi_epi_stk<kRStk>, dim3(P->nepi[1]), dim3(kBlock), 0, s,
                         P->epi_task[1], P->desc, in, s64, part_stk, out);
  }
  BIE_HIP_CHECK(hipGetLastError());
  // FMM items: independent geometries overlap on the stream pool; items of one geometry share
  // its workspace and stay on one stream, in item order
  std::vector<const bie_geom *> gseen;
  std::vector<int> on(n, -1);
  for (int i = 0; i < n; ++i) {
    if (!active[i] || !items[i].fmm) continue;
    size_t gi = std::find(gseen.begin(), gseen.end(), items[i].g) - gseen.begin();
    if (gi == gseen.size()) gseen.push_back(items[i].g);
    on[i] = (int)(gi % kFmmStreams);
  }
  if (gseen.empty()) return BIE_OK;
  if (!P->fork) {
    // all streams are on one device: no system-scope fence at the event markers
    constexpr unsigned kFlags = hipEventDisableTiming | hipEventDisableSystemFence;
    BIE_HIP_CHECK(hipEventCreateWithFlags(&P->fork, kFlags));
    for (int k = 0; k < kFmmStreams; ++k) {
      BIE_HIP_CHECK(hipStreamCreateWithFlags(&P->pool[k], hipStreamNonBlocking));
      BIE_HIP_CHECK(hipEventCreateWithFlags(&P->join[k], kFlags));
    }
  }
  const int used = (int)std::min<size_t>(gseen.size(), kFmmStreams);
  BIE_HIP_CHECK(hipEventRecord(P->fork, s));
  for (int k = 0; k < used; ++k) BIE_HIP_CHECK(hipStreamWaitEvent(P->pool[k], P->fork, 0));
  int rc = BIE_OK;
  for (int i = 0; i < n && rc == BIE_OK; ++i)
    if (on[i] >= 0) {
      items[i].g->fmm_order = items[i].fmm_order;  // the caller's expansion order and leaf size
      items[i].g->fmm_leaf = items[i].fmm_leaf;
      rc = apply_operator(items[i].g, items[i].kind, f32_of(i) ? BIE_MIXED : BIE_FP64, BIE_FMM, 1,
                          1.0, items[i].nrhs, in + items[i].io, out + items[i].io, P->pool[on[i]]);
    }
  for (int k = 0; k < used; ++k) {
    BIE_HIP_CHECK(hipEventRecord(P->join[k], P->pool[k]));
    BIE_HIP_CHECK(hipStreamWaitEvent(s, P->join[k], 0));
  }
  return rc;
}

}  // namespace bie
