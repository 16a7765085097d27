// 2D fast multipole method for the far field of the operator apply (the paper accelerates the
// layer potentials with an FMM and names it only; this design is the library's own).
//
// Both kernels reduce to Cauchy sums F(z) = sum_k Q_k / (z - zeta_k) over complex charges:
//   Laplace:  n_x . sum_k s_k (x - y_k) / |x - y_k|^2 = Re(nu F(z)), nu = n1 + i n2, Q_k = s_k real.
//   Stokes:   sum_k (r.n)(r.s_k) r / |r|^4 (as a complex number) =
//             (1/4) [conj(nu) conj(C'(z) - conj(z) A'(z)) + conj(nu) conj(B(z)) + nu conj(A(z)) + nu A(z)]
//             with A: Q = rho_k, B: Q = conj(rho_k), C: Q = rho_k conj(zeta_k), rho_k = s_k1 + i s_k2,
//             all coordinates taken relative to the root-box centre (the shift cancels in C' - z A').
// Tree: uniform quadtree over the bounding square whose depth makes the mean population of the
// non-empty leaves closest to `leaf` (nodes lie on curves, so populations are uneven); only
// non-empty boxes are stored, in Morton order, so each box is a contiguous run of sorted nodes. Expansions are scaled by the box size h:
//   multipole a_m = sum_k Q_k ((zeta_k - c)/h)^m,   F(z) = sum_m a_m h^m / (z - c)^{m+1}
//   local     F(z) = sum_n b_n ((z - c)/h)^n
// so the 40 M2L operators (offsets d with max(|dx|,|dy|) in {2,3}) and the 4 M2M operators are
// the same at every level (M2L carries one 1/h factor). There is no L2L pass: each target sums
// the local expansions of all its ancestors directly. Near field: the 3 x 3 neighbouring
// leaves, summed directly in float64 for every pair k != i, including pairs on the same body, so
// the epilogue adds only the diagonal limit, identity and completion. Deterministic: one wave per
// box with one lane per coefficient; fixed list orders.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <complex>
#include <cstdlib>
#include <string>
#include <map>
#include <type_traits>
#include <unordered_map>
#include <vector>

#include "internal.h"

namespace bie {

constexpr int kMaxP = 64;

struct FmmTree {
  int p = 0, L = 0, M = 0, nleaf = 0, nbox = 0;
  double size = 0.0, ox = 0.0, oy = 0.0;
  std::vector<int> level_off;  // [L+2]
  // device
  DevBuf buf;
  int *leaf_anc = nullptr;  // per leaf its boxes at levels L, L - 1, ..., 2 [nleaf][L - 1]
  int *perm = nullptr, *leaf_start = nullptr, *leaf_box = nullptr, *child = nullptr,
      *parent = nullptr, *run_ptr = nullptr, *chunk_leaf = nullptr,
      *chunk_start = nullptr;
  int nchunk = 0;
  // evaluation chunks (L2P): up to 64 consecutive sorted targets of at most kEvalLeaves
  // consecutive leaves; ev_start [nev + 1], ev_leaf [nev] (first leaf); ev_maxslot = most
  // ancestor expansions one chunk stages
  int *ev_start = nullptr, *ev_leaf = nullptr;
  int nev = 0, ev_maxslot = 0;
  // M2L groups: 16 target boxes each (grp_tgt, -1 = unused column), their level, and per group
  // the offsets it uses (item_off, increasing) with the 16 source boxes of each (item_src, -1 =
  // none)
  int ngroup = 0, nitem = 0;
  int *grp_ptr = nullptr, *grp_tgt = nullptr, *grp_lvl = nullptr, *item_off = nullptr,
      *item_src = nullptr;
  long long m2l_entries = 0, near_pairs = 0;  // work units for instrumentation
  int2 *run = nullptr;  // near field: per leaf, runs [k0, k1) of sorted nodes in neighbour leaves
  double2 *xs = nullptr, *center = nullptr, *nrm = nullptr;  // sorted coords (rel. root), centres
  double *T_c = nullptr;      // real Hankel vector C[k] = k! / s^k, [2p] (float64 M2L)
  double2 *T_dpow = nullptr;  // powers d^-k, k = 0 .. 16 ceil(p / 16), per offset [40][.]
  double2 *T_tau = nullptr;  // M2M Toeplitz vectors [4][2p] (p zeros, then tau)
  double *fact_out = nullptr, *fact_in = nullptr;  // (-1)^n c^n / n!  and  c^n / n!
  double *inv_h = nullptr;  // [L+1]
  DevBuf work;              // charges + expansions
  // evaluation at arbitrary points (treecode over this tree): per box its level, centre,
  // children and run [lo, hi) of sorted nodes (host); the log-expansion factors
  // T_log[m] = (m - 1)! / s^m (device); the interaction lists of the geometry's read-off points
  std::vector<int> h_level, h_child, h_lo, h_hi;
  std::vector<double2> h_center;
  double *T_log = nullptr;
  struct PointLists *rd = nullptr;
};

// Interaction lists of a set of evaluation points: boxes whose multipoles are evaluated at the
// point (every box at level >= 2 with |z - c| >= sqrt(2) h, i.e. twice its half-diagonal, whose
// parent is not), and the runs [k0, k1) of sorted nodes of the remaining leaves, summed directly.
struct PointLists {
  int npts = 0;
  long long nbox_total = 0, direct_pairs = 0;
  DevBuf buf;
  int *box_ptr = nullptr, *run_ptr = nullptr;  // [npts + 1] each
  int2 *box = nullptr;                         // (box, level)
  int2 *run = nullptr;                         // [k0, k1)
};

struct FmmPlan {
  std::map<std::pair<int, int>, FmmTree *> trees;  // by (order p, leaf population)
  hipStream_t side = nullptr;      // near field, concurrent with the expansion passes
  hipEvent_t fork = nullptr, join = nullptr;
  ~FmmPlan() {
    if (side) {
      (void)hipStreamSynchronize(side);
      (void)hipStreamDestroy(side);
    }
    if (fork) (void)hipEventDestroy(fork);
    if (join) (void)hipEventDestroy(join);
    for (auto &kv : trees) {
      if (kv.second->rd) {
        kv.second->rd->buf.release();
        delete kv.second->rd;
      }
      kv.second->buf.release();
      kv.second->work.release();
      delete kv.second;
    }
  }
};

void fmm_destroy(FmmPlan *p) { delete p; }

namespace {

using cd = std::complex<double>;

// Complex numbers as float2 / double2; the expansions of the mixed-precision Laplace apply are
// float, everything else double.
template <class T> struct cx_of;
template <> struct cx_of<double> { using type = double2; };
template <> struct cx_of<float> { using type = float2; };
template <class T>
using cx = typename cx_of<T>::type;

template <class T>
__device__ inline cx<T> mkc(T a, T b) {
  cx<T> r;
  r.x = a;
  r.y = b;
  return r;
}
template <class V>
__device__ inline V cmul(V a, V b) {
  V r;
  r.x = a.x * b.x - a.y * b.y;
  r.y = a.x * b.y + a.y * b.x;
  return r;
}
template <class V>
__device__ inline V cfma(V a, V b, V c) {  // a*b + c
  V r;
  r.x = fma(a.x, b.x, fma(-a.y, b.y, c.x));
  r.y = fma(a.x, b.y, fma(a.y, b.x, c.y));
  return r;
}

__device__ inline double rcp64(double a) {
  const double y = __builtin_amdgcn_rcp(a);
  const double e = fma(-a, y, 1.0);
  return fma(y, e, y);
}

// Source strengths s = w mu (written to s64 in node order, as the epilogue reads them) and, in
// sorted order, the charges: Laplace set r is (s, 0) (in float when Qf is given); Stokes sets 3r,
// 3r+1, 3r+2 are rho, conj(rho), rho conj(z). Also the near-field source records
// S4[r][j] = (x, y, s, 0), resp. (x, y, rho), always in float64.
__global__ void k_gather(int M, int R, int kind, const int *__restrict__ perm,
                         const double2 *__restrict__ xs, const double *__restrict__ wq,
                         const double *__restrict__ mu, double *__restrict__ s64,
                         double2 *__restrict__ Q, float2 *__restrict__ Qf,
                         double4 *__restrict__ S4) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= M) return;
  const int k = perm[j];
  const double2 z = xs[j];
  const double wk = wq[k];
  for (int r = 0; r < R; ++r) {
    if (kind == 0) {
      const double v = wk * mu[(size_t)r * M + k];
      s64[(size_t)r * M + k] = v;
      if (Qf)
        Qf[(size_t)r * M + j] = make_float2((float)v, 0.0f);
      else
        Q[(size_t)r * M + j] = make_double2(v, 0.0);
      S4[(size_t)r * M + j] = make_double4(z.x, z.y, v, 0.0);
    } else {
      const double2 rho = make_double2(wk * mu[(size_t)r * 2 * M + 2 * k],
                                       wk * mu[(size_t)r * 2 * M + 2 * k + 1]);
      s64[(size_t)r * 2 * M + 2 * k] = rho.x;
      s64[(size_t)r * 2 * M + 2 * k + 1] = rho.y;
      Q[(size_t)(3 * r) * M + j] = rho;
      Q[(size_t)(3 * r + 1) * M + j] = make_double2(rho.x, -rho.y);
      Q[(size_t)(3 * r + 2) * M + j] = cmul(rho, make_double2(z.x, -z.y));
      S4[(size_t)r * M + j] = make_double4(z.x, z.y, rho.x, rho.y);
    }
  }
}

// Wave-uniform read of lane l's value (l a compile-time or uniform index).
__device__ __forceinline__ double rl(double v, int l) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), l);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), l);
  return __hiloint2double(hi, lo);
}
__device__ __forceinline__ float rl(float v, int l) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}

// Launch order to XCD-contiguous work: consecutive workgroups go round-robin to the eight XCDs,
// each with its own L2. Workgroup i (of n along x) takes item (i % 8) * q + min(i % 8, r) + i / 8
// (q = n / 8, r = n % 8), so each XCD works through one contiguous range of items, and items
// that share inputs (neighbouring leaves and boxes in Morton order) share its L2. A bijection
// on [0, n).
__device__ __forceinline__ int xcd_item(int i, int n) {
  const int q = n >> 3, r = n & 7, x = i & 7;
  return x * q + min(x, r) + (i >> 3);
}

// Wave priority of the expansion chain (P2M, M2M, M2L, evaluation). The near field runs on a
// second stream beside the chain and shares its compute units; at equal priority it slows the
// chain's latency-bound kernels. Raised, the chain's waves issue first where both are resident
// and the near field takes the remaining issue slots (it stays at the default, 0).
constexpr int kChainPrio = 3;

// P2M: grid (leaves, nsets / NS), one wave per leaf and NS charge sets. Multipole coefficients of
// the leaf, u_n = (s^n/n!) sum_j q_j w_j^n with w_j = (z_j - c)/h and the table scale s (fact_in).
// Lane (g, b) = (lane % 8, lane / 8) takes the sources j = j0 + g, j0 + g + 8, ... and the P/8
// coefficients n = b P/8 .. (b + 1) P/8 - 1: per source it forms w^(b P/8) (w^(P/8) raised to b by
// squaring) and the following powers by running products, accumulating in registers. The eight
// lanes of each coefficient block are then added by three shuffle steps. Fixed order: the result
// is reproducible. With NS > 1 (the three charge sets of a Stokes right-hand side) the powers of
// w are formed once per source for all NS sets.
template <int P, class T, int NS>
__global__ __launch_bounds__(64) void k_p2m(int M, int nbox, double inv_h,
                                           const int *__restrict__ leaf_start,
                                           const int *__restrict__ leaf_box,
                                           const double2 *__restrict__ center,
                                           const double2 *__restrict__ xs,
                                           const cx<T> *__restrict__ Q,
                                           const double *__restrict__ fact_in,
                                           cx<T> *__restrict__ Mexp) {
  __builtin_amdgcn_s_setprio(kChainPrio);
  constexpr int NB = P / 8;          // coefficients per lane
  constexpr int U = NS == 1 ? 8 : 4;  // sources per lane in one batch of loads
  const int leaf = blockIdx.x, set0 = blockIdx.y * NS, lane = threadIdx.x;
  const int g = lane & 7, b = lane >> 3;
  const int box = leaf_box[leaf];
  const double2 c = center[box];
  cx<T> acc[NS][NB];
#pragma unroll
  for (int e = 0; e < NS; ++e)
#pragma unroll
    for (int k = 0; k < NB; ++k) acc[e][k] = mkc<T>(0, 0);
  const int j0 = leaf_start[leaf], j1 = leaf_start[leaf + 1];
  // 8 U sources at a time: every load of the batch is issued before the first product (lanes
  // past the leaf's end take the leaf's first coordinate and zero charges, so they add zero)
  for (int jb = j0; jb < j1; jb += 8 * U) {
    double2 zz[U];
    cx<T> qq[U][NS];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int j = jb + g + 8 * u;
      const bool ok = j < j1;
      zz[u] = xs[ok ? j : j0];
#pragma unroll
      for (int e = 0; e < NS; ++e) qq[u][e] = ok ? Q[(size_t)(set0 + e) * M + j] : mkc<T>(0, 0);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (jb + 8 * u >= j1) break;  // uniform over the wave
      // leaf-relative coordinates formed in float64
      const cx<T> w = mkc<T>((T)((zz[u].x - c.x) * inv_h), (T)((zz[u].y - c.y) * inv_h));
      cx<T> wb = w;  // w^NB
#pragma unroll
      for (int k = 1; k < NB; ++k) wb = cmul(wb, w);
      cx<T> t[NS];
      if constexpr (NS == 1) {
        t[0] = qq[u][0];  // q w^(b NB), by squaring over the three bits of b
#pragma unroll
        for (int bit = 0; bit < 3; ++bit) {
          const cx<T> tw = cmul(t[0], wb);
          const bool use = (b >> bit) & 1;  // per component (a select of the pair is not)
          t[0].x = use ? tw.x : t[0].x;
          t[0].y = use ? tw.y : t[0].y;
          wb = cmul(wb, wb);
        }
      } else {
        cx<T> pw = mkc<T>(1, 0);  // w^(b NB), by squaring over the three bits of b
#pragma unroll
        for (int bit = 0; bit < 3; ++bit) {
          const cx<T> tw = cmul(pw, wb);
          const bool use = (b >> bit) & 1;
          pw.x = use ? tw.x : pw.x;
          pw.y = use ? tw.y : pw.y;
          if (bit < 2) wb = cmul(wb, wb);
        }
#pragma unroll
        for (int e = 0; e < NS; ++e) t[e] = cmul(qq[u][e], pw);
      }
#pragma unroll
      for (int k = 0; k < NB; ++k) {
#pragma unroll
        for (int e = 0; e < NS; ++e) {
          acc[e][k].x += t[e].x;
          acc[e][k].y += t[e].y;
        }
        if (k + 1 < NB) {
#pragma unroll
          for (int e = 0; e < NS; ++e) t[e] = cmul(t[e], w);
        }
      }
    }
  }
#pragma unroll
  for (int e = 0; e < NS; ++e)
#pragma unroll
    for (int k = 0; k < NB; ++k)
#pragma unroll
      for (int off = 1; off < 8; off <<= 1) {
        acc[e][k].x += __shfl_xor(acc[e][k].x, off, 64);
        acc[e][k].y += __shfl_xor(acc[e][k].y, off, 64);
      }
  if (g == 0) {
#pragma unroll
    for (int e = 0; e < NS; ++e) {
      cx<T> *o = Mexp + ((size_t)(set0 + e) * nbox + box) * P;
#pragma unroll
      for (int k = 0; k < NB; ++k) {
        const int n = NB * b + k;
        const T f = (T)fact_in[n];
        o[n] = mkc<T>(acc[e][k].x * f, acc[e][k].y * f);
      }
    }
  }
}

// M2M is a Toeplitz product with one vector per child position: with d = (child centre - parent
// centre) / parent size = (+-1/4, +-1/4), the table scale s and tau[k] = (s d)^k / k!,
//   u_parent[n] = sum_{m <= n} 2^-m u_child[m] tau[n - m]   (stored u_n = a_n s^n / n!).
// The table holds, per position, p zeros followed by tau[0..p-1], so that the sum reads tau at a
// lane-dependent offset without a bound test. It sits in LDS; the source coefficient of step m
// is read from lane m (readlane, wave-uniform).

// M2M for one level: one workgroup per (parent box, set) with a grid stride; wave c translates
// the child at position c, and the four contributions are added through LDS in position order.
template <int P, class T>
__global__ __launch_bounds__(256) void k_m2m(int nb, int off, int nbox, int nsets,
                                            const int *__restrict__ child,
                                            const double2 *__restrict__ tau, cx<T> *Mexp) {
  __builtin_amdgcn_s_setprio(kChainPrio);
  __shared__ cx<T> tp[8 * P];
  __shared__ cx<T> part[4 * 64];
  for (int i = threadIdx.x; i < 8 * P; i += blockDim.x) tp[i] = mkc<T>((T)tau[i].x, (T)tau[i].y);
  __syncthreads();
  const int lane = threadIdx.x & 63;
  const int n = lane < P ? lane : P - 1;
  const int cpos = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const long long total = (long long)nb * nsets;
  for (long long item = blockIdx.x; item < total; item += gridDim.x) {
    const int set = (int)(item / nb);
    const int b = off + (int)(item % nb);
    cx<T> a0 = mkc<T>(0, 0), a1 = a0;
    const int ch = child[4 * b + cpos];
    if (ch >= 0) {
      const cx<T> u = Mexp[((size_t)set * nbox + ch) * P + n];
      const cx<T> v = mkc<T>(ldexp(u.x, -n), ldexp(u.y, -n));
      const cx<T> *tc = tp + cpos * 2 * P + P + n;  // tc[-m] = tau[n - m], zero for m > n
#pragma unroll
      for (int m = 0; m < P; m += 2) {
        a0 = cfma(mkc<T>(rl(v.x, m), rl(v.y, m)), tc[-m], a0);
        a1 = cfma(mkc<T>(rl(v.x, m + 1), rl(v.y, m + 1)), tc[-m - 1], a1);
      }
    }
    part[cpos * 64 + lane] = mkc<T>(a0.x + a1.x, a0.y + a1.y);
    __syncthreads();
    if (cpos == 0 && lane < P) {
      const cx<T> r0 = part[lane], r1 = part[64 + lane], r2 = part[128 + lane], r3 = part[192 + lane];
      Mexp[((size_t)set * nbox + b) * P + n] =
          mkc<T>((r0.x + r1.x) + (r2.x + r3.x), (r0.y + r1.y) + (r2.y + r3.y));
    }
    __syncthreads();
  }
}

// M2L for all boxes of levels >= 2, written into Lexp, on the matrix cores. Multipoles are stored
// as u_m = a_m s^m / m! (s: the table scale). For a box offset d (in units of the box size) the
// operator is the Hankel product b_n = (1/h) f_n sum_m u_m V_d[m + n] with f_n = (-1)^n s^n / n!
// and V_d[k] = k! / (s^k d^(k+1)) = C[k] d^-(k+1), where C[k] = k! / s^k is real. So
//   b_n = (1/h) f_n d^-(n+1) sum_m C[m + n] (u_m d^-m):
// a complex scaling of the source, one real Hankel matrix C shared by every offset, and a complex
// scaling of the product. Target boxes are grouped 16 at a time (same level, same position in the
// parent, so their interaction lists share most offsets); an item is one offset d of a group with
// the 16 sources at that offset (zero columns where a target has none). Per item, the real and
// imaginary parts of the 16 scaled sources form two 16-column B operands, C's row tiles (read
// from LDS per item) the A operands of 16x16x4 float64 MFMAs, and the lane scales
// the two results (the real and imaginary parts of C u~) by d^-(n+1) into its complex
// accumulators. MFMA lane layout: lane (j, q) = (lane % 16, lane / 16) holds A[j][q] and B[q][j]
// of a k-step and rows q + 4r of column j of an accumulator tile.
// One workgroup of four waves per (group, set): wave w takes items w, w + 4, ... in order, and
// the four partial sums are added in wave order through LDS at the end (a fixed order).
typedef double m2l_d4 __attribute__((ext_vector_type(4)));

template <int P>
struct M2lShape {
  static constexpr int RT = (P + 15) / 16;   // row tiles of C (rows >= P are zero)
  static constexpr int KS = P / 4;           // k-steps
  static constexpr int DP = 16 * RT + 1;     // powers d^-k, k = 0 .. 16 RT, per offset
  static constexpr int CN = 16 * RT + P;     // C[k] for k < CN (zeros from 2p - 1 on)
  static constexpr int TABLE = 40 * DP * 2 + CN;  // doubles
  static constexpr int RED = 4 * RT * 4 * 2 * 64;
  static constexpr int LDS = TABLE > RED ? TABLE : RED;
};
// whether an item's sources are loaded during the previous item's products: the extra registers
// leave two workgroups per CU (up to order 40); otherwise items run one after another in fewer
// registers, three workgroups per CU
template <int P>
constexpr bool kM2lPrefetch = P <= 40;

template <int P>
__global__ __launch_bounds__(256, kM2lPrefetch<P> ? 2 : 3) void k_m2l(int g0, int nbox, const int *__restrict__ grp_ptr,
                                               const int *__restrict__ grp_tgt,
                                               const int *__restrict__ grp_lvl,
                                               const int *__restrict__ item_off,
                                               const int *__restrict__ item_src,
                                               const double *__restrict__ inv_h,
                                               const double *__restrict__ fact_out,
                                               const double *__restrict__ Ctab,
                                               const double2 *__restrict__ Dpow,
                                               const double2 *__restrict__ Mexp,
                                               double2 *__restrict__ Lexp) {
  __builtin_amdgcn_s_setprio(kChainPrio);
  using S = M2lShape<P>;
  constexpr int RT = S::RT, KS = S::KS, DP = S::DP;
  __shared__ double lds[S::LDS];
  double2 *dps = reinterpret_cast<double2 *>(lds);
  double *cs = lds + 40 * DP * 2;
  for (int i = threadIdx.x; i < 40 * DP; i += blockDim.x) dps[i] = Dpow[i];
  for (int i = threadIdx.x; i < S::CN; i += blockDim.x) cs[i] = i < 2 * P - 1 ? Ctab[i] : 0.0;
  const int g = g0 + blockIdx.x, set = blockIdx.y;
  const int lane = threadIdx.x & 63, j = lane & 15, q = lane >> 4;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  double br[RT][4], bi[RT][4];
#pragma unroll
  for (int t = 0; t < RT; ++t)
#pragma unroll
    for (int r = 0; r < 4; ++r) br[t][r] = bi[t][r] = 0.0;
  const double2 *Ms = Mexp + (size_t)set * nbox * P;
  const int i0 = grp_ptr[g], i1 = grp_ptr[g + 1];
  // one item's products: one row tile at a time, the real and imaginary products, then the
  // scaling by d^-(n+1) into the accumulators. A[n][m] = C[n + m]; rows n >= P (the last
  // tile's padding) hold finite values that are never written out.
  auto products = [&](const double *bre, const double *bim, const double2 *dp, int zoff) {
#pragma unroll
    for (int t = 0; t < RT; ++t) {
      const double *ca = cs + 16 * t + j + q + zoff;
      m2l_d4 yr = {0.0, 0.0, 0.0, 0.0}, yi = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int kk = 0; kk < KS; ++kk) {
        const double a = ca[4 * kk];
        yr = __builtin_amdgcn_mfma_f64_16x16x4f64(a, bre[kk], yr, 0, 0, 0);
        yi = __builtin_amdgcn_mfma_f64_16x16x4f64(a, bim[kk], yi, 0, 0, 0);
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const double2 pw = dp[16 * t + q + 4 * r + 1];  // d^-(n+1)
        br[t][r] = fma(yr[r], pw.x, fma(-yi[r], pw.y, br[t][r]));
        bi[t][r] = fma(yr[r], pw.y, fma(yi[r], pw.x, bi[t][r]));
      }
    }
  };
  // this lane's sources u_src[m], m = 4 kk + q, scaled by d^-m; a missing source (src < 0)
  // reads box 0, then zeros
  auto prescale = [&](const double2 *u, int src, const double2 *dp, double *bre, double *bim) {
#pragma unroll
    for (int kk = 0; kk < KS; ++kk) {
      const double2 pw = dp[4 * kk + q];  // d^-m
      const double ur = src < 0 ? 0.0 : u[kk].x, ui = src < 0 ? 0.0 : u[kk].y;
      bre[kk] = fma(ur, pw.x, -ui * pw.y);
      bim[kk] = fma(ur, pw.y, ui * pw.x);
    }
  };
  __syncthreads();
  if constexpr (kM2lPrefetch<P>) {
    // software pipeline over the wave's items it = i0 + w, i0 + w + 4, ...: the sources of the
    // next item are loaded before this item's products and pre-scaled after them; the indices
    // run one item further ahead
    int it = i0 + w;
    int s1 = -1, o1 = 0, s2 = -1, o2 = 0;  // (source, offset) of items it, it + 4
    if (it < i1) { s1 = item_src[it * 16 + j]; o1 = item_off[it]; }
    if (it + 4 < i1) { s2 = item_src[(it + 4) * 16 + j]; o2 = item_off[it + 4]; }
    double bre[KS], bim[KS];
    double2 un[KS];
    if (it < i1) {
      const double2 *up = Ms + (size_t)max(s1, 0) * P + q;
#pragma unroll
      for (int kk = 0; kk < KS; ++kk) un[kk] = up[4 * kk];
      prescale(un, s1, dps + o1 * DP, bre, bim);
    }
    for (; it < i1; it += 4) {
      const double2 *dp = dps + o1 * DP;
      s1 = s2; o1 = o2;  // item it + 4
      const bool more = it + 4 < i1;
      if (more) {
        const double2 *up = Ms + (size_t)max(s1, 0) * P + q;
#pragma unroll
        for (int kk = 0; kk < KS; ++kk) un[kk] = up[4 * kk];
      }
      if (it + 8 < i1) { s2 = item_src[(it + 8) * 16 + j]; o2 = item_off[it + 8]; }
      // the C entries are read from LDS per item (an opaque zero keeps the compiler from
      // holding all of them in registers across items)
      int zoff = 0;
      asm volatile("" : "+v"(zoff));
      products(bre, bim, dp, zoff);
      if (more) prescale(un, s1, dps + o1 * DP, bre, bim);
    }
  } else {
    // one item after another: its sources, their scaling, the products
    for (int it = i0 + w; it < i1; it += 4) {
      const int src = item_src[it * 16 + j];
      const double2 *dp = dps + item_off[it] * DP;
      const double2 *up = Ms + (size_t)max(src, 0) * P + q;
      double2 u[KS];
#pragma unroll
      for (int kk = 0; kk < KS; ++kk) u[kk] = up[4 * kk];
      double bre[KS], bim[KS];
      prescale(u, src, dp, bre, bim);
      products(bre, bim, dp, 0);
    }
  }
  __syncthreads();  // the tables are no longer read: their LDS holds the partial sums
  double *red = lds;
#pragma unroll
  for (int t = 0; t < RT; ++t)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      red[(((w * RT + t) * 4 + r) * 2) * 64 + lane] = br[t][r];
      red[(((w * RT + t) * 4 + r) * 2 + 1) * 64 + lane] = bi[t][r];
    }
  __syncthreads();
  const int tb = grp_tgt[g * 16 + j];
  if (tb < 0) return;
  const double sc = inv_h[grp_lvl[g]];
  double2 *out = Lexp + ((size_t)set * nbox + tb) * P;
  for (int t = w; t < RT; t += 4)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int n = 16 * t + q + 4 * r;
      if (n >= P) continue;
      double vr = 0.0, vi = 0.0;
#pragma unroll
      for (int ww = 0; ww < 4; ++ww) {
        vr += red[(((ww * RT + t) * 4 + r) * 2) * 64 + lane];
        vi += red[(((ww * RT + t) * 4 + r) * 2 + 1) * 64 + lane];
      }
      const double f = sc * fact_out[n];
      out[n] = make_double2(vr * f, vi * f);
    }
}

// The factored M2L of k_m2l in float32 for the mixed-precision Laplace apply: the same tables
// (C[k] = k!/s^k, the powers d^-k of the 40 offsets) converted to float32 in LDS, the same
// groups and items, the Hankel product on 16x16x4 float32 MFMAs (twice the float64 rate). The
// operand layout is that of the float64 product; the accumulator layout differs: lane (j, q)
// holds rows 4q + r of column j, i.e. coefficient n = 16 t + 4 q + r of target column j.
typedef float m2l_f4v __attribute__((ext_vector_type(4)));

template <int P>
struct M2lShapeF {
  static constexpr int RT = (P + 15) / 16;
  static constexpr int KS = P / 4;
  static constexpr int DP = 16 * RT + 1;
  static constexpr int CN = 16 * RT + P;
  static constexpr int TABLE = 40 * DP * 2 + CN;  // floats
  static constexpr int RED = 4 * RT * 4 * 2 * 64;
  static constexpr int LDS = TABLE > RED ? TABLE : RED;
};

template <int P>
__global__ __launch_bounds__(256, 4) void k_m2l_fac_f32(
    int g0, int nbox, const int *__restrict__ grp_ptr, const int *__restrict__ grp_tgt,
    const int *__restrict__ grp_lvl, const int *__restrict__ item_off,
    const int *__restrict__ item_src, const double *__restrict__ inv_h,
    const double *__restrict__ fact_out, const double *__restrict__ Ctab,
    const double2 *__restrict__ Dpow, const float2 *__restrict__ Mexp,
    float2 *__restrict__ Lexp) {
  __builtin_amdgcn_s_setprio(kChainPrio);
  using S = M2lShapeF<P>;
  constexpr int RT = S::RT, KS = S::KS, DP = S::DP;
  __shared__ float lds[S::LDS];
  float2 *dps = reinterpret_cast<float2 *>(lds);
  float *cs = lds + 40 * DP * 2;
  for (int i = threadIdx.x; i < 40 * DP; i += blockDim.x) {
    const double2 v = Dpow[i];
    dps[i] = make_float2((float)v.x, (float)v.y);
  }
  for (int i = threadIdx.x; i < S::CN; i += blockDim.x) cs[i] = i < 2 * P - 1 ? (float)Ctab[i] : 0.0f;
  const int g = g0 + blockIdx.x, set = blockIdx.y;
  const int lane = threadIdx.x & 63, j = lane & 15, q = lane >> 4;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  float br[RT][4], bi[RT][4];
#pragma unroll
  for (int t = 0; t < RT; ++t)
#pragma unroll
    for (int r = 0; r < 4; ++r) br[t][r] = bi[t][r] = 0.0f;
  const float2 *Ms = Mexp + (size_t)set * nbox * P;
  const int i0 = grp_ptr[g], i1 = grp_ptr[g + 1];
  __syncthreads();
  for (int it = i0 + w; it < i1; it += 4) {
    const int src = item_src[it * 16 + j];
    const float2 *dp = dps + item_off[it] * DP;
    const float2 *up = Ms + (size_t)max(src, 0) * P + q;
    float2 u[KS];
#pragma unroll
    for (int kk = 0; kk < KS; ++kk) u[kk] = up[4 * kk];
    // this lane's sources u_m, m = 4 kk + q, scaled by d^-m (a missing source: zeros)
    float bre[KS], bim[KS];
#pragma unroll
    for (int kk = 0; kk < KS; ++kk) {
      const float2 pw = dp[4 * kk + q];
      const float ur = src < 0 ? 0.0f : u[kk].x, ui = src < 0 ? 0.0f : u[kk].y;
      bre[kk] = fmaf(ur, pw.x, -ui * pw.y);
      bim[kk] = fmaf(ur, pw.y, ui * pw.x);
    }
#pragma unroll
    for (int t = 0; t < RT; ++t) {
      const float *ca = cs + 16 * t + j + q;
      m2l_f4v yr = {0.0f, 0.0f, 0.0f, 0.0f}, yi = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
      for (int kk = 0; kk < KS; ++kk) {
        const float a = ca[4 * kk];
        yr = __builtin_amdgcn_mfma_f32_16x16x4f32(a, bre[kk], yr, 0, 0, 0);
        yi = __builtin_amdgcn_mfma_f32_16x16x4f32(a, bim[kk], yi, 0, 0, 0);
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const float2 pw = dp[16 * t + 4 * q + r + 1];  // d^-(n+1)
        br[t][r] = fmaf(yr[r], pw.x, fmaf(-yi[r], pw.y, br[t][r]));
        bi[t][r] = fmaf(yr[r], pw.y, fmaf(yi[r], pw.x, bi[t][r]));
      }
    }
  }
  __syncthreads();  // the tables are no longer read: their LDS holds the partial sums
  float *red = lds;
#pragma unroll
  for (int t = 0; t < RT; ++t)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      red[(((w * RT + t) * 4 + r) * 2) * 64 + lane] = br[t][r];
      red[(((w * RT + t) * 4 + r) * 2 + 1) * 64 + lane] = bi[t][r];
    }
  __syncthreads();
  const int tb = grp_tgt[g * 16 + j];
  if (tb < 0) return;
  const double sc = inv_h[grp_lvl[g]];
  float2 *out = Lexp + ((size_t)set * nbox + tb) * P;
  for (int t = w; t < RT; t += 4)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int n = 16 * t + 4 * q + r;
      if (n >= P) continue;
      float vr = 0.0f, vi = 0.0f;
#pragma unroll
      for (int ww = 0; ww < 4; ++ww) {
        vr += red[(((ww * RT + t) * 4 + r) * 2) * 64 + lane];
        vi += red[(((ww * RT + t) * 4 + r) * 2 + 1) * 64 + lane];
      }
      const float f = (float)(sc * fact_out[n]);
      out[n] = make_float2(vr * f, vi * f);
    }
}

// Local expansion value F and derivative F' at w = (z - c)/h (Horner); F' includes 1/h. The
// coefficients are wave-uniform (one box per wave) and P is a compile-time constant, so the
// loads batch into a few scalar loads.
template <int P>
__device__ inline void eval_local(const double2 *b, double2 w, double ih, double2 &F, double2 &dF) {
  F = b[P - 1];
  dF = make_double2(0.0, 0.0);
#pragma unroll
  for (int n = P - 1; n >= 1; --n) {
    dF = cfma(dF, w, F);
    F = cfma(F, w, b[n - 1]);
  }
  dF = make_double2(dF.x * ih, dF.y * ih);
}

template <int P, class V>
__device__ inline V eval_value(const V *b, V w) {
  V F = b[P - 1];
#pragma unroll
  for (int n = P - 1; n >= 1; --n) F = cfma(F, w, b[n - 1]);
  return F;
}

// Near field. The neighbour leaves of a leaf (itself included) form a few runs of consecutive
// sorted nodes, whose source records (x, y, s, 0) or (x, y, rho) are the same for all targets of
// the leaf. A workgroup of four waves takes a chunk of up to 64 targets of one leaf: wave w holds
// targets 16 w .. 16 w + 15 of the chunk (lane % 16), and lane group g = lane / 16 takes the
// records g, g + 4, g + 8, ... of the staged records, so a leaf of n targets keeps ceil(n / 16)
// waves busy with 16 lanes per target row instead of one wave with n of 64 lanes. The four
// groups' sums are added at the end in a fixed order.
//
// No pair is masked. The pair of a target with itself has r = 0 exactly (its record holds the
// same coordinates): |r|^2 is raised to kSelfFloor, far below the square of any distance between
// two nodes, so the factor stays finite and the pair adds r times it, i.e. zero. Staged segments
// are padded to a multiple of 32 records with zero-weight records far away, which add zero too.
constexpr double kSelfFloor = 1e-100;
constexpr double kNearPad = 1e50;  // coordinates of a padding record

// One step over the eight records rec (this lane's group). The reciprocals of |r|^2 are formed
// two at a time from one reciprocal of their product, 1/a = b / (ab) and 1/b = a / (ab): the
// quarter-rate reciprocal is issued once per two pairs. |r|^2 lies in [kSelfFloor, about
// 2 kNearPad^2], so ab stays within the float64 range.
template <bool STOKES>
__device__ __forceinline__ void near_step(const double4 *rec, double2 z, double2 nv, double &gx,
                                          double &gy) {
#pragma unroll
  for (int u = 0; u < 8; u += 2) {
    const double dx0 = z.x - rec[u].x, dy0 = z.y - rec[u].y;
    const double dx1 = z.x - rec[u + 1].x, dy1 = z.y - rec[u + 1].y;
    const double a = fmax(fma(dx0, dx0, dy0 * dy0), kSelfFloor);
    const double b = fmax(fma(dx1, dx1, dy1 * dy1), kSelfFloor);
    const double y = rcp64(a * b);
    const double inv0 = b * y, inv1 = a * y;
    double t0, t1;
    if (STOKES) {
      const double rn0 = fma(dx0, nv.x, dy0 * nv.y), rn1 = fma(dx1, nv.x, dy1 * nv.y);
      t0 = fma(dx0, rec[u].z, dy0 * rec[u].w) * rn0 * (inv0 * inv0);
      t1 = fma(dx1, rec[u + 1].z, dy1 * rec[u + 1].w) * rn1 * (inv1 * inv1);
    } else {
      t0 = rec[u].z * inv0;
      t1 = rec[u + 1].z * inv1;
    }
    gx = fma(dx0, t0, gx);
    gy = fma(dy0, t0, gy);
    gx = fma(dx1, t1, gx);
    gy = fma(dy1, t1, gy);
  }
}

// Sum over the staged records at LDS positions [0, n) (n a multiple of 32): this lane's group
// reads positions g, g + 4, ... by LDS broadcast (four addresses per read, one per group), eight
// per step.
template <bool STOKES>
__device__ __forceinline__ void near_seg(const double4 *buf, int n, int g, double2 z, double2 nv,
                                         double &gx, double &gy) {
  for (int k = 0; k < n; k += 32) {
    double4 rec[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) rec[u] = buf[k + 4 * u + g];
    near_step<STOKES>(rec, z, nv, gx, gy);
  }
}

// LDS records per workgroup (a multiple of 32). A leaf whose runs hold at most this many records
// (after padding) has them all staged at once, back to back: one load latency and one barrier.
// Larger neighbourhoods are read run by run in blocks of this size.
constexpr int kNearCap = 512;

// Copies n records src[0 .. n) to buf[at ..], then zero-weight padding up to a multiple of 32
// records; returns the padded count.
__device__ __forceinline__ int near_stage(const double4 *__restrict__ src, int n, double4 *buf,
                                          int at) {
  const int np = (n + 31) & ~31;
  for (int t = threadIdx.x; t < np; t += blockDim.x)
    buf[at + t] = t < n ? src[t] : make_double4(kNearPad, kNearPad, 0.0, 0.0);
  return np;
}

// Near field: grid (target chunks, R), 256 threads. Laplace writes -(1/2pi) n.(sum over the
// neighbour leaves, k != i, of s_k r/|r|^2); Stokes writes -(1/pi) sum over the neighbour leaves,
// k != i, of (r.n)(r.rho_k) r/|r|^4 (two components per node). Waves without targets (busy false,
// uniform over the wave) take part in the copies and barriers only. At least five waves per
// SIMD (at most 102 VGPRs instead of 104): the kernel shares the compute units with the
// expansion chain, and its smaller register footprint leaves room for the chain's waves.
// Chunks are taken in XCD-contiguous order (xcd_item): neighbouring leaves, which stage mostly
// the same source records, then run on one XCD and share its L2.
template <bool STOKES>
__global__ __launch_bounds__(256, 5) void k_near(
    int M, const int *__restrict__ leaf_start, const double2 *__restrict__ xs,
    const double2 *__restrict__ nrm, const int *__restrict__ perm,
    const int *__restrict__ run_ptr, const int2 *__restrict__ run,
    const int *__restrict__ chunk_leaf, const int *__restrict__ chunk_start,
    const double4 *__restrict__ S4, double *__restrict__ out) {
  const int cb = xcd_item(blockIdx.x, gridDim.x);
  const int leaf = chunk_leaf[cb], r = blockIdx.y;
  const int j1 = leaf_start[leaf + 1];
  const int lane = threadIdx.x & 63, g = lane >> 4;
  const int t0 = chunk_start[cb] + 16 * (threadIdx.x >> 6);  // the wave's first target
  const int j = t0 + (lane & 15);
  const bool valid = j < j1, busy = t0 < j1;
  const int jj = valid ? j : t0;
  const double2 z = xs[min(jj, M - 1)], nv = nrm[min(jj, M - 1)];
  const double4 *src = S4 + (size_t)r * M;
  __shared__ double4 buf[kNearCap];
  double gx = 0.0, gy = 0.0;
  const int e0 = run_ptr[leaf], e1 = run_ptr[leaf + 1];
  int total = 0;
  for (int e = e0; e < e1; ++e) total += run[e].y - run[e].x;
  const int padded = (total + 31) & ~31;
  if (padded <= kNearCap) {  // the runs back to back, one padding at the end
    int at = 0;
    for (int e = e0; e < e1; ++e) {
      const int2 kr = run[e];
      const int n = kr.y - kr.x;
      for (int t = threadIdx.x; t < n; t += blockDim.x) buf[at + t] = src[kr.x + t];
      at += n;
    }
    for (int t = total + threadIdx.x; t < padded; t += blockDim.x)
      buf[t] = make_double4(kNearPad, kNearPad, 0.0, 0.0);
    __syncthreads();
    if (busy) near_seg<STOKES>(buf, padded, g, z, nv, gx, gy);
  } else {
    for (int e = e0; e < e1; ++e) {
      const int2 kr = run[e];
      for (int base = kr.x; base < kr.y; base += kNearCap) {
        __syncthreads();  // the previous block is no longer read
        const int n = near_stage(src + base, min(kNearCap, kr.y - base), buf, 0);
        __syncthreads();
        if (busy) near_seg<STOKES>(buf, n, g, z, nv, gx, gy);
      }
    }
  }
  gx += __shfl_xor(gx, 16, 64);
  gy += __shfl_xor(gy, 16, 64);
  gx += __shfl_xor(gx, 32, 64);
  gy += __shfl_xor(gy, 32, 64);
  if (!valid || g != 0) return;
  const int i = perm[j];
  if (STOKES) {
    out[(size_t)r * 2 * M + 2 * i] = -gx / kPi;
    out[(size_t)r * 2 * M + 2 * i + 1] = -gy / kPi;
  } else {
    out[(size_t)r * M + i] = -(nv.x * gx + nv.y * gy) / (2.0 * kPi);
  }
}

// Float32 near field of the mixed-precision applies: k_near's neighbour lists,
// chunks and summation pattern, with the staged records converted to float32 coordinates
// relative to the chunk's first target (one float64 difference, rounded once, so a target and its
// own record still give r = 0 exactly) and float32 pair terms; each lane adds its eight-record
// partial sums into float64 accumulators. Coordinates relative to a point of the leaf keep the
// float32 rounding of r at eps32 times the neighbourhood size rather than the geometry's.
constexpr float kSelfFloor32 = 1e-20f;  // |r|^2 floor (self pair): s / floor stays finite
constexpr float kNearPad32 = 1e18f;     // padding record coordinates: |r|^2 stays finite

// Stokes (STOKES): records (x, y, rho_x, rho_y) and the term (r.n)(r.rho) r/|r|^4, formed as
// (((r.rho)(r.n)) / |r|^2) / |r|^2 so that the self pair, whose r.rho is 0, gives 0 and not 0
// times an overflowed square of the floored reciprocal.
template <bool STOKES>
__device__ __forceinline__ void near_seg32(const float4 *buf, int n, int g, float2 z, float2 nv,
                                           double &gx, double &gy) {
  for (int k = 0; k < n; k += 32) {
    float4 rec[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) rec[u] = buf[k + 4 * u + g];
    float sx = 0.0f, sy = 0.0f;
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const float dx = z.x - rec[u].x, dy = z.y - rec[u].y;
      const float inv = __builtin_amdgcn_rcpf(fmaxf(fmaf(dx, dx, dy * dy), kSelfFloor32));
      float t;
      if (STOKES) {
        const float rn = fmaf(dx, nv.x, dy * nv.y);
        t = ((fmaf(dx, rec[u].z, dy * rec[u].w) * rn) * inv) * inv;
      } else {
        t = rec[u].z * inv;
      }
      sx = fmaf(dx, t, sx);
      sy = fmaf(dy, t, sy);
    }
    gx += (double)sx;
    gy += (double)sy;
  }
}

// Stages n records src[0 .. n) at buf[at ..] relative to o, then padding up to a multiple of 32
// (the fourth component: rho_y for Stokes, 0 for Laplace).
template <bool STOKES>
__device__ __forceinline__ int near_stage32(const double4 *__restrict__ src, int n, float4 *buf,
                                            int at, double2 o) {
  const int np = (n + 31) & ~31;
  for (int t = threadIdx.x; t < np; t += blockDim.x) {
    float4 v = make_float4(kNearPad32, kNearPad32, 0.0f, 0.0f);
    if (t < n) {
      const double4 r = src[t];
      v = make_float4((float)(r.x - o.x), (float)(r.y - o.y), (float)r.z,
                      STOKES ? (float)r.w : 0.0f);
    }
    buf[at + t] = v;
  }
  return np;
}

template <bool STOKES>
__global__ __launch_bounds__(256, 6) void k_near_f32(
    int M, const int *__restrict__ leaf_start, const double2 *__restrict__ xs,
    const double2 *__restrict__ nrm, const int *__restrict__ perm,
    const int *__restrict__ run_ptr, const int2 *__restrict__ run,
    const int *__restrict__ chunk_leaf, const int *__restrict__ chunk_start,
    const double4 *__restrict__ S4, double *__restrict__ out) {
  const int cb = xcd_item(blockIdx.x, gridDim.x);
  const int leaf = chunk_leaf[cb], r = blockIdx.y;
  const int j1 = leaf_start[leaf + 1];
  const int lane = threadIdx.x & 63, g = lane >> 4;
  const int t0 = chunk_start[cb] + 16 * (threadIdx.x >> 6);  // the wave's first target
  const int j = t0 + (lane & 15);
  const bool valid = j < j1, busy = t0 < j1;
  const int jj = valid ? j : t0;
  const double2 o = xs[chunk_start[cb]];  // origin of the chunk's float32 coordinates
  const double2 zd = xs[min(jj, M - 1)], nv = nrm[min(jj, M - 1)];
  const float2 z = make_float2((float)(zd.x - o.x), (float)(zd.y - o.y));
  const float2 nvf = make_float2((float)nv.x, (float)nv.y);
  const double4 *src = S4 + (size_t)r * M;
  __shared__ float4 buf[kNearCap];
  double gx = 0.0, gy = 0.0;
  const int e0 = run_ptr[leaf], e1 = run_ptr[leaf + 1];
  int total = 0;
  for (int e = e0; e < e1; ++e) total += run[e].y - run[e].x;
  if (((total + 31) & ~31) <= kNearCap) {  // the runs back to back, one padding at the end
    int at = 0;
    for (int e = e0; e < e1; ++e) {
      const int2 kr = run[e];
      const int n = kr.y - kr.x;
      for (int t = threadIdx.x; t < n; t += blockDim.x) {
        const double4 v = src[kr.x + t];
        buf[at + t] = make_float4((float)(v.x - o.x), (float)(v.y - o.y), (float)v.z,
                                  STOKES ? (float)v.w : 0.0f);
      }
      at += n;
    }
    const int padded = (total + 31) & ~31;
    for (int t = total + threadIdx.x; t < padded; t += blockDim.x)
      buf[t] = make_float4(kNearPad32, kNearPad32, 0.0f, 0.0f);
    __syncthreads();
    if (busy) near_seg32<STOKES>(buf, padded, g, z, nvf, gx, gy);
  } else {
    for (int e = e0; e < e1; ++e) {
      const int2 kr = run[e];
      for (int base = kr.x; base < kr.y; base += kNearCap) {
        __syncthreads();  // the previous block is no longer read
        const int n = near_stage32<STOKES>(src + base, min(kNearCap, kr.y - base), buf, 0, o);
        __syncthreads();
        if (busy) near_seg32<STOKES>(buf, n, g, z, nvf, gx, gy);
      }
    }
  }
  gx += __shfl_xor(gx, 16, 64);
  gy += __shfl_xor(gy, 16, 64);
  gx += __shfl_xor(gx, 32, 64);
  gy += __shfl_xor(gy, 32, 64);
  if (!valid || g != 0) return;
  const int i = perm[j];
  if (STOKES) {
    out[(size_t)r * 2 * M + 2 * i] = -gx / kPi;
    out[(size_t)r * 2 * M + 2 * i + 1] = -gy / kPi;
  } else {
    out[(size_t)r * M + i] = -(nv.x * gx + nv.y * gy) / (2.0 * kPi);
  }
}

// Downward pass and evaluation in one: the local expansion of a leaf is the sum over its
// ancestors A (levels 2 to L, the leaf included) of A's M2L part re-expanded about the leaf, and
// re-expanding a polynomial about another centre is exact (L2L has no truncation). So each target
// evaluates the M2L part of every ancestor directly at its own scaled coordinate
// w_A = (z - c_A)/h_A and sums the values (levels in decreasing order), which replaces the
// level-by-level L2L passes. One wave per evaluation chunk: up to 64 consecutive sorted targets of
// at most kEvalLeaves consecutive leaves, so that nearly every lane has a target. At each level
// the ancestors of consecutive leaves are consecutive boxes (boxes of a level are numbered in
// Morton order and none is empty), so the chunk's ancestors at level index i (0 = leaf level)
// are the boxes lo_i .. hi_i. The wave first copies their coefficients into LDS with coalesced
// vector loads (one wait), at slots off_i .. off_i + hi_i - lo_i (levels in order), and the Horner
// steps then read them by LDS broadcast (one address per leaf of the chunk).
constexpr int kEvalLeaves = 4;

// Copies the ancestor coefficients of a chunk whose first and last leaves have the ancestor lists
// a0 and a1 ([nlev] each): per set k < nsets_here (from set0),
// cf[(k * nslot + off_i + b) * P + n] = Lexp[set0 + k][lo_i + b][n]. With DERIV_LAST the last set
// is staged as the coefficients of its derivative in w, (n + 1) Lexp[..][n + 1] (0 for n = P - 1).
template <int P, class T, bool DERIV_LAST = false>
__device__ __forceinline__ void stage_levels(const int *a0, const int *a1, int nlev, int nbox,
                                             int set0, int nsets_here, int nslot,
                                             const cx<T> *__restrict__ Lexp, cx<T> *cf) {
  int off = 0;
  for (int i = 0; i < nlev; ++i) {
    const int lo = a0[i], cnt = a1[i] - lo + 1;
    for (int k = 0; k < nsets_here; ++k) {
      const cx<T> *src = Lexp + ((size_t)(set0 + k) * nbox + lo) * P;
      cx<T> *dst = cf + ((size_t)k * nslot + off) * P;
      if (DERIV_LAST && k == nsets_here - 1) {
        for (int e = threadIdx.x; e < cnt * P; e += 64) {
          const int n = e % P;
          const T f = (T)(n + 1);
          dst[e] = n < P - 1 ? mkc<T>(f * src[e + 1].x, f * src[e + 1].y) : mkc<T>(0, 0);
        }
      } else {
        for (int e = threadIdx.x; e < cnt * P; e += 64) dst[e] = src[e];
      }
    }
    off += cnt;
  }
  __syncthreads();
}

// The chunk's leaves: first lf0, last lf1 (the leaf of its last target), and the number of
// ancestor slots.
__device__ __forceinline__ int chunk_leaves(const int *__restrict__ leaf_start,
                                            const int *__restrict__ leaf_anc, int nlev, int lf0,
                                            int j1, int &lf1) {
  lf1 = lf0;
  while (leaf_start[lf1 + 1] < j1) ++lf1;
  const int *a0 = leaf_anc + (size_t)lf0 * nlev, *a1 = leaf_anc + (size_t)lf1 * nlev;
  int nslot = 0;
  for (int i = 0; i < nlev; ++i) nslot += a1[i] - a0[i] + 1;
  return nslot;
}

// The apply's last terms, added by the Laplace evaluation when out is set (see FmmFinish):
// out = alpha (1/2 mu - s kappa / (4 pi) [+ charge of the node's body] + near + far), in the
// order of the separate epilogue, so that both give the same bits.
struct L2pFinish {
  const double *mu, *s64, *kappa, *charge;  // charge [R][N]: sum of s over each body
  const int *body_of;
  double *out;
  double alpha;
  int N, with_L;
};

// Per body b and rhs r: charge[r][b] = sum of s over the body's nodes (the epilogue's order).
__global__ __launch_bounds__(256) void k_body_sums(int M, int N, const int *__restrict__ body_ptr,
                                                   const double *__restrict__ s64,
                                                   double *__restrict__ charge) {
  __shared__ double sh[4];
  const int b = blockIdx.x, r = blockIdx.y;
  const int k0 = body_ptr[b], k1 = body_ptr[b + 1];
  const double *sr = s64 + (size_t)r * M;
  double part = 0.0;
  for (int k = k0 + threadIdx.x; k < k1; k += 256) part += sr[k];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) part += __shfl_down(part, off, 64);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) sh[wid] = part;
  __syncthreads();
  if (threadIdx.x == 0) charge[(size_t)r * N + b] = (sh[0] + sh[1]) + (sh[2] + sh[3]);
}

// Both evaluation kernels take their chunks in XCD-contiguous order (xcd_item): sibling leaves,
// which stage the same ancestors, then share one XCD's L2.
// L2P, Laplace: adds -(1/2pi) Re(nu F(z)) to the near-field sums in out, or (fin.out set) writes
// the finished apply. Grid (evaluation chunks, R); dynamic LDS: ev_maxslot P coefficients.
template <int P, class T>
__global__ __launch_bounds__(64) void k_l2p_laplace(
    int M, int nbox, int L, double ih_leaf, const int *__restrict__ leaf_start,
    const int *__restrict__ leaf_anc, const double2 *__restrict__ center,
    const double2 *__restrict__ xs, const double2 *__restrict__ nrm, const int *__restrict__ perm,
    const int *__restrict__ ev_start, const int *__restrict__ ev_leaf,
    const cx<T> *__restrict__ Lexp, double *__restrict__ out, const L2pFinish fin) {
  __builtin_amdgcn_s_setprio(kChainPrio);
  extern __shared__ char l2p_lds[];
  cx<T> *cf = reinterpret_cast<cx<T> *>(l2p_lds);
  const int c = xcd_item(blockIdx.x, gridDim.x), r = blockIdx.y;
  const int j0 = ev_start[c], j1 = ev_start[c + 1], lf0 = ev_leaf[c];
  const int nlev = L - 1;  // ancestor lists: levels L, L - 1, ..., 2
  int lf1;
  const int nslot = chunk_leaves(leaf_start, leaf_anc, nlev, lf0, j1, lf1);
  const int *a0 = leaf_anc + (size_t)lf0 * nlev, *a1 = leaf_anc + (size_t)lf1 * nlev;
  stage_levels<P, T>(a0, a1, nlev, nbox, r, 1, nslot, Lexp, cf);
  const int j = j0 + threadIdx.x;
  if (j >= j1) return;
  int lf = lf0;
  while (leaf_start[lf + 1] <= j) ++lf;
  const int *anc = leaf_anc + (size_t)lf * nlev;
  const double2 z = xs[j], nv = nrm[j];
  cx<T> F = mkc<T>(0, 0);
  double ih = ih_leaf;
  for (int i = 0, off = 0; i < nlev; ++i) {
    const int b = anc[i];
    const double2 cc = center[b];
    const cx<T> Fl = eval_value<P>(cf + (size_t)(off + b - a0[i]) * P,
                                   mkc<T>((T)((z.x - cc.x) * ih), (T)((z.y - cc.y) * ih)));
    F = mkc<T>(F.x + Fl.x, F.y + Fl.y);
    off += a1[i] - a0[i] + 1;
    ih *= 0.5;
  }
  const int i = perm[j];
  const size_t ri = (size_t)r * M + i;
  const double part = out[ri] - (nv.x * (double)F.x - nv.y * (double)F.y) / (2.0 * kPi);  // Re(nu F)
  if (fin.out) {
    double v = 0.5 * fin.mu[ri] - fin.s64[ri] * fin.kappa[i] / (4.0 * kPi);
    if (fin.with_L) v += fin.charge[(size_t)r * fin.N + fin.body_of[i]];
    v += part;
    fin.out[ri] = fin.alpha * v;
  } else {
    out[ri] = part;
  }
}

// L2P, Stokes: sets 3r, 3r+1, 3r+2 are the expansions of A, B, C; adds -(1/pi) of
// (1/4)[conj(nu) conj(C' - conj(z) A') + conj(nu) conj(B) + nu (conj(A) + A)].
template <int P>
__global__ __launch_bounds__(64) void k_l2p_stokes(
    int M, int nbox, int L, double ih_leaf, const int *__restrict__ leaf_start,
    const int *__restrict__ leaf_anc, const double2 *__restrict__ center,
    const double2 *__restrict__ xs, const double2 *__restrict__ nrm, const int *__restrict__ perm,
    const int *__restrict__ ev_start, const int *__restrict__ ev_leaf,
    const double2 *__restrict__ Lexp, double *__restrict__ out) {
  __builtin_amdgcn_s_setprio(kChainPrio);
  extern __shared__ char l2p_lds[];
  double2 *cf = reinterpret_cast<double2 *>(l2p_lds);  // sets A, B, C of every staged ancestor
  const int c = xcd_item(blockIdx.x, gridDim.x), r = blockIdx.y;
  const int j0 = ev_start[c], j1 = ev_start[c + 1], lf0 = ev_leaf[c];
  const int nlev = L - 1;
  int lf1;
  const int nslot = chunk_leaves(leaf_start, leaf_anc, nlev, lf0, j1, lf1);
  const int *a0 = leaf_anc + (size_t)lf0 * nlev, *a1 = leaf_anc + (size_t)lf1 * nlev;
  stage_levels<P, double, true>(a0, a1, nlev, nbox, 3 * r, 3, nslot, Lexp, cf);
  const int j = j0 + threadIdx.x;
  if (j >= j1) return;
  int lf = lf0;
  while (leaf_start[lf + 1] <= j) ++lf;
  const int *anc = leaf_anc + (size_t)lf * nlev;
  const double2 z = xs[j], nv = nrm[j];
  double2 A = make_double2(0.0, 0.0), dA = A, B = A, dC = A;
  double ih = ih_leaf;
  for (int i = 0, off = 0; i < nlev; ++i) {  // ancestors, as in the Laplace evaluation
    const int b = anc[i];
    const double2 cc = center[b];
    const double2 w = make_double2((z.x - cc.x) * ih, (z.y - cc.y) * ih);
    const size_t sl = (size_t)(off + b - a0[i]);
    off += a1[i] - a0[i] + 1;
    double2 Al, dAl;
    eval_local<P>(cf + (0 * (size_t)nslot + sl) * P, w, ih, Al, dAl);
    const double2 Bl = eval_value<P>(cf + (1 * (size_t)nslot + sl) * P, w);
    // C enters through its derivative only: staged as derivative coefficients (P - 1 terms)
    const double2 dCw = eval_value<P - 1>(cf + (2 * (size_t)nslot + sl) * P, w);
    const double2 dCl = make_double2(dCw.x * ih, dCw.y * ih);
    A = make_double2(A.x + Al.x, A.y + Al.y);
    dA = make_double2(dA.x + dAl.x, dA.y + dAl.y);
    B = make_double2(B.x + Bl.x, B.y + Bl.y);
    dC = make_double2(dC.x + dCl.x, dC.y + dCl.y);
    ih *= 0.5;
  }
  const double2 zA = cmul(make_double2(z.x, -z.y), dA);
  const double2 u = make_double2(dC.x - zA.x, -(dC.y - zA.y));  // conj(C' - conj(z) A')
  const double2 nc = make_double2(nv.x, -nv.y);
  const double2 t1 = cmul(nc, u);
  const double2 t2 = cmul(nc, make_double2(B.x, -B.y));
  const double2 t3 = cmul(nv, make_double2(2.0 * A.x, 0.0));  // conj(A) + A = 2 Re A
  const double fx = 0.25 * (t1.x + t2.x + t3.x), fy = 0.25 * (t1.y + t2.y + t3.y);
  const int i = perm[j];
  out[(size_t)r * 2 * M + 2 * i] -= fx / kPi;
  out[(size_t)r * 2 * M + 2 * i + 1] -= fy / kPi;
}

// ---- evaluation at arbitrary points (read-off, off-surface field) ----------------------------
// The single-layer potentials at points z off the curves, by a treecode over this tree: the
// multipoles of the boxes in the point's list (P2M and M2M of the density's strengths, as in
// the apply) evaluated at z, plus the nodes of the remaining leaves directly.
//   Laplace: sum_k q_k log(z - zeta_k) = a_0 log(z - c) - sum_{m>=1} a_m (h / (z - c))^m / m,
//   a_m = sum_k q_k ((zeta_k - c)/h)^m = u_m m! / s^m (stored u_m), so the m-th term is
//   u_m T_log[m] t^m with t = h / (z - c), T_log[m] = (m - 1)! / s^m; the potential needs its
//   real part (log|z - zeta|).
//   Stokes (traction strengths t_k = w_k (dens_1 + i dens_2)_k as complex numbers f):
//   sum_k G(z - zeta_k) f_k = (1/4pi) [ -sum f ln|r| + F/2 + (1/2) (z conj(A) - conj(C)) ],
//   with r = z - zeta, F = sum f, A(z) = sum f / (z - zeta), C(z) = sum f conj(zeta) / (z - zeta)
//   (the charge sets A and C of the apply), and sum f ln|r| = (L_A + conj(L_B)) / 2 with the log
//   sums L of the sets A (f) and B (conj f); half the vorticity is -(1/4pi) Im A(z).
//   Cauchy multipole: A(z) = (1/(z - c)) sum_m u_m (m! / s^m) t^m (T_c).

// Charges in sorted order only: Laplace set r = (w dens, 0); Stokes sets 3r, 3r + 1, 3r + 2 =
// f, conj f, f conj(z) with f = w (dens_1 + i dens_2).
__global__ void k_gather_q(int M, int R, int kind, const int *__restrict__ perm,
                           const double2 *__restrict__ xs, const double *__restrict__ wq,
                           const double *__restrict__ dens, double2 *__restrict__ Q) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= M) return;
  const int k = perm[j];
  const double wk = wq[k];
  for (int r = 0; r < R; ++r) {
    if (kind == 0) {
      Q[(size_t)r * M + j] = make_double2(wk * dens[(size_t)r * M + k], 0.0);
    } else {
      const double2 z = xs[j];
      const double2 f = make_double2(wk * dens[(size_t)r * 2 * M + 2 * k],
                                     wk * dens[(size_t)r * 2 * M + 2 * k + 1]);
      Q[(size_t)(3 * r) * M + j] = f;
      Q[(size_t)(3 * r + 1) * M + j] = make_double2(f.x, -f.y);
      Q[(size_t)(3 * r + 2) * M + j] = cmul(f, make_double2(z.x, -z.y));
    }
  }
}

__device__ __forceinline__ double2 cdiv1(double2 z) {  // 1 / z
  const double d = 1.0 / fma(z.x, z.x, z.y * z.y);
  return make_double2(z.x * d, -z.y * d);
}

// Wave sum in a fixed order (the same tree for every call).
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Laplace: phi(z) = -(1/2pi) sum_k q_k log|z - zeta_k|. Grid (points, R), one wave each.
template <int P>
__global__ __launch_bounds__(64) void k_eval_lap(
    int M, int nbox, double size, const double2 *__restrict__ pts, double ox, double oy,
    const int *__restrict__ box_ptr, const int2 *__restrict__ boxes,
    const int *__restrict__ run_ptr, const int2 *__restrict__ runs,
    const double2 *__restrict__ center, const double *__restrict__ T_log,
    const double2 *__restrict__ xs, const double2 *__restrict__ Q,
    const double2 *__restrict__ Mexp, int npts, double *__restrict__ out) {
  const int p = blockIdx.x, r = blockIdx.y, lane = threadIdx.x;
  const double2 z = make_double2(pts[p].x - ox, pts[p].y - oy);
  double acc = 0.0;
  for (int e = box_ptr[p] + lane; e < box_ptr[p + 1]; e += 64) {
    const int2 bl = boxes[e];
    const double h = size / (double)(1 << bl.y);
    const double2 c = center[bl.x];
    const double2 dz = make_double2(z.x - c.x, z.y - c.y);
    const double2 id = cdiv1(dz);
    const double2 t = make_double2(h * id.x, h * id.y);
    const double2 *u = Mexp + ((size_t)r * nbox + bl.x) * P;
    double2 S = make_double2(u[P - 1].x * T_log[P - 1], u[P - 1].y * T_log[P - 1]);
#pragma unroll
    for (int m = P - 2; m >= 1; --m)
      S = cfma(S, t, make_double2(u[m].x * T_log[m], u[m].y * T_log[m]));
    S = cmul(S, t);  // sum_{m>=1} u_m T_log[m] t^m
    acc += u[0].x * 0.5 * log(fma(dz.x, dz.x, dz.y * dz.y)) - S.x;
  }
  const double2 *q = Q + (size_t)r * M;
  for (int e = run_ptr[p]; e < run_ptr[p + 1]; ++e) {
    const int2 kr = runs[e];
    for (int k = kr.x + lane; k < kr.y; k += 64) {
      const double2 zk = xs[k];
      const double dx = z.x - zk.x, dy = z.y - zk.y;
      acc = fma(q[k].x, 0.5 * log(fma(dx, dx, dy * dy)), acc);
    }
  }
  acc = wave_sum(acc);
  if (lane == 0) out[(size_t)r * npts + p] = -acc / (2.0 * kPi);
}

// Stokes: u(z) (viscosity 1) and half the vorticity; with rigid, v = u - omega (p - x^c)^perp
// and omega for body p (out [R][npts][3]), else the velocity (out [R][npts][2]).
template <int P>
__global__ __launch_bounds__(64) void k_eval_stk(
    int M, int nbox, double size, const double2 *__restrict__ pts, double ox, double oy,
    const int *__restrict__ box_ptr, const int2 *__restrict__ boxes,
    const int *__restrict__ run_ptr, const int2 *__restrict__ runs,
    const double2 *__restrict__ center, const double *__restrict__ T_log,
    const double *__restrict__ T_c, const double2 *__restrict__ xs,
    const double2 *__restrict__ Q, const double2 *__restrict__ Mexp, int npts, int rigid,
    const double *__restrict__ xc, const double *__restrict__ yc, double *__restrict__ out) {
  const int p = blockIdx.x, r = blockIdx.y, lane = threadIdx.x;
  const double2 z = make_double2(pts[p].x - ox, pts[p].y - oy);
  double u1 = 0.0, u2 = 0.0, om = 0.0;  // raw sums: u = (1/4pi) (u1, u2), omega = -(1/4pi) om
  for (int e = box_ptr[p] + lane; e < box_ptr[p + 1]; e += 64) {
    const int2 bl = boxes[e];
    const double h = size / (double)(1 << bl.y);
    const double2 c = center[bl.x];
    const double2 dz = make_double2(z.x - c.x, z.y - c.y);
    const double2 id = cdiv1(dz);
    const double2 t = make_double2(h * id.x, h * id.y);
    const double2 *uA = Mexp + ((size_t)(3 * r) * nbox + bl.x) * P;
    const double2 *uB = Mexp + ((size_t)(3 * r + 1) * nbox + bl.x) * P;
    const double2 *uC = Mexp + ((size_t)(3 * r + 2) * nbox + bl.x) * P;
    double2 SA = make_double2(uA[P - 1].x * T_log[P - 1], uA[P - 1].y * T_log[P - 1]);
    double2 SB = make_double2(uB[P - 1].x * T_log[P - 1], uB[P - 1].y * T_log[P - 1]);
    double2 FA = make_double2(uA[P - 1].x * T_c[P - 1], uA[P - 1].y * T_c[P - 1]);
    double2 FC = make_double2(uC[P - 1].x * T_c[P - 1], uC[P - 1].y * T_c[P - 1]);
#pragma unroll
    for (int m = P - 2; m >= 0; --m) {
      if (m >= 1) {
        SA = cfma(SA, t, make_double2(uA[m].x * T_log[m], uA[m].y * T_log[m]));
        SB = cfma(SB, t, make_double2(uB[m].x * T_log[m], uB[m].y * T_log[m]));
      }
      FA = cfma(FA, t, make_double2(uA[m].x * T_c[m], uA[m].y * T_c[m]));
      FC = cfma(FC, t, make_double2(uC[m].x * T_c[m], uC[m].y * T_c[m]));
    }
    SA = cmul(SA, t);
    SB = cmul(SB, t);
    const double2 A = cmul(FA, id), C = cmul(FC, id);
    const double lnr = 0.5 * log(fma(dz.x, dz.x, dz.y * dz.y));
    // -F ln|dz| + (S_A + conj(S_B)) / 2 + F / 2 + (z conj(A) - conj(C)) / 2, F = a_0 of set A
    const double2 zA = cmul(z, make_double2(A.x, -A.y));
    u1 += -uA[0].x * lnr + 0.5 * (SA.x + SB.x) + 0.5 * uA[0].x + 0.5 * (zA.x - C.x);
    u2 += -uA[0].y * lnr + 0.5 * (SA.y - SB.y) + 0.5 * uA[0].y + 0.5 * (zA.y + C.y);
    om += A.y;
  }
  const double2 *f = Q + (size_t)(3 * r) * M;
  for (int e = run_ptr[p]; e < run_ptr[p + 1]; ++e) {
    const int2 kr = runs[e];
    for (int k = kr.x + lane; k < kr.y; k += 64) {
      const double2 zk = xs[k], fk = f[k];
      const double dx = z.x - zk.x, dy = z.y - zk.y;
      const double rr = fma(dx, dx, dy * dy);
      const double lg = 0.5 * log(rr), inv = 1.0 / rr;
      const double rt = fma(dx, fk.x, dy * fk.y) * inv;
      u1 += -lg * fk.x + dx * rt;
      u2 += -lg * fk.y + dy * rt;
      om += (dx * fk.y - dy * fk.x) * inv;
    }
  }
  u1 = wave_sum(u1);
  u2 = wave_sum(u2);
  om = wave_sum(om);
  if (lane != 0) return;
  const double U1 = u1 / (4.0 * kPi), U2 = u2 / (4.0 * kPi), OM = -om / (4.0 * kPi);
  if (rigid) {  // v = u(p) - omega (p - x^c)^perp, a^perp = (-a2, a1)
    const double e1 = pts[p].x - xc[p], e2 = pts[p].y - yc[p];
    double *o = out + ((size_t)r * npts + p) * 3;
    o[0] = U1 + OM * e2;
    o[1] = U2 - OM * e1;
    o[2] = OM;
  } else {
    double *o = out + ((size_t)r * npts + p) * 2;
    o[0] = U1;
    o[1] = U2;
  }
}

// ---- host: tree and translation operators ---------------------------------------------------

double binom(int n, int k) {
  double r = 1.0;
  for (int i = 1; i <= k; ++i) r = r * (n - k + i) / i;
  return r;
}

int build_tree(bie_geom *g, int p, int leaf_cap, FmmTree &t, hipStream_t s) {
  const int M = g->M;
  std::vector<double> x(M), y(M), nx(M), ny(M);
  BIE_HIP_CHECK(hipMemcpyAsync(x.data(), g->x, M * 8, hipMemcpyDeviceToHost, s));
  BIE_HIP_CHECK(hipMemcpyAsync(y.data(), g->y, M * 8, hipMemcpyDeviceToHost, s));
  BIE_HIP_CHECK(hipMemcpyAsync(nx.data(), g->nx, M * 8, hipMemcpyDeviceToHost, s));
  BIE_HIP_CHECK(hipMemcpyAsync(ny.data(), g->ny, M * 8, hipMemcpyDeviceToHost, s));
  BIE_HIP_CHECK(hipStreamSynchronize(s));
  double x0 = x[0], x1 = x[0], y0 = y[0], y1 = y[0];
  for (int k = 0; k < M; ++k) {
    x0 = std::min(x0, x[k]); x1 = std::max(x1, x[k]);
    y0 = std::min(y0, y[k]); y1 = std::max(y1, y[k]);
  }
  t.p = p;
  t.M = M;
  t.size = std::max(x1 - x0, y1 - y0) * (1.0 + 1e-9) + 1e-300;
  t.ox = 0.5 * (x0 + x1);
  t.oy = 0.5 * (y0 + y1);
  // cells at the finest level (14) and their Morton keys (x bits even, y bits odd); one sort
  // makes every box of every level a contiguous run of nodes
  constexpr int kTop = 14;
  const int nTop = 1 << kTop;
  auto cell = [&](double v, double o) {
    long long i = (long long)std::floor((v - o + 0.5 * t.size) / t.size * nTop);
    return (unsigned)std::min<long long>(std::max<long long>(i, 0), nTop - 1);
  };
  auto spread = [](unsigned v) {
    v &= 0xffff;
    v = (v | (v << 8)) & 0x00ff00ff;
    v = (v | (v << 4)) & 0x0f0f0f0f;
    v = (v | (v << 2)) & 0x33333333;
    v = (v | (v << 1)) & 0x55555555;
    return v;
  };
  std::vector<unsigned long long> kv(M);  // (morton << 32) | index
  for (int k = 0; k < M; ++k) {
    const unsigned mk = spread(cell(x[k], t.ox)) | (spread(cell(y[k], t.oy)) << 1);
    kv[k] = ((unsigned long long)mk << 32) | (unsigned)k;
  }
  std::sort(kv.begin(), kv.end());
  std::vector<int> perm(M);
  std::vector<unsigned> mort(M);
  for (int j = 0; j < M; ++j) {
    perm[j] = (int)(kv[j] & 0xffffffffu);
    mort[j] = (unsigned)(kv[j] >> 32);
  }
  // depth: mean population of non-empty leaves closest (in log) to leaf_cap; at least 2 levels
  int L = 2;
  double best = 1e300;
  for (int l = 2; l <= 12; ++l) {
    const int sh = 2 * (kTop - l);
    long long runs = 1;
    for (int j = 1; j < M; ++j) runs += (mort[j] >> sh) != (mort[j - 1] >> sh);
    const double mean = (double)M / (double)runs;
    const double d = std::fabs(std::log(mean / (double)leaf_cap));
    if (d < best) {
      best = d;
      L = l;
    }
    if (mean < 0.5 * leaf_cap) break;
  }
  t.L = L;
  const int nL = 1 << L;
  auto decode = [](unsigned v) {  // compact even bits
    v &= 0x55555555;
    v = (v | (v >> 1)) & 0x33333333;
    v = (v | (v >> 2)) & 0x0f0f0f0f;
    v = (v | (v >> 4)) & 0x00ff00ff;
    v = (v | (v >> 8)) & 0x0000ffff;
    return v;
  };
  // boxes per level: sorted unique Morton keys (at level l a key has 2l bits)
  std::vector<std::vector<long long>> keys(L + 1);
  std::vector<int> leaf_start;
  const int shL = 2 * (kTop - L);
  for (int j = 0; j < M; ++j) {
    const long long kk = mort[j] >> shL;
    if (keys[L].empty() || keys[L].back() != kk) {
      keys[L].push_back(kk);
      leaf_start.push_back(j);
    }
  }
  leaf_start.push_back(M);
  for (int l = L - 1; l >= 0; --l)
    for (long long kk : keys[l + 1])
      if (keys[l].empty() || keys[l].back() != (kk >> 2)) keys[l].push_back(kk >> 2);
  t.level_off.assign(L + 2, 0);
  for (int l = 0; l <= L; ++l) t.level_off[l + 1] = t.level_off[l] + (int)keys[l].size();
  t.nbox = t.level_off[L + 1];
  t.nleaf = (int)keys[L].size();
  auto enc = [&](int ix, int iy) { return (long long)(spread((unsigned)ix) | (spread((unsigned)iy) << 1)); };
  auto find = [&](int l, long long kk) -> int {
    auto it = std::lower_bound(keys[l].begin(), keys[l].end(), kk);
    if (it == keys[l].end() || *it != kk) return -1;
    return t.level_off[l] + (int)(it - keys[l].begin());
  };
  std::vector<double2> center(t.nbox);
  std::vector<int> child(4 * t.nbox, -1), parent(t.nbox, -1), box_level(t.nbox);
  for (int l = 0; l <= L; ++l) {
    const int n = 1 << l;
    const double h = t.size / n;
    for (size_t b = 0; b < keys[l].size(); ++b) {
      const long long kk = keys[l][b];
      const long long ix = decode((unsigned)kk), iy = decode((unsigned)(kk >> 1));
      const int gb = t.level_off[l] + (int)b;
      box_level[gb] = l;
      center[gb] = make_double2(-0.5 * t.size + (ix + 0.5) * h, -0.5 * t.size + (iy + 0.5) * h);
      if (l > 0) {
        const int pb = find(l - 1, kk >> 2);
        const int cpos = (int)((iy & 1) * 2 + (ix & 1));
        child[4 * pb + cpos] = gb;
        parent[gb] = pb * 4 + cpos;
      }
    }
    (void)n;
  }
  // host copies for the evaluation at arbitrary points: box levels, centres, children, and the
  // run of sorted nodes of every box (leaves first, then each parent spans its children)
  t.h_level = box_level;
  t.h_center = center;
  t.h_child = child;
  t.h_lo.assign(t.nbox, M);
  t.h_hi.assign(t.nbox, 0);
  for (int b = 0; b < (int)keys[L].size(); ++b) {
    t.h_lo[t.level_off[L] + b] = leaf_start[b];
    t.h_hi[t.level_off[L] + b] = leaf_start[b + 1];
  }
  for (int l = L - 1; l >= 0; --l)
    for (int b = t.level_off[l]; b < t.level_off[l + 1]; ++b)
      for (int c = 0; c < 4; ++c)
        if (child[4 * b + c] >= 0) {
          t.h_lo[b] = std::min(t.h_lo[b], t.h_lo[child[4 * b + c]]);
          t.h_hi[b] = std::max(t.h_hi[b], t.h_hi[child[4 * b + c]]);
        }
  // M2L lists (levels >= 2) and near lists (leaves)
  std::vector<int> m2l_ptr(1, 0), m2l_src, m2l_off;
  const int off2 = t.level_off[std::min(2, L)];
  for (int l = 2; l <= L; ++l) {
    const int n = 1 << l;
    for (long long kk : keys[l]) {
      const int ix = (int)decode((unsigned)kk), iy = (int)decode((unsigned)(kk >> 1));
      const int py = iy >> 1, px = ix >> 1, np = n >> 1;
      for (int dy = -1; dy <= 1; ++dy)
        for (int dx = -1; dx <= 1; ++dx) {
          const int qy = py + dy, qx = px + dx;
          if (qy < 0 || qx < 0 || qy >= np || qx >= np) continue;
          for (int cy = 0; cy < 2; ++cy)
            for (int cx = 0; cx < 2; ++cx) {
              const int sy = 2 * qy + cy, sx = 2 * qx + cx;
              if (std::max(std::abs(sx - ix), std::abs(sy - iy)) < 2) continue;
              const int sb = find(l, enc(sx, sy));
              if (sb < 0) continue;
              m2l_src.push_back(sb);
              m2l_off.push_back((ix - sx + 3) * 7 + (iy - sy + 3));
            }
        }
      m2l_ptr.push_back((int)m2l_src.size());
    }
  }
  t.m2l_entries = (long long)m2l_src.size();
  std::vector<int> near_ptr(1, 0), near_leaf, leaf_box(t.nleaf), leaf_anc((size_t)t.nleaf * (L - 1));
  std::vector<int> chunk_leaf, chunk_start;
  for (int b = 0; b < t.nleaf; ++b) {
    const long long kk = keys[L][b];
    const int ix = (int)decode((unsigned)kk), iy = (int)decode((unsigned)(kk >> 1));
    leaf_box[b] = t.level_off[L] + b;
    for (int i = 0, a = leaf_box[b]; i < L - 1; ++i, a = parent[a] >> 2) leaf_anc[(size_t)b * (L - 1) + i] = a;
    for (int j = leaf_start[b]; j < leaf_start[b + 1]; j += 64) {
      chunk_leaf.push_back(b);
      chunk_start.push_back(j);
    }
    for (int dy = -1; dy <= 1; ++dy)
      for (int dx = -1; dx <= 1; ++dx) {
        const int qy = iy + dy, qx = ix + dx;
        if (qy < 0 || qx < 0 || qy >= nL || qx >= nL) continue;
        const int nb = find(L, enc(qx, qy));
        if (nb >= 0) {
          near_leaf.push_back(nb - t.level_off[L]);
          const int nl = nb - t.level_off[L];
          t.near_pairs += (long long)(leaf_start[b + 1] - leaf_start[b]) *
                          (leaf_start[nl + 1] - leaf_start[nl]);
        }
      }
    near_ptr.push_back((int)near_leaf.size());
  }
  // evaluation chunks: from target j, up to 64 targets, adding whole or partial leaves while
  // the chunk spans at most kEvalLeaves leaves and `cap` ancestor slots (2 (L - 1), and at most
  // what keeps the Stokes evaluation's three sets within 64 KiB of LDS; one leaf: L - 1)
  std::vector<int> ev_start, ev_leaf;
  int ev_maxslot = 0;
  {
    const int nlev = L - 1;
    const int cap = std::min(2 * nlev, 65536 / (3 * 16 * p));
    auto slots = [&](int b0, int b1) {
      int n = 0;
      for (int i = 0; i < nlev; ++i)
        n += leaf_anc[(size_t)b1 * nlev + i] - leaf_anc[(size_t)b0 * nlev + i] + 1;
      return n;
    };
    int b = 0;
    for (int j = 0; j < M;) {
      while (leaf_start[b + 1] <= j) ++b;
      const int end = std::min(M, j + 64);
      int last = b;
      while (last + 1 < t.nleaf && leaf_start[last + 1] < end && last + 2 - b <= kEvalLeaves &&
             slots(b, last + 1) <= cap)
        ++last;
      ev_start.push_back(j);
      ev_leaf.push_back(b);
      ev_maxslot = std::max(ev_maxslot, slots(b, last));
      j = std::min(end, leaf_start[last + 1]);
    }
    ev_start.push_back(M);
  }
  // translation operators: the 40 M2L offsets (compact index) and, below, the M2L and M2M
  // tables
  std::vector<int> ocompact(49, -1);
  int nc = 0;
  for (int dx = -3; dx <= 3; ++dx)
    for (int dy = -3; dy <= 3; ++dy)
      if (std::max(std::abs(dx), std::abs(dy)) >= 2) ocompact[(dx + 3) * 7 + (dy + 3)] = nc++;
  for (auto &o : m2l_off) o = ocompact[o];
  // M2L groups (k_m2l): per level and position within the parent, up to 16 boxes; per group the
  // offsets its boxes use, in increasing order, with one source per box. A group costs one
  // item per offset any of its boxes uses, so boxes are grouped by the offsets they use: each
  // group starts from the first box not yet placed (Morton order) and adds, from the next
  // kGroupWindow boxes not yet placed, the one that enlarges the group's offset set least (ties:
  // more offsets, then the earlier box). For 1000 starfish this fills 76 % of the MFMA columns
  // instead of 64 % in plain Morton order.
  constexpr int kGroupWindow = 512;
  std::vector<int> grp_ptr(1, 0), grp_tgt, grp_lvl, item_off, item_src;
  for (int l = 2; l <= L; ++l) {
    std::vector<int> cls[4];
    for (size_t b = 0; b < keys[l].size(); ++b) {
      const long long kk = keys[l][b];
      const int ix = (int)decode((unsigned)kk), iy = (int)decode((unsigned)(kk >> 1));
      cls[(ix & 1) | ((iy & 1) << 1)].push_back(t.level_off[l] + (int)b);
    }
    for (int c = 0; c < 4; ++c) {
      const int n = (int)cls[c].size();
      std::vector<unsigned long long> mask(n, 0);
      std::vector<int> pc(n);
      for (int i = 0; i < n; ++i) {
        const int tb = cls[c][i];
        for (int e = m2l_ptr[tb - off2]; e < m2l_ptr[tb - off2 + 1]; ++e) mask[i] |= 1ull << m2l_off[e];
        pc[i] = __builtin_popcountll(mask[i]);
      }
      std::vector<char> placed(n, 0);
      std::vector<int> members;  // boxes of the groups, 16 slots per group (-1: empty)
      int first = 0;
      while (true) {
        while (first < n && placed[first]) ++first;
        if (first >= n) break;
        std::vector<int> cand;
        for (int i = first + 1; i < n && (int)cand.size() < kGroupWindow; ++i)
          if (!placed[i]) cand.push_back(i);
        placed[first] = 1;
        unsigned long long u = mask[first];
        int gcount = 1;
        members.push_back(cls[c][first]);
        while (gcount < 16 && !cand.empty()) {
          int best = -1, bu = 1 << 30, bp = -1;
          for (int k = 0; k < (int)cand.size(); ++k) {
            const int i = cand[k];
            const int cu = __builtin_popcountll(u | mask[i]);
            if (cu < bu || (cu == bu && pc[i] > bp)) {
              best = k;
              bu = cu;
              bp = pc[i];
            }
          }
          const int i = cand[best];
          cand.erase(cand.begin() + best);
          placed[i] = 1;
          u |= mask[i];
          members.push_back(cls[c][i]);
          ++gcount;
        }
        for (; gcount < 16; ++gcount) members.push_back(-1);
      }
      for (size_t g0 = 0; g0 < members.size(); g0 += 16) {
        std::vector<int> src_of(40 * 16, -1);
        std::vector<char> used(40, 0);
        for (int col = 0; col < 16; ++col) {
          const int tb = members[g0 + col];
          grp_tgt.push_back(tb);
          if (tb < 0) continue;
          for (int e = m2l_ptr[tb - off2]; e < m2l_ptr[tb - off2 + 1]; ++e) {
            src_of[m2l_off[e] * 16 + col] = m2l_src[e];
            used[m2l_off[e]] = 1;
          }
        }
        for (int o = 0; o < 40; ++o)
          if (used[o]) {
            item_off.push_back(o);
            for (int col = 0; col < 16; ++col) item_src.push_back(src_of[o * 16 + col]);
          }
        grp_lvl.push_back(l);
        grp_ptr.push_back((int)item_off.size());
      }
    }
  }
  {
    // Dispatch order. Workgroup i of the M2L launch runs on XCD i % 8, each XCD with its own L2:
    // the groups of every level are cut into eight contiguous parts of about equal work (items),
    // and XCD x takes part x of every level, so neighbouring groups, which read mostly the same
    // source multipoles, share one L2 while the work stays balanced over the XCDs. Only the order
    // of the groups changes (each group writes its own boxes' locals).
    const int G = (int)grp_lvl.size();
    auto xcd_order = [&](int ga, int gb, std::vector<int> &order) {
      std::vector<std::vector<int>> share(8);
      for (int a = ga; a < gb;) {
        int b = a;
        while (b < gb && grp_lvl[b] == grp_lvl[a]) ++b;
        const int i0 = grp_ptr[a], i1 = grp_ptr[b];  // group g's items: grp_ptr[g] .. [g + 1]
        int x = 0;
        for (int g = a; g < b; ++g) {
          const int mid = grp_ptr[g] + (grp_ptr[g + 1] - grp_ptr[g]) / 2;
          while (x < 7 && (long long)(mid - i0) * 8 >= (long long)(i1 - i0) * (x + 1)) ++x;
          share[x].push_back(g);
        }
        a = b;
      }
      std::vector<size_t> next(8, 0);
      for (int i = 0; i < gb - ga; ++i) {
        int x = i & 7;
        if (next[x] == share[x].size()) {  // this XCD's share is used up: take from the largest rest
          size_t best = 0;
          for (int y = 0; y < 8; ++y)
            if (share[y].size() - next[y] > best) best = share[y].size() - next[y], x = y;
        }
        order.push_back(share[x][next[x]++]);
      }
    };
    std::vector<int> order;
    order.reserve(G);
    xcd_order(0, G, order);
    std::vector<int> tgt2, lvl2, ptr2(1, 0), off2v, src2;
    tgt2.reserve(grp_tgt.size());
    src2.reserve(item_src.size());
    for (int g : order) {
      const int e0 = grp_ptr[g], e1 = grp_ptr[g + 1];
      tgt2.insert(tgt2.end(), grp_tgt.begin() + 16 * (size_t)g, grp_tgt.begin() + 16 * (size_t)g + 16);
      for (int e = e0; e < e1; ++e) {
        off2v.push_back(item_off[e]);
        src2.insert(src2.end(), item_src.begin() + 16 * (size_t)e, item_src.begin() + 16 * (size_t)e + 16);
      }
      lvl2.push_back(grp_lvl[g]);
      ptr2.push_back((int)off2v.size());
    }
    grp_tgt.swap(tgt2);
    grp_lvl.swap(lvl2);
    grp_ptr.swap(ptr2);
    item_off.swap(off2v);
    item_src.swap(src2);
  }
  t.ngroup = (int)grp_lvl.size();
  t.nitem = (int)item_off.size();
  // All tables carry a scale s = max(1, 2p/e): multipoles are stored as u_m = a_m s^m / m!, so
  // the M2L Hankel vectors become V_d[k] = k! / (s^k d^(k+1)), the output factor
  // (-1)^n s^n / n!, and the child-parent Toeplitz vectors tau[k] = (s d)^k / k!. The products
  // are unchanged; every table entry stays of moderate size (float32 range included).
  const double csc = std::max(1.0, 2.0 * p / 2.718281828459045);
  // float64 M2L: C[k] = k! / s^k and the powers d^-k of the 40 offsets
  const int dpn = 16 * ((p + 15) / 16) + 1;
  std::vector<double> Tc(2 * p);
  {
    double v = 1.0;
    for (int k = 0; k < 2 * p; ++k) {
      Tc[k] = v;
      v *= (double)(k + 1) / csc;
    }
  }
  std::vector<double2> Tdpow((size_t)40 * dpn);
  for (int dx = -3; dx <= 3; ++dx)
    for (int dy = -3; dy <= 3; ++dy) {
      const int o = ocompact[(dx + 3) * 7 + (dy + 3)];
      if (o < 0) continue;
      const cd dinv = 1.0 / cd(dx, dy);
      cd v = 1.0;
      for (int k = 0; k < dpn; ++k) {
        Tdpow[(size_t)o * dpn + k] = make_double2(v.real(), v.imag());
        v *= dinv;
      }
    }
  std::vector<double> fact_out(p), fact_in(p);
  {
    double f = 1.0;  // s^n / n!
    for (int n = 0; n < p; ++n) {
      if (n > 0) f *= csc / n;
      fact_in[n] = f;
      fact_out[n] = (n & 1) ? -f : f;
    }
  }
  // translation vectors: per child position, p zeros then tau[k] = (s d)^k / k!
  std::vector<double2> Ttau((size_t)8 * p, make_double2(0.0, 0.0));
  for (int cpos = 0; cpos < 4; ++cpos) {
    const cd delta(((cpos & 1) ? 0.25 : -0.25), ((cpos & 2) ? 0.25 : -0.25));
    cd v = 1.0;
    for (int k = 0; k < p; ++k) {
      Ttau[(size_t)cpos * 2 * p + p + k] = make_double2(v.real(), v.imag());
      v = v * delta * (csc / (double)(k + 1));
    }
  }
  std::vector<double> inv_h(L + 1);
  for (int l = 0; l <= L; ++l) inv_h[l] = (double)(1 << l) / t.size;
  std::vector<double> Tlog(p, 0.0);  // (m - 1)! / s^m, m >= 1
  for (int m = 1; m < p; ++m) Tlog[m] = Tc[m] / m;
  std::vector<double2> xs(M), nrm(M);
  std::vector<int> perm_i(M);
  for (int j = 0; j < M; ++j) {
    const int k = perm[j];
    xs[j] = make_double2(x[k] - t.ox, y[k] - t.oy);
    nrm[j] = make_double2(nx[k], ny[k]);
    perm_i[j] = k;
  }
  // upload (one arena)
  // near runs: the neighbour leaves of a leaf in increasing order, consecutive ones merged
  std::vector<int> run_ptr(1, 0), run_kk;
  for (int b = 0; b < t.nleaf; ++b) {
    std::vector<int> nb(near_leaf.begin() + near_ptr[b], near_leaf.begin() + near_ptr[b + 1]);
    std::sort(nb.begin(), nb.end());
    for (size_t i = 0; i < nb.size(); ++i) {
      if (i > 0 && nb[i] == nb[i - 1] + 1) {
        run_kk.back() = leaf_start[nb[i] + 1];
      } else {
        run_kk.push_back(leaf_start[nb[i]]);
        run_kk.push_back(leaf_start[nb[i] + 1]);
      }
    }
    run_ptr.push_back((int)run_kk.size() / 2);
  }
  const size_t nitem = std::max<size_t>(item_off.size(), 1), nnear = std::max<size_t>(run_kk.size(), 2);
  const size_t ints = (size_t)M + (t.nleaf + 1) + t.nleaf + 4 * (size_t)t.nbox + t.nbox +
                      grp_ptr.size() + 18 * (size_t)t.ngroup + 17 * nitem + run_ptr.size() +
                      nnear + 2 * chunk_leaf.size() + leaf_anc.size() + 2 * ev_start.size();
  const size_t d2 = 2 * (size_t)M + t.nbox + (size_t)80 * p + (size_t)8 * p * p + Tdpow.size();
  const size_t bytes = d2 * 16 + (L + 1 + 5 * p) * 8 + ints * 4 + 37 * 256;
  BIE_TRY(t.buf.reserve(bytes));
  char *q = t.buf.as<char>();
  auto take = [&](size_t nbytes) {
    char *r = q;
    q += (nbytes + 255) & ~size_t(255);
    return r;
  };
  t.xs = (double2 *)take(M * 16);
  t.nrm = (double2 *)take(M * 16);
  t.center = (double2 *)take(t.nbox * 16);
  t.T_c = (double *)take(Tc.size() * 8);
  t.T_dpow = (double2 *)take(Tdpow.size() * 16);
  t.fact_out = (double *)take(p * 8);
  t.fact_in = (double *)take(p * 8);
  t.T_tau = (double2 *)take((size_t)8 * p * 16);
  t.inv_h = (double *)take((L + 1) * 8);
  t.T_log = (double *)take(p * 8);
  t.perm = (int *)take(M * 4);
  t.leaf_start = (int *)take((t.nleaf + 1) * 4);
  t.leaf_box = (int *)take(t.nleaf * 4);
  t.leaf_anc = (int *)take(leaf_anc.size() * 4);
  t.child = (int *)take(4 * (size_t)t.nbox * 4);
  t.parent = (int *)take(t.nbox * 4);
  t.grp_ptr = (int *)take(grp_ptr.size() * 4);
  t.grp_tgt = (int *)take(std::max<size_t>(grp_tgt.size(), 1) * 4);
  t.grp_lvl = (int *)take(std::max<size_t>(grp_lvl.size(), 1) * 4);
  t.item_off = (int *)take(nitem * 4);
  t.item_src = (int *)take(nitem * 16 * 4);
  t.run_ptr = (int *)take(run_ptr.size() * 4);
  t.run = (int2 *)take(nnear * 4);
  t.nchunk = (int)chunk_leaf.size();
  t.chunk_leaf = (int *)take(chunk_leaf.size() * 4);
  t.chunk_start = (int *)take(chunk_start.size() * 4);
  t.nev = (int)ev_leaf.size();
  t.ev_maxslot = ev_maxslot;
  t.ev_start = (int *)take(ev_start.size() * 4);
  t.ev_leaf = (int *)take(ev_leaf.size() * 4);
  if ((size_t)(q - t.buf.as<char>()) > t.buf.bytes) {
    set_error("fmm: arena overflow");
    return BIE_EINVAL;
  }
  auto up = [&](void *dst, const void *src, size_t nbytes) -> int {
    if (nbytes == 0) return BIE_OK;
    BIE_HIP_CHECK(hipMemcpyAsync(dst, src, nbytes, hipMemcpyHostToDevice, s));
    return BIE_OK;
  };
  BIE_TRY(up(t.xs, xs.data(), M * 16));
  BIE_TRY(up(t.nrm, nrm.data(), M * 16));
  BIE_TRY(up(t.center, center.data(), t.nbox * 16));
  BIE_TRY(up(t.T_c, Tc.data(), Tc.size() * 8));
  BIE_TRY(up(t.T_dpow, Tdpow.data(), Tdpow.size() * 16));
  BIE_TRY(up(t.T_tau, Ttau.data(), Ttau.size() * 16));
  BIE_TRY(up(t.fact_out, fact_out.data(), p * 8));
  BIE_TRY(up(t.fact_in, fact_in.data(), p * 8));
  BIE_TRY(up(t.inv_h, inv_h.data(), (L + 1) * 8));
  BIE_TRY(up(t.T_log, Tlog.data(), p * 8));
  BIE_TRY(up(t.perm, perm_i.data(), M * 4));
  BIE_TRY(up(t.leaf_start, leaf_start.data(), leaf_start.size() * 4));
  BIE_TRY(up(t.leaf_box, leaf_box.data(), t.nleaf * 4));
  BIE_TRY(up(t.leaf_anc, leaf_anc.data(), leaf_anc.size() * 4));
  BIE_TRY(up(t.child, child.data(), child.size() * 4));
  BIE_TRY(up(t.parent, parent.data(), t.nbox * 4));
  BIE_TRY(up(t.grp_ptr, grp_ptr.data(), grp_ptr.size() * 4));
  BIE_TRY(up(t.grp_tgt, grp_tgt.data(), grp_tgt.size() * 4));
  BIE_TRY(up(t.grp_lvl, grp_lvl.data(), grp_lvl.size() * 4));
  BIE_TRY(up(t.item_off, item_off.data(), item_off.size() * 4));
  BIE_TRY(up(t.item_src, item_src.data(), item_src.size() * 4));
  BIE_TRY(up(t.run_ptr, run_ptr.data(), run_ptr.size() * 4));
  BIE_TRY(up(t.run, run_kk.data(), run_kk.size() * 4));
  BIE_TRY(up(t.chunk_leaf, chunk_leaf.data(), chunk_leaf.size() * 4));
  BIE_TRY(up(t.chunk_start, chunk_start.data(), chunk_start.size() * 4));
  BIE_TRY(up(t.ev_start, ev_start.data(), ev_start.size() * 4));
  BIE_TRY(up(t.ev_leaf, ev_leaf.data(), ev_leaf.size() * 4));
  BIE_HIP_CHECK(hipStreamSynchronize(s));  // host vectors go out of scope
  (void)off2;
  return BIE_OK;
}

// M2L for the groups [ga, gb) (in XCD-balanced dispatch order: each XCD takes a contiguous share
// of every level, so a level is not one contiguous range of groups), in float64 or, for the
// mixed Laplace apply, float32.
template <int P>
int launch_m2l(const FmmTree &t, int ga, int gb, int nsets, const double2 *Mexp, double2 *Lexp,
               hipStream_t s) {
  if (gb <= ga) return BIE_OK;
  static_assert(M2lShape<P>::LDS * sizeof(double) <= 65536, "M2L LDS exceeds 64 KiB");
  hipLaunchKernelGGL(k_m2l<P>, dim3(gb - ga, nsets), dim3(256), 0, s, ga, t.nbox, t.grp_ptr,
                     t.grp_tgt, t.grp_lvl, t.item_off, t.item_src, t.inv_h, t.fact_out, t.T_c,
                     t.T_dpow, Mexp, Lexp);
  BIE_HIP_CHECK(hipGetLastError());
  return BIE_OK;
}

template <int P>
int launch_m2l(const FmmTree &t, int ga, int gb, int nsets, const float2 *Mexp, float2 *Lexp,
               hipStream_t s) {
  if (gb <= ga) return BIE_OK;
  hipLaunchKernelGGL(k_m2l_fac_f32<P>, dim3(gb - ga, nsets), dim3(256), 0, s, ga, t.nbox,
                     t.grp_ptr, t.grp_tgt, t.grp_lvl, t.item_off, t.item_src, t.inv_h,
                     t.fact_out, t.T_c, t.T_dpow, Mexp, Lexp);
  BIE_HIP_CHECK(hipGetLastError());
  return BIE_OK;
}

// Multipoles of every box at levels >= 2: P2M at the leaves, then M2M level by level.
template <int P, class T>
void m2m_passes(const FmmTree &t, int nsets, cx<T> *Mexp, hipStream_t s) {
  for (int l = t.L - 1; l >= 2; --l) {
    const int nb = t.level_off[l + 1] - t.level_off[l];
    if (nb > 0)
      hipLaunchKernelGGL((k_m2m<P, T>), dim3((unsigned)std::min<long long>((long long)nb * nsets, 4096)),
                         dim3(256), 0, s, nb, t.level_off[l], t.nbox, nsets, t.child, t.T_tau, Mexp);
  }
}

template <int P, class T>
void p2m_pass(const FmmTree &t, int kind, int nsets, double ih_leaf, const cx<T> *Q, cx<T> *Mexp,
              hipStream_t s) {
  const int M = t.M;
  bool p2m_done = false;
  if constexpr (std::is_same<T, double>::value) {
    if (kind != 0 && nsets % 3 == 0) {  // Stokes: the three sets of a right-hand side in one wave
      hipLaunchKernelGGL((k_p2m<P, T, 3>), dim3(t.nleaf, nsets / 3), dim3(64), 0, s, M, t.nbox,
                         ih_leaf, t.leaf_start, t.leaf_box, t.center, t.xs, Q, t.fact_in, Mexp);
      p2m_done = true;
    }
  }
  if (!p2m_done)
    hipLaunchKernelGGL((k_p2m<P, T, 1>), dim3(t.nleaf, nsets), dim3(64), 0, s, M, t.nbox,
                       ih_leaf, t.leaf_start, t.leaf_box, t.center, t.xs, Q, t.fact_in, Mexp);
}

template <int P, class T>
void upward_pass(const FmmTree &t, int kind, int nsets, double ih_leaf, const cx<T> *Q,
                 cx<T> *Mexp, hipStream_t s) {
  p2m_pass<P, T>(t, kind, nsets, ih_leaf, Q, Mexp, s);
  m2m_passes<P, T>(t, nsets, Mexp, s);
}

constexpr int kNearAtF32 = 0;

template <int P, class T, class Near>
int expansion_passes(const FmmTree &t, FmmPlan &plan, int kind, int R, int nsets, double ih_leaf,
                     const cx<T> *Q, cx<T> *Mexp, cx<T> *Lexp, double *partial, hipStream_t s,
                     Near &&launch_near, const L2pFinish &fin) {
  const int M = t.M;
  // Where the near field is submitted. It waits on the GPU only for the gather (the fork event),
  // so the order below is the host's submission order: float64 expansions submit it after the
  // multipole passes, float32 ones at kNearAtF32 (0 before the P2M, 1 before the M2M passes, 2
  // after them). Either way it overlaps the latency-bound upward chain: making it wait on the
  // GPU for the whole upward pass measured 166 us per float64 apply against 150 us. A fused
  // upward pass (P2M and every M2M level in two launches, one workgroup per subtree) measured
  // slower as well: fewer, larger workgroups serialise the leaves' P2M and, at 1024 threads,
  // wait for the near field's waves to drain.
  constexpr int near_at = std::is_same<T, float>::value ? kNearAtF32 : 2;
  if (near_at == 0) BIE_TRY(launch_near());
  p2m_pass<P, T>(t, kind, nsets, ih_leaf, Q, Mexp, s);
  if (near_at == 1) BIE_TRY(launch_near());
  m2m_passes<P, T>(t, nsets, Mexp, s);
  if (near_at == 2) BIE_TRY(launch_near());
  if (t.ngroup > 0) {
    ProfScope pm(std::is_same<T, float>::value ? BIE_K_FMM_M2L_F32 : BIE_K_FMM_M2L, s,
                 t.m2l_entries * nsets);
    BIE_TRY(launch_m2l<P>(t, 0, t.ngroup, nsets, Mexp, Lexp, s));
  }
  BIE_HIP_CHECK(hipStreamWaitEvent(s, plan.join, 0));
  if (kind == 0) {
    hipLaunchKernelGGL((k_l2p_laplace<P, T>), dim3(t.nev, R), dim3(64),
                       (size_t)t.ev_maxslot * P * sizeof(cx<T>), s, M, t.nbox, t.L, ih_leaf,
                       t.leaf_start, t.leaf_anc, t.center, t.xs, t.nrm, t.perm, t.ev_start,
                       t.ev_leaf, Lexp, partial, fin);
  } else {
    if constexpr (std::is_same<T, double>::value)
      hipLaunchKernelGGL((k_l2p_stokes<P>), dim3(t.nev, R), dim3(64),
                         (size_t)3 * t.ev_maxslot * P * sizeof(double2), s, M, t.nbox, t.L,
                         ih_leaf, t.leaf_start, t.leaf_anc, t.center, t.xs, t.nrm, t.perm,
                         t.ev_start, t.ev_leaf, Lexp, partial);
  }
  BIE_HIP_CHECK(hipGetLastError());
  return BIE_OK;
}

// Calls f(std::integral_constant<int, P>) for the expansion length p (a multiple of 8).
template <class F>
int with_order(int p, F &&f) {
  switch (p) {
    case 8: return f(std::integral_constant<int, 8>{});
    case 16: return f(std::integral_constant<int, 16>{});
    case 24: return f(std::integral_constant<int, 24>{});
    case 32: return f(std::integral_constant<int, 32>{});
    case 40: return f(std::integral_constant<int, 40>{});
    case 48: return f(std::integral_constant<int, 48>{});
    case 56: return f(std::integral_constant<int, 56>{});
    case 64: return f(std::integral_constant<int, 64>{});
    default:
      set_error("fmm: internal order not a multiple of 8");
      return BIE_EINVAL;
  }
}

}  // namespace

// Expansion length the apply uses for a requested order (mixed precision: about half).
int fmm_length(int order, int precision) {
  int p = order > 0 ? order : 40;
  if (precision == BIE_MIXED) p = std::max(8, (p * 11 + 19) / 20);  // about sqrt of the accuracy
  return std::min((p + 7) / 8 * 8, kMaxP);  // expansions use a multiple of 8 terms (rounded up)
}

namespace {

// The tree of g for (order, leaf), built on first use.
int get_tree(bie_geom *g, int p, int leaf, hipStream_t s, FmmTree **out) {
  if (!g->fmm) g->fmm = new FmmPlan();
  FmmTree *&tp = g->fmm->trees[std::make_pair(p, leaf)];
  if (!tp) {
    tp = new FmmTree();
    const int rc = build_tree(g, p, leaf, *tp, s);
    if (rc != BIE_OK) {
      tp->buf.release();
      delete tp;
      tp = nullptr;
      return rc;
    }
  }
  *out = tp;
  return BIE_OK;
}

// Interaction lists of the points pts (absolute coordinates, host) on tree t: a descent from
// the level-2 boxes; a box at level l >= 2 with |z - c| >= sqrt(2) h_l (twice its half-diagonal:
// the multipole's terms fall at least as 2^-m) is evaluated by its multipole, a leaf closer
// than that contributes its nodes directly, any other box is replaced by its children.
int build_point_lists(const FmmTree &t, const std::vector<double2> &pts, PointLists &pl,
                      hipStream_t s) {
  const int n = (int)pts.size();
  std::vector<int> bptr(1, 0), rptr(1, 0);
  std::vector<int2> bx, rn;
  std::vector<int> stack;
  long long direct = 0;
  for (int i = 0; i < n; ++i) {
    const double zx = pts[i].x - t.ox, zy = pts[i].y - t.oy;
    stack.clear();
    const int l2 = std::min(2, t.L);
    for (int b = t.level_off[l2 + 1] - 1; b >= t.level_off[l2]; --b) stack.push_back(b);
    std::vector<int2> myruns;
    while (!stack.empty()) {
      const int b = stack.back();
      stack.pop_back();
      const int l = t.h_level[b];
      const double h = t.size / (double)(1 << l);
      const double dx = zx - t.h_center[b].x, dy = zy - t.h_center[b].y;
      if (l >= 2 && dx * dx + dy * dy >= 2.0 * h * h) {
        bx.push_back(make_int2(b, l));
      } else if (l == t.L) {
        myruns.push_back(make_int2(t.h_lo[b], t.h_hi[b]));
      } else {
        for (int c = 3; c >= 0; --c)
          if (t.h_child[4 * b + c] >= 0) stack.push_back(t.h_child[4 * b + c]);
      }
    }
    std::sort(myruns.begin(), myruns.end(), [](int2 a, int2 b) { return a.x < b.x; });
    for (const int2 &r : myruns) {
      direct += r.y - r.x;
      if (!rn.empty() && (int)rn.size() > rptr.back() && rn.back().y == r.x) rn.back().y = r.y;
      else rn.push_back(r);
    }
    bptr.push_back((int)bx.size());
    rptr.push_back((int)rn.size());
  }
  pl.npts = n;
  pl.nbox_total = (long long)bx.size();
  pl.direct_pairs = direct;
  const size_t bytes = (size_t)(2 * (n + 1)) * 4 + (bx.size() + rn.size()) * 8 + 4 * 256;
  BIE_TRY(pl.buf.reserve(bytes));
  char *q = pl.buf.as<char>();
  auto take = [&](size_t nb) {
    char *r = q;
    q += (nb + 255) & ~size_t(255);
    return r;
  };
  pl.box_ptr = (int *)take((n + 1) * 4);
  pl.run_ptr = (int *)take((n + 1) * 4);
  pl.box = (int2 *)take(std::max<size_t>(bx.size(), 1) * 8);
  pl.run = (int2 *)take(std::max<size_t>(rn.size(), 1) * 8);
  BIE_HIP_CHECK(hipMemcpyAsync(pl.box_ptr, bptr.data(), bptr.size() * 4, hipMemcpyHostToDevice, s));
  BIE_HIP_CHECK(hipMemcpyAsync(pl.run_ptr, rptr.data(), rptr.size() * 4, hipMemcpyHostToDevice, s));
  if (!bx.empty())
    BIE_HIP_CHECK(hipMemcpyAsync(pl.box, bx.data(), bx.size() * 8, hipMemcpyHostToDevice, s));
  if (!rn.empty())
    BIE_HIP_CHECK(hipMemcpyAsync(pl.run, rn.data(), rn.size() * 8, hipMemcpyHostToDevice, s));
  BIE_HIP_CHECK(hipStreamSynchronize(s));  // the host vectors go out of scope
  return BIE_OK;
}

}  // namespace

// Single-layer potentials of dens at npts points pts (device [npts][2]; the geometry's read-off
// points when pts == g->pint, whose lists are kept with the tree) by the treecode over the
// float64 FMM tree of the geometry's order and leaf size. Laplace: res [nrhs][npts]; Stokes:
// rigid (read-off) res [nrhs][npts][3] = (v, omega), else velocities [nrhs][npts][2].
int fmm_eval_points(bie_geom *g, int kind, int nrhs, const double *dens, int npts,
                    const double *pts, bool rigid, double *res, hipStream_t s) {
  const int p = fmm_length(g->fmm_order, BIE_FP64);
  const int leaf = g->fmm_leaf > 0 ? g->fmm_leaf : 64;
  FmmTree *tp = nullptr;
  BIE_TRY(get_tree(g, p, leaf, s, &tp));
  FmmTree &t = *tp;
  PointLists local, *pl = &local;
  const bool cached = pts == g->pint && npts == g->N;
  if (cached && t.rd) {
    pl = t.rd;
  } else {
    std::vector<double2> hp(npts);
    BIE_HIP_CHECK(hipMemcpyAsync(hp.data(), pts, (size_t)npts * 16, hipMemcpyDeviceToHost, s));
    BIE_HIP_CHECK(hipStreamSynchronize(s));
    if (cached) {
      t.rd = new PointLists();
      pl = t.rd;
    }
    const int rc = build_point_lists(t, hp, *pl, s);
    if (rc != BIE_OK) {
      if (cached) {
        t.rd->buf.release();
        delete t.rd;
        t.rd = nullptr;
      }
      return rc;
    }
  }
  const int M = t.M;
  const int Rmax = kind == 0 ? 8 : 4;
  const double ih_leaf = (double)(1 << t.L) / t.size;
  int rc = BIE_OK;
  for (int r0 = 0; r0 < nrhs && rc == BIE_OK; r0 += Rmax) {
    const int R = std::min(Rmax, nrhs - r0);
    const int nsets = kind == 0 ? R : 3 * R;
    // work: charges Q [nsets][M], multipoles [nsets][nbox][p] (float64)
    const size_t need = ((size_t)nsets * M + (size_t)nsets * t.nbox * p) * sizeof(double2) + 512;
    rc = t.work.reserve(need);
    if (rc != BIE_OK) break;
    double2 *Q = t.work.as<double2>();
    double2 *Mexp = Q + (size_t)nsets * M;
    const size_t len = (size_t)M * (kind == 0 ? 1 : 2);
    hipLaunchKernelGGL(k_gather_q, dim3((M + 255) / 256), dim3(256), 0, s, M, R, kind, t.perm,
                       t.xs, g->w, dens + (size_t)r0 * len, Q);
    const size_t w = kind == 0 ? 1 : (rigid ? 3 : 2);
    double *o = res + (size_t)r0 * npts * w;
    rc = with_order(p, [&](auto order) -> int {
      constexpr int P = decltype(order)::value;
      upward_pass<P, double>(t, kind, nsets, ih_leaf, Q, Mexp, s);
      if (kind == 0)
        hipLaunchKernelGGL(k_eval_lap<P>, dim3(npts, R), dim3(64), 0, s, M, t.nbox, t.size,
                           reinterpret_cast<const double2 *>(pts), t.ox, t.oy, pl->box_ptr, pl->box,
                           pl->run_ptr, pl->run, t.center, t.T_log, t.xs, Q, Mexp, npts, o);
      else
        hipLaunchKernelGGL(k_eval_stk<P>, dim3(npts, R), dim3(64), 0, s, M, t.nbox, t.size,
                           reinterpret_cast<const double2 *>(pts), t.ox, t.oy, pl->box_ptr, pl->box,
                           pl->run_ptr, pl->run, t.center, t.T_log, t.T_c, t.xs, Q, Mexp, npts,
                           rigid ? 1 : 0, g->xc, g->yc, o);
      BIE_HIP_CHECK(hipGetLastError());
      return BIE_OK;
    });
  }
  if (pl == &local) {
    (void)hipStreamSynchronize(s);  // the lists are freed on return
    local.buf.release();
  }
  return rc;
}


void fmm_drop_tree(bie_geom *g, int precision, int order, int leaf) {
  if (!g->fmm) return;
  auto it = g->fmm->trees.find(std::make_pair(fmm_length(order, precision), leaf));
  if (it == g->fmm->trees.end() || !it->second) return;
  (void)hipDeviceSynchronize();  // no apply may still use it
  FmmTree *t = it->second;
  if (t->rd) {
    t->rd->buf.release();
    delete t->rd;
  }
  t->buf.release();
  t->work.release();
  delete t;
  g->fmm->trees.erase(it);
}

long long fmm_state_bytes(const bie_geom *g, int kind, int precision, int order, int leaf) {
  if (leaf <= 0) leaf = 64;
  long long total = 0;
  // a mixed solve keeps both trees: the float64 residual applies and the shorter inner ones
  const int precs[2] = {BIE_FP64, BIE_MIXED};
  for (int k = 0; k < (precision == BIE_MIXED ? 2 : 1); ++k) {
    const int p = fmm_length(order, precs[k]);
    const int R = kind == 0 ? 8 : 4, nsets = kind == 0 ? R : 3 * R;
    const size_t csz = (precs[k] == BIE_MIXED && kind == 0) ? 8 : 16;
    long long nbox = 2LL * g->M / leaf + 64, tree = 0;
    if (g->fmm) {
      auto it = g->fmm->trees.find(std::make_pair(p, leaf));
      if (it != g->fmm->trees.end() && it->second) {
        nbox = it->second->nbox;
        tree = (long long)it->second->buf.bytes;
      }
    }
    if (tree == 0) tree = 96LL * g->M + 1024LL * nbox + 16LL * 8 * p * p;
    total += tree + (long long)R * g->M * 32 +
             (long long)((size_t)nsets * g->M + 2 * (size_t)nsets * nbox * p) * (long long)csz +
             (kind == 0 ? (long long)R * g->N * 8 + 64 : 0) + 512;
  }
  return total;
}

// Far field of all pairs k != i (sets: Laplace R, Stokes 3R) into partial [R][len] (nsplit 1).
int fmm_far_field(bie_geom *g, int kind, int precision, int R, const double *mu, double *s64,
                  double *partial,
                  hipStream_t s, int order, int leaf, const FmmFinish *finish) {
  const int p = fmm_length(order, precision);
  if (leaf <= 0) leaf = 64;
  FmmTree *tp = nullptr;
  BIE_TRY(get_tree(g, p, leaf, s, &tp));
  FmmTree &t = *tp;
  const int M = t.M;
  const int nsets = kind == 0 ? R : 3 * R;
  // float32 expansions for the mixed-precision Laplace apply (the near field of every mixed
  // apply is float32)
  const bool f32 = precision == BIE_MIXED && kind == 0;
  const size_t csz = f32 ? sizeof(float2) : sizeof(double2);
  // work: near-field source records S4 [R][M] (32 B), charges Q [nsets][M], multipoles and
  // locals [nsets][nbox][p]
  // (and, when the evaluation finishes the apply, the body charges [R][N])
  const bool fuse = finish && kind == 0;
  const size_t need = (size_t)R * M * 32 + ((size_t)nsets * M + 2 * (size_t)nsets * t.nbox * p) * csz +
                      (fuse ? (size_t)R * g->N * 8 + 64 : 0) + 512;
  BIE_TRY(t.work.reserve(need));
  double4 *S4 = t.work.as<double4>();
  char *wq = reinterpret_cast<char *>(S4 + (size_t)R * M);
  char *wm = wq + (size_t)nsets * M * csz;
  char *wl = wm + (size_t)nsets * t.nbox * p * csz;
  double *charge = reinterpret_cast<double *>(
      (reinterpret_cast<uintptr_t>(wl + (size_t)nsets * t.nbox * p * csz) + 63) & ~uintptr_t(63));
  L2pFinish fin{};
  if (fuse)
    fin = L2pFinish{finish->mu, s64, g->kappa, charge, g->body_of, finish->out, finish->alpha,
                    g->N, finish->with_L};
  FmmPlan &plan = *g->fmm;
  if (!plan.side) {  // side stream for the near field (default priority) and its fork/join events
    BIE_HIP_CHECK(hipStreamCreateWithFlags(&plan.side, hipStreamNonBlocking));
    // both streams are on one device: a device-scope release suffices, and the default
    // system-scope fence of the event marker (a cache write-back and invalidation) would leave
    // the stream idle for several microseconds at every fork and join
    constexpr unsigned kFlags = hipEventDisableTiming | hipEventDisableSystemFence;
    BIE_HIP_CHECK(hipEventCreateWithFlags(&plan.fork, kFlags));
    BIE_HIP_CHECK(hipEventCreateWithFlags(&plan.join, kFlags));
  }
  ProfScope prof(BIE_K_FMM, s, (long long)R * M * (long long)M);
  hipLaunchKernelGGL(k_gather, dim3((M + 255) / 256), dim3(256), 0, s, M, R, kind, t.perm, t.xs, g->w,
                     mu, s64,
                     f32 ? nullptr : reinterpret_cast<double2 *>(wq),
                     f32 ? reinterpret_cast<float2 *>(wq) : nullptr, S4);
  // the near field needs only the source records: it runs on the side stream while the
  // expansions are built, and writes `partial`; the L2P kernels add the far part after the join
  BIE_HIP_CHECK(hipEventRecord(plan.fork, s));
  auto launch_near = [&]() -> int {
    BIE_HIP_CHECK(hipStreamWaitEvent(plan.side, plan.fork, 0));
    if (fuse && finish->with_L)  // the body charges for the finishing evaluation
      hipLaunchKernelGGL(k_body_sums, dim3(g->N, R), dim3(256), 0, plan.side, M, g->N,
                         g->body_ptr, s64, charge);
    {
      // the float32 near field in every mixed apply (Laplace and Stokes)
      const bool near32 = precision == BIE_MIXED;
      ProfScope pe(near32 ? BIE_K_FMM_NEAR_F32 : BIE_K_FMM_EVAL, plan.side,
                   (t.near_pairs - M) * R);
      if (kind == 0 && near32)
        hipLaunchKernelGGL(k_near_f32<false>, dim3(t.nchunk, R), dim3(256), 0, plan.side, M,
                           t.leaf_start, t.xs, t.nrm, t.perm, t.run_ptr, t.run, t.chunk_leaf,
                           t.chunk_start, S4, partial);
      else if (near32)
        hipLaunchKernelGGL(k_near_f32<true>, dim3(t.nchunk, R), dim3(256), 0, plan.side, M,
                           t.leaf_start, t.xs, t.nrm, t.perm, t.run_ptr, t.run, t.chunk_leaf,
                           t.chunk_start, S4, partial);
      else if (kind == 0)
        hipLaunchKernelGGL(k_near<false>, dim3(t.nchunk, R), dim3(256), 0, plan.side, M,
                           t.leaf_start, t.xs, t.nrm, t.perm, t.run_ptr, t.run, t.chunk_leaf,
                           t.chunk_start, S4, partial);
      else
        hipLaunchKernelGGL(k_near<true>, dim3(t.nchunk, R), dim3(256), 0, plan.side, M,
                           t.leaf_start, t.xs, t.nrm, t.perm, t.run_ptr, t.run, t.chunk_leaf,
                           t.chunk_start, S4, partial);
      BIE_HIP_CHECK(hipGetLastError());
    }
    BIE_HIP_CHECK(hipEventRecord(plan.join, plan.side));
    return BIE_OK;
  };
  const double ih_leaf = (double)(1 << t.L) / t.size;
  BIE_TRY(with_order(p, [&](auto order) -> int {
    constexpr int P = decltype(order)::value;
    if (f32)
      return expansion_passes<P, float>(t, plan, kind, R, nsets, ih_leaf,
                                        reinterpret_cast<const float2 *>(wq),
                                        reinterpret_cast<float2 *>(wm),
                                        reinterpret_cast<float2 *>(wl), partial, s, launch_near,
                                        fin);
    return expansion_passes<P, double>(t, plan, kind, R, nsets, ih_leaf,
                                       reinterpret_cast<const double2 *>(wq),
                                       reinterpret_cast<double2 *>(wm),
                                       reinterpret_cast<double2 *>(wl), partial, s, launch_near,
                                       fin);
  }));
  BIE_HIP_CHECK(hipGetLastError());
  return BIE_OK;
}

}  // namespace bie
