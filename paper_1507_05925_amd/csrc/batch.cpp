// Batched solves over several geometries: each (item, rhs) is one system of the segmented GMRES
// (gmres.cpp); one Arnoldi step applies the operator of every geometry to its systems.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <string>
#include <vector>

#include "internal.h"

struct bie_batch {
  bie::SolverMem sm;
  bie::Segments seg;
  bie::DevBuf flat;  // incident densities, rhs, solutions [Ntot] each (and P u, preconditioned)
  bie::DevBuf pcitems;  // the batched preconditioner's item descriptors
  bie::DevBuf ident; // identity blocks
  bie::MultiPlan *plan = nullptr;
};

namespace bie {
namespace {

__global__ void k_identity(int n, int cols, int col0, double *out) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long long)n * cols) return;
  const int r = (int)(t / cols), c = (int)(t % cols);  // row r of the block = rhs r
  out[t] = (c == col0 + r) ? 1.0 : 0.0;
}

}  // namespace
}  // namespace bie

using namespace bie;

extern "C" {

int bie_batch_create(bie_batch **out) {
  if (!out) {
    set_error("bie_batch_create: NULL out");
    return BIE_EINVAL;
  }
  *out = new (std::nothrow) bie_batch();
  if (!*out) {
    set_error("host allocation failed");
    return BIE_ENOMEM;
  }
  return BIE_OK;
}

int bie_batch_destroy(bie_batch *b) {
  if (!b) return BIE_OK;
  (void)hipDeviceSynchronize();
  b->sm.release();
  b->seg.buf.release();
  b->flat.release();
  b->ident.release();
  b->pcitems.release();
  bie::multi_destroy(b->plan);
  delete b;
  return BIE_OK;
}

int bie_batch_solve(bie_batch *b, int nitems, const bie_batch_item *items, const bie_opts *opts,
                    bie_info *info, double *rel_residual, void *stream) {
  auto t0 = std::chrono::steady_clock::now();
  if (!b || nitems < 1 || !items) {
    set_error("bie_batch_solve: need a batch, nitems >= 1 and items");
    return BIE_EINVAL;
  }
  bie_opts o;
  if (opts) o = *opts; else bie_default_opts(&o);
  BIE_TRY(check_opts(o));
  if (o.l2_scaling) {
    set_error("bie_batch_solve: l2_scaling is supported by the single-geometry solves only");
    return BIE_EINVAL;
  }

  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  std::vector<long long> lens, starts, item_off(nitems + 1, 0), in_off(nitems + 1, 0);
  long long pairs = 0;
  for (int i = 0; i < nitems; ++i) {
    const bie_batch_item &it = items[i];
    if (!it.g || (it.kind != 0 && it.kind != 1) || it.nrhs < 1 || !it.out) {
      set_error("bie_batch_solve: item " + std::to_string(i) + " is invalid");
      return BIE_EINVAL;
    }
    const int cols = it.kind == 0 ? it.g->N : 3 * it.g->N;
    if (!it.in && it.nrhs != cols) {
      set_error("bie_batch_solve: identity block of item " + std::to_string(i) +
                " needs nrhs = " + std::to_string(cols));
      return BIE_EINVAL;
    }
    const long long n = it.kind == 0 ? it.g->M : 2LL * it.g->M;
    for (int r = 0; r < it.nrhs; ++r) {
      lens.push_back(n);
      starts.push_back(item_off[i] + r * n);
    }
    item_off[i + 1] = align8(item_off[i] + n * it.nrhs);  // 64-byte aligned item blocks
    in_off[i + 1] = in_off[i] + (long long)cols * (it.in ? 0 : it.nrhs);
    pairs += (long long)it.nrhs * it.g->M * (long long)it.g->M;
    it.g->fmm_order = effective_order(o, it.kind);
    // leaf sizes (fmm_leaf 0: the tuner's, for items the FMM applies)
    BIE_TRY(resolve_leaf(it.g, it.kind, o, it.nrhs, method_is_fmm(o.method, it.g->M), s));
  }
  const long long Ntot = item_off[nitems];
  BIE_TRY(b->seg.build(lens, s, &starts));
  const bool pcb = o.precond == BIE_PRECOND_BLOCK;
  BIE_TRY(b->flat.reserve((pcb ? 4 : 3) * (size_t)Ntot * sizeof(double)));
  double *dens = b->flat.as<double>(), *f = dens + Ntot, *mu = f + Ntot;
  double *ptmp = pcb ? mu + Ntot : nullptr;  // P u, the operator's input, when preconditioned
  if (in_off[nitems] > 0) BIE_TRY(b->ident.reserve((size_t)in_off[nitems] * sizeof(double)));
  // incident densities and right-hand sides, per item
  for (int i = 0; i < nitems; ++i) {
    const bie_batch_item &it = items[i];
    const double *in = it.in;
    if (!in) {
      const int cols = it.kind == 0 ? it.g->N : 3 * it.g->N;
      double *id = b->ident.as<double>() + in_off[i];
      const long long tot = (long long)cols * it.nrhs;
      hipLaunchKernelGGL(k_identity, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s,
                         it.nrhs, cols, 0, id);
      BIE_HIP_CHECK(hipGetLastError());
      in = id;
    }
    BIE_TRY(incident_density(it.g, it.kind, it.nrhs, in, dens + item_off[i], s));
    BIE_TRY(apply_operator(it.g, it.kind, BIE_FP64, o.method, 0, -1.0, it.nrhs, dens + item_off[i],
                           f + item_off[i], s));
  }
  SysSet ss;
  ss.seg = &b->seg;
  ss.mem = &b->sm;
  ss.pairs_per_apply = pairs;
  std::vector<MultiItem> mitems(nitems);
  std::vector<int> first_sys(nitems + 1, 0);
  for (int i = 0; i < nitems; ++i) {
    bie_geom *g = items[i].g;
    mitems[i] = {g, items[i].kind, items[i].nrhs, item_off[i],
                 method_is_fmm(o.method, g->M), effective_order(o, items[i].kind), g->fmm_leaf};
    first_sys[i + 1] = first_sys[i] + items[i].nrhs;
  }
  ss.group_ptr = first_sys;  // items: a relaxed mixed solve picks precisions per item
  for (int i = 0; i < nitems; ++i)
    ss.group_eta.push_back(
        mixed_apply_error(items[i].g, items[i].kind, o.method, effective_order(o, items[i].kind)));
  // right preconditioning (GMRES on (A P) u = f, x = P u): every item's geometry's blocks, one
  // batched launch per apply
  size_t pc_lds = 0;
  long long pc_blocks = 0, pc_macs = 0;
  const PcBatchItem *pc_items = nullptr;
  if (pcb) {
    std::vector<bie_geom *> gs(nitems);
    std::vector<int> kinds(nitems), nr(nitems);
    std::vector<long long> offs(nitems);
    for (int i = 0; i < nitems; ++i) {
      BIE_TRY(pc_build(items[i].g, items[i].kind, s));
      gs[i] = items[i].g;
      kinds[i] = items[i].kind;
      nr[i] = items[i].nrhs;
      offs[i] = item_off[i];
    }
    std::vector<PcBatchItem> pit;
    BIE_TRY(pc_batch_items(gs, kinds, nr, offs, pit, pc_lds, pc_blocks, pc_macs));
    BIE_TRY(b->pcitems.reserve(pit.size() * sizeof(PcBatchItem)));
    BIE_HIP_CHECK(hipMemcpyAsync(b->pcitems.ptr, pit.data(), pit.size() * sizeof(PcBatchItem),
                                 hipMemcpyHostToDevice, s));
    BIE_HIP_CHECK(hipStreamSynchronize(s));  // the host descriptors go out of scope
    pc_items = reinterpret_cast<const PcBatchItem *>(b->pcitems.ptr);
  }
  SysSet *ssp = &ss;
  MultiPlan **plan = &b->plan;
  ss.apply = [ssp, plan, mitems, first_sys, Ntot, pc_items, pc_lds, pc_blocks, pc_macs, ptmp,
              nitems](int precision, const double *in, double *out, hipStream_t st) {
    if (pc_items) {
      BIE_TRY(pc_apply_batch(nitems, pc_items, pc_lds, pc_blocks, pc_macs, in, ptmp, st));
      in = ptmp;
    }
    // an item is applied when any of its systems is still active
    std::vector<char> act(mitems.size(), 1);
    if (!ssp->active.empty())
      for (size_t i = 0; i < mitems.size(); ++i) {
        char a = 0;
        for (int k = first_sys[i]; k < first_sys[i + 1]; ++k) a |= ssp->active[k];
        act[i] = a;
      }
    if (precision == kPrecPerGroup)
      return multi_apply(*plan, mitems, act, BIE_FP64, in, out, Ntot, st, &ssp->group_f32);
    return multi_apply(*plan, mitems, act, precision, in, out, Ntot, st);
  };
  std::vector<double> rel;
  bie_info inf{};
  int rc = solve_systems(ss, o, f, mu, rel, &inf, s);
  if (rc != BIE_OK && rc != BIE_ENOCONV) return rc;
  if (pc_items)  // x = P u, in place (each body is staged before it is written)
    BIE_TRY(pc_apply_batch(nitems, pc_items, pc_lds, pc_blocks, pc_macs, mu, mu, s));
  BIE_TRY(vec_axpby(Ntot, 1.0, mu, 1.0, dens, s));
  for (int i = 0; i < nitems; ++i) {
    BIE_TRY(read_off(items[i].g, items[i].kind, items[i].nrhs, dens + item_off[i], items[i].out, s,
                     mitems[i].fmm ? BIE_FMM : BIE_DIRECT));
    if (items[i].kind == 1 && o.viscosity != 1.0)  // velocities for the caller's viscosity
      BIE_TRY(vec_axpby((long long)items[i].nrhs * 3 * items[i].g->N, 0.0, items[i].out,
                        1.0 / o.viscosity, items[i].out, s));
  }
  BIE_HIP_CHECK(hipStreamSynchronize(s));
  if (rel_residual) {
    size_t k = 0;
    for (int i = 0; i < nitems; ++i) {
      double w = 0.0;
      for (int r = 0; r < items[i].nrhs; ++r) w = std::max(w, rel[k++]);
      rel_residual[i] = w;
    }
  }
  inf.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  if (info) *info = inf;
  return rc;
}

}  // extern "C"
