"""Benchmark: elastance solves on 1000 starfish conductors x 256 nodes (256,000 unknowns).

One step = the whole path on one charge vector q ~ N(0,1), inputs resident in HBM:
  geometry and quadrature (bie_geom_create) -> incident charge and right-hand side ->
  GMRES with the operator apply (float32 far-field sweep + float64 self blocks, diagonal and
  completion) and float64 iterative refinement to a relative residual of 1e-10 -> potentials
  read off inside every conductor.
Reported value: pair interactions per second (M^2 per operator apply, all applies of the timed
steps, divided by the timed wall clock). Also solves/s and per-step latency percentiles.

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--precision mixed|fp64]
                  [--method direct|fmm] [--no-cpu-baseline]
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK = {"f32": 157.3, "f64": 78.6}  # MI355X vector TFLOP/s (datasheet)
HBM_PEAK = 8000.0  # GB/s
FLOPS_PER_PAIR = {"laplace": 11, "stokes": 19}


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=3)
    p.add_argument("--warmup", type=int, default=1)
    p.add_argument("--precision", choices=["mixed", "fp64"], default="mixed")
    p.add_argument("--method", choices=["direct", "fmm"], default="direct")
    p.add_argument("--tol", type=float, default=1e-10)
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--cpu-seconds", type=float, default=12.0)
    return p.parse_args()


def cpu_baseline(curves, target_seconds):
    """The float64 CPU oracle's matrix-free apply (plain C loops, OpenMP over targets) on a
    bounded sample of target rows of the same workload, scaled to pairs/s."""
    import numpy as np

    from oracle import matfree as mf
    from oracle import nystrom as ny

    geo = ny.geometry_of(curves)
    mu = np.random.default_rng(0).standard_normal(geo["M"])
    rows = np.arange(0, geo["M"], 997, dtype=np.int32)
    t = time.perf_counter()
    mf.laplace_apply(geo, mu, rows=rows)
    dt = time.perf_counter() - t
    # scale the sample so that the measured leg takes about target_seconds
    stride = max(1, int(997 * dt / target_seconds))
    rows = np.arange(0, geo["M"], stride, dtype=np.int32)
    t = time.perf_counter()
    mf.laplace_apply(geo, mu, rows=rows)
    dt = time.perf_counter() - t
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    pairs = len(rows) * geo["M"]
    return {"value": pairs / dt, "unit": "pair-interactions/s", "cores": cores, "kind": "oracle",
            "sample": f"float64 oracle apply (1/2 I + K + L), {len(rows)} of {geo['M']} target rows "
                      f"x all {geo['M']} sources ({pairs:.3e} pairs, {dt:.1f} s wall)"}


def main():
    a = parse()
    if a.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU; --gpus N > 1 is not "
                                   "supported (one-GPU build, no collectives)"}))
        sys.exit(2)
    import numpy as np
    import torch

    from paper_1507_05925_amd import bie2d
    from paper_1507_05925_amd import workloads as wl

    dev = "cuda:0"
    torch.cuda.set_device(0)
    curves, q = wl.elastance_starfish()
    c = np.stack([curves.x, curves.y, curves.dx, curves.dy, curves.ddx, curves.ddy])
    curve_d = torch.from_numpy(np.ascontiguousarray(c)).to(dev)
    q_d = torch.as_tensor(q[None], device=dev)
    prec = bie2d.BIE_MIXED if a.precision == "mixed" else bie2d.BIE_FP64
    meth = bie2d.BIE_DIRECT if a.method == "direct" else bie2d.BIE_FMM
    opts = bie2d.default_opts(precision=prec, method=meth, tol=a.tol, restart=100, max_iter=2000)

    def step():
        g = bie2d.Geometry(curves.nodes_per_body, curve_d)
        phi, info = bie2d.bie_elastance_solve(g, q_d, opts)
        g.close()
        return phi, info

    for _ in range(a.warmup):
        step()
    torch.cuda.synchronize()
    bie2d.bie_profile_enable(True)
    lat, pairs, infos = [], 0, []
    t0 = time.perf_counter()
    for _ in range(a.steps):
        s = time.perf_counter()
        phi, info = step()
        torch.cuda.synchronize()
        lat.append(time.perf_counter() - s)
        pairs += info["pairs"]
        infos.append(info)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    kc = bie2d.BIE_K_FAR_LAPLACE_F32 if prec == bie2d.BIE_MIXED else bie2d.BIE_K_FAR_LAPLACE_F64
    if meth == bie2d.BIE_FMM:
        kc = bie2d.BIE_K_FMM
    far = bie2d.bie_profile_read(kc)
    epi = bie2d.bie_profile_read(bie2d.BIE_K_EPILOGUE)
    bie2d.bie_profile_enable(False)

    # accuracy of the benchmarked result: against the float64 oracle's stored solution and
    # against this library's float64 path (untimed)
    acc = {}
    gold = os.path.join(ROOT, "tests", "golden", "starfish_1000x256_phi.json")
    if os.path.exists(gold):
        ref = np.asarray(json.load(open(gold))["phi"])
        acc["rel_err_vs_fp64_oracle"] = float(np.abs(phi.cpu().numpy()[0] - ref).max() / np.abs(ref).max())
    if prec == bie2d.BIE_MIXED:
        g = bie2d.Geometry(curves.nodes_per_body, curve_d)
        phi64, info64 = bie2d.bie_elastance_solve(
            g, q_d, bie2d.default_opts(precision=bie2d.BIE_FP64, method=meth, tol=1e-12, restart=100))
        g.close()
        acc["rel_err_vs_fp64_gpu"] = float((phi - phi64).abs().max() / phi64.abs().max())
        acc["fp64_gpu_solve_seconds"] = info64["seconds"]

    avg_ms = far["ms_total"] / max(far["launches"], 1)
    pairs_per_launch = far["pairs"] / max(far["launches"], 1)
    fl = FLOPS_PER_PAIR["laplace"]
    dtype_k = "f32" if prec == bie2d.BIE_MIXED else "f64"
    achieved = fl * pairs_per_launch / (avg_ms * 1e-3) / 1e12 if avg_ms > 0 else 0.0
    lat_sorted = sorted(lat)
    res = {
        "metric": "pair-interactions/s (M^2 per operator apply) of full elastance solves, "
                  "mixed precision refined to <=1e-9 vs float64",
        "value": pairs / elapsed,
        "unit": "pair-interactions/s",
        "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
        "ms_per_step": 1e3 * elapsed / a.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32+f64" if prec == bie2d.BIE_MIXED else "f64",
        "data": "synthetic (seeded starfish ensemble, q ~ N(0,1))",
        "config": {"workload": "elastance, 1000 starfish r0(1+0.3cos5t) x 256 nodes "
                               "(M=256000), q~N(0,1), GMRES tol 1e-10",
                   "precision": a.precision, "method": a.method, "nodes": curves.M,
                   "bodies": curves.nbodies},
        "solves_per_s": a.steps / elapsed,
        "latency_s": {"p50": lat_sorted[len(lat) // 2], "p99": lat_sorted[min(len(lat) - 1, int(0.99 * len(lat)))]},
        "gmres": {"iters": infos[-1]["iters"], "refinements": infos[-1]["refinements"],
                  "applies_fp32": infos[-1]["applies_fp32"], "applies_fp64": infos[-1]["applies_fp64"],
                  "rel_residual": infos[-1]["rel_residual"]},
        "accuracy": acc,
        "roofline": {"bound": "alu", "kernel": "k_lap_far_f32<1>" if dtype_k == "f32" else "k_lap_far_f64<1>",
                     "achieved": achieved, "peak": PEAK[dtype_k], "unit": "TFLOP/s",
                     "frac": achieved / PEAK[dtype_k], "traffic": None,
                     "avg_launch_ms": avg_ms, "launches": far["launches"],
                     "pairs_per_launch": pairs_per_launch, "flops_per_pair": fl},
        "epilogue_ms_per_launch": epi["ms_total"] / max(epi["launches"], 1),
    }
    if not a.no_cpu_baseline:
        res["cpu_baseline"] = cpu_baseline(curves, a.cpu_seconds)
    print(json.dumps(res))


if __name__ == "__main__":
    main()
