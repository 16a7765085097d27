"""Benchmark: elastance solves on 1000 starfish conductors x 256 nodes (256,000 unknowns).

Setup (untimed, reported): the curve samples and charges are put in HBM, the geometry and
quadrature data are built on the device (bie_geom_create), and one solve builds the FMM tree.
One timed step = one whole solve on that resident geometry: incident charge and right-hand side,
GMRES to a relative residual of 1e-10 with the operator apply (far field by the 2D FMM, float64
self terms, diagonal and completion), potentials read off inside every conductor.

Reported value: pair interactions per second, counted as M^2 per operator apply (for the FMM this
is the equivalent direct count, labelled as such in `metric`), over the timed steps.
`roofline` is for the kernel that takes the most time in the timed steps, measured with HIP
events on the launch stream; `roofline_direct_p2p` is the direct float32 far-field sweep on the
same workload.

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--method fmm|direct]
                  [--precision fp64|mixed] [--no-cpu-baseline]
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK = {"f32": 157.3, "f64": 78.6}  # MI355X vector TFLOP/s
FLOPS_PER_PAIR = 11  # Laplace traction kernel: 2 sub, r^2 (3), reciprocal (1), scale (1), 2 fma (4)
FLOPS_PER_CMAC = 8   # complex multiply-add


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=10)
    p.add_argument("--warmup", type=int, default=2)
    p.add_argument("--method", choices=["fmm", "direct"], default="fmm")
    p.add_argument("--precision", choices=["fp64", "mixed"], default=None)
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
    stride = 997
    while True:
        rows = np.arange(0, geo["M"], stride, dtype=np.int32)
        t = time.perf_counter()
        mf.laplace_apply(geo, mu, rows=rows)
        dt = time.perf_counter() - t
        if dt >= 0.5 * target_seconds or stride == 1:
            break
        stride = max(1, int(stride * dt / target_seconds))
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    pairs = len(rows) * geo["M"]
    return {"value": pairs / dt, "unit": "pair-interactions/s", "cores": cores, "kind": "oracle",
            "sample": f"float64 oracle apply of (1/2 I + K + L) (direct sum, no FMM): {len(rows)} "
                      f"of {geo['M']} target rows x all {geo['M']} sources = {pairs:.3e} pairs in "
                      f"{dt:.1f} s wall"}


def roofline(prof, kc, units_flops, dtype):
    ms = prof["ms_total"] / max(prof["launches"], 1)
    units = prof["pairs"] / max(prof["launches"], 1)
    ach = units_flops * units / (ms * 1e-3) / 1e12 if ms > 0 else 0.0
    return {"bound": "alu", "achieved": ach, "peak": PEAK[dtype], "unit": "TFLOP/s",
            "frac": ach / PEAK[dtype], "traffic": None, "avg_launch_ms": ms,
            "launches": prof["launches"], "units_per_launch": units, "flops_per_unit": units_flops}


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

    torch.cuda.set_device(0)
    dev = "cuda:0"
    curves, q = wl.elastance_starfish()
    c = np.stack([curves.x, curves.y, curves.dx, curves.dy, curves.ddx, curves.ddy])
    curve_d = torch.from_numpy(np.ascontiguousarray(c)).to(dev)
    q_d = torch.as_tensor(q[None], device=dev)
    meth = bie2d.BIE_FMM if a.method == "fmm" else bie2d.BIE_DIRECT
    precision = a.precision or ("fp64" if a.method == "fmm" else "mixed")
    prec = bie2d.BIE_MIXED if precision == "mixed" else bie2d.BIE_FP64
    opts = bie2d.default_opts(precision=prec, method=meth, tol=a.tol, restart=100, max_iter=2000)

    torch.cuda.synchronize()
    t = time.perf_counter()
    g = bie2d.Geometry(curves.nodes_per_body, curve_d)
    torch.cuda.synchronize()
    t_geom = time.perf_counter() - t
    t = time.perf_counter()
    bie2d.bie_elastance_solve(g, q_d, opts)
    t_first = time.perf_counter() - t
    for _ in range(a.warmup):
        bie2d.bie_elastance_solve(g, q_d, opts)
    torch.cuda.synchronize()

    bie2d.bie_profile_enable(True)
    lat, pairs, info = [], 0, None
    t0 = time.perf_counter()
    for _ in range(a.steps):
        s = time.perf_counter()
        phi, info = bie2d.bie_elastance_solve(g, q_d, opts)
        lat.append(time.perf_counter() - s)
        pairs += info["pairs"]
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    classes = {
        "k_lap_far_f32": (bie2d.BIE_K_FAR_LAPLACE_F32, FLOPS_PER_PAIR, "f32"),
        "k_lap_far_f64": (bie2d.BIE_K_FAR_LAPLACE_F64, FLOPS_PER_PAIR, "f64"),
        "k_m2l": (bie2d.BIE_K_FMM_M2L, FLOPS_PER_CMAC, "f64"),
        "k_eval_laplace": (bie2d.BIE_K_FMM_EVAL, FLOPS_PER_PAIR, "f64"),
        "k_lap_epilogue": (bie2d.BIE_K_EPILOGUE, 0, "f64"),
    }
    profs = {k: bie2d.bie_profile_read(v[0]) for k, v in classes.items()}
    fmm_total = bie2d.bie_profile_read(bie2d.BIE_K_FMM)
    bie2d.bie_profile_enable(False)
    dom = max((k for k in classes if classes[k][1] > 0), key=lambda k: profs[k]["ms_total"])
    rl = roofline(profs[dom], classes[dom][0], classes[dom][1], classes[dom][2])
    rl["kernel"] = dom

    # the direct float32 far-field sweep on the same workload (survey row a3), 5 applies
    mu = torch.randn(1, g.M, dtype=torch.float64, device=dev)
    bie2d.bie_laplace_apply(g, mu, bie2d.BIE_MIXED, bie2d.BIE_DIRECT)
    torch.cuda.synchronize()
    bie2d.bie_profile_enable(True)
    for _ in range(5):
        bie2d.bie_laplace_apply(g, mu, bie2d.BIE_MIXED, bie2d.BIE_DIRECT)
    torch.cuda.synchronize()
    p32 = bie2d.bie_profile_read(bie2d.BIE_K_FAR_LAPLACE_F32)
    bie2d.bie_profile_enable(False)
    rl_direct = roofline(p32, bie2d.BIE_K_FAR_LAPLACE_F32, FLOPS_PER_PAIR, "f32")
    rl_direct["kernel"] = "k_lap_far_f32<1>"

    acc = {}
    gold = os.path.join(ROOT, "tests", "golden", "starfish_1000x256_phi.json")
    if os.path.exists(gold):
        ref = np.asarray(json.load(open(gold))["phi"])
        acc["rel_err_vs_fp64_oracle"] = float(np.abs(phi.cpu().numpy()[0] - ref).max() / np.abs(ref).max())
    phi64, info64 = bie2d.bie_elastance_solve(
        g, q_d, bie2d.default_opts(precision=bie2d.BIE_FP64, method=bie2d.BIE_DIRECT, tol=1e-12,
                                   restart=100))
    acc["rel_err_vs_fp64_direct_gpu"] = float((phi - phi64).abs().max() / phi64.abs().max())
    acc["fp64_direct_gpu_solve_seconds"] = info64["seconds"]

    lat_sorted = sorted(lat)
    label = "equivalent direct " if meth == bie2d.BIE_FMM else ""
    res = {
        "metric": f"pair-interactions/s ({label}M^2 per operator apply) of full elastance solves "
                  f"to <=1e-9 rel err vs float64",
        "value": pairs / elapsed,
        "unit": "pair-interactions/s",
        "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
        "ms_per_step": 1e3 * elapsed / a.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32+f64" if prec == bie2d.BIE_MIXED else "f64",
        "data": "synthetic (seeded starfish ensemble, q ~ N(0,1))",
        "config": {"workload": "elastance, 1000 starfish r0(1+0.3cos5t) x 256 nodes (M=256000), "
                               "q~N(0,1), GMRES tol 1e-10",
                   "method": a.method, "precision": precision, "fmm_order": opts.fmm_order,
                   "nodes": curves.M, "bodies": curves.nbodies},
        "solves_per_s": a.steps / elapsed,
        "latency_s": {"p50": lat_sorted[len(lat) // 2],
                      "p99": lat_sorted[min(len(lat) - 1, int(0.99 * len(lat)))]},
        "setup_s": {"geometry": t_geom, "first_solve_incl_tree": t_first},
        "gmres": {k: info[k] for k in ("iters", "refinements", "applies_fp32", "applies_fp64",
                                       "rel_residual")},
        "accuracy": acc,
        "roofline": rl,
        "roofline_direct_p2p": rl_direct,
        "kernel_ms_per_step": {k: v["ms_total"] / a.steps for k, v in profs.items()},
        "fmm_ms_per_apply": fmm_total["ms_total"] / max(fmm_total["launches"], 1),
    }
    if not a.no_cpu_baseline:
        res["cpu_baseline"] = cpu_baseline(curves, a.cpu_seconds)
    g.close()
    print(json.dumps(res))


if __name__ == "__main__":
    main()
