"""Benchmark: elastance solves on 1000 starfish conductors x 256 nodes (256,000 unknowns).

Setup (untimed, reported): the curve samples and charges are put in HBM, the geometry and
quadrature data are built on the device (bie_geom_create), and one solve builds the FMM tree.
One timed step = one whole solve on that resident geometry: incident charge and right-hand side,
GMRES to a relative residual of 1e-10 with the operator apply (far field by the 2D FMM, float64
self terms, diagonal and completion), potentials read off inside every conductor. By default the
solves are mixed precision (float64 GMRES whose late steps apply the float32 operator) with the
block right preconditioner (two-grid blocks on 64 coarse nodes per body), checked against the
stored float64 oracle potentials; `fp64_path` times the same solves in float64,
`unpreconditioned` the mixed solves without the preconditioner (the paper's plain GMRES).

Reported value: solves per second over the timed steps; pair interactions per second (M^2 per
operator apply, for the FMM the equivalent direct count, labelled as such) alongside.
`roofline` is for the kernel that takes the most time in the timed steps, measured with HIP
events on the launch stream; `roofline_direct_p2p` is the direct float32 far-field sweep on the
same workload.

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--method fmm|direct]
                  [--precision fp64|mixed] [--mixed-strategy relaxed|refine]
                  [--no-cpu-baseline]

Other workloads (not the default line):
  --workload serve   Poisson stream of elastance (60%) and mobility (40%) queries on
                     device-resident geometries of 2-500 bodies x 64-256 nodes, served with
                     continuous batching at 0.7 x the measured saturation rate; p50/p99
                     latency and solves/s next to the plain float64 GPU path (one solve at a
                     time, FIFO, same arrival times).
  --workload mobility 200 rigid ellipses x 512 nodes (204,800 unknowns), FMM: solves in float64
                     and in the mixed mode, (v, omega) against the stored float64 oracle solution.
  --workload batched 32 geometries of 8-128 bodies: every P and M in one batched solve.
  --workload nanocomposite  every configuration of the paper's nanocomposite capacitance table
                     (two plates and m x 10 particles, m = 0, 1, 4, 16, five aspect ratios): the
                     capacitance and the solve time beside the printed ones.
  --workload crosstest  the paper's cross-tests (capacitance then elastance, resistance then
                     mobility) on two discs at three gaps and the splash curves.
  --workload copy    a plain 256 MiB device copy kernel (y = -x), 6 times: the known-size reference that
                     scales the FETCH_SIZE / WRITE_SIZE counters into HBM bytes.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK = {"f32": 157.3, "f64": 78.6}  # MI355X vector TFLOP/s (float64 MFMA: also 78.6)
FLOPS_PER_PAIR = 11  # Laplace traction kernel: 2 sub, r^2 (3), reciprocal (1), scale (1), 2 fma (4)
FLOPS_PER_CMAC = 8   # complex multiply-add
FLOPS_PER_PAIR_STOKES = 19  # stresslet kernel per node pair (two components)


PROFILE_EVERY = 8  # launches per timed launch of the roofline kernel in the timed solves


MIXED_STRATEGY = {"relaxed": 0, "refine": 1}  # BIE_MIXED_RELAXED, BIE_MIXED_REFINE


def m2l_flops_per_entry(p):
    """One M2L interaction-list entry as the kernel computes it: the source scaled by d^-m
    (p complex products, 6 flops each), the real Hankel matrix C (p x p) applied to its real and
    imaginary parts (2 p^2 multiply-adds, 4 p^2 flops), and the product scaled by d^-(n+1) and
    added (p complex multiply-adds, 8 flops each)."""
    return 4 * p * p + 14 * p


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=10)
    p.add_argument("--warmup", type=int, default=2)
    p.add_argument("--method", choices=["fmm", "direct"], default="fmm")
    p.add_argument("--precision", choices=["fp64", "mixed"], default=None)
    p.add_argument("--mixed-strategy", choices=["relaxed", "refine"], default="relaxed")
    p.add_argument("--fmm-leaf", type=int, default=0,
                   help="FMM mean nodes per leaf (0: the library's autotuner picks it)")
    # the workloads ask for an FMM at 1e-10 (24 terms in the float64 Laplace applies). Without
    # the preconditioner a 1e-12 FMM (32 terms) paid for itself (34 GMRES steps against 37 on the
    # 1000 starfish); with it both take 12 steps and the shorter expansions are faster
    p.add_argument("--fmm-eps", type=float, default=1e-10,
                   help="FMM accuracy target (float64 apply, relative); 0: --fmm-order")
    p.add_argument("--fmm-order", type=int, default=40)
    p.add_argument("--precond", choices=["none", "block"], default="block",
                   help="GMRES right preconditioner of the elastance and mobility solves (block: "
                        "two-grid inverses of the bodies' self blocks; the solution is the same)")
    p.add_argument("--tol", type=float, default=1e-10)
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--cpu-seconds", type=float, default=12.0)
    p.add_argument("--workload", choices=["starfish", "mobility", "serve", "batched", "nanocomposite",
                                          "crosstest", "copy"],
                   default="starfish")
    p.add_argument("--requests", type=int, default=2000)
    p.add_argument("--serve-restart", type=int, default=20)
    return p.parse_args()


def cpu_model():
    """The host CPU's model name (/proc/cpuinfo, as lscpu reports it)."""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def oracle_apply_rate(geo, mu, target_seconds):
    """Pairs/s of the float64 oracle's matrix-free apply on a strided sample of target rows
    sized to take about target_seconds; returns (rate, rows, seconds)."""
    import numpy as np

    from oracle import matfree as mf

    stride = 997
    while True:
        rows = np.arange(0, geo["M"], stride, dtype=np.int32)
        t = time.perf_counter()
        mf.laplace_apply(geo, mu, rows=rows)
        dt = time.perf_counter() - t
        if dt >= 0.5 * target_seconds or stride == 1:
            break
        stride = max(1, int(stride * dt / target_seconds))
    return len(rows) * geo["M"] / dt, len(rows), dt


def cpu_baseline(curves, target_seconds, applies_per_solve):
    """The float64 CPU oracle's matrix-free apply (plain C loops, OpenMP over targets) on a
    bounded sample of target rows of the same workload, scaled to pairs/s, with all host threads
    and with one, and to solves/s for a solve of `applies_per_solve` applies; and the dense
    oracle's solve (Nystrom matrix, LU) of the small 4-ellipse case next to the GPU solve of the
    same case."""
    import numpy as np

    from oracle import matfree as mf
    from oracle import nystrom as ny
    from paper_1507_05925_amd import bie2d
    from paper_1507_05925_amd import workloads as wl

    geo = ny.geometry_of(curves)
    mu = np.random.default_rng(0).standard_normal(geo["M"])
    threads = mf.set_threads(int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1)))
    rate, nrows, dt = oracle_apply_rate(geo, mu, target_seconds)
    mf.set_threads(1)
    rate1, nrows1, dt1 = oracle_apply_rate(geo, mu, target_seconds / 4)
    mf.set_threads(threads)
    # the 4-ellipse elastance case (512 unknowns): dense oracle solve vs the GPU float64 solve
    c1, q1 = wl.elastance_small()
    g1 = ny.geometry_of(c1)
    t = time.perf_counter()
    ref = ny.elastance_solve(g1, q1)
    t_lu = time.perf_counter() - t
    G = bie2d.Geometry.from_curves(c1)
    qd = __import__("torch").as_tensor(q1[None], device="cuda")
    o = bie2d.default_opts(precision=bie2d.BIE_FP64, tol=1e-12)
    bie2d.bie_elastance_solve(G, qd, o)
    t = time.perf_counter()
    phi, _ = bie2d.bie_elastance_solve(G, qd, o)
    __import__("torch").cuda.synchronize()
    t_gpu = time.perf_counter() - t
    G.close()
    err = float(np.abs(phi.cpu().numpy()[0] - ref["phi"]).max() / np.abs(ref["phi"]).max())
    pairs = nrows * geo["M"]
    per_solve = applies_per_solve * float(geo["M"]) ** 2
    return {"value": rate / per_solve, "unit": "solves/s", "cores": threads, "kind": "oracle",
            "cpu": cpu_model(),
            "sample": f"float64 oracle apply of (1/2 I + K + L) (direct sum, no FMM): {nrows} "
                      f"of {geo['M']} target rows x all {geo['M']} sources = {pairs:.3e} pairs in "
                      f"{dt:.1f} s wall on {threads} threads; solves/s for the oracle's plain "
                      f"GMRES taken at {applies_per_solve} applies of M^2 pairs (the GPU's "
                      f"unpreconditioned solve of the same system, with its right-hand side)",
            "pair_interactions_per_s": rate,
            "one_core": {"value": rate1 / per_solve, "unit": "solves/s",
                         "pair_interactions_per_s": rate1,
                         "sample": f"{nrows1} rows x {geo['M']} sources in {dt1:.1f} s, 1 thread"},
            "small_case_solve": {"workload": "elastance, 4 ellipses x 128 nodes (512 unknowns)",
                                 "oracle_dense_lu_s": t_lu, "gpu_fp64_solve_s": t_gpu,
                                 "gpu_rel_err_vs_oracle": err}}


def roofline(prof, kc, units_flops, dtype, bound="alu", kernel=None):
    """Achieved algorithmic FLOP/s of one kernel class from its live HIP-event launch timings."""
    ms = prof["ms_total"] / max(prof["launches"], 1)
    units = prof["pairs"] / max(prof["launches"], 1)
    ach = units_flops * units / (ms * 1e-3) / 1e12 if ms > 0 else 0.0
    peak = PEAK[dtype]
    return {"bound": bound, "achieved": ach, "peak": peak, "unit": "TFLOP/s",
            "frac": ach / peak, "traffic": traffic_bytes(kernel), "avg_launch_ms": ms,
            "launches": prof["launches"], "units_per_launch": units, "flops_per_unit": units_flops}


def traffic_bytes(kernel):
    """HBM bytes per launch of `kernel` from the committed counter summary (profiles/traffic.json:
    FETCH_SIZE and WRITE_SIZE per dispatch, scaled by the copy-kernel calibration), or None when
    there is none or the kernel's source file has changed since the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if kernel is None or not os.path.exists(path):
        return None
    rec = json.load(open(path)).get(kernel)
    if not rec:
        return None
    src = os.path.join(ROOT, rec["source"])
    if hashlib.sha256(open(src, "rb").read()).hexdigest() != rec["source_sha256"]:
        return None
    return rec["fetch_bytes"] + rec["write_bytes"]


def pct(v, q):
    v = sorted(v)
    return v[min(len(v) - 1, int(q * len(v)))]


def serve_bench(a):
    import threading

    import numpy as np
    import torch

    from paper_1507_05925_amd import bie2d
    from paper_1507_05925_amd import workloads as wl

    warm = 100
    sessions = wl.serving_sessions(a.requests + warm)
    geoms = [bie2d.Geometry.from_curves(c) for _, c, _ in sessions]
    queries = [(si, kind, q) for si, (kind, c, qs) in enumerate(sessions) for q in qs]
    pc = bie2d.BIE_PRECOND_BLOCK if a.precond == "block" else bie2d.BIE_PRECOND_NONE
    opts = bie2d.default_opts(precision=bie2d.BIE_MIXED, method=bie2d.BIE_AUTO, tol=1e-10,
                              restart=a.serve_restart, precond=pc)
    # geometries are resident: quadrature data, FMM trees for both precisions and the block
    # preconditioner, built once (the preconditioner by one solve)
    for (kind, _, qs), g in zip(sessions, geoms):
        width = g.M if kind == 0 else 2 * g.M
        mu = torch.zeros(1, width, dtype=torch.float64, device="cuda")
        f = bie2d.bie_laplace_apply if kind == 0 else bie2d.bie_stokes_apply
        for prec in (bie2d.BIE_FP64, bie2d.BIE_MIXED):
            f(g, mu, prec, bie2d.BIE_AUTO)
        if pc != bie2d.BIE_PRECOND_NONE:
            solve = bie2d.bie_elastance_solve if kind == 0 else bie2d.bie_mobility_solve
            solve(g, torch.as_tensor(np.asarray(qs[0]).reshape(1, -1), device="cuda"), opts)
    torch.cuda.synchronize()
    srv = bie2d.Server(opts, hbm_budget_bytes=64 << 30, max_cycles=400)
    for x in [srv.submit(geoms[si], kind, q) for si, kind, q in queries[:warm]]:
        srv.wait(x)
    run = queries[warm:]
    # saturation: a backlog of queries drawn from the run's own mix, all submitted at once
    rng = np.random.default_rng(11)
    sample = rng.choice(len(run), size=min(300, len(run)), replace=False)
    t = time.perf_counter()
    for x in [srv.submit(geoms[run[i][0]], run[i][1], run[i][2]) for i in sample]:
        srv.wait(x)
    sat = len(sample) / (time.perf_counter() - t)

    def stream(rate, reqs, seed):
        arrivals = np.cumsum(np.random.default_rng(seed).exponential(1.0 / rate, size=len(reqs)))
        tickets = [None] * len(reqs)

        def client():
            t0 = time.perf_counter()
            for i, (si, kind, q) in enumerate(reqs):
                dt = arrivals[i] - (time.perf_counter() - t0)
                if dt > 0:
                    time.sleep(dt)
                tickets[i] = srv.submit(geoms[si], kind, q)

        t0 = time.perf_counter()
        th = threading.Thread(target=client)
        th.start()
        lat, outs, statuses = [], [], []
        for i in range(len(reqs)):
            while tickets[i] is None:
                time.sleep(0.0005)
            out, info = srv.wait(tickets[i])
            lat.append(info["latency_s"])
            outs.append(out)
            statuses.append(info["status"])
        th.join()
        wall = time.perf_counter() - t0
        return arrivals, lat, outs, statuses, wall

    rate = 0.7 * sat
    c0 = srv.stats()["cycles"]
    arrivals, lat, outs, statuses, wall = stream(rate, run, 7)
    st = srv.stats()
    st["cycles_in_run"] = st["cycles"] - c0
    sweep = []
    for frac in (0.4, 0.9):
        part = run[: max(1, len(run) // 2)]
        _, l2, _, s2, w2 = stream(frac * sat, part, 8)
        sweep.append({"offered_fraction_of_saturation": frac, "offered_rate_per_s": frac * sat,
                      "solves_per_s": len(part) / w2, "p50": pct(l2, 0.5), "p99": pct(l2, 0.99),
                      "all_ok": all(x == 0 for x in s2)})
    srv.close()
    # the plain float64 GPU path: one solve at a time; FIFO queue with the same arrivals
    o64 = bie2d.default_opts(precision=bie2d.BIE_FP64, method=bie2d.BIE_AUTO, tol=1e-10,
                             restart=a.serve_restart)
    service, errs = [], []
    for i, (si, kind, q) in enumerate(run):
        qd = torch.as_tensor(q, device="cuda")
        s0 = time.perf_counter()
        f = bie2d.bie_elastance_solve if kind == 0 else bie2d.bie_mobility_solve
        ref, _ = f(geoms[si], qd, o64)
        ref = ref.cpu().numpy()
        service.append(time.perf_counter() - s0)
        errs.append(float(np.abs(outs[i] - ref).max() / np.abs(ref).max()))
    fin, lat64 = 0.0, []
    for i in range(len(run)):
        fin = max(arrivals[i], fin) + service[i]
        lat64.append(fin - arrivals[i])
    res = {
        "metric": "served solves/s and p50/p99 latency (continuous batching), elastance and "
                  "mobility queries, <=1e-9 rel err vs float64",
        "value": len(run) / wall, "unit": "solves/s", "n_gpus": 1,
        "steps": len(run), "warmup": warm, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32+f64", "data": "synthetic (seeded sessions)",
        "config": {"workload": "serving: Poisson queries, 60/40 elastance/mobility, 2-500 bodies "
                               "x 64-256 nodes, 1-16 queries per resident geometry, method auto "
                               "(FMM above 32768 nodes), mixed precision, tol 1e-10",
                   "offered_rate_per_s": rate, "saturation_rate_per_s": sat,
                   "saturation_backlog": len(sample), "geometries": len(sessions),
                   "restart": a.serve_restart, "precond": a.precond},
        "latency_s": {"p50": pct(lat, 0.5), "p99": pct(lat, 0.99), "mean": float(np.mean(lat))},
        "sweep": sweep,
        "plain_fp64_gpu": {"service_s_mean": float(np.mean(service)),
                           "throughput_solves_per_s": len(run) / float(np.sum(service)),
                           "latency_s": {"p50": pct(lat64, 0.5), "p99": pct(lat64, 0.99)}},
        "max_rel_err_vs_fp64": max(errs), "all_ok": all(x == 0 for x in statuses),
        "server": st,
    }
    print(json.dumps(res))


def batched_bench(a):
    from paper_1507_05925_amd import bie2d
    from paper_1507_05925_amd import workloads as wl
    import torch

    geoms = wl.batched_geometries()
    items = [(bie2d.Geometry.from_curves(c), 0 if k == "elastance" else 1, None) for k, c in geoms]
    b = bie2d.Batch()
    runs = {}
    pcs = [("precond", bie2d.BIE_PRECOND_BLOCK)] if a.precond == "block" else []
    for name, pc in pcs + [("unpreconditioned", bie2d.BIE_PRECOND_NONE)]:
        o = bie2d.default_opts(precision=bie2d.BIE_MIXED, tol=1e-10, restart=40, max_iter=3000,
                               precond=pc)
        torch.cuda.synchronize()
        t = time.perf_counter()
        outs, info, rel = bie2d.bie_batch_solve(b, items, o)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t
        systems = sum(x.shape[0] for x in outs)
        runs[name] = {"seconds": dt, "solves_per_s": systems / dt, "systems": systems,
                      "pair_interactions_per_s": info["pairs"] / dt,
                      "gmres": {k: info[k] for k in ("iters", "refinements", "applies_fp32",
                                                     "applies_fp64")},
                      "max_rel_residual": float(rel.max())}
    best = runs[pcs[0][0]] if pcs else runs["unpreconditioned"]
    print(json.dumps({
        "metric": "solves/s (pair-interactions/s, M^2 per apply per rhs, alongside), batched P "
                  "and M of 32 geometries", "value": best["solves_per_s"], "unit": "solves/s",
        "n_gpus": 1, "steps": 1, "warmup": 0, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32+f64", "data": "synthetic (seeded ensemble)",
        "config": {"workload": "32 geometries, 8-128 bodies, 64-512 nodes per body, identity "
                               "rhs blocks (P or M), mixed precision, tol 1e-10",
                   "precond": a.precond},
        **best, "runs": runs}))


def nanocomposite_bench(a):
    """The paper's nanocomposite table on the GPU: float64, method auto, GMRES tol 1e-10;
    geometry resident, one untimed solve first (builds the FMM tree where used), then the
    median of 5 timed solves."""
    import numpy as np
    import torch

    from paper_1507_05925_amd import bie2d
    from paper_1507_05925_amd import workloads as wl

    rows = json.load(open(os.path.join(ROOT, "tests", "golden", "nanocomposite_table3.json")))["rows"]
    out, total_t = [], 0.0
    for r in rows:
        c, q = wl.nanocomposite(r["m"], r["A"] if r["A"] is not None else 1.0)
        g = bie2d.Geometry.from_curves(c)
        qd = torch.as_tensor(q[None], device="cuda")
        o = bie2d.default_opts(precision=bie2d.BIE_FP64, method=bie2d.BIE_AUTO, tol=1e-10,
                               restart=100)
        bie2d.bie_elastance_solve(g, qd, o)
        ts = []
        for _ in range(5):
            torch.cuda.synchronize()
            t = time.perf_counter()
            phi, info = bie2d.bie_elastance_solve(g, qd, o)
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t)
        phi = phi.cpu().numpy()[0]
        C = 1.0 / (phi[0] - phi[1])
        t = float(np.median(ts))
        total_t += t
        out.append({"m": r["m"], "A": r["A"], "N_pts": int(c.M), "C": C, "C_paper": r["C"],
                    "abs_diff": abs(C - r["C"]), "iters": info["iters"], "t_solve_s": t,
                    "t_solve_paper_s": r["t_solve"], "paper_over_ours": r["t_solve"] / t})
        g.close()
    print(json.dumps({
        "metric": "solves/s over the nanocomposite capacitance table (16 configurations)",
        "value": len(out) / total_t, "unit": "solves/s", "n_gpus": 1, "steps": len(out),
        "warmup": 1, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "the paper's geometry (plates and particle lattice), synthetic charges +-1",
        "config": {"workload": "nanocomposite capacitance, m = 0, 1, 4, 16 rows of 10 particles, "
                               "A = 0.25..4, 800 nodes per plate, 600 per particle, method auto, "
                               "tol 1e-10"},
        "max_abs_diff_vs_paper_C": max(x["abs_diff"] for x in out), "rows": out}))


def mobility_bench(a):
    """Mobility of 200 rigid ellipses x 512 nodes (204,800 unknowns), FMM, GMRES tol 1e-10, in
    float64 and in the mixed mode (for Stokes the late GMRES steps apply an FMM of about half the
    order, still in float64): geometry resident, warm-up solves, then `steps` timed solves per
    mode; (v, omega) compared with the stored float64 oracle solution."""
    import numpy as np
    import torch

    from paper_1507_05925_amd import bie2d
    from paper_1507_05925_amd import workloads as wl

    torch.cuda.set_device(0)
    curves, FT = wl.mobility_ellipses()
    g = bie2d.Geometry.from_curves(curves)
    ft = torch.as_tensor(FT[None], device="cuda")
    gold = os.path.join(ROOT, "tests", "golden", "ellipses_200x512_vw.json")
    ref = np.asarray(json.load(open(gold))["VW"]).reshape(-1, 3) if os.path.exists(gold) else None
    runs = {}
    pc = bie2d.BIE_PRECOND_BLOCK if a.precond == "block" else bie2d.BIE_PRECOND_NONE
    cases = [("fp64", bie2d.BIE_FP64, pc), ("mixed", bie2d.BIE_MIXED, pc)]
    if pc != bie2d.BIE_PRECOND_NONE:  # the paper's plain GMRES beside it
        cases.append(("mixed_unpreconditioned", bie2d.BIE_MIXED, bie2d.BIE_PRECOND_NONE))
    for name, prec, pcn in cases:
        o = bie2d.default_opts(precision=prec, method=bie2d.BIE_FMM, tol=a.tol, restart=100,
                               max_iter=2000, mixed_strategy=MIXED_STRATEGY[a.mixed_strategy],
                               fmm_leaf=a.fmm_leaf, fmm_eps=a.fmm_eps, fmm_order=a.fmm_order,
                               precond=pcn)
        for _ in range(max(a.warmup, 1)):
            bie2d.bie_mobility_solve(g, ft, o)
        torch.cuda.synchronize()
        lat, pairs = [], 0
        t0 = time.perf_counter()
        for _ in range(a.steps):
            s = time.perf_counter()
            VW, info = bie2d.bie_mobility_solve(g, ft, o)
            lat.append(time.perf_counter() - s)
            pairs += info["pairs"]
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        r = {"solves_per_s": a.steps / el, "ms_per_solve": 1e3 * el / a.steps,
             "pair_interactions_per_s": pairs / el, "p50_s": pct(lat, 0.5), "p99_s": pct(lat, 0.99),
             "gmres": {k: info[k] for k in ("iters", "refinements", "applies_fp32", "applies_fp64",
                                            "rel_residual")}}
        if ref is not None:
            v = VW.cpu().numpy()[0].reshape(-1, 3)
            r["rel_err_v_vs_fp64_oracle"] = float(np.abs(v[:, :2] - ref[:, :2]).max()
                                                  / np.abs(ref[:, :2]).max())
            r["rel_err_omega_vs_fp64_oracle"] = float(np.abs(v[:, 2] - ref[:, 2]).max()
                                                      / np.abs(ref[:, 2]).max())
        runs[name] = r
    # the float64 FMM kernels timed with HIP events over one more solve, each class in a
    # solve of its own: the M2L (three charge sets per right-hand side) and the Stokes near field
    o = bie2d.default_opts(precision=bie2d.BIE_FP64, method=bie2d.BIE_FMM, tol=a.tol, restart=100,
                           max_iter=2000, fmm_leaf=a.fmm_leaf, fmm_eps=a.fmm_eps,
                           fmm_order=a.fmm_order)
    terms = bie2d.bie_fmm_terms(o, 1, bie2d.BIE_FP64)
    rls = {}
    for key, kc, flops, bound, kern in (
            ("roofline_m2l", bie2d.BIE_K_FMM_M2L, m2l_flops_per_entry(terms), "mfma",
             f"k_m2l<{terms}>"),
            ("roofline_near", bie2d.BIE_K_FMM_EVAL, FLOPS_PER_PAIR_STOKES, "alu", "k_near<true>")):
        bie2d.bie_profile_select([kc])
        bie2d.bie_profile_enable(True)
        bie2d.bie_mobility_solve(g, ft, o)
        torch.cuda.synchronize()
        # (kernel=None: the committed traffic counters were taken on the elastance workload)
        rl = roofline(bie2d.bie_profile_read(kc), kc, flops, "f64", bound=bound, kernel=None)
        rl["kernel"] = kern
        rls[key] = rl
        bie2d.bie_profile_enable(False)
    bie2d.bie_profile_select(None)
    leaf = a.fmm_leaf if a.fmm_leaf > 0 else \
        "autotuned (float64 %d, mixed %d)" % bie2d.bie_autotune(g, 1, bie2d.BIE_MIXED)
    g.close()
    best = max((k for k in runs if k in ("fp64", "mixed")), key=lambda k: runs[k]["solves_per_s"])
    print(json.dumps({
        "metric": "solves/s of full mobility solves (pair-interactions/s, equivalent direct M^2 "
                  "node pairs per operator apply, alongside)",
        "value": runs[best]["solves_per_s"], "unit": "solves/s",
        "pair_interactions_per_s": runs[best]["pair_interactions_per_s"],
        "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
        "ms_per_step": runs[best]["ms_per_solve"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None,
        # the mixed Stokes FMM: float64 expansions, float32 near field and float64 refinement
        "dtype": "f32+f64" if best == "mixed" else "f64",
        "data": "synthetic (seeded ellipse ensemble, F ~ N(0,1)^2 with zero total, T ~ N(0,1))",
        "config": {"workload": "mobility, 200 ellipses (aspect 1..3, gaps >= 0.2) x 512 nodes "
                               "(204,800 unknowns), FMM, GMRES tol %g" % a.tol,
                   "fastest": best, "fmm_eps": a.fmm_eps, "precond": a.precond,
                   "fmm_terms": {"fp64": terms, "mixed": bie2d.bie_fmm_terms(o, 1, bie2d.BIE_MIXED)},
                   "fmm_leaf": leaf},
        "runs": runs, **rls}))


def crosstest_bench(a):
    """The paper's cross-tests on the GPU: prescribed potentials (rigid motions) -> capacitance
    (resistance) solve -> elastance (mobility) solve with the resulting charges (forces, torques)
    -> the prescribed data up to u_inf. Cases: two discs at gaps 0.5, 0.05, 0.005 (256, 1024,
    6144 nodes per disc) and the five splash curves (1024 nodes each), float64 direct, GMRES tol
    1e-12. One untimed round, then the median of 5 timed rounds per case."""
    import numpy as np
    import torch

    from paper_1507_05925_amd import bie2d
    from paper_1507_05925_amd import workloads as wl

    tab = json.load(open(os.path.join(ROOT, "tests", "golden", "two_disc_tables.json")))
    spl = json.load(open(os.path.join(ROOT, "tests", "golden", "splash_prescribed.json")))
    cases = [(f"two discs d={d}", wl.two_discs(d, n), [tab["elastance"]["phi1"], tab["elastance"]["phi2"]],
              [*tab["mobility"]["v_body1"], tab["mobility"]["omega1"], *tab["mobility"]["v_body2"],
               tab["mobility"]["omega2"]]) for d, n in ((0.5, 256), (0.05, 1024), (0.005, 6144))]
    cases.append(("splash", wl.splash(1024), spl["phi"],
                  list(np.stack([spl["v1"], spl["v2"], spl["omega"]], 1).reshape(-1))))
    o = bie2d.default_opts(precision=bie2d.BIE_FP64, method=bie2d.BIE_DIRECT, tol=1e-12,
                           restart=300, max_iter=3000)
    bie2d.bie_profile_enable(True)
    out, total_t, nsolves = [], 0.0, 0
    for name, c, phi, VW in cases:
        g = bie2d.Geometry.from_curves(c)
        phid = torch.as_tensor(np.array(phi)[None], device="cuda")
        vwd = torch.as_tensor(np.array(VW)[None], device="cuda")

        def rounds():
            q, ui, i1 = bie2d.bie_capacitance_solve(g, phid, o, allow_noconv=True)
            back, i2 = bie2d.bie_elastance_solve(g, q, o, allow_noconv=True)
            FT, uv, i3 = bie2d.bie_resistance_solve(g, vwd, o, allow_noconv=True)
            bm, i4 = bie2d.bie_mobility_solve(g, FT, o, allow_noconv=True)
            return q, ui, back, FT, uv, bm, (i1, i2, i3, i4)

        rounds()
        ts = []
        for _ in range(5):
            torch.cuda.synchronize()
            t = time.perf_counter()
            q, ui, back, FT, uv, bm, infos = rounds()
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t)
        t = float(np.median(ts))
        total_t += t
        nsolves += 4
        e_phi = float(np.abs(back.cpu().numpy()[0] + float(ui.cpu().numpy()[0]) - np.array(phi)).max())
        want = np.array(VW).reshape(-1, 3).copy()
        want[:, 0:2] -= uv.cpu().numpy()[0][None, :]
        e_vw = float(np.abs(bm.cpu().numpy()[0].reshape(-1, 3) - want).max())
        out.append({"case": name, "M": int(c.M), "seconds_per_round": t,
                    "iters": [i["iters"] for i in infos],
                    "rel_residual": [i["rel_residual"] for i in infos],
                    "max_err_potential": e_phi, "max_err_rigid_motion": e_vw,
                    "u_inf_laplace": float(ui.cpu().numpy()[0]),
                    "u_inf_stokes": [float(v) for v in uv.cpu().numpy()[0]]})
        g.close()
    pr = bie2d.bie_profile_read(bie2d.BIE_K_DOUBLE_LAYER)
    n, ms, pairs = pr["launches"], pr["ms_total"], pr["pairs"]
    print(json.dumps({
        "metric": "solves/s of the paper's cross-tests (capacitance + elastance, resistance + "
                  "mobility; two discs at three gaps and the splash curves)",
        "value": nsolves / total_t, "unit": "solves/s", "n_gpus": 1, "steps": 5, "warmup": 1,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "the paper's geometries and prescribed data",
        "config": {"workload": "cross-tests: two discs d = 0.5, 0.05, 0.005 (256, 1024, 6144 "
                               "nodes per disc), splash (5 x 1024), float64 direct, tol 1e-12"},
        "double_layer_applies": {"launches": n, "ms_total": ms, "pairs": pairs,
                                 "pairs_per_s": pairs / (ms * 1e-3) if ms > 0 else None},
        "max_err_potential": max(x["max_err_potential"] for x in out),
        "max_err_rigid_motion": max(x["max_err_rigid_motion"] for x in out),
        "cases": out}))


def copy_bench(a):
    import torch

    n = 1 << 25  # 2^25 doubles = 256 MiB read + 256 MiB written per copy
    x = torch.ones(n, dtype=torch.float64, device="cuda:0")
    y = torch.empty_like(x)
    # an elementwise kernel (not a DMA blit), so the counters see an ordinary dispatch
    torch.neg(x, out=y)
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(5):
        torch.neg(x, out=y)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t) / 5
    print(json.dumps({"metric": "device copy bandwidth", "value": 2 * 8 * n / dt / 1e9,
                      "unit": "GB/s", "bytes_read_per_copy": 8 * n, "bytes_written_per_copy": 8 * n,
                      "copies": 6}))


def main():
    a = parse()
    if a.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU; --gpus N > 1 is not "
                                   "supported (one-GPU build, no collectives)"}))
        sys.exit(2)
    if a.workload == "serve":
        return serve_bench(a)
    if a.workload == "batched":
        return batched_bench(a)
    if a.workload == "copy":
        return copy_bench(a)
    if a.workload == "crosstest":
        return crosstest_bench(a)
    if a.workload == "nanocomposite":
        return nanocomposite_bench(a)
    if a.workload == "mobility":
        return mobility_bench(a)
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
    precision = a.precision or "mixed"
    prec = bie2d.BIE_MIXED if precision == "mixed" else bie2d.BIE_FP64
    pc = bie2d.BIE_PRECOND_BLOCK if a.precond == "block" else bie2d.BIE_PRECOND_NONE
    opts = bie2d.default_opts(precision=prec, method=meth, tol=a.tol, restart=100, max_iter=2000,
                              mixed_strategy=MIXED_STRATEGY[a.mixed_strategy],
                              fmm_leaf=a.fmm_leaf, fmm_eps=a.fmm_eps, fmm_order=a.fmm_order,
                              precond=pc)

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

    order = bie2d.bie_fmm_terms(opts, 0, bie2d.BIE_FP64)  # expansion terms, float64 applies
    order32 = bie2d.bie_fmm_terms(opts, 0, bie2d.BIE_MIXED)  # and float32 ones
    classes = {  # class, algorithmic flops per unit, dtype, bound, kernel name in the profiles
        "k_lap_far_f32": (bie2d.BIE_K_FAR_LAPLACE_F32, FLOPS_PER_PAIR, "f32", "alu",
                          "k_lap_far_f32<1>"),
        "k_lap_far_f64": (bie2d.BIE_K_FAR_LAPLACE_F64, FLOPS_PER_PAIR, "f64", "alu",
                          "k_lap_far_f64<1>"),
        "k_m2l": (bie2d.BIE_K_FMM_M2L, m2l_flops_per_entry(order), "f64", "mfma", f"k_m2l<{order}>"),
        "k_near": (bie2d.BIE_K_FMM_EVAL, FLOPS_PER_PAIR, "f64", "alu", "k_near<false>"),
        "k_m2l_f32": (bie2d.BIE_K_FMM_M2L_F32, m2l_flops_per_entry(order32), "f32", "mfma",
                      f"k_m2l_fac_f32<{order32}>"),
        "k_near_f32": (bie2d.BIE_K_FMM_NEAR_F32, FLOPS_PER_PAIR, "f32", "alu", "k_near_f32<false>"),
        "k_lap_epilogue": (bie2d.BIE_K_EPILOGUE, 0, "f64", "alu", "k_lap_epilogue"),
    }
    # one untimed solve with every class recorded picks the dominant kernel class; the timed
    # solves then record events around that class only (events around every class would add
    # their own cost to the timed region)
    bie2d.bie_profile_enable(True)
    bie2d.bie_elastance_solve(g, q_d, opts)
    profs = {k: bie2d.bie_profile_read(v[0]) for k, v in classes.items()}
    fmm_total = bie2d.bie_profile_read(bie2d.BIE_K_FMM)
    bie2d.bie_profile_enable(False)
    dom = max((k for k in classes if classes[k][1] > 0), key=lambda k: profs[k]["ms_total"])
    c = classes[dom]
    torch.cuda.synchronize()

    # events around every 8th launch of that class only: each event marker leaves the stream idle
    # for a few microseconds, which would otherwise lengthen the timed solves
    bie2d.bie_profile_select([c[0]])
    bie2d.bie_profile_sample(PROFILE_EVERY)
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
    rl = roofline(bie2d.bie_profile_read(c[0]), c[0], c[1], c[2], bound=c[3], kernel=c[4])
    rl["kernel"] = c[4]
    rl["sampled_every"] = PROFILE_EVERY
    bie2d.bie_profile_enable(False)
    bie2d.bie_profile_sample(1)
    # the matrix-core kernels (M2L, float64 and, in mixed solves, float32) on their own, from one
    # more solve that times only those classes
    rl_m2ls = {}
    for name in ("k_m2l", "k_m2l_f32"):
        cm = classes[name]
        bie2d.bie_profile_select([cm[0]])
        bie2d.bie_profile_enable(True)
        bie2d.bie_elastance_solve(g, q_d, opts)
        pr = bie2d.bie_profile_read(cm[0])
        bie2d.bie_profile_enable(False)
        if pr["launches"] > 0:
            rl_m2ls[name] = roofline(pr, cm[0], cm[1], cm[2], bound=cm[3], kernel=cm[4])
            rl_m2ls[name]["kernel"] = cm[4]
    # the preconditioner apply (two-grid blocks): algorithmic bytes = the float32 coarse
    # inverses (U^2 entries per body, U = the coarse node count: n up to 64, else the largest
    # divisor of n not above 64) and the float64 vector in and out
    rl_pre = None
    if pc != bie2d.BIE_PRECOND_NONE:
        bie2d.bie_profile_select([bie2d.BIE_K_PRECOND])
        bie2d.bie_profile_enable(True)
        bie2d.bie_elastance_solve(g, q_d, opts)
        pr = bie2d.bie_profile_read(bie2d.BIE_K_PRECOND)
        bie2d.bie_profile_enable(False)
        ms = pr["ms_total"] / max(pr["launches"], 1)
        coarse = lambda n: n if n <= 64 else max(d for d in range(16, 65) if n % d == 0)
        nbytes = sum(4.0 * coarse(int(n)) ** 2 for n in curves.nodes_per_body) + 16.0 * g.M
        ach = nbytes / (ms * 1e-3) / 1e9 if ms > 0 else 0.0
        kern = "k_pc_apply<512>"
        rl_pre = {"bound": "hbm", "achieved": ach, "peak": 8000.0, "unit": "GB/s",
                  "frac": ach / 8000.0, "traffic": traffic_bytes(kern), "avg_launch_ms": ms,
                  "launches": pr["launches"], "multiply_adds_per_launch": pr["pairs"] /
                  max(pr["launches"], 1), "bytes_per_launch": nbytes, "kernel": kern}
    bie2d.bie_profile_select(None)

    # where a solve's time goes: the FMM applies of each precision timed on their own (events on
    # the stream), times the counts of the timed solve, and the rest (Arnoldi, read-off, host)
    breakdown = None
    if meth == bie2d.BIE_FMM:
        mu_t = torch.randn(1, g.M, dtype=torch.float64, device=dev)
        ms_apply = {}
        for name, pr in (("fp64", bie2d.BIE_FP64), ("fp32", bie2d.BIE_MIXED)):
            bie2d.bie_laplace_apply(g, mu_t, pr, bie2d.BIE_FMM)
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(20):
                bie2d.bie_laplace_apply(g, mu_t, pr, bie2d.BIE_FMM)
            e1.record()
            torch.cuda.synchronize()
            ms_apply[name] = e0.elapsed_time(e1) / 20
        ms_solve = 1e3 * elapsed / a.steps
        n64, n32 = info["applies_fp64"], info["applies_fp32"]

        def apply_flops(near, m2l, order_):
            u = lambda k: profs[k]["pairs"] / max(profs[k]["launches"], 1)  # units per launch
            return u(near) * FLOPS_PER_PAIR + u(m2l) * m2l_flops_per_entry(order_)
        fl64 = apply_flops("k_near", "k_m2l", order) if profs["k_near"]["launches"] else None
        fl32 = apply_flops("k_near_f32", "k_m2l_f32", order32) if profs["k_near_f32"]["launches"] else None
        breakdown = {
            "ms_per_solve": ms_solve,
            "applies_fp64": n64, "apply_fp64_ms": ms_apply["fp64"],
            "applies_fp32": n32, "apply_fp32_ms": ms_apply["fp32"],
            "applies_ms": n64 * ms_apply["fp64"] + n32 * ms_apply["fp32"],
            **({"precond_applies": rl_pre["launches"],
                "precond_ms": rl_pre["launches"] * rl_pre["avg_launch_ms"]} if rl_pre else {}),
            "arnoldi_readoff_host_ms": ms_solve - n64 * ms_apply["fp64"] - n32 * ms_apply["fp32"]
            - (rl_pre["launches"] * rl_pre["avg_launch_ms"] if rl_pre else 0.0),
            "whole_apply_near_plus_m2l_flops": {
                "note": "algorithmic near-field and M2L flops of one apply over the whole apply's "
                        "time (P2M, M2M, evaluation and epilogue flops not counted)",
                **({"fp64_tflops": fl64 / (ms_apply["fp64"] * 1e-3) / 1e12,
                    "fp64_frac_of_78.6": fl64 / (ms_apply["fp64"] * 1e-3) / 1e12 / PEAK["f64"]}
                   if fl64 else {}),
                **({"fp32_tflops": fl32 / (ms_apply["fp32"] * 1e-3) / 1e12,
                    "fp32_frac_of_157.3": fl32 / (ms_apply["fp32"] * 1e-3) / 1e12 / PEAK["f32"]}
                   if fl32 else {}),
            },
        }

    # the same solves without the preconditioner (the paper's plain GMRES), for comparison
    unpre = None
    if pc != bie2d.BIE_PRECOND_NONE:
        onp = bie2d.default_opts(precision=prec, method=meth, tol=a.tol, restart=100,
                                 max_iter=2000, mixed_strategy=MIXED_STRATEGY[a.mixed_strategy],
                                 fmm_leaf=a.fmm_leaf, fmm_eps=a.fmm_eps, fmm_order=a.fmm_order)
        bie2d.bie_elastance_solve(g, q_d, onp)
        torch.cuda.synchronize()
        tn = time.perf_counter()
        for _ in range(a.steps):
            _, info_n = bie2d.bie_elastance_solve(g, q_d, onp)
        torch.cuda.synchronize()
        unpre = {"ms_per_solve": 1e3 * (time.perf_counter() - tn) / a.steps,
                 "gmres": {k: info_n[k] for k in ("iters", "applies_fp32", "applies_fp64")}}

    # the plain float64 GPU path on the same solves, for comparison with the mixed solves
    fp64 = None
    if prec == bie2d.BIE_MIXED:
        o64 = bie2d.default_opts(precision=bie2d.BIE_FP64, method=meth, tol=a.tol, restart=100,
                                 max_iter=2000, fmm_leaf=a.fmm_leaf, fmm_eps=a.fmm_eps,
                                 fmm_order=a.fmm_order, precond=pc)
        for _ in range(max(a.warmup, 1)):
            bie2d.bie_elastance_solve(g, q_d, o64)
        torch.cuda.synchronize()
        t64 = time.perf_counter()
        for _ in range(a.steps):
            phi64_, info64_ = bie2d.bie_elastance_solve(g, q_d, o64)
        torch.cuda.synchronize()
        el64 = time.perf_counter() - t64
        fp64 = {"ms_per_solve": 1e3 * el64 / a.steps, "solves_per_s": a.steps / el64,
                "gmres": {k: info64_[k] for k in ("iters", "applies_fp64", "rel_residual")},
                "mixed_speedup": el64 / elapsed}

    # the same solves replaying captured HIP graphs of every Arnoldi step (the timed solves
    # above launch each step's kernels on the stream, the library default)
    bie2d.bie_set_graphs(True)
    bie2d.bie_elastance_solve(g, q_d, opts)  # captures the steps
    torch.cuda.synchronize()
    t_g = time.perf_counter()
    for _ in range(a.steps):
        bie2d.bie_elastance_solve(g, q_d, opts)
    torch.cuda.synchronize()
    ms_graph = 1e3 * (time.perf_counter() - t_g) / a.steps
    captured, replayed = g.graph_stats()
    bie2d.bie_set_graphs(False)
    ms_stream = 1e3 * elapsed / a.steps
    graphs = {"ms_per_solve_stream_launch": ms_stream, "ms_per_solve_graph_replay": ms_graph,
              "arnoldi_steps_per_solve": info["iters"],
              "us_per_step_graph_minus_stream": 1e3 * (ms_graph - ms_stream) / max(info["iters"], 1),
              "steps_captured": captured, "steps_replayed": replayed}

    # the direct float32 far-field sweep on the same workload, 5 applies
    mu = torch.randn(1, g.M, dtype=torch.float64, device=dev)
    bie2d.bie_laplace_apply(g, mu, bie2d.BIE_MIXED, bie2d.BIE_DIRECT)
    torch.cuda.synchronize()
    bie2d.bie_profile_enable(True)
    for _ in range(5):
        bie2d.bie_laplace_apply(g, mu, bie2d.BIE_MIXED, bie2d.BIE_DIRECT)
    torch.cuda.synchronize()
    p32 = bie2d.bie_profile_read(bie2d.BIE_K_FAR_LAPLACE_F32)
    bie2d.bie_profile_enable(False)
    rl_direct = roofline(p32, bie2d.BIE_K_FAR_LAPLACE_F32, FLOPS_PER_PAIR, "f32",
                         kernel="k_lap_far_f32<1>")
    rl_direct["kernel"] = "k_lap_far_f32<1>"

    acc = {}
    gold = os.path.join(ROOT, "tests", "golden", "starfish_1000x256_phi.json")
    if os.path.exists(gold):
        ref = np.asarray(json.load(open(gold))["phi"])
        acc["rel_err_vs_fp64_oracle"] = float(np.abs(phi.cpu().numpy()[0] - ref).max() / np.abs(ref).max())
        if fp64 is not None:
            fp64["rel_err_vs_fp64_oracle"] = float(
                np.abs(phi64_.cpu().numpy()[0] - ref).max() / np.abs(ref).max())
    phi64, info64 = bie2d.bie_elastance_solve(
        g, q_d, bie2d.default_opts(precision=bie2d.BIE_FP64, method=bie2d.BIE_DIRECT, tol=1e-12,
                                   restart=100))
    acc["rel_err_vs_fp64_direct_gpu"] = float((phi - phi64).abs().max() / phi64.abs().max())
    acc["fp64_direct_gpu_solve_seconds"] = info64["seconds"]

    lat_sorted = sorted(lat)
    label = "equivalent direct " if meth == bie2d.BIE_FMM else ""
    # value: solves/s (a preconditioner that saves applies shows there; pair-interactions/s,
    # which counts M^2 per apply however few applies a solve needs, is reported beside it)
    res = {
        "metric": "solves/s of full elastance solves to <=1e-9 rel err vs float64 "
                  "(pair-interactions/s and p50/p99 latency alongside)",
        "value": a.steps / elapsed,
        "unit": "solves/s",
        "pair_interactions_per_s": pairs / elapsed,
        "pair_interactions_note": f"{label}M^2 per operator apply",
        "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
        "ms_per_step": 1e3 * elapsed / a.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32+f64" if prec == bie2d.BIE_MIXED else "f64",
        "data": "synthetic (seeded starfish ensemble, q ~ N(0,1))",
        "config": {"workload": "elastance, 1000 starfish r0(1+0.3cos5t) x 256 nodes (M=256000), "
                               "q~N(0,1), 2D FMM at <= 1e-10, GMRES tol 1e-10",
                   "method": a.method, "precision": precision, "fmm_eps": a.fmm_eps,
                   "fmm_terms": {"fp64": order, "mixed": order32}, "precond": a.precond,
                   "fmm_leaf": a.fmm_leaf if a.fmm_leaf > 0 else
                   "autotuned (float64 %d, mixed %d)" % bie2d.bie_autotune(g, 0, prec),
                   **({"mixed_strategy": a.mixed_strategy} if prec == bie2d.BIE_MIXED else {}),
                   "nodes": curves.M, "bodies": curves.nbodies},
        "solves_per_s": a.steps / elapsed,
        "latency_s": {"p50": lat_sorted[len(lat) // 2],
                      "p99": lat_sorted[min(len(lat) - 1, int(0.99 * len(lat)))]},
        "setup_s": {"geometry": t_geom, "first_solve_incl_tree": t_first},
        "gmres": {k: info[k] for k in ("iters", "refinements", "applies_fp32", "applies_fp64",
                                       "rel_residual")},
        "accuracy": acc,
        "roofline": rl,
        **({"roofline_m2l": rl_m2ls["k_m2l"]} if "k_m2l" in rl_m2ls else {}),
        **({"roofline_m2l_f32": rl_m2ls["k_m2l_f32"]} if "k_m2l_f32" in rl_m2ls else {}),
        **({"roofline_precond": rl_pre} if rl_pre else {}),
        "roofline_direct_p2p": rl_direct,
        **({"fp64_path": fp64} if fp64 is not None else {}),
        **({"unpreconditioned": unpre} if unpre is not None else {}),
        **({"solve_breakdown": breakdown} if breakdown is not None else {}),
        "kernel_ms_per_solve_untimed": {k: v["ms_total"] for k, v in profs.items()},
        "fmm_ms_per_apply": fmm_total["ms_total"] / max(fmm_total["launches"], 1),
        "graphs": graphs,
    }
    if not a.no_cpu_baseline:
        ref_gm = (unpre or {"gmres": info})["gmres"]
        n_app = ref_gm["applies_fp32"] + ref_gm["applies_fp64"] + 1  # + the right-hand side
        res["cpu_baseline"] = cpu_baseline(curves, a.cpu_seconds, n_app)
    g.close()
    print(json.dumps(res))


if __name__ == "__main__":
    main()
