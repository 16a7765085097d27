"""Write the full-size expected outputs used by the GPU parity tests.

Calls only oracle/ (matrix-free float64 apply + GMRES to 1e-13) on the seeded workloads of
paper_1507_05925_amd.workloads; nothing here comes from the HIP path.

  python tests/golden/make_golden.py starfish   # 1000 starfish x 256 nodes, q ~ N(0,1) -> phi
  python tests/golden/make_golden.py ellipses   # 200 ellipses x 512 nodes, (F, T) -> (v, omega)
  python tests/golden/make_golden.py batched    # columns of P / M of the largest batched geometries
  python tests/golden/make_golden.py fmm_items  # items above the FMM threshold of BIE_AUTO
  python tests/golden/make_golden.py near_touching  # two discs at gap 0.005, mobility
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

from oracle import matfree as mf  # noqa: E402
from oracle import nystrom as ny  # noqa: E402
from paper_1507_05925_amd import workloads as wl  # noqa: E402


def _dump(name, payload):
    path = os.path.join(HERE, name)
    with open(path, "w") as f:
        json.dump(payload, f, indent=1)
    print("wrote", path)


def starfish():
    g, q = wl.elastance_starfish()
    geo = ny.geometry_of(g)
    t = time.time()
    res = mf.elastance_solve(geo, q, tol=1e-13, restart=60, maxiter=10)
    mu = res["mu"]
    r = mf.laplace_apply(geo, mu) - res["f"]
    _dump("starfish_1000x256_phi.json", {
        "workload": "elastance, 1000 starfish r0(1+0.3cos5t) x 256 nodes, q ~ N(0,1)",
        "generator": "paper_1507_05925_amd.workloads.elastance_starfish()",
        "seed": wl.SEEDS["elastance_starfish"], "M": geo["M"], "N": geo["N"],
        "oracle": "oracle.matfree.elastance_solve (float64, GMRES rtol 1e-13)",
        "gmres_iters": res["iters"],
        "rel_residual": float(np.linalg.norm(r) / np.linalg.norm(res["f"])),
        "seconds": time.time() - t,
        "phi": [float(v) for v in res["phi"]],
        "body_charge_max": float(np.abs(ny.body_charge(geo, mu)).max()),
    })


def ellipses():
    g, FT = wl.mobility_ellipses()
    geo = ny.geometry_of(g)
    t = time.time()
    res = mf.mobility_solve(geo, FT, tol=1e-13, restart=80, maxiter=10)
    r = mf.stokes_apply(geo, res["mu"]) - res["f"]
    _dump("ellipses_200x512_vw.json", {
        "workload": "mobility, 200 ellipses AR~U[1,3] x 512 nodes, F ~ N(0,1)^2 zero-sum, T ~ N(0,1)",
        "generator": "paper_1507_05925_amd.workloads.mobility_ellipses()",
        "seed": wl.SEEDS["mobility_ellipses"], "M": geo["M"], "N": geo["N"],
        "oracle": "oracle.matfree.mobility_solve (float64, GMRES rtol 1e-13)",
        "gmres_iters": res["iters"],
        "rel_residual": float(np.linalg.norm(r) / np.linalg.norm(res["f"])),
        "seconds": time.time() - t,
        "VW": [float(v) for v in res["VW"]],
        "body_force_torque_max": float(np.abs(ny.body_force_torque(geo, res["mu"])).max()),
    })


def batched():
    """Columns of P (largest elastance geometry) and M (largest mobility geometry) of the
    32-geometry ensemble: unit charge on body 0; unit force (x) on body 0; unit torque on body 0."""
    geoms = wl.batched_geometries()
    out = {"workload": "32 geometries, 8-128 bodies, 64-512 nodes per body (batched ensemble)",
           "generator": "paper_1507_05925_amd.workloads.batched_geometries()",
           "seed": wl.SEEDS["batched"], "oracle": "oracle.matfree (float64, GMRES rtol 1e-13)",
           "columns": []}
    t = time.time()
    ie = max((i for i, (k, c) in enumerate(geoms) if k == "elastance"), key=lambda i: geoms[i][1].M)
    c = geoms[ie][1]
    geo = ny.geometry_of(c)
    q = np.zeros(c.nbodies)
    q[0] = 1.0
    r = mf.elastance_solve(geo, q, tol=1e-13, restart=100, maxiter=10)
    out["columns"].append({"geometry": ie, "kind": "elastance", "column": 0, "M": geo["M"],
                           "values": [float(v) for v in r["phi"]], "gmres_iters": r["iters"]})
    im = max((i for i, (k, c) in enumerate(geoms) if k == "mobility"), key=lambda i: geoms[i][1].M)
    c = geoms[im][1]
    geo = ny.geometry_of(c)
    for col in (0, 2):
        FT = np.zeros(3 * c.nbodies)
        FT[col] = 1.0
        r = mf.mobility_solve(geo, FT, tol=1e-13, restart=150, maxiter=10)
        out["columns"].append({"geometry": im, "kind": "mobility", "column": col, "M": geo["M"],
                               "values": [float(v) for v in r["VW"]], "gmres_iters": r["iters"]})
    out["seconds"] = time.time() - t
    _dump("batched_columns.json", out)


def fmm_items():
    """Outputs for the items of workloads.fmm_items() (two of them above the FMM threshold)."""
    out = {"workload": "130 starfish x 256 (2 q), 66 ellipses x 512 (2 (F, T)), 3 ellipses x 128 "
                       "(1 q), 5-body mixed grid (1 (F, T))",
           "generator": "paper_1507_05925_amd.workloads.fmm_items()",
           "seed": wl.SEEDS["fmm_items"], "oracle": "oracle.matfree (float64, GMRES rtol 1e-13)",
           "items": []}
    t = time.time()
    for kind, c, inputs in wl.fmm_items():
        geo = ny.geometry_of(c)
        vals, its = [], []
        for v in inputs:
            if kind == "elastance":
                r = mf.elastance_solve(geo, v, tol=1e-13, restart=100, maxiter=10)
                vals.append([float(x) for x in r["phi"]])
            else:
                r = mf.mobility_solve(geo, v, tol=1e-13, restart=150, maxiter=10)
                vals.append([float(x) for x in r["VW"]])
            its.append(r["iters"])
        out["items"].append({"kind": kind, "M": geo["M"], "N": geo["N"], "values": vals,
                             "gmres_iters": its})
        print(kind, geo["M"], its, time.time() - t)
    out["seconds"] = time.time() - t
    _dump("fmm_items.json", out)


def near_touching():
    """(v, omega) of the two unit discs at gap 0.005, 6144 nodes per disc, for the table row's
    forces and torques (two-disc mobility table) and the seeded vectors of
    workloads.near_touching_forces()."""
    tab = json.load(open(os.path.join(HERE, "two_disc_tables.json")))["mobility"]["rows"][2]
    c = wl.two_discs(0.005, 6144)
    geo = ny.geometry_of(c)
    inputs = [np.array([tab["F11"], tab["F21"], tab["T1"], -tab["F11"], -tab["F21"], tab["T2"]])]
    inputs += list(wl.near_touching_forces())
    t = time.time()
    vals, its, res = [], [], []
    for FT in inputs:
        r = mf.mobility_solve(geo, FT, tol=1e-13, restart=400, maxiter=10)
        rr = mf.stokes_apply(geo, r["mu"]) - r["f"]
        vals.append([float(x) for x in r["VW"]])
        its.append(r["iters"])
        res.append(float(np.linalg.norm(rr) / np.linalg.norm(r["f"])))
        print(its[-1], res[-1], time.time() - t)
    _dump("two_discs_0005_vw.json", {
        "workload": "mobility, two unit discs at gap 0.005, 6144 nodes per disc",
        "generator": "paper_1507_05925_amd.workloads.two_discs(0.005, 6144); inputs: the "
                     "two-disc mobility table row at d = 0.005, then "
                     "workloads.near_touching_forces()",
        "seed": wl.SEEDS["near_touching"], "oracle": "oracle.matfree.mobility_solve (float64, "
                                                      "GMRES rtol 1e-13)",
        "inputs": [[float(x) for x in v] for v in inputs], "VW": vals, "gmres_iters": its,
        "rel_residual": res, "seconds": time.time() - t})


if __name__ == "__main__":
    jobs = {"starfish": starfish, "ellipses": ellipses, "batched": batched,
            "fmm_items": fmm_items, "near_touching": near_touching}
    which = sys.argv[1:] or list(jobs)
    for w in which:
        jobs[w]()
