"""Write the full-size expected outputs used by the GPU parity tests.

Calls only oracle/ (matrix-free float64 apply + GMRES to 1e-13) on the seeded workloads of
paper_1507_05925_amd.workloads; nothing here comes from the HIP path.

  python tests/golden/make_golden.py starfish   # 1000 starfish x 256 nodes, q ~ N(0,1) -> phi
  python tests/golden/make_golden.py ellipses   # 200 ellipses x 512 nodes, (F, T) -> (v, omega)
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


if __name__ == "__main__":
    which = sys.argv[1:] or ["starfish", "ellipses"]
    for w in which:
        {"starfish": starfish, "ellipses": ellipses}[w]()
