"""GPU: nearly touching bodies through resolution (the two-disc tests at the paper's smallest gap,
d = 0.005). With equispaced trapezoidal nodes the error falls geometrically in the node count
(about 250x per 1024 nodes per disc at this gap, measured with the oracle); 6144 nodes per disc
(12,288 unknowns; 24,576 for Stokes) reach the exact bipolar solution to 1e-10 and the printed
table rows to their digits. The paper reaches this gap with panels and near-singular quadrature
instead."""
import json
import math
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_1507_05925_amd import bie2d  # noqa: E402
from paper_1507_05925_amd import workloads as wl  # noqa: E402

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs the GPU")]
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
D, NODES = 0.005, 6144


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64), device="cuda")


def test_two_discs_gap_0005_elastance():
    g = bie2d.Geometry.from_curves(wl.two_discs(D, NODES))
    o = bie2d.default_opts(tol=1e-13, restart=200, max_iter=2000)
    tab = json.load(open(os.path.join(GOLDEN, "two_disc_tables.json")))["elastance"]
    q_tab = -2 * math.pi * tab["rows"][2]["q1"]  # printed q1 = -q / (2 pi)
    phi, info = bie2d.bie_elastance_solve(g, dev([[1.0, -1.0], [q_tab, -q_tab]]), o)
    phi = phi.cpu().numpy()
    al = math.sqrt(D + D * D / 4)
    exact = math.log((D / 2 + al) / (al - D / 2)) / math.pi  # bipolar solution, unit charges
    assert abs((phi[0, 0] - phi[0, 1]) - exact) < 1e-10, info
    dphi = tab["phi1"] - tab["phi2"]
    assert abs((phi[1, 0] - phi[1, 1]) - dphi) / dphi < 3e-6


def test_two_discs_gap_0005_mobility():
    g = bie2d.Geometry.from_curves(wl.two_discs(D, NODES))
    o = bie2d.default_opts(tol=1e-13, restart=300, max_iter=5000)
    tab = json.load(open(os.path.join(GOLDEN, "two_disc_tables.json")))["mobility"]
    row = tab["rows"][2]
    FT = [row["F11"], row["F21"], row["T1"], -row["F11"], -row["F21"], row["T2"]]
    VW, info = bie2d.bie_mobility_solve(g, dev([FT]), o)
    VW = VW.cpu().numpy()[0]
    dv = np.array(tab["v_body1"]) - np.array(tab["v_body2"])
    got = VW[0:2] - VW[3:5]
    assert np.abs(got - dv).max() / np.abs(dv).max() < 5e-6, (got, dv, info)
    assert abs(VW[2] - tab["omega1"]) < 2e-5 and abs(VW[5] - tab["omega2"]) < 2e-5, (VW, info)


@pytest.mark.parametrize("precision,tol", [(bie2d.BIE_FP64, 1e-10), (bie2d.BIE_MIXED, 1e-9)])
def test_two_discs_gap_0005_mobility_vs_oracle(precision, tol):
    """(v, omega) at gap 0.005 against the stored float64 oracle solution of the same discrete
    system (tests/golden/two_discs_0005_vw.json, oracle/matfree only): the table row's forces and
    torques, a seeded (F, T) with net force, and the squeeze pair F_1 = -F_2."""
    gold = json.load(open(os.path.join(GOLDEN, "two_discs_0005_vw.json")))
    g = bie2d.Geometry.from_curves(wl.two_discs(D, NODES))
    o = bie2d.default_opts(precision=precision, tol=1e-13, restart=300, max_iter=6000,
                           max_refine=30)
    VW, info = bie2d.bie_mobility_solve(g, dev(gold["inputs"]), o)
    VW = VW.cpu().numpy()
    for k, ref in enumerate(gold["VW"]):
        ref = np.array(ref)
        err = float(np.abs(VW[k] - ref).max() / np.abs(ref).max())
        assert err < tol, (k, err, info)
