"""GPU: the capacitance and resistance solvers (completed double layers) against the oracle, and
the paper's cross-tests on the GPU (capacitance then elastance, resistance then mobility) on the
two-disc and splash geometries.

Parity: the double-layer applies element by element against the oracle's dense operators, on a
ragged geometry (M = 1030: four 256-node tiles and a tail, four source splits) with 1, 3 and 9
(Laplace) or 1 and 5 (Stokes) densities, so every rhs chunk width runs; the solves (charges,
forces, torques, u_inf and densities) against the oracle's LU solves."""
import json
import math
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import dirichlet as dr  # noqa: E402
from oracle import nystrom as ny  # noqa: E402
from paper_1507_05925_amd import bie2d  # noqa: E402
from paper_1507_05925_amd import workloads as wl  # noqa: E402

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs the GPU")]
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64), device="cuda")


def _ragged():
    rng = np.random.default_rng(41)
    return wl.mixed_grid(rng, 5, np.array([200, 150, 333, 97, 250]))


def _opts(**kw):
    kw.setdefault("tol", 1e-13)
    kw.setdefault("restart", 100)
    kw.setdefault("max_iter", 2000)
    return bie2d.default_opts(**kw)


@pytest.mark.parametrize("nrhs", [1, 3, 9])
def test_laplace_dl_apply_parity(nrhs):
    curves = _ragged()
    geo = ny.geometry_of(curves)
    g = bie2d.Geometry.from_curves(curves)
    mu = np.random.default_rng(nrhs).standard_normal((nrhs, geo["M"]))
    A = dr.capacitance_operator(geo)
    ref = mu @ A.T
    got = bie2d.bie_laplace_dl_apply(g, dev(mu)).cpu().numpy()
    assert np.abs(got - ref).max() < 1e-12 * np.abs(ref).max()
    A0 = 0.5 * np.eye(geo["M"]) + dr.laplace_D(geo)
    got0 = bie2d.bie_laplace_dl_apply(g, dev(mu), with_completion=False).cpu().numpy()
    assert np.abs(got0 - mu @ A0.T).max() < 1e-12 * np.abs(ref).max()


@pytest.mark.parametrize("nrhs", [1, 5])
def test_stokes_dl_apply_parity(nrhs):
    curves = _ragged()
    geo = ny.geometry_of(curves)
    g = bie2d.Geometry.from_curves(curves)
    mu = np.random.default_rng(10 + nrhs).standard_normal((nrhs, 2 * geo["M"]))
    A = dr.resistance_operator(geo)
    ref = mu @ A.T
    got = bie2d.bie_stokes_dl_apply(g, dev(mu)).cpu().numpy()
    assert np.abs(got - ref).max() < 1e-12 * np.abs(ref).max()
    A0 = 0.5 * np.eye(2 * geo["M"]) + dr.stokes_D(geo)
    got0 = bie2d.bie_stokes_dl_apply(g, dev(mu), with_completion=False).cpu().numpy()
    assert np.abs(got0 - mu @ A0.T).max() < 1e-12 * np.abs(ref).max()


def test_capacitance_solve_parity():
    curves = _ragged()
    geo = ny.geometry_of(curves)
    g = bie2d.Geometry.from_curves(curves)
    phi = np.random.default_rng(3).standard_normal((3, geo["N"]))
    ref = dr.capacitance_solve(geo, phi)
    q, uinf, info, mu = bie2d.bie_capacitance_solve(g, dev(phi), _opts(), want_mu=True)
    q, uinf, mu = q.cpu().numpy(), uinf.cpu().numpy(), mu.cpu().numpy()
    assert np.abs(q - ref["q"]).max() < 1e-10 * np.abs(ref["q"]).max(), info
    assert np.abs(uinf - ref["u_inf"]).max() < 1e-10 * np.abs(phi).max()
    assert np.abs(mu - ref["mu"]).max() < 1e-10 * np.abs(ref["mu"]).max()
    assert np.abs(q.sum(1)).max() < 1e-12 * np.abs(q).max()


def test_resistance_solve_parity():
    curves = _ragged()
    geo = ny.geometry_of(curves)
    g = bie2d.Geometry.from_curves(curves)
    VW = np.random.default_rng(4).standard_normal((2, 3 * geo["N"]))
    ref = dr.resistance_solve(geo, VW)
    FT, uinf, info, mu = bie2d.bie_resistance_solve(g, dev(VW), _opts(), want_mu=True)
    FT, uinf, mu = FT.cpu().numpy(), uinf.cpu().numpy(), mu.cpu().numpy()
    assert np.abs(FT - ref["FT"]).max() < 1e-10 * np.abs(ref["FT"]).max(), info
    assert np.abs(uinf - ref["u_inf"]).max() < 1e-10 * np.abs(VW).max()
    assert np.abs(mu - ref["mu"]).max() < 1e-10 * np.abs(ref["mu"]).max()
    F = FT.reshape(2, -1, 3)[:, :, 0:2].sum(1)
    assert np.abs(F).max() < 1e-12 * np.abs(FT).max()


def _bipolar_dphi_per_charge(d):
    """Exact two-disc solution: charges +q, -q give phi_1 - phi_2 = (q/pi) log((x0 + alpha) /
    (alpha - x0)), alpha = sqrt(d + d^2/4), x0 = d/2."""
    al = math.sqrt(d + d * d / 4)
    return math.log((d / 2 + al) / (al - d / 2)) / math.pi


@pytest.mark.parametrize("row,n,tol", [(0, 256, 1e-11), (1, 1024, 1e-10), (2, 6144, 1e-9)])
def test_two_disc_capacitance_cross_test(row, n, tol):
    """The two-disc test end to end on the GPU: prescribed 0.209 / -0.123 -> capacitance solve
    (q against the exact bipolar solution and the printed q1; u_inf = (phi_1 + phi_2)/2) ->
    elastance solve with those charges -> the prescribed potentials up to u_inf."""
    tab = json.load(open(os.path.join(GOLDEN, "two_disc_tables.json")))["elastance"]
    r = tab["rows"][row]
    g = bie2d.Geometry.from_curves(wl.two_discs(r["d"], n))
    phi = np.array([tab["phi1"], tab["phi2"]])
    q, uinf, info = bie2d.bie_capacitance_solve(g, dev(phi[None]), _opts(restart=200))
    q, uinf = q.cpu().numpy()[0], float(uinf.cpu().numpy()[0])
    q_exact = (phi[0] - phi[1]) / _bipolar_dphi_per_charge(r["d"])
    assert abs(q[0] - q_exact) < tol * q_exact, (q, q_exact, info)
    assert abs(-q[0] / (2 * np.pi) - r["q1"]) < 3e-6 * abs(r["q1"])
    assert abs(uinf - 0.5 * (phi[0] + phi[1])) < tol
    back, info = bie2d.bie_elastance_solve(g, dev(q[None]), _opts(restart=200))
    assert np.abs(back.cpu().numpy()[0] + uinf - phi).max() < tol, info


@pytest.mark.parametrize("row,n", [(0, 256), (1, 1024), (2, 6144)])
def test_two_disc_resistance_cross_test(row, n):
    """Prescribed motions (read as v_{k,j}) -> resistance solve (the printed forces and torques
    to the table's accuracy) -> mobility solve -> the prescribed motions up to u_inf."""
    tab = json.load(open(os.path.join(GOLDEN, "two_disc_tables.json")))["mobility"]
    r = tab["rows"][row]
    g = bie2d.Geometry.from_curves(wl.two_discs(r["d"], n))
    VW = np.array([*tab["v_body1"], tab["omega1"], *tab["v_body2"], tab["omega2"]])
    FT, uinf, info = bie2d.bie_resistance_solve(g, dev(VW[None]), _opts(tol=1e-12, restart=300,
                                                                        max_iter=3000),
                                                allow_noconv=True)
    assert info["rel_residual"] < 1e-10, info
    FT, uinf = FT.cpu().numpy()[0], uinf.cpu().numpy()[0]
    assert abs(FT[0] - r["F11"]) < 1e-5 * abs(r["F11"]), (FT, info)
    assert abs(FT[1] - r["F21"]) < 1e-5 * abs(r["F21"]), FT
    assert abs(FT[2] - r["T1"]) < 5e-5 * abs(r["T1"]), FT
    assert abs(FT[5] - r["T2"]) < 5e-5 * abs(r["T2"]), FT
    back, info = bie2d.bie_mobility_solve(g, dev(FT[None]), _opts(restart=300, max_iter=5000))
    want = VW.reshape(2, 3).copy()
    want[:, 0:2] -= uinf[None, :]
    assert np.abs(back.cpu().numpy()[0].reshape(2, 3) - want).max() < 1e-8, info


def test_splash_cross_tests():
    """The splash tests end to end on the GPU with the printed potentials and rigid motions,
    1024 nodes per curve (the paper reports errors of about 1e-5 for its discretisation)."""
    s = json.load(open(os.path.join(GOLDEN, "splash_prescribed.json")))
    curves = wl.splash(1024)
    g = bie2d.Geometry.from_curves(curves)
    phi = np.array(s["phi"])
    q, uinf, info = bie2d.bie_capacitance_solve(g, dev(phi[None]), _opts())
    back, info2 = bie2d.bie_elastance_solve(g, q, _opts())
    err = np.abs(back.cpu().numpy()[0] + float(uinf.cpu().numpy()[0]) - phi).max()
    assert err < 1e-11, (err, info, info2)
    VW = np.stack([s["v1"], s["v2"], s["omega"]], 1).reshape(-1)
    FT, uinf, info = bie2d.bie_resistance_solve(g, dev(VW[None]), _opts())
    back, info2 = bie2d.bie_mobility_solve(g, FT, _opts())
    want = VW.reshape(5, 3).copy()
    want[:, 0:2] -= uinf.cpu().numpy()[0][None, :]
    err = np.abs(back.cpu().numpy()[0].reshape(5, 3) - want).max()
    assert err < 1e-10, (err, info, info2)


def test_dirichlet_argument_errors():
    g = bie2d.Geometry.from_curves(wl.two_discs(0.5, 64))
    x = dev(np.zeros((1, g.M)))
    with pytest.raises(bie2d.BieError):
        bie2d.bie_laplace_dl_apply(g, x, out=x)
    with pytest.raises(bie2d.BieError):
        bie2d.bie_capacitance_solve(g, dev(np.zeros((0, g.N))))
