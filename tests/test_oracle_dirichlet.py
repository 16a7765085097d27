"""Pins of the capacitance and resistance oracle (the Dirichlet companions the paper's numerical
section solves to test the elastance and mobility solvers), no GPU.

Kernel entries are checked against independent complex-variable forms and curve limits; the
double layers against their Gauss-law and rigid-motion identities; the solutions against the
exact two-disc solution, the two printed two-disc tables, single-disc closed forms, the paper's
cross-test (capacitance then elastance, resistance then mobility), independence from the
completion's length scale, and symmetry.
"""
import json
import math
import os

import numpy as np
import pytest

from oracle import dirichlet as dr
from oracle import nystrom as ny
from paper_1507_05925_amd import workloads as wl

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _geo(curves):
    return ny.geometry_of(curves)


def _mixed(seed=11, nbodies=4, n=64):
    rng = np.random.default_rng(seed)
    return wl.mixed_grid(rng, nbodies, np.full(nbodies, n))


# ------------------------------------------------------------------------------------------
# Entries
# ------------------------------------------------------------------------------------------

def test_laplace_double_layer_complex_form():
    """dG/dn_y (x, y) = (1/2pi) Re(n_y / (x - y)) in complex notation."""
    geo = _geo(_mixed())
    D = dr.laplace_D(geo)
    z = geo["x"] + 1j * geo["y"]
    n = geo["nx"] + 1j * geo["ny"]
    r = z[:, None] - z[None, :]
    np.fill_diagonal(r, 1.0)
    ref = (1 / (2 * np.pi)) * np.real(n[None, :] / r) * geo["w"][None, :]
    off = ~np.eye(geo["M"], dtype=bool)
    assert np.allclose(D[off], ref[off], rtol=1e-13, atol=1e-15)


def test_stokes_double_layer_complex_form():
    """(1/pi)(r.n_y)(r.mu) r / |r|^4 as a complex number equals
    (1/4pi) [conj(n) conj(mu) r / conj(r)^2 + (conj(n) mu + n conj(mu)) / conj(r) + n mu / r]
    with n the source normal."""
    geo = _geo(_mixed(seed=12))
    M = geo["M"]
    D = dr.stokes_D(geo)
    rng = np.random.default_rng(6)
    mu = rng.standard_normal(2 * M)
    Dd = D.reshape(M, 2, M, 2)
    idx = np.arange(M)
    diag = np.einsum("iab,ib->ia", Dd[idx, :, idx, :], mu.reshape(M, 2))
    out = (D @ mu).reshape(M, 2) - diag
    z = geo["x"] + 1j * geo["y"]
    n = (geo["nx"] + 1j * geo["ny"])[None, :]
    m = ((mu[0::2] + 1j * mu[1::2]) * geo["w"])[None, :]
    r = z[:, None] - z[None, :]
    np.fill_diagonal(r, 1.0)
    v = 0.25 * (np.conj(n) * np.conj(m) * r / np.conj(r) ** 2
                + (np.conj(n) * m + n * np.conj(m)) / np.conj(r) + n * m / r)
    np.fill_diagonal(v, 0.0)
    ref = (1 / np.pi) * v.sum(1)
    assert np.allclose(out[:, 0], ref.real, rtol=1e-12, atol=1e-13)
    assert np.allclose(out[:, 1], ref.imag, rtol=1e-12, atol=1e-13)


@pytest.mark.parametrize("t0", [0.3, 1.7, 4.0])
def test_double_layer_diagonal_limits(t0):
    """The diagonal entries equal the limit of the off-diagonal kernels as the source approaches
    the target along the curve (symmetric average over +-eps)."""
    def starfish(t):
        r0, a = 0.7, 0.3
        r = r0 * (1 + a * np.cos(5 * t))
        dr_ = -r0 * a * 5 * np.sin(5 * t)
        ddr = -r0 * a * 25 * np.cos(5 * t)
        return wl._radial(t, 0.2, -0.1, r, dr_, ddr, 0.4)

    for eps, tol in ((1e-3, 3e-5), (1e-4, 3e-7)):  # the gap closes as eps^2
        ts = np.array([t0 - eps, t0, t0 + eps])
        geo = ny.geometry(np.array([3]), *starfish(ts))
        D = dr.laplace_D(geo) / geo["w"][None, :]
        assert abs(0.5 * (D[1, 0] + D[1, 2]) - D[1, 1]) < tol * max(1.0, abs(D[1, 1]))
        Ds = (dr.stokes_D(geo) / np.repeat(geo["w"], 2)[None, :]).reshape(3, 2, 3, 2)
        lim = 0.5 * (Ds[1, :, 0, :] + Ds[1, :, 2, :])
        assert np.abs(lim - Ds[1, :, 1, :]).max() < tol * max(1.0, np.abs(Ds[1, :, 1, :]).max())


# ------------------------------------------------------------------------------------------
# Double-layer identities: D[1] = -1 inside, -1/2 on the curve, 0 outside; the Stokes double
# layer reproduces minus a rigid motion inside, half of it on the curve, zero outside
# ------------------------------------------------------------------------------------------

def test_laplace_double_layer_gauss_law():
    g, _ = wl.mobility_ellipses(5, 128, seed=7)
    geo = _geo(g)
    D = dr.laplace_D(geo)
    B = geo["body"]
    for b in range(geo["N"]):
        one = (B == b).astype(float)
        v = D @ one
        assert np.abs(v[B == b] + 0.5).max() < 1e-12
        assert np.abs(v[B != b]).max() < 1e-12
    inside = geo["xc"]
    outside = geo["xc"] + np.array([0.0, 50.0])
    for b in range(geo["N"]):
        one = (B == b).astype(float)
        assert abs(dr.double_layer(geo, one, inside[b])[0] + 1.0) < 1e-12
        assert abs(dr.double_layer(geo, one, outside[b])[0]) < 1e-12


def test_stokes_double_layer_rigid_motions():
    g, _ = wl.mobility_ellipses(4, 128, seed=8)
    geo = _geo(g)
    M, B = geo["M"], geo["body"]
    D = dr.stokes_D(geo)
    z = np.array([0.3, -0.7])  # any centre of rotation
    for b in range(geo["N"]):
        m = np.repeat(B == b, 2)
        for e in ([1.0, 0.0], [0.0, 1.0]):
            mu = np.tile(e, M) * m
            v = (D @ mu).reshape(M, 2)
            want = np.zeros((M, 2))
            want[B == b] = -0.5 * np.array(e)
            assert np.abs(v - want).max() < 1e-12
        rot = np.stack([-(geo["y"] - z[1]), geo["x"] - z[0]], 1)
        mu = (rot * (B == b)[:, None]).reshape(-1)
        v = (D @ mu).reshape(M, 2)
        want = np.zeros((M, 2))
        want[B == b] = -0.5 * rot[B == b]
        assert np.abs(v - want).max() < 1e-11


# ------------------------------------------------------------------------------------------
# Closed forms and the printed tables
# ------------------------------------------------------------------------------------------

def _bipolar_dphi_per_charge(d):
    """Exact two-disc solution (two-disc test): charges +q, -q give
    phi_1 - phi_2 = (q / pi) log((x0 + alpha) / (alpha - x0)), alpha = sqrt(d + d^2/4),
    x0 = d/2; and u_inf = (phi_1 + phi_2) / 2 (the constant v_2 of the exact solution)."""
    al = math.sqrt(d + d * d / 4)
    x0 = d / 2
    return math.log((x0 + al) / (al - x0)) / math.pi


@pytest.mark.parametrize("d,n,tol", [(0.5, 192, 1e-12), (0.05, 768, 1e-9)])
def test_capacitance_two_disc_exact(d, n, tol):
    geo = _geo(wl.two_discs(d, n))
    phi = np.array([0.209, -0.123])
    res = dr.capacitance_solve(geo, phi)
    q_exact = (phi[0] - phi[1]) / _bipolar_dphi_per_charge(d)
    assert abs(res["q"][0] - q_exact) < tol * q_exact
    assert abs(res["q"][0] + res["q"][1]) < 1e-12 * q_exact
    assert abs(res["u_inf"] - 0.5 * (phi[0] + phi[1])) < 1e-12


def _u_exact(d, phi, pts):
    """The two-disc test's exact exterior potential (bipolar solution):
    u_ex(x) = -(v1 / 2 pi) log(|x - (alpha, 0)| / |x + (alpha, 0)|) + v2 with
    alpha = sqrt(d + d^2/4), v1 = pi (phi2 - phi1) / log(|x0 + (alpha, 0)| / |x0 - (alpha, 0)|),
    v2 = (phi1 + phi2) / 2, x0 = (d/2, 0) (the printed "(d/2)" read as the point)."""
    al = math.sqrt(d + d * d / 4)
    x0 = d / 2
    v1 = math.pi * (phi[1] - phi[0]) / math.log((x0 + al) / (al - x0))
    p = np.asarray(pts, dtype=np.float64)
    rm = np.hypot(p[:, 0] - al, p[:, 1])
    rp = np.hypot(p[:, 0] + al, p[:, 1])
    return -(v1 / (2 * math.pi)) * np.log(rm / rp) + 0.5 * (phi[0] + phi[1])


@pytest.mark.parametrize("d,n,tol", [(0.5, 256, 1e-11), (0.05, 1024, 1e-9)])
def test_capacitance_field_two_disc_exact(d, n, tol):
    """capacitance_field at exterior points equals the exact two-disc potential: near the gap,
    above and below the discs, and far out (where it tends to u_inf = v2)."""
    geo = _geo(wl.two_discs(d, n))
    phi = np.array([0.209, -0.123])
    res = dr.capacitance_solve(geo, phi)
    c = 1.0 + d / 2
    pts = np.array([[0.0, 0.6], [0.0, -1.5], [-c, 1.4], [c + 1.3, 0.2], [-c - 1.5, -0.7],
                    [2.0, 2.0], [40.0, -30.0]])
    u = dr.capacitance_field(geo, res, pts)
    ue = _u_exact(d, phi, pts)
    assert np.abs(u - ue).max() < tol * np.abs(phi).max(), (u, ue)
    # a planted mistake: the double-layer term with the wrong sign misses by O(1e-2)
    wrong = -dr.double_layer(geo, res["mu"], pts) + (u - dr.double_layer(geo, res["mu"], pts))
    assert np.abs(wrong - ue).max() > 1e-3


def test_capacitance_field_double_layer_identity():
    """D[1] = -1 inside a curve and 0 outside (the discrete Gauss law through double_layer,
    the kernel capacitance_field evaluates), and capacitance_field of the uniform data on one
    disc is the constant datum everywhere outside (q = 0, u_inf = phi)."""
    geo = _geo(wl.two_discs(0.5, 256))
    body0 = (geo["body"] == 0).astype(float)
    inside = dr.double_layer(geo, body0, np.array([[-1.25, 0.3], [-1.0, -0.5]]))
    outside = dr.double_layer(geo, body0, np.array([[1.25, 0.0], [0.0, 3.0], [-4.0, 0.0]]))
    assert np.abs(inside + 1.0).max() < 1e-13 and np.abs(outside).max() < 1e-13
    one = _geo(wl.single_disc(128, R=0.7, cx=0.3, cy=-0.2))
    res = dr.capacitance_solve(one, [0.42])
    u = dr.capacitance_field(one, res, np.array([[1.5, 0.0], [0.3, 2.0], [-5.0, 4.0]]))
    assert np.abs(u - 0.42).max() < 1e-13


def test_capacitance_table1():
    """The capacitance solve with the prescribed 0.209 and -0.123 reproduces the printed q1
    (= -q / (2 pi)) to its six digits."""
    tab = json.load(open(os.path.join(GOLDEN, "two_disc_tables.json")))["elastance"]
    for row, n in zip(tab["rows"][:2], (256, 1024)):
        geo = _geo(wl.two_discs(row["d"], n))
        q = dr.capacitance_solve(geo, [tab["phi1"], tab["phi2"]])["q"]
        q1 = -q[0] / (2 * np.pi)
        assert abs(q1 - row["q1"]) < 3e-6 * abs(row["q1"])


def test_resistance_table2():
    """The resistance solve with the prescribed motions (velocity components read as v_{k,j})
    reproduces the printed forces to 1e-5 and torques to 5e-5 relative. The oracle's values are
    converged (768 and 1536 nodes per disc agree to 1e-10); the paper iterates to 1e-6 and
    reports velocity errors of about 1e-5."""
    tab = json.load(open(os.path.join(GOLDEN, "two_disc_tables.json")))["mobility"]
    VW = [*tab["v_body1"], tab["omega1"], *tab["v_body2"], tab["omega2"]]
    for row, n in zip(tab["rows"][:2], (256, 1024)):
        geo = _geo(wl.two_discs(row["d"], n))
        FT = dr.resistance_solve(geo, VW)["FT"]
        assert abs(FT[0] - row["F11"]) < 1e-5 * abs(row["F11"])
        assert abs(FT[1] - row["F21"]) < 1e-5 * abs(row["F21"])
        assert abs(FT[2] - row["T1"]) < 5e-5 * abs(row["T1"])
        assert abs(FT[5] - row["T2"]) < 5e-5 * abs(row["T2"])
        assert np.abs(FT[3:5] + FT[0:2]).max() < 1e-9 * abs(row["F11"])  # F_2 = -F_1


@pytest.mark.parametrize("n,R,c", [(3, 1.0, (0, 0)), (16, 0.7, (0.3, -0.2)), (64, 2.3, (5.0, 1.0))])
def test_single_disc_dirichlet(n, R, c):
    """One conductor held at phi: u = phi everywhere, q = 0, u_inf = phi. One cylinder moving
    rigidly: a bounded flow carries no net force, so u = v uniformly plus the rotlet of
    T = 4 pi R^2 omega."""
    geo = _geo(wl.single_disc(n, R, *c))
    res = dr.capacitance_solve(geo, [0.4])
    assert abs(res["q"][0]) < 1e-14 and abs(res["u_inf"] - 0.4) < 1e-14
    res = dr.resistance_solve(geo, [0.3, -0.2, 1.1])
    FT = res["FT"]
    assert np.abs(FT[0:2]).max() < 1e-13
    assert abs(FT[2] - 4 * np.pi * R * R * 1.1) < 1e-12 * FT[2]
    assert np.allclose(res["u_inf"], [0.3, -0.2], atol=1e-13)


# ------------------------------------------------------------------------------------------
# The paper's cross-tests, scale independence and symmetry
# ------------------------------------------------------------------------------------------

def test_cross_test_capacitance_elastance():
    """Prescribed potentials -> capacitance solve -> (q, u_inf) -> elastance solve: the
    potentials come back, up to u_inf (the elastance field is grounded at infinity)."""
    geo = _geo(_mixed(seed=31, nbodies=5, n=128))
    phi = np.random.default_rng(4).standard_normal(5)
    res = dr.capacitance_solve(geo, phi)
    assert abs(res["q"].sum()) < 1e-13
    back = ny.elastance_solve(geo, res["q"])["phi"]
    assert np.abs(back + res["u_inf"] - phi).max() < 1e-12


@pytest.mark.parametrize("shift", [None, (0.05, -0.03)])
def test_cross_test_resistance_mobility(shift):
    """Prescribed rigid motions -> resistance solve -> (F, T, u_inf) -> mobility solve: the
    motions come back, translations up to u_inf; also with completion centres z_j away from the
    centroids (torques are about the centroid)."""
    g, _ = wl.mobility_ellipses(4, 128, seed=9)
    geo = _geo(g)
    VW = np.random.default_rng(5).standard_normal(12)
    z = None if shift is None else geo["xc"] + np.array(shift)
    res = dr.resistance_solve(geo, VW, interior=z)
    FT = res["FT"].reshape(4, 3)
    assert np.abs(FT[:, 0:2].sum(0)).max() < 1e-12
    back = ny.mobility_solve(geo, res["FT"])["VW"].reshape(4, 3)
    want = VW.reshape(4, 3).copy()
    want[:, 0:2] -= res["u_inf"][None, :]
    assert np.abs(back - want).max() < 1e-11


def test_completion_scale_independent():
    """The bounded solution is unique. Changing the completion's length scale R adds a multiple
    of a rank-one term that the superposition removes exactly: q, F, T, u_inf and the densities
    agree to roundoff. Moving the completion centres z_j changes the discrete equations, so the
    outputs agree to the discretisation error (spectrally small at 160 nodes per body); the
    density itself depends on z_j (D[mu] = u - sum q_j G(., z_j) - u_inf)."""
    geo = _geo(_mixed(seed=32, nbodies=4, n=160))
    phi = np.array([0.5, -0.2, 0.1, 0.9])
    a = dr.capacitance_solve(geo, phi)
    b = dr.capacitance_solve(geo, phi, R=3.7 * dr.scale_length(geo))
    c = dr.capacitance_solve(geo, phi, interior=geo["xc"] + 0.02)
    for o in (b, c):
        assert np.abs(o["q"] - a["q"]).max() < 1e-13 * np.abs(a["q"]).max()
        assert abs(o["u_inf"] - a["u_inf"]) < 1e-13
    assert np.abs(b["mu"] - a["mu"]).max() < 1e-13
    VW = np.arange(12, dtype=float) / 7 - 0.8
    a = dr.resistance_solve(geo, VW)
    b = dr.resistance_solve(geo, VW, R=3.7 * dr.scale_length(geo))
    c = dr.resistance_solve(geo, VW, interior=geo["xc"] + 0.02)
    for o in (b, c):
        assert np.abs(o["FT"] - a["FT"]).max() < 1e-13 * np.abs(a["FT"]).max()
        assert np.abs(o["u_inf"] - a["u_inf"]).max() < 1e-13
    assert np.abs(b["mu"] - a["mu"]).max() < 1e-12


def test_capacitance_and_resistance_matrices():
    """C = C^T, C 1 = 0 (equal potentials carry no charge), phi^T C phi >= 0, and C P q = q for
    neutral q (C is the inverse of P on the neutral subspace); the resistance matrix is
    symmetric, positive semi-definite and vanishes on uniform translations."""
    geo = _geo(_mixed(seed=33, nbodies=4, n=128))
    C = dr.capacitance_matrix(geo)
    assert np.abs(C - C.T).max() < 1e-12 * np.abs(C).max()
    assert np.abs(C.sum(1)).max() < 1e-12 * np.abs(C).max()
    assert np.linalg.eigvalsh(0.5 * (C + C.T)).min() > -1e-12
    P = ny.elastance_matrix(geo)
    q = np.array([1.0, -0.3, 0.5, -1.2])
    assert np.abs(C @ P @ q - q).max() < 1e-11
    g, _ = wl.mobility_ellipses(3, 128, seed=10)
    geo = _geo(g)
    Rm = dr.resistance_matrix(geo)
    assert np.abs(Rm - Rm.T).max() < 1e-10 * np.abs(Rm).max()
    assert np.linalg.eigvalsh(0.5 * (Rm + Rm.T)).min() > -1e-10 * np.abs(Rm).max()
    for e in ([1, 0, 0] * 3, [0, 1, 0] * 3):
        assert np.abs(Rm @ np.array(e, float)).max() < 1e-11 * np.abs(Rm).max()


# ------------------------------------------------------------------------------------------
# Planted mistakes (in the oracle, on the CPU): the pins above must catch each
# ------------------------------------------------------------------------------------------

def test_planted_double_layer_diagonal_sign_is_caught(monkeypatch):
    orig = dr.laplace_D

    def wrong(geo):
        D = orig(geo)
        np.fill_diagonal(D, +geo["kappa"] * geo["w"] / (4 * np.pi))
        return D

    monkeypatch.setattr(dr, "laplace_D", wrong)
    with pytest.raises(AssertionError):
        test_laplace_double_layer_gauss_law()
    with pytest.raises(AssertionError):
        test_cross_test_capacitance_elastance()


def test_planted_dropped_rotlet_is_caught(monkeypatch):
    """Without the rotlet the rotations of each body stay in the null space of the operator."""
    orig = dr.stokes_completion

    def wrong(geo, interior=None, R=None):
        M = geo["M"]
        R = dr.scale_length(geo) if R is None else R
        C = orig(geo, interior, R).reshape(M, 2, M, 2)
        z = ny.interior_points(geo, interior)[geo["body"]]
        d1 = geo["x"][:, None] - z[None, :, 0]
        d2 = geo["y"][:, None] - z[None, :, 1]
        dd = d1 * d1 + d2 * d2
        s1, s2 = -(geo["y"] - z[:, 1]), geo["x"] - z[:, 0]
        w = geo["w"][None, :] / (4 * np.pi)
        C[:, 0, :, 0] -= w * (-d2) * s1[None, :] / dd
        C[:, 0, :, 1] -= w * (-d2) * s2[None, :] / dd
        C[:, 1, :, 0] -= w * d1 * s1[None, :] / dd
        C[:, 1, :, 1] -= w * d1 * s2[None, :] / dd
        return C.reshape(2 * M, 2 * M)

    monkeypatch.setattr(dr, "stokes_completion", wrong)
    with pytest.raises((AssertionError, np.linalg.LinAlgError)):
        test_cross_test_resistance_mobility(None)


def test_planted_torque_about_wrong_point_is_caught(monkeypatch):
    """Torques taken about the completion centre z_j instead of the centroid x^c_j disagree with
    the mobility problem's torque once z_j != x^c_j."""
    orig = dr.resistance_solve

    def wrong(geo, VW, interior=None, R=None, lu=None):
        res = orig(geo, VW, interior, R, lu)
        N = geo["N"]
        mom = res["moments_systems"]
        FT = res["FT"].reshape(-1, N, 3)
        beta = np.atleast_2d(res["u_inf"])
        t = mom[:-2, :, 2] - beta[:, 0, None] * mom[-2][None, :, 2] - beta[:, 1, None] * mom[-1][None, :, 2]
        FT[:, :, 2] = t
        res["FT"] = FT.reshape(res["FT"].shape)
        return res

    monkeypatch.setattr(dr, "resistance_solve", wrong)
    with pytest.raises(AssertionError):
        test_cross_test_resistance_mobility((0.05, -0.03))


def test_splash_cross_tests():
    """The paper's splash tests: the printed potentials and rigid motions of the five splash
    curves go through the capacitance (resistance) solve and back through the elastance
    (mobility) solve. The paper reports errors of about 1e-5 for its discretisation; the
    trapezoidal rule reaches 1e-12 at 512 nodes per curve (Laplace) and 1e-9 at 768 (Stokes)."""
    s = json.load(open(os.path.join(GOLDEN, "splash_prescribed.json")))
    geo = _geo(wl.splash(512))
    res = dr.capacitance_solve(geo, s["phi"])
    back = ny.elastance_solve(geo, res["q"])["phi"]
    assert np.abs(back + res["u_inf"] - np.array(s["phi"])).max() < 1e-12
    geo = _geo(wl.splash(768))
    VW = np.stack([s["v1"], s["v2"], s["omega"]], 1).reshape(-1)
    res = dr.resistance_solve(geo, VW)
    back = ny.mobility_solve(geo, res["FT"])["VW"].reshape(5, 3)
    want = VW.reshape(5, 3).copy()
    want[:, 0:2] -= res["u_inf"][None, :]
    assert np.abs(back - want).max() < 1e-9
