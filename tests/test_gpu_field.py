"""GPU: off-surface evaluation of the solution (the representation formulas). Everywhere the field
matches the float64 oracle's layer potential of its own total density (1e-10). Inside body j the
elastance field is the constant phi_j and the mobility velocity the rigid motion
v_j + omega_j (p - x^c_j)^perp (the theorems after eqs. IntEqConstraints and the Stokes analogue),
up to the discretisation error of the curves (checked at 1e-7 for the potential and 1e-4 for the
velocity: the 128-node ellipses resolve the Stokes problem to about 2e-5)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import nystrom as ny  # noqa: E402
from paper_1507_05925_amd import bie2d  # noqa: E402
from paper_1507_05925_amd import workloads as wl  # noqa: E402

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs the GPU")]


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64), device="cuda")


def points(c, geo, rng):
    """Interior points (at most 0.35 of the way from the centroid to the curve: well inside, where
    the trapezoidal sums need no near-boundary correction) with their body, and
    exterior points at least 0.3 from every node."""
    inner, body = [], []
    for j in range(geo["N"]):
        k = np.arange(c.body_ptr[j], c.body_ptr[j + 1])
        pick = rng.choice(k, 4, replace=False)
        t = rng.uniform(0.05, 0.35, 4)[:, None]
        xc = geo["xc"][j]
        inner.append(xc + t * (np.stack([geo["x"][pick], geo["y"][pick]], 1) - xc))
        body += [j] * 4
    lo = np.array([geo["x"].min(), geo["y"].min()]) - 1.0
    hi = np.array([geo["x"].max(), geo["y"].max()]) + 1.0
    cand = rng.uniform(lo, hi, (4000, 2))
    d = np.hypot(cand[:, :1] - geo["x"][None], cand[:, 1:] - geo["y"][None]).min(1)
    # outside every body: not closer to a centroid than that body's nearest node
    out = cand[d > 0.3][:200]
    inside = np.zeros(len(out), bool)
    for j in range(geo["N"]):
        k = np.arange(c.body_ptr[j], c.body_ptr[j + 1])
        rmin = np.hypot(geo["x"][k] - geo["xc"][j, 0], geo["y"][k] - geo["xc"][j, 1]).min()
        inside |= np.hypot(out[:, 0] - geo["xc"][j, 0], out[:, 1] - geo["xc"][j, 1]) < rmin
    return np.concatenate(inner), np.array(body), out[~inside]


@pytest.mark.parametrize("name", ["ellipses", "splash"])
def test_elastance_field(name):
    rng = np.random.default_rng(41)
    c = wl.elastance_small()[0] if name == "ellipses" else wl.splash(256)
    geo = ny.geometry_of(c)
    g = bie2d.Geometry.from_curves(c)
    q = rng.standard_normal((2, geo["N"]))
    o = bie2d.default_opts(tol=1e-13, restart=200)
    phi, info, mu = bie2d.bie_elastance_solve(g, dev(q), o, want_mu=True)
    pin, body, pout = points(c, geo, rng)
    ref = ny.elastance_solve(geo, q)
    dens = ref["mu"] + ny.incident_charge(geo, q)
    for pts in (pin, pout):
        u = bie2d.bie_elastance_field(g, dev(q), mu, dev(pts)).cpu().numpy()
        uref = np.stack([ny.single_layer(geo, d, pts) for d in dens])
        assert np.abs(u - uref).max() / np.abs(uref).max() < 1e-10
    u_in = bie2d.bie_elastance_field(g, dev(q), mu, dev(pin)).cpu().numpy()
    ph = phi.cpu().numpy()
    assert np.abs(u_in - ph[:, body]).max() / np.abs(ph).max() < 1e-7


@pytest.mark.parametrize("name", ["ellipses", "splash"])
def test_mobility_field(name):
    rng = np.random.default_rng(42)
    c = wl.elastance_small()[0] if name == "ellipses" else wl.splash(256)
    geo = ny.geometry_of(c)
    g = bie2d.Geometry.from_curves(c)
    FT = rng.standard_normal((1, 3 * geo["N"]))
    o = bie2d.default_opts(tol=1e-13, restart=300)
    VW, info, mu = bie2d.bie_mobility_solve(g, dev(FT), o, want_mu=True)
    pin, body, pout = points(c, geo, rng)
    ref = ny.mobility_solve(geo, FT)
    dens = (ref["mu"] + ny.incident_traction(geo, FT))[0]
    for pts in (pin, pout):
        u = bie2d.bie_mobility_field(g, dev(FT), mu, dev(pts)).cpu().numpy()[0]
        uref = ny.stokes_single_layer(geo, dens, pts)
        assert np.abs(u - uref).max() / np.abs(uref).max() < 1e-10
    u_in = bie2d.bie_mobility_field(g, dev(FT), mu, dev(pin)).cpu().numpy()[0]
    vw = VW.cpu().numpy()[0].reshape(-1, 3)
    e = pin - geo["xc"][body]
    rigid = vw[body, :2] + vw[body, 2:3] * np.stack([-e[:, 1], e[:, 0]], 1)
    assert np.abs(u_in - rigid).max() / np.abs(rigid).max() < 1e-4


def test_field_arguments():
    c = wl.elastance_small()[0]
    g = bie2d.Geometry.from_curves(c)
    q = dev(np.ones((1, g.N)))
    mu = dev(np.zeros((1, g.M)))
    out = bie2d.bie_elastance_field(g, q, mu, dev(np.zeros((0, 2))))
    assert out.shape == (1, 0)
    lib = bie2d.lib()
    code = lib.bie_elastance_field(g.handle, 1, bie2d._dptr(q), bie2d._dptr(mu), -1, None, None,
                                   bie2d._stream())
    assert code == bie2d.BIE_EINVAL
