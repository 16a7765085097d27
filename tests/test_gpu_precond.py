"""GPU: the block right preconditioner (opts.precond = BIE_PRECOND_BLOCK; exact blocks for bodies
of at most 64 nodes, two-grid blocks beyond) leaves the solution unchanged (against the float64
oracle and against the unpreconditioned solves), for elastance and mobility, and cuts the GMRES
steps on multi-body problems; it is refused where it does not apply (bodies it cannot coarsen,
the capacitance and resistance solves)."""
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


def rel(a, b):
    a = a.cpu().numpy() if hasattr(a, "cpu") else np.asarray(a)
    return float(np.abs(a - b).max() / np.abs(b).max())


@pytest.mark.parametrize("precision,tol", [(bie2d.BIE_FP64, 1e-10), (bie2d.BIE_MIXED, 1e-9)])
def test_precond_small_vs_oracle(precision, tol):
    c, q = wl.elastance_small()
    g = bie2d.Geometry.from_curves(c)
    geo = ny.geometry_of(c)
    rng = np.random.default_rng(41)
    Q = np.vstack([q, rng.standard_normal((2, geo["N"]))])
    ref = ny.elastance_solve(geo, Q)
    o = bie2d.default_opts(precision=precision, precond=bie2d.BIE_PRECOND_BLOCK, tol=1e-12)
    phi, info, mu = bie2d.bie_elastance_solve(g, dev(Q), o, want_mu=True)
    assert rel(phi, ref["phi"]) < tol, info
    assert rel(mu, ref["mu"]) < 100 * tol, info
    P, _ = bie2d.bie_elastance_matrix(g, max_rhs=4, opts=o)
    assert rel(P, ny.elastance_matrix(geo)) < tol


@pytest.mark.parametrize("precision,tol", [(bie2d.BIE_FP64, 1e-10), (bie2d.BIE_MIXED, 1e-9)])
@pytest.mark.parametrize("n", [48, 192])
def test_precond_mobility_small_vs_oracle(precision, tol, n):
    """Four ellipses: exact blocks (48 nodes) and two-grid blocks (192 nodes, 64 coarse)."""
    c, FT = wl.mobility_ellipses(nbodies=4, n=n)
    g = bie2d.Geometry.from_curves(c)
    geo = ny.geometry_of(c)
    rng = np.random.default_rng(43)
    X = np.vstack([FT, rng.standard_normal((2, 3 * geo["N"]))])
    ref = ny.mobility_solve(geo, X)
    o = bie2d.default_opts(precision=precision, precond=bie2d.BIE_PRECOND_BLOCK, tol=1e-12)
    VW, info, mu = bie2d.bie_mobility_solve(g, dev(X), o, want_mu=True)
    assert rel(VW, ref["VW"]) < tol, info
    assert rel(mu, ref["mu"]) < 100 * tol, info
    Mm, _ = bie2d.bie_mobility_matrix(g, max_rhs=5, opts=o)
    assert rel(Mm, ny.mobility_matrix(geo)) < tol


@pytest.mark.parametrize("precision,tol", [(bie2d.BIE_FP64, 1e-10), (bie2d.BIE_MIXED, 1e-9)])
def test_precond_elastance_two_grid_vs_oracle(precision, tol):
    """Six starfish of 320 nodes: two-grid blocks on 64 coarse nodes (every fifth)."""
    c, q = wl.elastance_starfish(nbodies=6, n=320)
    g = bie2d.Geometry.from_curves(c)
    geo = ny.geometry_of(c)
    rng = np.random.default_rng(47)
    Q = np.vstack([q, rng.standard_normal((2, geo["N"]))])
    ref = ny.elastance_solve(geo, Q)
    o = bie2d.default_opts(precision=precision, precond=bie2d.BIE_PRECOND_BLOCK, tol=1e-12)
    phi, info, mu = bie2d.bie_elastance_solve(g, dev(Q), o, want_mu=True)
    assert rel(phi, ref["phi"]) < tol, info
    assert rel(mu, ref["mu"]) < 100 * tol, info
    base = bie2d.default_opts(precision=precision, tol=1e-12)
    _, i0 = bie2d.bie_elastance_solve(g, dev(Q), base)
    assert info["iters"] < i0["iters"], (info, i0)


@pytest.mark.parametrize("kind", [0, 1])
@pytest.mark.parametrize("precision,tol", [(bie2d.BIE_FP64, 1e-10), (bie2d.BIE_MIXED, 1e-9)])
def test_precond_uneven_bodies_vs_oracle(kind, precision, tol):
    """Every block regime in one geometry: exact blocks of 16, 40 and 64 nodes, two-grid blocks of
    66 nodes (33 coarse, every second), 100 nodes (50 coarse) and 2048 nodes (64 coarse, every
    32nd: the largest body the apply stages); for mobility the blocks of more than 32 coarse nodes
    take the 128-wide layout."""
    rng = np.random.default_rng(53)
    c = wl.mixed_grid(rng, 6, np.array([16, 40, 64, 66, 100, 2048]))
    g = bie2d.Geometry.from_curves(c)
    geo = ny.geometry_of(c)
    width = geo["N"] if kind == 0 else 3 * geo["N"]
    X = rng.standard_normal((2, width))
    ref = (ny.elastance_solve if kind == 0 else ny.mobility_solve)(geo, X)
    key = "phi" if kind == 0 else "VW"
    o = bie2d.default_opts(precision=precision, precond=bie2d.BIE_PRECOND_BLOCK, tol=1e-12)
    solve = bie2d.bie_elastance_solve if kind == 0 else bie2d.bie_mobility_solve
    out, info = solve(g, dev(X), o)
    assert rel(out, ref[key]) < tol, info


@pytest.mark.parametrize("method", [bie2d.BIE_DIRECT, bie2d.BIE_FMM])
def test_precond_same_solution_fewer_steps(method):
    """100 starfish of 256 nodes (gap >= 0.3; two-grid blocks on 64 nodes): the same potentials
    as without the preconditioner, in at most half the GMRES steps (34 -> 11 measured with exact
    blocks and the oracle)."""
    c, q = wl.elastance_starfish(nbodies=100)
    g = bie2d.Geometry.from_curves(c)
    qd = dev(q[None])
    base = bie2d.default_opts(method=method, tol=1e-11)
    phi0, i0 = bie2d.bie_elastance_solve(g, qd, base)
    pre = bie2d.default_opts(method=method, tol=1e-11, precond=bie2d.BIE_PRECOND_BLOCK)
    phi1, i1 = bie2d.bie_elastance_solve(g, qd, pre)
    assert float((phi1 - phi0).abs().max() / phi0.abs().max()) < 1e-10, (i0, i1)
    assert i1["rel_residual"] < 1e-11 and 2 * i1["iters"] <= i0["iters"], (i0, i1)
    # mixed precision keeps the solution too
    pm = bie2d.default_opts(method=method, tol=1e-11, precond=bie2d.BIE_PRECOND_BLOCK,
                            precision=bie2d.BIE_MIXED)
    phi2, i2 = bie2d.bie_elastance_solve(g, qd, pm)
    assert float((phi2 - phi0).abs().max() / phi0.abs().max()) < 1e-9, i2
    assert i2["rel_residual"] < 1e-11


@pytest.mark.parametrize("method", [bie2d.BIE_DIRECT, bie2d.BIE_FMM])
def test_precond_mobility_fewer_steps(method):
    """40 ellipses of 256 nodes (two-grid blocks on 64 nodes): the same rigid motions, in at
    most half the steps (55 -> 17 measured with the oracle on 20 such ellipses)."""
    c, FT = wl.mobility_ellipses(nbodies=40, n=256)
    g = bie2d.Geometry.from_curves(c)
    x = dev(FT[None])
    base = bie2d.default_opts(method=method, tol=1e-11)
    v0, i0 = bie2d.bie_mobility_solve(g, x, base)
    pre = bie2d.default_opts(method=method, tol=1e-11, precond=bie2d.BIE_PRECOND_BLOCK)
    v1, i1 = bie2d.bie_mobility_solve(g, x, pre)
    assert float((v1 - v0).abs().max() / v0.abs().max()) < 1e-9, (i0, i1)
    assert i1["rel_residual"] < 1e-11 and 2 * i1["iters"] <= i0["iters"], (i0, i1)


def test_precond_refused_where_it_does_not_apply():
    o = bie2d.default_opts(precond=bie2d.BIE_PRECOND_BLOCK)
    # 257 nodes: more than 64 and no divisor in [16, 64]
    odd = bie2d.Geometry.from_curves(wl.two_discs(0.5, 257))
    with pytest.raises(bie2d.BieError) as e:
        bie2d.bie_elastance_solve(odd, dev([[1.0, -1.0]]), o)
    assert e.value.code == bie2d.BIE_EINVAL and "divisor" in str(e.value)
    big = bie2d.Geometry.from_curves(wl.two_discs(0.5, 4096))
    with pytest.raises(bie2d.BieError) as e:
        bie2d.bie_mobility_solve(big, dev([[1.0, 0.0, 0.0, -1.0, 0.0, 0.0]]), o)
    assert e.value.code == bie2d.BIE_EINVAL and "2048" in str(e.value)
    c, _ = wl.elastance_small()
    g = bie2d.Geometry.from_curves(c)
    with pytest.raises(bie2d.BieError) as e:
        bie2d.bie_capacitance_solve(g, dev(np.ones((1, g.N))), o)
    assert e.value.code == bie2d.BIE_EINVAL and "elastance and mobility" in str(e.value)


def precond_batch():
    """Geometries whose every body the preconditioner takes (node counts with a divisor in
    [16, 64] past 64 nodes): exact blocks, two-grid blocks and a mix of both."""
    rng = np.random.default_rng(23)
    return [("elastance", wl.elastance_small()[0]),
            ("mobility", wl.mixed_grid(rng, 5, np.array([64, 96, 32, 130, 256]))),
            ("elastance", wl.splash(128)),
            ("mobility", wl.two_discs(0.5, 96)),
            ("elastance", wl.mixed_grid(rng, 9, np.full(9, 64)))]


@pytest.mark.parametrize("precision,tol", [(bie2d.BIE_FP64, 1e-10), (bie2d.BIE_MIXED, 1e-9)])
def test_precond_batch_matrices_vs_oracle(precision, tol):
    items, refs = [], []
    for kind, c in precond_batch():
        geo = ny.geometry_of(c)
        items.append((bie2d.Geometry.from_curves(c), 0 if kind == "elastance" else 1, None))
        refs.append(ny.elastance_matrix(geo) if kind == "elastance" else ny.mobility_matrix(geo))
    o = bie2d.default_opts(precision=precision, tol=1e-12, restart=120, max_iter=3000,
                           precond=bie2d.BIE_PRECOND_BLOCK)
    outs, info, rel = bie2d.bie_batch_solve(bie2d.Batch(), items, o)
    for out, r in zip(outs, refs):
        assert rel_err(out, r) < tol, info
    assert (rel <= 1e-12).all()
    base = bie2d.default_opts(precision=precision, tol=1e-12, restart=120, max_iter=3000)
    _, info0, _ = bie2d.bie_batch_solve(bie2d.Batch(), items, base)
    assert info["iters"] < info0["iters"], (info, info0)


def rel_err(a, b):
    return float(np.abs(a.cpu().numpy() - b).max() / np.abs(b).max())


@pytest.mark.parametrize("precision", [bie2d.BIE_FP64, bie2d.BIE_MIXED])
def test_precond_batch_alone_and_in_the_mix(precision):
    """Each item's preconditioned result is bitwise the same alone and in the mix, and equals
    the single-geometry preconditioned solve to rounding."""
    rng = np.random.default_rng(24)
    items = []
    for kind, c in precond_batch():
        g = bie2d.Geometry.from_curves(c)
        k = 0 if kind == "elastance" else 1
        width = g.N if k == 0 else 3 * g.N
        items.append((g, k, dev(rng.standard_normal((int(rng.integers(1, 4)), width)))))
    o = bie2d.default_opts(precision=precision, tol=1e-12, restart=120, max_iter=3000,
                           precond=bie2d.BIE_PRECOND_BLOCK)
    b = bie2d.Batch()
    mix, _, _ = bie2d.bie_batch_solve(b, items, o)
    for it, m in zip(items, mix):
        alone, _, _ = bie2d.bie_batch_solve(b, [it], o)
        assert torch.equal(alone[0], m)
    g, k, inp = items[1]
    vw, _ = bie2d.bie_mobility_solve(g, inp, o)
    assert float((vw - mix[1]).abs().max() / vw.abs().max()) < 1e-10


@pytest.mark.parametrize("kind", [0, 1])
@pytest.mark.parametrize("precision", [bie2d.BIE_FP64, bie2d.BIE_MIXED])
def test_zero_rhs_among_others(kind, precision):
    """A zero right-hand side among others (its first GMRES cycle runs on a zero vector before the
    norms of f reach the host): its result is exactly zero, the others match the oracle, with and
    without the preconditioner."""
    c, data = wl.elastance_small() if kind == 0 else wl.mobility_ellipses(nbodies=4, n=64)
    g = bie2d.Geometry.from_curves(c)
    geo = ny.geometry_of(c)
    rng = np.random.default_rng(59)
    width = geo["N"] if kind == 0 else 3 * geo["N"]
    X = np.vstack([rng.standard_normal((1, width)), np.zeros((1, width)),
                   rng.standard_normal((1, width))])
    key = "phi" if kind == 0 else "VW"
    ref = (ny.elastance_solve if kind == 0 else ny.mobility_solve)(geo, X[[0, 2]])[key]
    solve = bie2d.bie_elastance_solve if kind == 0 else bie2d.bie_mobility_solve
    tol = 1e-10 if precision == bie2d.BIE_FP64 else 1e-9
    for pc in (bie2d.BIE_PRECOND_NONE, bie2d.BIE_PRECOND_BLOCK):
        o = bie2d.default_opts(precision=precision, precond=pc, tol=1e-12)
        out, info = solve(g, dev(X), o)
        out = out.cpu().numpy()
        assert np.all(out[1] == 0.0), (pc, np.abs(out[1]).max())
        assert rel(out[[0, 2]], ref) < tol, (pc, info)
