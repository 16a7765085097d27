"""GPU: solves that replay captured HIP graphs of their Arnoldi steps (the operator apply with
the FMM near field on a forked stream, and the Gram-Schmidt kernels) give bitwise the result of
the same solves run eagerly, on every replay, with other eager work and synchronisations in
between; a change of configuration (right-hand-side count, order) recaptures instead of
replaying stale graphs. One case is also checked against the float64 oracle."""
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


def solve(g, kind, inp, o):
    f = bie2d.bie_elastance_solve if kind == 0 else bie2d.bie_mobility_solve
    out, info = f(g, inp, o)
    return out, info


@pytest.mark.parametrize("method", [bie2d.BIE_FMM, bie2d.BIE_DIRECT])
@pytest.mark.parametrize("kind", [0, 1])
@pytest.mark.parametrize("precision", [bie2d.BIE_FP64, bie2d.BIE_MIXED])
def test_graph_replays_are_bitwise_eager(method, kind, precision):
    rng = np.random.default_rng(60 + kind)
    if method == bie2d.BIE_FMM:
        c = wl.elastance_starfish(nbodies=60)[0] if kind == 0 else wl.mobility_ellipses(nbodies=20, n=256)[0]
    else:
        c = wl.mixed_grid(rng, 6, np.array([64, 96, 128, 160, 64, 200]))
    g = bie2d.Geometry.from_curves(c)
    other = bie2d.Geometry.from_curves(wl.elastance_small()[0])
    width = g.N if kind == 0 else 3 * g.N
    inp = dev(rng.standard_normal((2, width)))
    o = bie2d.default_opts(method=method, precision=precision, tol=1e-11, restart=40)
    try:
        bie2d.bie_set_graphs(False)
        eager, info_e = solve(g, kind, inp, o)
        bie2d.bie_set_graphs(True)
        for rep in range(4):
            out, info = solve(g, kind, inp, o)
            torch.cuda.synchronize()
            assert torch.equal(out, eager), (rep, float((out - eager).abs().max()))
            assert info["iters"] == info_e["iters"]
            # eager work of the program between replays
            bie2d.bie_laplace_apply(other, torch.ones(1, other.M, dtype=torch.float64, device="cuda"))
            torch.cuda.synchronize()
        captured, replayed = g.graph_stats()
        assert captured > 0 and replayed >= 3 * info_e["iters"] // 2, (captured, replayed)
        # another configuration (one rhs) must not replay the two-rhs graphs
        one, _ = solve(g, kind, inp[:1].contiguous(), o)
        bie2d.bie_set_graphs(False)
        one_e, _ = solve(g, kind, inp[:1].contiguous(), o)
        assert torch.equal(one, one_e)
    finally:
        bie2d.bie_set_graphs(False)  # the library default


def test_graph_solve_vs_oracle():
    c, q = wl.elastance_small()
    g = bie2d.Geometry.from_curves(c)
    ref = ny.elastance_solve(ny.geometry_of(c), q)["phi"]
    o = bie2d.default_opts(tol=1e-12)
    bie2d.bie_set_graphs(True)
    try:
        for _ in range(3):
            phi, _ = bie2d.bie_elastance_solve(g, dev(q[None]), o)
            assert float(np.abs(phi.cpu().numpy()[0] - ref).max() / np.abs(ref).max()) < 1e-10
        assert g.graph_stats()[1] > 0
    finally:
        bie2d.bie_set_graphs(False)
