"""GPU: batched and served items above the 32,768-node threshold of BIE_AUTO, i.e. through the
FMM on the multi-geometry stream pool, against stored float64 oracle outputs
(tests/golden/fmm_items.json, written by tests/golden/make_golden.py from oracle/ only), and
the reuse of one batch or server across methods and across geometries that replace each other
(the cached batched-apply plan is keyed on each geometry's creation id, kind, rhs count, method
and block offset)."""
import json
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import nystrom as ny  # noqa: E402
from paper_1507_05925_amd import bie2d  # noqa: E402
from paper_1507_05925_amd import workloads as wl  # noqa: E402

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs the GPU")]
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
TOL = {bie2d.BIE_FP64: 1e-10, bie2d.BIE_MIXED: 1e-9}


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64), device="cuda")


def golden():
    return json.load(open(os.path.join(GOLDEN, "fmm_items.json")))["items"]


_CACHE = {}


def items():
    """(kind, Geometry, inputs) for workloads.fmm_items(); geometries are built once."""
    if "items" not in _CACHE:
        _CACHE["items"] = [(0 if k == "elastance" else 1, bie2d.Geometry.from_curves(c), inp)
                           for k, c, inp in wl.fmm_items()]
    return _CACHE["items"]


def opts(precision, method=bie2d.BIE_AUTO, leaf=64):
    return bie2d.default_opts(precision=precision, method=method, tol=1e-12, restart=150,
                              max_iter=3000, fmm_leaf=leaf)


def check(outs, gold, tol, what):
    for k, (o, g) in enumerate(zip(outs, gold)):
        ref = np.array(g["values"])
        err = float(np.abs(o - ref).max() / np.abs(ref).max())
        assert err < tol, (what, k, g["M"], err)


def test_items_cross_the_threshold():
    its = items()
    assert its[0][1].M > 32768 and its[1][1].M > 32768
    assert its[2][1].M <= 32768 and its[3][1].M <= 32768


@pytest.mark.parametrize("leaf", [64, 0])
@pytest.mark.parametrize("precision", [bie2d.BIE_FP64, bie2d.BIE_MIXED])
def test_batch_fmm_items_vs_oracle(precision, leaf):
    """leaf 0: the FMM items take their leaf sizes from the autotuner (a tree built for a leaf
    size of 0 would have the minimum depth and turn the far field into near-field work)."""
    b = bie2d.Batch()
    req = [(g, k, dev(inp)) for k, g, inp in items()]
    outs, info, rel = bie2d.bie_batch_solve(b, req, opts(precision, leaf=leaf))
    check([o.cpu().numpy() for o in outs], golden(), TOL[precision], "batch")
    assert (rel <= 1e-12).all(), rel
    if leaf == 0:
        for k, g, _ in items()[:2]:  # the FMM items: the tuner's sizes, among those it times
            lf64, lfmx = bie2d.bie_autotune(g, k, precision)
            assert lf64 in (24, 32, 48, 64, 96, 128) and lfmx in (24, 32, 48, 64, 96, 128)


@pytest.mark.parametrize("precision", [bie2d.BIE_FP64, bie2d.BIE_MIXED])
def test_batch_fmm_items_preconditioned(precision):
    """The same items with the block preconditioner (two-grid blocks for the FMM items' 256- and
    512-node bodies): the oracle's outputs, in fewer lock-step steps."""
    req = [(g, k, dev(inp)) for k, g, inp in items()]
    o = opts(precision)
    o.precond = bie2d.BIE_PRECOND_BLOCK
    outs, info, rel = bie2d.bie_batch_solve(bie2d.Batch(), req, o)
    check([x.cpu().numpy() for x in outs], golden(), TOL[precision], "batch, preconditioned")
    assert (rel <= 1e-12).all(), rel
    _, info0, _ = bie2d.bie_batch_solve(bie2d.Batch(), req, opts(precision))
    assert info["iters"] < info0["iters"], (info, info0)


def test_one_batch_direct_then_auto_then_direct():
    """The same batch object is solved with BIE_DIRECT, BIE_AUTO (FMM for the two large items)
    and BIE_DIRECT again: each must match the oracle (a plan kept across the method switch
    would skip or double an item's far field)."""
    b = bie2d.Batch()
    req = [(g, k, dev(inp)) for k, g, inp in items()]
    for method in (bie2d.BIE_DIRECT, bie2d.BIE_AUTO, bie2d.BIE_DIRECT):
        outs, info, rel = bie2d.bie_batch_solve(b, req, opts(bie2d.BIE_FP64, method))
        check([o.cpu().numpy() for o in outs], golden(), 1e-10, method)


@pytest.mark.parametrize("precision,leaf", [(bie2d.BIE_FP64, 64), (bie2d.BIE_MIXED, 64),
                                          (bie2d.BIE_MIXED, 0)])
def test_server_fmm_items_vs_oracle(precision, leaf):
    srv = bie2d.Server(opts(precision, leaf=leaf), max_cycles=400)
    tickets = []
    for k, g, inp in items():
        tickets.append([srv.submit(g, k, v) for v in inp])
    outs = []
    for tk in tickets:
        vals = []
        for t in tk:
            out, info = srv.wait(t, timeout=300)
            assert info["status"] == 0, info
            vals.append(out[0])
        outs.append(np.array(vals))
    srv.close()
    check(outs, golden(), TOL[precision], "server")


def test_server_geometry_destroyed_and_recreated():
    """A geometry is destroyed between requests and another one (different node count, often
    at the same address) takes its place; the server's cached plan must not be reused."""
    srv = bie2d.Server(opts(bie2d.BIE_FP64, bie2d.BIE_DIRECT))
    rng = np.random.default_rng(17)
    for n in (64, 96, 160, 64):
        c = wl.mixed_grid(rng, 4, np.full(4, n))
        g = bie2d.Geometry.from_curves(c)
        q = rng.standard_normal(4)
        out, info = srv.wait(srv.submit(g, 0, q), timeout=120)
        ref = ny.elastance_solve(ny.geometry_of(c), q)["phi"]
        assert float(np.abs(out[0] - ref).max() / np.abs(ref).max()) < 1e-10, n
        g.close()
    srv.close()
