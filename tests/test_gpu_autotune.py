"""GPU: the FMM leaf-size autotuner. Solves with opts.fmm_leaf = 0 take the leaf sizes from the
tuner (timed on the geometry over 24..128 nodes per leaf, per precision) and still match the
stored float64 oracle outputs; the choice is cached per shape class in the context, so a second
geometry of the same class is not timed again."""
import json
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_1507_05925_amd import bie2d  # noqa: E402
from paper_1507_05925_amd import workloads as wl  # noqa: E402

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs the GPU")]
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64), device="cuda")


@pytest.mark.parametrize("precision,tol", [(bie2d.BIE_FP64, 1e-10), (bie2d.BIE_MIXED, 1e-9)])
def test_tuned_leaf_solves_match_oracle_and_cache(precision, tol):
    kind, c, inp = wl.fmm_items()[0]
    gold = json.load(open(os.path.join(GOLDEN, "fmm_items.json")))["items"][0]["values"]
    ctx = bie2d.Context(0, bie2d.default_opts(method=bie2d.BIE_FMM, precision=precision,
                                              fmm_leaf=0, tol=1e-12, restart=150))
    g = ctx.geometry(c)
    phi, info = bie2d.bie_elastance_solve(g, dev(inp))
    ref = np.array(gold)
    err = float(np.abs(phi.cpu().numpy() - ref).max() / np.abs(ref).max())
    assert err < tol, err
    tuned, hits = bie2d.bie_autotune_stats(ctx)
    assert tuned == (2 if precision == bie2d.BIE_MIXED else 1) and hits == 0
    a, b = bie2d.bie_autotune(g, 0, precision, 2)  # cached now
    assert a in (24, 32, 48, 64, 96, 128) and b in (24, 32, 48, 64, 96, 128)
    g2 = ctx.geometry(c)  # same shape class: looked up, not timed
    phi2, _ = bie2d.bie_elastance_solve(g2, dev(inp))
    assert torch.equal(phi2, phi)
    tuned2, hits2 = bie2d.bie_autotune_stats(ctx)
    assert tuned2 == tuned and hits2 >= 2 * tuned
    ctx.close()
