"""GPU: bie_apply_noalloc (the direct apply with the library's fixed per-device workspace)
against the allocating entry points bie_laplace_apply / bie_stokes_apply on the same inputs,
on two calls in a row (the second smaller, so the first call's leftovers sit in the shared
workspace), both kinds and both precisions; and a request too large for the workspace is
refused before any device work."""
import ctypes

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import matfree as mf  # noqa: E402
from oracle import nystrom as ny  # noqa: E402
from paper_1507_05925_amd import bie2d  # noqa: E402
from paper_1507_05925_amd import workloads as wl  # noqa: E402

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs the GPU")]


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64), device="cuda")


@pytest.mark.parametrize("kind", [0, 1])
@pytest.mark.parametrize("precision", [bie2d.BIE_FP64, bie2d.BIE_MIXED])
def test_noalloc_matches_allocating_apply(kind, precision):
    rng = np.random.default_rng(40 + kind)
    big = wl.elastance_starfish(nbodies=24, n=256)[0]
    small = wl.elastance_small()[0]
    ref_apply = bie2d.bie_laplace_apply if kind == 0 else bie2d.bie_stokes_apply
    for c, nrhs in ((big, 8 if kind == 0 else 4), (small, 3)):
        g = bie2d.Geometry.from_curves(c)
        n = g.M if kind == 0 else 2 * g.M
        mu = dev(rng.standard_normal((nrhs, n)))
        for with_L in (True, False):
            got = bie2d.bie_apply_noalloc(g, kind, mu, precision, with_L)
            ref = ref_apply(g, mu, precision, bie2d.BIE_DIRECT, with_L)
            torch.cuda.synchronize()
            assert torch.equal(got, ref), (kind, precision, g.M, with_L)
        if precision == bie2d.BIE_FP64:  # and the oracle's matrix-free apply
            geo = ny.geometry_of(c)
            f = mf.laplace_apply if kind == 0 else mf.stokes_apply
            o = f(geo, mu.cpu().numpy()[0], with_L=False)  # the last call above had L off
            assert float(np.abs(got.cpu().numpy()[0] - o).max() / np.abs(o).max()) < 1e-12


def test_noalloc_rejects_oversized_request():
    g = bie2d.Geometry.from_curves(wl.elastance_starfish(nbodies=100, n=256)[0])
    nrhs = 64  # 64 rhs x 25,600 nodes: strengths and partial sums exceed the fixed workspace
    mu = torch.zeros(nrhs, g.M, dtype=torch.float64, device="cuda")
    with pytest.raises(bie2d.BieError) as e:
        bie2d.bie_apply_noalloc(g, 0, mu)
    assert e.value.code == bie2d.BIE_EINVAL and "scratch" in str(e.value)
    L = bie2d.lib()
    assert L.bie_apply_noalloc(g.handle, 2, 0, 1, 1, ctypes.c_void_p(mu.data_ptr()),
                               ctypes.c_void_p(mu.data_ptr() + 8), None) == bie2d.BIE_EINVAL
