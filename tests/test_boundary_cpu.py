"""CPU: the C-ABI's host-side checks and error codes, forced from the host without a GPU.

bie_curves_check runs the checks that bie_geom_create applies to its curve samples (finite,
positively oriented, read-off points inside their bodies; the BIE_ERESOLVE warning for
under-resolved curves and gaps below a few node spacings). Context and server creation fail
with BIE_EDEVICE on a host without a device instead of handing back an object that cannot work;
option validation (viscosity, fmm_eps, l2_scaling) happens before any device call.
"""
import ctypes

import numpy as np
import pytest

from paper_1507_05925_amd import bie2d
from paper_1507_05925_amd import workloads as wl

torch = pytest.importorskip("torch")
no_gpu = pytest.mark.skipif(torch.cuda.is_available(), reason="checks the no-device path")


def banana(n=2048):
    """A smooth CCW body bent so that its arc-length centroid lies outside it:
    x = cos t, y = 0.15 sin t - 0.8 cos 2t (the branches t in (0, pi) and (pi, 2 pi) are 0.3 |sin t|
    apart at the same x, so the curve is simple)."""
    t = 2 * np.pi * np.arange(n) / n
    x, dx, ddx = np.cos(t), -np.sin(t), -np.cos(t)
    y = 0.15 * np.sin(t) - 0.8 * np.cos(2 * t)
    dy = 0.15 * np.cos(t) + 1.6 * np.sin(2 * t)
    ddy = -0.15 * np.sin(t) + 3.2 * np.cos(2 * t)
    return wl.assemble([(x, y, dx, dy, ddx, ddy)], [[0.0, 0.0]], [1.2])


def test_good_geometries_pass():
    for c in (wl.elastance_small()[0], wl.two_discs(0.5, 256), wl.two_discs(0.005, 6144),
              wl.mobility_ellipses(nbodies=20, n=512)[0]):
        code, msg = bie2d.bie_curves_check(c)
        assert code == bie2d.BIE_OK, msg


def test_clockwise_and_nonfinite_are_einval():
    c = wl.two_discs(0.5, 64)
    rev = wl.assemble([(c.x[:64][::-1], c.y[:64][::-1], -c.dx[:64][::-1], -c.dy[:64][::-1],
                        c.ddx[:64][::-1], c.ddy[:64][::-1])], [[0, 0]], [1])
    code, msg = bie2d.bie_curves_check(rev)
    assert code == bie2d.BIE_EINVAL and "positively oriented" in msg
    bad = wl.two_discs(0.5, 64)
    bad.ddy[70] = np.nan
    code, msg = bie2d.bie_curves_check(bad)
    assert code == bie2d.BIE_EINVAL and "non-finite" in msg and "body 1" in msg


def test_read_off_point_must_be_inside():
    c = wl.two_discs(0.5, 128)
    inside = np.array([[-1.25, 0.1], [1.25, -0.3]])
    assert bie2d.bie_curves_check(c, inside)[0] == bie2d.BIE_OK
    outside = np.array([[-1.25, 0.1], [3.0, 0.0]])
    code, msg = bie2d.bie_curves_check(c, outside)
    assert code == bie2d.BIE_EINVAL and "body 1" in msg and "not inside" in msg
    # default read-off point (the arc-length centroid) outside a bent body
    b = banana()
    code, msg = bie2d.bie_curves_check(b)
    assert code == bie2d.BIE_EINVAL and "centroid" in msg
    assert bie2d.bie_curves_check(b, np.array([[0.0, 0.8]]))[0] == bie2d.BIE_OK


def test_resolution_warning():
    # under-resolved curves: the splash bodies at 128 nodes (turning number off by 13 %)
    code, msg = bie2d.bie_curves_check(wl.splash(128))
    assert code == bie2d.BIE_ERESOLVE and "under-resolved" in msg
    # a gap of 0.005 between unit discs: 2048 nodes give 1.6 node spacings, 6144 give 4.9
    code, msg = bie2d.bie_curves_check(wl.two_discs(0.005, 2048))
    assert code == bie2d.BIE_ERESOLVE and "bodies 0 and 1" in msg
    assert bie2d.bie_curves_check(wl.two_discs(0.005, 6144))[0] == bie2d.BIE_OK
    # a read-off point outside is an error even when the curves are also under-resolved
    code, _ = bie2d.bie_curves_check(wl.splash(128), np.full((5, 2), 50.0))
    assert code == bie2d.BIE_EINVAL


def test_option_validation_before_device():
    L = bie2d.lib()
    b = ctypes.c_void_p()
    assert L.bie_batch_create(ctypes.byref(b)) == bie2d.BIE_OK
    item = bie2d.bie_batch_item()
    info = bie2d.bie_info()
    for field, value in (("viscosity", 0.0), ("viscosity", float("nan")), ("fmm_eps", -1e-3),
                         ("mixed_strategy", 2), ("mixed_strategy", -1), ("precond", 2),
                         ("l2_scaling", 2), ("l2_scaling", 1)):
        o = bie2d.default_opts(**{field: value})
        rc = L.bie_batch_solve(b, 1, ctypes.cast(ctypes.pointer(item), ctypes.c_void_p),
                               ctypes.byref(o), ctypes.byref(info), None, None)
        assert rc == bie2d.BIE_EINVAL, (field, value)
    assert b"l2_scaling" in L.bie_last_error()
    L.bie_batch_destroy(b)
    o = bie2d.default_opts()
    assert o.viscosity == 1.0 and o.fmm_eps == 0.0 and o.l2_scaling == 0
    assert o.mixed_strategy == bie2d.BIE_MIXED_RELAXED and o.precond == bie2d.BIE_PRECOND_NONE
    both = bie2d.default_opts(precond=bie2d.BIE_PRECOND_BLOCK, l2_scaling=1)
    L = bie2d.lib()
    b2 = ctypes.c_void_p()
    assert L.bie_batch_create(ctypes.byref(b2)) == bie2d.BIE_OK
    assert L.bie_batch_solve(b2, 1, ctypes.cast(ctypes.pointer(bie2d.bie_batch_item()), ctypes.c_void_p),
                             ctypes.byref(both), ctypes.byref(bie2d.bie_info()), None, None) == bie2d.BIE_EINVAL
    L.bie_batch_destroy(b2)


@no_gpu
def test_context_and_server_need_a_device():
    L = bie2d.lib()
    assert L.bie_create(None, 0, None) == bie2d.BIE_EINVAL
    h = ctypes.c_void_p()
    assert L.bie_create(ctypes.byref(h), 0, None) == bie2d.BIE_EDEVICE
    assert b"no HIP device" in L.bie_last_error()
    cfg = bie2d.bie_server_config()
    cfg.max_cycles = 10
    cfg.opts = bie2d.default_opts()
    assert L.bie_server_create(ctypes.byref(cfg), ctypes.byref(h)) == bie2d.BIE_EDEVICE
    cfg.opts = bie2d.default_opts(l2_scaling=1)
    assert L.bie_server_create(ctypes.byref(cfg), ctypes.byref(h)) == bie2d.BIE_EINVAL
    with pytest.raises(bie2d.BieError):
        bie2d.Context(0)
