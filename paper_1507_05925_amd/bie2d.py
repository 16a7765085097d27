"""Python binding of libbie2d (C ABI in include/bie2d.h): argument marshalling only.

Every numerical step runs in the HIP library; this module only checks tensor dtypes, devices and
shapes, passes data pointers and the current torch stream, and converts status codes into
exceptions. Device memory for inputs and outputs comes from torch (float64 CUDA/HIP tensors).
If libbie2d.so has not been built, loading fails with an error (there is no fallback path).
"""
from __future__ import annotations

import ctypes
import os
import re
import warnings
import weakref

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libbie2d.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "bie2d.h")

BIE_OK, BIE_EINVAL, BIE_ENOMEM, BIE_ENOCONV, BIE_EDEVICE, BIE_ERESOLVE = 0, -1, -2, -3, -4, -5
BIE_FP64, BIE_MIXED = 0, 1
BIE_DIRECT, BIE_FMM, BIE_AUTO = 0, 1, 2
BIE_MIXED_RELAXED, BIE_MIXED_REFINE = 0, 1
BIE_PRECOND_NONE, BIE_PRECOND_BLOCK = 0, 1


class BieError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"bie2d error {code}: {msg}")
        self.code = code


class ResolutionWarning(UserWarning):
    """bie_geom_create returned BIE_ERESOLVE: the geometry exists, but a curve is
    under-resolved or two bodies are closer than a few node spacings."""


class bie_opts(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int), ("method", ctypes.c_int), ("tol", ctypes.c_double),
                ("restart", ctypes.c_int), ("max_iter", ctypes.c_int),
                ("inner_tol", ctypes.c_double), ("max_refine", ctypes.c_int),
                ("fmm_order", ctypes.c_int), ("fmm_leaf", ctypes.c_int),
                ("viscosity", ctypes.c_double), ("fmm_eps", ctypes.c_double),
                ("mixed_strategy", ctypes.c_int), ("precond", ctypes.c_int),
                ("l2_scaling", ctypes.c_int)]


class bie_batch_item(ctypes.Structure):
    _fields_ = [("g", ctypes.c_void_p), ("kind", ctypes.c_int), ("nrhs", ctypes.c_int),
                ("in_", ctypes.c_void_p), ("out", ctypes.c_void_p)]


class bie_info(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int), ("refinements", ctypes.c_int),
                ("applies_fp64", ctypes.c_int), ("applies_fp32", ctypes.c_int),
                ("rel_residual", ctypes.c_double), ("seconds", ctypes.c_double),
                ("pairs", ctypes.c_longlong), ("net_charge_or_force", ctypes.c_double * 2)]

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_}
        d["net_charge_or_force"] = tuple(self.net_charge_or_force)
        return d


_P = ctypes.c_void_p
_I = ctypes.c_int
_SIGS = {
    "bie_last_error": ([], ctypes.c_char_p),
    "bie_default_opts": ([ctypes.POINTER(bie_opts)], _I),
    "bie_create": ([ctypes.POINTER(_P), _I, ctypes.POINTER(bie_opts)], _I),
    "bie_destroy": ([_P], _I),
    "bie_ctx_defaults": ([_P, ctypes.POINTER(bie_opts)], _I),
    "bie_ctx_geom_create": ([_P, _I, _P, _P, _P, _P, ctypes.POINTER(_P)], _I),
    "bie_geom_create": ([_I, _P, _P, _P, _P, ctypes.POINTER(_P)], _I),
    "bie_curves_check": ([_I, _P, _P, _P], _I),
    "bie_geom_destroy": ([_P], _I),
    "bie_geom_sizes": ([_P, ctypes.POINTER(_I), ctypes.POINTER(_I)], _I),
    "bie_geom_export": ([_P, _P, _P, _P], _I),
    "bie_geom_device_bytes": ([_P], ctypes.c_longlong),
    "bie_geom_set_fmm": ([_P, _I, _I], _I),
    "bie_laplace_apply": ([_P, _I, _I, _I, _I, _P, _P, _P], _I),
    "bie_stokes_apply": ([_P, _I, _I, _I, _I, _P, _P, _P], _I),
    "bie_apply_noalloc": ([_P, _I, _I, _I, _I, _P, _P, _P], _I),
    "bie_elastance_rhs": ([_P, _I, _P, _P, _P, _P], _I),
    "bie_mobility_rhs": ([_P, _I, _P, _P, _P, _P], _I),
    "bie_laplace_potential": ([_P, _I, _P, _P, _P], _I),
    "bie_stokes_rigid_motion": ([_P, _I, _P, _P, _P], _I),
    "bie_elastance_field": ([_P, _I, _P, _P, _I, _P, _P, _P], _I),
    "bie_mobility_field": ([_P, _I, _P, _P, _I, _P, _P, _P], _I),
    "bie_elastance_solve": ([_P, _I, _P, _P, _P, ctypes.POINTER(bie_opts),
                             ctypes.POINTER(bie_info), _P], _I),
    "bie_mobility_solve": ([_P, _I, _P, _P, _P, ctypes.POINTER(bie_opts),
                            ctypes.POINTER(bie_info), _P], _I),
    "bie_laplace_dl_apply": ([_P, _I, _I, _P, _P, _P], _I),
    "bie_stokes_dl_apply": ([_P, _I, _I, _P, _P, _P], _I),
    "bie_capacitance_solve": ([_P, _I, _P, _P, _P, _P, ctypes.POINTER(bie_opts),
                               ctypes.POINTER(bie_info), _P], _I),
    "bie_resistance_solve": ([_P, _I, _P, _P, _P, _P, ctypes.POINTER(bie_opts),
                              ctypes.POINTER(bie_info), _P], _I),
    "bie_elastance_matrix": ([_P, _P, _I, ctypes.POINTER(bie_opts), ctypes.POINTER(bie_info), _P], _I),
    "bie_mobility_matrix": ([_P, _P, _I, ctypes.POINTER(bie_opts), ctypes.POINTER(bie_info), _P], _I),
    "bie_batch_create": ([ctypes.POINTER(_P)], _I),
    "bie_batch_destroy": ([_P], _I),
    "bie_batch_solve": ([_P, _I, _P, ctypes.POINTER(bie_opts), ctypes.POINTER(bie_info), _P, _P], _I),
    "bie_server_create": ([_P, ctypes.POINTER(_P)], _I),
    "bie_server_submit": ([_P, _P, _I, _I, _P, _P, ctypes.POINTER(ctypes.c_longlong)], _I),
    "bie_server_wait": ([_P, ctypes.c_longlong, ctypes.c_double, _P], _I),
    "bie_server_stats": ([_P, ctypes.POINTER(ctypes.c_longlong), ctypes.POINTER(ctypes.c_longlong),
                          ctypes.POINTER(ctypes.c_longlong), ctypes.POINTER(ctypes.c_longlong)], _I),
    "bie_server_destroy": ([_P], _I),
    "bie_server_inject_failure": ([_P, _I], _I),
    "bie_set_graphs": ([_I], _I),
    "bie_autotune": ([_P, _I, _I, _I, ctypes.POINTER(_I), ctypes.POINTER(_I), _P], _I),
    "bie_autotune_stats": ([_P, ctypes.POINTER(ctypes.c_longlong),
                            ctypes.POINTER(ctypes.c_longlong)], _I),
    "bie_fmm_terms": ([ctypes.POINTER(bie_opts), _I, _I, ctypes.POINTER(_I)], _I),
    "bie_geom_graph_stats": ([_P, ctypes.POINTER(ctypes.c_longlong),
                              ctypes.POINTER(ctypes.c_longlong)], _I),
    "bie_profile_enable": ([_I], _I),
    "bie_profile_sample": ([ctypes.c_int], _I),
    "bie_profile_select": ([ctypes.c_uint], _I),
    "bie_profile_read": ([_I, ctypes.POINTER(ctypes.c_longlong), ctypes.POINTER(ctypes.c_double),
                          ctypes.POINTER(ctypes.c_longlong)], _I),
}

BIE_K_FAR_LAPLACE_F32, BIE_K_FAR_LAPLACE_F64, BIE_K_FAR_STOKES_F32, BIE_K_FAR_STOKES_F64 = 0, 1, 2, 3
BIE_K_EPILOGUE, BIE_K_FMM, BIE_K_FMM_M2L, BIE_K_FMM_EVAL = 4, 5, 6, 7
BIE_K_DOUBLE_LAYER, BIE_K_FMM_M2L_F32, BIE_K_FMM_NEAR_F32, BIE_K_PRECOND = 8, 9, 10, 11
BIE_K_COUNT = 12


def bie_autotune(g, kind, precision=BIE_FP64, nrhs=1):
    """Tune (or look up) the FMM leaf sizes for g's shape class -> (leaf_fp64, leaf_mixed)."""
    a, b = _I(), _I()
    _check(lib().bie_autotune(g.handle, int(kind), precision, int(nrhs), ctypes.byref(a),
                              ctypes.byref(b), _stream()))
    return a.value, b.value


def bie_fmm_terms(opts, kind, precision=BIE_FP64):
    """Expansion length (terms) of the FMM applies of a solve with these options."""
    t = _I()
    _check(lib().bie_fmm_terms(ctypes.byref(opts), int(kind), int(precision), ctypes.byref(t)))
    return t.value


def bie_autotune_stats(ctx=None):
    """-> (shape classes tuned, cache hits) of a context's cache (None: the process cache)."""
    t, h = ctypes.c_longlong(), ctypes.c_longlong()
    _check(lib().bie_autotune_stats(None if ctx is None else ctx.handle, ctypes.byref(t),
                                    ctypes.byref(h)))
    return t.value, h.value


def bie_set_graphs(on=True):
    """Replay captured HIP graphs of the solves' Arnoldi steps (process-wide, default off)."""
    _check(lib().bie_set_graphs(int(on)))


def bie_profile_enable(on=True):
    _check(lib().bie_profile_enable(int(on)))


def bie_profile_select(classes=None):
    """Record only the given kernel classes (None: all)."""
    mask = 0xFFFFFFFF if classes is None else sum(1 << int(k) for k in classes)
    _check(lib().bie_profile_select(mask))


def bie_profile_sample(every=1):
    """Record events around every `every`-th launch of each class only."""
    _check(lib().bie_profile_sample(int(every)))


def bie_profile_read(kclass):
    """-> dict(launches, ms_total, pairs) for one kernel class."""
    n, ms, pr = ctypes.c_longlong(), ctypes.c_double(), ctypes.c_longlong()
    _check(lib().bie_profile_read(kclass, ctypes.byref(n), ctypes.byref(ms), ctypes.byref(pr)))
    return {"launches": n.value, "ms_total": ms.value, "pairs": pr.value}

_lib = None


def header_symbols(path=HEADER):
    """Function names declared in include/bie2d.h."""
    text = open(path).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(bie_[a-z0-9_]+)\s*\(", text)))


def lib():
    """Load libbie2d.so (built by paper_1507_05925_amd.build); raises if it is missing."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built: run `python -m paper_1507_05925_amd.build`")
        try:  # torch's HIP runtime first, so that the library binds to the same one
            import torch  # noqa: F401
        except ImportError:
            pass
        L = ctypes.CDLL(LIB_PATH)
        for name, (args, res) in _SIGS.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = res
        _lib = L
    return _lib


def _check(code):
    if code not in (BIE_OK,):
        raise BieError(code, lib().bie_last_error().decode())
    return code


def _torch():
    import torch
    return torch


def _stream():
    torch = _torch()
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dptr(t, shape_last=None, name="tensor"):
    torch = _torch()
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda" or t.dtype != torch.float64:
        raise TypeError(f"{name} must be a float64 CUDA tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape_last is not None and t.shape[-1] != shape_last:
        raise ValueError(f"{name}: last dimension {t.shape[-1]} != {shape_last}")
    return ctypes.c_void_p(t.data_ptr())


def default_opts(**kw):
    o = bie_opts()
    _check(lib().bie_default_opts(ctypes.byref(o)))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise KeyError(k)
        setattr(o, k, v)
    return o


def bie_curves_check(curves, interior=None):
    """Host-side checks of curve samples (a Curves object) as bie_geom_create applies them:
    returns (code, message) with code BIE_OK, BIE_EINVAL or BIE_ERESOLVE."""
    c = np.ascontiguousarray(np.stack([curves.x, curves.y, curves.dx, curves.dy, curves.ddx,
                                       curves.ddy]), dtype=np.float64)
    npb = np.ascontiguousarray(curves.nodes_per_body, dtype=np.int32)
    ip = None if interior is None else np.ascontiguousarray(interior, dtype=np.float64).reshape(-1)
    code = lib().bie_curves_check(len(npb), npb.ctypes.data_as(ctypes.c_void_p),
                                  c.ctypes.data_as(ctypes.c_void_p),
                                  None if ip is None else ip.ctypes.data_as(ctypes.c_void_p))
    return code, (lib().bie_last_error().decode() if code != BIE_OK else "")


class Context:
    """Owns a bie_ctx: a device, default options, and the geometries created through it."""

    def __init__(self, device=0, defaults=None):
        h = ctypes.c_void_p()
        _check(lib().bie_create(ctypes.byref(h), int(device),
                                None if defaults is None else ctypes.byref(defaults)))
        self.handle = h
        self.device = int(device)
        self._geoms = weakref.WeakSet()

    def defaults(self):
        o = bie_opts()
        _check(lib().bie_ctx_defaults(self.handle, ctypes.byref(o)))
        return o

    def geometry(self, curves, interior=None):
        return Geometry.from_curves(curves, device=f"cuda:{self.device}", interior=interior,
                                    ctx=self)

    def close(self):
        if getattr(self, "handle", None):
            for g in list(self._geoms):  # bie_destroy frees them: forget the handles first
                g.handle = None
            lib().bie_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Geometry:
    """Owns a bie_geom (device-resident quadrature data and workspace)."""

    def __init__(self, nodes_per_body, curve, interior=None, ctx=None):
        self.nodes_per_body = np.ascontiguousarray(nodes_per_body, dtype=np.int32)
        M = int(self.nodes_per_body.sum())
        if tuple(curve.shape) != (6, M):
            raise ValueError(f"curve must have shape (6, {M})")
        h = ctypes.c_void_p()
        ip = None if interior is None else _dptr(interior, 2, "interior")
        args = (len(self.nodes_per_body), self.nodes_per_body.ctypes.data_as(ctypes.c_void_p),
                _dptr(curve, M, "curve"), ip, _stream(), ctypes.byref(h))
        code = (lib().bie_geom_create(*args) if ctx is None
                else lib().bie_ctx_geom_create(ctx.handle, *args))
        if code == BIE_ERESOLVE:
            warnings.warn(lib().bie_last_error().decode(), ResolutionWarning, stacklevel=3)
        else:
            _check(code)
        self.handle = h
        self.ctx = ctx  # keeps the context alive while the geometry is
        if ctx is not None:
            ctx._geoms.add(self)
        self.N, self.M = len(self.nodes_per_body), M
        self.device = curve.device

    @classmethod
    def from_curves(cls, curves, device="cuda", interior=None, ctx=None):
        torch = _torch()
        c = np.stack([curves.x, curves.y, curves.dx, curves.dy, curves.ddx, curves.ddy])
        t = torch.from_numpy(np.ascontiguousarray(c)).to(device)
        it = None if interior is None else torch.as_tensor(np.asarray(interior, np.float64),
                                                          device=device).reshape(-1, 2).contiguous()
        return cls(curves.nodes_per_body, t, it, ctx=ctx)

    def close(self):
        if getattr(self, "handle", None):
            lib().bie_geom_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def sizes(self):
        n, m = _I(), _I()
        _check(lib().bie_geom_sizes(self.handle, ctypes.byref(n), ctypes.byref(m)))
        return n.value, m.value

    def export(self):
        torch = _torch()
        out = torch.empty(8, self.M, dtype=torch.float64, device=self.device)
        ob = torch.empty(4, self.N, dtype=torch.float64, device=self.device)
        _check(lib().bie_geom_export(self.handle, _dptr(out, self.M), _dptr(ob, self.N), _stream()))
        keys = ["x", "y", "nx", "ny", "w", "kappa", "px", "py"]
        d = {k: out[i] for i, k in enumerate(keys)}
        d.update({"length": ob[0], "xc": ob[1], "yc": ob[2], "W": ob[3]})
        return d

    def device_bytes(self):
        return int(lib().bie_geom_device_bytes(self.handle))

    def graph_stats(self):
        """-> (Arnoldi steps captured as HIP graphs, steps replayed) of this geometry's solves."""
        c, r = ctypes.c_longlong(), ctypes.c_longlong()
        _check(lib().bie_geom_graph_stats(self.handle, ctypes.byref(c), ctypes.byref(r)))
        return c.value, r.value

    def set_fmm(self, order, leaf=64):
        _check(lib().bie_geom_set_fmm(self.handle, int(order), int(leaf)))


def _rows(t, width):
    return 1 if t.dim() == 1 else int(np.prod(t.shape[:-1]))


def bie_laplace_apply(g, mu, precision=BIE_FP64, method=BIE_DIRECT, with_L=True, out=None):
    torch = _torch()
    out = torch.empty_like(mu) if out is None else out
    _check(lib().bie_laplace_apply(g.handle, precision, method, int(with_L), _rows(mu, g.M),
                                   _dptr(mu, g.M, "mu"), _dptr(out, g.M, "out"), _stream()))
    return out


def bie_stokes_apply(g, mu, precision=BIE_FP64, method=BIE_DIRECT, with_L=True, out=None):
    torch = _torch()
    out = torch.empty_like(mu) if out is None else out
    _check(lib().bie_stokes_apply(g.handle, precision, method, int(with_L), _rows(mu, 2 * g.M),
                                  _dptr(mu, 2 * g.M, "mu"), _dptr(out, 2 * g.M, "out"), _stream()))
    return out


def bie_apply_noalloc(g, kind, mu, precision=BIE_FP64, with_L=True, out=None):
    """The direct apply with the library's fixed per-device workspace (no allocation)."""
    torch = _torch()
    n = g.M if kind == 0 else 2 * g.M
    out = torch.empty_like(mu) if out is None else out
    _check(lib().bie_apply_noalloc(g.handle, int(kind), precision, int(with_L), _rows(mu, n),
                                   _dptr(mu, n, "mu"), _dptr(out, n, "out"), _stream()))
    return out


def bie_elastance_rhs(g, q):
    torch = _torch()
    R = _rows(q, g.N)
    sigma = torch.empty(R, g.M, dtype=torch.float64, device=q.device)
    f = torch.empty_like(sigma)
    _check(lib().bie_elastance_rhs(g.handle, R, _dptr(q, g.N, "q"), _dptr(sigma), _dptr(f), _stream()))
    return sigma.reshape(q.shape[:-1] + (g.M,)), f.reshape(q.shape[:-1] + (g.M,))


def bie_mobility_rhs(g, FT):
    torch = _torch()
    R = _rows(FT, 3 * g.N)
    rho = torch.empty(R, 2 * g.M, dtype=torch.float64, device=FT.device)
    f = torch.empty_like(rho)
    _check(lib().bie_mobility_rhs(g.handle, R, _dptr(FT, 3 * g.N, "FT"), _dptr(rho), _dptr(f), _stream()))
    return rho.reshape(FT.shape[:-1] + (2 * g.M,)), f.reshape(FT.shape[:-1] + (2 * g.M,))


def bie_laplace_potential(g, dens):
    torch = _torch()
    R = _rows(dens, g.M)
    phi = torch.empty(R, g.N, dtype=torch.float64, device=dens.device)
    _check(lib().bie_laplace_potential(g.handle, R, _dptr(dens, g.M, "dens"), _dptr(phi), _stream()))
    return phi.reshape(dens.shape[:-1] + (g.N,))


def bie_stokes_rigid_motion(g, dens):
    torch = _torch()
    R = _rows(dens, 2 * g.M)
    VW = torch.empty(R, 3 * g.N, dtype=torch.float64, device=dens.device)
    _check(lib().bie_stokes_rigid_motion(g.handle, R, _dptr(dens, 2 * g.M, "dens"), _dptr(VW), _stream()))
    return VW.reshape(dens.shape[:-1] + (3 * g.N,))


def _solve(fn, g, data, width_in, width_mu, opts, want_mu, allow_noconv):
    torch = _torch()
    R = _rows(data, width_in)
    res = torch.empty(R, width_in, dtype=torch.float64, device=data.device)
    mu = torch.empty(R, width_mu, dtype=torch.float64, device=data.device) if want_mu else None
    info = bie_info()
    o = None if opts is None else ctypes.byref(opts)  # NULL: the library's (or context's) defaults
    code = fn(g.handle, R, _dptr(data, width_in, "input"), _dptr(res),
              _dptr(mu) if want_mu else None, o, ctypes.byref(info), _stream())
    if not (code == BIE_OK or (allow_noconv and code == BIE_ENOCONV)):
        _check(code)
    shape = data.shape[:-1]
    out = (res.reshape(shape + (width_in,)), info.as_dict())
    if want_mu:
        out = out + (mu.reshape(shape + (width_mu,)),)
    return out


def bie_elastance_solve(g, q, opts=None, want_mu=False, allow_noconv=False):
    """q [.., N] -> (phi [.., N], info[, mu [.., M]])."""
    return _solve(lib().bie_elastance_solve, g, q, g.N, g.M, opts, want_mu, allow_noconv)


def bie_mobility_solve(g, FT, opts=None, want_mu=False, allow_noconv=False):
    """FT [.., 3N] -> (VW [.., 3N], info[, mu [.., 2M]])."""
    return _solve(lib().bie_mobility_solve, g, FT, 3 * g.N, 2 * g.M, opts, want_mu, allow_noconv)


def _field(fn, g, inp, width, mu, mlen, pts, comps):
    torch = _torch()
    R = _rows(inp, width)
    P = pts.reshape(-1, 2).shape[0]
    out = torch.empty((R, P, comps) if comps > 1 else (R, P), dtype=torch.float64, device=g.device)
    _check(fn(g.handle, R, _dptr(inp, width, "input"), _dptr(mu, mlen, "mu"), int(P),
              _dptr(pts.reshape(-1), None, "pts"), _dptr(out), _stream()))
    return out


def bie_elastance_field(g, q, mu, pts):
    """Potential u = S[mu + sigma(q)] at points pts [P, 2]: q [R, N], mu [R, M] -> [R, P]."""
    return _field(lib().bie_elastance_field, g, q, g.N, mu, g.M, pts, 1)


def bie_mobility_field(g, FT, mu, pts):
    """Velocity Scal[mu + rho(F, T)] at points pts [P, 2]: FT [R, 3N], mu [R, 2M] -> [R, P, 2]."""
    return _field(lib().bie_mobility_field, g, FT, 3 * g.N, mu, 2 * g.M, pts, 2)


def bie_laplace_dl_apply(g, mu, with_completion=True, out=None):
    """(1/2 I + D + C) mu for mu [.., M] (capacitance operator)."""
    torch = _torch()
    out = torch.empty_like(mu) if out is None else out
    _check(lib().bie_laplace_dl_apply(g.handle, int(with_completion), _rows(mu, g.M),
                                      _dptr(mu, g.M, "mu"), _dptr(out, g.M, "out"), _stream()))
    return out


def bie_stokes_dl_apply(g, mu, with_completion=True, out=None):
    """(1/2 I + Dcal + C) mu for mu [.., 2M] node-major (resistance operator)."""
    torch = _torch()
    out = torch.empty_like(mu) if out is None else out
    _check(lib().bie_stokes_dl_apply(g.handle, int(with_completion), _rows(mu, 2 * g.M),
                                     _dptr(mu, 2 * g.M, "mu"), _dptr(out, 2 * g.M, "out"),
                                     _stream()))
    return out


def _dl_solve(fn, g, data, width_in, width_mu, width_inf, opts, want_mu, allow_noconv):
    torch = _torch()
    R = _rows(data, width_in)
    res = torch.empty(R, width_in, dtype=torch.float64, device=data.device)
    uinf = torch.empty(R, width_inf, dtype=torch.float64, device=data.device)
    mu = torch.empty(R, width_mu, dtype=torch.float64, device=data.device) if want_mu else None
    info = bie_info()
    o = None if opts is None else ctypes.byref(opts)
    code = fn(g.handle, R, _dptr(data, width_in, "input"), _dptr(res), _dptr(uinf),
              _dptr(mu) if want_mu else None, o, ctypes.byref(info), _stream())
    if not (code == BIE_OK or (allow_noconv and code == BIE_ENOCONV)):
        _check(code)
    shape = data.shape[:-1]
    uinf = uinf.reshape(shape + ((width_inf,) if width_inf > 1 else ()))
    out = (res.reshape(shape + (width_in,)), uinf, info.as_dict())
    if want_mu:
        out = out + (mu.reshape(shape + (width_mu,)),)
    return out


def bie_capacitance_solve(g, phi, opts=None, want_mu=False, allow_noconv=False):
    """Conductor potentials phi [.., N] -> (q [.., N], u_inf [..], info[, mu [.., M]])."""
    return _dl_solve(lib().bie_capacitance_solve, g, phi, g.N, g.M, 1, opts, want_mu,
                     allow_noconv)


def bie_resistance_solve(g, VW, opts=None, want_mu=False, allow_noconv=False):
    """Rigid motions VW [.., 3N] -> (FT [.., 3N], u_inf [.., 2], info[, mu [.., 2M]])."""
    return _dl_solve(lib().bie_resistance_solve, g, VW, 3 * g.N, 2 * g.M, 2, opts, want_mu,
                     allow_noconv)


def _matrix(fn, g, n, max_rhs, opts):
    torch = _torch()
    out = torch.empty(n, n, dtype=torch.float64, device=g.device)  # rows = columns of the matrix
    info = bie_info()
    o = None if opts is None else ctypes.byref(opts)
    _check(fn(g.handle, _dptr(out), int(max_rhs), o, ctypes.byref(info), _stream()))
    return out.t().contiguous(), info.as_dict()  # column-major buffer -> matrix


def bie_elastance_matrix(g, max_rhs=0, opts=None):
    return _matrix(lib().bie_elastance_matrix, g, g.N, max_rhs, opts)


def bie_mobility_matrix(g, max_rhs=0, opts=None):
    return _matrix(lib().bie_mobility_matrix, g, 3 * g.N, max_rhs, opts)


class Batch:
    """Owns a bie_batch (solver workspace reused across batched solves)."""

    def __init__(self):
        h = ctypes.c_void_p()
        _check(lib().bie_batch_create(ctypes.byref(h)))
        self.handle = h

    def close(self):
        if getattr(self, "handle", None):
            lib().bie_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def bie_batch_solve(batch, items, opts=None, allow_noconv=False):
    """items: list of (Geometry, kind, input tensor [nrhs, width] or None for the identity
    block). Returns (outputs, info, per-item worst relative residual); for identity items the
    output is the matrix P (kind 0) or M (kind 1)."""
    torch = _torch()
    arr = (bie_batch_item * len(items))()
    outs = []
    for k, (g, kind, inp) in enumerate(items):
        width = g.N if kind == 0 else 3 * g.N
        nrhs = width if inp is None else _rows(inp, width)
        out = torch.empty(nrhs, width, dtype=torch.float64, device=g.device)
        outs.append(out)
        arr[k].g = g.handle
        arr[k].kind = kind
        arr[k].nrhs = nrhs
        arr[k].in_ = None if inp is None else _dptr(inp, width, "input").value
        arr[k].out = _dptr(out).value
    info = bie_info()
    rel = np.zeros(len(items))
    o = opts if opts is not None else default_opts()
    code = lib().bie_batch_solve(batch.handle, len(items), ctypes.cast(arr, ctypes.c_void_p),
                                 ctypes.byref(o), ctypes.byref(info),
                                 rel.ctypes.data_as(ctypes.c_void_p), _stream())
    if not (code == BIE_OK or (allow_noconv and code == BIE_ENOCONV)):
        _check(code)
    res = [o_.t().contiguous() if it[2] is None else o_ for o_, it in zip(outs, items)]
    return res, info.as_dict(), rel


class bie_server_config(ctypes.Structure):
    _fields_ = [("hbm_budget_bytes", ctypes.c_longlong), ("max_systems", ctypes.c_int),
                ("max_cycles", ctypes.c_int), ("opts", bie_opts)]


class bie_request_info(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int), ("cycles", ctypes.c_int), ("queue_s", ctypes.c_double),
                ("latency_s", ctypes.c_double), ("rel_residual", ctypes.c_double),
                ("inflight", ctypes.c_int), ("footprint_bytes", ctypes.c_longlong)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class Server:
    """Owns a bie_server (worker thread with continuous batching). Inputs and outputs are host
    numpy arrays; geometries must stay alive while their requests are in flight."""

    def __init__(self, opts=None, hbm_budget_bytes=0, max_systems=0, max_cycles=200):
        cfg = bie_server_config()
        cfg.hbm_budget_bytes = int(hbm_budget_bytes)
        cfg.max_systems = int(max_systems)
        cfg.max_cycles = int(max_cycles)
        cfg.opts = opts if opts is not None else default_opts()
        h = ctypes.c_void_p()
        _check(lib().bie_server_create(ctypes.byref(cfg), ctypes.byref(h)))
        self.handle = h
        self._bufs = {}

    def submit(self, g, kind, inp):
        """inp: [nrhs, N] charges (kind 0) or [nrhs, 3N] (F, T) (kind 1) -> ticket."""
        width = g.N if kind == 0 else 3 * g.N
        a = np.ascontiguousarray(np.atleast_2d(inp), dtype=np.float64)
        if a.shape[-1] != width:
            raise ValueError(f"input width {a.shape[-1]} != {width}")
        out = np.empty_like(a)
        t = ctypes.c_longlong()
        _check(lib().bie_server_submit(self.handle, g.handle, int(kind), a.shape[0],
                                       a.ctypes.data_as(ctypes.c_void_p),
                                       out.ctypes.data_as(ctypes.c_void_p), ctypes.byref(t)))
        self._bufs[t.value] = (a, out)
        return t.value

    def wait(self, ticket, timeout=-1.0, raise_on_error=True):
        """-> (output array, info dict); raises on failure other than non-convergence unless
        raise_on_error is False (then info["status"] carries the code)."""
        info = bie_request_info()
        code = lib().bie_server_wait(self.handle, ctypes.c_longlong(ticket), float(timeout),
                                     ctypes.byref(info))
        if code != BIE_OK and (raise_on_error or ticket not in self._bufs):
            _check(code)
        a, out = self._bufs.pop(ticket)
        return out, info.as_dict()

    def inject_failure(self, cycles=1):
        """Testing hook: the next `cycles` worker cycles fail (bie_server_inject_failure)."""
        _check(lib().bie_server_inject_failure(self.handle, int(cycles)))

    def stats(self):
        v = [ctypes.c_longlong() for _ in range(4)]
        _check(lib().bie_server_stats(self.handle, *[ctypes.byref(x) for x in v]))
        return dict(zip(("requests", "solves", "cycles", "peak_bytes"), [x.value for x in v]))

    def close(self):
        if getattr(self, "handle", None):
            lib().bie_server_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
