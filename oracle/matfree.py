"""Matrix-free float64 oracle (test infrastructure only; see oracle/__init__.py).

The dense oracle's operators (oracle/nystrom.py) applied by the plain C loops of
oracle/matfree.c, for node counts where the dense matrix does not fit in memory, and solved with
scipy's restarted GMRES (a library routine used as one step) to a relative residual of 1e-13.
Geometry, incident densities and outputs reuse oracle.nystrom's definitions.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np
import scipy.sparse.linalg as spla

from . import nystrom as ny

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "matfree.c")
_LIB = os.path.join(_HERE, "libmatfree.so")
_lib = None


def build(force=True):
    """Compile oracle/matfree.c with gcc (plain -O2, no fast-math, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        build(force=False)  # compiles when missing or older than the source
        _lib = ctypes.CDLL(_LIB)
    return _lib


def _d(a):
    return np.ascontiguousarray(a, dtype=np.float64).ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _i(a):
    return np.ascontiguousarray(a, dtype=np.int32).ctypes.data_as(ctypes.POINTER(ctypes.c_int))


class _Keep:
    """Keeps contiguous copies alive for the duration of a C call."""

    def __init__(self):
        self.refs = []

    def d(self, a):
        a = np.ascontiguousarray(a, dtype=np.float64)
        self.refs.append(a)
        return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))

    def i(self, a):
        a = np.ascontiguousarray(a, dtype=np.int32)
        self.refs.append(a)
        return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int))


def set_threads(n):
    """OpenMP threads of the oracle's loops (for timing); returns the number in use."""
    return int(lib().oracle_set_threads(ctypes.c_int(n)))


def laplace_apply(geo, mu, with_L=True, rows=None):
    """(1/2 I + K + L) mu (with_L) or (1/2 I + K) mu, at all nodes or at `rows`."""
    k = _Keep()
    nrows = 0 if rows is None else len(rows)
    out = np.empty(geo["M"] if rows is None else nrows)
    lib().oracle_laplace_apply(
        ctypes.c_int(geo["M"]), ctypes.c_int(geo["N"]), k.i(geo["body"]), k.d(geo["x"]),
        k.d(geo["y"]), k.d(geo["nx"]), k.d(geo["ny"]), k.d(geo["w"]), k.d(geo["kappa"]), k.d(mu),
        ctypes.c_int(int(with_L)), None if rows is None else k.i(rows), ctypes.c_int(nrows),
        out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    return out


def stokes_apply(geo, mu, with_L=True, rows=None):
    """(1/2 I + Kcal + L) mu on node-major vectors [2M], at all nodes or at `rows` -> [2*len]."""
    k = _Keep()
    nrows = 0 if rows is None else len(rows)
    out = np.empty(2 * (geo["M"] if rows is None else nrows))
    lib().oracle_stokes_apply(
        ctypes.c_int(geo["M"]), ctypes.c_int(geo["N"]), k.i(geo["body"]), k.d(geo["x"]),
        k.d(geo["y"]), k.d(geo["nx"]), k.d(geo["ny"]), k.d(geo["w"]), k.d(geo["kappa"]),
        k.d(geo["px"]), k.d(geo["py"]), k.d(mu), ctypes.c_int(int(with_L)),
        None if rows is None else k.i(rows), ctypes.c_int(nrows),
        out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    return out


def single_layer(geo, dens, points):
    k = _Keep()
    p = np.ascontiguousarray(points, dtype=np.float64).reshape(-1, 2)
    out = np.empty(len(p))
    lib().oracle_laplace_single_layer(ctypes.c_int(geo["M"]), k.d(geo["x"]), k.d(geo["y"]),
                                      k.d(geo["w"]), k.d(dens), ctypes.c_int(len(p)), k.d(p),
                                      out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    return out


def stokes_velocity_vorticity(geo, dens, points):
    k = _Keep()
    p = np.ascontiguousarray(points, dtype=np.float64).reshape(-1, 2)
    out = np.empty((len(p), 3))
    lib().oracle_stokes_single_layer(ctypes.c_int(geo["M"]), k.d(geo["x"]), k.d(geo["y"]),
                                     k.d(geo["w"]), k.d(dens), ctypes.c_int(len(p)), k.d(p),
                                     out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    return out


def _gmres(apply, f, tol, restart, maxiter):
    n = f.shape[0]
    op = spla.LinearOperator((n, n), matvec=apply, dtype=np.float64)
    its = [0]

    def cb(_):
        its[0] += 1

    x, info = spla.gmres(op, f, rtol=tol, atol=0.0, restart=restart, maxiter=maxiter,
                         callback=cb, callback_type="pr_norm")
    if info != 0:
        raise RuntimeError(f"oracle GMRES did not converge (info={info})")
    return x, its[0]


def elastance_solve(geo, q, interior=None, tol=1e-13, restart=100, maxiter=20):
    """Matrix-free version of nystrom.elastance_solve for one charge vector q [N]."""
    sigma = ny.incident_charge(geo, q)
    f = -laplace_apply(geo, sigma, with_L=False)
    mu, its = _gmres(lambda v: laplace_apply(geo, v), f, tol, restart, maxiter)
    phi = single_layer(geo, mu + sigma, ny.interior_points(geo, interior))
    return dict(phi=phi, mu=mu, sigma=sigma, f=f, iters=its)


def mobility_solve(geo, FT, interior=None, tol=1e-13, restart=100, maxiter=20):
    """Matrix-free version of nystrom.mobility_solve for one (F, T) vector [3N]."""
    rho = ny.incident_traction(geo, FT)
    f = -stokes_apply(geo, rho, with_L=False)
    mu, its = _gmres(lambda v: stokes_apply(geo, v), f, tol, restart, maxiter)
    pts = ny.interior_points(geo, interior)
    uvo = stokes_velocity_vorticity(geo, mu + rho, pts)
    d = pts - geo["xc"]
    v = uvo[:, :2] - uvo[:, 2:3] * np.stack([-d[:, 1], d[:, 0]], 1)
    VW = np.concatenate([v, uvo[:, 2:3]], 1).reshape(-1)
    return dict(VW=VW, mu=mu, rho=rho, f=f, iters=its)
