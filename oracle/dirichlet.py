"""Dense trapezoidal Nystrom oracle for the capacitance and resistance problems, float64 (test
infrastructure only; see oracle/__init__.py).

The paper's numerical section tests the elastance (mobility) solver against an independent solve
of the inverse problem: prescribe conductor potentials phi_j (rigid motions v_j, omega_j), solve
the capacitance (resistance) problem for the charges q_j (forces and torques F_j, T_j) and the
value at infinity u_inf, feed those to the elastance (mobility) solver and recover the prescribed
data. The paper leaves the capacitance and resistance equations to the literature (Mikhlin;
Power and Miranda). The formulations used here are the classical completed double layers.

Capacitance (the Dirichlet problem of the introduction: u harmonic outside the conductors,
u = phi_j on Gamma_j, u bounded at infinity, so that u -> u_inf and sum_j q_j = 0 with
q_j = -int_{Gamma_j} du/dn ds):
    u = D[mu] + sum_j q~_j G_R(x, z_j),   q~_j = int_{Gamma_j} mu ds,
  with the double layer D[mu](x) = int dG/dn_y(x, y) mu(y) ds_y, G = -(1/2pi) log|x - y|,
  G_R(x, z) = -(1/2pi) log(|x - z| / R), z_j a point inside body j and R a length scale. The
  exterior limit of D is (1/2 I + D), so the boundary condition gives the second-kind equation
    (1/2 I + D + C) mu = f,   (C mu)(x) = sum_j G_R(x, z_j) int_{Gamma_j} mu ds,
  which is uniquely solvable when R differs from the logarithmic capacity of the union of the
  curves (here R = twice the diagonal of the nodes' bounding box; capacity <= half the diameter).
  D[mu] carries no charge (its normal derivative is continuous and it is harmonic inside each
  body), so body j carries the charge q~_j. Such a solution grows like
  -(sum q~ / 2pi) log(|x| / R). Bounded solution: solve with f = phi (per body) and with f = 1;
  with beta = sum q~[phi] / sum q~[1],
    u = u[phi] - beta (u[1] - 1),  q = q~[phi] - beta q~[1],  u_inf = beta,
  and the density of u is mu[phi] - beta mu[1] (its G_R constants cancel since sum q = 0).

Resistance (u = v_j + omega_j (x - x^c_j)^perp on Gamma_j, viscosity 1, u bounded at infinity,
sum_j F_j = 0):
    u = Dcal[mu] + sum_j [ Gcal_R(x, z_j) a_j + t_j (x - z_j)^perp / (4 pi |x - z_j|^2) ],
    a_j = int_{Gamma_j} mu ds,   t_j = int_{Gamma_j} ((y - z_j)^perp, mu(y)) ds_y,
  with the Stokes double layer Dcal[mu](x) = (1/pi) int (r.n_y)(r.mu(y)) r / |r|^4 ds_y,
  r = x - y, the Stokeslet Gcal_R(x, z) = (1/4pi) (-log(|x - z| / R) I + d d^T / |d|^2),
  d = x - z (the single-layer kernel of the mobility problem), and the rotlet, whose torque is
  t_j (a cylinder of radius a rotating at omega needs t = 4 pi a^2 omega). Dcal reproduces minus
  any rigid motion inside a body and zero outside, so (1/2 I + Dcal) annihilates rigid motions on
  each curve; the Stokeslet and rotlet completion removes that null space. Dcal carries no force
  and no torque, so body j exerts the force a_j and, about its centroid x^c_j, the torque
  T_j = t_j + (z_j - x^c_j) x a_j. Bounded solution: solve with the prescribed data and with the
  uniform velocities e_x and e_y; beta in R^2 solves [sum a[e_x], sum a[e_y]] beta = sum a[data];
  then F = a[data] - beta_1 a[e_x] - beta_2 a[e_y] (likewise t and the density) and
  u_inf = beta.

Diagonal entries are the smooth limits of the kernels along the curve: dG/dn_y -> -kappa/(4pi)
and (1/pi)(r.n_y) r r^T / |r|^4 -> -(kappa/2pi) tau tau^T. Vector densities are node-major.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg

from . import nystrom as ny

TWO_PI = 2.0 * np.pi


def scale_length(geo):
    """R of the completion: twice the diagonal of the nodes' bounding box."""
    dx = geo["x"].max() - geo["x"].min()
    dy = geo["y"].max() - geo["y"].min()
    return 2.0 * float(np.sqrt(dx * dx + dy * dy))


def _centres(geo, interior):
    return ny.interior_points(geo, interior)


# ------------------------------------------------------------------------------------------
# Capacitance
# ------------------------------------------------------------------------------------------

def laplace_D(geo):
    """Nystrom matrix of D: D[i, k] = w_k (1/2pi) (x_i - x_k).n_k / |x_i - x_k|^2, and the
    smooth limit -kappa_i w_i / (4 pi) on the diagonal."""
    r1 = geo["x"][:, None] - geo["x"][None, :]
    r2 = geo["y"][:, None] - geo["y"][None, :]
    rr = r1 * r1 + r2 * r2
    np.fill_diagonal(rr, 1.0)
    rn = r1 * geo["nx"][None, :] + r2 * geo["ny"][None, :]
    D = (1.0 / TWO_PI) * rn / rr * geo["w"][None, :]
    np.fill_diagonal(D, -geo["kappa"] * geo["w"] / (4.0 * np.pi))
    return D


def laplace_completion(geo, interior=None, R=None):
    """C[i, k] = w_k G_R(x_i, z_{body(k)})."""
    R = scale_length(geo) if R is None else R
    z = _centres(geo, interior)[geo["body"]]
    d = np.hypot(geo["x"][:, None] - z[None, :, 0], geo["y"][:, None] - z[None, :, 1])
    return -(1.0 / TWO_PI) * np.log(d / R) * geo["w"][None, :]


def capacitance_operator(geo, interior=None, R=None):
    return 0.5 * np.eye(geo["M"]) + laplace_D(geo) + laplace_completion(geo, interior, R)


def capacitance_solve(geo, phi, interior=None, R=None, lu=None):
    """Conductor potentials phi [N] or [nrhs, N] -> charges q (same shape), u_inf ([] or
    [nrhs]) and the density mu of the bounded solution; also the raw systems."""
    phi = np.asarray(phi, dtype=np.float64)
    one = phi.ndim == 1
    phi = np.atleast_2d(phi)
    if lu is None:
        lu = scipy.linalg.lu_factor(capacitance_operator(geo, interior, R))
    f = np.concatenate([phi[:, geo["body"]], np.ones((1, geo["M"]))])
    mus = scipy.linalg.lu_solve(lu, f.T).T
    qt = np.stack([np.bincount(geo["body"], weights=geo["w"] * m, minlength=geo["N"])
                   for m in mus])
    beta = qt[:-1].sum(1) / qt[-1].sum()
    q = qt[:-1] - beta[:, None] * qt[-1][None, :]
    mu = mus[:-1] - beta[:, None] * mus[-1][None, :]
    if one:
        q, beta, mu = q[0], beta[0], mu[0]
    return dict(q=q, u_inf=beta, mu=mu, mu_systems=mus, charges_systems=qt, f=f)


def capacitance_matrix(geo, interior=None, R=None):
    """C with column j = q for phi = e_j (eq. capeq)."""
    return capacitance_solve(geo, np.eye(geo["N"]), interior, R)["q"].T.copy()


def double_layer(geo, density, points):
    """D[density](p) at off-curve points p [P, 2]."""
    p = np.asarray(points, dtype=np.float64).reshape(-1, 2)
    r1 = p[:, 0:1] - geo["x"][None, :]
    r2 = p[:, 1:2] - geo["y"][None, :]
    k = (r1 * geo["nx"][None, :] + r2 * geo["ny"][None, :]) / (r1 * r1 + r2 * r2)
    return (1.0 / TWO_PI) * (k * geo["w"][None, :]) @ density


def capacitance_field(geo, res, points, interior=None):
    """u(p) = D[mu](p) + sum_j q_j G(p, z_j) + u_inf for a bounded solution `res` (one rhs)."""
    p = np.asarray(points, dtype=np.float64).reshape(-1, 2)
    z = _centres(geo, interior)
    d = np.hypot(p[:, 0:1] - z[None, :, 0], p[:, 1:2] - z[None, :, 1])
    return double_layer(geo, res["mu"], p) - (1.0 / TWO_PI) * np.log(d) @ res["q"] + res["u_inf"]


# ------------------------------------------------------------------------------------------
# Resistance
# ------------------------------------------------------------------------------------------

def stokes_D(geo):
    """Nystrom matrix of Dcal on node-major vectors: block [i, k] (2x2) is
    w_k (1/pi) (r.n_k) r r^T / |r|^4 with r = x_i - x_k; diagonal block
    -(kappa_i / 2 pi) w_i tau_i tau_i^T."""
    M = geo["M"]
    r1 = geo["x"][:, None] - geo["x"][None, :]
    r2 = geo["y"][:, None] - geo["y"][None, :]
    rr = r1 * r1 + r2 * r2
    np.fill_diagonal(rr, 1.0)
    rn = r1 * geo["nx"][None, :] + r2 * geo["ny"][None, :]
    c = (1.0 / np.pi) * rn / (rr * rr) * geo["w"][None, :]
    D = np.empty((M, 2, M, 2))
    D[:, 0, :, 0] = c * r1 * r1
    D[:, 0, :, 1] = c * r1 * r2
    D[:, 1, :, 0] = c * r2 * r1
    D[:, 1, :, 1] = c * r2 * r2
    idx = np.arange(M)
    dg = -(geo["kappa"] / TWO_PI) * geo["w"]
    t = (geo["tx"], geo["ty"])
    for a in range(2):
        for b in range(2):
            D[idx, a, idx, b] = dg * t[a] * t[b]
    return D.reshape(2 * M, 2 * M)


def stokes_completion(geo, interior=None, R=None):
    """Block [i, k] = w_k [Gcal_R(x_i, z_j) + (x_i - z_j)^perp ((x_k - z_j)^perp)^T
    / (4 pi |x_i - z_j|^2)], j = body(k)."""
    M = geo["M"]
    R = scale_length(geo) if R is None else R
    z = _centres(geo, interior)[geo["body"]]
    d1 = geo["x"][:, None] - z[None, :, 0]
    d2 = geo["y"][:, None] - z[None, :, 1]
    dd = d1 * d1 + d2 * d2
    lg = 0.5 * np.log(dd / (R * R))
    s1 = -(geo["y"] - z[:, 1])  # (x_k - z_j)^perp
    s2 = geo["x"] - z[:, 0]
    p1, p2 = -d2, d1  # (x_i - z_j)^perp
    w = geo["w"][None, :] / (4.0 * np.pi)
    C = np.empty((M, 2, M, 2))
    C[:, 0, :, 0] = w * (-lg + d1 * d1 / dd + p1 * s1[None, :] / dd)
    C[:, 0, :, 1] = w * (d1 * d2 / dd + p1 * s2[None, :] / dd)
    C[:, 1, :, 0] = w * (d2 * d1 / dd + p2 * s1[None, :] / dd)
    C[:, 1, :, 1] = w * (-lg + d2 * d2 / dd + p2 * s2[None, :] / dd)
    return C.reshape(2 * M, 2 * M)


def resistance_operator(geo, interior=None, R=None):
    return 0.5 * np.eye(2 * geo["M"]) + stokes_D(geo) + stokes_completion(geo, interior, R)


def rigid_data(geo, VW):
    """Boundary velocity v_j + omega_j (x - x^c_j)^perp, node-major [.., 2M], from
    VW = (v_1x, v_1y, omega_1, v_2x, ...) of shape [3N] or [nrhs, 3N]."""
    VW = np.asarray(VW, dtype=np.float64)
    lead = VW.shape[:-1]
    VW = VW.reshape(lead + (geo["N"], 3))
    b = geo["body"]
    u1 = VW[..., b, 0] + VW[..., b, 2] * geo["px"]
    u2 = VW[..., b, 1] + VW[..., b, 2] * geo["py"]
    return np.stack([u1, u2], -1).reshape(lead + (2 * geo["M"],))


def _force_moments(geo, mu, interior):
    """Per body: a_j = sum_k w_k mu_k and t_j = sum_k w_k ((x_k - z_j)^perp, mu_k)."""
    z = _centres(geo, interior)[geo["body"]]
    m = mu.reshape(-1, 2)
    w, b, N = geo["w"], geo["body"], geo["N"]
    a1 = np.bincount(b, weights=w * m[:, 0], minlength=N)
    a2 = np.bincount(b, weights=w * m[:, 1], minlength=N)
    t = np.bincount(b, weights=w * (-(geo["y"] - z[:, 1]) * m[:, 0] + (geo["x"] - z[:, 0]) * m[:, 1]),
                    minlength=N)
    return np.stack([a1, a2, t], 1)


def resistance_solve(geo, VW, interior=None, R=None, lu=None):
    """Rigid motions VW [3N] or [nrhs, 3N] -> forces and torques FT (same layout,
    (F_1x, F_1y, T_1, ...), torque about the centroid), u_inf ([2] or [nrhs, 2]) and the
    density of the bounded solution; also the raw systems."""
    VW = np.asarray(VW, dtype=np.float64)
    one = VW.ndim == 1
    VW = np.atleast_2d(VW)
    if lu is None:
        lu = scipy.linalg.lu_factor(resistance_operator(geo, interior, R))
    M, N = geo["M"], geo["N"]
    ex = np.zeros(2 * M)
    ex[0::2] = 1.0
    ey = np.zeros(2 * M)
    ey[1::2] = 1.0
    f = np.concatenate([rigid_data(geo, VW), ex[None, :], ey[None, :]])
    mus = scipy.linalg.lu_solve(lu, f.T).T
    mom = np.stack([_force_moments(geo, m, interior) for m in mus])  # [sys, N, 3]
    tot = mom[:, :, 0:2].sum(1)  # [sys, 2]
    B = np.stack([tot[-2], tot[-1]], 1)  # columns: total force of the e_x and e_y solutions
    beta = np.linalg.solve(B, tot[:-2].T).T  # [nrhs, 2]
    m = mom[:-2] - beta[:, 0, None, None] * mom[-2][None] - beta[:, 1, None, None] * mom[-1][None]
    mu = mus[:-2] - beta[:, 0:1] * mus[-2][None, :] - beta[:, 1:2] * mus[-1][None, :]
    z = _centres(geo, interior)
    e1 = z[:, 0] - geo["xc"][:, 0]
    e2 = z[:, 1] - geo["xc"][:, 1]
    T = m[:, :, 2] + e1[None, :] * m[:, :, 1] - e2[None, :] * m[:, :, 0]
    FT = np.stack([m[:, :, 0], m[:, :, 1], T], 2).reshape(-1, 3 * N)
    if one:
        FT, beta, mu = FT[0], beta[0], mu[0]
    return dict(FT=FT, u_inf=beta, mu=mu, mu_systems=mus, moments_systems=mom, f=f)


def resistance_matrix(geo, interior=None, R=None):
    """Column j = (F, T) for the rigid motion e_j, ordered (v_1x, v_1y, omega_1, ...)."""
    return resistance_solve(geo, np.eye(3 * geo["N"]), interior, R)["FT"].T.copy()
