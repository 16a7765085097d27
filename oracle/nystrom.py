"""Dense trapezoidal Nystrom oracle, float64 (test infrastructure only; see oracle/__init__.py).

The method (Rachh & Greengard):
  Elastance: u = S(mu + sigma) with sigma_i = q_i / |Gamma_i| (eq. sigma), and mu solving the
  completed interior-Neumann equation (1/2 I + K + L) mu = -(1/2 I + K) sigma (eq. ModRep2), where
  K is the normal derivative of the single layer at the target, dG/dn_x, with
  G(x, y) = -(1/2pi) log|x - y|, and (L_i mu)(x) = int_{Gamma_i} mu ds.
  Mobility: u = Scal(mu + rho) with rho_j = F_j/|Gamma_j| + T_j (x - x^c_j)^perp / W_j (eq. rho) and
  (1/2 I + Kcal + L) mu = -(1/2 I + Kcal) rho (eq. ModRep2Stokes), where
  (Kcal rho)_k(x) = n_{x,l} int T_{kml}(x, y) rho_m(y) ds_y with the stresslet
  T_{ijk} = -(1/pi) r_i r_j r_k / |r|^4, r = x - y (lemma with eq. SLnormaljumpStokes), and
  L_i mu = int mu ds + (x - x^c_i)^perp int ((y - x^c_i)^perp, mu) ds.

Discretisation readings (the paper uses Gauss-Legendre panels with GLQBX; here, as the
operator's own definition on smooth closed curves):
  * nodes t_k = 2 pi k / n_b, trapezoidal weights w_k = (2 pi / n_b) |x'(t_k)|;
  * the principal-value diagonal entries are the smooth limits of the kernels along the curve:
    dG/dn_x(x, y) -> -kappa(x) / (4 pi) and n_l T_{kml} -> -(kappa / 2 pi) tau_k tau_m,
    with kappa the signed curvature (positive on convex arcs of a positively oriented curve);
  * the outward normal of a positively oriented curve is n = (tau_2, -tau_1);
  * the centroid is the arc-length centroid x^c = (1/|Gamma|) int x ds (mobility problem
    statement), discretised as sum(w x) / sum(w);
  * phi_j and (v_j, omega_j) are read off inside each body, where u is constant, respectively a
    rigid motion (proofs of the two representation theorems): phi_j = S(mu + sigma)(p_j),
    omega_j = half the vorticity of Scal(mu + rho) at p_j, v_j = u(p_j) - omega_j (p_j - x^c_j)^perp.
Vector densities are stored node-major: entry 2k + a is component a of node k.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg

TWO_PI = 2.0 * np.pi


# ------------------------------------------------------------------------------------------
# Geometry (elastance problem statement; centroid of the mobility problem statement; eq. rho)
# ------------------------------------------------------------------------------------------

def geometry(nodes_per_body, x, y, dx, dy, ddx, ddy):
    """Per-node and per-body quadrature data of a body-contiguous node set."""
    npb = np.asarray(nodes_per_body, dtype=np.int64)
    N = len(npb)
    body = np.repeat(np.arange(N), npb)
    speed = np.hypot(dx, dy)
    tx, ty = dx / speed, dy / speed
    nx, ny = ty, -tx
    kappa = (dx * ddy - dy * ddx) / speed ** 3
    w = (TWO_PI / npb[body]) * speed
    length = np.bincount(body, weights=w, minlength=N)
    xc = np.bincount(body, weights=w * x, minlength=N) / length
    yc = np.bincount(body, weights=w * y, minlength=N) / length
    rx, ry = x - xc[body], y - yc[body]
    W = np.bincount(body, weights=w * (rx * rx + ry * ry), minlength=N)
    px, py = -ry, rx  # (x - x^c)^perp = (-(x2 - c2), x1 - c1)
    return dict(N=N, M=len(x), body=body, x=np.asarray(x, float), y=np.asarray(y, float),
                nx=nx, ny=ny, tx=tx, ty=ty, kappa=kappa, w=w, length=length,
                xc=np.stack([xc, yc], 1), W=W, px=px, py=py)


def geometry_of(curves):
    return geometry(curves.nodes_per_body, curves.x, curves.y, curves.dx, curves.dy,
                    curves.ddx, curves.ddy)


def _same_body(geo):
    b = geo["body"]
    return (b[:, None] == b[None, :]).astype(np.float64)


# ------------------------------------------------------------------------------------------
# Laplace: K (eq. IntegralEq and the K_{ij} definitions), L (eq. ModRep2), RHS, solve
# ------------------------------------------------------------------------------------------

def laplace_K(geo):
    """Nystrom matrix of K: K[i, k] = w_k dG/dn_x(x_i, x_k), diagonal by the smooth limit."""
    r1 = geo["x"][:, None] - geo["x"][None, :]
    r2 = geo["y"][:, None] - geo["y"][None, :]
    rr = r1 * r1 + r2 * r2
    np.fill_diagonal(rr, 1.0)
    rn = r1 * geo["nx"][:, None] + r2 * geo["ny"][:, None]
    K = -(1.0 / TWO_PI) * rn / rr * geo["w"][None, :]
    np.fill_diagonal(K, -geo["kappa"] * geo["w"] / (4.0 * np.pi))
    return K


def laplace_L(geo):
    """L[i, k] = w_k when nodes i and k lie on the same body, else 0."""
    return _same_body(geo) * geo["w"][None, :]


def laplace_operator(geo):
    return 0.5 * np.eye(geo["M"]) + laplace_K(geo) + laplace_L(geo)


def incident_charge(geo, q):
    """sigma at each node: q_i / |Gamma_i| (eq. sigma). q: [N] or [nrhs, N] -> [.., M]."""
    q = np.asarray(q, dtype=np.float64)
    return q[..., geo["body"]] / geo["length"][geo["body"]]


def laplace_rhs(geo, sigma, K=None):
    """Right-hand side -(1/2 I + K) sigma (eq. ModRep2)."""
    K = laplace_K(geo) if K is None else K
    return -(0.5 * sigma + sigma @ K.T)


def single_layer(geo, density, points):
    """S[density](p) = sum_k w_k G(p, x_k) density_k at off-curve points p [P, 2]."""
    p = np.asarray(points, dtype=np.float64).reshape(-1, 2)
    r = np.hypot(p[:, 0:1] - geo["x"][None, :], p[:, 1:2] - geo["y"][None, :])
    G = -(1.0 / TWO_PI) * np.log(r)
    return (density * geo["w"]) @ G.T


def interior_points(geo, interior=None):
    return geo["xc"] if interior is None else np.asarray(interior, dtype=np.float64).reshape(-1, 2)


def elastance_solve(geo, q, interior=None, lu=None):
    """Charges q [N] or [nrhs, N] -> potentials phi (same shape); also returns mu, sigma.

    phi_j = S(mu + sigma)(p_j) at an interior point p_j of body j (u is constant inside each
    conductor once (1/2 I + K) (mu + sigma) = 0)."""
    K = laplace_K(geo)
    A = 0.5 * np.eye(geo["M"]) + K + laplace_L(geo)
    lu = scipy.linalg.lu_factor(A) if lu is None else lu
    sigma = incident_charge(geo, q)
    f = laplace_rhs(geo, sigma, K)
    mu = scipy.linalg.lu_solve(lu, f.T).T
    pts = interior_points(geo, interior)
    dens = mu + sigma
    if dens.ndim == 1:
        phi = single_layer(geo, dens, pts)
    else:
        phi = np.stack([single_layer(geo, d, pts) for d in dens])
    return dict(phi=phi, mu=mu, sigma=sigma, f=f)


def elastance_matrix(geo, interior=None):
    """P with column j = phi for q = e_j (elastance problem statement)."""
    res = elastance_solve(geo, np.eye(geo["N"]), interior)
    return res["phi"].T.copy()


# ------------------------------------------------------------------------------------------
# Stokes: Kcal (eq. IntegralEqStokes and the Kcal_{ij} definitions), L (eq. ModRep2Stokes),
# incident traction (eq. rho), solve, outputs
# ------------------------------------------------------------------------------------------

def stokes_K(geo):
    """Nystrom matrix of Kcal on node-major vectors: block [i, k] (2x2) is
    w_k n_{i,l} T_{a b l}(x_i, x_k); diagonal block -(kappa_i / 2 pi) w_i tau_i tau_i^T."""
    M = geo["M"]
    r1 = geo["x"][:, None] - geo["x"][None, :]
    r2 = geo["y"][:, None] - geo["y"][None, :]
    rr = r1 * r1 + r2 * r2
    np.fill_diagonal(rr, 1.0)
    rn = r1 * geo["nx"][:, None] + r2 * geo["ny"][:, None]
    c = -(1.0 / np.pi) * rn / (rr * rr) * geo["w"][None, :]
    K = np.empty((M, 2, M, 2))
    K[:, 0, :, 0] = c * r1 * r1
    K[:, 0, :, 1] = c * r1 * r2
    K[:, 1, :, 0] = c * r2 * r1
    K[:, 1, :, 1] = c * r2 * r2
    idx = np.arange(M)
    d = -(geo["kappa"] / TWO_PI) * geo["w"]
    t = (geo["tx"], geo["ty"])
    for a in range(2):
        for b in range(2):
            K[idx, a, idx, b] = d * t[a] * t[b]
    return K.reshape(2 * M, 2 * M)


def stokes_L(geo):
    """L block [i, k] = [same body] w_k (I + p_i p_k^T), p = (x - x^c)^perp."""
    M = geo["M"]
    S = _same_body(geo) * geo["w"][None, :]
    p = (geo["px"], geo["py"])
    L = np.empty((M, 2, M, 2))
    for a in range(2):
        for b in range(2):
            L[:, a, :, b] = S * ((1.0 if a == b else 0.0) + p[a][:, None] * p[b][None, :])
    return L.reshape(2 * M, 2 * M)


def stokes_operator(geo):
    return 0.5 * np.eye(2 * geo["M"]) + stokes_K(geo) + stokes_L(geo)


def incident_traction(geo, FT):
    """rho at each node, node-major [.., 2M]: F_j / |Gamma_j| + T_j (x - x^c_j)^perp / W_j.
    FT is (F_1x, F_1y, T_1, F_2x, ...), shape [3N] or [nrhs, 3N]."""
    FT = np.asarray(FT, dtype=np.float64)
    lead = FT.shape[:-1]
    FT = FT.reshape(lead + (geo["N"], 3))
    b = geo["body"]
    F1, F2, T = FT[..., b, 0], FT[..., b, 1], FT[..., b, 2]
    L, W = geo["length"][b], geo["W"][b]
    rho = np.stack([F1 / L + T * geo["px"] / W, F2 / L + T * geo["py"] / W], -1)
    return rho.reshape(lead + (2 * geo["M"],))


def stokes_rhs(geo, rho, K=None):
    K = stokes_K(geo) if K is None else K
    return -(0.5 * rho + rho @ K.T)


def stokes_single_layer(geo, density, points):
    """Velocity Scal[density](p) = sum_k w_k G(p, x_k) density_k with the Stokeslet
    G_ij = (1/4pi)(-log|r| delta_ij + r_i r_j / |r|^2); density node-major [2M]; -> [P, 2]."""
    p = np.asarray(points, dtype=np.float64).reshape(-1, 2)
    t = density.reshape(-1, 2) * geo["w"][:, None]
    r1 = p[:, 0:1] - geo["x"][None, :]
    r2 = p[:, 1:2] - geo["y"][None, :]
    rr = r1 * r1 + r2 * r2
    lg = 0.5 * np.log(rr)
    rt = (r1 * t[None, :, 0] + r2 * t[None, :, 1]) / rr
    u1 = (-lg * t[None, :, 0] + r1 * rt).sum(1) / (4.0 * np.pi)
    u2 = (-lg * t[None, :, 1] + r2 * rt).sum(1) / (4.0 * np.pi)
    return np.stack([u1, u2], 1)


def stokes_half_vorticity(geo, density, points):
    """Half the vorticity (d u2/dx1 - d u1/dx2)/2 of Scal[density] at p; for the Stokeslet this
    is -(1/4pi) (r x f) / |r|^2 per source, r = p - x_k."""
    p = np.asarray(points, dtype=np.float64).reshape(-1, 2)
    t = density.reshape(-1, 2) * geo["w"][:, None]
    r1 = p[:, 0:1] - geo["x"][None, :]
    r2 = p[:, 1:2] - geo["y"][None, :]
    rr = r1 * r1 + r2 * r2
    cross = r1 * t[None, :, 1] - r2 * t[None, :, 0]
    return -(cross / rr).sum(1) / (4.0 * np.pi)


def rigid_motion(geo, density, interior=None):
    """(v_j, omega_j) of the rigid motion that u = Scal[density] performs inside body j."""
    pts = interior_points(geo, interior)
    u = stokes_single_layer(geo, density, pts)
    om = stokes_half_vorticity(geo, density, pts)
    d = pts - geo["xc"]
    v = u - om[:, None] * np.stack([-d[:, 1], d[:, 0]], 1)
    return np.concatenate([v, om[:, None]], 1).reshape(-1)  # (v1x, v1y, w1, v2x, ...)


def mobility_solve(geo, FT, interior=None, lu=None):
    """(F, T) [3N] or [nrhs, 3N] -> (v, omega) in the same layout; also returns mu, rho."""
    K = stokes_K(geo)
    A = 0.5 * np.eye(2 * geo["M"]) + K + stokes_L(geo)
    lu = scipy.linalg.lu_factor(A) if lu is None else lu
    rho = incident_traction(geo, FT)
    f = stokes_rhs(geo, rho, K)
    mu = scipy.linalg.lu_solve(lu, f.T).T
    dens = mu + rho
    if dens.ndim == 1:
        VW = rigid_motion(geo, dens, interior)
    else:
        VW = np.stack([rigid_motion(geo, d, interior) for d in dens])
    return dict(VW=VW, mu=mu, rho=rho, f=f)


def mobility_matrix(geo, interior=None):
    """M with column j = (v_1, omega_1, ...) for (F_1, T_1, ...) = e_j."""
    res = mobility_solve(geo, np.eye(3 * geo["N"]), interior)
    return res["VW"].T.copy()


# ------------------------------------------------------------------------------------------
# Diagnostics
# ------------------------------------------------------------------------------------------

def body_charge(geo, mu):
    """int_{Gamma_j} mu ds per body (the elastance constraints, eq. IntEqConstraints)."""
    return np.bincount(geo["body"], weights=geo["w"] * mu, minlength=geo["N"])


def body_force_torque(geo, mu):
    """(int mu ds, int (x - x^c)^perp . mu ds) per body (eqs. IntegralEqStokesForceConstraint and
    IntegralEqStokesTorqueConstraint); -> [N, 3]."""
    m = mu.reshape(-1, 2)
    b, w = geo["body"], geo["w"]
    f1 = np.bincount(b, weights=w * m[:, 0], minlength=geo["N"])
    f2 = np.bincount(b, weights=w * m[:, 1], minlength=geo["N"])
    t = np.bincount(b, weights=w * (geo["px"] * m[:, 0] + geo["py"] * m[:, 1]), minlength=geo["N"])
    return np.stack([f1, f2, t], 1)
