"""Seeded synthetic inputs: closed curves sampled at equispaced parameters, and right-hand sides.

This module is shared by the CPU oracle's tests and by the HIP path. It holds no arithmetic of the
integral-equation method itself: it only samples analytic parametrisations x(t), x'(t), x''(t) of
smooth, positively oriented closed curves (the setting of the elastance section of the paper),
places bodies with a guaranteed minimum gap, and draws charges q or forces and torques (F, T).

Curve families follow the paper's workloads:
  * discs (two-disc tests, numerical-examples section),
  * Fourier-perturbed circles r(t) = 1 + sum_k a_k sin(k t) (splash test),
  * ellipses (nanocomposite lattice),
  * starfish r(t) = r0 (1 + 0.3 cos 5t) (a smooth non-convex family of the same kind).

Node layout: bodies are contiguous; body b owns nodes body_ptr[b] .. body_ptr[b+1]-1, sampled at
t_k = 2 pi k / n_b, k = 0..n_b-1.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

SEEDS = {"elastance_small": 150701, "elastance_starfish": 150702, "mobility_ellipses": 150703,
         "batched": 150704, "serving": 150705, "fmm_items": 150706, "near_touching": 150707}


@dataclasses.dataclass
class Curves:
    """Samples of N closed curves, body-contiguous, all float64 [M] unless noted."""
    nodes_per_body: np.ndarray  # int32 [N]
    x: np.ndarray
    y: np.ndarray
    dx: np.ndarray
    dy: np.ndarray
    ddx: np.ndarray
    ddy: np.ndarray
    # per-body shape descriptors (for placement checks and documentation only)
    centers: np.ndarray  # float64 [N, 2]
    radii: np.ndarray  # float64 [N] bounding-circle radius about centers

    @property
    def nbodies(self) -> int:
        return int(self.nodes_per_body.shape[0])

    @property
    def M(self) -> int:
        return int(self.x.shape[0])

    @property
    def body_ptr(self) -> np.ndarray:
        bp = np.zeros(self.nbodies + 1, dtype=np.int32)
        np.cumsum(self.nodes_per_body, out=bp[1:])
        return bp

    def xy(self):
        return np.stack([self.x, self.y], 1)


# --------------------------------------------------------------------------------------------
# Analytic parametrisations. Each returns (x, y, x', y', x'', y'') at parameters t.
# --------------------------------------------------------------------------------------------

def _ellipse(t, cx, cy, a, b, theta):
    c, s = math.cos(theta), math.sin(theta)
    ex, ey = a * np.cos(t), b * np.sin(t)
    dex, dey = -a * np.sin(t), b * np.cos(t)
    ddex, ddey = -a * np.cos(t), -b * np.sin(t)
    rot = lambda u, v: (c * u - s * v, s * u + c * v)
    x, y = rot(ex, ey)
    dx, dy = rot(dex, dey)
    ddx, ddy = rot(ddex, ddey)
    return x + cx, y + cy, dx, dy, ddx, ddy


def _radial(t, cx, cy, r, dr, ddr, beta):
    """x(t) = c + r(t) (cos(t+beta), sin(t+beta)) with r, r', r'' given at t."""
    ct, st = np.cos(t + beta), np.sin(t + beta)
    x = cx + r * ct
    y = cy + r * st
    dx = dr * ct - r * st
    dy = dr * st + r * ct
    ddx = ddr * ct - 2.0 * dr * st - r * ct
    ddy = ddr * st + 2.0 * dr * ct - r * st
    return x, y, dx, dy, ddx, ddy


def disc_samples(n, cx, cy, R):
    t = 2.0 * np.pi * np.arange(n) / n
    one = np.ones_like(t)
    return _radial(t, cx, cy, R * one, 0.0 * one, 0.0 * one, 0.0)


def ellipse_samples(n, cx, cy, a, b, theta):
    t = 2.0 * np.pi * np.arange(n) / n
    return _ellipse(t, cx, cy, a, b, theta)


def starfish_samples(n, cx, cy, r0, theta, amp=0.3, arms=5):
    t = 2.0 * np.pi * np.arange(n) / n
    r = r0 * (1.0 + amp * np.cos(arms * t))
    dr = -r0 * amp * arms * np.sin(arms * t)
    ddr = -r0 * amp * arms * arms * np.cos(arms * t)
    return _radial(t, cx, cy, r, dr, ddr, theta)


def fourier_samples(n, cx, cy, coeffs, beta):
    """r(t) = 1 + sum_k a_k sin(k t), k = 1..len(coeffs) (splash-test curves)."""
    t = 2.0 * np.pi * np.arange(n) / n
    r = np.ones_like(t)
    dr = np.zeros_like(t)
    ddr = np.zeros_like(t)
    for k, a in enumerate(coeffs, start=1):
        r += a * np.sin(k * t)
        dr += a * k * np.cos(k * t)
        ddr -= a * k * k * np.sin(k * t)
    return _radial(t, cx, cy, r, dr, ddr, beta)


def assemble(samples, centers, radii) -> Curves:
    npb = np.array([len(s[0]) for s in samples], dtype=np.int32)
    cat = [np.concatenate([s[j] for s in samples]).astype(np.float64) for j in range(6)]
    return Curves(npb, *cat, centers=np.asarray(centers, dtype=np.float64).reshape(-1, 2),
                  radii=np.asarray(radii, dtype=np.float64))


# --------------------------------------------------------------------------------------------
# Paper geometries
# --------------------------------------------------------------------------------------------

def two_discs(d, n):
    """Two unit discs centred at (-1-d/2, 0) and (1+d/2, 0) (two-disc tests)."""
    c = 1.0 + 0.5 * d
    s = [disc_samples(n, -c, 0.0, 1.0), disc_samples(n, c, 0.0, 1.0)]
    return assemble(s, [[-c, 0.0], [c, 0.0]], [1.0, 1.0])


def single_disc(n, R=1.0, cx=0.0, cy=0.0):
    return assemble([disc_samples(n, cx, cy, R)], [[cx, cy]], [R])


# Splash-test geometry: centres, rotations and Fourier coefficients as printed in the paper's
# splash-test tables (used as printed, including the two entries outside the stated range).
SPLASH_CENTERS = [(-1.2, 0.0), (1.2, 0.0), (0.0, -2.2), (-1.2, -4.4), (1.2, -4.4)]
SPLASH_BETA = [math.pi, 0.0, math.pi / 8, 3 * math.pi / 4, -math.pi / 4]
SPLASH_COEFFS = np.array([
    [0.012065, 0.017038, 0.070082, 0.029959, 0.012613],
    [0.064385, 0.041668, 0.094629, 0.069290, 0.004017],
    [0.006234, 0.011991, 0.046520, 0.005102, 0.07413],
    [0.049028, 0.022743, 0.038905, 0.067634, 0.052361],
    [0.030608, 0.035266, 0.043884, 0.089215, 0.084973],
    [0.081641, 0.10864, 0.030143, 0.097489, 0.002916],
    [0.099718, 0.087338, 0.084480, 0.004693, 0.081962],
    [0.042460, 0.096291, 0.008018, 0.055024, 0.020443],
    [0.076748, 0.053323, 0.069852, 0.085238, 0.069016],
    [0.084684, 0.040564, 0.047617, 0.070539, 0.056950],
    [0.016811, 0.085034, 0.015078, 0.069771, 0.051020],
    [0.040454, 0.016044, 0.050553, 0.051137, 0.092286],
]).T  # [5 bodies, 12 modes]


def splash(n):
    s, radii = [], []
    for j in range(5):
        cx, cy = SPLASH_CENTERS[j]
        s.append(fourier_samples(n, cx, cy, SPLASH_COEFFS[j], SPLASH_BETA[j]))
        radii.append(1.0 + SPLASH_COEFFS[j].sum())
    return assemble(s, SPLASH_CENTERS, radii)


# --------------------------------------------------------------------------------------------
# Randomised ensembles
# --------------------------------------------------------------------------------------------

def _jittered_grid(rng, count, cols, pitch, jitter):
    rows = -(-count // cols)
    slots = [(i, j) for j in range(rows) for i in range(cols)][:count]
    c = np.array([[i * pitch, j * pitch] for i, j in slots], dtype=np.float64)
    c += rng.uniform(-jitter, jitter, size=c.shape)
    return c


def _min_gap(centers, radii):
    n = len(radii)
    if n < 2:
        return np.inf
    d = np.sqrt(((centers[:, None, :] - centers[None, :, :]) ** 2).sum(-1))
    g = d - radii[:, None] - radii[None, :]
    g[np.arange(n), np.arange(n)] = np.inf
    return float(g.min())


def random_ellipses_box(rng, nbodies, n, gap, box=3.0, axes=(0.5, 1.0)):
    """Semi-axes a, b ~ U[axes] independently, random rotation, random sequential placement in
    [-box, box]^2 with bounding-circle gap >= gap (4-ellipse elastance workload)."""
    centers, radii, s = [], [], []
    while len(s) < nbodies:
        a, b = rng.uniform(*axes, size=2)
        th = rng.uniform(0.0, 2.0 * np.pi)
        rad = max(a, b)
        for _ in range(10000):
            c = rng.uniform(-box, box, size=2)
            if all(np.hypot(*(c - c2)) - rad - r2 >= gap for c2, r2 in zip(centers, radii)):
                break
        else:
            raise RuntimeError("placement failed; enlarge the box")
        centers.append(c)
        radii.append(rad)
        s.append(ellipse_samples(n, c[0], c[1], a, b, th))
    return assemble(s, centers, radii)


def starfish_grid(rng, nbodies, n, cols=40, pitch=1.8, jitter=0.1, r0=(0.2, 0.5)):
    """Starfish r(t) = r0 (1 + 0.3 cos 5t), r0 ~ U[r0], random rotation, jittered grid. With the
    defaults the bounding-circle gap is >= pitch - 2*jitter - 2*1.3*0.5 = 0.3."""
    c = _jittered_grid(rng, nbodies, cols, pitch, jitter)
    r0s = rng.uniform(*r0, size=nbodies)
    th = rng.uniform(0.0, 2.0 * np.pi, size=nbodies)
    s = [starfish_samples(n, c[i, 0], c[i, 1], r0s[i], th[i]) for i in range(nbodies)]
    return assemble(s, c, 1.3 * r0s)


def ellipse_grid(rng, nbodies, n, cols=15, pitch=2.4, jitter=0.1, a=(0.5, 1.0), ar=(1.0, 3.0)):
    """Ellipses with aspect ratio ~ U[ar], semi-major ~ U[a], random rotation, jittered grid;
    bounding-circle gap >= pitch - 2*jitter - 2*max(a) = 0.2 with the defaults."""
    c = _jittered_grid(rng, nbodies, cols, pitch, jitter)
    A = rng.uniform(*a, size=nbodies)
    AR = rng.uniform(*ar, size=nbodies)
    th = rng.uniform(0.0, 2.0 * np.pi, size=nbodies)
    s = [ellipse_samples(n, c[i, 0], c[i, 1], A[i], A[i] / AR[i], th[i]) for i in range(nbodies)]
    return assemble(s, c, A)


def mixed_grid(rng, nbodies, nodes, pitch=2.4, jitter=0.1):
    """Uneven ensemble: per body a random node count from `nodes` (array [N]), shape 50/50
    ellipse (semi-axes ~ U[0.5,1]) or starfish (r0 ~ U[0.35,0.75]); jittered square grid."""
    cols = max(1, int(math.ceil(math.sqrt(nbodies))))
    c = _jittered_grid(rng, nbodies, cols, pitch, jitter)
    s, radii = [], []
    for i in range(nbodies):
        th = rng.uniform(0.0, 2.0 * np.pi)
        if rng.uniform() < 0.5:
            a, b = rng.uniform(0.5, 1.0, size=2)
            s.append(ellipse_samples(int(nodes[i]), c[i, 0], c[i, 1], a, b, th))
            radii.append(max(a, b))
        else:
            r0 = rng.uniform(0.35, 0.75)
            s.append(starfish_samples(int(nodes[i]), c[i, 0], c[i, 1], r0, th))
            radii.append(1.3 * r0)
    return assemble(s, c, radii)


# --------------------------------------------------------------------------------------------
# Named workloads (sizes of the benchmark configurations)
# --------------------------------------------------------------------------------------------

def elastance_small(seed=SEEDS["elastance_small"]):
    """4 ellipse conductors, semi-axes ~ U[0.5,1], gap >= 0.5, 128 nodes each; q ~ N(0,1)."""
    rng = np.random.default_rng(seed)
    g = random_ellipses_box(rng, 4, 128, gap=0.5)
    q = rng.standard_normal(4)
    return g, q


def elastance_starfish(nbodies=1000, n=256, seed=SEEDS["elastance_starfish"]):
    """1000 starfish, r0 ~ U[0.2,0.5], 40x25 jittered grid (pitch 1.8), gap >= 0.3, 256 nodes
    each; q ~ N(0,1). Smaller `nbodies` gives a prefix-shaped instance of the same recipe."""
    rng = np.random.default_rng(seed)
    g = starfish_grid(rng, nbodies, n, cols=min(40, nbodies))
    q = rng.standard_normal(nbodies)
    return g, q


def mobility_ellipses(nbodies=200, n=512, seed=SEEDS["mobility_ellipses"]):
    """200 ellipses, aspect ratio ~ U[1,3], semi-major ~ U[0.5,1], 15-column jittered grid
    (pitch 2.4), gap >= 0.2, 512 nodes each; F ~ N(0,1)^2 with zero total, T ~ N(0,1)."""
    rng = np.random.default_rng(seed)
    g = ellipse_grid(rng, nbodies, n, cols=min(15, nbodies))
    F = rng.standard_normal((nbodies, 2))
    F -= F.mean(0, keepdims=True)
    T = rng.standard_normal(nbodies)
    FT = np.concatenate([F, T[:, None]], 1).reshape(-1)
    return g, FT


def batched_geometries(count=32, seed=SEEDS["batched"], nb_range=(8, 128), nodes_range=(2, 16)):
    """`count` independent geometries: N_g = round(exp U[ln 8, ln 128]) bodies, per-body nodes
    32*round(exp U[ln 2, ln 16]) in {64..512}, shapes 50/50; kinds alternate elastance/mobility."""
    rng = np.random.default_rng(seed)
    out = []
    for gi in range(count):
        N = int(round(math.exp(rng.uniform(math.log(nb_range[0]), math.log(nb_range[1])))))
        nodes = 32 * np.round(np.exp(rng.uniform(math.log(nodes_range[0]), math.log(nodes_range[1]),
                                                 size=N))).astype(np.int64)
        g = mixed_grid(rng, N, nodes)
        kind = "elastance" if gi % 2 == 0 else "mobility"
        out.append((kind, g))
    return out


def plate_samples(n, shift):
    """Capacitor plate of the nanocomposite application: a rounded bar of length 2.2 and
    thickness 0.2, centred at (0, shift), sampled at s_k = -pi/2 + pi (k - 1/2) / (n/2),
    k = 1..n (a full period of the parameter, so the trapezoidal rule applies). On
    s in [-pi/2, pi/2]: x = 1.1 (1 - (2/pi) a(s)), y = 0.1 erf(7 s), with the smoothed |s|
    a(s) = s erf(10 s) + exp(-100 s^2) / (10 sqrt(pi)) (so a' = erf(10 s)); the other half
    mirrors it, x(s) = -x(pi - s), y(s) = y(pi - s). Counterclockwise."""
    from scipy.special import erf
    half = n // 2
    s = -0.5 * math.pi + math.pi * (np.arange(1, n + 1) - 0.5) / half
    right = s <= 0.5 * math.pi
    u = np.where(right, s, math.pi - s)  # parameter on the right half
    k = 2.2 / math.pi
    a = u * erf(10 * u) + np.exp(-100 * u * u) / (10 * math.sqrt(math.pi))
    x = 1.1 * (1 - (2 / math.pi) * a)
    dx = -k * erf(10 * u)
    ddx = -k * (20 / math.sqrt(math.pi)) * np.exp(-100 * u * u)
    y = 0.1 * erf(7 * u)
    dy = 0.1 * (14 / math.sqrt(math.pi)) * np.exp(-49 * u * u)
    ddy = dy * (-98 * u)
    # mirrored half: x(s) = -x(pi - s) so x' = x'(u), x'' = -x''(u); y(s) = y(pi - s) so
    # y' = -y'(u), y'' = y''(u)
    x = np.where(right, x, -x)
    ddx = np.where(right, ddx, -ddx)
    dy = np.where(right, dy, -dy)
    return x, y + shift, dx, dy, ddx, ddy


def nanocomposite(m, A, plate_nodes=800, particle_nodes=600):
    """The nanocomposite capacitance workload: two plates (shifted copies of plate_samples at
    y = +1.1 and -1.1, conductors 0 and 1) and an m x 10 lattice of ellipses of area 0.002/m and
    aspect ratio A (x semi-axis over y semi-axis) centred at (-0.9 + 1.8 (k-1)/10, y_j), each
    sampled at 600 equispaced parameter values. Charges +1 and -1 on
    the plates, 0 elsewhere. Returns (curves, q).
    Row centres: the printed -0.9 + 1.8 (j-1)/m puts a single row 0.075 from the lower plate and
    reproduces none of the printed capacitances for m = 1; the centred rows
    -0.9 + 1.8 (j - 1/2)/m reproduce them (to the printed digits for A = 1), and are used."""
    samples = [plate_samples(plate_nodes, 1.1), plate_samples(plate_nodes, -1.1)]
    centers = [[0.0, 1.1], [0.0, -1.1]]
    radii = [1.1, 1.1]
    if m > 0:
        b = math.sqrt(0.002 / (m * math.pi * A))
        a = A * b
        for j in range(1, m + 1):
            for kk in range(1, 11):
                cx = -0.9 + 1.8 * (kk - 1) / 10
                cy = -0.9 + 1.8 * (j - 0.5) / m
                samples.append(ellipse_samples(particle_nodes, cx, cy, a, b, 0.0))
                centers.append([cx, cy])
                radii.append(max(a, b))
    q = np.zeros(len(samples))
    q[0], q[1] = 1.0, -1.0
    return assemble(samples, centers, radii), q


def random_charges(rng, N, nrhs=1):
    return rng.standard_normal((nrhs, N))


def random_forces(rng, N, nrhs=1, zero_total=True):
    F = rng.standard_normal((nrhs, N, 2))
    if zero_total:
        F -= F.mean(1, keepdims=True)
    T = rng.standard_normal((nrhs, N, 1))
    return np.concatenate([F, T], 2).reshape(nrhs, 3 * N)


def min_gap(g: Curves) -> float:
    return _min_gap(g.centers, g.radii)


def serving_sessions(n_requests, seed=SEEDS["serving"]):
    """Query sessions for the serving workload: each session is one geometry with
    N = round(exp U[ln 2, ln 500]) bodies of 32*k nodes (64..256), shapes 50/50 starfish/ellipse,
    kind 60/40 elastance/mobility, and 1-16 queries (one rhs each: q ~ N(0,1), or F ~ N(0,1)^2
    with zero total and T ~ N(0,1)). Sessions are added until n_requests queries exist."""
    rng = np.random.default_rng(seed)
    out, total = [], 0
    while total < n_requests:
        N = int(round(math.exp(rng.uniform(math.log(2), math.log(500)))))
        nodes = 32 * rng.integers(2, 9, size=N)
        c = mixed_grid(rng, N, nodes)
        kind = 0 if rng.uniform() < 0.6 else 1
        nq = int(min(rng.integers(1, 17), n_requests - total))
        if kind == 0:
            qs = [random_charges(rng, N) for _ in range(nq)]
        else:
            qs = [random_forces(rng, N) for _ in range(nq)]
        out.append((kind, c, qs))
        total += nq
    return out


def fmm_items(seed=SEEDS["fmm_items"]):
    """Items above the 32,768-node threshold of BIE_AUTO (so batches and the server send them
    through the FMM): 130 starfish x 256 nodes (33,280; two charge vectors q ~ N(0,1)) and 66
    ellipses x 512 nodes (33,792; two (F, T) vectors, F zero-sum), with the recipes of the
    1000-starfish and 200-ellipse workloads; plus two small direct items (3 ellipses x 128,
    elastance; a 5-body mixed grid, mobility) so that FMM and direct items share a batch."""
    rng = np.random.default_rng(seed)
    star = starfish_grid(rng, 130, 256, cols=13)
    ell = ellipse_grid(rng, 66, 512, cols=11)
    small_e = random_ellipses_box(rng, 3, 128, gap=0.5)
    small_m = mixed_grid(rng, 5, np.array([64, 96, 128, 160, 64]))
    return [("elastance", star, random_charges(rng, 130, 2)),
            ("mobility", ell, random_forces(rng, 66, 2)),
            ("elastance", small_e, random_charges(rng, 3, 1)),
            ("mobility", small_m, random_forces(rng, 5, 1))]


def near_touching_forces(seed=SEEDS["near_touching"]):
    """Two (F, T) vectors for the two unit discs at gap 0.005: one seeded F ~ N(0,1)^2 (not
    zero-sum), T ~ N(0,1), and one net-force-free pair F_1 = -F_2 = (1, 0), T = 0 (the
    squeeze motion that the lubrication gap resists)."""
    rng = np.random.default_rng(seed)
    a = random_forces(rng, 2, 1, zero_total=False)[0]
    b = np.array([1.0, 0.0, 0.0, -1.0, 0.0, 0.0])
    return np.stack([a, b])
