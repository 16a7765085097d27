/* bie2d.h - C ABI of the MI355X (gfx950) second-kind integral-equation library for the 2D
 * elastance (Laplace) and mobility (Stokes) problems of Rachh & Greengard, "Integral equation
 * methods for elastance and mobility problems in two dimensions".
 *
 * Problem (elastance section): N disjoint smooth closed curves Gamma_j, positively oriented,
 * outward normal n. Given charges q_j, find conductor potentials phi_j (phi = P q) with u
 * harmonic outside, u = phi_j on Gamma_j, -int_{Gamma_j} du/dn = q_j, u -> 0 at infinity.
 * Mobility section: given forces and torques (F_j, T_j) on rigid bodies in Stokes flow of
 * viscosity 1, find rigid motions (v_j, omega_j) about the arc-length centroid x^c_j
 * (U = M F, ordered (F_1, T_1, F_2, T_2, ...) -> (v_1, omega_1, ...)).
 *
 * Method: u = S(mu + sigma), sigma_j = q_j/|Gamma_j| (eq. sigma), with
 *     (1/2 I + K + L) mu = -(1/2 I + K) sigma                          (eq. ModRep2)
 * K = normal derivative of the single layer at the target, L_i mu = int_{Gamma_i} mu ds; and
 * u = Scal(mu + rho), rho_j = F_j/|Gamma_j| + T_j (x - x^c_j)^perp / W_j (eq. rho), with
 *     (1/2 I + Kcal + L) mu = -(1/2 I + Kcal) rho                      (eq. ModRep2Stokes)
 * Kcal = stresslet traction operator, L_i mu = int mu + (x - x^c_i)^perp int (y - x^c_i)^perp . mu.
 * Discretisation: trapezoidal Nystrom on t_k = 2 pi k / n_b, w_k = (2 pi / n_b)|x'(t_k)|;
 * diagonal entries are the smooth kernel limits -kappa/(4 pi) and -(kappa/2 pi) tau tau^T.
 *
 * Conventions for every call below
 *   - Pointers marked (device) are HIP device pointers on the geometry's device; (host) are host
 *     memory. The caller owns every buffer it passes; the library copies what it keeps.
 *   - `stream` is a hipStream_t (NULL = the null stream). All work is enqueued on it; calls that
 *     return results needed on the host (iteration counts, info) synchronise that stream.
 *   - Vector densities are node-major: entry 2k + a is component a of node k. Multiple
 *     right-hand sides are stacked: rhs r occupies [r * len, (r + 1) * len).
 *   - Return value: BIE_OK (0) or a negative error code; bie_last_error() gives the message of
 *     the most recent failure on the calling thread. Outputs are written only on BIE_OK (and on
 *     BIE_ENOCONV, where the last iterate is returned and info is filled).
 *   - Thread safety: distinct geometries may be used from distinct threads; calls that overlap
 *     on one geometry (it owns the workspace) race.
 */
#ifndef BIE2D_H
#define BIE2D_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define BIE_OK 0
#define BIE_EINVAL (-1)   /* bad sizes or pointers, non-finite input, clockwise curve */
#define BIE_ENOMEM (-2)   /* device allocation failed */
#define BIE_ENOCONV (-3)  /* GMRES did not reach the tolerance within max_iter */
#define BIE_EDEVICE (-4)  /* HIP runtime error */
#define BIE_ERESOLVE (-5) /* warning from bie_geom_create / bie_ctx_geom_create only: the geometry
                             WAS created (*out is valid and usable) but a curve is under-resolved
                             (its trapezoidal turning number sum_k kappa_k w_k misses 2 pi by more
                             than 1e-8 relative) or a node of one body lies closer than 3 node
                             spacings of another body to it (the trapezoidal rule on that body
                             then loses accuracy like exp(-2 pi d / h)); bie_last_error() names the
                             bodies. Results stay the exact solution of the discrete system; only
                             their distance to the continuum solution is at risk. */

#define BIE_FP64 0   /* every step in float64 */
#define BIE_MIXED 1  /* float32 far field in the late GMRES steps (or the inner solves of a
                        refinement: mixed_strategy). Direct: float32 pair sums (body-relative
                        coordinates, float64 accumulation across source bodies), float64
                        self-body blocks. FMM: float32 near field pair terms (float64
                        accumulation), expansions of about half the order, float32 for Laplace
                        (multipoles, M2M, M2L, evaluation), float64 for Stokes. Both: float64
                        diagonal, completion, Arnoldi and true residuals (float64 operator). */

/* How BIE_MIXED wins the float64 accuracy back:
 * BIE_MIXED_RELAXED  one float64 GMRES (float64 Arnoldi and residuals) whose steps apply the
 *                    BIE_MIXED operator once the estimated relative residual of every system it
 *                    applies to is below tol / eta, eta that apply's relative error (1e-7
 *                    direct, 5e-7 FMM, or for FMM Stokes ten times the fitted error of its
 *                    expansion length where that is larger; measured values rounded up):
 *                    the error a step's apply may carry grows as the residual it reduces
 *                    falls (relaxed inexact Krylov, Simoncini & Szyld 2003). The solve stops
 *                    only on the float64 true residual of a cycle start, so a cycle that the
 *                    float32 steps left short is followed by another. The rhs of one geometry
 *                    share each step's precision; the items of a batch choose theirs apart (at
 *                    most 1024 items; larger batches choose together).
 * BIE_MIXED_REFINE   iterative refinement: inner GMRES on the float32 operator to inner_tol (one
 *                    Gram-Schmidt pass), x += d, float64 residual, repeat (max_refine). */
#define BIE_MIXED_RELAXED 0
#define BIE_MIXED_REFINE 1

/* GMRES preconditioning (opts.precond). BIE_PRECOND_BLOCK: right preconditioning by an
 * approximate inverse of the operator's block diagonal, one block per body (its self
 * interactions: identity, diagonal limit, same-body double-layer pairs, completion), built once
 * per geometry and kind on the device. A block's inverse is 2 I plus a smooth part, formed on a
 * coarse grid of the curve (n itself up to 64 nodes, exact; else every s-th node, n / s the
 * largest divisor of n in [16, 64]) with full-weighting restriction and linear interpolation;
 * the coarse blocks are inverted in float32 and applied in float64. The solution is that of the
 * unpreconditioned system (the stopping tests use true float64 residuals of A x = f); the
 * iteration count falls when the bodies interact weakly (37 -> 12 steps for 1000 starfish at
 * gap >= 0.3, 64 -> 18 for 200 ellipses at gap >= 0.2). Elastance and mobility solves,
 * matrices, batches and the server (one launch applies every item's blocks); BIE_EINVAL for the
 * capacitance and resistance solves, with l2_scaling, and for a body of more than 2048 nodes or
 * with no such divisor (a server request on such a geometry fails with it). */
#define BIE_PRECOND_NONE 0
#define BIE_PRECOND_BLOCK 1

#define BIE_DIRECT 0 /* all-pairs direct summation */
#define BIE_FMM 1    /* 2D fast multipole method for the far field */
#define BIE_AUTO 2   /* FMM for geometries with more than 32768 nodes, else direct */

typedef struct bie_geom bie_geom; /* device-resident geometry + workspace (opaque) */

typedef struct {
  int precision;    /* BIE_FP64 | BIE_MIXED                                            */
  int method;       /* BIE_DIRECT | BIE_FMM | BIE_AUTO                                 */
  double tol;       /* target relative residual ||f - A mu|| / ||f|| (float64 apply)    */
  int restart;      /* GMRES restart length m (Krylov vectors per cycle)               */
  int max_iter;     /* cap on GMRES iterations summed over cycles and refinements      */
  double inner_tol; /* BIE_MIXED: relative tolerance of each inner float32-apply solve */
  int max_refine;   /* BIE_MIXED: cap on outer refinement steps                       */
  int fmm_order;    /* BIE_FMM: expansion order p (terms per expansion)               */
  int fmm_leaf;     /* BIE_FMM: mean nodes per leaf box the tree depth aims at; 0 = tuned:
                       the solves and batches take it from the autotuner (bie_autotune)
                       for the geometry's shape class, per precision; the server uses 64 */
  double viscosity; /* mobility / resistance: fluid viscosity > 0 (mobility problem
                       statement: viscosity 1 there). Velocities scale as 1/viscosity,
                       forces and torques as viscosity; densities do not change.        */
  double fmm_eps;   /* BIE_FMM: > 0 sets the expansion order from a target for the float64
                       apply's relative error (2-norm against direct summation): the
                       smallest p with K 0.45^p <= fmm_eps, K = 2.1e-3 (Laplace), 4.3e-2
                       (Stokes), a fit of measured errors at p = 16, 24, 32; clamped to
                       [8, 64] (1e-10: order 24 Laplace, 32 Stokes). 0 = use fmm_order   */
  int mixed_strategy; /* BIE_MIXED: BIE_MIXED_RELAXED (default) or BIE_MIXED_REFINE   */
  int precond;      /* BIE_PRECOND_NONE (default) or BIE_PRECOND_BLOCK: elastance and
                       mobility solves run GMRES on (A P) u = f with P an approximate inverse
                       of the bodies' self blocks, x = P u                                 */
  int l2_scaling;   /* 1: GMRES on the symmetrised system D A D^-1 (D mu) = D f with
                       D = diag(sqrt(w)) (the paper's L2 rescaling of the numerical
                       section): same solution, the stopping test then uses the discrete
                       L2 norm ||D r|| / ||D f||. Single-geometry solves only (the batch
                       and the server reject it).                                       */
} bie_opts;

typedef struct {
  int iters;             /* GMRES iterations (all cycles, all refinements; max over rhs)  */
  int refinements;       /* outer refinement steps (BIE_MIXED), else 0                     */
  int applies_fp64;      /* float64 operator applications                                 */
  int applies_fp32;      /* float32 far-field operator applications                        */
  double rel_residual;   /* final true relative residual, float64 apply (max over rhs)    */
  double seconds;        /* wall time of the call                                         */
  long long pairs;       /* pair interactions evaluated (direct: M^2 per apply per rhs)   */
  double net_charge_or_force[2]; /* solves: sum_j q_j (elastance; [1] = 0) or sum_j F_j
                                    (mobility) of the right-hand side with the largest
                                    magnitude. The paper requires both to vanish (eqs.
                                    ChargeConservation, NoNetForce); any value is accepted
                                    (see the solves) and reported here. */
} bie_info;

/* Message of the last failure on this thread (never NULL). */
const char *bie_last_error(void);

/* Fills *o with the defaults: BIE_FP64, BIE_DIRECT, tol 1e-12, restart 100, max_iter 500,
 * inner_tol 1e-6, max_refine 10, fmm_order 40, fmm_leaf 64, viscosity 1, fmm_eps 0,
 * mixed_strategy BIE_MIXED_RELAXED, l2_scaling 0. With BIE_FMM and BIE_MIXED the float32-apply
 * steps use order ceil(0.55 fmm_order) (about the square root of the accuracy); the near field
 * stays float64, the Laplace expansions (multipoles, M2M, M2L, evaluation) are float32, the
 * Stokes expansions stay float64 (their C' - conj(z) A' combination cancels). The float64
 * applies use the full order. fmm_order must lie in [4, 64]; the library rounds the order up
 * to a multiple of 8. */
int bie_default_opts(bie_opts *o);

/* ---- context: device, default options, owned geometries -------------------------------------
 * A context binds one HIP device and a set of default options. Geometries created through it
 * (bie_ctx_geom_create) live on its device, are owned by it until bie_geom_destroy (bie_destroy
 * destroys the ones left), and take the context's defaults wherever a call passes opts = NULL.
 * Every call on such a geometry makes the context's device current for its duration. A context
 * is used from one host thread at a time; bie_last_error() reports per thread, hence per
 * context. Geometries from bie_geom_create have no context: process defaults, the current
 * device at creation.
 * bie_create: device = HIP device ordinal (0 .. count - 1); defaults NULL = bie_default_opts.
 * Errors: BIE_EINVAL (NULL out, bad device ordinal or options), BIE_EDEVICE (no device). */
typedef struct bie_ctx bie_ctx;
int bie_create(bie_ctx **out, int device, const bie_opts *defaults);
int bie_destroy(bie_ctx *ctx);
int bie_ctx_defaults(const bie_ctx *ctx, bie_opts *out);
/* As bie_geom_create, on the context's device and owned by the context. */
int bie_ctx_geom_create(bie_ctx *ctx, int nbodies, const int32_t *nodes_per_body,
                        const double *curve, const double *interior, void *stream,
                        bie_geom **out);

/* ---- a1: geometry and quadrature (elastance section; eq. rho for W; centroid of the mobility
 * problem statement) ------------------------------------------------------------------------
 * nbodies        N >= 1
 * nodes_per_body (host) [N], each n_b >= 3; bodies are contiguous, M = sum n_b
 * curve          (device) [6][M] float64: x, y, x'(t), y'(t), x''(t), y''(t) at t_k = 2 pi k / n_b
 * interior       (device) [N][2] float64 points p_j inside body j at which phi_j, (v_j, omega_j)
 *                are read off, or NULL for the arc-length centroids
 * Computes on the device: outward normal n = (y', -x')/|x'|, curvature, weights
 * w_k = (2 pi / n_b)|x'(t_k)|, |Gamma_j|, x^c_j = sum w x / sum w, W_j = sum w |x - x^c_j|^2,
 * p_k = (x_k - x^c_j)^perp, float32 body-relative coordinates.
 * Errors: BIE_EINVAL for N < 1, n_b < 3, NULL curve, non-finite samples, a body whose signed
 * area is not positive (clockwise), or a read-off point (given, or the default centroid) that
 * is not inside its body's node polygon (winding number 1; phi and (v, omega) are read there,
 * where u is constant, resp. a rigid motion). BIE_ERESOLVE: created, with the warning above. */
int bie_geom_create(int nbodies, const int32_t *nodes_per_body, const double *curve,
                    const double *interior, void *stream, bie_geom **out);
/* The checks bie_geom_create applies, on host copies of its inputs (curve (host) [6][M],
 * interior (host) [N][2] or NULL), without a device: BIE_OK, BIE_EINVAL or BIE_ERESOLVE with
 * the same messages. */
int bie_curves_check(int nbodies, const int32_t *nodes_per_body, const double *curve,
                     const double *interior);
int bie_geom_destroy(bie_geom *g);
int bie_geom_sizes(const bie_geom *g, int *nbodies, int *M);
/* Copies the per-node quadrature data (device out [8][M]: x, y, nx, ny, w, kappa, px, py) and
 * per-body data (device out_body [4][N]: |Gamma|, xc, yc, W). Either may be NULL. */
int bie_geom_export(const bie_geom *g, double *out, double *out_body, void *stream);
/* Device bytes held by the geometry including its current workspace. */
long long bie_geom_device_bytes(const bie_geom *g);
/* Expansion order p (4..64) and maximum leaf population used by BIE_FMM applies on g (the solve
 * entry points set them from bie_opts). The quadtree for each order is built on first use and
 * kept with the geometry. */
int bie_geom_set_fmm(bie_geom *g, int order, int leaf);

/* ---- a3 + a4: the operator apply (eqs. ModRep2 / ModRep2Stokes) ----------------------------
 * out = (1/2 I + K + L) mu      (with_L = 1)  or  (1/2 I + K) mu  (with_L = 0)
 * Laplace: mu, out (device) [nrhs][M].  Stokes: (device) [nrhs][2M] node-major.
 * precision: BIE_FP64, or BIE_MIXED (float32 far field, float64 self blocks and terms).
 * method: BIE_DIRECT or BIE_FMM (expansion order and leaf size of the last solve on this geometry,
 * default 40 and 64). mu and out must not alias. */
int bie_laplace_apply(bie_geom *g, int precision, int method, int with_L, int nrhs,
                      const double *mu, double *out, void *stream);
int bie_stokes_apply(bie_geom *g, int precision, int method, int with_L, int nrhs,
                     const double *mu, double *out, void *stream);

/* ---- the same apply without allocation ----------------------------------------------------
 * For callers that cannot allocate device memory: code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc. Same result as bie_laplace_apply (kind 0) or
 * bie_stokes_apply (kind 1) with method BIE_DIRECT and the same arguments (it runs the same
 * kernels), but its workspace (strengths and far-field partial sums) is a fixed 64 MiB array in
 * device memory that the library holds per device for the life of the process; the call
 * allocates and frees nothing (and records no profiling events). The workspace it needs,
 * 12 nrhs len + 8 nsplit R len bytes (len = M or 2M, R = 8 Laplace / 4 Stokes rhs per pass,
 * nsplit <= 64 source splits of the geometry), must fit: else BIE_EINVAL, with the size in the
 * message. All calls on one device share that array: calls that overlap on one device (any
 * geometry, any stream) race and must be ordered by the caller. Nothing in it needs clearing
 * between calls (every entry a call reads, it writes first). The geometry itself must already
 * exist (bie_geom_create allocates). */
int bie_apply_noalloc(bie_geom *g, int kind, int precision, int with_L, int nrhs,
                      const double *mu, double *out, void *stream);

/* ---- a2: incident densities and right-hand sides -------------------------------------------
 * sigma_k = q_j/|Gamma_j| (eq. sigma); f = -(1/2 I + K) sigma.  q (device) [nrhs][N];
 * sigma, f (device) [nrhs][M]; either output may be NULL.
 * rho_k = F_j/|Gamma_j| + T_j p_k / W_j (eq. rho); f = -(1/2 I + Kcal) rho.
 * FT (device) [nrhs][3N] as (F_1x, F_1y, T_1, ...); rho, f (device) [nrhs][2M]. */
int bie_elastance_rhs(bie_geom *g, int nrhs, const double *q, double *sigma, double *f,
                      void *stream);
int bie_mobility_rhs(bie_geom *g, int nrhs, const double *FT, double *rho, double *f,
                     void *stream);

/* ---- a7: outputs read off inside the bodies (u constant, resp. a rigid motion, inside) ------
 * phi_j = S(dens)(p_j) = -(1/2 pi) sum_k w_k dens_k log|p_j - x_k|. dens (device) [nrhs][M],
 * phi (device) [nrhs][N].
 * Stokes: u = Scal(dens), omega_j = half the vorticity at p_j, v_j = u(p_j) - omega_j
 * (p_j - x^c_j)^perp. dens (device) [nrhs][2M], VW (device) [nrhs][3N] as (v_1x, v_1y, w_1, ...). */
int bie_laplace_potential(bie_geom *g, int nrhs, const double *dens, double *phi, void *stream);
int bie_stokes_rigid_motion(bie_geom *g, int nrhs, const double *dens, double *VW, void *stream);

/* ---- a6 + the whole path: solves ------------------------------------------------------------
 * Elastance: q (device) [nrhs][N] -> phi (device) [nrhs][N]; mu_out (device) [nrhs][M] or NULL.
 * Mobility: FT (device) [nrhs][3N] -> VW (device) [nrhs][3N]; mu_out (device) [nrhs][2M] or NULL.
 * Any q is accepted: for sum q != 0 (or sum F != 0) the same representation gives the unique
 * field with u + (Q/2 pi) log|x| -> 0 (its potential is grounded at infinity in that sense);
 * info->net_charge_or_force reports the net charge, resp. force. Mobility velocities are for
 * opts.viscosity (mu_out, the traction density, does not depend on it).
 * opts NULL = defaults (the context's for a context geometry); info may be NULL.
 * Errors: BIE_EINVAL for a non-finite q, F or T (the input is read once to check it), bad
 * sizes or options. BIE_ENOCONV: outputs hold the last iterate. */
int bie_elastance_solve(bie_geom *g, int nrhs, const double *q, double *phi, double *mu_out,
                        const bie_opts *opts, bie_info *info, void *stream);
int bie_mobility_solve(bie_geom *g, int nrhs, const double *FT, double *VW, double *mu_out,
                       const bie_opts *opts, bie_info *info, void *stream);

/* ---- a8: assembly of P and M column by column (elastance / mobility statements) -------------
 * P (device) [N][N] column-major: column j = phi for q = e_j.
 * Mmat (device) [3N][3N] column-major: column j = (v_1, omega_1, ...) for (F_1, T_1, ...) = e_j.
 * The identity right-hand-side block is solved as one multi-rhs solve in chunks of at most
 * `max_rhs_per_pass` columns (0 = library default). */
int bie_elastance_matrix(bie_geom *g, double *P, int max_rhs_per_pass, const bie_opts *opts,
                         bie_info *info, void *stream);
int bie_mobility_matrix(bie_geom *g, double *Mmat, int max_rhs_per_pass, const bie_opts *opts,
                        bie_info *info, void *stream);

/* ---- off-surface evaluation: the field everywhere (the representation formulas) ------------
 * The solution is a layer potential of the total density everywhere, not only on the curves:
 * u = S[mu + sigma] for the elastance problem (eq. TotRepresentation; constant, = phi_j, inside
 * conductor j) and u = Scal[mu + rho] for the mobility problem (eq. TotRepresentationStokes;
 * the rigid motion of body j inside it), the fields the paper draws as contours and velocity
 * plots. Given the solve's input (q [nrhs][N], resp. (F, T) [nrhs][3N]) and its density mu
 * (mu_out of the solve: [nrhs][M], resp. [nrhs][2M] node-major), these evaluate that field at
 * npts points pts [2*npts] (x0, y0, x1, ...): u [nrhs][npts], resp. velocities [nrhs][npts][2]
 * (viscosity 1). All buffers are device memory. The trapezoidal rule is spectrally accurate for
 * points a few node spacings away from every curve; closer points get no near-singular
 * correction (the paper uses QBX there) and lose accuracy. npts = 0 is a no-op. */
int bie_elastance_field(bie_geom *g, int nrhs, const double *q, const double *mu, int npts,
                        const double *pts, double *u, void *stream);
int bie_mobility_field(bie_geom *g, int nrhs, const double *FT, const double *mu, int npts,
                       const double *pts, double *u, void *stream);

/* ---- the inverse problems: capacitance and resistance (the paper's cross-tests) -------------
 * The numerical section checks the elastance (mobility) solver by first solving the capacitance
 * (resistance) problem for prescribed potentials phi_j (rigid motions v_j + omega_j
 * (x - x^c_j)^perp), which gives the charges q_j (forces F_j and torques T_j about x^c_j) and the
 * value at infinity u_inf, then feeding those to the elastance (mobility) solver; the prescribed
 * data come back up to u_inf (introduction: the Dirichlet problem with u bounded at infinity; the
 * cross-test protocol of the numerical section). The paper cites the standard equations for
 * these problems; the ones used here are the completed double layers:
 *   Laplace: u = D[mu] + sum_j G_R(x, z_j) int_{Gamma_j} mu,
 *            D[mu](x) = int dG/dn_y(x, y) mu(y) ds_y, G = -(1/2pi) log|x - y|,
 *            G_R(x, z) = -(1/2pi) log(|x - z| / R);   (1/2 I + D + C) mu = f on the curves.
 *   Stokes:  u = Dcal[mu] + sum_j [Gcal_R(x, z_j) a_j + t_j (x - z_j)^perp / (4 pi |x - z_j|^2)],
 *            Dcal[mu](x) = (1/pi) int (r.n_y)(r.mu) r / |r|^4 ds_y (r = x - y),
 *            Gcal_R(x, z) = (1/4pi)(-log(|d| / R) I + d d^T / |d|^2), d = x - z,
 *            a_j = int_{Gamma_j} mu, t_j = int_{Gamma_j} ((y - z_j)^perp, mu);  viscosity 1.
 * z_j is body j's interior point (bie_geom_create; default its centroid), which must lie inside
 * the body; R is twice the diagonal of the nodes' bounding box. Nystrom discretisation on the
 * trapezoidal nodes, diagonal by the smooth kernel limits (-kappa/4pi; -(kappa/2pi) tau tau^T).
 * All applies and solves are float64 with direct summation (opts.precision and opts.method are
 * ignored).
 *
 * bie_laplace_dl_apply / bie_stokes_dl_apply: out = (1/2 I + D + C) mu (with_completion = 0 drops
 * C), mu and out (device) [nrhs][M], resp. [nrhs][2M] node-major; mu and out must not alias.
 *
 * bie_capacitance_solve: phi (device) [nrhs][N] -> q (device) [nrhs][N] (sum_j q_j = 0,
 * q_j = -int_{Gamma_j} du/dn, the charge of the elastance problem) and u_inf (device) [nrhs].
 * bie_resistance_solve: VW (device) [nrhs][3N] (v_1x, v_1y, omega_1, ...) -> FT (device)
 * [nrhs][3N] (F_1x, F_1y, T_1, ...; sum_j F_j = 0, the force and torque of the mobility problem)
 * and u_inf (device) [nrhs][2].
 * Each solves nrhs + 1 (Laplace) or nrhs + 2 (Stokes) systems in one multi-rhs GMRES: the data
 * and the uniform boundary values 1, resp. e_x and e_y, whose combination is the bounded
 * solution. mu_out (device) [nrhs][M], resp. [nrhs][2M], or NULL receives that solution's
 * density; then u = D[mu_out] + sum_j q_j G(x, z_j) + u_inf (Stokes: Dcal[mu_out] plus the
 * Stokeslet F_j and the rotlet of t_j = T_j - (z_j - x^c_j) x F_j at z_j, plus u_inf).
 * opts NULL = defaults; info may be NULL; BIE_ENOCONV: outputs from the last iterate. */
int bie_laplace_dl_apply(bie_geom *g, int with_completion, int nrhs, const double *mu, double *out,
                         void *stream);
int bie_stokes_dl_apply(bie_geom *g, int with_completion, int nrhs, const double *mu, double *out,
                        void *stream);
int bie_capacitance_solve(bie_geom *g, int nrhs, const double *phi, double *q, double *u_inf,
                          double *mu_out, const bie_opts *opts, bie_info *info, void *stream);
int bie_resistance_solve(bie_geom *g, int nrhs, const double *VW, double *FT, double *u_inf,
                         double *mu_out, const bie_opts *opts, bie_info *info, void *stream);

/* ---- batched solves over several geometries (many systems in one lock-step GMRES) ---------
 * Every right-hand side of every item is one system; all systems advance together, one batched
 * operator apply per Arnoldi step, each with its own Hessenberg matrix and convergence test, so
 * an item's iterates do not depend on the other items of the batch (reductions are per system
 * and deterministic; with BIE_MIXED_RELAXED the rhs of one item share each step's precision, and
 * batches of more than 1024 items share it across items). Used for P and M of many geometries at once and by the server.
 * kind: 0 = elastance (in [nrhs][N] charges, out [nrhs][N] potentials), 1 = mobility (in
 * [nrhs][3N] (F, T), out [nrhs][3N] (v, omega)). in == NULL means the identity block: nrhs must
 * equal N (kind 0) or 3N (kind 1) and out receives P or M column by column (column-major).
 * rel_residual (host [nitems] or NULL) receives each item's worst final relative residual. */
typedef struct bie_batch bie_batch; /* solver workspace reused across calls (opaque) */
typedef struct {
  bie_geom *g;
  int kind;
  int nrhs;
  const double *in; /* (device) or NULL */
  double *out;      /* (device) */
} bie_batch_item;
int bie_batch_create(bie_batch **out);
int bie_batch_destroy(bie_batch *b);
int bie_batch_solve(bie_batch *b, int nitems, const bie_batch_item *items, const bie_opts *opts,
                    bie_info *info, double *rel_residual, void *stream);

/* ---- serving: continuous batching of elastance and mobility requests ------------------------
 * A worker thread (own HIP stream, default priority, created with the server: BIE_EDEVICE
 * from bie_server_create when the device cannot be used) keeps a set of requests in flight. At every
 * GMRES-cycle boundary it (1) computes each active request's true residual f - A x with the
 * float64 operator, (2) retires the requests whose systems all reached opts.tol (potentials or
 * rigid motions read off inside the bodies, copied to the caller's host buffer), (3) admits
 * queued requests in arrival order while their solver state fits in hbm_budget_bytes, and
 * (4) runs one Arnoldi cycle of at most `restart` steps over all remaining systems with the
 * opts.precision operator (with BIE_MIXED each cycle is one float64 refinement step around a
 * float32 far field). Requests that arrive while others are on the GPU join at the next cycle
 * boundary; a request's arithmetic does not depend on the other requests in flight.
 * Geometries (and their FMM trees) stay resident with their bie_geom and must outlive the
 * requests that use them; several requests may share one geometry.
 * Callers: any host thread; submit copies the input; out must stay valid until wait returns. */
typedef struct bie_server bie_server;
typedef struct {
  long long hbm_budget_bytes; /* device bytes for solver state of requests in flight (0 = none) */
  int max_systems;            /* cap on systems (rhs) in flight, 0 = no cap                     */
  int max_cycles;             /* a request still above tol after this many cycles fails         */
  bie_opts opts;              /* precision, method, tol, inner_tol, restart (cycle length), fmm */
} bie_server_config;
typedef struct {
  int status;          /* BIE_OK, BIE_ENOCONV, or an error code                              */
  int cycles;          /* GMRES cycles the request took part in                             */
  double queue_s;      /* submit -> admitted                                                 */
  double latency_s;    /* submit -> result in the caller's buffer                           */
  double rel_residual; /* worst final relative residual over the request's rhs               */
  int inflight;        /* requests in flight right after this one was admitted (itself too) */
  long long footprint_bytes; /* bytes charged for it: its solver state plus, for the first
                                request on its geometry and kind, the geometry's FMM tree and
                                apply workspace (charged once while any of its requests run) */
} bie_request_info;
int bie_server_create(const bie_server_config *cfg, bie_server **out);
/* kind 0: in [nrhs][N] charges -> out [nrhs][N] potentials; kind 1: in [nrhs][3N] (F, T) ->
 * out [nrhs][3N] (v, omega); in and out are host pointers. *ticket identifies the request. */
int bie_server_submit(bie_server *srv, bie_geom *g, int kind, int nrhs, const double *in,
                      double *out, long long *ticket);
/* Blocks until the request is done (timeout_s < 0: no timeout); BIE_EINVAL on timeout or an
 * unknown ticket. */
int bie_server_wait(bie_server *srv, long long ticket, double timeout_s, bie_request_info *info);
/* Totals since creation: requests completed, rhs solved, cycles run, peak bytes in flight. */
int bie_server_stats(bie_server *srv, long long *requests, long long *solves, long long *cycles,
                     long long *peak_bytes);
/* Drains the queue and in-flight work, stops the worker and frees the server. */
int bie_server_destroy(bie_server *srv);
/* Testing hook for the error path: the next `cycles` worker cycles fail with BIE_EDEVICE
 * before doing any work. A failing cycle fails only the requests in flight in it (their wait
 * returns the error); the worker stays up and serves the requests that come after. */
int bie_server_inject_failure(bie_server *srv, int cycles);

/* ---- instrumentation (not a step of the method) ---------------------------------------------
 * When enabled, the library records a pair of HIP events on the launch stream around every
 * launch of the kernel classes below and accumulates, per class, the number of launches, their
 * summed durations and the work units they process (target-source pairs times rhs unless the
 * class says otherwise).
 * bie_profile_enable(1) clears the counters; bie_profile_read() waits for the recorded events
 * of that class and returns the totals. bie_profile_select(mask) limits the recording to the
 * classes whose bit (1 << class) is set (default: all), so that timing one class adds no events
 * around the others. bie_profile_sample(every) records only every every-th launch of each class
 * (default 1, every launch; every < 1 is BIE_EINVAL): an event marker on a stream leaves the GPU
 * idle for a few microseconds, so sampling keeps the timed work close to an unprofiled run; the
 * launch count and the totals then cover the sampled launches. Process-wide; not thread safe. */
#define BIE_K_FAR_LAPLACE_F32 0 /* float32 far-field sweep, Laplace            */
#define BIE_K_FAR_LAPLACE_F64 1 /* float64 far-field sweep, Laplace            */
#define BIE_K_FAR_STOKES_F32 2  /* float32 far-field sweep, Stokes             */
#define BIE_K_FAR_STOKES_F64 3  /* float64 far-field sweep, Stokes             */
#define BIE_K_EPILOGUE 4        /* self blocks + diagonal + completion + sum   */
#define BIE_K_FMM 5             /* FMM far field, all its kernels; units: M^2 per rhs (equivalent pairs) */
#define BIE_K_FMM_M2L 6         /* FMM multipole-to-local; units: interaction-list entries (box pairs) per set */
#define BIE_K_FMM_EVAL 7        /* FMM local evaluation + near field; units: near-field pairs */
#define BIE_K_DOUBLE_LAYER 8    /* double-layer applies of the capacitance / resistance solves; units: M^2 per rhs */
#define BIE_K_FMM_M2L_F32 9     /* float32 M2L of the mixed Laplace apply; units as BIE_K_FMM_M2L */
#define BIE_K_FMM_NEAR_F32 10   /* float32 near field of the mixed applies; units: pairs        */
#define BIE_K_PRECOND 11        /* block preconditioner apply; units: its multiply-adds         */
#define BIE_K_COUNT 12
/* ---- autotuning of the FMM leaf size -------------------------------------------------------
 * The leaf population trades near-field pair work against expansion work; the best value
 * depends on the kernel, the precision and the node density. bie_autotune times the operator
 * apply of `kind` at `precision` with nrhs right-hand sides (up to 8, resp. 4, per pass) on g
 * for leaf sizes 24, 32, 48, 64, 96, 128 (each with its own tree; the losers' trees are
 * freed), for the float64 apply and, with BIE_MIXED, also for the float32 inner apply, and
 * stores the fastest per shape class (kind, precision, rhs per pass, floor(log2 M),
 * floor(log2 M/N)) in the geometry's context (process-wide for a geometry without one). A
 * class already in the cache is not timed again. The leaf sizes are set on g and returned.
 * Solves with opts.fmm_leaf = 0 and the FMM call it themselves. bie_autotune_stats: classes
 * tuned and cache hits (ctx NULL: the process cache). */
int bie_autotune(bie_geom *g, int kind, int precision, int nrhs, int *leaf_fp64,
                 int *leaf_mixed, void *stream);
int bie_autotune_stats(const bie_ctx *ctx, long long *tunings, long long *hits);

/* Expansion length *terms (coefficients per expansion, a multiple of 8) of the FMM applies of a
 * solve of kind 0 (Laplace) or 1 (Stokes) with options *opts: the float64 applies
 * (precision BIE_FP64) or the BIE_MIXED ones (about half the order). Host only; BIE_EINVAL for
 * invalid options. */
int bie_fmm_terms(const bie_opts *opts, int kind, int precision, int *terms);

/* Graph replay of the solves' Arnoldi steps (default off: measured slower than stream
 * launches on the 1000-starfish solve, about 6 us more per step). A single-geometry solve runs each
 * Arnoldi step (the operator apply, with the FMM's near field forked onto a second stream and
 * joined back, and the Gram-Schmidt kernels) eagerly the first time, captures it as a HIP graph
 * and replays that graph in later cycles and solves of the same configuration; a different
 * configuration or a reallocated workspace drops the captured steps. Results are bitwise the
 * same either way. Process-wide. Batches and the server run their steps eagerly. */
int bie_set_graphs(int on);
/* Graph statistics of a geometry's solver: steps captured and steps replayed since creation. */
int bie_geom_graph_stats(const bie_geom *g, long long *captured, long long *replayed);

int bie_profile_enable(int on);
int bie_profile_select(unsigned mask);
int bie_profile_sample(int every);
int bie_profile_read(int kclass, long long *launches, double *ms_total, long long *pairs);

#ifdef __cplusplus
}
#endif

#endif /* BIE2D_H */
