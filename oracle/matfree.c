/* Matrix-free float64 oracle (test infrastructure only; see oracle/__init__.py).
 *
 * Plain double loops over (target, source) pairs, one OpenMP thread per block of targets and a
 * fixed source order per target, for node counts where the dense Nystrom matrix does not fit.
 * The operators are those of the dense oracle (oracle/nystrom.py), written out again:
 *
 *   Laplace (eq. ModRep2):  out_i = 1/2 mu_i + sum_{k != i} w_k dG/dn_x(x_i, x_k) mu_k
 *                                  - w_i kappa_i mu_i / (4 pi) + [with_L] sum_{k in body(i)} w_k mu_k
 *     with dG/dn_x(x, y) = -(1/2pi) (x - y).n_x / |x - y|^2.
 *   Stokes (eq. ModRep2Stokes): out_i = 1/2 mu_i + sum_{k != i} w_k n_{i,l} T_{a b l}(x_i, x_k) mu_{k,b}
 *                                  - w_i (kappa_i / 2pi) tau_i (tau_i . mu_i)
 *                                  + [with_L] (F_b + p_i tq_b),  F_b = sum w mu,  tq_b = sum w p . mu
 *     with T_{abl} = -(1/pi) r_a r_b r_l / |r|^4 and p = (x - x^c)^perp.
 *
 * Rows: if rows != NULL only the listed targets are computed (out has nrows entries, or 2*nrows
 * for Stokes); otherwise all M targets.
 */
#include <math.h>
#include <omp.h>
#include <stdlib.h>

/* Threads of the loops below (n >= 1); returns the number in use afterwards. Timing only. */
int oracle_set_threads(int n) {
  if (n >= 1) omp_set_num_threads(n);
  return omp_get_max_threads();
}

#define PI 3.14159265358979323846

static void body_sums_laplace(int M, int N, const int *body, const double *w, const double *mu,
                              double *m) {
  for (int b = 0; b < N; ++b) m[b] = 0.0;
  for (int k = 0; k < M; ++k) m[body[k]] += w[k] * mu[k];
}

void oracle_laplace_apply(int M, int N, const int *body, const double *x, const double *y,
                          const double *nx, const double *ny, const double *w,
                          const double *kappa, const double *mu, int with_L, const int *rows,
                          int nrows, double *out) {
  double *m = (double *)calloc((size_t)N, sizeof(double));
  body_sums_laplace(M, N, body, w, mu, m);
  int T = rows ? nrows : M;
#pragma omp parallel for schedule(dynamic, 16)
  for (int t = 0; t < T; ++t) {
    int i = rows ? rows[t] : t;
    double s = 0.0;
    for (int k = 0; k < M; ++k) {
      if (k == i) continue;
      double r1 = x[i] - x[k], r2 = y[i] - y[k];
      double rr = r1 * r1 + r2 * r2;
      s += w[k] * mu[k] * (r1 * nx[i] + r2 * ny[i]) / rr;
    }
    double v = 0.5 * mu[i] - s / (2.0 * PI) - w[i] * kappa[i] * mu[i] / (4.0 * PI);
    if (with_L) v += m[body[i]];
    out[t] = v;
  }
  free(m);
}

void oracle_stokes_apply(int M, int N, const int *body, const double *x, const double *y,
                         const double *nx, const double *ny, const double *w, const double *kappa,
                         const double *px, const double *py, const double *mu, int with_L,
                         const int *rows, int nrows, double *out) {
  double *F1 = (double *)calloc((size_t)N, sizeof(double));
  double *F2 = (double *)calloc((size_t)N, sizeof(double));
  double *TQ = (double *)calloc((size_t)N, sizeof(double));
  for (int k = 0; k < M; ++k) {
    F1[body[k]] += w[k] * mu[2 * k];
    F2[body[k]] += w[k] * mu[2 * k + 1];
    TQ[body[k]] += w[k] * (px[k] * mu[2 * k] + py[k] * mu[2 * k + 1]);
  }
  int T = rows ? nrows : M;
#pragma omp parallel for schedule(dynamic, 16)
  for (int t = 0; t < T; ++t) {
    int i = rows ? rows[t] : t;
    double s1 = 0.0, s2 = 0.0;
    for (int k = 0; k < M; ++k) {
      if (k == i) continue;
      double r1 = x[i] - x[k], r2 = y[i] - y[k];
      double rr = r1 * r1 + r2 * r2;
      double rn = r1 * nx[i] + r2 * ny[i];
      double rm = r1 * mu[2 * k] + r2 * mu[2 * k + 1];
      double c = w[k] * rn * rm / (rr * rr);
      s1 += c * r1;
      s2 += c * r2;
    }
    /* unit tangent from the outward normal n = (tau_2, -tau_1) */
    double t1 = -ny[i], t2 = nx[i];
    double tm = t1 * mu[2 * i] + t2 * mu[2 * i + 1];
    double d = -w[i] * kappa[i] / (2.0 * PI);
    double o1 = 0.5 * mu[2 * i] - s1 / PI + d * t1 * tm;
    double o2 = 0.5 * mu[2 * i + 1] - s2 / PI + d * t2 * tm;
    if (with_L) {
      int b = body[i];
      o1 += F1[b] + px[i] * TQ[b];
      o2 += F2[b] + py[i] * TQ[b];
    }
    out[2 * t] = o1;
    out[2 * t + 1] = o2;
  }
  free(F1);
  free(F2);
  free(TQ);
}

/* S[dens](p_j) = -(1/2pi) sum_k w_k dens_k log|p_j - x_k| */
void oracle_laplace_single_layer(int M, const double *x, const double *y, const double *w,
                                 const double *dens, int P, const double *p, double *out) {
#pragma omp parallel for schedule(dynamic, 1)
  for (int j = 0; j < P; ++j) {
    double s = 0.0;
    for (int k = 0; k < M; ++k) {
      double r1 = p[2 * j] - x[k], r2 = p[2 * j + 1] - y[k];
      s += w[k] * dens[k] * log(sqrt(r1 * r1 + r2 * r2));
    }
    out[j] = -s / (2.0 * PI);
  }
}

/* Stokeslet velocity u(p_j) and half-vorticity omega(p_j) of the density dens (node-major):
 * u = (1/4pi) sum_k [-log|r| t_k + r (r . t_k) / |r|^2],  omega = -(1/4pi) sum_k (r x t_k)/|r|^2,
 * r = p_j - x_k, t_k = w_k dens_k.  out is [P][3] = (u1, u2, omega). */
void oracle_stokes_single_layer(int M, const double *x, const double *y, const double *w,
                                const double *dens, int P, const double *p, double *out) {
#pragma omp parallel for schedule(dynamic, 1)
  for (int j = 0; j < P; ++j) {
    double u1 = 0.0, u2 = 0.0, om = 0.0;
    for (int k = 0; k < M; ++k) {
      double r1 = p[2 * j] - x[k], r2 = p[2 * j + 1] - y[k];
      double rr = r1 * r1 + r2 * r2;
      double t1 = w[k] * dens[2 * k], t2 = w[k] * dens[2 * k + 1];
      double lg = log(sqrt(rr));
      double rt = (r1 * t1 + r2 * t2) / rr;
      u1 += -lg * t1 + r1 * rt;
      u2 += -lg * t2 + r2 * rt;
      om += (r1 * t2 - r2 * t1) / rr;
    }
    out[3 * j] = u1 / (4.0 * PI);
    out[3 * j + 1] = u2 / (4.0 * PI);
    out[3 * j + 2] = -om / (4.0 * PI);
  }
}
