/*
 * Lax-Friedrichs sweeping with fifth-order WENO derivatives for one point
 * source on a 2D grid (test infrastructure of the HB tables; compiled with
 * gcc and called from oracle/hb_tables.py, never linked with the library).
 *
 * The discrete equations (Sec. 2.3 of the paper: the factored eikonal
 * eq. faceik and the transport recurrence eq. equVs, solved by LxF-WENO
 * sweeping with values near the source held at their Taylor expansions):
 *
 *   grid      nx x ny points, spacing h, point (i, j) at index i + nx j;
 *   p-, p+    one-sided x-derivatives at (i, j): the Jiang-Peng WENO5 forms
 *             (linear weights 0.1, 0.6, 0.3; epsilon given, h^2 by the
 *             caller: with 1e-6 the weights of the transport sweeps can
 *             switch back and forth without end) where the
 *             seven points i-3 .. i+3 lie in the grid, else first-order
 *             differences (u_i - u_{i-1})/h and (u_{i+1} - u_i)/h, the
 *             missing one replaced by the other at the first and last
 *             point; likewise q-, q+ in y;
 *   eikonal   unknown tb (tau = tt * tb, tt = n0 |r - r0| given with its
 *             gradient), H = |tt grad tb + tb grad tt|,
 *             LxF  Hh = H(mean p, mean q) - ax (p+ - p-)/2 - ay (q+ - q-)/2,
 *             update tb += omega (n - Hh) h / (ax + ay);
 *   transport unknown v, b . grad v + c v = f with b = 2 grad tau^2,
 *             LxF  Hh = b_x mean p + b_y mean q + c v - ax (p+ - p-)/2
 *                       - ay (q+ - q-)/2,
 *             update v += omega (f - Hh) h / (ax + ay);
 *   ax, ay    the viscosities, given per point (bounds of |dH/dp|, |dH/dq|
 *             chosen by the caller);
 *   points with fixed[k] != 0 are never updated.
 * Gauss-Seidel sweeps in the four alternating orderings (i, j ascending /
 * descending) repeat until the largest update of a full round is below tol
 * or maxrounds rounds have run; the return value is the number of rounds,
 * *last the largest update of the last round.
 */
#include <math.h>
#include <stddef.h>

static double weno5(double v1, double v2, double v3, double v4, double v5, double eps) {
  const double s1 = 13.0 / 12.0 * (v1 - 2 * v2 + v3) * (v1 - 2 * v2 + v3) +
                    0.25 * (v1 - 4 * v2 + 3 * v3) * (v1 - 4 * v2 + 3 * v3);
  const double s2 = 13.0 / 12.0 * (v2 - 2 * v3 + v4) * (v2 - 2 * v3 + v4) +
                    0.25 * (v2 - v4) * (v2 - v4);
  const double s3 = 13.0 / 12.0 * (v3 - 2 * v4 + v5) * (v3 - 2 * v4 + v5) +
                    0.25 * (3 * v3 - 4 * v4 + v5) * (3 * v3 - 4 * v4 + v5);
  const double a1 = 0.1 / ((eps + s1) * (eps + s1));
  const double a2 = 0.6 / ((eps + s2) * (eps + s2));
  const double a3 = 0.3 / ((eps + s3) * (eps + s3));
  return (a1 * (v1 / 3 - 7 * v2 / 6 + 11 * v3 / 6) + a2 * (-v2 / 6 + 5 * v3 / 6 + v4 / 3) +
          a3 * (v3 / 3 + 5 * v4 / 6 - v5 / 6)) /
         (a1 + a2 + a3);
}

/* one-sided derivatives at index k (position i of n along a line with
 * stride s) */
static void dpm(const double *u, size_t k, int i, int n, size_t s, double h, double eps,
                double *m, double *p) {
  if (i >= 3 && i <= n - 4) {
    double d[6];
    for (int q = 0; q < 6; ++q) d[q] = (u[k + (q - 2) * s] - u[k + (q - 3) * s]) / h;
    *m = weno5(d[0], d[1], d[2], d[3], d[4], eps);
    *p = weno5(d[5], d[4], d[3], d[2], d[1], eps);
    return;
  }
  const double bm = i > 0 ? (u[k] - u[k - s]) / h : 0.0;
  const double bp = i < n - 1 ? (u[k + s] - u[k]) / h : 0.0;
  *m = i > 0 ? bm : bp;
  *p = i < n - 1 ? bp : bm;
}

static double eik_update(const double *tb, size_t k, int i, int j, int nx, int ny, double h,
                         double eps, double n, double tt, double ttx, double tty, double ax,
                         double ay) {
  double pm, pp, qm, qp;
  dpm(tb, k, i, nx, 1, h, eps, &pm, &pp);
  dpm(tb, k, j, ny, (size_t)nx, h, eps, &qm, &qp);
  const double t = tb[k];
  const double ex = tt * 0.5 * (pm + pp) + t * ttx, ey = tt * 0.5 * (qm + qp) + t * tty;
  const double Hh = sqrt(ex * ex + ey * ey) - ax * (pp - pm) / 2 - ay * (qp - qm) / 2;
  return (n - Hh) * h / (ax + ay);
}

static double tr_update(const double *v, size_t k, int i, int j, int nx, int ny, double h,
                        double eps, double bx, double by, double c, double f, double ax,
                        double ay) {
  double pm, pp, qm, qp;
  dpm(v, k, i, nx, 1, h, eps, &pm, &pp);
  dpm(v, k, j, ny, (size_t)nx, h, eps, &qm, &qp);
  const double Hh = bx * 0.5 * (pm + pp) + by * 0.5 * (qm + qp) + c * v[k] - ax * (pp - pm) / 2 -
                    ay * (qp - qm) / 2;
  return (f - Hh) * h / (ax + ay);
}

/* kind 0: eikonal (c0 = n, c1 = tt, c2 = ttx, c3 = tty);
 * kind 1: transport (c0 = b_x, c1 = b_y, c2 = c, c3 = f);
 * ax, ay the viscosities, eps the WENO epsilon.  Every array is nx x ny. */
int hb_sweep(int kind, double *u, int nx, int ny, double h, double eps, const double *c0,
             const double *c1,
             const double *c2, const double *c3, const double *ax, const double *ay,
             const unsigned char *fixed, double omega, double tol, int maxrounds, double *last) {
  int round = 0;
  double mx = 0.0;
  for (round = 0; round < maxrounds; ++round) {
    mx = 0.0;
    for (int o = 0; o < 4; ++o) {
      const int sx = (o == 0 || o == 3) ? 1 : -1, sy = (o < 2) ? 1 : -1;
      for (int jj = 0; jj < ny; ++jj) {
        const int j = sy > 0 ? jj : ny - 1 - jj;
        for (int ii = 0; ii < nx; ++ii) {
          const int i = sx > 0 ? ii : nx - 1 - ii;
          const size_t k = (size_t)i + (size_t)nx * j;
          if (fixed[k]) continue;
          const double du =
              omega * (kind == 0
                           ? eik_update(u, k, i, j, nx, ny, h, eps, c0[k], c1[k], c2[k], c3[k],
                                        ax[k], ay[k])
                           : tr_update(u, k, i, j, nx, ny, h, eps, c0[k], c1[k], c2[k], c3[k],
                                       ax[k], ay[k]));
          u[k] += du;
          /* a NaN update counts as never converging */
          if (!(fabs(du) <= mx)) mx = du == du ? fabs(du) : INFINITY;
        }
      }
    }
    if (mx < tol) { ++round; break; }
  }
  if (last) *last = mx;
  return round;
}
