// Tables of tau^2, v0, v1 at pairs of Chebyshev nodes from the eikonal and
// transport solves (2D): for every source node, the factored eikonal
// (eq. faceik) and the transport recurrence (eq. equVs, v0 then v1) on a grid
// of spacing h0 aligned with the node, by Lax-Friedrichs sweeping with WENO5
// derivatives and the unknowns held at their Taylor expansions near the
// source (Sec. 2.2-2.3); then local cubic interpolation of the grid values to
// every node (Sec. 4.1, the tabulation of eq. chebinterp).
//
// One workgroup per source node.  A Gauss-Seidel sweep in ordering (sx, sy)
// visits the anti-diagonals i' + j' = t in order (i' = i or nx-1-i, likewise
// j'); the points of one anti-diagonal do not depend on each other, so the
// workgroup updates them together and meets at a barrier before the next.
// The unknown of the running solve sits in LDS when the grid fits, the
// coefficients in global memory (read-only, cached).
// The discrete equations:
//   * derivatives p-, p+ (q-, q+): Jiang-Peng WENO5 (epsilon h^2) where the
//     seven points i-3 .. i+3 lie in the grid, first-order one-sided
//     differences in the three outer layers (the missing one replaced by the
//     other on the first and last point);
//   * eikonal, tau = tt tb with tt = n0 |r - r0|:
//     Hh = |tt grad tb + tb grad tt|(mean p, mean q) - a (p+ - p-)/2 - a (q+ - q-)/2,
//     tb += (n - Hh) h / (2 a), a = the largest tt over the grid;
//   * transport, b . grad v + c v = f with b = 2 grad tau^2:
//     Hh = b_x mean p + b_y mean q + c v - a_x (p+ - p-)/2 - a_y (q+ - q-)/2,
//     v += (f - Hh) h / (a_x + a_y) / 2, a_x, a_y the largest |b_x|, |b_y|;
//   * v0: c = lap tau^2 - 4 n^2, f = 0; v1: c = lap tau^2, f = lap v0
//     (d = 2); gradients and Laplacians by sixth-order central differences,
//     second order in the three outer layers;
//   * held values: |i - i0|, |j - j0| <= P - 1 with P = 6 (tb), 4 (v0), 2 (v1).
#include <hip/hip_runtime.h>

#include "hbi_device.h"
#include "hbi_tabulate.h"

namespace hbi {

namespace {

// The WENO5 combination sum_k a_k f_k / sum_k a_k with a_k = d_k / (eps +
// s_k)^2, numerator and denominator both multiplied by the product of the
// three (eps + s_k)^2 so that one division remains; the stencil values f_k
// with constant multipliers instead of divisions.
__device__ __forceinline__ double weno5(double v1, double v2, double v3, double v4, double v5,
                                        double eps) {
  const double s1 = 13.0 / 12.0 * (v1 - 2 * v2 + v3) * (v1 - 2 * v2 + v3) +
                    0.25 * (v1 - 4 * v2 + 3 * v3) * (v1 - 4 * v2 + 3 * v3);
  const double s2 = 13.0 / 12.0 * (v2 - 2 * v3 + v4) * (v2 - 2 * v3 + v4) +
                    0.25 * (v2 - v4) * (v2 - v4);
  const double s3 = 13.0 / 12.0 * (v3 - 2 * v4 + v5) * (v3 - 2 * v4 + v5) +
                    0.25 * (3 * v3 - 4 * v4 + v5) * (3 * v3 - 4 * v4 + v5);
  const double q1 = (eps + s1) * (eps + s1), q2 = (eps + s2) * (eps + s2),
               q3 = (eps + s3) * (eps + s3);
  const double w1 = 0.1 * (q2 * q3), w2 = 0.6 * (q1 * q3), w3 = 0.3 * (q1 * q2);
  constexpr double c3 = 1.0 / 3.0, c6 = 1.0 / 6.0;
  const double f1 = c3 * v1 - 7 * c6 * v2 + 11 * c6 * v3;
  const double f2 = -c6 * v2 + 5 * c6 * v3 + c3 * v4;
  const double f3 = c3 * v3 + 5 * c6 * v4 - c6 * v5;
  return (w1 * f1 + w2 * f2 + w3 * f3) / (w1 + w2 + w3);
}

// one-sided derivatives of u at index k, position i of n along a line of
// stride s (ih = 1 / h)
__device__ __forceinline__ void dpm(const double *u, int64_t k, int i, int n, int64_t s, double ih,
                                    double eps, double &m, double &p) {
  if (i >= 3 && i <= n - 4) {
    double d[6];
#pragma unroll
    for (int q = 0; q < 6; ++q) d[q] = (u[k + (q - 2) * s] - u[k + (q - 3) * s]) * ih;
    m = weno5(d[0], d[1], d[2], d[3], d[4], eps);
    p = weno5(d[5], d[4], d[3], d[2], d[1], eps);
    return;
  }
  const double bm = i > 0 ? (u[k] - u[k - s]) * ih : 0.0;
  const double bp = i < n - 1 ? (u[k + s] - u[k]) * ih : 0.0;
  m = i > 0 ? bm : bp;
  p = i < n - 1 ? bp : bm;
}

// first and second derivative along a line (sixth order inside, second
// order in the three outer layers, one-sided on the first and last point)
__device__ double d1(const double *u, int64_t k, int i, int n, int64_t s, double h) {
  if (i >= 3 && i <= n - 4)
    return (-u[k - 3 * s] / 60 + 3 * u[k - 2 * s] / 20 - 3 * u[k - s] / 4 + 3 * u[k + s] / 4 -
            3 * u[k + 2 * s] / 20 + u[k + 3 * s] / 60) /
           h;
  if (i == 0) return (-3 * u[k] + 4 * u[k + s] - u[k + 2 * s]) / (2 * h);
  if (i == n - 1) return (3 * u[k] - 4 * u[k - s] + u[k - 2 * s]) / (2 * h);
  return (u[k + s] - u[k - s]) / (2 * h);
}
__device__ double d2(const double *u, int64_t k, int i, int n, int64_t s, double h) {
  if (i >= 3 && i <= n - 4)
    return (u[k - 3 * s] / 90 - 3 * u[k - 2 * s] / 20 + 3 * u[k - s] / 2 - 49 * u[k] / 18 +
            3 * u[k + s] / 2 - 3 * u[k + 2 * s] / 20 + u[k + 3 * s] / 90) /
           (h * h);
  if (i == 0) return (2 * u[k] - 5 * u[k + s] + 4 * u[k + 2 * s] - u[k + 3 * s]) / (h * h);
  if (i == n - 1) return (2 * u[k] - 5 * u[k - s] + 4 * u[k - 2 * s] - u[k - 3 * s]) / (h * h);
  return (u[k + s] - 2 * u[k] + u[k - s]) / (h * h);
}

// sum of c[a * TAB_PD + b] dx^a dy^b (degree < TAB_PD)
__device__ double poly(const double *c, double dx, double dy) {
  double acc = 0.0, xa = 1.0;
  for (int a = 0; a < TAB_PD; ++a) {
    double yb = 1.0;
    for (int b = 0; a + b < TAB_PD; ++b) {
      acc += c[a * TAB_PD + b] * xa * yb;
      yb *= dy;
    }
    xa *= dx;
  }
  return acc;
}

// largest value over the workgroup (all threads get it); a NaN counts as +inf
__device__ double block_max(double v, double *red) {
  if (!(v == v)) v = INFINITY;
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  const int w = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[w] = v;
  __syncthreads();
  double m = red[0];
  for (int q = 1; q < (int)(blockDim.x >> 6); ++q) m = fmax(m, red[q]);
  return m;
}

struct Grid {
  int nx, ny, i0, j0;
  double h, gx0, gy0;   // point (i, j) at (gx0 + i h, gy0 + j h); the source at (i0, j0)
};

// Gauss-Seidel rounds of one equation until the largest update of a round
// is below tol (returns the rounds, or -1 when maxrounds did not suffice).
// KIND 0: eikonal (c0 = n, c1 = tt, c2 = tt_x, c3 = tt_y), KIND 1:
// transport (c0 = b_x, c1 = b_y, c2 = c, c3 = f).  u may be the workgroup's
// LDS copy of the unknown.
template <int KIND>
__device__ __forceinline__ int sweep(double *u, const Grid &g, const double *c0, const double *c1,
                                     const double *c2, const double *c3, double ax, double ay,
                                     int hold, double omega, double tol, int maxrounds,
                                     double *red) {
  const int nx = g.nx, ny = g.ny;
  const double h = g.h, ih = 1.0 / h, eps = h * h;
  const double scale = omega * h / (ax + ay);
  for (int round = 0; round < maxrounds; ++round) {
    double mx = 0.0;
    for (int o = 0; o < 4; ++o) {
      const bool fx = (o == 0 || o == 3), fy = (o < 2);
      for (int t = 0; t < nx + ny - 1; ++t) {
        const int lo = t - (ny - 1) > 0 ? t - (ny - 1) : 0;
        const int hi = t < nx - 1 ? t : nx - 1;
        for (int ip = lo + (int)threadIdx.x; ip <= hi; ip += (int)blockDim.x) {
          const int i = fx ? ip : nx - 1 - ip;
          const int jp = t - ip;
          const int j = fy ? jp : ny - 1 - jp;
          if (abs(i - g.i0) <= hold && abs(j - g.j0) <= hold) continue;
          const int64_t k = (int64_t)i + (int64_t)nx * j;
          double pm, pp, qm, qp;
          dpm(u, k, i, nx, 1, ih, eps, pm, pp);
          dpm(u, k, j, ny, nx, ih, eps, qm, qp);
          double r;
          if (KIND == 0) {
            const double tt = c1[k];
            const double ex = tt * 0.5 * (pm + pp) + u[k] * c2[k];
            const double ey = tt * 0.5 * (qm + qp) + u[k] * c3[k];
            const double Hh = sqrt(ex * ex + ey * ey) - ax * (pp - pm) * 0.5 - ay * (qp - qm) * 0.5;
            r = c0[k] - Hh;
          } else {
            const double Hh = c0[k] * 0.5 * (pm + pp) + c1[k] * 0.5 * (qm + qp) + c2[k] * u[k] -
                              ax * (pp - pm) * 0.5 - ay * (qp - qm) * 0.5;
            r = c3[k] - Hh;
          }
          const double du = r * scale;
          u[k] += du;
          const double a = fabs(du);
          mx = (a == a) ? fmax(mx, a) : INFINITY;
        }
        __syncthreads();
      }
    }
    if (block_max(mx, red) < tol) return round + 1;
  }
  return -1;
}

// A workgroup barrier that waits only for this wave's LDS operations: the
// sweeps keep the unknown in LDS and only read global memory, so the loads
// of the next diagonal's coefficients may stay in flight across it (the
// memory clobber keeps the compiler from moving memory accesses over it).
__device__ __forceinline__ void lds_barrier() {
  __asm__ volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
}

// sweep() for an unknown in LDS on a grid whose anti-diagonals have at most
// blockDim.x points (min(nx, ny) <= blockDim.x): every thread updates at
// most one point per diagonal, and the coefficients of its point on the
// next diagonal are loaded before the barrier that ends the current one.
// Same updates in the same order as sweep().
template <int KIND>
__device__ __forceinline__ int sweep_lds(double *u, const Grid &g, const double *c0,
                                         const double *c1, const double *c2, const double *c3,
                                         double ax, double ay, int hold, double omega, double tol,
                                         int maxrounds, double *red) {
  const int nx = g.nx, ny = g.ny;
  const double h = g.h, ih = 1.0 / h, eps = h * h;
  const double scale = omega * h / (ax + ay);
  const int tid = (int)threadIdx.x;
  for (int round = 0; round < maxrounds; ++round) {
    double mx = 0.0;
    for (int o = 0; o < 4; ++o) {
      const bool fx = (o == 0 || o == 3), fy = (o < 2);
      // this thread's point on diagonal t: position ip = lo(t) + tid
      auto point = [&](int t, int &i, int &j) -> bool {
        const int lo = t - (ny - 1) > 0 ? t - (ny - 1) : 0;
        const int hi = t < nx - 1 ? t : nx - 1;
        const int ip = lo + tid;
        const int jp = t - ip;
        i = fx ? ip : nx - 1 - ip;
        j = fy ? jp : ny - 1 - jp;
        return t < nx + ny - 1 && ip <= hi &&
               !(abs(i - g.i0) <= hold && abs(j - g.j0) <= hold);
      };
      int i, j;
      bool have = point(0, i, j);
      int64_t k = have ? (int64_t)i + (int64_t)nx * j : 0;
      double e0 = c0[k], e1 = c1[k], e2 = c2[k], e3 = c3[k];
      for (int t = 0; t < nx + ny - 1; ++t) {
        int in, jn;
        const bool hn = point(t + 1, in, jn);
        const int64_t kn = hn ? (int64_t)in + (int64_t)nx * jn : 0;
        const double n0 = c0[kn], n1 = c1[kn], n2 = c2[kn], n3 = c3[kn];
        if (have) {
          double pm, pp, qm, qp;
          dpm(u, k, i, nx, 1, ih, eps, pm, pp);
          dpm(u, k, j, ny, nx, ih, eps, qm, qp);
          double r;
          if (KIND == 0) {
            const double ex = e1 * 0.5 * (pm + pp) + u[k] * e2;
            const double ey = e1 * 0.5 * (qm + qp) + u[k] * e3;
            const double Hh = sqrt(ex * ex + ey * ey) - ax * (pp - pm) * 0.5 - ay * (qp - qm) * 0.5;
            r = e0 - Hh;
          } else {
            const double Hh = e0 * 0.5 * (pm + pp) + e1 * 0.5 * (qm + qp) + e2 * u[k] -
                              ax * (pp - pm) * 0.5 - ay * (qp - qm) * 0.5;
            r = e3 - Hh;
          }
          const double du = r * scale;
          u[k] += du;
          const double a = fabs(du);
          mx = (a == a) ? fmax(mx, a) : INFINITY;
        }
        lds_barrier();
        have = hn;
        i = in;
        j = jn;
        k = kn;
        e0 = n0; e1 = n1; e2 = n2; e3 = n3;
      }
    }
    if (block_max(mx, red) < tol) return round + 1;
  }
  return -1;
}

// One solve with the unknown u (np points, global memory) copied into the
// workgroup's LDS array ul for the sweeps when LDS, written back after.
template <int KIND, bool LDS>
__device__ __forceinline__ int solve(double *u, double *ul, int64_t np, const Grid &g,
                                     const double *c0, const double *c1, const double *c2,
                                     const double *c3, double ax, double ay, int hold,
                                     double omega, double tol, int maxrounds, double *red) {
  if constexpr (LDS) {
    for (int64_t k = threadIdx.x; k < np; k += blockDim.x) ul[k] = u[k];
    __syncthreads();
    const int r =
        (g.nx <= (int)blockDim.x || g.ny <= (int)blockDim.x)
            ? sweep_lds<KIND>(ul, g, c0, c1, c2, c3, ax, ay, hold, omega, tol, maxrounds, red)
            : sweep<KIND>(ul, g, c0, c1, c2, c3, ax, ay, hold, omega, tol, maxrounds, red);
    for (int64_t k = threadIdx.x; k < np; k += blockDim.x) u[k] = ul[k];
    __syncthreads();
    return r;
  } else {
    return sweep<KIND>(u, g, c0, c1, c2, c3, ax, ay, hold, omega, tol, maxrounds, red);
  }
}

// n^2 of the medium at (x, y): tensor Lagrange quintic on the 6 x 6 grid
// points around it
__device__ double medium_n2(const TabMedium &m, double x, double y) {
  const double fx = (x - m.ox) / m.hm, fy = (y - m.oy) / m.hm;
  const int i = (int)floor(fx) - 2, j = (int)floor(fy) - 2;
  double wx[6], wy[6];
#pragma unroll
  for (int a = 0; a < 6; ++a) {
    double px = 1.0, py = 1.0;
#pragma unroll
    for (int b = 0; b < 6; ++b) {
      if (b == a) continue;
      px *= (fx - (i + b)) / (double)(a - b);
      py *= (fy - (j + b)) / (double)(a - b);
    }
    wx[a] = px;
    wy[a] = py;
  }
  double acc = 0.0;
  for (int b = 0; b < 6; ++b) {
    double r = 0.0;
#pragma unroll
    for (int a = 0; a < 6; ++a) r += wx[a] * m.n2[(int64_t)(i + a) + (int64_t)m.nx * (j + b)];
    acc += wy[b] * r;
  }
  return acc;
}

}  // namespace

template <bool LDS>
__global__ __launch_bounds__(256) void k_tab_source(const TabSource *srcs, TabMedium med,
                                                    double *ws, int64_t ws_stride,
                                                    const double *nodes, int32_t NT,
                                                    double *ftau2, double *fv0, double *fv1,
                                                    int32_t *status, double tol, int maxrounds) {
  __shared__ double red[4];
  extern __shared__ double ul[];   // the unknown during the sweeps (LDS)
  const int s = blockIdx.x;
  const TabSource S = srcs[s];
  Grid g{S.nx, S.ny, S.i0, S.j0, S.h, S.gx0, S.gy0};
  const int64_t np = (int64_t)g.nx * g.ny;
  double *W = ws + (int64_t)s * ws_stride;
  double *N = W, *TT = W + np, *TX = W + 2 * np, *TY = W + 3 * np, *U = W + 4 * np;
  double *V0 = W + 5 * np, *V1 = W + 6 * np, *BX = W + 7 * np, *BY = W + 8 * np;
  double *CC = W + 9 * np, *FF = W + 10 * np;
  // medium, factor tt = n0 |r - r0| and its gradient, held Taylor values
  double ttmax = 0.0;
  for (int64_t k = threadIdx.x; k < np; k += blockDim.x) {
    const int i = (int)(k % g.nx), j = (int)(k / g.nx);
    const double dx = (i - g.i0) * g.h, dy = (j - g.j0) * g.h;
    N[k] = sqrt(medium_n2(med, g.gx0 + i * g.h, g.gy0 + j * g.h));
    const double rho = sqrt(dx * dx + dy * dy);
    TT[k] = S.n0 * rho;
    TX[k] = rho > 0 ? S.n0 * dx / rho : 0.0;
    TY[k] = rho > 0 ? S.n0 * dy / rho : 0.0;
    ttmax = fmax(ttmax, TT[k]);
    const int di = abs(i - g.i0), dj = abs(j - g.j0);
    const double t2 = poly(S.T, dx, dy);
    U[k] = (di <= 5 && dj <= 5) ? (rho > 0 ? sqrt(fmax(t2, 0.0)) / TT[k] : 1.0) : 1.0;
    V0[k] = (di <= 3 && dj <= 3) ? poly(S.B, dx, dy) : S.B[0];
    V1[k] = (di <= 1 && dj <= 1) ? poly(S.C, dx, dy) : 0.0;
  }
  const double a_t = block_max(ttmax, red);
  int r1 = solve<0, LDS>(U, ul, np, g, N, TT, TX, TY, a_t, a_t, 5, 1.0, tol, maxrounds, red);
  // tau^2, b = 2 grad tau^2, lap tau^2
  for (int64_t k = threadIdx.x; k < np; k += blockDim.x) U[k] = (U[k] * TT[k]) * (U[k] * TT[k]);
  __syncthreads();
  double bxm = 0.0, bym = 0.0;
  for (int64_t k = threadIdx.x; k < np; k += blockDim.x) {
    const int i = (int)(k % g.nx), j = (int)(k / g.nx);
    BX[k] = 2.0 * d1(U, k, i, g.nx, 1, g.h);
    BY[k] = 2.0 * d1(U, k, j, g.ny, g.nx, g.h);
    CC[k] = d2(U, k, i, g.nx, 1, g.h) + d2(U, k, j, g.ny, g.nx, g.h) - 4.0 * N[k] * N[k];
    FF[k] = 0.0;
    bxm = fmax(bxm, fabs(BX[k]));
    bym = fmax(bym, fabs(BY[k]));
  }
  const double a_x = block_max(bxm, red), a_y = block_max(bym, red);
  int r2 = solve<1, LDS>(V0, ul, np, g, BX, BY, CC, FF, a_x, a_y, 3, 0.5, tol, maxrounds, red);
  // v1: c = lap tau^2, f = lap v0
  for (int64_t k = threadIdx.x; k < np; k += blockDim.x) {
    const int i = (int)(k % g.nx), j = (int)(k / g.nx);
    CC[k] += 4.0 * N[k] * N[k];
    FF[k] = d2(V0, k, i, g.nx, 1, g.h) + d2(V0, k, j, g.ny, g.nx, g.h);
  }
  __syncthreads();
  int r3 = solve<1, LDS>(V1, ul, np, g, BX, BY, CC, FF, a_x, a_y, 1, 0.5, tol, maxrounds, red);
  // the grid values at every node: tensor Lagrange cubic on the 4 x 4 points
  for (int A = threadIdx.x; A < NT; A += blockDim.x) {
    const double fx = (nodes[2 * A] - g.gx0) / g.h, fy = (nodes[2 * A + 1] - g.gy0) / g.h;
    const int i = (int)floor(fx), j = (int)floor(fy);
    const double tx = fx - i, ty = fy - j;
    const double wx[4] = {-tx * (tx - 1) * (tx - 2) / 6, (tx + 1) * (tx - 1) * (tx - 2) / 2,
                          -(tx + 1) * tx * (tx - 2) / 2, (tx + 1) * tx * (tx - 1) / 6};
    const double wy[4] = {-ty * (ty - 1) * (ty - 2) / 6, (ty + 1) * (ty - 1) * (ty - 2) / 2,
                          -(ty + 1) * ty * (ty - 2) / 2, (ty + 1) * ty * (ty - 1) / 6};
    double a0 = 0.0, a1 = 0.0, a2 = 0.0;
    for (int a = 0; a < 4; ++a)
      for (int b = 0; b < 4; ++b) {
        const int64_t k = (int64_t)(i - 1 + a) + (int64_t)g.nx * (j - 1 + b);
        const double w = wx[a] * wy[b];
        a0 += w * U[k];
        a1 += w * V0[k];
        a2 += w * V1[k];
      }
    ftau2[(int64_t)A * NT + s] = a0;
    fv0[(int64_t)A * NT + s] = a1;
    fv1[(int64_t)A * NT + s] = a2;
  }
  if (threadIdx.x == 0) {
    status[3 * s] = r1;
    status[3 * s + 1] = r2;
    status[3 * s + 2] = r3;
  }
}

// F <- (F + F^T) / 2 for the three tables (one thread per pair A < B)
__global__ void k_tab_symmetrise(double *f0, double *f1, double *f2, int32_t NT) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t A = q / NT, B = q % NT;
  if (A >= NT || B <= A) return;
  double *F[3] = {f0, f1, f2};
  for (int t = 0; t < 3; ++t) {
    const double m = 0.5 * (F[t][A * NT + B] + F[t][B * NT + A]);
    F[t][A * NT + B] = m;
    F[t][B * NT + A] = m;
  }
}

hipError_t launch_tabulate(const TabSource *srcs, int32_t nsrc, const TabMedium &med, double *ws,
                           int64_t ws_stride, int64_t npmax, const double *nodes, int32_t NT,
                           double *ftau2, double *fv0, double *fv1, int32_t *status, double tol,
                           int maxrounds, hipStream_t st) {
  if (nsrc <= 0) return hipSuccess;
  // the unknown in LDS when the largest grid fits (gfx950: 160 KiB per
  // workgroup, the attribute raises the dynamic limit)
  const size_t lds = sizeof(double) * (size_t)npmax;
  if (lds <= TAB_LDS_MAX_BYTES &&
      hipFuncSetAttribute((const void *)k_tab_source<true>,
                          hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) == hipSuccess) {
    hipLaunchKernelGGL(k_tab_source<true>, dim3(nsrc), dim3(256), lds, st, srcs, med, ws, ws_stride,
                       nodes, NT, ftau2, fv0, fv1, status, tol, maxrounds);
  } else {
    (void)hipGetLastError();
    hipLaunchKernelGGL(k_tab_source<false>, dim3(nsrc), dim3(256), 0, st, srcs, med, ws, ws_stride,
                       nodes, NT, ftau2, fv0, fv1, status, tol, maxrounds);
  }
  return hipGetLastError();
}

hipError_t launch_tab_symmetrise(double *f0, double *f1, double *f2, int32_t NT, hipStream_t st) {
  const int64_t n = (int64_t)NT * NT;
  hipLaunchKernelGGL(k_tab_symmetrise, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, f0, f1,
                     f2, NT);
  return hipGetLastError();
}

}  // namespace hbi
