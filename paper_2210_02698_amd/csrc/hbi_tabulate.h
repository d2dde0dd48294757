// Table generation from the eikonal and transport solves (hbi_tabulate.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hbi {

constexpr int TAB_PD = 7;   // polynomial coefficient arrays c[a * TAB_PD + b], a + b < TAB_PD
// largest LDS copy of a source grid's unknown (bytes); larger grids sweep in
// global memory
constexpr size_t TAB_LDS_MAX_BYTES = 150 * 1024;

// One source node: its grid (point (i, j) at (gx0 + i h, gy0 + j h), the
// node at (i0, j0)), n0 = n(node), and the summed Taylor polynomials of
// tau^2 (degrees <= 6), v0 (<= 4), v1 (<= 2) about it in (x - x0, y - y0).
struct TabSource {
  double h, gx0, gy0, n0;
  int32_t nx, ny, i0, j0;
  double T[TAB_PD * TAB_PD], B[TAB_PD * TAB_PD], C[TAB_PD * TAB_PD];
};

// The medium: n^2 on a regular grid (point (i, j) at (ox + i hm, oy + j hm)),
// device array, x fastest.
struct TabMedium {
  const double *n2;
  int32_t nx, ny;
  double ox, oy, hm;
};

// Solves every source of srcs (one workgroup each; workspace ws_stride
// doubles per source, at least 11 nx ny; npmax the largest nx ny) and
// writes column s of the three
// NT x NT tables (row A: the value at node A); status[3 s + e] = rounds of
// equation e, or -1 when maxrounds did not reach tol.
hipError_t launch_tabulate(const TabSource *srcs, int32_t nsrc, const TabMedium &med, double *ws,
                           int64_t ws_stride, int64_t npmax, const double *nodes, int32_t NT,
                           double *ftau2, double *fv0, double *fv1, int32_t *status, double tol,
                           int maxrounds, hipStream_t st);
hipError_t launch_tab_symmetrise(double *f0, double *f1, double *f2, int32_t NT, hipStream_t st);

}  // namespace hbi
