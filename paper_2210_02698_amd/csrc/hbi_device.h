// Small device helpers: complex arithmetic on interleaved pairs and
// wave64 reductions.
#pragma once
#include <hip/hip_runtime.h>

#include "hbi_internal.h"

namespace hbi {

template <typename R> struct cplx;
template <> struct cplx<double> { using type = double2; };
template <> struct cplx<float> { using type = float2; };
template <typename R> using cplx_t = typename cplx<R>::type;

template <typename C> __device__ __forceinline__ C cmul(C a, C b) {
  return C{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
// a * conj(b)
template <typename C> __device__ __forceinline__ C cmulc(C a, C b) {
  return C{a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y};
}
// acc += a * b
template <typename C> __device__ __forceinline__ void cfma(C &acc, C a, C b) {
  acc.x = fma(a.x, b.x, acc.x);
  acc.x = fma(-a.y, b.y, acc.x);
  acc.y = fma(a.x, b.y, acc.y);
  acc.y = fma(a.y, b.x, acc.y);
}
// acc += conj(a) * b
template <typename C> __device__ __forceinline__ void cfmac(C &acc, C a, C b) {
  acc.x = fma(a.x, b.x, acc.x);
  acc.x = fma(a.y, b.y, acc.x);
  acc.y = fma(a.x, b.y, acc.y);
  acc.y = fma(-a.y, b.x, acc.y);
}

// Table box of the point c and its 1D barycentric Lagrange weights in that
// box, lw[ax * nI + k].  First-kind Chebyshev nodes
// u_k = (1 + cos((2k+1)pi/(2nI)))/2 on [0,1] have barycentric weights
// (-1)^k sin((2k+1)pi/(2nI)) (Berrut & Trefethen, SIAM Rev. 2004);
// l_k(t) = (w_k/(t-u_k)) / sum_j w_j/(t-u_j).  A point on a box face
// belongs to the box floor((x - origin)/size), clamped to the table region.
__device__ inline int32_t box_weights(const DevProblem &P, const double c[3], double *lw) {
  constexpr double pi = 3.14159265358979323846;
  int32_t b = 0, stride = 1;
  const int nI = P.nI;
  for (int ax = 0; ax < P.dim; ++ax) {
    const double rel = (c[ax] - P.box_origin[ax]) / P.box_size;
    int bi = (int)floor(rel);
    bi = bi < 0 ? 0 : (bi >= P.nbox[ax] ? P.nbox[ax] - 1 : bi);
    b += bi * stride;
    stride *= P.nbox[ax];
    const double t = rel - bi;
    double *w = lw + ax * nI;
    int hit = -1;
    double den = 0.0;
    for (int k = 0; k < nI; ++k) {
      const double ang = (2.0 * k + 1.0) * pi / (2.0 * nI);
      const double u = 0.5 * (1.0 + cos(ang));
      const double d = t - u;
      if (d == 0.0) { hit = k; break; }
      const double q = ((k & 1) ? -sin(ang) : sin(ang)) / d;
      w[k] = q;
      den += q;
    }
    if (hit >= 0) {
      for (int k = 0; k < nI; ++k) w[k] = (k == hit) ? 1.0 : 0.0;
    } else {
      const double inv = 1.0 / den;
      for (int k = 0; k < nI; ++k) w[k] *= inv;
    }
  }
  return b;
}

// Orders the LDS writes of a wave before its later LDS reads by other lanes
// of the same wave (no other wave reads them).
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

}  // namespace hbi
