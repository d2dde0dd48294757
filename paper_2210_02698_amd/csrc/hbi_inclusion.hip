// HIP kernels of the curve inclusion (Sec. 3.2, domain with a sound-hard inclusion), 2D:
//
//   U = (K^{v2v} + K^{s2v} (K^{s2s})^{-1} K^{v2s}) h^d s      (eq. m_v2v_inclu)
//
// with K^{v2s}_ij = g(r^s_i, r_j), K^{s2v}_ij = g(r_i, r^s_j) w_j and
// K^{s2s}_ij = -g(r^s_i, r^s_j) w_j off the diagonal (eq. m_v2s, m_s2v, s2s).
// The tables are symmetric, so g is reciprocal and one operator G,
// G[j, i] = g(r_j, r^s_i) over cells j and segments i, serves both
// K^{v2s} = G^T and K^{s2v} = G W.  G is a single butterfly (hbi_s2v.hip),
// or, kept dense for comparison, stored in row chunks of `m` cells: chunk q
// holds cells [q m, q m + m_q) as an m_q x N_s column-major block at element
// offset q m N_s, so a segment's column within a chunk is contiguous.
//
//   k_point_setup           table box and Lagrange weights of every segment
//                           centre, and the K^{s2s} self factor
//   k_gj_pivot(_panel), k_gj_update(_panel), k_gj_copy_rows,
//   k_gj_block_update, k_gj_unpermute
//                           Gauss-Jordan inverse of K^{s2s} in FP64 with row
//                           pivoting, in place, by panels of 32 columns whose
//                           update of the rest is an MFMA GEMM
//   k_inc_gather, k_inc_reduce, k_inc_small(_sum), k_inc_scatter, k_inc_add
//                           the inclusion term of one product (or of its
//                           conjugate transpose), gathers only, fixed
//                           summation order (with a butterfly G, only the
//                           K^{s2s} step k_inc_small(_sum) runs here)
#include "hbi_kernels.h"
#include "hbi_device.h"

namespace hbi {

namespace {
constexpr double kPiI = 3.14159265358979323846;
constexpr double kEulerGamma = 0.57721566490153286061;
}  // namespace

// Segment i sits at position p0 + i of the per-point arrays (after the
// cells).  Its self factor sf_i is the value the entry kernels return on
// the diagonal: K^{s2s}_ii = -w_i sf_i with
//   -w_i sf_i = -(i w_i / 4) [1 + (2i/pi)(log(e^gamma omega n_i w_i / 4) - 1)],
// minus the integral of the leading HB term (i/4) H0(omega n |t|) over the
// segment, in its small-segment form (eq. s2s; the factor i of the leading
// term and e^gamma are read into the printed formula).
__global__ void k_point_setup(DevProblem P, const double *xy, const double *w,
                              const double *slow, int32_t ns, int64_t p0, double *xyz,
                              double *lw, int32_t *box, double2 *self) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= ns) return;
  const int64_t p = p0 + i;
  const double c[3] = {xy[2 * i], xy[2 * i + 1], 0.0};
  for (int ax = 0; ax < 3; ++ax) xyz[p * 3 + ax] = c[ax];
  box[p] = box_weights(P, c, lw + p * P.dim * P.nI);
  const double L = kEulerGamma + log(P.omega * slow[i] * w[i] / 4.0);
  self[p] = double2{-(L - 1.0) / (2.0 * kPiI), 0.25};
}

// ---------------------------------------------------------------------------
// Gauss-Jordan inverse, column-major n x n complex A, in place.  Step k:
// k_gj_pivot (one workgroup) picks the row p >= k with the largest |A[p,k]|
// (lowest index on ties), swaps rows k and p, saves column k to colk,
// replaces A[k,k] by 1/A[k,k] and scales the rest of row k by it;
// k_gj_update subtracts colk[i] times row k from every other row i, and
// sets A[i,k] = -colk[i] A[k,k].  Row k is only read in the update, column
// k only written from colk, so the step has no read/write overlap.  After
// the last step the columns are swapped back in reverse order.  A zero
// pivot sets *status and leaves the remaining steps as no-ops.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(1024) void k_gj_pivot(double2 *A, int n, int k, int32_t *perm,
                                                   double2 *colk, int32_t *status) {
  __shared__ double sv[1024];
  __shared__ int si[1024];
  __shared__ double2 sinv;
  __shared__ int sp;
  if (*status) return;
  const int t = threadIdx.x;
  double best = -1.0;
  int bi = n;
  for (int i = k + t; i < n; i += blockDim.x) {
    const double2 a = A[i + (int64_t)k * n];
    const double m = a.x * a.x + a.y * a.y;
    if (m > best) { best = m; bi = i; }
  }
  sv[t] = best;
  si[t] = bi;
  __syncthreads();
  for (int o = blockDim.x / 2; o > 0; o >>= 1) {
    if (t < o) {
      const double b2 = sv[t + o];
      const int i2 = si[t + o];
      if (b2 > sv[t] || (b2 == sv[t] && i2 < si[t])) { sv[t] = b2; si[t] = i2; }
    }
    __syncthreads();
  }
  if (t == 0) {
    sp = si[0];
    perm[k] = sp;
    if (!(sv[0] > 0.0)) *status = 1;
  }
  __syncthreads();
  if (!(sv[0] > 0.0)) return;
  const int p = sp;
  if (p != k)
    for (int j = t; j < n; j += blockDim.x) {
      const double2 a = A[k + (int64_t)j * n], b = A[p + (int64_t)j * n];
      A[k + (int64_t)j * n] = b;
      A[p + (int64_t)j * n] = a;
    }
  __syncthreads();
  for (int i = t; i < n; i += blockDim.x) colk[i] = A[i + (int64_t)k * n];
  if (t == 0) {
    const double2 a = A[k + (int64_t)k * n];
    const double d = a.x * a.x + a.y * a.y;
    sinv = double2{a.x / d, -a.y / d};
  }
  __syncthreads();
  const double2 inv = sinv;
  for (int j = t; j < n; j += blockDim.x) {
    double2 &a = A[k + (int64_t)j * n];
    a = j == k ? inv : cmul(a, inv);
  }
}

__global__ void k_gj_update(double2 *A, int n, int k, const double2 *colk,
                            const int32_t *status) {
  if (*status) return;
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= (int64_t)n * n) return;
  const int i = (int)(e % n), j = (int)(e / n);
  if (i == k) return;
  const double2 f = colk[i];
  const double2 rk = A[k + (int64_t)j * n];
  if (j == k) {
    const double2 v = cmul(f, rk);
    A[e] = double2{-v.x, -v.y};
  } else {
    const double2 v = cmul(f, rk);
    A[e] = double2{A[e].x - v.x, A[e].y - v.y};
  }
}

// Blocked form: the pivot steps of a panel of up to kGjPanel columns
// [j0, j0 + jb) swap whole rows but scale and eliminate only inside the
// panel (k_gj_pivot_panel, k_gj_update_panel), which leaves in the panel
// columns the panel's own Gauss-Jordan result Pn: A11^-1 on the pivot rows
// j0.., -A21 A11^-1 on the others.  The rest of the matrix then takes the
// whole panel at once: with S its pivot rows (copied to Sb first),
// A[:, rest] = (A[:, rest], pivot rows zeroed) + Pn S, a complex GEMM of
// rank jb on FP64 MFMA tiles (k_gj_block_update).  This is the same
// elimination as the column-by-column form, its row updates regrouped.
constexpr int kGjPanel = 32;

__global__ __launch_bounds__(1024) void k_gj_pivot_panel(double2 *A, int n, int k, int j0, int jb,
                                                         int32_t *perm, double2 *colk,
                                                         int32_t *status) {
  __shared__ double sv[1024];
  __shared__ int si[1024];
  __shared__ double2 sinv;
  __shared__ int sp;
  if (*status) return;
  const int t = threadIdx.x;
  double best = -1.0;
  int bi = n;
  for (int i = k + t; i < n; i += blockDim.x) {
    const double2 a = A[i + (int64_t)k * n];
    const double m = a.x * a.x + a.y * a.y;
    if (m > best) { best = m; bi = i; }
  }
  sv[t] = best;
  si[t] = bi;
  __syncthreads();
  for (int o = blockDim.x / 2; o > 0; o >>= 1) {
    if (t < o) {
      const double b2 = sv[t + o];
      const int i2 = si[t + o];
      if (b2 > sv[t] || (b2 == sv[t] && i2 < si[t])) { sv[t] = b2; si[t] = i2; }
    }
    __syncthreads();
  }
  if (t == 0) {
    sp = si[0];
    perm[k] = sp;
    if (!(sv[0] > 0.0)) *status = 1;
  }
  __syncthreads();
  if (!(sv[0] > 0.0)) return;
  const int p = sp;
  if (p != k)
    for (int j = t; j < n; j += blockDim.x) {
      const double2 a = A[k + (int64_t)j * n], b = A[p + (int64_t)j * n];
      A[k + (int64_t)j * n] = b;
      A[p + (int64_t)j * n] = a;
    }
  __syncthreads();
  for (int i = t; i < n; i += blockDim.x) colk[i] = A[i + (int64_t)k * n];
  if (t == 0) {
    const double2 a = A[k + (int64_t)k * n];
    const double d = a.x * a.x + a.y * a.y;
    sinv = double2{a.x / d, -a.y / d};
  }
  __syncthreads();
  const double2 inv = sinv;
  for (int j = j0 + t; j < j0 + jb; j += blockDim.x) {
    double2 &a = A[k + (int64_t)j * n];
    a = j == k ? inv : cmul(a, inv);
  }
}

__global__ void k_gj_update_panel(double2 *A, int n, int k, int j0, int jb, const double2 *colk,
                                  const int32_t *status) {
  if (*status) return;
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= (int64_t)n * jb) return;
  const int i = (int)(e % n), j = j0 + (int)(e / n);
  if (i == k) return;
  const double2 f = colk[i];
  const double2 rk = A[k + (int64_t)j * n];
  double2 &a = A[i + (int64_t)j * n];
  const double2 v = cmul(f, rk);
  a = j == k ? double2{-v.x, -v.y} : double2{a.x - v.x, a.y - v.y};
}

// Sb[q][j] = A[j0 + q][j] for the columns outside the panel (0 inside it),
// q < jb, row-major jb x n.
__global__ void k_gj_copy_rows(const double2 *A, int n, int j0, int jb, double2 *Sb,
                               const int32_t *status) {
  if (*status) return;
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= (int64_t)n * jb) return;
  const int q = (int)(e / n), j = (int)(e % n);
  Sb[e] = (j >= j0 && j < j0 + jb) ? double2{0.0, 0.0} : A[(j0 + q) + (int64_t)j * n];
}

// One wave per 16 x 16 tile of A outside the panel, computed transposed so
// that a lane's four results are 16 consecutive rows of a column: tile
// (rows i0.., columns c0..) = (pivot rows zeroed) + (Sb^T Pn^T)^T.
__global__ __launch_bounds__(256) void k_gj_block_update(double2 *A, int n, int j0, int jb,
                                                         const double2 *Sb,
                                                         const int32_t *status) {
  typedef double v4 __attribute__((ext_vector_type(4)));
  if (*status) return;
  const int nt = (n + 15) / 16;
  const int64_t t = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (t >= (int64_t)nt * nt) return;
  const int it = (int)(t % nt), ct = (int)(t / nt);
  const int c0 = ct * 16, i0 = it * 16;
  if (c0 >= j0 && c0 < j0 + jb) return;   // panel columns: tiles never straddle (j0 % 16 == 0)
  const int lane = threadIdx.x & 63, li = lane & 15, lk = lane >> 4;
  const int col = c0 + li, row = i0 + li;
  const bool cok = col < n, rok = row < n;
  v4 re = {0.0, 0.0, 0.0, 0.0}, im = {0.0, 0.0, 0.0, 0.0};
  for (int k0 = 0; k0 < jb; k0 += 4) {
    const int q = k0 + lk;
    const bool qok = q < jb;
    double2 s = Sb[(int64_t)(qok ? q : 0) * n + (cok ? col : 0)];
    double2 pn = A[(rok ? row : 0) + (int64_t)(j0 + (qok ? q : 0)) * n];
    if (!(qok && cok)) s = double2{0.0, 0.0};
    if (!(qok && rok)) pn = double2{0.0, 0.0};
    // (S^T)[col][q] * (Pn^T)[q][row]
    re = __builtin_amdgcn_mfma_f64_16x16x4f64(s.x, pn.x, re, 0, 0, 0);
    re = __builtin_amdgcn_mfma_f64_16x16x4f64(-s.y, pn.y, re, 0, 0, 0);
    im = __builtin_amdgcn_mfma_f64_16x16x4f64(s.x, pn.y, im, 0, 0, 0);
    im = __builtin_amdgcn_mfma_f64_16x16x4f64(s.y, pn.x, im, 0, 0, 0);
  }
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int j = c0 + lk + 4 * v, i = i0 + li;
    if (j >= n || i >= n) continue;
    double2 &a = A[i + (int64_t)j * n];
    const double2 o = (i >= j0 && i < j0 + jb) ? double2{0.0, 0.0} : a;
    a = double2{o.x + re[v], o.y + im[v]};
  }
}

__global__ __launch_bounds__(1024) void k_gj_unpermute(double2 *A, int n, const int32_t *perm,
                                                       const int32_t *status) {
  if (*status) return;
  for (int k = n - 1; k >= 0; --k) {
    const int p = perm[k];
    if (p != k)
      for (int i = threadIdx.x; i < n; i += blockDim.x) {
        const double2 a = A[i + (int64_t)k * n], b = A[i + (int64_t)p * n];
        A[i + (int64_t)k * n] = b;
        A[i + (int64_t)p * n] = a;
      }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// The inclusion term of one product.  Forward (CONJ = false), x = s:
//   part[q][i] = hd sum_{j in chunk q} G[j, i] x_j        (K^{v2s} h^d s)
//   z_i        = sum_q part[q][i]
//   y_i        = w_i sum_k M[i, k] z_k                   (W (K^{s2s})^{-1} z)
//   u_j       += sum_i G[j, i] y_i                        (K^{s2v} ...)
// Adjoint (CONJ = true) with Ma = M^H:
//   z_i = sum_j conj(G[j, i]) x_j,  y_i = sum_k Ma[i, k] w_k z_k,
//   u_j += hd sum_i conj(G[j, i]) y_i.
// ---------------------------------------------------------------------------
template <typename R, bool CONJ>
__global__ __launch_bounds__(256) void k_inc_gather(const cplx_t<R> *G, int64_t Nv, int32_t ns,
                                                    int32_t m, const cplx_t<R> *x, R scale,
                                                    cplx_t<R> *part) {
  using C = cplx_t<R>;
  const int lane = threadIdx.x & 63;
  const int i = blockIdx.y * 4 + (threadIdx.x >> 6);
  const int64_t q = blockIdx.x;
  if (i >= ns) return;
  const int64_t r0 = q * m;
  const int mq = (int)(Nv - r0 < m ? Nv - r0 : m);
  const C *col = G + r0 * ns + (int64_t)i * mq;
  const C *xq = x + r0;
  C acc{0, 0};
  for (int j = lane; j < mq; j += 64) {
    if (CONJ) cfmac(acc, col[j], xq[j]);
    else cfma(acc, col[j], xq[j]);
  }
  acc.x = wave_sum(acc.x);
  acc.y = wave_sum(acc.y);
  if (lane == 0) part[q * ns + i] = C{acc.x * scale, acc.y * scale};
}

template <typename R>
__global__ void k_inc_reduce(const cplx_t<R> *part, int64_t nchunk, int32_t ns, cplx_t<R> *z) {
  using C = cplx_t<R>;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= ns) return;
  C acc{0, 0};
  for (int64_t q = 0; q < nchunk; ++q) {
    const C v = part[q * ns + i];
    acc.x += v.x;
    acc.y += v.y;
  }
  z[i] = acc;
}

// y_i = sum_k A[i + k ns] v_k with v = z (forward, y scaled by w_i after the
// sum) or v = w z (adjoint).  k_inc_small: partial sums over column block
// kb = blockIdx.y of kIncCol columns, one thread per output row;
// k_inc_small_sum adds the blocks in order (256-column blocks keep that sum
// short: with 32 it was a few hundred terms per row on 32 workgroups).
constexpr int kIncCol = 256;

template <typename R, bool ADJ>
__global__ __launch_bounds__(256) void k_inc_small(const cplx_t<R> *A, int32_t ns, const R *w,
                                                   const cplx_t<R> *z, cplx_t<R> *part3) {
  using C = cplx_t<R>;
  __shared__ C vs[kIncCol];
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int k0 = blockIdx.y * kIncCol;
  const int kn = ns - k0 < kIncCol ? ns - k0 : kIncCol;
  if (threadIdx.x < kn) {
    const C v = z[k0 + threadIdx.x];
    vs[threadIdx.x] = ADJ ? C{v.x * w[k0 + threadIdx.x], v.y * w[k0 + threadIdx.x]} : v;
  }
  __syncthreads();
  if (i >= ns) return;
  C acc{0, 0};
  const C *col = A + i + (int64_t)k0 * ns;
#pragma unroll 8
  for (int k = 0; k < kn; ++k) cfma(acc, col[(int64_t)k * ns], vs[k]);
  part3[(int64_t)blockIdx.y * ns + i] = acc;
}

template <typename R, bool ADJ>
__global__ void k_inc_small_sum(const cplx_t<R> *part3, int32_t ns, int32_t nkb, const R *w,
                                cplx_t<R> *y) {
  using C = cplx_t<R>;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= ns) return;
  C acc{0, 0};
  for (int b = 0; b < nkb; ++b) {
    const C v = part3[(int64_t)b * ns + i];
    acc.x += v.x;
    acc.y += v.y;
  }
  y[i] = ADJ ? acc : C{acc.x * w[i], acc.y * w[i]};
}

// Partial sums of u_j over segment block b = blockIdx.y (kIncSeg segments):
// part2[b][j] = sum_{i in b} op(G[j, i]) y_i, loads issued 8 at a time.
constexpr int kIncSeg = 256;

template <typename R, bool CONJ>
__global__ __launch_bounds__(256) void k_inc_scatter(const cplx_t<R> *G, int64_t Nv, int32_t ns,
                                                     int32_t m, const cplx_t<R> *y,
                                                     cplx_t<R> *part2) {
  using C = cplx_t<R>;
  __shared__ C ys[kIncSeg];
  const int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int i0 = blockIdx.y * kIncSeg;
  const int in = ns - i0 < kIncSeg ? ns - i0 : kIncSeg;
  for (int k = threadIdx.x; k < in; k += blockDim.x) ys[k] = y[i0 + k];
  __syncthreads();
  if (j >= Nv) return;
  const int64_t r0 = (j / m) * m;
  const int mq = (int)(Nv - r0 < m ? Nv - r0 : m);
  const C *row = G + r0 * ns + (j - r0) + (int64_t)i0 * mq;
  C acc{0, 0};
  constexpr int B = 8;
  for (int k0 = 0; k0 < in; k0 += B) {
    C g[B];
#pragma unroll
    for (int b = 0; b < B; ++b) g[b] = k0 + b < in ? row[(int64_t)(k0 + b) * mq] : C{0, 0};
#pragma unroll
    for (int b = 0; b < B; ++b) {
      if (k0 + b < in) {
        if (CONJ) cfmac(acc, g[b], ys[k0 + b]);
        else cfma(acc, g[b], ys[k0 + b]);
      }
    }
  }
  part2[(int64_t)blockIdx.y * Nv + j] = acc;
}

// u_j += scale * sum_b part2[b][j], blocks in order.
template <typename R>
__global__ void k_inc_add(const cplx_t<R> *part2, int64_t Nv, int32_t nb, R scale, cplx_t<R> *u) {
  using C = cplx_t<R>;
  const int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (j >= Nv) return;
  C acc{0, 0};
  for (int b = 0; b < nb; ++b) {
    const C v = part2[(int64_t)b * Nv + j];
    acc.x += v.x;
    acc.y += v.y;
  }
  const C o = u[j];
  u[j] = C{o.x + scale * acc.x, o.y + scale * acc.y};
}

__global__ void k_scale_cols_neg(double2 *A, int32_t n, const double *w) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= (int64_t)n * n) return;
  const double s = -w[e / n];
  A[e] = double2{A[e].x * s, A[e].y * s};
}

// dst = src^H (column-major n x n)
__global__ void k_conj_transpose(const double2 *src, int32_t n, double2 *dst) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= (int64_t)n * n) return;
  const int64_t i = e % n, j = e / n;
  const double2 v = src[j + i * n];
  dst[e] = double2{v.x, -v.y};
}

// ---------------------------------------------------------------------------
// Host-side launchers.
// ---------------------------------------------------------------------------
hipError_t launch_point_setup(const DevProblem &P, const double *xy, const double *w,
                              const double *slow, int32_t ns, int64_t p0, double *xyz,
                              double *lw, int32_t *box, double2 *self, hipStream_t st) {
  if (ns <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_point_setup, dim3((ns + 255) / 256), dim3(256), 0, st, P, xy, w, slow,
                     ns, p0, xyz, lw, box, self);
  return hipGetLastError();
}

// -diag(w)-scaled columns, then the in-place Gauss-Jordan inverse, by
// panels of kGjPanel columns (Sb: kGjPanel x n scratch) or, with Sb null,
// column by column.
hipError_t launch_s2s_inverse(double2 *A, int32_t n, const double *w, int32_t *perm,
                              double2 *colk, double2 *Sb, int32_t *status, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  const int64_t nn = (int64_t)n * n;
  const int T = 256;
  hipLaunchKernelGGL(k_scale_cols_neg, dim3((nn + T - 1) / T), dim3(T), 0, st, A, n, w);
  if (!Sb) {
    for (int k = 0; k < n; ++k) {
      hipLaunchKernelGGL(k_gj_pivot, dim3(1), dim3(1024), 0, st, A, n, k, perm, colk, status);
      hipLaunchKernelGGL(k_gj_update, dim3((nn + T - 1) / T), dim3(T), 0, st, A, n, k, colk,
                         status);
    }
  } else {
    const int nt = (n + 15) / 16;
    const int64_t ntile = (int64_t)nt * nt;
    for (int j0 = 0; j0 < n; j0 += kGjPanel) {
      const int jb = n - j0 < kGjPanel ? n - j0 : kGjPanel;
      const int64_t np = (int64_t)n * jb;
      for (int k = j0; k < j0 + jb; ++k) {
        hipLaunchKernelGGL(k_gj_pivot_panel, dim3(1), dim3(1024), 0, st, A, n, k, j0, jb, perm,
                           colk, status);
        hipLaunchKernelGGL(k_gj_update_panel, dim3((np + T - 1) / T), dim3(T), 0, st, A, n, k, j0,
                           jb, colk, status);
      }
      if (jb == n) break;
      hipLaunchKernelGGL(k_gj_copy_rows, dim3((np + T - 1) / T), dim3(T), 0, st, A, n, j0, jb,
                         Sb, status);
      hipLaunchKernelGGL(k_gj_block_update, dim3((unsigned)((ntile + 3) / 4)), dim3(256), 0, st,
                         A, n, j0, jb, Sb, status);
    }
  }
  hipLaunchKernelGGL(k_gj_unpermute, dim3(1), dim3(1024), 0, st, A, n, perm, status);
  return hipGetLastError();
}

hipError_t launch_conj_transpose(const double2 *src, int32_t n, double2 *dst, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  const int64_t nn = (int64_t)n * n;
  hipLaunchKernelGGL(k_conj_transpose, dim3((nn + 255) / 256), dim3(256), 0, st, src, n, dst);
  return hipGetLastError();
}

template <typename R>
hipError_t launch_inclusion_apply(const InclusionPlan &ip, const void *x, void *u, R hd,
                                  bool adjoint, hipStream_t st) {
  using C = cplx_t<R>;
  const C *G = (const C *)ip.G;
  C *part = (C *)ip.part;
  C *z = (C *)ip.z;
  C *y = (C *)ip.y;
  const R *w = (const R *)ip.w;
  const int32_t nkb = (ip.ns + kIncCol - 1) / kIncCol;
  const dim3 gm((unsigned)((ip.ns + 255) / 256), (unsigned)nkb);
  C *part3 = (C *)ip.part3;
  if (ip.bf) {
    // z = h^d G^T x (forward) or G^H x (adjoint), then the K^{s2s} step, then
    // u += G y (forward) or h^d conj(G) y (adjoint)
    hipError_t e = launch_s2v<R>(*ip.bf, x, z, adjoint ? (R)1 : hd, true, adjoint, st);
    if (e != hipSuccess) return e;
    if (!adjoint) {
      hipLaunchKernelGGL((k_inc_small<R, false>), gm, dim3(256), 0, st, (const C *)ip.M, ip.ns, w,
                         (const C *)z, part3);
      hipLaunchKernelGGL((k_inc_small_sum<R, false>), dim3((ip.ns + 255) / 256), dim3(256), 0,
                         st, (const C *)part3, ip.ns, nkb, w, y);
    } else {
      hipLaunchKernelGGL((k_inc_small<R, true>), gm, dim3(256), 0, st, (const C *)ip.MH, ip.ns, w,
                         (const C *)z, part3);
      hipLaunchKernelGGL((k_inc_small_sum<R, true>), dim3((ip.ns + 255) / 256), dim3(256), 0,
                         st, (const C *)part3, ip.ns, nkb, w, y);
    }
    return launch_s2v<R>(*ip.bf, y, u, adjoint ? hd : (R)1, false, adjoint, st);
  }
  const int64_t nchunk = (ip.Nv + ip.m - 1) / ip.m;
  const dim3 gg((unsigned)nchunk, (unsigned)((ip.ns + 3) / 4));
  if (!adjoint) {
    hipLaunchKernelGGL((k_inc_gather<R, false>), gg, dim3(256), 0, st, G, ip.Nv, ip.ns, ip.m,
                       (const C *)x, hd, part);
  } else {
    hipLaunchKernelGGL((k_inc_gather<R, true>), gg, dim3(256), 0, st, G, ip.Nv, ip.ns, ip.m,
                       (const C *)x, (R)1, part);
  }
  hipLaunchKernelGGL((k_inc_reduce<R>), dim3((ip.ns + 255) / 256), dim3(256), 0, st,
                     (const C *)part, nchunk, ip.ns, z);
  const int32_t nb = (ip.ns + kIncSeg - 1) / kIncSeg;
  const dim3 gs((unsigned)((ip.Nv + 255) / 256), (unsigned)nb);
  C *part2 = (C *)ip.part2;
  if (!adjoint) {
    hipLaunchKernelGGL((k_inc_small<R, false>), gm, dim3(256), 0, st, (const C *)ip.M, ip.ns, w,
                       (const C *)z, part3);
    hipLaunchKernelGGL((k_inc_small_sum<R, false>), dim3((ip.ns + 255) / 256), dim3(256), 0, st,
                       (const C *)part3, ip.ns, nkb, w, y);
    hipLaunchKernelGGL((k_inc_scatter<R, false>), gs, dim3(256), 0, st, G, ip.Nv, ip.ns, ip.m,
                       (const C *)y, part2);
  } else {
    hipLaunchKernelGGL((k_inc_small<R, true>), gm, dim3(256), 0, st, (const C *)ip.MH, ip.ns, w,
                       (const C *)z, part3);
    hipLaunchKernelGGL((k_inc_small_sum<R, true>), dim3((ip.ns + 255) / 256), dim3(256), 0, st,
                       (const C *)part3, ip.ns, nkb, w, y);
    hipLaunchKernelGGL((k_inc_scatter<R, true>), gs, dim3(256), 0, st, G, ip.Nv, ip.ns, ip.m,
                       (const C *)y, part2);
  }
  hipLaunchKernelGGL((k_inc_add<R>), dim3((unsigned)((ip.Nv + 255) / 256)), dim3(256), 0, st,
                     (const C *)part2, ip.Nv, nb, adjoint ? hd : (R)1, (C *)u);
  return hipGetLastError();
}

template hipError_t launch_inclusion_apply<double>(const InclusionPlan &, const void *, void *,
                                                   double, bool, hipStream_t);
template hipError_t launch_inclusion_apply<float>(const InclusionPlan &, const void *, void *,
                                                  float, bool, hipStream_t);

}  // namespace hbi
