// HIP kernels of the single butterfly of the inclusion's cells x segments
// matrix G, G[j, i] = g(r_j, r^s_i) (Sec. 4.2, K^{s2v} compressed as one
// butterfly with L = min(L_v, L_s) levels; K^{s2v} = G W and K^{v2s} = G^T
// since g is reciprocal):
//
//   G = K^L W^L ... W^1 V^0          (eq. butterfly_mat)
//
// V^0 is block diagonal over the 2^L segment leaves, W^k over the units of
// level k (a sibling pair of row nodes over the same candidate columns),
// K^L over the 2^L cell nodes of depth L.  Every V and W block is an
// interpolation matrix X = [I, T] Pi^T of which only T is stored (column
// major), with the column order and its inverse in the index store.
//
//   k_s2v_v,  k_s2v_w,  k_s2v_k      y += scale op(G) x      (segments -> cells)
//   k_s2v_kt, k_s2v_wt, k_s2v_vt     z  = scale op(G)^T x    (cells -> segments)
//
// op(a) = conj(a) when CONJ, else a.  Gathers only, one writer per output
// element, sums in a fixed order: results are bitwise repeatable.  The
// transfer and K^L-transposed kernels give each output a wave (lanes over
// its sum), so that a sum of a few hundred terms is not one lane's chain of
// dependent loads; their workgroups (four outputs each) come from exact
// item lists, not a grid sized for the largest unit.
#include "hbi_kernels.h"
#include "hbi_device.h"

namespace hbi {

template <bool CONJ, typename C> __device__ __forceinline__ void fma_op(C &acc, C a, C b) {
  if (CONJ) cfmac(acc, a, b);
  else cfma(acc, a, b);
}

// V^0, forward: row i of leaf block X = [I, T] Pi^T (r x n, inputs the
// segments [lo, lo + n)) is x[lo + ord[i]] + sum_m T[i, m] x[lo + ord[r + m]].
template <typename R, bool CONJ>
__global__ __launch_bounds__(64) void k_s2v_v(const S2VLeaf *lv, const cplx_t<R> *F,
                                              const uint16_t *idx, const cplx_t<R> *x,
                                              cplx_t<R> *z) {
  using C = cplx_t<R>;
  const S2VLeaf d = lv[blockIdx.x];
  const uint16_t *ord = idx + d.ioff;
  const C *T = F + d.foff;
  const C *xl = x + d.lo;
  for (int i = threadIdx.x; i < d.r; i += 64) {
    C acc = xl[ord[i]];
    for (int m = 0; m < d.n - d.r; ++m) fma_op<CONJ>(acc, T[i + (int64_t)m * d.r], xl[ord[d.r + m]]);
    z[d.zoff + i] = acc;
  }
}

// W^k, forward: one wave per row of child a (then b) of a unit, over its c
// inputs zin = z[U.zin ..]: row i of X_a is zin[ia[i]] + sum_m T_a[i, m]
// zin[ia[ra + m]], the lanes taking m = lane, lane + 64, ... and their
// partial sums added in a fixed tree.
template <typename R, bool CONJ>
__global__ __launch_bounds__(256) void k_s2v_w(const WUnit *units, const int2 *items,
                                               const cplx_t<R> *F, const uint16_t *idx,
                                               cplx_t<R> *z) {
  using C = cplx_t<R>;
  const int2 it = items[blockIdx.x];
  const WUnit U = units[it.x];
  const int ii = it.y + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (ii >= U.ra + U.rb) return;
  const C *zin = z + U.zin;
  const bool b = ii >= U.ra;
  const int i = b ? ii - U.ra : ii, r = b ? U.rb : U.ra;
  const uint16_t *ord = idx + U.ioff + (b ? U.c : 0);
  const C *T = F + U.foff + (b ? (int64_t)U.ra * (U.c - U.ra) : 0);
  C acc{0, 0};
  for (int m = lane; m < U.c - r; m += 64) fma_op<CONJ>(acc, T[i + (int64_t)m * r], zin[ord[r + m]]);
  acc.x = wave_sum(acc.x);
  acc.y = wave_sum(acc.y);
  if (lane == 0) {
    const C x0 = zin[ord[i]];
    z[(b ? U.zoutb : U.zouta) + i] = C{acc.x + x0.x, acc.y + x0.y};
  }
}

// K^L, forward: y[perm[start + p]] += scale sum_k K[p, k] z[zoff + k] over
// the rows p of one cell node (K column major size x r).
template <typename R, bool CONJ>
__global__ __launch_bounds__(256) void k_s2v_k(const S2VNode *nodes, const cplx_t<R> *F,
                                               const int32_t *perm, const cplx_t<R> *z, R scale,
                                               cplx_t<R> *y) {
  using C = cplx_t<R>;
  const S2VNode d = nodes[blockIdx.x];
  const int p = blockIdx.y * 256 + threadIdx.x;
  if (p >= d.size) return;
  const C *K = F + d.foff + p;
  const C *zz = z + d.zoff;
  C acc{0, 0};
  // loads issued eight at a time before their products
  constexpr int B = 8;
  for (int k0 = 0; k0 < d.r; k0 += B) {
    C kv[B], zv[B];
#pragma unroll
    for (int q = 0; q < B; ++q) {
      const int k = k0 + q < d.r ? k0 + q : d.r - 1;
      kv[q] = K[(int64_t)k * d.size];
      zv[q] = zz[k];
    }
#pragma unroll
    for (int q = 0; q < B; ++q)
      if (k0 + q < d.r) fma_op<CONJ>(acc, kv[q], zv[q]);
  }
  const int64_t j = perm[d.start + p];
  const C o = y[j];
  y[j] = C{o.x + scale * acc.x, o.y + scale * acc.y};
}

// K^L, transposed: z[zoff + k] = scale sum_p K[p, k] x[perm[start + p]], one
// wave per skeleton column k (lane-strided partial sums, then a fixed tree);
// a workgroup's four columns share the node's inputs, gathered once into
// LDS when they fit (kKtLds entries).
constexpr int kKtLds = 2048;
template <typename R, bool CONJ>
__global__ __launch_bounds__(256) void k_s2v_kt(const S2VNode *nodes, const int2 *items,
                                                const cplx_t<R> *F, const int32_t *perm,
                                                const cplx_t<R> *x, R scale, cplx_t<R> *z) {
  using C = cplx_t<R>;
  __shared__ C xs[kKtLds];
  const int2 it = items[blockIdx.x];
  const S2VNode d = nodes[it.x];
  const bool lds = d.size <= kKtLds;
  if (lds)
    for (int p = threadIdx.x; p < d.size; p += 256) xs[p] = x[perm[d.start + p]];
  __syncthreads();
  const int k = it.y + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (k >= d.r) return;
  const C *K = F + d.foff + (int64_t)k * d.size;
  C acc{0, 0};
  if (lds) {
    int p = lane;
    for (; p + 192 < d.size; p += 256) {
      C kv[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) kv[u] = K[p + 64 * u];
#pragma unroll
      for (int u = 0; u < 4; ++u) fma_op<CONJ>(acc, kv[u], xs[p + 64 * u]);
    }
    for (; p < d.size; p += 64) fma_op<CONJ>(acc, K[p], xs[p]);
  } else {
    for (int p = lane; p < d.size; p += 64) fma_op<CONJ>(acc, K[p], x[perm[d.start + p]]);
  }
  acc.x = wave_sum(acc.x);
  acc.y = wave_sum(acc.y);
  if (lane == 0) z[d.zoff + k] = C{scale * acc.x, scale * acc.y};
}

// W^k, transposed: one wave per input q of a unit, which gets
// X_a[:, q]^T za + X_b[:, q]^T zb; with p = pa[q] the column of X_a is the
// unit vector e_p when p < ra, else column p - ra of T_a (likewise for b).
// The lanes take the rows i = lane, lane + 64, ...
template <typename R, bool CONJ>
__global__ __launch_bounds__(256) void k_s2v_wt(const WUnit *units, const int2 *items,
                                                const cplx_t<R> *F, const uint16_t *idx,
                                                cplx_t<R> *z) {
  using C = cplx_t<R>;
  const int2 it = items[blockIdx.x];
  const WUnit U = units[it.x];
  const int q = it.y + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (q >= U.c) return;
  const uint16_t *pa = idx + U.ioff + 2 * (int64_t)U.c, *pb = pa + U.c;
  const C *Ta = F + U.foff, *Tb = Ta + (int64_t)U.ra * (U.c - U.ra);
  const C *za = z + U.zouta, *zb = z + U.zoutb;
  const int p = pa[q], pq = pb[q];
  C acc{0, 0};
  if (p >= U.ra) {
    const C *t = Ta + (int64_t)(p - U.ra) * U.ra;
    for (int i = lane; i < U.ra; i += 64) fma_op<CONJ>(acc, t[i], za[i]);
  }
  if (pq >= U.rb) {
    const C *t = Tb + (int64_t)(pq - U.rb) * U.rb;
    for (int i = lane; i < U.rb; i += 64) fma_op<CONJ>(acc, t[i], zb[i]);
  }
  acc.x = wave_sum(acc.x);
  acc.y = wave_sum(acc.y);
  if (lane == 0) {
    if (p < U.ra) { acc.x += za[p].x; acc.y += za[p].y; }
    if (pq < U.rb) { acc.x += zb[pq].x; acc.y += zb[pq].y; }
    z[U.zin + q] = acc;
  }
}

// V^0, transposed: segment lo + q gets X[:, q]^T z_leaf (inverse order inv).
template <typename R, bool CONJ>
__global__ __launch_bounds__(64) void k_s2v_vt(const S2VLeaf *lv, const cplx_t<R> *F,
                                               const uint16_t *idx, const cplx_t<R> *z,
                                               cplx_t<R> *y) {
  using C = cplx_t<R>;
  const S2VLeaf d = lv[blockIdx.x];
  const uint16_t *inv = idx + d.ioff + d.n;
  const C *zl = z + d.zoff;
  for (int q = threadIdx.x; q < d.n; q += 64) {
    const int p = inv[q];
    C acc{0, 0};
    if (p < d.r) {
      acc = zl[p];
    } else {
      const C *t = F + d.foff + (int64_t)(p - d.r) * d.r;
      for (int i = 0; i < d.r; ++i) fma_op<CONJ>(acc, t[i], zl[i]);
    }
    y[d.lo + q] = acc;
  }
}

template <typename R, bool CONJ>
static void s2v_forward(const S2VPlan &p, const cplx_t<R> *x, cplx_t<R> *y, R scale,
                        hipStream_t st) {
  using C = cplx_t<R>;
  const C *F = (const C *)p.F;
  C *z = (C *)p.z;
  hipLaunchKernelGGL((k_s2v_v<R, CONJ>), dim3((unsigned)p.nleaf), dim3(64), 0, st, p.leaves, F,
                     p.idx, x, z);
  for (int k = 1; k <= p.L; ++k)
    if (p.nwitems[k])
      hipLaunchKernelGGL((k_s2v_w<R, CONJ>), dim3((unsigned)p.nwitems[k]), dim3(256), 0, st,
                         p.units[k], p.witems[k], F, p.idx, z);
  hipLaunchKernelGGL((k_s2v_k<R, CONJ>), dim3((unsigned)p.nnode, (p.size_max + 255) / 256),
                     dim3(256), 0, st, p.nodes, F, p.perm, (const C *)z, scale, y);
}

template <typename R, bool CONJ>
static void s2v_transpose(const S2VPlan &p, const cplx_t<R> *x, cplx_t<R> *y, R scale,
                          hipStream_t st) {
  using C = cplx_t<R>;
  const C *F = (const C *)p.F;
  C *z = (C *)p.z;
  hipLaunchKernelGGL((k_s2v_kt<R, CONJ>), dim3((unsigned)p.nktitems), dim3(256), 0, st, p.nodes,
                     p.ktitems, F, p.perm, x, scale, z);
  for (int k = p.L; k >= 1; --k)
    if (p.nwtitems[k])
      hipLaunchKernelGGL((k_s2v_wt<R, CONJ>), dim3((unsigned)p.nwtitems[k]), dim3(256), 0, st,
                         p.units[k], p.wtitems[k], F, p.idx, z);
  hipLaunchKernelGGL((k_s2v_vt<R, CONJ>), dim3((unsigned)p.nleaf), dim3(64), 0, st, p.leaves, F,
                     p.idx, (const C *)z, y);
}

template <typename R>
hipError_t launch_s2v(const S2VPlan &p, const void *x, void *y, R scale, bool transpose,
                      bool conj, hipStream_t st) {
  using C = cplx_t<R>;
  if (p.nleaf <= 0 || p.nnode <= 0 || (int)p.units.size() != p.L + 1 ||
      (int)p.nunits.size() != p.L + 1 || (int)p.witems.size() != p.L + 1 ||
      (int)p.wtitems.size() != p.L + 1 || (int)p.nwitems.size() != p.L + 1 ||
      (int)p.nwtitems.size() != p.L + 1 || p.size_max <= 0 || p.nktitems <= 0)
    return hipErrorInvalidValue;
  if (!transpose) {
    if (conj) s2v_forward<R, true>(p, (const C *)x, (C *)y, scale, st);
    else s2v_forward<R, false>(p, (const C *)x, (C *)y, scale, st);
  } else {
    if (conj) s2v_transpose<R, true>(p, (const C *)x, (C *)y, scale, st);
    else s2v_transpose<R, false>(p, (const C *)x, (C *)y, scale, st);
  }
  return hipGetLastError();
}

template hipError_t launch_s2v<float>(const S2VPlan &, const void *, void *, float, bool, bool,
                                      hipStream_t);
template hipError_t launch_s2v<double>(const S2VPlan &, const void *, void *, double, bool, bool,
                                       hipStream_t);

}  // namespace hbi
