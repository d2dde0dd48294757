// HIP kernels of the butterfly apply for gfx950 (wave64), one right-hand
// side at a time.
//
//   bf_apply  k_vstage, k_wstage, k_final             (u = K h^d s)
//   adjoint   k_final_adj, k_wstage_adj, k_vstage_adj  (u = h^d K^H s)
#include <type_traits>

#include "hbi_kernels.h"
#include "hbi_device.h"

namespace hbi {

// ---------------------------------------------------------------------------
// bf_apply (eq. butterfly_mat): V^0 per column leaf, transfer stages W^k,
// skeleton factor K^L plus the dense diagonal leaf per row leaf.  Gathers
// only: every output element is written by exactly one lane.
// ---------------------------------------------------------------------------
// acc += sum_{i < n} op(m(i), x(i)) in order of i, with the loads issued B
// at a time (predicated past n) before any of them is consumed: a plain
// unrolled loop leaves a short trip count to a remainder loop that waits for
// every load in turn.
template <int B, bool CONJ, typename C, typename MF, typename XF>
__device__ __forceinline__ void batched_dot(C &acc, int n, MF m, XF x) {
  for (int b = 0; b < n; b += B) {
    C mv[B], xv[B];
#pragma unroll
    for (int u = 0; u < B; ++u) {
      if (b + u < n) {
        mv[u] = m(b + u);
        xv[u] = x(b + u);
      } else {
        mv[u] = C{0, 0};
        xv[u] = C{0, 0};
      }
    }
#pragma unroll
    for (int u = 0; u < B; ++u) {
      if (CONJ) cfmac(acc, mv[u], xv[u]);
      else cfma(acc, mv[u], xv[u]);
    }
  }
}
template <typename C> struct LoadBatch { static constexpr int value = sizeof(C) == 8 ? 16 : 8; };
// Factor entries are read once per product: non-temporal loads keep them
// from displacing the skeleton vectors z in the caches.
template <typename C> __device__ __forceinline__ C ldf(const C *p) {
  using E = decltype(C{}.x);
  typedef E V __attribute__((ext_vector_type(2)));
  const V v = __builtin_nontemporal_load((const V *)p);
  return C{v[0], v[1]};
}
// Factor load with the non-temporal hint or without it.  Measured on the
// 1024^2 FP32 apply: the short per-wave streams of the FP32 transfer stages
// and of the adjoint's K^L stage run 3 % and 12 % faster with plain loads,
// while the leaf stages and every FP64 stage are faster with the hint.
template <bool NTL, typename C> __device__ __forceinline__ C ldx(const C *p) {
  if constexpr (NTL) return ldf(p);
  else return *p;
}
// FP32 transfer stages and adjoint K^L stage: plain loads
template <typename R> struct PlainF32 { static constexpr bool nt = sizeof(R) != 4; };

// y[0..R) = M x for a column-major R x c matrix M streamed by one wave.
// Lane l works on row l % R of column group l / R (G = 64 / R groups when
// R <= 32), so every load instruction of the wave reads one contiguous span
// of G*R entries; partial sums of a row are combined with lane permutes in a
// fixed order.  For R > 32 lanes take rows (64 at a time) and columns are
// walked in order.  Returns the result for row `lane` (lane < R, R <= 64) or
// writes through `store` for larger R.
template <typename C, typename XF, typename ST>
__device__ __forceinline__ void wave_gemv(const C *__restrict__ M, int Rt, int c, int lane,
                                          XF xat, ST store, int r0 = 0, int r1 = 1 << 30) {
  if (Rt <= 32) {
    const int G = 64 / Rt;
    const int grp = lane / Rt;
    const bool act = grp < G;
    C acc{0, 0};
    if (act) {
      const C *p = M + lane;
      const int step = G * Rt;
      const int nt = (c - grp + G - 1) / G;   // columns grp, grp + G, ...
      batched_dot<LoadBatch<C>::value, false>(
          acc, nt, [&](int t) { return ldf(p + (int64_t)t * step); },
          [&](int t) { return xat(grp + t * G); });
    }
    // combine the G partial sums of each row (lanes row, row+Rt, ...)
    C tot = acc;
    for (int g = 1; g < G; ++g) {
      const int src = lane + g * Rt;
      const auto re = __shfl(acc.x, src < 64 ? src : lane, 64);
      const auto im = __shfl(acc.y, src < 64 ? src : lane, 64);
      if (src < 64) { tot.x += re; tot.y += im; }
    }
    if (lane < Rt) store(lane, tot);
  } else {
    const int re_ = r1 < Rt ? r1 : Rt;
    for (int rb = r0; rb < re_; rb += 64) {
      const int row = rb + lane;
      if (row < re_) {
        C acc{0, 0};
        const C *p = M + row;
        batched_dot<LoadBatch<C>::value, false>(
            acc, c, [&](int col) { return ldf(p + (int64_t)col * Rt); }, [&](int col) { return xat(col); });
        store(row, acc);
      }
    }
  }
}

// One workgroup (4 waves) per leaf; wave w handles the HODBF levels
// l = w, w + 4, ... of the leaf (at most kVq of them).  Each block is
// V = [I, T] Pi^T: the leaf's inputs are permuted into the block's column
// order in the wave's LDS slice, then row k is xp[k] + sum_m T[k, m]
// xp[r + m].  A wave loads the descriptors and column orders of all its
// blocks at once, while the leaf's inputs are gathered, so that each block
// then waits only for its own factor stream (one block after another, each
// waited on three dependent loads).  Batches of 8 instead of 16 entries per
// lane (7 or 8 waves per SIMD instead of 5) measured the same; issuing the
// next block's first batch before the current block is consumed took 124
// registers (4 waves per SIMD) and was 7 % slower.
constexpr int kVq = 8;   // blocks per wave: L_v <= 4 kVq
template <typename R>
__global__ __launch_bounds__(256) void k_vstage(const cplx_t<R> *s,
                                                const LeafInfo *leaves,
                                                const int32_t *perm,
                                                const VDesc *vd, int Lv,
                                                const uint16_t *fidx,
                                                const cplx_t<R> *F,
                                                cplx_t<R> *z, R hd) {
  using C = cplx_t<R>;
  __shared__ C xs[HBI_MAX_LEAF];
  __shared__ C xp[4][HBI_MAX_LEAF];
  const int g = blockIdx.x;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const LeafInfo lf = leaves[g];
  const int sz = lf.size;
  const int nq = wave < Lv ? (Lv - wave + 3) / 4 : 0;
  VDesc dq[kVq];
  int ix[kVq];
#pragma unroll
  for (int q = 0; q < kVq; ++q)
    if (q < nq) dq[q] = vd[(int64_t)g * Lv + wave + 4 * q];
#pragma unroll
  for (int q = 0; q < kVq; ++q) ix[q] = (q < nq && lane < sz) ? fidx[dq[q].ioff + lane] : 0;
  if (threadIdx.x < sz) {
    const C v = s[perm[lf.start + threadIdx.x]];
    xs[threadIdx.x] = C{v.x * hd, v.y * hd};
  }
  __syncthreads();
  C *xw = xp[wave];
#pragma unroll
  for (int q = 0; q < kVq; ++q) {
    if (q >= nq) break;
    const VDesc d = dq[q];
    wave_lds_sync();   // the previous block's reads of xw are done
    if (lane < sz) xw[lane] = xs[ix[q]];
    wave_lds_sync();
    C *zo = z + d.zout;
    const int r = d.r;
    wave_gemv<C>(F + d.foff, r, sz - r, lane, [&](int col) { return xw[r + col]; },
                 [&](int row, C v) { zo[row] = C{v.x + xw[row].x, v.y + xw[row].y}; });
  }
}

// One lane's share of a row of a column-major factor block: entries
// T[0], T[step], ... (nt of them), streamed B at a time.  issue(q0) loads
// entries q0 .. q0 + B - 1 (zero past nt), so the first batch can be issued
// before the lane's inputs are ready.
template <typename C, int B, bool NTL> struct RowStream {
  const C *T;
  int64_t step;
  int nt;
  C mv[B];
  __device__ __forceinline__ void issue(int q0) {
#pragma unroll
    for (int u = 0; u < B; ++u)
      mv[u] = q0 + u < nt ? ldx<NTL>(T + (int64_t)(q0 + u) * step) : C{0, 0};
  }
  // sum_q T[q step] x(q) in order of q; the first batch must have been issued
  template <typename XF> __device__ __forceinline__ C dot(XF x) {
    C acc{0, 0};
    for (int q0 = 0; q0 < nt; q0 += B) {
      if (q0 > 0) issue(q0);
#pragma unroll
      for (int u = 0; u < B; ++u) {
        const int q = q0 + u < nt ? q0 + u : nt - 1;   // padding entries are zero
        cfma(acc, mv[u], x(q));
      }
    }
    return acc;
  }
};

// Lanes of a wave on rows [r0, r0 + wr) of a column-major block: lane l takes
// row r0 + l % wr and the columns g, g + G, ... with g = l / wr, G = 64 / wr.
// Sums the G partial sums of each row into its group-0 lane (a fixed tree
// order, so results are bitwise repeatable).
template <typename C>
__device__ __forceinline__ C group_sum(C acc, int lane, int wr, int G) {
  const int grp = lane / wr;
  for (int off = 1; off < G; off <<= 1) {
    const int src = lane + off * wr;
    const auto re = __shfl(acc.x, src < 64 ? src : lane, 64);
    const auto im = __shfl(acc.y, src < 64 ? src : lane, 64);
    if ((grp & (2 * off - 1)) == 0 && grp + off < G) { acc.x += re; acc.y += im; }
  }
  return acc;
}

// Forward transfer stage (FP64; FP32 runs k_wstage_pair below, the same
// work with rows in pairs).  Row i of child a of a unit is
// x[ia[i]] + sum_m T_a[i, m] x[ia[ra + m]] (X = [I, T] Pi^T), likewise for b
// with its own column order ib.  A work item is rows [r0, r0 + wr) of a unit
// (the pair stacked a then b; all rows when it has at most 32), one wave,
// lanes on (row, column group) as in group_sum.  A wave loads the item's
// descriptor, then at once the unit's first 128 inputs and column-order
// words and the first batch of T, so that the factor stream is in flight
// while the raw inputs and the orders ia, ib (as 32-bit words) land in the
// wave's LDS slice; each use then reads its input through the order in LDS.
// Units whose inputs and orders would not fit cap_lds entries of the slice
// gather their inputs from global memory.  Items are ordered by decreasing
// cost, and the factor store holds the units in that order.  Measured and
// dropped: the two permuted lists formed in LDS first (slower), persistent
// waves looping over items with the next descriptor prefetched (slower),
// the producers scattering their outputs straight into both consumer orders
// (twice the output writes, scattered: slower).  Factor batches of 4 to 16
// entries per lane, 2 to 6 staging loads per lane issued ahead and 5 to 8
// waves per SIMD all ran within 5 % of each other in FP32 (this
// configuration the fastest), so the stage is not bound by the loads one
// wave keeps in flight.
// Each wave is a workgroup of its own (1-2 % faster than four per
// workgroup: a finished wave's slot and LDS are not held by the others).
template <typename R, int B>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(8, 8))) void k_wstage(
    const WItem *items, int64_t nitems, const uint16_t *fidx, const cplx_t<R> *F,
    cplx_t<R> *z, int cap_lds) {
  using C = cplx_t<R>;
  constexpr int WX = HBI_WSTAGE_LDS_BYTES / (int)sizeof(C);   // LDS entries of the wave
  constexpr int NS = 2;   // staging loads per lane issued before T
  __shared__ C xs[WX];
  const int lane = threadIdx.x;
  const int64_t it = blockIdx.x;
  if (it >= nitems) return;
  const WItem U = items[it];
  const int ra = U.ra, rb = U.rb, c = U.c, Rt = ra + rb;
  const int wr = Rt <= 32 ? Rt : U.wr;
  const int G = 64 / wr;
  const int r0 = Rt <= 32 ? 0 : U.off;
  const int row = r0 + lane % wr, grp = lane / wr;
  const bool act = row < Rt && row < r0 + wr && grp < G;
  const bool isb = row >= ra;
  const int i = isb ? row - ra : row;
  const int rc = isb ? rb : ra;
  const int t = c - rc;
  const int ob = isb ? c : 0;          // this row's column order: ia or ib
  const int j0 = ob + rc + grp;        // its first non-skeleton column position
  const uint16_t *ia = fidx + U.ioff;  // ia, then ib at ia + c (4-byte aligned)
  const uint32_t *ia32 = (const uint32_t *)ia;
  const C *zin = z + U.zin;
  RowStream<C, B, PlainF32<R>::nt> S;
  S.T = F + U.foff + (isb ? (int64_t)ra * (c - ra) : 0) + i + (int64_t)grp * rc;
  S.step = (int64_t)G * rc;
  S.nt = act && t > grp ? (t - grp + G - 1) / G : 0;
  const int cw = (4 * c + (int)sizeof(C) - 1) / (int)sizeof(C);   // entries the orders take
  C acc, x0;
  if (c + cw <= cap_lds) {
    C *xw = xs;
    uint32_t *iw32 = (uint32_t *)(xw + c);
    const uint16_t *iw = (const uint16_t *)iw32;
    C xr[NS];
    uint32_t ir[NS];
#pragma unroll
    for (int u = 0; u < NS; ++u) {
      const int k = lane + 64 * u;
      xr[u] = k < c ? zin[k] : C{0, 0};
      ir[u] = k < c ? ia32[k] : 0u;
    }
    S.issue(0);
    for (int k = 64 * NS + lane; k < c; k += 64) { xw[k] = zin[k]; iw32[k] = ia32[k]; }
#pragma unroll
    for (int u = 0; u < NS; ++u) {
      const int k = lane + 64 * u;
      if (k < c) { xw[k] = xr[u]; iw32[k] = ir[u]; }
    }
    wave_lds_sync();
    acc = S.dot([&](int q) { return xw[iw[j0 + q * G]]; });
    x0 = xw[iw[ob + (act ? i : 0)]];
  } else {
    S.issue(0);
    acc = S.dot([&](int q) { return zin[ia[j0 + q * G]]; });
    x0 = zin[ia[ob + (act ? i : 0)]];
  }
  acc = group_sum(acc, lane, wr, G);
  if (act && grp == 0) (isb ? z + U.zoutb : z + U.zouta)[i] = C{acc.x + x0.x, acc.y + x0.y};
}

// FP32 forward transfer stage with row pairs: lane (p, g) takes rows i and
// i + 1 of one child (pairs never straddle the two children) and the
// columns g, g + G, ... (G = 64 / pairs), loading both entries of a column
// with one 16-byte load, so a wave issues half the factor-load
// instructions of k_wstage for the same bytes.  The pair's second entry of
// an odd child is the next column's first (or, for the last column, the
// entry after the block, inside the store's two spare entries) and is not
// used.  Staging and column orders as in k_wstage.  The stage's waves spend
// much of their life ready but waiting for issue behind the others' memory
// instructions: the pairs took it from 63.8 to 58.7 us per launch on the
// 1024^2 bump; staging the inputs and orders with 16-byte loads as well
// measured slower (59.6 us), as did 8 pairs per batch (spills).
template <int B>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(8, 8))) void k_wstage_pair(
    const WItem *items, int64_t nitems, const uint16_t *fidx, const cplx_t<float> *F,
    cplx_t<float> *z, int cap_lds) {
  using C = cplx_t<float>;
  typedef float F4 __attribute__((ext_vector_type(4), aligned(8)));
  constexpr int WX = HBI_WSTAGE_LDS_BYTES / (int)sizeof(C);
  constexpr int NS = 2;
  __shared__ C xs[WX];
  const int lane = threadIdx.x;
  const int64_t it = blockIdx.x;
  if (it >= nitems) return;
  const WItem U = items[it];
  const int ra = U.ra, rb = U.rb, c = U.c, Rt = ra + rb;
  const int wr = Rt <= 32 ? Rt : U.wr;
  const int r0 = Rt <= 32 ? 0 : U.off;
  const int r1 = r0 + wr < Rt ? r0 + wr : Rt;        // window [r0, r1) of the stacked rows
  // the window's rows of child a, [a0, a1), and of child b, [b0, b1) (local)
  const int a0 = r0 < ra ? r0 : ra, a1 = r1 < ra ? r1 : ra;
  const int b0 = (r0 > ra ? r0 : ra) - ra, b1 = r1 > ra ? r1 - ra : 0;
  const int npa = (a1 - a0 + 1) >> 1, npb = (b1 - b0 + 1) >> 1, P = npa + npb;
  const int G = 64 / P;
  const int pr = lane % P, grp = lane / P;
  const bool isb = pr >= npa;
  const int i = isb ? b0 + 2 * (pr - npa) : a0 + 2 * pr;   // first row, local to the child
  const int iend = isb ? b1 : a1;
  const bool act = grp < G;
  const bool two = i + 1 < iend;                     // the pair's second row is in the window
  const int rc = isb ? rb : ra;
  const int t = c - rc;
  const int ob = isb ? c : 0;
  const int j0 = ob + rc + grp;
  const uint16_t *ia = fidx + U.ioff;
  const uint32_t *ia32 = (const uint32_t *)ia;
  const C *zin = z + U.zin;
  const C *T = F + U.foff + (isb ? (int64_t)ra * (c - ra) : 0) + i + (int64_t)grp * rc;
  const int64_t step = (int64_t)G * rc;
  const int nt = act && t > grp ? (t - grp + G - 1) / G : 0;
  F4 mv[B];
  auto issue = [&](int q0) {
#pragma unroll
    for (int u = 0; u < B; ++u)
      mv[u] = q0 + u < nt ? *(const F4 *)(T + (int64_t)(q0 + u) * step) : F4{0, 0, 0, 0};
  };
  auto dot = [&](auto xat, C &acc0, C &acc1) {
    acc0 = C{0, 0};
    acc1 = C{0, 0};
    for (int q0 = 0; q0 < nt; q0 += B) {
      if (q0 > 0) issue(q0);
#pragma unroll
      for (int u = 0; u < B; ++u) {
        const int q = q0 + u < nt ? q0 + u : nt - 1;   // padding entries are zero
        const C x = xat(q);
        cfma(acc0, C{mv[u][0], mv[u][1]}, x);
        cfma(acc1, C{mv[u][2], mv[u][3]}, x);
      }
    }
  };
  const int cw = (4 * c + (int)sizeof(C) - 1) / (int)sizeof(C);
  C acc0, acc1, x0, x1;
  const int i1 = two ? i + 1 : i;
  if (c + cw <= cap_lds) {
    C *xw = xs;
    uint32_t *iw32 = (uint32_t *)(xw + c);
    const uint16_t *iw = (const uint16_t *)iw32;
    C xr[NS];
    uint32_t ir[NS];
#pragma unroll
    for (int u = 0; u < NS; ++u) {
      const int k = lane + 64 * u;
      xr[u] = k < c ? zin[k] : C{0, 0};
      ir[u] = k < c ? ia32[k] : 0u;
    }
    issue(0);
    for (int k = 64 * NS + lane; k < c; k += 64) { xw[k] = zin[k]; iw32[k] = ia32[k]; }
#pragma unroll
    for (int u = 0; u < NS; ++u) {
      const int k = lane + 64 * u;
      if (k < c) { xw[k] = xr[u]; iw32[k] = ir[u]; }
    }
    wave_lds_sync();
    dot([&](int q) { return xw[iw[j0 + q * G]]; }, acc0, acc1);
    x0 = xw[iw[ob + (act ? i : 0)]];
    x1 = xw[iw[ob + (act ? i1 : 0)]];
  } else {
    issue(0);
    dot([&](int q) { return zin[ia[j0 + q * G]]; }, acc0, acc1);
    x0 = zin[ia[ob + (act ? i : 0)]];
    x1 = zin[ia[ob + (act ? i1 : 0)]];
  }
  acc0 = group_sum(acc0, lane, P, G);
  acc1 = group_sum(acc1, lane, P, G);
  if (act && grp == 0) {
    C *zo = isb ? z + U.zoutb : z + U.zouta;
    zo[i] = C{acc0.x + x0.x, acc0.y + x0.y};
    if (two) zo[i + 1] = C{acc1.x + x1.x, acc1.y + x1.y};
  }
}

// One workgroup (4 waves) per row leaf: wave w accumulates the K^L blocks
// of levels l = w, w + 4, ... (wave 0 also the dense block); the four
// partial results are added in a fixed order.
template <typename R>
__global__ __launch_bounds__(256) void k_final(const cplx_t<R> *s,
                                               const LeafInfo *leaves,
                                               const int32_t *perm,
                                               const KDesc *kd, int Lv,
                                               const cplx_t<R> *F,
                                               const cplx_t<R> *z,
                                               cplx_t<R> *u, R hd) {
  using C = cplx_t<R>;
  __shared__ C xs[HBI_MAX_LEAF];
  __shared__ C part[4][HBI_MAX_LEAF];
  const int g = blockIdx.x;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const LeafInfo lf = leaves[g];
  const int sz = lf.size;
  if (threadIdx.x < sz) {
    const C v = s[perm[lf.start + threadIdx.x]];
    xs[threadIdx.x] = C{v.x * hd, v.y * hd};
  }
  __syncthreads();
  C acc{0, 0};
  if (lane < sz) {
    if (wave == 0) {
      const C *Dm = F + lf.dense_off + lane;
      batched_dot<LoadBatch<C>::value, false>(
          acc, sz, [&](int col) { return ldf(Dm + (int64_t)col * sz); }, [&](int col) { return xs[col]; });
    }
    for (int l = wave; l < Lv; l += 4) {
      const KDesc d = kd[(int64_t)g * Lv + l];
      const C *K = F + d.foff + lane;
      const C *zz = z + d.zin;
      batched_dot<LoadBatch<C>::value, false>(
          acc, d.r, [&](int q) { return ldf(K + (int64_t)q * sz); }, [&](int q) { return zz[q]; });
    }
  }
  part[wave][lane] = acc;
  __syncthreads();
  if (threadIdx.x < sz) {
    C t = part[0][threadIdx.x];
    for (int w = 1; w < 4; ++w) { t.x += part[w][threadIdx.x].x; t.y += part[w][threadIdx.x].y; }
    u[perm[lf.start + threadIdx.x]] = t;
  }
}

// ---------------------------------------------------------------------------
// Adjoint: the same factors read as conjugate transposes, stages reversed.
// Every product is a set of conjugate dot products down contiguous columns
// of a column-major block.  A wave takes four columns at a time: slot
// g = lane / 16 one column, lane r16 = lane % 16 of the slot the rows r16,
// r16 + 16, ..., so each load instruction reads four contiguous column
// segments; the 16 partial sums of a slot are added by DPP row shifts (a
// fixed order), leaving the column's result in the slot's lane 15.
// ---------------------------------------------------------------------------
template <int CTRL> __device__ __forceinline__ float dpp_row(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xf, 0xf, true));
}
template <int CTRL> __device__ __forceinline__ double dpp_row(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, 0xf, 0xf, true);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xf, 0xf, true);
  return __longlong_as_double(((long long)(unsigned)lo) | ((long long)hi << 32));
}
// Sum over each row of 16 lanes, complete in the row's lane 15 (row_shr 1,
// 2, 4, 8 with zero fill: a prefix sum within the row).
template <typename C> __device__ __forceinline__ C row16_sum(C v) {
  v.x += dpp_row<0x111>(v.x); v.y += dpp_row<0x111>(v.y);
  v.x += dpp_row<0x112>(v.x); v.y += dpp_row<0x112>(v.y);
  v.x += dpp_row<0x114>(v.x); v.y += dpp_row<0x114>(v.y);
  v.x += dpp_row<0x118>(v.x); v.y += dpp_row<0x118>(v.y);
  return v;
}

// This lane's share of sum_{i < R} conj(col[i]) w[i]: rows r16, r16 + 16,
// ...; the first four of them use wr[0..3] (w at those rows, loaded once by
// the caller), later ones read w.  Loads issued four at a time, predicated.
template <bool NTL = true, typename C>
__device__ __forceinline__ C col_share(const C *col, int R, int r16, const C (&wr)[4],
                                       const C *w) {
  C acc{0, 0};
  {
    C mv[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) mv[u] = r16 + 16 * u < R ? ldx<NTL>(col + r16 + 16 * u) : C{0, 0};
#pragma unroll
    for (int u = 0; u < 4; ++u) cfmac(acc, mv[u], wr[u]);
  }
  for (int k0 = r16 + 64; k0 < R; k0 += 64) {
    C mv[4], wv[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int i = k0 + 16 * u;
      mv[u] = i < R ? ldx<NTL>(col + i) : C{0, 0};
      wv[u] = i < R ? w[i] : C{0, 0};
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) cfmac(acc, mv[u], wv[u]);
  }
  return acc;
}
// w at this lane's first four rows (zero past R)
template <typename C>
__device__ __forceinline__ void load_w4(C (&wr)[4], const C *w, int R, int r16) {
#pragma unroll
  for (int u = 0; u < 4; ++u) wr[u] = r16 + 16 * u < R ? w[r16 + 16 * u] : C{0, 0};
}

// K^L part: z_l = (K^L_l)^H y_leaf for every level of a row leaf (one
// workgroup; wave w takes levels w, w + 4, ...); K^L_l is sz x r, column q
// contiguous.
template <typename R>
__global__ __launch_bounds__(256) void k_final_adj(const cplx_t<R> *y,
                                                   const LeafInfo *leaves,
                                                   const int32_t *perm,
                                                   const KDesc *kd, int Lv,
                                                   const cplx_t<R> *F,
                                                   cplx_t<R> *z) {
  using C = cplx_t<R>;
  __shared__ C ys[HBI_MAX_LEAF];
  const int g = blockIdx.x;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const int slot = lane >> 4, r16 = lane & 15;
  const LeafInfo lf = leaves[g];
  const int sz = lf.size;
  if (threadIdx.x < sz) ys[threadIdx.x] = y[perm[lf.start + threadIdx.x]];
  __syncthreads();
  C yr[4];
  load_w4(yr, ys, sz, r16);
  for (int l = wave; l < Lv; l += 4) {
    const KDesc d = kd[(int64_t)g * Lv + l];
    // eight columns per pass, two column groups in flight
    for (int q0 = 0; q0 < d.r; q0 += 8) {
      const int q1 = q0 + slot, q2 = q0 + 4 + slot;
      const C *K = F + d.foff;
      constexpr bool nt = PlainF32<R>::nt;
      C a1 = col_share<nt>(K + (int64_t)(q1 < d.r ? q1 : d.r - 1) * sz, sz, r16, yr, ys);
      C a2 = col_share<nt>(K + (int64_t)(q2 < d.r ? q2 : d.r - 1) * sz, sz, r16, yr, ys);
      a1 = row16_sum(a1);
      a2 = row16_sum(a2);
      if (r16 == 15 && q1 < d.r) z[d.zin + q1] = a1;
      if (r16 == 15 && q2 < d.r) z[d.zin + q2] = a2;
    }
  }
}

// Passes of the two adjoint kernels below for blocks of at most 16 U rows:
// U rows per lane and NT groups of four columns per pass (4 NT columns),
// all their loads in flight before the sums.  col(t) is the slot's column
// position in group t (its T column is pos - r when pos >= r).
template <int U, int NT, typename C, typename POS>
__device__ __forceinline__ void adj_pass(const C *T, int r, int r16, const C (&wr)[4], POS pos,
                                         C (&out)[NT]) {
  int pp[NT];
  C tv[NT][U];
#pragma unroll
  for (int t = 0; t < NT; ++t) pp[t] = pos(t);
#pragma unroll
  for (int t = 0; t < NT; ++t)
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int i = r16 + 16 * u;
      tv[t][u] = pp[t] >= r && i < r ? ldf(T + (int64_t)(pp[t] - r) * r + i) : C{0, 0};
    }
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    C acc{0, 0};
#pragma unroll
    for (int u = 0; u < U; ++u) cfmac(acc, tv[t][u], wr[u]);
    out[t] = row16_sum(acc);
  }
}

// Adjoint of a transfer unit for the inputs j of the window [off, off + 64):
// column j of X_a is e_k when pa[j] = k < ra, and column pa[j] - ra of T_a
// otherwise (ra contiguous entries), so (X_a^H w_a)_j is w_a[k] or a
// conjugate dot product with that column; child b adds the same way.  Four
// inputs at a time, one per slot; the results gather in the wave's LDS
// slice and are stored together.  One wave per workgroup (3 % faster than
// four).
template <typename R>
__global__ __launch_bounds__(64) void k_wstage_adj(const WItem *items, int64_t nitems,
                                                   const uint16_t *fidx, const cplx_t<R> *F,
                                                   cplx_t<R> *z) {
  using C = cplx_t<R>;
  __shared__ C res[64];
  const int lane = threadIdx.x;
  const int slot = lane >> 4, r16 = lane & 15;
  const int64_t it = blockIdx.x;
  if (it >= nitems) return;
  const WItem U = items[it];
  const int ra = U.ra, rb = U.rb, c = U.c;
  const uint16_t *pa = fidx + U.ioff + 2 * (int64_t)c, *pb = pa + c;
  const C *wa = z + U.zouta, *wb = z + U.zoutb;
  const C *Ta = F + U.foff, *Tb = Ta + (int64_t)ra * (c - ra);
  const int nw = c - U.off < 64 ? c - U.off : 64;   // inputs of this window
  // the window's inverse orders, one input per lane
  const int jl = U.off + (lane < nw ? lane : 0);
  const int ka_l = pa[jl], kb_l = pb[jl];
  C war[4], wbr[4];
  load_w4(war, wa, ra, r16);
  load_w4(wbr, wb, rb, r16);
  // blocks of at most 32 rows: two rows per lane, 16 inputs per pass with
  // all their column loads in flight (one row per lane and 32 inputs per
  // pass measured slower: twice the registers, half the waves)
  auto fast = [&](auto Uc) {
    constexpr int Uv = decltype(Uc)::value, NT = 4;
    for (int q0 = 0; q0 < nw; q0 += 4 * NT) {
      int ka[NT], kb[NT];
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        const int jw = q0 + 4 * t + slot < nw ? q0 + 4 * t + slot : nw - 1;
        ka[t] = __shfl(ka_l, jw, 64);
        kb[t] = __shfl(kb_l, jw, 64);
      }
      C sa[NT], sb[NT];
      adj_pass<Uv, NT>(Ta, ra, r16, war, [&](int t) { return ka[t]; }, sa);
      adj_pass<Uv, NT>(Tb, rb, r16, wbr, [&](int t) { return kb[t]; }, sb);
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        const int q = q0 + 4 * t + slot;
        if (r16 == 15 && q < nw) {
          const C xa = ka[t] < ra ? wa[ka[t]] : sa[t];
          const C xb = kb[t] < rb ? wb[kb[t]] : sb[t];
          res[q] = C{xa.x + xb.x, xa.y + xb.y};
        }
      }
    }
    wave_lds_sync();
    if (lane < nw) z[U.zin + U.off + lane] = res[lane];
  };
  if (ra <= 32 && rb <= 32) return fast(std::integral_constant<int, 2>());
  for (int q0 = 0; q0 < nw; q0 += 4) {
    const int jw = q0 + slot < nw ? q0 + slot : nw - 1;   // window position of this slot
    const int ka = __shfl(ka_l, jw, 64), kb = __shfl(kb_l, jw, 64);
    // a skeleton column has no T column: zero rows, no loads (T may be empty)
    C acc = col_share(Ta + (int64_t)(ka >= ra ? ka - ra : 0) * ra, ka >= ra ? ra : 0, r16, war,
                      wa);
    C accb = col_share(Tb + (int64_t)(kb >= rb ? kb - rb : 0) * rb, kb >= rb ? rb : 0, r16, wbr,
                       wb);
    acc = row16_sum(acc);
    accb = row16_sum(accb);
    if (r16 == 15 && q0 + slot < nw) {
      const C xa = ka < ra ? wa[ka] : acc;
      const C xb = kb < rb ? wb[kb] : accb;
      res[q0 + slot] = C{xa.x + xb.x, xa.y + xb.y};
    }
  }
  wave_lds_sync();
  if (lane < nw) z[U.zin + U.off + lane] = res[lane];
}

// Leaf part of the adjoint: u_leaf = hd (D^H y_leaf + sum_l V_l^H z_l), one
// workgroup per leaf: wave 0 the dense block (column-major sz x sz), wave w
// the levels w, w + 4, ...; column j of V_l = [I, T] Pi^T is e_p when the
// cell's position p < r, else column p - r of T (r contiguous entries).
// Per-wave sums in LDS, added over the waves in a fixed order.
template <typename R>
__global__ __launch_bounds__(256) void k_vstage_adj(const cplx_t<R> *y,
                                                    const LeafInfo *leaves,
                                                    const int32_t *perm,
                                                    const VDesc *vd, int Lv,
                                                    const uint16_t *fidx,
                                                    const cplx_t<R> *F,
                                                    const cplx_t<R> *z,
                                                    cplx_t<R> *u, R hd) {
  using C = cplx_t<R>;
  __shared__ C ys[HBI_MAX_LEAF];
  __shared__ C part[4][HBI_MAX_LEAF];
  const int g = blockIdx.x;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const int slot = lane >> 4, r16 = lane & 15;
  const LeafInfo lf = leaves[g];
  const int sz = lf.size;
  if (threadIdx.x < sz) ys[threadIdx.x] = y[perm[lf.start + threadIdx.x]];
  part[wave][lane] = C{0, 0};
  __syncthreads();
  if (wave == 0) {
    // dense leaf: (D^H y)[col], column col of D contiguous
    C yr[4];
    load_w4(yr, ys, sz, r16);
    for (int q0 = 0; q0 < sz; q0 += 8) {
      const int q1 = q0 + slot, q2 = q0 + 4 + slot;
      C a1 = col_share(F + lf.dense_off + (int64_t)(q1 < sz ? q1 : sz - 1) * sz, sz, r16, yr, ys);
      C a2 = col_share(F + lf.dense_off + (int64_t)(q2 < sz ? q2 : sz - 1) * sz, sz, r16, yr, ys);
      a1 = row16_sum(a1);
      a2 = row16_sum(a2);
      if (r16 == 15 && q1 < sz) part[0][q1] = a1;
      if (r16 == 15 && q2 < sz) part[0][q2] = a2;
    }
  }
  for (int l = wave; l < Lv; l += 4) {
    const VDesc d = vd[(int64_t)g * Lv + l];
    const C *w = z + d.zout;
    const int p_l = fidx[d.ioff + sz + (lane < sz ? lane : 0)];   // position of cell `lane`
    C wr[4];
    load_w4(wr, w, d.r, r16);
    // blocks of at most 32 rows: two rows per lane, 16 cells per pass with
    // all their column loads in flight
    auto fast = [&](auto Uc) {
      constexpr int Uv = decltype(Uc)::value, NT = 4;
      for (int q0 = 0; q0 < sz; q0 += 4 * NT) {
        int pp[NT];
#pragma unroll
        for (int t = 0; t < NT; ++t) {
          const int jw = q0 + 4 * t + slot < sz ? q0 + 4 * t + slot : sz - 1;
          pp[t] = __shfl(p_l, jw, 64);
        }
        C sv[NT];
        adj_pass<Uv, NT>(F + d.foff, d.r, r16, wr, [&](int t) { return pp[t]; }, sv);
#pragma unroll
        for (int t = 0; t < NT; ++t) {
          const int q = q0 + 4 * t + slot;
          if (r16 == 15 && q < sz) {
            const C x = pp[t] < d.r ? w[pp[t]] : sv[t];
            C &tt = part[wave][q];
            tt.x += x.x;
            tt.y += x.y;
          }
        }
      }
    };
    if (d.r <= 32) { fast(std::integral_constant<int, 2>()); continue; }
    for (int q0 = 0; q0 < sz; q0 += 4) {
      const int jw = q0 + slot < sz ? q0 + slot : sz - 1;
      const int p = __shfl(p_l, jw, 64);
      // a skeleton cell has no T column: zero rows, no loads (T may be empty)
      C acc = col_share(F + d.foff + (int64_t)(p >= d.r ? p - d.r : 0) * d.r, p >= d.r ? d.r : 0,
                        r16, wr, w);
      acc = row16_sum(acc);
      if (r16 == 15 && q0 + slot < sz) {
        const C x = p < d.r ? w[p] : acc;
        C &t = part[wave][q0 + slot];
        t.x += x.x;
        t.y += x.y;
      }
    }
  }
  __syncthreads();
  if (threadIdx.x < sz) {
    C t = part[0][threadIdx.x];
    for (int w = 1; w < 4; ++w) { t.x += part[w][threadIdx.x].x; t.y += part[w][threadIdx.x].y; }
    u[perm[lf.start + threadIdx.x]] = C{t.x * hd, t.y * hd};
  }
}

template <typename R>
hipError_t launch_apply(const ApplyPlan &ap, const void *s, void *u, void *z,
                        const void *F, R hd, bool adjoint, hipStream_t st, LaunchHook *hook) {
  using C = cplx_t<R>;
  const C *sc = (const C *)s;
  C *uc = (C *)u;
  C *zc = (C *)z;
  const C *Fc = (const C *)F;
  const double esz = sizeof(C);
  auto pre = [&](const char *name, double elems, double idx) {
    if (hook) hook->before(name, elems * esz + idx);
  };
  auto post = [&]() { if (hook) hook->after(); };
  // factor loads per batch of the FP64 transfer stage (64 VGPRs: 8 waves/SIMD)
  constexpr int WB = 4;
  if (ap.Lv > 4 * kVq) return hipErrorInvalidValue;   // N_v < 2^31 keeps L_v <= 25
  if (!adjoint) {
    if (ap.Lv > 0) {
      pre("k_vstage", ap.v_elems, ap.v_idx);
      hipLaunchKernelGGL((k_vstage<R>), dim3(ap.nleaf), dim3(256), 0, st, sc, ap.leaves,
                         ap.perm, ap.vd, ap.Lv, ap.fidx, Fc, zc, hd);
      post();
    }
    for (int k = 1; k <= ap.Lmax; ++k) {
      const int64_t nu = ap.nunits[k];
      if (nu == 0) continue;
      const int64_t ni = ap.nitems[k];
      pre(sizeof(R) == 4 ? "k_wstage_pair" : "k_wstage", ap.w_elems[k], ap.w_idx[k]);
      // FP32: rows in pairs, one 16-byte factor load per pair and column
      if constexpr (sizeof(R) == 4)
        hipLaunchKernelGGL((k_wstage_pair<4>), dim3(ni), dim3(64), 0, st, ap.items[k], ni,
                           ap.fidx, Fc, zc, ap.cap_lds);
      else
        hipLaunchKernelGGL((k_wstage<R, WB>), dim3(ni), dim3(64), 0, st, ap.items[k],
                           ni, ap.fidx, Fc, zc, ap.cap_lds);
      post();
    }
    pre("k_final", ap.f_elems, ap.f_idx);
    hipLaunchKernelGGL((k_final<R>), dim3(ap.nleaf), dim3(256), 0, st, sc, ap.leaves,
                       ap.perm, ap.kd, ap.Lv, Fc, (const C *)zc, uc, hd);
    post();
  } else {
    // the adjoint streams the same factors; its K^L part is the K^L share of
    // the final stage and its dense part rides with the V^H stage
    if (ap.Lv > 0) {
      pre("k_final_adj", ap.f_elems, ap.f_idx);
      hipLaunchKernelGGL((k_final_adj<R>), dim3(ap.nleaf), dim3(256), 0, st, sc, ap.leaves,
                         ap.perm, ap.kd, ap.Lv, Fc, zc);
      post();
    }
    for (int k = ap.Lmax; k >= 1; --k) {
      const int64_t nu = ap.nunits[k];
      if (nu == 0) continue;
      const int64_t ni = ap.nitems_adj[k];
      pre("k_wstage_adj", ap.w_elems[k], ap.w_idx[k]);
      hipLaunchKernelGGL((k_wstage_adj<R>), dim3(ni), dim3(64), 0, st,
                         ap.items_adj[k], ni, ap.fidx, Fc, zc);
      post();
    }
    pre("k_vstage_adj", ap.v_elems, ap.v_idx);
    hipLaunchKernelGGL((k_vstage_adj<R>), dim3(ap.nleaf), dim3(256), 0, st, sc, ap.leaves,
                       ap.perm, ap.vd, ap.Lv, ap.fidx, Fc, (const C *)zc, uc, hd);
    post();
  }
  return hipGetLastError();
}

template hipError_t launch_apply<double>(const ApplyPlan &, const void *, void *, void *,
                                         const void *, double, bool, hipStream_t, LaunchHook *);
template hipError_t launch_apply<float>(const ApplyPlan &, const void *, void *, void *,
                                        const void *, float, bool, hipStream_t, LaunchHook *);

}  // namespace hbi
