// HIP kernels of the butterfly apply for gfx950 (wave64), one right-hand
// side at a time.
//
//   bf_apply  k_vstage, k_wstage, k_final             (u = K h^d s)
//   adjoint   k_final_adj, k_wstage_adj, k_vstage_adj  (u = h^d K^H s)
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
// l = w, w + 4, ... of the leaf.  Each block is V = [I, T] Pi^T: the leaf's
// inputs are permuted into the block's column order in the wave's LDS slice,
// then row k is xp[k] + sum_m T[k, m] xp[r + m].
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
  if (threadIdx.x < sz) {
    const C v = s[perm[lf.start + threadIdx.x]];
    xs[threadIdx.x] = C{v.x * hd, v.y * hd};
  }
  __syncthreads();
  C *xw = xp[wave];
  for (int l = wave; l < Lv; l += 4) {
    const VDesc d = vd[(int64_t)g * Lv + l];
    wave_lds_sync();   // the previous block's reads of xw are done
    if (lane < sz) xw[lane] = xs[fidx[d.ioff + lane]];
    wave_lds_sync();
    C *zo = z + d.zout;
    const int r = d.r;
    wave_gemv<C>(F + d.foff, r, sz - r, lane, [&](int col) { return xw[r + col]; },
                 [&](int row, C v) { zo[row] = C{v.x + xw[row].x, v.y + xw[row].y}; });
  }
}

// Rows [off, off + wr) of a compact transfer unit (all rows when it has at
// most 32): row i of child a is X[i] + sum_m T_a[i, m] X[ra + m] with
// X = xv + xoff the inputs in a's column order (xoff = 0), likewise for b
// (xoff = c).  Per lane: T column stride rc, column count t, and the columns
// grp, grp + G, ... when G = 64 / wr > 1 lanes share a row.
template <typename C> struct RowLane {
  const C *T;        // the lane's first factor entry
  int64_t tstep;     // between its successive entries
  int nt, grp, G, wr, i, xo;
  bool act, isb;
};
template <typename C>
__device__ __forceinline__ RowLane<C> row_lane(const WItem &U, const C *__restrict__ Ta, int lane) {
  RowLane<C> L;
  const int ra = U.ra, rb = U.rb, c = U.c, Rt = ra + rb;
  L.wr = Rt <= 32 ? Rt : U.wr;   // rows of the window
  L.G = 64 / L.wr;
  const int row = (Rt <= 32 ? 0 : U.off) + lane % L.wr;
  L.grp = lane / L.wr;
  L.isb = row >= ra;
  L.i = L.isb ? row - ra : row;
  const int rc = L.isb ? rb : ra;
  L.xo = (L.isb ? c : 0) + rc;
  L.T = (L.isb ? Ta + (int64_t)ra * (c - ra) : Ta) + L.i + (int64_t)L.grp * rc;
  L.tstep = (int64_t)L.G * rc;
  L.act = row < Rt && L.grp < L.G;
  const int t = c - rc;
  L.nt = L.act && t > L.grp ? (t - L.grp + L.G - 1) / L.G : 0;
  return L;
}
template <typename C, int B, typename XF>
__device__ __forceinline__ void wstage_rows(const WItem &U, const RowLane<C> &L, int lane, XF xv,
                                            C *z) {
  const int nt = L.nt, G = L.G, grp = L.grp, xo = L.xo;
  C acc{0, 0};
  for (int q0 = 0; q0 < nt; q0 += B) {
    C mv[B], xq[B];
#pragma unroll
    for (int u = 0; u < B; ++u) {
      if (q0 + u < nt) {
        mv[u] = ldf(L.T + (q0 + u) * L.tstep);
        xq[u] = xv(xo + grp + (q0 + u) * G);
      } else {
        mv[u] = C{0, 0};
        xq[u] = C{0, 0};
      }
    }
#pragma unroll
    for (int u = 0; u < B; ++u) cfma(acc, mv[u], xq[u]);
  }
  if (G > 1) {
    // combine the G partial sums of each row (lanes row, row+Rt, ...)
    C tot = acc;
    for (int g = 1; g < G; ++g) {
      const int src = lane + g * L.wr;
      const auto re = __shfl(acc.x, src < 64 ? src : lane, 64);
      const auto im = __shfl(acc.y, src < 64 ? src : lane, 64);
      if (src < 64) { tot.x += re; tot.y += im; }
    }
    acc = tot;
  }
  if (L.act && grp == 0) {
    const C x0 = xv((L.isb ? U.c : 0) + L.i);
    (L.isb ? z + U.zoutb : z + U.zouta)[L.i] = C{acc.x + x0.x, acc.y + x0.y};
  }
}

// xw[0, c) = zin[0, c) and iw[0, 2c) = io[0, 2c) for c <= 64 NX and
// 2c <= 64 NI: every load is issued before the first LDS store, so the
// wave waits on one round trip (a plain strided copy loop waits on each).
template <int NX, int NI, typename C>
__device__ __forceinline__ void stage_raw(C *xw, uint16_t *iw, const C *zin, const uint16_t *io,
                                          int c, int lane) {
  C xr[NX];
  uint16_t ir[NI];
#pragma unroll
  for (int u = 0; u < NX; ++u) {
    const int k = lane + 64 * u;
    xr[u] = k < c ? zin[k] : C{0, 0};
  }
#pragma unroll
  for (int u = 0; u < NI; ++u) {
    const int k = lane + 64 * u;
    ir[u] = k < 2 * c ? io[k] : uint16_t(0);
  }
#pragma unroll
  for (int u = 0; u < NX; ++u)
    if (lane + 64 * u < c) xw[lane + 64 * u] = xr[u];
#pragma unroll
  for (int u = 0; u < NI; ++u)
    if (lane + 64 * u < 2 * c) iw[lane + 64 * u] = ir[u];
}

// One wave per work item: rows [r0, r0 + 64) of a transfer unit, the pair
// stacked a then b (the whole unit when it has <= 64 rows).  Items are
// ordered by decreasing cost, and the factor store holds the units in that
// order.  Row i of child a is x[ia[i]] + sum_m T_a[i, m] x[ia[ra + m]]
// (X = [I, T] Pi^T), likewise for b with its own column order ib.  Both
// gathered inputs are staged in the wave's own LDS slice when 2c <= WX, so
// the streamed T blocks are the only vector-memory traffic of the loop; the
// waves of a workgroup do not wait for each other.  Lanes are (row, column
// group) for units of at most 32 rows and rows otherwise, as in wave_gemv.
// (A persistent variant, each wave looping over items, measured slower.)
template <typename R>
__global__ __launch_bounds__(256) void k_wstage(const WItem *items, int64_t nitems,
                                                const uint16_t *fidx, const cplx_t<R> *F,
                                                cplx_t<R> *z) {
  using C = cplx_t<R>;
  constexpr int WX = 512;   // LDS entries per wave: both permuted inputs, c <= WX / 2
  __shared__ C xs[4][WX];
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const int64_t it = (int64_t)blockIdx.x * 4 + wave;
  if (it >= nitems) return;
  const WItem U = items[it];
  const int c = U.c;
  const uint16_t *ia = fidx + U.ioff;   // ia, then ib at ia + c
  const C *zin = z + U.zin;
  const bool lds = 2 * c <= WX;
  C *xw = xs[wave];
  const RowLane<C> L = row_lane(U, F + U.foff, lane);
  if (lds) {
    // the inputs in their own order and both column orders (three
    // independent contiguous loads), then the two gathers within LDS:
    // xw[0, c) = x[ia], xw[c, 2c) = x[ib]
    uint16_t *iw = (uint16_t *)(xw + c);
    stage_raw<WX / 128, WX / 64>(xw, iw, zin, ia, c, lane);
    wave_lds_sync();
    R ar[WX / 128], ai[WX / 128], br[WX / 128], bi[WX / 128];
#pragma unroll
    for (int u = 0; u < WX / 128; ++u) {
      const int k = lane + 64 * u < c ? lane + 64 * u : 0;
      const C va = xw[iw[k]], vb = xw[iw[c + k]];
      ar[u] = va.x; ai[u] = va.y;
      br[u] = vb.x; bi[u] = vb.y;
    }
    wave_lds_sync();
#pragma unroll
    for (int u = 0; u < WX / 128; ++u) {
      const int k = lane + 64 * u;
      if (k < c) {
        xw[k] = C{ar[u], ai[u]};
        xw[c + k] = C{br[u], bi[u]};
      }
    }
    wave_lds_sync();
    // 8 loads in flight (FP32) or 4 (FP64) keep the registers within 8 (6)
    // waves per SIMD
    wstage_rows<C, sizeof(R) == 4 ? 8 : 4>(U, L, lane, [&](int k) { return xw[k]; }, z);
    return;
  }
  // wider units whose raw inputs and both column orders still fit the slice
  constexpr int CM = WX * (int)sizeof(C) / (int)(sizeof(C) + 2 * sizeof(uint16_t));
  if (c <= CM) {
    // gathers through the column orders, both in LDS
    uint16_t *iw = (uint16_t *)(xw + c);
    stage_raw<(CM + 63) / 64, (2 * CM + 63) / 64>(xw, iw, zin, ia, c, lane);
    wave_lds_sync();
    wstage_rows<C, 4>(U, L, lane, [&](int k) { return xw[iw[k]]; }, z);
  } else {
    // the widest units: inputs gathered from global memory
    wstage_rows<C, 4>(U, L, lane, [&](int k) { return zin[ia[k]]; }, z);
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
// ---------------------------------------------------------------------------
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
  const LeafInfo lf = leaves[g];
  const int sz = lf.size;
  if (threadIdx.x < sz) ys[threadIdx.x] = y[perm[lf.start + threadIdx.x]];
  __syncthreads();
  for (int l = wave; l < Lv; l += 4) {
    const KDesc d = kd[(int64_t)g * Lv + l];
    if (lane < d.r) {
      const C *K = F + d.foff + (int64_t)lane * sz;
      C acc{0, 0};
      batched_dot<LoadBatch<C>::value, true>(
          acc, sz, [&](int row) { return ldf(K + row); }, [&](int row) { return ys[row]; });
      z[d.zin + lane] = acc;
    }
  }
}

// Adjoint of a transfer unit, one lane per input column j of the window
// [off, off + 64): column j of X_a is e_k when pa[j] = k < ra, and column
// pa[j] - ra of T_a otherwise, so (X_a^H w_a)_j is w_a[k] or a conjugate
// dot product with that column of T_a; child b adds the same way.
template <typename R>
__global__ __launch_bounds__(256) void k_wstage_adj(const WItem *items, int64_t nitems,
                                                    const uint16_t *fidx, const cplx_t<R> *F,
                                                    cplx_t<R> *z) {
  using C = cplx_t<R>;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const int64_t it = (int64_t)blockIdx.x * 4 + wave;
  if (it >= nitems) return;
  const WItem U = items[it];
  const int ra = U.ra, rb = U.rb, c = U.c;
  const uint16_t *pa = fidx + U.ioff + 2 * (int64_t)c, *pb = pa + c;
  const C *wa = z + U.zouta, *wb = z + U.zoutb;
  const C *Ta = F + U.foff, *Tb = Ta + (int64_t)ra * (c - ra);
  const int c1 = U.off + 64 < c ? U.off + 64 : c;
  const int col = U.off + lane;
  if (col < c1) {
    C acc{0, 0};
    const int ka = pa[col], kb = pb[col];
    if (ka < ra) {
      acc = wa[ka];
    } else {
      const C *cm = Ta + (int64_t)(ka - ra) * ra;
      batched_dot<LoadBatch<C>::value, true>(
          acc, ra, [&](int i) { return ldf(cm + i); }, [&](int i) { return wa[i]; });
    }
    if (kb < rb) {
      acc.x += wb[kb].x;
      acc.y += wb[kb].y;
    } else {
      const C *cm = Tb + (int64_t)(kb - rb) * rb;
      batched_dot<LoadBatch<C>::value, true>(
          acc, rb, [&](int i) { return ldf(cm + i); }, [&](int i) { return wb[i]; });
    }
    z[U.zin + col] = acc;
  }
}

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
  const LeafInfo lf = leaves[g];
  const int sz = lf.size;
  if (threadIdx.x < sz) ys[threadIdx.x] = y[perm[lf.start + threadIdx.x]];
  __syncthreads();
  C acc{0, 0};
  if (lane < sz) {
    if (wave == 0) {
      // dense leaf: (D^H y)[col], column `lane` of D is contiguous
      const C *Dc = F + lf.dense_off + (int64_t)lane * sz;
      batched_dot<LoadBatch<C>::value, true>(
          acc, sz, [&](int row) { return ldf(Dc + row); }, [&](int row) { return ys[row]; });
    }
    for (int l = wave; l < Lv; l += 4) {
      // column `lane` of V: e_p when p < r, else column p - r of T
      const VDesc d = vd[(int64_t)g * Lv + l];
      const C *w = z + d.zout;
      const int p = fidx[d.ioff + sz + lane];
      if (p < d.r) {
        acc.x += w[p].x;
        acc.y += w[p].y;
      } else {
        const C *V = F + d.foff + (int64_t)(p - d.r) * d.r;
        batched_dot<LoadBatch<C>::value, true>(
            acc, d.r, [&](int row) { return ldf(V + row); }, [&](int row) { return w[row]; });
      }
    }
  }
  part[wave][lane] = acc;
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
      pre("k_wstage", ap.w_elems[k], ap.w_idx[k]);
      hipLaunchKernelGGL((k_wstage<R>), dim3((ni + 3) / 4), dim3(256), 0, st,
                         ap.items[k], ni, ap.fidx, Fc, zc);
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
      hipLaunchKernelGGL((k_wstage_adj<R>), dim3((ni + 3) / 4), dim3(256), 0, st,
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
