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

// One lane's share of a row of a column-major factor block: entries
// T[0], T[step], ... (nt of them), streamed B at a time.  issue(q0) loads
// entries q0 .. q0 + B - 1 (zero past nt), so the first batch can be issued
// before the lane's inputs are ready.
template <typename C, int B> struct RowStream {
  const C *T;
  int64_t step;
  int nt;
  C mv[B];
  __device__ __forceinline__ void issue(int q0) {
#pragma unroll
    for (int u = 0; u < B; ++u) mv[u] = q0 + u < nt ? ldf(T + (int64_t)(q0 + u) * step) : C{0, 0};
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

// Forward transfer stage.  Row i of child a of a unit is
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
// (twice the output writes, scattered: slower).
template <typename R, int B>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(8, 8))) void k_wstage(
    const WItem *items, int64_t nitems, const uint16_t *fidx, const cplx_t<R> *F,
    cplx_t<R> *z, int cap_lds) {
  using C = cplx_t<R>;
  constexpr int WX = HBI_WSTAGE_LDS_BYTES / (int)sizeof(C);   // LDS entries per wave
  constexpr int NS = 2;   // staging loads per lane issued before T
  __shared__ C xs[4][WX];
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const int64_t it = (int64_t)blockIdx.x * 4 + wave;
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
  RowStream<C, B> S;
  S.T = F + U.foff + (isb ? (int64_t)ra * (c - ra) : 0) + i + (int64_t)grp * rc;
  S.step = (int64_t)G * rc;
  S.nt = act && t > grp ? (t - grp + G - 1) / G : 0;
  const int cw = (4 * c + (int)sizeof(C) - 1) / (int)sizeof(C);   // entries the orders take
  C acc, x0;
  if (c + cw <= cap_lds) {
    C *xw = xs[wave];
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
  // factor loads per batch of the transfer stages (64 VGPRs: 8 waves/SIMD)
  constexpr int WB = sizeof(R) == 4 ? 8 : 4;
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
      hipLaunchKernelGGL((k_wstage<R, WB>), dim3((ni + 3) / 4), dim3(256), 0, st, ap.items[k],
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
