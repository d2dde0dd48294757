// Many right-hand sides (and many problems) per launch: the factor
// products become small complex GEMMs Y = M Z, computed with 16x16x4 MFMA
// tiles (FP32: v_mfma_f32_16x16x4_f32, FP64: v_mfma_f64_16x16x4_f64).
//
// A complex GEMM step is four real MFMAs on the same operands:
//   Yr += Mr Zr - Mi Zi,   Yi += Mr Zi + Mi Zr.
// Operand layout of the 16x16x4 MFMA (one wave): lane l holds A[l%16][l/16]
// and B[l/16][l%16].  Accumulator v = 0..3 of lane l holds D[4*(l/16) + v]
// [l%16] for the FP32 instruction and D[l/16 + 4*v][l%16] for the FP64 one
// (measured on gfx950 for both builtins).
//
// Vectors are in tree order with the right-hand sides contiguous:
// element (row, j) of a block with offset zoff is z[(zoff + row) * Np + j],
// Np = nrhs rounded up to 16.  Factor blocks keep their single-RHS
// column-major layout, so every factor entry is loaded once per 16-row
// tile and reused for all Np right-hand sides.
//
// Each stage is one launch (the host replays them from a HIP graph), or all
// of them are phases of k_multi_persistent, one cooperative launch.  The
// column-tile width NB and the k-steps per load chunk are template
// parameters that the host tunes per batch.
#include <type_traits>

#include <hip/hip_cooperative_groups.h>

#include "hbi_device.h"
#include "hbi_multi.h"

namespace hbi {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef double v4d __attribute__((ext_vector_type(4)));

template <typename R> struct Mfma;
template <> struct Mfma<float> {
  using acc = v4f;
  static __device__ __forceinline__ acc zero() { return acc{0.f, 0.f, 0.f, 0.f}; }
  static __device__ __forceinline__ acc op(float a, float b, acc c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  // row of the result held by accumulator v of a lane in group g = l/16
  static __device__ __forceinline__ int row(int g, int v) { return 4 * g + v; }
};
template <> struct Mfma<double> {
  using acc = v4d;
  static __device__ __forceinline__ acc zero() { return acc{0.0, 0.0, 0.0, 0.0}; }
  static __device__ __forceinline__ acc op(double a, double b, acc c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int g, int v) { return g + 4 * v; }
};

// The descriptors carry generic pointers; loads and stores through these
// helpers use global-memory instructions (flat ones would also wait on LDS
// traffic and need a full address per lane).
template <typename T> using gptr = __attribute__((address_space(1))) T *;
template <typename C> __device__ __forceinline__ C ldg(const C *p, int64_t i) {
  using E = decltype(C{}.x);
  typedef E V __attribute__((ext_vector_type(2)));
  const V v = ((gptr<const V>)p)[i];
  return C{v[0], v[1]};
}
__device__ __forceinline__ int ldg16(const uint16_t *p, int64_t i) {
  return ((gptr<const uint16_t>)p)[i];
}
template <typename C> __device__ __forceinline__ void stg(C *p, int64_t i, C v) {
  using E = decltype(C{}.x);
  typedef E V __attribute__((ext_vector_type(2)));
  ((gptr<V>)p)[i] = V{v.x, v.y};
}

// Workspace column of lane li in column tile nb of the group [jt, jt + NB)
// (nbv tiles of it exist).  With NB >= 2 a full pair of tiles (2m, 2m + 1)
// takes the 32 columns jt*16 + 32m + [0, 32) interleaved, tile 2m the even
// ones and 2m + 1 the odd ones, so that one 16-byte load brings a lane's B
// entries of both; a pair with one tile takes its 16 columns in order.
// Every load and store of the tiles' columns goes through this map, and
// each output column is computed from the same input column, so the
// numbers do not depend on it.
template <int NB> __device__ __forceinline__ int tcol(int jt, int nb, int li, int nbv) {
  if (NB >= 2 && (nb | 1) < nbv) return jt * 16 + 32 * (nb >> 1) + 2 * li + (nb & 1);
  return (jt + nb) * 16 + li;
}
template <typename C> __device__ __forceinline__ void ldg2(const C *p, int64_t i, C &e0, C &e1) {
  using E = decltype(C{}.x);
  typedef E V __attribute__((ext_vector_type(4)));
  const V v = ((gptr<const V>)(p + i))[0];
  e0 = C{v[0], v[1]};
  e1 = C{v[2], v[3]};
}

// Accumulate a 16-row tile of M (rows r0.., column-major, leading dimension
// ldm, `rows` valid rows, `k` columns) times Z (k x Np, row stride Np),
// for column tiles [jt0, jt0 + NB) of 16 columns each.
// With `zrow` non-null, row kk of Z is zrow[kk] (a gather of the inputs).
// The A entries come from aload.value(row, aload.index(row, kk), valid)
// when an A loader is given, else M[row + kk ldm]; rows at or past ksplit
// come from Z2 (row - ksplit).
//
// The k columns go in chunks of KU MFMA k-steps (4 KU columns), software
// pipelined two deep: while the MFMAs of chunk i run, the data loads of
// chunk i + 1 (A entries and B rows) and the index loads of chunk i + 2
// (zrow, or the A loader's) are in flight, so a wave waits on memory only
// when the MFMAs cannot cover a round trip.  Loads of chunks past the end
// read clamped, valid addresses and are zeroed; so are out-of-range rows,
// columns and column tiles, whose MFMAs then add zeros (a wave-uniform
// branch around them would split the loop into blocks and let the compiler
// sink each load into the block that uses it).  An empty asm statement
// with a memory clobber after each batch of loads keeps them there.
struct NoLoad {};
__device__ __forceinline__ void load_fence() { __asm__ volatile("" ::: "memory"); }

template <typename R, int NB, int KUT = 0, typename AL = NoLoad, bool GATHER = false>
__device__ __forceinline__ void tile_gemm(const cplx_t<R> *__restrict__ M, int ldm, int r0,
                                          int rows, int k, const cplx_t<R> *__restrict__ Z,
                                          int Np, int jt0, int lane,
                                          typename Mfma<R>::acc (&ar)[NB],
                                          typename Mfma<R>::acc (&ai)[NB],
                                          const uint16_t *zrow = nullptr, AL aload = AL(),
                                          const cplx_t<R> *__restrict__ Z2 = nullptr,
                                          int ksplit = 1 << 30) {
  using C = cplx_t<R>;
  // k-steps per chunk: KUT, or by default 4 / 2 / 1 for NB = 1 / 2 / more
  constexpr int KU = KUT ? KUT : NB == 1 ? 4 : NB == 2 ? 2 : 1;
  constexpr int STEP = 4 * KU;                        // columns per chunk
  constexpr bool synth = !std::is_same<AL, NoLoad>::value;
  const int li = lane & 15, lk = lane >> 4;
  const int row = r0 + li;
  const bool rok = row < rows;
  const int zc = jt0 * 16 + li;
  // column tiles past Np (last group of a row) are never read
  const int nbv = (Np >> 4) - jt0 < NB ? (Np >> 4) - jt0 : NB;
  struct Idx { int zr[KU], pa[KU]; };
  struct Dat { C a[KU], b[KU][NB]; };
  auto load_idx = [&](int k0, Idx &I) {
#pragma unroll
    for (int u = 0; u < KU; ++u) {
      const int kk = k0 + 4 * u + lk;
      const bool kok = kk < k;
      if constexpr (GATHER) I.zr[u] = ldg16(zrow, kok ? kk : 0);
      else I.zr[u] = kk;
      if constexpr (synth) I.pa[u] = aload.index(row, (rok && kok) ? kk : 0);
    }
  };
  auto load_dat = [&](int k0, const Idx &I, Dat &D) {
#pragma unroll
    for (int u = 0; u < KU; ++u) {
      const int kk = k0 + 4 * u + lk;
      const bool kok = kk < k;
      const bool second = Z2 && kok && kk >= ksplit;
      const C *Zb = second ? Z2 : Z;
      const int zrb = second ? I.zr[u] - ksplit : I.zr[u];
      if constexpr (NB >= 2 && sizeof(R) == 4) {
        // one 16-byte load per pair of tiles (tcol's interleaved columns);
        // a pair with one tile loads the aligned pair of columns holding
        // the lane's column and keeps its half
#pragma unroll
        for (int nb = 0; nb < NB; nb += 2) {
          const bool full = nb + 1 < nbv;
          const bool ok0 = kok && nb < nbv, ok1 = kok && full;
          const int col = full ? jt0 * 16 + 16 * nb + 2 * li : (jt0 + nb) * 16 + (li & ~1);
          C e0, e1;
          ldg2(Zb, (int64_t)(ok0 ? zrb : 0) * Np + (ok0 ? col : 0), e0, e1);
          D.b[u][nb] = ok0 ? (full || !(li & 1) ? e0 : e1) : C{0, 0};
          D.b[u][nb + 1] = ok1 ? e1 : C{0, 0};
        }
      } else {
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) {
          const bool ok = kok && nb < nbv;
          const C v = ldg(Zb, (int64_t)(ok ? zrb : 0) * Np + (ok ? tcol<NB>(jt0, nb, li, nbv) : zc));
          D.b[u][nb] = ok ? v : C{0, 0};
        }
      }
      if constexpr (synth) {
        D.a[u] = aload.value(row, I.pa[u], rok && kok);
      } else {
        const C v = ldg(M, (rok && kok) ? row + (int64_t)kk * ldm : 0);
        D.a[u] = (rok && kok) ? v : C{0, 0};
      }
    }
  };
  auto mma = [&](const Dat &D) {
#pragma unroll
    for (int u = 0; u < KU; ++u) {
      const R nai = -D.a[u].y;
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) {
        ar[nb] = Mfma<R>::op(D.a[u].x, D.b[u][nb].x, ar[nb]);
        ar[nb] = Mfma<R>::op(nai, D.b[u][nb].y, ar[nb]);
        ai[nb] = Mfma<R>::op(D.a[u].x, D.b[u][nb].y, ai[nb]);
        ai[nb] = Mfma<R>::op(D.a[u].y, D.b[u][nb].x, ai[nb]);
      }
    }
  };
  // Loads complete in issue order, so the index loads of a chunk are issued
  // before the data loads of the chunk ahead of it: using the indices then
  // never waits for data loads.  One chunk per iteration (a single exit
  // keeps the accumulators in place); the buffers rotate at its end.
  Idx In, Inn;
  Dat Dc, Dn;
  load_idx(0, In);
  load_idx(STEP, Inn);
  load_dat(0, In, Dc);
  load_fence();
  for (int k0 = 0; k0 < k; k0 += STEP) {
    In = Inn;
    load_idx(k0 + 2 * STEP, Inn);
    load_dat(k0 + STEP, In, Dn);
    load_fence();
    mma(Dc);
    Dc = Dn;
  }
}

// A entries of a stacked compact unit (rows of child a, then of b, over
// all c inputs): entry (row, kk) of X = [I, T] Pi^T is 1 or 0 when the
// column's position p = pa[kk] (pb) is a skeleton, else T[i, p - r].  The
// load is issued either way, from `safe` (any valid entry) when no T entry
// is wanted, and the value selected after it, so that it needs no branch.
template <typename R> struct StackedA {
  const cplx_t<R> *Ta, *Tb, *safe;
  const uint16_t *pa, *pb;
  int ra, rb;
  __device__ __forceinline__ int index(int row, int kk) const {
    return row >= ra ? ldg16(pb, kk) : ldg16(pa, kk);
  }
  __device__ __forceinline__ cplx_t<R> value(int row, int p, bool ok) const {
    const bool isb = row >= ra;
    const int i = isb ? row - ra : row, rc = isb ? rb : ra;
    const bool t = ok && p >= rc;
    const cplx_t<R> v = ldg(t ? (isb ? Tb : Ta) + i + (int64_t)(p - rc) * rc : safe, 0);
    const R one = (ok && p == i) ? (R)1 : (R)0;
    return t ? v : cplx_t<R>{one, (R)0};
  }
};

// A entries of a conjugate transpose: A[row][kk] = conj(M[kk + row ldm]).
template <typename R> struct ConjTransA {
  const cplx_t<R> *M;
  int ldm;
  __device__ __forceinline__ int index(int, int kk) const { return kk; }
  __device__ __forceinline__ cplx_t<R> value(int row, int kk, bool ok) const {
    const cplx_t<R> v = ldg(M, ok ? kk + (int64_t)row * ldm : 0);
    return ok ? cplx_t<R>{v.x, -v.y} : cplx_t<R>{0, 0};
  }
};

// A entries of [X_a; X_b]^H for a transfer unit (rows: its c input columns,
// in their natural order; k: the ra rows of a, then the rb rows of b).  With
// p = pa[row] (the column's position in a's order), X_a[k][row] is 1 when
// p == k, T_a[k, p - ra] when p >= ra, else 0; likewise for b.  The lane's
// positions pa[row], pb[row] are loaded once, before the tile.
template <typename R> struct AdjStackedA {
  const cplx_t<R> *Ta, *Tb, *safe;
  int ra, rb, pja, pjb;
  __device__ __forceinline__ int index(int, int kk) const { return kk; }
  __device__ __forceinline__ cplx_t<R> value(int, int kk, bool ok) const {
    const bool isb = kk >= ra;
    const int k = isb ? kk - ra : kk, rc = isb ? rb : ra, p = isb ? pjb : pja;
    const bool t = ok && p >= rc;
    const cplx_t<R> v = ldg(t ? (isb ? Tb : Ta) + k + (int64_t)(p - rc) * rc : safe, 0);
    const R one = (ok && p == k) ? (R)1 : (R)0;
    return t ? cplx_t<R>{v.x, -v.y} : cplx_t<R>{one, (R)0};
  }
};

// A entries of V^H for a V^0 block V = [I, T] Pi^T (r x sz): row j of V^H
// (a cell of the leaf) has pv = the cell's position in the block's order;
// V[k][j] is 1 when pv == k, T[k, pv - r] when pv >= r, else 0.
template <typename R> struct AdjVA {
  const cplx_t<R> *T, *safe;
  int r, pj;
  __device__ __forceinline__ int index(int, int kk) const { return kk; }
  __device__ __forceinline__ cplx_t<R> value(int, int kk, bool ok) const {
    const bool t = ok && pj >= r;
    const cplx_t<R> v = ldg(t ? T + kk + (int64_t)(pj - r) * r : safe, 0);
    const R one = (ok && pj == kk) ? (R)1 : (R)0;
    return t ? cplx_t<R>{v.x, -v.y} : cplx_t<R>{one, (R)0};
  }
};

// Rows [r0, r0 + 16) of Y = X Z for X = [I, T] Pi^T with T Z_rest already
// in the accumulators: dst[row] = acc[row] + Z[idx[row]] for row < r.  The
// four row indices are loaded first, then the inputs, then the stores.
template <typename R, int NB>
__device__ __forceinline__ void add_skeleton_rows(const uint16_t *idx, int r, int r0,
                                                  const cplx_t<R> *Z, cplx_t<R> *dst, int Np,
                                                  int jt0, int nbv, int lane,
                                                  const typename Mfma<R>::acc (&ar)[NB],
                                                  const typename Mfma<R>::acc (&ai)[NB]) {
  using C = cplx_t<R>;
  const int li = lane & 15, lg = lane >> 4;
  int sr[4];
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int row = r0 + Mfma<R>::row(lg, v);
    sr[v] = ldg16(idx, row < r ? row : 0);   // idx[0] exists: r >= 1
  }
  C x0[4][NB];
#pragma unroll
  for (int v = 0; v < 4; ++v)
#pragma unroll
    for (int nb = 0; nb < NB; ++nb)
      x0[v][nb] = nb < nbv ? ldg(Z, (int64_t)sr[v] * Np + tcol<NB>(jt0, nb, li, nbv)) : C{0, 0};
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int row = r0 + Mfma<R>::row(lg, v);
    if (row >= r) continue;
#pragma unroll
    for (int nb = 0; nb < NB; ++nb)
      if (nb < nbv)
        stg(dst, (int64_t)row * Np + tcol<NB>(jt0, nb, li, nbv),
            C{ar[nb][v] + x0[v][nb].x, ai[nb][v] + x0[v][nb].y});
  }
}

// Transfer stage: one wave per (child of a unit, 16-row tile, group of NB
// column tiles).
template <typename R, int NB, int KUT = 0>
__device__ __forceinline__ void b_wstage_mr(const MWItem *items, int64_t nitems, int64_t bid) {
  using C = cplx_t<R>;
  using A = typename Mfma<R>::acc;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const int64_t it = bid * 4 + wave;
  if (it >= nitems) return;
  const MWItem W = items[it];
  if (W.Np == 0) return;   // a free slot of the XCD placement
  A ar[NB], ai[NB];
#pragma unroll
  for (int nb = 0; nb < NB; ++nb) { ar[nb] = Mfma<R>::zero(); ai[nb] = Mfma<R>::zero(); }
  const int jt0 = W.jt;
  const int nbv = (W.Np >> 4) - jt0 < NB ? (W.Np >> 4) - jt0 : NB;
  const C *Z = (const C *)W.zin;
  const int li = lane & 15, lg = lane >> 4;
  if (W.rb >= 0) {
    // a small unit as stacked 16-row tiles over all c inputs
    const int ra = W.r, rb = W.rb, c = W.c;
    StackedA<R> aload;
    aload.Ta = (const C *)W.T;
    aload.Tb = aload.Ta + (int64_t)ra * (c - ra);
    aload.safe = Z;
    aload.pa = W.idx + 2 * (int64_t)c;
    aload.pb = aload.pa + c;
    aload.ra = ra;
    aload.rb = rb;
    tile_gemm<R, NB, KUT>(aload.Ta, 0, W.r0, ra + rb, c, Z, W.Np, jt0, lane, ar, ai, nullptr, aload);
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int row = W.r0 + Mfma<R>::row(lg, v);
      if (row >= ra + rb) continue;
      C *dst = row < ra ? (C *)W.zout + (int64_t)row * W.Np
                        : (C *)W.zoutb + (int64_t)(row - ra) * W.Np;
#pragma unroll
      for (int nb = 0; nb < NB; ++nb)
        if (nb < nbv) stg(dst, tcol<NB>(jt0, nb, li, nbv), C{ar[nb][v], ai[nb][v]});
    }
    return;
  }
  // T times the non-skeleton inputs (rows idx[r..c) of Z)
  tile_gemm<R, NB, KUT, NoLoad, true>((const C *)W.T, W.r, W.r0, W.r, W.c - W.r, Z, W.Np, jt0, lane,
                                 ar, ai, W.idx + W.r);
  // plus the skeleton input of each row (the identity part of X)
  add_skeleton_rows<R, NB>(W.idx, W.r, W.r0, Z, (C *)W.zout, W.Np, jt0, nbv, lane, ar, ai);
}
template <typename R, int NB, int KUT = 0>
__global__ __launch_bounds__(256) void k_wstage_mr(const MWItem *items, int64_t nitems) {
  b_wstage_mr<R, NB, KUT>(items, nitems, blockIdx.x);
}

// V^0 stage: one wave per (leaf, level, 16-row tile, column-tile group).
template <typename R, int NB, int KUT = 0>
__device__ __forceinline__ void b_vstage_mr(const MVItem *items, int64_t nitems, int64_t bid) {
  using C = cplx_t<R>;
  using A = typename Mfma<R>::acc;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const int64_t it = bid * 4 + wave;
  if (it >= nitems) return;
  const MVItem W = items[it];
  if (W.Np == 0) return;   // a free slot of the XCD placement
  A ar[NB], ai[NB];
#pragma unroll
  for (int nb = 0; nb < NB; ++nb) { ar[nb] = Mfma<R>::zero(); ai[nb] = Mfma<R>::zero(); }
  const int nbv = (W.Np >> 4) - W.jt < NB ? (W.Np >> 4) - W.jt : NB;
  const C *X = (const C *)W.x;
  // T times the non-skeleton inputs (rows idx[r..sz) of x)
  tile_gemm<R, NB, KUT, NoLoad, true>((const C *)W.T, W.r, W.r0, W.r, W.sz - W.r, X, W.Np, W.jt,
                                 lane, ar, ai, W.idx + W.r);
  // plus the skeleton input of each row
  add_skeleton_rows<R, NB>(W.idx, W.r, W.r0, X, (C *)W.z, W.Np, W.jt, nbv, lane, ar, ai);
}
template <typename R, int NB, int KUT = 0>
__global__ __launch_bounds__(256) void k_vstage_mr(const MVItem *items, int64_t nitems) {
  b_vstage_mr<R, NB, KUT>(items, nitems, blockIdx.x);
}

// Final stage: one wave per (leaf, 16-row tile, column-tile group); the
// dense leaf block and every level's K^L accumulate into the same tiles in
// a fixed order.
template <typename R, int NB, int KUT = 0>
__device__ __forceinline__ void b_final_mr(const MFItem *items, int64_t nitems, int64_t bid) {
  using C = cplx_t<R>;
  using A = typename Mfma<R>::acc;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const int64_t it = bid * 4 + wave;
  if (it >= nitems) return;
  const MFItem W = items[it];
  if (W.Np == 0) return;   // a free slot of the XCD placement
  A ar[NB], ai[NB];
#pragma unroll
  for (int nb = 0; nb < NB; ++nb) { ar[nb] = Mfma<R>::zero(); ai[nb] = Mfma<R>::zero(); }
  const C *F = (const C *)W.F;
  const C *z = (const C *)W.z;
  const int sz = W.sz;
  tile_gemm<R, NB, KUT>(F + W.dense_off, sz, W.r0, sz, sz, (const C *)W.x, W.Np, W.jt, lane, ar, ai);
  for (int l = 0; l < W.Lv; ++l) {
    const KDesc d = W.kd[l];
    tile_gemm<R, NB, KUT>(F + d.foff, sz, W.r0, sz, d.r, z + d.zin * W.Np, W.Np, W.jt, lane, ar, ai);
  }
  const int nbv = (W.Np >> 4) - W.jt < NB ? (W.Np >> 4) - W.jt : NB;
  const int li = lane & 15, lg = lane >> 4;
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int row = W.r0 + Mfma<R>::row(lg, v);
    if (row >= sz) continue;
    C *dst = (C *)W.y + (int64_t)row * W.Np;
#pragma unroll
    for (int nb = 0; nb < NB; ++nb)
      if (nb < nbv) stg(dst, tcol<NB>(W.jt, nb, li, nbv), C{ar[nb][v], ai[nb][v]});
  }
}
template <typename R, int NB, int KUT = 0>
__global__ __launch_bounds__(256) void k_final_mr(const MFItem *items, int64_t nitems) {
  b_final_mr<R, NB, KUT>(items, nitems, blockIdx.x);
}

// Stores rows [r0, r0 + 16) (those below `rows`) of the accumulators to
// dst (row stride Np), times `scale`.
template <typename R, int NB>
__device__ __forceinline__ void store_tile(cplx_t<R> *dst, int r0, int rows, int Np, int jt,
                                           int lane, R scale,
                                           const typename Mfma<R>::acc (&ar)[NB],
                                           const typename Mfma<R>::acc (&ai)[NB]) {
  const int nbv = (Np >> 4) - jt < NB ? (Np >> 4) - jt : NB;
  const int li = lane & 15, lg = lane >> 4;
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int row = r0 + Mfma<R>::row(lg, v);
    if (row >= rows) continue;
#pragma unroll
    for (int nb = 0; nb < NB; ++nb)
      if (nb < nbv)
        stg(dst, (int64_t)row * Np + tcol<NB>(jt, nb, li, nbv),
            cplx_t<R>{ar[nb][v] * scale, ai[nb][v] * scale});
  }
}

// Adjoint, K^L part: z_l = (K^L_l)^H y_leaf for one (leaf, level, 16-row
// tile of the r skeleton rows, column-tile group).
template <typename R, int NB, int KUT = 0>
__device__ __forceinline__ void b_final_adj_mr(const MFAItem *items, int64_t nitems, int64_t bid) {
  using C = cplx_t<R>;
  using A = typename Mfma<R>::acc;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const int64_t it = bid * 4 + wave;
  if (it >= nitems) return;
  const MFAItem W = items[it];
  if (W.Np == 0) return;   // a free slot of the XCD placement
  A ar[NB], ai[NB];
#pragma unroll
  for (int nb = 0; nb < NB; ++nb) { ar[nb] = Mfma<R>::zero(); ai[nb] = Mfma<R>::zero(); }
  ConjTransA<R> aload{(const C *)W.K, W.sz};
  tile_gemm<R, NB, KUT>(aload.M, 0, W.r0, W.r, W.sz, (const C *)W.y, W.Np, W.jt, lane, ar, ai,
                   nullptr, aload);
  store_tile<R, NB>((C *)W.z, W.r0, W.r, W.Np, W.jt, lane, (R)1, ar, ai);
}
template <typename R, int NB, int KUT = 0>
__global__ __launch_bounds__(256) void k_final_adj_mr(const MFAItem *items, int64_t nitems) {
  b_final_adj_mr<R, NB, KUT>(items, nitems, blockIdx.x);
}

// Adjoint of a transfer unit: rows [r0, r0 + 16) of its c inputs,
// z_in = X_a^H w_a + X_b^H w_b as one product over the stacked ra + rb
// outputs (w_a and w_b are separate blocks).
template <typename R, int NB, int KUT = 0>
__device__ __forceinline__ void b_wstage_adj_mr(const MWAItem *items, int64_t nitems, int64_t bid) {
  using C = cplx_t<R>;
  using A = typename Mfma<R>::acc;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const int64_t it = bid * 4 + wave;
  if (it >= nitems) return;
  const MWAItem W = items[it];
  if (W.Np == 0) return;   // a free slot of the XCD placement
  A ar[NB], ai[NB];
#pragma unroll
  for (int nb = 0; nb < NB; ++nb) { ar[nb] = Mfma<R>::zero(); ai[nb] = Mfma<R>::zero(); }
  const int ra = W.ra, rb = W.rb, c = W.c;
  const int row = W.r0 + (lane & 15);
  const int rowc = row < c ? row : 0;
  AdjStackedA<R> aload;
  aload.Ta = (const C *)W.T;
  aload.Tb = aload.Ta + (int64_t)ra * (c - ra);
  aload.safe = aload.Ta;
  aload.ra = ra;
  aload.rb = rb;
  // inverse orders pa, pb of the unit's index lists (ia, ib, pa, pb)
  aload.pja = ldg16(W.idx, 2 * (int64_t)c + rowc);
  aload.pjb = ldg16(W.idx, 3 * (int64_t)c + rowc);
  tile_gemm<R, NB, KUT>(aload.Ta, 0, W.r0, c, ra + rb, (const C *)W.za, W.Np, W.jt, lane, ar, ai,
                   nullptr, aload, (const C *)W.zb, ra);
  store_tile<R, NB>((C *)W.zin, W.r0, c, W.Np, W.jt, lane, (R)1, ar, ai);
}
template <typename R, int NB, int KUT = 0>
__global__ __launch_bounds__(256) void k_wstage_adj_mr(const MWAItem *items, int64_t nitems) {
  b_wstage_adj_mr<R, NB, KUT>(items, nitems, blockIdx.x);
}

// Adjoint, leaf part: u_leaf = scale (D^H y_leaf + sum_l V_l^H z_l), rows
// [r0, r0 + 16) of the leaf's cells, every level in a fixed order.
template <typename R, int NB, int KUT = 0>
__device__ __forceinline__ void b_vstage_adj_mr(const MVAItem *items, int64_t nitems, int64_t bid) {
  using C = cplx_t<R>;
  using A = typename Mfma<R>::acc;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const int64_t it = bid * 4 + wave;
  if (it >= nitems) return;
  const MVAItem W = items[it];
  if (W.Np == 0) return;   // a free slot of the XCD placement
  A ar[NB], ai[NB];
#pragma unroll
  for (int nb = 0; nb < NB; ++nb) { ar[nb] = Mfma<R>::zero(); ai[nb] = Mfma<R>::zero(); }
  const C *F = (const C *)W.F;
  const C *z = (const C *)W.z;
  const int sz = W.sz;
  const int row = W.r0 + (lane & 15);
  const int rowc = row < sz ? row : 0;
  ConjTransA<R> dl{F + W.dense_off, sz};
  tile_gemm<R, NB, KUT>(dl.M, 0, W.r0, sz, sz, (const C *)W.y, W.Np, W.jt, lane, ar, ai, nullptr, dl);
  for (int l = 0; l < W.Lv; ++l) {
    const VDesc d = W.vd[l];
    AdjVA<R> vl;
    vl.T = F + d.foff;
    vl.safe = F;
    vl.r = d.r;
    vl.pj = ldg16(W.fidx + d.ioff, sz + rowc);   // the cell's position in the order
    tile_gemm<R, NB, KUT>(vl.T, 0, W.r0, sz, d.r, z + d.zout * W.Np, W.Np, W.jt, lane, ar, ai,
                     nullptr, vl);
  }
  store_tile<R, NB>((C *)W.u, W.r0, sz, W.Np, W.jt, lane, (R)W.scale, ar, ai);
}
template <typename R, int NB, int KUT = 0>
__global__ __launch_bounds__(256) void k_vstage_adj_mr(const MVAItem *items, int64_t nitems) {
  b_vstage_adj_mr<R, NB, KUT>(items, nitems, blockIdx.x);
}

// s (natural order, column-major N_v x nrhs, leading dimension ld) ->
// x (tree order, row stride Np), scaled by h^d; columns nrhs..Np-1 zeroed.
// 64 tree positions x 16 columns per workgroup through LDS.
template <typename R>
__device__ __forceinline__ void b_gather_in(const MTrans *jobs, int64_t bx, int by, int bz,
                                            cplx_t<R> (*tile)[17]) {
  using C = cplx_t<R>;
  const MTrans J = jobs[by];
  const int64_t p0 = bx * 64;
  const int jt = bz;
  if (p0 >= J.Nv || jt * 16 >= J.Np) return;
  const int t = threadIdx.x;
  // read: column j fastest-varying over threads' positions
  for (int q = t; q < 64 * 16; q += 256) {
    const int pl = q & 63, j = q >> 6;
    const int64_t p = p0 + pl;
    const int col = jt * 16 + j;
    C v{0, 0};
    if (p < J.Nv && col < J.nrhs) {
      const C s = ((const C *)J.src)[J.perm[p] + (int64_t)col * J.ld];
      v = C{s.x * (R)J.scale, s.y * (R)J.scale};
    }
    tile[pl][j] = v;
  }
  __syncthreads();
  for (int q = t; q < 64 * 16; q += 256) {
    const int j = q & 15, pl = q >> 4;
    const int64_t p = p0 + pl;
    if (p < J.Nv) ((C *)J.dst)[p * J.Np + jt * 16 + j] = tile[pl][j];
  }
}
template <typename R>
__global__ __launch_bounds__(256) void k_gather_in(const MTrans *jobs, int64_t njobs) {
  __shared__ cplx_t<R> tile[64][17];
  b_gather_in<R>(jobs, blockIdx.x, blockIdx.y, blockIdx.z, tile);
}

// y (tree order, row stride Np) -> u (natural order, column-major, ld).
template <typename R>
__device__ __forceinline__ void b_scatter_out(const MTrans *jobs, int64_t bx, int by, int bz,
                                              cplx_t<R> (*tile)[17]) {
  using C = cplx_t<R>;
  const MTrans J = jobs[by];
  const int64_t p0 = bx * 64;
  const int jt = bz;
  if (p0 >= J.Nv || jt * 16 >= J.Np) return;
  const int t = threadIdx.x;
  for (int q = t; q < 64 * 16; q += 256) {
    const int j = q & 15, pl = q >> 4;
    const int64_t p = p0 + pl;
    if (p < J.Nv) tile[pl][j] = ((const C *)J.src)[p * J.Np + jt * 16 + j];
  }
  __syncthreads();
  for (int q = t; q < 64 * 16; q += 256) {
    const int pl = q & 63, j = q >> 6;
    const int64_t p = p0 + pl;
    const int col = jt * 16 + j;
    if (p < J.Nv && col < J.nrhs) ((C *)J.dst)[J.perm[p] + (int64_t)col * J.ld] = tile[pl][j];
  }
}
template <typename R>
__global__ __launch_bounds__(256) void k_scatter_out(const MTrans *jobs, int64_t njobs) {
  __shared__ cplx_t<R> tile[64][17];
  b_scatter_out<R>(jobs, blockIdx.x, blockIdx.y, blockIdx.z, tile);
}

// The whole batched product in one persistent launch: the workgroups walk
// the phases (gather, every stage, scatter, pass after pass) in order, each
// taking the units b, b + gridDim.x, ... of a phase (workgroup b keeps XCD
// b % 8 since gridDim.x is a multiple of 8, so the XCD placement of the work
// items holds), and wait at a grid-wide barrier between phases.  Launched
// cooperatively: every workgroup is resident, so the barrier cannot wait on
// a workgroup that has not started.
template <typename R, int NB>
__global__ __launch_bounds__(256) void k_multi_persistent(const MPhase *phases, int nphase) {
  __shared__ cplx_t<R> tile[64][17];
  cooperative_groups::grid_group grid = cooperative_groups::this_grid();
  for (int q = 0; q < nphase; ++q) {
    const MPhase P = phases[q];
    const bool trans = P.kind >= 6;
    const int64_t nu = trans ? (int64_t)P.nx * P.n * P.maxjt : (P.n + 3) / 4;
    for (int64_t u = blockIdx.x; u < nu; u += gridDim.x) {
      switch (P.kind) {
        case 0: b_vstage_mr<R, NB>((const MVItem *)P.items, P.n, u); break;
        case 1: b_wstage_mr<R, NB>((const MWItem *)P.items, P.n, u); break;
        case 2: b_final_mr<R, NB>((const MFItem *)P.items, P.n, u); break;
        case 3: b_final_adj_mr<R, NB>((const MFAItem *)P.items, P.n, u); break;
        case 4: b_wstage_adj_mr<R, NB>((const MWAItem *)P.items, P.n, u); break;
        case 5: b_vstage_adj_mr<R, NB>((const MVAItem *)P.items, P.n, u); break;
        default: {
          const int64_t bx = u % P.nx, rest = u / P.nx;
          const int by = (int)(rest % P.n), bz = (int)(rest / P.n);
          if (P.kind == 6) b_gather_in<R>((const MTrans *)P.items, bx, by, bz, tile);
          else b_scatter_out<R>((const MTrans *)P.items, bx, by, bz, tile);
          __syncthreads();   // the tile is reused by the next unit
        }
      }
    }
    grid.sync();
  }
}

// ---------------------------------------------------------------------------
template <typename R, int NB, int KUT>
static void launch_stage_nb(const MStagePlan &sp, hipStream_t st) {
  if (sp.kind == 0 && sp.n)
    hipLaunchKernelGGL((k_vstage_mr<R, NB, KUT>), dim3((sp.n + 3) / 4), dim3(256), 0, st,
                       (const MVItem *)sp.items, sp.n);
  if (sp.kind == 1 && sp.n)
    hipLaunchKernelGGL((k_wstage_mr<R, NB, KUT>), dim3((sp.n + 3) / 4), dim3(256), 0, st,
                       (const MWItem *)sp.items, sp.n);
  if (sp.kind == 2 && sp.n)
    hipLaunchKernelGGL((k_final_mr<R, NB, KUT>), dim3((sp.n + 3) / 4), dim3(256), 0, st,
                       (const MFItem *)sp.items, sp.n);
  if (sp.kind == 3 && sp.n)
    hipLaunchKernelGGL((k_final_adj_mr<R, NB, KUT>), dim3((sp.n + 3) / 4), dim3(256), 0, st,
                       (const MFAItem *)sp.items, sp.n);
  if (sp.kind == 4 && sp.n)
    hipLaunchKernelGGL((k_wstage_adj_mr<R, NB, KUT>), dim3((sp.n + 3) / 4), dim3(256), 0, st,
                       (const MWAItem *)sp.items, sp.n);
  if (sp.kind == 5 && sp.n)
    hipLaunchKernelGGL((k_vstage_adj_mr<R, NB, KUT>), dim3((sp.n + 3) / 4), dim3(256), 0, st,
                       (const MVAItem *)sp.items, sp.n);
}

template <typename R>
hipError_t launch_multi_stage(const MStagePlan &sp, hipStream_t st) {
  // (column-tile width, k-steps per chunk); ku = 0 is the width's default
  switch (sp.nb * 16 + sp.ku) {
    case 16 + 0: case 16 + 4: launch_stage_nb<R, 1, 4>(sp, st); break;
    case 16 + 8: launch_stage_nb<R, 1, 8>(sp, st); break;
    case 16 + 2: launch_stage_nb<R, 1, 2>(sp, st); break;
    case 32 + 0: case 32 + 2: launch_stage_nb<R, 2, 2>(sp, st); break;
    case 32 + 4: launch_stage_nb<R, 2, 4>(sp, st); break;
    case 32 + 1: launch_stage_nb<R, 2, 1>(sp, st); break;
    case 64 + 0: case 64 + 1: launch_stage_nb<R, 4, 1>(sp, st); break;
    case 64 + 2: launch_stage_nb<R, 4, 2>(sp, st); break;
    case 128 + 0: case 128 + 1: launch_stage_nb<R, 8, 1>(sp, st); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <typename R>
hipError_t launch_gather_in(const MTrans *jobs, int64_t njobs, int64_t maxNv, int maxjt,
                            hipStream_t st) {
  if (njobs == 0) return hipSuccess;
  hipLaunchKernelGGL((k_gather_in<R>), dim3((maxNv + 63) / 64, njobs, maxjt), dim3(256), 0, st,
                     jobs, njobs);
  return hipGetLastError();
}

template <typename R>
hipError_t launch_scatter_out(const MTrans *jobs, int64_t njobs, int64_t maxNv, int maxjt,
                              hipStream_t st) {
  if (njobs == 0) return hipSuccess;
  hipLaunchKernelGGL((k_scatter_out<R>), dim3((maxNv + 63) / 64, njobs, maxjt), dim3(256), 0, st,
                     jobs, njobs);
  return hipGetLastError();
}

template <typename R> static const void *persistent_kernel(int nb) {
  switch (nb) {
    case 1: return (const void *)k_multi_persistent<R, 1>;
    case 2: return (const void *)k_multi_persistent<R, 2>;
    case 4: return (const void *)k_multi_persistent<R, 4>;
    case 8: return (const void *)k_multi_persistent<R, 8>;
    default: return nullptr;
  }
}

template <typename R> hipError_t persistent_grid(int nb, int device, int *grid) {
  const void *k = persistent_kernel<R>(nb);
  if (!k) return hipErrorInvalidValue;
  int per_cu = 0, ncu = 0;
  hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k, 256, 0);
  if (e != hipSuccess) return e;
  e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, device);
  if (e != hipSuccess) return e;
  const int g = per_cu * ncu - (per_cu * ncu) % 8;
  if (g < 8) return hipErrorInvalidConfiguration;
  *grid = g;
  return hipSuccess;
}

template <typename R>
hipError_t launch_multi_persistent(const MPhase *phases, int nphase, int nb, int grid,
                                   hipStream_t st) {
  const void *k = persistent_kernel<R>(nb);
  if (!k || grid < 8 || grid % 8) return hipErrorInvalidValue;
  void *args[] = {(void *)&phases, (void *)&nphase};
  return hipLaunchCooperativeKernel(k, dim3(grid), dim3(256), args, 0, st);
}

template hipError_t persistent_grid<float>(int, int, int *);
template hipError_t persistent_grid<double>(int, int, int *);
template hipError_t launch_multi_persistent<float>(const MPhase *, int, int, int, hipStream_t);
template hipError_t launch_multi_persistent<double>(const MPhase *, int, int, int, hipStream_t);
template hipError_t launch_multi_stage<float>(const MStagePlan &, hipStream_t);
template hipError_t launch_multi_stage<double>(const MStagePlan &, hipStream_t);
template hipError_t launch_gather_in<float>(const MTrans *, int64_t, int64_t, int, hipStream_t);
template hipError_t launch_gather_in<double>(const MTrans *, int64_t, int64_t, int, hipStream_t);
template hipError_t launch_scatter_out<float>(const MTrans *, int64_t, int64_t, int, hipStream_t);
template hipError_t launch_scatter_out<double>(const MTrans *, int64_t, int64_t, int, hipStream_t);

}  // namespace hbi
