// Work items and launchers of the multi-right-hand-side (MFMA) apply.
#pragma once

#include <vector>
#include "hbi_internal.h"

namespace hbi {

// Transfer-stage item, column tiles [jt, jt+NB), z_out = X z_in with
// X = [I, T] Pi^T (T column-major, r x (c - r)).  Two forms:
//  * one child (rb < 0): rows [r0, r0+16) of X, T of the child at T, idx its
//    column order (c entries: skeleton columns, then the others); B rows
//    are gathered through idx and the skeleton rows added;
//  * a unit of at most 32 rows (rb >= 0): rows [r0, r0+16) of the stacked
//    [X_a; X_b], its entries synthesised from T_a (at T), T_b (after it) and
//    the inverse orders pa, pb (idx: the unit's lists ia, ib, pa, pb), so a
//    small pair shares tiles and its B rows are read in order.
// Vector pointers are absolute.  In every item kind Np = 0 marks an empty
// slot (the wave returns at once).
struct MWItem {
  const void *T;
  const uint16_t *idx;
  const void *zin;     // c x Np
  void *zout, *zoutb;  // r x Np (the child, or a), rb x Np (b)
  int32_t r, rb, c, r0, jt, Np;
};

// V^0 item: rows [r0, r0+16) of V = [I, T] Pi^T (T r x (sz - r) at T, the
// column order idx: skeleton cells, then the others) times the leaf's
// inputs.
struct MVItem {
  const void *T;
  const uint16_t *idx;
  const void *x;       // sz x Np (tree-ordered input rows of the leaf)
  void *z;             // r x Np
  int32_t r, sz, r0, jt, Np, pad;
};

// Final item: rows [r0, r0+16) of one leaf: dense block plus the K^L of
// every HODBF level.
struct MFItem {
  const void *F;       // factor store (element offsets below)
  const void *z;       // z base of the problem (offsets in kd are rows)
  const void *x;       // sz x Np leaf inputs
  void *y;             // sz x Np leaf outputs
  const KDesc *kd;     // Lv descriptors of this leaf
  int64_t dense_off;
  int32_t sz, Lv, r0, jt, Np, pad;
};

// Adjoint items (u = h^d K^H s), in the reverse order of the stages:
// K^L part: z_l = (K^L)^H y_leaf, rows [r0, r0+16) of the r skeleton rows
// (K column-major sz x r).
struct MFAItem {
  const void *K;
  const void *y;       // sz x Np leaf inputs
  void *z;             // r x Np
  int32_t r, sz, r0, jt, Np, pad;
};
// A transfer unit: rows [r0, r0+16) of its c inputs, zin = X_a^H za + X_b^H zb
// (T_a at T, T_b after it; idx: the unit's lists ia, ib, pa, pb).
struct MWAItem {
  const void *T;
  const uint16_t *idx;
  void *zin;           // c x Np
  const void *za, *zb; // ra x Np, rb x Np
  int32_t ra, rb, c, r0, jt, Np;
};
// Leaf part: rows [r0, r0+16) of u_leaf = scale (D^H y + sum_l V_l^H z_l).
struct MVAItem {
  const void *F;       // factor store (element offsets in vd, dense_off)
  const uint16_t *fidx;
  const void *y;       // sz x Np leaf inputs
  void *u;             // sz x Np leaf outputs
  const VDesc *vd;     // Lv descriptors of this leaf
  const void *z;       // z base of the problem (offsets in vd are rows)
  int64_t dense_off;
  double scale;
  int32_t sz, Lv, r0, jt, Np, pad;
};

// Gather / scatter between natural column-major vectors and tree-ordered
// row-major blocks.
struct MTrans {
  const void *src;
  void *dst;
  const int32_t *perm;
  int64_t Nv, ld;
  int32_t nrhs, Np;
  double scale;
};

struct MStagePlan {
  int kind;            // 0 V, 1 W, 2 final; adjoint: 3 K^L, 4 W, 5 leaf
  int nb;              // column tiles per wave
  const void *items;
  int64_t n;
  int ku = 0;          // MFMA k-steps per load chunk (0: the default for nb)
};
// k-steps per chunk that launch_multi_stage accepts for a column-tile
// width, the default first
inline std::vector<int> multi_ku_candidates(int nb) {
  switch (nb) {
    case 1: return {4, 8, 2};
    case 2: return {2, 4, 1};
    case 4: return {1, 2};
    case 8: return {1};
    default: return {};
  }
}

// One phase of the persistent batched product: a stage (kind 0..5, as in
// MStagePlan, n work items) or a gather (6) / scatter (7) over n jobs, nx
// blocks of 64 tree positions and maxjt column tiles each.
struct MPhase {
  int kind;
  int nx, maxjt;
  const void *items;
  int64_t n;
};

template <typename R> hipError_t launch_multi_stage(const MStagePlan &sp, hipStream_t st);
// Co-resident workgroups of the persistent kernel for column-tile width nb
// (a multiple of 8), and its cooperative launch over device phases.
template <typename R> hipError_t persistent_grid(int nb, int device, int *grid);
template <typename R>
hipError_t launch_multi_persistent(const MPhase *phases, int nphase, int nb, int grid,
                                   hipStream_t st);
template <typename R>
hipError_t launch_gather_in(const MTrans *jobs, int64_t njobs, int64_t maxNv, int maxjt,
                            hipStream_t st);
template <typename R>
hipError_t launch_scatter_out(const MTrans *jobs, int64_t njobs, int64_t maxNv, int maxjt,
                              hipStream_t st);

}  // namespace hbi
