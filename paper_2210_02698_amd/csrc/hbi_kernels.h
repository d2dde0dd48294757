// Launchers of the HIP kernels (defined in hbi_kernels.hip).
#pragma once
#include <vector>

#include "hbi_internal.h"

namespace hbi {

// Compaction of a sibling pair's interpolation matrices: T_a = X_a[:, nsa]
// (ra x (c - ra)) then T_b = X_b[:, nsb] at dst, column-major; nsa and nsb
// list the non-skeleton columns (device, c - ra and c - rb entries).
struct PairDesc {
  const double2 *xa, *xb;
  double2 *dst;
  const uint16_t *nsa, *nsb;
  int32_t ra, rb, c, pad;
};
struct PlaceDesc { const double2 *src; int64_t dst; int64_t count; };   // dst: element offset

// Optional observer of apply launches (per-kernel event timing).
struct LaunchHook {
  virtual void before(const char *name, double bytes) = 0;
  virtual void after() = 0;
  virtual ~LaunchHook() = default;
};

// Device-side apply plan (all pointers are device pointers).
struct ApplyPlan {
  int Lv = 0, Lmax = 0;
  int64_t nleaf = 0;
  const LeafInfo *leaves = nullptr;
  const int32_t *perm = nullptr;
  const VDesc *vd = nullptr;
  const KDesc *kd = nullptr;
  const uint16_t *fidx = nullptr;   // index store of the transfer units
  std::vector<const WUnit *> units;   // index k = 1..Lmax
  std::vector<int64_t> nunits;
  std::vector<const WItem *> items, items_adj;   // index k
  std::vector<int64_t> nitems, nitems_adj;
  // forward transfer items stage their inputs and column orders in the
  // wave's LDS slice when they need at most cap_lds entries of it, else
  // gather the inputs from global memory
  int cap_lds = 0;
  // algorithmic traffic per launch, in complex elements and index bytes
  double v_elems = 0, v_idx = 0, f_elems = 0, f_idx = 0;
  std::vector<double> w_elems, w_idx;   // index k
};

hipError_t launch_cell_setup(const DevProblem &P, const int32_t *perm, int64_t Nv,
                             const int32_t ncell[3], const double origin[3],
                             double *xyz, double *lw, int32_t *box, hipStream_t st);
hipError_t launch_self_terms(const DevProblem &P, const double *slow, int64_t Nv,
                             const double *gx, const double *gw, int ng,
                             double2 *self, hipStream_t st);
hipError_t launch_colside(const DevProblem &P, const DevCells &C, const DevTables &T,
                          const EntryBlock *blks, const int32_t *work, int64_t nwork,
                          const int32_t *cols, const int32_t *slotbox, double *Hc,
                          hipStream_t st);
// Column-side contractions of every (cell, box) pair into Hcache
// (Nv * nbox * 3 * NTb doubles).
hipError_t launch_colside_cells(const DevProblem &P, const DevCells &C, const DevTables &T,
                                int64_t Nv, int nbox, double *Hcache, hipStream_t st);
// Entries of the blocks; the column side comes from the batch workspace Hc,
// or from Hcache (nbox boxes per cell) when that is non-null.
hipError_t launch_entries(const DevProblem &P, const DevCells &C, const EntryBlock *blks,
                          const ETile *tiles, int64_t ntiles, const int32_t *rows,
                          const int32_t *rord, const int32_t *cols, const double *Hc,
                          const int32_t *slotbox, const double *Hcache, int nbox,
                          hipStream_t st);
// Interpolative decompositions of the blocks blks[sel[0..nb)]: k_cpqr works
// on the block in global memory (any n); launch_id_onchip handles blocks of
// at most HBI_ID_ONCHIP_NMAX columns on chip (nmax = their largest n).
hipError_t launch_cpqr(const IdBlock *blks, const int32_t *sel, int64_t nb, int nmax, int mmax,
                       double tol, int32_t *rank, hipStream_t st);
hipError_t launch_id_onchip(const IdBlock *blks, const int32_t *sel, int64_t nb, int nmax,
                            double tol, int32_t *rank, hipStream_t st);
// Blocked (panel) form of k_cpqr for any n whose norms and panel fit in LDS
// (falls back to launch_cpqr otherwise).
hipError_t launch_cpqr_blocked(const IdBlock *blks, const int32_t *sel, int64_t nb, int nmax,
                               int mmax, double tol, int32_t *rank, hipStream_t st);
// Tall blocks (m >= n, every selected one): k_gram forms G = A^H A in X's
// space, k_pchol the pivoted Cholesky factorisation of G (the pivots and R of
// the column-pivoted QR of A) and X; nmax = their largest n.
hipError_t launch_id_gram(const IdBlock *blks, const int32_t *sel, int64_t nb, int nmax,
                          double tol, int32_t *rank, hipStream_t st);
hipError_t launch_pack_pairs(const PairDesc *d, int64_t np, hipStream_t st);
hipError_t launch_place_blocks(const PlaceDesc *d, int64_t nb, void *F, bool f32,
                               hipStream_t st);

template <typename R>
hipError_t launch_apply(const ApplyPlan &ap, const void *s, void *u, void *z,
                        const void *F, R hd, bool adjoint, hipStream_t st,
                        LaunchHook *hook = nullptr);

// Single butterfly of the inclusion's cells x segments matrix G (hbi_s2v.hip):
// V^0 over the segment leaves, W^1..W^L over the units of each level, K^L
// over the cell nodes of depth L.  Offsets are elements of the factor store
// F (T blocks column major), of the index store idx, and of the skeleton
// vector z.
struct S2VLeaf {
  int64_t foff, ioff, zoff;   // T (r x (n - r)); idx: column order, inverse (n each)
  int32_t r, n, lo, pad;      // rank, segments [lo, lo + n)
};
struct S2VNode {
  int64_t foff, zoff;         // K (size x r, column major); skeleton vector
  int32_t start, size, r, pad;   // cells at tree positions [start, start + size)
};
struct S2VPlan {
  int L = 0;
  const void *F = nullptr;
  const uint16_t *idx = nullptr;
  const int32_t *perm = nullptr;   // tree position -> natural cell index
  const S2VLeaf *leaves = nullptr;
  const S2VNode *nodes = nullptr;
  int64_t nleaf = 0, nnode = 0;
  std::vector<const WUnit *> units;   // index k = 1..L
  std::vector<int64_t> nunits;
  // work items (descriptor index, first of four outputs) of the wave-per-
  // output kernels: rows of level k's units, their inputs (transposed), and
  // the skeleton columns of the K^L nodes (transposed)
  std::vector<const int2 *> witems, wtitems;   // index k
  std::vector<int64_t> nwitems, nwtitems;
  const int2 *ktitems = nullptr;
  int64_t nktitems = 0;
  void *z = nullptr;
  int32_t size_max = 0;
};
// transpose = false: y (cells, natural order) += scale op(G) x (segments);
// transpose = true: y (segments) = scale op(G)^T x (cells); op = conj or not.
template <typename R>
hipError_t launch_s2v(const S2VPlan &p, const void *x, void *y, R scale, bool transpose,
                      bool conj, hipStream_t st);

// Curve inclusion (hbi_inclusion.hip).  G: the butterfly bf, or (bf null) a
// chunked N_v x N_s array of g(cell, segment); M = (K^{s2s})^{-1} and MH = M^H,
// column-major N_s x N_s;
// w the segment lengths; part, z, y, part2, part3 scratch of nchunk*N_s,
// N_s, N_s, ceil(N_s/256)*N_v and ceil(N_s/256)*N_s entries.
// Element type complex64/complex128 (w float/double) as for the factors.
struct InclusionPlan {
  const S2VPlan *bf = nullptr;   // G as a butterfly (then G is not used)
  const void *G = nullptr, *M = nullptr, *MH = nullptr, *w = nullptr;
  void *part = nullptr, *z = nullptr, *y = nullptr, *part2 = nullptr, *part3 = nullptr;
  int64_t Nv = 0;
  int32_t ns = 0, m = 0;
};
hipError_t launch_point_setup(const DevProblem &P, const double *xy, const double *w,
                              const double *slow, int32_t ns, int64_t p0, double *xyz,
                              double *lw, int32_t *box, double2 *self, hipStream_t st);
hipError_t launch_s2s_inverse(double2 *A, int32_t n, const double *w, int32_t *perm,
                              double2 *colk, double2 *Sb, int32_t *status, hipStream_t st);
hipError_t launch_conj_transpose(const double2 *src, int32_t n, double2 *dst, hipStream_t st);
template <typename R>
hipError_t launch_inclusion_apply(const InclusionPlan &ip, const void *x, void *u, R hd,
                                  bool adjoint, hipStream_t st);

}  // namespace hbi
