// Internal structures shared by the host driver and the HIP kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#define HBI_MAX_NI 16
#define HBI_MAX_LEAF 64
#define HBI_ID_THREADS 1024
#define HBI_ID_NMAX 4096   // largest candidate-column count an ID accepts
#define HBI_ID_ONCHIP_NMAX 64   // largest column count of the on-chip ID kernel
#define HBI_MAX_INCLUSION 32768  // segments of a curve inclusion
#define HBI_WSTAGE_LDS_BYTES 4096   // LDS of one forward transfer-stage wave

// Problem constants visible to the kernels.
struct DevProblem {
  int dim, nI, NT, NTb, nterms;
  int nbox[3];
  double box_origin[3], box_size;
  double omega, h, hd;   // hd = h^dim
};

// Per-cell data, in tree order (position p of the K-D permutation).
struct DevCells {
  const double *xyz;     // [Nv*3] centre coordinates
  const double *lw;      // [Nv*dim*nI] 1D Lagrange weights in the cell's box
  const int32_t *box;    // [Nv] table box of the cell
  const double2 *self;   // [Nv] self term K_ii
  const double *slow;    // [Nv] slowness
  const int32_t *perm;   // [Nv] tree position -> natural index
  // With a curve inclusion, segment centres follow the cells as points
  // Nv..Nv+ns-1 of xyz/lw/box/self, and cellof[p] is the position of the
  // cell containing point p (p itself for a cell); null without one.
  const int32_t *cellof;
};

// Which self value an entry (rp, cp) takes, or -1 for the HB value: the
// diagonal, and a segment centre paired with the cell that contains it
// (that cell's self term, the cell average of the leading HB term).
__host__ __device__ inline int32_t self_index(const DevCells &C, int32_t rp, int32_t cp) {
  if (rp == cp) return rp;
  if (C.cellof) {
    if (C.cellof[cp] == rp) return rp;
    if (C.cellof[rp] == cp) return cp;
  }
  return -1;
}

struct DevTables {
  const double *FT[3];   // transposed tables FT[t][B*NT + A] = F_t[A*NT + B]
};

// hb_entry work description for one block K(rows, cols).
struct EntryBlock {
  int64_t row_off;   // into rows[] / rowslot[]
  int64_t col_off;   // into cols[]
  int64_t slot_off;  // into slotbox[]
  int64_t hc_off;    // into the Hc workspace (doubles)
  double2 *out;      // column-major m x n output, leading dimension m
  int32_t m, n, nslot, pad;
};

// Entry tile: sorted rows [r0, r0 + nr) of block blk (all in row-box slot
// `slot`) x columns [j0, j0 + nj).
struct ETile { int32_t blk, r0, nr, j0, nj, slot; };

// One interpolative decomposition on a block already in the workspace.
struct IdBlock {
  double2 *A;        // m x n column-major (overwritten)
  double2 *X;        // output r x n column-major (capacity min(m,n)*n)
  int32_t *piv;      // output, n entries (first r are the skeleton)
  int32_t m, n;
};

// Apply descriptors (element offsets into the factor store / z workspace).
// V^0 block of a leaf and HODBF level: X = [I, T] Pi^T over the leaf's
// cells; only T (r x (|nu| - r), column-major) is stored at foff, and the
// index store holds at ioff the column order (skeleton cells in pivot
// order, then the others ascending) and its inverse, |nu| entries each.
struct VDesc { int64_t foff; int64_t zout; int64_t ioff; int32_t r; int32_t pad; };
struct KDesc { int64_t foff; int64_t zin; int32_t r; int32_t pad; };
// A transfer unit: the interpolation matrices X_a (ra x c) and X_b (rb x c)
// of a sibling pair over the same c candidate columns.  An interpolative
// decomposition gives X = [I, T] Pi^T, so only T is stored: T_a (ra x ta,
// ta = c - ra) at foff and T_b (rb x tb) at foff + ra ta, column-major.  The
// index store holds at ioff four lists of c entries: ia (the skeleton
// columns of a in pivot order, then its other columns in increasing order),
// ib, and their inverses pa (pa[ia[k]] = k), pb.  Row i of X_a x is
// x[ia[i]] + sum_m T_a[i, m] x[ia[ra + m]].
struct WUnit {
  int64_t foff;
  int64_t zin;       // c inputs (skeletons of nu_1 then nu_2)
  int64_t zouta, zoutb;
  int64_t ioff;
  int32_t ra, rb, c, pad;
};
// Work item of a transfer stage: rows (forward, of the pair stacked a then
// b) [off, off + wr) or columns (adjoint) [off, off + 64) of a unit, with
// the unit's fields copied in so that a wave needs one descriptor load.
// Forward windows of wr = 16 rows (64 / wr lanes per row) serve the widest
// units, whose rows are long.
struct WItem {
  int64_t foff, zin, zouta, zoutb, ioff;
  int32_t ra, rb, c;
  int16_t off, wr;
};
struct LeafInfo { int32_t start, size; int64_t dense_off; };
