/*
 * hbi.h -- C ABI of the butterfly-compressed Hadamard-Babich (HB) volume
 * integrator on AMD Instinct MI355X (gfx950).
 *
 * The library applies the discretised HB integrator U = K^{v2v} I of the
 * paper's Sec. 3.1 (eq. m_v2v): N_v cells of size h on a regular grid, the
 * source vector I_j = s(r_j) h^d, and the operator entries
 *   K_ij = v0 f_{-(d-2)/2}(omega, tau) + v1 f_{1-(d-2)/2}(omega, tau),  i != j
 * (eq. babich with N = 1 and the terms of eq. termf), with tau^2, v0, v1
 * taken from Chebyshev-interpolated tables (eq. chebinterp,
 * eq. chebinterpblock) and K_ii the cell integral of the leading HB term
 * (Appendix A).  K is compressed as a hierarchically off-diagonal butterfly
 * (HODBF) matrix (Sec. 4.2): a K-D cluster tree, one column-wise butterfly
 * per pair of sibling clusters (eq. butterfly_mat, eq. butterfly_factors)
 * built level by level from interpolative decompositions of proxy-row
 * blocks (eq. ID, eq. proxy, eq. proxyv2v), and dense diagonal leaf blocks.
 *
 * Conventions shared by every call:
 *  * Every function returns hbi_status; nothing throws across the ABI.  On
 *    failure hbi_last_error(ctx) (or hbi_last_error(NULL) when no context
 *    exists) gives a human-readable reason.
 *  * Cells are numbered naturally: i = x + ncell[0] * (y + ncell[1] * z).
 *    Cell (x, y, z) has centre origin + (idx + 0.5) * h.
 *  * Complex arrays are interleaved (re, im): complex128 for HBI_F64,
 *    complex64 for HBI_F32.
 *  * Device arrays are HIP device pointers on the context's device (for
 *    instance torch.Tensor.data_ptr()).  Host arrays are ordinary memory.
 */
#ifndef HBI_H
#define HBI_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct hbi_ctx hbi_ctx;

typedef enum {
  HBI_OK = 0,
  HBI_ERR_ARG = 1,      /* bad shape, null pointer, out-of-range value   */
  HBI_ERR_STATE = 2,    /* call out of order (apply before build, ...)   */
  HBI_ERR_OOM = 3,      /* device or host allocation failed              */
  HBI_ERR_HIP = 4,      /* a HIP runtime call failed (text in last_error) */
  HBI_ERR_NUMERIC = 5   /* non-finite value met where one is not allowed  */
} hbi_status;

typedef enum { HBI_F64 = 0, HBI_F32 = 1 } hbi_prec;

/* Problem statement (Sec. 3.1) and tabulated HB ingredients (Sec. 4.1,
 * eq. chebinterp).
 *
 * Table layout: the table region is nbox[0] x nbox[1] (x nbox[2]) cubic
 * boxes of side box_size from box_origin; box b = bx + nbox0*(by + nbox1*bz).
 * Each box carries nI first-kind Chebyshev nodes per axis at
 * lo + box_size*(1 + cos((2k+1)pi/(2 nI)))/2, k = 0..nI-1, node multi-index
 * a = k1 + nI*(k2 + nI*k3); global node A = b*nI^d + a, NT = nboxes*nI^d.
 * tau2, v0, v1 are NT x NT row-major: F[A*NT + B] = f(node A as observation
 * point, node B as source).  A point is interpolated with the nodes of the
 * box floor((x - box_origin)/box_size) (clamped), so cells must lie inside
 * the table region.  With nbox = {1,1,1} this is the paper's global table. */
typedef struct {
  int32_t dim;            /* 2 or 3                                        */
  int32_t ncell[3];       /* cells per axis (unused axes ignored)          */
  double origin[3];       /* lower corner of the cell grid                 */
  double h;               /* cell size (> 0)                               */
  double omega;           /* angular frequency (> 0)                       */
  int32_t nterms;         /* 1 (N = 0: v0 only) or 2 (N = 1: v0 and v1)    */
  int32_t nI;             /* Chebyshev nodes per axis per box, 2..16       */
  int32_t nbox[3];        /* table boxes per axis (>= 1)                   */
  double box_origin[3];
  double box_size;        /* > 0                                           */
  const double *tau2;     /* host [NT*NT]                                  */
  const double *v0;       /* host [NT*NT]                                  */
  const double *v1;       /* host [NT*NT]; may be NULL iff nterms == 1     */
  const double *slowness; /* host [N_v], n(r_i) at cell centres, natural
                             order (used by the self terms, Appendix A)    */
} hbi_tables;

/* Compression parameters (Sec. 4.2.2 and the parameter choices of
 * Sec. 5.1).  Zero / negative fields select the default in brackets. */
typedef struct {
  double chi;               /* proxy oversampling factor chi of eq. proxyv2v
                               [20 in 2D, 4 in 3D]                          */
  int32_t leaf_size;        /* max cells per leaf cluster [64]               */
  double neighbor_radius;   /* radius of the neighbour proxy rows n_i, in
                               cells [10 in 2D, 3 in 3D]                    */
  int32_t band_width;       /* width in cells of the boundary band that the
                               uniform proxy rows f_tau are drawn from [2]   */
  int64_t workspace_bytes;  /* device workspace budget per build batch
                               [1/8 of free device memory, clamped to
                               2..32 GiB]                                    */
} hbi_build_opts;

/* Create a context on HIP device `device`; all work is queued on
 * `hip_stream` (a hipStream_t, NULL = the null stream).  *out receives the
 * context, owned by the caller until hbi_destroy. */
hbi_status hbi_create(int device, void *hip_stream, hbi_ctx **out);

/* Free the context and every device allocation it owns.  NULL is a no-op. */
hbi_status hbi_destroy(hbi_ctx *ctx);

/* Change the stream later applies are queued on. */
hbi_status hbi_set_stream(hbi_ctx *ctx, void *hip_stream);

/* Deep-copy the problem statement and the tables to the device and build the
 * cluster tree.  The caller keeps ownership of t and its arrays.  Drops any
 * earlier factors.  Synchronous. */
hbi_status hbi_load_tables(hbi_ctx *ctx, const hbi_tables *t);

/* Tables and cells of `src` at another angular frequency.  The HB
 * ingredients tau, v0, v1 do not depend on omega (Sec. 2.3: tabulated once,
 * reused for many frequencies), so a frequency sweep loads its tables once
 * and gives every further context a device-to-device copy of them, with the
 * cluster tree and per-cell data copied when the leaf sizes agree; only the
 * self terms (App. A), which depend on omega, are evaluated again.  ctx and
 * src are two contexts on the same device, or the same context (then only
 * the frequency changes).  A curve inclusion of src (hbi_set_inclusion) is
 * copied too.  Drops the earlier factors of ctx; src keeps its own.  src
 * must have tables (HBI_ERR_STATE otherwise); omega must be finite and > 0
 * (HBI_ERR_ARG).  Synchronous. */
hbi_status hbi_load_tables_from(hbi_ctx *ctx, const hbi_ctx *src, double omega);

/* A curve inclusion (Sec. 3.2, domain with a sound-hard inclusion; 2D): ns straight
 * segments with centres (xy[2i], xy[2i+1]), lengths w[i] > 0 and slowness
 * slowness[i] > 0 of the medium at the centres (host arrays, copied; the
 * centres must lie in the table region; 0 <= ns <= 32768, ns = 0 removes the
 * inclusion; the segments are taken in the given order, which should follow
 * the curve).  Later builds assemble, besides the volume factors, the
 * operator G[j, i] = g(r_j, r^s_i) over cells and segments (read as
 * K^{v2s} = G^T and K^{s2v} = G diag(w): the tables are symmetric) as a
 * single butterfly (Sec. 4.2: L = min(L_v, L_s) levels over the cell tree
 * and a halving tree of the segment indices with leaves of at most 8
 * segments, compressed at tol / 100; O(N_v) entries instead of N_v x ns),
 * and the inverse of K^{s2s} (eq. s2s, by Gauss-Jordan elimination with row
 * pivoting in FP64; HBI_ERR_NUMERIC if it is singular), both in the factors'
 * precision.  With the environment variable HBI_INCLUSION_DENSE=1 at build
 * time G is kept dense instead (N_v x ns entries), for comparison.  hbi_apply and hbi_apply_adjoint then apply the total operator
 * of eq. m_v2v_inclu, (K^{v2v} + K^{s2v} (K^{s2s})^{-1} K^{v2s}) h^d, and its
 * conjugate transpose; hbi_apply_batched rejects such contexts.  The
 * diagonal of K^{s2s} is -(i w/4)[1 + (2i/pi)(log(e^gamma omega n w/4) - 1)],
 * minus the integral of the leading HB term over the segment.  Needs
 * tables (HBI_ERR_STATE); drops the factors; hbi_load_tables removes the
 * inclusion, hbi_load_tables_from copies the source's.  Synchronous. */
hbi_status hbi_set_inclusion(hbi_ctx *ctx, int32_t ns, const double *xy, const double *w,
                             const double *slowness);

/* Override compression parameters for later builds (NULL restores the
 * defaults). */
hbi_status hbi_set_build_opts(hbi_ctx *ctx, const hbi_build_opts *opts);

/* Build the HODBF factors (Sec. 4.2): interpolative decompositions by
 * column-pivoted QR with relative tolerance `tol` (eq. ID: a pivot is kept
 * while |R_kk| > tol |R_11|), in FP64.  `prec` selects the precision the
 * factors are stored and applied in (HBI_F32 rounds the FP64 factors).
 * Needs loaded tables; replaces earlier factors.  Synchronous. */
hbi_status hbi_build(hbi_ctx *ctx, double tol, hbi_prec prec);

/* u = K (h^d s) (eq. m_v2v) for nrhs right-hand sides.  s and u are device
 * arrays, column-major N_v x nrhs with leading dimension ld >= N_v, natural
 * cell order, complex128 (HBI_F64 build) or complex64 (HBI_F32 build); they
 * must not overlap.  Asynchronous on the context's stream. */
hbi_status hbi_apply(hbi_ctx *ctx, const void *s, void *u, int32_t nrhs,
                     int64_t ld);

/* u = h^d K^H s: the exact conjugate transpose of the compressed operator
 * applied by hbi_apply (same layout rules).  With L(s) = ||P K h^d s - d||^2
 * the gradient with respect to conj(s) is h^d K^H P^T (P K h^d s - d). */
hbi_status hbi_apply_adjoint(hbi_ctx *ctx, const void *s, void *u,
                             int32_t nrhs, int64_t ld);

/* The batched workload: for p = 0..nprob-1, u[p] = K_p (h^d s[p]) with
 * nrhs[p] right-hand sides (column-major N_v,p x nrhs[p], leading dimension
 * ld[p], same element type and rules as hbi_apply).  All contexts must be
 * built, in the same precision and on the same device; the work is queued
 * on ctx[0]'s stream.  The factor products of all problems become complex
 * GEMM tiles over the right-hand sides (16x16x4 MFMA), each stage of every
 * problem in one launch, and the whole call is captured once into a HIP
 * graph that later calls with the same contexts, builds and nrhs replay
 * (new vector pointers are patched in; a context rebuilt since, or a new
 * context at a freed one's address, makes the call capture again).  The
 * graph is kept by ctx[0] until its next rebuild or hbi_destroy.  On the first call the column-tile
 * width, then the MFMA k-steps whose loads are issued together, are chosen
 * by timing the candidates on the batch itself (hbi_get_info of ctx[0]:
 * "batched_tile_nb", "batched_tile_ku", 0 for the width's default); choices
 * are kept for the process and in the JSON file named by HBI_TUNE_CACHE
 * when set.  Vector workspace is bounded by HBI_MULTI_BYTES (default 8 GiB);
 * larger batches run as several passes inside the same graph.  hbi_apply
 * with nrhs >= 2 uses the same path for one problem.  With the environment
 * variable HBI_BATCHED_PERSISTENT=1 (read when a batch is planned) the call
 * is instead one persistent cooperative kernel launch per call: its
 * workgroups walk every pass's gather, stages and scatter in order with a
 * grid-wide barrier between them, with results identical to the graph's;
 * hbi_get_info counts these launches in "batched_persistent_launches". */
hbi_status hbi_apply_batched(hbi_ctx *const *ctx, int32_t nprob,
                             const void *const *s, void *const *u,
                             const int32_t *nrhs, const int64_t *ld);

/* A 2D medium for hbi_tabulate: n^2 on a regular grid, point (i, j) at
 * origin + (i, j) * spacing, and the Taylor coefficients of n^2 about every
 * table node. */
typedef struct {
  int32_t n[2];             /* grid points per axis (>= 6)                       */
  double origin[2];
  double spacing;           /* > 0                                                */
  const double *n2;         /* host [n[0] * n[1]], n(r)^2, x fastest              */
  const double *taylor;     /* host [NT * 25]: about node A, the coefficient of
                               (x - x_A)^i (y - y_A)^j at [25 A + 5 i + j],
                               i + j <= 4 (the other entries are ignored)       */
} hbi_medium2d;

/* The tables tau^2, v0, v1 of hbi_tables (Sec. 4.1: values at every pair of
 * table nodes) computed from the medium, 2D: for every node as a point
 * source, the factored eikonal (eq. faceik) and the transport recurrence
 * (eq. equVs) for v0 and v1 on a grid of spacing h0 aligned with the node and
 * covering the table region plus `margin` points on every side, by
 * Lax-Friedrichs sweeping with fifth-order WENO derivatives (epsilon h0^2),
 * Gauss-Seidel in the four orderings until the largest update of a round is
 * below 1e-13, the unknowns held at their Taylor expansions (Sec. 2.2,
 * truncation 6, 4, 2) within 5, 3 and 1 grid points of the node; then the 4 x 4 Lagrange cubic of the grid
 * values at every other node.  The tables are symmetrised ((F + F^T) / 2)
 * and written to the host arrays tau2, v0, v1 (NT x NT row-major, layout of
 * hbi_tables).  The medium grid must cover every source grid with 3 more
 * points (n^2 is interpolated by local quintics); nI 2..16, nbox >= 1,
 * h0 > 0, margin >= 4 (HBI_ERR_ARG otherwise).  HBI_ERR_NUMERIC when a solve
 * does not converge (the sweeps stop after 20000 rounds).  Needs a context
 * for its device and stream only (tables and factors are untouched).
 * Synchronous. */
hbi_status hbi_tabulate(hbi_ctx *ctx, const hbi_medium2d *m, int32_t nI, const int32_t nbox[2],
                        const double box_origin[2], double box_size, double h0, int32_t margin,
                        double *tau2, double *v0, double *v1);

/* Bytes of the fixed per-device scratch array of hbi_apply_noalloc. */
#define HBI_NOALLOC_SCRATCH_BYTES (128u << 20)

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * product as hbi_apply, u = K (h^d s) for nrhs right-hand sides (same
 * layout rules; the right-hand sides are applied one after another with the
 * single-RHS kernels), with the per-level vectors z in a fixed scratch
 * array of HBI_NOALLOC_SCRATCH_BYTES bytes that the library holds on every
 * device it runs on until the process ends, instead of memory the library
 * allocates.  Nothing is allocated or freed, and no per-kernel timing is
 * recorded.  The scratch needed, "apply_scratch_bytes" of hbi_get_info,
 * must fit that array (HBI_ERR_ARG otherwise, with the sizes in the
 * message); contexts with a curve inclusion are rejected (HBI_ERR_ARG).
 * Every call on a device shares that device's array and leaves its
 * contents behind (no part of it needs to start at zero: a product writes
 * every entry it reads first), so calls that overlap in time on one device
 * (several streams, several threads) race and must be serialised by the
 * caller.  Asynchronous on the context's stream. */
hbi_status hbi_apply_noalloc(hbi_ctx *ctx, const void *s, void *u, int32_t nrhs, int64_t ld);

/* hb_entry on its own: out[i + m*j] = K[rows[i], cols[j]] (natural cell
 * indices, host int32 arrays) as complex128 into the device array `out`
 * (column-major m x n), including the self term where rows[i] == cols[j].
 * Needs loaded tables.  Synchronous. */
hbi_status hbi_entries(hbi_ctx *ctx, const int32_t *rows, int32_t m,
                       const int32_t *cols, int32_t n, void *out);

/* Per-kernel timing of applies.  While enabled (enable != 0), every
 * hbi_apply / hbi_apply_adjoint records a HIP event pair on the context's
 * stream around each of its kernel launches.  Used to report achieved
 * bandwidth against the HBM roofline; costs a few microseconds per launch. */
hbi_status hbi_set_profiling(hbi_ctx *ctx, int32_t enable);

/* Synchronise the context's stream and write JSON
 * {"kernels": {name: {"launches": n, "ms": total, "bytes": total}}} for
 * the launches recorded since profiling was enabled (bytes are the
 * algorithmic HBM bytes of each launch: factor entries streamed, vector
 * entries read and written, descriptors), then clear the record. */
hbi_status hbi_get_profile(hbi_ctx *ctx, char *json, int64_t cap);

/* JSON description of the context into json[0..cap): sizes, ranks, stored
 * factor entries and bytes, build timings.  Fails with HBI_ERR_ARG when cap
 * is too small. */
hbi_status hbi_get_info(const hbi_ctx *ctx, char *json, int64_t cap);

/* Text of the last error on ctx (or of the last context-free error when ctx
 * is NULL).  Valid until the next call on the same context. */
const char *hbi_last_error(const hbi_ctx *ctx);

#ifdef __cplusplus
}
#endif
#endif /* HBI_H */
