// HIP kernels of the HB integrator build for gfx950 (wave64).
//
//   hb_entry  k_cell_setup, k_self_terms, k_colside, k_colside_cells,
//             k_entries
//   bf_build  k_id_onchip, k_cpqr, k_cpqr_blocked (column-pivoted Householder
//             QR + interpolation matrix), k_pack_pairs,
//             k_place_blocks
// The apply kernels are in hbi_apply.hip, the multi-RHS ones in hbi_multi.hip.
#include "hbi_kernels.h"
#include "hbi_device.h"
#include "hbi_hankel.h"

namespace hbi {

// ---------------------------------------------------------------------------
// Per-cell setup: centre, table box and 1D barycentric Lagrange weights.
// ---------------------------------------------------------------------------
__global__ void k_cell_setup(DevProblem P, const int32_t *perm, int64_t Nv,
                             int32_t ncx, int32_t ncy, double ox, double oy,
                             double oz, double *xyz, double *lw, int32_t *box) {
  const int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (p >= Nv) return;
  const int64_t nat = perm[p];
  const int64_t ix = nat % ncx, iy = (nat / ncx) % ncy, iz = nat / ((int64_t)ncx * ncy);
  double c[3];
  c[0] = ox + (ix + 0.5) * P.h;
  c[1] = oy + (iy + 0.5) * P.h;
  c[2] = P.dim == 3 ? oz + (iz + 0.5) * P.h : 0.0;
  for (int ax = 0; ax < 3; ++ax) xyz[p * 3 + ax] = c[ax];
  box[p] = box_weights(P, c, lw + p * P.dim * P.nI);
}

// ---------------------------------------------------------------------------
// Self terms K_ii = h^-d x (cell integral of the leading HB term), Appendix A.
// 2D: (i/4) (n w)^-2 [8 int_0^{pi/4} X H1(X) dtheta + 4i] / h^2,
//     X = h n w / (2 cos theta).
// 3D: i Q_s / (4 pi w^2 n^2 h^3), Q_s = -48i int_0^{pi/4} dphi int_0^1 drho'
//     [e^{i r1}(1 - i r1) - 1] rho / (1 + rho^2)^{3/2} / cos phi,
//     rho = rho'/cos phi, r1 = w n (h/2) sqrt(1 + rho^2).
// Both integrands are smooth; Gauss-Legendre with `ng` nodes (gx, gw on
// [0,1]) converges to machine precision.
// ---------------------------------------------------------------------------
__global__ void k_self_terms(DevProblem P, const double *slow, int64_t Nv,
                             const double *gx, const double *gw, int ng,
                             double2 *self) {
  const int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (p >= Nv) return;
  const double n = slow[p], w = P.omega, h = P.h;
  double2 out;
  if (P.dim == 2) {
    const double a = 0.5 * h * n * w;
    double sr = 0.0, si = 0.0;
    for (int q = 0; q < ng; ++q) {
      const double th = 0.25 * kPi * gx[q];
      const double X = a / cos(th);
      const Hankel01 H = hankel01(X);
      sr += gw[q] * X * H.j1;
      si += gw[q] * X * H.y1;
    }
    sr *= 0.25 * kPi;
    si *= 0.25 * kPi;
    // (i/4)(8 s + 4i) = 2 i s - 1
    const double sc = 1.0 / ((n * w) * (n * w) * h * h);
    out.x = (-2.0 * si - 1.0) * sc;
    out.y = (2.0 * sr) * sc;
  } else {
    double qr = 0.0, qi = 0.0;
    for (int a = 0; a < ng; ++a) {
      const double phi = 0.25 * kPi * gx[a];
      const double cph = cos(phi);
      double ir = 0.0, ii = 0.0;
      for (int b = 0; b < ng; ++b) {
        const double rho = gx[b] / cph;
        const double s2 = 1.0 + rho * rho;
        const double r1 = w * n * 0.5 * h * sqrt(s2);
        double sn, cs;
        sincos(r1, &sn, &cs);
        // e^{i r1}(1 - i r1) - 1
        const double er = cs + r1 * sn - 1.0;
        const double ei = sn - r1 * cs;
        const double g = rho / (s2 * sqrt(s2)) / cph;
        ir += gw[b] * er * g;
        ii += gw[b] * ei * g;
      }
      qr += gw[a] * ir;
      qi += gw[a] * ii;
    }
    qr *= 0.25 * kPi;
    qi *= 0.25 * kPi;
    // Q_s = -48 i (qr + i qi) = 48 qi - 48 i qr ; I = i Q_s / (4 pi w^2 n^2)
    const double Qr = 48.0 * qi, Qi = -48.0 * qr;
    const double sc = 1.0 / (4.0 * kPi * w * w * n * n * h * h * h);
    out.x = -Qi * sc;
    out.y = Qr * sc;
  }
  self[p] = out;
}

// ---------------------------------------------------------------------------
// hb_entry, column side of eq. chebinterpblock: for a source cell in table
// box beta and a row box alpha,
//   Hc[t][a] = sum_b F_t[alpha*NTb + a, beta*NTb + b] T_b(r_j).
// One wave per (source cell, row box); lanes run over a, reading the
// transposed table so that the loads are contiguous.  k_colside does this
// per (block, column, row-box slot) into the batch workspace; k_colside_cells
// fills a cache for every (cell, box) pair once per build when it fits in
// memory, which the entry kernel then reads instead.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void colside_item(const DevProblem &P, const DevCells &C,
                                             const DevTables &T, int32_t cp, int beta, int alpha,
                                             double *out, double *sT) {
  const int nI = P.nI, NTb = P.NTb, NT = P.NT, D = P.dim;
  const double *lwc = C.lw + (int64_t)cp * D * nI;
  for (int b = threadIdx.x; b < NTb; b += 64) {
    int r = b;
    double v = 1.0;
    for (int ax = 0; ax < D; ++ax) {
      v *= lwc[ax * nI + r % nI];
      r /= nI;
    }
    sT[b] = v;
  }
  __syncthreads();
  const int ntab = P.nterms == 2 ? 3 : 2;
  for (int a = threadIdx.x; a < NTb; a += 64) {
    const int64_t col = (int64_t)alpha * NTb + a;
    double acc[3] = {0.0, 0.0, 0.0};
    for (int b = 0; b < NTb; ++b) {
      const double tb = sT[b];
      const int64_t rowB = ((int64_t)beta * NTb + b) * NT + col;
      acc[0] = fma(tb, T.FT[0][rowB], acc[0]);
      acc[1] = fma(tb, T.FT[1][rowB], acc[1]);
      if (ntab == 3) acc[2] = fma(tb, T.FT[2][rowB], acc[2]);
    }
    out[a] = acc[0];
    out[NTb + a] = acc[1];
    out[2 * NTb + a] = acc[2];
  }
}

__global__ __launch_bounds__(64) void k_colside(
    DevProblem P, DevCells C, DevTables T, const EntryBlock *blks,
    const int32_t *work, int64_t nwork, const int32_t *cols,
    const int32_t *slotbox, double *Hc) {
  extern __shared__ double sT[];
  const int64_t w = blockIdx.x;
  if (w >= nwork) return;
  const int blk = work[2 * w], js = work[2 * w + 1];
  const EntryBlock B = blks[blk];
  const int j = js / B.nslot, slot = js % B.nslot;
  const int32_t cp = cols[B.col_off + j];
  double *out = Hc + B.hc_off + ((int64_t)j * B.nslot + slot) * 3 * P.NTb;
  colside_item(P, C, T, cp, C.box[cp], slotbox[B.slot_off + slot], out, sT);
}

// Cache entry (cell p, box alpha) at Hcache[(p * nbox + alpha) * 3 NTb].
__global__ __launch_bounds__(64) void k_colside_cells(DevProblem P, DevCells C, DevTables T,
                                                      int64_t Nv, int nbox, double *Hcache) {
  extern __shared__ double sT[];
  const int64_t w = blockIdx.x;
  if (w >= Nv * nbox) return;
  const int32_t p = (int32_t)(w / nbox);
  const int alpha = (int)(w % nbox);
  colside_item(P, C, T, p, C.box[p], alpha, Hcache + w * 3 * P.NTb, sT);
}

// HB entry from interpolated tau^2, v0, v1 (eq. babich, eq. termf).
__device__ __forceinline__ double2 hb_value(int D, int nterms, double omega,
                                            double tau2, double v0, double v1) {
  const double tau = sqrt(fmax(tau2, 0.0));
  const double x = omega * tau;
  double2 K;
  if (D == 2) {
    // f0 = i sqrt(pi)/2 H0 = (sqrt(pi)/2)(-Y0 + i J0)
    // f1 = -i sqrt(pi) (tau/omega) H1 = sqrt(pi)(tau/omega)(Y1 - i J1)
    const Hankel01 H = hankel01(x);
    const double c0 = 0.88622692545275801365 * v0;   // sqrt(pi)/2
    K.x = -c0 * H.y0;
    K.y = c0 * H.j0;
    if (nterms == 2) {
      const double c1 = 1.77245385090551602730 * (tau / omega) * v1;
      K.x += c1 * H.y1;
      K.y -= c1 * H.j1;
    }
  } else {
    // e^{i x} (v0/(2 tau) + i v1/omega)
    double sn, cs;
    sincos(x, &sn, &cs);
    const double A = v0 / (2.0 * tau);
    const double B = nterms == 2 ? v1 / omega : 0.0;
    K.x = cs * A - sn * B;
    K.y = sn * A + cs * B;
  }
  return K;
}

// ---------------------------------------------------------------------------
// hb_entry, row side of eq. chebinterpblock as a tiled product: for a tile of
// up to kET_I rows (all in one table box) and kET_J columns of a block,
//   g_t(i, j) = sum_A T_A(r_i) Hc_t(j, box)[A],   T_A = prod_s l_{a_s}(r_i),
// for t = tau^2, v0, v1.  T and Hc pass through LDS in chunks of kET_K nodes;
// each thread keeps a 4 x 2 x 3 register tile.  Then the HB value of
// (tau^2, v0, v1) (eq. babich, eq. termf), or the self term on the diagonal,
// goes to out(i, j).  Rows are visited in slot order through `rord`.
// In 2D the Hankel pair H0, H1 of x = omega tau takes one of three branches
// (series, Miller recurrence, asymptotic expansion); the tile's entries are
// first sorted by branch through LDS so that every wave runs one branch at a
// time over full lanes, then written out in place.
// ---------------------------------------------------------------------------
constexpr int kET_I = 128, kET_K = 32;
// tile columns: 16 in 2D (entries are Hankel-heavy; the branch sort needs
// the tile in LDS), 32 in 3D (entries are contraction-heavy)
constexpr int et_cols(int D) { return D == 3 ? 32 : 16; }

// HB value from the Hankel pair: (sqrt(pi)/2) v0 i H0 - sqrt(pi) (tau/omega) v1 i H1
__device__ __forceinline__ double2 hb2d(const Hankel01 &H, double c0, double c1) {
  return double2{-c0 * H.y0 + c1 * H.y1, c0 * H.j0 - c1 * H.j1};
}

template <int D, int NI>
__global__ __launch_bounds__(256, 2) void k_entries(
    DevProblem P, DevCells C, const EntryBlock *blks, const ETile *tiles, int64_t ntiles,
    const int32_t *rows, const int32_t *rord, const int32_t *cols, const double *Hc,
    const int32_t *slotbox, const double *Hcache, int nbox) {
  // contraction staging (sW: kET_K x kET_I, sH: 3 x kET_K x kET_J), reused by
  // the 2D epilogue as x, c0, c1 per entry plus the branch-sorted entry list
  constexpr int kET_J = et_cols(D), CJ = kET_J / 8, kET_N = kET_I * kET_J;
  constexpr int kStage = kET_K * kET_I + 3 * kET_K * kET_J;
  constexpr int kEpi = D == 2 ? 3 * kET_N + kET_N / 4 : 0;
  __shared__ double smem[kStage > kEpi ? kStage : kEpi];
  __shared__ int32_t srp[kET_I];
  __shared__ const double *shp[kET_J];
  __shared__ int32_t cls_cnt[4][3];
  double(*sW)[kET_I] = (double(*)[kET_I])smem;
  double(*sH)[kET_K][kET_J] = (double(*)[kET_K][kET_J])(smem + kET_K * kET_I);
  const int64_t tb = blockIdx.x;
  if (tb >= ntiles) return;
  const ETile T = tiles[tb];
  const EntryBlock B = blks[T.blk];
  const int NTb = P.NTb;
  const int ntab = P.nterms == 2 ? 3 : 2;
  const int tid = threadIdx.x;
  const int box = slotbox[B.slot_off + T.slot];
  for (int r = tid; r < kET_I; r += 256)
    srp[r] = r < T.nr ? rows[B.row_off + rord[B.row_off + T.r0 + r]] : -1;
  for (int c = tid; c < kET_J; c += 256) {
    const double *h = nullptr;
    if (c < T.nj) {
      const int j = T.j0 + c;
      h = Hcache ? Hcache + ((int64_t)cols[B.col_off + j] * nbox + box) * 3 * NTb
                 : Hc + B.hc_off + ((int64_t)j * B.nslot + T.slot) * 3 * NTb;
    }
    shp[c] = h;
  }
  __syncthreads();
  const int ty = tid >> 3, tx = tid & 7;
  double acc[4][CJ][3];
#pragma unroll
  for (int r = 0; r < 4; ++r)
#pragma unroll
    for (int c = 0; c < CJ; ++c)
#pragma unroll
      for (int t = 0; t < 3; ++t) acc[r][c][t] = 0.0;
  for (int a0 = 0; a0 < NTb; a0 += kET_K) {
    for (int e = tid; e < kET_K * kET_I; e += 256) {
      const int k = e / kET_I, r = e % kET_I;
      const int A = a0 + k, rp = srp[r];
      double w = 0.0;
      if (rp >= 0 && A < NTb) {
        const double *lw = C.lw + (int64_t)rp * D * NI;
        const int a1 = A % NI, a23 = A / NI;
        w = lw[a1] * lw[NI + a23 % NI];
        if (D == 3) w *= lw[2 * NI + a23 / NI];
      }
      sW[k][r] = w;
    }
    for (int e = tid; e < 3 * kET_K * kET_J; e += 256) {
      const int k = e % kET_K, cr = e / kET_K, c = cr % kET_J, t = cr / kET_J;
      const double *h = shp[c];
      const int A = a0 + k;
      sH[t][k][c] = (h && A < NTb && t < ntab) ? h[(int64_t)t * NTb + A] : 0.0;
    }
    __syncthreads();
#pragma unroll 4
    for (int k = 0; k < kET_K; ++k) {
      double w[4], h[3][CJ];
#pragma unroll
      for (int r = 0; r < 4; ++r) w[r] = sW[k][ty * 4 + r];
#pragma unroll
      for (int t = 0; t < 3; ++t)
#pragma unroll
        for (int c = 0; c < CJ; ++c) h[t][c] = sH[t][k][tx * CJ + c];
#pragma unroll
      for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int c = 0; c < CJ; ++c)
#pragma unroll
          for (int t = 0; t < 3; ++t) acc[r][c][t] = fma(w[r], h[t][c], acc[r][c][t]);
    }
    __syncthreads();
  }
  if constexpr (D == 3) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int rr = ty * 4 + r;
      if (rr >= T.nr) continue;
      const int i = rord[B.row_off + T.r0 + rr];
      const int32_t rp = srp[rr];
#pragma unroll
      for (int c = 0; c < CJ; ++c) {
        const int cc = tx * CJ + c;
        if (cc >= T.nj) continue;
        const int j = T.j0 + cc;
        const int32_t cp = cols[B.col_off + j];
        const int32_t si = self_index(C, rp, cp);
        const double2 K = si >= 0 ? C.self[si]
                                  : hb_value(D, P.nterms, P.omega, acc[r][c][0], acc[r][c][1],
                                             acc[r][c][2]);
        B.out[i + (int64_t)j * B.m] = K;
      }
    }
    return;
  } else {
  // ---- 2D: x, c0, c1 per entry (entry e = rr * kET_J + cc), branch 0..2 or
  // 3 (value already final: self term) or -1 (outside the tile)
  double *ex = smem, *ec0 = smem + kET_N, *ec1 = smem + 2 * kET_N;
  uint16_t *elist = (uint16_t *)(smem + 3 * kET_N);
  const int lane = tid & 63, wave = tid >> 6;
  int cls[4][2];
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int rr = ty * 4 + r;
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      const int cc = tx * 2 + c;
      const int e = rr * kET_J + cc;
      cls[r][c] = -1;
      if (rr < T.nr && cc < T.nj) {
        const int32_t rp = srp[rr];
        const int32_t cp = cols[B.col_off + T.j0 + cc];
        const int32_t si = self_index(C, rp, cp);
        if (si >= 0) {
          const double2 sf = C.self[si];
          ec0[e] = sf.x;
          ec1[e] = sf.y;
          cls[r][c] = 3;
        } else {
          const double tau = sqrt(fmax(acc[r][c][0], 0.0));
          const double x = P.omega * tau;
          ex[e] = x;
          ec0[e] = 0.88622692545275801365 * acc[r][c][1];   // sqrt(pi)/2 v0
          ec1[e] = P.nterms == 2 ? 1.77245385090551602730 * (tau / P.omega) * acc[r][c][2] : 0.0;
          cls[r][c] = x < 3.0 ? 0 : (x < 20.0 ? 1 : 2);
        }
      }
    }
  }
  // branch-sorted list: per-wave counts by ballot, then positions
  int cnt[3] = {0, 0, 0};
#pragma unroll
  for (int r = 0; r < 4; ++r)
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
      for (int q = 0; q < 3; ++q) cnt[q] += __popcll(__ballot(cls[r][c] == q));
  if (lane == 0)
    for (int q = 0; q < 3; ++q) cls_cnt[wave][q] = cnt[q];
  __syncthreads();
  int base[3], tot[3];
  {
    int run = 0;
    for (int q = 0; q < 3; ++q) {
      int before = 0, all = 0;
      for (int w2 = 0; w2 < 4; ++w2) {
        if (w2 < wave) before += cls_cnt[w2][q];
        all += cls_cnt[w2][q];
      }
      base[q] = run + before;
      tot[q] = all;
      run += all;
    }
  }
  const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
#pragma unroll
  for (int r = 0; r < 4; ++r)
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
      for (int q = 0; q < 3; ++q) {
        const uint64_t mk = __ballot(cls[r][c] == q);
        if (cls[r][c] == q)
          elist[base[q] + __popcll(mk & below)] = (uint16_t)((ty * 4 + r) * kET_J + tx * 2 + c);
        base[q] += __popcll(mk);
      }
  __syncthreads();
  // one branch at a time over full lanes; results overwrite c0, c1
  {
    int off = 0;
    for (int q = 0; q < 3; ++q) {
      for (int t = tid; t < tot[q]; t += 256) {
        const int e = elist[off + t];
        const double x = ex[e];
        const Hankel01 H = q == 0 ? hankel01_series(x)
                                  : (q == 1 ? hankel01_miller(x) : hankel01_asym(x));
        const double2 K = hb2d(H, ec0[e], ec1[e]);
        ec0[e] = K.x;
        ec1[e] = K.y;
      }
      off += tot[q];
    }
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int rr = ty * 4 + r;
    if (rr >= T.nr) continue;
    const int i = rord[B.row_off + T.r0 + rr];
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      const int cc = tx * 2 + c;
      if (cc >= T.nj) continue;
      const int e = rr * kET_J + cc;
      B.out[i + (int64_t)(T.j0 + cc) * B.m] = double2{ec0[e], ec1[e]};
    }
  }
  }
}

// ---------------------------------------------------------------------------
// Interpolative decomposition of one block (eq. ID): Householder QR with
// column pivoting on the largest remaining column norm (ties: first in
// pivot order), stopped at the first k with |R_kk| <= tol |R_11|; rank
// r = k (at least 1).  Then X = [I, R11^-1 R12] Pi^T (r x n) so that
// A ~ A(:, skel) X.  Column norms are recomputed exactly from the updated
// entries at every step.
//
// One 1024-thread workgroup (16 waves) per block; the block stays in global
// memory and the waves split the trailing columns.  Each step: thread 0
// picks the pivot from the waves' candidates and forms the reflector
// H = I - tau v v^H (beta, tau and the scale of x below the diagonal); the
// workgroup writes v into LDS; each wave applies H^H to its columns
// (w = v^H a, a -= conj(tau) w v) and reports its best next pivot.  Rows
// [k, k + 64 kCpqrRPL) of a column stay in registers between the dot product
// and the update, so they are read once; rows past that are streamed twice
// with kCpqrCH loads in flight per lane.  After the last step the top r rows
// of R (pivoted order) are staged in LDS and R11^-1 R12 is solved there by
// back substitution, one column per thread.
//
// LDS: norms (8 B per column) and column map (4 B per column), then a region
// of `cap` complex entries that holds v during the factorisation and R's top
// rows during the solve.  A block whose m (or r n) exceeds `cap` uses the
// global-memory forms of those two parts instead.
// ---------------------------------------------------------------------------
constexpr int kCpqrRPL = 8;
constexpr int kCpqrCH = 2;

// Reflector entries read from LDS, or formed from the pivot column.
struct ReflLds {
  const double2 *v;
  __device__ __forceinline__ double2 operator()(int i) const { return v[i]; }
};
struct ReflGlobal {
  const double2 *x;
  double2 scale;
  int k;
  __device__ __forceinline__ double2 operator()(int i) const {
    return i == k ? double2{1.0, 0.0} : cmul(x[i], scale);
  }
};

// Apply H^H to column a (rows [k, m)) by one wave; returns the new squared
// norm of a below row k.
template <class Refl>
__device__ __forceinline__ double apply_reflector(double2 *a, const Refl &v, int k, int m,
                                                  int lane, double2 ctau) {
  double2 seg[kCpqrRPL];
  double2 wv = double2{0.0, 0.0};
#pragma unroll
  for (int t = 0; t < kCpqrRPL; ++t) {
    const int i = k + lane + 64 * t;
    seg[t] = i < m ? a[i] : double2{0.0, 0.0};
  }
#pragma unroll
  for (int t = 0; t < kCpqrRPL; ++t) {
    const int i = k + lane + 64 * t;
    if (i < m) cfmac(wv, v(i), seg[t]);
  }
  const int kr = k + 64 * kCpqrRPL;
  for (int b = kr; b < m; b += 64 * kCpqrCH) {
    double2 t2[kCpqrCH];
#pragma unroll
    for (int u = 0; u < kCpqrCH; ++u) {
      const int i = b + lane + 64 * u;
      t2[u] = i < m ? a[i] : double2{0.0, 0.0};
    }
#pragma unroll
    for (int u = 0; u < kCpqrCH; ++u) {
      const int i = b + lane + 64 * u;
      if (i < m) cfmac(wv, v(i), t2[u]);
    }
  }
  wv.x = wave_sum(wv.x);
  wv.y = wave_sum(wv.y);
  const double2 f = cmul(ctau, wv);
  double s = 0.0;
#pragma unroll
  for (int t = 0; t < kCpqrRPL; ++t) {
    const int i = k + lane + 64 * t;
    if (i < m) {
      const double2 vi = v(i);
      double2 ai = seg[t];
      ai.x -= f.x * vi.x - f.y * vi.y;
      ai.y -= f.x * vi.y + f.y * vi.x;
      a[i] = ai;
      if (i > k) s += ai.x * ai.x + ai.y * ai.y;
    }
  }
  for (int b = kr; b < m; b += 64 * kCpqrCH) {
    double2 t2[kCpqrCH];
#pragma unroll
    for (int u = 0; u < kCpqrCH; ++u) {
      const int i = b + lane + 64 * u;
      t2[u] = i < m ? a[i] : double2{0.0, 0.0};
    }
#pragma unroll
    for (int u = 0; u < kCpqrCH; ++u) {
      const int i = b + lane + 64 * u;
      if (i < m) {
        const double2 vi = v(i);
        double2 ai = t2[u];
        ai.x -= f.x * vi.x - f.y * vi.y;
        ai.y -= f.x * vi.y + f.y * vi.x;
        a[i] = ai;
        s += ai.x * ai.x + ai.y * ai.y;
      }
    }
  }
  return wave_sum(s);
}

// Back substitution x <- R11^-1 x for one column (x holds R12's column on
// entry); R(i, l) at R[i + l * ldr].  A zero or singular diagonal gives 0.
template <class RAt>
__device__ __forceinline__ void solve_upper(const RAt &R, double2 *x, int r, bool zero) {
  for (int i = r - 1; i >= 0; --i) {
    double2 acc = x[i];
    for (int l = i + 1; l < r; ++l) {
      const double2 ril = R(i, l);
      const double2 xl = x[l];
      acc.x -= ril.x * xl.x - ril.y * xl.y;
      acc.y -= ril.x * xl.y + ril.y * xl.x;
    }
    const double2 d = R(i, i);
    const double dd = d.x * d.x + d.y * d.y;
    x[i] = (zero || dd == 0.0)
               ? double2{0.0, 0.0}
               : double2{(acc.x * d.x + acc.y * d.y) / dd, (acc.y * d.x - acc.x * d.y) / dd};
  }
}

__global__ __launch_bounds__(HBI_ID_THREADS) void k_cpqr(const IdBlock *blks, const int32_t *sel,
                                                          double tol, int32_t *rank_out, int nmax,
                                                          int cap) {
  extern __shared__ double lds_id[];
  constexpr int NW = HBI_ID_THREADS / 64;
  __shared__ double red_v[NW];
  __shared__ int red_i[NW];
  __shared__ double2 sh_tau, sh_scale;
  __shared__ int sh_stop, sh_rank, sh_c;
  __shared__ double sh_r11;

  const int blk = sel[blockIdx.x];
  const IdBlock B = blks[blk];
  const int m = B.m, n = B.n;
  double *nrm2 = lds_id;
  int *colmap = (int *)(lds_id + nmax);
  double2 *shared_c = (double2 *)(lds_id + ((nmax + (nmax + 1) / 2 + 2) & ~1));
  const bool vlds = m <= cap;
  double2 *A = B.A;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;

  // initial norms; each wave also tracks its best candidate
  double bv = -1.0;
  int bq = n;
  for (int j = wave; j < n; j += NW) {
    const double2 *a = A + (int64_t)j * m;
    double s = 0.0;
    for (int b = 0; b < m; b += 64 * kCpqrCH) {
      double2 t2[kCpqrCH];
#pragma unroll
      for (int u = 0; u < kCpqrCH; ++u) {
        const int i = b + lane + 64 * u;
        t2[u] = i < m ? a[i] : double2{0.0, 0.0};
      }
#pragma unroll
      for (int u = 0; u < kCpqrCH; ++u) s += t2[u].x * t2[u].x + t2[u].y * t2[u].y;
    }
    s = wave_sum(s);
    if (lane == 0) nrm2[j] = s;
    if (s > bv) { bv = s; bq = j; }
  }
  if (lane == 0) { red_v[wave] = bv; red_i[wave] = bq; }
  for (int j = tid; j < n; j += HBI_ID_THREADS) colmap[j] = j;
  if (tid == 0) { sh_rank = m < n ? m : n; sh_r11 = 0.0; }
  __syncthreads();

  const int kmax = m < n ? m : n;
  for (int k = 0; k < kmax; ++k) {
    if (tid == 0) {
      double v = red_v[0];
      int q = red_i[0];
      for (int w2 = 1; w2 < NW; ++w2)
        if (red_v[w2] > v || (red_v[w2] == v && red_i[w2] < q)) { v = red_v[w2]; q = red_i[w2]; }
      const double nrm = sqrt(fmax(v, 0.0));
      if (k == 0) sh_r11 = nrm;
      const int stop = (q >= n) || (nrm == 0.0) || (k > 0 && nrm <= tol * sh_r11);
      sh_stop = stop;
      if (stop) {
        sh_rank = k > 0 ? k : 1;
      } else {
        const int t = colmap[k];
        colmap[k] = colmap[q];
        colmap[q] = t;
        const int c = colmap[k];
        double2 *ac = A + (int64_t)c * m;
        const double2 al = ac[k];
        const double beta = al.x >= 0.0 ? -nrm : nrm;
        // H = I - tau v v^H with v = (1, x_{k+1:}/(alpha - beta)), H^H x = beta e_k
        sh_tau = double2{(beta - al.x) / beta, -al.y / beta};
        const double dr = al.x - beta, di = al.y;
        const double dd = dr * dr + di * di;
        sh_scale = double2{dr / dd, -di / dd};
        ac[k] = double2{beta, 0.0};
        sh_c = c;
      }
    }
    __syncthreads();
    if (sh_stop) break;
    const double2 *x = A + (int64_t)sh_c * m;
    const double2 scale = sh_scale;
    const double2 ctau = double2{sh_tau.x, -sh_tau.y};
    bv = -1.0;
    bq = n;
    if (vlds) {
      for (int i = k + tid; i < m; i += HBI_ID_THREADS)
        shared_c[i] = (i == k) ? double2{1.0, 0.0} : cmul(x[i], scale);
      __syncthreads();
      const ReflLds v{shared_c};
      for (int q = k + 1 + wave; q < n; q += NW) {
        const int j = colmap[q];
        const double s = apply_reflector(A + (int64_t)j * m, v, k, m, lane, ctau);
        if (lane == 0) nrm2[j] = s;
        if (s > bv) { bv = s; bq = q; }
      }
    } else {
      const ReflGlobal v{x, scale, k};
      for (int q = k + 1 + wave; q < n; q += NW) {
        const int j = colmap[q];
        const double s = apply_reflector(A + (int64_t)j * m, v, k, m, lane, ctau);
        if (lane == 0) nrm2[j] = s;
        if (s > bv) { bv = s; bq = q; }
      }
    }
    if (lane == 0) { red_v[wave] = bv; red_i[wave] = bq; }
    __syncthreads();
  }

  const int r = sh_rank;
  const bool zero = !(sh_r11 > 0.0);
  double2 *X = B.X;
  for (int idx = tid; idx < r * r; idx += HBI_ID_THREADS) {
    const int q = idx / r, i = idx % r;
    X[i + (int64_t)colmap[q] * r] = double2{i == q ? 1.0 : 0.0, 0.0};
  }
  for (int q = tid; q < r; q += HBI_ID_THREADS) B.piv[q] = colmap[q];
  if ((int64_t)r * n <= cap) {
    // top r rows of R in pivoted column order, column q at shared_c[q r]
    for (int idx = tid; idx < r * n; idx += HBI_ID_THREADS) {
      const int q = idx / r, i = idx % r;
      shared_c[idx] = A[i + (int64_t)colmap[q] * m];
    }
    __syncthreads();
    const double2 *Rs = shared_c;
    auto R = [Rs, r](int i, int l) { return Rs[i + l * r]; };
    for (int q = r + tid; q < n; q += HBI_ID_THREADS) solve_upper(R, shared_c + q * r, r, zero);
    __syncthreads();
    for (int idx = tid; idx < r * (n - r); idx += HBI_ID_THREADS) {
      const int q = r + idx / r, i = idx % r;
      X[i + (int64_t)colmap[q] * r] = shared_c[i + q * r];
    }
  } else {
    // in global memory: R12's column is copied into X's and solved there
    auto R = [A, colmap, m](int i, int l) { return A[i + (int64_t)colmap[l] * m]; };
    for (int q = r + tid; q < n; q += HBI_ID_THREADS) {
      const int col = colmap[q];
      double2 *xo = X + (int64_t)col * r;
      for (int i = 0; i < r; ++i) xo[i] = A[i + (int64_t)col * m];
      solve_upper(R, xo, r, zero);
    }
  }
  if (tid == 0) rank_out[blk] = r;
}

// ---------------------------------------------------------------------------
// Interpolative decomposition of a block with at most NW NS columns, done on
// chip.  The pivoted QR of A (m x n) is taken as the pivoted QR of the n x n
// triangular factor R0 of an unpivoted Householder QR A = Q0 R0: Q0 has
// orthonormal columns, so every column norm, pivot choice and R factor of
// the pivoted QR is the same for A and for R0, and A is read once.
//   Phase 1 streams A in panels of 64 PR rows and folds each panel P into
//   R0 with Householder reflections of the stacked matrix [R0; P].
//   Phase 2 is the column-pivoted QR of R0 with the rule and stopping test
//   of k_cpqr (norms recomputed exactly at each step).
//   Phase 3 stages the top r rows of R in LDS (or, when r n exceeds `cap`,
//   in A's storage) and solves R11 T = R12 one column per thread.
// Layout: wave w owns columns c = w + NW s (s < NS); lane l holds rows
// l + 64 u of R0 (u < RR = NW NS / 64) and rows l + 64 t of the panel
// (t < PR).  Launched as 8 waves x 8 slots with 128-row panels (n <= 64):
// within 128 VGPRs, so two workgroups share a CU.
// ---------------------------------------------------------------------------
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ double dpp_add(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, ROW_MASK, 0xf, true);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, ROW_MASK, 0xf, true);
  return v + __longlong_as_double(((long long)(unsigned)lo) | ((long long)hi << 32));
}

__device__ __forceinline__ double readlane_d(double v, int l) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)b, l);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
  return __longlong_as_double(((long long)(unsigned)lo) | ((long long)hi << 32));
}

// Sum over the wave's 64 lanes, the same value in every lane: DPP row
// shifts by 1, 2, 4, 8 leave each row's sum in its lane 15; row broadcasts
// of lanes 15 and 31 then carry the total to lane 63, which is read out.
__device__ __forceinline__ double wave_sum_u(double v) {
  v = dpp_add<0x111, 0xf>(v);   // row_shr:1
  v = dpp_add<0x112, 0xf>(v);   // row_shr:2
  v = dpp_add<0x114, 0xf>(v);   // row_shr:4
  v = dpp_add<0x118, 0xf>(v);   // row_shr:8
  v = dpp_add<0x142, 0xa>(v);   // row_bcast:15 into rows 1 and 3
  v = dpp_add<0x143, 0xc>(v);   // row_bcast:31 into rows 2 and 3
  return readlane_d(v, 63);
}

// A value the whole wave holds alike (read from LDS), made wave-uniform so
// that branches on it are scalar.
__device__ __forceinline__ double uniform_d(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readfirstlane((int)b);
  const int hi = __builtin_amdgcn_readfirstlane((int)(b >> 32));
  return __longlong_as_double(((long long)(unsigned)lo) | ((long long)hi << 32));
}
__device__ __forceinline__ double2 uniform_c(double2 v) {
  return double2{uniform_d(v.x), uniform_d(v.y)};
}

__device__ __forceinline__ double2 readlane_c(double2 v, int l) {
  return double2{readlane_d(v.x, l), readlane_d(v.y, l)};
}

// Phase 1 of the on-chip decomposition: R0 (the triangular factor of an
// unpivoted Householder QR of the m x n block A, n <= NW NS) accumulated in
// registers (lane l holds rows l + 64 u of R0 for its wave's columns) by
// folding panels of 64 PR rows into [R0; P].  vsh holds two reflector
// buffers of VS entries, tsh two reflector scalars (LDS).
template <int NW, int NS, int PR, int VS>
__device__ __forceinline__ void tsqr_panels(const double2 *A, int m, int n, int w, int lane,
                                            double2 (&R)[NS * NW / 64][NS], double2 *vsh,
                                            double2 *tsh) {
  constexpr int RR = NS * NW / 64;
  const double2 zero2 = double2{0.0, 0.0};
#pragma unroll
  for (int u = 0; u < RR; ++u)
#pragma unroll
    for (int s = 0; s < NS; ++s) R[u][s] = zero2;
  int buf = 0;
  for (int p0 = 0; p0 < m; p0 += 64 * PR) {
    double2 P[PR][NS];
#pragma unroll
    for (int t = 0; t < PR; ++t)
#pragma unroll
      for (int s = 0; s < NS; ++s) {
        const int c = w + NW * s, i = p0 + lane + 64 * t;
        P[t][s] = (c < n && i < m) ? A[i + (int64_t)c * m] : zero2;
      }
    for (int j = 0; j < n; ++j) {
      const int sj = j / NW, uj = j >> 6, lj = j & 63;
      if (w == j % NW) {
        double2 x[PR], rj = zero2;
#pragma unroll
        for (int s = 0; s < NS; ++s)
          if (s == sj) {
#pragma unroll
            for (int t = 0; t < PR; ++t) x[t] = P[t][s];
#pragma unroll
            for (int u = 0; u < RR; ++u)
              if (u == uj) rj = R[u][s];
          }
        double xn = 0.0;
#pragma unroll
        for (int t = 0; t < PR; ++t) xn += x[t].x * x[t].x + x[t].y * x[t].y;
        xn = wave_sum_u(xn);
        const double2 al = readlane_c(rj, lj);
        double2 tau = zero2;
        if (xn != 0.0 || al.y != 0.0) {
          const double nrm = sqrt(al.x * al.x + al.y * al.y + xn);
          const double beta = al.x >= 0.0 ? -nrm : nrm;
          tau = double2{(beta - al.x) / beta, -al.y / beta};
          const double dr = al.x - beta, di = al.y, dd = dr * dr + di * di;
          const double2 scale = double2{dr / dd, -di / dd};
#pragma unroll
          for (int t = 0; t < PR; ++t) vsh[buf * VS + (lane + 64 * t)] = cmul(x[t], scale);
#pragma unroll
          for (int s = 0; s < NS; ++s)
            if (s == sj) {
#pragma unroll
              for (int t = 0; t < PR; ++t) P[t][s] = zero2;
#pragma unroll
              for (int u = 0; u < RR; ++u)
                if (u == uj && lane == lj) R[u][s] = double2{beta, 0.0};
            }
        }
        if (lane == 0) tsh[buf] = tau;
      }
      __syncthreads();
      const double2 tau = uniform_c(tsh[buf]);
      if (tau.x != 0.0 || tau.y != 0.0) {
        double2 v[PR];
#pragma unroll
        for (int t = 0; t < PR; ++t) v[t] = vsh[buf * VS + (lane + 64 * t)];
        const double2 ctau = double2{tau.x, -tau.y};
#pragma unroll
        for (int s = 0; s < NS; ++s) {
          const int c = w + NW * s;
          if (c > j && c < n) {
            double2 d = zero2;
#pragma unroll
            for (int t = 0; t < PR; ++t) cfmac(d, v[t], P[t][s]);
            d.x = wave_sum_u(d.x);
            d.y = wave_sum_u(d.y);
            double2 rl = R[0][s];
#pragma unroll
            for (int u = 1; u < RR; ++u)
              if (u == uj) rl = R[u][s];
            const double2 rjc = readlane_c(rl, lj);
            const double2 f = cmul(ctau, double2{rjc.x + d.x, rjc.y + d.y});
#pragma unroll
            for (int t = 0; t < PR; ++t) {
              P[t][s].x -= f.x * v[t].x - f.y * v[t].y;
              P[t][s].y -= f.x * v[t].y + f.y * v[t].x;
            }
#pragma unroll
            for (int u = 0; u < RR; ++u)
              if (u == uj && lane == lj) { R[u][s].x -= f.x; R[u][s].y -= f.y; }
          }
        }
      }
      buf ^= 1;
    }
  }

}

template <int NW, int NS, int PR, int WPE>
__global__ __launch_bounds__(NW * 64, WPE) void k_id_onchip(
    const IdBlock *blks, const int32_t *sel, double tol, int32_t *rank_out, int cap) {
  constexpr int NC = NS * NW;      // column capacity
  constexpr int RR = NC / 64;      // R0 rows per lane
  constexpr int T = NW * 64;
  static_assert(NC % 64 == 0, "column capacity must be a multiple of 64");
  extern __shared__ double2 lds_rs[];
  __shared__ double2 v_sh[2][NC > 64 * PR ? NC : 64 * PR];
  __shared__ double2 tau_sh[2];
  __shared__ int colmap[NC], pos[NC];
  __shared__ double red_v[NW];
  __shared__ int red_q[NW], red_c[NW];

  const int blk = sel[blockIdx.x];
  const IdBlock B = blks[blk];
  const int m = B.m, n = B.n;
  const int tid = threadIdx.x, lane = tid & 63;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);   // wave-uniform
  const double2 *A = B.A;
  const double2 zero2 = double2{0.0, 0.0};

  double2 R[RR][NS];
#pragma unroll
  for (int u = 0; u < RR; ++u)
#pragma unroll
    for (int s = 0; s < NS; ++s) R[u][s] = zero2;

  // ---- phase 1: R0 of A, one panel of 64 PR rows at a time
  constexpr int VS = NC > 64 * PR ? NC : 64 * PR;
  tsqr_panels<NW, NS, PR, VS>(A, m, n, w, lane, R, &v_sh[0][0], tau_sh);
  int buf = 0;

  // ---- phase 2: column-pivoted QR of R0
  for (int c = tid; c < NC; c += T) { colmap[c] = c; pos[c] = c; }
  {
    double bv = -1.0;
    int bq = n, bc = -1;
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      const int c = w + NW * s;
      if (c < n) {
        double sn = 0.0;
#pragma unroll
        for (int u = 0; u < RR; ++u) sn += R[u][s].x * R[u][s].x + R[u][s].y * R[u][s].y;
        sn = wave_sum_u(sn);
        if (sn > bv || (sn == bv && c < bq)) { bv = sn; bq = c; bc = c; }
      }
    }
    if (lane == 0) { red_v[w] = bv; red_q[w] = bq; red_c[w] = bc; }
  }
  __syncthreads();
  const int kmax = m < n ? m : n;
  int rank = kmax;
  double r11 = 0.0;
  // single-exit loop (a break would make the compiler copy R at the exit)
  bool go = kmax > 0;
  for (int k = 0; go; ++k) {
    double best = uniform_d(red_v[0]);
    int q = __builtin_amdgcn_readfirstlane(red_q[0]), p = __builtin_amdgcn_readfirstlane(red_c[0]);
    for (int w2 = 1; w2 < NW; ++w2) {
      const double bw = uniform_d(red_v[w2]);
      const int qw = __builtin_amdgcn_readfirstlane(red_q[w2]);
      if (bw > best || (bw == best && qw < q)) {
        best = bw; q = qw; p = __builtin_amdgcn_readfirstlane(red_c[w2]);
      }
    }
    const double nrm = sqrt(fmax(best, 0.0));
    if (k == 0) r11 = nrm;
    if (q >= n || nrm == 0.0 || (k > 0 && nrm <= tol * r11)) {
      rank = k > 0 ? k : 1;
      go = false;
      continue;
    }
    go = k + 1 < kmax;
    const int uk = k >> 6, lk = k & 63;
    if (w == p % NW) {
      const int sp = p / NW;
      double2 col[RR];
#pragma unroll
      for (int u = 0; u < RR; ++u) col[u] = zero2;
#pragma unroll
      for (int s = 0; s < NS; ++s)
        if (s == sp) {
#pragma unroll
          for (int u = 0; u < RR; ++u) col[u] = R[u][s];
        }
      double2 al = col[0];
#pragma unroll
      for (int u = 1; u < RR; ++u)
        if (u == uk) al = col[u];
      al = readlane_c(al, lk);
      const double beta = al.x >= 0.0 ? -nrm : nrm;
      const double dr = al.x - beta, di = al.y, dd = dr * dr + di * di;
      const double2 scale = double2{dr / dd, -di / dd};
#pragma unroll
      for (int u = 0; u < RR; ++u) {
        const int row = lane + 64 * u;
        v_sh[buf][row] = row < k ? zero2 : (row == k ? double2{1.0, 0.0} : cmul(col[u], scale));
      }
#pragma unroll
      for (int s = 0; s < NS; ++s)
        if (s == sp) {
#pragma unroll
          for (int u = 0; u < RR; ++u) {
            const int row = lane + 64 * u;
            if (row == k) R[u][s] = double2{beta, 0.0};
            else if (row > k) R[u][s] = zero2;
          }
        }
      if (lane == 0) tau_sh[buf] = double2{(beta - al.x) / beta, -al.y / beta};
    }
    if (tid == 0) {
      const int ck = colmap[k];
      colmap[k] = p;
      colmap[q] = ck;
      pos[p] = k;
      pos[ck] = q;
    }
    __syncthreads();
    const double2 tau = uniform_c(tau_sh[buf]);
    const double2 ctau = double2{tau.x, -tau.y};
    double2 v[RR];
#pragma unroll
    for (int u = 0; u < RR; ++u) v[u] = v_sh[buf][lane + 64 * u];
    double bv = -1.0;
    int bq = n, bc = -1;
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      const int c = w + NW * s;
      if (c < n) {
        const int pc = __builtin_amdgcn_readfirstlane(pos[c]);
        if (pc > k) {
          double2 d = zero2;
#pragma unroll
          for (int u = 0; u < RR; ++u) cfmac(d, v[u], R[u][s]);
          d.x = wave_sum_u(d.x);
          d.y = wave_sum_u(d.y);
          const double2 f = cmul(ctau, d);
          double sn = 0.0;
#pragma unroll
          for (int u = 0; u < RR; ++u) {
            R[u][s].x -= f.x * v[u].x - f.y * v[u].y;
            R[u][s].y -= f.x * v[u].y + f.y * v[u].x;
            if (lane + 64 * u > k) sn += R[u][s].x * R[u][s].x + R[u][s].y * R[u][s].y;
          }
          sn = wave_sum_u(sn);
          if (sn > bv || (sn == bv && pc < bq)) { bv = sn; bq = pc; bc = c; }
        }
      }
    }
    if (lane == 0) { red_v[w] = bv; red_q[w] = bq; red_c[w] = bc; }
    __syncthreads();
    buf ^= 1;
  }

  // ---- phase 3: X = [I, R11^-1 R12] Pi^T
  const int r = rank;
  const bool zero = !(r11 > 0.0);
  double2 *Rs = (int64_t)r * n <= cap ? lds_rs : (double2 *)B.A;
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    const int c = w + NW * s;
    if (c < n) {
      const int q = __builtin_amdgcn_readfirstlane(pos[c]);
#pragma unroll
      for (int u = 0; u < RR; ++u) {
        const int row = lane + 64 * u;
        if (row < r) Rs[row + q * r] = R[u][s];
      }
    }
  }
  __syncthreads();
  double2 *X = B.X;
  for (int idx = tid; idx < r * r; idx += T) {
    const int q = idx / r, i = idx % r;
    X[i + (int64_t)colmap[q] * r] = double2{i == q ? 1.0 : 0.0, 0.0};
  }
  for (int q = tid; q < r; q += T) B.piv[q] = colmap[q];
  const double2 *Rc = Rs;
  auto Rat = [Rc, r](int i, int l) { return Rc[i + l * r]; };
  for (int q = r + tid; q < n; q += T) solve_upper(Rat, Rs + q * r, r, zero);
  __syncthreads();
  for (int idx = tid; idx < r * (n - r); idx += T) {
    const int q = r + idx / r, i = idx % r;
    X[i + (int64_t)colmap[q] * r] = Rs[i + q * r];
  }
  if (tid == 0) rank_out[blk] = r;
}

// ---------------------------------------------------------------------------
// Interpolative decomposition of a block in global memory with the
// reflectors applied in panels of nb steps: the blocked form of column-
// pivoted Householder QR (deferred trailing update with downdated column
// norms, as in LAPACK's xGEQP3 / xLAQPS).  Same pivot rule, stopping test
// and output as k_cpqr.  Inside a panel that starts at row k0 the trailing
// block is A^(k) = A - V F^H, V holding the panel's reflectors (stored below
// the diagonal of the pivot columns) and F = [f_0 ...], f_l = tau_l A^(l)^H v_l.
// Step k, pivot p, trailing columns T:
//   a_p    = A(k:, p) - V(k:, :) F(p, :)^H        (pivot column brought up to date)
//   beta, tau, v from a_p (as in k_cpqr); v stored in A(k+1:, p)
//   g      = A(k:, T)^H v,  y = V(k:, :)^H v       (one read of the trailing block)
//   f      = tau (g - F(T, :) y)                    (new column of F)
//   R(k,T) = A(k, T) - V(k, :) F(T, :)^H - conj(f)  (written to A(k, T))
//   |a_j|^2 -= |R(k, j)|^2                          (norm downdate)
// A downdated norm that falls below sqrt(eps) of its last exact value is
// recomputed exactly; at the end of a panel A(k+1:, T) -= V F(T, :)^H is
// applied explicitly and all norms are recomputed.  Per step the trailing
// block is read once, against two reads and a write in k_cpqr.
// LDS: norms, reference norms, column map and recompute list (24 B per
// column), F (16 nb B per column), y and V(k, :) (nb entries each), then a
// region holding v (m entries, when it fits; else v is read from A), the
// panel-end chunk of V (64 nb entries) and, at the end, R's top rows.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(HBI_ID_THREADS) void k_cpqr_blocked(const IdBlock *blks,
                                                                  const int32_t *sel, double tol,
                                                                  int32_t *rank_out, int nmax,
                                                                  int nb, int vcap, int rcap) {
  extern __shared__ double lds_bq[];
  constexpr int NW = HBI_ID_THREADS / 64;
  constexpr double kTol3z = 1.4901161193847656e-08;   // sqrt(2^-52)
  __shared__ double red_v[NW], red_s[NW];
  __shared__ int red_q[NW], red_c[NW];
  __shared__ double2 sh_alpha;
  __shared__ int sh_nflag;

  const int blk = sel[blockIdx.x];
  const IdBlock B = blks[blk];
  const int m = B.m, n = B.n;
  double *nrm2 = lds_bq;
  double *nref = nrm2 + nmax;
  int *colmap = (int *)(nref + nmax);
  int *flist = colmap + nmax;
  double2 *F = (double2 *)(lds_bq + ((3 * nmax + 1) & ~1));   // nmax x nb, F(j, l) at F[j + l nmax]
  double2 *yv = F + (int64_t)nmax * nb;
  double2 *vr = yv + nb;
  double2 *reg = vr + nb;                         // v / V chunk / R's top rows
  const bool vlds = m <= vcap;
  double2 *A = B.A;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;

  // exact initial norms; each wave reports its best candidate
  {
    double bv = -1.0;
    int bq = n;
    for (int j = wave; j < n; j += NW) {
      const double2 *a = A + (int64_t)j * m;
      double s = 0.0;
      for (int r = lane; r < m; r += 64) s += a[r].x * a[r].x + a[r].y * a[r].y;
      s = wave_sum(s);
      if (lane == 0) { nrm2[j] = s; nref[j] = s; }
      if (s > bv) { bv = s; bq = j; }
    }
    if (lane == 0) { red_v[wave] = bv; red_q[wave] = bq; red_c[wave] = bq < n ? bq : 0; }
    for (int j = tid; j < n; j += HBI_ID_THREADS) colmap[j] = j;
  }
  __syncthreads();

  const int kmax = m < n ? m : n;
  int rank = kmax;
  double r11 = 0.0;
  int k0 = 0, i = 0;
  for (int k = 0; k < kmax; ++k) {
    // ---- pivot (every thread takes the same decision)
    double best = red_v[0];
    int q = red_q[0], p = red_c[0];
    for (int w2 = 1; w2 < NW; ++w2)
      if (red_v[w2] > best || (red_v[w2] == best && red_q[w2] < q)) {
        best = red_v[w2]; q = red_q[w2]; p = red_c[w2];
      }
    if (q >= n) { rank = k > 0 ? k : 1; break; }
    if (tid == 0) { colmap[q] = colmap[k]; colmap[k] = p; }
    // ---- pivot column a_p(k:) = A(k:, p) - V(k:, :) F(p, :)^H, its norm
    {
      double sp = 0.0;
      double2 *ap = A + (int64_t)p * m;
      for (int r = k + tid; r < m; r += HBI_ID_THREADS) {
        double2 a = ap[r];
        for (int l = 0; l < i; ++l) {
          const double2 vv = A[r + (int64_t)colmap[k0 + l] * m];
          const double2 fl = F[p + l * nmax];
          // a -= vv * conj(fl)
          a.x -= vv.x * fl.x + vv.y * fl.y;
          a.y -= vv.y * fl.x - vv.x * fl.y;
        }
        ap[r] = a;
        if (r == k) sh_alpha = a;
        else sp += a.x * a.x + a.y * a.y;
      }
      sp = wave_sum(sp);
      if (lane == 0) red_s[wave] = sp;
    }
    __syncthreads();
    // ---- reflector (every thread), v
    double s = 0.0;
    for (int w2 = 0; w2 < NW; ++w2) s += red_s[w2];
    const double2 al = sh_alpha;
    const double nrm = sqrt(al.x * al.x + al.y * al.y + s);
    if (k == 0) r11 = nrm;
    if (nrm == 0.0 || (k > 0 && nrm <= tol * r11)) { rank = k > 0 ? k : 1; break; }
    const double beta = al.x >= 0.0 ? -nrm : nrm;
    const double2 tau = double2{(beta - al.x) / beta, -al.y / beta};
    const double dr = al.x - beta, di = al.y, dd = dr * dr + di * di;
    const double2 scale = double2{dr / dd, -di / dd};
    {
      double2 *ap = A + (int64_t)p * m;
      for (int r = k + 1 + tid; r < m; r += HBI_ID_THREADS) {
        const double2 v = cmul(ap[r], scale);
        ap[r] = v;
        if (vlds) reg[r] = v;
      }
      if (tid == 0) {
        ap[k] = double2{beta, 0.0};
        if (vlds) reg[k] = double2{1.0, 0.0};
        sh_nflag = 0;
      }
      if (tid < i) vr[tid] = A[k + (int64_t)colmap[k0 + tid] * m];
    }
    __syncthreads();
    // ---- g = A(k:, T)^H v into F(:, i); y = V(k:, :)^H v
    {
      const double2 *pv = A + (int64_t)p * m;
      const int items = i + (n - k - 1);
      for (int it = wave; it < items; it += NW) {
        const int col = it < i ? colmap[k0 + it] : colmap[k + 1 + (it - i)];
        const double2 *a = A + (int64_t)col * m;
        double2 d = double2{0.0, 0.0};
        // rows k + lane + 64 t, kCpqrCB loads in flight per lane
        constexpr int CB = 8;
        for (int b = k; b < m; b += 64 * CB) {
          double2 av[CB];
#pragma unroll
          for (int u = 0; u < CB; ++u) {
            const int r = b + lane + 64 * u;
            av[u] = r < m ? a[r] : double2{0.0, 0.0};
          }
#pragma unroll
          for (int u = 0; u < CB; ++u) {
            const int r = b + lane + 64 * u;
            if (r < m) {
              const double2 v = r == k ? double2{1.0, 0.0} : (vlds ? reg[r] : pv[r]);
              cfmac(d, av[u], v);   // d += conj(a) v
            }
          }
        }
        d.x = wave_sum(d.x);
        d.y = wave_sum(d.y);
        if (lane == 0) {
          if (it < i) yv[it] = d;
          else F[col + i * nmax] = d;
        }
      }
    }
    __syncthreads();
    // ---- f, R(k, T), norm downdate (one thread per trailing column)
    for (int qq = k + 1 + tid; qq < n; qq += HBI_ID_THREADS) {
      const int j = colmap[qq];
      const double2 g = F[j + i * nmax];
      double2 fy = double2{0.0, 0.0};
      double2 vf = double2{0.0, 0.0};
      for (int l = 0; l < i; ++l) {
        const double2 fl = F[j + l * nmax];
        const double2 yl = yv[l], vl = vr[l];
        fy.x += fl.x * yl.x - fl.y * yl.y;
        fy.y += fl.x * yl.y + fl.y * yl.x;
        vf.x += vl.x * fl.x + vl.y * fl.y;   // vl * conj(fl)
        vf.y += vl.y * fl.x - vl.x * fl.y;
      }
      const double2 f = cmul(tau, double2{g.x - fy.x, g.y - fy.y});
      F[j + i * nmax] = f;
      double2 *akj = A + k + (int64_t)j * m;
      const double2 a0 = *akj;
      const double2 rk = double2{a0.x - vf.x - f.x, a0.y - vf.y + f.y};
      *akj = rk;
      const double nw = nrm2[j] - (rk.x * rk.x + rk.y * rk.y);
      if (nw <= kTol3z * nref[j]) {
        flist[atomicAdd(&sh_nflag, 1)] = j;
      } else {
        nrm2[j] = nw;
      }
    }
    ++i;
    const bool flush = i == nb && k + 1 < kmax;
    __syncthreads();
    if (flush) {
      // ---- panel end: A(k+1:, T) -= V F(T, :)^H, exact norms
      for (int qq = k + 1 + tid; qq < n; qq += HBI_ID_THREADS) nref[colmap[qq]] = 0.0;
      __syncthreads();
      for (int r0 = k + 1; r0 < m; r0 += 64) {
        __syncthreads();
        if (tid < 64 * nb) {
          const int rr = tid & 63, l = tid >> 6, r = r0 + rr;   // V chunk, row fastest
          reg[tid] = r < m ? A[r + (int64_t)colmap[k0 + l] * m] : double2{0.0, 0.0};
        }
        __syncthreads();
        const int r = r0 + lane;
        for (int qq = k + 1 + wave; qq < n; qq += NW) {
          const int j = colmap[qq];
          double sq = 0.0;
          if (r < m) {
            double2 a = A[r + (int64_t)j * m];
            for (int l = 0; l < nb; ++l) {
              const double2 vv = reg[l * 64 + lane];
              const double2 fl = F[j + l * nmax];
              a.x -= vv.x * fl.x + vv.y * fl.y;
              a.y -= vv.y * fl.x - vv.x * fl.y;
            }
            A[r + (int64_t)j * m] = a;
            sq = a.x * a.x + a.y * a.y;
          }
          sq = wave_sum(sq);
          if (lane == 0) nref[j] += sq;
        }
      }
      // the same wave owns column j in the loop above and below
      for (int qq = k + 1 + wave; qq < n; qq += NW)
        if (lane == 0) nrm2[colmap[qq]] = nref[colmap[qq]];
      k0 = k + 1;
      i = 0;
    } else if (sh_nflag > 0) {
      // ---- exact norms of the flagged columns: rows k+1.., all panel terms
      const int nf = sh_nflag;
      for (int t = wave; t < nf; t += NW) {
        const int j = flist[t];
        double sq = 0.0;
        for (int r = k + 1 + lane; r < m; r += 64) {
          double2 a = A[r + (int64_t)j * m];
          for (int l = 0; l < i; ++l) {
            const double2 vv = A[r + (int64_t)colmap[k0 + l] * m];
            const double2 fl = F[j + l * nmax];
            a.x -= vv.x * fl.x + vv.y * fl.y;
            a.y -= vv.y * fl.x - vv.x * fl.y;
          }
          sq += a.x * a.x + a.y * a.y;
        }
        sq = wave_sum(sq);
        if (lane == 0) { nrm2[j] = sq; nref[j] = sq; }
      }
      __syncthreads();
    }
    // ---- next candidates (the flush owner of column j reads it back itself)
    {
      double bv = -1.0;
      int bq = n, bc = 0;
      for (int qq = k + 1 + wave; qq < n; qq += NW) {
        const int j = colmap[qq];
        const double v = nrm2[j];
        if (v > bv) { bv = v; bq = qq; bc = j; }
      }
      if (lane == 0) { red_v[wave] = bv; red_q[wave] = bq; red_c[wave] = bc; }
    }
    __syncthreads();
  }
  __syncthreads();

  // ---- X = [I, R11^-1 R12] Pi^T from the top rows of R (in A, pivot order)
  const int r = rank;
  const bool zero = !(r11 > 0.0);
  double2 *X = B.X;
  for (int idx = tid; idx < r * r; idx += HBI_ID_THREADS) {
    const int qq = idx / r, ii = idx % r;
    X[ii + (int64_t)colmap[qq] * r] = double2{ii == qq ? 1.0 : 0.0, 0.0};
  }
  for (int qq = tid; qq < r; qq += HBI_ID_THREADS) B.piv[qq] = colmap[qq];
  double2 *Rs = F;   // F, y, V(k, :) and the region are free now
  if ((int64_t)r * n <= rcap) {
    for (int idx = tid; idx < r * n; idx += HBI_ID_THREADS) {
      const int qq = idx / r, ii = idx % r;
      Rs[idx] = A[ii + (int64_t)colmap[qq] * m];
    }
    __syncthreads();
    const double2 *Rc = Rs;
    auto Rat = [Rc, r](int a, int b) { return Rc[a + b * r]; };
    for (int qq = r + tid; qq < n; qq += HBI_ID_THREADS) solve_upper(Rat, Rs + qq * r, r, zero);
    __syncthreads();
    for (int idx = tid; idx < r * (n - r); idx += HBI_ID_THREADS) {
      const int qq = r + idx / r, ii = idx % r;
      X[ii + (int64_t)colmap[qq] * r] = Rs[ii + qq * r];
    }
  } else {
    auto Rat = [A, colmap, m](int a, int b) { return A[a + (int64_t)colmap[b] * m]; };
    for (int qq = r + tid; qq < n; qq += HBI_ID_THREADS) {
      const int col = colmap[qq];
      double2 *xo = X + (int64_t)col * r;
      for (int ii = 0; ii < r; ++ii) xo[ii] = A[ii + (int64_t)col * m];
      solve_upper(Rat, xo, r, zero);
    }
  }
  if (tid == 0) rank_out[blk] = r;
}

// The non-skeleton columns of interpolation matrices X = [I, T] Pi^T (the
// skeleton columns are unit vectors and are not stored): T_a = X_a[:, nsa],
// then, for a sibling pair (rb > 0), T_b = X_b[:, nsb].
__global__ void k_pack_pairs(const PairDesc *d, int64_t np) {
  const int64_t b = blockIdx.x;
  if (b >= np) return;
  const PairDesc p = d[b];
  const int ta = p.c - p.ra, tb = p.c - p.rb;
  const int64_t na = (int64_t)p.ra * ta, n = na + (int64_t)p.rb * tb;
  for (int64_t i = threadIdx.x; i < n; i += blockDim.x) {
    if (i < na) {
      const int m = (int)(i / p.ra), row = (int)(i % p.ra);
      p.dst[i] = p.xa[row + (int64_t)p.nsa[m] * p.ra];
    } else {
      const int64_t e = i - na;
      const int m = (int)(e / p.rb), row = (int)(e % p.rb);
      p.dst[i] = p.xb[row + (int64_t)p.nsb[m] * p.rb];
    }
  }
}

// Copy FP64 blocks to their places in the factor store (FP64 or rounded to
// FP32), one workgroup per block.
template <typename T>
__global__ void k_place_blocks(const PlaceDesc *d, int64_t nb, T *F) {
  const int64_t b = blockIdx.x;
  if (b >= nb) return;
  const PlaceDesc p = d[b];
  T *dst = F + p.dst;
  for (int64_t i = threadIdx.x; i < p.count; i += blockDim.x) {
    const double2 v = p.src[i];
    dst[i] = T{(decltype(T{}.x))v.x, (decltype(T{}.x))v.y};
  }
}


// ---------------------------------------------------------------------------
// Host-side launchers.
// ---------------------------------------------------------------------------
hipError_t launch_cell_setup(const DevProblem &P, const int32_t *perm, int64_t Nv,
                             const int32_t ncell[3], const double origin[3],
                             double *xyz, double *lw, int32_t *box, hipStream_t st) {
  const int T = 256;
  hipLaunchKernelGGL(k_cell_setup, dim3((Nv + T - 1) / T), dim3(T), 0, st, P, perm, Nv,
                     ncell[0], ncell[1], origin[0], origin[1], origin[2], xyz, lw, box);
  return hipGetLastError();
}

hipError_t launch_self_terms(const DevProblem &P, const double *slow, int64_t Nv,
                             const double *gx, const double *gw, int ng,
                             double2 *self, hipStream_t st) {
  const int T = 128;
  hipLaunchKernelGGL(k_self_terms, dim3((Nv + T - 1) / T), dim3(T), 0, st, P, slow, Nv,
                     gx, gw, ng, self);
  return hipGetLastError();
}

hipError_t launch_colside(const DevProblem &P, const DevCells &C, const DevTables &T,
                          const EntryBlock *blks, const int32_t *work, int64_t nwork,
                          const int32_t *cols, const int32_t *slotbox, double *Hc,
                          hipStream_t st) {
  if (nwork == 0) return hipSuccess;
  const size_t lds = sizeof(double) * (size_t)P.NTb;
  hipLaunchKernelGGL(k_colside, dim3(nwork), dim3(64), lds, st, P, C, T, blks, work, nwork,
                     cols, slotbox, Hc);
  return hipGetLastError();
}

hipError_t launch_colside_cells(const DevProblem &P, const DevCells &C, const DevTables &T,
                                int64_t Nv, int nbox, double *Hcache, hipStream_t st) {
  const int64_t n = Nv * nbox;
  if (n == 0) return hipSuccess;
  const size_t lds = sizeof(double) * (size_t)P.NTb;
  hipLaunchKernelGGL(k_colside_cells, dim3(n), dim3(64), lds, st, P, C, T, Nv, nbox, Hcache);
  return hipGetLastError();
}

template <int D, int NI>
static void entries_launch(const DevProblem &P, const DevCells &C, const EntryBlock *blks,
                           const ETile *tiles, int64_t ntiles, const int32_t *rows,
                           const int32_t *rord, const int32_t *cols, const double *Hc,
                           const int32_t *slotbox, const double *Hcache, int nbox,
                           hipStream_t st) {
  hipLaunchKernelGGL((k_entries<D, NI>), dim3(ntiles), dim3(256), 0, st, P, C, blks, tiles,
                     ntiles, rows, rord, cols, Hc, slotbox, Hcache, nbox);
}

hipError_t launch_entries(const DevProblem &P, const DevCells &C, const EntryBlock *blks,
                          const ETile *tiles, int64_t ntiles, const int32_t *rows,
                          const int32_t *rord, const int32_t *cols, const double *Hc,
                          const int32_t *slotbox, const double *Hcache, int nbox,
                          hipStream_t st) {
  if (ntiles == 0) return hipSuccess;
#define HBI_NI_CASE(D, NI)                                                                  \
  case NI:                                                                                  \
    entries_launch<D, NI>(P, C, blks, tiles, ntiles, rows, rord, cols, Hc, slotbox, Hcache, \
                          nbox, st);                                                        \
    break;
#define HBI_NI_SWITCH(D)                                                              \
  switch (P.nI) {                                                                     \
    HBI_NI_CASE(D, 2) HBI_NI_CASE(D, 3) HBI_NI_CASE(D, 4) HBI_NI_CASE(D, 5)           \
    HBI_NI_CASE(D, 6) HBI_NI_CASE(D, 7) HBI_NI_CASE(D, 8) HBI_NI_CASE(D, 9)           \
    HBI_NI_CASE(D, 10) HBI_NI_CASE(D, 11) HBI_NI_CASE(D, 12) HBI_NI_CASE(D, 13)       \
    HBI_NI_CASE(D, 14) HBI_NI_CASE(D, 15) HBI_NI_CASE(D, 16)                          \
    default: return hipErrorInvalidValue;                                            \
  }
  if (P.dim == 2) {
    HBI_NI_SWITCH(2)
  } else {
    HBI_NI_SWITCH(3)
  }
#undef HBI_NI_SWITCH
#undef HBI_NI_CASE
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Interpolative decomposition of a tall block (m >= n) from its Gram matrix.
// The column-pivoted QR of A and the pivoted Cholesky factorisation of
// G = A^H A choose the same pivots and the same R in exact arithmetic (the
// remaining column norms of the QR are the square roots of the remaining
// diagonal of the Cholesky factorisation), so A is read once, by an MFMA
// product, instead of once per pivot step:
//   k_gram   G = A^H A (n x n, row major, in X's space, which holds
//            min(m, n) n >= n^2 entries), FP64 16x16x4 MFMA tiles of the
//            upper triangle, mirrored;
//   k_pchol  left-looking pivoted Cholesky of G with the pivot rule and
//            stopping test of k_cpqr (largest remaining norm, stop once it
//            is at most tol |R_00|): the rows of R, row major in A's space
//            (A is not needed any more), then X = R11^-1 [R11 R12] written
//            as k_cpqr writes it.
// Rounding: the Gram matrix squares the condition number.  A remaining
// diagonal entry carries an absolute error of about eps |a_j|^2 per step,
// which can swap pivots that are within rounding of each other and keep
// columns of norm up to about sqrt(k eps) |A|; the interpolation residual
// stays at about eps times the skeleton's condition number.  The caller
// takes this path only for tolerances where that was measured harmless.
// ---------------------------------------------------------------------------
constexpr int kGramWG = 8;   // workgroups per block in k_gram

__global__ __launch_bounds__(256) void k_gram(const IdBlock *blks, const int32_t *sel) {
  typedef double v4 __attribute__((ext_vector_type(4)));
  const int blk = sel[blockIdx.x / kGramWG];
  const int part = blockIdx.x % kGramWG;
  const IdBlock B = blks[blk];
  const int m = B.m, n = B.n;
  const int nt = (n + 15) / 16, ntri = nt * (nt + 1) / 2;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int li = lane & 15, lk = lane >> 4;
  double2 *G = B.X;
  constexpr int KS = 4;   // MFMA k-steps whose loads are issued together
  for (int t = part * 4 + wave; t < ntri; t += kGramWG * 4) {
    int I = 0, rem = t;
    while (rem >= nt - I) { rem -= nt - I; ++I; }
    const int J = I + rem;
    const int ci = I * 16 + li, cj = J * 16 + li;
    const bool oi = ci < n, oj = cj < n;
    const double2 *ai = B.A + (int64_t)(oi ? ci : 0) * m;
    const double2 *aj = B.A + (int64_t)(oj ? cj : 0) * m;
    v4 re = {0.0, 0.0, 0.0, 0.0}, im = {0.0, 0.0, 0.0, 0.0};
    for (int k0 = 0; k0 < m; k0 += 4 * KS) {
      double2 x[KS], y[KS];
#pragma unroll
      for (int q = 0; q < KS; ++q) {
        const int k = k0 + 4 * q + lk;
        const int kc = k < m ? k : 0;
        x[q] = ai[kc];
        y[q] = aj[kc];
        if (!(oi && k < m)) x[q] = double2{0.0, 0.0};
        if (!(oj && k < m)) y[q] = double2{0.0, 0.0};
      }
#pragma unroll
      for (int q = 0; q < KS; ++q) {
        // conj(x) y
        re = __builtin_amdgcn_mfma_f64_16x16x4f64(x[q].x, y[q].x, re, 0, 0, 0);
        re = __builtin_amdgcn_mfma_f64_16x16x4f64(x[q].y, y[q].y, re, 0, 0, 0);
        im = __builtin_amdgcn_mfma_f64_16x16x4f64(x[q].x, y[q].y, im, 0, 0, 0);
        im = __builtin_amdgcn_mfma_f64_16x16x4f64(-x[q].y, y[q].x, im, 0, 0, 0);
      }
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int row = I * 16 + lk + 4 * v, col = J * 16 + li;
      if (row < n && col < n) {
        G[(int64_t)row * n + col] = double2{re[v], im[v]};
        if (I != J) G[(int64_t)col * n + row] = double2{re[v], -im[v]};
      }
    }
  }
}

__global__ __launch_bounds__(HBI_ID_THREADS) void k_pchol(const IdBlock *blks, const int32_t *sel,
                                                           double tol, int32_t *rank_out) {
  extern __shared__ double lds_pc[];
  constexpr int T = HBI_ID_THREADS, NW = T / 64;
  __shared__ double red_v[NW];
  __shared__ int red_i[NW];
  __shared__ int sh_stop, sh_rank, sh_p;
  __shared__ double sh_nrm, sh_r11;
  const int blk = sel[blockIdx.x];
  const IdBlock B = blks[blk];
  const int n = B.n;
  const double2 *G = B.X;
  double2 *R = B.A;                                  // row k of R at R + k n
  double2 *rp = (double2 *)lds_pc;                   // n: R[l][p], l < k
  double *d = lds_pc + 2 * (int64_t)n;               // n: remaining diagonal
  int *colmap = (int *)(d + n);                      // n: pivot order
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  for (int j = tid; j < n; j += T) {
    d[j] = fmax(G[(int64_t)j * n + j].x, 0.0);
    colmap[j] = j;
  }
  if (tid == 0) { sh_rank = n; sh_r11 = 0.0; }
  __syncthreads();
  for (int k = 0; k < n; ++k) {
    // largest remaining diagonal over positions [k, n) (lowest position on ties)
    double bv = -1.0;
    int bq = n;
    for (int q = k + tid; q < n; q += T) {
      const double v = d[colmap[q]];
      if (v > bv) { bv = v; bq = q; }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      const double ov = __shfl_xor(bv, o, 64);
      const int oq = __shfl_xor(bq, o, 64);
      if (ov > bv || (ov == bv && oq < bq)) { bv = ov; bq = oq; }
    }
    if (lane == 0) { red_v[wave] = bv; red_i[wave] = bq; }
    __syncthreads();
    if (tid == 0) {
      double v = red_v[0];
      int q = red_i[0];
      for (int w2 = 1; w2 < NW; ++w2)
        if (red_v[w2] > v || (red_v[w2] == v && red_i[w2] < q)) { v = red_v[w2]; q = red_i[w2]; }
      const double nrm = sqrt(fmax(v, 0.0));
      if (k == 0) sh_r11 = nrm;
      const int stop = (q >= n) || (nrm == 0.0) || (k > 0 && nrm <= tol * sh_r11);
      sh_stop = stop;
      if (stop) {
        sh_rank = k > 0 ? k : 1;
      } else {
        const int t = colmap[k];
        colmap[k] = colmap[q];
        colmap[q] = t;
        sh_p = colmap[k];
        sh_nrm = nrm;
      }
    }
    __syncthreads();
    if (sh_stop) break;
    const int p = sh_p;
    const double nrm = sh_nrm, inv = 1.0 / nrm;
    for (int l = tid; l < k; l += T) rp[l] = R[(int64_t)l * n + p];
    if (tid == 0) R[(int64_t)k * n + p] = double2{nrm, 0.0};
    __syncthreads();
    // row k over the remaining columns: (G[p][j] - sum_l conj(R[l][p]) R[l][j]) / R_kk
    for (int q = k + 1 + tid; q < n; q += T) {
      const int j = colmap[q];
      double2 acc = G[(int64_t)p * n + j];
      int l = 0;
      for (; l + 4 <= k; l += 4) {
        double2 rv[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) rv[u] = R[(int64_t)(l + u) * n + j];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const double2 a = rp[l + u];
          acc.x -= a.x * rv[u].x + a.y * rv[u].y;
          acc.y -= a.x * rv[u].y - a.y * rv[u].x;
        }
      }
      for (; l < k; ++l) {
        const double2 a = rp[l], b = R[(int64_t)l * n + j];
        acc.x -= a.x * b.x + a.y * b.y;
        acc.y -= a.x * b.y - a.y * b.x;
      }
      const double2 rkj = double2{acc.x * inv, acc.y * inv};
      R[(int64_t)k * n + j] = rkj;
      d[j] = fmax(d[j] - (rkj.x * rkj.x + rkj.y * rkj.y), 0.0);
    }
    __syncthreads();
  }
  const int r = sh_rank;
  const bool zero = !(sh_r11 > 0.0);
  double2 *X = B.X;   // G is not read any more
  for (int idx = tid; idx < r * r; idx += T) {
    const int q = idx / r, i = idx % r;
    X[i + (int64_t)colmap[q] * r] = double2{i == q ? 1.0 : 0.0, 0.0};
  }
  for (int q = tid; q < r; q += T) B.piv[q] = colmap[q];
  auto Rat = [R, colmap, n](int i, int l) { return R[(int64_t)i * n + colmap[l]]; };
  for (int q = r + tid; q < n; q += T) {
    const int col = colmap[q];
    double2 *xo = X + (int64_t)col * r;
    for (int i = 0; i < r; ++i) xo[i] = R[(int64_t)i * n + col];
    solve_upper(Rat, xo, r, zero);
  }
  if (tid == 0) rank_out[blk] = r;
}

static hipError_t lds_limit(int *ldsmax) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  return hipDeviceGetAttribute(ldsmax, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
}

hipError_t launch_cpqr(const IdBlock *blks, const int32_t *sel, int64_t nb, int nmax, int mmax,
                       double tol, int32_t *rank, hipStream_t st) {
  if (nb == 0) return hipSuccess;
  int ldsmax = 65536;
  hipError_t e = lds_limit(&ldsmax);
  if (e != hipSuccess) return e;
  // norms + column map, then the region for v (m entries) and R's top rows
  // (r n <= min(m, n) n entries), as far as the device's LDS allows
  const size_t head = sizeof(double) * (((size_t)nmax + (nmax + 1) / 2 + 2) & ~(size_t)1);
  const size_t want = std::max<size_t>((size_t)mmax, (size_t)std::min(mmax, nmax) * nmax);
  const size_t avail = (size_t)ldsmax > head + 1024 ? ((size_t)ldsmax - head - 1024) / 16 : 0;
  const int cap = (int)std::min(want, avail);
  const size_t lds = head + sizeof(double2) * (size_t)cap;
  if (lds > 65536) {
    e = hipFuncSetAttribute((const void *)k_cpqr, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)lds);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_cpqr, dim3(nb), dim3(HBI_ID_THREADS), lds, st, blks, sel, tol, rank, nmax,
                     cap);
  return hipGetLastError();
}

hipError_t launch_cpqr_blocked(const IdBlock *blks, const int32_t *sel, int64_t nb, int nmax,
                               int mmax, double tol, int32_t *rank, hipStream_t st) {
  if (nb == 0) return hipSuccess;
  int ldsmax = 65536;
  hipError_t e = lds_limit(&ldsmax);
  if (e != hipSuccess) return e;
  const size_t avail = ldsmax > 4096 ? (size_t)ldsmax - 4096 : 0;   // static LDS and slack
  const size_t head = sizeof(double) * ((3 * (size_t)nmax + 1) & ~(size_t)1);
  auto bytes = [&](int pw, size_t regcap) {
    return head + sizeof(double2) * ((size_t)nmax * pw + 2 * pw + regcap);
  };
  int pw = 16;
  while (pw >= 2 && bytes(pw, 64 * (size_t)pw) > avail) pw /= 2;
  if (pw < 2) return launch_cpqr(blks, sel, nb, nmax, mmax, tol, rank, st);
  size_t regcap = 64 * (size_t)pw;
  int vcap = 0;
  if (bytes(pw, std::max(regcap, (size_t)mmax)) <= avail) {
    regcap = std::max(regcap, (size_t)mmax);
    vcap = (int)regcap;
  }
  const int rcap = (int)((size_t)nmax * pw + 2 * pw + regcap);
  const size_t lds = bytes(pw, regcap);
  if (lds > 65536) {
    e = hipFuncSetAttribute((const void *)k_cpqr_blocked,
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_cpqr_blocked, dim3(nb), dim3(HBI_ID_THREADS), lds, st, blks, sel, tol,
                     rank, nmax, pw, vcap, rcap);
  return hipGetLastError();
}

hipError_t launch_id_onchip(const IdBlock *blks, const int32_t *sel, int64_t nb, int nmax,
                            double tol, int32_t *rank, hipStream_t st) {
  if (nb == 0) return hipSuccess;
  if (nmax > HBI_ID_ONCHIP_NMAX) return hipErrorInvalidValue;
  int ldsmax = 65536;
  hipError_t e = lds_limit(&ldsmax);
  if (e != hipSuccess) return e;
  // R's top rows: 64 KiB (two workgroups share a CU), within what the
  // device allows
  const size_t lds = std::min((size_t)64 << 10, ldsmax > 8192 ? (size_t)ldsmax - 8192 : (size_t)0);
  const int cap = (int)(lds / sizeof(double2));
  e = hipFuncSetAttribute((const void *)k_id_onchip<8, 8, 2, 4>,
                          hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_id_onchip<8, 8, 2, 4>), dim3(nb), dim3(512), lds, st, blks, sel, tol, rank,
                     cap);
  return hipGetLastError();
}

hipError_t launch_id_gram(const IdBlock *blks, const int32_t *sel, int64_t nb, int nmax,
                          double tol, int32_t *rank, hipStream_t st) {
  if (nb == 0) return hipSuccess;
  int ldsmax = 65536;
  hipError_t e = lds_limit(&ldsmax);
  if (e != hipSuccess) return e;
  // rp (16 B), d (8 B) and colmap (4 B) per column
  const size_t lds = (size_t)28 * nmax + 64;
  if (lds > (size_t)ldsmax) return hipErrorInvalidValue;
  if (lds > 65536) {
    e = hipFuncSetAttribute((const void *)k_pchol, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)lds);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_gram, dim3((unsigned)(nb * kGramWG)), dim3(256), 0, st, blks, sel);
  hipLaunchKernelGGL(k_pchol, dim3((unsigned)nb), dim3(HBI_ID_THREADS), lds, st, blks, sel, tol,
                     rank);
  return hipGetLastError();
}

hipError_t launch_pack_pairs(const PairDesc *d, int64_t np, hipStream_t st) {
  if (np == 0) return hipSuccess;
  hipLaunchKernelGGL(k_pack_pairs, dim3(np), dim3(256), 0, st, d, np);
  return hipGetLastError();
}

hipError_t launch_place_blocks(const PlaceDesc *d, int64_t nb, void *F, bool f32,
                               hipStream_t st) {
  if (nb == 0) return hipSuccess;
  if (f32)
    hipLaunchKernelGGL(k_place_blocks<float2>, dim3(nb), dim3(256), 0, st, d, nb, (float2 *)F);
  else
    hipLaunchKernelGGL(k_place_blocks<double2>, dim3(nb), dim3(256), 0, st, d, nb, (double2 *)F);
  return hipGetLastError();
}


}  // namespace hbi
