// C ABI, context and the level-synchronous HODBF build driver.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <deque>
#include <functional>
#include <limits>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/hbi.h"
#include "hbi_geometry.h"
#include "hbi_internal.h"
#include "hbi_kernels.h"
#include "hbi_multi.h"
#include "hbi_tabulate.h"

#include <cstdlib>
#include <fstream>
#include <map>
#include <sstream>

using namespace hbi;

namespace {

thread_local std::string g_err;
// Every successful build gets a new number: a cached batched-apply graph
// names its contexts by address and by this number, so that it is never
// replayed on factors that a rebuild (or a new context at the same
// address) has replaced.
std::atomic<uint64_t> g_build_gen{0};

}  // namespace

// Fixed per-device scratch of the allocation-free apply (hbi_apply_noalloc):
// the per-level vectors z of the single-RHS product live here instead of in
// memory the library allocates.  Host code never uses this name as an
// address: the device address of each GPU's copy comes from
// hipGetSymbolAddress, taken once per device when a context is created on
// it, and kept in g_scratch below.
static __device__ __align__(256) unsigned char scratch[HBI_NOALLOC_SCRATCH_BYTES];

namespace {

struct ScratchSlot {
  bool done = false;
  hipError_t status = hipSuccess;
  void *ptr = nullptr;
};
std::mutex g_scratch_mu;
std::map<int, ScratchSlot> g_scratch;

// The device address of `scratch` on `device` (the current device), looked
// up once per device.
void setup_scratch(int device) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  ScratchSlot &sl = g_scratch[device];
  if (sl.done) return;
  sl.done = true;
  void *ptr = nullptr;
  sl.status = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (sl.status != hipSuccess) {
    (void)hipGetLastError();
    sl.ptr = nullptr;
  } else {
    sl.ptr = ptr;
  }
}


// Test hook: with HBI_FAIL_ALLOC_BYTES=X set, every device allocation of at
// least X bytes fails as out of memory (the error paths of HBI_ERR_OOM).
bool forced_oom(size_t bytes) {
  const char *e = std::getenv("HBI_FAIL_ALLOC_BYTES");
  if (!e || !*e) return false;
  const unsigned long long x = std::strtoull(e, nullptr, 10);
  return x > 0 && bytes >= x;
}

struct DevBuf {
  void *p = nullptr;
  size_t n = 0;
  DevBuf() = default;
  DevBuf(const DevBuf &) = delete;
  DevBuf &operator=(const DevBuf &) = delete;
  DevBuf(DevBuf &&o) noexcept : p(o.p), n(o.n) { o.p = nullptr; o.n = 0; }
  DevBuf &operator=(DevBuf &&o) noexcept {
    if (this != &o) { release(); p = o.p; n = o.n; o.p = nullptr; o.n = 0; }
    return *this;
  }
  ~DevBuf() { release(); }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    n = 0;
  }
  hipError_t alloc(size_t bytes) {
    release();
    if (bytes == 0) return hipSuccess;
    if (forced_oom(bytes)) return hipErrorOutOfMemory;
    hipError_t e = hipMalloc(&p, bytes);
    if (e != hipSuccess) { p = nullptr; (void)hipGetLastError(); return e; }
    n = bytes;
    return hipSuccess;
  }
  // grow-only reuse
  hipError_t reserve(size_t bytes) { return bytes <= n ? hipSuccess : alloc(bytes); }
  template <class T> T *as() const { return (T *)p; }
};

// Pinned (page-locked) host memory, grow-only.
struct HostBuf {
  void *p = nullptr;
  size_t n = 0;
  HostBuf() = default;
  HostBuf(const HostBuf &) = delete;
  HostBuf &operator=(const HostBuf &) = delete;
  ~HostBuf() { release(); }
  void release() {
    if (p) (void)hipHostFree(p);
    p = nullptr;
    n = 0;
  }
  hipError_t reserve(size_t bytes) {
    if (bytes <= n) return hipSuccess;
    release();
    hipError_t e = hipHostMalloc(&p, bytes, hipHostMallocDefault);
    if (e != hipSuccess) { p = nullptr; (void)hipGetLastError(); return e; }
    n = bytes;
    return hipSuccess;
  }
  template <class T> T *as() const { return (T *)p; }
};

struct Status {
  hbi_status code;
  std::string msg;
};

struct Error {
  hbi_status code;
  std::string msg;
};

#define HBI_HIP(expr)                                                                  \
  do {                                                                                 \
    hipError_t e_ = (expr);                                                            \
    if (e_ != hipSuccess) {                                                            \
      throw Error{e_ == hipErrorOutOfMemory ? HBI_ERR_OOM : HBI_ERR_HIP,               \
                  std::string(#expr) + ": " + hipGetErrorString(e_)};                  \
    }                                                                                  \
  } while (0)

#define HBI_REQUIRE(cond, code, msg) \
  do {                               \
    if (!(cond)) throw Error{code, msg}; \
  } while (0)

void *scratch_ptr(int device) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  auto it = g_scratch.find(device);
  if (it == g_scratch.end() || !it->second.done)
    throw Error{HBI_ERR_STATE, "scratch of this device not set up (no context created on it)"};
  if (it->second.status != hipSuccess)
    throw Error{HBI_ERR_HIP, std::string("hipGetSymbolAddress(scratch): ") +
                                 hipGetErrorString(it->second.status)};
  return it->second.ptr;
}

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// Gauss-Legendre nodes/weights on [0,1] by Newton iteration on P_n.
void gauss_legendre01(int n, std::vector<double> &x, std::vector<double> &w) {
  x.resize(n);
  w.resize(n);
  for (int i = 0; i < n; ++i) {
    double z = std::cos(M_PI * (i + 0.75) / (n + 0.5));
    double dp = 1.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = z;
      for (int k = 2; k <= n; ++k) {
        const double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      dp = n * (z * p1 - p0) / (z * z - 1.0);
      const double dz = p1 / dp;
      z -= dz;
      if (std::fabs(dz) < 1e-16) break;
    }
    x[i] = 0.5 * (1.0 - z);
    w[i] = 1.0 / ((1.0 - z * z) * dp * dp);   // = 0.5 * 2/((1-z^2) P'^2)
  }
}

struct Chunk {
  DevBuf buf;
  int64_t goff;     // global element offset in the final factor store
  int64_t count;    // complex elements
};

// Records an event pair around every apply launch while enabled.
struct Profiler : LaunchHook {
  hipStream_t st = nullptr;
  struct Rec { const char *name; hipEvent_t a, b; double bytes; };
  std::vector<Rec> recs;
  void before(const char *name, double bytes) override {
    Rec r{name, nullptr, nullptr, bytes};
    if (hipEventCreate(&r.a) != hipSuccess || hipEventCreate(&r.b) != hipSuccess) return;
    (void)hipEventRecord(r.a, st);
    recs.push_back(r);
  }
  void after() override {
    if (!recs.empty()) (void)hipEventRecord(recs.back().b, st);
  }
  void clear() {
    for (auto &r : recs) { (void)hipEventDestroy(r.a); (void)hipEventDestroy(r.b); }
    recs.clear();
  }
  ~Profiler() override { clear(); }
};

}  // namespace

struct BatchCache;

struct hbi_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  std::string err;
  int state = 0;   // 0 created, 1 tables, 2 built
  // problem
  int dim = 2, nterms = 2, nI = 3, NTb = 0, NT = 0;
  int32_t ncell[3] = {1, 1, 1}, nbox[3] = {1, 1, 1};
  double origin[3] = {0, 0, 0}, h = 1, omega = 1, box_origin[3] = {0, 0, 0}, box_size = 1;
  std::vector<double> slow_nat;
  hbi_build_opts opts{};
  int geo_leaf = -1, geo_band = -1;   // leaf size and band width the tree was built with
  Geometry geo;
  std::vector<int32_t> box_h;   // table box per tree position (host copy)
  // device cell data
  DevBuf perm_d, xyz_d, lw_d, box_d, self_d, slow_d, FT_d[3];
  // build workspace; hc_cache holds the column side of every (cell, box)
  // pair during a build when it fits (hc_nbox boxes per cell, else empty)
  DevBuf ws, idx_d, hc_cache;
  int hc_nbox = 0;
  // factors and plan
  hbi_prec prec = HBI_F64;
  DevBuf F;
  int64_t Felems = 0;
  DevBuf Fi;   // uint16 index store of the transfer units (WUnit)
  DevBuf leaves_d, vd_d, kd_d;
  std::vector<DevBuf> units_d, items_d, items_adj_d;
  ApplyPlan plan;
  int64_t ztotal = 0;
  int64_t zalloc = 0;   // entries of z_d (the per-level vectors of one single-RHS product)
  DevBuf z_d;
  // forward transfer items with inputs staged in LDS / gathered from global
  // memory, and those on 16-row windows
  int64_t wst_lds = 0, wst_global = 0, wst_wide = 0;
  // the last hbi_tabulate: sources, largest sweep count, point updates (rounds
  // x four orderings x updated points, over every equation), solve time
  int32_t tab_sources = 0, tab_rounds_max = 0;
  double tab_point_updates = 0, tab_s = 0;
  // batched products issued by this context as one persistent launch
  int64_t n_persistent = 0;
  int32_t wst_cq[5] = {0, 0, 0, 0, 0};   // unit widths c: min, quartiles, max
  // curve inclusion (2D): segments at positions [Nv, Nv + inc_ns) of the
  // per-point arrays; inputs on the host and the device, and the dense
  // operators built with the factors
  int32_t inc_ns = 0;
  std::vector<double> inc_xy, inc_w, inc_n;
  DevBuf inc_xy_d, inc_w_d, inc_n_d;
  DevBuf cellof_d;   // [Nv + inc_ns]: the cell containing each point (DevCells::cellof)
  DevBuf inc_G, inc_M, inc_MH, inc_wf, inc_part, inc_z, inc_y, inc_part2, inc_part3;
  InclusionPlan inc_plan;
  // G as a single butterfly (the default; HBI_INCLUSION_DENSE=1 keeps G dense)
  DevBuf s2v_F, s2v_idx, s2v_leaves, s2v_nodes, s2v_z;
  std::vector<DevBuf> s2v_units;
  S2VPlan s2v_plan;
  int s2v_L = -1;
  int64_t s2v_entries = 0, s2v_ztotal = 0;
  int32_t s2v_rank_max = 0;
  double t_inc = 0;
  bool profiling = false;
  Profiler prof;
  // host copies of the apply plan (used to assemble batched work items)
  std::vector<LeafInfo> leaves_h;
  std::vector<VDesc> vd_h;
  std::vector<KDesc> kd_h;
  std::vector<std::vector<WUnit>> units_h;
  std::shared_ptr<BatchCache> batch, batch_adj;   // forward / adjoint graphs
  uint64_t build_gen = 0;   // g_build_gen of the current factors (0: none)
  // statistics
  double t_build = 0, t_geo = 0, t_host = 0, t_gpu = 0, t_final = 0;
  double t_prep = 0, t_wait = 0, t_compact = 0;   // inside t_gpu: batch host set-up, batch total, compaction
  int64_t nnz_v = 0, nnz_w = 0, nnz_k = 0, nnz_d = 0, entries_eval = 0, nid = 0;
  int64_t entry_slots = 0;   // entry-tile capacity launched (fill = entries_eval / entry_slots)
  int64_t nid_path[3] = {0, 0, 0};   // IDs per kernel group (on chip, Gram matrix, global QR)
  int32_t rank_max = 0, id_m_max = 0;
  double rank_sum = 0, id_m_sum = 0, id_n_sum = 0, id_work = 0, id_work_wide = 0, id_work_128 = 0;
  int64_t nid_wide = 0;
  double tol = 0;

  DevProblem devprob() const {
    DevProblem P{};
    P.dim = dim; P.nI = nI; P.NT = NT; P.NTb = NTb; P.nterms = nterms;
    for (int a = 0; a < 3; ++a) { P.nbox[a] = nbox[a]; P.box_origin[a] = box_origin[a]; }
    P.box_size = box_size; P.omega = omega; P.h = h; P.hd = std::pow(h, dim);
    return P;
  }
  DevCells devcells() const {
    DevCells C{};
    C.xyz = xyz_d.as<double>(); C.lw = lw_d.as<double>(); C.box = box_d.as<int32_t>();
    C.self = self_d.as<double2>(); C.slow = slow_d.as<double>(); C.perm = perm_d.as<int32_t>();
    C.cellof = inc_ns ? cellof_d.as<int32_t>() : nullptr;
    return C;
  }
  DevTables devtables() const {
    DevTables T{};
    for (int t = 0; t < 3; ++t) T.FT[t] = FT_d[t].as<double>();
    return T;
  }
  double chi() const { return opts.chi > 0 ? opts.chi : (dim == 2 ? 20.0 : 4.0); }
  int leaf() const { return opts.leaf_size > 0 ? std::min(opts.leaf_size, HBI_MAX_LEAF) : 64; }
  double radius() const { return opts.neighbor_radius > 0 ? opts.neighbor_radius : (dim == 2 ? 10.0 : 3.0); }
  int band() const { return opts.band_width > 0 ? opts.band_width : 2; }
  // batch workspace budget: the option, else an eighth of the free device
  // memory within [2 GiB, 32 GiB] (more blocks per batch keep more CUs busy
  // while the largest decompositions run)
  int64_t wsbytes() const {
    if (opts.workspace_bytes > 0) return opts.workspace_bytes;
    size_t fr = 0, tot = 0;
    if (hipMemGetInfo(&fr, &tot) != hipSuccess) { (void)hipGetLastError(); fr = 0; }
    const int64_t lo = (int64_t)2 << 30, hi = (int64_t)32 << 30;
    return std::min(hi, std::max(lo, (int64_t)(fr / 8)));
  }
  void drop_factors() {
    F.release(); Felems = 0; Fi.release(); leaves_d.release(); vd_d.release(); kd_d.release();
    units_d.clear(); items_d.clear(); items_adj_d.clear(); plan = ApplyPlan();
    inc_G.release(); inc_M.release(); inc_MH.release(); inc_wf.release();
    inc_part.release(); inc_z.release(); inc_y.release(); inc_part2.release();
    inc_part3.release();
    inc_plan = InclusionPlan(); t_inc = 0;
    s2v_F.release(); s2v_idx.release(); s2v_leaves.release(); s2v_nodes.release();
    s2v_z.release(); s2v_units.clear(); s2v_plan = S2VPlan();
    s2v_L = -1; s2v_entries = s2v_ztotal = 0; s2v_rank_max = 0;
    leaves_h.clear(); vd_h.clear(); kd_h.clear(); units_h.clear(); batch.reset(); batch_adj.reset(); ztotal = 0;
    zalloc = 0;
    z_d.release(); wst_lds = wst_global = wst_wide = 0;
    build_gen = 0;
    nnz_v = nnz_w = nnz_k = nnz_d = entries_eval = nid = 0; rank_max = 0; rank_sum = 0;
    t_prep = t_wait = t_compact = 0; entry_slots = 0;
    nid_path[0] = nid_path[1] = nid_path[2] = 0;
    id_m_max = 0; id_m_sum = id_n_sum = id_work = id_work_wide = id_work_128 = 0; nid_wide = 0;
    if (state > 1) state = 1;
  }
};

namespace {

hbi_status fail(hbi_ctx *ctx, const Error &e) {
  if (ctx) ctx->err = e.msg; else g_err = e.msg;
  return e.code;
}

template <class F> hbi_status guarded(hbi_ctx *ctx, F &&f) {
  try {
    if (ctx) {
      ctx->err.clear();
      HBI_HIP(hipSetDevice(ctx->device));
    }
    f();
    return HBI_OK;
  } catch (const Error &e) {
    return fail(ctx, e);
  } catch (const std::bad_alloc &) {
    return fail(ctx, Error{HBI_ERR_OOM, "host allocation failed"});
  } catch (const std::exception &e) {
    return fail(ctx, Error{HBI_ERR_HIP, e.what()});
  }
}

template <class T> void upload(DevBuf &d, const std::vector<T> &h) {
  HBI_HIP(d.alloc(h.size() * sizeof(T)));
  if (!h.empty()) HBI_HIP(hipMemcpy(d.p, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice));
}

// Geometry + per-cell device arrays for the current leaf size.
// Self terms (App. A) of every cell at the context's omega, and the
// per-point data of the inclusion's segments (their K^{s2s} self factor
// depends on omega too).
void eval_self_terms(hbi_ctx *c) {
  const int64_t Nv = c->geo.Nv;
  HBI_HIP(c->self_d.alloc(sizeof(double2) * (Nv + c->inc_ns)));
  std::vector<double> gx, gw;
  gauss_legendre01(32, gx, gw);
  DevBuf gx_d, gw_d;
  upload(gx_d, gx);
  upload(gw_d, gw);
  HBI_HIP(launch_self_terms(c->devprob(), c->slow_d.as<double>(), Nv, gx_d.as<double>(),
                            gw_d.as<double>(), 32, c->self_d.as<double2>(), c->stream));
  HBI_HIP(launch_point_setup(c->devprob(), c->inc_xy_d.as<double>(), c->inc_w_d.as<double>(),
                             c->inc_n_d.as<double>(), c->inc_ns, Nv, c->xyz_d.as<double>(),
                             c->lw_d.as<double>(), c->box_d.as<int32_t>(),
                             c->self_d.as<double2>(), c->stream));
  HBI_HIP(hipStreamSynchronize(c->stream));
}

void setup_cells(hbi_ctx *c) {
  const double t0 = now_s();
  c->geo.build(c->dim, c->ncell, c->leaf());
  c->geo.build_bands(c->band());
  c->geo_leaf = c->leaf();
  c->geo_band = c->band();
  const int64_t Nv = c->geo.Nv;
  upload(c->perm_d, c->geo.perm);
  std::vector<double> slow_t(Nv);
  for (int64_t p = 0; p < Nv; ++p) slow_t[p] = c->slow_nat[c->geo.perm[p]];
  upload(c->slow_d, slow_t);
  const int64_t np = Nv + c->inc_ns;   // cells, then the inclusion's segments
  HBI_HIP(c->xyz_d.alloc(sizeof(double) * 3 * np));
  HBI_HIP(c->lw_d.alloc(sizeof(double) * c->dim * c->nI * np));
  HBI_HIP(c->box_d.alloc(sizeof(int32_t) * np));
  const DevProblem P = c->devprob();
  HBI_HIP(launch_cell_setup(P, c->perm_d.as<int32_t>(), Nv, c->ncell, c->origin,
                            c->xyz_d.as<double>(), c->lw_d.as<double>(), c->box_d.as<int32_t>(),
                            c->stream));
  if (c->inc_ns > 0) {
    // a segment centre belongs to the cell floor((x - origin) / h), clamped
    std::vector<int32_t> cellof(np);
    for (int64_t p = 0; p < Nv; ++p) cellof[p] = (int32_t)p;
    for (int32_t i = 0; i < c->inc_ns; ++i) {
      int64_t nat = 0, stride = 1;
      for (int a = 0; a < 2; ++a) {
        int64_t k = (int64_t)std::floor((c->inc_xy[2 * i + a] - c->origin[a]) / c->h);
        k = std::min<int64_t>(std::max<int64_t>(k, 0), c->ncell[a] - 1);
        nat += k * stride;
        stride *= c->ncell[a];
      }
      cellof[Nv + i] = c->geo.ipos[nat];
    }
    upload(c->cellof_d, cellof);
  } else {
    c->cellof_d.release();
  }
  eval_self_terms(c);
  c->box_h.resize(np);
  HBI_HIP(hipMemcpyAsync(c->box_h.data(), c->box_d.p, sizeof(int32_t) * np,
                         hipMemcpyDeviceToHost, c->stream));
  HBI_HIP(hipStreamSynchronize(c->stream));
  c->t_geo = now_s() - t0;
}

// ---------------------------------------------------------------------------
// Batched hb_entry (+ optional interpolative decomposition) on the GPU.
// ---------------------------------------------------------------------------
struct BlockIn {
  const int32_t *rows; int32_t m;
  const int32_t *cols; int32_t n;
  double2 *out;        // entry-only blocks: destination (column-major, ld m)
};

struct BlockOut {
  int32_t rank = 0;
  std::vector<int32_t> piv;   // first `rank` pivots
  const double2 *X = nullptr; // device, rank x n (valid until the next batch)
};

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// Widest block of the Gram-matrix ID path: its per-column LDS (28 B) within
// a workgroup's share.
static int id_gram_nmax() { return 4096; }
// Smallest build tolerance of the Gram-matrix ID path (HBI_ID_GRAM_MIN_TOL
// overrides it).  Forming A^H A costs the remaining column norms an absolute
// error of about sqrt(k eps) |a_j| after k steps (1.5e-7 of the column at
// k = 100), the order of the stopping threshold at tol 1e-7: measured on
// the 1024^2 bump in FP64 at tol 1e-7 it gives 1.49e-7 against the oracle
// where the pivoted QR gives 1.37e-7, with 0.2 % more factor entries, and
// builds in 9.0 s instead of 13.2 s.  At tol 1e-9 it fell short of the
// tolerance (1.05e-6 on a gradient that the pivoted QR computes to 1e-7), so
// tighter builds keep the pivoted QR of A itself.
constexpr double kGramMinTol = 1e-7;
static double gram_min_tol() {
  const char *e = std::getenv("HBI_ID_GRAM_MIN_TOL");
  return e && std::atof(e) > 0 ? std::atof(e) : kGramMinTol;
}

// Which kernels decompose the blocks (HBI_ID_KERNEL, for comparisons):
// by default blocks of at most HBI_ID_ONCHIP_NMAX columns on chip and wider
// ones by the global-memory pivoted QR (k_cpqr); "global" sends every block
// to k_cpqr, "blocked" every block to its panel form (k_cpqr_blocked, which
// measured slower than k_cpqr on the 2D and 3D workloads).
// "cpqr" keeps the default's on-chip kernel for narrow blocks but sends
// every wider block to k_cpqr instead of the Gram-matrix path.
enum IdKernels { ID_AUTO = 0, ID_GLOBAL = 1, ID_BLOCKED = 2, ID_CPQR = 3 };
static IdKernels id_kernels() {
  const char *e = std::getenv("HBI_ID_KERNEL");
  if (e && std::strcmp(e, "global") == 0) return ID_GLOBAL;
  if (e && std::strcmp(e, "blocked") == 0) return ID_BLOCKED;
  if (e && std::strcmp(e, "cpqr") == 0) return ID_CPQR;
  return ID_AUTO;
}

// entry tile shape (rows of one table box x columns), as k_entries takes it:
// 16 columns in 2D, 32 in 3D
constexpr int32_t kEntryTileRows = 128;
static int32_t entry_tile_cols(int dim) { return dim == 3 ? 32 : 16; }

// One GPU batch of blocks.  prep() does all of its host-side set-up into a
// pinned staging buffer without touching device memory; submit() sizes the
// workspace, writes the device pointers, uploads and launches; finish()
// waits and reads the ranks and pivots back.  Two staging buffers let the
// host prepare batch j + 1 while the GPU runs batch j.
struct Prepared {
  const std::vector<BlockIn> *blocks = nullptr;
  std::vector<BlockOut> *outs = nullptr;
  std::function<void(int64_t, int64_t)> on_batch;   // after finish(), X still in the workspace
  int64_t i0 = 0, i1 = 0, nb = 0;
  int sbuf = 0;
  bool id = false;
  size_t ws_used = 0, idx_bytes = 0, up_bytes = 0;
  size_t o_rows = 0, o_cols = 0, o_slot = 0, o_wc = 0, o_tl = 0, o_ro = 0, o_eb = 0, o_ib = 0,
         o_sel = 0, o_piv = 0, o_rank = 0;
  int64_t ncw = 0, ntiles = 0, po = 0;
  int64_t nsel[3] = {0, 0, 0};
  int nmax_g[3] = {1, 1, 1}, mmax_w = 1;
  IdKernels idk = ID_AUTO;
  double tol = 0;
  std::vector<int64_t> wsoff, pivoff;
  std::vector<int32_t> nslot;   // table slots per block of the batch
  double t_submit = 0;
};

struct Batcher {
  hbi_ctx *c;
  HostBuf stage[2];   // pinned staging: uploads and the rank/pivot read-back
  explicit Batcher(hbi_ctx *ctx) : c(ctx) {}

  // bytes of workspace a block needs
  size_t ws_need(int32_t m, int32_t n, int nslot, bool id) const {
    size_t b = c->hc_cache.p ? 0 : align256((size_t)n * nslot * 3 * c->NTb * sizeof(double));
    if (id) b += align256((size_t)m * n * sizeof(double2)) +
                 align256((size_t)std::min(m, n) * n * sizeof(double2));
    return b;
  }

  int count_slots(const BlockIn &b, std::vector<int32_t> &slotbox) const {
    slotbox.clear();
    for (int32_t i = 0; i < b.m; ++i) {
      const int32_t bx = c->box_h[b.rows[i]];
      if (std::find(slotbox.begin(), slotbox.end(), bx) == slotbox.end()) slotbox.push_back(bx);
    }
    return (int)slotbox.size();
  }

  // Table slots of every block and the batch boundaries under the workspace
  // budget; with `pairs`, blocks 2q and 2q+1 always go to the same batch.
  struct Plan {
    std::vector<std::vector<int32_t>> slots;
    std::vector<int> nslot;
    std::vector<std::pair<int64_t, int64_t>> batches;
  };
  Plan plan(const std::vector<BlockIn> &blocks, bool id, bool pairs) const {
    Plan pl;
    const int64_t nb = (int64_t)blocks.size();
    const size_t budget = (size_t)c->wsbytes();
    pl.slots.resize(nb);
    pl.nslot.resize(nb);
    parallel_for(nb, [&](int64_t a, int64_t b) {
      for (int64_t i = a; i < b; ++i) pl.nslot[i] = count_slots(blocks[i], pl.slots[i]);
    });
    const int step = pairs ? 2 : 1;
    int64_t i0 = 0;
    while (i0 < nb) {
      size_t used = 0;
      int64_t i1 = i0;
      while (i1 < nb) {
        size_t need = 0;
        for (int q = 0; q < step && i1 + q < nb; ++q)
          need += ws_need(blocks[i1 + q].m, blocks[i1 + q].n, pl.nslot[i1 + q], id);
        if (need > budget)
          throw Error{HBI_ERR_OOM, "a single block (m=" + std::to_string(blocks[i1].m) + ", n=" +
                                       std::to_string(blocks[i1].n) + ") exceeds the workspace"};
        if (used + need > budget) break;
        used += need;
        i1 = std::min<int64_t>(nb, i1 + step);
      }
      pl.batches.push_back({i0, i1});
      i0 = i1;
    }
    return pl;
  }

  // Runs batches handed out by next(P) (false when there are none left):
  // batch j + 1 is prepared on the host while the GPU runs batch j.
  template <class Next>
  void pipeline(Next &&next) {
    Prepared pa, pb;
    Prepared *cur = &pa, *nxt = &pb;
    int sb = 0;
    cur->sbuf = sb;
    try {
      bool have = next(*cur);
      while (have) {
        submit(*cur);
        sb ^= 1;
        *nxt = Prepared();
        nxt->sbuf = sb;
        const bool have2 = next(*nxt);
        finish(*cur);
        std::swap(cur, nxt);
        have = have2;
      }
    } catch (...) {
      // no staging buffer or workspace may go while a copy or kernel uses it
      (void)hipStreamSynchronize(c->stream);
      throw;
    }
  }

  // Process blocks [0, nb) in as many GPU batches as the workspace needs.
  // id = true: evaluate into the workspace and run the ID, fill outs.
  // id = false: evaluate straight into blocks[i].out.
  // `on_batch(first, count)` is called after each ID batch while its X
  // matrices are still in the workspace.
  template <class CB>
  void run(const std::vector<BlockIn> &blocks, bool id, double tol, std::vector<BlockOut> *outs,
           CB &&on_batch, bool pairs = false) {
    const Plan pl = plan(blocks, id, pairs);
    size_t j = 0;
    pipeline([&](Prepared &P) {
      if (j == pl.batches.size()) return false;
      prep(P, blocks, pl, pl.batches[j].first, pl.batches[j].second, id, tol);
      ++j;
      P.outs = outs;
      P.on_batch = on_batch;
      return true;
    });
  }

  // Host-side set-up of blocks [i0, i1) into staging buffer P.sbuf.
  void prep(Prepared &P, const std::vector<BlockIn> &blocks, const Plan &pl, int64_t i0,
            int64_t i1, bool id, double tol) {
    const double tb = now_s();
    P.tol = tol;
    P.blocks = &blocks;
    P.i0 = i0; P.i1 = i1; P.id = id;
    const int64_t nb = i1 - i0;
    P.nb = nb;
    const auto &slots = pl.slots;
    const auto &nslot = pl.nslot;
    // offsets of every block's rows, columns, slots and column-side work
    std::vector<int64_t> ro(nb + 1, 0), co(nb + 1, 0), so(nb + 1, 0), wco(nb + 1, 0), to(nb + 1, 0);
    P.pivoff.assign(nb + 1, 0);
    P.wsoff.assign(nb + 1, 0);
    P.nslot.assign(nslot.begin() + i0, nslot.begin() + i1);
    for (int64_t q = 0; q < nb; ++q) {
      const BlockIn &b = blocks[i0 + q];
      const int ns = nslot[i0 + q];
      ro[q + 1] = ro[q] + b.m;
      co[q + 1] = co[q] + b.n;
      so[q + 1] = so[q] + ns;
      wco[q + 1] = wco[q] + (int64_t)b.n * ns;
      P.pivoff[q + 1] = P.pivoff[q] + (id ? b.n : 0);
      P.wsoff[q + 1] = P.wsoff[q] + (int64_t)ws_need(b.m, b.n, ns, id);
    }
    P.ws_used = (size_t)P.wsoff[nb];
    const int64_t nrows = ro[nb], ncols = co[nb], nsl = so[nb], ncw = wco[nb], po = P.pivoff[nb];
    P.ncw = ncw;
    P.po = po;
    // rows in slot order (counting sort) and the number of entry tiles
    // (kEntryTileRows rows of one slot x tcols columns) per block
    const int32_t tcols = entry_tile_cols(c->dim);
    std::vector<int32_t> rslot(nrows);
    std::vector<int64_t> ntile(nb);
    // ID kernel per block: on chip up to HBI_ID_ONCHIP_NMAX columns (group
    // 0); wider blocks with at least as many rows as columns through their
    // Gram matrix (group 1), the others by the global-memory pivoted QR
    // (group 2); sel lists the groups.
    std::vector<int32_t> sel;
    P.idk = id ? id_kernels() : ID_AUTO;
    if (id) {
      std::vector<int32_t> g[3];
      const int gram_nmax = id_gram_nmax();
      const double gram_tol = gram_min_tol();
      for (int64_t q = 0; q < nb; ++q) {
        const BlockIn &b = blocks[i0 + q];
        int k = (P.idk == ID_AUTO || P.idk == ID_CPQR) && b.n <= HBI_ID_ONCHIP_NMAX ? 0 : 2;
        if (k == 2 && P.idk == ID_AUTO && tol >= gram_tol && b.m >= b.n && b.n <= gram_nmax)
          k = 1;
        g[k].push_back((int32_t)q);
        P.nmax_g[k] = std::max(P.nmax_g[k], (int)b.n);
        if (k == 2) P.mmax_w = std::max(P.mmax_w, (int)b.m);
      }
      for (int k = 0; k < 3; ++k) {
        P.nsel[k] = (int64_t)g[k].size();
        sel.insert(sel.end(), g[k].begin(), g[k].end());
      }
    }
    // the tile count needs the slot runs: first pass over the rows
    parallel_for(nb, [&](int64_t qa, int64_t qb) {
      std::vector<int32_t> cnt;
      for (int64_t q = qa; q < qb; ++q) {
        const BlockIn &b = blocks[i0 + q];
        const std::vector<int32_t> &sl = slots[i0 + q];
        const int ns = nslot[i0 + q];
        cnt.assign(ns + 1, 0);
        int32_t *rs = rslot.data() + ro[q];
        for (int32_t i = 0; i < b.m; ++i) {
          const int32_t bx = c->box_h[b.rows[i]];
          rs[i] = (int32_t)(std::find(sl.begin(), sl.end(), bx) - sl.begin());
          cnt[rs[i] + 1] += 1;
        }
        int64_t nt = 0;
        const int64_t cj = (b.n + tcols - 1) / tcols;
        for (int s2 = 0; s2 < ns; ++s2)
          nt += (cnt[s2 + 1] + kEntryTileRows - 1) / kEntryTileRows * cj;
        ntile[q] = nt;
      }
    });
    for (int64_t q = 0; q < nb; ++q) to[q + 1] = to[q] + ntile[q];
    const int64_t ntiles = to[nb];
    P.ntiles = ntiles;
    // staging layout: rows, cols, slotbox, workc, tiles, rord, eb, ib, sel
    // (uploaded), then piv and rank (read back)
    size_t off = 0;
    auto place = [&](size_t bytes) { size_t o = off; off = align256(off + bytes); return o; };
    P.o_rows = place(nrows * 4); P.o_cols = place(ncols * 4); P.o_slot = place(nsl * 4);
    P.o_wc = place(ncw * 8); P.o_tl = place(ntiles * sizeof(ETile)); P.o_ro = place(nrows * 4);
    P.o_eb = place(nb * sizeof(EntryBlock)); P.o_ib = place(id ? nb * sizeof(IdBlock) : 0);
    P.o_sel = place(id ? (size_t)nb * 4 : 0); P.o_piv = place((size_t)po * 4);
    P.o_rank = place((size_t)nb * 4);
    P.idx_bytes = off;
    P.up_bytes = P.o_piv;
    HBI_HIP(stage[P.sbuf].reserve(off));
    char *st = stage[P.sbuf].as<char>();
    int32_t *rows = (int32_t *)(st + P.o_rows), *cols = (int32_t *)(st + P.o_cols),
            *slotbox = (int32_t *)(st + P.o_slot), *workc = (int32_t *)(st + P.o_wc),
            *rord = (int32_t *)(st + P.o_ro);
    ETile *tiles = (ETile *)(st + P.o_tl);
    if (id) std::memcpy(st + P.o_sel, sel.data(), sel.size() * 4);
    parallel_for(nb, [&](int64_t qa, int64_t qb) {
      std::vector<int32_t> cnt;
      for (int64_t q = qa; q < qb; ++q) {
        const BlockIn &b = blocks[i0 + q];
        const std::vector<int32_t> &sl = slots[i0 + q];
        const int ns = nslot[i0 + q];
        const int32_t *rs = rslot.data() + ro[q];
        // rows in slot order
        cnt.assign(ns + 1, 0);
        for (int32_t i = 0; i < b.m; ++i) cnt[rs[i] + 1] += 1;
        for (int s2 = 0; s2 < ns; ++s2) cnt[s2 + 1] += cnt[s2];
        int32_t *rq = rord + ro[q];
        for (int32_t i = 0; i < b.m; ++i) rq[cnt[rs[i]]++] = i;
        std::copy(b.rows, b.rows + b.m, rows + ro[q]);
        std::copy(b.cols, b.cols + b.n, cols + co[q]);
        std::copy(sl.begin(), sl.end(), slotbox + so[q]);
        int32_t *w = workc + 2 * wco[q];
        for (int32_t j = 0; j < b.n; ++j)
          for (int s2 = 0; s2 < ns; ++s2) {
            *w++ = (int32_t)q;
            *w++ = j * ns + s2;
          }
        // tiles: slot runs of the sorted rows
        ETile *t = tiles + to[q];
        int32_t r0 = 0;
        while (r0 < b.m) {
          const int s2 = rs[rq[r0]];
          int32_t r1 = r0;
          while (r1 < b.m && rs[rq[r1]] == s2) ++r1;
          for (int32_t a = r0; a < r1; a += kEntryTileRows)
            for (int32_t j0 = 0; j0 < b.n; j0 += tcols)
              *t++ = ETile{(int32_t)q, a, std::min(kEntryTileRows, r1 - a), j0,
                           std::min(tcols, b.n - j0), s2};
          r0 = r1;
        }
      }
    });
    for (int64_t q = 0; q < nb; ++q) c->entries_eval += (int64_t)blocks[i0 + q].m * blocks[i0 + q].n;
    c->entry_slots += ntiles * kEntryTileRows * tcols;
    for (int k = 0; k < 3; ++k) c->nid_path[k] += P.nsel[k];
    c->t_prep += now_s() - tb;   // host-side set-up of the batch
  }

  // Workspace and index buffer sized for P (the previous batch has
  // finished), device pointers written into the staging copy of the block
  // descriptors, upload and launches.
  void submit(Prepared &P) {
    P.t_submit = now_s();
    const std::vector<BlockIn> &blocks = *P.blocks;
    HBI_HIP(c->ws.reserve(P.ws_used));
    HBI_HIP(c->idx_d.reserve(P.idx_bytes));
    char *ix = c->idx_d.as<char>();
    char *ws = c->ws.as<char>();
    char *st = stage[P.sbuf].as<char>();
    EntryBlock *eb = (EntryBlock *)(st + P.o_eb);
    IdBlock *ib = (IdBlock *)(st + P.o_ib);
    int64_t ro = 0, co = 0, so = 0;
    for (int64_t q = 0; q < P.nb; ++q) {
      const BlockIn &b = blocks[P.i0 + q];
      const int32_t ns = P.nslot[q];
      EntryBlock e{};
      e.row_off = ro; e.col_off = co; e.slot_off = so;
      e.m = b.m; e.n = b.n; e.nslot = ns;
      size_t wso = (size_t)P.wsoff[q];
      e.hc_off = (int64_t)(wso / sizeof(double));
      if (!c->hc_cache.p) wso += align256((size_t)b.n * ns * 3 * c->NTb * sizeof(double));
      if (P.id) {
        IdBlock d{};
        d.A = (double2 *)(ws + wso);
        wso += align256((size_t)b.m * b.n * sizeof(double2));
        d.X = (double2 *)(ws + wso);
        d.m = b.m; d.n = b.n;
        d.piv = (int32_t *)(ix + P.o_piv) + P.pivoff[q];
        ib[q] = d;
        e.out = d.A;
      } else {
        e.out = b.out;
      }
      eb[q] = e;
      ro += b.m; co += b.n; so += ns;
    }
    HBI_HIP(hipMemcpyAsync(ix, st, P.up_bytes, hipMemcpyHostToDevice, c->stream));
    const DevProblem Pr = c->devprob();
    const DevCells C = c->devcells();
    const DevTables T = c->devtables();
    const double *hcache = c->hc_cache.as<double>();
    if (!hcache)
      HBI_HIP(launch_colside(Pr, C, T, (const EntryBlock *)(ix + P.o_eb),
                             (const int32_t *)(ix + P.o_wc), P.ncw, (const int32_t *)(ix + P.o_cols),
                             (const int32_t *)(ix + P.o_slot), c->ws.as<double>(), c->stream));
    HBI_HIP(launch_entries(Pr, C, (const EntryBlock *)(ix + P.o_eb), (const ETile *)(ix + P.o_tl),
                           P.ntiles, (const int32_t *)(ix + P.o_rows),
                           (const int32_t *)(ix + P.o_ro), (const int32_t *)(ix + P.o_cols),
                           c->ws.as<double>(), (const int32_t *)(ix + P.o_slot), hcache,
                           c->hc_nbox, c->stream));
    if (P.id) {
      const IdBlock *ibd = (const IdBlock *)(ix + P.o_ib);
      const int32_t *seld = (const int32_t *)(ix + P.o_sel);
      int32_t *rankd = (int32_t *)(ix + P.o_rank);
      HBI_HIP(launch_id_onchip(ibd, seld, P.nsel[0], P.nmax_g[0], P.tol, rankd, c->stream));
      HBI_HIP(launch_id_gram(ibd, seld + P.nsel[0], P.nsel[1], P.nmax_g[1], P.tol, rankd, c->stream));
      if (P.idk == ID_BLOCKED)
        HBI_HIP(launch_cpqr_blocked(ibd, seld + P.nsel[0] + P.nsel[1], P.nsel[2], P.nmax_g[2],
                                    P.mmax_w, P.tol, rankd, c->stream));
      else
        HBI_HIP(launch_cpqr(ibd, seld + P.nsel[0] + P.nsel[1], P.nsel[2], P.nmax_g[2], P.mmax_w,
                            P.tol, rankd, c->stream));
      // pivots and ranks back into the same staging buffer
      HBI_HIP(hipMemcpyAsync(st + P.o_piv, ix + P.o_piv, P.idx_bytes - P.o_piv,
                             hipMemcpyDeviceToHost, c->stream));
    }
  }

  // Wait for P, take its ranks and pivots, then the caller's compaction.
  void finish(Prepared &P) {
    HBI_HIP(hipStreamSynchronize(c->stream));
    c->t_wait += now_s() - P.t_submit;
    if (P.id) {
      const char *st = stage[P.sbuf].as<char>();
      const IdBlock *ib = (const IdBlock *)(st + P.o_ib);
      const int32_t *rank = (const int32_t *)(st + P.o_rank);
      const int32_t *piv = (const int32_t *)(st + P.o_piv);
      for (int64_t q = 0; q < P.nb; ++q) {
        BlockOut &o = (*P.outs)[P.i0 + q];
        o.rank = rank[q];
        if (o.rank < 1 || o.rank > std::min(ib[q].m, ib[q].n))
          throw Error{HBI_ERR_NUMERIC, "interpolative decomposition returned an invalid rank"};
        o.piv.assign(piv + P.pivoff[q], piv + P.pivoff[q] + o.rank);
        o.X = ib[q].X;
        c->nid += 1;
        c->rank_max = std::max(c->rank_max, o.rank);
        c->rank_sum += o.rank;
        c->id_m_max = std::max(c->id_m_max, ib[q].m);
        c->id_m_sum += ib[q].m;
        c->id_n_sum += ib[q].n;
        // complex multiply-adds of the Householder steps actually taken
        double wk = 0.0;
        for (int32_t k = 0; k < o.rank; ++k)
          wk += 2.0 * (double)(ib[q].m - k) * (double)(ib[q].n - k - 1);
        c->id_work += wk;
        if (ib[q].n > 64) { c->id_work_wide += wk; c->nid_wide += 1; }
        if (ib[q].n > 128) c->id_work_128 += wk;
      }
      const double tc = now_s();
      if (P.on_batch) P.on_batch(P.i0, P.nb);
      c->t_compact += now_s() - tc;
    }
  }
};

struct BF { int lev; int64_t oi, si; int L; };

struct LevelState {
  std::vector<int32_t> rank;
  std::vector<int64_t> skel_off;   // into skel, size nblk+1
  std::vector<int32_t> skel;       // tree positions
  std::vector<int64_t> foff;
  std::vector<int64_t> ioff;   // transfer blocks: the pair's index lists
  std::vector<int64_t> zoff;
  void reset(int64_t nblk) {
    rank.assign(nblk, 0); skel_off.assign(nblk + 1, 0); skel.clear();
    foff.assign(nblk, 0); ioff.assign(nblk, -1); zoff.assign(nblk, 0);
  }
};

// The column-side cache: Nv * nbox * 3 * NTb doubles, used when at most
// HBI_HC_CACHE_BYTES (default 16 GiB) and a quarter of the free device memory.
// Each cell then gets its column side once instead of once per block.
static void fill_hc_cache(hbi_ctx *c) {
  c->hc_cache.release();
  c->hc_nbox = 0;
  const int nbox = c->NT / c->NTb;
  const int64_t Nv = c->geo.Nv;
  const size_t bytes = (size_t)Nv * nbox * 3 * c->NTb * sizeof(double);
  size_t cap = (size_t)16 << 30;
  if (const char *e = std::getenv("HBI_HC_CACHE_BYTES")) cap = (size_t)std::strtoull(e, nullptr, 10);
  size_t fr = 0, tot = 0;
  if (hipMemGetInfo(&fr, &tot) != hipSuccess) { (void)hipGetLastError(); return; }
  if (bytes == 0 || bytes > cap || bytes > fr / 4) return;
  if (c->hc_cache.alloc(bytes) != hipSuccess) return;   // not fatal: per-block path
  HBI_HIP(launch_colside_cells(c->devprob(), c->devcells(), c->devtables(), Nv, nbox,
                               c->hc_cache.as<double>(), c->stream));
  c->hc_nbox = nbox;
}

struct HcCacheScope {
  hbi_ctx *c;
  ~HcCacheScope() { c->hc_cache.release(); c->hc_nbox = 0; }
};

int env_int(const char *name, int def) {
  const char *e = std::getenv(name);
  if (!e || !*e) return def;
  char *end = nullptr;
  const long v = std::strtol(e, &end, 10);
  return (end && *end == 0) ? (int)v : def;
}

// Units with more candidate columns than this get forward windows of 16
// rows, four lanes a row (HBI_WSTAGE_WIDE_C, default 256).
int wide_columns() { return env_int("HBI_WSTAGE_WIDE_C", 256); }
int window_rows(const WUnit &U, int wide_c) { return U.c > wide_c && U.ra + U.rb > 32 ? 16 : 64; }

// Final layout of the factor store.  The build leaves its blocks in chunks
// in production order; the store places each block where its apply kernel
// streams it, so that waves running at the same time read neighbouring
// memory:
//   V^0 blocks   leaf-major, level-minor (one workgroup per leaf);
//   W^k units    per level, in the order of the forward stage's work items
//                (heaviest first);
//   leaf blocks  per leaf: the dense block, then its K^L blocks by level.
// Every block offset (vd, units, leaves, kd) is rewritten to the new place;
// the returned descriptors copy each block from its chunk.
std::vector<PlaceDesc> layout_store(const std::vector<Chunk> &chunks, int Lv, int64_t nleaf,
                                    std::vector<VDesc> &vd, std::vector<KDesc> &kd,
                                    std::vector<LeafInfo> &leaves,
                                    std::vector<std::vector<WUnit>> &units, int64_t Fg) {
  const int wide_c = wide_columns();
  // chunks are in store order (appended as the store grows)
  auto src = [&](int64_t off, int64_t n) -> const double2 * {
    auto it = std::upper_bound(chunks.begin(), chunks.end(), off,
                               [](int64_t o, const Chunk &ch) { return o < ch.goff; });
    if (it == chunks.begin() || off + n > (it - 1)->goff + (it - 1)->count)
      throw Error{HBI_ERR_NUMERIC, "internal layout error in the factor store"};
    return (it - 1)->buf.as<double2>() + (off - (it - 1)->goff);
  };
  std::vector<PlaceDesc> out;
  int64_t cur = 0;
  auto place = [&](int64_t &foff, int64_t n) {
    if (n > 0) out.push_back(PlaceDesc{src(foff, n), cur, n});
    foff = cur;
    cur += n;
  };
  for (int64_t g = 0; g < nleaf; ++g)
    for (int l = 0; l < Lv; ++l) {
      VDesc &d = vd[g * Lv + l];
      place(d.foff, (int64_t)d.r * (leaves[g].size - d.r));
    }
  for (size_t k = 1; k < units.size(); ++k) {
    std::vector<WUnit> &us = units[k];
    // a unit's first forward item is its heaviest (64-row windows); items
    // of equal weight keep the unit order
    std::vector<std::pair<int64_t, int32_t>> ord(us.size());
    for (size_t u = 0; u < us.size(); ++u) {
      const int Rt = us[u].ra + us[u].rb;
      const int wr = window_rows(us[u], wide_c);   // as the work items
      ord[u] = {(int64_t)std::min(Rt, wr) * us[u].c, (int32_t)u};
    }
    std::stable_sort(ord.begin(), ord.end(), [](const std::pair<int64_t, int32_t> &a,
                                                const std::pair<int64_t, int32_t> &b) {
      return a.first > b.first;
    });
    for (const auto &o : ord) {
      WUnit &U = us[o.second];
      place(U.foff, (int64_t)U.ra * (U.c - U.ra) + (int64_t)U.rb * (U.c - U.rb));
    }
  }
  for (int64_t g = 0; g < nleaf; ++g) {
    const int64_t sz = leaves[g].size;
    place(leaves[g].dense_off, sz * sz);
    for (int l = 0; l < Lv; ++l) {
      KDesc &d = kd[g * Lv + l];
      place(d.foff, sz * d.r);
    }
  }
  if (cur != Fg) throw Error{HBI_ERR_NUMERIC, "internal layout error: factor store size"};
  return out;
}

// The apply plan of a finished build: descriptors on the device, the work
// items of every transfer stage, and the algorithmic traffic of each launch.
void make_apply_plan(hbi_ctx *c, std::vector<LeafInfo> &leaves, std::vector<VDesc> &vd,
                     std::vector<KDesc> &kd, std::vector<std::vector<WUnit>> &units, int Lv,
                     int Lmax) {
  const int64_t nleaf = (int64_t)leaves.size();
  const int wide_c = wide_columns();
  // LDS entries of one forward wave for a unit of c columns: the raw inputs
  // and both column orders (4 bytes per column)
  const int esz = c->prec == HBI_F64 ? 16 : 8;
  const int lds_max = HBI_WSTAGE_LDS_BYTES / esz;
  const int cap_lds = std::max(0, std::min(env_int("HBI_WSTAGE_LDS_CAP", lds_max), lds_max));
  auto slice = [&](int cc) { return cc + (4 * cc + esz - 1) / esz; };
  for (int k = 1; k <= Lmax; ++k)
    for (const WUnit &U : units[k])
      if (U.ioff % 2 != 0) throw Error{HBI_ERR_NUMERIC, "internal layout error: index alignment"};
  upload(c->leaves_d, leaves);
  upload(c->vd_d, vd);
  upload(c->kd_d, kd);
  c->leaves_h = leaves;
  c->vd_h = vd;
  c->kd_h = kd;
  c->units_h = units;
  c->units_d.clear();
  c->units_d.resize(Lmax + 1);
  c->plan = ApplyPlan();
  ApplyPlan &ap = c->plan;
  ap.Lv = Lv;
  ap.Lmax = Lv >= 1 ? Lmax : 0;
  ap.nleaf = nleaf;
  ap.leaves = c->leaves_d.as<LeafInfo>();
  ap.perm = c->perm_d.as<int32_t>();
  ap.vd = c->vd_d.as<VDesc>();
  ap.kd = c->kd_d.as<KDesc>();
  ap.fidx = c->Fi.as<uint16_t>();
  ap.cap_lds = cap_lds;
  ap.units.assign(Lmax + 1, nullptr);
  ap.nunits.assign(Lmax + 1, 0);
  c->items_d.clear();
  c->items_d.resize(Lmax + 1);
  c->items_adj_d.clear();
  c->items_adj_d.resize(Lmax + 1);
  ap.items.assign(Lmax + 1, nullptr);
  ap.items_adj.assign(Lmax + 1, nullptr);
  ap.nitems.assign(Lmax + 1, 0);
  ap.nitems_adj.assign(Lmax + 1, 0);
  ap.w_elems.assign(Lmax + 1, 0.0);
  ap.w_idx.assign(Lmax + 1, 0.0);
  c->wst_lds = c->wst_global = c->wst_wide = 0;
  for (int k = 1; k <= Lmax; ++k) {
    upload(c->units_d[k], units[k]);
    ap.units[k] = c->units_d[k].as<WUnit>();
    ap.nunits[k] = (int64_t)units[k].size();
    // forward: windows of 64 (or 16) rows of every unit; adjoint: windows
    // of 64 columns; heaviest first so the long items do not form the tail
    std::vector<std::pair<int64_t, WItem>> fw, bw;
    for (int32_t u = 0; u < (int32_t)units[k].size(); ++u) {
      const WUnit &U = units[k][u];
      const int Rt = U.ra + U.rb;
      const int wr = window_rows(U, wide_c);
      auto item = [&U](int32_t off, int32_t w) {
        return WItem{U.foff, U.zin, U.zouta, U.zoutb, U.ioff, U.ra, U.rb, U.c, (int16_t)off,
                     (int16_t)w};
      };
      for (int r0 = 0; r0 < Rt; r0 += wr) {
        const int r1 = Rt <= 32 ? Rt : std::min(Rt, r0 + wr);
        fw.push_back({(int64_t)(r1 - r0) * U.c, item(Rt <= 32 ? 0 : r0, wr)});
        if (slice(U.c) <= cap_lds) ++c->wst_lds; else ++c->wst_global;
        if (wr == 16) ++c->wst_wide;
        if (Rt <= 32) break;
      }
      for (int c0 = 0; c0 < U.c; c0 += 64)
        bw.push_back({(int64_t)std::min(64, U.c - c0) * Rt, item(c0, 64)});
      // traffic of the unit: T of both children, its c inputs and Rt
      // outputs; the two column orders the inputs are gathered through
      ap.w_elems[k] += (double)U.ra * (U.c - U.ra) + (double)U.rb * (U.c - U.rb) + U.c + Rt;
      ap.w_idx[k] += 2.0 * sizeof(uint16_t) * U.c;
    }
    auto order = [](std::vector<std::pair<int64_t, WItem>> &v) {
      std::stable_sort(v.begin(), v.end(), [](const std::pair<int64_t, WItem> &a,
                                              const std::pair<int64_t, WItem> &b) {
        return a.first > b.first;
      });
      std::vector<WItem> out(v.size());
      for (size_t q = 0; q < v.size(); ++q) out[q] = v[q].second;
      return out;
    };
    upload(c->items_d[k], order(fw));
    upload(c->items_adj_d[k], order(bw));
    ap.items[k] = c->items_d[k].as<WItem>();
    ap.items_adj[k] = c->items_adj_d[k].as<WItem>();
    ap.nitems[k] = (int64_t)fw.size();
    ap.nitems_adj[k] = (int64_t)bw.size();
    ap.w_idx[k] += (double)sizeof(WItem) * ap.nitems[k];
  }
  {
    std::vector<int32_t> cs;
    for (int k = 1; k <= Lmax; ++k)
      for (const WUnit &U : units[k]) cs.push_back(U.c);
    std::sort(cs.begin(), cs.end());
    for (int q = 0; q < 5; ++q)
      c->wst_cq[q] = cs.empty() ? 0 : cs[std::min(cs.size() - 1, (size_t)(q * (cs.size() - 1) / 4))];
  }
  // traffic of the V^0 and final launches (complex elements + index bytes)
  double ve = 0, vi = 0, fe = 0, fi = 0;
  for (int64_t g = 0; g < nleaf; ++g) {
    const double sz = leaves[g].size;
    vi += sizeof(LeafInfo) + 4.0 * sz;
    fi += sizeof(LeafInfo) + 4.0 * sz;
    if (Lv > 0) ve += sz;                 // s read by the V stage
    fe += sz * sz + 2.0 * sz;             // dense leaf, s read, u written
    for (int l = 0; l < Lv; ++l) {
      const VDesc &v = vd[g * Lv + l];
      const KDesc &q = kd[g * Lv + l];
      ve += (double)v.r * (sz - v.r) + v.r;
      fe += (double)q.r * sz + q.r;
      vi += sizeof(VDesc) + sizeof(uint16_t) * sz;   // descriptor, column order
      fi += sizeof(KDesc);
    }
  }
  ap.v_elems = ve; ap.v_idx = vi; ap.f_elems = fe; ap.f_idx = fi;
  c->zalloc = c->ztotal;
  HBI_HIP(c->z_d.alloc((size_t)esz * std::max<int64_t>(c->zalloc, 1)));
}

void build_factors(hbi_ctx *c, double tol) {
  const double tb0 = now_s();
  if (c->geo_leaf != c->leaf() || c->geo_band != c->band()) setup_cells(c);
  HcCacheScope hc_scope{c};
  fill_hc_cache(c);
  Geometry &G = c->geo;
  const int Lv = G.Lv;
  const int64_t nleaf = (int64_t)1 << Lv;
  std::vector<BF> bfs;
  for (int lev = 1; lev <= Lv; ++lev)
    for (int64_t p = 0; p < ((int64_t)1 << (lev - 1)); ++p) {
      bfs.push_back({lev, 2 * p, 2 * p + 1, Lv - lev});
      bfs.push_back({lev, 2 * p + 1, 2 * p, Lv - lev});
    }
  const int64_t nbf = (int64_t)bfs.size();
  const int Lmax = Lv >= 1 ? Lv - 1 : 0;
  std::vector<LevelState> prev(nbf), cur(nbf);
  std::vector<Chunk> chunks;
  int64_t Fg = 0;   // running global element offset
  std::vector<VDesc> vd((size_t)nleaf * Lv);
  std::vector<KDesc> kd((size_t)nleaf * Lv);
  std::vector<std::vector<WUnit>> units(Lmax + 1);
  ProxyParams pp;
  pp.chi = c->chi();
  pp.radius = c->radius();
  Batcher B(c);
  c->ztotal = 0;
  double t_host = 0, t_gpu = 0;

  // Compact the X matrices of an ID batch into a new chunk: only the
  // non-skeleton columns T of X = [I, T] Pi^T are kept.  Level 0 keeps T of
  // each V_{tau,nu} and appends its column order and inverse (ia, pa) to the
  // index store fi_h; higher levels keep, for the sibling pair (2t', j),
  // (2t'+1, j), T_a then T_b, and append (ia, ib, pa, pb).
  std::vector<uint16_t> fi_h;
  auto compact = [&](std::vector<BlockOut> &outs, int64_t first, int64_t cnt,
                     const std::vector<int32_t> &ncols, std::vector<int64_t> &foff_out,
                     std::vector<int64_t> &ioff_out, bool pairs) {
    int64_t tot = 0;
    for (int64_t q = 0; q < cnt; ++q)
      tot += (int64_t)outs[first + q].rank * (ncols[first + q] - outs[first + q].rank);
    Chunk ch;
    HBI_HIP(ch.buf.alloc(sizeof(double2) * std::max<int64_t>(tot, 1)));
    ch.goff = Fg;
    ch.count = tot;
    DevBuf d_d, ns_d;
    int64_t o = 0;
    // column order of one block (skeleton columns in pivot order, then the
    // others ascending) and its inverse
    std::vector<uint16_t> ord, inv;
    std::vector<uint8_t> mark;
    auto orders = [&](const BlockOut &x, int32_t cc) {
      mark.assign(cc, 0);
      ord.clear();
      for (int32_t k = 0; k < x.rank; ++k) { ord.push_back((uint16_t)x.piv[k]); mark[x.piv[k]] = 1; }
      for (int32_t j = 0; j < cc; ++j)
        if (!mark[j]) ord.push_back((uint16_t)j);
      if ((int32_t)ord.size() != cc) throw Error{HBI_ERR_NUMERIC, "internal error: repeated pivot"};
      inv.assign(cc, 0);
      for (int32_t k = 0; k < cc; ++k) inv[ord[k]] = (uint16_t)k;
    };
    if (!pairs) {
      // V^0 blocks: T of each, lists [ia, pa]
      std::vector<PairDesc> pd(cnt);
      std::vector<uint16_t> ns_h;
      std::vector<int64_t> nso(cnt);
      for (int64_t q = 0; q < cnt; ++q) {
        const BlockOut &x = outs[first + q];
        const int32_t cc = ncols[first + q];
        const int64_t io = (int64_t)fi_h.size();
        orders(x, cc);
        fi_h.insert(fi_h.end(), ord.begin(), ord.end());
        fi_h.insert(fi_h.end(), inv.begin(), inv.end());
        nso[q] = (int64_t)ns_h.size();
        ns_h.insert(ns_h.end(), ord.begin() + x.rank, ord.end());
        pd[q] = PairDesc{x.X, nullptr, ch.buf.as<double2>() + o, nullptr, nullptr, x.rank, 0,
                         cc, 0};
        foff_out[first + q] = Fg + o;
        ioff_out[first + q] = io;
        o += (int64_t)x.rank * (cc - x.rank);
      }
      upload(ns_d, ns_h);
      for (int64_t q = 0; q < cnt; ++q) pd[q].nsa = ns_d.as<uint16_t>() + nso[q];
      upload(d_d, pd);
      HBI_HIP(launch_pack_pairs(d_d.as<PairDesc>(), cnt, c->stream));
    } else {
      if (cnt % 2 != 0) throw Error{HBI_ERR_NUMERIC, "internal error: unpaired transfer block"};
      const int64_t np = cnt / 2;
      std::vector<PairDesc> pd(np);
      std::vector<uint16_t> ns_h;        // non-skeleton lists for the pack kernel
      std::vector<int64_t> nso(2 * np);
      for (int64_t q = 0; q < cnt; q += 2) {
        const BlockOut &a = outs[first + q], &b = outs[first + q + 1];
        const int32_t cc = ncols[first + q];
        if (ncols[first + q + 1] != cc) throw Error{HBI_ERR_NUMERIC, "internal error: pair width"};
        const int64_t io = (int64_t)fi_h.size();
        fi_h.resize(io + 4 * (int64_t)cc);
        for (int h = 0; h < 2; ++h) {
          const BlockOut &x = h ? b : a;
          orders(x, cc);
          std::copy(ord.begin(), ord.end(), fi_h.begin() + io + (int64_t)h * cc);
          std::copy(inv.begin(), inv.end(), fi_h.begin() + io + (int64_t)(2 + h) * cc);
          nso[q + h] = (int64_t)ns_h.size();
          ns_h.insert(ns_h.end(), ord.begin() + x.rank, ord.end());
        }
        const int64_t ea = (int64_t)a.rank * (cc - a.rank);
        pd[q / 2] = PairDesc{a.X, b.X, ch.buf.as<double2>() + o, nullptr, nullptr,
                             a.rank, b.rank, cc, 0};
        foff_out[first + q] = Fg + o;
        foff_out[first + q + 1] = Fg + o + ea;
        ioff_out[first + q] = io;
        ioff_out[first + q + 1] = io;
        o += ea + (int64_t)b.rank * (cc - b.rank);
      }
      upload(ns_d, ns_h);
      for (int64_t q = 0; q < np; ++q) {
        pd[q].nsa = ns_d.as<uint16_t>() + nso[2 * q];
        pd[q].nsb = ns_d.as<uint16_t>() + nso[2 * q + 1];
      }
      upload(d_d, pd);
      HBI_HIP(launch_pack_pairs(d_d.as<PairDesc>(), np, c->stream));
    }
    HBI_HIP(hipStreamSynchronize(c->stream));
    Fg += tot;
    chunks.push_back(std::move(ch));
  };

  for (int k = 0; k <= Lmax && Lv >= 1; ++k) {
    // enumerate blocks of level k in processing order
    struct Blk { int32_t b; int32_t t; int64_t j; };
    std::vector<Blk> blks;
    for (int64_t b = 0; b < nbf; ++b) {
      const int L = bfs[b].L;
      if (L < k) continue;
      cur[b].reset((int64_t)1 << L);
      if (k == 0) {
        for (int64_t j = 0; j < ((int64_t)1 << L); ++j) blks.push_back({(int32_t)b, 0, j});
      } else {
        for (int64_t tp = 0; tp < ((int64_t)1 << (k - 1)); ++tp)
          for (int64_t j = 0; j < ((int64_t)1 << (L - k)); ++j)
            for (int cc = 0; cc < 2; ++cc) blks.push_back({(int32_t)b, (int32_t)(2 * tp + cc), j});
      }
    }
    const int64_t nblk = (int64_t)blks.size();
    // per-block skeleton staging (filled as batches finish)
    std::vector<std::vector<int32_t>> skel_tmp(nblk);
    std::vector<int32_t> rank_tmp(nblk);
    std::vector<int64_t> foff_tmp(nblk), ioff_tmp(nblk);
    // Blocks go to the GPU in chunks of CH: proxy rows and candidate columns
    // on the host, then the chunk's batches.  The host builds chunk i + 1
    // and prepares every next batch while the GPU runs the current one.
    const int64_t CH = 16384;
    struct ChunkJob {
      int64_t c0 = 0, c1 = 0;
      std::vector<std::vector<int32_t>> rows, cands;
      std::vector<BlockIn> bin;
      std::vector<int32_t> ncols;
      std::vector<BlockOut> outs;
      std::vector<int64_t> foff_local, ioff_local;
      Batcher::Plan plan;
      size_t next = 0, done = 0;
    };
    auto make_chunk = [&](int64_t c0) {
      auto J = std::make_unique<ChunkJob>();
      J->c0 = c0;
      J->c1 = std::min(nblk, c0 + CH);
      const int64_t n = J->c1 - c0;
      const double th = now_s();
      auto &rows = J->rows;
      auto &cands = J->cands;
      rows.resize(n);
      cands.resize(n);
      parallel_for(n, [&](int64_t a, int64_t e) {
        std::vector<int32_t> stamp(G.Nv, 0);
        int32_t tag = 0;
        for (int64_t q = a; q < e; ++q) {
          const Blk &bk = blks[c0 + q];
          const BF &bf = bfs[bk.b];
          const int L = bf.L;
          std::vector<int32_t> &cd = cands[q];
          if (k == 0) {
            const int64_t nd = Geometry::node(bf.lev + L, (bf.si << L) + bk.j);
            for (int32_t p = G.nstart[nd]; p < G.nend[nd]; ++p) cd.push_back(p);
          } else {
            const LevelState &ps = prev[bk.b];
            const int64_t in = (int64_t)(bk.t >> 1) * ((int64_t)1 << (L - k + 1)) + 2 * bk.j;
            cd.insert(cd.end(), ps.skel.begin() + ps.skel_off[in], ps.skel.begin() + ps.skel_off[in + 2]);
          }
          const int64_t tnode = Geometry::node(bf.lev + k, (bf.oi << k) + bk.t);
          if (k == L) {
            rows[q].resize(G.nend[tnode] - G.nstart[tnode]);
            for (size_t i = 0; i < rows[q].size(); ++i) rows[q][i] = G.nstart[tnode] + (int32_t)i;
          } else {
            proxy_rows(G, tnode, cd.data(), (int)cd.size(), pp, rows[q], stamp, ++tag);
          }
        }
      });
      t_host += now_s() - th;
      J->bin.resize(n);
      J->ncols.resize(n);
      for (int64_t q = 0; q < n; ++q) {
        J->bin[q] = BlockIn{rows[q].data(), (int32_t)rows[q].size(), cands[q].data(),
                            (int32_t)cands[q].size(), nullptr};
        J->ncols[q] = (int32_t)cands[q].size();
        if (J->ncols[q] > HBI_ID_NMAX)
          throw Error{HBI_ERR_NUMERIC, "candidate set larger than the ID kernel supports"};
      }
      J->outs.resize(n);
      J->foff_local.resize(n);
      J->ioff_local.resize(n);
      J->plan = B.plan(J->bin, true, k > 0);
      return J;
    };
    auto chunk_done = [&](ChunkJob &J) {
      for (int64_t q = 0; q < J.c1 - J.c0; ++q) {
        const BlockOut &o = J.outs[q];
        skel_tmp[J.c0 + q].resize(o.rank);
        for (int32_t r = 0; r < o.rank; ++r) skel_tmp[J.c0 + q][r] = J.cands[q][o.piv[r]];
        rank_tmp[J.c0 + q] = o.rank;
        foff_tmp[J.c0 + q] = J.foff_local[q];
        ioff_tmp[J.c0 + q] = J.ioff_local[q];
        const int64_t e = (int64_t)o.rank * (J.ncols[q] - o.rank);
        if (k == 0) c->nnz_v += e; else c->nnz_w += e;
      }
    };
    {
      std::deque<std::unique_ptr<ChunkJob>> live;   // chunks with batches not yet finished
      std::vector<std::unique_ptr<ChunkJob>> finished;
      // results of finished chunks into the level state, and their host
      // arrays freed: done while the GPU runs the next batch
      auto drain = [&]() {
        for (auto &J : finished) chunk_done(*J);
        finished.clear();
      };
      int64_t cnext = 0;
      const double tg = now_s();
      const double th0 = t_host;
      B.pipeline([&](Prepared &P) {
        drain();
        if (live.empty() || live.back()->next == live.back()->plan.batches.size()) {
          if (cnext >= nblk) return false;
          live.push_back(make_chunk(cnext));
          cnext = live.back()->c1;
        }
        ChunkJob *J = live.back().get();
        const std::pair<int64_t, int64_t> bt = J->plan.batches[J->next++];
        B.prep(P, J->bin, J->plan, bt.first, bt.second, true, tol);
        P.outs = &J->outs;
        P.on_batch = [&, J](int64_t first, int64_t cnt) {
          compact(J->outs, first, cnt, J->ncols, J->foff_local, J->ioff_local, k > 0);
          if (++J->done == J->plan.batches.size()) {
            finished.push_back(std::move(live.front()));   // chunks finish in order
            live.pop_front();
          }
        };
        return true;
      });
      drain();
      t_gpu += now_s() - tg - (t_host - th0);
    }
    // scatter into per-butterfly state (block index t * 2^(L-k) + j)
    for (int64_t q = 0; q < nblk; ++q) {
      const Blk &bk = blks[q];
      const int L = bfs[bk.b].L;
      const int64_t bi = (int64_t)bk.t * ((int64_t)1 << (L - k)) + bk.j;
      cur[bk.b].rank[bi] = rank_tmp[q];
      cur[bk.b].foff[bi] = foff_tmp[q];
      cur[bk.b].ioff[bi] = ioff_tmp[q];
    }
    for (int64_t b = 0; b < nbf; ++b) {
      if (bfs[b].L < k) continue;
      LevelState &cs = cur[b];
      const int64_t n = (int64_t)cs.rank.size();
      for (int64_t bi = 0; bi < n; ++bi) cs.skel_off[bi + 1] = cs.skel_off[bi] + cs.rank[bi];
      cs.skel.resize(cs.skel_off[n]);
    }
    for (int64_t q = 0; q < nblk; ++q) {
      const Blk &bk = blks[q];
      const int L = bfs[bk.b].L;
      const int64_t bi = (int64_t)bk.t * ((int64_t)1 << (L - k)) + bk.j;
      std::copy(skel_tmp[q].begin(), skel_tmp[q].end(), cur[bk.b].skel.begin() + cur[bk.b].skel_off[bi]);
    }
    // z offsets in (t, j) order, then descriptors
    for (int64_t b = 0; b < nbf; ++b) {
      const BF &bf = bfs[b];
      if (bf.L < k) continue;
      LevelState &cs = cur[b];
      for (size_t bi = 0; bi < cs.rank.size(); ++bi) { cs.zoff[bi] = c->ztotal; c->ztotal += cs.rank[bi]; }
      const int L = bf.L;
      if (k == 0) {
        for (int64_t j = 0; j < ((int64_t)1 << L); ++j) {
          const int64_t g = (bf.si << L) + j;
          vd[g * Lv + (bf.lev - 1)] = VDesc{cs.foff[j], cs.zoff[j], cs.ioff[j], cs.rank[j], 0};
        }
      } else {
        const LevelState &ps = prev[b];
        for (int64_t tp = 0; tp < ((int64_t)1 << (k - 1)); ++tp)
          for (int64_t j = 0; j < ((int64_t)1 << (L - k)); ++j) {
            const int64_t a = (2 * tp) * ((int64_t)1 << (L - k)) + j;
            const int64_t bb = (2 * tp + 1) * ((int64_t)1 << (L - k)) + j;
            const int64_t in = tp * ((int64_t)1 << (L - k + 1)) + 2 * j;
            WUnit U{};
            U.ra = cs.rank[a]; U.rb = cs.rank[bb];
            U.c = ps.rank[in] + ps.rank[in + 1];
            U.foff = cs.foff[a];
            U.ioff = cs.ioff[a];
            U.zin = ps.zoff[in];
            U.zouta = cs.zoff[a];
            U.zoutb = cs.zoff[bb];
            if (ps.zoff[in + 1] != ps.zoff[in] + ps.rank[in] ||
                cs.foff[bb] != cs.foff[a] + (int64_t)U.ra * (U.c - U.ra) ||
                cs.ioff[bb] != cs.ioff[a] || U.ioff < 0)
              throw Error{HBI_ERR_NUMERIC, "internal layout error in the transfer stage"};
            units[k].push_back(U);
          }
      }
    }
    // skeleton factors K^L for butterflies ending at this level
    {
      std::vector<std::pair<int64_t, int64_t>> kl;   // (butterfly, t)
      int64_t tot = 0;
      for (int64_t b = 0; b < nbf; ++b) {
        if (bfs[b].L != k) continue;
        for (int64_t t = 0; t < ((int64_t)1 << k); ++t) {
          const int64_t nd = Geometry::node(bfs[b].lev + k, (bfs[b].oi << k) + t);
          tot += (int64_t)(G.nend[nd] - G.nstart[nd]) * cur[b].rank[t];
          kl.push_back({b, t});
        }
      }
      if (!kl.empty()) {
        const double tg = now_s();
        Chunk ch;
        HBI_HIP(ch.buf.alloc(sizeof(double2) * tot));
        ch.goff = Fg;
        ch.count = tot;
        std::vector<BlockIn> bin;
        std::vector<std::vector<int32_t>> rws(kl.size());
        int64_t o = 0;
        for (size_t q = 0; q < kl.size(); ++q) {
          const auto [b, t] = kl[q];
          const BF &bf = bfs[b];
          const int64_t nd = Geometry::node(bf.lev + k, (bf.oi << k) + t);
          const int32_t sz = G.nend[nd] - G.nstart[nd];
          rws[q].resize(sz);
          for (int32_t i = 0; i < sz; ++i) rws[q][i] = G.nstart[nd] + i;
          const LevelState &cs = cur[b];
          bin.push_back(BlockIn{rws[q].data(), sz, cs.skel.data() + cs.skel_off[t], cs.rank[t],
                                ch.buf.as<double2>() + o});
          const int64_t g = (bf.oi << k) + t;
          kd[g * Lv + (bf.lev - 1)] = KDesc{Fg + o, cs.zoff[t], cs.rank[t], 0};
          o += (int64_t)sz * cs.rank[t];
        }
        B.run(bin, false, tol, nullptr, [](int64_t, int64_t) {});
        Fg += tot;
        c->nnz_k += tot;
        chunks.push_back(std::move(ch));
        t_gpu += now_s() - tg;
      }
    }
    std::swap(prev, cur);
  }

  // dense diagonal leaves
  std::vector<LeafInfo> leaves(nleaf);
  {
    const double tg = now_s();
    int64_t tot = 0;
    for (int64_t g = 0; g < nleaf; ++g) {
      const int64_t nd = Geometry::node(Lv, g);
      const int64_t sz = G.nend[nd] - G.nstart[nd];
      tot += sz * sz;
    }
    Chunk ch;
    HBI_HIP(ch.buf.alloc(sizeof(double2) * tot));
    ch.goff = Fg;
    ch.count = tot;
    std::vector<std::vector<int32_t>> rws(nleaf);
    std::vector<BlockIn> bin(nleaf);
    int64_t o = 0;
    for (int64_t g = 0; g < nleaf; ++g) {
      const int64_t nd = Geometry::node(Lv, g);
      const int32_t sz = G.nend[nd] - G.nstart[nd];
      rws[g].resize(sz);
      for (int32_t i = 0; i < sz; ++i) rws[g][i] = G.nstart[nd] + i;
      bin[g] = BlockIn{rws[g].data(), sz, rws[g].data(), sz, ch.buf.as<double2>() + o};
      leaves[g] = LeafInfo{G.nstart[nd], sz, Fg + o};
      o += (int64_t)sz * sz;
    }
    B.run(bin, false, tol, nullptr, [](int64_t, int64_t) {});
    Fg += tot;
    c->nnz_d += tot;
    chunks.push_back(std::move(ch));
    t_gpu += now_s() - tg;
  }

  // final factor store (FP64 or rounded to FP32); the batch workspace is not
  // needed any more
  const double tf = now_s();
  c->ws.release();
  c->idx_d.release();
  B.stage[0].release();
  B.stage[1].release();
  c->Felems = Fg;
  const size_t esz = c->prec == HBI_F64 ? sizeof(double2) : sizeof(float2);
  // two spare entries: the FP32 transfer stage loads rows in pairs, which
  // reads at most one entry past a block
  HBI_HIP(c->F.alloc(esz * (std::max<int64_t>(Fg, 1) + 2)));
  upload(c->Fi, fi_h);
  {
    const std::vector<PlaceDesc> place = layout_store(chunks, Lv, nleaf, vd, kd, leaves, units, Fg);
    DevBuf pd;
    upload(pd, place);
    HBI_HIP(launch_place_blocks(pd.as<PlaceDesc>(), (int64_t)place.size(), c->F.p,
                                c->prec == HBI_F32, c->stream));
    HBI_HIP(hipStreamSynchronize(c->stream));
  }
  chunks.clear();
  make_apply_plan(c, leaves, vd, kd, units, Lv, Lmax);
  c->t_final = now_s() - tf;
  c->t_host = t_host;
  c->t_gpu = t_gpu;
  c->t_build = now_s() - tb0;
}

// The inclusion's G[j, i] = g(r_j, r^s_i) (cells j, segments i) as a single
// butterfly (Sec. 4.2: K^{s2v} compressed as one butterfly of
// L = min(L_v, L_s) levels, rows on the cell tree, columns on a tree of the
// segments; proxy rows by eq. proxyv2v with the uniform rows spread over the
// whole node).  The segment tree halves index ranges of the segments (they
// follow the curve) down to leaves of at most kSegLeaf segments.  Level k
// holds the blocks (t, j) of cell node t at depth k and segment node j at
// depth L - k (block index t 2^(L-k) + j): level 0 takes a leaf's segments
// as candidate columns, level k > 0 the skeletons of (t/2, 2j) and
// (t/2, 2j + 1), and level L all rows of its node; K^L then holds every
// cell of a depth-L node against that node's skeleton.  Factors are
// rounded to the context's precision like the volume ones.
constexpr int32_t kSegLeaf = 8;

// The inclusion term passes through (K^{s2s})^{-1}, which amplifies the
// compression error of G by its condition number; G's butterfly is small
// next to the volume factors, so it is compressed kIncTolFactor times
// tighter than the build tolerance (HBI_INCLUSION_TOL sets it outright).
constexpr double kIncTolFactor = 0.01;
double inclusion_tol(const hbi_ctx *c) {
  const char *e = std::getenv("HBI_INCLUSION_TOL");
  if (e && std::atof(e) > 0 && std::atof(e) < 1) return std::atof(e);
  return c->tol * kIncTolFactor;
}

void build_s2v(hbi_ctx *c, double tol) {
  const Geometry &G = c->geo;
  const int32_t ns = c->inc_ns;
  const int64_t Nv = G.Nv;
  int Ls = 0;
  while ((((int64_t)ns + ((int64_t)1 << Ls) - 1) >> Ls) > kSegLeaf) ++Ls;
  const int L = std::min(G.Lv, Ls);
  auto seg_lo = [&](int l, int64_t i) { return (int32_t)((i * ns) >> l); };
  // the cell holding each segment centre (the proxy rule's neighbours)
  std::vector<int32_t> segcell(ns);
  for (int32_t i = 0; i < ns; ++i) {
    int64_t nat = 0, stride = 1;
    for (int a = 0; a < 2; ++a) {
      int64_t k = (int64_t)std::floor((c->inc_xy[2 * i + a] - c->origin[a]) / c->h);
      k = std::min<int64_t>(std::max<int64_t>(k, 0), c->ncell[a] - 1);
      nat += k * stride;
      stride *= c->ncell[a];
    }
    segcell[i] = G.ipos[nat];
  }
  ProxyParams pp;
  pp.chi = c->chi();
  pp.radius = c->radius();
  pp.band = false;
  // the volume operator's ID statistics are kept apart
  const int64_t s_nid = c->nid, s_nw = c->nid_wide;
  const int32_t s_rmax = c->rank_max, s_mmax = c->id_m_max;
  const double s_rsum = c->rank_sum, s_msum = c->id_m_sum, s_nsum = c->id_n_sum,
               s_w = c->id_work, s_ww = c->id_work_wide, s_w128 = c->id_work_128;
  const int64_t s_path[3] = {c->nid_path[0], c->nid_path[1], c->nid_path[2]};

  struct Lev {
    std::vector<int32_t> rank, skel;
    std::vector<int64_t> soff, zoff, foff, ioff;
  };
  Lev prev, cur;
  std::vector<Chunk> chunks;
  int64_t Fg = 0, ztot = 0;
  std::vector<uint16_t> ih;
  std::vector<S2VLeaf> leaves((size_t)1 << L);
  std::vector<std::vector<WUnit>> units(L + 1);
  Batcher B(c);
  std::vector<int32_t> stamp(Nv, 0);
  int32_t tag = 0, rmax = 0;
  std::vector<uint16_t> ord, inv;
  std::vector<uint8_t> mark;
  auto orders = [&](const BlockOut &x, int32_t n) {
    mark.assign(n, 0);
    ord.clear();
    for (int32_t k = 0; k < x.rank; ++k) { ord.push_back((uint16_t)x.piv[k]); mark[x.piv[k]] = 1; }
    for (int32_t j = 0; j < n; ++j)
      if (!mark[j]) ord.push_back((uint16_t)j);
    if ((int32_t)ord.size() != n) throw Error{HBI_ERR_NUMERIC, "internal error: repeated pivot"};
    inv.assign(n, 0);
    for (int32_t k = 0; k < n; ++k) inv[ord[k]] = (uint16_t)k;
  };
  for (int k = 0; k <= L; ++k) {
    const int64_t nt = (int64_t)1 << k, nj = (int64_t)1 << (L - k), nblk = nt * nj;
    // processing order: level 0 by leaf, higher levels the sibling pairs
    // (2t', j), (2t' + 1, j) side by side (they share their candidates)
    std::vector<int64_t> bi(nblk);
    {
      int64_t q = 0;
      if (k == 0) {
        for (int64_t j = 0; j < nj; ++j) bi[q++] = j;
      } else {
        for (int64_t tp = 0; tp < nt / 2; ++tp)
          for (int64_t j = 0; j < nj; ++j)
            for (int h = 0; h < 2; ++h) bi[q++] = (2 * tp + h) * nj + j;
      }
    }
    std::vector<std::vector<int32_t>> cand(nblk), rows(nblk), colpt(nblk);
    std::vector<BlockIn> bin(nblk);
    std::vector<int32_t> cells;
    for (int64_t q = 0; q < nblk; ++q) {
      const int64_t b = bi[q], t = b / nj, j = b % nj;
      std::vector<int32_t> &cd = cand[q];
      if (k == 0) {
        for (int32_t i = seg_lo(L, j); i < seg_lo(L, j + 1); ++i) cd.push_back(i);
      } else {
        const int64_t in = (t >> 1) * (2 * nj) + 2 * j;
        cd.assign(prev.skel.begin() + prev.soff[in], prev.skel.begin() + prev.soff[in + 2]);
      }
      if ((int64_t)cd.size() > HBI_ID_NMAX)
        throw Error{HBI_ERR_NUMERIC, "inclusion candidate set larger than the ID kernel supports"};
      const int64_t nd = Geometry::node(k, t);
      if (k == L) {
        rows[q].resize(G.nend[nd] - G.nstart[nd]);
        for (size_t i = 0; i < rows[q].size(); ++i) rows[q][i] = G.nstart[nd] + (int32_t)i;
      } else {
        cells.resize(cd.size());
        for (size_t i = 0; i < cd.size(); ++i) cells[i] = segcell[cd[i]];
        proxy_rows(G, nd, cells.data(), (int)cells.size(), pp, rows[q], stamp, ++tag);
      }
      colpt[q].resize(cd.size());
      for (size_t i = 0; i < cd.size(); ++i) colpt[q][i] = (int32_t)(Nv + cd[i]);
      bin[q] = BlockIn{rows[q].data(), (int32_t)rows[q].size(), colpt[q].data(),
                       (int32_t)cd.size(), nullptr};
    }
    cur.rank.assign(nblk, 0);
    cur.foff.assign(nblk, 0);
    cur.ioff.assign(nblk, 0);
    std::vector<BlockOut> outs(nblk);
    // each batch's T blocks packed into a chunk of the store, while its
    // interpolation matrices are still in the workspace
    B.run(bin, true, tol, &outs, [&](int64_t first, int64_t cnt) {
      const bool pairs = k > 0;
      if (pairs && (first % 2 || cnt % 2))
        throw Error{HBI_ERR_NUMERIC, "internal error: unpaired inclusion block"};
      int64_t tot = 0;
      for (int64_t q = first; q < first + cnt; ++q)
        tot += (int64_t)outs[q].rank * ((int64_t)cand[q].size() - outs[q].rank);
      Chunk ch;
      HBI_HIP(ch.buf.alloc(sizeof(double2) * std::max<int64_t>(tot, 1)));
      ch.goff = Fg;
      ch.count = tot;
      std::vector<PairDesc> pd;
      std::vector<uint16_t> nsl;
      std::vector<int64_t> nso;
      int64_t o = 0;
      for (int64_t q = first; q < first + cnt; q += pairs ? 2 : 1) {
        const int64_t io = (int64_t)ih.size();
        const int32_t n = (int32_t)cand[q].size();
        PairDesc d{outs[q].X, nullptr, ch.buf.as<double2>() + o, nullptr, nullptr, outs[q].rank,
                   0, n, 0};
        if (!pairs) {
          orders(outs[q], n);
          ih.insert(ih.end(), ord.begin(), ord.end());
          ih.insert(ih.end(), inv.begin(), inv.end());
          nso.push_back((int64_t)nsl.size());
          nsl.insert(nsl.end(), ord.begin() + outs[q].rank, ord.end());
          nso.push_back(-1);
        } else {
          if ((int32_t)cand[q + 1].size() != n)
            throw Error{HBI_ERR_NUMERIC, "internal error: inclusion pair width"};
          ih.resize(io + 4 * (int64_t)n);
          for (int h = 0; h < 2; ++h) {
            orders(outs[q + h], n);
            std::copy(ord.begin(), ord.end(), ih.begin() + io + (int64_t)h * n);
            std::copy(inv.begin(), inv.end(), ih.begin() + io + (int64_t)(2 + h) * n);
            nso.push_back((int64_t)nsl.size());
            nsl.insert(nsl.end(), ord.begin() + outs[q + h].rank, ord.end());
          }
          d.xb = outs[q + 1].X;
          d.rb = outs[q + 1].rank;
        }
        for (int h = 0; h < (pairs ? 2 : 1); ++h) {
          const int64_t b = bi[q + h];
          cur.rank[b] = outs[q + h].rank;
          cur.foff[b] = Fg + o;
          cur.ioff[b] = io;
          o += (int64_t)outs[q + h].rank * (n - outs[q + h].rank);
          rmax = std::max(rmax, outs[q + h].rank);
        }
        pd.push_back(d);
      }
      DevBuf ns_d, pd_d;
      upload(ns_d, nsl);
      for (size_t e = 0; e < pd.size(); ++e) {
        pd[e].nsa = ns_d.as<uint16_t>() + nso[2 * e];
        if (pairs) pd[e].nsb = ns_d.as<uint16_t>() + nso[2 * e + 1];
      }
      upload(pd_d, pd);
      HBI_HIP(launch_pack_pairs(pd_d.as<PairDesc>(), (int64_t)pd.size(), c->stream));
      HBI_HIP(hipStreamSynchronize(c->stream));
      Fg += tot;
      chunks.push_back(std::move(ch));
    }, k > 0);
    // skeletons and vector offsets in block order
    cur.soff.assign(nblk + 1, 0);
    for (int64_t b = 0; b < nblk; ++b) cur.soff[b + 1] = cur.soff[b] + cur.rank[b];
    cur.skel.assign(cur.soff[nblk], 0);
    for (int64_t q = 0; q < nblk; ++q) {
      const int64_t b = bi[q];
      for (int32_t r = 0; r < outs[q].rank; ++r) cur.skel[cur.soff[b] + r] = cand[q][outs[q].piv[r]];
    }
    cur.zoff.assign(nblk, 0);
    for (int64_t b = 0; b < nblk; ++b) { cur.zoff[b] = ztot; ztot += cur.rank[b]; }
    if (k == 0) {
      for (int64_t j = 0; j < nj; ++j)
        leaves[j] = S2VLeaf{cur.foff[j], cur.ioff[j], cur.zoff[j], cur.rank[j],
                            seg_lo(L, j + 1) - seg_lo(L, j), seg_lo(L, j), 0};
    } else {
      for (int64_t tp = 0; tp < nt / 2; ++tp)
        for (int64_t j = 0; j < nj; ++j) {
          const int64_t a = (2 * tp) * nj + j, bb = a + nj, in = tp * (2 * nj) + 2 * j;
          WUnit U{};
          U.ra = cur.rank[a];
          U.rb = cur.rank[bb];
          U.c = prev.rank[in] + prev.rank[in + 1];
          U.foff = cur.foff[a];
          U.ioff = cur.ioff[a];
          U.zin = prev.zoff[in];
          U.zouta = cur.zoff[a];
          U.zoutb = cur.zoff[bb];
          if (prev.zoff[in + 1] != prev.zoff[in] + prev.rank[in] ||
              cur.foff[bb] != cur.foff[a] + (int64_t)U.ra * (U.c - U.ra) || cur.ioff[bb] != U.ioff)
            throw Error{HBI_ERR_NUMERIC, "internal layout error in the inclusion butterfly"};
          units[k].push_back(U);
        }
    }
    std::swap(prev, cur);
  }
  // K^L: every cell of a depth-L node against the node's skeleton
  std::vector<S2VNode> nodes((size_t)1 << L);
  int32_t size_max = 0;
  {
    int64_t tot = 0;
    for (int64_t t = 0; t < ((int64_t)1 << L); ++t) {
      const int64_t nd = Geometry::node(L, t);
      tot += (int64_t)(G.nend[nd] - G.nstart[nd]) * prev.rank[t];
    }
    Chunk ch;
    HBI_HIP(ch.buf.alloc(sizeof(double2) * std::max<int64_t>(tot, 1)));
    ch.goff = Fg;
    ch.count = tot;
    std::vector<std::vector<int32_t>> rws(nodes.size()), cls(nodes.size());
    std::vector<BlockIn> bin(nodes.size());
    int64_t o = 0;
    for (int64_t t = 0; t < (int64_t)nodes.size(); ++t) {
      const int64_t nd = Geometry::node(L, t);
      const int32_t sz = G.nend[nd] - G.nstart[nd], r = prev.rank[t];
      rws[t].resize(sz);
      for (int32_t i = 0; i < sz; ++i) rws[t][i] = G.nstart[nd] + i;
      cls[t].resize(r);
      for (int32_t i = 0; i < r; ++i) cls[t][i] = (int32_t)(Nv + prev.skel[prev.soff[t] + i]);
      bin[t] = BlockIn{rws[t].data(), sz, cls[t].data(), r, ch.buf.as<double2>() + o};
      nodes[t] = S2VNode{Fg + o, prev.zoff[t], G.nstart[nd], sz, r, 0};
      size_max = std::max(size_max, sz);
      o += (int64_t)sz * r;
    }
    B.run(bin, false, tol, nullptr, [](int64_t, int64_t) {});
    Fg += tot;
    chunks.push_back(std::move(ch));
  }
  c->nid = s_nid; c->nid_wide = s_nw; c->rank_max = s_rmax; c->id_m_max = s_mmax;
  c->rank_sum = s_rsum; c->id_m_sum = s_msum; c->id_n_sum = s_nsum; c->id_work = s_w;
  c->id_work_wide = s_ww; c->id_work_128 = s_w128;
  for (int q = 0; q < 3; ++q) c->nid_path[q] = s_path[q];
  // the store: chunks in order, rounded to the context's precision
  const bool f32 = c->prec == HBI_F32;
  const size_t esz = f32 ? sizeof(float2) : sizeof(double2);
  HBI_HIP(c->s2v_F.alloc(esz * std::max<int64_t>(Fg, 1)));
  {
    std::vector<PlaceDesc> pd;
    for (const Chunk &ch : chunks)
      if (ch.count) pd.push_back(PlaceDesc{ch.buf.as<double2>(), ch.goff, ch.count});
    DevBuf pd_d;
    upload(pd_d, pd);
    HBI_HIP(launch_place_blocks(pd_d.as<PlaceDesc>(), (int64_t)pd.size(), c->s2v_F.p, f32,
                                c->stream));
    HBI_HIP(hipStreamSynchronize(c->stream));
  }
  chunks.clear();
  if (ih.empty()) ih.push_back(0);
  upload(c->s2v_idx, ih);
  upload(c->s2v_leaves, leaves);
  upload(c->s2v_nodes, nodes);
  c->s2v_units.clear();
  S2VPlan &P = c->s2v_plan;
  P = S2VPlan();
  P.L = L;
  P.F = c->s2v_F.p;
  P.idx = c->s2v_idx.as<uint16_t>();
  P.perm = c->perm_d.as<int32_t>();
  P.leaves = c->s2v_leaves.as<S2VLeaf>();
  P.nodes = c->s2v_nodes.as<S2VNode>();
  P.nleaf = (int64_t)leaves.size();
  P.nnode = (int64_t)nodes.size();
  P.units.assign(L + 1, nullptr);
  P.nunits.assign(L + 1, 0);
  P.witems.assign(L + 1, nullptr);
  P.wtitems.assign(L + 1, nullptr);
  P.nwitems.assign(L + 1, 0);
  P.nwtitems.assign(L + 1, 0);
  // four outputs per workgroup: (descriptor, first output)
  auto quads = [](std::vector<int2> &v, int32_t d, int32_t n) {
    for (int32_t o = 0; o < n; o += 4) v.push_back(int2{d, o});
  };
  for (int k = 1; k <= L; ++k) {
    std::vector<int2> wi, wti;
    for (size_t u = 0; u < units[k].size(); ++u) {
      quads(wi, (int32_t)u, units[k][u].ra + units[k][u].rb);
      quads(wti, (int32_t)u, units[k][u].c);
    }
    c->s2v_units.emplace_back();
    upload(c->s2v_units.back(), units[k]);
    P.units[k] = c->s2v_units.back().as<WUnit>();
    P.nunits[k] = (int64_t)units[k].size();
    c->s2v_units.emplace_back();
    upload(c->s2v_units.back(), wi);
    P.witems[k] = c->s2v_units.back().as<int2>();
    P.nwitems[k] = (int64_t)wi.size();
    c->s2v_units.emplace_back();
    upload(c->s2v_units.back(), wti);
    P.wtitems[k] = c->s2v_units.back().as<int2>();
    P.nwtitems[k] = (int64_t)wti.size();
  }
  {
    std::vector<int2> kti;
    for (size_t t = 0; t < nodes.size(); ++t) quads(kti, (int32_t)t, nodes[t].r);
    c->s2v_units.emplace_back();
    upload(c->s2v_units.back(), kti);
    P.ktitems = c->s2v_units.back().as<int2>();
    P.nktitems = (int64_t)kti.size();
  }
  HBI_HIP(c->s2v_z.alloc(esz * std::max<int64_t>(ztot, 1)));
  P.z = c->s2v_z.p;
  P.size_max = size_max;
  c->s2v_L = L;
  c->s2v_entries = Fg;
  c->s2v_rank_max = rmax;
  c->s2v_ztotal = ztot;
}

// Dense operators of the curve inclusion (Sec. 3.2, eq. m_v2v_inclu):
// G[j, i] = g(r_j, r^s_i) over cells j (natural order, chunks of kIncChunk
// cells) and segments i, evaluated by the entry kernels with the segments as
// points after the cells; K^{s2s} from g between segments, its columns
// scaled by -w_j (self factors on the diagonal), inverted by Gauss-Jordan in
// FP64.  Stored in the factors' precision.
constexpr int32_t kIncChunk = 4096;   // cells per chunk of G (a multiple of 256)
constexpr int32_t kS2sChunk = 512;    // columns per block of the K^{s2s} entries

void build_inclusion(hbi_ctx *c) {
  const double t0 = now_s();
  const int64_t Nv = c->geo.Nv;
  const int32_t ns = c->inc_ns;
  const int32_t m = kIncChunk;
  const int64_t nchunk = (Nv + m - 1) / m;
  const bool f32 = c->prec == HBI_F32;
  const size_t esz = f32 ? sizeof(float2) : sizeof(double2);
  std::vector<int32_t> segpos(ns), rowpos(Nv);
  for (int32_t i = 0; i < ns; ++i) segpos[i] = (int32_t)(Nv + i);
  for (int64_t j = 0; j < Nv; ++j) rowpos[j] = c->geo.ipos[j];
  const bool dense = env_int("HBI_INCLUSION_DENSE", 0) != 0;
  if (!dense) build_s2v(c, inclusion_tol(c));
  else HBI_HIP(c->inc_G.alloc(esz * (size_t)Nv * ns));
  Batcher B(c);
  if (dense) {
    // groups of chunks whose FP64 values fit a 1 GiB scratch
    const int64_t per = (int64_t)m * ns * (int64_t)sizeof(double2);
    const int64_t gch = std::max<int64_t>(1, ((int64_t)1 << 30) / per);
    DevBuf scratch, pd_d;
    HBI_HIP(scratch.alloc((size_t)std::min(nchunk, gch) * per));
    for (int64_t g0 = 0; g0 < nchunk; g0 += gch) {
      const int64_t g1 = std::min(nchunk, g0 + gch);
      std::vector<BlockIn> bin;
      std::vector<PlaceDesc> pd;
      int64_t off = 0;
      for (int64_t q = g0; q < g1; ++q) {
        const int64_t r0 = q * m;
        const int32_t mq = (int32_t)std::min<int64_t>(m, Nv - r0);
        double2 *out = scratch.as<double2>() + off;
        bin.push_back(BlockIn{rowpos.data() + r0, mq, segpos.data(), ns, out});
        pd.push_back(PlaceDesc{out, r0 * ns, (int64_t)mq * ns});
        off += (int64_t)mq * ns;
      }
      B.run(bin, false, 0.0, nullptr, [](int64_t, int64_t) {});
      upload(pd_d, pd);
      HBI_HIP(launch_place_blocks(pd_d.as<PlaceDesc>(), (int64_t)pd.size(), c->inc_G.p, f32,
                                  c->stream));
      HBI_HIP(hipStreamSynchronize(c->stream));
    }
  }
  {
    DevBuf S, SH, perm, colk, status, pd_d, Sb;
    HBI_HIP(S.alloc(sizeof(double2) * (size_t)ns * ns));
    // panel rows of the blocked inverse (32 x ns); HBI_S2S_INVERSE=columns
    // keeps the column-by-column form
    const char *iv = std::getenv("HBI_S2S_INVERSE");
    const bool blocked = !(iv && std::strcmp(iv, "columns") == 0);
    if (blocked) HBI_HIP(Sb.alloc(sizeof(double2) * (size_t)32 * ns));
    HBI_HIP(SH.alloc(sizeof(double2) * (size_t)ns * ns));
    HBI_HIP(perm.alloc(sizeof(int32_t) * ns));
    HBI_HIP(colk.alloc(sizeof(double2) * ns));
    HBI_HIP(status.alloc(sizeof(int32_t)));
    HBI_HIP(hipMemsetAsync(status.p, 0, sizeof(int32_t), c->stream));
    // K^{s2s} entries in column chunks (each chunk's column side then needs
    // a bounded workspace whatever N_s is)
    std::vector<BlockIn> bin;
    for (int32_t j0 = 0; j0 < ns; j0 += kS2sChunk)
      bin.push_back(BlockIn{segpos.data(), ns, segpos.data() + j0, std::min(kS2sChunk, ns - j0),
                            S.as<double2>() + (int64_t)j0 * ns});
    B.run(bin, false, 0.0, nullptr, [](int64_t, int64_t) {});
    HBI_HIP(launch_s2s_inverse(S.as<double2>(), ns, c->inc_w_d.as<double>(), perm.as<int32_t>(),
                               colk.as<double2>(), blocked ? Sb.as<double2>() : nullptr,
                               status.as<int32_t>(), c->stream));
    int32_t st = 0;
    HBI_HIP(hipMemcpyAsync(&st, status.p, sizeof(int32_t), hipMemcpyDeviceToHost, c->stream));
    HBI_HIP(hipStreamSynchronize(c->stream));
    HBI_REQUIRE(st == 0, HBI_ERR_NUMERIC, "the surface-to-surface matrix is singular");
    HBI_HIP(launch_conj_transpose(S.as<double2>(), ns, SH.as<double2>(), c->stream));
    HBI_HIP(c->inc_M.alloc(esz * (size_t)ns * ns));
    HBI_HIP(c->inc_MH.alloc(esz * (size_t)ns * ns));
    std::vector<PlaceDesc> pd{PlaceDesc{S.as<double2>(), 0, (int64_t)ns * ns}};
    upload(pd_d, pd);
    HBI_HIP(launch_place_blocks(pd_d.as<PlaceDesc>(), 1, c->inc_M.p, f32, c->stream));
    HBI_HIP(hipStreamSynchronize(c->stream));
    pd[0].src = SH.as<double2>();
    upload(pd_d, pd);
    HBI_HIP(launch_place_blocks(pd_d.as<PlaceDesc>(), 1, c->inc_MH.p, f32, c->stream));
    HBI_HIP(hipStreamSynchronize(c->stream));
  }
  if (f32) {
    std::vector<float> wf(c->inc_w.begin(), c->inc_w.end());
    upload(c->inc_wf, wf);
  } else {
    upload(c->inc_wf, c->inc_w);
  }
  if (dense) {
    HBI_HIP(c->inc_part.alloc(esz * (size_t)nchunk * ns));
    HBI_HIP(c->inc_part2.alloc(esz * (size_t)Nv * ((ns + 255) / 256)));
  }
  HBI_HIP(c->inc_z.alloc(esz * (size_t)ns));
  HBI_HIP(c->inc_y.alloc(esz * (size_t)ns));
  HBI_HIP(c->inc_part3.alloc(esz * (size_t)ns * ((ns + 255) / 256)));
  InclusionPlan &ip = c->inc_plan;
  ip.bf = dense ? nullptr : &c->s2v_plan;
  ip.G = c->inc_G.p; ip.M = c->inc_M.p; ip.MH = c->inc_MH.p; ip.w = c->inc_wf.p;
  ip.part = c->inc_part.p; ip.z = c->inc_z.p; ip.y = c->inc_y.p; ip.part2 = c->inc_part2.p;
  ip.part3 = c->inc_part3.p;
  ip.Nv = Nv; ip.ns = ns; ip.m = m;
  c->t_inc = now_s() - t0;
}

// The inclusion term of eq. m_v2v_inclu (or of its conjugate transpose),
// added to u after the volume product of every column.
void apply_inclusion(hbi_ctx *c, const void *s, void *u, int32_t nrhs, int64_t ld, bool adj) {
  if (c->inc_ns == 0) return;
  const size_t esz = c->prec == HBI_F64 ? 16 : 8;
  for (int32_t r = 0; r < nrhs; ++r) {
    const char *sc = (const char *)s + esz * (size_t)ld * r;
    char *uc = (char *)u + esz * (size_t)ld * r;
    if (c->prec == HBI_F64)
      HBI_HIP(launch_inclusion_apply<double>(c->inc_plan, sc, uc, std::pow(c->h, c->dim), adj,
                                             c->stream));
    else
      HBI_HIP(launch_inclusion_apply<float>(c->inc_plan, sc, uc, (float)std::pow(c->h, c->dim),
                                            adj, c->stream));
  }
}

bool overlap(const void *a, size_t na, const void *b, size_t nb) {
  const char *x = (const char *)a, *y = (const char *)b;
  return x < y + nb && y < x + na;
}

void check_apply_args(hbi_ctx *c, const void *s, void *u, int32_t nrhs, int64_t ld) {
  HBI_REQUIRE(c->state == 2, HBI_ERR_STATE, "apply before build");
  HBI_REQUIRE(s && u, HBI_ERR_ARG, "null s or u");
  HBI_REQUIRE(nrhs >= 1, HBI_ERR_ARG, "nrhs must be >= 1");
  HBI_REQUIRE(ld >= c->geo.Nv, HBI_ERR_ARG, "ld must be >= N_v");
  const size_t esz = c->prec == HBI_F64 ? 16 : 8;
  const size_t span = esz * ((size_t)ld * (nrhs - 1) + c->geo.Nv);
  HBI_REQUIRE(!overlap(s, span, u, span), HBI_ERR_ARG, "s and u overlap");
}

// The single-RHS product column by column, with the per-level vectors in z
// (the context's own buffer unless another one is given; no profiling
// events are recorded then).
void do_apply(hbi_ctx *c, const void *s, void *u, int32_t nrhs, int64_t ld, bool adj,
              void *zbuf = nullptr) {
  check_apply_args(c, s, u, nrhs, ld);
  const size_t esz = c->prec == HBI_F64 ? 16 : 8;
  c->prof.st = c->stream;
  LaunchHook *hook = c->profiling && !zbuf ? &c->prof : nullptr;
  void *z = zbuf ? zbuf : c->z_d.p;
  for (int32_t r = 0; r < nrhs; ++r) {
    const char *sc = (const char *)s + esz * (size_t)ld * r;
    char *uc = (char *)u + esz * (size_t)ld * r;
    if (c->prec == HBI_F64) {
      HBI_HIP(launch_apply<double>(c->plan, sc, uc, z, c->F.p, std::pow(c->h, c->dim), adj,
                                   c->stream, hook));
    } else {
      HBI_HIP(launch_apply<float>(c->plan, sc, uc, z, c->F.p, (float)std::pow(c->h, c->dim),
                                  adj, c->stream, hook));
    }
  }
}

}  // namespace

// ===========================================================================
// Many right-hand sides / many problems (MFMA tiles, one HIP graph)
// ===========================================================================
struct MultiJob {
  hbi_ctx *c;
  int32_t j0, nrhs, Np;     // right-hand-side columns [j0, j0 + nrhs) of problem p
  int prob;
  int64_t xt_off = 0, yt_off = 0, z_off = 0;   // element offsets in the pass workspace
};

struct MultiPass {
  std::vector<int> jobs;
  std::vector<MStagePlan> stages;
  std::vector<DevBuf> bufs;
  std::vector<MTrans> jin, jout;
  DevBuf jin_d, jout_d;
  int64_t maxNv = 0;
  int maxjt = 0;
  size_t bytes = 0;
};

struct BatchCache {
  std::vector<hbi_ctx *> ctxs;
  std::vector<uint64_t> gens;   // build_gen of each context when captured
  std::vector<int32_t> nrhs;
  std::vector<const void *> s_ptr;
  std::vector<void *> u_ptr;
  std::vector<int64_t> ld;
  int prec = 0, nb = 4, ku = 0;   // column-tile width, k-steps per chunk (0: default)
  bool adj = false;   // the conjugate-transpose product
  std::vector<MultiJob> jobs;
  std::vector<MultiPass> passes;
  DevBuf ws;
  hipStream_t gst = nullptr;
  hipEvent_t e_in = nullptr, e_out = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  // one persistent cooperative launch instead of the graph
  bool persistent = false;
  int pgrid = 0, nphase = 0;
  DevBuf phases_d;
  double tuned_ms = 0;
  ~BatchCache() {
    // the graph may still run: its workspace and job tables go with it
    if (gst) (void)hipStreamSynchronize(gst);
    if (gexec) (void)hipGraphExecDestroy(gexec);
    if (graph) (void)hipGraphDestroy(graph);
    if (e_in) (void)hipEventDestroy(e_in);
    if (e_out) (void)hipEventDestroy(e_out);
    if (gst) (void)hipStreamDestroy(gst);
  }
};

namespace {

size_t multi_budget() {
  const char *e = std::getenv("HBI_MULTI_BYTES");
  if (e && *e) return (size_t)std::strtoull(e, nullptr, 10);
  return (size_t)8 << 30;
}

int round16(int n) { return (n + 15) & ~15; }

// Split the problems' right-hand sides into jobs and pack them into passes
// whose vector workspace (x, y and all butterfly vectors, Np wide) fits.
void plan_passes(BatchCache &B, const std::vector<int32_t> &nrhs) {
  const size_t budget = multi_budget();
  const size_t esz = B.prec == HBI_F64 ? 16 : 8;
  B.jobs.clear();
  B.passes.clear();
  for (size_t p = 0; p < B.ctxs.size(); ++p) {
    hbi_ctx *c = B.ctxs[p];
    const size_t per_col = (size_t)(2 * c->geo.Nv + c->ztotal) * esz;
    int cmax = (int)std::min<size_t>(256, (budget / per_col) & ~(size_t)15);
    if (cmax < 16) throw Error{HBI_ERR_OOM, "batched apply workspace too small for a problem"};
    for (int j0 = 0; j0 < nrhs[p]; j0 += cmax) {
      MultiJob J{};
      J.c = c;
      J.prob = (int)p;
      J.j0 = j0;
      J.nrhs = std::min(cmax, nrhs[p] - j0);
      J.Np = round16(J.nrhs);
      B.jobs.push_back(J);
    }
  }
  MultiPass cur;
  for (int q = 0; q < (int)B.jobs.size(); ++q) {
    MultiJob &J = B.jobs[q];
    const size_t b = (size_t)(2 * J.c->geo.Nv + J.c->ztotal) * J.Np * esz;
    if (!cur.jobs.empty() && cur.bytes + b > budget) {
      B.passes.push_back(std::move(cur));
      cur = MultiPass();
    }
    cur.jobs.push_back(q);
    cur.bytes += b;
  }
  if (!cur.jobs.empty()) B.passes.push_back(std::move(cur));
  size_t wsmax = 0;
  for (auto &P : B.passes) {
    int64_t o = 0;
    for (int q : P.jobs) { B.jobs[q].xt_off = o; o += B.jobs[q].c->geo.Nv * B.jobs[q].Np; }
    for (int q : P.jobs) { B.jobs[q].yt_off = o; o += B.jobs[q].c->geo.Nv * B.jobs[q].Np; }
    for (int q : P.jobs) { B.jobs[q].z_off = o; o += std::max<int64_t>(B.jobs[q].c->ztotal, 1) * B.jobs[q].Np; }
    wsmax = std::max(wsmax, (size_t)o * esz);
  }
  HBI_HIP(B.ws.reserve(std::max<size_t>(wsmax, 256)));
}

// XCD-aware placement of one stage's work items (four per workgroup, one
// per wave).  Workgroups are dispatched round-robin to the GPU's eight
// XCDs (workgroup b to XCD b % 8), each with its own L2, so items that read
// the same operands (a transfer unit's inputs and factors, a leaf's inputs)
// are put on one XCD, in consecutive slots of its sequence of workgroups
// b = 8 q + x: their repeated reads then hit that L2 instead of going to
// memory once per XCD.  Groups are taken in decreasing `key` (the longest
// items first) and each goes to the XCD with the least work so far; slots
// left over are empty items (Np = 0).
constexpr int kXcds = 8;

template <typename It> struct ItemGroups {
  std::vector<It> items;              // group g = items[start[g] .. start[g + 1])
  std::vector<size_t> start{0};
  std::vector<double> key, work;
  void close(double k, double w) {
    if (items.size() == start.back()) return;
    start.push_back(items.size());
    key.push_back(k);
    work.push_back(w);
  }
};

template <typename It> std::vector<It> xcd_place(const ItemGroups<It> &G) {
  const size_t ng = G.key.size();
  std::vector<size_t> order(ng);
  for (size_t g = 0; g < ng; ++g) order[g] = g;
  std::stable_sort(order.begin(), order.end(),
                   [&](size_t a, size_t b) { return G.key[a] > G.key[b]; });
  std::vector<std::vector<It>> q(kXcds);
  std::vector<double> load(kXcds, 0.0);
  for (size_t g : order) {
    const int x = (int)(std::min_element(load.begin(), load.end()) - load.begin());
    q[x].insert(q[x].end(), G.items.begin() + G.start[g], G.items.begin() + G.start[g + 1]);
    load[x] += G.work[g];
  }
  size_t nwg = 0;
  for (auto &v : q) nwg = std::max(nwg, (v.size() + 3) / 4);
  std::vector<It> out(nwg * kXcds * 4, It{});
  for (int x = 0; x < kXcds; ++x)
    for (size_t p = 0; p < q[x].size(); ++p) out[4 * (kXcds * (p / 4) + x) + p % 4] = q[x][p];
  return out;
}

// Work items of every stage of every pass for `nb` column tiles per wave.
void build_items(BatchCache &B, int nb) {
  const size_t esz = B.prec == HBI_F64 ? 16 : 8;
  char *ws = B.ws.as<char>();
  for (auto &P : B.passes) {
    P.stages.clear();
    P.bufs.clear();
    P.jin.clear();
    P.jout.clear();
    P.maxNv = 0;
    P.maxjt = 0;
    int Lmax = 0;
    ItemGroups<MVItem> vi;
    ItemGroups<MFItem> fi;
    for (int q : P.jobs) {
      const MultiJob &J = B.jobs[q];
      hbi_ctx *c = J.c;
      const char *F = c->F.as<char>();
      char *xt = ws + J.xt_off * esz, *yt = ws + J.yt_off * esz, *zb = ws + J.z_off * esz;
      const int Lv = c->geo.Lv;
      Lmax = std::max(Lmax, c->plan.Lmax);
      P.maxNv = std::max(P.maxNv, c->geo.Nv);
      P.maxjt = std::max(P.maxjt, J.Np / 16);
      const int ngrp = (J.Np / 16 + nb - 1) / nb;
      for (int64_t g = 0; g < (int64_t)c->leaves_h.size(); ++g) {
        const LeafInfo &lf = c->leaves_h[g];
        const char *x = xt + (int64_t)lf.start * J.Np * esz;
        // one group per leaf: every item reads the leaf's inputs x
        double vw = 0.0, fw = lf.size;
        for (int gq = 0; gq < ngrp; ++gq)
          for (int l = 0; l < Lv; ++l) {
            const VDesc &d = c->vd_h[g * Lv + l];
            for (int r0 = 0; r0 < d.r; r0 += 16) {
              vi.items.push_back(MVItem{F + d.foff * esz, c->Fi.as<uint16_t>() + d.ioff, x,
                                        zb + d.zout * J.Np * esz, d.r, lf.size, r0, gq * nb,
                                        J.Np, 0});
              vw += lf.size - d.r;
            }
          }
        vi.close(lf.size, vw);
        for (int l = 0; l < Lv; ++l) fw += c->kd_h[g * Lv + l].r;
        for (int gq = 0; gq < ngrp; ++gq)
          for (int r0 = 0; r0 < lf.size; r0 += 16)
            fi.items.push_back(MFItem{F, zb, x, yt + (int64_t)lf.start * J.Np * esz,
                                      c->kd_d.as<KDesc>() + g * Lv, lf.dense_off, lf.size, Lv, r0,
                                      gq * nb, J.Np, 0});
        fi.close(fw, fw * ((lf.size + 15) / 16) * ngrp);
      }
      const size_t cofs = (size_t)J.j0 * esz;
      P.jin.push_back(MTrans{(const char *)B.s_ptr[J.prob] + cofs * B.ld[J.prob], xt,
                             c->perm_d.as<int32_t>(), c->geo.Nv, B.ld[J.prob], J.nrhs, J.Np,
                             std::pow(c->h, c->dim)});
      P.jout.push_back(MTrans{yt, (char *)B.u_ptr[J.prob] + cofs * B.ld[J.prob],
                              c->perm_d.as<int32_t>(), c->geo.Nv, B.ld[J.prob], J.nrhs, J.Np, 1.0});
    }
    auto add_stage = [&](int kind, const void *data, size_t bytes, int64_t n) {
      DevBuf d;
      HBI_HIP(d.alloc(bytes));
      if (bytes) HBI_HIP(hipMemcpy(d.p, data, bytes, hipMemcpyHostToDevice));
      P.stages.push_back(MStagePlan{kind, nb, d.p, n});
      P.bufs.push_back(std::move(d));
    };
    const std::vector<MVItem> vp = xcd_place(vi);
    add_stage(0, vp.data(), vp.size() * sizeof(MVItem), (int64_t)vp.size());
    for (int k = 1; k <= Lmax; ++k) {
      ItemGroups<MWItem> wi;
      for (int q : P.jobs) {
        const MultiJob &J = B.jobs[q];
        hbi_ctx *c = J.c;
        if (k > c->plan.Lmax) continue;
        const char *F = c->F.as<char>();
        char *zb = ws + J.z_off * esz;
        const int ngrp = (J.Np / 16 + nb - 1) / nb;
        const uint16_t *fidx = c->Fi.as<uint16_t>();
        // one group per unit (its inputs and factors are read by every
        // item), column-tile groups outermost
        for (const WUnit &U : c->units_h[k]) {
          const size_t n0 = wi.items.size();
          for (int gq = 0; gq < ngrp; ++gq) {
            if (U.ra + U.rb <= 32) {
              // a small pair: stacked tiles, entries synthesised from T
              for (int r0 = 0; r0 < U.ra + U.rb; r0 += 16)
                wi.items.push_back(MWItem{F + U.foff * esz, fidx + U.ioff, zb + U.zin * J.Np * esz,
                                          zb + U.zouta * J.Np * esz, zb + U.zoutb * J.Np * esz,
                                          U.ra, U.rb, U.c, r0, gq * nb, J.Np});
              continue;
            }
            for (int h = 0; h < 2; ++h) {
              // child a, then child b (T_b after T_a, ib after ia)
              const int32_t r = h ? U.rb : U.ra;
              const int64_t toff = U.foff + (h ? (int64_t)U.ra * (U.c - U.ra) : 0);
              const uint16_t *idx = fidx + U.ioff + (h ? U.c : 0);
              char *zo = zb + (h ? U.zoutb : U.zouta) * J.Np * esz;
              for (int r0 = 0; r0 < r; r0 += 16)
                wi.items.push_back(MWItem{F + toff * esz, idx, zb + U.zin * J.Np * esz, zo,
                                          nullptr, r, -1, U.c, r0, gq * nb, J.Np});
            }
          }
          wi.close(U.c, (double)U.c * (wi.items.size() - n0));
        }
      }
      const std::vector<MWItem> w = xcd_place(wi);
      add_stage(1, w.data(), w.size() * sizeof(MWItem), (int64_t)w.size());
    }
    const std::vector<MFItem> fp = xcd_place(fi);
    add_stage(2, fp.data(), fp.size() * sizeof(MFItem), (int64_t)fp.size());
    upload(P.jin_d, P.jin);
    upload(P.jout_d, P.jout);
  }
  B.nb = nb;
}

// Work items of the adjoint product for `nb` column tiles per wave: the
// K^L part, the transfer units from the top level down, then every leaf's
// D^H and V^H parts (scaled by h^d); the inputs are gathered unscaled.
void build_items_adj(BatchCache &B, int nb) {
  const size_t esz = B.prec == HBI_F64 ? 16 : 8;
  char *ws = B.ws.as<char>();
  for (auto &P : B.passes) {
    P.stages.clear();
    P.bufs.clear();
    P.jin.clear();
    P.jout.clear();
    P.maxNv = 0;
    P.maxjt = 0;
    int Lmax = 0;
    ItemGroups<MFAItem> ki;
    ItemGroups<MVAItem> li;
    for (int q : P.jobs) {
      const MultiJob &J = B.jobs[q];
      hbi_ctx *c = J.c;
      const char *F = c->F.as<char>();
      char *xt = ws + J.xt_off * esz, *yt = ws + J.yt_off * esz, *zb = ws + J.z_off * esz;
      const int Lv = c->geo.Lv;
      Lmax = std::max(Lmax, c->plan.Lmax);
      P.maxNv = std::max(P.maxNv, c->geo.Nv);
      P.maxjt = std::max(P.maxjt, J.Np / 16);
      const int ngrp = (J.Np / 16 + nb - 1) / nb;
      const double hd = std::pow(c->h, c->dim);
      for (int64_t g = 0; g < (int64_t)c->leaves_h.size(); ++g) {
        const LeafInfo &lf = c->leaves_h[g];
        const char *y = xt + (int64_t)lf.start * J.Np * esz;
        // one group per leaf: every item reads the leaf's inputs y
        double kw = 0.0, lw = lf.size;
        for (int gq = 0; gq < ngrp; ++gq)
          for (int l = 0; l < Lv; ++l) {
            const KDesc &d = c->kd_h[g * Lv + l];
            for (int r0 = 0; r0 < d.r; r0 += 16) {
              ki.items.push_back(MFAItem{F + d.foff * esz, y, zb + d.zin * J.Np * esz, d.r,
                                         lf.size, r0, gq * nb, J.Np, 0});
              kw += lf.size;
            }
          }
        ki.close(lf.size, kw);
        for (int l = 0; l < Lv; ++l) lw += c->vd_h[g * Lv + l].r;
        for (int gq = 0; gq < ngrp; ++gq)
          for (int r0 = 0; r0 < lf.size; r0 += 16)
            li.items.push_back(MVAItem{F, c->Fi.as<uint16_t>(), y,
                                       yt + (int64_t)lf.start * J.Np * esz,
                                       c->vd_d.as<VDesc>() + g * Lv, zb, lf.dense_off, hd, lf.size,
                                       Lv, r0, gq * nb, J.Np, 0});
        li.close(lw, lw * ((lf.size + 15) / 16) * ngrp);
      }
      const size_t cofs = (size_t)J.j0 * esz;
      P.jin.push_back(MTrans{(const char *)B.s_ptr[J.prob] + cofs * B.ld[J.prob], xt,
                             c->perm_d.as<int32_t>(), c->geo.Nv, B.ld[J.prob], J.nrhs, J.Np, 1.0});
      P.jout.push_back(MTrans{yt, (char *)B.u_ptr[J.prob] + cofs * B.ld[J.prob],
                              c->perm_d.as<int32_t>(), c->geo.Nv, B.ld[J.prob], J.nrhs, J.Np, 1.0});
    }
    auto add_stage = [&](int kind, const void *data, size_t bytes, int64_t n) {
      DevBuf d;
      HBI_HIP(d.alloc(bytes));
      if (bytes) HBI_HIP(hipMemcpy(d.p, data, bytes, hipMemcpyHostToDevice));
      P.stages.push_back(MStagePlan{kind, nb, d.p, n});
      P.bufs.push_back(std::move(d));
    };
    const std::vector<MFAItem> kp = xcd_place(ki);
    add_stage(3, kp.data(), kp.size() * sizeof(MFAItem), (int64_t)kp.size());
    for (int k = Lmax; k >= 1; --k) {
      ItemGroups<MWAItem> wi;
      for (int q : P.jobs) {
        const MultiJob &J = B.jobs[q];
        hbi_ctx *c = J.c;
        if (k > c->plan.Lmax) continue;
        const char *F = c->F.as<char>();
        char *zb = ws + J.z_off * esz;
        const int ngrp = (J.Np / 16 + nb - 1) / nb;
        const uint16_t *fidx = c->Fi.as<uint16_t>();
        // one group per unit (every item reads its za, zb and factors)
        for (const WUnit &U : c->units_h[k]) {
          for (int gq = 0; gq < ngrp; ++gq)
            for (int r0 = 0; r0 < U.c; r0 += 16)
              wi.items.push_back(MWAItem{F + U.foff * esz, fidx + U.ioff, zb + U.zin * J.Np * esz,
                                         zb + U.zouta * J.Np * esz, zb + U.zoutb * J.Np * esz,
                                         U.ra, U.rb, U.c, r0, gq * nb, J.Np});
          wi.close(U.ra + U.rb, (double)(U.ra + U.rb) * ((U.c + 15) / 16) * ngrp);
        }
      }
      const std::vector<MWAItem> w = xcd_place(wi);
      add_stage(4, w.data(), w.size() * sizeof(MWAItem), (int64_t)w.size());
    }
    const std::vector<MVAItem> lp = xcd_place(li);
    add_stage(5, lp.data(), lp.size() * sizeof(MVAItem), (int64_t)lp.size());
    upload(P.jin_d, P.jin);
    upload(P.jout_d, P.jout);
  }
  B.nb = nb;
}

void launch_passes(BatchCache &B, hipStream_t st) {
  for (auto &P : B.passes) {
    if (B.prec == HBI_F64) {
      HBI_HIP(launch_gather_in<double>(P.jin_d.as<MTrans>(), (int64_t)P.jin.size(), P.maxNv,
                                       P.maxjt, st));
      for (auto &sp : P.stages) HBI_HIP(launch_multi_stage<double>(sp, st));
      HBI_HIP(launch_scatter_out<double>(P.jout_d.as<MTrans>(), (int64_t)P.jout.size(), P.maxNv,
                                         P.maxjt, st));
    } else {
      HBI_HIP(launch_gather_in<float>(P.jin_d.as<MTrans>(), (int64_t)P.jin.size(), P.maxNv,
                                      P.maxjt, st));
      for (auto &sp : P.stages) HBI_HIP(launch_multi_stage<float>(sp, st));
      HBI_HIP(launch_scatter_out<float>(P.jout_d.as<MTrans>(), (int64_t)P.jout.size(), P.maxNv,
                                        P.maxjt, st));
    }
  }
}

// Tuned column-tile width per (architecture, precision, direction, widest
// column-tile count, rank bucket), shared by every batch of the process and
// optionally kept in the JSON file named by HBI_TUNE_CACHE.
std::map<std::string, int> &tune_table() {
  static std::map<std::string, int> t;
  static bool loaded = false;
  if (!loaded) {
    loaded = true;
    const char *path = std::getenv("HBI_TUNE_CACHE");
    if (path && *path) {
      std::ifstream f(path);
      std::string line;
      while (std::getline(f, line)) {
        const auto q1 = line.find('"'), q2 = line.find('"', q1 + 1), colon = line.find(':', q2);
        if (q1 == std::string::npos || q2 == std::string::npos || colon == std::string::npos) continue;
        t[line.substr(q1 + 1, q2 - q1 - 1)] = std::atoi(line.c_str() + colon + 1);
      }
    }
  }
  return t;
}

void save_tune_table() {
  const char *path = std::getenv("HBI_TUNE_CACHE");
  if (!path || !*path) return;
  std::ofstream f(path);
  f << "{\n";
  size_t i = 0;
  for (auto &kv : tune_table())
    f << "  \"" << kv.first << "\": " << kv.second << (++i < tune_table().size() ? ",\n" : "\n");
  f << "}\n";
}

double time_passes(BatchCache &B, int reps) {
  hipEvent_t a, b;
  HBI_HIP(hipEventCreate(&a));
  HBI_HIP(hipEventCreate(&b));
  launch_passes(B, B.gst);   // warm
  HBI_HIP(hipEventRecord(a, B.gst));
  for (int r = 0; r < reps; ++r) launch_passes(B, B.gst);
  HBI_HIP(hipEventRecord(b, B.gst));
  HBI_HIP(hipEventSynchronize(b));
  float ms = 0;
  HBI_HIP(hipEventElapsedTime(&ms, a, b));
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  return ms / reps;
}

void multi_apply(hbi_ctx *c0, const std::vector<hbi_ctx *> &ctxs, const std::vector<const void *> &s,
                 const std::vector<void *> &u, const std::vector<int32_t> &nrhs,
                 const std::vector<int64_t> &ld, bool adj = false) {
  const int prec = ctxs[0]->prec;
  for (size_t p = 0; p < ctxs.size(); ++p) {
    HBI_REQUIRE(ctxs[p] && ctxs[p]->state == 2, HBI_ERR_STATE, "batched apply before build");
    HBI_REQUIRE(ctxs[p]->prec == prec, HBI_ERR_ARG, "batched problems differ in precision");
    HBI_REQUIRE(ctxs[p]->device == c0->device, HBI_ERR_ARG, "batched problems on different devices");
    check_apply_args(ctxs[p], s[p], u[p], nrhs[p], ld[p]);
  }
  std::vector<uint64_t> gens(ctxs.size());
  for (size_t p = 0; p < ctxs.size(); ++p) gens[p] = ctxs[p]->build_gen;
  std::shared_ptr<BatchCache> &slot = adj ? c0->batch_adj : c0->batch;
  std::shared_ptr<BatchCache> B = slot;
  const bool persistent = env_int("HBI_BATCHED_PERSISTENT", 0) != 0;
  const bool same = B && B->ctxs == ctxs && B->gens == gens && B->nrhs == nrhs &&
                    B->prec == prec && B->persistent == persistent;
  if (!same) {
    // the previous graph, if any, finishes and frees its workspace first
    B.reset();
    slot.reset();
    B = std::make_shared<BatchCache>();
    B->adj = adj;
    B->ctxs = ctxs;
    B->gens = gens;
    B->nrhs = nrhs;
    B->prec = prec;
    B->s_ptr = s;
    B->u_ptr = u;
    B->ld = ld;
    HBI_HIP(hipStreamCreateWithFlags(&B->gst, hipStreamNonBlocking));
    HBI_HIP(hipEventCreateWithFlags(&B->e_in, hipEventDisableTiming));
    HBI_HIP(hipEventCreateWithFlags(&B->e_out, hipEventDisableTiming));
    HBI_HIP(hipEventRecord(B->e_in, c0->stream));
    HBI_HIP(hipStreamWaitEvent(B->gst, B->e_in, 0));
    plan_passes(*B, nrhs);
    // autotune the column-tile width on this batch (cached per process)
    // key: architecture, precision, direction, widest column-tile count and
    // the rank bucket (power of two >= the largest transfer unit's rows)
    int maxjt = 1;
    for (auto &J : B->jobs) maxjt = std::max(maxjt, J.Np / 16);
    int rmax = 1;
    for (hbi_ctx *cc : ctxs)
      if (cc)
        for (const auto &lev : cc->units_h)
          for (const WUnit &U : lev) rmax = std::max(rmax, U.ra + U.rb);
    int rbucket = 16;
    while (rbucket < rmax) rbucket *= 2;
    hipDeviceProp_t prop;
    HBI_HIP(hipGetDeviceProperties(&prop, c0->device));
    std::string arch(prop.gcnArchName);
    arch = arch.substr(0, arch.find(':'));
    const std::string key = arch + ":" + (prec == HBI_F64 ? "f64" : "f32") + (adj ? ":adj" : "") +
                            ":jt" + std::to_string(maxjt) + ":r" + std::to_string(rbucket);
    auto items = [&](int nb) { if (adj) build_items_adj(*B, nb); else build_items(*B, nb); };
    auto &tt = tune_table();
    // the tuned choice is kept as nb * 16 + ku (ku = 0: the width's default
    // k-steps per chunk; entries written before the k-step knob are nb alone)
    auto set_ku = [&](int ku) {
      for (auto &P : B->passes)
        for (auto &sp : P.stages) sp.ku = ku;
    };
    auto valid = [&](int nb, int ku) {
      if (!(nb == 1 || nb == 2 || nb == 4 || nb == 8) || (nb > 1 && nb > maxjt)) return false;
      if (ku == 0) return true;
      for (int k : multi_ku_candidates(nb))
        if (k == ku) return true;
      return false;
    };
    int best = -1, best_ku = 0;
    // a cached choice is used only if it is one of the candidates this batch
    // would time (a corrupt or stale file entry is ignored and re-tuned)
    if (tt.count(key)) {
      const int v = tt[key];
      const int nb = v < 16 ? v : v / 16, ku = v < 16 ? 0 : v % 16;
      if (valid(nb, ku)) { best = nb; best_ku = ku; }
    }
    if (best < 0) {
      // the width at its default k-steps, then the k-steps at that width
      double bt = 1e300;
      for (int nb : {1, 2, 4, 8}) {
        if (nb > 1 && nb > maxjt) break;
        items(nb);
        const double t = time_passes(*B, 2);
        if (t < bt) { bt = t; best = nb; }
      }
      items(best);
      const std::vector<int> kus = multi_ku_candidates(best);
      for (size_t q = 1; q < kus.size(); ++q) {
        set_ku(kus[q]);
        const double t = time_passes(*B, 2);
        if (t < bt) { bt = t; best_ku = kus[q]; }
      }
      B->tuned_ms = bt;
      tt[key] = best * 16 + best_ku;
      save_tune_table();
    }
    items(best);
    // the persistent kernel runs every width at its default k-steps
    set_ku(persistent ? 0 : best_ku);
    B->ku = persistent ? 0 : best_ku;
    B->persistent = persistent;
    if (persistent) {
      // the passes' gathers, stages and scatters as the phases of one launch
      std::vector<MPhase> ph;
      for (auto &P : B->passes) {
        const int nx = (int)((P.maxNv + 63) / 64);
        ph.push_back(MPhase{6, nx, P.maxjt, P.jin_d.p, (int64_t)P.jin.size()});
        for (auto &sp : P.stages)
          if (sp.n) ph.push_back(MPhase{sp.kind, 0, 0, sp.items, sp.n});
        ph.push_back(MPhase{7, nx, P.maxjt, P.jout_d.p, (int64_t)P.jout.size()});
      }
      upload(B->phases_d, ph);
      B->nphase = (int)ph.size();
      if (prec == HBI_F64) HBI_HIP(persistent_grid<double>(best, c0->device, &B->pgrid));
      else HBI_HIP(persistent_grid<float>(best, c0->device, &B->pgrid));
    } else {
      HBI_HIP(hipStreamBeginCapture(B->gst, hipStreamCaptureModeRelaxed));
      launch_passes(*B, B->gst);
      HBI_HIP(hipStreamEndCapture(B->gst, &B->graph));
      HBI_HIP(hipGraphInstantiate(&B->gexec, B->graph, nullptr, nullptr, 0));
    }
    slot = B;
  } else if (B->s_ptr != s || B->u_ptr != u || B->ld != ld) {
    // new vector pointers: refresh the gather/scatter job tables
    HBI_HIP(hipStreamSynchronize(B->gst));
    B->s_ptr = s;
    B->u_ptr = u;
    B->ld = ld;
    const size_t esz = prec == HBI_F64 ? 16 : 8;
    for (auto &P : B->passes) {
      for (size_t q = 0; q < P.jobs.size(); ++q) {
        const MultiJob &J = B->jobs[P.jobs[q]];
        const size_t cofs = (size_t)J.j0 * esz * ld[J.prob];
        P.jin[q].src = (const char *)s[J.prob] + cofs;
        P.jin[q].ld = ld[J.prob];
        P.jout[q].dst = (char *)u[J.prob] + cofs;
        P.jout[q].ld = ld[J.prob];
      }
      HBI_HIP(hipMemcpy(P.jin_d.p, P.jin.data(), P.jin.size() * sizeof(MTrans), hipMemcpyHostToDevice));
      HBI_HIP(hipMemcpy(P.jout_d.p, P.jout.data(), P.jout.size() * sizeof(MTrans), hipMemcpyHostToDevice));
    }
  }
  HBI_HIP(hipEventRecord(B->e_in, c0->stream));
  HBI_HIP(hipStreamWaitEvent(B->gst, B->e_in, 0));
  if (B->persistent) {
    const MPhase *ph = B->phases_d.as<MPhase>();
    if (prec == HBI_F64) HBI_HIP(launch_multi_persistent<double>(ph, B->nphase, B->nb, B->pgrid, B->gst));
    else HBI_HIP(launch_multi_persistent<float>(ph, B->nphase, B->nb, B->pgrid, B->gst));
    ++c0->n_persistent;
  } else {
    HBI_HIP(hipGraphLaunch(B->gexec, B->gst));
  }
  HBI_HIP(hipEventRecord(B->e_out, B->gst));
  HBI_HIP(hipStreamWaitEvent(c0->stream, B->e_out, 0));
}

}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================
// ---------------------------------------------------------------------------
// Tables from the eikonal and transport solves (hbi_tabulate)
// ---------------------------------------------------------------------------
namespace tabgen {

constexpr int DEG = 8;   // polynomials keep degrees <= DEG
struct Poly {
  double c[DEG + 1][DEG + 1] = {};   // c[i][j]: coefficient of x^i y^j
};
Poly hom(const Poly &A, int k) {
  Poly B;
  for (int i = 0; i <= k && i <= DEG; ++i)
    if (k - i <= DEG) B.c[i][k - i] = A.c[i][k - i];
  return B;
}
Poly mul(const Poly &A, const Poly &B) {
  Poly C;
  for (int i = 0; i <= DEG; ++i)
    for (int j = 0; i + j <= DEG; ++j) {
      if (A.c[i][j] == 0.0) continue;
      for (int k = 0; i + j + k <= DEG; ++k)
        for (int l = 0; i + j + k + l <= DEG; ++l) C.c[i + k][j + l] += A.c[i][j] * B.c[k][l];
    }
  return C;
}
Poly ddx(const Poly &A) {
  Poly C;
  for (int i = 1; i <= DEG; ++i)
    for (int j = 0; j <= DEG; ++j) C.c[i - 1][j] = i * A.c[i][j];
  return C;
}
Poly ddy(const Poly &A) {
  Poly C;
  for (int i = 0; i <= DEG; ++i)
    for (int j = 1; j <= DEG; ++j) C.c[i][j - 1] = j * A.c[i][j];
  return C;
}
void axpy(Poly &Y, double a, const Poly &X) {
  for (int i = 0; i <= DEG; ++i)
    for (int j = 0; j <= DEG; ++j) Y.c[i][j] += a * X.c[i][j];
}
Poly lap(const Poly &A) {
  Poly L = ddx(ddx(A));
  axpy(L, 1.0, ddy(ddy(A)));
  return L;
}
Poly gdot(const Poly &A, const Poly &B) {
  Poly G = mul(ddx(A), ddx(B));
  axpy(G, 1.0, mul(ddy(A), ddy(B)));
  return G;
}

// Homogeneous parts of tau^2 (T_0..T_6), v0 (B_0..B_4), v1 (C_0..C_2) about
// a source from the Taylor coefficients S[i][j] of n^2 (i + j <= 4), by the
// recursions of Sec. 2.2 (eq. recursiveT, eq. recursiveB, eq. C0, C1 and
// recursiveC; d = 2), summed into TAB_PD x TAB_PD arrays.
void taylor_sums(const double *S25, TabSource &src) {
  const int PT = 6, PS = 4, PB = 4, PC = 2, d = 2;
  Poly Sf;
  for (int i = 0; i <= 4; ++i)
    for (int j = 0; i + j <= 4; ++j) Sf.c[i][j] = S25[5 * i + j];
  std::vector<Poly> Sk(PS + 1), T(PT + 1), B(PB + 1), C(PC + 1);
  for (int k = 0; k <= PS; ++k) Sk[k] = hom(Sf, k);
  const double S0 = Sk[0].c[0][0];
  if (!(S0 > 0)) throw Error{HBI_ERR_ARG, "hbi_tabulate: n^2 must be positive at every node"};
  T[2].c[2][0] = T[2].c[0][2] = S0;
  for (int P = 3; P <= PT; ++P) {
    Poly acc;
    for (int k = 1; k <= P - 2; ++k)
      if (k <= PS) axpy(acc, 1.0, mul(Sk[k], T[P - k]));
    for (int k = 2; k <= P - 2; ++k) axpy(acc, -0.25, gdot(T[k + 1], T[P - k + 1]));
    T[P] = hom(acc, P);
    for (auto &row : T[P].c)
      for (double &v : row) v /= (P - 1) * S0;
  }
  B[0].c[0][0] = 1.0 / (2.0 * std::sqrt(M_PI));   // n0^(d-2) / (2 pi^((d-1)/2)), d = 2
  for (int P = 1; P <= PB; ++P) {
    Poly acc;
    for (int k = 1; k <= P - 1; ++k) axpy(acc, -1.0, gdot(B[k], T[P + 2 - k]));
    for (int k = 0; k <= P - 1; ++k) {
      axpy(acc, -0.5, mul(B[k], lap(T[P + 2 - k])));
      axpy(acc, (double)d, mul(B[k], Sk[P - k]));
    }
    B[P] = hom(acc, P);
    for (auto &row : B[P].c)
      for (double &v : row) v /= 2.0 * P * S0;
  }
  for (int P = 0; P <= PC; ++P) {
    Poly acc = lap(B[P + 2]);
    for (auto &row : acc.c)
      for (double &v : row) v *= 0.5;
    for (int k = 1; k <= P - 1; ++k) axpy(acc, -1.0, gdot(C[k], T[P + 2 - k]));
    for (int k = 0; k <= P - 1; ++k) {
      axpy(acc, -0.5, mul(C[k], lap(T[P + 2 - k])));
      axpy(acc, -(2.0 - d), mul(C[k], Sk[P - k]));
    }
    C[P] = hom(acc, P);
    for (auto &row : C[P].c)
      for (double &v : row) v /= 2.0 * (P + 1) * S0;
  }
  for (int a = 0; a < TAB_PD; ++a)
    for (int b = 0; a + b < TAB_PD; ++b) {
      double t = 0, v = 0, w = 0;
      for (int k = 0; k <= PT; ++k) t += T[k].c[a][b];
      for (int k = 0; k <= PB; ++k) v += B[k].c[a][b];
      for (int k = 0; k <= PC; ++k) w += C[k].c[a][b];
      src.T[a * TAB_PD + b] = t;
      src.B[a * TAB_PD + b] = v;
      src.C[a * TAB_PD + b] = w;
    }
  src.n0 = std::sqrt(S0);
}

void tabulate(hbi_ctx *c, const hbi_medium2d *m, int32_t nI, const int32_t nbox[2],
              const double box_origin[2], double box_size, double h0, int32_t margin,
              double *tau2, double *v0, double *v1) {
  HBI_REQUIRE(m && nbox && box_origin && tau2 && v0 && v1 && m->n2 && m->taylor, HBI_ERR_ARG,
              "hbi_tabulate: null argument");
  HBI_REQUIRE(nI >= 2 && nI <= HBI_MAX_NI, HBI_ERR_ARG, "hbi_tabulate: nI must be in 2..16");
  HBI_REQUIRE(nbox[0] >= 1 && nbox[1] >= 1 && box_size > 0 && h0 > 0 && margin >= 4,
              HBI_ERR_ARG, "hbi_tabulate: bad nbox, box_size, h0 or margin");
  HBI_REQUIRE(m->n[0] >= 6 && m->n[1] >= 6 && m->spacing > 0, HBI_ERR_ARG,
              "hbi_tabulate: the medium grid needs >= 6 points per axis and spacing > 0");
  const int64_t NT64 = (int64_t)nbox[0] * nbox[1] * nI * nI;
  HBI_REQUIRE(NT64 <= 16384, HBI_ERR_ARG, "hbi_tabulate: more than 16384 table nodes");
  const int32_t NT = (int32_t)NT64;
  // nodes in table order (box b = bx + nbox0 by, node a = k1 + nI k2)
  std::vector<double> nodes(2 * (size_t)NT);
  for (int32_t b = 0; b < nbox[0] * nbox[1]; ++b)
    for (int32_t a = 0; a < nI * nI; ++a) {
      const int32_t q = b * nI * nI + a, bx = b % nbox[0], by = b / nbox[0];
      const int32_t k1 = a % nI, k2 = a / nI;
      nodes[2 * q] = box_origin[0] +
                     (bx + 0.5 * (1.0 + std::cos((2.0 * k1 + 1.0) * M_PI / (2.0 * nI)))) * box_size;
      nodes[2 * q + 1] = box_origin[1] +
                         (by + 0.5 * (1.0 + std::cos((2.0 * k2 + 1.0) * M_PI / (2.0 * nI)))) * box_size;
    }
  const double lo[2] = {box_origin[0], box_origin[1]};
  const double hi[2] = {box_origin[0] + nbox[0] * box_size, box_origin[1] + nbox[1] * box_size};
  // source grids: aligned with the node, covering the region plus margin
  std::vector<TabSource> src(NT);
  int64_t npmax = 0;
  for (int32_t q = 0; q < NT; ++q) {
    TabSource &S = src[q];
    const double x0 = nodes[2 * q], y0 = nodes[2 * q + 1];
    const int32_t ia = (int32_t)std::floor((lo[0] - x0) / h0) - margin;
    const int32_t ib = (int32_t)std::ceil((hi[0] - x0) / h0) + margin;
    const int32_t ja = (int32_t)std::floor((lo[1] - y0) / h0) - margin;
    const int32_t jb = (int32_t)std::ceil((hi[1] - y0) / h0) + margin;
    S.h = h0;
    S.nx = ib - ia + 1;
    S.ny = jb - ja + 1;
    S.i0 = -ia;
    S.j0 = -ja;
    S.gx0 = x0 + ia * h0;
    S.gy0 = y0 + ja * h0;
    HBI_REQUIRE((int64_t)S.nx * S.ny <= ((int64_t)1 << 24), HBI_ERR_ARG,
                "hbi_tabulate: source grid larger than 2^24 points (h0 too small)");
    // the quintic of the medium needs points -2 .. +3 around every grid point
    const double fx0 = (S.gx0 - m->origin[0]) / m->spacing, fy0 = (S.gy0 - m->origin[1]) / m->spacing;
    const double fx1 = (S.gx0 + (S.nx - 1) * h0 - m->origin[0]) / m->spacing;
    const double fy1 = (S.gy0 + (S.ny - 1) * h0 - m->origin[1]) / m->spacing;
    HBI_REQUIRE(std::floor(fx0) - 2 >= 0 && std::floor(fy0) - 2 >= 0 &&
                    std::floor(fx1) + 3 <= m->n[0] - 1 && std::floor(fy1) + 3 <= m->n[1] - 1,
                HBI_ERR_ARG, "hbi_tabulate: the medium grid does not cover the source grids");
    taylor_sums(m->taylor + 25 * (size_t)q, S);
    npmax = std::max<int64_t>(npmax, (int64_t)S.nx * S.ny);
  }
  const hipStream_t st = c->stream;
  DevBuf n2d, nodes_d, tabs, stat_d, src_d, ws;
  upload(n2d, std::vector<double>(m->n2, m->n2 + (size_t)m->n[0] * m->n[1]));
  upload(nodes_d, nodes);
  upload(src_d, src);
  HBI_HIP(tabs.alloc(3 * sizeof(double) * (size_t)NT * NT));
  HBI_HIP(stat_d.alloc(3 * sizeof(int32_t) * (size_t)NT));
  TabMedium med{n2d.as<double>(), m->n[0], m->n[1], m->origin[0], m->origin[1], m->spacing};
  const int64_t stride = 11 * npmax;
  // sources in batches whose workspace fits about 2 GiB
  const int64_t per = std::max<int64_t>(1, ((int64_t)2 << 30) / (stride * (int64_t)sizeof(double)));
  const int32_t batch = (int32_t)std::min<int64_t>(NT, per);
  HBI_HIP(ws.alloc(sizeof(double) * (size_t)stride * batch));
  double *F0 = tabs.as<double>(), *F1 = F0 + (size_t)NT * NT, *F2 = F1 + (size_t)NT * NT;
  const double t0 = now_s();
  for (int32_t s0 = 0; s0 < NT; s0 += batch) {
    const int32_t nb = std::min(batch, NT - s0);
    // column s0 + s of every table: offset the table pointers by s0 columns
    HBI_HIP(launch_tabulate(src_d.as<TabSource>() + s0, nb, med, ws.as<double>(), stride, npmax,
                            nodes_d.as<double>(), NT, F0 + s0, F1 + s0, F2 + s0,
                            stat_d.as<int32_t>() + 3 * s0, 1e-13, 20000, st));
    HBI_HIP(hipStreamSynchronize(st));
  }
  HBI_HIP(launch_tab_symmetrise(F0, F1, F2, NT, st));
  std::vector<int32_t> status(3 * (size_t)NT);
  HBI_HIP(hipMemcpyAsync(status.data(), stat_d.p, status.size() * sizeof(int32_t),
                         hipMemcpyDeviceToHost, st));
  HBI_HIP(hipMemcpyAsync(tau2, F0, sizeof(double) * (size_t)NT * NT, hipMemcpyDeviceToHost, st));
  HBI_HIP(hipMemcpyAsync(v0, F1, sizeof(double) * (size_t)NT * NT, hipMemcpyDeviceToHost, st));
  HBI_HIP(hipMemcpyAsync(v1, F2, sizeof(double) * (size_t)NT * NT, hipMemcpyDeviceToHost, st));
  HBI_HIP(hipStreamSynchronize(st));
  c->tab_s = now_s() - t0;
  c->tab_sources = NT;
  c->tab_rounds_max = 0;
  c->tab_point_updates = 0;
  for (int32_t q = 0; q < NT; ++q)
    for (int e = 0; e < 3; ++e) {
      if (status[3 * q + e] < 0)
        throw Error{HBI_ERR_NUMERIC, "hbi_tabulate: the sweeps of node " + std::to_string(q) +
                                         " (equation " + std::to_string(e) + ") did not converge"};
      c->tab_rounds_max = std::max(c->tab_rounds_max, status[3 * q + e]);
      // held points: the (2 P - 1)^2 square, P = 6, 4, 2 (inside the grid)
      const int64_t held = (int64_t)(11 - 4 * e) * (11 - 4 * e);
      c->tab_point_updates +=
          4.0 * status[3 * q + e] * (double)((int64_t)src[q].nx * src[q].ny - held);
    }
}

}  // namespace tabgen

namespace {
// Index and descriptor bytes one forward apply reads (algorithmic).
double apply_index_bytes(const ApplyPlan &ap) {
  double b = ap.v_idx + ap.f_idx;
  for (double w : ap.w_idx) b += w;
  return b;
}
// Algorithmic bytes of one forward single-RHS product: factor entries,
// vectors read and written, index lists, positions and descriptors.
double apply_bytes(const ApplyPlan &ap, double esz) {
  double e = ap.v_elems + ap.f_elems;
  for (double w : ap.w_elems) e += w;
  return e * esz + apply_index_bytes(ap);
}
// Bytes of the inclusion operators one apply streams: G twice (the
// K^{v2s} gather and the K^{s2v} scatter), (K^{s2s})^{-1} once, and the
// cell vectors read and written.
// With G as a butterfly: its factors twice (the transposed and the forward
// product), (K^{s2s})^{-1} once, the cell vectors read and written, and the
// index store twice.
double inclusion_apply_bytes(const hbi_ctx *c) {
  if (!c->inc_ns || c->state < 2) return 0.0;
  const double esz = c->prec == HBI_F64 ? 16.0 : 8.0;
  const double nv = (double)c->geo.Nv, ns = (double)c->inc_ns;
  if (c->inc_plan.bf)
    return esz * (2.0 * (double)c->s2v_entries + ns * ns + 2.0 * nv) + 2.0 * (double)c->s2v_idx.n;
  return esz * (2.0 * nv * ns + ns * ns + 2.0 * nv);
}
}  // namespace

extern "C" {

hbi_status hbi_create(int device, void *hip_stream, hbi_ctx **out) {
  return guarded(nullptr, [&]() {
    HBI_REQUIRE(out, HBI_ERR_ARG, "out is NULL");
    *out = nullptr;
    int n = 0;
    HBI_HIP(hipGetDeviceCount(&n));
    HBI_REQUIRE(device >= 0 && device < n, HBI_ERR_ARG, "device index out of range");
    HBI_HIP(hipSetDevice(device));
    setup_scratch(device);
    auto c = std::make_unique<hbi_ctx>();
    c->device = device;
    c->stream = (hipStream_t)hip_stream;
    *out = c.release();
  });
}

hbi_status hbi_destroy(hbi_ctx *ctx) {
  if (!ctx) return HBI_OK;
  (void)hipSetDevice(ctx->device);
  delete ctx;
  return HBI_OK;
}

hbi_status hbi_set_stream(hbi_ctx *ctx, void *hip_stream) {
  if (!ctx) { g_err = "ctx is NULL"; return HBI_ERR_ARG; }
  ctx->stream = (hipStream_t)hip_stream;
  return HBI_OK;
}

namespace {
void clear_inclusion(hbi_ctx *c) {
  c->inc_ns = 0;
  c->inc_xy.clear(); c->inc_w.clear(); c->inc_n.clear();
  c->inc_xy_d.release(); c->inc_w_d.release(); c->inc_n_d.release();
}
}  // namespace

hbi_status hbi_load_tables(hbi_ctx *ctx, const hbi_tables *t) {
  if (!ctx) { g_err = "ctx is NULL"; return HBI_ERR_ARG; }
  return guarded(ctx, [&]() {
    HBI_REQUIRE(t, HBI_ERR_ARG, "tables is NULL");
    HBI_REQUIRE(t->dim == 2 || t->dim == 3, HBI_ERR_ARG, "dim must be 2 or 3");
    const int d = t->dim;
    int64_t Nv = 1;
    for (int a = 0; a < d; ++a) {
      HBI_REQUIRE(t->ncell[a] >= 1, HBI_ERR_ARG, "ncell must be >= 1");
      HBI_REQUIRE(t->nbox[a] >= 1, HBI_ERR_ARG, "nbox must be >= 1");
      Nv *= t->ncell[a];
    }
    HBI_REQUIRE(Nv <= ((int64_t)1 << 30), HBI_ERR_ARG, "N_v too large");
    HBI_REQUIRE(t->h > 0 && std::isfinite(t->h), HBI_ERR_ARG, "h must be > 0");
    HBI_REQUIRE(t->omega > 0 && std::isfinite(t->omega), HBI_ERR_ARG, "omega must be > 0");
    HBI_REQUIRE(t->nterms == 1 || t->nterms == 2, HBI_ERR_ARG, "nterms must be 1 or 2");
    HBI_REQUIRE(t->nI >= 2 && t->nI <= HBI_MAX_NI, HBI_ERR_ARG, "nI must be in [2, 16]");
    HBI_REQUIRE(t->box_size > 0, HBI_ERR_ARG, "box_size must be > 0");
    HBI_REQUIRE(t->tau2 && t->v0 && t->slowness, HBI_ERR_ARG, "null table or slowness");
    HBI_REQUIRE(t->nterms == 1 || t->v1, HBI_ERR_ARG, "v1 is NULL but nterms == 2");
    for (int a = 0; a < d; ++a) {
      const double lo = t->origin[a], hi = t->origin[a] + t->ncell[a] * t->h;
      const double blo = t->box_origin[a], bhi = t->box_origin[a] + t->nbox[a] * t->box_size;
      const double eps = 1e-12 * std::max(1.0, std::fabs(bhi - blo));
      HBI_REQUIRE(lo + 0.5 * t->h >= blo - eps && hi - 0.5 * t->h <= bhi + eps, HBI_ERR_ARG,
                  "cell centres lie outside the table region");
    }
    hbi_ctx *c = ctx;
    c->drop_factors();
    c->state = 0;
    clear_inclusion(c);
    c->dim = d;
    c->nterms = t->nterms;
    c->nI = t->nI;
    c->NTb = 1;
    int64_t nboxes = 1;
    for (int a = 0; a < 3; ++a) {
      c->ncell[a] = a < d ? t->ncell[a] : 1;
      c->nbox[a] = a < d ? t->nbox[a] : 1;
      c->origin[a] = a < d ? t->origin[a] : 0.0;
      c->box_origin[a] = a < d ? t->box_origin[a] : 0.0;
    }
    for (int a = 0; a < d; ++a) { c->NTb *= t->nI; nboxes *= t->nbox[a]; }
    HBI_REQUIRE(nboxes * c->NTb <= (1 << 16), HBI_ERR_ARG, "table too large");
    c->NT = (int)(nboxes * c->NTb);
    c->h = t->h;
    c->omega = t->omega;
    c->box_size = t->box_size;
    c->slow_nat.assign(t->slowness, t->slowness + Nv);
    for (double v : c->slow_nat)
      HBI_REQUIRE(std::isfinite(v) && v > 0, HBI_ERR_ARG, "slowness must be finite and > 0");
    // transposed tables (FT[B*NT + A] = F[A*NT + B]) so the kernels read them contiguously
    const int64_t NT = c->NT;
    const double *src[3] = {t->tau2, t->v0, t->nterms == 2 ? t->v1 : nullptr};
    std::vector<double> tr((size_t)NT * NT);
    for (int k = 0; k < 3; ++k) {
      if (!src[k]) { std::fill(tr.begin(), tr.end(), 0.0); }
      else {
        const double *F = src[k];
        parallel_for(NT, [&](int64_t b0, int64_t b1) {
          for (int64_t B = b0; B < b1; ++B)
            for (int64_t A = 0; A < NT; ++A) tr[B * NT + A] = F[A * NT + B];
        });
      }
      upload(c->FT_d[k], tr);
    }
    setup_cells(c);
    c->state = 1;
  });
}

namespace {
void copy_dev(DevBuf &dst, const DevBuf &src, hipStream_t st) {
  HBI_HIP(dst.alloc(src.n));
  if (src.n) HBI_HIP(hipMemcpyAsync(dst.p, src.p, src.n, hipMemcpyDeviceToDevice, st));
}
}  // namespace

hbi_status hbi_load_tables_from(hbi_ctx *ctx, const hbi_ctx *src, double omega) {
  if (!ctx) { g_err = "ctx is NULL"; return HBI_ERR_ARG; }
  return guarded(ctx, [&]() {
    HBI_REQUIRE(src, HBI_ERR_ARG, "src is NULL");
    HBI_REQUIRE(std::isfinite(omega) && omega > 0, HBI_ERR_ARG, "omega must be finite and > 0");
    HBI_REQUIRE(src->device == ctx->device, HBI_ERR_ARG, "src is on another device");
    HBI_REQUIRE(src->state >= 1, HBI_ERR_STATE, "src has no tables");
    hbi_ctx *c = ctx;
    c->drop_factors();
    if (c == src) {
      c->omega = omega;
      eval_self_terms(c);
      c->state = 1;
      return;
    }
    c->state = 0;
    // tables are constant once loaded; src's stream may still run its own
    // builds or applies, which only read them
    HBI_HIP(hipStreamSynchronize(src->stream));
    c->inc_ns = src->inc_ns;
    c->inc_xy = src->inc_xy; c->inc_w = src->inc_w; c->inc_n = src->inc_n;
    copy_dev(c->inc_xy_d, src->inc_xy_d, c->stream);
    copy_dev(c->inc_w_d, src->inc_w_d, c->stream);
    copy_dev(c->inc_n_d, src->inc_n_d, c->stream);
    c->dim = src->dim; c->nterms = src->nterms; c->nI = src->nI;
    c->NTb = src->NTb; c->NT = src->NT;
    for (int a = 0; a < 3; ++a) {
      c->ncell[a] = src->ncell[a]; c->nbox[a] = src->nbox[a];
      c->origin[a] = src->origin[a]; c->box_origin[a] = src->box_origin[a];
    }
    c->h = src->h; c->box_size = src->box_size;
    c->omega = omega;
    c->slow_nat = src->slow_nat;
    for (int k = 0; k < 3; ++k) copy_dev(c->FT_d[k], src->FT_d[k], c->stream);
    if (src->geo_leaf == c->leaf() && src->geo_band == c->band()) {
      // same cluster tree: copy it and the per-cell data
      c->geo = src->geo;
      c->geo_leaf = src->geo_leaf;
      c->geo_band = src->geo_band;
      copy_dev(c->perm_d, src->perm_d, c->stream);
      copy_dev(c->slow_d, src->slow_d, c->stream);
      copy_dev(c->xyz_d, src->xyz_d, c->stream);
      copy_dev(c->lw_d, src->lw_d, c->stream);
      copy_dev(c->box_d, src->box_d, c->stream);
      copy_dev(c->cellof_d, src->cellof_d, c->stream);
      c->box_h = src->box_h;
      eval_self_terms(c);
    } else {
      setup_cells(c);
    }
    HBI_HIP(hipStreamSynchronize(c->stream));
    c->state = 1;
  });
}

hbi_status hbi_set_inclusion(hbi_ctx *ctx, int32_t ns, const double *xy, const double *w,
                             const double *slowness) {
  if (!ctx) { g_err = "ctx is NULL"; return HBI_ERR_ARG; }
  return guarded(ctx, [&]() {
    hbi_ctx *c = ctx;
    HBI_REQUIRE(c->state >= 1, HBI_ERR_STATE, "inclusion before tables");
    HBI_REQUIRE(c->dim == 2, HBI_ERR_ARG, "curve inclusions are 2D");
    HBI_REQUIRE(ns >= 0 && ns <= HBI_MAX_INCLUSION, HBI_ERR_ARG,
                "ns must be in [0, " + std::to_string(HBI_MAX_INCLUSION) + "]");
    if (ns > 0) {
      HBI_REQUIRE(xy && w && slowness, HBI_ERR_ARG, "null segment array");
      for (int32_t i = 0; i < ns; ++i) {
        HBI_REQUIRE(std::isfinite(w[i]) && w[i] > 0, HBI_ERR_ARG, "segment lengths must be > 0");
        HBI_REQUIRE(std::isfinite(slowness[i]) && slowness[i] > 0, HBI_ERR_ARG,
                    "slowness must be finite and > 0");
        for (int a = 0; a < 2; ++a) {
          const double x = xy[2 * i + a];
          const double blo = c->box_origin[a], bhi = blo + c->nbox[a] * c->box_size;
          HBI_REQUIRE(std::isfinite(x) && x >= blo && x <= bhi, HBI_ERR_ARG,
                      "segment centres lie outside the table region");
        }
      }
    }
    c->drop_factors();
    c->state = 0;
    clear_inclusion(c);
    if (ns > 0) {
      c->inc_ns = ns;
      c->inc_xy.assign(xy, xy + 2 * (size_t)ns);
      c->inc_w.assign(w, w + ns);
      c->inc_n.assign(slowness, slowness + ns);
      upload(c->inc_xy_d, c->inc_xy);
      upload(c->inc_w_d, c->inc_w);
      upload(c->inc_n_d, c->inc_n);
    }
    setup_cells(c);
    c->state = 1;
  });
}

hbi_status hbi_set_build_opts(hbi_ctx *ctx, const hbi_build_opts *opts) {
  if (!ctx) { g_err = "ctx is NULL"; return HBI_ERR_ARG; }
  return guarded(ctx, [&]() {
    if (!opts) { ctx->opts = hbi_build_opts{}; return; }
    HBI_REQUIRE(opts->leaf_size <= HBI_MAX_LEAF, HBI_ERR_ARG, "leaf_size must be <= 64");
    HBI_REQUIRE(std::isfinite(opts->chi) && std::isfinite(opts->neighbor_radius), HBI_ERR_ARG,
                "non-finite option");
    ctx->opts = *opts;
  });
}

hbi_status hbi_build(hbi_ctx *ctx, double tol, hbi_prec prec) {
  if (!ctx) { g_err = "ctx is NULL"; return HBI_ERR_ARG; }
  return guarded(ctx, [&]() {
    HBI_REQUIRE(ctx->state >= 1, HBI_ERR_STATE, "build before tables");
    HBI_REQUIRE(tol > 0 && tol < 1, HBI_ERR_ARG, "tol must be in (0, 1)");
    HBI_REQUIRE(prec == HBI_F64 || prec == HBI_F32, HBI_ERR_ARG, "bad precision");
    ctx->drop_factors();
    ctx->prec = prec;
    ctx->tol = tol;
    build_factors(ctx, tol);
    if (ctx->inc_ns > 0) {
      build_inclusion(ctx);
      ctx->t_build += ctx->t_inc;
    }
    ctx->build_gen = ++g_build_gen;
    ctx->state = 2;
  });
}

hbi_status hbi_apply(hbi_ctx *ctx, const void *s, void *u, int32_t nrhs, int64_t ld) {
  if (!ctx) { g_err = "ctx is NULL"; return HBI_ERR_ARG; }
  return guarded(ctx, [&]() {
    if (nrhs >= 2 && !ctx->profiling)
      multi_apply(ctx, {ctx}, {s}, {u}, {nrhs}, {ld});
    else
      do_apply(ctx, s, u, nrhs, ld, false);
    apply_inclusion(ctx, s, u, nrhs, ld, false);
  });
}

hbi_status hbi_apply_batched(hbi_ctx *const *ctx, int32_t nprob, const void *const *s,
                             void *const *u, const int32_t *nrhs, const int64_t *ld) {
  if (!ctx || nprob < 1 || !ctx[0]) { g_err = "ctx is NULL or nprob < 1"; return HBI_ERR_ARG; }
  return guarded(ctx[0], [&]() {
    HBI_REQUIRE(s && u && nrhs && ld, HBI_ERR_ARG, "null argument array");
    for (int32_t p = 0; p < nprob; ++p)
      HBI_REQUIRE(!ctx[p] || ctx[p]->inc_ns == 0, HBI_ERR_ARG,
                  "operators with an inclusion are applied by hbi_apply");
    std::vector<hbi_ctx *> cs(ctx, ctx + nprob);
    std::vector<const void *> sv(s, s + nprob);
    std::vector<void *> uv(u, u + nprob);
    std::vector<int32_t> nv(nrhs, nrhs + nprob);
    std::vector<int64_t> lv(ld, ld + nprob);
    multi_apply(ctx[0], cs, sv, uv, nv, lv);
  });
}

hbi_status hbi_tabulate(hbi_ctx *ctx, const hbi_medium2d *m, int32_t nI, const int32_t nbox[2],
                        const double box_origin[2], double box_size, double h0, int32_t margin,
                        double *tau2, double *v0, double *v1) {
  if (!ctx) { g_err = "ctx is NULL"; return HBI_ERR_ARG; }
  return guarded(ctx, [&]() {
    tabgen::tabulate(ctx, m, nI, nbox, box_origin, box_size, h0, margin, tau2, v0, v1);
  });
}

hbi_status hbi_apply_noalloc(hbi_ctx *ctx, const void *s, void *u, int32_t nrhs, int64_t ld) {
  if (!ctx) { g_err = "ctx is NULL"; return HBI_ERR_ARG; }
  return guarded(ctx, [&]() {
    HBI_REQUIRE(ctx->state == 2, HBI_ERR_STATE, "apply before build");
    HBI_REQUIRE(ctx->inc_ns == 0, HBI_ERR_ARG,
                "hbi_apply_noalloc applies the volume operator only (the context has a curve "
                "inclusion)");
    const size_t esz = ctx->prec == HBI_F64 ? 16 : 8;
    const size_t need = esz * (size_t)std::max<int64_t>(ctx->zalloc, 1);
    if (need > (size_t)HBI_NOALLOC_SCRATCH_BYTES)
      throw Error{HBI_ERR_ARG, "hbi_apply_noalloc: the product needs " + std::to_string(need) +
                                   " bytes of scratch, more than the fixed " +
                                   std::to_string((size_t)HBI_NOALLOC_SCRATCH_BYTES) +
                                   " bytes per device"};
    do_apply(ctx, s, u, nrhs, ld, false, scratch_ptr(ctx->device));
  });
}
hbi_status hbi_apply_adjoint(hbi_ctx *ctx, const void *s, void *u, int32_t nrhs, int64_t ld) {
  if (!ctx) { g_err = "ctx is NULL"; return HBI_ERR_ARG; }
  return guarded(ctx, [&]() {
    if (nrhs >= 2 && !ctx->profiling)
      multi_apply(ctx, {ctx}, {s}, {u}, {nrhs}, {ld}, true);
    else
      do_apply(ctx, s, u, nrhs, ld, true);
    apply_inclusion(ctx, s, u, nrhs, ld, true);
  });
}

hbi_status hbi_entries(hbi_ctx *ctx, const int32_t *rows, int32_t m, const int32_t *cols,
                       int32_t n, void *out) {
  if (!ctx) { g_err = "ctx is NULL"; return HBI_ERR_ARG; }
  return guarded(ctx, [&]() {
    HBI_REQUIRE(ctx->state >= 1, HBI_ERR_STATE, "entries before tables");
    HBI_REQUIRE(m >= 0 && n >= 0, HBI_ERR_ARG, "negative size");
    if (m == 0 || n == 0) return;
    HBI_REQUIRE(rows && cols && out, HBI_ERR_ARG, "null pointer");
    const int64_t Nv = ctx->geo.Nv;
    std::vector<int32_t> rp(m), cp(n);
    for (int32_t i = 0; i < m; ++i) {
      HBI_REQUIRE(rows[i] >= 0 && rows[i] < Nv, HBI_ERR_ARG, "row index out of range");
      rp[i] = ctx->geo.ipos[rows[i]];
    }
    for (int32_t j = 0; j < n; ++j) {
      HBI_REQUIRE(cols[j] >= 0 && cols[j] < Nv, HBI_ERR_ARG, "column index out of range");
      cp[j] = ctx->geo.ipos[cols[j]];
    }
    std::vector<BlockIn> bin;
    const int32_t CW = 256;
    for (int32_t j0 = 0; j0 < n; j0 += CW) {
      const int32_t nn = std::min(CW, n - j0);
      bin.push_back(BlockIn{rp.data(), m, cp.data() + j0, nn, (double2 *)out + (int64_t)j0 * m});
    }
    Batcher B(ctx);
    B.run(bin, false, 0.0, nullptr, [](int64_t, int64_t) {});
  });
}

hbi_status hbi_set_profiling(hbi_ctx *ctx, int32_t enable) {
  if (!ctx) { g_err = "ctx is NULL"; return HBI_ERR_ARG; }
  return guarded(ctx, [&]() {
    ctx->profiling = enable != 0;
    if (ctx->profiling) {
      HBI_HIP(hipStreamSynchronize(ctx->stream));
      ctx->prof.clear();
    }
  });
}

hbi_status hbi_get_profile(hbi_ctx *ctx, char *json, int64_t cap) {
  if (!ctx) { g_err = "ctx is NULL"; return HBI_ERR_ARG; }
  return guarded(ctx, [&]() {
    HBI_REQUIRE(json && cap > 0, HBI_ERR_ARG, "null or empty output buffer");
    HBI_HIP(hipStreamSynchronize(ctx->stream));
    struct Agg { std::string name; int64_t n = 0; double ms = 0, bytes = 0; };
    std::vector<Agg> agg;
    for (auto &r : ctx->prof.recs) {
      float ms = 0.f;
      HBI_HIP(hipEventElapsedTime(&ms, r.a, r.b));
      auto it = std::find_if(agg.begin(), agg.end(), [&](const Agg &a) { return a.name == r.name; });
      if (it == agg.end()) { agg.push_back(Agg{r.name}); it = agg.end() - 1; }
      it->n += 1;
      it->ms += ms;
      it->bytes += r.bytes;
    }
    ctx->prof.clear();
    std::string out = "{\"kernels\": {";
    char buf[256];
    for (size_t i = 0; i < agg.size(); ++i) {
      std::snprintf(buf, sizeof buf, "%s\"%s\": {\"launches\": %lld, \"ms\": %.6f, \"bytes\": %.0f}",
                    i ? ", " : "", agg[i].name.c_str(), (long long)agg[i].n, agg[i].ms, agg[i].bytes);
      out += buf;
    }
    out += "}}";
    HBI_REQUIRE((int64_t)out.size() < cap, HBI_ERR_ARG, "output buffer too small");
    std::memcpy(json, out.c_str(), out.size() + 1);
  });
}

hbi_status hbi_get_info(const hbi_ctx *cctx, char *json, int64_t cap) {
  hbi_ctx *ctx = const_cast<hbi_ctx *>(cctx);
  if (!ctx) { g_err = "ctx is NULL"; return HBI_ERR_ARG; }
  if (!json || cap <= 0) { ctx->err = "null or empty output buffer"; return HBI_ERR_ARG; }
  const int64_t Nv = ctx->geo.Nv;
  const size_t esz = ctx->prec == HBI_F64 ? 16 : 8;
  // algorithmic bytes of each forward transfer launch (levels 1..L_max)
  std::string wl = "[";
  for (size_t k = 1; k < ctx->plan.w_elems.size(); ++k) {
    char t[32];
    std::snprintf(t, sizeof t, "%s%.0f", k > 1 ? ", " : "",
                  ctx->plan.w_elems[k] * (double)esz + ctx->plan.w_idx[k]);
    wl += t;
  }
  wl += "]";
  char buf[12288];
  const int len = std::snprintf(
      buf, sizeof buf,
      "{\"state\": %d, \"dim\": %d, \"N_v\": %lld, \"L_v\": %d, \"NT\": %d, \"nI\": %d, "
      "\"prec\": \"%s\", \"tol\": %.3e, \"chi\": %.3f, \"leaf_size\": %d, "
      "\"nnz_v\": %lld, \"nnz_w\": %lld, \"nnz_k\": %lld, \"nnz_dense\": %lld, "
      "\"nnz_total\": %lld, \"factor_bytes\": %lld, \"index_bytes\": %lld, \"z_entries\": %lld, "
      "\"n_id\": %lld, \"rank_max\": %d, \"rank_mean\": %.3f, \"entries_evaluated\": %lld, "
      "\"entry_tile_fill\": %.4f, \"n_id_onchip\": %lld, \"n_id_global\": %lld, \"n_id_gram\": %lld, "
      "\"id_rows_mean\": %.1f, \"id_rows_max\": %d, \"id_cols_mean\": %.1f, \"id_cmac\": %.6e, "
      "\"n_id_cols_gt64\": %lld, \"id_cmac_cols_gt64\": %.6e, \"id_cmac_cols_gt128\": %.6e, "
      "\"build_s\": %.6f, \"build_geometry_s\": %.6f, \"build_proxy_host_s\": %.6f, "
      "\"build_gpu_s\": %.6f, \"build_batch_host_setup_s\": %.6f, \"build_batch_total_s\": %.6f, "
      "\"build_compact_s\": %.6f, \"build_finalize_s\": %.6f, "
      "\"inclusion_ns\": %d, \"inclusion_bytes\": %lld, \"build_inclusion_s\": %.6f, "
      "\"inclusion_bf_levels\": %d, \"inclusion_bf_entries\": %lld, "
      "\"inclusion_bf_rank_max\": %d, "
      "\"apply_index_bytes\": %.0f, \"inclusion_apply_bytes\": %.0f, "
      "\"apply_scratch_bytes\": %lld, \"apply_bytes\": %.0f, \"wstage_items_lds\": %lld, "
      "\"wstage_items_global\": %lld, \"wstage_items_wide\": %lld, \"wstage_cap_lds\": %d, "
      "\"wstage_c_quantiles\": [%d, %d, %d, %d, %d], \"nnz_per_cell\": %.3f, "
      "\"nnz_per_cell_over_log2sq\": %.5f, \"tab_sources\": %d, \"tab_rounds_max\": %d, "
      "\"tab_point_updates\": %.0f, \"tab_s\": %.6f, \"batched_persistent_launches\": %lld, "
      "\"batched_tile_nb\": %d, \"batched_tile_ku\": %d, \"wstage_bytes_per_level\": %s}",
      ctx->state, ctx->dim, (long long)Nv, ctx->geo.Lv, ctx->NT, ctx->nI,
      ctx->prec == HBI_F64 ? "f64" : "f32", ctx->tol, ctx->chi(), ctx->leaf(),
      (long long)ctx->nnz_v, (long long)ctx->nnz_w, (long long)ctx->nnz_k, (long long)ctx->nnz_d,
      (long long)ctx->Felems, (long long)(ctx->Felems * (int64_t)esz), (long long)ctx->Fi.n,
      (long long)ctx->ztotal,
      (long long)ctx->nid, ctx->rank_max, ctx->nid ? ctx->rank_sum / ctx->nid : 0.0,
      (long long)ctx->entries_eval,
      ctx->entry_slots ? (double)ctx->entries_eval / (double)ctx->entry_slots : 0.0,
      (long long)ctx->nid_path[0], (long long)ctx->nid_path[2], (long long)ctx->nid_path[1],
      ctx->nid ? ctx->id_m_sum / ctx->nid : 0.0, ctx->id_m_max,
      ctx->nid ? ctx->id_n_sum / ctx->nid : 0.0, ctx->id_work, (long long)ctx->nid_wide,
      ctx->id_work_wide, ctx->id_work_128, ctx->t_build, ctx->t_geo, ctx->t_host, ctx->t_gpu, ctx->t_prep,
      ctx->t_wait, ctx->t_compact,
      ctx->t_final, ctx->inc_ns,
      (long long)(ctx->inc_G.n + ctx->inc_M.n + ctx->inc_MH.n + ctx->s2v_F.n + ctx->s2v_idx.n +
                  ctx->s2v_z.n),
      ctx->t_inc, ctx->inc_plan.bf ? ctx->s2v_L : -1, (long long)ctx->s2v_entries,
      ctx->s2v_rank_max,
      apply_index_bytes(ctx->plan), inclusion_apply_bytes(ctx),
      (long long)(ctx->zalloc * (int64_t)esz), apply_bytes(ctx->plan, (double)esz),
      (long long)ctx->wst_lds, (long long)ctx->wst_global, (long long)ctx->wst_wide,
      ctx->plan.cap_lds, ctx->wst_cq[0], ctx->wst_cq[1], ctx->wst_cq[2],
      ctx->wst_cq[3], ctx->wst_cq[4], Nv ? (double)ctx->Felems / (double)Nv : 0.0,
      Nv > 1 ? (double)ctx->Felems / (double)Nv / (std::log2((double)Nv) * std::log2((double)Nv))
             : 0.0,
      ctx->tab_sources, ctx->tab_rounds_max, ctx->tab_point_updates, ctx->tab_s,
      (long long)ctx->n_persistent, ctx->batch ? ctx->batch->nb : -1,
      ctx->batch ? ctx->batch->ku : -1, wl.c_str());
  if (len < 0 || len >= cap) { ctx->err = "output buffer too small"; return HBI_ERR_ARG; }
  std::memcpy(json, buf, len + 1);
  return HBI_OK;
}

const char *hbi_last_error(const hbi_ctx *ctx) {
  return ctx ? ctx->err.c_str() : g_err.c_str();
}

}  // extern "C"
