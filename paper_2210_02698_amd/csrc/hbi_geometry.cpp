#include "hbi_geometry.h"

#include <algorithm>
#include <cmath>
#include <thread>

namespace hbi {

void parallel_for(int64_t n, const std::function<void(int64_t, int64_t)> &fn) {
  if (n <= 0) return;
  unsigned hw = std::thread::hardware_concurrency();
  int64_t nt = std::max<int64_t>(1, std::min<int64_t>(hw ? hw : 4, 32));
  nt = std::min(nt, n);
  if (nt == 1) { fn(0, n); return; }
  std::vector<std::thread> th;
  const int64_t chunk = (n + nt - 1) / nt;
  for (int64_t t = 0; t < nt; ++t) {
    const int64_t a = t * chunk, b = std::min(n, a + chunk);
    if (a >= b) break;
    th.emplace_back([&fn, a, b]() { fn(a, b); });
  }
  for (auto &x : th) x.join();
}

void Geometry::build(int d, const int32_t ncell[3], int leaf) {
  dim = d;
  nc[0] = ncell[0];
  nc[1] = d >= 2 ? ncell[1] : 1;
  nc[2] = d >= 3 ? ncell[2] : 1;
  Nv = (int64_t)nc[0] * nc[1] * nc[2];
  Lv = 0;
  while (((Nv + ((int64_t)1 << Lv) - 1) >> Lv) > leaf) ++Lv;
  perm.resize(Nv);
  for (int64_t i = 0; i < Nv; ++i) perm[i] = (int32_t)i;
  const int64_t nn = ((int64_t)2 << Lv) - 1;
  nstart.assign(nn, 0);
  nend.assign(nn, 0);
  bblo.assign(nn * 3, 0);
  bbhi.assign(nn * 3, 0);
  nstart[0] = 0;
  nend[0] = (int32_t)Nv;
  for (int l = 0; l <= Lv; ++l) {
    const int64_t cnt = (int64_t)1 << l;
    parallel_for(cnt, [&](int64_t i0, int64_t i1) {
      std::vector<std::pair<int32_t, int32_t>> key;
      for (int64_t i = i0; i < i1; ++i) {
        const int64_t nd = node(l, i);
        const int32_t a = nstart[nd], b = nend[nd];
        int32_t lo[3] = {INT32_MAX, INT32_MAX, INT32_MAX}, hi[3] = {-1, -1, -1};
        for (int32_t p = a; p < b; ++p) {
          int32_t g[3];
          grid_coords(perm[p], g);
          for (int ax = 0; ax < 3; ++ax) {
            lo[ax] = std::min(lo[ax], g[ax]);
            hi[ax] = std::max(hi[ax], g[ax]);
          }
        }
        if (a == b) { for (int ax = 0; ax < 3; ++ax) { lo[ax] = 0; hi[ax] = -1; } }
        for (int ax = 0; ax < 3; ++ax) {
          bblo[nd * 3 + ax] = lo[ax];
          bbhi[nd * 3 + ax] = hi[ax];
        }
        if (l == Lv) continue;
        int axis = 0;
        for (int ax = 1; ax < dim; ++ax)
          if (hi[ax] - lo[ax] > hi[axis] - lo[axis]) axis = ax;
        key.resize(b - a);
        for (int32_t p = a; p < b; ++p) {
          int32_t g[3];
          grid_coords(perm[p], g);
          key[p - a] = {g[axis], perm[p]};
        }
        std::stable_sort(key.begin(), key.end(),
                         [](const std::pair<int32_t, int32_t> &x,
                            const std::pair<int32_t, int32_t> &y) { return x.first < y.first; });
        for (int32_t p = a; p < b; ++p) perm[p] = key[p - a].second;
        const int32_t mid = a + (b - a) / 2;
        const int64_t c0 = node(l + 1, 2 * i), c1 = node(l + 1, 2 * i + 1);
        nstart[c0] = a;
        nend[c0] = mid;
        nstart[c1] = mid;
        nend[c1] = b;
      }
    });
  }
  ipos.resize(Nv);
  for (int64_t p = 0; p < Nv; ++p) ipos[perm[p]] = (int32_t)p;
}

void Geometry::build_bands(int width) {
  const int64_t nn = node(Lv, 0);   // nodes at levels < Lv
  band_off.assign(nn + 1, 0);
  std::vector<std::vector<int32_t>> per(nn);
  parallel_for(nn, [&](int64_t n0, int64_t n1) {
    for (int64_t nd = n0; nd < n1; ++nd) {
      const int32_t a = nstart[nd], b = nend[nd];
      auto &out = per[nd];
      for (int32_t p = a; p < b; ++p) {
        int32_t g[3];
        grid_coords(perm[p], g);
        bool edge = false;
        const int wz = dim == 3 ? width : 0;
        for (int dz = -wz; dz <= wz && !edge; ++dz)
          for (int dy = -width; dy <= width && !edge; ++dy)
            for (int dx = -width; dx <= width && !edge; ++dx) {
              const int32_t q[3] = {g[0] + dx, g[1] + dy, g[2] + dz};
              if (q[0] < 0 || q[0] >= nc[0] || q[1] < 0 || q[1] >= nc[1] || q[2] < 0 ||
                  q[2] >= nc[2]) {
                edge = true;
                break;
              }
              const int64_t nat = q[0] + (int64_t)nc[0] * (q[1] + (int64_t)nc[1] * q[2]);
              const int32_t qp = ipos[nat];
              if (qp < a || qp >= b) edge = true;
            }
        if (edge) out.push_back(p);
      }
    }
  });
  for (int64_t nd = 0; nd < nn; ++nd) band_off[nd + 1] = band_off[nd] + (int64_t)per[nd].size();
  band.resize(band_off[nn]);
  parallel_for(nn, [&](int64_t n0, int64_t n1) {
    for (int64_t nd = n0; nd < n1; ++nd)
      std::copy(per[nd].begin(), per[nd].end(), band.begin() + band_off[nd]);
  });
}

void proxy_rows(const Geometry &G, int64_t nd, const int32_t *cand, int ncand,
                const ProxyParams &pp, std::vector<int32_t> &out,
                std::vector<int32_t> &stamp, int32_t tag) {
  const int32_t a = G.nstart[nd], b = G.nend[nd];
  const int64_t size = b - a;
  out.clear();
  const int64_t nf = (int64_t)std::ceil(pp.chi * ncand);
  auto all_rows = [&]() {
    out.resize(size);
    for (int64_t i = 0; i < size; ++i) out[i] = a + (int32_t)i;
  };
  if (nf >= size || (pp.band && nd >= (int64_t)G.band_off.size() - 1)) { all_rows(); return; }
  auto add = [&](int32_t p) {
    if (stamp[p] != tag) { stamp[p] = tag; out.push_back(p); }
  };
  // f_tau: half over the boundary band, half over the whole node
  int64_t nb = 0;
  if (pp.band) {
    const int64_t b0 = G.band_off[nd], nb_all = G.band_off[nd + 1] - b0;
    nb = std::min<int64_t>(nb_all, (nf + 1) / 2);
    for (int64_t q = 0; q < nb; ++q) add(G.band[b0 + (q * nb_all) / nb]);
  }
  const int64_t nu = nf - nb;
  for (int64_t q = 0; q < nu; ++q) add(a + (int32_t)((q * size + size / 2) / nu));
  // nearest-neighbour rows: cells of the node within `radius` of a candidate
  const int R = (int)std::floor(pp.radius);
  const double R2 = pp.radius * pp.radius;
  const int32_t *lo = &G.bblo[nd * 3], *hi = &G.bbhi[nd * 3];
  for (int c = 0; c < ncand; ++c) {
    int32_t g[3];
    G.grid_coords(G.perm[cand[c]], g);
    double d2 = 0.0;
    for (int ax = 0; ax < G.dim; ++ax) {
      const int32_t dd = g[ax] < lo[ax] ? lo[ax] - g[ax] : (g[ax] > hi[ax] ? g[ax] - hi[ax] : 0);
      d2 += double(dd) * dd;
    }
    if (d2 > R2) continue;
    const int Rz = G.dim == 3 ? R : 0;
    for (int dz = -Rz; dz <= Rz; ++dz)
      for (int dy = -R; dy <= R; ++dy)
        for (int dx = -R; dx <= R; ++dx) {
          if (double(dx) * dx + double(dy) * dy + double(dz) * dz > R2) continue;
          const int32_t q[3] = {g[0] + dx, g[1] + dy, g[2] + dz};
          if (q[0] < lo[0] || q[0] > hi[0] || q[1] < lo[1] || q[1] > hi[1] ||
              q[2] < lo[2] || q[2] > hi[2])
            continue;
          const int64_t nat = q[0] + (int64_t)G.nc[0] * (q[1] + (int64_t)G.nc[1] * q[2]);
          const int32_t p = G.ipos[nat];
          if (p >= a && p < b) add(p);
        }
  }
  if ((int64_t)out.size() >= size) { all_rows(); return; }
  std::sort(out.begin(), out.end());
}

}  // namespace hbi
