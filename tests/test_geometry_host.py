"""The host geometry (csrc/hbi_geometry.cpp: K-D cluster tree, boundary
bands, proxy rows of eq. proxyv2v) compiled with g++ and checked against
brute force on small grids: the tree rule (median split along the longest
extent, ties to the lowest axis, lower half first), the node boxes, the
bands (cells within `width` cells, Chebyshev distance, of a cell outside the
node or the grid) and the proxy-row rule (every cell of the node within the
neighbour radius of a candidate, half of the uniform rows from the band)."""
import ctypes
import math
import os
import subprocess
import tempfile

import numpy as np
import pytest
from scipy import ndimage

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(os.path.dirname(HERE), "paper_2210_02698_amd", "csrc")

SHIM = r'''
#include "hbi_geometry.h"
using namespace hbi;
extern "C" {
void *geo_new(int dim, int nx, int ny, int nz, int leaf, int width) {
  Geometry *g = new Geometry;
  const int32_t nc[3] = {nx, ny, nz};
  g->build(dim, nc, leaf);
  g->build_bands(width);
  return g;
}
void geo_free(void *h) { delete (Geometry *)h; }
long long geo_nv(void *h) { return ((Geometry *)h)->Nv; }
int geo_lv(void *h) { return ((Geometry *)h)->Lv; }
void geo_perm(void *h, int32_t *perm, int32_t *ipos) {
  const Geometry &g = *(Geometry *)h;
  for (long long i = 0; i < g.Nv; ++i) { perm[i] = g.perm[i]; ipos[i] = g.ipos[i]; }
}
void geo_nodes(void *h, int32_t *s, int32_t *e, int32_t *lo, int32_t *hi) {
  const Geometry &g = *(Geometry *)h;
  for (size_t i = 0; i < g.nstart.size(); ++i) { s[i] = g.nstart[i]; e[i] = g.nend[i]; }
  for (size_t i = 0; i < g.bblo.size(); ++i) { lo[i] = g.bblo[i]; hi[i] = g.bbhi[i]; }
}
long long geo_band(void *h, long long nd, int32_t *out) {
  const Geometry &g = *(Geometry *)h;
  const long long a = g.band_off[nd], b = g.band_off[nd + 1];
  if (out) for (long long i = a; i < b; ++i) out[i - a] = g.band[i];
  return b - a;
}
int geo_proxy(void *h, long long nd, const int32_t *cand, int ncand, double chi,
              double radius, int32_t *out) {
  const Geometry &g = *(Geometry *)h;
  std::vector<int32_t> stamp(g.Nv, 0), rows;
  ProxyParams pp;
  pp.chi = chi;
  pp.radius = radius;
  proxy_rows(g, nd, cand, ncand, pp, rows, stamp, 1);
  for (size_t i = 0; i < rows.size(); ++i) out[i] = rows[i];
  return (int)rows.size();
}
}
'''

I32 = ctypes.POINTER(ctypes.c_int32)


@pytest.fixture(scope="module")
def geo_lib():
    d = tempfile.mkdtemp()
    shim, so = os.path.join(d, "shim.cpp"), os.path.join(d, "geo.so")
    open(shim, "w").write(SHIM)
    subprocess.check_call(["g++", "-O2", "-std=c++17", "-shared", "-fPIC", "-pthread", "-I", CSRC,
                           shim, os.path.join(CSRC, "hbi_geometry.cpp"), "-o", so])
    lib = ctypes.CDLL(so)
    lib.geo_new.restype = ctypes.c_void_p
    lib.geo_new.argtypes = [ctypes.c_int] * 6
    for f in ("geo_free", "geo_nv", "geo_lv", "geo_perm", "geo_nodes", "geo_band", "geo_proxy"):
        getattr(lib, f).argtypes = None
    lib.geo_free.argtypes = [ctypes.c_void_p]
    lib.geo_nv.argtypes = [ctypes.c_void_p]
    lib.geo_nv.restype = ctypes.c_longlong
    lib.geo_lv.argtypes = [ctypes.c_void_p]
    lib.geo_perm.argtypes = [ctypes.c_void_p, I32, I32]
    lib.geo_nodes.argtypes = [ctypes.c_void_p, I32, I32, I32, I32]
    lib.geo_band.argtypes = [ctypes.c_void_p, ctypes.c_longlong, I32]
    lib.geo_band.restype = ctypes.c_longlong
    lib.geo_proxy.argtypes = [ctypes.c_void_p, ctypes.c_longlong, I32, ctypes.c_int,
                              ctypes.c_double, ctypes.c_double, I32]
    return lib


def ptr(a):
    return a.ctypes.data_as(I32)


class Geo:
    """The library's geometry for one grid, read back into numpy."""

    def __init__(self, lib, dim, nc, leaf, width):
        self.lib, self.dim = lib, dim
        self.nc = tuple(nc) + (1,) * (3 - len(nc))
        self.h = lib.geo_new(dim, *self.nc, leaf, width)
        self.Nv, self.Lv = lib.geo_nv(self.h), lib.geo_lv(self.h)
        self.perm = np.empty(self.Nv, np.int32)
        self.ipos = np.empty(self.Nv, np.int32)
        lib.geo_perm(self.h, ptr(self.perm), ptr(self.ipos))
        nn = (2 << self.Lv) - 1
        self.s, self.e = np.empty(nn, np.int32), np.empty(nn, np.int32)
        self.lo, self.hi = np.empty(3 * nn, np.int32), np.empty(3 * nn, np.int32)
        lib.geo_nodes(self.h, ptr(self.s), ptr(self.e), ptr(self.lo), ptr(self.hi))
        nat = np.arange(self.Nv)
        self.coords = np.stack([nat % self.nc[0], (nat // self.nc[0]) % self.nc[1],
                                nat // (self.nc[0] * self.nc[1])], axis=1)

    def cells(self, nd):
        """Grid coordinates of node nd's cells, in tree order."""
        return self.coords[self.perm[self.s[nd]:self.e[nd]]]

    def band(self, nd):
        n = self.lib.geo_band(self.h, nd, None)
        out = np.empty(max(n, 1), np.int32)
        self.lib.geo_band(self.h, nd, ptr(out))
        return out[:n]

    def proxy(self, nd, cand, chi, radius):
        out = np.empty(self.e[nd] - self.s[nd] + 1, np.int32)
        cand = np.ascontiguousarray(cand, np.int32)
        n = self.lib.geo_proxy(self.h, nd, ptr(cand), len(cand), chi, radius, ptr(out))
        return out[:n]

    def close(self):
        self.lib.geo_free(self.h)


GRIDS = [(2, (37, 29), 64), (2, (64, 64), 64), (2, (5, 7), 64), (2, (64, 1), 8),
         (2, (24, 40), 8), (3, (9, 7, 5), 16), (3, (16, 16, 16), 64)]


@pytest.mark.parametrize("dim,nc,leaf", GRIDS)
def test_tree_rule(geo_lib, dim, nc, leaf):
    g = Geo(geo_lib, dim, nc, leaf, 2)
    assert g.Nv == math.prod(nc)
    assert np.array_equal(np.sort(g.perm), np.arange(g.Nv))
    assert np.array_equal(g.ipos[g.perm], np.arange(g.Nv))
    # fewest levels whose leaves hold at most `leaf` cells
    L = 0
    while math.ceil(g.Nv / 2 ** L) > leaf:
        L += 1
    assert g.Lv == L
    assert g.s[0] == 0 and g.e[0] == g.Nv
    for l in range(g.Lv + 1):
        for i in range(2 ** l):
            nd = 2 ** l - 1 + i
            c = g.cells(nd)
            n = len(c)
            assert n in (g.Nv // 2 ** l, -(-g.Nv // 2 ** l))   # complete tree
            assert np.array_equal(g.lo[3 * nd:3 * nd + 3], c.min(axis=0))
            assert np.array_equal(g.hi[3 * nd:3 * nd + 3], c.max(axis=0))
            if l == g.Lv:
                assert n <= leaf
                continue
            c0, c1 = 2 ** (l + 1) - 1 + 2 * i, 2 ** (l + 1) + 2 * i
            assert g.s[c0] == g.s[nd] and g.e[c0] == g.s[c1] and g.e[c1] == g.e[nd]
            assert g.e[c0] - g.s[c0] == n // 2          # lower half first
            ext = (c.max(axis=0) - c.min(axis=0))[:dim]
            ax = int(np.argmax(ext))                     # first maximum: lowest axis
            assert g.cells(c0)[:, ax].max() <= g.cells(c1)[:, ax].min()
    g.close()


@pytest.mark.parametrize("dim,nc,leaf", GRIDS[:3] + GRIDS[5:6])
@pytest.mark.parametrize("width", [1, 2])
def test_boundary_bands(geo_lib, dim, nc, leaf, width):
    g = Geo(geo_lib, dim, nc, leaf, width)
    shape = tuple(reversed(g.nc[:dim]))                  # numpy order (z,) y, x
    for nd in range(2 ** g.Lv - 1):                      # nodes above the leaves
        mask = np.zeros(shape, bool)
        c = g.cells(nd)
        mask[tuple(c[:, a] for a in reversed(range(dim)))] = True
        # a cell is inside the band when its (2 width + 1)^dim window reaches
        # a cell outside the node or outside the grid (padding counts as out)
        inner = ndimage.minimum_filter(np.pad(mask, width, constant_values=False),
                                       size=2 * width + 1, mode="constant", cval=False)
        inner = inner[tuple(slice(width, -width) for _ in range(dim))]
        want = np.sort(g.ipos[[x + g.nc[0] * (y + g.nc[1] * z)
                               for x, y, z in g.coords[g.perm[g.s[nd]:g.e[nd]]]
                               if not inner[(z, y, x)[3 - dim:]]]])
        assert np.array_equal(np.sort(g.band(nd)), want), nd
    g.close()


@pytest.mark.parametrize("dim,nc,leaf,radius", [(2, (64, 64), 64, 10.0), (2, (37, 29), 64, 3.5),
                                                (3, (16, 16, 16), 64, 3.0)])
def test_proxy_rows(geo_lib, dim, nc, leaf, radius):
    g = Geo(geo_lib, dim, nc, leaf, 2)
    rng = np.random.default_rng(7)
    for l in range(1, g.Lv + 1):
        for i in range(0, 2 ** l, max(1, 2 ** l // 4)):
            nd, sib = 2 ** l - 1 + i, 2 ** l - 1 + (i ^ 1)
            # candidate columns: a few cells of the sibling node
            pool = np.arange(g.s[sib], g.e[sib])
            for ncand in (1, 3, 12):
                cand = rng.choice(pool, size=min(ncand, len(pool)), replace=False)
                for chi in (0.5, 4.0, 20.0):
                    rows = g.proxy(nd, cand, chi, radius)
                    a, b = g.s[nd], g.e[nd]
                    size = b - a
                    assert np.all(np.diff(rows) > 0) and rows[0] >= a and rows[-1] < b
                    nf = math.ceil(chi * len(cand))
                    if nf >= size or l == g.Lv:
                        assert len(rows) == size            # all rows of the node
                        continue
                    # every cell of the node within the radius of a candidate
                    cc = g.coords[g.perm[np.arange(a, b)]][:, :dim].astype(float)
                    gc = g.coords[g.perm[cand]][:, :dim].astype(float)
                    d2 = ((cc[:, None, :] - gc[None, :, :]) ** 2).sum(-1).min(axis=1)
                    near = np.arange(a, b)[d2 <= radius * radius]
                    assert np.all(np.isin(near, rows))
                    if len(rows) == size:
                        continue                            # fell back to all rows
                    band = g.band(nd)
                    assert np.isin(rows, band).sum() >= min(len(band), (nf + 1) // 2)
                    assert len(rows) <= nf + len(near)
    g.close()
