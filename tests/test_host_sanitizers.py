"""The host C++ of the library (csrc/hbi_geometry.cpp: cluster tree, bands,
proxy rows, the thread pool) built with AddressSanitizer and
UndefinedBehaviorSanitizer by g++ into a standalone driver and run as its own
process on 2D and 3D grids, ragged and degenerate ones included: every node
of every level gets its band and, with candidates drawn from a sibling, its
proxy rows.  Any sanitizer report fails the test (halt_on_error)."""
import os
import shutil
import subprocess
import tempfile

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(os.path.dirname(HERE), "paper_2210_02698_amd", "csrc")

DRIVER = r'''
#include <cstdio>
#include <cstdlib>
#include <vector>
#include "hbi_geometry.h"
using namespace hbi;

static int run(int dim, int nx, int ny, int nz, int leaf, int width, double chi, double rad) {
  Geometry g;
  const int32_t nc[3] = {nx, ny, nz};
  g.build(dim, nc, leaf);
  g.build_bands(width);
  std::vector<int32_t> stamp(g.Nv, 0), rows;
  int32_t tag = 0;
  long long total = 0;
  for (int l = 1; l <= g.Lv; ++l) {
    for (int64_t i = 0; i < ((int64_t)1 << l); ++i) {
      const int64_t nd = Geometry::node(l, i), sib = Geometry::node(l, i ^ 1);
      std::vector<int32_t> cand;
      const int32_t step = (g.nend[sib] - g.nstart[sib]) / 3 > 0 ? (g.nend[sib] - g.nstart[sib]) / 3 : 1;
      for (int32_t p = g.nstart[sib]; p < g.nend[sib]; p += step) cand.push_back(p);
      proxy_rows(g, nd, cand.data(), (int)cand.size(), ProxyParams{chi, rad}, rows, stamp, ++tag);
      for (int32_t r : rows)
        if (r < g.nstart[nd] || r >= g.nend[nd]) { std::printf("row outside node\n"); return 1; }
      total += (long long)rows.size();
    }
  }
  // the thread pool over an uneven range
  std::vector<int> hit(1000003, 0);
  parallel_for((int64_t)hit.size(), [&](int64_t a, int64_t b) {
    for (int64_t q = a; q < b; ++q) hit[q] += 1;
  });
  for (int h : hit)
    if (h != 1) { std::printf("parallel_for covered an index %d times\n", h); return 1; }
  std::printf("dim %d %dx%dx%d leaf %d: Nv %lld Lv %d proxy rows %lld\n", dim, nx, ny, nz, leaf,
              (long long)g.Nv, g.Lv, total);
  return 0;
}

int main() {
  int bad = 0;
  bad |= run(2, 64, 64, 1, 64, 2, 20.0, 10.0);
  bad |= run(2, 37, 29, 1, 64, 2, 20.0, 10.0);
  bad |= run(2, 5, 7, 1, 64, 2, 20.0, 10.0);
  bad |= run(2, 200, 1, 1, 64, 2, 20.0, 10.0);
  bad |= run(2, 96, 80, 1, 16, 3, 4.0, 2.5);
  bad |= run(2, 256, 256, 1, 64, 2, 2.0, 3.0);
  bad |= run(3, 16, 16, 16, 64, 2, 4.0, 3.0);
  bad |= run(3, 9, 13, 7, 64, 2, 4.0, 3.0);
  return bad;
}
'''


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not available")
def test_geometry_under_address_and_ub_sanitizers():
    d = tempfile.mkdtemp()
    src, exe = os.path.join(d, "driver.cpp"), os.path.join(d, "driver")
    open(src, "w").write(DRIVER)
    subprocess.check_call(["g++", "-O1", "-g", "-std=c++17", "-pthread",
                           "-fsanitize=address,undefined", "-fno-omit-frame-pointer",
                           "-I", CSRC, src, os.path.join(CSRC, "hbi_geometry.cpp"), "-o", exe])
    env = dict(os.environ, ASAN_OPTIONS="halt_on_error=1:detect_leaks=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    env.pop("LD_PRELOAD", None)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=600, env=env)
    print(r.stdout)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr
