"""Host-side logic that needs no GPU: the W-cycle stage structure of the
multi-level driver and the bench's lookup of committed counter profiles."""

import json
import os

import pytest

torch = pytest.importorskip("torch")

from paper_1712_07070_amd import hydro  # noqa: E402

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _driver(n_levels):
    ml = object.__new__(hydro.MultiLevel)   # the stage logic only reads the level count
    ml.L = n_levels
    return ml


@pytest.mark.parametrize("n_levels", [1, 2, 3, 4])
def test_wcycle_stage_membership(n_levels):
    """Over the 2^(L-1) stages of a coarse step level l advances 2^l times
    (dt_l = dt_0 / 2^l), every stage advances the finest level, and a level
    that advances in a stage also advances every finer level there."""
    ml = _driver(n_levels)
    stages = [ml.stage_levels(s) for s in range(2 ** (n_levels - 1))]
    for l in range(n_levels):
        assert sum(l in st for st in stages) == 2 ** l
    for st in stages:
        assert n_levels - 1 in st
        assert st == list(range(st[0], n_levels))
    assert stages[0] == list(range(n_levels))


def test_wcycle_three_levels_exact():
    assert [_driver(3).stage_levels(s) for s in range(4)] == [[0, 1, 2], [2], [1, 2], [2]]


def test_measured_profile_guards(monkeypatch):
    import bench
    with open(os.path.join(ROOT, "profiles", "traffic.json")) as fh:
        rec = json.load(fh)
    key = next(iter(rec))
    variants = rec[key]["by_variant"]
    v = next(iter(variants))
    # a record is used only for the sources it was measured on
    monkeypatch.setattr(bench, "kernel_source_sha", lambda: rec[key]["source_sha256"])
    assert bench.measured_traffic(key, v) == variants[v]["bytes_per_launch"]
    assert bench.measured_profile(key, 99, "bytes_per_launch") is None
    assert bench.measured_profile("no such kernel", v, "bytes_per_launch") is None
    monkeypatch.setattr(bench, "kernel_source_sha", lambda: "0" * 64)
    assert bench.measured_traffic(key, v) is None


# The level kernel maps workgroups to groups with index arithmetic that runs
# only on the device; a mapping that left a group out, or named one twice or
# outside the level, would write wrong cells (or outside the buffers).  The
# functions are taken from the kernel header as written and compiled for the
# host.
_GROUP_ORDER_CHECK = r"""
#include <cstdint>
#include <cstdio>
#include <vector>
struct LevelGeom { int ngx, ngy, ngz; };
%s
int main() {
  long bad = 0, cases = 0;
  for (int nx = 1; nx <= 40; ++nx) for (int ny = 1; ny <= 24; ++ny) for (int nz = 1; nz <= 9; ++nz) {
    const LevelGeom g{nx, ny, nz};
    const int64_t G = int64_t(nx) * ny * nz;
    if (tile_slots(g) != G) { ++bad; continue; }
    for (int gpw = 1; gpw <= 2; ++gpw)
      for (int order = 0; order < 4; ++order) {
        std::vector<int> seen(G, 0);
        const int64_t wslots = (G + gpw - 1) / gpw;
        const int64_t blocks = (order & 1) ? ((wslots + 7) / 8) * 8 : wslots;   // as the launcher sizes it
        for (int64_t b = 0; b < blocks; ++b) {
          const int64_t w = (order & 1) ? xcd_group(b, wslots) : b;
          if (w >= wslots) continue;
          for (int h = 0; h < gpw; ++h) {
            const int64_t sl = w * gpw + h;
            if (sl >= G) continue;
            const int64_t q = (order & 2) ? tile_group(sl, g) : sl;
            if (q < 0 || q >= G) { ++bad; continue; }
            seen[q]++;
          }
        }
        for (int64_t i = 0; i < G; ++i) bad += seen[i] != 1;
        ++cases;
      }
  }
  printf("%%ld %%ld\n", cases, bad);
  return bad != 0;
}
"""


def _device_functions(path, names):
    """The text of the named __device__ functions (and the constants before
    them) of a header, made host functions."""
    import re
    src = open(path).read()
    out = []
    for m in re.finditer(r"constexpr int kTileGroups = \d+;", src):
        out.append(m.group(0))
    for n in names:
        i = src.index("__device__ __forceinline__ int64_t %s(" % n)
        depth, j = 0, src.index("{", i)
        while True:
            depth += {"{": 1, "}": -1}.get(src[j], 0)
            j += 1
            if depth == 0:
                break
        out.append(src[i:j].replace("__device__ __forceinline__", "inline"))
    return "\n".join(out)


def test_level_group_orders_cover_every_group_once(tmp_path):
    """Plain, XCD-blocked, linear and column-tile orders, one and two groups
    per workgroup: every group of every lattice up to 40 x 24 x 9 is taken by
    exactly one workgroup slot."""
    import shutil
    import subprocess
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("no host C++ compiler")
    body = _device_functions(os.path.join(ROOT, "paper_1712_07070_amd", "csrc", "mhm_level.h"),
                             ["xcd_group", "tile_slots", "tile_group"])
    cpp = tmp_path / "orders.cpp"
    cpp.write_text(_GROUP_ORDER_CHECK % body)
    exe = tmp_path / "orders"
    subprocess.run([gxx, "-O2", "-std=c++17", str(cpp), "-o", str(exe)], check=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True)
    cases, bad = (int(v) for v in r.stdout.split())
    assert r.returncode == 0 and bad == 0 and cases == 40 * 24 * 9 * 8
