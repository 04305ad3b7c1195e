"""The workgroup -> (output block, time tile) maps of tile_order.h are bijections.

Every kernel launches one workgroup per (output block, time tile) pair and
finds its pair through tile_of(); a pair produced twice or never would be
computed twice or left unwritten.  The header is compiled for the host with
g++ and checked for every order on all grids up to 24 x 40 (tails in both
dimensions against the 8 XCDs and the groups of 4 output blocks) and on the
workloads' own grid sizes.
"""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

HARNESS = r"""
#define __device__
#define __forceinline__ inline
#include "tile_order.h"
#include <cstdio>
#include <vector>
static int check(int n_oblk, int n_tiles, int order) {
  std::vector<int> seen((size_t)n_oblk * n_tiles, 0);
  for (int w = 0; w < n_oblk * n_tiles; ++w) {
    int o = -1, t = -1;
    dd::tile_of(w, n_oblk, n_tiles, order, o, t);
    if (o < 0 || o >= n_oblk || t < 0 || t >= n_tiles) return 1;
    if (seen[(size_t)o * n_tiles + t]++) return 1;
  }
  return 0;
}
int main() {
  const int big[][2] = {{125, 993}, {16, 993}, {64, 1024}, {32, 407}, {4, 2}, {1, 1}, {250, 1985}};
  int bad = 0;
  for (int order = 0; order < 4; ++order) {
    for (int a = 1; a <= 24; ++a)
      for (int b = 1; b <= 40; ++b)
        if (check(a, b, order)) { printf("order %d grid %d x %d\n", order, a, b); ++bad; }
    for (auto &g : big)
      if (check(g[0], g[1], order)) { printf("order %d grid %d x %d\n", order, g[0], g[1]); ++bad; }
  }
  if (!bad) printf("ok\n");
  return bad ? 1 : 0;
}
"""


def test_tile_orders_are_bijections(tmp_path):
    src = tmp_path / "tile_order_check.cpp"
    src.write_text(HARNESS)
    exe = tmp_path / "tile_order_check"
    subprocess.run(["g++", "-O2", "-std=c++17", "-I", os.path.join(ROOT, "paper_2311_05341_amd", "csrc"), str(src),
                    "-o", str(exe)], check=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0 and r.stdout.strip() == "ok", r.stdout
