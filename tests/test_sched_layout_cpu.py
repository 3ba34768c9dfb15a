"""The work-list layout of the persistent projection launch (csrc/sched_layout.h), checked on the
host: for every capacity max_batch and every batch size up to it, each index the list builder
writes (the per-XCD prefix offsets and the eight totals) and each index the persistent kernel
reads lies inside the allocation, and no two writes share an index."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2505_22718_amd", "csrc")

PROGRAM = r"""
#include "sched_layout.h"
#include <stdio.h>
#include <vector>
int main() {
  const int NXCD = 8;
  for (int maxb = 1; maxb <= 200; ++maxb) {
    const int stride = sched_stride_for(maxb);
    const size_t n = sched_ints(stride);
    for (int batch = 1; batch <= maxb; ++batch) {
      std::vector<int> hits(n, 0);
      for (int x = 0; x < NXCD; ++x) {
        // the builder: offs[i] for i = 0..nx (nx points of this XCD), then the total
        int i = 0;
        for (int b = x; b < batch; b += NXCD, ++i) {
          const size_t at = sched_list_index(stride, x, i);
          if (at >= n) { printf("list write past the end: maxb %d batch %d x %d i %d\n", maxb, batch, x, i); return 1; }
          hits[at]++;
        }
        const size_t last = sched_list_index(stride, x, i);
        if (last >= n || i >= stride) { printf("list end past its row: maxb %d batch %d x %d\n", maxb, batch, x); return 1; }
        hits[last]++;
        const size_t tot = sched_total_index(stride, x);
        if (tot >= n) { printf("total past the end: maxb %d batch %d x %d\n", maxb, batch, x); return 1; }
        hits[tot]++;
        // the reader: a binary search over offs[0..nx], nx = ceil((batch - x) / 8)
        const int nx = (batch - x + NXCD - 1) / NXCD;
        if (nx > 0 && sched_list_index(stride, x, nx) >= n) { printf("read past the end\n"); return 1; }
      }
      for (size_t k = 0; k < n; ++k)
        if (hits[k] > 1) { printf("two writes at %zu: maxb %d batch %d\n", k, maxb, batch); return 1; }
    }
  }
  printf("ok\n");
  return 0;
}
"""


def test_schedule_indices_stay_inside_the_allocation(tmp_path):
    if shutil.which("g++") is None:
        pytest.skip("no g++")
    src = tmp_path / "sched.cpp"
    src.write_text(PROGRAM)
    exe = tmp_path / "sched"
    subprocess.run(["g++", "-std=c++17", "-Wall", "-Werror", "-I", CSRC, str(src), "-o", str(exe)], check=True)
    res = subprocess.run([str(exe)], capture_output=True, text=True)
    assert res.returncode == 0 and res.stdout.strip() == "ok", res.stdout
