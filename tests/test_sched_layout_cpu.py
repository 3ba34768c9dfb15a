"""The work-list layout of the persistent projection launch (csrc/sched_layout.h), checked on the
host: for every capacity max_batch and every batch size up to it, each index the list builder
writes (the per-XCD prefix offsets and the eight totals) and each index the persistent kernel
reads lies inside the allocation, and no two writes share an index.  The packed lists: on random
and adversarial tracer / multipole counts, the pairing (sched_pack) places every (point,
multipole) item in exactly one task, never more than 16 tracer rows in a task, at most 43
segments, and the per-XCD regions stay inside the allocation without overlapping."""
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


PACKED = r"""
#include "sched_layout.h"
#include <stdio.h>
#include <stdlib.h>
#include <vector>
// the device builder's steps on the host: counting sort by descending tracer count, prefix
// offsets over that order, sched_pack; then every task decoded as the persistent kernel does
static int check(int batch, int Lm, const std::vector<int>& ntr, const std::vector<int>& nell, int* maxseg) {
  const int NXCD = 8, NC = SCHED_ROWS + 1;
  const int st = sched_stride_for(batch);
  const size_t n = sched_ints(st);
  std::vector<int> sched(n, -7), hits(n, 0);
  for (int x = 0; x < NXCD; ++x) {
    int cnt[NC] = {0}, rem[NC] = {0}, cur[NC] = {0};
    for (int b = x; b < batch; b += NXCD) { ++cnt[ntr[b]]; rem[ntr[b]] += nell[b]; }
    int pos = 0, items = 0;
    for (int c = SCHED_ROWS; c >= 0; --c) { const int k = cnt[c]; cnt[c] = pos; cur[c] = items; pos += k; items += rem[c]; }
    for (int b = x; b < batch; b += NXCD) {  // place the point; its first item is cur[count]
      const int c = ntr[b], at = cnt[c]++;
      hits[sched_pts_index(st, x, at)]++;
      sched[sched_pts_index(st, x, at)] = b;
      hits[sched_list_index(st, x, at)]++;
      sched[sched_list_index(st, x, at)] = cur[c];
      cur[c] += nell[b];
    }
    hits[sched_list_index(st, x, pos)]++;
    sched[sched_list_index(st, x, pos)] = items;
    for (int c = SCHED_ROWS, at = 0; c >= 0; --c) { cur[c] = at; at += rem[c]; }
    // the offsets are the prefix sums of the multipole counts in the new order
    for (int i = 0, acc = 0; i <= pos; ++i) {
      if (sched[sched_list_index(st, x, i)] != acc) { printf("offs[%d] is not a prefix sum\n", i); return 1; }
      if (i < pos) acc += nell[sched[sched_pts_index(st, x, i)]];
    }
    for (int j = 0; j < SCHED_SEG_INTS; ++j) hits[sched_seg_index(st, x, j)]++;
    hits[sched_ctr_index(st, x)]++;
    int* seg = &sched[sched_seg_index(st, x, 0)];
    const int total = sched_pack(rem, cur, seg);
    hits[sched_total_index(st, x)]++;
    if (seg[0] > *maxseg) *maxseg = seg[0];
    if (seg[0] > 43) { printf("%d segments\n", seg[0]); return 1; }
    // decode every task
    std::vector<int> seen(items, 0);
    const int* offs = &sched[sched_list_index(st, x, 0)];
    auto locate = [&](int q) { int i = 0, hi = pos; while (hi - i > 1) { int mid = (i + hi) / 2; if (offs[mid] <= q) i = mid; else hi = mid; } return i; };
    int sg = 0;
    for (int k = 0; k < total; ++k) {
      while (sg + 1 < seg[0] && seg[1 + 3 * (sg + 1)] <= k) ++sg;
      const int d = k - seg[1 + 3 * sg];
      const int qa = seg[2 + 3 * sg] + d, qb = seg[3 + 3 * sg] < 0 ? -1 : seg[3 + 3 * sg] + d;
      if (qa < 0 || qa >= items || qb >= items) { printf("stream index out of range\n"); return 1; }
      const int ia = locate(qa), ba = sched[sched_pts_index(st, x, ia)], la = qa - offs[ia];
      if (ba % NXCD != x || la < 0 || la >= nell[ba]) { printf("bad item a\n"); return 1; }
      seen[qa]++;
      if (qb >= 0) {
        const int ib = locate(qb), bb = sched[sched_pts_index(st, x, ib)], lb = qb - offs[ib];
        if (bb % NXCD != x || lb < 0 || lb >= nell[bb]) { printf("bad item b\n"); return 1; }
        if (ntr[ba] + ntr[bb] > SCHED_ROWS) { printf("task of %d + %d rows\n", ntr[ba], ntr[bb]); return 1; }
        seen[qb]++;
      }
    }
    for (int q = 0; q < items; ++q)
      if (seen[q] != 1) { printf("item %d seen %d times (x %d)\n", q, seen[q], x); return 1; }
  }
  for (size_t k = 0; k < n; ++k)
    if (hits[k] > 1) { printf("two writes at %zu\n", k); return 1; }
  if (sched_ctr_index(st, 7) != n - 1) { printf("counters not at the end\n"); return 1; }
  return 0;
}
int main() {
  srand(12345);
  int maxseg = 0;
  for (int trial = 0; trial < 3000; ++trial) {
    const int batch = 1 + rand() % 300, Lm = 1 + rand() % 120;
    std::vector<int> ntr(batch), nell(batch);
    const int mode = trial % 4;
    for (int b = 0; b < batch; ++b) {
      // uniform counts; a 6/10/15 mix; one count per point index; many distinct small counts
      ntr[b] = mode == 0 ? rand() % 17 : mode == 1 ? (int[]){6, 10, 15}[rand() % 3] : mode == 2 ? b % 17 : 1 + rand() % 8;
      nell[b] = (trial % 7 == 0 && rand() % 5 == 0) ? 0 : rand() % (Lm + 1);
    }
    if (check(batch, Lm, ntr, nell, &maxseg)) { printf("trial %d batch %d\n", trial, batch); return 1; }
  }
  printf("ok %d\n", maxseg);
  return 0;
}
"""


def test_packed_lists_cover_every_item_once(tmp_path):
    if shutil.which("g++") is None:
        pytest.skip("no g++")
    src = tmp_path / "packed.cpp"
    src.write_text(PACKED)
    exe = tmp_path / "packed"
    subprocess.run(["g++", "-std=c++17", "-O1", "-Wall", "-Werror", "-I", CSRC, str(src), "-o", str(exe)], check=True)
    res = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    assert res.returncode == 0 and res.stdout.startswith("ok"), res.stdout


def test_schedule_indices_stay_inside_the_allocation(tmp_path):
    if shutil.which("g++") is None:
        pytest.skip("no g++")
    src = tmp_path / "sched.cpp"
    src.write_text(PROGRAM)
    exe = tmp_path / "sched"
    subprocess.run(["g++", "-std=c++17", "-Wall", "-Werror", "-I", CSRC, str(src), "-o", str(exe)], check=True)
    res = subprocess.run([str(exe)], capture_output=True, text=True)
    assert res.returncode == 0 and res.stdout.strip() == "ok", res.stdout
