// Layout of the work lists of the persistent projection launch (k_schedule / k_schedule_packed
// write them, the persistent k_windows_cl reads them).  Plain C++ (no HIP) so that a host test can
// check the arithmetic for every batch size; constexpr functions are usable in device code as well.
//
// For XCD x (0..7) the list holds offs[x][i] = sum of the multipole counts of the XCD's points
// before position i, for i = 0..nx with nx = ceil((batch - x) / 8) (nx + 1 entries, the last the
// list's total); the eight totals follow the eight lists.  Plain persistent mode: position i is
// point 8 i + x.  Packed mode: the XCD's points in descending order of tracer count, pts[x][i]
// naming the point at position i, so that the (point, multipole) items of each tracer count form
// one contiguous range of the XCD's item stream; the segments then pair items whose tracer counts
// sum to at most 16 into one workgroup (rows 0..T_a - 1 for the first, T_a.. for the second).
#pragma once

#include <stddef.h>

// largest tracer count a workgroup of the fused projection holds (rows of its Gram tile)
constexpr int SCHED_ROWS = 16;
// segments of one XCD's packed list: at most 43 for 17 tracer counts (sched_pack)
constexpr int SCHED_MAXSEG = 48;
// ints of one XCD's segment record: nseg, then (first packed item, first a item, first b item or
// -1) per segment
constexpr int SCHED_SEG_INTS = 1 + 3 * SCHED_MAXSEG;

// row stride of one XCD's list: room for nx + 1 <= max_batch / 8 + 2 entries
constexpr int sched_stride_for(int max_batch) { return max_batch / 8 + 2; }
// ints to allocate: eight lists, eight totals, eight point orders, eight segment records, eight
// task counters (packed mode: the blocks of an XCD take their next task from its counter)
constexpr size_t sched_ints(int stride) { return (size_t)16 * stride + 8 + (size_t)8 * SCHED_SEG_INTS + 8; }
constexpr size_t sched_list_index(int stride, int x, int i) { return (size_t)x * stride + i; }
constexpr size_t sched_total_index(int stride, int x) { return (size_t)8 * stride + x; }
constexpr size_t sched_pts_index(int stride, int x, int i) { return (size_t)8 * stride + 8 + (size_t)x * stride + i; }
constexpr size_t sched_seg_index(int stride, int x, int j) {
  return (size_t)16 * stride + 8 + (size_t)x * SCHED_SEG_INTS + j;
}
constexpr size_t sched_ctr_index(int stride, int x) { return (size_t)16 * stride + 8 + (size_t)8 * SCHED_SEG_INTS + x; }
// largest point count per XCD the packed builder stages in LDS (larger batches run mode 1)
constexpr int SCHED_PACK_MAXNX = 2048;

// Greedy pairing of one XCD's items by tracer count.  rem[c] (c = 0..16): the number of items
// with c tracers, cur[c]: the stream index of the first of them (both updated in place).  Tracer
// counts are taken largest first; each is paired with items of the largest count c' <= min(c, 16 - c)
// that has items left (two of c itself when c' = c), and what finds no partner runs alone.  Writes
// seg[0] = the segment count and seg[1 + 3 s ..] = (first packed item, first a item, first b item
// or -1) of segment s; returns the number of packed items (workgroup tasks).  Every step that does
// not end count c's turn exhausts a partner count for good, or halves count c's own items once, so
// the segments number at most 17 + 17 + 9 = 43.
constexpr int sched_pack(int* rem, int* cur, int* seg) {
  int nseg = 0, k = 0;
  for (int c = SCHED_ROWS; c >= 0; --c) {
    while (rem[c] > 0) {
      int p = -1;
      for (int q = (c < SCHED_ROWS - c ? c : SCHED_ROWS - c); q >= 0; --q)
        if (rem[q] > (q == c ? 1 : 0)) { p = q; break; }
      int m = rem[c], qa = cur[c], qb = -1;
      if (p == c) {
        m = rem[c] / 2;
        qb = cur[c] + m;
        cur[c] += 2 * m;
        rem[c] -= 2 * m;
      } else if (p >= 0) {
        m = rem[c] < rem[p] ? rem[c] : rem[p];
        qb = cur[p];
        cur[c] += m;
        rem[c] -= m;
        cur[p] += m;
        rem[p] -= m;
      } else {
        cur[c] += m;
        rem[c] = 0;
      }
      if (nseg < SCHED_MAXSEG) {
        seg[1 + 3 * nseg] = k;
        seg[2 + 3 * nseg] = qa;
        seg[3 + 3 * nseg] = qb;
      }
      ++nseg;
      k += m;
    }
  }
  seg[0] = nseg;
  return k;
}
