// Layout of the work lists of the persistent projection launch (k_schedule writes them, the
// persistent k_windows_cl reads them).  Plain C++ (no HIP) so that a host test can check the
// arithmetic for every batch size; constexpr functions are usable in device code as well.
//
// For XCD x (0..7) the list holds offs[x][i] = sum of the multipole counts of points 8 j + x, j < i,
// for i = 0..nx with nx = ceil((batch - x) / 8) (nx + 1 entries, the last the list's total); the
// eight totals follow the eight lists.
#pragma once

#include <stddef.h>

// row stride of one XCD's list: room for nx + 1 <= max_batch / 8 + 2 entries
constexpr int sched_stride_for(int max_batch) { return max_batch / 8 + 2; }
// ints to allocate: eight lists, then eight totals
constexpr size_t sched_ints(int stride) { return (size_t)8 * stride + 8; }
constexpr size_t sched_list_index(int stride, int x, int i) { return (size_t)x * stride + i; }
constexpr size_t sched_total_index(int stride, int x) { return (size_t)8 * stride + x; }
