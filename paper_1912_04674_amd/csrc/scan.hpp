// scan.hpp -- the counting sort's scans (device side): per tile, the
// exclusive scan of its cells' counts into the per-cell cursors (work groups
// of the field-stage kernel); over all tiles, the exclusive scan of the tile
// totals into the next layout's offsets and work items (one work group,
// launched after it).
#pragma once
#include "common.hpp"

namespace envpic {

// Tile t's 16 x 16 cells (column-major, radius fastest) by 256 consecutive
// threads of the block (lt = 0..255, s: their 256 LDS ints): exclusive scan
// of the counts into the per-cell cursors, the total into hist[t], counts
// cleared.  Every thread of the block calls it (it synchronizes the block);
// inactive halves pass t < 0.
__device__ inline void cell_scan_tile(const Geo& g, int t, int lt, int* ccount, int* ccur, int* hist, int* s) {
  const bool active = t >= 0 && t < g.ntiles;
  int c = 0;
  size_t o = 0;
  bool valid = false;
  if (active) {
    const int tcx = t / g.ntr, tcr = t - (t / g.ntr) * g.ntr;
    const int a = lt / TR, b = lt - (lt / TR) * TR;
    const long long col = (long long)lab_tile(g, tcx) * TX + a;
    const int rel = (int)(col - g.shift), j = tcr * TR + b;
    valid = rel >= 0 && rel < g.nx && j < g.nr;
    o = valid ? (size_t)phys_col(g, rel) * g.pitch + j : 0;
    c = valid ? ccount[o] : 0;
  }
  s[lt] = c;
  __syncthreads();
  for (int off = 1; off < TX * TR; off <<= 1) {
    const int v = lt >= off ? s[lt - off] : 0;
    __syncthreads();
    s[lt] += v;
    __syncthreads();
  }
  if (valid) {
    ccur[o] = s[lt] - c;
    ccount[o] = 0;
  }
  if (active && lt == TX * TR - 1) hist[t] = s[lt];
}

// One block of NT threads: the items (pending[0]) and slots (pending[1]) of
// a column injected since the last scan are added to the layout in use
// (*bump_items, *bump_fill); with sort set, the tile totals in hist become
// the offsets, cursors and work items of layout `out` (a tile of v
// particles gives ceil(v / chunk) items of equal size) and hist is cleared.
// Flags when the particles plus the columns injected before the next sort
// would not fit.
template <int NT>
__device__ inline void layout_scan(const Geo& g, int* hist, Layout out, long long capacity, int inj_max, int max_items,
                                   int* bump_items, int* bump_fill, int* pending, int* err, int sort, int* s_c,
                                   int* s_m) {
  const int nt = g.ntiles;
  const int tid = threadIdx.x;
  if (tid == 0 && pending[0] != 0) {
    *bump_items += pending[0];
    *bump_fill += pending[1];
    pending[0] = 0;
    pending[1] = 0;
  }
  if (!sort) return;
  const int per = (nt + NT - 1) / NT;
  const int t0 = min(nt, tid * per), t1 = min(nt, t0 + per);
  int c = 0, m = 0;
  for (int t = t0; t < t1; ++t) {
    const int v = hist[t];
    c += v;
    m += (v + g.chunk - 1) / g.chunk;
  }
  s_c[tid] = c;
  s_m[tid] = m;
  __syncthreads();
  for (int off = 1; off < NT; off <<= 1) {
    const int vc = tid >= off ? s_c[tid - off] : 0;
    const int vm = tid >= off ? s_m[tid - off] : 0;
    __syncthreads();
    s_c[tid] += vc;
    s_m[tid] += vm;
    __syncthreads();
  }
  int ec = s_c[tid] - c, em = s_m[tid] - m;
  const int total = s_c[NT - 1], n_items = s_m[NT - 1];
  // room kept for the columns injected before the next sort (one per step)
  const int item_cap = max_items - SORT_EVERY * g.ntr;
  for (int t = t0; t < t1; ++t) {
    const int v = hist[t];
    out.offsets[t] = ec;
    out.cursor[t] = ec;
    const int nm = (v + g.chunk - 1) / g.chunk;
    for (int k = 0; k < nm; ++k) {
      // the nm items of a tile share its particles evenly
      const int lo = (int)((long long)k * v / nm), hi = (int)((long long)(k + 1) * v / nm);
      const int st = ec + lo, cn = hi - lo;
      // items never reach past the buffer (an overflow is flagged below)
      out.items[em + k] = (em + k < item_cap && (long long)st + cn <= capacity) ? make_int4(t, st, cn, 0)
                                                                                : make_int4(t, 0, 0, 0);
    }
    ec += v;
    em += nm;
    hist[t] = 0;
  }
  if (tid == NT - 1) {
    out.offsets[nt] = total;
    *out.fill = total;
    *out.n_items = min(n_items, item_cap);
    if (n_items > item_cap) atomicOr(err, ERR_ITEMS);
    if ((long long)total + (long long)SORT_EVERY * inj_max > capacity) atomicOr(err, ERR_CAPACITY);
  }
}

}  // namespace envpic
