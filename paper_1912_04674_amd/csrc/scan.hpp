// scan.hpp -- the sort's scans (device side): per tile, the exclusive scan
// of its cells' counts into the per-cell cursors (work groups of the
// field-stage kernel); over all tiles, the scans of the tile totals into the
// next layout's segments and work items, or of the arrivals into the free
// slots and overflow ranges of an incremental sort (one work group,
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

// Exclusive scan of one int per thread over the NT threads of a block
// (NT a multiple of 64, at most 64 wavefronts): shuffles inside each
// wavefront, then the wavefront totals through s_w (NT / 64 ints).  Returns
// the sum of the lower threads' values; *total gets the block's sum.  Every
// thread calls it.
template <int NT> __device__ inline int block_scan(int v, int* s_w, int* total) {
  const int lane = (int)(threadIdx.x & 63), w = (int)(threadIdx.x >> 6);
  int x = v;
  for (int o = 1; o < 64; o <<= 1) {
    const int y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  if (lane == 63) s_w[w] = x;
  __syncthreads();
  int pre = 0, tot = 0;
  for (int k = 0; k < NT / 64; ++k) {
    const int t = s_w[k];
    pre += k < w ? t : 0;
    tot += t;
  }
  __syncthreads();  // s_w is free again
  *total = tot;
  return pre + x - v;
}

// The items (pending[0]) and slots past the used ones (pending[1]) of a
// column injected since the last scan join layout L, the layout in use: an
// item placed at the end of its tile's segment extends the segment's used
// slots (the items of one column lie in distinct tiles).  Every thread of
// the block calls it; the caller synchronizes before reading L.
__device__ inline void bump_pending(const Geo& g, Layout L, int* pending) {
  const int np = pending[0];
  if (np == 0) return;
  const int n0 = *L.n_items, seg_end = L.offsets[g.ntiles];
  for (int i = threadIdx.x; i < np; i += blockDim.x) {
    const int4 it = L.items[n0 + i];
    if (it.y < seg_end) L.ext[it.x] += it.z;
  }
  __syncthreads();  // every thread has read n_items and pending
  if (threadIdx.x == 0) {
    *L.n_items = n0 + np;
    *L.fill += pending[1];
    pending[0] = 0;
    pending[1] = 0;
  }
}

// Work items of v particles from slot st: ceil(v / chunk) items of equal
// size, written from items[em] on (none past max_em); returns their number.
__device__ inline int emit_items(const Geo& g, int4* items, int em, int max_em, int key, int st, int v,
                                 long long capacity) {
  const int nm = (v + g.chunk - 1) / g.chunk;
  for (int k = 0; k < nm; ++k) {
    const int lo = (int)((long long)k * v / nm), hi = (int)((long long)(k + 1) * v / nm);
    // items never reach past the buffer (an overflow is flagged by the caller)
    if (em + k < max_em)
      items[em + k] = ((long long)st + hi <= capacity) ? make_int4(key, st + lo, hi - lo, 0) : make_int4(key, 0, 0, 0);
  }
  return nm;
}

// Slots a rebuilt layout holds for tile t of v particles: v, or a full tile
// when the tile lies in the `entering` tile columns ahead of a moving window
// (or in the one its front is in), which fill as columns are injected.
// Other tiles get no free slots: measured on the LWFA workload, free slots of
// 1/16 of each tile made the passes that stream the particles 5 % slower
// (their arrivals, rare, take overflow ranges instead).
__device__ inline int seg_room(const Geo& g, int t, int v, int entering) {
  if (entering <= 0) return v;
  const int tcx = t / g.ntr, tr = t - (t / g.ntr) * g.ntr;
  const long long T = lab_tile(g, tcx), front = (g.shift + g.nx - 1) / TX;
  if (T < front || T > front + entering) return v;
  return max(v, TX * min(TR, g.nr - tr * TR) * g.ppc_x * g.ppc_r * g.ppc_t);
}

// One block of NT threads: the tile totals in hist become layout `out` of
// the other buffer, the whole layout rebuilt: the segment of a tile of v
// particles holds seg_room slots (the room for entering tiles only when
// `reserve` slots past the segments stay free), and its particles form
// ceil(v / chunk) items of equal size.  hist stays (the kernels keep it
// current).  Flags when the particles plus the columns injected before the
// next sort would not fit.
template <int NT>
__device__ inline void full_layout(const Geo& g, int* hist, Layout out, long long capacity, int inj_max,
                                   long long reserve, int entering, int max_items, int* err, int* s_w) {
  const int nt = g.ntiles;
  const int tid = threadIdx.x;
  const int per = (nt + NT - 1) / NT;
  const int t0 = min(nt, tid * per), t1 = min(nt, t0 + per);
  int c = 0, m = 0, rs = 0;
  for (int t = t0; t < t1; ++t) {
    const int v = hist[t];
    c += v;
    rs += seg_room(g, t, v, entering);
    m += (v + g.chunk - 1) / g.chunk;
  }
  int total_c = 0, n_items = 0, total_rs = 0, seg_end = 0;
  block_scan<NT>(c, s_w, &total_c);
  int em = block_scan<NT>(m, s_w, &n_items);
  block_scan<NT>(rs, s_w, &total_rs);
  const int ent = (long long)total_rs + reserve <= capacity ? entering : 0;
  int cs = 0;
  for (int t = t0; t < t1; ++t) cs += seg_room(g, t, hist[t], ent);
  int ec = block_scan<NT>(cs, s_w, &seg_end);
  // room kept for the columns injected before the next sort (one per step)
  const int item_cap = max_items - SORT_EVERY * g.ntr;
  for (int t = t0; t < t1; ++t) {
    const int v = hist[t];
    out.offsets[t] = ec;
    out.ext[t] = v;
    out.cursor[t] = ec;
    out.ovb[t] = 0;
    out.ovn[t] = 0;
    em += emit_items(g, out.items, em, item_cap, t, ec, v, capacity);
    ec += seg_room(g, t, v, ent);
  }
  if (tid == NT - 1) {
    out.offsets[nt] = seg_end;
    *out.fill = seg_end;
    *out.n_items = min(n_items, item_cap);
    *out.mode = LAYOUT_FULL;
    if (n_items > item_cap) atomicOr(err, ERR_ITEMS);
    if ((long long)seg_end + (long long)SORT_EVERY * inj_max > capacity) atomicOr(err, ERR_CAPACITY);
  }
}

// One block of NT threads, before a tile sort: layout `out` of the same
// buffer as `in`, where only the particles that change tile move.  arr[t]
// holds the arrivals of tile t (particles of other tiles' items whose cell
// is now in t, and every particle of t's items past the segments: injected
// columns, earlier overflows), hist[t] its particles after the sort.  The
// arrivals fill the free slots at the end of t's segment, then a range of
// their own past the used slots (from ovb[t], ovn[t] of them).  When the
// overflow or the items would not fit, the layout is rebuilt as by
// full_layout instead (mode LAYOUT_FULL: the sort then scatters every
// particle).  arr is cleared; stats[0] counts the incremental layouts,
// stats[1] the rebuilt ones.
template <int NT>
__device__ inline void move_layout(const Geo& g, int* hist, int* arr, Layout in, Layout out, long long capacity,
                                   int inj_max, long long reserve, int entering, int max_items, int* err, int* stats,
                                   int* s_w) {
  const int nt = g.ntiles;
  const int tid = threadIdx.x;
  const int per = (nt + NT - 1) / NT;
  const int t0 = min(nt, tid * per), t1 = min(nt, t0 + per);
  const int seg_end = in.offsets[nt];
  const int fill0 = *in.fill;
  int ov = 0, m = 0;
  for (int t = t0; t < t1; ++t) {
    const int a = arr[t], e = in.ext[t], cap = in.offsets[t + 1] - in.offsets[t];
    const int tail = min(a, cap - e);
    ov += a - tail;
    m += (e + tail + g.chunk - 1) / g.chunk + (a - tail + g.chunk - 1) / g.chunk;
  }
  int total_ov = 0, n_items = 0;
  const int ov_pre = block_scan<NT>(ov, s_w, &total_ov);
  int em = block_scan<NT>(m, s_w, &n_items);
  const long long fill_new = (long long)fill0 + total_ov;
  const int item_cap = max_items - SORT_EVERY * g.ntr;
  if (fill_new + (long long)SORT_EVERY * inj_max > capacity || n_items > item_cap) {
    // every thread takes the same branch
    __syncthreads();
    if (tid == 0) stats[1] += 1;
    for (int t = t0; t < t1; ++t) arr[t] = 0;
    full_layout<NT>(g, hist, out, capacity, inj_max, reserve, entering, max_items, err, s_w);
    return;
  }
  int ob = fill0 + ov_pre;
  for (int t = t0; t < t1; ++t) {
    const int a = arr[t], e = in.ext[t], base = in.offsets[t], cap = in.offsets[t + 1] - base;
    const int tail = min(a, cap - e);
    out.offsets[t] = base;
    out.ext[t] = e + tail;
    out.cursor[t] = 0;
    out.ovb[t] = ob;
    out.ovn[t] = a - tail;
    em += emit_items(g, out.items, em, item_cap, t, base, e + tail, capacity);
    em += emit_items(g, out.items, em, item_cap, t, ob, a - tail, capacity);
    ob += a - tail;
    arr[t] = 0;
  }
  if (tid == NT - 1) {
    out.offsets[nt] = seg_end;
    *out.fill = (int)fill_new;
    *out.n_items = n_items;
    *out.mode = LAYOUT_MOVE;
    stats[0] += 1;
  }
}

// After a tile sort whose scan rebuilt the layout (LAYOUT_FULL), the sort
// wrote every particle into the other buffer: copy the used slots back (b of
// nb groups of 256 threads), so that the particles stay in the buffer they
// were in.  Nothing to do after an incremental sort.  Each lane moves four
// consecutive slots of every record array per pass with 16-byte accesses
// (the arrays start 256-byte aligned), so that enough bytes are in flight to
// stream at the copy rate; the slots past the last multiple of four go one
// by one.
template <class T> __device__ inline void copy4(T* to, const T* from, long long i) {
  static_assert(sizeof(T) == 4, "4-byte record arrays");
  *reinterpret_cast<uint4*>(to + i) = *reinterpret_cast<const uint4*>(from + i);
}
template <class R>
__device__ inline void settle_copy(const SettleArgs<R>& sa, int b, int nb) {
  if (*sa.L.mode != LAYOUT_FULL) return;
  const long long n = min((long long)*sa.L.fill, sa.cap);
  const long long n4 = n & ~3LL;
  if constexpr (sizeof(R) == 4) {
    for (long long i = ((long long)b * 256 + threadIdx.x) * 4; i < n4; i += (long long)nb * 256 * 4) {
      copy4(sa.to.cell, sa.from.cell, i);
      copy4(sa.to.fx, sa.from.fx, i);
      copy4(sa.to.fr, sa.from.fr, i);
      copy4(sa.to.th, sa.from.th, i);
      copy4(sa.to.px, sa.from.px, i);
      copy4(sa.to.py, sa.from.py, i);
      copy4(sa.to.pz, sa.from.pz, i);
      copy4(sa.to.w, sa.from.w, i);
      copy4(sa.to.id, sa.from.id, i);
    }
  }
  const long long i0 = sizeof(R) == 4 ? n4 : 0;
  for (long long i = i0 + (long long)b * 256 + threadIdx.x; i < n; i += (long long)nb * 256) {
    sa.to.cell[i] = sa.from.cell[i];
    sa.to.fx[i] = sa.from.fx[i];
    sa.to.fr[i] = sa.from.fr[i];
    sa.to.th[i] = sa.from.th[i];
    sa.to.px[i] = sa.from.px[i];
    sa.to.py[i] = sa.from.py[i];
    sa.to.pz[i] = sa.from.pz[i];
    sa.to.w[i] = sa.from.w[i];
    sa.to.id[i] = sa.from.id[i];
  }
}

}  // namespace envpic
