// common.hpp -- state layout and device helpers shared by the envpic kernels.
//
// Method: arXiv:1912.04674 (cylindrical envelope PIC).  Data layout in HBM:
//   * grids: one array per field, [column][row] with the radius contiguous
//     (pitch >= nr + 1, a multiple of 16), columns kept in a ring of `nxa`
//     entries indexed by lab column mod nxa, so a moving-window shift moves
//     no data;
//   * particles: structure of arrays, cell word (lab column, radial row),
//     offsets in the cell along x and r, azimuth, momenta, weight (R), id
//     (uint32), grouped by tile: each tile owns a segment of a buffer (the
//     tiles a moving window is about to enter, room for a full tile).  The
//     sort by tile runs every third step (every second with quadratic
//     shapes); it moves only the particles that changed tile (into free
//     slots of their new tile's segment, or into an overflow range of that
//     tile past all segments), and every CELL_SORT_EVERY-th sort rebuilds
//     the whole layout, ordered by cell, in the second buffer (the two
//     buffers ping-pong at those sorts);
//   * the envelope rows j = 0, 1 additionally in FP64 (FP32 mode).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace envpic {

constexpr int TX = 16;      // tile width along x (cells)
constexpr int TR = 16;      // tile height along r (cells)
// Particles move at most one cell per step and are re-sorted by tile every
// SORT_EVERY steps, so a particle is at most SORT_EVERY cells outside its
// tile at a gather (SORT_EVERY + 1 at the end of a push); one more cell of
// margin holds the linear and half-cell-staggered stencils.  Quadratic
// stencils reach one node further and re-sort every SORT_EVERY - 1 steps,
// which keeps them inside the same margin.
constexpr int SORT_EVERY = 3;
constexpr int HALO = SORT_EVERY + 1;  // LDS region margin around a tile (cells)
constexpr int LX = TX + 2 * HALO + 1;
constexpr int LR = TR + 2 * HALO + 1;
constexpr int LN = LX * LR; // nodes of an LDS tile region
// cells a tile's particles can occupy at a sort (its 16 x 16 cells plus
// SORT_EVERY on each side): the per-cell counts of a work item live here
constexpr int CR = TX + 2 * SORT_EVERY;
constexpr int CRN = CR * CR;
// how a sort moves the particles: by tile (only the particles that changed
// tile move; if the layout has no room for them, every particle is
// scattered into the other buffer and copied back), or by cell with the
// placement of loading (every CELL_SORT_EVERY-th sort, into the other
// buffer)
constexpr int SCAT_NONE = 0, SCAT_TILE = 1, SCAT_CELL = 2;
constexpr int CELL_SORT_EVERY = 8;
// the layout a scan produced for a tile sort: incremental, or every particle
// scattered (not enough free slots, overflow room or work items)
constexpr int LAYOUT_MOVE = 0, LAYOUT_FULL = 1;
// flag of a cell-sort layout: the cell-ordered copy is gathered (k_permute)
// instead of scattered by the momentum pass
constexpr int LAYOUT_GATHER = 2;
// Tile columns ahead of a moving window whose segments get room for a full
// tile when the layout is rebuilt (the window enters at most one column per
// step, SORT_EVERY * CELL_SORT_EVERY steps between rebuilds), with the tile
// column the window's front is in
constexpr int ENTERING_TILES = (SORT_EVERY * CELL_SORT_EVERY + TX - 1) / TX + 1;
constexpr int WG = 512;     // work-group size of the particle kernels
constexpr int CHUNK = 4096; // largest work item (particles); small runs use smaller items
// particle buffers at least this large (one buffer's records) stream past the
// 256 MB last-level cache: their records are accessed non-temporally
constexpr long long STREAM_PARTS_BYTES = 256LL << 20;
// A particle's cell is one 32-bit word: lab column << 12 | radial row.  The
// position inside the cell is kept as FP32 (or FP64) offsets along x and r,
// so neither a long moving-window run nor a large radius erodes the
// resolution of the offsets; the azimuth is kept separately.
constexpr int JR_BITS = 12;
constexpr unsigned JR_MASK = (1u << JR_BITS) - 1u;
constexpr int NR_MAX = (1 << JR_BITS) - 2;           // rows
constexpr long long COL_MAX = (1LL << (32 - JR_BITS)) - 2;  // lab columns
constexpr unsigned kDead = 0xFFFFFFFFu;              // cell word of a removed particle
__host__ __device__ inline unsigned pack_cell(int ix, int jr) { return ((unsigned)ix << JR_BITS) | (unsigned)jr; }
__host__ __device__ inline int cell_ix(unsigned c) { return (int)(c >> JR_BITS); }
__host__ __device__ inline int cell_jr(unsigned c) { return (int)(c & JR_MASK); }

// error bits of the device error word
constexpr int ERR_HALO = 1;      // a particle left the LDS halo of its tile
constexpr int ERR_CAPACITY = 2;  // particle buffer capacity exceeded
constexpr int ERR_ITEMS = 4;     // work-item list overflow
constexpr int ERR_LAYOUT = 8;    // a sort met more arrivals at a tile than its scan counted

template <class R> struct cplx_of;
template <> struct cplx_of<float> { using type = float2; };
template <> struct cplx_of<double> { using type = double2; };

struct Geo {
  int nx, nr;        // cells
  int nxa;           // ring columns (multiple of TX)
  int pitch;         // elements per column
  int ntxa, ntr, ntiles;
  int modes;
  int ppc_x, ppc_r, ppc_t;
  int base;          // shift mod nxa (physical column of the window's left edge)
  int t_lo;          // lab tile index of column shift - 2
  long long shift;   // lab column of the window's left edge
  long long cap;     // particle slots per buffer
  double dx, dr, dt;
  float fix;         // fixed-point scale of the FP32 path's mode-1 current sums
  double unfix;      // 1 / fix
  float fix0;        // fixed-point scale of the FP32 path's chi and mode-0 current sums
  double unfix0;     // 1 / fix0
  int chunk;         // particles per work item at most (<= CHUNK, a multiple of WG)
  int order;         // particle shape order: 1 linear, 2 quadratic
  int stream_parts;  // 1: a particle buffer exceeds the last-level cache (non-temporal record access)
};

template <class R> struct Parts {
  unsigned* cell;  // lab column << 12 | radial row
  R* fx;           // offset in the cell along x, [0, 1)
  R* fr;           // offset in the cell along r, [0, 1] (1 only at r_max)
  R* th;           // azimuth, [-pi, pi]
  R* px;
  R* py;
  R* pz;
  R* w;
  uint32_t* id;
};

template <class R> struct Grids {
  using C = typename cplx_of<R>::type;
  R *ex, *er, *bt, *btb, *jx, *jr, *chi;
  C *env, *envp;
  double2 *ax, *axp;  // FP64 envelope rows 0, 1 of A^n and A^{n-1}: [phys col][2]
  C *ex1, *er1, *et1, *bx1, *br1, *bt1, *bxb1, *brb1, *btb1, *jx1, *jr1, *jt1;
  // second copies of E and B: the field update writes E^{n+1}, B^{n+3/2}
  // here and the host swaps them with the current ones
  R *ex_n, *er_n, *bt_n;
  C *ex1_n, *er1_n, *et1_n, *bx1_n, *br1_n, *bt1_n;
};

// A layout of one particle buffer.  Tile t owns the segment
// [offsets[t], offsets[t + 1]) and uses its first ext[t] slots (live or
// removed particles); slots from offsets[ntiles] to *fill hold the columns
// injected since the layout was built and particles that found no room in
// their tile's segment (work items of their own, keyed by their tile).
struct Layout {
  int* offsets;  // [ntiles + 1]
  int* ext;      // [ntiles] slots in use at the start of each segment
  int* cursor;   // [ntiles] scatter cursors (full) or arrival tickets (incremental)
  int* ovb;      // [ntiles] first overflow slot of each tile's arrivals (incremental)
  int* ovn;      // [ntiles] arrivals of each tile that go to its overflow range (incremental)
  int4* items;   // {key, start, count, 0}
  int* n_items;  // scalar
  int* fill;     // scalar: end of the used slots (injected columns are appended here)
  int* mode;     // scalar: LAYOUT_MOVE or LAYOUT_FULL (tile sorts)
};

// The copy back after a tile sort that rebuilt its layout (settle_copy):
// from the other buffer into the one in use, over the used slots of L, by
// `blocks` extra groups of the launch that carries it (none: 0)
constexpr int SETTLE_BLOCKS = 256;  // groups of 256 threads (they exit at once when no copy is due)
template <class R> struct SettleArgs {
  Parts<R> to, from;
  Layout L;
  long long cap;
  int blocks;
};

struct Plasma {
  int profile;
  double n0, ramp_len, perturb, bump_x, bump_w;
  unsigned long long seed;
};

struct Laser {
  double a0, w0, tau, x_c, x_f;
};

// ------------------------------------------------------------- helpers --
__host__ __device__ inline int wrap_col(int p, int nxa) { return p >= nxa ? p - nxa : p; }

// physical column of window-relative column rel (0 <= rel < nxa)
__host__ __device__ inline int phys_col(const Geo& g, int rel) { return wrap_col(g.base + rel, g.nxa); }

// lab tile index of ring tile column tcx
__device__ inline int lab_tile(const Geo& g, int tcx) {
  int d = tcx - (int)(((long long)g.t_lo % g.ntxa + g.ntxa) % g.ntxa);
  if (d < 0) d += g.ntxa;
  return g.t_lo + d;
}

__host__ __device__ inline int tile_key(const Geo& g, long long col, int jr) {
  long long t = col / TX;
  int tcx = (int)(t % g.ntxa);
  return tcx * g.ntr + jr / TR;
}

// node volume of primal row j: axis disc of radius dr/2, else 2 pi r_j dr dx
template <class R> __device__ inline R inv_vol_node(const Geo& g, int j) {
  const double pi = 3.14159265358979323846;
  double v = j == 0 ? pi * g.dr * g.dr * g.dx * 0.25 : 2.0 * pi * j * g.dr * g.dr * g.dx;
  return (R)(1.0 / v);
}
template <class R> __device__ inline R inv_vol_half(const Geo& g, int j) {
  const double pi = 3.14159265358979323846;
  return (R)(1.0 / (2.0 * pi * (j + 0.5) * g.dr * g.dr * g.dx));
}

// SplitMix64 (Steele, Lea, Flood 2014) used counter-style: the deviate for
// a key is the mix of seed + (key + 1) * golden gamma.
__host__ __device__ inline unsigned long long sm64_mix(unsigned long long z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
__host__ __device__ inline double counter_uniform(unsigned long long seed, unsigned long long stream,
                                                  long long col, long long j) {
  unsigned long long key = (stream << 56) ^ (((unsigned long long)col & 0xFFFFFFFFull) << 20) ^
                           ((unsigned long long)j & 0xFFFFFull);
  unsigned long long z = sm64_mix(seed + (key + 1ull) * 0x9E3779B97F4A7C15ull);
  return (double)(z >> 11) * (1.0 / 9007199254740992.0);
}
constexpr unsigned long long STREAM_ANGLE = 1;
constexpr unsigned long long STREAM_DENSITY = 2;

__host__ __device__ inline double plasma_density(const Plasma& p, double xlab, long long col, int j) {
  switch (p.profile) {
    case 1: return p.n0;
    case 2:
      if (xlab <= 0.0) return 0.0;
      if (xlab < p.ramp_len) return p.n0 * xlab / p.ramp_len;
      return p.n0;
    case 3: return p.n0 * (1.0 + p.perturb * (2.0 * counter_uniform(p.seed, STREAM_DENSITY, col, j) - 1.0));
    case 4: {
      double u = (xlab - p.bump_x) / p.bump_w;
      return p.n0 * (1.0 + exp(-u * u));
    }
    default: return 0.0;
  }
}

template <class T> __device__ inline T lds_get(const T* a, int x, int r) { return a[x * LR + r]; }

}  // namespace envpic
