// particles.hip -- per-macroparticle kernels of the cylindrical envelope PIC
// step (arXiv:1912.04674): the momentum pass (gather of E, Bbar, Phi and
// grad Phi, ponderomotive Boris push, chi deposit, scatter into the tile
// order of the next pass), the position pass (gather of Phi^{n+1/2}, push,
// current deposit, tile histogram), loading and injection.
//
// Work decomposition: particles are counting-sorted by 16 x 16-cell tiles
// every SORT_EVERY steps (SORT_EVERY - 1 for quadratic shapes); a work item
// is (tile, contiguous range of at most g.chunk particles).  A work group
// stages the fields of its tile plus a
// HALO-cell margin in LDS, accumulates the deposits of its particles in LDS
// and flushes them to HBM once (atomic adds, since halos overlap).
// Particles drift at most one cell per step (dt < dx, dt < dr), so between
// two sorts they stay inside the margin.
//
// Positions: lab cell (column, row) in one word plus offsets in the cell
// along x and r and the azimuth; the push is Cartesian (Sec. 3), and the
// new radius is obtained from the radial and azimuthal components of the
// displacement without cancellation, so the offsets keep their resolution at
// any radius.
#include <algorithm>

#include "common.hpp"
#include "cplx.hpp"
#include "launch.hpp"
#include "scan.hpp"

namespace envpic {

// ------------------------------------------------------------ shapes --
template <class R> struct Lin {
  int i;   // first node (local LDS index)
  R a, b;  // weights of nodes i and i+1
};

template <class R> __device__ inline Lin<R> primal_w(int c, R f) { return Lin<R>{c, (R)1 - f, f}; }
template <class R> __device__ inline Lin<R> dual_w(int c, R f) {
  R v = f - (R)0.5;
  if (v < (R)0) return Lin<R>{c - 1, (R)0.5 - f, f + (R)0.5};
  return Lin<R>{c, (R)1 - v, v};
}

// (RL: the row length of the LDS region the values are staged in)
template <class R, int RL = LR> __device__ inline R interp2(const R* a, Lin<R> sx, Lin<R> sr) {
  return sx.a * (sr.a * a[sx.i * RL + sr.i] + sr.b * a[sx.i * RL + sr.i + 1]) +
         sx.b * (sr.a * a[(sx.i + 1) * RL + sr.i] + sr.b * a[(sx.i + 1) * RL + sr.i + 1]);
}
template <class C, class R, int RL = LR> __device__ inline C interp2c(const C* a, Lin<R> sx, Lin<R> sr) {
  C v00 = a[sx.i * RL + sr.i], v01 = a[sx.i * RL + sr.i + 1];
  C v10 = a[(sx.i + 1) * RL + sr.i], v11 = a[(sx.i + 1) * RL + sr.i + 1];
  R w00 = sx.a * sr.a, w01 = sx.a * sr.b, w10 = sx.b * sr.a, w11 = sx.b * sr.b;
  return mk<C>(w00 * v00.x + w01 * v01.x + w10 * v10.x + w11 * v11.x,
               w00 * v00.y + w01 * v01.y + w10 * v10.y + w11 * v11.y);
}

// Quadratic B-spline (order 2) on three nodes i, i+1, i+2 around the nearest
// node m = i + 1, d = u - m in [-1/2, 1/2): (1/2 - d)^2/2, 3/4 - d^2,
// (1/2 + d)^2/2.  Primal nodes sit at the cell corners (nearest node a or
// a + 1), dual nodes at the cell centres (nearest node always a).
// The outer weights differ by d, so the last is formed as the first plus d
// (four operations per stencil instead of seven; the absolute error stays
// within an ulp of 1/2).
template <class R> struct Quad {
  int i;
  R w[3];
};
template <class R> __device__ inline Quad<R> quad_of(int i, R d) {
  const R w0 = fma(d, fma(d, (R)0.5, (R)-0.5), (R)0.125);  // (1/2 - d)^2 / 2
  return Quad<R>{i, {w0, fma(-d, d, (R)0.75), w0 + d}};
}
template <class R> __device__ inline Quad<R> quad_primal(int c, R f) {
  return f < (R)0.5 ? quad_of<R>(c - 1, f) : quad_of<R>(c, f - (R)1);
}
template <class R> __device__ inline Quad<R> quad_dual(int c, R f) { return quad_of<R>(c - 1, f - (R)0.5); }

template <class R, int RL = LR> __device__ inline R interp3(const R* a, const Quad<R>& sx, const Quad<R>& sr) {
  R acc = 0;
#pragma unroll
  for (int u = 0; u < 3; ++u) {
    const R* col = a + (sx.i + u) * RL + sr.i;
    acc += sx.w[u] * (sr.w[0] * col[0] + sr.w[1] * col[1] + sr.w[2] * col[2]);
  }
  return acc;
}
template <class C, class R, int RL = LR>
__device__ inline C interp3c(const C* a, const Quad<R>& sx, const Quad<R>& sr) {
  R re = 0, im = 0;
#pragma unroll
  for (int u = 0; u < 3; ++u) {
    const C* col = a + (sx.i + u) * RL + sr.i;
    re += sx.w[u] * (sr.w[0] * col[0].x + sr.w[1] * col[1].x + sr.w[2] * col[2].x);
    im += sx.w[u] * (sr.w[0] * col[0].y + sr.w[1] * col[1].y + sr.w[2] * col[2].y);
  }
  return mk<C>(re, im);
}

// Phi and its centred differences (times 1/(2 dx), 1/(2 dr)) interpolated
// with one quadratic stencil, from Phi on the 5 x 5 nodes around the 3 x 3 of
// the stencil (corners unused).  j0 is the grid row of the stencil's first
// node (at least -1): the radial difference is zero on the axis row and, on
// the ghost row below it, minus its value on row 1.
template <class R, int RL>
__device__ inline void phi_grad3(const R* phi, const Quad<R>& sx, const Quad<R>& sr, int j0, R i2dx, R i2dr,
                                 R& ph, R& gx, R& gr) {
  // the differences taken through the weights: a node's Phi enters the x
  // difference with the weight of the node behind it minus that of the node
  // ahead; the radial weights of the axis row and the ghost row are moved
  // (zero on the axis, the ghost row folded onto row 1 with a sign)
  const R k0 = j0 >= 1 ? sr.w[0] : (R)0, k1 = j0 >= 0 ? sr.w[1] : (R)0;
  const R k2 = j0 == -1 ? sr.w[2] - sr.w[0] : sr.w[2];
  const R dx[5] = {-sx.w[0], -sx.w[1], sx.w[0] - sx.w[2], sx.w[1], sx.w[2]};
  const R dr[5] = {-k0, -k1, k0 - k2, k1, k2};
  const R* p = phi + sx.i * RL + sr.i;
  R a = 0, b = 0, d = 0;
#pragma unroll
  for (int u = -1; u < 4; ++u) {
    const R* c = p + u * RL;
    if (u >= 0 && u <= 2) {
      const R c0 = c[0], c1 = c[1], c2 = c[2];
      a += sx.w[u] * (sr.w[0] * c0 + sr.w[1] * c1 + sr.w[2] * c2);
      d += sx.w[u] * (dr[0] * c[-1] + dr[1] * c0 + dr[2] * c1 + dr[3] * c2 + dr[4] * c[3]);
      b += dx[u + 1] * (sr.w[0] * c0 + sr.w[1] * c1 + sr.w[2] * c2);
    } else {
      b += dx[u + 1] * (sr.w[0] * c[0] + sr.w[1] * c[1] + sr.w[2] * c[2]);
    }
  }
  ph = a;
  gx = b * i2dx;
  gr = d * i2dr;
}

// v clamped to [lo, hi]; bad is set when it was outside (one min/max and one
// compare)
__device__ inline int clampi(int v, int lo, int hi, bool& bad) {
  const int c = min(max(v, lo), hi);
  bad |= c != v;
  return c;
}

__device__ inline void lds_add(float* a, float v) { atomicAdd(a, v); }
__device__ inline void lds_add(double* a, double v) { atomicAdd(a, v); }

// Mode-1 current accumulators.  The FP64 path sums in FP64 LDS words.  The
// FP32 path sums fixed-point integers in 64-bit LDS words: on gfx950 integer
// LDS atomics issue faster than FP64 ones (and FP32 LDS atomics are far
// slower than either, measured), and an integer sum is exact and independent
// of the order in which the lanes land.  Each contribution is scaled by
// g.fix = 2^32 / (2 w_max / V_0), the bound of any |2 q w v S / V| (|v| < 1,
// S <= 1, V_0 the smallest node volume), so one contribution is at most 2^32
// in magnitude and the <= 2 CHUNK contributions of a work item to one node
// (and a fold of two such nodes) stay below 2^46.
//
// The float -> fixed conversion is one FP64 FMA: u x + 1.5 2^52 rounds u x
// to the nearest integer v and its bit pattern is 0x4338 2^48 + v (exact for
// |v| < 2^51).  The words add those patterns as they are; the constant parts
// only reach bits 48..63, so the low 48 bits of a word hold the sum of the v
// modulo 2^48, which is the sum itself, as |sum| < 2^47 (fixed_sum reads it).
// On the hot path this saves the subtraction of the constant per atomic.
// add_prod(a, u, x, y) adds u x and u y, formed in FP64.
template <class R> struct Acc1;
template <> struct Acc1<double> {
  using T = double2;
  using S = double;  // one word (real or imaginary part)
  __device__ static T zero() { return make_double2(0.0, 0.0); }
  __device__ static double scale(const Geo&) { return 1.0; }
  template <class A> __device__ static void add_prod(A& a, int k, double u, double x, double y) {
    atomicAdd(&a.re[k], u * x);
    atomicAdd(&a.im[k], u * y);
  }
  __device__ static bool nonzero(const T& v) { return v.x != 0.0 || v.y != 0.0; }
  __device__ static double re(const T& v, const Geo&) { return v.x; }
  __device__ static double im(const T& v, const Geo&) { return v.y; }
};
// bit pattern of u x + 1.5 2^52: 0x4338 2^48 + the nearest integer to u x
// (|u x| < 2^51)
__device__ inline unsigned long long fixed_bits(double u, double x) {
  return (unsigned long long)__double_as_longlong(fma(u, x, 6755399441055744.0));  // 1.5 * 2^52
}
// the sum held by a word of fixed_bits patterns: its low 48 bits, signed
__device__ inline long long fixed_sum(long long w) {
  return (long long)((unsigned long long)w << 16) >> 16;
}
template <> struct Acc1<float> {
  using T = longlong2;
  using S = long long;  // one word (real or imaginary part)
  __device__ static T zero() { return make_longlong2(0, 0); }
  __device__ static float scale(const Geo& g) { return g.fix; }
  template <class A> __device__ static void add_prod(A& a, int k, double u, double x, double y) {  // already scaled
    atomicAdd((unsigned long long*)&a.re[k], fixed_bits(u, x));
    atomicAdd((unsigned long long*)&a.im[k], fixed_bits(u, y));
  }
  __device__ static bool nonzero(const T& v) { return fixed_sum(v.x) != 0 || fixed_sum(v.y) != 0; }
  __device__ static float re(const T& v, const Geo& g) { return (float)((double)fixed_sum(v.x) * g.unfix); }
  __device__ static float im(const T& v, const Geo& g) { return (float)((double)fixed_sum(v.y) * g.unfix); }
};

// Mode-0 deposit accumulators (chi, and J_x, J_r of the Esirkepov scheme).
// A contribution is w S: the weight times shape factors (or, for the
// currents, a partial sum of shape differences in [-1, 1]) without the
// inverse node volume or face area, which depend on the row only and are
// applied once per node at the flush.  The FP64 path sums FP64 words; the
// FP32 path sums fixed point as the mode-1 accumulators do, scaled by g.fix0
// = 2^32 / w_max, so a contribution is at most 2^32 and the <= 2 CHUNK
// contributions of a work item to one node (and a fold of two such nodes)
// stay below 2^46 (exact, order-independent sums).
template <class R> struct Acc0;
template <> struct Acc0<double> {
  using T = double;
  __device__ static double scale(const Geo&) { return 1.0; }
  __device__ static void add_prod(T* a, double u, double x) { atomicAdd(a, u * x); }
  __device__ static bool nonzero(T v) { return v != 0.0; }
  __device__ static double val(T v, const Geo&) { return v; }
};
template <> struct Acc0<float> {
  using T = long long;
  __device__ static double scale(const Geo& g) { return g.fix0; }
  __device__ static void add_prod(T* a, double u, double x) { atomicAdd((unsigned long long*)a, fixed_bits(u, x)); }
  __device__ static bool nonzero(T v) { return fixed_sum(v) != 0; }
  __device__ static double val(T v, const Geo& g) { return (double)fixed_sum(v) * g.unfix0; }
};

// Elementary functions.  The FP32 path uses the hardware reciprocal, square
// root, reciprocal square root and sine/cosine (about 1 ulp, or ~1e-6 for
// the direction cosines of the azimuth, far inside the FP32 path's
// tolerance); the FP64 path uses the libm calls.
__device__ inline float rsqrt_r(float x) { return __builtin_amdgcn_rsqf(x); }  // x >= 1 here
__device__ inline double rsqrt_r(double x) { return rsqrt(x); }
__device__ inline float sqrt_r(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ inline double sqrt_r(double x) { return sqrt(x); }
__device__ inline float rcp_r(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ inline double rcp_r(double x) { return 1.0 / x; }
__device__ inline void sincos_r(float t, float* s, float* c) {
  *s = __sinf(t);
  *c = __cosf(t);
}
__device__ inline void sincos_r(double t, double* s, double* c) { sincos(t, s, c); }
// azimuth increment atan2(b, ra); in FP32, for ra > 0 and |b/ra| < 0.05 the
// odd series beta - beta^3/3 + beta^5/5 (truncation below beta^7/7 < 1.2e-10,
// under the FP32 resolution of the azimuth)
__device__ inline float dtheta(float b, float ra) {
  if (ra > 0.0f) {
    const float beta = b * rcp_r(ra);
    if (fabsf(beta) < 0.05f) {
      const float b2 = beta * beta;
      return beta * (1.0f - b2 * (1.0f / 3.0f - b2 * 0.2f));
    }
  }
  return atan2f(b, ra);
}
__device__ inline double dtheta(double b, double ra) { return atan2(b, ra); }

// carry an offset back into [0, 1): cell += floor(off), off -= floor(off)
template <class R> __device__ inline void carry(int& cell, R& off) {
  const R c = floor(off);
  cell += (int)c;
  off -= c;
  if (off >= (R)1) {  // rounding of 1 - tiny
    off = 0;
    cell += 1;
  }
}

// New radius and azimuth after a Cartesian transverse displacement with
// radial component a and azimuthal component b (lengths) from radius r:
// r' = |(r + a, b)|, written r' - r = a + (r + a)(sqrt(1 + beta^2) - 1) with
// beta = b/(r + a) so that small displacements keep full relative precision.
template <class R> __device__ inline void radial_step(R r, R a, R b, R& dr_out, R& dth) {
  const R ra = r + a;
  if (ra > (R)0) {
    const R beta = b * rcp_r(ra);
    const R q = sqrt_r((R)1 + beta * beta);
    dr_out = a + ra * beta * beta * rcp_r((R)1 + q);
  } else {
    dr_out = sqrt_r(ra * ra + b * b) - r;
  }
  dth = dtheta(b, ra);
}

template <class R> __device__ inline R wrap_angle(R t) {
  const R pi = (R)3.14159265358979323846, two_pi = (R)6.28318530717958647692;
  if (t > pi) t -= two_pi;
  if (t < -pi) t += two_pi;
  return t;
}

// Access to the particle records.  Each pass reads and writes a record once;
// when a simulation's particle buffers are larger than the last-level cache
// (NT), the records are read and written with non-temporal hints so that
// streaming them does not evict the grids, which the tiles' regions re-read
// and the field stage reads next (measured: the field stage of the
// 2048 x 256 LWFA workload 37 -> 28 us, its step 5.6 % shorter).  Runs whose
// buffers fit in that cache keep ordinary accesses, which let the next pass
// find the records there.
template <bool NT, class T> __device__ inline T pld(const T* p) {
  if constexpr (NT) return __builtin_nontemporal_load(p);
  else return *p;
}
template <bool NT, class T> __device__ inline void pst(T* p, T v) {
  if constexpr (NT) __builtin_nontemporal_store(v, p);
  else *p = v;
}
// Element i of a record array: for 4-byte elements the byte offset is formed
// in 32 bits (slots < 2^30), so the access takes the array's address from
// scalar registers and the 32-bit offset from a vector register, with no
// 64-bit address arithmetic per lane.
template <class T> __device__ inline T* elem(T* a, int i) {
  if constexpr (sizeof(T) == 4) return (T*)((char*)a + (unsigned)i * 4u);
  else return a + i;
}
template <class T> __device__ inline const T* elem(const T* a, int i) {
  if constexpr (sizeof(T) == 4) return (const T*)((const char*)a + (unsigned)i * 4u);
  else return a + i;
}

// Loading order inside a tile: the R particles of a tile, enumerated cell
// by cell, fill a K-column matrix row by row (K = ceil(R/64)) and are stored
// column by column.  The 64 lanes of a wavefront then hold particles K apart
// in the enumeration, i.e. from cells at least four rows apart, so their
// deposit stencils do not share LDS addresses.  The per-step scatter keeps
// the relative order of the particles it moves, so the interleaving made at
// loading persists while every pass reads and writes contiguously.
__device__ inline int transpose_rank(int r, int R) {
  const int K = (R + 63) / 64;
  const int rows = (R + K - 1) / K;
  const int L = R - (rows - 1) * K;  // columns holding `rows` entries
  const int m = r % K, q = r / K;
  return m * rows - max(0, m - L) + q;
}

// slot of the r-th particle (in cell order) of a tile of v particles: the
// tile splits into nm = ceil(v / chunk) equal work items (as the scan makes
// them), and inside an item the particles are placed as at loading.  With
// linear shapes (O = 1) an item takes a contiguous range of ranks.  With
// quadratic shapes the ranks are dealt to the items in turn (listed by
// r mod nm, then r / nm, and cut into the items' sizes), so that every item
// spans all cells of the tile and a wavefront's lanes stay four cells apart
// in cell order with the smaller items of that order (measured: the
// position pass 5 % faster on the LWFA workload; with linear shapes the
// 8192 x 768 workload, six particles per cell more than an item holds,
// became 5 % slower, so they keep contiguous ranges)
template <int O> __device__ inline int placed_rank(int r, int v, int chunk) {
  const int nm = (v + chunk - 1) / chunk;
  int t = r;
  if constexpr (O == 2) {
    if (nm == 1) return transpose_rank(r, v);
    const int a = v / nm, b = v - a * nm, m = r % nm;
    t = m * a + min(m, b) + r / nm;  // (the first b residues hold a + 1 ranks)
  }
  int k = (int)((long long)t * nm / v);
  if (k + 1 < nm && (int)((long long)(k + 1) * v / nm) <= t) ++k;
  const int lo = (int)((long long)k * v / nm), hi = (int)((long long)(k + 1) * v / nm);
  return lo + transpose_rank(t - lo, hi - lo);
}

// the tile region of a work item with a margin of h cells: lab column
// X0 = T TX - h, row R0 = tcr TR - h
struct Region {
  int T, tcx, tcr;
  int X0;  // lab column (lab columns fit 20 bits)
  int relX0, R0;
};
__device__ inline Region region_of(const Geo& g, int key, int h = HALO) {
  Region q;
  q.tcx = key / g.ntr;
  q.tcr = key - q.tcx * g.ntr;
  q.T = lab_tile(g, q.tcx);
  q.X0 = q.T * TX - h;
  q.relX0 = (int)((long long)q.X0 - g.shift);
  q.R0 = q.tcr * TR - h;
  return q;
}

// ================================================== momentum pass ==
// The chi deposit accumulates in 64-bit LDS words (Acc0): 64-bit atomics
// run at a much higher rate than ds_add_f32 on gfx950 (measured), and the
// accumulated sums are rounded once, at the flush.
// A region with a margin of H cells: (TX + 2H + 1) x (TR + 2H + 1) nodes.
template <int H> struct Halo {
  static constexpr int X = TX + 2 * H + 1, R = TR + 2 * H + 1, N = X * R;
};
// The gradient of Phi is staged only by the scattering passes with quadratic
// shapes (their registers are the tighter limit); the others difference the
// staged Phi where they read it.  The sort counters exist only in the
// scattering variants.
template <class R, bool M1, int H, int O, bool SC> struct SmemMom {
  using C = typename cplx_of<R>::type;
  static constexpr int N = Halo<H>::N;
  static constexpr int NG = (O == 2 && SC) ? N : 1;
  R ex[N], er[N], bt[N], phi[N], gx[NG], gr[NG];
  typename Acc0<R>::T chi[N];
  C ex1[M1 ? N : 1], er1[M1 ? N : 1], et1[M1 ? N : 1];
  C bx1[M1 ? N : 1], br1[M1 ? N : 1], bt1[M1 ? N : 1];
  R ivol[Halo<H>::R];
  int ccell[SC ? CRN : 1];  // sort: particles per destination cell, then their first slot
};
constexpr int PPT = CHUNK / WG;  // particles per thread of a work item

// Work item of work group b (of n groups).  Work groups are dealt to the 8
// XCDs in turn; runs of XG consecutive items (radially adjacent tiles, whose
// LDS regions overlap) are given to one XCD so that the halo lines they
// share are fetched into that XCD's L2 once, and the runs rotate over the
// XCDs, which keeps their loads even.  A bijection of [0, n).
constexpr int XCDS = 8, XG = 4;
__device__ inline int item_of(int b, int n) {
  constexpr int sg = XCDS * XG;
  if (b >= (n / sg) * sg) return b;
  const int q = b / XCDS, x = b - q * XCDS;
  return ((q / XG) * XCDS + x) * XG + (q - (q / XG) * XG);
}

// sum over the 64 lanes of a wavefront (every lane active)
__device__ inline int wave_sum_i(int v) {
  for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
  return v;
}

// Rank of this lane among the lanes of its wavefront with the same slot
// (slot < 0: none), added to a counter per slot with one LDS atomic per
// distinct slot in the wavefront.  The lanes of a wavefront mostly share
// one destination, which a per-lane atomic serialises on one LDS word.
// Ranks follow lane order within a slot.  Call from wavefront-uniform
// control flow.
__device__ inline int wave_slot_rank(int slot, int* counters) {
  const int lane = (int)__lane_id();
  const unsigned long long below = (1ull << lane) - 1ull;
  unsigned long long pending = __ballot(slot >= 0);
  int rank = 0;
  while (pending) {
    const int leader = __ffsll((unsigned long long)pending) - 1;
    const int s = __shfl(slot, leader);
    const unsigned long long m = __ballot(slot == s);
    int base = 0;
    if (lane == leader) base = atomicAdd(&counters[s], (int)__popcll(m));
    base = __shfl(base, leader);
    if (slot == s) rank = base + (int)__popcll(m & below);
    pending &= ~m;
  }
  return rank;
}

// SCAT: SCAT_NONE updates p in place and keeps the layout.  SCAT_TILE
// re-sorts by tile into the next layout (the tiles of x^n), as its scan
// made it: incrementally (LAYOUT_MOVE: a particle that stays in its tile
// keeps its slot and has p updated in place; one that changed tile is
// written, whole, to a free slot of its new tile's segment or to that
// tile's overflow range, and its old slot is marked removed), or, when the
// scan found no room (LAYOUT_FULL), every particle is written into the other
// buffer keeping the particles' relative order (coalesced writes), from where
// settle_copy copies them back (in the envelope stage's launch).  SCAT_CELL
// orders each tile by cell and places every work item as at loading, so that
// the lanes of a wavefront hold particles of distinct cells again (the
// deposits' LDS atomics do not collide), at the price of strided writes.
// O: particle shape order (1 linear, 2 quadratic; order 2 re-sorts every
// second step, so its wider stencil stays inside the same halo).
// Waves per SIMD the compiler must allow: the FP32 in-place pass fits four
// work groups per CU in LDS (its smaller region, no staged gradient), so its
// registers are held to 64 per lane (eight waves per SIMD); the others are
// not constrained.
template <class R, bool DEFER, int SCAT, int O> constexpr int mom_waves_per_simd() {
  return (sizeof(R) == 4 && !DEFER && SCAT == SCAT_NONE) ? 8 : 1;
}

// Margin: a scattering pass gathers at most SORT_EVERY cells of drift from
// the tile (SORT_EVERY - 1 with quadratic shapes) and needs the full HALO;
// the passes in between have drifted one cell less and stage a region with
// one cell less of margin (fewer bytes staged, less LDS per work group).
template <class R, bool M1, bool DEFER, int SCAT, int O, bool NT>
__global__ __launch_bounds__(WG, (mom_waves_per_simd<R, DEFER, SCAT, O>())) void k_momentum(
    Geo g, Grids<R> f, R* __restrict__ chi_out,
                                                 Parts<R> src, Parts<R> dst, Layout Ls, Layout Ld,
                                                 int* __restrict__ ccur, R* __restrict__ gscr,
                                                 unsigned* __restrict__ inv, int* err) {
  using C = typename cplx_of<R>::type;
  constexpr int H = (SCAT == SCAT_NONE && !DEFER) ? HALO - 1 : HALO;
  constexpr int RX = Halo<H>::X, RL = Halo<H>::R, RN = Halo<H>::N;
  __shared__ SmemMom<R, M1, H, O, SCAT != SCAT_NONE> sm;
  const int item = item_of(blockIdx.x, gridDim.x);
  if (item >= *Ls.n_items) return;
  const int4 it = Ls.items[item];
  const int start = it.y, count = it.z;
  const Region q = region_of(g, it.x, H);
  const R hdt = (R)(0.5 * g.dt);

  // ---- stage E, Bbar, Phi (and mode 1) of the region in LDS.  Every load
  // reads a valid address (the index falls back to the column start) and the
  // value is selected afterwards; outside the grid the value is zero, and on
  // the ghost row j = -1 the radial-staggered values mirror row 1/2 with the
  // parity of the component (odd for mode-0 E_r and Bbar_t and mode-1 B_x).
  // The quadratic stencil also reaches the primal ghost row j = -1, which
  // mirrors row 1 (odd: mode-1 E_x; even: the others).
  for (int k = threadIdx.x; k < RN; k += WG) {
    const int a = k / RL, b = k - (k / RL) * RL;
    const int rel = q.relX0 + a, j = q.R0 + b;
    const bool px = rel >= 0 && rel <= g.nx, dxok = rel >= 0 && rel <= g.nx - 1;
    const size_t o = (px || dxok) ? (size_t)phys_col(g, rel) * g.pitch : 0;
    const bool pr = j >= 0 && j <= g.nr, drok = j >= 0 && j <= g.nr - 1, ghost = j == -1;
    const bool pg = O == 2 && ghost && g.nr >= 1;      // primal ghost row (order 2)
    const bool pv = pr || pg;
    const size_t in = pr ? o + j : (pg ? o + 1 : o);   // primal row (clamped), ghost -> row 1
    const size_t ih = drok ? o + j : o;                // half row, ghost -> row 1/2
    const R hs = drok ? (R)1 : (ghost ? (R)-1 : (R)0); // odd parity on the ghost row
    const R hp = drok ? (R)1 : (ghost ? (R)1 : (R)0);  // even parity on the ghost row
    const R vex = f.ex[in], ver = f.er[ih], vbt = f.btb[ih];
    const C venv = f.env[in];
    sm.ex[k] = (dxok && pv) ? vex : (R)0;
    sm.er[k] = px ? hs * ver : (R)0;
    sm.bt[k] = dxok ? hs * vbt : (R)0;
    sm.phi[k] = (px && pv) ? (R)0.5 * cnorm(venv) : (R)0;
    sm.chi[k] = 0;
    if (M1) {
      const C z = mk<C>((R)0, (R)0);
      const C e1 = f.ex1[in], r1 = f.er1[ih], t1 = f.et1[in];
      const C bx = f.bxb1[ih], br = f.brb1[in], bt = f.btb1[ih];
      sm.ex1[k] = (dxok && pv) ? (pg ? cscale(e1, (R)-1) : e1) : z;
      sm.er1[k] = px ? cscale(r1, hp) : z;
      sm.et1[k] = (px && pv) ? t1 : z;
      sm.bx1[k] = px ? cscale(bx, hs) : z;
      sm.br1[k] = (dxok && pv) ? br : z;
      sm.bt1[k] = dxok ? cscale(bt, hp) : z;
    }
  }
  for (int k = threadIdx.x; k < RL; k += WG) {
    const int j = q.R0 + k;
    sm.ivol[k] = (j >= 0 && j <= g.nr) ? inv_vol_node<R>(g, j) : (R)0;
  }
  if (SCAT != SCAT_NONE)
    for (int k = threadIdx.x; k < (SCAT == SCAT_CELL ? CRN : 9); k += WG) sm.ccell[k] = 0;
  __syncthreads();
  // grad Phi by centred differences on the primal nodes (zero radial
  // derivative on the axis, odd below it).  A scattering pass with quadratic
  // shapes stages it (the outermost ring of the region is unused); the
  // other gathers form it from the staged Phi (below).
  const R i2dx = (R)(0.5 / g.dx), i2dr = (R)(0.5 / g.dr);
  if constexpr (O == 2 && SCAT != SCAT_NONE) {
    for (int k = threadIdx.x; k < RN; k += WG) {
      const int a = k / RL, b = k - (k / RL) * RL;
      R vx = 0, vr = 0;
      if (a >= 1 && a <= RX - 2 && b >= 1 && b <= RL - 2) {
        vx = (sm.phi[k + RL] - sm.phi[k - RL]) * i2dx;
        if (q.R0 + b == -1)  // odd below the axis: minus the value on row 1
          vr = -((sm.phi[k + 3] - sm.phi[k + 1]) * i2dr);
        else if (q.R0 + b != 0)
          vr = (sm.phi[k + 1] - sm.phi[k - 1]) * i2dr;
      }
      sm.gx[k] = vx;
      sm.gr[k] = vr;
    }
  }

  // ---- destination (tile of the 3 x 3 neighbourhood, or cell) and rank
  // of each particle, kept in registers (the loops over a thread's
  // particles are unrolled).  Without the scatter only the live flag is kept.
  // An incremental tile sort ranks the particles that change tile only.
  const bool move = SCAT == SCAT_TILE && *Ld.mode == LAYOUT_MOVE;
  // a cell sort whose copy is gathered afterwards (k_permute)
  const bool gather = SCAT == SCAT_CELL && !DEFER && (*Ld.mode & LAYOUT_GATHER) != 0;
  // the particles of an item past the segments all join their tiles' segments
  const bool fill_item = start >= Ls.offsets[g.ntiles];
  constexpr int STAY = 1 << 30;  // slot_rank of a particle that keeps its slot
  int slot_rank[PPT];
  bool bad = false;
#pragma unroll
  for (int u = 0; u < PPT; ++u) {
    const int k = threadIdx.x + u * WG;
    slot_rank[u] = -1;
    int tslot = -1;  // SCAT_TILE: destination tile of the 3 x 3 neighbourhood
    if (k < count) {
      const unsigned cw = *elem(src.cell, start + k);
      if (cw != kDead) {
        if (SCAT == SCAT_TILE) {
          const int dtx = clampi(cell_ix(cw) / TX - q.T, -1, 1, bad);
          const int dtr = clampi(cell_jr(cw) / TR - q.tcr, -1, 1, bad);
          tslot = (dtx + 1) * 3 + (dtr + 1);
          if (move && tslot == 4 && !fill_item) {
            slot_rank[u] = STAY;
            tslot = -1;
          }
        } else if (SCAT == SCAT_CELL) {
          const int sx = clampi(cell_ix(cw) - (q.T * TX - SORT_EVERY), 0, CR - 1, bad);
          const int sr = clampi(cell_jr(cw) - (q.tcr * TR - SORT_EVERY), 0, CR - 1, bad);
          const int slot = sx * CR + sr;
          slot_rank[u] = (slot << 16) | atomicAdd(&sm.ccell[slot], 1);
        } else {
          slot_rank[u] = 0;
        }
      }
    }
    if (SCAT == SCAT_TILE) {  // the loop is wavefront-uniform (PPT iterations)
      const int r = wave_slot_rank(tslot, sm.ccell);
      if (tslot >= 0) slot_rank[u] = (tslot << 16) | r;
    }
  }
  __syncthreads();
  // one reservation per destination tile, or per destination cell (its
  // slots in cell order).  An incremental sort reserves arrival tickets and
  // keeps, per destination, where its free slots and overflow range start
  // and how many each holds.
  if (SCAT == SCAT_TILE) {
    if (threadIdx.x < 9) {
      const int c = sm.ccell[threadIdx.x];
      if (c > 0) {
        int tx2 = q.tcx + threadIdx.x / 3 - 1;
        if (tx2 < 0) tx2 += g.ntxa;
        if (tx2 >= g.ntxa) tx2 -= g.ntxa;
        const int tr2 = q.tcr + threadIdx.x % 3 - 1;
        const int key = tx2 * g.ntr + tr2;
        if (tr2 < 0 || tr2 >= g.ntr) {
          sm.ccell[threadIdx.x] = -1;  // no cell lies there: its particles are flagged, not written
        } else {
          sm.ccell[threadIdx.x] = atomicAdd(&Ld.cursor[key], c);
        }
        if (move && sm.ccell[threadIdx.x] >= 0) {
          int* pl = &sm.ccell[9 + 4 * threadIdx.x];
          pl[0] = Ls.offsets[key] + Ls.ext[key];
          pl[1] = Ld.ext[key] - Ls.ext[key];
          pl[2] = Ld.ovb[key];
          pl[3] = Ld.ovn[key];
        }
      }
    }
    __syncthreads();
  }
  if (SCAT == SCAT_CELL) {
    for (int k = threadIdx.x; k < CRN; k += WG) {
      const int c = sm.ccell[k];
      if (c > 0) {
        const int rel = (int)((long long)q.T * TX - SORT_EVERY + k / CR - g.shift);
        const int j = q.tcr * TR - SORT_EVERY + k % CR;
        sm.ccell[k] = atomicAdd(&ccur[(size_t)phys_col(g, rel) * g.pitch + j], c);
      }
    }
    __syncthreads();
  }

  // ---- gather, push, deposit, scatter
  bool lost = false;
#pragma unroll
  for (int u = 0; u < PPT; ++u) {
    if (slot_rank[u] < 0) continue;
    const int p = start + threadIdx.x + u * WG;
    const unsigned cw = pld<NT>(elem(src.cell, p));  // its second read (the first above)
    int d = p;
    const bool stay = SCAT == SCAT_TILE && slot_rank[u] == STAY;
    if (SCAT == SCAT_TILE && !stay) {
      const int sl = slot_rank[u] >> 16;
      if (sm.ccell[sl] < 0) {
        bad = true;
        continue;
      }
      const int tk = sm.ccell[sl] + (slot_rank[u] & 0xFFFF);
      d = tk;
      if (move) {
        // ticket tk of the destination: its free slots, then its overflow
        const int* pl = &sm.ccell[9 + 4 * sl];
        d = tk < pl[1] ? pl[0] + tk : (tk - pl[1] < pl[3] ? pl[2] + tk - pl[1] : -1);
        if (d < 0) {  // more arrivals than the scan counted: never written
          lost = true;
          continue;
        }
      }
      if ((long long)d >= g.cap) {  // the scan has flagged the overflow
        bad = true;
        continue;
      }
    }
    if (SCAT == SCAT_CELL) {
      // rank in the destination tile's cell order, then the transposed
      // placement inside its work item (as at loading)
      const int r = sm.ccell[slot_rank[u] >> 16] + (slot_rank[u] & 0xFFFF);
      const int key = tile_key(g, cell_ix(cw), cell_jr(cw));
      const int off = Ld.offsets[key], v = Ld.ext[key];
      if (r >= v) {  // counts and particles disagree: flagged, never written
        bad = true;
        continue;
      }
      d = off + placed_rank<O>(r, v, g.chunk);
      if ((long long)d >= g.cap) {  // the scan has flagged the overflow
        bad = true;
        continue;
      }
    }
    const R fx = pld<NT>(elem(src.fx, p)), fr = pld<NT>(elem(src.fr, p)), th = pld<NT>(elem(src.th, p)), w = pld<NT>(elem(src.w, p));
    R pv[3] = {pld<NT>(elem(src.px, p)), pld<NT>(elem(src.py, p)), pld<NT>(elem(src.pz, p))};
    // the cell relative to the region: [1, RX - 3] for the linear stencils
    // (and the differences of Phi one node further out); order 2 keeps
    // [2, RX - 4], the range its position pass needs for the current
    // stencil of the old and new cells
    const int a = O == 2 ? clampi(cell_ix(cw) - q.X0, 2, RX - 4, bad) : clampi(cell_ix(cw) - q.X0, 1, RX - 3, bad);
    const int b = O == 2 ? clampi(cell_jr(cw) - q.R0, 2, RL - 4, bad) : clampi(cell_jr(cw) - q.R0, 1, RL - 3, bad);
    R s, c;
    sincos_r(th, &s, &c);
    R ex, er, bt, et = 0, bx = 0, br = 0, ph, gx, gr;
    Lin<R> Px, Pr;
    Quad<R> Qx, Qr;
    if constexpr (O == 2) {
      Qx = quad_primal<R>(a, fx);
      Qr = quad_primal<R>(b, fr);
      const Quad<R> Ux = quad_dual<R>(a, fx), Ur = quad_dual<R>(b, fr);
      ex = interp3<R, RL>(sm.ex, Ux, Qr);
      er = interp3<R, RL>(sm.er, Qx, Ur);
      bt = interp3<R, RL>(sm.bt, Ux, Ur);
      if constexpr (SCAT != SCAT_NONE) {
        ph = interp3<R, RL>(sm.phi, Qx, Qr);
        gx = interp3<R, RL>(sm.gx, Qx, Qr);
        gr = interp3<R, RL>(sm.gr, Qx, Qr);
      } else {
        phi_grad3<R, RL>(sm.phi, Qx, Qr, q.R0 + Qr.i, i2dx, i2dr, ph, gx, gr);
      }
      if (M1) {
        ex += mode1_at<C, R>(interp3c<C, R, RL>(sm.ex1, Ux, Qr), c, s);
        er += mode1_at<C, R>(interp3c<C, R, RL>(sm.er1, Qx, Ur), c, s);
        et = mode1_at<C, R>(interp3c<C, R, RL>(sm.et1, Qx, Qr), c, s);
        bx = mode1_at<C, R>(interp3c<C, R, RL>(sm.bx1, Qx, Ur), c, s);
        br = mode1_at<C, R>(interp3c<C, R, RL>(sm.br1, Ux, Qr), c, s);
        bt += mode1_at<C, R>(interp3c<C, R, RL>(sm.bt1, Ux, Ur), c, s);
      }
    } else {
      Px = primal_w<R>(a, fx);
      Pr = primal_w<R>(b, fr);
      const Lin<R> Dx = dual_w<R>(a, fx), Dr = dual_w<R>(b, fr);
      ex = interp2<R, RL>(sm.ex, Dx, Pr);
      er = interp2<R, RL>(sm.er, Px, Dr);
      bt = interp2<R, RL>(sm.bt, Dx, Dr);
      // Phi on the 4 x 4 nodes around the cell (corners unused): itself on
      // the inner 2 x 2, its centred differences at those four nodes (the
      // radial one zero on the axis row)
      const R* pc = &sm.phi[a * RL + b];
      const R p00 = pc[0], p01 = pc[1], p10 = pc[RL], p11 = pc[RL + 1];
      ph = Px.a * (Pr.a * p00 + Pr.b * p01) + Px.b * (Pr.a * p10 + Pr.b * p11);
      const R gx00 = (p10 - pc[-RL]) * i2dx, gx01 = (p11 - pc[1 - RL]) * i2dx;
      const R gx10 = (pc[2 * RL] - p00) * i2dx, gx11 = (pc[2 * RL + 1] - p01) * i2dx;
      gx = Px.a * (Pr.a * gx00 + Pr.b * gx01) + Px.b * (Pr.a * gx10 + Pr.b * gx11);
      const bool axis = q.R0 + b == 0;
      const R gr00 = axis ? (R)0 : (p01 - pc[-1]) * i2dr, gr10 = axis ? (R)0 : (p11 - pc[RL - 1]) * i2dr;
      const R gr01 = (pc[2] - p00) * i2dr, gr11 = (pc[RL + 2] - p10) * i2dr;
      gr = Px.a * (Pr.a * gr00 + Pr.b * gr01) + Px.b * (Pr.a * gr10 + Pr.b * gr11);
      if (M1) {
        ex += mode1_at<C, R>(interp2c<C, R, RL>(sm.ex1, Dx, Pr), c, s);
        er += mode1_at<C, R>(interp2c<C, R, RL>(sm.er1, Px, Dr), c, s);
        et = mode1_at<C, R>(interp2c<C, R, RL>(sm.et1, Px, Pr), c, s);
        bx = mode1_at<C, R>(interp2c<C, R, RL>(sm.bx1, Px, Dr), c, s);
        br = mode1_at<C, R>(interp2c<C, R, RL>(sm.br1, Dx, Pr), c, s);
        bt += mode1_at<C, R>(interp2c<C, R, RL>(sm.bt1, Dx, Dr), c, s);
      }
    }
    // (x, r, theta) -> Cartesian, r-hat = (0, c, s), theta-hat = (0, -s, c)
    const R E[3] = {ex, er * c - et * s, er * s + et * c};
    const R B[3] = {bx, br * c - bt * s, br * s + bt * c};
    const R G[3] = {gx, gr * c, gr * s};
    // ponderomotive Boris: half kick with gbar(p^{n-1/2}), rotation and chi
    // with gbar of the half-kicked momentum, second half kick
    const R ig0 = (R)0.5 * rsqrt_r((R)1 + pv[0] * pv[0] + pv[1] * pv[1] + pv[2] * pv[2] + ph);
    R F[3], pm[3];
#pragma unroll
    for (int e = 0; e < 3; ++e) {
      F[e] = -E[e] - G[e] * ig0;
      pm[e] = pv[e] + hdt * F[e];
    }
    const R igb = rsqrt_r((R)1 + pm[0] * pm[0] + pm[1] * pm[1] + pm[2] * pm[2] + ph);
    const R tf = -hdt * igb;
    const R t[3] = {tf * B[0], tf * B[1], tf * B[2]};
    const R sf = (R)2 * rcp_r((R)1 + t[0] * t[0] + t[1] * t[1] + t[2] * t[2]);
    const R sv[3] = {sf * t[0], sf * t[1], sf * t[2]};
    const R pp[3] = {pm[0] + pm[1] * t[2] - pm[2] * t[1], pm[1] + pm[2] * t[0] - pm[0] * t[2],
                     pm[2] + pm[0] * t[1] - pm[1] * t[0]};
    pv[0] = pm[0] + pp[1] * sv[2] - pp[2] * sv[1] + hdt * F[0];
    pv[1] = pm[1] + pp[2] * sv[0] - pp[0] * sv[2] + hdt * F[1];
    pv[2] = pm[2] + pp[0] * sv[1] - pp[1] * sv[0] + hdt * F[2];
    if (DEFER) {
      gscr[d] = (R)1 / igb;
    } else if constexpr (O == 2) {
      // rows below the axis are folded onto their mirrors at the flush
      const R wg = w * igb * (R)Acc0<R>::scale(g);
#pragma unroll
      for (int aa = 0; aa < 3; ++aa) {
        const double wa = (double)(wg * Qx.w[aa]);
#pragma unroll
        for (int bb = 0; bb < 3; ++bb)
          Acc0<R>::add_prod(&sm.chi[(Qx.i + aa) * RL + Qr.i + bb], wa, (double)Qr.w[bb]);
      }
    } else {
      const R wg = w * igb * (R)Acc0<R>::scale(g);
#pragma unroll
      for (int aa = 0; aa < 2; ++aa) {
        const double wa = (double)(wg * (aa ? Px.b : Px.a));
#pragma unroll
        for (int bb = 0; bb < 2; ++bb)
          Acc0<R>::add_prod(&sm.chi[(Px.i + aa) * RL + Pr.i + bb], wa, (double)(bb ? Pr.b : Pr.a));
      }
    }
    if (gather) {
      // the cell-ordered copy is gathered afterwards (k_permute): p is
      // updated in place and the destination slot records where it comes from
      pst<NT>(elem(src.px, p), pv[0]);
      pst<NT>(elem(src.py, p), pv[1]);
      pst<NT>(elem(src.pz, p), pv[2]);
      *elem(inv, d) = (unsigned)p;
    } else if (SCAT != SCAT_NONE && !stay) {
      // an incremental sort writes within the same buffer, into slots no
      // work item of this pass reads (free or overflow slots)
      const Parts<R>& out = move ? src : dst;
      pst<NT>(elem(out.cell, d), cw);
      pst<NT>(elem(out.fx, d), fx);
      pst<NT>(elem(out.fr, d), fr);
      pst<NT>(elem(out.th, d), th);
      pst<NT>(elem(out.px, d), pv[0]);
      pst<NT>(elem(out.py, d), pv[1]);
      pst<NT>(elem(out.pz, d), pv[2]);
      pst<NT>(elem(out.w, d), w);
      pst<NT>(elem(out.id, d), pld<NT>(elem(src.id, p)));
      if (move && !fill_item) *elem(src.cell, p) = kDead;  // its old slot
    } else {
      pst<NT>(elem(src.px, p), pv[0]);
      pst<NT>(elem(src.py, p), pv[1]);
      pst<NT>(elem(src.pz, p), pv[2]);
    }
  }
  if (bad) atomicOr(err, ERR_HALO);
  if (lost) atomicOr(err, ERR_LAYOUT);
  if (DEFER) return;
  __syncthreads();
  for (int k = threadIdx.x; k < RN; k += WG) {
    const int a = k / RL, b = k - (k / RL) * RL;
    const int rel = q.relX0 + a, j = q.R0 + b;
    typename Acc0<R>::T v = sm.chi[k];
    // order 2: the row below the axis (two LDS rows down) belongs to row 1
    if (O == 2 && j == 1 && b >= 2) v += sm.chi[k - 2];
    if (!Acc0<R>::nonzero(v)) continue;
    if (rel < 0 || rel > g.nx || j < 0 || j > g.nr) continue;
    atomicAdd(&chi_out[(size_t)phys_col(g, rel) * g.pitch + j], (R)(Acc0<R>::val(v, g) * sm.ivol[b]));
  }
}

// ================================================== position pass ==
// A mode-1 accumulator grid of N nodes, real and imaginary words in
// separate arrays: one atomic instruction then touches words 8 bytes apart
// across the lanes' nodes, not 16 as with interleaved pairs, which halves the
// LDS bank conflicts of the deposit (measured: they took 40 % of the
// position pass's LDS cycles with pairs).
template <class R, int N> struct Acc1Grid {
  using T = typename Acc1<R>::T;
  typename Acc1<R>::S re[N], im[N];
  __device__ T operator[](int k) const {
    T v;
    v.x = re[k];
    v.y = im[k];
    return v;
  }
  __device__ void clear(int k) {
    re[k] = 0;
    im[k] = 0;
  }
};

template <class R, bool M1> struct SmemPos {
  using C = typename cplx_of<R>::type;
  R phh[LN];
  typename Acc0<R>::T jx[LN], jr[LN];
  Acc1Grid<R, M1 ? LN : 1> jx1, jr1, jt1;
  R iax[LR], iar[LR], ivn[LR], ivh[LR];
  int ccell[CRN];  // before a cell sort: particles per cell of x^{n+1}
  int tcnt[11];    // per-tile counts of the work item (flush_tiles)
};

// one particle's move: old and new cells/offsets, transverse displacement
// (radial a, azimuthal b, lengths) at the old azimuth, new azimuth, velocity
template <class R> struct Move {
  int ix0, jr0, ix1, jr1;
  R fx0, fr0, fx1, fr1;
  R th0, th1, a, b;
  R c0, s0;  // cos, sin of the old azimuth
  bool refl;
  R vx, vy, vz;
};

// The push x^{n+1} = x^n + dt v in Cartesian space, expressed on the cell
// representation; specular reflection at r_max (p updated).
template <class R>
__device__ inline void push_position(const Geo& g, unsigned cw, R fx, R fr, R th, R& py, R& pz, R vx, R vy, R vz,
                                     Move<R>& mv) {
  const R dt = (R)g.dt, dr = (R)g.dr;
  mv.ix0 = cell_ix(cw);
  mv.jr0 = cell_jr(cw);
  mv.fx0 = fx;
  mv.fr0 = fr;
  mv.th0 = th;
  mv.vx = vx;
  mv.vy = vy;
  mv.vz = vz;
  mv.ix1 = mv.ix0;
  mv.fx1 = fx + vx * (R)(g.dt / g.dx);
  carry(mv.ix1, mv.fx1);
  R s, c;
  sincos_r(th, &s, &c);
  mv.c0 = c;
  mv.s0 = s;
  const R dy = dt * vy, dz = dt * vz;
  mv.a = c * dy + s * dz;
  mv.b = -s * dy + c * dz;
  const R r = ((R)mv.jr0 + fr) * dr;
  R drad, dth;
  radial_step(r, mv.a, mv.b, drad, dth);
  mv.jr1 = mv.jr0;
  mv.fr1 = fr + drad * (R)(1.0 / g.dr);
  carry(mv.jr1, mv.fr1);
  if (mv.jr1 < 0) {
    mv.jr1 = 0;
    mv.fr1 = 0;
  }
  mv.th1 = wrap_angle(th + dth);
  mv.refl = false;
  if (mv.jr1 >= g.nr) {
    // r' = r_max + e with 0 <= e < dr  ->  r_max - e; reverse p_r
    const R e = (R)(mv.jr1 - g.nr) + mv.fr1;
    mv.jr1 = g.nr - 1;
    mv.fr1 = (R)1 - e;
    if (mv.fr1 < (R)0) mv.fr1 = 0;
    R s1, c1;
    sincos_r(mv.th1, &s1, &c1);
    const R prad = py * c1 + pz * s1;
    py -= (R)2 * prad * c1;
    pz -= (R)2 * prad * s1;
    mv.refl = true;
  }
}

// Esirkepov current of one particle between two positions (mode 0) and the
// direct mid-point current of mode 1, into the LDS accumulators.
template <class R, bool M1>
__device__ inline void deposit_current(SmemPos<R, M1>& sm, const Region& q, const Geo& g, const Move<R>& mv, R w,
                                       bool& bad) {
  // the stencil spans min(a0, a1) .. min(a0, a1) + 2: the push moves a
  // particle less than a cell (dt < dx and dt < dr, checked at init), so the
  // new cell is the old one's neighbour or itself; that step, bounded to one
  // cell, keeps every index inside the region once the old cell is
  const int a0 = clampi(mv.ix0 - q.X0, 1, LX - 4, bad);
  const int a1 = a0 + min(max(mv.ix1 - mv.ix0, -1), 1);
  const int b0 = clampi(mv.jr0 - q.R0, 1, LR - 4, bad);
  const int b1 = b0 + min(max(mv.jr1 - mv.jr0, -1), 1);
  // node weights on the 3-node union of the old and new supports, without
  // indexing into register arrays: d = a1 - a0 in {-1, 0, 1}
  const int dxs = a1 - a0, drs = b1 - b0;
  const int amin = a0 + min(dxs, 0), bmin = b0 + min(drs, 0);
  const R u0 = (R)1 - mv.fx0, u1 = (R)1 - mv.fx1, v0 = (R)1 - mv.fr0, v1 = (R)1 - mv.fr1;
  const R S0x[3] = {dxs >= 0 ? u0 : (R)0, dxs >= 0 ? mv.fx0 : u0, dxs >= 0 ? (R)0 : mv.fx0};
  const R S1x[3] = {dxs <= 0 ? u1 : (R)0, dxs <= 0 ? mv.fx1 : u1, dxs <= 0 ? (R)0 : mv.fx1};
  const R S0r[3] = {drs >= 0 ? v0 : (R)0, drs >= 0 ? mv.fr0 : v0, drs >= 0 ? (R)0 : mv.fr0};
  const R S1r[3] = {drs <= 0 ? v1 : (R)0, drs <= 0 ? mv.fr1 : v1, drs <= 0 ? (R)0 : mv.fr1};
  // J_x (i+1/2, j): flux accumulated along x; the third partial sum is zero
  const R cx0 = S1x[0] - S0x[0], cx1 = cx0 + S1x[1] - S0x[1];
  const R cr0 = S1r[0] - S0r[0], cr1 = cr0 + S1r[1] - S0r[1];
  // (the face areas are applied at the flush)
  using A0 = Acc0<R>;
  typename A0::T* jx = &sm.jx[amin * LR + bmin];
  typename A0::T* jr = &sm.jr[amin * LR + bmin];
  const double hw = 0.5 * (double)w * A0::scale(g);
  const double cx0d = cx0, cx1d = cx1, cr0d = cr0, cr1d = cr1;
  // the second partial sum is non-zero only when the particle changed
  // column (row); a zero first one adds nothing
#pragma unroll
  for (int bb = 0; bb < 3; ++bb) {
    const double sr = (double)(S0r[bb] + S1r[bb]) * hw;
    A0::add_prod(&jx[bb], cx0d, sr);
    if (dxs != 0) A0::add_prod(&jx[LR + bb], cx1d, sr);
  }
  // J_r (i, j+1/2): flux accumulated along r
#pragma unroll
  for (int aa = 0; aa < 3; ++aa) {
    const double sx = (double)(S0x[aa] + S1x[aa]) * hw;
    A0::add_prod(&jr[aa * LR], cr0d, sx);
    if (drs != 0) A0::add_prod(&jr[aa * LR + 1], cr1d, sx);
  }
  if (M1) {
    // Cartesian mid-point of the old and new positions: in the frame of the
    // old azimuth it sits at (r0 + a/2, b/2); its radius and direction follow
    // without trigonometric calls
    const R dr = (R)g.dr;
    const R r0 = ((R)mv.jr0 + mv.fr0) * dr;
    int jm = mv.jr0;
    R frm, c, s;
    if (!mv.refl) {
      const R u = r0 + (R)0.5 * mv.a, v = (R)0.5 * mv.b;
      R cd, sd;
      if (u > (R)0) {
        const R beta = v * rcp_r(u);
        const R q2b = (R)1 + beta * beta;
        cd = rsqrt_r(q2b);  // 1 / sqrt(1 + beta^2)
        const R qq = q2b * cd;
        frm = mv.fr0 + ((R)0.5 * mv.a + u * beta * beta * rcp_r((R)1 + qq)) * (R)(1.0 / g.dr);
        sd = beta * cd;
      } else {
        const R rm = sqrt_r(u * u + v * v);
        frm = mv.fr0 + (rm - r0) / dr;
        cd = rm > (R)0 ? u / rm : (R)1;
        sd = rm > (R)0 ? v / rm : (R)0;
      }
      c = mv.c0 * cd - mv.s0 * sd;
      s = mv.s0 * cd + mv.c0 * sd;
    } else {
      R s1, c1;
      sincos_r(mv.th1, &s1, &c1);
      const R r1 = ((R)mv.jr1 + mv.fr1) * dr;
      const R ym = (R)0.5 * (r0 * mv.c0 + r1 * c1), zm = (R)0.5 * (r0 * mv.s0 + r1 * s1);
      const R rm = sqrt_r(ym * ym + zm * zm);
      jm = 0;
      frm = rm / dr;
      c = rm > (R)0 ? ym / rm : (R)1;
      s = rm > (R)0 ? zm / rm : (R)0;
    }
    carry(jm, frm);
    if (jm < 0) {
      jm = 0;
      frm = 0;
    }
    if (jm > g.nr - 1) {
      frm += (R)(jm - (g.nr - 1));
      jm = g.nr - 1;
    }
    const R um = (R)0.5 * ((R)a0 + mv.fx0 + (R)a1 + mv.fx1);
    const int am = (int)floor(um);
    const R fm = um - (R)am;
    const int bm = clampi(jm - q.R0, 1, LR - 3, bad);
    const int amc = clampi(am, 1, LX - 3, bad);
    const Lin<R> Px = primal_w<R>(amc, fm), Dx = dual_w<R>(amc, fm);
    const Lin<R> Pr = primal_w<R>(bm, frm), Dr = dual_w<R>(bm, frm);
    // 2 q w v e^{i theta} per component (electrons, q = -1), with the
    // accumulator scale folded in; radial weights times inverse volumes
    const R q2 = (R)-2 * w * Acc1<R>::scale(g);
    const R vx = q2 * mv.vx, vr = q2 * (mv.vy * c + mv.vz * s), vt = q2 * (mv.vz * c - mv.vy * s);
    const double xc = vx * c, xs = vx * s, rc = vr * c, rs = vr * s, tc = vt * c, ts = vt * s;
    const R pv[2] = {Pr.a * sm.ivn[Pr.i], Pr.b * sm.ivn[Pr.i + 1]};
    // J_r1 rows; row -1/2 folds onto +1/2 (even for mode 1)
    const int dn0 = (q.R0 + Dr.i == -1) ? Dr.i + 1 : Dr.i, dn1 = Dr.i + 1;
    const R dv[2] = {Dr.a * sm.ivh[dn0], Dr.b * sm.ivh[dn1]};
    const int dn[2] = {dn0, dn1};
#pragma unroll
    for (int aa = 0; aa < 2; ++aa) {
      const R wdx = aa ? Dx.b : Dx.a, wpx = aa ? Px.b : Px.a;
#pragma unroll
      for (int bb = 0; bb < 2; ++bb) {
        const double ux = wdx * pv[bb], ur = wpx * dv[bb], ut = wpx * pv[bb];
        Acc1<R>::add_prod(sm.jx1, (Dx.i + aa) * LR + Pr.i + bb, ux, xc, xs);  // (i+1/2, j)
        Acc1<R>::add_prod(sm.jr1, (Px.i + aa) * LR + dn[bb], ur, rc, rs);     // (i, j+1/2)
        Acc1<R>::add_prod(sm.jt1, (Px.i + aa) * LR + Pr.i + bb, ut, tc, ts);  // (i, j)
      }
    }
  }
}

// Order-2 currents: the Esirkepov decomposition of the change between the
// old and new quadratic stencils on their 4-node union (mode 0), and the
// quadratic mid-point deposit of mode 1.  Contributions to the rows below
// the axis stay in the LDS ghost rows and are folded at the flush, except
// the mode-1 J_r of the half row -1/2, which lands on +1/2 directly (even).
template <class R, bool M1>
__device__ inline void deposit_current2(SmemPos<R, M1>& sm, const Region& q, const Geo& g, const Move<R>& mv, R w,
                                        bool& bad) {
  const int a0 = clampi(mv.ix0 - q.X0, 2, LX - 4, bad);
  const int a1 = a0 + min(max(mv.ix1 - mv.ix0, -1), 1);  // (a step of at most one cell, as above)
  const int b0 = clampi(mv.jr0 - q.R0, 2, LR - 4, bad);
  const int b1 = b0 + min(max(mv.jr1 - mv.jr0, -1), 1);
  const Quad<R> X0 = quad_primal<R>(a0, mv.fx0), X1 = quad_primal<R>(a1, mv.fx1);
  const Quad<R> Y0 = quad_primal<R>(b0, mv.fr0), Y1 = quad_primal<R>(b1, mv.fr1);
  // nearest nodes move by at most one (less than a cell per step)
  const int ax = min(X0.i, X1.i), by = min(Y0.i, Y1.i);
  const int ox0 = clampi(X0.i - ax, 0, 1, bad), ox1 = clampi(X1.i - ax, 0, 1, bad);
  const int or0 = clampi(Y0.i - by, 0, 1, bad), or1 = clampi(Y1.i - by, 0, 1, bad);
  // the stencils on the union (placed without indexing register arrays)
  auto place = [](const Quad<R>& Q, int o, R* S) {
    S[0] = o ? (R)0 : Q.w[0];
    S[1] = o ? Q.w[0] : Q.w[1];
    S[2] = o ? Q.w[1] : Q.w[2];
    S[3] = o ? Q.w[2] : (R)0;
  };
  R S0x[4], S1x[4], S0r[4], S1r[4];
  place(X0, ox0, S0x);
  place(X1, ox1, S1x);
  place(Y0, or0, S0r);
  place(Y1, or1, S1r);
  // partial sums of the change from the low side (the fourth is zero)
  R cx[3], cr[3];
  cx[0] = S1x[0] - S0x[0];
  cr[0] = S1r[0] - S0r[0];
#pragma unroll
  for (int k = 1; k < 3; ++k) {
    cx[k] = cx[k - 1] + (S1x[k] - S0x[k]);
    cr[k] = cr[k - 1] + (S1r[k] - S0r[k]);
  }
  using A0 = Acc0<R>;
  typename A0::T* jx = &sm.jx[ax * LR + by];
  typename A0::T* jr = &sm.jr[ax * LR + by];
  const double hw = 0.5 * (double)w * A0::scale(g);
#pragma unroll
  for (int bb = 0; bb < 4; ++bb) {
    const double sr = (double)(S0r[bb] + S1r[bb]) * hw;
#pragma unroll
    for (int aa = 0; aa < 3; ++aa)
      if (cx[aa] != (R)0) A0::add_prod(&jx[aa * LR + bb], (double)cx[aa], sr);
  }
#pragma unroll
  for (int aa = 0; aa < 4; ++aa) {
    const double sx = (double)(S0x[aa] + S1x[aa]) * hw;
#pragma unroll
    for (int bb = 0; bb < 3; ++bb)
      if (cr[bb] != (R)0) A0::add_prod(&jr[aa * LR + bb], (double)cr[bb], sx);
  }
  if (M1) {
    // mid-point as in the linear deposit
    const R dr = (R)g.dr;
    const R r0 = ((R)mv.jr0 + mv.fr0) * dr;
    int jm = mv.jr0;
    R frm, c, s;
    if (!mv.refl) {
      const R u = r0 + (R)0.5 * mv.a, v = (R)0.5 * mv.b;
      R cd, sd;
      if (u > (R)0) {
        const R beta = v * rcp_r(u);
        const R q2b = (R)1 + beta * beta;
        cd = rsqrt_r(q2b);  // 1 / sqrt(1 + beta^2)
        const R qq = q2b * cd;
        frm = mv.fr0 + ((R)0.5 * mv.a + u * beta * beta * rcp_r((R)1 + qq)) * (R)(1.0 / g.dr);
        sd = beta * cd;
      } else {
        const R rm = sqrt_r(u * u + v * v);
        frm = mv.fr0 + (rm - r0) / dr;
        cd = rm > (R)0 ? u / rm : (R)1;
        sd = rm > (R)0 ? v / rm : (R)0;
      }
      c = mv.c0 * cd - mv.s0 * sd;
      s = mv.s0 * cd + mv.c0 * sd;
    } else {
      R s1, c1;
      sincos_r(mv.th1, &s1, &c1);
      const R r1 = ((R)mv.jr1 + mv.fr1) * dr;
      const R ym = (R)0.5 * (r0 * mv.c0 + r1 * c1), zm = (R)0.5 * (r0 * mv.s0 + r1 * s1);
      const R rm = sqrt_r(ym * ym + zm * zm);
      jm = 0;
      frm = rm / dr;
      c = rm > (R)0 ? ym / rm : (R)1;
      s = rm > (R)0 ? zm / rm : (R)0;
    }
    carry(jm, frm);
    if (jm < 0) {
      jm = 0;
      frm = 0;
    }
    if (jm > g.nr - 1) {
      frm += (R)(jm - (g.nr - 1));
      jm = g.nr - 1;
    }
    const R um = (R)0.5 * ((R)a0 + mv.fx0 + (R)a1 + mv.fx1);
    const int am = (int)floor(um);
    const R fm = um - (R)am;
    const int bm = clampi(jm - q.R0, 1, LR - 3, bad);
    const int amc = clampi(am, 1, LX - 3, bad);
    const Quad<R> Qx = quad_primal<R>(amc, fm), Ux = quad_dual<R>(amc, fm);
    const Quad<R> Qr = quad_primal<R>(bm, frm), Ur = quad_dual<R>(bm, frm);
    const R q2 = (R)-2 * w * Acc1<R>::scale(g);
    const R vx = q2 * mv.vx, vr = q2 * (mv.vy * c + mv.vz * s), vt = q2 * (mv.vz * c - mv.vy * s);
    const double xc = vx * c, xs = vx * s, rc = vr * c, rs = vr * s, tc = vt * c, ts = vt * s;
    // radial weights times the inverse volume of the row they land on (the
    // primal ghost row carries row 1's); the half row -1/2 is row +1/2
    R pv[3], dv[3];
    int dn[3];
#pragma unroll
    for (int bb = 0; bb < 3; ++bb) {
      pv[bb] = Qr.w[bb] * sm.ivn[Qr.i + bb];
      dn[bb] = (q.R0 + Ur.i + bb == -1) ? Ur.i + bb + 1 : Ur.i + bb;
      dv[bb] = Ur.w[bb] * sm.ivh[dn[bb]];
    }
    // each radial factor times the velocity's cosine and sine parts in FP64,
    // then one FMA per word with the axial weight (converted once per node)
#pragma unroll
    for (int bb = 0; bb < 3; ++bb) {
      const double p = pv[bb], d = dv[bb];
      const double pxc = p * xc, pxs = p * xs, drc = d * rc, drs = d * rs, ptc = p * tc, pts = p * ts;
#pragma unroll
      for (int aa = 0; aa < 3; ++aa) {
        const double ux = Ux.w[aa], qx = Qx.w[aa];
        Acc1<R>::add_prod(sm.jx1, (Ux.i + aa) * LR + Qr.i + bb, ux, pxc, pxs);  // (i+1/2, j)
        Acc1<R>::add_prod(sm.jr1, (Qx.i + aa) * LR + dn[bb], qx, drc, drs);     // (i, j+1/2)
        Acc1<R>::add_prod(sm.jt1, (Qx.i + aa) * LR + Qr.i + bb, qx, ptc, pts);  // (i, j)
      }
    }
  }
}

template <class R, bool M1>
__device__ inline void stage_pos_constants(SmemPos<R, M1>& sm, const Region& q, const Geo& g) {
  const double pi = 3.14159265358979323846;
  for (int k = threadIdx.x; k < LR; k += WG) {
    const int j = q.R0 + k;
    // 1 / (face area * dt): axial face of row j (V_j / dx), radial face at r_{j+1/2}
    double ax = (j == 0 ? pi * g.dr * g.dr * 0.25 : 2.0 * pi * j * g.dr * g.dr);
    double ar = 2.0 * pi * (j + 0.5) * g.dr * g.dx;
    sm.iax[k] = (j >= 0 && j <= g.nr) ? (R)(1.0 / (ax * g.dt)) : (R)0;
    sm.iar[k] = (j >= 0 && j <= g.nr - 1) ? (R)(1.0 / (ar * g.dt)) : (R)0;
    // the primal ghost row j = -1 carries the volume of row 1, onto which
    // its (order-2) deposits are folded
    sm.ivn[k] = (j >= 0 && j <= g.nr) ? inv_vol_node<R>(g, j) : (j == -1 ? inv_vol_node<R>(g, 1) : (R)0);
    sm.ivh[k] = (j >= 0 && j <= g.nr - 1) ? inv_vol_half<R>(g, j) : (R)0;
  }
}

template <class R, bool M1>
__device__ inline void zero_pos_acc(SmemPos<R, M1>& sm) {
  for (int k = threadIdx.x; k < LN; k += WG) {
    sm.jx[k] = 0;
    sm.jr[k] = 0;
    if (M1) {
      sm.jx1.clear(k);
      sm.jr1.clear(k);
      sm.jt1.clear(k);
    }
  }
  for (int k = threadIdx.x; k < CRN; k += WG) sm.ccell[k] = 0;
  if (threadIdx.x < 11) sm.tcnt[threadIdx.x] = 0;
}

// a + sg b of two mode-1 accumulator words (exact for the fixed point, whose
// words add modulo 2^64)
template <class T> __device__ inline T acc_axpy(T a, const T& b, int sg) {
  a.x += sg * b.x;
  a.y += sg * b.y;
  return a;
}

// O = 2: the deposits on the rows below the axis are folded onto their
// mirrors with the component's parity (R23): J_x row -1 onto row 1 (even for
// mode 0, odd for mode 1), J_r face -1/2 onto +1/2 (odd for mode 0), mode-1
// J_theta row -1 onto row 1 (even).
template <class R, bool M1, int O>
__device__ inline void flush_current(SmemPos<R, M1>& sm, const Region& q, const Geo& g, R* jx_out,
                                     R* jr_out, typename cplx_of<R>::type* jx1_out,
                                     typename cplx_of<R>::type* jr1_out,
                                     typename cplx_of<R>::type* jt1_out) {
  for (int k = threadIdx.x; k < LN; k += WG) {
    const int a = k / LR, b = k - (k / LR) * LR;
    const int rel = q.relX0 + a, j = q.R0 + b;
    if (rel < 0 || rel > g.nx || j < 0 || j > g.nr) continue;
    const size_t o = (size_t)phys_col(g, rel) * g.pitch + j;
    const bool dxok = rel <= g.nx - 1, drok = j <= g.nr - 1;
    if constexpr (O == 2) {
      const bool fold_row = j == 1 && b >= 2, fold_face = j == 0 && b >= 1;
      typename Acc0<R>::T vjx = sm.jx[k], vjr = sm.jr[k];
      if (fold_row) vjx += sm.jx[k - 2];
      if (fold_face) vjr -= sm.jr[k - 1];
      if (dxok && Acc0<R>::nonzero(vjx)) atomicAdd(&jx_out[o], (R)(Acc0<R>::val(vjx, g) * sm.iax[b]));
      if (drok && Acc0<R>::nonzero(vjr)) atomicAdd(&jr_out[o], (R)(Acc0<R>::val(vjr, g) * sm.iar[b]));
      if (M1) {
        using A = Acc1<R>;
        typename A::T v1x = sm.jx1[k], v1t = sm.jt1[k];
        if (fold_row) {
          v1x = acc_axpy(v1x, sm.jx1[k - 2], -1);
          v1t = acc_axpy(v1t, sm.jt1[k - 2], 1);
        }
        if (dxok && A::nonzero(v1x)) {
          atomicAdd(&jx1_out[o].x, (R)A::re(v1x, g));
          atomicAdd(&jx1_out[o].y, (R)A::im(v1x, g));
        }
        if (drok && A::nonzero(sm.jr1[k])) {
          atomicAdd(&jr1_out[o].x, (R)A::re(sm.jr1[k], g));
          atomicAdd(&jr1_out[o].y, (R)A::im(sm.jr1[k], g));
        }
        if (A::nonzero(v1t)) {
          atomicAdd(&jt1_out[o].x, (R)A::re(v1t, g));
          atomicAdd(&jt1_out[o].y, (R)A::im(v1t, g));
        }
      }
    } else {
      if (dxok && Acc0<R>::nonzero(sm.jx[k])) atomicAdd(&jx_out[o], (R)(Acc0<R>::val(sm.jx[k], g) * sm.iax[b]));
      if (drok && Acc0<R>::nonzero(sm.jr[k])) atomicAdd(&jr_out[o], (R)(Acc0<R>::val(sm.jr[k], g) * sm.iar[b]));
      if (M1) {
        using A = Acc1<R>;
        if (dxok && A::nonzero(sm.jx1[k])) {
          atomicAdd(&jx1_out[o].x, (R)A::re(sm.jx1[k], g));
          atomicAdd(&jx1_out[o].y, (R)A::im(sm.jx1[k], g));
        }
        if (drok && A::nonzero(sm.jr1[k])) {
          atomicAdd(&jr1_out[o].x, (R)A::re(sm.jr1[k], g));
          atomicAdd(&jr1_out[o].y, (R)A::im(sm.jr1[k], g));
        }
        if (A::nonzero(sm.jt1[k])) {
          atomicAdd(&jt1_out[o].x, (R)A::re(sm.jt1[k], g));
          atomicAdd(&jt1_out[o].y, (R)A::im(sm.jt1[k], g));
        }
      }
    }
  }
}

// the per-cell counts of a work item into the global per-cell counts
__device__ inline void flush_cells(const int* cc, const Region& q, const Geo& g, int* ccount) {
  for (int k = threadIdx.x; k < CRN; k += WG) {
    const int c = cc[k];
    if (c > 0) {
      const int rel = (int)((long long)q.T * TX - SORT_EVERY + k / CR - g.shift);
      const int j = q.tcr * TR - SORT_EVERY + k % CR;
      atomicAdd(&ccount[(size_t)phys_col(g, rel) * g.pitch + j], c);
    }
  }
}

// The per-tile counts of a work item, t[d] for d = 3 (dx + 1) + (dr + 1)
// the particles that moved to the neighbouring tile (dx, dr) (counted
// before a tile sort), t[9] the particles removed, t[10] the live ones at
// the start of a fill item.  hist (particles per tile, kept current from
// step to step) loses the removed and moved ones and gains the moved ones
// at their new tiles; before a tile sort, arr gains the moved ones, and
// every particle of a fill item that stays in its tile.
__device__ inline void flush_tiles(const int* t, const Region& q, const Geo& g, const SortCounts& sc, bool fill_item) {
  if (threadIdx.x >= 9) return;
  const int d = threadIdx.x;
  int v = t[d];
  if (d == 4) {
    int moved = 0;
    for (int e = 0; e < 9; ++e) moved += e == 4 ? 0 : t[e];
    const int key = q.tcx * g.ntr + q.tcr;
    if (t[9] + moved != 0) atomicAdd(&sc.hist[key], -(t[9] + moved));
    if (sc.mode == SCAT_TILE && fill_item) {
      const int stay = t[10] - t[9] - moved;
      if (stay != 0) atomicAdd(&sc.arr[key], stay);
    }
    return;
  }
  if (v == 0) return;
  int tx = q.tcx + d / 3 - 1;
  if (tx < 0) tx += g.ntxa;
  if (tx >= g.ntxa) tx -= g.ntxa;
  const int tr = q.tcr + d % 3 - 1;
  if (tr < 0 || tr >= g.ntr) return;  // (no cell lies there)
  atomicAdd(&sc.hist[tx * g.ntr + tr], v);
  atomicAdd(&sc.arr[tx * g.ntr + tr], v);
}

// ============================================== loading / injection ==
// Plasma of lab cell column `col`, radial cell j: regular in x and r, one
// SplitMix64 angle per cell with equally spaced angles inside the cell,
// weights n 2 pi r (dr/N_r)(dx/N_x)/N_theta.  Particle k of the cell is
// stored at base + transpose_rank(r0 + k, n_range).  Returns 1 if live.
template <class R>
__device__ inline int load_particle(const Geo& g, const Plasma& pl, Parts<R> P, int base, int r0, int n_range,
                                    long long col, int j, int k) {
  const double pi = 3.14159265358979323846;
  const int ppc = g.ppc_x * g.ppc_r * g.ppc_t;
  const int t = k % g.ppc_t, b = (k / g.ppc_t) % g.ppc_r, a = k / (g.ppc_t * g.ppc_r);
  const double fx = (a + 0.5) / g.ppc_x, fr = (b + 0.5) / g.ppc_r;
  const double xl = ((double)col + fx) * g.dx;
  const double r = (j + fr) * g.dr;
  const double n = plasma_density(pl, xl, col, j);
  const int s = base + transpose_rank(r0 + k, n_range);
  P.px[s] = 0;
  P.py[s] = 0;
  P.pz[s] = 0;
  P.id[s] = (uint32_t)(col * (long long)g.nr * ppc + (long long)j * ppc + k);
  if (!(n > 0.0)) {
    P.cell[s] = kDead;
    P.fx[s] = 0;
    P.fr[s] = 0;
    P.th[s] = 0;
    P.w[s] = 0;
    return 0;
  }
  const double th0 = 2.0 * pi * counter_uniform(pl.seed, STREAM_ANGLE, col, j);
  double th = th0 + 2.0 * pi * t / g.ppc_t;  // in [0, 4 pi): fold into (-pi, pi]
  if (th > pi) th -= 2.0 * pi;
  if (th > pi) th -= 2.0 * pi;
  P.cell[s] = pack_cell((int)col, j);
  P.fx[s] = (R)fx;
  P.fr[s] = (R)fr;
  P.th[s] = (R)th;
  P.w[s] = (R)(n * 2.0 * pi * r * (g.dr / g.ppc_r) * (g.dx / g.ppc_x) / g.ppc_t);
  return 1;
}

// One work group (WG threads, group index blk) of the injection: the
// plasma of lab column gn.shift + nx - 1, tile by tile, with one work item
// per tile.  A row tile goes to the end of its tile's segment when the free
// slots hold it, else past the used slots (after the row tiles before it
// that went there); every group of the injection finds the same placement
// (the layout does not change during the pass).  s_cnt holds WG + 1 ints,
// s_base ntr + 1.  The field stage adds the items to the layout (and their
// slots to the segments or the fill pointer).
template <class R>
__device__ void inject_block(const InjectArgs& ia, Parts<R> P, const Layout& L, const SortCounts& sc, int* err,
                             int blk, int* s_cnt, int* s_base) {
  const Geo& g = ia.gn;
  const long long col = g.shift + g.nx - 1;
  const int ppc = g.ppc_x * g.ppc_r * g.ppc_t;
  const int total = *L.fill;  // end of the used slots
  const int base_items = *L.n_items;
  const int seg_end = L.offsets[g.ntiles];
  if ((long long)total + (long long)g.nr * ppc > ia.capacity || base_items + g.ntr > ia.max_items || col > COL_MAX) {
    if (blk == 0 && threadIdx.x == 0) atomicOr(err, ERR_CAPACITY);
    return;
  }
  // first slot of each row tile: its segment's end (>= 0) or, for now, the
  // negated slot count of a row tile that goes past the used slots
  for (int t = threadIdx.x; t < g.ntr; t += WG) {
    const int key = tile_key(g, col, t * TR), n = min(TR, g.nr - t * TR) * ppc;
    const int off = L.offsets[key], e = L.ext[key];
    s_base[t] = e + n <= L.offsets[key + 1] - off ? off + e : -n;
  }
  for (int k = threadIdx.x; k < WG + 1; k += WG) s_cnt[k] = 0;
  __syncthreads();
  if (threadIdx.x == 0) {
    int fill = total;
    for (int t = 0; t < g.ntr; ++t)
      if (s_base[t] < 0) {
        const int n = -s_base[t];
        s_base[t] = fill;
        fill += n;
      }
    s_base[g.ntr] = fill - total;  // slots past the used ones
  }
  __syncthreads();
  // live particles per cell (one cell = ppc consecutive threads), counted in
  // LDS first: a group spans WG / ppc + 1 rows at most
  const int idx = blk * WG + threadIdx.x;
  const int j_first = (blk * WG) / ppc;
  if (idx < g.nr * ppc) {
    const int j = idx / ppc, k = idx - (idx / ppc) * ppc;
    const int t = j / TR, trt = min(TR, g.nr - t * TR);
    if (load_particle<R>(g, ia.pl, P, s_base[t], (j - t * TR) * ppc, trt * ppc, col, j, k))
      atomicAdd(&s_cnt[j - j_first], 1);
  }
  __syncthreads();
  if (sc.mode == SCAT_CELL) {
    const int pc = phys_col(g, g.nx - 1);
    for (int k = threadIdx.x; k < WG + 1; k += WG)
      if (s_cnt[k] > 0 && j_first + k < g.nr) atomicAdd(&sc.ccount[(size_t)pc * g.pitch + j_first + k], s_cnt[k]);
  }
  // the particles per tile, kept current; before a tile sort the particles
  // of a row tile placed past the segments also arrive in their tile's
  // segment
  for (int k = threadIdx.x; k < WG + 1; k += WG)
    if (s_cnt[k] > 0 && j_first + k < g.nr) {
      const int j = j_first + k;
      const int key = tile_key(g, col, j);
      atomicAdd(&sc.hist[key], s_cnt[k]);
      if (sc.mode == SCAT_TILE && s_base[j / TR] >= seg_end) atomicAdd(&sc.arr[key], s_cnt[k]);
    }
  if (idx < g.ntr) {
    const int trt = min(TR, g.nr - idx * TR);
    L.items[base_items + idx] = make_int4(tile_key(g, col, idx * TR), s_base[idx], trt * ppc, 0);
  }
  if (idx == 0) {
    ia.pending[0] = g.ntr;           // items appended
    ia.pending[1] = s_base[g.ntr];   // slots appended past the used ones
  }
}

// vacate: 1 when the window moves after this step (particles whose new
// column is the window's first one are dropped after depositing); sc: what
// to count for a sort at the next step (SortCounts)
// The FP32 quadratic pass is held to six waves per SIMD (80 registers per
// lane, the count the LDS allows), at the price of 12 bytes of spills per
// lane.
template <class R, int O> constexpr int pos_waves_per_simd() { return (sizeof(R) == 4 && O == 2) ? 6 : 1; }

template <class R, bool M1, bool DEFER, int O, bool NT>
__global__ __launch_bounds__(WG, (pos_waves_per_simd<R, O>())) void k_position(Geo g, Grids<R> f, R* __restrict__ jx_out,
                                                 R* __restrict__ jr_out,
                                                 typename cplx_of<R>::type* __restrict__ jx1_out,
                                                 typename cplx_of<R>::type* __restrict__ jr1_out,
                                                 typename cplx_of<R>::type* __restrict__ jt1_out,
                                                 Parts<R> P, Layout L, SortCounts sc, int vacate,
                                                 Parts<R> scr, int* err, int item_blocks,
                                                 InjectArgs inj) {
  __shared__ SmemPos<R, M1> sm;
  if ((int)blockIdx.x >= item_blocks) {
    // the phi staging area and the J_x accumulators are free in these
    // groups: they hold the row counts and the row tiles' first slots
    static_assert(sizeof(sm.phh) >= (WG + 1) * sizeof(int), "row counts do not fit");
    static_assert(sizeof(sm.jx) >= (NR_MAX / TR + 2) * sizeof(int), "row tile slots do not fit");
    inject_block<R>(inj, P, L, sc, err, blockIdx.x - item_blocks, reinterpret_cast<int*>(sm.phh),
                    reinterpret_cast<int*>(sm.jx));
    return;
  }
  const int item = item_of(blockIdx.x, item_blocks);
  if (item >= *L.n_items) return;
  const int4 it = L.items[item];
  const int start = it.y, count = it.z;
  const Region q = region_of(g, it.x);

  // Phi^{n+1/2} = (|A^{n+1}|^2 + |A^n|^2)/4 on the primal nodes (order 2:
  // the ghost row j = -1 mirrors row 1, even)
  for (int k = threadIdx.x; k < LN; k += WG) {
    const int a = k / LR, b = k - (k / LR) * LR;
    const int rel = q.relX0 + a, j0 = q.R0 + b;
    const int j = (O == 2 && j0 == -1) ? 1 : j0;
    R v = 0;
    if (rel >= 0 && rel <= g.nx && j >= 0 && j <= g.nr) {
      const size_t o = (size_t)phys_col(g, rel) * g.pitch + j;
      v = (R)0.25 * (cnorm(f.env[o]) + cnorm(f.envp[o]));
    }
    sm.phh[k] = v;
  }
  stage_pos_constants(sm, q, g);
  zero_pos_acc(sm);
  __syncthreads();
  // Before a tile sort, the particles of an item past the tiles' segments
  // (an injected column, an overflow range) all join their tiles'
  // segments: their live count, taken before the pass removes any
  const bool fill_item = start >= L.offsets[g.ntiles];
  if (sc.mode == SCAT_TILE && fill_item) {
    int c = 0;
    for (int k = threadIdx.x; k < count; k += WG) c += P.cell[start + k] != kDead ? 1 : 0;
    c = wave_sum_i(c);
    if (__lane_id() == 0 && c != 0) atomicAdd(&sm.tcnt[10], c);
    __syncthreads();
  }

  bool bad = false;
  // the next particle's record is loaded before this one is processed
  // (the stores below would otherwise keep the loads from moving up)
  struct Rec {
    unsigned cw;
    R fx, fr, th, w, px, py, pz;
  };
  auto fetch = [&](int k) {
    Rec r;
    const int p = start + k;
    r.cw = pld<NT>(elem(P.cell, p));
    r.fx = pld<NT>(elem(P.fx, p));
    r.fr = pld<NT>(elem(P.fr, p));
    r.th = pld<NT>(elem(P.th, p));
    r.w = pld<NT>(elem(P.w, p));
    r.px = pld<NT>(elem(P.px, p));
    r.py = pld<NT>(elem(P.py, p));
    r.pz = pld<NT>(elem(P.pz, p));
    return r;
  };
  Rec nxt;
  if (threadIdx.x < count) nxt = fetch(threadIdx.x);
  for (int k = threadIdx.x; k < count; k += WG) {
    const Rec cur = nxt;
    if (k + WG < count) nxt = fetch(k + WG);
    const int p = start + k;
    const unsigned cw = cur.cw;
    if (cw == kDead) continue;
    const R fx = cur.fx, fr = cur.fr, th = cur.th, w = cur.w;
    const R px = cur.px;
    R py = cur.py, pz = cur.pz;
    R ph;
    if constexpr (O == 2) {
      const int a = clampi(cell_ix(cw) - q.X0, 2, LX - 4, bad);
      const int b = clampi(cell_jr(cw) - q.R0, 2, LR - 4, bad);
      ph = interp3<R>(sm.phh, quad_primal<R>(a, fx), quad_primal<R>(b, fr));
    } else {
      // the old cell is at most two cells out of the tile: the range of the
      // current stencil's old cell, the same clamp as the deposit's (shared)
      const int a = clampi(cell_ix(cw) - q.X0, 1, LX - 4, bad);
      const int b = clampi(cell_jr(cw) - q.R0, 1, LR - 4, bad);
      ph = interp2<R>(sm.phh, primal_w<R>(a, fx), primal_w<R>(b, fr));
    }
    const R ig = rsqrt_r((R)1 + px * px + py * py + pz * pz + ph);
    Move<R> mv;
    push_position<R>(g, cw, fx, fr, th, py, pz, px * ig, py * ig, pz * ig, mv);
    if (mv.refl) {
      *elem(P.py, p) = py;
      *elem(P.pz, p) = pz;
    }
    const int reln = mv.ix1 - (int)g.shift;  // (lab columns stay below COL_MAX)
    if ((unsigned)reln >= (unsigned)g.nx) {
      *elem(P.cell, p) = kDead;  // left the window: removed without deposit
      atomicAdd(&sm.tcnt[9], 1);
      continue;
    }
    if (DEFER) {
      scr.cell[p] = cw;
      scr.fx[p] = fx;
      scr.fr[p] = fr;
      scr.th[p] = th;
      scr.w[p] = mv.refl ? -ig : ig;
    } else if constexpr (O == 2) {
      deposit_current2<R, M1>(sm, q, g, mv, w, bad);
    } else {
      deposit_current<R, M1>(sm, q, g, mv, w, bad);
    }
    pst<NT>(elem(P.cell, p), pack_cell(mv.ix1, mv.jr1));
    pst<NT>(elem(P.fx, p), mv.fx1);
    pst<NT>(elem(P.fr, p), mv.fr1);
    pst<NT>(elem(P.th, p), mv.th1);
    if (vacate && reln < 1) {
      if (!DEFER) *elem(P.cell, p) = kDead;  // vacated column: dropped after depositing
      atomicAdd(&sm.tcnt[9], 1);
      continue;
    }
    if (sc.mode == SCAT_CELL) {
      const int sx = clampi(mv.ix1 - (q.T * TX - SORT_EVERY), 0, CR - 1, bad);
      const int sr = clampi(mv.jr1 - (q.tcr * TR - SORT_EVERY), 0, CR - 1, bad);
      atomicAdd(&sm.ccell[sx * CR + sr], 1);
    } else if (sc.mode == SCAT_TILE) {
      // a particle that changes tile (rare) counts for its new tile
      const int dtx = clampi(mv.ix1 / TX - q.T, -1, 1, bad);
      const int dtr = clampi(mv.jr1 / TR - q.tcr, -1, 1, bad);
      if (dtx != 0 || dtr != 0) atomicAdd(&sm.tcnt[(dtx + 1) * 3 + dtr + 1], 1);
    }
  }
  if (bad) atomicOr(err, ERR_HALO);
  __syncthreads();
  if (!DEFER) flush_current<R, M1, O>(sm, q, g, jx_out, jr_out, jx1_out, jr1_out, jt1_out);
  if (sc.mode == SCAT_CELL) flush_cells(sm.ccell, q, g, sc.ccount);
  flush_tiles(sm.tcnt, q, g, sc, fill_item);
}

// ============================= deferred deposits (stage-by-stage API) ==
// chi^n from x^n and the gbar^n kept by a deferred momentum pass
template <class R>
__global__ __launch_bounds__(WG) void k_deposit_chi(Geo g, R* __restrict__ chi_out, Parts<R> P,
                                                    Layout L, const R* __restrict__ gscr, int* err) {
  __shared__ double acc[LN];
  __shared__ R ivol[LR];
  const int item = item_of(blockIdx.x, gridDim.x);
  if (item >= *L.n_items) return;
  const int4 it = L.items[item];
  const Region q = region_of(g, it.x);
  for (int k = threadIdx.x; k < LN; k += WG) acc[k] = 0;
  for (int k = threadIdx.x; k < LR; k += WG) {
    const int j = q.R0 + k;
    ivol[k] = (j >= 0 && j <= g.nr) ? inv_vol_node<R>(g, j) : (R)0;
  }
  __syncthreads();
  bool bad = false;
  for (int k = threadIdx.x; k < it.z; k += WG) {
    const int p = it.y + k;
    const unsigned cw = P.cell[p];
    if (cw == kDead) continue;
    const int a = clampi(cell_ix(cw) - q.X0, 0, LX - 2, bad);
    const int b = clampi(cell_jr(cw) - q.R0, 0, LR - 2, bad);
    const Lin<R> Px = primal_w<R>(a, P.fx[p]), Pr = primal_w<R>(b, P.fr[p]);
    const R wg = P.w[p] / gscr[p];
#pragma unroll
    for (int aa = 0; aa < 2; ++aa)
#pragma unroll
      for (int bb = 0; bb < 2; ++bb)
        lds_add(&acc[(Px.i + aa) * LR + Pr.i + bb], (double)(wg * (aa ? Px.b : Px.a) * (bb ? Pr.b : Pr.a) * ivol[Pr.i + bb]));
  }
  if (bad) atomicOr(err, ERR_HALO);
  __syncthreads();
  for (int k = threadIdx.x; k < LN; k += WG) {
    const R v = (R)acc[k];
    if (v == (R)0) continue;
    const int a = k / LR, b = k - (k / LR) * LR;
    const int rel = q.relX0 + a, j = q.R0 + b;
    if (rel < 0 || rel > g.nx || j < 0 || j > g.nr) continue;
    atomicAdd(&chi_out[(size_t)phys_col(g, rel) * g.pitch + j], v);
  }
}

// J^{n+1/2} from the old positions and gbar kept by a deferred position pass
template <class R, bool M1>
__global__ __launch_bounds__(WG) void k_deposit_J(Geo g, R* __restrict__ jx_out, R* __restrict__ jr_out,
                                                  typename cplx_of<R>::type* __restrict__ jx1_out,
                                                  typename cplx_of<R>::type* __restrict__ jr1_out,
                                                  typename cplx_of<R>::type* __restrict__ jt1_out,
                                                  Parts<R> P, Layout L, int vacate, Parts<R> scr, int* err) {
  __shared__ SmemPos<R, M1> sm;
  const int item = item_of(blockIdx.x, gridDim.x);
  if (item >= *L.n_items) return;
  const int4 it = L.items[item];
  const Region q = region_of(g, it.x);
  stage_pos_constants(sm, q, g);
  zero_pos_acc(sm);
  __syncthreads();
  bool bad = false;
  for (int k = threadIdx.x; k < it.z; k += WG) {
    const int p = it.y + k;
    const unsigned cw = P.cell[p];
    if (cw == kDead) continue;
    const R gm = scr.w[p];
    R py = P.py[p], pz = P.pz[p];
    if (gm < (R)0) {
      // undo the specular reflection of p (an involution about r-hat)
      R s1, c1;
      sincos_r(P.th[p], &s1, &c1);
      const R prad = py * c1 + pz * s1;
      py -= (R)2 * prad * c1;
      pz -= (R)2 * prad * s1;
    }
    const R ig = fabs(gm);
    // replay the push from the kept old position: the same arithmetic as the
    // fused position pass, hence the same move
    Move<R> mv;
    R py2 = py, pz2 = pz;
    push_position<R>(g, scr.cell[p], scr.fx[p], scr.fr[p], scr.th[p], py2, pz2, P.px[p] * ig, py * ig, pz * ig, mv);
    deposit_current<R, M1>(sm, q, g, mv, P.w[p], bad);
    if (vacate && (long long)cell_ix(cw) - g.shift < 1) P.cell[p] = kDead;
  }
  if (bad) atomicOr(err, ERR_HALO);
  __syncthreads();
  flush_current<R, M1, 1>(sm, q, g, jx_out, jr_out, jx1_out, jr1_out, jt1_out);
}

// The copy back of a tile sort whose scan rebuilt the layout, as a launch of
// its own (the deferred-deposit stages, which read the particles before the
// envelope stage that otherwise carries it).
template <class R>
__global__ __launch_bounds__(256) void k_settle(SettleArgs<R> sa) {
  settle_copy(sa, blockIdx.x, gridDim.x);
}

// initial loading of window cells in tile-major order (offsets per tile
// from the host, cells of a tile column-major inside the tile)
template <class R>
__global__ void k_init_particles(Geo g, Plasma pl, Parts<R> P, const int* __restrict__ offsets) {
  const long long cell = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (cell >= (long long)g.nx * g.nr) return;
  const int col = (int)(cell / g.nr), j = (int)(cell - (long long)col * g.nr);
  const int T = col / TX, tcr = j / TR;
  const int trt = min(TR, g.nr - tcr * TR);
  const int tct = min(TX, g.nx - T * TX);
  const int key = tile_key(g, col, j);
  const int local = (col - T * TX) * trt + (j - tcr * TR);
  const int ppc = g.ppc_x * g.ppc_r * g.ppc_t;
  for (int k = 0; k < ppc; ++k) load_particle<R>(g, pl, P, offsets[key], local * ppc, tct * trt * ppc, col, j, k);
}

// ====================================================== cell-sort copy ==
// The cell-ordered copy of a cell sort whose layout carries LAYOUT_GATHER:
// slot s of the new layout's work items takes the record of slot inv[s] of
// the buffer in use (the momentum pass wrote inv and updated p there).  One group per item moves one record
// array after the other, so the reads of a group stay within its tile's few
// tens of kilobytes of that array (cached in the L2) and every store is
// contiguous.  A direct scatter of whole records from the momentum pass
// wrote partial cache lines across every array of a tile at once once the
// particles had moved (measured: 2.5x its bytes written, 650 us for the
// cell sort late in the LWFA run).  A slot whose source index is not valid
// (possible only after a count mismatch, which the pass flags) gets a
// removed particle.
template <bool NT, int PPT, class T>
__device__ inline void gather_array(T* __restrict__ to, const T* __restrict__ from, const unsigned* sp, int start,
                                    int count, T none) {
  T v[PPT];
#pragma unroll
  for (int u = 0; u < PPT; ++u) {
    const int k = threadIdx.x + u * WG;
    v[u] = (k < count && sp[u] != ~0u) ? *elem(from, (int)sp[u]) : none;
  }
#pragma unroll
  for (int u = 0; u < PPT; ++u) {
    const int k = threadIdx.x + u * WG;
    if (k < count) pst<NT>(elem(to, start + k), v[u]);
  }
}
template <class R, bool NT>
__global__ __launch_bounds__(WG) void k_permute(Parts<R> src, Parts<R> dst, Layout L, const unsigned* __restrict__ inv,
                                                long long cap) {
  constexpr int PPT = CHUNK / WG;
  if ((*L.mode & LAYOUT_GATHER) == 0) return;  // the momentum pass scattered the records
  const int item = item_of(blockIdx.x, gridDim.x);
  if (item >= *L.n_items) return;
  const int4 it = L.items[item];
  const int start = it.y, count = it.z;  // count <= chunk <= CHUNK
  unsigned sp[PPT];
#pragma unroll
  for (int u = 0; u < PPT; ++u) {
    const int k = threadIdx.x + u * WG;
    const unsigned v = k < count ? *elem(inv, start + k) : ~0u;
    sp[u] = (long long)v < cap ? v : ~0u;
  }
  gather_array<NT, PPT>(dst.cell, src.cell, sp, start, count, kDead);
  gather_array<NT, PPT>(dst.fx, src.fx, sp, start, count, (R)0);
  gather_array<NT, PPT>(dst.fr, src.fr, sp, start, count, (R)0);
  gather_array<NT, PPT>(dst.th, src.th, sp, start, count, (R)0);
  gather_array<NT, PPT>(dst.px, src.px, sp, start, count, (R)0);
  gather_array<NT, PPT>(dst.py, src.py, sp, start, count, (R)0);
  gather_array<NT, PPT>(dst.pz, src.pz, sp, start, count, (R)0);
  gather_array<NT, PPT>(dst.w, src.w, sp, start, count, (R)0);
  gather_array<NT, PPT>(dst.id, src.id, sp, start, count, 0u);
}

// ============================================================ launchers ==
template <class R, bool M1, bool DEFER, int SCAT, int O, bool NT>
static void launch_momentum_k(const Geo& g, const Grids<R>& f, R* chi, const Parts<R>& src, const Parts<R>& dst,
                              const Layout& Ls, const Layout& Ld, int* ccur, R* gscr, unsigned* inv, int* err,
                              int max_items, hipStream_t st, const KEvents& ev) {
  launch_k(k_momentum<R, M1, DEFER, SCAT, O, NT>, dim3(max_items), dim3(WG), st, ev, g, f, chi, src, dst, Ls, Ld,
           ccur, gscr, inv, err);
}
template <class R, bool M1, bool DEFER, int O, bool NT>
static void launch_momentum_nt(const Geo& g, const Grids<R>& f, R* chi, const Parts<R>& src, const Parts<R>& dst,
                               const Layout& Ls, const Layout& Ld, int* ccur, R* gscr, unsigned* inv, int* err,
                               int grid, int scatter, hipStream_t st, const KEvents& ev) {
  if (scatter == SCAT_TILE && DEFER) {
    // the deferred chi deposit reads the particles before the envelope stage
    launch_momentum_k<R, M1, DEFER, SCAT_TILE, O, NT>(g, f, chi, src, dst, Ls, Ld, ccur, gscr, inv, err, grid, st,
                                                      KEvents{ev.start, nullptr});
    launch_k(k_settle<R>, dim3(SETTLE_BLOCKS), dim3(256), st, KEvents{nullptr, ev.stop},
             SettleArgs<R>{src, dst, Ld, g.cap, SETTLE_BLOCKS});
  } else if (scatter == SCAT_TILE) {
    // (the envelope stage carries the copy back)
    launch_momentum_k<R, M1, DEFER, SCAT_TILE, O, NT>(g, f, chi, src, dst, Ls, Ld, ccur, gscr, inv, err, grid, st, ev);
  } else if (scatter == SCAT_CELL && !DEFER) {
    // the pass scatters the records, or records their destinations for the
    // gather that follows (the layout scan chose)
    launch_momentum_k<R, M1, DEFER, SCAT_CELL, O, NT>(g, f, chi, src, dst, Ls, Ld, ccur, gscr, inv, err, grid, st,
                                                      KEvents{ev.start, nullptr});
    launch_k(k_permute<R, NT>, dim3(grid), dim3(WG), st, KEvents{nullptr, ev.stop}, src, dst, Ld,
             (const unsigned*)inv, g.cap);
  } else if (scatter == SCAT_CELL) {
    launch_momentum_k<R, M1, DEFER, SCAT_CELL, O, NT>(g, f, chi, src, dst, Ls, Ld, ccur, gscr, inv, err, grid, st, ev);
  } else {
    launch_momentum_k<R, M1, DEFER, SCAT_NONE, O, NT>(g, f, chi, src, dst, Ls, Ld, ccur, gscr, inv, err, grid, st, ev);
  }
}
// non-temporal record access for the fused passes of large runs only
template <class R, bool M1, bool DEFER, int O>
static void launch_momentum_sc(const Geo& g, const Grids<R>& f, R* chi, const Parts<R>& src, const Parts<R>& dst,
                               const Layout& Ls, const Layout& Ld, int* ccur, R* gscr, unsigned* inv, int* err,
                               int grid, int scatter, hipStream_t st, const KEvents& ev) {
  if (!DEFER && g.stream_parts)
    launch_momentum_nt<R, M1, DEFER, O, true>(g, f, chi, src, dst, Ls, Ld, ccur, gscr, inv, err, grid, scatter, st, ev);
  else
    launch_momentum_nt<R, M1, DEFER, O, false>(g, f, chi, src, dst, Ls, Ld, ccur, gscr, inv, err, grid, scatter, st, ev);
}

// order 2 has no deferred-deposit variant (the library rejects the request)
template <class R>
void launch_momentum(const Geo& g, const Grids<R>& f, R* chi, const Parts<R>& src, const Parts<R>& dst,
                     const Layout& Ls, const Layout& Ld, int* ccur, R* gscr, unsigned* inv, int* err, int grid,
                     bool defer, int scatter, hipStream_t st, const KEvents& ev) {
  if (grid <= 0) return;
  if (g.order == 2) {
    if (g.modes >= 2)
      launch_momentum_sc<R, true, false, 2>(g, f, chi, src, dst, Ls, Ld, ccur, gscr, inv, err, grid, scatter, st, ev);
    else
      launch_momentum_sc<R, false, false, 2>(g, f, chi, src, dst, Ls, Ld, ccur, gscr, inv, err, grid, scatter, st, ev);
  } else if (g.modes >= 2) {
    if (defer)
      launch_momentum_sc<R, true, true, 1>(g, f, chi, src, dst, Ls, Ld, ccur, gscr, inv, err, grid, scatter, st, ev);
    else
      launch_momentum_sc<R, true, false, 1>(g, f, chi, src, dst, Ls, Ld, ccur, gscr, inv, err, grid, scatter, st, ev);
  } else {
    if (defer)
      launch_momentum_sc<R, false, true, 1>(g, f, chi, src, dst, Ls, Ld, ccur, gscr, inv, err, grid, scatter, st, ev);
    else
      launch_momentum_sc<R, false, false, 1>(g, f, chi, src, dst, Ls, Ld, ccur, gscr, inv, err, grid, scatter, st, ev);
  }
}

template <class R> int inject_blocks(const Geo& g) {
  const int n = std::max(g.nr * g.ppc_x * g.ppc_r * g.ppc_t, g.ntr);
  return (n + WG - 1) / WG;
}

template <class R, bool M1, bool DEFER, int O, bool NT>
static void launch_position_nt(const Geo& g, const Grids<R>& f, const DepositBufs<R>& d, const Parts<R>& P,
                               const Layout& L, const SortCounts& sc, int vacate, const Parts<R>& scr, int* err,
                               int max_items, const InjectArgs& inj, hipStream_t st, const KEvents& ev) {
  launch_k(k_position<R, M1, DEFER, O, NT>, dim3(max_items + inj.blocks), dim3(WG), st, ev, g, f, d.jx, d.jr, d.jx1,
           d.jr1, d.jt1, P, L, sc, vacate, scr, err, max_items, inj);
}
template <class R, bool M1, bool DEFER, int O>
static void launch_position_k(const Geo& g, const Grids<R>& f, const DepositBufs<R>& d, const Parts<R>& P,
                              const Layout& L, const SortCounts& sc, int vacate, const Parts<R>& scr, int* err,
                              int grid, const InjectArgs& inj, hipStream_t st, const KEvents& ev) {
  if (!DEFER && g.stream_parts)
    launch_position_nt<R, M1, DEFER, O, true>(g, f, d, P, L, sc, vacate, scr, err, grid, inj, st, ev);
  else
    launch_position_nt<R, M1, DEFER, O, false>(g, f, d, P, L, sc, vacate, scr, err, grid, inj, st, ev);
}

template <class R>
void launch_position(const Geo& g, const Grids<R>& f, const DepositBufs<R>& d, const Parts<R>& P, const Layout& L,
                     const SortCounts& sc, int vacate, const Parts<R>& scr, int* err, int grid, bool defer,
                     const InjectArgs& inj, hipStream_t st, const KEvents& ev) {
  if (grid <= 0) return;
  if (g.order == 2) {
    if (g.modes >= 2)
      launch_position_k<R, true, false, 2>(g, f, d, P, L, sc, vacate, scr, err, grid, inj, st, ev);
    else
      launch_position_k<R, false, false, 2>(g, f, d, P, L, sc, vacate, scr, err, grid, inj, st, ev);
  } else if (g.modes >= 2) {
    if (defer)
      launch_position_k<R, true, true, 1>(g, f, d, P, L, sc, vacate, scr, err, grid, inj, st, ev);
    else
      launch_position_k<R, true, false, 1>(g, f, d, P, L, sc, vacate, scr, err, grid, inj, st, ev);
  } else {
    if (defer)
      launch_position_k<R, false, true, 1>(g, f, d, P, L, sc, vacate, scr, err, grid, inj, st, ev);
    else
      launch_position_k<R, false, false, 1>(g, f, d, P, L, sc, vacate, scr, err, grid, inj, st, ev);
  }
}

template <class R>
void launch_deposit_chi(const Geo& g, R* chi, const Parts<R>& P, const Layout& L, const R* gscr, int* err, int grid,
                        hipStream_t st) {
  if (grid <= 0) return;
  hipLaunchKernelGGL((k_deposit_chi<R>), dim3(grid), dim3(WG), 0, st, g, chi, P, L, gscr, err);
}

template <class R>
void launch_deposit_J(const Geo& g, const DepositBufs<R>& d, const Parts<R>& P, const Layout& L, int vacate,
                      const Parts<R>& scr, int* err, int grid, hipStream_t st) {
  if (grid <= 0) return;
  if (g.modes >= 2)
    hipLaunchKernelGGL((k_deposit_J<R, true>), dim3(grid), dim3(WG), 0, st, g, d.jx, d.jr, d.jx1, d.jr1, d.jt1, P, L, vacate, scr, err);
  else
    hipLaunchKernelGGL((k_deposit_J<R, false>), dim3(grid), dim3(WG), 0, st, g, d.jx, d.jr, d.jx1, d.jr1, d.jt1, P, L, vacate, scr, err);
}

template <class R>
void launch_init_particles(const Geo& g, const Plasma& pl, const Parts<R>& P, const int* offsets, hipStream_t st) {
  const long long cells = (long long)g.nx * g.nr;
  const int grid = (int)((cells + 255) / 256);
  hipLaunchKernelGGL((k_init_particles<R>), dim3(grid), dim3(256), 0, st, g, pl, P, offsets);
}



#define ENVPIC_INST(R)                                                                                          \
  template void launch_momentum<R>(const Geo&, const Grids<R>&, R*, const Parts<R>&, const Parts<R>&,           \
                                   const Layout&, const Layout&, int*, R*, unsigned*, int*, int, bool, int,     \
                                   hipStream_t, const KEvents&);                                                \
  template void launch_position<R>(const Geo&, const Grids<R>&, const DepositBufs<R>&, const Parts<R>&,         \
                                   const Layout&, const SortCounts&, int, const Parts<R>&, int*, int, bool,     \
                                   const InjectArgs&, hipStream_t, const KEvents&);                             \
  template int inject_blocks<R>(const Geo&);                                                                    \
  template void launch_deposit_chi<R>(const Geo&, R*, const Parts<R>&, const Layout&, const R*, int*, int,      \
                                      hipStream_t);                                                             \
  template void launch_deposit_J<R>(const Geo&, const DepositBufs<R>&, const Parts<R>&, const Layout&, int,     \
                                    const Parts<R>&, int*, int, hipStream_t);                                   \
  template void launch_init_particles<R>(const Geo&, const Plasma&, const Parts<R>&, const int*, hipStream_t);
ENVPIC_INST(float)
ENVPIC_INST(double)
#undef ENVPIC_INST

}  // namespace envpic
