// grid.hip -- grid kernels of the cylindrical envelope PIC step
// (arXiv:1912.04674): the explicit envelope update (Sec. 3, Eq.
// envelope_solver with the cylindrical Laplacian), the Yee/FDTD update of the
// low-frequency fields (Sec. 2, Eq. MaxwellEqsCylindrical; Sec. 3), the
// moving-window column reset and the initial envelope.
//
// One thread per window node (i, j), radius fastest, so a wavefront reads a
// contiguous run of one column; columns live in a ring indexed by lab column
// mod nxa.  All kernels are bound by HBM bandwidth (a few flops per byte).
#include "envpic.h"
#include "common.hpp"
#include "cplx.hpp"
#include "launch.hpp"
#include "scan.hpp"

namespace envpic {

// -------------------------------------------------------------- envelope --
// A^{n+1} = (1 + i dt)/(1 + dt^2) [2 A^n - (1 + i dt) A^{n-1}
//            + dt^2 (lap A^n - chi^n A^n + 2i (A_{i+1} - A_{i-1})/(2 dx))]
// radial Laplacian: 5-point form with (1/r_j)(A_{j+1} - A_{j-1})/(2 dr) for
// j >= 1, and its on-axis limit 4 (A_1 - A_0)/dr^2 at j = 0.  Dirichlet at
// the x ends and at r_max.  A^{n+1} overwrites A^{n-1} in place.  With
// fp64_rows the rows j = 0, 1 are advanced in FP64 from their own FP64
// copies and rounded into the FP32 bulk array for the gathers.
// reciprocal in the grid precision: FP64 division on the FP64 path, the
// hardware reciprocal (about 1 ulp) on the FP32 path
__device__ inline double recip_r(double x) { return 1.0 / x; }
__device__ inline float recip_r(float x) { return __builtin_amdgcn_rcpf(x); }

template <class R>
__global__ void k_envelope(Geo g, Grids<R> f, const R* __restrict__ chi, int fp64_rows, SettleArgs<R> sa) {
  using C = typename cplx_of<R>::type;
  const int node_groups = (int)gridDim.x - sa.blocks;
  if ((int)blockIdx.x >= node_groups) {  // the copy back of a rebuilt tile sort
    settle_copy(sa, (int)blockIdx.x - node_groups, sa.blocks);
    return;
  }
  const int nr1 = g.nr + 1;
  const int idx = (int)(blockIdx.x * blockDim.x + threadIdx.x);  // nodes < 2^31
  if (idx >= (g.nx + 1) * nr1) return;
  const int i = idx / nr1, j = idx - i * nr1;
  const int pc = phys_col(g, i);
  const size_t o = (size_t)pc * g.pitch + j;
  const bool rows64 = fp64_rows && j <= 1;
  if (i == 0 || i == g.nx || j == g.nr) {
    f.envp[o] = mk<C>((R)0, (R)0);
    if (rows64) f.axp[pc * 2 + j] = make_double2(0.0, 0.0);
    return;
  }
  const int pp = phys_col(g, i + 1), pm = phys_col(g, i - 1);
  const double dt = g.dt;
  const double pre_r = 1.0 / (1.0 + dt * dt), pre_i = dt / (1.0 + dt * dt);
  if (rows64) {
    const double2 a = f.ax[pc * 2 + j], aip = f.ax[pp * 2 + j], aim = f.ax[pm * 2 + j];
    const double idx2 = 1.0 / (g.dx * g.dx), idr2 = 1.0 / (g.dr * g.dr);
    double2 lap = make_double2((aip.x - 2.0 * a.x + aim.x) * idx2, (aip.y - 2.0 * a.y + aim.y) * idx2);
    if (j == 0) {
      const double2 up = f.ax[pc * 2 + 1];
      lap.x += 4.0 * (up.x - a.x) * idr2;
      lap.y += 4.0 * (up.y - a.y) * idr2;
    } else {
      const C u = f.env[o + 1];
      const double2 up = make_double2((double)u.x, (double)u.y), dn = f.ax[pc * 2 + 0];
      const double ir = 1.0 / (2.0 * g.dr * g.dr);  // 1/(2 r_1 dr), r_1 = dr
      lap.x += (up.x - 2.0 * a.x + dn.x) * idr2 + (up.x - dn.x) * ir;
      lap.y += (up.y - 2.0 * a.y + dn.y) * idr2 + (up.y - dn.y) * ir;
    }
    const double ch = (double)chi[o];
    const double i2dx = 1.0 / g.dx;  // 2i (d)/(2 dx) = i d / dx
    const double rr = lap.x - ch * a.x - (aip.y - aim.y) * i2dx;
    const double ri = lap.y - ch * a.y + (aip.x - aim.x) * i2dx;
    const double2 ap = f.axp[pc * 2 + j];
    const double br = 2.0 * a.x - (ap.x - dt * ap.y) + dt * dt * rr;
    const double bi = 2.0 * a.y - (ap.y + dt * ap.x) + dt * dt * ri;
    const double2 an = make_double2(pre_r * br - pre_i * bi, pre_r * bi + pre_i * br);
    f.axp[pc * 2 + j] = an;
    f.envp[o] = mk<C>((R)an.x, (R)an.y);
    return;
  }
  const R rdt = (R)dt;
  const C a = f.env[o], aip = f.env[(size_t)pp * g.pitch + j], aim = f.env[(size_t)pm * g.pitch + j];
  const R idx1 = recip_r((R)g.dx), idr1 = recip_r((R)g.dr);
  const R idx2 = idx1 * idx1, idr2 = idr1 * idr1;
  R lx = (aip.x - (R)2 * a.x + aim.x) * idx2, ly = (aip.y - (R)2 * a.y + aim.y) * idx2;
  const C up = f.env[o + 1];
  if (j == 0) {
    lx += (R)4 * (up.x - a.x) * idr2;
    ly += (R)4 * (up.y - a.y) * idr2;
  } else {
    const C dn = f.env[o - 1];
    const R ir = (R)0.5 * idr2 * recip_r((R)j);
    lx += (up.x - (R)2 * a.x + dn.x) * idr2 + (up.x - dn.x) * ir;
    ly += (up.y - (R)2 * a.y + dn.y) * idr2 + (up.y - dn.y) * ir;
  }
  const R ch = chi[o];
  const R i2dx = idx1;
  const R rr = lx - ch * a.x - (aip.y - aim.y) * i2dx;
  const R ri = ly - ch * a.y + (aip.x - aim.x) * i2dx;
  const C ap = f.envp[o];
  const R br = (R)2 * a.x - (ap.x - rdt * ap.y) + rdt * rdt * rr;
  const R bi = (R)2 * a.y - (ap.y + rdt * ap.x) + rdt * rdt * ri;
  const R pr = recip_r((R)1 + rdt * rdt), pim = rdt * pr;
  f.envp[o] = mk<C>(pr * br - pim * bi, pr * bi + pim * br);
}

// ----------------------------------------------- Ampere and Faraday --
// Ampere: E^{n+1} from E^n, B^{n+1/2}, J^{n+1/2}
//   E_r(i, j+1/2) -= dt [(B_t(i+1/2) - B_t(i-1/2))/dx + J_r];   E_r = 0 at x ends
//   E_x(i+1/2, j) += dt [(r_{j+1/2} B_t(j+1/2) - r_{j-1/2} B_t(j-1/2))/(r_j dr) - J_x]
//     axis: (1/r) d(r B_t)/dr -> 4 B_t(1/2)/dr (flux through the disc r < dr/2);
//     E_x = 0 at r_max (perfect conductor).
//   Mode 1: d/dtheta -> -i (F = Re[F_1 e^{-i theta}]); axial components
//   vanish on the axis, E_t there from the odd ghost B_x(-1/2) = -B_x(1/2).
// Faraday: B^{n+3/2} from B^{n+1/2} and E^{n+1}, and Bbar^{n+1} = (B^{n+1/2} + B^{n+3/2})/2
//   B_t(i+1/2, j+1/2) += dt [(E_x(j+1) - E_x(j))/dr - (E_r(i+1) - E_r(i))/dx]
//   B_x(i, j+1/2) -= dt [((j+1) E_t(j+1) - j E_t(j))/((j+1/2) dr) + (i/r_{j+1/2}) E_r]
//   B_r(i+1/2, j) += dt [(i/r) E_x + (E_t(i+1) - E_t(i))/dx]; on the axis E_x/r -> E_x(1)/dr
// One kernel: a work group computes E^{n+1} on its tile of nodes plus one
// column and one row beyond (recomputed by the neighbour that owns them,
// with the same arithmetic), keeps it in LDS, then advances B on its tile.
// E^n and B^{n+1/2} are only read and the new values go to the second
// copies (ex_n, ..., bt1_n), so no work group sees another's output; Bbar
// is written in place.  The deposits of the next step (chi, J) are cleared
// on the way.
template <class R, bool M1> struct ENew {
  using C = typename cplx_of<R>::type;
  R ex, er;
  C ex1, er1, et1;
};

template <class R, bool M1>
__device__ inline ENew<R, M1> ampere(const Geo& g, const Grids<R>& f, const DepositBufs<R>& din, int i, int j) {
  using C = typename cplx_of<R>::type;
  ENew<R, M1> e;
  const int pc = phys_col(g, i);
  const size_t o = (size_t)pc * g.pitch + j;
  const size_t om = i > 0 ? (size_t)phys_col(g, i - 1) * g.pitch + j : o;
  const R dt = (R)g.dt, idx_ = recip_r((R)g.dx), idr = recip_r((R)g.dr);
  const bool xin = i > 0 && i < g.nx;
  e.er = (j <= g.nr - 1 && xin) ? f.er[o] - dt * ((f.bt[o] - f.bt[om]) * idx_ + din.jr[o]) : (R)0;
  e.ex = 0;
  if (i <= g.nx - 1) {
    if (j == 0) {
      e.ex = f.ex[o] + dt * ((R)4 * f.bt[o] * idr - din.jx[o]);
    } else if (j < g.nr) {
      e.ex = f.ex[o] + dt * (((R)(j + 0.5) * f.bt[o] - (R)(j - 0.5) * f.bt[o - 1]) * (recip_r((R)j) * idr) - din.jx[o]);
    }
  }
  if (M1) {
    const C z = mk<C>((R)0, (R)0);
    e.ex1 = z;
    e.er1 = z;
    e.et1 = z;
    if (i <= g.nx - 1 && j >= 1 && j <= g.nr - 1) {
      const R irj = recip_r((R)j) * idr;
      const C curl = cadd(cscale(csub(cscale(f.bt1[o], (R)(j + 0.5)), cscale(f.bt1[o - 1], (R)(j - 0.5))), irj),
                          cscale(cmuli(f.br1[o]), irj));
      e.ex1 = cadd(f.ex1[o], cscale(csub(curl, din.jx1[o]), dt));
    }
    if (j <= g.nr - 1 && xin) {
      const R irh = recip_r((R)(j + 0.5)) * idr;
      const C curl = csub(cscale(cmuli(f.bx1[o]), -irh), cscale(csub(f.bt1[o], f.bt1[om]), idx_));
      e.er1 = cadd(f.er1[o], cscale(csub(curl, din.jr1[o]), dt));
      const C dbr = cscale(csub(f.br1[o], f.br1[om]), idx_);
      const C dbx = j == 0 ? cscale(f.bx1[o], (R)2 * idr) : cscale(csub(f.bx1[o], f.bx1[o - 1]), idr);
      e.et1 = cadd(f.et1[o], cscale(csub(csub(dbr, dbx), din.jt1[o]), dt));
    }
  }
  return e;
}

constexpr int MW_TI = 8, MW_TJ = 64;  // tile of a Maxwell work group: 8 columns x 64 rows
constexpr int MW_T = MW_TI * MW_TJ;   // threads of a field-stage work group

template <class R, bool M1> struct MwShared {
  using C = typename cplx_of<R>::type;
  static constexpr int HI = MW_TI + 1, HJ = MW_TJ + 1, HN = HI * HJ;
  R ex[HN], er[HN];
  C ex1[M1 ? HN : 1], er1[M1 ? HN : 1], et1[M1 ? HN : 1];
};

// B^{n+1/2} of one node
template <class R, bool M1> struct MwB {
  using C = typename cplx_of<R>::type;
  R bt;
  C bx1, br1, bt1;
};

// One owned node (i, j) of a Maxwell tile, LDS index k (E^{n+1} of the tile
// and its +1 column / row in sm), grid offset o, B^{n+1/2} in bo: the new E
// stored, B^{n+3/2} and Bbar^{n+1}, the next deposits cleared.
template <class R, bool M1>
__device__ inline void tile_node(const Geo& g, const Grids<R>& f, const DepositBufs<R>& dnext, int i, int j, int k,
                                 size_t o, const MwB<R, M1>& bo, bool left_edge_zero, const MwShared<R, M1>& sm) {
  using C = typename cplx_of<R>::type;
  constexpr int HJ = MwShared<R, M1>::HJ;
  const int kp = k + HJ;  // (i+1, j); k + 1 is (i, j+1)
  const R dt = (R)g.dt, idx_ = recip_r((R)g.dx), idr = recip_r((R)g.dr);
  const bool ez = left_edge_zero && i == 1;
  // the new E of the owned node
  if (j <= g.nr - 1) f.er_n[o] = ez ? (R)0 : sm.er[k];
  if (i <= g.nx - 1) f.ex_n[o] = sm.ex[k];
  if (M1) {
    const C z = mk<C>((R)0, (R)0);
    if (i <= g.nx - 1) f.ex1_n[o] = sm.ex1[k];
    if (j <= g.nr - 1) f.er1_n[o] = ez ? z : sm.er1[k];
    f.et1_n[o] = ez ? z : sm.et1[k];
  }
  // ---- B^{n+3/2} and Bbar^{n+1}
  if (i <= g.nx - 1 && j <= g.nr - 1) {
    const R b0 = bo.bt;
    const R b1 = b0 + dt * ((sm.ex[k + 1] - sm.ex[k]) * idr - (sm.er[kp] - sm.er[k]) * idx_);
    f.bt_n[o] = b1;
    f.btb[o] = (R)0.5 * (b0 + b1);
  }
  if (M1) {
    if (j <= g.nr - 1) {
      const R irh = recip_r((R)(j + 0.5)) * idr;
      const C b0 = bo.bx1;
      const C curl = cadd(cscale(csub(cscale(sm.et1[k + 1], (R)(j + 1)), cscale(sm.et1[k], (R)j)), irh),
                          cscale(cmuli(sm.er1[k]), irh));
      const C b1 = csub(b0, cscale(curl, dt));
      f.bx1_n[o] = b1;
      f.bxb1[o] = cscale(cadd(b0, b1), (R)0.5);
    }
    if (i <= g.nx - 1) {
      const C exr = j == 0 ? cscale(sm.ex1[k + 1], idr) : cscale(sm.ex1[k], recip_r((R)j) * idr);
      const C b0 = bo.br1;
      const C b1 = cadd(b0, cscale(cadd(cmuli(exr), cscale(csub(sm.et1[kp], sm.et1[k]), idx_)), dt));
      f.br1_n[o] = b1;
      f.brb1[o] = cscale(cadd(b0, b1), (R)0.5);
      if (j <= g.nr - 1) {
        const C c0 = bo.bt1;
        const C c1 = cadd(c0, cscale(csub(cscale(csub(sm.ex1[k + 1], sm.ex1[k]), idr),
                                          cscale(csub(sm.er1[kp], sm.er1[k]), idx_)), dt));
        f.bt1_n[o] = c1;
        f.btb1[o] = cscale(cadd(c0, c1), (R)0.5);
      }
    }
  }
  dnext.chi[o] = 0;
  dnext.jx[o] = 0;
  dnext.jr[o] = 0;
  if (M1) {
    const C z = mk<C>((R)0, (R)0);
    dnext.jx1[o] = z;
    dnext.jr1[o] = z;
    dnext.jt1[o] = z;
  }
}

// The Maxwell tile (i0, j0): E^{n+1} on the tile and its +1 column / +1 row
// into LDS, then the owned nodes' E^{n+1}, B^{n+3/2}, Bbar^{n+1} and the
// cleared next deposits.  left_edge_zero: the window moves after this step
// and column 1 becomes its left edge, where E_r (both modes) and E_t of
// mode 1 are set to zero (B still sees the computed values).
template <class R, bool M1>
__device__ inline void maxwell_tile(const Geo& g, const Grids<R>& f, const DepositBufs<R>& din,
                                    const DepositBufs<R>& dnext, int i0, int j0, bool left_edge_zero,
                                    MwShared<R, M1>& sm) {
  constexpr int HJ = MwShared<R, M1>::HJ, HN = MwShared<R, M1>::HN;
  static_assert(HN <= 2 * MW_T, "two nodes per thread at most");
  auto put = [&](int k, const ENew<R, M1>& e) {
    sm.ex[k] = e.ex;
    sm.er[k] = e.er;
    if (M1) {
      sm.ex1[k] = e.ex1;
      sm.er1[k] = e.er1;
      sm.et1[k] = e.et1;
    }
  };
  // E^{n+1} on the tile and its +1 column / row: node k and, in the first
  // wavefronts, node k + MW_T as well, both in one straight-line block so
  // that their loads are in flight together (indices clamped into the grid;
  // nodes outside it are not stored and never read)
  {
    const int k0 = threadIdx.x, k1 = threadIdx.x + MW_T;
    const int a0 = k0 / HJ, b0 = k0 - (k0 / HJ) * HJ;
    const bool ok0 = i0 + a0 <= g.nx && j0 + b0 <= g.nr;
    if ((int)(threadIdx.x & ~63u) < HN - MW_T) {  // wavefront-uniform
      const int k1c = min(k1, HN - 1);
      const int a1 = k1c / HJ, b1 = k1c - (k1c / HJ) * HJ;
      const bool ok1 = k1 < HN && i0 + a1 <= g.nx && j0 + b1 <= g.nr;
      const ENew<R, M1> e0 = ampere<R, M1>(g, f, din, min(i0 + a0, g.nx), min(j0 + b0, g.nr));
      const ENew<R, M1> e1 = ampere<R, M1>(g, f, din, min(i0 + a1, g.nx), min(j0 + b1, g.nr));
      if (ok0) put(k0, e0);
      if (ok1) put(k1, e1);
    } else if (ok0) {
      put(k0, ampere<R, M1>(g, f, din, i0 + a0, j0 + b0));
    }
  }
  const int a = threadIdx.x / MW_TJ, b = threadIdx.x - (threadIdx.x / MW_TJ) * MW_TJ;
  const int i = i0 + a, j = j0 + b;
  const bool own = i <= g.nx && j <= g.nr;
  const size_t o = (size_t)phys_col(g, own ? i : 0) * g.pitch + (own ? j : 0);
  // B^{n+1/2} of the owned node, loaded before the barrier
  MwB<R, M1> bo;
  bo.bt = f.bt[o];
  if (M1) {
    bo.bx1 = f.bx1[o];
    bo.br1 = f.br1[o];
    bo.bt1 = f.bt1[o];
  }
  __syncthreads();
  if (own) tile_node<R, M1>(g, f, dnext, i, j, a * HJ + b, o, bo, left_edge_zero, sm);
}

// ----------------------------------------------------- window shift --
// After the shift (g holds the new shift), row j: the primal column entering
// at the right (rel = nx) and the half-shifted column entering (rel = nx - 1)
// start at zero, and the new left edge (rel = 0) takes its boundary values
// (zero envelope; E_r and mode-1 E_t there are zeroed by the Maxwell tile).
// Runs in the field-stage kernel before the host swaps the E/B copies, so
// E and B are written in their new (_n) copies.
template <class R, bool M1>
__device__ inline void window_row(const Geo& g, const Grids<R>& f, const DepositBufs<R>& d0,
                                  const DepositBufs<R>& d1, int fp64_rows, int j) {
  using C = typename cplx_of<R>::type;
  if (j > g.nr) return;
  const C z = mk<C>((R)0, (R)0);
  const int pn = phys_col(g, g.nx), pd = phys_col(g, g.nx - 1), pl = phys_col(g, 0);
  const size_t on = (size_t)pn * g.pitch + j, od = (size_t)pd * g.pitch + j, ol = (size_t)pl * g.pitch + j;
  // primal-x grids at the entering column
  f.env[on] = z;
  f.envp[on] = z;
  f.er_n[on] = 0;
  d0.chi[on] = 0; d1.chi[on] = 0;
  d0.jr[on] = 0; d1.jr[on] = 0;
  // half-shifted-x grids at the entering column
  f.ex_n[od] = 0;
  f.bt_n[od] = 0;
  f.btb[od] = 0;
  d0.jx[od] = 0; d1.jx[od] = 0;
  // boundary values at the new left edge
  f.env[ol] = z;
  f.envp[ol] = z;
  if (fp64_rows && j <= 1) {
    f.ax[pn * 2 + j] = make_double2(0.0, 0.0);
    f.axp[pn * 2 + j] = make_double2(0.0, 0.0);
    f.ax[pl * 2 + j] = make_double2(0.0, 0.0);
    f.axp[pl * 2 + j] = make_double2(0.0, 0.0);
  }
  if (M1) {
    f.er1_n[on] = z; f.et1_n[on] = z; f.bx1_n[on] = z; f.bxb1[on] = z;
    d0.jr1[on] = z; d1.jr1[on] = z; d0.jt1[on] = z; d1.jt1[on] = z;
    f.ex1_n[od] = z; f.br1_n[od] = z; f.bt1_n[od] = z; f.brb1[od] = z; f.btb1[od] = z;
    d0.jx1[od] = z; d1.jx1[od] = z;
  }
}

// --------------------------------------------------------- field stage --
// One kernel for the field stage, its work groups in three roles: Maxwell
// tiles (geometry before the shift); if the window moves, the rows of its
// column resets (geometry after it); before a sort, the per-tile cell scans
// (two tiles per group).  No role reads another's output.  On a step
// without a sort, one thread also adds the items and slots of a column
// injected by the position pass to the layout in use.
template <class R, bool M1>
__global__ __launch_bounds__(MW_T) void k_field(Geo g, Grids<R> f, DepositBufs<R> din, DepositBufs<R> dnext,
                                               DepositBufs<R> d0, DepositBufs<R> d1, FieldArgs fa) {
  __shared__ MwShared<R, M1> sm;
  __shared__ int s_a[MW_T];
  const int blk = blockIdx.x;
  // an injected column's items and slots join the layout in use
  if (!fa.presort && blk == 0) bump_pending(fa.gn, fa.in, fa.pending);
  if (blk < fa.nb_mw) {
    maxwell_tile<R, M1>(g, f, din, dnext, (blk / fa.nbx_mw) * MW_TI, (blk % fa.nbx_mw) * MW_TJ, fa.shifting != 0, sm);
  } else if (blk < fa.nb_mw + fa.nb_win) {
    window_row<R, M1>(fa.gn, f, d0, d1, fa.fp64_rows, (blk - fa.nb_mw) * MW_T + threadIdx.x);
  } else {
    const int t = 2 * (blk - fa.nb_mw - fa.nb_win) + threadIdx.x / (TX * TR);
    const int lt = threadIdx.x % (TX * TR);
    cell_scan_tile(fa.gn, t, lt, fa.ccount, fa.ccur, fa.hist, s_a + (threadIdx.x / (TX * TR)) * (TX * TR));
  }
}

// before a sort: the injected column's items and slots added to the layout
// in use, then the next layout (one group): rebuilt from the tile totals
// before a cell sort, from the arrivals before a tile sort
constexpr int SCAN_T = 1024;
__global__ __launch_bounds__(SCAN_T) void k_layout_scan(FieldArgs fa) {
  __shared__ int s_w[SCAN_T / 64];
  bump_pending(fa.gn, fa.in, fa.pending);
  __syncthreads();
  if (fa.presort == SCAT_CELL) {
    full_layout<SCAN_T>(fa.gn, fa.hist, fa.out, fa.capacity, fa.inj_max, fa.reserve, fa.entering, fa.max_items,
                        fa.err, s_w);
    // The cell order is gathered once the overflow ranges used since the last
    // rebuild exceed 1/32 of the segments: the particles have moved, and a
    // direct scatter of whole records from the momentum pass would write
    // partial cache lines of every record array.  While the particles are
    // still close to cell order the pass scatters them directly (cheaper).
    __syncthreads();
    if (threadIdx.x == 0) {
      const long long seg = fa.in.offsets[fa.gn.ntiles], over = (long long)*fa.in.fill - seg;
      if (over * 32 > seg) {
        *fa.out.mode = LAYOUT_FULL | LAYOUT_GATHER;
        fa.stats[2] += 1;
      }
    }
  } else {
    move_layout<SCAN_T>(fa.gn, fa.hist, fa.arr, fa.in, fa.out, fa.capacity, fa.inj_max, fa.reserve, fa.entering,
                        fa.max_items, fa.err, fa.stats, s_w);
  }
}

// ---------------------------------------------------- initial envelope --
// Paraxial Gaussian: a0 exp(-r^2/(w0^2 q))/q exp(-(x - x_c - t)^2/sigma^2),
// q = 1 + i (x - x_f)/Z_R, Z_R = w0^2/2, sigma = tau/(2 sqrt(ln 2)), at
// t = 0 (A^0) and t = -dt (A^{-1}); zero on the Dirichlet boundary nodes.
__device__ inline double2 pulse_at(const Laser& L, double x, double r, double t) {
  if (L.a0 == 0.0) return make_double2(0.0, 0.0);
  const double zr = 0.5 * L.w0 * L.w0;
  const double qi = (x - L.x_f) / zr;  // q = 1 + i qi
  const double den = 1.0 + qi * qi;
  // 1/q = (1 - i qi)/den ; -r^2/(w0^2 q) = -r^2 (1 - i qi)/(w0^2 den)
  const double er = -r * r / (L.w0 * L.w0 * den), ei = r * r * qi / (L.w0 * L.w0 * den);
  const double sig = L.tau / (2.0 * sqrt(log(2.0)));
  const double xi = x - L.x_c - t;
  const double mag = L.a0 * exp(er) * exp(-xi * xi / (sig * sig)) / den;
  double sn, cs;
  sincos(ei, &sn, &cs);
  // (cs + i sn)(1 - i qi)
  return make_double2(mag * (cs + sn * qi), mag * (sn - cs * qi));
}

template <class R>
__global__ void k_init_envelope(Geo g, Grids<R> f, Laser L, int fp64_rows) {
  using C = typename cplx_of<R>::type;
  const int nr1 = g.nr + 1;
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (long long)(g.nx + 1) * nr1) return;
  const int i = (int)(idx / nr1), j = (int)(idx - (long long)i * nr1);
  const int pc = phys_col(g, i);
  const size_t o = (size_t)pc * g.pitch + j;
  const bool edge = i == 0 || i == g.nx || j == g.nr;
  const double x = (double)(g.shift + i) * g.dx, r = j * g.dr;
  const double2 a0 = edge ? make_double2(0.0, 0.0) : pulse_at(L, x, r, 0.0);
  const double2 am = edge ? make_double2(0.0, 0.0) : pulse_at(L, x, r, -g.dt);
  f.env[o] = mk<C>((R)a0.x, (R)a0.y);
  f.envp[o] = mk<C>((R)am.x, (R)am.y);
  if (fp64_rows && j <= 1) {
    f.ax[pc * 2 + j] = a0;
    f.axp[pc * 2 + j] = am;
  }
}

// ------------------------------------------------------------ launchers --
static inline int node_blocks(const Geo& g) {
  const long long n = (long long)(g.nx + 1) * (g.nr + 1);
  return (int)((n + 255) / 256);
}

template <class R>
void launch_envelope(const Geo& g, const Grids<R>& f, const R* chi, int fp64_rows, const SettleArgs<R>& sa,
                     hipStream_t st, const KEvents& ev) {
  launch_k(k_envelope<R>, dim3(node_blocks(g) + sa.blocks), dim3(256), st, ev, g, f, chi, fp64_rows, sa);
}

template <class R>
void launch_field(const Geo& g, const Grids<R>& f, const DepositBufs<R>& din, const DepositBufs<R>& dnext,
                  const DepositBufs<R>& d0, const DepositBufs<R>& d1, FieldArgs fa, hipStream_t st,
                  const KEvents& ev) {
  fa.nbx_mw = (g.nr + 1 + MW_TJ - 1) / MW_TJ;
  fa.nb_mw = fa.nbx_mw * ((g.nx + 1 + MW_TI - 1) / MW_TI);
  fa.nb_win = fa.shifting ? (g.nr + 1 + MW_T - 1) / MW_T : 0;
  const int nb_cs = fa.presort == SCAT_CELL ? (g.ntiles + 1) / 2 : 0;
  const int grid = fa.nb_mw + fa.nb_win + nb_cs;
  // the stage's stop event goes on its last kernel
  const KEvents ev_field{ev.start, fa.presort ? nullptr : ev.stop};
  if (g.modes >= 2)
    launch_k(k_field<R, true>, dim3(grid), dim3(MW_T), st, ev_field, g, f, din, dnext, d0, d1, fa);
  else
    launch_k(k_field<R, false>, dim3(grid), dim3(MW_T), st, ev_field, g, f, din, dnext, d0, d1, fa);
  if (fa.presort) launch_k(k_layout_scan, dim3(1), dim3(SCAN_T), st, KEvents{nullptr, ev.stop}, fa);
}

// ------------------------------------------------- binomial J filter --
// The uncompensated binomial filter of the paper's nonlinear benchmark
// (Sec. 4), read as N passes of 1-2-1 in index space, each along x then
// along r, on J^{n+1/2} of both modes before the field update: zero current
// outside the window and beyond r_max, rows below the axis mirrored with the
// component's parity (axial components (-1)^m, radial and azimuthal
// (-1)^{m+1}); the odd mode-1 J_x is zero on the axis row (it vanishes
// there, and the field update never reads it).
// Zeroing the node beyond an end before every pass is the same as filtering
// the signal extended oddly about that node, and the axis rule is the same
// as filtering its parity extension; 1-2-1 keeps both symmetries, and the x
// and r passes commute (with each other and with those extensions).  So the
// N passes are, exactly, one (2N+1)-tap convolution with the binomial
// weights C(2N, N+m)/4^N along x and one along r, of the extended signal.
// A work group owns one component of a FT x FT tile, loads it with an
// N-node halo (the extension applied at the load) into LDS, convolves along
// x, then along r, and writes the owned nodes to the filtered copy the field
// update reads.
// The grid must be at least N + 1 nodes wide in each direction.
constexpr int FT = 32;                 // owned nodes per tile side
constexpr int FH = ENVPIC_FILTER_MAX;  // largest halo
constexpr int FR = FT + 2 * FH;        // LDS region side (at most)
constexpr int FTH = 256;               // threads of a filter work group

__device__ inline float vscale(float a, float s) { return a * s; }
__device__ inline double vscale(double a, double s) { return a * s; }
__device__ inline float2 vscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }
__device__ inline double2 vscale(double2 a, double s) { return make_double2(a.x * s, a.y * s); }
__device__ inline float vfma(float w, float a, float acc) { return fmaf(w, a, acc); }
__device__ inline double vfma(double w, double a, double acc) { return fma(w, a, acc); }
__device__ inline float2 vfma(float w, float2 a, float2 acc) { return make_float2(fmaf(w, a.x, acc.x), fmaf(w, a.y, acc.y)); }
__device__ inline double2 vfma(double w, double2 a, double2 acc) { return make_double2(fma(w, a.x, acc.x), fma(w, a.y, acc.y)); }

// index of the extended signal's node i in the valid range [0, m] and its
// sign: odd reflection about -1 and about m + 1 (the zeroed neighbours);
// returns -1 where the extension is zero
__device__ inline int reflect_end(int i, int m, float& sign) {
  if (i >= 0 && i <= m) return i;
  if (i == -1 || i == m + 1) return -1;
  sign = -sign;
  return i < 0 ? -2 - i : 2 * (m + 1) - i;
}

// One component of the tile (i0, j0): valid for 0 <= i <= imax, 0 <= j <=
// jmax; half_r: staggered by half a cell in r (the mirror of row j < 0 is
// -1 - j, else -j).  A: FR x FR values (the tile and a halo of FH >= N
// nodes; the outer FH - N rings are not needed), B: FT x FR.
template <class V, class R>
__device__ void filter_component(const Geo& g, const V* __restrict__ src, V* __restrict__ dst, int imax, int jmax,
                                 bool half_r, R parity, int N, const R* cw, int i0, int j0, V* A, V* B) {
  const V zero = vscale(V{}, (R)0);
  const int lo = FH - N, hi = FH + FT + N;  // the region rows and columns used
  // every lane issues all of its loads before it writes any of them to LDS,
  // so that they are in flight together: each load reads a valid address
  // (the array's first element stands in for a node that is not read) and
  // the value is selected afterwards; entries outside the rows and columns
  // used are written as zero and never read
  constexpr int NLD = (FR * FR + FTH - 1) / FTH;
  size_t off[NLD];
  R sc[NLD];
#pragma unroll
  for (int u = 0; u < NLD; ++u) {
    const int k = threadIdx.x + u * FTH;
    const int a = k / FR, b = k - (k / FR) * FR;
    float sx = 1.0f, sr = 1.0f;
    const int i = reflect_end(i0 - FH + a, imax, sx);
    int j = j0 - FH + b;
    if (j < 0) {  // below the axis: the parity mirror
      j = half_r ? -1 - j : -j;
      sr = (float)parity;
    }
    j = reflect_end(j, jmax, sr);
    const bool odd_axis = !half_r && parity < (R)0 && j == 0;  // an odd function's axis value
    const bool ok = k < FR * FR && a >= lo && a < hi && b >= lo && b < hi && i >= 0 && j >= 0 && !odd_axis;
    off[u] = ok ? (size_t)phys_col(g, i) * g.pitch + j : 0;
    sc[u] = ok ? (R)(sx * sr) : (R)0;
  }
  V v[NLD];
#pragma unroll
  for (int u = 0; u < NLD; ++u) v[u] = src[off[u]];
#pragma unroll
  for (int u = 0; u < NLD; ++u) {
    const int k = threadIdx.x + u * FTH;
    if (k < FR * FR) A[k] = sc[u] != (R)0 ? vscale(v[u], sc[u]) : zero;
  }
  __syncthreads();
  // along x: owned columns, the rows used
  for (int k = threadIdx.x; k < FT * FR; k += FTH) {
    const int a = k / FR, b = k - (k / FR) * FR;
    if (b < lo || b >= hi) continue;
    V acc = zero;
    for (int m = 0; m <= 2 * N; ++m) acc = vfma(cw[m], A[(a + lo + m) * FR + b], acc);
    B[k] = acc;
  }
  __syncthreads();
  // along r: owned nodes
  for (int k = threadIdx.x; k < FT * FT; k += FTH) {
    const int a = k / FT, b = k - (k / FT) * FT;
    const int i = i0 + a, j = j0 + b;
    if (i > g.nx || j > g.nr) continue;
    V acc = zero;
    for (int m = 0; m <= 2 * N; ++m) acc = vfma(cw[m], B[a * FR + b + lo + m], acc);
    dst[(size_t)phys_col(g, i) * g.pitch + j] = (i <= imax && j <= jmax) ? acc : zero;
  }
}

// work group: tile blockIdx.x / ncomp, component blockIdx.x % ncomp
template <class R, bool M1>
__global__ __launch_bounds__(FTH) void k_filter(Geo g, DepositBufs<R> din, DepositBufs<R> dout, int N) {
  using C = typename cplx_of<R>::type;
  constexpr int ncomp = M1 ? 5 : 2;
  __shared__ C a_buf[FR * FR];
  __shared__ C b_buf[FT * FR];
  __shared__ R cw[2 * FH + 1];
  const int tile = blockIdx.x / ncomp, comp = blockIdx.x % ncomp;
  const int ntr = (g.nr + 1 + FT - 1) / FT;
  const int i0 = (tile / ntr) * FT, j0 = (tile % ntr) * FT;
  if (threadIdx.x <= 2 * N) {  // binomial weights C(2N, m) / 4^N (exact)
    double c = 1.0;
    for (int q = 0; q < (int)threadIdx.x; ++q) c = c * (2 * N - q) / (q + 1);
    cw[threadIdx.x] = (R)std::ldexp(c, -2 * N);
  }
  __syncthreads();
  R* ra = reinterpret_cast<R*>(a_buf);
  R* rb = reinterpret_cast<R*>(b_buf);
  switch (comp) {
    case 0: filter_component<R, R>(g, din.jx, dout.jx, g.nx - 1, g.nr, false, (R)1, N, cw, i0, j0, ra, rb); break;
    case 1: filter_component<R, R>(g, din.jr, dout.jr, g.nx, g.nr - 1, true, (R)-1, N, cw, i0, j0, ra, rb); break;
    case 2: filter_component<C, R>(g, din.jx1, dout.jx1, g.nx - 1, g.nr, false, (R)-1, N, cw, i0, j0, a_buf, b_buf); break;
    case 3: filter_component<C, R>(g, din.jr1, dout.jr1, g.nx, g.nr - 1, true, (R)1, N, cw, i0, j0, a_buf, b_buf); break;
    default: filter_component<C, R>(g, din.jt1, dout.jt1, g.nx, g.nr, false, (R)1, N, cw, i0, j0, a_buf, b_buf); break;
  }
}

template <class R>
void launch_filter(const Geo& g, const DepositBufs<R>& din, const DepositBufs<R>& dout, int passes, hipStream_t st,
                   const KEvents& ev) {
  if (passes <= 0) return;
  const int tiles = ((g.nx + 1 + FT - 1) / FT) * ((g.nr + 1 + FT - 1) / FT);
  const int grid = tiles * (g.modes >= 2 ? 5 : 2);
  if (g.modes >= 2)
    launch_k(k_filter<R, true>, dim3(grid), dim3(FTH), st, ev, g, din, dout, passes);
  else
    launch_k(k_filter<R, false>, dim3(grid), dim3(FTH), st, ev, g, din, dout, passes);
}

template <class R>
void launch_init_envelope(const Geo& g, const Grids<R>& f, const Laser& L, int fp64_rows, hipStream_t st) {
  hipLaunchKernelGGL((k_init_envelope<R>), dim3(node_blocks(g)), dim3(256), 0, st, g, f, L, fp64_rows);
}

#define ENVPIC_INST(R)                                                                                      \
  template void launch_envelope<R>(const Geo&, const Grids<R>&, const R*, int, const SettleArgs<R>&,        \
                                   hipStream_t, const KEvents&);                                            \
  template void launch_field<R>(const Geo&, const Grids<R>&, const DepositBufs<R>&, const DepositBufs<R>&,   \
                                const DepositBufs<R>&, const DepositBufs<R>&, FieldArgs, hipStream_t,       \
                                const KEvents&);                                                            \
  template void launch_init_envelope<R>(const Geo&, const Grids<R>&, const Laser&, int, hipStream_t);        \
  template void launch_filter<R>(const Geo&, const DepositBufs<R>&, const DepositBufs<R>&, int, hipStream_t, \
                                 const KEvents&);
ENVPIC_INST(float)
ENVPIC_INST(double)
#undef ENVPIC_INST

}  // namespace envpic
