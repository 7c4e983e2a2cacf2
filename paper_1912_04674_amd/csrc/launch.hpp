// launch.hpp -- host-side launchers of the envpic kernels (internal).
#pragma once
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include "common.hpp"

namespace envpic {

// Stage timing: events that the command processor stamps when a kernel's
// dispatch starts (start) and when it completes (stop), as the kernel trace
// measures it (no gaps between launches inside the interval).  Null events
// launch the kernel the ordinary way.
struct KEvents {
  hipEvent_t start = nullptr, stop = nullptr;
};
template <typename... Args, typename F = void (*)(Args...)>
inline void launch_k(F kernel, dim3 grid, dim3 block, hipStream_t st, const KEvents& ev, Args... args) {
  if (ev.start || ev.stop)
    hipExtLaunchKernelGGL(kernel, grid, block, 0, st, ev.start, ev.stop, 0, args...);
  else
    hipLaunchKernelGGL(kernel, grid, block, 0, st, args...);
}

// chi and current deposits of one step (double-buffered by step parity)
template <class R> struct DepositBufs {
  using C = typename cplx_of<R>::type;
  R *chi, *jx, *jr;
  C *jx1, *jr1, *jt1;
};

// scatter (SCAT_*): re-sort into the layout Ld, by tile (cursors of Ld) or
// by cell (per-cell cursors ccur); inv (one word per slot) holds the cell
// order's source slots between the pass and the copy that follows it
template <class R>
void launch_momentum(const Geo& g, const Grids<R>& f, R* chi, const Parts<R>& src, const Parts<R>& dst,
                     const Layout& Ls, const Layout& Ld, int* ccur, R* gscr, unsigned* inv, int* err, int grid,
                     bool defer, int scatter, hipStream_t st, const KEvents& ev = KEvents{});
// the plasma of the column entering the window at this step's shift,
// loaded by extra work groups of the position pass (blocks == 0: none)
struct InjectArgs {
  Geo gn;  // geometry after the shift
  Plasma pl;
  long long capacity;
  int max_items;
  int* pending;  // items and slots appended, added to the layout by the field stage
  int blocks;
};
// What a position pass counts for the sort at the next step: nothing
// (mode 0); the particles per cell of x^{n+1} into ccount (SCAT_CELL); or
// the particles per tile into hist and the arrivals (particles of another
// tile's work item) per tile into arr (SCAT_TILE).
struct SortCounts {
  int mode;
  int* ccount;
  int* hist;
  int* arr;
};
template <class R>
void launch_position(const Geo& g, const Grids<R>& f, const DepositBufs<R>& d, const Parts<R>& P, const Layout& L,
                     const SortCounts& sc, int vacate, const Parts<R>& scr, int* err, int grid, bool defer,
                     const InjectArgs& inj, hipStream_t st, const KEvents& ev = KEvents{});
template <class R> int inject_blocks(const Geo& g);
template <class R>
void launch_deposit_chi(const Geo& g, R* chi, const Parts<R>& P, const Layout& L, const R* gscr, int* err, int grid,
                        hipStream_t st);
template <class R>
void launch_deposit_J(const Geo& g, const DepositBufs<R>& d, const Parts<R>& P, const Layout& L, int vacate,
                      const Parts<R>& scr, int* err, int grid, hipStream_t st);
template <class R>
void launch_init_particles(const Geo& g, const Plasma& pl, const Parts<R>& P, const int* offsets, hipStream_t st);

// sa: the copy back of a tile sort that rebuilt its layout, run by extra
// groups of the same launch (it reads no grid the update writes)
template <class R>
void launch_envelope(const Geo& g, const Grids<R>& f, const R* chi, int fp64_rows, const SettleArgs<R>& sa,
                     hipStream_t st,
                     const KEvents& ev = KEvents{});
// `passes` passes of the binomial filter on the currents of din into dout
// (chi is not touched)
template <class R>
void launch_filter(const Geo& g, const DepositBufs<R>& din, const DepositBufs<R>& dout, int passes, hipStream_t st,
                   const KEvents& ev = KEvents{});
// arguments of the field-stage kernel besides the grids and deposits
struct FieldArgs {
  Geo gn;                      // geometry after the window shift (as before it when there is none)
  int shifting, fp64_rows;
  int presort;                 // before a sort: 0 none, SCAT_CELL (cell scans, rebuilt layout), SCAT_TILE (arrivals)
  int nb_mw, nbx_mw, nb_win;   // work-group roles (set by the launcher)
  int* ccount;                 // per-cell counts -> cursors (ccur), tile totals (hist)
  int* ccur;
  int* hist;                   // particles per tile after the sort
  int* arr;                    // arrivals per tile (tile sorts)
  Layout in;                   // the layout in use
  Layout out;                  // the next layout
  long long capacity;
  long long reserve;           // slots kept free past the segments when a layout is rebuilt
  int entering;                // tile columns ahead of the window given a full tile of slots when it is rebuilt
  int inj_max, max_items;
  int* pending;
  int* err;
  int* stats;                  // [incremental, rebuilt] tile-sort layouts, gathered cell sorts
};
// E^{n+1}, B^{n+3/2}, Bbar^{n+1} into the second E/B copies (the caller
// swaps them), the next deposits cleared, the window's column resets (if
// shifting), the per-cell and layout scans (before a sort) or the injected
// column's items added to the layout in use
template <class R>
void launch_field(const Geo& g, const Grids<R>& f, const DepositBufs<R>& din, const DepositBufs<R>& dnext,
                  const DepositBufs<R>& d0, const DepositBufs<R>& d1, FieldArgs fa, hipStream_t st,
                  const KEvents& ev = KEvents{});
template <class R>
void launch_init_envelope(const Geo& g, const Grids<R>& f, const Laser& L, int fp64_rows, hipStream_t st);

// FP64 diagnostics (sort_diag.hip): a fixed number of work groups, so the
// partial sums take diag_scratch_doubles() doubles for any simulation size
constexpr int DIAG_BLOCKS = 1024;
int diag_scratch_doubles();
// device address and size (doubles) of the library's own diagnostics scratch
// on `device` (a file-scope device array; resolved once per device); 0 on
// success
int static_scratch(int device, double** ptr, size_t* doubles);
template <class R>
void launch_diag(const Geo& g, const Parts<R>& P, const Layout& L, const Grids<R>& f, const R* chi, int fp64_rows,
                 double* scratch, double* out, hipStream_t st);

// injected-beam parameters (beam.hip)
constexpr int BEAM_MAX_BINS = 4096;
constexpr int BEAM_PARTS = 8;  // partial sums per work item in each moment pass
struct BeamArgs {
  double e_lo, e_hi, de;  // spectrum range (gamma - 1) and bin width (e_hi - e_lo) / nbins
  double scale;           // fixed-point scale of the histogram: sum |w| scale < 2^62
  int nbins;
};
// slots of the small state vector the beam kernels pass on to each other
enum {
  BS_NONEMPTY = 0, BS_PEAK, BS_FWHM, BS_LO, BS_HI, BS_W, BS_COUNT, BS_QSPEC,
  BS_EMEAN, BS_YMEAN, BS_ZMEAN, BS_PYMEAN, BS_PZMEAN, BEAM_STATE = 16
};
struct BeamScratch {
  unsigned long long* hist;  // [BEAM_MAX_BINS] fixed-point charge per bin
  double* hist_f;            // [BEAM_MAX_BINS] the same as FP64 (charge units)
  double* part;              // [max_items][BEAM_PARTS] per-item partial sums
  double* st;                // [BEAM_STATE]
  double* out;               // [ENVPIC_NBEAM]
};
template <class R>
void launch_beam(const Geo& g, const Parts<R>& P, const Layout& L, int max_items, const BeamArgs& a,
                 const BeamScratch& b, hipStream_t st);

// self-consistent fields of an injected bunch (bunch.hip): conjugate
// gradients on the (nx - 1) x nr interior potential nodes, FP64
constexpr int CG_CHECK = 25;  // iterations between residual reads
constexpr int CG_NS = 8;      // device scalars
struct CgVecs {
  double *x, *r, *p, *p2, *q;  // [unknowns] each (p, p2: two direction buffers)
  double* idiag;          // [nr] inverse diagonal of each row
  double* part;           // [blocks][2] partial sums
  double* s;              // [CG_NS]
};
long long cg_unknowns(int nx, int nr);
int cg_blocks(int nx, int nr);
template <class R>
int bunch_solve(const Geo& g, const Parts<R>& P, const Layout& L, int max_items, const Grids<R>& f,
                unsigned id_lo, unsigned id_hi, double beta, double tol, int max_iter, const CgVecs& v,
                hipStream_t st, int* iters, double* resid);

}  // namespace envpic
