// launch.hpp -- host-side launchers of the envpic kernels (internal).
#pragma once
#include <hip/hip_runtime.h>

#include "common.hpp"

namespace envpic {

// chi and current deposits of one step (double-buffered by step parity)
template <class R> struct DepositBufs {
  using C = typename cplx_of<R>::type;
  R *chi, *jx, *jr;
  C *jx1, *jr1, *jt1;
};

// scatter (SCAT_*): re-sort into the layout Ld, by tile (cursors of Ld) or
// by cell (per-cell cursors ccur)
template <class R>
void launch_momentum(const Geo& g, const Grids<R>& f, R* chi, const Parts<R>& src, const Parts<R>& dst,
                     const Layout& Ls, const Layout& Ld, int* ccur, R* gscr, int* err, int grid, bool defer,
                     int scatter, hipStream_t st);
// count_cells: add the particles' new cells into ccount (before a sort)
template <class R>
void launch_position(const Geo& g, const Grids<R>& f, const DepositBufs<R>& d, const Parts<R>& P, const Layout& L,
                     int* ccount, int vacate, int count_cells, const Parts<R>& scr, int* err, int grid, bool defer,
                     hipStream_t st);
template <class R>
void launch_deposit_chi(const Geo& g, R* chi, const Parts<R>& P, const Layout& L, const R* gscr, int* err, int grid,
                        hipStream_t st);
template <class R>
void launch_deposit_J(const Geo& g, const DepositBufs<R>& d, const Parts<R>& P, const Layout& L, int vacate,
                      const Parts<R>& scr, int* err, int grid, hipStream_t st);
template <class R>
void launch_init_particles(const Geo& g, const Plasma& pl, const Parts<R>& P, const int* offsets, hipStream_t st);
template <class R>
void launch_inject(const Geo& g, const Plasma& pl, const Parts<R>& P, const Layout& L, int* ccount, int count_cells,
                   long long capacity, int max_items, int* pending, int* err, hipStream_t st);

template <class R>
void launch_envelope(const Geo& g, const Grids<R>& f, const R* chi, int fp64_rows, hipStream_t st);
template <class R>
void launch_maxwell(const Geo& g, const Grids<R>& f, const DepositBufs<R>& din, const DepositBufs<R>& dnext,
                    hipStream_t st);
template <class R>
void launch_window(const Geo& g, const Grids<R>& f, const DepositBufs<R>& d0, const DepositBufs<R>& d1,
                   int fp64_rows, hipStream_t st);
template <class R>
void launch_init_envelope(const Geo& g, const Grids<R>& f, const Laser& L, int fp64_rows, hipStream_t st);

// per tile: exclusive scan of its cells' counts into the per-cell cursors
// (cell order within the tile), the tile total into hist, counts cleared
void launch_cell_scan(const Geo& g, int* ccount, int* ccur, int* hist, hipStream_t st);
// the items (pending[0]) and slots (pending[1]) appended by an injection
// are first added to *bump_items and *bump_fill of the layout in use; with
// sort = 0 that is all it does
void launch_scan(const Geo& g, int* hist, const Layout& out, long long capacity, int inj_max, int max_items,
                 int* bump_items, int* bump_fill, int* pending, int* err, int sort, hipStream_t st);

int diag_scratch_doubles(int max_items, const Geo& g);
template <class R>
void launch_diag(const Geo& g, const Parts<R>& P, const Layout& L, int max_items, const Grids<R>& f, const R* chi,
                 int fp64_rows, double* scratch, double* out, hipStream_t st);

}  // namespace envpic
