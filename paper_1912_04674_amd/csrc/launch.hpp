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

template <class R>
void launch_momentum(const Geo& g, const Grids<R>& f, R* chi, const Parts<R>& src, const Parts<R>& dst,
                     const Layout& Ls, const Layout& Ld, R* gscr, int* err, int grid, bool defer, bool scatter,
                     hipStream_t st);
template <class R>
void launch_position(const Geo& g, const Grids<R>& f, const DepositBufs<R>& d, const Parts<R>& P, const Layout& L,
                     int* hist, int vacate, const Parts<R>& scr, int* err, int grid, bool defer, hipStream_t st);
template <class R>
void launch_deposit_chi(const Geo& g, R* chi, const Parts<R>& P, const Layout& L, const R* gscr, int* err, int grid,
                        hipStream_t st);
template <class R>
void launch_deposit_J(const Geo& g, const DepositBufs<R>& d, const Parts<R>& P, const Layout& L, int vacate,
                      const Parts<R>& scr, int* err, int grid, hipStream_t st);
template <class R>
void launch_init_particles(const Geo& g, const Plasma& pl, const Parts<R>& P, const int* offsets, hipStream_t st);
template <class R>
void launch_inject(const Geo& g, const Plasma& pl, const Parts<R>& P, const Layout& L, int* hist, long long capacity,
                   int max_items, int* pending, int* err, hipStream_t st);
template <class R>
void launch_hist(const Geo& g, const Parts<R>& P, const Layout& L, int* hist, int grid, hipStream_t st);

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

// the items (pending[0]) and slots (pending[1]) appended by an injection
// are first added to *bump_items and *bump_fill of the layout in use
void launch_scan(const Geo& g, int* hist, const Layout& out, long long capacity, int inj_max, int max_items,
                 int* bump_items, int* bump_fill, int* pending, int* err, hipStream_t st);

int diag_scratch_doubles(int max_items, const Geo& g);
template <class R>
void launch_diag(const Geo& g, const Parts<R>& P, const Layout& L, int max_items, const Grids<R>& f, const R* chi,
                 int fp64_rows, double* scratch, double* out, hipStream_t st);

}  // namespace envpic
