// sort_diag.hip -- the counting-sort scan of the per-tile histogram into the
// next particle layout and its work items, and the FP64 conserved-sum
// diagnostics (wavefront/work-group tree reductions, summed in a fixed order).
#include "common.hpp"
#include "cplx.hpp"
#include "launch.hpp"

namespace envpic {

// ------------------------------------------------------------ cell scan --
// One work group per tile: exclusive scan of its 16 x 16 cells' counts
// (column-major, radius fastest) into the per-cell cursors the scatter
// reserves from, the tile total into hist, and the counts cleared.
__global__ __launch_bounds__(TX * TR) void k_cell_scan(Geo g, int* __restrict__ ccount, int* __restrict__ ccur,
                                                       int* __restrict__ hist) {
  __shared__ int s[TX * TR];
  const int t = blockIdx.x;
  const int tcx = t / g.ntr, tcr = t - (t / g.ntr) * g.ntr;
  const int a = threadIdx.x / TR, b = threadIdx.x - (threadIdx.x / TR) * TR;
  const long long col = (long long)lab_tile(g, tcx) * TX + a;
  const int rel = (int)(col - g.shift), j = tcr * TR + b;
  const bool valid = rel >= 0 && rel < g.nx && j < g.nr;
  const size_t o = valid ? (size_t)phys_col(g, rel) * g.pitch + j : 0;
  const int c = valid ? ccount[o] : 0;
  s[threadIdx.x] = c;
  __syncthreads();
  for (int off = 1; off < TX * TR; off <<= 1) {
    const int v = (int)threadIdx.x >= off ? s[threadIdx.x - off] : 0;
    __syncthreads();
    s[threadIdx.x] += v;
    __syncthreads();
  }
  if (valid) {
    ccur[o] = s[threadIdx.x] - c;
    ccount[o] = 0;
  }
  if (threadIdx.x == TX * TR - 1) hist[t] = s[threadIdx.x];
}

void launch_cell_scan(const Geo& g, int* ccount, int* ccur, int* hist, hipStream_t st) {
  hipLaunchKernelGGL(k_cell_scan, dim3(g.ntiles), dim3(TX * TR), 0, st, g, ccount, ccur, hist);
}

// ----------------------------------------------------------------- scan --
// One work group of 1024 threads: exclusive scan of the tile totals into
// offsets (and the scatter cursors), work items (a tile of v particles gives
// ceil(v / chunk) items of equal size), and a reset of the histogram for the
// next step.  Flags when the particles plus one injected column would not
// fit.
constexpr int SCAN_T = 1024;

__global__ __launch_bounds__(SCAN_T) void k_scan(Geo g, int* __restrict__ hist, Layout out, long long capacity,
                                                 int inj_max, int max_items, int* bump_items, int* bump_fill,
                                                 int* pending, int* err, int sort) {
  __shared__ int s_c[SCAN_T], s_m[SCAN_T];
  const int nt = g.ntiles;
  const int tid = threadIdx.x;
  if (tid == 0 && pending != nullptr && pending[0] != 0) {
    *bump_items += pending[0];  // items and slots of the column injected before this scan
    *bump_fill += pending[1];
    pending[0] = 0;
    pending[1] = 0;
  }
  if (!sort) return;
  const int per = (nt + SCAN_T - 1) / SCAN_T;
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
  for (int off = 1; off < SCAN_T; off <<= 1) {
    const int vc = tid >= off ? s_c[tid - off] : 0;
    const int vm = tid >= off ? s_m[tid - off] : 0;
    __syncthreads();
    s_c[tid] += vc;
    s_m[tid] += vm;
    __syncthreads();
  }
  int ec = s_c[tid] - c, em = s_m[tid] - m;
  const int total = s_c[SCAN_T - 1], n_items = s_m[SCAN_T - 1];
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
  if (tid == SCAN_T - 1) {
    out.offsets[nt] = total;
    *out.fill = total;
    *out.n_items = min(n_items, item_cap);
    if (n_items > item_cap) atomicOr(err, ERR_ITEMS);
    if ((long long)total + (long long)SORT_EVERY * inj_max > capacity) atomicOr(err, ERR_CAPACITY);
  }
}

void launch_scan(const Geo& g, int* hist, const Layout& out, long long capacity, int inj_max, int max_items,
                 int* bump_items, int* bump_fill, int* pending, int* err, int sort, hipStream_t st) {
  hipLaunchKernelGGL(k_scan, dim3(1), dim3(sort ? SCAN_T : 64), 0, st, g, hist, out, capacity, inj_max, max_items,
                     bump_items, bump_fill, pending, err, sort);
}

// ---------------------------------------------------------- diagnostics --
constexpr int DG = 256;

template <int N>
__device__ inline void block_sum(double (&v)[N], double* red /* [N][DG] */, double* out) {
  for (int k = 0; k < N; ++k) red[k * DG + threadIdx.x] = v[k];
  __syncthreads();
  for (int s = DG / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s)
      for (int k = 0; k < N; ++k) red[k * DG + threadIdx.x] += red[k * DG + threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x < N) out[threadIdx.x] = red[threadIdx.x * DG];
}

// per work item: count, charge, kinetic energy, L_x, P_x, non-finite count
constexpr int NPD = 6;
template <class R>
__global__ __launch_bounds__(DG) void k_diag_particles(Geo g, Parts<R> P, Layout L, double* __restrict__ part) {
  __shared__ double red[NPD * DG];
  double v[NPD] = {0, 0, 0, 0, 0, 0};
  const int item = blockIdx.x;
  if (item < *L.n_items) {
    const int4 it = L.items[item];
    for (int k = threadIdx.x; k < it.z; k += DG) {
      const int p = it.y + k;
      const unsigned cw = P.cell[p];
      if (cw == kDead) continue;
      const double w = P.w[p], px = P.px[p], py = P.py[p], pz = P.pz[p];
      const double fr = P.fr[p], th = P.th[p], fx = P.fx[p];
      const double r = (cell_jr(cw) + fr) * g.dr;
      double s, c;
      sincos(th, &s, &c);
      const double p2 = px * px + py * py + pz * pz;
      v[0] += 1.0;
      v[1] += -w;
      v[2] += w * p2 / (1.0 + sqrt(1.0 + p2));
      v[3] += w * r * (c * pz - s * py);  // y p_z - z p_y
      v[4] += w * px;
      const double vals[7] = {w, px, py, pz, fr, th, fx};
      for (int e = 0; e < 7; ++e)
        if (!isfinite(vals[e])) v[5] += 1.0;
    }
  }
  block_sum<NPD>(v, red, part + (size_t)item * NPD);
}

// per block of nodes: sum chi V, sum |A|^2 V, mode-0 and mode-1 energy, non-finite count
constexpr int NGD = 5;
template <class R>
__global__ __launch_bounds__(DG) void k_diag_grid(Geo g, Grids<R> f, const R* __restrict__ chi, int fp64_rows,
                                                  double* __restrict__ part) {
  using C = typename cplx_of<R>::type;
  __shared__ double red[NGD * DG];
  double v[NGD] = {0, 0, 0, 0, 0};
  const int nr1 = g.nr + 1;
  const long long idx = (long long)blockIdx.x * DG + threadIdx.x;
  if (idx < (long long)(g.nx + 1) * nr1) {
    const double pi = 3.14159265358979323846;
    const int i = (int)(idx / nr1), j = (int)(idx - (long long)i * nr1);
    const int pc = phys_col(g, i);
    const size_t o = (size_t)pc * g.pitch + j;
    const double vn = j == 0 ? pi * g.dr * g.dr * g.dx * 0.25 : 2.0 * pi * j * g.dr * g.dr * g.dx;
    const double vh = 2.0 * pi * (j + 0.5) * g.dr * g.dr * g.dx;
    double ar, ai;
    if (fp64_rows && j <= 1) {
      ar = f.ax[pc * 2 + j].x;
      ai = f.ax[pc * 2 + j].y;
    } else {
      ar = f.env[o].x;
      ai = f.env[o].y;
    }
    const double ch = chi[o];
    v[0] = ch * vn;
    v[1] = (ar * ar + ai * ai) * vn;
    const double ex = f.ex[o], er = f.er[o], bt = f.bt[o];
    if (i <= g.nx - 1) v[2] += ex * ex * vn;
    if (j <= g.nr - 1) v[2] += er * er * vh;
    if (i <= g.nx - 1 && j <= g.nr - 1) v[2] += bt * bt * vh;
    const double vals[7] = {ch, ar, ai, ex, er, bt, (double)f.btb[o]};
    for (int e = 0; e < 7; ++e)
      if (!isfinite(vals[e])) v[4] += 1.0;
    if (g.modes >= 2) {
      const C ex1 = f.ex1[o], er1 = f.er1[o], et1 = f.et1[o], bx1 = f.bx1[o], br1 = f.br1[o], bt1 = f.bt1[o];
      if (i <= g.nx - 1) v[3] += (double)cnorm(ex1) * vn;
      if (j <= g.nr - 1) v[3] += (double)cnorm(er1) * vh;
      v[3] += (double)cnorm(et1) * vn;
      if (j <= g.nr - 1) v[3] += (double)cnorm(bx1) * vh;
      if (i <= g.nx - 1) v[3] += (double)cnorm(br1) * vn;
      if (i <= g.nx - 1 && j <= g.nr - 1) v[3] += (double)cnorm(bt1) * vh;
    }
  }
  block_sum<NGD>(v, red, part + (size_t)blockIdx.x * NGD);
}

// fixed-order final sums (one thread per quantity)
__global__ void k_diag_final(const double* __restrict__ pp, int np_blocks, const double* __restrict__ pg,
                             int ng_blocks, double* __restrict__ out) {
  // wavefront q sums quantity q: lane l takes blocks l, l + 64, ..., then a
  // fixed-order tree over the lanes (the result does not depend on timing)
  __shared__ double lanes[NPD + NGD][64];
  const int q = threadIdx.x / 64, l = threadIdx.x % 64;
  double s = 0.0;
  if (q < NPD) {
    for (int b = l; b < np_blocks; b += 64) s += pp[(size_t)b * NPD + q];
  } else if (q < NPD + NGD) {
    for (int b = l; b < ng_blocks; b += 64) s += pg[(size_t)b * NGD + (q - NPD)];
  }
  if (q < NPD + NGD) lanes[q][l] = s;
  __syncthreads();
  for (int h = 32; h > 0; h >>= 1) {
    if (q < NPD + NGD && l < h) lanes[q][l] += lanes[q][l + h];
    __syncthreads();
  }
  // map onto the public diagnostics vector
  // pp: 0 count, 1 charge, 2 kin, 3 lx, 4 px, 5 nonfinite
  // pg: 0 chi V, 1 |A|^2 V, 2 u0, 3 u1, 4 nonfinite
  __shared__ double t[NPD + NGD];
  if (l == 0 && q < NPD + NGD) t[q] = lanes[q][0];
  __syncthreads();
  if (threadIdx.x == 0) {
    out[0] = t[0];
    out[1] = t[1];
    out[2] = t[NPD + 0];
    out[3] = t[2];
    out[4] = 0.5 * t[NPD + 2] + 0.25 * t[NPD + 3];
    out[5] = t[NPD + 1];
    out[6] = t[3];
    out[7] = t[4];
    out[8] = t[5] + t[NPD + 4];
  }
}

int diag_scratch_doubles(int max_items, const Geo& g) {
  const long long nb = ((long long)(g.nx + 1) * (g.nr + 1) + DG - 1) / DG;
  return max_items * NPD + (int)nb * NGD;
}

template <class R>
void launch_diag(const Geo& g, const Parts<R>& P, const Layout& L, int max_items, const Grids<R>& f, const R* chi,
                 int fp64_rows, double* scratch, double* out, hipStream_t st) {
  const int nb = (int)(((long long)(g.nx + 1) * (g.nr + 1) + DG - 1) / DG);
  double* pp = scratch;
  double* pg = scratch + (size_t)max_items * NPD;
  hipLaunchKernelGGL((k_diag_particles<R>), dim3(max_items), dim3(DG), 0, st, g, P, L, pp);
  hipLaunchKernelGGL((k_diag_grid<R>), dim3(nb), dim3(DG), 0, st, g, f, chi, fp64_rows, pg);
  hipLaunchKernelGGL(k_diag_final, dim3(1), dim3(64 * (NPD + NGD)), 0, st, pp, max_items, pg, nb, out);
}

template void launch_diag<float>(const Geo&, const Parts<float>&, const Layout&, int, const Grids<float>&,
                                 const float*, int, double*, double*, hipStream_t);
template void launch_diag<double>(const Geo&, const Parts<double>&, const Layout&, int, const Grids<double>&,
                                  const double*, int, double*, double*, hipStream_t);

}  // namespace envpic
