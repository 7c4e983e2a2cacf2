// sort_diag.hip -- the FP64 conserved-sum diagnostics (work-group tree
// reductions, summed in a fixed order).  The counting sort's scans are in
// scan.hpp (run inside the field-stage kernel).
#include "common.hpp"
#include "cplx.hpp"
#include "launch.hpp"

namespace envpic {

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
