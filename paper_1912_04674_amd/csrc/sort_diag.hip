// sort_diag.hip -- the FP64 conserved-sum diagnostics: charge, chi V,
// kinetic energy, field energy, envelope norm, L_x, P_x and a non-finite
// count of the state.  (The counting sort's scans are in scan.hpp, run inside
// the field-stage kernel.)
//
// Reduction order is fixed, so a sum is bitwise the same from run to run:
//   * a fixed number of work groups (DIAG_BLOCKS) strides over the work
//     items (particle sums) or the grid nodes (grid sums), each thread adding
//     its own elements in index order;
//   * each wavefront sums its 64 lanes with a shuffle butterfly (lanes l and
//     l ^ m exchange and add, m = 32 .. 1; IEEE addition is commutative, so
//     every lane ends with the same total);
//   * the group adds its wavefronts' totals in wavefront order, and a last
//     one-group kernel adds the groups' totals, lane-strided, then one more
//     butterfly.
// The partial sums need DIAG_BLOCKS * (NPD + NGD) doubles whatever the
// simulation's size.
#include <mutex>

#include "common.hpp"
#include "cplx.hpp"
#include "launch.hpp"

namespace envpic {

constexpr int DG = 256;            // threads per group (4 wavefronts)
constexpr int DWAVES = DG / 64;
constexpr int NPD = 6;             // count, charge, kinetic energy, L_x, P_x, non-finite
constexpr int NGD = 5;             // chi V, |A|^2 V, mode-0 energy, mode-1 energy, non-finite

// sum of v over the lanes of this wavefront, in the same order on every call
__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
  return v;
}

// the group's sums of v[0..N) into out[0..N): wavefront butterflies, then
// the wavefront totals in wavefront order
template <int N>
__device__ inline void group_sum(const double (&v)[N], double* out) {
  __shared__ double wv[DWAVES][N];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < N; ++k) {
    const double s = wave_sum(v[k]);
    if (lane == 0) wv[wave][k] = s;
  }
  __syncthreads();
  if (threadIdx.x < N) {
    double s = 0.0;
    for (int w = 0; w < DWAVES; ++w) s += wv[w][threadIdx.x];
    out[threadIdx.x] = s;
  }
}

// per group: count, charge, kinetic energy, L_x, P_x, non-finite count over
// the work items b, b + DIAG_BLOCKS, ...
template <class R>
__global__ __launch_bounds__(DG) void k_diag_particles(Geo g, Parts<R> P, Layout L, double* __restrict__ part) {
  double v[NPD] = {0, 0, 0, 0, 0, 0};
  const int n_items = *L.n_items;
  for (int item = blockIdx.x; item < n_items; item += DIAG_BLOCKS) {
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
      v[2] += w * p2 / (1.0 + sqrt(1.0 + p2));  // w (gamma - 1) without cancellation
      v[3] += w * r * (c * pz - s * py);        // y p_z - z p_y
      v[4] += w * px;
      const double vals[7] = {w, px, py, pz, fr, th, fx};
      for (int e = 0; e < 7; ++e)
        if (!isfinite(vals[e])) v[5] += 1.0;
    }
  }
  group_sum<NPD>(v, part + (size_t)blockIdx.x * NPD);
}

// per group: sum chi V, sum |A|^2 V, mode-0 and mode-1 field energy sums,
// non-finite count over the nodes idx = (b + k DIAG_BLOCKS) DG + t
template <class R>
__global__ __launch_bounds__(DG) void k_diag_grid(Geo g, Grids<R> f, const R* __restrict__ chi, int fp64_rows,
                                                  double* __restrict__ part) {
  using C = typename cplx_of<R>::type;
  double v[NGD] = {0, 0, 0, 0, 0};
  const int nr1 = g.nr + 1;
  const long long nodes = (long long)(g.nx + 1) * nr1;
  const double pi = 3.14159265358979323846;
  for (long long idx = (long long)blockIdx.x * DG + threadIdx.x; idx < nodes; idx += (long long)DIAG_BLOCKS * DG) {
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
    v[0] += ch * vn;
    v[1] += (ar * ar + ai * ai) * vn;
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
  group_sum<NGD>(v, part + (size_t)blockIdx.x * NGD);
}

// the groups' sums in a fixed order (wavefront q sums quantity q), mapped
// onto the public diagnostics vector
__global__ __launch_bounds__(64 * (NPD + NGD)) void k_diag_final(const double* __restrict__ pp,
                                                                 const double* __restrict__ pg,
                                                                 double* __restrict__ out) {
  __shared__ double t[NPD + NGD];
  const int q = threadIdx.x >> 6, l = threadIdx.x & 63;
  double s = 0.0;
  if (q < NPD) {
    for (int b = l; b < DIAG_BLOCKS; b += 64) s += pp[(size_t)b * NPD + q];
  } else {
    for (int b = l; b < DIAG_BLOCKS; b += 64) s += pg[(size_t)b * NGD + (q - NPD)];
  }
  s = wave_sum(s);
  if (l == 0) t[q] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    // pp: count, charge, kinetic, L_x, P_x, non-finite;
    // pg: chi V, |A|^2 V, mode-0 energy, mode-1 energy, non-finite
    out[0] = t[0];
    out[1] = t[1];
    out[2] = t[NPD + 0];
    out[3] = t[2];
    // a mode-1 amplitude F carries a mean square |F|^2 / 2 over the azimuth
    out[4] = 0.5 * t[NPD + 2] + 0.25 * t[NPD + 3];
    out[5] = t[NPD + 1];
    out[6] = t[3];
    out[7] = t[4];
    out[8] = t[5] + t[NPD + 4];
  }
}

int diag_scratch_doubles() { return DIAG_BLOCKS * (NPD + NGD); }

// The partial sums of the allocation-free diagnostics entry point: one copy
// per GPU the library runs on, held until the process ends.  Host code never
// passes this name to a kernel: it is a host-side stand-in, and the device
// address comes from hipGetSymbolAddress, per device (static_scratch below).
constexpr int STATIC_SCRATCH_DOUBLES = DIAG_BLOCKS * (NPD + NGD);
static __device__ __align__(256) double scratch[STATIC_SCRATCH_DOUBLES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_addr[kMaxDevices] = {};
}  // namespace

int static_scratch(int device, double** ptr, size_t* doubles) {
  if (device < 0 || device >= kMaxDevices) return -1;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_addr[device]) {
    int cur = -1;
    if (hipGetDevice(&cur) != hipSuccess) return -1;
    if (cur != device && hipSetDevice(device) != hipSuccess) return -1;
    void* a = nullptr;
    const hipError_t e = hipGetSymbolAddress(&a, HIP_SYMBOL(scratch));
    if (cur != device) (void)hipSetDevice(cur);
    if (e != hipSuccess || !a) return -1;
    g_scratch_addr[device] = static_cast<double*>(a);
  }
  *ptr = g_scratch_addr[device];
  *doubles = STATIC_SCRATCH_DOUBLES;
  return 0;
}

template <class R>
void launch_diag(const Geo& g, const Parts<R>& P, const Layout& L, const Grids<R>& f, const R* chi, int fp64_rows,
                 double* scratch, double* out, hipStream_t st) {
  double* pp = scratch;
  double* pg = scratch + (size_t)DIAG_BLOCKS * NPD;
  hipLaunchKernelGGL((k_diag_particles<R>), dim3(DIAG_BLOCKS), dim3(DG), 0, st, g, P, L, pp);
  hipLaunchKernelGGL((k_diag_grid<R>), dim3(DIAG_BLOCKS), dim3(DG), 0, st, g, f, chi, fp64_rows, pg);
  hipLaunchKernelGGL(k_diag_final, dim3(1), dim3(64 * (NPD + NGD)), 0, st, pp, pg, out);
}

template void launch_diag<float>(const Geo&, const Parts<float>&, const Layout&, const Grids<float>&, const float*,
                                 int, double*, double*, hipStream_t);
template void launch_diag<double>(const Geo&, const Parts<double>&, const Layout&, const Grids<double>&,
                                  const double*, int, double*, double*, hipStream_t);

}  // namespace envpic
