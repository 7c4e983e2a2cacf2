// bunch.hip -- self-consistent initial fields of an externally injected
// relativistic electron bunch (arXiv:1912.04674, Sec. 3: the field
// initialisation of external injection carries over to cylindrical
// symmetry).  The bunch moves along x with velocity beta; its potential
// solves the relativistic Poisson equation
//     (1/gamma^2) d2phi/dx2 + (1/r) d/dr (r dphi/dr) = -rho
// on the primal nodes, discretised so that the Gauss law of the field update
// holds exactly:
//     E_x(i+1/2, j) = -(phi_{i+1,j} - phi_{i,j}) / (gamma^2 dx),
//     E_r(i, j+1/2) = -(phi_{i,j+1} - phi_{i,j}) / dr,
//     B_theta(i+1/2, j+1/2) = beta (E_r(i, j+1/2) + E_r(i+1, j+1/2)) / 2,
// with phi = 0 on the x ends and at r_max.  Multiplied by the node volume
// V_j the system K phi = q sum w S is symmetric positive definite:
//     (K phi)_{ij} = V_j/(gamma^2 dx^2) (2 phi_ij - phi_{i-1,j} - phi_{i+1,j})
//                  + A_{j+1/2}/dr (phi_ij - phi_{i,j+1})
//                  + A_{j-1/2}/dr (phi_ij - phi_{i,j-1}),
// A_{j+1/2} = 2 pi (j + 1/2) dr dx, A_{-1/2} = 0, V_0 = pi dr^2 dx / 4.
//
// Solved by conjugate gradients with the diagonal as preconditioner, in
// FP64.  Per iteration: a stencil kernel that forms the new direction
// p = r/diag + beta p_old on the fly for its node and the four neighbours
// (two direction buffers, swapped by the host), applies K and sums p.Kp per
// block; an update kernel (x, r and the partial sums of r.z and r.r); and two
// one-group reductions in a fixed order, so a solve is reproducible.  The
// scalars stay on the device; the host reads the residual every CG_CHECK
// iterations.
#include <algorithm>

#include "common.hpp"
#include "launch.hpp"

namespace envpic {

constexpr int SB = 256;  // threads of the grid kernels

struct CgOp {
  int ni, nj;       // unknowns: interior columns i = 1 .. nx-1, rows j = 0 .. nr-1
  double g2;        // 1 / gamma^2
  double dx, dr;
};

__device__ inline double vol_j(const CgOp& o, int j) {
  const double pi = 3.14159265358979323846;
  return j == 0 ? pi * o.dr * o.dr * o.dx * 0.25 : 2.0 * pi * j * o.dr * o.dr * o.dx;
}
__device__ inline double face_j(const CgOp& o, int j) {  // A_{j+1/2} / dr
  const double pi = 3.14159265358979323846;
  return 2.0 * pi * (j + 0.5) * o.dx;
}
__device__ inline double diag_j(const CgOp& o, int j) {
  const double cx = vol_j(o, j) * o.g2 / (o.dx * o.dx);
  return 2.0 * cx + face_j(o, j) + (j >= 1 ? face_j(o, j - 1) : 0.0);
}

// q sum w S of the particles with id in [id_lo, id_hi) onto the unknowns
// (boundary nodes hold none), with the loop's shape and the axis fold
template <class R>
__global__ __launch_bounds__(SB) void k_bunch_charge(Geo g, Parts<R> P, Layout L, unsigned id_lo, unsigned id_hi,
                                                     CgOp o, double* __restrict__ rhs) {
  const int item = blockIdx.x;
  if (item >= *L.n_items) return;
  const int4 it = L.items[item];
  for (int k = threadIdx.x; k < it.z; k += SB) {
    const int p = it.y + k;
    const unsigned cw = P.cell[p];
    if (cw == kDead) continue;
    const unsigned id = P.id[p];
    if (id < id_lo || id >= id_hi) continue;
    const double ux = (double)((long long)cell_ix(cw) - g.shift) + (double)P.fx[p];
    const double ur = (double)cell_jr(cw) + (double)P.fr[p];
    const double w = -(double)P.w[p];  // q = -1
    int i0, j0, n;
    double wx[3], wr[3];
    if (g.order == 2) {
      const double mx = floor(ux + 0.5), dxo = ux - mx, mr = floor(ur + 0.5), dro = ur - mr;
      i0 = (int)mx - 1;
      j0 = (int)mr - 1;
      n = 3;
      wx[0] = 0.5 * (0.5 - dxo) * (0.5 - dxo);
      wx[1] = 0.75 - dxo * dxo;
      wx[2] = 0.5 * (0.5 + dxo) * (0.5 + dxo);
      wr[0] = 0.5 * (0.5 - dro) * (0.5 - dro);
      wr[1] = 0.75 - dro * dro;
      wr[2] = 0.5 * (0.5 + dro) * (0.5 + dro);
    } else {
      const double fx0 = floor(ux), fr0 = floor(ur);
      i0 = (int)fx0;
      j0 = (int)fr0;
      n = 2;
      wx[0] = 1.0 - (ux - fx0);
      wx[1] = ux - fx0;
      wr[0] = 1.0 - (ur - fr0);
      wr[1] = ur - fr0;
      wx[2] = wr[2] = 0.0;
    }
    for (int a = 0; a < n; ++a) {
      const int i = i0 + a;
      if (i < 1 || i > o.ni) continue;
      for (int b = 0; b < n; ++b) {
        int j = j0 + b;
        if (j < 0) j = -j;  // below the axis: the mirror row (charge is even)
        if (j >= o.nj) continue;
        atomicAdd(&rhs[(size_t)(i - 1) * o.nj + j], w * wx[a] * wr[b]);
      }
    }
  }
}

template <int N>
__device__ inline void cg_block_sum(double (&v)[N], double* red /* [N][SB] */, double* out) {
  for (int k = 0; k < N; ++k) red[k * SB + threadIdx.x] = v[k];
  __syncthreads();
  for (int s = SB / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s)
      for (int k = 0; k < N; ++k) red[k * SB + threadIdx.x] += red[k * SB + threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x < N) out[(size_t)blockIdx.x * N + threadIdx.x] = red[threadIdx.x * SB];
}

// scalars on the device: [0] r.z, [1] alpha, [2] beta, [3] r.r, [4] b.b
enum { CG_RZ = 0, CG_ALPHA, CG_BETA, CG_RR, CG_BB };

__global__ __launch_bounds__(SB) void k_cg_zero(double* __restrict__ a, long long n) {
  const long long k = (long long)blockIdx.x * SB + threadIdx.x;
  if (k < n) a[k] = 0.0;
}

// the preconditioner: 1 / diag of each row (the diagonal depends on j only)
__global__ __launch_bounds__(SB) void k_cg_idiag(CgOp o, CgVecs v) {
  const int j = blockIdx.x * SB + threadIdx.x;
  if (j < o.nj) v.idiag[j] = 1.0 / diag_j(o, j);
}

// x = 0, p_old = 0 (so the first direction is z); partial sums of r.z, r.r
__global__ __launch_bounds__(SB) void k_cg_start(CgOp o, CgVecs v) {
  __shared__ double red[2 * SB];
  double s[2] = {0.0, 0.0};
  const long long k = (long long)blockIdx.x * SB + threadIdx.x;
  const long long n = (long long)o.ni * o.nj;
  if (k < n) {
    const int j = (int)(k % o.nj);
    const double r = v.r[k], z = r * v.idiag[j];
    v.x[k] = 0.0;
    v.p[k] = 0.0;
    s[0] = r * z;
    s[1] = r * r;
  }
  cg_block_sum<2>(s, red, v.part);
}

// p_new = r / diag + beta p_old (at the node and its neighbours), q = K p_new;
// partial sums of p_new.q
__global__ __launch_bounds__(SB) void k_cg_apply(CgOp o, CgVecs v, const double* __restrict__ p_old,
                                                 double* __restrict__ p_new) {
  __shared__ double red[SB];
  double s[1] = {0.0};
  const long long k = (long long)blockIdx.x * SB + threadIdx.x;
  const long long n = (long long)o.ni * o.nj;
  const double beta = v.s[CG_BETA];
  if (k < n) {
    const int i = (int)(k / o.nj), j = (int)(k - (long long)i * o.nj);
    auto dir = [&](long long m, int jj) { return v.r[m] * v.idiag[jj] + beta * p_old[m]; };
    const double pc = dir(k, j);
    const double cx = vol_j(o, j) * o.g2 / (o.dx * o.dx);
    const double pl = i > 0 ? dir(k - o.nj, j) : 0.0, pr = i < o.ni - 1 ? dir(k + o.nj, j) : 0.0;
    const double pu = j < o.nj - 1 ? dir(k + 1, j + 1) : 0.0, pd = j > 0 ? dir(k - 1, j - 1) : 0.0;
    double q = cx * (2.0 * pc - pl - pr) + face_j(o, j) * (pc - pu);
    if (j > 0) q += face_j(o, j - 1) * (pc - pd);
    p_new[k] = pc;
    v.q[k] = q;
    s[0] = pc * q;
  }
  cg_block_sum<1>(s, red, v.part);
}

// fixed-order sum of NQ partial sums per block into sums[0 .. NQ)
template <int NQ>
__device__ inline void cg_sum_parts(const double* part, int nb, double* sums) {
  __shared__ double lanes[NQ][256];
  const int l = threadIdx.x;
  for (int q = 0; q < NQ; ++q) {
    double s = 0.0;
    for (int b = l; b < nb; b += 256) s += part[(size_t)b * NQ + q];
    lanes[q][l] = s;
  }
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (l < h)
      for (int q = 0; q < NQ; ++q) lanes[q][l] += lanes[q][l + h];
    __syncthreads();
  }
  if (l == 0)
    for (int q = 0; q < NQ; ++q) sums[q] = lanes[q][0];
}

// after k_cg_start: r.z, r.r and b.b (= r.r at the start)
__global__ __launch_bounds__(256) void k_cg_init_scalars(int nb, CgVecs v) {
  __shared__ double t[2];
  cg_sum_parts<2>(v.part, nb, t);
  if (threadIdx.x == 0) {
    v.s[CG_RZ] = t[0];
    v.s[CG_RR] = t[1];
    v.s[CG_BB] = t[1];
    v.s[CG_BETA] = 0.0;
  }
}

// alpha = r.z / p.Kp
__global__ __launch_bounds__(256) void k_cg_alpha(int nb, CgVecs v) {
  __shared__ double t[1];
  cg_sum_parts<1>(v.part, nb, t);
  if (threadIdx.x == 0) v.s[CG_ALPHA] = t[0] != 0.0 ? v.s[CG_RZ] / t[0] : 0.0;
}

// x += alpha p, r -= alpha q; partial sums of r.z (z = r / diag) and r.r
__global__ __launch_bounds__(SB) void k_cg_update(CgOp o, CgVecs v, const double* __restrict__ p) {
  __shared__ double red[2 * SB];
  double s[2] = {0.0, 0.0};
  const long long k = (long long)blockIdx.x * SB + threadIdx.x;
  const long long n = (long long)o.ni * o.nj;
  const double alpha = v.s[CG_ALPHA];
  if (k < n) {
    const int j = (int)(k % o.nj);
    v.x[k] += alpha * p[k];
    const double r = v.r[k] - alpha * v.q[k];
    v.r[k] = r;
    s[0] = r * (r * v.idiag[j]);
    s[1] = r * r;
  }
  cg_block_sum<2>(s, red, v.part);
}

// beta = r.z(new) / r.z(old)
__global__ __launch_bounds__(256) void k_cg_beta(int nb, CgVecs v) {
  __shared__ double t[2];
  cg_sum_parts<2>(v.part, nb, t);
  if (threadIdx.x == 0) {
    v.s[CG_BETA] = v.s[CG_RZ] != 0.0 ? t[0] / v.s[CG_RZ] : 0.0;
    v.s[CG_RZ] = t[0];
    v.s[CG_RR] = t[1];
  }
}

// E_x, E_r, B_theta (and Bbar_theta) of phi, added to the mode-0 grids
template <class R>
__global__ __launch_bounds__(SB) void k_bunch_fields(Geo g, Grids<R> f, CgOp o, double beta, CgVecs v) {
  const long long k = (long long)blockIdx.x * SB + threadIdx.x;
  const int nr1 = g.nr + 1;
  if (k >= (long long)(g.nx + 1) * nr1) return;
  const int i = (int)(k / nr1), j = (int)(k - (long long)i * nr1);
  auto phi = [&](int a, int b) -> double {  // zero on the x ends and at r_max
    if (a < 1 || a > o.ni || b < 0 || b >= o.nj) return 0.0;
    return v.x[(size_t)(a - 1) * o.nj + b];
  };
  const size_t at = (size_t)phys_col(g, i) * g.pitch + j;
  if (i <= g.nx - 1) {
    const double ex = -(phi(i + 1, j) - phi(i, j)) * o.g2 / o.dx;
    f.ex[at] = (R)((double)f.ex[at] + ex);
  }
  if (j <= g.nr - 1) {
    const double er = -(phi(i, j + 1) - phi(i, j)) / o.dr;
    f.er[at] = (R)((double)f.er[at] + er);
    if (i <= g.nx - 1) {
      const double er1 = -(phi(i + 1, j + 1) - phi(i + 1, j)) / o.dr;
      const double bt = beta * 0.5 * (er + er1);
      f.bt[at] = (R)((double)f.bt[at] + bt);
      f.btb[at] = (R)((double)f.btb[at] + bt);
    }
  }
}

long long cg_unknowns(int nx, int nr) { return (long long)(nx - 1) * nr; }
int cg_blocks(int nx, int nr) { return (int)((cg_unknowns(nx, nr) + SB - 1) / SB); }

template <class R>
int bunch_solve(const Geo& g, const Parts<R>& P, const Layout& L, int max_items, const Grids<R>& f,
                unsigned id_lo, unsigned id_hi, double beta, double tol, int max_iter, const CgVecs& v,
                hipStream_t st, int* iters, double* resid) {
  CgOp o;
  o.ni = g.nx - 1;
  o.nj = g.nr;
  o.g2 = 1.0 - beta * beta;
  o.dx = g.dx;
  o.dr = g.dr;
  const long long n = cg_unknowns(g.nx, g.nr);
  const int nb = cg_blocks(g.nx, g.nr);
  hipLaunchKernelGGL(k_cg_zero, dim3(nb), dim3(SB), 0, st, v.r, n);
  hipLaunchKernelGGL(k_cg_idiag, dim3((o.nj + SB - 1) / SB), dim3(SB), 0, st, o, v);
  hipLaunchKernelGGL((k_bunch_charge<R>), dim3(max_items), dim3(SB), 0, st, g, P, L, id_lo, id_hi, o, v.r);
  hipLaunchKernelGGL(k_cg_start, dim3(nb), dim3(SB), 0, st, o, v);
  hipLaunchKernelGGL(k_cg_init_scalars, dim3(1), dim3(256), 0, st, nb, v);
  double hs[CG_NS];
  if (hipMemcpyAsync(hs, v.s, sizeof(hs), hipMemcpyDeviceToHost, st) != hipSuccess) return -1;
  if (hipStreamSynchronize(st) != hipSuccess) return -1;
  const double bb = hs[CG_BB];
  *iters = 0;
  *resid = 0.0;
  if (bb == 0.0) return 0;  // no charge: nothing to add (x = 0)
  const double stop = tol * tol * bb;
  double* pa = v.p;   // direction of the previous iteration (zero at the start)
  double* pb = v.p2;  // the new one
  int it = 0;
  double rr = bb;
  while (it < max_iter && rr > stop) {
    const int burst = std::min(CG_CHECK, max_iter - it);
    for (int k = 0; k < burst; ++k) {
      hipLaunchKernelGGL(k_cg_apply, dim3(nb), dim3(SB), 0, st, o, v, pa, pb);
      hipLaunchKernelGGL(k_cg_alpha, dim3(1), dim3(256), 0, st, nb, v);
      hipLaunchKernelGGL(k_cg_update, dim3(nb), dim3(SB), 0, st, o, v, pb);
      hipLaunchKernelGGL(k_cg_beta, dim3(1), dim3(256), 0, st, nb, v);
      std::swap(pa, pb);
    }
    it += burst;
    if (hipMemcpyAsync(hs, v.s, sizeof(hs), hipMemcpyDeviceToHost, st) != hipSuccess) return -1;
    if (hipStreamSynchronize(st) != hipSuccess) return -1;
    rr = hs[CG_RR];
  }
  *iters = it;
  *resid = std::sqrt(rr / bb);
  const long long nodes = (long long)(g.nx + 1) * (g.nr + 1);
  hipLaunchKernelGGL((k_bunch_fields<R>), dim3((unsigned)((nodes + SB - 1) / SB)), dim3(SB), 0, st, g, f, o, beta, v);
  return 0;
}

template int bunch_solve<float>(const Geo&, const Parts<float>&, const Layout&, int, const Grids<float>&, unsigned,
                                unsigned, double, double, int, const CgVecs&, hipStream_t, int*, double*);
template int bunch_solve<double>(const Geo&, const Parts<double>&, const Layout&, int, const Grids<double>&,
                                 unsigned, unsigned, double, double, int, const CgVecs&, hipStream_t, int*, double*);

}  // namespace envpic
