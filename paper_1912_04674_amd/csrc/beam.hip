// beam.hip -- injected-beam parameters of the particle set (Sec. 4, Table
// BeamParams of arXiv:1912.04674): peak of the electron energy spectrum,
// beam charge, relative energy spread and normalized transverse emittance
// sqrt(s_xx s_pp - s_xp^2), over the particles within two FWHM widths in
// energy around the spectrum peak.
//
// Definitions (the table gives the quantities only):
//   energy     gamma - 1 = |p|^2 / (1 + sqrt(1 + |p|^2)) of the momentum, FP64;
//   spectrum   charge histogram sum |q| w over nbins equal bins of
//              [e_lo, e_hi), summed as 64-bit fixed point (exact and
//              independent of the order of the atomics);
//   peak       the fullest bin (lowest on a tie), energy at its centre;
//   FWHM       first bin below half maximum on each side of the peak, the
//              crossing interpolated between bin centres; a side that stays
//              above ends at the range edge;
//   window     [E_peak - FWHM, E_peak + FWHM] within [e_lo, e_hi);
//   moments    weighted by w, centred (a pass for the means, one for the
//              second moments), FP64 tree sums per work item, then a
//              fixed-order sum over the items.
//
// Four launches on the simulation's stream: clear, histogram (one work
// group per work item of the tile layout, LDS histogram flushed with
// integer atomics), peak (one work group), and for each moment pass a
// per-item kernel plus a one-group fixed-order reduction.
#include <algorithm>

#include "common.hpp"
#include "envpic.h"
#include "launch.hpp"

// the energy, bin and moment arithmetic is written out term by term; keep
// the compiler from fusing it into FMAs so the rounding is that of the
// expressions as written
#pragma clang fp contract(off)

namespace envpic {

constexpr int BG = 256;      // threads of the per-item kernels
constexpr int BPK = 1024;    // threads of the peak kernel
constexpr int NBM = BEAM_PARTS;  // partial sums per item in each moment pass

__device__ inline double kin_energy(double px, double py, double pz) {
  const double p2 = px * px + py * py + pz * pz;
  return p2 / (1.0 + sqrt(1.0 + p2));
}

__device__ inline int energy_bin(const BeamArgs& a, double e) {
  if (!(e >= a.e_lo && e < a.e_hi)) return -1;
  int k = (int)floor((e - a.e_lo) / a.de);
  return k < a.nbins - 1 ? k : a.nbins - 1;
}

__global__ __launch_bounds__(BG) void k_beam_clear(BeamScratch b, int nbins) {
  const int k = blockIdx.x * BG + threadIdx.x;
  if (k < nbins) b.hist[k] = 0;
  if (k < BEAM_STATE) b.st[k] = 0.0;
}

template <class R>
__global__ __launch_bounds__(BG) void k_beam_hist(Parts<R> P, Layout L, BeamArgs a, BeamScratch b) {
  __shared__ long long h[BEAM_MAX_BINS];
  for (int k = threadIdx.x; k < a.nbins; k += BG) h[k] = 0;
  __syncthreads();
  const int item = blockIdx.x;
  if (item < *L.n_items) {
    const int4 it = L.items[item];
    for (int k = threadIdx.x; k < it.z; k += BG) {
      const int p = it.y + k;
      if (P.cell[p] == kDead) continue;
      const int bin = energy_bin(a, kin_energy((double)P.px[p], (double)P.py[p], (double)P.pz[p]));
      if (bin < 0) continue;
      // |q| w in fixed point (q = -1): the scale keeps every sum below 2^62
      const long long c = __double2ll_rn((double)P.w[p] * a.scale);
      atomicAdd((unsigned long long*)&h[bin], (unsigned long long)c);
    }
  }
  __syncthreads();
  for (int k = threadIdx.x; k < a.nbins; k += BG)
    if (h[k] != 0) atomicAdd((unsigned long long*)&b.hist[k], (unsigned long long)h[k]);
}

// block reductions of the peak kernel
__device__ inline void argmax_block(long long v, int k, long long* sv, int* sk) {
  // value, then the lower index on a tie
  sv[threadIdx.x] = v;
  sk[threadIdx.x] = k;
  __syncthreads();
  for (int s = BPK / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
      const long long v2 = sv[threadIdx.x + s];
      const int k2 = sk[threadIdx.x + s];
      if (v2 > sv[threadIdx.x] || (v2 == sv[threadIdx.x] && k2 < sk[threadIdx.x])) {
        sv[threadIdx.x] = v2;
        sk[threadIdx.x] = k2;
      }
    }
    __syncthreads();
  }
}
__device__ inline int reduce_idx(int k, bool take_max, int* sk) {
  sk[threadIdx.x] = k;
  __syncthreads();
  for (int s = BPK / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
      const int k2 = sk[threadIdx.x + s];
      if (take_max ? k2 > sk[threadIdx.x] : k2 < sk[threadIdx.x]) sk[threadIdx.x] = k2;
    }
    __syncthreads();
  }
  const int r = sk[0];
  __syncthreads();
  return r;
}

__global__ __launch_bounds__(BPK) void k_beam_peak(BeamArgs a, BeamScratch b) {
  __shared__ long long sv[BPK];
  __shared__ int sk[BPK];
  const int n = a.nbins;
  // the fullest bin, lowest index on a tie
  long long best = -1;
  int kbest = n;
  for (int k = threadIdx.x; k < n; k += BPK) {
    const long long v = (long long)b.hist[k];
    if (v > best) {  // strided in increasing k: the first of equal values stays
      best = v;
      kbest = k;
    }
  }
  argmax_block(best, kbest, sv, sk);
  const long long hmax = sv[0];
  const int kp = sk[0];
  __syncthreads();
  const double inv = 1.0 / a.scale;
  for (int k = threadIdx.x; k < n; k += BPK) b.hist_f[k] = (double)(long long)b.hist[k] * inv;
  if (hmax <= 0) {  // empty spectrum: nothing is selected, every output is zero
    if (threadIdx.x == 0) {
      b.st[BS_NONEMPTY] = 0.0;
      b.st[BS_LO] = 1.0;
      b.st[BS_HI] = -1.0;
    }
    return;
  }
  // first bin below half maximum on each side (2 H < H_max, exact integers)
  int kl = -1, kr = n;
  for (int k = threadIdx.x; k < n; k += BPK) {
    const bool below = 2 * (long long)b.hist[k] < hmax;
    if (below && k < kp && k > kl) kl = k;
    if (below && k > kp && k < kr) kr = k;
  }
  kl = reduce_idx(kl, true, sk);
  kr = reduce_idx(kr, false, sk);
  if (threadIdx.x == 0) {
    const double h = (double)hmax * inv, half = 0.5 * h;
    const double e_peak = a.e_lo + (kp + 0.5) * a.de;
    double left = a.e_lo, right = a.e_hi;
    if (kl >= 0) {
      const double hl = (double)(long long)b.hist[kl] * inv, hl1 = (double)(long long)b.hist[kl + 1] * inv;
      left = (a.e_lo + (kl + 0.5) * a.de) + (half - hl) / (hl1 - hl) * a.de;
    }
    if (kr < n) {
      const double hr = (double)(long long)b.hist[kr] * inv, hr0 = (double)(long long)b.hist[kr - 1] * inv;
      right = (a.e_lo + (kr - 1 + 0.5) * a.de) + (hr0 - half) / (hr0 - hr) * a.de;
    }
    const double fwhm = right - left;
    b.st[BS_NONEMPTY] = 1.0;
    b.st[BS_PEAK] = e_peak;
    b.st[BS_FWHM] = fwhm;
    b.st[BS_LO] = fmax(a.e_lo, e_peak - fwhm);
    b.st[BS_HI] = e_peak + fwhm;
  }
}

template <int N>
__device__ inline void beam_block_sum(double (&v)[N], double* red /* [N][BG] */, double* out) {
  for (int k = 0; k < N; ++k) red[k * BG + threadIdx.x] = v[k];
  __syncthreads();
  for (int s = BG / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s)
      for (int k = 0; k < N; ++k) red[k * BG + threadIdx.x] += red[k * BG + threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x < N) out[threadIdx.x] = red[threadIdx.x * BG];
}

// PASS 1: sums of w, w E, w y, w z, w p_y, w p_z, count over the window and
// w over the whole spectrum range; PASS 2: centred second moments
// w dE^2, w dy^2, w dpy^2, w dy dpy, w dz^2, w dpz^2, w dz dpz
template <class R, int PASS>
__global__ __launch_bounds__(BG) void k_beam_moments(Geo g, Parts<R> P, Layout L, BeamArgs a, BeamScratch b) {
  __shared__ double red[NBM * BG];
  double v[NBM] = {0, 0, 0, 0, 0, 0, 0, 0};
  const int item = blockIdx.x;
  const double lo = b.st[BS_LO], hi = b.st[BS_HI];
  const double em = b.st[BS_EMEAN], ym = b.st[BS_YMEAN], zm = b.st[BS_ZMEAN];
  const double pym = b.st[BS_PYMEAN], pzm = b.st[BS_PZMEAN];
  if (item < *L.n_items) {
    const int4 it = L.items[item];
    for (int k = threadIdx.x; k < it.z; k += BG) {
      const int p = it.y + k;
      const unsigned cw = P.cell[p];
      if (cw == kDead) continue;
      const double px = P.px[p], py = P.py[p], pz = P.pz[p];
      const double e = kin_energy(px, py, pz);
      if (!(e >= a.e_lo && e < a.e_hi)) continue;
      const double w = P.w[p];
      if (PASS == 1) v[7] += w;
      if (!(e >= lo && e <= hi)) continue;
      const double r = ((double)cell_jr(cw) + (double)P.fr[p]) * g.dr;
      const double th = (double)P.th[p];
      const double y = r * cos(th), z = r * sin(th);
      if (PASS == 1) {
        v[0] += w;
        v[1] += w * e;
        v[2] += w * y;
        v[3] += w * z;
        v[4] += w * py;
        v[5] += w * pz;
        v[6] += 1.0;
      } else {
        const double de = e - em, dy = y - ym, dz = z - zm, dpy = py - pym, dpz = pz - pzm;
        v[0] += w * de * de;
        v[1] += w * dy * dy;
        v[2] += w * dpy * dpy;
        v[3] += w * dy * dpy;
        v[4] += w * dz * dz;
        v[5] += w * dpz * dpz;
        v[6] += w * dz * dpz;
      }
    }
  }
  beam_block_sum<NBM>(v, red, b.part + (size_t)item * NBM);
}

// fixed-order sum of the per-item partials (wavefront q sums quantity q),
// then the means (PASS 1) or the outputs (PASS 2)
template <int PASS>
__global__ __launch_bounds__(64 * NBM) void k_beam_reduce(int n_items, BeamArgs a, BeamScratch b) {
  __shared__ double lanes[NBM][64];
  __shared__ double t[NBM];
  const int q = threadIdx.x / 64, l = threadIdx.x % 64;
  double s = 0.0;
  for (int i = l; i < n_items; i += 64) s += b.part[(size_t)i * NBM + q];
  lanes[q][l] = s;
  __syncthreads();
  for (int h = 32; h > 0; h >>= 1) {
    if (l < h) lanes[q][l] += lanes[q][l + h];
    __syncthreads();
  }
  if (l == 0) t[q] = lanes[q][0];
  __syncthreads();
  if (threadIdx.x != 0) return;
  double* st = b.st;
  if (PASS == 1) {
    const double W = t[0];
    st[BS_W] = W;
    st[BS_COUNT] = t[6];
    st[BS_QSPEC] = -t[7];
    if (W != 0.0) {
      st[BS_EMEAN] = t[1] / W;
      st[BS_YMEAN] = t[2] / W;
      st[BS_ZMEAN] = t[3] / W;
      st[BS_PYMEAN] = t[4] / W;
      st[BS_PZMEAN] = t[5] / W;
    }
    return;
  }
  double* out = b.out;
  for (int k = 0; k < ENVPIC_NBEAM; ++k) out[k] = 0.0;
  const double W = st[BS_W];
  if (st[BS_NONEMPTY] == 0.0 || W == 0.0) return;
  const double e_rms = sqrt(t[0] / W);
  const double syy = t[1] / W, spp = t[2] / W, syp = t[3] / W;
  const double szz = t[4] / W, sqq = t[5] / W, szq = t[6] / W;
  out[ENVPIC_B_PEAK] = st[BS_PEAK];
  out[ENVPIC_B_FWHM] = st[BS_FWHM];
  out[ENVPIC_B_CHARGE] = -W;
  out[ENVPIC_B_EMEAN] = st[BS_EMEAN];
  out[ENVPIC_B_ERMS] = e_rms;
  out[ENVPIC_B_SPREAD] = e_rms / st[BS_PEAK];
  out[ENVPIC_B_EMIT_Y] = sqrt(fmax(0.0, syy * spp - syp * syp));
  out[ENVPIC_B_EMIT_Z] = sqrt(fmax(0.0, szz * sqq - szq * szq));
  out[ENVPIC_B_COUNT] = st[BS_COUNT];
  out[ENVPIC_B_QSPEC] = st[BS_QSPEC];
  out[ENVPIC_B_WIN_LO] = st[BS_LO];
  out[ENVPIC_B_WIN_HI] = fmin(st[BS_HI], a.e_hi);
}

template <class R>
void launch_beam(const Geo& g, const Parts<R>& P, const Layout& L, int max_items, const BeamArgs& a,
                 const BeamScratch& b, hipStream_t st) {
  const int nclr = (std::max(a.nbins, (int)BEAM_STATE) + BG - 1) / BG;
  hipLaunchKernelGGL(k_beam_clear, dim3(nclr), dim3(BG), 0, st, b, a.nbins);
  hipLaunchKernelGGL((k_beam_hist<R>), dim3(max_items), dim3(BG), 0, st, P, L, a, b);
  hipLaunchKernelGGL(k_beam_peak, dim3(1), dim3(BPK), 0, st, a, b);
  hipLaunchKernelGGL((k_beam_moments<R, 1>), dim3(max_items), dim3(BG), 0, st, g, P, L, a, b);
  hipLaunchKernelGGL(k_beam_reduce<1>, dim3(1), dim3(64 * NBM), 0, st, max_items, a, b);
  hipLaunchKernelGGL((k_beam_moments<R, 2>), dim3(max_items), dim3(BG), 0, st, g, P, L, a, b);
  hipLaunchKernelGGL(k_beam_reduce<2>, dim3(1), dim3(64 * NBM), 0, st, max_items, a, b);
}

template void launch_beam<float>(const Geo&, const Parts<float>&, const Layout&, int, const BeamArgs&,
                                 const BeamScratch&, hipStream_t);
template void launch_beam<double>(const Geo&, const Parts<double>&, const Layout&, int, const BeamArgs&,
                                  const BeamScratch&, hipStream_t);

}  // namespace envpic
