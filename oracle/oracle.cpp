/*
 * oracle.cpp -- plain FP64 CPU reference of the cylindrical envelope PIC loop.
 *
 * TEST INFRASTRUCTURE ONLY (see oracle.h).  Plain loops, no blocking, no
 * fusion, no reordering beyond what the method states, so that each stage
 * can be read against the paper:
 *   Massimo, Zemzemi, Beck, Derouillat, Specka, arXiv:1912.04674.
 *
 * Readings taken where the paper is silent, garbled or delegates to other
 * work (each is listed with its reason in the design notes of the repo):
 *   R1  ponderomotive force  -grad(Phi)/(2 gbar)       (Sec. 2, Eq. EquationsOfMotion,
 *       read as the gradient of gbar = sqrt(1+p^2+Phi) w.r.t. position)
 *   R2  Cartesian force signs from the vector form of Eq. EquationsOfMotion with
 *       the right-handed frame r = (0, cos, sin), theta = (0, -sin, cos)
 *       (Sec. 3, Eq. motion_equations_cartesian is garbled)
 *   R3  envelope scheme: dt^2 multiplies the whole bracket, "dz" is dx
 *       (Sec. 3, Eq. envelope_solver, re-derived from Eq. envelope_equation)
 *   R4  on-axis radial Laplacian 4 (A_1 - A_0)/dr^2
 *   R5  Yee-like layout after Lifschitz: A, chi, E_t at (i,j); E_x, J_x at
 *       (i+1/2, j); E_r, J_r at (i, j+1/2); B_t at (i+1/2, j+1/2); mode 1 adds
 *       B_x at (i, j+1/2) and B_r at (i+1/2, j); axis on the primal node j=0
 *   R6  step order: momentum + chi -> envelope -> position + J -> Maxwell -> window
 *   R7  gbar for the kick from p^{n-1/2}; gbar^n from the half-kicked momentum
 *       for the rotation and chi
 *   R8  Phi^{n+1/2} = (Phi^n + Phi^{n+1})/2 gathered at x^n for the position push
 *   R9  linear (cloud-in-cell) shapes for gather and deposit
 *   R10 chi = sum w S / (gbar V) > 0 (electrons, q^2/m = 1)
 *   R11 mode-0 current by the Esirkepov decomposition in (x, r) index space;
 *       mode-1 current deposited directly at the mid-point
 *   R12 node volumes V_0 = pi dr^2 dx / 4, V_j = 2 pi r_j dr dx
 *   R13 initial A^{-1}: the paraxial pulse one time step earlier
 *   R14 tau is the FWHM of |A|
 *   R16 Dirichlet envelope / perfect conductor at the x ends and r_max;
 *       particles reflect at r_max and leave through the x ends
 *   R17 loading regular in x and r, one random angle per cell, equally spaced
 *       angles inside the cell, weights proportional to r
 *   R21 Bbar^n = (B^{n-1/2} + B^{n+1/2}) / 2
 * Threads (oracle_set_threads, default 1): the particle loops of the
 * momentum and position stages split the particles into equal contiguous
 * ranges, one per thread; each thread deposits chi or J into grids of its
 * own, which are then added in thread order.  Results are therefore
 * identical for a given thread count; one thread is the plain loop.
 *   R24 optional binomial current filter (Sec. 4, nonlinear benchmark: an
 *       uncompensated binomial filter of 7 passes): N passes of 1-2-1 in
 *       index space, each along x then along r, on J^{n+1/2} of both modes
 *       before the field update; zero current outside the window and beyond
 *       r_max, ghost rows below the axis by the component's parity (R23);
 *       a component odd on the primal axis row (mode-1 J_x) is zero there
 */
#include "oracle.h"

#include <cmath>
#include <complex>
#include <cstring>
#include <new>
#include <thread>
#include <vector>

namespace {

typedef std::complex<double> cplx;
const double kPi = 3.14159265358979323846;
const cplx kI(0.0, 1.0);

/* ------------------------------------------------------------------ RNG --
 * SplitMix64 (Steele, Lea, Flood, OOPSLA 2014), used counter-style: the
 * deviate for a key is the mix of seed + (key + 1) * golden-gamma.        */
uint64_t splitmix64_mix(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

double uniform_of(uint64_t seed, uint64_t stream, int64_t col, int64_t j) {
  uint64_t key = (stream << 56) ^ (((uint64_t)col & 0xFFFFFFFFull) << 20) ^
                 ((uint64_t)j & 0xFFFFFull);
  uint64_t z = splitmix64_mix(seed + (key + 1ull) * 0x9E3779B97F4A7C15ull);
  return (double)(z >> 11) * (1.0 / 9007199254740992.0);
}

const uint64_t kStreamAngle = 1;
const uint64_t kStreamDensity = 2;

/* ------------------------------------------------------------ threads -- */
int g_threads = 1;

/* fn(t, lo, hi) for t = 0..T-1 over the contiguous ranges [lo, hi) of n
 * items, thread t on its own std::thread (t = 0 on the caller's)           */
template <class F>
void for_ranges(size_t n, int T, F fn) {
  if (T <= 1) {
    fn(0, (size_t)0, n);
    return;
  }
  std::vector<std::thread> th;
  for (int t = 1; t < T; ++t) th.emplace_back(fn, t, n * t / T, n * (t + 1) / T);
  fn(0, (size_t)0, n / T);
  for (auto& x : th) x.join();
}

/* ---------------------------------------------------------------- state -- */
struct Sim {
  oracle_params p;
  int Nx, Nr, NR1;
  size_t ng;
  double dx, dr, dt;
  int64_t n, shift;
  std::vector<cplx> A, Ap;                                   /* A^n, A^{n-1} */
  std::vector<double> chi, Ex, Er, Bt, Btb, Jx, Jr;          /* mode 0 */
  std::vector<cplx> Ex1, Er1, Et1, Bx1, Br1, Bt1, Bxb1, Brb1, Btb1, Jx1, Jr1, Jt1;
  std::vector<double> x, y, z, px, py, pz, w, gbar;
  std::vector<uint32_t> id;

  size_t at(int i, int j) const { return (size_t)i * NR1 + j; }
  bool m1() const { return p.n_modes >= 2; }

  /* per-thread deposit grids (threads > 1 only) */
  std::vector<std::vector<double>> t_chi, t_jx, t_jr;
  std::vector<std::vector<cplx>> t_jx1, t_jr1, t_jt1;
};

/* where one thread's deposits go: the simulation's own grids (one thread)
 * or that thread's grids                                                  */
struct Dep {
  double* chi;
  double *jx, *jr;
  cplx *jx1, *jr1, *jt1;
};

/* T deposit targets, zeroed; for one thread the simulation's own grids */
std::vector<Dep> deposit_targets(Sim& s, int T, bool chi) {
  std::vector<Dep> d(T);
  if (T == 1) {
    if (chi) {
      std::fill(s.chi.begin(), s.chi.end(), 0.0);
    } else {
      std::fill(s.Jx.begin(), s.Jx.end(), 0.0);
      std::fill(s.Jr.begin(), s.Jr.end(), 0.0);
      if (s.m1()) {
        std::fill(s.Jx1.begin(), s.Jx1.end(), 0.0);
        std::fill(s.Jr1.begin(), s.Jr1.end(), 0.0);
        std::fill(s.Jt1.begin(), s.Jt1.end(), 0.0);
      }
    }
    d[0] = Dep{s.chi.data(), s.Jx.data(), s.Jr.data(), s.m1() ? s.Jx1.data() : nullptr,
               s.m1() ? s.Jr1.data() : nullptr, s.m1() ? s.Jt1.data() : nullptr};
    return d;
  }
  const size_t ng = s.ng, n1 = s.m1() ? s.ng : 0;
  if (chi) {
    s.t_chi.resize(T);
    for_ranges((size_t)T, T, [&](int, size_t lo, size_t hi) {
      for (size_t t = lo; t < hi; ++t) s.t_chi[t].assign(ng, 0.0);
    });
    for (int t = 0; t < T; ++t) d[t] = Dep{s.t_chi[t].data(), nullptr, nullptr, nullptr, nullptr, nullptr};
  } else {
    s.t_jx.resize(T);
    s.t_jr.resize(T);
    s.t_jx1.resize(T);
    s.t_jr1.resize(T);
    s.t_jt1.resize(T);
    for_ranges((size_t)T, T, [&](int, size_t lo, size_t hi) {
      for (size_t t = lo; t < hi; ++t) {
        s.t_jx[t].assign(ng, 0.0);
        s.t_jr[t].assign(ng, 0.0);
        s.t_jx1[t].assign(n1, 0.0);
        s.t_jr1[t].assign(n1, 0.0);
        s.t_jt1[t].assign(n1, 0.0);
      }
    });
    for (int t = 0; t < T; ++t)
      d[t] = Dep{nullptr, s.t_jx[t].data(), s.t_jr[t].data(), s.t_jx1[t].data(), s.t_jr1[t].data(),
                 s.t_jt1[t].data()};
  }
  return d;
}

/* out[k] = sum over threads t = 0..T-1 (in that order) of parts[t][k] */
template <class V>
void sum_in_thread_order(V& out, const std::vector<V>& parts, int T) {
  for_ranges(out.size(), T, [&](int, size_t lo, size_t hi) {
    for (size_t k = lo; k < hi; ++k) {
      typename V::value_type acc = parts[0][k];
      for (int t = 1; t < T; ++t) acc += parts[t][k];
      out[k] = acc;
    }
  });
}

/* ------------------------------------------------ cylindrical volumes --
 * R12: node volume of the primal row j (axis disc of radius dr/2 for j=0),
 * volume of the half-integer row j+1/2, radial face area at r_{j+1/2} and
 * axial face area of row j.                                               */
double vol_node(const Sim& s, int j) {
  return j == 0 ? kPi * s.dr * s.dr * s.dx / 4.0 : 2.0 * kPi * j * s.dr * s.dr * s.dx;
}
double vol_half(const Sim& s, int j) { return 2.0 * kPi * (j + 0.5) * s.dr * s.dr * s.dx; }
double area_r(const Sim& s, int j) { return 2.0 * kPi * (j + 0.5) * s.dr * s.dx; }
double area_x(const Sim& s, int j) { return vol_node(s, j) / s.dx; }

/* ------------------------------------------------------------ loading -- */
double density(const Sim& s, double xlab, int64_t col, int j) {
  const oracle_params& p = s.p;
  switch (p.profile) {
    case ORACLE_PROFILE_UNIFORM:
      return p.n0;
    case ORACLE_PROFILE_RAMP:
      if (xlab <= 0.0) return 0.0;
      if (xlab < p.ramp_len) return p.n0 * xlab / p.ramp_len;
      return p.n0;
    case ORACLE_PROFILE_PERTURB:
      return p.n0 * (1.0 + p.perturb * (2.0 * uniform_of(p.seed, kStreamDensity, col, j) - 1.0));
    case ORACLE_PROFILE_BUMP: {
      double u = (xlab - p.bump_x) / p.bump_w;
      return p.n0 * (1.0 + std::exp(-u * u));
    }
    default:
      return 0.0;
  }
}

/* R17: particles of lab cell column `col`, radial cell j. */
void load_cell(Sim& s, int64_t col, int j) {
  const oracle_params& p = s.p;
  const int ppc = p.ppc_x * p.ppc_r * p.ppc_t;
  const double th0 = 2.0 * kPi * uniform_of(p.seed, kStreamAngle, col, j);
  for (int a = 0; a < p.ppc_x; ++a)
    for (int b = 0; b < p.ppc_r; ++b)
      for (int k = 0; k < p.ppc_t; ++k) {
        double xl = ((double)col + (a + 0.5) / p.ppc_x) * s.dx;
        double r = (j + (b + 0.5) / p.ppc_r) * s.dr;
        double nloc = density(s, xl, col, j);
        if (!(nloc > 0.0)) continue;
        double th = th0 + 2.0 * kPi * k / p.ppc_t;
        s.x.push_back(xl);
        s.y.push_back(r * std::cos(th));
        s.z.push_back(r * std::sin(th));
        s.px.push_back(0.0);
        s.py.push_back(0.0);
        s.pz.push_back(0.0);
        s.w.push_back(nloc * 2.0 * kPi * r * (s.dr / p.ppc_r) * (s.dx / p.ppc_x) / p.ppc_t);
        s.gbar.push_back(1.0);
        s.id.push_back((uint32_t)(col * (int64_t)s.Nr * ppc + (int64_t)j * ppc +
                                  (a * p.ppc_r + b) * p.ppc_t + k));
      }
}

/* Paraxial Gaussian pulse (R13, R14): the beam a0 exp(-r^2/(w0^2 q))/q with
 * q = 1 + i (x - x_f)/Z_R, Z_R = w0^2/2, solves 2i dA/dx + lap_perp A = 0;
 * it is modulated by exp(-xi^2/sigma^2), xi = x - x_c - t.                 */
cplx pulse(const Sim& s, double xl, double r, double t) {
  const oracle_params& p = s.p;
  if (p.a0 == 0.0) return 0.0;
  double zr = 0.5 * p.w0 * p.w0;
  cplx q(1.0, (xl - p.x_f) / zr);
  double sig = p.tau / (2.0 * std::sqrt(std::log(2.0)));
  double xi = xl - p.x_c - t;
  return p.a0 * std::exp(-r * r / (p.w0 * p.w0 * q)) / q * std::exp(-xi * xi / (sig * sig));
}

/* ------------------------------------------------------------- shapes --
 * Order 1 (R9, cloud in cell): nodes floor(u), floor(u)+1 with weights
 * 1-f, f.  Order 2 (R26, quadratic B-spline): around the nearest node
 * m = floor(u + 1/2), d = u - m in [-1/2, 1/2), nodes m-1, m, m+1 with
 * weights (1/2 - d)^2/2, 3/4 - d^2, (1/2 + d)^2/2.  u is in node units
 * (cell units for the primal nodes, shifted by 1/2 for the dual ones).   */
struct Sh {
  int i;       /* first node */
  int n;       /* number of nodes (order + 1) */
  double w[3]; /* weights of nodes i .. i+n-1 */
};
Sh shape(double u, int order) {
  Sh r{};
  if (order == 2) {
    double m = std::floor(u + 0.5), d = u - m;
    r.i = (int)m - 1;
    r.n = 3;
    r.w[0] = 0.5 * (0.5 - d) * (0.5 - d);
    r.w[1] = 0.75 - d * d;
    r.w[2] = 0.5 * (0.5 + d) * (0.5 + d);
  } else {
    double f = std::floor(u);
    r.i = (int)f;
    r.n = 2;
    r.w[0] = 1.0 - (u - f);
    r.w[1] = u - f;
  }
  return r;
}
int order_of(const Sim& s) { return s.p.shape_order == 2 ? 2 : 1; }
Sh primal(const Sim& s, double u) { return shape(u, order_of(s)); }
Sh dual(const Sim& s, double u) { return shape(u - 0.5, order_of(s)); }

/* Radial staggering of a grid: primal rows sit at r = j dr, half rows at
 * r = (j + 1/2) dr.  Below the axis a grid continues by its parity (R23):
 * primal row -j mirrors row j, half row -1-j mirrors row j.              */
enum Stag { PRIMAL_R = 0, HALF_R = 1 };
int mirror_row(int j, Stag st) { return st == HALF_R ? -1 - j : -j; }

/* value of a grid at (i, j); (imax, jmax) is the last stored index of this
 * staggering; rows below the axis mirror with sign `par`; anything else
 * outside is zero.                                                        */
template <class T>
T val(const Sim& s, const std::vector<T>& f, int i, int j, int imax, int jmax, Stag st, double par) {
  if (i < 0 || i > imax) return T(0.0);
  if (j < 0) {
    int m = mirror_row(j, st);
    if (m > jmax) return T(0.0);
    return par * f[s.at(i, m)];
  }
  if (j > jmax) return T(0.0);
  return f[s.at(i, j)];
}
template <class T>
T interp(const Sim& s, const std::vector<T>& f, Sh sx, Sh sr, int imax, int jmax, Stag st, double par) {
  T acc(0.0);
  for (int a = 0; a < sx.n; ++a) {
    T col(0.0);
    for (int b = 0; b < sr.n; ++b) col += sr.w[b] * val(s, f, sx.i + a, sr.i + b, imax, jmax, st, par);
    acc += sx.w[a] * col;
  }
  return acc;
}

/* mode-1 contribution at azimuth (c, s) = (cos, sin): Re[F e^{-i theta}] */
double mode1(cplx f, double c, double sn) { return f.real() * c + f.imag() * sn; }

void init_fields(Sim& s) {
  const size_t ng = s.ng;
  s.A.assign(ng, 0.0);
  s.Ap.assign(ng, 0.0);
  s.chi.assign(ng, 0.0);
  s.Ex.assign(ng, 0.0);
  s.Er.assign(ng, 0.0);
  s.Bt.assign(ng, 0.0);
  s.Btb.assign(ng, 0.0);
  s.Jx.assign(ng, 0.0);
  s.Jr.assign(ng, 0.0);
  std::vector<cplx>* m1f[] = {&s.Ex1, &s.Er1, &s.Et1, &s.Bx1, &s.Br1, &s.Bt1,
                              &s.Bxb1, &s.Brb1, &s.Btb1, &s.Jx1, &s.Jr1, &s.Jt1};
  for (auto* f : m1f) f->assign(s.m1() ? ng : 0, 0.0);
  for (int i = 0; i <= s.Nx; ++i)
    for (int j = 0; j <= s.Nr; ++j) {
      double xl = (double)(s.shift + i) * s.dx, r = j * s.dr;
      bool edge = (s.p.env_bc_x == 0 && (i == 0 || i == s.Nx)) ||
                  (s.p.env_bc_r == 0 && j == s.Nr);
      s.A[s.at(i, j)] = edge ? 0.0 : pulse(s, xl, r, 0.0);
      s.Ap[s.at(i, j)] = edge ? 0.0 : pulse(s, xl, r, -s.dt);
    }
}

/* -------------------------------------------- momentum stage (Sec. 3) --
 * Gather E^n, Bbar^n, Phi^n and grad Phi^n at x^n, push p^{n-1/2} ->
 * p^{n+1/2} with the ponderomotive Boris scheme (R1, R2, R7), deposit
 * chi^n (R10).  grad Phi by centred differences on the primal nodes.     */
void momentum_chi(Sim& s) {
  const int Nx = s.Nx, Nr = s.Nr;
  const double dx = s.dx, dr = s.dr, dt = s.dt;
  std::vector<double> phi(s.ng), gx(s.ng), gr(s.ng);
  for (size_t k = 0; k < s.ng; ++k) phi[k] = 0.5 * std::norm(s.A[k]);
  for (int i = 0; i <= Nx; ++i)
    for (int j = 0; j <= Nr; ++j) {
      double pl = i + 1 <= Nx ? phi[s.at(i + 1, j)] : 0.0;
      double mi = i - 1 >= 0 ? phi[s.at(i - 1, j)] : 0.0;
      gx[s.at(i, j)] = (pl - mi) / (2.0 * dx);
      if (j == 0) {
        gr[s.at(i, j)] = 0.0;
      } else {
        double up = j + 1 <= Nr ? phi[s.at(i, j + 1)] : 0.0;
        gr[s.at(i, j)] = (up - phi[s.at(i, j - 1)]) / (2.0 * dr);
      }
    }
  const size_t np = s.x.size();
  s.gbar.assign(np, 1.0);
  const int T = np >= 4096 ? g_threads : 1;
  std::vector<Dep> dep = deposit_targets(s, T, true);
  for_ranges(np, T, [&](int t, size_t k_lo, size_t k_hi) {
    double* chi = dep[t].chi;
    for (size_t k = k_lo; k < k_hi; ++k) {
      double ux = s.x[k] / dx - (double)s.shift;
      double r = std::sqrt(s.y[k] * s.y[k] + s.z[k] * s.z[k]);
      double ur = r / dr;
      Sh Px = primal(s, ux), Dx = dual(s, ux), Pr = primal(s, ur), Dr = dual(s, ur);
      double c = 1.0, sn = 0.0;
      if (r > 0.0) {
        c = s.y[k] / r;
        sn = s.z[k] / r;
      }
      /* parities across the axis (R23): axial components (-1)^m, radial and
       * azimuthal ones (-1)^(m+1); Phi and its x-derivative even, its
       * r-derivative odd */
      double ex = interp(s, s.Ex, Dx, Pr, Nx - 1, Nr, PRIMAL_R, 1.0);
      double er = interp(s, s.Er, Px, Dr, Nx, Nr - 1, HALF_R, -1.0);
      double bt = interp(s, s.Btb, Dx, Dr, Nx - 1, Nr - 1, HALF_R, -1.0);
      double et = 0.0, bx = 0.0, br = 0.0;
      double ph = interp(s, phi, Px, Pr, Nx, Nr, PRIMAL_R, 1.0);
      double gxp = interp(s, gx, Px, Pr, Nx, Nr, PRIMAL_R, 1.0);
      double grp = interp(s, gr, Px, Pr, Nx, Nr, PRIMAL_R, -1.0);
      if (s.m1()) {
        ex += mode1(interp(s, s.Ex1, Dx, Pr, Nx - 1, Nr, PRIMAL_R, -1.0), c, sn);
        er += mode1(interp(s, s.Er1, Px, Dr, Nx, Nr - 1, HALF_R, 1.0), c, sn);
        et += mode1(interp(s, s.Et1, Px, Pr, Nx, Nr, PRIMAL_R, 1.0), c, sn);
        bx += mode1(interp(s, s.Bxb1, Px, Dr, Nx, Nr - 1, HALF_R, -1.0), c, sn);
        br += mode1(interp(s, s.Brb1, Dx, Pr, Nx - 1, Nr, PRIMAL_R, 1.0), c, sn);
        bt += mode1(interp(s, s.Btb1, Dx, Dr, Nx - 1, Nr - 1, HALF_R, 1.0), c, sn);
      }
      /* rotate (x, r, theta) components to Cartesian */
      double E[3] = {ex, er * c - et * sn, er * sn + et * c};
      double B[3] = {bx, br * c - bt * sn, br * sn + bt * c};
      double G[3] = {gxp, grp * c, grp * sn};
      double p[3] = {s.px[k], s.py[k], s.pz[k]};
      double g0 = std::sqrt(1.0 + p[0] * p[0] + p[1] * p[1] + p[2] * p[2] + ph);
      double F[3], pm[3];
      for (int d = 0; d < 3; ++d) {
        F[d] = -E[d] - G[d] / (2.0 * g0);
        pm[d] = p[d] + 0.5 * dt * F[d];
      }
      double gb = std::sqrt(1.0 + pm[0] * pm[0] + pm[1] * pm[1] + pm[2] * pm[2] + ph);
      double t[3], sv[3];
      for (int d = 0; d < 3; ++d) t[d] = -0.5 * dt * B[d] / gb;
      double t2 = t[0] * t[0] + t[1] * t[1] + t[2] * t[2];
      for (int d = 0; d < 3; ++d) sv[d] = 2.0 * t[d] / (1.0 + t2);
      double pp[3] = {pm[0] + pm[1] * t[2] - pm[2] * t[1], pm[1] + pm[2] * t[0] - pm[0] * t[2],
                      pm[2] + pm[0] * t[1] - pm[1] * t[0]};
      double pl[3] = {pm[0] + pp[1] * sv[2] - pp[2] * sv[1], pm[1] + pp[2] * sv[0] - pp[0] * sv[2],
                      pm[2] + pp[0] * sv[1] - pp[1] * sv[0]};
      s.px[k] = pl[0] + 0.5 * dt * F[0];
      s.py[k] = pl[1] + 0.5 * dt * F[1];
      s.pz[k] = pl[2] + 0.5 * dt * F[2];
      s.gbar[k] = gb;
      /* chi^n deposit at the primal nodes around x^n (even across the
       * axis); the volume is that of the row the contribution lands on */
      for (int a = 0; a < Px.n; ++a)
        for (int b = 0; b < Pr.n; ++b) {
          int i = Px.i + a, j = Pr.i + b;
          if (j < 0) j = mirror_row(j, PRIMAL_R);
          if (i < 0 || i > Nx || j < 0 || j > Nr) continue;
          chi[s.at(i, j)] += s.w[k] * Px.w[a] * Pr.w[b] / (gb * vol_node(s, j));
        }
    }
  });
  if (T > 1) sum_in_thread_order(s.chi, s.t_chi, T);
}

/* -------------------------------------------- envelope stage (Sec. 3) --
 * Centred differences of Eq. envelope_equation (R3, R4):
 *   A^{n+1} = (1+i dt)/(1+dt^2) [ 2A^n - (1+i dt) A^{n-1}
 *             + dt^2 ( lap A^n - chi^n A^n + 2i (A_{i+1} - A_{i-1})/(2dx) ) ]  */
void envelope(Sim& s) {
  const int Nx = s.Nx, Nr = s.Nr;
  const double dx = s.dx, dr = s.dr, dt = s.dt;
  const bool per = s.p.env_bc_x == 1, mir = s.p.env_bc_r == 1;
  std::vector<cplx> An(s.ng, 0.0);
  const cplx pref = (1.0 + kI * dt) / (1.0 + dt * dt);
  int i_lo = per ? 0 : 1, i_hi = per ? Nx - 1 : Nx - 1;
  int j_hi = mir ? Nr : Nr - 1;
  for (int i = i_lo; i <= i_hi; ++i)
    for (int j = 0; j <= j_hi; ++j) {
      int ip = i + 1, im = i - 1;
      if (per) {
        ip = (i + 1) % Nx;
        im = (i - 1 + Nx) % Nx;
      }
      cplx a = s.A[s.at(i, j)];
      cplx aip = s.A[s.at(ip, j)], aim = s.A[s.at(im, j)];
      cplx lap = (aip - 2.0 * a + aim) / (dx * dx);
      if (j == 0) {
        lap += 4.0 * (s.A[s.at(i, 1)] - a) / (dr * dr);
      } else {
        cplx up = (j + 1 <= Nr) ? s.A[s.at(i, j + 1)] : s.A[s.at(i, Nr - 1)];
        cplx dn = s.A[s.at(i, j - 1)];
        double rj = j * dr;
        lap += (up - 2.0 * a + dn) / (dr * dr) + (up - dn) / (2.0 * rj * dr);
      }
      cplx R = lap - s.chi[s.at(i, j)] * a + 2.0 * kI * (aip - aim) / (2.0 * dx);
      An[s.at(i, j)] = pref * (2.0 * a - (1.0 + kI * dt) * s.Ap[s.at(i, j)] + dt * dt * R);
    }
  if (per)
    for (int j = 0; j <= Nr; ++j) An[s.at(Nx, j)] = An[s.at(0, j)];
  s.Ap.swap(s.A);
  s.A.swap(An);
}

/* ------------------------------------- current deposit (R11, mode 0) --
 * Esirkepov decomposition of the change of the linear node weights
 * between (ux0, ur0) and (ux1, ur1) (cell units, window-relative):
 *   W_x = (S1x - S0x)(S0r + S1r)/2,  W_r = (S1r - S0r)(S0x + S1x)/2,
 * fluxes accumulated from the low side, divided by face area and dt.    */
void deposit_J_mode0(const Sim& s, const Dep& d, double w, double ux0, double ur0, double ux1, double ur1) {
  const int Nx = s.Nx, Nr = s.Nr;
  const double q = -1.0;
  Sh a0 = primal(s, ux0), a1 = primal(s, ux1), b0 = primal(s, ur0), b1 = primal(s, ur1);
  /* the two stencils, on the union of their nodes (one node more than a
   * stencil, since a particle moves less than a cell per step) */
  const int K = a0.n + 1;
  int imin = std::min(a0.i, a1.i), jmin = std::min(b0.i, b1.i);
  double S0x[4] = {0, 0, 0, 0}, S1x[4] = {0, 0, 0, 0}, S0r[4] = {0, 0, 0, 0}, S1r[4] = {0, 0, 0, 0};
  for (int m = 0; m < a0.n; ++m) {
    S0x[a0.i - imin + m] += a0.w[m];
    S1x[a1.i - imin + m] += a1.w[m];
    S0r[b0.i - jmin + m] += b0.w[m];
    S1r[b1.i - jmin + m] += b1.w[m];
  }
  /* J_x on row j: even across the axis (a row below folds onto its mirror) */
  for (int b = 0; b < K; ++b) {
    double acc = 0.0;
    for (int a = 0; a < K; ++a) {
      acc += (S1x[a] - S0x[a]) * (S0r[b] + S1r[b]) * 0.5;
      int i = imin + a, j = jmin + b;
      if (j < 0) j = mirror_row(j, PRIMAL_R);
      if (i < 0 || i > Nx - 1 || j < 0 || j > Nr) continue;
      d.jx[s.at(i, j)] += -q * w * acc / (area_x(s, j) * s.dt);
    }
  }
  /* J_r at the face j + 1/2: odd across the axis (the face at -1/2 folds
   * onto +1/2 with the opposite sign) */
  for (int a = 0; a < K; ++a) {
    double acc = 0.0;
    for (int b = 0; b < K; ++b) {
      acc += (S1r[b] - S0r[b]) * (S0x[a] + S1x[a]) * 0.5;
      int i = imin + a, j = jmin + b;
      double sg = 1.0;
      if (j < 0) {
        j = mirror_row(j, HALF_R);
        sg = -1.0;
      }
      if (i < 0 || i > Nx || j < 0 || j > Nr - 1) continue;
      d.jr[s.at(i, j)] += sg * -q * w * acc / (area_r(s, j) * s.dt);
    }
  }
}

/* mode-1 current, deposited directly with the particle's mid-point shape:
 * J_1 += 2 q w v S e^{+i theta} / V (factor 2 and e^{+i theta} from the
 * Fourier coefficient of a point current at azimuth theta).              */
void deposit_J_mode1(const Sim& s, const Dep& d, double w, double ux, double ur, double c, double sn,
                     const double v[3]) {
  const int Nx = s.Nx, Nr = s.Nr;
  const double q = -1.0;
  double vr = v[1] * c + v[2] * sn, vt = -v[1] * sn + v[2] * c;
  cplx e(c, sn);
  Sh Px = primal(s, ux), Dx = dual(s, ux), Pr = primal(s, ur), Dr = dual(s, ur);
  /* J_x1 at (i+1/2, j): odd across the axis for mode 1 */
  for (int a = 0; a < Dx.n; ++a)
    for (int b = 0; b < Pr.n; ++b) {
      int i = Dx.i + a, j = Pr.i + b;
      double sg = 1.0;
      if (j < 0) {
        j = mirror_row(j, PRIMAL_R);
        sg = -1.0;
      }
      if (i < 0 || i > Nx - 1 || j < 0 || j > Nr) continue;
      d.jx1[s.at(i, j)] += sg * 2.0 * q * w * v[0] * Dx.w[a] * Pr.w[b] * e / vol_node(s, j);
    }
  /* J_r1 at (i, j+1/2): even for mode 1 (row -1/2 folds onto +1/2) */
  for (int a = 0; a < Px.n; ++a)
    for (int b = 0; b < Dr.n; ++b) {
      int i = Px.i + a, j = Dr.i + b;
      if (j < 0) j = mirror_row(j, HALF_R);
      if (i < 0 || i > Nx || j < 0 || j > Nr - 1) continue;
      d.jr1[s.at(i, j)] += 2.0 * q * w * vr * Px.w[a] * Dr.w[b] * e / vol_half(s, j);
    }
  /* J_t1 at (i, j): even for mode 1 */
  for (int a = 0; a < Px.n; ++a)
    for (int b = 0; b < Pr.n; ++b) {
      int i = Px.i + a, j = Pr.i + b;
      if (j < 0) j = mirror_row(j, PRIMAL_R);
      if (i < 0 || i > Nx || j < 0 || j > Nr) continue;
      d.jt1[s.at(i, j)] += 2.0 * q * w * vt * Px.w[a] * Pr.w[b] * e / vol_node(s, j);
    }
}

/* -------------------------------------------- position stage (Sec. 3) --
 * gbar^{n+1/2} from p^{n+1/2} and Phi^{n+1/2} (R8); x^{n+1} = x^n + dt p/gbar
 * in Cartesian space; reflect at r_max, remove outside the window (R16);
 * deposit J^{n+1/2} (R11).                                               */
void position_J(Sim& s) {
  const int Nx = s.Nx, Nr = s.Nr;
  const double dx = s.dx, dr = s.dr, dt = s.dt;
  /* after the envelope stage A = A^{n+1}, Ap = A^n */
  std::vector<double> phh(s.ng);
  for (size_t k = 0; k < s.ng; ++k) phh[k] = 0.25 * (std::norm(s.A[k]) + std::norm(s.Ap[k]));
  const double rmax = Nr * dr;
  const double xlo = (double)s.shift * dx, xhi = (double)(s.shift + Nx) * dx;
  const size_t np = s.x.size();
  std::vector<char> keep(np, 1);
  const int T = np >= 4096 ? g_threads : 1;
  std::vector<Dep> dep = deposit_targets(s, T, false);
  for_ranges(np, T, [&](int t, size_t k_lo, size_t k_hi) {
    const Dep& d = dep[t];
    for (size_t k = k_lo; k < k_hi; ++k) {
      double ux = s.x[k] / dx - (double)s.shift;
      double r = std::sqrt(s.y[k] * s.y[k] + s.z[k] * s.z[k]);
      double ph = interp(s, phh, primal(s, ux), primal(s, r / dr), Nx, Nr, PRIMAL_R, 1.0);
      double p[3] = {s.px[k], s.py[k], s.pz[k]};
      double g = std::sqrt(1.0 + p[0] * p[0] + p[1] * p[1] + p[2] * p[2] + ph);
      double v[3] = {p[0] / g, p[1] / g, p[2] / g};
      double xn = s.x[k] + dt * v[0], yn = s.y[k] + dt * v[1], zn = s.z[k] + dt * v[2];
      double rn = std::sqrt(yn * yn + zn * zn);
      if (rn >= rmax) {
        double f = (2.0 * rmax - rn) / rn;
        double cr = yn / rn, sr = zn / rn;
        yn *= f;
        zn *= f;
        rn = 2.0 * rmax - rn;
        double prad = s.py[k] * cr + s.pz[k] * sr;
        s.py[k] -= 2.0 * prad * cr;
        s.pz[k] -= 2.0 * prad * sr;
      }
      if (xn < xlo || xn >= xhi) {
        keep[k] = 0;
        continue;
      }
      deposit_J_mode0(s, d, s.w[k], ux, r / dr, xn / dx - (double)s.shift, rn / dr);
      if (s.m1()) {
        double xm = 0.5 * (s.x[k] + xn), ym = 0.5 * (s.y[k] + yn), zm = 0.5 * (s.z[k] + zn);
        double rm = std::sqrt(ym * ym + zm * zm);
        double c = 1.0, sn = 0.0;
        if (rm > 0.0) {
          c = ym / rm;
          sn = zm / rm;
        }
        deposit_J_mode1(s, d, s.w[k], xm / dx - (double)s.shift, rm / dr, c, sn, v);
      }
      s.x[k] = xn;
      s.y[k] = yn;
      s.z[k] = zn;
    }
  });
  if (T > 1) {
    sum_in_thread_order(s.Jx, s.t_jx, T);
    sum_in_thread_order(s.Jr, s.t_jr, T);
    if (s.m1()) {
      sum_in_thread_order(s.Jx1, s.t_jx1, T);
      sum_in_thread_order(s.Jr1, s.t_jr1, T);
      sum_in_thread_order(s.Jt1, s.t_jt1, T);
    }
  }
  size_t m = 0;
  for (size_t k = 0; k < np; ++k) {
    if (!keep[k]) continue;
    s.x[m] = s.x[k]; s.y[m] = s.y[k]; s.z[m] = s.z[k];
    s.px[m] = s.px[k]; s.py[m] = s.py[k]; s.pz[m] = s.pz[k];
    s.w[m] = s.w[k]; s.gbar[m] = s.gbar[k]; s.id[m] = s.id[k];
    ++m;
  }
  for (auto* v : {&s.x, &s.y, &s.z, &s.px, &s.py, &s.pz, &s.w, &s.gbar}) v->resize(m);
  s.id.resize(m);
}

/* --------------------------------------- binomial current filter (R24) --
 * One pass on a component f valid for 0 <= i <= imax, 0 <= j <= jmax:
 * f <- (f_{i-1} + 2 f_i + f_{i+1})/4 along x, then the same along r.  Zero
 * beyond the valid ranges; the row below the axis is the mirror of row 1
 * (primal in r: J(-1) = parity J(1)) or of row 0 (half-integer in r:
 * J(-1/2) = parity J(1/2)).                                                */
template <class T>
void binomial_pass(const Sim& s, std::vector<T>& f, int imax, int jmax, bool half_r, double parity) {
  std::vector<T> g(f.size(), T(0));
  for (int i = 0; i <= imax; ++i)
    for (int j = 0; j <= jmax; ++j) {
      const T lo = i > 0 ? f[s.at(i - 1, j)] : T(0);
      const T hi = i < imax ? f[s.at(i + 1, j)] : T(0);
      g[s.at(i, j)] = 0.25 * lo + 0.5 * f[s.at(i, j)] + 0.25 * hi;
    }
  for (int i = 0; i <= imax; ++i)
    for (int j = 0; j <= jmax; ++j) {
      const T lo = j > 0 ? g[s.at(i, j - 1)] : parity * g[s.at(i, half_r ? 0 : std::min(1, jmax))];
      const T hi = j < jmax ? g[s.at(i, j + 1)] : T(0);
      f[s.at(i, j)] = 0.25 * lo + 0.5 * g[s.at(i, j)] + 0.25 * hi;
    }
}

/* R24 on J^{n+1/2}: mode 0 J_x (axial, even; i+1/2, j) and J_r (radial,
 * odd; i, j+1/2); mode 1 J_x (axial, odd), J_r (radial, even; i, j+1/2)
 * and J_t (azimuthal, even; i, j).  The odd mode-1 J_x vanishes on the axis
 * (R23), so its axis row is zeroed first (the field update never reads it):
 * the passes then act on an odd function.                                 */
void filter_J(Sim& s) {
  const int Nx = s.Nx, Nr = s.Nr;
  if (s.m1() && s.p.filter_passes > 0)
    for (int i = 0; i <= Nx; ++i) s.Jx1[s.at(i, 0)] = 0.0;
  for (int k = 0; k < s.p.filter_passes; ++k) {
    binomial_pass(s, s.Jx, Nx - 1, Nr, false, +1.0);
    binomial_pass(s, s.Jr, Nx, Nr - 1, true, -1.0);
    if (s.m1()) {
      binomial_pass(s, s.Jx1, Nx - 1, Nr, false, -1.0);
      binomial_pass(s, s.Jr1, Nx, Nr - 1, true, +1.0);
      binomial_pass(s, s.Jt1, Nx, Nr, false, +1.0);
    }
  }
}

/* ---------------------------------------------- Maxwell (Sec. 2, 3) --
 * Yee leap-frog of Eq. MaxwellEqsCylindrical with dt/2 staggering:
 * E^{n+1} from B^{n+1/2} and J^{n+1/2}, then B^{n+3/2} from E^{n+1};
 * Bbar^{n+1} = (B^{n+1/2} + B^{n+3/2})/2.  On the axis the E_x update uses
 * the flux through the disc r < dr/2: (1/r) d(r B)/dr -> 4 B(1/2)/dr.
 * Mode 1 (not in the paper; from the Fourier-mode curl with d/dtheta ->
 * -i): axial components vanish on the axis, r/theta components use even
 * ghosts and axial ones odd ghosts.                                        */
void maxwell(Sim& s) {
  const int Nx = s.Nx, Nr = s.Nr;
  const double dx = s.dx, dr = s.dr, dt = s.dt;
  /* Ampere, mode 0 */
  for (int i = 1; i <= Nx - 1; ++i)
    for (int j = 0; j <= Nr - 1; ++j)
      s.Er[s.at(i, j)] -= dt * ((s.Bt[s.at(i, j)] - s.Bt[s.at(i - 1, j)]) / dx + s.Jr[s.at(i, j)]);
  for (int j = 0; j <= Nr - 1; ++j) {
    s.Er[s.at(0, j)] = 0.0;
    s.Er[s.at(Nx, j)] = 0.0;
  }
  for (int i = 0; i <= Nx - 1; ++i) {
    s.Ex[s.at(i, 0)] += dt * (4.0 * s.Bt[s.at(i, 0)] / dr - s.Jx[s.at(i, 0)]);
    for (int j = 1; j <= Nr - 1; ++j)
      s.Ex[s.at(i, j)] +=
          dt * (((j + 0.5) * s.Bt[s.at(i, j)] - (j - 0.5) * s.Bt[s.at(i, j - 1)]) / (j * dr) -
                s.Jx[s.at(i, j)]);
    s.Ex[s.at(i, Nr)] = 0.0;
  }
  /* Ampere, mode 1 */
  if (s.m1()) {
    for (int i = 0; i <= Nx - 1; ++i) {
      s.Ex1[s.at(i, 0)] = 0.0;
      for (int j = 1; j <= Nr - 1; ++j)
        s.Ex1[s.at(i, j)] +=
            dt * (((j + 0.5) * s.Bt1[s.at(i, j)] - (j - 0.5) * s.Bt1[s.at(i, j - 1)]) / (j * dr) +
                  kI * s.Br1[s.at(i, j)] / (j * dr) - s.Jx1[s.at(i, j)]);
      s.Ex1[s.at(i, Nr)] = 0.0;
    }
    for (int i = 1; i <= Nx - 1; ++i)
      for (int j = 0; j <= Nr - 1; ++j)
        s.Er1[s.at(i, j)] += dt * (-kI * s.Bx1[s.at(i, j)] / ((j + 0.5) * dr) -
                                   (s.Bt1[s.at(i, j)] - s.Bt1[s.at(i - 1, j)]) / dx -
                                   s.Jr1[s.at(i, j)]);
    for (int i = 1; i <= Nx - 1; ++i) {
      s.Et1[s.at(i, 0)] += dt * ((s.Br1[s.at(i, 0)] - s.Br1[s.at(i - 1, 0)]) / dx -
                                 2.0 * s.Bx1[s.at(i, 0)] / dr - s.Jt1[s.at(i, 0)]);
      for (int j = 1; j <= Nr - 1; ++j)
        s.Et1[s.at(i, j)] += dt * ((s.Br1[s.at(i, j)] - s.Br1[s.at(i - 1, j)]) / dx -
                                   (s.Bx1[s.at(i, j)] - s.Bx1[s.at(i, j - 1)]) / dr -
                                   s.Jt1[s.at(i, j)]);
      s.Et1[s.at(i, Nr)] = 0.0;
    }
    for (int j = 0; j <= Nr; ++j) {
      if (j <= Nr - 1) {
        s.Er1[s.at(0, j)] = 0.0;
        s.Er1[s.at(Nx, j)] = 0.0;
      }
      s.Et1[s.at(0, j)] = 0.0;
      s.Et1[s.at(Nx, j)] = 0.0;
    }
  }
  /* Faraday, mode 0, and the time-centred average */
  for (int i = 0; i <= Nx - 1; ++i)
    for (int j = 0; j <= Nr - 1; ++j) {
      double b0 = s.Bt[s.at(i, j)];
      double b1 = b0 + dt * ((s.Ex[s.at(i, j + 1)] - s.Ex[s.at(i, j)]) / dr -
                             (s.Er[s.at(i + 1, j)] - s.Er[s.at(i, j)]) / dx);
      s.Bt[s.at(i, j)] = b1;
      s.Btb[s.at(i, j)] = 0.5 * (b0 + b1);
    }
  /* Faraday, mode 1 */
  if (s.m1()) {
    for (int i = 0; i <= Nx; ++i)
      for (int j = 0; j <= Nr - 1; ++j) {
        cplx b0 = s.Bx1[s.at(i, j)];
        cplx b1 = b0 - dt * (((j + 1.0) * s.Et1[s.at(i, j + 1)] - (double)j * s.Et1[s.at(i, j)]) /
                                 ((j + 0.5) * dr) +
                             kI * s.Er1[s.at(i, j)] / ((j + 0.5) * dr));
        s.Bx1[s.at(i, j)] = b1;
        s.Bxb1[s.at(i, j)] = 0.5 * (b0 + b1);
      }
    for (int i = 0; i <= Nx - 1; ++i)
      for (int j = 0; j <= Nr; ++j) {
        cplx b0 = s.Br1[s.at(i, j)];
        cplx ex_over_r = j == 0 ? s.Ex1[s.at(i, 1)] / dr : s.Ex1[s.at(i, j)] / (j * dr);
        cplx b1 = b0 + dt * (kI * ex_over_r + (s.Et1[s.at(i + 1, j)] - s.Et1[s.at(i, j)]) / dx);
        s.Br1[s.at(i, j)] = b1;
        s.Brb1[s.at(i, j)] = 0.5 * (b0 + b1);
      }
    for (int i = 0; i <= Nx - 1; ++i)
      for (int j = 0; j <= Nr - 1; ++j) {
        cplx b0 = s.Bt1[s.at(i, j)];
        cplx b1 = b0 + dt * ((s.Ex1[s.at(i, j + 1)] - s.Ex1[s.at(i, j)]) / dr -
                             (s.Er1[s.at(i + 1, j)] - s.Er1[s.at(i, j)]) / dx);
        s.Bt1[s.at(i, j)] = b1;
        s.Btb1[s.at(i, j)] = 0.5 * (b0 + b1);
      }
  }
}

/* ------------------------------------------------------ moving window --
 * After step n the window moves by one cell when (n+1) dt >= (shift+1) dx
 * (Sec. 4 uses a moving window; timing, drop and injection are R18):
 * particles of the vacated cell column are dropped, every grid moves one
 * column, the entering column starts at zero, the new left edge takes its
 * boundary values, and the entering cell column is loaded with plasma.   */
template <class T>
void shift_grid(Sim& s, std::vector<T>& f, bool dual_x) {
  if (f.empty()) return;
  const int last = dual_x ? s.Nx - 1 : s.Nx;
  for (int i = 0; i < last; ++i)
    for (int j = 0; j <= s.Nr; ++j) f[s.at(i, j)] = f[s.at(i + 1, j)];
  for (int i = last; i <= s.Nx; ++i)
    for (int j = 0; j <= s.Nr; ++j) f[s.at(i, j)] = T(0);
}

void window(Sim& s) {
  if (!s.p.moving_window) return;
  if ((double)(s.n + 1) * s.dt < (double)(s.shift - s.p.start_col + 1) * s.dx) return;
  const double xcut = (double)(s.shift + 1) * s.dx;
  size_t m = 0;
  for (size_t k = 0; k < s.x.size(); ++k) {
    if (s.x[k] < xcut) continue;
    s.x[m] = s.x[k]; s.y[m] = s.y[k]; s.z[m] = s.z[k];
    s.px[m] = s.px[k]; s.py[m] = s.py[k]; s.pz[m] = s.pz[k];
    s.w[m] = s.w[k]; s.gbar[m] = s.gbar[k]; s.id[m] = s.id[k];
    ++m;
  }
  for (auto* v : {&s.x, &s.y, &s.z, &s.px, &s.py, &s.pz, &s.w, &s.gbar}) v->resize(m);
  s.id.resize(m);
  /* primal-x grids */
  shift_grid(s, s.A, false);
  shift_grid(s, s.Ap, false);
  shift_grid(s, s.chi, false);
  shift_grid(s, s.Er, false);
  shift_grid(s, s.Jr, false);
  shift_grid(s, s.Er1, false);
  shift_grid(s, s.Et1, false);
  shift_grid(s, s.Bx1, false);
  shift_grid(s, s.Bxb1, false);
  shift_grid(s, s.Jr1, false);
  shift_grid(s, s.Jt1, false);
  /* dual-x grids */
  shift_grid(s, s.Ex, true);
  shift_grid(s, s.Bt, true);
  shift_grid(s, s.Btb, true);
  shift_grid(s, s.Jx, true);
  shift_grid(s, s.Ex1, true);
  shift_grid(s, s.Br1, true);
  shift_grid(s, s.Bt1, true);
  shift_grid(s, s.Brb1, true);
  shift_grid(s, s.Btb1, true);
  shift_grid(s, s.Jx1, true);
  s.shift += 1;
  for (int j = 0; j <= s.Nr; ++j) {
    s.A[s.at(0, j)] = 0.0;
    s.Ap[s.at(0, j)] = 0.0;
    s.Er[s.at(0, j)] = 0.0;
    if (s.m1()) {
      s.Er1[s.at(0, j)] = 0.0;
      s.Et1[s.at(0, j)] = 0.0;
    }
  }
  const int64_t col = s.shift + s.Nx - 1;
  for (int j = 0; j < s.Nr; ++j) load_cell(s, col, j);
}

Sim* as_sim(void* h) { return static_cast<Sim*>(h); }

bool check_params(const oracle_params* p) {
  if (!p || p->size != (int32_t)sizeof(oracle_params) || p->version != ORACLE_PARAMS_VERSION)
    return false;
  if (p->nx < 2 || p->nr < 2 || p->n_modes < 1 || p->n_modes > 2) return false;
  if (p->ppc_x < 1 || p->ppc_r < 1 || p->ppc_t < 1) return false;
  if (!(p->dx > 0 && p->dr > 0 && p->dt > 0)) return false;
  /* one cell at most per step along each axis (the current deposit needs it) */
  if (!(p->dt < p->dx && p->dt < p->dr)) return false;
  if (p->start_col < 0) return false;
  if (p->filter_passes < 0 || p->filter_passes > 64) return false;
  if (p->shape_order < 0 || p->shape_order > 2) return false;
  return true;
}

}  // namespace

/* ============================================================= C ABI == */
extern "C" {

int oracle_set_threads(int n) {
  if (n < 1 || n > 256) return ORACLE_EINVAL;
  g_threads = n;
  return ORACLE_OK;
}

double oracle_uniform(uint64_t seed, uint64_t stream, int64_t col, int64_t j) {
  return uniform_of(seed, stream, col, j);
}

int oracle_create(const oracle_params* p, void** out) {
  if (!out || !check_params(p)) return ORACLE_EINVAL;
  Sim* s = new (std::nothrow) Sim();
  if (!s) return ORACLE_EINVAL;
  s->p = *p;
  s->Nx = p->nx;
  s->Nr = p->nr;
  s->NR1 = p->nr + 1;
  s->ng = (size_t)(p->nx + 1) * (p->nr + 1);
  s->dx = p->dx;
  s->dr = p->dr;
  s->dt = p->dt;
  s->n = 0;
  s->shift = p->start_col;
  init_fields(*s);
  if (p->profile != ORACLE_PROFILE_NONE)
    for (int64_t c = 0; c < p->nx; ++c)
      for (int j = 0; j < p->nr; ++j) load_cell(*s, p->start_col + c, j);
  *out = s;
  return ORACLE_OK;
}

void oracle_destroy(void* h) { delete as_sim(h); }

int oracle_momentum_chi(void* h) {
  momentum_chi(*as_sim(h));
  return ORACLE_OK;
}
int oracle_envelope(void* h) {
  envelope(*as_sim(h));
  return ORACLE_OK;
}
int oracle_position_J(void* h) {
  position_J(*as_sim(h));
  return ORACLE_OK;
}
int oracle_field_step(void* h) {
  Sim& s = *as_sim(h);
  if (s.p.filter_passes > 0) filter_J(s);
  maxwell(s);
  window(s);
  s.n += 1;
  return ORACLE_OK;
}
int oracle_filter_J(void* h) {
  filter_J(*as_sim(h));
  return ORACLE_OK;
}
int oracle_step(void* h, int nsteps) {
  for (int k = 0; k < nsteps; ++k) {
    oracle_momentum_chi(h);
    oracle_envelope(h);
    oracle_position_J(h);
    oracle_field_step(h);
  }
  return ORACLE_OK;
}

int oracle_state(void* h, int64_t* n, int64_t* shift, int64_t* np) {
  Sim& s = *as_sim(h);
  if (n) *n = s.n;
  if (shift) *shift = s.shift;
  if (np) *np = (int64_t)s.x.size();
  return ORACLE_OK;
}

int oracle_get_particles(void* h, double* x, double* y, double* z, double* px, double* py,
                         double* pz, double* w, uint32_t* id) {
  Sim& s = *as_sim(h);
  size_t np = s.x.size();
  if (x) std::memcpy(x, s.x.data(), np * sizeof(double));
  if (y) std::memcpy(y, s.y.data(), np * sizeof(double));
  if (z) std::memcpy(z, s.z.data(), np * sizeof(double));
  if (px) std::memcpy(px, s.px.data(), np * sizeof(double));
  if (py) std::memcpy(py, s.py.data(), np * sizeof(double));
  if (pz) std::memcpy(pz, s.pz.data(), np * sizeof(double));
  if (w) std::memcpy(w, s.w.data(), np * sizeof(double));
  if (id) std::memcpy(id, s.id.data(), np * sizeof(uint32_t));
  return ORACLE_OK;
}

int oracle_set_particles(void* h, int64_t n, const double* x, const double* y, const double* z,
                         const double* px, const double* py, const double* pz, const double* w,
                         const uint32_t* id) {
  Sim& s = *as_sim(h);
  if (n < 0 || (n > 0 && (!x || !y || !z || !px || !py || !pz || !w || !id)))
    return ORACLE_EINVAL;
  s.x.assign(x, x + n);
  s.y.assign(y, y + n);
  s.z.assign(z, z + n);
  s.px.assign(px, px + n);
  s.py.assign(py, py + n);
  s.pz.assign(pz, pz + n);
  s.w.assign(w, w + n);
  s.id.assign(id, id + n);
  s.gbar.assign(n, 1.0);
  return ORACLE_OK;
}

int oracle_get_gbar(void* h, double* g) {
  Sim& s = *as_sim(h);
  std::memcpy(g, s.gbar.data(), s.gbar.size() * sizeof(double));
  return ORACLE_OK;
}

static std::vector<double>* real_field(Sim& s, int f) {
  switch (f) {
    case ORACLE_F_CHI: return &s.chi;
    case ORACLE_F_EX: return &s.Ex;
    case ORACLE_F_ER: return &s.Er;
    case ORACLE_F_BT: return &s.Bt;
    case ORACLE_F_BT_BAR: return &s.Btb;
    case ORACLE_F_JX: return &s.Jx;
    case ORACLE_F_JR: return &s.Jr;
    default: return nullptr;
  }
}
static std::vector<cplx>* cplx_field(Sim& s, int f) {
  switch (f) {
    case ORACLE_F_ENV: return &s.A;
    case ORACLE_F_ENV_PREV: return &s.Ap;
    case ORACLE_F_EX1: return &s.Ex1;
    case ORACLE_F_ER1: return &s.Er1;
    case ORACLE_F_ET1: return &s.Et1;
    case ORACLE_F_BX1: return &s.Bx1;
    case ORACLE_F_BR1: return &s.Br1;
    case ORACLE_F_BT1: return &s.Bt1;
    case ORACLE_F_BX1_BAR: return &s.Bxb1;
    case ORACLE_F_BR1_BAR: return &s.Brb1;
    case ORACLE_F_BT1_BAR: return &s.Btb1;
    case ORACLE_F_JX1: return &s.Jx1;
    case ORACLE_F_JR1: return &s.Jr1;
    case ORACLE_F_JT1: return &s.Jt1;
    default: return nullptr;
  }
}

int oracle_get_field(void* h, int f, double* out) {
  Sim& s = *as_sim(h);
  if (auto* r = real_field(s, f)) {
    std::memcpy(out, r->data(), s.ng * sizeof(double));
    return ORACLE_OK;
  }
  if (auto* c = cplx_field(s, f)) {
    if (c->empty()) return ORACLE_EINVAL;
    for (size_t k = 0; k < s.ng; ++k) {
      out[2 * k] = (*c)[k].real();
      out[2 * k + 1] = (*c)[k].imag();
    }
    return ORACLE_OK;
  }
  return ORACLE_EINVAL;
}

int oracle_set_field(void* h, int f, const double* in) {
  Sim& s = *as_sim(h);
  if (auto* r = real_field(s, f)) {
    std::memcpy(r->data(), in, s.ng * sizeof(double));
    return ORACLE_OK;
  }
  if (auto* c = cplx_field(s, f)) {
    if (c->empty()) return ORACLE_EINVAL;
    for (size_t k = 0; k < s.ng; ++k) (*c)[k] = cplx(in[2 * k], in[2 * k + 1]);
    return ORACLE_OK;
  }
  return ORACLE_EINVAL;
}

int oracle_diagnostics(void* h, double* out) {
  Sim& s = *as_sim(h);
  for (int k = 0; k < ORACLE_NDIAG; ++k) out[k] = 0.0;
  double nonfinite = 0.0;
  const size_t np = s.x.size();
  out[ORACLE_D_COUNT] = (double)np;
  for (size_t k = 0; k < np; ++k) {
    double p2 = s.px[k] * s.px[k] + s.py[k] * s.py[k] + s.pz[k] * s.pz[k];
    double g = std::sqrt(1.0 + p2);
    out[ORACLE_D_CHARGE] += -s.w[k];
    out[ORACLE_D_KIN] += s.w[k] * p2 / (1.0 + g);
    out[ORACLE_D_LX] += s.w[k] * (s.y[k] * s.pz[k] - s.z[k] * s.py[k]);
    out[ORACLE_D_PX] += s.w[k] * s.px[k];
    double vals[7] = {s.x[k], s.y[k], s.z[k], s.px[k], s.py[k], s.pz[k], s.w[k]};
    for (double v : vals)
      if (!std::isfinite(v)) nonfinite += 1.0;
  }
  const int Nx = s.Nx, Nr = s.Nr;
  double u0 = 0.0, u1 = 0.0;
  for (int i = 0; i <= Nx; ++i)
    for (int j = 0; j <= Nr; ++j) {
      size_t k = s.at(i, j);
      out[ORACLE_D_CHI_V] += s.chi[k] * vol_node(s, j);
      out[ORACLE_D_ENV2_V] += std::norm(s.A[k]) * vol_node(s, j);
      if (i <= Nx - 1) u0 += s.Ex[k] * s.Ex[k] * vol_node(s, j);
      if (j <= Nr - 1) u0 += s.Er[k] * s.Er[k] * vol_half(s, j);
      if (i <= Nx - 1 && j <= Nr - 1) u0 += s.Bt[k] * s.Bt[k] * vol_half(s, j);
      double vals[7] = {s.chi[k], s.A[k].real(), s.A[k].imag(), s.Ex[k], s.Er[k], s.Bt[k],
                        s.Btb[k]};
      for (double v : vals)
        if (!std::isfinite(v)) nonfinite += 1.0;
      if (s.m1()) {
        if (i <= Nx - 1) u1 += std::norm(s.Ex1[k]) * vol_node(s, j);
        if (j <= Nr - 1) u1 += std::norm(s.Er1[k]) * vol_half(s, j);
        u1 += std::norm(s.Et1[k]) * vol_node(s, j);
        if (j <= Nr - 1) u1 += std::norm(s.Bx1[k]) * vol_half(s, j);
        if (i <= Nx - 1) u1 += std::norm(s.Br1[k]) * vol_node(s, j);
        if (i <= Nx - 1 && j <= Nr - 1) u1 += std::norm(s.Bt1[k]) * vol_half(s, j);
      }
    }
  /* a mode-1 amplitude F carries <Re[F e^{-i theta}]^2> = |F|^2/2 */
  out[ORACLE_D_UEM] = 0.5 * u0 + 0.25 * u1;
  out[ORACLE_D_NONFINITE] = nonfinite;
  return ORACLE_OK;
}

}  // extern "C"
