/*
 * envpic.h -- C ABI of the MI355X (gfx950) cylindrical envelope PIC library.
 *
 * Method: Massimo, Zemzemi, Beck, Derouillat, Specka, "Efficient cylindrical
 * envelope modeling for laser wakefield acceleration", arXiv:1912.04674.
 * One step advances the state {x^n, p^{n-1/2}, A^n, A^{n-1}, E^n, B^{n+1/2},
 * Bbar^n} to n+1:
 *   1. momentum stage  (Sec. 3, Eq. motion_equations_cartesian; Sec. 2,
 *      Eq. EquationsOfMotion): gather E, Bbar, Phi = |A|^2/2 and grad Phi at
 *      x^n, ponderomotive Boris push p^{n-1/2} -> p^{n+1/2}, deposit chi^n;
 *   2. envelope stage  (Sec. 3, Eq. envelope_solver and the cylindrical
 *      Laplacian after it): A^{n+1} from A^n, A^{n-1}, chi^n;
 *   3. position stage  (Sec. 2, Eq. EquationsOfMotion): x^n -> x^{n+1} with
 *      gbar from Phi^{n+1/2}, deposit J^{n+1/2}; when the window moves at
 *      this step, the plasma of the entering column is loaded (Sec. 4);
 *   4. field stage     (Sec. 2, Eq. MaxwellEqsCylindrical; Sec. 3, FDTD with
 *      dt/2 staggering): E^{n+1}, B^{n+3/2}, Bbar^{n+1}; moving window
 *      (Sec. 4); particle tile sort for the next step.
 *
 * Units (Sec. 2): lengths c/w0, time 1/w0, momenta m_e c, fields
 * m_e c w0 / e, densities n_c.  Electrons only (charge -1, mass 1).
 *
 * Conventions
 *   - Return 0 on success or a negative ENVPIC_E* code; the message is kept
 *     in envpic_last_error().  No C++ exception crosses this interface.
 *   - Device memory is caller-owned: envpic_sim_init lays the whole state out
 *     inside the arena it is given (size from envpic_footprint) and never
 *     allocates device memory itself.  The handle is host memory owned by the
 *     library until envpic_sim_destroy; the arena stays the caller's.
 *   - A simulation is bound to the HIP stream given at init.  Every non-IO
 *     call is asynchronous on that stream; IO and diagnostics calls are
 *     synchronous.  A simulation is not thread-safe; distinct simulations may
 *     be driven from distinct threads.
 *   - Host-side IO is always FP64.  Grids are exchanged window-relative as
 *     (nx+1) x (nr+1) arrays, row-major [i][j] (radius fastest); a quantity
 *     staggered by half a cell in x (r) at (i, j) sits at x = (i+1/2) dx
 *     (r = (j+1/2) dr) and unused trailing entries are zero.  Complex grids
 *     are interleaved (re, im).  Particles are exchanged as separate arrays
 *     in lab-frame Cartesian coordinates, ordered by id.
 */
#ifndef ENVPIC_H
#define ENVPIC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ENVPIC_PARAMS_VERSION 3

enum envpic_status {
  ENVPIC_OK = 0,
  ENVPIC_EINVAL = -1,   /* bad parameters, unstable time step, bad argument */
  ENVPIC_ENOMEM = -2,   /* arena smaller than the footprint, capacity exceeded */
  ENVPIC_EORDER = -3,   /* a stage called out of sequence */
  ENVPIC_EDEVICE = -4,  /* HIP runtime error (text in envpic_last_error) */
  ENVPIC_ENUMERIC = -5, /* non-finite value or out-of-range particle detected */
};

enum envpic_precision {
  ENVPIC_FP32_BULK = 0, /* FP32 particles and grids, FP64 envelope rows j=0,1 */
  ENVPIC_FP64 = 1,      /* FP64 everywhere */
};

enum envpic_profile {
  ENVPIC_PROFILE_NONE = 0,    /* vacuum */
  ENVPIC_PROFILE_UNIFORM = 1, /* n0 */
  ENVPIC_PROFILE_RAMP = 2,    /* linear 0 -> n0 over lab x in [0, ramp_len], then n0 */
  ENVPIC_PROFILE_PERTURB = 3, /* n0 (1 + perturb (2u - 1)), u uniform per cell */
  ENVPIC_PROFILE_BUMP = 4,    /* n0 (1 + exp(-((x - bump_x)/bump_w)^2)) */
};

/* Plain-old-data parameter block.  `size` must be sizeof(envpic_params) and
 * `version` ENVPIC_PARAMS_VERSION.  tau is the FWHM duration of |A|; the
 * pulse is A = a0 exp(-r^2/(w0^2 q))/q exp(-(x - x_c - t)^2/sigma^2),
 * q = 1 + i (x - x_f)/Z_R, Z_R = w0^2/2, sigma = tau/(2 sqrt(ln 2)). */
typedef struct envpic_params {
  int32_t size, version;
  int32_t nx, nr;          /* cells along x and r (r_max = nr dr) */
  int32_t n_modes;         /* 1: azimuthal mode 0; 2: modes 0 and 1 */
  int32_t ppc_x, ppc_r, ppc_t; /* particles per cell along x, r, theta */
  int32_t profile;         /* enum envpic_profile */
  int32_t moving_window;   /* 1: window moves one cell when (n+1) dt >= (shift+1) dx */
  int32_t tile_x, tile_r;  /* sort tile in cells (0: defaults 16 x 16) */
  uint64_t seed;           /* loading RNG seed (SplitMix64, counter based) */
  double dx, dr, dt;
  double a0, w0, tau, x_c, x_f;
  double n0, ramp_len, perturb, bump_x, bump_w;
  int64_t capacity;        /* particle slots per buffer (0: derived; at most 2^30 - 1) */
  int32_t filter_passes;   /* passes of the 1-2-1 binomial filter on J (0: none, at most
                              ENVPIC_FILTER_MAX, below nx/2 and nr/2); each pass
                              smooths along x, then r */
  int32_t shape_order;     /* particle shape of gather and deposit: 0 or 1 linear
                              (cloud in cell), 2 quadratic B-spline (Sec. 4's
                              nonlinear benchmark configuration); order 2 re-sorts
                              every second step and has no deferred deposits */
  int32_t sort_every;      /* steps between two tile sorts of the particles: 0 for
                              the default (3 linear, 2 quadratic, the most the LDS
                              halo allows), or 1 .. that default */
  int32_t reserved;        /* must be 0 */
} envpic_params;
#define ENVPIC_FILTER_MAX 8

/* grid identifiers for envpic_get_field / envpic_set_field */
enum envpic_field {
  ENVPIC_F_ENV = 0,      /* A^n         complex (i, j)          */
  ENVPIC_F_ENV_PREV = 1, /* A^{n-1}     complex (i, j)          */
  ENVPIC_F_CHI = 2,      /* chi^n       real    (i, j)          */
  ENVPIC_F_EX = 3,       /* E_x^n       real    (i+1/2, j)      */
  ENVPIC_F_ER = 4,       /* E_r^n       real    (i, j+1/2)      */
  ENVPIC_F_BT = 5,       /* B_t^{n+1/2} real    (i+1/2, j+1/2)  */
  ENVPIC_F_BT_BAR = 6,   /* Bbar_t^n    real    (i+1/2, j+1/2)  */
  ENVPIC_F_JX = 7,       /* J_x^{n+1/2} real    (i+1/2, j)      */
  ENVPIC_F_JR = 8,       /* J_r^{n+1/2} real    (i, j+1/2)      */
  ENVPIC_F_EX1 = 9,      /* mode 1, complex: E_x (i+1/2, j)     */
  ENVPIC_F_ER1 = 10,     /* E_r (i, j+1/2)                      */
  ENVPIC_F_ET1 = 11,     /* E_t (i, j)                          */
  ENVPIC_F_BX1 = 12,     /* B_x (i, j+1/2)                      */
  ENVPIC_F_BR1 = 13,     /* B_r (i+1/2, j)                      */
  ENVPIC_F_BT1 = 14,     /* B_t (i+1/2, j+1/2)                  */
  ENVPIC_F_BX1_BAR = 15,
  ENVPIC_F_BR1_BAR = 16,
  ENVPIC_F_BT1_BAR = 17,
  ENVPIC_F_JX1 = 18,
  ENVPIC_F_JR1 = 19,
  ENVPIC_F_JT1 = 20,
  ENVPIC_NFIELDS = 21
};

enum envpic_stage { ENVPIC_MOMENTUM = 0, ENVPIC_POSITION = 1 };
/* OR-ed into the stage of envpic_gather_push: skip the fused deposit and keep
 * what envpic_project_chi_J needs in a scratch area instead. */
#define ENVPIC_DEFER_DEPOSIT 0x100
enum envpic_deposit { ENVPIC_CHI = 1, ENVPIC_J = 2 };

/* diagnostics vector, FP64 reductions on the device */
enum envpic_diag {
  ENVPIC_D_COUNT = 0,     /* live macro-particles */
  ENVPIC_D_CHARGE = 1,    /* sum q w */
  ENVPIC_D_CHI_V = 2,     /* sum over nodes of chi V (chi of the last momentum stage) */
  ENVPIC_D_KIN = 3,       /* sum w (gamma - 1), gamma = sqrt(1 + |p|^2) */
  ENVPIC_D_UEM = 4,       /* low-frequency field energy */
  ENVPIC_D_ENV2_V = 5,    /* sum over nodes |A^n|^2 V */
  ENVPIC_D_LX = 6,        /* sum w (y p_z - z p_y) */
  ENVPIC_D_PX = 7,        /* sum w p_x */
  ENVPIC_D_NONFINITE = 8, /* count of non-finite state values */
  ENVPIC_NDIAG = 9
};

/* injected-beam parameters (envpic_beam_diagnostics), FP64 */
enum envpic_beam {
  ENVPIC_B_PEAK = 0,    /* energy of the spectrum peak, gamma - 1 (m_e c^2) */
  ENVPIC_B_FWHM = 1,    /* full width at half maximum of the peak (m_e c^2) */
  ENVPIC_B_CHARGE = 2,  /* sum q w over the window (q = -1) */
  ENVPIC_B_EMEAN = 3,   /* weighted mean energy over the window */
  ENVPIC_B_ERMS = 4,    /* weighted rms energy spread over the window */
  ENVPIC_B_SPREAD = 5,  /* ERMS / PEAK */
  ENVPIC_B_EMIT_Y = 6,  /* normalized emittance of (y, p_y), c/w0 */
  ENVPIC_B_EMIT_Z = 7,  /* normalized emittance of (z, p_z), c/w0 */
  ENVPIC_B_COUNT = 8,   /* macro-particles in the window */
  ENVPIC_B_QSPEC = 9,   /* sum q w over the whole spectrum range */
  ENVPIC_B_WIN_LO = 10, /* window [WIN_LO, WIN_HI] in energy */
  ENVPIC_B_WIN_HI = 11,
  ENVPIC_NBEAM = 12
};
#define ENVPIC_BEAM_MAX_BINS 4096

typedef struct envpic_sim envpic_sim;

/* Fill `p` with a preset: 0 custom (small vacuum defaults); 1..5 the
 * workloads C1..C5 (C4 gives its 2048 x 256 job shape). */
void envpic_params_default(envpic_params* p, int preset);

/* Validate `p` (sizes, one-cell-per-step CFL dt < dx, dt < dr, envelope and
 * Yee stability on this grid, finite floating-point fields, a non-negative
 * density and capacity) and report the arena bytes a simulation needs at
 * `precision`.  Returns ENVPIC_EINVAL with a message if invalid. */
int envpic_footprint(const envpic_params* p, int precision, size_t* bytes);

/* Lay out and initialise a simulation inside `dev_arena` (device memory of
 * `arena_bytes` >= footprint, 256-byte aligned) on `hip_stream` (a
 * hipStream_t; NULL = default stream): particles x^0 (regular in x, r,
 * one SplitMix64 angle per cell), p^{-1/2} = 0, A^0 and A^{-1} from the
 * paraxial pulse at t = 0 and t = -dt, E^0 = 0, B^{1/2} = 0, and the initial
 * tile sort.  ENVPIC_ENOMEM if the arena is too small. */
int envpic_sim_init(const envpic_params* p, int precision, void* dev_arena, size_t arena_bytes,
                    void* hip_stream, envpic_sim** out);

/* Stage calls of one step, in this order: gather_push(MOMENTUM),
 * envelope_step, gather_push(POSITION), field_step.  ENVPIC_EORDER if called
 * out of sequence.  With ENVPIC_DEFER_DEPOSIT the push leaves the deposit to
 * envpic_project_chi_J (CHI after MOMENTUM, J after POSITION). */
int envpic_gather_push(envpic_sim* s, int stage);
int envpic_envelope_step(envpic_sim* s);
int envpic_project_chi_J(envpic_sim* s, int what);
int envpic_field_step(envpic_sim* s);

/* `nsteps` whole steps with the fused kernels (deposits inside the pushes).
 * ENVPIC_EINVAL for nsteps < 0; ENVPIC_EORDER inside a step. */
int envpic_step_n(envpic_sim* s, int nsteps);

/* Graph mode of envpic_step_n: with steps = k > 0, envpic_step_n captures
 * its kernels from the simulation's stream in chunks of up to k steps, one
 * HIP graph per chunk (each captured, instantiated and launched once: a
 * step's kernel arguments depend on the step), which replaces the per-kernel
 * launches of a chunk by one graph launch; 0 (the default) launches every
 * kernel directly.  Results are those of direct launches.  Ignored while
 * stage timing is on.  ENVPIC_EINVAL for k < 0. */
int envpic_set_graph(envpic_sim* s, int steps);

/* Advance `count` resident simulations by `nsteps` each, interleaving their
 * stages on `hip_stream` so that their kernels overlap on the device.  Each
 * simulation keeps its own state; results equal envpic_step_n's within the
 * rounding of the deposit order.  ENVPIC_EINVAL for count < 0, nsteps < 0,
 * or a NULL or repeated simulation; ENVPIC_EORDER if one is inside a step. */
int envpic_batch_step(envpic_sim* const* sims, int count, int nsteps, void* hip_stream);

/* Synchronous IO (host buffers caller-owned, FP64).  `out`/`in` hold
 * (nx+1)(nr+1) values, twice that for complex grids.  Mode-1 grids need
 * n_modes = 2 (else ENVPIC_EINVAL). */
int envpic_get_field(const envpic_sim* s, int field, double* out);
int envpic_set_field(envpic_sim* s, int field, const double* in);

/* step counter, window shift (cells) and live particle count */
int envpic_state(const envpic_sim* s, int64_t* n, int64_t* shift, int64_t* n_particles);
/* How the particle sorts ran so far (synchronous), out[4]: the sorts that
 * rebuilt the layout ordered by cell (every 8th sort, into the other
 * particle buffer); the tile sorts that moved only the particles that
 * changed tile; the tile sorts whose scan found too few free slots, too
 * little overflow room or too few work items and rebuilt the layout instead
 * (every particle scattered and copied back: correct, slower); the cell
 * sorts whose cell-ordered copy was gathered slot by slot after the momentum
 * pass (chosen once the particles have moved enough that the pass's direct
 * scatter writes partial cache lines; the same result).  The counts start at
 * envpic_sim_init. */
int envpic_sort_stats(const envpic_sim* s, int64_t* out);
/* Particles ordered by id; each pointer may be NULL to skip that array;
 * arrays hold n_particles entries. */
int envpic_get_particles(const envpic_sim* s, double* x, double* y, double* z, double* px,
                         double* py, double* pz, double* w, uint32_t* id);
/* Replace all particles (positions must lie inside the window and below
 * r_max, momenta and weights finite: ENVPIC_EINVAL otherwise; ENVPIC_ENOMEM
 * beyond the capacity); they are tile-sorted on the host before upload. */
int envpic_set_particles(envpic_sim* s, int64_t n, const double* x, const double* y,
                         const double* z, const double* px, const double* py, const double* pz,
                         const double* w, const uint32_t* id);

/* Stage timing: with enable = k > 0, every step whose index is a multiple of
 * k times each stage (momentum; envelope; position = push, deposit,
 * injection; field = [filter,] Maxwell, window, sort scans) with a pair of
 * HIP events that the dispatch of the stage's first kernel stamps at its
 * start and the dispatch of its last kernel stamps at its end
 * (hipExtLaunchKernelGGL), the interval a kernel trace reports, without the
 * gaps between launches (k = 1: every step; a k coprime to the sort periods
 * 3 and 24 samples every variant evenly); enable = 0 turns timing off.
 * envpic_get_timing synchronises and writes the average milliseconds per
 * timed launch into out_ms[4] and the timed launch counts into counts[4]
 * (either may be NULL); every call of envpic_set_timing resets the sums. */
int envpic_set_timing(envpic_sim* s, int enable);
int envpic_get_timing(envpic_sim* s, double* out_ms, int64_t* counts);

/* FP64 device reductions of the current state into out[ENVPIC_NDIAG]. */
int envpic_diagnostics(const envpic_sim* s, double* out);

/* For callers that cannot allocate device memory, nor synchronise: code under
 * HIP graph capture, tight serving loops, harnesses that forbid allocation.
 * The same sums as envpic_diagnostics, from the same kernels, written to
 * dev_out[ENVPIC_NDIAG] (caller-owned device memory, FP64) asynchronously on
 * the simulation's stream.  The partial sums live in a scratch array of the
 * library's own (1024 x 11 doubles, 88 KiB per GPU, kept until the process
 * ends), not in the arena; its size does not depend on the simulation, so no
 * simulation is too large for it.  The call allocates nothing, copies
 * nothing to the host and does not read the error word (envpic_diagnostics
 * does).  Calls on one GPU share that scratch: two of them that overlap in
 * time (different streams) race, so order them.  ENVPIC_EORDER in the middle
 * of a step; ENVPIC_EDEVICE if the scratch could not be located on the
 * simulation's GPU at init. */
int envpic_diagnostics_noalloc(const envpic_sim* s, double* dev_out);

/* Injected-beam parameters of the current particles (Sec. 4, Table
 * BeamParams: spectrum peak energy, beam charge, relative energy spread and
 * normalized transverse emittance sqrt(s_uu s_pp - s_up^2), all over the
 * particles within two FWHM widths in energy around the spectrum peak),
 * as FP64 device reductions into out[ENVPIC_NBEAM].
 *   energy     gamma - 1 with gamma = sqrt(1 + |p|^2);
 *   spectrum   charge histogram sum |q| w over `nbins` equal bins of
 *              [e_lo, e_hi) (e_lo leaves out the bulk plasma), copied to
 *              `hist` (nbins doubles, caller-owned; NULL to skip);
 *   peak       centre of the fullest bin (the lowest on a tie);
 *   FWHM       half-maximum crossings interpolated between bin centres, the
 *              range edge where a side stays above half maximum;
 *   window     [peak - FWHM, peak + FWHM] within [e_lo, e_hi);
 *   moments    weighted by w and centred; y = r cos(theta), z = r sin(theta).
 * An empty spectrum gives all zeros.  Synchronous; only between steps
 * (ENVPIC_EORDER otherwise).  ENVPIC_EINVAL unless e_lo < e_hi (finite)
 * and 1 <= nbins <= ENVPIC_BEAM_MAX_BINS. */
int envpic_beam_diagnostics(const envpic_sim* s, double e_lo, double e_hi, int nbins, double* out,
                            double* hist);

/* Self-consistent initial fields of an externally injected relativistic
 * electron bunch (Sec. 3: the field initialisation of external injection,
 * carried over to cylindrical symmetry).  The bunch is the set of resident
 * particles with id in [id_lo, id_hi) (load it with envpic_set_particles);
 * it moves along x with velocity beta.  Its potential solves
 *   (1/gamma^2) d2phi/dx2 + (1/r) d/dr (r dphi/dr) = -rho
 * on the primal nodes, with phi = 0 on the x ends and at r_max and rho the
 * bunch's charge deposited with the simulation's particle shape, so that
 * the Gauss law of the field update holds exactly; then
 *   E_x(i+1/2, j) = -(phi_{i+1,j} - phi_{i,j}) / (gamma^2 dx),
 *   E_r(i, j+1/2) = -(phi_{i,j+1} - phi_{i,j}) / dr,
 *   B_theta = Bbar_theta = beta (E_r(i) + E_r(i+1)) / 2 at (i+1/2, j+1/2)
 * are ADDED to the mode-0 E^n, B^{n+1/2} and Bbar^n (mode 1 untouched: an
 * axisymmetric bunch).  FP64 conjugate gradients (diagonal preconditioner)
 * until the relative residual |b - K phi| / |b| is at most tol, in at most
 * max_iter iterations; *iters and *resid (each may be NULL) receive the
 * iterations and the final relative residual.  A range holding no charge
 * changes nothing.  Synchronous; only between steps (ENVPIC_EORDER).
 * ENVPIC_EINVAL unless 0 <= beta < 1, tol > 0, max_iter >= 1 and
 * id_hi > id_lo; ENVPIC_ENUMERIC if tol is not reached (the fields are
 * added all the same). */
int envpic_bunch_fields(envpic_sim* s, uint32_t id_lo, uint32_t id_hi, double beta, double tol, int max_iter,
                        int* iters, double* resid);

/* Checkpoint: with host_blob == NULL, *bytes receives the size needed; else
 * the full state (step, shift, both envelope levels, E, B, Bbar, particles,
 * parameters) is written.  envpic_load restores a blob written by a
 * simulation with the same parameters and precision (ENVPIC_EINVAL for any
 * other blob, a truncated one or one whose counts are out of range). */
int envpic_save(const envpic_sim* s, void* host_blob, size_t* bytes);
int envpic_load(envpic_sim* s, const void* host_blob, size_t bytes);

/* Debug hook: write a NaN into one node of a grid (tests of failure
 * detection through the diagnostics). */
int envpic_debug_poison(envpic_sim* s, int field);

/* Frees the handle.  It first waits for every kernel the simulation has
 * queued on its stream, so the caller may release or reuse the arena as soon
 * as this returns.  NULL is ignored. */
void envpic_sim_destroy(envpic_sim* s);

/* A plain streaming device-to-device copy of `bytes` bytes (a multiple of 16;
 * both pointers 16-byte aligned, caller-owned device memory, not
 * overlapping), asynchronous on `stream`: the bandwidth reference the
 * kernels' HBM rates are compared with.  variant: 0 and 1 ordinary loads and
 * stores with 4 or 8 16-byte accesses in flight per lane, 2 and 3 the same
 * with non-temporal loads and stores.  ENVPIC_EINVAL on a bad size,
 * alignment or variant; ENVPIC_EDEVICE if the launch fails. */
int envpic_stream_copy(void* dst, const void* src, size_t bytes, int variant, void* stream);

/* Message of the last error on this thread (s may be NULL). */
const char* envpic_last_error(const envpic_sim* s);

#ifdef __cplusplus
}
#endif
#endif
