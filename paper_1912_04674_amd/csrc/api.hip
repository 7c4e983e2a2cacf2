// api.hip -- host implementation of the envpic C ABI (include/envpic.h).
//
// The library never allocates device memory: every array lives in the
// caller's arena, carved by `plan()` below.  Kernel launches are
// asynchronous on the simulation's stream; IO and diagnostics synchronise.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/envpic.h"
#include "common.hpp"
#include "launch.hpp"

using namespace envpic;

namespace {

thread_local std::string g_last_error;

int fail(int code, const std::string& msg) {
  g_last_error = msg;
  return code;
}

int hip_check(hipError_t e, const char* what) {
  if (e == hipSuccess) return ENVPIC_OK;
  return fail(ENVPIC_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

inline size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// ------------------------------------------------------------ geometry --
struct Sizes {
  int nxa, pitch, ntxa, ntr, ntiles, ppc, max_items, chunk;
  long long capacity;
  size_t ngrid;  // elements per grid
};

Sizes sizes_of(const envpic_params& p) {
  Sizes s;
  s.ntxa = (p.nx + 2 + TX - 1) / TX + 3;
  s.nxa = s.ntxa * TX;
  s.pitch = (int)align_up((size_t)p.nr + 1, 16);
  s.ntr = (p.nr + TR - 1) / TR;
  s.ntiles = s.ntxa * s.ntr;
  s.ppc = p.ppc_x * p.ppc_r * p.ppc_t;
  const long long window = (long long)p.nx * p.nr * s.ppc;
  // one window of particles, overflow ranges for particles that change
  // tile (1/4 of them: an incremental sort moves the earlier overflow again
  // with the new arrivals, so the ranges grow over the tile sorts between
  // two cell sorts; with 1/16 the late LWFA wake ran out of them and rebuilt
  // the layout about once per cell-sort cycle), room for the tiles about to
  // enter a moving window, and the columns injected until the layout is
  // rebuilt
  const long long column = (long long)p.nr * s.ppc;
  s.capacity = p.capacity > 0 ? p.capacity
                              : window + window / 4 + (long long)(ENTERING_TILES + 1) * TX * column +
                                    (SORT_EVERY * (CELL_SORT_EVERY + 1LL) + 1) * column + 1024;
  // work-item size: about four items per compute unit (256 of them) so that
  // small runs fill the device, at most CHUNK (CHUNK / 2 with quadratic
  // shapes, whose particles cost more than the staging and flush of an
  // item: measured faster on the LWFA workload, and CHUNK / 4 slower), a
  // multiple of WG
  const long long per = window / (4LL * 256);
  const long long cmax = p.shape_order == 2 ? CHUNK / 2 : CHUNK;
  s.chunk = (int)std::max<long long>(WG, std::min<long long>(cmax, per / WG * WG));
  // items: those of any layout of the tiles' particles, and those of the
  // columns injected between two sorts (a tile sort whose overflow would
  // need more rebuilds the layout instead)
  s.max_items = (int)(s.ntiles + s.capacity / s.chunk + SORT_EVERY * s.ntr + 16);
  s.ngrid = (size_t)s.nxa * s.pitch;
  return s;
}

// slots a rebuilt layout keeps free past the tiles' segments: the columns
// injected until it is rebuilt again (at most one per step)
long long slot_reserve(const envpic_params& p, const Sizes& s) {
  return SORT_EVERY * (CELL_SORT_EVERY + 1LL) * p.nr * s.ppc;
}

int validate(const envpic_params* p) {
  if (!p) return fail(ENVPIC_EINVAL, "params is NULL");
  if (p->size != (int32_t)sizeof(envpic_params) || p->version != ENVPIC_PARAMS_VERSION)
    return fail(ENVPIC_EINVAL, "params size/version mismatch");
  if (p->nx < 4 || p->nr < 2) return fail(ENVPIC_EINVAL, "grid needs nx >= 4 and nr >= 2");
  if (p->nr > NR_MAX) return fail(ENVPIC_EINVAL, "nr exceeds the 12-bit radial cell index");
  if (p->nx > COL_MAX / 2) return fail(ENVPIC_EINVAL, "nx exceeds the 20-bit lab column index");
  if (p->n_modes < 1 || p->n_modes > 2) return fail(ENVPIC_EINVAL, "n_modes must be 1 or 2");
  if (p->ppc_x < 1 || p->ppc_r < 1 || p->ppc_t < 1 || p->ppc_x * p->ppc_r * p->ppc_t > 256)
    return fail(ENVPIC_EINVAL, "particles per cell must be in [1, 256]");
  if ((p->tile_x != 0 && p->tile_x != TX) || (p->tile_r != 0 && p->tile_r != TR))
    return fail(ENVPIC_EINVAL, "tile shape must be 16 x 16 (or 0 for the default)");
  for (const double v : {p->dx, p->dr, p->dt, p->a0, p->w0, p->tau, p->x_c, p->x_f, p->n0, p->ramp_len, p->perturb,
                         p->bump_x, p->bump_w})
    if (!std::isfinite(v)) return fail(ENVPIC_EINVAL, "every floating-point parameter must be finite");
  if (p->capacity < 0) return fail(ENVPIC_EINVAL, "capacity must be >= 0 (0: derived)");
  if (!(p->dx > 0 && p->dr > 0 && p->dt > 0)) return fail(ENVPIC_EINVAL, "dx, dr, dt must be positive");
  if (!(p->dt < p->dx && p->dt < p->dr))
    return fail(ENVPIC_EINVAL, "dt must be below dx and dr (particles move at most one cell per step)");
  // Stability: both the envelope scheme and the cylindrical Yee scheme are
  // about 2 % stricter than the Cartesian bound 1/sqrt(1/dx^2 + 1/dr^2) once
  // the axis rows are included; 0.97 of that bound keeps a margin.
  const double cart = 1.0 / std::sqrt(1.0 / (p->dx * p->dx) + 1.0 / (p->dr * p->dr));
  if (p->dt > 0.97 * cart) {
    char buf[160];
    std::snprintf(buf, sizeof buf, "dt = %g exceeds the stability limit ~%.4f for dx = %g, dr = %g", p->dt,
                  0.97 * cart, p->dx, p->dr);
    return fail(ENVPIC_EINVAL, buf);
  }
  if (p->profile < 0 || p->profile > 4) return fail(ENVPIC_EINVAL, "unknown plasma profile");
  if (p->filter_passes < 0 || p->filter_passes > ENVPIC_FILTER_MAX)
    return fail(ENVPIC_EINVAL, "filter_passes must be in [0, ENVPIC_FILTER_MAX]");
  if (p->filter_passes > 0 && (p->nx <= 2 * p->filter_passes || p->nr <= 2 * p->filter_passes))
    return fail(ENVPIC_EINVAL, "the binomial filter needs nx and nr above twice its passes");
  if (p->shape_order < 0 || p->shape_order > 2) return fail(ENVPIC_EINVAL, "shape_order must be 0, 1 (linear) or 2 (quadratic)");
  if (p->sort_every < 0 || p->sort_every > (p->shape_order == 2 ? SORT_EVERY - 1 : SORT_EVERY))
    return fail(ENVPIC_EINVAL, "sort_every must be 0 (default) or between 1 and 3 (2 for quadratic shapes)");
  if (p->reserved != 0) return fail(ENVPIC_EINVAL, "reserved must be 0");
  if (p->n0 < 0) return fail(ENVPIC_EINVAL, "n0 must be >= 0");
  if (p->profile == ENVPIC_PROFILE_RAMP && !(p->ramp_len > 0)) return fail(ENVPIC_EINVAL, "ramp_len must be > 0");
  if (p->profile == ENVPIC_PROFILE_BUMP && !(p->bump_w > 0)) return fail(ENVPIC_EINVAL, "bump_w must be > 0");
  if (p->profile == ENVPIC_PROFILE_PERTURB && !(p->perturb >= 0 && p->perturb <= 1))
    return fail(ENVPIC_EINVAL, "perturb must be in [0, 1] (a non-negative density)");
  if (p->a0 < 0 || (p->a0 > 0 && !(p->w0 > 0 && p->tau > 0))) return fail(ENVPIC_EINVAL, "bad laser parameters");
  const Sizes s = sizes_of(*p);
  // slots < 2^30: the particle passes form 4-byte records' byte offsets in 32 bits
  if (s.capacity >= (1LL << 30)) return fail(ENVPIC_EINVAL, "too many particles: at most 2^30 - 1 slots");
  if (s.capacity < (long long)p->nx * p->nr * s.ppc + (long long)SORT_EVERY * p->nr * s.ppc)
    return fail(ENVPIC_EINVAL, "capacity below one window of particles plus the columns injected between sorts");
  return ENVPIC_OK;
}

// -------------------------------------------------------- arena layout --
struct Carver {
  char* base;
  size_t off = 0;
  template <class T> T* take(size_t count) {
    off = align_up(off, 256);
    T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
    off += count * sizeof(T);
    return p;
  }
};

template <class R> struct State {
  using C = typename cplx_of<R>::type;
  Parts<R> parts[2], scr;
  Grids<R> grids;
  DepositBufs<R> dep[2];
  DepositBufs<R> jf;  // filtered currents (chi unused) when the binomial filter is on
  Layout lay[2];
  int* hist;    // particles per tile at the next sort
  int* arr;     // particles arriving from other tiles at the next (tile) sort
  int* sort_stats;  // [incremental, rebuilt] layouts of the tile sorts, gathered cell sorts
  int* ccount;  // particles per cell at the next sort ([phys col][row], as the grids)
  int* ccur;    // per-cell scatter cursors of the next sort
  int* err;
  int* pending;  // [items, slots] appended by the last injection, not yet counted
  double* diag_scratch;
  double* diag_out;
  BeamScratch beam;
  CgVecs cg;
};

template <class R> size_t plan(const envpic_params& p, const Sizes& s, bool fp64_rows, char* base, State<R>* st) {
  using C = typename cplx_of<R>::type;
  Carver cv{base};
  State<R> S{};
  const size_t cap = (size_t)s.capacity;
  for (int b = 0; b < 2; ++b) {
    Parts<R>& P = S.parts[b];
    P.cell = cv.take<unsigned>(cap);
    P.fx = cv.take<R>(cap);
    P.fr = cv.take<R>(cap);
    P.th = cv.take<R>(cap);
    P.px = cv.take<R>(cap);
    P.py = cv.take<R>(cap);
    P.pz = cv.take<R>(cap);
    P.w = cv.take<R>(cap);
    P.id = cv.take<uint32_t>(cap);
  }
  S.scr.cell = cv.take<unsigned>(cap);
  S.scr.fx = cv.take<R>(cap);
  S.scr.fr = cv.take<R>(cap);
  S.scr.th = cv.take<R>(cap);
  S.scr.w = cv.take<R>(cap);
  const size_t ng = s.ngrid;
  Grids<R>& f = S.grids;
  f.ex = cv.take<R>(ng);
  f.er = cv.take<R>(ng);
  f.bt = cv.take<R>(ng);
  f.btb = cv.take<R>(ng);
  f.env = cv.take<C>(ng);
  f.envp = cv.take<C>(ng);
  f.ax = fp64_rows ? cv.take<double2>((size_t)s.nxa * 2) : nullptr;
  f.axp = fp64_rows ? cv.take<double2>((size_t)s.nxa * 2) : nullptr;
  const bool m1 = p.n_modes >= 2;
  const size_t n1 = m1 ? ng : 0;
  f.ex1 = cv.take<C>(n1);
  f.er1 = cv.take<C>(n1);
  f.et1 = cv.take<C>(n1);
  f.bx1 = cv.take<C>(n1);
  f.br1 = cv.take<C>(n1);
  f.bt1 = cv.take<C>(n1);
  f.bxb1 = cv.take<C>(n1);
  f.brb1 = cv.take<C>(n1);
  f.btb1 = cv.take<C>(n1);
  f.ex_n = cv.take<R>(ng);
  f.er_n = cv.take<R>(ng);
  f.bt_n = cv.take<R>(ng);
  f.ex1_n = cv.take<C>(n1);
  f.er1_n = cv.take<C>(n1);
  f.et1_n = cv.take<C>(n1);
  f.bx1_n = cv.take<C>(n1);
  f.br1_n = cv.take<C>(n1);
  f.bt1_n = cv.take<C>(n1);
  for (int b = 0; b < 2; ++b) {
    DepositBufs<R>& d = S.dep[b];
    d.chi = cv.take<R>(ng);
    d.jx = cv.take<R>(ng);
    d.jr = cv.take<R>(ng);
    d.jx1 = cv.take<C>(n1);
    d.jr1 = cv.take<C>(n1);
    d.jt1 = cv.take<C>(n1);
  }
  {
    const bool filt = p.filter_passes > 0;
    DepositBufs<R>& d = S.jf;
    d.chi = nullptr;
    d.jx = cv.take<R>(filt ? ng : 0);
    d.jr = cv.take<R>(filt ? ng : 0);
    d.jx1 = cv.take<C>(filt ? n1 : 0);
    d.jr1 = cv.take<C>(filt ? n1 : 0);
    d.jt1 = cv.take<C>(filt ? n1 : 0);
  }
  f.chi = nullptr;
  f.jx = nullptr;
  f.jr = nullptr;
  f.jx1 = f.jr1 = f.jt1 = nullptr;
  for (int b = 0; b < 2; ++b) {
    Layout& L = S.lay[b];
    L.offsets = cv.take<int>((size_t)s.ntiles + 1);
    L.ext = cv.take<int>((size_t)s.ntiles);
    L.cursor = cv.take<int>((size_t)s.ntiles);
    L.ovb = cv.take<int>((size_t)s.ntiles);
    L.ovn = cv.take<int>((size_t)s.ntiles);
    L.items = cv.take<int4>((size_t)s.max_items);
    L.n_items = cv.take<int>(1);
    L.fill = cv.take<int>(1);
    L.mode = cv.take<int>(1);
  }
  S.hist = cv.take<int>((size_t)s.ntiles);
  S.arr = cv.take<int>((size_t)s.ntiles);
  S.sort_stats = cv.take<int>(3);
  S.ccount = cv.take<int>(ng);
  S.ccur = cv.take<int>(ng);
  S.err = cv.take<int>(1);
  S.pending = cv.take<int>(2);
  S.diag_scratch = cv.take<double>((size_t)diag_scratch_doubles());
  S.diag_out = cv.take<double>(ENVPIC_NDIAG);
  S.beam.hist = cv.take<unsigned long long>(BEAM_MAX_BINS);
  S.beam.hist_f = cv.take<double>(BEAM_MAX_BINS);
  S.beam.part = cv.take<double>((size_t)s.max_items * BEAM_PARTS);
  S.beam.st = cv.take<double>(BEAM_STATE);
  S.beam.out = cv.take<double>(ENVPIC_NBEAM);
  {
    const size_t nu = (size_t)cg_unknowns(p.nx, p.nr);
    S.cg.x = cv.take<double>(nu);
    S.cg.r = cv.take<double>(nu);
    S.cg.p = cv.take<double>(nu);
    S.cg.p2 = cv.take<double>(nu);
    S.cg.q = cv.take<double>(nu);
    S.cg.idiag = cv.take<double>((size_t)p.nr);
    S.cg.part = cv.take<double>((size_t)cg_blocks(p.nx, p.nr) * 2);
    S.cg.s = cv.take<double>(CG_NS);
  }
  if (st) *st = S;
  return align_up(cv.off, 256);
}

size_t footprint_bytes(const envpic_params& p, int prec) {
  const Sizes s = sizes_of(p);
  if (prec == ENVPIC_FP64) return plan<double>(p, s, false, nullptr, nullptr);
  return plan<float>(p, s, true, nullptr, nullptr);
}

}  // namespace

// ================================================================ sim ==
struct envpic_sim {
  envpic_params p;
  int prec;
  hipStream_t stream;
  int device = -1;                  // the GPU current at init (the stream's)
  double* diag_static = nullptr;    // that GPU's static diagnostics scratch
  size_t diag_static_doubles = 0;
  Sizes sz;
  int64_t n = 0, shift = 0;
  int stage = 0;     // next expected stage: 0 momentum, 1 envelope, 2 position, 3 field
  int cur = 0;       // particle buffer holding the current state
  int lay = 0;       // its layout (a tile sort changes the layout, not the buffer)
  int64_t sorted_at = 0;  // step whose positions the layout of P[cur] is sorted by
  int64_t n_sorts = 0;    // sorts so far (selects tile or cell order)
  int64_t n_cell_sorts = 0;
  bool settle_due = false;  // the envelope stage carries the copy back of this step's tile sort
  bool deferred = false, deposit_done = true;
  int chi_last = 0;  // deposit buffer of the last momentum stage
  bool jf_valid = false;  // the filtered copy holds the current of the last field stage
  // stage timing (events on the simulation's stream)
  struct Tick {
    int stage;
    hipEvent_t a, b;
  };
  int timing = 0;  // record the stage events on every timing-th step (0: off)
  std::vector<hipEvent_t> ev_pool;
  std::vector<Tick> ticks;
  double t_ms[4] = {0, 0, 0, 0};
  int64_t t_n[4] = {0, 0, 0, 0};

  hipEvent_t take_event() {
    if (!ev_pool.empty()) {
      hipEvent_t e = ev_pool.back();
      ev_pool.pop_back();
      return e;
    }
    // timing only: no system-scope fence (no cache writeback and
    // invalidation between the stages being timed)
    hipEvent_t e = nullptr;
    if (hipEventCreateWithFlags(&e, hipEventDisableSystemFence) != hipSuccess) return nullptr;
    return e;
  }
  // the stage's start and stop events on every timing-th step (none
  // otherwise): the launchers hand them to the stage's first and last
  // kernel, whose dispatch stamps them
  KEvents tick_events() {
    if (timing <= 0 || n % timing != 0) return KEvents{};
    hipEvent_t a = take_event(), b = a ? take_event() : nullptr;
    if (!a || !b) {
      if (a) ev_pool.push_back(a);
      return KEvents{};
    }
    return KEvents{a, b};
  }
  void tick_end(int stage, const KEvents& ev) {
    if (!ev.start) return;
    ticks.push_back(Tick{stage, ev.start, ev.stop});
    if (ticks.size() >= 4096) resolve_ticks();
  }
  int resolve_ticks() {
    if (ticks.empty()) return ENVPIC_OK;
    if (hipEventSynchronize(ticks.back().b) != hipSuccess) return ENVPIC_EDEVICE;
    for (const Tick& t : ticks) {
      float ms = 0.0f;
      if (hipEventElapsedTime(&ms, t.a, t.b) == hipSuccess) {
        t_ms[t.stage] += ms;
        t_n[t.stage] += 1;
      }
      ev_pool.push_back(t.a);
      ev_pool.push_back(t.b);
    }
    ticks.clear();
    return ENVPIC_OK;
  }
  // graph mode: envpic_step_n records chunks of graph_steps steps into one
  // HIP graph each and launches it on the simulation's stream; an executable
  // graph is destroyed once the event recorded after its launch has
  // completed.  The kernels are recorded from a private stream (the
  // simulation's stream may be the null stream, which cannot be captured).
  int graph_steps = 0;
  std::vector<std::pair<hipGraphExec_t, hipEvent_t>> graphs;
  hipStream_t cap_stream = nullptr;

  void reap_graphs(bool wait) {
    for (size_t k = 0; k < graphs.size();) {
      if (wait) (void)hipEventSynchronize(graphs[k].second);
      if (wait || hipEventQuery(graphs[k].second) == hipSuccess) {
        (void)hipGraphExecDestroy(graphs[k].first);
        (void)hipEventDestroy(graphs[k].second);
        graphs.erase(graphs.begin() + (long)k);
      } else {
        ++k;
      }
    }
  }
  int step_graph(int k) {
    reap_graphs(false);
    int rc = ENVPIC_OK;
    if (!cap_stream && (rc = hip_check(hipStreamCreateWithFlags(&cap_stream, hipStreamNonBlocking), "capture stream")))
      return rc;
    if ((rc = hip_check(hipStreamBeginCapture(cap_stream, hipStreamCaptureModeThreadLocal), "begin capture"))) return rc;
    hipStream_t own = stream;
    stream = cap_stream;  // the stages issue their kernels on `stream`
    for (int i = 0; i < k && !rc; ++i) rc = step();
    stream = own;
    hipGraph_t graph = nullptr;
    const hipError_t ec = hipStreamEndCapture(cap_stream, &graph);
    if (rc || ec != hipSuccess) {
      if (graph) (void)hipGraphDestroy(graph);
      return rc ? rc : hip_check(ec, "end capture");
    }
    hipGraphExec_t exec = nullptr;
    rc = hip_check(hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0), "graph instantiate");
    (void)hipGraphDestroy(graph);
    if (rc) return rc;
    hipEvent_t done = nullptr;
    if ((rc = hip_check(hipGraphLaunch(exec, stream), "graph launch")) ||
        (rc = hip_check(hipEventCreateWithFlags(&done, hipEventDisableTiming), "graph event")) ||
        (rc = hip_check(hipEventRecord(done, stream), "graph event record"))) {
      (void)hipStreamSynchronize(stream);
      (void)hipGraphExecDestroy(exec);
      if (done) (void)hipEventDestroy(done);
      return rc;
    }
    graphs.emplace_back(exec, done);
    return ENVPIC_OK;
  }

  virtual ~envpic_sim() {
    reap_graphs(true);
    if (cap_stream) (void)hipStreamDestroy(cap_stream);
    if (!ticks.empty()) (void)hipEventSynchronize(ticks.back().b);
    for (const Tick& t : ticks) {
      (void)hipEventDestroy(t.a);
      (void)hipEventDestroy(t.b);
    }
    for (hipEvent_t e : ev_pool) (void)hipEventDestroy(e);
  }
  virtual int init() = 0;
  virtual int momentum(bool defer) = 0;
  virtual int project(int what) = 0;
  virtual int envelope() = 0;
  virtual int position(bool defer) = 0;
  virtual int field() = 0;
  virtual int get_field(int f, double* out) = 0;
  virtual int set_field(int f, const double* in) = 0;
  virtual int get_particles(std::vector<double>* cols, std::vector<uint32_t>* ids) = 0;
  virtual int set_particles(int64_t n, const double* const* cols, const uint32_t* id) = 0;
  virtual int diagnostics(double* out) = 0;
  virtual int diagnostics_noalloc(double* dev_out) = 0;
  virtual int beam(double e_lo, double e_hi, int nbins, double* out, double* hist) = 0;
  virtual int bunch(uint32_t id_lo, uint32_t id_hi, double beta, double tol, int max_iter, int* iters,
                    double* resid) = 0;
  virtual int poison(int f) = 0;
  virtual int check_err() = 0;
  virtual int clear_deposits() = 0;
  virtual int sort_counts(int64_t* incremental, int64_t* rebuilt, int64_t* gathered) = 0;

  // the momentum stage of the next step re-sorts the particles
  // Steps between sorts: particles drift at most one cell per step, and the
  // LDS halo holds SORT_EVERY cells of drift plus the linear stencil, or
  // SORT_EVERY - 1 cells plus the wider quadratic one.
  int sort_every() const {
    const int most = p.shape_order == 2 ? SORT_EVERY - 1 : SORT_EVERY;
    return p.sort_every > 0 && p.sort_every < most ? p.sort_every : most;
  }
  bool presort() const { return n + 1 - sorted_at >= sort_every(); }
  // the kind of sort at the momentum stage of the next step (0: none);
  // every CELL_SORT_EVERY-th sort orders the tiles by cell again
  int next_sort() const {
    if (!presort()) return 0;
    return n_sorts % CELL_SORT_EVERY == 0 ? SCAT_CELL : SCAT_TILE;
  }
  bool shift_due() const {
    return p.moving_window && (double)(n + 1) * p.dt >= (double)(shift + 1) * p.dx;
  }
  int step() {
    int rc;
    if ((rc = momentum(false))) return rc;
    if ((rc = envelope())) return rc;
    if ((rc = position(false))) return rc;
    return field();
  }
};

namespace {

template <class R> struct SimT : envpic_sim {
  using C = typename cplx_of<R>::type;
  State<R> S;
  bool fp64_rows;
  char* arena;
  double wmax = 0.0;  // bound of |w| over every particle loaded, injected or set

  // largest weight the loading rule gives: n_max 2 pi r (dr/ppc_r)(dx/ppc_x)/ppc_t at r <= r_max
  double loading_weight_bound() const {
    double nmax = 0.0;
    switch (p.profile) {
      case ENVPIC_PROFILE_UNIFORM:
      case ENVPIC_PROFILE_RAMP: nmax = std::fabs(p.n0); break;
      case ENVPIC_PROFILE_PERTURB: nmax = std::fabs(p.n0) * (1.0 + std::fabs(p.perturb)); break;
      case ENVPIC_PROFILE_BUMP: nmax = 2.0 * std::fabs(p.n0); break;
      default: nmax = 0.0;
    }
    const double pi = 3.14159265358979323846;
    return nmax * 2.0 * pi * (p.nr * p.dr) * (p.dr / p.ppc_r) * (p.dx / p.ppc_x) / p.ppc_t;
  }

  Geo geo() const { return geo_at(shift); }
  // the geometry with the window's left edge at lab column sh
  Geo geo_at(int64_t sh) const {
    Geo g{};
    g.nx = p.nx;
    g.nr = p.nr;
    g.nxa = sz.nxa;
    g.pitch = sz.pitch;
    g.ntxa = sz.ntxa;
    g.ntr = sz.ntr;
    g.ntiles = sz.ntiles;
    g.modes = p.n_modes;
    g.ppc_x = p.ppc_x;
    g.ppc_r = p.ppc_r;
    g.ppc_t = p.ppc_t;
    g.shift = sh;
    g.cap = sz.capacity;
    g.base = (int)(sh % sz.nxa);
    const long long c = sh - 2;
    g.t_lo = (int)(c >= 0 ? c / TX : -((-c + TX - 1) / TX));
    g.dx = p.dx;
    g.dr = p.dr;
    g.dt = p.dt;
    g.chunk = sz.chunk;
    g.order = p.shape_order == 2 ? 2 : 1;
    // one buffer's records: cell word and id, six reals and the weight
    g.stream_parts = sz.capacity * (long long)(8 + 7 * sizeof(R)) >= STREAM_PARTS_BYTES ? 1 : 0;
    // fixed-point scale of the mode-1 current sums: 2^32 over the largest
    // |2 q w v S / V| = 2 w_max / V_0, V_0 = pi dr^2 dx / 4
    const double cmax = 2.0 * wmax * 4.0 / (3.14159265358979323846 * p.dr * p.dr * p.dx);
    const double fix = cmax > 0.0 ? std::min(std::max(std::ldexp(1.0, 32) / cmax, std::ldexp(1.0, -100)), std::ldexp(1.0, 100)) : 1.0;
    g.fix = (float)fix;
    g.unfix = 1.0 / (double)g.fix;
    // the chi and mode-0 current sums: 2^32 over the largest |w S| = w_max
    const double fix0 = wmax > 0.0 ? std::min(std::max(std::ldexp(1.0, 32) / wmax, std::ldexp(1.0, -100)), std::ldexp(1.0, 100)) : 1.0;
    g.fix0 = (float)fix0;
    g.unfix0 = 1.0 / (double)g.fix0;
    return g;
  }
  Plasma plasma() const {
    Plasma pl;
    pl.profile = p.profile;
    pl.n0 = p.n0;
    pl.ramp_len = p.ramp_len;
    pl.perturb = p.perturb;
    pl.bump_x = p.bump_x;
    pl.bump_w = p.bump_w;
    pl.seed = p.seed;
    return pl;
  }
  Laser laser() const {
    Laser L;
    L.a0 = p.a0;
    L.w0 = p.w0;
    L.tau = p.tau;
    L.x_c = p.x_c;
    L.x_f = p.x_f;
    return L;
  }
  int launched(const char* what) { return hip_check(hipGetLastError(), what); }

  // host-built layout of a particle set sorted by tile key: offsets per key
  // and work items of <= chunk particles
  int upload_layout(int b, const std::vector<int>& counts) {
    std::vector<int> off(sz.ntiles + 1, 0);
    std::vector<int4> items;
    for (int t = 0; t < sz.ntiles; ++t) {
      off[t + 1] = off[t] + counts[t];
      const int nm = (counts[t] + sz.chunk - 1) / sz.chunk;  // equal shares, as in the device scan
      for (int k = 0; k < nm; ++k) {
        const int lo = (int)((long long)k * counts[t] / nm), hi = (int)((long long)(k + 1) * counts[t] / nm);
        items.push_back(make_int4(t, off[t] + lo, hi - lo, 0));
      }
    }
    if ((int)items.size() > sz.max_items - sz.ntr) return fail(ENVPIC_ENOMEM, "work-item list overflow");
    const int ni = (int)items.size();
    int rc;
    if ((rc = hip_check(hipMemcpyAsync(S.lay[b].offsets, off.data(), off.size() * sizeof(int), hipMemcpyHostToDevice, stream), "upload offsets"))) return rc;
    if ((rc = hip_check(hipMemcpyAsync(S.lay[b].cursor, off.data(), (size_t)sz.ntiles * sizeof(int), hipMemcpyHostToDevice, stream), "upload cursor"))) return rc;
    if ((rc = hip_check(hipMemcpyAsync(S.lay[b].ext, counts.data(), (size_t)sz.ntiles * sizeof(int), hipMemcpyHostToDevice, stream), "upload extents"))) return rc;
    // the particles per tile, which the kernels keep current (exact for a
    // particle upload; the first sort after loading is a cell sort, which
    // counts them afresh)
    if ((rc = hip_check(hipMemcpyAsync(S.hist, counts.data(), (size_t)sz.ntiles * sizeof(int), hipMemcpyHostToDevice, stream), "upload tile counts"))) return rc;
    const int full = LAYOUT_FULL;
    if ((rc = hip_check(hipMemcpyAsync(S.lay[b].mode, &full, sizeof(int), hipMemcpyHostToDevice, stream), "upload mode"))) return rc;
    if (ni && (rc = hip_check(hipMemcpyAsync(S.lay[b].items, items.data(), items.size() * sizeof(int4), hipMemcpyHostToDevice, stream), "upload items"))) return rc;
    if ((rc = hip_check(hipMemcpyAsync(S.lay[b].n_items, &ni, sizeof(int), hipMemcpyHostToDevice, stream), "upload n_items"))) return rc;
    if ((rc = hip_check(hipMemcpyAsync(S.lay[b].fill, &off[sz.ntiles], sizeof(int), hipMemcpyHostToDevice, stream), "upload fill"))) return rc;
    return hip_check(hipStreamSynchronize(stream), "layout upload");
  }



  int init() override {
    int rc;
    wmax = loading_weight_bound();
    if ((rc = hip_check(hipMemsetAsync(arena, 0, footprint_bytes(p, prec), stream), "arena clear"))) return rc;
    const Geo g = geo();
    // initial layout: window cells in tile-major order, ppc slots per cell
    std::vector<int> counts(sz.ntiles, 0);
    if (p.profile != ENVPIC_PROFILE_NONE)
      for (int T = 0; T * TX < p.nx; ++T)
        for (int tr = 0; tr < sz.ntr; ++tr) {
          const int cols = std::min(TX, p.nx - T * TX), rows = std::min(TR, p.nr - tr * TR);
          counts[(T % sz.ntxa) * sz.ntr + tr] = cols * rows * sz.ppc;
        }
    lay = cur;
    if ((rc = upload_layout(lay, counts))) return rc;
    if (p.profile != ENVPIC_PROFILE_NONE) launch_init_particles<R>(g, plasma(), S.parts[cur], S.lay[lay].offsets, stream);
    launch_init_envelope<R>(g, S.grids, laser(), fp64_rows ? 1 : 0, stream);
    if ((rc = launched("init kernels"))) return rc;
    sorted_at = n;  // the particles of P[cur] sit in their tiles
    if ((rc = hip_check(hipStreamSynchronize(stream), "init"))) return rc;
    return check_err();
  }

  int clear_deposits() override {
    const size_t ng = sz.ngrid;
    const size_t n1 = p.n_modes >= 2 ? ng : 0;
    for (int b = 0; b < 2; ++b) {
      int rc;
      if ((rc = hip_check(hipMemsetAsync(S.dep[b].chi, 0, ng * sizeof(R), stream), "clear chi"))) return rc;
      if ((rc = hip_check(hipMemsetAsync(S.dep[b].jx, 0, ng * sizeof(R), stream), "clear jx"))) return rc;
      if ((rc = hip_check(hipMemsetAsync(S.dep[b].jr, 0, ng * sizeof(R), stream), "clear jr"))) return rc;
      if (n1) {
        if ((rc = hip_check(hipMemsetAsync(S.dep[b].jx1, 0, n1 * sizeof(C), stream), "clear jx1"))) return rc;
        if ((rc = hip_check(hipMemsetAsync(S.dep[b].jr1, 0, n1 * sizeof(C), stream), "clear jr1"))) return rc;
        if ((rc = hip_check(hipMemsetAsync(S.dep[b].jt1, 0, n1 * sizeof(C), stream), "clear jt1"))) return rc;
      }
    }
    return hip_check(hipStreamSynchronize(stream), "clear deposits");
  }

  int sort_counts(int64_t* incremental, int64_t* rebuilt, int64_t* gathered) override {
    int c[3] = {0, 0, 0};
    int rc = hip_check(hipMemcpyAsync(c, S.sort_stats, sizeof c, hipMemcpyDeviceToHost, stream), "sort counts");
    if (rc || (rc = hip_check(hipStreamSynchronize(stream), "sync"))) return rc;
    *incremental = c[0];
    *rebuilt = c[1];
    *gathered = c[2];
    return ENVPIC_OK;
  }

  int check_err() override {
    int e = 0;
    int rc = hip_check(hipMemcpyAsync(&e, S.err, sizeof(int), hipMemcpyDeviceToHost, stream), "read error word");
    if (rc) return rc;
    if ((rc = hip_check(hipStreamSynchronize(stream), "sync"))) return rc;
    if (e & ERR_CAPACITY) return fail(ENVPIC_ENOMEM, "particle capacity exceeded");
    if (e & ERR_ITEMS) return fail(ENVPIC_ENOMEM, "work-item list overflow");
    if (e & ERR_LAYOUT) return fail(ENVPIC_EDEVICE, "a sort met more particles changing tile than its scan counted");
    if (e & ERR_HALO) return fail(ENVPIC_ENUMERIC, "a particle moved beyond its tile halo (non-finite or super-luminal state)");
    return ENVPIC_OK;
  }

  int momentum(bool defer) override {
    if (stage != 0) return fail(ENVPIC_EORDER, "momentum stage out of order");
    const Geo g = geo();
    const int d = (int)(n & 1);
    // re-sort when the particles have had sort_every() steps to drift from
    // their tiles; in between, p is updated in place
    const bool scatter = n - sorted_at >= sort_every();
    // every CELL_SORT_EVERY-th sort orders the tiles by cell again (into the
    // other buffer); the others move only the particles that changed tile
    const int mode = !scatter ? SCAT_NONE : (n_sorts % CELL_SORT_EVERY == 0 ? SCAT_CELL : SCAT_TILE);
    const KEvents ev = tick_events();
    // (the position scratch's cell words are free until the position stage)
    launch_momentum<R>(g, S.grids, S.dep[d].chi, S.parts[cur], S.parts[1 - cur], S.lay[lay], S.lay[1 - lay], S.ccur,
                       S.scr.w, S.scr.cell, S.err, sz.max_items, defer, mode, stream, ev);
    tick_end(0, ev);
    if (scatter) {
      if (mode == SCAT_CELL) {
        cur = 1 - cur;
        n_cell_sorts += 1;
      }
      settle_due = mode == SCAT_TILE && !defer;  // (the deferred form copies back at once)
      lay = 1 - lay;
      sorted_at = n;
      n_sorts += 1;
    }
    chi_last = d;
    stage = 1;
    deferred = defer;
    deposit_done = !defer;
    return launched("momentum pass");
  }

  int project(int what) override {
    const Geo g = geo();
    const int d = (int)(n & 1);
    if (what == ENVPIC_CHI) {
      if (stage != 1 || !deferred || deposit_done) return fail(ENVPIC_EORDER, "chi deposit needs a deferred momentum stage");
      launch_deposit_chi<R>(g, S.dep[d].chi, S.parts[cur], S.lay[lay], S.scr.w, S.err, sz.max_items, stream);
    } else if (what == ENVPIC_J) {
      if (stage != 3 || !deferred || deposit_done) return fail(ENVPIC_EORDER, "J deposit needs a deferred position stage");
      launch_deposit_J<R>(g, S.dep[d], S.parts[cur], S.lay[lay], shift_due() ? 1 : 0, S.scr, S.err, sz.max_items, stream);
    } else {
      return fail(ENVPIC_EINVAL, "project_chi_J: what must be ENVPIC_CHI or ENVPIC_J");
    }
    deposit_done = true;
    return launched("deposit");
  }

  int envelope() override {
    if (stage != 1 || !deposit_done) return fail(ENVPIC_EORDER, "envelope stage out of order");
    const Geo g = geo();
    const KEvents ev = tick_events();
    // a tile sort of this step that rebuilt its layout is copied back here
    SettleArgs<R> sa{};
    if (settle_due) {
      sa = SettleArgs<R>{S.parts[cur], S.parts[1 - cur], S.lay[lay], sz.capacity, SETTLE_BLOCKS};
      settle_due = false;
    }
    launch_envelope<R>(g, S.grids, S.dep[n & 1].chi, fp64_rows ? 1 : 0, sa, stream, ev);
    tick_end(1, ev);
    std::swap(S.grids.env, S.grids.envp);
    std::swap(S.grids.ax, S.grids.axp);
    stage = 2;
    return launched("envelope");
  }

  int position(bool defer) override {
    if (stage != 2) return fail(ENVPIC_EORDER, "position stage out of order");
    jf_valid = false;
    const Geo g = geo();
    const bool shifting = shift_due();
    // the plasma of the column entering the window at this step's shift is
    // loaded by extra work groups of the same launch (particles appended
    // past the live range; the field stage adds its items to the layout)
    InjectArgs inj{};
    inj.gn = geo_at(shift + 1);
    inj.pl = plasma();
    inj.capacity = sz.capacity;
    inj.max_items = sz.max_items;
    inj.pending = S.pending;
    inj.blocks = (shifting && p.profile != ENVPIC_PROFILE_NONE) ? inject_blocks<R>(inj.gn) : 0;
    const KEvents ev = tick_events();
    const SortCounts sc{next_sort(), S.ccount, S.hist, S.arr};
    launch_position<R>(g, S.grids, S.dep[n & 1], S.parts[cur], S.lay[lay], sc, shifting ? 1 : 0, S.scr, S.err,
                       sz.max_items, defer, inj, stream, ev);
    tick_end(2, ev);
    stage = 3;
    deferred = defer;
    deposit_done = !defer;
    return launched("position pass");
  }

  int field() override {
    if (stage != 3 || !deposit_done) return fail(ENVPIC_EORDER, "field stage out of order");
    const KEvents ev = tick_events();
    const Geo g = geo();
    const bool shifting = shift_due();
    const int pre = next_sort();
    if (shifting) shift += 1;
    const Geo gn = geo();
    FieldArgs fa{};
    fa.gn = gn;
    fa.shifting = shifting ? 1 : 0;
    fa.fp64_rows = fp64_rows ? 1 : 0;
    fa.presort = pre;
    fa.ccount = S.ccount;
    fa.ccur = S.ccur;
    fa.hist = S.hist;
    fa.arr = S.arr;
    fa.in = S.lay[lay];
    fa.out = S.lay[1 - lay];
    fa.capacity = sz.capacity;
    fa.inj_max = p.nr * sz.ppc;
    fa.reserve = slot_reserve(p, sz);
    fa.entering = (p.moving_window && p.profile != ENVPIC_PROFILE_NONE) ? ENTERING_TILES : 0;
    fa.max_items = sz.max_items;
    fa.pending = S.pending;
    fa.err = S.err;
    fa.stats = S.sort_stats;
    DepositBufs<R> din = S.dep[n & 1];
    if (p.filter_passes > 0) {
      // the field update reads the filtered current
      launch_filter<R>(g, din, S.jf, p.filter_passes, stream, KEvents{ev.start, nullptr});
      din.jx = S.jf.jx;
      din.jr = S.jf.jr;
      din.jx1 = S.jf.jx1;
      din.jr1 = S.jf.jr1;
      din.jt1 = S.jf.jt1;
      jf_valid = true;
    }
    launch_field<R>(g, S.grids, din, S.dep[(n + 1) & 1], S.dep[0], S.dep[1], fa, stream,
                    KEvents{p.filter_passes > 0 ? nullptr : ev.start, ev.stop});
    {
      Grids<R>& G = S.grids;  // the new E, B become the current ones
      std::swap(G.ex, G.ex_n);
      std::swap(G.er, G.er_n);
      std::swap(G.bt, G.bt_n);
      std::swap(G.ex1, G.ex1_n);
      std::swap(G.er1, G.er1_n);
      std::swap(G.et1, G.et1_n);
      std::swap(G.bx1, G.bx1_n);
      std::swap(G.br1, G.br1_n);
      std::swap(G.bt1, G.bt1_n);
    }
    tick_end(3, ev);
    n += 1;
    stage = 0;
    return launched("field stage");
  }


  // ---------------------------------------------------------------- IO --
  struct FieldRef {
    void* ptr;
    bool cplx, dual_x, dual_r;
  };
  int field_ref(int f, FieldRef& r) {
    const bool m1 = p.n_modes >= 2;
    Grids<R>& G = S.grids;
    switch (f) {
      case ENVPIC_F_ENV: r = {G.env, true, false, false}; return 0;
      case ENVPIC_F_ENV_PREV: r = {G.envp, true, false, false}; return 0;
      case ENVPIC_F_CHI: r = {S.dep[chi_last].chi, false, false, false}; return 0;
      case ENVPIC_F_EX: r = {G.ex, false, true, false}; return 0;
      case ENVPIC_F_ER: r = {G.er, false, false, true}; return 0;
      case ENVPIC_F_BT: r = {G.bt, false, true, true}; return 0;
      case ENVPIC_F_BT_BAR: r = {G.btb, false, true, true}; return 0;
      case ENVPIC_F_JX: r = {(jf_valid ? S.jf : S.dep[chi_last]).jx, false, true, false}; return 0;
      case ENVPIC_F_JR: r = {(jf_valid ? S.jf : S.dep[chi_last]).jr, false, false, true}; return 0;
      default: break;
    }
    if (!m1 || f < ENVPIC_F_EX1 || f >= ENVPIC_NFIELDS) return fail(ENVPIC_EINVAL, "unknown field (or mode 1 not enabled)");
    switch (f) {
      case ENVPIC_F_EX1: r = {G.ex1, true, true, false}; return 0;
      case ENVPIC_F_ER1: r = {G.er1, true, false, true}; return 0;
      case ENVPIC_F_ET1: r = {G.et1, true, false, false}; return 0;
      case ENVPIC_F_BX1: r = {G.bx1, true, false, true}; return 0;
      case ENVPIC_F_BR1: r = {G.br1, true, true, false}; return 0;
      case ENVPIC_F_BT1: r = {G.bt1, true, true, true}; return 0;
      case ENVPIC_F_BX1_BAR: r = {G.bxb1, true, false, true}; return 0;
      case ENVPIC_F_BR1_BAR: r = {G.brb1, true, true, false}; return 0;
      case ENVPIC_F_BT1_BAR: r = {G.btb1, true, true, true}; return 0;
      case ENVPIC_F_JX1: r = {(jf_valid ? S.jf : S.dep[chi_last]).jx1, true, true, false}; return 0;
      case ENVPIC_F_JR1: r = {(jf_valid ? S.jf : S.dep[chi_last]).jr1, true, false, true}; return 0;
      case ENVPIC_F_JT1: r = {(jf_valid ? S.jf : S.dep[chi_last]).jt1, true, false, false}; return 0;
    }
    return fail(ENVPIC_EINVAL, "unknown field");
  }

  int get_field(int f, double* out) override {
    FieldRef r;
    int rc = field_ref(f, r);
    if (rc) return rc;
    const int comp = r.cplx ? 2 : 1;
    std::vector<R> buf(sz.ngrid * comp);
    if ((rc = hip_check(hipMemcpyAsync(buf.data(), r.ptr, buf.size() * sizeof(R), hipMemcpyDeviceToHost, stream), "get_field"))) return rc;
    std::vector<double2> ax;
    const bool env = f == ENVPIC_F_ENV || f == ENVPIC_F_ENV_PREV;
    if (fp64_rows && env) {
      ax.resize((size_t)sz.nxa * 2);
      const double2* src = f == ENVPIC_F_ENV ? S.grids.ax : S.grids.axp;
      if ((rc = hip_check(hipMemcpyAsync(ax.data(), src, ax.size() * sizeof(double2), hipMemcpyDeviceToHost, stream), "get_field rows"))) return rc;
    }
    if ((rc = hip_check(hipStreamSynchronize(stream), "get_field sync"))) return rc;
    const Geo g = geo();
    const int nr1 = p.nr + 1;
    for (int i = 0; i <= p.nx; ++i) {
      const int pc = phys_col(g, i);
      for (int j = 0; j <= p.nr; ++j) {
        const bool valid = (!r.dual_x || i <= p.nx - 1) && (!r.dual_r || j <= p.nr - 1);
        const size_t o = (size_t)pc * sz.pitch + j;
        const size_t k = (size_t)i * nr1 + j;
        if (r.cplx) {
          double re = valid ? (double)buf[2 * o] : 0.0, im = valid ? (double)buf[2 * o + 1] : 0.0;
          if (fp64_rows && env && j <= 1) {
            re = ax[pc * 2 + j].x;
            im = ax[pc * 2 + j].y;
          }
          out[2 * k] = re;
          out[2 * k + 1] = im;
        } else {
          out[k] = valid ? (double)buf[o] : 0.0;
        }
      }
    }
    return ENVPIC_OK;
  }

  int set_field(int f, const double* in) override {
    FieldRef r;
    int rc = field_ref(f, r);
    if (rc) return rc;
    const int comp = r.cplx ? 2 : 1;
    std::vector<R> buf(sz.ngrid * comp, (R)0);
    if ((rc = hip_check(hipMemcpyAsync(buf.data(), r.ptr, buf.size() * sizeof(R), hipMemcpyDeviceToHost, stream), "set_field read"))) return rc;
    const bool env = f == ENVPIC_F_ENV || f == ENVPIC_F_ENV_PREV;
    std::vector<double2> ax;
    double2* axdev = nullptr;
    if (fp64_rows && env) {
      ax.resize((size_t)sz.nxa * 2);
      axdev = f == ENVPIC_F_ENV ? S.grids.ax : S.grids.axp;
      if ((rc = hip_check(hipMemcpyAsync(ax.data(), axdev, ax.size() * sizeof(double2), hipMemcpyDeviceToHost, stream), "set_field rows"))) return rc;
    }
    if ((rc = hip_check(hipStreamSynchronize(stream), "set_field sync"))) return rc;
    const Geo g = geo();
    const int nr1 = p.nr + 1;
    for (int i = 0; i <= p.nx; ++i) {
      const int pc = phys_col(g, i);
      for (int j = 0; j <= p.nr; ++j) {
        const size_t o = (size_t)pc * sz.pitch + j, k = (size_t)i * nr1 + j;
        if (r.cplx) {
          buf[2 * o] = (R)in[2 * k];
          buf[2 * o + 1] = (R)in[2 * k + 1];
          if (axdev && j <= 1) ax[pc * 2 + j] = make_double2(in[2 * k], in[2 * k + 1]);
        } else {
          buf[o] = (R)in[k];
        }
      }
    }
    if ((rc = hip_check(hipMemcpyAsync(r.ptr, buf.data(), buf.size() * sizeof(R), hipMemcpyHostToDevice, stream), "set_field write"))) return rc;
    if (axdev && (rc = hip_check(hipMemcpyAsync(axdev, ax.data(), ax.size() * sizeof(double2), hipMemcpyHostToDevice, stream), "set_field rows write"))) return rc;
    return hip_check(hipStreamSynchronize(stream), "set_field sync");
  }

  // the slots of P[cur] that work items cover (the free slots of the
  // tiles' segments hold stale records): [0, used) and a flag per slot
  int used_slots(int& used, std::vector<char>& covered) {
    int ni = 0;
    int rc = hip_check(hipMemcpyAsync(&ni, S.lay[lay].n_items, sizeof(int), hipMemcpyDeviceToHost, stream), "n_items");
    if (rc) return rc;
    if ((rc = hip_check(hipStreamSynchronize(stream), "sync"))) return rc;
    std::vector<int4> items(ni);
    if (ni && (rc = hip_check(hipMemcpyAsync(items.data(), S.lay[lay].items, ni * sizeof(int4), hipMemcpyDeviceToHost, stream), "items"))) return rc;
    if ((rc = hip_check(hipStreamSynchronize(stream), "sync"))) return rc;
    used = 0;
    for (const int4& it : items) used = std::max(used, it.y + it.z);
    covered.assign(used, 0);
    for (const int4& it : items)
      for (int k = it.y; k < it.y + it.z; ++k) covered[k] = 1;
    return ENVPIC_OK;
  }

  int get_particles(std::vector<double>* cols, std::vector<uint32_t>* ids) override {
    int used = 0;
    std::vector<char> covered;
    int rc = used_slots(used, covered);
    if (rc) return rc;
    const Parts<R>& P = S.parts[cur];
    std::vector<unsigned> cell(used);
    std::vector<R> a[7];
    const R* src[7] = {P.fx, P.fr, P.th, P.px, P.py, P.pz, P.w};
    std::vector<uint32_t> id(used);
    if (used) {
      if ((rc = hip_check(hipMemcpyAsync(cell.data(), P.cell, used * sizeof(unsigned), hipMemcpyDeviceToHost, stream), "cell"))) return rc;
      for (int k = 0; k < 7; ++k) {
        a[k].resize(used);
        if ((rc = hip_check(hipMemcpyAsync(a[k].data(), src[k], used * sizeof(R), hipMemcpyDeviceToHost, stream), "parts"))) return rc;
      }
      if ((rc = hip_check(hipMemcpyAsync(id.data(), P.id, used * sizeof(uint32_t), hipMemcpyDeviceToHost, stream), "id"))) return rc;
    }
    if ((rc = hip_check(hipStreamSynchronize(stream), "sync"))) return rc;
    std::vector<int> order;
    for (int k = 0; k < used; ++k)
      if (covered[k] && cell[k] != kDead) order.push_back(k);
    std::sort(order.begin(), order.end(), [&](int u, int v) { return id[u] < id[v]; });
    for (int c = 0; c < 7; ++c) cols[c].resize(order.size());
    ids->resize(order.size());
    for (size_t m = 0; m < order.size(); ++m) {
      const int k = order[m];
      const double r = ((double)cell_jr(cell[k]) + (double)a[1][k]) * p.dr;
      const double th = (double)a[2][k];
      cols[0][m] = ((double)cell_ix(cell[k]) + (double)a[0][k]) * p.dx;
      cols[1][m] = r * std::cos(th);
      cols[2][m] = r * std::sin(th);
      for (int c = 3; c < 7; ++c) cols[c][m] = (double)a[c][k];
      (*ids)[m] = id[k];
    }
    return ENVPIC_OK;
  }

  int set_particles(int64_t np, const double* const* in, const uint32_t* id) override {
    if (stage != 0) return fail(ENVPIC_EORDER, "set_particles only between steps");
    if (np < 0) return fail(ENVPIC_EINVAL, "negative particle count");
    if (np + (long long)p.nr * sz.ppc > sz.capacity) return fail(ENVPIC_ENOMEM, "too many particles for the capacity");
    const Geo g = geo();
    const double rmax = p.nr * p.dr;
    std::vector<int> key(np), counts(sz.ntiles, 0);
    std::vector<int> ixv(np), jrv(np);
    std::vector<double> fxv(np), frv(np), thv(np);
    for (int64_t k = 0; k < np; ++k) {
      if (!(std::isfinite(in[3][k]) && std::isfinite(in[4][k]) && std::isfinite(in[5][k]) && std::isfinite(in[6][k])))
        return fail(ENVPIC_EINVAL, "non-finite particle momentum or weight");
      const double u = in[0][k] / p.dx;
      const double c = std::floor(u);
      const double r = std::sqrt(in[1][k] * in[1][k] + in[2][k] * in[2][k]);
      if (!(c >= (double)shift && c < (double)(shift + p.nx)) || !(r <= rmax))
        return fail(ENVPIC_EINVAL, "particle outside the window or beyond r_max");
      ixv[k] = (int)c;
      fxv[k] = u - c;
      const double ur = r / p.dr;
      int jr = (int)std::floor(ur);
      if (jr > p.nr - 1) jr = p.nr - 1;
      jrv[k] = jr;
      frv[k] = ur - jr;
      thv[k] = std::atan2(in[2][k], in[1][k]);
      key[k] = tile_key(g, ixv[k], jr);
      counts[key[k]]++;
    }
    std::vector<int> off(sz.ntiles + 1, 0);
    for (int t = 0; t < sz.ntiles; ++t) off[t + 1] = off[t] + counts[t];
    std::vector<int> pos(off.begin(), off.end() - 1);
    std::vector<unsigned> hcell(np);
    std::vector<R> h[7];
    for (int c = 0; c < 7; ++c) h[c].resize(np);
    std::vector<uint32_t> hid(np);
    for (int64_t k = 0; k < np; ++k) {
      const int d = pos[key[k]]++;
      int ix = ixv[k], jr = jrv[k];
      R fx = (R)fxv[k], fr = (R)frv[k];
      if (fx >= (R)1) fx = (R)0, ix += 1;  // rounding of the offsets
      if (fr > (R)1) fr = (R)1;
      hcell[d] = pack_cell(ix, jr);
      h[0][d] = fx;
      h[1][d] = fr;
      h[2][d] = (R)thv[k];
      for (int c = 3; c < 7; ++c) h[c][d] = (R)in[c][k];
      hid[d] = id[k];
      wmax = std::max(wmax, std::fabs((double)h[6][d]));
    }
    int rc;
    lay = cur;
    if ((rc = upload_layout(lay, counts))) return rc;
    Parts<R>& P = S.parts[cur];
    R* dst[7] = {P.fx, P.fr, P.th, P.px, P.py, P.pz, P.w};
    if (np) {
      if ((rc = hip_check(hipMemcpyAsync(P.cell, hcell.data(), np * sizeof(unsigned), hipMemcpyHostToDevice, stream), "cell"))) return rc;
      for (int c = 0; c < 7; ++c)
        if ((rc = hip_check(hipMemcpyAsync(dst[c], h[c].data(), np * sizeof(R), hipMemcpyHostToDevice, stream), "parts"))) return rc;
      if ((rc = hip_check(hipMemcpyAsync(P.id, hid.data(), np * sizeof(uint32_t), hipMemcpyHostToDevice, stream), "id"))) return rc;
    }
    sorted_at = n;  // the particles of P[cur] sit in their tiles
    return hip_check(hipStreamSynchronize(stream), "set_particles");
  }

  int diagnostics(double* out) override {
    const Geo g = geo();
    launch_diag<R>(g, S.parts[cur], S.lay[lay], S.grids, S.dep[chi_last].chi, fp64_rows ? 1 : 0, S.diag_scratch,
                   S.diag_out, stream);
    int rc = launched("diagnostics");
    if (rc) return rc;
    if ((rc = hip_check(hipMemcpyAsync(out, S.diag_out, ENVPIC_NDIAG * sizeof(double), hipMemcpyDeviceToHost, stream), "diag read"))) return rc;
    if ((rc = hip_check(hipStreamSynchronize(stream), "diag sync"))) return rc;
    return check_err();
  }

  // the same kernels with the partial sums in the library's static scratch
  // and the result written to caller-owned device memory, asynchronously
  int diagnostics_noalloc(double* dev_out) override {
    if (!diag_static) return fail(ENVPIC_EDEVICE, "the static diagnostics scratch is not available on this device");
    if ((size_t)diag_scratch_doubles() > diag_static_doubles)
      return fail(ENVPIC_EINVAL, "diagnostics partial sums exceed the static scratch");
    launch_diag<R>(geo(), S.parts[cur], S.lay[lay], S.grids, S.dep[chi_last].chi, fp64_rows ? 1 : 0, diag_static,
                   dev_out, stream);
    return launched("diagnostics (static scratch)");
  }

  int beam(double e_lo, double e_hi, int nbins, double* out, double* hist) override {
    BeamArgs a{};
    a.e_lo = e_lo;
    a.e_hi = e_hi;
    a.nbins = nbins;
    a.de = (e_hi - e_lo) / nbins;
    // fixed-point histogram: a power of two with capacity * w_max * scale <= 2^61
    const double wb = std::max(wmax, 1e-300) * (double)sz.capacity;
    a.scale = std::ldexp(1.0, std::min(1000, (int)std::floor(std::log2(std::ldexp(1.0, 61) / wb))));
    launch_beam<R>(geo(), S.parts[cur], S.lay[lay], sz.max_items, a, S.beam, stream);
    int rc = launched("beam diagnostics");
    if (rc) return rc;
    if ((rc = hip_check(hipMemcpyAsync(out, S.beam.out, ENVPIC_NBEAM * sizeof(double), hipMemcpyDeviceToHost, stream), "beam read"))) return rc;
    if (hist && (rc = hip_check(hipMemcpyAsync(hist, S.beam.hist_f, nbins * sizeof(double), hipMemcpyDeviceToHost, stream), "beam hist"))) return rc;
    if ((rc = hip_check(hipStreamSynchronize(stream), "beam sync"))) return rc;
    return check_err();
  }

  int bunch(uint32_t id_lo, uint32_t id_hi, double beta, double tol, int max_iter, int* iters,
            double* resid) override {
    int it = 0;
    double res = 0.0;
    if (bunch_solve<R>(geo(), S.parts[cur], S.lay[lay], sz.max_items, S.grids, id_lo, id_hi, beta, tol, max_iter,
                       S.cg, stream, &it, &res)) {
      const int rc = launched("bunch fields");
      return rc ? rc : fail(ENVPIC_EDEVICE, "bunch fields: residual transfer failed");
    }
    int rc = launched("bunch fields");
    if (rc) return rc;
    if ((rc = hip_check(hipStreamSynchronize(stream), "bunch sync"))) return rc;
    if (iters) *iters = it;
    if (resid) *resid = res;
    if (!(res <= tol)) return fail(ENVPIC_ENUMERIC, "bunch field solve did not reach the tolerance");
    return check_err();
  }

  int poison(int f) override {
    std::vector<double> buf;
    FieldRef r;
    int rc = field_ref(f, r);
    if (rc) return rc;
    buf.resize((size_t)(p.nx + 1) * (p.nr + 1) * (r.cplx ? 2 : 1));
    if ((rc = get_field(f, buf.data()))) return rc;
    const size_t k = (size_t)(p.nx / 2) * (p.nr + 1) + p.nr / 2;
    buf[r.cplx ? 2 * k : k] = std::nan("");
    return set_field(f, buf.data());
  }
};

template <class R>
int create(const envpic_params* p, int prec, void* arena, size_t bytes, void* stream, envpic_sim** out) {
  SimT<R>* s = new (std::nothrow) SimT<R>();
  if (!s) return fail(ENVPIC_ENOMEM, "host allocation failed");
  s->p = *p;
  s->prec = prec;
  s->stream = (hipStream_t)stream;
  s->sz = sizes_of(*p);
  s->fp64_rows = (prec == ENVPIC_FP32_BULK);
  s->arena = (char*)arena;
  // set-up of the static diagnostics scratch of this GPU (once per device;
  // only the allocation-free diagnostics call needs it)
  if (hipGetDevice(&s->device) != hipSuccess || static_scratch(s->device, &s->diag_static, &s->diag_static_doubles))
    s->diag_static = nullptr;
  plan<R>(*p, s->sz, s->fp64_rows, (char*)arena, &s->S);
  int rc = s->init();
  if (rc) {
    delete s;
    return rc;
  }
  *out = s;
  return ENVPIC_OK;
}

}  // namespace

// ============================================================== C ABI ==
extern "C" {

void envpic_params_default(envpic_params* p, int preset) {
  if (!p) return;
  std::memset(p, 0, sizeof *p);
  p->size = sizeof(envpic_params);
  p->version = ENVPIC_PARAMS_VERSION;
  p->dx = 0.8;
  p->dr = 1.5;
  p->dt = 0.6;
  p->n_modes = 1;
  p->ppc_x = 2;
  p->ppc_r = 2;
  p->ppc_t = 1;
  p->seed = 191204674ull + (uint64_t)preset;
  p->w0 = 1.0;
  p->tau = 1.0;
  p->bump_w = 1.0;
  switch (preset) {
    case 1:  // mode-0 parity case
      p->nx = 256; p->nr = 32; p->profile = ENVPIC_PROFILE_UNIFORM; p->n0 = 0.002;
      p->a0 = 1.0; p->w0 = 20.0; p->tau = 30.0; p->x_c = p->x_f = 102.4;
      break;
    case 2:  // LWFA-shaped run with a moving window
      p->nx = 2048; p->nr = 256; p->n_modes = 2; p->ppc_t = 4; p->profile = ENVPIC_PROFILE_RAMP;
      p->n0 = 0.0017; p->ramp_len = 200.0; p->a0 = 2.0; p->w0 = 100.0; p->tau = 60.0;
      p->x_c = p->x_f = 2048 * 0.8 - 180.0; p->moving_window = 1;
      break;
    case 3:  // bandwidth case
      p->nx = 4096; p->nr = 512; p->n_modes = 2; p->ppc_t = 4; p->profile = ENVPIC_PROFILE_PERTURB;
      p->n0 = 0.001; p->perturb = 0.01; p->a0 = 2.5; p->w0 = 150.0; p->tau = 80.0;
      p->x_c = p->x_f = 4096 * 0.8 / 2; p->sort_every = 1;
      break;
    case 4:  // largest scan-job shape
      p->nx = 2048; p->nr = 256; p->ppc_t = 2; p->profile = ENVPIC_PROFILE_UNIFORM; p->n0 = 0.0025;
      p->a0 = 1.75; p->w0 = 80.0; p->tau = 30.0; p->x_c = p->x_f = 2048 * 0.8 - 90.0; p->moving_window = 1;
      break;
    case 5:  // scale case
      p->nx = 8192; p->nr = 768; p->n_modes = 2; p->ppc_t = 6; p->profile = ENVPIC_PROFILE_BUMP;
      p->n0 = 0.0015; p->bump_x = 8192 * 0.8 + 400.0; p->bump_w = 100.0; p->a0 = 3.0; p->w0 = 200.0;
      p->tau = 90.0; p->x_c = p->x_f = 8192 * 0.8 - 270.0; p->moving_window = 1;
      break;
    default:  // small vacuum grid
      p->nx = 64; p->nr = 16; p->profile = ENVPIC_PROFILE_NONE;
      break;
  }
}

int envpic_footprint(const envpic_params* p, int precision, size_t* bytes) {
  int rc = validate(p);
  if (rc) return rc;
  if (precision != ENVPIC_FP32_BULK && precision != ENVPIC_FP64) return fail(ENVPIC_EINVAL, "unknown precision");
  if (!bytes) return fail(ENVPIC_EINVAL, "bytes is NULL");
  *bytes = footprint_bytes(*p, precision);
  return ENVPIC_OK;
}

int envpic_sim_init(const envpic_params* p, int precision, void* dev_arena, size_t arena_bytes, void* hip_stream,
                    envpic_sim** out) {
  size_t need = 0;
  int rc = envpic_footprint(p, precision, &need);
  if (rc) return rc;
  if (!out || !dev_arena) return fail(ENVPIC_EINVAL, "NULL arena or output handle");
  if (((uintptr_t)dev_arena & 255) != 0) return fail(ENVPIC_EINVAL, "arena must be 256-byte aligned");
  if (arena_bytes < need) {
    char buf[128];
    std::snprintf(buf, sizeof buf, "arena of %zu bytes is smaller than the footprint %zu", arena_bytes, need);
    return fail(ENVPIC_ENOMEM, buf);
  }
  if (precision == ENVPIC_FP64) return create<double>(p, precision, dev_arena, arena_bytes, hip_stream, out);
  return create<float>(p, precision, dev_arena, arena_bytes, hip_stream, out);
}

int envpic_gather_push(envpic_sim* s, int stage) {
  if (!s) return fail(ENVPIC_EINVAL, "NULL sim");
  const bool defer = (stage & ENVPIC_DEFER_DEPOSIT) != 0;
  stage &= ~ENVPIC_DEFER_DEPOSIT;
  if (defer && s->p.shape_order == 2)
    return fail(ENVPIC_EINVAL, "deferred deposits are built for linear shapes only");
  if (stage == ENVPIC_MOMENTUM) return s->momentum(defer);
  if (stage == ENVPIC_POSITION) return s->position(defer);
  return fail(ENVPIC_EINVAL, "stage must be ENVPIC_MOMENTUM or ENVPIC_POSITION");
}

int envpic_envelope_step(envpic_sim* s) { return s ? s->envelope() : fail(ENVPIC_EINVAL, "NULL sim"); }
int envpic_project_chi_J(envpic_sim* s, int what) { return s ? s->project(what) : fail(ENVPIC_EINVAL, "NULL sim"); }
int envpic_field_step(envpic_sim* s) { return s ? s->field() : fail(ENVPIC_EINVAL, "NULL sim"); }

int envpic_step_n(envpic_sim* s, int nsteps) {
  if (!s) return fail(ENVPIC_EINVAL, "NULL sim");
  if (nsteps < 0) return fail(ENVPIC_EINVAL, "nsteps must be >= 0");
  if (s->stage != 0) return fail(ENVPIC_EORDER, "step_n called in the middle of a step");
  if (s->graph_steps > 0 && s->timing == 0) {
    for (int done = 0; done < nsteps;) {
      const int k = std::min(s->graph_steps, nsteps - done);
      int rc = s->step_graph(k);
      if (rc) return rc;
      done += k;
    }
    return ENVPIC_OK;
  }
  for (int k = 0; k < nsteps; ++k) {
    int rc = s->step();
    if (rc) return rc;
  }
  return ENVPIC_OK;
}

int envpic_batch_step(envpic_sim* const* sims, int count, int nsteps, void* hip_stream) {
  if (count < 0 || nsteps < 0 || (count > 0 && !sims)) return fail(ENVPIC_EINVAL, "bad simulation list or step count");
  for (int k = 0; k < count; ++k) {
    if (!sims[k]) return fail(ENVPIC_EINVAL, "NULL simulation in the list");
    for (int m = 0; m < k; ++m)
      if (sims[m] == sims[k]) return fail(ENVPIC_EINVAL, "a simulation appears twice in the list");
  }
  for (int k = 0; k < count; ++k)
    if (sims[k]->stage != 0) return fail(ENVPIC_EORDER, "batch_step needs every simulation between steps");
  // interleave: step k of every simulation before step k+1 of any, each on
  // its own stream so that the kernels of different simulations overlap
  for (int st = 0; st < nsteps; ++st)
    for (int k = 0; k < count; ++k) {
      int rc = sims[k]->step();
      if (rc) return rc;
    }
  hipStream_t join = (hipStream_t)hip_stream;
  for (int k = 0; k < count; ++k) {
    if (sims[k]->stream == join) continue;
    hipEvent_t ev;
    int rc = hip_check(hipEventCreateWithFlags(&ev, hipEventDisableTiming), "event");
    if (rc) return rc;
    if ((rc = hip_check(hipEventRecord(ev, sims[k]->stream), "event record"))) return rc;
    if ((rc = hip_check(hipStreamWaitEvent(join, ev, 0), "stream wait"))) return rc;
    if ((rc = hip_check(hipEventDestroy(ev), "event destroy"))) return rc;
  }
  return hip_check(hipGetLastError(), "batch_step");
}

int envpic_get_field(const envpic_sim* s, int field, double* out) {
  if (!s || !out) return fail(ENVPIC_EINVAL, "NULL argument");
  return const_cast<envpic_sim*>(s)->get_field(field, out);
}
int envpic_set_field(envpic_sim* s, int field, const double* in) {
  if (!s || !in) return fail(ENVPIC_EINVAL, "NULL argument");
  return s->set_field(field, in);
}

int envpic_sort_stats(const envpic_sim* s, int64_t* out) {
  if (!s || !out) return fail(ENVPIC_EINVAL, "NULL argument");
  out[0] = s->n_cell_sorts;
  return const_cast<envpic_sim*>(s)->sort_counts(&out[1], &out[2], &out[3]);
}

int envpic_state(const envpic_sim* s, int64_t* n, int64_t* shift, int64_t* n_particles) {
  if (!s) return fail(ENVPIC_EINVAL, "NULL sim");
  if (n) *n = s->n;
  if (shift) *shift = s->shift;
  if (n_particles) {
    double d[ENVPIC_NDIAG];
    int rc = const_cast<envpic_sim*>(s)->diagnostics(d);
    if (rc) return rc;
    *n_particles = (int64_t)d[ENVPIC_D_COUNT];
  }
  return ENVPIC_OK;
}

int envpic_get_particles(const envpic_sim* s, double* x, double* y, double* z, double* px, double* py, double* pz,
                         double* w, uint32_t* id) {
  if (!s) return fail(ENVPIC_EINVAL, "NULL sim");
  std::vector<double> cols[7];
  std::vector<uint32_t> ids;
  int rc = const_cast<envpic_sim*>(s)->get_particles(cols, &ids);
  if (rc) return rc;
  double* outs[7] = {x, y, z, px, py, pz, w};
  for (int c = 0; c < 7; ++c)
    if (outs[c] && !cols[c].empty()) std::memcpy(outs[c], cols[c].data(), cols[c].size() * sizeof(double));
  if (id && !ids.empty()) std::memcpy(id, ids.data(), ids.size() * sizeof(uint32_t));
  return ENVPIC_OK;
}

int envpic_set_particles(envpic_sim* s, int64_t n, const double* x, const double* y, const double* z,
                         const double* px, const double* py, const double* pz, const double* w, const uint32_t* id) {
  if (!s) return fail(ENVPIC_EINVAL, "NULL sim");
  if (n > 0 && (!x || !y || !z || !px || !py || !pz || !w || !id)) return fail(ENVPIC_EINVAL, "NULL particle array");
  const double* cols[7] = {x, y, z, px, py, pz, w};
  return s->set_particles(n, cols, id);
}

int envpic_set_timing(envpic_sim* s, int enable) {
  if (!s) return fail(ENVPIC_EINVAL, "NULL sim");
  int rc = s->resolve_ticks();
  if (rc) return fail(rc, "timing events failed");
  for (int k = 0; k < 4; ++k) {
    s->t_ms[k] = 0.0;
    s->t_n[k] = 0;
  }
  s->timing = enable > 0 ? enable : 0;
  return ENVPIC_OK;
}

int envpic_set_graph(envpic_sim* s, int steps) {
  if (!s) return fail(ENVPIC_EINVAL, "NULL sim");
  if (steps < 0) return fail(ENVPIC_EINVAL, "negative graph length");
  s->graph_steps = steps;
  return ENVPIC_OK;
}

int envpic_get_timing(envpic_sim* s, double* out_ms, int64_t* counts) {
  if (!s) return fail(ENVPIC_EINVAL, "NULL sim");
  int rc = s->resolve_ticks();
  if (rc) return fail(rc, "timing events failed");
  for (int k = 0; k < 4; ++k) {
    if (out_ms) out_ms[k] = s->t_n[k] ? s->t_ms[k] / (double)s->t_n[k] : 0.0;
    if (counts) counts[k] = s->t_n[k];
  }
  return ENVPIC_OK;
}

int envpic_diagnostics(const envpic_sim* s, double* out) {
  if (!s || !out) return fail(ENVPIC_EINVAL, "NULL argument");
  return const_cast<envpic_sim*>(s)->diagnostics(out);
}

int envpic_diagnostics_noalloc(const envpic_sim* cs, double* dev_out) {
  envpic_sim* s = const_cast<envpic_sim*>(cs);
  if (!s || !dev_out) return fail(ENVPIC_EINVAL, "NULL argument");
  if (s->stage != 0) return fail(ENVPIC_EORDER, "diagnostics only between steps");
  return s->diagnostics_noalloc(dev_out);
}

int envpic_beam_diagnostics(const envpic_sim* cs, double e_lo, double e_hi, int nbins, double* out, double* hist) {
  static_assert(ENVPIC_BEAM_MAX_BINS == envpic::BEAM_MAX_BINS, "beam histogram bound");
  envpic_sim* s = const_cast<envpic_sim*>(cs);
  if (!s || !out) return fail(ENVPIC_EINVAL, "NULL argument");
  if (!(std::isfinite(e_lo) && std::isfinite(e_hi) && e_hi > e_lo))
    return fail(ENVPIC_EINVAL, "beam diagnostics need finite e_lo < e_hi");
  if (nbins < 1 || nbins > ENVPIC_BEAM_MAX_BINS) return fail(ENVPIC_EINVAL, "nbins outside [1, ENVPIC_BEAM_MAX_BINS]");
  if (s->stage != 0) return fail(ENVPIC_EORDER, "beam diagnostics only between steps");
  return s->beam(e_lo, e_hi, nbins, out, hist);
}

int envpic_bunch_fields(envpic_sim* s, uint32_t id_lo, uint32_t id_hi, double beta, double tol, int max_iter,
                        int* iters, double* resid) {
  if (!s) return fail(ENVPIC_EINVAL, "NULL sim");
  if (!(beta >= 0.0 && beta < 1.0)) return fail(ENVPIC_EINVAL, "beta must be in [0, 1)");
  if (!(tol > 0.0 && std::isfinite(tol)) || max_iter < 1) return fail(ENVPIC_EINVAL, "need tol > 0 and max_iter >= 1");
  if (id_hi <= id_lo) return fail(ENVPIC_EINVAL, "empty id range");
  if (s->stage != 0) return fail(ENVPIC_EORDER, "bunch fields only between steps");
  return s->bunch(id_lo, id_hi, beta, tol, max_iter, iters, resid);
}

// checkpoint blob: header, the persistent grids (FP64, window-relative),
// particles (FP64 columns ordered by id)
namespace {
struct BlobHeader {
  char magic[8];
  int32_t version, prec, nx, nr, modes, nfields;
  int64_t n, shift, nparticles;
  envpic_params params;
};
const int kCkptFields[] = {ENVPIC_F_ENV, ENVPIC_F_ENV_PREV, ENVPIC_F_EX, ENVPIC_F_ER, ENVPIC_F_BT, ENVPIC_F_BT_BAR,
                           ENVPIC_F_EX1, ENVPIC_F_ER1, ENVPIC_F_ET1, ENVPIC_F_BX1, ENVPIC_F_BR1, ENVPIC_F_BT1,
                           ENVPIC_F_BX1_BAR, ENVPIC_F_BR1_BAR, ENVPIC_F_BT1_BAR};
int n_ckpt_fields(const envpic_params& p) { return p.n_modes >= 2 ? 15 : 6; }
size_t field_doubles(const envpic_params& p, int f) {
  const bool c = f == ENVPIC_F_ENV || f == ENVPIC_F_ENV_PREV || f >= ENVPIC_F_EX1;
  return (size_t)(p.nx + 1) * (p.nr + 1) * (c ? 2 : 1);
}
}  // namespace

int envpic_save(const envpic_sim* cs, void* blob, size_t* bytes) {
  envpic_sim* s = const_cast<envpic_sim*>(cs);
  if (!s || !bytes) return fail(ENVPIC_EINVAL, "NULL argument");
  if (s->stage != 0) return fail(ENVPIC_EORDER, "save only between steps");
  std::vector<double> cols[7];
  std::vector<uint32_t> ids;
  int rc = s->get_particles(cols, &ids);
  if (rc) return rc;
  size_t need = sizeof(BlobHeader);
  for (int k = 0; k < n_ckpt_fields(s->p); ++k) need += field_doubles(s->p, kCkptFields[k]) * sizeof(double);
  need += ids.size() * (7 * sizeof(double) + sizeof(uint32_t));
  if (!blob) {
    *bytes = need;
    return ENVPIC_OK;
  }
  if (*bytes < need) return fail(ENVPIC_ENOMEM, "checkpoint buffer too small");
  char* q = (char*)blob;
  BlobHeader h{};
  std::memcpy(h.magic, "ENVPIC01", 8);
  h.version = 1;
  h.prec = s->prec;
  h.nx = s->p.nx;
  h.nr = s->p.nr;
  h.modes = s->p.n_modes;
  h.nfields = n_ckpt_fields(s->p);
  h.n = s->n;
  h.shift = s->shift;
  h.nparticles = (int64_t)ids.size();
  h.params = s->p;
  std::memcpy(q, &h, sizeof h);
  q += sizeof h;
  for (int k = 0; k < h.nfields; ++k) {
    if ((rc = s->get_field(kCkptFields[k], (double*)q))) return rc;
    q += field_doubles(s->p, kCkptFields[k]) * sizeof(double);
  }
  for (int c = 0; c < 7; ++c) {
    if (!ids.empty()) std::memcpy(q, cols[c].data(), ids.size() * sizeof(double));
    q += ids.size() * sizeof(double);
  }
  if (!ids.empty()) std::memcpy(q, ids.data(), ids.size() * sizeof(uint32_t));
  *bytes = need;
  return ENVPIC_OK;
}

int envpic_load(envpic_sim* s, const void* blob, size_t bytes) {
  if (!s || !blob) return fail(ENVPIC_EINVAL, "NULL argument");
  if (s->stage != 0) return fail(ENVPIC_EORDER, "load only between steps");
  if (bytes < sizeof(BlobHeader)) return fail(ENVPIC_EINVAL, "checkpoint too short");
  BlobHeader h;
  std::memcpy(&h, blob, sizeof h);
  if (std::memcmp(h.magic, "ENVPIC01", 8) != 0 || h.prec != s->prec || h.nx != s->p.nx || h.nr != s->p.nr ||
      h.modes != s->p.n_modes)
    return fail(ENVPIC_EINVAL, "checkpoint does not match this simulation");
  // the parameter block has no padding: equal parameters are equal bytes
  static_assert(sizeof(envpic_params) == 12 * 4 + 8 + 13 * 8 + 8 + 4 * 4, "envpic_params has padding");
  if (std::memcmp(&h.params, &s->p, sizeof(envpic_params)) != 0)
    return fail(ENVPIC_EINVAL, "checkpoint written with other parameters");
  if (h.nfields != n_ckpt_fields(s->p)) return fail(ENVPIC_EINVAL, "checkpoint field count does not match");
  if (h.n < 0 || h.shift < 0 || h.nparticles < 0 || h.nparticles > s->sz.capacity)
    return fail(ENVPIC_EINVAL, "checkpoint step, shift or particle count out of range");
  const char* q = (const char*)blob + sizeof h;
  size_t need = sizeof h;
  for (int k = 0; k < h.nfields; ++k) need += field_doubles(s->p, kCkptFields[k]) * sizeof(double);
  need += (size_t)h.nparticles * (7 * sizeof(double) + sizeof(uint32_t));
  if (bytes < need) return fail(ENVPIC_EINVAL, "checkpoint truncated");
  // step counter and window first: the IO below is window-relative
  s->n = h.n;
  s->shift = h.shift;
  s->chi_last = (int)((h.n + 1) & 1);
  s->jf_valid = false;
  int rc;
  if ((rc = s->clear_deposits())) return rc;
  for (int k = 0; k < h.nfields; ++k) {
    if ((rc = s->set_field(kCkptFields[k], (const double*)q))) return rc;
    q += field_doubles(s->p, kCkptFields[k]) * sizeof(double);
  }
  const double* cols[7];
  for (int c = 0; c < 7; ++c) {
    cols[c] = (const double*)q;
    q += (size_t)h.nparticles * sizeof(double);
  }
  return s->set_particles(h.nparticles, cols, (const uint32_t*)q);
}

int envpic_debug_poison(envpic_sim* s, int field) { return s ? s->poison(field) : fail(ENVPIC_EINVAL, "NULL sim"); }

void envpic_sim_destroy(envpic_sim* s) {
  if (!s) return;
  // the arena returns to the caller: no kernel of this simulation may still
  // be reading or writing it
  (void)hipStreamSynchronize(s->stream);
  delete s;
}

const char* envpic_last_error(const envpic_sim*) { return g_last_error.c_str(); }

}  // extern "C"
