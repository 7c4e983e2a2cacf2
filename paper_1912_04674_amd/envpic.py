"""ctypes binding of libenvpic.so (include/envpic.h).

Argument marshalling only: every stage of the step runs in the HIP kernels.
PyTorch provides the device arena and the stream.  If the library has not
been built this module raises on first use; there is no other code path.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libenvpic.so")
HEADER = os.path.join(_HERE, "..", "include", "envpic.h")

PARAMS_VERSION = 3
FP32_BULK, FP64 = 0, 1
MOMENTUM, POSITION = 0, 1
DEFER_DEPOSIT = 0x100
CHI, J = 1, 2

PROFILES = {"none": 0, "uniform": 1, "ramp": 2, "perturb": 3, "bump": 4}
FIELDS = {
    "env": 0, "env_prev": 1, "chi": 2, "ex": 3, "er": 4, "bt": 5, "bt_bar": 6,
    "jx": 7, "jr": 8, "ex1": 9, "er1": 10, "et1": 11, "bx1": 12, "br1": 13,
    "bt1": 14, "bx1_bar": 15, "br1_bar": 16, "bt1_bar": 17, "jx1": 18,
    "jr1": 19, "jt1": 20,
}
COMPLEX_FIELDS = {"env", "env_prev", "ex1", "er1", "et1", "bx1", "br1", "bt1",
                  "bx1_bar", "br1_bar", "bt1_bar", "jx1", "jr1", "jt1"}
DIAG_NAMES = ["count", "charge", "chi_v", "kin", "uem", "env2_v", "lx", "px", "nonfinite"]
BEAM_NAMES = ["e_peak", "fwhm", "charge", "e_mean", "e_rms", "rel_spread", "emit_y", "emit_z", "count",
              "charge_spectrum", "win_lo", "win_hi"]
BEAM_MAX_BINS = 4096
ERRORS = {-1: "EINVAL", -2: "ENOMEM", -3: "EORDER", -4: "EDEVICE", -5: "ENUMERIC"}


class EnvpicError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"envpic {ERRORS.get(code, code)}: {msg}")
        self.code = code


class Params(ctypes.Structure):
    _fields_ = [
        ("size", ctypes.c_int32), ("version", ctypes.c_int32),
        ("nx", ctypes.c_int32), ("nr", ctypes.c_int32), ("n_modes", ctypes.c_int32),
        ("ppc_x", ctypes.c_int32), ("ppc_r", ctypes.c_int32), ("ppc_t", ctypes.c_int32),
        ("profile", ctypes.c_int32), ("moving_window", ctypes.c_int32),
        ("tile_x", ctypes.c_int32), ("tile_r", ctypes.c_int32),
        ("seed", ctypes.c_uint64),
        ("dx", ctypes.c_double), ("dr", ctypes.c_double), ("dt", ctypes.c_double),
        ("a0", ctypes.c_double), ("w0", ctypes.c_double), ("tau", ctypes.c_double),
        ("x_c", ctypes.c_double), ("x_f", ctypes.c_double),
        ("n0", ctypes.c_double), ("ramp_len", ctypes.c_double), ("perturb", ctypes.c_double),
        ("bump_x", ctypes.c_double), ("bump_w", ctypes.c_double),
        ("capacity", ctypes.c_int64),
        ("filter_passes", ctypes.c_int32), ("shape_order", ctypes.c_int32),
        ("sort_every", ctypes.c_int32), ("reserved", ctypes.c_int32),
    ]


_lib = None
EXPORTS = [
    "envpic_params_default", "envpic_footprint", "envpic_sim_init", "envpic_gather_push",
    "envpic_envelope_step", "envpic_project_chi_J", "envpic_field_step", "envpic_step_n",
    "envpic_batch_step", "envpic_get_field", "envpic_set_field", "envpic_state",
    "envpic_get_particles", "envpic_set_particles", "envpic_diagnostics", "envpic_save",
    "envpic_load", "envpic_debug_poison", "envpic_sim_destroy", "envpic_last_error",
    "envpic_set_timing", "envpic_get_timing", "envpic_set_graph", "envpic_beam_diagnostics",
    "envpic_bunch_fields", "envpic_stream_copy", "envpic_diagnostics_noalloc", "envpic_sort_stats",
]


def lib():
    """Load libenvpic.so (raises if it is not built).  ENVPIC_LIB in the
    environment names another build of the library to load instead."""
    global _lib
    if _lib is not None:
        return _lib
    path = os.environ.get("ENVPIC_LIB") or LIB_PATH
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with "
                           "`python -m paper_1912_04674_amd.build_lib`")
    L = ctypes.CDLL(path)
    vp, dp = ctypes.c_void_p, ctypes.POINTER(ctypes.c_double)
    up, i64p = ctypes.POINTER(ctypes.c_uint32), ctypes.POINTER(ctypes.c_int64)
    pp = ctypes.POINTER(Params)
    L.envpic_params_default.argtypes = [pp, ctypes.c_int]
    L.envpic_params_default.restype = None
    L.envpic_footprint.argtypes = [pp, ctypes.c_int, ctypes.POINTER(ctypes.c_size_t)]
    L.envpic_sim_init.argtypes = [pp, ctypes.c_int, vp, ctypes.c_size_t, vp, ctypes.POINTER(vp)]
    L.envpic_gather_push.argtypes = [vp, ctypes.c_int]
    L.envpic_envelope_step.argtypes = [vp]
    L.envpic_project_chi_J.argtypes = [vp, ctypes.c_int]
    L.envpic_field_step.argtypes = [vp]
    L.envpic_step_n.argtypes = [vp, ctypes.c_int]
    L.envpic_batch_step.argtypes = [ctypes.POINTER(vp), ctypes.c_int, ctypes.c_int, vp]
    L.envpic_get_field.argtypes = [vp, ctypes.c_int, dp]
    L.envpic_set_field.argtypes = [vp, ctypes.c_int, dp]
    L.envpic_state.argtypes = [vp, i64p, i64p, i64p]
    L.envpic_sort_stats.argtypes = [vp, i64p]
    L.envpic_get_particles.argtypes = [vp] + [dp] * 7 + [up]
    L.envpic_set_particles.argtypes = [vp, ctypes.c_int64] + [dp] * 7 + [up]
    L.envpic_diagnostics.argtypes = [vp, dp]
    L.envpic_diagnostics_noalloc.argtypes = [vp, vp]
    L.envpic_beam_diagnostics.argtypes = [vp, ctypes.c_double, ctypes.c_double, ctypes.c_int, dp, dp]
    L.envpic_bunch_fields.argtypes = [vp, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_double, ctypes.c_double,
                                      ctypes.c_int, ctypes.POINTER(ctypes.c_int), dp]
    L.envpic_set_timing.argtypes = [vp, ctypes.c_int]
    L.envpic_set_graph.argtypes = [vp, ctypes.c_int]
    L.envpic_get_timing.argtypes = [vp, dp, i64p]
    L.envpic_save.argtypes = [vp, vp, ctypes.POINTER(ctypes.c_size_t)]
    L.envpic_load.argtypes = [vp, vp, ctypes.c_size_t]
    L.envpic_debug_poison.argtypes = [vp, ctypes.c_int]
    L.envpic_sim_destroy.argtypes = [vp]
    L.envpic_stream_copy.argtypes = [vp, vp, ctypes.c_size_t, ctypes.c_int, vp]
    L.envpic_sim_destroy.restype = None
    L.envpic_last_error.argtypes = [vp]
    L.envpic_last_error.restype = ctypes.c_char_p
    _lib = L
    return L


def _check(rc):
    if rc != 0:
        raise EnvpicError(rc, lib().envpic_last_error(None).decode())
    return rc


def _dptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def params_default(preset=0):
    p = Params()
    lib().envpic_params_default(ctypes.byref(p), int(preset))
    return p


def make_params(cfg):
    """Params from a workload dictionary (keys as in the parameter block)."""
    p = params_default(0)
    p.nx, p.nr = int(cfg["nx"]), int(cfg["nr"])
    p.n_modes = int(cfg.get("n_modes", 1))
    p.ppc_x, p.ppc_r, p.ppc_t = (int(v) for v in cfg.get("ppc", (2, 2, 1)))
    p.profile = PROFILES[cfg.get("profile", "uniform")]
    p.moving_window = int(cfg.get("moving_window", 0))
    p.seed = int(cfg.get("seed", 191204674))
    p.dx, p.dr, p.dt = float(cfg["dx"]), float(cfg["dr"]), float(cfg["dt"])
    p.a0, p.w0, p.tau = float(cfg.get("a0", 0.0)), float(cfg.get("w0", 1.0)), float(cfg.get("tau", 1.0))
    p.x_c, p.x_f = float(cfg.get("x_c", 0.0)), float(cfg.get("x_f", 0.0))
    p.n0 = float(cfg.get("n0", 0.0))
    p.ramp_len = float(cfg.get("ramp_len", 0.0))
    p.perturb = float(cfg.get("perturb", 0.0))
    p.bump_x = float(cfg.get("bump_x", 0.0))
    p.bump_w = float(cfg.get("bump_w", 1.0))
    p.capacity = int(cfg.get("capacity", 0))
    p.filter_passes = int(cfg.get("filter_passes", 0))
    p.shape_order = int(cfg.get("shape_order", 0))
    p.sort_every = int(cfg.get("sort_every", 0))
    return p


def footprint(cfg_or_params, precision=FP32_BULK):
    p = cfg_or_params if isinstance(cfg_or_params, Params) else make_params(cfg_or_params)
    n = ctypes.c_size_t()
    _check(lib().envpic_footprint(ctypes.byref(p), int(precision), ctypes.byref(n)))
    return n.value


class Sim:
    """One simulation resident in a caller-owned device arena."""

    def __init__(self, cfg, precision=FP32_BULK, arena=None, stream=None):
        import torch
        self.params = cfg if isinstance(cfg, Params) else make_params(cfg)
        self.nx, self.nr = self.params.nx, self.params.nr
        self.precision = precision
        need = footprint(self.params, precision)
        own = arena is None
        if own:
            arena = torch.empty(need, dtype=torch.uint8, device="cuda")
        self.arena = arena
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        if own and self.stream != torch.cuda.current_stream():
            # the caching allocator must not hand the block out again while
            # kernels queued on the simulation's stream may still use it
            arena.record_stream(self.stream)
        h = ctypes.c_void_p()
        _check(lib().envpic_sim_init(ctypes.byref(self.params), int(precision),
                                     ctypes.c_void_p(arena.data_ptr()), arena.numel() * arena.element_size(),
                                     ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h)))
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            lib().envpic_sim_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def handle(self):
        return self._h

    # stages
    def gather_push(self, stage, defer=False):
        _check(lib().envpic_gather_push(self._h, int(stage) | (DEFER_DEPOSIT if defer else 0)))

    def momentum(self, defer=False):
        self.gather_push(MOMENTUM, defer)

    def position(self, defer=False):
        self.gather_push(POSITION, defer)

    def envelope_step(self):
        _check(lib().envpic_envelope_step(self._h))

    def project_chi_J(self, what):
        _check(lib().envpic_project_chi_J(self._h, int(what)))

    def field_step(self):
        _check(lib().envpic_field_step(self._h))

    def step(self, nsteps=1):
        _check(lib().envpic_step_n(self._h, int(nsteps)))

    # state
    def state(self):
        n, s, npart = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        _check(lib().envpic_state(self._h, ctypes.byref(n), ctypes.byref(s), ctypes.byref(npart)))
        return n.value, s.value, npart.value

    def sort_stats(self):
        """How the particle sorts ran: {"cell": sorts that rebuilt the layout
        ordered by cell, "incremental": tile sorts that moved only the
        particles that changed tile, "rebuilt": tile sorts that found no room
        and rebuilt the layout, "gathered": cell sorts whose copy in cell
        order was gathered after the momentum pass}."""
        out = (ctypes.c_int64 * 4)()
        _check(lib().envpic_sort_stats(self._h, out))
        return {"cell": out[0], "incremental": out[1], "rebuilt": out[2], "gathered": out[3]}

    def get_field(self, name):
        shape = (self.nx + 1, self.nr + 1)
        cplx = name in COMPLEX_FIELDS
        buf = np.zeros(shape[0] * shape[1] * (2 if cplx else 1))
        _check(lib().envpic_get_field(self._h, FIELDS[name], _dptr(buf)))
        if cplx:
            return (buf[0::2] + 1j * buf[1::2]).reshape(shape)
        return buf.reshape(shape)

    def set_field(self, name, arr):
        shape = (self.nx + 1, self.nr + 1)
        arr = np.asarray(arr)
        assert arr.shape == shape, (arr.shape, shape)
        if name in COMPLEX_FIELDS:
            flat = arr.astype(np.complex128).ravel()
            buf = np.empty(2 * flat.size)
            buf[0::2], buf[1::2] = flat.real, flat.imag
        else:
            buf = np.ascontiguousarray(arr, dtype=np.float64).ravel()
        _check(lib().envpic_set_field(self._h, FIELDS[name], _dptr(buf)))

    def get_particles(self):
        npart = self.state()[2]
        out = {k: np.zeros(npart) for k in ("x", "y", "z", "px", "py", "pz", "w")}
        ids = np.zeros(npart, dtype=np.uint32)
        _check(lib().envpic_get_particles(self._h, *(_dptr(out[k]) for k in
                                                     ("x", "y", "z", "px", "py", "pz", "w")),
                                          ids.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32))))
        out["id"] = ids
        return out

    def set_particles(self, parts):
        n = len(parts["x"])
        arrs = [np.ascontiguousarray(parts[k], dtype=np.float64)
                for k in ("x", "y", "z", "px", "py", "pz", "w")]
        ids = np.ascontiguousarray(parts["id"], dtype=np.uint32)
        _check(lib().envpic_set_particles(self._h, n, *(_dptr(a) for a in arrs),
                                          ids.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32))))

    def set_graph(self, steps):
        """step() issues chunks of up to `steps` steps as one HIP graph each (0: off)."""
        _check(lib().envpic_set_graph(self._h, int(steps)))

    def set_timing(self, enable=True, every=1):
        """Record stage events on every `every`-th step (off if not enable)."""
        _check(lib().envpic_set_timing(self._h, int(every) if enable else 0))

    def timing(self):
        """Average ms per launch and launch counts of the momentum, envelope,
        position and field stages since timing was enabled."""
        ms = np.zeros(4)
        cnt = np.zeros(4, dtype=np.int64)
        _check(lib().envpic_get_timing(self._h, _dptr(ms), cnt.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))))
        names = ("momentum", "envelope", "position", "field")
        return {n: (float(ms[k]), int(cnt[k])) for k, n in enumerate(names)}

    def diagnostics(self):
        out = np.zeros(len(DIAG_NAMES))
        _check(lib().envpic_diagnostics(self._h, _dptr(out)))
        return dict(zip(DIAG_NAMES, out))

    def diagnostics_noalloc(self, out):
        """The diagnostics into the caller's device tensor `out` (9 float64),
        asynchronously on the simulation's stream, with no allocation (the
        library's static scratch holds the partial sums)."""
        import torch
        assert out.dtype == torch.float64 and out.is_cuda and out.numel() >= len(DIAG_NAMES)
        _check(lib().envpic_diagnostics_noalloc(self._h, ctypes.c_void_p(out.data_ptr())))
        return out

    def beam(self, e_lo, e_hi, nbins, with_hist=False):
        """Injected-beam parameters (dict of BEAM_NAMES), and the charge
        spectrum over [e_lo, e_hi) when with_hist."""
        out = np.zeros(len(BEAM_NAMES))
        hist = np.zeros(max(int(nbins), 1)) if with_hist else None
        _check(lib().envpic_beam_diagnostics(self._h, float(e_lo), float(e_hi), int(nbins), _dptr(out),
                                             _dptr(hist) if with_hist else None))
        res = dict(zip(BEAM_NAMES, out))
        return (res, hist) if with_hist else res

    def bunch_fields(self, id_lo, id_hi, beta, tol=1e-12, max_iter=50000):
        """Add the self-consistent fields of the bunch of particles with id in
        [id_lo, id_hi) moving at beta; returns (iterations, relative residual)."""
        it, res = ctypes.c_int(), ctypes.c_double()
        _check(lib().envpic_bunch_fields(self._h, int(id_lo), int(id_hi), float(beta), float(tol), int(max_iter),
                                         ctypes.byref(it), ctypes.byref(res)))
        return it.value, res.value

    def save(self):
        n = ctypes.c_size_t()
        _check(lib().envpic_save(self._h, None, ctypes.byref(n)))
        blob = (ctypes.c_char * n.value)()
        _check(lib().envpic_save(self._h, ctypes.cast(blob, ctypes.c_void_p), ctypes.byref(n)))
        return bytes(blob)

    def load(self, blob):
        buf = ctypes.create_string_buffer(blob, len(blob))
        _check(lib().envpic_load(self._h, ctypes.cast(buf, ctypes.c_void_p), len(blob)))

    def poison(self, name):
        _check(lib().envpic_debug_poison(self._h, FIELDS[name]))


def stream_copy(dst, src, variant=0, stream=None):
    """Plain streaming copy of the device tensor src into dst (same number of
    bytes) with the library's copy kernel, on `stream` (default: torch's
    current stream)."""
    import torch
    n = src.numel() * src.element_size()
    assert dst.numel() * dst.element_size() == n
    stream = stream if stream is not None else torch.cuda.current_stream()
    _check(lib().envpic_stream_copy(ctypes.c_void_p(dst.data_ptr()), ctypes.c_void_p(src.data_ptr()), n,
                                    int(variant), ctypes.c_void_p(stream.cuda_stream)))


def batch_step(sims, nsteps, stream=None):
    """Advance resident simulations together (their kernels overlap)."""
    import torch
    stream = stream if stream is not None else torch.cuda.current_stream()
    arr = (ctypes.c_void_p * len(sims))(*[s.handle for s in sims])
    _check(lib().envpic_batch_step(arr, len(sims), int(nsteps), ctypes.c_void_p(stream.cuda_stream)))
