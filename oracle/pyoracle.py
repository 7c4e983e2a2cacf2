"""ctypes binding of the FP64 CPU oracle (oracle/oracle.h).

TEST INFRASTRUCTURE ONLY: imported by the test suite, the smoke check and the
CPU-baseline leg of the benchmark.  It does not import the GPU package and the
GPU package does not import it.  Marshalling only: every stage of the method
runs in oracle.cpp.
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liboracle.so")

PARAMS_VERSION = 2

PROFILES = {"none": 0, "uniform": 1, "ramp": 2, "perturb": 3, "bump": 4}

FIELDS = {
    "env": 0, "env_prev": 1, "chi": 2, "ex": 3, "er": 4, "bt": 5, "bt_bar": 6,
    "jx": 7, "jr": 8, "ex1": 9, "er1": 10, "et1": 11, "bx1": 12, "br1": 13,
    "bt1": 14, "bx1_bar": 15, "br1_bar": 16, "bt1_bar": 17, "jx1": 18,
    "jr1": 19, "jt1": 20,
}
COMPLEX_FIELDS = {"env", "env_prev", "ex1", "er1", "et1", "bx1", "br1", "bt1",
                  "bx1_bar", "br1_bar", "bt1_bar", "jx1", "jr1", "jt1"}
DIAG_NAMES = ["count", "charge", "chi_v", "kin", "uem", "env2_v", "lx", "px",
              "nonfinite"]


class OracleParams(ctypes.Structure):
    _fields_ = [
        ("size", ctypes.c_int32), ("version", ctypes.c_int32),
        ("nx", ctypes.c_int32), ("nr", ctypes.c_int32),
        ("n_modes", ctypes.c_int32),
        ("ppc_x", ctypes.c_int32), ("ppc_r", ctypes.c_int32), ("ppc_t", ctypes.c_int32),
        ("profile", ctypes.c_int32), ("moving_window", ctypes.c_int32),
        ("env_bc_x", ctypes.c_int32), ("env_bc_r", ctypes.c_int32),
        ("seed", ctypes.c_uint64),
        ("dx", ctypes.c_double), ("dr", ctypes.c_double), ("dt", ctypes.c_double),
        ("a0", ctypes.c_double), ("w0", ctypes.c_double), ("tau", ctypes.c_double),
        ("x_c", ctypes.c_double), ("x_f", ctypes.c_double),
        ("n0", ctypes.c_double), ("ramp_len", ctypes.c_double),
        ("perturb", ctypes.c_double), ("bump_x", ctypes.c_double),
        ("bump_w", ctypes.c_double),
        ("start_col", ctypes.c_int64),
        ("filter_passes", ctypes.c_int32), ("shape_order", ctypes.c_int32),
    ]


def build(force=False):
    """Compile liboracle.so with g++ (-O2, no fast-math)."""
    src = os.path.join(_HERE, "oracle.cpp")
    if force or not os.path.exists(LIB_PATH) or os.path.getmtime(LIB_PATH) < max(
            os.path.getmtime(src), os.path.getmtime(os.path.join(_HERE, "oracle.h"))):
        subprocess.check_call(["g++", "-std=c++17", "-O2", "-fPIC", "-shared", "-Wall", "-pthread",
                               "-o", LIB_PATH, src])
    return LIB_PATH


_libs = {}


def lib(path=None):
    """The loaded oracle library (by default liboracle.so next to this file;
    `path` loads another build of the same source, e.g. a planted-mistake
    variant made by build_variant)."""
    path = path or LIB_PATH
    if path not in _libs:
        if path == LIB_PATH and not os.path.exists(LIB_PATH):
            build()
        L = ctypes.CDLL(path)
        vp = ctypes.c_void_p
        dp = ctypes.POINTER(ctypes.c_double)
        up = ctypes.POINTER(ctypes.c_uint32)
        i64p = ctypes.POINTER(ctypes.c_int64)
        L.oracle_create.argtypes = [ctypes.POINTER(OracleParams), ctypes.POINTER(vp)]
        L.oracle_destroy.argtypes = [vp]
        L.oracle_destroy.restype = None
        for name in ("oracle_momentum_chi", "oracle_envelope", "oracle_position_J",
                     "oracle_field_step", "oracle_filter_J"):
            getattr(L, name).argtypes = [vp]
        L.oracle_step.argtypes = [vp, ctypes.c_int]
        L.oracle_state.argtypes = [vp, i64p, i64p, i64p]
        L.oracle_get_particles.argtypes = [vp] + [dp] * 7 + [up]
        L.oracle_set_particles.argtypes = [vp, ctypes.c_int64] + [dp] * 7 + [up]
        L.oracle_get_gbar.argtypes = [vp, dp]
        L.oracle_get_field.argtypes = [vp, ctypes.c_int, dp]
        L.oracle_set_field.argtypes = [vp, ctypes.c_int, dp]
        L.oracle_diagnostics.argtypes = [vp, dp]
        L.oracle_uniform.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int64,
                                     ctypes.c_int64]
        L.oracle_uniform.restype = ctypes.c_double
        L.oracle_set_threads.argtypes = [ctypes.c_int]
        _libs[path] = L
    return _libs[path]


def build_variant(edits, workdir):
    """Compile a copy of oracle.cpp with textual edits [(old, new), ...] into
    `workdir` and return the library path.  Used only to show that the pins
    catch planted mistakes; every `old` must occur exactly once."""
    src = open(os.path.join(_HERE, "oracle.cpp")).read()
    for old, new in edits:
        assert src.count(old) == 1, f"edit target not unique: {old!r}"
        src = src.replace(old, new)
    os.makedirs(workdir, exist_ok=True)
    cpp = os.path.join(workdir, "oracle.cpp")
    with open(cpp, "w") as f:
        f.write(src)
    out = os.path.join(workdir, "liboracle.so")
    subprocess.check_call(["g++", "-std=c++17", "-O2", "-fPIC", "-shared", "-pthread", "-I", _HERE,
                           "-o", out, cpp])
    return out


class Variant:
    """Module-like view of another oracle build (same interface as this
    module's OracleSim and uniform)."""

    def __init__(self, path):
        self.path = path

    def OracleSim(self, cfg):
        return OracleSim(cfg, lib_path=self.path)

    def uniform(self, seed, stream, col, j):
        return lib(self.path).oracle_uniform(seed, stream, col, j)


def _dptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def make_params(cfg):
    """OracleParams from a plain workload dictionary (see tests/inputs.py)."""
    p = OracleParams()
    p.size = ctypes.sizeof(OracleParams)
    p.version = PARAMS_VERSION
    p.nx, p.nr = int(cfg["nx"]), int(cfg["nr"])
    p.n_modes = int(cfg.get("n_modes", 1))
    p.ppc_x, p.ppc_r, p.ppc_t = (int(v) for v in cfg.get("ppc", (2, 2, 1)))
    p.profile = PROFILES[cfg.get("profile", "uniform")]
    p.moving_window = int(cfg.get("moving_window", 0))
    p.env_bc_x = int(cfg.get("env_bc_x", 0))
    p.env_bc_r = int(cfg.get("env_bc_r", 0))
    p.seed = int(cfg.get("seed", 191204674))
    p.dx, p.dr, p.dt = float(cfg["dx"]), float(cfg["dr"]), float(cfg["dt"])
    p.a0, p.w0, p.tau = float(cfg.get("a0", 0.0)), float(cfg.get("w0", 1.0)), float(cfg.get("tau", 1.0))
    p.x_c, p.x_f = float(cfg.get("x_c", 0.0)), float(cfg.get("x_f", 0.0))
    p.n0 = float(cfg.get("n0", 0.0))
    p.ramp_len = float(cfg.get("ramp_len", 0.0))
    p.perturb = float(cfg.get("perturb", 0.0))
    p.bump_x = float(cfg.get("bump_x", 0.0))
    p.bump_w = float(cfg.get("bump_w", 1.0))
    p.start_col = int(cfg.get("start_col", 0))
    p.filter_passes = int(cfg.get("filter_passes", 0))
    p.shape_order = int(cfg.get("shape_order", 1))
    return p


class OracleSim:
    """One oracle simulation (host memory)."""

    def __init__(self, cfg, lib_path=None):
        self._L = lib(lib_path)
        self.cfg = dict(cfg)
        self.nx, self.nr = int(cfg["nx"]), int(cfg["nr"])
        self._p = make_params(cfg)
        h = ctypes.c_void_p()
        rc = self._L.oracle_create(ctypes.byref(self._p), ctypes.byref(h))
        if rc != 0:
            raise ValueError(f"oracle_create failed ({rc}) for {cfg}")
        self._h = h

    def close(self):
        if self._h:
            self._L.oracle_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # stages
    def momentum_chi(self):
        self._L.oracle_momentum_chi(self._h)

    def envelope(self):
        self._L.oracle_envelope(self._h)

    def position_J(self):
        self._L.oracle_position_J(self._h)

    def field_step(self):
        self._L.oracle_field_step(self._h)

    def filter_J(self):
        self._L.oracle_filter_J(self._h)

    def step(self, n=1):
        self._L.oracle_step(self._h, int(n))

    # state
    def state(self):
        n, s, npart = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        self._L.oracle_state(self._h, ctypes.byref(n), ctypes.byref(s), ctypes.byref(npart))
        return n.value, s.value, npart.value

    @property
    def n_particles(self):
        return self.state()[2]

    def get_particles(self):
        npart = self.n_particles
        out = {k: np.zeros(npart) for k in ("x", "y", "z", "px", "py", "pz", "w")}
        ids = np.zeros(npart, dtype=np.uint32)
        self._L.oracle_get_particles(self._h, *(_dptr(out[k]) for k in
                                              ("x", "y", "z", "px", "py", "pz", "w")),
                                   ids.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)))
        out["id"] = ids
        return out

    def set_particles(self, parts):
        n = len(parts["x"])
        arrs = [np.ascontiguousarray(parts[k], dtype=np.float64)
                for k in ("x", "y", "z", "px", "py", "pz", "w")]
        ids = np.ascontiguousarray(parts["id"], dtype=np.uint32)
        rc = self._L.oracle_set_particles(self._h, n, *(_dptr(a) for a in arrs),
                                        ids.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)))
        if rc != 0:
            raise ValueError("oracle_set_particles failed")

    def get_gbar(self):
        g = np.zeros(self.n_particles)
        self._L.oracle_get_gbar(self._h, _dptr(g))
        return g

    def get_field(self, name):
        shape = (self.nx + 1, self.nr + 1)
        if name in COMPLEX_FIELDS:
            buf = np.zeros(2 * shape[0] * shape[1])
            rc = self._L.oracle_get_field(self._h, FIELDS[name], _dptr(buf))
            if rc != 0:
                raise ValueError(f"field {name} unavailable")
            return (buf[0::2] + 1j * buf[1::2]).reshape(shape)
        buf = np.zeros(shape[0] * shape[1])
        rc = self._L.oracle_get_field(self._h, FIELDS[name], _dptr(buf))
        if rc != 0:
            raise ValueError(f"field {name} unavailable")
        return buf.reshape(shape)

    def set_field(self, name, arr):
        shape = (self.nx + 1, self.nr + 1)
        arr = np.asarray(arr)
        assert arr.shape == shape, (arr.shape, shape)
        if name in COMPLEX_FIELDS:
            buf = np.empty(2 * arr.size)
            flat = arr.astype(np.complex128).ravel()
            buf[0::2], buf[1::2] = flat.real, flat.imag
        else:
            buf = np.ascontiguousarray(arr, dtype=np.float64).ravel()
        rc = self._L.oracle_set_field(self._h, FIELDS[name], _dptr(buf))
        if rc != 0:
            raise ValueError(f"field {name} unavailable")

    def diagnostics(self):
        out = np.zeros(len(DIAG_NAMES))
        self._L.oracle_diagnostics(self._h, _dptr(out))
        return dict(zip(DIAG_NAMES, out))


def uniform(seed, stream, col, j):
    return lib().oracle_uniform(seed, stream, col, j)


def set_threads(n):
    """Threads of the oracle's particle loops (process-wide; 1 is the plain
    serial loop).  Results are identical for a given count."""
    if lib().oracle_set_threads(int(n)) != 0:
        raise ValueError(f"bad thread count {n}")


def host_threads(cap=16):
    """The CPUs this process may run on, at most `cap`."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(cap, n))
