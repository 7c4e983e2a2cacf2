"""Workload definitions and seeded input generators.

Shared by the GPU-path tests and the oracle tests (and the benchmark).  This
module holds configuration numbers and random-number draws only: none of the
method's arithmetic lives here.

Workloads are synthetic stand-ins for the laser-wakefield set-ups of the
paper's benchmarks (Sec. 4): a Gaussian envelope in vacuum or in a cold
electron plasma on an (x, r) grid, cell sizes dx = 0.8, dr = 1.5 (c/w0) and
dt = 0.75 dx.  Units are normalized as in Sec. 2.
"""
import numpy as np

BASE_SEED = 191204674

_COMMON = dict(dx=0.8, dr=1.5, dt=0.6)


def _cfg(**kw):
    c = dict(_COMMON)
    c.update(kw)
    return c


# C1: mode-0 parity case, 256 x 32 cells, 2x2x1 particles per cell (32768),
# uniform n = 0.002, a0 = 1, w0 = 20, tau = 30 centred in the box, 100 steps.
C1 = _cfg(name="c1_parity_256x32", nx=256, nr=32, n_modes=1, ppc=(2, 2, 1),
          profile="uniform", n0=0.002, a0=1.0, w0=20.0, tau=30.0,
          x_c=102.4, x_f=102.4, moving_window=0, seed=BASE_SEED + 1, steps=100)

# C2: LWFA-shaped run, 2048 x 256, modes 0 and 1, 2x2x4 (8.4 M particles),
# n0 = 0.0017 with a linear up-ramp over 200, a0 = 2, w0 = 100, tau = 60,
# moving window, 1000 steps.
C2 = _cfg(name="c2_lwfa_2048x256", nx=2048, nr=256, n_modes=2, ppc=(2, 2, 4),
          profile="ramp", n0=0.0017, ramp_len=200.0, a0=2.0, w0=100.0, tau=60.0,
          x_c=2048 * 0.8 - 180.0, x_f=2048 * 0.8 - 180.0, moving_window=1,
          seed=BASE_SEED + 2, steps=1000)

# C3: bandwidth case, 4096 x 512, modes 0 and 1, 2x2x4 (33.5 M particles),
# n = 0.001 (1 +- 1 % per cell), a0 = 2.5, w0 = 150, tau = 80, 500 steps,
# particle sort every step.
C3 = _cfg(name="c3_bandwidth_4096x512", nx=4096, nr=512, n_modes=2, ppc=(2, 2, 4),
          profile="perturb", n0=0.001, perturb=0.01, a0=2.5, w0=150.0, tau=80.0,
          x_c=4096 * 0.8 / 2, x_f=4096 * 0.8 / 2, moving_window=0, sort_every=1,
          seed=BASE_SEED + 3, steps=500)

# C5: scale case, 8192 x 768, modes 0 and 1, 2x2x6 (151 M particles),
# n0 = 0.0015 plateau with a Gaussian bump entering through injection,
# a0 = 3, w0 = 200, tau = 90, moving window, 2000 steps.
C5 = _cfg(name="c5_extreme_8192x768", nx=8192, nr=768, n_modes=2, ppc=(2, 2, 6),
          profile="bump", n0=0.0015, bump_x=8192 * 0.8 + 400.0, bump_w=100.0,
          a0=3.0, w0=200.0, tau=90.0, x_c=8192 * 0.8 - 270.0, x_f=8192 * 0.8 - 270.0,
          moving_window=1, seed=BASE_SEED + 5, steps=2000)

CONFIGS = {"C1": C1, "C2": C2, "C3": C3, "C5": C5}

# a small window of the LWFA shape (host-side checks of the parameter block)
C2_SMALL_LIKE = _cfg(name="c2_small_like", nx=192, nr=48, n_modes=2, ppc=(2, 2, 4), profile="ramp",
                     n0=0.004, ramp_len=40.0, a0=2.0, w0=20.0, tau=15.0, x_c=108.6, x_f=108.6,
                     moving_window=1, seed=BASE_SEED + 6)

# C4: serving scan -- 64 jobs, Poisson arrivals at 4 jobs/s, grids drawn
# from {512x64, 1024x128, 2048x256}, mode 0, 2x2x2 particles per cell,
# n ~ U[0.001, 0.004], a0 ~ U[0.5, 3], w0 ~ U[40, 120], tau = 30, window on,
# 300 steps each.
C4_GRIDS = [(512, 64), (1024, 128), (2048, 256)]


def c4_job(j, rng):
    nx, nr = C4_GRIDS[int(rng.integers(0, 3))]
    lx = nx * 0.8
    return _cfg(name=f"c4_job{j}_{nx}x{nr}", nx=nx, nr=nr, n_modes=1, ppc=(2, 2, 2),
                profile="uniform", n0=float(rng.uniform(0.001, 0.004)),
                a0=float(rng.uniform(0.5, 3.0)), w0=float(rng.uniform(40.0, 120.0)),
                tau=30.0, x_c=lx - 90.0, x_f=lx - 90.0, moving_window=1,
                seed=BASE_SEED + 100 + j, steps=300)


def c4_trace(n_jobs=64, rate=4.0, seed=BASE_SEED + 99):
    """Job list and Poisson arrival times (exponential gaps, mean 1/rate)."""
    rng = np.random.default_rng(seed)
    jobs = [c4_job(j, rng) for j in range(n_jobs)]
    gaps = rng.exponential(1.0 / rate, size=n_jobs)
    arrivals = np.cumsum(gaps) - gaps[0]
    return jobs, arrivals


def scaled(cfg, **kw):
    c = dict(cfg)
    c.update(kw)
    return c


# ---------------------------------------------------------------- states --
def random_particles(cfg, n, seed, margin=2.0, pmax=0.5, r_frac=0.95):
    """n particles uniformly inside the window (x in [margin, Lx - margin] cells,
    r up to r_frac r_max) with uniform random momenta in [-pmax, pmax]^3 and
    positive weights.  Lab-frame Cartesian FP64 arrays plus ids."""
    rng = np.random.default_rng(seed)
    dx, dr = cfg["dx"], cfg["dr"]
    nx, nr = cfg["nx"], cfg["nr"]
    x = rng.uniform(margin * dx, (nx - margin) * dx, n)
    r = r_frac * nr * dr * np.sqrt(rng.uniform(0.0, 1.0, n))
    th = rng.uniform(0.0, 2 * np.pi, n)
    return dict(
        x=x, y=r * np.cos(th), z=r * np.sin(th),
        px=rng.uniform(-pmax, pmax, n), py=rng.uniform(-pmax, pmax, n),
        pz=rng.uniform(-pmax, pmax, n),
        w=rng.uniform(0.5, 1.5, n) * 1e-3, id=np.arange(n, dtype=np.uint32))


def random_grid(cfg, seed, amp=1.0, complex_=False):
    """Smooth random (nx+1) x (nr+1) grid: a few random Fourier modes."""
    rng = np.random.default_rng(seed)
    nx, nr = cfg["nx"], cfg["nr"]
    i = np.arange(nx + 1)[:, None] / nx
    j = np.arange(nr + 1)[None, :] / nr
    out = np.zeros((nx + 1, nr + 1), dtype=np.complex128 if complex_ else np.float64)
    for _ in range(4):
        kx, kr = rng.uniform(0.5, 4.0, 2)
        ph = rng.uniform(0, 2 * np.pi, 2)
        a = rng.normal() + (1j * rng.normal() if complex_ else 0.0)
        out = out + a * np.cos(2 * np.pi * kx * i + ph[0]) * np.cos(2 * np.pi * kr * j + ph[1])
    return amp * out / 4.0


def beam_particles(cfg, n_bulk, n_beam, seed, p_beam=400.0, dp_beam=8.0, sig_r=2.0):
    """A cold bulk plasma near rest plus an accelerated electron bunch, as
    after self-injection: the bunch has p_x ~ N(p_beam, dp_beam), transverse
    positions ~ N(0, sig_r) and transverse momenta correlated with them, and
    a low-energy tail (a fifth of the bunch with p_x ~ U[20, p_beam]).
    Lab-frame Cartesian FP64 arrays plus ids; all inside the window."""
    rng = np.random.default_rng(seed)
    dx, dr = cfg["dx"], cfg["dr"]
    nx, nr = cfg["nx"], cfg["nr"]
    bulk = random_particles(cfg, n_bulk, seed + 1, margin=4.0, pmax=0.05)
    x = rng.uniform(0.3 * nx * dx, 0.5 * nx * dx, n_beam)
    y = np.clip(rng.normal(0.0, sig_r, n_beam), -0.3 * nr * dr, 0.3 * nr * dr)
    z = np.clip(rng.normal(0.0, sig_r, n_beam), -0.3 * nr * dr, 0.3 * nr * dr)
    px = rng.normal(p_beam, dp_beam, n_beam)
    tail = rng.uniform(0.0, 1.0, n_beam) < 0.2
    px[tail] = rng.uniform(20.0, p_beam, int(tail.sum()))
    py = 0.5 * y + rng.normal(0.0, 1.0, n_beam)
    pz = -0.3 * z + rng.normal(0.0, 0.7, n_beam)
    w = rng.uniform(0.2, 1.0, n_beam) * 1e-3
    ids = np.arange(n_bulk, n_bulk + n_beam, dtype=np.uint32)
    return {k: np.concatenate([bulk[k], v]) for k, v in
            dict(x=x, y=y, z=z, px=px, py=py, pz=pz, w=w, id=ids).items()}


def bunch_particles(n, seed, x0, sig_x, sig_r, p0, w_total=1.0, id0=0, r_cut=4.0):
    """An externally injected electron bunch: Gaussian in x (centre x0, rms
    sig_x) and in each transverse coordinate (rms sig_r, cut at r_cut sig_r
    from the axis), momentum p0 along x, equal weights summing to w_total.
    Lab-frame Cartesian FP64 arrays plus ids."""
    rng = np.random.default_rng(seed)
    x = rng.normal(x0, sig_x, n)
    y = rng.normal(0.0, sig_r, n)
    z = rng.normal(0.0, sig_r, n)
    r = np.hypot(y, z)
    scale = np.where(r > r_cut * sig_r, r_cut * sig_r / np.maximum(r, 1e-300), 1.0)
    return dict(x=x, y=y * scale, z=z * scale, px=np.full(n, p0), py=np.zeros(n), pz=np.zeros(n),
                w=np.full(n, w_total / n), id=np.arange(id0, id0 + n, dtype=np.uint32))
