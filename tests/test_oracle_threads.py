"""The oracle's threaded particle loops: each thread deposits into grids of
its own, added in thread order, so a run is reproducible for a given thread
count and differs from the one-thread run only by the order of the deposit
sums (round-off)."""
import numpy as np
import pytest

from inputs import scaled

CFG = dict(name="threads", nx=96, nr=32, dx=0.8, dr=1.5, dt=0.6, n_modes=2, ppc=(2, 2, 2),
           profile="ramp", n0=0.004, ramp_len=30.0, a0=2.0, w0=15.0, tau=15.0,
           x_c=96 * 0.8 - 35.0, x_f=96 * 0.8 - 35.0, moving_window=1, seed=191204690)
NAMES = ("env", "chi", "ex", "er", "bt", "jx", "jr", "ex1", "er1", "jx1", "jr1", "jt1")
# mode-1 grids of a theta-symmetric loading are round-off: scaled by mode 0
SCALE = {"ex1": "ex", "er1": "er", "jx1": "jx", "jr1": "jr", "jt1": "jr"}


def _run(oracle_mod, threads, cfg, steps=30):
    oracle_mod.set_threads(threads)
    try:
        s = oracle_mod.OracleSim(cfg)
        s.step(steps)
        return {n: s.get_field(n) for n in NAMES}, s.get_particles()
    finally:
        oracle_mod.set_threads(1)


@pytest.mark.parametrize("order", [1, 2])
def test_thread_counts_agree(oracle_mod, order):
    cfg = scaled(CFG, shape_order=order)
    f1, p1 = _run(oracle_mod, 1, cfg)
    f5, p5 = _run(oracle_mod, 5, cfg)
    f5b, p5b = _run(oracle_mod, 5, cfg)
    for n in NAMES:
        assert np.array_equal(f5[n], f5b[n]), n  # reproducible for a given count
        ref = np.abs(f1[SCALE.get(n, n)]).max()
        assert np.abs(f5[n] - f1[n]).max() <= 1e-11 * ref, n
    assert np.array_equal(p1["id"], p5["id"])
    for k in ("x", "y", "z", "px", "py", "pz"):
        assert np.array_equal(p5[k], p5b[k])
        assert np.abs(p5[k] - p1[k]).max() <= 1e-10 * max(np.abs(p1[k]).max(), 1.0), k


def test_thread_count_is_validated(oracle_mod):
    with pytest.raises(ValueError):
        oracle_mod.set_threads(0)
