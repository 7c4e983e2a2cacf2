"""Parity of the injected-bunch field initialisation (R27) of the HIP path,
through the C ABI, with the oracle's direct solve (oracle/bunch.py), and the
discrete Gauss law of its result at the full 2048 x 256 LWFA size.

Bars: FP64 fields 1e-9 of each field's maximum (conjugate gradients to a
relative residual of 1e-13 against a direct solve), FP32 fields 1e-6 (the
grids are FP32); the run that follows, at the usual loop bars.
"""
import time

import numpy as np
import pytest

from inputs import C2, bunch_particles
from test_gpu_parity import compare_fields, compare_particles, ferr, say, staggered

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def E():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1912_04674_amd as E
    E.lib()
    return E


@pytest.fixture(scope="module")
def bunch_mod():
    from oracle import bunch
    return bunch


def _prec(E, name):
    return E.FP64 if name == "fp64" else E.FP32_BULK


def _subset(parts, lo, hi):
    m = (parts["id"] >= lo) & (parts["id"] < hi)
    return {k: v[m] for k, v in parts.items()}


BETA = 0.99
GAMMA = 1.0 / np.sqrt(1.0 - BETA * BETA)


@pytest.mark.parametrize("order", [1, 2])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_bunch_fields_match_direct_solve(E, bunch_mod, prec, order):
    cfg = dict(nx=96, nr=24, dx=0.8, dr=1.5, dt=0.6, n_modes=2, profile="none", a0=0.0, ppc=(1, 1, 1),
               shape_order=order, capacity=20000)
    say("bunch solve", prec, "order", order)
    g = E.Sim(cfg, _prec(E, prec))
    g.set_particles(bunch_particles(5000, 8, x0=38.0, sig_x=5.0, sig_r=2.5, p0=GAMMA * BETA, w_total=0.5))
    it, res = g.bunch_fields(0, 5000, BETA, tol=1e-13)
    say("iterations", it, "residual", res)
    assert 0 < it and res <= 1e-13
    ex, er, bt, phi, qv = bunch_mod.bunch_fields(cfg, g.get_particles(), BETA)
    tol = 1e-9 if prec == "fp64" else 1e-6
    for name, ref in (("ex", ex), ("er", er), ("bt", bt), ("bt_bar", bt)):
        e = ferr(staggered(name, g.get_field(name)), ref)
        say("field", name, f"{e:.2e}")
        assert e <= tol, (name, e)
    for name in ("ex1", "er1", "bt1"):  # mode 1 untouched
        assert np.abs(g.get_field(name)).max() == 0.0


def test_bunch_fields_arguments_and_empty_range(E):
    cfg = dict(nx=48, nr=12, dx=0.8, dr=1.5, dt=0.6, n_modes=1, profile="none", a0=0.0, ppc=(1, 1, 1),
               capacity=4000)
    g = E.Sim(cfg, E.FP32_BULK)
    g.set_particles(bunch_particles(500, 9, x0=19.0, sig_x=3.0, sig_r=2.0, p0=3.0))
    for bad in [dict(beta=1.0), dict(beta=-0.1), dict(tol=0.0), dict(max_iter=0), dict(id_lo=5, id_hi=5)]:
        kw = dict(id_lo=0, id_hi=500, beta=0.9, tol=1e-10, max_iter=100)
        kw.update(bad)
        with pytest.raises(E.EnvpicError) as ei:
            g.bunch_fields(**kw)
        assert ei.value.code == -1, bad
    it, res = g.bunch_fields(1000, 2000, 0.9)  # no particle in the range: nothing added
    assert it == 0 and np.abs(g.get_field("ex")).max() == 0.0
    with pytest.raises(E.EnvpicError) as ei:  # far too few iterations
        g.bunch_fields(0, 500, 0.9, tol=1e-14, max_iter=2)
    assert ei.value.code == -5
    g.momentum()
    with pytest.raises(E.EnvpicError) as ei:
        g.bunch_fields(0, 500, 0.9)
    assert ei.value.code == -3


@pytest.mark.parametrize("prec,tf,tp", [("fp64", 1e-9, 1e-9), ("fp32", 1e-4, 1e-3)])
def test_bunch_in_plasma_run_parity(E, oracle_mod, bunch_mod, prec, tf, tp):
    """A relativistic bunch entering a uniform plasma behind a laser pulse:
    bunch fields initialised on both sides, then 40 steps of the loop
    (modes 0 and 1, quadratic shapes)."""
    cfg = dict(nx=160, nr=32, dx=0.8, dr=1.5, dt=0.6, n_modes=2, profile="uniform", n0=0.003, ppc=(2, 2, 2),
               a0=1.5, w0=10.0, tau=12.0, x_c=100.0, x_f=100.0, shape_order=2, seed=191204690,
               capacity=160 * 32 * 8 + 20000)
    say("bunch in plasma", prec)
    g = E.Sim(cfg, _prec(E, prec))
    r = oracle_mod.OracleSim(cfg)
    plasma = r.get_particles()
    nb = 4000
    b = bunch_particles(nb, 10, x0=40.0, sig_x=4.0, sig_r=1.5, p0=GAMMA * BETA, w_total=0.05, id0=1 << 24)
    parts = {k: np.concatenate([plasma[k], b[k]]) for k in plasma}
    g.set_particles(parts)
    r.set_particles(parts)
    it, res = g.bunch_fields(1 << 24, (1 << 24) + nb, BETA, tol=1e-13)
    say("iterations", it, "residual", res)
    ex, er, bt, _, _ = bunch_mod.bunch_fields(cfg, _subset(r.get_particles(), 1 << 24, (1 << 24) + nb), BETA)
    r.set_field("ex", ex)
    r.set_field("er", er)
    r.set_field("bt", bt)
    r.set_field("bt_bar", bt)
    compare_fields(g, r, tf if prec == "fp32" else 1e-9, names=("ex", "er", "bt", "bt_bar"))
    g.step(40)
    r.step(40)
    compare_fields(g, r, tf, modes=2)
    compare_particles(g.get_particles(), r.get_particles(), tp, 1e-8 if prec == "fp64" else 1e-3)


def test_full_size_bunch_gauss_law(E):
    """The 2048 x 256 LWFA workload (8.4 M plasma particles) plus a 200 000-
    particle bunch behind the pulse: the solve on 524 032 unknowns, then the
    discrete Gauss law V div E = q sum w S (this file's own linear deposit of
    the bunch, the field update's divergence) at every interior node."""
    cfg = dict(C2, capacity=9_000_000)
    g = E.Sim(cfg, E.FP32_BULK)
    plasma = g.get_particles()
    dx, dr = cfg["dx"], cfg["dr"]
    nb = 200_000
    x0 = (cfg["nx"] - 600) * dx
    b = bunch_particles(nb, 11, x0=x0, sig_x=8.0, sig_r=3.0, p0=GAMMA * BETA, w_total=20.0, id0=1 << 26)
    g.set_particles({k: np.concatenate([plasma[k], b[k]]) for k in plasma})
    t0 = time.perf_counter()
    it, res = g.bunch_fields(1 << 26, (1 << 26) + nb, BETA, tol=1e-12)
    dt = time.perf_counter() - t0
    say("full size solve", it, "iterations", f"{res:.1e}", f"{dt * 1e3:.1f} ms")
    bp = _subset(g.get_particles(), 1 << 26, (1 << 26) + nb)
    nx, nr = cfg["nx"], cfg["nr"]
    ux, ur = bp["x"] / dx - g.state()[1], np.hypot(bp["y"], bp["z"]) / dr
    i0, j0 = np.floor(ux).astype(int), np.floor(ur).astype(int)
    fx, fr = ux - i0, ur - j0
    qv = np.zeros((nx + 2, nr + 2))
    for a, wa in ((0, 1 - fx), (1, fx)):
        for c, wc in ((0, 1 - fr), (1, fr)):
            np.add.at(qv, (i0 + a, j0 + c), -bp["w"] * wa * wc)
    qv = qv[: nx + 1, : nr + 1]
    ex, er = g.get_field("ex"), g.get_field("er")
    j = np.arange(nr + 1)
    V = np.where(j == 0, np.pi * dr * dr * dx / 4, 2 * np.pi * j * dr * dr * dx)
    A = 2 * np.pi * (j + 0.5) * dr * dx
    dv = np.zeros_like(ex)
    dv[1:, :] += V[None, :] * (ex[1:, :] - ex[:-1, :]) / dx
    flux = A[None, :] * er
    dv[:, 0] += flux[:, 0]
    dv[:, 1:] += flux[:, 1:] - flux[:, :-1]
    sl = (slice(1, nx), slice(0, nr))
    err = np.abs(dv - qv)[sl].max() / np.abs(qv).max()
    say("Gauss law error", f"{err:.2e}", "max |E_r|", np.abs(er).max())
    assert err < 1e-4
    assert np.abs(er).max() > 0
