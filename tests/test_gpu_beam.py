"""Parity of the injected-beam parameters (Table BeamParams, Sec. 4) of the
HIP path, through the C ABI, with the FP64 oracle (oracle/beam.py).

Both sides read the same particle values: the oracle takes the particles the
GPU simulation holds (envpic_get_particles, FP64 on the host), so every
selection decision (energy bin, window) is taken on identical inputs in FP64.
Bars: histogram 1e-10 of its maximum (the GPU sums 64-bit fixed point with a
per-particle quantum of about 2^-35 of the largest weight), outputs 1e-9
relative (FP64 sums in a different order), counts exact.
"""
import sys

import numpy as np
import pytest

from inputs import C2, beam_particles

pytestmark = pytest.mark.gpu

NAMES = ["e_peak", "fwhm", "charge", "e_mean", "e_rms", "rel_spread", "emit_y", "emit_z", "count",
         "charge_spectrum", "win_lo", "win_hi"]


def say(*a):
    print("[gpu]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def E():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1912_04674_amd as E
    E.lib()
    return E


@pytest.fixture(scope="module")
def beam_mod():
    from oracle import beam
    return beam


def check(gpu_out, gpu_hist, ref_out, ref_hist, tol=1e-9):
    hmax = np.abs(ref_hist).max()
    if hmax > 0:
        herr = float(np.abs(gpu_hist - ref_hist).max() / hmax)
    else:
        herr = float(np.abs(gpu_hist).max())
    say("hist err", f"{herr:.1e}", "peak", ref_out["e_peak"], "count", ref_out["count"])
    assert herr <= 1e-10, herr
    for k in NAMES:
        a, b = gpu_out[k], ref_out[k]
        if k == "count":
            assert a == b, (k, a, b)
        else:
            assert abs(a - b) <= tol * max(abs(b), 1e-300) or a == b, (k, a, b)


CFG = dict(nx=128, nr=48, dx=0.8, dr=1.5, dt=0.6, n_modes=2, profile="none", a0=0.0, ppc=(1, 1, 1),
           capacity=40000)
QUERIES = [
    (100.0, 600.0, 250),   # the bunch, bulk left out
    (0.0, 600.0, 4096),    # everything, the bulk peak near zero
    (300.0, 420.0, 1),     # one bin
    (390.0, 420.0, 7),     # peak at the lower range edge, few bins
    (1000.0, 2000.0, 64),  # empty spectrum
]


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_beam_parity_synthetic_bunch(E, beam_mod, prec):
    g = E.Sim(CFG, E.FP64 if prec == "fp64" else E.FP32_BULK)
    g.set_particles(beam_particles(CFG, 20000, 6000, seed=71))
    parts = g.get_particles()
    for q in QUERIES:
        say(prec, "query", q)
        out, hist = g.beam(*q, with_hist=True)
        ref, rhist = beam_mod.beam_parameters(parts, *q)
        check(out, hist, ref, rhist)
    empty, _ = g.beam(1000.0, 2000.0, 64, with_hist=True)
    assert all(v == 0.0 for v in empty.values())


def test_beam_arguments_rejected(E):
    g = E.Sim(CFG, E.FP32_BULK)
    g.set_particles(beam_particles(CFG, 100, 100, seed=72))
    for bad in [(10.0, 10.0, 8), (20.0, 10.0, 8), (0.0, 10.0, 0), (0.0, 10.0, E.envpic.BEAM_MAX_BINS + 1),
                (float("nan"), 10.0, 8), (0.0, float("inf"), 8)]:
        with pytest.raises(E.EnvpicError) as ei:
            g.beam(*bad)
        assert ei.value.code == -1, bad
    g.momentum()
    with pytest.raises(E.EnvpicError) as ei:
        g.beam(0.0, 10.0, 8)
    assert ei.value.code == -3
    g.envelope_step()
    g.position()
    g.field_step()
    g.beam(0.0, 10.0, 8)  # between steps again


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_beam_after_a_driven_run(E, beam_mod, prec):
    """After 80 steps of a strong pulse in plasma (moving window, modes 0
    and 1) the spectrum of the pushed electrons."""
    cfg = dict(nx=192, nr=48, dx=0.8, dr=1.5, dt=0.6, n_modes=2, ppc=(2, 2, 2), profile="uniform", n0=0.004,
               a0=3.0, w0=12.0, tau=15.0, x_c=120.0, x_f=120.0, moving_window=1, seed=191204674 + 61)
    g = E.Sim(cfg, E.FP64 if prec == "fp64" else E.FP32_BULK)
    g.step(80)
    parts = g.get_particles()
    for q in [(0.0, 0.05, 200), (1e-3, 1.0, 100)]:
        say(prec, "query", q)
        out, hist = g.beam(*q, with_hist=True)
        ref, rhist = beam_mod.beam_parameters(parts, *q)
        assert ref["count"] > 0
        check(out, hist, ref, rhist)


def test_beam_full_size_c2(E, beam_mod):
    """The 8.4 M-particle LWFA workload (2048 x 256, modes 0 and 1) after 30
    steps: every particle through the same launch configuration as the
    benchmark's beam pass."""
    g = E.Sim(C2, E.FP32_BULK)
    g.step(30)
    parts = g.get_particles()
    say("c2 particles", len(parts["x"]))
    for q in [(0.0, 2e-3, 256), (1e-5, 1e-2, 128)]:
        out, hist = g.beam(*q, with_hist=True)
        ref, rhist = beam_mod.beam_parameters(parts, *q)
        assert ref["count"] > 0
        check(out, hist, ref, rhist)
