"""Pins of the oracle's injected-beam parameters (Table BeamParams, Sec. 4).

Each test checks oracle/beam.py against a value fixed by the definition in
the table caption or by mathematics, never against the oracle itself: closed
forms of symmetric phase-space sets, invariances of the emittance, the
Gaussian spectrum's FWHM, captured charge and truncated rms spread, and
hand-computed histogram cases.
"""
import math

import numpy as np
import pytest
from scipy.special import ndtri

from oracle import beam


def _parts(px, py, pz, y, z, w):
    n = len(px)
    return {"x": np.zeros(n), "y": np.asarray(y, float), "z": np.asarray(z, float),
            "px": np.asarray(px, float), "py": np.asarray(py, float),
            "pz": np.asarray(pz, float), "w": np.asarray(w, float)}


def _px_for(e_kin, py=0.0, pz=0.0):
    """p_x giving kinetic energy e_kin (gamma - 1) with the given p_y, p_z."""
    return np.sqrt((e_kin + 1.0) ** 2 - 1.0 - py * py - pz * pz)


def test_kinetic_energy_of_known_momenta():
    def ek(px, py, pz):
        return float(beam.kinetic_energy(np.array(px), np.array(py), np.array(pz)))

    assert ek(0.0, 0.0, 0.0) == 0.0
    # |p| = sqrt(3): gamma = 2
    assert ek(1.0, 1.0, 1.0) == pytest.approx(1.0, rel=1e-15)
    # small |p|: p^2/2 - p^4/8 + ... (no cancellation)
    p = 1e-4
    assert ek(p, 0.0, 0.0) == pytest.approx(p * p / 2 - p ** 4 / 8, rel=1e-14, abs=0.0)


def test_emittance_of_symmetric_point_sets():
    """(y, p_y) = (+-a, +-b) and (z, p_z) = (+-c, +-d): eps_y = a b, eps_z = c d."""
    a, b, c, d = 1.5, 0.25, 0.7, 2.0
    rows = [(sy * a, sp * b, sz * c, sq * d) for sy in (-1, 1) for sp in (-1, 1)
            for sz in (-1, 1) for sq in (-1, 1)]
    y, py, z, pz = (np.array(v) for v in zip(*rows))
    px = _px_for(300.0, py, pz)  # every particle at the same energy
    out, hist = beam.beam_parameters(_parts(px, py, pz, y, z, np.full(16, 2.0)), 250.0, 350.0, 100)
    assert out["count"] == 16
    assert out["emit_y"] == pytest.approx(a * b, rel=1e-12)
    assert out["emit_z"] == pytest.approx(c * d, rel=1e-12)
    assert out["charge"] == pytest.approx(-32.0, rel=1e-15)
    assert out["e_rms"] < 1e-9 and out["e_mean"] == pytest.approx(300.0, rel=1e-12)


def _random_beam(seed, n=4000, e0=400.0):
    rng = np.random.default_rng(seed)
    y = rng.normal(0.3, 2.0, n)
    py = 0.4 * y + rng.normal(0.1, 1.5, n)
    z = rng.normal(-0.2, 1.0, n)
    pz = -0.3 * z + rng.normal(0.0, 0.8, n)
    px = np.full(n, e0)
    w = rng.uniform(0.5, 2.0, n)
    return y, py, z, pz, px, w


def test_emittance_invariant_under_shear_and_translation():
    """A linear shear p -> p + k u and a translation of u and p preserve the
    phase-space area; one wide bin selects every particle."""
    y, py, z, pz, px, w = _random_beam(1)
    base, _ = beam.beam_parameters(_parts(px, py, pz, y, z, w), 100.0, 1000.0, 1)
    assert base["count"] == len(y)
    for k in (0.5, -3.0):
        sh, _ = beam.beam_parameters(_parts(px, py + k * y, pz - k * z, y, z, w), 100.0, 1000.0, 1)
        assert sh["emit_y"] == pytest.approx(base["emit_y"], rel=1e-10)
        assert sh["emit_z"] == pytest.approx(base["emit_z"], rel=1e-10)
    tr, _ = beam.beam_parameters(_parts(px, py + 5.0, pz - 2.0, y - 7.0, z + 3.0, w), 100.0, 1000.0, 1)
    assert tr["emit_y"] == pytest.approx(base["emit_y"], rel=1e-10)
    assert tr["emit_z"] == pytest.approx(base["emit_z"], rel=1e-10)
    # an affine line p = k u + p0 has zero area
    ln, _ = beam.beam_parameters(_parts(px, 0.4 * y + 3.0, -2.0 * z + 1.0, y, z, w), 100.0, 1000.0, 1)
    assert ln["emit_y"] < 1e-6 * base["emit_y"] and ln["emit_z"] < 1e-6 * base["emit_z"]


def test_gaussian_spectrum_fwhm_window_and_spread():
    """Energies at the quantiles of N(mu, sigma): FWHM = 2 sqrt(2 ln 2) sigma,
    the window [peak - FWHM, peak + FWHM] holds erf(a / sqrt 2) of the charge
    (a = FWHM / sigma) and the rms spread of a normal truncated at +-a."""
    mu, sigma, n = 200.0, 4.0, 200000
    e = mu + sigma * ndtri((np.arange(n) + 0.5) / n)
    px = _px_for(e)
    zeros = np.zeros(n)
    out, hist = beam.beam_parameters(_parts(px, zeros, zeros, zeros, zeros, np.ones(n)), 150.0, 250.0, 1000)
    de = 0.1
    assert abs(out["e_peak"] - mu) <= de
    assert out["fwhm"] == pytest.approx(2.0 * math.sqrt(2.0 * math.log(2.0)) * sigma, abs=0.25 * de)
    a = out["fwhm"] / sigma
    frac = math.erf(a / math.sqrt(2.0))
    assert -out["charge"] / n == pytest.approx(frac, abs=2e-3)
    phi = math.exp(-0.5 * a * a) / math.sqrt(2.0 * math.pi)
    trunc = sigma * math.sqrt(1.0 - 2.0 * a * phi / frac)
    assert out["e_rms"] == pytest.approx(trunc, rel=5e-3)
    assert out["rel_spread"] == pytest.approx(trunc / out["e_peak"], rel=5e-3)
    assert out["charge_spectrum"] == pytest.approx(-n, rel=1e-12)


def test_particles_below_the_range_are_left_out():
    y, py, z, pz, px, w = _random_beam(2, n=3000)
    rng = np.random.default_rng(3)
    m = 20000  # bulk plasma near rest, heavy weights
    bg = _parts(rng.normal(0, 0.01, m), rng.normal(0, 0.01, m), rng.normal(0, 0.01, m),
                rng.normal(0, 50, m), rng.normal(0, 50, m), np.full(m, 100.0))
    fg = _parts(px, py, pz, y, z, w)
    both = {k: np.concatenate([fg[k], bg[k]]) for k in fg}
    alone, _ = beam.beam_parameters(fg, 100.0, 1000.0, 300)
    mixed, _ = beam.beam_parameters(both, 100.0, 1000.0, 300)
    assert alone == mixed
    low, _ = beam.beam_parameters(both, 0.0, 1000.0, 300)
    assert low["e_peak"] < 5.0  # the bulk dominates once the range includes it


def test_weights_equal_repeated_particles():
    rng = np.random.default_rng(4)
    n = 2500
    e = rng.normal(120.0, 6.0, n)
    py, pz = rng.normal(0, 1.0, n), rng.normal(0, 1.0, n)
    px = _px_for(e, py, pz)
    y, z = rng.normal(0, 3.0, n), rng.normal(0, 3.0, n)
    mult = rng.integers(1, 4, n)
    weighted, hw = beam.beam_parameters(_parts(px, py, pz, y, z, mult.astype(float)), 80.0, 160.0, 80)
    rep = np.repeat(np.arange(n), mult)
    repeated, hr = beam.beam_parameters(_parts(px[rep], py[rep], pz[rep], y[rep], z[rep], np.ones(rep.size)),
                                        80.0, 160.0, 80)
    np.testing.assert_array_equal(hw, hr)
    for k in beam.BEAM_NAMES:
        if k != "count":
            assert weighted[k] == pytest.approx(repeated[k], rel=1e-12, abs=1e-14), k


def test_peak_and_fwhm_hand_computed():
    de = 0.5
    # peak in the first bin: the left side ends at e_lo; right crossing between
    # the centres of bins 0 and 1 at (10 - 5) / (10 - 4) of a bin
    peak, fwhm, kp = beam.peak_and_fwhm(np.array([10.0, 4.0, 0.0, 0.0]), 1.0, 3.0)
    assert kp == 0 and peak == 1.25
    assert fwhm == pytest.approx(0.5 * de + 5.0 / 6.0 * de, rel=1e-15)
    # a tie picks the lower bin; contents at exactly half maximum stay inside
    peak, fwhm, kp = beam.peak_and_fwhm(np.array([0.0, 6.0, 3.0, 6.0, 1.0]), 0.0, 5.0)
    assert kp == 1 and peak == 1.5
    # left: bin 0 (0 < 3) at 0.5 of the way from centre 0 to centre 1 -> 1.0;
    # right: bins 2 (3, not below) and 3 stay inside, bin 4 (1 < 3) crosses
    # at centre 3 + (6 - 3) / (6 - 1) -> 4.1
    assert fwhm == pytest.approx(4.1 - 1.0, rel=1e-14)


def test_empty_spectrum_and_bad_arguments():
    p = _parts([0.0], [0.0], [0.0], [0.0], [0.0], [1.0])
    out, hist = beam.beam_parameters(p, 10.0, 20.0, 8)
    assert all(v == 0.0 for v in out.values()) and not hist.any()
    with pytest.raises(ValueError):
        beam.beam_parameters(p, 10.0, 10.0, 8)
    with pytest.raises(ValueError):
        beam.beam_parameters(p, 10.0, 20.0, 0)


def test_lab_units_of_the_paper_set_up():
    """lambda0 = 0.8 um: E = 1 GeV is 1956.95 m_e c^2, c/w0 = 0.1273 um."""
    out = dict.fromkeys(beam.BEAM_NAMES, 0.0)
    out.update(e_peak=1000.0 / 0.51099895, charge=-1.0, rel_spread=0.02, emit_y=1.0, emit_z=2.0)
    lab = beam.to_lab_units(out)
    assert lab["e_peak_GeV"] == pytest.approx(1.0, rel=1e-12)
    assert lab["emit_y_mm_mrad"] == pytest.approx(0.8 / (2 * math.pi), rel=1e-9)
    assert lab["rel_spread_pct"] == pytest.approx(2.0)
    # n_c (c/w0)^3 e for 0.8 um: 1.742e27 m^-3 * (1.2732e-7 m)^3 * e
    assert lab["charge_pC"] == pytest.approx(1.742e27 * (1.2732e-7) ** 3 * 1.602176634e-19 * 1e12, rel=2e-3)
