"""Injected-beam parameters of a particle set, plain FP64 numpy (the oracle).

TEST INFRASTRUCTURE ONLY: imported by the test suite, the smoke check and the
CPU-baseline leg of the benchmark; it imports nothing from the GPU package.

What is computed (Sec. 4, Table BeamParams of arXiv:1912.04674): the peak of
the electron energy spectrum, the beam charge, the relative energy spread and
the normalized transverse emittance
    eps_n = sqrt(sigma_x^2 sigma_p^2 - sigma_xp^2),
all over the particles that lie within two FWHM widths in energy around the
spectrum peak.  The table defines the quantities; the paper gives no
histogram or window rule beyond that, so this module takes the readings
below (R25), each in plain code:

  * energy: kinetic energy gamma - 1 in m_e c^2, gamma = sqrt(1 + |p|^2) of
    the particle's momentum (the envelope's quiver term is not beam energy),
    evaluated as |p|^2 / (1 + sqrt(1 + |p|^2)), the same number without the
    cancellation of sqrt(.) - 1 at small |p|;
  * spectrum: the charge histogram sum |q| w over `nbins` equal bins on the
    caller's range [e_lo, e_hi); particles outside the range are not part of
    the spectrum (e_lo is how a caller leaves out the bulk plasma);
  * peak: the bin of largest content (the lowest such bin on a tie); the
    peak energy is its centre;
  * FWHM: from the peak outwards, the first bin on each side whose content is
    below half the peak's; the half-maximum crossing is interpolated linearly
    between that bin's centre and its neighbour's towards the peak; a side
    that never drops below half maximum inside the range ends at the range
    edge;
  * window: "two FWHM widths around the peak" is [E_peak - FWHM,
    E_peak + FWHM] (two widths in total), intersected with [e_lo, e_hi);
  * moments: weighted by the macro-particle weight, centred (two passes);
    the energy spread is the rms spread divided by the peak energy; the
    transverse planes are y = r cos(theta) with p_y and z = r sin(theta)
    with p_z, one emittance each.

Charge is sum q w with q = -1 (electrons), in the units of the weights
(densities in n_c times volumes in (c/w0)^3); emittance is in c/w0.
Pinned by tests/test_oracle_beam.py: closed-form emittances of symmetric
point sets and their invariance under phase-space shear and translation, the
FWHM, captured charge and truncated rms spread of a Gaussian spectrum, the
exclusion of particles below the range, weights equal to repeated particles,
and the kinetic energy of known momenta.
"""
import math

import numpy as np

BEAM_NAMES = ["e_peak", "fwhm", "charge", "e_mean", "e_rms", "rel_spread",
              "emit_y", "emit_z", "count", "charge_spectrum", "win_lo", "win_hi"]
Q_ELECTRON = -1.0


def kinetic_energy(px, py, pz):
    """gamma - 1 in m_e c^2 for momenta in m_e c."""
    p2 = px * px + py * py + pz * pz
    return p2 / (1.0 + np.sqrt(1.0 + p2))


def spectrum(energy, w, e_lo, e_hi, nbins):
    """Charge histogram sum |q| w per bin of [e_lo, e_hi) and the mask of the
    particles inside the range."""
    de = (e_hi - e_lo) / nbins
    inside = (energy >= e_lo) & (energy < e_hi)
    k = np.floor((energy[inside] - e_lo) / de).astype(np.int64)
    k = np.minimum(k, nbins - 1)
    hist = np.zeros(nbins)
    wk = np.abs(Q_ELECTRON) * w[inside]
    for b in range(nbins):  # exact per-bin sums
        sel = wk[k == b]
        hist[b] = math.fsum(sel) if sel.size else 0.0
    return hist, inside


def peak_and_fwhm(hist, e_lo, e_hi):
    """Peak energy (centre of the fullest bin) and the FWHM interpolated
    between bin centres at half maximum."""
    nbins = len(hist)
    de = (e_hi - e_lo) / nbins

    def centre(b):
        return e_lo + (b + 0.5) * de

    kp = 0
    for b in range(1, nbins):
        if hist[b] > hist[kp]:
            kp = b
    hmax = hist[kp]
    half = 0.5 * hmax
    # left side
    left = e_lo
    for b in range(kp - 1, -1, -1):
        if hist[b] < half:
            left = centre(b) + (half - hist[b]) / (hist[b + 1] - hist[b]) * de
            break
    right = e_hi
    for b in range(kp + 1, nbins):
        if hist[b] < half:
            right = centre(b - 1) + (hist[b - 1] - half) / (hist[b - 1] - hist[b]) * de
            break
    return centre(kp), right - left, kp


def _emittance(u, pu, w):
    """sqrt(<du^2><dpu^2> - <du dpu>^2), moments weighted by w and centred."""
    W = math.fsum(w)
    um = math.fsum(w * u) / W
    pm = math.fsum(w * pu) / W
    du, dp = u - um, pu - pm
    s_uu = math.fsum(w * du * du) / W
    s_pp = math.fsum(w * dp * dp) / W
    s_up = math.fsum(w * du * dp) / W
    return math.sqrt(max(0.0, s_uu * s_pp - s_up * s_up))


def beam_parameters(parts, e_lo, e_hi, nbins):
    """Beam parameters of a particle set (dict of FP64 arrays x, y, z, px,
    py, pz, w as the oracle and the GPU library export them).  Returns
    (dict of BEAM_NAMES, histogram).  An empty spectrum gives all zeros."""
    if not (nbins >= 1 and e_hi > e_lo):
        raise ValueError("need nbins >= 1 and e_hi > e_lo")
    px, py, pz = (np.asarray(parts[k], dtype=np.float64) for k in ("px", "py", "pz"))
    y, z, w = (np.asarray(parts[k], dtype=np.float64) for k in ("y", "z", "w"))
    energy = kinetic_energy(px, py, pz)
    hist, inside = spectrum(energy, w, e_lo, e_hi, nbins)
    out = dict.fromkeys(BEAM_NAMES, 0.0)
    if not np.any(hist > 0.0):
        return out, hist
    e_peak, fwhm, _ = peak_and_fwhm(hist, e_lo, e_hi)
    lo, hi = max(e_lo, e_peak - fwhm), e_peak + fwhm
    sel = inside & (energy >= lo) & (energy <= hi)
    ws = w[sel]
    W = math.fsum(ws)
    es = energy[sel]
    e_mean = math.fsum(ws * es) / W
    e_rms = math.sqrt(math.fsum(ws * (es - e_mean) ** 2) / W)
    out.update(
        e_peak=e_peak, fwhm=fwhm, charge=Q_ELECTRON * W, e_mean=e_mean,
        e_rms=e_rms, rel_spread=e_rms / e_peak,
        emit_y=_emittance(y[sel], py[sel], ws), emit_z=_emittance(z[sel], pz[sel], ws),
        count=float(np.count_nonzero(sel)),
        charge_spectrum=Q_ELECTRON * math.fsum(w[inside]), win_lo=lo, win_hi=min(hi, e_hi))
    return out, hist


# Conversion of code units to the units of Table BeamParams for a laser
# wavelength lambda0 (the paper's set-up reproduces its 15 J with 0.8 um).
E_MC2_MEV = 0.51099895
E_CHARGE = 1.602176634e-19
EPS0 = 8.8541878128e-12
M_E = 9.1093837015e-31
C_LIGHT = 299792458.0


def to_lab_units(out, lambda0_m=0.8e-6):
    """Peak energy in GeV, charge in pC, spread in %, emittance in mm mrad."""
    omega0 = 2.0 * math.pi * C_LIGHT / lambda0_m
    n_c = EPS0 * M_E * omega0 ** 2 / E_CHARGE ** 2
    l0 = C_LIGHT / omega0
    return {
        "e_peak_GeV": out["e_peak"] * E_MC2_MEV * 1e-3,
        "charge_pC": abs(out["charge"]) * n_c * l0 ** 3 * E_CHARGE * 1e12,
        "rel_spread_pct": 100.0 * out["rel_spread"],
        "emit_y_mm_mrad": out["emit_y"] * l0 * 1e6,
        "emit_z_mm_mrad": out["emit_z"] * l0 * 1e6,
    }
