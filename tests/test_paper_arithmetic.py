"""The paper's own arithmetic, from the values it prints (tests/golden/
sec4_nonlinear_benchmark.json): Eq. Speedup gives about 1200; a 0.8 um
wavelength reproduces the quoted 15 J; and the unit conversions of the
beam-parameter oracle carry Table BeamParams to code units and back."""
import json
import math
import os

import pytest

from oracle import beam

G = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "sec4_nonlinear_benchmark.json")))

C = 299792458.0
E_CHARGE = 1.602176634e-19
M_E = 9.1093837015e-31
EPS0 = 8.8541878128e-12


def test_speedup_equation():
    """Eq. Speedup: particles of the 3D run over those of the cylindrical run
    (half the transverse domain), with the printed cell counts and ppc."""
    g = G["grids"]
    s = (g["n_cells_perp"] ** 2 * g["n_cells_parallel"] * g["ppc_3d"]) / (
        g["n_cells_perp"] / 2 * g["n_cells_parallel"] * g["ppc_cyl"])
    assert s == pytest.approx(1194.67, abs=0.01)
    assert s == pytest.approx(G["cost"]["ratio_3d_over_cyl"], rel=0.005)


def test_laser_energy_with_0p8_um():
    """A Gaussian pulse of peak a0 (linear polarisation): E0 = a0 m_e c w0 / e,
    I0 = eps0 c E0^2 / 2; energy = I0 (pi w^2 / 2) tau_I sqrt(pi / (4 ln 2))
    for an intensity FWHM tau_I.  With lambda0 = 0.8 um it is the quoted 15 J."""
    L = G["laser"]
    lam = L["lambda0_um_not_printed"] * 1e-6
    w0 = 2 * math.pi * C / lam
    e0 = L["a0"] * M_E * C * w0 / E_CHARGE
    i0 = EPS0 * C * e0 ** 2 / 2
    area = math.pi * (L["waist_um"] * 1e-6) ** 2 / 2
    energy = i0 * area * L["fwhm_intensity_fs"] * 1e-15 * math.sqrt(math.pi / (4 * math.log(2)))
    assert energy == pytest.approx(L["energy_J"], rel=0.01)
    # the plateau density in units of the critical density
    n_c = EPS0 * M_E * w0 ** 2 / E_CHARGE ** 2 * 1e-6  # cm^-3
    assert L["plateau_density_cm3"] / n_c == pytest.approx(4.59e-4, rel=0.01)


@pytest.mark.parametrize("which", ["3d", "cylindrical"])
def test_beam_table_units_round_trip(which):
    """The table's peak energy, charge and emittance, put in code units
    (m_e c^2, weights in n_c (c/w0)^3, c/w0) and back through the oracle's
    conversion."""
    t = G["beam_params"][which]
    lam = 0.8e-6
    w0 = 2 * math.pi * C / lam
    l0 = C / w0
    n_c = EPS0 * M_E * w0 ** 2 / E_CHARGE ** 2
    out = dict.fromkeys(beam.BEAM_NAMES, 0.0)
    out["e_peak"] = t["e_peak_GeV"] * 1e3 / 0.51099895
    out["charge"] = -t["charge_pC"] * 1e-12 / (E_CHARGE * n_c * l0 ** 3)
    out["rel_spread"] = t["rel_spread_pct"] / 100
    out["emit_y"] = t["emit_n_mm_mrad"] * 1e-6 / l0
    lab = beam.to_lab_units(out, lambda0_m=lam)
    assert lab["e_peak_GeV"] == pytest.approx(t["e_peak_GeV"], rel=1e-12)
    assert lab["charge_pC"] == pytest.approx(t["charge_pC"], rel=1e-12)
    assert lab["rel_spread_pct"] == pytest.approx(t["rel_spread_pct"], rel=1e-12)
    assert lab["emit_y_mm_mrad"] == pytest.approx(t["emit_n_mm_mrad"], rel=1e-12)
    assert out["e_peak"] == pytest.approx({"3d": 2211.35, "cylindrical": 2152.64}[which], rel=1e-5)
