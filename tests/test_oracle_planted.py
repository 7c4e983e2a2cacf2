"""The pins of the diagnostic sums and of the plasma profiles catch planted
mistakes: each variant below is the oracle source with one plausible error
(a dropped factor, a wrong volume, a sign, an unweighted sum, a wrong slope),
compiled on the CPU into a scratch folder; at least one pin must fail on it.
"""
import concurrent.futures as cf

import pytest

import test_oracle_diagnostics as P

PLANTED = {
    "U_EM without the 1/2 of mode 0": [("0.5 * u0 + 0.25 * u1", "u0 + 0.25 * u1")],
    "U_EM with mode 1 weighted 1/2": [("0.5 * u0 + 0.25 * u1", "0.5 * u0 + 0.5 * u1")],
    "U_EM of E_r on node volumes": [("u0 += s.Er[k] * s.Er[k] * vol_half(s, j)",
                                     "u0 += s.Er[k] * s.Er[k] * vol_node(s, j)")],
    "U_EM of E_theta1 on half volumes": [("u1 += std::norm(s.Et1[k]) * vol_node(s, j)",
                                          "u1 += std::norm(s.Et1[k]) * vol_half(s, j)")],
    "kinetic energy as p^2 / (2 gamma)": [("s.w[k] * p2 / (1.0 + g)", "s.w[k] * p2 / (2.0 * g)")],
    "kinetic energy by cancellation": [("s.w[k] * p2 / (1.0 + g)", "s.w[k] * (g - 1.0 + 1e-9 * p2)")],
    "L_x with the opposite sense": [("(s.y[k] * s.pz[k] - s.z[k] * s.py[k])",
                                     "(s.z[k] * s.py[k] - s.y[k] * s.pz[k])")],
    "P_x unweighted": [("out[ORACLE_D_PX] += s.w[k] * s.px[k]", "out[ORACLE_D_PX] += s.px[k]")],
    "axis node volume pi dr^2 dx / 3": [("kPi * s.dr * s.dr * s.dx / 4.0", "kPi * s.dr * s.dr * s.dx / 3.0")],
    "|A|^2 V on half-row volumes": [("std::norm(s.A[k]) * vol_node(s, j)", "std::norm(s.A[k]) * vol_half(s, j)")],
    "ramp twice as long": [("return p.n0 * xlab / p.ramp_len;", "return p.n0 * xlab / (2.0 * p.ramp_len);")],
    "ramp starting one cell late": [("if (xlab <= 0.0) return 0.0;", "if (xlab <= s.dx) return 0.0;")],
    "perturbation one-sided": [("p.perturb * (2.0 * uniform_of(p.seed, kStreamDensity, col, j) - 1.0)",
                                "p.perturb * uniform_of(p.seed, kStreamDensity, col, j)")],
    "perturbation keyed by the wrong stream": [("uniform_of(p.seed, kStreamDensity, col, j)",
                                                "uniform_of(p.seed, kStreamAngle, col, j)")],
    "bump of width w_b sqrt 2": [("std::exp(-u * u)", "std::exp(-0.5 * u * u)")],
    "bump centred one width off": [("double u = (xlab - p.bump_x) / p.bump_w;",
                                    "double u = (xlab - p.bump_x) / p.bump_w - 1.0;")],
}

PINS = [P.test_field_energy_mode0_closed_forms, P.test_field_energy_mode1_uniform_transverse_field,
        P.test_field_energy_mode1_axial_components, P.test_kinetic_energy_of_known_momenta,
        P.test_uniform_field_kick_momentum_and_energy, P.test_angular_momentum_of_a_rotating_ring,
        lambda m: P.test_envelope_norm_of_the_initial_pulse(m, 20.0, 0.0),
        P.test_ramp_profile_column_charge, P.test_perturbed_profile_cell_charge,
        P.test_bump_profile_column_charge]


@pytest.fixture(scope="module")
def variants(oracle_mod, tmp_path_factory):
    root = tmp_path_factory.mktemp("planted")
    with cf.ThreadPoolExecutor(max_workers=4) as ex:
        futs = {name: ex.submit(oracle_mod.build_variant, edits, str(root / f"v{k}"))
                for k, (name, edits) in enumerate(PLANTED.items())}
        return {name: oracle_mod.Variant(f.result()) for name, f in futs.items()}


def _fails(pin, mod):
    try:
        pin(mod)
    except AssertionError:
        return True
    return False


def test_unmodified_source_passes_every_pin(oracle_mod, tmp_path):
    ref = oracle_mod.Variant(oracle_mod.build_variant([], str(tmp_path / "ref")))
    for pin in PINS:
        pin(ref)


@pytest.mark.parametrize("name", list(PLANTED))
def test_planted_mistake_fails_a_pin(variants, name):
    caught = [k for k, pin in enumerate(PINS) if _fails(pin, variants[name])]
    assert caught, f"no pin catches: {name}"
