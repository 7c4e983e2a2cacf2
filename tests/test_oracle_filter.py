"""Pins of the oracle's binomial current filter (the uncompensated binomial
filter of the paper's nonlinear benchmark, Sec. 4): N passes of 1-2-1, each
along x then along r, with zero current outside the window and beyond r_max
and parity ghosts below the axis.

The pins are closed forms of the filter, not the oracle's own formula:
  * a Fourier mode cos(k i) far from the ends is multiplied by
    (cos^2(k/2))^N (the transfer function of N passes of 1-2-1);
  * 1-2-1 leaves a linear function unchanged, so a radial profile whose
    parity extension through the axis is linear (odd: r-linear through the
    right point; even: constant) stays exact at the axis rows: a wrong ghost
    sign or a ghost taken from the wrong row breaks it at j = 0;
  * one pass on a constant gives 3/4 next to a zero boundary."""
import numpy as np
import pytest

from inputs import C1, scaled

NX, NR = 64, 40


def _sim(oracle_mod, passes, modes=2):
    cfg = scaled(C1, nx=NX, nr=NR, n_modes=modes, profile="none", a0=0.0, filter_passes=passes)
    return oracle_mod.OracleSim(cfg)


def _grid():
    i = np.arange(NX + 1)[:, None] * np.ones((1, NR + 1))
    j = np.ones((NX + 1, 1)) * np.arange(NR + 1)[None, :]
    return i, j


@pytest.mark.parametrize("passes", [1, 3, 7])
def test_transfer_function_and_axis_parity(oracle_mod, passes):
    k = 2 * np.pi / 13.0
    g = (np.cos(k / 2) ** 2) ** passes
    i, j = _grid()
    c1 = 0.7 - 0.4j
    # component: (profile, x-valid max, r-valid max, is the radial part exact)
    cases = {
        "jx": (np.cos(k * i), NX - 1, NR),                   # mode 0 axial: even, primal r -> constant
        "jr": (np.cos(k * i) * (j + 0.5), NX, NR - 1),       # mode 0 radial: odd about j = -1/2 -> j + 1/2
        "jx1": (c1 * np.cos(k * i) * j, NX - 1, NR),         # mode 1 axial: odd about j = 0 -> j
        "jr1": (c1 * np.cos(k * i), NX, NR - 1),             # mode 1 radial: even, half-integer r -> constant
        "jt1": (c1 * np.cos(k * i) * np.ones_like(j), NX, NR),  # mode 1 azimuthal: even, primal r
    }
    s = _sim(oracle_mod, passes)
    for name, (f, imax, jmax) in cases.items():
        f = np.array(f)
        f[imax + 1:, :] = 0
        f[:, jmax + 1:] = 0
        s.set_field(name, f)
    s.filter_J()
    for name, (f, imax, jmax) in cases.items():
        out = s.get_field(name)
        # interior: N from the x ends and from r_max (the axis is included)
        sl = (slice(passes, imax - passes + 1), slice(0, jmax - passes + 1))
        want = g * np.array(f)[sl]
        np.testing.assert_allclose(out[sl], want, rtol=0, atol=1e-13 * np.abs(f).max(), err_msg=name)


def test_one_pass_at_the_zero_boundaries(oracle_mod):
    s = _sim(oracle_mod, 1, modes=1)
    one = np.zeros((NX + 1, NR + 1))
    one[: NX, :] = 1.0  # J_x valid for i <= nx - 1, j <= nr
    s.set_field("jx", one)
    s.filter_J()
    out = s.get_field("jx")
    mid = NR // 2
    assert out[0, mid] == pytest.approx(0.75, abs=1e-15)         # x end: (0 + 2 + 1)/4
    assert out[NX - 1, mid] == pytest.approx(0.75, abs=1e-15)
    assert out[NX // 2, NR] == pytest.approx(0.75, abs=1e-15)     # r_max: (1 + 2 + 0)/4
    assert out[NX // 2, 0] == pytest.approx(1.0, abs=1e-15)       # axis, even ghost
    assert out[0, NR] == pytest.approx(0.75 * 0.75, abs=1e-15)    # corner: both
    assert np.all(out[NX:, :] == 0)


def test_odd_axial_current_vanishes_on_the_axis(oracle_mod):
    """Mode-1 J_x is odd about the axis: a current on the axis row alone is
    not a current at all, and filters to zero everywhere."""
    s = _sim(oracle_mod, 4)
    f = np.zeros((NX + 1, NR + 1), complex)
    f[: NX, 0] = 1.0 - 2.0j
    s.set_field("jx1", f)
    s.filter_J()
    assert np.abs(s.get_field("jx1")).max() == 0.0


def test_no_filter_is_identity(oracle_mod):
    s = _sim(oracle_mod, 0)
    rng = np.random.default_rng(3)
    f = rng.standard_normal((NX + 1, NR + 1))
    s.set_field("jr", f)
    s.filter_J()
    np.testing.assert_array_equal(s.get_field("jr"), f)
