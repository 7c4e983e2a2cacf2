"""Pins of the oracle's mode-1 field update by the normal modes of the
conducting cylinder (closed forms, no oracle arithmetic retyped).

Inside a perfectly conducting cylinder of radius R, an azimuthal-mode m = 1
field varying as cos or sin along x is a normal mode with
    TM: E_x = J_1(k r) cos(k_x x),  J_1(k R) = 0   (k R = j_{1,1} = 3.8317),
    TE: B_x = J_1(k r) sin(k_x x),  J_1'(k R) = 0  (k R = j'_{1,1} = 1.8412),
and frequency w^2 = k^2 + k_x^2.  The leapfrog Yee scheme changes this in
two known ways: a sine profile along x sees (2/dx) sin(k_x dx/2) for k_x,
and the time step gives w_d = (2/dt) asin((dt/2) sqrt(k_x'^2 + k^2)).  What
remains is the radial discretisation, which must vanish at second order:
the TM frequency error falls by 4 when dr halves.  Together these pin the
mode-1 E_x, E_r, E_theta, B_x, B_r, B_theta updates (the m/r terms, the
axis rows and the wall rows).  The frequency is read from the zero crossings
of one field component, a least-squares line through the crossing times.
"""
import numpy as np
import pytest
from scipy.special import j1, jn_zeros, jnp_zeros, jvp


def _freq(ts, vs):
    zc = []
    for a in range(len(vs) - 1):
        if vs[a] * vs[a + 1] < 0:
            zc.append(ts[a] + (ts[a + 1] - ts[a]) * vs[a] / (vs[a] - vs[a + 1]))
    zc = np.array(zc)
    assert len(zc) >= 6, "too few zero crossings"
    k = np.arange(len(zc))
    half = np.polyfit(k, zc, 1)[0]  # crossings are half a period apart
    return np.pi / half


def _run(oracle_mod, pol, dr, nr, nx, dx=0.8, periods=4):
    dt = 0.3 * dr
    rmax, L = nr * dr, nx * dx
    s = oracle_mod.OracleSim(dict(nx=nx, nr=nr, dx=dx, dr=dr, dt=dt, n_modes=2, profile="none", a0=0.0))
    i = np.arange(nx + 1)[:, None]
    if pol == "TM":  # uniform along x: E_x1 on the primal rows
        k, kx = jn_zeros(1, 1)[0] / rmax, 0.0
        r = np.arange(nr + 1)[None, :] * dr
        f = (j1(k * r) * np.ones_like(i)).astype(complex)
        f[-1, :] = 0
        s.set_field("ex1", f)
        probe = "ex1"
    else:  # one half wave along x: B_x1 on the half rows, read E_r1
        k, kx = jnp_zeros(1, 1)[0] / rmax, np.pi / L
        rh = (np.arange(nr + 1)[None, :] + 0.5) * dr
        f = (j1(k * rh) * np.sin(kx * i * dx)).astype(complex)
        f[:, -1] = 0
        s.set_field("bx1", f)
        s.set_field("bx1_bar", f)
        probe = "er1"
    kxd = (2 / dx) * np.sin(kx * dx / 2)
    w_d = (2 / dt) * np.arcsin((dt / 2) * np.sqrt(kxd ** 2 + k ** 2))
    nsteps = int(periods * 2 * np.pi / w_d / dt) + 2
    ts, vs = [], []
    for n in range(nsteps):
        s.step(1)
        v = s.get_field(probe)[nx // 2, nr // 3]
        vs.append(v.real if abs(v.real) >= abs(v.imag) else v.imag)
        ts.append((n + 1) * dt)
    return (_freq(np.array(ts), np.array(vs)) - w_d) / w_d


def test_tm11_frequency_second_order(oracle_mod):
    e1 = _run(oracle_mod, "TM", 1.0, 24, 4)
    e2 = _run(oracle_mod, "TM", 0.5, 48, 4)
    assert abs(e2) < 2e-4
    assert 3.5 < e1 / e2 < 4.5


def test_te111_frequency(oracle_mod):
    for dr, nr in ((1.0, 24), (0.5, 48)):
        assert abs(_run(oracle_mod, "TE", dr, nr, 40)) < 1e-5


def _profile_error(oracle_mod, pol, dr, nr, nx, dx=0.8, nsteps=400):
    """Largest deviation, over all rows from the axis to the wall, of one
    component's radial profile (taken when its amplitude peaks, mid-box in x)
    from its closed-form mode shape, after a best-fit scale:
      TE: E_theta ~ J_1'(k r) on the primal rows (J_1'(0) = 1/2 on the axis);
      TM: B_r ~ J_1(k r) / (k r) on the primal rows (1/2 on the axis)."""
    dt = 0.3 * dr
    rmax, L = nr * dr, nx * dx
    s = oracle_mod.OracleSim(dict(nx=nx, nr=nr, dx=dx, dr=dr, dt=dt, n_modes=2, profile="none", a0=0.0))
    i = np.arange(nx + 1)[:, None]
    r = np.arange(nr + 1) * dr
    if pol == "TE":
        k, kx = jnp_zeros(1, 1)[0] / rmax, np.pi / L
        rh = (np.arange(nr + 1)[None, :] + 0.5) * dr
        f = (j1(k * rh) * np.sin(kx * i * dx)).astype(complex)
        f[:, -1] = 0
        s.set_field("bx1", f)
        s.set_field("bx1_bar", f)
        name, ref = "et1", jvp(1, k * r)
    else:
        k = jn_zeros(1, 1)[0] / rmax
        f = (j1(k * r)[None, :] * np.ones_like(i)).astype(complex)
        f[-1, :] = 0
        s.set_field("ex1", f)
        kr = np.where(r > 0, k * r, 1.0)
        name, ref = "br1", np.where(r > 0, j1(kr) / kr, 0.5)
    best = None
    for _ in range(nsteps):
        s.step(1)
        v = s.get_field(name)[nx // 2]
        if best is None or np.abs(v).max() > best[0]:
            best = (np.abs(v).max(), v.copy())
    v = best[1][:nr]
    ref = ref[:nr]
    c = np.vdot(ref, v) / np.vdot(ref, ref)
    return np.abs(v - c * ref).max() / np.abs(c * ref).max()


def test_te111_profile_through_the_axis(oracle_mod):
    assert _profile_error(oracle_mod, "TE", 0.5, 24, 40) < 2.5e-3


def test_tm110_profile_through_the_axis(oracle_mod):
    assert _profile_error(oracle_mod, "TM", 0.5, 24, 4) < 7e-3
