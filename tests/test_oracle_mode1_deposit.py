"""Pins of the oracle's mode-1 current deposit (reading R11: the direct
deposit at the mid-point of the move, amplitude and phase of the azimuthal
Fourier coefficient) by closed forms of smooth states, for both shape orders.

A mode-1 field F is seen at azimuth theta as Re[F e^{-i theta}].  A plasma
moving with a uniform velocity v then carries, in the interior of the grid
(away from the axis rows, r_max and the window ends):

  * v along y, density n(x): J = q n v y-hat, so J_r(theta) = q n v
    cos(theta) and J_theta(theta) = -q n v sin(theta), i.e.
        J_r1 = q n v,  J_theta1 = -i q n v,  J_x1 = 0;
  * v along x, density n(x, r) (1 + eps cos(theta - theta0)):
        J_x1 = q n v eps e^{+i theta0},  J_r1 = J_theta1 = 0.

Densities are linear in x and r, n = n0 (1 + gx (x - xc)) (1 + gr r), so that
the deposit also sees where each shape sits: a shape S of unit mass and
variance sigma^2 gives, at a node of radius r_j whose stencil stays off the
axis, the x factor at the node (at the mid-point of the move, x - v dt/2)
and the r factor 1 + gr (r_j + sigma^2 / r_j), from the cylindrical volume
2 pi r_j dr dx of the node (sigma^2 = dr^2/6 for the linear hat, dr^2/4 for
the quadratic B-spline).

The states are quiet starts: strata in x at equal steps, off-centre in each
cell, 3-point Gauss-Legendre nodes on each half cell in r, equally spaced
azimuths, each macroparticle weighted by the density times its share of the
stratum volume.  These sums equal the continuum integrals exactly (along x a
B-spline of width dx summed over a lattice of step dx/n reproduces linear
functions; across r the integrands are polynomials of degree at most 4
between the half-cell breakpoints of the shapes), so the bar is rounding,
1e-12 of q n0 v: a dropped factor, a conjugated phase, a swapped component,
a wrong volume or a misplaced stencil fails it by far.
"""
import numpy as np
import pytest

Q = -1.0
GX, GR, XC = 0.02, 0.03, 10.0


def _cfg(order):
    return dict(nx=24, nr=16, dx=0.8, dr=1.5, dt=0.3, n_modes=2, profile="none", a0=0.0, shape_order=order)


def _quiet_start(cfg, n0, gr=0.0, eps=0.0, theta0=0.0, nsx=2, nth=8):
    """Plasma of density n0 (1 + GX (x - XC)) (1 + gr r) (1 + eps cos(theta
    - theta0)) on x cells [2, nx - 2) and r cells [0, nr - 1)."""
    nx, nr, dx, dr = cfg["nx"], cfg["nr"], cfg["dx"], cfg["dr"]
    xs = (np.arange(2 * nsx, (nx - 2) * nsx) + 0.3) * dx / nsx  # off-centre: no mirror symmetry in a cell
    gl, gw = np.polynomial.legendre.leggauss(3)
    h = 0.5 * dr
    lo = np.arange(2 * (nr - 1)) * h
    rs = (lo[:, None] + 0.5 * h * (1.0 + gl[None, :])).ravel()
    vr = (2 * np.pi * rs * 0.5 * h * np.tile(gw, len(lo))) * (dx / nsx) / nth
    th = (np.arange(nth) + 0.37) * 2 * np.pi / nth
    X, R, T = np.meshgrid(xs, rs, th, indexing="ij")
    V = np.broadcast_to(vr[None, :, None], X.shape)
    w = n0 * V * (1.0 + GX * (X - XC)) * (1.0 + gr * R) * (1.0 + eps * np.cos(T - theta0))
    n = X.size
    return dict(x=X.ravel(), y=(R * np.cos(T)).ravel(), z=(R * np.sin(T)).ravel(), px=np.zeros(n),
                py=np.zeros(n), pz=np.zeros(n), w=w.ravel(), id=np.arange(n, dtype=np.uint32))


def _interior(cfg, order):
    jlo = 2 if order == 2 else 1
    return slice(4, cfg["nx"] - 4), slice(jlo, cfg["nr"] - 3)


def _run(oracle_mod, cfg, parts):
    s = oracle_mod.OracleSim(cfg)
    s.set_particles(parts)
    s.position_J()
    return s


@pytest.mark.parametrize("order", [1, 2])
def test_transverse_drift_gives_real_jr1_and_minus_i_jtheta1(oracle_mod, order):
    cfg = _cfg(order)
    n0, p = 0.01, 1e-3
    parts = _quiet_start(cfg, n0)
    parts["py"][:] = p
    s = _run(oracle_mod, cfg, parts)
    v = p / np.sqrt(1.0 + p * p)
    sx, sr = _interior(cfg, order)
    x = np.arange(cfg["nx"] + 1)[sx] * cfg["dx"]  # J_r1 and J_theta1 sit on primal x
    j0 = (Q * n0 * v * (1.0 + GX * (x - XC)))[:, None]
    jr1, jt1, jx1 = (s.get_field(n)[sx, sr] for n in ("jr1", "jt1", "jx1"))
    scale = abs(Q * n0 * v)
    assert np.abs(jr1 - j0).max() <= 1e-12 * scale
    assert np.abs(jt1 - (-1j) * j0).max() <= 1e-12 * scale
    assert np.abs(jx1).max() <= 1e-12 * scale


@pytest.mark.parametrize("order", [1, 2])
def test_modulated_axial_drift_gives_jx1_with_the_modulation_phase(oracle_mod, order):
    cfg = _cfg(order)
    n0, p, eps, th0 = 0.01, 1e-3, 0.3, 2.1
    dx, dr, dt = cfg["dx"], cfg["dr"], cfg["dt"]
    parts = _quiet_start(cfg, n0, GR, eps, th0)
    parts["px"][:] = p
    s = _run(oracle_mod, cfg, parts)
    v = p / np.sqrt(1.0 + p * p)
    sx, sr = _interior(cfg, order)
    x = (np.arange(cfg["nx"] + 1)[sx] + 0.5) * dx - 0.5 * v * dt  # J_x1 on dual x, mid-point shift
    rj = np.arange(cfg["nr"] + 1)[sr] * dr
    var = dr * dr / (4.0 if order == 2 else 6.0)
    fr = 1.0 + GR * (rj + var / rj)
    want = Q * n0 * v * eps * np.exp(1j * th0) * (1.0 + GX * (x - XC))[:, None] * fr[None, :]
    scale = abs(Q * n0 * v)
    assert np.abs(s.get_field("jx1")[sx, sr] - want).max() <= 1e-12 * scale
    for name in ("jr1", "jt1"):
        assert np.abs(s.get_field(name)[sx, sr]).max() <= 1e-12 * scale


@pytest.mark.parametrize("order", [1, 2])
def test_single_particle_phase_is_the_azimuth_of_the_mid_point(oracle_mod, order):
    """One electron moving along y: its mode-1 J_r and J_theta carry e^{+i
    theta_m}, theta_m the azimuth of the mid-point of its move (not of its
    start), and their ratio is v_theta / v_r there; J_x1 is zero."""
    cfg = _cfg(order)
    th, r, p = 0.6, 3.7, 0.5
    x0, y0, z0 = 9.3, r * np.cos(th), r * np.sin(th)
    parts = dict(x=np.array([x0]), y=np.array([y0]), z=np.array([z0]), px=np.zeros(1), py=np.array([p]),
                 pz=np.zeros(1), w=np.array([1.0]), id=np.zeros(1, np.uint32))
    s = _run(oracle_mod, cfg, parts)
    v = p / np.sqrt(1.0 + p * p)
    ym = y0 + 0.5 * cfg["dt"] * v
    thm = np.arctan2(z0, ym)
    assert abs(thm - th) > 1e-2
    vr, vt = v * np.cos(thm), -v * np.sin(thm)
    jr1, jt1 = s.get_field("jr1"), s.get_field("jt1")
    nz = np.abs(jr1) > 0
    assert nz.sum() == (4 if order == 1 else 9)
    # q < 0 and v_r > 0: -J_r1 points along e^{i theta_m}
    assert np.allclose(np.angle(-jr1[nz]), thm, rtol=0, atol=1e-12)
    nzt = np.abs(jt1) > 0
    assert np.allclose(np.angle(-np.sign(vt) * jt1[nzt]), thm, rtol=0, atol=1e-12)
    # both use the same (primal x) stencil, J_r on half rows and J_theta on primal rows;
    # summed over the stencil with the node volumes, the ratio is v_theta / v_r
    dr, dx = cfg["dr"], cfg["dx"]
    j = np.arange(cfg["nr"] + 1)
    vh = 2 * np.pi * (j + 0.5) * dr * dr * dx
    vn = np.where(j == 0, np.pi * dr * dr * dx / 4, 2 * np.pi * j * dr * dr * dx)
    qr = (jr1 * vh[None, :]).sum()
    qt = (jt1 * vn[None, :]).sum()
    assert abs(qt / qr - vt / vr) <= 1e-12 * abs(vt / vr)
    assert abs(qr - 2 * Q * vr * np.exp(1j * thm)) <= 1e-12 * abs(qr)
    assert np.abs(s.get_field("jx1")).max() == 0.0
