"""Pins of the oracle's self-consistent bunch fields (oracle/bunch.py, R27):
the discrete Gauss law against this file's own charge deposit, the radial
field of a long uniform cylinder, the 1/gamma^2 scaling of E_x, the total
charge, and the 1/gamma^2 cancellation of the radial self-force on a
co-moving electron in the oracle's own pusher."""
import numpy as np
import pytest

from inputs import bunch_particles
from oracle import bunch


def _cfg(**kw):
    c = dict(nx=96, nr=24, dx=0.8, dr=1.5, dt=0.6, profile="none", a0=0.0)
    c.update(kw)
    return c


def _own_rho_v(cfg, parts, order):
    """q sum w S with this file's own weights (and the axis fold for order 2)."""
    nx, nr, dx, dr = cfg["nx"], cfg["nr"], cfg["dx"], cfg["dr"]
    ux = parts["x"] / dx
    ur = np.hypot(parts["y"], parts["z"]) / dr
    out = np.zeros((nx + 3, nr + 3))
    if order == 1:
        i0, j0 = np.floor(ux).astype(int), np.floor(ur).astype(int)
        fx, fr = ux - i0, ur - j0
        for a, wa in ((0, 1 - fx), (1, fx)):
            for b, wb in ((0, 1 - fr), (1, fr)):
                np.add.at(out, (i0 + a, j0 + b), -parts["w"] * wa * wb)
    else:
        def w3(u):
            m = np.floor(u + 0.5)
            d = u - m
            return m.astype(int), [0.5 * (0.5 - d) ** 2, 0.75 - d * d, 0.5 * (0.5 + d) ** 2]
        mx, wx = w3(ux)
        mr, wr = w3(ur)
        for a in range(3):
            for b in range(3):
                jj = np.abs(mr - 1 + b)
                np.add.at(out, (mx - 1 + a, jj), -parts["w"] * wx[a] * wr[b])
    return out[: nx + 1, : nr + 1]


def _div_times_v(cfg, ex, er):
    """V_j div E at the primal nodes, divergence of the field update: node
    volumes 2 pi r_j dr dx (pi dr^2 dx / 4 on the axis), radial faces
    2 pi r_{j+1/2} dx."""
    dx, dr, nr = cfg["dx"], cfg["dr"], cfg["nr"]
    j = np.arange(nr + 1)
    V = np.where(j == 0, np.pi * dr * dr * dx / 4, 2 * np.pi * j * dr * dr * dx)
    A = 2 * np.pi * (j + 0.5) * dr * dx
    d = np.zeros_like(ex)
    d[1:, :] += V[None, :] * (ex[1:, :] - ex[:-1, :]) / dx
    flux = A[None, :] * er
    d[:, 0] += flux[:, 0]
    d[:, 1:] += flux[:, 1:] - flux[:, :-1]
    return d


@pytest.mark.parametrize("order", [1, 2])
@pytest.mark.parametrize("beta", [0.0, 0.9, 0.999])
def test_discrete_gauss_law(order, beta):
    cfg = _cfg(shape_order=order)
    parts = bunch_particles(3000, 5, x0=38.0, sig_x=6.0, sig_r=3.0, p0=1.0, w_total=2.0)
    ex, er, bt, phi, qv = bunch.bunch_fields(cfg, parts, beta)
    own = _own_rho_v(cfg, parts, order)
    assert np.abs(qv - own).max() < 1e-14 * np.abs(own).max()
    dv = _div_times_v(cfg, ex, er)
    sl = (slice(1, cfg["nx"]), slice(0, cfg["nr"]))
    assert np.abs(dv - own)[sl].max() < 1e-10 * np.abs(own).max()
    assert qv.sum() == pytest.approx(-2.0, rel=1e-13)  # every particle inside
    assert np.array_equal(bt[:-1, :-1], beta * 0.5 * (er[:-1, :-1] + er[1:, :-1]))


def test_long_uniform_cylinder_radial_field():
    """A long cylinder of uniform density n_b and radius R (regular loading,
    weights ~ r, linear shapes: exactly n_b on the nodes off the axis)
    moving at beta -> 1.  In its middle, between two radii inside, r E_r
    changes by -n_b (r2^2 - r1^2) / 2 (Gauss's law over the ring between
    them); outside, r E_r is constant, -n_b R^2 / 2 up to the axis node's
    deposit excess, whatever the wall radius."""
    cfg = _cfg(nx=200, nr=30)
    dx, dr = cfg["dx"], cfg["dr"]
    nb, R = 0.01, 12 * dr
    xs = (np.arange(40 * 4, 160 * 4) + 0.5) * dx / 4
    rs = (np.arange(0, 12 * 4) + 0.5) * dr / 4
    X, Rr = np.meshgrid(xs, rs, indexing="ij")
    w = nb * 2 * np.pi * Rr * (dx / 4) * (dr / 4)
    parts = dict(x=X.ravel(), y=Rr.ravel(), z=np.zeros(X.size), w=w.ravel())
    ex, er, bt, phi, qv = bunch.bunch_fields(cfg, parts, 0.9999)
    i = 100  # middle of the bunch
    rh = (np.arange(cfg["nr"]) + 0.5) * dr
    rE = rh * er[i, : cfg["nr"]]
    for k, j in ((1, 5), (2, 10), (3, 9)):
        assert rE[j] - rE[k] == pytest.approx(-nb * (rh[j] ** 2 - rh[k] ** 2) / 2, rel=1e-6)
    out = rh > R + 2 * dr
    assert np.ptp(rE[out]) < 1e-6 * np.abs(rE[out]).max()
    assert rE[out][0] == pytest.approx(-nb * R * R / 2, rel=5e-3)


def test_ex_scales_as_inverse_gamma_squared():
    """For gamma sigma_x far beyond the wall radius the potential tends to
    the column-by-column transverse one, so E_x -> (1/gamma^2) x a limit:
    doubling gamma quarters E_x."""
    cfg = _cfg(nx=128, nr=24)
    parts = bunch_particles(4000, 6, x0=51.2, sig_x=10.0, sig_r=2.0, p0=1.0)
    b1, b2 = np.sqrt(1 - 1e-6), np.sqrt(1 - 0.25e-6)  # gamma = 1000, 2000
    e1 = bunch.bunch_fields(cfg, parts, b1)[0]
    e2 = bunch.bunch_fields(cfg, parts, b2)[0]
    ratio = np.abs(e2).max() / np.abs(e1).max()
    assert ratio == pytest.approx(0.25, rel=1e-3)


def test_radial_self_force_cancels_to_inverse_gamma_squared(oracle_mod):
    """A co-moving electron inside the bunch feels q (E_r - beta B_theta) =
    q E_r / gamma^2 (the magnetic pull cancels the electric push): one
    momentum stage of the oracle in the bunch fields gives dp_r = -dt E_r /
    gamma^2 to within the offset of the B and E interpolation points."""
    cfg = _cfg(nx=160, nr=24)
    beta = 0.94
    gam = 1 / np.sqrt(1 - beta * beta)
    parts = bunch_particles(6000, 7, x0=64.0, sig_x=40.0, sig_r=3.0, p0=gam * beta, w_total=5.0)
    ex, er, bt, phi, qv = bunch.bunch_fields(cfg, parts, beta)
    s = oracle_mod.OracleSim(cfg)
    s.set_field("ex", ex)
    s.set_field("er", er)
    s.set_field("bt", bt)
    s.set_field("bt_bar", bt)
    r0 = 2.1
    s.set_particles(dict(x=np.array([64.3]), y=np.array([r0]), z=np.array([0.0]), px=np.array([gam * beta]),
                         py=np.array([0.0]), pz=np.array([0.0]), w=np.array([1e-9]), id=np.zeros(1, np.uint32)))
    s.momentum_chi()
    p = s.get_particles()

    def lin(f, ux, ur):  # this file's own bilinear interpolation at node coordinates
        i, j = int(np.floor(ux)), int(np.floor(ur))
        fx, fr = ux - i, ur - j
        return ((1 - fx) * ((1 - fr) * f[i, j] + fr * f[i, j + 1]) +
                fx * ((1 - fr) * f[i + 1, j] + fr * f[i + 1, j + 1]))

    ux, ur = 64.3 / cfg["dx"], r0 / cfg["dr"]
    e_p = lin(er, ux, ur - 0.5)        # E_r at (i, j+1/2)
    b_p = lin(bt, ux - 0.5, ur - 0.5)  # B_theta at (i+1/2, j+1/2)
    assert abs(e_p) > 1e-4
    # q = -1: dp_r = -dt (E_r - v_x B_theta), v_x = beta; about E_r / gamma^2
    expect = -cfg["dt"] * (e_p - beta * b_p)
    assert p["py"][0] == pytest.approx(expect, rel=2e-3)
    assert expect == pytest.approx(-cfg["dt"] * e_p / gam ** 2, rel=0.06)
    assert abs(p["py"][0]) < 0.2 * cfg["dt"] * abs(e_p)  # far below the unscreened push
