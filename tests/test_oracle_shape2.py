"""Pins of the oracle's quadratic (order-2) particle shapes (R26): the
weights, the parity ghosts below the axis in the gathers, the folded
deposits, and charge conservation of the order-2 Esirkepov current.

The checks use closed forms only: moments of the quadratic B-spline
(partition of unity, first moment u, variance 1/4), fields that are exactly
linear or even-quadratic through the axis with their own parity, the
ponderomotive kick in Phi ~ r^2, the chi sum rule, and the discrete Gauss
law and continuity equation against a charge density this file computes on
its own (quadratic weights, contributions below the axis folded onto their
mirror rows).
"""
import numpy as np
import pytest

from inputs import random_particles


def _cfg(**kw):
    c = dict(nx=32, nr=16, dx=0.8, dr=1.5, dt=0.6, profile="none", a0=0.0, shape_order=2)
    c.update(kw)
    return c


def _one(x, y, z, px=0.0, py=0.0, pz=0.0, w=1.0):
    return dict(x=np.array([x]), y=np.array([y]), z=np.array([z]), px=np.array([px]),
                py=np.array([py]), pz=np.array([pz]), w=np.array([w]), id=np.zeros(1, np.uint32))


def _kick(oracle_mod, cfg, fields, x, r, th=0.0):
    """Momentum after one momentum stage of a particle at rest: -dt F."""
    s = oracle_mod.OracleSim(cfg)
    for name, arr in fields.items():
        s.set_field(name, arr)
    s.set_particles(_one(x, r * np.cos(th), r * np.sin(th)))
    s.momentum_chi()
    P = s.get_particles()
    return np.array([P["px"][0], P["py"][0], P["pz"][0]])


def _grid(cfg, fn, complex_=False):
    i = np.arange(cfg["nx"] + 1)[:, None] * np.ones((1, cfg["nr"] + 1))
    j = np.ones((cfg["nx"] + 1, 1)) * np.arange(cfg["nr"] + 1)[None, :]
    return fn(i, j).astype(complex if complex_ else float)


def _variance(order, u):
    if order == 2:
        return 0.25
    f = u - np.floor(u)
    return f * (1 - f)


@pytest.mark.parametrize("order", [1, 2])
@pytest.mark.parametrize("ur", [5.3, 7.71, 9.5])
def test_shape_moments_in_r_primal_and_dual(oracle_mod, order, ur):
    """E_x on primal rows k (r = k dr) and E_r on half rows (r = (k + 1/2) dr)
    set to g(r/dr) for g = 1, u, u^2: the gathered value is the shape's
    moment, 1, u and u^2 + var, with var = 1/4 for the quadratic B-spline
    and f(1 - f) for the linear one (f the offset from the node below, in
    the node coordinate of that staggering: u for primal, u - 1/2 for half
    rows)."""
    cfg = _cfg(shape_order=order)
    dt, dr = cfg["dt"], cfg["dr"]
    x = 12.34
    cases = [(lambda u: u ** 0, 1.0, 1.0),
             (lambda u: u, ur, ur),
             (lambda u: u * u, ur * ur + _variance(order, ur), ur * ur + _variance(order, ur - 0.5))]
    for g, primal, half in cases:
        p = _kick(oracle_mod, cfg, {"ex": _grid(cfg, lambda i, j: g(j))}, x, ur * dr)
        assert -p[0] / dt == pytest.approx(primal, rel=1e-13)
        p = _kick(oracle_mod, cfg, {"er": _grid(cfg, lambda i, j: g(j + 0.5))}, x, ur * dr)
        assert -p[1] / dt == pytest.approx(half, rel=1e-13)


@pytest.mark.parametrize("order", [1, 2])
def test_shape_moments_in_x(oracle_mod, order):
    """E_r on primal columns = i^2 gives u_x^2 + var along x."""
    cfg = _cfg(shape_order=order)
    dt, dx = cfg["dt"], cfg["dx"]
    ux = 14.62
    p = _kick(oracle_mod, cfg, {"er": _grid(cfg, lambda i, j: i * i)}, ux * dx, 6.0)
    assert -p[1] / dt == pytest.approx(ux * ux + _variance(order, ux), rel=1e-13)


@pytest.mark.parametrize("ur", [0.05, 0.3, 0.49, 0.5, 0.8, 1.2, 1.7])
def test_axis_ghosts_follow_parity(oracle_mod, ur):
    """Near the axis the quadratic stencil reaches the row below it.  Fields
    that are exactly reproduced through the axis with their parity:
      mode-0 E_r = alpha r (odd, half rows: ghost -1/2 mirrors +1/2),
      mode-0 E_x = beta r^2 (even, primal rows: ghost -1 mirrors +1),
      mode-1 E_x = gamma r (odd), mode-1 E_theta = c (even)."""
    cfg = _cfg(n_modes=2)
    dt, dr = cfg["dt"], cfg["dr"]
    r = ur * dr
    x, th = 11.9, 0.9
    alpha, beta = 0.02, 0.003
    p = _kick(oracle_mod, cfg, {"er": _grid(cfg, lambda i, j: alpha * (j + 0.5) * dr)}, x, r, th)
    assert -p[1] / dt == pytest.approx(alpha * r * np.cos(th), rel=1e-12)
    assert -p[2] / dt == pytest.approx(alpha * r * np.sin(th), rel=1e-12)
    p = _kick(oracle_mod, cfg, {"ex": _grid(cfg, lambda i, j: beta * (j * dr) ** 2)}, x, r, th)
    assert -p[0] / dt == pytest.approx(beta * (r * r + 0.25 * dr * dr), rel=1e-12)
    gam = 0.01 - 0.004j
    p = _kick(oracle_mod, cfg, {"ex1": _grid(cfg, lambda i, j: gam * j * dr, True)}, x, r, th)
    # mode-1 field at azimuth theta: Re[F e^{-i theta}]
    assert -p[0] / dt == pytest.approx((gam * r * np.exp(-1j * th)).real, rel=1e-12)
    c1 = 0.015 + 0.01j
    p = _kick(oracle_mod, cfg, {"et1": _grid(cfg, lambda i, j: c1 + 0 * j, True)}, x, r, th)
    et = (c1 * np.exp(-1j * th)).real
    # theta-hat = (0, -sin, cos)
    assert -p[1] / dt == pytest.approx(-et * np.sin(th), rel=1e-12)
    assert -p[2] / dt == pytest.approx(et * np.cos(th), rel=1e-12)


@pytest.mark.parametrize("ur", [0.2, 0.6, 1.3, 4.4])
def test_ponderomotive_kick_in_quadratic_phi(oracle_mod, ur):
    """A = a r gives Phi = a^2 r^2 / 2; its centred radial difference on the
    nodes is exactly a^2 r_j (zero on the axis, odd below it), so a particle
    at rest is kicked by p_r = -dt a^2 r / (2 sqrt(1 + Phi_p)) with the
    gathered Phi_p = a^2 (r^2 + dr^2/4) / 2."""
    cfg = _cfg()
    dt, dr = cfg["dt"], cfg["dr"]
    a = 0.05
    A = _grid(cfg, lambda i, j: a * j * dr, True)
    r, th = ur * dr, -0.4
    p = _kick(oracle_mod, cfg, {"env": A, "env_prev": A}, 12.0, r, th)
    phi = 0.5 * a * a * (r * r + 0.25 * dr * dr)
    pr = -dt * a * a * r / (2 * np.sqrt(1 + phi))
    assert p[1] == pytest.approx(pr * np.cos(th), rel=1e-12)
    assert p[2] == pytest.approx(pr * np.sin(th), rel=1e-12)
    assert abs(p[0]) < 1e-17


def test_chi_sum_rule_with_axis_fold(oracle_mod):
    """sum_nodes chi V = sum_p w / gbar_p: the contributions below the axis
    are folded, none is lost (particles crowd the axis here)."""
    cfg = _cfg(nx=40, nr=16, a0=1.2, w0=8.0, tau=10.0, x_c=16.0, x_f=16.0)
    s = oracle_mod.OracleSim(cfg)
    parts = random_particles(cfg, 3000, seed=17, margin=2.5, r_frac=0.2)
    s.set_particles(parts)
    s.momentum_chi()
    g = s.get_gbar()
    assert g.max() > 1.05
    d = s.diagnostics()
    assert d["chi_v"] == pytest.approx(np.sum(parts["w"] / g), rel=1e-13)


def _vols(cfg):
    dx, dr, nr = cfg["dx"], cfg["dr"], cfg["nr"]
    j = np.arange(nr + 1)
    V = 2 * np.pi * j * dr * dr * dx
    V[0] = np.pi * dr * dr * dx / 4
    Ar = 2 * np.pi * (j + 0.5) * dr * dx
    return V, Ar


def _rho2(cfg, parts, shift=0):
    """Electron charge density on the primal nodes with quadratic weights
    (nearest node m, d = u - m: (1/2 - d)^2/2, 3/4 - d^2, (1/2 + d)^2/2),
    the row below the axis folded onto row 1."""
    nx, nr, dx, dr = cfg["nx"], cfg["nr"], cfg["dx"], cfg["dr"]
    V, _ = _vols(cfg)
    ux = parts["x"] / dx - shift
    ur = np.hypot(parts["y"], parts["z"]) / dr

    def w3(u):
        m = np.floor(u + 0.5)
        d = u - m
        return m.astype(int), [0.5 * (0.5 - d) ** 2, 0.75 - d * d, 0.5 * (0.5 + d) ** 2]

    mx, wx = w3(ux)
    mr, wr = w3(ur)
    rho = np.zeros((nx + 4, nr + 4))
    for a in range(3):
        for b in range(3):
            jj = mr - 1 + b
            jj = np.where(jj < 0, -jj, jj)
            np.add.at(rho, (mx - 1 + a + 1, jj), -parts["w"] * wx[a] * wr[b])
    return rho[1: nx + 2, : nr + 1] / V[None, :]


def _div(cfg, fx, fr):
    dx = cfg["dx"]
    V, Ar = _vols(cfg)
    d = np.zeros_like(fx)
    d[1:, :] += (fx[1:, :] - fx[:-1, :]) / dx
    flux = Ar[None, :] * fr
    d[:, 0] += flux[:, 0] / V[0]
    d[:, 1:] += (flux[:, 1:] - flux[:, :-1]) / V[None, 1:]
    return d


def test_gauss_law_and_continuity_order2(oracle_mod):
    """The order-2 Esirkepov current with the axis folds and the Yee update
    conserve charge exactly: div E^n = rho^n - rho^0 and (rho^{n+1} -
    rho^n)/dt + div J^{n+1/2} = 0 on every node but the outer x columns and
    r_max, with electrons crossing the axis."""
    cfg = _cfg(nx=64, nr=16, profile="uniform", n0=0.01, ppc=(2, 2, 1), a0=2.0, w0=6.0,
               tau=10.0, x_c=25.6, x_f=25.6)
    s = oracle_mod.OracleSim(cfg)
    rho0 = _rho2(cfg, s.get_particles())
    for _ in range(40):
        s.step(1)
    rho_n = _rho2(cfg, s.get_particles())
    s.momentum_chi()
    s.envelope()
    s.position_J()
    rho_n1 = _rho2(cfg, s.get_particles())
    divJ = _div(cfg, s.get_field("jx"), s.get_field("jr"))
    divE = _div(cfg, s.get_field("ex"), s.get_field("er"))
    sl = (slice(4, cfg["nx"] - 4), slice(0, cfg["nr"] - 1))
    scale = np.abs(rho0).max()
    assert np.abs(rho_n - rho0)[sl].max() > 1e-3 * scale
    assert np.abs(divE - (rho_n - rho0))[sl].max() < 1e-11 * scale
    cont = (rho_n1 - rho_n) / cfg["dt"] + divJ
    assert np.abs(cont)[sl].max() < 1e-11 * scale / cfg["dt"]


def test_mode1_symmetric_ring_deposits_zero_order2(oracle_mod):
    cfg = _cfg(nx=48, nr=12, n_modes=2, profile="uniform", n0=0.005, ppc=(1, 1, 4),
               a0=1.5, w0=6.0, tau=8.0, x_c=19.2, x_f=19.2)
    s = oracle_mod.OracleSim(cfg)
    s.step(6)
    s.momentum_chi()
    s.envelope()
    s.position_J()
    j0 = max(np.abs(s.get_field("jx")).max(), np.abs(s.get_field("jr")).max())
    assert j0 > 0
    for n in ("jx1", "jr1", "jt1"):
        assert np.abs(s.get_field(n)).max() < 1e-12 * j0


def test_mode1_deposit_folds_with_parity(oracle_mod):
    """One electron near the axis moving along x at azimuth theta_p: its
    mode-1 J_x stencil reaches the row below the axis, which folds onto row 1
    with the odd parity of an axial mode-1 component; the reconstructed
    J_x(r, theta_p) = Re[J_x1 e^{-i theta_p}] on rows 0..2 then equals the
    direct sum of its weights: row 0 gets 2 q w v S_0 / V_0, row 1 gets
    2 q w v (S_1 - S_-1) / V_1."""
    cfg = _cfg(nx=16, nr=8, n_modes=2)
    dx, dr = cfg["dx"], cfg["dr"]
    s = oracle_mod.OracleSim(cfg)
    th, ur, ux = 0.6, 0.3, 6.3
    px = 0.5
    s.set_particles(_one(ux * dx, ur * dr * np.cos(th), ur * dr * np.sin(th), px=px))
    s.position_J()
    jx1 = s.get_field("jx1")
    V, _ = _vols(cfg)
    v = px / np.sqrt(1 + px * px)
    um = ur  # the particle moves along x only: the mid-point radius is ur
    d = um - np.floor(um + 0.5)
    S = [0.5 * (0.5 - d) ** 2, 0.75 - d * d, 0.5 * (0.5 + d) ** 2]  # rows -1, 0, 1
    col = jx1.sum(axis=0) * np.exp(-1j * th)
    q = -1.0
    assert col[0].real == pytest.approx(2 * q * v * S[1] / V[0], rel=1e-12)
    assert col[1].real == pytest.approx(2 * q * v * (S[2] - S[0]) / V[1], rel=1e-12)
    assert np.abs(col[2:]).max() == 0.0
    assert np.abs(col.imag).max() < 1e-15 * np.abs(col).max()
