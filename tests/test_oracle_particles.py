"""Pins of the oracle's particle stages (gather, ponderomotive Boris push,
position push, chi deposit) against closed forms, invariants and brute force.

Equations of motion: Sec. 2, Eq. EquationsOfMotion; Cartesian form and the
modified Boris pusher: Sec. 3, Eq. motion_equations_cartesian; chi: Sec. 2
(definition after Eq. EquationsOfMotion) and Sec. 3 (projection).
"""
import numpy as np
import pytest

from inputs import random_particles, random_grid


def _vac(nx=32, nr=16, dx=0.8, dr=1.5, dt=0.6, **kw):
    cfg = dict(nx=nx, nr=nr, dx=dx, dr=dr, dt=dt, profile="none", a0=0.0)
    cfg.update(kw)
    return cfg


def _one(x, y, z, px=0.0, py=0.0, pz=0.0, w=1.0):
    return dict(x=np.array([x]), y=np.array([y]), z=np.array([z]), px=np.array([px]),
                py=np.array([py]), pz=np.array([pz]), w=np.array([w]),
                id=np.zeros(1, np.uint32))


def _const(cfg, v, complex_=False):
    return np.full((cfg["nx"] + 1, cfg["nr"] + 1), v, dtype=complex if complex_ else float)


# ------------------------------------------------------------------ chi --
def test_chi_uniform_plasma_at_rest_exact(oracle_mod):
    """Uniform loading at rest, Phi = 0: chi = n0 exactly at interior nodes
    (weights ~ r with linear shapes sum to r_j on both sides of a node), and
    the closed forms of the boundary rows: 1.5 n0 on the axis (2 radial
    particles per cell, axis volume pi dr^2 dx/4), n0 (N_r - 3/8)/(2 N_r) at
    r_max, n0/2 on the x end columns."""
    n0 = 0.002
    cfg = _vac(nx=24, nr=12, profile="uniform", n0=n0, ppc=(2, 2, 1))
    s = oracle_mod.OracleSim(cfg)
    s.momentum_chi()
    chi = s.get_field("chi")
    assert np.allclose(chi[1:-1, 1:-1], n0, rtol=1e-13, atol=0)
    assert np.allclose(chi[1:-1, 0], 1.5 * n0, rtol=1e-13, atol=0)
    nr = cfg["nr"]
    assert np.allclose(chi[1:-1, nr], n0 * (nr - 3 / 8) / (2 * nr), rtol=1e-13, atol=0)
    assert np.allclose(chi[0, 1:-1], 0.5 * n0, rtol=1e-13, atol=0)


@pytest.mark.parametrize("ppc", [(2, 2, 1), (1, 3, 2), (2, 4, 4)])
def test_chi_uniform_any_loading(oracle_mod, ppc):
    n0 = 0.0017
    cfg = _vac(nx=16, nr=10, profile="uniform", n0=n0, ppc=ppc)
    s = oracle_mod.OracleSim(cfg)
    s.momentum_chi()
    chi = s.get_field("chi")
    assert np.allclose(chi[1:-1, 1:-1], n0, rtol=1e-13, atol=0)


def test_chi_sum_rule_and_charge(oracle_mod):
    """sum_nodes chi V = sum_p w / gbar_p and total charge = -sum w, with a
    laser present and random momenta (gbar != 1)."""
    cfg = _vac(nx=48, nr=20, a0=1.5, w0=12.0, tau=10.0, x_c=19.2, x_f=19.2)
    s = oracle_mod.OracleSim(cfg)
    parts = random_particles(cfg, 4000, seed=7, margin=1.5)
    s.set_particles(parts)
    s.momentum_chi()
    g = s.get_gbar()
    assert g.min() > 1.0 and g.max() > 1.2
    d = s.diagnostics()
    assert d["chi_v"] == pytest.approx(np.sum(parts["w"] / g), rel=1e-13)
    assert d["charge"] == pytest.approx(-parts["w"].sum(), rel=1e-14)


# ---------------------------------------------------------------- Boris --
def test_pure_static_E_kick_exact(oracle_mod):
    """E only: the electron momentum changes by -E dt exactly (two half kicks,
    identity rotation); E_x along x, E_r along r-hat = (0, cos, sin)."""
    cfg = _vac()
    s = oracle_mod.OracleSim(cfg)
    s.set_field("ex", _const(cfg, 0.03))
    s.set_field("er", _const(cfg, -0.02))
    th = 0.7
    r = 7.3
    s.set_particles(_one(10.1, r * np.cos(th), r * np.sin(th), px=0.1, py=-0.2, pz=0.05))
    s.momentum_chi()
    p = s.get_particles()
    dt = cfg["dt"]
    assert p["px"][0] == pytest.approx(0.1 - 0.03 * dt, abs=1e-15)
    assert p["py"][0] == pytest.approx(-0.2 + 0.02 * dt * np.cos(th), abs=1e-15)
    assert p["pz"][0] == pytest.approx(0.05 + 0.02 * dt * np.sin(th), abs=1e-15)


def test_pure_B_rotation_with_phi(oracle_mod):
    """B_theta only, uniform Phi: |p| is conserved, the momentum turns about
    theta-hat = (0, -sin, cos) by 2 atan(B dt / (2 gbar)) with gbar including
    Phi, and the turn follows dp/dt = -v x B (electron)."""
    cfg = _vac()
    s = oracle_mod.OracleSim(cfg)
    b0, a = 0.4, 0.9
    s.set_field("bt_bar", _const(cfg, b0))
    s.set_field("env", _const(cfg, a, True))
    s.set_field("env_prev", _const(cfg, a, True))
    th, r = 1.1, 9.0
    p0 = np.array([0.3, 0.2, -0.4])
    s.set_particles(_one(12.3, r * np.cos(th), r * np.sin(th), *p0))
    s.momentum_chi()
    P = s.get_particles()
    p1 = np.array([P["px"][0], P["py"][0], P["pz"][0]])
    dt = cfg["dt"]
    assert np.linalg.norm(p1) == pytest.approx(np.linalg.norm(p0), rel=1e-14)
    that = np.array([0.0, -np.sin(th), np.cos(th)])
    assert p1 @ that == pytest.approx(p0 @ that, abs=1e-15)
    gbar = np.sqrt(1 + p0 @ p0 + a * a / 2)
    q0, q1 = p0 - (p0 @ that) * that, p1 - (p1 @ that) * that
    ang = np.arccos(np.clip(q0 @ q1 / (np.linalg.norm(q0) * np.linalg.norm(q1)), -1, 1))
    assert ang == pytest.approx(2 * np.arctan(b0 * dt / (2 * gbar)), rel=1e-12)
    B = b0 * that
    assert (p1 - p0) @ (-np.cross(p0 / gbar, B)) > 0


def test_ponderomotive_kick_direction_and_factor(oracle_mod):
    """Phi = alpha x + beta, particle at rest: p = -dt alpha / (2 sqrt(1 + Phi))
    along x (kick down the intensity gradient, factor 1/2 from gbar =
    sqrt(1 + p^2 + Phi))."""
    cfg = _vac()
    s = oracle_mod.OracleSim(cfg)
    alpha, beta = 0.01, 0.2
    xg = np.arange(cfg["nx"] + 1)[:, None] * cfg["dx"] * np.ones((1, cfg["nr"] + 1))
    phi = alpha * xg + beta
    s.set_field("env", np.sqrt(2 * phi).astype(complex))
    xp = 11.37
    s.set_particles(_one(xp, 3.0, 4.0))
    s.momentum_chi()
    P = s.get_particles()
    expect = -cfg["dt"] * alpha / (2 * np.sqrt(1 + alpha * xp + beta))
    assert P["px"][0] == pytest.approx(expect, rel=1e-12)
    assert abs(P["py"][0]) < 1e-16 and abs(P["pz"][0]) < 1e-16


def test_Lx_conserved_in_mode0_fields(oracle_mod):
    """Mode-0 forces lie in span(x-hat, r-hat) and the rotation is about
    theta-hat, and the drift is straight: L_x = y p_z - z p_y of each particle
    is an exact invariant of the discrete map (away from the r_max wall)."""
    cfg = _vac(nx=48, nr=24)
    s = oracle_mod.OracleSim(cfg)
    for f, sd in (("ex", 1), ("er", 2), ("bt_bar", 3)):
        s.set_field(f, random_grid(cfg, sd, amp=0.01))
    A = random_grid(cfg, 4, amp=0.3, complex_=True)
    parts = random_particles(cfg, 500, seed=11, margin=12, r_frac=0.5, pmax=0.04)
    s.set_particles(parts)
    L0 = parts["y"] * parts["pz"] - parts["z"] * parts["py"]
    for _ in range(150):
        s.set_field("env", A)
        s.set_field("env_prev", A)
        s.momentum_chi()
        s.position_J()
    P = s.get_particles()
    L1 = P["y"] * P["pz"] - P["z"] * P["py"]
    assert len(P["id"]) > 400
    assert np.abs(L1 - L0[P["id"]]).max() < 1e-13 * max(1.0, np.abs(L0).max())
    moved = np.abs(P["px"] - parts["px"][P["id"]]).max()
    assert moved > 1e-3


# ---------------------------------------------------- luminal invariant --
def _luminal(oracle_mod, dx, dt, a0=1.0, sig=10.0):
    nx, nr = int(round(200 / dx)), 8
    cfg = _vac(nx=nx, nr=nr, dx=dx, dr=1.5, dt=dt)
    s = oracle_mod.OracleSim(cfg)
    x0 = 100.0
    s.set_particles(_one(x0, 0.0, 0.0))
    xg = np.arange(nx + 1) * dx
    xc0 = x0 - 5 * sig

    def env(t):
        a = a0 * np.exp(-(((xg - xc0 - t) / sig) ** 2))
        return np.repeat(a[:, None], nr + 1, axis=1).astype(complex)

    err = pxmax = 0.0
    for n in range(int(round(10 * sig / dt))):
        t = n * dt
        s.set_field("env", env(t))
        s.set_field("env_prev", env(t - dt))
        s.momentum_chi()
        s.set_field("env", env(t + dt))
        s.set_field("env_prev", env(t))
        xold = s.get_particles()["x"][0]
        s.position_J()
        P = s.get_particles()
        xh, th = 0.5 * (xold + P["x"][0]), t + 0.5 * dt
        phi = 0.5 * (a0 * np.exp(-(((xh - xc0 - th) / sig) ** 2))) ** 2
        g = np.sqrt(1 + P["px"][0] ** 2 + P["py"][0] ** 2 + P["pz"][0] ** 2 + phi)
        err = max(err, abs(g - P["px"][0] - 1))
        pxmax = max(pxmax, P["px"][0])
    return err, pxmax, P["px"][0]


def test_luminal_invariant(oracle_mod):
    """Plane envelope moving at c, E = B = 0, electron from rest: the
    Hamiltonian gbar(x - t, p) gives gbar - p_x = 1 exactly, p_x = |A|^2/4 at
    the peak (a0^2/4 for a0 = 1), and p_x -> 0 after the pulse.  The discrete
    map converges to it (dx and dt refined together)."""
    errs = []
    for dx in (0.5, 0.25, 0.125):
        e, pxm, pxf = _luminal(oracle_mod, dx, 0.8 * dx)
        errs.append(e)
        assert pxm == pytest.approx(0.25, abs=2e-3)
        assert abs(pxf) < 2e-4
    assert errs[0] < 1e-3
    assert errs[0] / errs[1] > 1.8 and errs[1] / errs[2] > 1.8


# ------------------------------------------------------ brute force RK4 --
def _fields(x, r):
    """Smooth static test fields (E_r, B_theta vanish on the axis)."""
    ex = 0.02 * np.sin(0.2 * x) * np.exp(-(r**2) / 200.0)
    er = 0.015 * (r / 10.0) * np.cos(0.15 * x) * np.exp(-(r**2) / 200.0)
    bt = 0.01 * (r / 10.0) * np.exp(-(r**2) / 300.0)
    phi = 0.3 * np.exp(-((x - 12.0) ** 2) / 40.0 - r**2 / 150.0)
    dphix = phi * (-2 * (x - 12.0) / 40.0)
    dphir = phi * (-2 * r / 150.0)
    return ex, er, bt, phi, dphix, dphir


def _rhs(y):
    x, yy, zz, px, py, pz = y
    r = np.hypot(yy, zz)
    c, s = (yy / r, zz / r) if r > 0 else (1.0, 0.0)
    ex, er, bt, phi, gx, gr = _fields(x, r)
    g = np.sqrt(1 + px * px + py * py + pz * pz + phi)
    v = np.array([px, py, pz]) / g
    E = np.array([ex, er * c, er * s])
    B = bt * np.array([0.0, -s, c])
    G = np.array([gx, gr * c, gr * s])
    dp = -(E + np.cross(v, B)) - G / (2 * g)
    return np.concatenate([v, dp])


def _reference(y0, t0, t1):
    """High-order adaptive integration of the continuous equations of motion
    (dense output on [t0, t1])."""
    from scipy.integrate import solve_ivp
    sol = solve_ivp(lambda t, y: _rhs(y), (t0, t1), y0, method="DOP853", rtol=1e-12,
                    atol=1e-14, dense_output=True)
    return sol.sol


def _pic_track(oracle_mod, dx, dt, y0, T):
    dr = dx
    nx, nr = int(round(30 / dx)), int(round(20 / dr))
    cfg = _vac(nx=nx, nr=nr, dx=dx, dr=dr, dt=dt)
    s = oracle_mod.OracleSim(cfg)
    i = np.arange(nx + 1)[:, None]
    j = np.arange(nr + 1)[None, :]
    full = lambda f: np.broadcast_to(f, (nx + 1, nr + 1)).copy()
    s.set_field("ex", full(_fields((i + 0.5) * dx, j * dr)[0]))
    s.set_field("er", full(_fields(i * dx, (j + 0.5) * dr)[1]))
    s.set_field("bt_bar", full(_fields((i + 0.5) * dx, (j + 0.5) * dr)[2]))
    A = full(np.sqrt(2 * _fields(i * dx, j * dr)[3]).astype(complex))
    # leap-frog start: p^{-1/2} from the reference trajectory
    ym = _reference(y0, 0.0, -0.5 * dt)(-0.5 * dt)
    s.set_particles(_one(y0[0], y0[1], y0[2], ym[3], ym[4], ym[5]))
    for _ in range(int(round(T / dt))):
        s.set_field("env", A)
        s.set_field("env_prev", A)
        s.momentum_chi()
        s.position_J()
    P = s.get_particles()
    return np.array([P["x"][0], P["y"][0], P["z"][0]]), np.array([P["px"][0], P["py"][0], P["pz"][0]])


def test_pusher_vs_ode_brute_force(oracle_mod):
    """A single particle in smooth static fields sampled on the grid follows the
    continuous equations of motion (integrated to 1e-12 by an adaptive
    8th-order Runge-Kutta method):
    the difference shrinks at least linearly when dx and dt are halved."""
    y0 = np.array([6.0, 3.0, -2.0, 0.05, 0.02, 0.03])
    T = 12.0
    errs = []
    for dx in (0.4, 0.2, 0.1):
        dt = 0.75 * dx
        x, p = _pic_track(oracle_mod, dx, dt, y0, T)
        ref = _reference(y0, 0.0, T)
        errs.append(np.abs(x - ref(T)[:3]).max() + np.abs(p - ref(T - 0.5 * dt)[3:]).max())
    assert errs[0] < 5e-3
    assert errs[0] / errs[1] > 1.8 and errs[1] / errs[2] > 1.8
