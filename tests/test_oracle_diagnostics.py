"""Pins of the oracle's FP64 conserved-sum diagnostics and of its plasma
density profiles, against closed forms (no oracle arithmetic retyped).

Diagnostics (the sums listed with the hot path):
  * U_EM, the low-frequency field energy.  A field set on the grid must carry
    the energy (1/2) integral |E|^2 + |B|^2 dV of the continuous field it
    samples.  Along x a sine that vanishes at both ends sums exactly to half
    the length on either staggering.  Along r the node volumes of the axis
    row (pi dr^2 dx / 4) and of the others (2 pi r_j dr dx), and the half-row
    volumes 2 pi r_{j+1/2} dr dx, integrate 1 - (r/R)^2 with known defects:
    -pi dr^2/4 on the primal rows and +pi dr^2/4 on the half rows (the
    Euler-Maclaurin remainder of the trapezoid rule, worked out in the test).
    A uniform transverse field E_y = E0 f(x) h(r) written as azimuthal mode 1
    (E_r1 = E0 f h, E_theta1 = -i E0 f h, Sec. 2 mode convention) therefore
    carries exactly (1/2) E0^2 integral f^2 h^2 dV: the two defects cancel.
    This fixes the weight 1/2 of mode 0 and 1/4 of mode 1 (a field
    Re[F e^{-i theta}] has a mean square |F|^2/2 over the azimuth).
  * kinetic energy sum w (gamma - 1) and momentum sum w p_x: particles with
    momenta of rational gamma; electrons at rest kicked by a uniform static
    E_x for one step (the Lorentz force of Eq. EquationsOfMotion).
  * L_x = sum w (y p_z - z p_y): a ring of electrons with azimuthal momentum
    carries w r p_theta each.
  * sum |A|^2 V of the initial Gaussian envelope: the paraxial beam carries
    pi a0^2 w0^2 / 2 per unit length at every distance from focus; the node
    volumes add dr^2 / (6 W^2) - dr^4 / (15 W^4) - ... of it (W the local
    waist).

Profiles (the workloads' plasma): each cell holds ppc_x ppc_r ppc_theta
particles whose weights are n(x_lab) times the volume each stands for, so a
cell column's weights sum to n pi R^2 dx per x sub-position (midpoint radii
integrate r dr exactly).  The ramp rises linearly from 0 at x = 0 to n0 at
x = ramp_len; the perturbed density is n0 (1 + eps (2u - 1)) with u the
counter-based uniform of the cell; the bump is n0 (1 + exp(-((x - x_b)/w_b)^2)).
"""
import numpy as np
import pytest

NX, NR, DX, DR = 40, 24, 0.8, 1.5


def vac(oracle_mod, modes=2, nx=NX, nr=NR):
    return oracle_mod.OracleSim(dict(nx=nx, nr=nr, dx=DX, dr=DR, dt=0.6, n_modes=modes,
                                     profile="none", a0=0.0))


def grids(nx=NX, nr=NR):
    i = np.arange(nx + 1)[:, None]
    j = np.arange(nr + 1)[None, :]
    R = nr * DR
    sx_p = np.sin(np.pi * i / nx) * np.ones((1, nr + 1))           # primal in x: i dx
    sx_d = np.sin(np.pi * (i + 0.5) / nx) * np.ones((1, nr + 1))   # dual in x: (i + 1/2) dx
    h_p = np.sqrt(np.clip(1 - (j * DR / R) ** 2, 0, None)) * np.ones((nx + 1, 1))
    h_d = np.sqrt(np.clip(1 - ((j + 0.5) * DR / R) ** 2, 0, None)) * np.ones((nx + 1, 1))
    return sx_p, sx_d, h_p, h_d


def trim(a, dual_x, dual_r):
    a = np.array(a, copy=True)
    if dual_x:
        a[-1, :] = 0
    if dual_r:
        a[:, -1] = 0
    return a


# ----------------------------------------------------------------- U_EM --
def test_field_energy_mode0_closed_forms(oracle_mod):
    """E_r = E0 sin(pi x / L) and B_theta = B0 sin(pi x / L), uniform in r:
    (1/2) E0^2 (L/2) pi R^2 exactly.  E_x = E0 sin(pi x/L) sqrt(1 - (r/R)^2):
    (1/2) E0^2 (L/2) (pi R^2 / 2)(1 - 1/(2 nr^2)) (the primal-row defect)."""
    L, R = NX * DX, NR * DR
    sx_p, sx_d, h_p, _ = grids()
    for name, f, dual_x, dual_r in (("er", sx_p, False, True), ("bt", sx_d, True, True)):
        s = vac(oracle_mod, modes=1)
        a = 0.37
        s.set_field(name, trim(a * f, dual_x, dual_r))
        got = s.diagnostics()["uem"]
        want = 0.5 * a * a * (L / 2) * np.pi * R * R
        assert got == pytest.approx(want, rel=1e-13), name
    s = vac(oracle_mod, modes=1)
    a = 0.21
    s.set_field("ex", trim(a * sx_d * h_p, True, False))
    got = s.diagnostics()["uem"]
    want = 0.5 * a * a * (L / 2) * (np.pi * R * R / 2) * (1 - 1 / (2 * NR * NR))
    assert got == pytest.approx(want, rel=1e-13)


def test_field_energy_mode1_uniform_transverse_field(oracle_mod):
    """E_y = E0 f(x) h(r) as mode 1 (E_r1 = E0 f h, E_theta1 = -i E0 f h) and
    the same for B_y (B_r1, B_theta1): the energy is (1/2) E0^2 integral of
    f^2 h^2 over the cylinder, exactly, with h = sqrt(1 - (r/R)^2)."""
    L, R = NX * DX, NR * DR
    sx_p, sx_d, h_p, h_d = grids()
    exact = (L / 2) * (np.pi * R * R / 2)  # integral of f^2 h^2 dV
    e0, b0 = 0.29, 0.17
    s = vac(oracle_mod)
    s.set_field("er1", trim(e0 * sx_p * h_d, False, True).astype(complex))
    s.set_field("et1", -1j * e0 * sx_p * h_p)
    assert s.diagnostics()["uem"] == pytest.approx(0.5 * e0 * e0 * exact, rel=1e-13)
    s = vac(oracle_mod)
    s.set_field("br1", trim(b0 * sx_d * h_p, True, False).astype(complex))
    s.set_field("bt1", -1j * trim(b0 * sx_d * h_d, True, True))
    assert s.diagnostics()["uem"] == pytest.approx(0.5 * b0 * b0 * exact, rel=1e-13)
    # both at once, plus a mode-0 E_r: energies add
    s = vac(oracle_mod)
    s.set_field("er1", trim(e0 * sx_p * h_d, False, True).astype(complex))
    s.set_field("et1", -1j * e0 * sx_p * h_p)
    s.set_field("br1", trim(b0 * sx_d * h_p, True, False).astype(complex))
    s.set_field("bt1", -1j * trim(b0 * sx_d * h_d, True, True))
    s.set_field("er", trim(e0 * sx_p, False, True))
    want = 0.5 * (e0 * e0 + b0 * b0) * exact + 0.5 * e0 * e0 * (L / 2) * np.pi * R * R
    assert s.diagnostics()["uem"] == pytest.approx(want, rel=1e-13)


def test_field_energy_mode1_axial_components(oracle_mod):
    """E_x = E0 f(x) h(r) cos(theta) (mode-1 E_x1 = E0 f h on primal rows) and
    B_x = B0 f(x) h(r) cos(theta) (B_x1 on half rows): (1/2) E0^2 (L/2)
    (pi R^2 / 4) times 1 - 1/(2 nr^2) and 1 + 1/(2 nr^2) respectively."""
    L, R = NX * DX, NR * DR
    sx_p, sx_d, h_p, h_d = grids()
    cont = (L / 2) * (np.pi * R * R / 4)
    s = vac(oracle_mod)
    s.set_field("ex1", trim(0.4 * sx_d * h_p, True, False).astype(complex))
    assert s.diagnostics()["uem"] == pytest.approx(0.5 * 0.16 * cont * (1 - 1 / (2 * NR * NR)), rel=1e-13)
    s = vac(oracle_mod)
    s.set_field("bx1", (0.4j * trim(sx_p * h_d, False, True)))
    assert s.diagnostics()["uem"] == pytest.approx(0.5 * 0.16 * cont * (1 + 1 / (2 * NR * NR)), rel=1e-13)


# ------------------------------------------------ kinetic energy, P_x, L_x --
def _set(s, x, y, z, px, py, pz, w):
    n = len(x)
    s.set_particles(dict(x=np.asarray(x, float), y=np.asarray(y, float), z=np.asarray(z, float),
                         px=np.asarray(px, float), py=np.asarray(py, float), pz=np.asarray(pz, float),
                         w=np.asarray(w, float), id=np.arange(n, dtype=np.uint32)))


def test_kinetic_energy_of_known_momenta(oracle_mod):
    """|p| = 3/4 gives gamma - 1 = 1/4; |p| = 4/3 gives 2/3; |p| = 1e-4 gives
    p^2/2 - p^4/8 (no cancellation allowed); |p| = 1000 gives
    sqrt(1000001) - 1.  Weights 1, 2, 3, 4: P_x = 0.75 + 3 p_x3."""
    s = vac(oracle_mod, modes=1)
    x = [10.0, 12.0, 14.0, 16.0]
    y = [3.0, -2.0, 0.5, 5.0]
    z = [1.0, 4.0, -6.0, 0.0]
    px = [0.75, 0.0, 0.6e-4, 0.0]
    py = [0.0, 0.8, 0.0, 600.0]
    pz = [0.0, 16.0 / 15.0, 0.8e-4, -800.0]
    w = [1.0, 2.0, 3.0, 4.0]
    _set(s, x, y, z, px, py, pz, w)
    d = s.diagnostics()
    p3 = 1e-4
    kin = 1 * 0.25 + 2 * (2.0 / 3.0) + 3 * (p3 ** 2 / 2 - p3 ** 4 / 8) + 4 * (np.sqrt(1000001.0) - 1)
    assert d["kin"] == pytest.approx(kin, rel=1e-14)
    assert d["px"] == pytest.approx(0.75 + 3 * 0.6e-4, rel=1e-14)
    assert d["count"] == 4
    assert d["charge"] == pytest.approx(-10.0, rel=1e-15)
    # the small-momentum particle alone: relative precision of p^2/2
    s = vac(oracle_mod, modes=1)
    _set(s, [10.0], [1.0], [0.0], [1e-7], [0.0], [0.0], [1.0])
    assert s.diagnostics()["kin"] == pytest.approx(0.5e-14, rel=1e-12)


def test_uniform_field_kick_momentum_and_energy(oracle_mod):
    """Electrons (q = -1) at rest in a uniform static E_x = E0, no envelope:
    after one momentum stage every p = -E0 dt x, so P_x = -E0 dt sum w and
    the kinetic energy is (sqrt(1 + (E0 dt)^2) - 1) sum w."""
    rng = np.random.default_rng(5)
    s = vac(oracle_mod, modes=2)
    n = 200
    x = rng.uniform(2 * DX, (NX - 2) * DX, n)
    r = rng.uniform(0.0, (NR - 1) * DR, n)
    th = rng.uniform(0, 2 * np.pi, n)
    w = rng.uniform(0.5, 1.5, n)
    _set(s, x, r * np.cos(th), r * np.sin(th), np.zeros(n), np.zeros(n), np.zeros(n), w)
    e0, dt = 0.05, 0.6
    s.set_field("ex", trim(np.full((NX + 1, NR + 1), e0), True, False))
    s.momentum_chi()
    d = s.diagnostics()
    assert d["px"] == pytest.approx(-e0 * dt * w.sum(), rel=1e-12)
    assert d["kin"] == pytest.approx((np.sqrt(1 + (e0 * dt) ** 2) - 1) * w.sum(), rel=1e-12)
    assert abs(d["lx"]) < 1e-15 * w.sum()


def test_angular_momentum_of_a_rotating_ring(oracle_mod):
    """Electrons on a ring of radius r0 moving along theta-hat with p_theta:
    L_x = sum w r0 p_theta; a single electron at (y, z) = (0, r0) moving along
    +y has L_x = -w r0 p (right-handed sense about +x)."""
    s = vac(oracle_mod, modes=1)
    m, r0, pt = 48, 7.3, 0.35
    th = 2 * np.pi * (np.arange(m) + 0.3) / m
    w = 1.0 + 0.01 * np.arange(m)
    _set(s, np.full(m, 15.0), r0 * np.cos(th), r0 * np.sin(th), np.full(m, 0.2),
         -pt * np.sin(th), pt * np.cos(th), w)
    assert s.diagnostics()["lx"] == pytest.approx(r0 * pt * w.sum(), rel=1e-13)
    s = vac(oracle_mod, modes=1)
    _set(s, [15.0], [0.0], [r0], [0.0], [0.5], [0.0], [2.0])
    assert s.diagnostics()["lx"] == pytest.approx(-2.0 * r0 * 0.5, rel=1e-14)


# ------------------------------------------------------- sum |A|^2 V --
@pytest.mark.parametrize("w0,xf_off", [(20.0, 0.0), (12.0, 60.0)])
def test_envelope_norm_of_the_initial_pulse(oracle_mod, w0, xf_off):
    """The paraxial beam a0 exp(-r^2/(w0^2 q))/q carries pi a0^2 w0^2 / 2 per
    unit length at any distance from focus (|A|^2 is a Gaussian of waist
    W = w0 |q| and height a0^2/|q|^2).  On the node volumes each column adds
    dr^2/(6 W^2) - dr^4/(15 W^4) - 2 dr^6/(63 W^6) of it: the axis row's
    pi dr^2/4 against the trapezoid rule's end corrections (Euler-Maclaurin
    with the Bernoulli numbers 1/6, -1/30, 1/42), worked out for a Gaussian.  Along x, the pulse exp(-2 xi^2/sigma^2) summed on the
    nodes is its integral to machine precision."""
    nx, nr, dx, dr = 320, 64, 0.8, 1.5
    a0, tau = 0.7, 30.0
    xc = 0.5 * nx * dx
    xf = xc + xf_off
    s = oracle_mod.OracleSim(dict(nx=nx, nr=nr, dx=dx, dr=dr, dt=0.6, n_modes=1, profile="none",
                                  a0=a0, w0=w0, tau=tau, x_c=xc, x_f=xf))
    got = s.diagnostics()["env2_v"]
    sig = tau / (2 * np.sqrt(np.log(2)))
    x = np.arange(nx + 1) * dx
    zr = w0 * w0 / 2
    W2 = w0 * w0 * (1 + ((x - xf) / zr) ** 2)
    col = np.pi * a0 * a0 * w0 * w0 / 2 * np.exp(-2 * (x - xc) ** 2 / sig ** 2)
    want = np.sum(col * (1 + dr * dr / (6 * W2) - dr ** 4 / (15 * W2 * W2)
                         - 2 * dr ** 6 / (63 * W2 ** 3))) * dx
    assert got == pytest.approx(want, rel=2e-9)
    # the axis correction is visible at this tolerance: without it the sum
    # would be off by about dr^2 / (6 w0^2)
    plain = np.sum(col) * dx
    assert abs(got / plain - 1) > 1000 * 2e-9


# -------------------------------------------------------------- profiles --
def _column_weights(s, nx, dx, start_col=0):
    p = s.get_particles()
    col = np.floor(p["x"] / dx + 1e-9).astype(int) - start_col
    return np.bincount(col, weights=p["w"], minlength=nx)[:nx], p


def _expected_columns(nfun, nx, dx, nr, dr, ppc_x, start_col=0):
    R = nr * dr
    out = np.zeros(nx)
    for c in range(nx):
        for a in range(ppc_x):
            xl = (start_col + c + (a + 0.5) / ppc_x) * dx
            out[c] += nfun(xl) * np.pi * R * R * dx / ppc_x
    return out


def test_ramp_profile_column_charge(oracle_mod):
    """Linear up-ramp 0 -> n0 over lab x in [0, ramp_len], then n0: every
    column's weights sum to n pi R^2 dx over its x sub-positions, and chi at
    interior nodes follows the linear ramp exactly (a cloud-in-cell deposit
    of a linear density is exact)."""
    nx, nr, n0, rl = 60, 12, 0.003, 20.0
    cfg = dict(nx=nx, nr=nr, dx=DX, dr=DR, dt=0.6, n_modes=1, ppc=(2, 2, 2), profile="ramp",
               n0=n0, ramp_len=rl, a0=0.0, seed=7)
    s = oracle_mod.OracleSim(cfg)

    def n(x):
        return 0.0 if x <= 0 else (n0 * x / rl if x < rl else n0)

    got, _ = _column_weights(s, nx, DX)
    want = _expected_columns(n, nx, DX, nr, DR, 2)
    np.testing.assert_allclose(got, want, rtol=1e-13, atol=1e-18)
    s.momentum_chi()
    chi = s.get_field("chi")
    for i in range(1, nx):
        xi = i * DX
        if xi < rl - DX:  # both neighbouring cells on the linear part
            np.testing.assert_allclose(chi[i, 1:nr], n(xi), rtol=1e-12)


def test_perturbed_profile_cell_charge(oracle_mod):
    """n0 (1 + eps (2u - 1)) per cell, u the counter-based uniform (stream 2)
    of the cell: each cell's weights sum to that density times the annulus
    volume 2 pi r_{j+1/2} dr dx; the densities fill [n0 (1-eps), n0 (1+eps)]
    with the mean and variance of a uniform deviate."""
    nx, nr, n0, eps, seed = 64, 32, 0.001, 0.01, 123
    cfg = dict(nx=nx, nr=nr, dx=DX, dr=DR, dt=0.6, n_modes=1, ppc=(2, 2, 1), profile="perturb",
               n0=n0, perturb=eps, a0=0.0, seed=seed)
    s = oracle_mod.OracleSim(cfg)
    p = s.get_particles()
    col = np.floor(p["x"] / DX + 1e-9).astype(int)
    row = np.floor(np.hypot(p["y"], p["z"]) / DR + 1e-9).astype(int)
    cw = np.zeros((nx, nr))
    np.add.at(cw, (col, row), p["w"])
    vol = 2 * np.pi * (np.arange(nr)[None, :] + 0.5) * DR * DR * DX
    dens = cw / vol
    u = np.array([[oracle_mod.uniform(seed, 2, c, j) for j in range(nr)] for c in range(nx)])
    np.testing.assert_allclose(dens, n0 * (1 + eps * (2 * u - 1)), rtol=1e-12)
    v = dens / n0 - 1
    assert v.min() >= -eps and v.max() <= eps
    m = v.size
    assert abs(v.mean()) < 4 * eps / np.sqrt(3 * m)
    assert v.var() == pytest.approx(eps * eps / 3, rel=0.1)


def test_bump_profile_column_charge(oracle_mod):
    """n0 (1 + exp(-((x - x_b)/w_b)^2)): twice the plateau at the bump centre,
    n0 (1 + 1/e) one width away, the plateau far from it; column sums as for
    the ramp.  A window shifted by start_col loads the same lab columns."""
    nx, nr, n0, xb, wb = 80, 10, 0.0015, 30.0, 8.0
    for start in (0, 25):
        cfg = dict(nx=nx, nr=nr, dx=DX, dr=DR, dt=0.6, n_modes=1, ppc=(2, 2, 1), profile="bump",
                   n0=n0, bump_x=xb, bump_w=wb, a0=0.0, seed=9, start_col=start)
        s = oracle_mod.OracleSim(cfg)
        got, _ = _column_weights(s, nx, DX, start_col=start)
        want = _expected_columns(lambda x: n0 * (1 + np.exp(-((x - xb) / wb) ** 2)), nx, DX, nr, DR, 2, start)
        np.testing.assert_allclose(got, want, rtol=1e-13)
    R = nr * DR
    per_len = lambda x: n0 * (1 + np.exp(-((x - xb) / wb) ** 2)) * np.pi * R * R
    assert per_len(xb) == pytest.approx(2 * n0 * np.pi * R * R)
    assert per_len(xb + wb) == pytest.approx(n0 * (1 + np.exp(-1)) * np.pi * R * R)
