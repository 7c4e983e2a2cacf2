"""Parity of the quadratic-shape (order-2) HIP path, through the C ABI, with
the FP64 oracle's order-2 step (R26): stage by stage from random states that
crowd the axis (parity ghosts and folded deposits), whole runs with the
moving window and modes 0 and 1, a ragged grid, axis crossings and wall
reflections.  Bars as for the linear path: FP64 1e-9 (1e-12 per stage),
FP32-bulk 1e-4 on grids and 1e-3 on momenta (2e-5 per stage).
"""
import numpy as np
import pytest

from inputs import C2, random_grid, random_particles, scaled
from test_gpu_parity import (C2_SMALL, DEPOSIT_TOL_FP32, PRECS, RAGGED, compare_fields, compare_particles, ferr,
                             say, staggered)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def E():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1912_04674_amd as E
    E.lib()
    return E


def _prec(E, name):
    return E.FP64 if name == "fp64" else E.FP32_BULK


def _near_axis_and_bulk(cfg, seed):
    a = random_particles(cfg, 4000, seed=seed, margin=3, pmax=0.6)
    b = random_particles(cfg, 2000, seed=seed + 1, margin=3, pmax=0.6, r_frac=0.08)
    b["id"] = b["id"] + 4000
    return {k: np.concatenate([a[k], b[k]]) for k in a}


@pytest.mark.parametrize("modes", [1, 2])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_stage_parity_random_state_order2(E, oracle_mod, prec, modes):
    cfg = dict(nx=64, nr=32, dx=0.8, dr=1.5, dt=0.6, n_modes=modes, profile="none", a0=0.0, ppc=(2, 2, 1),
               shape_order=2)
    say("order-2 stage parity", prec, "modes", modes)
    g = E.Sim(cfg, _prec(E, prec))
    r = oracle_mod.OracleSim(cfg)
    parts = _near_axis_and_bulk(cfg, 121)
    g.set_particles(parts)
    r.set_particles(parts)
    fields = {"ex": random_grid(cfg, 1, 0.05), "er": random_grid(cfg, 2, 0.05),
              "bt": random_grid(cfg, 3, 0.05), "bt_bar": random_grid(cfg, 4, 0.05),
              "env": random_grid(cfg, 5, 0.8, True), "env_prev": random_grid(cfg, 6, 0.8, True)}
    if modes == 2:
        for k, n in enumerate(("ex1", "er1", "et1", "bx1", "br1", "bt1", "bx1_bar", "br1_bar", "bt1_bar")):
            fields[n] = random_grid(cfg, 10 + k, 0.02, True)
    for n, a in fields.items():
        g.set_field(n, staggered(n, a))
        r.set_field(n, staggered(n, a))
    tol = 1e-12 if prec == "fp64" else 2e-5
    g.momentum()
    r.momentum_chi()
    compare_particles(g.get_particles(), r.get_particles(), tol, 1e-12 if prec == "fp64" else 1e-5)
    compare_fields(g, r, tol, names=("chi",))
    g.envelope_step()
    r.envelope()
    g.position()
    r.position_J()
    compare_particles(g.get_particles(), r.get_particles(), tol, 1e-11 if prec == "fp64" else 1e-5)
    jn = ("jx", "jr") + (("jx1", "jr1", "jt1") if modes == 2 else ())
    for n in jn:
        e = ferr(g.get_field(n), r.get_field(n))
        say("deposit", n, e)
        assert e <= tol, (n, e)
    g.field_step()
    r.field_step()
    names = ("ex", "er", "bt", "bt_bar")
    if modes == 2:
        names += ("ex1", "er1", "et1", "bx1", "br1", "bt1", "bx1_bar", "br1_bar", "bt1_bar")
    for n in names:
        e = ferr(g.get_field(n), r.get_field(n))
        assert e <= tol, (n, e)


@pytest.mark.parametrize("prec,tf,tp", PRECS)
def test_window_modes01_parity_order2(E, oracle_mod, prec, tf, tp):
    """Moving window with injection, modes 0 and 1, up-ramp: 100 steps with
    quadratic shapes (re-sorted every second step)."""
    cfg = dict(C2_SMALL, shape_order=2)
    say("order-2 window + mode 1", prec)
    g = E.Sim(cfg, _prec(E, prec))
    r = oracle_mod.OracleSim(cfg)
    g.step(100)
    r.step(100)
    assert g.state() == r.state()
    compare_fields(g, r, tf, modes=2)
    compare_particles(g.get_particles(), r.get_particles(), tp, 1e-8 if prec == "fp64" else 1e-3)


@pytest.mark.parametrize("prec,tf,tp", PRECS)
def test_ragged_grid_parity_order2(E, oracle_mod, prec, tf, tp):
    cfg = dict(RAGGED, shape_order=2)
    say("order-2 ragged", prec)
    g = E.Sim(cfg, _prec(E, prec))
    r = oracle_mod.OracleSim(cfg)
    g.step(60)
    r.step(60)
    assert g.state() == r.state()
    compare_fields(g, r, tf, modes=2)
    compare_particles(g.get_particles(), r.get_particles(), tp, 1e-8 if prec == "fp64" else 1e-3)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_axis_crossing_and_wall_reflection_order2(E, oracle_mod, prec):
    cfg = dict(nx=48, nr=12, dx=0.8, dr=1.5, dt=0.6, n_modes=2, profile="none", a0=0.0, ppc=(1, 1, 1),
               shape_order=2)
    rng = np.random.default_rng(141)
    n = 400
    x = rng.uniform(8.0, 30.0, n)
    th = rng.uniform(-np.pi, np.pi, n)
    near = np.arange(n) < n // 2
    r = np.where(near, rng.uniform(0.05, 2.0, n), rng.uniform(16.0, 17.9, n))
    y, z = r * np.cos(th), r * np.sin(th)
    sgn = np.where(near, -1.0, 1.0)
    pr = sgn * rng.uniform(0.5, 3.0, n)
    pt = rng.uniform(-0.3, 0.3, n)
    parts = dict(x=x, y=y, z=z, px=rng.uniform(-0.2, 0.2, n), py=pr * np.cos(th) - pt * np.sin(th),
                 pz=pr * np.sin(th) + pt * np.cos(th), w=rng.uniform(0.5, 1.5, n) * 1e-3,
                 id=np.arange(n, dtype=np.uint32))
    g = E.Sim(cfg, _prec(E, prec))
    o = oracle_mod.OracleSim(cfg)
    g.set_particles(parts)
    o.set_particles(parts)
    g.step(12)
    o.step(12)
    tol = 1e-9 if prec == "fp64" else 1e-4
    compare_fields(g, o, tol, names=("chi", "ex", "er", "bt", "jx", "jr"), modes=2)
    compare_particles(g.get_particles(), o.get_particles(), 1e-9 if prec == "fp64" else 1e-3,
                      1e-9 if prec == "fp64" else 1e-3)


def test_order2_rejects_deferred_deposits(E):
    g = E.Sim(scaled(C2_SMALL, shape_order=2), E.FP64)
    with pytest.raises(E.EnvpicError) as ei:
        g.gather_push(E.MOMENTUM, defer=True)
    assert ei.value.code == -1
    g.step(2)  # the fused path still runs


@pytest.mark.parametrize("order", [1, 2])
def test_c2_full_window_100_steps(E, oracle_mod, order):
    """The 2048 x 256, modes 0-1, 8.4 M-particle LWFA workload (moving window,
    injection at the leading edge) for 100 steps in the benchmark's launch
    configuration, FP32-bulk and FP64 paths, against the oracle run on the
    whole window (threaded over the host's cores): every grid of both modes
    (the deposits of the FP32 path, chi and J, to DEPOSIT_TOL_FP32), every particle
    by id and the nine conserved sums."""
    import torch
    cfg = dict(C2, shape_order=order)
    nthr = oracle_mod.host_threads()
    say("C2 full window, 100 steps, order", order, "oracle threads", nthr)
    oracle_mod.set_threads(nthr)
    try:
        r = oracle_mod.OracleSim(cfg)
        r.step(100)
    finally:
        oracle_mod.set_threads(1)
    ref_parts = r.get_particles()
    dref = r.diagnostics()
    say("oracle done", r.state())
    for prec, tf, tj, tp in (("fp32", 1e-4, DEPOSIT_TOL_FP32, 1e-3), ("fp64", 1e-9, 1e-9, 1e-9)):
        say("gpu", prec)
        g = E.Sim(cfg, _prec(E, prec))
        g.step(100)
        assert g.state() == r.state()
        compare_fields(g, r, tf, modes=2, tol_j=tj)
        compare_particles(g.get_particles(), ref_parts, tp, 1e-3 if prec == "fp32" else 1e-8)
        dg = g.diagnostics()
        assert dg["count"] == dref["count"] and dg["nonfinite"] == 0
        for k in ("charge", "chi_v", "kin", "uem", "env2_v", "px"):
            assert abs(dg[k] - dref[k]) <= (2e-4 if prec == "fp32" else 1e-9) * abs(dref[k]), (k, dg[k], dref[k])
        g.close()
        del g
        torch.cuda.empty_cache()


@pytest.mark.parametrize("prec,tf,tp", PRECS)
def test_order2_with_filter_window_parity(E, oracle_mod, prec, tf, tp):
    """The paper's nonlinear-benchmark configuration on a small window:
    quadratic shapes and the 7-pass binomial current filter, modes 0 and 1,
    moving window with injection, 60 steps."""
    cfg = dict(C2_SMALL, shape_order=2, filter_passes=7)
    say("order-2 + filter window", prec)
    g = E.Sim(cfg, _prec(E, prec))
    r = oracle_mod.OracleSim(cfg)
    g.step(60)
    r.step(60)
    assert g.state() == r.state()
    compare_fields(g, r, tf, modes=2)
    compare_particles(g.get_particles(), r.get_particles(), tp, 1e-8 if prec == "fp64" else 1e-3)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_order2_checkpoint_and_graph_mode(E, prec):
    """2N steps equal N steps + save + load + N steps, and graph-mode chunks
    equal direct launches, with the two-step sort period of order 2."""
    cfg = dict(C2_SMALL, shape_order=2)
    P = _prec(E, prec)
    a = E.Sim(cfg, P)
    a.step(15)
    blob = a.save()
    a.step(16)
    b = E.Sim(cfg, P)
    b.load(blob)
    b.set_graph(5)
    b.step(16)
    assert a.state() == b.state()
    tol_f, tol_p = (1e-10, 1e-10) if prec == "fp64" else (1e-4, 1e-3)
    compare_fields(b, a, tol_f, names=("env", "env_prev", "chi", "ex", "er", "bt", "bt_bar"), modes=2)
    compare_particles(b.get_particles(), a.get_particles(), tol_p, 1e-8 if prec == "fp64" else 1e-3)


def test_beam_parameters_after_order2_run(E):
    """The beam-parameter pass on the state of an order-2 run equals the
    oracle's computation on the same particles."""
    from oracle import beam
    cfg = dict(C2_SMALL, shape_order=2, a0=3.0)
    g = E.Sim(cfg, E.FP32_BULK)
    g.step(50)
    parts = g.get_particles()
    for q in [(0.0, 0.05, 128), (1e-3, 2.0, 64)]:
        out, hist = g.beam(*q, with_hist=True)
        ref, rhist = beam.beam_parameters(parts, *q)
        assert ref["count"] > 0
        assert np.abs(hist - rhist).max() <= 1e-10 * np.abs(rhist).max()
        for k, v in ref.items():
            assert out[k] == v if k == "count" else abs(out[k] - v) <= 1e-9 * abs(v), (q, k, out[k], v)
