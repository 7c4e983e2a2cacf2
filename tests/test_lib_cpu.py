"""Host-side checks of the HIP library that need no GPU: the shared object
loads, exports every entry point the header declares, validates parameters
and reports footprints.  No kernel runs here."""
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def E():
    import paper_1912_04674_amd as E
    if not os.path.exists(E.envpic.LIB_PATH):
        pytest.skip("libenvpic.so not built")
    return E


def test_exports_every_declared_entry_point(E):
    header = open(os.path.join(ROOT, "include", "envpic.h")).read()
    declared = set(re.findall(r"\b(envpic_[a-z_0-9A-Z]+)\s*\(", header))
    assert len(declared) >= 20
    L = E.lib()
    for name in sorted(declared):
        assert hasattr(L, name), name
    assert set(E.envpic.EXPORTS) <= declared


def test_presets_match_workload_table(E):
    from inputs import C1, C2, C3, C5
    for preset, cfg in ((1, C1), (2, C2), (3, C3), (5, C5)):
        p = E.params_default(preset)
        q = E.make_params(cfg)
        for f, _ in E.Params._fields_:
            if f in ("seed",):
                continue
            a, b = getattr(p, f), getattr(q, f)
            assert a == pytest.approx(b), (preset, f, a, b)


def test_footprint_sizes(E):
    from inputs import C1, C3, C5
    f1 = E.footprint(C1, E.FP32_BULK)
    f64 = E.footprint(C1, E.FP64)
    assert 0 < f1 < f64 < 2 * f1 + (1 << 20)
    f3 = E.footprint(C3, E.FP32_BULK)
    npart = 4096 * 512 * 16
    # two particle buffers of 36 B plus scratch of 20 B per slot, slots for
    # 1/4 more particles than the window holds (overflow ranges of the
    # particles that change tile), and grids
    assert 92 * 1.25 * npart < f3 < 145 * npart
    f5 = E.footprint(C5, E.FP32_BULK)
    assert f5 < 20 * 2**30  # well inside one GPU's 288 GB


@pytest.mark.parametrize("bad", [
    dict(dt=0.85),                 # dt > dx: more than one cell per step
    dict(dt=0.69),                 # beyond the stability limit for dx = 0.8, dr = 1.5
    dict(nx=2),
    dict(n_modes=3),
    dict(ppc=(0, 2, 1)),
    dict(a0=-1.0),
    dict(n0=float("nan")),
    dict(x_c=float("inf")),
    dict(a0=float("nan")),
    dict(profile="perturb", perturb=1.5),
    dict(capacity=-5),
    dict(capacity=2**30),          # slots must stay below 2^30 (32-bit byte offsets)
])
def test_validation_rejects(E, bad):
    from inputs import C1, scaled
    with pytest.raises(E.EnvpicError) as ei:
        E.footprint(scaled(C1, **bad))
    assert ei.value.code == -1


def test_stability_guard_matches_oracle_growth(oracle_mod):
    """The unstable case the guard rejects (dt = 0.6 with dr = 0.75) really
    grows in the oracle, and the accepted neighbour does not."""
    base = dict(nx=64, nr=48, dx=0.8, dt=0.6, profile="none", a0=1.0, w0=10.0, tau=10.0,
                x_c=25.6, x_f=25.6)
    bad = oracle_mod.OracleSim(dict(base, dr=0.75))
    ok = oracle_mod.OracleSim(dict(base, dr=1.5))
    for _ in range(200):
        bad.envelope()
        ok.envelope()
    assert np.abs(bad.get_field("env")).max() > 1e3
    assert np.abs(ok.get_field("env")).max() < 1.5


def test_beam_diagnostics_null_sim_rejected(E):
    """Argument checks of the beam diagnostics run on the host before any
    device work: a NULL simulation or output is ENVPIC_EINVAL."""
    import ctypes
    out = np.zeros(len(E.envpic.BEAM_NAMES))
    dp = out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    assert E.lib().envpic_beam_diagnostics(None, 0.0, 1.0, 8, dp, None) == -1
    assert len(E.envpic.BEAM_NAMES) == 12


def test_sort_period_is_validated(E):
    """sort_every: 0 (default) or 1 .. 3, and at most 2 with quadratic
    shapes (the LDS halo holds that many steps of drift)."""
    from inputs import C2_SMALL_LIKE
    for v, order, ok in ((0, 1, True), (1, 1, True), (3, 1, True), (4, 1, False), (-1, 1, False),
                         (2, 2, True), (3, 2, False)):
        cfg = dict(C2_SMALL_LIKE, sort_every=v, shape_order=order)
        if ok:
            assert E.footprint(cfg) > 0
        else:
            with pytest.raises(E.EnvpicError):
                E.footprint(cfg)
