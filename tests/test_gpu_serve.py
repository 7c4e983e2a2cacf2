"""Scan serving on the GPU: jobs stepped together on their own streams inside
one arena give each the result it gets alone (FP32 tolerance: 1e-4 of the
field maximum, 1e-3 of the momentum maximum)."""
import sys

import numpy as np
import pytest

from inputs import c4_job, scaled

pytestmark = pytest.mark.gpu


def say(*a):
    print("[gpu-serve]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def E():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1912_04674_amd as E
    E.lib()
    return E


def _small_jobs(n):
    rng = np.random.default_rng(191204900)
    out = []
    for k in range(n):
        c = c4_job(k, rng)
        nx, nr = [(128, 32), (256, 32), (256, 64)][k % 3]
        lx = nx * 0.8
        out.append(scaled(c, name=f"serve{k}_{nx}x{nr}", nx=nx, nr=nr, x_c=lx - 40.0, x_f=lx - 40.0,
                          w0=min(c["w0"], 30.0), tau=20.0))
    return out


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_jobs_same_alone_and_in_the_mix(E, prec):
    from oracle import beam
    from paper_1912_04674_amd.serve import GpuBackend, ScanServer, DONE
    P = E.FP32_BULK if prec == "fp32" else E.FP64
    cfgs = _small_jobs(6)
    need = sum(E.footprint(c, P) for c in cfgs)
    be = GpuBackend(budget_bytes=need // 2 + (1 << 20), precision=P, full=True,  # not all fit at once
                    beam_query=(0.0, 0.05, 64))
    srv = ScanServer(be, chunk=7, depth=2)
    say("serving", prec, [c["name"] for c in cfgs])
    jobs = srv.run_trace(cfgs, [0.0, 0.0, 0.001, 0.002, 0.003, 0.004], steps=40, timeout=120)
    assert all(j.status == DONE for j in jobs), [(j.status, j.error) for j in jobs]
    assert max(j.admit for j in jobs) > min(j.finish for j in jobs)  # admitted as others ended
    tol_f, tol_p = (1e-4, 1e-3) if prec == "fp32" else (1e-10, 1e-10)
    for c, j in zip(cfgs, jobs):
        alone = E.Sim(c, P)
        alone.step(40)
        for n, v in j.result["fields"].items():
            ref = alone.get_field(n)
            e = float(np.abs(v - ref).max() / max(np.abs(ref).max(), 1e-300))
            assert e <= tol_f, (c["name"], n, e)
        a = alone.get_particles()
        b = j.result["particles"]
        oa, ob = np.argsort(a["id"]), np.argsort(b["id"])
        assert np.array_equal(a["id"][oa], b["id"][ob])
        pm = max(np.abs(a[k]).max() for k in ("px", "py", "pz")) or 1.0
        for k in ("px", "py", "pz"):
            assert np.abs(a[k][oa] - b[k][ob]).max() / pm <= tol_p, (c["name"], k)
        # the beam parameters returned with the job are those of its final particles
        ref, _ = beam.beam_parameters(b, *be.beam_query)
        assert ref["count"] > 0
        for k, v in ref.items():
            got = j.result["beam"][k]
            assert got == v if k == "count" else abs(got - v) <= 1e-9 * abs(v), (c["name"], k, got, v)
        alone.close()
    say("ok", prec)
