#!/usr/bin/env python
"""Throughput benchmark of the HIP cylindrical envelope PIC step (one GPU).

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload c2|c3|c5]

Prints one JSON line.  A step is one full PIC step (momentum pass with chi,
envelope update, position pass with J, fields, moving window with injection,
tile sort) of the whole workload, all inputs resident in HBM.  `value` is
particle pushes per second of the FP32-bulk path; the FP64 path, the
per-kernel HBM roofline and the CPU oracle baseline are reported beside it.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
for _p in (ROOT, os.path.join(ROOT, "tests"), os.path.join(ROOT, "oracle")):
    if _p not in sys.path:
        sys.path.insert(0, _p)

METRIC = "particle-pushes/s FP32 vs FP64 path at oracle tol; scan-job p50/p99 latency"
HBM_PEAK_GBS = 8000.0


def algorithmic_bytes(cfg, n_particles, prec_bytes=4):
    """Bytes the method must move per launch of the two particle kernels
    (each array read or written once; no sort, halo or re-read traffic).
    Per particle: momentum pass reads cell, offsets, azimuth, p, w (8 words)
    and writes p (3 words); position pass reads the same 8 words and writes
    cell, offsets, azimuth (4 words).  Per cell: the gathered grids and the
    deposited grids of each pass (mode 1 adds six complex gathers and three
    complex currents)."""
    w = prec_bytes
    cells = cfg["nx"] * cfg["nr"]
    m1 = cfg.get("n_modes", 1) >= 2
    mom_p = 4 + 7 * w + 3 * w                 # read 8 words, write p
    pos_p = 4 + 7 * w + 4 + 3 * w             # read 8 words, write cell + 3 offsets
    mom_c = 3 * w + 2 * w + w + (12 * w if m1 else 0)   # E_x, E_r, Bbar_t, A; chi; mode-1 gathers
    pos_c = 4 * w + 2 * w + (6 * w if m1 else 0)        # A^n, A^{n+1}; J_x, J_r; mode-1 J
    # field update per cell: mode 0 reads E_x, E_r, B_t, J_x, J_r and writes
    # E_x, E_r, B_t, Bbar_t (9 words); mode 1 reads six complex E/B and three
    # complex J and writes six complex E/B and three complex Bbar (18 complex)
    fld_c = 9 * w + (36 * w if m1 else 0)
    env_c = 7 * w                                       # A^n, A^{n-1}, chi read; A^{n+1} written
    return {"k_momentum": mom_p * n_particles + mom_c * cells,
            "k_position": pos_p * n_particles + pos_c * cells,
            "k_field": fld_c * cells, "k_envelope": env_c * cells,
            "per_particle": {"k_momentum": mom_p, "k_position": pos_p, "k_field": 0, "k_envelope": 0},
            "per_cell": {"k_momentum": mom_c, "k_position": pos_c, "k_field": fld_c, "k_envelope": env_c}}


def source_digest():
    """sha256 (first 16 hex digits) of the HIP sources, in name order."""
    d = os.path.join(ROOT, "paper_1912_04674_amd", "csrc")
    h = hashlib.sha256()
    for name in sorted(os.listdir(d)):
        if name.endswith((".hip", ".hpp")):
            h.update(name.encode())
            h.update(open(os.path.join(d, name), "rb").read())
    return h.hexdigest()[:16]


def traffic_record(kernel, workload):
    """Measured HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, scaled
    by a copy-kernel calibration) from profiles/, valid only while the kernel
    sources are unchanged."""
    path = os.path.join(ROOT, "profiles", f"traffic_{kernel}_{workload}.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    if rec.get("source_sha256_16") != source_digest():
        return None
    return rec.get("bytes_per_launch")


# Per-kernel times come from a pass after the timed region (the timed steps
# carry no events): HIP events around each stage on every step, for two full
# cycles of the sort schedule (a tile sort every third step, a cell-ordered
# one every 24th; every second and 16th with quadratic shapes), so each
# variant of the momentum pass counts with its share of the launches.
KERNEL_PASS_STEPS = 48
STAGE_KERNEL = {"momentum": "k_momentum", "envelope": "k_envelope", "position": "k_position", "field": "k_field"}


# beam parameters of the final state (Table BeamParams): electrons above
# 1e-3 m_e c^2 of kinetic energy, 512 bins up to 20 m_e c^2
BEAM_QUERY = (1e-3, 20.0, 512)


def time_beam(sim, torch, reps=20):
    """Average wall time of the synchronous beam-parameter call (histogram,
    peak and two moment passes over every particle, read back to the host)."""
    out = sim.beam(*BEAM_QUERY)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        sim.beam(*BEAM_QUERY)
    dt = (time.perf_counter() - t0) / reps
    return {"ms": 1e3 * dt, "query": list(BEAM_QUERY), "count": out["count"], "e_peak": out["e_peak"],
            "charge": out["charge"], "rel_spread": out["rel_spread"], "emit_y": out["emit_y"]}


def run_gpu(E, torch, cfg, prec, steps, warmup, per_kernel=True, beam=False):
    """Warm up, then time `steps` steps issued by the library's own loop
    (envpic_step_n) on the simulation's stream.  With `per_kernel`, a pass of
    KERNEL_PASS_STEPS more steps follows with HIP events around each stage
    on that stream on every step (the library's stage timing)."""
    stream = torch.cuda.current_stream()
    sim = E.Sim(cfg, prec, stream=stream)
    sim.step(warmup)
    torch.cuda.synchronize()
    n0 = sim.state()[2]
    t_start = torch.cuda.Event(enable_timing=True)
    t_end = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    wall0 = time.perf_counter()
    t_start.record(stream)
    sim.step(steps)
    t_end.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    n1 = sim.state()[2]
    gpu_ms = t_start.elapsed_time(t_end)
    out = {"wall_s": wall, "gpu_ms": gpu_ms, "particles": 0.5 * (n0 + n1), "n0": n0, "n1": n1}
    if per_kernel:
        sim.set_timing(True, every=1)
        sim.step(KERNEL_PASS_STEPS)
        t = sim.timing()
        sim.set_timing(False)
        assert all(v[1] == KERNEL_PASS_STEPS for v in t.values()), t
        out["stage_ms"] = {k: round(v[0], 5) for k, v in t.items()}
        out["kernel_ms"] = {STAGE_KERNEL[k]: v[0] for k, v in t.items()}
        out["kernel_pass_particles"] = sim.state()[2]
    if beam:
        out["beam"] = time_beam(sim, torch)
    sim.close()
    del sim
    torch.cuda.empty_cache()
    return out


def run_serving(E, prec, budget_bytes, steps=300, repeat=0, burst=False):
    """The scan-serving trace: 64 jobs arriving as a Poisson process (mean
    4 jobs/s; repeat r draws jobs and arrivals from seed base + 99 + 10 r),
    grids from {512x64, 1024x128, 2048x256}, 300 steps each, served by
    continuous batching inside one arena of `budget_bytes`.  With `burst`
    every job arrives at t = 0 (the server saturated)."""
    import numpy as np
    from inputs import BASE_SEED, c4_trace
    from paper_1912_04674_amd.serve import DONE, GpuBackend, ScanServer, latency_stats
    cfgs, arrivals = c4_trace(seed=BASE_SEED + 99 + 10 * repeat)
    if burst:
        arrivals = np.zeros_like(arrivals)
    be = GpuBackend(budget_bytes, precision=prec, lineout=True)
    # load the kernels' code objects before the trace starts
    warm = ScanServer(be, chunk=5)
    warm.run_trace([dict(cfgs[0], nx=64, nr=16, x_c=20.0, x_f=20.0)], [0.0], steps=3)
    srv = ScanServer(be, max_slots=32, chunk=25, depth=2)
    jobs = srv.run_trace(cfgs, arrivals, steps=steps, timeout=600)
    ok = [j for j in jobs if j.status == DONE]
    makespan = max(j.finish for j in jobs) - min(j.arrival for j in jobs)
    pushes = sum(j.result["diag"]["count"] * j.steps for j in ok)
    st = latency_stats(jobs)
    by_grid = {}
    for j in ok:
        by_grid.setdefault(f"{j.cfg['nx']}x{j.cfg['nr']}", []).append(j.latency)
    del be, srv, warm
    return {"jobs": len(jobs), "done": len(ok), "p50_s": st["p50"], "p99_s": st["p99"], "mean_s": st["mean"],
            "makespan_s": makespan, "aggregate_pushes_per_s": pushes / makespan,
            "median_latency_s_by_grid": {k: float(sorted(v)[(len(v) - 1) // 2]) for k, v in sorted(by_grid.items())},
            "budget_bytes": budget_bytes, "arrival_seed": int(BASE_SEED + 99 + 10 * repeat), "burst": burst}


def cpu_model():
    """CPU model name of the host (from /proc/cpuinfo)."""
    try:
        for ln in open("/proc/cpuinfo"):
            if ln.lower().startswith("model name"):
                return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _oracle_rate(pyoracle, cfg, steps, threads):
    """Pushes and cell updates per second of the oracle on cfg (creation not
    timed)."""
    pyoracle.set_threads(threads)
    try:
        sim = pyoracle.OracleSim(cfg)
        n0 = sim.n_particles
        t0 = time.perf_counter()
        sim.step(steps)
        dt = time.perf_counter() - t0
        n1 = sim.n_particles
        sim.close()
    finally:
        pyoracle.set_threads(1)
    return {"pushes_per_s": 0.5 * (n0 + n1) * steps / dt, "cell_updates_per_s": cfg["nx"] * cfg["nr"] * steps / dt,
            "particles": int(0.5 * (n0 + n1)), "steps": steps, "seconds": round(dt, 3)}


def cpu_baseline(cfg, cols=256, steps=100):
    """The FP64 oracle, as it stands, on the host's cores: the particle loops
    on 1 thread and on every core this process may use (at most 16, the host
    share of one GPU).  The headline sample is a slab of the benchmarked
    workload (its last `cols` cell columns, where the pulse is; full radius,
    same loading) for `steps` steps (a fifth as many on 1 thread); beside
    it, on all threads: the mode-0 parity workload in full (100 steps), a
    256-column slab of the bandwidth workload (20 steps), the leading
    256-column slab of the largest workload (5 steps) and one scan job per
    grid size for 30 of its 300 steps (the job's CPU latency is scaled from
    those)."""
    import pyoracle
    from inputs import C1, C3, C5, C4_GRIDS, c4_job, scaled
    import numpy as np
    pyoracle.build()
    nthr = pyoracle.host_threads()
    start = cfg["nx"] - cols
    sub = scaled(cfg, nx=cols, start_col=start)
    one = _oracle_rate(pyoracle, sub, max(4, steps // 5), 1)
    many = _oracle_rate(pyoracle, sub, steps, nthr)
    others = {"c1_parity_256x32 (full, 100 steps)": _oracle_rate(pyoracle, C1, 100, nthr),
              "c3_bandwidth_4096x512 columns [1920, 2176), 20 steps":
                  _oracle_rate(pyoracle, scaled(C3, nx=256, start_col=1920), 20, nthr),
              "c5_extreme_8192x768 columns [7936, 8192), 5 steps":
                  _oracle_rate(pyoracle, scaled(C5, nx=256, start_col=7936), 5, nthr)}
    rng = np.random.default_rng(7)
    for nx, nr in C4_GRIDS:
        job = c4_job(0, rng)
        job = scaled(job, nx=nx, nr=nr, x_c=nx * 0.8 - 90.0, x_f=nx * 0.8 - 90.0, name=f"c4_{nx}x{nr}")
        r = _oracle_rate(pyoracle, job, 30, nthr)
        r["job_latency_s_300_steps"] = round(r["seconds"] * 300 / 30, 2)
        others[f"c4 scan job {nx}x{nr} (30 of 300 steps)"] = r
    return {"value": many["pushes_per_s"], "unit": "particle-pushes/s", "cores": nthr, "kind": "oracle",
            "sample": f"{cfg['name']} columns [{start}, {cfg['nx']}) x {cfg['nr']} rows, {many['particles']} particles, "
                      f"{steps} steps, FP64, {nthr} threads ({many['seconds']:.1f} s)",
            "cpu_model": cpu_model(),
            "one_thread": {"value": one["pushes_per_s"], "cores": 1,
                           "sample": f"same slab, {one['steps']} steps ({one['seconds']:.1f} s)"},
            "cell_updates_per_s": many["cell_updates_per_s"],
            "other_samples": others}


def bunch_solve_line(workload):
    """The field initialisation of an injected bunch (gamma = 7.09) on the
    workload's grid: conjugate-gradient iterations, wall time of the
    synchronous call, and the algorithmic bytes of the iterations (per
    unknown and iteration: stencil 16 B, update 48 B, direction 24 B)."""
    import numpy as np
    import torch
    import paper_1912_04674_amd as E
    from inputs import C2, C3, C5, bunch_particles
    base = {"c2": C2, "c3": C3, "c5": C5}[workload]
    cfg = dict(base, capacity=base["nx"] * base["nr"] * int(np.prod(base["ppc"])) + 300_000)
    torch.cuda.set_device(0)
    g = E.Sim(cfg, E.FP32_BULK)
    plasma = g.get_particles()
    beta = 0.99
    nb = 200_000
    b = bunch_particles(nb, 11, x0=(cfg["nx"] - 600) * cfg["dx"], sig_x=8.0, sig_r=3.0,
                        p0=beta / np.sqrt(1 - beta * beta), w_total=20.0, id0=1 << 26)
    g.set_particles({k: np.concatenate([plasma[k], b[k]]) for k in plasma})
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    it, res = g.bunch_fields(1 << 26, (1 << 26) + nb, beta, tol=1e-12)
    dt = time.perf_counter() - t0
    n = (cfg["nx"] - 1) * cfg["nr"]
    return {"workload": cfg["name"], "unknowns": n, "bunch_particles": nb, "beta": beta, "iterations": it,
            "relative_residual": res, "ms": 1e3 * dt, "us_per_iteration": 1e6 * dt / max(it, 1),
            "alg_GBps": 88.0 * n * it / dt / 1e9}


def progress(*a):
    """One line on stderr as each part of the benchmark ends."""
    print("[bench]", *a, file=sys.stderr, flush=True)



def copy_seconds(torch, n, reps, variant=None):
    """Seconds per plain device copy of n bytes (read n, write n), averaged
    over reps copies after one untimed copy: torch's copy (variant None) or
    the library's streaming copy kernel (variant 0-3)."""
    import paper_1912_04674_amd as E
    src = torch.ones(n, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)

    def once():
        if variant is None:
            dst.copy_(src)
        else:
            E.stream_copy(dst, src, variant)
    once()
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        once()
    b.record()
    torch.cuda.synchronize()
    dt = a.elapsed_time(b) * 1e-3 / reps
    del src, dst
    return dt


def copy_ceiling(torch, n=512 * 2**20, reps=10):
    """The measured streaming ceiling: the library's hand-written copy kernel
    (16 B per lane, 4 or 8 accesses in flight, ordinary or non-temporal) and
    torch's copy, each moving n bytes in and n out (n above the 256 MB
    Infinity Cache)."""
    names = {0: "hip_copy_u4", 1: "hip_copy_u8", 2: "hip_copy_u4_nt", 3: "hip_copy_u8_nt", None: "torch_copy"}
    rates = {names[v]: round(2 * n / copy_seconds(torch, n, reps, v) / 1e9, 1) for v in (0, 1, 2, 3, None)}
    best = max((k for k in rates if k.startswith("hip")), key=lambda k: rates[k])
    return {"GBps": rates[best], "frac_of_peak": round(rates[best] / HBM_PEAK_GBS, 4), "kernel": best,
            "bytes": 2 * n, "all_GBps": rates}


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="c2", choices=["c2", "c3", "c5"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-serving", action="store_true", help="skip the scan-serving trace")
    ap.add_argument("--serving-budget-gib", type=float, default=4.0)
    ap.add_argument("--filter-passes", type=int, default=0,
                    help="binomial current filter passes (the paper's nonlinear benchmark uses 7)")
    ap.add_argument("--shape-order", type=int, default=1, choices=[1, 2],
                    help="particle shape order of gather and deposit (2: quadratic B-spline)")
    ap.add_argument("--bunch-solve", action="store_true",
                    help="only time the self-consistent field solve of a 200 000-particle relativistic "
                         "bunch added to the workload's plasma (one JSON line)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MiB",
                    help="only run a plain device copy of this many MiB, 10 times (reference for "
                         "the FETCH_SIZE / WRITE_SIZE counters)")
    ap.add_argument("--copy-variant", type=int, default=0, choices=[0, 1, 2, 3],
                    help="the library copy kernel's variant for --copy-calibration")
    ap.add_argument("--serving-repeats", type=int, default=1,
                    help="run the scan trace this many times (arrival seeds base + 99 + 10 r)")
    ap.add_argument("--serving-burst", action="store_true",
                    help="also serve the 64 jobs of the trace all arriving at t = 0 (saturation)")
    args = ap.parse_args()
    if args.copy_calibration:
        import torch
        n = args.copy_calibration * 2**20
        dt = copy_seconds(torch, n, 10, variant=args.copy_variant)
        print(json.dumps({"copy_bytes_read": n, "copy_bytes_written": n, "seconds": dt,
                          "GBps_read_plus_write": 2 * n / dt / 1e9}))
        return
    if args.bunch_solve:
        print(json.dumps(bunch_solve_line(args.workload)))
        return
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU; the multi-GPU x-slab "
                                   "decomposition is a design only, not built", "n_gpus": args.gpus}))
        sys.exit(2)

    import torch
    import paper_1912_04674_amd as E
    from inputs import C2, C3, C5
    cfg = {"c2": C2, "c3": C3, "c5": C5}[args.workload]
    if args.filter_passes:
        cfg = dict(cfg, filter_passes=args.filter_passes, name=f"{cfg['name']}_filter{args.filter_passes}")
    if args.shape_order == 2:
        cfg = dict(cfg, shape_order=2, name=f"{cfg['name']}_order2")
    E.lib()
    torch.cuda.set_device(0)

    r32 = run_gpu(E, torch, cfg, E.FP32_BULK, args.steps, args.warmup, beam=True)
    progress(f"fp32 timed run done: {1e3 * r32['wall_s'] / args.steps:.4f} ms/step")
    pushes = r32["particles"] * args.steps
    value = pushes / r32["wall_s"]
    cells = cfg["nx"] * cfg["nr"]
    ab = algorithmic_bytes(cfg, r32["kernel_pass_particles"], 4)
    kernels = {}
    for k, ms in r32["kernel_ms"].items():
        kernels[k] = {"avg_ms": ms, "alg_bytes": ab[k], "GBps": ab[k] / (ms * 1e-3) / 1e9,
                      "frac": ab[k] / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS}
    # every kernel runs once per step: the dominant one takes the most time
    dom = max(kernels, key=lambda k: kernels[k]["avg_ms"])
    achieved = kernels[dom]["GBps"]
    tr = traffic_record(dom, cfg["name"])
    ceiling = copy_ceiling(torch)
    progress(f"copy ceiling {ceiling['all_GBps']}")
    roofline = {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": tr,
                "copy_ceiling": ceiling,
                "alg_bytes_per_particle": ab["per_particle"][dom], "alg_bytes_per_cell": ab["per_cell"][dom],
                "kernel_times": f"HIP events around each stage on every step of {KERNEL_PASS_STEPS} steps "
                                "after the timed region (two cycles of the sort schedule)",
                "kernels": {k: {kk: round(vv, 4) if isinstance(vv, float) else vv for kk, vv in v.items()}
                            for k, v in kernels.items()}}
    extra = {"cell_updates_per_s": cells * args.steps / r32["wall_s"],
             "gpu_event_ms_per_step": r32["gpu_ms"] / args.steps,
             "stage_avg_ms": r32["stage_ms"],
             "particles_start_end": [r32["n0"], r32["n1"]]}
    # the beam pass reads cell, momentum and weight of every particle three
    # times (histogram, means, centred moments): 60 B per particle
    bm = r32["beam"]
    bm["alg_bytes"] = 3 * (4 + 3 * 4 + 4) * r32["n1"]
    bm["GBps_alg_incl_host_sync"] = bm["alg_bytes"] / (bm["ms"] * 1e-3) / 1e9
    extra["beam_diag"] = bm
    if args.workload == "c3" and cfg.get("sort_every") == 1:
        # the same workload with the default sort period (every third step)
        r3 = run_gpu(E, torch, dict(cfg, sort_every=0), E.FP32_BULK, args.steps, args.warmup)
        extra["sort_every_3"] = {"ms_per_step": 1e3 * r3["wall_s"] / args.steps,
                                 "pushes_per_s": r3["particles"] * args.steps / r3["wall_s"],
                                 "stage_avg_ms": r3["stage_ms"]}
        progress("c3 with the default sort period done")
    if not args.no_fp64:
        s64 = max(10, args.steps // 5)
        r64 = run_gpu(E, torch, cfg, E.FP64, s64, min(args.warmup, 5), per_kernel=False)
        extra["fp64_pushes_per_s"] = r64["particles"] * s64 / r64["wall_s"]
        extra["fp64_steps"] = s64
        extra["fp32_over_fp64"] = value / extra["fp64_pushes_per_s"]
        progress("fp64 run done")
    line = {
        "metric": METRIC, "value": value, "unit": "particle-pushes/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": 1e3 * r32["wall_s"] / args.steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": cfg["name"], "grid": [cfg["nx"], cfg["nr"]], "modes": cfg["n_modes"],
                   "filter_passes": int(cfg.get("filter_passes", 0)),
                   "shape_order": int(cfg.get("shape_order", 1)),
                   "ppc": list(cfg["ppc"]), "particles": int(r32["particles"]),
                   "moving_window": bool(cfg["moving_window"]), "precision": "fp32-bulk (fp64 axis rows)"},
        "roofline": roofline,
    }
    if not args.no_serving:
        budget = int(args.serving_budget_gib * 2**30)
        line["serving"] = {"trace": "64 jobs, Poisson 4 jobs/s, grids {512x64, 1024x128, 2048x256}, m=0, "
                                    "2x2x2 ppc, 300 steps, window on"}
        precs = [("fp32", E.FP32_BULK)] + ([] if args.no_fp64 else [("fp64", E.FP64)])
        for name, prec in precs:
            runs = []
            for r in range(args.serving_repeats):
                runs.append(run_serving(E, prec, budget, repeat=r))
                progress(f"{name} serving trace {r} done")
            line["serving"][name] = runs[0] if len(runs) == 1 else runs
            if args.serving_burst:
                line["serving"][name + "_burst"] = run_serving(E, prec, budget, burst=True)
                progress(f"{name} serving burst done")
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(cfg)
        progress("cpu baseline done")
    line["extra"] = extra
    print(json.dumps(line))


if __name__ == "__main__":
    main()
