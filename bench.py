"""Benchmark: staggered FFT phase-field fracture solve on one MI355X.

Headline workload ("batched"): 64 independent realizations of a 512x512
periodic microstructure, E = max(1 + 0.2 z, 0.5) with z a unit-variance
Gaussian random field of correlation length 16 px (seeds 3000..3063), AT1,
strain-spectral split, l = 2 px, crack-set irreversibility, uniaxial-strain
ramp of 200 load steps to 1.5 eps_M; FP32 fields with FP64 reductions; all
realizations in one batched launch per kernel, independent per-problem
progression, launch plans from the shipped autotuner cache.

A "step" is one load step (alternating minimisation to Tol_AM: mechanics
Newton-CG + phase-field BCCG, Algorithm 2) of every realization.  The ramp's
early steps run untimed to reach the window (preparation), then W warmup
steps, then exactly K timed steps.  value = (mechanics CG + BCCG
iterations) x grid points / seconds of the timed steps, inputs resident in
HBM.  The library's device-clock kernel timers run during the timed steps
(they cost about 3% of the kernel time, so `value` is slightly pessimistic)
and give the per-kernel launch times of the roofline object; the timed steps
are bracketed by roctxProfilerResume / Pause inside a roctx range
(`bench_timed`; the large leg's timed steps: `bench_large_timed`), so that
`rocprofv3 --selected-regions --kernel-trace --stats` profiles exactly them.

The whole run keeps to a wall-clock budget (--budget seconds from the start
of the process): the headline runs first, then the secondary legs in order,
each only if its minimum time still fits, each bounded by what is left; legs
that did not fit are listed under "skipped".  Exactly one JSON line is
printed on stdout.

Secondary legs (same JSON line):
  cpu_baseline  the FP64 NumPy oracle on the host: a bounded window of
                mechanics CG and BCCG iterations per realization, started
                from the GPU state after the timed steps, on one core and on
                all cores (one realization per core)
  plain_gpu     the plain single-instance path (256x256, one problem, host
                check after every tick, no graph) over its 200-step ramp
                (AT1 spectral, the headline's model; vs_plain = value / its
                value)
  serving       continuous batching of load-step requests over resident
                problems of mixed grid sizes at staggered ramp positions:
                saturation rate, then p50/p99 latency (from arrival) and
                throughput under Poisson arrivals
  large         one 2048x2048 problem, l = 1 px, load steps through crack
                nucleation
  variants      model and evolution variants on 16 x 256^2
"""

import argparse
import json
import os
import subprocess
import sys
import time

T_START = time.time()
ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "grid-pt CG iters/s & HBM GB/s, batched FP32 vs plain GPU @1e-4 err; p50/p99"
HBM_PEAK_GBS = 8000.0
KERNELS = ("rowfwd", "col", "rowinv")


def log(*a):
    print(f"[bench {time.time() - T_START:6.1f}s]", *a, file=sys.stderr, flush=True)


class _Roctx:
    """roctx markers: a named range around the timed steps, and profiler
    resume / pause around them for `rocprofv3 --selected-regions`; no-ops
    when the library is absent."""

    def __init__(self):
        import ctypes
        self.lib = None
        for name in ("librocprofiler-sdk-roctx.so.1", "libroctx64.so"):
            try:
                self.lib = ctypes.CDLL(name)
                break
            except OSError:
                continue
        self.ok = self.lib is not None and hasattr(self.lib, "roctxProfilerResume")
        if self.ok:
            self.lib.roctxProfilerResume.argtypes = [ctypes.c_uint64]
            self.lib.roctxProfilerPause.argtypes = [ctypes.c_uint64]

    # resume before the push and pop before the pause: a marker issued while
    # the profiler is paused is not recorded
    def begin(self, name):
        if self.ok:
            self.lib.roctxProfilerResume(0)
            self.lib.roctxRangePushA(name.encode())

    def end(self):
        if self.ok:
            self.lib.roctxRangePop()
            self.lib.roctxProfilerPause(0)


ROCTX = _Roctx()


def left(args):
    return args.budget - (time.time() - T_START)


def iters(stats):
    cg = sum(s["cg_iters"] for row in stats for s in row)
    pf = sum(s["bccg_iters"] for row in stats for s in row)
    return cg, pf


def kernel_figures(pr):
    """Per-kernel launch time from the device-clock timers: a launch's span,
    from its first work-group's start to the next kernel's first start (its
    work-group activity plus its drain and end-of-kernel write-back, plus the
    next dispatch).  A profiler's kernel-trace duration lies between the
    activity and the span, within 2% of the span on the benchmark's window
    (the dispatch itself is short), so the span is the launch time used, a
    slight overestimate."""
    kt = {k: pr["kernel_span_ms"][k] for k in KERNELS}
    dom = max(KERNELS, key=lambda k: kt[k])
    nl = max(pr["launches"][dom], 1)
    ms = kt[dom]
    return {"kernel_ms": kt, "dominant": dom, "avg_launch_us": ms * 1e3 / nl,
            "alg_bytes_per_launch": pr["alg_bytes"][dom] / nl,
            "achieved_GBs": pr["alg_bytes"][dom] / (ms * 1e-3) / 1e9 if ms > 0 else 0.0}


# ---------------------------------------------------------------------------
# headline
# ---------------------------------------------------------------------------
def batched_leg(args):
    import numpy as np
    import torch

    import spff_inputs as si
    from paper_2203_16467_amd import autotune, spff

    n, B = args.grid, args.batch
    E = np.stack([si.young_modulus(n, args.corr, args.amp, 3000 + i) for i in range(B)])
    ramp = si.uniaxial_ramp(200, 0.2, 2.0)
    t = time.time()
    plans, timing, source = autotune.tune(n, n, B, cache=args.plan_cache or autotune.DEFAULT_CACHE)
    tuned = {"source": source, "seconds": time.time() - t, "plans": {str(v): plans[v] for v in plans}}
    log(f"launch plans for {len(plans)} buckets ({source})")
    cfg = spff.default_config(nx=n, ny=n, use_graph=1, ticks_per_sync=args.ticks_per_sync)
    p = spff.Problem(torch.as_tensor(E, device="cuda:0"), cfg)
    autotune.apply(p, plans)
    s0 = args.start - args.warmup
    t = time.time()
    steady = None
    a0, a1 = args.all_active
    if s0 >= a1 > a0 >= 0:
        # the kernels at full occupancy: every realization active (elastic
        # steps before any nucleates), timed on the way to the window
        p.run_sequence(ramp[:a0])
        p.profile_enable(True)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        _, sst = p.run_sequence(ramp[a0:a1])
        torch.cuda.synchronize()
        dt1 = time.perf_counter() - t1
        pr = p.profile_read()
        p.profile_enable(False)
        cg1, pf1 = iters(sst)
        steady = {"steps": f"{a0}..{a1 - 1}", "seconds": dt1, "value": (cg1 + pf1) * n * n / dt1,
                  "cg_iters": cg1, "bccg_iters": pf1, "prof": pr}
        p.run_sequence(ramp[a1:s0])
    elif s0 > 0:
        p.run_sequence(ramp[:s0])
    log(f"prepared {B}x{n}^2 to load step {s0} in {time.time() - t:.1f}s")
    if args.warmup > 0:
        p.run_sequence(ramp[s0:args.start])
    log(f"warmup steps {s0}..{args.start - 1} done")
    p.profile_enable(True)
    torch.cuda.synchronize()
    ROCTX.begin("bench_timed")
    t0 = time.perf_counter()
    st, stats = p.run_sequence(ramp[args.start:args.start + args.steps])
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ROCTX.end()
    prof = p.profile_read()
    p.profile_enable(False)
    # the GPU state after the timed steps seeds the CPU baseline's sample (the
    # next load step of the ramp, with cracks nucleating in several of them)
    st_all, _ = p.get_state()
    ncpu = min(args.cpu_states, B)
    cpu_states = st_all[:ncpu].double().cpu().numpy()
    del st_all
    cg, pf = iters(stats)
    am = [sum(s["am_iters"] for s in row) for row in stats]
    capped = sum(1 for row in stats for s in row if s["status"] == spff.WARN_NOT_CONVERGED)
    ncrack = sum(1 for row in stats if row[-1]["crack_px"] > 0)
    log(f"timed {args.steps} steps in {dt:.2f}s: cg {cg} bccg {pf}, cracked {ncrack}/{B}, status {st}")
    p.close()
    return {"dt": dt, "cg": cg, "pf": pf, "status": st, "prof": prof, "ncrack": ncrack, "E": E[:ncpu],
            "cpu_states": cpu_states, "cpu_eps": ramp[min(args.start + args.steps, 199)],
            "cpu_step": min(args.start + args.steps, 199), "ramp": ramp, "n": n, "B": B, "tuned": tuned,
            "am_iters": int(sum(am)), "am_max_step": int(max(s["am_iters"] for row in stats for s in row)),
            "steps_capped": capped, "steady": steady}


# ---------------------------------------------------------------------------
# CPU baseline (the oracle, in child processes that never touch the GPU)
# ---------------------------------------------------------------------------
def cpu_worker(spec_path, indices, cg_cap, pf_cap):
    """Realizations `indices` one after the other: for each, the oracle's
    mechanics Newton-CG (one Newton step, at most cg_cap CG iterations) and
    phase-field BCCG (at most pf_cap iterations) of the first
    alternating-minimisation iteration of the load step after the timed
    window, from the GPU state.  Prints one JSON line."""
    import numpy as np

    import oracle
    from oracle import constitutive as ocm
    from oracle import phasefield as opf
    d = np.load(spec_path)
    cg = pf = 0
    t0 = time.perf_counter()
    for index in indices:
        E, s, eb = d["E"][index], d["states"][index].astype(np.float64), d["eps"]
        o = oracle.Problem(E.astype(np.float64), nu=0.2, ell=2.0, gc=1.0, at=1, split="spectral", tol_mech=1e-6,
                           tol_pf=1e-6, max_cg=cg_cap, max_newton=1, max_bccg=pf_cap, max_am=1)
        o.set_state({"eps_star": ocm.sym_tensor(s[0], s[1], s[2]), "phi": s[3], "phi_ref": s[4]})
        o.eps_bar = ocm.sym_tensor(*eb)
        mi = o.solve_mechanics()
        lo = opf.constraint_field(o.phi_ref, o.irr, o.threshold)
        _, pi = o.solve_phase_field(lo)
        cg += int(mi["cg"])
        pf += int(pi["iterations"])
    dt = time.perf_counter() - t0
    print(json.dumps({"cg": cg, "bccg": pf, "seconds": dt, "n": int(d["E"].shape[-1])}), flush=True)


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_leg(res, args):
    """The FP64 oracle on the host, one realization per process (OpenMP /
    BLAS threads pinned to one per process): first one process alone (one
    core), then one per core of the machine's CPU share at once (all cores).
    grid-pt-iters/s = sum of (CG + BCCG iterations) x grid points / wall."""
    import tempfile

    import numpy as np

    spec = os.path.join(tempfile.gettempdir(), f"spff_cpu_sample_{os.getpid()}.npz")
    np.savez(spec, E=res["E"], states=res["cpu_states"].astype(np.float32), eps=res["cpu_eps"])
    env = dict(os.environ, OMP_NUM_THREADS="1", OPENBLAS_NUM_THREADS="1", MKL_NUM_THREADS="1",
               HIP_VISIBLE_DEVICES="", ROCR_VISIBLE_DEVICES="")
    n = res["n"]

    def run(groups, cg_cap, pf_cap):
        t0 = time.perf_counter()
        procs = [subprocess.Popen([sys.executable, os.path.abspath(__file__), "--cpu-worker", spec,
                                   ",".join(str(i) for i in g), str(cg_cap), str(pf_cap)],
                                  stdout=subprocess.PIPE, env=env, cwd=ROOT) for g in groups]
        outs = []
        for pr in procs:
            out, _ = pr.communicate(timeout=max(30.0, left(args)))
            if pr.returncode != 0:
                raise RuntimeError(f"cpu worker failed ({pr.returncode})")
            outs.append(json.loads(out.decode().strip().splitlines()[-1]))
        wall = time.perf_counter() - t0
        it = sum(o["cg"] + o["bccg"] for o in outs)
        return {"value": it * n * n / wall, "seconds": wall, "cg_iters": sum(o["cg"] for o in outs),
                "bccg_iters": sum(o["bccg"] for o in outs), "processes": len(groups),
                "realizations": sum(len(g) for g in groups)}

    try:
        cores = len(os.sched_getaffinity(0))
    except AttributeError:  # pragma: no cover
        cores = os.cpu_count() or 1
    nst = len(res["cpu_states"])
    cores = max(1, min(cores, args.cpu_cores, nst))
    one = run([list(range(min(args.cpu_one, nst)))], args.cpu_cg, args.cpu_bccg)
    log(f"cpu baseline, one core: {one['value']:.3e} grid-pt-iters/s ({one['seconds']:.1f}s)")
    allc = None
    if cores > 1 and left(args) > 1.5 * one["seconds"] + 20:
        groups = [list(range(j, nst, cores)) for j in range(cores)]
        allc = run(groups, args.cpu_cg, args.cpu_bccg)
        log(f"cpu baseline, {cores} cores: {allc['value']:.3e} grid-pt-iters/s ({allc['seconds']:.1f}s)")
    os.remove(spec)
    best = allc if allc is not None else one
    return {"value": best["value"], "unit": "grid-pt-iters/s", "cores": best["processes"], "kind": "oracle",
            "sample": f"FP64 NumPy oracle, {n}x{n} realizations of the batched workload from the GPU state "
                      f"after the timed steps, load step {res['cpu_step']}: one alternating-minimisation "
                      f"iteration with the mechanics Newton-CG capped at {args.cpu_cg} CG iterations and the "
                      f"BCCG at {args.cpu_bccg}; one core: {one['realizations']} realizations in one "
                      f"single-threaded process; all cores: {nst} realizations over {cores} single-threaded "
                      f"processes",
            "one_core": one, "all_cores": allc, "cpu_model": cpu_model(), "host_cpus": os.cpu_count()}


# ---------------------------------------------------------------------------
# plain single-instance path
# ---------------------------------------------------------------------------
def plain_leg(args, budget):
    import torch

    import spff_inputs as si
    from paper_2203_16467_amd import spff

    n = 256
    E = si.young_modulus(n, 8.0, 0.1, 2000)
    ramp = si.uniaxial_ramp(200, 0.2, 2.0)
    t_end = time.time() + budget
    runs = {}
    for at, split in ((1, spff.SPLIT_SPECTRAL), (2, spff.SPLIT_SPECTRAL), (1, spff.SPLIT_NONE), (2, spff.SPLIT_NONE)):
        name = f"AT{at}-{'spectral' if split else 'none'}"
        if runs and time.time() > t_end - 5:
            break
        cfg = spff.default_config(nx=n, ny=n, at=at, split=split, use_graph=0, ticks_per_sync=1)
        p = spff.Problem(torch.as_tensor(E, device="cuda:0"), cfg)
        cg = pf = 0
        dt = 0.0
        done = 0
        st = 0
        for c0 in range(0, 200, 20):
            if time.time() > t_end:
                break
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            st_c, stats = p.run_sequence(ramp[c0:c0 + 20])
            torch.cuda.synchronize()
            dt += time.perf_counter() - t0
            a, b = iters(stats)
            cg, pf, done = cg + a, pf + b, c0 + 20
            st = max(st, st_c)
        p.close()
        runs[name] = {"seconds": dt, "steps": done, "cg_iters": cg, "bccg_iters": pf, "status": st,
                      "value": (cg + pf) * n * n / dt if dt > 0 else 0.0}
        log(f"plain 256^2 {name}: {done} steps in {dt:.2f}s, {runs[name]['value']:.3e} grid-pt-iters/s")
    return {"value": runs["AT1-spectral"]["value"], "unit": "grid-pt-iters/s",
            "workload": "plain: one 256x256 problem (E = max(1+0.1z,0.5), corr 8 px, seed 2000), l = 2 px, "
                        "crack-set, 200-step ramp to 1.5 eps_M; host status check after every tick, no graph; "
                        "value = the AT1 spectral-split run (the batched workload's model); the other variants "
                        "as the budget allows",
            "runs": runs}


# ---------------------------------------------------------------------------
# serving
# ---------------------------------------------------------------------------
def serving_leg(args, budget):
    """Resident microstructures with grid sizes drawn uniformly from {128,
    256, 512, 1024}^2, AT1/AT2 half and half; request = the next load step
    of the problem's 200-step ramp.  Each problem joins at its own point of
    the ramp, drawn uniformly from [serve_start_lo, serve_start_hi): its
    first request equilibrates it there from zero strain fluctuation and
    phi = 0.  Before any pixel reaches the crack-set threshold the
    irreversibility bound is phi >= 0 alone, so that state is the one the
    ramp itself reaches (AT1 stays at phi = 0 before the onset of damage);
    positions late in the range put AT2 problems a few requests before
    crack nucleation.  A closed-loop run (serve_closed_steps requests per
    problem) gives the saturation rate of this mix and the latency under
    saturation; Poisson arrivals at fractions of that rate then give
    throughput and p50/p99 latency from arrival.  Requests of the closed
    loop still running after a tenth of the budget run on under the open
    loop as a backlog.  Each load level gets an equal share of the remaining
    budget; requests still running when its share ends are censored
    (counted with their age, a lower bound) and stay on the device, so the
    next level starts behind them.  Request costs are heavy-tailed: a load
    step of elastic growth takes milliseconds, a crack nucleation step of a
    1024^2 problem tens of seconds."""
    import numpy as np
    import torch

    import spff_inputs as si
    from paper_2203_16467_amd import serving, spff

    t_end = time.time() + budget
    rng = np.random.default_rng(4000)
    sizes = rng.choice([128, 256, 512, 1024], size=args.serve_problems)
    ats = np.arange(args.serve_problems) % 2 + 1
    starts = rng.integers(args.serve_start_lo, args.serve_start_hi, size=args.serve_problems)
    sv = spff.Server(arena_bytes=int(args.serve_arena_gb * (1 << 30)),
                     scratch_budget_bytes=int(args.serve_scratch_gb * (1 << 30)), ticks_per_sync=8, use_graph=1)
    ramps, cursor = {}, {}
    for i, (n, at) in enumerate(zip(sizes, ats)):
        E = si.young_modulus(int(n), 8.0, 0.1, 4000 + i)
        pid = sv.register(spff.default_config(nx=int(n), ny=int(n), at=int(at)), torch.as_tensor(E, device="cuda:0"))
        ramps[pid] = si.uniaxial_ramp(200, 0.2, 2.0)
        cursor[pid] = int(starts[i])
    pos = np.asarray(starts)
    log(f"serving: {len(ramps)} problems joining at ramp steps {pos.min()}..{pos.max()}")
    sat, lat0, wall0, res0, running = serving.run_closed(sv, ramps, cursor, args.serve_closed_steps,
                                                          deadline=time.perf_counter() + 0.3 * budget)
    info = sv.info()
    log(f"serving: saturation {sat:.1f} req/s ({len(lat0)} requests in {wall0:.1f}s, {len(running)} still "
        f"running), {info['slots']} slots in {info['classes']} classes")
    lat0 = np.asarray(lat0)
    out = {"workload": None, "join_steps": {"min": int(pos.min()), "median": int(np.median(pos)),
                                            "max": int(pos.max())},
           "saturation_req_per_s": sat, "saturation_requests": int(lat0.size),
           "saturation_p50_ms": float(np.percentile(lat0, 50)) if lat0.size else None,
           "saturation_p99_ms": float(np.percentile(lat0, 99)) if lat0.size else None,
           "saturation_max_am_iters": int(max((r["am_iters"] for r in res0), default=0)),
           "slots": info["slots"], "classes": info["classes"], "loads": []}
    # requests of the saturation run still running get a tenth of the budget
    # to finish; any left run on under the open-loop levels (a backlog)
    drain_end = time.perf_counter() + 0.1 * budget
    while running and time.perf_counter() < drain_end:
        sv.progress(1)
        running = [t for t in running if sv.poll(t) is None]
    out["backlog_from_saturation_run"] = len(running)
    for k, f in enumerate(args.serve_loads if sat > 0 else []):
        share = (t_end - time.time()) / (len(args.serve_loads) - k)
        if share < 10:
            break
        rate = f * sat
        nreq = int(min(args.serve_requests, max(0.0, 0.6 * share) * rate))
        if nreq < 50:
            break
        warm = max(10, nreq // 20)
        log(f"serving load {f}: {nreq} requests at {rate:.1f} req/s")
        thr, lat, offered, res, cens = serving.run_poisson(sv, ramps, cursor, rate=rate, n_requests=nreq, seed=k,
                                                           warmup=warm, deadline=time.perf_counter() + share - 2)
        lat = np.asarray(lat)
        pfw = np.asarray([r["bccg_iters"] > 0 for r in res], dtype=bool)
        done_lat = lat[:len(res)]
        out["loads"].append({"load": f, "offered_req_per_s": offered, "throughput_req_per_s": thr,
                             "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
                             "requests": int(lat.size), "censored": int(cens),
                             "requests_with_phase_field_work": int(pfw.sum()),
                             "p99_ms_phase_field_requests":
                                 float(np.percentile(done_lat[pfw], 99)) if pfw.any() else None,
                             "max_am_iters": int(max((r["am_iters"] for r in res), default=0)),
                             "requests_nucleating": int(sum(1 for r in res if r["am_iters"] >= 20))})
        L = out["loads"][-1]
        log(f"serving load {f}: {thr:.1f} req/s, p50 {L['p50_ms']:.1f} ms, p99 {L['p99_ms']:.1f} ms, "
            f"{L['requests_with_phase_field_work']} with phase-field work, max AM {L['max_am_iters']}, "
            f"censored {cens}")
        # requests still running stay on the device: the next level starts
        # behind them, as a server would
    sv.close()
    out["workload"] = (f"serving: {args.serve_problems} resident problems, grid uniform over {{128,256,512,1024}}^2 "
                       f"(E = max(1+0.1z,0.5), corr 8 px), AT1/AT2 alternating, strain-spectral, crack set; each "
                       f"problem joins at its own ramp step (uniform over {args.serve_start_lo}.."
                       f"{args.serve_start_hi - 1}); request = next load step; scratch budget "
                       f"{args.serve_scratch_gb:g} GB (admission by footprint); latency from arrival to observed "
                       f"completion")
    return out


# ---------------------------------------------------------------------------
# large single instance
# ---------------------------------------------------------------------------
def large_leg(args, budget):
    """2048^2 (E = max(1+0.3z, 0.5), corr 32 px, seed 5000), AT1, spectral
    split, l = 1 px, crack set, 500-step uniaxial ramp to 1.5 eps_M.  Load
    steps before `large_start` run untimed; then single load steps are timed
    with the kernel timers on, through at most `large_pf_steps` steps with
    phase-field work (by default the onset of damage itself, load step 212;
    the next step is unstable crack growth across the 2048 px cell, which
    runs the alternating minimisation for minutes), or until the budget is
    spent."""
    import torch

    import spff_inputs as si
    from paper_2203_16467_amd import autotune, spff

    n = 2048
    t_end = time.time() + budget
    E = si.young_modulus(n, 32.0, 0.3, 5000)
    ramp = si.uniaxial_ramp(500, 0.2, 1.0)
    cfg = spff.default_config(nx=n, ny=n, ell=1.0, use_graph=1, ticks_per_sync=16)
    p = spff.Problem(torch.as_tensor(E, device="cuda:0"), cfg)
    plans, _, source = autotune.tune(n, n, 1, cache=args.plan_cache or autotune.DEFAULT_CACHE)
    autotune.apply(p, plans)
    for c0 in range(0, args.large_start, 40):
        p.run_sequence(ramp[c0:min(c0 + 40, args.large_start)])
    log(f"large 2048^2: load steps 0..{args.large_start - 1} untimed")
    p.profile_enable(True)
    dt, cg, pf, st, steps, pf_steps, am = 0.0, 0, 0, 0, 0, 0, 0
    k = args.large_start
    ROCTX.begin("bench_large_timed")
    # a step after the onset of damage may run the alternating minimisation
    # to its cap (about a minute on this grid): start one only with that
    # much of the budget left
    while k < 500 and pf_steps < args.large_pf_steps and time.time() < t_end - (70 if pf_steps else 5):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st_c, stats = p.run_sequence(ramp[k:k + 1])
        torch.cuda.synchronize()
        dt += time.perf_counter() - t0
        s0 = stats[0][0]
        cg, pf, st, steps, k = cg + s0["cg_iters"], pf + s0["bccg_iters"], max(st, st_c), steps + 1, k + 1
        am += s0["am_iters"]
        if s0["bccg_iters"] > 0:
            pf_steps += 1
            log(f"large 2048^2: load step {k - 1} with phase-field work: {s0['am_iters']} AM, "
                f"{s0['bccg_iters']} BCCG, {s0['cg_iters']} CG iterations")
    ROCTX.end()
    pr = p.profile_read()
    p.close()
    kf = kernel_figures(pr)
    out = {"workload": f"one 2048x2048 problem (E = max(1+0.3z,0.5), corr 32 px, seed 5000), AT1, spectral, "
                       f"l = 1 px, crack set, 500-step ramp to 1.5 eps_M; load steps {args.large_start}.."
                       f"{args.large_start + steps - 1} (from before to after the onset of damage)",
           "seconds": dt, "value": (cg + pf) * n * n / dt if dt > 0 else 0.0, "unit": "grid-pt-iters/s",
           "cg_iters": cg, "bccg_iters": pf, "am_iters": am, "steps_with_phase_field_work": pf_steps,
           "status": st, "dominant_kernel": kf["dominant"], "avg_launch_us": kf["avg_launch_us"],
           "alg_bytes_per_launch": kf["alg_bytes_per_launch"], "achieved_GBs": kf["achieved_GBs"],
           "frac_hbm": kf["achieved_GBs"] / HBM_PEAK_GBS, "kernel_ms": kf["kernel_ms"],
           "kernel_GBs": {q: pr["alg_bytes"][q] / (kf["kernel_ms"][q] * 1e-3) / 1e9
                          for q in KERNELS if kf["kernel_ms"][q] > 0},
           "plan": {"source": source, "plan": plans[1]}}
    log(f"large 2048^2: {out['value']:.3e} grid-pt-iters/s over {steps} steps ({cg} CG, {pf} BCCG), "
        f"{kf['dominant']} {kf['achieved_GBs']:.0f} GB/s")
    return out


# ---------------------------------------------------------------------------
# variants
# ---------------------------------------------------------------------------
def variants_leg(args, budget):
    """The model and evolution variants beyond the headline configuration,
    each on a batch of 16 realizations of 256^2 (E = max(1+0.2z, 0.5), corr
    8 px, seeds 6000..), l = 2 px, 100-step uniaxial ramp to 1.5 eps_M,
    captured graphs, built-in launch plans: vol.-dev. split; the production
    model (spectral driving force, stress-free isotropic contact, damage);
    Algorithm 3 (eta = 0.5, dt in [1e-3, 1], dphi_max 20 px, dphi_min
    1e-3); Algorithm 4 ((-F_phi)_max = 0.7 G_c/l, threshold 1 G_c/l).  Steps
    (iterations) 0..1 untimed, then chunks of 8 timed with the kernel timers
    while the variant's share of the budget lasts."""
    import numpy as np
    import torch

    import spff_inputs as si
    from paper_2203_16467_amd import spff

    n, B = 256, 16
    E = np.stack([si.young_modulus(n, 8.0, 0.2, 6000 + i) for i in range(B)])
    ramp = si.uniaxial_ramp(100, 0.2, 2.0)
    deps = ramp[0].copy()
    ell = 2.0
    variants = {
        "voldev": (dict(split=spff.SPLIT_VOLDEV), "seq"),
        "production": (dict(split=spff.SPLIT_SPECTRAL, contact=spff.SPLIT_NONE,
                            irreversibility=spff.IRR_DAMAGE), "seq"),
        "time_alg3": (dict(evolution=spff.EVOL_TIME, eta=0.5, dt_max=1.0, dt_min=1e-3, dphi_max=20.0,
                           dphi_min=1e-3), "evo"),
        "near_eq_alg4": (dict(evolution=spff.EVOL_NEAR_EQ, fphi_max=0.7 / ell, drive_threshold=1.0 / ell,
                              deps_max=float(np.abs(deps).max()), dphi_min=1e-3), "evo"),
    }
    out = {}
    t_end = time.time() + budget
    for j, (name, (kw, kind)) in enumerate(variants.items()):
        share = (t_end - time.time()) / (len(variants) - j)
        if share < 5:
            break
        v_end = time.time() + share
        cfg = spff.default_config(nx=n, ny=n, ell=ell, use_graph=1, ticks_per_sync=16, **kw)
        p = spff.Problem(torch.as_tensor(E, device="cuda:0"), cfg)
        if kind == "seq":
            p.run_sequence(ramp[:2])
        else:
            p.run_evolution(deps, nsteps=2)
        p.profile_enable(True)
        cg = pf = adv = 0
        dt, st, done = 0.0, 0, 2
        Kv = 50 if kind == "seq" else 120
        while done < Kv and time.time() < v_end:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            m = min(8, Kv - done)
            if kind == "seq":
                st_c, s_c = p.run_sequence(ramp[done:done + m])
            else:
                st_c, s_c = p.run_evolution(deps, nsteps=m)
            torch.cuda.synchronize()
            dt += time.perf_counter() - t0
            a, b = iters(s_c)
            cg, pf, done = cg + a, pf + b, done + m
            adv += sum(s["advance"] for row in s_c for s in row)
            st = min(st, st_c) if st_c < 0 or st < 0 else max(st, st_c)
        pr = p.profile_read()
        p.close()
        kf = kernel_figures(pr)
        out[name] = {"seconds": dt, "steps": [2, done - 1], "value": (cg + pf) * n * n / dt if dt > 0 else 0.0,
                     "unit": "grid-pt-iters/s", "cg_iters": cg, "bccg_iters": pf, "status": st,
                     "dominant_kernel": kf["dominant"], "achieved_GBs": kf["achieved_GBs"],
                     "frac_hbm": kf["achieved_GBs"] / HBM_PEAK_GBS}
        if kind == "evo":
            out[name]["advanced"] = adv
        log(f"variant {name}: {out[name]['value']:.3e} grid-pt-iters/s in {dt:.2f}s")
    return {"workload": "16 realizations of 256x256 (E = max(1+0.2z,0.5), corr 8 px, seeds 6000..), l = 2 px, "
                        "load steps (iterations) from 2 of a 100-step uniaxial ramp to 1.5 eps_M (Algorithms 3, "
                        "4: the ramp's increment per advancing iteration)", "runs": out}


# ---------------------------------------------------------------------------
# measured traffic (committed rocprofv3 --pmc record)
# ---------------------------------------------------------------------------
KERNEL_SOURCES = ("spff_kernels.hip", "spff_device.hpp", "spff_engine.hpp")
PMC_RECORD = os.path.join(ROOT, "profiles", "pmc_traffic_batched_64x512.txt")


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2203_16467_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(role, window):
    """HBM-side bytes per launch of a kernel role from the committed
    rocprofv3 --pmc record: read bytes from the L2's read requests counted
    by size (TCC_EA0_RDREQ_32B/64B/128B) and write bytes (WRITE_SIZE), per
    dispatch of the role in the record's window.  None if the record is
    missing, covers another window, or was taken on kernel sources other
    than the ones built here."""
    if not os.path.exists(PMC_RECORD):
        return None
    rec = {}
    with open(PMC_RECORD) as f:
        for line in f:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                rec[k.strip()] = v.strip()
    try:
        if rec.get("kernel_source_sha256") != kernel_source_hash() or rec.get("window") != window:
            return None
        read = float(rec[f"{role}.read_kib_per_dispatch"])
        write = float(rec[f"{role}.write_kib_per_dispatch"])
    except (KeyError, ValueError):
        return None
    return (read + write) * 1024.0


LEGS = ("cpu_baseline", "plain", "large", "variants", "serving")
# minimum seconds a leg needs to produce a figure, and the most it may take
LEG_MIN = {"cpu_baseline": 40, "plain": 30, "serving": 90, "large": 60, "variants": 40}
LEG_MAX = {"cpu_baseline": 120, "plain": 90, "serving": 240, "large": 120, "variants": 100}


def main():
    if len(sys.argv) > 1 and sys.argv[1] == "--cpu-worker":
        cpu_worker(sys.argv[2], [int(v) for v in sys.argv[3].split(",")], int(sys.argv[4]), int(sys.argv[5]))
        return
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--start", type=int, default=82,
                    help="first timed load step of the 200-step ramp (the default window 82..101 holds the "
                         "first wave of crack nucleation: eight realizations nucleate, three run the "
                         "alternating minimisation to its cap)")
    ap.add_argument("--budget", type=float, default=420.0, help="wall-clock seconds for the whole run")
    ap.add_argument("--all-active", type=int, nargs=2, default=[40, 45],
                    help="load steps [a, b) timed on the way to the window with every realization active")
    ap.add_argument("--legs", nargs="*", default=list(LEGS), help=f"secondary legs to run, in order: {LEGS}")
    ap.add_argument("--grid", type=int, default=512)
    ap.add_argument("--batch", type=int, default=64)
    ap.add_argument("--corr", type=float, default=16.0)
    ap.add_argument("--amp", type=float, default=0.2)
    ap.add_argument("--ticks-per-sync", type=int, default=32,
                    help="solver ticks per captured graph block between host status checks")
    ap.add_argument("--plan-cache", default=None, help="JSON cache of autotuned launch plans (default: the "
                                                       "package's gfx950 cache; missing buckets are tuned live)")
    ap.add_argument("--cpu-cores", type=int, default=16, help="processes of the all-cores CPU baseline (the "
                                                              "box's CPU share)")
    ap.add_argument("--cpu-states", type=int, default=32, help="realizations of the CPU baseline's sample")
    ap.add_argument("--cpu-one", type=int, default=8, help="realizations of the one-core run")
    ap.add_argument("--cpu-cg", type=int, default=20)
    ap.add_argument("--cpu-bccg", type=int, default=20)
    ap.add_argument("--serve-problems", type=int, default=200)
    ap.add_argument("--serve-requests", type=int, default=2000)
    ap.add_argument("--serve-loads", type=float, nargs="+", default=[0.5, 0.8, 0.95])
    ap.add_argument("--serve-closed-steps", type=int, default=5,
                    help="load steps per problem of the closed-loop saturation run")
    ap.add_argument("--serve-start-lo", type=int, default=0)
    ap.add_argument("--serve-start-hi", type=int, default=90)
    ap.add_argument("--serve-arena-gb", type=float, default=8.0)
    ap.add_argument("--serve-scratch-gb", type=float, default=1.0)
    ap.add_argument("--large-start", type=int, default=170)
    ap.add_argument("--large-pf-steps", type=int, default=1,
                    help="load steps with phase-field work timed in the large leg (the step after the onset of "
                         "damage of this instance is unstable crack growth that runs for minutes)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU: this build runs one process on one MI355X "
              f"(--gpus {args.gpus} is not supported; independent problems shard across GPUs by "
              f"placement, see the design notes)", file=sys.stderr)
        sys.exit(2)
    if args.start < args.warmup or args.start + args.steps > 200:
        sys.exit("window must lie inside the 200-step ramp")

    res = batched_leg(args)
    value = (res["cg"] + res["pf"]) * res["n"] ** 2 / res["dt"]
    kf = kernel_figures(res["prof"])
    dom = kf["dominant"]
    window = f"{args.start}..{args.start + args.steps - 1}"
    all_ms = sum(kf["kernel_ms"][k] for k in KERNELS)
    all_b = sum(res["prof"]["alg_bytes"][k] for k in KERNELS)
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "grid-pt-iters/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": res["dt"] * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": f"batched: {res['B']} realizations of {res['n']}x{res['n']} (E = max(1+{args.amp}z, 0.5), "
                        f"corr {args.corr:g} px, seeds 3000..), AT1, strain-spectral split, l = 2 px, crack-set, "
                        f"uniaxial-strain ramp of 200 steps to 1.5 eps_M; timed load steps {window}; FP32 fields, "
                        f"FP64 reductions",
            "batch": res["B"], "grid": [res["n"], res["n"]], "parallelism": "single GPU",
        },
        "breakdown": {"cg_iters": res["cg"], "bccg_iters": res["pf"], "am_iters": res["am_iters"],
                      "am_iters_max_step": res["am_max_step"], "problem_steps_at_a_cap": res["steps_capped"],
                      "seconds": res["dt"], "realizations_cracked": res["ncrack"], "status": res["status"],
                      "kernel_ms": kf["kernel_ms"], "kernel_activity_ms": res["prof"]["kernel_ms"],
                      "kernel_span_ms": res["prof"]["kernel_span_ms"], "kernel_launches": res["prof"]["launches"],
                      "kernel_alg_bytes": res["prof"]["alg_bytes"],
                      "alg_GBs_all_fft_kernels": all_b / (all_ms * 1e-3) / 1e9 if all_ms > 0 else None},
        "autotune": res["tuned"],
        "kernel_source_sha256": kernel_source_hash(),
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": kf["achieved_GBs"], "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": kf["achieved_GBs"] / HBM_PEAK_GBS,
                     "traffic": measured_traffic(dom, window), "alg_bytes_per_launch": kf["alg_bytes_per_launch"],
                     "avg_launch_us": kf["avg_launch_us"]},
    }
    if res["steady"] is not None:
        sd = res["steady"]
        sk = kernel_figures(sd["prof"])
        out["all_active"] = {
            "steps": sd["steps"], "seconds": sd["seconds"], "value": sd["value"], "unit": "grid-pt-iters/s",
            "cg_iters": sd["cg_iters"], "bccg_iters": sd["bccg_iters"],
            "note": "every realization active (elastic load steps before any nucleates), same launch plans; "
                    "the kernels at full occupancy",
            "roofline": {"bound": "hbm", "kernel": sk["dominant"], "achieved": sk["achieved_GBs"],
                         "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": sk["achieved_GBs"] / HBM_PEAK_GBS,
                         "traffic": measured_traffic(sk["dominant"], sd["steps"]),
                         "alg_bytes_per_launch": sk["alg_bytes_per_launch"], "avg_launch_us": sk["avg_launch_us"]},
            "kernel_GBs": {q: sd["prof"]["alg_bytes"][q] / (sk["kernel_ms"][q] * 1e-3) / 1e9
                           for q in KERNELS if sk["kernel_ms"][q] > 0},
            "kernel_alg_MB_per_launch": {q: sd["prof"]["alg_bytes"][q] / max(sd["prof"]["launches"][q], 1) / 1e6
                                         for q in KERNELS},
            "kernel_traffic_MB_per_launch": {q: (measured_traffic(q, sd["steps"]) or 0.0) / 1e6 or None
                                             for q in KERNELS}}
        log(f"all active {sd['steps']}: {sd['value']:.3e} grid-pt-iters/s; {sk['dominant']} "
            f"{sk['achieved_GBs']:.0f} GB/s")
    log(f"headline {value:.3e} grid-pt-iters/s; {dom} {kf['achieved_GBs']:.0f} GB/s")
    skipped = []
    for leg in args.legs:
        rem = left(args)
        if rem < LEG_MIN[leg]:
            skipped.append(leg)
            log(f"skip {leg}: {rem:.0f}s left")
            continue
        budget = min(rem - 5, LEG_MAX[leg])
        try:
            if leg == "cpu_baseline":
                out["cpu_baseline"] = cpu_leg(res, args)
            elif leg == "plain":
                out["plain_gpu"] = plain_leg(args, budget)
                out["vs_plain"] = value / out["plain_gpu"]["value"] if out["plain_gpu"]["value"] > 0 else None
            elif leg == "serving":
                out["serving"] = serving_leg(args, budget)
            elif leg == "large":
                out["large"] = large_leg(args, budget)
            elif leg == "variants":
                out["variants"] = variants_leg(args, budget)
        except Exception as e:  # a failed secondary leg must not cost the headline line
            skipped.append(leg)
            out.setdefault("errors", {})[leg] = repr(e)
            log(f"{leg} failed: {e!r}")
    out["skipped"] = skipped
    out["wall_s"] = time.time() - T_START
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
