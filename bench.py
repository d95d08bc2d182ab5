"""Benchmark: staggered FFT phase-field fracture solve on one MI355X.

Workload (default, "batched"): 64 independent realizations of a 512x512
periodic microstructure, E = max(1 + 0.2 z, 0.5) with z a unit-variance
Gaussian random field of correlation length 16 px (seeds 3000..3063), AT1,
strain-spectral split, l = 2 px, crack-set irreversibility, uniaxial-strain
ramp of 200 load steps to 1.5 eps_M; FP32 fields with FP64 reductions; all
realizations in one batched launch per kernel, independent per-problem
progression.

A "step" is one load step (alternating minimisation to Tol_AM: mechanics
Newton-CG + phase-field BCCG) of every realization.  The ramp's early steps
are run untimed to reach the window (preparation), then W warmup steps, then
K timed steps.  value = (mechanics CG + BCCG iterations) x grid points per
second over the timed steps.

Before the timed steps the launch plans of the FFT kernels are autotuned
per bucket of active problems (untimed; reported under "autotune"), and a
steady window of load steps before any realization nucleates (all 64 active)
is measured on its own (reported under breakdown.steady_all_active).

Also reported on the same line:
  roofline      dominant kernel's algorithmic HBM bytes per launch / its
                average time per launch, both over the timed steps (the
                library's device-clock kernel timers on the solver stream,
                also inside captured graphs: a launch's work-group activity
                plus half of the dead time to the next kernel's first start,
                which brackets a kernel trace's duration);
                traffic = measured HBM bytes per launch from the committed
                rocprofv3 --pmc record when it was taken on these kernel
                sources, else null
  plain_gpu     the plain single-instance path (256x256, one problem, host
                check after every tick, no graph) over its full 200-step
                ramp, for each of AT1/AT2 x no split/spectral split
  serving       continuous batching of load-step requests over resident
                problems of mixed grid sizes: saturation rate, then p50/p99
                latency and throughput under Poisson arrivals
  cpu_baseline  the FP64 NumPy oracle on one host core, on a bounded sample
"""

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "grid-pt CG iters/s & HBM GB/s, batched FP32 vs plain GPU @1e-4 err; p50/p99"
HBM_PEAK_GBS = 8000.0
KERNELS = ("rowfwd", "col", "rowinv")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


class _Roctx:
    """roctx range around the timed steps, so that a profiler run (rocprofv3
    --marker-trace) can restrict its kernel statistics to them; a no-op when
    the library is absent."""

    def __init__(self):
        import ctypes
        self.lib = None
        for name in ("librocprofiler-sdk-roctx.so.1", "libroctx64.so"):
            try:
                self.lib = ctypes.CDLL(name)
                break
            except OSError:
                continue

    def push(self, name):
        if self.lib:
            self.lib.roctxRangePushA(name.encode())

    def pop(self):
        if self.lib:
            self.lib.roctxRangePop()


ROCTX = _Roctx()


def iters(stats):
    cg = sum(s["cg_iters"] for row in stats for s in row)
    pf = sum(s["bccg_iters"] for row in stats for s in row)
    return cg, pf


def batched_leg(args):
    import numpy as np
    import torch

    import spff_inputs as si
    from paper_2203_16467_amd import spff

    n, B = args.grid, args.batch
    E = np.stack([si.young_modulus(n, args.corr, args.amp, 3000 + i) for i in range(B)])
    ramp = si.uniaxial_ramp(200, 0.2, 2.0)
    tuned = None
    if args.autotune:
        from paper_2203_16467_amd import autotune
        t = time.time()
        plans, timing, source = autotune.tune(n, n, B, cache=args.plan_cache or autotune.DEFAULT_CACHE,
                                              log=log if args.verbose else None)
        tuned = {"source": source, "seconds": time.time() - t,
                 "plans": {str(v): plans[v] for v in plans}, "timing_us_per_tick": {str(v): timing[v] for v in timing}}
        log(f"[bench] autotuned launch plans for {len(plans)} buckets ({source}) in {tuned['seconds']:.1f}s")
    cfg = spff.default_config(nx=n, ny=n, use_graph=1, ticks_per_sync=args.ticks_per_sync)
    p = spff.Problem(torch.as_tensor(E, device="cuda:0"), cfg)
    if tuned:
        autotune.apply(p, plans)
    steady = None
    s0 = args.start - args.warmup
    t = time.time()
    if args.steady and s0 > args.steady_start + args.steady_steps:
        # all realizations active (before any nucleates): the batched
        # kernels at full occupancy
        p.run_sequence(ramp[:args.steady_start])
        p.profile_enable(True)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        st, stats = p.run_sequence(ramp[args.steady_start:args.steady_start + args.steady_steps])
        torch.cuda.synchronize()
        dt1 = time.perf_counter() - t1
        pr = p.profile_read()
        p.profile_enable(False)
        cg1, pf1 = iters(stats)
        kt1 = {k: 0.5 * (pr["kernel_ms"][k] + pr["kernel_span_ms"][k]) for k in KERNELS}
        steady = {"steps": [args.steady_start, args.steady_start + args.steady_steps - 1], "seconds": dt1,
                  "value": (cg1 + pf1) * n * n / dt1, "unit": "grid-pt-iters/s", "cg_iters": cg1,
                  "bccg_iters": pf1, "kernel_ms": kt1, "kernel_alg_bytes": pr["alg_bytes"],
                  "kernel_alg_GBs": {k: pr["alg_bytes"][k] / (kt1[k] * 1e-3) / 1e9 for k in KERNELS if kt1[k] > 0}}
        log(f"[bench] steady window {steady['steps']}: {steady['value']:.3e} grid-pt-iters/s, "
            f"kernel GB/s {steady['kernel_alg_GBs']}")
        if s0 > args.steady_start + args.steady_steps:
            p.run_sequence(ramp[args.steady_start + args.steady_steps:s0])
    elif s0 > 0:
        p.run_sequence(ramp[:s0])
    log(f"[bench] prepared {B}x{n}^2 to load step {s0} in {time.time() - t:.1f}s")
    p.profile_enable(True)
    if args.warmup > 0:
        p.run_sequence(ramp[s0:args.start])
    log(f"[bench] warmup steps {s0}..{args.start - 1} done")
    # the timed region runs without the kernel timers (they cost a few
    # percent: every work-group stamps its start and end, the controller
    # folds them); it is then replayed from the same state with the timers
    # on for the per-kernel figures (deterministic: same iterations, same
    # launches)
    snap = p.get_state() if args.profile else None
    p.profile_enable(False)
    torch.cuda.synchronize()
    ROCTX.push("bench_timed")
    t0 = time.perf_counter()
    st, stats = p.run_sequence(ramp[args.start:args.start + args.steps])
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ROCTX.pop()
    cg, pf = iters(stats)
    prof, replay = None, None
    if args.profile:
        p.set_state(*snap)
        del snap
        p.profile_enable(True)
        torch.cuda.synchronize()
        ROCTX.push("bench_profiled")
        t1 = time.perf_counter()
        _, stats2 = p.run_sequence(ramp[args.start:args.start + args.steps])
        torch.cuda.synchronize()
        replay = {"seconds": time.perf_counter() - t1, "iterations_equal": iters(stats2) == (cg, pf)}
        ROCTX.pop()
        prof = p.profile_read()
        log(f"[bench] profiled replay in {replay['seconds']:.2f}s (same iterations: {replay['iterations_equal']})")
    ncrack = sum(1 for row in stats if row[-1]["crack_px"] > 0)
    log(f"[bench] timed {args.steps} steps in {dt:.2f}s: cg {cg} bccg {pf}, cracked {ncrack}/{B}, status {st}")
    p.close()
    return {"dt": dt, "cg": cg, "pf": pf, "status": st, "prof": prof, "ncrack": ncrack, "E0": E[0],
            "ramp": ramp, "n": n, "B": B, "tuned": tuned, "steady": steady, "replay": replay}


def plain_leg(args):
    import torch

    import spff_inputs as si
    from paper_2203_16467_amd import spff

    n = 256
    E = si.young_modulus(n, 8.0, 0.1, 2000)
    ramp = si.uniaxial_ramp(200, 0.2, 2.0)
    runs, tot_it, tot_s = {}, 0, 0.0
    for at in (1, 2):
        for split in (spff.SPLIT_NONE, spff.SPLIT_SPECTRAL):
            cfg = spff.default_config(nx=n, ny=n, at=at, split=split, use_graph=0, ticks_per_sync=1)
            p = spff.Problem(torch.as_tensor(E, device="cuda:0"), cfg)
            p.run_sequence(ramp[:2])  # warmup
            p.close()
            p = spff.Problem(torch.as_tensor(E, device="cuda:0"), cfg)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            st, stats = p.run_sequence(ramp)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            cg, pf = iters(stats)
            p.close()
            name = f"AT{at}-{'spectral' if split else 'none'}"
            runs[name] = {"seconds": dt, "cg_iters": cg, "bccg_iters": pf, "status": st,
                          "value": (cg + pf) * n * n / dt}
            tot_it += cg + pf
            tot_s += dt
            log(f"[bench] plain 256^2 single {name}: 200 steps in {dt:.2f}s, cg {cg} bccg {pf}")
    return {"value": runs["AT1-spectral"]["value"], "unit": "grid-pt-iters/s",
            "value_all_variants": tot_it * n * n / tot_s,
            "workload": "plain: one 256x256 problem (E = max(1+0.1z,0.5), corr 8 px, seed 2000), l = 2 px, "
                        "crack-set, 200-step ramp to 1.5 eps_M, run for AT1/AT2 x no split/spectral split; host "
                        "status check after every tick, no graph; value = the AT1 spectral-split run (the "
                        "batched workload's model), value_all_variants = all four runs' iterations x grid "
                        "points / their summed time",
            "seconds": tot_s, "runs": runs}


def variants_leg(args):
    """The model and evolution variants beyond the headline configuration,
    each on a batch of 16 realizations of 256^2 (E = max(1+0.2z, 0.5), corr
    8 px, seeds 6000..), l = 2 px, 100-step uniaxial ramp to 1.5 eps_M,
    captured graphs, autotuned-plan-free built-in plans:
      voldev          alternating minimisation, vol.-dev. split (variational)
      production      alternating minimisation, spectral driving force,
                      stress-free isotropic contact, damage irreversibility
      time_alg3       Algorithm 3 (eta = 0.5, dt in [1e-3, 1], dphi_max 20 px,
                      dphi_min 1e-3), device-driven iterations
      near_eq_alg4    Algorithm 4 ((-F_phi)_max = 0.7 G_c/l, threshold
                      1 G_c/l), device-driven iterations
    Steps (iterations) 0..1 untimed (graph capture); timed with the kernel
    timers in chunks of 8: load steps 2..49 (through crack nucleation,
    before complete separation), iterations 2..119 for Algorithms 3 and 4
    (whose iterations do not advance the load while phi evolves): grid-point
    Krylov iterations per second and the achieved algorithmic bandwidth of
    the dominant kernel."""
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
    K, K_EVO, CH = 50, 120, 8
    for name, (kw, kind) in variants.items():
        cfg = spff.default_config(nx=n, ny=n, ell=ell, use_graph=1, ticks_per_sync=16, **kw)
        p = spff.Problem(torch.as_tensor(E, device="cuda:0"), cfg)
        # untimed: the first two steps (captures the full-batch graphs)
        if kind == "seq":
            p.run_sequence(ramp[:2])
        else:
            p.run_evolution(deps, nsteps=2)
        p.profile_enable(True)
        stats = [[] for _ in range(B)]
        dt, st = 0.0, 0
        Kv = K if kind == "seq" else K_EVO
        for c0 in range(2, Kv, CH):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            if kind == "seq":
                st_c, s_c = p.run_sequence(ramp[c0:min(c0 + CH, Kv)])
            else:
                st_c, s_c = p.run_evolution(deps, nsteps=min(CH, Kv - c0))
            torch.cuda.synchronize()
            dt += time.perf_counter() - t0
            st = min(st, st_c) if st_c < 0 or st < 0 else max(st, st_c)
            for b in range(B):
                stats[b] += s_c[b]
            log(f"[bench] variant {name}: steps {c0}..{min(c0 + CH, Kv) - 1} done ({dt:.2f}s)")
        pr = p.profile_read()
        p.close()
        cg, pf = iters(stats)
        kt = {k: 0.5 * (pr["kernel_ms"][k] + pr["kernel_span_ms"][k]) for k in KERNELS}
        dom = max(KERNELS, key=lambda k: kt[k])
        gbs = pr["alg_bytes"][dom] / (kt[dom] * 1e-3) / 1e9 if kt[dom] > 0 else 0.0
        res = {"seconds": dt, "value": (cg + pf) * n * n / dt, "unit": "grid-pt-iters/s",
               "cg_iters": cg, "bccg_iters": pf, "status": st,
               "cracked": sum(1 for row in stats if row[-1]["crack_px"] > 0),
               "dominant_kernel": dom, "achieved_GBs": gbs, "frac_hbm": gbs / HBM_PEAK_GBS}
        if kind == "evo":
            res["advanced"] = sum(s["advance"] for row in stats for s in row)
            res["final_eps_yy_mean"] = float(np.mean([row[-1]["eps_bar"][1] for row in stats]))
        out[name] = res
        log(f"[bench] variant {name}: {res['value']:.3e} grid-pt-iters/s in {res['seconds']:.2f}s, "
            f"{res['dominant_kernel']} {res['achieved_GBs']:.0f} GB/s")
    return {"workload": "16 realizations of 256x256 (E = max(1+0.2z,0.5), corr 8 px, seeds 6000..), l = 2 px, "
                        "alternating minimisation: load steps 2..49 of a 100-step uniaxial ramp to 1.5 eps_M "
                        "(crack nucleation from about step 42); Algorithms 3, 4: iterations 2..119 with the "
                        "ramp's increment (eps_M / 66.7); timed in chunks of 8", "runs": out}


def large_leg(args):
    """One large instance: 2048^2 (E = max(1+0.3z, 0.5), corr 32 px, seed
    5000), AT1, spectral split, l = 1 px, crack set, 500-step uniaxial ramp
    to 1.5 eps_M; load steps 0..39 untimed, 40..59 timed without the kernel
    timers, then replayed from the same state with them on for the dominant
    kernel's achieved algorithmic bandwidth."""
    import torch

    import spff_inputs as si
    from paper_2203_16467_amd import spff

    n = 2048
    E = si.young_modulus(n, 32.0, 0.3, 5000)
    ramp = si.uniaxial_ramp(500, 0.2, 1.0)
    cfg = spff.default_config(nx=n, ny=n, ell=1.0, use_graph=1, ticks_per_sync=16)
    p = spff.Problem(torch.as_tensor(E, device="cuda:0"), cfg)
    tuned = None
    if args is None or args.autotune:
        from paper_2203_16467_amd import autotune
        plans, _, source = autotune.tune(n, n, 1, cache=(args.plan_cache if args else None) or autotune.DEFAULT_CACHE)
        autotune.apply(p, plans)
        tuned = {"source": source, "plan": plans[1]}
    p.run_sequence(ramp[:40])
    snap = p.get_state()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st, stats = p.run_sequence(ramp[40:60])
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    cg, pf = iters(stats)
    p.set_state(*snap)
    del snap
    p.profile_enable(True)
    _, stats2 = p.run_sequence(ramp[40:60])
    pr = p.profile_read()
    p.close()
    kt = {k: 0.5 * (pr["kernel_ms"][k] + pr["kernel_span_ms"][k]) for k in KERNELS}
    dom = max(KERNELS, key=lambda k: kt[k])
    gbs = pr["alg_bytes"][dom] / (kt[dom] * 1e-3) / 1e9 if kt[dom] > 0 else 0.0
    out = {"workload": "one 2048x2048 problem (E = max(1+0.3z,0.5), corr 32 px, seed 5000), AT1, spectral, "
                       "l = 1 px, crack set, 500-step ramp to 1.5 eps_M; load steps 40..59 (elastic)",
           "seconds": dt, "value": (cg + pf) * n * n / dt, "unit": "grid-pt-iters/s", "cg_iters": cg,
           "bccg_iters": pf, "status": st, "replay_iterations_equal": iters(stats2) == (cg, pf),
           "dominant_kernel": dom, "avg_launch_us": kt[dom] * 1e3 / max(pr["launches"][dom], 1),
           "alg_bytes_per_launch": pr["alg_bytes"][dom] / max(pr["launches"][dom], 1),
           "achieved_GBs": gbs, "frac_hbm": gbs / HBM_PEAK_GBS, "plan": tuned}
    log(f"[bench] large 2048^2: {out['value']:.3e} grid-pt-iters/s in {dt:.2f}s, {dom} {gbs:.0f} GB/s")
    return out


def serving_leg(args):
    """Serving workload: resident microstructures with grid sizes drawn
    uniformly from {128, 256, 512, 1024}^2, AT1/AT2 half and half, requests =
    the next load step of a problem's 200-step ramp; closed-loop saturation
    run, then Poisson arrivals at fractions of the saturation rate."""
    import numpy as np
    import torch

    import spff_inputs as si
    from paper_2203_16467_amd import serving, spff

    rng = np.random.default_rng(4000)
    sizes = rng.choice([128, 256, 512, 1024], size=args.serve_problems)
    ats = np.arange(args.serve_problems) % 2 + 1
    sv = spff.Server(arena_bytes=int(args.serve_arena_gb * (1 << 30)),
                     scratch_budget_bytes=int(args.serve_scratch_gb * (1 << 30)), ticks_per_sync=8, use_graph=1)
    ramps = {}
    t = time.time()
    for i, (n, at) in enumerate(zip(sizes, ats)):
        E = si.young_modulus(int(n), 8.0, 0.1, 4000 + i)
        pid = sv.register(spff.default_config(nx=int(n), ny=int(n), at=int(at)), torch.as_tensor(E, device="cuda:0"))
        ramps[pid] = si.uniaxial_ramp(200, 0.2, 2.0)
    info = sv.info()
    log(f"[bench] serving: registered {len(ramps)} problems in {time.time() - t:.1f}s")
    # saturation: two steps of every problem submitted at once
    sat, lat0, wall0, res0 = serving.run_closed(sv, ramps, 2)
    info = sv.info()
    log(f"[bench] serving: saturation {sat:.1f} req/s ({len(lat0)} requests in {wall0:.1f}s), "
        f"{info['slots']} slots in {info['classes']} classes")
    loads = []
    for k, f in enumerate(args.serve_loads):
        thr, lat, offered = serving.run_poisson(sv, ramps, 2, rate=f * sat, n_requests=args.serve_requests,
                                                seed=k, warmup=max(10, args.serve_requests // 20))
        lat = np.asarray(lat)
        loads.append({"load": f, "offered_req_per_s": offered, "throughput_req_per_s": thr,
                      "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
                      "requests": int(lat.size)})
        log(f"[bench] serving load {f}: {thr:.1f} req/s, p50 {loads[-1]['p50_ms']:.1f} ms, "
            f"p99 {loads[-1]['p99_ms']:.1f} ms")
    sv.close()
    return {"workload": f"serving: {args.serve_problems} resident problems, grid uniform over "
                        f"{{128,256,512,1024}}^2 (E = max(1+0.1z,0.5), corr 8 px), AT1/AT2 alternating, "
                        f"strain-spectral, crack set; request = next load step of the problem's 200-step ramp; "
                        f"scratch budget {args.serve_scratch_gb:g} GB (admission by footprint)",
            "saturation_req_per_s": sat, "slots": info["slots"], "classes": info["classes"],
            "loads": loads}


KERNEL_SOURCES = ("spff_kernels.hip", "spff_device.hpp", "spff_engine.hpp")
PMC_RECORD = os.path.join(ROOT, "profiles", "pmc_traffic_row_kernels_batched_64x512.txt")


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2203_16467_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(role):
    """HBM bytes per launch of the dominant kernel from the committed
    rocprofv3 --pmc record (FETCH_SIZE and WRITE_SIZE in KiB per dispatch,
    each scaled by the factor the same counter reads for a copy kernel of
    known size), or None if the record is missing, covers another kernel
    role, or was taken on kernel sources other than the ones built here."""
    if not os.path.exists(PMC_RECORD):
        return None
    rec = {}
    with open(PMC_RECORD) as f:
        for line in f:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                rec[k.strip()] = v.strip()
    try:
        if rec.get("kernel_source_sha256") != kernel_source_hash():
            return None
        fetch = float(rec[f"{role}.fetch_kib_per_dispatch"]) * float(rec["fetch_scale"])
        write = float(rec[f"{role}.write_kib_per_dispatch"]) * float(rec["write_scale"])
    except (KeyError, ValueError):
        return None
    return (fetch + write) * 1024.0


def cpu_leg(res, budget_s):
    """The FP64 oracle on one host core, realization 0 of the workload, for as
    many load steps as fit the budget (at least one)."""
    import numpy as np

    import oracle
    try:
        from threadpoolctl import threadpool_limits
        limiter = threadpool_limits(limits=1)
    except Exception:  # pragma: no cover
        limiter = None
    E = res["E0"].astype(np.float64)
    o = oracle.Problem(E, nu=0.2, ell=2.0, gc=1.0, at=1, split="spectral", tol_mech=1e-6, tol_pf=1e-6)
    # sample: mechanics-dominated steps from an early state of the ramp
    # (the oracle at a nucleation step can take hours)
    ramp = res["ramp"]
    t0 = time.perf_counter()
    cg = pf = 0
    k = 0
    while True:
        stt = o.load_step(ramp[20 + k])
        cg += stt["cg"]
        pf += stt["bccg"]
        k += 1
        if time.perf_counter() - t0 > budget_s:
            break
    dt = time.perf_counter() - t0
    if limiter is not None:
        limiter.unregister()
    n = E.shape[0]
    return {"value": (cg + pf) * n * n / dt, "unit": "grid-pt-iters/s", "cores": 1, "kind": "oracle",
            "sample": f"FP64 NumPy oracle, realization 0 ({n}x{n}), load steps 21..{20 + k} of the ramp from a "
                      f"zero state (mechanics Newton-CG dominated; {cg} CG + {pf} BCCG iterations in {dt:.1f}s), "
                      f"one thread",
            "host_cpus": os.cpu_count()}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--start", type=int, default=88, help="first timed load step of the 200-step ramp")
    ap.add_argument("--grid", type=int, default=512)
    ap.add_argument("--batch", type=int, default=64)
    ap.add_argument("--corr", type=float, default=16.0)
    ap.add_argument("--amp", type=float, default=0.2)
    ap.add_argument("--no-plain", dest="plain", action="store_false")
    ap.add_argument("--no-cpu-baseline", dest="cpu_baseline", action="store_false")
    ap.add_argument("--cpu-budget", type=float, default=15.0)
    ap.add_argument("--no-serving", dest="serving", action="store_false")
    ap.add_argument("--no-variants", dest="variants", action="store_false")
    ap.add_argument("--no-large", dest="large", action="store_false")
    ap.add_argument("--ticks-per-sync", type=int, default=32,
                    help="solver ticks per captured graph block between host status checks (32: the host "
                         "turnaround is ~1%% of the window; 16 costs ~2%%)")
    ap.add_argument("--serve-problems", type=int, default=200)
    ap.add_argument("--serve-requests", type=int, default=2000)
    ap.add_argument("--serve-loads", type=float, nargs="+", default=[0.5, 0.8, 0.95])
    ap.add_argument("--serve-arena-gb", type=float, default=8.0)
    ap.add_argument("--serve-scratch-gb", type=float, default=1.0)
    ap.add_argument("--no-autotune", dest="autotune", action="store_false")
    ap.add_argument("--plan-cache", default=None,
                    help="JSON cache of autotuned launch plans (default: the package's gfx950 cache; buckets "
                         "missing from it are tuned live)")
    ap.add_argument("--no-steady", dest="steady", action="store_false")
    ap.add_argument("--steady-start", type=int, default=40)
    ap.add_argument("--steady-steps", type=int, default=10)
    ap.add_argument("--verbose", action="store_true")
    ap.add_argument("--no-profile", dest="profile", action="store_false",
                    help="skip the replay of the window with the kernel timers (no roofline figures)")
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
    prof = res["prof"]
    if prof is None:  # --no-profile: no per-kernel figures
        prof = {"kernel_ms": {k: 0.0 for k in KERNELS + ("ctrl",)}, "kernel_span_ms": {k: 0.0 for k in KERNELS + ("ctrl",)},
                "launches": {k: 0 for k in KERNELS + ("ctrl",)}, "alg_bytes": {k: 0.0 for k in KERNELS + ("ctrl",)}}
    # a launch's time: its work-group activity plus half of the dead time to
    # the next kernel (drain and write-back belong to it, the next dispatch
    # does not); a kernel trace's duration lies between the two figures
    ktime = {k: 0.5 * (prof["kernel_ms"][k] + prof["kernel_span_ms"][k]) for k in KERNELS}
    dom = max(KERNELS, key=lambda k: ktime[k])
    ms = ktime[dom]
    achieved = prof["alg_bytes"][dom] / (ms * 1e-3) / 1e9 if ms > 0 else 0.0
    all_ms = sum(ktime[k] for k in KERNELS)
    all_b = sum(prof["alg_bytes"][k] for k in KERNELS)
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
                        f"uniaxial-strain ramp of 200 steps to 1.5 eps_M; timed load steps {args.start}.."
                        f"{args.start + args.steps - 1}; FP32 fields, FP64 reductions",
            "batch": res["B"], "grid": [res["n"], res["n"]], "parallelism": "single GPU",
        },
        "breakdown": {"cg_iters": res["cg"], "bccg_iters": res["pf"], "seconds": res["dt"],
                      "realizations_cracked": res["ncrack"], "status": res["status"],
                      "kernel_ms": ktime, "kernel_activity_ms": prof["kernel_ms"],
                      "kernel_span_ms": prof["kernel_span_ms"], "kernel_launches": prof["launches"],
                      "kernel_alg_bytes": prof["alg_bytes"],
                      "alg_GBs_all_fft_kernels": all_b / (all_ms * 1e-3) / 1e9 if all_ms > 0 else None,
                      "profiled_replay": res["replay"],
                      "steady_all_active": res["steady"]},
        "autotune": res["tuned"],
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": measured_traffic(dom),
                     "alg_bytes_per_launch": prof["alg_bytes"][dom] / max(prof["launches"][dom], 1),
                     "avg_launch_us": ms * 1e3 / max(prof["launches"][dom], 1)},
    }
    if args.plain:
        pl = plain_leg(args)
        out["plain_gpu"] = pl
        out["vs_plain"] = value / pl["value"]
    if args.serving:
        out["serving"] = serving_leg(args)
    if args.variants:
        out["variants"] = variants_leg(args)
    if args.large:
        out["large"] = large_leg(args)
    if args.cpu_baseline:
        out["cpu_baseline"] = cpu_leg(res, args.cpu_budget)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
