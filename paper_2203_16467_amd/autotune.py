"""Autotuner for the FFT launch plans.

A handle launches its three FFT kernels (row-forward, column, row-inverse)
over a power-of-two bucket of active problem slots; for every bucket the
library holds a launch plan (``spff_plan``): the kind of FFT kernel for rows
and for columns (LDS Stockham radix-4/2 with one point pair per thread, or
register-resident radix-8 with eight points per lane -- sixteen for
1024- and 2048-point transforms, columns of those sizes also eight --, or for
rows radix-4 with four), rows / columns per work-group and threads per
work-group.  The built-in plans come from a
heuristic; this module times the alternatives on the device and installs the
fastest.

Method: for a bucket of v slots a tuning handle holds v identical copies of
a synthetic microstructure (so that all v stay active together), AT2 so that
every load step runs both the mechanics CG (three-component ticks) and the
phase-field BCCG (one-component ticks).  Each candidate runs the same capped
load step from the same saved state, once to warm up (graph capture), once
timed with the library's device-clock kernel timers.  Row plans are ranked by
row-forward + row-inverse time per tick, column plans by column time per
tick (the kernels are timed apart, so the two searches are independent).
Results are kept in a JSON cache keyed by grid, precision and bucket size.
"""

import json
import os
import time

import numpy as np

from . import spff

THREADS = 256
LDS_BYTES = 160 * 1024


def _pow2_range(lo, hi):
    v, out = lo, []
    while v <= hi:
        out.append(v)
        v *= 2
    return out


def row_candidates(cfg):
    """Row halves of the candidate plans: (kind, rows, threads)."""
    M = cfg.nx // 2
    csize = 8 if cfg.precision == spff.FP32 else 16
    out = []
    for R in _pow2_range(1, min(cfg.ny, 32)):
        for T in (128, 256):
            if T * 8 >= M and 3 * R * (M + 1) * csize <= LDS_BYTES // 2:
                out.append((spff.FFT_LDS, R, T))
    for kind, E, Mmax in ((spff.FFT_REG, 8 if M <= 512 else 16, 1024), (spff.FFT_REG4, 4, 256)):
        if cfg.precision == spff.FP32 and 64 <= M <= Mmax:
            L = M // E
            for R in _pow2_range(max(1, 64 // L), THREADS // L):
                if R <= cfg.ny:
                    out.append((kind, R, R * L))
    return out


def col_candidates(cfg):
    """Column halves of the candidate plans: (kind, cols, threads)."""
    M = cfg.nx // 2
    csize = 8 if cfg.precision == spff.FP32 else 16
    out = []
    for W in _pow2_range(1, min(M, 16)):
        for T in (128, 256):
            if T * 8 >= cfg.ny and 3 * W * (cfg.ny + 1) * csize <= LDS_BYTES // 2:
                out.append((spff.FFT_LDS, W, T))
    if cfg.precision == spff.FP32 and cfg.ny in (128, 256, 512, 1024, 2048):
        L = cfg.ny // (8 if cfg.ny <= 512 else 16)
        # 16 points per lane for 1024 and 2048 points: a 2048-point column
        # (128 lanes) is alone in its work-group
        for W in _pow2_range(max(1, 64 // L), 1 if L > 64 else THREADS // L):
            if W <= M:
                out.append((spff.FFT_REG, W, W * L))
        if cfg.ny >= 1024:
            # 8 points per lane: ny/8 lanes, one column per work-group
            out.append((spff.FFT_REG, 1, cfg.ny // 8))
    return out


def _key(nx, ny, precision, v):
    return f"{nx}x{ny}:{'fp64' if precision == spff.FP64 else 'fp32'}:b{v}"


def _time_plan(prob, bidx, plan, state, eps):
    """Per-tick kernel times (ms) of one plan on the tuning handle."""
    prob.set_plan(bidx, plan)
    st, eb = state
    prob.set_state(st, eb)
    prob.load_step(eps)  # warm-up: captures the bucket's graph
    prob.set_state(st, eb)
    prob.profile_enable(True)
    prob.load_step(eps)
    pr = prob.profile_read()
    prob.profile_enable(False)
    t = max(pr["ticks"], 1)
    # activity plus half the dead time to the next kernel (write-back heavy
    # plans pay for it there)
    km = {k: 0.5 * (pr["kernel_ms"][k] + pr["kernel_span_ms"][k]) for k in pr["kernel_ms"]}
    return (km["rowfwd"] + km["rowinv"]) / t, km["col"] / t


def tune_bucket(nx, ny, v, precision=spff.FP32, seed=7, log=None):
    """Best plan for a bucket of v slots of an nx x ny grid."""
    import torch
    import spff_inputs as si

    E1 = si.young_modulus(nx, max(2.0, nx / 32.0), 0.2, seed, ny=ny)
    E = torch.as_tensor(np.broadcast_to(E1, (v, ny, nx)).copy(), device="cuda:0")
    if precision == spff.FP64:
        E = E.double()
    cfg = spff.default_config(nx=nx, ny=ny, at=2, precision=precision, use_graph=1, ticks_per_sync=16)
    cfg.max_am, cfg.max_cg, cfg.max_bccg = 2, 24, 24
    prob = spff.Problem(E, cfg)
    ramp = si.uniaxial_ramp(20, cfg.nu, cfg.ell)
    prob.load_step(ramp[8])
    state = prob.get_state()
    eps = ramp[10]
    bidx = prob.plan_buckets().index(v)
    base = prob.get_plan(bidx)
    best_row, best_col = None, None
    for kind, R, T in row_candidates(cfg):
        plan = dict(base, row_kind=kind, rows=R, row_threads=T)
        try:
            tr, _ = _time_plan(prob, bidx, plan, state, eps)
        except spff.SpffError:
            continue
        if log:
            log(f"[autotune] {nx}x{ny} b{v} rows kind {kind} R {R} T {T}: {tr * 1e3:.1f} us/tick")
        if best_row is None or tr < best_row[0]:
            best_row = (tr, kind, R, T)
    for kind, W, T in col_candidates(cfg):
        plan = dict(base, row_kind=best_row[1], rows=best_row[2], row_threads=best_row[3], col_kind=kind,
                    cols=W, col_threads=T)
        try:
            _, tc = _time_plan(prob, bidx, plan, state, eps)
        except spff.SpffError:
            continue
        if log:
            log(f"[autotune] {nx}x{ny} b{v} cols kind {kind} W {W} T {T}: {tc * 1e3:.1f} us/tick")
        if best_col is None or tc < best_col[0]:
            best_col = (tc, kind, W, T)
    prob.close()
    plan = dict(row_kind=best_row[1], rows=best_row[2], row_threads=best_row[3], col_kind=best_col[1],
                cols=best_col[2], col_threads=best_col[3])
    return plan, {"row_us_per_tick": best_row[0] * 1e3, "col_us_per_tick": best_col[0] * 1e3}


DEFAULT_CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "plans_gfx950.json")


def tune(nx, ny, batch, precision=spff.FP32, cache=DEFAULT_CACHE, write_cache=False, log=None):
    """Plans for every bucket of a batch of `batch` problems; returns
    ({bucket size: plan}, {bucket size: timings}, source) where source is
    "cache" if every bucket was found in the cache file (buckets missing
    from it are tuned; the file is rewritten only with write_cache)."""
    sizes = []
    v = 1
    while True:
        sizes.append(min(v, batch))
        if v >= batch:
            break
        v *= 2
    store = {}
    if cache and os.path.exists(cache):
        with open(cache) as f:
            store = json.load(f)
    plans, times, hit = {}, {}, True
    for v in sizes:
        k = _key(nx, ny, precision, v)
        if k in store:
            plans[v] = store[k]["plan"]
            times[v] = store[k]["timing"]
            continue
        hit = False
        t0 = time.time()
        plans[v], times[v] = tune_bucket(nx, ny, v, precision, log=log)
        store[k] = {"plan": plans[v], "timing": times[v]}
        if log:
            log(f"[autotune] {k}: {plans[v]} ({time.time() - t0:.1f} s)")
    if cache and write_cache and not hit:
        os.makedirs(os.path.dirname(os.path.abspath(cache)), exist_ok=True)
        with open(cache, "w") as f:
            json.dump(store, f, indent=1, sort_keys=True)
    return plans, times, "cache" if hit else "tuned"


def apply(prob, plans):
    """Install tuned plans ({bucket size: plan}) on a handle."""
    for i, v in enumerate(prob.plan_buckets()):
        if v in plans:
            prob.set_plan(i, plans[v])


def main(argv=None):
    """python -m paper_2203_16467_amd.autotune NX NY BATCH [--out FILE]:
    tune every bucket and write the plans to FILE (default: the package's
    gfx950 cache)."""
    import argparse
    import sys
    ap = argparse.ArgumentParser()
    ap.add_argument("nx", type=int)
    ap.add_argument("ny", type=int)
    ap.add_argument("batch", type=int)
    ap.add_argument("--out", default=DEFAULT_CACHE)
    ap.add_argument("--fp64", action="store_true")
    a = ap.parse_args(argv)
    log = lambda *m: print(*m, file=sys.stderr, flush=True)  # noqa: E731
    plans, _, src = tune(a.nx, a.ny, a.batch, spff.FP64 if a.fp64 else spff.FP32, cache=a.out, write_cache=True,
                         log=log)
    print(json.dumps({str(k): v for k, v in plans.items()}), src)


if __name__ == "__main__":
    main()
