"""GPU: continuous-batching server.  Each result is the same alone and in
the mix (bitwise with fixed launch plans, within the FP32 contract without),
admission respects the scratch budget, requests of one problem run in order."""

import numpy as np
import pytest

import spff_inputs as si
from gpu_common import device
from paper_2203_16467_amd import serving, spff

pytestmark = pytest.mark.gpu

PLAN = dict(plan_rows=2, plan_cols=1, plan_threads=256)


def _problems():
    """(cfg kwargs, E) for a small mixed population: two grid sizes, AT1 and
    AT2, different seeds."""
    out = []
    for i, (n, at) in enumerate([(64, 1), (64, 2), (128, 1), (64, 1), (128, 2), (64, 2)]):
        E = si.young_modulus(n, 4.0 if n == 64 else 8.0, 0.2, 4000 + i)
        out.append((dict(nx=n, ny=n, at=at), E))
    return out


def _ramp(n_steps=4, first=8):
    return si.uniaxial_ramp(20, 0.2, 2.0)[first:first + n_steps]


def _alone(kw, E, ramp, plan):
    import torch
    cfg = spff.default_config(**kw, **plan)
    p = spff.Problem(torch.as_tensor(E, device=device()), cfg)
    stats = [p.load_step(eb)[1][0] for eb in ramp]
    f = p.get_fields(spff.FIELD_PHI | spff.FIELD_EPS_STAR, 0)
    out = {k: v.double().cpu().numpy() for k, v in f.items()}
    p.close()
    return stats, out


@pytest.mark.parametrize("fixed_plan", [True, False])
def test_alone_equals_mix(fixed_plan):
    import torch
    plan = PLAN if fixed_plan else {}
    probs = _problems()
    ramp = _ramp()
    # scratch for about two slots per class: forces queueing and admission
    sv = spff.Server(arena_bytes=256 << 20, scratch_budget_bytes=3 * (128 * 128 * 48 + 64 * 64 * 48) * 2,
                     ticks_per_sync=4, use_graph=1)
    ids = [sv.register(spff.default_config(**kw, **plan), torch.as_tensor(E, device=device())) for kw, E in probs]
    # interleaved submissions: step k of every problem before step k+1
    tickets = {i: [] for i in ids}
    for k in range(len(ramp)):
        for i in ids:
            tickets[i].append(sv.submit(i, ramp[k]))
    while True:
        done, pending = sv.progress(4)
        if pending == 0:
            break
    info = sv.info()
    assert info["classes"] == 2 and info["slots"] >= 2
    for i, (kw, E) in zip(ids, probs):
        mix = [sv.poll(t) for t in tickets[i]]
        assert all(m is not None for m in mix)
        stats, alone = _alone(kw, E, ramp, plan)
        f = sv.get_fields(i, spff.FIELD_PHI | spff.FIELD_EPS_STAR)
        phi = f["phi"].double().cpu().numpy()[0]
        eps = f["eps_star"].double().cpu().numpy()
        assert phi.shape == alone["phi"][0].shape and eps.shape == alone["eps_star"].shape
        if fixed_plan:
            assert np.array_equal(phi, alone["phi"][0]), (i, np.abs(phi - alone["phi"][0]).max())
            assert np.array_equal(eps, alone["eps_star"]), i
            for a, b in zip(mix, stats):
                assert (a["cg_iters"], a["bccg_iters"], a["am_iters"]) == \
                    (b["cg_iters"], b["bccg_iters"], b["am_iters"])
        else:
            assert np.abs(phi - alone["phi"][0]).max() <= 1e-3
            assert np.linalg.norm(eps - alone["eps_star"]) <= 1e-4 * np.linalg.norm(alone["eps_star"]) + 1e-12
    sv.close()


def test_requests_of_one_problem_run_in_order_and_poll_semantics():
    import torch
    kw, E = _problems()[1]
    sv = spff.Server(arena_bytes=64 << 20, ticks_per_sync=2)
    pid = sv.register(spff.default_config(**kw), torch.as_tensor(E, device=device()))
    ramp = _ramp(3)
    ts = [sv.submit(pid, eb) for eb in ramp]
    assert sv.poll(ts[-1]) is None  # pending
    while sv.progress(8)[1] > 0:
        pass
    got = [sv.poll(t) for t in ts]
    stats, _ = _alone(kw, E, ramp, {})
    assert [g["sigma_bar"][1] for g in got] == pytest.approx([s["sigma_bar"][1] for s in stats], rel=1e-5)
    with pytest.raises(spff.SpffError):
        sv.poll(ts[0])  # already collected
    with pytest.raises(spff.SpffError):
        sv.poll(10 ** 9)
    sv.close()


def test_register_validates_and_arena_bounds():
    import torch
    sv = spff.Server(arena_bytes=1 << 20)
    E = np.ones((64, 64), np.float32)
    E[1, 1] = 0.0
    with pytest.raises(spff.SpffError) as ei:
        sv.register(spff.default_config(nx=64, ny=64), torch.as_tensor(E, device=device()))
    assert ei.value.status == spff.E_INVALID
    with pytest.raises(spff.SpffError) as ei:
        sv.register(spff.default_config(nx=512, ny=512), torch.ones((512, 512), device=device()))
    assert ei.value.status == spff.E_NOMEM
    sv.close()


def test_poisson_driver_smoke():
    import torch
    sv = spff.Server(arena_bytes=128 << 20, ticks_per_sync=4)
    ramps = {}
    for kw, E in _problems()[:4]:
        pid = sv.register(spff.default_config(**kw), torch.as_tensor(E, device=device()))
        ramps[pid] = si.uniaxial_ramp(20, 0.2, 2.0)
    cursor = {pid: 2 for pid in ramps}
    rate, lat, wall, _, left = serving.run_closed(sv, ramps, cursor, 2)
    assert left == []
    assert rate > 0 and len(lat) == 8 and all(c == 4 for c in cursor.values())
    thr, lat2, offered, res, cens = serving.run_poisson(sv, ramps, cursor, rate=0.5 * rate, n_requests=12,
                                                        seed=1)
    assert cens == 0
    assert len(lat2) == 12 and thr > 0 and sum(cursor.values()) == 16 + 12
    # latency from arrival includes the server's own submit-to-completion time
    assert all(l >= r["wall_ms"] - 1e-6 for l, r in zip(lat2, res))
    sv.close()


@pytest.mark.parametrize("mode", ["time", "near_eq"])
def test_evolution_state_is_kept_per_problem(mode):
    """Algorithms 3 and 4 carry state between iterations (dt, the trigger
    flag).  Served problems share slots (the scratch budget holds two slots
    for four problems), so the server keeps that state per problem: each
    problem's iterations equal those of the same problem run alone, bit for
    bit with fixed launch plans, whatever slot served each request."""
    import torch
    ramp = si.uniaxial_ramp(20, 0.2, 2.0)
    deps = ramp[1] - ramp[0]
    if mode == "time":
        extra = dict(evolution=spff.EVOL_TIME, eta=0.5, dt_max=1.0, dt_min=1e-3, dphi_max=20.0, dphi_min=1e-3)
    else:
        extra = dict(evolution=spff.EVOL_NEAR_EQ, fphi_max=0.35, drive_threshold=0.5,
                     deps_max=float(np.abs(deps).max()), dphi_min=1e-3)
    Es = [si.young_modulus(64, 4.0, 0.1, 1000)] + [si.young_modulus(64, 4.0, 0.2, 1001 + i) for i in range(3)]
    kw = dict(nx=64, ny=64, at=1, **extra, **PLAN)
    sv = spff.Server(arena_bytes=64 << 20, scratch_budget_bytes=2 * 64 * 64 * 48 * 2, ticks_per_sync=4,
                     use_graph=1)
    ids = [sv.register(spff.default_config(**kw), torch.as_tensor(E, device=device())) for E in Es]
    K = 10
    eb = {i: np.asarray(ramp[11], dtype=np.float64) for i in ids}
    hist = {i: [] for i in ids}
    for k in range(K):
        tickets = {i: sv.submit(i, eb[i]) for i in ids}
        while True:
            _, pending = sv.progress(4)
            if pending == 0:
                break
        for i in ids:
            s = sv.poll(tickets[i])
            hist[i].append(s)
            eb[i] = np.asarray(s["eps_bar"]) + (deps if s["advance"] else 0.0)
    for i, E in zip(ids, Es):
        p = spff.Problem(torch.as_tensor(E, device=device()), spff.default_config(**kw))
        e = np.asarray(ramp[11], dtype=np.float64)
        for k in range(K):
            _, st = p.load_step(e)
            a, b = hist[i][k], st[0]
            for key in ("cg_iters", "bccg_iters", "advance", "halvings", "ne_flag"):
                assert a[key] == b[key], (i, k, key)
            assert a["dt"] == b["dt"] and a["gamma"] == b["gamma"] and a["eps_bar"] == b["eps_bar"], (i, k)
            e = np.asarray(b["eps_bar"]) + (deps if b["advance"] else 0.0)
        f = sv.get_fields(i, spff.FIELD_PHI)["phi"].double().cpu().numpy()
        g = p.get_fields(spff.FIELD_PHI, 0)["phi"].double().cpu().numpy()
        assert np.array_equal(f, g), i
        p.close()
    if mode == "time":
        assert any(s["halvings"] > 0 for h in hist.values() for s in h)
    else:
        assert any(s["gamma"] < 1.0 for h in hist.values() for s in h)
    sv.close()


def _onset_step(kw, E, ramp, chunk=40):
    """First load step whose phase field leaves zero (AT1: onset of damage),
    running the problem alone with alternating minimisation capped as in kw."""
    import torch
    p = spff.Problem(torch.as_tensor(E, device=device()), spff.default_config(**kw))
    try:
        for c0 in range(0, len(ramp), chunk):
            _, stats = p.run_sequence(ramp[c0:c0 + chunk])
            for k, s in enumerate(stats[0]):
                if s["phi_max"] > 0.0:
                    return c0 + k
    finally:
        p.close()
    return None


@pytest.mark.parametrize("n", [512, 1024])
def test_served_nucleation_step_large_grids(n):
    """The serving workload's large grids (C4 recipe: E = max(1 + 0.1 z,
    0.5), corr 8 px, AT1, strain-spectral split) at the load step where the
    phase field first leaves zero: a problem served in a mix with a smaller
    one (requests walking its ramp from the start) ends that step bit for bit
    where the same problem run alone does, and the alone step matches the
    FP64 oracle started from the same state (FP32 contract).  Alternating
    minimisation is capped at 2 iterations on every side (the uncapped
    onset of a crack runs hundreds of iterations, a path FP32 and FP64 need
    not share iteration by iteration; the oracle at 1024^2 takes minutes per
    uncapped step)."""
    import torch
    ramp = si.uniaxial_ramp(200, 0.2, 2.0)
    E = si.young_modulus(n, 8.0, 0.1, 4000 + n // 256)
    kw = dict(nx=n, ny=n, at=1, max_am=2, **PLAN)
    k = _onset_step(kw, E, ramp)
    assert k is not None and k > 20
    print(f"{n}^2: onset at load step {k}", flush=True)
    # alone: to step k - 1, snapshot, step k
    p = spff.Problem(torch.as_tensor(E, device=device()), spff.default_config(**kw))
    p.run_sequence(ramp[:k])
    before, eb = p.get_state()
    _, alone = p.load_step(ramp[k])
    after, _ = p.get_state()
    assert alone[0]["phi_max"] > 0.0 and alone[0]["bccg_iters"] > 0
    # served in a mix with a small AT2 problem
    sv = spff.Server(arena_bytes=int(24 * n * n * 4 + (64 << 20)), ticks_per_sync=4, use_graph=1)
    small = sv.register(spff.default_config(nx=128, ny=128, at=2, **PLAN),
                        torch.as_tensor(si.young_modulus(128, 8.0, 0.1, 4100), device=device()))
    pid = sv.register(spff.default_config(**kw), torch.as_tensor(E, device=device()))
    tks = [sv.submit(pid, ramp[j]) for j in range(k + 1)]
    for j in range(2 * k):
        sv.submit(small, ramp[j % 120])
    while sv.progress(8)[1] > 0:
        pass
    served = [sv.poll(t) for t in tks][-1]
    f = sv.get_fields(pid, spff.FIELD_PHI | spff.FIELD_PHI_REF | spff.FIELD_EPS_STAR)
    got = torch.cat([f["eps_star"], f["phi"], f["phi_ref"]]).cpu()
    assert torch.equal(got, after[0].cpu())
    for key in ("am_iters", "cg_iters", "bccg_iters", "F_e", "F_f"):
        assert served[key] == alone[0][key], key
    sv.close()
    # alone against the oracle from the same state
    from gpu_common import oracle_for, planes_to_tensor, gpu_fields, oracle_fields
    from oracle import constitutive as ocm
    from test_gpu_parity import compare
    cfg = spff.default_config(**kw)
    o = oracle_for(E, cfg, tol=1e-8, max_am=2)
    s = before[0].double().cpu().numpy()
    o.set_state({"eps_star": planes_to_tensor(s[0:3]), "phi": s[3], "phi_ref": s[4],
                 "eps_bar": ocm.sym_tensor(*eb[0])})
    ost = o.load_step(ramp[k])
    cmp = compare(gpu_fields(p), oracle_fields(o), "fp32")
    print(n, k, cmp, alone[0]["am_iters"], ost["am"], alone[0]["bccg_iters"], ost["bccg"], flush=True)
    assert alone[0]["am_iters"] == ost["am"]
    tot = ost["F_e"] + ost["F_f"]
    assert abs(alone[0]["F_e"] - ost["F_e"]) <= 1e-4 * tot
    assert abs(alone[0]["F_f"] - ost["F_f"]) <= 1e-4 * tot
    p.close()
