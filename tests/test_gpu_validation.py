"""Validation workloads of Sec. 4.1.1 on the GPU path (homogeneous domain
L = 100 l with a centred 50 l crack or a small void as initial phase field,
E = E0 = 1e4 G_c / l, nu = 0.2, AT1, damage irreversibility, strain-spectral
driving force with the stress-free isotropic contact model, tolerances
1e-6, uniaxial strain increments of 1e-4, until C_bar < 0.01 E0).

The grid is 512^2 (l = 5.12 px) where the paper uses the odd 511^2: the
GPU transforms need powers of two, and on an even grid the Nyquist
component of the strain is not representable (its gradient is zeroed), so
a pixel-wide crack cannot open freely.  Measured here (FP32, alternating
minimisation): crack IC stiffness 0.76 sigma_M/eps_M (printed 0.65; the
oracle gives 0.665 on the odd 255^2 grid, see the oracle tests), peak
stress 0.158 sigma_M (printed 0.16), final F_f 108.8 G_c l; void IC
stiffness 1.00 (printed: nearly 1), peak 0.757 sigma_M (printed 0.77),
final F_f 109.1 G_c l (printed 103.0).  The final profiles are about 19%
(L1) from the analytical one, against 5.6% / 6.6% printed: on the even grid
the crack band widens as the load grows (the oracle on 256^2 shows the
same, on 255^2 it does not).  Bounds on stiffness and profile are loose for
that reason.

The near-equilibrium runs (Algorithm 4 as a device-driven evolution,
(-F_phi)_max = 0.7 G_c/l, trigger 1 G_c/l, (d phi)_min = 1e-3 l^2) show the
paper's snap-back: the macroscopic strain falls while the crack runs (void:
from 0.0045 to 0.0004, the paper reports almost 3x).  Measured: crack IC
1761 iterations, peak 0.167 sigma_M; void IC 2299 iterations (paper 3024),
peak 0.774 sigma_M, F_f 108.1 (paper 102.6)."""

import numpy as np
import pytest

import spff_inputs as si
from oracle import phasefield as opf
from paper_2203_16467_amd import spff
from test_gpu_parity import torch_E

pytestmark = pytest.mark.gpu

N = 512
ELL = N / 100.0
E0 = 1e4 / ELL
EPS_M = 0.005809            # Sec. 3.3, uniaxial strain, AT1, nu = 0.2
SIGMA_M = 64.55 / ELL       # 64.55 G_c / l
STIFF = SIGMA_M / EPS_M     # sigma_M / eps_M = lambda + 2 mu at E0


def _run(phi0, nyquist=spff.NYQ_ZERO):
    import torch
    cfg = spff.default_config(nx=N, ny=N, at=1, split=spff.SPLIT_SPECTRAL, contact=spff.SPLIT_NONE,
                              irreversibility=spff.IRR_DAMAGE, ell=ELL, gc=1.0, nu=0.2, tol_mech=1e-6,
                              tol_pf=1e-6, use_graph=1, ticks_per_sync=16, nyquist=nyquist)
    p = spff.Problem(torch_E(np.full((N, N), E0), "fp32"), cfg, phi_init=torch.as_tensor(phi0, device="cuda:0"))
    hist = []
    for k in range(1, 120):
        _, st = p.load_step((0.0, k * 1e-4, 0.0))
        s = st[0]
        assert s["status"] >= 0
        hist.append(s)
        if s["C_bar"] < 0.01 * E0:
            break
    phi = p.get_fields(spff.FIELD_PHI, index=0)["phi"][0].double().cpu().numpy()
    p.close()
    return hist, phi


def _final_checks(hist, phi):
    """Broken sample, a crack near the centre row through the whole periodic
    width, no damage away from it; returns F_f / (G_c l) and the relative L1
    distance of phi from the analytical crack profile centred, column by
    column, on the crack (the crack may step by a few pixels where the two
    tips of a void's crack meet across the periodic boundary)."""
    assert hist[-1]["C_bar"] < 0.01 * E0
    c = N // 2
    band = int(np.ceil(2 * ELL))
    assert (phi[c - band:c + band + 1].max(axis=0) >= 0.95).all()
    d = np.abs(np.arange(N) - c)
    far = np.minimum(d, N - d) > 4 * ELL
    assert phi[far].max() < 1e-3
    ff = hist[-1]["F_f"] / ELL
    assert 95.0 <= ff <= 115.0, ff
    err = tot = 0.0
    for x in range(N):
        r = int(np.argmax(phi[:, x]))
        dd = np.abs(np.arange(N) - r)
        ana = opf.optimal_profile(np.minimum(dd, N - dd), 1, ELL)
        err += np.abs(phi[:, x] - ana).sum()
        tot += ana.sum()
    err /= tot
    assert err < 0.3, err
    return ff, err


def test_homogeneous_tension_initial_crack():
    hist, phi = _run(si.centre_crack(N, N, ELL, 50 * ELL))
    c0 = hist[0]["C_bar"] / STIFF
    peak = max(s["sigma_bar"][1] for s in hist) / SIGMA_M
    ff, err = _final_checks(hist, phi)
    print(f"crack IC: C0 {c0:.3f} sigma_M/eps_M, peak {peak:.3f} sigma_M, steps {len(hist)}, "
          f"F_f {ff:.2f} G_c l, L1 {err:.3f}")
    # the even grid stiffens the cracked domain (Nyquist gradient zeroed):
    # 0.76 here, 0.665 for the oracle on the odd 255^2 grid (printed: 0.65)
    assert 0.6 < c0 < 0.85
    assert peak == pytest.approx(0.16, rel=0.1)


def test_homogeneous_tension_small_void():
    hist, phi = _run(si.round_void(N, N, ELL))
    c0 = hist[0]["C_bar"] / STIFF
    peak = max(s["sigma_bar"][1] for s in hist) / SIGMA_M
    ff, err = _final_checks(hist, phi)
    print(f"void IC: C0 {c0:.3f} sigma_M/eps_M, peak {peak:.3f} sigma_M, steps {len(hist)}, "
          f"F_f {ff:.2f} G_c l, L1 {err:.3f}")
    assert c0 == pytest.approx(1.0, abs=0.02)
    assert peak == pytest.approx(0.77, rel=0.05)


def _run_near_eq(phi0, max_iter=6000):
    import torch
    cfg = spff.default_config(nx=N, ny=N, at=1, split=spff.SPLIT_SPECTRAL, contact=spff.SPLIT_NONE,
                              irreversibility=spff.IRR_DAMAGE, ell=ELL, gc=1.0, nu=0.2, tol_mech=1e-6,
                              tol_pf=1e-6, use_graph=1, ticks_per_sync=16, evolution=spff.EVOL_NEAR_EQ,
                              fphi_max=0.7 / ELL, drive_threshold=1.0 / ELL, deps_max=1e-4, eta=0.0,
                              dt_max=1.0, dphi_min=1e-3 * ELL * ELL)
    p = spff.Problem(torch_E(np.full((N, N), E0), "fp32"), cfg, phi_init=torch.as_tensor(phi0, device="cuda:0"))
    hist = []
    while len(hist) < max_iter:
        st, stats = p.run_evolution((0.0, 1e-4, 0.0), nsteps=200)
        assert st >= 0
        done = False
        for s in stats[0]:
            hist.append(s)
            if s["C_bar"] < 0.01 * E0:
                done = True
                break
        if done:
            break
    phi = p.get_fields(spff.FIELD_PHI, index=0)["phi"][0].double().cpu().numpy()
    p.close()
    return hist, phi


@pytest.mark.parametrize("ic", ["crack", "void"])
def test_homogeneous_tension_near_equilibrium(ic):
    phi0 = si.centre_crack(N, N, ELL, 50 * ELL) if ic == "crack" else si.round_void(N, N, ELL)
    hist, phi = _run_near_eq(phi0)
    i_peak = int(np.argmax([s["sigma_bar"][1] for s in hist]))
    peak = hist[i_peak]["sigma_bar"][1] / SIGMA_M
    eps_peak = hist[i_peak]["eps_bar"][1]
    eps_min_after = min(s["eps_bar"][1] for s in hist[i_peak:])
    ff, err = _final_checks(hist, phi)
    print(f"near-eq {ic} IC: {len(hist)} iterations, peak {peak:.3f} sigma_M at eps {eps_peak:.5f}, "
          f"strain falls to {eps_min_after:.5f}, F_f {ff:.2f} G_c l, L1 {err:.3f}")
    assert any(s["gamma"] < 1.0 for s in hist)
    # snap-back: the algorithm lowers the macroscopic strain during fracture
    assert eps_min_after < 0.7 * eps_peak
    if ic == "void":
        assert peak == pytest.approx(0.77, rel=0.05)


@pytest.mark.parametrize("ic", ["crack", "void"])
def test_homogeneous_tension_free_nyquist_matches_printed_results(ic):
    """With the Nyquist modes of the strain fluctuation left free (the even
    grid then behaves like the paper's odd ones), alternating minimisation
    reproduces the printed figures of Sec. 4.1.1: stiffness before fracture
    0.65 sigma_M/eps_M (crack) and nearly 1 (void), peak stress 0.16 and
    0.77 sigma_M, a final crack with the analytical profile (printed L1
    errors 5.6% and 6.6%) and about G_c per unit length of crack (printed
    F_f 103.0 G_c l for the void; 100 is ideal)."""
    phi0 = si.centre_crack(N, N, ELL, 50 * ELL) if ic == "crack" else si.round_void(N, N, ELL)
    hist, phi = _run(phi0, spff.NYQ_FREE)
    c0 = hist[0]["C_bar"] / STIFF
    peak = max(s["sigma_bar"][1] for s in hist) / SIGMA_M
    ff, err = _final_checks(hist, phi)
    print(f"free Nyquist, {ic} IC: C0 {c0:.3f} sigma_M/eps_M, peak {peak:.3f} sigma_M, steps {len(hist)}, "
          f"F_f {ff:.2f} G_c l, L1 {err:.3f}")
    if ic == "crack":
        assert c0 == pytest.approx(0.65, rel=0.05)
        assert peak == pytest.approx(0.16, rel=0.1)
    else:
        assert c0 == pytest.approx(1.0, abs=0.02)
        assert peak == pytest.approx(0.77, rel=0.05)
    assert err < 0.1
    assert 95.0 <= ff <= 110.0
