"""Pins for oracle.phasefield: F_phi as the variation of the energy, the 1-D
optimal profiles and unit crack energy (Sec. 2.1), brute-force box QP and
KKT conditions for BCCG (Sec. 3.1.2, Alg. 1), homogeneous fixed points."""

import numpy as np
import pytest
from scipy.optimize import minimize

from oracle import phasefield as pf
from oracle import spectral as sp


def total_pf_energy(phi, psi_plus, at, gc, ell):
    """sum_x h(phi) psi0+ + F_f(phi): the phi-dependent part of F."""
    return float(np.sum((1 - phi) ** 2 * psi_plus)) + pf.fracture_energy(phi, at, gc, ell)


@pytest.mark.parametrize("at", [1, 2])
def test_f_phi_is_energy_variation(at):
    """F_phi (with the factor-2 reading) is the gradient of
    sum h psi0+ + F_f over the grid values, by central differences."""
    rng = np.random.default_rng(20)
    shape = (6, 8)
    phi = rng.uniform(0, 1, shape)
    psi = rng.uniform(0, 0.5, shape)
    gc, ell = 1.3, 1.7
    g = pf.f_phi(phi, psi, at, gc, ell)
    h = 1e-6
    for _ in range(5):
        d = rng.standard_normal(shape)
        fd = (total_pf_energy(phi + h * d, psi, at, gc, ell)
              - total_pf_energy(phi - h * d, psi, at, gc, ell)) / (2 * h)
        assert fd == pytest.approx(float(np.sum(g * d)), rel=1e-7, abs=1e-9)


def line_crack(at, nx, ell, ny=4):
    phi_ref = np.zeros((ny, nx))
    phi_ref[:, nx // 2] = 1.0
    lo = pf.constraint_field(phi_ref, "crack_set")
    op = pf.Operator(np.zeros((ny, nx)), at, 1.0, ell)
    phi, info = pf.bccg(phi_ref, lo, np.ones_like(lo), op, 1e-11, max_iter=20000)
    ana = pf.optimal_profile(np.arange(nx) - nx // 2, at, ell)
    err = np.abs(phi[0] - ana).sum() / ana.sum()
    return phi, err, pf.fracture_energy(phi, at, 1.0, ell) / ny


@pytest.mark.parametrize("at,nx", [(1, 128), (2, 256)])
def test_one_d_profiles_and_unit_crack_energy(at, nx):
    """Sec. 2.1: the optimal 1-D profiles are (1 - |x|/2l)^2 (AT1) and
    exp(-|x|/l) (AT2) and F_f is G_c per unit crack length.  A phi = 1 line
    held by crack-set irreversibility at zero strain relaxes to the profile;
    the discretisation error shrinks as l/dx grows (the paper reports about
    6% relative L1 at l/dx ~ 5 in 2-D, Sec. 4.1.1)."""
    errs, energies = [], []
    for ell in (4.0, 8.0):
        phi, err, ff = line_crack(at, nx, ell)
        assert np.all(phi >= -1e-12) and np.all(phi <= 1 + 1e-12)
        # the solution does not depend on y
        np.testing.assert_allclose(phi, phi[:1].repeat(phi.shape[0], 0), atol=1e-9)
        errs.append(err)
        energies.append(ff)
    assert errs[1] < 0.05
    assert errs[1] < 0.7 * errs[0]
    assert abs(energies[1] - 1.0) < 0.03
    assert abs(energies[1] - 1.0) < abs(energies[0] - 1.0)


def _tiny_problem(seed, shape=(4, 5), at=1):
    rng = np.random.default_rng(seed)
    psi = rng.uniform(0.0, 0.6, shape)
    phi_ref = np.where(rng.uniform(0, 1, shape) < 0.3, rng.uniform(0.85, 1.0, shape), rng.uniform(0, 0.5, shape))
    return psi, phi_ref


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
@pytest.mark.parametrize("at", [1, 2])
@pytest.mark.parametrize("irr", ["crack_set", "damage"])
def test_bccg_matches_brute_force_box_qp(seed, at, irr):
    """BCCG returns the minimiser of 1/2 phi.J phi - b.phi on the box
    [phi_con(phi_ref), 1]; brute force with a bound-constrained quasi-Newton
    solver on the dense J of a 4x5 grid."""
    psi, phi_ref = _tiny_problem(seed, at=at)
    gc, ell = 1.0, 0.8
    op = pf.Operator(psi, at, gc, ell)
    lo = pf.constraint_field(phi_ref, irr)
    hi = np.ones_like(lo)
    phi, info = pf.bccg(np.zeros_like(psi), lo, hi, op, 1e-13)
    J = op.dense()
    b = op.b.ravel()
    res = minimize(lambda x: (0.5 * x @ J @ x - b @ x, J @ x - b), lo.ravel().copy(), jac=True,
                   method="L-BFGS-B", bounds=list(zip(lo.ravel(), hi.ravel())),
                   options={"gtol": 1e-14, "ftol": 1e-16, "maxiter": 10000})
    np.testing.assert_allclose(phi.ravel(), res.x, atol=2e-6)
    # KKT conditions on the BCCG output
    r = op.J(phi) - op.b
    free = (phi > lo + 1e-12) & (phi < hi - 1e-12)
    assert np.all(np.abs(r[free]) < 1e-9)
    assert np.all(r[(phi <= lo + 1e-12) & ~free] > -1e-9)
    assert np.all(r[(phi >= hi - 1e-12) & ~free] < 1e-9)


def test_bccg_without_active_bounds_is_linear_solve():
    """With bounds far away BCCG is plain CG: phi = J^-1 b."""
    rng = np.random.default_rng(21)
    psi = rng.uniform(0.3, 0.6, (6, 6))
    op = pf.Operator(psi, 2, 1.0, 1.0)
    J = op.dense()
    want = np.linalg.solve(J, op.b.ravel())
    assert want.min() > 0 and want.max() < 1
    phi, _ = pf.bccg(np.full((6, 6), 0.5), np.full((6, 6), -10.0), np.full((6, 6), 10.0), op, 1e-13)
    np.testing.assert_allclose(phi.ravel(), want, atol=1e-10)


@pytest.mark.parametrize("psi", [0.05, 0.2, 0.6, 3.0])
def test_homogeneous_fixed_points(psi):
    """Uniform psi0+ with no Laplacian contribution: AT1 phi = 1 - 3 G_c/(16 l
    psi0+) when 2 psi0+ > 3 G_c/(8 l), else 0; AT2 phi = 2 psi0+/(2 psi0+ +
    G_c/l)."""
    gc, ell = 1.0, 2.0
    field = np.full((8, 8), psi)
    lo, hi = np.zeros((8, 8)), np.ones((8, 8))
    phi1, _ = pf.bccg(np.zeros((8, 8)), lo, hi, pf.Operator(field, 1, gc, ell), 1e-12)
    want1 = max(0.0, 1 - 3 * gc / (16 * ell * psi))
    np.testing.assert_allclose(phi1, want1, atol=1e-10)
    phi2, _ = pf.bccg(np.zeros((8, 8)), lo, hi, pf.Operator(field, 2, gc, ell), 1e-12)
    np.testing.assert_allclose(phi2, 2 * psi / (2 * psi + gc / ell), atol=1e-10)


def test_constraint_field_threshold_inclusive():
    ref = np.array([0.0, 0.5, 0.9, 0.95, 1.0])
    np.testing.assert_array_equal(pf.constraint_field(ref, "crack_set"), [0, 0, 0.9, 0.95, 1.0])
    np.testing.assert_array_equal(pf.constraint_field(ref, "damage"), ref)


def test_fracture_energy_gradient_term_is_laplacian_form():
    rng = np.random.default_rng(22)
    phi = rng.uniform(0, 1, (8, 10))
    assert sp.grad_sq_sum(phi) >= 0
    # plane wave: sum |grad|^2 = |xi|^2 sum phi^2
    y, x = np.meshgrid(np.arange(8), np.arange(10), indexing="ij")
    f = np.cos(2 * np.pi * (2 * x / 10 + 1 * y / 8))
    xi2 = (2 * np.pi * 2 / 10) ** 2 + (2 * np.pi / 8) ** 2
    assert sp.grad_sq_sum(f) == pytest.approx(xi2 * np.sum(f * f), rel=1e-12)
