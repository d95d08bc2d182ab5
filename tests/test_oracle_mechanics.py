"""Pins for oracle.mechanics: closed forms (homogeneous, laminate), energy
minimisation by brute force on a tiny grid, equivariances, symmetry of the
effective stiffness (Sec. 3.1.1)."""

import numpy as np
import pytest
from scipy.optimize import minimize

from oracle import constitutive as cm
from oracle import mechanics as mech
from oracle import spectral as sp


def solve(E, phi, eps_bar, split, nu=0.2, tol=1e-11, k_res=0.0):
    lam, mu = cm.lame(E, nu)
    eps_star = np.zeros(E.shape + (2, 2))
    eps_star, info = mech.solve(eps_star, np.asarray(eps_bar, float), phi, lam, mu, split,
                                k_res=k_res, tol_rel=tol, max_newton=50)
    assert info["converged"], info
    sig = cm.stress(eps_bar + eps_star, phi, lam, mu, split, k_res)
    return eps_star, sig, info


@pytest.mark.parametrize("split", ["none", "spectral"])
def test_homogeneous_closed_form(split):
    """Uniform E and phi: eps* = 0 and sigma = C : eps_bar; for uniaxial
    strain e: sigma_yy = h (lam + 2 mu) e, sigma_xx = h lam e."""
    E = np.full((8, 8), 1.3)
    phi = np.full((8, 8), 0.25)
    e = 0.37
    eps_star, sig, _ = solve(E, phi, np.diag([0.0, e]), split)
    np.testing.assert_allclose(eps_star, 0.0, atol=1e-14)
    lam, mu = cm.lame(1.3, 0.2)
    h = 0.75 ** 2
    np.testing.assert_allclose(sig[..., 1, 1], h * (lam + 2 * mu) * e, rtol=1e-13)
    np.testing.assert_allclose(sig[..., 0, 0], h * lam * e, rtol=1e-13)


@pytest.mark.parametrize("shape", [(9, 9), (15, 7)])
@pytest.mark.parametrize("split", ["none", "spectral"])
def test_laminate_uniaxial(shape, split):
    """E varying along y only (odd grid: every grid function is a trig
    polynomial): sigma_yy is uniform and equals e / mean(1/M),
    M = lam + 2 mu; eps_xx = 0 (compatibility across the layers)."""
    ny, nx = shape
    rng = np.random.default_rng(10)
    Ey = rng.uniform(0.5, 1.5, ny)
    E = Ey[:, None] * np.ones((1, nx))
    phi = np.zeros(shape)
    e = 0.2
    eps_star, sig, _ = solve(E, phi, np.diag([0.0, e]), split)
    lam, mu = cm.lame(Ey, 0.2)
    want = e / np.mean(1.0 / (lam + 2 * mu))
    np.testing.assert_allclose(sig[..., 1, 1], want, rtol=1e-9)
    np.testing.assert_allclose(eps_star[..., 0, 0], 0.0, atol=1e-10)


@pytest.mark.parametrize("shape", [(9, 9), (7, 11)])
def test_laminate_shear(shape):
    """Laminate in y under shear eps_bar_xy = g: sigma_xy uniform
    = 2 g / mean(1/mu), sigma_yy = 0."""
    ny, nx = shape
    rng = np.random.default_rng(11)
    Ey = rng.uniform(0.5, 1.5, ny)
    E = Ey[:, None] * np.ones((1, nx))
    g = 0.1
    _, sig, _ = solve(E, np.zeros(shape), np.array([[0.0, g], [g, 0.0]]), "none")
    _, mu = cm.lame(Ey, 0.2)
    np.testing.assert_allclose(sig[..., 0, 1], 2 * g / np.mean(1.0 / mu), rtol=1e-9)
    np.testing.assert_allclose(sig[..., 1, 1], 0.0, atol=1e-10)


def _sym_grad_basis(ny, nx):
    n = ny * nx
    basis = np.empty((2 * n, ny, nx, 2, 2))
    for k in range(2 * n):
        u = np.zeros(2 * n)
        u[k] = 1.0
        basis[k] = sp.symmetric_gradient(u.reshape(2, ny, nx).transpose(1, 2, 0))
    return basis


@pytest.mark.parametrize("eps_bar", [np.array([[0.05, 0.12], [0.12, 0.3]]),
                                     np.array([[-0.2, 0.05], [0.05, 0.1]])])
def test_spectral_split_energy_minimiser(eps_bar):
    """The Galerkin solution minimises sum_x psi(eps_bar + sym grad u) over
    periodic trig-polynomial displacements.  Brute force on a 5x5 grid with a
    quasi-Newton minimiser, compared stress field by stress field."""
    ny = nx = 5
    rng = np.random.default_rng(12)
    E = rng.uniform(0.5, 1.5, (ny, nx))
    phi = rng.uniform(0.0, 0.8, (ny, nx))
    lam, mu = cm.lame(E, 0.2)
    basis = _sym_grad_basis(ny, nx)

    def energy(u):
        eps = eps_bar + np.einsum("k,kyxij->yxij", u, basis)
        f = np.sum(cm.energy_density(eps, phi, lam, mu, "spectral"))
        sig = cm.stress(eps, phi, lam, mu, "spectral")
        return f, np.einsum("yxij,kyxij->k", sig, basis)

    res = minimize(energy, np.zeros(2 * ny * nx), jac=True, method="L-BFGS-B",
                   options={"gtol": 1e-13, "ftol": 1e-16, "maxiter": 20000, "maxcor": 50})
    eps_bf = eps_bar + np.einsum("k,kyxij->yxij", res.x, basis)
    sig_bf = cm.stress(eps_bf, phi, lam, mu, "spectral")
    _, sig, _ = solve(E, phi, eps_bar, "spectral")
    np.testing.assert_allclose(sig, sig_bf, atol=2e-6 * np.abs(sig).max())


@pytest.mark.parametrize("split", ["none", "spectral"])
def test_homogeneity_in_load(split):
    """Degree-1 homogeneity of the stress (Sec. 3.2.3) carries to the
    solution: eps*(g eps_bar) = g eps*(eps_bar) for g > 0."""
    rng = np.random.default_rng(13)
    E = rng.uniform(0.6, 1.4, (8, 8))
    phi = rng.uniform(0, 0.5, (8, 8))
    eb = np.array([[0.1, -0.05], [-0.05, 0.2]])
    e1, _, _ = solve(E, phi, eb, split)
    e2, _, _ = solve(E, phi, 2.5 * eb, split)
    np.testing.assert_allclose(e2, 2.5 * e1, atol=1e-8)


@pytest.mark.parametrize("split", ["none", "spectral"])
def test_rotation_and_translation_equivariance(split):
    """Rotating the microstructure by 90 degrees (x -> y) and swapping the
    load components rotates the solution; a periodic shift shifts it."""
    rng = np.random.default_rng(14)
    E = rng.uniform(0.6, 1.4, (8, 6))
    phi = rng.uniform(0, 0.5, (8, 6))
    eb = np.array([[0.05, 0.08], [0.08, 0.2]])
    _, sig, _ = solve(E, phi, eb, split)
    # 90-degree rotation: new field f'(y', x') = f(x', y') with axes swapped,
    # i.e. transpose of the grid plus swap of tensor indices x<->y
    Et, pt = E.T.copy(), phi.T.copy()
    P = np.array([[0.0, 1.0], [1.0, 0.0]])
    ebt = P @ eb @ P.T
    _, sigt, _ = solve(Et, pt, ebt, split)
    back = np.einsum("ij,yxjk,lk->xyil", P, sigt, P)
    np.testing.assert_allclose(back, sig, atol=1e-8)
    _, sigs, _ = solve(np.roll(E, (3, 2), (0, 1)), np.roll(phi, (3, 2), (0, 1)), eb, split)
    np.testing.assert_allclose(np.roll(sig, (3, 2), (0, 1)), sigs, atol=1e-8)


def test_effective_stiffness_symmetric():
    """For the linear (isotropic) model the effective stiffness
    eps_a : sigma_bar(eps_b) is symmetric."""
    rng = np.random.default_rng(15)
    E = rng.uniform(0.5, 1.5, (10, 10))
    phi = rng.uniform(0, 0.6, (10, 10))
    loads = [np.diag([1.0, 0.0]), np.diag([0.0, 1.0]), np.array([[0.0, 1.0], [1.0, 0.0]])]
    sb = [solve(E, phi, L, "none")[1].mean(axis=(0, 1)) for L in loads]
    M = np.array([[np.sum(loads[a] * sb[b]) for b in range(3)] for a in range(3)])
    np.testing.assert_allclose(M, M.T, rtol=1e-8)
    assert np.all(np.linalg.eigvalsh(M) > 0)


def test_residual_small_after_solve():
    rng = np.random.default_rng(16)
    E = rng.uniform(0.5, 1.5, (12, 12))
    phi = rng.uniform(0, 0.9, (12, 12))
    eb = np.array([[0.0, 0.03], [0.03, 0.3]])
    eps_star, sig, info = solve(E, phi, eb, "spectral", tol=1e-10)
    R = sp.project(sig)
    assert np.sqrt(np.sum(R * R)) <= info["target"] * (1 + 1e-12)
    # eps* stays compatible and zero mean
    np.testing.assert_allclose(sp.project(eps_star), eps_star, atol=1e-12)


@pytest.mark.parametrize("shape", [(8, 8), (16, 6)])
@pytest.mark.parametrize("split", ["none", "spectral"])
def test_laminate_uniaxial_even_grid_nyquist_free(shape, split):
    """On an even grid the layer strain e_yy(y) has a Nyquist component.
    With the Nyquist modes of the strain fluctuation unconstrained
    (nyquist='free') the laminate is exact again: sigma_yy uniform,
    e / mean(1/M); with them suppressed (nyquist='zero') it is not (here
    the layers alternate pixel by pixel, the pure Nyquist pattern)."""
    ny, nx = shape
    Ey = np.where(np.arange(ny) % 2 == 0, 1.0, 0.1)
    E = Ey[:, None] * np.ones((1, nx))
    phi = np.zeros(shape)
    e = 0.2
    lam, mu = cm.lame(E, 0.2)
    lam1, mu1 = cm.lame(Ey, 0.2)
    want = e / np.mean(1.0 / (lam1 + 2 * mu1))
    out = {}
    for nyq in ("free", "zero"):
        eps_star, info = mech.solve(np.zeros(shape + (2, 2)), np.diag([0.0, e]), phi, lam, mu, split,
                                    tol_rel=1e-11, max_newton=50, nyquist=nyq)
        assert info["converged"], info
        out[nyq] = cm.stress(np.diag([0.0, e]) + eps_star, phi, lam, mu, split, 0.0)
    np.testing.assert_allclose(out["free"][..., 1, 1], want, rtol=1e-9)
    assert np.abs(out["zero"][..., 1, 1].mean() / want - 1) > 0.5
