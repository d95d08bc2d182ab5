"""Pins for oracle.constitutive against the paper's worked examples
(Sec. 4.2.1), closed forms (Sec. 3.3, 4.2.2) and calculus identities."""

import json
import os

import numpy as np
import pytest

from oracle import constitutive as cm

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "strength_closed_forms.json")
SQ2 = np.sqrt(2.0)


def rot(theta):
    c, s = np.cos(theta), np.sin(theta)
    return np.array([[c, -s], [s, c]])


def principal(e1, e2, theta):
    R = rot(theta)
    return R @ np.diag([e1, e2]) @ R.T


@pytest.mark.parametrize("a,b,theta", [(0.3, 0.0, 0.0), (0.3, 0.2, 0.7), (1.0, 2.5, -1.1),
                                       (0.01, 0.05, 2.0)])
def test_worked_example_driving_forces(a, b, theta):
    """Sec. 4.2.1: principal strains (a, -a-b): psi0+ is
    1/2 lam b^2 + 2 mu (a^2 + ab + b^2/2) for the isotropic model and mu a^2
    for the strain-spectral split, in any frame."""
    lam, mu = cm.lame(1.7, 0.23)
    eps = principal(a, -a - b, theta)
    iso, _ = cm.psi0(eps, lam, mu, "none")
    spec, _ = cm.psi0(eps, lam, mu, "spectral")
    assert iso == pytest.approx(0.5 * lam * b * b + 2 * mu * (a * a + a * b + b * b / 2), rel=1e-12)
    assert spec == pytest.approx(mu * a * a, rel=1e-12)


@pytest.mark.parametrize("b", [0.1, 1.0, 3.0])
def test_worked_example_contact_compression(b):
    """Sec. 4.2.1: at phi = 1, eps = diag(0, -b): isotropic sigma = 0,
    strain-spectral sigma = diag(-lam b, -(lam + 2 mu) b)."""
    lam, mu = cm.lame(2.3, 0.3)
    eps = np.diag([0.0, -b])
    np.testing.assert_allclose(cm.stress(eps, 1.0, lam, mu, "none"), 0.0, atol=1e-15)
    np.testing.assert_allclose(cm.stress(eps, 1.0, lam, mu, "spectral"),
                               np.diag([-lam * b, -(lam + 2 * mu) * b]), rtol=1e-12, atol=1e-14)


@pytest.mark.parametrize("b", [0.1, 1.0, 3.0])
def test_worked_example_contact_mixed(b):
    """Sec. 4.2.1: at phi = 1, eps = [[0, b], [b, 2b]]: strain-spectral
    sigma = mu/sqrt2 [[-b, (sqrt2-1) b], [(sqrt2-1) b, (2 sqrt2 - 3) b]];
    isotropic sigma = 0."""
    lam, mu = cm.lame(1.3, 0.2)
    eps = np.array([[0.0, b], [b, 2 * b]])
    want = mu / SQ2 * np.array([[-b, (SQ2 - 1) * b], [(SQ2 - 1) * b, (2 * SQ2 - 3) * b]])
    np.testing.assert_allclose(cm.stress(eps, 1.0, lam, mu, "spectral"), want, rtol=1e-12, atol=1e-14)
    np.testing.assert_allclose(cm.stress(eps, 1.0, lam, mu, "none"), 0.0, atol=1e-15)


@pytest.mark.parametrize("b", [0.1, 1.0, 3.0])
def test_worked_example_voldev_contact(b):
    """Sec. 4.2.1, volumetric-deviatoric split at phi = 1: eps = diag(0, -b)
    gives sigma = (lam + 2 mu/3) diag(-b, -b); eps = [[0, b], [b, 2b]]
    (tension along y) gives sigma = 0."""
    lam, mu = cm.lame(2.3, 0.3)
    np.testing.assert_allclose(cm.stress(np.diag([0.0, -b]), 1.0, lam, mu, "voldev"),
                               (lam + 2 * mu / 3) * np.diag([-b, -b]), rtol=1e-12, atol=1e-14)
    np.testing.assert_allclose(cm.stress(np.array([[0.0, b], [b, 2 * b]]), 1.0, lam, mu, "voldev"), 0.0,
                               atol=1e-14)


@pytest.mark.parametrize("a,b,theta", [(0.3, 0.0, 0.0), (0.3, 0.2, 0.7), (1.0, 2.5, -1.1),
                                       (0.01, 0.05, 2.0)])
def test_worked_example_voldev_driving_force(a, b, theta):
    """Sec. 4.2.1, principal strains (a, -a-b): the volumetric-deviatoric
    driving force equals the isotropic one for pure shear (b = 0) and lies
    between the isotropic and the strain-spectral ones,
    iso >= vol.-dev. > spectral.  With the plane-strain deviator (out-of-plane
    strain zero) its value is 2 mu (a^2 + ab + b^2/3)."""
    lam, mu = cm.lame(1.7, 0.23)
    eps = principal(a, -a - b, theta)
    iso = cm.psi0(eps, lam, mu, "none")[0]
    vd = cm.psi0(eps, lam, mu, "voldev")[0]
    spec = cm.psi0(eps, lam, mu, "spectral")[0]
    if b == 0.0:
        assert vd == pytest.approx(iso, rel=1e-12)
    assert iso >= vd - 1e-15 and vd > spec
    assert vd == pytest.approx(2 * mu * (a * a + a * b + b * b / 3), rel=1e-12)


def test_degradation_properties():
    """Sec. 2.1: h(0) = 1, h(1) = 0, h'(1) = 0."""
    assert cm.degradation(0.0) == 1.0 and cm.degradation(1.0) == 0.0
    d = 1e-6
    assert abs((cm.degradation(1 + d) - cm.degradation(1 - d)) / (2 * d)) < 1e-9


def _rand_eps(rng, n):
    a = rng.standard_normal((n, 2, 2))
    return 0.5 * (a + np.swapaxes(a, -1, -2))


def test_split_sums_to_isotropic():
    rng = np.random.default_rng(5)
    eps = _rand_eps(rng, 200)
    lam, mu = cm.lame(rng.uniform(0.5, 2, 200), 0.2)
    sp_, sm = cm.sigma0(eps, lam, mu, "spectral")
    si, _ = cm.sigma0(eps, lam, mu, "none")
    np.testing.assert_allclose(sp_ + sm, si, atol=1e-13)
    pp, pm = cm.psi0(eps, lam, mu, "spectral")
    pi, _ = cm.psi0(eps, lam, mu, "none")
    np.testing.assert_allclose(pp + pm, pi, atol=1e-13)
    assert np.all(pp >= 0) and np.all(pm >= 0)
    # Sec. 4.2.1: at phi = 0 every model gives the isotropic response
    sp_, sm = cm.sigma0(eps, lam, mu, "voldev")
    np.testing.assert_allclose(sp_ + sm, si, atol=1e-13)
    pp, pm = cm.psi0(eps, lam, mu, "voldev")
    np.testing.assert_allclose(pp + pm, pi, atol=1e-13)
    assert np.all(pp >= 0) and np.all(pm >= 0)


@pytest.mark.parametrize("split", ["none", "spectral", "voldev"])
def test_homogeneity(split):
    """Sec. 3.2.3: psi0+ is degree-2 and the stress degree-1 homogeneous."""
    rng = np.random.default_rng(6)
    eps = _rand_eps(rng, 100)
    lam, mu = cm.lame(1.0, 0.2)
    phi = rng.uniform(0, 1, 100)
    for g in (0.3, 2.0, 7.5):
        np.testing.assert_allclose(cm.psi0(g * eps, lam, mu, split)[0],
                                   g * g * cm.psi0(eps, lam, mu, split)[0], rtol=1e-11, atol=1e-14)
        np.testing.assert_allclose(cm.stress(g * eps, phi, lam, mu, split),
                                   g * cm.stress(eps, phi, lam, mu, split), rtol=1e-11, atol=1e-14)


@pytest.mark.parametrize("split", ["none", "spectral", "voldev"])
def test_stress_is_energy_gradient(split):
    """sigma = d psi / d eps (Sec. 2.1), by central differences."""
    rng = np.random.default_rng(7)
    eps = _rand_eps(rng, 64)
    phi = rng.uniform(0, 1, 64)
    lam, mu = cm.lame(rng.uniform(0.5, 2, 64), 0.25)
    sig = cm.stress(eps, phi, lam, mu, split, k_res=1e-3)
    h = 1e-6
    for _ in range(4):
        d = _rand_eps(rng, 64)
        fp = cm.energy_density(eps + h * d, phi, lam, mu, split, 1e-3)
        fm = cm.energy_density(eps - h * d, phi, lam, mu, split, 1e-3)
        np.testing.assert_allclose((fp - fm) / (2 * h), cm.ddot(sig, d), rtol=1e-6, atol=1e-8)


@pytest.mark.parametrize("split", ["none", "spectral", "voldev"])
def test_tangent_is_stress_derivative(split):
    """C : d equals the central difference of sigma (Sec. 3.1.1), away from
    the kinks of the ramps."""
    rng = np.random.default_rng(8)
    eps = _rand_eps(rng, 300)
    w, _ = np.linalg.eigh(eps)
    ok = (np.min(np.abs(w), axis=-1) > 0.05) & (np.abs(w[:, 0] - w[:, 1]) > 0.05) & \
         (np.abs(w.sum(-1)) > 0.05)
    eps = eps[ok]
    n = len(eps)
    phi = rng.uniform(0, 1, n)
    lam, mu = cm.lame(rng.uniform(0.5, 2, n), 0.2)
    h = 1e-7
    for _ in range(4):
        d = _rand_eps(rng, n)
        fd = (cm.stress(eps + h * d, phi, lam, mu, split) - cm.stress(eps - h * d, phi, lam, mu, split)) / (2 * h)
        np.testing.assert_allclose(cm.tangent_action(eps, d, phi, lam, mu, split), fd, rtol=1e-5, atol=1e-6)


def test_tangent_repeated_eigenvalues_limit():
    """At eps = m I the spectral tangent is the isotropic one (m > 0) or 0
    (m < 0) for the degraded part; the repeated-eigenvalue limit is used."""
    lam, mu = cm.lame(1.0, 0.2)
    rng = np.random.default_rng(9)
    d = _rand_eps(rng, 10)
    for m, want_plus in ((0.4, 1.0), (-0.4, 0.0)):
        eps = np.broadcast_to(m * np.eye(2), (10, 2, 2))
        iso = cm.dsigma0(eps, d, lam, mu, "none", +1)
        np.testing.assert_allclose(cm.dsigma0(eps, d, lam, mu, "spectral", +1), want_plus * iso, atol=1e-13)
        np.testing.assert_allclose(cm.dsigma0(eps, d, lam, mu, "spectral", -1), (1 - want_plus) * iso, atol=1e-13)


def test_strength_closed_forms_golden():
    """Sec. 3.3 and 4.2.2: the homogeneous AT1 strength values printed in
    the paper follow from the oracle's Lame constants and energy split."""
    g = json.load(open(GOLDEN))
    u = g["uniaxial_strain_AT1"]
    lam, mu = cm.lame(u["E0"], u["nu"])
    # onset where 2 psi0+ (eps_M) = 3 G_c / (8 l) for uniaxial strain
    e = np.sqrt(3 * u["gc"] / (8 * u["ell"] * (lam + 2 * mu)))
    eps = np.diag([0.0, e])
    psi = cm.psi0(eps, lam, mu, "spectral")[0]
    assert 2 * psi == pytest.approx(3 * u["gc"] / (8 * u["ell"]), rel=1e-12)
    assert e == pytest.approx(u["eps_M"], abs=5e-7)
    sig = cm.stress(eps, 0.0, lam, mu, "spectral")
    assert sig[1, 1] == pytest.approx(u["sigma_M"], abs=5e-3)
    s = g["pure_shear_AT1_spectral"]
    lam, mu = cm.lame(s["E0"], s["nu"])
    # spectral driving force of pure shear eps_12 = g is mu g^2 ... per
    # eigenvalue +-g: psi0+ = mu g^2; onset 2 psi0+ = 3 G_c / (8 l)
    gam = np.sqrt(3 * s["gc"] / (16 * s["ell"] * mu))
    eps = np.array([[0.0, gam], [gam, 0.0]])
    assert 2 * cm.psi0(eps, lam, mu, "spectral")[0] == pytest.approx(3 * s["gc"] / (8 * s["ell"]), rel=1e-12)
    assert gam == pytest.approx(s["eps12_M"], abs=5e-7)
    assert cm.stress(eps, 0.0, lam, mu, "spectral")[0, 1] == pytest.approx(s["sigma12_M"], abs=5e-3)
