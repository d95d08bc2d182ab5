"""Seeded input generators: the two-phase microstructure and the initial
phase fields of Sec. 3.4 and 4.1.1 (host-side inputs, no solver
arithmetic)."""

import numpy as np
import pytest

import spff_inputs as si


def test_two_phase_structure():
    """Two bulk phases E = 1 -+ a (modulus ratio 15 at a = 0.875) in about
    equal fractions, separated by diffuse interfaces about two pixels wide;
    the structure is set by the seed."""
    n, a = 128, 0.875
    E = si.two_phase(n, 32.0, a, seed=11)
    assert E.dtype == np.float32 and E.shape == (n, n)
    xi = (E.astype(np.float64) - 1.0) / a
    assert xi.min() >= -1.0 - 1e-6 and xi.max() <= 1.0 + 1e-6
    bulk = np.abs(xi) > 0.9
    assert bulk.mean() > 0.75
    assert 0.3 < (xi > 0).mean() < 0.7
    assert (1 + a) / (1 - a) == pytest.approx(15.0)
    assert np.isclose(E.max(), 1 + a, atol=0.02) and np.isclose(E.min(), 1 - a, atol=0.02)
    np.testing.assert_array_equal(E, si.two_phase(n, 32.0, a, seed=11))
    assert not np.array_equal(E, si.two_phase(n, 32.0, a, seed=12))
    # l_cut sets the feature size: a smaller cutoff wavelength, more interfaces
    fine = si.two_phase(n, 12.0, a, seed=11)
    assert (np.abs((fine - 1) / a) < 0.5).mean() > 2 * (np.abs(xi) < 0.5).mean()


def test_allen_cahn_smoothing_relaxes_to_the_equilibrium_interface():
    """The smoothing iteration is explicit Allen-Cahn with unit coefficients,
    xi_t = xi - xi^3 + lap xi, whose 1-D equilibrium interface is
    tanh(x / sqrt 2): a periodic stripe with two such interfaces barely
    moves in 21 steps, and a sharp sgn stripe relaxes to within a few
    percent of it (from 0.6 away)."""
    n = 64
    x = np.arange(n) - n / 2

    def smooth(prof):
        out = np.broadcast_to(prof[None, :], (8, n)).copy()
        for _ in range(21):
            nb = np.roll(out, 1, 0) + np.roll(out, -1, 0) + np.roll(out, 1, 1) + np.roll(out, -1, 1)
            out = out - 0.1 * ((out ** 3 - out) + (4.0 * out - nb))
        return out[0]

    eq = np.tanh((np.abs(x) - 16.5) / np.sqrt(2.0))
    assert np.abs(smooth(eq) - eq).max() < 0.05
    step = np.sign(np.abs(x) - 16.5)
    assert np.abs(step - eq).max() > 0.5
    assert np.abs(smooth(step) - eq).max() < 0.06
    # the generator runs the same iteration: its interfaces have the same width
    E = si.two_phase(256, 64.0, 1.0, seed=3)
    xi = E.astype(np.float64) - 1.0
    frac = (np.abs(xi) < np.tanh(1.0 / np.sqrt(2.0))).mean()   # |dist| < 1 px
    per = (np.abs(np.diff(np.sign(xi), axis=1)) > 0).mean()     # interface crossings per pixel
    assert 1.0 < frac / per < 3.5


def test_initial_crack_and_void_fields():
    """Sec. 4.1.1: the crack is the AT1 profile (1 - |r|/(2 l))^2 around a
    segment of y = 0 (centred: |x| <= L/2; the literal printed form: x <= L/2
    on a grid centred at the origin); the void is the same profile around
    the origin."""
    n, ell = 64, 3.0
    phi = si.edge_crack(n, n, ell, 20.0)
    assert phi[n // 2, 0] == 1.0 and phi[n // 2, n // 2 + 10] == 1.0 and phi[n // 2, n // 2 + 17] == 0.0
    assert phi[n // 2 + 3, 5] == pytest.approx(0.25)
    c = si.centre_crack(n, n, ell, 20.0)
    assert c[n // 2, n // 2 - 10] == 1.0 and c[n // 2, n // 2 + 10] == 1.0 and c[n // 2, 0] == 0.0
    assert c[n // 2, n // 2 + 13] == pytest.approx(0.25) and c[n // 2, n // 2 - 13] == pytest.approx(0.25)
    np.testing.assert_array_equal(c[:, n // 2 + 1:n // 2 + 31], c[:, n // 2 - 1:n // 2 - 31:-1])
    v = si.round_void(n, n, ell)
    assert v[n // 2, n // 2] == 1.0 and v.sum() > 0
    assert v[n // 2 + 3, n // 2] == pytest.approx(0.25) and v[n // 2, n // 2 - 3] == pytest.approx(0.25)
    assert v[n // 2 + 6, n // 2] == 0.0 and np.count_nonzero(v) < 0.05 * n * n
