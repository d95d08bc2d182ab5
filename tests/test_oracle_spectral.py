"""Pins for oracle.spectral: transform convention, compatibility projection,
collocation Laplacian, displacement recovery (Sec. 3.1, 3.1.1, 3.1.2)."""

import numpy as np
import pytest

from oracle import spectral as sp

GRIDS = [(4, 4), (5, 7), (6, 6), (8, 16), (5, 4)]


def brute_dft(f):
    """The paper's forward transform written out (Sec. 3.1), with the 1/|N|
    factor, on the index set in grid order."""
    ny, nx = f.shape
    out = np.zeros((ny, nx), dtype=complex)
    for ky in range(ny):
        for kx in range(nx):
            s = 0.0
            for jy in range(ny):
                for jx in range(nx):
                    s += f[jy, jx] * np.exp(-2j * np.pi * (kx * jx / nx + ky * jy / ny))
            out[ky, kx] = s / (nx * ny)
    return out


@pytest.mark.parametrize("shape", GRIDS)
def test_fft_matches_brute_force_dft(shape):
    rng = np.random.default_rng(1)
    f = rng.standard_normal(shape)
    np.testing.assert_allclose(sp.fft_field(f) / f.size, brute_dft(f), atol=1e-13)
    np.testing.assert_allclose(sp.ifft_field(sp.fft_field(f)), f, atol=1e-13)


def _rand_sym(rng, shape):
    a = rng.standard_normal(shape + (2, 2))
    return 0.5 * (a + np.swapaxes(a, -1, -2))


def ddot_sum(a, b):
    return float(np.sum(a * b))


@pytest.mark.parametrize("shape", GRIDS)
def test_projection_idempotent_selfadjoint(shape):
    rng = np.random.default_rng(2)
    a, b = _rand_sym(rng, shape), _rand_sym(rng, shape)
    ga = sp.project(a)
    np.testing.assert_allclose(sp.project(ga), ga, atol=1e-12)
    assert abs(ddot_sum(ga, b) - ddot_sum(a, sp.project(b))) < 1e-10
    # symmetric output, zero mean
    np.testing.assert_allclose(ga, np.swapaxes(ga, -1, -2), atol=1e-13)
    np.testing.assert_allclose(ga.mean(axis=(0, 1)), 0.0, atol=1e-13)
    # constants are removed
    c = np.broadcast_to(np.array([[1.0, 0.3], [0.3, -2.0]]), shape + (2, 2)).copy()
    np.testing.assert_allclose(sp.project(c), 0.0, atol=1e-13)


@pytest.mark.parametrize("shape", GRIDS)
def test_projection_keeps_gradients(shape):
    rng = np.random.default_rng(3)
    u = rng.standard_normal(shape + (2,))
    eps = sp.symmetric_gradient(u)
    np.testing.assert_allclose(sp.project(eps), eps, atol=1e-12)


def _dense_range_projector(ny, nx):
    """Orthogonal projector (in the A:B metric) onto the range of the
    discrete symmetric gradient, from dense linear algebra.  Coordinates per
    pixel: (e_xx, sqrt2 e_xy, e_yy), which turns A:B into the dot product."""
    n = ny * nx
    cols = []
    for k in range(2 * n):
        u = np.zeros(2 * n)
        u[k] = 1.0
        e = sp.symmetric_gradient(u.reshape(2, ny, nx).transpose(1, 2, 0))
        cols.append(np.concatenate([e[..., 0, 0].ravel(), np.sqrt(2) * e[..., 0, 1].ravel(),
                                    e[..., 1, 1].ravel()]))
    B = np.array(cols).T
    U, s, _ = np.linalg.svd(B, full_matrices=False)
    rank = int(np.sum(s > 1e-9 * s.max()))
    Ur = U[:, :rank]
    return Ur @ Ur.T


@pytest.mark.parametrize("shape", [(4, 4), (5, 5), (4, 6), (5, 6), (3, 5)])
def test_projection_equals_dense_projector(shape):
    ny, nx = shape
    n = ny * nx
    P = _dense_range_projector(ny, nx)
    G = np.zeros((3 * n, 3 * n))
    for k in range(3 * n):
        v = np.zeros(3 * n)
        v[k] = 1.0
        a = np.zeros((ny, nx, 2, 2))
        a[..., 0, 0] = v[:n].reshape(ny, nx)
        a[..., 0, 1] = a[..., 1, 0] = v[n:2 * n].reshape(ny, nx) / np.sqrt(2)
        a[..., 1, 1] = v[2 * n:].reshape(ny, nx)
        g = sp.project(a)
        G[:, k] = np.concatenate([g[..., 0, 0].ravel(), np.sqrt(2) * g[..., 0, 1].ravel(),
                                  g[..., 1, 1].ravel()])
    np.testing.assert_allclose(G, P, atol=1e-10)


@pytest.mark.parametrize("shape", [(8, 8), (7, 9), (6, 10)])
def test_laplacian_plane_waves(shape):
    ny, nx = shape
    y, x = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
    for ky in range(ny // 2 + 1):
        for kx in range(nx // 2 + 1):
            f = np.cos(2 * np.pi * (kx * x / nx + ky * y / ny))
            lam = (2 * np.pi * kx / nx) ** 2 + (2 * np.pi * ky / ny) ** 2
            np.testing.assert_allclose(sp.laplacian(f), -lam * f, atol=1e-11)


def test_laplacian_nyquist_checkerboard_kept():
    f = np.fromfunction(lambda y, x: (-1.0) ** (x + y), (8, 8))
    np.testing.assert_allclose(sp.laplacian(f), -2 * np.pi ** 2 * f, atol=1e-11)


def _plane_wave_displacement(ny, nx, kx, ky, ax, ay, phase):
    """u = (ax sin(t), ay cos(t)), t = 2 pi (kx x / nx + ky y / ny) + phase,
    and its symmetric gradient written out by hand from the continuum
    derivatives d/dx t = 2 pi kx / nx, d/dy t = 2 pi ky / ny (exact on the
    grid for a wave below the Nyquist index).  Returns u (ny, nx, 2) and eps
    (ny, nx, 2, 2), vector index order (x, y)."""
    y, x = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
    t = 2 * np.pi * (kx * x / nx + ky * y / ny) + phase
    gx, gy = 2 * np.pi * kx / nx, 2 * np.pi * ky / ny
    u = np.stack([ax * np.sin(t), ay * np.cos(t)], axis=-1)
    dux_dx, dux_dy = ax * gx * np.cos(t), ax * gy * np.cos(t)
    duy_dx, duy_dy = -ay * gx * np.sin(t), -ay * gy * np.sin(t)
    eps = np.zeros((ny, nx, 2, 2))
    eps[..., 0, 0] = dux_dx
    eps[..., 1, 1] = duy_dy
    eps[..., 0, 1] = eps[..., 1, 0] = 0.5 * (dux_dy + duy_dx)
    return u, eps


WAVES = [(1, 0, 1.0, 0.0, 0.0), (0, 1, 0.0, 1.0, 0.0), (0, 1, 1.0, 0.0, 0.0), (1, 0, 0.0, 1.0, 0.0),
         (2, 3, 0.7, -1.3, 0.4), (-3, 1, -0.5, 0.9, 1.1), (1, -2, 1.2, 0.3, -0.6)]


@pytest.mark.parametrize("shape", [(8, 8), (9, 7), (12, 10), (16, 16)])
@pytest.mark.parametrize("wave", WAVES)
def test_symmetric_gradient_plane_waves(shape, wave):
    """sym(grad u) of a single plane-wave displacement equals the hand-written
    derivative (Sec. 3.1.1: compatible strains are symmetric gradients).
    Covers pure extension in x and y, pure shear (eps_xy = d u_x / dy / 2),
    and oblique waves with both components."""
    ny, nx = shape
    u, eps = _plane_wave_displacement(ny, nx, *wave)
    np.testing.assert_allclose(sp.symmetric_gradient(u), eps, atol=1e-12)


@pytest.mark.parametrize("shape", [(8, 8), (9, 7), (12, 10), (16, 16)])
@pytest.mark.parametrize("wave", WAVES)
def test_displacement_from_strain_plane_waves(shape, wave):
    """The displacement recovered from a plane-wave strain is the plane-wave
    displacement itself (zero mean), e.g. eps_xx = (2 pi / N) cos(2 pi x / N)
    gives u = (sin(2 pi x / N), 0): checked against the hand-written wave, not
    against ``symmetric_gradient``."""
    ny, nx = shape
    u, eps = _plane_wave_displacement(ny, nx, *wave)
    np.testing.assert_allclose(sp.displacement_from_strain(eps), u, atol=1e-12)


def test_displacement_from_strain_superposition_and_mean():
    """Linear in the strain, and a constant offset of u is not recoverable:
    the result is the zero-mean fluctuation of the sum of several waves."""
    ny, nx = 10, 12
    us, es = zip(*[_plane_wave_displacement(ny, nx, *w) for w in WAVES[4:]])
    u = sum(us) + np.array([0.3, -0.2])
    eps = sum(es)
    np.testing.assert_allclose(sp.displacement_from_strain(eps), u - u.mean(axis=(0, 1)), atol=1e-12)


def test_symmetric_gradient_of_nyquist_waves_vanishes():
    """Even grids: cos(pi x) and cos(pi y) sampled on the grid are (-1)^x,
    (-1)^y, whose continuum derivative -pi sin(pi x) vanishes at every grid
    point; the gradient (Nyquist component zero) gives zero strain, and the
    displacement recovered from zero strain is zero."""
    y, x = np.meshgrid(np.arange(8), np.arange(8), indexing="ij")
    for wave in ((-1.0) ** x, (-1.0) ** y, (-1.0) ** (x + y)):
        for c in range(2):
            u = np.zeros((8, 8, 2))
            u[..., c] = wave
            np.testing.assert_allclose(sp.symmetric_gradient(u), 0.0, atol=1e-13)


@pytest.mark.parametrize("shape", [(8, 8), (9, 7), (6, 10)])
def test_displacement_recovery_roundtrip(shape):
    rng = np.random.default_rng(4)
    u = rng.standard_normal(shape + (2,))
    eps = sp.symmetric_gradient(u)
    u2 = sp.displacement_from_strain(eps)
    np.testing.assert_allclose(sp.symmetric_gradient(u2), eps, atol=1e-11)
    np.testing.assert_allclose(u2.mean(axis=(0, 1)), 0.0, atol=1e-12)


def _dense_projector_with_nyquist(ny, nx):
    """Orthogonal projector onto the symmetric gradients plus every real
    tensor field supported on the modes with a Nyquist index (same
    coordinates as _dense_range_projector)."""
    n = ny * nx
    P = _dense_range_projector(ny, nx)
    U0 = np.linalg.svd(P)[0][:, :int(round(np.trace(P)))]
    extra = []
    yy, xx = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
    mask = sp.nyquist_modes(ny, nx)
    for ky, kx in zip(*np.nonzero(mask)):
        ph = 2 * np.pi * (sp.signed_indices(nx)[kx] * xx / nx + sp.signed_indices(ny)[ky] * yy / ny)
        for wave in (np.cos(ph), np.sin(ph)):
            for c in range(3):
                v = np.zeros(3 * n)
                v[c * n:(c + 1) * n] = wave.ravel()
                extra.append(v)
    B = np.concatenate([U0, np.array(extra).T], axis=1) if extra else U0
    U, s, _ = np.linalg.svd(B, full_matrices=False)
    rank = int(np.sum(s > 1e-9 * s.max()))
    return U[:, :rank] @ U[:, :rank].T


@pytest.mark.parametrize("shape", [(4, 4), (4, 6), (5, 6), (3, 5)])
def test_projection_nyquist_free_equals_dense_projector(shape):
    """nyquist='free' (even grids): G is the orthogonal projector onto the
    compatible fields plus all fields on the Nyquist modes; on odd grids it
    is the same operator as nyquist='zero'."""
    ny, nx = shape
    n = ny * nx
    P = _dense_projector_with_nyquist(ny, nx)
    G = np.zeros((3 * n, 3 * n))
    for k in range(3 * n):
        v = np.zeros(3 * n)
        v[k] = 1.0
        a = np.zeros((ny, nx, 2, 2))
        a[..., 0, 0] = v[:n].reshape(ny, nx)
        a[..., 0, 1] = a[..., 1, 0] = v[n:2 * n].reshape(ny, nx) / np.sqrt(2)
        a[..., 1, 1] = v[2 * n:].reshape(ny, nx)
        g = sp.project(a, "free")
        G[:, k] = np.concatenate([g[..., 0, 0].ravel(), np.sqrt(2) * g[..., 0, 1].ravel(),
                                  g[..., 1, 1].ravel()])
    np.testing.assert_allclose(G, P, atol=1e-10)
    if ny % 2 and nx % 2:
        rng = np.random.default_rng(5)
        a = _rand_sym(rng, shape)
        np.testing.assert_allclose(sp.project(a, "free"), sp.project(a, "zero"), atol=1e-14)
