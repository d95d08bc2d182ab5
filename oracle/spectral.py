"""Grid, wavevectors, compatibility projection and collocation Laplacian.

Oracle (test infrastructure only).  Follows Sec. 3.1 (periodic grid, discrete
Fourier transform), Sec. 3.1.1 (projection onto compatible strain fields) and
Sec. 3.1.2 (collocation Laplacian).

Conventions
  * Fields are sampled on an ny x nx periodic grid with unit spacing; arrays
    are indexed [y, x].
  * Forward transform = ``numpy.fft.fft2`` (no normalisation), inverse =
    ``numpy.fft.ifft2`` (1/(nx ny)).  The paper puts 1/|N| on the forward
    transform (Sec. 3.1); the placement is a convention with no effect on any
    operator used here.
  * Angular wavevector xi = 2 pi q with q = k / L, k the signed index in
    numpy's fftfreq order.

Reading of the paper for even grids: the paper uses odd N only (trapezoidal
exactness, Sec. 3.1).  For even N the Nyquist index k = N/2 has no signed
partner, and a real field's gradient there is ambiguous.  The gradient (and
therefore the compatibility projection) uses xi with any component at
|k| = N/2 set to zero; the Laplacian keeps the true |xi|^2 at Nyquist so the
phase-field operator stays positive definite on checkerboard modes.
"""

import numpy as np


def signed_indices(n):
    """Signed integer wave indices k of an n-point DFT, fftfreq order."""
    return np.rint(np.fft.fftfreq(n) * n).astype(np.int64)


def wavevectors(ny, nx):
    """Angular wavevectors (xi_y, xi_x), each of shape (ny, nx), unit spacing.

    Sec. 3.1: q^k = (k_x / L_x, k_y / L_y); xi = 2 pi q.
    """
    ky = signed_indices(ny)
    kx = signed_indices(nx)
    xi_y = 2.0 * np.pi * ky[:, None] / ny * np.ones((1, nx))
    xi_x = 2.0 * np.pi * kx[None, :] / nx * np.ones((ny, 1))
    return xi_y, xi_x


def gradient_wavevectors(ny, nx):
    """Wavevectors used for gradients and the compatibility projection.

    Identical to ``wavevectors`` except that a component whose index sits on
    the Nyquist frequency |k| = N/2 (even N only) is set to zero.
    """
    xi_y, xi_x = wavevectors(ny, nx)
    ky = signed_indices(ny)[:, None] * np.ones((1, nx), dtype=np.int64)
    kx = signed_indices(nx)[None, :] * np.ones((ny, 1), dtype=np.int64)
    if ny % 2 == 0:
        xi_y = np.where(np.abs(ky) == ny // 2, 0.0, xi_y)
    if nx % 2 == 0:
        xi_x = np.where(np.abs(kx) == nx // 2, 0.0, xi_x)
    return xi_y, xi_x


def laplacian_symbol(ny, nx):
    """|2 pi q|^2 for every mode, so that the collocation Laplacian is
    nabla_N^2 g = -F^{-1}[ |2 pi q|^2 F g ]  (Sec. 3.1.2)."""
    xi_y, xi_x = wavevectors(ny, nx)
    return xi_x ** 2 + xi_y ** 2


def fft_field(a):
    """Forward 2-D DFT over the two leading (grid) axes of a real field."""
    return np.fft.fft2(a, axes=(0, 1))


def ifft_field(a_hat):
    """Inverse 2-D DFT over the two leading axes; returns the real part."""
    return np.fft.ifft2(a_hat, axes=(0, 1)).real


def nyquist_modes(ny, nx):
    """Boolean (ny, nx) mask of the modes with a Nyquist index |k| = N/2 in
    either direction (even N only)."""
    ky = signed_indices(ny)[:, None] * np.ones((1, nx), dtype=np.int64)
    kx = signed_indices(nx)[None, :] * np.ones((ny, 1), dtype=np.int64)
    m = np.zeros((ny, nx), dtype=bool)
    if ny % 2 == 0:
        m |= np.abs(ky) == ny // 2
    if nx % 2 == 0:
        m |= np.abs(kx) == nx // 2
    return m


def project_hat(a_hat, nyquist="zero"):
    """Apply the Fourier-space compatibility projection G^ to a tensor field.

    Sec. 3.1.1: G projects an arbitrary symmetric tensor field onto the
    subspace of compatible (symmetrised-gradient) fields; its Fourier form is
    block diagonal, one 2x2-tensor map per mode.  Its form is not printed in
    the paper; the reading taken is the orthogonal projector, in the A:B
    metric, onto {sym(a (x) xi) : a in C^2}.  In 2-D the orthogonal
    complement of that space at a mode xi != 0 is spanned by t (x) t with
    t = (-xi_y, xi_x)/|xi|, so
        G^ : A = A - (t . A . t) t (x) t        (xi != 0)
        G^ : A = 0                               (xi  = 0; the mean strain is
                                                  fixed by the load).
    ``a_hat`` has shape (ny, nx, 2, 2), complex; vector index order is (x, y).

    Even grids (not covered by the paper, which uses odd ones): with
    ``nyquist="zero"`` the gradient wavevector component at a Nyquist index
    is zero, so the strain fluctuation has no Nyquist component along that
    direction; with ``nyquist="free"`` the modes with a Nyquist index are
    left unconstrained (G^ = identity there), i.e. G is the orthogonal
    projector onto the compatible fields plus every field supported on
    those modes.
    """
    ny, nx = a_hat.shape[:2]
    xi_y, xi_x = gradient_wavevectors(ny, nx)
    norm2 = xi_x ** 2 + xi_y ** 2
    nz = norm2 > 0.0
    inv = np.zeros_like(norm2)
    inv[nz] = 1.0 / np.sqrt(norm2[nz])
    t = np.stack([-xi_y * inv, xi_x * inv], axis=-1)  # (ny, nx, 2), x first
    tt = t[..., :, None] * t[..., None, :]
    tat = np.einsum("...i,...ij,...j->...", t, a_hat, t)
    out = a_hat - tat[..., None, None] * tt
    out[~nz] = 0.0
    if nyquist == "free":
        m = nyquist_modes(ny, nx)
        out[m] = a_hat[m]
    elif nyquist != "zero":
        raise ValueError(nyquist)
    return out


def project(a, nyquist="zero"):
    """G applied to a real tensor field of shape (ny, nx, 2, 2)."""
    return ifft_field(project_hat(fft_field(a), nyquist))


def laplacian(g):
    """Collocation Laplacian of a real scalar field (Sec. 3.1.2)."""
    ny, nx = g.shape
    return -ifft_field(laplacian_symbol(ny, nx) * fft_field(g))


def grad_sq_sum(g):
    """sum_x |grad_N g|^2 over the grid, defined through the collocation
    Laplacian as sum_x g (-nabla_N^2 g) (Parseval), so that it is exactly the
    quadratic form whose variation is -2 nabla_N^2 g."""
    return float(np.sum(g * (-laplacian(g))))


def symmetric_gradient(u):
    """Compatible strain sym(grad u) of a periodic displacement u.

    ``u`` has shape (ny, nx, 2) (components x, y).  Derivatives are spectral
    with the gradient wavevectors (Nyquist component zero for even N).
    Returns shape (ny, nx, 2, 2).  Used for displacement recovery checks and
    the brute-force tests.
    """
    ny, nx = u.shape[:2]
    xi_y, xi_x = gradient_wavevectors(ny, nx)
    xi = np.stack([xi_x, xi_y], axis=-1)
    u_hat = fft_field(u)
    grad_hat = 1j * u_hat[..., :, None] * xi[..., None, :]  # d u_i / d x_j
    eps_hat = 0.5 * (grad_hat + np.swapaxes(grad_hat, -1, -2))
    return ifft_field(eps_hat)


def displacement_from_strain(eps_star):
    """Zero-mean periodic displacement u* whose symmetric gradient is the
    compatible field ``eps_star`` (shape (ny, nx, 2, 2)).

    The paper does not solve for u (Sec. 3.1.1 uses strain as the unknown).
    Reading: invert eps^ = sym(i u^ (x) xi) mode by mode,
        u^ = -i [ 2 eps^ xi / |xi|^2 - xi (xi . eps^ . xi) / |xi|^4 ],
    with u^ = 0 where the gradient wavevector vanishes (mean and Nyquist).
    """
    ny, nx = eps_star.shape[:2]
    xi_y, xi_x = gradient_wavevectors(ny, nx)
    xi = np.stack([xi_x, xi_y], axis=-1)
    n2 = xi_x ** 2 + xi_y ** 2
    nz = n2 > 0.0
    e_hat = fft_field(eps_star)
    exi = np.einsum("...ij,...j->...i", e_hat, xi)
    xexi = np.einsum("...i,...i->...", xi, exi)
    u_hat = np.zeros(e_hat.shape[:2] + (2,), dtype=complex)
    u_hat[nz] = -1j * (2.0 * exi[nz] / n2[nz][:, None]
                       - xi[nz] * (xexi[nz] / n2[nz] ** 2)[:, None])
    return ifft_field(u_hat)
