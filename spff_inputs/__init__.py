"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the
benchmark.  Holds no solver arithmetic: only microstructure fields, load
ramps and initial phase fields.

Young's modulus recipe (stands in for the paper's generated microstructures,
Sec. 3.4, whose realisations are not available):
    w  ~ N(0, 1) white noise on the ny x nx grid (numpy PCG64, ``seed``)
    z  = irfft2( rfft2(w) * exp(-|xi|^2 c^2 / 4) ),  xi = 2 pi k / N
         (covariance proportional to exp(-r^2 / (2 c^2)); c = correlation
         length in pixels)
    z  <- (z - mean z) / std z
    E  = max(1 + a z, floor)            rounded to float32
Realisation i of workload configuration j uses seed = 1000 j + i.

Also: the paper's two-phase ("slit island") microstructure (Sec. 3.4) and
its initial phase fields for a crack and a small void (Sec. 4.1.1).
"""

import numpy as np


def gaussian_random_field(ny, nx, corr_len, seed):
    """Unit-variance, zero-mean Gaussian random field with a Gaussian
    correlation of length ``corr_len`` pixels (float64, shape (ny, nx))."""
    rng = np.random.default_rng(seed)
    w = rng.standard_normal((ny, nx))
    ky = np.fft.fftfreq(ny)[:, None] * 2.0 * np.pi
    kx = np.fft.rfftfreq(nx)[None, :] * 2.0 * np.pi
    filt = np.exp(-(kx ** 2 + ky ** 2) * corr_len ** 2 / 4.0)
    z = np.fft.irfft2(np.fft.rfft2(w) * filt, s=(ny, nx))
    z = z - z.mean()
    return z / z.std()


def young_modulus(n, corr_len, amp, seed, floor=0.5, ny=None):
    """E = max(1 + amp * z, floor) as float32, shape (ny or n, n)."""
    ny = n if ny is None else ny
    z = gaussian_random_field(ny, n, corr_len, seed)
    return np.maximum(1.0 + amp * z, floor).astype(np.float32)


def strength_strain(nu, ell, gc=1.0, E0=1.0):
    """Uniaxial-strain strength eps_M = sqrt(3 G_c / (8 l (lambda + 2 mu)))
    of a homogeneous AT1 material with modulus E0 (Sec. 3.3); used only to
    scale load ramps."""
    lam = E0 * nu / (1.0 - nu - 2.0 * nu * nu)
    mu = E0 / (2.0 + 2.0 * nu)
    return float(np.sqrt(3.0 * gc / (8.0 * ell * (lam + 2.0 * mu))))


def uniaxial_ramp(steps, nu, ell, gc=1.0, factor=1.5):
    """Macroscopic strains (xx, yy, xy) of a uniaxial-strain ramp in ``steps``
    equal increments of eps_yy up to ``factor`` * eps_M; array (steps, 3)."""
    em = strength_strain(nu, ell, gc)
    e = np.arange(1, steps + 1, dtype=np.float64) / steps * factor * em
    out = np.zeros((steps, 3))
    out[:, 1] = e
    return out


def centre_crack(ny, nx, ell, length, dx=1.0):
    """Initial phase field of a straight crack of length ``length`` centred
    on the grid (Sec. 4.1.1): phi = (1 - |r| / (2 l))^2 where |r| <= 2 l, 0
    elsewhere, r = (max(|x| - L_crack/2, 0), y) on a grid centred at the
    origin.  Readings: the printed r lost the absolute value of x (with it
    the crack has the stated length L_crack; without it the crack would run
    from the periodic boundary to x = L_crack/2); the cut-off "|r| <= 2" is
    |r| <= 2 l.  Returns float32."""
    y = (np.arange(ny) - ny // 2)[:, None] * dx
    x = (np.arange(nx) - nx // 2)[None, :] * dx
    rx = np.maximum(np.abs(x) - 0.5 * length, 0.0)
    r = np.sqrt(rx ** 2 + y ** 2)
    phi = np.where(r <= 2.0 * ell, (1.0 - r / (2.0 * ell)) ** 2, 0.0)
    return phi.astype(np.float32)


def edge_crack(ny, nx, ell, length, dx=1.0):
    """Initial phase field of a straight crack (Sec. 4.1.1, initial crack
    condition): phi = (1 - |r| / (2 l))^2 where |r| <= 2 l, 0 elsewhere, with
    r = (max(x - L_crack/2, 0), y) on a grid centred at the origin.  The
    printed cut-off "|r| <= 2" is read as |r| <= 2 l.  Returns float32."""
    y = (np.arange(ny) - ny // 2)[:, None] * dx
    x = (np.arange(nx) - nx // 2)[None, :] * dx
    rx = np.maximum(x - 0.5 * length, 0.0)
    r = np.sqrt(rx ** 2 + y ** 2)
    phi = np.where(r <= 2.0 * ell, (1.0 - r / (2.0 * ell)) ** 2, 0.0)
    return phi.astype(np.float32)


WORKLOADS = {
    # name: (n, corr_len, amp, ell, steps, seed_base)
    "c1_64": dict(n=64, corr_len=4.0, amp=0.1, ell=2.0, steps=20, seed=1000),
    "c2_256": dict(n=256, corr_len=8.0, amp=0.1, ell=2.0, steps=200, seed=2000),
    "c3_512x64": dict(n=512, corr_len=16.0, amp=0.2, ell=2.0, steps=200, seed=3000, batch=64),
    "c5_2048": dict(n=2048, corr_len=32.0, amp=0.3, ell=1.0, steps=500, seed=5000),
}


def two_phase(n, l_cut, a, seed, iters=21, ny=None):
    """Two-phase Young's modulus field of Sec. 3.4, E0 = 1: white noise
    N(0, 1) (numpy PCG64, ``seed``), low-pass filtered, thresholded to
    sgn(xi) in {-1, 0, 1}, smoothed by ``iters`` explicit Allen-Cahn steps
    xi <- xi - 0.1 [(xi^3 - xi) + (4 xi_k - sum of the four periodic
    neighbours)], and mapped to E = a xi + 1 (bulk phases 1 - a and 1 + a,
    ratio (1 + a) / (1 - a)).  Readings: the filter keeps the modes with
    |q| <= 2 pi / l_cut (the text removes wavelengths shorter than l_cut;
    the printed inequality is reversed); the iteration index runs over
    n = 0 .. 20, i.e. 21 steps.  Returns float32, shape (ny or n, n)."""
    ny = n if ny is None else ny
    rng = np.random.default_rng(seed)
    w = rng.standard_normal((ny, n))
    qy = np.fft.fftfreq(ny)[:, None] * 2.0 * np.pi
    qx = np.fft.fftfreq(n)[None, :] * 2.0 * np.pi
    keep = np.sqrt(qx ** 2 + qy ** 2) <= 2.0 * np.pi / l_cut
    xi = np.sign(np.fft.ifft2(np.fft.fft2(w) * keep).real)
    for _ in range(iters):
        nb = np.roll(xi, 1, 0) + np.roll(xi, -1, 0) + np.roll(xi, 1, 1) + np.roll(xi, -1, 1)
        xi = xi - 0.1 * ((xi ** 3 - xi) + (4.0 * xi - nb))
    return (a * xi + 1.0).astype(np.float32)


def round_void(ny, nx, ell, dx=1.0):
    """Initial phase field of a small void (Sec. 4.1.1): the crack profile
    with r = (x, y) on a grid centred at the origin, phi = (1 - |r| / (2 l))^2
    where |r| <= 2 l, 0 elsewhere.  Returns float32."""
    y = (np.arange(ny) - ny // 2)[:, None] * dx
    x = (np.arange(nx) - nx // 2)[None, :] * dx
    r = np.sqrt(x ** 2 + y ** 2)
    phi = np.where(r <= 2.0 * ell, (1.0 - r / (2.0 * ell)) ** 2, 0.0)
    return phi.astype(np.float32)

