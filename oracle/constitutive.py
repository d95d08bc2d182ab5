"""Pointwise constitutive model: degradation, energy splits, stress, tangent.

Oracle (test infrastructure only).  Follows Sec. 2.1 (isotropic energy,
split schema, strain-spectral split, stresses) and Sec. 3.1.1 (tangent C).

Tensors are full symmetric 2x2 matrices with shape (..., 2, 2).  Eigenvalues
and eigenvectors come from ``numpy.linalg.eigh``.

Readings of the paper:
  * Sec. 2.1 gives lambda = E nu / (1 - nu - 2 nu^2), the three-dimensional
    Lame constant, while Sec. 3.1.1 speaks of plane stress with a 2x2 strain.
    The printed strength values of Sec. 3.3 use lambda + 2 mu = 10/9 E at
    nu = 0.2, i.e. the 3-D constants on a 2x2 strain: plane strain.  That is
    the reading taken (out-of-plane strain zero, not represented).
  * The strain-spectral split runs over the two in-plane eigenvalues.
  * Ramp derivatives: H+(x) = [x > 0], H-(x) = [x < 0] (value 0 at x = 0).
  * An optional residual stiffness k_res is added to h(phi) in the elastic
    energy and the stress, psi = (h + k_res) psi0+ + psi0-; the paper has
    k_res = 0, which is the default everywhere.
  * Volumetric-deviatoric split (Sec. 2.1): K = lambda + 2 mu / 3 and the
    deviator with the 1/3 trace are three-dimensional; in plane strain the
    out-of-plane strain is zero, so the deviatoric energy sums the in-plane
    components and the zz component -tr/3:  mu (eps:eps - tr^2 / 3).  This
    makes psi0+ + psi0- the isotropic energy and sigma0+ + sigma0- the
    isotropic stress, as Sec. 4.2.1 states for all models at phi = 0; the
    printed psi0+ = 2 mu (a^2 + ab + 5 b^2/18) of Sec. 4.2.1 instead sums the
    in-plane components only (giving b^2/3 in place of 5 b^2/18 here) and
    would break that statement.  The stresses are the derivatives:
    sigma0+ = K <tr>+ I + 2 mu (eps - tr/3 I), sigma0- = K <tr>- I (the
    worked contact example of Sec. 4.2.1 gives K tr I for the negative part).
  * Non-variational models (Sec. 2.1, 4.2.1) pair the crack driving force of
    one split with the stress ("contact model") of another; the functions
    here take one model each, the caller chooses which one feeds the stress
    and which the driving force psi0+.
"""

import numpy as np

SPLITS = ("none", "spectral", "voldev")

I2 = np.eye(2)


def lame(E, nu):
    """Lame constants (lambda, mu) from Young's modulus and Poisson ratio
    (Sec. 2.1, after the isotropic energy density)."""
    E = np.asarray(E, dtype=np.float64)
    mu = E / (2.0 + 2.0 * nu)
    lam = E * nu / (1.0 - nu - 2.0 * nu * nu)
    return lam, mu


def degradation(phi):
    """h(phi) = (1 - phi)^2 (Sec. 2.1)."""
    return (1.0 - phi) ** 2


def ramp(x, sign):
    """<x>_+ (sign=+1) or <x>_- (sign=-1) (Sec. 2.1)."""
    return np.maximum(x, 0.0) if sign > 0 else np.minimum(x, 0.0)


def step(x, sign):
    """Derivative of the ramp: [x > 0] for sign=+1, [x < 0] for sign=-1."""
    return (x > 0.0).astype(np.float64) if sign > 0 else (x < 0.0).astype(np.float64)


def trace(eps):
    return eps[..., 0, 0] + eps[..., 1, 1]


def ddot(a, b):
    """A:B = sum_ij A_ij B_ij, pointwise."""
    return np.einsum("...ij,...ij->...", a, b)


def _outer(u, v):
    return u[..., :, None] * v[..., None, :]


def eig(eps):
    """Eigenvalues (ascending) and eigenvectors (columns) of symmetric 2x2
    tensors."""
    return np.linalg.eigh(eps)


def psi0(eps, lam, mu, split):
    """(psi0+, psi0-) of the split schema psi = psi0+ h + psi0- (Sec. 2.1).

    none      (isotropic energy): psi0+ = 1/2 (lam tr^2 + 2 mu eps:eps),
                                  psi0- = 0
    spectral  (strain-spectral):  psi0+- = 1/2 lam <tr>+-^2
                                           + mu sum_a <eps_a>+-^2
    """
    tr = trace(eps)
    if split == "none":
        plus = 0.5 * (lam * tr ** 2 + 2.0 * mu * ddot(eps, eps))
        return plus, np.zeros_like(plus)
    if split == "spectral":
        w, _ = eig(eps)
        out = []
        for s in (+1, -1):
            out.append(0.5 * lam * ramp(tr, s) ** 2
                       + mu * np.sum(ramp(w, s) ** 2, axis=-1))
        return out[0], out[1]
    if split == "voldev":
        K = lam + 2.0 * mu / 3.0
        dev2 = ddot(eps, eps) - tr ** 2 / 3.0
        return 0.5 * K * ramp(tr, +1) ** 2 + mu * dev2, 0.5 * K * ramp(tr, -1) ** 2
    raise ValueError(split)


def sigma0(eps, lam, mu, split):
    """(sigma0+, sigma0-) (Sec. 2.1, isotropic and strain-spectral stresses).

    none:      sigma0+ = lam tr I + 2 mu eps, sigma0- = 0
    spectral:  sigma0+- = sum_a (lam <tr>+- + 2 mu <eps_a>+-) n_a (x) n_a
    """
    lam = np.asarray(lam)[..., None, None]
    mu = np.asarray(mu)[..., None, None]
    tr = trace(eps)
    if split == "none":
        plus = lam * tr[..., None, None] * I2 + 2.0 * mu * eps
        return plus, np.zeros_like(plus)
    if split == "spectral":
        w, v = eig(eps)
        out = []
        for s in (+1, -1):
            acc = np.zeros(eps.shape)
            for a in range(2):
                n = v[..., :, a]
                coef = lam[..., 0, 0] * ramp(tr, s) + 2.0 * mu[..., 0, 0] * ramp(w[..., a], s)
                acc = acc + coef[..., None, None] * _outer(n, n)
            out.append(acc)
        return out[0], out[1]
    if split == "voldev":
        lam0, mu0 = lam[..., 0, 0], mu[..., 0, 0]
        K = lam0 + 2.0 * mu0 / 3.0
        plus = (K * ramp(tr, +1) - 2.0 * mu0 * tr / 3.0)[..., None, None] * I2 + 2.0 * mu * eps
        minus = (K * ramp(tr, -1))[..., None, None] * I2
        return plus, minus
    raise ValueError(split)


def energy_density(eps, phi, lam, mu, split, k_res=0.0):
    """psi(phi, eps) = (h(phi) + k_res) psi0+ + psi0- (Sec. 2.1 schema)."""
    p, m = psi0(eps, lam, mu, split)
    return (degradation(phi) + k_res) * p + m


def stress(eps, phi, lam, mu, split, k_res=0.0):
    """sigma = (h(phi) + k_res) sigma0+ + sigma0- (Sec. 2.1)."""
    p, m = sigma0(eps, lam, mu, split)
    g = np.asarray(degradation(np.asarray(phi, dtype=np.float64)) + k_res)
    return g[..., None, None] * p + m


def dsigma0(eps, d, lam, mu, split, sign):
    """Directional derivative of sigma0+ (sign=+1) or sigma0- (sign=-1) at
    ``eps`` along ``d``.

    Sec. 3.1.1 says the tangents are available in the literature; the reading
    taken is the exact directional derivative, written in the eigenbasis:
      d sigma0 = lam H(tr) tr(d) I
               + 2 mu sum_a H(eps_a) (n_a.d.n_a) n_a (x) n_a
               + 2 mu c12 (n_1.d.n_2) (n_1 (x) n_2 + n_2 (x) n_1),
      c12 = (<eps_1> - <eps_2>) / (eps_1 - eps_2), or H(eps_1) when the two
      eigenvalues coincide (the limit of the quotient).
    """
    lam_ = np.asarray(lam)
    mu_ = np.asarray(mu)
    trd = trace(d)
    if split == "none":
        if sign < 0:
            return np.zeros(np.broadcast_shapes(eps.shape, d.shape))
        return lam_[..., None, None] * trd[..., None, None] * I2 + 2.0 * mu_[..., None, None] * d
    if split == "voldev":
        # d sigma0+ = K H+(tr) tr(d) I + 2 mu (d - tr(d)/3 I),
        # d sigma0- = K H-(tr) tr(d) I
        K = lam_ + 2.0 * mu_ / 3.0
        vol = (K * step(trace(eps), sign) * trd)[..., None, None] * I2
        if sign < 0:
            return vol + np.zeros(np.broadcast_shapes(eps.shape, d.shape))
        return vol + 2.0 * mu_[..., None, None] * (d - (trd / 3.0)[..., None, None] * I2)
    w, v = eig(eps)
    n1, n2 = v[..., :, 0], v[..., :, 1]
    e1, e2 = w[..., 0], w[..., 1]
    out = (lam_ * step(trace(eps), sign) * trd)[..., None, None] * I2
    for a, n in ((0, n1), (1, n2)):
        dn = np.einsum("...i,...ij,...j->...", n, d, n)
        out = out + (2.0 * mu_ * step(w[..., a], sign) * dn)[..., None, None] * _outer(n, n)
    diff = e1 - e2
    same = diff == 0.0
    safe = np.where(same, 1.0, diff)
    c12 = np.where(same, step(e1, sign), (ramp(e1, sign) - ramp(e2, sign)) / safe)
    d12 = np.einsum("...i,...ij,...j->...", n1, d, n2)
    out = out + (2.0 * mu_ * c12 * d12)[..., None, None] * (_outer(n1, n2) + _outer(n2, n1))
    return out


def tangent_action(eps, d, phi, lam, mu, split, k_res=0.0):
    """C : d with C = d sigma / d eps at ``eps`` (Sec. 3.1.1):
    (h + k_res) dsigma0+[d] + dsigma0-[d]."""
    g = np.asarray(degradation(np.asarray(phi, dtype=np.float64)) + k_res)[..., None, None]
    return g * dsigma0(eps, d, lam, mu, split, +1) + dsigma0(eps, d, lam, mu, split, -1)


def sym_tensor(xx, yy, xy):
    """Assemble full symmetric tensors from (xx, yy, xy) tensor components."""
    xx, yy, xy = np.broadcast_arrays(np.asarray(xx, float), np.asarray(yy, float),
                                     np.asarray(xy, float))
    out = np.empty(xx.shape + (2, 2))
    out[..., 0, 0] = xx
    out[..., 1, 1] = yy
    out[..., 0, 1] = xy
    out[..., 1, 0] = xy
    return out
