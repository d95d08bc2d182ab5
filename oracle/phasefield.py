"""Phase-field sub-problem: F_phi, its Jacobian J, bound-constrained CG.

Oracle (test infrastructure only).  Follows Sec. 2.1 (fracture energy,
AT1/AT2 local terms, constraint field), Sec. 3.1.2 (collocation Laplacian,
backward-Euler inequality, Jacobian) and Algorithm 1 (BCCG).

Readings of the paper (the printed factors disagree with each other):
  * Fracture energy F_f = G_c/(c_w l) int [ w(phi) + l^2 |grad phi|^2 ] with
    AT1: w = phi,   c_w = 8/3
    AT2: w = phi^2, c_w = 2
    and F_phi = h'(phi) psi0+ + G_c/(c_w l) (w'(phi) - 2 l^2 lap phi)
              + (eta/dt)(phi - phi_old).
    This is the only choice under which the printed 1-D optimal profiles
    (1-|x|/2l)^2 and exp(-|x|/l) and the unit energy per crack length both
    hold; the printed "f = phi^2/2" for AT2 and the missing factor 2 on the
    Laplacian term in F_phi are taken as typesetting slips.
  * With h = (1-phi)^2 every term is affine in phi, so the backward-Euler
    inequality is a linear complementarity problem  J phi - b >= 0,
    phi >= lo, (phi - lo)(J phi - b) = 0 (and the mirror condition at the
    upper bound), with  J x = F_phi(x) - F_phi(0)  and  b = -F_phi(0).
  * Bounds: lo = phi_con(phi_ref) (Sec. 2.1 constraint field; crack set uses
    phi_ref >= threshold, inclusive), hi = 1.  Algorithm 1 has only the lower
    bound; the upper bound phi <= 1 is added with the mirrored active-set rule.
  * Algorithm 1 is written for the update v; it is applied here to phi
    itself (phi = phi_prev + v shifts bounds and right-hand side only), with
    the loop condition read as "while ||r|| > tol" and the step length
    alpha = -(r.p)/(p.Jp), the sign that makes alpha > 0 for p = -r.
  * Stopping rule (relative l2, what "relative" refers to is unstated):
    ||r||_2 <= tol_rel max(||b||_2, ||r0||_2) + tol_abs, r0 the masked
    residual of the clipped initial guess.  ||b|| alone can vanish (AT2 at
    zero strain, where only the bounds drive the solution).
  * Not in the paper (tie-break): if p.Jp <= 0 the iteration stops.
"""

import numpy as np

from . import spectral as sp

MODELS = {1: {"cw": 8.0 / 3.0}, 2: {"cw": 2.0}}


def cw(at):
    """Normalisation constant c_w of Sec. 2.1 (AT1: 8/3, AT2: 2)."""
    return MODELS[at]["cw"]


def local_w(phi, at):
    """Local fracture energy density w(phi): AT1 phi, AT2 phi^2."""
    return phi if at == 1 else phi ** 2


def local_dw(phi, at):
    """w'(phi): AT1 1, AT2 2 phi."""
    return np.ones_like(phi) if at == 1 else 2.0 * phi


def constraint_field(phi_ref, irreversibility, threshold=0.9):
    """phi_con(phi_ref) of Sec. 2.1: 'crack_set' keeps phi_ref where
    phi_ref >= threshold and 0 elsewhere; 'damage' keeps phi_ref."""
    if irreversibility == "damage":
        return phi_ref.copy()
    if irreversibility == "crack_set":
        return np.where(phi_ref >= threshold, phi_ref, 0.0)
    raise ValueError(irreversibility)


def f_phi(phi, psi_plus, at, gc, ell, eta_dt=0.0, phi_old=None):
    """Variational derivative F_phi (Sec. 2.1 with the reading above) plus
    the backward-Euler viscous term (Sec. 3.1.2).  h'(phi) = -2 (1 - phi)."""
    c = gc / (cw(at) * ell)
    out = -2.0 * (1.0 - phi) * psi_plus + c * (local_dw(phi, at) - 2.0 * ell ** 2 * sp.laplacian(phi))
    if eta_dt != 0.0:
        out = out + eta_dt * (phi - (phi_old if phi_old is not None else 0.0))
    return out


class Operator:
    """The affine map phi -> F_phi(phi) split into J (linear) and b."""

    def __init__(self, psi_plus, at, gc, ell, eta_dt=0.0, phi_old=None):
        self.args = (psi_plus, at, gc, ell, eta_dt, phi_old)
        zero = np.zeros_like(psi_plus)
        self.f0 = f_phi(zero, *self.args)
        self.b = -self.f0

    def J(self, x):
        """J x = F_phi(x) - F_phi(0)."""
        return f_phi(x, *self.args) - self.f0

    def dense(self):
        """Dense J (tiny grids only; used by brute-force tests)."""
        ny, nx = self.b.shape
        n = ny * nx
        out = np.empty((n, n))
        for j in range(n):
            e = np.zeros(n)
            e[j] = 1.0
            out[:, j] = self.J(e.reshape(ny, nx)).ravel()
        return out


def _active(phi, r, lo, hi):
    """Active set: at the lower bound with r > 0, or at the upper bound with
    r < 0 (complementary slackness in terms of the residual, Alg. 1)."""
    return ((phi <= lo) & (r > 0.0)) | ((phi >= hi) & (r < 0.0))


def bccg(phi0, lo, hi, op, tol_rel=1e-8, tol_abs=0.0, max_iter=10000):
    """Bound-constrained conjugate gradients (Algorithm 1) on lo <= phi <= hi.

    Returns (phi, info)."""
    b = op.b
    phi = np.clip(phi0, lo, hi)
    r = op.J(phi) - b
    act = _active(phi, r, lo, hi)
    r[act] = 0.0
    p = -r
    ref = max(np.sqrt(np.sum(b * b)), np.sqrt(np.sum(r * r)))
    target = tol_rel * ref + tol_abs
    it = 0
    stopped = "converged"
    while np.sqrt(np.sum(r * r)) > target:
        if it >= max_iter:
            stopped = "max_iter"
            break
        q = op.J(p)
        pq = float(np.sum(p * q))
        if pq <= 0.0:
            stopped = "nonpositive_curvature"
            break
        alpha = -float(np.sum(r * p)) / pq
        phi = np.clip(phi + alpha * p, lo, hi)
        r_old = r
        r = op.J(phi) - b
        act = _active(phi, r, lo, hi)
        r[act] = 0.0
        beta = float(np.sum(r * (r - r_old))) / (alpha * pq)
        p = -r + beta * p
        p[act] = 0.0
        it += 1
    return phi, {"iterations": it, "residual": float(np.sqrt(np.sum(r * r))),
                 "target": float(target), "stopped": stopped}


def optimal_profile(d, at, ell):
    """Optimal 1-D phase-field profile across a straight crack at distance
    d from its centre line (Sec. 2.1): AT1 (1 - |d| / (2 l))^2 for
    |d| <= 2 l, else 0; AT2 exp(-|d| / l)."""
    d = np.abs(np.asarray(d, dtype=np.float64))
    if at == 1:
        return np.where(d <= 2.0 * ell, (1.0 - d / (2.0 * ell)) ** 2, 0.0)
    return np.exp(-d / ell)


def fracture_energy(phi, at, gc, ell):
    """F_f = G_c/(c_w l) [ sum w(phi) + l^2 sum |grad_N phi|^2 ] with unit
    pixel area (Sec. 2.1; the gradient term is the Laplacian quadratic form,
    see ``spectral.grad_sq_sum``)."""
    c = gc / (cw(at) * ell)
    return c * (float(np.sum(local_w(phi, at))) + ell ** 2 * sp.grad_sq_sum(phi))
