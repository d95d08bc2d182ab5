"""Fourier-Galerkin mechanics sub-problem: Newton on eps*, CG on the update.

Oracle (test infrastructure only).  Follows Sec. 3.1.1: strain eps = eps_bar
+ eps* with eps* compatible and zero-mean, loading by eps_bar; nodal
equilibrium G^ : sigma^ = 0; Newton update theta from CG on
G^ : (C_m : theta)^ = -G^ : sigma^_m; one Newton step for the linear
(isotropic) model, a looser inner tolerance for the split model.

Readings of the paper:
  * The sign of the Newton system is not printed; the consistent one is
    G[C_m : theta] = -G[sigma_m].
  * The mechanics tolerance is printed for the L-infinity norm while the
    evolution section says sub-problems are converged in the l2 norm; l2 is
    used.  Stop when ||G[sigma]||_2 <= tol_rel max(||sigma_hom||_2, ||R0||_2)
    + tol_abs, where sigma_hom = sigma(eps_bar) evaluated pixel by pixel with
    the current phi and material (the stress if eps* were 0) and R0 the
    residual of the warm start (it sets the scale when eps_bar = 0).
  * "A lower relative tolerance" for the Newton inner CG of the split model is
    unspecified: the inner CG stops at max(0.1 ||R_m||, final tolerance).
  * All inner products are sum over pixels of A:B, the metric in which G is
    an orthogonal projector and C is symmetric.
"""

import numpy as np

from . import constitutive as cm
from . import spectral as sp


def inner(a, b):
    """sum over pixels of A:B."""
    return float(np.sum(a * b))


def residual(eps_star, eps_bar, phi, lam, mu, split, k_res, nyquist="zero"):
    """R = G[sigma(eps_bar + eps*)] (Sec. 3.1.1, nodal equilibrium)."""
    eps = eps_bar + eps_star
    return sp.project(cm.stress(eps, phi, lam, mu, split, k_res), nyquist)


def cg(apply_k, b, tol_abs, max_iter):
    """Plain conjugate gradients from x = 0 for K x = b, K symmetric positive
    (semi)definite on the compatible subspace; stop when ||r|| <= tol_abs.

    Returns (x, iterations, final ||r||, converged)."""
    x = np.zeros_like(b)
    r = b.copy()
    p = r.copy()
    rr = inner(r, r)
    it = 0
    while np.sqrt(rr) > tol_abs and it < max_iter:
        q = apply_k(p)
        pq = inner(p, q)
        if pq <= 0.0:
            break
        alpha = rr / pq
        x = x + alpha * p
        r = r - alpha * q
        rr_new = inner(r, r)
        beta = rr_new / rr
        p = r + beta * p
        rr = rr_new
        it += 1
    return x, it, float(np.sqrt(rr)), bool(np.sqrt(rr) <= tol_abs)


def solve(eps_star, eps_bar, phi, lam, mu, split, k_res=0.0, tol_rel=1e-8,
          tol_abs=0.0, max_newton=30, max_cg=10000, nyquist="zero"):
    """Solve the mechanics sub-problem at fixed phi and eps_bar.

    ``eps_star`` is the warm start (shape (ny, nx, 2, 2)); ``eps_bar`` a
    2x2 tensor.  Returns (eps_star, info) with Newton / CG iteration counts.
    """
    eps_bar = np.asarray(eps_bar, dtype=np.float64)
    hom = eps_bar * np.ones_like(eps_star)
    sig_hom = cm.stress(hom, phi, lam, mu, split, k_res)
    R0 = residual(eps_star, eps_bar, phi, lam, mu, split, k_res, nyquist)
    ref = max(np.sqrt(inner(sig_hom, sig_hom)), np.sqrt(inner(R0, R0)))
    target = tol_rel * ref + tol_abs
    newton = 0
    cg_total = 0
    converged = False
    while True:
        R = residual(eps_star, eps_bar, phi, lam, mu, split, k_res, nyquist)
        res = np.sqrt(inner(R, R))
        if res <= target:
            converged = True
            break
        if newton >= max_newton:
            break
        eps_m = eps_bar + eps_star
        if split == "none":
            inner_tol = target
        else:
            inner_tol = max(0.1 * res, target)

        def apply_k(d):
            return sp.project(cm.tangent_action(eps_m, d, phi, lam, mu, split, k_res), nyquist)

        theta, its, _, _ = cg(apply_k, -R, inner_tol, max_cg)
        cg_total += its
        eps_star = eps_star + theta
        newton += 1
        if its == 0:
            break
    return eps_star, {"newton": newton, "cg": cg_total, "residual": float(res),
                      "target": float(target), "converged": converged}
