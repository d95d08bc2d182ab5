"""Alternating-minimisation load step and per-step statistics.

Oracle (test infrastructure only).  Follows Sec. 3.2.1 and Algorithm 2:
for each strain increment, alternate the mechanics solve at fixed phi and the
phase-field solve at fixed strain until ||phi_n+1 - phi_n||_1 < Tol_AM, with
the irreversibility constraint taken from the phase field at the start of the
load step.  Sec. 3.2.1 also defines the stiffness measure C.

Readings of the paper:
  * ``load_step(eps_bar)`` takes the macroscopic strain of the step directly
    (Algorithm 2 increments it by a fixed Delta eps_bar).
  * Tol_AM is stated in units where lengths are scaled by l (Sec. 3.3): the
    default here is 1e-3 l^2 in pixel units; the L1 norm sums |.| times the
    pixel area.
  * Fields follow Algorithm 2 literally: after a step the strain is the one of
    the last mechanics solve and phi the one of the last phase-field solve.
  * With an initial phase field the phase-field problem is first solved at
    zero strain with phi_con(phi_init) (Algorithm 2, first two lines).
  * C = sigma_bar_ij / eps_bar_ij at the component with the largest
    |eps_bar_ij| (Sec. 3.2.1).
  * ``time_step`` is one iteration of the time-discretized evolution
    (Algorithm 3, Sec. 3.2.2); the caller increments eps_bar when the
    returned ``advance`` is set.
  * Non-variational models (Sec. 2.1, 4.2.1): ``split`` is the crack driving
    force model (psi0+ of the phase-field problem), ``contact`` the model of
    the stress (mechanics problem); contact=None means the same model
    (variational).  The elastic energy reported is the one of the contact
    model, whose derivative the stress is.
  * ``near_equilibrium_step`` is one iteration of the near-equilibrium
    evolution (Algorithm 4, Sec. 3.2.2), with these readings of its printed
    formulas: the crack driving force that gates the rescaling is
    -h'(phi) psi0+ = 2 (1 - phi) psi0+ (the printed -h psi0+ is never
    positive); psi0+ is degree-two homogeneous, psi0+(g eps) = g^2 psi0+(eps)
    (the printed right-hand side lost psi0+); so g solves
    g^2 (-h' psi0+)(x*) + [-F_phi - (-h' psi0+)](x*) = (-F_phi)_max, i.e. the
    denominator is -h' psi0+ > 0 (printed with the opposite sign); a
    negative g^2 (the part of -F_phi that does not scale already exceeds the
    bound) gives g = 0, and a vanishing driving force at x* leaves the strain
    unscaled; F_phi carries no viscous term (at phi = phi_n it is zero
    anyway); x* is the first maximiser in row-major order; the trigger flag
    persists once set.
"""

import numpy as np

from . import constitutive as cm
from . import mechanics as mech
from . import phasefield as pf
from . import spectral as sp


class Problem:
    """One periodic 2-D microstructure and its evolving state.

    Parameters mirror the library's problem configuration: Young's modulus
    field E (ny, nx), Poisson ratio nu, length scale ell (pixels), G_c, AT
    model (1 or 2), split ('none' | 'spectral' | 'voldev': the crack
    driving force model), contact (the stress model; None: same as split),
    irreversibility ('crack_set' | 'damage'), nyquist ('zero' | 'free':
    the strain fluctuation's Nyquist modes on even grids, see
    ``spectral.project_hat``).
    """

    def __init__(self, E, nu=0.2, ell=2.0, gc=1.0, at=1, split="spectral", contact=None,
                 irreversibility="crack_set", threshold=0.9, k_res=0.0,
                 eta_over_dt=0.0, tol_mech=1e-8, tol_pf=1e-8, tol_am=None,
                 tol_abs_mech=0.0, tol_abs_pf=0.0, max_cg=10000,
                 max_newton=30, max_bccg=10000, max_am=1000, phi_init=None, nyquist="zero"):
        self.E = np.asarray(E, dtype=np.float64)
        self.ny, self.nx = self.E.shape
        self.nu, self.ell, self.gc, self.at = float(nu), float(ell), float(gc), int(at)
        self.split, self.irr, self.threshold = split, irreversibility, float(threshold)
        self.contact = split if contact is None else contact
        self.k_res, self.eta_dt = float(k_res), float(eta_over_dt)
        self.tol_mech, self.tol_pf = float(tol_mech), float(tol_pf)
        self.tol_abs_mech, self.tol_abs_pf = float(tol_abs_mech), float(tol_abs_pf)
        self.tol_am = 1e-3 * self.ell ** 2 if tol_am is None else float(tol_am)
        self.max_cg, self.max_newton = int(max_cg), int(max_newton)
        self.max_bccg, self.max_am = int(max_bccg), int(max_am)
        self.nyquist = nyquist
        self.lam, self.mu = cm.lame(self.E, self.nu)
        self.eps_star = np.zeros((self.ny, self.nx, 2, 2))
        self.eps_bar = np.zeros((2, 2))
        self.phi = np.zeros((self.ny, self.nx))
        if phi_init is not None:
            phi_init = np.asarray(phi_init, dtype=np.float64)
            lo = pf.constraint_field(phi_init, self.irr, self.threshold)
            op = pf.Operator(np.zeros_like(self.phi), self.at, self.gc, self.ell)
            self.phi, _ = pf.bccg(phi_init, lo, np.ones_like(lo), op, self.tol_pf,
                                  self.tol_abs_pf, self.max_bccg)
        self.phi_ref = self.phi.copy()
        self.step_count = 0

    # -- pointwise fields ------------------------------------------------
    def strain(self):
        return self.eps_bar + self.eps_star

    def stress(self):
        return cm.stress(self.strain(), self.phi, self.lam, self.mu, self.contact, self.k_res)

    def psi_plus(self):
        return cm.psi0(self.strain(), self.lam, self.mu, self.split)[0]

    def displacement(self):
        """Periodic fluctuation u* (zero mean); the affine part is eps_bar x."""
        return sp.displacement_from_strain(self.eps_star)

    # -- energies --------------------------------------------------------
    def elastic_energy(self, phi=None, eps_star=None):
        phi = self.phi if phi is None else phi
        eps = self.eps_bar + (self.eps_star if eps_star is None else eps_star)
        return float(np.sum(cm.energy_density(eps, phi, self.lam, self.mu, self.contact, self.k_res)))

    def fracture_energy(self, phi=None):
        return pf.fracture_energy(self.phi if phi is None else phi, self.at, self.gc, self.ell)

    # -- sub-problems ----------------------------------------------------
    def solve_mechanics(self):
        self.eps_star, info = mech.solve(self.eps_star, self.eps_bar, self.phi, self.lam,
                                         self.mu, self.contact, self.k_res, self.tol_mech,
                                         self.tol_abs_mech, self.max_newton, self.max_cg,
                                         self.nyquist)
        return info

    def solve_phase_field(self, lo, phi_old=None):
        op = pf.Operator(self.psi_plus(), self.at, self.gc, self.ell, self.eta_dt, phi_old)
        phi, info = pf.bccg(self.phi, lo, np.ones_like(lo), op, self.tol_pf,
                            self.tol_abs_pf, self.max_bccg)
        return phi, info

    # -- Algorithm 2, one strain increment --------------------------------
    def load_step(self, eps_bar, trace=None):
        """Advance one load step at macroscopic strain ``eps_bar`` (2x2 or
        (xx, yy, xy)).  ``trace`` (a list) receives (F_e, F_f) after every
        sub-solve.  Returns a stats dict."""
        eps_bar = np.asarray(eps_bar, dtype=np.float64)
        if eps_bar.shape == (3,):
            eps_bar = cm.sym_tensor(*eps_bar)
        self.eps_bar = eps_bar
        self.phi_ref = self.phi.copy()
        lo = pf.constraint_field(self.phi_ref, self.irr, self.threshold)
        phi_old = self.phi_ref if self.eta_dt != 0.0 else None
        am = newton = cg = bccg = 0
        dphi = np.inf
        converged = True
        while dphi > self.tol_am:
            if am >= self.max_am:
                converged = False
                break
            mi = self.solve_mechanics()
            newton += mi["newton"]
            cg += mi["cg"]
            converged &= mi["converged"]
            if trace is not None:
                trace.append((self.elastic_energy(), self.fracture_energy()))
            phi_new, pi = self.solve_phase_field(lo, phi_old)
            bccg += pi["iterations"]
            converged &= pi["stopped"] == "converged"
            dphi = float(np.sum(np.abs(phi_new - self.phi)))
            self.phi = phi_new
            am += 1
            if trace is not None:
                trace.append((self.elastic_energy(), self.fracture_energy()))
        self.step_count += 1
        return self.stats(am=am, newton=newton, cg=cg, bccg=bccg, dphi=dphi,
                          converged=converged)

    # -- Algorithm 3, one iteration n of the time-discretized evolution ----
    def time_step(self, eps_bar, eta, dt_max, dt_min, dphi_max, dphi_min):
        """One outer iteration of Algorithm 3 (Sec. 3.2.2) at macroscopic
        strain ``eps_bar``: the elasticity sub-problem at phi_n, then the
        phase-field sub-problem with the viscous term eta/dt and phi_con(phi_n)
        (phi_old = phi_n), halving dt until ||phi_n+1 - phi_n||_1 < dphi_max
        or dt <= dt_min; dt doubles (up to dt_max) when the accepted change is
        below dphi_max / 2.  dt persists between calls (initially dt_max).
        Returns the stats dict with dt (the next step's), the halvings and
        ``advance``: the condition under which Algorithm 3 increments the
        macroscopic strain (dphi < dphi_min and dt >= dt_max).

        Readings: the doubling is capped at dt_max (the text bounds dt by
        (dt)_max); each retry restarts the phase-field solve from phi_n."""
        eps_bar = np.asarray(eps_bar, dtype=np.float64)
        if eps_bar.shape == (3,):
            eps_bar = cm.sym_tensor(*eps_bar)
        if not hasattr(self, "dt"):
            self.dt = float(dt_max)
        self.eps_bar = eps_bar
        phi_n = self.phi.copy()
        self.phi_ref = phi_n
        lo = pf.constraint_field(phi_n, self.irr, self.threshold)
        mi = self.solve_mechanics()
        halvings = bccg = 0
        converged = bool(mi["converged"])
        while True:
            op = pf.Operator(self.psi_plus(), self.at, self.gc, self.ell, eta / self.dt, phi_n)
            phi_new, pi = pf.bccg(phi_n, lo, np.ones_like(lo), op, self.tol_pf, self.tol_abs_pf, self.max_bccg)
            bccg += pi["iterations"]
            dphi = float(np.sum(np.abs(phi_new - phi_n)))
            if dphi < dphi_max or self.dt <= dt_min:
                if dphi < 0.5 * dphi_max:
                    self.dt = min(2.0 * self.dt, float(dt_max))
                break
            self.dt *= 0.5
            halvings += 1
        converged &= pi["stopped"] == "converged"
        self.phi = phi_new
        self.step_count += 1
        advance = dphi < dphi_min and self.dt >= dt_max
        return self.stats(am=1, newton=mi["newton"], cg=mi["cg"], bccg=bccg, dphi=dphi, converged=converged,
                          dt=self.dt, halvings=halvings, advance=bool(advance))

    # -- Algorithm 4, one iteration n of the near-equilibrium evolution ----
    def near_equilibrium_step(self, eps_bar, deps, fphi_max, drive_threshold, eta=0.0, dt_max=1.0,
                              dphi_min=0.0):
        """One outer iteration of Algorithm 4 (Sec. 3.2.2) at macroscopic
        strain ``eps_bar``: the elasticity sub-problem at phi_n; if the
        largest -F_phi(phi_n, eps_n) exceeds ``fphi_max`` (and the trigger
        flag is set: the largest crack driving force -h'(phi_n) psi0+ has
        once exceeded ``drive_threshold``), the whole strain (eps_bar and
        eps*) is scaled by g so that -F_phi = fphi_max at the maximiser x*,
        with g capped at 1 + max|deps| / max|eps_bar|; then the phase-field
        sub-problem with phi_con(phi_n) and the viscous term eta/dt_max.
        ``deps`` is the load increment (xx, yy, xy).  Returns the stats dict
        with ``gamma``, ``fphi_max`` (the largest -F_phi before scaling),
        ``eps_bar`` (the scaled macroscopic strain), ``ne_flag`` and
        ``advance`` (||phi_n+1 - phi_n||_1 < dphi_min: the caller then adds
        deps to the returned eps_bar)."""
        eps_bar = np.asarray(eps_bar, dtype=np.float64)
        if eps_bar.shape == (3,):
            eps_bar = cm.sym_tensor(*eps_bar)
        if not hasattr(self, "ne_flag"):
            self.ne_flag = False
        self.eps_bar = eps_bar
        phi_n = self.phi.copy()
        self.phi_ref = phi_n
        lo = pf.constraint_field(phi_n, self.irr, self.threshold)
        mi = self.solve_mechanics()
        psi = self.psi_plus()
        neg_f = -pf.f_phi(phi_n, psi, self.at, self.gc, self.ell)
        drive = 2.0 * (1.0 - phi_n) * psi
        fmax = float(neg_f.max())
        if fmax > fphi_max and float(drive.max()) > drive_threshold:
            self.ne_flag = True
        gamma = 1.0
        if fmax > fphi_max and self.ne_flag:
            i = int(np.argmax(neg_f))
            dx, fx = float(drive.flat[i]), float(neg_f.flat[i])
            if dx > 0.0:
                gamma = float(np.sqrt(max((fphi_max - (fx - dx)) / dx, 0.0)))
            eb = max(abs(eps_bar[0, 0]), abs(eps_bar[1, 1]), abs(eps_bar[0, 1]))
            if eb > 0.0:
                gamma = min(gamma, 1.0 + float(np.max(np.abs(deps))) / eb)
            self.eps_star = gamma * self.eps_star
            self.eps_bar = gamma * self.eps_bar
        op = pf.Operator(self.psi_plus(), self.at, self.gc, self.ell, eta / dt_max, phi_n)
        phi_new, pi = pf.bccg(phi_n, lo, np.ones_like(lo), op, self.tol_pf, self.tol_abs_pf, self.max_bccg)
        dphi = float(np.sum(np.abs(phi_new - phi_n)))
        self.phi = phi_new
        self.step_count += 1
        converged = bool(mi["converged"]) and pi["stopped"] == "converged"
        ebar = [float(self.eps_bar[0, 0]), float(self.eps_bar[1, 1]), float(self.eps_bar[0, 1])]
        return self.stats(am=1, newton=mi["newton"], cg=mi["cg"], bccg=pi["iterations"], dphi=dphi,
                          converged=converged, gamma=gamma, fphi_max=fmax, eps_bar=ebar,
                          ne_flag=bool(self.ne_flag), advance=bool(dphi < dphi_min))

    def stats(self, **extra):
        sig = self.stress()
        sbar = sig.mean(axis=(0, 1))
        comps = [(0, 0), (1, 1), (0, 1)]
        ebar = [self.eps_bar[i, j] for i, j in comps]
        k = int(np.argmax(np.abs(ebar)))
        stiff = sbar[comps[k]] / ebar[k] if ebar[k] != 0.0 else float("nan")
        out = {
            "F_e": self.elastic_energy(),
            "F_f": self.fracture_energy(),
            "sigma_bar": [float(sbar[i, j]) for i, j in comps],
            "C_bar": float(stiff),
            "phi_max": float(self.phi.max()),
            "phi_mean": float(self.phi.mean()),
            "crack_px": int(np.count_nonzero(self.phi > 0.9)),
        }
        out.update(extra)
        return out

    # -- state transfer ---------------------------------------------------
    def get_state(self):
        return {"eps_star": self.eps_star.copy(), "phi": self.phi.copy(),
                "phi_ref": self.phi_ref.copy(), "eps_bar": self.eps_bar.copy(),
                "step": self.step_count}

    def set_state(self, state):
        self.eps_star = np.asarray(state["eps_star"], dtype=np.float64).copy()
        self.phi = np.asarray(state["phi"], dtype=np.float64).copy()
        self.phi_ref = np.asarray(state.get("phi_ref", self.phi), dtype=np.float64).copy()
        self.eps_bar = np.asarray(state.get("eps_bar", np.zeros((2, 2))), dtype=np.float64).copy()
        self.step_count = int(state.get("step", 0))
