"""Poisson-Boltzmann pieces of the oracle (Sec. III; test infrastructure only).

Ionic charge (Eq. rhoions) with concentrations from the Boltzmann law
(Eq. ionsconcPB) or the steric Bikerman/Langmuir form (Eq. ionsconcMPB with
c_max from Eq. maxconc), weighted by an ion-accessibility field gamma in
[0, 1] that keeps ions out of the solute cavity.  Units are Hartree atomic
units: phi in Ha/e, kT in Ha, concentrations in bohr^-3, charge in e/bohr^3;
the factor e N_A of the paper's SI-style notation is absorbed into the
concentration unit.

Readings of the paper taken here:
  * Eq. ionsconcMPB prints "+1" inside the denominator's bracket; the bulk
    limit c_i(phi = 0) = c_i^inf requires "-1", which is used.
  * Algorithm SCPBimproved: "phi_k = phi_k + phi'_k" is read as accumulating
    the corrections, phi <- phi + phi'; the unspecified rho^ions_1 is 0,
    matching the stated input guess rho^ions_0 = 0.
  * Inner tolerance of SCPBimproved: equal to the outer one expressed on the
    PCG residual (||r|| <= 4 pi tol ||rho||), except in the first two outer
    iterations, which stop at 1e-2 relative to their own initial residual.
  * The outer stopping test is ||rho^ions_{k+1} - rho^ions_k||_2 <= tol ||rho||_2.
"""
import numpy as np

from .pcg import pcg_solve, fixed_fields, FOUR_PI, STATUS_OK, STATUS_NONFINITE, \
    STATUS_NOT_CONVERGED
from .green import VacuumSolver


class Electrolyte:
    """Species valences Z, bulk concentrations c (bohr^-3), optional c_max."""

    def __init__(self, Z, c_bulk, kT, c_max=None, eps_bulk=78.36, gamma=None):
        self.Z = np.asarray(Z, dtype=np.float64)
        self.c = np.asarray(c_bulk, dtype=np.float64)
        self.kT = float(kT)
        self.c_max = None if c_max is None else np.asarray(c_max, dtype=np.float64)
        self.eps_bulk = float(eps_bulk)
        self.gamma = gamma

    def accessibility(self, eps):
        """gamma(r): given field, else (eps - 1)/(eps_bulk - 1)."""
        if self.gamma is not None:
            return np.asarray(self.gamma, dtype=np.float64)
        return (np.asarray(eps, dtype=np.float64) - 1.0) / (self.eps_bulk - 1.0)

    def kappa2(self, eps):
        """Linear-PB coefficient of Eq. corrPB: (4 pi / kT) sum Z^2 c * gamma."""
        return FOUR_PI / self.kT * float(np.sum(self.Z ** 2 * self.c)) * self.accessibility(eps)


def max_concentration(packing, radius_bohr):
    """Eq. maxconc in atomic units: c_max = p / (4/3 pi R^3)."""
    return packing / (4.0 / 3.0 * np.pi * radius_bohr ** 3)


def ionic_charge(phi, ions, gamma):
    """rho^ions[phi] = gamma sum_i Z_i c_i[phi]   (Eqs. rhoions, ionsconc(M)PB).

    Boltzmann: c_i = c_i^inf exp(x_i), x_i = -Z_i phi / kT.  May overflow; the
    caller sees a non-finite value.
    MPB: c_i = c_i^inf exp(x_i) / (1 + sum_j a_j (exp(x_j) - 1)), a_j = c_j/c_j^max.
    Numerator and denominator are both multiplied by exp(-xm), with
    xm = max(0, max_j x_j), which is exact and cannot overflow.
    """
    phi = np.asarray(phi, dtype=np.float64)
    x = [-z * phi / ions.kT for z in ions.Z]
    if ions.c_max is None:
        with np.errstate(over="ignore", invalid="ignore"):
            tot = sum(z * c * np.exp(xi) for z, c, xi in zip(ions.Z, ions.c, x))
        return gamma * tot
    a = ions.c / ions.c_max
    xm = np.maximum(0.0, np.max(np.stack(x), axis=0))
    denom = np.exp(-xm) * (1.0 - float(np.sum(a))) + sum(
        aj * np.exp(xj - xm) for aj, xj in zip(a, x))
    num = sum(z * c * np.exp(xi - xm) for z, c, xi in zip(ions.Z, ions.c, x))
    return gamma * num / denom


class PBResult:
    def __init__(self, phi, rho_ion, status, outer, inner_iterations, residuals,
                 rho_ion_used=None, rprime=None):
        self.phi = phi
        self.rho_ion_used = rho_ion_used      # ionic charge of the last solve
        self.rprime = rprime                  # left-over residual (as a charge)
        self.rho_ion = rho_ion
        self.status = status
        self.outer = outer
        self.inner_iterations = inner_iterations
        self.residuals = residuals

    @property
    def converged(self):
        return self.status == STATUS_OK


def solve_linear_pb(rho, eps, h, bc, ions, tol, **kw):
    """Linear PB: Algorithm PCG with the operator of Eq. corrPB."""
    return pcg_solve(rho, eps, h, bc, tol=tol, kappa2=ions.kappa2(eps), **kw)


def scpb(rho, eps, h, bc, ions, tol, eta=0.3, outer_maxit=200, inner_tol=1e-11,
         fd_order=16, solver=None, maxit=1000):
    """Algorithm SCPB: full generalized-Poisson solve on rho + rho^ions each step."""
    rho = np.asarray(rho, dtype=np.float64)
    if solver is None:
        solver = VacuumSolver(rho.shape, h, bc)
    fields = fixed_fields(eps, h, bc, fd_order)
    gamma = ions.accessibility(eps)
    rho_norm = float(np.sqrt(np.sum(rho * rho)))
    rho_ion = np.zeros_like(rho)
    phi = np.zeros_like(rho)
    inner, res = [], []
    status = STATUS_NOT_CONVERGED
    for k in range(outer_maxit):
        used = rho_ion
        sol = pcg_solve(rho + rho_ion, eps, h, bc, tol=inner_tol, solver=solver,
                        fields=fields, maxit=maxit)
        inner.append(sol.iterations)
        phi = sol.phi
        new = ionic_charge(phi, ions, gamma)
        mixed = eta * new + (1.0 - eta) * rho_ion
        dr = float(np.sqrt(np.sum((mixed - rho_ion) ** 2)))
        res.append(dr)
        rho_ion = mixed
        if not np.isfinite(dr):
            status = STATUS_NONFINITE
            break
        if dr <= tol * rho_norm:
            status = STATUS_OK
            break
    return PBResult(phi, rho_ion, status, len(res), inner, res, rho_ion_used=used)


def inner_threshold(k, tol, rho_norm, rnorm0_inner):
    """PCG stop threshold for outer step k (1-based) of Algorithm SCPBimproved."""
    absolute = FOUR_PI * tol * rho_norm
    if k <= 2:
        return max(absolute, 1e-2 * rnorm0_inner)
    return absolute


def scpb_improved(rho, eps, h, bc, ions, tol, eta=0.3, outer_maxit=200,
                  fd_order=16, solver=None, maxit=1000):
    """Algorithm SCPBimproved: each step solves only for the correction phi'.

    State: phi, rho^ions_k, rho^ions_{k-1}, r' (left-over residual as a charge).
    rho_tot = r' + rho^ions_k - rho^ions_{k-1}; PCG from phi' = 0 returns its
    final residual r_fin and r' <- -r_fin/(4 pi), so that at every step
    A phi = -4 pi (rho + rho^ions_k - r') holds exactly.
    """
    rho = np.asarray(rho, dtype=np.float64)
    if solver is None:
        solver = VacuumSolver(rho.shape, h, bc)
    fields = fixed_fields(eps, h, bc, fd_order)
    gamma = ions.accessibility(eps)
    rho_norm = float(np.sqrt(np.sum(rho * rho)))
    phi = np.zeros_like(rho)
    rho_ion_prev = np.zeros_like(rho)
    rho_ion = np.zeros_like(rho)
    rprime = rho.copy()
    inner, res = [], []
    status = STATUS_NOT_CONVERGED
    for k in range(1, outer_maxit + 1):
        rho_tot = rprime + rho_ion - rho_ion_prev
        used = rho_ion
        r0 = FOUR_PI * float(np.sqrt(np.sum(rho_tot * rho_tot)))
        thr = inner_threshold(k, tol, rho_norm, r0)
        sol = pcg_solve(rho_tot, eps, h, bc, abs_threshold=thr, solver=solver,
                        fields=fields, maxit=maxit)
        inner.append(sol.iterations)
        rprime = -sol.r / FOUR_PI
        phi = phi + sol.phi
        new = ionic_charge(phi, ions, gamma)
        rho_ion_prev = rho_ion
        rho_ion = eta * new + (1.0 - eta) * rho_ion
        dr = float(np.sqrt(np.sum((rho_ion - rho_ion_prev) ** 2)))
        res.append(dr)
        if not np.isfinite(dr):
            status = STATUS_NONFINITE
            break
        if dr <= tol * rho_norm:
            status = STATUS_OK
            break
    return PBResult(phi, rho_ion, status, len(res), inner, res, rho_ion_used=used,
                    rprime=rprime)
