"""Pins of the oracle's Algorithm PCG (Sec. II.B) and linear PB (Eq. corrPB)
against invariants, a dense direct solve, closed forms and limits."""
import math

import numpy as np
import pytest
from scipy import integrate
from scipy.special import erf, erfc

from oracle import green, pcg, dense, pb
from paper_1509_00680_amd import workloads as W

BCS = ("free", "surface", "periodic", "wire")


def _small_problem(bc, n=8, h=0.6, seed=1):
    return W.molecule(n, h, seed=seed, n_atoms=4, ball=1.0, bc=bc)


@pytest.mark.parametrize("bc", BCS)
@pytest.mark.parametrize("eps_value", [1.0, 5.0])
def test_constant_eps_one_iteration(bc, eps_value):
    # eps constant => q = 0, the preconditioner is exact: one iteration,
    # alpha_0 = -1/(4 pi), phi = G rho / eps
    p = _small_problem(bc, 12, 0.5)
    eps = np.full(p.shape, eps_value)
    res = pcg.pcg_solve(p.rho, eps, p.h, bc, tol=1e-12)
    assert res.iterations == 1
    assert abs(res.history[0]["alpha"] * 4 * math.pi + 1.0) < 1e-12
    u = green.VacuumSolver(p.shape, p.h, bc).apply(p.rho) / eps_value
    assert np.abs(res.phi - u).max() < 1e-12 * np.abs(u).max()


@pytest.mark.parametrize("bc", BCS)
@pytest.mark.parametrize("ions", [None, "uniform", "accessibility"])
def test_pcg_equals_dense_direct_solve(bc, ions):
    p = _small_problem(bc)
    kappa2 = None
    if ions == "uniform":
        kappa2 = np.full(p.shape, 0.3)
    elif ions == "accessibility":
        kappa2 = 0.8 * (p.eps - 1.0) / (W.EPS_WATER - 1.0)
    phi_d = dense.dense_solve(p.rho, p.eps, p.h, bc, kappa2=kappa2)
    res = pcg.pcg_solve(p.rho, p.eps, p.h, bc, tol=1e-14, kappa2=kappa2)
    assert res.converged
    assert np.abs(res.phi - phi_d).max() < 1e-12 * np.abs(phi_d).max()


def test_periodic_gauge():
    p = _small_problem("periodic", 12, 0.5)
    res = pcg.pcg_solve(p.rho, p.eps, p.h, "periodic", tol=1e-12)
    assert abs(np.sum(np.sqrt(p.eps) * res.phi)) < 1e-10 * np.abs(res.phi).sum()


def test_zero_charge_zero_iterations():
    p = _small_problem("free")
    res = pcg.pcg_solve(np.zeros(p.shape), p.eps, p.h, "free", tol=1e-8)
    assert res.iterations == 0 and res.converged and not res.phi.any()


def test_breakdown_reported_for_indefinite_preconditioner():
    # the unshifted surface kernel is indefinite (see green); PCG must say so
    p = _small_problem("surface")
    res = pcg.pcg_solve(p.rho, p.eps, p.h, "surface", tol=1e-12, surface_k0_offset=0.0)
    assert res.status == pcg.STATUS_BREAKDOWN


def test_action_decreases_monotonically():
    # CG minimizes the action of Eq. AIntegral over growing Krylov spaces
    p = W.molecule(24, 0.5, seed=3, n_atoms=8, ball=2.0)
    solver = green.VacuumSolver(p.shape, p.h, "free")
    fields = pcg.fixed_fields(p.eps, p.h, "free")
    vals = []
    for it in range(0, 12):
        res = pcg.pcg_solve(p.rho, p.eps, p.h, "free", tol=0.0, maxit=it, solver=solver,
                            fields=fields)
        vals.append(pcg.discrete_action(res.phi, res.r, p.rho))
    assert all(b < a for a, b in zip(vals, vals[1:]))


def _sphere_continuum_energy(sigma=1.0, q=1.0, d0=3.0, delta=0.5, eps0=W.EPS_WATER):
    # Gauss: phi' = -q_enc/(eps r^2)  =>  E = (1/2) int_0^inf q_enc^2 / (eps r^2) dr
    def qenc(r):
        return q * (erf(r / (math.sqrt(2) * sigma))
                    - math.sqrt(2 / math.pi) * (r / sigma) * math.exp(-r * r / (2 * sigma ** 2)))

    def integrand(r):
        eps = 1 + (eps0 - 1) * 0.5 * (1 + erf((r - d0) / delta))
        return qenc(r) ** 2 / (eps * r * r) if r > 0 else 0.0
    val = sum(integrate.quad(integrand, a, b, limit=200, epsabs=1e-14, epsrel=1e-13)[0]
              for a, b in [(0, 2), (2, 4), (4, 12), (12, np.inf)])
    return 0.5 * val


def test_sphere_in_dielectric_energy_converges_to_gauss_law():
    E = _sphere_continuum_energy()
    Eh = []
    for n, h in [(48, 0.35), (96, 0.175)]:
        p = W.single_sphere(n, h)
        res = pcg.pcg_solve(p.rho, p.eps, p.h, "free", tol=1e-10)
        assert res.converged
        Eh.append(pcg.electrostatic_energy(p.rho, res.phi, p.h))
    e1, e2 = abs(Eh[0] - E), abs(Eh[1] - E)
    assert e1 / E < 2e-2
    assert 3.0 < e1 / e2 < 5.0                      # second order
    assert abs((4 * Eh[1] - Eh[0]) / 3 - E) / E < 1e-3


def test_sphere_iteration_count():
    # the paper reports about ten iterations for smooth cavities (Sec. II.C)
    p = W.single_sphere()
    res = pcg.pcg_solve(p.rho, p.eps, p.h, "free", tol=1e-8)
    assert res.converged and 8 <= res.iterations <= 16


def _screened_gaussian(r, q, sigma, kappa, eps):
    a = math.exp(kappa * kappa * sigma * sigma / 2) / (2 * eps * r)
    s2 = math.sqrt(2) * sigma
    return q * a * (np.exp(-kappa * r) * erfc((kappa * sigma ** 2 - r) / s2)
                    - np.exp(kappa * r) * erfc((kappa * sigma ** 2 + r) / s2))


def test_debye_huckel_limit():
    # uniform eps and kappa2: (eps lap - kappa2) phi = -4 pi rho has the screened
    # Gaussian solution; errors are O(h^2) plus box-edge effects ~ exp(-kappa L/2)
    eps0, lam, sigma = 10.0, 1.5, 1.0
    kappa = 1.0 / lam
    errs = []
    for n, h in [(32, 0.6), (64, 0.3)]:
        shape = (n, n, n)
        rho = W.gaussian_sum(shape, h, [(0, 0, 0)], [sigma], [1.0])
        eps = np.full(shape, eps0)
        kappa2 = np.full(shape, eps0 * kappa * kappa)
        res = pcg.pcg_solve(rho, eps, h, "free", tol=1e-11, kappa2=kappa2)
        x, y, z = W.grid_coords(shape, h)
        r = np.sqrt(x * x + y * y + z * z)
        exact = _screened_gaussian(np.maximum(r, 1e-9), 1.0, sigma, kappa, eps0)
        inner = r < 5.0
        errs.append(np.abs(res.phi - exact)[inner].max() / np.abs(exact).max())
    assert errs[1] < 5e-3
    assert errs[0] / errs[1] > 3.0


def test_debye_huckel_point_limit_and_vacuum_limit():
    # the closed form itself: kappa -> 0 gives erf(r/(sqrt2 sigma))/(eps r),
    # sigma -> 0 gives exp(-kappa r)/(eps r)
    r = np.linspace(0.5, 6, 12)
    v = _screened_gaussian(r, 1.0, 0.7, 1e-7, 3.0)
    assert np.abs(v - erf(r / (math.sqrt(2) * 0.7)) / (3.0 * r)).max() < 1e-6
    v = _screened_gaussian(r, 1.0, 1e-3, 0.8, 3.0)
    assert np.abs(v - np.exp(-0.8 * r) / (3.0 * r)).max() < 1e-5


def test_manufactured_solution_second_order():
    # Sec. II.C test: phi Gaussian, rho from div(eps grad phi); the discrete
    # solution approaches phi as O(h^2) with the cell-averaged kernel
    errs = []
    for n in (40, 80):
        p, phi = W.manufactured_gaussian(n)
        res = pcg.pcg_solve(p.rho, p.eps, p.h, "free", tol=1e-11)
        assert res.converged and res.iterations <= 20
        errs.append(np.abs(res.phi - phi).max() / np.abs(phi).max())
    assert errs[1] < 2e-2
    assert errs[0] / errs[1] > 3.0


# ---- true-residual refinement (sqrt(eps) phi = G s, restart from b - A phi) ----------

@pytest.mark.parametrize("bc", ("free", "surface"))
@pytest.mark.parametrize("ions", [None, "accessibility"])
def test_refined_pcg_equals_dense_direct_solve(bc, ions):
    p = _small_problem(bc)
    kappa2 = None if ions is None else 0.8 * (p.eps - 1.0) / (W.EPS_WATER - 1.0)
    phi_d = dense.dense_solve(p.rho, p.eps, p.h, bc, kappa2=kappa2)
    res = pcg.pcg_solve(p.rho, p.eps, p.h, bc, tol=1e-14, kappa2=kappa2, refine_every=3)
    assert res.converged
    assert np.abs(res.phi - phi_d).max() < 1e-12 * np.abs(phi_d).max()


@pytest.mark.parametrize("bc", ("free", "surface"))
def test_refinement_representation_and_true_residual(bc):
    # At every refinement point, before the restart: the accumulated iterate
    # equals the source representation S^-1 G s, and the residual recomputed
    # from its definition equals the recursively updated one (both FP64, so
    # they differ only by rounding).  A wrong term or sign in either formula
    # would show up as an O(1) mismatch.
    p = _small_problem(bc, 12, 0.5)
    solver = green.VacuumSolver(p.shape, p.h, bc)
    log = []
    res = pcg.pcg_solve(p.rho, p.eps, p.h, bc, tol=1e-12, solver=solver, refine_every=4,
                        refine_log=log)
    assert res.converged and len(log) >= 2
    r0 = 4 * math.pi * np.sqrt(np.sum(p.rho ** 2))
    isq = 1.0 / np.sqrt(p.eps)
    for e in log:
        assert np.abs(e["r_true"] - e["r"]).max() < 1e-10 * r0, e["k"]
        rep = isq * solver.apply(e["src"])
        assert np.abs(rep - e["phi"]).max() < 1e-10 * np.abs(e["phi"]).max(), e["k"]
    plain = pcg.pcg_solve(p.rho, p.eps, p.h, bc, tol=1e-12, solver=solver)
    assert np.abs(res.phi - plain.phi).max() < 1e-9 * np.abs(plain.phi).max()


def test_refinement_rejected_for_periodic():
    p = _small_problem("periodic")
    with pytest.raises(ValueError):
        pcg.pcg_solve(p.rho, p.eps, p.h, "periodic", tol=1e-8, refine_every=4)
