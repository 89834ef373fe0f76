"""Pins of the oracle's Algorithm SC and PSD minimization (Sec. II.A):
SC equals PSD with the fixed step -eta/(4 pi) iterate by iterate, both reach
the dense solve of the operator they discretize, and constant eps is solved
at once."""
import numpy as np
import pytest

from oracle import green, sc
from paper_1509_00680_amd import workloads as W


def _problem(bc, n=8, h=0.6, seed=2):
    return W.molecule(n, h, seed=seed, n_atoms=4, ball=1.0, bc=bc)


@pytest.mark.parametrize("bc", ["free", "wire"])
@pytest.mark.parametrize("eta", [1.0, 0.6])
def test_sc_equals_psd_with_fixed_step(bc, eta):
    p = _problem(bc, 10, 0.5)
    phis = []
    for k in range(1, 7):
        phi_sc, _, _ = sc.sc_solve(p.rho, p.eps, p.h, bc, eta, tol=0.0, maxit=k)
        phis.append(phi_sc)
    rec = []
    sc.psd_solve(p.rho, p.eps, p.h, bc, tol=0.0, alpha=-eta / (4 * np.pi),
                 alpha_first=-1.0 / (4 * np.pi), maxit=7, record=rec)
    for k in range(6):
        # SC after k + 1 iterations holds phi_{k+1}; PSD after k + 2 steps
        assert np.abs(rec[k + 1] - phis[k]).max() <= 1e-11 * np.abs(phis[k]).max(), k


@pytest.mark.parametrize("bc", ["free", "surface", "wire"])
def test_fixed_points_are_the_dense_solve(bc):
    p = _problem(bc, 6, 0.6)
    a = sc.dense_sc_operator(p.eps, p.h, bc)
    ref = np.linalg.solve(a, -4 * np.pi * p.rho.ravel()).reshape(p.shape)
    phi_sc, it_sc, _ = sc.sc_solve(p.rho, p.eps, p.h, bc, 0.6, tol=1e-13, maxit=2000)
    phi_psd, it_psd, st = sc.psd_solve(p.rho, p.eps, p.h, bc, tol=1e-13, maxit=2000)
    assert st == "ok"
    scale = np.abs(ref).max()
    assert np.abs(phi_sc - ref).max() <= 1e-9 * scale
    assert np.abs(phi_psd - ref).max() <= 1e-9 * scale


def test_constant_eps_one_step():
    p = _problem("free", 8, 0.5)
    eps = np.full(p.shape, 7.0)
    u = green.VacuumSolver(p.shape, p.h, "free").apply(p.rho) / 7.0
    phi, it, _ = sc.sc_solve(p.rho, eps, p.h, "free", 0.6, tol=1e-12)
    assert it == 1 and np.abs(phi - u).max() <= 1e-13 * np.abs(u).max()
    phi, it, st = sc.psd_solve(p.rho, eps, p.h, "free", tol=1e-12)
    assert st == "ok" and it == 1 and np.abs(phi - u).max() <= 1e-12 * np.abs(u).max()
