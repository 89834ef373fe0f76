"""Pins of the oracle's Poisson-Boltzmann pieces (Sec. III): ionic charge of
Eqs. ionsconcPB/ionsconcMPB/maxconc and Algorithms SCPB / SCPBimproved."""
import math

import numpy as np
import pytest

from oracle import pcg, pb, dense
from paper_1509_00680_amd import workloads as W

KT = W.KT_ROOM


def _ions(c=1e-4, c_max=None, gamma=None):
    return pb.Electrolyte([1.0, -1.0], [c, c], KT,
                          c_max=None if c_max is None else [c_max, c_max], gamma=gamma)


def test_boltzmann_1to1_is_sinh():
    phi = np.linspace(-0.02, 0.02, 41)
    g = np.linspace(0.0, 1.0, 41)
    got = pb.ionic_charge(phi, _ions(), g)
    assert np.allclose(got, -2e-4 * g * np.sinh(phi / KT), rtol=1e-13, atol=0)


def test_mpb_1to1_closed_form():
    # 1:1 steric: rho = -2 c gamma sinh(x) / (1 - 2a + 2a cosh x), x = phi/kT
    cmax = 9.7e-4
    a = 1e-4 / cmax
    phi = np.linspace(-0.05, 0.05, 101)
    x = phi / KT
    expect = -2e-4 * np.sinh(x) / (1 - 2 * a + 2 * a * np.cosh(x))
    got = pb.ionic_charge(phi, _ions(c_max=cmax), 1.0)
    assert np.allclose(got, expect, rtol=1e-12, atol=0)


def test_mpb_tends_to_boltzmann_and_saturates():
    phi = np.linspace(-0.01, 0.01, 21)
    big = pb.ionic_charge(phi, _ions(c_max=1e30), 1.0)
    assert np.allclose(big, pb.ionic_charge(phi, _ions(), 1.0), rtol=1e-12)
    cmax = 9.7e-4
    sat = pb.ionic_charge(np.array([-5.0, 5.0]), _ions(c_max=cmax), 1.0)
    assert np.allclose(sat, [cmax, -cmax], rtol=1e-12)      # no overflow, capped
    assert np.all(np.isfinite(pb.ionic_charge(np.array([-1e3, 1e3]), _ions(c_max=cmax), 1.0)))


def test_mpb_bulk_limit_single_species():
    # reading of Eq. ionsconcMPB: c_i(phi = 0) = c_i^inf (with "-1" in the bracket)
    ions = pb.Electrolyte([2.0], [3e-4], KT, c_max=[1e-3])
    assert abs(pb.ionic_charge(np.zeros(1), ions, 1.0)[0] - 2.0 * 3e-4) < 1e-18


def test_maxconc_paper_values():
    # Sec. III.A: p = 0.74, R = 3 Angstrom
    cm = pb.max_concentration(0.74, 3.0 * W.ANGSTROM_BOHR)
    assert abs(cm - W.steric_cmax()) < 1e-18
    mol = cm / W.MOLAR_BOHR3
    assert 10.8 < mol < 10.9          # about 10.9 mol/L for 3 Angstrom spheres


def _pb_problem(n=24, h=0.5, seed=6, net=2.0, scale=1.0):
    p = W.molecule(n, h, seed=seed, n_atoms=6, ball=2.0, net_charge=net)
    return p.rho * scale, p.eps, p.h


def test_linear_and_nonlinear_agree_for_weak_charge():
    rho, eps, h = _pb_problem(scale=1e-5)
    ions = _ions(c=W.MOLAR_BOHR3 * 0.1)
    lin = pb.solve_linear_pb(rho, eps, h, "free", ions, 1e-12)
    nl = pb.scpb_improved(rho, eps, h, "free", ions, 1e-10, eta=0.6)
    assert nl.converged
    assert np.abs(lin.phi).max() / KT < 0.05
    assert np.abs(nl.phi - lin.phi).max() < 2e-3 * np.abs(lin.phi).max()


def test_scpb_and_improved_share_fixed_point():
    rho, eps, h = _pb_problem()
    ions = _ions(c=W.MOLAR_BOHR3 * 0.1, c_max=W.steric_cmax())
    a3 = pb.scpb(rho, eps, h, "free", ions, 1e-9, eta=0.3)
    a4 = pb.scpb_improved(rho, eps, h, "free", ions, 1e-9, eta=0.3)
    assert a3.converged and a4.converged
    assert np.abs(a3.phi - a4.phi).max() < 1e-6 * np.abs(a3.phi).max()
    assert sum(a4.inner_iterations) < sum(a3.inner_iterations)


def test_improved_invariant_with_dense_operator():
    # after every outer step A phi = -4 pi (rho + rho_ion_used - r'), no
    # residual is lost; checked with the dense operator assembled independently
    rho, eps, h = _pb_problem(n=8, h=0.6, seed=2)
    ions = _ions(c=W.MOLAR_BOHR3 * 0.1, c_max=W.steric_cmax())
    a = dense.dense_operator(eps, h, "free")
    for steps in (1, 2, 3, 5):
        res = pb.scpb_improved(rho, eps, h, "free", ions, 1e-30, eta=0.3, outer_maxit=steps)
        lhs = (a @ res.phi.ravel()).reshape(rho.shape)
        rhs = -4 * math.pi * (rho + res.rho_ion_used - res.rprime)
        assert np.abs(lhs - rhs).max() < 1e-10 * np.abs(rhs).max()
    # the converged solution solves the nonlinear equation itself
    res = pb.scpb_improved(rho, eps, h, "free", ions, 1e-12, eta=0.3)
    assert res.converged
    rhs = -4 * math.pi * (rho + pb.ionic_charge(res.phi, ions, ions.accessibility(eps)))
    lhs = (a @ res.phi.ravel()).reshape(rho.shape)
    assert np.abs(lhs - rhs).max() < 1e-8 * np.abs(rhs).max()


def test_nonlinear_pb_outer_convergence_mpb():
    # reduced charged-solute case, steric ions, eta = 0.3: converges in tens of steps
    p = W.charged_solute_mpb(n=32, h=0.5, n_atoms=12, ball=3.0, net_charge=2.0)
    io = p.ions
    ions = pb.Electrolyte(io["Z"], io["c_bulk"], io["kT"], c_max=io["c_max"])
    res = pb.scpb_improved(p.rho, p.eps, p.h, "free", ions, 1e-8, eta=0.3)
    assert res.converged and res.outer < 60
    # late inner solves are cheap (warm start through the carried residual)
    assert res.inner_iterations[-1] <= max(res.inner_iterations[:3])
