"""GPU parity of Algorithm SC and the PSD minimization (Sec. II.A) through
gps_solve_sc, against the oracle: iterates after a fixed number of steps
(FP64, 1e-10 of max|phi|), converged solutions (iterations within one,
1e-7), mixed precision (1e-5 Ha/e), and the argument checks."""
import numpy as np
import pytest

from oracle import sc
from paper_1509_00680_amd import workloads as W
from paper_1509_00680_amd import gps
from gpu_util import dev, host, empty, plan, require_gpu

pytestmark = pytest.mark.gpu


def _problem(bc):
    return W.molecule(16, 0.5, seed=4, n_atoms=5, ball=1.5, bc=bc)


@pytest.mark.parametrize("bc", ["free", "surface", "wire"])
@pytest.mark.parametrize("method", ["sc", "psd"])
def test_iterates_match_oracle(bc, method):
    require_gpu()
    p = _problem(bc)
    steps = 8
    if method == "sc":
        ref, _, _ = sc.sc_solve(p.rho, p.eps, p.h, bc, 0.6, tol=0.0, maxit=steps)
    else:
        ref, _, _ = sc.psd_solve(p.rho, p.eps, p.h, bc, tol=0.0, maxit=steps)
    pl = plan(p.shape, p.h, bc, "fp64", maxit=steps)
    phi = empty(p.shape)
    print("sc iterates", bc, method, flush=True)
    st = pl.solve_sc(dev(p.rho), dev(p.eps), phi, 1e-30, method=method, eta=0.6)
    assert st == gps.GPS_E_NOT_CONVERGED, gps.STATUS[st]
    assert pl.info()["iterations"] == steps
    assert np.abs(host(phi) - ref).max() <= 1e-10 * np.abs(ref).max()


@pytest.mark.parametrize("bc", ["free", "wire"])
@pytest.mark.parametrize("method", ["sc", "psd"])
def test_converged_solution_matches_oracle(bc, method):
    require_gpu()
    p = _problem(bc)
    if method == "sc":
        ref, it, _ = sc.sc_solve(p.rho, p.eps, p.h, bc, 0.6, tol=1e-9, maxit=2000)
    else:
        ref, it, _ = sc.psd_solve(p.rho, p.eps, p.h, bc, tol=1e-9, maxit=2000)
    pl = plan(p.shape, p.h, bc, "fp64", maxit=2000)
    phi = empty(p.shape)
    print("sc converged", bc, method, flush=True)
    assert pl.solve_sc(dev(p.rho), dev(p.eps), phi, 1e-9, method=method, eta=0.6) == gps.GPS_OK
    assert abs(pl.info()["iterations"] - it) <= 1
    assert np.abs(host(phi) - ref).max() <= 1e-7 * np.abs(ref).max()
    if method == "sc":
        # mixed precision: FP32 vacuum solves
        pm = plan(p.shape, p.h, bc, "mixed", maxit=2000)
        assert pm.solve_sc(dev(p.rho), dev(p.eps), phi, 1e-6, method="sc", eta=0.6) == gps.GPS_OK
        assert np.abs(host(phi) - ref).max() <= 1e-5


def test_sc_arguments_checked():
    require_gpu()
    shape = (8, 8, 8)
    rho, eps, phi = dev(np.zeros(shape)), dev(np.ones(shape)), empty(shape)
    pp = plan(shape, 0.5, "periodic", "fp64")
    assert pp.solve_sc(rho, eps, phi, 1e-6) == gps.GPS_E_INVALID
    pf = plan(shape, 0.5, "free", "fp64")
    assert pf.solve_sc(rho, eps, phi, 1e-6, eta=0.0) == gps.GPS_E_INVALID
    assert pf.solve_sc(rho, eps, phi, 1e-6, eta=1.5) == gps.GPS_E_INVALID
    assert gps.load().gps_solve_sc(pf.handle, None, None, None, 1e-6, 0, 0.5) == gps.GPS_E_INVALID
    assert gps.load().gps_solve_sc(pf.handle, gps._ptr(rho), gps._ptr(eps), gps._ptr(phi),
                                   1e-6, 7, 0.5) == gps.GPS_E_INVALID
    # zero charge: nothing to do
    assert pf.solve_sc(rho, eps, phi, 1e-6) == gps.GPS_OK
    assert pf.info()["iterations"] == 0 and not host(phi).any()
