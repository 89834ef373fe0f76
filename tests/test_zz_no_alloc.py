"""gps_polarization_charge_noalloc (the entry point for callers that cannot
allocate) against gps_polarization_charge through the C ABI: identical bits
on two calls in a row, the second on a smaller grid, and the size limit."""
import numpy as np
import pytest

from paper_1509_00680_amd import gps
from paper_1509_00680_amd import workloads as W
from gpu_util import dev, host, empty, plan, require_gpu

pytestmark = pytest.mark.gpu


def _fields(n, bc, seed):
    p = W.molecule(n, 0.5, seed=seed, n_atoms=6, ball=2.0, bc=bc)
    rng = np.random.default_rng(seed)
    phi = rng.normal(size=p.shape) * 0.1
    return p, phi


def test_noalloc_equals_allocating_entry_point():
    require_gpu()
    # two calls in a row on one GPU; the second grid is smaller, so its call
    # finds the first call's values in the scratch array beyond its own range
    for n, bc, order in ((40, "free", 16), (24, "surface", 6)):
        p, phi = _fields(n, bc, seed=n)
        pl = plan(p.shape, p.h, bc, "fp64", fd_order=order)
        rho, eps, ph = dev(p.rho), dev(p.eps), dev(phi)
        ref, got = empty(p.shape), empty(p.shape)
        print("noalloc", n, bc, order, flush=True)
        assert pl.polarization_charge(rho, eps, ph, ref) == gps.GPS_OK
        assert pl.polarization_charge_noalloc(rho, eps, ph, got) == gps.GPS_OK
        a, b = host(ref), host(got)
        assert np.isfinite(a).all()
        assert np.array_equal(a, b), np.abs(a - b).max()
        pl.close()


def test_noalloc_rejects_grids_beyond_its_scratch():
    require_gpu()
    shape = (256, 128, 140)                    # 4,587,520 points > 4,194,304
    assert shape[0] * shape[1] * shape[2] > gps.NOALLOC_MAX_POINTS
    pl = plan(shape, 0.3, "free", "fp64")
    f = empty(shape)
    print("noalloc limit", flush=True)
    assert pl.polarization_charge_noalloc(f, f, f, f) == gps.GPS_E_INVALID
    pl.close()
