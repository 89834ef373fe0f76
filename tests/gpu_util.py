"""Helpers of the GPU tests: device transfer and library access."""
import numpy as np


def require_gpu():
    import torch
    assert torch.cuda.is_available(), "these tests need an MI355X GPU (HIP device not found)"
    return torch


def dev(a):
    torch = require_gpu()
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to("cuda")


def host(t):
    return t.detach().cpu().numpy()


def empty(shape):
    torch = require_gpu()
    return torch.empty(shape, dtype=torch.float64, device="cuda")


def plan(shape, h, bc, precision="fp64", **kw):
    from paper_1509_00680_amd import gps
    return gps.Plan(shape, h, bc, precision=precision, **kw)


def oracle_ions(d):
    from oracle import pb
    return pb.Electrolyte(d["Z"], d["c_bulk"], d["kT"], c_max=d.get("c_max"),
                          eps_bulk=d.get("eps_bulk", 78.36))
