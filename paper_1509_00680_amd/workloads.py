"""Seeded synthetic inputs: charge densities and dielectric cavities.

This module builds the solver's INPUTS only (rho, eps, electrolyte
parameters, request streams).  It contains none of the solver's arithmetic
and is shared by the tests, the benchmark and the serving harness; both the
GPU library and the CPU oracle receive exactly the arrays it returns.

Conventions: Hartree atomic units (bohr, Ha, e); arrays of shape (nz, ny, nx),
x fastest; cell-centred grid, point (i, j, k) at ((i-(nx-1)/2) h, ...), i.e.
the box is symmetric about the origin.

Dielectric cavities follow the paper's definitions:
  * erf switch h(d0, Delta; r) = (1 + erf((r - d0)/Delta))/2   (Eq. hfunc),
    eps = 1 + (eps0 - 1) h(d0, Delta; r) for a sphere (Sec. II.C), the same
    in |z| for a slab;
  * density-dependent cavity (Eq. sccs): eps = 1 above rho_max, eps0 below
    rho_min and eps0 ** w(rho) in between, with
    w = (zeta - sin zeta)/(2 pi), zeta = 2 pi ln(rho_max/rho)/ln(rho_max/rho_min).
    The printed "eps0 e^{w}" cannot be continuous with eps = 1 at rho_max; the
    continuous reading exp(ln(eps0) w) is used.
The cavity density of a synthetic solute is the sum of unit-weight atomic
Gaussians (independent of the atomic charges).
"""
import math

import numpy as np
from scipy.special import erf

EPS_WATER = 78.36                 # Sec. IV.C
KB_HARTREE_PER_K = 3.166811563e-6
T_ROOM = 298.15
KT_ROOM = KB_HARTREE_PER_K * T_ROOM
BOHR_M = 5.29177210903e-11
AVOGADRO = 6.02214076e23
ANGSTROM_BOHR = 1e-10 / BOHR_M
MOLAR_BOHR3 = AVOGADRO * 1e3 * BOHR_M ** 3        # 1 mol/L in bohr^-3
RHO_MAX_SCCS = 5e-3                                # Sec. IV.C
RHO_MIN_SCCS = 1e-4

BC_FREE, BC_SURFACE, BC_PERIODIC, BC_WIRE = "free", "surface", "periodic", "wire"


# --------------------------------------------------------------------------
# grids and fields
# --------------------------------------------------------------------------
def axis_coords(n, h):
    return (np.arange(n) - (n - 1) / 2.0) * h


def grid_coords(shape, h):
    nz, ny, nx = shape
    return (axis_coords(nx, h)[None, None, :], axis_coords(ny, h)[None, :, None],
            axis_coords(nz, h)[:, None, None])


def periodic_flags(bc):
    """(x, y, z) periodicity of a boundary condition."""
    return {BC_FREE: (False, False, False), BC_SURFACE: (True, True, False),
            BC_PERIODIC: (True, True, True), BC_WIRE: (False, False, True)}[bc]


def _min_image(d, length, periodic):
    if periodic:
        return d - length * np.round(d / length)
    return d


def gaussian_sum(shape, h, centres, sigmas, weights, bc=BC_FREE, discrete_norm=False):
    """sum_i w_i (2 pi s_i^2)^-3/2 exp(-|r - c_i|^2 / (2 s_i^2)).

    Minimum image along periodic axes.  With discrete_norm each Gaussian is
    rescaled so that h^3 * (its grid sum) equals w_i exactly, which makes a
    set of charges with sum(w) = 0 exactly neutral on the grid.
    """
    nz, ny, nx = shape
    x, y, z = grid_coords(shape, h)
    px, py, pz = periodic_flags(bc)
    out = np.zeros(shape)
    for c, s, w in zip(np.asarray(centres), np.asarray(sigmas), np.asarray(weights)):
        dx = _min_image(x - c[0], nx * h, px)
        dy = _min_image(y - c[1], ny * h, py)
        dz = _min_image(z - c[2], nz * h, pz)
        e = (np.exp(-dx * dx / (2 * s * s)) * np.exp(-dy * dy / (2 * s * s))
             * np.exp(-dz * dz / (2 * s * s)))
        if discrete_norm:
            g = e / (h ** 3 * e.sum())
        else:
            g = e * (2 * np.pi * s * s) ** -1.5
        out += w * g
    return out


def erf_switch(r, d0, delta):
    """h(d0, Delta; r) of Eq. hfunc."""
    return 0.5 * (1.0 + erf((r - d0) / delta))


def sphere_cavity(shape, h, d0, delta, eps0=EPS_WATER, centre=(0.0, 0.0, 0.0)):
    x, y, z = grid_coords(shape, h)
    r = np.sqrt((x - centre[0]) ** 2 + (y - centre[1]) ** 2 + (z - centre[2]) ** 2)
    return 1.0 + (eps0 - 1.0) * erf_switch(r, d0, delta)


def slab_cavity(shape, h, d0, delta, eps0=EPS_WATER):
    _, _, z = grid_coords(shape, h)
    e = 1.0 + (eps0 - 1.0) * erf_switch(np.abs(z), d0, delta)
    return np.broadcast_to(e, shape).copy()


def sccs_eps(rho_elec, rho_max=RHO_MAX_SCCS, rho_min=RHO_MIN_SCCS, eps0=EPS_WATER):
    """Density-dependent cavity (Eq. sccs, continuous reading)."""
    rho = np.asarray(rho_elec, dtype=np.float64)
    out = np.full(rho.shape, eps0)
    out[rho > rho_max] = 1.0
    mid = (rho <= rho_max) & (rho >= rho_min)
    zeta = 2 * np.pi * np.log(rho_max / rho[mid]) / np.log(rho_max / rho_min)
    w = (zeta - np.sin(zeta)) / (2 * np.pi)
    out[mid] = np.exp(np.log(eps0) * w)
    return out


# --------------------------------------------------------------------------
# solutes and workload recipes
# --------------------------------------------------------------------------
def random_solute(rng, n_atoms, ball_radius, net_charge=0.0):
    """Draw order: sigma, q, direction, radius (all from rng)."""
    sig = rng.uniform(0.6, 1.2, n_atoms)
    q = rng.uniform(-1.0, 1.0, n_atoms)
    q = q - q.mean() + net_charge / n_atoms
    d = rng.normal(size=(n_atoms, 3))
    d /= np.linalg.norm(d, axis=1)[:, None]
    rad = ball_radius * rng.uniform(size=n_atoms) ** (1.0 / 3.0)
    return d * rad[:, None], sig, q


class Problem:
    """One solve: rho, eps and what the solver needs besides them."""

    def __init__(self, name, shape, h, bc, rho, eps, tol, ions=None, kind="gpe",
                 meta=None):
        self.name = name
        self.shape = tuple(shape)
        self.h = float(h)
        self.bc = bc
        self.rho = np.ascontiguousarray(rho, dtype=np.float64)
        self.eps = np.ascontiguousarray(eps, dtype=np.float64)
        self.tol = tol
        self.ions = ions          # dict or None
        self.kind = kind          # "gpe" | "pb_linear" | "pb_nonlinear"
        self.meta = meta or {}

    @property
    def npoints(self):
        return int(np.prod(self.shape))


def electrolyte_1to1(conc_bohr3, kT=KT_ROOM, c_max=None, eps_bulk=EPS_WATER,
                     linear=False, eta=0.3, outer_maxit=100):
    return {"Z": [1.0, -1.0], "c_bulk": [conc_bohr3, conc_bohr3],
            "c_max": None if c_max is None else [c_max, c_max], "kT": kT,
            "eps_bulk": eps_bulk, "linear": linear, "eta": eta,
            "outer_maxit": outer_maxit}


def debye_concentration(debye_length, eps_bulk=EPS_WATER, kT=KT_ROOM):
    """1:1 concentration whose bulk Debye length is debye_length (bohr):
    (4 pi / kT) 2 c = eps_bulk / lambda^2."""
    return eps_bulk * kT / (8 * np.pi * debye_length ** 2)


def steric_cmax(packing=0.74, radius_angstrom=3.0):
    """Eq. maxconc, c_max = p / (4/3 pi R^3), in bohr^-3 (Sec. III.A values)."""
    r = radius_angstrom * ANGSTROM_BOHR
    return packing / (4.0 / 3.0 * np.pi * r ** 3)


def single_sphere(n=48, h=0.35, sigma=1.0, q=1.0, d0=3.0, delta=0.5, eps0=EPS_WATER,
                  tol=1e-8):
    """One Gaussian charge in a spherical erf cavity at the box centre."""
    shape = (n, n, n)
    rho = gaussian_sum(shape, h, [(0.0, 0.0, 0.0)], [sigma], [q])
    eps = sphere_cavity(shape, h, d0, delta, eps0)
    return Problem("sphere%d" % n, shape, h, BC_FREE, rho, eps, tol,
                   meta={"sigma": sigma, "q": q, "d0": d0, "delta": delta, "eps0": eps0})


def molecule(n=96, h=0.3, seed=2, n_atoms=24, ball=6.0, net_charge=0.0, tol=1e-6,
             bc=BC_FREE, eps0=EPS_WATER):
    """Molecule-like solute in a density-dependent (sccs) cavity."""
    rng = np.random.default_rng(seed)
    centres, sig, q = random_solute(rng, n_atoms, ball, net_charge)
    shape = (n, n, n)
    periodic = bc != BC_FREE
    rho = gaussian_sum(shape, h, centres, sig, q, bc=bc, discrete_norm=periodic)
    cav = gaussian_sum(shape, h, centres, sig, np.ones(n_atoms), bc=bc)
    eps = sccs_eps(cav, eps0=eps0)
    return Problem("molecule%d_s%d" % (n, seed), shape, h, bc, rho, eps, tol,
                   meta={"seed": seed, "n_atoms": n_atoms, "net_charge": net_charge})


def rigid_solute(n=48, h=0.35, seed=6, n_atoms=6, ball=2.0, radii=(2.2, 2.8), delta=0.4,
                 eps0=EPS_WATER, net_charge=0.0, bc=BC_FREE, shape=None):
    """Inputs of a rigid-cavity solve (Eq. RigCav): the atom table
    (natoms x 4: X, Y, Z, cavity radius d_i), Delta, eps0 and the solute's
    Gaussian charge.  The cavity itself is left to the solver."""
    rng = np.random.default_rng(seed)
    centres, sig, q = random_solute(rng, n_atoms, ball, net_charge)
    d = rng.uniform(radii[0], radii[1], n_atoms)
    shape = tuple(shape) if shape is not None else (n, n, n)
    rho = gaussian_sum(shape, h, centres, sig, q, bc=bc, discrete_norm=bc != BC_FREE)
    atoms = np.concatenate([np.asarray(centres), d[:, None]], axis=1)
    return {"shape": shape, "h": h, "bc": bc, "rho": rho, "atoms": atoms, "delta": delta,
            "eps0": eps0, "name": "rigid%d_s%d" % (shape[0], seed)}


def charged_solute_mpb(n=160, h=0.3, seed=4, n_atoms=48, ball=6.0, net_charge=4.0,
                       molar=1.0, eta=0.15, tol=1e-6, steric=True, outer_maxit=200):
    """Nonlinear PB: charged solute, 1:1 electrolyte, accessibility from eps.

    eta = 0.15: in this 48-bohr box at 1 M the plain linear mixing of the
    self-consistent loop settles into a non-contracting cycle for eta >= 0.2
    (the screening response of the box-scale mode is about -10); 0.15
    converges in about 50 outer steps."""
    p = molecule(n, h, seed, n_atoms, ball, net_charge, tol)
    c = molar * MOLAR_BOHR3
    ions = electrolyte_1to1(c, c_max=steric_cmax() if steric else None, eta=eta,
                            outer_maxit=outer_maxit)
    return Problem("mpb%d_s%d" % (n, seed), p.shape, h, BC_FREE, p.rho, p.eps, tol,
                   ions=ions, kind="pb_nonlinear", meta=p.meta)


def slab(nxy=128, nz=192, h=0.3, seed=3, n_atoms=64, half_width=4.0, debye=10.0,
         tol=1e-6, eps0=EPS_WATER):
    """Surface BC: charges in a slab |z| < 4 with eps = 1 inside; linear PB."""
    rng = np.random.default_rng(seed)
    sig = rng.uniform(0.6, 1.2, n_atoms)
    q = rng.uniform(-1.0, 1.0, n_atoms)
    q = q - q.mean()
    L = nxy * h
    xy = rng.uniform(-L / 2, L / 2, size=(n_atoms, 2))
    z = rng.uniform(-half_width, half_width, size=n_atoms)
    centres = np.column_stack([xy, z])
    shape = (nz, nxy, nxy)
    rho = gaussian_sum(shape, h, centres, sig, q, bc=BC_SURFACE, discrete_norm=True)
    eps = slab_cavity(shape, h, half_width, 0.5, eps0)
    ions = electrolyte_1to1(debye_concentration(debye, eps0), linear=True)
    return Problem("slab%dx%d_s%d" % (nxy, nz, seed), shape, h, BC_SURFACE, rho, eps,
                   tol, ions=ions, kind="pb_linear", meta={"seed": seed})


def manufactured_gaussian(n, box=10.0, sigma=0.5, d0=1.7, delta=0.3, eps0=EPS_WATER,
                          bc=BC_FREE):
    """Sec. II.C test: normalized Gaussian phi, erf cavity, rho from the operator.

    rho = -(1/4 pi) div(eps grad phi), evaluated analytically in the radial
    variable: eps (phi'' + 2 phi'/r) + eps' phi'.
    Returns (Problem, phi_exact).
    """
    h = box / n
    shape = (n, n, n)
    x, y, z = grid_coords(shape, h)
    r = np.sqrt(x * x + y * y + z * z)
    s2 = sigma * sigma
    phi = (2 * np.pi * s2) ** -1.5 * np.exp(-r * r / (2 * s2))
    dphi_over_r = -phi / s2                      # phi'/r
    d2phi = (r * r / (s2 * s2) - 1.0 / s2) * phi
    eps = 1.0 + (eps0 - 1.0) * erf_switch(r, d0, delta)
    deps = (eps0 - 1.0) / (delta * np.sqrt(np.pi)) * np.exp(-((r - d0) / delta) ** 2)
    lap = d2phi + 2.0 * dphi_over_r
    rho = -(eps * lap + deps * dphi_over_r * r) / (4 * np.pi)
    return Problem("manufactured%d" % n, shape, h, bc, rho, eps, 1e-10), phi


# --------------------------------------------------------------------------
# serving stream
# --------------------------------------------------------------------------
SERVING_GRIDS = (32, 48, 64, 96, 128)
SERVING_BOX = 19.2


def serving_params(rng, grids=SERVING_GRIDS, box=SERVING_BOX, tol=1e-6):
    """Draws one request's parameters: grid, BC, kind, solute (in this order)."""
    n = int(rng.choice(grids))
    bc = (BC_FREE, BC_SURFACE, BC_PERIODIC)[int(rng.integers(3))]
    n_atoms = int(rng.integers(4, 49))
    kind = ("gpe", "pb_linear")[int(rng.integers(2))]
    centres, sig, q = random_solute(rng, n_atoms, 3.0, 0.0)
    ions = electrolyte_1to1(debye_concentration(10.0), linear=True) if kind == "pb_linear" else None
    return {"n": n, "h": box / n, "bc": bc, "kind": kind, "n_atoms": n_atoms,
            "centres": centres, "sigmas": sig, "charges": q, "ions": ions, "tol": tol}


def serving_request(rng, grids=SERVING_GRIDS, box=SERVING_BOX, tol=1e-6):
    """One request: grid, BC, solute and kind drawn from rng."""
    return request_problem(serving_params(rng, grids, box, tol))


def request_problem(prm):
    """Fields of a request on the host (numpy)."""
    n, h, bc = prm["n"], prm["h"], prm["bc"]
    shape = (n, n, n)
    rho = gaussian_sum(shape, h, prm["centres"], prm["sigmas"], prm["charges"], bc=bc,
                       discrete_norm=True)
    cav = gaussian_sum(shape, h, prm["centres"], prm["sigmas"], np.ones(prm["n_atoms"]), bc=bc)
    eps = sccs_eps(cav)
    return Problem("req_n%d_%s_%s" % (n, bc, prm["kind"]), shape, h, bc, rho, eps, prm["tol"],
                   ions=prm["ions"], kind=prm["kind"], meta={"n_atoms": prm["n_atoms"]})


def request_fields_torch(prm, device):
    """(rho, eps) of a request as float64 torch tensors on `device`: the same
    recipe as request_problem, evaluated by torch (for large request streams)."""
    import torch
    n, h, bc = prm["n"], prm["h"], prm["bc"]
    ax = (torch.arange(n, dtype=torch.float64, device=device) - (n - 1) / 2.0) * h
    px, py, pz = periodic_flags(bc)
    length = n * h

    def mi(d, periodic):
        return d - length * torch.round(d / length) if periodic else d

    rho = torch.zeros((n, n, n), dtype=torch.float64, device=device)
    cav = torch.zeros_like(rho)
    for c, s, w in zip(prm["centres"], prm["sigmas"], prm["charges"]):
        k = 1.0 / (2.0 * s * s)
        ex = torch.exp(-mi(ax - c[0], px) ** 2 * k)
        ey = torch.exp(-mi(ax - c[1], py) ** 2 * k)
        ez = torch.exp(-mi(ax - c[2], pz) ** 2 * k)
        e = ez[:, None, None] * ey[None, :, None] * ex[None, None, :]
        rho += (w / (h ** 3 * e.sum())) * e
        cav += (2 * math.pi * s * s) ** -1.5 * e
    eps = torch.full_like(cav, EPS_WATER)
    eps[cav > RHO_MAX_SCCS] = 1.0
    mid = (cav <= RHO_MAX_SCCS) & (cav >= RHO_MIN_SCCS)
    zeta = 2 * math.pi * torch.log(RHO_MAX_SCCS / cav[mid]) / math.log(RHO_MAX_SCCS / RHO_MIN_SCCS)
    w = (zeta - torch.sin(zeta)) / (2 * math.pi)
    eps[mid] = torch.exp(math.log(EPS_WATER) * w)
    return rho, eps


def serving_stream(n_requests=512, seed=5, rate=None, **kw):
    """Requests with exponential inter-arrival times (Poisson process)."""
    rng = np.random.default_rng(seed)
    reqs = [serving_request(rng, **kw) for _ in range(n_requests)]
    gaps = rng.exponential(1.0, n_requests)
    if rate is not None:
        gaps = gaps / rate
    return reqs, np.cumsum(gaps)


def serving_stream_params(n_requests=512, seed=5, **kw):
    """Parameters of the same stream as serving_stream (no fields) and the
    unit-rate inter-arrival gaps (divide by the rate)."""
    rng = np.random.default_rng(seed)
    prms = [serving_params(rng, **kw) for _ in range(n_requests)]
    return prms, rng.exponential(1.0, n_requests)
