"""Algorithm PCG of Sec. II.B in plain binary64 (test infrastructure only).

Discrete problem.  The paper's PCG never applies a finite-difference form of
div(eps grad).  With the preconditioner of Eq. PCGdef,
    P v = sqrt(eps) lap (sqrt(eps) v) = -4 pi r   =>   v = S^-1 G S^-1 r,
where S = diag(sqrt(eps)) and G is the vacuum Poisson solver, Eq. corr gives
the operator on v without differentiating:  A v = -q v - 4 pi r.  For linear
Poisson-Boltzmann (Eq. corrPB) q is replaced by q + kappa2 with
kappa2 = (4 pi / kT) sum_i Z_i^2 c_i gamma.  The discrete operator solved is
therefore the one implied by the vacuum solver,
    A = S L_G S - diag(q + kappa2),   L_G = -4 pi G^-1 .

Periodic boundaries: the spectral Laplacian annihilates constants, so
whatever G does with the k = 0 component, lap(sqrt(eps) v) equals
-4 pi (r/sqrt(eps) - mean(r/sqrt(eps))) and the exact form of Eq. corr is
A v = -(q + kappa2) v - 4 pi (r - sqrt(eps) mean(r/sqrt(eps))).  For free and
surface boundaries G is invertible and the mean term is absent.  Without ions
the periodic G drops k = 0 (the iterates then satisfy sum sqrt(eps) phi = 0,
which fixes the free constant); with ions it uses 4 pi / mean(kappa2/eps).

Steps per iteration k (Algorithm PCG):
    v_k   = S^-1 G S^-1 r_k
    delta = (v_k, r_k);  beta = delta / delta_prev  (beta = 0 at k = 0)
    p_k   = v_k + beta p_{k-1}
    A p_k = A v_k + beta A p_{k-1}          (A v_k from Eq. corr)
    alpha = delta / (p_k, A p_k)
    phi  += alpha p_k ;   r -= alpha A p_k
Inner products are plain sums over grid points (the h^3 weight cancels in
alpha and beta).  A is negative definite, so delta > 0 and (p, Ap) < 0 (alpha
< 0); a violation is reported as a breakdown.  The solve starts from phi = 0,
r_0 = -4 pi rho and stops when ||r_k||_2 <= threshold, with threshold
tol * ||r_0||_2 (relative) or an absolute value.
"""
import numpy as np

from . import BC_PERIODIC
from .green import VacuumSolver
from .stencil import q_field

FOUR_PI = 4.0 * np.pi

STATUS_OK = "ok"
STATUS_NOT_CONVERGED = "not_converged"
STATUS_BREAKDOWN = "breakdown"
STATUS_NONFINITE = "nonfinite"


class PCGResult:
    def __init__(self, phi, r, iterations, status, history, rnorm0):
        self.phi = phi
        self.r = r
        self.iterations = iterations
        self.status = status
        self.history = history
        self.rnorm0 = rnorm0

    @property
    def converged(self):
        return self.status == STATUS_OK

    @property
    def rel_residual(self):
        if self.rnorm0 == 0.0:
            return 0.0
        return float(np.sqrt(np.sum(self.r * self.r)) / self.rnorm0)


def fixed_fields(eps, h, bc, fd_order=16, kappa2=None):
    """sqrt(eps), 1/sqrt(eps) and q + kappa2, computed once per dielectric."""
    eps = np.asarray(eps, dtype=np.float64)
    s = np.sqrt(eps)
    qk = q_field(eps, h, bc, fd_order)
    if kappa2 is not None:
        qk = qk + kappa2
    return s, 1.0 / s, qk


def periodic_k0_value(eps, kappa2):
    """k = 0 multiplier of the periodic preconditioner: 0 without ions (the
    singular Poisson case), else 4 pi / mean(kappa2 / eps)."""
    if kappa2 is None:
        return 0.0
    m = float(np.mean(np.broadcast_to(kappa2, np.shape(eps)) / np.asarray(eps)))
    return 0.0 if m == 0.0 else 4.0 * np.pi / m


def pcg_solve(rho, eps, h, bc, *, tol=None, abs_threshold=None, kappa2=None,
              solver=None, fd_order=16, maxit=1000, fields=None,
              surface_k0_offset=None, refine_every=None, refine_log=None):
    """Solve -div(eps grad phi) + kappa2 phi = 4 pi rho (A phi = -4 pi rho).

    refine_every = m (free and surface boundaries): true-residual refinement.
    Every direction is the preconditioner image of a source,
        p_k = S^-1 G sigma_k,   sigma_k = S^-1 r_k + beta_k sigma_{k-1},
    so the iterate keeps the representation sqrt(eps) phi = G s with
    s = sum_k alpha_k sigma_k.  Every m iterations phi is recomputed as
    S^-1 G s and the residual from its definition b - A phi, which with
    A = S L_G S - diag(q + kappa2), L_G G = -4 pi I and b = -4 pi rho is
        r = -4 pi rho + 4 pi sqrt(eps) s + (q + kappa2) phi ;
    PCG then restarts from that residual with beta = 0.  On exit phi is
    recomputed from s.  refine_log (a list) receives, at each refinement,
    the recursive residual, the recomputed one, the accumulated phi and s.
    """
    rho = np.asarray(rho, dtype=np.float64)
    shape = rho.shape
    if solver is None:
        solver = VacuumSolver(shape, h, bc, surface_k0_offset=surface_k0_offset)
    if fields is None:
        fields = fixed_fields(eps, h, bc, fd_order, kappa2)
    s, isq, qk = fields
    periodic = bc == BC_PERIODIC
    k0 = periodic_k0_value(eps, kappa2) if periodic else None

    r = -FOUR_PI * rho
    phi = np.zeros(shape)
    p = np.zeros(shape)
    ap = np.zeros(shape)
    rnorm0 = float(np.sqrt(np.sum(r * r)))
    if abs_threshold is not None:
        threshold = float(abs_threshold)
    else:
        threshold = float(tol) * rnorm0
    history = []
    delta_prev = None
    status = STATUS_NOT_CONVERGED
    k = 0
    rnorm = rnorm0
    refine = refine_every is not None and refine_every > 0
    if refine and periodic:
        raise ValueError("refinement needs an invertible vacuum solver (free or surface)")
    sig = np.zeros(shape)
    src = np.zeros(shape)
    while True:
        if not np.isfinite(rnorm):
            status = STATUS_NONFINITE
            break
        if rnorm <= threshold:
            status = STATUS_OK
            break
        if k >= maxit:
            status = STATUS_NOT_CONVERGED
            break
        # preconditioner, Eq. PCGdef
        v = isq * solver.apply(isq * r, periodic_k0=k0)
        delta = float(np.sum(v * r))
        if not delta > 0.0:
            status = STATUS_BREAKDOWN if np.isfinite(delta) else STATUS_NONFINITE
            break
        beta = 0.0 if delta_prev is None else delta / delta_prev
        p = v + beta * p
        if refine:
            sig = isq * r + beta * sig
        # operator on v without derivatives, Eq. corr / Eq. corrPB
        if periodic:
            mu = float(np.mean(isq * r))
            av = -qk * v - FOUR_PI * (r - s * mu)
        else:
            av = -qk * v - FOUR_PI * r
        ap = av + beta * ap
        pap = float(np.sum(p * ap))
        if not pap < 0.0:
            status = STATUS_BREAKDOWN if np.isfinite(pap) else STATUS_NONFINITE
            break
        alpha = delta / pap
        phi = phi + alpha * p
        r = r - alpha * ap
        if refine:
            src = src + alpha * sig
        delta_prev = delta
        k += 1
        if refine and k % refine_every == 0:
            phi_s = isq * solver.apply(src)
            r_true = -FOUR_PI * rho + FOUR_PI * s * src + qk * phi_s
            if refine_log is not None:
                refine_log.append({"k": k, "r": r, "r_true": r_true, "phi": phi, "src": src})
            phi, r = phi_s, r_true
            delta_prev = None                  # restart: beta = 0 next
            p = np.zeros(shape)
            ap = np.zeros(shape)
        rnorm = float(np.sqrt(np.sum(r * r)))
        history.append({"delta": delta, "beta": beta, "pAp": pap, "alpha": alpha,
                        "rnorm": rnorm})
    if refine:
        phi = isq * solver.apply(src)
    return PCGResult(phi, r, k, status, history, rnorm0)


def electrostatic_energy(rho, phi, h):
    """E = (1/2) h^3 sum rho phi  (Sec. IV.B, energy of the solute charge)."""
    return 0.5 * h ** 3 * float(np.sum(np.asarray(rho) * np.asarray(phi)))


def discrete_action(phi, r, rho):
    """CG functional J(phi) = (1/2)(phi, r) - 2 pi (rho, phi).

    With r = -4 pi rho - A phi this equals -(1/2)(phi, A phi) - 4 pi (rho, phi),
    the grid form of the action integral of Eq. AIntegral divided by h^3.
    """
    return 0.5 * float(np.sum(phi * r)) - 2.0 * np.pi * float(np.sum(rho * phi))
