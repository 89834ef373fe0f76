"""Algorithm SC and the PSD minimization of Sec. II.A in plain binary64
(test infrastructure only).

Algorithm SC (self-consistent iteration with linear mixing eta):
    rho_iter_0 = 0;  for k = 0, 1, ...:
        phi_k          = G (rho/eps + rho_iter_k)          (Eq. remap, the SPe solve)
        rho_new        = (1/4 pi) grad ln eps . grad phi_k  (Eq. rhoiter)
        rho_iter_{k+1} = eta rho_new + (1 - eta) rho_iter_k
        r_{k+1}        = rho_iter_{k+1} - rho_iter_k
Gradients are the order-2M central differences of the polarization charge
(oracle/cavity.py); G is the plan's vacuum solver.

PSD (Algorithm PCG with beta = 0 and the preconditioner of Eq. PrePSD,
eps lap v = -4 pi r, i.e. v = G(r/eps)).  The operator on v follows Eq.
PrePSD's identity, A v = div(eps grad v) = eps lap v + grad eps . grad v =
-4 pi r + eps grad ln eps . grad v, with grad eps written as eps grad ln eps so
that PSD and SC discretize the same operator,
    A phi = eps L_G phi + eps (grad_h ln eps) . grad_h phi,  L_G = -4 pi G^-1.
    r_0 = -4 pi rho;  v_k = G(r_k/eps);  A v_k = -4 pi r_k + eps grad ln eps . grad v_k
    phi += alpha_k v_k;  r -= alpha_k A v_k.
Two steps alpha_k are provided:
  * step "paper" (the default): Algorithm PCG's own step with p_k = v_k,
    alpha_k = (v_k, r_k) / (v_k, A v_k), stopping like Algorithm PCG at
    ||r_k||_2 <= tol ||4 pi rho||_2.  This is the exact line minimum of the
    quadratic functional only for a symmetric operator and preconditioner; here
    neither A (written with grad eps) nor P = eps lap is symmetric, and the
    iteration stalls: on the paper's Gaussian test (Sec. II.C) and on small
    molecules the relative residual stays near 1 (1.05 and 3.4) for hundreds of
    steps.  It ends with status "not_converged" at maxit.
  * step "weighted": the step minimizing ||r/eps||_2, the norm of SC's own
    residual below, along A v_k:
        alpha_k = (A v_k, r_k / eps^2) / (A v_k, A v_k / eps^2),
    stopping at ||r_k / eps||_2 <= tol ||4 pi rho / eps||_2.  It converges
    like SC (47 steps against SC's 48 at eta = 0.6 on a 16^3 molecule).
With the same operator, one SC step with mixing eta is the PSD step with the
fixed alpha = -eta / (4 pi): since v = G(r/eps) = -4 pi (phi_SC - phi) for the
SC update phi_SC = G(rho/eps + rho_new(phi)), and the mixing is linear in
rho_iter, phi_{k+1} = phi_k + eta (phi_SC(phi_k) - phi_k).  SC's first
potential is unmixed (phi_0 = G(rho/eps)), so PSD from phi = 0 reproduces the
SC iterates with alpha = -1/(4 pi) in its first step and -eta/(4 pi) after
(the paper's remark that PSD with a fixed unit step is SC, in the sign and
scale conventions of Algorithm PCG used here).  SC's residual is
rho_iter_{k+1} - rho_iter_k = -(eta / 4 pi) r_k / eps at the current iterate.
SC stops when ||rho_iter_{k+1} - rho_iter_k||_2 <= tol ||rho||_2.
"""
import numpy as np

from .cavity import gradient_fd
from .green import VacuumSolver

FOUR_PI = 4.0 * np.pi


def grad_dot(a, b, h, m_half, bc):
    ga = gradient_fd(a, h, m_half, bc)
    gb = gradient_fd(b, h, m_half, bc)
    return ga[0] * gb[0] + ga[1] * gb[1] + ga[2] * gb[2]


def sc_solve(rho, eps, h, bc, eta, tol, maxit=1000, fd_order=16, solver=None):
    """Algorithm SC: returns (phi, iterations, history of ||r_k||_2)."""
    rho = np.asarray(rho, dtype=np.float64)
    eps = np.asarray(eps, dtype=np.float64)
    if solver is None:
        solver = VacuumSolver(rho.shape, h, bc)
    lne = np.log(eps)
    m = fd_order // 2
    rho_iter = np.zeros(rho.shape)
    hist = []
    phi = solver.apply(rho / eps)
    for k in range(maxit):
        rho_new = grad_dot(lne, phi, h, m, bc) / FOUR_PI
        nxt = eta * rho_new + (1.0 - eta) * rho_iter
        r = nxt - rho_iter
        rho_iter = nxt
        phi = solver.apply(rho / eps + rho_iter)
        hist.append(float(np.sqrt(np.sum(r * r))))
        if hist[-1] <= tol * float(np.sqrt(np.sum(rho * rho))):
            return phi, k + 1, hist
    return phi, maxit, hist


def psd_solve(rho, eps, h, bc, tol, alpha=None, alpha_first=None, maxit=1000, fd_order=16,
              solver=None, record=None, step="paper", res_hist=None):
    """PSD (beta = 0).  alpha None: the step of `step` ("paper" or
    "weighted", see the module docstring); else the fixed alpha (the first
    step may take alpha_first instead), stopping like "weighted".  Returns
    (phi, iterations, status) with status "ok", "not_converged",
    "breakdown" (a zero or non-finite denominator of the step) or
    "nonfinite".  record (a list) receives phi after every step, res_hist
    (a list) the stopping norm of r relative to its initial value."""
    if step not in ("paper", "weighted"):
        raise ValueError("unknown PSD step %r" % (step,))
    rho = np.asarray(rho, dtype=np.float64)
    eps = np.asarray(eps, dtype=np.float64)
    if solver is None:
        solver = VacuumSolver(rho.shape, h, bc)
    lne = np.log(eps)
    m = fd_order // 2
    r = -FOUR_PI * rho
    phi = np.zeros(rho.shape)
    if step == "paper" and alpha is None:
        norm = lambda x: float(np.sqrt(np.sum(x * x)))
    else:
        norm = lambda x: float(np.sqrt(np.sum((x / eps) ** 2)))
    thr = tol * norm(r)
    for k in range(maxit):
        if norm(r) <= thr:
            return phi, k, "ok"
        v = solver.apply(r / eps)
        av = -FOUR_PI * r + eps * grad_dot(lne, v, h, m, bc)
        a = alpha_first if (k == 0 and alpha_first is not None) else alpha
        if a is None:
            if step == "paper":
                num, den = float(np.sum(v * r)), float(np.sum(v * av))
            else:
                num = float(np.sum(av * r / (eps * eps)))
                den = float(np.sum((av / eps) ** 2))
            if not (np.isfinite(num) and np.isfinite(den)):
                return phi, k, "nonfinite"
            if den == 0.0:
                return phi, k, "breakdown"
            a = num / den
        phi = phi + a * v
        r = r - a * av
        if record is not None:
            record.append(phi.copy())
        if res_hist is not None:
            res_hist.append(norm(r) / norm(-FOUR_PI * rho))
    if norm(r) <= thr:
        return phi, maxit, "ok"
    return phi, maxit, "not_converged"


def dense_sc_operator(eps, h, bc, fd_order=16):
    """The matrix of A phi = eps L_G phi + eps grad_h ln eps . grad_h phi
    (tiny grids), assembled column by column from unit vectors."""
    from .green import dense_green
    eps = np.asarray(eps, dtype=np.float64)
    shape = eps.shape
    n = eps.size
    g = dense_green(shape, h, bc)
    lg = -FOUR_PI * np.linalg.inv(g)
    lne = np.log(eps)
    m = fd_order // 2
    cols = np.empty((n, n))
    for j in range(n):
        e = np.zeros(n)
        e[j] = 1.0
        cols[:, j] = grad_dot(lne, e.reshape(shape), h, m, bc).ravel()
    return eps.ravel()[:, None] * (lg + cols)
