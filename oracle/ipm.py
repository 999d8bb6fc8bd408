"""Discrete Benamou-Brenier system, its KKT Jacobian and the interior-point
continuation, in plain FP64 with sparse direct Newton solves.

Notation follows the paper: K density/slack time levels, K+1 potential levels,
dt = 1/(K+1), rho^0 = rho_in and rho^{K+1} = rho_f (Sec. 2.2).  Arrays are
slice-major: phi has shape (K+1, n_fine), rho and s have shape (K, n_coarse);
python index k-1 holds the paper's level k.

Readings where the paper is silent or inconsistent:
  * the time-difference term of F_rho uses Omega^T = J^T M (the transpose of the
    term of F_phi); the printed M' J^T differs from it by the child count and
    would break the symmetry of the Jacobian that Sec. 3 states;
  * mu schedule mu_l = mu0 * 0.2^l from mu0 = 1, stop after the first mu < tol;
  * Newton stops on the absolute Euclidean norm of (F_phi; F_rho; F_s - mu);
  * line search: one step length alpha = min(1, 0.99 alpha_max) for all
    variables, alpha_max keeping rho and s positive;
  * renormalisation of rho after every update is multiplicative per slice;
  * start point phi = 0, rho uniform with the marginals' mass, s = mu0 / rho.

Pins (tests/test_oracle_ipm.py): Taylor test of the Jacobian against F,
symmetry of the (phi, rho) Hessian block, per-slice mass conservation, the
exact gap identity KE - D* = mu K dt |Omega| at a converged solution, the
closed-form uniform-marginal solution, a brute-force minimisation of the
barrier problem on tiny meshes (independent of F and of the Jacobian), and
convergence of 2 * cost to |d|^2 for a translated narrow Gaussian.
"""

from __future__ import annotations

import dataclasses
import time

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .mesh import Mesh
from .operators import Operators


@dataclasses.dataclass
class Problem:
    """One OT problem: mesh, K and the two coarse-cell marginals."""

    mesh: Mesh
    K: int
    rho_in: np.ndarray
    rho_f: np.ndarray

    def __post_init__(self):
        self.ops = Operators(self.mesh)
        self.dt = 1.0 / (self.K + 1)
        self.rho_in = np.asarray(self.rho_in, dtype=np.float64)
        self.rho_f = np.asarray(self.rho_f, dtype=np.float64)

    @property
    def nf(self):
        return self.mesh.n_fine

    @property
    def nc(self):
        return self.mesh.n_coarse

    def rho_full(self, rho):
        """(rho^0; rho^1..rho^K; rho^{K+1}) as a (K+2, nc) array."""
        return np.vstack([self.rho_in[None, :], rho, self.rho_f[None, :]])


# ---------------------------------------------------------------------------
# Nonlinear residual (Sec. 2.3 and the relaxed system of Sec. 2.4)
# ---------------------------------------------------------------------------

def residual(prob: Problem, phi, rho, s, mu):
    """Return (F_phi, F_rho, F_s - mu) with shapes (K+1,nf), (K,nc), (K,nc).

    F_phi^k = -M J (rho^k - rho^{k-1})/dt - div(R_E((rho^k+rho^{k-1})/2) * grad phi^k)
    F_rho^k = Omega^T (phi^{k+1}-phi^k)/dt + 1/4 R_T((grad phi^k)^2 + (grad phi^{k+1})^2) + M' s^k
    F_s^k   = rho^k * s^k  (minus mu in the relaxed system)
    """
    o, K, dt = prob.ops, prob.K, prob.dt
    rf = prob.rho_full(rho)
    g = np.stack([o.grad @ phi[k] for k in range(K + 1)])
    Fphi = np.empty_like(phi)
    for k in range(1, K + 2):
        rt = o.RE @ (0.5 * (rf[k] + rf[k - 1]))
        Fphi[k - 1] = -(o.Om @ (rf[k] - rf[k - 1])) / dt - o.div @ (rt * g[k - 1])
    Frho = np.empty_like(rho)
    for k in range(1, K + 1):
        Frho[k - 1] = (o.Om.T @ (phi[k] - phi[k - 1])) / dt \
            + 0.25 * (o.RT @ (g[k - 1] ** 2 + g[k] ** 2)) + o.ac * s[k - 1]
    Fs = rho * s - mu
    return Fphi, Frho, Fs


def residual_norm(F):
    return float(np.sqrt(sum(float(np.sum(x * x)) for x in F)))


# ---------------------------------------------------------------------------
# KKT Jacobian blocks (Sec. 3) and the reduced saddle system (Sec. 3.1)
# ---------------------------------------------------------------------------

def edge_density(prob: Problem, rho):
    """rho~^k = R_E((rho^k + rho^{k-1})/2), k = 1..K+1, shape (K+1, ne)."""
    o = prob.ops
    rf = prob.rho_full(rho)
    return np.stack([o.RE @ (0.5 * (rf[k] + rf[k - 1])) for k in range(1, prob.K + 2)])


def kkt_blocks(prob: Problem, phi, rho, s):
    """Return the sparse blocks (A, B, C) of the Newton system at (phi, rho, s).

    A = BlkDiag(A^k), A^k = -div Diag(rho~^k) grad                (K+1 blocks)
    B = J^T D_t M + H G D_x,  G^k = R_T Diag(grad phi^k)          (K x (K+1))
    C = M' Diag(rho)^-1 Diag(s)                                     (diagonal)
    """
    o, K, dt = prob.ops, prob.K, prob.dt
    rt = edge_density(prob, rho)
    A = sp.block_diag([o.laplacian(rt[k]) for k in range(K + 1)], format="csr")
    G = [(o.RT @ sp.diags(o.grad @ phi[k])).tocsr() for k in range(K + 1)]
    OmT = o.Om.T.tocsr()
    blocks = [[None] * (K + 1) for _ in range(K)]
    for k in range(K):          # row block = paper level k+1
        # J^T D_t M: (phi^{k+2} - phi^{k+1}) / dt restricted by Omega^T
        # H G D_x: average of G^{k+1} grad and G^{k+2} grad
        blocks[k][k] = -OmT / dt + 0.5 * (G[k] @ o.grad)
        blocks[k][k + 1] = OmT / dt + 0.5 * (G[k + 1] @ o.grad)
    B = sp.bmat(blocks, format="csr")
    C = sp.diags((np.tile(o.ac, K) * (s / rho).ravel())).tocsr()
    return A, B, C


def kkt_matrix(prob: Problem, phi, rho, s):
    """Full 3x3 Jacobian of (F_phi; F_rho; F_s - mu) w.r.t. (phi, rho, s)."""
    A, B, _ = kkt_blocks(prob, phi, rho, s)
    Mc = sp.block_diag([prob.ops.Mc] * prob.K, format="csr")
    Ds = sp.diags(s.ravel())
    Dr = sp.diags(rho.ravel())
    return sp.bmat([[A, B.T, None], [B, None, Mc], [None, Ds, Dr]], format="csr")


def saddle_matrix(prob: Problem, phi, rho, s):
    """J_s = [[A, B^T], [B, -C]] after eliminating delta s (Sec. 3.1)."""
    A, B, C = kkt_blocks(prob, phi, rho, s)
    return sp.bmat([[A, B.T], [B, -C]], format="csr")


def newton_rhs(prob: Problem, phi, rho, s, mu):
    """(f, g, h) = -(F_phi, F_rho, F_s - mu) and g~ = g - M' Diag(rho)^-1 h."""
    Fphi, Frho, Fs = residual(prob, phi, rho, s, mu)
    f, g, h = -Fphi, -Frho, -Fs
    gt = g - prob.ops.ac[None, :] * h / rho
    return f, g, h, gt


def solve_saddle_direct(J, rhs):
    """Solve the singular saddle system by grounding the first phi unknown.

    The kernel of J_s is the global constant in phi (remark on the kernel,
    Sec. 3); the system is consistent when the marginals have equal mass, so
    fixing delta phi_0 = 0 and dropping its (redundant) row gives a regular
    system, solved by sparse LU.
    """
    n = J.shape[0]
    keep = np.arange(1, n)
    Jg = J[keep][:, keep].tocsc()
    b = rhs[1:]
    x = np.zeros(n)
    # symmetric ordering and diagonal pivots first (the matrix is symmetric);
    # fall back to the default partial-pivoting LU if that is not accurate
    lu = spla.splu(Jg, permc_spec="MMD_AT_PLUS_A", diag_pivot_thresh=0.0,
                   options=dict(SymmetricMode=True))
    x[1:] = lu.solve(b)
    bn = np.linalg.norm(b)
    if not np.all(np.isfinite(x)) or np.linalg.norm(Jg @ x[1:] - b) > 1e-11 * max(bn, 1e-300):
        x[1:] = spla.splu(Jg).solve(b)
    return x


# ---------------------------------------------------------------------------
# Interior point continuation (Sec. 2.4)
# ---------------------------------------------------------------------------

def slice_mass(prob: Problem, rho):
    return rho @ prob.ops.ac


def renormalize(prob: Problem, rho, m0):
    """Multiplicative per-slice renormalisation a'^T rho^k = m0 (Sec. 3.1 remark)."""
    return rho * (m0 / slice_mass(prob, rho))[:, None]


def step_length(x, dx, tau=0.99):
    """alpha = min(1, tau * sup{alpha: x + alpha dx > 0}) over all entries."""
    neg = dx < 0
    if not np.any(neg):
        return 1.0
    amax = float(np.min(-x[neg] / dx[neg]))
    return min(1.0, tau * amax)


def central_step(rho, s, drho, ds, gmu, amax):
    """Largest step t <= amax with (rho + t drho)(s + t ds) >= gmu in every
    cell where rho s > gmu holds at t = 0: per cell the first positive root
    of the quadratic a t^2 + b t + c, a = drho ds, b = rho ds + s drho,
    c = rho s - gmu (np.roots per cell, plain and slow)."""
    t = amax
    for r, sv, dr, d in zip(rho.ravel(), s.ravel(), drho.ravel(), ds.ravel()):
        c = r * sv - gmu
        if c <= 0:
            continue
        roots = np.roots([dr * d, r * d + sv * dr, c])
        pos = [x.real for x in roots if abs(x.imag) == 0.0 and x.real > 0]
        if pos:
            t = min(t, min(pos))
    return t


def solve_reduced_direct(prob: Problem, phi, rho, s, f, gt):
    """(delta phi, delta rho) of the Sec. 3.1 system J_s (dphi; drho) =
    (f; g~), with delta rho eliminated (C is diagonal):

        (A + B^T C^-1 B) dphi = f + B^T C^-1 g~,   drho = C^-1 (B dphi - g~).

    The potential-only matrix is symmetric positive semidefinite with the
    global constant as kernel (the kernel of J_s); the system is grounded at
    the first potential unknown like solve_saddle_direct.  Same solution,
    far less fill in the sparse LU at 64^2 and beyond."""
    A, B, C = kkt_blocks(prob, phi, rho, s)
    cinv = 1.0 / C.diagonal()
    S = (A + B.T @ sp.diags(cinv) @ B).tocsc()
    rhs = np.ravel(f) + B.T @ (cinv * np.ravel(gt))
    n = S.shape[0]
    dphi = np.zeros(n)
    Sg = S[1:, :][:, 1:].tocsc()
    lu = spla.splu(Sg, permc_spec="MMD_AT_PLUS_A", diag_pivot_thresh=0.0, options=dict(SymmetricMode=True))
    dphi[1:] = lu.solve(rhs[1:])
    if not np.all(np.isfinite(dphi)) or np.linalg.norm(Sg @ dphi[1:] - rhs[1:]) > 1e-11 * max(
            np.linalg.norm(rhs[1:]), 1e-300):
        dphi[1:] = spla.splu(Sg).solve(rhs[1:])
    drho = cinv * (B @ dphi - np.ravel(gt))
    return dphi, drho


def newton_step(prob: Problem, phi, rho, s, mu, tau=0.99, step_rule="common", neighborhood=0.0,
                direct="saddle"):
    """One Newton update of (phi, rho, s) at fixed mu with a direct solve.

    step_rule "common" (the reading of the positivity line search of Sec. 2.4):
    one step length for all three blocks, tau times the largest that keeps rho
    and s positive.  "split": phi and rho take tau times the largest step that
    keeps rho positive, s the one that keeps s positive (a primal / dual split
    of that line search).  neighborhood = gamma > 0 (common rule only)
    shortens the step further so that rho s >= gamma mu holds in every cell
    that satisfied it before (a neighbourhood of the central path).
    direct "saddle" solves J_s as it stands, "reduced" through the
    potential-only system of solve_reduced_direct (same solution)."""
    K, nf, nc = prob.K, prob.nf, prob.nc
    f, g, h, gt = newton_rhs(prob, phi, rho, s, mu)
    if direct == "reduced":
        dphi, drho = solve_reduced_direct(prob, phi, rho, s, f, gt)
        dphi = dphi.reshape(K + 1, nf)
        drho = drho.reshape(K, nc)
    elif direct == "saddle":
        J = saddle_matrix(prob, phi, rho, s)
        x = solve_saddle_direct(J, np.concatenate([f.ravel(), gt.ravel()]))
        dphi = x[: (K + 1) * nf].reshape(K + 1, nf)
        drho = x[(K + 1) * nf:].reshape(K, nc)
    else:
        raise ValueError(f"unknown direct solver {direct}")
    ds = (h - s * drho) / rho
    a_p, a_d = step_length(rho, drho, tau), step_length(s, ds, tau)
    alpha = min(a_p, a_d)
    if step_rule == "split":
        return phi + a_p * dphi, rho + a_p * drho, s + a_d * ds, alpha
    if step_rule != "common":
        raise ValueError(f"unknown step rule {step_rule}")
    if neighborhood > 0:
        alpha = central_step(rho, s, drho, ds, neighborhood * mu, alpha)
    return phi + alpha * dphi, rho + alpha * drho, s + alpha * ds, alpha


@dataclasses.dataclass
class IPMResult:
    phi: np.ndarray        # normalised: sum_k a^T phi^k = 0
    rho: np.ndarray
    s: np.ndarray
    mu: float
    cost: float            # kinetic energy KE
    dual: float            # D*
    gap: float             # KE - D*
    newton_per_mu: list
    residuals: list
    seconds: float
    converged: bool


def initial_point(prob: Problem, mu0=1.0):
    m0 = float(prob.ops.ac @ prob.rho_in)
    area = prob.mesh.domain_area
    phi = np.zeros((prob.K + 1, prob.nf))
    rho = np.full((prob.K, prob.nc), m0 / area)
    s = mu0 / rho
    return phi, rho, s


def solve_ipm(prob: Problem, tol=1e-6, mu0=1.0, mu_factor=0.2, tau=0.99,
              max_newton=20, final_tol=None, start=None, mu_start=None,
              max_mu_steps=200, mu_target=None, step_rule="common", neighborhood=0.0, direct="saddle"):
    """IP continuation: for mu_l = mu0 mu_factor^l, Newton until |F_mu| <= tol,
    warm-started from the previous mu; stop after the first mu < tol.

    final_tol, when given, replaces tol for the last mu (tighter solves for
    parity and finite-difference checks).  start = (phi, rho, s) and mu_start
    resume a previous run.  mu_target, when given, clamps the schedule at that
    value and stops after solving it (solutions at a prescribed mu).  direct
    selects the Newton systems' direct solver (newton_step).
    """
    t0 = time.perf_counter()
    m0 = float(prob.ops.ac @ prob.rho_in)
    if start is None:
        phi, rho, s = initial_point(prob, mu0)
    else:
        phi, rho, s = (np.array(x, dtype=np.float64) for x in start)
    mu = mu0 if mu_start is None else mu_start
    newton_counts, residuals = [], []
    converged = True
    for _ in range(max_mu_steps):
        if mu_target is not None:
            mu = max(mu, mu_target)
            last = mu <= mu_target
        else:
            last = mu < tol
        tol_l = final_tol if (last and final_tol is not None) else tol
        count = 0
        ok = False
        for it in range(max_newton + 1):
            F = residual(prob, phi, rho, s, mu)
            nrm = residual_norm(F)
            residuals.append((mu, nrm))
            if nrm <= tol_l:
                ok = True
                break
            if it == max_newton:
                break
            phi, rho, s, _ = newton_step(prob, phi, rho, s, mu, tau, step_rule, neighborhood, direct)
            rho = renormalize(prob, rho, m0)
            count += 1
        newton_counts.append(count)
        converged = converged and ok
        if last:
            break
        mu *= mu_factor
    phi_n = normalize_phi(prob, phi)
    ke = kinetic_energy(prob, phi_n, rho)
    ds = dual_value(prob, phi_n)
    return IPMResult(phi=phi_n, rho=rho, s=s, mu=mu, cost=ke, dual=ds, gap=ke - ds,
                     newton_per_mu=newton_counts, residuals=residuals,
                     seconds=time.perf_counter() - t0, converged=converged)


# ---------------------------------------------------------------------------
# Outputs
# ---------------------------------------------------------------------------

def normalize_phi(prob: Problem, phi):
    """Shift phi by a global constant so that sum_k a^T phi^k = 0 (phi is
    defined up to a global constant, remark on the kernel in Sec. 3)."""
    a = prob.ops.a
    c = float(np.sum(phi @ a)) / ((prob.K + 1) * float(a.sum()))
    return phi - c


def kinetic_energy(prob: Problem, phi, rho):
    """KE = dt/2 sum_k sum_e W_e rho~^k_e (grad phi^k)_e^2: the discrete value
    of the kinetic energy of the transport problem (Sec. 1 objective)."""
    o = prob.ops
    rt = edge_density(prob, rho)
    tot = 0.0
    for k in range(prob.K + 1):
        gk = o.grad @ phi[k]
        tot += float(np.sum(o.Wvec * rt[k] * gk * gk))
    return 0.5 * prob.dt * tot


def dual_value(prob: Problem, phi):
    """D* = phi^{K+1,T} Omega rho_f - phi^{1,T} Omega rho_in
            - dt/4 [rho_in^T R_T (grad phi^1)^2 + rho_f^T R_T (grad phi^{K+1})^2].

    Summation by parts of the continuity and Hamilton-Jacobi equations gives
    KE = D* + mu K dt |Omega| at an exact solution of the relaxed system.
    """
    o, dt = prob.ops, prob.dt
    g1 = o.grad @ phi[0]
    gK = o.grad @ phi[-1]
    return float(phi[-1] @ (o.Om @ prob.rho_f) - phi[0] @ (o.Om @ prob.rho_in)
                 - 0.25 * dt * (prob.rho_in @ (o.RT @ (g1 * g1))
                                + prob.rho_f @ (o.RT @ (gK * gK))))
