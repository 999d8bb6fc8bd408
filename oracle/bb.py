"""Projected saddle system and the BB preconditioner with exact inner solves.

Sec. 4.4.1-4.4.2: the potential is split into a zero-mean part and a
time-only shift; eliminating the shift gives the projected system
    J_P = [[A, B^T P^T], [P B, -P C P^T]],   P = I - M' E'^T E' / |Omega|,
acting on (delta phi_hat; delta rho).  A solution of it is turned into a
solution of the reduced Newton system J_s by the recovery below.

Sec. 4.4.3: the dual Schur complement is approximated through the commutator
-B^T M'^-1 A~ ~= A M^-1 B~, which leaves the pseudo-Schur system
    (Diag(s) A~ - Diag(rho) B M^-1 B~) z = -Diag(rho) d,     y = M'^-1 A~ z,
followed by the block-triangular back-substitution A x = c - B^T P^T y over
the K+1 independent Laplacians.

Readings where the paper is silent or its formula does not type-check:
  * A~^k is the positive coarse Laplacian -div' Diag(R'_E rho^k) grad';
  * B~ = -Omega D~_t^T + G_f D_x J H^T with G_f^k = R_Tf Diag(grad phi^k) and
    J = M^-1 Omega: the fine operator M (d/dt + grad phi . grad) composed with
    the coarse-to-fine lift, i.e. the discrete right factor of the commutator;
    the printed formula does not type-check (block sizes), this is the reading
    whose time part equals the printed one;
  * the sign follows the printed pseudo-Schur system (right-hand side
    -Diag(rho) d) with A x = c - B^T P^T y: the preconditioner is then the
    block upper-triangular matrix with the true (negative) Schur complement,
    and J_P times its inverse is identity plus nilpotent;
  * the Laplacian right-hand sides are projected onto zero sum and the
    Laplacian solutions are returned with zero sum (their constant is in the
    kernel of J_P);
  * the time shift enters the potential at level k as dt * sum_{i<k} delta
    lambda^i (the shift has K components, one per density level).

Pins (tests/test_oracle_bb.py, tests/test_oracle_bb_pins.py): P^2 = P,
E' M' E'^T = |Omega| I, the kernel relations of Sec. 3 and Sec. 4.4.2; the
pseudo-Schur operator against a dense matrix assembled entry by entry from
the definitions of Sec. 4.4.3 (from the raw mesh arrays, not these sparse
operators); apply_bb_exact's outputs satisfying the pseudo-Schur system, the
definition of y and the K+1 Laplacian equations in that dense form; with the
exact Schur complement routed through apply_bb_exact itself, GMRES on
J_P P^-1 converging in two steps and (J_P P^-1 - I)^2 vanishing on the range;
planted mistakes (y with the other sign, P^T dropped, a sign slip inside the
pseudo-Schur operator) each failing one of these pins; the commutator being
small for a translation and large when B~ is misread; and projected solve +
recovery agreeing with the grounded direct solve of J_s.
"""

from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .ipm import Problem, kkt_blocks


# ---------------------------------------------------------------- projector
def proj(prob: Problem, v):
    """(P v)^k = v^k - a' (1^T v^k) / |Omega|, v of shape (K, nc)."""
    ac = prob.ops.ac
    return v - ac[None, :] * (v.sum(axis=1) / ac.sum())[:, None]


def proj_t(prob: Problem, v):
    """(P^T v)^k = v^k - 1 (a'^T v^k) / |Omega|."""
    ac = prob.ops.ac
    return v - ((v @ ac) / ac.sum())[:, None]


def proj_matrix(prob: Problem):
    ac = prob.ops.ac
    Pk = sp.identity(prob.nc, format="csr") - sp.csr_matrix(np.outer(ac, np.ones(prob.nc)) / ac.sum())
    return sp.block_diag([Pk] * prob.K, format="csr")


def projected_matrix(prob: Problem, phi, rho, s):
    """J_P of the projected Newton system (Sec. 4.4.2)."""
    A, B, C = kkt_blocks(prob, phi, rho, s)
    P = proj_matrix(prob)
    return sp.bmat([[A, B.T @ P.T], [P @ B, -(P @ C @ P.T)]], format="csr")


def apply_projected(prob: Problem, phi, rho, s, x):
    """y = J_P x for a flat x = (x_phi; x_rho)."""
    return projected_matrix(prob, phi, rho, s) @ x


# ---------------------------------------------------------------- BB pieces
def coarse_laplacian_blocks(prob: Problem, rho):
    """A~ = BlkDiag(A~^k), k = 1..K."""
    return sp.block_diag([prob.ops.coarse_laplacian(rho[k]) for k in range(prob.K)],
                         format="csr")


def btilde(prob: Problem, phi):
    """B~ (n_phi x m_rho): (B~ z)^k = Omega (z^k - z^{k-1})/dt
    + R_Tf[grad phi^k * grad(J (z^{k-1} + z^k)/2)], z^0 = z^{K+1} = 0."""
    o, K, dt = prob.ops, prob.K, prob.dt
    # time part: -Omega D~_t^T, with (D~_t u)^k = (u^{k+1} - u^k)/dt
    Dt = sp.bmat([[(-sp.identity(prob.nc) if j == k else
                    (sp.identity(prob.nc) if j == k + 1 else None))
                   for j in range(K + 1)] for k in range(K)], format="csr") / dt
    OmB = sp.block_diag([o.Om] * (K + 1), format="csr")
    # gradient part: G_f D_x J H^T
    Gf = sp.block_diag([(o.RTf @ sp.diags(o.grad @ phi[k]) @ o.grad).tocsr()
                        for k in range(K + 1)], format="csr")
    Jb = sp.block_diag([o.Jlift] * (K + 1), format="csr")
    Hm = sp.bmat([[(0.5 * sp.identity(prob.nc) if j in (k, k + 1) else None)
                   for j in range(K + 1)] for k in range(K)], format="csr")
    return (-(OmB @ Dt.T) + Gf @ Jb @ Hm.T).tocsr()


def pseudo_schur(prob: Problem, phi, rho, s):
    """S_BB = Diag(s) A~ - Diag(rho) B M^-1 B~ (scaled pseudo-Schur operator)."""
    _, B, _ = kkt_blocks(prob, phi, rho, s)
    At = coarse_laplacian_blocks(prob, rho)
    Minv = sp.diags(1.0 / np.tile(prob.ops.a, prob.K + 1))
    return (sp.diags(s.ravel()) @ At - sp.diags(rho.ravel()) @ B @ Minv @ btilde(prob, phi)).tocsr()


def _solve_laplacian_zero_sum(L, b):
    """Solve L x = b - mean(b) with sum(x) = 0 (L a connected graph Laplacian)."""
    n = L.shape[0]
    b = b - b.mean()
    x = np.zeros(n)
    x[1:] = spla.spsolve(L[1:, 1:].tocsc(), b[1:])
    return x - x.mean()


def exact_schur_solve(prob: Problem, phi, rho, s, rhs):
    """Least-squares solution w of P (C + B A^+ B^T) P^T w = rhs (dense).

    The exact projected Schur complement of J_P is -P (C + B A^+ B^T) P^T
    (Sec. 4.4.2).  TEST-ONLY and for tiny meshes: it forms the dense
    pseudo-inverse of the K+1 Laplacians.  It stands in for the pseudo-Schur
    step of the BB preconditioner, so that the rest of apply_bb_exact can be
    checked against the ideal block-triangular preconditioner.
    """
    A, B, C = kkt_blocks(prob, phi, rho, s)
    P = proj_matrix(prob).toarray()
    Ap = np.linalg.pinv(A.toarray(), rcond=1e-12)
    Bd = B.toarray()
    Shat = P @ (C.toarray() + Bd @ Ap @ Bd.T) @ P.T
    return np.linalg.lstsq(Shat, np.ravel(rhs), rcond=1e-12)[0].reshape(prob.K, prob.nc)


def apply_bb_exact(prob: Problem, phi, rho, s, c, d, schur="bb", return_zeta=False):
    """(x; y) = P_BB^-1 (c; d) with exact inner solves.

    c: (K+1, nf), d: (K, nc).  Steps (Sec. 4.4.3):
      z = S_BB^-1 (-Diag(rho) P d);  w = M'^-1 A~ z;  y = P^T w;
      b = c - B^T y;  x^k = (A^k)^+ (b^k - mean), zero-sum.
    schur="exact" (test-only, tiny meshes) replaces the first two steps by
    the exact projected Schur solve w = [P (C + B A^+ B^T) P^T]^+ (-P d),
    which turns the whole application into the ideal block upper-triangular
    preconditioner of Sec. 4.4.2.  return_zeta=True also returns z (None in
    the exact mode).
    """
    o, K = prob.ops, prob.K
    _, B, _ = kkt_blocks(prob, phi, rho, s)
    z = None
    if schur == "bb":
        S = pseudo_schur(prob, phi, rho, s)
        z = spla.spsolve(S.tocsc(), -(rho * proj(prob, d)).ravel())
        At = coarse_laplacian_blocks(prob, rho)
        w = ((At @ z).reshape(K, prob.nc)) / o.ac[None, :]
    elif schur == "exact":
        w = exact_schur_solve(prob, phi, rho, s, -proj(prob, d))
    else:
        raise ValueError(f"unknown schur mode {schur}")
    y = proj_t(prob, w)
    b = c.ravel() - B.T @ y.ravel()
    b = b.reshape(K + 1, prob.nf)
    from .ipm import edge_density
    rt = edge_density(prob, rho)
    x = np.stack([_solve_laplacian_zero_sum(o.laplacian(rt[k]), b[k]) for k in range(K + 1)])
    if return_zeta:
        return x, y, (None if z is None else z.reshape(K, prob.nc))
    return x, y


# ---------------------------------------------------------------- recovery
def recover(prob: Problem, phi, rho, s, dphi_hat, drho, gt):
    """Turn a solution of the projected system into one of J_s (Sec. 4.4.1-2).

    drho <- P^T drho (zero slice mass);  dphi_bar^k = dphi_hat^k minus its
    area mean;  delta lambda = E'(g~ - B dphi_bar + C drho) / |Omega|;
    dphi^k = dphi_bar^k + dt sum_{i<k} delta lambda^i.
    """
    o, K, dt = prob.ops, prob.K, prob.dt
    _, B, C = kkt_blocks(prob, phi, rho, s)
    drho = proj_t(prob, drho)
    a = o.a
    dphib = dphi_hat - ((dphi_hat @ a) / a.sum())[:, None]
    r = gt.ravel() - B @ dphib.ravel() + C @ drho.ravel()
    dlam = r.reshape(K, prob.nc).sum(axis=1) / o.ac.sum()
    shift = np.concatenate([[0.0], np.cumsum(dt * dlam)])
    return dphib + shift[:, None], drho
