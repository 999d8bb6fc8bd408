"""The SIMPLE preconditioner of Sec. 4.3 with exact inner solves, applied to
the projected saddle system J_P of Sec. 4.4.2 (test infrastructure only).

For a saddle matrix [[A, B^T], [B, -C]] the paper factors

    P^-1 = [[I, -D^-1 B^T], [0, I]] . diag(D^-1, S~^-1) . [[I, 0], [-B D^-1, I]]

with D = Diag(A) and S~ = -(C + B D^-1 B^T), i.e. P = [[D, B^T], [B, -C]]:
the saddle matrix with A replaced by its diagonal.  On the projected system
B becomes P B and C becomes P C P^T (P the per-slice projector of
Sec. 4.4.2), so

    S~_P = -P (C + B D^-1 B^T) P^T,

which is singular with the per-slice constants as kernel; the systems met
here are consistent (their right-hand sides sum to zero per slice), and the
zero-sum solution is taken (the constant is annihilated by P^T wherever y
enters J_P).  The paper solves S~ y = c after scaling both sides by
Diag(rho) (its eq. for the second mode of the SIMPLE system) to tame the
spread of C as mu -> 0; that scaling changes the inner iteration, not the
exact solution, so it does not appear here.

Pins (tests/test_oracle_simple.py): P^-1 applied to P z returns z, with P
assembled densely as the projected saddle matrix with A replaced by Diag(A);
planted mistakes (S~ with the other sign, the D^-1 dropped in the
back-substitution, P dropped from B) each fail that pin.
"""

from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .bb import proj, proj_t
from .ipm import Problem, kkt_blocks


def simple_blocks(prob: Problem, phi, rho, s):
    """(D, B, C) at an iterate: D = Diag(A) as a vector, B and C the KKT
    blocks of Sec. 3.1."""
    A, B, C = kkt_blocks(prob, phi, rho, s)
    return A.diagonal(), B, C


def simple_schur(prob: Problem, phi, rho, s):
    """S~_P = -P (C + B D^-1 B^T) P^T as a dense matrix (tiny meshes), built
    column by column: (P X P^T) e_j = P X (P^T e_j)."""
    D, B, C = simple_blocks(prob, phi, rho, s)
    X = (C + B @ sp.diags(1.0 / D) @ B.T).tocsr()
    K, nc = prob.K, prob.nc
    eye = np.eye(K * nc)
    cols = []
    for j in range(K * nc):
        v = proj_t(prob, eye[:, j].reshape(K, nc)).ravel()
        cols.append(proj(prob, (X @ v).reshape(K, nc)).ravel())
    return -np.stack(cols, axis=1)


def apply_simple_exact(prob: Problem, phi, rho, s, c, d):
    """(x; y) = P_SIMPLE^-1 (c; d) on the projected system, exact S~ solve.

    c: (K+1, nf), d: (K, nc).  Steps (Sec. 4.3):
      u = D^-1 c;  v = d - P B u;  y = S~_P^+ v (zero sum per slice);
      x = u - D^-1 B^T P^T y.
    """
    K, nc = prob.K, prob.nc
    D, B, _ = simple_blocks(prob, phi, rho, s)
    u = c.ravel() / D
    v = np.ravel(d) - proj(prob, (B @ u).reshape(K, nc)).ravel()
    S = simple_schur(prob, phi, rho, s)
    y = np.linalg.lstsq(S, v, rcond=1e-13)[0].reshape(K, nc)
    y = y - y.mean(axis=1, keepdims=True)
    x = u - (B.T @ proj_t(prob, y).ravel()) / D
    return x.reshape(K + 1, prob.nf), y


def simple_matrix(prob: Problem, phi, rho, s):
    """P_SIMPLE on the projected system: [[D, B^T P^T], [P B, -P C P^T]]
    (dense, tiny meshes), assembled from the KKT blocks with A replaced by
    its diagonal."""
    D, B, C = simple_blocks(prob, phi, rho, s)
    K, nc = prob.K, prob.nc
    m = K * nc
    P = np.zeros((m, m))
    eye = np.eye(m)
    for j in range(m):
        P[:, j] = proj(prob, eye[:, j].reshape(K, nc)).ravel()
    Bd, Cd = B.toarray(), C.toarray()
    return np.block([[np.diag(D), Bd.T @ P.T], [P @ Bd, -(P @ Cd @ P.T)]])


def gmres_solve(prob: Problem, phi, rho, s, b, tol=1e-10, maxit=400):
    """Right-preconditioned GMRES on J_P with P_SIMPLE^-1 (exact inner
    solves); returns the residual history (relative)."""
    from .bb import projected_matrix
    J = projected_matrix(prob, phi, rho, s)
    K, nf, nc = prob.K, prob.nf, prob.nc
    nphi = (K + 1) * nf
    N = J.shape[0]

    def prec(v):
        x, y = apply_simple_exact(prob, phi, rho, s, v[:nphi].reshape(K + 1, nf), v[nphi:].reshape(K, nc))
        return np.concatenate([x.ravel(), y.ravel()])

    op = spla.LinearOperator((N, N), matvec=lambda v: J @ prec(v))
    hist = []
    spla.gmres(op, b, rtol=tol, restart=maxit, maxiter=1, callback=lambda r: hist.append(r),
               callback_type="pr_norm")
    return hist
