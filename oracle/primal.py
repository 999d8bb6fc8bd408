"""The primal-Schur preconditioner of Sec. 4.2 with an exact inner solve,
applied to the projected saddle system J_P of Sec. 4.4.2 (test
infrastructure only).

For a saddle matrix [[A, B^T], [B, -C]] with C diagonal, the paper's
preconditioner (Sec. 4.2) is the block factorisation built on the primal
Schur complement S_p = A + B^T C^-1 B:

    P^-1 = [[I, 0], [C^-1 B, I]] . diag(S_p^-1, -C^-1) . [[I, B^T C^-1], [0, I]],

the exact inverse of [[A, B^T], [B, -C]].  On the projected system B
becomes P B while the (2,2) block P C P^T is no longer diagonal; the
factorisation keeps the diagonal C there, so it is the exact inverse of

    J^ = [[A, B^T P^T], [P B, -C]],

which differs from J_P only in C - P C P^T (rank at most two per slice).
Then S_p = A + B^T P^T C^-1 P B.  P B annihilates the per-slice constants
of phi (B maps them to multiples of a' per slice, and P removes those), and
so does A: S_p is symmetric positive semidefinite with exactly the K+1
per-slice constants as kernel (the same kernel J_P has in phi; the Newton
step recovers those constants afterwards).  The inner right-hand side is
made zero-sum per slice and the zero-sum solution taken.

Pins (tests/test_oracle_primal.py): P^-1 applied to J^ z returns z for z
whose phi part is zero-sum per slice, with J^ assembled densely from the
KKT blocks; planted mistakes (C with the other sign, the projector
dropped from P B, the zero-sum solution replaced by a shifted one) each
fail that pin.
"""

from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .bb import proj_matrix
from .ipm import Problem, kkt_blocks


def primal_schur(prob: Problem, phi, rho, s):
    """S_p = A + B^T P^T C^-1 P B (sparse, with P as a sparse matrix: its
    rank-one part per slice makes S_p denser than A, so tiny meshes only)."""
    A, B, C = kkt_blocks(prob, phi, rho, s)
    PB = (proj_matrix(prob) @ B).tocsr()
    return (A + PB.T @ sp.diags(1.0 / C.diagonal()) @ PB).tocsr()


def _zero_sum_per_slice(prob: Problem, x):
    x = np.array(x, dtype=float).reshape(prob.K + 1, prob.nf)
    return x - x.mean(axis=1, keepdims=True)


def apply_primal_exact(prob: Problem, phi, rho, s, f, g):
    """(x; y) = P^-1 (f; g) for the projected system (Sec. 4.2 factorisation).

    f: (K+1, nf), g: (K, nc).  Steps:
      t = f + B^T P^T C^-1 g, made zero-sum per slice;
      x = S_p^+ t (zero-sum per slice);
      y = C^-1 (P B x - g).
    """
    K, nf, nc = prob.K, prob.nf, prob.nc
    _, B, C = kkt_blocks(prob, phi, rho, s)
    P = proj_matrix(prob)
    cinv = 1.0 / C.diagonal()
    t = np.ravel(f) + B.T @ (P.T @ (cinv * np.ravel(g)))
    t = _zero_sum_per_slice(prob, t).ravel()
    S = primal_schur(prob, phi, rho, s)
    # the kernel is spanned by the per-slice constants: add Q Q^T (Q the
    # normalised per-slice indicator vectors) to make the matrix regular;
    # for t orthogonal to Q the solution is the zero-sum one
    Q = sp.block_diag([sp.csr_matrix(np.full((nf, 1), 1.0 / np.sqrt(nf)))] * (K + 1), format="csr")
    x = spla.spsolve((S + Q @ Q.T).tocsc(), t)
    x = _zero_sum_per_slice(prob, x)
    y = cinv * (P @ (B @ x.ravel()) - np.ravel(g))
    return x, y.reshape(K, nc)


def primal_matrix(prob: Problem, phi, rho, s):
    """J^ = [[A, B^T P^T], [P B, -C]] (dense, tiny meshes)."""
    A, B, C = kkt_blocks(prob, phi, rho, s)
    P = proj_matrix(prob).toarray()
    Bd = B.toarray()
    return np.block([[A.toarray(), Bd.T @ P.T], [P @ Bd, -C.toarray()]])
