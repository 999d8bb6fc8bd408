"""Sparse discrete operators of the two-level FV scheme (Sec. 2.1) and of the
BB approximation (Sec. 4.4.3), assembled as scipy CSR matrices in FP64.

Per time slice:
  M   = Diag(fine areas),  M' = Diag(coarse areas)
  Om  = M J  (overlap areas; with a 0/1 injection J this is exactly M J)
  E   signed incidence, E[K, e] = +1, E[L, e] = -1
  grad = Diag(d)^-1 E^T                 (two-point gradient on edges)
  W    = Diag(d * len)
  div  = -grad^T W = -E Diag(len)
  R_E  coarse cell -> fine edge, lambda-weighted mean of the two sides
  R_T  = R_E^T W                         (fine edge -> coarse cell)
  R_Ef fine cell -> fine edge lambda mean, R_Tf = R_Ef^T W (used by B~)
  coarse-level grad', W', R'_E for the coarse weighted Laplacian A~.

Pins (tests/test_oracle_operators.py): grad 1 = 0, 1^T div = 0, R_E 1 = 1,
the unit-weight Laplacian equals the textbook 5-point graph Laplacian built
from Kronecker products, R_T of the squared gradient of a linear function is
|d|^2 a' on interior coarse cells, and Omega row/column sums.
"""

from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .mesh import Mesh


class Operators:
    """All per-slice operators of one mesh."""

    def __init__(self, mesh: Mesh):
        self.mesh = m = mesh
        nf, nc, ne = m.n_fine, m.n_coarse, m.n_fedge
        self.a = m.fine_area.copy()
        self.ac = m.coarse_area.copy()
        self.M = sp.diags(self.a).tocsr()
        self.Mc = sp.diags(self.ac).tocsr()
        self.Om = sp.csr_matrix((m.ov_area, (m.ov_fine, m.ov_coarse)), shape=(nf, nc))
        e = np.arange(ne)
        self.E = sp.csr_matrix(
            (np.concatenate([np.ones(ne), -np.ones(ne)]),
             (np.concatenate([m.fe_K, m.fe_L]), np.concatenate([e, e]))),
            shape=(nf, ne))
        self.grad = (sp.diags(1.0 / m.fe_dist) @ self.E.T).tocsr()
        self.Wvec = m.fe_dist * m.fe_len
        self.W = sp.diags(self.Wvec).tocsr()
        self.div = (-self.grad.T @ self.W).tocsr()
        self.RE = sp.csr_matrix(
            (np.concatenate([m.fe_lam, 1.0 - m.fe_lam]),
             (np.concatenate([e, e]), np.concatenate([m.fe_rK, m.fe_rL]))),
            shape=(ne, nc))
        self.RT = (self.RE.T @ self.W).tocsr()
        self.REf = sp.csr_matrix(
            (np.concatenate([m.fe_lam, 1.0 - m.fe_lam]),
             (np.concatenate([e, e]), np.concatenate([m.fe_K, m.fe_L]))),
            shape=(ne, nf))
        self.RTf = (self.REf.T @ self.W).tocsr()
        # lift coarse -> fine by area-weighted overlap (J = M^-1 Om)
        self.Jlift = (sp.diags(1.0 / self.a) @ self.Om).tocsr()
        # coarse level (BB approximation only)
        nce = m.n_cedge
        ce = np.arange(nce)
        self.Ec = sp.csr_matrix(
            (np.concatenate([np.ones(nce), -np.ones(nce)]),
             (np.concatenate([m.ce_i, m.ce_j]), np.concatenate([ce, ce]))),
            shape=(nc, nce))
        self.gradc = (sp.diags(1.0 / m.ce_dist) @ self.Ec.T).tocsr()
        self.Wc = sp.diags(m.ce_dist * m.ce_len).tocsr()
        self.REc = sp.csr_matrix(
            (np.concatenate([m.ce_lam, 1.0 - m.ce_lam]),
             (np.concatenate([ce, ce]), np.concatenate([m.ce_i, m.ce_j]))),
            shape=(nce, nc))

    # ---- per-slice building blocks ------------------------------------
    def laplacian(self, edge_weight: np.ndarray) -> sp.csr_matrix:
        """-div Diag(w) grad  (Sec. 3: the weighted Laplacian blocks A^k)."""
        return (-self.div @ sp.diags(edge_weight) @ self.grad).tocsr()

    def coarse_laplacian(self, rho: np.ndarray) -> sp.csr_matrix:
        """A~^k = -div' Diag(R'_E rho) grad' on the coarse mesh (Sec. 4.4.3).

        The printed definition carries no minus sign; A~ discretises the
        positive operator -div(rho grad) like A^k does, so the sign of A^k is
        used.
        """
        w = self.REc @ rho
        return (self.gradc.T @ self.Wc @ sp.diags(w) @ self.gradc).tocsr()
