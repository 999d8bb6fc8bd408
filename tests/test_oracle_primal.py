"""Pins of the oracle's primal-Schur preconditioner (Sec. 4.2) on the
projected saddle system (test infrastructure).

The factorisation inverts J^ = [[A, B^T P^T], [P B, -C]]: the projected
saddle matrix with its (2,2) block kept diagonal.  J^ is assembled here
densely from the KKT blocks (which the Taylor and symmetry tests pin),
independently of the factorised form, and apply_primal_exact(J^ z) must
return z for z whose phi part is zero-sum per slice (the kernel of S_p is
the per-slice constants).  Planted mistakes each fail the pin.
"""

import numpy as np
import pytest
import scipy.sparse as sp

import otinputs
from oracle import primal as PR
from oracle.bb import proj_matrix
from oracle.ipm import Problem, kkt_blocks, solve_ipm
from oracle.mesh import cartesian3d_mesh, structured_mesh


def _dense(prob, phi, rho, s):
    A, B, C = kkt_blocks(prob, phi, rho, s)
    P = proj_matrix(prob).toarray()
    Bd = B.toarray()
    return np.block([[A.toarray(), Bd.T @ P.T], [P @ Bd, -np.diag(C.diagonal())]])


@pytest.fixture(scope="module", params=["tri4K3", "cube2K2"])
def state(request):
    if request.param == "tri4K3":
        n, K = 4, 3
        ri, rf = otinputs.mixture_pair(n, 2, config=8, problem=1)
        prob = Problem(structured_mesh(n), K, ri, rf)
    else:
        K = 2
        ri, rf = otinputs.gaussian3d_pair(2)
        prob = Problem(cartesian3d_mesh(2), K, ri, rf)
    r = solve_ipm(prob, tol=1e-6, mu_target=0.04)
    return prob, r.phi, r.rho, r.s


def _pin_err(prob, phi, rho, s, Jh, seed):
    rng = np.random.default_rng(seed)
    K, nf, nc = prob.K, prob.nf, prob.nc
    nphi = (K + 1) * nf
    x = rng.standard_normal((K + 1, nf))
    x -= x.mean(axis=1, keepdims=True)
    y = rng.standard_normal((K, nc))
    r = Jh @ np.concatenate([x.ravel(), y.ravel()])
    xx, yy = PR.apply_primal_exact(prob, phi, rho, s, r[:nphi].reshape(K + 1, nf), r[nphi:].reshape(K, nc))
    return max(np.abs(xx - x).max() / np.abs(x).max(), np.abs(yy - y).max() / np.abs(y).max())


def test_inverse_of_dense_primal(state):
    prob, phi, rho, s = state
    Jh = _dense(prob, phi, rho, s)
    assert np.allclose(Jh, PR.primal_matrix(prob, phi, rho, s), rtol=0, atol=1e-13 * np.abs(Jh).max())
    for seed in (1, 2):
        assert _pin_err(prob, phi, rho, s, Jh, seed) < 1e-8


def test_kernel_of_primal_schur_is_the_slice_constants(state):
    prob, phi, rho, s = state
    S = PR.primal_schur(prob, phi, rho, s).toarray()
    K, nf = prob.K, prob.nf
    assert np.allclose(S, S.T, rtol=0, atol=1e-12 * np.abs(S).max())
    ev = np.linalg.eigvalsh(S)
    # K+1 zero eigenvalues (one constant per slice), the rest positive
    assert np.all(np.abs(ev[:K + 1]) < 1e-10 * ev[-1])
    assert ev[K + 1] > 1e-8 * ev[-1]
    for k in range(K + 1):
        e = np.zeros((K + 1, nf))
        e[k] = 1.0
        assert np.abs(S @ e.ravel()).max() < 1e-10 * np.abs(S).max()


def test_pin_detects_planted_mistakes(state, monkeypatch):
    prob, phi, rho, s = state
    Jh = _dense(prob, phi, rho, s)
    orig_blocks, orig_proj, orig_zs = PR.kkt_blocks, PR.proj_matrix, PR._zero_sum_per_slice

    def neg_c(*a):                                    # C with the other sign
        A, B, C = orig_blocks(*a)
        return A, B, -C
    monkeypatch.setattr(PR, "kkt_blocks", neg_c)
    assert _pin_err(prob, phi, rho, s, Jh, 3) > 1e-3
    monkeypatch.setattr(PR, "kkt_blocks", orig_blocks)
    monkeypatch.setattr(PR, "proj_matrix", lambda p: sp.identity(p.K * p.nc, format="csr"))   # P dropped
    assert _pin_err(prob, phi, rho, s, Jh, 4) > 1e-3
    monkeypatch.setattr(PR, "proj_matrix", orig_proj)
    monkeypatch.setattr(PR, "_zero_sum_per_slice",
                        lambda p, x: np.array(x, dtype=float).reshape(p.K + 1, p.nf) + 1.0)    # not zero-sum
    assert _pin_err(prob, phi, rho, s, Jh, 5) > 1e-3
    monkeypatch.setattr(PR, "_zero_sum_per_slice", orig_zs)
