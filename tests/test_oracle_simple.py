"""Pins of the oracle's SIMPLE preconditioner (Sec. 4.3) on the projected
saddle system (test infrastructure).

The SIMPLE factorisation inverts P_SIMPLE = [[D, B^T P^T], [P B, -P C P^T]]
with D = Diag(A): the projected saddle matrix with A replaced by its
diagonal.  That matrix is assembled here densely from the KKT blocks (which
the Taylor and symmetry tests pin), independently of the factorised form
the oracle applies, and apply_simple_exact(P_SIMPLE z) must return z on the
space where the projected system acts (rho block zero-sum per slice).
Planted mistakes in the oracle (S~ with the other sign, the diagonal D
replaced, the projector dropped from P B) each fail the pin.
"""

import numpy as np
import pytest

import otinputs
from oracle import simple as S
from oracle.bb import proj
from oracle.ipm import Problem, kkt_blocks, solve_ipm
from oracle.mesh import structured_mesh, cartesian3d_mesh


def _dense_simple(prob, phi, rho, s):
    A, B, C = kkt_blocks(prob, phi, rho, s)
    K, nc = prob.K, prob.nc
    m = K * nc
    P = np.zeros((m, m))
    for j in range(m):
        e = np.zeros(m)
        e[j] = 1.0
        P[:, j] = proj(prob, e.reshape(K, nc)).ravel()
    Bd, Cd = B.toarray(), C.toarray()
    return np.block([[np.diag(A.diagonal()), Bd.T @ P.T], [P @ Bd, -(P @ Cd @ P.T)]])


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


def _pin_err(prob, phi, rho, s, Pm, seed):
    rng = np.random.default_rng(seed)
    K, nf, nc = prob.K, prob.nf, prob.nc
    nphi = (K + 1) * nf
    x = rng.standard_normal((K + 1, nf))
    y = rng.standard_normal((K, nc))
    y -= y.mean(axis=1, keepdims=True)
    r = Pm @ np.concatenate([x.ravel(), y.ravel()])
    xx, yy = S.apply_simple_exact(prob, phi, rho, s, r[:nphi].reshape(K + 1, nf), r[nphi:].reshape(K, nc))
    return max(np.abs(xx - x).max() / np.abs(x).max(), np.abs(yy - y).max() / np.abs(y).max())


def test_inverse_of_dense_simple(state):
    prob, phi, rho, s = state
    Pm = _dense_simple(prob, phi, rho, s)
    assert np.allclose(Pm, S.simple_matrix(prob, phi, rho, s), rtol=0, atol=1e-13 * np.abs(Pm).max())
    for seed in (1, 2):
        assert _pin_err(prob, phi, rho, s, Pm, seed) < 1e-9


def test_pin_detects_planted_mistakes(state, monkeypatch):
    prob, phi, rho, s = state
    Pm = _dense_simple(prob, phi, rho, s)
    orig_schur, orig_blocks, orig_proj = S.simple_schur, S.simple_blocks, S.proj
    monkeypatch.setattr(S, "simple_schur", lambda *a: -orig_schur(*a))          # S~ with the other sign
    assert _pin_err(prob, phi, rho, s, Pm, 3) > 1e-3
    monkeypatch.setattr(S, "simple_schur", orig_schur)

    def doubled(*a):                                                              # D not the diagonal of A
        D, B, C = orig_blocks(*a)
        return 2.0 * D, B, C
    monkeypatch.setattr(S, "simple_blocks", doubled)
    assert _pin_err(prob, phi, rho, s, Pm, 4) > 1e-3
    monkeypatch.setattr(S, "simple_blocks", orig_blocks)
    monkeypatch.setattr(S, "proj", lambda p, v: np.array(v, dtype=float))        # projector dropped
    assert _pin_err(prob, phi, rho, s, Pm, 5) > 1e-3
    monkeypatch.setattr(S, "proj", orig_proj)
