"""Pins of the projected system and the BB preconditioner (Sec. 4.4)."""

import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import otinputs
from oracle.mesh import structured_mesh
from oracle.ipm import (Problem, solve_ipm, kkt_blocks, saddle_matrix, newton_rhs,
                        solve_saddle_direct, edge_density)
from oracle.bb import (proj, proj_t, proj_matrix, projected_matrix, apply_bb_exact,
                       btilde, coarse_laplacian_blocks, recover)


@pytest.fixture(scope="module")
def state8():
    """An interior-point iterate at mu = 0.04 on the 8 x 8 grid, K = 3."""
    n, K = 8, 3
    ri, rf = otinputs.mixture_pair(n, 2, config=9)
    prob = Problem(structured_mesh(n), K, ri, rf)
    r = solve_ipm(prob, tol=1e-8, mu_target=0.04)
    return prob, r.phi, r.rho, r.s, r.mu


def test_projector_identities():
    rng = np.random.default_rng(0)
    prob = Problem(structured_mesh(4), 3, np.ones(8), np.ones(8))
    P = proj_matrix(prob).toarray()
    assert np.allclose(P @ P, P, atol=1e-15)                         # P^2 = P
    Eb = np.kron(np.eye(prob.K), np.ones((1, prob.nc)))               # E'
    Mc = np.kron(np.eye(prob.K), np.diag(prob.ops.ac))
    assert np.allclose(Eb @ Mc @ Eb.T, np.eye(prob.K) * 1.0)          # E'M'E'^T = |Omega| I
    assert np.allclose(P @ Mc @ Eb.T, 0)                              # Ker P = Im M'E'^T
    v = rng.standard_normal((prob.K, prob.nc))
    assert np.allclose(proj(prob, v).ravel(), P @ v.ravel())
    assert np.allclose(proj_t(prob, v).ravel(), P.T @ v.ravel())


def test_kernels(state8):
    """Ker A = per-slice constants (dim K+1), Ker A in Ker P B, and the
    projected matrix has kernel dimension 2K+1 (Sec. 3, Sec. 4.4.2)."""
    prob, phi, rho, s, mu = state8
    K, nf, nc = prob.K, prob.nf, prob.nc
    A, B, C = kkt_blocks(prob, phi, rho, s)
    P = proj_matrix(prob)
    ones = np.kron(np.eye(K + 1), np.ones((nf, 1)))
    assert np.abs(A @ ones).max() < 1e-12
    assert np.abs(P @ (B @ ones)).max() < 1e-10
    # B restricted to Ker A is the time difference of slice constants
    Bk = B @ ones
    assert np.linalg.matrix_rank(Bk, tol=1e-8) == K
    JP = projected_matrix(prob, phi, rho, s).toarray()
    sv = np.linalg.svd(JP, compute_uv=False)
    assert np.sum(sv < 1e-10 * sv[0]) == 2 * K + 1
    # Im(B^T P^T) is orthogonal to Ker A
    assert np.abs(ones.T @ (B.T @ P.T).toarray()).max() < 1e-10


def test_ideal_schur_two_steps(state8):
    """With the exact Schur complement, the block upper-triangular
    preconditioner in the sign convention of the printed pseudo-Schur system
    makes J_P P^-1 equal to identity plus nilpotent on the range of J_P, so
    GMRES needs two iterations."""
    prob, phi, rho, s, mu = state8
    K, nf = prob.K, prob.nf
    A, B, C = kkt_blocks(prob, phi, rho, s)
    P = proj_matrix(prob).toarray()
    Ad = A.toarray()
    Ap = np.linalg.pinv(Ad, rcond=1e-12)
    Bd, Cd = B.toarray(), C.toarray()
    Shat = P @ (Cd + Bd @ Ap @ Bd.T) @ P.T
    JP = projected_matrix(prob, phi, rho, s).toarray()
    n_phi = (K + 1) * nf

    def prec(v):
        c, d = v[:n_phi], v[n_phi:]
        y = np.linalg.lstsq(Shat, -P @ d, rcond=1e-12)[0]
        y = P.T @ y
        x = Ap @ (c - Bd.T @ y)
        return np.concatenate([x, y])

    f, g, h, gt = newton_rhs(prob, phi, rho, s, mu * 0.2)
    b = np.concatenate([f.ravel(), (P @ gt.ravel())])
    # two Arnoldi steps on J_P prec
    V = [b / np.linalg.norm(b)]
    Hm = np.zeros((3, 2))
    for j in range(2):
        w = JP @ prec(V[j])
        for i in range(j + 1):
            Hm[i, j] = V[i] @ w
            w = w - Hm[i, j] * V[i]
        Hm[j + 1, j] = np.linalg.norm(w)
        V.append(w / Hm[j + 1, j] if Hm[j + 1, j] > 0 else w)
    e1 = np.zeros(3)
    e1[0] = np.linalg.norm(b)
    y = np.linalg.lstsq(Hm, e1, rcond=None)[0]
    res = np.linalg.norm(e1 - Hm @ y) / np.linalg.norm(b)
    assert res < 1e-8
    # identity plus nilpotent: (T - I)^2 vanishes on the range
    T = JP @ np.column_stack([prec(e) for e in np.eye(JP.shape[0])])
    R = T - np.eye(T.shape[0])
    Q = np.linalg.svd(JP)[0][:, : JP.shape[0] - (2 * K + 1)]
    assert np.abs((R @ R) @ Q).max() < 1e-6 * np.abs(T).max()


def _translation_state(n, K, shift=0.3):
    """rho^k: a Gaussian translated with unit speed along x, phi^k = d . x:
    the continuity residual is small and grad^2 phi = 0 (Prop. 1 terms)."""
    dt = 1.0 / (K + 1)
    x0 = 0.5 - shift / 2
    mk = lambda c: otinputs.structured_marginal(otinputs.gaussian(c, 0.5, 0.12), n)
    ri, rf = mk(x0), mk(x0 + shift)
    rho = np.stack([mk(x0 + shift * (k + 1) * dt) for k in range(K)])
    h = 1.0 / n
    b, a = np.divmod(np.arange(n * n), n)
    xc = (a + 0.5) * h
    phi = np.tile(shift * xc, (K + 1, 1))
    prob = Problem(structured_mesh(n), K, ri, rf)
    return prob, phi, rho, np.ones_like(rho)


def _lap_pinv_solve(L, b):
    """L^+ b for a connected graph Laplacian L and b orthogonal to the
    constants: the zero-mean solution, from the system grounded at node 0."""
    L = sp.csc_matrix(L)
    x = np.zeros(L.shape[0])
    x[1:] = spla.spsolve(L[1:, 1:], b[1:])
    return x - x.mean()


def _commutator_ratio(prob, phi, rho, variant):
    """Relative gap between A^+ B^T y and -M^-1 B~ A~^+ M' y on a smooth,
    zero-mass y (the approximation the BB preconditioner rests on), compared
    in the potential space after removing per-slice means."""
    o, K = prob.ops, prob.K
    _, B, _ = kkt_blocks(prob, phi, rho, np.ones_like(rho))
    rt = edge_density(prob, rho)
    Bt = btilde(prob, phi)
    if variant == "flip":
        # misread: transport part of B~ with the opposite sign
        Bt0 = btilde(prob, np.zeros_like(phi))
        Bt = Bt0 - (Bt - Bt0)
    n = int(round(np.sqrt(prob.nc * 2)))
    H = 2.0 / n
    cx = np.array([((A_ + 0.5) * H, (B_ + 0.5) * H)
                   for B_ in range(n // 2) for A_ in range(n // 2) for _ in range(2)])
    t = np.arange(1, K + 1) / (K + 1)
    y = proj_t(prob, np.outer(np.sin(np.pi * t), np.cos(np.pi * cx[:, 0]) * np.cos(np.pi * cx[:, 1])))
    BTy = (B.T @ y.ravel()).reshape(K + 1, -1)
    # both right-hand sides are orthogonal to the constants: 1^T (B^T y)^k
    # pairs y with B 1_k, a multiple of a' per slice, and a'^T y^k = 0
    assert np.abs(BTy.sum(axis=1)).max() < 1e-10 * np.abs(BTy).max()
    Y = np.stack([_lap_pinv_solve(o.laplacian(rt[k]), BTy[k]) for k in range(K + 1)])
    w = np.stack([_lap_pinv_solve(o.coarse_laplacian(rho[k]), o.ac * y[k]) for k in range(K)])
    X = -(Bt @ w.ravel()).reshape(K + 1, -1) / o.a[None, :]
    X = X - X.mean(1, keepdims=True)
    Y = Y - Y.mean(1, keepdims=True)
    return np.linalg.norm(X - Y) / np.linalg.norm(Y)


def test_commutator_translation():
    """For a translation the neglected terms of Prop. 1 vanish, so
    A^+ B^T ~= -M^-1 B~ A~^+ M' holds up to discretisation error: the gap
    shrinks under joint refinement of h and dt.  Flipping the sign of the
    transport part of B~ leaves an O(1) gap that does not shrink."""
    ok = [_commutator_ratio(*_translation_state(n, K)[:3], "ok") for n, K in [(16, 7), (32, 15)]]
    bad = [_commutator_ratio(*_translation_state(n, K)[:3], "flip") for n, K in [(16, 7), (32, 15)]]
    assert ok[1] < 0.7 * ok[0]
    assert bad[1] > 1.5 * ok[1] and bad[1] > 0.9 * bad[0]


def test_recovery_matches_direct_solve(state8):
    """A solution of J_P, shifted by kernel elements, recovers the solution of
    the reduced Newton system J_s up to the global constant (Sec. 4.4.1-2)."""
    prob, phi, rho, s, mu = state8
    K, nf, nc = prob.K, prob.nf, prob.nc
    f, g, h, gt = newton_rhs(prob, phi, rho, s, mu * 0.2)
    Js = saddle_matrix(prob, phi, rho, s)
    x = solve_saddle_direct(Js, np.concatenate([f.ravel(), gt.ravel()]))
    dphi_ref = x[: (K + 1) * nf].reshape(K + 1, nf)
    drho_ref = x[(K + 1) * nf:].reshape(K, nc)
    JP = projected_matrix(prob, phi, rho, s).toarray()
    b = np.concatenate([f.ravel(), proj(prob, gt).ravel()])
    xp = np.linalg.lstsq(JP, b, rcond=1e-13)[0]
    rng = np.random.default_rng(3)
    dphi_hat = xp[: (K + 1) * nf].reshape(K + 1, nf) + rng.standard_normal((K + 1, 1))
    drho = xp[(K + 1) * nf:].reshape(K, nc) + rng.standard_normal((K, 1))
    dphi, drho2 = recover(prob, phi, rho, s, dphi_hat, drho, gt)
    c = (dphi - dphi_ref).mean()
    assert np.abs(dphi - c - dphi_ref).max() < 1e-9 * np.abs(dphi_ref).max()
    assert np.abs(drho2 - drho_ref).max() < 1e-9 * np.abs(drho_ref).max()


def test_bb_preconditioned_gmres(state8):
    """The exact-inner BB preconditioner cuts GMRES iterations on J_P."""
    prob, phi, rho, s, mu = state8
    K, nf = prob.K, prob.nf
    n_phi = (K + 1) * nf
    JP = projected_matrix(prob, phi, rho, s)
    f, g, h, gt = newton_rhs(prob, phi, rho, s, mu * 0.2)
    b = np.concatenate([f.ravel(), proj(prob, gt).ravel()])

    def count(M):
        it = [0]

        def cb(_):
            it[0] += 1
        spla.gmres(JP, b, M=M, rtol=1e-8, restart=400, maxiter=400, callback=cb,
                   callback_type="pr_norm")
        return it[0]

    def pbb(v):
        x, y = apply_bb_exact(prob, phi, rho, s, v[:n_phi].reshape(K + 1, nf),
                              v[n_phi:].reshape(K, prob.nc))
        return np.concatenate([x.ravel(), y.ravel()])

    M = spla.LinearOperator(JP.shape, matvec=pbb)
    it_bb = count(M)
    it_none = count(None)
    assert it_bb < 40 and it_bb * 3 < it_none
