"""Pins of the oracle's nonlinear system and interior-point solve."""

import numpy as np
import pytest

import otinputs
from oracle.mesh import structured_mesh, cartesian_mesh
from oracle.ipm import (Problem, residual, kkt_matrix, solve_ipm, kinetic_energy,
                        dual_value, residual_norm, initial_point, newton_step)


def _random_state(prob, rng):
    K, nf, nc = prob.K, prob.nf, prob.nc
    phi = rng.standard_normal((K + 1, nf))
    rho = rng.uniform(0.5, 2.0, (K, nc))
    s = rng.uniform(0.5, 2.0, (K, nc))
    return phi, rho, s


def _flat(F):
    return np.concatenate([x.ravel() for x in F])


@pytest.mark.parametrize("mk", [structured_mesh, cartesian_mesh])
def test_taylor_jacobian(mk):
    """|F(x + eps v) - F(x) - eps K v| = O(eps^2)  (Jacobian of Sec. 3)."""
    rng = np.random.default_rng(0)
    m = mk(4)
    prob = Problem(m, 3, rng.uniform(0.5, 1.5, m.n_coarse), rng.uniform(0.5, 1.5, m.n_coarse))
    phi, rho, s = _random_state(prob, rng)
    v = _random_state(prob, rng)
    J = kkt_matrix(prob, phi, rho, s)
    F0 = _flat(residual(prob, phi, rho, s, 0.1))
    Jv = J @ np.concatenate([x.ravel() for x in v])
    errs = []
    for eps in (1e-2, 1e-3, 1e-4):
        F1 = _flat(residual(prob, phi + eps * v[0], rho + eps * v[1], s + eps * v[2], 0.1))
        errs.append(np.linalg.norm(F1 - F0 - eps * Jv))
    assert errs[1] / errs[0] < 0.011 and errs[2] / errs[1] < 0.011


def test_hessian_symmetry_complex_step():
    """The (phi, rho) block of dF/dx, computed by complex-step differentiation
    of F itself, is symmetric (F is the gradient of a Lagrangian).  This pins
    the time-difference term of F_rho to Omega^T = J^T M."""
    rng = np.random.default_rng(1)
    m = structured_mesh(4)
    K = 2
    prob = Problem(m, K, rng.uniform(0.5, 1.5, m.n_coarse), rng.uniform(0.5, 1.5, m.n_coarse))
    phi, rho, s = _random_state(prob, rng)
    nphi, nrho = phi.size, rho.size
    n = nphi + nrho
    J = np.zeros((n, n))
    h = 1e-30
    for j in range(n):
        dphi = np.zeros(nphi, dtype=complex)
        drho = np.zeros(nrho, dtype=complex)
        if j < nphi:
            dphi[j] = 1j * h
        else:
            drho[j - nphi] = 1j * h
        F = residual(prob, phi + dphi.reshape(phi.shape), rho + drho.reshape(rho.shape), s, 0.0)
        J[:, j] = np.concatenate([F[0].ravel(), F[1].ravel()]).imag / h
    assert np.abs(J - J.T).max() < 1e-10 * np.abs(J).max()


@pytest.fixture(scope="module")
def gaussian16():
    n, K, ri, rf = otinputs.config_marginals(1)
    prob = Problem(structured_mesh(n), K, ri, rf)
    return prob, solve_ipm(prob, tol=1e-6, final_tol=1e-11)


def test_mass_per_slice(gaussian16):
    prob, r = gaussian16
    m0 = prob.ops.ac @ prob.rho_in
    assert np.abs(r.rho @ prob.ops.ac - m0).max() < 1e-14
    assert r.rho.min() > 0 and r.s.min() > 0


def test_gap_identity(gaussian16):
    """KE - D* = mu K dt |Omega| exactly at a solution of the relaxed system."""
    prob, r = gaussian16
    expect = r.mu * prob.K * prob.dt * 1.0
    assert r.converged
    assert abs(r.gap - expect) < 1e-9 * expect
    # mu schedule 0.2^l down to the first value below 1e-6
    assert r.mu == pytest.approx(0.2 ** 9)


def test_newton_counts(gaussian16):
    _, r = gaussian16
    assert len(r.newton_per_mu) == 10
    assert max(r.newton_per_mu[:-1]) <= 10


def test_split_step_rule_reaches_same_solution(gaussian16):
    """The relaxed system has one solution per mu (strictly convex barrier
    problem), so the primal / dual split of the positivity line search must
    end where the common step ends, with the gap identity intact."""
    prob, r = gaussian16
    r2 = solve_ipm(prob, tol=1e-6, final_tol=1e-11, step_rule="split")
    assert r2.converged
    assert abs(r2.cost - r.cost) < 1e-9 * r.cost
    assert np.abs(r2.rho - r.rho).max() < 1e-7 * np.abs(r.rho).max()
    expect = r2.mu * prob.K * prob.dt
    assert abs(r2.gap - expect) < 1e-9 * expect
    with pytest.raises(ValueError):
        solve_ipm(prob, tol=1e-6, step_rule="bogus")


def test_neighborhood_rule_reaches_same_solution(gaussian16):
    """The central-path neighbourhood step rule (rho s >= gamma mu kept in
    every cell) changes the path only: the solution of the final relaxed
    system is unique."""
    prob, r = gaussian16
    r2 = solve_ipm(prob, tol=1e-6, final_tol=1e-11, neighborhood=0.1)
    assert r2.converged
    assert abs(r2.cost - r.cost) < 1e-9 * r.cost
    assert np.abs(r2.rho - r.rho).max() < 1e-7 * np.abs(r.rho).max()


def test_central_step_keeps_products_above_bound():
    """central_step against a brute-force scan of the step length."""
    from oracle.ipm import central_step
    rng = np.random.default_rng(7)
    rho = rng.uniform(0.1, 2.0, 50)
    s = rng.uniform(0.1, 2.0, 50)
    drho = rng.standard_normal(50)
    ds = rng.standard_normal(50)
    gmu = 0.05
    t = central_step(rho, s, drho, ds, gmu, 1.0)
    ok = (rho * s) > gmu
    grid = np.linspace(0.0, 1.0, 20001)
    prod = (rho[ok, None] + grid[None, :] * drho[ok, None]) * (s[ok, None] + grid[None, :] * ds[ok, None])
    feasible = np.all(prod >= gmu, axis=0)
    t_scan = grid[np.argmin(feasible)] if not feasible.all() else 1.0
    assert abs(t - t_scan) <= 1.0 / 20000 + 1e-12
    assert np.all((rho[ok] + t * drho[ok]) * (s[ok] + t * ds[ok]) >= gmu * (1 - 1e-12))


def test_uniform_marginals_closed_form():
    """rho_in = rho_f = 1: rho = 1, s = mu, phi^k = -(k-1) dt mu + c, KE = 0."""
    for mk in (structured_mesh, cartesian_mesh):
        m = mk(4)
        K = 3
        one = np.ones(m.n_coarse)
        prob = Problem(m, K, one, one)
        r = solve_ipm(prob, tol=1e-6, final_tol=1e-12)
        assert np.abs(r.rho - 1).max() < 1e-12
        assert np.abs(r.s - r.mu).max() < 1e-12
        steps = np.diff(r.phi, axis=0)
        assert np.abs(steps + prob.dt * r.mu).max() < 1e-12
        assert abs(r.cost) < 1e-20
        assert r.gap == pytest.approx(r.mu * K / (K + 1), rel=1e-9)


# ---------------------------------------------------------------------------
# Brute force: minimise the barrier problem directly (no F, no Jacobian)
# ---------------------------------------------------------------------------

def _bf_operators(mesh):
    """Dense per-slice pieces built from the mesh arrays with plain loops."""
    nf, nc = mesh.n_fine, mesh.n_coarse
    Om = np.zeros((nf, nc))
    for i, j, a in zip(mesh.ov_fine, mesh.ov_coarse, mesh.ov_area):
        Om[i, j] += a
    return Om


def _bf_energy(mesh, Om, K, rho_in, rho_f, rho):
    """KE(rho) = 1/2 sum_k phi^k . Omega (rho^k - rho^{k-1}) where phi^k solves
    the rho~-weighted Laplacian system A^k phi^k = Omega (rho^k - rho^{k-1})/dt.
    Works for complex rho (complex-step derivatives)."""
    dt = 1.0 / (K + 1)
    nf = mesh.n_fine
    full = [rho_in] + [rho[k] for k in range(K)] + [rho_f]
    tot = 0.0
    for k in range(1, K + 2):
        A = np.zeros((nf, nf), dtype=complex)
        for e in range(mesh.n_fedge):
            i, j = mesh.fe_K[e], mesh.fe_L[e]
            rm = 0.5 * (full[k] + full[k - 1])
            rt = mesh.fe_lam[e] * rm[mesh.fe_rK[e]] + (1 - mesh.fe_lam[e]) * rm[mesh.fe_rL[e]]
            w = rt * mesh.fe_len[e] / mesh.fe_dist[e]
            A[i, i] += w
            A[j, j] += w
            A[i, j] -= w
            A[j, i] -= w
        b = Om @ (full[k] - full[k - 1]) / dt
        phi = np.zeros(nf, dtype=complex)
        phi[1:] = np.linalg.solve(A[1:, 1:], b[1:])
        tot = tot + 0.5 * phi @ (Om @ (full[k] - full[k - 1]))
    return tot


def _brute_force(mesh, K, rho_in, rho_f, mu):
    """Damped Newton on the barrier objective in a basis of the mass-preserving
    subspace; gradient by complex step (exact), Hessian by central differences
    of that gradient."""
    nc = mesh.n_coarse
    ac = mesh.coarse_area
    dt = 1.0 / (K + 1)
    Om = _bf_operators(mesh)
    m0 = ac @ rho_in
    # orthonormal basis of {v : a'^T v = 0}
    Q, _ = np.linalg.qr(np.column_stack([ac, np.eye(nc)[:, :-1]]))
    Z = Q[:, 1:]
    nz = Z.shape[1]
    base = np.full(nc, m0 / ac.sum())

    def rho_of(y):
        return base[None, :] + (Z @ y.reshape(K, nz).T).T

    def obj(y):
        r = rho_of(y)
        return _bf_energy(mesh, Om, K, rho_in, rho_f, r) - mu * dt * np.sum(ac[None, :] * np.log(r))

    def grad(y):
        g = np.zeros(y.size)
        for i in range(y.size):
            yy = y.astype(complex)
            yy[i] += 1e-30j
            g[i] = obj(yy).imag / 1e-30
        return g

    y = np.zeros(K * nz)
    for _ in range(60):
        g = grad(y)
        if np.linalg.norm(g) < 1e-14:
            break
        Hm = np.zeros((y.size, y.size))
        for i in range(y.size):
            e = np.zeros(y.size)
            e[i] = 1e-6
            Hm[:, i] = (grad(y + e) - grad(y - e)) / 2e-6
        Hm = 0.5 * (Hm + Hm.T)
        step = -np.linalg.solve(Hm, g)
        t = 1.0
        f0 = obj(y).real
        while True:
            yn = y + t * step
            if rho_of(yn).min() > 0 and obj(yn).real <= f0 + 1e-4 * t * (g @ step):
                break
            t *= 0.5
        y = yn
    r = rho_of(y)
    return r, _bf_energy(mesh, Om, K, rho_in, rho_f, r).real


@pytest.mark.parametrize("n,K,mu", [(2, 1, 0.3), (2, 2, 0.05), (4, 1, 0.1), (4, 2, 0.02)])
def test_brute_force_barrier_minimum(n, K, mu):
    rng = np.random.default_rng(100 + n + K)
    m = structured_mesh(n)
    ac = m.coarse_area
    ri = rng.uniform(0.2, 2.0, m.n_coarse)
    rf = rng.uniform(0.2, 2.0, m.n_coarse)
    ri /= ac @ ri
    rf /= ac @ rf
    prob = Problem(m, K, ri, rf)
    r = solve_ipm(prob, tol=1e-6, final_tol=1e-13, mu_target=mu)
    rho_bf, ke_bf = _brute_force(m, K, ri, rf, mu)
    assert np.abs(r.rho - rho_bf).max() < 1e-8 * np.abs(rho_bf).max()
    assert abs(r.cost - ke_bf) < 1e-8 * abs(ke_bf)


def test_translation_w2_convergence():
    """2 * cost -> |d|^2 = 0.09 for a translated narrow Gaussian, with the
    error decreasing under joint refinement of h and dt."""
    errs = []
    for n, K in [(8, 3), (16, 7), (24, 11)]:
        ri, rf = otinputs.translation_pair(n)
        prob = Problem(structured_mesh(n), K, ri, rf)
        r = solve_ipm(prob, tol=1e-6)
        errs.append(abs(2 * r.cost - 0.09))
    assert errs[0] > errs[1] > errs[2]
    assert errs[2] < 0.005


def test_reduced_direct_solve_equals_saddle_solve():
    """Eliminating delta rho through the diagonal C gives the solution of
    the full reduced saddle system J_s: Newton steps at the start point and
    at a later iterate agree, and so do whole continuations."""
    n, K = 8, 4
    ri, rf = otinputs.mixture_pair(n, 2, config=8, problem=1)
    prob = Problem(structured_mesh(n), K, ri, rf)
    p0, r0, s0 = initial_point(prob)
    it = solve_ipm(prob, tol=1e-6, mu_target=0.04)
    for phi, rho, s, mu in ((p0, r0, s0, 1.0), (it.phi, it.rho, it.s, 0.008)):
        a = newton_step(prob, phi, rho, s, mu, direct="saddle")
        b = newton_step(prob, phi, rho, s, mu, direct="reduced")
        for xa, xb in zip(a[:3], b[:3]):
            # phi up to the global constant (the kernel)
            d = xa - xb
            d = d - d.mean() if xa.shape[0] == K + 1 else d
            assert np.abs(d).max() < 1e-9 * np.abs(xa).max()
        assert abs(a[3] - b[3]) < 1e-12
    ra = solve_ipm(prob, tol=1e-6, final_tol=1e-10)
    rb = solve_ipm(prob, tol=1e-6, final_tol=1e-10, direct="reduced")
    assert abs(ra.cost - rb.cost) < 1e-10 * ra.cost
    assert np.abs(ra.rho - rb.rho).max() < 1e-8 * np.abs(ra.rho).max()
