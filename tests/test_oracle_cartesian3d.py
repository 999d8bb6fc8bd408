"""Pins of the oracle on the three-dimensional workload (Sec. 4.1, fourth test
case): the n^3 grid of cubes, J = identity, faces as TPFA edges.

What fixes the values here, independently of the oracle's own formulas:
  * the unit-weight Laplacian equals h times the textbook 7-point graph
    Laplacian written as a sum of Kronecker products;
  * no-flux identities, R_E 1 = 1 and the overlap sums;
  * for a linear potential d . x the face gradients are d . n_e and R_T of
    their squares is a' |d|^2 on interior cells (6 faces of weight h^3 / 2);
  * uniform marginals: rho = 1, s = mu, phi linear in time, KE = 0;
  * a brute-force minimisation of the barrier problem on the 2^3 grid
    (independent of F and of the Jacobian);
  * the exact gap identity KE - D* = mu K dt |Omega| at a converged solution.
"""

import numpy as np
import pytest
import scipy.sparse as sp

import otinputs
from oracle.ipm import Problem, solve_ipm
from oracle.mesh import cartesian3d_mesh
from oracle.operators import Operators
from test_oracle_ipm import _brute_force


def _path_laplacian(n):
    main = np.full(n, 2.0)
    main[0] = main[-1] = 1.0
    return sp.diags([main, -np.ones(n - 1), -np.ones(n - 1)], [0, 1, -1])


def _centres(n):
    h = 1.0 / n
    c, rem = np.divmod(np.arange(n ** 3), n * n)
    b, a = np.divmod(rem, n)
    return (a + 0.5) * h, (b + 0.5) * h, (c + 0.5) * h


@pytest.mark.parametrize("n", [2, 4])
def test_no_flux_and_overlaps(n):
    o = Operators(cartesian3d_mesh(n))
    N = n ** 3
    assert o.mesh.n_fedge == 3 * n * n * (n - 1)
    assert np.abs(o.grad @ np.ones(N)).max() == 0.0
    assert np.abs(np.ones(N) @ o.div).max() < 1e-16
    assert np.allclose(o.RE @ np.ones(N), 1.0)
    assert np.allclose(np.asarray(o.Om.sum(1)).ravel(), o.a)
    assert np.allclose(np.asarray(o.Om.sum(0)).ravel(), o.ac)
    assert o.a.sum() == pytest.approx(1.0, rel=1e-14)


def test_unit_weight_laplacian_is_7_point():
    n = 5
    o = Operators(cartesian3d_mesh(n))
    L = o.laplacian(np.ones(o.mesh.n_fedge))
    I = sp.identity(n)
    T = _path_laplacian(n)
    # index (c n + b) n + a: kron(I_c, I_b, T_a) + kron(I_c, T_b, I_a) + kron(T_c, I_b, I_a)
    ref = sp.kron(sp.kron(I, I), T) + sp.kron(sp.kron(I, T), I) + sp.kron(sp.kron(T, I), I)
    assert abs(L - (1.0 / n) * ref).max() < 1e-12


def test_linear_potential():
    n = 6
    o = Operators(cartesian3d_mesh(n))
    x, y, z = _centres(n)
    d = np.array([0.3, -0.7, 0.45])
    g = o.grad @ (d[0] * x + d[1] * y + d[2] * z)
    m = o.mesh
    step = m.fe_L - m.fe_K
    for axis, off in enumerate((1, n, n * n)):
        assert np.allclose(g[step == off], -d[axis])
    rt = o.RT @ (g * g)
    c, rem = np.divmod(np.arange(n ** 3), n * n)
    b, a = np.divmod(rem, n)
    inner = (a > 0) & (a < n - 1) & (b > 0) & (b < n - 1) & (c > 0) & (c < n - 1)
    assert np.allclose(rt[inner], o.ac[inner] * (d @ d), rtol=1e-13)


def test_uniform_marginals_closed_form():
    m = cartesian3d_mesh(3)
    K = 2
    one = np.ones(m.n_coarse)
    prob = Problem(m, K, one, one)
    r = solve_ipm(prob, tol=1e-6, final_tol=1e-12)
    assert np.abs(r.rho - 1).max() < 1e-12
    assert np.abs(r.s - r.mu).max() < 1e-12
    assert np.abs(np.diff(r.phi, axis=0) + prob.dt * r.mu).max() < 1e-12
    assert abs(r.cost) < 1e-20


@pytest.mark.parametrize("K,mu", [(1, 0.2), (2, 0.05)])
def test_brute_force_barrier_minimum(K, mu):
    rng = np.random.default_rng(300 + K)
    m = cartesian3d_mesh(2)
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


def test_gaussian_pair_gap_identity_and_mass():
    n, K = 6, 5
    ri, rf = otinputs.gaussian3d_pair(n)
    prob = Problem(cartesian3d_mesh(n), K, ri, rf)
    r = solve_ipm(prob, tol=1e-6, final_tol=1e-11)
    assert r.converged
    expect = r.mu * K * prob.dt * 1.0
    assert abs(r.gap - expect) < 1e-7 * expect
    mass = r.rho @ prob.ops.ac
    assert np.abs(mass - 1.0).max() < 1e-13
    # the marginals' centres are d = (0.4, 0.4, 0.4) apart: 2 KE stays below
    # |d|^2 (the Gaussians are clipped by the cube, which shortens transport)
    assert 0.0 < 2 * r.cost < 0.48
