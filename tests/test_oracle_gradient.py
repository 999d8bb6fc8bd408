"""Pin of the oracle's cost gradient: central finite differences of the
oracle cost along mass-preserving directions."""

import numpy as np
import pytest

import otinputs
from oracle.mesh import structured_mesh
from oracle.ipm import Problem, solve_ipm
from oracle.gradient import cost_gradient


@pytest.mark.parametrize("n,K,mu", [(4, 2, 0.05), (8, 3, 0.01)])
def test_gradient_finite_differences(n, K, mu):
    ri, rf = otinputs.mixture_pair(n, 2, config=8, problem=n)
    m = structured_mesh(n)
    prob = Problem(m, K, ri, rf)
    r = solve_ipm(prob, tol=1e-8, final_tol=1e-13, mu_target=mu)
    g_in, g_f = cost_gradient(prob, r.phi, r.rho, r.s)
    ac = m.coarse_area
    assert abs(g_in @ ac) < 1e-12 * np.linalg.norm(g_in) * np.linalg.norm(ac)
    dirs = otinputs.mass_preserving_directions(ri, ac, 2, seed=5)
    eps = 1e-5
    for which in ("in", "f"):
        for d in dirs:
            vals = []
            for sgn in (1, -1):
                a = ri + sgn * eps * d if which == "in" else ri
                b = rf + sgn * eps * d if which == "f" else rf
                p = Problem(m, K, a, b)
                vals.append(solve_ipm(p, tol=1e-8, final_tol=1e-13, mu_target=mu,
                                      start=(r.phi, r.rho, r.s), mu_start=mu).cost)
            fd = (vals[0] - vals[1]) / (2 * eps)
            an = (g_in if which == "in" else g_f) @ d
            assert abs(fd - an) < 1e-6 * max(abs(an), 1e-3)
