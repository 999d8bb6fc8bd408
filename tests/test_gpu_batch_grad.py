"""Batched solves and the differentiable cost on the GPU against the oracle.

- ot_solve_batched on problems of different grid sizes, K and mixtures gives
  the single-problem results (the members are independent) and the oracle's
  costs (1e-6 relative in FP64, 1e-5 in the mixed path).
- OTCost (torch.autograd.Function over ot_solve / ot_gradient): forward
  equals the oracle's cost; backward equals the oracle's gradient (envelope
  term plus adjoint solve) and central finite differences of the GPU cost
  along mass-preserving directions.
"""

import functools

import numpy as np
import pytest

import otinputs
from oracle.gradient import cost_gradient
from oracle.ipm import Problem, solve_ipm
from oracle.mesh import structured_mesh

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
ot = pytest.importorskip("paper_2209_00315_amd")

BATCH = [(8, 3, 1), (12, 4, 2), (16, 5, 3)]     # (n, K, mixture components)


def _say(*a):
    print(*a, flush=True)


@functools.lru_cache(maxsize=None)
def _oracle_cost(i):
    n, K, k = BATCH[i]
    ri, rf = otinputs.mixture_pair(n, k, config=4, problem=i)
    return solve_ipm(Problem(structured_mesh(n), K, ri, rf), tol=1e-6, final_tol=1e-10).cost


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-6), ("mixed", 1e-5)])
def test_solve_batched(precision, tol):
    meshes, ris, rfs, Ks, refs = [], [], [], [], []
    for i, (n, K, k) in enumerate(BATCH):
        ri, rf = otinputs.mixture_pair(n, k, config=4, problem=i)
        meshes.append(ot.Mesh.structured(n))
        ris.append(ri)
        rfs.append(rf)
        Ks.append(K)
        refs.append(_oracle_cost(i))
    _say(f"[batched {precision}] members {BATCH}")
    out = ot.solve_batched(meshes, ris, rfs, Ks, tol=1e-6, final_tol=1e-10, precision=precision)
    for i, (n, K, _) in enumerate(BATCH):
        single = ot.solve(meshes[i], ris[i], rfs[i], K, tol=1e-6, final_tol=1e-10, precision=precision)
        e_or = abs(out["cost"][i] - refs[i]) / refs[i]
        e_single = abs(out["cost"][i] - single["cost"]) / single["cost"]
        _say(f"  member {i} n={n} K={K}: cost rel err vs oracle {e_or:.2e}, vs single solve {e_single:.2e}")
        assert e_or < tol
        assert e_single < 1e-12
        assert np.abs(out["rho"][i] - single["rho"]).max() <= 1e-12 * np.abs(single["rho"]).max()


CFG4_SMALL = [0, 1, 3, 4, 6, 10, 14, 16]          # members of the 32-problem batch with n <= 48


def test_batch_of_the_32_problem_spec_concurrent_vs_sequential():
    """Eight members of the 32-problem batch (n 32 or 48, K 8 or 16, 1-4
    Gaussians): the concurrent batch (4 streams) equals the sequential one
    member by member (each member runs the same kernels on its own stream),
    and the 32^2, K = 8 member equals the oracle (mixed path, 1e-5)."""
    import time
    meshes, ris, rfs, Ks = [], [], [], []
    for p in CFG4_SMALL:
        n, K, ri, rf = otinputs.config_marginals(4, p)
        meshes.append(ot.Mesh.structured(n))
        ris.append(ri)
        rfs.append(rf)
        Ks.append(K)
    _say(f"[cfg4 subset] members {[otinputs.batch_spec(p) for p in CFG4_SMALL]}")
    t0 = time.perf_counter()
    seq = ot.solve_batched(meshes, ris, rfs, Ks, tol=1e-6, batch_streams=1)
    t1 = time.perf_counter()
    con = ot.solve_batched(meshes, ris, rfs, Ks, tol=1e-6, batch_streams=4)
    t2 = time.perf_counter()
    _say(f"  sequential {t1 - t0:.2f}s, 4 streams {t2 - t1:.2f}s (x{(t1 - t0) / (t2 - t1):.2f})")
    assert seq["rc"] == ot.OT_OK and con["rc"] == ot.OT_OK
    for i in range(len(CFG4_SMALL)):
        assert con["cost"][i] == seq["cost"][i]
        assert np.array_equal(con["rho"][i], seq["rho"][i])
    j = CFG4_SMALL.index(10)
    n, K, ri, rf = otinputs.config_marginals(4, 10)
    ref = solve_ipm(Problem(structured_mesh(n), K, ri, rf), tol=1e-6).cost
    err = abs(con["cost"][j] - ref) / ref
    _say(f"  member 10 (n={n}, K={K}) cost rel err vs oracle {err:.2e}")
    assert err < 1e-5


def _otcost(ri, rf, mesh, K, opts):
    a = torch.tensor(ri, dtype=torch.float64, device="cuda", requires_grad=True)
    b = torch.tensor(rf, dtype=torch.float64, device="cuda", requires_grad=True)
    c = ot.OTCost.apply(a, b, mesh, K, dict(opts))
    return a, b, c


def test_otcost_autograd():
    n, K = 8, 3
    ri, rf = otinputs.mixture_pair(n, 2, config=5, problem=0)
    prob = Problem(structured_mesh(n), K, ri, rf)
    ref = solve_ipm(prob, tol=1e-6, final_tol=1e-12)
    gi_ref, gf_ref = cost_gradient(prob, ref.phi, ref.rho, ref.s)
    mesh = ot.Mesh.structured(n)
    opts = dict(precision="fp64", final_tol=1e-12, eps_out=1e-12, eps_in_S=1e-8, eps_in_A=1e-8,
                max_inner_S=200, max_fgmres=600)
    _say(f"[otcost n={n} K={K}]")
    a, b, c = _otcost(ri, rf, mesh, K, opts)
    c.backward()
    e_cost = abs(c.item() - ref.cost) / ref.cost
    gi, gf = a.grad.cpu().numpy(), b.grad.cpu().numpy()
    e_gi = np.abs(gi - gi_ref).max() / np.abs(gi_ref).max()
    e_gf = np.abs(gf - gf_ref).max() / np.abs(gf_ref).max()
    _say(f"  cost rel err {e_cost:.2e}; gradient rel err in {e_gi:.2e} f {e_gf:.2e}")
    assert e_cost < 1e-9
    assert e_gi < 1e-6 and e_gf < 1e-6
    # central differences of the GPU cost along mass-preserving directions
    ac = prob.ops.ac
    eps = 1e-6
    for side, rho, g in (("in", ri, gi), ("f", rf, gf)):
        for d in otinputs.mass_preserving_directions(rho, ac, 2, seed=17 if side == "in" else 18):
            args_p = (ri + eps * d, rf) if side == "in" else (ri, rf + eps * d)
            args_m = (ri - eps * d, rf) if side == "in" else (ri, rf - eps * d)
            cp = _otcost(*args_p, mesh, K, opts)[2].item()
            cm = _otcost(*args_m, mesh, K, opts)[2].item()
            fd = (cp - cm) / (2 * eps)
            an = float(g @ d)
            err = abs(fd - an) / max(abs(an), 1e-3 * np.abs(g).max())
            _say(f"  FD rho_{side}: fd {fd:.6e} analytic {an:.6e} rel {err:.1e}")
            assert err < 1e-4


@pytest.mark.timeout(600)
def test_gradient_fd_member_of_the_differentiable_batch():
    """A member of the differentiable batch (128^2, K = 32, mixed path):
    ot_gradient against central differences along mass-preserving
    directions of rho_in and rho_f, for the cost of the relaxed problem at
    mu = 1.6e-3 (the continuation stopped there with mu_stop).  The
    perturbed problems start from the unperturbed solution
    (ot_state_import) and are solved at the same mu to the same residual;
    the solution of the relaxed system is unique, so this changes the path,
    not the result.  Below mu ~ 1e-4 the Newton systems of this
    size need hundreds of FGMRES iterations each, which puts eight
    perturbed solves beyond a test's time; the full continuation's gradient
    is checked against the oracle and finite differences at 8^2 above.
    Step 1e-4, central quotient; the base and the perturbed problems are
    solved to |F| <= 1e-12, since the quotient divides the cost's own
    error by the step: at |F| <= 1e-10 that error (about 1e-13 absolute)
    moved the quotient by up to 7e-3 of the derivative, and a smaller step
    made it worse, not better (the h^2 term is not the limit).  The adjoint
    solve of the gradient runs to eps_out = 1e-9: at the default 1e-5 its
    error reached 1e-3 of the smaller directional derivatives."""
    n, K, ri, rf = otinputs.config_marginals(5, 0)
    mesh = ot.Mesh.structured(n)
    mu_stop = 1.6e-3 * (1 + 1e-9)
    opts = dict(precision="mixed", final_tol=1e-12, mu_stop=mu_stop)
    _say(f"[gradient FD n={n} K={K} mu_stop {mu_stop:.3e}]")
    st = ot.State(mesh, ri, rf, K, **opts)
    rc, stats = st.solve(1e-6)
    st.set_options(eps_out=1e-9)              # adjoint solve well below the quotient's accuracy
    gi, gf = st.gradient()
    phi, rho, s, mu = st.export()
    assert abs(mu - 1.6e-3) < 1e-12
    _say(f"  base cost {stats.cost:.12g} newton {stats.newton_steps} simple systems {stats.simple_systems}")
    ac = np.full(mesh.n_coarse, 0.5 / (n // 2) ** 2)              # coarse triangle areas
    eps = 1e-4

    def cost(a, b):
        p = ot.State(mesh, a, b, K, **opts)
        p.import_(phi, rho, s, mu)
        rc2, st2 = p.solve(1e-6)
        assert abs(st2.mu - mu) < 1e-15
        return st2.cost

    for side, r0, g in (("in", ri, gi), ("f", rf, gf)):
        for d in otinputs.mass_preserving_directions(r0, ac, 2, seed=51 if side == "in" else 52):
            assert abs(ac @ d) < 1e-14
            plus = (ri + eps * d, rf) if side == "in" else (ri, rf + eps * d)
            minus = (ri - eps * d, rf) if side == "in" else (ri, rf - eps * d)
            fd = (cost(*plus) - cost(*minus)) / (2 * eps)
            an = float(g @ d)
            err = abs(fd - an) / max(abs(an), 1e-3 * np.abs(g).max())
            _say(f"  FD rho_{side}: fd {fd:.6e} analytic {an:.6e} rel {err:.1e}")
            assert err < 1e-3
