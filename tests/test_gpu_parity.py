"""Parity of the HIP path (called through the C ABI) against the FP64 oracle.

Tolerances: operators are FP64 on both sides and differ only by summation
order, so they must agree to 1e-12 relative.  Preconditioner applications
with inner tolerances of 1e-13 agree with the oracle's direct inner solves
to 1e-8 relative (the inner GMRES stops on the residual; the pseudo-Schur
operator's condition number converts it into a solution error).  Full
solves compare the cost to 1e-6 (FP64 path) and 1e-5 (mixed path), rho and
phi in area-weighted norms to 1e-5 / 1e-4, with both sides solving the last
mu to 1e-10.
"""

import numpy as np
import pytest

import otinputs
from oracle.mesh import structured_mesh, cartesian_mesh, cartesian3d_mesh, mesh_from_arrays
from oracle.ipm import Problem, residual, solve_ipm, newton_step, renormalize, initial_point
from oracle.bb import projected_matrix, apply_bb_exact
from oracle.gradient import cost_gradient

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

ot = pytest.importorskip("paper_2209_00315_amd")


def _say(*a):
    print(*a, flush=True)


def _random_state(prob, seed):
    rng = np.random.default_rng(seed)
    K, nf, nc = prob.K, prob.nf, prob.nc
    phi = rng.standard_normal((K + 1, nf)) * 0.1
    rho = rng.uniform(0.5, 2.0, (K, nc))
    s = rng.uniform(0.1, 1.0, (K, nc))
    return phi, rho, s


def _gpu_state(mesh, prob, phi, rho, s, mu, **opts):
    st = ot.State(mesh, prob.rho_in, prob.rho_f, prob.K, device=False, **opts)
    st.import_(phi.ravel(), rho.ravel(), s.ravel(), mu)
    return st


CASES = [
    ("tri8K3", lambda: structured_mesh(8), lambda: ot.Mesh.structured(8), 3),
    ("tri16K8", lambda: structured_mesh(16), lambda: ot.Mesh.structured(16), 8),
    ("cart6K1", lambda: cartesian_mesh(6), lambda: ot.Mesh.structured(6, cartesian=True), 1),
    ("tri2K2", lambda: structured_mesh(2), lambda: ot.Mesh.structured(2), 2),
    ("cube4K3", lambda: cartesian3d_mesh(4), lambda: ot.Mesh.cartesian3d(4), 3),
    # several blocks per slice and a ragged last block: 1024 fine cells, 512
    # coarse cells, 33 potential levels
    ("tri32K32", lambda: structured_mesh(32), lambda: ot.Mesh.structured(32), 32),
]


def _random_generic(seed):
    d = otinputs.random_mesh_arrays(300, 70, seed)
    return mesh_from_arrays(d), ot.Mesh.from_arrays(**d)


@pytest.fixture(params=CASES + [("generic300", None, None, 4)], ids=lambda c: c[0])
def case(request):
    name, mk_o, mk_g, K = request.param
    if mk_o is None:
        mo, mg = _random_generic(7)
    else:
        mo, mg = mk_o(), mk_g()
    ri = np.random.default_rng(1).uniform(0.2, 2.0, mo.n_coarse)
    rf = np.random.default_rng(2).uniform(0.2, 2.0, mo.n_coarse)
    ri /= mo.coarse_area @ ri
    rf /= mo.coarse_area @ rf
    _say(f"[case {name}] nf={mo.n_fine} nc={mo.n_coarse} K={K}")
    return name, Problem(mo, K, ri, rf), mg


def test_residual_parity(case):
    name, prob, mg = case
    phi, rho, s = _random_state(prob, 10)
    st = _gpu_state(mg, prob, phi, rho, s, 0.3)
    F, nrm = st.residual()
    Fo = residual(prob, phi, rho, s, 0.3)
    ref = np.concatenate([x.ravel() for x in Fo])
    err = np.abs(F - ref).max() / np.abs(ref).max()
    _say(f"  residual rel err {err:.2e}")
    assert err < 1e-12
    assert abs(nrm - np.linalg.norm(ref)) < 1e-12 * np.linalg.norm(ref)


def test_apply_saddle_parity(case):
    name, prob, mg = case
    phi, rho, s = _random_state(prob, 11)
    st = _gpu_state(mg, prob, phi, rho, s, 0.3)
    x = np.random.default_rng(12).standard_normal(st.N)
    y = st.apply_saddle(x)
    ref = projected_matrix(prob, phi, rho, s) @ x
    err = np.abs(y - ref).max() / np.abs(ref).max()
    _say(f"  apply_saddle rel err {err:.2e}")
    assert err < 1e-12


_ITERATES = {}


def _iterate_at_004(name, prob):
    """The oracle's solution at mu = 0.04, once per case (both precisions)."""
    if name not in _ITERATES:
        _ITERATES[name] = solve_ipm(prob, tol=1e-6, mu_target=0.04)
    return _ITERATES[name]


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-8), ("mixed", 2e-4)])
def test_schur_prec_exact_inner(case, precision, tol):
    name, prob, mg = case
    r = _iterate_at_004(name, prob)                      # an interior-point iterate
    phi, rho, s = r.phi, r.rho, r.s
    inner = 1e-13 if precision == "fp64" else 1e-6
    st = _gpu_state(mg, prob, phi, rho, s, r.mu, precision=precision, eps_in_S=inner, eps_in_A=inner,
                    max_inner=2000, max_inner_S=2000, inner_restart=40)
    r = np.random.default_rng(14).standard_normal(st.N)
    z = st.apply_schur_prec(r)
    K, nf = prob.K, prob.nf
    n_phi = (K + 1) * nf
    x, y = apply_bb_exact(prob, phi, rho, s, r[:n_phi].reshape(K + 1, nf), r[n_phi:].reshape(K, prob.nc))
    ex = np.abs(z[:n_phi] - x.ravel()).max() / np.abs(x).max()
    ey = np.abs(z[n_phi:] - y.ravel()).max() / np.abs(y).max()
    _say(f"  schur_prec[{precision}] rel err x {ex:.2e} y {ey:.2e}")
    assert ex < tol and ey < tol


def test_newton_step_parity(case):
    """One Newton step from the start point with tight inner/outer tolerances
    equals the oracle's direct step."""
    name, prob, mg = case
    st = ot.State(mg, prob.rho_in, prob.rho_f, prob.K, precision="fp64", eps_out=1e-12, eps_in_S=1e-6,
                  eps_in_A=1e-6, max_fgmres=600, restart=60, max_inner_S=200, tol=1e-14)
    rc, stats, res = st.newton_step()
    phi, rho, s, mu = st.export()
    p0, r0, s0 = initial_point(prob)
    p1, r1, s1, _ = newton_step(prob, p0, r0, s0, 1.0)
    r1 = renormalize(prob, r1, float(prob.ops.ac @ prob.rho_in))
    er = np.abs(rho - r1.ravel()).max() / np.abs(r1).max()
    es = np.abs(s - s1.ravel()).max() / np.abs(s1).max()
    dp = phi.reshape(prob.K + 1, -1) - p1
    ep = np.abs(dp - dp.mean()).max() / max(np.abs(p1).max(), 1e-300)
    _say(f"  newton step: fgmres {stats.outer_iters} rel err rho {er:.2e} s {es:.2e} phi {ep:.2e}")
    assert er < 1e-8 and es < 1e-8 and ep < 1e-8


def _norm_a(x, w):
    return np.sqrt(np.sum(w * x * x))


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_full_solve_gaussian16(precision):
    """The 16 x 16 Gaussian pair, K = 8: cost, rho, phi against the oracle."""
    n, K, ri, rf = otinputs.config_marginals(1)
    _say(f"[full solve n={n} K={K} {precision}]")
    prob = Problem(structured_mesh(n), K, ri, rf)
    ref = solve_ipm(prob, tol=1e-6, final_tol=1e-10)
    mesh = ot.Mesh.structured(n)
    out = ot.solve(mesh, ri, rf, K, tol=1e-6, final_tol=1e-10, precision=precision)
    st = out["stats"]
    cost_err = abs(out["cost"] - ref.cost) / ref.cost
    ac = prob.ops.ac
    rho = out["rho"].reshape(K, -1)
    rho_err = _norm_a(rho - ref.rho, ac[None, :]) / _norm_a(ref.rho, ac[None, :])
    phi = out["phi"].reshape(K + 1, -1)
    a = prob.ops.a
    phi_err = _norm_a(phi - ref.phi, a[None, :]) / _norm_a(ref.phi, a[None, :])
    _say(f"  cost {out['cost']:.12f} ref {ref.cost:.12f} rel {cost_err:.2e} rho {rho_err:.2e} "
         f"phi {phi_err:.2e} newton {st.newton_steps} outer {st.outer_iters} gap {st.gap:.3e}")
    ctol, ftol = (1e-6, 1e-5) if precision == "fp64" else (1e-5, 1e-4)
    assert cost_err < ctol and rho_err < ftol and phi_err < ftol
    assert st.ip_steps == 10 and st.failures == 0


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_full_solve_cube8(precision):
    """The three-dimensional workload at its first size: 8^3 cubes, K+1 = 8,
    Gaussians of variance 0.1 at (0.3, 0.3, 0.3) -> (0.7, 0.7, 0.7)."""
    n, K = 8, 7
    ri, rf = otinputs.gaussian3d_pair(n)
    _say(f"[full solve cube n={n} K={K} {precision}]")
    prob = Problem(cartesian3d_mesh(n), K, ri, rf)
    ref = solve_ipm(prob, tol=1e-6, final_tol=1e-10)
    out = ot.solve(ot.Mesh.cartesian3d(n), ri, rf, K, tol=1e-6, final_tol=1e-10, precision=precision)
    st = out["stats"]
    cost_err = abs(out["cost"] - ref.cost) / ref.cost
    ac, a = prob.ops.ac, prob.ops.a
    rho_err = _norm_a(out["rho"].reshape(K, -1) - ref.rho, ac[None, :]) / _norm_a(ref.rho, ac[None, :])
    phi_err = _norm_a(out["phi"].reshape(K + 1, -1) - ref.phi, a[None, :]) / _norm_a(ref.phi, a[None, :])
    _say(f"  cost {out['cost']:.12f} ref {ref.cost:.12f} rel {cost_err:.2e} rho {rho_err:.2e} phi {phi_err:.2e} "
         f"newton {st.newton_steps} outer {st.outer_iters}")
    ctol, ftol = (1e-6, 1e-5) if precision == "fp64" else (1e-5, 1e-4)
    assert out["rc"] == ot.OT_OK
    assert cost_err < ctol and rho_err < ftol and phi_err < ftol


def test_full_solve_generic_mesh():
    mo, mg = _random_generic(21)
    K = 3
    rng = np.random.default_rng(5)
    ri = rng.uniform(0.2, 2.0, mo.n_coarse)
    rf = rng.uniform(0.2, 2.0, mo.n_coarse)
    ri /= mo.coarse_area @ ri
    rf /= mo.coarse_area @ rf
    _say(f"[full solve generic nf={mo.n_fine} K={K}]")
    prob = Problem(mo, K, ri, rf)
    ref = solve_ipm(prob, tol=1e-6, final_tol=1e-10)
    out = ot.solve(mg, ri, rf, K, tol=1e-6, final_tol=1e-10, precision="fp64")
    err = abs(out["cost"] - ref.cost) / ref.cost
    _say(f"  cost rel err {err:.2e}")
    assert err < 1e-6


def test_gradient_parity():
    n, K = 8, 3
    ri, rf = otinputs.mixture_pair(n, 2, config=8, problem=n)
    _say(f"[gradient n={n} K={K}]")
    prob = Problem(structured_mesh(n), K, ri, rf)
    mu = 5.12e-7
    ref = solve_ipm(prob, tol=1e-6, final_tol=1e-12)
    gi_ref, gf_ref = cost_gradient(prob, ref.phi, ref.rho, ref.s)
    mesh = ot.Mesh.structured(n)
    st = ot.State(mesh, ri, rf, K, precision="fp64", eps_out=1e-12, eps_in_S=1e-8, eps_in_A=1e-8,
                  max_fgmres=600, restart=60, max_inner_S=200)
    st.import_(ref.phi.ravel(), ref.rho.ravel(), ref.s.ravel(), ref.mu)
    gi, gf = st.gradient()
    e1 = np.abs(gi - gi_ref).max() / np.abs(gi_ref).max()
    e2 = np.abs(gf - gf_ref).max() / np.abs(gf_ref).max()
    _say(f"  gradient rel err in {e1:.2e} f {e2:.2e}")
    assert e1 < 1e-7 and e2 < 1e-7


def test_error_codes_on_device_states():
    mesh = ot.Mesh.structured(8)
    nc = mesh.n_coarse
    ri = np.ones(nc)
    with pytest.raises(ot.OTError) as e:
        ot.State(mesh, ri, 2 * ri, 3)
    assert e.value.code == ot.OT_EMASS
    bad = ri.copy()
    bad[3] = -1
    with pytest.raises(ot.OTError) as e:
        ot.State(mesh, bad, ri, 3)
    assert e.value.code == ot.OT_ENEG
    bad[3] = np.nan
    with pytest.raises(ot.OTError) as e:
        ot.State(mesh, bad, ri, 3)
    assert e.value.code == ot.OT_ENEG
    # forced non-convergence: FGMRES cap of 1 -> OT_ELINSOLVE, state untouched
    ga, gb = otinputs.gaussian_pair(8)
    st = ot.State(mesh, ga, gb, 3, max_fgmres=1, precision="fp64")
    before = st.export()
    rc, stats, _ = st.newton_step(raise_on_error=False)
    after = st.export()
    assert rc == ot.OT_ELINSOLVE
    assert np.array_equal(before[1], after[1])
    # Newton cap of 1 at a tight tolerance -> OT_ENEWTON from ot_solve
    ri2, rf2 = otinputs.gaussian_pair(8)
    out = ot.solve(mesh, ri2, rf2, 3, tol=1e-6, max_newton=1, raise_on_error=False)
    assert out["rc"] == ot.OT_ENEWTON
