"""The SIMPLE preconditioner (Sec. 4.3) of the HIP path against the oracle.

apply_schur_prec on a state using OT_PREC_SIMPLE with an inner tolerance of
1e-13 must equal the oracle's apply_simple_exact (dense S~ solve) to 1e-8
relative (the inner PCG stops on the residual; the conditioning of S~
turns it into a solution error).  A full interior-point solve with SIMPLE
must reach the oracle's solution: cost to 1e-6, rho and phi in area
weighted norms to 1e-5 (FP64 path; the final mu solved to 1e-10 on both
sides).
"""

import numpy as np
import pytest

import otinputs
from oracle.ipm import Problem, solve_ipm
from oracle.mesh import structured_mesh, cartesian3d_mesh
from oracle.simple import apply_simple_exact

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
ot = pytest.importorskip("paper_2209_00315_amd")

CASES = [
    ("tri8K3", lambda: structured_mesh(8), lambda: ot.Mesh.structured(8), 3),
    ("tri16K8", lambda: structured_mesh(16), lambda: ot.Mesh.structured(16), 8),
    ("cube4K3", lambda: cartesian3d_mesh(4), lambda: ot.Mesh.cartesian3d(4), 3),
]


@pytest.mark.parametrize("name,mk_o,mk_g,K", CASES, ids=[c[0] for c in CASES])
def test_simple_apply_exact_inner(name, mk_o, mk_g, K):
    mo = mk_o()
    ri = np.random.default_rng(1).uniform(0.2, 2.0, mo.n_coarse)
    rf = np.random.default_rng(2).uniform(0.2, 2.0, mo.n_coarse)
    ri /= mo.coarse_area @ ri
    rf /= mo.coarse_area @ rf
    print(f"[simple {name}] nf={mo.n_fine} nc={mo.n_coarse} K={K}", flush=True)
    prob = Problem(mo, K, ri, rf)
    r = solve_ipm(prob, tol=1e-6, mu_target=0.04)
    st = ot.State(mk_g(), ri, rf, K, precision="fp64", preconditioner="simple", eps_in_S=1e-13, max_inner=5000)
    st.import_(r.phi.ravel(), r.rho.ravel(), r.s.ravel(), r.mu)
    v = np.random.default_rng(3).standard_normal(st.N)
    nphi = (K + 1) * prob.nf
    # a right-hand side of the projected system: rho block zero-sum per slice
    d = v[nphi:].reshape(K, prob.nc)
    v[nphi:] = (d - d.mean(axis=1, keepdims=True)).ravel()
    z = st.apply_schur_prec(v)
    x, y = apply_simple_exact(prob, r.phi, r.rho, r.s, v[:nphi].reshape(K + 1, prob.nf),
                              v[nphi:].reshape(K, prob.nc))
    zy = z[nphi:].reshape(K, prob.nc)
    zy = zy - zy.mean(axis=1, keepdims=True)          # y is defined up to per-slice constants
    ex = np.abs(z[:nphi] - x.ravel()).max() / np.abs(x).max()
    ey = np.abs(zy - y).max() / np.abs(y).max()
    print(f"  rel err x {ex:.2e} y {ey:.2e}", flush=True)
    assert ex < 1e-8 and ey < 1e-8


def _norm_a(x, w):
    return np.sqrt(np.sum(w * x * x))


def test_full_solve_with_simple():
    n, K, ri, rf = otinputs.config_marginals(1)
    print(f"[simple full solve n={n} K={K}]", flush=True)
    prob = Problem(structured_mesh(n), K, ri, rf)
    ref = solve_ipm(prob, tol=1e-6, final_tol=1e-10)
    out = ot.solve(ot.Mesh.structured(n), ri, rf, K, tol=1e-6, final_tol=1e-10, precision="fp64",
                   preconditioner="simple", raise_on_error=False)
    st = out["stats"]
    cost_err = abs(out["cost"] - ref.cost) / ref.cost
    ac, a = prob.ops.ac, prob.ops.a
    rho_err = _norm_a(out["rho"].reshape(K, -1) - ref.rho, ac[None, :]) / _norm_a(ref.rho, ac[None, :])
    phi_err = _norm_a(out["phi"].reshape(K + 1, -1) - ref.phi, a[None, :]) / _norm_a(ref.phi, a[None, :])
    print(f"  rc {out['rc']} cost rel {cost_err:.2e} rho {rho_err:.2e} phi {phi_err:.2e} newton {st.newton_steps} "
          f"outer {st.outer_iters} outer/system {st.outer_iters / max(st.linear_systems, 1):.1f} "
          f"inner/outer {st.inner_S_iters / max(st.prec_applies, 1):.1f}", flush=True)
    assert out["rc"] == ot.OT_OK
    assert cost_err < 1e-6 and rho_err < 1e-5 and phi_err < 1e-5
