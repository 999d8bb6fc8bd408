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
