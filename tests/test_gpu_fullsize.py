"""Parity at the benchmark's full size (256 x 256 grid, K = 64, 5-Gaussian
mixtures plus a 1e-3 background) in the launch configuration bench.py times
(device tensors, mixed precision).

The first interior-point step (mu = 1) is solved on the GPU.  At that
iterate the oracle evaluates, at full size, what it can compute directly:
the residual vector (FP64 on both sides, so it must agree to rounding), the
kinetic energy and the dual value.  Properties that hold at any size are
checked too: the gap identity KE - D* = mu K dt |Omega| of a solution of the
relaxed system, the per-slice mass of rho, and positivity of rho and s.
"""

import numpy as np
import pytest

import otinputs
from oracle.ipm import Problem, dual_value, kinetic_energy, normalize_phi, residual
from oracle.mesh import structured_mesh

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
ot = pytest.importorskip("paper_2209_00315_amd")


def test_first_mu_at_full_size():
    n, K, ri, rf = otinputs.config_marginals(3)
    print(f"[full size] n={n} K={K} mixed, mu = 1", flush=True)
    mesh = ot.Mesh.structured(n)
    dev = torch.device("cuda")
    st = ot.State(mesh, torch.as_tensor(ri, device=dev), torch.as_tensor(rf, device=dev), K, device=True,
                  precision="mixed", mu_stop=1.0)
    rc, _ = st.solve(1e-6)
    assert rc == ot.OT_OK
    F_gpu, nrm = st.residual()
    phi, rho, s, mu = st.export()
    cost, dual, _ = st.outputs()
    torch.cuda.synchronize()
    assert mu == 1.0 and nrm <= 1e-6
    phi, rho, s = (x.cpu().numpy() for x in (phi, rho, s))
    F_gpu = F_gpu.cpu().numpy()

    prob = Problem(structured_mesh(n), K, ri, rf)
    nf, nc = prob.nf, prob.nc
    P, R, S = phi.reshape(K + 1, nf), rho.reshape(K, nc), s.reshape(K, nc)
    F_ref = np.concatenate([f.ravel() for f in residual(prob, P, R, S, mu)])
    # size of the terms that cancel in F at a solution: the residual without
    # the slack terms, and rho s (about mu)
    terms = np.concatenate([f.ravel() for f in residual(prob, P, R, S * 0.0, 0.0)])
    scale = max(np.abs(terms).max(), np.abs(R * S).max())
    err = np.abs(F_gpu - F_ref).max() / scale
    print(f"  residual: |F| {nrm:.2e}, max |F_gpu - F_oracle| / max|terms| {err:.2e}", flush=True)
    assert err < 1e-12

    ke = kinetic_energy(prob, normalize_phi(prob, P), R)
    ds = dual_value(prob, normalize_phi(prob, P))
    e_ke = abs(cost - ke) / ke
    e_ds = abs(dual - ds) / abs(ds)
    gap = cost - dual
    expect = mu * K * prob.dt * 1.0
    print(f"  KE rel err {e_ke:.2e}, D* rel err {e_ds:.2e}, gap {gap:.10f} vs mu K dt |Omega| {expect:.10f}",
          flush=True)
    assert e_ke < 1e-12 and e_ds < 1e-10
    assert abs(gap - expect) < 1e-6 * expect

    m0 = float(prob.ops.ac @ ri)
    mass = R @ prob.ops.ac
    assert np.abs(mass - m0).max() < 1e-12 * m0
    assert R.min() > 0.0 and S.min() > 0.0
