"""Parity of the BB preconditioner's components on the GPU against the
oracle's sparse matrices: pseudo-Schur operator, its probed time diagonals,
the pseudo-Schur GMRES solve, the multigrid-preconditioned Laplacian solves."""

import ctypes as C

import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from oracle.mesh import structured_mesh
from oracle.ipm import Problem, edge_density
from oracle.bb import pseudo_schur

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
ot = pytest.importorskip("paper_2209_00315_amd")


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


@pytest.fixture(params=[("fp64", 1e-12), ("mixed", 1e-5)], ids=["fp64", "mixed"])
def setup(request):
    precision, tol = request.param
    n, K = 8, 4
    rng = np.random.default_rng(3)
    m = structured_mesh(n)
    ri = rng.uniform(0.2, 2.0, m.n_coarse)
    rf = rng.uniform(0.2, 2.0, m.n_coarse)
    ri /= m.coarse_area @ ri
    rf /= m.coarse_area @ rf
    prob = Problem(m, K, ri, rf)
    phi = rng.standard_normal((K + 1, prob.nf)) * 0.2
    rho = rng.uniform(0.5, 2.0, (K, prob.nc))
    s = rng.uniform(0.1, 1.0, (K, prob.nc))
    st = ot.State(ot.Mesh.structured(n), ri, rf, K, precision=precision)
    st.import_(phi.ravel(), rho.ravel(), s.ravel(), 0.3)
    print(f"[components {precision}] n={n} K={K}", flush=True)
    return prob, phi, rho, s, st, tol


def test_schur_operator(setup):
    prob, phi, rho, s, st, tol = setup
    S = pseudo_schur(prob, phi, rho, s)
    z = np.random.default_rng(4).standard_normal(st.m_rho)
    out = np.zeros(st.m_rho)
    ot.check(ot.lib().otbb_debug_schur_apply(st._h, _dp(z), _dp(out)))
    ref = S @ z
    err = np.abs(out - ref).max() / np.abs(ref).max()
    print(f"  schur apply rel err {err:.2e}", flush=True)
    assert err < tol


def test_probed_diagonals(setup):
    prob, phi, rho, s, st, tol = setup
    S = pseudo_schur(prob, phi, rho, s)
    nc = prob.nc
    d0, dl, du = np.zeros(st.m_rho), np.zeros(st.m_rho), np.zeros(st.m_rho)
    ot.check(ot.lib().otbb_debug_tri_diagonals(st._h, _dp(d0), _dp(dl), _dp(du)))
    e0 = np.abs(d0 - S.diagonal(0)).max() / np.abs(S.diagonal(0)).max()
    el = np.abs(dl[nc:] - S.diagonal(-nc)).max() / np.abs(S.diagonal(-nc)).max()
    eu = np.abs(du[:-nc] - S.diagonal(nc)).max() / np.abs(S.diagonal(nc)).max()
    print(f"  diagonals rel err {e0:.2e} {el:.2e} {eu:.2e}", flush=True)
    assert max(e0, el, eu) < tol


def test_schur_solve(setup):
    """GMRES on the pseudo-Schur system at an interior-point iterate."""
    prob, phi, rho, s, st, tol = setup
    from oracle.ipm import solve_ipm
    r = solve_ipm(prob, tol=1e-6, mu_target=0.04)
    phi, rho, s = r.phi, r.rho, r.s
    st.import_(phi.ravel(), rho.ravel(), s.ravel(), r.mu)
    S = pseudo_schur(prob, phi, rho, s)
    b = np.random.default_rng(5).standard_normal(st.m_rho)
    z = np.zeros(st.m_rho)
    its = C.c_int32()
    itol = 1e-12 if tol < 1e-8 else 1e-5
    ot.check(ot.lib().otbb_debug_schur_solve(st._h, _dp(b), _dp(z), itol, 1000, C.byref(its)))
    res = np.linalg.norm(S @ z - b) / np.linalg.norm(b)
    print(f"  schur solve its {its.value} rel res {res:.2e}", flush=True)
    assert res < 10 * itol


def test_laplace_solve(setup):
    prob, phi, rho, s, st, tol = setup
    K, nf = prob.K, prob.nf
    rt = edge_density(prob, rho)
    rng = np.random.default_rng(6)
    b = rng.standard_normal((K + 1, nf))
    b -= b.mean(axis=1, keepdims=True)
    x = np.zeros(b.size)
    its = C.c_int32()
    itol = 1e-12 if tol < 1e-8 else 1e-5
    ot.check(ot.lib().otbb_debug_laplace_solve(st._h, _dp(b.ravel().copy()), _dp(x), itol, 500, C.byref(its)))
    x = x.reshape(K + 1, nf)
    worst = 0.0
    for k in range(K + 1):
        A = prob.ops.laplacian(rt[k])
        worst = max(worst, np.linalg.norm(A @ x[k] - b[k]) / np.linalg.norm(b[k]))
    print(f"  laplace solve its {its.value} worst rel res {worst:.2e}", flush=True)
    assert worst < 10 * itol


def _thomas_reference(d0, dl, du, r, K, nc):
    """Host Thomas solve of the time-line tridiagonals with the library's
    factorisation rule (a pivot that loses three digits to elimination is
    replaced by the plain diagonal)."""
    d0, dl, du, r = (a.reshape(K, nc) for a in (d0, dl, du, r))
    inv, L, U = np.zeros((K, nc)), np.zeros((K, nc)), np.zeros((K, nc))
    prev, prev_up = np.zeros(nc), np.zeros(nc)
    for k in range(K):
        d, l = d0[k].copy(), np.zeros(nc)
        if k > 0:
            ok = prev != 0.0
            l = np.where(ok, dl[k] / np.where(ok, prev, 1.0), 0.0)
            dd = d - l * prev_up
            weak = ~(np.abs(dd) > 1e-3 * np.abs(d)) | ~np.isfinite(dd)
            l = np.where(weak, 0.0, l)
            d = np.where(weak, d, dd)
        d = np.where(~(np.abs(d) > 0.0) | ~np.isfinite(d), 1.0, d)
        u = du[k] if k + 1 < K else np.zeros(nc)
        inv[k], L[k], U[k] = 1.0 / d, l, u
        prev, prev_up = d, u
    y, acc = np.zeros((K, nc)), np.zeros(nc)
    for k in range(K):
        acc = r[k] - L[k] * acc
        y[k] = acc
    x, xn = np.zeros((K, nc)), np.zeros(nc)
    for k in reversed(range(K)):
        xn = (y[k] - U[k] * xn) * inv[k]
        x[k] = xn
    return x.ravel()


@pytest.mark.parametrize("K", [4, 64, 70, 130, 300])
@pytest.mark.parametrize("precision,tol", [("fp64", 1e-9), ("mixed", 2e-4)])
def test_time_line_solve(K, precision, tol):
    """Time-line tridiagonal solve on the density cells: one wavefront per
    cell with a scan over time (K <= 256: one full chunk, a ragged chunk,
    several chunks) and the one-thread-per-cell recurrence (K = 300), both
    against the host Thomas solve of the probed diagonals."""
    n = 8
    rng = np.random.default_rng(21 + K)
    m = structured_mesh(n)
    ri = rng.uniform(0.2, 2.0, m.n_coarse)
    rf = rng.uniform(0.2, 2.0, m.n_coarse)
    ri /= m.coarse_area @ ri
    rf /= m.coarse_area @ rf
    nf, nc = m.n_fine, m.n_coarse
    print(f"[time-line solve {precision}] n={n} K={K}", flush=True)
    st = ot.State(ot.Mesh.structured(n), ri, rf, K, precision=precision)
    st.import_(rng.standard_normal((K + 1) * nf) * 0.2, rng.uniform(0.5, 2.0, K * nc),
               rng.uniform(0.1, 1.0, K * nc), 0.3)
    d0, dl, du = np.zeros(st.m_rho), np.zeros(st.m_rho), np.zeros(st.m_rho)
    ot.check(ot.lib().otbb_debug_tri_diagonals(st._h, _dp(d0), _dp(dl), _dp(du)))
    r = rng.standard_normal(st.m_rho)
    x = np.zeros(st.m_rho)
    ot.check(ot.lib().otbb_debug_tri_solve(st._h, _dp(r), _dp(x)))
    ref = _thomas_reference(d0, dl, du, r, K, nc)
    err = np.abs(x - ref).max() / np.abs(ref).max()
    print(f"  time-line solve rel err {err:.2e}", flush=True)
    assert err < tol


@pytest.mark.parametrize("levels", [0, 1, 8, 16])
@pytest.mark.parametrize("K", [4, 8, 12, 17])
@pytest.mark.parametrize("precision,tol", [("fp64", 1e-12), ("mixed", 1e-5)])
def test_schur_operator_time_blocks(K, precision, tol, levels):
    """Pseudo-Schur operator through the time-blocked passes (levels per
    thread; 0 = per-level kernels): K below, at, and past one block, with a
    ragged last block."""
    w = 4 if precision == "mixed" else 8
    ot.check(ot.lib().otbb_debug_set_schur_blocking(w, levels, levels))
    try:
        _schur_blocks_case(K, precision, tol, levels)
    finally:
        ot.check(ot.lib().otbb_debug_set_schur_blocking(w, -1, -1))          # back to the autotuner


def _schur_blocks_case(K, precision, tol, levels):
    n = 8
    rng = np.random.default_rng(40 + K)
    m = structured_mesh(n)
    ri = rng.uniform(0.2, 2.0, m.n_coarse)
    rf = rng.uniform(0.2, 2.0, m.n_coarse)
    ri /= m.coarse_area @ ri
    rf /= m.coarse_area @ rf
    prob = Problem(m, K, ri, rf)
    phi = rng.standard_normal((K + 1, prob.nf)) * 0.2
    rho = rng.uniform(0.5, 2.0, (K, prob.nc))
    s = rng.uniform(0.1, 1.0, (K, prob.nc))
    print(f"[schur blocks {precision}] n={n} K={K} levels={levels}", flush=True)
    st = ot.State(ot.Mesh.structured(n), ri, rf, K, precision=precision)
    st.import_(phi.ravel(), rho.ravel(), s.ravel(), 0.3)
    S = pseudo_schur(prob, phi, rho, s)
    z = rng.standard_normal(st.m_rho)
    out = np.zeros(st.m_rho)
    ot.check(ot.lib().otbb_debug_schur_apply(st._h, _dp(z), _dp(out)))
    ref = S @ z
    err = np.abs(out - ref).max() / np.abs(ref).max()
    print(f"  schur apply rel err {err:.2e}", flush=True)
    assert err < tol
