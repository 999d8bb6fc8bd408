"""Pins of the oracle's discrete operators (Sec. 2.1, Sec. 4.4.3)."""

import numpy as np
import pytest
import scipy.sparse as sp

from oracle.mesh import structured_mesh, cartesian_mesh
from oracle.operators import Operators


def _path_laplacian(n):
    main = np.full(n, 2.0)
    main[0] = main[-1] = 1.0
    return sp.diags([main, -np.ones(n - 1), -np.ones(n - 1)], [0, 1, -1])


def _cell_centres(n):
    h = 1.0 / n
    b, a = np.divmod(np.arange(n * n), n)
    return (a + 0.5) * h, (b + 0.5) * h


@pytest.mark.parametrize("mk", [structured_mesh, cartesian_mesh])
@pytest.mark.parametrize("n", [4, 8])
def test_no_flux_and_consistency(mk, n):
    o = Operators(mk(n))
    assert np.abs(o.grad @ np.ones(o.mesh.n_fine)).max() == 0.0          # grad 1 = 0
    assert np.abs(np.ones(o.mesh.n_fine) @ o.div).max() < 1e-16           # 1^T div = 0
    assert np.allclose(o.RE @ np.ones(o.mesh.n_coarse), 1.0)               # R_E 1 = 1
    assert np.allclose(o.REf @ np.ones(o.mesh.n_fine), 1.0)
    assert np.allclose(np.asarray(o.Om.sum(1)).ravel(), o.a)              # Omega 1 = a
    assert np.allclose(np.asarray(o.Om.sum(0)).ravel(), o.ac)             # 1^T Omega = a'


@pytest.mark.parametrize("mk", [structured_mesh, cartesian_mesh])
def test_unit_weight_laplacian_is_5_point(mk):
    n = 8
    o = Operators(mk(n))
    L = o.laplacian(np.ones(o.mesh.n_fedge))
    I = sp.identity(n)
    T = _path_laplacian(n)
    ref = sp.kron(I, T) + sp.kron(T, I)       # index b*n + a: kron(I_b, T_a) + kron(T_b, I_a)
    assert abs(L - ref).max() < 1e-12


@pytest.mark.parametrize("mk", [structured_mesh, cartesian_mesh])
def test_linear_potential(mk):
    """phi = d . x: (grad phi)_e = d . n_e with n_e from L to K, and
    R_T((grad phi)^2) = a' |d|^2 on interior coarse cells (4 horizontal and
    4 vertical edge-sides of weight h^2/2 each on the triangle grid)."""
    n = 16
    o = Operators(mk(n))
    x, y = _cell_centres(n)
    d = np.array([0.3, -0.7])
    phi = d[0] * x + d[1] * y
    g = o.grad @ phi
    m = o.mesh
    vertical = (m.fe_L - m.fe_K) == 1
    assert np.allclose(g[vertical], -d[0]) and np.allclose(g[~vertical], -d[1])
    rt = o.RT @ (g * g)
    # interior coarse cells: every neighbouring fine square exists
    wsum = o.RT @ np.ones(m.n_fedge)
    interior = np.isclose(wsum, 2.0 * o.ac)   # all edge-sides present
    assert interior.sum() > 0
    assert np.allclose(rt[interior], o.ac[interior] * (d @ d))


def test_coarse_laplacian_unit_density():
    o = Operators(structured_mesh(8))
    At = o.coarse_laplacian(np.ones(o.mesh.n_coarse))
    assert abs(At - At.T).max() < 1e-14
    assert np.abs(At @ np.ones(o.mesh.n_coarse)).max() < 1e-13
    w = np.linalg.eigvalsh(At.toarray())
    assert w.min() > -1e-12 and np.sum(w < 1e-10) == 1      # connected, PSD
    # leg weight length/dist = 1, diagonal weight sqrt(2)H / (sqrt(2)H/3) = 3
    diag_pairs = np.abs(At[0, 1])
    assert diag_pairs == pytest.approx(3.0)
