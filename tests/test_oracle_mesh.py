"""Pins of the oracle's meshes (two-level FV meshes, Sec. 2.1).

Every check recomputes the geometry directly (polygon clipping, point
location) instead of re-reading the mesh builder's index logic.
"""

import numpy as np
import pytest

from oracle.mesh import structured_mesh, cartesian_mesh


def _coarse_tri_vertices(n):
    """Coarse triangles by direct geometry: square (A, B) of side H split
    SW-NE; t = 0 the part with x >= y (relative to the square)."""
    H = 2.0 / n
    out = {}
    for B in range(n // 2):
        for A in range(n // 2):
            x0, y0 = A * H, B * H
            j = 2 * (B * (n // 2) + A)
            out[j] = np.array([(x0, y0), (x0 + H, y0), (x0 + H, y0 + H)])
            out[j + 1] = np.array([(x0, y0), (x0 + H, y0 + H), (x0, y0 + H)])
    return out


def _clip(subject, clipper):
    """Sutherland-Hodgman clipping of a polygon by a convex CCW polygon."""
    out = list(subject)
    m = len(clipper)
    for i in range(m):
        a, b = clipper[i], clipper[(i + 1) % m]
        inp, out = out, []
        if not inp:
            break

        def inside(p):
            return (b[0] - a[0]) * (p[1] - a[1]) - (b[1] - a[1]) * (p[0] - a[0]) >= -1e-15

        def inter(p, q):
            d1 = (b[0] - a[0]) * (p[1] - a[1]) - (b[1] - a[1]) * (p[0] - a[0])
            d2 = (b[0] - a[0]) * (q[1] - a[1]) - (b[1] - a[1]) * (q[0] - a[0])
            t = d1 / (d1 - d2)
            return (p[0] + t * (q[0] - p[0]), p[1] + t * (q[1] - p[1]))

        for k in range(len(inp)):
            p, q = inp[k], inp[(k + 1) % len(inp)]
            if inside(q):
                if not inside(p):
                    out.append(inter(p, q))
                out.append(q)
            elif inside(p):
                out.append(inter(p, q))
    return out


def _area(poly):
    if len(poly) < 3:
        return 0.0
    x = np.array([p[0] for p in poly])
    y = np.array([p[1] for p in poly])
    return 0.5 * abs(np.dot(x, np.roll(y, -1)) - np.dot(y, np.roll(x, -1)))


def _locate(tris, p):
    for j, t in tris.items():
        a, b, c = t
        d = lambda u, v, w: (v[0] - u[0]) * (w[1] - u[1]) - (v[1] - u[1]) * (w[0] - u[0])
        if d(a, b, p) >= 0 and d(b, c, p) >= 0 and d(c, a, p) >= 0:
            return j
    raise AssertionError("point outside mesh")


@pytest.mark.parametrize("n", [2, 4, 8])
def test_counts_and_areas(n):
    m = structured_mesh(n)
    assert m.n_fine == n * n
    assert m.n_coarse == n * n // 2
    assert m.n_fedge == 2 * n * (n - 1)
    nc = n // 2
    assert m.n_cedge == nc * nc + 2 * nc * (nc - 1)
    assert np.isclose(m.fine_area.sum(), 1.0, rtol=0, atol=1e-14)
    assert np.isclose(m.coarse_area.sum(), 1.0, rtol=0, atol=1e-14)


@pytest.mark.parametrize("n", [2, 4, 6])
def test_overlaps_by_clipping(n):
    """Omega_ij = area(fine square i intersected with coarse triangle j)."""
    m = structured_mesh(n)
    tris = _coarse_tri_vertices(n)
    h = 1.0 / n
    dense = np.zeros((m.n_fine, m.n_coarse))
    dense[m.ov_fine, m.ov_coarse] = m.ov_area
    for b in range(n):
        for a in range(n):
            sq = [(a * h, b * h), ((a + 1) * h, b * h), ((a + 1) * h, (b + 1) * h), (a * h, (b + 1) * h)]
            for j, t in tris.items():
                ar = _area(_clip(sq, [tuple(v) for v in t]))
                assert abs(ar - dense[b * n + a, j]) < 1e-14, (a, b, j)
    # row sums = fine areas, column sums = coarse areas
    assert np.allclose(dense.sum(1), m.fine_area, atol=1e-15)
    assert np.allclose(dense.sum(0), m.coarse_area, atol=1e-15)


@pytest.mark.parametrize("n", [2, 4, 8])
def test_edge_geometry_and_density_sides(n):
    """K/L are the left/bottom and right/top squares; the density side of each
    is the coarse triangle containing the point just inside that square next
    to the edge midpoint, off the square's own diagonal."""
    m = structured_mesh(n)
    tris = _coarse_tri_vertices(n)
    h = 1.0 / n
    eps = 1e-3 * h
    for e in range(m.n_fedge):
        K, L = m.fe_K[e], m.fe_L[e]
        aK, bK = K % n, K // n
        aL, bL = L % n, L // n
        if bK == bL:      # vertical edge at x = (aK+1) h
            assert aL == aK + 1
            xm, ym = (aK + 1) * h, (bK + 0.5) * h
            pK, pL = (xm - eps, ym - 0.25 * h), (xm + eps, ym + 0.25 * h)
            # pK lies below the SW-NE diagonal of square K (the LR triangle
            # touching the edge); pL above that of square L.
        else:             # horizontal edge at y = (bK+1) h
            assert aL == aK and bL == bK + 1
            xm, ym = (aK + 0.5) * h, (bK + 1) * h
            pK, pL = (xm - 0.25 * h, ym - eps), (xm + 0.25 * h, ym + eps)
        assert _locate(tris, pK) == m.fe_rK[e]
        assert _locate(tris, pL) == m.fe_rL[e]
        assert m.fe_len[e] == pytest.approx(h) and m.fe_dist[e] == pytest.approx(h)
    assert np.all(m.fe_lam == 0.5)


@pytest.mark.parametrize("n", [4, 8])
def test_coarse_edges_share_a_side(n):
    m = structured_mesh(n)
    tris = _coarse_tri_vertices(n)
    H = 2.0 / n
    for e in range(m.n_cedge):
        ti, tj = tris[m.ce_i[e]], tris[m.ce_j[e]]
        common = [p for p in ti if any(np.allclose(p, q) for q in tj)]
        assert len(common) == 2
        length = np.linalg.norm(common[0] - common[1])
        assert m.ce_len[e] == pytest.approx(length)
        ci, cj = ti.mean(0), tj.mean(0)
        if np.isclose(length, H):
            # legs: circumcentre distance = distance of the hypotenuse midpoints
            cci = 0.5 * (ti[0] + ti[2]) if m.ce_i[e] % 2 == 0 else 0.5 * (ti[0] + ti[1])
            ccj = 0.5 * (tj[0] + tj[2]) if m.ce_j[e] % 2 == 0 else 0.5 * (tj[0] + tj[1])
            assert m.ce_dist[e] == pytest.approx(np.linalg.norm(cci - ccj))
        else:
            assert m.ce_dist[e] == pytest.approx(np.linalg.norm(ci - cj))
    # every interior coarse side appears exactly once
    nc = n // 2
    assert m.n_cedge == 3 * nc * nc - 2 * nc


def test_cartesian_is_single_grid():
    m = cartesian_mesh(4)
    assert m.n_fine == m.n_coarse == 16
    assert np.array_equal(m.fe_rK, m.fe_K) and np.array_equal(m.fe_rL, m.fe_L)
    assert np.allclose(m.ov_area, 1.0 / 16)
