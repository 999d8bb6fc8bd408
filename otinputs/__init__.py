"""Seeded synthetic inputs shared by the oracle side and the HIP side.

This module holds no arithmetic of the transport method: it only draws
Gaussian-mixture densities, averages them over the coarse cells of the
benchmark meshes by a fixed quadrature, floors and normalises them, and draws
mass-preserving perturbation directions.  Both the oracle and the GPU library
receive its arrays as plain inputs.

Workloads (all on the unit square, marginals on the coarse/density cells):
  * gaussian pair: isotropic N(c, sigma^2 I), sigma = 0.1, centres (0.3, 0.3)
    and (0.7, 0.7); seed-free (the paper's first test case, with the sigma of
    the benchmark configuration);
  * mixtures: k Gaussians with centres U[0.2, 0.8]^2, sigma U[0.05, 0.15],
    weights Dirichlet(1, ..., 1), optional uniform background;
  * translation: sigma = 0.05 Gaussian moved from (0.35, 0.5) to (0.65, 0.5);
  * three dimensions: Gaussians of variance 0.1 at (0.3, 0.3, 0.3) and
    (0.7, 0.7, 0.7) on the n^3 grid of cubes of [0,1]^3 (cube averages by the
    4^3 midpoint rule).
Cell averages: every coarse triangle is cut into 64 congruent sub-triangles
(8 per edge), density sampled at their centroids; Cartesian squares use the
8 x 8 midpoint rule.  Then floor at 1e-8 and scale to unit mass a'^T rho = 1.
Seeds: numpy default_rng(1000 * config + 2 * problem + {0: rho_in, 1: rho_f}).
"""

from __future__ import annotations

import numpy as np

FLOOR = 1e-8


# ---------------------------------------------------------------- geometry
def coarse_triangles(n: int) -> np.ndarray:
    """Vertices (n_coarse, 3, 2) of the density triangles of the n x n
    right-triangle grid: coarse square (A, B) of side 2/n split SW-NE,
    index 2 * (B * n/2 + A) + t with t = 0 below the diagonal, 1 above."""
    nc = n // 2
    H = 2.0 / n
    tris = np.empty((2 * nc * nc, 3, 2))
    for B in range(nc):
        for A in range(nc):
            x0, y0 = A * H, B * H
            j = 2 * (B * nc + A)
            tris[j] = [(x0, y0), (x0 + H, y0), (x0 + H, y0 + H)]
            tris[j + 1] = [(x0, y0), (x0 + H, y0 + H), (x0, y0 + H)]
    return tris


def triangle_areas(tris: np.ndarray) -> np.ndarray:
    p0, p1, p2 = tris[:, 0], tris[:, 1], tris[:, 2]
    return 0.5 * np.abs((p1[:, 0] - p0[:, 0]) * (p2[:, 1] - p0[:, 1])
                        - (p2[:, 0] - p0[:, 0]) * (p1[:, 1] - p0[:, 1]))


def _subtriangle_centroids(m: int = 8) -> np.ndarray:
    """Barycentric centroids of the m^2 congruent sub-triangles."""
    pts = []
    for i in range(m):
        for j in range(m - i):
            # upward triangle (i, j), (i+1, j), (i, j+1)
            pts.append(((3 * i + 1) / (3 * m), (3 * j + 1) / (3 * m)))
            if i + j < m - 1:
                # downward triangle (i+1, j), (i, j+1), (i+1, j+1)
                pts.append(((3 * i + 2) / (3 * m), (3 * j + 2) / (3 * m)))
    uv = np.array(pts)
    assert uv.shape[0] == m * m
    return uv


def triangle_averages(fn, tris: np.ndarray, m: int = 8) -> np.ndarray:
    uv = _subtriangle_centroids(m)
    p0, p1, p2 = tris[:, 0], tris[:, 1], tris[:, 2]
    x = p0[:, None, :] + uv[None, :, 0:1] * (p1 - p0)[:, None, :] \
        + uv[None, :, 1:2] * (p2 - p0)[:, None, :]
    return fn(x[..., 0], x[..., 1]).mean(axis=1)


def square_averages(fn, n: int, m: int = 8) -> np.ndarray:
    """Averages over the n x n squares, index b * n + a, midpoint rule."""
    h = 1.0 / n
    off = (np.arange(m) + 0.5) / m * h
    a = np.arange(n) * h
    xs = (a[:, None] + off[None, :]).ravel()
    X, Y = np.meshgrid(xs, xs)                       # Y row = y, X col = x
    vals = fn(X, Y).reshape(n, m, n, m)              # (b, sy, a, sx)
    return vals.mean(axis=(1, 3)).ravel()


# ---------------------------------------------------------------- densities
def gaussian(cx, cy, sigma):
    def f(x, y):
        r2 = (x - cx) ** 2 + (y - cy) ** 2
        return np.exp(-r2 / (2 * sigma * sigma)) / (2 * np.pi * sigma * sigma)
    return f


def mixture(centres, sigmas, weights, background=0.0):
    comps = [gaussian(c[0], c[1], s) for c, s in zip(centres, sigmas)]

    def f(x, y):
        out = np.full(np.broadcast(x, y).shape, float(background))
        for w, g in zip(weights, comps):
            out = out + w * g(x, y)
        return out
    return f


def random_mixture(rng, k, background=0.0):
    centres = rng.uniform(0.2, 0.8, size=(k, 2))
    sigmas = rng.uniform(0.05, 0.15, size=k)
    weights = rng.dirichlet(np.ones(k))
    return mixture(centres, sigmas, weights, background)


def cube_averages(fn, n: int, m: int = 4) -> np.ndarray:
    """Averages of fn(x, y, z) over the n^3 cubes of [0,1]^3 (cell
    (c n + b) n + a), m^3-point midpoint rule per cube."""
    h = 1.0 / n
    t = (np.arange(m) + 0.5) / m
    centres = (np.arange(n) * h)[:, None] + h * t[None, :]          # (n, m)
    xs = centres.ravel()
    X = xs[None, None, :]
    Y = xs[None, :, None]
    Z = xs[:, None, None]
    vals = fn(X, Y, Z)                                                # [z, y, x] samples
    vals = vals.reshape(n, m, n, m, n, m).mean(axis=(1, 3, 5))
    return vals.ravel()


def floor_normalize(vals, areas, floor=FLOOR):
    v = np.maximum(vals, floor)
    return v / float(areas @ v)


def structured_marginal(fn, n):
    tris = coarse_triangles(n)
    return floor_normalize(triangle_averages(fn, tris), triangle_areas(tris))


def cartesian_marginal(fn, n):
    return floor_normalize(square_averages(fn, n), np.full(n * n, 1.0 / (n * n)))


# ---------------------------------------------------------------- workloads
def gaussian_pair(n, mesh="structured", sigma=0.1):
    """The seed-free Gaussian pair: (0.3, 0.3) -> (0.7, 0.7)."""
    mk = structured_marginal if mesh == "structured" else cartesian_marginal
    return (mk(gaussian(0.3, 0.3, sigma), n), mk(gaussian(0.7, 0.7, sigma), n))


def translation_pair(n, mesh="structured", sigma=0.05, shift=0.3):
    mk = structured_marginal if mesh == "structured" else cartesian_marginal
    x0 = 0.5 - shift / 2
    return (mk(gaussian(x0, 0.5, sigma), n), mk(gaussian(x0 + shift, 0.5, sigma), n))


def gaussian3d(cx, cy, cz, sigma):
    c = 1.0 / ((2.0 * np.pi) ** 1.5 * sigma ** 3)

    def f(x, y, z):
        return c * np.exp(-((x - cx) ** 2 + (y - cy) ** 2 + (z - cz) ** 2) / (2.0 * sigma * sigma))
    return f


def gaussian3d_pair(n, sigma=np.sqrt(0.1), centres=((0.3, 0.3, 0.3), (0.7, 0.7, 0.7))):
    """The three-dimensional workload on the n^3 cube grid: isotropic
    Gaussians of variance 0.1 at (0.3, 0.3, 0.3) and (0.7, 0.7, 0.7) (the
    paper's fourth test case; no benchmark configuration overrides the
    variance here), cube averages by the 4^3 midpoint rule, floored and
    normalised to unit mass; seed-free."""
    vol = np.full(n ** 3, 1.0 / n ** 3)
    return tuple(floor_normalize(cube_averages(gaussian3d(*c, sigma), n), vol) for c in centres)


def mixture_pair(n, k, config, problem=0, background=0.0, mesh="structured"):
    mk = structured_marginal if mesh == "structured" else cartesian_marginal
    out = []
    for side in (0, 1):
        rng = np.random.default_rng(1000 * config + 2 * problem + side)
        out.append(mk(random_mixture(rng, k, background), n))
    return tuple(out)


def config_marginals(cfg: int, problem: int = 0):
    """(n, K, rho_in, rho_f) of the benchmark configurations 1..5."""
    if cfg == 1:
        return (16, 8) + gaussian_pair(16)
    if cfg == 2:
        return (64, 32) + mixture_pair(64, 3, 2, problem)
    if cfg == 3:
        return (256, 64) + mixture_pair(256, 5, 3, problem, background=1e-3)
    if cfg == 4:
        n, K, k = batch_spec(problem)
        return (n, K) + mixture_pair(n, k, 4, problem)
    if cfg == 5:
        return (128, 32) + mixture_pair(128, 3, 5, problem)
    raise ValueError(cfg)


def batch_spec(problem: int):
    """(n, K, components) of member `problem` of the 32-problem batch."""
    rng = np.random.default_rng(1000 * 4 + 2 * problem + 100000)
    n = int(rng.choice([32, 48, 64, 96, 128]))
    K = int(rng.choice([8, 16, 32]))
    k = int(rng.integers(1, 5))
    return n, K, k


def mass_preserving_directions(rho, areas, count, seed):
    """Unit directions delta = rho*xi - rho (a'^T(rho*xi)) / (a'^T rho),
    xi ~ N(0, I): a'^T delta = 0, and rho +- eps delta stays positive."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        xi = rng.standard_normal(rho.size)
        d = rho * xi - rho * float(areas @ (rho * xi)) / float(areas @ rho)
        out.append(d / np.linalg.norm(d))
    return np.array(out)


def random_mesh_arrays(nf, nc, seed):
    """A random, valid generic two-level mesh description (graph-based, not
    geometric) for exercising the generic mesh interface: positive areas,
    overlaps summing to both cell areas, a connected fine edge graph with
    random lengths, distances and lambdas, density sides taken among the
    parents of each edge cell, and coarse edges between parents of
    neighbouring fine cells."""
    rng = np.random.default_rng(seed)
    assert nf >= nc >= 2
    parent = np.concatenate([np.arange(nc), rng.integers(0, nc, nf - nc)])
    rng.shuffle(parent)
    ov = {}
    for i in range(nf):
        ov[(i, int(parent[i]))] = rng.uniform(0.5, 1.5)
        if rng.random() < 0.3:
            j2 = int(rng.integers(0, nc))
            if j2 != parent[i]:
                ov[(i, j2)] = rng.uniform(0.2, 0.8)
    keys = sorted(ov)
    ov_f = np.array([k[0] for k in keys], dtype=np.int32)
    ov_c = np.array([k[1] for k in keys], dtype=np.int32)
    ov_a = np.array([ov[k] for k in keys])
    ov_a /= ov_a.sum()
    fine_area = np.bincount(ov_f, weights=ov_a, minlength=nf)
    coarse_area = np.bincount(ov_c, weights=ov_a, minlength=nc)
    parents = [[] for _ in range(nf)]
    for f, c in zip(ov_f, ov_c):
        parents[f].append(int(c))
    perm = rng.permutation(nf)
    edges = set()
    for t in range(1, nf):
        a, b = int(perm[t]), int(perm[rng.integers(0, t)])
        edges.add((min(a, b), max(a, b)))
    while len(edges) < 2 * nf:
        a, b = rng.integers(0, nf, 2)
        if a != b:
            edges.add((int(min(a, b)), int(max(a, b))))
    edges = sorted(edges)
    ne = len(edges)
    fe_cell = np.array(edges, dtype=np.int32).ravel()
    fe_rho = np.array([[parents[a][rng.integers(len(parents[a]))], parents[b][rng.integers(len(parents[b]))]]
                       for a, b in edges], dtype=np.int32).ravel()
    scale = 1.0 / np.sqrt(nf)
    fe_len = rng.uniform(0.5, 1.5, ne) * scale
    fe_dist = rng.uniform(0.5, 1.5, ne) * scale
    fe_lambda = rng.uniform(0.0, 1.0, ne)
    cset = set()
    for a, b in edges:
        for ca in parents[a]:
            for cb in parents[b]:
                if ca != cb:
                    cset.add((min(ca, cb), max(ca, cb)))
    cperm = rng.permutation(nc)
    for t in range(1, nc):
        a, b = int(cperm[t]), int(cperm[rng.integers(0, t)])
        cset.add((min(a, b), max(a, b)))
    cedges = sorted(cset)
    nce = len(cedges)
    return dict(
        fine_area=fine_area, coarse_area=coarse_area, ov_fine=ov_f, ov_coarse=ov_c, ov_area=ov_a,
        fe_cell=fe_cell, fe_rho=fe_rho, fe_len=fe_len, fe_dist=fe_dist, fe_lambda=fe_lambda,
        ce_cell=np.array(cedges, dtype=np.int32).ravel(),
        ce_len=rng.uniform(0.5, 1.5, nce) * np.sqrt(2.0 / nc),
        ce_dist=rng.uniform(0.5, 1.5, nce) * np.sqrt(2.0 / nc),
        ce_lambda=rng.uniform(0.0, 1.0, nce))
