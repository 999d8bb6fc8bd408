"""Value pins of the oracle's BB preconditioner pieces (Sec. 4.4.2-4.4.3).

The reference here is a dense assembly of every operator written entry by
entry from the definitions, straight from the raw mesh arrays (edge cells,
density sides, lengths, distances, lambdas, overlaps, coarse edges).  It does
not use oracle/operators.py or the sparse blocks of oracle/ipm.py, so a slip
in either shows up as a mismatch:

  A^p     = grad^T W Diag(rho~^p) grad        rho~^p = R_E (rho^p + rho^{p+1})/2
  B  rows q, cols p = q, q+1: -+ Omega^T/dt + 1/2 R_T Diag(grad phi^p) grad
  C       = Diag(a' s / rho)
  A~^q    = E' Diag(len'/dist' R'_E rho^q) E'^T
  B~ rows p, cols q = p, p-1: +- Omega/dt + 1/2 R_Tf Diag(grad phi^p) grad J
  S_BB    = Diag(s) A~ - Diag(rho) B M^-1 B~
  (P v)^q = v^q - a' (1^T v^q)/|Omega|,  P^T its transpose.

(p: potential level 0..K, q: density level 0..K-1; the density indices
0..K+1 of rho~ address rho_in, rho^1..rho^K, rho_f.)

The random generic mesh has unequal coarse areas, so P is not symmetric and
dropping P^T changes the result; on the structured grids it would not.
"""

import numpy as np
import pytest

import otinputs
import oracle.bb as bb
from oracle.ipm import Problem, kkt_blocks
from oracle.mesh import mesh_from_arrays, structured_mesh


# ---------------------------------------------------------------- dense reference
class Dense:
    def __init__(self, mesh, K, rho_in, rho_f, phi, rho, s):
        self.K, self.nf, self.nc = K, mesh.n_fine, mesh.n_coarse
        nf, nc = self.nf, self.nc
        self.dt = dt = 1.0 / (K + 1)
        a, ac = mesh.fine_area, mesh.coarse_area
        self.a, self.ac, self.area = a, ac, float(ac.sum())
        Om = np.zeros((nf, nc))
        for i, j, w in zip(mesh.ov_fine, mesh.ov_coarse, mesh.ov_area):
            Om[i, j] += w
        edges = list(zip(mesh.fe_K, mesh.fe_L, mesh.fe_rK, mesh.fe_rL, mesh.fe_len, mesh.fe_dist, mesh.fe_lam))

        def grad_rows():          # grad as a dense (ne x nf) matrix
            G = np.zeros((len(edges), nf))
            for e, (k, l, _, _, _, d, _) in enumerate(edges):
                G[e, k] += 1.0 / d
                G[e, l] -= 1.0 / d
            return G

        grad = grad_rows()
        rfull = np.vstack([rho_in, rho, rho_f])
        # A^p
        self.A = []
        for p in range(K + 1):
            Ap = np.zeros((nf, nf))
            for k, l, rk, rl, ln, d, lam in edges:
                mk = 0.5 * (rfull[p][rk] + rfull[p + 1][rk])
                ml = 0.5 * (rfull[p][rl] + rfull[p + 1][rl])
                w = ln / d * (lam * mk + (1.0 - lam) * ml)
                Ap[k, k] += w
                Ap[l, l] += w
                Ap[k, l] -= w
                Ap[l, k] -= w
            self.A.append(Ap)

        def rt_g_grad(g, fine_side):
            """R_T Diag(g) grad (nc x nf), or R_Tf Diag(g) grad (nf x nf)."""
            out = np.zeros((nf if fine_side else nc, nf))
            for e, (k, l, rk, rl, ln, d, lam) in enumerate(edges):
                c = ln * d * g[e] / d          # W_e g_e times the 1/d_e of grad
                sk, sl = (k, l) if fine_side else (rk, rl)
                for row, wt in ((sk, lam), (sl, 1.0 - lam)):
                    out[row, k] += wt * c
                    out[row, l] -= wt * c
            return out

        gphi = [grad @ phi[p] for p in range(K + 1)]
        n_phi, m_rho = (K + 1) * nf, K * nc
        self.n_phi, self.m_rho = n_phi, m_rho
        B = np.zeros((m_rho, n_phi))
        for q in range(K):
            B[q * nc:(q + 1) * nc, q * nf:(q + 1) * nf] = -Om.T / dt + 0.5 * rt_g_grad(gphi[q], False)
            B[q * nc:(q + 1) * nc, (q + 1) * nf:(q + 2) * nf] = Om.T / dt + 0.5 * rt_g_grad(gphi[q + 1], False)
        self.B = B
        self.C = np.diag((ac[None, :] * s / rho).ravel())
        At = np.zeros((m_rho, m_rho))
        for q in range(K):
            for i, j, ln, d, lam in zip(mesh.ce_i, mesh.ce_j, mesh.ce_len, mesh.ce_dist, mesh.ce_lam):
                w = ln / d * (lam * rho[q][i] + (1.0 - lam) * rho[q][j])
                o = q * nc
                At[o + i, o + i] += w
                At[o + j, o + j] += w
                At[o + i, o + j] -= w
                At[o + j, o + i] -= w
        self.At = At
        Jl = Om / a[:, None]
        Bt = np.zeros((n_phi, m_rho))
        for p in range(K + 1):
            G = 0.5 * rt_g_grad(gphi[p], True) @ Jl
            rows = slice(p * nf, (p + 1) * nf)
            if p < K:
                Bt[rows, p * nc:(p + 1) * nc] += Om / dt + G
            if p >= 1:
                Bt[rows, (p - 1) * nc:p * nc] += -Om / dt + G
        self.Bt = Bt
        Minv = np.diag(1.0 / np.tile(a, K + 1))
        self.S = np.diag(s.ravel()) @ At - np.diag(rho.ravel()) @ B @ Minv @ Bt
        Pk = np.eye(nc) - np.outer(ac, np.ones(nc)) / self.area
        self.P = np.kron(np.eye(K), Pk)
        Ablk = np.zeros((n_phi, n_phi))
        for p in range(K + 1):
            Ablk[p * nf:(p + 1) * nf, p * nf:(p + 1) * nf] = self.A[p]
        self.Ablk = Ablk
        self.JP = np.block([[Ablk, B.T @ self.P.T], [self.P @ B, -self.P @ self.C @ self.P.T]])


def _generic(seed=5, nf=40, nc=12, K=2):
    d = otinputs.random_mesh_arrays(nf, nc, seed)
    return mesh_from_arrays(d), K


def _state(mesh, K, seed):
    rng = np.random.default_rng(seed)
    nf, nc = mesh.n_fine, mesh.n_coarse
    ri = rng.uniform(0.3, 2.0, nc)
    rf = rng.uniform(0.3, 2.0, nc)
    ri /= mesh.coarse_area @ ri
    rf /= mesh.coarse_area @ rf
    phi = 0.3 * rng.standard_normal((K + 1, nf))
    rho = rng.uniform(0.5, 2.0, (K, nc))
    s = rng.uniform(0.1, 1.0, (K, nc))
    prob = Problem(mesh, K, ri, rf)
    return prob, phi, rho, s, Dense(mesh, K, ri, rf, phi, rho, s)


def _rel(a, b):
    return float(np.abs(np.asarray(a) - np.asarray(b)).max() / max(np.abs(b).max(), 1e-300))


MESHES = {"generic40": lambda: _generic(), "tri4K3": lambda: (structured_mesh(4), 3)}


# ---------------------------------------------------------------- pin metrics
def pseudo_schur_err(prob, phi, rho, s, D):
    return _rel(bb.pseudo_schur(prob, phi, rho, s).toarray(), D.S)


def bb_equation_errs(prob, phi, rho, s, D, seed=0):
    """apply_bb_exact's outputs checked against the dense equations:
    S_BB z = -Diag(rho) P d, y = P^T M'^-1 A~ z, A^p x^p = (c - B^T y)^p - mean,
    sum x^p = 0."""
    rng = np.random.default_rng(seed)
    K, nf, nc = prob.K, prob.nf, prob.nc
    c = rng.standard_normal((K + 1, nf))
    d = rng.standard_normal((K, nc))
    x, y, z = bb.apply_bb_exact(prob, phi, rho, s, c, d, return_zeta=True)
    rhs = -(rho.ravel() * (D.P @ d.ravel()))
    e_z = np.linalg.norm(D.S @ z.ravel() - rhs) / np.linalg.norm(rhs)
    w = (D.At @ z.ravel()) / np.tile(D.ac, K)
    e_y = _rel(y.ravel(), D.P.T @ w)
    b = (c.ravel() - D.B.T @ y.ravel()).reshape(K + 1, nf)
    e_x = 0.0
    for p in range(K + 1):
        bp = b[p] - b[p].mean()
        e_x = max(e_x, np.linalg.norm(D.A[p] @ x[p] - bp) / np.linalg.norm(bp), abs(x[p].sum()) / np.abs(x[p]).max())
    return e_z, e_y, e_x


def exact_mode_errs(prob, phi, rho, s, D, seed=1):
    """With the exact Schur complement routed through apply_bb_exact: GMRES
    on T = J_P P^-1 after two steps, and |(T - I)^2| on the range of J_P."""
    K, nf, nc = prob.K, prob.nf, prob.nc
    n_phi, N = D.n_phi, D.n_phi + D.m_rho

    def prec(v):
        x, y = bb.apply_bb_exact(prob, phi, rho, s, v[:n_phi].reshape(K + 1, nf), v[n_phi:].reshape(K, nc),
                                 schur="exact")
        return np.concatenate([x.ravel(), y.ravel()])

    Pinv = np.column_stack([prec(e) for e in np.eye(N)])
    T = D.JP @ Pinv
    b = D.JP @ np.random.default_rng(seed).standard_normal(N)
    V = [b / np.linalg.norm(b)]
    H = np.zeros((3, 2))
    for j in range(2):
        w = T @ V[j]
        for i in range(j + 1):
            H[i, j] = V[i] @ w
            w = w - H[i, j] * V[i]
        H[j + 1, j] = np.linalg.norm(w)
        V.append(w / H[j + 1, j] if H[j + 1, j] > 0 else w)
    e1 = np.zeros(3)
    e1[0] = np.linalg.norm(b)
    yls = np.linalg.lstsq(H, e1, rcond=None)[0]
    gm = np.linalg.norm(e1 - H @ yls) / np.linalg.norm(b)
    U, sv, _ = np.linalg.svd(D.JP)
    Q = U[:, sv > 1e-10 * sv[0]]
    R = T - np.eye(N)
    nil = np.abs((R @ R) @ Q).max() / np.abs(T).max()
    return gm, nil


# ---------------------------------------------------------------- tests
@pytest.mark.parametrize("name", list(MESHES))
def test_kkt_blocks_match_dense_definitions(name):
    mesh, K = MESHES[name]()
    prob, phi, rho, s, D = _state(mesh, K, 3)
    A, B, C = kkt_blocks(prob, phi, rho, s)
    assert _rel(A.toarray(), D.Ablk) < 1e-12
    assert _rel(B.toarray(), D.B) < 1e-12
    assert _rel(C.toarray(), D.C) < 1e-12
    assert _rel(bb.coarse_laplacian_blocks(prob, rho).toarray(), D.At) < 1e-12
    assert _rel(bb.btilde(prob, phi).toarray(), D.Bt) < 1e-12
    assert _rel(bb.projected_matrix(prob, phi, rho, s).toarray(), D.JP) < 1e-12


@pytest.mark.parametrize("name", list(MESHES))
def test_pseudo_schur_matches_dense_definition(name):
    mesh, K = MESHES[name]()
    prob, phi, rho, s, D = _state(mesh, K, 4)
    assert pseudo_schur_err(prob, phi, rho, s, D) < 1e-12


@pytest.mark.parametrize("name", list(MESHES))
def test_apply_bb_satisfies_its_equations(name):
    mesh, K = MESHES[name]()
    prob, phi, rho, s, D = _state(mesh, K, 5)
    e_z, e_y, e_x = bb_equation_errs(prob, phi, rho, s, D)
    assert e_z < 1e-10 and e_y < 1e-10 and e_x < 1e-9, (e_z, e_y, e_x)


@pytest.mark.parametrize("name", list(MESHES))
def test_exact_schur_through_apply_bb_two_steps(name):
    mesh, K = MESHES[name]()
    prob, phi, rho, s, D = _state(mesh, K, 6)
    gm, nil = exact_mode_errs(prob, phi, rho, s, D)
    assert gm < 1e-8 and nil < 1e-8, (gm, nil)


def test_pins_detect_planted_mistakes(monkeypatch):
    """Each plausible slip, planted in the oracle on the CPU, fails a pin."""
    mesh, K = _generic()
    prob, phi, rho, s, D = _state(mesh, K, 7)
    orig_proj_t, orig_ps = bb.proj_t, bb.pseudo_schur

    def failing():
        e_z, e_y, e_x = bb_equation_errs(prob, phi, rho, s, D)
        gm, nil = exact_mode_errs(prob, phi, rho, s, D)
        return {"ps": pseudo_schur_err(prob, phi, rho, s, D) > 1e-6, "z": e_z > 1e-6, "y": e_y > 1e-6,
                "x": e_x > 1e-6, "gmres2": gm > 1e-6, "nilpotent": nil > 1e-6}

    assert not any(failing().values())
    # y with the other sign convention: J_P P^-1 then has eigenvalues +-1,
    # so GMRES still takes two steps, but it is no longer I + nilpotent
    monkeypatch.setattr(bb, "proj_t", lambda p, v: -orig_proj_t(p, v))
    f = failing()
    assert f["y"] and f["nilpotent"], f
    monkeypatch.setattr(bb, "proj_t", orig_proj_t)
    # P^T dropped.  On the BB path it is a no-op: a'^T M'^-1 A~ z = 1^T A~ z
    # = 0 for a graph Laplacian A~, so y is unchanged there; with the exact
    # Schur complement it is not, and the two-step pins fail
    monkeypatch.setattr(bb, "proj_t", lambda p, v: np.array(v, dtype=float))
    f = failing()
    assert not f["y"] and f["gmres2"] and f["nilpotent"], f
    monkeypatch.setattr(bb, "proj_t", orig_proj_t)

    # a sign slip inside the pseudo-Schur operator
    def slipped(p, ph, r, sl):
        _, B, _ = kkt_blocks(p, ph, r, sl)
        At = bb.coarse_laplacian_blocks(p, r)
        import scipy.sparse as sp
        Minv = sp.diags(1.0 / np.tile(p.ops.a, p.K + 1))
        return (sp.diags(sl.ravel()) @ At + sp.diags(r.ravel()) @ B @ Minv @ bb.btilde(p, ph)).tocsr()

    monkeypatch.setattr(bb, "pseudo_schur", slipped)
    f = failing()
    assert f["ps"] and f["z"], f
    monkeypatch.setattr(bb, "pseudo_schur", orig_ps)
