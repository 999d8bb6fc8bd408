"""MI355X interior-point solver for finite-volume dynamical optimal transport
with the BB-preconditioned inexact Newton method (arXiv 2209.00315).

Thin Python binding over the C ABI of libotbb.so (include/otbb.h): argument
marshalling only.  Vectors are numpy float64 arrays (host) or torch float64
CUDA tensors (device, read and written on torch's current stream).
"""

import ctypes as C

import numpy as np

from . import _lib
from ._lib import (OT_OK, OT_EINVAL, OT_EMESH, OT_EMASS, OT_ENEG, OT_ELINSOLVE, OT_ENEWTON,  # noqa: F401
                   OT_EDEVICE, OT_ENOMEM, OT_ETIME, OT_FP64, OT_MIXED, OT_HOST, OT_DEVICE, OT_PREC_BB,
                   OT_PREC_SIMPLE, OT_PREC_HYBRID, OT_PREC_PRIMAL, OTError, Options, Stats, check, lib)

__all__ = ["Mesh", "State", "solve", "solve_batched", "options", "OTCost", "OTError", "Stats",
           "kprof_select", "kprof_read", "KPROF"]

# kernel ids of ot_kprof_select (include/otbb.h)
KPROF = {"none": 0, "cheb_fine": 1, "schur_btilde": 2, "schur_out": 3, "tri_fine": 4, "multidot": 5,
         "saddle_phi": 6}


def kprof_select(kernel, elem_bytes=0):
    """Time every launch of one hot-path kernel with HIP events (process-wide);
    elem_bytes 4 / 8 restricts it to the FP32 / FP64 instantiation."""
    check(lib().ot_kprof_select(KPROF[kernel] if isinstance(kernel, str) else int(kernel), int(elem_bytes)))


def kprof_read():
    """(launches, total kernel ms, total algorithmic bytes) since the last select."""
    n, ms, b = C.c_int64(), C.c_double(), C.c_double()
    check(lib().ot_kprof_read(C.byref(n), C.byref(ms), C.byref(b)))
    return n.value, ms.value, b.value


def _is_torch(x):
    return type(x).__module__.startswith("torch")


def _dev_ptr(x):
    if not (x.is_cuda and x.dtype.is_floating_point and x.element_size() == 8 and x.is_contiguous()):
        raise ValueError("device vectors must be contiguous float64 CUDA tensors")
    return C.c_void_p(x.data_ptr())


def _host(x):
    a = np.ascontiguousarray(np.asarray(x, dtype=np.float64))
    return a, C.c_void_p(a.ctypes.data)


def options(**kw):
    """Options with the library defaults, overridden by keyword arguments.
    precision may be 'mixed' / 'fp64' or the OT_* constant."""
    o = Options()
    lib().ot_options_default(C.byref(o))
    for k, v in kw.items():
        if k == "precision" and isinstance(v, str):
            v = {"mixed": OT_MIXED, "fp64": OT_FP64}[v]
        if k == "preconditioner" and isinstance(v, str):
            v = {"bb": OT_PREC_BB, "simple": OT_PREC_SIMPLE, "hybrid": OT_PREC_HYBRID, "primal": OT_PREC_PRIMAL}[v]
        if not hasattr(o, k):
            raise TypeError(f"unknown option {k}")
        setattr(o, k, v)
    return o


class Mesh:
    """Two-level FV mesh (Sec. 2.1 of the paper)."""

    def __init__(self, handle):
        self._h = handle

    @classmethod
    def structured(cls, n, cartesian=False):
        h = C.c_void_p()
        check(lib().ot_mesh_create_structured(int(n), 1 if cartesian else 0, C.byref(h)))
        return cls(h)

    @classmethod
    def cartesian3d(cls, n):
        """n^3 grid of cubes, J = identity (the three-dimensional workload)."""
        h = C.c_void_p()
        check(lib().ot_mesh_create_cartesian3d(int(n), C.byref(h)))
        return cls(h)

    @classmethod
    def from_arrays(cls, fine_area, coarse_area, ov_fine, ov_coarse, ov_area, fe_cell, fe_rho, fe_len,
                    fe_dist, fe_lambda, ce_cell, ce_len, ce_dist, ce_lambda):
        keep = []

        def d(x):
            a = np.ascontiguousarray(np.asarray(x, dtype=np.float64))
            keep.append(a)
            return a.ctypes.data_as(_lib.dptr)

        def i(x):
            a = np.ascontiguousarray(np.asarray(x, dtype=np.int32))
            keep.append(a)
            return a.ctypes.data_as(_lib.iptr)

        desc = _lib.MeshDesc(
            n_fine=len(fine_area), n_coarse=len(coarse_area), fine_area=d(fine_area), coarse_area=d(coarse_area),
            n_overlap=len(ov_area), ov_fine=i(ov_fine), ov_coarse=i(ov_coarse), ov_area=d(ov_area),
            n_fedge=len(fe_len), fe_cell=i(fe_cell), fe_rho=i(fe_rho), fe_len=d(fe_len), fe_dist=d(fe_dist),
            fe_lambda=d(fe_lambda), n_cedge=len(ce_len), ce_cell=i(ce_cell), ce_len=d(ce_len),
            ce_dist=d(ce_dist), ce_lambda=d(ce_lambda))
        h = C.c_void_p()
        check(lib().ot_mesh_create(C.byref(desc), C.byref(h)))
        return cls(h)

    def sizes(self):
        v = [C.c_int32() for _ in range(4)]
        check(lib().ot_mesh_sizes(self._h, *[C.byref(x) for x in v]))
        return tuple(x.value for x in v)

    @property
    def n_fine(self):
        return self.sizes()[0]

    @property
    def n_coarse(self):
        return self.sizes()[1]

    def __del__(self):
        if getattr(self, "_h", None) and _lib._lib is not None:
            _lib._lib.ot_mesh_destroy(self._h)
            self._h = None


class State:
    """Interior-point state (phi, rho, s, mu) on one mesh.

    device=True keeps every vector on the GPU as torch tensors; otherwise
    numpy arrays are used and copied through host memory."""

    def __init__(self, mesh, rho_in, rho_f, K, device=False, **opts):
        self.mesh = mesh
        self.K = int(K)
        self.device = bool(device)
        if self.device:
            import torch
            self._torch = torch
            opts.setdefault("stream", torch.cuda.current_stream().cuda_stream)
            opts["mem_kind"] = OT_DEVICE
        else:
            opts["mem_kind"] = OT_HOST
        self.opt = options(**opts)
        ri, pi = self._in(rho_in)
        rf, pf = self._in(rho_f)
        h = C.c_void_p()
        check(lib().ot_state_create(mesh._h, pi, pf, self.K, C.byref(self.opt), C.byref(h)))
        self._h = h
        nphi, mrho = C.c_int64(), C.c_int64()
        check(lib().ot_state_sizes(h, C.byref(nphi), C.byref(mrho)))
        self.n_phi, self.m_rho = nphi.value, mrho.value
        self.N = self.n_phi + self.m_rho

    # -- marshalling helpers
    def _in(self, x):
        if self.device:
            t = x if _is_torch(x) else self._torch.as_tensor(np.asarray(x, dtype=np.float64))
            t = t.to(device="cuda", dtype=self._torch.float64).contiguous()
            return t, _dev_ptr(t)
        return _host(x)

    def _out(self, n):
        if self.device:
            t = self._torch.empty(n, dtype=self._torch.float64, device="cuda")
            return t, _dev_ptr(t)
        a = np.empty(n)
        return a, C.c_void_p(a.ctypes.data)

    def set_options(self, **kw):
        for k, v in kw.items():
            if k == "precision" and isinstance(v, str):
                v = {"mixed": OT_MIXED, "fp64": OT_FP64}[v]
            if k == "preconditioner" and isinstance(v, str):
                v = {"bb": OT_PREC_BB, "simple": OT_PREC_SIMPLE, "hybrid": OT_PREC_HYBRID, "primal": OT_PREC_PRIMAL}[v]
            setattr(self.opt, k, v)
        check(lib().ot_state_set_options(self._h, C.byref(self.opt)))

    def set_mu(self, mu):
        check(lib().ot_state_set_mu(self._h, float(mu)))

    def residual(self):
        F, pF = self._out(self.n_phi + 2 * self.m_rho)
        nrm = C.c_double()
        check(lib().ot_residual(self._h, pF, C.byref(nrm)))
        return F, nrm.value

    def newton_step(self, raise_on_error=True):
        st = Stats()
        res = C.c_double()
        rc = lib().ot_newton_step(self._h, C.byref(st), C.byref(res))
        if raise_on_error and rc not in (OT_OK,):
            check(rc)
        return rc, st, res.value

    def apply_saddle(self, x):
        xi, px = self._in(x)
        y, py = self._out(self.N)
        check(lib().ot_apply_saddle(self._h, px, py))
        return y

    def apply_schur_prec(self, r):
        ri, pr = self._in(r)
        z, pz = self._out(self.N)
        check(lib().ot_apply_schur_prec(self._h, pr, pz))
        return z

    def export(self):
        phi, p1 = self._out(self.n_phi)
        rho, p2 = self._out(self.m_rho)
        s, p3 = self._out(self.m_rho)
        mu = C.c_double()
        check(lib().ot_state_export(self._h, p1, p2, p3, C.byref(mu)))
        return phi, rho, s, mu.value

    def import_(self, phi, rho, s, mu):
        a, p1 = self._in(phi)
        b, p2 = self._in(rho)
        c, p3 = self._in(s)
        check(lib().ot_state_import(self._h, p1, p2, p3, float(mu)))

    def outputs(self):
        cost, dual = C.c_double(), C.c_double()
        phi, p = self._out(self.n_phi)
        check(lib().ot_outputs(self._h, C.byref(cost), C.byref(dual), p))
        return cost.value, dual.value, phi

    def solve(self, tol=0.0, raise_on_error=True):
        """Interior-point continuation from the current iterate and mu
        (ot_state_solve); returns (rc, stats)."""
        st = Stats()
        rc = lib().ot_state_solve(self._h, float(tol), C.byref(st))
        if raise_on_error and rc != OT_OK:
            check(rc)
        return rc, st

    def gradient(self, raise_on_error=True):
        nc = self.mesh.n_coarse
        gi, p1 = self._out(nc)
        gf, p2 = self._out(nc)
        rc = lib().ot_gradient(self._h, p1, p2)
        if raise_on_error and rc != OT_OK:
            check(rc)
        return gi, gf

    def __del__(self):
        if getattr(self, "_h", None) and _lib._lib is not None:
            _lib._lib.ot_state_destroy(self._h)
            self._h = None


def solve(mesh, rho_in, rho_f, K, tol=1e-6, device=False, raise_on_error=True, **opts):
    """Full interior-point solve.  Returns dict(rho, phi, cost, stats, rc)."""
    nf, nc, _, _ = mesh.sizes()
    if device:
        import torch
        opts.setdefault("stream", torch.cuda.current_stream().cuda_stream)
        opts["mem_kind"] = OT_DEVICE
        ri = torch.as_tensor(rho_in, dtype=torch.float64).to("cuda").contiguous()
        rf = torch.as_tensor(rho_f, dtype=torch.float64).to("cuda").contiguous()
        rho = torch.empty(K * nc, dtype=torch.float64, device="cuda")
        phi = torch.empty((K + 1) * nf, dtype=torch.float64, device="cuda")
        ptrs = [_dev_ptr(t) for t in (ri, rf, rho, phi)]
    else:
        opts["mem_kind"] = OT_HOST
        ri, p1 = _host(rho_in)
        rf, p2 = _host(rho_f)
        rho, phi = np.empty(K * nc), np.empty((K + 1) * nf)
        ptrs = [p1, p2, C.c_void_p(rho.ctypes.data), C.c_void_p(phi.ctypes.data)]
    o = options(**opts)
    cost = C.c_double()
    st = Stats()
    rc = lib().ot_solve(mesh._h, ptrs[0], ptrs[1], int(K), float(tol), C.byref(o), ptrs[2], ptrs[3],
                        C.byref(cost), C.byref(st))
    if raise_on_error and rc != OT_OK:
        check(rc)
    return dict(rho=rho, phi=phi, cost=cost.value, stats=st, rc=rc)


def solve_batched(meshes, rho_ins, rho_fs, Ks, tol=1e-6, raise_on_error=True, **opts):
    """Solve independent problems with one call (host arrays)."""
    n = len(meshes)
    opts["mem_kind"] = OT_HOST
    o = options(**opts)
    keep, outs_r, outs_p = [], [], []
    arr = lambda L: (C.c_void_p * n)(*L)
    mh, pi, pf, pr, pp = [], [], [], [], []
    for m, a, b, K in zip(meshes, rho_ins, rho_fs, Ks):
        nf, nc, _, _ = m.sizes()
        ai, p1 = _host(a)
        bi, p2 = _host(b)
        r, p = np.empty(K * nc), np.empty((K + 1) * nf)
        keep += [ai, bi]
        outs_r.append(r)
        outs_p.append(p)
        mh.append(m._h.value); pi.append(p1.value); pf.append(p2.value)
        pr.append(r.ctypes.data); pp.append(p.ctypes.data)
    costs = np.zeros(n)
    stats = (Stats * n)()
    Karr = (C.c_int32 * n)(*[int(k) for k in Ks])
    rc = lib().ot_solve_batched(n, arr(mh), arr(pi), arr(pf), Karr, float(tol), C.byref(o), arr(pr), arr(pp),
                                costs.ctypes.data_as(_lib.dptr), stats)
    if raise_on_error and rc != OT_OK:
        check(rc)
    return dict(rho=outs_r, phi=outs_p, cost=costs, stats=list(stats), rc=rc)


def _make_otcost():
    import torch

    class OTCost(torch.autograd.Function):
        """cost = discrete kinetic energy of the transport from rho_in to
        rho_f; backward returns d cost / d rho_in and d cost / d rho_f
        (envelope term + adjoint saddle solve), orthogonal to the coarse areas."""

        @staticmethod
        def forward(ctx, rho_in, rho_f, mesh, K, opts):
            opts = dict(opts or {})
            tol = opts.pop("tol", 1e-6)
            dev = rho_in.is_cuda
            st = State(mesh, rho_in.detach().double().contiguous(), rho_f.detach().double().contiguous(), K,
                       device=dev, **opts)
            _, stats = st.solve(tol)
            cost = stats.cost
            ctx.state = st
            return torch.tensor(cost, dtype=torch.float64, device=rho_in.device)

        @staticmethod
        def backward(ctx, g):
            gi, gf = ctx.state.gradient()
            if not _is_torch(gi):
                gi, gf = torch.as_tensor(gi), torch.as_tensor(gf)
            gi = gi.to(g.device) * g
            gf = gf.to(g.device) * g
            return gi, gf, None, None, None

    return OTCost


class _LazyOTCost:
    _cls = None

    def __getattr__(self, name):
        if _LazyOTCost._cls is None:
            _LazyOTCost._cls = _make_otcost()
        return getattr(_LazyOTCost._cls, name)


OTCost = _LazyOTCost()
