"""MI355X (gfx950) hot path of the isogeometric Galerkin BEM of Bembel (arXiv 1906.00785).

Thin object layer over the C ABI (include/bem.h, libbem_hip.so).  Torch provides device
memory and the stream; every numerical step runs in the library's HIP kernels.

    geom = Geometry(BEM_GEOM_SPHERE6)
    space = Space(geom, BEM_LAPLACE_SINGLE, 0.0, degree=2, level=6)
    A = Operator(space, q=5, eta=1.6, leaf_level=4)        # plan + assemble on the GPU
    b = space.rhs(BEM_DATA_POINT_SOURCE, [(0.1, -0.2, 0.15)])
    rho, stats = A.solve(b, tol=1e-8)
    u = space.potential(points, rho)
"""
from __future__ import annotations

import numpy as np
import torch

from . import _bem as C
from ._bem import (BEM_DATA_DIPOLE, BEM_DATA_PLANE_WAVE, BEM_DATA_PLANE_WAVE_E, BEM_DATA_POINT_SOURCE,
                   BEM_GEOM_ELLIPSOID6, BEM_GEOM_FLAT1, BEM_GEOM_NURBS, BEM_GEOM_SPHERE6, BEM_GEOM_TORUS16,
                   BEM_HELMHOLTZ_SINGLE, BEM_LAPLACE_SINGLE, BEM_MAXWELL_SINGLE, BEM_PREC_BF16, BEM_PREC_FP32,
                   BEM_PREC_FP64, BemError)

__all__ = ["Geometry", "Space", "Operator", "BemError", "BEM_GEOM_SPHERE6", "BEM_GEOM_ELLIPSOID6",
           "BEM_GEOM_TORUS16", "BEM_GEOM_FLAT1", "BEM_GEOM_NURBS", "BEM_LAPLACE_SINGLE", "BEM_HELMHOLTZ_SINGLE",
           "BEM_MAXWELL_SINGLE", "BEM_DATA_POINT_SOURCE", "BEM_DATA_PLANE_WAVE", "BEM_DATA_DIPOLE",
           "BEM_DATA_PLANE_WAVE_E", "BEM_PREC_FP64", "BEM_PREC_FP32", "BEM_PREC_BF16"]


def _stream() -> int:
    return torch.cuda.current_stream().cuda_stream


def _dev() -> torch.device:
    if not torch.cuda.is_available():
        raise RuntimeError("no GPU visible: the BEM path runs only on the GPU")
    return torch.device("cuda", torch.cuda.current_device())


class Geometry:
    """Analytic geometry (kind, params), or NURBS patches via the constructors below."""

    def __init__(self, kind: int, params=(), _handle=None):
        self.kind, self.params = kind, tuple(params)
        self.h = _handle if _handle is not None else C.bem_geometry_analytic(kind, self.params)

    @classmethod
    def nurbs(cls, patches):
        """patches: list of {"degree": (p1, p2), "knots": (Xi_1, Xi_2), "cw": (k1, k2, 4)}."""
        return cls(BEM_GEOM_NURBS, (), _handle=C.bem_geometry_nurbs(patches))

    @classmethod
    def load(cls, path: str):
        """NURBS patches from a BEMNURBS text file."""
        return cls(BEM_GEOM_NURBS, (), _handle=C.bem_geometry_load(path))

    @classmethod
    def user(cls, npatch: int, fn, degree: int = 5, intervals: int = 8):
        """User patch maps fn(patch, st) -> xyz, replaced by their tensor B-spline interpolants."""
        return cls(BEM_GEOM_NURBS, (), _handle=C.bem_geometry_user(npatch, fn, degree, intervals))

    def save(self, path: str):
        C.bem_geometry_save(self.h, path)

    def __del__(self):
        if getattr(self, "h", None):
            try:
                C.bem_geometry_destroy(self.h)
            except Exception:
                pass
            self.h = None


class Space:
    def __init__(self, geom: Geometry, kernel: int = BEM_LAPLACE_SINGLE, kappa: complex = 0.0, degree: int = 1,
                 knot_repetition: int = 1, level: int = 0, continuous: bool = False):
        """continuous=True: the S^0 space (glued across patches, 0-form lifting); else S^2.  The
        Maxwell single layer (kernel BEM_MAXWELL_SINGLE) takes the div-conforming S^1 space of
        that degree (vector densities, complex)."""
        self.vector = kernel == C.BEM_MAXWELL_SINGLE
        kind = C.BEM_SPACE_S1 if self.vector else (C.BEM_SPACE_S0 if continuous else C.BEM_SPACE_S2)
        self.h = C.bem_space_create(geom.h, kernel, kappa, degree, knot_repetition, level, kind)
        self.continuous = bool(continuous)
        self.geom = geom
        self.kernel, self.kappa, self.degree, self.level = kernel, complex(kappa), degree, level
        self.knot_repetition = knot_repetition
        self.ndof = C.bem_space_ndof(self.h)
        self.dtype = torch.complex128 if kernel != BEM_LAPLACE_SINGLE else torch.float64

    def glue(self) -> np.ndarray:
        """Global function of every local function (the identity for S^2; -1: dropped S^1 function)."""
        return C.bem_space_glue(self.h)[1]

    def glue_sign(self) -> np.ndarray:
        """Sign of every local function in its global function (+1 except on S^1 spaces)."""
        return C.bem_space_glue_sign(self.h)

    def __del__(self):
        if getattr(self, "h", None):
            try:
                C.bem_space_destroy(self.h)
            except Exception:
                pass
            self.h = None

    def rhs(self, data_kind: int, params) -> torch.Tensor:
        """Load vectors, one per row of params (3 numbers each; 6 for the Maxwell data kinds):
        tensor (nrhs, N)."""
        params = [tuple(float(v) for v in p) for p in params]
        b = torch.empty((len(params), self.ndof), dtype=self.dtype, device=_dev())
        C.bem_rhs(self.h, data_kind, params, len(params), b.data_ptr(), self.ndof, _stream())
        return b

    def quadpoints(self) -> torch.Tensor:
        """The load vector's quadrature points, tensor (npts, 3) on the GPU."""
        n = C.bem_rhs_quadpoints(self.h, None, _stream())
        xyz = torch.empty((n, 3), dtype=torch.float64, device=_dev())
        C.bem_rhs_quadpoints(self.h, xyz.data_ptr(), _stream())
        return xyz

    def rhs_from_samples(self, g: torch.Tensor) -> torch.Tensor:
        """Load vectors from data sampled at quadpoints(): g of shape (nrhs, npts) or (npts,)."""
        gg = g.reshape(-1, g.shape[-1]).to(self.dtype).contiguous()
        assert gg.is_cuda
        b = torch.empty((gg.shape[0], self.ndof), dtype=self.dtype, device=_dev())
        C.bem_rhs_from_samples(self.h, gg.data_ptr(), gg.shape[1], gg.shape[0], b.data_ptr(), self.ndof, _stream())
        return b if g.dim() > 1 else b[0]

    def write_vtk(self, path: str, rho=None, nsub: int = 4):
        """Surface mesh and density (rows of rho: (nrhs, N) or (N,), host or device) as VTK."""
        if rho is None:
            C.bem_write_vtk(self.h, None, self.ndof, 0, nsub, path)
            return
        r = torch.as_tensor(rho).reshape(-1, self.ndof).to("cpu", self.dtype).contiguous()
        C.bem_write_vtk(self.h, r.data_ptr(), self.ndof, r.shape[0], nsub, path)

    def potential(self, pts, rho: torch.Tensor) -> torch.Tensor:
        """Potential at points (npts, 3) for densities rho (nrhs, N) or (N,); for the Maxwell
        single layer the field (MS), shape (nrhs, npts, 3) or (npts, 3)."""
        pts = torch.as_tensor(np.asarray(pts, dtype=np.float64)).to(_dev()).contiguous()
        r = rho.reshape(-1, self.ndof).contiguous()
        if self.vector:
            E = torch.empty((r.shape[0], pts.shape[0], 3), dtype=self.dtype, device=_dev())
            C.bem_eval_potential(self.h, pts.data_ptr(), pts.shape[0], r.data_ptr(), self.ndof, r.shape[0],
                                 E.data_ptr(), 3 * pts.shape[0], _stream())
            return E[0] if rho.dim() == 1 else E
        u = torch.empty((r.shape[0], pts.shape[0]), dtype=self.dtype, device=_dev())
        C.bem_eval_potential(self.h, pts.data_ptr(), pts.shape[0], r.data_ptr(), self.ndof, r.shape[0], u.data_ptr(),
                             pts.shape[0], _stream())
        return u.reshape(rho.shape[:-1] + (pts.shape[0],)) if rho.dim() == 1 else u


class Operator:
    """Compressed single-layer operator: plan on the host, assemble on the GPU."""

    def __init__(self, space: Space, q: int = 5, eta: float | None = None, leaf_level: int = -1, qg: int = 8, qs: int = 8,
                 assemble: bool = True, chunk_cols: int = 0, far_low: int = 0, batch_rhs: int = 0,
                 far_eval: bool = False, kappa_adm: float = 0.0):
        self.space = space
        if eta is None:
            eta = 0.0 if space.vector else 1.6  # Maxwell operators are dense
        self.far_low = far_low
        self.batch_rhs = batch_rhs
        self.far_eval = bool(far_eval)
        self.h, self.info = C.bem_assemble_plan(space.h, q, eta, leaf_level, qg, qs, chunk_cols, far_low, batch_rhs,
                                                int(far_eval), float(kappa_adm))
        self.q, self.eta = q, eta
        self.ndof = self.info.ndof
        self.op_ws = None
        if assemble:
            self.assemble()

    def __del__(self):
        if getattr(self, "h", None):
            try:
                C.bem_operator_destroy(self.h)
            except Exception:
                pass
            self.h = None

    def assemble(self):
        dev = _dev()
        self.op_ws = torch.empty(self.info.op_bytes, dtype=torch.uint8, device=dev)
        tmp = torch.empty(self.info.tmp_bytes, dtype=torch.uint8, device=dev)
        C.bem_assemble(self.h, self.op_ws.data_ptr(), self.info.op_bytes, tmp.data_ptr(), self.info.tmp_bytes,
                       _stream())
        torch.cuda.current_stream().synchronize()
        del tmp

    def apply(self, x: torch.Tensor, out: torch.Tensor | None = None, prec: int = BEM_PREC_FP64) -> torch.Tensor:
        """y = A x for x of shape (N,) or (nrhs, N); prec selects the far-field coupling's
        precision (BEM_PREC_FP64 or the far_low the operator was assembled with).  With
        batch_rhs > 1 several columns go through the many-RHS kernels together."""
        xx = x.reshape(-1, self.ndof).contiguous()
        y = out if out is not None else torch.empty_like(xx)
        C.bem_apply_ex(self.h, prec, xx.data_ptr(), self.ndof, y.data_ptr(), self.ndof, xx.shape[0], _stream())
        return y.reshape(x.shape)

    def solve(self, b: torch.Tensor, tol: float = 1e-8, restart: int = 30, maxit: int = 2000, refine: bool = False,
              inner_tol: float = 0.0, max_outer: int = 0, precond: bool = False, inner_maxit: int = 0):
        """GMRES(restart), optionally right-preconditioned with the block preconditioner
        (precond_build first) and/or inside FP64 iterative refinement with the
        low-precision far field; returns (x, [(iterations, converged, relres, outer)])."""
        bb = b.reshape(-1, self.ndof).contiguous()
        x = torch.empty_like(bb)
        nbytes = C.bem_solve_plan(self.h, bb.shape[0], restart, maxit, tol, int(refine), max_outer)
        ws = torch.empty(nbytes, dtype=torch.uint8, device=bb.device)
        _, stats = C.bem_solve(self.h, bb.data_ptr(), self.ndof, x.data_ptr(), self.ndof, bb.shape[0], restart, maxit,
                               tol, ws.data_ptr(), nbytes, _stream(), int(refine), max_outer, inner_tol, int(precond),
                               inner_maxit)
        return x.reshape(b.shape), stats

    # ---- block-Jacobi preconditioner and its learned correction
    def precond_build(self):
        """Extracts and inverts the 8 x 8-tile diagonal blocks of the near field."""
        self.ntiles, nbytes = C.bem_precond_info(self.h)
        self.prec_ws = torch.empty(nbytes, dtype=torch.uint8, device=_dev())
        C.bem_precond_build(self.h, self.prec_ws.data_ptr(), nbytes, _stream())

    def precond_apply(self, r: torch.Tensor) -> torch.Tensor:
        rr = r.reshape(-1, self.ndof).contiguous()
        z = torch.empty_like(rr)
        C.bem_precond_apply(self.h, rr.data_ptr(), self.ndof, z.data_ptr(), self.ndof, rr.shape[0], _stream())
        return z.reshape(r.shape)

    def precond_export(self, which: int = 0) -> np.ndarray:
        npdt = np.complex128 if self.space.dtype == torch.complex128 else np.float64
        out = np.zeros((self.ntiles, 64, 64), dtype=npdt)
        C.bem_precond_export(self.h, which, out.ctypes.data, _stream())
        return out

    def precond_features(self) -> torch.Tensor:
        f = torch.empty((self.ntiles, 99), dtype=torch.float32, device=_dev())
        C.bem_precond_features(self.h, f.data_ptr(), _stream())
        return f

    def precond_targets(self, ring: int = 2, per_pass: int = 256) -> torch.Tensor:
        """(X_b - D_b^{-1}) / s_b for every tile, float (ntiles, 64, 64[, 2]), X_b the block
        least-squares approximate inverse on the tile extended by `ring` indices."""
        cplx = self.space.dtype == torch.complex128
        shape = (self.ntiles, 64, 64, 2) if cplx else (self.ntiles, 64, 64)
        delta = torch.empty(shape, dtype=torch.float32, device=_dev())
        per_pass = max(1, min(per_pass, self.ntiles))
        nbytes = C.bem_precond_target_bytes(self.h, ring, per_pass)
        work = torch.empty(nbytes, dtype=torch.uint8, device=_dev())
        for t0 in range(0, self.ntiles, per_pass):
            nt = min(per_pass, self.ntiles - t0)
            C.bem_precond_targets(self.h, ring, t0, nt, work.data_ptr(), nbytes, delta.data_ptr(), _stream())
        return delta

    def precond_correct(self, uv: torch.Tensor | None, mode: int = 2, ring: int = 2) -> np.ndarray:
        """Install the learned correction from the network output (mode 2: per-block probe
        test, 1: keep all, 0: plain block-Jacobi); returns the accepted flags."""
        acc = np.zeros(self.ntiles, dtype=np.int32)
        ptr = uv.contiguous().data_ptr() if uv is not None else None
        C.bem_precond_correct(self.h, ptr, mode, ring, acc.ctypes.data, _stream())
        return acc

    def profile(self, on: bool):
        """Enable/disable HIP-event timing of the four apply stages."""
        C.bem_profile_enable(self.h, on)

    def profile_read(self):
        """(mean ms per stage [near + forward/upward, coupling, gather, downward/backward],
        number of applies)."""
        return C.bem_profile_read(self.h)

    def apply_stage(self, stage: int, x: torch.Tensor, y: torch.Tensor, prec: int = BEM_PREC_FP64):
        """Launch one stage of a one-column apply alone (profiling aid; see bem_apply_stage)."""
        assert x.is_cuda and y.is_cuda and x.numel() >= self.ndof and y.numel() >= self.ndof
        assert x.dtype == self.space.dtype and y.dtype == self.space.dtype and x.is_contiguous() and y.is_contiguous()
        C.bem_apply_stage(self.h, prec, stage, x.data_ptr(), y.data_ptr(), _stream())

    # ---- parity exports
    def potential(self, pts, rho: torch.Tensor, eta: float | None = None) -> torch.Tensor:
        """Potential at points (npts, 3) for densities rho (nrhs, N) or (N,) through the
        cluster tree (eta: admissibility of point and cluster, default the operator's)."""
        pts = torch.as_tensor(np.asarray(pts, dtype=np.float64)).to(_dev()).contiguous()
        r = rho.reshape(-1, self.ndof).contiguous()
        u = torch.empty((r.shape[0], pts.shape[0]), dtype=self.space.dtype, device=_dev())
        C.bem_eval_potential_h2(self.h, pts.data_ptr(), pts.shape[0], r.data_ptr(), self.ndof, r.shape[0],
                                u.data_ptr(), pts.shape[0], float(self.eta if eta is None else eta), _stream())
        return u.reshape(rho.shape[:-1] + (pts.shape[0],)) if rho.dim() == 1 else u

    def export_near(self):
        """Near field on the local functions (patch by patch), CSR."""
        n = self.info.nlocal
        rowptr = np.zeros(n + 1, dtype=np.int64)
        col = np.zeros(self.info.near_nnz, dtype=np.int32)
        npdt = np.complex128 if self.space.dtype == torch.complex128 else np.float64
        val = np.zeros(self.info.near_nnz, dtype=npdt)
        C.bem_export_near(self.h, rowptr.ctypes.data, col.ctypes.data, val.ctypes.data, _stream())
        return rowptr, col, val

    def export_far(self):
        q2 = self.q * self.q
        pairs = np.zeros((self.info.nfar, 2), dtype=np.int64)
        npdt = np.complex128 if self.space.dtype == torch.complex128 else np.float64
        blocks = np.zeros((self.info.nfar, q2, q2), dtype=npdt)
        C.bem_export_far(self.h, pairs.ctypes.data, blocks.ctypes.data, _stream())
        return pairs, blocks

    def moments(self, x: torch.Tensor) -> np.ndarray:
        q2 = self.q * self.q
        npdt = np.complex128 if self.space.dtype == torch.complex128 else np.float64
        m = np.zeros((self.info.nclusters, q2), dtype=npdt)
        xx = x.contiguous()
        C.bem_export_moments(self.h, xx.data_ptr(), m.ctypes.data, _stream())
        return m


class Group:
    """Columns of several operators (same PDE kind and q) applied with one launch per
    matvec stage.  xs, ys: lists of (ncols_i, N_i) tensors (contiguous rows = columns)."""

    def __init__(self, ops, xs, ys):
        self.ops = list(ops)
        ncols = [int(x.reshape(-1, op.ndof).shape[0]) for op, x in zip(self.ops, xs)]
        self.h, nbytes = C.bem_group_create([op.h for op in self.ops], ncols)
        self.ws = torch.empty(nbytes, dtype=torch.uint8, device=_dev())
        xp, yp = [], []
        for op, x, y in zip(self.ops, xs, ys):
            xx, yy = x.reshape(-1, op.ndof), y.reshape(-1, op.ndof)
            assert xx.is_contiguous() and yy.is_contiguous()
            for c in range(xx.shape[0]):
                xp.append(xx[c].data_ptr())
                yp.append(yy[c].data_ptr())
        self.xs, self.ys = xs, ys  # keep the bound buffers alive
        C.bem_group_bind(self.h, self.ws.data_ptr(), nbytes, xp, yp, _stream())

    def apply(self):
        C.bem_group_apply(self.h, _stream())

    def __del__(self):
        if getattr(self, "h", None):
            try:
                C.bem_group_destroy(self.h)
            except Exception:  # interpreter shutdown: the binding module may already be gone
                pass
            self.h = None


class Graph:
    """Stream capture of library calls (kernel launches only), replayed with one launch.
    Usage: g = Graph(); with g: ...calls...; g.launch()."""

    def __init__(self):
        self.h = None

    def __enter__(self):
        C.bem_capture_begin(_stream())
        return self

    def __exit__(self, et, ev, tb):
        h = C.bem_capture_end(_stream())
        if et is None:
            self.h = h
        else:
            C.bem_graph_destroy(h)
        return False

    def launch(self):
        C.bem_graph_launch(self.h, _stream())

    def __del__(self):
        if getattr(self, "h", None):
            try:
                C.bem_graph_destroy(self.h)
            except Exception:  # interpreter shutdown: the binding module may already be gone
                pass
            self.h = None
