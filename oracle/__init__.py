"""Oracle of the isogeometric Galerkin BEM hot path (ctypes binding of bem_oracle.cpp).

TEST INFRASTRUCTURE ONLY.  Only tests/, the smoke check in __graft_entry__ and the
cpu_baseline leg of bench.py may import this package.  The product path (the HIP library
and its Python binding) never imports, links or executes anything here, and this package
never imports the product path.

The oracle is plain serial FP64 C++ (oracle/bem_oracle.cpp); this module only marshals
numpy arrays.  Complex quantities are numpy complex128 arrays, passed as interleaved
(re, im) doubles.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "bem_oracle.cpp")
_LIB = os.path.join(_HERE, "_build", "liboracle.so")

# geometry kinds, PDEs and data kinds (same numbering as the C code)
SPHERE, ELLIPSOID, TORUS, FLAT, NURBS = 0, 1, 2, 3, 4
LAPLACE, HELMHOLTZ = 0, 1
POINT_SOURCE, PLANE_WAVE = 0, 1


def build(force: bool = True) -> str:
    """Compile liboracle.so with g++ (plain -O2, no fast-math; OpenMP for the timing mode)."""
    os.makedirs(os.path.dirname(_LIB), exist_ok=True)
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        cmd = ["g++", "-std=c++17", "-O2", "-fPIC", "-fopenmp", "-shared", "-o", tmp, _SRC]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        L = ctypes.CDLL(_LIB)
        P, I, I64, D = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, ctypes.c_double
        sig = {
            "orc_last_error": (ctypes.c_char_p, []),
            "orc_gauss01": (I, [I, P, P]),
            "orc_bspline": (I, [I, I, I, I, I64, P, P]),
            "orc_bspline_count": (I, [I, I, I]),
            "orc_space_new": (I, [I, P, I, I, D, D, I, I, I, P]),
            "orc_space_new_nurbs": (I, [I, P, P, P, I, D, D, I, I, I, P]),
            "orc_h2_potential": (I, [P, P, I64, P, D, P]),
            "orc_space_set_form": (I, [P, I]),
            "orc_space_glue": (I, [P, P, P]),
            "orc_set_threads": (I, [I]),
            "orc_space_free": (None, [P]),
            "orc_space_ndof": (I64, [P]),
            "orc_space_nelem": (I64, [P]),
            "orc_gamma": (I, [P, I, I64, P, P, P, P]),
            "orc_area": (I, [P, I, P]),
            "orc_classify": (I, [P, I64, I64, P]),
            "orc_pair_block": (I, [P, I64, I64, I, I, P]),
            "orc_dense": (I, [P, I, I, P]),
            "orc_density_pairing": (I, [P, I, I, I, I, P]),
            "orc_rhs": (I, [P, I, P, I, I, P]),
            "orc_potential": (I, [P, I, P, I64, P, P]),
            "orc_h2_new": (I, [P, I, D, I, I, I, I, D, P]),
            "orc_h2_free": (None, [P]),
            "orc_h2_info": (I, [P, P]),
            "orc_h2_lists": (I, [P, P, P]),
            "orc_h2_clusters": (I, [P, P, P]),
            "orc_h2_tables": (I, [P, P, P, P, P]),
            "orc_h2_near_csr": (I, [P, P, P, P]),
            "orc_h2_moments": (I, [P, P, I, P]),
            "orc_h2_apply": (I, [P, P, P, I]),
            "orc_h2_apply_rows": (I, [P, P, P, I64, I, P]),
            "orc_h2_gmres": (I, [P, P, P, D, I, I, P]),
            "orc_h2_near_rows": (I, [P, P, I64]),
            "orc_dense_gmres": (I, [I64, I, P, P, P, D, I, I, P]),
            "orc_bj_new": (I, [P, I, P]),
            "orc_bj_free": (None, [P]),
            "orc_bj_ntiles": (I64, [P]),
            "orc_bj_tile": (I, [P, I64, P, P]),
            "orc_bj_block": (I, [P, I64, P]),
            "orc_bj_apply": (I, [P, P, P]),
            "orc_bj_target": (I, [P, I64, I, P]),
            "orc_h2_gmres_bj": (I, [P, P, P, P, D, I, I, P]),
            "orc_tile_features": (I, [P, I, P]),
            "orc_mspace_new": (I, [I, P, I, D, D, I, I, P]),
            "orc_mspace_new_nurbs": (I, [I, P, P, P, D, D, I, I, P]),
            "orc_mspace_free": (None, [P]),
            "orc_mspace_info": (I, [P, P]),
            "orc_mspace_glue": (I, [P, P, P]),
            "orc_m_elem_eval": (I, [P, I64, D, D, P, P, P, P]),
            "orc_m_pair_block": (I, [P, I64, I64, I, I, I, P]),
            "orc_m_dense": (I, [P, I, I, I, P]),
            "orc_m_h2_dense": (I, [P, I, D, I, I, I, D, I, P]),
            "orc_m_rhs": (I, [P, I, P, I, I, P]),
            "orc_m_potential": (I, [P, I, P, I64, P, P]),
            "orc_m_field": (I, [I, P, D, D, I64, P, P]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _check(rc):
    if rc != 0:
        raise RuntimeError("oracle: " + lib().orc_last_error().decode())


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def set_threads(n: int) -> int:
    """Threads of the oracle's timing mode (parallel loops over independent rows, clusters
    and target runs; results are the same for any count).  Returns the count in effect."""
    return lib().orc_set_threads(int(n))


def gauss01(n: int):
    x = np.zeros(n)
    w = np.zeros(n)
    _check(lib().orc_gauss01(n, _p(x), _p(w)))
    return x, w


def bspline(d: int, r: int, L: int, j: int, x) -> np.ndarray:
    x = np.ascontiguousarray(x, dtype=np.float64)
    out = np.zeros_like(x)
    _check(lib().orc_bspline(d, r, L, j, x.size, _p(x), _p(out)))
    return out


def bspline_count(d: int, r: int, L: int) -> int:
    return lib().orc_bspline_count(d, r, L)


class Space:
    """Discrete space S^2 on an analytic multi-patch geometry, with its PDE."""

    def __init__(self, geom: int, gparams=(), pde: int = LAPLACE, kappa: complex = 0.0,
                 degree: int = 1, knot_rep: int = 1, level: int = 0, form: int = 2):
        """geom: an analytic kind with its parameters, or NURBS with gparams a list of patches,
        each a dict with "degree" (p1, p2), "knots" (Xi_1, Xi_2) and "cw", an array
        (k1, k2, 4) of control points and weights (App. C)."""
        h = ctypes.c_void_p()
        if geom == NURBS:
            meta, knots, cw = [], [], []
            for P in gparams:
                c = np.asarray(P["cw"], dtype=np.float64)
                meta += [int(P["degree"][0]), int(P["degree"][1]), c.shape[0], c.shape[1]]
                knots += [np.asarray(P["knots"][0], dtype=np.float64), np.asarray(P["knots"][1], dtype=np.float64)]
                cw.append(c.reshape(-1))
            m = np.ascontiguousarray(meta, dtype=np.int32)
            kn = np.ascontiguousarray(np.concatenate(knots))
            cc = np.ascontiguousarray(np.concatenate(cw))
            _check(lib().orc_space_new_nurbs(len(gparams), m.ctypes.data, _p(kn), _p(cc), pde,
                                             float(np.real(kappa)), float(np.imag(kappa)), degree, knot_rep, level,
                                             ctypes.byref(h)))
        else:
            gp = np.ascontiguousarray(np.asarray(gparams, dtype=np.float64).reshape(-1))
            if gp.size == 0:
                gp = np.zeros(1)
            _check(lib().orc_space_new(geom, _p(gp), int(len(gparams)), pde, float(np.real(kappa)),
                                       float(np.imag(kappa)), degree, knot_rep, level, ctypes.byref(h)))
        self._h = h
        self.form = form
        if form != 2:
            _check(lib().orc_space_set_form(self._h, form))
        self.pde = pde
        self.complex = pde == HELMHOLTZ
        self.degree, self.level, self.knot_rep = degree, level, knot_rep
        self.geom = geom
        self.dtype = np.complex128 if self.complex else np.float64

    def __del__(self):
        if getattr(self, "_h", None):
            try:
                lib().orc_space_free(self._h)
            except Exception:
                pass
            self._h = None

    @property
    def ndof(self) -> int:
        """Local functions (patch by patch); the glued space has glue()[1] of them."""
        return lib().orc_space_ndof(self._h)

    def glue(self):
        """S^0 continuity: (map local -> global, number of global functions)."""
        m = np.zeros(self.ndof, dtype=np.int64)
        n = ctypes.c_int64()
        _check(lib().orc_space_glue(self._h, _p(m), ctypes.byref(n)))
        return m, int(n.value)

    @property
    def nelem(self) -> int:
        return lib().orc_space_nelem(self._h)

    def gamma(self, patch: int, st):
        st = np.ascontiguousarray(st, dtype=np.float64).reshape(-1, 2)
        n = st.shape[0]
        xyz = np.zeros((n, 3))
        kap = np.zeros(n)
        nrm = np.zeros((n, 3))
        _check(lib().orc_gamma(self._h, patch, n, _p(st), _p(xyz), _p(kap), _p(nrm)))
        return xyz, kap, nrm

    def area(self, q: int = 8) -> float:
        a = ctypes.c_double()
        _check(lib().orc_area(self._h, q, ctypes.byref(a)))
        return a.value

    def classify(self, e1: int, e2: int):
        out = np.zeros(3, dtype=np.int32)
        _check(lib().orc_classify(self._h, e1, e2, _p(out)))
        return tuple(int(v) for v in out)

    def pair_block(self, e1: int, e2: int, qg: int = 8, qs: int = 8) -> np.ndarray:
        nb = (self.degree + 1) ** 2
        B = np.zeros((nb, nb), dtype=self.dtype)
        _check(lib().orc_pair_block(self._h, e1, e2, qg, qs, _p(B)))
        return B

    def dense(self, qg: int = 8, qs: int = 8) -> np.ndarray:
        N = self.ndof
        A = np.zeros((N, N), dtype=self.dtype)
        _check(lib().orc_dense(self._h, qg, qs, _p(A)))
        return A

    def density_pairing(self, fid: int, gid: int, qg: int = 8, qs: int = 8) -> complex:
        out = np.zeros(2)
        _check(lib().orc_density_pairing(self._h, fid, gid, qg, qs, _p(out)))
        return complex(out[0], out[1])

    def rhs(self, kind: int, params, q: int = 8) -> np.ndarray:
        prm = np.ascontiguousarray(np.asarray(params, dtype=np.float64).reshape(-1, 3))
        nrhs = prm.shape[0]
        b = np.zeros((nrhs, self.ndof), dtype=self.dtype)
        _check(lib().orc_rhs(self._h, kind, _p(prm), nrhs, q, _p(b)))
        return b.T.copy() if nrhs > 1 else b[0]

    def potential(self, rho, pts, q: int = 8) -> np.ndarray:
        rho = np.ascontiguousarray(rho, dtype=self.dtype)
        pts = np.ascontiguousarray(pts, dtype=np.float64).reshape(-1, 3)
        u = np.zeros(pts.shape[0], dtype=self.dtype)
        _check(lib().orc_potential(self._h, q, _p(rho), pts.shape[0], _p(pts), _p(u)))
        return u


class H2:
    """H^2 operator of a Space (near field optional: assemble_near=False keeps it lazy)."""

    def __init__(self, space: Space, q: int = 5, eta: float = 1.6, leaf: int = 0, qg: int = 8,
                 qs: int = 8, assemble_near: bool = True, kappa_adm: float = 0.0):
        self.space = space
        h = ctypes.c_void_p()
        _check(lib().orc_h2_new(space._h, q, eta, leaf, qg, qs, int(assemble_near), float(kappa_adm),
                                ctypes.byref(h)))
        self._h = h
        self.q, self.eta, self.leaf = q, eta, leaf
        info = np.zeros(6, dtype=np.int64)
        _check(lib().orc_h2_info(self._h, _p(info)))
        self.nclusters, self.nfar, self.nnear, self.nnz, self.nloc, self.qm = (int(v) for v in info)

    def __del__(self):
        if getattr(self, "_h", None):
            try:
                lib().orc_h2_free(self._h)
            except Exception:
                pass
            self._h = None

    def lists(self):
        far = np.zeros((self.nfar, 2), dtype=np.int64)
        near = np.zeros((self.nnear, 2), dtype=np.int64)
        _check(lib().orc_h2_lists(self._h, _p(far), _p(near)))
        return far, near

    def clusters(self):
        ids = np.zeros((self.nclusters, 4), dtype=np.int32)
        balls = np.zeros((self.nclusters, 4))
        _check(lib().orc_h2_clusters(self._h, _p(ids), _p(balls)))
        return ids, balls

    def tables(self):
        q2 = self.q * self.q
        K = np.zeros((self.nfar, q2, q2), dtype=self.space.dtype)
        E0 = np.zeros((self.q, self.q))
        E1 = np.zeros((self.q, self.q))
        nl = 1 << self.leaf
        V1 = np.zeros((nl, self.q, self.nloc))
        _check(lib().orc_h2_tables(self._h, _p(K), _p(E0), _p(E1), _p(V1)))
        return K, E0, E1, V1

    def near_csr(self):
        N = self.space.ndof
        rowptr = np.zeros(N + 1, dtype=np.int64)
        col = np.zeros(self.nnz, dtype=np.int64)
        val = np.zeros(self.nnz, dtype=self.space.dtype)
        _check(lib().orc_h2_near_csr(self._h, _p(rowptr), _p(col), _p(val)))
        return rowptr, col, val

    def moments(self, x, direct: bool = False):
        x = np.ascontiguousarray(x, dtype=self.space.dtype)
        m = np.zeros((self.nclusters, self.q * self.q), dtype=self.space.dtype)
        _check(lib().orc_h2_moments(self._h, _p(x), int(direct), _p(m)))
        return m

    def apply(self, x) -> np.ndarray:
        x = np.asarray(x, dtype=self.space.dtype)
        N = self.space.ndof
        X = np.ascontiguousarray(x.reshape(N, -1).T)
        Y = np.zeros_like(X)
        _check(lib().orc_h2_apply(self._h, _p(X), _p(Y), X.shape[0]))
        return Y.T.reshape(x.shape)

    def apply_rows(self, x, rows, far: bool = True, near: bool = True) -> np.ndarray:
        x = np.ascontiguousarray(x, dtype=self.space.dtype)
        rows = np.ascontiguousarray(rows, dtype=np.int64)
        y = np.zeros(rows.size, dtype=self.space.dtype)
        parts = (1 if far else 0) | (2 if near else 0)
        _check(lib().orc_h2_apply_rows(self._h, _p(x), _p(rows), rows.size, parts, _p(y)))
        return y

    def potential(self, rho, pts, eta: float | None = None) -> np.ndarray:
        """Potential at points (n, 3) by the cluster tree: admissible clusters through their
        moments and Chebyshev points, near leaves by 8x8 Gauss (eta: admissibility of
        point and cluster; default the operator's; 0 gives the plain quadrature)."""
        rho = np.ascontiguousarray(rho, dtype=self.space.dtype)
        pts = np.ascontiguousarray(pts, dtype=np.float64).reshape(-1, 3)
        u = np.zeros(pts.shape[0], dtype=self.space.dtype)
        _check(lib().orc_h2_potential(self._h, _p(rho), pts.shape[0], _p(pts), float(self.eta if eta is None else eta),
                                      _p(u)))
        return u

    def assemble_near_rows(self, rows):
        """Assemble and keep the near-field rows of a subset of DOFs (lazy operators)."""
        rows = np.ascontiguousarray(rows, dtype=np.int64)
        _check(lib().orc_h2_near_rows(self._h, _p(rows), rows.size))

    def gmres(self, b, tol: float = 1e-8, restart: int = 30, maxit: int = 2000):
        b = np.ascontiguousarray(b, dtype=self.space.dtype)
        x = np.zeros_like(b)
        st = np.zeros(3)
        _check(lib().orc_h2_gmres(self._h, _p(b), _p(x), tol, restart, maxit, _p(st)))
        return x, int(st[0]), float(st[1]), bool(st[2])


def dense_gmres(A, b, tol: float = 1e-8, restart: int = 30, maxit: int = 2000):
    A = np.ascontiguousarray(A)
    cplx = np.iscomplexobj(A) or np.iscomplexobj(b)
    dt = np.complex128 if cplx else np.float64
    A = np.ascontiguousarray(A, dtype=dt)
    b = np.ascontiguousarray(b, dtype=dt)
    x = np.zeros_like(b)
    st = np.zeros(3)
    _check(lib().orc_dense_gmres(A.shape[0], int(cplx), _p(A), _p(b), _p(x), tol, restart, maxit, _p(st)))
    return x, int(st[0]), float(st[1]), bool(st[2])


class BlockJacobi:
    """Block-Jacobi preconditioner of an H2 oracle operator: tiles of `tile` x `tile`
    B-spline indices per patch, blocks from the near field, LU with partial pivoting."""

    def __init__(self, h2: "H2", tile: int = 8):
        self.h2 = h2
        h = ctypes.c_void_p()
        _check(lib().orc_bj_new(h2._h, tile, ctypes.byref(h)))
        self._h = h.value
        self.ntiles = lib().orc_bj_ntiles(self._h)
        self.dtype = h2.space.dtype

    def __del__(self):
        if getattr(self, "_h", None):
            lib().orc_bj_free(self._h)
            self._h = None

    def tile(self, k: int):
        t5 = np.zeros(5, dtype=np.int32)
        _check(lib().orc_bj_tile(self._h, k, _p(t5), None))
        n = int((t5[2] - t5[1]) * (t5[4] - t5[3]))
        dofs = np.zeros(n, dtype=np.int64)
        _check(lib().orc_bj_tile(self._h, k, _p(t5), _p(dofs)))
        return tuple(int(v) for v in t5), dofs

    def block(self, k: int) -> np.ndarray:
        _, dofs = self.tile(k)
        D = np.zeros((dofs.size, dofs.size), dtype=self.dtype)
        _check(lib().orc_bj_block(self._h, k, _p(D)))
        return D

    def target(self, k: int, ring: int) -> np.ndarray:
        """Block least-squares approximate inverse X_b of tile k on the tile extended by ring."""
        _, dofs = self.tile(k)
        C = np.zeros((dofs.size, dofs.size), dtype=self.dtype)
        _check(lib().orc_bj_target(self._h, k, ring, _p(C)))
        return C

    def apply(self, r) -> np.ndarray:
        r = np.ascontiguousarray(r, dtype=self.dtype)
        z = np.zeros_like(r)
        _check(lib().orc_bj_apply(self._h, _p(r), _p(z)))
        return z

    def gmres(self, b, tol: float = 1e-8, restart: int = 30, maxit: int = 2000):
        """Right-preconditioned GMRES on the H2 operator; returns (x, iterations, relres, converged)."""
        b = np.ascontiguousarray(b, dtype=self.dtype)
        x = np.zeros_like(b)
        st = np.zeros(3)
        _check(lib().orc_h2_gmres_bj(self.h2._h, self._h, _p(b), _p(x), tol, restart, maxit, _p(st)))
        return x, int(st[0]), float(st[1]), bool(st[2])


def tile_features(space: "Space", tile: int = 8) -> np.ndarray:
    """Features of every tile of `tile` x `tile` B-spline indices (ntiles x 99), analytic
    Jacobians of the patch maps (see bem_oracle.cpp, tile_features)."""
    nb = space.degree + 1 + (2 ** space.level - 1) * space.knot_rep
    npatch = {SPHERE: 6, ELLIPSOID: 6, TORUS: 16, FLAT: 1}[space.geom]
    nt = -(-nb // tile)
    out = np.zeros((npatch * nt * nt, 99))
    _check(lib().orc_tile_features(space._h, tile, _p(out)))
    return out


def user_map_patches(fn, npatch: int, degree: int = 5, intervals: int = 8):
    """Reading of a user-supplied patch map (Sec. 4 "Geometry" allows arbitrary smooth
    maps): each patch map is replaced by its tensor B-spline interpolant of `degree` on
    `intervals` (a power of two) uniform intervals per direction, interpolating at the
    Greville abscissae of the clamped knot vector; the result is a set of NURBS patches
    with unit weights.  fn(patch, st) -> xyz for st an (n, 2) array of parameter points.
    The collocation matrices use the oracle's own B-splines (App. C recursion)."""
    L = int(round(np.log2(intervals)))
    if 1 << L != intervals:
        raise ValueError("intervals must be a power of two")
    k = bspline_count(degree, 1, L)
    knots = [0.0] * (degree + 1) + [j / intervals for j in range(1, intervals)] + [1.0] * (degree + 1)
    kn = np.asarray(knots)
    grev = np.array([kn[j + 1:j + degree + 1].mean() for j in range(k)]) if degree > 0 else \
        0.5 * (kn[:k] + kn[1:k + 1])
    B = np.stack([bspline(degree, 1, L, j, grev) for j in range(k)], axis=1)  # B[i, j] = b_j(x_i)
    s1, s2 = np.meshgrid(grev, grev, indexing="ij")
    st = np.stack([s1.ravel(), s2.ravel()], axis=1)
    out = []
    for f in range(npatch):
        F = np.asarray(fn(f, st), dtype=np.float64).reshape(k, k, 3)
        C = np.empty_like(F)
        for d in range(3):  # B C_d B^T = F_d
            C[:, :, d] = np.linalg.solve(B, np.linalg.solve(B, F[:, :, d]).T).T
        cw = np.concatenate([C, np.ones((k, k, 1))], axis=2)
        out.append({"degree": (degree, degree), "knots": (knots, knots), "cw": cw})
    return out


# ---------------------------------------------------------------------------------------
# Maxwell single layer (App. A (MP), App. B (MS)) on the div-conforming spaces S^1 (App. E)
DIPOLE, PLANE_WAVE_E = 0, 1


class MSpace:
    """S^1 = S_p x S_{p-1} (x) S_{p-1} x S_p on every patch, lifted by the Piola transform and
    glued by normal continuity (p >= 1), with the wavenumber of (MS)."""

    def __init__(self, geom: int, gparams=(), kappa: complex = 1.0, p: int = 1, level: int = 0):
        h = ctypes.c_void_p()
        if geom == NURBS:
            meta, knots, cw = [], [], []
            for P in gparams:
                c = np.asarray(P["cw"], dtype=np.float64)
                meta += [int(P["degree"][0]), int(P["degree"][1]), c.shape[0], c.shape[1]]
                knots += [np.asarray(P["knots"][0], dtype=np.float64), np.asarray(P["knots"][1], dtype=np.float64)]
                cw.append(c.reshape(-1))
            m = np.ascontiguousarray(meta, dtype=np.int32)
            kn = np.ascontiguousarray(np.concatenate(knots))
            cc = np.ascontiguousarray(np.concatenate(cw))
            _check(lib().orc_mspace_new_nurbs(len(gparams), m.ctypes.data, _p(kn), _p(cc), float(np.real(kappa)),
                                              float(np.imag(kappa)), p, level, ctypes.byref(h)))
        else:
            gp = np.ascontiguousarray(np.asarray(gparams, dtype=np.float64).reshape(-1))
            if gp.size == 0:
                gp = np.zeros(1)
            _check(lib().orc_mspace_new(geom, _p(gp), int(len(gparams)), float(np.real(kappa)),
                                        float(np.imag(kappa)), p, level, ctypes.byref(h)))
        self._h = h
        self.kappa, self.p, self.level = complex(kappa), p, level
        info = np.zeros(4, dtype=np.int64)
        _check(lib().orc_mspace_info(self._h, _p(info)))
        self.nloc, self.nglob, self.nelem, self.nl = (int(v) for v in info)

    def __del__(self):
        if getattr(self, "_h", None):
            try:
                lib().orc_mspace_free(self._h)
            except Exception:
                pass
            self._h = None

    def glue(self):
        """(local -> global map with -1 for dropped functions, sign of each local function)."""
        g = np.zeros(self.nloc, dtype=np.int64)
        sg = np.zeros(self.nloc, dtype=np.int32)
        _check(lib().orc_mspace_glue(self._h, _p(g), sg.ctypes.data))
        return g, sg

    def elem_eval(self, e: int, s: float, t: float):
        """(point, lifted fields (nl, 3), reference divergences (nl,), local indices (nl,))."""
        x = np.zeros(3)
        V = np.zeros((self.nl, 3))
        D = np.zeros(self.nl)
        lid = np.zeros(self.nl, dtype=np.int64)
        _check(lib().orc_m_elem_eval(self._h, e, s, t, _p(x), _p(V), _p(D), _p(lid)))
        return x, V, D, lid

    def pair_block(self, e1: int, e2: int, qg: int = 8, qs: int = 8, part: int = 0) -> np.ndarray:
        B = np.zeros((self.nl, self.nl), dtype=np.complex128)
        _check(lib().orc_m_pair_block(self._h, e1, e2, qg, qs, part, _p(B)))
        return B

    def dense(self, qg: int = 8, qs: int = 8, part: int = 0) -> np.ndarray:
        """Galerkin matrix on the global functions (row: test, column: trial); part 1: the
        vector term only, 2: the divergence term only."""
        M = np.zeros((self.nglob, self.nglob), dtype=np.complex128)
        _check(lib().orc_m_dense(self._h, qg, qs, part, _p(M)))
        return M

    def h2_dense(self, q: int = 5, eta: float = 1.6, leaf: int = 0, qg: int = 8, qs: int = 8,
                 kappa_adm: float = 0.0, part: int = 0) -> np.ndarray:
        """The Galerkin matrix with the far field of the scalar H^2 partition replaced by the
        Chebyshev interpolation of the kernel on both clusters (four channels)."""
        M = np.zeros((self.nglob, self.nglob), dtype=np.complex128)
        _check(lib().orc_m_h2_dense(self._h, q, float(eta), leaf, qg, qs, float(kappa_adm), part, _p(M)))
        return M

    def rhs(self, kind: int, params, q: int = 8) -> np.ndarray:
        prm = np.ascontiguousarray(np.asarray(params, dtype=np.float64).reshape(-1, 6))
        b = np.zeros((prm.shape[0], self.nglob), dtype=np.complex128)
        _check(lib().orc_m_rhs(self._h, kind, _p(prm), prm.shape[0], q, _p(b)))
        return b[0] if prm.shape[0] == 1 else b

    def potential(self, j, pts, q: int = 8) -> np.ndarray:
        j = np.ascontiguousarray(j, dtype=np.complex128)
        pts = np.ascontiguousarray(pts, dtype=np.float64).reshape(-1, 3)
        E = np.zeros((pts.shape[0], 3), dtype=np.complex128)
        _check(lib().orc_m_potential(self._h, q, _p(j), pts.shape[0], _p(pts), _p(E)))
        return E


def m_field(kind: int, params, kappa: complex, pts) -> np.ndarray:
    """Data fields of (MP): kind DIPOLE (x0, moment) or PLANE_WAVE_E (direction, polarisation)."""
    prm = np.ascontiguousarray(np.asarray(params, dtype=np.float64).reshape(6))
    pts = np.ascontiguousarray(pts, dtype=np.float64).reshape(-1, 3)
    E = np.zeros((pts.shape[0], 3), dtype=np.complex128)
    _check(lib().orc_m_field(kind, _p(prm), float(np.real(kappa)), float(np.imag(kappa)), pts.shape[0], _p(pts),
                             _p(E)))
    return E
