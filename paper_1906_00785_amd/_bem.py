"""ctypes binding of libbem_hip.so (include/bem.h): the same entry points, argument
marshalling only.  Every step of the computation runs in the library's HIP kernels; if the
library is missing this module raises at import, there is no fallback."""
from __future__ import annotations

import ctypes
import os
import re

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libbem_hip.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "bem.h")

BEM_OK, BEM_EINVAL, BEM_ENOMEM, BEM_EDEVICE, BEM_ENOCONV, BEM_EUNSUPPORTED = 0, -1, -2, -3, -4, -5
BEM_LAPLACE_SINGLE, BEM_HELMHOLTZ_SINGLE, BEM_MAXWELL_SINGLE = 0, 1, 2
BEM_GEOM_SPHERE6, BEM_GEOM_ELLIPSOID6, BEM_GEOM_TORUS16, BEM_GEOM_FLAT1, BEM_GEOM_NURBS = 0, 1, 2, 3, 4
BEM_SPACE_S2, BEM_SPACE_S0, BEM_SPACE_S1 = 2, 0, 1
BEM_DATA_POINT_SOURCE, BEM_DATA_PLANE_WAVE, BEM_DATA_DIPOLE, BEM_DATA_PLANE_WAVE_E = 0, 1, 2, 3
BEM_PREC_FP64, BEM_PREC_FP32, BEM_PREC_BF16 = 0, 1, 2
BEM_PRECOND_NONE, BEM_PRECOND_BLOCK = 0, 1

_c_int, _c_dbl, _c_i64, _c_sz, _vp = ctypes.c_int, ctypes.c_double, ctypes.c_int64, ctypes.c_size_t, ctypes.c_void_p


class bem_h2_params(ctypes.Structure):
    _fields_ = [("q", _c_int), ("eta", _c_dbl), ("leaf_level", _c_int), ("qg", _c_int), ("qs", _c_int),
                ("chunk_cols", _c_int), ("far_low", _c_int), ("batch_rhs", _c_int),
                ("far_eval", _c_int), ("kappa_adm", _c_dbl)]


class bem_operator_info(ctypes.Structure):
    _fields_ = [("ndof", _c_i64), ("nclusters", _c_i64), ("nfar", _c_i64), ("nnear", _c_i64), ("ntouch", _c_i64),
                ("near_nnz", _c_i64), ("leaf_level", _c_i64), ("op_bytes", _c_sz), ("tmp_bytes", _c_sz),
                ("far_bytes", _c_dbl), ("near_bytes", _c_dbl), ("nstored", _c_i64), ("nchunks", _c_i64),
                ("transposed_bytes", _c_dbl), ("nlocal", _c_i64)]


class bem_solve_params(ctypes.Structure):
    _fields_ = [("restart", _c_int), ("maxit", _c_int), ("tol", _c_dbl), ("refine", _c_int), ("max_outer", _c_int),
                ("inner_tol", _c_dbl), ("precond", _c_int), ("inner_maxit", _c_int),
                ("reserved", _c_int * 2)]


class bem_solve_stats(ctypes.Structure):
    _fields_ = [("iterations", _c_int), ("converged", _c_int), ("relres", _c_dbl), ("outer", _c_int),
                ("reserved", _c_int)]


class BemError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"bem error {code}: {msg}")
        self.code = code


_P = ctypes.POINTER
_SIGNATURES = {
    "bem_last_error": (ctypes.c_char_p, []),
    "bem_geometry_analytic": (_c_int, [_c_int, _P(_c_dbl), _c_int, _P(_vp)]),
    "bem_geometry_destroy": (None, [_vp]),
    "bem_geometry_nurbs": (_c_int, [_c_int, _vp, _vp, _vp, _P(_vp)]),
    "bem_write_vtk": (_c_int, [_vp, _vp, _c_i64, _c_int, _c_int, ctypes.c_char_p]),
    "bem_eval_potential_h2": (_c_int, [_vp, _vp, _c_i64, _vp, _c_i64, _c_int, _vp, _c_i64, _c_dbl, _vp]),
    "bem_geometry_load": (_c_int, [ctypes.c_char_p, _P(_vp)]),
    "bem_geometry_save": (_c_int, [_vp, ctypes.c_char_p]),
    "bem_geometry_user": (_c_int, [_c_int, _vp, _vp, _c_int, _c_int, _P(_vp)]),
    "bem_space_create": (_c_int, [_vp, _c_int, _c_dbl, _c_dbl, _c_int, _c_int, _c_int, _P(_vp)]),
    "bem_space_create_ex": (_c_int, [_vp, _c_int, _c_dbl, _c_dbl, _c_int, _c_int, _c_int, _c_int, _P(_vp)]),
    "bem_space_glue": (_c_int, [_vp, _P(_c_i64), _vp]),
    "bem_space_glue_sign": (_c_int, [_vp, _vp]),
    "bem_space_ndof": (_c_int, [_vp, _P(_c_i64)]),
    "bem_space_destroy": (None, [_vp]),
    "bem_rhs": (_c_int, [_vp, _c_int, _P(_c_dbl), _c_int, _vp, _c_i64, _vp]),
    "bem_rhs_quadpoints": (_c_int, [_vp, _vp, _P(_c_i64), _vp]),
    "bem_rhs_from_samples": (_c_int, [_vp, _vp, _c_i64, _c_int, _vp, _c_i64, _vp]),
    "bem_assemble_plan": (_c_int, [_vp, _P(bem_h2_params), _P(_vp), _P(bem_operator_info)]),
    "bem_assemble": (_c_int, [_vp, _vp, _c_sz, _vp, _c_sz, _vp]),
    "bem_operator_info_get": (_c_int, [_vp, _P(bem_operator_info)]),
    "bem_operator_dims": (_c_int, [_vp, _P(_c_i64), _P(_c_i64)]),
    "bem_apply": (_c_int, [_vp, _vp, _c_i64, _vp, _c_i64, _c_int, _vp]),
    "bem_apply_ex": (_c_int, [_vp, _c_int, _vp, _c_i64, _vp, _c_i64, _c_int, _vp]),
    "bem_solve_plan": (_c_int, [_vp, _c_int, _P(bem_solve_params), _P(_c_sz)]),
    "bem_solve": (_c_int, [_vp, _vp, _c_i64, _vp, _c_i64, _c_int, _P(bem_solve_params), _P(bem_solve_stats), _vp,
                           _c_sz, _vp]),
    "bem_eval_potential": (_c_int, [_vp, _vp, _c_i64, _vp, _c_i64, _c_int, _vp, _c_i64, _vp]),
    "bem_operator_destroy": (None, [_vp]),
    "bem_profile_enable": (_c_int, [_vp, _c_int]),
    "bem_profile_read": (_c_int, [_vp, _P(_c_dbl), _c_int, _P(_c_int)]),
    "bem_apply_stage": (_c_int, [_vp, _c_int, _c_int, _vp, _vp, _vp]),
    "bem_export_near": (_c_int, [_vp, _vp, _vp, _vp, _vp]),
    "bem_export_far": (_c_int, [_vp, _vp, _vp, _vp]),
    "bem_export_moments": (_c_int, [_vp, _vp, _vp, _vp]),
    "bem_precond_info": (_c_int, [_vp, _P(_c_i64), _P(_c_sz)]),
    "bem_precond_build": (_c_int, [_vp, _vp, _c_sz, _vp]),
    "bem_precond_apply": (_c_int, [_vp, _vp, _c_i64, _vp, _c_i64, _c_int, _vp]),
    "bem_precond_export": (_c_int, [_vp, _c_int, _vp, _vp]),
    "bem_precond_features": (_c_int, [_vp, _vp, _vp]),
    "bem_precond_target_bytes": (_c_int, [_vp, _c_int, _c_i64, _P(_c_sz)]),
    "bem_precond_targets": (_c_int, [_vp, _c_int, _c_i64, _c_i64, _vp, _c_sz, _vp, _vp]),
    "bem_precond_correct": (_c_int, [_vp, _vp, _c_int, _c_int, _vp, _vp]),
    "bem_precond_select": (_c_int, [_vp, _vp, _vp, _c_int, _vp, _c_sz, _P(_c_int), _P(_c_dbl), _vp]),
    "bem_group_create": (_c_int, [_c_int, _P(_vp), _P(_c_int), _P(_vp), _P(_c_sz)]),
    "bem_group_bind": (_c_int, [_vp, _vp, _c_sz, _P(_vp), _P(_vp), _vp]),
    "bem_group_apply": (_c_int, [_vp, _vp]),
    "bem_group_destroy": (None, [_vp]),
    "bem_capture_begin": (_c_int, [_vp]),
    "bem_capture_end": (_c_int, [_vp, _P(_vp)]),
    "bem_graph_launch": (_c_int, [_vp, _vp]),
    "bem_graph_destroy": (None, [_vp]),
    "bem_mlp_sizes": (_c_int, [_c_int, _c_int, _c_int, _c_int, _P(_c_i64), _P(_c_sz)]),
    "bem_mlp_init": (_c_int, [_c_int, _c_int, _c_int, ctypes.c_uint64, _vp, _vp]),
    "bem_mlp_forward": (_c_int, [_c_int, _c_int, _c_int, _c_int, _vp, _vp, _vp, _c_int, _vp, _c_sz, _vp]),
    "bem_mlp_forward_noalloc": (_c_int, [_c_int, _c_int, _c_int, _c_int, _vp, _vp, _vp, _c_int, _vp]),
    "bem_mlp_loss_grad": (_c_int, [_c_int, _c_int, _c_int, _c_int, _c_int, _vp, _vp, _vp, _vp, _vp, _c_int, _vp, _c_sz,
                                   _vp]),
    "bem_mlp_adam": (_c_int, [_c_i64, _vp, _vp, _vp, _vp, _c_int, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                              ctypes.c_float, _vp]),
}


def header_symbols() -> list[str]:
    """Names of the functions declared in include/bem.h."""
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(bem_[a-z0-9_]+)\s*\(", txt)))


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build() (hipcc for gfx950)")
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in _SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


lib = _load()


def check(rc: int):
    if rc != BEM_OK:
        raise BemError(rc, lib.bem_last_error().decode())


def _dbl_array(vals):
    vals = [float(v) for v in vals]
    return (ctypes.c_double * max(1, len(vals)))(*vals)


# ----------------------------------------------------------------------------- entry points
def bem_geometry_analytic(kind: int, params=()) -> int:
    h = _vp()
    check(lib.bem_geometry_analytic(kind, _dbl_array(params), len(params), ctypes.byref(h)))
    return h.value


def bem_geometry_nurbs(patches) -> int:
    """patches: list of {"degree": (p1, p2), "knots": (Xi_1, Xi_2), "cw": array (k1, k2, 4)}."""
    import numpy as np

    meta, knots, cw = [], [], []
    for P in patches:
        c = np.asarray(P["cw"], dtype=np.float64)
        meta += [int(P["degree"][0]), int(P["degree"][1]), c.shape[0], c.shape[1]]
        knots += [float(v) for v in P["knots"][0]] + [float(v) for v in P["knots"][1]]
        cw.append(c.reshape(-1))
    m = np.ascontiguousarray(meta, dtype=np.int32)
    kn = np.ascontiguousarray(knots, dtype=np.float64)
    cc = np.ascontiguousarray(np.concatenate(cw))
    h = _vp()
    check(lib.bem_geometry_nurbs(len(patches), m.ctypes.data, kn.ctypes.data, cc.ctypes.data, ctypes.byref(h)))
    return h.value


def bem_geometry_load(path: str) -> int:
    h = _vp()
    check(lib.bem_geometry_load(os.fsencode(path), ctypes.byref(h)))
    return h.value


def bem_geometry_save(g: int, path: str):
    check(lib.bem_geometry_save(g, os.fsencode(path)))


USER_MAP = ctypes.CFUNCTYPE(None, _c_int, _P(_c_dbl), _c_i64, _P(_c_dbl), _P(_c_dbl), _vp)


def bem_geometry_user(npatch: int, fn, degree: int, intervals: int) -> int:
    """fn(patch, st) -> xyz for an (n, 2) numpy array of parameter points (host callback;
    called during this call only)."""
    import numpy as np

    err = []

    def cb(patch, st, n, xyz, jac, user):
        try:
            pts = np.ctypeslib.as_array(st, shape=(n, 2)).copy()
            out = np.ctypeslib.as_array(xyz, shape=(n, 3))
            out[:] = np.asarray(fn(patch, pts), dtype=np.float64).reshape(n, 3)
        except Exception as e:  # leave NaN in xyz: the library reports it
            err.append(e)

    h = _vp()
    c = USER_MAP(cb)
    rc = lib.bem_geometry_user(npatch, ctypes.cast(c, _vp), None, degree, intervals, ctypes.byref(h))
    if err:
        raise err[0]
    check(rc)
    return h.value


def bem_geometry_destroy(g: int):
    lib.bem_geometry_destroy(g)


def bem_space_create(g: int, kernel: int, kappa: complex, degree: int, knot_repetition: int, level: int,
                     space_kind: int = BEM_SPACE_S2) -> int:
    h = _vp()
    kappa = complex(kappa)
    check(lib.bem_space_create_ex(g, kernel, kappa.real, kappa.imag, degree, knot_repetition, level, space_kind,
                                  ctypes.byref(h)))
    return h.value


def bem_space_glue(s: int):
    """(number of local functions, int32 array of their global functions)."""
    import numpy as np

    n = _c_i64()
    check(lib.bem_space_glue(s, ctypes.byref(n), None))
    m = np.zeros(n.value, dtype=np.int32)
    check(lib.bem_space_glue(s, ctypes.byref(n), m.ctypes.data))
    return n.value, m


def bem_space_glue_sign(s: int):
    """int32 array: sign of every local function in its global function."""
    import numpy as np

    n = _c_i64()
    check(lib.bem_space_glue(s, ctypes.byref(n), None))
    m = np.zeros(n.value, dtype=np.int32)
    check(lib.bem_space_glue_sign(s, m.ctypes.data))
    return m


def bem_space_ndof(s: int) -> int:
    n = _c_i64()
    check(lib.bem_space_ndof(s, ctypes.byref(n)))
    return n.value


def bem_space_destroy(s: int):
    lib.bem_space_destroy(s)


def bem_rhs(s: int, data_kind: int, data_params, nrhs: int, b_ptr: int, ldb: int, stream: int):
    flat = [float(v) for row in data_params for v in row]
    check(lib.bem_rhs(s, data_kind, _dbl_array(flat), nrhs, b_ptr, ldb, stream))


def bem_rhs_quadpoints(s: int, xyz_ptr, stream: int) -> int:
    n = ctypes.c_int64()
    check(lib.bem_rhs_quadpoints(s, xyz_ptr, ctypes.byref(n), stream))
    return n.value


def bem_rhs_from_samples(s: int, g_ptr: int, ldg: int, nrhs: int, b_ptr: int, ldb: int, stream: int):
    check(lib.bem_rhs_from_samples(s, g_ptr, ldg, nrhs, b_ptr, ldb, stream))


def bem_assemble_plan(s: int, q: int, eta: float, leaf_level: int, qg: int, qs: int, chunk_cols: int = 0,
                      far_low: int = 0, batch_rhs: int = 0, far_eval: int = 0, kappa_adm: float = 0.0):
    p = bem_h2_params(q, eta, leaf_level, qg, qs, chunk_cols, far_low, batch_rhs, far_eval, kappa_adm)
    h = _vp()
    info = bem_operator_info()
    check(lib.bem_assemble_plan(s, ctypes.byref(p), ctypes.byref(h), ctypes.byref(info)))
    return h.value, info


def bem_assemble(A: int, op_ptr: int, op_bytes: int, tmp_ptr: int, tmp_bytes: int, stream: int):
    check(lib.bem_assemble(A, op_ptr, op_bytes, tmp_ptr, tmp_bytes, stream))


def bem_operator_info_get(A: int) -> bem_operator_info:
    info = bem_operator_info()
    check(lib.bem_operator_info_get(A, ctypes.byref(info)))
    return info


def bem_operator_dims(A: int):
    r, c = _c_i64(), _c_i64()
    check(lib.bem_operator_dims(A, ctypes.byref(r), ctypes.byref(c)))
    return r.value, c.value


def bem_apply(A: int, x_ptr: int, ldx: int, y_ptr: int, ldy: int, nrhs: int, stream: int):
    check(lib.bem_apply(A, x_ptr, ldx, y_ptr, ldy, nrhs, stream))


def _solve_params(restart, maxit, tol, refine=0, max_outer=0, inner_tol=0.0, precond=0, inner_maxit=0):
    return bem_solve_params(restart, maxit, tol, int(refine), max_outer, inner_tol, int(precond), int(inner_maxit),
                            (_c_int * 2)(0, 0))


def bem_apply_ex(A: int, prec: int, x_ptr: int, ldx: int, y_ptr: int, ldy: int, nrhs: int, stream: int):
    check(lib.bem_apply_ex(A, prec, x_ptr, ldx, y_ptr, ldy, nrhs, stream))


def bem_solve_plan(A: int, nrhs: int, restart: int, maxit: int, tol: float, refine: int = 0,
                   max_outer: int = 0) -> int:
    p = _solve_params(restart, maxit, tol, refine, max_outer)
    n = _c_sz()
    check(lib.bem_solve_plan(A, nrhs, ctypes.byref(p), ctypes.byref(n)))
    return n.value


def bem_solve(A: int, b_ptr: int, ldb: int, x_ptr: int, ldx: int, nrhs: int, restart: int, maxit: int, tol: float,
              ws_ptr: int, ws_bytes: int, stream: int, refine: int = 0, max_outer: int = 0, inner_tol: float = 0.0,
              precond: int = 0, inner_maxit: int = 0):
    """Returns (rc, stats list); rc is BEM_OK or BEM_ENOCONV (other codes raise)."""
    p = _solve_params(restart, maxit, tol, refine, max_outer, inner_tol, precond, inner_maxit)
    st = (bem_solve_stats * nrhs)()
    rc = lib.bem_solve(A, b_ptr, ldb, x_ptr, ldx, nrhs, ctypes.byref(p), st, ws_ptr, ws_bytes, stream)
    if rc not in (BEM_OK, BEM_ENOCONV):
        check(rc)
    return rc, [(s.iterations, bool(s.converged), s.relres, s.outer) for s in st]


def bem_write_vtk(s: int, rho_host_ptr, ldr: int, nrhs: int, nsub: int, path: str):
    check(lib.bem_write_vtk(s, rho_host_ptr, ldr, nrhs, nsub, os.fsencode(path)))


def bem_eval_potential_h2(A: int, pts_ptr: int, npts: int, rho_ptr: int, ldr: int, nrhs: int, u_ptr: int, ldu: int,
                          eta: float, stream: int):
    check(lib.bem_eval_potential_h2(A, pts_ptr, npts, rho_ptr, ldr, nrhs, u_ptr, ldu, eta, stream))


def bem_eval_potential(s: int, pts_ptr: int, npts: int, rho_ptr: int, ldr: int, nrhs: int, u_ptr: int, ldu: int,
                       stream: int):
    check(lib.bem_eval_potential(s, pts_ptr, npts, rho_ptr, ldr, nrhs, u_ptr, ldu, stream))


def bem_operator_destroy(A: int):
    lib.bem_operator_destroy(A)


def bem_profile_enable(A: int, on: bool):
    check(lib.bem_profile_enable(A, int(bool(on))))


def bem_profile_read(A: int):
    """Mean milliseconds of the 4 apply stages and the number of recorded applies."""
    ms = (ctypes.c_double * 4)()
    n = _c_int()
    check(lib.bem_profile_read(A, ms, 4, ctypes.byref(n)))
    return list(ms), n.value


def bem_apply_stage(A: int, prec: int, stage: int, x_ptr: int, y_ptr: int, stream: int):
    check(lib.bem_apply_stage(A, prec, stage, x_ptr, y_ptr, stream))


def bem_export_near(A: int, rowptr_ptr: int, col_ptr: int, val_ptr: int, stream: int):
    check(lib.bem_export_near(A, rowptr_ptr, col_ptr, val_ptr, stream))


def bem_export_far(A: int, pairs_ptr: int, blocks_ptr: int, stream: int):
    check(lib.bem_export_far(A, pairs_ptr, blocks_ptr, stream))


def bem_export_moments(A: int, x_ptr: int, mom_ptr: int, stream: int):
    check(lib.bem_export_moments(A, x_ptr, mom_ptr, stream))


def bem_precond_info(A: int):
    n, b = _c_i64(), _c_sz()
    check(lib.bem_precond_info(A, ctypes.byref(n), ctypes.byref(b)))
    return n.value, b.value


def bem_precond_build(A: int, ws_ptr: int, ws_bytes: int, stream: int):
    check(lib.bem_precond_build(A, ws_ptr, ws_bytes, stream))


def bem_precond_apply(A: int, r_ptr: int, ldr: int, z_ptr: int, ldz: int, nrhs: int, stream: int):
    check(lib.bem_precond_apply(A, r_ptr, ldr, z_ptr, ldz, nrhs, stream))


def bem_precond_export(A: int, which: int, out_ptr: int, stream: int):
    check(lib.bem_precond_export(A, which, out_ptr, stream))


def bem_precond_features(A: int, feats_ptr: int, stream: int):
    check(lib.bem_precond_features(A, feats_ptr, stream))


def bem_precond_target_bytes(A: int, ring: int, nt: int) -> int:
    b = _c_sz()
    check(lib.bem_precond_target_bytes(A, ring, nt, ctypes.byref(b)))
    return b.value


def bem_precond_targets(A: int, ring: int, t0: int, nt: int, work_ptr: int, work_bytes: int, delta_ptr: int,
                        stream: int):
    check(lib.bem_precond_targets(A, ring, t0, nt, work_ptr, work_bytes, delta_ptr, stream))


def bem_precond_correct(A: int, uv_ptr, mode: int, ring: int, accepted_ptr, stream: int):
    check(lib.bem_precond_correct(A, uv_ptr, mode, ring, accepted_ptr, stream))


def bem_precond_select(A: int, uv_ptr: int, b_ptr: int, restart: int, ws_ptr: int, ws_bytes: int, stream: int):
    kept = _c_int()
    rr = (_c_dbl * 2)()
    check(lib.bem_precond_select(A, uv_ptr, b_ptr, restart, ws_ptr, ws_bytes, ctypes.byref(kept), rr, stream))
    return bool(kept.value), (rr[0], rr[1])


def bem_mlp_sizes(n_in: int, hidden: int, out: int, batch: int):
    n, b = _c_i64(), _c_sz()
    check(lib.bem_mlp_sizes(n_in, hidden, out, batch, ctypes.byref(n), ctypes.byref(b)))
    return n.value, b.value


def bem_mlp_init(n_in: int, hidden: int, out: int, seed: int, params_ptr: int, stream: int):
    check(lib.bem_mlp_init(n_in, hidden, out, seed, params_ptr, stream))


def bem_mlp_forward(n_in, hidden, out, batch, params_ptr, x_ptr, y_ptr, precision, ws_ptr, ws_bytes, stream):
    check(lib.bem_mlp_forward(n_in, hidden, out, batch, params_ptr, x_ptr, y_ptr, precision, ws_ptr, ws_bytes, stream))


def bem_mlp_forward_noalloc(n_in, hidden, out, batch, params_ptr, x_ptr, y_ptr, precision, stream):
    check(lib.bem_mlp_forward_noalloc(n_in, hidden, out, batch, params_ptr, x_ptr, y_ptr, precision, stream))


def bem_mlp_loss_grad(n_in, hidden, out, batch, is_complex, params_ptr, x_ptr, t_ptr, grad_ptr, loss_ptr, precision,
                      ws_ptr, ws_bytes, stream):
    check(lib.bem_mlp_loss_grad(n_in, hidden, out, batch, is_complex, params_ptr, x_ptr, t_ptr, grad_ptr, loss_ptr,
                                precision, ws_ptr, ws_bytes, stream))


def bem_mlp_adam(n, params_ptr, grad_ptr, m_ptr, v_ptr, step, lr, beta1, beta2, eps, stream):
    check(lib.bem_mlp_adam(n, params_ptr, grad_ptr, m_ptr, v_ptr, step, lr, beta1, beta2, eps, stream))


def bem_group_create(ops, ncols):
    n = len(ops)
    h = _vp()
    b = _c_sz()
    check(lib.bem_group_create(n, (_vp * n)(*ops), (_c_int * n)(*ncols), ctypes.byref(h), ctypes.byref(b)))
    return h.value, b.value


def bem_group_bind(G: int, ws_ptr: int, ws_bytes: int, x_ptrs, y_ptrs, stream: int):
    n = len(x_ptrs)
    check(lib.bem_group_bind(G, ws_ptr, ws_bytes, (_vp * n)(*x_ptrs), (_vp * n)(*y_ptrs), stream))


def bem_group_apply(G: int, stream: int):
    check(lib.bem_group_apply(G, stream))


def bem_group_destroy(G: int):
    lib.bem_group_destroy(G)


def bem_capture_begin(stream: int):
    check(lib.bem_capture_begin(stream))


def bem_capture_end(stream: int) -> int:
    g = _vp()
    check(lib.bem_capture_end(stream, ctypes.byref(g)))
    return g.value


def bem_graph_launch(g: int, stream: int):
    check(lib.bem_graph_launch(g, stream))


def bem_graph_destroy(g: int):
    lib.bem_graph_destroy(g)
