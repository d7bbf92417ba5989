"""GPU: NURBS patch geometries (App. C), file import and user-supplied maps, against the
oracle on the same patch data.

Bar: FP64 near-field values, load vectors, potentials and H^2 products within 1e-11
(max-norm, relative to the largest oracle entry); near patterns exact.  A NURBS patch
whose map is the identity gives the flat square's operator (1e-14); a saved and reloaded
geometry gives a bitwise-equal product; the user map's interpolant agrees with the oracle's
reading of the same map (1e-11) and with the analytic sphere to the interpolation error.
"""
import math

import numpy as np
import pytest
import torch

import workloads as W

pytestmark = pytest.mark.gpu

TOL = 1e-11


@pytest.fixture(scope="module")
def B():
    import paper_1906_00785_amd as B

    return B


def relerr(a, b):
    return float(np.max(np.abs(np.asarray(a) - np.asarray(b))) / max(np.max(np.abs(b)), 1e-300))


CASES = {
    # id: (patches, pde, kappa, L, d, q, leaf)
    "torus_laplace_d1": (lambda: W.nurbs_torus(1.0, 0.4), 0, 0.0, 2, 1, 4, 1),
    "torus_helmholtz_d2": (lambda: W.nurbs_torus(1.0, 0.3), 1, 2.5, 2, 2, 4, 1),
    "flat_laplace_d2": (lambda: W.nurbs_flat(1.5), 0, 0.0, 2, 2, 3, 1),
}
_cache = {}


def case(B, orc, cid):
    if cid not in _cache:
        mk, pde, kappa, L, d, q, leaf = CASES[cid]
        print(f"[nurbs {cid}] assemble on GPU and in the oracle", flush=True)
        patches = mk()
        g = B.Geometry.nurbs(patches)
        s = B.Space(g, pde, kappa, degree=d, level=L)
        A = B.Operator(s, q=q, eta=1.6, leaf_level=leaf)
        So = orc.Space(orc.NURBS, patches, pde, kappa, degree=d, level=L)
        Ho = orc.H2(So, q=q, eta=1.6, leaf=leaf)
        _cache[cid] = (patches, g, s, A, So, Ho)
    return _cache[cid]


@pytest.mark.parametrize("cid", list(CASES))
def test_near_field_and_apply(B, orc, cid):
    patches, g, s, A, So, Ho = case(B, orc, cid)
    rowptr, col, val = A.export_near()
    rp, cl, vo = Ho.near_csr()
    assert np.array_equal(rowptr, rp) and np.array_equal(col, cl)
    assert relerr(val, vo) <= TOL
    x = W.random_vector(W.rng(9, 20), s.ndof, is_complex=So.complex)
    y = A.apply(torch.from_numpy(x).cuda()).cpu().numpy()
    assert relerr(y, Ho.apply(x)) <= TOL


@pytest.mark.parametrize("cid", ["torus_laplace_d1", "torus_helmholtz_d2"])
def test_rhs_and_potential(B, orc, cid):
    patches, g, s, A, So, Ho = case(B, orc, cid)
    x0 = (0.9, 0.3, 0.05)
    b = s.rhs(B.BEM_DATA_POINT_SOURCE, [x0]).cpu().numpy()[0]
    assert relerr(b, So.rhs(orc.POINT_SOURCE, x0)) <= TOL
    rho = W.random_vector(W.rng(9, 21), s.ndof, is_complex=So.complex)
    pts = W.exterior_points(W.rng(9, 22), 32, 2.0, 4.0)
    u = s.potential(pts, torch.from_numpy(rho).cuda()).cpu().numpy()
    assert relerr(u, So.potential(rho, pts)) <= TOL


def test_exterior_dirichlet_on_nurbs_torus(B, orc):
    """Solved on the GPU (H^2, GMRES to 1e-12), the potential reproduces 1/(4 pi |x - x0|)
    and agrees with the oracle's solution of the same system."""
    patches, g, s, A, So, Ho = case(B, orc, "torus_laplace_d1")
    x0 = np.array([0.9, 0.3, 0.05])
    b = s.rhs(B.BEM_DATA_POINT_SOURCE, [tuple(x0)])
    rho, st = A.solve(b, tol=1e-12)
    assert st[0][1]
    pts = W.exterior_points(W.rng(9, 4), 24, 2.0, 4.0)
    u = s.potential(pts, rho[0]).cpu().numpy()
    ex = 1.0 / (4 * math.pi * np.linalg.norm(pts - x0, axis=1))
    assert np.max(np.abs(u - ex)) / np.max(np.abs(ex)) < 1e-4
    xo, _, _, ok = Ho.gmres(So.rhs(orc.POINT_SOURCE, tuple(x0)), tol=1e-12)
    assert ok and np.linalg.norm(rho.cpu().numpy()[0] - xo) / np.linalg.norm(xo) <= 1e-8


def test_identity_patch_equals_flat_square(B):
    gn = B.Geometry.nurbs(W.nurbs_flat(1.5))
    gf = B.Geometry(B.BEM_GEOM_FLAT1, (1.5,))
    vals = []
    for g in (gn, gf):
        s = B.Space(g, B.BEM_LAPLACE_SINGLE, 0.0, degree=2, level=2)
        vals.append(B.Operator(s, q=3, eta=1.6, leaf_level=1).export_near()[2])
    assert relerr(vals[0], vals[1]) <= 1e-14


def test_file_round_trip_is_bitwise(B, tmp_path):
    g = B.Geometry.nurbs(W.nurbs_torus(1.0, 0.4))
    path = str(tmp_path / "torus.bemnurbs")
    g.save(path)
    ys = []
    for gg in (g, B.Geometry.load(path)):
        s = B.Space(gg, B.BEM_HELMHOLTZ_SINGLE, 3.0, degree=1, level=2)
        A = B.Operator(s, q=4, eta=1.6, leaf_level=1)
        x = torch.from_numpy(W.random_vector(W.rng(9, 23), s.ndof, is_complex=True)).cuda()
        ys.append(A.apply(x))
    assert torch.equal(ys[0], ys[1])


def test_user_map_matches_oracle_and_sphere(B, orc):
    """The sphere's patch maps passed as a host callback: the library's interpolant
    (degree 5, 8 intervals) gives the oracle's operator for the same reading, and the
    analytic sphere's operator to the interpolation error (measured 2e-5 on the dense
    operator)."""
    L, d = 3, 2
    g = B.Geometry.user(6, W.sphere6_map, degree=5, intervals=8)
    s = B.Space(g, B.BEM_LAPLACE_SINGLE, 0.0, degree=d, level=L)
    A = B.Operator(s, q=5, eta=1.6, leaf_level=1)
    So = orc.Space(orc.NURBS, orc.user_map_patches(W.sphere6_map, 6, 5, 8), orc.LAPLACE, 0.0, degree=d, level=L)
    Ho = orc.H2(So, q=5, eta=1.6, leaf=1, assemble_near=False)
    x = W.random_vector(W.rng(9, 24), s.ndof)
    y = A.apply(torch.from_numpy(x).cuda()).cpu().numpy()
    rows = W.sample_rows(9, s.ndof, 8)
    Ho.assemble_near_rows(rows)
    assert relerr(y[rows], Ho.apply_rows(x, rows)) <= TOL
    ga = B.Geometry(B.BEM_GEOM_SPHERE6)
    sa = B.Space(ga, B.BEM_LAPLACE_SINGLE, 0.0, degree=d, level=L)
    ya = B.Operator(sa, q=5, eta=1.6, leaf_level=1).apply(torch.from_numpy(x).cuda()).cpu().numpy()
    assert relerr(y, ya) <= 1e-4
