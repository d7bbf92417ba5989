"""GPU parity of the continuous spaces S^0 (App. E: 0-form lifting, continuity across patch
boundaries) against the oracle's S^0 spaces, which are pinned on the CPU.

The HIP path works on the global (glued) functions; the oracle works on the local ones and
its global quantities are composed here with the 0/1 gluing matrix P (P[k, m[k]] = 1):
matrix P^T A P, load vector P^T b, density P rho.  Bar: the gluing map exactly; FP64 results
within 1e-11 (max-norm relative, element by element) of the oracle's; the solution of the
exterior Dirichlet problem within 1e-8 of the oracle's solution of the same H^2 system.
"""
import math

import numpy as np
import pytest
import torch

import workloads as W

pytestmark = pytest.mark.gpu

TOL = 1e-11

CASES = {
    # id: (geometry maker, oracle geometry, pde, kappa, L, d, q, eta, leaf)
    "sphere_L2_d1_laplace_h2": (lambda B: B.Geometry(B.BEM_GEOM_SPHERE6), (0, []), 0, 0.0, 2, 1, 4, 1.6, 1),
    "ellipsoid_L2_d1_laplace_dense": (lambda B: B.Geometry(B.BEM_GEOM_ELLIPSOID6, (0.8, 1.1, 1.3)),
                                      (1, [0.8, 1.1, 1.3]), 0, 0.0, 2, 1, 3, 0.0, 0),
    "torus_L2_d2_helmholtz_h2": (lambda B: B.Geometry(B.BEM_GEOM_TORUS16, (1.0, 0.4)), (2, [1.0, 0.4]), 1, 2.0, 2,
                                 2, 4, 1.6, 1),
    "ellipsoid_L1_d2_helmholtz_cplx_h2": (lambda B: B.Geometry(B.BEM_GEOM_ELLIPSOID6, (0.7, 1.2, 1.6)),
                                          (1, [0.7, 1.2, 1.6]), 1, 1.5 + 0.3j, 1, 2, 3, 1.6, 1),
    "nurbs_torus_L1_d2_laplace_h2": (lambda B: B.Geometry.nurbs(W.nurbs_torus(1.0, 0.4)),
                                     (4, W.nurbs_torus(1.0, 0.4)), 0, 0.0, 1, 2, 4, 1.6, 1),
    "flat_L2_d1_laplace_h2": (lambda B: B.Geometry(B.BEM_GEOM_FLAT1, (1.7,)), (3, [1.7]), 0, 0.0, 2, 1, 3, 1.6, 1),
}


@pytest.fixture(scope="module")
def B():
    import paper_1906_00785_amd as B

    assert torch.cuda.is_available()
    return B


def relerr(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def gluing(m, n):
    P = np.zeros((len(m), n))
    P[np.arange(len(m)), m] = 1.0
    return P


_cache = {}


def case(B, orc, cid):
    if cid not in _cache:
        mk, (og, oprm), pde, kappa, L, d, q, eta, leaf = CASES[cid]
        print(f"[s0 case {cid}] assemble on GPU and in the oracle", flush=True)
        s = B.Space(mk(B), pde, kappa, degree=d, level=L, continuous=True)
        A = B.Operator(s, q=q, eta=eta, leaf_level=leaf)
        So = orc.Space(og, oprm, pde, kappa, degree=d, level=L, form=0)
        Ho = orc.H2(So, q=q, eta=eta, leaf=leaf)
        m, n = So.glue()
        _cache[cid] = (s, A, So, Ho, gluing(m, n))
    return _cache[cid]


@pytest.mark.parametrize("cid", list(CASES))
def test_gluing_matches_oracle(B, orc, cid):
    s, A, So, Ho, P = case(B, orc, cid)
    m, n = So.glue()
    assert s.ndof == n == A.ndof and A.info.nlocal == So.ndof
    assert np.array_equal(s.glue(), m.astype(np.int32))


@pytest.mark.parametrize("cid", list(CASES))
def test_near_field_on_local_functions(B, orc, cid):
    s, A, So, Ho, P = case(B, orc, cid)
    rowptr, col, val = A.export_near()
    rp, cl, vo = Ho.near_csr()
    assert np.array_equal(rowptr, rp) and np.array_equal(col, cl)
    assert relerr(val, vo) <= TOL


@pytest.mark.parametrize("cid", list(CASES))
def test_apply_is_glued_product(B, orc, cid):
    s, A, So, Ho, P = case(B, orc, cid)
    x = W.random_vector(W.rng(9, 70), s.ndof, is_complex=So.complex, ncols=2).T.copy()
    y = A.apply(torch.from_numpy(x).cuda()).cpu().numpy()
    for r in range(2):
        yo = P.T @ Ho.apply(P @ x[r])
        assert relerr(y[r], yo) <= TOL, r


def test_dense_mode_is_glued_galerkin_matrix(B, orc):
    """eta = 0: P^T A P for the dense 0-form Galerkin matrix, and symmetric."""
    s, A, So, Ho, P = case(B, orc, "ellipsoid_L2_d1_laplace_dense")
    N = s.ndof
    Ag = A.apply(torch.eye(N, dtype=torch.float64, device="cuda")).cpu().numpy().T
    Ad = P.T @ So.dense(8, 8) @ P
    assert relerr(Ag, Ad) <= TOL
    assert np.abs(Ag - Ag.T).max() <= 1e-13 * np.abs(Ag).max()


@pytest.mark.parametrize("cid", list(CASES))
def test_load_vector_and_moments(B, orc, cid):
    s, A, So, Ho, P = case(B, orc, cid)
    x0 = (0.05, -0.1, 0.08) if "flat" not in cid else (0.3, 0.2, 0.9)
    b = s.rhs(B.BEM_DATA_POINT_SOURCE, [x0]).cpu().numpy().reshape(-1)
    assert relerr(b, P.T @ So.rhs(orc.POINT_SOURCE, x0)) <= TOL
    if So.complex:
        kv = (0.0, 0.6, 0.8)
        bp = s.rhs(B.BEM_DATA_PLANE_WAVE, [kv]).cpu().numpy().reshape(-1)
        assert relerr(bp, P.T @ So.rhs(orc.PLANE_WAVE, kv)) <= TOL
    if not So.complex:
        # samples of the Laplace point source at the exported points reproduce the load vector
        xyz = s.quadpoints().cpu().numpy()
        g = 1.0 / (4 * math.pi * np.linalg.norm(xyz - np.array(x0), axis=1))
        bs = s.rhs_from_samples(torch.from_numpy(g).cuda()).cpu().numpy().reshape(-1)
        assert relerr(bs, b) <= 1e-13
    rho = W.random_vector(W.rng(9, 71), s.ndof, is_complex=So.complex)
    if CASES[cid][7] > 0.0:
        assert relerr(A.moments(torch.from_numpy(rho).cuda()), Ho.moments(P @ rho)) <= TOL


@pytest.mark.parametrize("cid", list(CASES))
def test_potential(B, orc, cid):
    s, A, So, Ho, P = case(B, orc, cid)
    rho = W.random_vector(W.rng(9, 72), s.ndof, is_complex=So.complex)
    pts = np.concatenate([W.exterior_points(W.rng(9, 73), 24, 1.05, 2.0), W.exterior_points(W.rng(9, 74), 8, 3.0, 6.0)])
    rt = torch.from_numpy(rho).cuda()
    u = s.potential(pts, rt).cpu().numpy()
    assert relerr(u, So.potential(P @ rho, pts)) <= TOL
    if CASES[cid][7] > 0.0:
        ut = A.potential(pts, rt).cpu().numpy()
        assert relerr(ut, Ho.potential(P @ rho, pts)) <= TOL


def test_exterior_dirichlet_solve(B, orc):
    """GMRES on the glued system matches the oracle's direct solution of the same H^2 system,
    and the potential reproduces the point source outside the sphere."""
    s, A, So, Ho, P = case(B, orc, "sphere_L2_d1_laplace_h2")
    x0, pts = W.c0_inputs()
    b = s.rhs(B.BEM_DATA_POINT_SOURCE, [x0])
    x, st = A.solve(b, tol=1e-13, maxit=5000)
    assert st[0][1] and st[0][2] <= 1e-13
    N = s.ndof
    Ah = np.stack([P.T @ Ho.apply(P[:, j]) for j in range(N)], 1)
    xo = np.linalg.solve(Ah, P.T @ So.rhs(orc.POINT_SOURCE, x0))
    xg = x.cpu().numpy().reshape(-1)
    assert np.linalg.norm(xg - xo) <= 1e-8 * np.linalg.norm(xo)
    u = A.space.potential(pts, x.reshape(-1)).cpu().numpy()
    ex = 1.0 / (4 * math.pi * np.linalg.norm(pts - np.array(x0), axis=1))
    err = relerr(u, ex)
    print(f"S0 exterior Dirichlet on the GPU: potential error {err:.2e}")
    assert err <= 1e-4


def test_unsupported_combinations(B):
    g = B.Geometry(B.BEM_GEOM_SPHERE6)
    s = B.Space(g, B.BEM_LAPLACE_SINGLE, 0.0, degree=1, level=2, continuous=True)
    A = B.Operator(s, q=3, eta=1.6, leaf_level=1)
    for call in (A.precond_build, lambda: A.profile(True)):
        with pytest.raises(B.BemError) as e:
            call()
        assert e.value.code == B._bem.BEM_EUNSUPPORTED
    x = torch.zeros(s.ndof, dtype=torch.float64, device="cuda")
    with pytest.raises(B.BemError) as e:
        A.apply_stage(0, x, torch.empty_like(x))
    assert e.value.code == B._bem.BEM_EUNSUPPORTED
    with pytest.raises(B.BemError) as e:
        B.Group([A], [x.reshape(1, -1)], [torch.empty_like(x).reshape(1, -1)])
    assert e.value.code == B._bem.BEM_EUNSUPPORTED


def test_sampled_rows_at_size(B, orc):
    """Sphere, L = 5, d = 2, q = 5, leaf 3 (about 7,000 glued functions): sampled global rows,
    each the sum over its local functions of the oracle's rows, including functions glued
    at patch edges and vertices."""
    print("[s0 sampled rows] sphere L5 d2", flush=True)
    g = B.Geometry(B.BEM_GEOM_SPHERE6)
    s = B.Space(g, B.BEM_LAPLACE_SINGLE, 0.0, degree=2, level=5, continuous=True)
    A = B.Operator(s, q=5, eta=1.6, leaf_level=3)
    So = orc.Space(orc.SPHERE, [], orc.LAPLACE, 0.0, degree=2, level=5, form=0)
    Ho = orc.H2(So, q=5, eta=1.6, leaf=3, assemble_near=False)
    m, n = So.glue()
    assert s.ndof == n and np.array_equal(s.glue(), m.astype(np.int32))
    x = W.random_vector(W.rng(9, 75), n)
    y = A.apply(torch.from_numpy(x).cuda()).cpu().numpy()
    xl = x[m]
    sizes = np.bincount(m, minlength=n)
    glob = sorted(set(W.sample_rows(1, n, 4).tolist()) | {int(np.argmax(sizes == 2)), int(np.argmax(sizes == 3))})
    assert sizes[glob].max() == 3
    for G in glob:
        loc = np.nonzero(m == G)[0].astype(np.int64)
        Ho.assemble_near_rows(loc)
        yo = Ho.apply_rows(xl, loc).sum()
        assert abs(y[G] - yo) <= TOL * np.max(np.abs(y)), G
