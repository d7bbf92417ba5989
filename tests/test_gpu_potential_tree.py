"""GPU: potential through the cluster tree (bem_eval_potential_h2) against the oracle's
tree potential on the same operator parameters, and against the plain quadrature.

Bar: within 1e-11 (max-norm relative) of the oracle's tree potential with the same q, leaf
level and eta, for points near and far from the surface, Laplace and Helmholtz, analytic and
NURBS geometries, one and several columns; eta = 0 equals bem_eval_potential to 1e-13 (same
quadrature, different summation order).  At the benchmark size: sampled points against
the oracle, and a grid of 100,000 points.
"""
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
    return float(np.max(np.abs(np.asarray(a) - np.asarray(b))) / np.max(np.abs(b)))


CASES = {
    # id: (geometry maker, oracle geometry, pde, kappa, L, d, q, leaf)
    "sphere_laplace": (lambda B: B.Geometry(B.BEM_GEOM_SPHERE6), (0, []), 0, 0.0, 3, 2, 5, 1),
    "ellipsoid_helmholtz": (lambda B: B.Geometry(B.BEM_GEOM_ELLIPSOID6, (0.8, 1.1, 1.3)), (1, [0.8, 1.1, 1.3]), 1,
                            3.0, 3, 1, 4, 2),
    "nurbs_torus_laplace": (lambda B: B.Geometry.nurbs(W.nurbs_torus(1.0, 0.4)), (4, W.nurbs_torus(1.0, 0.4)), 0,
                            0.0, 2, 1, 4, 1),
}


@pytest.mark.parametrize("cid", list(CASES))
def test_tree_potential_matches_oracle(B, orc, cid):
    mk, (og, oprm), pde, kappa, L, d, q, leaf = CASES[cid]
    print(f"[potential {cid}]", flush=True)
    s = B.Space(mk(B), pde, kappa, degree=d, level=L)
    A = B.Operator(s, q=q, eta=1.6, leaf_level=leaf)
    So = orc.Space(og, oprm, pde, kappa, degree=d, level=L)
    Ho = orc.H2(So, q=q, eta=1.6, leaf=leaf, assemble_near=False)
    rho = W.random_vector(W.rng(9, 50), s.ndof, is_complex=bool(pde), ncols=2).T.copy()
    pts = np.concatenate([W.exterior_points(W.rng(9, 51), 40, 1.02, 2.0), W.exterior_points(W.rng(9, 52), 24, 3.0, 9.0)])
    u = A.potential(pts, torch.from_numpy(rho).cuda()).cpu().numpy()
    for r in range(2):
        assert relerr(u[r], Ho.potential(rho[r], pts)) <= TOL, r
    # eta = 0: the plain quadrature over every leaf
    u0 = A.potential(pts, torch.from_numpy(rho[0]).cuda(), eta=0.0).cpu().numpy()
    ud = s.potential(pts, torch.from_numpy(rho[0]).cuda()).cpu().numpy()
    assert relerr(u0, ud) <= 1e-13


def test_tree_potential_full_size(B, orc):
    """The benchmark operator (sphere, L = 6, d = 2, q = 5, leaf 4): sampled points against
    the oracle, and 100,000 points against the plain quadrature's error scale."""
    c = W.CONFIGS[1]
    g = B.Geometry(B.BEM_GEOM_SPHERE6)
    s = B.Space(g, B.BEM_LAPLACE_SINGLE, 0.0, degree=c["degree"], level=c["level"])
    A = B.Operator(s, q=c["q"], eta=c["eta"], leaf_level=c["leaf"], far_eval=True)
    So = orc.Space(orc.SPHERE, [], orc.LAPLACE, 0.0, degree=c["degree"], level=c["level"])
    Ho = orc.H2(So, q=c["q"], eta=c["eta"], leaf=c["leaf"], assemble_near=False)
    rho = W.random_vector(W.rng(1, 53), s.ndof)
    pts = np.concatenate([W.exterior_points(W.rng(1, 54), 12, 1.01, 1.2), W.exterior_points(W.rng(1, 55), 12, 2.0, 4.0)])
    rt = torch.from_numpy(rho).cuda()
    u = A.potential(pts, rt).cpu().numpy()
    assert relerr(u, Ho.potential(rho, pts)) <= TOL
    # a grid of 100,000 points; a random density (measured 2.1e-3 against the plain quadrature,
    # relative to the largest value: its potential is small by cancellation while the
    # interpolation error scales with the density) and the smooth solution of the exterior
    # Dirichlet problem, whose potential is 1/(4 pi |x - x0|)
    grid = W.exterior_points(W.rng(1, 56), 100000, 1.5, 5.0)
    ug = A.potential(grid, rt).cpu().numpy()
    ud = s.potential(grid[:2000], rt).cpu().numpy()
    err = relerr(ug[:2000], ud)
    x0, _ = W.c1_inputs()
    b = s.rhs(B.BEM_DATA_POINT_SOURCE, [x0])
    sol, st = A.solve(b, tol=1e-10)
    assert st[0][1]
    us = A.potential(grid, sol[0]).cpu().numpy()
    uq = s.potential(grid[:2000], sol[0]).cpu().numpy()
    ex = 1.0 / (4 * np.pi * np.linalg.norm(grid - np.array(x0), axis=1))
    e_tree, e_plain = relerr(us, ex), relerr(uq, ex[:2000])
    print(f"[potential full size] 100000 points; random density: tree vs plain quadrature {err:.2e}; "
          f"solved density: tree vs exact {e_tree:.2e}, plain quadrature vs exact {e_plain:.2e}")
    assert np.isfinite(ug).all() and err <= 5e-3
    assert e_tree <= 1e-3
