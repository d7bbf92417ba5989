"""Pins of the oracle's NURBS patch maps (App. C) against facts outside the oracle.

- The map against scipy's B-splines: numerator and denominator of the rational map built
  from scipy.interpolate.BSpline design matrices (library), at random points, knots and
  the patch corners; its surface element against central differences of that map.
- The NURBS torus (rational biquadratic arcs): every point on the torus (implicit
  equation), area 4 pi^2 R r (closed form), outward normals.
- A flat NURBS patch with non-uniform knots and equal weights whose control points sit at
  the Greville abscissae is the identity map (linear precision): its Galerkin matrix equals
  the flat square's (special case reducing to an existing, pinned geometry).
- Exterior Dirichlet problem on the NURBS torus: the potential reproduces
  1/(4 pi |x - x0|) (closed form).
All run on the CPU.
"""
import math

import numpy as np
import pytest
from scipy.interpolate import BSpline

import workloads as W


def scipy_map(P, s, t):
    """Rational map of a patch from scipy B-spline design matrices."""
    (p1, p2), (k1, k2) = P["degree"], P["knots"]
    c = np.asarray(P["cw"])
    B1 = BSpline.design_matrix(np.atleast_1d(s), np.asarray(k1, float), p1, extrapolate=False).toarray()
    B2 = BSpline.design_matrix(np.atleast_1d(t), np.asarray(k2, float), p2, extrapolate=False).toarray()
    w = c[:, :, 3]
    num = np.einsum("pi,pj,ijd->pd", B1, B2, c[:, :, :3] * w[:, :, None])
    den = np.einsum("pi,pj,ij->p", B1, B2, w)
    return num / den[:, None]


def random_patch(g, p=(3, 2), k1=(0.0, 0.0, 0.0, 0.0, 0.15, 0.5, 0.5, 0.8, 1.0, 1.0, 1.0, 1.0),
                 k2=(0.0, 0.0, 0.0, 0.3, 0.6, 1.0, 1.0, 1.0)):
    n1, n2 = len(k1) - p[0] - 1, len(k2) - p[1] - 1
    cw = np.zeros((n1, n2, 4))
    cw[:, :, :3] = g.normal(size=(n1, n2, 3))
    cw[:, :, 3] = g.uniform(0.5, 2.0, size=(n1, n2))
    return {"degree": p, "knots": (list(k1), list(k2)), "cw": cw}


def test_map_matches_scipy_bsplines(orc):
    g = W.rng(9, 1)
    P = random_patch(g)
    S = orc.Space(orc.NURBS, [P], orc.LAPLACE, 0.0, degree=1, level=1)
    st = np.concatenate([g.uniform(size=(200, 2)),
                         [[0.0, 0.0], [1.0, 1.0], [0.0, 1.0], [1.0, 0.0], [0.5, 0.3], [0.15, 0.6], [0.8, 1.0]]])
    xyz, kap, nrm = S.gamma(0, st)
    ref = np.stack([scipy_map(P, s, t)[0] for s, t in st])
    assert np.max(np.abs(xyz - ref)) <= 1e-14 * np.max(np.abs(ref))
    # surface element against central differences of the scipy map (interior points, away
    # from the knots where the cubic direction is only C^1 across the double knot 0.5)
    h = 1e-6
    for s, t in g.uniform(0.02, 0.98, size=(40, 2)):
        if min(abs(s - k) for k in (0.15, 0.5, 0.8)) < 2 * h or min(abs(t - k) for k in (0.3, 0.6)) < 2 * h:
            continue
        xs = (scipy_map(P, s + h, t)[0] - scipy_map(P, s - h, t)[0]) / (2 * h)
        xt = (scipy_map(P, s, t + h)[0] - scipy_map(P, s, t - h)[0]) / (2 * h)
        kfd = np.linalg.norm(np.cross(xs, xt))
        _, k, n = S.gamma(0, [[s, t]])
        assert abs(k[0] - kfd) <= 1e-7 * kfd
        assert np.allclose(n[0], np.cross(xs, xt), rtol=0, atol=1e-7 * kfd)


def test_torus_points_area_normals(orc):
    R, r = 1.0, 0.35
    S = orc.Space(orc.NURBS, W.nurbs_torus(R, r), orc.LAPLACE, 0.0, degree=1, level=2)
    g = W.rng(9, 2)
    for f in range(16):
        st = g.uniform(size=(50, 2))
        xyz, _, nrm = S.gamma(f, st)
        rho = np.hypot(xyz[:, 0], xyz[:, 1])
        assert np.max(np.abs((rho - R) ** 2 + xyz[:, 2] ** 2 - r * r)) <= 1e-14
        ctr = np.stack([R * xyz[:, 0] / rho, R * xyz[:, 1] / rho, np.zeros_like(rho)], axis=1)
        assert np.all(np.sum(nrm * (xyz - ctr), axis=1) > 0)  # outward
    assert abs(S.area(8) - 4 * math.pi ** 2 * R * r) <= 1e-12 * 4 * math.pi ** 2 * R * r


def test_flat_identity_patch_equals_flat_square(orc):
    a = 1.7
    S_n = orc.Space(orc.NURBS, W.nurbs_flat(a), orc.LAPLACE, 0.0, degree=1, level=2)
    S_f = orc.Space(orc.FLAT, [a], orc.LAPLACE, 0.0, degree=1, level=2)
    st = W.rng(9, 3).uniform(size=(100, 2))
    xn, kn, _ = S_n.gamma(0, st)
    xf, kf, _ = S_f.gamma(0, st)
    assert np.max(np.abs(xn - xf)) <= 1e-15 * a and np.max(np.abs(kn - a * a)) <= 1e-14
    An, Af = S_n.dense(8, 8), S_f.dense(8, 8)
    assert np.max(np.abs(An - Af)) <= 1e-14 * np.max(np.abs(Af))


def test_exterior_dirichlet_on_nurbs_torus(orc):
    R, r = 1.0, 0.4
    x0 = np.array([0.9, 0.3, 0.05])  # inside the tube
    pts = W.exterior_points(W.rng(9, 4), 24, 2.0, 4.0)
    ex = 1.0 / (4 * math.pi * np.linalg.norm(pts - x0, axis=1))
    # level 2, degree 1 (400 DOFs, dense; 6 Gauss points per direction for regular pairs and
    # 5 for the Duffy cubes): measured 2.9e-6 (8.4e-6 with 8 and 8; the analytic torus map
    # gives 2.9e-5 at the same level; level 1 gives 1.8e-3)
    S = orc.Space(orc.NURBS, W.nurbs_torus(R, r), orc.LAPLACE, 0.0, degree=1, level=2)
    rho = np.linalg.solve(S.dense(6, 5), S.rhs(orc.POINT_SOURCE, x0))
    err = np.max(np.abs(S.potential(rho, pts) - ex)) / np.max(np.abs(ex))
    print("NURBS torus exterior Dirichlet error", err)
    assert err < 5e-5


# ---------------------------------------------------------------- user-supplied maps (reading)
def test_user_map_reproduces_polynomial_maps(orc):
    """A map that is a polynomial of degree <= the interpolant's degree is reproduced
    exactly: the flat square's user map gives the flat square's Galerkin matrix."""
    a = 1.3
    P = orc.user_map_patches(lambda f, st: np.stack([a * st[:, 0], a * st[:, 1], 0 * st[:, 0]], 1), 1, 3, 4)
    S_u = orc.Space(orc.NURBS, P, orc.LAPLACE, 0.0, degree=2, level=1)
    S_f = orc.Space(orc.FLAT, [a], orc.LAPLACE, 0.0, degree=2, level=1)
    Au, Af = S_u.dense(8, 8), S_f.dense(8, 8)
    assert np.max(np.abs(Au - Af)) <= 1e-14 * np.max(np.abs(Af))


def test_user_map_interpolant_converges(orc):
    """The interpolant of the sphere's patch maps converges at the spline order p + 1
    (measured: degree 5, 8 -> 16 intervals: 1.3e-5 -> 1.2e-7), its patches still meet edge
    to edge (the Galerkin matrix stays symmetric, which the Duffy rules of touching pairs
    need), and its operator approaches the analytic sphere's by the interpolation error."""
    Sa = orc.Space(orc.SPHERE, [], orc.LAPLACE, 0.0, degree=1, level=1)
    st = W.rng(9, 5).uniform(size=(200, 2))
    errs = []
    for m in (8, 16):
        Su = orc.Space(orc.NURBS, orc.user_map_patches(W.sphere6_map, 6, 5, m), orc.LAPLACE, 0.0, degree=1,
                       level=1)
        errs.append(max(np.abs(Su.gamma(f, st)[0] - Sa.gamma(f, st)[0]).max() for f in range(6)))
    assert errs[0] < 3e-5 and math.log2(errs[0] / errs[1]) > 5.5
    Au, Aa = Su.dense(6, 6), Sa.dense(6, 6)  # the same rules on both (measured difference 4.4e-8)
    assert np.max(np.abs(Au - Au.T)) <= 1e-14 * np.max(np.abs(Au))
    assert np.max(np.abs(Au - Aa)) <= 1e-5 * np.max(np.abs(Aa))
