"""Pins of the oracle's continuous spaces S^0 (App. E: 0-form lifting, continuity across
patch boundaries) against facts outside the oracle.

- Glued counts: closed forms for the cube-sphere (6 faces, 12 edges, 8 vertices) and the
  torus (16 faces, 32 edges, 16 vertices).
- Continuity: a glued function evaluated from both sides of every shared patch edge agrees.
- Flat square: the 0-form matrix is a^4 times the 2-form one (kappa = a^2), exactly.
- Unit sphere, Laplace: the constant is in S^0 and V 1 = 1 on the sphere, so
  1^T A 1 = <V 1, 1> = 4 pi; the load vector of G(., x0), x0 inside, sums to
  int G(x, x0) dsigma = 1 (single-layer potential of the unit density inside the sphere).
- Exterior Dirichlet problem: the S^0 Galerkin solution reproduces 1/(4 pi |x - x0|).
- H^2 on S^0: eta = 0 equals the dense matrix; transferred moments equal directly
  integrated ones.
All run on the CPU.
"""
import math

import numpy as np
import pytest

import workloads as W


def glued(S):
    m, n = S.glue()
    P = np.zeros((S.ndof, n))
    P[np.arange(S.ndof), m] = 1.0
    return P


@pytest.mark.parametrize("d,L", [(1, 1), (2, 1), (1, 2), (2, 2)])
def test_glued_counts(orc, d, L):
    nb = (1 << L) + d
    S = orc.Space(orc.SPHERE, [], orc.LAPLACE, 0.0, degree=d, level=L, form=0)
    assert S.glue()[1] == 6 * (nb - 2) ** 2 + 12 * (nb - 2) + 8
    T = orc.Space(orc.TORUS, [1.0, 0.4], orc.LAPLACE, 0.0, degree=d, level=L, form=0)
    assert T.glue()[1] == 16 * (nb - 2) ** 2 + 32 * (nb - 2) + 16


def test_glued_functions_are_continuous(orc):
    """Every global function of the glued space, evaluated on both sides of the edges of
    patch 0 of the sphere, gives the same values."""
    d, L = 2, 1
    S = orc.Space(orc.SPHERE, [], orc.LAPLACE, 0.0, degree=d, level=L, form=0)
    m, n = S.glue()
    nb = (1 << L) + d
    ts = np.linspace(0.0, 1.0, 7)
    st = {k: np.array(pts) for k, pts in
          {"s0": [[0.0, t] for t in ts], "s1": [[1.0, t] for t in ts], "t0": [[t, 0.0] for t in ts],
           "t1": [[t, 1.0] for t in ts]}.items()}

    def values(f, pts, coeff):
        """sum_j c_j b_j1(s) b_j2(t) on patch f at parameter points."""
        B1 = np.stack([orc.bspline(d, 1, L, j, pts[:, 0]) for j in range(nb)], 1)
        B2 = np.stack([orc.bspline(d, 1, L, j, pts[:, 1]) for j in range(nb)], 1)
        return np.einsum("pi,pj,ij->p", B1, B2, coeff.reshape(6, nb, nb)[f])

    hits = 0
    for gdof in range(n):
        coeff = (m == gdof).astype(float)
        for edge, pts in st.items():
            x0, _, _ = S.gamma(0, pts)
            v0 = values(0, pts, coeff)
            # the same physical points on the neighbouring patch, found by their images
            for f in range(1, 6):
                grid = np.array([[a, b] for a in np.linspace(0, 1, 7) for b in np.linspace(0, 1, 7)])
                xf, _, _ = S.gamma(f, grid)
                for k, x in enumerate(x0):
                    hit = np.where(np.linalg.norm(xf - x, axis=1) < 1e-12)[0]
                    if hit.size:
                        hits += 1
                        assert abs(values(f, grid[hit[:1]], coeff)[0] - v0[k]) <= 1e-14
    assert hits >= n * 4 * 7  # every edge point of patch 0 lies on a neighbour


def test_flat_square_zero_form_scales(orc):
    a = 1.7
    A2 = orc.Space(orc.FLAT, [a], orc.LAPLACE, 0.0, degree=2, level=1).dense(8, 8)
    A0 = orc.Space(orc.FLAT, [a], orc.LAPLACE, 0.0, degree=2, level=1, form=0).dense(8, 8)
    assert np.max(np.abs(A0 - a ** 4 * A2)) <= 1e-13 * np.max(np.abs(A0))


def test_constant_density_on_the_unit_sphere(orc):
    S = orc.Space(orc.SPHERE, [], orc.LAPLACE, 0.0, degree=1, level=2, form=0)
    P = glued(S)
    A = P.T @ S.dense(8, 8) @ P
    one = np.ones(P.shape[1])
    assert abs(one @ A @ one - 4 * math.pi) <= 1e-8 * 4 * math.pi
    b = P.T @ S.rhs(orc.POINT_SOURCE, (0.1, -0.2, 0.15))
    assert abs(b.sum() - 1.0) <= 1e-10
    assert np.max(np.abs(A - A.T)) <= 1e-13 * np.max(np.abs(A))


def test_exterior_dirichlet_s0(orc):
    S = orc.Space(orc.SPHERE, [], orc.LAPLACE, 0.0, degree=1, level=2, form=0)
    P = glued(S)
    x0, pts = W.c0_inputs()
    A = P.T @ S.dense(8, 8) @ P
    rho = P @ np.linalg.solve(A, P.T @ S.rhs(orc.POINT_SOURCE, x0))
    u = S.potential(rho, pts)
    ex = 1.0 / (4 * math.pi * np.linalg.norm(pts - x0, axis=1))
    err = np.max(np.abs(u - ex)) / np.max(np.abs(ex))
    print("S0 exterior Dirichlet error", err)
    assert err < 1e-4


@pytest.mark.parametrize("pde,kappa", [(0, 0.0), (1, 2.0)])
def test_h2_on_s0(orc, pde, kappa):
    S1 = orc.Space(orc.ELLIPSOID, [0.8, 1.1, 1.3], pde, kappa, degree=2, level=1, form=0)
    x1 = W.random_vector(W.rng(9, 61), S1.ndof, is_complex=bool(pde))
    H0 = orc.H2(S1, q=4, eta=0.0, leaf=1)
    D = S1.dense(8, 8)
    assert np.max(np.abs(H0.apply(x1) - D @ x1)) <= 1e-13 * np.max(np.abs(D @ x1))
    S = orc.Space(orc.ELLIPSOID, [0.8, 1.1, 1.3], pde, kappa, degree=2, level=2, form=0)
    x = W.random_vector(W.rng(9, 60), S.ndof, is_complex=bool(pde))
    H = orc.H2(S, q=4, eta=1.6, leaf=2, assemble_near=False)
    m_t, m_d = H.moments(x), H.moments(x, direct=True)
    assert np.max(np.abs(m_t - m_d)) <= 1e-13 * np.max(np.abs(m_d))
