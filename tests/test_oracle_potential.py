"""Pins of the oracle's tree-accelerated potential (source-side interpolation over the
cluster tree, near leaves by plain quadrature) against the plain quadrature of the
potential (Sec. 4 "Evaluation of the Solution"), which the exterior Dirichlet pins tie to
closed forms.

- eta = 0: no cluster is admissible, every point takes the plain quadrature over all
  leaves: equal to the dense potential up to summation order (special case).
- The difference to the dense potential decays geometrically in q (interpolation of the
  kernel in the source variable), for Laplace and Helmholtz, near and far points.
All run on the CPU.
"""
import numpy as np
import pytest

import workloads as W


def rel(a, b):
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


@pytest.mark.parametrize("pde,kappa", [(0, 0.0), (1, 3.0)])
def test_eta_zero_is_the_plain_quadrature(orc, pde, kappa):
    S = orc.Space(orc.SPHERE, [], pde, kappa, degree=1, level=3)
    H = orc.H2(S, q=4, eta=1.6, leaf=1, assemble_near=False)
    rho = W.random_vector(W.rng(9, 30), S.ndof, is_complex=bool(pde))
    pts = W.exterior_points(W.rng(9, 31), 40, 1.05, 3.0)
    assert rel(H.potential(rho, pts, eta=0.0), S.potential(rho, pts)) <= 1e-14


@pytest.mark.parametrize("pde,kappa", [(0, 0.0), (1, 3.0)])
def test_geometric_convergence_in_q(orc, pde, kappa):
    S = orc.Space(orc.ELLIPSOID, [0.8, 1.1, 1.3], pde, kappa, degree=2, level=3)
    rho = W.random_vector(W.rng(9, 32), S.ndof, is_complex=bool(pde))
    pts = np.concatenate([W.exterior_points(W.rng(9, 33), 30, 1.4, 2.0), W.exterior_points(W.rng(9, 34), 10, 5.0, 9.0)])
    ref = S.potential(rho, pts)
    errs = []
    for q in (3, 4, 5, 6, 7):
        H = orc.H2(S, q=q, eta=1.6, leaf=2, assemble_near=False)
        errs.append(rel(H.potential(rho, pts), ref))
    print("tree potential errors q=3..7:", errs)
    # measured, Laplace: 4.4e-3, 9.4e-4, 3.4e-4, 8.6e-5, 2.0e-5; Helmholtz (kappa 3, whose
    # oscillation across the top-level clusters needs the larger q): 0.10, 2.6e-2, 1.7e-2, 5.9e-3, 2.4e-3
    assert all(b < a / 1.3 for a, b in zip(errs, errs[1:]))
    assert errs[0] / errs[-1] > (100 if pde == 0 else 30)
