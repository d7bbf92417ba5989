"""CPU pins of the oracle's block-Jacobi preconditioner (tiles, blocks, LU apply,
right-preconditioned GMRES, learned-correction targets).

Pinned by: the partition of the DOFs, the dense Galerkin matrix (eta = 0: everything is near
field, so the blocks are principal submatrices of the dense matrix), numpy's solve and
inverse, the unpreconditioned oracle GMRES (same system, same solution), and the exact
preconditioner (one tile that covers the whole system converges in one step).
"""
import numpy as np
import pytest

import workloads as W


def _h2(orc, geom, prm, pde, kappa, L, d, q, eta, leaf):
    S = orc.Space(geom, list(prm), pde, kappa, degree=d, level=L)
    return S, orc.H2(S, q=q, eta=eta, leaf=leaf)


@pytest.mark.parametrize("L,d,T", [(2, 1, 8), (2, 2, 4)])
def test_tiles_partition_the_dofs(orc, L, d, T):
    S, H = _h2(orc, orc.SPHERE, (), orc.LAPLACE, 0.0, L, d, 3, 1.6, 1)
    bj = orc.BlockJacobi(H, tile=T)
    nb = d + 1 + (2 ** L - 1)
    nt = -(-nb // T)
    assert bj.ntiles == 6 * nt * nt
    seen = np.concatenate([bj.tile(k)[1] for k in range(bj.ntiles)])
    assert np.array_equal(np.sort(seen), np.arange(S.ndof))
    for k in range(bj.ntiles):
        (f, a1, b1, a2, b2), dofs = bj.tile(k)
        assert b1 - a1 == min(T, nb - a1) and b2 - a2 == min(T, nb - a2)
        j1, j2 = np.divmod(dofs - f * nb * nb, nb)
        assert np.all((j1 >= a1) & (j1 < b1) & (j2 >= a2) & (j2 < b2))


@pytest.mark.parametrize("pde,kappa", [(0, 0.0), (1, 2.5)])
def test_blocks_are_principal_submatrices_in_dense_mode(orc, pde, kappa):
    S, H = _h2(orc, orc.SPHERE, (), pde, kappa, 2, 1, 3, 0.0, 0)
    A = S.dense(8, 8)
    bj = orc.BlockJacobi(H, tile=3)  # nb = 5: tiles of 3 and 2 indices, including short ones
    for k in range(bj.ntiles):
        _, dofs = bj.tile(k)
        D = bj.block(k)
        assert np.max(np.abs(D - A[np.ix_(dofs, dofs)])) <= 1e-13 * np.max(np.abs(A))


@pytest.mark.parametrize("pde,kappa", [(0, 0.0), (1, 2.5)])
def test_apply_solves_every_block(orc, pde, kappa):
    S, H = _h2(orc, orc.SPHERE, (), pde, kappa, 2, 2, 4, 1.6, 1)
    bj = orc.BlockJacobi(H, tile=4)
    r = W.random_vector(W.rng(0, 70), S.ndof, is_complex=S.complex)
    z = bj.apply(r)
    for k in range(bj.ntiles):
        _, dofs = bj.tile(k)
        zk = np.linalg.solve(bj.block(k), r[dofs])
        assert np.max(np.abs(z[dofs] - zk)) <= 1e-12 * np.max(np.abs(zk))


@pytest.mark.parametrize("pde,kappa", [(0, 0.0), (1, 2.5)])
def test_preconditioned_gmres_solves_the_same_system(orc, pde, kappa):
    S, H = _h2(orc, orc.SPHERE, (), pde, kappa, 2, 2, 4, 1.6, 1)
    bj = orc.BlockJacobi(H, tile=4)
    b = S.rhs(orc.POINT_SOURCE, W.CONFIGS[0]["x0"])
    x0, it0, rr0, ok0 = H.gmres(b, tol=1e-12)
    x1, it1, rr1, ok1 = bj.gmres(b, tol=1e-12)
    assert ok0 and ok1 and rr1 <= 1e-12
    # two solutions of the same system to a residual of 1e-12 differ by up to cond * 2e-12
    assert np.linalg.norm(x1 - x0) / np.linalg.norm(x0) <= 1e-8
    # the true residual of the preconditioned solution, through the operator itself
    assert np.linalg.norm(H.apply(x1) - b) / np.linalg.norm(b) <= 1e-12
    assert it1 < it0


def test_exact_preconditioner_converges_in_one_step(orc):
    # one patch, nb = 5 <= 8: one tile holds every DOF, and eta = 0 makes the near field the
    # whole matrix, so M = A
    S, H = _h2(orc, orc.FLAT, (1.0,), orc.LAPLACE, 0.0, 2, 1, 3, 0.0, 0)
    bj = orc.BlockJacobi(H, tile=8)
    assert bj.ntiles == 1
    b = S.rhs(orc.POINT_SOURCE, (0.3, 0.4, 0.5))
    x, it, rr, ok = bj.gmres(b, tol=1e-12)
    assert ok and it == 1
    A = S.dense(8, 8)
    assert np.linalg.norm(x - np.linalg.solve(A, b)) <= 1e-11 * np.linalg.norm(x)


def test_targets(orc):
    # ring 0: N(b) = b, so the least-squares inverse is D_b^{-1}
    S, H = _h2(orc, orc.SPHERE, (), orc.HELMHOLTZ, 2.5, 2, 1, 4, 1.6, 1)
    bj = orc.BlockJacobi(H, tile=3)
    for k in (0, 3):
        C = bj.target(k, 0)
        assert np.max(np.abs(C - np.linalg.inv(bj.block(k)))) <= 1e-10 * np.max(np.abs(C))
    # ring 2: numpy's least-squares solution of A[N(b), b] X = I[N(b), b] from the near field
    rowptr, col, val = H.near_csr()
    nb = 5
    for k in (0, 4, 8):
        (f, a1, b1, a2, b2), dofs = bj.tile(k)
        nbh = [(f * nb + j1) * nb + j2 for j1 in range(max(0, a1 - 2), min(nb, b1 + 2))
               for j2 in range(max(0, a2 - 2), min(nb, b2 + 2))]
        Anb = np.zeros((len(nbh), len(dofs)), dtype=complex)
        for i, g in enumerate(nbh):
            cols = col[rowptr[g]:rowptr[g + 1]]
            for j, h in enumerate(dofs):
                hit = np.nonzero(cols == h)[0]
                if hit.size:
                    Anb[i, j] = val[rowptr[g] + hit[0]]
        I = np.array([[1.0 if g == h else 0.0 for h in dofs] for g in nbh])
        X = np.linalg.lstsq(Anb, I, rcond=None)[0]
        C = bj.target(k, 2)
        assert np.max(np.abs(C - X)) <= 1e-9 * np.max(np.abs(X)), k
