"""Pins of the oracle against facts that do not come from the oracle itself.

Each test names what it pins: a closed form, an invariant, a library routine or brute force.
All run on the CPU.  A plausible mistake (dropped term, wrong sign or index, transposed
operand, wrong rotation) in any oracle function should fail at least one of them.
"""
import json
import math
import os

import numpy as np
import pytest
from scipy.interpolate import BSpline
from scipy.special import elliprg, spherical_jn, spherical_yn

import workloads as W

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "closed_forms.json")))
I_ID = GOLDEN["flat_identical_1_over_r"]["value"]


@pytest.fixture(scope="module")
def c0(orc):
    """Dense C0 operator: sphere6, L=2, d=1, Laplace."""
    S = orc.Space(orc.SPHERE, [], orc.LAPLACE, 0.0, degree=1, level=2)
    A = S.dense(8, 8)
    return S, A


# ---------------------------------------------------------------- quadrature (library)
@pytest.mark.parametrize("n", [1, 2, 3, 5, 8, 13, 20])
def test_gauss_matches_numpy_and_is_exact(orc, n):
    x, w = orc.gauss01(n)
    xr, wr = np.polynomial.legendre.leggauss(n)
    np.testing.assert_allclose(x, 0.5 * (xr + 1.0), rtol=0, atol=2e-15)
    np.testing.assert_allclose(w, 0.5 * wr, rtol=0, atol=2e-15)
    for k in range(2 * n):  # exact for degree <= 2n-1
        assert abs(np.dot(w, x ** k) - 1.0 / (k + 1)) < 5e-15


# ---------------------------------------------------------------- B-splines (library)
@pytest.mark.parametrize("d,r,L", [(0, 1, 0), (0, 1, 3), (1, 1, 2), (2, 1, 3), (3, 1, 2), (2, 2, 2), (3, 3, 1), (2, 3, 2)])
def test_bsplines_match_scipy(orc, d, r, L):
    nel = 1 << L
    knots = [0.0] * (d + 1) + [k / nel for k in range(1, nel) for _ in range(r)] + [1.0] * (d + 1)
    nb = orc.bspline_count(d, r, L)
    assert nb == len(knots) - d - 1 == d + 1 + (nel - 1) * r
    xs = np.random.default_rng(5).uniform(0, 1, 200)
    tot = np.zeros_like(xs)
    for j in range(nb):
        mine = orc.bspline(d, r, L, j, xs)
        c = np.zeros(nb)
        c[j] = 1.0
        ref = BSpline(np.array(knots), c, d, extrapolate=False)(xs)
        np.testing.assert_allclose(mine, ref, rtol=0, atol=1e-14)
        tot += mine
    np.testing.assert_allclose(tot, 1.0, rtol=0, atol=1e-14)  # partition of unity


# ---------------------------------------------------------------- geometry (closed forms)
def test_areas_closed_forms(orc):
    S = orc.Space(orc.SPHERE, [], orc.LAPLACE, 0, degree=0, level=2)
    assert abs(S.area(10) - 4 * math.pi) < 1e-12
    a, b, c = 0.7, 1.3, 2.0
    S = orc.Space(orc.ELLIPSOID, [a, b, c], orc.LAPLACE, 0, degree=0, level=3)
    ref = 4 * math.pi * a * b * c * elliprg(a ** -2, b ** -2, c ** -2)
    assert abs(S.area(12) - ref) / ref < 1e-12
    R, r = 1.0, 0.35
    S = orc.Space(orc.TORUS, [R, r], orc.LAPLACE, 0, degree=0, level=2)
    assert abs(S.area(10) - 4 * math.pi ** 2 * R * r) / (4 * math.pi ** 2 * R * r) < 1e-12


@pytest.mark.parametrize("geom,prm", [(0, []), (1, [0.6, 1.1, 1.9]), (2, [1.0, 0.3])])
def test_normals_point_outward(orc, geom, prm):
    S = orc.Space(geom, prm, orc.LAPLACE, 0, degree=0, level=0)
    st = np.random.default_rng(3).uniform(0.01, 0.99, size=(50, 2))
    npatch = 16 if geom == orc.TORUS else 6
    for f in range(npatch):
        x, kap, n = S.gamma(f, st)
        if geom == orc.TORUS:
            R = prm[0]
            rad = np.hypot(x[:, 0], x[:, 1])
            centre = np.stack([R * x[:, 0] / rad, R * x[:, 1] / rad, np.zeros_like(rad)], axis=1)
            out = x - centre
        else:
            out = x
        assert np.all(np.sum(out * n, axis=1) > 0)
        np.testing.assert_allclose(np.linalg.norm(n, axis=1), kap, rtol=1e-14)


def test_patches_match_along_shared_edges(orc):
    """App. D matching condition, checked by counting touching element pairs: on the cube
    sphere every element touches 4 others by an edge and 4 by a vertex only, except the 24
    elements at the 8 cube corners (vertices of valence 3), which touch only 3 by a vertex."""
    S = orc.Space(orc.SPHERE, [], orc.LAPLACE, 0, degree=0, level=2)
    counts = np.zeros(4, dtype=int)
    for e1 in range(S.nelem):
        for e2 in range(S.nelem):
            counts[S.classify(e1, e2)[0]] += 1
    ne = S.nelem
    assert counts[3] == ne
    assert counts[2] == 4 * ne
    assert counts[1] == 4 * ne - 24


# ---------------------------------------------------------------- Duffy rules (closed form + invariants)
def test_flat_duffy_identical_closed_form_and_invariants(orc):
    """Flat 4x4 grid of unit squares (side 4, L=2, degree 0): every identical block equals
    I_id/(4 pi) after the parameter measure 4^-4 is undone; all edge blocks are equal and
    all vertex blocks are equal whatever their orientation; self-similarity of the square
    gives I_id = 2 I_e + I_v and the 4x4 grid gives 64 I_id = 16 I_id + 48 I_e + 36 I_v + F."""
    a = 4.0
    S = orc.Space(orc.FLAT, [a], orc.LAPLACE, 0, degree=0, level=2)
    scale = 4 * math.pi * a ** 4
    A = S.dense(8, 8) * scale
    ne = S.nelem
    types = np.array([[S.classify(i, j)[0] for j in range(ne)] for i in range(ne)])
    Iid = A[types == 3]
    Ie = A[types == 2]
    Iv = A[types == 1]
    far = A[types == 0].sum()
    assert len(Iid) == 16 and len(Ie) == 48 and len(Iv) == 36
    np.testing.assert_allclose(Iid, I_ID, rtol=1e-11)
    assert np.ptp(Ie) < 1e-13 and np.ptp(Iv) < 1e-13
    ie, iv = Ie.mean(), Iv.mean()
    assert abs(I_ID - (2 * ie + iv)) < 1e-11
    # far sum at higher order for the second invariant
    A20 = S.dense(20, 8) * scale
    far20 = A20[types == 0].sum()
    assert abs(64 * I_ID - (16 * I_ID + 48 * ie + 36 * iv + far20)) < 1e-10 * 64 * I_ID
    assert abs(far - far20) < 1e-9 * far20


# ---------------------------------------------------------------- sphere eigenvalues (closed forms)
def _h2(l, k):
    return spherical_jn(l, k) - 1j * spherical_yn(l, k)


@pytest.mark.parametrize("fid,gid,expect", [
    (0, 0, 4 * math.pi),                       # <S 1, 1> = lambda_0 * 4 pi
    (3, 3, (1 / 3) * 4 * math.pi / 3),         # <S z, z> = lambda_1 * 4 pi/3
    (4, 4, (1 / 5) * 4 * math.pi / 15),        # <S xy, xy> = lambda_2 * 4 pi/15
    (3, 4, 0.0),                               # orthogonality of harmonics
    (0, 3, 0.0),
])
def test_sphere_laplace_eigenvalues(orc, fid, gid, expect):
    S = orc.Space(orc.SPHERE, [], orc.LAPLACE, 0, degree=0, level=2)
    v = S.density_pairing(fid, gid, 8, 8)
    assert abs(v - expect) <= 1e-10 * 4 * math.pi


@pytest.mark.parametrize("k", [2.5, -1.7])
def test_sphere_helmholtz_eigenvalues(orc, k):
    S = orc.Space(orc.SPHERE, [], orc.HELMHOLTZ, k, degree=0, level=2)
    lam0 = np.exp(-1j * k) * math.sin(k) / k
    v = S.density_pairing(0, 0, 8, 8)
    assert abs(v - 4 * math.pi * lam0) <= 1e-10 * 4 * math.pi
    lam1 = -1j * k * spherical_jn(1, k) * _h2(1, k)
    v = S.density_pairing(3, 3, 8, 8)
    assert abs(v - (4 * math.pi / 3) * lam1) <= 1e-10 * 4 * math.pi


# ---------------------------------------------------------------- Galerkin matrix invariants
def test_dense_symmetric_and_spd(c0):
    S, A = c0
    assert A.shape == (150, 150)
    assert np.abs(A - A.T).max() <= 1e-13 * np.abs(A).max()
    np.linalg.cholesky(0.5 * (A + A.T))


def test_helmholtz_complex_symmetric(orc):
    S = orc.Space(orc.SPHERE, [], orc.HELMHOLTZ, 3.1 + 0.2j, degree=1, level=1)
    A = S.dense(8, 8)
    assert np.iscomplexobj(A)
    assert np.abs(A - A.T).max() <= 1e-13 * np.abs(A).max()


def test_degree0_dense_equals_pair_blocks(orc):
    """For piecewise constants A[e1, e2] is exactly the pair integral of the two elements."""
    S = orc.Space(orc.SPHERE, [], orc.LAPLACE, 0, degree=0, level=1)
    A = S.dense(8, 8)
    rng = np.random.default_rng(2)
    for _ in range(10):
        e1, e2 = rng.integers(0, S.nelem, 2)
        assert A[e1, e2] == S.pair_block(int(e1), int(e2))[0, 0]


def test_self_convergence_of_quadrature(orc):
    """Duffy q_s=8 against q_s=16 and regular Gauss 8 against 20 on the curved cube sphere."""
    S = orc.Space(orc.SPHERE, [], orc.LAPLACE, 0, degree=1, level=1)
    for e2 in range(S.nelem):
        t = S.classify(0, e2)[0]
        B8 = S.pair_block(0, e2, 8, 8)
        Bf = S.pair_block(0, e2, 20, 16)
        assert np.abs(B8 - Bf).max() <= 1e-9 * np.abs(Bf).max(), (e2, t)


# ---------------------------------------------------------------- exterior Dirichlet (closed form + rate)
def test_exterior_dirichlet_c0(orc, c0):
    S, A = c0
    x0, pts = W.c0_inputs()
    b = S.rhs(orc.POINT_SOURCE, x0)
    rho = np.linalg.solve(A, b)
    u = S.potential(rho, pts)
    ex = 1.0 / (4 * math.pi * np.linalg.norm(pts - x0, axis=1))
    assert np.max(np.abs(u - ex)) / np.max(np.abs(ex)) < 2e-4


def test_convergence_order(orc, c0):
    """Potential error decays like h^(2d+3) (Fig. 1's 2P+1 orders): measured pre-asymptotic
    orders are above 2.7 for d=0 (L=1->2) and above 4.0 for d=1 (L=1->2)."""
    x0, pts = W.c0_inputs()
    ex = 1.0 / (4 * math.pi * np.linalg.norm(pts - x0, axis=1))

    def err(S, A=None):
        if A is None:
            A = S.dense(8, 8)
        rho = np.linalg.solve(A, S.rhs(orc.POINT_SOURCE, x0))
        return np.max(np.abs(S.potential(rho, pts) - ex)) / np.max(np.abs(ex))

    e01 = err(orc.Space(orc.SPHERE, [], orc.LAPLACE, 0, degree=0, level=1))
    e02 = err(orc.Space(orc.SPHERE, [], orc.LAPLACE, 0, degree=0, level=2))
    assert math.log2(e01 / e02) > 2.7
    e11 = err(orc.Space(orc.SPHERE, [], orc.LAPLACE, 0, degree=1, level=1))
    e12 = err(c0[0], c0[1])
    assert math.log2(e11 / e12) > 4.0


def test_exterior_dirichlet_helmholtz(orc):
    k = 2.0
    S = orc.Space(orc.SPHERE, [], orc.HELMHOLTZ, k, degree=1, level=1)
    A = S.dense(8, 8)
    x0, pts = W.c0_inputs()
    b = S.rhs(orc.POINT_SOURCE, x0)
    rho = np.linalg.solve(A, b)
    u = S.potential(rho, pts)
    r = np.linalg.norm(pts - x0, axis=1)
    ex = np.exp(-1j * k * r) / (4 * math.pi * r)
    assert np.max(np.abs(u - ex)) / np.max(np.abs(ex)) < 2e-2


def test_plane_wave_mie_series(orc):
    """Sound-soft sphere, incident exp(-i k d.x): the scattered field of the single-layer
    solution with data -u_inc equals minus the incident wave's partial-wave sum
    sum_l (2l+1)(-i)^l j_l(k) h2_l(k|x|)/h2_l(k) P_l(d.x^)."""
    from scipy.special import eval_legendre

    k = 2.0
    S = orc.Space(orc.SPHERE, [], orc.HELMHOLTZ, k, degree=1, level=2)
    A = S.dense(8, 8)
    d = np.array([0.3, -0.4, np.sqrt(1 - 0.25)])
    b = S.rhs(orc.PLANE_WAVE, d)  # data g = exp(-i k d.x)
    rho = np.linalg.solve(A, b)
    _, pts = W.c0_inputs()
    u = S.potential(rho, pts[:16])
    r = np.linalg.norm(pts[:16], axis=1)
    c = pts[:16] @ d / r
    ex = np.zeros(16, dtype=complex)
    for l in range(40):
        ex += (2 * l + 1) * (-1j) ** l * spherical_jn(l, k) * _h2(l, k * r) / _h2(l, k) * eval_legendre(l, c)
    assert np.max(np.abs(u - ex)) / np.max(np.abs(ex)) < 1e-3


# ---------------------------------------------------------------- H^2 special cases
def test_h2_eta0_is_dense(orc, c0):
    S, A = c0
    H = orc.H2(S, q=3, eta=0.0, leaf=2)
    assert H.nfar == 0 and H.nnear == S.nelem ** 2
    x = W.random_vector(W.rng(0, 1), S.ndof)
    y = H.apply(x)
    assert np.abs(y - A @ x).max() <= 1e-14 * np.abs(A @ x).max()


def test_h2_transfer_exact_and_counts(orc, c0):
    S, A = c0
    H = orc.H2(S, q=5, eta=1.6, leaf=2)
    # far and near counts of the ball rule with eta = 1.6 on the cube sphere at leaf level 2
    assert (H.nfar, H.nnear) == (6672, 2184)
    x = W.random_vector(W.rng(0, 2), S.ndof)
    m1, m2 = H.moments(x), H.moments(x, direct=True)
    assert np.abs(m1 - m2).max() <= 1e-14 * np.abs(m2).max()


def test_h2_error_decays_in_q(orc, c0):
    """The compression error decays geometrically in q at fixed eta (its value is pinned by
    test_h2_equals_its_definition)."""
    S, A = c0
    x = W.random_vector(W.rng(0, 3), S.ndof)
    ref = A @ x
    errs = []
    for q in (2, 3, 4, 5, 6):
        H = orc.H2(S, q=q, eta=1.6, leaf=2)
        errs.append(np.linalg.norm(H.apply(x) - ref) / np.linalg.norm(ref))
    assert all(e2 < 0.5 * e1 for e1, e2 in zip(errs, errs[1:]))
    assert errs[3] < 1e-6


def test_h2_apply_rows_matches_apply(orc, c0):
    S, _ = c0
    H = orc.H2(S, q=4, eta=1.6, leaf=1)
    Hl = orc.H2(S, q=4, eta=1.6, leaf=1, assemble_near=False)
    x = W.random_vector(W.rng(0, 4), S.ndof)
    rows = W.sample_rows(0, S.ndof, 12)
    np.testing.assert_allclose(Hl.apply_rows(x, rows), H.apply(x)[rows], rtol=0,
                               atol=1e-14 * np.abs(H.apply(x)).max())


def test_h2_near_pattern(orc, c0):
    S, _ = c0
    H = orc.H2(S, q=4, eta=1.6, leaf=2)
    rowptr, col, val = H.near_csr()
    assert rowptr[-1] == H.nnz
    assert np.all(np.diff(rowptr) > 0)
    # symmetric pattern and values (both triangles integrated independently)
    Ad = np.zeros((S.ndof, S.ndof))
    for r in range(S.ndof):
        Ad[r, col[rowptr[r]:rowptr[r + 1]]] = val[rowptr[r]:rowptr[r + 1]]
    assert np.abs(Ad - Ad.T).max() <= 1e-13 * np.abs(Ad).max()


# ---------------------------------------------------------------- GMRES (library)
def test_gmres_matches_numpy_solve(orc, c0):
    S, A = c0
    b = S.rhs(orc.POINT_SOURCE, W.CONFIGS[0]["x0"])
    x, it, rr, ok = orc.dense_gmres(A, b, tol=1e-13, restart=30)
    ref = np.linalg.solve(A, b)
    assert ok and rr <= 1e-13
    assert np.linalg.norm(x - ref) / np.linalg.norm(ref) <= 1e-10


def test_gmres_complex_matches_numpy_solve(orc):
    g = np.random.default_rng(11)
    n = 60
    A = np.eye(n) * 3 + (g.normal(size=(n, n)) + 1j * g.normal(size=(n, n))) / np.sqrt(n)
    b = g.normal(size=n) + 1j * g.normal(size=n)
    x, it, rr, ok = orc.dense_gmres(A, b, tol=1e-13, restart=10)
    ref = np.linalg.solve(A, b)
    assert ok and np.linalg.norm(x - ref) / np.linalg.norm(ref) <= 1e-11


def test_gmres_reports_nonconvergence(orc):
    g = np.random.default_rng(12)
    n = 50
    A = g.normal(size=(n, n))
    b = g.normal(size=n)
    x, it, rr, ok = orc.dense_gmres(A, b, tol=1e-12, restart=5, maxit=5)
    assert not ok and it == 5 and rr > 1e-12


def _h2_by_definition(orc, S, H, A, a, L, d, q, kernel):
    """The compressed operator written out from its definition (Sec. 2, embedded FMM on
    the unit square): the dense matrix with, on every far cluster pair (tau, sigma), the
    kernel replaced by its tensor Chebyshev interpolant on the two cluster squares,
    k(gamma(s), gamma(t)) ~ sum_ab L_a(s) k(gamma(xi_a), gamma(xi_b)) L_b(t).  Built from
    scratch here on a flat square gamma(s, t) = (a s, a t, 0): scipy B-splines, Gauss rules,
    Lagrange polynomials; the far part of the dense matrix is replaced by the interpolated
    one, each integrated with the 8-point Gauss rule per element direction."""
    nb, ne = 2 ** L + d, 2 ** L
    knots = np.r_[np.zeros(d), np.linspace(0.0, 1.0, ne + 1), np.ones(d)]
    xg, wg = np.polynomial.legendre.leggauss(8)
    xi = 0.5 * (1.0 + np.cos((2 * np.arange(q) + 1) * np.pi / (2 * q)))

    def basis(u):  # (len(u), nb)
        return np.stack([BSpline(knots, np.eye(nb)[j], d, extrapolate=False)(u) for j in range(nb)], axis=1)

    def lagrange(u, nodes):  # (len(u), q)
        out = np.ones((len(u), q))
        for k in range(q):
            for m in range(q):
                if m != k:
                    out[:, k] *= (u - nodes[m]) / (nodes[k] - nodes[m])
        return out

    def cluster(lev, i, j):
        w = 1.0 / (1 << lev)
        ee = (1 << L) >> lev  # elements per cluster direction
        u = np.concatenate([(e + 0.5 * (xg + 1.0)) / ne for e in range(i * ee, (i + 1) * ee)])
        v = np.concatenate([(e + 0.5 * (xg + 1.0)) / ne for e in range(j * ee, (j + 1) * ee)])
        wu = np.tile(0.5 * wg / ne, ee)
        U, Vv = np.meshgrid(u, v, indexing="ij")
        Wt = np.outer(wu, wu).ravel()
        Bu, Bv = basis(u), basis(v)
        Phi = np.einsum("ab,cd->acbd", Bu, Bv).reshape(len(u) * len(v), nb * nb)
        Lu, Lv = lagrange(u, i * w + xi * w), lagrange(v, j * w + xi * w)
        Lam = np.einsum("ab,cd->acbd", Lu, Lv).reshape(len(u) * len(v), q * q)
        pts = a * np.stack([U.ravel(), Vv.ravel(), np.zeros(U.size)], axis=1)
        nu, nv = np.meshgrid(i * w + xi * w, j * w + xi * w, indexing="ij")
        nodes = a * np.stack([nu.ravel(), nv.ravel(), np.zeros(q * q)], axis=1)
        return Phi, Wt, Lam, pts, nodes

    ids, _ = H.clusters()
    far, _ = H.lists()
    AH = A.astype(S.dtype).copy()
    for t, s in far:
        Pt, Wt, Lt, Xt, Nt = cluster(ids[t, 0], ids[t, 2], ids[t, 3])
        Ps, Ws, Ls, Xs, Ns = cluster(ids[s, 0], ids[s, 2], ids[s, 3])
        Kd = kernel(np.linalg.norm(Xt[:, None, :] - Xs[None, :, :], axis=2))
        Kn = kernel(np.linalg.norm(Nt[:, None, :] - Ns[None, :, :], axis=2))
        exact = (Pt * Wt[:, None]).T @ Kd @ (Ps * Ws[:, None])
        Vt, Vs = (Lt * Wt[:, None]).T @ Pt, (Ls * Ws[:, None]).T @ Ps
        AH += Vt.T @ Kn @ Vs - exact
    return AH, far


@pytest.mark.parametrize("pde,kappa", [(0, 0.0), (1, 2.5)])
def test_h2_equals_its_definition(orc, pde, kappa):
    """Pins the value of the compressed operator (not only its decay in q): the oracle's H2
    matvec equals the operator built from the definition on a flat square, L = 2, d = 1,
    q = 3, leaf level 2, eta = 1.6, to rounding, while differing from the dense matrix by
    the compression error."""
    a, L, d, q = 2.0, 2, 1, 3
    S = orc.Space(orc.FLAT, [a], pde, kappa, degree=d, level=L)
    H = orc.H2(S, q=q, eta=1.6, leaf=2)
    A = S.dense(8, 8)
    if pde == 0:
        kernel = lambda r: 1.0 / (4.0 * np.pi * r)
    else:
        kernel = lambda r: np.exp(-1j * kappa * r) / (4.0 * np.pi * r)
    AH, far = _h2_by_definition(orc, S, H, A, a, L, d, q, kernel)
    assert len(far) > 0 and {(t, s) for t, s in far} == {(s, t) for t, s in far}
    x = W.random_vector(W.rng(0, 40), S.ndof, is_complex=S.complex)
    y, yd, yh = H.apply(x), A @ x, AH @ x
    comp = np.linalg.norm(y - yd) / np.linalg.norm(yd)
    assert comp > 1e-6  # the far field really is approximated
    assert np.linalg.norm(y - yh) / np.linalg.norm(yh) <= 1e-13 * max(1.0, 1e3 * comp)
