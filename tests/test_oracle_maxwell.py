"""Pins of the oracle's Maxwell single layer (App. A (MP), App. B (MS)) on the
div-conforming spaces S^1 (App. E) against facts outside the Maxwell code.

- Glued counts: every patch edge of a closed surface glues its nbq edge functions in pairs
  (cube-sphere: 12 edges, torus: 32); on an open surface (flat square) they are dropped.
- Normal continuity: at the midpoint of every element edge on a patch boundary the normal
  component of each glued global function is the same from both sides (geometry: the two
  patches evaluated at the same point, the edge normal from the surface normal).
- The divergence term equals -kappa^-2 D^T V D with V the Helmholtz single-layer matrix of
  the S^2 space of degree p - 1 (the scalar oracle, pinned on its own) and D the B-spline
  derivative identity of App. C mapping S^1 coefficients to S^2 coefficients.
- The data field of a point dipole solves (MP): curl curl E = kappa^2 E and div E = 0
  (central differences); the field (MS) of a random density solves it too, which fixes the
  sign of its gradient term and needs the glued divergences (integration by parts on the
  closed surface).
- Complex symmetry of the Galerkin matrix.
- Exterior problem: the field of the solved density reproduces the dipole's field outside
  the sphere, converging with order about 3 for p = 1 and about 5 for p = 2 (Fig. 1 reports
  orders 3, 5 and 7 for P = 1, 2, 3).
- The compressed form (the far field of the scalar H^2 partition interpolated, four
  channels): with eta = 0 it is the Galerkin matrix; its error against the Galerkin matrix
  decays geometrically in q (Sec. 2); its divergence channel is -kappa^-2 D^T H D with H the
  scalar oracle's H^2 matrix of the S^2 space of degree p - 1 (pinned on its own).
All run on the CPU.
"""
import numpy as np
import pytest

import workloads as W

KAPPA = 1.5  # below the first interior resonance of the unit sphere (about 2.74)
X0 = [0.1, 0.2, -0.1]
MOM = (np.array([0.3, -0.5, 1.0]) / np.linalg.norm([0.3, -0.5, 1.0])).tolist()


def exterior_points(n, seed):
    return W.exterior_points(W.rng(9, seed), n, 2.0, 4.0)


@pytest.mark.parametrize("p,L", [(1, 0), (1, 2), (2, 1), (3, 1)])
def test_glued_counts(orc, p, L):
    nbp, nbq = (1 << L) + p, (1 << L) + p - 1
    S = orc.MSpace(orc.SPHERE, [], KAPPA, p=p, level=L)
    g, sg = S.glue()
    assert S.nloc == 6 * 2 * nbp * nbq and S.nglob == S.nloc - 12 * nbq
    assert (g >= 0).all() and set(np.unique(sg)) <= {-1, 1}
    assert np.array_equal(np.bincount(g), np.where(np.arange(S.nglob) >= 0, np.bincount(g), 0))
    assert np.bincount(g).max() == 2
    T = orc.MSpace(orc.TORUS, [1.0, 0.4], KAPPA, p=p, level=L)
    assert T.nglob == 16 * 2 * nbp * nbq - 32 * nbq
    F = orc.MSpace(orc.FLAT, [1.0], KAPPA, p=p, level=L)
    gf, sf = F.glue()
    assert F.nglob == 2 * nbp * nbq - 4 * nbq and (gf < 0).sum() == 4 * nbq and (sf[gf < 0] == 0).all()


def test_normal_component_is_continuous(orc):
    p, L = 2, 1
    S = orc.MSpace(orc.SPHERE, [], KAPPA, p=p, level=L)
    Ssc = orc.Space(orc.SPHERE, [], orc.HELMHOLTZ, KAPPA, degree=0, level=L)
    g, sg = S.glue()
    n = 1 << L
    h = 1.0 / n

    def edge_points(f):
        """(element, s, t, point) at the midpoints of the element edges on patch f's boundary."""
        out = []
        for i in range(n):
            m = (i + 0.5) * h
            for (s, t, i1, i2) in ((0.0, m, 0, i), (1.0, m, n - 1, i), (m, 0.0, i, 0), (m, 1.0, i, n - 1)):
                e = (f * n + i1) * n + i2
                x, _, _ = Ssc.gamma(f, [[s, t]])
                out.append((e, s, t, x[0]))
        return out

    pts = {f: edge_points(f) for f in range(6)}
    checked = 0
    for f in range(6):
        for (e, s, t, x) in pts[f]:
            # the same point on the neighbouring patch
            match = [(f2, e2, s2, t2) for f2 in range(6) if f2 != f for (e2, s2, t2, x2) in pts[f2]
                     if np.linalg.norm(x2 - x) < 1e-12]
            assert len(match) == 1
            f2, e2, s2, t2 = match[0]
            xa, Va, _, la = S.elem_eval(e, s, t)
            xb, Vb, _, lb = S.elem_eval(e2, s2, t2)
            _, ka, nrm = Ssc.gamma(f, [[s, t]])
            _, kb, _ = Ssc.gamma(f2, [[s2, t2]])
            # edge tangent: the parametric direction along the edge
            d = 1e-6
            st2 = [[s, t + d]] if s in (0.0, 1.0) else [[s + d, t]]
            xn, _, _ = Ssc.gamma(f, st2)
            tau = (xn[0] - x) / d
            nu = np.cross(tau, nrm[0])
            nu /= np.linalg.norm(nu)
            for G in np.unique(g[la]):
                ja = sum((sg[l] * Va[k] for k, l in enumerate(la) if g[l] == G), np.zeros(3)) / ka[0]
                jb = sum((sg[l] * Vb[k] for k, l in enumerate(lb) if g[l] == G), np.zeros(3)) / kb[0]
                assert abs(ja @ nu - jb @ nu) <= 1e-6 * max(1.0, abs(ja @ nu)), (f, f2, G)
                checked += 1
    assert checked > 100


def divergence_map(S, p, L, nrows):
    """D: glued S^1 coefficients -> coefficients of the S^2 space of degree p - 1 of their
    surface divergences (times the surface element), from the B-spline derivative identity:
    on the degree-p knots d/dx b^p_j = p b^{p-1}_j / (xi_{j+p} - xi_j)
    - p b^{p-1}_{j+1} / (xi_{j+p+1} - xi_{j+1}), the degree-(p-1) functions of the degree-p
    knots being those of the truncated knots shifted by one index (App. C, App. E)."""
    g, sg = S.glue()
    nbp, nbq = (1 << L) + p, (1 << L) + p - 1
    xi = np.concatenate([np.zeros(p + 1), np.arange(1, 1 << L) / (1 << L), np.ones(p + 1)])

    def dcoef(j):
        """derivative of b^p_j as {truncated-knot index: coefficient}"""
        out = {}
        if xi[j + p] > xi[j]:
            out[j - 1] = p / (xi[j + p] - xi[j])
        if xi[j + p + 1] > xi[j + 1]:
            out[j] = out.get(j, 0.0) - p / (xi[j + p + 1] - xi[j + 1])
        return {k: v for k, v in out.items() if 0 <= k < nbq}

    D = np.zeros((nrows, S.nglob))
    per = nbp * nbq
    for f in range(6):
        for c in range(2):
            for a in range(nbp):
                for b in range(nbq):
                    # a: index of the degree-p factor, b: of the degree-(p-1) factor
                    lid = (f * 2 + c) * per + (a * nbq + b if c == 0 else b * nbp + a)
                    for k, v in dcoef(a).items():
                        j1, j2 = (k, b) if c == 0 else (b, k)
                        D[(f * nbq + j1) * nbq + j2, g[lid]] += sg[lid] * v
    return D


@pytest.mark.parametrize("p,L", [(1, 1), (2, 1)])
def test_divergence_term_is_the_scalar_single_layer_of_the_divergences(orc, p, L):
    S = orc.MSpace(orc.SPHERE, [], KAPPA, p=p, level=L)
    Md = S.dense(part=2)
    V = orc.Space(orc.SPHERE, [], orc.HELMHOLTZ, KAPPA, degree=p - 1, level=L).dense()
    D = divergence_map(S, p, L, V.shape[0])
    ref = -(D.T @ V @ D) / KAPPA ** 2
    assert np.max(np.abs(Md - ref)) <= 1e-12 * np.max(np.abs(ref))


# ---- the compressed form (Sec. 2 interpolation on the scalar block partition)

def test_compressed_form_without_admissible_blocks_is_the_galerkin_matrix(orc):
    """eta = 0 admits no block: every element pair keeps its Galerkin block."""
    S = orc.MSpace(orc.TORUS, [1.0, 0.4], KAPPA, p=2, level=1)
    M = S.dense(qg=6, qs=5)
    H = S.h2_dense(q=3, eta=0.0, leaf=1, qg=6, qs=5)
    assert np.max(np.abs(H - M)) <= 1e-14 * np.max(np.abs(M))


@pytest.mark.parametrize("p,L,leaf", [(1, 2, 2), (2, 1, 1)])
def test_compressed_form_converges_geometrically_in_q(orc, p, L, leaf):
    """The interpolation error of an analytic kernel on admissible blocks decays
    geometrically with the number of Chebyshev nodes (Sec. 2): the compressed matrix tends
    to the pinned Galerkin matrix, more than an order of magnitude per two more nodes."""
    S = orc.MSpace(orc.SPHERE, [], KAPPA, p=p, level=L)
    M = S.dense()
    errs = [np.max(np.abs(S.h2_dense(q=q, eta=1.6, leaf=leaf) - M)) / np.max(np.abs(M)) for q in (2, 4, 6)]
    print(f"p = {p}: compressed-form errors for q = 2, 4, 6: {errs}")
    assert errs[0] / errs[1] >= 20 and errs[1] / errs[2] >= 20 and errs[2] <= 1e-6


def test_compressed_divergence_term_is_the_scalar_compressed_operator(orc):
    """The divergence channel of the compressed form is the scalar H^2 operator of the
    divergences: -kappa^-2 D^T H D with H the oracle's own (separately pinned) H^2 matrix of
    the S^2 space of degree p - 1 on the same partition; both moment rules are exact for
    these polynomial integrands, so the two agree to rounding."""
    p, L, q, leaf = 2, 1, 4, 1
    S = orc.MSpace(orc.SPHERE, [], KAPPA, p=p, level=L)
    Md = S.h2_dense(q=q, eta=1.6, leaf=leaf, part=2)
    Sc = orc.Space(orc.SPHERE, [], orc.HELMHOLTZ, KAPPA, degree=p - 1, level=L)
    Hs = orc.H2(Sc, q=q, eta=1.6, leaf=leaf)
    assert Hs.nfar > 0
    Hm = Hs.apply(np.eye(Sc.ndof, dtype=np.complex128))
    D = divergence_map(S, p, L, Sc.ndof)
    ref = -(D.T @ Hm @ D) / KAPPA ** 2
    assert np.max(np.abs(Md - ref)) <= 1e-12 * np.max(np.abs(ref))
    # and it is not the uncompressed term (the far field is really replaced)
    assert np.max(np.abs(Md - S.dense(part=2))) >= 1e-8 * np.max(np.abs(ref))


def curl_curl_residual(field, x, kappa, d=1e-3):
    """|curl curl E - kappa^2 E| and |div E| at x by central differences of E."""
    def E(y):
        return field(np.asarray(y).reshape(1, 3))[0]

    J = np.zeros((3, 3), dtype=complex)  # J[i, k] = d E_i / d x_k
    H = np.zeros((3, 3, 3), dtype=complex)  # H[i, k, l] = d2 E_i / dx_k dx_l
    e = np.eye(3) * d
    E0 = E(x)
    for k in range(3):
        J[:, k] = (E(x + e[k]) - E(x - e[k])) / (2 * d)
        for l in range(3):
            H[:, k, l] = (E(x + e[k] + e[l]) - E(x + e[k] - e[l]) - E(x - e[k] + e[l]) + E(x - e[k] - e[l])) / (4 * d * d)
    grad_div = np.array([sum(H[k, k, i] for k in range(3)) for i in range(3)])
    lap = np.array([sum(H[i, k, k] for k in range(3)) for i in range(3)])
    cc = grad_div - lap  # curl curl E
    return np.abs(cc - kappa ** 2 * E0).max() / (kappa ** 2 * np.abs(E0).max()), abs(np.trace(J)) / np.abs(J).max()


def test_dipole_field_solves_the_wave_equation(orc):
    for x in exterior_points(4, 70):
        r, dv = curl_curl_residual(lambda y: orc.m_field(orc.DIPOLE, X0 + MOM, KAPPA, y), x, KAPPA)
        assert r <= 1e-5 and dv <= 1e-5


def test_single_layer_field_solves_the_wave_equation(orc):
    S = orc.MSpace(orc.SPHERE, [], KAPPA, p=1, level=1)
    rng = W.rng(9, 71)
    j = rng.normal(size=S.nglob) + 1j * rng.normal(size=S.nglob)
    for x in exterior_points(3, 72):
        r, dv = curl_curl_residual(lambda y: S.potential(j, y), x, KAPPA)
        assert r <= 1e-5 and dv <= 1e-5


def test_galerkin_matrix_is_complex_symmetric(orc):
    for p in (1, 2):
        M = orc.MSpace(orc.ELLIPSOID, [0.8, 1.1, 1.3], KAPPA, p=p, level=1).dense()
        assert np.max(np.abs(M - M.T)) <= 1e-13 * np.max(np.abs(M))


@pytest.mark.parametrize("p,levels,rate,bar", [(1, (1, 2), 6.0, 1e-2), (2, (0, 1), 3.0, 2e-2)])
def test_exterior_dipole_problem_converges(orc, p, levels, rate, bar):
    pts = exterior_points(20, 73)
    ex = orc.m_field(orc.DIPOLE, X0 + MOM, KAPPA, pts)
    errs = []
    for L in levels:
        S = orc.MSpace(orc.SPHERE, [], KAPPA, p=p, level=L)
        j = np.linalg.solve(S.dense(), S.rhs(orc.DIPOLE, X0 + MOM))
        E = S.potential(j, pts)
        errs.append(np.abs(E - ex).max() / np.abs(ex).max())
    print(f"p = {p}: field errors {errs}")
    assert errs[-1] <= bar and errs[0] / errs[-1] >= rate
