"""CPU checks of the C ABI library: it loads, exports every function that include/bem.h
declares, validates its arguments, and its host plan (cluster tree, block partition, near
pattern) equals the oracle's.  No compute call touches a GPU here."""
import ctypes
import os

import numpy as np
import pytest

import workloads as W


@pytest.fixture(scope="module")
def B():
    import paper_1906_00785_amd as B

    return B


def test_exports_every_declared_symbol(B):
    names = B._bem.header_symbols()
    assert len(names) >= 20
    lib = ctypes.CDLL(B._bem.LIB_PATH)
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


def test_argument_validation(B):
    C = B._bem
    with pytest.raises(C.BemError) as e:
        B.Geometry(99)
    assert e.value.code == C.BEM_EINVAL
    with pytest.raises(C.BemError) as e:
        B.Geometry(B.BEM_GEOM_TORUS16, (0.3, 0.5))  # R < r
    assert e.value.code == C.BEM_EINVAL
    g = B.Geometry(B.BEM_GEOM_SPHERE6)
    for kw, code in [(dict(degree=-1), C.BEM_EINVAL), (dict(level=-1), C.BEM_EINVAL),
                     (dict(degree=1, knot_repetition=3), C.BEM_EINVAL),
                     (dict(degree=1, knot_repetition=0), C.BEM_EINVAL), (dict(degree=3), C.BEM_EUNSUPPORTED)]:
        with pytest.raises(C.BemError) as e:
            B.Space(g, B.BEM_LAPLACE_SINGLE, 0.0, **kw)
        assert e.value.code == code, kw
    with pytest.raises(C.BemError) as e:
        B.Space(g, B.BEM_HELMHOLTZ_SINGLE, 0.0, degree=1, level=1)  # kappa = 0
    assert e.value.code == C.BEM_EINVAL
    s = B.Space(g, B.BEM_LAPLACE_SINGLE, 0.0, degree=1, level=2)
    for q, eta, leaf in [(0, 1.6, 1), (5, -1.0, 1), (5, 1.6, 3), (9, 1.6, 1)]:
        with pytest.raises(C.BemError) as e:
            B.Operator(s, q=q, eta=eta, leaf_level=leaf, assemble=False)
        assert e.value.code == C.BEM_EINVAL
    # on-the-fly coupling excludes the stored low-precision copy and the many-RHS slabs
    for kw, code in [(dict(far_eval=True, far_low=1), C.BEM_EUNSUPPORTED),
                     (dict(far_eval=True, batch_rhs=8), C.BEM_EUNSUPPORTED)]:
        with pytest.raises(C.BemError) as e:
            B.Operator(s, q=5, eta=1.6, leaf_level=2, assemble=False, **kw)
        assert e.value.code == code, kw
    # the on-the-fly sine and cosine take Re(kappa) r < 2^20
    sh = B.Space(g, B.BEM_HELMHOLTZ_SINGLE, 5e5, degree=1, level=2)
    with pytest.raises(C.BemError) as e:
        B.Operator(sh, q=5, eta=1.6, leaf_level=2, assemble=False, far_eval=True)
    assert e.value.code == C.BEM_EUNSUPPORTED
    B.Operator(sh, q=5, eta=1.6, leaf_level=2, assemble=False)  # stored blocks: no bound
    Ao = B.Operator(s, q=5, eta=1.6, leaf_level=2, assemble=False, far_eval=True)
    Ast = B.Operator(s, q=5, eta=1.6, leaf_level=2, assemble=False)
    assert Ao.info.far_bytes == 0.0 and Ast.info.far_bytes > 0.0
    assert Ao.info.op_bytes < Ast.info.op_bytes
    A = B.Operator(s, q=5, eta=1.6, leaf_level=2, assemble=False)
    with pytest.raises(C.BemError):  # not assembled yet
        C.bem_apply(A.h, 1, A.ndof, 2, A.ndof, 1, 0)
    assert C.bem_operator_dims(A.h) == (150, 150)


def test_degenerate_sizes(B):
    g = B.Geometry(B.BEM_GEOM_SPHERE6)
    s = B.Space(g, B.BEM_LAPLACE_SINGLE, 0.0, degree=0, level=0)
    A = B.Operator(s, q=1, eta=1.6, leaf_level=0, assemble=False)
    assert A.info.ndof == 6 and A.info.nfar == 0 and A.info.nnear == 36
    assert A.info.ntouch == 6 + 24 + 0  # identical, edge; no vertex-only pairs at L=0
    s = B.Space(g, B.BEM_LAPLACE_SINGLE, 0.0, degree=2, knot_repetition=3, level=2)
    assert s.ndof == 6 * (3 + 3 * 3) ** 2


def _plan_lists(B, A):
    C = B._bem
    info = A.info
    pairs = np.zeros((info.nfar, 2), dtype=np.int64)
    C.bem_export_far(A.h, pairs.ctypes.data, 0, 0)
    rowptr = np.zeros(info.ndof + 1, dtype=np.int64)
    col = np.zeros(info.near_nnz, dtype=np.int32)
    C.bem_export_near(A.h, rowptr.ctypes.data, col.ctypes.data, 0, 0)
    return pairs, rowptr, col


@pytest.mark.parametrize("geom,prm,L,d,leaf,eta", [
    (0, (), 2, 1, 2, 1.6), (0, (), 2, 1, 1, 1.6), (2, (1.0, 0.4), 2, 1, 1, 1.6),
    (1, (0.7, 1.2, 1.6), 2, 2, 1, 1.6), (3, (2.0,), 2, 0, 1, 1.6), (0, (), 2, 1, 0, 0.0), (0, (), 1, 2, 1, 3.0),
])
def test_plan_equals_oracle(B, orc, geom, prm, L, d, leaf, eta):
    g = B.Geometry(geom, prm)
    s = B.Space(g, B.BEM_LAPLACE_SINGLE, 0.0, degree=d, level=L)
    A = B.Operator(s, q=4, eta=eta, leaf_level=leaf, assemble=False)
    pairs, rowptr, col = _plan_lists(B, A)
    So = orc.Space(geom, list(prm), orc.LAPLACE, 0.0, degree=d, level=L)
    Ho = orc.H2(So, q=4, eta=eta, leaf=leaf, assemble_near=(L <= 1 or (L == 2 and d <= 1 and leaf >= 1)))
    far, near = Ho.lists()
    assert np.array_equal(far, pairs)
    assert A.info.nnear == Ho.nnear
    if Ho.nnz:
        rp, cl, _ = Ho.near_csr()
        assert np.array_equal(rp, rowptr) and np.array_equal(cl, col)


def test_plan_counts_at_full_size(B, orc):
    """The benchmark workload's partition: far and near lists equal the oracle's."""
    c = W.CONFIGS[1]
    g = B.Geometry(B.BEM_GEOM_SPHERE6)
    s = B.Space(g, B.BEM_LAPLACE_SINGLE, 0.0, degree=c["degree"], level=c["level"])
    A = B.Operator(s, q=c["q"], eta=c["eta"], leaf_level=c["leaf"], assemble=False)
    pairs, rowptr, col = _plan_lists(B, A)
    So = orc.Space(orc.SPHERE, [], orc.LAPLACE, 0.0, degree=c["degree"], level=c["level"])
    Ho = orc.H2(So, q=c["q"], eta=c["eta"], leaf=c["leaf"], assemble_near=False)
    far, near = Ho.lists()
    assert np.array_equal(far, pairs)
    assert A.info.nfar == 143520 and A.info.nnear == Ho.nnear
    assert A.info.ndof == 26136
    # touching element pairs: identical + edge + vertex = nelem + 4 nelem + (4 nelem - 24)
    ne = 6 * 64 * 64
    assert A.info.ntouch == ne + 4 * ne + 4 * ne - 24


def test_bench_refuses_several_gpus():
    """bench.py measures one GPU; --gpus N > 1 exits with a message before touching a GPU."""
    import subprocess
    import sys

    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"], capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr


@pytest.mark.parametrize("kappa,kadm", [(4.0, 4.0), (12.0, 3.0), (6.0 + 1.0j, 2.5), (4.0, 0.0)])
def test_plan_equals_oracle_wavenumber_bound(B, orc, kappa, kadm):
    """Reading A12: with the wavenumber bound the far list equals the oracle's and is a
    subset of the unbounded one (pairs too wide for the wavenumber are refined)."""
    g = B.Geometry(B.BEM_GEOM_SPHERE6)
    s = B.Space(g, B.BEM_HELMHOLTZ_SINGLE, kappa, degree=1, level=3)
    A = B.Operator(s, q=4, eta=1.6, leaf_level=3, assemble=False, kappa_adm=kadm)
    pairs, _, _ = _plan_lists(B, A)
    So = orc.Space(orc.SPHERE, [], orc.HELMHOLTZ, kappa, degree=1, level=3)
    Ho = orc.H2(So, q=4, eta=1.6, leaf=3, assemble_near=False, kappa_adm=kadm)
    far, _ = Ho.lists()
    assert np.array_equal(far, pairs)
    A0 = B.Operator(s, q=4, eta=1.6, leaf_level=3, assemble=False)
    if kadm > 0:
        assert A.info.nnear >= A0.info.nnear
        # every far pair satisfies the bound: |kappa| times the larger cluster diameter; the
        # clusters of a level-l pair have diameters of order 2^-l, so the coarsest far level
        # moves down as the bound tightens
        lev_of = lambda c: int(np.searchsorted(np.cumsum([6 * 4 ** l for l in range(4)]), c, side="right"))
        assert min(lev_of(t) for t, _ in pairs) >= min(lev_of(t) for t, _ in _plan_lists(B, A0)[0])
    else:
        assert A.info.nfar == A0.info.nfar


def test_autotune_cache_key_separates_instances():
    """Two instances that differ only in a geometry parameter, the wavenumber, the knot
    repetition or the far-field mode get different cache entries."""
    from types import SimpleNamespace as NS

    import paper_1906_00785_amd.autotune as AT

    def sp(params=(1.0, 0.4), kappa=2.0, rep=1):
        return NS(geom=NS(kind=2, params=params), level=3, degree=2, knot_repetition=rep, kernel=1, kappa=kappa)

    base = AT.cache_key(sp(), 5, 1.6, 1, False, 0.0)
    others = [AT.cache_key(sp(params=(1.0, 0.45)), 5, 1.6, 1, False, 0.0),
              AT.cache_key(sp(kappa=2.5), 5, 1.6, 1, False, 0.0),
              AT.cache_key(sp(kappa=2.0 + 0.1j), 5, 1.6, 1, False, 0.0),
              AT.cache_key(sp(rep=2), 5, 1.6, 1, False, 0.0),
              AT.cache_key(sp(), 5, 1.6, 1, True, 0.0),
              AT.cache_key(sp(), 5, 1.6, 1, False, 6.0),
              AT.cache_key(sp(), 5, 1.6, 8, False, 0.0)]
    assert len(set(others + [base])) == len(others) + 1
    assert AT.cache_key(sp(), 5, 1.6, 1, False, 0.0) == base


# ---------------------------------------------------------------- NURBS geometries (host side)
def test_nurbs_plan_equals_oracle(B, orc):
    """The NURBS torus: the host plan (partition, near pattern) equals the oracle's."""
    patches = W.nurbs_torus(1.0, 0.4)
    g = B.Geometry.nurbs(patches)
    s = B.Space(g, B.BEM_LAPLACE_SINGLE, 0.0, degree=1, level=2)
    A = B.Operator(s, q=4, eta=1.6, leaf_level=1, assemble=False)
    pairs, rowptr, col = _plan_lists(B, A)
    So = orc.Space(orc.NURBS, patches, orc.LAPLACE, 0.0, degree=1, level=2)
    Ho = orc.H2(So, q=4, eta=1.6, leaf=1, assemble_near=False)
    far, _ = Ho.lists()
    assert np.array_equal(far, pairs) and A.info.nnear == Ho.nnear
    # touching element pairs on the closed torus: every vertex has valence 4
    ne = 16 * 4 * 4
    assert A.info.ntouch == ne + 4 * ne + 4 * ne


def test_nurbs_file_round_trip(B, tmp_path):
    """A NURBS geometry saved and loaded again plans the same operator; malformed files
    and tables are refused with EINVAL."""
    C = B._bem
    g = B.Geometry.nurbs(W.nurbs_torus(1.0, 0.3) + [])
    path = str(tmp_path / "torus.bemnurbs")
    g.save(path)
    g2 = B.Geometry.load(path)
    plans = []
    for gg in (g, g2):
        s = B.Space(gg, B.BEM_LAPLACE_SINGLE, 0.0, degree=1, level=2)
        plans.append(_plan_lists(B, B.Operator(s, q=4, eta=1.6, leaf_level=1, assemble=False)))
    for a, b in zip(*plans):
        assert np.array_equal(a, b)
    bad = tmp_path / "bad.bemnurbs"
    txt = open(path).read()
    for mutate in (lambda t: t.replace("BEMNURBS 1", "BEMNURBS 2"), lambda t: t[: len(t) // 2]):
        bad.write_text(mutate(txt))
        with pytest.raises(C.BemError) as e:
            B.Geometry.load(str(bad))
        assert e.value.code == C.BEM_EINVAL
    P = W.nurbs_torus(1.0, 0.3)[0]
    for change in ({"knots": ([0.0, 0.0, 0.5, 1.0, 1.0, 1.0], P["knots"][1])},  # not clamped
                   {"cw": np.concatenate([P["cw"][:, :, :3], -np.ones((3, 3, 1))], axis=2)}):  # weights
        with pytest.raises(C.BemError) as e:
            B.Geometry.nurbs([dict(P, **change)])
        assert e.value.code == C.BEM_EINVAL
    with pytest.raises(C.BemError) as e:
        B.Geometry(B.BEM_GEOM_SPHERE6).save(path)
    assert e.value.code == C.BEM_EINVAL


def test_user_map_plan_equals_oracle(B, orc):
    """A user map (the sphere's patch maps as a host callback): the library's interpolant
    plans the same partition as the oracle's reading of the same map, and a callback that
    returns non-finite points is refused."""
    C = B._bem
    g = B.Geometry.user(6, W.sphere6_map, degree=5, intervals=8)
    s = B.Space(g, B.BEM_LAPLACE_SINGLE, 0.0, degree=1, level=3)
    A = B.Operator(s, q=4, eta=1.6, leaf_level=2, assemble=False)
    pairs, _, _ = _plan_lists(B, A)
    So = orc.Space(orc.NURBS, orc.user_map_patches(W.sphere6_map, 6, 5, 8), orc.LAPLACE, 0.0, degree=1, level=3)
    Ho = orc.H2(So, q=4, eta=1.6, leaf=2, assemble_near=False)
    far, _ = Ho.lists()
    assert np.array_equal(far, pairs) and A.info.nnear == Ho.nnear
    with pytest.raises(C.BemError) as e:
        B.Geometry.user(1, lambda f, st: np.full((st.shape[0], 3), np.nan), degree=3, intervals=4)
    assert e.value.code == C.BEM_EINVAL


def _read_vtk(path):
    """Minimal reader of the legacy ASCII unstructured grid the library writes."""
    tok = open(path).read().split("\n")
    i = tok.index("DATASET UNSTRUCTURED_GRID") + 1
    n = int(tok[i].split()[1])
    pts = np.array([[float(v) for v in tok[i + 1 + k].split()] for k in range(n)])
    i += 1 + n
    nc = int(tok[i].split()[1])
    cells = np.array([[int(v) for v in tok[i + 1 + k].split()] for k in range(nc)])
    i += 1 + nc
    types = np.array([int(tok[i + 1 + k]) for k in range(nc)])
    i += 1 + nc
    data = {}
    assert tok[i].startswith("POINT_DATA")
    i += 1
    while i < len(tok) and tok[i].startswith("SCALARS"):
        name = tok[i].split()[1]
        data[name] = np.array([float(tok[i + 2 + k]) for k in range(n)])
        i += 2 + n
    return pts, cells, types, data


@pytest.mark.parametrize("geom,prm,pde,kappa", [(0, (), 0, 0.0), (2, (1.0, 0.4), 1, 2.0)])
def test_vtk_output_matches_oracle_geometry_and_density(B, orc, tmp_path, geom, prm, pde, kappa):
    """Points are gamma at the stated parameters, kappa the surface element, and the density
    rho_hat / kappa with rho_hat = sum_g rho_g b_j1(s) b_j2(t), all against the oracle's maps,
    surface elements and B-splines (App. C)."""
    L, d, nsub = 1, 2, 3
    g = B.Geometry(geom, prm)
    s = B.Space(g, pde, kappa, degree=d, level=L)
    rho = W.random_vector(W.rng(9, 40), s.ndof, is_complex=bool(pde), ncols=2).T.copy()
    path = str(tmp_path / "out.vtk")
    s.write_vtk(path, torch_free(rho), nsub=nsub)
    pts, cells, types, data = _read_vtk(path)
    np1 = nsub + 1
    nel = 1 << L
    assert pts.shape == (s.ndof // (nel + d) ** 2 * nel * nel * np1 * np1, 3)
    assert cells.shape[1] == 5 and np.all(cells[:, 0] == 4) and np.all(types == 9)
    So = orc.Space(geom, list(prm), pde, kappa, degree=d, level=L)
    nb = nel + d
    k = 0
    for e in range(So.nelem):
        f, i1, i2 = e // (nel * nel), (e // nel) % nel, e % nel
        st = np.array([[(i1 + a / nsub) / nel, (i2 + b / nsub) / nel] for a in range(np1) for b in range(np1)])
        xyz, kap, _ = So.gamma(f, st)
        np.testing.assert_allclose(pts[k:k + np1 * np1], xyz, rtol=0, atol=1e-14)
        np.testing.assert_allclose(data["kappa"][k:k + np1 * np1], kap, rtol=1e-8)
        B1 = np.stack([orc.bspline(d, 1, L, j, st[:, 0]) for j in range(nb)], 1)
        B2 = np.stack([orc.bspline(d, 1, L, j, st[:, 1]) for j in range(nb)], 1)
        for r in range(2):
            c = rho[r].reshape(-1, nb, nb)[f]
            rh = np.einsum("pi,pj,ij->p", B1, B2, c) / kap
            if pde:
                np.testing.assert_allclose(data[f"rho_re_{r}"][k:k + np1 * np1], rh.real, rtol=1e-7, atol=1e-12)
                np.testing.assert_allclose(data[f"rho_im_{r}"][k:k + np1 * np1], rh.imag, rtol=1e-7, atol=1e-12)
            else:
                np.testing.assert_allclose(data[f"rho_{r}"][k:k + np1 * np1], rh, rtol=1e-7, atol=1e-12)
        k += np1 * np1


def torch_free(a):
    import torch

    return torch.from_numpy(np.ascontiguousarray(a))


@pytest.mark.parametrize("geom,prm,d,L", [(0, (), 1, 2), (0, (), 2, 3), (2, (1.0, 0.4), 2, 2), (1, (0.8, 1.1, 1.3), 1, 1),
                                          (3, (1.7,), 2, 2)])
def test_s0_gluing_equals_oracle(B, orc, geom, prm, d, L):
    """The host gluing of a continuous space (App. E) equals the oracle's map, function by
    function, and its count is the space's N."""
    g = B.Geometry(geom, prm)
    s = B.Space(g, B.BEM_LAPLACE_SINGLE, 0.0, degree=d, level=L, continuous=True)
    So = orc.Space(geom, list(prm), orc.LAPLACE, 0.0, degree=d, level=L, form=0)
    m, n = So.glue()
    assert s.ndof == n and np.array_equal(s.glue(), m.astype(np.int32))
    A = B.Operator(s, q=4, eta=1.6, leaf_level=min(L, 1), assemble=False)
    assert A.ndof == n and A.info.nlocal == So.ndof
    # the discontinuous space of the same geometry: the identity map
    s2 = B.Space(g, B.BEM_LAPLACE_SINGLE, 0.0, degree=d, level=L)
    assert s2.ndof == So.ndof and np.array_equal(s2.glue(), np.arange(So.ndof, dtype=np.int32))


def test_s0_nurbs_gluing_equals_oracle(B, orc):
    g = B.Geometry.nurbs(W.nurbs_torus(1.0, 0.4))
    s = B.Space(g, B.BEM_LAPLACE_SINGLE, 0.0, degree=2, level=2, continuous=True)
    So = orc.Space(4, W.nurbs_torus(1.0, 0.4), orc.LAPLACE, 0.0, degree=2, level=2, form=0)
    m, n = So.glue()
    assert s.ndof == n == 16 * 4 ** 2 + 32 * 4 + 16 and np.array_equal(s.glue(), m.astype(np.int32))


def test_s0_argument_validation(B):
    C = B._bem
    g = B.Geometry(B.BEM_GEOM_SPHERE6)
    with pytest.raises(C.BemError) as e:
        B.Space(g, B.BEM_LAPLACE_SINGLE, 0.0, degree=0, level=2, continuous=True)
    assert e.value.code == C.BEM_EINVAL
    h = ctypes.c_void_p()
    assert C.lib.bem_space_create_ex(g.h, 0, 0.0, 0.0, 1, 1, 2, 7, ctypes.byref(h)) == C.BEM_EINVAL
    s = B.Space(g, B.BEM_LAPLACE_SINGLE, 0.0, degree=1, level=2, continuous=True)
    for kw in (dict(far_low=1), dict(far_low=2), dict(batch_rhs=8)):
        with pytest.raises(C.BemError) as e:
            B.Operator(s, q=4, eta=1.6, leaf_level=1, assemble=False, **kw)
        assert e.value.code == C.BEM_EUNSUPPORTED, kw
    B.Operator(s, q=4, eta=1.6, leaf_level=1, assemble=False, far_eval=True)


def test_vtk_output_of_a_continuous_density(B, orc, tmp_path):
    """S^0: the density written is rho_hat = sum over local functions of the coefficient of
    their global function times the B-splines (no division by kappa), and it is continuous:
    points shared by neighbouring patches carry the same value."""
    L, d, nsub = 1, 2, 2
    g = B.Geometry(B.BEM_GEOM_SPHERE6)
    s = B.Space(g, B.BEM_LAPLACE_SINGLE, 0.0, degree=d, level=L, continuous=True)
    rho = W.random_vector(W.rng(9, 41), s.ndof)
    path = str(tmp_path / "s0.vtk")
    s.write_vtk(path, torch_free(rho), nsub=nsub)
    pts, cells, types, data = _read_vtk(path)
    So = orc.Space(orc.SPHERE, [], orc.LAPLACE, 0.0, degree=d, level=L, form=0)
    m, _ = So.glue()
    nel, nb, np1 = 1 << L, (1 << L) + d, nsub + 1
    k = 0
    for e in range(So.nelem):
        f, i1, i2 = e // (nel * nel), (e // nel) % nel, e % nel
        st = np.array([[(i1 + a / nsub) / nel, (i2 + b / nsub) / nel] for a in range(np1) for b in range(np1)])
        B1 = np.stack([orc.bspline(d, 1, L, j, st[:, 0]) for j in range(nb)], 1)
        B2 = np.stack([orc.bspline(d, 1, L, j, st[:, 1]) for j in range(nb)], 1)
        c = rho[m].reshape(-1, nb, nb)[f]
        np.testing.assert_allclose(data["rho_0"][k:k + np1 * np1], np.einsum("pi,pj,ij->p", B1, B2, c), rtol=1e-12,
                                   atol=1e-13)
        k += np1 * np1
    # continuity: equal points, equal values
    order = np.lexsort(np.round(pts, 9).T)
    ps, vs = pts[order], data["rho_0"][order]
    same = np.all(np.abs(np.diff(ps, axis=0)) <= 1e-12, axis=1)
    assert same.sum() > 0
    assert np.max(np.abs(np.diff(vs)[same])) <= 1e-12 * np.max(np.abs(vs))


@pytest.mark.parametrize("geom,prm,p,L", [(0, (), 1, 0), (0, (), 2, 1), (0, (), 1, 2), (1, (0.8, 1.1, 1.3), 2, 1),
                                          (2, (1.0, 0.4), 1, 1), (2, (1.0, 0.4), 2, 1), (3, (1.7,), 1, 1),
                                          (3, (1.7,), 2, 2)])
def test_s1_gluing_equals_oracle(B, orc, geom, prm, p, L):
    """The host gluing of a div-conforming space (App. E: normal continuity across patch
    edges, dropped edge functions on open surfaces) equals the oracle's, map and signs."""
    g = B.Geometry(geom, prm)
    s = B.Space(g, B.BEM_MAXWELL_SINGLE, 1.5, degree=p, level=L)
    So = orc.MSpace(geom, list(prm), 1.5, p=p, level=L)
    m, sg = So.glue()
    assert s.ndof == So.nglob
    assert np.array_equal(s.glue(), m.astype(np.int32)) and np.array_equal(s.glue_sign(), sg)
    A = B.Operator(s, qg=6, qs=5, assemble=False)
    assert A.ndof == So.nglob and A.info.nlocal == So.nloc
    # the touching element pairs are those of the scalar near field at the finest leaf level
    s2 = B.Space(g, B.BEM_HELMHOLTZ_SINGLE, 1.5, degree=0, level=L)
    A2 = B.Operator(s2, q=3, eta=1.6, leaf_level=L, assemble=False)
    assert A.info.ntouch == A2.info.ntouch and A.info.nnear == (s2.ndof) ** 2
    assert A.info.op_bytes >= 16 * So.nglob ** 2


def test_s1_nurbs_gluing_equals_oracle(B, orc):
    g = B.Geometry.nurbs(W.nurbs_torus(1.0, 0.4))
    s = B.Space(g, B.BEM_MAXWELL_SINGLE, 1.5, degree=2, level=1)
    So = orc.MSpace(4, W.nurbs_torus(1.0, 0.4), 1.5, p=2, level=1)
    m, sg = So.glue()
    assert s.ndof == So.nglob == 16 * 2 * 4 * 3 - 32 * 3
    assert np.array_equal(s.glue(), m.astype(np.int32)) and np.array_equal(s.glue_sign(), sg)


def test_s1_argument_validation(B, tmp_path):
    C = B._bem
    g = B.Geometry(B.BEM_GEOM_SPHERE6)
    h = ctypes.c_void_p()
    # kernel and space kind go together
    assert C.lib.bem_space_create_ex(g.h, 2, 1.0, 0.0, 1, 1, 1, C.BEM_SPACE_S2, ctypes.byref(h)) == C.BEM_EINVAL
    assert C.lib.bem_space_create_ex(g.h, 1, 1.0, 0.0, 1, 1, 1, C.BEM_SPACE_S1, ctypes.byref(h)) == C.BEM_EINVAL
    for kw, code in [(dict(degree=0), C.BEM_EINVAL), (dict(degree=3), C.BEM_EUNSUPPORTED),
                     (dict(degree=2, knot_repetition=2), C.BEM_EUNSUPPORTED), (dict(kappa=0.0), C.BEM_EINVAL)]:
        args = dict(kappa=1.5, degree=1, level=1)
        args.update(kw)
        with pytest.raises(C.BemError) as e:
            B.Space(g, B.BEM_MAXWELL_SINGLE, **args)
        assert e.value.code == code, kw
    s = B.Space(g, B.BEM_MAXWELL_SINGLE, 1.5, degree=1, level=1)
    for kw, code in [(dict(eta=-1.0), C.BEM_EINVAL), (dict(eta=1.6, q=9), C.BEM_EINVAL),
                     (dict(eta=1.6, leaf_level=2), C.BEM_EINVAL), (dict(far_low=1), C.BEM_EUNSUPPORTED),
                     (dict(batch_rhs=8), C.BEM_EUNSUPPORTED), (dict(far_eval=True), C.BEM_EUNSUPPORTED),
                     (dict(qg=9), C.BEM_EINVAL), (dict(qs=0), C.BEM_EINVAL)]:
        with pytest.raises(C.BemError) as e:
            B.Operator(s, assemble=False, **kw)
        assert e.value.code == code, kw
    A = B.Operator(s, assemble=False)
    Ah = B.Operator(s, eta=1.6, q=3, assemble=False)  # compressed: the same operations are unsupported
    assert Ah.info.leaf_level == 0  # default leaf level L - 1
    n64, sz = ctypes.c_int64(), ctypes.c_size_t()
    for call in (lambda: C.check(C.lib.bem_export_near(A.h, None, None, None, None)),
                 lambda: C.check(C.lib.bem_export_far(A.h, None, None, None)),
                 lambda: C.check(C.lib.bem_precond_info(A.h, ctypes.byref(n64), ctypes.byref(sz))),
                 lambda: s.write_vtk(str(tmp_path / "s1.vtk")),
                 lambda: C.check(C.lib.bem_rhs_quadpoints(s.h, None, ctypes.byref(ctypes.c_int64()), None)),
                 lambda: C.check(C.lib.bem_profile_enable(A.h, 1)),
                 lambda: C.check(C.lib.bem_apply_stage(A.h, 0, 0, ctypes.c_void_p(8), ctypes.c_void_p(8), None))):
        with pytest.raises(C.BemError) as e:
            call()
        assert e.value.code in (C.BEM_EUNSUPPORTED, C.BEM_EINVAL)
    # scalar spaces: all signs +1
    s2 = B.Space(g, B.BEM_LAPLACE_SINGLE, 0.0, degree=1, level=1, continuous=True)
    assert (s2.glue_sign() == 1).all() and s2.glue_sign().size == C.bem_space_glue(s2.h)[0]


@pytest.mark.parametrize("geom,prm,p,L,q,leaf", [(0, (), 2, 2, 5, 2), (2, (1.0, 0.4), 1, 2, 4, 1), (3, (1.7,), 2, 3, 3, 2)])
def test_s1_compressed_partition_equals_oracle(B, orc, geom, prm, p, L, q, leaf):
    """The compressed S^1 operator plans on the block partition of the scalar operators of
    the same surface: far and near counts equal the oracle's scalar partition."""
    g = B.Geometry(geom, prm)
    s = B.Space(g, B.BEM_MAXWELL_SINGLE, 1.5, degree=p, level=L)
    A = B.Operator(s, q=q, eta=1.6, leaf_level=leaf, assemble=False)
    Ho = orc.H2(orc.Space(geom, list(prm), orc.HELMHOLTZ, 1.5, degree=0, level=L), q=q, eta=1.6, leaf=leaf,
                assemble_near=False)
    nl = 2 * p * (p + 1)
    m = 1 << (L - leaf)
    assert (A.info.nfar, A.info.nnear, A.info.nclusters) == (Ho.nfar, Ho.nnear, Ho.nclusters)
    assert A.info.near_nnz == Ho.nnear * m ** 4 * nl * nl and A.info.leaf_level == leaf
