"""GPU: mixed-precision far field and FP64 iterative refinement.

The low-precision coupling (blocks in FP32 or BF16, FP32 accumulation) is not a parity
quantity by itself: its error against the FP64 operator is stated and bounded here.  The
refined solve is: its solution must lie within 1e-8 (relative) of the FP64 oracle's
solution of the same H^2 system, and its FP64 residual must meet the tolerance.
"""
import numpy as np
import pytest
import torch

import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def B():
    import paper_1906_00785_amd as B

    return B


CASES = {
    # id: (geom, params, pde, kappa, L, d, q, eta, leaf)
    "sphere_L2_d1_laplace": (0, (), 0, 0.0, 2, 1, 5, 1.6, 2),
    "sphere_L2_d1_helmholtz": (0, (), 1, 2.5, 2, 1, 5, 1.6, 2),
    "torus_L2_d1_laplace": (2, (1.0, 0.4), 0, 0.0, 2, 1, 4, 1.6, 1),
}
# stated bounds of the low-precision matvec against the FP64 matvec (max-norm relative)
LOW_BOUND = {1: 1e-5, 2: 2e-2}

_cache = {}


def case(B, orc, cid, low):
    key = (cid, low)
    if key not in _cache:
        geom, prm, pde, kappa, L, d, q, eta, leaf = CASES[cid]
        print(f"[case {cid} far_low={low}] assemble", flush=True)
        g = B.Geometry(geom, prm)
        s = B.Space(g, pde, kappa, degree=d, level=L)
        A = B.Operator(s, q=q, eta=eta, leaf_level=leaf, far_low=low)
        if cid not in _cache:
            So = orc.Space(geom, list(prm), pde, kappa, degree=d, level=L)
            _cache[cid] = (So, orc.H2(So, q=q, eta=eta, leaf=leaf))
        _cache[key] = (g, s, A)
    return _cache[key] + _cache[cid]


@pytest.mark.parametrize("low", [1, 2])
@pytest.mark.parametrize("cid", list(CASES))
def test_low_precision_apply_error_is_bounded(B, orc, cid, low):
    g, s, A, So, Ho = case(B, orc, cid, low)
    x = torch.from_numpy(W.random_vector(W.rng(0, 40), s.ndof, is_complex=So.complex)).cuda()
    y64 = A.apply(x).cpu().numpy()
    ylo = A.apply(x, prec=low).cpu().numpy()
    err = np.max(np.abs(ylo - y64)) / np.max(np.abs(y64))
    print(f"low-precision matvec error ({cid}, {'fp32' if low == 1 else 'bf16'}): {err:.2e}")
    assert 0.0 < err <= LOW_BOUND[low]
    # the FP64 path of the same operator is untouched by the extra copy
    assert np.max(np.abs(y64 - Ho.apply(x.cpu().numpy()))) <= 1e-11 * np.max(np.abs(y64))


@pytest.mark.parametrize("low", [1, 2])
@pytest.mark.parametrize("cid", list(CASES))
def test_refined_solution_matches_fp64_oracle(B, orc, cid, low):
    g, s, A, So, Ho = case(B, orc, cid, low)
    x0 = W.CONFIGS[0]["x0"]
    b = s.rhs(B.BEM_DATA_POINT_SOURCE, [x0])
    x, stats = A.solve(b, tol=1e-10, refine=True, inner_tol=1e-4)
    it, ok, rr, outer = stats[0]
    assert ok and rr <= 1e-10 and outer >= 1
    bo = So.rhs(orc.POINT_SOURCE, x0)
    xo, _, _, oko = Ho.gmres(bo, tol=1e-13)
    xg = x.cpu().numpy()[0]
    err = np.linalg.norm(xg - xo) / np.linalg.norm(xo)
    print(f"refined solution error vs FP64 oracle ({cid}, low={low}): {err:.2e} after {outer} refinements, {it} its")
    assert oko and err <= 1e-8


def test_precision_errors(B, orc):
    g, s, A, So, Ho = case(B, orc, "sphere_L2_d1_laplace", 1)
    x = torch.zeros(s.ndof, dtype=torch.float64, device="cuda")
    with pytest.raises(B.BemError) as e:
        A.apply(x, prec=2)  # only FP32 was assembled
    assert e.value.code == B._bem.BEM_EINVAL
    g2 = B.Geometry(B.BEM_GEOM_SPHERE6)
    s2 = B.Space(g2, B.BEM_LAPLACE_SINGLE, 0.0, degree=1, level=1)
    A2 = B.Operator(s2, q=3, eta=1.6, leaf_level=1)
    with pytest.raises(B.BemError) as e:
        A2.solve(torch.ones(s2.ndof, dtype=torch.float64, device="cuda"), refine=True)
    assert e.value.code == B._bem.BEM_EINVAL


@pytest.fixture(scope="module")
def c1_fp64(B):
    """The benchmark workload's FP64 solution at a relative residual of 1e-13 (its matvec is
    pinned to the oracle by the parity tests), the reference of the refined solves."""
    c = W.CONFIGS[1]
    g = B.Geometry(B.BEM_GEOM_SPHERE6)
    s = B.Space(g, B.BEM_LAPLACE_SINGLE, 0.0, degree=c["degree"], level=c["level"])
    ops = {low: B.Operator(s, q=c["q"], eta=c["eta"], leaf_level=c["leaf"], far_low=low) for low in (1, 2)}
    x0, pts = W.c1_inputs()
    b = s.rhs(B.BEM_DATA_POINT_SOURCE, [x0])
    x64, st64 = ops[1].solve(b, tol=1e-13, restart=c["restart"], maxit=20000)
    assert st64[0][1] and st64[0][2] <= 1e-13
    return s, ops, b, x64, pts


@pytest.mark.parametrize("low", [1, 2])
def test_full_size_refined_solve(B, c1_fp64, low):
    """The refined solve at the benchmark size reaches the same FP64 residual and a solution
    within 1e-8 (relative) of the FP64 solution, both solved to 1e-13."""
    s, ops, b, x64, pts = c1_fp64
    A = ops[low]
    xm, stm = A.solve(b, tol=1e-13, restart=30, maxit=20000, refine=True, max_outer=40)
    it, ok, rr, outer = stm[0]
    assert ok and rr <= 1e-13
    r = (b[0] - A.apply(xm[0])).norm() / b[0].norm()
    assert float(r) <= 1e-13 * (1 + 1e-6)
    d = float((xm - x64).norm() / x64.norm())
    u64 = s.potential(pts, x64[0]).cpu().numpy()
    um = s.potential(pts, xm[0]).cpu().numpy()
    du = float(np.max(np.abs(um - u64)) / np.max(np.abs(u64)))
    print(f"full size: refined ({'fp32' if low == 1 else 'bf16'}) vs FP64 solution {d:.2e}, potential {du:.2e}; "
          f"{it} its, {outer} outer steps")
    assert d <= 1e-8 and du <= 1e-10
