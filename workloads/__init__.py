"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the benchmark.

This module holds none of the method's arithmetic: only the sizes of the workloads and the
random draws (points, directions, wavenumbers, vectors).  Both sides of every parity check
take their inputs from here, so the oracle and the HIP path never feed each other.

Every random draw uses ``numpy.random.default_rng([1906, config_index, *extra])``.
"""
from __future__ import annotations

import numpy as np

# Workloads (geometries are the analytic multi-patch maps; sizes as in the paper's example
# of refinement levels and degrees, Sec. 5, at the scale of the benchmark).
CONFIGS = {
    0: dict(
        name="laplace_sphere6_L2_d1_dense",
        geom="sphere", gparams=(), pde="laplace", kappa=0.0,
        level=2, degree=1, knot_rep=1,
        dense=True, qg=8, qs=8,
        x0=(0.1, -0.2, 0.15), npts=64, r_range=(2.0, 4.0),
    ),
    1: dict(
        name="laplace_sphere6_L6_d2_h2_q5_eta1.6",
        geom="sphere", gparams=(), pde="laplace", kappa=0.0,
        level=6, degree=2, knot_rep=1,
        q=5, eta=1.6, leaf=4, qg=8, qs=8,
        tol=1e-8, restart=30, maxit=2000,
        x0=(0.1, -0.2, 0.15), npts=64, r_range=(2.0, 4.0),
    ),
    2: dict(
        name="helmholtz_sphere6_L5_d2_h2_128rhs",
        geom="sphere", gparams=(), pde="helmholtz", kappa_range=(2.0, 16.0),
        level=5, degree=2, knot_rep=1,
        q=5, eta=1.6, leaf=3, qg=8, qs=8, nrhs=128,
        tol=1e-8, restart=30, maxit=2000,
    ),
}

CONFIGS[3] = dict(
    name="batched_uneven_ellipsoid_torus_512",
    ninst=512, levels=(2, 3, 4, 5), degrees=(1, 2), kappa_range=(1.0, 8.0), nrhs_range=(1, 16),
    semiaxes=(0.5, 2.0), torus_R=1.0, torus_r=(0.2, 0.5), q=5, eta=1.6,
)
CONFIGS[4] = dict(
    name="learned_precond_ellipsoid_torus_L5-6_d2_helmholtz_k4-20",
    level=5, levels=(5, 6), degree=2, kappa_range=(4.0, 20.0), semiaxes=(0.5, 2.0), torus_R=1.0,
    torus_r=(0.2, 0.5), q=5, eta=1.6, tol=1e-8, restart=64, maxit=15000, ring=2, train_blocks=10000,
)
# At wavenumbers up to 20 on these meshes GMRES(30) stalls even with block-Jacobi (measured
# on the held-out instances: relative residuals 1e-6..7e-3 after 12,000 steps), so this
# family solves with the longest restart the library takes and a step cap of 15,000.

# Maxwell single layer (electric field integral equation) on the unit sphere with the field
# of an electric dipole inside as data, the setting of the paper's example (Sec. 5, Fig. 1:
# field error at exterior points against the level): degree 2 on level 5 for the timings,
# levels 1..5 at degrees 1 and 2 for the convergence series; wavenumber below the first
# interior resonance of the unit sphere (about 2.74).
MAXWELL = dict(
    name="maxwell_efie_sphere6_L5_p2_h2_q5_eta1.6",
    level=5, degree=2, kappa=1.5, q=5, eta=1.6, qg=8, qs=8,
    x0=(0.1, 0.2, -0.1), moment=(0.3, -0.5, 1.0), npts=20, r_range=(2.0, 4.0),
    tol=1e-8, restart=64, maxit=5000, levels=(1, 2, 3, 4, 5), dense_level=3,
    # the convergence series interpolates with 7 nodes: at q = 5 the compression error
    # (about 1e-6 in the field) hides the discretisation error of degree 2 from level 4 on
    series_q=7, series_tol=1e-10, series_maxit=10000,
)

GEOM_KIND = {"sphere": 0, "ellipsoid": 1, "torus": 2, "flat": 3}
PDE_KIND = {"laplace": 0, "helmholtz": 1}


def rng(config_index: int, *extra: int) -> np.random.Generator:
    return np.random.default_rng([1906, config_index, *extra])


def maxwell_inputs():
    """(dipole parameters x0 + unit moment, exterior evaluation points) of the Maxwell workload."""
    c = MAXWELL
    mom = np.asarray(c["moment"], dtype=np.float64)
    mom = mom / np.linalg.norm(mom)
    pts = exterior_points(rng(9, 73), c["npts"], *c["r_range"])
    return list(c["x0"]) + mom.tolist(), pts


def ndof(npatch: int, level: int, degree: int, knot_rep: int = 1) -> int:
    n1 = degree + 1 + ((1 << level) - 1) * knot_rep
    return npatch * n1 * n1


def unit_vectors(g: np.random.Generator, n: int) -> np.ndarray:
    """Directions uniform on the unit sphere (normalised Gaussian 3-vectors)."""
    v = g.normal(size=(n, 3))
    return v / np.linalg.norm(v, axis=1)[:, None]


def exterior_points(g: np.random.Generator, n: int, rmin: float = 2.0, rmax: float = 4.0) -> np.ndarray:
    """Points with uniform direction and radius uniform in [rmin, rmax]."""
    d = unit_vectors(g, n)
    r = g.uniform(rmin, rmax, size=(n, 1))
    return d * r


def random_vector(g: np.random.Generator, n: int, is_complex: bool = False, ncols: int = 1) -> np.ndarray:
    if is_complex:
        v = g.normal(size=(n, ncols)) + 1j * g.normal(size=(n, ncols))
    else:
        v = g.normal(size=(n, ncols))
    return v[:, 0].copy() if ncols == 1 else v


def _near_sphere_resonance(k: float, lmax: int, margin: float) -> bool:
    """True if k lies within `margin` of a zero of some spherical Bessel j_l, l <= lmax
    (the interior Dirichlet eigenvalues of the unit ball, at which the single-layer operator
    on the unit sphere is singular)."""
    from scipy.special import spherical_jn

    for l in range(lmax + 1):
        ks = np.linspace(k - margin, k + margin, 9)
        v = spherical_jn(l, ks)
        if np.any(np.sign(v[:-1]) != np.sign(v[1:])) or np.any(v == 0.0):
            return True
    return False


def draw_wavenumber(g: np.random.Generator, lo: float, hi: float, lmax: int = 20,
                    margin: float = 0.02, avoid_sphere_resonance: bool = True) -> float:
    """Wavenumber uniform in [lo, hi], redrawn while it is near a resonance of the sphere."""
    while True:
        k = float(g.uniform(lo, hi))
        if not avoid_sphere_resonance or not _near_sphere_resonance(k, lmax, margin):
            return k


def c0_inputs():
    """Point-source centre and the 64 exterior evaluation points of the dense sphere case."""
    c = CONFIGS[0]
    g = rng(0)
    pts = exterior_points(g, c["npts"], *c["r_range"])
    return np.array(c["x0"]), pts


def c1_inputs():
    c = CONFIGS[1]
    g = rng(1)
    pts = exterior_points(g, c["npts"], *c["r_range"])
    return np.array(c["x0"]), pts


def c2_inputs():
    """Wavenumber and plane-wave directions of the Helmholtz many-RHS case."""
    c = CONFIGS[2]
    g = rng(2)
    k = draw_wavenumber(g, *c["kappa_range"])
    dirs = unit_vectors(g, c["nrhs"])
    return k, dirs


def sample_rows(config_index: int, n: int, nrows: int) -> np.ndarray:
    """Sorted distinct row indices for sampled parity checks at full size; always includes
    the first and the last row."""
    g = rng(config_index, 7)
    rows = set(g.choice(n, size=min(nrows, n), replace=False).tolist())
    rows.update({0, n - 1})
    return np.array(sorted(rows), dtype=np.int64)



def shape_draw(g: np.random.Generator, cfg: dict):
    """Ellipsoid (semi-axes uniform) or torus (R fixed, r uniform), 50/50."""
    if g.uniform() < 0.5:
        a = g.uniform(*cfg["semiaxes"], size=3)
        return GEOM_KIND["ellipsoid"], tuple(float(v) for v in a)
    return GEOM_KIND["torus"], (float(cfg["torus_R"]), float(g.uniform(*cfg["torus_r"])))


def c4_levels(n: int, stream: int = 0):
    """Levels of the first n instances of a stream of the learned-preconditioner family,
    uniform over the configured levels (a draw of its own, so the instances' shapes and
    wavenumbers do not depend on it)."""
    g = rng(4, 100 + stream)
    return [int(v) for v in g.choice(CONFIGS[4]["levels"], size=n)]


def c4_instances(n: int, stream: int = 0, kappa_range=None):
    """Instances of the learned-preconditioner family: (geom, params, kappa) with kappa
    uniform in the configured range (or kappa_range); stream 0 trains, other streams are
    held out."""
    cfg = CONFIGS[4]
    g = rng(4, stream)
    out = []
    for _ in range(n):
        geom, prm = shape_draw(g, cfg)
        out.append((geom, prm, float(g.uniform(*(kappa_range or cfg["kappa_range"])))))
    return out


def c3_instances(n: int | None = None):
    """Instances of the batched uneven workload: geometry, level, degree, PDE, wavenumber,
    number of right-hand sides, and one interior point source per right-hand side."""
    cfg = CONFIGS[3]
    n = cfg["ninst"] if n is None else n
    g = rng(3)
    out = []
    for _ in range(n):
        geom, prm = shape_draw(g, cfg)
        L = int(g.choice(cfg["levels"]))
        d = int(g.choice(cfg["degrees"]))
        helm = bool(g.uniform() < 0.5)
        kappa = float(g.uniform(*cfg["kappa_range"])) if helm else 0.0
        nrhs = int(g.integers(cfg["nrhs_range"][0], cfg["nrhs_range"][1] + 1))
        srcs = []
        for _ in range(nrhs):
            if geom == GEOM_KIND["ellipsoid"]:
                u = unit_vectors(g, 1)[0] * g.uniform() ** (1 / 3)
                srcs.append(tuple(0.5 * np.array(prm) * u))
            else:
                R, r = prm
                phi = g.uniform(0, 2 * np.pi)
                rho = 0.5 * r * np.sqrt(g.uniform())
                th = g.uniform(0, 2 * np.pi)
                rr = R + rho * np.cos(th)
                srcs.append((rr * np.cos(phi), rr * np.sin(phi), rho * np.sin(th)))
        out.append(dict(geom=geom, params=prm, level=L, degree=d, pde=1 if helm else 0, kappa=kappa, sources=srcs))
    return out


# ------------------------------------------------------------------ NURBS patch sets
# Geometry inputs given as NURBS patches (control points and weights): each patch is a dict
# {"degree": (p1, p2), "knots": (Xi_1, Xi_2), "cw": array (k1, k2, 4) of x, y, z, w}.

def _quarter_arc(k: int):
    """The unit circle over the angles [k pi/2, (k+1) pi/2] as a rational quadratic Bezier
    arc: control points (end, corner of the end tangents, end) and weights (1, 1/sqrt 2, 1)."""
    t0 = 0.5 * np.pi * k
    c, s = np.cos(t0), np.sin(t0)
    pts = np.array([[c, s], [c - s, s + c], [-s, c]])
    w = np.array([1.0, np.sqrt(0.5), 1.0])
    return pts, w


def nurbs_torus(R: float, r: float):
    """The torus of radii R > r as 16 biquadratic rational patches, patch 4 a + b covering
    the quarter turns a (around the z axis) and b (around the tube), oriented like the
    analytic torus patches (outward normal); control points are the products of the two
    circles' arc control points."""
    knots = [0.0, 0.0, 0.0, 1.0, 1.0, 1.0]
    out = []
    for a in range(4):
        P, wP = _quarter_arc(a)
        for b in range(4):
            Q, wQ = _quarter_arc(b)
            cw = np.zeros((3, 3, 4))
            for i in range(3):
                for j in range(3):
                    rad = R + r * Q[j, 0]
                    cw[i, j] = (rad * P[i, 0], rad * P[i, 1], r * Q[j, 1], wP[i] * wQ[j])
            out.append({"degree": (2, 2), "knots": (knots, knots), "cw": cw})
    return out


def greville(knots, p: int) -> np.ndarray:
    """Greville abscissae of a knot vector (averages of p consecutive interior knots)."""
    kn = np.asarray(knots, dtype=np.float64)
    k = kn.size - p - 1
    if p == 0:
        return 0.5 * (kn[:k] + kn[1:k + 1])
    return np.array([kn[j + 1:j + p + 1].mean() for j in range(k)])


def nurbs_flat(a: float, degree=(2, 3), knots=None, weight: float = 2.5):
    """The square [0, a]^2 x {0} as one NURBS patch whose map is (a s, a t, 0): control
    points at the Greville abscissae (linear precision of B-splines), every weight equal.
    knots: (Xi_1, Xi_2), default non-uniform open knot vectors."""
    if knots is None:
        knots = ([0.0] * (degree[0] + 1) + [0.2, 0.45, 0.5] + [1.0] * (degree[0] + 1),
                 [0.0] * (degree[1] + 1) + [0.3, 0.7] + [1.0] * (degree[1] + 1))
    g1, g2 = greville(knots[0], degree[0]), greville(knots[1], degree[1])
    cw = np.zeros((g1.size, g2.size, 4))
    for i, u in enumerate(g1):
        for j, v in enumerate(g2):
            cw[i, j] = (a * u, a * v, 0.0, weight)
    return [{"degree": tuple(degree), "knots": (list(knots[0]), list(knots[1])), "cw": cw}]


def sphere6_map(f: int, st) -> np.ndarray:
    """The unit sphere's patch f (cube face projected radially, faces +z, -z, +x, -x, +y, -y
    with u = 2s - 1, v = 2t - 1 placed as (u,v,1), (v,u,-1), (1,u,v), (-1,v,u), (v,1,u),
    (u,-1,v)), as a user-supplied map: xyz for an (n, 2) array of parameter points."""
    st = np.asarray(st, dtype=np.float64).reshape(-1, 2)
    u, v = 2.0 * st[:, 0] - 1.0, 2.0 * st[:, 1] - 1.0
    one = np.ones_like(u)
    c = [np.stack([u, v, one], 1), np.stack([v, u, -one], 1), np.stack([one, u, v], 1),
         np.stack([-one, v, u], 1), np.stack([v, one, u], 1), np.stack([u, -one, v], 1)][f]
    return c / np.linalg.norm(c, axis=1, keepdims=True)


def torus16_map(R: float, r: float):
    """The torus's 16 quarter-turn patches as a user-supplied map (same parametrisation as
    the analytic torus)."""
    def fn(f: int, st):
        st = np.asarray(st, dtype=np.float64).reshape(-1, 2)
        u = 0.5 * np.pi * ((f >> 2) + st[:, 0])
        v = 0.5 * np.pi * ((f & 3) + st[:, 1])
        rr = R + r * np.cos(v)
        return np.stack([rr * np.cos(u), rr * np.sin(u), r * np.sin(v)], 1)
    return fn
