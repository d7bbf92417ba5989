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
    name="learned_precond_ellipsoid_torus_L5_d2_helmholtz",
    level=5, degree=2, kappa_range=(4.0, 20.0), semiaxes=(0.5, 2.0), torus_R=1.0, torus_r=(0.2, 0.5),
    q=5, eta=1.6, tol=1e-8, restart=30, maxit=2000, ring=2,
)

GEOM_KIND = {"sphere": 0, "ellipsoid": 1, "torus": 2, "flat": 3}
PDE_KIND = {"laplace": 0, "helmholtz": 1}


def rng(config_index: int, *extra: int) -> np.random.Generator:
    return np.random.default_rng([1906, config_index, *extra])


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
