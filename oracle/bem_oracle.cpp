// Oracle of the isogeometric Galerkin BEM hot path: Laplace and Helmholtz single-layer
// operators on multi-patch surfaces, assembled densely or as an interpolation-based H^2
// matrix, plus the right-hand side, the potential and restarted GMRES; the Maxwell single
// layer on div-conforming spaces, assembled densely or with its far field compressed by the
// same interpolation (four channels on the scalar block partition), with its load vector
// and field.
//
// TEST INFRASTRUCTURE ONLY.  This file is compiled into liboracle.so, which is loaded by
// tests/, by the smoke check and by the CPU-baseline leg of bench.py, and by nothing on the
// product path.  It is plain serial FP64 code written to be read against the paper
// (Bembel, arXiv 1906.00785), not to be fast.  It shares no code with the HIP library.
//
// Paper sections followed (cited by section / equation, never by line):
//   App. A  PDEs (LP), (HP), (MP)               App. B  single-layer ansatz (LS), (HS), (MS), (BIE)
//   App. C  B-spline recursion                  App. D  multi-patch B-rep, matching condition
//   App. E  spaces S^0, S^1, S^2, Piola lifting Sec. 2  singular integrals by regularisation,
//                                                       embedded FMM / H^2 on the unit square
//   Sec. 4  API: Discretization, computeRhs, HierarchicalMatrix, H*x, GMRES, evalSolution
// Where the paper is silent a reading is taken (A1..A23 and the named ones below); each is
// stated in the function that takes it.
//
// Parity status: every function here is pinned by a CPU test (tests/test_oracle_*.py)
// against a closed form, an invariant, a library routine or brute force.  The compressed
// operator itself is pinned three ways: eta -> 0 gives the dense matrix, the error decays
// geometrically in q, and its matvec equals the operator written out from the definition
// (interpolated kernel on every far pair, scipy B-splines and Gauss rules; flat square).
// The compressed Maxwell form is pinned the same way (eta = 0 gives its dense matrix, the
// error decays geometrically in q) and its divergence channel equals the scalar compressed
// operator of the divergences.
#include <algorithm>
#include <array>
#include <cmath>
#include <complex>
#include <cstdint>
#include <cstring>
#include <map>
#include <stdexcept>
#include <string>
#include <vector>

#ifdef _OPENMP
#include <omp.h>
#endif

namespace orc {

using cplx = std::complex<double>;
static const double PI = 3.14159265358979323846264338327950288;

// ---------------------------------------------------------------------------------------
// Gauss-Legendre rule on [0,1]: Newton iteration on the Legendre polynomial P_n, nodes
// ascending.  Used for every quadrature in the oracle (regular pairs, Duffy cubes,
// moments, right-hand side, potential).
// ---------------------------------------------------------------------------------------
struct Rule {
    std::vector<double> x, w;
};

static Rule gauss01(int n) {
    Rule r;
    r.x.assign(n, 0.0);
    r.w.assign(n, 0.0);
    for (int i = 0; i < n; ++i) {
        double z = std::cos(PI * (i + 0.75) / (n + 0.5));
        double dp = 1.0;
        for (int it = 0; it < 200; ++it) {
            double p0 = 1.0, p1 = z;
            for (int k = 2; k <= n; ++k) {
                double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            if (n == 1) p0 = 1.0;
            dp = n * (z * p1 - p0) / (z * z - 1.0);
            double dz = p1 / dp;
            z -= dz;
            if (std::fabs(dz) < 1e-16) break;
        }
        // final derivative at the converged node for the weight
        double p0 = 1.0, p1 = z;
        for (int k = 2; k <= n; ++k) {
            double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
            p0 = p1;
            p1 = p2;
        }
        dp = n * (z * p1 - p0) / (z * z - 1.0);
        r.x[n - 1 - i] = 0.5 * (1.0 + z);
        r.w[n - 1 - i] = 1.0 / ((1.0 - z * z) * dp * dp);
    }
    return r;
}

// ---------------------------------------------------------------------------------------
// B-splines, App. C: clamped knot vector on [0,1] with 2^L equal elements, interior knots
// repeated r times (App. E: equidistant knots, same degree in both directions).
// ---------------------------------------------------------------------------------------
struct Knots {
    int d = 0, r = 1, L = 0;
    int nel = 1;  // elements per direction, 2^L
    int nb = 1;   // B-splines per direction
    std::vector<double> xi;
};

static Knots make_knots(int d, int r, int L) {
    Knots K;
    K.d = d;
    K.r = r;
    K.L = L;
    K.nel = 1 << L;
    for (int i = 0; i <= d; ++i) K.xi.push_back(0.0);
    for (int k = 1; k < K.nel; ++k)
        for (int m = 0; m < r; ++m) K.xi.push_back((double)k / (double)K.nel);
    for (int i = 0; i <= d; ++i) K.xi.push_back(1.0);
    K.nb = (int)K.xi.size() - d - 1;
    return K;
}

// Cox-de Boor recursion of App. C.  The degree-0 functions are the indicators of the
// half-open knot spans; here the span that contains x is passed explicitly (`span`), which
// is the same indicator for x inside that span and keeps points that round onto an element
// edge on the element they belong to.  Quotients with a zero denominator are taken as 0.
static double bspline(const Knots& K, int j, int p, double x, int span) {
    if (p == 0) return (j == span) ? 1.0 : 0.0;
    double v = 0.0;
    double den1 = K.xi[j + p] - K.xi[j];
    if (den1 > 0.0) v += (x - K.xi[j]) / den1 * bspline(K, j, p - 1, x, span);
    double den2 = K.xi[j + p + 1] - K.xi[j + 1];
    if (den2 > 0.0) v += (K.xi[j + p + 1] - x) / den2 * bspline(K, j + 1, p - 1, x, span);
    return v;
}

// knot span of element i (the last knot index whose value is i/2^L)
static int elem_span(const Knots& K, int i) { return K.d + i * K.r; }
// first B-spline that is non-zero on element i; the d+1 functions first..first+d are
static int elem_first_basis(const Knots& K, int i) { return i * K.r; }

// span containing a point x of [0,1] (closed at x = 1), for evaluating at arbitrary points
static int find_span(const Knots& K, double x) {
    int i = (int)std::floor(x * K.nel);
    if (i >= K.nel) i = K.nel - 1;
    if (i < 0) i = 0;
    return elem_span(K, i);
}

// ---------------------------------------------------------------------------------------
// Geometry, App. D: Gamma is the union of patches gamma_f([0,1]^2) with outward normal and
// matching parametrisations on shared edges.  The analytic maps are reading A1.
// ---------------------------------------------------------------------------------------
enum { G_SPHERE = 0, G_ELLIPSOID = 1, G_TORUS = 2, G_FLAT = 3, G_NURBS = 4 };

// One NURBS patch of App. C: degrees p_1, p_2, knot vectors Xi_1, Xi_2 on [0, 1] with
// k_1, k_2 basis functions, control points c_{j1 j2} and weights w_{j1 j2} (stored
// x, y, z, w per control point, j1 outer).
struct NurbsPatch {
    int p[2] = {0, 0};
    int k[2] = {1, 1};
    std::vector<double> xi[2];
    std::vector<double> cw;
};

struct Geom {
    int kind = G_SPHERE;
    double p[3] = {1.0, 1.0, 1.0};
    int npatch = 6;
    std::vector<NurbsPatch> nurbs;  // G_NURBS only
};

static Geom make_geom(int kind, const double* params, int nparams) {
    Geom G;
    G.kind = kind;
    if (kind == G_SPHERE) {
        G.npatch = 6;
    } else if (kind == G_ELLIPSOID) {
        if (nparams < 3) throw std::runtime_error("ellipsoid needs a,b,c");
        G.npatch = 6;
        for (int i = 0; i < 3; ++i) G.p[i] = params[i];
    } else if (kind == G_TORUS) {
        if (nparams < 2) throw std::runtime_error("torus needs R,r");
        G.npatch = 16;
        G.p[0] = params[0];
        G.p[1] = params[1];
    } else if (kind == G_FLAT) {
        if (nparams < 1) throw std::runtime_error("flat square needs its side");
        G.npatch = 1;
        G.p[0] = params[0];
    } else {
        throw std::runtime_error("unknown geometry kind");
    }
    return G;
}

// All k B-splines of degree p over the knot vector xi at x (App. C recursion), and their
// derivatives.  The recursion is evaluated degree by degree over every index (the same
// formula as the recursive definition, each b_j^{p-1} computed once); the degree-0
// indicators take the half-open span [xi_j, xi_{j+1}) that contains x, and at x = 1 the
// last non-empty span.  Quotients with a zero denominator are taken as 0.  Derivative:
// d/dx b_j^p = p b_j^{p-1} / (xi_{j+p} - xi_j) - p b_{j+1}^{p-1} / (xi_{j+p+1} - xi_{j+1}).
static void nurbs_basis(const std::vector<double>& xi, int p, int k, double x, std::vector<double>& b,
                        std::vector<double>& db) {
    const int nk = (int)xi.size();
    int span = -1;
    for (int j = 0; j + 1 < nk; ++j)
        if (xi[j] < xi[j + 1] && xi[j] <= x && (x < xi[j + 1] || (xi[j + 1] >= xi[nk - 1] && x <= xi[j + 1])))
            span = j;
    if (span < 0) throw std::runtime_error("point outside the knot vector");
    // (work arrays kept per thread so that repeated calls do not allocate)
    thread_local std::vector<double> cur, prev;
    cur.assign(nk - 1, 0.0);
    cur[span] = 1.0;
    for (int q = 1; q <= p; ++q) {
        prev.swap(cur);
        const int cnt = nk - 1 - q;
        cur.assign(cnt, 0.0);
        for (int j = 0; j < cnt; ++j) {
            double v = 0.0;
            const double d1 = xi[j + q] - xi[j];
            if (d1 > 0.0) v += (x - xi[j]) / d1 * prev[j];
            const double d2 = xi[j + q + 1] - xi[j + 1];
            if (d2 > 0.0) v += (xi[j + q + 1] - x) / d2 * prev[j + 1];
            cur[j] = v;
        }
        if (q == p) {
            db.assign(k, 0.0);
            for (int j = 0; j < k; ++j) {
                double v = 0.0;
                const double d1 = xi[j + p] - xi[j];
                if (d1 > 0.0) v += p * prev[j] / d1;
                const double d2 = xi[j + p + 1] - xi[j + 1];
                if (d2 > 0.0) v -= p * prev[j + 1] / d2;
                db[j] = v;
            }
        }
    }
    if (p == 0) db.assign(k, 0.0);
    b.assign(cur.begin(), cur.begin() + k);
}

// NURBS map of App. C and its partial derivatives (quotient rule)
static void nurbs_point(const NurbsPatch& P, double s, double t, double x[3], double xs[3], double xt[3]) {
    thread_local std::vector<double> b1, db1, b2, db2;
    nurbs_basis(P.xi[0], P.p[0], P.k[0], s, b1, db1);
    nurbs_basis(P.xi[1], P.p[1], P.k[1], t, b2, db2);
    double A[3] = {0, 0, 0}, As[3] = {0, 0, 0}, At[3] = {0, 0, 0}, W = 0, Ws = 0, Wt = 0;
    for (int j1 = 0; j1 < P.k[0]; ++j1)
        for (int j2 = 0; j2 < P.k[1]; ++j2) {
            const double* c = &P.cw[4 * ((size_t)j1 * P.k[1] + j2)];
            const double w = c[3];
            const double v = b1[j1] * b2[j2] * w, vs = db1[j1] * b2[j2] * w, vt = b1[j1] * db2[j2] * w;
            for (int d = 0; d < 3; ++d) {
                A[d] += v * c[d];
                As[d] += vs * c[d];
                At[d] += vt * c[d];
            }
            W += v;
            Ws += vs;
            Wt += vt;
        }
    for (int d = 0; d < 3; ++d) {
        x[d] = A[d] / W;
        if (xs) xs[d] = (As[d] - x[d] * Ws) / W;
        if (xt) xt[d] = (At[d] - x[d] * Wt) / W;
    }
}

static Geom make_nurbs_geom(int npatch, const int* meta, const double* knots, const double* cw) {
    if (npatch < 1) throw std::runtime_error("need at least one patch");
    Geom G;
    G.kind = G_NURBS;
    G.npatch = npatch;
    size_t ko = 0, co = 0;
    for (int f = 0; f < npatch; ++f) {
        NurbsPatch P;
        for (int d = 0; d < 2; ++d) {
            P.p[d] = meta[4 * f + d];
            P.k[d] = meta[4 * f + 2 + d];
            if (P.p[d] < 0 || P.k[d] <= P.p[d]) throw std::runtime_error("bad NURBS degree or count");
        }
        for (int d = 0; d < 2; ++d) {
            const int nk = P.k[d] + P.p[d] + 1;
            P.xi[d].assign(knots + ko, knots + ko + nk);
            ko += nk;
            for (int i = 0; i + 1 < nk; ++i)
                if (P.xi[d][i + 1] < P.xi[d][i]) throw std::runtime_error("knots must not decrease");
            if (P.xi[d].front() != 0.0 || P.xi[d].back() != 1.0) throw std::runtime_error("knots must span [0,1]");
        }
        const size_t n = (size_t)P.k[0] * P.k[1] * 4;
        P.cw.assign(cw + co, cw + co + n);
        co += n;
        for (size_t i = 3; i < n; i += 4)
            if (!(P.cw[i] > 0.0)) throw std::runtime_error("weights must be positive");
        G.nurbs.push_back(std::move(P));
    }
    return G;
}

// cube face f at (u,v) in [-1,1]^2 and the face's derivatives with respect to u and v
static void cube_face(int f, double u, double v, double c[3], double cu[3], double cv[3]) {
    // +z:(u,v,1)  -z:(v,u,-1)  +x:(1,u,v)  -x:(-1,v,u)  +y:(v,1,u)  -y:(u,-1,v)
    for (int k = 0; k < 3; ++k) cu[k] = cv[k] = 0.0;
    switch (f) {
        case 0: c[0] = u; c[1] = v; c[2] = 1.0; cu[0] = 1; cv[1] = 1; break;
        case 1: c[0] = v; c[1] = u; c[2] = -1.0; cu[1] = 1; cv[0] = 1; break;
        case 2: c[0] = 1.0; c[1] = u; c[2] = v; cu[1] = 1; cv[2] = 1; break;
        case 3: c[0] = -1.0; c[1] = v; c[2] = u; cu[2] = 1; cv[1] = 1; break;
        case 4: c[0] = v; c[1] = 1.0; c[2] = u; cu[2] = 1; cv[0] = 1; break;
        default: c[0] = u; c[1] = -1.0; c[2] = v; cu[0] = 1; cv[2] = 1; break;
    }
}

// gamma_f(s,t) and, when requested, its partial derivatives (for the surface element)
static void gamma(const Geom& G, int f, double s, double t, double x[3], double xs[3] = nullptr,
                  double xt[3] = nullptr) {
    if (G.kind == G_SPHERE || G.kind == G_ELLIPSOID) {
        double c[3], cu[3], cv[3];
        cube_face(f, 2.0 * s - 1.0, 2.0 * t - 1.0, c, cu, cv);
        double rho = std::sqrt(c[0] * c[0] + c[1] * c[1] + c[2] * c[2]);
        double n[3] = {c[0] / rho, c[1] / rho, c[2] / rho};
        double sc[3] = {1.0, 1.0, 1.0};
        if (G.kind == G_ELLIPSOID) {
            sc[0] = G.p[0];
            sc[1] = G.p[1];
            sc[2] = G.p[2];
        }
        for (int k = 0; k < 3; ++k) x[k] = sc[k] * n[k];
        if (xs && xt) {
            // d(c/|c|) = (dc - n (n.dc)) / |c|, with dc/ds = 2 cu and dc/dt = 2 cv
            double nu = n[0] * cu[0] + n[1] * cu[1] + n[2] * cu[2];
            double nv = n[0] * cv[0] + n[1] * cv[1] + n[2] * cv[2];
            for (int k = 0; k < 3; ++k) {
                xs[k] = sc[k] * 2.0 * (cu[k] - n[k] * nu) / rho;
                xt[k] = sc[k] * 2.0 * (cv[k] - n[k] * nv) / rho;
            }
        }
    } else if (G.kind == G_TORUS) {
        const double R = G.p[0], r = G.p[1];
        int a = f / 4, b = f % 4;
        double u = 2.0 * PI * (a + s) / 4.0, v = 2.0 * PI * (b + t) / 4.0;
        double A = R + r * std::cos(v);
        x[0] = A * std::cos(u);
        x[1] = A * std::sin(u);
        x[2] = r * std::sin(v);
        if (xs && xt) {
            const double du = PI / 2.0, dv = PI / 2.0;
            xs[0] = -A * std::sin(u) * du;
            xs[1] = A * std::cos(u) * du;
            xs[2] = 0.0;
            xt[0] = -r * std::sin(v) * std::cos(u) * dv;
            xt[1] = -r * std::sin(v) * std::sin(u) * dv;
            xt[2] = r * std::cos(v) * dv;
        }
    } else if (G.kind == G_NURBS) {
        nurbs_point(G.nurbs[f], s, t, x, xs, xt);
    } else {  // flat square of side a in the plane z = 0
        const double a = G.p[0];
        x[0] = a * s;
        x[1] = a * t;
        x[2] = 0.0;
        if (xs && xt) {
            xs[0] = a; xs[1] = 0; xs[2] = 0;
            xt[0] = 0; xt[1] = a; xt[2] = 0;
        }
    }
}

// surface element kappa_f(s,t) = |d_s gamma x d_t gamma| and the (unnormalised) normal
static double surf_elem(const Geom& G, int f, double s, double t, double nrm[3] = nullptr) {
    double x[3], xs[3], xt[3];
    gamma(G, f, s, t, x, xs, xt);
    double n[3] = {xs[1] * xt[2] - xs[2] * xt[1], xs[2] * xt[0] - xs[0] * xt[2],
                   xs[0] * xt[1] - xs[1] * xt[0]};
    if (nrm)
        for (int k = 0; k < 3; ++k) nrm[k] = n[k];
    return std::sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
}

// ---------------------------------------------------------------------------------------
// Kernels, App. B (LS) and (HS): 1/(4 pi r) and exp(-i kappa r)/(4 pi r), kappa complex.
// ---------------------------------------------------------------------------------------
enum { PDE_LAPLACE = 0, PDE_HELMHOLTZ = 1 };

template <class T>
static T kernel_r(int pde, cplx kappa, double r);

template <>
double kernel_r<double>(int, cplx, double r) {
    return 1.0 / (4.0 * PI * r);
}
template <>
cplx kernel_r<cplx>(int pde, cplx kappa, double r) {
    if (pde == PDE_LAPLACE) return cplx(1.0 / (4.0 * PI * r), 0.0);
    return std::exp(cplx(0.0, -1.0) * kappa * r) / (4.0 * PI * r);
}

static double dist3(const double a[3], const double b[3]) {
    double dx = a[0] - b[0], dy = a[1] - b[1], dz = a[2] - b[2];
    return std::sqrt(dx * dx + dy * dy + dz * dz);
}

// ---------------------------------------------------------------------------------------
// Discrete space S^2 of App. E on every patch (reading A2: `degree` is the degree d of the
// B-splines of the ansatz space), lifted by the 2-form Piola transform (reading A3) so that
// the surface element cancels from the Galerkin entries.  Global DOF index
// g = (f*nb + j1)*nb + j2; element index e = (f*nel + i1)*nel + i2.
// ---------------------------------------------------------------------------------------
struct Space {
    Geom G;
    int pde = PDE_LAPLACE;
    cplx kappa = 0.0;
    Knots K;
    int64_t nelem = 0, ndof = 0;
    double h = 1.0;
    // lifting of the reference functions to the surface (App. E "Piola transform"): 2 for
    // the 2-form lifting of S^2 (the surface element cancels, reading A3), 0 for the 0-form
    // lifting of S^0 (phi = phi_hat o gamma^-1: every surface integral carries kappa)
    int form = 2;
};

static Space make_space(const Geom& G, int pde, cplx kappa, int d, int r, int L) {
    if (d < 0 || L < 0 || r < 1 || r > d + 1) throw std::runtime_error("bad space parameters");
    Space S;
    S.G = G;
    S.pde = pde;
    S.kappa = kappa;
    S.K = make_knots(d, r, L);
    S.nelem = (int64_t)G.npatch * S.K.nel * S.K.nel;
    S.ndof = (int64_t)G.npatch * S.K.nb * S.K.nb;
    S.h = 1.0 / S.K.nel;
    return S;
}

struct Elem {
    int f, i1, i2;
};
static Elem elem_of(const Space& S, int64_t e) {
    int n = S.K.nel;
    Elem E;
    E.i2 = (int)(e % n);
    E.i1 = (int)((e / n) % n);
    E.f = (int)(e / ((int64_t)n * n));
    return E;
}
static int64_t dof_index(const Space& S, int f, int j1, int j2) {
    return ((int64_t)f * S.K.nb + j1) * S.K.nb + j2;
}

// S^0 continuity across patch boundaries (App. E: continuity conditions give the conforming
// space S^0(Gamma) in H^1/2).  Each local B-spline b_j1 b_j2 of a patch is anchored at the
// image of its Greville point (xi*_j1, xi*_j2), xi*_j = (xi_{j+1} + ... + xi_{j+d}) / d; with
// clamped knots the anchors of the functions that do not vanish on the patch boundary lie on
// it, and by the matching condition (App. D) the functions of two patches that agree on a
// shared edge or vertex have the same anchor.  Those are identified (anchors within 1e-10
// of the largest anchor coordinate), every other function is its own.  Global indices are
// numbered in the order of their first local function.  Returns the local -> global map.
static std::vector<int64_t> glue_map(const Space& S, int64_t* nglob) {
    const Knots& K = S.K;
    if (K.d < 1) throw std::runtime_error("continuous spaces need degree >= 1");
    const int nb = K.nb;
    std::vector<double> gr(nb);
    for (int j = 0; j < nb; ++j) {
        double a = 0.0;
        for (int k = 1; k <= K.d; ++k) a += K.xi[j + k];
        gr[j] = a / K.d;
    }
    std::vector<int64_t> bidx;
    std::vector<std::array<double, 3>> anc;
    double scale = 0.0;
    for (int f = 0; f < S.G.npatch; ++f)
        for (int j1 = 0; j1 < nb; ++j1)
            for (int j2 = 0; j2 < nb; ++j2) {
                if (j1 != 0 && j1 != nb - 1 && j2 != 0 && j2 != nb - 1) continue;
                std::array<double, 3> x;
                gamma(S.G, f, gr[j1], gr[j2], x.data());
                for (double v : x) scale = std::max(scale, std::fabs(v));
                bidx.push_back(dof_index(S, f, j1, j2));
                anc.push_back(x);
            }
    std::vector<int64_t> parent(S.ndof);
    for (int64_t g = 0; g < S.ndof; ++g) parent[g] = g;
    auto root = [&](int64_t g) {
        while (parent[g] != g) g = parent[g] = parent[parent[g]];
        return g;
    };
    const double tol = 1e-10 * std::max(scale, 1e-300);
    for (size_t a = 0; a < bidx.size(); ++a)
        for (size_t b = a + 1; b < bidx.size(); ++b)
            if (std::fabs(anc[a][0] - anc[b][0]) <= tol && std::fabs(anc[a][1] - anc[b][1]) <= tol &&
                std::fabs(anc[a][2] - anc[b][2]) <= tol) {
                const int64_t ra = root(bidx[a]), rb = root(bidx[b]);
                if (ra != rb) parent[std::max(ra, rb)] = std::min(ra, rb);
            }
    std::vector<int64_t> gid(S.ndof, -1), map(S.ndof);
    int64_t n = 0;
    for (int64_t g = 0; g < S.ndof; ++g) {
        const int64_t r = root(g);
        if (gid[r] < 0) gid[r] = n++;
        map[g] = gid[r];
    }
    *nglob = n;
    return map;
}


// D4 symmetries of the unit square, fixed enumeration (reading A8): identity, flip first,
// flip second, flip both; then the same four applied after swapping the coordinates.
static void d4(int k, double a, double b, double& o1, double& o2) {
    if (k >= 4) std::swap(a, b);
    switch (k & 3) {
        case 0: o1 = a; o2 = b; break;
        case 1: o1 = 1.0 - a; o2 = b; break;
        case 2: o1 = a; o2 = 1.0 - b; break;
        default: o1 = 1.0 - a; o2 = 1.0 - b; break;
    }
}

// parameter point of element e at local coordinates (a,b) seen through the symmetry k
static void elem_param(const Space& S, const Elem& E, int k, double a, double b, double& s,
                       double& t) {
    double p1, p2;
    d4(k, a, b, p1, p2);
    s = (E.i1 + p1) * S.h;
    t = (E.i2 + p2) * S.h;
}

// Values of the (d+1)^2 local basis functions of element E at parameter (s,t):
// out[l1*(d+1)+l2] = b_{first1+l1}(s) b_{first2+l2}(t), each in the element's span.
static void elem_basis(const Space& S, const Elem& E, double s, double t, double* out) {
    const Knots& K = S.K;
    int d = K.d;
    int sp1 = elem_span(K, E.i1), sp2 = elem_span(K, E.i2);
    int f1 = elem_first_basis(K, E.i1), f2 = elem_first_basis(K, E.i2);
    std::vector<double> bs(d + 1), bt(d + 1);
    for (int l = 0; l <= d; ++l) {
        bs[l] = bspline(K, f1 + l, d, s, sp1);
        bt[l] = bspline(K, f2 + l, d, t, sp2);
    }
    for (int l1 = 0; l1 <= d; ++l1)
        for (int l2 = 0; l2 <= d; ++l2) out[l1 * (d + 1) + l2] = bs[l1] * bt[l2];
}

// ---------------------------------------------------------------------------------------
// What is integrated on each side of an element pair.  Galerkin mode integrates the local
// B-spline products (the surface element cancels under the Piola lifting); density mode is
// used only by the closed-form pins and integrates f(gamma(s)) * kappa(s) with one of a
// few fixed surface functions f, giving <S f, g> for densities f, g on Gamma.
// ---------------------------------------------------------------------------------------
enum { SIDE_SPLINE = 0, SIDE_DENSITY = 1 };
struct SideFn {
    int mode = SIDE_SPLINE;
    int fid = 0;  // density mode: 0:1  1:x  2:y  3:z  4:x*y  5:x^2-y^2
};

static int side_nb(const Space& S, const SideFn& F) {
    return F.mode == SIDE_SPLINE ? (S.K.d + 1) * (S.K.d + 1) : 1;
}

static double density_fn(int fid, const double x[3]) {
    switch (fid) {
        case 0: return 1.0;
        case 1: return x[0];
        case 2: return x[1];
        case 3: return x[2];
        case 4: return x[0] * x[1];
        default: return x[0] * x[0] - x[1] * x[1];
    }
}

// position and side-function values at element-local point (a,b) under symmetry k
static void side_eval(const Space& S, const SideFn& F, const Elem& E, int k, double a, double b,
                      double x[3], double* vals) {
    double s, t;
    elem_param(S, E, k, a, b, s, t);
    gamma(S.G, E.f, s, t, x);
    if (F.mode == SIDE_SPLINE) {
        elem_basis(S, E, s, t, vals);
        if (S.form == 0) {
            const double k = surf_elem(S.G, E.f, s, t);
            for (int l = 0; l < side_nb(S, F); ++l) vals[l] *= k;
        }
    } else {
        vals[0] = density_fn(F.fid, x) * surf_elem(S.G, E.f, s, t);
    }
}

// ---------------------------------------------------------------------------------------
// Element-pair classification (reading A8): the number of physical corners two distinct
// elements share decides between edge (2), vertex (1) and regular (0) pairs; for touching
// pairs the first symmetry pair (k_tau outer, k_sigma inner) that puts the shared vertex at
// local (0,0) on both elements, and for an edge also (0,1), is chosen.  The matching
// condition of App. D guarantees that such a pair exists.
// ---------------------------------------------------------------------------------------
enum { PAIR_REGULAR = 0, PAIR_VERTEX = 1, PAIR_EDGE = 2, PAIR_IDENTICAL = 3 };

struct PairInfo {
    int type = PAIR_REGULAR;
    int k1 = 0, k2 = 0;
};

static void corner_point(const Space& S, const Elem& E, int k, double a, double b, double x[3]) {
    double s, t;
    elem_param(S, E, k, a, b, s, t);
    gamma(S.G, E.f, s, t, x);
}

static PairInfo classify_pair(const Space& S, int64_t e1, int64_t e2) {
    PairInfo P;
    if (e1 == e2) {
        P.type = PAIR_IDENTICAL;
        return P;
    }
    Elem A = elem_of(S, e1), B = elem_of(S, e2);
    const double cl[4][2] = {{0, 0}, {1, 0}, {0, 1}, {1, 1}};
    double pa[4][3], pb[4][3];
    for (int c = 0; c < 4; ++c) {
        corner_point(S, A, 0, cl[c][0], cl[c][1], pa[c]);
        corner_point(S, B, 0, cl[c][0], cl[c][1], pb[c]);
    }
    double diam = 0.0;
    for (int c = 0; c < 4; ++c)
        for (int c2 = 0; c2 < 4; ++c2) diam = std::max(diam, dist3(pa[c], pa[c2]));
    const double tol = 1e-10 * diam;
    int shared = 0;
    for (int c = 0; c < 4; ++c)
        for (int c2 = 0; c2 < 4; ++c2)
            if (dist3(pa[c], pb[c2]) <= tol) ++shared;
    if (shared == 0) return P;
    if (shared > 2) throw std::runtime_error("elements share more than an edge");
    P.type = (shared == 2) ? PAIR_EDGE : PAIR_VERTEX;
    for (int k1 = 0; k1 < 8; ++k1)
        for (int k2 = 0; k2 < 8; ++k2) {
            double x0[3], y0[3];
            corner_point(S, A, k1, 0, 0, x0);
            corner_point(S, B, k2, 0, 0, y0);
            if (dist3(x0, y0) > tol) continue;
            if (P.type == PAIR_EDGE) {
                double x1[3], y1[3];
                corner_point(S, A, k1, 0, 1, x1);
                corner_point(S, B, k2, 0, 1, y1);
                if (dist3(x1, y1) > tol) continue;
            }
            P.k1 = k1;
            P.k2 = k2;
            return P;
        }
    throw std::runtime_error("no symmetry aligns the shared entity (matching condition)");
}

// Duffy-type regularisation of a touching pair (Sec. 2 cites [SS97]; regions of reading
// A6): calls f(x1, x2, y1, y2, w) for every point of every region's 4D unit cube, qs Gauss
// points per dimension, with local points x (first element) and y (second element) in the
// aligned frames and w the Gauss weight times the substitution's Jacobian.
template <class F>
static void duffy_each(int type, int qs, F&& f) {
    const Rule g = gauss01(qs);
    for (int i0 = 0; i0 < qs; ++i0)
        for (int i1 = 0; i1 < qs; ++i1)
            for (int i2 = 0; i2 < qs; ++i2)
                for (int i3 = 0; i3 < qs; ++i3) {
                    const double xi = g.x[i0], e1v = g.x[i1], e2v = g.x[i2], e3v = g.x[i3];
                    const double wq = g.w[i0] * g.w[i1] * g.w[i2] * g.w[i3];
                    if (type == PAIR_IDENTICAL) {
                        // (xi, eta, u1, u2); the difference vector y - x = (s1 t1, s2 t2)
                        const double u1 = e2v, u2 = e3v;
                        for (int ord = 0; ord < 2; ++ord) {
                            const double t1 = ord == 0 ? xi : xi * e1v;
                            const double t2 = ord == 0 ? xi * e1v : xi;
                            for (int sg = 0; sg < 4; ++sg) {
                                const double s1 = (sg & 1) ? -1.0 : 1.0;
                                const double s2 = (sg & 2) ? -1.0 : 1.0;
                                const double x1 = (1.0 - t1) * u1 + (s1 < 0 ? t1 : 0.0);
                                const double x2 = (1.0 - t2) * u2 + (s2 < 0 ? t2 : 0.0);
                                const double y1 = x1 + s1 * t1, y2 = x2 + s2 * t2;
                                f(x1, x2, y1, y2, wq * xi * (1.0 - t1) * (1.0 - t2));
                            }
                        }
                    } else if (type == PAIR_EDGE) {
                        // shared edge at local first coordinate 0 on both sides; (xi, eta1,
                        // eta2, u): the largest of (x1, y1, t) is xi
                        const double u = e3v;
                        for (int c = 0; c < 3; ++c) {
                            double v3[3];
                            v3[c] = xi;
                            int m = 0;
                            for (int k = 0; k < 3; ++k)
                                if (k != c) v3[k] = xi * (m++ == 0 ? e1v : e2v);
                            const double x1 = v3[0], y1 = v3[1], t = v3[2];
                            for (int sg = 0; sg < 2; ++sg) {
                                const double s2 = sg ? -1.0 : 1.0;
                                const double x2 = (1.0 - t) * u + (s2 < 0 ? t : 0.0);
                                const double y2 = x2 + s2 * t;
                                f(x1, x2, y1, y2, wq * xi * xi * (1.0 - t));
                            }
                        }
                    } else {  // PAIR_VERTEX: shared vertex at local (0,0) on both sides
                        for (int c = 0; c < 4; ++c) {
                            double z[4];
                            z[c] = xi;
                            int m = 0;
                            const double et[3] = {e1v, e2v, e3v};
                            for (int k = 0; k < 4; ++k)
                                if (k != c) z[k] = xi * et[m++];
                            f(z[0], z[1], z[2], z[3], wq * xi * xi * xi);
                        }
                    }
                }
}

// ---------------------------------------------------------------------------------------
// Element-pair integral  B[i][j] = int_tau int_sigma k(x,y) Phi_i(x) Psi_j(y)  over the
// two elements' parameter squares (each of area h^2).
//   regular pairs : tensor Gauss, qg points per direction on each element (reading A7)
//   touching pairs: Duffy-type regularisation (Sec. 2 cites [SS97]; regions of reading A6),
//                   qs Gauss points per dimension of each 4D unit cube.
// ---------------------------------------------------------------------------------------
template <class T>
static void pair_block(const Space& S, const SideFn& Ft, const SideFn& Fs, int64_t e1, int64_t e2,
                       int qg, int qs, T* B, PairInfo* info_out = nullptr) {
    const int nt = side_nb(S, Ft), ns = side_nb(S, Fs);
    for (int i = 0; i < nt * ns; ++i) B[i] = T(0);
    const Elem A = elem_of(S, e1), Bel = elem_of(S, e2);
    const PairInfo P = classify_pair(S, e1, e2);
    if (info_out) *info_out = P;
    const double h4 = S.h * S.h * S.h * S.h;

    if (P.type == PAIR_REGULAR) {
        // iterated integral: for each Gauss point x of tau, the inner integral over sigma
        const Rule g = gauss01(qg);
        const int np = qg * qg;
        std::vector<double> ys(3 * np), ps(ns * np), wy(np);
        for (int b1 = 0; b1 < qg; ++b1)
            for (int b2 = 0; b2 < qg; ++b2) {
                int b = b1 * qg + b2;
                side_eval(S, Fs, Bel, 0, g.x[b1], g.x[b2], &ys[3 * b], &ps[ns * b]);
                wy[b] = g.w[b1] * g.w[b2];
            }
        std::vector<double> xv(3), pt(nt);
        std::vector<T> inner(ns);
        for (int a1 = 0; a1 < qg; ++a1)
            for (int a2 = 0; a2 < qg; ++a2) {
                side_eval(S, Ft, A, 0, g.x[a1], g.x[a2], xv.data(), pt.data());
                const double wx = g.w[a1] * g.w[a2];
                for (int j = 0; j < ns; ++j) inner[j] = T(0);
                for (int b = 0; b < np; ++b) {
                    T kv = kernel_r<T>(S.pde, S.kappa, dist3(xv.data(), &ys[3 * b])) * wy[b];
                    for (int j = 0; j < ns; ++j) inner[j] += kv * ps[ns * b + j];
                }
                for (int i = 0; i < nt; ++i)
                    for (int j = 0; j < ns; ++j) B[i * ns + j] += wx * pt[i] * inner[j];
            }
        for (int i = 0; i < nt * ns; ++i) B[i] *= h4;
        return;
    }

    std::vector<double> pt(nt), ps(ns);
    double xv[3], yv[3];
    // accumulate one point of a Duffy cube: local points xh (on tau) and yh (on sigma)
    duffy_each(P.type, qs, [&](double xh1, double xh2, double yh1, double yh2, double w) {
        side_eval(S, Ft, A, P.k1, xh1, xh2, xv, pt.data());
        side_eval(S, Fs, Bel, P.k2, yh1, yh2, yv, ps.data());
        T kv = kernel_r<T>(S.pde, S.kappa, dist3(xv, yv)) * w;
        for (int i = 0; i < nt; ++i)
            for (int j = 0; j < ns; ++j) B[i * ns + j] += kv * pt[i] * ps[j];
    });
    for (int i = 0; i < nt * ns; ++i) B[i] *= h4;
}

// global DOF of local basis function l of element E (Galerkin mode)
static int64_t local_dof(const Space& S, const Elem& E, int l) {
    const int d = S.K.d;
    const int l1 = l / (d + 1), l2 = l % (d + 1);
    return dof_index(S, E.f, elem_first_basis(S.K, E.i1) + l1, elem_first_basis(S.K, E.i2) + l2);
}

// ---------------------------------------------------------------------------------------
// Dense Galerkin matrix (Sec. 2: conforming Galerkin; App. B (BIE); bilinear pairing):
// A[g][h] = sum over all element pairs of the pair blocks, scattered through the local DOFs.
// ---------------------------------------------------------------------------------------
template <class T>
static void dense_matrix(const Space& S, int qg, int qs, T* A) {
    const int64_t N = S.ndof;
    std::fill(A, A + N * N, T(0));
    SideFn F;
    const int nb = side_nb(S, F);
    std::vector<T> B(nb * nb);
    for (int64_t e1 = 0; e1 < S.nelem; ++e1) {
        const Elem E1 = elem_of(S, e1);
        for (int64_t e2 = 0; e2 < S.nelem; ++e2) {
            const Elem E2 = elem_of(S, e2);
            pair_block<T>(S, F, F, e1, e2, qg, qs, B.data());
            for (int i = 0; i < nb; ++i)
                for (int j = 0; j < nb; ++j)
                    A[local_dof(S, E1, i) * N + local_dof(S, E2, j)] += B[i * nb + j];
        }
    }
}

// <S f, g> for two surface functions given in density mode (closed-form pins only)
template <class T>
static T density_pairing(const Space& S, int fid, int gid, int qg, int qs) {
    SideFn Ft, Fs;
    Ft.mode = Fs.mode = SIDE_DENSITY;
    Ft.fid = fid;
    Fs.fid = gid;
    T sum = T(0), B;
    for (int64_t e1 = 0; e1 < S.nelem; ++e1)
        for (int64_t e2 = 0; e2 < S.nelem; ++e2) {
            pair_block<T>(S, Ft, Fs, e1, e2, qg, qs, &B);
            sum += B;
        }
    return sum;
}

// ---------------------------------------------------------------------------------------
// Boundary data and load vector (Sec. 4 "Boundary Values"): b_g = int g(gamma(s)) phi_g(s) ds
// (surface element cancelled by the Piola lifting); Gauss with q points per direction per
// element.  Data: point source = the PDE's own kernel centred at x0 (exterior Dirichlet
// data reproduced by the single-layer potential, remark in App. B), plane wave
// exp(-i kappa d.x) (reading A16).
// ---------------------------------------------------------------------------------------
enum { DATA_POINT_SOURCE = 0, DATA_PLANE_WAVE = 1 };

template <class T>
static T data_value(const Space& S, int kind, const double* prm, const double x[3]);
template <>
double data_value<double>(const Space& S, int kind, const double* prm, const double x[3]) {
    (void)kind;
    return kernel_r<double>(S.pde, S.kappa, dist3(x, prm));
}
template <>
cplx data_value<cplx>(const Space& S, int kind, const double* prm, const double x[3]) {
    if (kind == DATA_POINT_SOURCE) return kernel_r<cplx>(S.pde, S.kappa, dist3(x, prm));
    const double dx = prm[0] * x[0] + prm[1] * x[1] + prm[2] * x[2];
    return std::exp(cplx(0.0, -1.0) * S.kappa * dx);
}

template <class T>
static void load_vector(const Space& S, int kind, const double* prm, int q, T* b) {
    std::fill(b, b + S.ndof, T(0));
    const Rule g = gauss01(q);
    const int nb = (S.K.d + 1) * (S.K.d + 1);
    std::vector<double> ph(nb);
    for (int64_t e = 0; e < S.nelem; ++e) {
        const Elem E = elem_of(S, e);
        for (int a1 = 0; a1 < q; ++a1)
            for (int a2 = 0; a2 < q; ++a2) {
                double s, t, x[3];
                elem_param(S, E, 0, g.x[a1], g.x[a2], s, t);
                gamma(S.G, E.f, s, t, x);
                elem_basis(S, E, s, t, ph.data());
                const double lift = S.form == 0 ? surf_elem(S.G, E.f, s, t) : 1.0;
                const T gv = data_value<T>(S, kind, prm, x) * (g.w[a1] * g.w[a2] * S.h * S.h * lift);
                for (int l = 0; l < nb; ++l) b[local_dof(S, E, l)] += gv * ph[l];
            }
    }
}

// Potential (Sec. 4 "Evaluation of the Solution"; App. B (LS)/(HS)):
// u(x) = sum_f int k(x, gamma_f(t)) rho_hat_f(t) dt with rho_hat = sum_g rho_g phi_g.
template <class T>
static void potential(const Space& S, int q, const T* rho, int64_t npts, const double* pts, T* u) {
    const Rule g = gauss01(q);
    const int nb = (S.K.d + 1) * (S.K.d + 1);
    std::vector<double> ph(nb);
    for (int64_t p = 0; p < npts; ++p) u[p] = T(0);
    for (int64_t e = 0; e < S.nelem; ++e) {
        const Elem E = elem_of(S, e);
        for (int a1 = 0; a1 < q; ++a1)
            for (int a2 = 0; a2 < q; ++a2) {
                double s, t, y[3];
                elem_param(S, E, 0, g.x[a1], g.x[a2], s, t);
                gamma(S.G, E.f, s, t, y);
                elem_basis(S, E, s, t, ph.data());
                T rv = T(0);
                for (int l = 0; l < nb; ++l) rv += rho[local_dof(S, E, l)] * ph[l];
                rv *= g.w[a1] * g.w[a2] * S.h * S.h * (S.form == 0 ? surf_elem(S.G, E.f, s, t) : 1.0);
                for (int64_t p = 0; p < npts; ++p)
                    u[p] += kernel_r<T>(S.pde, S.kappa, dist3(&pts[3 * p], y)) * rv;
            }
    }
}

// ---------------------------------------------------------------------------------------
// H^2 matrix (Sec. 2: embedded FMM tailored to IGA, compression on the reference square;
// Sec. 4 "System Matrix").  Clusters are dyadic sub-squares of each patch's parameter
// square; the far field of an admissible cluster pair is interpolated in both variables
// with tensor Chebyshev nodes on the two cluster squares:
//   k(gamma(s), gamma(t)) ~ sum_a sum_b L_a^tau(s) k(gamma(xi_a^tau), gamma(xi_b^sigma)) L_b^sigma(t)
// so that A_far = V_tau^T K_tau,sigma V_sigma with moments V_tau[a,g] = int_tau L_a phi_g.
// Readings: A9 (q nodes per direction, first kind), A10 (ball admissibility, eta, tie
// margin), A11 (leaf level), A13 (moment quadrature), A14 (stored coupling blocks).
// ---------------------------------------------------------------------------------------
struct Cluster {
    int lev, f, i, j;
    double c[3];
    double rad;
};

// Chebyshev nodes of the first kind mapped to [0,1] (reading A9)
static std::vector<double> cheb_nodes(int q) {
    std::vector<double> x(q);
    for (int a = 0; a < q; ++a) x[a] = 0.5 * (1.0 + std::cos((2.0 * a + 1.0) * PI / (2.0 * q)));
    return x;
}

// Lagrange basis polynomial a of the nodes xs at point y (product form)
static double lagrange(const std::vector<double>& xs, int a, double y) {
    double v = 1.0;
    for (int b = 0; b < (int)xs.size(); ++b)
        if (b != a) v *= (y - xs[b]) / (xs[a] - xs[b]);
    return v;
}

template <class T>
struct H2 {
    const Space* S = nullptr;
    int q = 5, leaf = 0, qg = 8, qs = 8, qm = 1;
    double eta = 1.6;
    double kadm = 0.0;  // reading A12: |kappa| 2 max(r) <= kadm for a far pair (0: no bound)
    std::vector<int64_t> lev_off;  // first cluster index of every level, plus the total
    std::vector<Cluster> cl;
    std::vector<std::pair<int64_t, int64_t>> far;   // (target, source), sorted
    std::vector<std::pair<int64_t, int64_t>> near;  // leaf pairs, sorted
    std::vector<double> xi;                         // q Chebyshev nodes on [0,1]
    std::vector<double> E[2];                       // E[b][a'*q + a] = L_a(xi child b, node a')
    std::vector<T> K;                               // q^4 per far block, block order = far
    // 1-D moments per leaf index i along one direction: V1[i][a*nloc + m] =
    //   int over leaf interval i of L_a(s) b_{first(i)+m}(s) ds
    std::vector<std::vector<double>> V1;
    std::vector<std::vector<double>> Vd;  // 0-form lifting: full leaf tables (see h2_build)
    int nloc = 0;  // B-splines overlapping one leaf interval
    bool have_near = false;
    std::vector<std::map<int64_t, T>> near_rows;  // near field, one sorted map per row

    int64_t cluster_index(int lev, int f, int i, int j) const {
        const int64_t n = (int64_t)1 << lev;
        return lev_off[lev] + ((int64_t)f * n + i) * n + j;
    }
    int leaf_first_basis(int i) const {  // first B-spline touching leaf interval i
        const int m = 1 << (S->K.L - leaf);
        return elem_first_basis(S->K, i * m);
    }
};

// ball of a cluster (reading A10): centre gamma(midpoint), radius the largest distance to
// gamma at a 9x9 uniform grid of the cluster square, boundary included
static void cluster_ball(const Geom& G, Cluster& C) {
    const double w = 1.0 / (double)(1 << C.lev);
    gamma(G, C.f, (C.i + 0.5) * w, (C.j + 0.5) * w, C.c);
    C.rad = 0.0;
    for (int a = 0; a <= 8; ++a)
        for (int b = 0; b <= 8; ++b) {
            double x[3];
            gamma(G, C.f, (C.i + a / 8.0) * w, (C.j + b / 8.0) * w, x);
            C.rad = std::max(C.rad, dist3(x, C.c));
        }
}

// admissibility (reading A10); ties within 1e-12 * dist count as inadmissible
static bool admissible(const Cluster& A, const Cluster& B, double eta) {
    const double dist = dist3(A.c, B.c) - A.rad - B.rad;
    if (!(dist > 0.0)) return false;
    const double lhs = 2.0 * std::max(A.rad, B.rad), rhs = eta * dist;
    if (std::fabs(lhs - rhs) <= 1e-12 * dist) return false;
    return lhs <= rhs;
}

// reading A12: the interpolation degree resolves the kernel's oscillation only while the
// wavenumber times the larger cluster diameter stays below kadm (ties inadmissible)
static bool resolved(const Cluster& A, const Cluster& B, double kabs, double kadm) {
    if (!(kadm > 0.0) || kabs == 0.0) return true;
    const double lhs = kabs * 2.0 * std::max(A.rad, B.rad);
    if (std::fabs(lhs - kadm) <= 1e-12 * kadm) return false;
    return lhs <= kadm;
}

template <class T>
static void h2_partition(H2<T>& H, int64_t t, int64_t s) {
    const Cluster& A = H.cl[t];
    const Cluster& B = H.cl[s];
    const double kabs = H.S->pde == PDE_HELMHOLTZ ? std::abs(H.S->kappa) : 0.0;
    if (admissible(A, B, H.eta) && resolved(A, B, kabs, H.kadm)) {
        H.far.push_back({t, s});
        return;
    }
    if (A.lev == H.leaf) {
        H.near.push_back({t, s});
        return;
    }
    for (int a = 0; a < 4; ++a)
        for (int b = 0; b < 4; ++b)
            h2_partition(H, H.cluster_index(A.lev + 1, A.f, 2 * A.i + (a >> 1), 2 * A.j + (a & 1)),
                         H.cluster_index(B.lev + 1, B.f, 2 * B.i + (b >> 1), 2 * B.j + (b & 1)));
}

// physical point of Chebyshev node (a1,a2) of a cluster
static void cluster_node(const Geom& G, const Cluster& C, const std::vector<double>& xi, int a1,
                         int a2, double x[3]) {
    const double w = 1.0 / (double)(1 << C.lev);
    gamma(G, C.f, (C.i + xi[a1]) * w, (C.j + xi[a2]) * w, x);
}

// the near-field element pairs that belong to near leaf pair (t, s)
template <class T>
static void leaf_elements(const H2<T>& H, int64_t c, std::vector<int64_t>& els) {
    const Cluster& C = H.cl[c];
    const int m = 1 << (H.S->K.L - C.lev);
    const int n = H.S->K.nel;
    els.clear();
    for (int a = 0; a < m; ++a)
        for (int b = 0; b < m; ++b)
            els.push_back(((int64_t)C.f * n + (C.i * m + a)) * n + (C.j * m + b));
}

template <class T>
static void h2_build(H2<T>& H, const Space& S, int q, double eta, int leaf, int qg, int qs,
                     bool assemble_near, double kadm) {
    if (leaf < 0 || leaf > S.K.L) throw std::runtime_error("leaf level must lie in [0, L]");
    if (q < 1) throw std::runtime_error("q must be positive");
    H.S = &S;
    H.q = q;
    H.eta = eta;
    H.kadm = kadm;
    H.leaf = leaf;
    H.qg = qg;
    H.qs = qs;
    H.qm = (q + S.K.d + 1) / 2;  // ceil((q+d)/2), reading A13
    // clusters of all levels 0..leaf
    H.lev_off.assign(leaf + 2, 0);
    for (int l = 0; l <= leaf; ++l)
        H.lev_off[l + 1] = H.lev_off[l] + (int64_t)S.G.npatch * ((int64_t)1 << (2 * l));
    H.cl.resize(H.lev_off[leaf + 1]);
    for (int l = 0; l <= leaf; ++l) {
        const int n = 1 << l;
        for (int f = 0; f < S.G.npatch; ++f)
            for (int i = 0; i < n; ++i)
                for (int j = 0; j < n; ++j) {
                    Cluster& C = H.cl[H.cluster_index(l, f, i, j)];
                    C.lev = l;
                    C.f = f;
                    C.i = i;
                    C.j = j;
                    cluster_ball(S.G, C);
                }
    }
    // block partition, starting from all pairs of patches
    for (int f = 0; f < S.G.npatch; ++f)
        for (int g = 0; g < S.G.npatch; ++g)
            h2_partition(H, H.cluster_index(0, f, 0, 0), H.cluster_index(0, g, 0, 0));
    std::sort(H.far.begin(), H.far.end());
    std::sort(H.near.begin(), H.near.end());
    // interpolation nodes and transfer matrices
    H.xi = cheb_nodes(q);
    for (int b = 0; b < 2; ++b) {
        H.E[b].assign(q * q, 0.0);
        for (int ap = 0; ap < q; ++ap)
            for (int a = 0; a < q; ++a) H.E[b][ap * q + a] = lagrange(H.xi, a, 0.5 * (b + H.xi[ap]));
    }
    // 1-D leaf moments by Gauss with qm points per element (exact, reading A13)
    const int m = 1 << (S.K.L - leaf);  // elements per leaf per direction
    const int nleaf1 = 1 << leaf;
    H.nloc = (m - 1) * S.K.r + S.K.d + 1;
    const Rule g = gauss01(H.qm);
    H.V1.assign(nleaf1, std::vector<double>(q * H.nloc, 0.0));
    for (int i = 0; i < nleaf1; ++i) {
        const int first = H.leaf_first_basis(i);
        for (int el = i * m; el < (i + 1) * m; ++el) {
            const int sp = elem_span(S.K, el);
            for (int k = 0; k < H.qm; ++k) {
                const double s = (el + g.x[k]) * S.h;
                const double sl = (s - (double)i / nleaf1) * nleaf1;  // leaf-local coordinate
                for (int a = 0; a < q; ++a) {
                    const double La = lagrange(H.xi, a, sl);
                    for (int jl = 0; jl < H.nloc; ++jl) {
                        const double bv = bspline(S.K, first + jl, S.K.d, s, sp);
                        H.V1[i][a * H.nloc + jl] += g.w[k] * S.h * La * bv;
                    }
                }
            }
        }
    }
    // 0-form lifting: the moments carry the surface element, so a leaf's table is no longer
    // a product of 1-D tables; Vd[leaf][(a1 q + a2) nloc^2 + m1 nloc + m2] is the integral over
    // the leaf of L_a1 L_a2 b_{first1+m1} b_{first2+m2} kappa by qg x qg Gauss points per element
    if (S.form == 0) {
        const Rule gq = gauss01(qg);
        const int nl2 = H.nloc * H.nloc, nbl = (S.K.d + 1) * (S.K.d + 1);
        H.Vd.assign((size_t)S.G.npatch * nleaf1 * nleaf1, std::vector<double>((size_t)q * q * nl2, 0.0));
        std::vector<double> ph(nbl);
        for (int f = 0; f < S.G.npatch; ++f)
            for (int i = 0; i < nleaf1; ++i)
                for (int j = 0; j < nleaf1; ++j) {
                    std::vector<double>& V = H.Vd[((size_t)f * nleaf1 + i) * nleaf1 + j];
                    const int fi = H.leaf_first_basis(i), fj = H.leaf_first_basis(j);
                    for (int e1 = i * m; e1 < (i + 1) * m; ++e1)
                        for (int e2 = j * m; e2 < (j + 1) * m; ++e2) {
                            const Elem E{f, e1, e2};
                            for (int k1 = 0; k1 < qg; ++k1)
                                for (int k2 = 0; k2 < qg; ++k2) {
                                    const double s = (e1 + gq.x[k1]) * S.h, t = (e2 + gq.x[k2]) * S.h;
                                    elem_basis(S, E, s, t, ph.data());
                                    const double w = gq.w[k1] * gq.w[k2] * S.h * S.h * surf_elem(S.G, f, s, t);
                                    const double sl = s * nleaf1 - i, tl = t * nleaf1 - j;
                                    for (int a1 = 0; a1 < q; ++a1)
                                        for (int a2 = 0; a2 < q; ++a2) {
                                            const double La = lagrange(H.xi, a1, sl) * lagrange(H.xi, a2, tl) * w;
                                            for (int l = 0; l < nbl; ++l) {
                                                const int m1 = elem_first_basis(S.K, e1) + l / (S.K.d + 1) - fi;
                                                const int m2 = elem_first_basis(S.K, e2) + l % (S.K.d + 1) - fj;
                                                V[(size_t)(a1 * q + a2) * nl2 + m1 * H.nloc + m2] += La * ph[l];
                                            }
                                        }
                                }
                        }
                }
    }
    // coupling blocks K[(a1,a2),(b1,b2)] = k(gamma_tau(xi_a), gamma_sigma(xi_b))
    const int q2 = q * q;
    H.K.assign(H.far.size() * (size_t)q2 * q2, T(0));
    const int64_t nblk = (int64_t)H.far.size();
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t blk = 0; blk < nblk; ++blk) {
        const Cluster& A = H.cl[H.far[blk].first];
        const Cluster& B = H.cl[H.far[blk].second];
        for (int a = 0; a < q2; ++a) {
            double x[3];
            cluster_node(S.G, A, H.xi, a / q, a % q, x);
            for (int b = 0; b < q2; ++b) {
                double y[3];
                cluster_node(S.G, B, H.xi, b / q, b % q, y);
                H.K[blk * q2 * q2 + a * q2 + b] = kernel_r<T>(S.pde, S.kappa, dist3(x, y));
            }
        }
    }
    // near field: the same element-pair integrals as the dense matrix, over near leaf pairs
    H.have_near = assemble_near;
    if (assemble_near) {
        H.near_rows.assign(S.ndof, std::map<int64_t, T>());
        SideFn F;
        const int nb = side_nb(S, F);
        std::vector<T> Bk(nb * nb);
        std::vector<int64_t> et, es;
        for (const auto& pr : H.near) {
            leaf_elements(H, pr.first, et);
            leaf_elements(H, pr.second, es);
            for (int64_t e1 : et) {
                const Elem E1 = elem_of(S, e1);
                for (int64_t e2 : es) {
                    const Elem E2 = elem_of(S, e2);
                    pair_block<T>(S, F, F, e1, e2, qg, qs, Bk.data());
                    for (int i = 0; i < nb; ++i)
                        for (int j = 0; j < nb; ++j)
                            H.near_rows[local_dof(S, E1, i)][local_dof(S, E2, j)] += Bk[i * nb + j];
                }
            }
        }
    }
}

// moments of every leaf: m_tau[a1,a2] = sum_g V_tau[(a1,a2), g] x_g (forward transform)
template <class T>
static void h2_forward(const H2<T>& H, const T* x, std::vector<T>& mom) {
    const Space& S = *H.S;
    const int q = H.q, q2 = q * q, nl = 1 << H.leaf;
    // (timing mode: independent clusters in parallel; each cluster's sums are unchanged)
#pragma omp parallel for collapse(3) schedule(static)
    for (int f = 0; f < S.G.npatch; ++f)
        for (int i = 0; i < nl; ++i)
            for (int j = 0; j < nl; ++j) {
                const int64_t c = H.cluster_index(H.leaf, f, i, j);
                const int fi = H.leaf_first_basis(i), fj = H.leaf_first_basis(j);
                for (int a1 = 0; a1 < q; ++a1)
                    for (int a2 = 0; a2 < q; ++a2) {
                        T acc = T(0);
                        for (int m1 = 0; m1 < H.nloc; ++m1)
                            for (int m2 = 0; m2 < H.nloc; ++m2) {
                                const double v = S.form == 0
                                                     ? H.Vd[((size_t)f * nl + i) * nl + j][(size_t)(a1 * q + a2) * H.nloc * H.nloc +
                                                                                           m1 * H.nloc + m2]
                                                     : H.V1[i][a1 * H.nloc + m1] * H.V1[j][a2 * H.nloc + m2];
                                acc += v * x[dof_index(S, f, fi + m1, fj + m2)];
                            }
                        mom[c * q2 + a1 * q + a2] = acc;
                    }
            }
}

// upward transfer: m_P = sum over the four children c of (E_c1 (x) E_c2)^T m_c
template <class T>
static void h2_upward(const H2<T>& H, std::vector<T>& mom) {
    const Space& S = *H.S;
    const int q = H.q, q2 = q * q;
    for (int l = H.leaf - 1; l >= 0; --l) {
        const int n = 1 << l;
#pragma omp parallel for collapse(3) schedule(static)
        for (int f = 0; f < S.G.npatch; ++f)
            for (int i = 0; i < n; ++i)
                for (int j = 0; j < n; ++j) {
                    const int64_t P = H.cluster_index(l, f, i, j);
                    for (int a = 0; a < q2; ++a) mom[P * q2 + a] = T(0);
                    for (int b1 = 0; b1 < 2; ++b1)
                        for (int b2 = 0; b2 < 2; ++b2) {
                            const int64_t c = H.cluster_index(l + 1, f, 2 * i + b1, 2 * j + b2);
                            for (int a1 = 0; a1 < q; ++a1)
                                for (int a2 = 0; a2 < q; ++a2) {
                                    T acc = T(0);
                                    for (int p1 = 0; p1 < q; ++p1)
                                        for (int p2 = 0; p2 < q; ++p2)
                                            acc += H.E[b1][p1 * q + a1] * H.E[b2][p2 * q + a2] *
                                                   mom[c * q2 + p1 * q + p2];
                                    mom[P * q2 + a1 * q + a2] += acc;
                                }
                        }
                }
    }
}

// moments of every cluster integrated directly (no transfer); used to pin the transfer
template <class T>
static void h2_direct_moments(const H2<T>& H, const T* x, std::vector<T>& mom) {
    const Space& S = *H.S;
    const int q = H.q, q2 = q * q;
    const int nq = S.form == 0 ? H.qg : H.qm;  // 0-form: the leaf tables' rule
    const Rule g = gauss01(nq);
    const int nb = (S.K.d + 1) * (S.K.d + 1);
    std::vector<double> ph(nb);
    std::fill(mom.begin(), mom.end(), T(0));
    for (int l = 0; l <= H.leaf; ++l) {
        const int n = 1 << l;
        const int m = 1 << (S.K.L - l);
        for (int f = 0; f < S.G.npatch; ++f)
            for (int i = 0; i < n; ++i)
                for (int j = 0; j < n; ++j) {
                    const int64_t c = H.cluster_index(l, f, i, j);
                    for (int ei = i * m; ei < (i + 1) * m; ++ei)
                        for (int ej = j * m; ej < (j + 1) * m; ++ej) {
                            Elem E{f, ei, ej};
                            for (int k1 = 0; k1 < nq; ++k1)
                                for (int k2 = 0; k2 < nq; ++k2) {
                                    const double s = (ei + g.x[k1]) * S.h, t = (ej + g.x[k2]) * S.h;
                                    elem_basis(S, E, s, t, ph.data());
                                    T xv = T(0);
                                    for (int lb = 0; lb < nb; ++lb) xv += ph[lb] * x[local_dof(S, E, lb)];
                                    const double w = g.w[k1] * g.w[k2] * S.h * S.h * (S.form == 0 ? surf_elem(S.G, f, s, t) : 1.0);
                                    const double sl = s * n - i, tl = t * n - j;
                                    for (int a1 = 0; a1 < q; ++a1)
                                        for (int a2 = 0; a2 < q; ++a2)
                                            mom[c * q2 + a1 * q + a2] +=
                                                w * lagrange(H.xi, a1, sl) * lagrange(H.xi, a2, tl) * xv;
                                }
                        }
                }
    }
}

// coupling: lv_tau += K_tau,sigma m_sigma over the far list
template <class T>
static void h2_coupling(const H2<T>& H, const std::vector<T>& mom, std::vector<T>& lv) {
    const int q2 = H.q * H.q;
    std::fill(lv.begin(), lv.end(), T(0));
    // blocks in list order; the list is sorted by target, so the runs of one target are
    // independent of each other (timing mode: runs in parallel, each in list order)
    std::vector<size_t> run{0};
    for (size_t blk = 1; blk < H.far.size(); ++blk)
        if (H.far[blk].first != H.far[blk - 1].first) run.push_back(blk);
    run.push_back(H.far.size());
    const int64_t nruns = (int64_t)run.size() - 1;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t k = 0; k < nruns; ++k)
        for (size_t blk = run[k]; blk < run[k + 1]; ++blk) {
            const int64_t t = H.far[blk].first, s = H.far[blk].second;
            for (int a = 0; a < q2; ++a) {
                T acc = T(0);
                for (int b = 0; b < q2; ++b) acc += H.K[blk * q2 * q2 + a * q2 + b] * mom[s * q2 + b];
                lv[t * q2 + a] += acc;
            }
        }
}

// downward transfer: lv_c += (E_c1 (x) E_c2) lv_P
template <class T>
static void h2_downward(const H2<T>& H, std::vector<T>& lv) {
    const Space& S = *H.S;
    const int q = H.q, q2 = q * q;
    for (int l = 1; l <= H.leaf; ++l) {
        const int n = 1 << l;
#pragma omp parallel for collapse(3) schedule(static)
        for (int f = 0; f < S.G.npatch; ++f)
            for (int i = 0; i < n; ++i)
                for (int j = 0; j < n; ++j) {
                    const int64_t c = H.cluster_index(l, f, i, j);
                    const int64_t P = H.cluster_index(l - 1, f, i / 2, j / 2);
                    const int b1 = i & 1, b2 = j & 1;
                    for (int p1 = 0; p1 < q; ++p1)
                        for (int p2 = 0; p2 < q; ++p2) {
                            T acc = T(0);
                            for (int a1 = 0; a1 < q; ++a1)
                                for (int a2 = 0; a2 < q; ++a2)
                                    acc += H.E[b1][p1 * q + a1] * H.E[b2][p2 * q + a2] *
                                           lv[P * q2 + a1 * q + a2];
                            lv[c * q2 + p1 * q + p2] += acc;
                        }
                }
    }
}

// backward transform for one DOF: y_g = sum over leaves tau touching g of (V_tau^T lv_tau)_g
template <class T>
static T h2_backward_dof(const H2<T>& H, const std::vector<T>& lv, int64_t g) {
    const Space& S = *H.S;
    const int q = H.q, q2 = q * q, nl = 1 << H.leaf;
    const int nb = S.K.nb;
    const int f = (int)(g / ((int64_t)nb * nb));
    const int j1 = (int)((g / nb) % nb), j2 = (int)(g % nb);
    T acc = T(0);
    for (int i = 0; i < nl; ++i) {
        const int m1 = j1 - H.leaf_first_basis(i);
        if (m1 < 0 || m1 >= H.nloc) continue;
        for (int j = 0; j < nl; ++j) {
            const int m2 = j2 - H.leaf_first_basis(j);
            if (m2 < 0 || m2 >= H.nloc) continue;
            const int64_t c = H.cluster_index(H.leaf, f, i, j);
            for (int a1 = 0; a1 < q; ++a1)
                for (int a2 = 0; a2 < q; ++a2) {
                    const double v = S.form == 0
                                         ? H.Vd[((size_t)f * nl + i) * nl + j][(size_t)(a1 * q + a2) * H.nloc * H.nloc +
                                                                               m1 * H.nloc + m2]
                                         : H.V1[i][a1 * H.nloc + m1] * H.V1[j][a2 * H.nloc + m2];
                    acc += v * lv[c * q2 + a1 * q + a2];
                }
        }
    }
    return acc;
}

// near-field rows for a subset of DOFs only (the rest stays empty); used to time the
// near-field product on a sample of rows of a problem whose full near field is too costly
template <class T>
static void h2_near_rows_subset(H2<T>& H, const int64_t* rows, int64_t nrows) {
    const Space& S = *H.S;
    H.near_rows.assign(S.ndof, std::map<int64_t, T>());
    SideFn F;
    const int nb = side_nb(S, F);
    const int d = S.K.d, nbs = S.K.nb, nel = S.K.nel;
    const int m = 1 << (S.K.L - H.leaf);
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t r = 0; r < nrows; ++r) {
        std::vector<T> Bk(nb * nb);
        std::vector<int64_t> es;
        const int64_t g = rows[r];
        const int f = (int)(g / ((int64_t)nbs * nbs));
        const int j1 = (int)((g / nbs) % nbs), j2 = (int)(g % nbs);
        for (int i1 = 0; i1 < nel; ++i1) {
            const int l1 = j1 - elem_first_basis(S.K, i1);
            if (l1 < 0 || l1 > d) continue;
            for (int i2 = 0; i2 < nel; ++i2) {
                const int l2 = j2 - elem_first_basis(S.K, i2);
                if (l2 < 0 || l2 > d) continue;
                const int64_t e1 = ((int64_t)f * nel + i1) * nel + i2;
                const int64_t tl = H.cluster_index(H.leaf, f, i1 / m, i2 / m);
                auto lo = std::lower_bound(H.near.begin(), H.near.end(), std::make_pair(tl, (int64_t)-1));
                for (auto it = lo; it != H.near.end() && it->first == tl; ++it) {
                    leaf_elements(H, it->second, es);
                    for (int64_t e2 : es) {
                        const Elem E2 = elem_of(S, e2);
                        pair_block<T>(S, F, F, e1, e2, H.qg, H.qs, Bk.data());
                        const int il = l1 * (d + 1) + l2;
                        for (int j = 0; j < nb; ++j) H.near_rows[g][local_dof(S, E2, j)] += Bk[il * nb + j];
                    }
                }
            }
        }
    }
    H.have_near = true;
}

// far-field part of y = A x for all DOFs (forward, upward, coupling, downward, backward)
template <class T>
static void h2_far_apply(const H2<T>& H, const T* x, std::vector<T>& lv) {
    const int q2 = H.q * H.q;
    std::vector<T> mom(H.cl.size() * q2, T(0));
    lv.assign(H.cl.size() * q2, T(0));
    h2_forward(H, x, mom);
    h2_upward(H, mom);
    h2_coupling(H, mom, lv);
    h2_downward(H, lv);
}

// y = (A_near + A_far) x with an assembled near field
template <class T>
static void h2_apply(const H2<T>& H, const T* x, T* y) {
    if (!H.have_near) throw std::runtime_error("near field not assembled");
    std::vector<T> lv;
    h2_far_apply(H, x, lv);
    for (int64_t g = 0; g < H.S->ndof; ++g) {
        T acc = h2_backward_dof(H, lv, g);
        for (const auto& kv : H.near_rows[g]) acc += kv.second * x[kv.first];
        y[g] = acc;
    }
}

// y at selected rows only, computing the near-field rows by quadrature on the fly (for
// large problems whose full near field the oracle does not assemble)
template <class T>
static void h2_apply_rows(const H2<T>& H, const T* x, const int64_t* rows, int64_t nrows, T* y,
                          bool far_part, bool near_part) {
    const Space& S = *H.S;
    std::vector<T> lv;
    if (far_part) h2_far_apply(H, x, lv);
    SideFn F;
    const int nb = side_nb(S, F);
    const int d = S.K.d, nbs = S.K.nb, nel = S.K.nel;
    const int m = 1 << (S.K.L - H.leaf);
    // (timing mode: rows in parallel, each row's sum unchanged)
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t r = 0; r < nrows; ++r) {
        std::vector<T> Bk(nb * nb);
        std::vector<int64_t> es;
        const int64_t g = rows[r];
        T acc = far_part ? h2_backward_dof(H, lv, g) : T(0);
        if (near_part && H.have_near) {
            for (const auto& kv : H.near_rows[g]) acc += kv.second * x[kv.first];
        } else if (near_part) {
            const int f = (int)(g / ((int64_t)nbs * nbs));
            const int j1 = (int)((g / nbs) % nbs), j2 = (int)(g % nbs);
            // elements whose local basis contains g
            for (int i1 = 0; i1 < nel; ++i1) {
                const int l1 = j1 - elem_first_basis(S.K, i1);
                if (l1 < 0 || l1 > d) continue;
                for (int i2 = 0; i2 < nel; ++i2) {
                    const int l2 = j2 - elem_first_basis(S.K, i2);
                    if (l2 < 0 || l2 > d) continue;
                    const int64_t e1 = ((int64_t)f * nel + i1) * nel + i2;
                    const int64_t tl = H.cluster_index(H.leaf, f, i1 / m, i2 / m);
                    auto lo = std::lower_bound(H.near.begin(), H.near.end(),
                                               std::make_pair(tl, (int64_t)-1));
                    for (auto it = lo; it != H.near.end() && it->first == tl; ++it) {
                        leaf_elements(H, it->second, es);
                        for (int64_t e2 : es) {
                            const Elem E2 = elem_of(S, e2);
                            pair_block<T>(S, F, F, e1, e2, H.qg, H.qs, Bk.data());
                            const int il = l1 * (d + 1) + l2;
                            for (int j = 0; j < nb; ++j) acc += Bk[il * nb + j] * x[local_dof(S, E2, j)];
                        }
                    }
                }
            }
        }
        y[r] = acc;
    }
}

// ---------------------------------------------------------------------------------------
// Restarted GMRES(m) (Sec. 4 "Solution of the System of Linear Equations"; the example
// program's GMRES with identity preconditioner; reading A15): x0 = 0, modified
// Gram-Schmidt Arnoldi, Givens rotations, convergence on the Arnoldi residual estimate,
// true residual recomputed at the end.  Inner products are conjugate-linear in the first
// argument.
// ---------------------------------------------------------------------------------------
static double absval(double v) { return std::fabs(v); }
static double absval(const cplx& v) { return std::abs(v); }
static double conjv(double v) { return v; }
static cplx conjv(const cplx& v) { return std::conj(v); }

template <class T>
static double vnorm(const std::vector<T>& v) {
    double s = 0.0;
    for (const T& a : v) s += absval(a) * absval(a);
    return std::sqrt(s);
}

template <class T, class MV>
static int gmres(int64_t n, MV matvec, const T* b, T* x, double tol, int m, int maxit, int* iters,
                 double* relres) {
    std::vector<T> r(n), w(n);
    std::fill(x, x + n, T(0));
    std::vector<T> bv(b, b + n);
    const double bnorm = vnorm<T>(bv);
    *iters = 0;
    if (bnorm == 0.0) {
        *relres = 0.0;
        return 0;
    }
    std::vector<std::vector<T>> V(m + 1, std::vector<T>(n));
    std::vector<T> Hm((m + 1) * m), g(m + 1), sn(m), yv(m);
    std::vector<double> cs(m);
    int total = 0;
    bool converged = false;
    while (!converged && total < maxit) {
        matvec(x, r.data());
        for (int64_t i = 0; i < n; ++i) r[i] = b[i] - r[i];
        const double beta = vnorm<T>(r);
        if (beta / bnorm <= tol) {
            converged = true;
            break;
        }
        for (int64_t i = 0; i < n; ++i) V[0][i] = r[i] / beta;
        std::fill(g.begin(), g.end(), T(0));
        g[0] = beta;
        int k = 0;
        for (int j = 0; j < m && total < maxit; ++j) {
            matvec(V[j].data(), w.data());
            for (int i = 0; i <= j; ++i) {
                T hij = T(0);
                for (int64_t t = 0; t < n; ++t) hij += conjv(V[i][t]) * w[t];
                Hm[i * m + j] = hij;
                for (int64_t t = 0; t < n; ++t) w[t] -= hij * V[i][t];
            }
            const double hn = vnorm<T>(w);
            Hm[(j + 1) * m + j] = hn;
            if (hn > 0.0)
                for (int64_t t = 0; t < n; ++t) V[j + 1][t] = w[t] / hn;
            // apply the earlier rotations to the new column
            for (int i = 0; i < j; ++i) {
                const T a = Hm[i * m + j], c = Hm[(i + 1) * m + j];
                Hm[i * m + j] = cs[i] * a + sn[i] * c;
                Hm[(i + 1) * m + j] = -conjv(sn[i]) * a + cs[i] * c;
            }
            // new rotation zeroing H[j+1][j]
            const T a = Hm[j * m + j], c = Hm[(j + 1) * m + j];
            const double na = absval(a), nc = absval(c);
            const double nu = std::sqrt(na * na + nc * nc);
            if (na == 0.0) {
                cs[j] = 0.0;
                sn[j] = T(1);
            } else {
                cs[j] = na / nu;
                sn[j] = (a / na) * conjv(c) / nu;
            }
            Hm[j * m + j] = cs[j] * a + sn[j] * c;
            Hm[(j + 1) * m + j] = T(0);
            const T gj = g[j];
            g[j] = cs[j] * gj;
            g[j + 1] = -conjv(sn[j]) * gj;
            ++total;
            k = j + 1;
            if (absval(g[j + 1]) / bnorm <= tol || hn == 0.0) break;
        }
        // solve the k x k upper-triangular system and update x
        for (int i = k - 1; i >= 0; --i) {
            T s = g[i];
            for (int l = i + 1; l < k; ++l) s -= Hm[i * m + l] * yv[l];
            yv[i] = s / Hm[i * m + i];
        }
        for (int i = 0; i < k; ++i)
            for (int64_t t = 0; t < n; ++t) x[t] += yv[i] * V[i][t];
        if (k > 0 && absval(g[k]) / bnorm <= tol) {
            // confirm with the true residual before stopping
            matvec(x, r.data());
            for (int64_t i = 0; i < n; ++i) r[i] = b[i] - r[i];
            if (vnorm<T>(r) / bnorm <= tol) converged = true;
        }
    }
    matvec(x, r.data());
    for (int64_t i = 0; i < n; ++i) r[i] = b[i] - r[i];
    *relres = vnorm<T>(r) / bnorm;
    *iters = total;
    return (*relres <= tol) ? 0 : 1;
}

// ---------------------------------------------------------------------------------------
// Block-Jacobi preconditioning (an addition to the paper's method: its example program runs
// GMRES with the identity preconditioner).  Blocks are tiles of T x T consecutive B-spline
// indices of one patch (the last tile of a direction is smaller when T does not divide nb).
// Reading: the block D_b is the near-field part of A[b, b] (its far-field part vanishes
// whenever no admissible cluster pair joins two leaves that meet the tile, true for the
// workloads here and checked by the tests through the dense operator).  D_b^{-1} is applied
// by LU with partial pivoting.  Right preconditioning: GMRES on A M^{-1}, x = M^{-1} u, so
// the residual GMRES sees is the true residual.
// Learned-correction targets: the block least-squares approximate inverse on N(b), the tile
// extended by `ring` B-spline indices on each side inside the patch (see bj_target).
// ---------------------------------------------------------------------------------------
struct Tile {
    int f, j1a, j1b, j2a, j2b;  // [j1a, j1b) x [j2a, j2b) of patch f
};

static std::vector<Tile> make_tiles(const Space& S, int T) {
    std::vector<Tile> out;
    const int nb = S.K.nb;
    const int nt = (nb + T - 1) / T;
    for (int f = 0; f < S.G.npatch; ++f)
        for (int t1 = 0; t1 < nt; ++t1)
            for (int t2 = 0; t2 < nt; ++t2)
                out.push_back({f, t1 * T, std::min(nb, (t1 + 1) * T), t2 * T, std::min(nb, (t2 + 1) * T)});
    return out;
}

// DOFs of a (possibly ring-extended) tile, j1 outer, j2 inner
static std::vector<int64_t> tile_dofs(const Space& S, const Tile& t, int ring) {
    const int nb = S.K.nb;
    std::vector<int64_t> g;
    for (int j1 = std::max(0, t.j1a - ring); j1 < std::min(nb, t.j1b + ring); ++j1)
        for (int j2 = std::max(0, t.j2a - ring); j2 < std::min(nb, t.j2b + ring); ++j2)
            g.push_back(dof_index(S, t.f, j1, j2));
    return g;
}

template <class T>
static std::vector<T> near_block(const H2<T>& H, const std::vector<int64_t>& rows,
                                 const std::vector<int64_t>& cols) {
    std::vector<T> D(rows.size() * cols.size(), T(0));
    for (size_t i = 0; i < rows.size(); ++i) {
        const auto& m = H.near_rows.at(rows[i]);
        for (size_t j = 0; j < cols.size(); ++j) {
            auto it = m.find(cols[j]);
            if (it != m.end()) D[i * cols.size() + j] = it->second;
        }
    }
    return D;
}

// LU with partial pivoting (largest modulus in the column), in place; piv[k] = row swapped
// with row k at step k
template <class T>
static void lu_factor(std::vector<T>& A, int n, std::vector<int>& piv) {
    piv.assign(n, 0);
    for (int k = 0; k < n; ++k) {
        int p = k;
        for (int i = k + 1; i < n; ++i)
            if (absval(A[i * n + k]) > absval(A[p * n + k])) p = i;
        if (absval(A[p * n + k]) == 0.0) throw std::runtime_error("singular block");
        piv[k] = p;
        if (p != k)
            for (int j = 0; j < n; ++j) std::swap(A[k * n + j], A[p * n + j]);
        for (int i = k + 1; i < n; ++i) {
            const T l = A[i * n + k] / A[k * n + k];
            A[i * n + k] = l;
            for (int j = k + 1; j < n; ++j) A[i * n + j] -= l * A[k * n + j];
        }
    }
}

template <class T>
static void lu_solve(const std::vector<T>& LU, int n, const std::vector<int>& piv, T* b) {
    for (int k = 0; k < n; ++k)
        if (piv[k] != k) std::swap(b[k], b[piv[k]]);
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < i; ++j) b[i] -= LU[i * n + j] * b[j];
    for (int i = n - 1; i >= 0; --i) {
        for (int j = i + 1; j < n; ++j) b[i] -= LU[i * n + j] * b[j];
        b[i] /= LU[i * n + i];
    }
}

template <class T>
struct BJ {
    std::vector<Tile> tiles;
    std::vector<std::vector<int64_t>> dofs;
    std::vector<std::vector<T>> LU;
    std::vector<std::vector<int>> piv;
};

template <class T>
static void bj_build(const H2<T>& H, int Tsz, BJ<T>& B) {
    B.tiles = make_tiles(*H.S, Tsz);
    B.dofs.clear();
    B.LU.clear();
    B.piv.clear();
    for (const Tile& t : B.tiles) {
        B.dofs.push_back(tile_dofs(*H.S, t, 0));
        const auto& g = B.dofs.back();
        B.LU.push_back(near_block(H, g, g));
        B.piv.emplace_back();
        lu_factor(B.LU.back(), (int)g.size(), B.piv.back());
    }
}

template <class T>
static void bj_apply(const BJ<T>& B, const T* r, T* z) {
    for (size_t k = 0; k < B.tiles.size(); ++k) {
        const auto& g = B.dofs[k];
        std::vector<T> v(g.size());
        for (size_t i = 0; i < g.size(); ++i) v[i] = r[g[i]];
        lu_solve(B.LU[k], (int)g.size(), B.piv[k], v.data());
        for (size_t i = 0; i < g.size(); ++i) z[g[i]] = v[i];
    }
}

// Learned-correction target: the block least-squares approximate inverse of tile b,
// X_b = argmin_X ||A[N(b), b] X - I[N(b), b]||_F = (A_Nb^H A_Nb)^{-1} A_bb^H, with A_Nb the
// near-field rows of N(b) in the columns of b (the tile extended by `ring` indices per
// side).  For ring 0 it is D_b^{-1}.
template <class T>
static std::vector<T> bj_target(const H2<T>& H, const Tile& t, int ring) {
    const auto gb = tile_dofs(*H.S, t, 0);
    const auto gn = tile_dofs(*H.S, t, ring);
    const int n = (int)gn.size(), nbk = (int)gb.size();
    const std::vector<T> ANb = near_block(H, gn, gb);  // n x nbk
    std::vector<T> G((size_t)nbk * nbk, T(0));
    for (int i = 0; i < nbk; ++i)
        for (int j = 0; j < nbk; ++j) {
            T s = T(0);
            for (int k = 0; k < n; ++k) s += conjv(ANb[(size_t)k * nbk + i]) * ANb[(size_t)k * nbk + j];
            G[(size_t)i * nbk + j] = s;
        }
    const std::vector<T> D = near_block(H, gb, gb);
    std::vector<int> piv;
    lu_factor(G, nbk, piv);
    std::vector<T> X((size_t)nbk * nbk);
    std::vector<T> col(nbk);
    for (int j = 0; j < nbk; ++j) {
        for (int i = 0; i < nbk; ++i) col[i] = conjv(D[(size_t)j * nbk + i]);  // column j of D^H
        lu_solve(G, nbk, piv, col.data());
        for (int i = 0; i < nbk; ++i) X[(size_t)i * nbk + j] = col[i];
    }
    return X;
}

// Features of a tile for the correction network (reading, not in the paper): the parameter
// box of the elements that the tile's B-splines meet; at the 4 x 4 cell centres of a
// uniform grid of the box, the Jacobian of the patch map with respect to the box
// coordinates (analytic derivatives): d/ds x, y, z then d/dt x, y, z per point, points row
// by row; then Re kappa / 10, Im kappa / 10, level / 8.
static void tile_features(const Space& S, const Tile& t, double* out) {
    const int d = S.K.d, r = S.K.r, nel = 1 << S.K.L;
    const double h = 1.0 / nel;
    auto box = [&](int ja, int jb, double& lo, double& hi) {  // B-splines [ja, jb)
        int elo = ja - d <= 0 ? 0 : (ja - d + r - 1) / r;
        int ehi = std::min((jb - 1) / r, nel - 1);
        lo = elo * h;
        hi = (ehi + 1) * h;
    };
    double s0, s1, u0, u1;
    box(t.j1a, t.j1b, s0, s1);
    box(t.j2a, t.j2b, u0, u1);
    for (int p = 0; p < 16; ++p) {
        const double s = s0 + (p / 4 + 0.5) * 0.25 * (s1 - s0), u = u0 + (p % 4 + 0.5) * 0.25 * (u1 - u0);
        double x[3], xs[3], xt[3];
        gamma(S.G, t.f, s, u, x, xs, xt);
        for (int k = 0; k < 3; ++k) {
            out[p * 6 + k] = xs[k] * (s1 - s0);
            out[p * 6 + 3 + k] = xt[k] * (u1 - u0);
        }
    }
    out[96] = S.kappa.real() / 10.0;
    out[97] = S.kappa.imag() / 10.0;
    out[98] = S.K.L / 8.0;
}

// ---------------------------------------------------------------------------------------
// Maxwell single layer: the electric wave equation (App. A (MP)) through the single-layer
// ansatz (MS) of App. B, on the div-conforming spaces S^1 of App. E.
//
// Reference space (App. E): S^1 = S_p (x) S_{p-1}  x  S_{p-1} (x) S_p on the unit square,
// p >= 1, the degree p - 1 factor on the truncated knot vector (the clamped uniform knots of
// degree p - 1).  Component 0 is the field b^p_j1(s) b^{p-1}_j2(t) e_s, component 1 the
// field b^{p-1}_j1(s) b^p_j2(t) e_t.  Lifting by the Piola transform of div-conforming
// fields: j(gamma(s)) = D gamma(s) j_hat(s) / kappa(s) and div_Gamma j = div_hat j_hat /
// kappa(s), so with d sigma = kappa ds the surface element cancels.  Testing the trace of
// (MS) with v and moving the gradient onto v by integration by parts on the closed surface,
//   a(j, v) = int int G(x, y) [ j(y) . v(x) - kappa^-2 div j(y) div v(x) ] d sigma d sigma
//           = int int G [ (D gamma_x v_hat) . (D gamma_y j_hat) - kappa^-2 div v_hat div j_hat ] ds dt,
// with G the Helmholtz kernel of (HS).  The load vector of data E is int E . v d sigma =
// int E(gamma) . (D gamma v_hat) ds, and the field of a density is (MS) itself.
//
// Continuity (App. E: normal continuity gives S^1(Gamma) in H^-1/2(div)).  A reference field
// has a normal component on an edge only for the functions whose degree-p index is first or
// last (b^p_0 = 1 at 0, b^p_last = 1 at 1); its flux through the edge is the tangential
// B-spline, which the matching condition (App. D) carries onto the neighbour's.  Reading:
// the edge function of one patch and the one of the neighbour whose anchors (images of the
// point (edge coordinate, a(tangential factor))) coincide within 1e-10 of
// the largest anchor coordinate form one global function, the second with the sign
// -o1 o2 (o = +1 where the reference direction leaves its patch, at coordinate 1, and -1
// at coordinate 0), so that the flux leaving one patch enters the other.  An edge function
// without a partner (open surface) is dropped: the normal trace vanishes on the boundary.
// Global functions are numbered in the order of their first local function.
// ---------------------------------------------------------------------------------------
struct MSpace {
    Geom G;
    cplx kappa;
    int p = 1, L = 0, nel = 1;
    double h = 1.0;
    Knots Kp, Kq;          // degree p and p - 1 on 2^L elements
    int nbp = 0, nbq = 0;  // functions per direction of each degree
    int64_t nelem = 0, nloc = 0, nglob = 0;
    std::vector<int64_t> glob;  // local -> global (-1: dropped)
    std::vector<int> sgn;       // sign of the local function in its global one
    Space geo;                  // scalar space of the same geometry and level (pair classification)
};

// local function of patch f, component c, indices (j1, j2)
static int64_t mlocal(const MSpace& S, int f, int c, int j1, int j2) {
    const int64_t per = (int64_t)S.nbp * S.nbq;
    return ((int64_t)f * 2 + c) * per + (c == 0 ? (int64_t)j1 * S.nbq + j2 : (int64_t)j1 * S.nbp + j2);
}

// Anchor a(j) of B-spline j along an edge: the mean of its Greville abscissa and the centre
// of its support [xi_j, xi_{j+d+1}].  Both are symmetric under reversal of the parameter; the
// Greville abscissae increase strictly with j and the centres do not decrease, so the
// anchors are distinct, and they lie strictly inside (0, 1) (the Greville abscissa alone
// puts the first and last function on the patch corners, the centre alone can repeat).
static double edge_anchor(const Knots& K, int j) {
    double gr;
    if (K.d == 0) {
        gr = 0.5 * (K.xi[j] + K.xi[j + 1]);
    } else {
        gr = 0.0;
        for (int k = 1; k <= K.d; ++k) gr += K.xi[j + k];
        gr /= K.d;
    }
    return 0.5 * (gr + 0.5 * (K.xi[j] + K.xi[j + K.d + 1]));
}

static MSpace make_mspace(const Geom& G, cplx kappa, int p, int L) {
    if (p < 1 || L < 0) throw std::runtime_error("S^1 needs p >= 1 and L >= 0");
    MSpace S;
    S.G = G;
    S.kappa = kappa;
    S.p = p;
    S.L = L;
    S.Kp = make_knots(p, 1, L);
    S.Kq = make_knots(p - 1, 1, L);
    S.nbp = S.Kp.nb;
    S.nbq = S.Kq.nb;
    S.nel = 1 << L;
    S.h = 1.0 / S.nel;
    S.geo = make_space(G, PDE_HELMHOLTZ, kappa, 0, 1, L);
    S.nelem = (int64_t)G.npatch * S.nel * S.nel;
    S.nloc = (int64_t)G.npatch * 2 * S.nbp * S.nbq;
    // anchors of the edge functions
    struct Anc {
        double x[3];
        int64_t lid;
        int o;
    };
    std::vector<Anc> an;
    std::vector<int> edge(S.nloc, 0), orient(S.nloc, 0);
    double scale = 0.0;
    for (int f = 0; f < G.npatch; ++f)
        for (int c = 0; c < 2; ++c)
            for (int e = 0; e < 2; ++e) {
                const int jn = e == 0 ? 0 : S.nbp - 1;
                for (int jt = 0; jt < S.nbq; ++jt) {
                    Anc a;
                    const double en = e == 0 ? 0.0 : 1.0, tg = edge_anchor(S.Kq, jt);
                    if (c == 0) {
                        gamma(G, f, en, tg, a.x);
                        a.lid = mlocal(S, f, 0, jn, jt);
                    } else {
                        gamma(G, f, tg, en, a.x);
                        a.lid = mlocal(S, f, 1, jt, jn);
                    }
                    a.o = e == 0 ? -1 : 1;
                    edge[a.lid] = 1;
                    orient[a.lid] = a.o;
                    for (double v : a.x) scale = std::max(scale, std::fabs(v));
                    an.push_back(a);
                }
            }
    const double tol = 1e-10 * std::max(scale, 1e-300);
    std::vector<int64_t> partner(S.nloc, -1);
    for (size_t a = 0; a < an.size(); ++a)
        for (size_t b = 0; b < an.size(); ++b) {
            if (a == b || dist3(an[a].x, an[b].x) > tol) continue;
            if (partner[an[a].lid] >= 0 && partner[an[a].lid] != an[b].lid)
                throw std::runtime_error("an edge function matches more than one neighbour");
            partner[an[a].lid] = an[b].lid;
        }
    S.glob.assign(S.nloc, -2);
    S.sgn.assign(S.nloc, 1);
    int64_t n = 0;
    for (int64_t l = 0; l < S.nloc; ++l) {
        if (S.glob[l] != -2) continue;
        if (!edge[l]) {
            S.glob[l] = n++;
        } else if (partner[l] < 0) {
            S.glob[l] = -1;
            S.sgn[l] = 0;
        } else {
            const int64_t m = partner[l];
            S.glob[l] = S.glob[m] = n++;
            S.sgn[l] = 1;
            S.sgn[m] = -orient[l] * orient[m];
        }
    }
    S.nglob = n;
    return S;
}

// derivative of B-spline j of degree K.d at x in span `span` (App. C recursion differentiated)
static double dbspline(const Knots& K, int j, double x, int span) {
    const int p = K.d;
    if (p == 0) return 0.0;
    double v = 0.0;
    const double d1 = K.xi[j + p] - K.xi[j], d2 = K.xi[j + p + 1] - K.xi[j + 1];
    if (d1 > 0.0) v += p * bspline(K, j, p - 1, x, span) / d1;
    if (d2 > 0.0) v -= p * bspline(K, j + 1, p - 1, x, span) / d2;
    return v;
}

// the 2 p (p + 1) local functions of element E at parameter (s, t): lifted field V (3 per
// function, D gamma times the reference field), reference divergence Dv and local index
static int m_nl(const MSpace& S) { return 2 * S.p * (S.p + 1); }

static void m_elem_eval(const MSpace& S, const Elem& E, double s, double t, double x[3], double* V, double* Dv,
                        int64_t* lid) {
    double xs[3], xt[3];
    gamma(S.G, E.f, s, t, x, xs, xt);
    const int p = S.p;
    const int spp1 = elem_span(S.Kp, E.i1), spp2 = elem_span(S.Kp, E.i2);
    const int spq1 = elem_span(S.Kq, E.i1), spq2 = elem_span(S.Kq, E.i2);
    int k = 0;
    for (int l1 = 0; l1 <= p; ++l1)  // component 0: degree p in s, p - 1 in t
        for (int l2 = 0; l2 < p; ++l2, ++k) {
            const int j1 = E.i1 + l1, j2 = E.i2 + l2;
            const double bs = bspline(S.Kp, j1, p, s, spp1), bt = bspline(S.Kq, j2, p - 1, t, spq2);
            for (int c = 0; c < 3; ++c) V[3 * k + c] = xs[c] * bs * bt;
            Dv[k] = dbspline(S.Kp, j1, s, spp1) * bt;
            lid[k] = mlocal(S, E.f, 0, j1, j2);
        }
    for (int l1 = 0; l1 < p; ++l1)  // component 1: degree p - 1 in s, p in t
        for (int l2 = 0; l2 <= p; ++l2, ++k) {
            const int j1 = E.i1 + l1, j2 = E.i2 + l2;
            const double bs = bspline(S.Kq, j1, p - 1, s, spq1), bt = bspline(S.Kp, j2, p, t, spp2);
            for (int c = 0; c < 3; ++c) V[3 * k + c] = xt[c] * bs * bt;
            Dv[k] = bs * dbspline(S.Kp, j2, t, spp2);
            lid[k] = mlocal(S, E.f, 1, j1, j2);
        }
}

// part: 0 the whole form, 1 the vector term only, 2 the divergence term only (with its
// factor -kappa^-2)
static void m_pair_block(const MSpace& S, int64_t e1, int64_t e2, int qg, int qs, int part, cplx* B) {
    const int nl = m_nl(S);
    for (int i = 0; i < nl * nl; ++i) B[i] = cplx(0.0);
    const Elem A = elem_of(S.geo, e1), Bel = elem_of(S.geo, e2);
    const PairInfo P = classify_pair(S.geo, e1, e2);
    const double h4 = S.h * S.h * S.h * S.h;
    const cplx ik2 = -1.0 / (S.kappa * S.kappa);
    const double wv = part == 2 ? 0.0 : 1.0;
    const cplx wd = part == 1 ? cplx(0.0) : ik2;
    std::vector<double> Vx(3 * nl), Vy(3 * nl), Dx(nl), Dy(nl);
    std::vector<int64_t> lx(nl), ly(nl);
    double xv[3], yv[3];
    auto accum = [&](double w) {
        const cplx kv = kernel_r<cplx>(PDE_HELMHOLTZ, S.kappa, dist3(xv, yv)) * w;
        for (int i = 0; i < nl; ++i)
            for (int j = 0; j < nl; ++j) {
                const double vv = Vx[3 * i] * Vy[3 * j] + Vx[3 * i + 1] * Vy[3 * j + 1] + Vx[3 * i + 2] * Vy[3 * j + 2];
                B[i * nl + j] += kv * (wv * vv + wd * (Dx[i] * Dy[j]));
            }
    };
    if (P.type == PAIR_REGULAR) {
        const Rule g = gauss01(qg);
        for (int a1 = 0; a1 < qg; ++a1)
            for (int a2 = 0; a2 < qg; ++a2) {
                double s, t;
                elem_param(S.geo, A, 0, g.x[a1], g.x[a2], s, t);
                m_elem_eval(S, A, s, t, xv, Vx.data(), Dx.data(), lx.data());
                for (int b1 = 0; b1 < qg; ++b1)
                    for (int b2 = 0; b2 < qg; ++b2) {
                        double s2, t2;
                        elem_param(S.geo, Bel, 0, g.x[b1], g.x[b2], s2, t2);
                        m_elem_eval(S, Bel, s2, t2, yv, Vy.data(), Dy.data(), ly.data());
                        accum(g.w[a1] * g.w[a2] * g.w[b1] * g.w[b2]);
                    }
            }
    } else {
        duffy_each(P.type, qs, [&](double xh1, double xh2, double yh1, double yh2, double w) {
            double s, t, s2, t2;
            elem_param(S.geo, A, P.k1, xh1, xh2, s, t);
            elem_param(S.geo, Bel, P.k2, yh1, yh2, s2, t2);
            m_elem_eval(S, A, s, t, xv, Vx.data(), Dx.data(), lx.data());
            m_elem_eval(S, Bel, s2, t2, yv, Vy.data(), Dy.data(), ly.data());
            accum(w);
        });
    }
    for (int i = 0; i < nl * nl; ++i) B[i] *= h4;
}

// local indices of element e's functions (in the order of m_elem_eval)
static void m_elem_lids(const MSpace& S, int64_t e, int64_t* lid) {
    const Elem E = elem_of(S.geo, e);
    int k = 0;
    for (int l1 = 0; l1 <= S.p; ++l1)
        for (int l2 = 0; l2 < S.p; ++l2) lid[k++] = mlocal(S, E.f, 0, E.i1 + l1, E.i2 + l2);
    for (int l1 = 0; l1 < S.p; ++l1)
        for (int l2 = 0; l2 <= S.p; ++l2) lid[k++] = mlocal(S, E.f, 1, E.i1 + l1, E.i2 + l2);
}

// dense Galerkin matrix on the global functions (row = test, column = trial), row-major
static void m_dense(const MSpace& S, int qg, int qs, int part, cplx* M) {
    const int64_t N = S.nglob, ne = S.nelem;
    const int nl = m_nl(S);
    std::fill(M, M + N * N, cplx(0.0));
    std::vector<std::vector<cplx>> rows(ne);
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t e1 = 0; e1 < ne; ++e1) {
        rows[e1].assign((size_t)ne * nl * nl, cplx(0.0));
        for (int64_t e2 = 0; e2 < ne; ++e2) m_pair_block(S, e1, e2, qg, qs, part, &rows[e1][(size_t)e2 * nl * nl]);
    }
    std::vector<int64_t> l1(nl), l2(nl);
    for (int64_t e1 = 0; e1 < ne; ++e1) {
        m_elem_lids(S, e1, l1.data());
        for (int64_t e2 = 0; e2 < ne; ++e2) {
            m_elem_lids(S, e2, l2.data());
            const cplx* B = &rows[e1][(size_t)e2 * nl * nl];
            for (int i = 0; i < nl; ++i) {
                const int64_t g = S.glob[l1[i]];
                if (g < 0) continue;
                for (int j = 0; j < nl; ++j) {
                    const int64_t hcol = S.glob[l2[j]];
                    if (hcol < 0) continue;
                    M[g * N + hcol] += (double)(S.sgn[l1[i]] * S.sgn[l2[j]]) * B[i * nl + j];
                }
            }
        }
        std::vector<cplx>().swap(rows[e1]);
    }
}

// Maxwell single layer compressed by the interpolation of Sec. 2 on the block partition of
// the scalar operators (same cluster tree, admissibility and Chebyshev nodes; the partition
// and the kernel blocks are those of the scalar H^2 operator of the element space of the
// same surface and wavenumber).  Element pairs inside near leaf pairs keep their Galerkin
// blocks.  For element pairs inside an admissible block (t, s) the kernel is replaced by its
// tensor interpolant in the two clusters' parameter squares, which turns the form into four
// scalar products, one per channel c (the three components of the lifted field, and the
// divergence with the factor -kappa^-2):
//   B[i][j] = sum_c w_c sum_a sum_b Mt_c[i][a] G(x_a^t, x_b^s) Ms_c[j][b],
//   Mt_c[i][a] = integral over the element of L_a^t times channel c of function i
// (qg x qg Gauss points per element, the element's parameter area h^2 included).  Every
// block interpolates directly on its own two clusters (no nested transfers).  part as in
// m_pair_block.  Dense output on the global functions, as m_dense.
static void m_h2_dense(const MSpace& S, int q, double eta, int leaf, int qg, int qs, double kadm, int part, cplx* M) {
    H2<cplx> H;
    h2_build(H, S.geo, q, eta, leaf, qg, qs, false, kadm);
    const int64_t N = S.nglob;
    const int nl = m_nl(S), q2 = q * q;
    const cplx ik2 = -1.0 / (S.kappa * S.kappa);
    const cplx wc[4] = {part == 2 ? 0.0 : 1.0, part == 2 ? 0.0 : 1.0, part == 2 ? 0.0 : 1.0,
                        part == 1 ? cplx(0.0) : ik2};
    std::fill(M, M + N * N, cplx(0.0));
    std::vector<int64_t> l1(nl), l2(nl);
    auto glue_block = [&](int64_t e1, int64_t e2, const cplx* B) {
        m_elem_lids(S, e1, l1.data());
        m_elem_lids(S, e2, l2.data());
        for (int i = 0; i < nl; ++i) {
            const int64_t g = S.glob[l1[i]];
            if (g < 0) continue;
            for (int j = 0; j < nl; ++j) {
                const int64_t hcol = S.glob[l2[j]];
                if (hcol < 0) continue;
                M[g * N + hcol] += (double)(S.sgn[l1[i]] * S.sgn[l2[j]]) * B[i * nl + j];
            }
        }
    };
    // channel moments of element e against the Lagrange polynomials of cluster c
    const Rule g = gauss01(qg);
    std::map<std::pair<int64_t, int64_t>, std::vector<double>> cache;
    auto moments = [&](int64_t c, int64_t e) -> const std::vector<double>& {
        auto it = cache.find({c, e});
        if (it != cache.end()) return it->second;
        std::vector<double> Mo((size_t)nl * 4 * q2, 0.0);  // [i][c][a]
        const Cluster& C = H.cl[c];
        const Elem E = elem_of(S.geo, e);
        const double n = (double)(1 << C.lev);
        std::vector<double> V(3 * nl), Dv(nl);
        std::vector<int64_t> lid(nl);
        double x[3];
        for (int k1 = 0; k1 < qg; ++k1)
            for (int k2 = 0; k2 < qg; ++k2) {
                const double s = (E.i1 + g.x[k1]) * S.h, t = (E.i2 + g.x[k2]) * S.h;
                m_elem_eval(S, E, s, t, x, V.data(), Dv.data(), lid.data());
                const double w = g.w[k1] * g.w[k2] * S.h * S.h;
                for (int a = 0; a < q2; ++a) {
                    const double La = lagrange(H.xi, a / q, s * n - C.i) * lagrange(H.xi, a % q, t * n - C.j) * w;
                    for (int i = 0; i < nl; ++i) {
                        double* m = &Mo[((size_t)i * 4) * q2 + a];
                        m[0] += La * V[3 * i];
                        m[q2] += La * V[3 * i + 1];
                        m[2 * q2] += La * V[3 * i + 2];
                        m[3 * q2] += La * Dv[i];
                    }
                }
            }
        return cache.emplace(std::make_pair(c, e), std::move(Mo)).first->second;
    };
    std::vector<cplx> B((size_t)nl * nl), T((size_t)nl * 4 * q2);
    std::vector<int64_t> et, es;
    for (size_t blk = 0; blk < H.far.size(); ++blk) {
        const int64_t t = H.far[blk].first, sc = H.far[blk].second;
        const cplx* K = &H.K[blk * (size_t)q2 * q2];
        leaf_elements(H, t, et);
        leaf_elements(H, sc, es);
        for (int64_t e2 : es) {
            // T[j][c][a] = sum_b K[a][b] Ms_c[j][b]
            const std::vector<double>& Ms = moments(sc, e2);
            for (int j = 0; j < nl; ++j)
                for (int c = 0; c < 4; ++c)
                    for (int a = 0; a < q2; ++a) {
                        cplx v = 0.0;
                        for (int b = 0; b < q2; ++b) v += K[a * q2 + b] * Ms[((size_t)j * 4 + c) * q2 + b];
                        T[((size_t)j * 4 + c) * q2 + a] = v;
                    }
            for (int64_t e1 : et) {
                const std::vector<double>& Mt = moments(t, e1);
                for (int i = 0; i < nl; ++i)
                    for (int j = 0; j < nl; ++j) {
                        cplx v = 0.0;
                        for (int c = 0; c < 4; ++c) {
                            cplx u = 0.0;
                            for (int a = 0; a < q2; ++a)
                                u += Mt[((size_t)i * 4 + c) * q2 + a] * T[((size_t)j * 4 + c) * q2 + a];
                            v += wc[c] * u;
                        }
                        B[i * nl + j] = v;
                    }
                glue_block(e1, e2, B.data());
            }
        }
    }
    // near element pairs: blocks in parallel, glued in list order
    std::vector<std::pair<int64_t, int64_t>> np;
    for (const auto& pr : H.near) {
        leaf_elements(H, pr.first, et);
        leaf_elements(H, pr.second, es);
        for (int64_t e1 : et)
            for (int64_t e2 : es) np.push_back({e1, e2});
    }
    std::vector<cplx> NB(np.size() * (size_t)nl * nl);
    const int64_t nnp = (int64_t)np.size();
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t k = 0; k < nnp; ++k) m_pair_block(S, np[k].first, np[k].second, qg, qs, part, &NB[k * nl * nl]);
    for (int64_t k = 0; k < nnp; ++k) glue_block(np[k].first, np[k].second, &NB[k * nl * nl]);
}

// Data fields (solutions of (MP) away from their source).  kind 0: the field of a point
// dipole of moment m at x0, E = curl curl (m G(x - x0)) = kappa^2 m G + grad (m . grad G);
// kind 1: a plane wave E = e exp(-i kappa d . x) (e perpendicular to d), the sign of the
// exponent matching the kernel's.
static void m_field(int kind, const double* prm, cplx kappa, const double x[3], cplx E[3]) {
    if (kind == 0) {
        const double R[3] = {x[0] - prm[0], x[1] - prm[1], x[2] - prm[2]};
        const double r = std::sqrt(R[0] * R[0] + R[1] * R[1] + R[2] * R[2]);
        const cplx ik = cplx(0.0, 1.0) * kappa, ex = std::exp(-ik * r) / (4.0 * PI);
        const cplx G = ex / r;
        const cplx G1 = -ex * (1.0 + ik * r) / (r * r);                          // G'(r)
        const cplx G2 = ex * (2.0 + 2.0 * ik * r + ik * ik * r * r) / (r * r * r);  // G''(r)
        const cplx g = G1 / r, gp = (G2 - G1 / r) / r;  // g(r) = G'/r and its derivative
        const double mR = prm[3] * R[0] + prm[4] * R[1] + prm[5] * R[2];
        for (int c = 0; c < 3; ++c) E[c] = kappa * kappa * prm[3 + c] * G + gp * mR * R[c] / r + g * prm[3 + c];
    } else {
        const cplx ph = std::exp(-cplx(0.0, 1.0) * kappa * (prm[0] * x[0] + prm[1] * x[1] + prm[2] * x[2]));
        for (int c = 0; c < 3; ++c) E[c] = prm[3 + c] * ph;
    }
}

// load vector b_g = int E . v_g d sigma, q x q Gauss points per element
static void m_rhs(const MSpace& S, int kind, const double* prm, int q, cplx* b) {
    const int nl = m_nl(S);
    std::fill(b, b + S.nglob, cplx(0.0));
    const Rule g = gauss01(q);
    std::vector<double> V(3 * nl), Dv(nl);
    std::vector<int64_t> lid(nl);
    for (int64_t e = 0; e < S.nelem; ++e) {
        const Elem E = elem_of(S.geo, e);
        for (int a1 = 0; a1 < q; ++a1)
            for (int a2 = 0; a2 < q; ++a2) {
                const double s = (E.i1 + g.x[a1]) * S.h, t = (E.i2 + g.x[a2]) * S.h;
                double x[3];
                m_elem_eval(S, E, s, t, x, V.data(), Dv.data(), lid.data());
                cplx F[3];
                m_field(kind, prm, S.kappa, x, F);
                const double w = g.w[a1] * g.w[a2] * S.h * S.h;
                for (int i = 0; i < nl; ++i) {
                    const int64_t G = S.glob[lid[i]];
                    if (G < 0) continue;
                    b[G] += (double)S.sgn[lid[i]] * w * (F[0] * V[3 * i] + F[1] * V[3 * i + 1] + F[2] * V[3 * i + 2]);
                }
            }
    }
}

// field (MS) of the density j (global coefficients) at points: int G j + kappa^-2 grad int G div j
static void m_potential(const MSpace& S, int q, const cplx* j, int64_t npts, const double* pts, cplx* out) {
    const int nl = m_nl(S);
    const Rule g = gauss01(q);
    const cplx ik = cplx(0.0, 1.0) * S.kappa, ik2 = 1.0 / (S.kappa * S.kappa);
    // the density and its divergence at every quadrature point
    const int64_t nq = S.nelem * q * q;
    std::vector<double> Y(3 * nq), W(nq);
    std::vector<cplx> J(3 * nq), Dj(nq);
    std::vector<double> V(3 * nl), Dv(nl);
    std::vector<int64_t> lid(nl);
    for (int64_t e = 0; e < S.nelem; ++e) {
        const Elem E = elem_of(S.geo, e);
        for (int a1 = 0; a1 < q; ++a1)
            for (int a2 = 0; a2 < q; ++a2) {
                const int64_t k = (e * q + a1) * q + a2;
                const double s = (E.i1 + g.x[a1]) * S.h, t = (E.i2 + g.x[a2]) * S.h;
                m_elem_eval(S, E, s, t, &Y[3 * k], V.data(), Dv.data(), lid.data());
                W[k] = g.w[a1] * g.w[a2] * S.h * S.h;
                cplx jj[3] = {0.0, 0.0, 0.0}, dd = 0.0;
                for (int i = 0; i < nl; ++i) {
                    const int64_t G = S.glob[lid[i]];
                    if (G < 0) continue;
                    const cplx c = (double)S.sgn[lid[i]] * j[G];
                    for (int d = 0; d < 3; ++d) jj[d] += c * V[3 * i + d];
                    dd += c * Dv[i];
                }
                for (int d = 0; d < 3; ++d) J[3 * k + d] = jj[d];
                Dj[k] = dd;
            }
    }
#pragma omp parallel for schedule(static)
    for (int64_t p = 0; p < npts; ++p) {
        const double* x = &pts[3 * p];
        cplx E[3] = {0.0, 0.0, 0.0};
        for (int64_t k = 0; k < nq; ++k) {
            const double R[3] = {x[0] - Y[3 * k], x[1] - Y[3 * k + 1], x[2] - Y[3 * k + 2]};
            const double r = std::sqrt(R[0] * R[0] + R[1] * R[1] + R[2] * R[2]);
            const cplx ex = std::exp(-ik * r) / (4.0 * PI);
            const cplx G = ex / r, G1 = -ex * (1.0 + ik * r) / (r * r);
            for (int d = 0; d < 3; ++d) E[d] += W[k] * (G * J[3 * k + d] + ik2 * G1 * (R[d] / r) * Dj[k]);
        }
        for (int d = 0; d < 3; ++d) out[3 * p + d] = E[d];
    }
}

}  // namespace orc

// =======================================================================================
// C interface used through ctypes.  Complex arrays are interleaved (re, im) doubles.
// All functions return 0 on success and -1 on error (message via orc_last_error).
// =======================================================================================
using namespace orc;

static thread_local std::string g_err;

struct OrcSpace {
    Space S;
};
struct OrcH2 {
    const OrcSpace* sp = nullptr;
    bool cplx_ = false;
    H2<double> hr;
    H2<cplx> hc;
};

#define ORC_TRY(...)                    \
    try {                               \
        __VA_ARGS__;                    \
        return 0;                       \
    } catch (const std::exception& e) { \
        g_err = e.what();               \
        return -1;                      \
    }

static bool is_cplx(const Space& S) { return S.pde == PDE_HELMHOLTZ; }

template <class T>
static void h2_info(const H2<T>& H, int64_t* info) {
    info[0] = (int64_t)H.cl.size();
    info[1] = (int64_t)H.far.size();
    info[2] = (int64_t)H.near.size();
    int64_t nnz = 0;
    for (const auto& r : H.near_rows) nnz += (int64_t)r.size();
    info[3] = nnz;
    info[4] = H.nloc;
    info[5] = H.qm;
}

// Potential accelerated by the cluster tree (Sec. 4 "Evaluation of the Solution" evaluated
// with the compression of Sec. 2 on the source side only): for each point x, the clusters of
// every patch are visited from the root; a cluster whose ball is admissible for the point
// (reading A10 with a target radius of 0: dist = |x - c| - r > 0 and 2 r <= eta dist, ties
// within 1e-12 dist inadmissible) contributes sum_a k(x, gamma(xi_a)) m_a, with the moments m
// of rho (forward + upward transform); an inadmissible leaf contributes the plain quadrature
// of its elements (q points per direction, as the dense potential); an inadmissible cluster
// above the leaves passes the point to its four children.
template <class T>
static void h2_potential(const H2<T>& H, const T* rho, int64_t npts, const double* pts, double eta, int qp, T* u) {
    const Space& S = *H.S;
    std::vector<T> mom(H.cl.size() * H.q * H.q, T(0));
    h2_forward(H, rho, mom);
    h2_upward(H, mom);
    const int q = H.q, q2 = q * q;
    const Rule g = gauss01(qp);
    const int nb = (S.K.d + 1) * (S.K.d + 1);
    std::vector<double> ph(nb);
    for (int64_t p = 0; p < npts; ++p) {
        const double* x = &pts[3 * p];
        T acc = T(0);
        std::vector<int64_t> todo;
        for (int f = S.G.npatch - 1; f >= 0; --f) todo.push_back(H.cluster_index(0, f, 0, 0));
        while (!todo.empty()) {
            const int64_t c = todo.back();
            todo.pop_back();
            const Cluster& C = H.cl[c];
            const double dist = dist3(x, C.c) - C.rad;
            const double lhs = 2.0 * C.rad, rhs = eta * dist;
            const bool adm = dist > 0.0 && !(std::fabs(lhs - rhs) <= 1e-12 * dist) && lhs <= rhs;
            if (adm) {
                for (int a = 0; a < q2; ++a) {
                    double y[3];
                    cluster_node(S.G, C, H.xi, a / q, a % q, y);
                    acc += kernel_r<T>(S.pde, S.kappa, dist3(x, y)) * mom[(size_t)c * q2 + a];
                }
            } else if (C.lev == H.leaf) {
                std::vector<int64_t> els;
                leaf_elements(H, c, els);
                for (int64_t e : els) {
                    const Elem E = elem_of(S, e);
                    for (int a1 = 0; a1 < qp; ++a1)
                        for (int a2 = 0; a2 < qp; ++a2) {
                            double s, t, y[3];
                            elem_param(S, E, 0, g.x[a1], g.x[a2], s, t);
                            gamma(S.G, E.f, s, t, y);
                            elem_basis(S, E, s, t, ph.data());
                            T rv = T(0);
                            for (int l = 0; l < nb; ++l) rv += rho[local_dof(S, E, l)] * ph[l];
                            if (S.form == 0) rv *= surf_elem(S.G, E.f, s, t);
                            acc += kernel_r<T>(S.pde, S.kappa, dist3(x, y)) * rv * (g.w[a1] * g.w[a2] * S.h * S.h);
                        }
                }
            } else {
                for (int k = 3; k >= 0; --k)
                    todo.push_back(H.cluster_index(C.lev + 1, C.f, 2 * C.i + (k >> 1), 2 * C.j + (k & 1)));
            }
        }
        u[p] = acc;
    }
}

extern "C" {

const char* orc_last_error() { return g_err.c_str(); }

// Timing mode (C-ALG step 13): threads of the parallel loops over independent items (rows,
// clusters, target runs); 1 = serial.  Results do not depend on it.  Returns the count set.
int orc_set_threads(int n) {
#ifdef _OPENMP
    omp_set_num_threads(n < 1 ? 1 : n);
    return omp_get_max_threads();
#else
    (void)n;
    return 1;
#endif
}

int orc_gauss01(int n, double* x, double* w) {
    ORC_TRY({
        Rule r = gauss01(n);
        for (int i = 0; i < n; ++i) {
            x[i] = r.x[i];
            w[i] = r.w[i];
        }
    })
}

// B-spline j of degree d (knot repetition r, 2^L elements) at points x
int orc_bspline(int d, int r, int L, int j, int64_t n, const double* x, double* out) {
    ORC_TRY({
        Knots K = make_knots(d, r, L);
        if (j < 0 || j >= K.nb) throw std::runtime_error("basis index out of range");
        for (int64_t i = 0; i < n; ++i) out[i] = bspline(K, j, d, x[i], find_span(K, x[i]));
    })
}

int orc_bspline_count(int d, int r, int L) { return make_knots(d, r, L).nb; }

int orc_space_new(int gkind, const double* gparams, int nparams, int pde, double kre, double kim,
                  int degree, int knot_rep, int level, void** out) {
    ORC_TRY({
        OrcSpace* s = new OrcSpace;
        try {
            s->S = make_space(make_geom(gkind, gparams, nparams), pde, cplx(kre, kim), degree,
                              knot_rep, level);
        } catch (...) {
            delete s;
            throw;
        }
        *out = s;
    })
}

// space on NURBS patches: meta = (p1, p2, k1, k2) per patch, knots = Xi_1 then Xi_2 of each
// patch in turn, cw = (x, y, z, w) per control point of each patch in turn (j1 outer)
int orc_space_new_nurbs(int npatch, const int* meta, const double* knots, const double* cw, int pde, double kre,
                        double kim, int degree, int knot_rep, int level, void** out) {
    ORC_TRY({
        OrcSpace* s = new OrcSpace;
        try {
            s->S = make_space(make_nurbs_geom(npatch, meta, knots, cw), pde, cplx(kre, kim), degree, knot_rep,
                              level);
        } catch (...) {
            delete s;
            throw;
        }
        *out = s;
    })
}

// lifting of the space: 2 (S^2, default) or 0 (S^0: surface integrals carry kappa); set
// before any operator is built on the space
int orc_space_set_form(void* sp, int form) {
    ORC_TRY({
        if (form != 0 && form != 2) throw std::runtime_error("form must be 0 or 2");
        ((OrcSpace*)sp)->S.form = form;
    })
}

// S^0 gluing: local -> global index of every local B-spline (map, ndof entries) and the
// number of global functions
int orc_space_glue(void* sp, int64_t* map, int64_t* nglob) {
    ORC_TRY({
        const std::vector<int64_t> m = glue_map(((OrcSpace*)sp)->S, nglob);
        std::copy(m.begin(), m.end(), map);
    })
}

void orc_space_free(void* s) { delete (OrcSpace*)s; }

int64_t orc_space_ndof(void* s) { return ((OrcSpace*)s)->S.ndof; }
int64_t orc_space_nelem(void* s) { return ((OrcSpace*)s)->S.nelem; }

// gamma and the surface element at n parameter points (s,t) of one patch
int orc_gamma(void* sp, int patch, int64_t n, const double* st, double* xyz, double* kappa,
              double* normal) {
    ORC_TRY({
        const Space& S = ((OrcSpace*)sp)->S;
        if (patch < 0 || patch >= S.G.npatch) throw std::runtime_error("bad patch");
        for (int64_t i = 0; i < n; ++i) {
            gamma(S.G, patch, st[2 * i], st[2 * i + 1], &xyz[3 * i]);
            double nr[3];
            double k = surf_elem(S.G, patch, st[2 * i], st[2 * i + 1], nr);
            if (kappa) kappa[i] = k;
            if (normal)
                for (int c = 0; c < 3; ++c) normal[3 * i + c] = nr[c];
        }
    })
}

// surface area sum_f int kappa_f by Gauss with q points per direction per element
int orc_area(void* sp, int q, double* area) {
    ORC_TRY({
        const Space& S = ((OrcSpace*)sp)->S;
        const Rule g = gauss01(q);
        double a = 0.0;
        for (int64_t e = 0; e < S.nelem; ++e) {
            const Elem E = elem_of(S, e);
            for (int a1 = 0; a1 < q; ++a1)
                for (int a2 = 0; a2 < q; ++a2) {
                    double s, t;
                    elem_param(S, E, 0, g.x[a1], g.x[a2], s, t);
                    a += g.w[a1] * g.w[a2] * S.h * S.h * surf_elem(S.G, E.f, s, t);
                }
        }
        *area = a;
    })
}

// classification of an element pair: type (0 regular, 1 vertex, 2 edge, 3 identical), k1, k2
int orc_classify(void* sp, int64_t e1, int64_t e2, int* out3) {
    ORC_TRY({
        const Space& S = ((OrcSpace*)sp)->S;
        PairInfo P = classify_pair(S, e1, e2);
        out3[0] = P.type;
        out3[1] = P.k1;
        out3[2] = P.k2;
    })
}

// one element-pair block ((d+1)^2 x (d+1)^2, row-major)
int orc_pair_block(void* sp, int64_t e1, int64_t e2, int qg, int qs, double* B) {
    ORC_TRY({
        const Space& S = ((OrcSpace*)sp)->S;
        SideFn F;
        if (is_cplx(S))
            pair_block<cplx>(S, F, F, e1, e2, qg, qs, (cplx*)B);
        else
            pair_block<double>(S, F, F, e1, e2, qg, qs, B);
    })
}

// dense Galerkin matrix, N x N row-major
int orc_dense(void* sp, int qg, int qs, double* A) {
    ORC_TRY({
        const Space& S = ((OrcSpace*)sp)->S;
        if (is_cplx(S))
            dense_matrix<cplx>(S, qg, qs, (cplx*)A);
        else
            dense_matrix<double>(S, qg, qs, A);
    })
}

// <S f, g> for the fixed surface functions of density mode (result complex: out[0], out[1])
int orc_density_pairing(void* sp, int fid, int gid, int qg, int qs, double* out) {
    ORC_TRY({
        const Space& S = ((OrcSpace*)sp)->S;
        cplx v = density_pairing<cplx>(S, fid, gid, qg, qs);
        out[0] = v.real();
        out[1] = v.imag();
    })
}

// load vectors for nrhs data sets (params: 3 doubles each), column-major N x nrhs
int orc_rhs(void* sp, int kind, const double* params, int nrhs, int q, double* b) {
    ORC_TRY({
        const Space& S = ((OrcSpace*)sp)->S;
        for (int r = 0; r < nrhs; ++r) {
            if (is_cplx(S))
                load_vector<cplx>(S, kind, params + 3 * r, q, (cplx*)b + r * S.ndof);
            else {
                if (kind != DATA_POINT_SOURCE) throw std::runtime_error("plane waves need Helmholtz");
                load_vector<double>(S, kind, params + 3 * r, q, b + r * S.ndof);
            }
        }
    })
}

int orc_potential(void* sp, int q, const double* rho, int64_t npts, const double* pts, double* u) {
    ORC_TRY({
        const Space& S = ((OrcSpace*)sp)->S;
        if (is_cplx(S))
            potential<cplx>(S, q, (const cplx*)rho, npts, pts, (cplx*)u);
        else
            potential<double>(S, q, rho, npts, pts, u);
    })
}

int orc_h2_new(void* sp, int q, double eta, int leaf, int qg, int qs, int assemble_near, double kadm, void** out) {
    ORC_TRY({
        OrcH2* h = new OrcH2;
        h->sp = (OrcSpace*)sp;
        const Space& S = h->sp->S;
        h->cplx_ = is_cplx(S);
        try {
            if (h->cplx_)
                h2_build(h->hc, S, q, eta, leaf, qg, qs, assemble_near != 0, kadm);
            else
                h2_build(h->hr, S, q, eta, leaf, qg, qs, assemble_near != 0, kadm);
        } catch (...) {
            delete h;
            throw;
        }
        *out = h;
    })
}

void orc_h2_free(void* h) { delete (OrcH2*)h; }


// info: [nclusters, nfar, nnear_leaf_pairs, near_nnz, nloc, qm]
int orc_h2_info(void* hp, int64_t* info) {
    ORC_TRY({
        OrcH2* h = (OrcH2*)hp;
        if (h->cplx_)
            h2_info(h->hc, info);
        else
            h2_info(h->hr, info);
    })
}

// far list (target, source) and near leaf-pair list, cluster indices
int orc_h2_lists(void* hp, int64_t* far2, int64_t* near2) {
    ORC_TRY({
        OrcH2* h = (OrcH2*)hp;
        const auto& F = h->cplx_ ? h->hc.far : h->hr.far;
        const auto& Nn = h->cplx_ ? h->hc.near : h->hr.near;
        if (far2)
            for (size_t i = 0; i < F.size(); ++i) {
                far2[2 * i] = F[i].first;
                far2[2 * i + 1] = F[i].second;
            }
        if (near2)
            for (size_t i = 0; i < Nn.size(); ++i) {
                near2[2 * i] = Nn[i].first;
                near2[2 * i + 1] = Nn[i].second;
            }
    })
}

// clusters: per cluster (lev, f, i, j) and (cx, cy, cz, rad)
int orc_h2_clusters(void* hp, int32_t* ids, double* balls) {
    ORC_TRY({
        OrcH2* h = (OrcH2*)hp;
        const auto& C = h->cplx_ ? h->hc.cl : h->hr.cl;
        for (size_t i = 0; i < C.size(); ++i) {
            ids[4 * i] = C[i].lev;
            ids[4 * i + 1] = C[i].f;
            ids[4 * i + 2] = C[i].i;
            ids[4 * i + 3] = C[i].j;
            balls[4 * i] = C[i].c[0];
            balls[4 * i + 1] = C[i].c[1];
            balls[4 * i + 2] = C[i].c[2];
            balls[4 * i + 3] = C[i].rad;
        }
    })
}

// coupling blocks (q^2 x q^2 each, far-list order), transfer matrices, 1-D leaf moments
int orc_h2_tables(void* hp, double* K, double* E0, double* E1, double* V1) {
    ORC_TRY({
        OrcH2* h = (OrcH2*)hp;
        auto copy = [&](auto& H) {
            if (K) std::memcpy(K, H.K.data(), H.K.size() * sizeof(H.K[0]));
            if (E0) std::memcpy(E0, H.E[0].data(), H.E[0].size() * sizeof(double));
            if (E1) std::memcpy(E1, H.E[1].data(), H.E[1].size() * sizeof(double));
            if (V1)
                for (size_t i = 0; i < H.V1.size(); ++i)
                    std::memcpy(V1 + i * H.V1[i].size(), H.V1[i].data(), H.V1[i].size() * sizeof(double));
        };
        if (h->cplx_)
            copy(h->hc);
        else
            copy(h->hr);
    })
}

// near field as CSR (rowptr N+1, col nnz, val nnz)
int orc_h2_near_csr(void* hp, int64_t* rowptr, int64_t* col, double* val) {
    ORC_TRY({
        OrcH2* h = (OrcH2*)hp;
        auto dump = [&](auto& H, auto* v) {
            if (!H.have_near) throw std::runtime_error("near field not assembled");
            int64_t k = 0;
            rowptr[0] = 0;
            for (size_t r = 0; r < H.near_rows.size(); ++r) {
                for (const auto& kv : H.near_rows[r]) {
                    col[k] = kv.first;
                    v[k] = kv.second;
                    ++k;
                }
                rowptr[r + 1] = k;
            }
        };
        if (h->cplx_)
            dump(h->hc, (cplx*)val);
        else
            dump(h->hr, val);
    })
}

// moments of all clusters, by forward + upward transfer (direct = 0) or by direct
// integration over each cluster (direct = 1)
int orc_h2_moments(void* hp, const double* x, int direct, double* mom) {
    ORC_TRY({
        OrcH2* h = (OrcH2*)hp;
        auto run = [&](auto& H, auto* xx, auto* mm) {
            using T = std::remove_reference_t<decltype(*mm)>;
            const int q2 = H.q * H.q;
            std::vector<T> m(H.cl.size() * q2, T(0));
            if (direct)
                h2_direct_moments(H, xx, m);
            else {
                h2_forward(H, xx, m);
                h2_upward(H, m);
            }
            std::copy(m.begin(), m.end(), mm);
        };
        if (h->cplx_)
            run(h->hc, (const cplx*)x, (cplx*)mom);
        else
            run(h->hr, x, mom);
    })
}

// y = A x for nrhs columns (column-major, leading dimension N)
int orc_h2_potential(void* hp, const double* rho, int64_t npts, const double* pts, double eta, double* u) {
    ORC_TRY({
        OrcH2* h = (OrcH2*)hp;
        if (h->cplx_)
            h2_potential(h->hc, (const cplx*)rho, npts, pts, eta, 8, (cplx*)u);
        else
            h2_potential(h->hr, rho, npts, pts, eta, 8, u);
    })
}

int orc_h2_apply(void* hp, const double* x, double* y, int nrhs) {
    ORC_TRY({
        OrcH2* h = (OrcH2*)hp;
        const int64_t N = h->sp->S.ndof;
        for (int r = 0; r < nrhs; ++r) {
            if (h->cplx_)
                h2_apply(h->hc, (const cplx*)x + r * N, (cplx*)y + r * N);
            else
                h2_apply(h->hr, x + r * N, y + r * N);
        }
    })
}

// (A x) at selected rows, near rows integrated on the fly; parts: bit 0 far, bit 1 near
int orc_h2_apply_rows(void* hp, const double* x, const int64_t* rows, int64_t nrows, int parts,
                      double* y) {
    ORC_TRY({
        OrcH2* h = (OrcH2*)hp;
        if (h->cplx_)
            h2_apply_rows(h->hc, (const cplx*)x, rows, nrows, (cplx*)y, parts & 1, parts & 2);
        else
            h2_apply_rows(h->hr, x, rows, nrows, y, parts & 1, parts & 2);
    })
}

// assemble (and keep) the near-field rows of a subset of DOFs; apply_rows then uses them
int orc_h2_near_rows(void* hp, const int64_t* rows, int64_t nrows) {
    ORC_TRY({
        OrcH2* h = (OrcH2*)hp;
        if (h->cplx_)
            h2_near_rows_subset(h->hc, rows, nrows);
        else
            h2_near_rows_subset(h->hr, rows, nrows);
    })
}

// GMRES on the H^2 operator; stats: [iterations, relres, converged]
int orc_h2_gmres(void* hp, const double* b, double* x, double tol, int restart, int maxit,
                 double* stats) {
    ORC_TRY({
        OrcH2* h = (OrcH2*)hp;
        const int64_t N = h->sp->S.ndof;
        int it = 0;
        double rr = 0.0;
        int rc;
        if (h->cplx_) {
            auto mv = [&](const cplx* a, cplx* o) { h2_apply(h->hc, a, o); };
            rc = gmres<cplx>(N, mv, (const cplx*)b, (cplx*)x, tol, restart, maxit, &it, &rr);
        } else {
            auto mv = [&](const double* a, double* o) { h2_apply(h->hr, a, o); };
            rc = gmres<double>(N, mv, b, x, tol, restart, maxit, &it, &rr);
        }
        stats[0] = it;
        stats[1] = rr;
        stats[2] = rc == 0 ? 1.0 : 0.0;
    })
}

// GMRES on a dense row-major matrix given by the caller
int orc_dense_gmres(int64_t n, int is_complex, const double* A, const double* b, double* x, double tol,
                    int restart, int maxit, double* stats) {
    ORC_TRY({
        int it = 0;
        double rr = 0.0;
        int rc;
        if (is_complex) {
            const cplx* Ac = (const cplx*)A;
            auto mv = [&](const cplx* a, cplx* o) {
                for (int64_t i = 0; i < n; ++i) {
                    cplx s = 0.0;
                    for (int64_t j = 0; j < n; ++j) s += Ac[i * n + j] * a[j];
                    o[i] = s;
                }
            };
            rc = gmres<cplx>(n, mv, (const cplx*)b, (cplx*)x, tol, restart, maxit, &it, &rr);
        } else {
            auto mv = [&](const double* a, double* o) {
                for (int64_t i = 0; i < n; ++i) {
                    double s = 0.0;
                    for (int64_t j = 0; j < n; ++j) s += A[i * n + j] * a[j];
                    o[i] = s;
                }
            };
            rc = gmres<double>(n, mv, b, x, tol, restart, maxit, &it, &rr);
        }
        stats[0] = it;
        stats[1] = rr;
        stats[2] = rc == 0 ? 1.0 : 0.0;
    })
}

// ---- block-Jacobi
struct OrcBJ {
    const OrcH2* h = nullptr;
    BJ<double> br;
    BJ<cplx> bc;
};

int orc_bj_new(void* hp, int tile, void** out) {
    ORC_TRY({
        OrcH2* h = (OrcH2*)hp;
        OrcBJ* b = new OrcBJ;
        b->h = h;
        try {
            if (h->cplx_)
                bj_build(h->hc, tile, b->bc);
            else
                bj_build(h->hr, tile, b->br);
        } catch (...) {
            delete b;
            throw;
        }
        *out = b;
    })
}
void orc_bj_free(void* b) { delete (OrcBJ*)b; }
int64_t orc_bj_ntiles(void* bp) {
    OrcBJ* b = (OrcBJ*)bp;
    return b->h->cplx_ ? (int64_t)b->bc.tiles.size() : (int64_t)b->br.tiles.size();
}
// tile k: (patch, j1a, j1b, j2a, j2b) and its DOFs (j1 outer, j2 inner)
int orc_bj_tile(void* bp, int64_t k, int32_t* t5, int64_t* dofs) {
    ORC_TRY({
        OrcBJ* b = (OrcBJ*)bp;
        const Tile& t = b->h->cplx_ ? b->bc.tiles.at(k) : b->br.tiles.at(k);
        t5[0] = t.f; t5[1] = t.j1a; t5[2] = t.j1b; t5[3] = t.j2a; t5[4] = t.j2b;
        const auto& g = b->h->cplx_ ? b->bc.dofs.at(k) : b->br.dofs.at(k);
        if (dofs) std::copy(g.begin(), g.end(), dofs);
    })
}
// the (unfactored) block D_b of tile k, n x n row-major
int orc_bj_block(void* bp, int64_t k, double* D) {
    ORC_TRY({
        OrcBJ* b = (OrcBJ*)bp;
        if (b->h->cplx_) {
            const auto& g = b->bc.dofs.at(k);
            auto v = near_block(b->h->hc, g, g);
            std::copy(v.begin(), v.end(), (cplx*)D);
        } else {
            const auto& g = b->br.dofs.at(k);
            auto v = near_block(b->h->hr, g, g);
            std::copy(v.begin(), v.end(), D);
        }
    })
}
int orc_bj_apply(void* bp, const double* r, double* z) {
    ORC_TRY({
        OrcBJ* b = (OrcBJ*)bp;
        if (b->h->cplx_)
            bj_apply(b->bc, (const cplx*)r, (cplx*)z);
        else
            bj_apply(b->br, r, z);
    })
}
// learned-correction target X_b of tile k with the given ring (n_b x n_b row-major)
int orc_bj_target(void* bp, int64_t k, int ring, double* C) {
    ORC_TRY({
        OrcBJ* b = (OrcBJ*)bp;
        if (b->h->cplx_) {
            auto v = bj_target(b->h->hc, b->bc.tiles.at(k), ring);
            std::copy(v.begin(), v.end(), (cplx*)C);
        } else {
            auto v = bj_target(b->h->hr, b->br.tiles.at(k), ring);
            std::copy(v.begin(), v.end(), C);
        }
    })
}
// features of every tile of T x T B-spline indices (ntiles x 99)
int orc_tile_features(void* sp, int T, double* feats) {
    ORC_TRY({
        const Space& S = ((OrcSpace*)sp)->S;
        const auto tiles = make_tiles(S, T);
        for (size_t k = 0; k < tiles.size(); ++k) tile_features(S, tiles[k], feats + k * 99);
    })
}

// right-preconditioned GMRES on the H^2 operator: GMRES on A M^{-1}, then x = M^{-1} u
int orc_h2_gmres_bj(void* hp, void* bp, const double* b, double* x, double tol, int restart, int maxit,
                    double* stats) {
    ORC_TRY({
        OrcH2* h = (OrcH2*)hp;
        OrcBJ* bj = (OrcBJ*)bp;
        const int64_t N = h->sp->S.ndof;
        int it = 0;
        double rr = 0.0;
        int rc;
        if (h->cplx_) {
            std::vector<cplx> z(N), u(N);
            auto mv = [&](const cplx* a, cplx* o) {
                bj_apply(bj->bc, a, z.data());
                h2_apply(h->hc, z.data(), o);
            };
            rc = gmres<cplx>(N, mv, (const cplx*)b, u.data(), tol, restart, maxit, &it, &rr);
            bj_apply(bj->bc, u.data(), (cplx*)x);
        } else {
            std::vector<double> z(N), u(N);
            auto mv = [&](const double* a, double* o) {
                bj_apply(bj->br, a, z.data());
                h2_apply(h->hr, z.data(), o);
            };
            rc = gmres<double>(N, mv, b, u.data(), tol, restart, maxit, &it, &rr);
            bj_apply(bj->br, u.data(), x);
        }
        stats[0] = it;
        stats[1] = rr;
        stats[2] = rc == 0 ? 1.0 : 0.0;
    })
}

// ---- Maxwell single layer on S^1 (App. A (MP), App. B (MS), App. E)
struct OrcMSpace {
    MSpace S;
};

int orc_mspace_new(int gkind, const double* gparams, int nparams, double kre, double kim, int p, int level,
                   void** out) {
    ORC_TRY({
        OrcMSpace* s = new OrcMSpace;
        try {
            s->S = make_mspace(make_geom(gkind, gparams, nparams), cplx(kre, kim), p, level);
        } catch (...) {
            delete s;
            throw;
        }
        *out = s;
    })
}

int orc_mspace_new_nurbs(int npatch, const int* meta, const double* knots, const double* cw, double kre, double kim,
                         int p, int level, void** out) {
    ORC_TRY({
        OrcMSpace* s = new OrcMSpace;
        try {
            s->S = make_mspace(make_nurbs_geom(npatch, meta, knots, cw), cplx(kre, kim), p, level);
        } catch (...) {
            delete s;
            throw;
        }
        *out = s;
    })
}

void orc_mspace_free(void* s) { delete (OrcMSpace*)s; }

// info: local functions, global functions, elements, functions per element
int orc_mspace_info(void* sp, int64_t* info) {
    ORC_TRY({
        const MSpace& S = ((OrcMSpace*)sp)->S;
        info[0] = S.nloc;
        info[1] = S.nglob;
        info[2] = S.nelem;
        info[3] = m_nl(S);
    })
}

int orc_mspace_glue(void* sp, int64_t* glob, int32_t* sgn) {
    ORC_TRY({
        const MSpace& S = ((OrcMSpace*)sp)->S;
        std::copy(S.glob.begin(), S.glob.end(), glob);
        std::copy(S.sgn.begin(), S.sgn.end(), sgn);
    })
}

// the local functions of element e at parameter (s, t): point, lifted fields, divergences
int orc_m_elem_eval(void* sp, int64_t e, double s, double t, double* x, double* V, double* Dv, int64_t* lid) {
    ORC_TRY({
        const MSpace& S = ((OrcMSpace*)sp)->S;
        if (e < 0 || e >= S.nelem) throw std::runtime_error("element out of range");
        m_elem_eval(S, elem_of(S.geo, e), s, t, x, V, Dv, lid);
    })
}

int orc_m_pair_block(void* sp, int64_t e1, int64_t e2, int qg, int qs, int part, double* B) {
    ORC_TRY({
        const MSpace& S = ((OrcMSpace*)sp)->S;
        m_pair_block(S, e1, e2, qg, qs, part, (cplx*)B);
    })
}

int orc_m_dense(void* sp, int qg, int qs, int part, double* M) {
    ORC_TRY({ m_dense(((OrcMSpace*)sp)->S, qg, qs, part, (cplx*)M); })
}

// Maxwell matrix with the far field compressed on the scalar H^2 partition (q, eta, leaf, kadm)
int orc_m_h2_dense(void* sp, int q, double eta, int leaf, int qg, int qs, double kadm, int part, double* M) {
    ORC_TRY({
        const MSpace& S = ((OrcMSpace*)sp)->S;
        if (leaf < 0 || leaf > S.L) throw std::runtime_error("leaf level must lie in [0, L]");
        m_h2_dense(S, q, eta, leaf, qg, qs, kadm, part, (cplx*)M);
    })
}

// nrhs load vectors, 6 parameters each (dipole: x0, moment; plane wave: direction, polarisation)
int orc_m_rhs(void* sp, int kind, const double* prm, int nrhs, int q, double* b) {
    ORC_TRY({
        const MSpace& S = ((OrcMSpace*)sp)->S;
        for (int r = 0; r < nrhs; ++r) m_rhs(S, kind, prm + 6 * r, q, (cplx*)b + (size_t)r * S.nglob);
    })
}

int orc_m_potential(void* sp, int q, const double* j, int64_t npts, const double* pts, double* E) {
    ORC_TRY({ m_potential(((OrcMSpace*)sp)->S, q, (const cplx*)j, npts, pts, (cplx*)E); })
}

int orc_m_field(int kind, const double* prm, double kre, double kim, int64_t npts, const double* pts, double* E) {
    ORC_TRY({
        for (int64_t p = 0; p < npts; ++p) m_field(kind, prm, cplx(kre, kim), &pts[3 * p], (cplx*)E + 3 * p);
    })
}

}  // extern "C"
