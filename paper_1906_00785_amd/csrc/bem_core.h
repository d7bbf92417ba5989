// Internal definitions shared by the host plan and the gfx950 kernels of libbem_hip.so:
// scalar types, the analytic patch maps, the single-layer kernels, and the plain-old-data
// descriptors that kernels receive by value.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace bem {

constexpr double kPi = 3.14159265358979323846264338327950288;
constexpr double kInv4Pi = 0.07957747154594766788444188168625718;  // 1/(4 pi)

// ------------------------------------------------------------------ complex scalar
struct cdbl {
    double re, im;
};
__host__ __device__ inline cdbl operator+(cdbl a, cdbl b) { return {a.re + b.re, a.im + b.im}; }
__host__ __device__ inline cdbl operator-(cdbl a, cdbl b) { return {a.re - b.re, a.im - b.im}; }
__host__ __device__ inline cdbl operator*(cdbl a, cdbl b) {
    return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
__host__ __device__ inline cdbl operator*(double s, cdbl a) { return {s * a.re, s * a.im}; }
__host__ __device__ inline cdbl operator*(cdbl a, double s) { return {s * a.re, s * a.im}; }
__host__ __device__ inline cdbl& operator+=(cdbl& a, cdbl b) {
    a.re += b.re;
    a.im += b.im;
    return a;
}
__host__ __device__ inline cdbl& operator-=(cdbl& a, cdbl b) {
    a.re -= b.re;
    a.im -= b.im;
    return a;
}

template <class T>
__host__ __device__ inline T zero();
template <>
__host__ __device__ inline double zero<double>() { return 0.0; }
template <>
__host__ __device__ inline cdbl zero<cdbl>() { return {0.0, 0.0}; }

__host__ __device__ inline double conj_(double a) { return a; }
__host__ __device__ inline cdbl conj_(cdbl a) { return {a.re, -a.im}; }
__host__ __device__ inline double abs2(double a) { return a * a; }
__host__ __device__ inline double abs2(cdbl a) { return a.re * a.re + a.im * a.im; }

// ------------------------------------------------------------------ geometry
enum GeomKind : int { GEOM_SPHERE6 = 0, GEOM_ELLIPSOID6 = 1, GEOM_TORUS16 = 2, GEOM_FLAT1 = 3, GEOM_NURBS = 4 };

// Patches given by NURBS maps (App. C) live in one table of doubles, a copy in host memory
// for the planner and one in device memory for the kernels:
//   [1 + 6 f .. 1 + 6 f + 5]  patch f: p1, p2, k1, k2 (degrees, basis counts), offset of its
//                             knots (Xi_1 then Xi_2, clamped), offset of its control points
//                             (x, y, z, w per point, j1 outer, k1 x k2 points)
constexpr int kNurbsMaxDeg = 8;

struct GeomDesc {
    int kind;
    int npatch;
    double a, b, c;  // ellipsoid semi-axes; torus R = a, r = b; flat side a
    const double* tab_host;  // NURBS table (GEOM_NURBS only)
    const double* tab_dev;
};

// Knot span of x in a clamped knot vector xi with k basis functions of degree p: the
// largest mu in [p, k-1] with xi[mu] <= x (x = 1 falls in the last span).
__host__ __device__ inline int nurbs_span(const double* xi, int p, int k, double x) {
    if (x >= xi[k]) return k - 1;
    int lo = p, hi = k;  // xi[lo] <= x < xi[hi]
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (x < xi[mid])
            hi = mid;
        else
            lo = mid;
    }
    return lo;
}

// The p + 1 B-splines of degree p that do not vanish in span mu, N[r] = b_{mu-p+r}(x),
// by the triangular scheme (each degree from the previous one over the span's knot
// differences; no division by a zero-length interval occurs inside a non-empty span).
__host__ __device__ inline void nurbs_funs(const double* xi, int p, int mu, double x, double* N) {
    double left[kNurbsMaxDeg + 1], right[kNurbsMaxDeg + 1];
    N[0] = 1.0;
    for (int j = 1; j <= p; ++j) {
        left[j] = x - xi[mu + 1 - j];
        right[j] = xi[mu + j] - x;
        double saved = 0.0;
        for (int r = 0; r < j; ++r) {
            const double tmp = N[r] / (right[r + 1] + left[j - r]);
            N[r] = saved + right[r + 1] * tmp;
            saved = left[j - r] * tmp;
        }
        N[j] = saved;
    }
}

// gamma_f(s, t) of a NURBS patch: the rational combination of the (p1+1)(p2+1) control
// points whose basis functions do not vanish at (s, t).  Kept out of line so that the
// analytic maps' callers do not carry its registers.
__host__ __device__ __attribute__((noinline)) inline void nurbs_point(const double* tab, int f, double s, double t,
                                                                     double* x) {
    const double* h = tab + 1 + 6 * f;
    const int p1 = (int)h[0], p2 = (int)h[1], k1 = (int)h[2], k2 = (int)h[3];
    const double* xi1 = tab + (int64_t)h[4];
    const double* xi2 = xi1 + k1 + p1 + 1;
    const double* cw = tab + (int64_t)h[5];
    const int m1 = nurbs_span(xi1, p1, k1, s), m2 = nurbs_span(xi2, p2, k2, t);
    double N1[kNurbsMaxDeg + 1], N2[kNurbsMaxDeg + 1];
    nurbs_funs(xi1, p1, m1, s, N1);
    nurbs_funs(xi2, p2, m2, t, N2);
    double a0 = 0.0, a1 = 0.0, a2 = 0.0, aw = 0.0;
    for (int i = 0; i <= p1; ++i) {
        const double* row = cw + 4 * ((int64_t)(m1 - p1 + i) * k2 + (m2 - p2));
        double b0 = 0.0, b1 = 0.0, b2 = 0.0, bw = 0.0;
        for (int j = 0; j <= p2; ++j) {
            const double* c = row + 4 * j;
            const double v = N2[j] * c[3];
            b0 += v * c[0];
            b1 += v * c[1];
            b2 += v * c[2];
            bw += v;
        }
        a0 += N1[i] * b0;
        a1 += N1[i] * b1;
        a2 += N1[i] * b2;
        aw += N1[i] * bw;
    }
    const double inv = 1.0 / aw;
    x[0] = a0 * inv;
    x[1] = a1 * inv;
    x[2] = a2 * inv;
}

// Cube face f of the cube-sphere: which coordinate receives u = 2s-1, which receives
// v = 2t-1, which is the constant +-1.  Faces: +z, -z, +x, -x, +y, -y, each with the
// orientation that makes d_s x d_t point outward.
__host__ __device__ inline void cube_face_layout(int f, int& iu, int& iv, int& ic, double& cval) {
    switch (f) {
        case 0: iu = 0; iv = 1; ic = 2; cval = 1.0; break;
        case 1: iu = 1; iv = 0; ic = 2; cval = -1.0; break;
        case 2: iu = 1; iv = 2; ic = 0; cval = 1.0; break;
        case 3: iu = 2; iv = 1; ic = 0; cval = -1.0; break;
        case 4: iu = 2; iv = 0; ic = 1; cval = 1.0; break;
        default: iu = 0; iv = 2; ic = 1; cval = -1.0; break;
    }
}

// Point gamma_f(s, t) of the analytic multi-patch surface.
__host__ __device__ inline void patch_point(const GeomDesc& g, int f, double s, double t, double* x) {
    if (g.kind == GEOM_SPHERE6 || g.kind == GEOM_ELLIPSOID6) {
        int iu, iv, ic;
        double cv;
        cube_face_layout(f, iu, iv, ic, cv);
        double c[3];
        c[iu] = 2.0 * s - 1.0;
        c[iv] = 2.0 * t - 1.0;
        c[ic] = cv;
        const double inv = 1.0 / sqrt(c[0] * c[0] + c[1] * c[1] + c[2] * c[2]);
        if (g.kind == GEOM_SPHERE6) {
            x[0] = c[0] * inv;
            x[1] = c[1] * inv;
            x[2] = c[2] * inv;
        } else {
            x[0] = g.a * (c[0] * inv);
            x[1] = g.b * (c[1] * inv);
            x[2] = g.c * (c[2] * inv);
        }
    } else if (g.kind == GEOM_TORUS16) {
        const double u = 0.5 * kPi * ((f >> 2) + s);
        const double v = 0.5 * kPi * ((f & 3) + t);
        double su, cu, sv, cvv;
        sincos(u, &su, &cu);
        sincos(v, &sv, &cvv);
        const double rr = g.a + g.b * cvv;
        x[0] = rr * cu;
        x[1] = rr * su;
        x[2] = g.b * sv;
    } else if (g.kind == GEOM_NURBS) {
        double px[3];  // own array for the out-of-line evaluation (see patch_jac)
#if defined(__HIP_DEVICE_COMPILE__)
        nurbs_point(g.tab_dev, f, s, t, px);
#else
        nurbs_point(g.tab_host, f, s, t, px);
#endif
        x[0] = px[0];
        x[1] = px[1];
        x[2] = px[2];
    } else {
        x[0] = g.a * s;
        x[1] = g.a * t;
        x[2] = 0.0;
    }
}

// Surface element |d_s gamma x d_t gamma| of a NURBS patch at (s, t): the derivatives of
// the p + 1 basis functions of a span follow from the p functions of degree p - 1,
// d/dx b_j^p = p (b_j^{p-1} / (xi_{j+p} - xi_j) - b_{j+1}^{p-1} / (xi_{j+p+1} - xi_{j+1})),
// and the map's derivatives from the quotient rule.
__host__ __device__ inline void nurbs_dfuns(const double* xi, int p, int mu, double x, double* N, double* dN) {
    nurbs_funs(xi, p, mu, x, N);
    if (p == 0) {
        dN[0] = 0.0;
        return;
    }
    double Nm[kNurbsMaxDeg + 1];
    nurbs_funs(xi, p - 1, mu, x, Nm);  // Nm[k] = b_{mu-p+1+k}^{p-1}
    for (int r = 0; r <= p; ++r) {
        double v = 0.0;
        if (r >= 1) v += Nm[r - 1] / (xi[mu + r] - xi[mu - p + r]);
        if (r <= p - 1) v -= Nm[r] / (xi[mu + r + 1] - xi[mu - p + r + 1]);
        dN[r] = p * v;
    }
}

// Point and first derivatives d_s gamma, d_t gamma of a NURBS patch at (s, t) (quotient rule
// on the rational map, basis derivatives from nurbs_dfuns).
__host__ __device__ __attribute__((noinline)) inline void nurbs_jac(const double* tab, int f, double s, double t,
                                                                    double* x, double* xs, double* xt) {
    const double* h = tab + 1 + 6 * f;
    const int p1 = (int)h[0], p2 = (int)h[1], k1 = (int)h[2], k2 = (int)h[3];
    const double* xi1 = tab + (int64_t)h[4];
    const double* xi2 = xi1 + k1 + p1 + 1;
    const double* cw = tab + (int64_t)h[5];
    const int m1 = nurbs_span(xi1, p1, k1, s), m2 = nurbs_span(xi2, p2, k2, t);
    double N1[kNurbsMaxDeg + 1], N2[kNurbsMaxDeg + 1], D1[kNurbsMaxDeg + 1], D2[kNurbsMaxDeg + 1];
    nurbs_dfuns(xi1, p1, m1, s, N1, D1);
    nurbs_dfuns(xi2, p2, m2, t, N2, D2);
    double A[3] = {0, 0, 0}, As[3] = {0, 0, 0}, At[3] = {0, 0, 0}, W = 0.0, Ws = 0.0, Wt = 0.0;
    for (int i = 0; i <= p1; ++i)
        for (int j = 0; j <= p2; ++j) {
            const double* c = cw + 4 * ((int64_t)(m1 - p1 + i) * k2 + (m2 - p2 + j));
            const double v = N1[i] * N2[j] * c[3], vs = D1[i] * N2[j] * c[3], vt = N1[i] * D2[j] * c[3];
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
        xs[d] = (As[d] - x[d] * Ws) / W;
        xt[d] = (At[d] - x[d] * Wt) / W;
    }
}

__host__ __device__ inline double nurbs_kappa(const double* tab, int f, double s, double t) {
    double x[3], xs[3], xt[3];
    nurbs_jac(tab, f, s, t, x, xs, xt);
    const double n0 = xs[1] * xt[2] - xs[2] * xt[1], n1 = xs[2] * xt[0] - xs[0] * xt[2], n2 = xs[0] * xt[1] - xs[1] * xt[0];
    return sqrt(n0 * n0 + n1 * n1 + n2 * n2);
}

// Surface element kappa_f(s, t) = |d_s gamma_f x d_t gamma_f| of every patch kind, from the
// maps' derivatives (the 0-form lifting multiplies every surface integral by it).
__host__ __device__ inline double patch_kappa(const GeomDesc& g, int f, double s, double t) {
    if (g.kind == GEOM_SPHERE6 || g.kind == GEOM_ELLIPSOID6) {
        int iu, iv, ic;
        double cv;
        cube_face_layout(f, iu, iv, ic, cv);
        double c[3];
        c[iu] = 2.0 * s - 1.0;
        c[iv] = 2.0 * t - 1.0;
        c[ic] = cv;
        const double rr = sqrt(c[0] * c[0] + c[1] * c[1] + c[2] * c[2]);
        const double n[3] = {c[0] / rr, c[1] / rr, c[2] / rr};
        // d(c/|c|)/ds = (dc/ds - n (n . dc/ds)) / |c| with dc/ds = 2 e_iu (and e_iv for t)
        double xs[3], xt[3];
        const double sc[3] = {g.kind == GEOM_SPHERE6 ? 1.0 : g.a, g.kind == GEOM_SPHERE6 ? 1.0 : g.b,
                              g.kind == GEOM_SPHERE6 ? 1.0 : g.c};
        for (int d = 0; d < 3; ++d) {
            xs[d] = sc[d] * 2.0 * ((d == iu ? 1.0 : 0.0) - n[d] * n[iu]) / rr;
            xt[d] = sc[d] * 2.0 * ((d == iv ? 1.0 : 0.0) - n[d] * n[iv]) / rr;
        }
        const double n0 = xs[1] * xt[2] - xs[2] * xt[1], n1 = xs[2] * xt[0] - xs[0] * xt[2],
                     n2 = xs[0] * xt[1] - xs[1] * xt[0];
        return sqrt(n0 * n0 + n1 * n1 + n2 * n2);
    } else if (g.kind == GEOM_TORUS16) {
        // d_s gamma and d_t gamma are orthogonal, of lengths pi/2 (R + r cos v) and pi/2 r
        const double v = 0.5 * kPi * ((f & 3) + t);
        return 0.25 * kPi * kPi * g.b * (g.a + g.b * cos(v));
    } else if (g.kind == GEOM_NURBS) {
#if defined(__HIP_DEVICE_COMPILE__)
        return nurbs_kappa(g.tab_dev, f, s, t);
#else
        return nurbs_kappa(g.tab_host, f, s, t);
#endif
    }
    return g.a * g.a;
}

// gamma_f(s, t) and its partial derivatives d_s gamma, d_t gamma (the Piola transform of
// div-conforming fields is D gamma (x) e_s, e_t)
__host__ __device__ inline void patch_jac(const GeomDesc& g, int f, double s, double t, double* x, double* xs,
                                          double* xt) {
    if (g.kind == GEOM_SPHERE6 || g.kind == GEOM_ELLIPSOID6) {
        int iu, iv, ic;
        double cv;
        cube_face_layout(f, iu, iv, ic, cv);
        double c[3];
        c[iu] = 2.0 * s - 1.0;
        c[iv] = 2.0 * t - 1.0;
        c[ic] = cv;
        const double rr = sqrt(c[0] * c[0] + c[1] * c[1] + c[2] * c[2]);
        const double n[3] = {c[0] / rr, c[1] / rr, c[2] / rr};
        const double sc[3] = {g.kind == GEOM_SPHERE6 ? 1.0 : g.a, g.kind == GEOM_SPHERE6 ? 1.0 : g.b,
                              g.kind == GEOM_SPHERE6 ? 1.0 : g.c};
        // d(c/|c|)/ds = (dc/ds - n (n . dc/ds)) / |c| with dc/ds = 2 e_iu (and e_iv for t)
        for (int d = 0; d < 3; ++d) {
            x[d] = sc[d] * n[d];
            xs[d] = sc[d] * 2.0 * ((d == iu ? 1.0 : 0.0) - n[d] * n[iu]) / rr;
            xt[d] = sc[d] * 2.0 * ((d == iv ? 1.0 : 0.0) - n[d] * n[iv]) / rr;
        }
    } else if (g.kind == GEOM_TORUS16) {
        const double u = 0.5 * kPi * ((f >> 2) + s), v = 0.5 * kPi * ((f & 3) + t);
        double su, cu, sv, cvv;
        sincos(u, &su, &cu);
        sincos(v, &sv, &cvv);
        const double rr = g.a + g.b * cvv, du = 0.5 * kPi;
        x[0] = rr * cu;
        x[1] = rr * su;
        x[2] = g.b * sv;
        xs[0] = -rr * su * du;
        xs[1] = rr * cu * du;
        xs[2] = 0.0;
        xt[0] = -g.b * sv * cu * du;
        xt[1] = -g.b * sv * su * du;
        xt[2] = g.b * cvv * du;
    } else if (g.kind == GEOM_NURBS) {
        // the out-of-line evaluation writes through pointers: it gets arrays of its own, so
        // that the caller's x, xs, xt can stay in registers on the other branches
        double px[3], ps[3], pt[3];
#if defined(__HIP_DEVICE_COMPILE__)
        nurbs_jac(g.tab_dev, f, s, t, px, ps, pt);
#else
        nurbs_jac(g.tab_host, f, s, t, px, ps, pt);
#endif
        for (int d = 0; d < 3; ++d) {
            x[d] = px[d];
            xs[d] = ps[d];
            xt[d] = pt[d];
        }
    } else {
        x[0] = g.a * s;
        x[1] = g.a * t;
        x[2] = 0.0;
        xs[0] = g.a;
        xs[1] = 0.0;
        xs[2] = 0.0;
        xt[0] = 0.0;
        xt[1] = g.a;
        xt[2] = 0.0;
    }
}

// ------------------------------------------------------------------ single-layer kernels
enum PdeKind : int { PDE_LAPLACE = 0, PDE_HELMHOLTZ = 1 };

struct KernelDesc {
    int pde;
    double kre, kim;  // wavenumber (Helmholtz)
};

// k(r) for Laplace: 1/(4 pi r)
__device__ inline double kernel_val(const KernelDesc&, double r2, double) {
    return kInv4Pi * rsqrt(r2);
}
// k(r) for Helmholtz: exp(-i kappa r)/(4 pi r), kappa = kre + i kim
__device__ inline cdbl kernel_val(const KernelDesc& k, double r2, cdbl) {
    const double ir = rsqrt(r2);
    const double r = r2 * ir;
    double s, c;
    sincos(k.kre * r, &s, &c);
    double mag = kInv4Pi * ir;
    if (k.kim != 0.0) mag *= exp(k.kim * r);
    return {mag * c, -mag * s};
}

// ------------------------------------------------------------------ space description
struct SpaceDesc {
    GeomDesc geom;
    KernelDesc ker;
    int d, r, L;       // degree, knot repetition, level
    int nel, nb;       // elements and B-splines per direction
    int64_t nelem, ndof;  // ndof: local functions (patch by patch)
    double h;          // element width 2^-L
    // Lifting to the surface: 2 for S^2 (2-form: the surface element cancels), 0 for S^0
    // (0-form: every surface integral carries kappa), whose local functions are glued across
    // patch boundaries into nglob global ones: glue[local] = global (device), and the local
    // functions of global g are ginv_idx[ginv_ptr[g] .. ginv_ptr[g+1]) (device).  S^2:
    // nglob = ndof and no maps.
    int form;
    int64_t nglob;
    const int32_t* glue;
    const int64_t* ginv_ptr;
    const int32_t* ginv_idx;
};

__host__ __device__ inline int64_t dof_id(const SpaceDesc& S, int f, int j1, int j2) {
    return ((int64_t)f * S.nb + j1) * S.nb + j2;
}
__host__ __device__ inline int64_t elem_id(const SpaceDesc& S, int f, int i1, int i2) {
    return ((int64_t)f * S.nel + i1) * S.nel + i2;
}

// D4 symmetry k of the unit square applied to (a, b): identity, flip first, flip second,
// flip both, then the same four after exchanging the coordinates.
__host__ __device__ inline void d4_apply(int k, double a, double b, double& o1, double& o2) {
    if (k >= 4) {
        const double tmp = a;
        a = b;
        b = tmp;
    }
    o1 = (k & 1) ? 1.0 - a : a;
    o2 = (k & 2) ? 1.0 - b : b;
}

// Touching element pair types
enum PairType : int { PT_REGULAR = 0, PT_VERTEX = 1, PT_EDGE = 2, PT_IDENTICAL = 3 };

// Duffy-type substitution of region `reg` for a touching pair of type `type` at the cube
// point (xi, e1, e2, e3): local points xh (first element) and yh (second element) with the
// Jacobian of the substitution.  Identical: 8 regions (4 sign patterns of y - x times the
// 2 simplices of (t1, t2)); edge (shared edge at first local coordinate 0 on both sides):
// 6 regions (sign of y2 - x2 times which of x1, y1, t is largest); vertex (shared vertex at
// the local origin on both sides): 4 regions (which of the 4 coordinates is largest).
__host__ __device__ inline void duffy_point(int type, int reg, double xi, double e1, double e2, double e3, double& x1,
                                   double& x2, double& y1, double& y2, double& jac) {
    if (type == PT_IDENTICAL) {
        const int ord = reg >> 2, sg = reg & 3;
        const double t1 = ord == 0 ? xi : xi * e1;
        const double t2 = ord == 0 ? xi * e1 : xi;
        const double u1 = e2, u2 = e3;
        const bool n1 = sg & 1, n2 = sg & 2;
        x1 = (1.0 - t1) * u1 + (n1 ? t1 : 0.0);
        x2 = (1.0 - t2) * u2 + (n2 ? t2 : 0.0);
        y1 = n1 ? x1 - t1 : x1 + t1;
        y2 = n2 ? x2 - t2 : x2 + t2;
        jac = xi * (1.0 - t1) * (1.0 - t2);
    } else if (type == PT_EDGE) {
        const int c = reg >> 1;
        const bool neg = reg & 1;
        double v[3];
        v[0] = c == 0 ? xi : xi * e1;
        v[1] = c == 1 ? xi : (c == 0 ? xi * e1 : xi * e2);
        v[2] = c == 2 ? xi : xi * e2;
        const double t = v[2];
        x1 = v[0];
        y1 = v[1];
        x2 = (1.0 - t) * e3 + (neg ? t : 0.0);
        y2 = neg ? x2 - t : x2 + t;
        jac = xi * xi * (1.0 - t);
    } else {
        // coordinate `reg` of (x1, x2, y1, y2) is xi, the others xi*e1, xi*e2, xi*e3 in order
        x1 = reg == 0 ? xi : xi * e1;
        x2 = reg == 1 ? xi : (reg < 1 ? xi * e1 : xi * e2);
        y1 = reg == 2 ? xi : (reg < 2 ? xi * e2 : xi * e3);
        y2 = reg == 3 ? xi : xi * e3;
        jac = xi * xi * xi;
    }
}

}  // namespace bem
