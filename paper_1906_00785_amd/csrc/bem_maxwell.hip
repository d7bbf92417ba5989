// gfx950 kernels of the Maxwell single layer on the div-conforming spaces S^1 (App. E):
// element-pair blocks (regular pairs by tensor Gauss rules, touching pairs by the Duffy
// rules of the scalar operators), the glued dense matrix and its product, load vectors and
// the field (MS).
#include "bem_device.h"
#include "bem_maxwell.h"

namespace bem {

namespace {

__device__ inline cdbl cmul(cdbl a, cdbl b) { return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; }

// exp(-i kappa r) with kappa = kre + i kim
__device__ inline cdbl cexp_mikr(const KernelDesc& k, double r) {
    double s, c;
    sincos(k.kre * r, &s, &c);
    const double mag = k.kim != 0.0 ? exp(k.kim * r) : 1.0;
    return {mag * c, -mag * s};
}

// the local functions of element (f, i1, i2) at element coordinates (u1, u2): point x, the
// lifted fields V[k] = D gamma (reference field) and the reference divergences D[k], in the
// order: component 0 (degree p in s, p - 1 in t; l1 outer), then component 1
template <int P>
__device__ inline void mx_eval(const MxDev& d, int f, int i1, int i2, double u1, double u2, double* x,
                               double (*V)[3], double* D) {
    double xs[3], xt[3];
    patch_jac(d.geom, f, (i1 + u1) * d.h, (i2 + u2) * d.h, x, xs, xt);
    const double ih = 1.0 / d.h;
    double bp1[P + 1], dp1[P + 1], bp2[P + 1], dp2[P + 1], bq1[P], bq2[P];
    const double* c1 = d.polp + (int64_t)i1 * (P + 1) * (P + 1);
    const double* c2 = d.polp + (int64_t)i2 * (P + 1) * (P + 1);
#pragma unroll
    for (int l = 0; l <= P; ++l) {
        double v1 = c1[l * (P + 1) + P], v2 = c2[l * (P + 1) + P], w1 = 0.0, w2 = 0.0;
#pragma unroll
        for (int k = P - 1; k >= 0; --k) {
            w1 = w1 * u1 + v1;  // derivative by Horner alongside the value
            w2 = w2 * u2 + v2;
            v1 = v1 * u1 + c1[l * (P + 1) + k];
            v2 = v2 * u2 + c2[l * (P + 1) + k];
        }
        bp1[l] = v1;
        bp2[l] = v2;
        dp1[l] = w1 * ih;
        dp2[l] = w2 * ih;
    }
    const double* q1 = d.polq + (int64_t)i1 * P * P;
    const double* q2 = d.polq + (int64_t)i2 * P * P;
#pragma unroll
    for (int l = 0; l < P; ++l) {
        double v1 = q1[l * P + P - 1], v2 = q2[l * P + P - 1];
#pragma unroll
        for (int k = P - 2; k >= 0; --k) {
            v1 = v1 * u1 + q1[l * P + k];
            v2 = v2 * u2 + q2[l * P + k];
        }
        bq1[l] = v1;
        bq2[l] = v2;
    }
    int k = 0;
#pragma unroll
    for (int l1 = 0; l1 <= P; ++l1)
#pragma unroll
        for (int l2 = 0; l2 < P; ++l2, ++k) {
            const double b = bp1[l1] * bq2[l2];
            V[k][0] = xs[0] * b;
            V[k][1] = xs[1] * b;
            V[k][2] = xs[2] * b;
            D[k] = dp1[l1] * bq2[l2];
        }
#pragma unroll
    for (int l1 = 0; l1 < P; ++l1)
#pragma unroll
        for (int l2 = 0; l2 <= P; ++l2, ++k) {
            const double b = bq1[l1] * bp2[l2];
            V[k][0] = xt[0] * b;
            V[k][1] = xt[1] * b;
            V[k][2] = xt[2] * b;
            D[k] = bq1[l1] * dp2[l2];
        }
}

// The local functions of element (f, i1, i2) at (u1, u2) in factored form: point x, the
// tangents xs = d_s gamma and xt = d_t gamma, the scalar factors b[k] (the lifted field of
// function k is xs b[k] for component 0, k < p (p + 1), and xt b[k] for component 1) and the
// reference divergences dv[k]; the order of mx_eval.
template <int P>
__device__ inline void mx_eval_f(const MxDev& d, int f, int i1, int i2, double u1, double u2, double* x,
                                 double* xs, double* xt, double* bv, double* dv) {
    patch_jac(d.geom, f, (i1 + u1) * d.h, (i2 + u2) * d.h, x, xs, xt);
    const double ih = 1.0 / d.h;
    double bp1[P + 1], dp1[P + 1], bp2[P + 1], dp2[P + 1], bq1[P], bq2[P];
    const double* c1 = d.polp + (int64_t)i1 * (P + 1) * (P + 1);
    const double* c2 = d.polp + (int64_t)i2 * (P + 1) * (P + 1);
#pragma unroll
    for (int l = 0; l <= P; ++l) {
        double v1 = c1[l * (P + 1) + P], v2 = c2[l * (P + 1) + P], w1 = 0.0, w2 = 0.0;
#pragma unroll
        for (int k = P - 1; k >= 0; --k) {
            w1 = w1 * u1 + v1;
            w2 = w2 * u2 + v2;
            v1 = v1 * u1 + c1[l * (P + 1) + k];
            v2 = v2 * u2 + c2[l * (P + 1) + k];
        }
        bp1[l] = v1;
        bp2[l] = v2;
        dp1[l] = w1 * ih;
        dp2[l] = w2 * ih;
    }
    const double* q1 = d.polq + (int64_t)i1 * P * P;
    const double* q2 = d.polq + (int64_t)i2 * P * P;
#pragma unroll
    for (int l = 0; l < P; ++l) {
        double v1 = q1[l * P + P - 1], v2 = q2[l * P + P - 1];
#pragma unroll
        for (int k = P - 2; k >= 0; --k) {
            v1 = v1 * u1 + q1[l * P + k];
            v2 = v2 * u2 + q2[l * P + k];
        }
        bq1[l] = v1;
        bq2[l] = v2;
    }
    int k = 0;
#pragma unroll
    for (int l1 = 0; l1 <= P; ++l1)
#pragma unroll
        for (int l2 = 0; l2 < P; ++l2, ++k) {
            bv[k] = bp1[l1] * bq2[l2];
            dv[k] = dp1[l1] * bq2[l2];
        }
#pragma unroll
    for (int l1 = 0; l1 < P; ++l1)
#pragma unroll
        for (int l2 = 0; l2 <= P; ++l2, ++k) {
            bv[k] = bq1[l1] * bp2[l2];
            dv[k] = bq1[l1] * dp2[l2];
        }
}

// Element-pair block B[i][j] = int_tau int_sigma G(x, y) [V_i(x) . V_j(y) - kappa^-2 D_i(x) D_j(y)]
// over the parameter squares (times h^4), i test, j trial.  Block blk = blist[...] of the
// launch; its element pair is plist[blk] (or blk itself without a list), its type tinfo[blk].
__device__ inline void mx_pair_of(const MxDev& d, int64_t blk, int& tf, int& ti1, int& ti2, int& sf, int& si1,
                                  int& si2) {
    const int64_t pr = d.plist ? d.plist[blk] : blk;
    const int64_t e1 = pr / d.nelem, e2 = pr % d.nelem;
    const int n = d.nel;
    ti2 = (int)(e1 % n);
    ti1 = (int)((e1 / n) % n);
    tf = (int)(e1 / ((int64_t)n * n));
    si2 = (int)(e2 % n);
    si1 = (int)((e2 / n) % n);
    sf = (int)(e2 / ((int64_t)n * n));
}

// B = (vector part - kappa^-2 divergence part) h^4 for this lane's entries
template <int NL, int NE>
__device__ inline void mx_store_block(const MxDev& d, int64_t blk, int lane, const double (*accr)[2],
                                      const double (*acci)[2]) {
    const double h2 = d.h * d.h, h4 = h2 * h2;
    const cdbl k2 = cmul(cdbl{d.ker.kre, d.ker.kim}, cdbl{d.ker.kre, d.ker.kim});
    const double den = k2.re * k2.re + k2.im * k2.im;
    const cdbl mik2 = {-k2.re / den, k2.im / den};  // -1 / kappa^2
    cdbl* B = (cdbl*)d.B + blk * NL * NL;
#pragma unroll
    for (int e = 0; e < NE; ++e) {
        const int ent = lane + 64 * e;
        if (ent >= NL * NL) continue;
        const cdbl dv = cmul(mik2, cdbl{accr[e][1], acci[e][1]});
        B[ent] = cdbl{(accr[e][0] + dv.re) * h4, (acci[e][0] + dv.im) * h4};
    }
}

// Regular pairs, one wave each: lane b is trial point b and sums F_b[i][c] =
// sum_a w_a G(x_a, y_b) Wx_a[i][c] over the qg^2 test points (uniform, from LDS), channel c =
// field component 0..2 or the divergence 3; then B[i][j] += sum_b F_b[i][c] w_b Wy_b[j][c]
// from LDS.  The test-side tables and the contraction operands share the LDS.
template <int P>
__global__ __launch_bounds__(64) void k_mx_regular(MxDev d) {
    constexpr int NL = 2 * P * (P + 1), NC = 4 * NL, NE = (NL * NL + 63) / 64;
    extern __shared__ double sm[];
    double* WX = sm;               // [64][NC] test-side values times weights (phase 1)
    double* Xt = sm + 64 * NC;     // [64][3] test points (phase 1)
    double* Fr = sm;               // [64][NC] (phase 2)
    double* Fi = sm + 64 * NC;     // [64][NC]
    double* Wl = sm + 128 * NC;    // [64][NC]
    const int64_t blk = d.blist[blockIdx.x];
    int tf, ti1, ti2, sf, si1, si2;
    mx_pair_of(d, blk, tf, ti1, ti2, sf, si1, si2);
    const int lane = threadIdx.x;
    const int qg = d.qg, np = qg * qg;  // qg * qg <= 64 (checked at planning)
    double x[3], V[NL][3], D[NL];
    if (lane < np) {
        const int a1 = lane / qg, a2 = lane % qg;
        mx_eval<P>(d, tf, ti1, ti2, d.gx[a1], d.gx[a2], x, V, D);
        const double w = d.gw[a1] * d.gw[a2];
        Xt[3 * lane] = x[0];
        Xt[3 * lane + 1] = x[1];
        Xt[3 * lane + 2] = x[2];
#pragma unroll
        for (int k = 0; k < NL; ++k) {
            WX[lane * NC + 4 * k] = w * V[k][0];
            WX[lane * NC + 4 * k + 1] = w * V[k][1];
            WX[lane * NC + 4 * k + 2] = w * V[k][2];
            WX[lane * NC + 4 * k + 3] = w * D[k];
        }
    }
    __syncthreads();
    double Sr[NC], Si[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) Sr[c] = Si[c] = 0.0;
    const int b1 = lane / qg, b2 = lane % qg;
    if (lane < np) {
        double y[3], ys[3], yt[3];
        patch_jac(d.geom, sf, (si1 + d.gx[b1]) * d.h, (si2 + d.gx[b2]) * d.h, y, ys, yt);
        for (int a = 0; a < np; ++a) {
            const double dx = Xt[3 * a] - y[0], dy = Xt[3 * a + 1] - y[1], dz = Xt[3 * a + 2] - y[2];
            const cdbl G = kernel_val(d.ker, dx * dx + dy * dy + dz * dz, cdbl{0.0, 0.0});
            const double* wx = WX + a * NC;
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                Sr[c] += G.re * wx[c];
                Si[c] += G.im * wx[c];
            }
        }
    }
    __syncthreads();  // phase 1 tables dead
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        Fr[lane * NC + c] = Sr[c];
        Fi[lane * NC + c] = Si[c];
    }
    double wb = 0.0;
    if (lane < np) {
        mx_eval<P>(d, sf, si1, si2, d.gx[b1], d.gx[b2], x, V, D);
        wb = d.gw[b1] * d.gw[b2];
    }
#pragma unroll
    for (int k = 0; k < NL; ++k) {
        Wl[lane * NC + 4 * k] = lane < np ? wb * V[k][0] : 0.0;
        Wl[lane * NC + 4 * k + 1] = lane < np ? wb * V[k][1] : 0.0;
        Wl[lane * NC + 4 * k + 2] = lane < np ? wb * V[k][2] : 0.0;
        Wl[lane * NC + 4 * k + 3] = lane < np ? wb * D[k] : 0.0;
    }
    __syncthreads();
    double accr[NE][2], acci[NE][2];  // [entry][vector part, divergence part]
#pragma unroll
    for (int e = 0; e < NE; ++e) {
        accr[e][0] = accr[e][1] = acci[e][0] = acci[e][1] = 0.0;
        const int ent = lane + 64 * e;
        if (ent >= NL * NL) continue;
        const int i = ent / NL, j = ent % NL;
        for (int b = 0; b < 64; ++b) {
            const double* fr = Fr + b * NC + 4 * i;
            const double* fi = Fi + b * NC + 4 * i;
            const double* w = Wl + b * NC + 4 * j;
            accr[e][0] += fr[0] * w[0] + fr[1] * w[1] + fr[2] * w[2];
            acci[e][0] += fi[0] * w[0] + fi[1] * w[1] + fi[2] * w[2];
            accr[e][1] += fr[3] * w[3];
            acci[e][1] += fi[3] * w[3];
        }
    }
    mx_store_block<NL, NE>(d, blk, lane, accr, acci);
}

// Touching pairs (identical, common edge, common vertex), one wave each, over the Duffy
// points of the scalar operators in batches of 32: the lower half-wave evaluates the test
// side of point p, the upper half the trial side of the same point, and the lower half
// takes the trial geometry from its partner lane.  Per point the lower lane stores the five
// kernel weights w G (t_a(x) . t_b(y)) (a, b = s, t: the tangents of the two components) and
// w G, and both halves their factors b and divergences; each lane then adds its block
// entries over the batch: B_vec[i][j] += w G (t_(c i)(x) . t_(c j)(y)) b_i(x) b_j(y),
// B_div[i][j] += w G dv_i(x) dv_j(y).
template <int P>
__global__ __launch_bounds__(64) void k_mx_touch(MxDev d) {
    constexpr int NL = 2 * P * (P + 1), NE = (NL * NL + 63) / 64, NC0 = (P + 1) * P;
    constexpr int ST = 10 + 4 * NL;  // per point: 5 complex weights, bx, dx, by, dy
    __shared__ double T[32][ST];
    const int64_t blk = d.blist[d.nreg + blockIdx.x];
    int tf, ti1, ti2, sf, si1, si2;
    mx_pair_of(d, blk, tf, ti1, ti2, sf, si1, si2);
    const int info = d.tinfo[blk];
    const int type = info & 15, k1 = (info >> 4) & 15, k2 = (info >> 8) & 15;
    const int lane = threadIdx.x, half = lane >> 5, pl = lane & 31;
    const int qs = d.qs, qs4 = qs * qs * qs * qs;
    const int nreg = type == PT_IDENTICAL ? 8 : (type == PT_EDGE ? 6 : 4);
    const int npts = nreg * qs4;
    double accr[NE][2], acci[NE][2];
#pragma unroll
    for (int e = 0; e < NE; ++e) accr[e][0] = accr[e][1] = acci[e][0] = acci[e][1] = 0.0;
    for (int p0 = 0; p0 < npts; p0 += 32) {
        const int pt = p0 + pl;
        double X[3] = {0.0, 0.0, 0.0}, Xs[3] = {0.0, 0.0, 0.0}, Xt[3] = {0.0, 0.0, 0.0}, bv[NL], dv[NL], w = 0.0;
#pragma unroll
        for (int k = 0; k < NL; ++k) bv[k] = dv[k] = 0.0;
        if (pt < npts) {
            const int reg = pt / qs4;
            int rem = pt - reg * qs4;
            const int i3 = rem % qs;
            rem /= qs;
            const int i2 = rem % qs;
            rem /= qs;
            const int i1 = rem % qs, i0 = rem / qs;
            double xh1, xh2, yh1, yh2, jac, u1, u2;
            duffy_point(type, reg, d.sx[i0], d.sx[i1], d.sx[i2], d.sx[i3], xh1, xh2, yh1, yh2, jac);
            if (half == 0) {
                d4_apply(k1, xh1, xh2, u1, u2);
                mx_eval_f<P>(d, tf, ti1, ti2, u1, u2, X, Xs, Xt, bv, dv);
            } else {
                d4_apply(k2, yh1, yh2, u1, u2);
                mx_eval_f<P>(d, sf, si1, si2, u1, u2, X, Xs, Xt, bv, dv);
            }
            w = d.sw[i0] * d.sw[i1] * d.sw[i2] * d.sw[i3] * jac;
        }
        double Y[3], Ys[3], Yt[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            Y[c] = __shfl_xor(X[c], 32, 64);
            Ys[c] = __shfl_xor(Xs[c], 32, 64);
            Yt[c] = __shfl_xor(Xt[c], 32, 64);
        }
        __syncthreads();  // the previous batch has been read
        double* t = T[pl];
        if (half == 0) {
            cdbl g = {0.0, 0.0};
            if (pt < npts) {
                const double dx = X[0] - Y[0], dy = X[1] - Y[1], dz = X[2] - Y[2];
                g = kernel_val(d.ker, dx * dx + dy * dy + dz * dz, cdbl{0.0, 0.0}) * w;
            }
            const double ss = Xs[0] * Ys[0] + Xs[1] * Ys[1] + Xs[2] * Ys[2];
            const double st = Xs[0] * Yt[0] + Xs[1] * Yt[1] + Xs[2] * Yt[2];
            const double ts = Xt[0] * Ys[0] + Xt[1] * Ys[1] + Xt[2] * Ys[2];
            const double tt = Xt[0] * Yt[0] + Xt[1] * Yt[1] + Xt[2] * Yt[2];
            t[0] = g.re * ss;
            t[1] = g.im * ss;
            t[2] = g.re * st;
            t[3] = g.im * st;
            t[4] = g.re * ts;
            t[5] = g.im * ts;
            t[6] = g.re * tt;
            t[7] = g.im * tt;
            t[8] = g.re;
            t[9] = g.im;
#pragma unroll
            for (int k = 0; k < NL; ++k) {
                t[10 + k] = bv[k];
                t[10 + NL + k] = dv[k];
            }
        } else {
#pragma unroll
            for (int k = 0; k < NL; ++k) {
                t[10 + 2 * NL + k] = bv[k];
                t[10 + 3 * NL + k] = dv[k];
            }
        }
        __syncthreads();
        for (int p = 0; p < 32; ++p) {
            const double* u = T[p];
            const double gdr = u[8], gdi = u[9];
#pragma unroll
            for (int e = 0; e < NE; ++e) {
                const int ent = lane + 64 * e;
                if (ent >= NL * NL) continue;
                const int i = ent / NL, j = ent % NL;
                const int gi = 2 * (2 * (i >= NC0) + (j >= NC0));
                const double bb = u[10 + i] * u[10 + 2 * NL + j];
                const double dd = u[10 + NL + i] * u[10 + 3 * NL + j];
                accr[e][0] += u[gi] * bb;
                acci[e][0] += u[gi + 1] * bb;
                accr[e][1] += gdr * dd;
                acci[e][1] += gdi * dd;
            }
        }
    }
    mx_store_block<NL, NE>(d, blk, lane, accr, acci);
}

// M[g][h]: one thread per entry, the pieces of g (outer) and h (inner) in table order
__global__ __launch_bounds__(256) void k_mx_gather(MxDev d) {
    const int64_t id = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t N = d.nglob;
    if (id >= N * N) return;
    const int64_t g = id / N, hc = id % N;
    const int nl = d.nl;
    const cdbl* B = (const cdbl*)d.B;
    double sr = 0.0, si = 0.0;
    for (int64_t a = d.gptr[g]; a < d.gptr[g + 1]; ++a) {
        const int pa = d.gpos[a], ea = pa / nl, ia = pa % nl;
        const double sa = d.gsgn[a];
        for (int64_t b = d.gptr[hc]; b < d.gptr[hc + 1]; ++b) {
            const int pb = d.gpos[b], eb = pb / nl, ib = pb % nl;
            const cdbl v = B[((int64_t)ea * d.nelem + eb) * nl * nl + ia * nl + ib];
            const double s = sa * d.gsgn[b];
            sr += s * v.re;
            si += s * v.im;
        }
    }
    ((cdbl*)d.M)[id] = cdbl{sr, si};
}

// y = M x, one wave per row
__global__ __launch_bounds__(256) void k_mx_matvec(MxDev d, const cdbl* __restrict__ x, cdbl* __restrict__ y) {
    const int64_t g = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (g >= d.nglob) return;
    const cdbl* row = (const cdbl*)d.M + g * d.nglob;
    double sr = 0.0, si = 0.0;
    for (int64_t h = lane; h < d.nglob; h += 64) {
        const cdbl a = row[h], b = x[h];
        sr += a.re * b.re - a.im * b.im;
        si += a.re * b.im + a.im * b.re;
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        sr += __shfl_xor(sr, o, 64);
        si += __shfl_xor(si, o, 64);
    }
    if (lane == 0) y[g] = cdbl{sr, si};
}

// data fields: 0 the point dipole curl curl (m G(x - x0)) = kappa^2 m G + grad (m . grad G),
// 1 the plane wave e exp(-i kappa d . x)
__device__ inline void mx_data(const KernelDesc& kd, int kind, const double* p, const double* x, cdbl* E) {
    if (kind == 0) {
        const double R[3] = {x[0] - p[0], x[1] - p[1], x[2] - p[2]};
        const double r = sqrt(R[0] * R[0] + R[1] * R[1] + R[2] * R[2]);
        const cdbl ex = cexp_mikr(kd, r) * (0.07957747154594767);  // exp(-i kappa r) / (4 pi)
        const cdbl ik = {-kd.kim, kd.kre};                        // i kappa
        const cdbl one_ikr = {1.0 + ik.re * r, ik.im * r};
        const cdbl ikr2 = cmul(ik, ik) * (r * r);
        const cdbl G = ex * (1.0 / r);
        const cdbl G1 = cmul(ex, one_ikr) * (-1.0 / (r * r));
        const cdbl G2 = cmul(ex, cdbl{2.0 + 2.0 * ik.re * r + ikr2.re, 2.0 * ik.im * r + ikr2.im}) * (1.0 / (r * r * r));
        const cdbl g = G1 * (1.0 / r);
        const cdbl gp = (G2 - G1 * (1.0 / r)) * (1.0 / r);
        const cdbl k2 = cmul(cdbl{kd.kre, kd.kim}, cdbl{kd.kre, kd.kim});
        const double mR = p[3] * R[0] + p[4] * R[1] + p[5] * R[2];
        for (int c = 0; c < 3; ++c)
            E[c] = cmul(k2, G) * p[3 + c] + gp * (mR * R[c] / r) + g * p[3 + c];
    } else {
        const cdbl ph = cexp_mikr(kd, p[0] * x[0] + p[1] * x[1] + p[2] * x[2]);
        for (int c = 0; c < 3; ++c) E[c] = ph * p[3 + c];
    }
}

// b_g = sum over the pieces (element, position, sign) of g of the 8 x 8 Gauss sums of
// E(gamma) . V; one wave per global function, lane = Gauss point
template <int P>
__global__ __launch_bounds__(256) void k_mx_rhs(MxDev d, Gauss8 g8, int kind, double p0, double p1, double p2,
                                                double p3, double p4, double p5, cdbl* b) {
    constexpr int NL = 2 * P * (P + 1);
    const int64_t G = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (G >= d.nglob) return;
    const double prm[6] = {p0, p1, p2, p3, p4, p5};
    const int n = d.nel, a1 = lane >> 3, a2 = lane & 7;
    double sr = 0.0, si = 0.0;
    for (int64_t a = d.gptr[G]; a < d.gptr[G + 1]; ++a) {
        const int pa = d.gpos[a], e = pa / NL, pos = pa % NL;
        const int i2 = e % n, i1 = (e / n) % n, f = e / (n * n);
        double x[3], V[NL][3], D[NL];
        mx_eval<P>(d, f, i1, i2, g8.x[a1], g8.x[a2], x, V, D);
        cdbl E[3];
        mx_data(d.ker, kind, prm, x, E);
        const double w = g8.w[a1] * g8.w[a2] * d.h * d.h * d.gsgn[a];
        sr += w * (E[0].re * V[pos][0] + E[1].re * V[pos][1] + E[2].re * V[pos][2]);
        si += w * (E[0].im * V[pos][0] + E[1].im * V[pos][1] + E[2].im * V[pos][2]);
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        sr += __shfl_xor(sr, o, 64);
        si += __shfl_xor(si, o, 64);
    }
    if (lane == 0) b[G] = cdbl{sr, si};
}

// E(x_p) = sum over elements and 8 x 8 Gauss points of w [G J + kappa^-2 G'(r) (x - y)/r Div],
// J and Div the density and its divergence at the point; one workgroup per point
template <int P>
__global__ __launch_bounds__(256) void k_mx_field(MxDev d, Gauss8 g8, const double* __restrict__ pts,
                                                  const cdbl* __restrict__ j, cdbl* __restrict__ out) {
    constexpr int NL = 2 * P * (P + 1);
    __shared__ double red[6][4];
    const int64_t p = blockIdx.x;
    const double px = pts[3 * p], py = pts[3 * p + 1], pz = pts[3 * p + 2];
    const int n = d.nel;
    const cdbl k2 = cmul(cdbl{d.ker.kre, d.ker.kim}, cdbl{d.ker.kre, d.ker.kim});
    const double den = k2.re * k2.re + k2.im * k2.im;
    const cdbl ik2 = {k2.re / den, -k2.im / den};  // 1 / kappa^2
    const cdbl ik = {-d.ker.kim, d.ker.kre};
    double acc[6] = {0, 0, 0, 0, 0, 0};
    const int64_t total = d.nelem * 64;
    for (int64_t idx = threadIdx.x; idx < total; idx += blockDim.x) {
        const int a = (int)(idx & 63);
        const int64_t e = idx >> 6;
        const int i2 = (int)(e % n), i1 = (int)((e / n) % n), f = (int)(e / ((int64_t)n * n));
        double y[3], V[NL][3], D[NL];
        mx_eval<P>(d, f, i1, i2, g8.x[a >> 3], g8.x[a & 7], y, V, D);
        cdbl J[3] = {{0, 0}, {0, 0}, {0, 0}}, Dv = {0, 0};
#pragma unroll
        for (int k = 0; k < NL; ++k) {
            const int gk = d.eglob[e * NL + k];
            if (gk < 0) continue;
            const cdbl c = j[gk] * (double)d.esgn[e * NL + k];
            J[0] = J[0] + c * V[k][0];
            J[1] = J[1] + c * V[k][1];
            J[2] = J[2] + c * V[k][2];
            Dv = Dv + c * D[k];
        }
        const double R[3] = {px - y[0], py - y[1], pz - y[2]};
        const double r = sqrt(R[0] * R[0] + R[1] * R[1] + R[2] * R[2]);
        const cdbl ex = cexp_mikr(d.ker, r) * 0.07957747154594767;
        const cdbl G = ex * (1.0 / r);
        const cdbl G1 = cmul(ex, cdbl{1.0 + ik.re * r, ik.im * r}) * (-1.0 / (r * r));
        const double w = g8.w[a >> 3] * g8.w[a & 7] * d.h * d.h;
        const cdbl gd = cmul(cmul(ik2, G1), Dv) * (w / r);
        for (int c = 0; c < 3; ++c) {
            const cdbl v = cmul(G, J[c]) * w + gd * R[c];
            acc[2 * c] += v.re;
            acc[2 * c + 1] += v.im;
        }
    }
#pragma unroll
    for (int c = 0; c < 6; ++c) {
        double v = acc[c];
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
        if ((threadIdx.x & 63) == 0) red[c][threadIdx.x >> 6] = v;
    }
    __syncthreads();
    if (threadIdx.x < 3) {
        const int c = threadIdx.x;
        out[3 * p + c] = cdbl{red[2 * c][0] + red[2 * c][1] + red[2 * c][2] + red[2 * c][3],
                              red[2 * c + 1][0] + red[2 * c + 1][1] + red[2 * c + 1][2] + red[2 * c + 1][3]};
    }
}

// ------------------------------------------------------------------ compressed operator
// Cluster c = (level, patch, i, j) of the uniform quadtree of every patch.
__device__ inline void cluster_of(const MxhDev& d, int64_t c, int& lev, int& f, int& i, int& j) {
    lev = 0;
    while (c >= d.lev_off[lev + 1]) ++lev;
    const int64_t loc = c - d.lev_off[lev];
    const int n = 1 << lev;
    j = (int)(loc % n);
    i = (int)((loc / n) % n);
    f = (int)(loc / ((int64_t)n * n));
}

// element of leaf l (leaf-local index) at position v (row-major m x m); the leaves per
// direction and the elements per leaf and direction are powers of two
__device__ inline int64_t leaf_elem(const MxhDev& d, int64_t l, int v) {
    const int s1 = __builtin_ctz(d.nleaf1), sm = __builtin_ctz(d.m);
    const int64_t f = l >> (2 * s1);
    const int li = (int)(l >> s1) & (d.nleaf1 - 1), lj = (int)l & (d.nleaf1 - 1);
    return (f * d.s.nel + (li << sm) + (v >> sm)) * d.s.nel + (lj << sm) + (v & (d.m - 1));
}

// Chebyshev points of every cluster on the surface; one thread per (cluster, node)
__global__ __launch_bounds__(256) void k_mxh_points(MxhDev d) {
    const int64_t id = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (id >= d.ncl * d.q2) return;
    const int64_t c = id / d.q2;
    const int a = (int)(id % d.q2);
    int lev, f, i, j;
    cluster_of(d, c, lev, f, i, j);
    const double w = 1.0 / (double)(1 << lev);
    patch_point(d.s.geom, f, (i + d.cheb[a / d.q]) * w, (j + d.cheb[a % d.q]) * w, d.xc + 3 * id);
}

// kernel at the nodes of every stored admissible pair, stored [block][partner node b][owner node a]
__global__ __launch_bounds__(256) void k_mxh_far(MxhDev d) {
    const int64_t id = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t per = (int64_t)d.q2 * d.q2;
    if (id >= d.nstored * per) return;
    const int64_t pr = id / per;
    const int rem = (int)(id % per), b = rem / d.q2, a = rem % d.q2;
    const double* x = d.xc + ((int64_t)d.own_t[pr] * d.q2 + a) * 3;
    const double* y = d.xc + ((int64_t)d.own_s[pr] * d.q2 + b) * 3;
    const double dx = x[0] - y[0], dy = x[1] - y[1], dz = x[2] - y[2];
    ((cdbl*)d.K)[id] = kernel_val(d.s.ker, dx * dx + dy * dy + dz * dz, cdbl{0.0, 0.0});
}

// Channel moments of every element against its leaf's Lagrange polynomials:
// Mt[e][k][c][a] = h^2 sum over the qg x qg Gauss points of w W_c,k L_a1 L_a2.
// One 64-lane block per element, lane = Gauss point; the products are summed from LDS.
template <int P>
__global__ __launch_bounds__(64) void k_mxh_moments(MxhDev d) {
    constexpr int NL = 2 * P * (P + 1), NC = 4 * NL;
    __shared__ double W[64][NC];
    __shared__ double L1[64][8], L2[64][8];
    const int64_t e = blockIdx.x;
    const int lane = threadIdx.x;
    const int n = d.s.nel, qg = d.s.qg, q = d.q, m = d.m;
    const int i2 = (int)(e % n), i1 = (int)((e / n) % n), f = (int)(e / ((int64_t)n * n));
    const int np = qg * qg;
    if (lane < np) {
        const int k1 = lane / qg, k2 = lane % qg;
        double x[3], V[NL][3], D[NL];
        mx_eval<P>(d.s, f, i1, i2, d.s.gx[k1], d.s.gx[k2], x, V, D);
        const double w = d.s.gw[k1] * d.s.gw[k2] * d.s.h * d.s.h;
#pragma unroll
        for (int k = 0; k < NL; ++k) {
            W[lane][4 * k] = w * V[k][0];
            W[lane][4 * k + 1] = w * V[k][1];
            W[lane][4 * k + 2] = w * V[k][2];
            W[lane][4 * k + 3] = w * D[k];
        }
        for (int a = 0; a < q; ++a) {
            L1[lane][a] = d.Lg[((i1 % m) * qg + k1) * q + a];
            L2[lane][a] = d.Lg[((i2 % m) * qg + k2) * q + a];
        }
    }
    __syncthreads();
    const int q2 = d.q2, nout = NC * q2;
    double* out = d.Mt + e * (int64_t)nout;
    for (int o = lane; o < nout; o += 64) {
        const int kc = o / q2, a = o % q2, a1 = a / q, a2 = a % q;
        double acc = 0.0;
        for (int pt = 0; pt < np; ++pt) acc += W[pt][kc] * L1[pt][a1] * L2[pt][a2];
        out[o] = acc;
    }
}

// Leaf moments (forward transform): mom[leaf][c][a] = sum over its elements and their
// functions of Mt[e][k][c][a] xl[e][k], xl[e][k] = sign * x[global function of (e, k)] (0
// for dropped functions) read straight from x; lanes over (c, a).  With one element per leaf, one
// wave per leaf; otherwise one workgroup per leaf, wave w taking the leaf's elements w,
// w + 4, ..., and the four waves' sums added in a fixed order.  All loads of an element are
// issued before its products.
template <int P, int NO>
__global__ __launch_bounds__(256) void k_mxh_forward(MxhDev d, const cdbl* __restrict__ x) {
    constexpr int NL = 2 * P * (P + 1);
    __shared__ cdbl red[4][64 * NO];
    const int w = uniform_int(threadIdx.x >> 6), lane = threadIdx.x & 63;
    const int m2 = d.m * d.m, nout = 4 * d.q2;
    const bool one = m2 == 1;
    const int64_t l = one ? (int64_t)blockIdx.x * 4 + w : (int64_t)blockIdx.x;
    if (l >= d.nleaves) return;  // uniform over the workgroup unless one == true
    cdbl acc[NO];
#pragma unroll
    for (int u = 0; u < NO; ++u) acc[u] = cdbl{0.0, 0.0};
    for (int v = one ? 0 : w; v < m2; v += 4) {
        const int64_t e = leaf_elem(d, l, v);
        const double* mt = d.Mt + e * NL * (int64_t)nout;
        cdbl xv[NL];
        double mv[NL][NO];
#pragma unroll
        for (int k = 0; k < NL; ++k) {
            const int gk = d.s.eglob[e * NL + k];  // the element's signed coefficients
            xv[k] = gk < 0 ? cdbl{0.0, 0.0} : x[gk] * (double)d.s.esgn[e * NL + k];
#pragma unroll
            for (int u = 0; u < NO; ++u) {
                const int o = lane + 64 * u;
                const double x = mt[k * nout + (o < nout ? o : 0)];  // loads without branches
                mv[k][u] = o < nout ? x : 0.0;
            }
        }
#pragma unroll
        for (int k = 0; k < NL; ++k)
#pragma unroll
            for (int u = 0; u < NO; ++u) acc[u] = acc[u] + xv[k] * mv[k][u];
    }
    cdbl* mom = (cdbl*)d.mom + (d.lev_off[d.leaf] + l) * nout;
    if (one) {
#pragma unroll
        for (int u = 0; u < NO; ++u) {
            const int o = lane + 64 * u;
            if (o < nout) mom[o] = acc[u];
        }
        return;
    }
#pragma unroll
    for (int u = 0; u < NO; ++u) red[w][lane + 64 * u] = acc[u];
    __syncthreads();
    if (w == 0)
#pragma unroll
        for (int u = 0; u < NO; ++u) {
            const int o = lane + 64 * u;
            if (o < nout) mom[o] = (red[0][o] + red[1][o]) + (red[2][o] + red[3][o]);
        }
}

typedef const __attribute__((address_space(4))) double* mx_cdptr;
typedef const __attribute__((address_space(4))) int32_t* mx_ciptr;

// Upward transfer to level lev: m_P[c][a] = sum over the four children b and their nodes p
// of E_b1[p1][a1] E_b2[p2][a2] m_child[c][p]; one wave per parent, lanes over (c, a).  The
// children's moments are staged in the wave's LDS slice (coalesced); each lane holds the
// transfer entries of its node in registers, so the sums run without memory waits.
// sm: the four children [b = 2 b1 + b2][c][p]; the parent's moments go to out (and to lds
// when given).
template <int Q>
__device__ inline void mxh_up_transfer(const MxhDev& d, const cdbl* sm, int lane, cdbl* out, cdbl* lds) {
    constexpr int Q2 = Q * Q, NOUT = 4 * Q2, NO = (NOUT + 63) / 64;
#pragma unroll
    for (int u = 0; u < NO; ++u) {
        const int o = lane + 64 * u;
        if (o >= NOUT) continue;
        const int c = o / Q2, a = o % Q2, a1 = a / Q, a2 = a % Q;
        double e1[2][Q], e2[2][Q];
#pragma unroll
        for (int bb = 0; bb < 2; ++bb)
#pragma unroll
            for (int p = 0; p < Q; ++p) {
                e1[bb][p] = d.E[(bb * Q + p) * Q + a1];
                e2[bb][p] = d.E[(bb * Q + p) * Q + a2];
            }
        cdbl acc = {0.0, 0.0};
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const int b1 = b >> 1, b2 = b & 1;
            const cdbl* m = sm + b * NOUT + c * Q2;
#pragma unroll
            for (int p1 = 0; p1 < Q; ++p1) {
                cdbl t = {0.0, 0.0};
#pragma unroll
                for (int p2 = 0; p2 < Q; ++p2) t = t + m[p1 * Q + p2] * e2[b2][p2];
                acc = acc + t * e1[b1][p1];
            }
        }
        out[o] = acc;
        if (lds) lds[o] = acc;
    }
}

// stages the four children of cluster (f, i, j) at level lev (children at lev + 1) into sm
template <int Q>
__device__ inline void mxh_stage_children(const MxhDev& d, int lev, int64_t f, int i, int j, int lane, cdbl* sm) {
    constexpr int NOUT = 4 * Q * Q;
    const int n = 1 << lev;
    // the four children are consecutive in pairs along j: (2i + b1, 2j), (2i + b1, 2j + 1)
    for (int b1 = 0; b1 < 2; ++b1) {
        const int64_t ch = d.lev_off[lev + 1] + (f * 2 * n + 2 * i + b1) * 2 * n + 2 * j;
        const cdbl* src = (const cdbl*)d.mom + ch * NOUT;
        for (int o = lane; o < 2 * NOUT; o += 64) sm[b1 * 2 * NOUT + o] = src[o];
    }
}

template <int Q>
__global__ __launch_bounds__(256) void k_mxh_up(MxhDev d, int lev) {
    constexpr int NOUT = 4 * Q * Q;
    __shared__ cdbl mc[4][4 * NOUT];  // [wave][child][c][p]
    const int n = 1 << lev;
    const int64_t nc = (int64_t)d.s.geom.npatch * n * n;
    const int w = uniform_int(threadIdx.x >> 6);
    const int64_t loc = (int64_t)blockIdx.x * 4 + w;
    const int lane = threadIdx.x & 63;
    if (loc >= nc) return;
    const int64_t f = loc / ((int64_t)n * n);
    const int i = (int)((loc / n) % n), j = (int)(loc % n);
    mxh_stage_children<Q>(d, lev, f, i, j, lane, mc[w]);
    wave_sync();
    mxh_up_transfer<Q>(d, mc[w], lane, (cdbl*)d.mom + (d.lev_off[lev] + loc) * NOUT, nullptr);
}

// Coupling.  For every stored block (u, v) of a work chunk (consecutive stored blocks of one
// owner u), with entries K[b][a] = G(x_a^u, x_b^v):
//   partial[chunk][c][a] += sum_b K[b][a] mom[v][c][b]   (the owner's expansion)
//   tprod[block][c][b]   = sum_a K[b][a] mom[u][c][a]    (the partner's)
// With q^2 <= 32 (q <= 5): one workgroup per chunk, one wave per block of the chunk.  The
// wave copies its block into its LDS slice with global-to-LDS loads (no registers held, all
// of the workgroup's loads in flight at once) and waits for its own copy only; both passes
// then read LDS, lane (0, i) forming the real and lane (1, i) the imaginary part of node
// i's sum, so that the moments (the partner's in the column pass, the owner's in the row
// pass) are uniform over the wave and enter the products straight from scalar registers.
// The waves' column sums are added in a fixed order.
template <int Q>
__global__ __launch_bounds__(64 * kMxhChunk) void k_mxh_coupling_wg(MxhDev d) {
    constexpr int W = kMxhChunk;  // waves, one block each
    constexpr int Q2 = Q * Q, QQ = Q2 * Q2, NL = W * QQ > 4 * W * Q2 ? W * QQ : 4 * W * Q2;
    static_assert(Q2 <= 32, "a node per lane and half-wave");
    __shared__ cdbl kls[NL];  // block j of the chunk at j q^4, [b][a]; then the waves' column sums
    const int64_t k = blockIdx.x;
    const int w = uniform_int(threadIdx.x >> 6), lane = threadIdx.x & 63, h = lane >> 5, i = lane & 31;
    const mx_ciptr cp0 = (mx_ciptr)d.ch_p0, cp1 = (mx_ciptr)d.ch_p1, cos_ = (mx_ciptr)d.own_s, cot = (mx_ciptr)d.own_t;
    const int p0 = cp0[k], p1 = cp1[k];
    const int pb = p0 + w;  // the wave's block
    const int ic = i < Q2 ? i : 0;  // lanes past the nodes work on node 0; their results are dropped
    // x K + y K' with (x, y) = (re, -im) of the entry for the real part, (im, re) for the
    // imaginary part, and (K, K') = (re, im) of the moment
    const int hx = h, hy = 1 - h;
    const uint64_t neg = h ? 0ull : 0x8000000000000000ull;
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    if (pb < p1) {
        {
            // 16 bytes per lane, 1 KiB per instruction: lane l of the instruction at byte off
            // lands at LDS byte off + 16 l of the wave's slice
            const char* src = (const char*)d.K + (int64_t)pb * QQ * 16;
            char* dst = (char*)(kls + w * QQ);
            for (int off = 0; off < QQ * 16; off += 1024)
                if (off + 16 * lane < QQ * 16)
                    __builtin_amdgcn_global_load_lds((const __attribute__((address_space(1))) void*)(src + off + 16 * lane),
                                                     (__attribute__((address_space(3))) void*)(dst + off), 16, 0, 0);
            __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0): the copy has landed
            wave_sync();
        }
        const double* ks = (const double*)(kls + w * QQ);
        const mx_cdptr mom = (mx_cdptr)d.mom;
        // column pass: lane i takes column i against the partner's moments
        const mx_cdptr mp = mom + (int64_t)cos_[pb] * 8 * Q2;
#pragma unroll 5
        for (int b = 0; b < Q2; ++b) {
            const int e = 2 * (b * Q2 + ic);
            const double x = ks[e + hx];
            const double y = __longlong_as_double(__double_as_longlong(ks[e + hy]) ^ (long long)neg);
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const int o = 2 * (c * Q2 + b);
                acc[c] = fma(x, mp[o], fma(y, mp[o + 1], acc[c]));
            }
        }
        // row pass: lane i takes row i against the owner's moments
        const mx_cdptr mo = mom + (int64_t)cot[p0] * 8 * Q2;
        double tp[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll 5
        for (int a = 0; a < Q2; ++a) {
            const int e = 2 * (ic * Q2 + a);
            const double x = ks[e + hx];
            const double y = __longlong_as_double(__double_as_longlong(ks[e + hy]) ^ (long long)neg);
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const int o = 2 * (c * Q2 + a);
                tp[c] = fma(x, mo[o], fma(y, mo[o + 1], tp[c]));
            }
        }
        if (i < Q2) {
            double* out = (double*)d.tprod + (int64_t)pb * 8 * Q2;
#pragma unroll
            for (int c = 0; c < 4; ++c) out[2 * (c * Q2 + i) + h] = tp[c];
        }
    }
    __syncthreads();  // every wave is done with its block
    if (i < Q2)
#pragma unroll
        for (int c = 0; c < 4; ++c) ((double*)kls)[2 * (w * 4 * Q2 + c * Q2 + i) + h] = acc[c];
    __syncthreads();
    if (threadIdx.x < 4 * Q2) {
        const int o = threadIdx.x;
        cdbl s = kls[o];
#pragma unroll
        for (int v = 1; v < W; ++v) s = s + kls[v * 4 * Q2 + o];
        ((cdbl*)d.partial)[k * 4 * Q2 + o] = s;
    }
}

// The same for q^2 > 32: one wave per work chunk, looping over its blocks; lane b reads row
// b of the block for the transposed product right after the column pass fetched it.
template <int Q>
__global__ __launch_bounds__(256) void k_mxh_coupling(MxhDev d) {
    constexpr int Q2 = Q * Q;
    static_assert(Q2 > 32 && Q2 <= 64, "one block per wave");
    const int64_t k = (int64_t)blockIdx.x * 4 + uniform_int(threadIdx.x >> 6);
    if (k >= d.nchunks) return;
    const int a = threadIdx.x & 63;
    const mx_ciptr cp0 = (mx_ciptr)d.ch_p0, cp1 = (mx_ciptr)d.ch_p1, cos_ = (mx_ciptr)d.own_s, cot = (mx_ciptr)d.own_t;
    const mx_cdptr mom = (mx_cdptr)d.mom;
    const int p0 = cp0[k], p1 = cp1[k];
    // the owner's moments, staged in the wave's LDS slice (read uniformly by the row pass)
    __shared__ cdbl mus[4][4 * Q2];
    const int w = threadIdx.x >> 6;
    {
        const cdbl* mu = (const cdbl*)d.mom + (int64_t)cot[p0] * 4 * Q2;
        for (int o = a; o < 4 * Q2; o += 64) mus[w][o] = mu[o];
        wave_sync();
    }
    const cdbl* __restrict__ Kb = (const cdbl*)d.K;
    cdbl acc[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) acc[c] = cdbl{0.0, 0.0};
    const bool on = a < Q2;
    for (int pp = p0; pp < p1; ++pp) {
        const cdbl* __restrict__ K = Kb + (int64_t)pp * Q2 * Q2;
        const mx_cdptr m0 = mom + (int64_t)cos_[pp] * 8 * Q2;
        // the lane's column of the block, all loads of a slice in flight before the products
        constexpr int KB = 16;
#pragma unroll 1
        for (int b0 = 0; b0 < Q2; b0 += KB) {
            cdbl kcol[KB];
#pragma unroll
            for (int bb = 0; bb < KB; ++bb)
                kcol[bb] = (on && b0 + bb < Q2) ? K[(b0 + bb) * Q2 + a] : cdbl{0.0, 0.0};
#pragma unroll
            for (int bb = 0; bb < KB; ++bb) {
                const int b = b0 + bb;
                if (b >= Q2) break;
                const cdbl kv = kcol[bb];
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    const int o = 2 * (c * Q2 + b);
                    const double mr = m0[o], mi = m0[o + 1];
                    acc[c].re += kv.re * mr - kv.im * mi;
                    acc[c].im += kv.re * mi + kv.im * mr;
                }
            }
        }
        // the transposed product: lane b = a takes row b of the block
        cdbl tp[4];
#pragma unroll
        for (int c = 0; c < 4; ++c) tp[c] = cdbl{0.0, 0.0};
        constexpr int KT = 8;  // row entries in flight
#pragma unroll 1
        for (int a0 = 0; a0 < Q2; a0 += KT) {
            cdbl krow[KT];
#pragma unroll
            for (int aa = 0; aa < KT; ++aa)
                krow[aa] = (on && a0 + aa < Q2) ? K[a * Q2 + a0 + aa] : cdbl{0.0, 0.0};
#pragma unroll
            for (int aa = 0; aa < KT; ++aa) {
                const int ai = a0 + aa;
                if (ai >= Q2) break;
                const cdbl kv = krow[aa];
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    const cdbl mv = mus[w][c * Q2 + ai];
                    tp[c].re += kv.re * mv.re - kv.im * mv.im;
                    tp[c].im += kv.re * mv.im + kv.im * mv.re;
                }
            }
        }
        if (on) {
            cdbl* out = (cdbl*)d.tprod + (int64_t)pp * 4 * Q2;
#pragma unroll
            for (int c = 0; c < 4; ++c) out[c * Q2 + a] = tp[c];
        }
    }
    if (on) {
        cdbl* out = (cdbl*)d.partial + k * 4 * Q2;
#pragma unroll
        for (int c = 0; c < 4; ++c) out[c * Q2 + a] = acc[c];
    }
}

// Local expansions, first part: lv[cl][c] = the sum of the cluster's chunk partials and of
// the transposed products of the blocks in which it is the partner, for the clusters of
// every level at once.  One workgroup per cluster, lanes over (c, a): the rows (partials in
// chunk order, then the transposed products in block order) are dealt to the four waves in
// turn, each wave keeps four running sums (row t to sum (t / 4) mod 4, the rows past the
// last full group of sixteen to the first), and the sums are added pairwise, then the waves'
// in wave order.
template <int NO>
__global__ __launch_bounds__(256) void k_mxh_collect(MxhDev d) {
    __shared__ cdbl red[4][64 * NO];
    const int64_t cl = blockIdx.x;
    const int w = uniform_int(threadIdx.x >> 6), lane = threadIdx.x & 63;
    const int nout = 4 * d.q2;
    const cdbl* part = (const cdbl*)d.partial;
    const cdbl* tp = (const cdbl*)d.tprod;
    const mx_ciptr tb = (mx_ciptr)d.tr_blk;
    const int64_t k0 = d.cl_chunk[cl], nk = d.cl_chunk[cl + 1] - k0;
    const int64_t e0 = d.tr_ptr[cl], ni = nk + d.tr_ptr[cl + 1] - e0;
    // lanes past the outputs read output 0 (loads without branches); their sums are not used
    bool on[NO];
    int oc[NO];
#pragma unroll
    for (int u = 0; u < NO; ++u) {
        on[u] = lane + 64 * u < nout;
        oc[u] = on[u] ? lane + 64 * u : 0;
    }
    cdbl a4[4][NO];
#pragma unroll
    for (int v = 0; v < 4; ++v)
#pragma unroll
        for (int u = 0; u < NO; ++u) a4[v][u] = cdbl{0.0, 0.0};
    int64_t t = w;
    for (; t + 12 < ni; t += 16) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int64_t r = t + 4 * v;
            const cdbl* row = r < nk ? part + (k0 + r) * nout : tp + (int64_t)tb[e0 + r - nk] * nout;
#pragma unroll
            for (int u = 0; u < NO; ++u) a4[v][u] = a4[v][u] + row[oc[u]];
        }
    }
    for (; t < ni; t += 4) {
        const cdbl* row = t < nk ? part + (k0 + t) * nout : tp + (int64_t)tb[e0 + t - nk] * nout;
#pragma unroll
        for (int u = 0; u < NO; ++u) a4[0][u] = a4[0][u] + row[oc[u]];
    }
#pragma unroll
    for (int u = 0; u < NO; ++u) red[w][lane + 64 * u] = (a4[0][u] + a4[1][u]) + (a4[2][u] + a4[3][u]);
    __syncthreads();
    if (w == 0) {
        cdbl* lc = (cdbl*)d.lv + cl * nout;
#pragma unroll
        for (int u = 0; u < NO; ++u) {
            const int o = lane + 64 * u;
            if (on[u]) lc[o] = (red[0][o] + red[1][o]) + (red[2][o] + red[3][o]);
        }
    }
}

// Local expansions, second part, at level lev >= 1, top down: lv[cl][c][p] += sum_a
// E_b1[p1][a1] E_b2[p2][a2] lv[parent][c][a].  One wave per cluster, lanes over (c, p); the
// parent's expansion is staged in the wave's LDS slice, the transfer entries of the lane's
// node are held in registers.  ps: the parent's expansion [c][a]; the result also goes to
// lds when given.
template <int Q>
__device__ inline void mxh_down_transfer(const MxhDev& d, const cdbl* ps, int b1, int b2, int lane, cdbl* lc,
                                         cdbl* lds) {
    constexpr int Q2 = Q * Q, NOUT = 4 * Q2, NO = (NOUT + 63) / 64;
#pragma unroll
    for (int u = 0; u < NO; ++u) {
        const int o = lane + 64 * u;
        if (o >= NOUT) continue;
        const int c = o / Q2, p = o % Q2, p1 = p / Q, p2 = p % Q;
        double e1[Q], e2[Q];
#pragma unroll
        for (int a = 0; a < Q; ++a) {
            e1[a] = d.E[(b1 * Q + p1) * Q + a];
            e2[a] = d.E[(b2 * Q + p2) * Q + a];
        }
        cdbl s = lc[o];
#pragma unroll
        for (int a1 = 0; a1 < Q; ++a1) {
            cdbl t = {0.0, 0.0};
#pragma unroll
            for (int a2 = 0; a2 < Q; ++a2) t = t + ps[c * Q2 + a1 * Q + a2] * e2[a2];
            s = s + t * e1[a1];
        }
        lc[o] = s;
        if (lds) lds[o] = s;
    }
}

template <int Q>
__global__ __launch_bounds__(256) void k_mxh_down(MxhDev d, int lev) {
    constexpr int NOUT = 4 * Q * Q;
    const int n = 1 << lev, hh = n / 2;
    const int64_t nc = (int64_t)d.s.geom.npatch * n * n;
    const int w = uniform_int(threadIdx.x >> 6);
    const int64_t loc = (int64_t)blockIdx.x * 4 + w;
    const int lane = threadIdx.x & 63;
    if (loc >= nc) return;
    const int f = (int)(loc / ((int64_t)n * n)), i = (int)((loc / n) % n), j = (int)(loc % n);
    __shared__ cdbl ps[4][NOUT];  // [wave][c][a]: the parent's expansion
    const cdbl* src = (const cdbl*)d.lv + (d.lev_off[lev - 1] + ((int64_t)f * hh + i / 2) * hh + j / 2) * NOUT;
    for (int o = lane; o < NOUT; o += 64) ps[w][o] = src[o];
    wave_sync();
    mxh_down_transfer<Q>(d, ps[w], i & 1, j & 1, lane, (cdbl*)d.lv + (d.lev_off[lev] + loc) * NOUT, nullptr);
}

// Two levels in one launch: one workgroup per cluster at level lev >= 1; wave 0 adds the
// parent's transfer to the cluster's expansion (kept in LDS), then wave w adds the cluster's
// transfer to child w (level lev + 1).
template <int Q>
__global__ __launch_bounds__(256) void k_mxh_down2(MxhDev d, int lev) {
    constexpr int NOUT = 4 * Q * Q;
    const int n = 1 << lev, hh = n / 2;
    const int64_t loc = blockIdx.x;
    const int w = uniform_int(threadIdx.x >> 6), lane = threadIdx.x & 63;
    const int64_t f = loc / ((int64_t)n * n);
    const int i = (int)((loc / n) % n), j = (int)(loc % n);
    __shared__ cdbl ps[NOUT];   // the parent's expansion
    __shared__ cdbl own[NOUT];  // the cluster's
    if (w == 0) {
        const cdbl* src = (const cdbl*)d.lv + (d.lev_off[lev - 1] + (f * hh + i / 2) * hh + j / 2) * NOUT;
        for (int o = lane; o < NOUT; o += 64) ps[o] = src[o];
        wave_sync();
        mxh_down_transfer<Q>(d, ps, i & 1, j & 1, lane, (cdbl*)d.lv + (d.lev_off[lev] + loc) * NOUT, own);
    }
    __syncthreads();
    const int ci = 2 * i + (w >> 1), cj = 2 * j + (w & 1);  // child w at level lev + 1
    const int64_t ch = d.lev_off[lev + 1] + (f * 2 * n + ci) * 2 * n + cj;
    mxh_down_transfer<Q>(d, own, w >> 1, w & 1, lane, (cdbl*)d.lv + ch * NOUT, nullptr);
}

// y[g] = sum over the pieces (e, k, s) of g of s sum_c w_c sum_a Mt[e][k][c][a] lv[leaf(e)][c][a]
// (the backward transform of the far field, w = 1, 1, 1, -kappa^-2) + sum_h M[g][h] x[h] (the
// glued near field).  One wave per global function: lanes over the (c, a) terms of each piece,
// then over the row's entries (four at a time in flight), then a wave sum.
__global__ __launch_bounds__(256) void k_mxh_scatter(MxhDev d, const cdbl* __restrict__ x, cdbl* __restrict__ y) {
    const int64_t g = (int64_t)blockIdx.x * 4 + uniform_int(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (g >= d.s.nglob) return;
    const int nl = d.s.nl, n = d.s.nel, m = d.m, q2 = d.q2, nout = 4 * q2;
    const KernelDesc& kd = d.s.ker;
    const double k2r = kd.kre * kd.kre - kd.kim * kd.kim, k2i = 2.0 * kd.kre * kd.kim;
    const double den = k2r * k2r + k2i * k2i;
    const cdbl mik2 = {-k2r / den, k2i / den};
    const cdbl* lvb = (const cdbl*)d.lv + d.lev_off[d.leaf] * nout;
    cdbl s = {0.0, 0.0};
    for (int64_t t = d.s.gptr[g]; t < d.s.gptr[g + 1]; ++t) {  // uniform over the wave
        const int p = d.s.gpos[t];
        const int64_t e = p / nl;
        const int i1 = (int)((e / n) % n), i2 = (int)(e % n);
        const int64_t l = ((e / ((int64_t)n * n)) * d.nleaf1 + i1 / m) * d.nleaf1 + i2 / m;
        const double* mt = d.Mt + (int64_t)p * nout;
        const cdbl* lv = lvb + l * nout;
        const double sg = (double)d.s.gsgn[t];
        for (int o = lane; o < nout; o += 64) {
            const cdbl v = lv[o];
            s = s + (o >= 3 * q2 ? cmul(mik2, v) : v) * (mt[o] * sg);
        }
    }
    const cdbl* val = (const cdbl*)d.nval;
    const int64_t r0 = d.nrowptr[g], r1 = d.nrowptr[g + 1];
#pragma unroll 4
    for (int64_t r = r0 + lane; r < r1; r += 64) s = s + val[r] * x[d.ncol[r]];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        s.re += __shfl_xor(s.re, o, 64);
        s.im += __shfl_xor(s.im, o, 64);
    }
    if (lane == 0) y[g] = s;
}

// Glued near field: M[g][h] = sum over the pieces (e1, k1, s1) of g and (e2, k2, s2) of h whose
// elements lie in a near leaf pair of s1 s2 B[pair][k1][k2]; one thread per stored entry,
// its row found by bisection of the row pointers.
__global__ __launch_bounds__(256) void k_mxh_near_glue(MxhDev d) {
    const int64_t id = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (id >= d.nnzg) return;
    int64_t lo = 0, hi = d.s.nglob;  // nrowptr[lo] <= id < nrowptr[hi]
    while (hi - lo > 1) {
        const int64_t mid = (lo + hi) / 2;
        if (d.nrowptr[mid] <= id) lo = mid;
        else hi = mid;
    }
    const int64_t g = lo, h = d.ncol[id];
    const int nl = d.s.nl, n = d.s.nel, m = d.m, m2 = m * m;
    const cdbl* B = (const cdbl*)d.s.B;
    cdbl acc = {0.0, 0.0};
    for (int64_t t1 = d.s.gptr[g]; t1 < d.s.gptr[g + 1]; ++t1) {
        const int p1 = d.s.gpos[t1], k1 = p1 % nl;
        const int64_t e1 = p1 / nl;
        const int i1 = (int)((e1 / n) % n), j1 = (int)(e1 % n);
        const int64_t l1 = ((e1 / ((int64_t)n * n)) * d.nleaf1 + i1 / m) * d.nleaf1 + j1 / m;
        const int u1 = (i1 % m) * m + j1 % m;
        for (int64_t t2 = d.s.gptr[h]; t2 < d.s.gptr[h + 1]; ++t2) {
            const int p2 = d.s.gpos[t2], k2 = p2 % nl;
            const int64_t e2 = p2 / nl;
            const int i2 = (int)((e2 / n) % n), j2 = (int)(e2 % n);
            const int64_t l2 = ((e2 / ((int64_t)n * n)) * d.nleaf1 + i2 / m) * d.nleaf1 + j2 / m;
            const int v2 = (i2 % m) * m + j2 % m;
            for (int64_t lp = d.near_rowptr[l1]; lp < d.near_rowptr[l1 + 1]; ++lp)
                if (d.near_s[lp] == l2) {
                    const cdbl b = B[((lp * m2 + u1) * m2 + v2) * (int64_t)(nl * nl) + k1 * nl + k2];
                    acc = acc + b * (double)(d.s.gsgn[t1] * d.s.gsgn[t2]);
                    break;
                }
        }
    }
    ((cdbl*)d.nval)[id] = acc;
}

inline unsigned nb(int64_t n, int per) { return (unsigned)((n + per - 1) / per); }

template <int P>
constexpr size_t mx_regular_lds() {
    constexpr int NC = 4 * 2 * P * (P + 1);
    return sizeof(double) * (size_t)(64 * NC * 3);
}

template <int P>
hipError_t mx_pairs_p(const MxDev& d, hipStream_t st) {
    constexpr size_t lds = mx_regular_lds<P>();
    if (lds > 64 * 1024) {
        const hipError_t e = hipFuncSetAttribute((const void*)k_mx_regular<P>,
                                                 hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    if (d.nreg > 0) hipLaunchKernelGGL(k_mx_regular<P>, dim3((unsigned)d.nreg), dim3(64), lds, st, d);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int64_t nt = d.npairs - d.nreg;
    if (nt > 0) hipLaunchKernelGGL(k_mx_touch<P>, dim3((unsigned)nt), dim3(64), 0, st, d);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_mx_pairs(const MxDev& d, hipStream_t st) {
    if (d.npairs == 0) return hipSuccess;
    if (d.p == 1) return mx_pairs_p<1>(d, st);
    if (d.p == 2) return mx_pairs_p<2>(d, st);
    return hipErrorInvalidValue;
}

hipError_t launch_mx_gather(const MxDev& d, hipStream_t st) {
    if (d.nglob == 0) return hipSuccess;
    hipLaunchKernelGGL(k_mx_gather, dim3(nb(d.nglob * d.nglob, 256)), dim3(256), 0, st, d);
    return hipGetLastError();
}

hipError_t launch_mx_matvec(const MxDev& d, const void* x, void* y, hipStream_t st) {
    if (d.nglob == 0) return hipSuccess;
    hipLaunchKernelGGL(k_mx_matvec, dim3(nb(d.nglob, 4)), dim3(256), 0, st, d, (const cdbl*)x, (cdbl*)y);
    return hipGetLastError();
}

hipError_t launch_mx_rhs(const MxDev& d, const Gauss8& g8, int kind, const double* q, void* b, hipStream_t st) {
    if (d.nglob == 0) return hipSuccess;
    const dim3 g(nb(d.nglob, 4)), blk(256);
    if (d.p == 1)
        hipLaunchKernelGGL(k_mx_rhs<1>, g, blk, 0, st, d, g8, kind, q[0], q[1], q[2], q[3], q[4], q[5], (cdbl*)b);
    else if (d.p == 2)
        hipLaunchKernelGGL(k_mx_rhs<2>, g, blk, 0, st, d, g8, kind, q[0], q[1], q[2], q[3], q[4], q[5], (cdbl*)b);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_mx_field(const MxDev& d, const Gauss8& g8, const double* pts, int64_t npts, const void* j, void* E,
                           hipStream_t st) {
    if (npts == 0) return hipSuccess;
    if (d.p == 1)
        hipLaunchKernelGGL(k_mx_field<1>, dim3((unsigned)npts), dim3(256), 0, st, d, g8, pts, (const cdbl*)j, (cdbl*)E);
    else if (d.p == 2)
        hipLaunchKernelGGL(k_mx_field<2>, dim3((unsigned)npts), dim3(256), 0, st, d, g8, pts, (const cdbl*)j, (cdbl*)E);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_mxh_assemble(const MxhDev& d, hipStream_t st) {
    if (d.ncl * d.q2 > 0) hipLaunchKernelGGL(k_mxh_points, dim3(nb(d.ncl * d.q2, 256)), dim3(256), 0, st, d);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int64_t nk = d.nstored * d.q2 * d.q2;
    if (nk > 0) hipLaunchKernelGGL(k_mxh_far, dim3(nb(nk, 256)), dim3(256), 0, st, d);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (d.s.nelem > 0) {
        if (d.s.p == 1)
            hipLaunchKernelGGL(k_mxh_moments<1>, dim3((unsigned)d.s.nelem), dim3(64), 0, st, d);
        else if (d.s.p == 2)
            hipLaunchKernelGGL(k_mxh_moments<2>, dim3((unsigned)d.s.nelem), dim3(64), 0, st, d);
        else
            return hipErrorInvalidValue;
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    if ((e = launch_mx_pairs(d.s, st)) != hipSuccess) return e;
    if (d.nnzg > 0) hipLaunchKernelGGL(k_mxh_near_glue, dim3(nb(d.nnzg, 256)), dim3(256), 0, st, d);
    return hipGetLastError();
}

template <int Q>
static hipError_t mxh_apply_q(const MxhDev& d, const void* x, void* y, hipStream_t st) {
    constexpr int NO = (4 * Q * Q + 63) / 64;
    const dim3 gf(d.m == 1 ? nb(d.nleaves, 4) : d.nleaves);
    if (d.s.p == 1)
        hipLaunchKernelGGL((k_mxh_forward<1, NO>), gf, dim3(256), 0, st, d, (const cdbl*)x);
    else
        hipLaunchKernelGGL((k_mxh_forward<2, NO>), gf, dim3(256), 0, st, d, (const cdbl*)x);
    for (int lev = d.leaf - 1; lev >= 0; --lev) {
        const int64_t nc = (int64_t)d.s.geom.npatch << (2 * lev);
        hipLaunchKernelGGL(k_mxh_up<Q>, dim3(nb(nc, 4)), dim3(256), 0, st, d, lev);
    }
    if (d.nchunks > 0) {
        if constexpr (Q * Q <= 32)
            hipLaunchKernelGGL(k_mxh_coupling_wg<Q>, dim3(d.nchunks), dim3(64 * kMxhChunk), 0, st, d);
        else
            hipLaunchKernelGGL(k_mxh_coupling<Q>, dim3(nb(d.nchunks, 4)), dim3(256), 0, st, d);
    }
    hipLaunchKernelGGL(k_mxh_collect<NO>, dim3(d.ncl), dim3(256), 0, st, d);
    {
        // levels 1 .. leaf, two per launch where they pair up
        int lev = 1;
        for (; lev + 1 <= d.leaf; lev += 2) {
            const int64_t nc = (int64_t)d.s.geom.npatch << (2 * lev);
            hipLaunchKernelGGL(k_mxh_down2<Q>, dim3((unsigned)nc), dim3(256), 0, st, d, lev);
        }
        if (lev == d.leaf) {
            const int64_t nc = (int64_t)d.s.geom.npatch << (2 * lev);
            hipLaunchKernelGGL(k_mxh_down<Q>, dim3(nb(nc, 4)), dim3(256), 0, st, d, lev);
        }
    }
    hipLaunchKernelGGL(k_mxh_scatter, dim3(nb(d.s.nglob, 4)), dim3(256), 0, st, d, (const cdbl*)x, (cdbl*)y);
    return hipGetLastError();
}

hipError_t launch_mxh_apply(const MxhDev& d, const void* x, void* y, hipStream_t st) {
    if (d.s.nglob == 0) return hipSuccess;
    if (d.s.p != 1 && d.s.p != 2) return hipErrorInvalidValue;
    switch (d.q) {
        case 1: return mxh_apply_q<1>(d, x, y, st);
        case 2: return mxh_apply_q<2>(d, x, y, st);
        case 3: return mxh_apply_q<3>(d, x, y, st);
        case 4: return mxh_apply_q<4>(d, x, y, st);
        case 5: return mxh_apply_q<5>(d, x, y, st);
        case 6: return mxh_apply_q<6>(d, x, y, st);
        case 7: return mxh_apply_q<7>(d, x, y, st);
        case 8: return mxh_apply_q<8>(d, x, y, st);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace bem
