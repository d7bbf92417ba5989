// gfx950 kernels of the isogeometric Galerkin BEM hot path: near-field quadrature, coupling
// blocks, the H^2 matvec, load vector, potential and the GMRES vector operations.
#include "bem_kernels.h"
#include "bem_device.h"

#include <type_traits>

namespace bem {

namespace {

constexpr int kGroupRowsDev = 16;  // rows per near-field row group at most (host: kGroupRows)

__device__ inline double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
    return v;
}
__device__ inline cdbl wave_sum(cdbl v) { return {wave_sum(v.re), wave_sum(v.im)}; }

__device__ inline double shfl_xor_t(double v, int off) { return __shfl_xor(v, off, kWave); }
__device__ inline cdbl shfl_xor_t(cdbl v, int off) { return {__shfl_xor(v.re, off, kWave), __shfl_xor(v.im, off, kWave)}; }
__device__ inline float shfl_xor_t(float v, int off) { return __shfl_xor(v, off, kWave); }
__device__ inline cflt shfl_xor_t(cflt v, int off) { return {__shfl_xor(v.re, off, kWave), __shfl_xor(v.im, off, kWave)}; }
__device__ inline double shfl_t(double v, int src) { return __shfl(v, src, kWave); }
__device__ inline cdbl shfl_t(cdbl v, int src) { return {__shfl(v.re, src, kWave), __shfl(v.im, src, kWave)}; }

// leaf-local index -> (patch, i, j)
__device__ inline void leaf_decode(int l, int n1, int& f, int& i, int& j) {
    j = l % n1;
    i = (l / n1) % n1;
    f = l / (n1 * n1);
}


// ------------------------------------------------------------------ geometry tables
__global__ void k_gauss_points(SpaceDesc S, int qg, const double* __restrict__ gx, double* __restrict__ gpos,
                               double* __restrict__ gkap) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int qg2 = qg * qg;
    if (idx >= S.nelem * qg2) return;
    const int a = (int)(idx % qg2);
    const int64_t e = idx / qg2;
    const int i2 = (int)(e % S.nel), i1 = (int)((e / S.nel) % S.nel), f = (int)(e / ((int64_t)S.nel * S.nel));
    const double ps = (i1 + gx[a / qg]) * S.h, pt = (i2 + gx[a % qg]) * S.h;
    double x[3];
    patch_point(S.geom, f, ps, pt, x);
    gpos[3 * idx] = x[0];
    gpos[3 * idx + 1] = x[1];
    gpos[3 * idx + 2] = x[2];
    if (gkap) gkap[idx] = patch_kappa(S.geom, f, ps, pt);  // 0-form lifting only
}

// 1/r for NS values r^2 > 0 (finite).  From the hardware estimate y (relative error
// about 5e-8), e = 1 - r^2 y^2 and the series (1 - e)^(-1/2) = 1 + e/2 + 3e^2/8 + ...
// give y (1 + e/2 + 3e^2/8), whose truncation error (5e^3/16) lies far below FP64
// rounding; the NS chains are interleaved step by step.
template <int NS>
__device__ inline void rinv_nr(const double* r2, double* y) {
#pragma unroll
    for (int u = 0; u < NS; ++u) y[u] = __builtin_amdgcn_rsq(r2[u]);
#pragma unroll
    for (int u = 0; u < NS; ++u) {
        const double e = __builtin_fma(-(r2[u] * y[u]), y[u], 1.0);
        const double c = __builtin_fma(e, 0.375, 0.5);
        y[u] = __builtin_fma(y[u] * e, c, y[u]);
    }
}

// The single-layer kernel without its factor 1/(4 pi), for the near-field quadrature: 1/r
// by rinv_nr (Laplace); exp(-i kappa r)/r with the library's sine, cosine and exponential
// (Helmholtz: near pairs put no bound on kappa r).
__device__ inline double near_kernel(const KernelDesc&, double r2, double) {
    double y;
    rinv_nr<1>(&r2, &y);
    return y;
}
__device__ inline cdbl near_kernel(const KernelDesc& k, double r2, cdbl) {
    double ir;
    rinv_nr<1>(&r2, &ir);
    const double r = r2 * ir;
    double s, c;
    sincos(k.kre * r, &s, &c);
    const double mag = k.kim != 0.0 ? ir * exp(k.kim * r) : ir;
    return {mag * c, -mag * s};
}

// Read-only tables addressed through the constant address space: loads at wave-uniform
// addresses become scalar loads (the tables are not written while a kernel reads them).
typedef const __attribute__((address_space(4))) double* cdptr;
__device__ inline cdptr as_const(const double* p) { return (cdptr)p; }

typedef double f64x4n __attribute__((ext_vector_type(4)));

// ------------------------------------------------------------------ near field: regular pairs
// One workgroup per near leaf pair (tau, sigma).  Wave w takes the tau-elements w, w+W, ...
// and integrates each against every sigma-element that does not touch it.  Lane a holds
// Gauss point a of the tau-element (64 points per pass); the sigma-element's points and
// weighted basis values are wave-uniform and come through scalar loads.  Per lane the inner
// integral over sigma is accumulated in tensor form (first over b2, then b1):
// T[a][j] = sum_b k(x_a, y_b) w_b phi_j(y_b).  The outer sum over tau's points,
// B[k][j] = sum_a w_a phi_k(x_a) T[a][j], runs on the matrix cores (v_mfma_f64_16x16x4f64,
// the pass's 64 points in 16 steps of 4): lane l holds the weight of point 4 s + l / 16 for
// basis l % 16 (built once per tau-element and pass) and reads T of that point from LDS.
// Element-pair blocks are accumulated into the wave's own copy of the leaf-pair block
// (DOFs of tau x DOFs of sigma), the copies summed in a fixed order.
// QG: the Gauss points per direction when fixed at compile time (0: op.qg); K0: 0-form lifting.
template <class T, int D, int QG, bool K0>
__global__ __launch_bounds__(256) void k_near_regular(OpDev op, AsmDev as, int W, int lb_in_lds) {
    constexpr int D1 = D + 1, NB = D1 * D1;
    static_assert(NB <= 16, "element blocks of at most 16 x 16");
    constexpr bool kCplx = std::is_same<T, cdbl>::value;
    const SpaceDesc S = op.S;
    const int qg = QG > 0 ? QG : op.qg, qg2 = qg * qg, m = op.m, m2 = m * m, nloc = op.nloc, nl2 = nloc * nloc;
    const int64_t blk = (int64_t)nl2 * nl2;
    const int64_t lp = blockIdx.x;
    int tf, ti, tj, sf, si, sj;
    leaf_decode(as.near_t[lp], op.nleaf1, tf, ti, tj);
    leaf_decode(as.near_s[lp], op.nleaf1, sf, si, sj);
    extern __shared__ double smem[];
    T* out = (T*)as.lb + lp * blk;
    T* LB = lb_in_lds ? (T*)smem : out;
    T* TB = (T*)smem + (lb_in_lds ? (int64_t)W * blk : 0);
    const int wave = uniform_int(threadIdx.x >> 6), lane = threadIdx.x & 63;
    T* myLB = LB + (lb_in_lds ? wave * blk : 0);
    T* myTB = TB + wave * kWave * NB;
    const int64_t nzero = lb_in_lds ? W * blk : blk;
    for (int64_t i = threadIdx.x; i < nzero; i += blockDim.x) LB[i] = zero<T>();
    __syncthreads();
    const KernelDesc kd = S.ker;
    const double h2 = S.h * S.h, scale = kInv4Pi * h2 * h2;
    const cdptr gpos = as_const(as.gpos), psiw = as_const(as.psiw);
    const cdptr gkap = K0 ? as_const(as.gkap) : nullptr;  // 0-form lifting: kappa at the points
    const int kq = lane & 15, aq = lane >> 4;                 // matrix-core operand roles of this lane
    for (int et = wave; et < m2; et += W) {
        const int ei1 = ti * m + et / m, ei2 = tj * m + et % m;
        const int64_t e = elem_id(S, tf, ei1, ei2);
        const int v0 = as.vid[4 * e], v1 = as.vid[4 * e + 1], v2 = as.vid[4 * e + 2], v3 = as.vid[4 * e + 3];
        for (int chunk = 0; chunk < qg2; chunk += kWave) {
            const int a = chunk + lane;
            const bool valid = a < qg2;
            double xa0 = 0.0, xa1 = 0.0, xa2 = 0.0;
            if (valid) {
                const double* xp = as.gpos + (e * qg2 + a) * 3;
                xa0 = xp[0];
                xa1 = xp[1];
                xa2 = xp[2];
            }
            // first operand: w_a phi_k(x_a) for point a = chunk + 4 s + aq and basis k = kq
            double wA[16];
#pragma unroll
            for (int st = 0; st < 16; ++st) {
                const int ap = chunk + 4 * st + aq;
                double w = 0.0;
                if (ap < qg2 && kq < NB) {
                    w = as.psiw[((int64_t)ei1 * qg + ap / qg) * D1 + kq / D1] *
                        as.psiw[((int64_t)ei2 * qg + ap % qg) * D1 + kq % D1];
                    if (K0) w *= as.gkap[e * qg2 + ap];
                }
                wA[st] = w;
            }
            for (int es = 0; es < m2; ++es) {
                const int fi1 = si * m + es / m, fi2 = sj * m + es % m;
                const int64_t e2 = elem_id(S, sf, fi1, fi2);
                const int* w2 = as.vid + 4 * e2;
                bool touch = false;
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    const int vv = w2[c];
                    touch |= (vv == v0) | (vv == v1) | (vv == v2) | (vv == v3);
                }
                if (touch) continue;
                T acc[NB];
#pragma unroll
                for (int j = 0; j < NB; ++j) acc[j] = zero<T>();
                const cdptr yp = gpos + e2 * qg2 * 3;
                const cdptr p1 = psiw + (int64_t)fi1 * qg * D1;
                const cdptr p2 = psiw + (int64_t)fi2 * qg * D1;
                const cdptr yk = K0 ? gkap + e2 * qg2 : nullptr;
                for (int b1 = 0; b1 < qg; ++b1) {
                    T sacc[D1];
#pragma unroll
                    for (int l = 0; l < D1; ++l) sacc[l] = zero<T>();
#pragma unroll 8
                    for (int b2 = 0; b2 < qg; ++b2) {
                        const cdptr y = yp + (b1 * qg + b2) * 3;
                        const double dx = xa0 - y[0], dy = xa1 - y[1], dz = xa2 - y[2];
                        T kv = near_kernel(kd, dx * dx + dy * dy + dz * dz, T());
                        if (K0) kv = kv * yk[b1 * qg + b2];
#pragma unroll
                        for (int l = 0; l < D1; ++l) sacc[l] += kv * p2[b2 * D1 + l];
                    }
#pragma unroll
                    for (int l1 = 0; l1 < D1; ++l1) {
                        const double c1 = p1[b1 * D1 + l1];
#pragma unroll
                        for (int l2 = 0; l2 < D1; ++l2) acc[l1 * D1 + l2] += c1 * sacc[l2];
                    }
                }
#pragma unroll
                for (int j = 0; j < NB; ++j) myTB[lane * NB + j] = valid ? acc[j] : zero<T>();
                wave_sync();
                // B = sum over the pass's points of w_a phi_k(x_a) T[a][j]; lane l, entry u of
                // the result: tau basis aq + 4 u, sigma basis kq
                f64x4n cre = {0.0, 0.0, 0.0, 0.0}, cim = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
                for (int st = 0; st < 16; ++st) {
                    const T tb = kq < NB ? myTB[(4 * st + aq) * NB + kq] : zero<T>();
                    if constexpr (kCplx) {
                        cre = __builtin_amdgcn_mfma_f64_16x16x4f64(wA[st], tb.re, cre, 0, 0, 0);
                        cim = __builtin_amdgcn_mfma_f64_16x16x4f64(wA[st], tb.im, cim, 0, 0, 0);
                    } else {
                        cre = __builtin_amdgcn_mfma_f64_16x16x4f64(wA[st], tb, cre, 0, 0, 0);
                    }
                }
                if (kq < NB) {
                    const int c1 = (es / m) * S.r + kq / D1, c2 = (es % m) * S.r + kq % D1;
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        const int kk = aq + 4 * u;
                        if (kk >= NB) continue;
                        const int r1 = (et / m) * S.r + kk / D1, r2 = (et % m) * S.r + kk % D1;
                        T v;
                        if constexpr (kCplx) v = cdbl{cre[u] * scale, cim[u] * scale};
                        else v = cre[u] * scale;
                        myLB[(int64_t)(r1 * nloc + r2) * nl2 + c1 * nloc + c2] += v;
                    }
                }
                wave_sync();
            }
        }
    }
    __syncthreads();
    if (lb_in_lds) {
        for (int64_t i = threadIdx.x; i < blk; i += blockDim.x) {
            T v = LB[i];
            for (int w = 1; w < W; ++w) v += LB[w * blk + i];
            out[i] = v;
        }
    }
}

// ------------------------------------------------------------------ near field: touching pairs
// gamma_f(s, t) with the geometry kind fixed at compile time (GK < 0: any kind).  Sphere and
// ellipsoid: the radial projection of the cube face with 1/|c| from rinv_nr.
template <int GK>
__device__ inline void patch_point_k(const GeomDesc& g, int f, double s, double t, double* x) {
    if constexpr (GK == GEOM_SPHERE6 || GK == GEOM_ELLIPSOID6) {
        int iu, iv, ic;
        double cv;
        cube_face_layout(f, iu, iv, ic, cv);
        double c[3];
        c[iu] = 2.0 * s - 1.0;
        c[iv] = 2.0 * t - 1.0;
        c[ic] = cv;
        double inv;
        const double n2 = c[0] * c[0] + c[1] * c[1] + c[2] * c[2];
        rinv_nr<1>(&n2, &inv);
        if constexpr (GK == GEOM_SPHERE6) {
            x[0] = c[0] * inv;
            x[1] = c[1] * inv;
            x[2] = c[2] * inv;
        } else {
            x[0] = g.a * (c[0] * inv);
            x[1] = g.b * (c[1] * inv);
            x[2] = g.c * (c[2] * inv);
        }
    } else if constexpr (GK >= 0) {
        GeomDesc h = g;
        h.kind = GK;  // the other branches of patch_point fold away
        patch_point(h, f, s, t, x);
    } else {
        patch_point(g, f, s, t, x);
    }
}

// One workgroup per touching element pair (identical, common edge or common vertex).  The
// pair's Duffy cube points are (xi, e1, e2, e3) per region; thread t takes the (e1, e2, e3)
// combinations t, t + 256, ... of the qs^3 and, for each, every region and every xi, so the
// region and xi are wave-uniform and no point index is divided.  The element block is
// reduced over the workgroup and written to the pair's slot in sblk (ROWS rows of the block
// per pass, to bound registers); k_near_singular_add adds the slots of each leaf pair to its
// leaf-pair block in a fixed order.
template <class T, int D, int ROWS, int FORM, int GK>
__global__ __launch_bounds__(256) void k_near_singular(OpDev op, AsmDev as) {
    constexpr int D1 = D + 1, NB = D1 * D1;
    __shared__ T red[4][ROWS * NB];
    const SpaceDesc S = op.S;
    const BasisTab& bt = op.bt;
    const int m = op.m, qs = op.qs, qs3 = qs * qs * qs;
    const int64_t tp = blockIdx.x;
    // the leaf pair of tp: the last lp with touch_rowptr[lp] <= tp
    int lo = 0, hi = (int)op.nnear;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (as.touch_rowptr[mid] <= tp) lo = mid;
        else hi = mid;
    }
    int tf, ti, tj, sf, si, sj;
    leaf_decode(as.near_t[lo], op.nleaf1, tf, ti, tj);
    leaf_decode(as.near_s[lo], op.nleaf1, sf, si, sj);
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const KernelDesc kd = S.ker;
    const double h2 = S.h * S.h, h4 = h2 * h2;
    const int et = as.touch[5 * tp], es = as.touch[5 * tp + 1], type = as.touch[5 * tp + 2];
    const int k1 = as.touch[5 * tp + 3], k2 = as.touch[5 * tp + 4];
    const int ei1 = ti * m + et / m, ei2 = tj * m + et % m;
    const int fi1 = si * m + es / m, fi2 = sj * m + es % m;
    const int c1a = basis_class(bt, ei1), c1b = basis_class(bt, ei2);
    const int c2a = basis_class(bt, fi1), c2b = basis_class(bt, fi2);
    const int nreg = type == PT_IDENTICAL ? 8 : (type == PT_EDGE ? 6 : 4);
    const cdptr sx = as_const(as.sx), sw = as_const(as.sw);
    T* sb = (T*)as.sblk + tp * NB * NB;
#pragma unroll
    for (int r0 = 0; r0 < NB; r0 += ROWS) {
        T acc[ROWS * NB];
#pragma unroll
        for (int v = 0; v < ROWS * NB; ++v) acc[v] = zero<T>();
        for (int c = threadIdx.x; c < qs3; c += blockDim.x) {
            const int i3 = c % qs, i2 = (c / qs) % qs, i1 = c / (qs * qs);
            const double e1 = as.sx[i1], e2 = as.sx[i2], e3 = as.sx[i3];
            const double w123 = as.sw[i1] * as.sw[i2] * as.sw[i3] * h4;
            for (int reg = 0; reg < nreg; ++reg)
                for (int i0 = 0; i0 < qs; ++i0) {
                    double xh1, xh2, yh1, yh2, jac;
                    duffy_point(type, reg, sx[i0], e1, e2, e3, xh1, xh2, yh1, yh2, jac);
                    double wq = sw[i0] * w123 * jac;
                    double u1, u2, w1, w2, X[3], Y[3];
                    d4_apply(k1, xh1, xh2, u1, u2);
                    d4_apply(k2, yh1, yh2, w1, w2);
                    patch_point_k<GK>(S.geom, tf, (ei1 + u1) * S.h, (ei2 + u2) * S.h, X);
                    patch_point_k<GK>(S.geom, sf, (fi1 + w1) * S.h, (fi2 + w2) * S.h, Y);
                    if (FORM == 0)  // 0-form lifting: both surface elements
                        wq *= patch_kappa(S.geom, tf, (ei1 + u1) * S.h, (ei2 + u2) * S.h) *
                              patch_kappa(S.geom, sf, (fi1 + w1) * S.h, (fi2 + w2) * S.h);
                    double pa[D1], pb[D1], qa[D1], qb[D1];
#pragma unroll
                    for (int l = 0; l < D1; ++l) {
                        pa[l] = basis_eval_d<D>(bt, c1a, l, u1);
                        pb[l] = basis_eval_d<D>(bt, c1b, l, u2);
                        qa[l] = basis_eval_d<D>(bt, c2a, l, w1);
                        qb[l] = basis_eval_d<D>(bt, c2b, l, w2);
                    }
                    const double dx = X[0] - Y[0], dy = X[1] - Y[1], dz = X[2] - Y[2];
                    const T kv = near_kernel(kd, dx * dx + dy * dy + dz * dz, T()) * (wq * kInv4Pi);
#pragma unroll
                    for (int ii = 0; ii < ROWS; ++ii) {
                        const int i = r0 + ii;
                        if (i < NB) {
                            const T fi = kv * (pa[i / D1] * pb[i % D1]);
#pragma unroll
                            for (int j = 0; j < NB; ++j) acc[ii * NB + j] += fi * (qa[j / D1] * qb[j % D1]);
                        }
                    }
                }
        }
#pragma unroll
        for (int v = 0; v < ROWS * NB; ++v) {
            const T s = wave_sum(acc[v]);
            if (lane == 0) red[wave][v] = s;
        }
        __syncthreads();
        for (int t = threadIdx.x; t < ROWS * NB; t += blockDim.x) {
            const int i = r0 + t / NB;
            if (i < NB) sb[i * NB + t % NB] = red[0][t] + red[1][t] + red[2][t] + red[3][t];
        }
        __syncthreads();
    }
}

// One workgroup per near leaf pair with touching element pairs: their element blocks, in
// the order of the pairs, added to the leaf-pair block.
template <class T, int D>
__global__ __launch_bounds__(128) void k_near_singular_add(OpDev op, AsmDev as) {
    constexpr int D1 = D + 1, NB = D1 * D1;
    const int m = op.m, nloc = op.nloc, nl2 = nloc * nloc, r = op.S.r;
    const int lp = as.touch_lp[blockIdx.x];
    T* out = (T*)as.lb + (int64_t)lp * nl2 * nl2;
    const T* sb = (const T*)as.sblk;
    for (int tp = as.touch_rowptr[lp]; tp < as.touch_rowptr[lp + 1]; ++tp) {
        const int et = as.touch[5 * tp], es = as.touch[5 * tp + 1];
        for (int t = threadIdx.x; t < NB * NB; t += blockDim.x) {
            const int i = t / NB, j = t % NB;
            const int r1 = (et / m) * r + i / D1, r2 = (et % m) * r + i % D1;
            const int cc1 = (es / m) * r + j / D1, cc2 = (es % m) * r + j % D1;
            out[(int64_t)(r1 * nloc + r2) * nl2 + cc1 * nloc + cc2] += sb[(int64_t)tp * NB * NB + t];
        }
        __syncthreads();
    }
}

// ------------------------------------------------------------------ near field: CSR values
// One wave per row g; each lane sums, for its column h, the leaf-pair blocks of every near
// leaf pair (tau, sigma) with g in dofs(tau) and h in dofs(sigma), in a fixed order.

template <class T>
__global__ __launch_bounds__(256) void k_near_gather(OpDev op, AsmDev as) {
    const SpaceDesc S = op.S;
    const int64_t g = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (g >= S.ndof) return;
    const int nb = S.nb, n1 = op.nleaf1, nloc = op.nloc, stride = op.m * S.r;
    const int64_t nl2 = (int64_t)nloc * nloc;
    const int j2 = (int)(g % nb), j1 = (int)((g / nb) % nb), f = (int)(g / ((int64_t)nb * nb));
    int lo1, hi1, lo2, hi2;
    leaf_range(j1, stride, nloc, n1, lo1, hi1);
    leaf_range(j2, stride, nloc, n1, lo2, hi2);
    const T* lb = (const T*)as.lb;
    const int64_t grp = as.row_grp[g];
    const int64_t rbeg = op.rowptr[g], ncol = op.rowptr[g + 1] - rbeg;
    T* val = (T*)op.val + op.grp_voff[grp] + as.row_pos[g] * ncol - rbeg;
    for (int64_t k = op.rowptr[g] + lane; k < op.rowptr[g + 1]; k += kWave) {
        const int h = op.col[k];
        const int h2 = h % nb, h1 = (h / nb) % nb, hf = h / (nb * nb);
        int mlo1, mhi1, mlo2, mhi2;
        leaf_range(h1, stride, nloc, n1, mlo1, mhi1);
        leaf_range(h2, stride, nloc, n1, mlo2, mhi2);
        T v = zero<T>();
        for (int a = lo1; a <= hi1; ++a)
            for (int b = lo2; b <= hi2; ++b) {
                const int tl = (f * n1 + a) * n1 + b;
                const int gl = (j1 - a * stride) * nloc + (j2 - b * stride);
                const int beg = as.near_rowptr[tl], end = as.near_rowptr[tl + 1];
                for (int c = mlo1; c <= mhi1; ++c)
                    for (int d = mlo2; d <= mhi2; ++d) {
                        const int sl = (hf * n1 + c) * n1 + d;
                        int lo = beg, hi = end;
                        while (lo < hi) {
                            const int mid = (lo + hi) >> 1;
                            if (as.near_s[mid] < sl)
                                lo = mid + 1;
                            else
                                hi = mid;
                        }
                        if (lo < end && as.near_s[lo] == sl) {
                            const int hl = (h1 - c * stride) * nloc + (h2 - d * stride);
                            v += lb[(int64_t)lo * nl2 * nl2 + gl * nl2 + hl];
                        }
                    }
            }
        val[k] = v;
    }
}

// ------------------------------------------------------------------ far field assembly
__device__ inline int cluster_level(const int64_t* lev_off, int leaf, int64_t c) {
    int l = 0;
    while (l < leaf && c >= lev_off[l + 1]) ++l;
    return l;
}

__global__ void k_cluster_points(OpDev op, AsmDev as) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= op.ncl * op.q2) return;
    const int a = (int)(idx % op.q2);
    const int64_t c = idx / op.q2;
    const int lev = cluster_level(op.lev_off, op.leaf, c);
    const int n = 1 << lev;
    const int64_t loc = c - op.lev_off[lev];
    const int j = (int)(loc % n), i = (int)((loc / n) % n), f = (int)(loc / ((int64_t)n * n));
    const double w = 1.0 / n;
    double x[3];
    patch_point(op.S.geom, f, (i + as.cheb[a / op.q]) * w, (j + as.cheb[a % op.q]) * w, x);
    as.xc[3 * idx] = x[0];
    as.xc[3 * idx + 1] = x[1];
    as.xc[3 * idx + 2] = x[2];
}

template <class T>
__global__ void k_far_assemble(OpDev op, AsmDev as) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int q2 = op.q2;
    const int64_t per = (int64_t)q2 * q2;
    if (idx >= op.nstored * per) return;
    const int64_t blk = idx / per;
    const int rem = (int)(idx - blk * per), a = rem / q2, b = rem % q2;
    const int t = as.own_t[blk], s = op.own_src[blk];
    const int64_t slot = blk - op.own_rowptr[t];
    const double* x = as.xc + ((int64_t)t * q2 + a) * 3;
    const double* y = as.xc + ((int64_t)s * q2 + b) * 3;
    const double dx = x[0] - y[0], dy = x[1] - y[1], dz = x[2] - y[2];
    ((T*)op.K)[op.koff[t] + (int64_t)a * op.krs[t] + slot * q2 + b] = kernel_val(op.S.ker, dx * dx + dy * dy + dz * dz, T());
}

// Reduce-scatter of Q2 per-lane values across the wave: after the six butterfly steps
// lane l holds the wave sum of one index (returned in `idx`, valid if `ok`).
template <class T, int C>
__device__ inline void rs_step(T* v, bool upper, int off) {
    constexpr int H = (C + 1) / 2;
#pragma unroll
    for (int i = 0; i < H; ++i) {
        const T lo = v[i];
        const T hi = (i + H < C) ? v[i + H] : T{};
        const T send = upper ? lo : hi;
        const T keep = upper ? hi : lo;
        v[i] = keep + shfl_xor_t(send, off);
    }
}

template <int C>
__device__ inline void rs_index(int lane, int off, int& base, int& real) {
    constexpr int H = (C + 1) / 2;
    if (lane & off) {
        base += H;
        real = real > H ? real - H : 0;
    } else {
        real = real < H ? real : H;
    }
}

template <class T, int Q2>
__device__ inline void wave_reduce_scatter(T* v, int lane, int& idx, bool& ok) {
    constexpr int C1 = Q2, C2 = (C1 + 1) / 2, C3 = (C2 + 1) / 2, C4 = (C3 + 1) / 2, C5 = (C4 + 1) / 2,
                  C6 = (C5 + 1) / 2;
    rs_step<T, C1>(v, lane & 32, 32);
    rs_step<T, C2>(v, lane & 16, 16);
    rs_step<T, C3>(v, lane & 8, 8);
    rs_step<T, C4>(v, lane & 4, 4);
    rs_step<T, C5>(v, lane & 2, 2);
    rs_step<T, C6>(v, lane & 1, 1);
    int base = 0, real = Q2;
    rs_index<C1>(lane, 32, base, real);
    rs_index<C2>(lane, 16, base, real);
    rs_index<C3>(lane, 8, base, real);
    rs_index<C4>(lane, 4, base, real);
    rs_index<C5>(lane, 2, base, real);
    rs_index<C6>(lane, 1, base, real);
    idx = base;
    ok = real > 0;
}

// ------------------------------------------------------------------ 0-form leaf tables
// Lagrange basis polynomial a of the q nodes at y (product form)
__device__ inline double lagrange_dev(const double* nodes, int q, int a, double y) {
    double v = 1.0;
    for (int b = 0; b < q; ++b)
        if (b != a) v *= (y - nodes[b]) / (nodes[a] - nodes[b]);
    return v;
}

// Vd[leaf][a][m1 nloc + m2] = integral over the leaf of L_a1 L_a2 b_{first1+m1} b_{first2+m2} kappa,
// by the qg x qg Gauss rule of the regular near field on every element (points, weights,
// basis values and kappa from its tables), one block per leaf, the leaf's elements one after
// the other (the map from a thread to its (a, l1, l2) entries does not depend on the element,
// so each entry is only ever added to by one thread).
template <int Q>
__global__ __launch_bounds__(256) void k_leaf_tables0(OpDev op, AsmDev as, double* __restrict__ Vd) {
    constexpr int Q2 = Q * Q;
    __shared__ double wk[256], L1[256][Q], L2[256][Q], B1[256][3], B2[256][3];
    const SpaceDesc& S = op.S;
    const int n1 = op.nleaf1, m = op.m, nloc = op.nloc, D1 = S.d + 1, r = S.r, qg = op.qg, qg2 = qg * qg;
    const int64_t leaf = blockIdx.x;
    const int j = (int)(leaf % n1), i = (int)((leaf / n1) % n1), f = (int)(leaf / ((int64_t)n1 * n1));
    double* V = Vd + leaf * Q2 * nloc * nloc;
    for (int t = threadIdx.x; t < Q2 * nloc * nloc; t += blockDim.x) V[t] = 0.0;
    for (int e = 0; e < m * m; ++e) {
        const int e1 = e / m, e2 = e % m, ei1 = i * m + e1, ei2 = j * m + e2;
        const int64_t eid = elem_id(S, f, ei1, ei2);
        __syncthreads();
        for (int pq = threadIdx.x; pq < qg2; pq += blockDim.x) {
            const int a1 = pq / qg, a2 = pq % qg;
            wk[pq] = as.gw[a1] * as.gw[a2] * S.h * S.h * as.gkap[eid * qg2 + pq];
            const double sl = (e1 + as.gx[a1]) / m, tl = (e2 + as.gx[a2]) / m;
            for (int a = 0; a < Q; ++a) {
                L1[pq][a] = lagrange_dev(as.cheb, Q, a, sl);
                L2[pq][a] = lagrange_dev(as.cheb, Q, a, tl);
            }
            for (int l = 0; l < D1; ++l) {
                B1[pq][l] = as.psi[((int64_t)ei1 * qg + a1) * D1 + l];
                B2[pq][l] = as.psi[((int64_t)ei2 * qg + a2) * D1 + l];
            }
        }
        __syncthreads();
        for (int t = threadIdx.x; t < Q2 * D1 * D1; t += blockDim.x) {
            const int a = t / (D1 * D1), l = t % (D1 * D1), a1 = a / Q, a2 = a % Q, l1 = l / D1, l2 = l % D1;
            double acc = 0.0;
            for (int pq = 0; pq < qg2; ++pq) acc += wk[pq] * L1[pq][a1] * L2[pq][a2] * B1[pq][l1] * B2[pq][l2];
            V[(int64_t)a * nloc * nloc + (e1 * r + l1) * nloc + (e2 * r + l2)] += acc;
        }
    }
}

// ------------------------------------------------------------------ H^2 matvec
// Stage 0.  Blocks [0, nup): forward transform of the leaves of one subtree rooted at level
// up_root and upward transfer inside it (LDS).  Blocks [nup, ...): near-field product
// by row groups, overwriting y.  The levels above up_root follow in k_up_top.
template <class T, int Q>
__device__ inline void up_subtree(const OpDev& op, int blk, const T* __restrict__ x) {
    constexpr int Q2 = Q * Q;
    __shared__ double Es[2 * Q * Q];
    __shared__ T tree[21][Q2];  // levels below the root: 16 + 4 + 1 clusters at most
    for (int i = threadIdx.x; i < 2 * Q * Q; i += blockDim.x) Es[i] = op.E[i];
    T* mom = (T*)op.mom;
    const int r0 = op.up_root, s = op.up_depth, leaf = op.leaf;
    const int nr = 1 << r0, w = 1 << s;  // roots per direction, leaves per root direction
    const int f = blk / (nr * nr), loc = blk % (nr * nr), ri = loc / nr, rj = loc % nr;
    const int n1 = op.nleaf1, nloc = op.nloc, stride = op.m * op.S.r;
    // LDS slots of the subtree: depth-2 clusters (16) at 0, depth-1 (4) at 16, root at 20
    const int lb = s == 2 ? 0 : (s == 1 ? 16 : 20);
    // the coefficients under the subtree's leaves form an E x E square; when it fits, it
    // is staged in LDS with coalesced loads, so that the transforms below read LDS instead
    // of issuing dependent global loads
    constexpr int kStage = 24;
    __shared__ T xs[kStage * kStage];
    const int E = (w - 1) * stride + nloc;
    const bool staged = E <= kStage;
    if (staged) {
        const int b1 = ri * w * stride, b2 = rj * w * stride;
        for (int idx = threadIdx.x; idx < E * E; idx += blockDim.x) {
            const int e1 = idx / E, e2 = idx - e1 * E;
            xs[idx] = x[dof_id(op.S, f, b1 + e1, b2 + e2)];
        }
        __syncthreads();
    }
    // leaves of this subtree
    for (int idx = threadIdx.x; idx < w * w * Q2; idx += blockDim.x) {
        const int a = idx % Q2, l = idx / Q2;
        const int i = ri * w + l / w, j = rj * w + l % w, a1 = a / Q, a2 = a % Q;
        const double* Vi = op.V1 + ((int64_t)i * Q + a1) * nloc;
        const double* Vj = op.V1 + ((int64_t)j * Q + a2) * nloc;
        T acc = zero<T>();
        if (op.Vd) {
            // 0-form lifting: the leaf's full table (the surface element does not separate)
            const double* V = op.Vd + (((int64_t)f * n1 + i) * n1 + j) * Q2 * nloc * nloc + (int64_t)a * nloc * nloc;
            for (int m1 = 0; m1 < nloc; ++m1)
                for (int m2 = 0; m2 < nloc; ++m2)
                    acc += V[m1 * nloc + m2] *
                           (staged ? xs[((l / w) * stride + m1) * E + (l % w) * stride + m2]
                                   : x[dof_id(op.S, f, i * stride + m1, j * stride + m2)]);
        } else if (staged) {
            const T* xl = xs + (l / w) * stride * E + (l % w) * stride;
#pragma unroll 2
            for (int m1 = 0; m1 < nloc; ++m1) {
                T in = zero<T>();
#pragma unroll 6
                for (int m2 = 0; m2 < nloc; ++m2) in += Vj[m2] * xl[m1 * E + m2];
                acc += Vi[m1] * in;
            }
        } else {
#pragma unroll 2
            for (int m1 = 0; m1 < nloc; ++m1) {
                const T* xr = x + dof_id(op.S, f, i * stride + m1, j * stride);
                T in = zero<T>();
#pragma unroll 6
                for (int m2 = 0; m2 < nloc; ++m2) in += Vj[m2] * xr[m2];
                acc += Vi[m1] * in;
            }
        }
        mom[(op.lev_off[leaf] + ((int64_t)f * n1 + i) * n1 + j) * Q2 + a] = acc;
        tree[lb + l][a] = acc;
    }
    // upward inside the subtree, depth s-1 .. 0 (level r0 + depth)
    for (int d = s - 1; d >= 0; --d) {
        __syncthreads();
        const int cw = 1 << d, lev = r0 + d;
        const int cb = (d + 1 == s) ? lb : 16, ob = d == 1 ? 16 : 20;
        for (int idx = threadIdx.x; idx < cw * cw * Q2; idx += blockDim.x) {
            const int a = idx % Q2, l = idx / Q2, u = l / cw, v = l % cw, a1 = a / Q, a2 = a % Q;
            T acc = zero<T>();
#pragma unroll 1
            for (int b1 = 0; b1 < 2; ++b1)
#pragma unroll 1
                for (int b2 = 0; b2 < 2; ++b2) {
                    const T* mc = tree[cb + (2 * u + b1) * (2 * cw) + 2 * v + b2];
#pragma unroll 1
                    for (int p1 = 0; p1 < Q; ++p1) {
                        T in = zero<T>();
#pragma unroll
                        for (int p2 = 0; p2 < Q; ++p2) in += Es[(b2 * Q + p2) * Q + a2] * mc[p1 * Q + p2];
                        acc += Es[(b1 * Q + p1) * Q + a1] * in;
                    }
                }
            tree[ob + l][a] = acc;
            const int gi = ri * cw + u, gj = rj * cw + v;
            mom[(op.lev_off[lev] + ((int64_t)f * (nr * cw) + gi) * (nr * cw) + gj) * Q2 + a] = acc;
        }
    }
}

// Stage 0b.  Upper levels of one patch's tree (levels up_root-1 .. 0), one block per
// patch, level by level from the moments written by stage 0.
template <class T, int Q>
__device__ inline void up_top_body(const OpDev& op, int64_t blk_) {
    constexpr int Q2 = Q * Q;
    __shared__ double Es[2 * Q * Q];
    for (int i = threadIdx.x; i < 2 * Q * Q; i += blockDim.x) Es[i] = op.E[i];
    T* mom = (T*)op.mom;
    const int f = blk_;
    for (int lev = op.up_root - 1; lev >= 0; --lev) {
        __syncthreads();
        const int n = 1 << lev, nc = n * n;
        for (int idx = threadIdx.x; idx < nc * Q2; idx += blockDim.x) {
            const int a = idx % Q2, loc = idx / Q2, i = loc / n, j = loc % n, a1 = a / Q, a2 = a % Q;
            T acc = zero<T>();
#pragma unroll 1
            for (int ch = 0; ch < 4; ++ch) {
                const int b1 = ch >> 1, b2 = ch & 1;
                const int64_t c = op.lev_off[lev + 1] + ((int64_t)f * 2 * n + 2 * i + b1) * 2 * n + 2 * j + b2;
                const T* mc = mom + c * Q2;
#pragma unroll
                for (int p1 = 0; p1 < Q; ++p1) {
                    T in = zero<T>();
#pragma unroll
                    for (int p2 = 0; p2 < Q; ++p2) in += Es[(b2 * Q + p2) * Q + a2] * mc[p1 * Q + p2];
                    acc += Es[(b1 * Q + p1) * Q + a1] * in;
                }
            }
            mom[(op.lev_off[lev] + (int64_t)f * nc + loc) * Q2 + a] = acc;
        }
    }
}

template <class T, int Q>
__global__ __launch_bounds__(256) void k_up_top(OpDev op) {
    up_top_body<T, Q>(op, blockIdx.x);
}

// rows of one near-field row group (R <= RMAX rows sharing C columns), see k_near_up.
// Columns are taken in blocks of U*64: per block every lane first issues its U column
// indices, then its U gathers of x, then the values of all rows, so that a block costs
// about two dependent memory round trips.
template <class T, int RMAX>
__device__ inline void near_group_rows(const int32_t* __restrict__ col, const T* __restrict__ val,
                                       const T* __restrict__ x, T* __restrict__ y, const int32_t* rows, int R, int C,
                                       int lane) {
    constexpr int U = RMAX <= 4 ? (sizeof(T) == 8 ? 8 : 4) : (sizeof(T) == 8 ? 4 : 2);
    T acc[RMAX];
#pragma unroll
    for (int r = 0; r < RMAX; ++r) acc[r] = zero<T>();
    for (int c0 = lane; c0 < C; c0 += U * kWave) {
        int cc[U];
        T xv[U];
#pragma unroll
        for (int u = 0; u < U; ++u) cc[u] = c0 + u * kWave < C ? col[c0 + u * kWave] : -1;
#pragma unroll
        for (int u = 0; u < U; ++u) xv[u] = cc[u] >= 0 ? x[cc[u]] : zero<T>();
#pragma unroll
        for (int r = 0; r < RMAX; ++r) {
            if (r < R) {
                T vv[U];
#pragma unroll
                for (int u = 0; u < U; ++u) vv[u] = cc[u] >= 0 ? val[(int64_t)r * C + c0 + u * kWave] : zero<T>();
#pragma unroll
                for (int u = 0; u < U; ++u) acc[r] += vv[u] * xv[u];
            }
        }
    }
    int idx;
    bool ok;
    wave_reduce_scatter<T, RMAX>(acc, lane, idx, ok);
    if (ok && idx < R) y[rows[idx]] = acc[0];
}

template <class T, int Q>
__device__ inline void near_up_body(const OpDev& op, int64_t blk_, const T* __restrict__ x, T* __restrict__ y) {
    const int nup = op.S.geom.npatch << (2 * op.up_root);
    if ((int)blk_ < nup) {
        up_subtree<T, Q>(op, blk_, x);
        return;
    }
    // near-field product of one row group: every lane takes columns c, c+64, ...; per
    // step it issues 4 column indices, then the 4 gathers of x, then the values of all the
    // group's rows (row-major, so each row's loads are coalesced across the wave)
    const int64_t G = (int64_t)(blk_ - nup) * 4 + uniform_int(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (G >= op.ngroups) return;
    const int64_t rb = op.grp_rowptr[G];
    const int R = (int)(op.grp_rowptr[G + 1] - rb);
    const int64_t first = op.grp_rows[rb];
    const int64_t cb = op.rowptr[first];
    const int C = (int)(op.rowptr[first + 1] - cb);
    const int32_t* __restrict__ col = op.col + cb;
    const T* __restrict__ val = (const T*)op.val + op.grp_voff[G];
    if (R <= 4)
        near_group_rows<T, 4>(col, val, x, y, op.grp_rows + rb, R, C, lane);
    else
        near_group_rows<T, kGroupRowsDev>(col, val, x, y, op.grp_rows + rb, R, C, lane);
}

// Stage 0 in one launch: the subtree blocks, then the levels above up_root by the last
// subtree block of each patch to finish.  Each subtree block releases its moments at device
// scope and counts itself in up_count[patch]; the block that brings the count to the
// number of subtrees acquires the others' moments, sums the upper levels and resets the
// count for the next apply (so no clearing is needed between applies or graph replays).
// No block waits for another.
template <class T, int Q>
__global__ __launch_bounds__(256) void k_near_up(OpDev op, const T* __restrict__ x, T* __restrict__ y) {
    const int nup = op.S.geom.npatch << (2 * op.up_root);
    if (op.up_count && op.up_root > 0 && (int)blockIdx.x < nup) {
        up_subtree<T, Q>(op, blockIdx.x, x);
        __shared__ int last;
        const int per = 1 << (2 * op.up_root), f = (int)blockIdx.x / per;
        __syncthreads();
        if (threadIdx.x == 0) {
            __threadfence();
            const int before = atomicAdd(op.up_count + f, 1);
            __threadfence();
            last = before == per - 1;
        }
        __syncthreads();
        if (last) {
            __threadfence();
            up_top_body<T, Q>(op, f);
            if (threadIdx.x == 0) op.up_count[f] = 0;
        }
        return;
    }
    near_up_body<T, Q>(op, blockIdx.x, x, y);
}

template <class T>
struct Pair {
    T x, y;
};

typedef double dvec2 __attribute__((ext_vector_type(2)));

// two adjacent scalars of a stream that is read once per matvec (non-temporal hint)
__device__ inline Pair<double> load_stream(const double* p) {
    const dvec2 v = __builtin_nontemporal_load((const dvec2*)p);
    return {v.x, v.y};
}
__device__ inline Pair<cdbl> load_stream(const cdbl* p) {
    const dvec2 a = __builtin_nontemporal_load((const dvec2*)p);
    const dvec2 b = __builtin_nontemporal_load((const dvec2*)p + 1);
    return {{a.x, a.y}, {b.x, b.y}};
}
// the same pairs with ordinary (cached) loads, for blocks that other blocks read again
__device__ inline Pair<double> load_cached(const double* p) {
    const dvec2 v = *(const dvec2*)p;
    return {v.x, v.y};
}
__device__ inline Pair<cdbl> load_cached(const cdbl* p) {
    const dvec2 a = *(const dvec2*)p;
    const dvec2 b = *((const dvec2*)p + 1);
    return {{a.x, a.y}, {b.x, b.y}};
}

// Stage 1.  Far-field coupling over the stored blocks, one wave per chunk of an owner's
// row-concatenated coupling rows.  Each lane takes two adjacent columns (sigma, b) per
// step: it loads the owner's Q2 row entries of both (16-byte loads, coalesced across the
// wave), accumulates K m_sigma into Q2 row sums, and forms the transposed product
// (K^T m_owner) of its columns, stored once per column.  Row sums are reduce-scattered
// across the wave into the chunk's partial sums.
template <class T, int Q, bool kStream = true>
__device__ inline void coupling_body(const OpDev& op, int64_t blk_) {
    constexpr int Q2 = Q * Q;
    const int64_t c = (int64_t)blk_ * 4 + uniform_int(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (c >= op.nchunks) return;
    const int t = op.ch_t[c], k0 = op.ch_k0[c], k1 = op.ch_k1[c];
    const int64_t rs = op.krs[t];
    const int64_t beg = op.own_rowptr[t];
    const int ncols = (int)(op.own_rowptr[t + 1] - beg) * Q2;
    const T* __restrict__ base = (const T*)op.K + op.koff[t];
    const int32_t* __restrict__ src = op.own_src + beg;
    const T* __restrict__ mom = (const T*)op.mom;
    T* __restrict__ P = (T*)op.P + op.pcol[t];
    T mown[Q2];
#pragma unroll
    for (int a = 0; a < Q2; ++a) mown[a] = mom[(int64_t)t * Q2 + a];
    T acc[Q2];
#pragma unroll
    for (int a = 0; a < Q2; ++a) acc[a] = zero<T>();
    for (int k = k0 + 2 * lane; k < k1; k += 2 * kWave) {
        const int s0 = k / Q2, b0 = k - s0 * Q2;
        const T m0 = mom[(int64_t)src[s0] * Q2 + b0];
        T m1 = zero<T>();
        if (k + 1 < ncols) {
            const int s1 = (k + 1) / Q2, b1 = (k + 1) - s1 * Q2;
            m1 = mom[(int64_t)src[s1] * Q2 + b1];
        }
        T p0 = zero<T>(), p1 = zero<T>();
#pragma unroll
        for (int a = 0; a < Q2; ++a) {
            const Pair<T> kv = kStream ? load_stream(base + a * rs + k) : load_cached(base + a * rs + k);
            acc[a] += kv.x * m0 + kv.y * m1;
            p0 += kv.x * mown[a];
            p1 += kv.y * mown[a];
        }
        *(Pair<T>*)(P + k) = Pair<T>{p0, p1};
    }
    int idx;
    bool ok;
    wave_reduce_scatter<T, Q2>(acc, lane, idx, ok);
    if (ok) ((T*)op.partial)[c * Q2 + idx] = acc[0];
}


// sin x and cos x for |x| < 2^20: x = k pi/2 + y with |y| <= pi/4 (pi/2 split into three
// doubles, each product subtracted with one rounding), then the Taylor series of sin and
// cos about 0 through y^17 and y^18 (truncation below 1e-19 at pi/4) and the quadrant k mod 4.
__device__ inline void sincos_reduced(double x, double* sn, double* cs) {
    const double k = __builtin_rint(x * 0.6366197723675814);  // 2 / pi
    double y = __builtin_fma(-k, 1.5707963267948966, x);
    y = __builtin_fma(-k, 6.123233995736766e-17, y);
    y = __builtin_fma(-k, -1.4973849048591698e-33, y);
    const double z = y * y;
    // coefficients (-1)^m / (2m+1)! and (-1)^m / (2m)!
    double ps = 2.8114572543455206e-15;
    ps = __builtin_fma(ps, z, -7.647163731819816e-13);
    ps = __builtin_fma(ps, z, 1.6059043836821613e-10);
    ps = __builtin_fma(ps, z, -2.505210838544172e-08);
    ps = __builtin_fma(ps, z, 2.7557319223985893e-06);
    ps = __builtin_fma(ps, z, -0.0001984126984126984);
    ps = __builtin_fma(ps, z, 0.008333333333333333);
    ps = __builtin_fma(ps, z, -0.16666666666666666);
    const double s = __builtin_fma(ps * z, y, y);
    double pc = -1.5619206968586225e-16;
    pc = __builtin_fma(pc, z, 4.779477332387385e-14);
    pc = __builtin_fma(pc, z, -1.1470745597729725e-11);
    pc = __builtin_fma(pc, z, 2.08767569878681e-09);
    pc = __builtin_fma(pc, z, -2.755731922398589e-07);
    pc = __builtin_fma(pc, z, 2.48015873015873e-05);
    pc = __builtin_fma(pc, z, -0.001388888888888889);
    pc = __builtin_fma(pc, z, 0.041666666666666664);
    pc = __builtin_fma(pc, z, -0.5);
    const double c = __builtin_fma(pc, z, 1.0);
    const int q = (int)k & 3;
    const double s1 = (q & 1) ? c : s, c1 = (q & 1) ? s : c;
    *sn = (q & 2) ? -s1 : s1;
    *cs = ((q + 1) & 2) ? -c1 : c1;
}

// the single-layer kernel without its constant factor 1/(4 pi), at NS distances r^2 > 0
template <int NS>
__device__ inline void kernel_unscaled(const KernelDesc&, const double* r2, double* kv) {
    rinv_nr<NS>(r2, kv);
}
template <int NS>
__device__ inline void kernel_unscaled(const KernelDesc& k, const double* r2, cdbl* kv) {
    double ir[NS];
    rinv_nr<NS>(r2, ir);
#pragma unroll
    for (int u = 0; u < NS; ++u) {
        const double r = r2[u] * ir[u];
        double sn, cs;
        sincos_reduced(k.kre * r, &sn, &cs);  // |Re kappa| r < 2^20, checked at planning
        const double mag = k.kim != 0.0 ? ir[u] * exp(k.kim * r) : ir[u];
        kv[u] = {mag * cs, -mag * sn};
    }
}

// One pass of the on-the-fly coupling over NS * 64 columns from kb (see coupling_otf_body).
template <class T, int Q, int NS>
__device__ inline void otf_pass(const OpDev& op, int kb, int k1, int kend, int lane, int w,
                                const int32_t* __restrict__ src, double o0, double o1, double o2,
                                const double4 (*opt)[Q * Q], const T (*omo)[Q * Q], T (*racc)[Q * Q],
                                T* __restrict__ P, const KernelDesc& kd) {
    constexpr int Q2 = Q * Q;
    constexpr int G = Q < 5 ? Q : 5;
    const T* __restrict__ mom = (const T*)op.mom;
    const double* __restrict__ xc = op.xc;
    double y0[NS], y1[NS], y2[NS], yy[NS];
    T ms[NS], p[NS];
#pragma unroll
    for (int u = 0; u < NS; ++u) {
        const int k = kb + u * kWave + lane;
        p[u] = zero<T>();
        if (k < kend) {
            const int sl = k / Q2, b = k - sl * Q2;
            const int64_t g = (int64_t)src[sl] * Q2 + b;
            y0[u] = xc[3 * g] - o0;
            y1[u] = xc[3 * g + 1] - o1;
            y2[u] = xc[3 * g + 2] - o2;
            ms[u] = mom[g];
        } else {
            y0[u] = y1[u] = y2[u] = 64.0;
            ms[u] = zero<T>();
        }
        yy[u] = y0[u] * y0[u] + y1[u] * y1[u] + y2[u] * y2[u];
    }
#pragma unroll 1
    for (int a0 = 0; a0 < Q2; a0 += G) {
        T sa[G];
#pragma unroll
        for (int g = 0; g < G; ++g) {
            sa[g] = zero<T>();
            const int a = a0 + g;
            if (Q2 % G != 0 && a >= Q2) continue;
            const double4 pa = opt[w][a];
            const T ma = omo[w][a];
            double r2[NS];
            T kv[NS];
#pragma unroll
            for (int u = 0; u < NS; ++u)
                r2[u] = __builtin_fma(pa.x, y0[u], __builtin_fma(pa.y, y1[u], __builtin_fma(pa.z, y2[u], pa.w + yy[u])));
            kernel_unscaled<NS>(kd, r2, kv);
#pragma unroll
            for (int u = 0; u < NS; ++u) {
                sa[g] += kv[u] * ms[u];
                p[u] += kv[u] * ma;
            }
        }
        int idx;
        bool ok;
        wave_reduce_scatter<T, G>(sa, lane, idx, ok);
        if (ok && a0 + idx < Q2) racc[w][a0 + idx] += sa[0];
    }
#pragma unroll
    for (int u = 0; u < NS; ++u) {
        const int k = kb + u * kWave + lane;
        if (k < k1) P[k] = p[u] * kInv4Pi;
    }
}

// Stage 1 without stored blocks: every coupling entry is the kernel at a pair of the
// clusters' Chebyshev points on the surface, evaluated where it is used (the stored
// blocks hold the same values).  Same chunks, row sums and transposed products as
// coupling_body.  Each lane takes NS columns (sigma, b) of a pass and keeps their points
// and moments in registers.  The owner's rows a are visited G at a time (points and
// moments staged in LDS per chunk): every lane adds k * m_owner[a] to its columns' transposed
// products, and the G row sums of the pass are reduce-scattered across the wave and
// added to the wave's row accumulators in LDS.  Columns past the row (its padding) or the
// chunk get a distant point and a zero moment; a pass skips the 64-column slices that hold
// padding only.
template <class T, int Q, int NS>
__device__ inline void coupling_otf_body(const OpDev& op, int64_t blk_) {
    constexpr int Q2 = Q * Q;
    static_assert(Q2 <= kWave, "one lane per row of the owner");
    __shared__ T racc[4][Q2];
    const int w = uniform_int(threadIdx.x >> 6);
    const int64_t c = (int64_t)blk_ * 4 + w;
    const int lane = threadIdx.x & 63;
    if (c >= op.nchunks) return;
    const int t = uniform_int(op.ch_t[c]), k0 = uniform_int(op.ch_k0[c]), k1 = uniform_int(op.ch_k1[c]);
    const int64_t beg = op.own_rowptr[t];
    const int32_t* __restrict__ src = op.own_src + beg;
    const int ncols = (int)(op.own_rowptr[t + 1] - beg) * Q2;  // rows are padded past this
    const int kend = k1 < ncols ? k1 : ncols;                   // last real column of the chunk
    const T* __restrict__ mom = (const T*)op.mom;
    const double* __restrict__ xc = op.xc;
    const double* __restrict__ xt = xc + (int64_t)t * Q2 * 3;
    const T* __restrict__ mt = mom + (int64_t)t * Q2;
    T* __restrict__ P = (T*)op.P + op.pcol[t];
    const KernelDesc kd = op.S.ker;
    // the owner's points and moments, staged once per chunk: the row loop reads them from
    // LDS (all lanes the same address) instead of waiting on global loads
    // Coordinates are taken relative to the owner's first point o, and the squared
    // distance is expanded as |x'|^2 + |y'|^2 - 2 x'.y' (three multiply-adds per entry).
    // For an admissible pair |x'|, |y'| and r are of one order, so the expansion loses
    // only a few units of rounding.  Staged per owner row: (-2 x', |x'|^2).
    __shared__ double4 opt[4][Q2];
    __shared__ T omo[4][Q2];
    const double o0 = xt[0], o1 = xt[1], o2 = xt[2];
    if (lane < Q2) {
        racc[w][lane] = zero<T>();
        const double d0 = xt[3 * lane] - o0, d1 = xt[3 * lane + 1] - o1, d2 = xt[3 * lane + 2] - o2;
        opt[w][lane] = double4{-2.0 * d0, -2.0 * d1, -2.0 * d2, d0 * d0 + d1 * d1 + d2 * d2};
        omo[w][lane] = mt[lane];
    }
    wave_sync();
    for (int kb = k0; kb < k1; kb += NS * kWave) {
        // 64-column slices past the row's last real column carry only padding: the last
        // pass of a row runs with as many slices as reach real columns
        const int nu = kend - kb >= NS * kWave ? NS : (kend - kb + kWave - 1) / kWave;  // uniform
        if (nu <= 0) continue;
        // the narrowest pass that covers the nu slices: 1, 2, 4 or NS
        if (nu == 1)
            otf_pass<T, Q, 1>(op, kb, k1, kend, lane, w, src, o0, o1, o2, opt, omo, racc, P, kd);
        else if (nu == 2 && NS > 2)
            otf_pass<T, Q, (NS > 2 ? 2 : NS)>(op, kb, k1, kend, lane, w, src, o0, o1, o2, opt, omo, racc, P, kd);
        else if (nu <= 4 && NS > 4)
            otf_pass<T, Q, (NS > 4 ? 4 : NS)>(op, kb, k1, kend, lane, w, src, o0, o1, o2, opt, omo, racc, P, kd);
        else
            otf_pass<T, Q, NS>(op, kb, k1, kend, lane, w, src, o0, o1, o2, opt, omo, racc, P, kd);
    }
    if (lane < Q2) ((T*)op.partial)[c * Q2 + lane] = racc[w][lane] * kInv4Pi;
}

// columns per lane and pass: 8 real (2 complex), or 4 real when the chunks are
// narrower than 512 columns
template <class T>
__host__ __device__ constexpr int otf_ns(bool wide) {
    return sizeof(T) == 16 ? 2 : (wide ? 8 : 4);
}

template <class T, int Q>
__global__ __launch_bounds__(256) void k_coupling(OpDev op) {
    coupling_body<T, Q>(op, blockIdx.x);
}

template <class T, int Q, int NS>
__global__ __launch_bounds__(256) void k_coupling_otf(OpDev op) {
    coupling_otf_body<T, Q, NS>(op, blockIdx.x);
}


// ------------------------------------------------------------------ low-precision far field


// storage types: FP32 (4 bytes per real scalar) or BF16 (2 bytes)
struct StFp32 {};
struct StBf16 {};

// two adjacent columns of a coupling row, converted to FP32
__device__ inline Pair<float> load_low(StFp32, const void* base, int64_t off) {
    const float2 v = *((const float2*)base + off / 2);
    return {v.x, v.y};
}
__device__ inline Pair<float> load_low(StBf16, const void* base, int64_t off) {
    const uint32_t v = *((const uint32_t*)base + off / 2);
    return {bf2f(v & 0xFFFFu), bf2f(v >> 16)};
}
__device__ inline Pair<cflt> load_low_c(StFp32, const void* base, int64_t off) {
    const float4 v = *((const float4*)base + off / 2);
    return {{v.x, v.y}, {v.z, v.w}};
}
__device__ inline Pair<cflt> load_low_c(StBf16, const void* base, int64_t off) {
    const uint2 v = *((const uint2*)base + off / 2);
    return {{bf2f(v.x & 0xFFFFu), bf2f(v.x >> 16)}, {bf2f(v.y & 0xFFFFu), bf2f(v.y >> 16)}};
}
template <class St>
__device__ inline Pair<float> load_pair(St st, const void* base, int64_t off, float) {
    return load_low(st, base, off);
}
template <class St>
__device__ inline Pair<cflt> load_pair(St st, const void* base, int64_t off, cflt) {
    return load_low_c(st, base, off);
}

__global__ void k_cast_low(int64_t n_scalars, const double* __restrict__ K, void* __restrict__ out, int kind) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_scalars) return;
    if (kind == 1)
        ((float*)out)[i] = (float)K[i];
    else
        ((uint16_t*)out)[i] = f2bf((float)K[i]);
}

// Stage 1 with the low-precision copy: as k_coupling, with the blocks and moments in
// FP32 arithmetic (FP32 accumulation); the row sums and transposed products are written
// back in FP64 for the rest of the pipeline.
template <class T, class F, class St, int Q>
__global__ __launch_bounds__(256) void k_coupling_low(OpDev op) {
    constexpr int Q2 = Q * Q;
    const int64_t c = (int64_t)blockIdx.x * 4 + uniform_int(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (c >= op.nchunks) return;
    const int t = op.ch_t[c], k0 = op.ch_k0[c], k1 = op.ch_k1[c];
    const int64_t rs = op.krs[t];
    const int64_t beg = op.own_rowptr[t];
    const int ncols = (int)(op.own_rowptr[t + 1] - beg) * Q2;
    const int64_t koff = op.koff[t];
    const int32_t* __restrict__ src = op.own_src + beg;
    const T* __restrict__ mom = (const T*)op.mom;
    T* __restrict__ P = (T*)op.P + op.pcol[t];
    F mown[Q2];
#pragma unroll
    for (int a = 0; a < Q2; ++a) mown[a] = to_f(mom[(int64_t)t * Q2 + a]);
    F acc[Q2];
#pragma unroll
    for (int a = 0; a < Q2; ++a) acc[a] = zero_f<F>();
    for (int k = k0 + 2 * lane; k < k1; k += 2 * kWave) {
        const int s0 = k / Q2, b0 = k - s0 * Q2;
        const F m0 = to_f(mom[(int64_t)src[s0] * Q2 + b0]);
        F m1 = zero_f<F>();
        if (k + 1 < ncols) {
            const int s1 = (k + 1) / Q2, b1 = (k + 1) - s1 * Q2;
            m1 = to_f(mom[(int64_t)src[s1] * Q2 + b1]);
        }
        F p0 = zero_f<F>(), p1 = zero_f<F>();
#pragma unroll
        for (int a = 0; a < Q2; ++a) {
            const Pair<F> kv = load_pair(St(), op.Klow, koff + a * rs + k, F());
            acc[a] += kv.x * m0 + kv.y * m1;
            p0 += kv.x * mown[a];
            p1 += kv.y * mown[a];
        }
        *(Pair<T>*)(P + k) = Pair<T>{to_d(p0), to_d(p1)};
    }
    int idx;
    bool ok;
    wave_reduce_scatter<F, Q2>(acc, lane, idx, ok);
    if (ok) ((T*)op.partial)[c * Q2 + idx] = to_d(acc[0]);
}

// Stage 2a.  Local expansion of every cluster: its chunks' row sums plus the transposed
// products of the blocks stored in its partners' rows.  One wave per cluster; the two
// half-waves take alternate entries (lane & 31 = component), then add.
template <class T, int Q>
__device__ inline void lv_gather_body(const OpDev& op, int64_t blk_) {
    constexpr int Q2 = Q * Q;
    static_assert(Q2 <= 64, "q <= 8");
    const int64_t t = (int64_t)blk_ * 4 + uniform_int(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (t >= op.ncl) return;
    const T* __restrict__ partial = (const T*)op.partial;
    const T* __restrict__ P = (const T*)op.P;
    T v = zero<T>();
    if (Q2 <= 32) {
        const int a = lane & 31, h = lane >> 5;
        if (a < Q2) {
            for (int64_t c = op.cl_chunk[t] + h; c < op.cl_chunk[t + 1]; c += 2) v += partial[c * Q2 + a];
            const int64_t e0 = op.tr_rowptr[t], e1 = op.tr_rowptr[t + 1];
#pragma unroll 4
            for (int64_t e = e0 + h; e < e1; e += 2) v += P[op.tr_off[e] + a];
        }
        v += shfl_xor_t(v, 32);
        if (lane < Q2) ((T*)op.lv)[t * Q2 + lane] = v;
    } else {
        if (lane < Q2) {
            for (int64_t c = op.cl_chunk[t]; c < op.cl_chunk[t + 1]; ++c) v += partial[c * Q2 + lane];
#pragma unroll 4
            for (int64_t e = op.tr_rowptr[t]; e < op.tr_rowptr[t + 1]; ++e) v += P[op.tr_off[e] + lane];
            ((T*)op.lv)[t * Q2 + lane] = v;
        }
    }
}

template <class T, int Q>
__global__ __launch_bounds__(256) void k_lv_gather(OpDev op) {
    lv_gather_body<T, Q>(op, blockIdx.x);
}

// Stage 2b + 3.  Downward transfer and backward transform per tile of TxT leaves: every
// leaf of the tile and of a one-leaf halo gets its total local expansion along its
// ancestor chain (v_0 = lv(patch), v_l = (E_b1 (x) E_b2) v_{l-1} + lv(ancestor at level
// l)) in LDS; then every DOF whose first B-spline lies in the tile adds
// sum over its leaves of (V_tau^T v_tau) to y.
template <class T, int Q>
__device__ inline void down_back_body(const OpDev& op, int64_t blk_, T* __restrict__ y) {
    constexpr int Q2 = Q * Q;
    constexpr int TMAX = 4, HW = TMAX + 2;  // tile and tile + halo (leaves per direction)
    __shared__ double Es[2 * Q * Q];
    __shared__ T vbuf[2][HW * HW][Q2];
    for (int i = threadIdx.x; i < 2 * Q * Q; i += blockDim.x) Es[i] = op.E[i];
    const int T1 = op.tile, n1 = op.nleaf1, nt = n1 / T1;
    const int f = blk_ / (nt * nt), loc = blk_ % (nt * nt);
    const int ti = (loc / nt) * T1, tj = (loc % nt) * T1;
    // halo-extended leaf range, clamped to the patch
    const int i0 = max(ti - 1, 0), i1 = min(ti + T1, n1 - 1), j0 = max(tj - 1, 0), j1 = min(tj + T1, n1 - 1);
    const int wi = i1 - i0 + 1, wj = j1 - j0 + 1, nl = wi * wj;
    const T* lv = (const T*)op.lv;
    int cur = 0;
    // level 0: the patch's own expansion for every leaf
    for (int idx = threadIdx.x; idx < nl * Q2; idx += blockDim.x)
        vbuf[0][idx / Q2][idx % Q2] = lv[(op.lev_off[0] + f) * Q2 + idx % Q2];
    for (int lev = 1; lev <= op.leaf; ++lev) {
        __syncthreads();
        const int sh = op.leaf - lev, n = 1 << lev;
        for (int idx = threadIdx.x; idx < nl * Q2; idx += blockDim.x) {
            const int p = idx % Q2, l = idx / Q2, p1 = p / Q, p2 = p % Q;
            const int li = i0 + l / wj, lj = j0 + l % wj;
            const int ai = li >> sh, aj = lj >> sh, b1 = ai & 1, b2 = aj & 1;
            const T* v = vbuf[cur][l];
            T acc = zero<T>();
#pragma unroll
            for (int a1 = 0; a1 < Q; ++a1) {
                T in = zero<T>();
#pragma unroll
                for (int a2 = 0; a2 < Q; ++a2) in += Es[(b2 * Q + p2) * Q + a2] * v[a1 * Q + a2];
                acc += Es[(b1 * Q + p1) * Q + a1] * in;
            }
            vbuf[cur ^ 1][l][p] = acc + lv[(op.lev_off[lev] + ((int64_t)f * n + ai) * n + aj) * Q2 + p];
        }
        cur ^= 1;
    }
    __syncthreads();
    // DOFs owned by the tile: first B-spline index in [ti*stride, (ti+T1)*stride), the last
    // tile also owning the trailing ones
    const int nb = op.S.nb, nloc = op.nloc, stride = op.m * op.S.r;
    const int g1a = ti * stride, g1b = (ti + T1 >= n1) ? nb : (ti + T1) * stride;
    const int g2a = tj * stride, g2b = (tj + T1 >= n1) ? nb : (tj + T1) * stride;
    const int nw = g2b - g2a;
    for (int idx = threadIdx.x; idx < (g1b - g1a) * nw; idx += blockDim.x) {
        const int jj1 = g1a + idx / nw, jj2 = g2a + idx % nw;
        int lo1, hi1, lo2, hi2;
        leaf_range(jj1, stride, nloc, n1, lo1, hi1);
        leaf_range(jj2, stride, nloc, n1, lo2, hi2);
        T acc = zero<T>();
        for (int li = lo1; li <= hi1; ++li)
            for (int lj = lo2; lj <= hi2; ++lj) {
                const T* L = vbuf[cur][(li - i0) * wj + (lj - j0)];
                if (op.Vd) {  // 0-form lifting: the leaf's full table
                    const double* V = op.Vd + (((int64_t)f * n1 + li) * n1 + lj) * Q2 * nloc * nloc +
                                      (jj1 - li * stride) * nloc + (jj2 - lj * stride);
#pragma unroll
                    for (int a = 0; a < Q2; ++a) acc += V[(int64_t)a * nloc * nloc] * L[a];
                    continue;
                }
                const double* Vi = op.V1 + (int64_t)li * Q * nloc + (jj1 - li * stride);
                const double* Vj = op.V1 + (int64_t)lj * Q * nloc + (jj2 - lj * stride);
#pragma unroll
                for (int a1 = 0; a1 < Q; ++a1) {
                    T in = zero<T>();
#pragma unroll
                    for (int a2 = 0; a2 < Q; ++a2) in += Vj[a2 * nloc] * L[a1 * Q + a2];
                    acc += Vi[a1 * nloc] * in;
                }
            }
        y[dof_id(op.S, f, jj1, jj2)] += acc;
    }
}

template <class T, int Q>
__global__ __launch_bounds__(256) void k_down_back(OpDev op, T* __restrict__ y) {
    down_back_body<T, Q>(op, blockIdx.x, y);
}

// ------------------------------------------------------------------ load vector and potential
template <class T>
__device__ inline T data_value(int kind, const KernelDesc& kd, double p0, double p1, double p2, const double* x);
template <>
__device__ inline double data_value<double>(int, const KernelDesc& kd, double p0, double p1, double p2,
                                            const double* x) {
    const double dx = x[0] - p0, dy = x[1] - p1, dz = x[2] - p2;
    return kernel_val(kd, dx * dx + dy * dy + dz * dz, 0.0);
}
template <>
__device__ inline cdbl data_value<cdbl>(int kind, const KernelDesc& kd, double p0, double p1, double p2,
                                        const double* x) {
    if (kind == 0) {
        const double dx = x[0] - p0, dy = x[1] - p1, dz = x[2] - p2;
        return kernel_val(kd, dx * dx + dy * dy + dz * dz, cdbl{0.0, 0.0});
    }
    // plane wave exp(-i kappa d.x), kappa = kre + i kim
    const double dd = p0 * x[0] + p1 * x[1] + p2 * x[2];
    double s, c;
    sincos(kd.kre * dd, &s, &c);
    const double mag = kd.kim != 0.0 ? exp(kd.kim * dd) : 1.0;
    return {mag * c, -mag * s};
}

// Local functions of global function G: itself (S^2) or its glued ones (S^0)
__device__ inline void glue_range(const SpaceDesc& S, int64_t G, int64_t& k0, int64_t& k1) {
    if (S.ginv_ptr) {
        k0 = S.ginv_ptr[G];
        k1 = S.ginv_ptr[G + 1];
    } else {
        k0 = G;
        k1 = G + 1;
    }
}
__device__ inline int64_t glue_local(const SpaceDesc& S, int64_t k) { return S.ginv_ptr ? S.ginv_idx[k] : k; }
__device__ inline int64_t glue_global(const SpaceDesc& S, int64_t g) { return S.glue ? S.glue[g] : g; }

// b_G = sum over the local functions g of G (S^0: the glued ones, in ascending order) and the
// elements of supp(g) of 8x8 Gauss sums of g(x) phi_g (times kappa for the 0-form lifting);
// one wave per global function
template <class T>
__global__ __launch_bounds__(256) void k_rhs(SpaceDesc S, BasisTab bt, Gauss8 g8, int kind, double p0, double p1,
                                             double p2, T* b) {
    const int64_t G = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (G >= S.nglob) return;
    const int nb = S.nb, d = S.d, r = S.r;
    const int a1 = lane >> 3, a2 = lane & 7;
    T acc = zero<T>();
    int64_t k0, k1;
    glue_range(S, G, k0, k1);
    for (int64_t k = k0; k < k1; ++k) {
        const int64_t g = glue_local(S, k);
        const int j2 = (int)(g % nb), j1 = (int)((g / nb) % nb), f = (int)(g / ((int64_t)nb * nb));
        const int i1lo = j1 - d <= 0 ? 0 : (j1 - d + r - 1) / r, i1hi = min(j1 / r, S.nel - 1);
        const int i2lo = j2 - d <= 0 ? 0 : (j2 - d + r - 1) / r, i2hi = min(j2 / r, S.nel - 1);
        for (int i1 = i1lo; i1 <= i1hi; ++i1)
            for (int i2 = i2lo; i2 <= i2hi; ++i2) {
                const int l1 = j1 - i1 * r, l2 = j2 - i2 * r;
                if (l1 > d || l2 > d) continue;
                double x[3];
                const double ps = (i1 + g8.x[a1]) * S.h, pt = (i2 + g8.x[a2]) * S.h;
                patch_point(S.geom, f, ps, pt, x);
                double phi = basis_eval(bt, basis_class(bt, i1), l1, g8.x[a1]) *
                             basis_eval(bt, basis_class(bt, i2), l2, g8.x[a2]);
                if (S.form == 0) phi *= patch_kappa(S.geom, f, ps, pt);
                acc += data_value<T>(kind, S.ker, p0, p1, p2, x) * (g8.w[a1] * g8.w[a2] * S.h * S.h * phi);
            }
    }
    const T s = wave_sum(acc);
    if (lane == 0) b[G] = s;
}

// The load vector's quadrature points: point e * 64 + 8 a1 + a2 is the Gauss point (a1, a2)
// of element e = (patch, i1, i2), as used by k_rhs.
__global__ __launch_bounds__(256) void k_quadpoints(SpaceDesc S, Gauss8 g8, double* xyz) {
    const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (p >= S.nelem * 64) return;
    const int64_t e = p / 64;
    const int q = (int)(p % 64), a1 = q >> 3, a2 = q & 7;
    const int i2 = (int)(e % S.nel), i1 = (int)((e / S.nel) % S.nel), f = (int)(e / ((int64_t)S.nel * S.nel));
    double x[3];
    patch_point(S.geom, f, (i1 + g8.x[a1]) * S.h, (i2 + g8.x[a2]) * S.h, x);
    xyz[3 * p] = x[0];
    xyz[3 * p + 1] = x[1];
    xyz[3 * p + 2] = x[2];
}

// b_g from data sampled at those points (gv[e * 64 + q]): the quadrature of k_rhs with
// the samples in place of the built-in data
template <class T>
__global__ __launch_bounds__(256) void k_rhs_samples(SpaceDesc S, BasisTab bt, Gauss8 g8, const T* __restrict__ gv,
                                                     T* b) {
    const int64_t G = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (G >= S.nglob) return;
    const int nb = S.nb, d = S.d, r = S.r;
    const int a1 = lane >> 3, a2 = lane & 7;
    T acc = zero<T>();
    int64_t k0, k1;
    glue_range(S, G, k0, k1);
    for (int64_t k = k0; k < k1; ++k) {
        const int64_t g = glue_local(S, k);
        const int j2 = (int)(g % nb), j1 = (int)((g / nb) % nb), f = (int)(g / ((int64_t)nb * nb));
        const int i1lo = j1 - d <= 0 ? 0 : (j1 - d + r - 1) / r, i1hi = min(j1 / r, S.nel - 1);
        const int i2lo = j2 - d <= 0 ? 0 : (j2 - d + r - 1) / r, i2hi = min(j2 / r, S.nel - 1);
        for (int i1 = i1lo; i1 <= i1hi; ++i1)
            for (int i2 = i2lo; i2 <= i2hi; ++i2) {
                const int l1 = j1 - i1 * r, l2 = j2 - i2 * r;
                if (l1 > d || l2 > d) continue;
                double phi = basis_eval(bt, basis_class(bt, i1), l1, g8.x[a1]) *
                             basis_eval(bt, basis_class(bt, i2), l2, g8.x[a2]);
                if (S.form == 0) phi *= patch_kappa(S.geom, f, (i1 + g8.x[a1]) * S.h, (i2 + g8.x[a2]) * S.h);
                acc += gv[elem_id(S, f, i1, i2) * 64 + lane] * (g8.w[a1] * g8.w[a2] * S.h * S.h * phi);
            }
    }
    const T s = wave_sum(acc);
    if (lane == 0) b[G] = s;
}

// u(x_p) = sum_e 8x8 Gauss sum of k(x_p, y) rho_hat(y); one workgroup per point
template <class T>
__global__ __launch_bounds__(256) void k_potential(SpaceDesc S, BasisTab bt, Gauss8 g8, const double* pts,
                                                   const T* __restrict__ rho, T* u) {
    __shared__ T red[4];
    const int64_t p = blockIdx.x;
    const double px = pts[3 * p], py = pts[3 * p + 1], pz = pts[3 * p + 2];
    const int d = S.d, r = S.r;
    T acc = zero<T>();
    const int64_t total = S.nelem * 64;
    for (int64_t idx = threadIdx.x; idx < total; idx += blockDim.x) {
        const int a = (int)(idx & 63);
        const int64_t e = idx >> 6;
        const int i2 = (int)(e % S.nel), i1 = (int)((e / S.nel) % S.nel), f = (int)(e / ((int64_t)S.nel * S.nel));
        const double u1 = g8.x[a >> 3], u2 = g8.x[a & 7];
        double y[3];
        patch_point(S.geom, f, (i1 + u1) * S.h, (i2 + u2) * S.h, y);
        const int ca = basis_class(bt, i1), cb = basis_class(bt, i2);
        T rh = zero<T>();
        for (int l1 = 0; l1 <= d; ++l1) {
            const double ba = basis_eval(bt, ca, l1, u1);
            for (int l2 = 0; l2 <= d; ++l2)
                rh += (ba * basis_eval(bt, cb, l2, u2)) * rho[glue_global(S, dof_id(S, f, i1 * r + l1, i2 * r + l2))];
        }
        if (S.form == 0) rh = rh * patch_kappa(S.geom, f, (i1 + u1) * S.h, (i2 + u2) * S.h);
        const double dx = px - y[0], dy = py - y[1], dz = pz - y[2];
        acc += kernel_val(S.ker, dx * dx + dy * dy + dz * dz, T()) * rh * (g8.w[a >> 3] * g8.w[a & 7] * S.h * S.h);
    }
    acc = wave_sum(acc);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) u[p] = red[0] + red[1] + red[2] + red[3];
}

// u(x_p) through the cluster tree, one wave per point (four per block).  The wave walks
// every patch's quadtree from its root with a stack in LDS (every lane writes the same
// entries, so each lane reads back its own writes): a cluster whose ball is admissible for
// the point (dist = |x - c| - r > 0, 2 r <= eta dist, ties within 1e-12 dist inadmissible)
// adds sum_a k(x, xi_a) m_a over its q^2 Chebyshev points (lane a); an inadmissible leaf adds
// the 8x8 Gauss sums of its elements (lane = Gauss point); other clusters push their four
// children.  The walk is the same for all lanes, so the wave never diverges on it.
template <class T>
__global__ __launch_bounds__(256) void k_potential_tree(OpDev op, Gauss8 g8, double eta, const double* __restrict__ pts,
                                                        int64_t npts, const T* __restrict__ rho, T* __restrict__ u) {
    __shared__ int stk[4][64];
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t p = (int64_t)blockIdx.x * 4 + wv;
    if (p >= npts) return;  // whole waves only; no block barrier follows
    const SpaceDesc& S = op.S;
    const double px = pts[3 * p], py = pts[3 * p + 1], pz = pts[3 * p + 2];
    const T* __restrict__ mom = (const T*)op.mom;
    const int q2 = op.q2, d = S.d, r = S.r;
    const int m = 1 << (S.L - op.leaf);  // elements per leaf per direction
    int* st = stk[wv];
    T acc = zero<T>();
    for (int f = 0; f < S.geom.npatch; ++f) {
        int top = 0;
        st[top++] = 0;  // (level 0, i 0, j 0), packed as level << 24 | i << 12 | j
        while (top > 0) {
            const int code = st[--top];
            const int l = code >> 24, ci = (code >> 12) & 4095, cj = code & 4095;
            const int n = 1 << l;
            const int64_t c = op.lev_off[l] + ((int64_t)f * n + ci) * n + cj;
            const double* bl = op.ball + 4 * c;
            const double dx = px - bl[0], dy = py - bl[1], dz = pz - bl[2];
            const double dist = sqrt(dx * dx + dy * dy + dz * dz) - bl[3];
            const double lhs = 2.0 * bl[3], rhs = eta * dist;
            const bool adm = dist > 0.0 && !(fabs(lhs - rhs) <= 1e-12 * dist) && lhs <= rhs;
            if (adm) {
                if (lane < q2) {
                    const double* y = op.xc + (c * q2 + lane) * 3;
                    const double ex = px - y[0], ey = py - y[1], ez = pz - y[2];
                    acc += kernel_val(S.ker, ex * ex + ey * ey + ez * ez, T()) * mom[c * q2 + lane];
                }
            } else if (l == op.leaf) {
                const double u1 = g8.x[lane >> 3], u2 = g8.x[lane & 7];
                const double wq = g8.w[lane >> 3] * g8.w[lane & 7] * S.h * S.h;
                for (int e1 = 0; e1 < m; ++e1)
                    for (int e2 = 0; e2 < m; ++e2) {
                        const int i1 = ci * m + e1, i2 = cj * m + e2;
                        double y[3];
                        patch_point(S.geom, f, (i1 + u1) * S.h, (i2 + u2) * S.h, y);
                        const int ca = basis_class(op.bt, i1), cb = basis_class(op.bt, i2);
                        T rh = zero<T>();
                        for (int l1 = 0; l1 <= d; ++l1) {
                            const double ba = basis_eval(op.bt, ca, l1, u1);
                            for (int l2 = 0; l2 <= d; ++l2)
                                rh += (ba * basis_eval(op.bt, cb, l2, u2)) *
                                      rho[glue_global(S, dof_id(S, f, i1 * r + l1, i2 * r + l2))];
                        }
                        if (S.form == 0) rh = rh * patch_kappa(S.geom, f, (i1 + u1) * S.h, (i2 + u2) * S.h);
                        const double ex = px - y[0], ey = py - y[1], ez = pz - y[2];
                        acc += kernel_val(S.ker, ex * ex + ey * ey + ez * ez, T()) * rh * wq;
                    }
            } else {
                for (int k = 3; k >= 0; --k)
                    st[top++] = ((l + 1) << 24) | ((2 * ci + (k >> 1)) << 12) | (2 * cj + (k & 1));
            }
        }
    }
    acc = wave_sum(acc);
    if (lane == 0) u[p] = acc;
}

// ------------------------------------------------------------------ grouped launches
// apply of block b: the largest a < napply with prefix[a] <= b (empty applies skipped)
__device__ inline int64_t group_find(const int64_t* pre, int64_t napply, int64_t b) {
    int64_t lo = 0, hi = napply;
    while (hi - lo > 1) {
        const int64_t mid = (lo + hi) >> 1;
        if (pre[mid] <= b)
            lo = mid;
        else
            hi = mid;
    }
    return lo;
}

template <class T, int Q, int S>
__global__ __launch_bounds__(256) void kg_stage(GroupDev g) {
    const int64_t* pre = g.prefix + (int64_t)S * (g.nop + 1);
    // consecutive logical blocks on one XCD, where an operator's columns share its data
    const int64_t b = xcd_block(blockIdx.x, gridDim.x);
    const int64_t o = group_find(pre, g.nop, b);
    const int64_t j = b - pre[o];
    const int nc = g.ncol[o];
    const int64_t a = g.first[o] + j % nc;
    const int64_t blk = j / nc;
    const OpDev& op = g.ops[a];
    if constexpr (S == 0)
        near_up_body<T, Q>(op, blk, (const T*)g.x[a], (T*)g.y[a]);
    else if constexpr (S == 1)
        up_top_body<T, Q>(op, blk);
    else if constexpr (S == 2)
        coupling_body<T, Q, false>(op, blk);  // the operator's other columns read the same blocks
    else if constexpr (S == 5) {
        // the operator's own pass width, so that the sums match its one-operator apply
        if (op.otf_wide)
            coupling_otf_body<T, Q, otf_ns<T>(true)>(op, blk);
        else
            coupling_otf_body<T, Q, otf_ns<T>(false)>(op, blk);
    }
    else if constexpr (S == 3)
        lv_gather_body<T, Q>(op, blk);
    else
        down_back_body<T, Q>(op, blk, (T*)g.y[a]);
}

template <class T, int Q>
hipError_t group_tq(const GroupDev& g, hipStream_t st) {
    if (g.nblocks[0] > 0) hipLaunchKernelGGL((kg_stage<T, Q, 0>), dim3((unsigned)g.nblocks[0]), dim3(256), 0, st, g);
    if (g.nblocks[1] > 0) hipLaunchKernelGGL((kg_stage<T, Q, 1>), dim3((unsigned)g.nblocks[1]), dim3(256), 0, st, g);
    if (g.nblocks[2] > 0) hipLaunchKernelGGL((kg_stage<T, Q, 2>), dim3((unsigned)g.nblocks[2]), dim3(256), 0, st, g);
    if (g.nblocks[5] > 0) hipLaunchKernelGGL((kg_stage<T, Q, 5>), dim3((unsigned)g.nblocks[5]), dim3(256), 0, st, g);
    if (g.nblocks[3] > 0) hipLaunchKernelGGL((kg_stage<T, Q, 3>), dim3((unsigned)g.nblocks[3]), dim3(256), 0, st, g);
    if (g.nblocks[4] > 0) hipLaunchKernelGGL((kg_stage<T, Q, 4>), dim3((unsigned)g.nblocks[4]), dim3(256), 0, st, g);
    return hipGetLastError();
}

template <class T>
hipError_t group_t(const GroupDev& g, int q, hipStream_t st) {
    switch (q) {
        case 1: return group_tq<T, 1>(g, st);
        case 2: return group_tq<T, 2>(g, st);
        case 3: return group_tq<T, 3>(g, st);
        case 4: return group_tq<T, 4>(g, st);
        case 5: return group_tq<T, 5>(g, st);
        case 6: return group_tq<T, 6>(g, st);
        case 7: return group_tq<T, 7>(g, st);
        default: return group_tq<T, 8>(g, st);
    }
}

inline unsigned nblk(int64_t n, int per) { return (unsigned)((n + per - 1) / per); }

}  // namespace

// =========================================================================== launchers
hipError_t launch_leaf_tables0(const OpDev& op, const AsmDev& as, hipStream_t st) {
    if (!op.Vd || op.nleaves == 0) return hipSuccess;
    if (op.qg * op.qg > 256 || op.S.d > 2) return hipErrorInvalidValue;  // the kernel's LDS tables
    const dim3 g((unsigned)op.nleaves), b(256);
    switch (op.q) {
        case 1: hipLaunchKernelGGL(k_leaf_tables0<1>, g, b, 0, st, op, as, (double*)op.Vd); break;
        case 2: hipLaunchKernelGGL(k_leaf_tables0<2>, g, b, 0, st, op, as, (double*)op.Vd); break;
        case 3: hipLaunchKernelGGL(k_leaf_tables0<3>, g, b, 0, st, op, as, (double*)op.Vd); break;
        case 4: hipLaunchKernelGGL(k_leaf_tables0<4>, g, b, 0, st, op, as, (double*)op.Vd); break;
        case 5: hipLaunchKernelGGL(k_leaf_tables0<5>, g, b, 0, st, op, as, (double*)op.Vd); break;
        case 6: hipLaunchKernelGGL(k_leaf_tables0<6>, g, b, 0, st, op, as, (double*)op.Vd); break;
        case 7: hipLaunchKernelGGL(k_leaf_tables0<7>, g, b, 0, st, op, as, (double*)op.Vd); break;
        default: hipLaunchKernelGGL(k_leaf_tables0<8>, g, b, 0, st, op, as, (double*)op.Vd); break;
    }
    return hipGetLastError();
}

template <class T>
__global__ __launch_bounds__(256) void k_glue_gather(int64_t n, const int32_t* __restrict__ glue,
                                                     const T* __restrict__ x, T* __restrict__ xl) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) xl[i] = x[glue[i]];
}
template <class T>
__global__ __launch_bounds__(256) void k_glue_scatter(int64_t n, const int64_t* __restrict__ ptr,
                                                      const int32_t* __restrict__ idx, const T* __restrict__ yl,
                                                      T* __restrict__ y) {
    const int64_t g = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (g >= n) return;
    T acc = zero<T>();
    for (int64_t k = ptr[g]; k < ptr[g + 1]; ++k) acc += yl[idx[k]];  // ascending local order
    y[g] = acc;
}

hipError_t launch_glue_gather(const SpaceDesc& S, int cplx, const void* x, void* x_loc, hipStream_t st) {
    const dim3 g(nblk(S.ndof, 256));
    if (cplx)
        hipLaunchKernelGGL(k_glue_gather<cdbl>, g, dim3(256), 0, st, S.ndof, S.glue, (const cdbl*)x, (cdbl*)x_loc);
    else
        hipLaunchKernelGGL(k_glue_gather<double>, g, dim3(256), 0, st, S.ndof, S.glue, (const double*)x,
                           (double*)x_loc);
    return hipGetLastError();
}

hipError_t launch_glue_scatter(const SpaceDesc& S, int cplx, const void* y_loc, void* y, hipStream_t st) {
    const dim3 g(nblk(S.nglob, 256));
    if (cplx)
        hipLaunchKernelGGL(k_glue_scatter<cdbl>, g, dim3(256), 0, st, S.nglob, S.ginv_ptr, S.ginv_idx,
                           (const cdbl*)y_loc, (cdbl*)y);
    else
        hipLaunchKernelGGL(k_glue_scatter<double>, g, dim3(256), 0, st, S.nglob, S.ginv_ptr, S.ginv_idx,
                           (const double*)y_loc, (double*)y);
    return hipGetLastError();
}

hipError_t launch_gauss_points(const OpDev& op, const AsmDev& as, hipStream_t st) {
    const int64_t n = op.S.nelem * op.qg * op.qg;
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_gauss_points, dim3(nblk(n, 256)), dim3(256), 0, st, op.S, op.qg, as.gx, (double*)as.gpos,
                       (double*)as.gkap);
    return hipGetLastError();
}

template <class T, int D, int QG, bool K0>
static hipError_t near_regular_launch(const OpDev& op, const AsmDev& as, int W, int in_lds, size_t shm,
                                      hipStream_t st) {
    if (shm > 64 * 1024) {
        hipError_t e = hipFuncSetAttribute((const void*)k_near_regular<T, D, QG, K0>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL((k_near_regular<T, D, QG, K0>), dim3((unsigned)op.nnear), dim3(64 * W), shm, st, op, as, W,
                       in_lds);
    return hipGetLastError();
}

template <class T, int D>
static hipError_t near_regular_t(const OpDev& op, const AsmDev& as, hipStream_t st) {
    constexpr int NB = (D + 1) * (D + 1);
    const size_t lb = (size_t)op.nloc * op.nloc * op.nloc * op.nloc * sizeof(T);
    const size_t tb = (size_t)kWave * NB * sizeof(T);
    const size_t budget = 96 * 1024;
    int W = 4;
    while (W > 1 && W * (lb + tb) > budget) --W;
    int in_lds = W * (lb + tb) <= budget ? 1 : 0;
    if (!in_lds) W = 1;
    const size_t shm = in_lds ? W * (lb + tb) : tb;
    const bool k0 = as.gkap != nullptr;
    if (op.qg == 8)
        return k0 ? near_regular_launch<T, D, 8, true>(op, as, W, in_lds, shm, st)
                  : near_regular_launch<T, D, 8, false>(op, as, W, in_lds, shm, st);
    return k0 ? near_regular_launch<T, D, 0, true>(op, as, W, in_lds, shm, st)
              : near_regular_launch<T, D, 0, false>(op, as, W, in_lds, shm, st);
}

hipError_t launch_near_regular(const OpDev& op, const AsmDev& as, hipStream_t st) {
    if (op.nnear == 0) return hipSuccess;
    const int d = op.S.d;
    if (op.cplx) {
        if (d == 0) return near_regular_t<cdbl, 0>(op, as, st);
        if (d == 1) return near_regular_t<cdbl, 1>(op, as, st);
        return near_regular_t<cdbl, 2>(op, as, st);
    }
    if (d == 0) return near_regular_t<double, 0>(op, as, st);
    if (d == 1) return near_regular_t<double, 1>(op, as, st);
    return near_regular_t<double, 2>(op, as, st);
}

template <class T, int D, int ROWS, int FORM>
static void near_singular_geom(const OpDev& op, const AsmDev& as, hipStream_t st) {
    const dim3 g((unsigned)op.ntouch), b(256);
    switch (FORM == 2 ? op.S.geom.kind : -1) {
        case GEOM_SPHERE6: hipLaunchKernelGGL((k_near_singular<T, D, ROWS, FORM, GEOM_SPHERE6>), g, b, 0, st, op, as); break;
        case GEOM_ELLIPSOID6:
            hipLaunchKernelGGL((k_near_singular<T, D, ROWS, FORM, GEOM_ELLIPSOID6>), g, b, 0, st, op, as);
            break;
        case GEOM_TORUS16: hipLaunchKernelGGL((k_near_singular<T, D, ROWS, FORM, GEOM_TORUS16>), g, b, 0, st, op, as); break;
        default: hipLaunchKernelGGL((k_near_singular<T, D, ROWS, FORM, -1>), g, b, 0, st, op, as); break;
    }
    hipLaunchKernelGGL((k_near_singular_add<T, D>), dim3((unsigned)as.ntouch_lp), dim3(128), 0, st, op, as);
}

hipError_t launch_near_singular(const OpDev& op, const AsmDev& as, hipStream_t st) {
    if (as.ntouch_lp == 0 || op.ntouch == 0) return hipSuccess;
    const int d = op.S.d;
    if (op.S.form == 0) {  // S^0 (degree >= 1)
        if (op.cplx) {
            if (d == 1) near_singular_geom<cdbl, 1, 4, 0>(op, as, st);
            else near_singular_geom<cdbl, 2, 5, 0>(op, as, st);
        } else {
            if (d == 1) near_singular_geom<double, 1, 4, 0>(op, as, st);
            else near_singular_geom<double, 2, 9, 0>(op, as, st);
        }
        return hipGetLastError();
    }
    if (op.cplx) {
        if (d == 0) near_singular_geom<cdbl, 0, 1, 2>(op, as, st);
        else if (d == 1) near_singular_geom<cdbl, 1, 4, 2>(op, as, st);
        else near_singular_geom<cdbl, 2, 5, 2>(op, as, st);
    } else {
        if (d == 0) near_singular_geom<double, 0, 1, 2>(op, as, st);
        else if (d == 1) near_singular_geom<double, 1, 4, 2>(op, as, st);
        else near_singular_geom<double, 2, 9, 2>(op, as, st);
    }
    return hipGetLastError();
}

hipError_t launch_near_gather(const OpDev& op, const AsmDev& as, hipStream_t st) {
    const dim3 g(nblk(op.S.ndof, 4)), b(256);
    if (op.cplx)
        hipLaunchKernelGGL(k_near_gather<cdbl>, g, b, 0, st, op, as);
    else
        hipLaunchKernelGGL(k_near_gather<double>, g, b, 0, st, op, as);
    return hipGetLastError();
}

hipError_t launch_far_assemble(const OpDev& op, const AsmDev& as, hipStream_t st) {
    const int64_t np = op.ncl * op.q2;
    hipLaunchKernelGGL(k_cluster_points, dim3(nblk(np, 256)), dim3(256), 0, st, op, as);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int64_t n = op.nstored * op.q2 * op.q2;
    if (n == 0 || op.otf) return hipSuccess;
    if (op.cplx)
        hipLaunchKernelGGL(k_far_assemble<cdbl>, dim3(nblk(n, 256)), dim3(256), 0, st, op, as);
    else
        hipLaunchKernelGGL(k_far_assemble<double>, dim3(nblk(n, 256)), dim3(256), 0, st, op, as);
    return hipGetLastError();
}

template <class T, int Q>
static hipError_t apply_stage_tq(const OpDev& op, int stage, const T* x, T* y, bool with_near, int prec,
                                 hipStream_t st) {
    switch (stage) {
        case 0: {
            const unsigned nup = (unsigned)op.S.geom.npatch << (2 * op.up_root);
            const unsigned nb = nup + (with_near ? nblk(op.ngroups, 4) : 0u);
            hipLaunchKernelGGL((k_near_up<T, Q>), dim3(nb), dim3(256), 0, st, op, x, y);
            if (op.up_root > 0 && !op.up_count)
                hipLaunchKernelGGL((k_up_top<T, Q>), dim3((unsigned)op.S.geom.npatch), dim3(256), 0, st, op);
            break;
        }
        case 1: {
            if (op.nchunks == 0) break;
            const dim3 g(nblk(op.nchunks, 4)), b(256);
            using F = typename std::conditional<std::is_same<T, double>::value, float, cflt>::type;
            if (op.otf && op.otf_wide)
                hipLaunchKernelGGL((k_coupling_otf<T, Q, otf_ns<T>(true)>), g, b, 0, st, op);
            else if (op.otf)
                hipLaunchKernelGGL((k_coupling_otf<T, Q, otf_ns<T>(false)>), g, b, 0, st, op);
            else if (prec == 0)
                hipLaunchKernelGGL((k_coupling<T, Q>), g, b, 0, st, op);
            else if (op.low == 1)
                hipLaunchKernelGGL((k_coupling_low<T, F, StFp32, Q>), g, b, 0, st, op);
            else
                hipLaunchKernelGGL((k_coupling_low<T, F, StBf16, Q>), g, b, 0, st, op);
            break;
        }
        case 2:
            if (op.nstored > 0) hipLaunchKernelGGL((k_lv_gather<T, Q>), dim3(nblk(op.ncl, 4)), dim3(256), 0, st, op);
            break;
        default:
            if (op.nstored > 0) {
                const int nt = op.nleaf1 / op.tile;
                hipLaunchKernelGGL((k_down_back<T, Q>), dim3((unsigned)(op.S.geom.npatch * nt * nt)), dim3(256), 0, st,
                                   op, y);
            }
            break;
    }
    return hipGetLastError();
}

template <class T>
static hipError_t apply_stage_t(const OpDev& op, int stage, const T* x, T* y, bool with_near, int prec,
                                hipStream_t st) {
    switch (op.q) {
        case 1: return apply_stage_tq<T, 1>(op, stage, x, y, with_near, prec, st);
        case 2: return apply_stage_tq<T, 2>(op, stage, x, y, with_near, prec, st);
        case 3: return apply_stage_tq<T, 3>(op, stage, x, y, with_near, prec, st);
        case 4: return apply_stage_tq<T, 4>(op, stage, x, y, with_near, prec, st);
        case 5: return apply_stage_tq<T, 5>(op, stage, x, y, with_near, prec, st);
        case 6: return apply_stage_tq<T, 6>(op, stage, x, y, with_near, prec, st);
        case 7: return apply_stage_tq<T, 7>(op, stage, x, y, with_near, prec, st);
        default: return apply_stage_tq<T, 8>(op, stage, x, y, with_near, prec, st);
    }
}

hipError_t launch_apply_stage(const OpDev& op, int stage, const void* x, void* y, int prec, hipStream_t st) {
    if (op.cplx) return apply_stage_t<cdbl>(op, stage, (const cdbl*)x, (cdbl*)y, true, prec, st);
    return apply_stage_t<double>(op, stage, (const double*)x, (double*)y, true, prec, st);
}

hipError_t launch_apply(const OpDev& op, const void* x, void* y, int prec, hipStream_t st) {
    for (int s = 0; s < kApplyStages; ++s) {
        hipError_t e = launch_apply_stage(op, s, x, y, prec, st);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_moments(const OpDev& op, const void* x, hipStream_t st) {
    if (op.cplx) return apply_stage_t<cdbl>(op, 0, (const cdbl*)x, nullptr, false, 0, st);
    return apply_stage_t<double>(op, 0, (const double*)x, nullptr, false, 0, st);
}

hipError_t launch_cast_low(const OpDev& op, hipStream_t st) {
    const int64_t n = (int64_t)op.nchunks > 0 ? (int64_t)op.ktotal_scalars : 0;
    if (n == 0 || op.low == 0) return hipSuccess;
    hipLaunchKernelGGL(k_cast_low, dim3(nblk(n, 256)), dim3(256), 0, st, n, (const double*)op.K, op.Klow, op.low);
    return hipGetLastError();
}

// blocks of each grouped stage for one operator (the one-column launch shapes)
void group_stage_blocks(const OpDev& op, int ncols, int64_t out[kGroupStages]) {
    const int64_t nc = op.nchunks > 0 ? (op.nchunks + 3) / 4 : 0;
    const int64_t nt = op.nleaf1 / op.tile;
    out[0] = ((int64_t)op.S.geom.npatch << (2 * op.up_root)) + (op.ngroups + 3) / 4;
    out[1] = op.up_root > 0 ? op.S.geom.npatch : 0;
    out[2] = op.otf ? 0 : nc;
    out[5] = op.otf ? nc : 0;
    out[3] = op.nstored > 0 ? (op.ncl + 3) / 4 : 0;
    out[4] = op.nstored > 0 ? (int64_t)op.S.geom.npatch * nt * nt : 0;
    for (int s = 0; s < kGroupStages; ++s) out[s] *= ncols;
}

hipError_t launch_group_apply(const GroupDev& g, int cplx, int q, hipStream_t st) {
    if (g.napply <= 0) return hipSuccess;
    return cplx ? group_t<cdbl>(g, q, st) : group_t<double>(g, q, st);
}

hipError_t launch_rhs(const SpaceDesc& S, const BasisTab& bt, const Gauss8& g8, int kind, const double* prm,
                      void* b, hipStream_t st) {
    const dim3 g(nblk(S.nglob, 4)), blk(256);
    if (S.ker.pde == PDE_HELMHOLTZ)
        hipLaunchKernelGGL(k_rhs<cdbl>, g, blk, 0, st, S, bt, g8, kind, prm[0], prm[1], prm[2], (cdbl*)b);
    else
        hipLaunchKernelGGL(k_rhs<double>, g, blk, 0, st, S, bt, g8, kind, prm[0], prm[1], prm[2], (double*)b);
    return hipGetLastError();
}

hipError_t launch_quadpoints(const SpaceDesc& S, const Gauss8& g8, double* xyz, hipStream_t st) {
    const int64_t n = S.nelem * 64;
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_quadpoints, dim3(nblk(n, 256)), dim3(256), 0, st, S, g8, xyz);
    return hipGetLastError();
}

hipError_t launch_rhs_samples(const SpaceDesc& S, const BasisTab& bt, const Gauss8& g8, const void* gv, void* b,
                              hipStream_t st) {
    const dim3 g(nblk(S.nglob, 4)), blk(256);
    if (S.ker.pde == PDE_HELMHOLTZ)
        hipLaunchKernelGGL(k_rhs_samples<cdbl>, g, blk, 0, st, S, bt, g8, (const cdbl*)gv, (cdbl*)b);
    else
        hipLaunchKernelGGL(k_rhs_samples<double>, g, blk, 0, st, S, bt, g8, (const double*)gv, (double*)b);
    return hipGetLastError();
}

hipError_t launch_potential_tree(const OpDev& op, const Gauss8& g8, double eta, const double* pts, int64_t npts,
                                 const void* rho, void* u, hipStream_t st) {
    if (npts == 0) return hipSuccess;
    const dim3 grid((unsigned)((npts + 3) / 4));
    if (op.cplx)
        hipLaunchKernelGGL(k_potential_tree<cdbl>, grid, dim3(256), 0, st, op, g8, eta, pts, npts, (const cdbl*)rho,
                           (cdbl*)u);
    else
        hipLaunchKernelGGL(k_potential_tree<double>, grid, dim3(256), 0, st, op, g8, eta, pts, npts,
                           (const double*)rho, (double*)u);
    return hipGetLastError();
}

hipError_t launch_potential(const SpaceDesc& S, const BasisTab& bt, const Gauss8& g8, const double* pts,
                            int64_t npts, const void* rho, void* u, hipStream_t st) {
    if (npts == 0) return hipSuccess;
    if (S.ker.pde == PDE_HELMHOLTZ)
        hipLaunchKernelGGL(k_potential<cdbl>, dim3((unsigned)npts), dim3(256), 0, st, S, bt, g8, pts, (const cdbl*)rho,
                           (cdbl*)u);
    else
        hipLaunchKernelGGL(k_potential<double>, dim3((unsigned)npts), dim3(256), 0, st, S, bt, g8, pts,
                           (const double*)rho, (double*)u);
    return hipGetLastError();
}

}  // namespace bem
