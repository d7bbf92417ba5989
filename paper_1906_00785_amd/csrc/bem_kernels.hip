// gfx950 kernels of the isogeometric Galerkin BEM hot path: near-field quadrature, coupling
// blocks, the H^2 matvec, load vector, potential and the GMRES vector operations.
#include "bem_kernels.h"

namespace bem {

namespace {

constexpr int kWave = 64;

__device__ inline int uniform_int(int v) { return __builtin_amdgcn_readfirstlane(v); }

__device__ inline void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ inline double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
    return v;
}
__device__ inline cdbl wave_sum(cdbl v) { return {wave_sum(v.re), wave_sum(v.im)}; }

// leaf-local index -> (patch, i, j)
__device__ inline void leaf_decode(int l, int n1, int& f, int& i, int& j) {
    j = l % n1;
    i = (l / n1) % n1;
    f = l / (n1 * n1);
}

// Duffy-type substitution of region `reg` for a touching pair of type `type` at the cube
// point (xi, e1, e2, e3): local points xh (first element) and yh (second element) with the
// Jacobian of the substitution.  Identical: 8 regions (4 sign patterns of y - x times the
// 2 simplices of (t1, t2)); edge (shared edge at first local coordinate 0 on both sides):
// 6 regions (sign of y2 - x2 times which of x1, y1, t is largest); vertex (shared vertex at
// the local origin on both sides): 4 regions (which of the 4 coordinates is largest).
__device__ inline void duffy_point(int type, int reg, double xi, double e1, double e2, double e3, double& x1,
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

// ------------------------------------------------------------------ geometry tables
__global__ void k_gauss_points(SpaceDesc S, int qg, const double* __restrict__ gx, double* __restrict__ gpos) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int qg2 = qg * qg;
    if (idx >= S.nelem * qg2) return;
    const int a = (int)(idx % qg2);
    const int64_t e = idx / qg2;
    const int i2 = (int)(e % S.nel), i1 = (int)((e / S.nel) % S.nel), f = (int)(e / ((int64_t)S.nel * S.nel));
    double x[3];
    patch_point(S.geom, f, (i1 + gx[a / qg]) * S.h, (i2 + gx[a % qg]) * S.h, x);
    gpos[3 * idx] = x[0];
    gpos[3 * idx + 1] = x[1];
    gpos[3 * idx + 2] = x[2];
}

// ------------------------------------------------------------------ near field: regular pairs
// One workgroup per near leaf pair (tau, sigma).  Wave w takes the tau-elements w, w+W, ...
// and integrates each against every sigma-element that does not touch it: lane a holds
// Gauss point a of the tau-element; the sigma-element's points, weights and 1-D basis
// values are wave-uniform (scalar loads).  Per lane the inner integral over sigma is
// accumulated in tensor form (first over b2, then b1); the outer sum over the lanes is a
// small LDS contraction.  Element-pair blocks are accumulated into the wave's own copy of
// the leaf-pair block (DOFs of tau x DOFs of sigma), the copies summed in a fixed order.
template <class T, int D>
__global__ __launch_bounds__(256) void k_near_regular(OpDev op, AsmDev as, int W, int lb_in_lds) {
    constexpr int D1 = D + 1, NB = D1 * D1;
    const SpaceDesc S = op.S;
    const int qg = op.qg, qg2 = qg * qg, m = op.m, m2 = m * m, nloc = op.nloc, nl2 = nloc * nloc;
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
    const double h2 = S.h * S.h, h4 = h2 * h2;
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
                const double* yp = as.gpos + e2 * qg2 * 3;
                const double* p1 = as.psi + (int64_t)fi1 * qg * D1;
                const double* p2 = as.psi + (int64_t)fi2 * qg * D1;
                for (int b1 = 0; b1 < qg; ++b1) {
                    T sacc[D1];
#pragma unroll
                    for (int l = 0; l < D1; ++l) sacc[l] = zero<T>();
                    for (int b2 = 0; b2 < qg; ++b2) {
                        const double* y = yp + (b1 * qg + b2) * 3;
                        const double dx = xa0 - y[0], dy = xa1 - y[1], dz = xa2 - y[2];
                        const T kv = kernel_val(kd, dx * dx + dy * dy + dz * dz, T());
                        const double wb = as.gw[b2];
#pragma unroll
                        for (int l = 0; l < D1; ++l) sacc[l] += kv * (wb * p2[b2 * D1 + l]);
                    }
                    const double wb = as.gw[b1];
#pragma unroll
                    for (int l1 = 0; l1 < D1; ++l1) {
                        const double c1 = wb * p1[b1 * D1 + l1];
#pragma unroll
                        for (int l2 = 0; l2 < D1; ++l2) acc[l1 * D1 + l2] += c1 * sacc[l2];
                    }
                }
#pragma unroll
                for (int j = 0; j < NB; ++j) myTB[lane * NB + j] = valid ? acc[j] : zero<T>();
                wave_sync();
                const double* q1 = as.psi + (int64_t)ei1 * qg * D1;
                const double* q2 = as.psi + (int64_t)ei2 * qg * D1;
                const int amax = min(kWave, qg2 - chunk);
                for (int t = lane; t < NB * NB; t += kWave) {
                    const int i = t / NB, j = t % NB, k1 = i / D1, k2 = i % D1;
                    T B = zero<T>();
                    for (int aa = 0; aa < amax; ++aa) {
                        const int ag = chunk + aa, a1 = ag / qg, a2 = ag % qg;
                        B += (as.gw[a1] * q1[a1 * D1 + k1] * as.gw[a2] * q2[a2 * D1 + k2]) * myTB[aa * NB + j];
                    }
                    const int r1 = (et / m) * S.r + k1, r2 = (et % m) * S.r + k2;
                    const int c1 = (es / m) * S.r + j / D1, c2 = (es % m) * S.r + j % D1;
                    myLB[(int64_t)(r1 * nloc + r2) * nl2 + c1 * nloc + c2] += B * h4;
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
// One workgroup per near leaf pair that contains touching element pairs; the pairs are
// integrated one after the other (all 256 threads share the Duffy cube points of a pair),
// each block reduced over the workgroup and added to the leaf-pair block in a fixed order.
// ROWS rows of the element-pair block are accumulated per pass to bound registers.
template <class T, int D, int ROWS>
__global__ __launch_bounds__(256) void k_near_singular(OpDev op, AsmDev as) {
    constexpr int D1 = D + 1, NB = D1 * D1;
    __shared__ T red[4][ROWS * NB];
    const SpaceDesc S = op.S;
    const BasisTab& bt = op.bt;
    const int m = op.m, nloc = op.nloc, nl2 = nloc * nloc, qs = op.qs, qs2 = qs * qs, qs4 = qs2 * qs2;
    const int64_t blk = (int64_t)nl2 * nl2;
    const int lp = as.touch_lp[blockIdx.x];
    int tf, ti, tj, sf, si, sj;
    leaf_decode(as.near_t[lp], op.nleaf1, tf, ti, tj);
    leaf_decode(as.near_s[lp], op.nleaf1, sf, si, sj);
    T* out = (T*)as.lb + (int64_t)lp * blk;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const KernelDesc kd = S.ker;
    const double h2 = S.h * S.h, h4 = h2 * h2;
    for (int tp = as.touch_rowptr[lp]; tp < as.touch_rowptr[lp + 1]; ++tp) {
        const int et = as.touch[5 * tp], es = as.touch[5 * tp + 1], type = as.touch[5 * tp + 2];
        const int k1 = as.touch[5 * tp + 3], k2 = as.touch[5 * tp + 4];
        const int ei1 = ti * m + et / m, ei2 = tj * m + et % m;
        const int fi1 = si * m + es / m, fi2 = sj * m + es % m;
        const int c1a = basis_class(bt, ei1), c1b = basis_class(bt, ei2);
        const int c2a = basis_class(bt, fi1), c2b = basis_class(bt, fi2);
        const int nreg = type == PT_IDENTICAL ? 8 : (type == PT_EDGE ? 6 : 4);
        const int npts = nreg * qs4;
#pragma unroll
        for (int r0 = 0; r0 < NB; r0 += ROWS) {
            T acc[ROWS * NB];
#pragma unroll
            for (int v = 0; v < ROWS * NB; ++v) acc[v] = zero<T>();
            for (int p = threadIdx.x; p < npts; p += blockDim.x) {
                const int reg = p / qs4;
                int rem = p - reg * qs4;
                const int i3 = rem % qs;
                rem /= qs;
                const int i2 = rem % qs;
                rem /= qs;
                const int i1 = rem % qs, i0 = rem / qs;
                double xh1, xh2, yh1, yh2, jac;
                duffy_point(type, reg, as.sx[i0], as.sx[i1], as.sx[i2], as.sx[i3], xh1, xh2, yh1, yh2, jac);
                const double wq = as.sw[i0] * as.sw[i1] * as.sw[i2] * as.sw[i3] * jac * h4;
                double u1, u2, w1, w2, X[3], Y[3];
                d4_apply(k1, xh1, xh2, u1, u2);
                d4_apply(k2, yh1, yh2, w1, w2);
                patch_point(S.geom, tf, (ei1 + u1) * S.h, (ei2 + u2) * S.h, X);
                patch_point(S.geom, sf, (fi1 + w1) * S.h, (fi2 + w2) * S.h, Y);
                double pa[D1], pb[D1], qa[D1], qb[D1];
#pragma unroll
                for (int l = 0; l < D1; ++l) {
                    pa[l] = basis_eval(bt, c1a, l, u1);
                    pb[l] = basis_eval(bt, c1b, l, u2);
                    qa[l] = basis_eval(bt, c2a, l, w1);
                    qb[l] = basis_eval(bt, c2b, l, w2);
                }
                const double dx = X[0] - Y[0], dy = X[1] - Y[1], dz = X[2] - Y[2];
                const T kv = kernel_val(kd, dx * dx + dy * dy + dz * dz, T()) * wq;
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
#pragma unroll
            for (int v = 0; v < ROWS * NB; ++v) {
                const T s = wave_sum(acc[v]);
                if (lane == 0) red[wave][v] = s;
            }
            __syncthreads();
            for (int t = threadIdx.x; t < ROWS * NB; t += blockDim.x) {
                const int i = r0 + t / NB, j = t % NB;
                if (i >= NB) continue;
                const T B = red[0][t] + red[1][t] + red[2][t] + red[3][t];
                const int r1 = (et / m) * S.r + i / D1, r2 = (et % m) * S.r + i % D1;
                const int cc1 = (es / m) * S.r + j / D1, cc2 = (es % m) * S.r + j % D1;
                out[(int64_t)(r1 * nloc + r2) * nl2 + cc1 * nloc + cc2] += B;
            }
            __syncthreads();
        }
    }
}

// ------------------------------------------------------------------ near field: CSR values
// One wave per row g; each lane sums, for its column h, the leaf-pair blocks of every near
// leaf pair (tau, sigma) with g in dofs(tau) and h in dofs(sigma), in a fixed order.
__device__ inline void leaf_range(int j, int stride, int nloc, int nleaf1, int& lo, int& hi) {
    hi = j / stride;
    if (hi > nleaf1 - 1) hi = nleaf1 - 1;
    const int l = j - nloc + 1;
    lo = l <= 0 ? 0 : (l + stride - 1) / stride;
}

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
    T* val = (T*)op.val;
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
    if (idx >= op.nfar * per) return;
    const int64_t blk = idx / per;
    const int rem = (int)(idx - blk * per), a = rem / q2, b = rem % q2;
    const int t = as.far_t[blk], s = op.far_s[blk];
    const int64_t slot = blk - op.far_rowptr[t];
    const double* x = as.xc + ((int64_t)t * q2 + a) * 3;
    const double* y = as.xc + ((int64_t)s * q2 + b) * 3;
    const double dx = x[0] - y[0], dy = x[1] - y[1], dz = x[2] - y[2];
    ((T*)op.K)[op.koff[t] + (int64_t)a * op.krs[t] + slot * q2 + b] = kernel_val(op.S.ker, dx * dx + dy * dy + dz * dz, T());
}

// ------------------------------------------------------------------ H^2 matvec
// forward transform: moments of every leaf, m[a1,a2] = sum V1_i[a1,m1] V1_j[a2,m2] x[...]
template <class T>
__global__ void k_forward(OpDev op, const T* __restrict__ x) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= op.nleaves * op.q2) return;
    const int a = (int)(idx % op.q2);
    const int l = (int)(idx / op.q2);
    const int q = op.q, nloc = op.nloc, stride = op.m * op.S.r;
    int f, i, j;
    leaf_decode(l, op.nleaf1, f, i, j);
    const int a1 = a / q, a2 = a % q;
    const double* Vi = op.V1 + ((int64_t)i * q + a1) * nloc;
    const double* Vj = op.V1 + ((int64_t)j * q + a2) * nloc;
    T acc = zero<T>();
    for (int m1 = 0; m1 < nloc; ++m1) {
        T in = zero<T>();
        const T* xr = x + dof_id(op.S, f, i * stride + m1, j * stride);
        for (int m2 = 0; m2 < nloc; ++m2) in += Vj[m2] * xr[m2];
        acc += Vi[m1] * in;
    }
    ((T*)op.mom)[(op.lev_off[op.leaf] + l) * op.q2 + a] = acc;
}

// upward transfer at level lev: m_P = sum_children (E_b1 (x) E_b2)^T m_child
template <class T>
__global__ void k_upward(OpDev op, int lev) {
    const int n = 1 << lev;
    const int64_t ncl = (int64_t)op.S.geom.npatch * n * n;
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= ncl * op.q2) return;
    const int q = op.q, q2 = op.q2;
    const int a = (int)(idx % q2);
    const int64_t loc = idx / q2;
    const int j = (int)(loc % n), i = (int)((loc / n) % n), f = (int)(loc / ((int64_t)n * n));
    const int a1 = a / q, a2 = a % q;
    const T* mom = (const T*)op.mom;
    T acc = zero<T>();
    for (int b1 = 0; b1 < 2; ++b1)
        for (int b2 = 0; b2 < 2; ++b2) {
            const int64_t c = op.lev_off[lev + 1] + ((int64_t)f * 2 * n + 2 * i + b1) * 2 * n + 2 * j + b2;
            const T* mc = mom + c * q2;
            for (int p1 = 0; p1 < q; ++p1) {
                T in = zero<T>();
                for (int p2 = 0; p2 < q; ++p2) in += op.E[(b2 * q + p2) * q + a2] * mc[p1 * q + p2];
                acc += op.E[(b1 * q + p1) * q + a1] * in;
            }
        }
    ((T*)op.mom)[(op.lev_off[lev] + loc) * q2 + a] = acc;
}

// coupling: lv_tau = sum over admissible sigma of K_tau,sigma m_sigma.  One wave per target;
// the target's coupling rows are stored contiguously (row a = all its blocks' row a), each
// lane streams columns k and keeps the Q*Q row sums, reduced across the wave at the end.
template <class T, int Q>
__global__ __launch_bounds__(256) void k_coupling(OpDev op) {
    constexpr int Q2 = Q * Q;
    const int64_t t = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (t >= op.ncl) return;
    const int64_t beg = op.far_rowptr[t], n = op.far_rowptr[t + 1] - beg;
    const int64_t rs = op.krs[t];
    const T* base = (const T*)op.K + op.koff[t];
    const T* mom = (const T*)op.mom;
    T acc[Q2];
#pragma unroll
    for (int a = 0; a < Q2; ++a) acc[a] = zero<T>();
    for (int64_t k = lane; k < n * Q2; k += kWave) {
        const int64_t s = k / Q2;
        const int b = (int)(k - s * Q2);
        const T mv = mom[(int64_t)op.far_s[beg + s] * Q2 + b];
#pragma unroll
        for (int a = 0; a < Q2; ++a) acc[a] += base[a * rs + k] * mv;
    }
    T* lv = (T*)op.lv + t * Q2;
#pragma unroll
    for (int a = 0; a < Q2; ++a) {
        const T s = wave_sum(acc[a]);
        if (lane == 0) lv[a] = s;
    }
}

// downward transfer at level lev >= 1: lv_c += (E_b1 (x) E_b2) lv_parent
template <class T>
__global__ void k_downward(OpDev op, int lev) {
    const int n = 1 << lev;
    const int64_t ncl = (int64_t)op.S.geom.npatch * n * n;
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= ncl * op.q2) return;
    const int q = op.q, q2 = op.q2;
    const int p = (int)(idx % q2);
    const int64_t loc = idx / q2;
    const int j = (int)(loc % n), i = (int)((loc / n) % n), f = (int)(loc / ((int64_t)n * n));
    const int p1 = p / q, p2 = p % q, b1 = i & 1, b2 = j & 1;
    const int64_t P = op.lev_off[lev - 1] + ((int64_t)f * (n / 2) + i / 2) * (n / 2) + j / 2;
    T* lv = (T*)op.lv;
    const T* lp = lv + P * q2;
    T acc = zero<T>();
    for (int a1 = 0; a1 < q; ++a1) {
        T in = zero<T>();
        for (int a2 = 0; a2 < q; ++a2) in += op.E[(b2 * q + p2) * q + a2] * lp[a1 * q + a2];
        acc += op.E[(b1 * q + p1) * q + a1] * in;
    }
    lv[(op.lev_off[lev] + loc) * q2 + p] += acc;
}

// backward transform plus near field: y_g = sum_tau (V_tau^T lv_tau)_g + sum_h A_near[g,h] x_h.
// One wave per row.
template <class T>
__global__ __launch_bounds__(256) void k_back_near(OpDev op, const T* __restrict__ x, T* __restrict__ y) {
    const SpaceDesc S = op.S;
    const int64_t g = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (g >= S.ndof) return;
    const T* val = (const T*)op.val;
    T acc = zero<T>();
    for (int64_t k = op.rowptr[g] + lane; k < op.rowptr[g + 1]; k += kWave) acc += val[k] * x[op.col[k]];
    const int nb = S.nb, n1 = op.nleaf1, nloc = op.nloc, stride = op.m * S.r, q = op.q, q2 = op.q2;
    const int j2 = (int)(g % nb), j1 = (int)((g / nb) % nb), f = (int)(g / ((int64_t)nb * nb));
    int lo1, hi1, lo2, hi2;
    leaf_range(j1, stride, nloc, n1, lo1, hi1);
    leaf_range(j2, stride, nloc, n1, lo2, hi2);
    const int nl_a = hi1 - lo1 + 1, nl_b = hi2 - lo2 + 1;
    const T* lv = (const T*)op.lv + op.lev_off[op.leaf] * q2;
    for (int t = lane; t < nl_a * nl_b * q2; t += kWave) {
        const int a = t % q2, lf = t / q2;
        const int li = lo1 + lf / nl_b, lj = lo2 + lf % nl_b;
        const int a1 = a / q, a2 = a % q;
        const double c = op.V1[((int64_t)li * q + a1) * nloc + (j1 - li * stride)] *
                         op.V1[((int64_t)lj * q + a2) * nloc + (j2 - lj * stride)];
        acc += c * lv[((int64_t)(f * n1 + li) * n1 + lj) * q2 + a];
    }
    const T s = wave_sum(acc);
    if (lane == 0) y[g] = s;
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

// b_g = sum over the elements of supp(g) of 8x8 Gauss sums of g(x) phi_g; one wave per DOF
template <class T>
__global__ __launch_bounds__(256) void k_rhs(SpaceDesc S, BasisTab bt, Gauss8 g8, int kind, double p0, double p1,
                                             double p2, T* b) {
    const int64_t g = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (g >= S.ndof) return;
    const int nb = S.nb, d = S.d, r = S.r;
    const int j2 = (int)(g % nb), j1 = (int)((g / nb) % nb), f = (int)(g / ((int64_t)nb * nb));
    const int a1 = lane >> 3, a2 = lane & 7;
    T acc = zero<T>();
    const int i1lo = j1 - d <= 0 ? 0 : (j1 - d + r - 1) / r, i1hi = min(j1 / r, S.nel - 1);
    const int i2lo = j2 - d <= 0 ? 0 : (j2 - d + r - 1) / r, i2hi = min(j2 / r, S.nel - 1);
    for (int i1 = i1lo; i1 <= i1hi; ++i1)
        for (int i2 = i2lo; i2 <= i2hi; ++i2) {
            const int l1 = j1 - i1 * r, l2 = j2 - i2 * r;
            if (l1 > d || l2 > d) continue;
            double x[3];
            patch_point(S.geom, f, (i1 + g8.x[a1]) * S.h, (i2 + g8.x[a2]) * S.h, x);
            const double phi = basis_eval(bt, basis_class(bt, i1), l1, g8.x[a1]) *
                               basis_eval(bt, basis_class(bt, i2), l2, g8.x[a2]);
            acc += data_value<T>(kind, S.ker, p0, p1, p2, x) * (g8.w[a1] * g8.w[a2] * S.h * S.h * phi);
        }
    const T s = wave_sum(acc);
    if (lane == 0) b[g] = s;
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
                rh += (ba * basis_eval(bt, cb, l2, u2)) * rho[dof_id(S, f, i1 * r + l1, i2 * r + l2)];
        }
        const double dx = px - y[0], dy = py - y[1], dz = pz - y[2];
        acc += kernel_val(S.ker, dx * dx + dy * dy + dz * dz, T()) * rh * (g8.w[a >> 3] * g8.w[a & 7] * S.h * S.h);
    }
    acc = wave_sum(acc);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) u[p] = red[0] + red[1] + red[2] + red[3];
}

// ------------------------------------------------------------------ GMRES vector operations
// partial[blk][i] = sum over the block's slice of conj(V_i) w, 8 vectors per pass
template <class T>
__global__ __launch_bounds__(256) void k_dots(int64_t n, int k, const T* __restrict__ V, int64_t ldv,
                                              const T* __restrict__ w, T* partial) {
    __shared__ T red[4][8];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    for (int i0 = 0; i0 < k; i0 += 8) {
        T acc[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) acc[u] = zero<T>();
        for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x) {
            const T wv = w[t];
#pragma unroll
            for (int u = 0; u < 8; ++u)
                if (i0 + u < k) acc[u] += conj_(V[(int64_t)(i0 + u) * ldv + t]) * wv;
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const T s = wave_sum(acc[u]);
            if (lane == 0) red[wave][u] = s;
        }
        __syncthreads();
        if (threadIdx.x < 8 && i0 + (int)threadIdx.x < k) {
            const int u = threadIdx.x;
            partial[(int64_t)blockIdx.x * k + i0 + u] = red[0][u] + red[1][u] + red[2][u] + red[3][u];
        }
        __syncthreads();
    }
}

template <class T>
__global__ void k_reduce_partials(int k, int nblocks, const T* partial, T* out) {
    for (int i = threadIdx.x; i < k; i += blockDim.x) {
        T s = zero<T>();
        for (int b = 0; b < nblocks; ++b) s += partial[(int64_t)b * k + i];
        out[i] = s;
    }
}

template <class T>
__global__ void k_update(int64_t n, int k, const T* __restrict__ V, int64_t ldv, const T* __restrict__ c, double alpha,
                         T* w) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    T s = zero<T>();
    for (int i = 0; i < k; ++i) s += c[i] * V[(int64_t)i * ldv + t];
    w[t] += alpha * s;
}

template <class T>
__global__ __launch_bounds__(256) void k_norm_partial(int64_t n, const T* __restrict__ w, double* partial) {
    __shared__ double red[4];
    double acc = 0.0;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x)
        acc += abs2(w[t]);
    acc = wave_sum(acc);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) partial[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

__global__ void k_norm_final(int nblocks, const double* partial, double* out) {
    if (threadIdx.x != 0) return;
    double s = 0.0;
    for (int b = 0; b < nblocks; ++b) s += partial[b];
    *out = sqrt(s);
}

template <class T>
__global__ void k_scale(int64_t n, const T* __restrict__ w, const double* nrm, T* v) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    v[t] = w[t] * (1.0 / *nrm);
}

template <class T>
__global__ void k_axpby(int64_t n, double a, const T* __restrict__ x, double b, T* y) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    y[t] = a * x[t] + b * y[t];
}

inline unsigned nblk(int64_t n, int per) { return (unsigned)((n + per - 1) / per); }

}  // namespace

// =========================================================================== launchers
hipError_t launch_gauss_points(const OpDev& op, const AsmDev& as, hipStream_t st) {
    const int64_t n = op.S.nelem * op.qg * op.qg;
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_gauss_points, dim3(nblk(n, 256)), dim3(256), 0, st, op.S, op.qg, as.gx, (double*)as.gpos);
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
    if (shm > 64 * 1024) {
        hipError_t e = hipFuncSetAttribute((const void*)k_near_regular<T, D>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL((k_near_regular<T, D>), dim3((unsigned)op.nnear), dim3(64 * W), shm, st, op, as, W, in_lds);
    return hipGetLastError();
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

hipError_t launch_near_singular(const OpDev& op, const AsmDev& as, hipStream_t st) {
    if (as.ntouch_lp == 0) return hipSuccess;
    const dim3 g((unsigned)as.ntouch_lp), b(256);
    const int d = op.S.d;
    if (op.cplx) {
        if (d == 0) hipLaunchKernelGGL((k_near_singular<cdbl, 0, 1>), g, b, 0, st, op, as);
        else if (d == 1) hipLaunchKernelGGL((k_near_singular<cdbl, 1, 4>), g, b, 0, st, op, as);
        else hipLaunchKernelGGL((k_near_singular<cdbl, 2, 5>), g, b, 0, st, op, as);
    } else {
        if (d == 0) hipLaunchKernelGGL((k_near_singular<double, 0, 1>), g, b, 0, st, op, as);
        else if (d == 1) hipLaunchKernelGGL((k_near_singular<double, 1, 4>), g, b, 0, st, op, as);
        else hipLaunchKernelGGL((k_near_singular<double, 2, 9>), g, b, 0, st, op, as);
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
    if (e != hipSuccess || op.nfar == 0) return e;
    const int64_t n = op.nfar * op.q2 * op.q2;
    if (op.cplx)
        hipLaunchKernelGGL(k_far_assemble<cdbl>, dim3(nblk(n, 256)), dim3(256), 0, st, op, as);
    else
        hipLaunchKernelGGL(k_far_assemble<double>, dim3(nblk(n, 256)), dim3(256), 0, st, op, as);
    return hipGetLastError();
}

template <class T>
static hipError_t moments_t(const OpDev& op, const T* x, hipStream_t st) {
    const int64_t n = op.nleaves * op.q2;
    hipLaunchKernelGGL(k_forward<T>, dim3(nblk(n, 256)), dim3(256), 0, st, op, x);
    for (int lev = op.leaf - 1; lev >= 0; --lev) {
        const int64_t nc = (int64_t)op.S.geom.npatch * (1LL << (2 * lev)) * op.q2;
        hipLaunchKernelGGL(k_upward<T>, dim3(nblk(nc, 256)), dim3(256), 0, st, op, lev);
    }
    return hipGetLastError();
}

template <class T>
static hipError_t coupling_t(const OpDev& op, hipStream_t st) {
    const dim3 g(nblk(op.ncl, 4)), b(256);
    switch (op.q) {
        case 1: hipLaunchKernelGGL((k_coupling<T, 1>), g, b, 0, st, op); break;
        case 2: hipLaunchKernelGGL((k_coupling<T, 2>), g, b, 0, st, op); break;
        case 3: hipLaunchKernelGGL((k_coupling<T, 3>), g, b, 0, st, op); break;
        case 4: hipLaunchKernelGGL((k_coupling<T, 4>), g, b, 0, st, op); break;
        case 5: hipLaunchKernelGGL((k_coupling<T, 5>), g, b, 0, st, op); break;
        case 6: hipLaunchKernelGGL((k_coupling<T, 6>), g, b, 0, st, op); break;
        case 7: hipLaunchKernelGGL((k_coupling<T, 7>), g, b, 0, st, op); break;
        default: hipLaunchKernelGGL((k_coupling<T, 8>), g, b, 0, st, op); break;
    }
    return hipGetLastError();
}

template <class T>
static hipError_t apply_stage_t(const OpDev& op, int stage, const T* x, T* y, hipStream_t st) {
    switch (stage) {
        case 0:
            return moments_t<T>(op, x, st);
        case 1:
            return coupling_t<T>(op, st);
        case 2:
            for (int lev = 1; lev <= op.leaf; ++lev) {
                const int64_t nc = (int64_t)op.S.geom.npatch * (1LL << (2 * lev)) * op.q2;
                hipLaunchKernelGGL(k_downward<T>, dim3(nblk(nc, 256)), dim3(256), 0, st, op, lev);
            }
            return hipGetLastError();
        default:
            hipLaunchKernelGGL(k_back_near<T>, dim3(nblk(op.S.ndof, 4)), dim3(256), 0, st, op, x, y);
            return hipGetLastError();
    }
}

hipError_t launch_apply_stage(const OpDev& op, int stage, const void* x, void* y, hipStream_t st) {
    if (op.cplx) return apply_stage_t<cdbl>(op, stage, (const cdbl*)x, (cdbl*)y, st);
    return apply_stage_t<double>(op, stage, (const double*)x, (double*)y, st);
}

hipError_t launch_apply(const OpDev& op, const void* x, void* y, hipStream_t st) {
    for (int s = 0; s < kApplyStages; ++s) {
        hipError_t e = launch_apply_stage(op, s, x, y, st);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_moments(const OpDev& op, const void* x, hipStream_t st) {
    if (op.cplx) return moments_t<cdbl>(op, (const cdbl*)x, st);
    return moments_t<double>(op, (const double*)x, st);
}

hipError_t launch_rhs(const SpaceDesc& S, const BasisTab& bt, const Gauss8& g8, int kind, const double* prm,
                      void* b, hipStream_t st) {
    const dim3 g(nblk(S.ndof, 4)), blk(256);
    if (S.ker.pde == PDE_HELMHOLTZ)
        hipLaunchKernelGGL(k_rhs<cdbl>, g, blk, 0, st, S, bt, g8, kind, prm[0], prm[1], prm[2], (cdbl*)b);
    else
        hipLaunchKernelGGL(k_rhs<double>, g, blk, 0, st, S, bt, g8, kind, prm[0], prm[1], prm[2], (double*)b);
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

hipError_t launch_dots(int cplx, int64_t n, int k, const void* V, int64_t ldv, const void* w, void* partial,
                       void* out, hipStream_t st) {
    if (cplx) {
        hipLaunchKernelGGL(k_dots<cdbl>, dim3(kDotBlocks), dim3(256), 0, st, n, k, (const cdbl*)V, ldv,
                           (const cdbl*)w, (cdbl*)partial);
        hipLaunchKernelGGL(k_reduce_partials<cdbl>, dim3(1), dim3(64), 0, st, k, kDotBlocks, (const cdbl*)partial,
                           (cdbl*)out);
    } else {
        hipLaunchKernelGGL(k_dots<double>, dim3(kDotBlocks), dim3(256), 0, st, n, k, (const double*)V, ldv,
                           (const double*)w, (double*)partial);
        hipLaunchKernelGGL(k_reduce_partials<double>, dim3(1), dim3(64), 0, st, k, kDotBlocks,
                           (const double*)partial, (double*)out);
    }
    return hipGetLastError();
}

hipError_t launch_update(int cplx, int64_t n, int k, const void* V, int64_t ldv, const void* c, double alpha,
                         void* w, hipStream_t st) {
    if (cplx)
        hipLaunchKernelGGL(k_update<cdbl>, dim3(nblk(n, 256)), dim3(256), 0, st, n, k, (const cdbl*)V, ldv,
                           (const cdbl*)c, alpha, (cdbl*)w);
    else
        hipLaunchKernelGGL(k_update<double>, dim3(nblk(n, 256)), dim3(256), 0, st, n, k, (const double*)V, ldv,
                           (const double*)c, alpha, (double*)w);
    return hipGetLastError();
}

hipError_t launch_norm(int cplx, int64_t n, const void* w, void* partial, double* out, hipStream_t st) {
    if (cplx)
        hipLaunchKernelGGL(k_norm_partial<cdbl>, dim3(kDotBlocks), dim3(256), 0, st, n, (const cdbl*)w,
                           (double*)partial);
    else
        hipLaunchKernelGGL(k_norm_partial<double>, dim3(kDotBlocks), dim3(256), 0, st, n, (const double*)w,
                           (double*)partial);
    hipLaunchKernelGGL(k_norm_final, dim3(1), dim3(64), 0, st, kDotBlocks, (const double*)partial, out);
    return hipGetLastError();
}

hipError_t launch_scale(int cplx, int64_t n, const void* w, const double* nrm, void* v, hipStream_t st) {
    if (cplx)
        hipLaunchKernelGGL(k_scale<cdbl>, dim3(nblk(n, 256)), dim3(256), 0, st, n, (const cdbl*)w, nrm, (cdbl*)v);
    else
        hipLaunchKernelGGL(k_scale<double>, dim3(nblk(n, 256)), dim3(256), 0, st, n, (const double*)w, nrm,
                           (double*)v);
    return hipGetLastError();
}

hipError_t launch_axpby(int cplx, int64_t n, double a, const void* x, double b, void* y, hipStream_t st) {
    if (cplx)
        hipLaunchKernelGGL(k_axpby<cdbl>, dim3(nblk(n, 256)), dim3(256), 0, st, n, a, (const cdbl*)x, b, (cdbl*)y);
    else
        hipLaunchKernelGGL(k_axpby<double>, dim3(nblk(n, 256)), dim3(256), 0, st, n, a, (const double*)x, b,
                           (double*)y);
    return hipGetLastError();
}

}  // namespace bem
