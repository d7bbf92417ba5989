// GMRES(m) for R right-hand sides in lockstep (Sec. 4 "Solution of the System of Linear
// Equations", one Krylov space per right-hand side).  Every vector is a slab v[g][r]; a
// wave handles rows of one slice for 64 consecutive right-hand sides (one per lane), so
// each right-hand side keeps its own inner products, Hessenberg matrix, Givens rotations
// and step count.  Reductions go through per-slice partials that a separate kernel sums in
// a fixed order (deterministic).
#include "bem_solve.h"

namespace bem {

namespace {

constexpr int kT = 256;
constexpr int kC = 64;  // right-hand sides per wave
constexpr int kJT = 4;  // inner products per block of the dots kernel
constexpr int kGivensThreads = 16;  // right-hand sides per block of the rotation kernel (LDS)

__device__ inline double absval(double v) { return fabs(v); }
__device__ inline double absval(cdbl v) { return sqrt(v.re * v.re + v.im * v.im); }
__device__ inline double div_(double a, double b) { return a / b; }
__device__ inline cdbl div_(cdbl a, cdbl b) {
    const double d = b.re * b.re + b.im * b.im;
    return {(a.re * b.re + a.im * b.im) / d, (a.im * b.re - a.re * b.im) / d};
}
__device__ inline double from_real(double v, double) { return v; }
__device__ inline cdbl from_real(double v, cdbl) { return {v, 0.0}; }

// rows [t0, t1) of slice blockIdx.x (of gridDim.x)
__device__ inline void bslice(int64_t n, int64_t& t0, int64_t& t1) {
    const int64_t len = (n + gridDim.x - 1) / gridDim.x;
    t0 = (int64_t)blockIdx.x * len;
    t1 = t0 + len < n ? t0 + len : n;
}

// part[s][j][r] = sum over the rows of slice s of conj(V_j[g][r]) w[g][r], for the kJT
// values of j of this block (blockIdx.z); the four waves take every fourth row
template <class T>
__global__ __launch_bounds__(kT) void kbs_dots(int64_t n, int R, int k, const T* __restrict__ V,
                                               const T* __restrict__ w, T* __restrict__ part) {
    __shared__ T red[4][kJT][kC];
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int r = blockIdx.y * kC + lane;
    const int j0 = blockIdx.z * kJT;
    int64_t t0, t1;
    bslice(n, t0, t1);
    T acc[kJT];
#pragma unroll
    for (int u = 0; u < kJT; ++u) acc[u] = zero<T>();
    if (r < R) {
        const int64_t slab = n * R;
        for (int64_t t = t0 + wv; t < t1; t += 4) {
            const T x = w[t * R + r];
#pragma unroll
            for (int u = 0; u < kJT; ++u)
                if (j0 + u < k) acc[u] += conj_(V[(int64_t)(j0 + u) * slab + t * R + r]) * x;
        }
    }
#pragma unroll
    for (int u = 0; u < kJT; ++u) red[wv][u][lane] = acc[u];
    __syncthreads();
    if (wv == 0 && r < R) {
#pragma unroll
        for (int u = 0; u < kJT; ++u)
            if (j0 + u < k)
                part[((int64_t)blockIdx.x * k + j0 + u) * R + r] =
                    ((red[0][u][lane] + red[1][u][lane]) + red[2][u][lane]) + red[3][u][lane];
    }
}

// h[j][r] = sum over slices of part[s][j][r] (slices in order)
template <class T>
__global__ __launch_bounds__(kT) void kbs_reduce(int S, int R, int k, const T* __restrict__ part, T* __restrict__ h) {
    const int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (i >= (int64_t)k * R) return;
    // eight interleaved partial sums (independent loads in flight), added in a fixed order
    T s8[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) s8[u] = zero<T>();
    int b = 0;
    for (; b + 8 <= S; b += 8)
#pragma unroll
        for (int u = 0; u < 8; ++u) s8[u] += part[(int64_t)(b + u) * k * R + i];
    for (; b < S; ++b) s8[0] += part[(int64_t)b * k * R + i];
    h[i] = ((s8[0] + s8[1]) + (s8[2] + s8[3])) + ((s8[4] + s8[5]) + (s8[6] + s8[7]));
}

// w[g][r] -= sum_{j<k} V_j[g][r] h[j][r] over the slice; with norm != 0 also the partial
// squared norms npart[s][r] of the updated rows
template <class T>
__global__ __launch_bounds__(kT) void kbs_update(int64_t n, int R, int k, const T* __restrict__ V,
                                                 const T* __restrict__ h, T* w, double* __restrict__ npart, int norm) {
    __shared__ T hs[kMaxRestart + 1][kC];
    __shared__ double red[4][kC];
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int r = blockIdx.y * kC + lane;
    for (int i = threadIdx.x; i < k * kC; i += kT) {
        const int j = i / kC, l = i % kC, rr = blockIdx.y * kC + l;
        hs[j][l] = rr < R ? h[(int64_t)j * R + rr] : zero<T>();
    }
    __syncthreads();
    int64_t t0, t1;
    bslice(n, t0, t1);
    double acc = 0.0;
    if (r < R) {
        const int64_t slab = n * R;
        for (int64_t t = t0 + wv; t < t1; t += 4) {
            T s = zero<T>();
            for (int j = 0; j < k; ++j) s += hs[j][lane] * V[(int64_t)j * slab + t * R + r];
            const T x = w[t * R + r] - s;
            w[t * R + r] = x;
            acc += abs2(x);
        }
    }
    if (!norm) return;
    red[wv][lane] = acc;
    __syncthreads();
    if (wv == 0 && r < R) npart[(int64_t)blockIdx.x * R + r] = ((red[0][lane] + red[1][lane]) + red[2][lane]) + red[3][lane];
}

// w = b - w (or w = b) and the partial squared norms
template <class T>
__global__ __launch_bounds__(kT) void kbs_residual(int64_t n, int R, const T* __restrict__ b, T* w,
                                                   double* __restrict__ npart, int copy_b) {
    __shared__ double red[4][kC];
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int r = blockIdx.y * kC + lane;
    int64_t t0, t1;
    bslice(n, t0, t1);
    double acc = 0.0;
    if (r < R)
        for (int64_t t = t0 + wv; t < t1; t += 4) {
            const T x = copy_b ? b[t * R + r] : b[t * R + r] - w[t * R + r];
            w[t * R + r] = x;
            acc += abs2(x);
        }
    red[wv][lane] = acc;
    __syncthreads();
    if (wv == 0 && r < R) npart[(int64_t)blockIdx.x * R + r] = ((red[0][lane] + red[1][lane]) + red[2][lane]) + red[3][lane];
}

__device__ inline double norm_of(const double* npart, int S, int R, int r) {
    double s8[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    int b = 0;
    for (; b + 8 <= S; b += 8)
#pragma unroll
        for (int u = 0; u < 8; ++u) s8[u] += npart[(int64_t)(b + u) * R + r];
    for (; b < S; ++b) s8[0] += npart[(int64_t)b * R + r];
    return sqrt(((s8[0] + s8[1]) + (s8[2] + s8[3])) + ((s8[4] + s8[5]) + (s8[6] + s8[7])));
}

// per right-hand side: beta = ||w||, g = beta e_1, sc = 1/beta (0 if beta = 0)
template <class T>
__global__ void kbs_start(int S, int R, int m, const double* __restrict__ npart, BGmresState st) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= R) return;
    const double beta = norm_of(npart, S, R, r);
    T* g = (T*)st.g + (int64_t)r * (m + 1);
    for (int i = 0; i <= m; ++i) g[i] = i == 0 ? from_real(beta, T()) : zero<T>();
    st.beta[r] = beta;
    st.sc[r] = beta > 0.0 ? 1.0 / beta : 0.0;
}

// v[g][r] = w[g][r] * sc[r]
template <class T>
__global__ __launch_bounds__(kT) void kbs_scale(int64_t n, int R, const T* __restrict__ w, const double* __restrict__ sc,
                                                T* __restrict__ v) {
    const int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (i >= n * R) return;
    v[i] = w[i] * sc[i % R];
}

// Hessenberg column j of every right-hand side: h1 + h2 above the diagonal, ||w|| below,
// the previous rotations, a new rotation, the rotated right-hand side g, the residual
// estimate est[j][r] = |g_{j+1}| and the scale 1/||w|| of the next basis vector
template <class T>
__global__ __launch_bounds__(kGivensThreads) void kbs_givens(int S, int R, int m, int j, const double* __restrict__ npart,
                                                           const T* __restrict__ h1, const T* __restrict__ h2,
                                                           BGmresState st) {
    // the new column and the previous rotations of each right-hand side staged in LDS
    // (one column of kGivensThreads right-hand sides per block), then the serial rotation
    // chain on LDS
    __shared__ T col[kMaxRestart + 1][kGivensThreads];
    __shared__ T snl[kMaxRestart][kGivensThreads];
    __shared__ double csl[kMaxRestart][kGivensThreads];
    const int tl = threadIdx.x;
    const int r = blockIdx.x * kGivensThreads + tl;
    if (r >= R) return;
    const double nrm = norm_of(npart, S, R, r);
    T* H = (T*)st.H + (int64_t)r * (m + 1) * m;
    double* cs = st.cs + (int64_t)r * m;
    T* sn = (T*)st.sn + (int64_t)r * m;
    T* g = (T*)st.g + (int64_t)r * (m + 1);
    for (int i = 0; i <= j; ++i) col[i][tl] = h1[(int64_t)i * R + r] + h2[(int64_t)i * R + r];
    for (int i = 0; i < j; ++i) {
        csl[i][tl] = cs[i];
        snl[i][tl] = sn[i];
    }
    col[j + 1][tl] = from_real(nrm, T());
    for (int i = 0; i < j; ++i) {
        const T a = col[i][tl], c = col[i + 1][tl];
        col[i][tl] = csl[i][tl] * a + snl[i][tl] * c;
        col[i + 1][tl] = csl[i][tl] * c - conj_(snl[i][tl]) * a;
    }
    const T a = col[j][tl], c = col[j + 1][tl];
    const double na = absval(a), nc = absval(c), nu = sqrt(na * na + nc * nc);
    double cj;
    T sj;
    if (na == 0.0) {
        cj = 0.0;
        sj = from_real(1.0, T());
    } else {
        cj = na / nu;
        sj = (a * (1.0 / na)) * conj_(c) * (1.0 / nu);
    }
    cs[j] = cj;
    sn[j] = sj;
    col[j][tl] = cj * a + sj * c;
    for (int i = 0; i <= j; ++i) H[i * m + j] = col[i][tl];
    H[(j + 1) * m + j] = zero<T>();
    const T gj = g[j];
    g[j] = cj * gj;
    g[j + 1] = zero<T>() - conj_(sj) * gj;
    st.est[(int64_t)j * R + r] = absval(g[j + 1]);
    st.sc[r] = nrm > 0.0 ? 1.0 / nrm : 0.0;
}

// y = H_k^{-1} g_k with k = kr[r] steps of right-hand side r (0: no update)
template <class T>
__global__ void kbs_backsolve(int R, int m, BGmresState st) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= R) return;
    const int k = st.kr[r];
    const T* H = (const T*)st.H + (int64_t)r * (m + 1) * m;
    const T* g = (const T*)st.g + (int64_t)r * (m + 1);
    T* y = (T*)st.y;
    for (int i = m - 1; i >= k; --i) y[(int64_t)i * R + r] = zero<T>();
    for (int i = k - 1; i >= 0; --i) {
        T s = g[i];
        for (int l = i + 1; l < k; ++l) s -= H[i * m + l] * y[(int64_t)l * R + r];
        y[(int64_t)i * R + r] = div_(s, H[i * m + i]);
    }
}

// x[g][r] += sum_{j<k} y[j][r] V_j[g][r]  (y is zero beyond each right-hand side's steps)
template <class T>
__global__ __launch_bounds__(kT) void kbs_xupdate(int64_t n, int R, int k, const T* __restrict__ V,
                                                  const T* __restrict__ y, T* x) {
    __shared__ T ys[kMaxRestart][kC];
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int r = blockIdx.y * kC + lane;
    for (int i = threadIdx.x; i < k * kC; i += kT) {
        const int j = i / kC, l = i % kC, rr = blockIdx.y * kC + l;
        ys[j][l] = rr < R ? y[(int64_t)j * R + rr] : zero<T>();
    }
    __syncthreads();
    if (r >= R) return;
    int64_t t0, t1;
    bslice(n, t0, t1);
    const int64_t slab = n * R;
    for (int64_t t = t0 + wv; t < t1; t += 4) {
        T s = zero<T>();
        for (int j = 0; j < k; ++j) s += ys[j][lane] * V[(int64_t)j * slab + t * R + r];
        x[t * R + r] += s;
    }
}

// U[g][r] = u[g][r] / ||u_r||, D[g][r] = d[g][r] / ||u_r|| (zero if ||u_r|| = 0)
template <class T>
__global__ __launch_bounds__(kT) void kbs_scale2(int64_t n, int R, const double* __restrict__ npart,
                                                 const T* __restrict__ u, const T* __restrict__ d, T* __restrict__ U,
                                                 T* __restrict__ D) {
    __shared__ double inv[kC];
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int r = blockIdx.y * kC + lane;
    if (wv == 0) {
        const double nrm = r < R ? norm_of(npart, kBSolveSlices, R, r) : 0.0;
        inv[lane] = nrm > 0.0 ? 1.0 / nrm : 0.0;
    }
    __syncthreads();
    if (r >= R) return;
    int64_t t0, t1;
    bslice(n, t0, t1);
    const double s = inv[lane];
    for (int64_t t = t0 + wv; t < t1; t += 4) {
        U[t * R + r] = u[t * R + r] * s;
        D[t * R + r] = d[t * R + r] * s;
    }
}

// y += x, and columns whose flag is set are cleared in y (mask != nullptr)
template <class T>
__global__ __launch_bounds__(kT) void kbs_axpy(int64_t n, int R, const T* __restrict__ x, T* y) {
    const int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (i < n * R) y[i] += x[i];
}
template <class T>
__global__ __launch_bounds__(kT) void kbs_mask(int64_t n, int R, const int* __restrict__ flag, T* y) {
    const int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (i < n * R && flag[i % R]) y[i] = zero<T>();
}
template <class T>
__global__ __launch_bounds__(kT) void kbs_fill0(int64_t n, T* y) {
    const int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (i < n) y[i] = zero<T>();
}

inline unsigned nb(int64_t n, int per) { return (unsigned)((n + per - 1) / per); }

template <class T>
struct BL {
    static hipError_t dots(int64_t n, int R, int k, const void* V, const void* w, void* part, void* h, hipStream_t s) {
        const unsigned nch = nb(R, kC);
        hipLaunchKernelGGL(kbs_dots<T>, dim3(kBSolveSlices, nch, nb(k, kJT)), dim3(kT), 0, s, n, R, k, (const T*)V,
                           (const T*)w, (T*)part);
        hipLaunchKernelGGL(kbs_reduce<T>, dim3(nb((int64_t)k * R, kT)), dim3(kT), 0, s, kBSolveSlices, R, k,
                           (const T*)part, (T*)h);
        return hipGetLastError();
    }
    static hipError_t update(int64_t n, int R, int k, const void* V, const void* h, void* w, double* npart, int norm,
                             hipStream_t s) {
        hipLaunchKernelGGL(kbs_update<T>, dim3(kBSolveSlices, nb(R, kC)), dim3(kT), 0, s, n, R, k, (const T*)V,
                           (const T*)h, (T*)w, npart, norm);
        return hipGetLastError();
    }
};

}  // namespace

#define BSOLVE_DISPATCH(cplx, call) ((cplx) ? BL<cdbl>::call : BL<double>::call)

hipError_t bsolve_dots(int cplx, int64_t n, int R, int k, const void* V, const void* w, void* part, void* h,
                       hipStream_t s) {
    return BSOLVE_DISPATCH(cplx, dots(n, R, k, V, w, part, h, s));
}

hipError_t bsolve_update(int cplx, int64_t n, int R, int k, const void* V, const void* h, void* w, double* npart,
                         int norm, hipStream_t s) {
    return BSOLVE_DISPATCH(cplx, update(n, R, k, V, h, w, npart, norm, s));
}

hipError_t bsolve_residual(int cplx, int64_t n, int R, const void* b, void* w, double* npart, int copy_b,
                           hipStream_t s) {
    const dim3 g(kBSolveSlices, nb(R, kC));
    if (cplx)
        hipLaunchKernelGGL(kbs_residual<cdbl>, g, dim3(kT), 0, s, n, R, (const cdbl*)b, (cdbl*)w, npart, copy_b);
    else
        hipLaunchKernelGGL(kbs_residual<double>, g, dim3(kT), 0, s, n, R, (const double*)b, (double*)w, npart, copy_b);
    return hipGetLastError();
}

hipError_t bsolve_start(int cplx, int64_t n, int R, const double* npart, const void* w, void* v0,
                        const BGmresState& st, hipStream_t s) {
    if (cplx) {
        hipLaunchKernelGGL(kbs_start<cdbl>, dim3(nb(R, 64)), dim3(64), 0, s, kBSolveSlices, R, st.m, npart, st);
        hipLaunchKernelGGL(kbs_scale<cdbl>, dim3(nb(n * R, kT)), dim3(kT), 0, s, n, R, (const cdbl*)w, st.sc,
                           (cdbl*)v0);
    } else {
        hipLaunchKernelGGL(kbs_start<double>, dim3(nb(R, 64)), dim3(64), 0, s, kBSolveSlices, R, st.m, npart, st);
        hipLaunchKernelGGL(kbs_scale<double>, dim3(nb(n * R, kT)), dim3(kT), 0, s, n, R, (const double*)w, st.sc,
                           (double*)v0);
    }
    return hipGetLastError();
}

hipError_t bsolve_givens_scale(int cplx, int64_t n, int R, int j, const double* npart, const void* h1, const void* h2,
                               const void* w, void* vnext, const BGmresState& st, hipStream_t s) {
    if (cplx) {
        hipLaunchKernelGGL(kbs_givens<cdbl>, dim3(nb(R, kGivensThreads)), dim3(kGivensThreads), 0, s, kBSolveSlices, R, st.m, j, npart,
                           (const cdbl*)h1, (const cdbl*)h2, st);
        hipLaunchKernelGGL(kbs_scale<cdbl>, dim3(nb(n * R, kT)), dim3(kT), 0, s, n, R, (const cdbl*)w, st.sc,
                           (cdbl*)vnext);
    } else {
        hipLaunchKernelGGL(kbs_givens<double>, dim3(nb(R, kGivensThreads)), dim3(kGivensThreads), 0, s, kBSolveSlices, R, st.m, j, npart,
                           (const double*)h1, (const double*)h2, st);
        hipLaunchKernelGGL(kbs_scale<double>, dim3(nb(n * R, kT)), dim3(kT), 0, s, n, R, (const double*)w, st.sc,
                           (double*)vnext);
    }
    return hipGetLastError();
}

hipError_t bsolve_backsolve_update(int cplx, int64_t n, int R, int k, const void* V, void* x, const BGmresState& st,
                                   hipStream_t s) {
    if (k <= 0) return hipSuccess;
    const dim3 g(kBSolveSlices, nb(R, kC));
    if (cplx) {
        hipLaunchKernelGGL(kbs_backsolve<cdbl>, dim3(nb(R, 64)), dim3(64), 0, s, R, st.m, st);
        hipLaunchKernelGGL(kbs_xupdate<cdbl>, g, dim3(kT), 0, s, n, R, k, (const cdbl*)V, (const cdbl*)st.y, (cdbl*)x);
    } else {
        hipLaunchKernelGGL(kbs_backsolve<double>, dim3(nb(R, 64)), dim3(64), 0, s, R, st.m, st);
        hipLaunchKernelGGL(kbs_xupdate<double>, g, dim3(kT), 0, s, n, R, k, (const double*)V, (const double*)st.y,
                           (double*)x);
    }
    return hipGetLastError();
}

hipError_t bsolve_xupdate(int cplx, int64_t n, int R, int k, const void* V, const void* y, void* x, hipStream_t s) {
    if (k <= 0) return hipSuccess;
    if (k > kMaxRestart) return hipErrorInvalidValue;
    const dim3 g(kBSolveSlices, nb(R, kC));
    if (cplx)
        hipLaunchKernelGGL(kbs_xupdate<cdbl>, g, dim3(kT), 0, s, n, R, k, (const cdbl*)V, (const cdbl*)y, (cdbl*)x);
    else
        hipLaunchKernelGGL(kbs_xupdate<double>, g, dim3(kT), 0, s, n, R, k, (const double*)V, (const double*)y,
                           (double*)x);
    return hipGetLastError();
}

hipError_t bsolve_scale2(int cplx, int64_t n, int R, const double* npart, const void* u, const void* d, void* U,
                         void* D, hipStream_t s) {
    const dim3 g(kBSolveSlices, nb(R, kC));
    if (cplx)
        hipLaunchKernelGGL(kbs_scale2<cdbl>, g, dim3(kT), 0, s, n, R, npart, (const cdbl*)u, (const cdbl*)d, (cdbl*)U,
                           (cdbl*)D);
    else
        hipLaunchKernelGGL(kbs_scale2<double>, g, dim3(kT), 0, s, n, R, npart, (const double*)u, (const double*)d,
                           (double*)U, (double*)D);
    return hipGetLastError();
}

hipError_t bsolve_axpy(int cplx, int64_t n, int R, const void* x, void* y, hipStream_t s) {
    if (cplx)
        hipLaunchKernelGGL(kbs_axpy<cdbl>, dim3(nb(n * R, kT)), dim3(kT), 0, s, n, R, (const cdbl*)x, (cdbl*)y);
    else
        hipLaunchKernelGGL(kbs_axpy<double>, dim3(nb(n * R, kT)), dim3(kT), 0, s, n, R, (const double*)x, (double*)y);
    return hipGetLastError();
}

hipError_t bsolve_mask(int cplx, int64_t n, int R, const int* flag, void* y, hipStream_t s) {
    if (cplx)
        hipLaunchKernelGGL(kbs_mask<cdbl>, dim3(nb(n * R, kT)), dim3(kT), 0, s, n, R, flag, (cdbl*)y);
    else
        hipLaunchKernelGGL(kbs_mask<double>, dim3(nb(n * R, kT)), dim3(kT), 0, s, n, R, flag, (double*)y);
    return hipGetLastError();
}

hipError_t bsolve_zero(int cplx, int64_t n_scalars, void* y, hipStream_t s) {
    if (n_scalars <= 0) return hipSuccess;
    if (cplx)
        hipLaunchKernelGGL(kbs_fill0<cdbl>, dim3(nb(n_scalars, kT)), dim3(kT), 0, s, n_scalars, (cdbl*)y);
    else
        hipLaunchKernelGGL(kbs_fill0<double>, dim3(nb(n_scalars, kT)), dim3(kT), 0, s, n_scalars, (double*)y);
    return hipGetLastError();
}

}  // namespace bem
