// GMRES(m) vector kernels: classical Gram-Schmidt with one reorthogonalisation, Givens
// rotations and the triangular solve on the device.  Every vector kernel splits the
// N entries into kSolveBlocks contiguous slices, one per block, and writes its per-block
// partial sums; the next kernel reduces those partials in its prologue (fixed order, so
// results are deterministic).
#include "bem_solve.h"

namespace bem {

namespace {

constexpr int kThreads = 256;

__device__ inline double wsum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
__device__ inline cdbl wsum(cdbl v) { return {wsum(v.re), wsum(v.im)}; }

__device__ inline double absval(double v) { return fabs(v); }
__device__ inline double absval(cdbl v) { return sqrt(v.re * v.re + v.im * v.im); }
__device__ inline double div_(double a, double b) { return a / b; }
__device__ inline cdbl div_(cdbl a, cdbl b) {
    const double d = b.re * b.re + b.im * b.im;
    return {(a.re * b.re + a.im * b.im) / d, (a.im * b.re - a.re * b.im) / d};
}
__device__ inline double from_real(double v, double) { return v; }
__device__ inline cdbl from_real(double v, cdbl) { return {v, 0.0}; }

// slice of block b
__device__ inline void slice(int64_t n, int64_t& t0, int64_t& t1) {
    const int64_t len = (n + gridDim.x - 1) / gridDim.x;
    t0 = (int64_t)blockIdx.x * len;
    t1 = t0 + len < n ? t0 + len : n;
}

// block-wide sum of one value per thread (256 threads), result valid in thread 0
template <class T>
__device__ inline T block_sum(T v, T* red) {
    v = wsum(v);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    T s = zero<T>();
    if (threadIdx.x == 0) s = red[0] + red[1] + red[2] + red[3];
    __syncthreads();
    return s;
}

// part[b][i] = sum over slice b of conj(V_i) w, i < k: wave v of the block takes the
// vectors i = v, v + 4, ..., each lane every 64th entry of the slice, then a butterfly
// (no block barrier per vector)
template <class T>
__device__ inline void slice_dots(int64_t n, int k, const T* __restrict__ V, const T* w, int64_t t0, int64_t t1,
                                  T* __restrict__ part) {
    const int v = threadIdx.x >> 6, lane = threadIdx.x & 63;
#pragma unroll 4
    for (int i = v; i < k; i += kThreads / 64) {
        T acc = zero<T>();
        for (int64_t t = t0 + lane; t < t1; t += 64) acc += conj_(V[(int64_t)i * n + t]) * w[t];
        acc = wsum(acc);
        if (lane == 0) part[(int64_t)blockIdx.x * k + i] = acc;
    }
}

template <class T>
__global__ __launch_bounds__(kThreads) void k_s_dots(int64_t n, int k, const T* __restrict__ V, const T* __restrict__ w,
                                                     T* __restrict__ part) {
    int64_t t0, t1;
    slice(n, t0, t1);
    slice_dots(n, k, V, w, t0, t1, part);
}

// h = sum of the partials (k values) -> w -= V h over the slice -> partials of the next
// reduction of the updated slice: mode 0 -> V^H w (k values), mode 1 -> ||w||^2
template <class T>
__global__ __launch_bounds__(kThreads) void k_s_update(int64_t n, int k, const T* __restrict__ V,
                                                       const T* __restrict__ part_in, T* __restrict__ hout, T* w,
                                                       T* __restrict__ part_out, double* __restrict__ npart, int mode) {
    __shared__ T h[65];
    __shared__ double redd[4];
    {
        // h_i = sum over the blocks' partials: wave v takes i = v, v + 4, ..., each lane
        // every 64th block, then a butterfly (fixed order)
        const int v = threadIdx.x >> 6, lane = threadIdx.x & 63;
        for (int i = v; i < k; i += kThreads / 64) {
            T s = zero<T>();
            for (int b = lane; b < (int)gridDim.x; b += 64) s += part_in[(int64_t)b * k + i];
            s = wsum(s);
            if (lane == 0) {
                h[i] = s;
                if (blockIdx.x == 0) hout[i] = s;
            }
        }
    }
    __syncthreads();
    int64_t t0, t1;
    slice(n, t0, t1);
    for (int64_t t = t0 + threadIdx.x; t < t1; t += kThreads) {
        T s = zero<T>();
        for (int i = 0; i < k; ++i) s += h[i] * V[(int64_t)i * n + t];
        w[t] -= s;
    }
    __syncthreads();
    if (mode == 0) {
        slice_dots(n, k, V, w, t0, t1, part_out);
    } else {
        double acc = 0.0;
        for (int64_t t = t0 + threadIdx.x; t < t1; t += kThreads) acc += abs2(w[t]);
        const double s = block_sum(acc, redd);
        if (threadIdx.x == 0) npart[blockIdx.x] = s;
    }
}

// sqrt of the sum of the nb per-block squared-norm partials, computed by every wave in the
// same fixed order (each lane every 64th partial, then a butterfly)
__device__ inline double reduce_npart(const double* npart, int nb) {
    double s = 0.0;
    for (int b = threadIdx.x & 63; b < nb; b += 64) s += npart[b];
    return sqrt(wsum(s));
}

// v_{j+1} = w / ||w|| over the slice; block 0 applies the Givens rotations to the new
// Hessenberg column j (h1 + h2 above the diagonal, ||w|| below) and records the residual
// estimate |g_{j+1}| in scal[2 + j]
template <class T>
__global__ __launch_bounds__(kThreads) void k_s_scale_givens(int64_t n, int j, const double* __restrict__ npart,
                                                             const T* __restrict__ w, T* __restrict__ vnext,
                                                             GmresState st) {
    const double nrm = reduce_npart(npart, gridDim.x);
    int64_t t0, t1;
    slice(n, t0, t1);
    const double inv = 1.0 / nrm;
    for (int64_t t = t0 + threadIdx.x; t < t1; t += kThreads) vnext[t] = w[t] * inv;
    if (blockIdx.x != 0) return;
    // block 0: the new column and the rotations so far are staged in LDS by all threads,
    // then one thread applies the rotations (a serial chain, now on LDS)
    __shared__ T col[66];
    __shared__ T snl[64];
    __shared__ double csl[64];
    const int m = st.m;
    T* H = (T*)st.H;
    T* sn = (T*)st.sn;
    T* g = (T*)st.g;
    const T* h1 = (const T*)st.h1;
    const T* h2 = (const T*)st.h2;
    for (int i = threadIdx.x; i <= j; i += kThreads) {
        col[i] = h1[i] + h2[i];
        if (i < j) {
            snl[i] = sn[i];
            csl[i] = st.cs[i];
        }
    }
    __syncthreads();
    if (threadIdx.x != 0) return;
    col[j + 1] = from_real(nrm, T());
    for (int i = 0; i < j; ++i) {
        const T a = col[i], c = col[i + 1];
        col[i] = csl[i] * a + snl[i] * c;
        col[i + 1] = csl[i] * c - conj_(snl[i]) * a;
    }
    const T a = col[j], c = col[j + 1];
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
    st.cs[j] = cj;
    sn[j] = sj;
    col[j] = cj * a + sj * c;
    for (int i = 0; i <= j; ++i) H[i * m + j] = col[i];
    H[(j + 1) * m + j] = zero<T>();
    const T gj = g[j];
    g[j] = cj * gj;
    g[j + 1] = zero<T>() - conj_(sj) * gj;
    st.scal[2 + j] = absval(g[j + 1]);
}

// w = b - w (residual of the current iterate) and its squared-norm partials
template <class T>
__global__ __launch_bounds__(kThreads) void k_s_residual(int64_t n, const T* __restrict__ b, T* w,
                                                         double* __restrict__ npart, int copy_b) {
    __shared__ double redd[4];
    int64_t t0, t1;
    slice(n, t0, t1);
    double acc = 0.0;
    for (int64_t t = t0 + threadIdx.x; t < t1; t += kThreads) {
        const T r = copy_b ? b[t] : b[t] - w[t];
        w[t] = r;
        acc += abs2(r);
    }
    const double s = block_sum(acc, redd);
    if (threadIdx.x == 0) npart[blockIdx.x] = s;
}

// beta = ||w||, v_0 = w / beta, g = beta e_1, scal[1] = beta
template <class T>
__global__ __launch_bounds__(kThreads) void k_s_start(int64_t n, const double* __restrict__ npart,
                                                      const T* __restrict__ w, T* __restrict__ v0, GmresState st) {
    const double beta = reduce_npart(npart, gridDim.x);
    int64_t t0, t1;
    slice(n, t0, t1);
    const double inv = beta > 0.0 ? 1.0 / beta : 0.0;
    for (int64_t t = t0 + threadIdx.x; t < t1; t += kThreads) v0[t] = w[t] * inv;
    if (blockIdx.x == 0) {
        T* g = (T*)st.g;
        for (int i = threadIdx.x; i <= st.m; i += kThreads) g[i] = i == 0 ? from_real(beta, T()) : zero<T>();
        if (threadIdx.x == 0) st.scal[1] = beta;
    }
}

// y = H_k^{-1} g_k (upper triangular, k <= m), one thread
template <class T>
__global__ void k_s_backsolve(int k, GmresState st) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const int m = st.m;
    const T* H = (const T*)st.H;
    const T* g = (const T*)st.g;
    T* y = (T*)st.y;
    for (int i = k - 1; i >= 0; --i) {
        T s = g[i];
        for (int l = i + 1; l < k; ++l) s -= H[i * m + l] * y[l];
        y[i] = div_(s, H[i * m + i]);
    }
}

// x += sum_{i<k} y_i v_i
template <class T>
__global__ __launch_bounds__(kThreads) void k_s_xupdate(int64_t n, int k, const T* __restrict__ V,
                                                        const T* __restrict__ y, T* x) {
    __shared__ T ys[64];
    for (int i = threadIdx.x; i < k; i += kThreads) ys[i] = y[i];
    __syncthreads();
    int64_t t0, t1;
    slice(n, t0, t1);
    for (int64_t t = t0 + threadIdx.x; t < t1; t += kThreads) {
        T s = zero<T>();
        for (int i = 0; i < k; ++i) s += ys[i] * V[(int64_t)i * n + t];
        x[t] += s;
    }
}

template <class T>
__global__ __launch_bounds__(kThreads) void k_s_axpy(int64_t n, double a, const T* __restrict__ x, T* y) {
    const int64_t t = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (t < n) y[t] += a * x[t];
}

template <class T>
struct Launch {
    static hipError_t dots(int64_t n, int k, const void* V, const void* w, void* part, hipStream_t s) {
        hipLaunchKernelGGL(k_s_dots<T>, dim3(kSolveBlocks), dim3(kThreads), 0, s, n, k, (const T*)V, (const T*)w,
                           (T*)part);
        return hipGetLastError();
    }
};

}  // namespace

hipError_t solve_dots(int cplx, int64_t n, int k, const void* V, const void* w, void* part, hipStream_t s) {
    return cplx ? Launch<cdbl>::dots(n, k, V, w, part, s) : Launch<double>::dots(n, k, V, w, part, s);
}

hipError_t solve_update(int cplx, int64_t n, int k, const void* V, const void* part_in, void* hout, void* w,
                        void* part_out, double* npart, int mode, hipStream_t s) {
    if (cplx)
        hipLaunchKernelGGL(k_s_update<cdbl>, dim3(kSolveBlocks), dim3(kThreads), 0, s, n, k, (const cdbl*)V,
                           (const cdbl*)part_in, (cdbl*)hout, (cdbl*)w, (cdbl*)part_out, npart, mode);
    else
        hipLaunchKernelGGL(k_s_update<double>, dim3(kSolveBlocks), dim3(kThreads), 0, s, n, k, (const double*)V,
                           (const double*)part_in, (double*)hout, (double*)w, (double*)part_out, npart, mode);
    return hipGetLastError();
}

hipError_t solve_scale_givens(int cplx, int64_t n, int j, const double* npart, const void* w, void* vnext,
                              const GmresState& st, hipStream_t s) {
    if (cplx)
        hipLaunchKernelGGL(k_s_scale_givens<cdbl>, dim3(kSolveBlocks), dim3(kThreads), 0, s, n, j, npart,
                           (const cdbl*)w, (cdbl*)vnext, st);
    else
        hipLaunchKernelGGL(k_s_scale_givens<double>, dim3(kSolveBlocks), dim3(kThreads), 0, s, n, j, npart,
                           (const double*)w, (double*)vnext, st);
    return hipGetLastError();
}

hipError_t solve_residual(int cplx, int64_t n, const void* b, void* w, double* npart, int copy_b, hipStream_t s) {
    if (cplx)
        hipLaunchKernelGGL(k_s_residual<cdbl>, dim3(kSolveBlocks), dim3(kThreads), 0, s, n, (const cdbl*)b, (cdbl*)w,
                           npart, copy_b);
    else
        hipLaunchKernelGGL(k_s_residual<double>, dim3(kSolveBlocks), dim3(kThreads), 0, s, n, (const double*)b,
                           (double*)w, npart, copy_b);
    return hipGetLastError();
}

hipError_t solve_start(int cplx, int64_t n, const double* npart, const void* w, void* v0, const GmresState& st,
                       hipStream_t s) {
    if (cplx)
        hipLaunchKernelGGL(k_s_start<cdbl>, dim3(kSolveBlocks), dim3(kThreads), 0, s, n, npart, (const cdbl*)w,
                           (cdbl*)v0, st);
    else
        hipLaunchKernelGGL(k_s_start<double>, dim3(kSolveBlocks), dim3(kThreads), 0, s, n, npart, (const double*)w,
                           (double*)v0, st);
    return hipGetLastError();
}

hipError_t solve_axpy(int cplx, int64_t n, double a, const void* x, void* y, hipStream_t s) {
    const unsigned nb = (unsigned)((n + kThreads - 1) / kThreads);
    if (cplx)
        hipLaunchKernelGGL(k_s_axpy<cdbl>, dim3(nb), dim3(kThreads), 0, s, n, a, (const cdbl*)x, (cdbl*)y);
    else
        hipLaunchKernelGGL(k_s_axpy<double>, dim3(nb), dim3(kThreads), 0, s, n, a, (const double*)x, (double*)y);
    return hipGetLastError();
}

hipError_t solve_backsolve_update(int cplx, int64_t n, int k, const void* V, void* x, const GmresState& st,
                                  hipStream_t s) {
    if (k <= 0) return hipSuccess;
    if (cplx) {
        hipLaunchKernelGGL(k_s_backsolve<cdbl>, dim3(1), dim3(64), 0, s, k, st);
        hipLaunchKernelGGL(k_s_xupdate<cdbl>, dim3(kSolveBlocks), dim3(kThreads), 0, s, n, k, (const cdbl*)V,
                           (const cdbl*)st.y, (cdbl*)x);
    } else {
        hipLaunchKernelGGL(k_s_backsolve<double>, dim3(1), dim3(64), 0, s, k, st);
        hipLaunchKernelGGL(k_s_xupdate<double>, dim3(kSolveBlocks), dim3(kThreads), 0, s, n, k, (const double*)V,
                           (const double*)st.y, (double*)x);
    }
    return hipGetLastError();
}

}  // namespace bem
