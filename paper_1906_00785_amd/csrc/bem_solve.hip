// GMRES(m) vector kernels: classical Gram-Schmidt with one reorthogonalisation, Givens
// rotations and the triangular solve on the device.  Every vector kernel splits the
// N entries into kSolveBlocks contiguous slices, one per block, and writes its per-block
// partial sums; the next kernel reduces those partials in its prologue (fixed order, so
// results are deterministic).  The Givens rotations of step j run in one extra block of
// step j+1's dot-product kernel, beside the slices, so that their serial chain is off the
// path from one matrix-vector product to the next.
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

// Givens step j: the new Hessenberg column (h1 + h2 above the diagonal, ||w|| from the
// squared-norm partials below it) is rotated by the rotations so far, the new rotation
// annihilates its subdiagonal entry, and the residual estimate |g_{j+1}| goes to
// scal[2 + j].  One block: the column and the rotations are staged in LDS by all threads,
// then one thread applies the rotations (a serial chain).
template <class T>
__device__ inline void givens_body(int j, const double* __restrict__ npart, const GmresState& st) {
    const double nrm = reduce_npart(npart, kSolveBlocks);
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
    const T gn = zero<T>() - conj_(sj) * gj;
    g[j + 1] = gn;
    const double est = absval(gn);
    st.scal[2 + j] = est;
    if (st.hest) {
        st.hest[j] = est;
        __threadfence_system();  // the estimate is visible to the host before its stamp
        *(volatile unsigned*)(st.hseq + j) = st.stamp;
    }
}

// Dot products of step j+1 (blocks 0 .. kSolveBlocks-1, see slice_dots) and, when
// gj >= 0, the Givens step gj in block kSolveBlocks.  The inputs of Givens step gj (h1,
// h2, the squared-norm partials) are rewritten only by the update kernels that follow.
template <class T>
__global__ __launch_bounds__(kThreads) void k_s_dots(int64_t n, int k, const T* __restrict__ V, const T* __restrict__ w,
                                                     T* __restrict__ part, int gj, const double* __restrict__ npart,
                                                     GmresState st) {
    if ((int)blockIdx.x == kSolveBlocks) {
        if (gj >= 0) givens_body<T>(gj, npart, st);
        return;
    }
    const int64_t len = (n + kSolveBlocks - 1) / kSolveBlocks;
    const int64_t t0 = (int64_t)blockIdx.x * len, t1 = t0 + len < n ? t0 + len : n;
    slice_dots(n, k, V, w, t0, t1, part);
}

// the Givens step on its own (the last step of a cycle)
template <class T>
__global__ __launch_bounds__(kThreads) void k_s_givens(int j, const double* __restrict__ npart, GmresState st) {
    givens_body<T>(j, npart, st);
}

// v_{j+1} = w / ||w|| over the slice
template <class T>
__global__ __launch_bounds__(kThreads) void k_s_scale(int64_t n, const double* __restrict__ npart,
                                                      const T* __restrict__ w, T* __restrict__ vnext) {
    const double nrm = reduce_npart(npart, gridDim.x);
    int64_t t0, t1;
    slice(n, t0, t1);
    const double inv = nrm > 0.0 ? 1.0 / nrm : 0.0;  // a zero vector stays zero
    for (int64_t t = t0 + threadIdx.x; t < t1; t += kThreads) vnext[t] = w[t] * inv;
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

// y = H_k^{-1} g_k (upper triangular, k <= m <= 64), one wave by columns: lane i holds the
// running right-hand side of row i; for l = k-1 down to 0 lane l divides by H_ll and every
// lane above the diagonal subtracts H_il y_l (its next H entry is loaded a column ahead)
template <class T>
__global__ __launch_bounds__(64) void k_s_backsolve(int k, GmresState st) {
    const int i = threadIdx.x;
    const int m = st.m;
    const T* H = (const T*)st.H;
    T* y = (T*)st.y;
    __shared__ T yl;
    T r = i < k ? ((const T*)st.g)[i] : zero<T>();
    T h = k >= 1 && i < k - 1 ? H[i * m + k - 1] : zero<T>();
    for (int l = k - 1; l >= 0; --l) {
        const T hn = l >= 1 && i < l - 1 ? H[i * m + l - 1] : zero<T>();
        if (i == l) {
            const T v = div_(r, H[l * m + l]);
            y[l] = v;
            yl = v;
        }
        __syncthreads();
        if (i < l) r -= h * yl;
        __syncthreads();
        h = hn;
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

// x += sign * sum_{i<k} y_i v_i  (y on the device, k <= 64)
template <class T>
__global__ __launch_bounds__(kThreads) void k_s_combine(int64_t n, int k, const T* __restrict__ V,
                                                        const T* __restrict__ y, double sign, T* x) {
    __shared__ T ys[64];
    for (int i = threadIdx.x; i < k; i += kThreads) ys[i] = y[i] * sign;
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
    static hipError_t dots(int64_t n, int k, const void* V, const void* w, void* part, int gj, const double* npart,
                           const GmresState& st, hipStream_t s) {
        hipLaunchKernelGGL(k_s_dots<T>, dim3(kSolveBlocks + (gj >= 0 ? 1 : 0)), dim3(kThreads), 0, s, n, k,
                           (const T*)V, (const T*)w, (T*)part, gj, npart, st);
        return hipGetLastError();
    }
    static hipError_t givens(int j, const double* npart, const GmresState& st, hipStream_t s) {
        hipLaunchKernelGGL(k_s_givens<T>, dim3(1), dim3(kThreads), 0, s, j, npart, st);
        return hipGetLastError();
    }
    static hipError_t scale(int64_t n, const double* npart, const void* w, void* vnext, hipStream_t s) {
        hipLaunchKernelGGL(k_s_scale<T>, dim3(kSolveBlocks), dim3(kThreads), 0, s, n, npart, (const T*)w, (T*)vnext);
        return hipGetLastError();
    }
};

}  // namespace

hipError_t solve_dots(int cplx, int64_t n, int k, const void* V, const void* w, void* part, int gj,
                      const double* npart, const GmresState& st, hipStream_t s) {
    if (gj >= st.m) return hipErrorInvalidValue;
    return cplx ? Launch<cdbl>::dots(n, k, V, w, part, gj, npart, st, s)
                : Launch<double>::dots(n, k, V, w, part, gj, npart, st, s);
}

hipError_t solve_givens(int cplx, int j, const double* npart, const GmresState& st, hipStream_t s) {
    if (j < 0 || j >= st.m) return hipErrorInvalidValue;
    return cplx ? Launch<cdbl>::givens(j, npart, st, s) : Launch<double>::givens(j, npart, st, s);
}

hipError_t solve_scale(int cplx, int64_t n, const double* npart, const void* w, void* vnext, hipStream_t s) {
    return cplx ? Launch<cdbl>::scale(n, npart, w, vnext, s) : Launch<double>::scale(n, npart, w, vnext, s);
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

hipError_t solve_combine(int cplx, int64_t n, int k, const void* V, const void* y, double sign, void* x,
                         hipStream_t s) {
    if (k <= 0) return hipSuccess;
    if (k > 64) return hipErrorInvalidValue;
    if (cplx)
        hipLaunchKernelGGL(k_s_combine<cdbl>, dim3(kSolveBlocks), dim3(kThreads), 0, s, n, k, (const cdbl*)V,
                           (const cdbl*)y, sign, (cdbl*)x);
    else
        hipLaunchKernelGGL(k_s_combine<double>, dim3(kSolveBlocks), dim3(kThreads), 0, s, n, k, (const double*)V,
                           (const double*)y, sign, (double*)x);
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
