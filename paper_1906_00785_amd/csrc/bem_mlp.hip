// The correction network of the learned preconditioner: a 3-layer perceptron
// in -> hidden -> hidden -> out with ReLU, trained on the device by these kernels
// (forward, loss and gradient of the rank-8 correction, backward, Adam).
//
// Parameters (FP32, one flat array): W1 [in][hid], b1 [hid], W2 [hid][hid], b2 [hid],
// W3 [hid][out], b3 [out] (row-major).  The products run as FP32 on the vector units
// (precision 0) or with BF16 operands on the matrix cores and FP32 accumulation
// (precision 1, v_mfma_f32_16x16x32_bf16).
#include "bem_mlp.h"

#include <mutex>

#include "bem_device.h"

namespace bem {

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef unsigned short u16x8 __attribute__((ext_vector_type(8)));

inline unsigned nblk(int64_t n, int per) { return (unsigned)((n + per - 1) / per); }

// C[M][N] = op(A)[M][K] op(B)[K][N] (+ bias[N]) (ReLU) (* (mask[M][N] > 0)), 64 x 64 tile
// per block, K in steps of 32 through LDS.  op(A)(i,k) = ta ? A[k*lda + i] : A[i*lda + k],
// op(B)(k,j) = tb ? B[j*ldb + k] : B[k*ldb + j].
struct GemmArgs {
    int M, N, K;
    const float* A;
    int lda, ta;
    const float* B;
    int ldb, tb;
    float* C;
    int ldc;
    const float* bias;
    int relu;
    const float* mask;  // optional, ld = ldc
};

__device__ inline float lda_at(const GemmArgs& g, int i, int k) {
    if (i >= g.M || k >= g.K) return 0.0f;
    return g.ta ? g.A[(int64_t)k * g.lda + i] : g.A[(int64_t)i * g.lda + k];
}
__device__ inline float ldb_at(const GemmArgs& g, int k, int j) {
    if (k >= g.K || j >= g.N) return 0.0f;
    return g.tb ? g.B[(int64_t)j * g.ldb + k] : g.B[(int64_t)k * g.ldb + j];
}

__device__ inline void gemm_store(const GemmArgs& g, int i, int j, float v) {
    if (i >= g.M || j >= g.N) return;
    if (g.bias) v += g.bias[j];
    if (g.relu) v = v > 0.0f ? v : 0.0f;
    if (g.mask && !(g.mask[(int64_t)i * g.ldc + j] > 0.0f)) v = 0.0f;
    g.C[(int64_t)i * g.ldc + j] = v;
}

__global__ __launch_bounds__(256) void k_gemm_f32(GemmArgs g) {
    __shared__ float As[64][33];
    __shared__ float Bs[32][65];
    const int i0 = blockIdx.y * 64, j0 = blockIdx.x * 64;
    const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;  // 16 x 16 threads, 4 x 4 outputs each
    float acc[4][4] = {};
    for (int k0 = 0; k0 < g.K; k0 += 32) {
        for (int e = threadIdx.x; e < 64 * 32; e += 256) {
            const int r = e / 32, c = e % 32;
            As[r][c] = lda_at(g, i0 + r, k0 + c);
        }
        for (int e = threadIdx.x; e < 32 * 64; e += 256) {
            const int r = e / 64, c = e % 64;
            Bs[r][c] = ldb_at(g, k0 + r, j0 + c);
        }
        __syncthreads();
        for (int k = 0; k < 32; ++k) {
            float a[4], b[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) a[u] = As[ty * 4 + u][k];
#pragma unroll
            for (int u = 0; u < 4; ++u) b[u] = Bs[k][tx * 4 + u];
#pragma unroll
            for (int u = 0; u < 4; ++u)
#pragma unroll
                for (int v = 0; v < 4; ++v) acc[u][v] += a[u] * b[v];
        }
        __syncthreads();
    }
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) gemm_store(g, i0 + ty * 4 + u, j0 + tx * 4 + v, acc[u][v]);
}

// BF16 operands, FP32 accumulation: the four waves of a block take 32 x 32 quadrants of the
// 64 x 64 tile (2 x 2 MFMA tiles each).  Lane l holds A[l % 16][8 (l / 16) + e] and
// B[8 (l / 16) + e][l % 16] and receives C[4 (l / 16) + e][l % 16].
__global__ __launch_bounds__(256) void k_gemm_bf16(GemmArgs g) {
    __shared__ uint16_t As[64][32 + 8];
    __shared__ uint16_t Bs[64][32 + 8];  // stored transposed: Bs[j][k]
    const int i0 = blockIdx.y * 64, j0 = blockIdx.x * 64;
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int wi = (w >> 1) * 32, wj = (w & 1) * 32;
    f32x4 acc[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
    for (int k0 = 0; k0 < g.K; k0 += 32) {
        for (int e = threadIdx.x; e < 64 * 32; e += 256) {
            const int r = e / 32, c = e % 32;
            As[r][c] = f2bf(lda_at(g, i0 + r, k0 + c));
            Bs[r][c] = f2bf(ldb_at(g, k0 + c, j0 + r));
        }
        __syncthreads();
        const int kk = 8 * (lane >> 4);
        bf16x8 af[2], bfr[2];
#pragma unroll
        for (int a = 0; a < 2; ++a) {
            u16x8 v;
#pragma unroll
            for (int e = 0; e < 8; ++e) v[e] = As[wi + 16 * a + (lane & 15)][kk + e];
            af[a] = __builtin_bit_cast(bf16x8, v);
        }
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            u16x8 v;
#pragma unroll
            for (int e = 0; e < 8; ++e) v[e] = Bs[wj + 16 * b + (lane & 15)][kk + e];
            bfr[b] = __builtin_bit_cast(bf16x8, v);
        }
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < 2; ++b) acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[a], bfr[b], acc[a][b], 0, 0, 0);
        __syncthreads();
    }
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int e = 0; e < 4; ++e)
                gemm_store(g, i0 + wi + 16 * a + 4 * (lane >> 4) + e, j0 + wj + 16 * b + (lane & 15), acc[a][b][e]);
}

hipError_t gemm(const GemmArgs& g, int precision, hipStream_t st) {
    const dim3 grid(nblk(g.N, 64), nblk(g.M, 64));
    if (precision == 1)
        hipLaunchKernelGGL(k_gemm_bf16, grid, dim3(256), 0, st, g);
    else
        hipLaunchKernelGGL(k_gemm_f32, grid, dim3(256), 0, st, g);
    return hipGetLastError();
}

// column sums of dY [M][N] into db [N] (row order fixed)
__global__ void k_colsum(int M, int N, const float* dY, float* db) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= N) return;
    float s = 0.0f;
    for (int i = 0; i < M; ++i) s += dY[(int64_t)i * N + j];
    db[j] = s;
}

// Loss of the rank-kRankN correction for one sample per block: E = T - U V^T (64 x 64;
// complex when cplx), L_b = ||E||_F^2 / ||T||_F^2, loss[b] = L_b / batch, and the gradient of
// the batch mean with respect to the network outputs (U, V; real and imaginary parts).
// Output layout: real [U (64 x 8) | V (64 x 8)]; complex [Re U | Im U | Re V | Im V].
__global__ __launch_bounds__(256) void k_lowrank_loss(int batch, int cplx, const float* O, const float* T, float* dO,
                                                      float* loss) {
    constexpr int n = kMlpSlots, r = kMlpRank;
    __shared__ float Ur[n][r], Ui[n][r], Vr[n][r], Vi[n][r];
    __shared__ float Er[n][n + 1], Ei[n][n + 1];
    __shared__ float red[2][256];
    const int b = blockIdx.x;
    const int out = (cplx ? 4 : 2) * n * r;
    const float* o = O + (int64_t)b * out;
    for (int e = threadIdx.x; e < n * r; e += 256) {
        const int i = e / r, k = e % r;
        if (cplx) {
            Ur[i][k] = o[e];
            Ui[i][k] = o[n * r + e];
            Vr[i][k] = o[2 * n * r + e];
            Vi[i][k] = o[3 * n * r + e];
        } else {
            Ur[i][k] = o[e];
            Ui[i][k] = 0.0f;
            Vr[i][k] = o[n * r + e];
            Vi[i][k] = 0.0f;
        }
    }
    __syncthreads();
    const float* t = T + (int64_t)b * n * n * (cplx ? 2 : 1);
    float se = 0.0f, st = 0.0f;
    for (int e = threadIdx.x; e < n * n; e += 256) {
        const int i = e / n, j = e % n;
        float pr = 0.0f, pi = 0.0f;
#pragma unroll
        for (int k = 0; k < r; ++k) {
            pr += Ur[i][k] * Vr[j][k] - Ui[i][k] * Vi[j][k];
            pi += Ur[i][k] * Vi[j][k] + Ui[i][k] * Vr[j][k];
        }
        const float tr = cplx ? t[2 * e] : t[e], ti = cplx ? t[2 * e + 1] : 0.0f;
        Er[i][j] = tr - pr;
        Ei[i][j] = ti - pi;
        se += Er[i][j] * Er[i][j] + Ei[i][j] * Ei[i][j];
        st += tr * tr + ti * ti;
    }
    red[0][threadIdx.x] = se;
    red[1][threadIdx.x] = st;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) {
            red[0][threadIdx.x] += red[0][threadIdx.x + off];
            red[1][threadIdx.x] += red[1][threadIdx.x + off];
        }
        __syncthreads();
    }
    const float den = red[1][0] > 0.0f ? red[1][0] : 1.0f;
    if (threadIdx.x == 0) loss[b] = red[0][0] / den / (float)batch;
    const float sc = 2.0f / den / (float)batch;
    float* d = dO + (int64_t)b * out;
    // dL/dRe U_ik = -sc Re(sum_j conj(E_ij) V_jk), dL/dIm U_ik = sc Im(sum_j conj(E_ij) V_jk)
    for (int e = threadIdx.x; e < n * r; e += 256) {
        const int i = e / r, k = e % r;
        float gr = 0.0f, gi = 0.0f, hr = 0.0f, hi = 0.0f;
        for (int j = 0; j < n; ++j) {
            // conj(E_ij) V_jk
            gr += Er[i][j] * Vr[j][k] + Ei[i][j] * Vi[j][k];
            gi += Er[i][j] * Vi[j][k] - Ei[i][j] * Vr[j][k];
            // conj(E_ji) U_jk  (for V_ik)
            hr += Er[j][i] * Ur[j][k] + Ei[j][i] * Ui[j][k];
            hi += Er[j][i] * Ui[j][k] - Ei[j][i] * Ur[j][k];
        }
        if (cplx) {
            d[e] = -sc * gr;
            d[n * r + e] = sc * gi;
            d[2 * n * r + e] = -sc * hr;
            d[3 * n * r + e] = sc * hi;
        } else {
            d[e] = -sc * gr;
            d[n * r + e] = -sc * hr;
        }
    }
}

__global__ void k_sum(int n, const float* v, float* out) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    float s = 0.0f;
    for (int i = 0; i < n; ++i) s += v[i];
    out[0] = s;
}

__global__ void k_adam(int64_t n, float* p, const float* g, float* m, float* v, float lr, float b1, float b2, float eps,
                       float c1, float c2) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// He-uniform weights from a counter-based generator (splitmix64 of seed and index), zero biases
__global__ void k_init(int in, int hid, int out, uint64_t seed, float* p) {
    const int64_t n = (int64_t)in * hid + hid + (int64_t)hid * hid + hid + (int64_t)hid * out + out;
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const int64_t o1 = (int64_t)in * hid, o2 = o1 + hid, o3 = o2 + (int64_t)hid * hid, o4 = o3 + hid,
                  o5 = o4 + (int64_t)hid * out;
    int fan = 0;
    if (i < o1)
        fan = in;
    else if (i >= o2 && i < o3)
        fan = hid;
    else if (i >= o4 && i < o5)
        fan = hid;
    if (fan == 0) {
        p[i] = 0.0f;
        return;
    }
    uint64_t x = seed * 0x9E3779B97F4A7C15ull + (uint64_t)i;
    x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
    x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
    x ^= x >> 31;
    const double u = (double)(x >> 11) * (1.0 / 9007199254740992.0);  // [0, 1)
    const double lim = sqrt(6.0 / fan);
    p[i] = (float)((2.0 * u - 1.0) * lim);
}

struct Net {
    int in, hid, out;
    const float *W1, *b1, *W2, *b2, *W3, *b3;
};
inline Net net_of(int in, int hid, int out, const float* p) {
    Net n{in, hid, out};
    n.W1 = p;
    n.b1 = n.W1 + (int64_t)in * hid;
    n.W2 = n.b1 + hid;
    n.b2 = n.W2 + (int64_t)hid * hid;
    n.W3 = n.b2 + hid;
    n.b3 = n.W3 + (int64_t)hid * out;
    return n;
}

}  // namespace

int64_t mlp_nparams(int in, int hid, int out) {
    return (int64_t)in * hid + hid + (int64_t)hid * hid + hid + (int64_t)hid * out + out;
}

size_t mlp_ws_bytes(int hid, int out, int batch) {
    return sizeof(float) * ((size_t)batch * (4 * (size_t)hid + 2 * (size_t)out) + (size_t)batch + 64) + 1024;
}

hipError_t mlp_init(int in, int hid, int out, uint64_t seed, float* params, hipStream_t st) {
    hipLaunchKernelGGL(k_init, dim3(nblk(mlp_nparams(in, hid, out), 256)), dim3(256), 0, st, in, hid, out, seed,
                       params);
    return hipGetLastError();
}

// workspace: H1, H2 [batch][hid], O [batch][out], dO [batch][out], dH2, dH1 [batch][hid], loss [batch]
struct MlpWs {
    float *H1, *H2, *O, *dO, *dH2, *dH1, *loss;
};
static MlpWs ws_of(int hid, int out, int batch, void* ws) {
    float* p = (float*)ws;
    MlpWs w;
    w.H1 = p;
    w.H2 = w.H1 + (size_t)batch * hid;
    w.O = w.H2 + (size_t)batch * hid;
    w.dO = w.O + (size_t)batch * out;
    w.dH2 = w.dO + (size_t)batch * out;
    w.dH1 = w.dH2 + (size_t)batch * hid;
    w.loss = w.dH1 + (size_t)batch * hid;
    return w;
}

static hipError_t forward(const Net& n, int batch, const float* X, float* Y, const MlpWs& w, int precision,
                          hipStream_t st) {
    hipError_t e;
    e = gemm({batch, n.hid, n.in, X, n.in, 0, n.W1, n.hid, 0, w.H1, n.hid, n.b1, 1, nullptr}, precision, st);
    if (e != hipSuccess) return e;
    e = gemm({batch, n.hid, n.hid, w.H1, n.hid, 0, n.W2, n.hid, 0, w.H2, n.hid, n.b2, 1, nullptr}, precision, st);
    if (e != hipSuccess) return e;
    return gemm({batch, n.out, n.hid, w.H2, n.hid, 0, n.W3, n.out, 0, Y, n.out, n.b3, 0, nullptr}, precision, st);
}

hipError_t mlp_forward(int in, int hid, int out, int batch, const float* params, const float* X, float* Y,
                       int precision, void* ws, hipStream_t st) {
    const Net n = net_of(in, hid, out, params);
    return forward(n, batch, X, Y, ws_of(hid, out, batch, ws), precision, st);
}

// Forward pass with its hidden activations in a fixed device array instead of a caller
// workspace, for callers that cannot allocate (graph capture, serving loops).  The array is
// a file-scope device variable; its address differs per device and is looked up once per
// device with hipGetSymbolAddress (the variable's name in host code is only a stand-in).
// Every call on a device shares that device's array, so calls that overlap in time on one
// device race.  Nothing in the array needs clearing: the forward pass writes H1 and H2 in
// full before reading them.
static __device__ __align__(256) char scratch[kMlpScratchBytes];

namespace {
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMlpMaxDevices] = {};
}  // namespace

hipError_t mlp_scratch(void** ptr) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMlpMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_ptr[dev] = p;
    }
    *ptr = g_scratch_ptr[dev];
    return hipSuccess;
}

size_t mlp_forward_scratch_bytes(int hid, int batch) { return sizeof(float) * 2 * (size_t)batch * (size_t)hid; }

hipError_t mlp_forward_noalloc(int in, int hid, int out, int batch, const float* params, const float* X, float* Y,
                               int precision, void* scratch_ptr, hipStream_t st) {
    const Net n = net_of(in, hid, out, params);
    MlpWs w{};
    w.H1 = (float*)scratch_ptr;
    w.H2 = w.H1 + (size_t)batch * hid;
    return forward(n, batch, X, Y, w, precision, st);
}

hipError_t mlp_loss_grad(int in, int hid, int out, int batch, int cplx, const float* params, const float* X,
                         const float* T, float* grad, float* loss, int precision, void* ws, hipStream_t st) {
    const Net n = net_of(in, hid, out, params);
    const MlpWs w = ws_of(hid, out, batch, ws);
    hipError_t e = forward(n, batch, X, w.O, w, precision, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_lowrank_loss, dim3(batch), dim3(256), 0, st, batch, cplx, w.O, T, w.dO, w.loss);
    hipLaunchKernelGGL(k_sum, dim3(1), dim3(64), 0, st, batch, w.loss, loss);
    // gradient layout matches the parameters
    Net gn = net_of(in, hid, out, grad);
    float* gW1 = (float*)gn.W1;
    float* gb1 = (float*)gn.b1;
    float* gW2 = (float*)gn.W2;
    float* gb2 = (float*)gn.b2;
    float* gW3 = (float*)gn.W3;
    float* gb3 = (float*)gn.b3;
    // layer 3: dW3 = H2^T dO, db3 = sum dO, dH2 = (dO W3^T) * (H2 > 0)
    e = gemm({hid, out, batch, w.H2, hid, 1, w.dO, out, 0, gW3, out, nullptr, 0, nullptr}, precision, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_colsum, dim3(nblk(out, 256)), dim3(256), 0, st, batch, out, w.dO, gb3);
    e = gemm({batch, hid, out, w.dO, out, 0, n.W3, out, 1, w.dH2, hid, nullptr, 0, w.H2}, precision, st);
    if (e != hipSuccess) return e;
    // layer 2
    e = gemm({hid, hid, batch, w.H1, hid, 1, w.dH2, hid, 0, gW2, hid, nullptr, 0, nullptr}, precision, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_colsum, dim3(nblk(hid, 256)), dim3(256), 0, st, batch, hid, w.dH2, gb2);
    e = gemm({batch, hid, hid, w.dH2, hid, 0, n.W2, hid, 1, w.dH1, hid, nullptr, 0, w.H1}, precision, st);
    if (e != hipSuccess) return e;
    // layer 1
    e = gemm({in, hid, batch, X, in, 1, w.dH1, hid, 0, gW1, hid, nullptr, 0, nullptr}, precision, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_colsum, dim3(nblk(hid, 256)), dim3(256), 0, st, batch, hid, w.dH1, gb1);
    return hipGetLastError();
}

hipError_t mlp_adam(int64_t n, float* params, const float* grad, float* m, float* v, int step, float lr, float b1,
                    float b2, float eps, hipStream_t st) {
    const float c1 = 1.0f - powf(b1, (float)step), c2 = 1.0f - powf(b2, (float)step);
    hipLaunchKernelGGL(k_adam, dim3(nblk(n, 256)), dim3(256), 0, st, n, params, grad, m, v, lr, b1, b2, eps, c1, c2);
    return hipGetLastError();
}

}  // namespace bem
