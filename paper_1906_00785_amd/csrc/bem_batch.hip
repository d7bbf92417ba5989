// gfx950 kernels of the H^2 matvec over many right-hand sides (see bem_batch.h).
//
// Stages of one batched product Y = A X (Sec. 2 "compressed system matrix", Sec. 4
// "System Matrix"): column-major X to the slab layout, forward transform at the leaves,
// upward transfer level by level, far-field coupling per target cluster, downward transfer
// level by level, backward transform per leaf, then per near-field row group the near
// product plus the gathered backward transforms, written back column-major.  Every kernel
// is deterministic: no atomics, fixed summation order.
#include "bem_batch.h"
#include "bem_device.h"

#include <type_traits>

namespace bem {

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef unsigned short u16x8 __attribute__((ext_vector_type(8)));

inline unsigned nblk(int64_t n, int per) { return (unsigned)((n + per - 1) / per); }
__device__ inline int nchunks(int R) { return (R + kBatchChunk - 1) / kBatchChunk; }

// conversions of a moment to the coupling's arithmetic type
template <class F>
__device__ inline F cvt(double v);
template <>
__device__ inline double cvt<double>(double v) { return v; }
template <>
__device__ inline float cvt<float>(double v) { return (float)v; }
template <class F>
__device__ inline F cvt(cdbl v);
template <>
__device__ inline cdbl cvt<cdbl>(cdbl v) { return v; }
template <>
__device__ inline cflt cvt<cflt>(cdbl v) { return {(float)v.re, (float)v.im}; }

__device__ inline double part_re(double v) { return v; }
__device__ inline double part_re(cdbl v) { return v.re; }
__device__ inline double part_im(double) { return 0.0; }
__device__ inline double part_im(cdbl v) { return v.im; }

// ------------------------------------------------------------------ slab transposes
// 64 DOFs x 32 right-hand sides per block through LDS
template <class T>
__global__ __launch_bounds__(256) void kb_to_slab(int64_t N, int R, const T* __restrict__ x, int64_t ldx,
                                                  T* __restrict__ xs) {
    __shared__ T tile[32][65];
    const int64_t g0 = (int64_t)blockIdx.x * 64;
    const int r0 = blockIdx.y * 32;
    {
        const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
        const int64_t g = g0 + tx;
        for (int i = ty; i < 32; i += 4)
            if (r0 + i < R && g < N) tile[i][tx] = x[g + (int64_t)(r0 + i) * ldx];
    }
    __syncthreads();
    const int tr = threadIdx.x & 31, tg = threadIdx.x >> 5;
    for (int i = tg; i < 64; i += 8)
        if (r0 + tr < R && g0 + i < N) xs[(g0 + i) * R + r0 + tr] = tile[tr][i];
}

template <class T>
__global__ __launch_bounds__(256) void kb_from_slab(int64_t N, int R, const T* __restrict__ ys, T* __restrict__ y,
                                                    int64_t ldy) {
    __shared__ T tile[32][65];
    const int64_t g0 = (int64_t)blockIdx.x * 64;
    const int r0 = blockIdx.y * 32;
    {
        const int tr = threadIdx.x & 31, tg = threadIdx.x >> 5;
        for (int i = tg; i < 64; i += 8)
            if (r0 + tr < R && g0 + i < N) tile[tr][i] = ys[(g0 + i) * R + r0 + tr];
    }
    __syncthreads();
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    const int64_t g = g0 + tx;
    for (int i = ty; i < 32; i += 4)
        if (r0 + i < R && g < N) y[g + (int64_t)(r0 + i) * ldy] = tile[i][tx];
}

// ------------------------------------------------------------------ coupling (vector units)
// Local expansion of target cluster t for 64 right-hand sides: l_t = sum over its
// admissible sources s of K_ts m_s, in the arithmetic type F (FP64, or FP32 from the FP32
// copy).  The four waves of a block take every fourth source; each wave stages the block
// K_ts (transposed when it is stored in the source's rows) in its LDS slice, with the
// next block already in flight in registers, and every lane applies it to its own
// right-hand side.  The four partial sums are added in wave order.
template <class T, class F, int Q>
__global__ __launch_bounds__(256) void kb_coupling(OpDev op, BatchDev bd, const F* __restrict__ K) {
    constexpr int Q2 = Q * Q;
    __shared__ F Ks[4][Q2 * Q2];
    __shared__ F red[Q2][kBatchChunk];
    const int nch = nchunks(bd.R);
    const int64_t t = blockIdx.x / nch;
    const int ch = blockIdx.x % nch;
    const int w = uniform_int(threadIdx.x >> 6), lane = threadIdx.x & 63;
    const int R = bd.R, r = ch * kBatchChunk + lane;
    const bool on = r < R;
    const int64_t beg = bd.far_rowptr[t], end = bd.far_rowptr[t + 1];
    const T* __restrict__ mom = (const T*)bd.mom;
    F* ks = Ks[w];
    F acc[Q2];
#pragma unroll
    for (int a = 0; a < Q2; ++a) acc[a] = zero_f<F>();
    // the next block's entries are loaded into registers while the current one is applied
    constexpr int KR = (Q2 * Q2 + kWave - 1) / kWave;  // block entries per lane
    F kreg[KR];
    auto load_block = [&](int64_t p) {
        const int64_t off = bd.fb_off[p];
        const int rs = bd.fb_rs[p];
        const int ars = rs < 0 ? -rs : rs;
#pragma unroll
        for (int u = 0; u < KR; ++u) {
            const int idx = lane + u * kWave;
            const int i = idx / Q2, jj = idx - i * Q2;
            kreg[u] = idx < Q2 * Q2 ? K[off + (int64_t)i * ars + jj] : zero_f<F>();
        }
    };
    int64_t p = beg + w;
    if (p < end) load_block(p);
    for (; p < end; p += 4) {
        const int s = bd.far_s[p];
        const bool tr = bd.fb_rs[p] < 0;
#pragma unroll
        for (int u = 0; u < KR; ++u) {
            const int idx = lane + u * kWave;
            const int i = idx / Q2, jj = idx - i * Q2;
            if (idx < Q2 * Q2) ks[tr ? jj * Q2 + i : idx] = kreg[u];
        }
        wave_sync();
        if (p + 4 < end) load_block(p + 4);
        const T* ms = mom + (int64_t)s * Q2 * R + r;
#pragma unroll 1
        for (int b0 = 0; b0 < Q2; b0 += Q) {
            F mv[Q];
#pragma unroll
            for (int u = 0; u < Q; ++u) mv[u] = on ? cvt<F>(ms[(int64_t)(b0 + u) * R]) : zero_f<F>();
#pragma unroll
            for (int a = 0; a < Q2; ++a)
#pragma unroll
                for (int u = 0; u < Q; ++u) acc[a] += ks[a * Q2 + b0 + u] * mv[u];
        }
        wave_sync();
    }
    for (int step = 0; step < 4; ++step) {
        if (w == step)
#pragma unroll
            for (int a = 0; a < Q2; ++a) red[a][lane] = step == 0 ? acc[a] : red[a][lane] + acc[a];
        __syncthreads();
    }
    if (w == 0 && on) {
        T* lv = (T*)bd.lv + t * Q2 * R + r;
#pragma unroll
        for (int a = 0; a < Q2; ++a) lv[(int64_t)a * R] = to_d(red[a][lane]);
    }
}

// ------------------------------------------------------------------ coupling (matrix cores)
// BF16 fragments.  v_mfma_f32_16x16x32_bf16: lane l holds A[l % 16][8 (l / 16) + e] and
// B[8 (l / 16) + e][l % 16], e = 0..7, and receives C[4 (l / 16) + e][l % 16], e = 0..3.
// A (one ordered block): rows = target nodes a (real), or [Re K; Im K] (complex), columns
// = source nodes b, zero-padded to 32.  B (one cluster, 64 right-hand sides): rows =
// source nodes b, columns = the right-hand sides (real) or [Re m | Im m] (complex).
template <class T, int Q>
__global__ __launch_bounds__(256) void kb_bf_blocks(OpDev op, BatchDev bd, int64_t npairs) {
    constexpr int Q2 = Q * Q;
    constexpr bool CP = sizeof(T) == 16;
    constexpr int RT = CP ? 4 : 2;
    const int64_t item = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (item >= npairs * RT) return;
    const int64_t p = item / RT;
    const int rt = (int)(item % RT);
    const int64_t off = bd.fb_off[p];
    const int rs = bd.fb_rs[p];
    const bool tr = rs < 0;
    const int ars = tr ? -rs : rs;
    const T* __restrict__ K = (const T*)op.K;
    const int row = 16 * rt + (lane & 15), k0 = 8 * (lane >> 4);
    const int a = row < Q2 ? row : row - Q2;
    const bool im = row >= Q2;
    u16x8 v;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        const int b = k0 + e;
        float x = 0.0f;
        if (b < Q2 && a < Q2 && (CP || !im)) {
            const T kv = K[off + (tr ? (int64_t)b * ars + a : (int64_t)a * ars + b)];
            x = (float)(im ? part_im(kv) : part_re(kv));
        }
        v[e] = f2bf(x);
    }
    ((u16x8*)bd.Af)[item * kWave + lane] = v;
}

template <class T, int Q>
__global__ __launch_bounds__(256) void kb_bf_moments(OpDev op, BatchDev bd) {
    constexpr int Q2 = Q * Q;
    constexpr bool CP = sizeof(T) == 16;
    constexpr int NT = CP ? 8 : 4;
    const int nch = nchunks(bd.R);
    const int64_t item = (int64_t)blockIdx.x * 4 + uniform_int(threadIdx.x >> 6);
    if (item >= op.ncl * nch) return;
    const int64_t c = item / nch;
    const int ch = (int)(item % nch);
    const int lane = threadIdx.x & 63, R = bd.R;
    const T* __restrict__ mom = (const T*)bd.mom + c * Q2 * R;
    const int k0 = 8 * (lane >> 4);
#pragma unroll 1
    for (int nt = 0; nt < NT; ++nt) {
        const int col = 16 * nt + (lane & 15);
        const bool im = CP && col >= kBatchChunk;
        const int r = ch * kBatchChunk + (im ? col - kBatchChunk : col);
        u16x8 v;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const int b = k0 + e;
            float x = 0.0f;
            if (b < Q2 && r < R) {
                const T mv = mom[(int64_t)b * R + r];
                x = (float)(im ? part_im(mv) : part_re(mv));
            }
            v[e] = f2bf(x);
        }
        ((u16x8*)bd.Bf)[(item * NT + nt) * kWave + lane] = v;
    }
}

// l_t = sum_s K_ts m_s on the matrix cores for 64 right-hand sides: per source one row of
// RT x NT MFMA tiles over a k-step of 32 (the q^2 <= 32 source nodes); the four waves of a
// block take every fourth source and their FP32 tiles are added in wave order in LDS.
template <class T, int Q>
__global__ __launch_bounds__(256) void kb_coupling_mfma(OpDev op, BatchDev bd) {
    constexpr int Q2 = Q * Q;
    static_assert(Q2 <= 32, "one k-step of 32 per block");
    constexpr bool CP = sizeof(T) == 16;
    constexpr int RT = CP ? 4 : 2, NT = CP ? 8 : 4;
    __shared__ float red[RT * 16][NT * 16 + 1];
    const int nch = nchunks(bd.R);
    const int64_t lb = xcd_block(blockIdx.x, gridDim.x);  // neighbouring blocks on one XCD
    const int64_t t = lb / nch;
    const int ch = (int)(lb % nch);
    const int w = uniform_int(threadIdx.x >> 6), lane = threadIdx.x & 63;
    const int64_t beg = bd.far_rowptr[t], end = bd.far_rowptr[t + 1];
    const u16x8* __restrict__ Af = (const u16x8*)bd.Af;
    const u16x8* __restrict__ Bf = (const u16x8*)bd.Bf;
    f32x4 acc[RT][NT];
#pragma unroll
    for (int i = 0; i < RT; ++i)
#pragma unroll
        for (int j = 0; j < NT; ++j) acc[i][j] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
    // fragments of the next source are loaded before the products of the current one
    u16x8 a[RT], b[NT];
    auto load = [&](int64_t p, u16x8* fa, u16x8* fb) {
        const int64_t s = bd.far_s[p];
#pragma unroll
        for (int i = 0; i < RT; ++i) fa[i] = Af[(p * RT + i) * kWave + lane];
#pragma unroll
        for (int j = 0; j < NT; ++j) fb[j] = Bf[((s * nch + ch) * NT + j) * kWave + lane];
    };
    int64_t p = beg + w;
    if (p < end) load(p, a, b);
    while (p < end) {
        const int64_t pn = p + 4;
        u16x8 an[RT], bn[NT];
        if (pn < end) load(pn, an, bn);
#pragma unroll
        for (int i = 0; i < RT; ++i)
#pragma unroll
            for (int j = 0; j < NT; ++j)
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a[i]),
                                                                    __builtin_bit_cast(bf16x8, b[j]), acc[i][j], 0, 0, 0);
        if (pn < end) {
#pragma unroll
            for (int i = 0; i < RT; ++i) a[i] = an[i];
#pragma unroll
            for (int j = 0; j < NT; ++j) b[j] = bn[j];
        }
        p = pn;
    }
    const int rq = 4 * (lane >> 4), cq = lane & 15;
    for (int step = 0; step < 4; ++step) {
        if (w == step)
#pragma unroll
            for (int i = 0; i < RT; ++i)
#pragma unroll
                for (int j = 0; j < NT; ++j)
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        float& dst = red[16 * i + rq + e][16 * j + cq];
                        dst = step == 0 ? acc[i][j][e] : dst + acc[i][j][e];
                    }
        __syncthreads();
    }
    T* lv = (T*)bd.lv + t * Q2 * bd.R;
    for (int idx = threadIdx.x; idx < Q2 * kBatchChunk; idx += blockDim.x) {
        const int a = idx / kBatchChunk, rl = idx % kBatchChunk, r = ch * kBatchChunk + rl;
        if (r >= bd.R) continue;
        if constexpr (CP) {
            // (Re K + i Im K)(Re m + i Im m)
            const double re = (double)red[a][rl] - (double)red[Q2 + a][kBatchChunk + rl];
            const double im = (double)red[a][kBatchChunk + rl] + (double)red[Q2 + a][rl];
            ((cdbl*)lv)[(int64_t)a * bd.R + r] = cdbl{re, im};
        } else {
            ((double*)lv)[(int64_t)a * bd.R + r] = (double)red[a][rl];
        }
    }
}

// ------------------------------------------------------------------ downward + backward
// Downward transfer and backward transform of one leaf: the leaf's local expansion plus
// those of all its ancestors carried down in one step each (l_leaf[p] += sum_a
// E^(k)_b1[p1][a1] E^(k)_b2[p2][a2] l_anc[a], E^(k) the leaf-to-ancestor transfer k levels
// up), then its contribution V_tau^T l_tau to each of the nloc^2 B-splines that meet it,
// stored per leaf (added per DOF by the near-field kernel).
template <class T, int Q>
__global__ __launch_bounds__(256) void kb_leaf_back(OpDev op, BatchDev bd) {
    constexpr int Q2 = Q * Q;
    const int nch = nchunks(bd.R);
    const int64_t item = (int64_t)blockIdx.x * 4 + uniform_int(threadIdx.x >> 6);
    if (item >= op.nleaves * nch) return;
    const int l = (int)(item / nch), ch = (int)(item % nch);
    const int R = bd.R, r = ch * kBatchChunk + (threadIdx.x & 63);
    if (r >= R) return;
    const int n1 = op.nleaf1, nloc = op.nloc;
    const int j = l % n1, i = (l / n1) % n1, f = l / (n1 * n1);
    const double* __restrict__ Vi = op.V1 + (int64_t)i * Q * nloc;
    const double* __restrict__ Vj = op.V1 + (int64_t)j * Q * nloc;
    const T* lvp = (const T*)bd.lv + (op.lev_off[op.leaf] + l) * Q2 * R + r;
    T v[Q2];
#pragma unroll
    for (int a = 0; a < Q2; ++a) v[a] = lvp[(int64_t)a * R];
    for (int k = 1; k <= op.leaf; ++k) {
        const int na = n1 >> k, b1 = i & ((1 << k) - 1), b2 = j & ((1 << k) - 1);
        const int64_t anc = op.lev_off[op.leaf - k] + ((int64_t)f * na + (i >> k)) * na + (j >> k);
        const double* __restrict__ Ek = bd.Ec + (int64_t)Q2 * ((1 << k) - 2);
        const T* vp = (const T*)bd.lv + anc * Q2 * R + r;
        T vall[Q2];
#pragma unroll
        for (int a = 0; a < Q2; ++a) vall[a] = vp[(int64_t)a * R];
#pragma unroll
        for (int a1 = 0; a1 < Q; ++a1) {
            T in[Q];
#pragma unroll
            for (int p2 = 0; p2 < Q; ++p2) in[p2] = zero<T>();
#pragma unroll
            for (int a2 = 0; a2 < Q; ++a2) {
                const T w = vall[a1 * Q + a2];
#pragma unroll
                for (int p2 = 0; p2 < Q; ++p2) in[p2] += Ek[(b2 * Q + p2) * Q + a2] * w;
            }
#pragma unroll
            for (int p1 = 0; p1 < Q; ++p1) {
                const double e = Ek[(b1 * Q + p1) * Q + a1];
#pragma unroll
                for (int p2 = 0; p2 < Q; ++p2) v[p1 * Q + p2] += e * in[p2];
            }
        }
    }
    T* yl = (T*)bd.yl + (int64_t)l * nloc * nloc * R + r;
    for (int m2 = 0; m2 < nloc; ++m2) {
        T t[Q];
#pragma unroll
        for (int a1 = 0; a1 < Q; ++a1) {
            T s = zero<T>();
#pragma unroll
            for (int a2 = 0; a2 < Q; ++a2) s += Vj[a2 * nloc + m2] * v[a1 * Q + a2];
            t[a1] = s;
        }
        for (int m1 = 0; m1 < nloc; ++m1) {
            T s = zero<T>();
#pragma unroll
            for (int a1 = 0; a1 < Q; ++a1) s += Vi[a1 * nloc + m1] * t[a1];
            yl[(int64_t)(m1 * nloc + m2) * R] = s;
        }
    }
}

// ------------------------------------------------------------------ near field + output
typedef double f64x4 __attribute__((ext_vector_type(4)));

__device__ inline f64x4 mfma64(double a, double b, f64x4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// value of the near field at (g, h), 0 outside the pattern (binary search in row g)
template <class T>
__device__ inline T near_at(const OpDev& op, const BatchDev& bd, int64_t g, int64_t h) {
    const int64_t b = op.rowptr[g], e = op.rowptr[g + 1];
    int64_t lo = b, hi = e;
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (op.col[mid] < h)
            lo = mid + 1;
        else
            hi = mid;
    }
    if (lo >= e || op.col[lo] != h) return zero<T>();
    const int64_t G = bd.row_grp[g];
    return ((const T*)op.val)[op.grp_voff[G] + (int64_t)bd.row_pos[g] * (e - b) + (lo - b)];
}

// dense tile values in fragment order (assembly; one block per tile)
template <class T>
__global__ __launch_bounds__(256) void kb_tile_fill(OpDev op, BatchDev bd) {
    const int64_t t = blockIdx.x;
    const int64_t rb = bd.tile_rowptr[t], cb = bd.tile_colptr[t];
    const int nr = (int)(bd.tile_rowptr[t + 1] - rb), C = (int)(bd.tile_colptr[t + 1] - cb);
    const int64_t v0 = bd.tile_voff[t], nv = bd.tile_voff[t + 1] - v0;
    T* out = (T*)bd.tile_val + v0;
    for (int64_t idx = threadIdx.x; idx < nv; idx += blockDim.x) {
        const int l = (int)(idx % kWave);
        const int row = l % 16, kc = (int)(idx / kWave) * 4 + l / 16;
        out[idx] = (row < nr && kc < C) ? near_at<T>(op, bd, bd.tile_rows[rb + row], bd.tile_cols[cb + kc]) : zero<T>();
    }
}

// Near field on the matrix cores (v_mfma_f64_16x16x4f64): one block per (tile, 64
// right-hand sides), wave w takes 16 of them.  Per step of 4 columns, lane l holds the tile
// value A[l % 16][l / 16] and x[column l / 16][rhs l % 16]; a complex product is four real
// products (Re, Im of A times Re, Im of x).  Four steps' fragments are loaded before their
// products; the tile's column indices are staged in LDS (up to kColStage at a time), so
// the x gathers of a round wait on one memory round trip, not two.  Epilogue: lane l
// holds rows l / 16 + 4 i,
// right-hand side l % 16; each adds the backward transforms of the leaves that meet its
// B-spline and is written to ys.
template <class T>
__global__ __launch_bounds__(256) void kb_near_mfma(OpDev op, BatchDev bd) {
    constexpr bool CP = sizeof(T) == 16;
    const int nch = nchunks(bd.R);
    const int64_t lb = xcd_block(blockIdx.x, gridDim.x);  // neighbouring blocks on one XCD
    const int64_t t = lb / nch;
    const int ch = (int)(lb % nch);
    const int w = uniform_int(threadIdx.x >> 6), lane = threadIdx.x & 63;
    const int R = bd.R;
    const int rb_n = ch * kBatchChunk + 16 * w;  // first right-hand side of this wave
    const int r = rb_n + (lane & 15);
    const bool on = r < R;
    const int64_t rb = bd.tile_rowptr[t], cb = bd.tile_colptr[t];
    const int nr = (int)(bd.tile_rowptr[t + 1] - rb), C = (int)(bd.tile_colptr[t + 1] - cb);
    const T* __restrict__ val = (const T*)bd.tile_val + bd.tile_voff[t] + lane;
    const int32_t* __restrict__ cols = bd.tile_cols + cb;
    const T* __restrict__ xs = (const T*)bd.xs;
    const int kk = lane >> 4;
    f64x4 ar = {0.0, 0.0, 0.0, 0.0}, ai = {0.0, 0.0, 0.0, 0.0};
    // DEPTH steps per round: all their value and x loads, then the products (steps past
    // the end carry zero values and a valid column)
    constexpr int DEPTH = 8;
    constexpr int kColStage = 1024;  // multiple of 4 DEPTH: a round never crosses a stage
    static_assert(kColStage % (4 * DEPTH) == 0, "whole rounds per stage");
    __shared__ int32_t cst[kColStage];
    for (int c0 = 0; c0 < C; c0 += kColStage) {
        const int cn = C - c0 < kColStage ? C - c0 : kColStage;
        __syncthreads();  // the previous stage's columns are no longer read
        for (int i = threadIdx.x; i < kColStage; i += blockDim.x) cst[i] = cols[c0 + (i < cn ? i : 0)];
        __syncthreads();
        const int sb = c0 / 4, se = (c0 + cn + 3) / 4;  // steps of this stage
        for (int s0 = sb; s0 < se; s0 += DEPTH) {
            T a[DEPTH], xv[DEPTH];
#pragma unroll
            for (int u = 0; u < DEPTH; ++u) {
                const int64_t h = cst[(s0 + u - sb) * 4 + kk];
                a[u] = s0 + u < se ? val[(int64_t)(s0 + u) * kWave] : zero<T>();
                xv[u] = on ? xs[h * R + r] : zero<T>();
            }
#pragma unroll
            for (int u = 0; u < DEPTH; ++u) {
                if constexpr (CP) {
                    const cdbl ac = *(const cdbl*)&a[u], xc = *(const cdbl*)&xv[u];
                    ar = mfma64(ac.re, xc.re, ar);
                    ar = mfma64(-ac.im, xc.im, ar);
                    ai = mfma64(ac.re, xc.im, ai);
                    ai = mfma64(ac.im, xc.re, ai);
                } else {
                    ar = mfma64(*(const double*)&a[u], *(const double*)&xv[u], ar);
                }
            }
        }
    }
    if (!on) return;
    const SpaceDesc& S = op.S;
    const int n1 = op.nleaf1, nloc = op.nloc, stride = op.m * S.r, nb = S.nb;
    const T* __restrict__ yl = (const T*)bd.yl;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int q = kk + 4 * i;  // v_mfma_f64_16x16x4f64: lane l holds rows l / 16 + 4 i
        if (q >= nr) continue;
        const int64_t g = bd.tile_rows[rb + q];
        const int j2 = (int)(g % nb), j1 = (int)((g / nb) % nb), f = (int)(g / ((int64_t)nb * nb));
        int lo1, hi1, lo2, hi2;
        leaf_range(j1, stride, nloc, n1, lo1, hi1);
        leaf_range(j2, stride, nloc, n1, lo2, hi2);
        T sum;
        if constexpr (CP)
            *(cdbl*)&sum = cdbl{ar[i], ai[i]};
        else
            *(double*)&sum = ar[i];
        for (int li = lo1; li <= hi1; ++li)
            for (int lj = lo2; lj <= hi2; ++lj) {
                const int64_t l = ((int64_t)f * n1 + li) * n1 + lj;
                const int m1 = j1 - li * stride, m2 = j2 - lj * stride;
                sum += yl[((l * nloc + m1) * nloc + m2) * R + r];
            }
        ((T*)bd.ys)[g * R + r] = sum;
    }
}

// ------------------------------------------------------------------ coupling (matrix cores, FP64 / FP32)
// One real MFMA step per arithmetic: v_mfma_f64_16x16x4f64 (lane l receives rows
// l / 16 + 4 e of column l % 16) or v_mfma_f32_16x16x4f32 (rows 4 (l / 16) + e); both take
// A[l % 16][l / 16] and B[l / 16][l % 16].
template <class Bt>
struct Mfma16;
template <>
struct Mfma16<double> {
    using acc = f64x4;
    __device__ static acc step(double a, double b, acc c) { return mfma64(a, b, c); }
    __device__ static int row(int kq, int e) { return kq + 4 * e; }
};
template <>
struct Mfma16<float> {
    using acc = f32x4;
    __device__ static acc step(float a, float b, acc c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
    __device__ static int row(int kq, int e) { return 4 * kq + e; }
};

// ------------------------------------------------------------------ forward + upward (matrix cores)
// Leaf moments m_tau[a][r] = sum over the nloc^2 B-splines g meeting the leaf of
// V_tau[a][g] x[g][r], V_tau[(a1, a2)][(m1, m2)] = V1_i[a1][m1] V1_j[a2][m2] (the 1-D moment
// tables of the two directions), as FP64 matrix-core steps: A = V_tau (rows a in tiles of
// 16, columns g in steps of 4), B = the slab rows of the leaf's B-splines for 16 right-hand
// sides per tile; a complex slab takes one real step per part.  One wave per leaf and
// 16 NTW right-hand sides.
template <class T, int Q, int NTW>
__global__ __launch_bounds__(256) void kb_leaf_moments(OpDev op, BatchDev bd) {
    constexpr int Q2 = Q * Q, RT = (Q2 + 15) / 16;
    constexpr bool CP = sizeof(T) == 16;
    const int R = bd.R, CW = 16 * NTW, ng = (R + CW - 1) / CW;
    const int64_t item = (int64_t)blockIdx.x * 4 + uniform_int(threadIdx.x >> 6);
    if (item >= op.nleaves * ng) return;
    const int l = (int)(item / ng), grp = (int)(item % ng);
    const int lane = threadIdx.x & 63, kq = lane >> 4, rl = lane & 15;
    const int n1 = op.nleaf1, nloc = op.nloc, stride = op.m * op.S.r, nl2 = nloc * nloc;
    const int j = l % n1, i = (l / n1) % n1, f = l / (n1 * n1);
    const double* __restrict__ Vi = op.V1 + (int64_t)i * Q * nloc;
    const double* __restrict__ Vj = op.V1 + (int64_t)j * Q * nloc;
    const T* __restrict__ xs = (const T*)bd.xs;
    int rr[NTW];
    bool on[NTW];
#pragma unroll
    for (int t = 0; t < NTW; ++t) {
        rr[t] = grp * CW + 16 * t + rl;
        on[t] = rr[t] < R;
    }
    f64x4 ar[RT][NTW], ai[RT][NTW];
#pragma unroll
    for (int u = 0; u < RT; ++u)
#pragma unroll
        for (int t = 0; t < NTW; ++t) ar[u][t] = ai[u][t] = f64x4{0.0, 0.0, 0.0, 0.0};
    for (int b0 = 0; b0 < nl2; b0 += 4) {
        const int b = b0 + kq;
        const bool bon = b < nl2;
        const int m1 = bon ? b / nloc : 0, m2 = bon ? b % nloc : 0;
        const int64_t g = dof_id(op.S, f, i * stride + m1, j * stride + m2);
        T xv[NTW];
#pragma unroll
        for (int t = 0; t < NTW; ++t) xv[t] = (bon && on[t]) ? xs[g * R + rr[t]] : zero<T>();
#pragma unroll
        for (int u = 0; u < RT; ++u) {
            const int a = 16 * u + rl;
            const double av = (bon && a < Q2) ? Vi[(a / Q) * nloc + m1] * Vj[(a % Q) * nloc + m2] : 0.0;
#pragma unroll
            for (int t = 0; t < NTW; ++t) {
                if constexpr (CP) {
                    ar[u][t] = mfma64(av, part_re(xv[t]), ar[u][t]);
                    ai[u][t] = mfma64(av, part_im(xv[t]), ai[u][t]);
                } else {
                    ar[u][t] = mfma64(av, *(const double*)&xv[t], ar[u][t]);
                }
            }
        }
    }
    T* mom = (T*)bd.mom + (op.lev_off[op.leaf] + l) * (int64_t)Q2 * R;
#pragma unroll
    for (int t = 0; t < NTW; ++t) {
        if (!on[t]) continue;
#pragma unroll
        for (int u = 0; u < RT; ++u)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int a = 16 * u + kq + 4 * e;
                if (a >= Q2) continue;
                if constexpr (CP)
                    ((cdbl*)mom)[(int64_t)a * R + rr[t]] = cdbl{ar[u][t][e], ai[u][t][e]};
                else
                    ((double*)mom)[(int64_t)a * R + rr[t]] = ar[u][t][e];
            }
    }
}

// Moments at level lev from the four children at lev + 1 (upward transfer):
// m_P[a][r] = sum over the children b and their nodes p of E_b1[p1][a1] E_b2[p2][a2]
// m_child[p][r], as FP64 matrix-core steps with A[(a1, a2)][(b, p)] formed from the two
// 1-D transfers and B the children's slab rows.  One wave per parent and 16 NTW
// right-hand sides.
template <class T, int Q, int NTW>
__global__ __launch_bounds__(256) void kb_upward(OpDev op, BatchDev bd, int lev) {
    constexpr int Q2 = Q * Q, RT = (Q2 + 15) / 16, KS = (4 * Q2 + 3) / 4;
    constexpr bool CP = sizeof(T) == 16;
    const int R = bd.R, CW = 16 * NTW, ng = (R + CW - 1) / CW;
    const int n = 1 << lev;
    const int64_t nl = (int64_t)op.S.geom.npatch * n * n;
    const int64_t item = (int64_t)blockIdx.x * 4 + uniform_int(threadIdx.x >> 6);
    const int64_t loc = item / ng;
    const int grp = (int)(item % ng);
    const int lane = threadIdx.x & 63, kq = lane >> 4, rl = lane & 15;
    const int f = (int)(loc / ((int64_t)n * n)), i = (int)((loc / n) % n), j = (int)(loc % n);
    __shared__ double Es[2 * Q * Q];
    for (int idx = threadIdx.x; idx < 2 * Q * Q; idx += blockDim.x) Es[idx] = op.E[idx];
    __syncthreads();
    if (item >= nl * ng) return;
    const T* __restrict__ mom = (const T*)bd.mom;
    int rr[NTW];
    bool on[NTW];
#pragma unroll
    for (int t = 0; t < NTW; ++t) {
        rr[t] = grp * CW + 16 * t + rl;
        on[t] = rr[t] < R;
    }
    // all of the lane's slab values first (independent loads in flight), then the steps
    T mv[KS][NTW];
#pragma unroll
    for (int k = 0; k < KS; ++k) {
        const int kk = 4 * k + kq;  // (child, node) = (kk / Q2, kk % Q2)
        const int b = kk / Q2, p = kk % Q2;
        const int64_t ch = op.lev_off[lev + 1] + ((int64_t)f * 2 * n + 2 * i + (b >> 1)) * 2 * n + 2 * j + (b & 1);
#pragma unroll
        for (int t = 0; t < NTW; ++t) mv[k][t] = on[t] ? mom[(ch * Q2 + p) * R + rr[t]] : zero<T>();
    }
    f64x4 ar[RT][NTW], ai[RT][NTW];
#pragma unroll
    for (int u = 0; u < RT; ++u)
#pragma unroll
        for (int t = 0; t < NTW; ++t) ar[u][t] = ai[u][t] = f64x4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int k = 0; k < KS; ++k) {
        const int kk = 4 * k + kq;
        const int b = kk / Q2, p = kk % Q2, b1 = b >> 1, b2 = b & 1;
#pragma unroll
        for (int u = 0; u < RT; ++u) {
            const int a = 16 * u + rl;
            const double av =
                a < Q2 ? Es[(b1 * Q + p / Q) * Q + a / Q] * Es[(b2 * Q + p % Q) * Q + a % Q] : 0.0;
#pragma unroll
            for (int t = 0; t < NTW; ++t) {
                if constexpr (CP) {
                    ar[u][t] = mfma64(av, part_re(mv[k][t]), ar[u][t]);
                    ai[u][t] = mfma64(av, part_im(mv[k][t]), ai[u][t]);
                } else {
                    ar[u][t] = mfma64(av, *(const double*)&mv[k][t], ar[u][t]);
                }
            }
        }
    }
    T* out = (T*)bd.mom + (op.lev_off[lev] + loc) * (int64_t)Q2 * R;
#pragma unroll
    for (int t = 0; t < NTW; ++t) {
        if (!on[t]) continue;
#pragma unroll
        for (int u = 0; u < RT; ++u)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int a = 16 * u + kq + 4 * e;
                if (a >= Q2) continue;
                if constexpr (CP)
                    ((cdbl*)out)[(int64_t)a * R + rr[t]] = cdbl{ar[u][t][e], ai[u][t][e]};
                else
                    ((double*)out)[(int64_t)a * R + rr[t]] = ar[u][t][e];
            }
    }
}

// l_t = sum_s K_ts m_s on the matrix cores for 64 NTW right-hand sides, in FP64 (F = T,
// the stored blocks) or FP32 (F = float / cflt, the FP32 copy; moments rounded to FP32,
// FP32 accumulation).  The block walks the sources of t in order; every source's block
// K_ts is staged once in LDS (transposed when it is stored in the source's rows; double
// buffered, the next block in flight in registers during the products) and wave w takes
// NTW column tiles of 16 right-hand sides.  Per step of 4 source nodes b, lane l takes
// A[16 i + l % 16][b] from the staged block and B[b][l % 16] of each column tile from the
// moments' slab (zero past q^2); a complex product is four real products.
// the moments' slab rounded to FP32 (read by the FP32 coupling at half the bytes)
template <class T, class F>
__global__ __launch_bounds__(256) void kb_moments_low(int64_t n, const T* __restrict__ m, F* __restrict__ ml) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) ml[i] = cvt<F>(m[i]);
}

template <class T, class F, int Q, int NTW>
__global__ __launch_bounds__(256) void kb_coupling_mx(OpDev op, BatchDev bd, const F* __restrict__ K) {
    constexpr int Q2 = Q * Q;
    constexpr bool CP = sizeof(T) == 16;
    using Bt = typename std::conditional<sizeof(F) == 4 || (sizeof(F) == 8 && CP), float, double>::type;
    using M = Mfma16<Bt>;
    using A4 = typename M::acc;
    constexpr int RT = (Q2 + 15) / 16, KS = (Q2 + 3) / 4, CW = 64 * NTW;
    constexpr int KR = (Q2 * Q2 + 255) / 256;  // block entries per thread
    __shared__ F ks[2][Q2 * Q2];
    const int nch = (bd.R + CW - 1) / CW;
    // consecutive targets (siblings, sharing most of their sources' moments) on one XCD
    const int64_t lb = xcd_block(blockIdx.x, gridDim.x);
    const int64_t t = lb / nch;
    const int ch = (int)(lb % nch);
    const int w = uniform_int(threadIdx.x >> 6), lane = threadIdx.x & 63;
    const int R = bd.R, kq = lane >> 4, rl = lane & 15;
    int rr[NTW];
    bool on[NTW];
#pragma unroll
    for (int j = 0; j < NTW; ++j) {
        rr[j] = ch * CW + 16 * (w * NTW + j) + rl;  // this lane's right-hand sides
        on[j] = rr[j] < R;
    }
    const int64_t beg = bd.far_rowptr[t], end = bd.far_rowptr[t + 1];
    // FP32 arithmetic reads the FP32 copy of the moments when there is one
    constexpr bool kLow = sizeof(F) < sizeof(T);
    const T* __restrict__ mom = (const T*)bd.mom;
    const F* __restrict__ moml = (const F*)bd.mlow;
    A4 ar[RT][NTW], ai[RT][NTW];
#pragma unroll
    for (int i = 0; i < RT; ++i)
#pragma unroll
        for (int j = 0; j < NTW; ++j) ar[i][j] = ai[i][j] = A4{0, 0, 0, 0};
    F kreg[KR];
    auto load_block = [&](int64_t p) {
        const int64_t off = bd.fb_off[p];
        const int rs = bd.fb_rs[p];
        const int ars = rs < 0 ? -rs : rs;
#pragma unroll
        for (int u = 0; u < KR; ++u) {
            const int idx = threadIdx.x + u * 256;
            const int i = idx / Q2, jj = idx - i * Q2;
            kreg[u] = idx < Q2 * Q2 ? K[off + (int64_t)i * ars + jj] : zero_f<F>();
        }
    };
    auto store_block = [&](int64_t p, F* dst) {
        const bool tr = bd.fb_rs[p] < 0;
#pragma unroll
        for (int u = 0; u < KR; ++u) {
            const int idx = threadIdx.x + u * 256;
            const int i = idx / Q2, jj = idx - i * Q2;
            if (idx < Q2 * Q2) dst[tr ? jj * Q2 + i : idx] = kreg[u];
        }
    };
    int buf = 0;
    if (beg < end) {
        load_block(beg);
        store_block(beg, ks[0]);
    }
    __syncthreads();
    for (int64_t p = beg; p < end; ++p) {
        if (p + 1 < end) load_block(p + 1);
        const int64_t mo = (int64_t)bd.far_s[p] * Q2 * R;
        const F* kb = ks[buf];
        F bv[KS][NTW];
#pragma unroll
        for (int k = 0; k < KS; ++k) {
            const int b = 4 * k + kq;
#pragma unroll
            for (int j = 0; j < NTW; ++j) {
                const int64_t idx = mo + (int64_t)b * R + rr[j];
                bv[k][j] = !(b < Q2 && on[j]) ? zero_f<F>() : (kLow && moml ? moml[idx] : cvt<F>(mom[idx]));
            }
        }
#pragma unroll
        for (int k = 0; k < KS; ++k) {
            const int b = 4 * k + kq;
#pragma unroll
            for (int i = 0; i < RT; ++i) {
                const int a = 16 * i + rl;
                const F av = (a < Q2 && b < Q2) ? kb[a * Q2 + b] : zero_f<F>();
#pragma unroll
                for (int j = 0; j < NTW; ++j) {
                    if constexpr (CP) {
                        ar[i][j] = M::step(av.re, bv[k][j].re, ar[i][j]);
                        ar[i][j] = M::step(-av.im, bv[k][j].im, ar[i][j]);
                        ai[i][j] = M::step(av.re, bv[k][j].im, ai[i][j]);
                        ai[i][j] = M::step(av.im, bv[k][j].re, ai[i][j]);
                    } else {
                        ar[i][j] = M::step(av, bv[k][j], ar[i][j]);
                    }
                }
            }
        }
        if (p + 1 < end) store_block(p + 1, ks[buf ^ 1]);
        __syncthreads();
        buf ^= 1;
    }
    T* lv = (T*)bd.lv + t * Q2 * R;
#pragma unroll
    for (int j = 0; j < NTW; ++j) {
        if (!on[j]) continue;
#pragma unroll
        for (int i = 0; i < RT; ++i)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int a = 16 * i + M::row(kq, e);
                if (a >= Q2) continue;
                if constexpr (CP)
                    ((cdbl*)lv)[(int64_t)a * R + rr[j]] = cdbl{(double)ar[i][j][e], (double)ai[i][j][e]};
                else
                    ((double*)lv)[(int64_t)a * R + rr[j]] = (double)ar[i][j][e];
            }
    }
}

// ------------------------------------------------------------------ launchers
template <class T, int Q>
hipError_t stage_tq(const OpDev& op, const BatchDev& bd, int stage, const void* x, int64_t ldx, void* y, int64_t ldy,
                    int prec, hipStream_t st) {
    const int R = bd.R, nch = (R + kBatchChunk - 1) / kBatchChunk;
    const int64_t N = op.S.ndof;
    if (stage == 0) {
        if (x)
            hipLaunchKernelGGL(kb_to_slab<T>, dim3(nblk(N, 64), nblk(R, 32)), dim3(256), 0, st, N, R, (const T*)x, ldx,
                               (T*)bd.xs);
        constexpr int NTW = 2;  // 32 right-hand sides per wave
        const int ng = (R + 16 * NTW - 1) / (16 * NTW);
        hipLaunchKernelGGL((kb_leaf_moments<T, Q, NTW>), dim3(nblk(op.nleaves * ng, 4)), dim3(256), 0, st, op, bd);
        for (int lev = op.leaf - 1; lev >= 0; --lev) {
            const int64_t nl = (int64_t)op.S.geom.npatch << (2 * lev);
            hipLaunchKernelGGL((kb_upward<T, Q, NTW>), dim3(nblk(nl * ng, 4)), dim3(256), 0, st, op, bd, lev);
        }
        if (prec == 2) hipLaunchKernelGGL((kb_bf_moments<T, Q>), dim3(nblk(op.ncl * nch, 4)), dim3(256), 0, st, op, bd);
        if (prec == 1 && bd.mlow) {
            using F32 = typename std::conditional<sizeof(T) == 16, cflt, float>::type;
            const int64_t nm = op.ncl * op.q2 * (int64_t)R;
            hipLaunchKernelGGL((kb_moments_low<T, F32>), dim3(nblk(nm, 256)), dim3(256), 0, st, nm, (const T*)bd.mom,
                               (F32*)bd.mlow);
        }
    } else if (stage == 1) {
        const unsigned nb = (unsigned)(op.ncl * nch);
        using F32 = typename std::conditional<sizeof(T) == 16, cflt, float>::type;
        // 128 right-hand sides per block once there are more than 64
        const unsigned nb2 = (unsigned)(op.ncl * ((R + 127) / 128));
        if (prec == 0) {
            if constexpr (Q * Q <= 28) {
                if (R > kBatchChunk)
                    hipLaunchKernelGGL((kb_coupling_mx<T, T, Q, 2>), dim3(nb2), dim3(256), 0, st, op, bd, (const T*)op.K);
                else
                    hipLaunchKernelGGL((kb_coupling_mx<T, T, Q, 1>), dim3(nb), dim3(256), 0, st, op, bd, (const T*)op.K);
            } else {
                hipLaunchKernelGGL((kb_coupling<T, T, Q>), dim3(nb), dim3(256), 0, st, op, bd, (const T*)op.K);
            }
        } else if (prec == 1) {
            if constexpr (Q * Q <= 28) {
                if (R > kBatchChunk)
                    hipLaunchKernelGGL((kb_coupling_mx<T, F32, Q, 2>), dim3(nb2), dim3(256), 0, st, op, bd,
                                       (const F32*)op.Klow);
                else
                    hipLaunchKernelGGL((kb_coupling_mx<T, F32, Q, 1>), dim3(nb), dim3(256), 0, st, op, bd,
                                       (const F32*)op.Klow);
            } else {
                hipLaunchKernelGGL((kb_coupling<T, F32, Q>), dim3(nb), dim3(256), 0, st, op, bd, (const F32*)op.Klow);
            }
        } else {
            if constexpr (Q * Q <= 32)
                hipLaunchKernelGGL((kb_coupling_mfma<T, Q>), dim3(nb), dim3(256), 0, st, op, bd);
            else
                return hipErrorInvalidValue;
        }
    } else if (stage == 2) {
        hipLaunchKernelGGL((kb_leaf_back<T, Q>), dim3(nblk(op.nleaves * nch, 4)), dim3(256), 0, st, op, bd);
    } else {
        hipLaunchKernelGGL(kb_near_mfma<T>, dim3((unsigned)(bd.ntiles * nch)), dim3(256), 0, st, op, bd);
        if (y)
            hipLaunchKernelGGL(kb_from_slab<T>, dim3(nblk(N, 64), nblk(R, 32)), dim3(256), 0, st, N, R,
                               (const T*)bd.ys, (T*)y, ldy);
    }
    return hipGetLastError();
}

template <class T>
hipError_t stage_t(const OpDev& op, const BatchDev& bd, int stage, const void* x, int64_t ldx, void* y, int64_t ldy,
                   int prec, hipStream_t st) {
    switch (op.q) {
        case 1: return stage_tq<T, 1>(op, bd, stage, x, ldx, y, ldy, prec, st);
        case 2: return stage_tq<T, 2>(op, bd, stage, x, ldx, y, ldy, prec, st);
        case 3: return stage_tq<T, 3>(op, bd, stage, x, ldx, y, ldy, prec, st);
        case 4: return stage_tq<T, 4>(op, bd, stage, x, ldx, y, ldy, prec, st);
        case 5: return stage_tq<T, 5>(op, bd, stage, x, ldx, y, ldy, prec, st);
        case 6: return stage_tq<T, 6>(op, bd, stage, x, ldx, y, ldy, prec, st);
        default: return hipErrorInvalidValue;
    }
}

template <class T, int Q>
hipError_t bf_blocks_tq(const OpDev& op, const BatchDev& bd, int64_t npairs, hipStream_t st) {
    if constexpr (Q * Q <= 32) {
        const int RT = bf_row_tiles(sizeof(T) == 16);
        hipLaunchKernelGGL((kb_bf_blocks<T, Q>), dim3(nblk(npairs * RT, 4)), dim3(256), 0, st, op, bd, npairs);
        return hipGetLastError();
    } else {
        return hipErrorInvalidValue;
    }
}

}  // namespace

hipError_t launch_apply_batched_stage(const OpDev& op, const BatchDev& bd, int stage, const void* x, int64_t ldx,
                                      void* y, int64_t ldy, int prec, hipStream_t st) {
    if (bd.R < 1 || bd.R > bd.rmax) return hipErrorInvalidValue;
    return op.cplx ? stage_t<cdbl>(op, bd, stage, x, ldx, y, ldy, prec, st)
                   : stage_t<double>(op, bd, stage, x, ldx, y, ldy, prec, st);
}

hipError_t launch_apply_batched(const OpDev& op, const BatchDev& bd, const void* x, int64_t ldx, void* y, int64_t ldy,
                                int prec, hipStream_t st) {
    for (int s = 0; s < kBatchStages; ++s) {
        const hipError_t e = launch_apply_batched_stage(op, bd, s, x, ldx, y, ldy, prec, st);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_to_slab(int cplx, int64_t N, int R, const void* x, int64_t ldx, void* xs, hipStream_t st) {
    const dim3 g(nblk(N, 64), nblk(R, 32));
    if (cplx)
        hipLaunchKernelGGL(kb_to_slab<cdbl>, g, dim3(256), 0, st, N, R, (const cdbl*)x, ldx, (cdbl*)xs);
    else
        hipLaunchKernelGGL(kb_to_slab<double>, g, dim3(256), 0, st, N, R, (const double*)x, ldx, (double*)xs);
    return hipGetLastError();
}

hipError_t launch_from_slab(int cplx, int64_t N, int R, const void* ys, void* y, int64_t ldy, hipStream_t st) {
    const dim3 g(nblk(N, 64), nblk(R, 32));
    if (cplx)
        hipLaunchKernelGGL(kb_from_slab<cdbl>, g, dim3(256), 0, st, N, R, (const cdbl*)ys, (cdbl*)y, ldy);
    else
        hipLaunchKernelGGL(kb_from_slab<double>, g, dim3(256), 0, st, N, R, (const double*)ys, (double*)y, ldy);
    return hipGetLastError();
}

hipError_t launch_tile_fill(const OpDev& op, const BatchDev& bd, hipStream_t st) {
    if (bd.ntiles == 0) return hipSuccess;
    if (op.cplx)
        hipLaunchKernelGGL(kb_tile_fill<cdbl>, dim3((unsigned)bd.ntiles), dim3(256), 0, st, op, bd);
    else
        hipLaunchKernelGGL(kb_tile_fill<double>, dim3((unsigned)bd.ntiles), dim3(256), 0, st, op, bd);
    return hipGetLastError();
}

hipError_t launch_build_bf_blocks(const OpDev& op, const BatchDev& bd, int64_t npairs, hipStream_t st) {
    if (npairs == 0) return hipSuccess;
    if (op.cplx) {
        switch (op.q) {
            case 1: return bf_blocks_tq<cdbl, 1>(op, bd, npairs, st);
            case 2: return bf_blocks_tq<cdbl, 2>(op, bd, npairs, st);
            case 3: return bf_blocks_tq<cdbl, 3>(op, bd, npairs, st);
            case 4: return bf_blocks_tq<cdbl, 4>(op, bd, npairs, st);
            case 5: return bf_blocks_tq<cdbl, 5>(op, bd, npairs, st);
            default: return hipErrorInvalidValue;
        }
    }
    switch (op.q) {
        case 1: return bf_blocks_tq<double, 1>(op, bd, npairs, st);
        case 2: return bf_blocks_tq<double, 2>(op, bd, npairs, st);
        case 3: return bf_blocks_tq<double, 3>(op, bd, npairs, st);
        case 4: return bf_blocks_tq<double, 4>(op, bd, npairs, st);
        case 5: return bf_blocks_tq<double, 5>(op, bd, npairs, st);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace bem
