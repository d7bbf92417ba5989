// gfx950 kernels of the block-Jacobi preconditioner and its learned correction (see
// bem_precond.h).  Not part of the paper's method (its example solves with unpreconditioned
// GMRES); added to cut GMRES iterations on the first-kind single-layer systems.
#include "bem_precond.h"
#include "bem_device.h"

namespace bem {

namespace {

inline unsigned nblk(int64_t n, int per) { return (unsigned)((n + per - 1) / per); }

__device__ inline double absval(double v) { return fabs(v); }
__device__ inline double absval(cdbl v) { return sqrt(v.re * v.re + v.im * v.im); }
__device__ inline double inv_(double v) { return 1.0 / v; }
__device__ inline cdbl inv_(cdbl v) {
    const double d = v.re * v.re + v.im * v.im;
    return {v.re / d, -v.im / d};
}
__device__ inline cdbl neg(cdbl v) { return {-v.re, -v.im}; }
__device__ inline double neg(double v) { return -v; }
template <class T>
__device__ inline T one();
template <>
__device__ inline double one<double>() { return 1.0; }
template <>
__device__ inline cdbl one<cdbl>() { return {1.0, 0.0}; }

// tile and slot of DOF g; false if g is not in a tile (never for g < ndof)
__device__ inline void tile_of(const SpaceDesc& S, int nt, int64_t g, int64_t& tb, int& slot) {
    const int nb = S.nb;
    const int j2 = (int)(g % nb), j1 = (int)((g / nb) % nb), f = (int)(g / ((int64_t)nb * nb));
    tb = ((int64_t)f * nt + j1 / kTile) * nt + j2 / kTile;
    slot = (j1 % kTile) * kTile + j2 % kTile;
}
// DOF of slot l of tile tb, or -1 for an unused slot of a short tile
__device__ inline int64_t slot_dof(const SpaceDesc& S, int nt, int64_t tb, int l) {
    const int t2 = (int)(tb % nt), t1 = (int)((tb / nt) % nt), f = (int)(tb / ((int64_t)nt * nt));
    const int j1 = t1 * kTile + l / kTile, j2 = t2 * kTile + l % kTile;
    if (j1 >= S.nb || j2 >= S.nb) return -1;
    return dof_id(S, f, j1, j2);
}

// ------------------------------------------------------------------ block extraction
// D_b = 0, with the unused slots of short tiles set to identity
template <class T>
__global__ __launch_bounds__(256) void kp_init(OpDev op, PrecDev pc) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= pc.ntiles * kTileN * kTileN) return;
    const int64_t tb = i / (kTileN * kTileN);
    const int r = (int)((i / kTileN) % kTileN), c = (int)(i % kTileN);
    T v = zero<T>();
    if (r == c && slot_dof(op.S, pc.nt, tb, r) < 0) v = one<T>();
    ((T*)pc.D0inv)[i] = v;
}

// near-field entries (g, h) with g and h in the same tile: one wave per row group
template <class T>
__global__ __launch_bounds__(256) void kp_extract(OpDev op, PrecDev pc) {
    const int64_t G = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (G >= op.ngroups) return;
    const int64_t rb = op.grp_rowptr[G];
    const int Rg = (int)(op.grp_rowptr[G + 1] - rb);
    const int64_t first = op.grp_rows[rb];
    const int64_t cb = op.rowptr[first];
    const int C = (int)(op.rowptr[first + 1] - cb);
    const T* val = (const T*)op.val + op.grp_voff[G];
    T* D = (T*)pc.D0inv;
    for (int q = 0; q < Rg; ++q) {
        int64_t tg;
        int lg;
        tile_of(op.S, pc.nt, op.grp_rows[rb + q], tg, lg);
        for (int c = lane; c < C; c += kWave) {
            int64_t th;
            int lh;
            tile_of(op.S, pc.nt, op.col[cb + c], th, lh);
            if (th == tg) D[(tg * kTileN + lg) * kTileN + lh] = val[(int64_t)q * C + c];
        }
    }
}

// ------------------------------------------------------------------ inversion
// In-place Gauss-Jordan inversion of the 64 x 64 matrix a (LDS) with partial pivoting
// (largest modulus in the column) by the whole block; the row interchanges are undone as
// column interchanges in reverse order.  status[0] = 1 on a zero pivot.
template <class T>
__device__ void gj_invert(T (*a)[kTileN + 1], T* colk, int* perm, int* piv_s, int* status) {
    for (int k = 0; k < kTileN; ++k) {
        if (threadIdx.x < 64) {
            const int i = threadIdx.x;
            double v = i >= k ? absval(a[i][k]) : -1.0;
            int p = i;
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) {
                const double v2 = __shfl_xor(v, o, 64);
                const int p2 = __shfl_xor(p, o, 64);
                if (v2 > v || (v2 == v && p2 < p)) {
                    v = v2;
                    p = p2;
                }
            }
            if (i == 0) {
                *piv_s = p;
                perm[k] = p;
                if (v == 0.0) status[0] = 1;
            }
        }
        __syncthreads();
        const int p = *piv_s;
        if (p != k)
            for (int j = threadIdx.x; j < kTileN; j += blockDim.x) {
                const T tmp = a[k][j];
                a[k][j] = a[p][j];
                a[p][j] = tmp;
            }
        __syncthreads();
        const T inv = inv_(a[k][k]);
        __syncthreads();
        for (int j = threadIdx.x; j < kTileN; j += blockDim.x) a[k][j] = j == k ? inv : a[k][j] * inv;
        for (int i = threadIdx.x; i < kTileN; i += blockDim.x) colk[i] = a[i][k];
        __syncthreads();
        for (int idx = threadIdx.x; idx < kTileN * kTileN; idx += blockDim.x) {
            const int i = idx / kTileN, j = idx % kTileN;
            if (i == k) continue;
            if (j == k)
                a[i][k] = neg(colk[i] * inv);
            else
                a[i][j] -= colk[i] * a[k][j];
        }
        __syncthreads();
    }
    for (int k = kTileN - 1; k >= 0; --k) {
        const int p = perm[k];
        if (p != k)
            for (int i = threadIdx.x; i < kTileN; i += blockDim.x) {
                const T tmp = a[i][k];
                a[i][k] = a[i][p];
                a[i][p] = tmp;
            }
        __syncthreads();
    }
}

template <class T>
__global__ __launch_bounds__(256) void kp_invert(PrecDev pc) {
    __shared__ T a[kTileN][kTileN + 1];
    __shared__ T colk[kTileN];
    __shared__ int perm[kTileN];
    __shared__ int piv_s;
    const int64_t tb = blockIdx.x;
    T* src = (T*)pc.D0inv + tb * kTileN * kTileN;
    for (int i = threadIdx.x; i < kTileN * kTileN; i += 256) a[i / kTileN][i % kTileN] = src[i];
    __syncthreads();
    gj_invert<T>(a, colk, perm, &piv_s, pc.status);
    T* dst0 = (T*)pc.D0inv + tb * kTileN * kTileN;
    T* dst1 = (T*)pc.Dinv + tb * kTileN * kTileN;
    double fro = 0.0;
    for (int i = threadIdx.x; i < kTileN * kTileN; i += 256) {
        const T v = a[i / kTileN][i % kTileN];
        dst0[i] = v;
        dst1[i] = v;
        fro += absval(v) * absval(v);
    }
    // s_b = ||D_b^{-1}||_F / 64: block sum in a fixed order
    __shared__ double red[256];
    red[threadIdx.x] = fro;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) pc.scale[tb] = sqrt(red[0]) / kTileN;
}

// ------------------------------------------------------------------ apply
// z_b = Dinv_b r_b on slabs: one block per (tile, 64 right-hand sides); the inverse is
// staged in LDS, the four waves take 16 rows each, lanes are right-hand sides
template <class T>
__global__ __launch_bounds__(256) void kp_apply(OpDev op, PrecDev pc, int R, const T* __restrict__ r,
                                                T* __restrict__ z) {
    __shared__ T a[kTileN][kTileN];
    __shared__ int64_t dof[kTileN];
    const int nch = (R + 63) / 64;
    const int64_t tb = blockIdx.x / nch;
    const int ch = blockIdx.x % nch;
    const T* src = (const T*)pc.Dinv + tb * kTileN * kTileN;
    for (int i = threadIdx.x; i < kTileN * kTileN; i += 256) a[i / kTileN][i % kTileN] = src[i];
    if (threadIdx.x < kTileN) dof[threadIdx.x] = slot_dof(op.S, pc.nt, tb, threadIdx.x);
    __syncthreads();
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63, rr = ch * 64 + lane;
    if (rr >= R) return;
    T acc[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) acc[i] = zero<T>();
    for (int j = 0; j < kTileN; ++j) {
        const int64_t h = dof[j];
        if (h < 0) continue;
        const T v = r[h * R + rr];
#pragma unroll
        for (int i = 0; i < 16; ++i) acc[i] += a[16 * w + i][j] * v;
    }
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        const int64_t g = dof[16 * w + i];
        if (g >= 0) z[g * R + rr] = acc[i];
    }
}

// ------------------------------------------------------------------ features
// Per tile: the parameter box of the elements its B-splines meet; at 4 x 4 points (cell
// centres of a uniform 4 x 4 grid of the box) the Jacobian of the patch map with respect to
// the box coordinates (central differences of the analytic map), then Re k, Im k, level.
__global__ __launch_bounds__(64) void kp_features(OpDev op, PrecDev pc, float* feats) {
    const int64_t tb = blockIdx.x;
    const int p = threadIdx.x;
    const SpaceDesc& S = op.S;
    const int nt = pc.nt;
    const int t2 = (int)(tb % nt), t1 = (int)((tb / nt) % nt), f = (int)(tb / ((int64_t)nt * nt));
    auto box = [&](int t, double& lo, double& hi) {
        const int ja = t * kTile, jb = min((t + 1) * kTile, S.nb) - 1;
        int elo = ja - S.d <= 0 ? 0 : (ja - S.d + S.r - 1) / S.r;
        int ehi = min(jb / S.r, S.nel - 1);
        lo = elo * S.h;
        hi = (ehi + 1) * S.h;
    };
    double s0, s1, u0, u1;
    box(t1, s0, s1);
    box(t2, u0, u1);
    float* out = feats + tb * kFeat;
    if (p < 16) {
        const int i1 = p / 4, i2 = p % 4;
        const double s = s0 + (i1 + 0.5) * 0.25 * (s1 - s0), t = u0 + (i2 + 0.5) * 0.25 * (u1 - u0);
        const double dl = 1e-6;
        double xp[3], xm[3], yp[3], ym[3];
        patch_point(S.geom, f, s + dl, t, xp);
        patch_point(S.geom, f, s - dl, t, xm);
        patch_point(S.geom, f, s, t + dl, yp);
        patch_point(S.geom, f, s, t - dl, ym);
        for (int k = 0; k < 3; ++k) {
            out[p * 6 + k] = (float)((xp[k] - xm[k]) / (2.0 * dl) * (s1 - s0));
            out[p * 6 + 3 + k] = (float)((yp[k] - ym[k]) / (2.0 * dl) * (u1 - u0));
        }
    }
    if (p == 16) {
        out[96] = (float)(S.ker.kre / 10.0);
        out[97] = (float)(S.ker.kim / 10.0);
        out[98] = (float)(S.L / 8.0);
    }
}

// ------------------------------------------------------------------ training targets
// Neighbourhood N(b): the tile extended by `ring` B-spline indices on each side inside the
// patch, DOFs j1 outer, j2 inner.
struct Nbhd {
    int f, j1a, j1b, j2a, j2b, n;
    __device__ int64_t dof(const SpaceDesc& S, int i) const {
        const int w2 = j2b - j2a;
        return dof_id(S, f, j1a + i / w2, j2a + i % w2);
    }
};
__device__ inline Nbhd nbhd_of(const SpaceDesc& S, int nt, int64_t tb, int ring) {
    const int t2 = (int)(tb % nt), t1 = (int)((tb / nt) % nt), f = (int)(tb / ((int64_t)nt * nt));
    Nbhd N;
    N.f = f;
    N.j1a = max(0, t1 * kTile - ring);
    N.j1b = min(S.nb, (t1 + 1) * kTile + ring);
    N.j2a = max(0, t2 * kTile - ring);
    N.j2b = min(S.nb, (t2 + 1) * kTile + ring);
    N.n = (N.j1b - N.j1a) * (N.j2b - N.j2a);
    return N;
}

// near-field value A[g][h] (0 if h is not in row g's pattern): binary search in the row
template <class T>
__device__ inline T near_entry(const OpDev& op, const int64_t* grp_of_row, const int32_t* pos_of_row, int64_t g,
                               int64_t h) {
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
    const int64_t G = grp_of_row[g];
    return ((const T*)op.val)[op.grp_voff[G] + (int64_t)pos_of_row[g] * (e - b) + (lo - b)];
}

__device__ inline double conj_(double v) { return v; }
__device__ inline cdbl conj_(cdbl v) { return {v.re, -v.im}; }

// Block least-squares approximate inverse of one tile (one block per tile):
// X_b = argmin ||A[N(b), b] X - I[N(b), b]||_F = (A_Nb^H A_Nb)^{-1} D_b^H, with A_Nb the near
// field on the rows of N(b) and the slots of b (in `work`, n x 64); unused slots of a short
// tile keep identity.  Target: (X_b - D_b^{-1}) / s_b.
template <class T>
__global__ __launch_bounds__(256) void kp_targets(OpDev op, PrecDev pc, int ring, int64_t t0, T* work, int64_t wstride,
                                                  float* delta) {
    __shared__ T G[kTileN][kTileN + 1];
    __shared__ T colk[kTileN];
    __shared__ int perm[kTileN];
    __shared__ int piv_s;
    const int64_t* grp_of_row = pc.grp_of_row;
    const int32_t* pos_of_row = pc.pos_of_row;
    const int64_t tb = t0 + blockIdx.x;
    const Nbhd N = nbhd_of(op.S, pc.nt, tb, ring);
    const int n = N.n;
    T* Anb = work + blockIdx.x * wstride;  // [n][64]
    T* DH = Anb + (int64_t)n * kTileN;     // [64][64]: D_b^H (identity on unused slots)
    for (int64_t idx = threadIdx.x; idx < (int64_t)n * kTileN; idx += 256) {
        const int i = (int)(idx / kTileN), l = (int)(idx % kTileN);
        const int64_t h = slot_dof(op.S, pc.nt, tb, l);
        Anb[idx] = h >= 0 ? near_entry<T>(op, grp_of_row, pos_of_row, N.dof(op.S, i), h) : zero<T>();
    }
    for (int idx = threadIdx.x; idx < kTileN * kTileN; idx += 256) {
        const int i = idx / kTileN, j = idx % kTileN;
        const int64_t gi = slot_dof(op.S, pc.nt, tb, i), gj = slot_dof(op.S, pc.nt, tb, j);
        T v = zero<T>();
        if (gi >= 0 && gj >= 0)
            v = conj_(near_entry<T>(op, grp_of_row, pos_of_row, gj, gi));  // (D^H)_ij = conj(D_ji)
        else if (i == j)
            v = one<T>();
        DH[idx] = v;
    }
    __syncthreads();
    for (int idx = threadIdx.x; idx < kTileN * kTileN; idx += 256) {
        const int i = idx / kTileN, j = idx % kTileN;
        T acc = zero<T>();
        for (int k = 0; k < n; ++k) acc += conj_(Anb[(int64_t)k * kTileN + i]) * Anb[(int64_t)k * kTileN + j];
        if (i == j && slot_dof(op.S, pc.nt, tb, i) < 0) acc = one<T>();
        G[i][j] = acc;
    }
    __syncthreads();
    gj_invert<T>(G, colk, perm, &piv_s, pc.status);
    const T* Dinv = (const T*)pc.D0inv + tb * kTileN * kTileN;
    const double sinv = 1.0 / pc.scale[tb];
    constexpr int CPX = sizeof(T) == 16 ? 2 : 1;
    float* out = delta + tb * kTileN * kTileN * CPX;
    for (int idx = threadIdx.x; idx < kTileN * kTileN; idx += 256) {
        const int i = idx / kTileN, j = idx % kTileN;
        T x = zero<T>();
        for (int k = 0; k < kTileN; ++k) x += G[i][k] * DH[k * kTileN + j];
        const T d = x - Dinv[idx];
        if constexpr (CPX == 2) {
            const cdbl c = *(const cdbl*)&d;
            out[2 * idx] = (float)(c.re * sinv);
            out[2 * idx + 1] = (float)(c.im * sinv);
        } else {
            out[idx] = (float)(*(const double*)&d * sinv);
        }
    }
}

// ------------------------------------------------------------------ learned correction
// counter-based probe entries: splitmix64 of (tile, probe, slot), mapped to [-1, 1)
__device__ inline double probe_val(int64_t tb, int k, int l) {
    uint64_t x = ((uint64_t)tb * 4 + (uint64_t)k) * 64 + (uint64_t)l + 0x9E3779B97F4A7C15ull;
    x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
    x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
    x ^= x >> 31;
    return (double)(x >> 11) * (2.0 / 9007199254740992.0) - 1.0;
}

// One block per tile: W = s_b U V^T (from the network output, FP32 -> FP64), then for 4
// probe vectors p on the tile the neighbourhood residuals ||[p; 0] - A[N(b), b] z|| of
// z = D0inv p and z = (D0inv + W) p; the correction is kept if it lowers every residual
// (mode 2), always (mode 1) or never (mode 0).
template <class T>
__global__ __launch_bounds__(256) void kp_correct(OpDev op, PrecDev pc, const float* uv, int mode, int ring,
                                                  int* accepted) {
    const int64_t* grp_of_row = pc.grp_of_row;
    const int32_t* pos_of_row = pc.pos_of_row;
    constexpr bool CP = sizeof(T) == 16;
    constexpr int OUT = (CP ? 4 : 2) * kTileN * kRank;
    __shared__ T U[kTileN][kRank], V[kTileN][kRank];
    __shared__ T W[kTileN][kTileN + 1];
    __shared__ T Z[8][kTileN];  // z for 4 probes x (plain, corrected)
    __shared__ double res[256][8];
    const int64_t tb = blockIdx.x;
    const float* o = uv + tb * OUT;
    const double s = pc.scale[tb];
    for (int i = threadIdx.x; i < kTileN * kRank; i += 256) {
        if constexpr (CP) {
            ((cdbl*)&U[0][0])[i] = cdbl{o[i], o[kTileN * kRank + i]};
            ((cdbl*)&V[0][0])[i] = cdbl{o[2 * kTileN * kRank + i], o[3 * kTileN * kRank + i]};
        } else {
            ((double*)&U[0][0])[i] = o[i];
            ((double*)&V[0][0])[i] = o[kTileN * kRank + i];
        }
    }
    __syncthreads();
    const T* D0 = (const T*)pc.D0inv + tb * kTileN * kTileN;
    for (int idx = threadIdx.x; idx < kTileN * kTileN; idx += 256) {
        const int i = idx / kTileN, j = idx % kTileN;
        T acc = zero<T>();
        if (slot_dof(op.S, pc.nt, tb, i) >= 0 && slot_dof(op.S, pc.nt, tb, j) >= 0)
            for (int k = 0; k < kRank; ++k) acc += U[i][k] * V[j][k];
        W[i][j] = acc * s;
    }
    __syncthreads();
    bool keep = mode == 1;
    if (mode == 2) {
        // z for the probes
        for (int idx = threadIdx.x; idx < 8 * kTileN; idx += 256) {
            const int v = idx / kTileN, i = idx % kTileN, k = v >> 1;
            T acc = zero<T>();
            for (int j = 0; j < kTileN; ++j) {
                if (slot_dof(op.S, pc.nt, tb, j) < 0) continue;
                const T pj = one<T>() * probe_val(tb, k, j);
                T a = D0[i * kTileN + j];
                if (v & 1) a += W[i][j];
                acc += a * pj;
            }
            Z[v][i] = slot_dof(op.S, pc.nt, tb, i) >= 0 ? acc : zero<T>();
        }
        __syncthreads();
        // residuals over the rows of N(b)
        const Nbhd N = nbhd_of(op.S, pc.nt, tb, ring);
        double rl[8];
        for (int v = 0; v < 8; ++v) rl[v] = 0.0;
        for (int i = threadIdx.x; i < N.n; i += 256) {
            const int64_t g = N.dof(op.S, i);
            T acc[8];
            for (int v = 0; v < 8; ++v) acc[v] = zero<T>();
            for (int j = 0; j < kTileN; ++j) {
                const int64_t h = slot_dof(op.S, pc.nt, tb, j);
                if (h < 0) continue;
                const T a = near_entry<T>(op, grp_of_row, pos_of_row, g, h);
                for (int v = 0; v < 8; ++v) acc[v] += a * Z[v][j];
            }
            int64_t tg;
            int lg;
            tile_of(op.S, pc.nt, g, tg, lg);
            for (int v = 0; v < 8; ++v) {
                const T pv = tg == tb ? one<T>() * probe_val(tb, v >> 1, lg) : zero<T>();
                rl[v] += absval(pv - acc[v]) * absval(pv - acc[v]);
            }
        }
        for (int v = 0; v < 8; ++v) res[threadIdx.x][v] = rl[v];
        __syncthreads();
        for (int off = 128; off > 0; off >>= 1) {
            if ((int)threadIdx.x < off)
                for (int v = 0; v < 8; ++v) res[threadIdx.x][v] += res[threadIdx.x + off][v];
            __syncthreads();
        }
        keep = true;
        for (int k = 0; k < 4; ++k) keep = keep && res[0][2 * k + 1] < res[0][2 * k];
    }
    T* Dn = (T*)pc.Dinv + tb * kTileN * kTileN;
    for (int idx = threadIdx.x; idx < kTileN * kTileN; idx += 256) {
        const int i = idx / kTileN, j = idx % kTileN;
        Dn[idx] = keep ? D0[idx] + W[i][j] : D0[idx];
    }
    if (threadIdx.x == 0) accepted[tb] = keep ? 1 : 0;
}

// row -> group and position in group (from the group lists)
__global__ void kp_row_maps(OpDev op, int64_t* grp_of_row, int32_t* pos_of_row) {
    const int64_t G = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (G >= op.ngroups) return;
    for (int64_t k = op.grp_rowptr[G]; k < op.grp_rowptr[G + 1]; ++k) {
        grp_of_row[op.grp_rows[k]] = G;
        pos_of_row[op.grp_rows[k]] = (int32_t)(k - op.grp_rowptr[G]);
    }
}

template <class T>
hipError_t build_t(const OpDev& op, const PrecDev& pc, hipStream_t st) {
    hipLaunchKernelGGL(kp_row_maps, dim3(nblk(op.ngroups, 256)), dim3(256), 0, st, op, pc.grp_of_row, pc.pos_of_row);
    hipLaunchKernelGGL(kp_init<T>, dim3(nblk(pc.ntiles * kTileN * kTileN, 256)), dim3(256), 0, st, op, pc);
    hipLaunchKernelGGL(kp_extract<T>, dim3(nblk(op.ngroups, 4)), dim3(256), 0, st, op, pc);
    hipLaunchKernelGGL(kp_invert<T>, dim3((unsigned)pc.ntiles), dim3(256), 0, st, pc);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_prec_build(const OpDev& op, const PrecDev& pc, hipStream_t st) {
    return op.cplx ? build_t<cdbl>(op, pc, st) : build_t<double>(op, pc, st);
}

hipError_t launch_prec_apply(const OpDev& op, const PrecDev& pc, int R, const void* r, void* z, hipStream_t st) {
    const unsigned nb = (unsigned)(pc.ntiles * ((R + 63) / 64));
    if (op.cplx)
        hipLaunchKernelGGL(kp_apply<cdbl>, dim3(nb), dim3(256), 0, st, op, pc, R, (const cdbl*)r, (cdbl*)z);
    else
        hipLaunchKernelGGL(kp_apply<double>, dim3(nb), dim3(256), 0, st, op, pc, R, (const double*)r, (double*)z);
    return hipGetLastError();
}

hipError_t launch_prec_features(const OpDev& op, const PrecDev& pc, float* feats, hipStream_t st) {
    hipLaunchKernelGGL(kp_features, dim3((unsigned)pc.ntiles), dim3(64), 0, st, op, pc, feats);
    return hipGetLastError();
}

size_t prec_layout(const OpDev& op, int64_t ntiles, void* base, PrecDev* pc) {
    const size_t sc = op.cplx ? 16 : 8;
    char* b = (char*)base;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        off = (off + 255) / 256 * 256;
        char* p = b ? b + off : nullptr;
        off += bytes;
        return p;
    };
    PrecDev d{};
    d.ntiles = ntiles;
    d.Dinv = take((size_t)ntiles * kTileN * kTileN * sc);
    d.D0inv = take((size_t)ntiles * kTileN * kTileN * sc);
    d.scale = (double*)take((size_t)ntiles * 8);
    d.status = (int*)take(8);
    d.accepted = (int*)take((size_t)ntiles * 4);
    d.grp_of_row = (int64_t*)take((size_t)op.S.ndof * 8);
    d.pos_of_row = (int32_t*)take((size_t)op.S.ndof * 4);
    if (pc) *pc = d;
    return off + 256;
}

static int64_t nbhd_max(int ring) {
    const int w = kTile + 2 * ring;
    return (int64_t)w * w;
}
size_t prec_target_bytes(const OpDev& op, int ring, int64_t ntiles_per_launch) {
    const int64_t n = nbhd_max(ring);
    const size_t sc = op.cplx ? 16 : 8;
    return (size_t)ntiles_per_launch * (n + kTileN) * kTileN * sc;
}

hipError_t launch_prec_targets(const OpDev& op, const PrecDev& pc, int ring, int64_t t0, int64_t nt, void* work,
                               float* delta, hipStream_t st) {
    if (ring < 0 || ring > 8 || nt <= 0) return hipErrorInvalidValue;
    const int64_t n = nbhd_max(ring), ws = (n + kTileN) * kTileN;
    if (op.cplx)
        hipLaunchKernelGGL(kp_targets<cdbl>, dim3((unsigned)nt), dim3(256), 0, st, op, pc, ring, t0, (cdbl*)work, ws,
                           delta);
    else
        hipLaunchKernelGGL(kp_targets<double>, dim3((unsigned)nt), dim3(256), 0, st, op, pc, ring, t0, (double*)work, ws,
                           delta);
    return hipGetLastError();
}

hipError_t launch_prec_correct(const OpDev& op, const PrecDev& pc, const float* uv, int mode, int ring,
                               int* accepted, hipStream_t st) {
    if (ring < 0 || ring > 8) return hipErrorInvalidValue;
    if (op.cplx)
        hipLaunchKernelGGL(kp_correct<cdbl>, dim3((unsigned)pc.ntiles), dim3(256), 0, st, op, pc, uv, mode, ring,
                           accepted);
    else
        hipLaunchKernelGGL(kp_correct<double>, dim3((unsigned)pc.ntiles), dim3(256), 0, st, op, pc, uv, mode, ring,
                           accepted);
    return hipGetLastError();
}

}  // namespace bem
