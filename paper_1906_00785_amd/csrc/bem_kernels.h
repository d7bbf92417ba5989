// Launch interface of the gfx950 kernels (bem_kernels.hip) used by the C ABI layer.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "bem_core.h"

namespace bem {

// Local B-spline polynomials of every element class, small enough to pass by value: with
// more than 2w+1 elements per direction (w = d+1) only the first w elements, the interior
// ones and the last w elements differ (uniform knots); otherwise every element is stored.
// The host checks every element against its class before use.
struct BasisTab {
    int d, nel, ncls, w;
    double c[7][3][3];  // [class][local basis][monomial coefficient], d <= 2
};
__host__ __device__ inline int basis_class(const BasisTab& t, int i) {
    if (t.ncls == t.nel) return i;
    if (i < t.w) return i;
    if (i >= t.nel - t.w) return 2 * t.w - (t.nel - 1 - i);
    return t.w;
}
__host__ __device__ inline double basis_eval(const BasisTab& t, int cls, int l, double x) {
    double v = t.c[cls][l][t.d];
    for (int k = t.d - 1; k >= 0; --k) v = v * x + t.c[cls][l][k];
    return v;
}
// the same with the degree D = t.d known at compile time
template <int D>
__host__ __device__ inline double basis_eval_d(const BasisTab& t, int cls, int l, double x) {
    double v = t.c[cls][l][D];
#pragma unroll
    for (int k = D - 1; k >= 0; --k) v = v * x + t.c[cls][l][k];
    return v;
}

struct Gauss8 {
    double x[8], w[8];
};

// Device arrays of an assembled operator (all inside the caller's workspaces).
struct OpDev {
    SpaceDesc S;
    BasisTab bt;
    int q, q2, leaf, m, nloc, nleaf1, qg, qs;
    int64_t ncl, nleaves, nfar, nnear, ntouch, nnz;
    int cplx;
    const int64_t* lev_off;  // device copy (leaf+2)
    // near field: CSR pattern; values stored by row groups (see the host plan)
    const int64_t* rowptr;
    const int32_t* col;
    void* val;
    int64_t ngroups;
    const int64_t* grp_rowptr;
    const int32_t* grp_rows;
    const int64_t* grp_voff;
    // far field: stored blocks in owner rows (see the host plan)
    const int64_t* own_rowptr;
    const int32_t* own_src;
    const int64_t* koff;
    const int32_t* krs;
    void* K;
    const int64_t* pcol;       // owner row -> start in P
    void* P;                   // transposed products, one scalar per stored column
    const int64_t* tr_rowptr;  // per cluster: its entries in tr_off
    const int64_t* tr_off;     // start of a q*q column group in P
    int64_t nchunks, nstored;
    const int32_t* ch_t;
    const int32_t* ch_k0;
    const int32_t* ch_k1;
    const int64_t* cl_chunk;   // per cluster: its chunks
    void* partial;             // per chunk: q*q row sums
    void* Klow;                // optional low-precision copy of K (same layout), see low
    int low;                   // 0 none, 1 FP32, 2 BF16
    int64_t ktotal_scalars;    // real scalars in K (2 per complex entry)
    // coupling evaluated in every apply instead of stored (K unused): the clusters'
    // Chebyshev points on the surface, [ncl][q2][3]
    int otf;
    int otf_wide;  // chunks of at least 512 columns (8 real columns per lane and pass)
    const double* xc;
    const double* ball;  // [ncl][4]: centre and radius of every cluster (admissibility)
    // transforms
    const double* V1;  // [nleaf1][q][nloc]
    const double* Vd;  // 0-form lifting: [nleaves][q*q][nloc*nloc] full leaf tables (else null)
    void* xl;          // S^0: the applied vector on the local functions (and the product)
    void* yl;
    const double* E;   // [2][q][q]
    // matvec scratch: moments and local expansions of all clusters (one RHS)
    void* mom;
    void* lv;
    // upward pass: subtrees rooted at level up_root are summed by one block each; the
    // levels above follow per patch
    int up_root, up_depth;
    int* up_count;  // per patch: subtree blocks done in the current apply (0 between applies)
    // downward pass + backward transform: square tiles of leaves per block
    int tile;
};

// Temporary arrays used only during assembly.
struct AsmDev {
    const int32_t* near_t;
    const int32_t* near_s;
    const int32_t* near_rowptr;
    const int32_t* touch_rowptr;
    const int32_t* touch;
    const int32_t* touch_lp;  // near leaf pairs that contain touching pairs
    const int32_t* row_grp;   // row group of every row
    const int32_t* row_pos;   // position of every row in its group
    int64_t ntouch_lp;
    const int32_t* vid;
    const double* gx;     // [qg]
    const double* gpos;   // [nelem][qg*qg][3]
    const double* gkap;   // [nelem][qg*qg] surface element at the Gauss points (0-form lifting only)
    const double* psi;    // [nel][qg][d+1]
    const double* psiw;   // [nel][qg][d+1] psi times the Gauss weights
    const double* gw;     // [qg]
    const double* sx;     // [qs]
    const double* sw;     // [qs]
    const double* cheb;   // [q]
    const int32_t* own_t; // owner of each stored block
    double* xc;           // [ncl][q2][3] Chebyshev points on the surface
    void* lb;             // [nnear][nloc^2][nloc^2] leaf-pair blocks
    void* sblk;           // [ntouch][(d+1)^2][(d+1)^2] element blocks of the touching pairs
};

hipError_t launch_gauss_points(const OpDev& op, const AsmDev& as, hipStream_t st);
hipError_t launch_leaf_tables0(const OpDev& op, const AsmDev& as, hipStream_t st);
// S^0: x_loc[i] = x[glue[i]] and y[g] = sum of y_loc over the local functions of g
hipError_t launch_glue_gather(const SpaceDesc& S, int cplx, const void* x, void* x_loc, hipStream_t st);
hipError_t launch_glue_scatter(const SpaceDesc& S, int cplx, const void* y_loc, void* y, hipStream_t st);
hipError_t launch_near_regular(const OpDev& op, const AsmDev& as, hipStream_t st);
hipError_t launch_near_singular(const OpDev& op, const AsmDev& as, hipStream_t st);
hipError_t launch_near_gather(const OpDev& op, const AsmDev& as, hipStream_t st);
hipError_t launch_far_assemble(const OpDev& op, const AsmDev& as, hipStream_t st);

// y = A x for one RHS column, as four stages: 0 near-field product with the forward
// transform + upward transfer beside it, 1 far-field coupling, 2 gather of the local
// expansions, 3 downward transfer + backward transform added to y
// prec: 0 FP64 coupling, otherwise the low-precision copy (op.low must be set)
constexpr int kApplyStages = 4;
hipError_t launch_apply_stage(const OpDev& op, int stage, const void* x, void* y, int prec, hipStream_t st);
hipError_t launch_apply(const OpDev& op, const void* x, void* y, int prec, hipStream_t st);
// low-precision copy of the stored coupling blocks
hipError_t launch_cast_low(const OpDev& op, hipStream_t st);
// moments of all clusters for x (forward + upward) into op.mom
hipError_t launch_moments(const OpDev& op, const void* x, hipStream_t st);

// Many operators and columns in one launch per stage: apply a runs the one-column stages
// of ops[a] (its own scratch) on x[a] -> y[a].  Stages: 0 near field + forward/upward
// inside subtrees, 1 upper levels of the upward pass, 2 coupling of the operators with
// stored blocks, 5 coupling of those evaluating it on the fly (launched right after 2, so
// that neither launch carries the other's registers), 3 gather of the local expansions,
// 4 downward + backward.  Within a launch the blocks of one operator's columns are
// interleaved (block j of the operator's range is block j / ncol of its column j % ncol),
// so that its columns read the same stored values one after the other.
// prefix[s * (nop + 1) + i] = first block of operator i in stage s's launch; first[i] =
// its first apply, ncol[i] its columns; nblocks[s] = blocks of that launch.  All operators
// share the scalar type and q.
constexpr int kGroupStages = 6;
struct GroupDev {
    int64_t napply, nop;
    const OpDev* ops;  // per apply
    const void* const* x;
    void* const* y;
    const int64_t* prefix;
    const int64_t* first;
    const int32_t* ncol;
    int64_t nblocks[kGroupStages];
};
// blocks of each grouped stage for one operator with ncols columns
void group_stage_blocks(const OpDev& op, int ncols, int64_t out[kGroupStages]);
hipError_t launch_group_apply(const GroupDev& g, int cplx, int q, hipStream_t st);

// load vector (one RHS) and potential (one RHS)
hipError_t launch_rhs(const SpaceDesc& S, const BasisTab& bt, const Gauss8& g8, int kind, const double* prm,
                      void* b, hipStream_t st);
// the load vector's quadrature points (nelem * 64 x 3) and the load vector from data sampled there
hipError_t launch_quadpoints(const SpaceDesc& S, const Gauss8& g8, double* xyz, hipStream_t st);
hipError_t launch_rhs_samples(const SpaceDesc& S, const BasisTab& bt, const Gauss8& g8, const void* gv, void* b,
                              hipStream_t st);
// potential through the cluster tree: moments of rho (launch_moments first, in op.mom),
// admissible clusters (point-ball rule with eta) by their Chebyshev points, near leaves by
// 8x8 Gauss
hipError_t launch_potential_tree(const OpDev& op, const Gauss8& g8, double eta, const double* pts, int64_t npts,
                                 const void* rho, void* u, hipStream_t st);
hipError_t launch_potential(const SpaceDesc& S, const BasisTab& bt, const Gauss8& g8, const double* pts,
                            int64_t npts, const void* rho, void* u, hipStream_t st);

}  // namespace bem
