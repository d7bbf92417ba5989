// Maxwell single layer (App. A (MP), App. B (MS)) on the div-conforming spaces S^1 of App. E,
// assembled on the device densely (element-pair blocks, the glued dense matrix and its
// product) or with the far field compressed by the interpolation of Sec. 2; the load vector
// of dipole and plane-wave data and the field (MS) of a density.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "bem_kernels.h"

namespace bem {

constexpr int kMxMaxP = 2;    // degrees p of the device kernels (register budget of the pair kernel)
constexpr int kMxhChunk = 4;  // stored admissible pairs per coupling work chunk

struct MxDev {
    GeomDesc geom;
    KernelDesc ker;          // Helmholtz kernel of (MS)
    int p, nel, nl;          // degree, elements per direction, local functions per element 2p(p+1)
    int qg, qs;              // Gauss points per direction of regular pairs, of the Duffy cubes
    double h;
    int64_t nelem, nglob;
    const double* polp;      // [nel][p+1][p+1] local B-splines of degree p (monomial coefficients)
    const double* polq;      // [nel][p][p] local B-splines of degree p - 1
    const int32_t* eglob;    // [nelem][nl] global function of each local function (-1: dropped)
    const int32_t* esgn;     // [nelem][nl] its sign
    const int64_t* gptr;     // [nglob + 1] (element, position) pieces of every global function,
    const int32_t* gpos;     // as element * nl + position,
    const int32_t* gsgn;     // with their signs
    const int32_t* tinfo;    // [nelem * nelem] touching pairs: type | k1 << 4 | k2 << 8; 0: regular
    const double* gx;        // [qg] Gauss rule of regular pairs
    const double* gw;
    const double* sx;        // [qs] Gauss rule of the Duffy cubes
    const double* sw;
    void* B;                 // [npairs][nl][nl] complex element-pair blocks (test x trial)
    void* M;                 // [nglob][nglob] complex dense matrix, row-major (test x trial)
    const int64_t* plist;    // [npairs] e1 * nelem + e2 of each block (null: all pairs, in order)
    int64_t npairs;          // blocks to compute (nelem * nelem without a list)
    const int64_t* blist;    // [npairs] the blocks by kind: the nreg regular ones, then the touching ones
    int64_t nreg;
};

// The compressed operator (Sec. 2 interpolation on the scalar block partition, four
// channels: the three components of the lifted field and the divergence).
struct MxhDev {
    MxDev s;                     // space, Gauss rules; s.B: near element-pair blocks (assembly)
    int q, q2, leaf, m, nleaf1;  // m: elements per leaf per direction
    int64_t ncl, nleaves, nfar, nnear;
    const int64_t* lev_off;      // [leaf + 2] first cluster of every level
    const double* cheb;          // [q] Chebyshev nodes on [0, 1]
    const double* E;             // [2][q][q]: E[b][p][a] = L_a(child b's node p in the parent)
    // admissible pairs stored once: block s joins its owner own_t[s] and partner own_s[s]
    // (the owner's blocks consecutive)
    int64_t nstored;
    const int32_t* own_t;        // [nstored]
    const int32_t* own_s;        // [nstored]
    void* K;                     // [nstored][q2 (partner b)][q2 (owner a)] complex G(x_a^owner, x_b^partner)
    // coupling work chunks: up to kMxhChunk consecutive stored blocks of one owner each
    int64_t nchunks;
    const int32_t* ch_p0;        // [nchunks] first stored block
    const int32_t* ch_p1;        // [nchunks] end stored block
    const int64_t* cl_chunk;     // [ncl + 1] chunks of every cluster (as owner)
    void* partial;               // [nchunks][4][q2] complex partial local expansions of the owners
    void* tprod;                 // [nstored][4][q2] complex products of the blocks' transposes with
                                 // the owners' moments (the partners' contributions)
    const int64_t* tr_ptr;       // [ncl + 1] stored blocks in which each cluster is the partner
    const int32_t* tr_blk;
    const int32_t* near_rowptr;  // [nleaves + 1] near leaf pairs by target leaf
    const int32_t* near_s;       // [nnear] source leaf (leaf-local index)
    // glued near field over the global functions (CSR, ascending columns): entry (g, h) sums
    // the signed entries of the near element-pair blocks between the pieces of g and of h
    int64_t nnzg;
    const int64_t* nrowptr;      // [nglob + 1]
    const int32_t* ncol;         // [nnzg]
    void* nval;                  // [nnzg] complex
    double* Mt;                  // [nelem][nl][4][q2] channel moments against the leaf's Lagrange polynomials
    double* xc;                  // [ncl][q2][3] Chebyshev points on the surface (assembly)
    const double* Lg;            // [m][qg][q] L_a at Gauss point k of element position i in its
                                 // leaf, (i + x_k) / m (assembly)
    void* mom;                   // [ncl][4][q2] complex moments
    void* lv;                    // [ncl][4][q2] complex local expansions
};

// element-pair blocks (tau test, sigma trial) of every pair, or of the pairs in d.plist
hipError_t launch_mx_pairs(const MxDev& d, hipStream_t st);
// compressed operator: cluster points, kernel blocks, channel moments, near blocks
hipError_t launch_mxh_assemble(const MxhDev& d, hipStream_t st);
// y = A x with the compressed operator (complex, one column)
hipError_t launch_mxh_apply(const MxhDev& d, const void* x, void* y, hipStream_t st);
// M[g][h] = sum over the pieces of g and h of the signed block entries
hipError_t launch_mx_gather(const MxDev& d, hipStream_t st);
// y = M x (complex, one column)
hipError_t launch_mx_matvec(const MxDev& d, const void* x, void* y, hipStream_t st);
// load vector of data kind (0 dipole: x0, moment; 1 plane wave: direction, polarisation)
hipError_t launch_mx_rhs(const MxDev& d, const Gauss8& g8, int kind, const double* prm6, void* b, hipStream_t st);
// field (MS) of the density j at npts points: 3 complex per point
hipError_t launch_mx_field(const MxDev& d, const Gauss8& g8, const double* pts, int64_t npts, const void* j, void* E,
                           hipStream_t st);

}  // namespace bem
