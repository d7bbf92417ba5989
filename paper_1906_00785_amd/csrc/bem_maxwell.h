// Maxwell single layer (App. A (MP), App. B (MS)) on the div-conforming spaces S^1 of App. E,
// assembled densely on the device: element-pair blocks, the glued dense matrix, its
// product, the load vector of dipole and plane-wave data and the field (MS) of a density.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "bem_kernels.h"

namespace bem {

constexpr int kMxMaxP = 2;  // degrees p of the device kernels (register budget of the pair kernel)

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
    void* B;                 // [nelem * nelem][nl][nl] complex element-pair blocks (test x trial)
    void* M;                 // [nglob][nglob] complex dense matrix, row-major (test x trial)
};

// element-pair blocks of every pair (tau test, sigma trial)
hipError_t launch_mx_pairs(const MxDev& d, hipStream_t st);
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
