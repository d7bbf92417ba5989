// Host-side plan of the H^2 operator: cluster tree on the patches' parameter squares, block
// partition, near-field pattern, touching element pairs and the small quadrature and
// interpolation tables that the kernels read.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "bem_core.h"

namespace bem {

// Gauss-Legendre rule on [0,1], n points, ascending
void gauss_legendre01(int n, std::vector<double>& x, std::vector<double>& w);

// Monomial coefficients (in the element-local coordinate xhat in [0,1]) of the d+1
// B-splines that are non-zero on each 1-D element: out[(i*(d+1) + l)*(d+1) + k] is the
// coefficient of xhat^k of B-spline i*r + l on element i.
void bspline_local_polys(int d, int r, int L, std::vector<double>& out);

// Lagrange basis polynomial a of the nodes xs evaluated at y (barycentric form)
double lagrange_bary(const std::vector<double>& xs, int a, double y);

constexpr int kGroupRows = 16;  // rows per near-field row group at most

struct H2Params {
    int q = 5;
    double eta = 1.6;
    int leaf = -1;
    int qg = 8;
    int qs = 8;
    int chunk = 128;  // columns per coupling work chunk (multiple of 128)
    double kadm = 0.0;  // far pairs also need |kappa| 2 max(r) <= kadm (Helmholtz; 0: no bound)
};

struct Plan {
    SpaceDesc S;
    H2Params P;
    int leaf = 0;          // leaf level used
    int m = 1;             // elements per leaf per direction
    int nloc = 1;          // B-splines overlapping one leaf interval
    int nleaf1 = 1;        // leaves per direction per patch
    int q2 = 1;            // q*q
    int64_t ncl = 0;       // clusters of all levels
    int64_t nleaves = 0;   // clusters at the leaf level
    std::vector<int64_t> lev_off;  // first cluster of each level (size leaf+2)
    std::vector<double> ball;      // centre xyz + radius per cluster

    // far field: all admissible pairs in both orientations, sorted by (target, source)
    std::vector<int32_t> far_t, far_s;
    std::vector<int64_t> far_rowptr;  // per cluster

    // Stored coupling blocks.  K_st = K_ts^T, so every unordered admissible pair is stored
    // once, in the rows of its owner: the smaller index if the index sum is odd, else the
    // larger (this splits each cluster's partners about evenly between the two roles).
    std::vector<int64_t> own_rowptr;  // per cluster: range of its stored blocks
    std::vector<int32_t> own_src;     // the partner of each stored block
    std::vector<int32_t> own_t;       // the owner of each stored block
    std::vector<int64_t> koff;        // start of each owner's coupling rows (scalars)
    std::vector<int32_t> krs;         // row stride of each owner's rows (even)
    int64_t ktotal = 0;               // scalars in all coupling rows
    // transposed products: one scalar per stored column, owner rows laid out like K's row 0
    std::vector<int64_t> pcol;        // start of each owner's columns in that buffer
    int64_t ptotal = 0;
    std::vector<int64_t> tr_rowptr;   // per cluster: stored blocks in which it is the partner
    std::vector<int64_t> tr_off;      // ... as offsets of their q*q columns in the buffer
    // work chunks of the coupling kernel: (owner, first column, end column), per owner
    // contiguous; every chunk but an owner's last has P.chunk columns
    std::vector<int32_t> ch_t, ch_k0, ch_k1;
    std::vector<int64_t> cl_chunk;    // per cluster: its chunk range

    // near field: leaf pairs (leaf-local indices), sorted
    std::vector<int32_t> near_t, near_s;
    std::vector<int32_t> near_rowptr;  // per leaf (size nleaves+1)
    // touching element pairs grouped by near leaf pair: packed (et, es, type, k1, k2)
    std::vector<int32_t> touch_rowptr;  // size nnear+1
    std::vector<int32_t> touch;         // 5 ints per pair
    std::vector<int32_t> vid;           // corner vertex ids, 4 per element (corner c1*2+c2)

    // near-field sparsity pattern in the B-spline basis
    std::vector<int64_t> rowptr;
    std::vector<int32_t> col;
    // Row groups: rows whose supports meet the same leaves have the same columns; up to
    // kGroupRows of them form a group whose values are stored row-major after each other
    // (value (r, c) of group G at grp_voff[G] + r * ncols(G) + c).  The columns of a group
    // are those of its first row in the pattern above.
    std::vector<int64_t> grp_rowptr;  // per group: range in grp_rows
    std::vector<int32_t> grp_rows;    // rows of each group, ascending
    std::vector<int64_t> grp_voff;    // per group: first value (size ngroups+1)
    std::vector<int32_t> row_grp, row_pos;  // group and position of every row

    // tables
    std::vector<double> gx, gw;   // qg-point rule
    std::vector<double> sx, sw;   // qs-point rule
    std::vector<double> bpoly;    // local B-spline polynomials (see bspline_local_polys)
    std::vector<double> psi;      // [nel][qg][d+1] B-spline values at the qg Gauss points
    std::vector<double> psiw;     // [nel][qg][d+1] the same times the Gauss weights
    std::vector<double> cheb;     // q Chebyshev nodes on [0,1]
    std::vector<double> E;        // [2][q][q]: E[b][a'][a] = L_a((b + x_a')/2)
    std::vector<double> V1;       // [nleaf1][q][nloc] 1-D leaf moments
};

// Builds the whole plan; returns false and sets err on invalid input.
bool build_plan(const SpaceDesc& S, const H2Params& P, Plan& plan, std::string& err);

// All touching element pairs of a space (sharing at least a vertex; both orders and e1 == e2
// included), as (e1, e2) in pairs and type | k1 << 4 | k2 << 8 in info (k1, k2 the symmetries
// of the unit square that bring the common vertex, or edge, to the origin, or to t = 0).
bool element_touch_pairs(const SpaceDesc& S, std::vector<int64_t>& pairs, std::vector<int32_t>& info,
                         std::string& err);

// Leaf-interval index range [lo, hi] that contains B-spline j (per direction)
inline void leaves_of_basis(const Plan& p, int j, int& lo, int& hi) {
    const int stride = p.m * p.S.r;  // first basis of leaf i is i*stride
    hi = j / stride;
    if (hi > p.nleaf1 - 1) hi = p.nleaf1 - 1;
    int l = j - p.nloc + 1;
    lo = l <= 0 ? 0 : (l + stride - 1) / stride;
}

}  // namespace bem
