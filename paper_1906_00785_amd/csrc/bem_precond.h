// Block-Jacobi preconditioner with an optional learned low-rank correction
// (bem_precond.hip), and the small dense kernels that build its training data.
//
// Blocks are tiles of kTile x kTile consecutive B-spline indices of one patch (64 DOFs;
// the last tile of a direction is smaller, its unused slots are identity).  Tile of DOF
// g = (f, j1, j2): (f, j1 / kTile, j2 / kTile), slot (j1 % kTile) * kTile + j2 % kTile.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "bem_kernels.h"

namespace bem {

constexpr int kTile = 8;
constexpr int kTileN = kTile * kTile;  // 64 slots per block
constexpr int kRank = 8;               // rank of the learned correction
constexpr int kFeat = 99;              // features per block: 16 x (3 x 2) Jacobian + Re k, Im k, level

struct PrecDev {
    int nt;          // tiles per direction per patch
    int64_t ntiles;
    void* Dinv;      // [ntiles][64][64] active inverse (row-major)
    void* D0inv;     // [ntiles][64][64] plain block-Jacobi inverse (fallback)
    double* scale;   // [ntiles] s_b = ||D_b^{-1}||_F / 64
    int* status;     // [1] 0 ok, 1 singular pivot met
    int* accepted;   // [ntiles] learned correction kept
    int64_t* grp_of_row;  // [N] near-field row group of every row
    int32_t* pos_of_row;  // [N] position of every row in its group
};

// bytes of the preconditioner's device workspace and its layout
size_t prec_layout(const OpDev& op, int64_t ntiles, void* base, PrecDev* pc);

// D_b from the near field, inverted by Gauss-Jordan with partial pivoting; Dinv = D0inv
hipError_t launch_prec_build(const OpDev& op, const PrecDev& pc, hipStream_t st);
// z = M^{-1} r on slabs [N][R] (R = 1: plain vectors)
hipError_t launch_prec_apply(const OpDev& op, const PrecDev& pc, int R, const void* r, void* z, hipStream_t st);
// features of every tile (float, [ntiles][kFeat])
hipError_t launch_prec_features(const OpDev& op, const PrecDev& pc, float* feats, hipStream_t st);
// training targets: (X_b - D_b^{-1}) / s_b as float [ntiles][64][64] (x2 interleaved if
// complex), X_b = (A_Nb^H A_Nb)^{-1} D_b^H the block least-squares approximate inverse on
// N(b), the tile plus `ring` (<= 8) indices per side; work: scratch of
// prec_target_bytes(); tiles [t0, t0 + nt) per launch
size_t prec_target_bytes(const OpDev& op, int ring, int64_t ntiles_per_launch);
hipError_t launch_prec_targets(const OpDev& op, const PrecDev& pc, int ring, int64_t t0, int64_t nt, void* work,
                               float* delta, hipStream_t st);
// installs Dinv_b = D0inv_b + s_b U_b V_b^T from uv ([ntiles][out], out = 2*64*kRank, x2 if
// complex) where the probe test accepts it (accept = 1: always, 0: never, 2: test); writes
// accepted flags [ntiles]
hipError_t launch_prec_correct(const OpDev& op, const PrecDev& pc, const float* uv, int mode, int ring,
                               int* accepted, hipStream_t st);

}  // namespace bem
