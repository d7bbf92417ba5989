// Many right-hand sides at once: the H^2 matvec over a block of R columns (bem_batch.hip).
//
// Inside a batched launch every DOF vector is held as a slab x[g][r] (the R values of one
// DOF contiguous), and so are moments and local expansions ([cluster][a][r]); a wave
// handles one item (leaf, cluster, row group) for 64 consecutive right-hand sides, one per
// lane, so every load of a slab row is coalesced and every table entry is shared by the
// wave.  The far-field coupling runs per target cluster over all its admissible sources:
// in FP64/FP32 on the vector units from the stored blocks, or in BF16 on the matrix cores
// (MFMA) from a copy of the blocks laid out as matrix fragments.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "bem_kernels.h"

namespace bem {

constexpr int kBatchChunk = 64;  // right-hand sides per wave

struct BatchDev {
    int rmax;  // right-hand sides per launch at most
    int R;     // right-hand sides of this launch (slab row length)
    // far list per target: sources and where each block sits in the stored coupling rows
    const int64_t* far_rowptr;  // per cluster
    const int32_t* far_s;       // source of each ordered pair
    const int64_t* fb_off;      // first scalar of the block (row 0) in K
    const int32_t* fb_rs;       // row stride of the stored rows; negative: stored transposed
    // near field as dense tiles for the matrix cores: rows of a 4 x 4 block of B-spline
    // indices of a patch, columns the union of their patterns; values in FP64 MFMA
    // fragment order (per step of 4 columns, lane l: row l % 16, column 4 step + l / 16)
    int64_t ntiles;
    const int64_t* tile_rowptr;  // [ntiles + 1] into tile_rows
    const int32_t* tile_rows;
    const int64_t* tile_colptr;  // [ntiles + 1] into tile_cols
    const int32_t* tile_cols;
    const int64_t* tile_voff;    // [ntiles + 1] first value (multiple of 64)
    void* tile_val;
    const int32_t* row_grp;      // near-field row group and position of every row
    const int32_t* row_pos;
    void* xs;                   // [N][R] input slab
    void* ys;                   // [N][R] output slab
    void* mom;                  // [ncl][q2][R] moments
    void* lv;                   // [ncl][q2][R] local expansions
    void* yl;                   // [nleaves][nloc^2][R] backward transform per leaf
    // BF16 matrix-core coupling (op.low == 2): fragments of every ordered block and of the
    // moments of every cluster
    void* Af;                   // [npairs][RT][64 lanes] x 8 bf16
    void* Bf;                   // [ncl][nchunks][NT][64 lanes] x 8 bf16
    void* mlow;                 // FP32 copy of the moments' slab (FP32 coupling), or null
    // transfer from a leaf to its ancestor k levels up, k = 1..leaf: for each leaf position
    // b in [0, 2^k) along one direction a q x q matrix [p][a] (leaf index p, ancestor index
    // a); level k starts at q^2 (2^k - 2)
    const double* Ec;
};

// fragment counts of the BF16 coupling: row tiles of 16 (real: K padded to 32 rows;
// complex: [Re K; Im K] padded to 64) and column tiles of 16 per 64 right-hand sides
// (real: 64 columns; complex: [Re m | Im m], 128 columns)
inline int bf_row_tiles(int cplx) { return cplx ? 4 : 2; }
inline int bf_col_tiles(int cplx) { return cplx ? 8 : 4; }

// Y = A X for R <= rmax columns.  x, y: column-major N x R with leading dimensions ldx, ldy
// (x == nullptr: the input is already in bd.xs; y == nullptr: the result stays in bd.ys).
// prec: 0 FP64 coupling, 1 FP32 (op.low == 1), 2 BF16 matrix cores (op.low == 2).
hipError_t launch_apply_batched(const OpDev& op, const BatchDev& bd, const void* x, int64_t ldx, void* y,
                                int64_t ldy, int prec, hipStream_t st);
// per-stage variant for timing: 0 slab in + leaf moments + upward, 1 coupling, 2 downward +
// backward, 3 near field + slab out
constexpr int kBatchStages = 4;
hipError_t launch_apply_batched_stage(const OpDev& op, const BatchDev& bd, int stage, const void* x, int64_t ldx,
                                      void* y, int64_t ldy, int prec, hipStream_t st);
// column-major (leading dimension ld) <-> slab [N][R]
hipError_t launch_to_slab(int cplx, int64_t N, int R, const void* x, int64_t ldx, void* xs, hipStream_t st);
hipError_t launch_from_slab(int cplx, int64_t N, int R, const void* ys, void* y, int64_t ldy, hipStream_t st);
// dense near-field tile values (assembly, after the near field)
hipError_t launch_tile_fill(const OpDev& op, const BatchDev& bd, hipStream_t st);
// BF16 fragments of every ordered far block (assembly, after the coupling blocks)
hipError_t launch_build_bf_blocks(const OpDev& op, const BatchDev& bd, int64_t npairs, hipStream_t st);

}  // namespace bem
