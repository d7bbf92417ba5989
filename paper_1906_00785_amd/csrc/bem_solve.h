// GMRES(m) device kernels (bem_solve.hip) and the device state they share.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "bem_core.h"

namespace bem {

constexpr int kSolveBlocks = 256;  // slices of every vector kernel
constexpr int kMaxRestart = 64;    // Krylov dimension per cycle at most

// Device-resident state of one GMRES cycle (pointers into the solver workspace).
struct GmresState {
    int m;
    void* H;       // (m+1) x m rotated Hessenberg matrix, row-major
    double* cs;    // m cosines
    void* sn;      // m sines
    void* g;       // m+1 rotated right-hand side
    void* y;       // m coefficients of the update
    void* h1;      // m+1 first Gram-Schmidt coefficients
    void* h2;      // m+1 second Gram-Schmidt coefficients
    double* scal;  // [0] unused, [1] beta of the cycle, [2 + j] residual estimate after step j
    // optional host-mapped status (coherent pinned memory): after Givens step j the estimate
    // goes to hest[j] and then stamp to hseq[j], so the host can read it without a copy
    double* hest = nullptr;
    unsigned* hseq = nullptr;
    unsigned stamp = 0;
};

// dot products of the new vector against V (k vectors); gj >= 0 also runs Givens step gj
hipError_t solve_dots(int cplx, int64_t n, int k, const void* V, const void* w, void* part, int gj,
                      const double* npart, const GmresState& st, hipStream_t s);
hipError_t solve_givens(int cplx, int j, const double* npart, const GmresState& st, hipStream_t s);
hipError_t solve_scale(int cplx, int64_t n, const double* npart, const void* w, void* vnext, hipStream_t s);
hipError_t solve_update(int cplx, int64_t n, int k, const void* V, const void* part_in, void* hout, void* w,
                        void* part_out, double* npart, int mode, hipStream_t s);
hipError_t solve_residual(int cplx, int64_t n, const void* b, void* w, double* npart, int copy_b, hipStream_t s);
hipError_t solve_start(int cplx, int64_t n, const double* npart, const void* w, void* v0, const GmresState& st,
                       hipStream_t s);
hipError_t solve_axpy(int cplx, int64_t n, double a, const void* x, void* y, hipStream_t s);
hipError_t solve_backsolve_update(int cplx, int64_t n, int k, const void* V, void* x, const GmresState& st,
                                  hipStream_t s);
// x += sign * sum_{i<k} y_i V_i, y device (k <= 64)
hipError_t solve_combine(int cplx, int64_t n, int k, const void* V, const void* y, double sign, void* x,
                         hipStream_t s);

// ---- many right-hand sides in lockstep (bem_bsolve.hip): slab vectors v[g][r]
constexpr int kBSolveSlices = 64;  // row slices of every slab kernel

// Device-resident per-RHS state of one batched GMRES cycle.
struct BGmresState {
    int m;
    void* H;      // [R][(m+1) x m]
    double* cs;   // [R][m]
    void* sn;     // [R][m]
    void* g;      // [R][m+1]
    void* y;      // [m][R]
    double* est;  // [m][R] residual estimate after each step
    double* beta; // [R] norm of the cycle's initial residual
    double* sc;   // [R] scale of the next basis vector
    int* kr;      // [R] steps of each right-hand side used for the update
};

hipError_t bsolve_dots(int cplx, int64_t n, int R, int k, const void* V, const void* w, void* part, void* h,
                       hipStream_t s);
hipError_t bsolve_update(int cplx, int64_t n, int R, int k, const void* V, const void* h, void* w, double* npart,
                         int norm, hipStream_t s);
hipError_t bsolve_residual(int cplx, int64_t n, int R, const void* b, void* w, double* npart, int copy_b,
                           hipStream_t s);
hipError_t bsolve_start(int cplx, int64_t n, int R, const double* npart, const void* w, void* v0,
                        const BGmresState& st, hipStream_t s);
hipError_t bsolve_givens_scale(int cplx, int64_t n, int R, int j, const double* npart, const void* h1, const void* h2,
                               const void* w, void* vnext, const BGmresState& st, hipStream_t s);
hipError_t bsolve_backsolve_update(int cplx, int64_t n, int R, int k, const void* V, void* x, const BGmresState& st,
                                   hipStream_t s);
hipError_t bsolve_axpy(int cplx, int64_t n, int R, const void* x, void* y, hipStream_t s);
// x[g][r] += sum_{j<k} y[j][r] V_j[g][r]  (y device [k][R], k <= 64)
hipError_t bsolve_xupdate(int cplx, int64_t n, int R, int k, const void* V, const void* y, void* x, hipStream_t s);
// U = u / ||u_r|| and D = d / ||u_r|| per right-hand side r (norms from the partials of u;
// a zero column stays zero)
hipError_t bsolve_scale2(int cplx, int64_t n, int R, const double* npart, const void* u, const void* d, void* U,
                         void* D, hipStream_t s);
hipError_t bsolve_mask(int cplx, int64_t n, int R, const int* flag, void* y, hipStream_t s);
hipError_t bsolve_zero(int cplx, int64_t n_scalars, void* y, hipStream_t s);

}  // namespace bem
