/*
 * bem.h -- C ABI of libbem_hip.so, the MI355X (gfx950) implementation of the hot path of the
 * isogeometric Galerkin boundary element method of Bembel (arXiv 1906.00785): assembling
 * and applying the Laplace and Helmholtz single-layer operators on multi-patch surfaces,
 * compressed as an interpolation-based H^2 matrix, and solving with restarted GMRES.
 *
 * The calls follow the paper's problem statement and API (Sec. 4): geometry (Sec. 4
 * "Geometry", App. D) + PDE (Sec. 4 "PDE", App. B) + discrete space of level L and degree
 * (Sec. 4 "Discretization", App. E) -> load vector (Sec. 4 "Boundary Values") -> compressed
 * system matrix (Sec. 4 "System Matrix", Sec. 2) -> H*x -> GMRES (Sec. 4 "Solution of the
 * System of Linear Equations") -> potential (Sec. 4 "Evaluation of the Solution").
 *
 * Conventions shared by every call
 *  - Return value: BEM_OK (0) or a negative BEM_E* code.  No C++ exception crosses the ABI.
 *    bem_last_error() returns a thread-local message describing the last failure.
 *  - Handles (bem_geometry, bem_space, bem_operator) are created and destroyed by the
 *    library.  Destroying NULL is a no-op.  A space keeps its geometry alive by copy; an
 *    operator refers to its space, which must outlive it.
 *  - Device buffers are raw device pointers owned by the caller (e.g. torch tensors);
 *    every call that takes a hipStream_t enqueues its device work on that stream and
 *    returns without synchronising unless stated otherwise.
 *  - Scalars are double for Laplace and interleaved (re, im) double pairs for Helmholtz
 *    (std::complex<double> / torch.complex128 layout).
 *  - Vectors over the degrees of freedom (DOFs) use the global index
 *        g = (patch * n1 + j1) * n1 + j2,   n1 = d + 1 + (2^L - 1) * knot_repetition,
 *    where j1, j2 index the B-splines along the two parameter directions of the patch.
 *    Elements are numbered e = (patch * 2^L + i1) * 2^L + i2.
 *  - Several right-hand sides are stored column-major, N x nrhs, with a leading dimension.
 *  - The operator's device memory is a caller-provided workspace whose size is returned by
 *    bem_assemble_plan; calls on one operator that overlap in time (on different streams)
 *    race on its internal matvec buffers.
 */
#ifndef BEM_H
#define BEM_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define BEM_OK 0
#define BEM_EINVAL (-1)       /* invalid argument (message says which) */
#define BEM_ENOMEM (-2)       /* workspace too small or host allocation failed */
#define BEM_EDEVICE (-3)      /* a HIP call failed */
#define BEM_ENOCONV (-4)      /* solver did not reach the tolerance; best iterate written */
#define BEM_EUNSUPPORTED (-5) /* valid request this build does not implement */

/* PDEs of Sec. 4 "PDE": single-layer kernels (LS) 1/(4 pi r) and (HS) exp(-i kappa r)/(4 pi r) */
#define BEM_LAPLACE_SINGLE 0
#define BEM_HELMHOLTZ_SINGLE 1
/* Maxwell single layer (App. A (MP), App. B (MS)): for test and trial fields v, j on the
 * surface, the bilinear form of the integrals over Gamma x Gamma of the Helmholtz kernel
 * (HS) times v(x) . j(y) - kappa^-2 div_Gamma v(x) div_Gamma j(y) (the electric field
 * integral operator); lives on S^1 spaces (bem_space_create_ex with BEM_SPACE_S1). */
#define BEM_MAXWELL_SINGLE 2

/* multi-patch geometries (App. D; arbitrary smooth maps are allowed, Sec. 4).  Analytic:
 *   SPHERE6     unit sphere, 6 cube faces projected radially               params: none
 *   ELLIPSOID6  diag(a,b,c) applied to SPHERE6                             params: a, b, c
 *   TORUS16     torus of radii R > r, 16 patches of a quarter turn each    params: R, r
 *   FLAT1       one flat square patch [0,a]^2 x {0} (open surface; tests) params: a        */
#define BEM_GEOM_SPHERE6 0
#define BEM_GEOM_ELLIPSOID6 1
#define BEM_GEOM_TORUS16 2
#define BEM_GEOM_FLAT1 3
/* patches given by NURBS maps (App. C): bem_geometry_nurbs, bem_geometry_load,
 * bem_geometry_user */
#define BEM_GEOM_NURBS 4

/* boundary data for bem_rhs (Sec. 4 "Boundary Values"):
 *   POINT_SOURCE  g(x) = k(x, x0), the PDE's own kernel centred at x0       params: x0 (3)
 *   PLANE_WAVE    g(x) = exp(-i kappa d.x), Helmholtz only                  params: d (3)  */
#define BEM_DATA_POINT_SOURCE 0
#define BEM_DATA_PLANE_WAVE 1
/* tangential data of the Maxwell single layer (S^1 spaces; b_g = int_Gamma E . psi_g with the
 * lifted vector field psi_g of the global function g; 6 params per RHS):
 *   DIPOLE        E = curl curl (m G(x - x0)) = kappa^2 G m + grad (m . grad G), G the (HS)
 *                 kernel: the field of an electric dipole of moment m at x0, a solution of
 *                 the Maxwell equations (App. A) away from x0          params: x0 (3), m (3)
 *   PLANE_WAVE_E  E = e exp(-i kappa d . x)                            params: d (3), e (3)
 *                 (a Maxwell solution when |d| = 1 and e . d = 0; not checked)           */
#define BEM_DATA_DIPOLE 2
#define BEM_DATA_PLANE_WAVE_E 3

typedef struct bem_geometry_s* bem_geometry;
typedef struct bem_space_s* bem_space;
typedef struct bem_operator_s* bem_operator;

/* Parameters of the compressed system matrix (Sec. 4 "System Matrix": a discretisation
 * plus the polynomial degree of the H^2 compression; Sec. 2: singular quadrature by
 * regularisation, embedded FMM on the reference square). */
typedef struct bem_h2_params {
    int q;            /* Chebyshev points per direction of each cluster (degree q-1), >= 1 */
    double eta;       /* admissibility: 2 max(r_t, r_s) <= eta * dist(balls); 0 = dense   */
    int leaf_level;   /* cluster-tree leaf level, 0..L; -1 picks max(L-2, 0)             */
    int qg;           /* Gauss points per direction on each element of a regular pair   */
    int qs;           /* Gauss points per dimension of each Duffy cube (touching pairs)  */
    int chunk_cols;   /* coupling columns per work chunk, a multiple of 128; 0 = 128 (256
                         with far_eval)                                                 */
    int far_low;      /* extra low-precision copy of the coupling blocks for mixed-precision
                         applies and solves: 0 none, BEM_PREC_FP32 or BEM_PREC_BF16      */
    int batch_rhs;    /* right-hand sides per batched apply: with batch_rhs > 1 the operator
                         workspace holds slabs for that many columns and bem_apply /
                         bem_apply_ex with nrhs > 1 run the many-RHS kernels on up to
                         batch_rhs columns per pass (q <= 6; with q <= 5 the coupling
                         runs on the matrix cores in FP64, FP32 or BF16 and the near field
                         in FP64; BEM_PREC_BF16 there needs q <= 5); 0 or 1: one column
                         at a time                                                        */
    int far_eval;     /* 1: no stored coupling blocks; every apply evaluates the kernel at the
                         clusters' Chebyshev points where the blocks are used (same entries
                         as the stored blocks, Sec. 4: the coupling matrices are the kernel
                         sampled at the interpolation points).  Needs far_low = 0 and
                         batch_rhs <= 1; bem_export_far then returns BEM_EUNSUPPORTED.
                         0: blocks computed once at assembly and stored               */
    double kappa_adm; /* Helmholtz: a far pair also needs |kappa| * 2 max(r_t, r_s) <= kappa_adm,
                         so that q nodes resolve the kernel's oscillation over the clusters
                         (survey reading of the paper's silence on large wavenumbers); 0: no
                         such bound.  Ignored for Laplace. */
} bem_h2_params;

/* arithmetic of the far-field coupling in bem_apply_ex / refined solves */
#define BEM_PREC_FP64 0
#define BEM_PREC_FP32 1 /* blocks stored in FP32, products accumulated in FP32 */
#define BEM_PREC_BF16 2 /* blocks stored in BF16, products accumulated in FP32 */

/* Sizes and counts of an operator, filled by bem_assemble_plan. */
typedef struct bem_operator_info {
    int64_t ndof;            /* rows = cols = N */
    int64_t nclusters;       /* clusters of all levels 0..leaf */
    int64_t nfar;            /* admissible (far) cluster pairs, both orientations */
    int64_t nnear;           /* near leaf pairs */
    int64_t ntouch;          /* touching element pairs (singular quadrature) */
    int64_t near_nnz;        /* non-zeros of the near field in the B-spline basis */
    int64_t leaf_level;      /* leaf level actually used */
    size_t op_bytes;         /* persistent device workspace for bem_assemble */
    size_t tmp_bytes;        /* temporary device workspace, free after bem_assemble */
    double far_bytes;        /* bytes of stored coupling blocks (each pair stored once) */
    double near_bytes;       /* bytes of near-field values + column indices */
    int64_t nstored;         /* stored coupling blocks (= nfar / 2) */
    int64_t nchunks;         /* work chunks of the coupling kernel */
    double transposed_bytes; /* bytes of the per-column transposed products */
    int64_t nlocal;          /* local functions (patch by patch); = ndof except on S^0 and S^1 spaces */
} bem_operator_info;

/* GMRES(m) parameters (reading: restart 30, x0 = 0, relative residual tolerance). */
typedef struct bem_solve_params {
    int restart;      /* Krylov dimension m per cycle, 1..64 */
    int maxit;        /* total Arnoldi steps over all cycles (and refinement steps), >= 1 */
    double tol;       /* stop when ||b - A x|| <= tol ||b|| (true FP64 residual, checked) */
    int refine;       /* 0: GMRES on the FP64 operator.  1: FP64 refinement: each outer step
                         solves A_low d = r (inner GMRES on the operator with the
                         low-precision far field, far_low at assembly) to inner_tol, and
                         x moves along d and the earlier outer directions by the
                         combination that minimises the FP64 residual ||b - A x|| (a
                         flexible outer Krylov loop: generalised conjugate residuals over
                         the images A d, orthonormalised in FP64; up to 16 directions are
                         kept, then the loop restarts from x); r = b - A x is recomputed in
                         FP64 after every step, until it meets tol */
    int max_outer;    /* refinement steps at most (0 = 20) */
    double inner_tol; /* relative tolerance of each inner solve (0: 1e-4 with an FP32 far
                         field, 1e-2 with BF16, whose rounded moments leave the inner
                         operator's residual near 1e-3 of the right-hand side) */
    int precond;      /* BEM_PRECOND_NONE, or BEM_PRECOND_BLOCK: right preconditioning with
                         the operator's block preconditioner (bem_precond_build first) */
    int inner_maxit;  /* Arnoldi steps of one inner solve at most (0 = 3 * restart); the outer
                         loop takes whatever the inner solve reached (measured: with the
                         flexible outer loop, short inner solves cost fewer steps in all) */
    int reserved[2];  /* must be zero */
} bem_solve_params;

#define BEM_PRECOND_NONE 0
#define BEM_PRECOND_BLOCK 1

/* per-RHS solver statistics */
typedef struct bem_solve_stats {
    int iterations;       /* Arnoldi steps taken (all inner solves) */
    int converged;        /* 1 if the true relative residual is <= tol */
    double relres;        /* true relative FP64 residual ||b - A x|| / ||b|| at exit */
    int outer;            /* refinement steps (0 without refinement) */
    int reserved;
} bem_solve_stats;

/* Message of the last failed call on this thread (never NULL). */
const char* bem_last_error(void);

/* Analytic geometry (Sec. 4 "Geometry"; App. D multi-patch boundary representation with
 * outward normals and matching parametrisations on shared edges).
 * kind: BEM_GEOM_*; params/nparams as listed above (host array).  -> *out. */
int bem_geometry_analytic(int kind, const double* params, int nparams, bem_geometry* out);
void bem_geometry_destroy(bem_geometry g);

/* Patches given by NURBS maps (App. C: gamma(x, y) = sum c_{j1 j2} b_{j1}(x) b_{j2}(y) w_{j1 j2}
 * / sum b_{i1}(x) b_{i2}(y) w_{i1 i2}, App. D: outward normals, matching parametrisations on
 * shared edges; the caller guarantees both, the library does not check them).
 * meta: host, 4 ints per patch: degrees p1, p2 (0..8) and basis counts k1 > p1, k2 > p2
 *       (<= 4096).
 * knots: host, per patch the k1 + p1 + 1 knots of the first direction then the k2 + p2 + 1
 *       of the second, patch after patch; non-decreasing and clamped (the first and the
 *       last degree + 1 knots are 0 and 1).
 * cw:   host, per patch k1 * k2 control points x, y, z, w (w > 0), j1 outer, patch after
 *       patch.
 * The library copies the tables (a small device copy is allocated here and freed with the
 * last space made from the geometry).  EINVAL names the offending patch. */
int bem_geometry_nurbs(int npatch, const int* meta, const double* knots, const double* cw, bem_geometry* out);

/* File import and export of NURBS patch sets (Sec. 4 "Geometry": the geometry is imported
 * from a file).  Plain text, '#' starts a comment to the end of its line: the word BEMNURBS
 * and the version 1, the number of patches, then per patch "p1 p2 k1 k2", the knots of the
 * two directions and k1 * k2 lines "x y z w" (j1 outer); the same checks as
 * bem_geometry_nurbs.  bem_geometry_save writes a NURBS geometry (EINVAL for analytic ones)
 * with 17 significant digits, so that a saved and reloaded geometry is the same. */
int bem_geometry_load(const char* path, bem_geometry* out);
int bem_geometry_save(bem_geometry g, const char* path);

/* User-supplied patch maps (Sec. 4 "Geometry": arbitrary smooth maps; App. D conditions are
 * the caller's).  The library calls gamma(patch, st, n, xyz, jac, user) once per patch at
 * setup, on the host, for n = (intervals + degree)^2 parameter points st (n x 2, row-major)
 * and reads xyz (n x 3, row-major; every entry must be finite); jac (n x 6) may be filled
 * or ignored, it is not used.  Reading of the paper's arbitrary maps: each patch map is
 * replaced by its tensor B-spline interpolant of the given degree (1..8) on `intervals`
 * (1..1024) uniform intervals per direction, interpolating at the Greville abscissae of the
 * clamped knot vector (so that shared edges, sampled at the same points from both sides,
 * stay shared); the result is a NURBS geometry with unit weights.  Its error against the
 * map decays like intervals^-(degree + 1) for smooth maps and is zero for polynomial maps of
 * at most that degree. */
typedef void (*bem_user_map)(int patch, const double* st, int64_t n, double* xyz, double* jac, void* user);
int bem_geometry_user(int npatch, bem_user_map gamma, void* user, int degree, int intervals, bem_geometry* out);

/* Discrete space (Sec. 4 "Discretization"; App. E): the spline space S^2 of tensor
 * B-splines of degree `degree` over 2^level equal elements per direction on every patch,
 * interior knots repeated `knot_repetition` times (1 <= knot_repetition <= degree + 1),
 * lifted to the surface by the Piola transform, for the PDE `kernel`
 * (BEM_LAPLACE_SINGLE or BEM_HELMHOLTZ_SINGLE with wavenumber kappa_re + i kappa_im != 0;
 * non-resonance is assumed, Sec. 2).  EINVAL on degree < 0, level < 0 or > 12, bad knot
 * repetition, or kappa = 0 for Helmholtz.  The geometry may be destroyed afterwards.
 * Build limit: degree <= 2 (EUNSUPPORTED above).  The singular-quadrature kernel keeps the
 * (d+1)^2 x (d+1)^2 element-pair block of every Duffy region in registers; at d = 2 it
 * already takes all 256 VGPRs of a lane (FP64: 256 VGPRs + 8 AGPRs, complex: 256 + 59,
 * occupancy 1 wave per SIMD, from the compiler's kernel resource report), so d = 3 (256
 * accumulators, 512 for complex) would spill; the element basis tables hold polynomials of
 * degree <= 2. */
int bem_space_create(bem_geometry g, int kernel, double kappa_re, double kappa_im, int degree,
                     int knot_repetition, int level, bem_space* out);

/* The spline spaces of App. E on the patches: */
#define BEM_SPACE_S2 2 /* S^2: discontinuous across patches, 2-form (Piola) lifting (default) */
#define BEM_SPACE_S0 0 /* S^0: continuous across patch boundaries, 0-form lifting */
#define BEM_SPACE_S1 1 /* S^1: div-conforming vector fields, normal continuity across patches */
/* bem_space_create with the space kind.  S^0 (conforming in H^1/2; degree >= 1): the local
 * B-splines of a patch are lifted as phi = phi_hat o gamma^-1, so every surface integral
 * (Galerkin entries, moments, load vector, potential) carries the surface element kappa;
 * the local functions that do not vanish on a shared edge or vertex are glued into one
 * global function (reading: functions whose Greville-point images coincide within 1e-10 of
 * the largest coordinate are the same; the matching condition of App. D makes these the
 * traces that agree).  Global functions are numbered in the order of their first local
 * function (patch, j1, j2).  Every vector over the DOFs of an S^0 space (load vectors,
 * densities, products, solutions) has the global length bem_space_ndof returns.  Operators
 * on S^0 spaces: FP64, one column per pass (far_low = 0, batch_rhs <= 1), no block
 * preconditioner, no grouped launches, no stage timing (EUNSUPPORTED). */
/* S^1 (conforming in H^-1/2(div); kernel BEM_MAXWELL_SINGLE, which needs this space kind and
 * kappa != 0; degree p = 1 or 2, EINVAL below, EUNSUPPORTED above; knot_repetition 1 only,
 * EUNSUPPORTED otherwise): on every patch the reference fields of component 0,
 * b^p_j1(s) b^{p-1}_j2(t) e_s (j1 < 2^L + p, j2 < 2^L + p - 1), and of component 1,
 * b^{p-1}_j1(s) b^p_j2(t) e_t (j1 < 2^L + p - 1, j2 < 2^L + p), with the B-splines b of the
 * indicated degrees on simple interior knots; local index
 * (patch * 2 + component) * (2^L + p) * (2^L + p - 1) + (component 0: j1 * (2^L + p - 1) + j2,
 * component 1: j1 * (2^L + p) + j2).  They are lifted by the Piola transform of vector fields
 * (D gamma v_hat / kappa on the surface; divergence div v_hat / kappa).  The functions whose
 * degree-p index is first or last have a normal component on that patch edge; by the
 * matching condition (App. D) each meets one function of the neighbouring patch with the
 * same trace of its tangential factor, and the two are glued into one global function, the
 * second taken with the sign that makes the flux leaving one patch enter the other (reading:
 * partners are the functions whose anchors coincide within 1e-10 of the largest coordinate,
 * the anchor being the image of the edge point at the mean of the Greville abscissa and the
 * support centre of the tangential factor).  Edge functions without a partner (open
 * surfaces) are dropped.  Global functions are numbered in the order of their first local
 * function; bem_space_glue gives the map (-1: dropped), bem_space_glue_sign the signs.
 * Operators on S^1 spaces (FP64 complex; far_low = 0, batch_rhs <= 1, far_eval = 0;
 * 1 <= qg <= 8, 1 <= qs <= 16):
 *   eta = 0: dense Galerkin matrix (at most 32768 elements; tmp workspace of every element
 *     pair's block, nelem^2 (2p(p+1))^2 complex);
 *   eta > 0: compressed by the interpolation of Sec. 2 on the block partition of the scalar
 *     operators of the same surface (cluster tree, admissibility, q Chebyshev nodes per
 *     direction, 1 <= q <= 8, leaf_level; default leaf level L - 1).  The form splits into
 *     four scalar kernel products, one per channel: the three components of the lifted
 *     field and the divergence (weight -kappa^-2), so one coupling block of the kernel serves
 *     all four; element pairs in near leaf pairs keep their Galerkin blocks, which are
 *     summed with the gluing signs into a sparse matrix over the global functions at
 *     assembly (the apply reads that matrix).  The channel moments of every element
 *     against its leaf's Lagrange polynomials use the qg x qg Gauss rule per element.
 *     info.nfar/nnear/nclusters describe the partition, near_nnz the near element-pair block
 *     entries, near_bytes the bytes of the glued near matrix (values, columns, row pointers).
 * bem_apply and bem_solve (no preconditioner, no refinement) work as for the other spaces;
 * the block preconditioner, grouped launches, stage timing, the exports, the cluster-tree
 * potential, sampled data and VTK output return EUNSUPPORTED. */
int bem_space_create_ex(bem_geometry g, int kernel, double kappa_re, double kappa_im, int degree,
                        int knot_repetition, int level, int space_kind, bem_space* out);
/* N: the space's functions (S^0: global, glued ones). */
int bem_space_ndof(bem_space s, int64_t* n);
/* Local functions (patch by patch, the numbering of the near field's CSR export) into
 * *nlocal and, if glue_host is not NULL, the global function of each (host, nlocal entries;
 * the identity for S^2). */
int bem_space_glue(bem_space s, int64_t* nlocal, int32_t* glue_host);
/* Sign of every local function in its global function (host, nlocal entries): S^1 +1 or -1
 * (0 for dropped functions), +1 on the other spaces. */
int bem_space_glue_sign(bem_space s, int32_t* sign_host);
void bem_space_destroy(bem_space s);

/* Load vectors (Sec. 4 "Boundary Values"): b_g = int_Gamma g psi_g for nrhs data sets.
 * data_params: host array of 3 doubles per RHS.  b_dev: device, N x nrhs column-major with
 * leading dimension ldb >= N, written (not accumulated).  Gauss with 8 points per direction
 * per element.  EINVAL on PLANE_WAVE for Laplace.  S^1 spaces: the kinds DIPOLE and
 * PLANE_WAVE_E only, 6 doubles per RHS, complex b. */
int bem_rhs(bem_space s, int data_kind, const double* data_params, int nrhs, void* b_dev,
            int64_t ldb, hipStream_t stream);

/* Load vectors from user data (Sec. 4 "Boundary Values" takes the Dirichlet data as a
 * function; here it is sampled where the quadrature needs it).  bem_rhs_quadpoints writes
 * the number of quadrature points, nelem * 64, to *npts and, if xyz_dev is not NULL, the
 * points themselves (device, npts x 3 row-major; point e * 64 + 8 a1 + a2 is Gauss point
 * (a1, a2) of element e = (patch, i1, i2), the rule of bem_rhs).  bem_rhs_from_samples
 * computes b_g = int_Gamma g psi_g by that rule from g_dev (device, npts x nrhs
 * column-major, leading dimension ldg >= npts; FP64, interleaved complex for Helmholtz)
 * into b_dev (N x nrhs, ldb >= N, written).  With samples of a built-in data function it
 * reproduces bem_rhs. */
int bem_rhs_quadpoints(bem_space s, double* xyz_dev, int64_t* npts, hipStream_t stream);
int bem_rhs_from_samples(bem_space s, const void* g_dev, int64_t ldg, int nrhs, void* b_dev, int64_t ldb,
                         hipStream_t stream);

/* Host plan of the compressed system matrix (Sec. 4 "System Matrix"): cluster tree on the
 * patches' parameter squares, block partition into admissible (far) cluster pairs and
 * near leaf pairs, near-field sparsity pattern, touching element pairs.  Creates *out (no
 * device memory yet) and fills *info with counts and workspace sizes.  Host work only. */
int bem_assemble_plan(bem_space s, const bem_h2_params* p, bem_operator* out,
                      bem_operator_info* info);

/* Assembles the operator on the device (near-field Galerkin quadrature with Duffy rules
 * for touching pairs, coupling blocks at Chebyshev nodes, moment and transfer tables).
 * op_ws: device workspace of >= info.op_bytes bytes, owned by the caller and used by the
 * operator until it is destroyed.  tmp_ws: device workspace of >= info.tmp_bytes bytes,
 * free again once the stream has passed this call.  ENOMEM if a size is too small. */
int bem_assemble(bem_operator A, void* op_ws, size_t op_bytes, void* tmp_ws, size_t tmp_bytes,
                 hipStream_t stream);

int bem_operator_info_get(bem_operator A, bem_operator_info* info);

/* rows() and cols() of the system matrix (Sec. 4 "System Matrix"). */
int bem_operator_dims(bem_operator A, int64_t* rows, int64_t* cols);

/* y = A x, the GEMV H*x of Sec. 4 "System Matrix": forward transform to leaf moments,
 * upward transfer, far-field coupling, downward transfer, backward transform, plus the
 * near-field product.  x_dev, y_dev: device, N x nrhs column-major, leading dimensions
 * ldx, ldy >= N, must not overlap.  y is overwritten.  nrhs >= 1. */
int bem_apply(bem_operator A, const void* x_dev, int64_t ldx, void* y_dev, int64_t ldy, int nrhs,
              hipStream_t stream);

/* y = A x like bem_apply with the far-field coupling in the given precision:
 * BEM_PREC_FP64, or the low precision the operator was assembled with (far_low); EINVAL
 * if that copy does not exist.  Near field, transforms and transfers stay FP64.  With
 * batch_rhs > 1 at planning and nrhs > 1, columns go through the many-RHS kernels in
 * passes of up to batch_rhs columns; BEM_PREC_BF16 there multiplies BF16 blocks and BF16
 * moments on the matrix cores with FP32 accumulation. */
int bem_apply_ex(bem_operator A, int precision, const void* x_dev, int64_t ldx, void* y_dev, int64_t ldy,
                 int nrhs, hipStream_t stream);

/* Device workspace bytes bem_solve needs for nrhs right-hand sides with parameters p
 * (refinement adds 2 min(max_outer, 16) vectors per right-hand side of a pass). */
int bem_solve_plan(bem_operator A, int nrhs, const bem_solve_params* p, size_t* bytes);

/* Restarted GMRES(m) on A (Sec. 4 "Solution of the System of Linear Equations"), x0 = 0,
 * classical Gram-Schmidt with one reorthogonalisation, Givens rotations and the triangular
 * solve on the device; a cycle ends early when the rotated residual estimate of a step
 * reaches tol, and convergence is decided on the true relative residual computed at the
 * start of the next cycle.  1 <= restart <= 64.  b_dev, x_dev: device N x nrhs
 * column-major; x is overwritten with the last iterate.  stats: host array of nrhs
 * entries.  ws: device workspace of >= the bytes from bem_solve_plan.  Blocks the calling
 * thread until the solve is done.  Returns ENOCONV (stats and x still written) if some
 * right-hand side misses the tolerance within maxit steps. */
int bem_solve(bem_operator A, const void* b_dev, int64_t ldb, void* x_dev, int64_t ldx, int nrhs,
              const bem_solve_params* p, bem_solve_stats* stats, void* ws, size_t ws_bytes,
              hipStream_t stream);

/* Potential u(x) = int_Gamma k(x, y) rho(y) dsigma_y at npts points (Sec. 4 "Evaluation of
 * the Solution"; App. B (LS)/(HS)), Gauss with 8 points per direction per element.
 * pts_dev: device, npts x 3 row-major.  rho_dev: device N x nrhs (leading dim ldr).
 * u_dev: device npts x nrhs column-major (leading dim ldu >= npts), overwritten.
 * With npts == 0 nothing is done and pts_dev, u_dev may be NULL.  S^1 spaces (Maxwell): the
 * field (MS), E(x) = int_Gamma G(x - y) j(y) dsigma_y + kappa^-2 grad_x int_Gamma G(x - y)
 * div_Gamma j(y) dsigma_y with the (HS) kernel G and the surface current j of the
 * coefficients rho, by the same rule; u_dev then holds 3 complex values per point (npts x 3
 * row-major per column, ldu >= 3 npts). */
int bem_eval_potential(bem_space s, const double* pts_dev, int64_t npts, const void* rho_dev,
                       int64_t ldr, int nrhs, void* u_dev, int64_t ldu, hipStream_t stream);

/* Potential at many points through the operator's cluster tree (Sec. 4 "Evaluation of the
 * Solution", accelerated by the interpolation of Sec. 2 on the source side): for every
 * point, each patch's clusters are visited from the root; a cluster whose ball (centre c,
 * radius r) satisfies dist = |x - c| - r > 0 and 2 r <= eta * dist (ties within 1e-12 dist
 * count as not admissible) contributes sum_a k(x, gamma(xi_a)) m_a over its q x q Chebyshev
 * points with the moments m of rho (the operator's forward transform and upward transfer);
 * a leaf that is not admissible contributes the 8 x 8 Gauss sums of its elements, as
 * bem_eval_potential; other clusters pass the point to their children.  eta >= 0 (0: every
 * point takes the plain quadrature, identical to bem_eval_potential up to summation order;
 * the operator's own eta is the usual choice).  The error against bem_eval_potential decays
 * geometrically with the operator's q.  Cost per point O(q^2 log N) for points away from
 * the surface instead of O(N).  pts_dev: device npts x 3 row-major; rho_dev: device N x
 * nrhs (ld ldr); u_dev: device npts x nrhs (ld ldu >= npts), overwritten.  Uses the
 * operator's matvec scratch (moments): overlapping calls on one operator race. */
int bem_eval_potential_h2(bem_operator A, const double* pts_dev, int64_t npts, const void* rho_dev, int64_t ldr,
                          int nrhs, void* u_dev, int64_t ldu, double eta, hipStream_t stream);

/* Visualisation of the density and the geometry in VTK format (Sec. 4 "Visualization"):
 * writes a legacy ASCII VTK unstructured grid with (nsub + 1)^2 points and nsub^2
 * quadrilaterals (cell type 9) per element, point e * (nsub + 1)^2 + a * (nsub + 1) + b at
 * parameter (i1 + a / nsub, i2 + b / nsub) 2^-L of element e = (patch, i1, i2), and point
 * data "kappa" (surface element |d_s gamma x d_t gamma|, by central differences with step
 * 1e-6) and, per column r of rho, the density on the surface, rho_hat / kappa (2-form
 * lifting, S^2) or rho_hat (0-form, S^0, coefficients of the global functions), as "rho_r"
 * (Laplace) or "rho_re_r", "rho_im_r" (Helmholtz).  rho_host: host,
 * N x nrhs column-major (leading dimension ldr >= N), may be NULL with nrhs = 0 (geometry
 * only); 0 <= nrhs <= 64, 1 <= nsub <= 64.  Host work only. */
int bem_write_vtk(bem_space s, const void* rho_host, int64_t ldr, int nrhs, int nsub, const char* path);

/* Stage timing of bem_apply (tracing).  While enabled (on != 0), every one-column apply
 * records HIP events on its stream around its four stages: 0 near-field product (y
 * overwritten) beside the forward transform and upward transfer (Sec. 4: moments of every
 * cluster), 1 far-field coupling, 2 gather of the local expansions, 3 downward transfer +
 * backward transform added to y.  Many-RHS applies (batch_rhs > 1) record their own five
 * stages.  Enabling or disabling clears the record.  bem_profile_read waits for the last
 * recorded event, writes the mean milliseconds of each stage over the recorded applies
 * into stage_ms[0..nstages-1] (nstages >= 4), their number into *napplies, and clears the
 * record. */
int bem_profile_enable(bem_operator A, int on);
int bem_profile_read(bem_operator A, double* stage_ms, int nstages, int* napplies);

/* Profiling aid: launch stage `stage` (0..3 as above) of a one-column apply of x into y
 * on `stream`, alone.  The stages pass their results through the operator's scratch
 * (moments, transposed products, row sums, local expansions), so a stage computes from
 * what the previous stages of the last apply left there; stages 0-2 are idempotent when
 * repeated, stage 3 adds to y again.  Back-to-back launches of one stage time its kernel
 * without the launch gaps that the stage events include.  prec as in bem_apply_ex.
 * x_dev, y_dev: device, N scalars each (stage 0 reads x and writes y; 3 adds to y).
 * EINVAL: bad stage, precision not available, operator not assembled. */
int bem_apply_stage(bem_operator A, int prec, int stage, const void* x_dev, void* y_dev, hipStream_t stream);

/* ---- block-Jacobi preconditioner with a learned low-rank correction -------------------
 * Not part of the paper (its example program runs GMRES unpreconditioned); an addition to
 * cut iterations on the first-kind single-layer systems.  Blocks are tiles of 8 x 8
 * consecutive B-spline indices of a patch (64 DOFs, shorter at a patch's end; DOF
 * (f, j1, j2) sits in slot (j1 % 8) * 8 + j2 % 8 of tile (f, j1 / 8, j2 / 8), tiles
 * numbered (f * nt + j1 / 8) * nt + j2 / 8 with nt = ceil(nb / 8)).  D_b is the near-field
 * part of A[b, b]; its inverse is formed by Gauss-Jordan elimination with partial pivoting
 * (unused slots of short tiles carry identity).  GMRES uses M^{-1} as a right
 * preconditioner (bem_solve_params.precond), so its residual is the true residual. */

/* Number of tiles and bytes of the device workspace bem_precond_build needs. */
int bem_precond_info(bem_operator A, int64_t* ntiles, size_t* ws_bytes);

/* Extracts and inverts every block (the plain inverse becomes the active one).  ws: device
 * workspace of >= ws_bytes, owned by the caller, used until the operator is destroyed or
 * the preconditioner is rebuilt.  EDEVICE if a block is singular. */
int bem_precond_build(bem_operator A, void* ws, size_t ws_bytes, hipStream_t stream);

/* z = M^{-1} r for nrhs columns (device, column-major, leading dimensions >= N). */
int bem_precond_apply(bem_operator A, const void* r, int64_t ldr, void* z, int64_t ldz, int nrhs,
                      hipStream_t stream);

/* Host copy of the active (which = 0) or plain (which = 1) inverses: ntiles x 64 x 64
 * scalars, row-major per tile, in slot order. */
int bem_precond_export(bem_operator A, int which, double* inv_host, hipStream_t stream);

/* Features of every tile for the correction network (device float, ntiles x 99): the
 * Jacobian of the patch map at the 4 x 4 cell centres of the parameter box of the
 * elements the tile's B-splines meet, with respect to box coordinates (d/ds x 3, d/dt x 3
 * per point, points row by row), then Re kappa / 10, Im kappa / 10, level / 8. */
int bem_precond_features(bem_operator A, float* feats_dev, hipStream_t stream);

/* Training targets of the correction network: for tiles [t0, t0 + nt), (X_b - D_b^{-1}) / s_b
 * as device float ntiles x 64 x 64 (interleaved re, im for Helmholtz; written at tile
 * index), where X_b is the block least-squares approximate inverse
 * X_b = argmin ||A[N(b), b] X - I[N(b), b]||_F = (A_Nb^H A_Nb)^{-1} D_b^H on N(b), the tile
 * extended by `ring` (0..8) B-spline indices per side inside the patch, A_Nb the near field
 * on the rows of N(b) and the columns of b, and s_b = ||D_b^{-1}||_F / 64.  work: device
 * scratch of >= the bytes from bem_precond_target_bytes(A, ring, nt). */
int bem_precond_target_bytes(bem_operator A, int ring, int64_t nt, size_t* bytes);
int bem_precond_targets(bem_operator A, int ring, int64_t t0, int64_t nt, void* work, size_t work_bytes,
                        float* delta_dev, hipStream_t stream);

/* Installs the learned correction M_b^{-1} = D_b^{-1} + s_b U_b V_b^T from the network output
 * uv_dev (device float, ntiles x out; out = [U (64 x 8, row-major), V (64 x 8)] for Laplace,
 * [Re U, Im U, Re V, Im V] for Helmholtz).  mode 2: keep it only for blocks where it lowers
 * the least-squares residual ||[p; 0] - A[N(b), b] z|| (the quantity X_b minimises) for each
 * of 4 seeded probe vectors p, else fall back to D_b^{-1}; mode 1: keep all; mode 0: plain
 * block-Jacobi again.
 * accepted_host (may be NULL): ntiles flags. */
int bem_precond_correct(bem_operator A, const float* uv_dev, int mode, int ring, int* accepted_host,
                        hipStream_t stream);

/* Keeps the learned correction (uv_dev as for bem_precond_correct, installed for every
 * block) only if one GMRES(restart) cycle of the preconditioned true operator on b_dev
 * (device, one column) ends with a lower residual than the same cycle with plain
 * block-Jacobi; otherwise plain block-Jacobi is installed again.  ws: device workspace of
 * >= the bytes from bem_solve_plan(A, 1, ...) plus N scalars.  *kept: 1 if the correction
 * stays; relres2 (may be NULL): the two cycles' relative residuals (plain, learned). */
int bem_precond_select(bem_operator A, const float* uv_dev, const void* b_dev, int restart, void* ws,
                       size_t ws_bytes, int* kept, double* relres2, hipStream_t stream);

/* ---- the correction network: in -> hidden -> hidden -> out, ReLU, trained on the device --
 * Parameters: one FP32 device array, W1 [in][hidden], b1, W2 [hidden][hidden], b2,
 * W3 [hidden][out], b3 (row-major).  precision 0: FP32 products; 1: BF16 operands on the
 * matrix cores with FP32 accumulation.  ws: device workspace of >= ws_bytes for the batch. */
int bem_mlp_sizes(int in, int hidden, int out, int batch, int64_t* nparams, size_t* ws_bytes);
/* He-uniform weights from a counter-based generator (splitmix64 of seed and index), zero biases. */
int bem_mlp_init(int in, int hidden, int out, uint64_t seed, float* params_dev, hipStream_t stream);
/* Y [batch][out] = net(X [batch][in]) (device, row-major). */
int bem_mlp_forward(int in, int hidden, int out, int batch, const float* params_dev, const float* X_dev, float* Y_dev,
                    int precision, void* ws, size_t ws_bytes, hipStream_t stream);
/* Y = net(X) like bem_mlp_forward, for callers that cannot allocate device memory (code under
 * HIP graph capture, serving loops, harnesses that forbid allocation): no workspace argument
 * and no allocation of any kind.  The hidden activations (2 * batch * hidden floats) live in a
 * fixed 32 MiB device array of the library, one per GPU, held until the process ends; its
 * address is looked up on the first call on each device.  EINVAL if 8 * batch * hidden
 * exceeds 32 MiB (33554432 bytes) or batch > 1048576, as for bad sizes.  Every call on one
 * GPU shares that GPU's array: calls that overlap in time on one device (different streams
 * or threads) race and must be serialised by the caller.  Same kernels and results as
 * bem_mlp_forward. */
int bem_mlp_forward_noalloc(int in, int hidden, int out, int batch, const float* params_dev, const float* X_dev,
                            float* Y_dev, int precision, hipStream_t stream);
/* Loss of the rank-8 block correction and its gradient: the network output of sample b is
 * U_b, V_b (64 x 8; out = 1024: [U | V] real, out = 2048: [Re U | Im U | Re V | Im V]);
 * loss = mean_b ||T_b - U_b V_b^T||_F^2 / ||T_b||_F^2 with T (device float, batch x 64 x 64,
 * interleaved complex if is_complex) into loss_dev[0], d loss / d params into grad_dev. */
int bem_mlp_loss_grad(int in, int hidden, int out, int batch, int is_complex, const float* params_dev,
                      const float* X_dev, const float* T_dev, float* grad_dev, float* loss_dev, int precision,
                      void* ws, size_t ws_bytes, hipStream_t stream);
/* One Adam step (bias-corrected moments m, v; step counts from 1). */
int bem_mlp_adam(int64_t n, float* params_dev, const float* grad_dev, float* m_dev, float* v_dev, int step, float lr,
                 float beta1, float beta2, float eps, hipStream_t stream);

/* Destroys the operator (its workspace stays with the caller). */
void bem_operator_destroy(bem_operator A);

/* ---- many operators in one launch per stage, and captured launch sequences -----------
 * A group binds columns of several assembled operators (uneven sizes, the same PDE kind and
 * q) so that y = A x for all of them runs as one launch per matvec stage (five launches in
 * all) instead of several launches per operator and column.  Each bound column gets its
 * own scratch, so the group does not disturb the operators' own applies. */
typedef struct bem_group_s* bem_group;

/* ncols[i] >= 1 columns of ops[i]; all assembled, all Laplace or all Helmholtz, one q.
 * *ws_bytes: device workspace bem_group_bind needs. */
int bem_group_create(int nops, const bem_operator* ops, const int* ncols, bem_group* out, size_t* ws_bytes);
/* Binds the columns: x_cols, y_cols are host arrays of sum(ncols) device pointers (column c
 * of operator i at position ncols[0] + ... + ncols[i-1] + c), each an N_i-vector; y must not
 * overlap x.  ws: device workspace of >= ws_bytes (caller-owned).  Synchronises the stream. */
int bem_group_bind(bem_group G, void* ws, size_t ws_bytes, const void* const* x_cols, void* const* y_cols,
                   hipStream_t stream);
/* y = A x for every bound column (FP64), five launches on `stream`, nothing else (capturable). */
int bem_group_apply(bem_group G, hipStream_t stream);
void bem_group_destroy(bem_group G);

/* Stream capture of a sequence of library calls that only launch kernels (bem_apply,
 * bem_apply_ex, bem_group_apply, bem_precond_apply) into a HIP graph, replayed with one
 * launch.  Between begin and end nothing may synchronise the stream. */
typedef struct bem_graph_s* bem_graph;
int bem_capture_begin(hipStream_t stream);
int bem_capture_end(hipStream_t stream, bem_graph* out);
int bem_graph_launch(bem_graph g, hipStream_t stream);
void bem_graph_destroy(bem_graph g);

/* ---- introspection for parity checks (host copies; each synchronises the stream) ----- */

/* Near field in CSR form: rowptr (N+1, int64), col (nnz, int32), val (nnz scalars).
 * Any pointer may be NULL to skip it; the pattern is available right after
 * bem_assemble_plan, the values only after bem_assemble. */
int bem_export_near(bem_operator A, int64_t* rowptr, int32_t* col, double* val, hipStream_t stream);

/* Far list as (target, source) cluster index pairs (int64, 2 per block), cluster index =
 * level offset + (patch * 2^level + i) * 2^level + j, and the q^2 x q^2 coupling block of
 * each pair (row-major, target node index a = a1*q + a2), in the order of the list.
 * Either pointer may be NULL; the list is available right after bem_assemble_plan. */
int bem_export_far(bem_operator A, int64_t* pairs, double* blocks, hipStream_t stream);

/* Moments of all clusters (nclusters x q^2 per RHS column) after forward + upward
 * transfer of x (1 RHS). */
int bem_export_moments(bem_operator A, const void* x_dev, double* mom_host, hipStream_t stream);

#ifdef __cplusplus
}
#endif

#endif /* BEM_H */
