// C ABI of libbem_hip.so (declared in include/bem.h): handles, workspace layout, the
// assembly and matvec drivers, GMRES and the parity exports.
#include "../../include/bem.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <complex>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <iterator>
#include <memory>
#include <new>
#include <sstream>
#include <string>
#include <vector>

#include "bem_batch.h"
#include "bem_kernels.h"
#include "bem_mlp.h"
#include "bem_maxwell.h"
#include "bem_plan.h"
#include "bem_precond.h"
#include "bem_solve.h"

using namespace bem;

namespace {

thread_local std::string g_err = "";

int fail(int code, const std::string& msg) {
    g_err = msg;
    return code;
}

#define HIP_CHECK(expr)                                                                       \
    do {                                                                                      \
        hipError_t e_ = (expr);                                                               \
        if (e_ != hipSuccess)                                                                 \
            return fail(BEM_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_));      \
    } while (0)

// bump allocator over a caller workspace (base == nullptr: size computation only)
struct Bump {
    char* base;
    size_t off = 0;
    explicit Bump(void* b) : base((char*)b) {}
    template <class X>
    X* take(size_t n) {
        off = (off + 255) / 256 * 256;
        X* p = base ? (X*)(base + off) : nullptr;
        off += n * sizeof(X);
        return p;
    }
};

}  // namespace

// NURBS table of a geometry (layout in bem_core.h): the host copy and a device copy of the
// same doubles; shared by the geometry and every space made from it
struct GeomTab {
    std::vector<double> host;
    double* dev = nullptr;
    ~GeomTab() {
        if (dev) (void)hipFree(dev);
    }
};

struct bem_geometry_s {
    GeomDesc g;
    std::shared_ptr<GeomTab> tab;
};

// S^0 gluing of a space: local -> global map and the inverse in CSR form, host and device
struct GlueTab {
    std::vector<int32_t> glue, ginv_idx;
    std::vector<int64_t> ginv_ptr;
    int32_t* d_glue = nullptr;
    int64_t* d_ptr = nullptr;
    int32_t* d_idx = nullptr;
    ~GlueTab() {
        if (d_glue) (void)hipFree(d_glue);
        if (d_ptr) (void)hipFree(d_ptr);
        if (d_idx) (void)hipFree(d_idx);
    }
};

// S^1 (div-conforming) tables of a space: local B-spline polynomials of degrees p and p - 1,
// the local -> global map with signs per element position, and the pieces of every global
// function; host copies and device copies
struct MxTab {
    int p = 1, nbp = 0, nbq = 0, nl = 0;
    int64_t nloc = 0, nglob = 0;
    std::vector<double> polp, polq;
    std::vector<int32_t> glob, sgn;    // per local function
    std::vector<int32_t> eglob, esgn;  // per element position
    std::vector<int64_t> gptr;
    std::vector<int32_t> gpos, gsgn;
    double* d_polp = nullptr;
    double* d_polq = nullptr;
    int32_t* d_eglob = nullptr;
    int32_t* d_esgn = nullptr;
    int64_t* d_gptr = nullptr;
    int32_t* d_gpos = nullptr;
    int32_t* d_gsgn = nullptr;
    ~MxTab() {
        for (void* q : {(void*)d_polp, (void*)d_polq, (void*)d_eglob, (void*)d_esgn, (void*)d_gptr, (void*)d_gpos,
                        (void*)d_gsgn})
            if (q) (void)hipFree(q);
    }
};

struct bem_space_s {
    SpaceDesc S;
    BasisTab bt;
    std::shared_ptr<GeomTab> tab;    // keeps a NURBS geometry's tables alive
    std::shared_ptr<GlueTab> glue;   // S^0 only
    std::shared_ptr<MxTab> mx;       // S^1 only
};

struct bem_operator_s {
    bem_space_s* sp = nullptr;
    Plan plan;
    bool cplx = false;
    bool assembled = false;
    bem_operator_info info{};
    std::vector<int32_t> touch_lp;
    std::vector<int64_t> fb_off;  // host copies of the per-pair block table (kept until destroy,
    std::vector<int32_t> fb_rs;   // the uploads above are asynchronous)
    std::vector<double> ec;       // leaf-to-ancestor transfers of the many-RHS path (same)
    // dense near-field tiles of the many-RHS path (see BatchDev)
    std::vector<int64_t> tile_rowptr, tile_colptr, tile_voff;
    std::vector<int32_t> tile_rows, tile_cols;
    OpDev dev{};
    // Maxwell single layer on S^1: dense operator (element-pair classification in plan)
    bool mx = false;
    MxDev mxd{};
    bool mxh = false;  // far field compressed (Sec. 2 interpolation, four channels)
    MxhDev mxhd{};
    std::vector<int64_t> mxh_plist;  // near element pairs (host copy, as the pair types)
    std::vector<double> mxh_lg;      // leaf Lagrange values at the Gauss points (same)
    std::vector<int32_t> mxh_ch_p0, mxh_ch_p1;  // coupling work chunks (same)
    std::vector<int64_t> mxh_tr_ptr;            // per cluster: stored blocks where it is the partner
    std::vector<int32_t> mxh_tr_blk;
    std::vector<int64_t> mx_blist;              // pair blocks by kind: regular, then touching (same)
    std::vector<int64_t> mxh_cl_chunk;
    std::vector<int64_t> mxh_nrowptr;  // glued near field: CSR pattern over the global functions
    std::vector<int32_t> mxh_ncol;
    std::vector<int32_t> mx_tinfo;  // host copies of the pair types and the Gauss rules (kept,
    std::vector<double> mx_rules;   // the uploads are asynchronous)
    size_t scal = 8;  // bytes per scalar
    int far_low = 0;  // low-precision copy of the coupling blocks: 0 none, 1 FP32, 2 BF16
    int batch_rhs = 0;  // columns per many-RHS pass (slabs in the operator workspace)
    bool far_eval = false;  // coupling evaluated in every apply (no stored blocks)
    BatchDev bdev{};
    // block preconditioner (bem_precond_*)
    bool prec_built = false;
    PrecDev pdev{};
    // stage timing of bem_apply (bem_profile_*)
    bool prof = false;
    std::vector<hipEvent_t> ev;  // kApplyStages + 1 events per recorded apply
    size_t ev_used = 0;
    // GMRES: pinned status words and per-step events
    double* pinned = nullptr;
    double* hstat = nullptr;  // coherent host-mapped estimates and stamps (GmresState::hest)
    unsigned stamp = 0;
    double* bpin = nullptr;  // batched GMRES: per-RHS estimates, norms and step counts
    size_t bpin_doubles = 0;
    std::vector<hipEvent_t> sev;
    ~bem_operator_s() {
        for (hipEvent_t e : ev) (void)hipEventDestroy(e);
        for (hipEvent_t e : sev) (void)hipEventDestroy(e);
        if (pinned) (void)hipHostFree(pinned);
        if (hstat) (void)hipHostFree(hstat);
        if (bpin) (void)hipHostFree(bpin);
    }
};

// root level of the subtrees summed by one block each in the upward pass (depth <= 2)
static int up_root_of(const Plan& p) { return std::max(p.leaf - 2, 0); }

static size_t op_layout(const bem_operator_s& A, void* base, OpDev* d, BatchDev* bdo = nullptr) {
    const Plan& p = A.plan;
    Bump b(base);
    OpDev o{};
    o.lev_off = b.take<int64_t>(p.lev_off.size());
    o.rowptr = b.take<int64_t>(p.rowptr.size());
    o.col = b.take<int32_t>(p.col.size());
    o.val = b.take<char>(p.col.size() * A.scal);
    o.grp_rowptr = b.take<int64_t>(p.grp_rowptr.size());
    o.grp_rows = b.take<int32_t>(p.grp_rows.size());
    o.grp_voff = b.take<int64_t>(p.grp_voff.size());
    o.own_rowptr = b.take<int64_t>(p.own_rowptr.size());
    o.own_src = b.take<int32_t>(p.own_src.size());
    o.koff = b.take<int64_t>(p.koff.size());
    o.krs = b.take<int32_t>(p.krs.size());
    o.K = A.far_eval ? nullptr : b.take<char>((size_t)p.ktotal * A.scal);
    o.otf = A.far_eval ? 1 : 0;
    o.otf_wide = p.P.chunk >= 512 ? 1 : 0;
    o.xc = b.take<double>((size_t)p.ncl * p.q2 * 3);
    o.ball = b.take<double>((size_t)p.ncl * 4);
    o.up_count = b.take<int>((size_t)p.S.geom.npatch);
    o.pcol = b.take<int64_t>(p.pcol.size());
    o.P = b.take<char>((size_t)p.ptotal * A.scal);
    o.tr_rowptr = b.take<int64_t>(p.tr_rowptr.size());
    o.tr_off = b.take<int64_t>(p.tr_off.size());
    o.ch_t = b.take<int32_t>(p.ch_t.size());
    o.ch_k0 = b.take<int32_t>(p.ch_k0.size());
    o.ch_k1 = b.take<int32_t>(p.ch_k1.size());
    o.cl_chunk = b.take<int64_t>(p.cl_chunk.size());
    o.partial = b.take<char>(p.ch_t.size() * p.q2 * A.scal);
    o.low = A.far_low;
    o.ktotal_scalars = p.ktotal * (A.cplx ? 2 : 1);
    o.Klow = A.far_low ? b.take<char>((size_t)o.ktotal_scalars * (A.far_low == 1 ? 4 : 2)) : nullptr;
    o.V1 = b.take<double>(p.V1.size());
    o.E = b.take<double>(p.E.size());
    o.mom = b.take<char>((size_t)p.ncl * p.q2 * A.scal);
    o.lv = b.take<char>((size_t)p.ncl * p.q2 * A.scal);
    if (p.S.form == 0) {
        // 0-form lifting: full leaf tables; S^0: local copies of the applied vectors
        o.Vd = b.take<double>((size_t)p.nleaves * p.q2 * p.nloc * p.nloc);
        o.xl = b.take<char>((size_t)p.S.ndof * A.scal);
        o.yl = b.take<char>((size_t)p.S.ndof * A.scal);
    }
    if (A.batch_rhs > 1) {
        // many-RHS slabs and the per-pair block table
        const size_t Rb = (size_t)A.batch_rhs, nch = (Rb + kBatchChunk - 1) / kBatchChunk, N = (size_t)p.S.ndof;
        const size_t np = p.far_t.size();
        BatchDev bd{};
        bd.rmax = A.batch_rhs;
        bd.ntiles = (int64_t)A.tile_rowptr.size() - 1;
        bd.tile_rowptr = b.take<int64_t>(A.tile_rowptr.size());
        bd.tile_rows = b.take<int32_t>(A.tile_rows.size());
        bd.tile_colptr = b.take<int64_t>(A.tile_colptr.size());
        bd.tile_cols = b.take<int32_t>(A.tile_cols.size());
        bd.tile_voff = b.take<int64_t>(A.tile_voff.size());
        bd.tile_val = b.take<char>((size_t)A.tile_voff.back() * A.scal);
        bd.row_grp = b.take<int32_t>(p.row_grp.size());
        bd.row_pos = b.take<int32_t>(p.row_pos.size());
        bd.far_rowptr = b.take<int64_t>(p.far_rowptr.size());
        bd.far_s = b.take<int32_t>(np);
        bd.fb_off = b.take<int64_t>(np);
        bd.fb_rs = b.take<int32_t>(np);
        bd.xs = b.take<char>(N * Rb * A.scal);
        bd.ys = b.take<char>(N * Rb * A.scal);
        bd.mom = b.take<char>((size_t)p.ncl * p.q2 * Rb * A.scal);
        bd.lv = b.take<char>((size_t)p.ncl * p.q2 * Rb * A.scal);
        bd.yl = b.take<char>((size_t)p.nleaves * p.nloc * p.nloc * Rb * A.scal);
        if (A.far_low == 2) {
            bd.Af = b.take<char>(np * bf_row_tiles(A.cplx) * kBatchChunk * 16);
            bd.Bf = b.take<char>((size_t)p.ncl * nch * bf_col_tiles(A.cplx) * kBatchChunk * 16);
        }
        if (A.far_low == 1) bd.mlow = b.take<char>((size_t)p.ncl * p.q2 * Rb * (A.scal / 2));
        bd.Ec = b.take<double>((size_t)p.q2 * ((size_t(2) << p.P.leaf) - 2) + 1);
        if (bdo) *bdo = bd;
    }
    if (d) *d = o;
    return b.off + 256;
}

static size_t tmp_layout(const bem_operator_s& A, void* base, AsmDev* d) {
    const Plan& p = A.plan;
    const SpaceDesc& S = p.S;
    Bump b(base);
    AsmDev a{};
    a.near_t = b.take<int32_t>(p.near_t.size());
    a.near_s = b.take<int32_t>(p.near_s.size());
    a.near_rowptr = b.take<int32_t>(p.near_rowptr.size());
    a.touch_rowptr = b.take<int32_t>(p.touch_rowptr.size());
    a.touch = b.take<int32_t>(p.touch.size());
    a.touch_lp = b.take<int32_t>(A.touch_lp.size());
    a.row_grp = b.take<int32_t>(p.row_grp.size());
    a.row_pos = b.take<int32_t>(p.row_pos.size());
    a.ntouch_lp = (int64_t)A.touch_lp.size();
    a.vid = b.take<int32_t>(p.vid.size());
    a.gx = b.take<double>(p.gx.size());
    a.gw = b.take<double>(p.gw.size());
    a.gpos = b.take<double>((size_t)S.nelem * p.P.qg * p.P.qg * 3);
    a.gkap = S.form == 0 ? b.take<double>((size_t)S.nelem * p.P.qg * p.P.qg) : nullptr;
    a.psi = b.take<double>(p.psi.size());
    a.psiw = b.take<double>(p.psiw.size());
    a.sx = b.take<double>(p.sx.size());
    a.sw = b.take<double>(p.sw.size());
    a.cheb = b.take<double>(p.cheb.size());
    a.own_t = b.take<int32_t>(p.own_t.size());
    a.xc = b.take<double>((size_t)p.ncl * p.q2 * 3);
    a.lb = b.take<char>((size_t)p.near_t.size() * p.nloc * p.nloc * p.nloc * p.nloc * A.scal);
    const size_t nb2 = (size_t)(S.d + 1) * (S.d + 1) * (S.d + 1) * (S.d + 1);
    a.sblk = b.take<char>(p.touch.size() / 5 * nb2 * A.scal);
    if (d) *d = a;
    return b.off + 256;
}

static bool make_basis_tab(const SpaceDesc& S, BasisTab& bt) {
    std::vector<double> poly;
    bspline_local_polys(S.d, S.r, S.L, poly);
    const int d1 = S.d + 1;
    std::memset(&bt, 0, sizeof(bt));
    bt.d = S.d;
    bt.nel = S.nel;
    bt.w = d1;
    bt.ncls = S.nel <= 2 * bt.w + 1 ? S.nel : 2 * bt.w + 1;
    auto coef = [&](int i, int l, int k) { return poly[((size_t)i * d1 + l) * d1 + k]; };
    std::vector<int> rep(bt.ncls, -1);
    for (int i = 0; i < S.nel; ++i) {
        const int c = basis_class(bt, i);
        if (rep[c] < 0) {
            rep[c] = i;
            for (int l = 0; l < d1; ++l)
                for (int k = 0; k < d1; ++k) bt.c[c][l][k] = coef(i, l, k);
        } else {
            for (int l = 0; l < d1; ++l)
                for (int k = 0; k < d1; ++k)
                    if (std::fabs(bt.c[c][l][k] - coef(i, l, k)) > 1e-12 * (1.0 + std::fabs(coef(i, l, k))))
                        return false;
        }
    }
    return true;
}

static Gauss8 gauss8() {
    std::vector<double> x, w;
    gauss_legendre01(8, x, w);
    Gauss8 g;
    for (int i = 0; i < 8; ++i) {
        g.x[i] = x[i];
        g.w[i] = w[i];
    }
    return g;
}

// ------------------------------------------------------------------------------ GMRES
struct SolveWs {
    char* V;       // (m+1) x N Krylov basis
    char* w;       // N
    char* r;       // N  (refinement: FP64 residual)
    char* d;       // N  (refinement: correction)
    char* z;       // N  (preconditioned vector)
    char* partA;   // kSolveBlocks x (m+1) partial sums
    char* partB;
    double* npart; // kSolveBlocks partial squared norms
    // refinement: the flexible outer loop's directions D_j and their images U_j = A D_j
    // (orthonormal), hist vectors each, with their own partial sums and coefficients
    int hist = 0;
    char* U;
    char* D;
    char* gpA;
    char* gpB;
    char* gh1;
    char* gh2;
    GmresState st;
};

// directions kept by the flexible outer loop of a refined solve (restarted beyond that)
constexpr int kRefineHist = 16;

// Inner tolerance of a refined solve: the caller's, else 1e-4 with an FP32 far field and
// 1e-2 with BF16 (its moments are rounded to BF16 in every apply, which leaves the inner
// operator's residual near 1e-3 of the right-hand side, so a tighter inner tolerance is
// never met).
static double refine_inner_tol(const bem_operator_s* A, const bem_solve_params* p) {
    if (p->inner_tol > 0.0) return p->inner_tol;
    return A->far_low == BEM_PREC_BF16 ? 1e-2 : 1e-4;
}

static int refine_hist(const bem_solve_params* p) {
    const int mo = p->max_outer > 0 ? p->max_outer : 20;
    return p->refine ? std::min(mo, kRefineHist) : 0;
}

static size_t solve_layout(int64_t N, int m, size_t sc, void* base, SolveWs* ws, int hist = 0) {
    Bump b(base);
    SolveWs w{};
    w.V = b.take<char>((size_t)(m + 1) * N * sc);
    w.w = b.take<char>((size_t)N * sc);
    w.r = b.take<char>((size_t)N * sc);
    w.d = b.take<char>((size_t)N * sc);
    w.z = b.take<char>((size_t)N * sc);
    w.partA = b.take<char>((size_t)kSolveBlocks * (m + 1) * sc);
    w.partB = b.take<char>((size_t)kSolveBlocks * (m + 1) * sc);
    w.npart = b.take<double>(kSolveBlocks);
    w.st.m = m;
    w.st.H = b.take<char>((size_t)(m + 1) * m * sc);
    w.st.cs = b.take<double>(m);
    w.st.sn = b.take<char>((size_t)m * sc);
    w.st.g = b.take<char>((size_t)(m + 1) * sc);
    w.st.y = b.take<char>((size_t)m * sc);
    w.st.h1 = b.take<char>((size_t)(m + 1) * sc);
    w.st.h2 = b.take<char>((size_t)(m + 1) * sc);
    w.st.scal = b.take<double>(m + 2);
    w.hist = hist;
    if (hist > 0) {
        w.U = b.take<char>((size_t)hist * N * sc);
        w.D = b.take<char>((size_t)hist * N * sc);
        w.gpA = b.take<char>((size_t)kSolveBlocks * hist * sc);
        w.gpB = b.take<char>((size_t)kSolveBlocks * hist * sc);
        w.gh1 = b.take<char>((size_t)hist * sc);
        w.gh2 = b.take<char>((size_t)hist * sc);
    }
    if (ws) *ws = w;
    return b.off + 256;
}

// y = A x for one column of global functions: on an S^0 space the column is spread to the
// local functions, multiplied, and the local products of each global function summed.
static hipError_t op_apply(const bem_operator_s* A, int prec, const void* x, void* y, hipStream_t stream) {
    if (A->mxh) return launch_mxh_apply(A->mxhd, x, y, stream);
    if (A->mx) return launch_mx_matvec(A->mxd, x, y, stream);
    const SpaceDesc& S = A->dev.S;
    if (S.form != 0) return launch_apply(A->dev, x, y, prec, stream);
    const int cp = A->cplx ? 1 : 0;
    hipError_t e = launch_glue_gather(S, cp, x, A->dev.xl, stream);
    if (e != hipSuccess) return e;
    e = launch_apply(A->dev, A->dev.xl, A->dev.yl, prec, stream);
    if (e != hipSuccess) return e;
    return launch_glue_scatter(S, cp, A->dev.yl, y, stream);
}

// One right-hand side.  The Givens step of Arnoldi step j runs inside step j+1's
// dot-product kernel and writes its residual estimate straight to coherent host memory,
// with a stamp (no copy, no event in the stream); having enqueued step j the host waits
// only for the estimate of step j-2, so the device always has more than a step queued.
// Convergence is therefore seen up to two steps late; those steps' columns are dropped,
// so the iterate is that of the step that converged.  The true residual is read once per
// cycle.
static int gmres_one(bem_operator A, int prec, const void* b, void* x, int m, int maxit, double tol,
                     bem_solve_stats* out, SolveWs& W, hipStream_t stream, bool pc = false) {
    const int64_t N = A->info.ndof;
    const int cp = A->cplx ? 1 : 0;
    const size_t sc = A->scal;
    auto Vj = [&](int j) { return W.V + (size_t)j * N * sc; };
    if (!A->pinned) HIP_CHECK(hipHostMalloc((void**)&A->pinned, sizeof(double) * (kMaxRestart + 2 + kSolveBlocks)));
    if (!A->hstat) {
        HIP_CHECK(hipHostMalloc((void**)&A->hstat, (sizeof(double) + sizeof(unsigned)) * kMaxRestart,
                                hipHostMallocMapped | hipHostMallocCoherent));
        std::memset(A->hstat, 0, (sizeof(double) + sizeof(unsigned)) * kMaxRestart);
        A->stamp = 0;
    }
    {
        void* dp = nullptr;
        HIP_CHECK(hipHostGetDevicePointer(&dp, A->hstat, 0));
        W.st.hest = (double*)dp;
        W.st.hseq = (unsigned*)((double*)dp + kMaxRestart);
    }
    const volatile double* hest = A->hstat;
    const volatile unsigned* hseq = (const volatile unsigned*)(A->hstat + kMaxRestart);
    // residual estimate of step jj of the current cycle: spin on its stamp; should it not
    // arrive within seconds (not expected), wait for the stream and copy the device value
    auto estimate = [&](int jj, double& e) -> int {
        const auto t0 = std::chrono::steady_clock::now();
        for (unsigned spin = 1; hseq[jj] != W.st.stamp; ++spin) {
            if ((spin & 4095u) == 0 && std::chrono::steady_clock::now() - t0 > std::chrono::seconds(5)) {
                HIP_CHECK(hipStreamSynchronize(stream));
                HIP_CHECK(hipMemcpy(&e, W.st.scal + 2 + jj, sizeof(double), hipMemcpyDeviceToHost));
                return BEM_OK;
            }
        }
        std::atomic_thread_fence(std::memory_order_acquire);
        e = hest[jj];
        return BEM_OK;
    };
    double* pin = A->pinned;
    out->iterations = 0;
    out->converged = 0;
    out->relres = 0.0;
    HIP_CHECK(hipMemsetAsync(x, 0, N * sc, stream));
    // ||b||: squared-norm partials of b, summed on the host in the device's order
    HIP_CHECK(solve_residual(cp, N, b, W.w, W.npart, 1, stream));
    HIP_CHECK(hipMemcpyAsync(pin + kMaxRestart + 2, W.npart, sizeof(double) * kSolveBlocks, hipMemcpyDeviceToHost,
                             stream));
    HIP_CHECK(hipStreamSynchronize(stream));
    double bb = 0.0;
    for (int i = 0; i < kSolveBlocks; ++i) bb += pin[kMaxRestart + 2 + i];
    const double bnorm = std::sqrt(bb);
    if (bnorm == 0.0) {
        out->converged = 1;
        return BEM_OK;
    }
    int total = 0;
    double relres = 1.0;
    for (int cycle = 0;; ++cycle) {
        W.st.stamp = ++A->stamp;
        if (cycle > 0) {
            HIP_CHECK(op_apply(A, prec, x, W.w, stream));
            HIP_CHECK(solve_residual(cp, N, b, W.w, W.npart, 0, stream));
        }  // in the first cycle x = 0 and w already holds b
        HIP_CHECK(solve_start(cp, N, W.npart, W.w, Vj(0), W.st, stream));
        HIP_CHECK(hipMemcpyAsync(pin, W.st.scal + 1, sizeof(double), hipMemcpyDeviceToHost, stream));
        HIP_CHECK(hipStreamSynchronize(stream));
        relres = pin[0] / bnorm;
        if (relres <= tol || total >= maxit || !std::isfinite(relres)) break;
        int k = 0;
        bool done = false;  // convergence seen: the Givens steps of columns 0..k-1 have run
        for (int j = 0; j < m && total + j < maxit; ++j) {
            if (pc) {
                HIP_CHECK(launch_prec_apply(A->dev, A->pdev, 1, Vj(j), W.z, stream));
                HIP_CHECK(op_apply(A, prec, W.z, W.w, stream));
            } else {
                HIP_CHECK(op_apply(A, prec, Vj(j), W.w, stream));
            }
            // the dot products of step j and the Givens step of step j-1
            HIP_CHECK(solve_dots(cp, N, j + 1, W.V, W.w, W.partA, j - 1, W.npart, W.st, stream));
            HIP_CHECK(solve_update(cp, N, j + 1, W.V, W.partA, W.st.h1, W.w, W.partB, W.npart, 0, stream));
            HIP_CHECK(solve_update(cp, N, j + 1, W.V, W.partB, W.st.h2, W.w, W.partA, W.npart, 1, stream));
            HIP_CHECK(solve_scale(cp, N, W.npart, W.w, Vj(j + 1), stream));
            k = j + 1;
            if (j >= 2) {
                double e;
                const int rc = estimate(j - 2, e);
                if (rc != BEM_OK) return rc;
                if (e <= tol * bnorm || !std::isfinite(e)) {
                    k = j - 1;  // converged after step j-2; the columns of steps j-1 and j are not used
                    done = true;
                    break;
                }
            }
        }
        // the last step's Givens step, and the convergence check of the steps not yet read
        if (k > 0 && !done) {
            HIP_CHECK(solve_givens(cp, k - 1, W.npart, W.st, stream));
            for (int j = k >= 2 ? k - 2 : 0; j < k; ++j) {
                double e;
                const int rc = estimate(j, e);
                if (rc != BEM_OK) return rc;
                if (e <= tol * bnorm || !std::isfinite(e)) {
                    k = j + 1;
                    break;
                }
            }
        }
        total += k;
        if (pc) {
            // x += M^{-1} (V y)
            if (k > 0) {
                HIP_CHECK(bsolve_zero(cp, N, W.z, stream));
                HIP_CHECK(solve_backsolve_update(cp, N, k, W.V, W.z, W.st, stream));
                HIP_CHECK(launch_prec_apply(A->dev, A->pdev, 1, W.z, W.w, stream));
                HIP_CHECK(solve_axpy(cp, N, 1.0, W.w, x, stream));
            }
        } else {
            HIP_CHECK(solve_backsolve_update(cp, N, k, W.V, x, W.st, stream));
        }
    }
    out->iterations = total;
    out->relres = relres;
    out->converged = relres <= tol ? 1 : 0;
    out->outer = 0;
    return BEM_OK;
}

// FP64 refinement around GMRES on the operator with the low-precision far field, as a
// flexible outer Krylov loop (generalised conjugate residuals): each outer step solves
// A_low d = r to inner_tol, forms u = A d with the FP64 operator, orthonormalises u against
// the previous images (classical Gram-Schmidt, two passes, the same combination applied to
// d), and moves x along d by the coefficient that minimises the FP64 residual over all
// kept directions; the residual is then recomputed as b - A x in FP64.  Plain refinement
// (x += d) is the first step of this; the later steps also converge when the low-precision
// operator's error times the condition number is near 1.
static int refine_one(bem_operator A, const void* b, void* x, const bem_solve_params* p, bem_solve_stats* out,
                      SolveWs& W, hipStream_t stream) {
    const int64_t N = A->info.ndof;
    const int cp = A->cplx ? 1 : 0;
    const size_t sc = A->scal;
    const int max_outer = p->max_outer > 0 ? p->max_outer : 20;
    const double inner_tol = refine_inner_tol(A, p);
    const int inner_cap = p->inner_maxit > 0 ? p->inner_maxit : 3 * p->restart;
    if (W.hist < 1) return fail(BEM_EINVAL, "refinement workspace missing");
    auto Uj = [&](int j) { return W.U + (size_t)j * N * sc; };
    auto Dj = [&](int j) { return W.D + (size_t)j * N * sc; };
    double* pin = A->pinned;
    HIP_CHECK(hipMemsetAsync(x, 0, N * sc, stream));
    HIP_CHECK(hipMemcpyAsync(W.r, b, N * sc, hipMemcpyDeviceToDevice, stream));
    HIP_CHECK(solve_residual(cp, N, b, W.w, W.npart, 1, stream));
    auto host_norm = [&](double& v) -> int {
        HIP_CHECK(hipMemcpyAsync(pin + kMaxRestart + 2, W.npart, sizeof(double) * kSolveBlocks,
                                 hipMemcpyDeviceToHost, stream));
        HIP_CHECK(hipStreamSynchronize(stream));
        double s2 = 0.0;
        for (int i = 0; i < kSolveBlocks; ++i) s2 += pin[kMaxRestart + 2 + i];
        v = std::sqrt(s2);
        return BEM_OK;
    };
    double bnorm = 0.0, rnorm = 0.0;
    if (host_norm(bnorm) != BEM_OK) return BEM_EDEVICE;
    rnorm = bnorm;
    int total = 0, outer = 0, k = 0;
    while (bnorm > 0.0 && rnorm > p->tol * bnorm && outer < max_outer && total < p->maxit && std::isfinite(rnorm)) {
        bem_solve_stats in{};
        const int rc = gmres_one(A, A->far_low, W.r, W.d, p->restart, std::min(p->maxit - total, inner_cap),
                                 inner_tol, &in, W, stream, p->precond != 0);
        if (rc != BEM_OK) return rc;
        total += in.iterations;
        ++outer;
        if (in.iterations == 0) break;  // no progress possible
        if (k == W.hist) k = 0;         // history full: restart the outer loop from x
        // u = A d (FP64), orthonormalised against U_0..U_{k-1}; d follows the same combination
        HIP_CHECK(op_apply(A, 0, W.d, W.w, stream));
        if (k > 0) {
            HIP_CHECK(solve_dots(cp, N, k, W.U, W.w, W.gpA, -1, W.npart, W.st, stream));
            HIP_CHECK(solve_update(cp, N, k, W.U, W.gpA, W.gh1, W.w, W.gpB, W.npart, 0, stream));
            HIP_CHECK(solve_combine(cp, N, k, W.D, W.gh1, -1.0, W.d, stream));
            HIP_CHECK(solve_update(cp, N, k, W.U, W.gpB, W.gh2, W.w, W.gpA, W.npart, 1, stream));
            HIP_CHECK(solve_combine(cp, N, k, W.D, W.gh2, -1.0, W.d, stream));
        } else {
            HIP_CHECK(solve_update(cp, N, 0, W.U, W.gpA, W.gh1, W.w, W.gpB, W.npart, 1, stream));  // ||u|| only
        }
        HIP_CHECK(solve_scale(cp, N, W.npart, W.w, Uj(k), stream));
        HIP_CHECK(solve_scale(cp, N, W.npart, W.d, Dj(k), stream));
        // alpha = U_k^H r; x += alpha D_k
        HIP_CHECK(solve_dots(cp, N, 1, Uj(k), W.r, W.gpA, -1, W.npart, W.st, stream));
        HIP_CHECK(solve_update(cp, N, 1, Uj(k), W.gpA, W.gh1, W.r, W.gpB, W.npart, 1, stream));
        HIP_CHECK(solve_combine(cp, N, 1, Dj(k), W.gh1, 1.0, x, stream));
        ++k;
        // the FP64 residual of the new iterate
        HIP_CHECK(op_apply(A, 0, x, W.w, stream));
        HIP_CHECK(solve_residual(cp, N, b, W.w, W.npart, 0, stream));
        HIP_CHECK(hipMemcpyAsync(W.r, W.w, N * sc, hipMemcpyDeviceToDevice, stream));
        if (host_norm(rnorm) != BEM_OK) return BEM_EDEVICE;
    }
    out->iterations = total;
    out->outer = outer;
    out->relres = bnorm > 0.0 ? rnorm / bnorm : 0.0;
    out->converged = out->relres <= p->tol ? 1 : 0;
    return BEM_OK;
}

// ------------------------------------------------------------------ GMRES, many RHS
struct BSolveWs {
    char* V;        // (m+1) slabs [N][R]
    char* w;        // slab
    char* r;        // slab (refinement: FP64 residual)
    char* d;        // slab (refinement: correction)
    char* bs;       // slab of the right-hand sides
    char* xs;       // slab of the solutions
    char* z;        // slab (preconditioned vectors)
    char* part;     // [slices][m+1][R] partial inner products
    char* h1;       // [m+1][R]
    char* h2;       // [m+1][R]
    double* npart;  // [slices][R]
    int* flag;      // [R]
    // refinement: directions D_j and orthonormal images U_j = A D_j (hist slabs each),
    // partial sums [slices][hist][R] and coefficients [hist][R]
    int hist = 0;
    char* U;
    char* D;
    char* gpart;
    char* gh1;
    char* gh2;
    BGmresState st;
};

static size_t bsolve_layout(int64_t N, int m, int R, size_t sc, void* base, BSolveWs* ws, int hist = 0) {
    Bump b(base);
    BSolveWs w{};
    const size_t slab = (size_t)N * R * sc;
    w.V = b.take<char>((size_t)(m + 1) * slab);
    w.w = b.take<char>(slab);
    w.r = b.take<char>(slab);
    w.d = b.take<char>(slab);
    w.bs = b.take<char>(slab);
    w.xs = b.take<char>(slab);
    w.z = b.take<char>(slab);
    w.part = b.take<char>((size_t)kBSolveSlices * (m + 1) * R * sc);
    w.h1 = b.take<char>((size_t)(m + 1) * R * sc);
    w.h2 = b.take<char>((size_t)(m + 1) * R * sc);
    w.npart = b.take<double>((size_t)kBSolveSlices * R);
    w.flag = b.take<int>(R);
    w.st.m = m;
    w.st.H = b.take<char>((size_t)R * (m + 1) * m * sc);
    w.st.cs = b.take<double>((size_t)R * m);
    w.st.sn = b.take<char>((size_t)R * m * sc);
    w.st.g = b.take<char>((size_t)R * (m + 1) * sc);
    w.st.y = b.take<char>((size_t)m * R * sc);
    w.st.est = b.take<double>((size_t)m * R);
    w.st.beta = b.take<double>(R);
    w.st.sc = b.take<double>(R);
    w.st.kr = b.take<int>(R);
    w.hist = hist;
    if (hist > 0) {
        w.U = b.take<char>((size_t)hist * slab);
        w.D = b.take<char>((size_t)hist * slab);
        w.gpart = b.take<char>((size_t)kBSolveSlices * hist * R * sc);
        w.gh1 = b.take<char>((size_t)hist * R * sc);
        w.gh2 = b.take<char>((size_t)hist * R * sc);
    }
    if (ws) *ws = w;
    return b.off + 256;
}

// y = A x on slabs of R columns (R <= batch_rhs)
static int bapply(bem_operator A, int prec, const void* xs, void* ys, int R, hipStream_t stream) {
    BatchDev bd = A->bdev;
    bd.R = R;
    bd.xs = (void*)xs;
    bd.ys = ys;
    HIP_CHECK(launch_apply_batched(A->dev, bd, nullptr, 0, nullptr, 0, prec, stream));
    return BEM_OK;
}

static int ensure_bpin(bem_operator A, int R) {
    const size_t need = (size_t)(kMaxRestart + 4) * R;
    if (A->bpin && A->bpin_doubles >= need) return BEM_OK;
    if (A->bpin) HIP_CHECK(hipHostFree(A->bpin));
    A->bpin = nullptr;
    HIP_CHECK(hipHostMalloc((void**)&A->bpin, sizeof(double) * need));
    A->bpin_doubles = need;
    while ((int)A->sev.size() < kMaxRestart) {
        hipEvent_t e;
        HIP_CHECK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
        A->sev.push_back(e);
    }
    return BEM_OK;
}

// R right-hand sides in lockstep (slabs b, x).  Each right-hand side stops on its own:
// a cycle's Arnoldi steps go on while some active one has not reached tol on its rotated
// residual estimate (checked one step late, as in the one-column solver), and each one
// updates its iterate with the steps it needed.  Convergence is decided on the true
// residual at the start of the next cycle.
static int gmres_batched(bem_operator A, int prec, const void* b, void* x, int R, int m, int maxit, double tol,
                         bem_solve_stats* out, BSolveWs& W, hipStream_t stream, bool pc = false) {
    const int64_t N = A->info.ndof;
    const int cp = A->cplx ? 1 : 0;
    const size_t sc = A->scal;
    auto Vj = [&](int j) { return W.V + (size_t)j * N * R * sc; };
    if (ensure_bpin(A, R) != BEM_OK) return BEM_EDEVICE;
    double* est_h = A->bpin;                       // [kMaxRestart][R]
    double* beta_h = est_h + (size_t)kMaxRestart * R;  // [R]
    int* kr_h = (int*)(beta_h + R);               // [R]
    auto read_beta = [&]() -> int {
        HIP_CHECK(hipMemcpyAsync(beta_h, W.st.beta, sizeof(double) * R, hipMemcpyDeviceToHost, stream));
        HIP_CHECK(hipStreamSynchronize(stream));
        return BEM_OK;
    };
    HIP_CHECK(bsolve_zero(cp, N * R, x, stream));
    HIP_CHECK(bsolve_residual(cp, N, R, b, W.w, W.npart, 1, stream));
    HIP_CHECK(bsolve_start(cp, N, R, W.npart, W.w, Vj(0), W.st, stream));
    if (read_beta() != BEM_OK) return BEM_EDEVICE;
    std::vector<double> bnorm(beta_h, beta_h + R), rel(R, 0.0);
    std::vector<int> total(R, 0);
    std::vector<char> conv(R, 0), act(R, 0);
    for (int cycle = 0;; ++cycle) {
        if (cycle > 0) {
            if (bapply(A, prec, x, W.w, R, stream) != BEM_OK) return BEM_EDEVICE;
            HIP_CHECK(bsolve_residual(cp, N, R, b, W.w, W.npart, 0, stream));
            HIP_CHECK(bsolve_start(cp, N, R, W.npart, W.w, Vj(0), W.st, stream));
            if (read_beta() != BEM_OK) return BEM_EDEVICE;
        }
        bool any = false;
        int room = 0;
        for (int r = 0; r < R; ++r) {
            rel[r] = bnorm[r] > 0.0 ? beta_h[r] / bnorm[r] : 0.0;
            conv[r] = rel[r] <= tol;
            act[r] = !conv[r] && total[r] < maxit && std::isfinite(rel[r]);
            if (act[r]) {
                any = true;
                room = std::max(room, maxit - total[r]);
            }
        }
        if (!any) break;
        int k = 0;
        for (int j = 0; j < m && j < room; ++j) {
            if (pc) {
                HIP_CHECK(launch_prec_apply(A->dev, A->pdev, R, Vj(j), W.z, stream));
                if (bapply(A, prec, W.z, W.w, R, stream) != BEM_OK) return BEM_EDEVICE;
            } else if (bapply(A, prec, Vj(j), W.w, R, stream) != BEM_OK) {
                return BEM_EDEVICE;
            }
            HIP_CHECK(bsolve_dots(cp, N, R, j + 1, W.V, W.w, W.part, W.h1, stream));
            HIP_CHECK(bsolve_update(cp, N, R, j + 1, W.V, W.h1, W.w, W.npart, 0, stream));
            HIP_CHECK(bsolve_dots(cp, N, R, j + 1, W.V, W.w, W.part, W.h2, stream));
            HIP_CHECK(bsolve_update(cp, N, R, j + 1, W.V, W.h2, W.w, W.npart, 1, stream));
            HIP_CHECK(bsolve_givens_scale(cp, N, R, j, W.npart, W.h1, W.h2, W.w, Vj(j + 1), W.st, stream));
            HIP_CHECK(hipMemcpyAsync(est_h + (size_t)j * R, W.st.est + (size_t)j * R, sizeof(double) * R,
                                     hipMemcpyDeviceToHost, stream));
            HIP_CHECK(hipEventRecord(A->sev[j], stream));
            k = j + 1;
            if (j >= 1) {
                HIP_CHECK(hipEventSynchronize(A->sev[j - 1]));
                bool all = true;
                for (int r = 0; r < R && all; ++r) {
                    const double e = est_h[(size_t)(j - 1) * R + r];
                    if (act[r] && e > tol * bnorm[r] && std::isfinite(e)) all = false;
                }
                if (all) {
                    k = j;  // every active one converged after step j-1
                    break;
                }
            }
        }
        if (k > 0) HIP_CHECK(hipEventSynchronize(A->sev[k - 1]));
        for (int r = 0; r < R; ++r) {
            int kr = 0;
            if (act[r]) {
                kr = std::min(k, maxit - total[r]);
                for (int s2 = 0; s2 < kr; ++s2)
                    if (!(est_h[(size_t)s2 * R + r] > tol * bnorm[r])) {
                        kr = s2 + 1;
                        break;
                    }
            }
            kr_h[r] = kr;
            total[r] += kr;
        }
        HIP_CHECK(hipMemcpyAsync(W.st.kr, kr_h, sizeof(int) * R, hipMemcpyHostToDevice, stream));
        if (pc) {
            if (k > 0) {
                HIP_CHECK(bsolve_zero(cp, N * R, W.z, stream));
                HIP_CHECK(bsolve_backsolve_update(cp, N, R, k, W.V, W.z, W.st, stream));
                HIP_CHECK(launch_prec_apply(A->dev, A->pdev, R, W.z, W.w, stream));
                HIP_CHECK(bsolve_axpy(cp, N, R, W.w, x, stream));
            }
        } else {
            HIP_CHECK(bsolve_backsolve_update(cp, N, R, k, W.V, x, W.st, stream));
        }
    }
    for (int r = 0; r < R; ++r) {
        out[r].iterations = total[r];
        out[r].relres = rel[r];
        out[r].converged = conv[r] ? 1 : 0;
        out[r].outer = 0;
    }
    return BEM_OK;
}

// FP64 refinement around the lockstep GMRES on the low-precision operator, with the same
// flexible outer loop as the one-column solver, per right-hand side (each keeps its own
// coefficients; right-hand sides that have met tol are masked out of further inner solves,
// their new directions are zero and leave them unchanged).
static int refine_batched(bem_operator A, const void* b, void* x, int R, const bem_solve_params* p,
                          bem_solve_stats* out, BSolveWs& W, hipStream_t stream) {
    const int64_t N = A->info.ndof;
    const int cp = A->cplx ? 1 : 0;
    const size_t slab = (size_t)N * R * A->scal;
    const int max_outer = p->max_outer > 0 ? p->max_outer : 20;
    const double inner_tol = refine_inner_tol(A, p);
    const int inner_cap = p->inner_maxit > 0 ? p->inner_maxit : 3 * p->restart;
    if (W.hist < 1) return fail(BEM_EINVAL, "refinement workspace missing");
    auto Uj = [&](int j) { return W.U + (size_t)j * slab; };
    auto Dj = [&](int j) { return W.D + (size_t)j * slab; };
    if (ensure_bpin(A, R) != BEM_OK) return BEM_EDEVICE;
    double* beta_h = A->bpin + (size_t)kMaxRestart * R;
    int* flag_h = (int*)(beta_h + R);
    auto norms = [&](std::vector<double>& v) -> int {
        // norms of the slab in W.r (partials in W.npart) via the start kernel's reduction
        HIP_CHECK(bsolve_start(cp, N, R, W.npart, W.r, W.V, W.st, stream));
        HIP_CHECK(hipMemcpyAsync(beta_h, W.st.beta, sizeof(double) * R, hipMemcpyDeviceToHost, stream));
        HIP_CHECK(hipStreamSynchronize(stream));
        v.assign(beta_h, beta_h + R);
        return BEM_OK;
    };
    HIP_CHECK(bsolve_zero(cp, N * R, x, stream));
    HIP_CHECK(bsolve_residual(cp, N, R, b, W.r, W.npart, 1, stream));
    std::vector<double> bnorm, rnorm;
    if (norms(bnorm) != BEM_OK) return BEM_EDEVICE;
    rnorm = bnorm;
    std::vector<int> total(R, 0), outer(R, 0), done(R, 0);
    std::vector<bem_solve_stats> in(R);
    int k = 0;
    for (int it = 0; it < max_outer; ++it) {
        bool any = false;
        for (int r = 0; r < R; ++r) {
            done[r] = bnorm[r] == 0.0 || rnorm[r] <= p->tol * bnorm[r] || total[r] >= p->maxit ||
                      !std::isfinite(rnorm[r]);
            flag_h[r] = done[r];
            any = any || !done[r];
        }
        if (!any) break;
        // (the pinned flags are read by the copy before the inner solve reuses that memory:
        // the inner solve synchronises the stream before its first host write)
        HIP_CHECK(hipMemcpyAsync(W.flag, flag_h, sizeof(int) * R, hipMemcpyHostToDevice, stream));
        HIP_CHECK(bsolve_mask(cp, N, R, W.flag, W.r, stream));
        // every inner solve stays within the budget of each right-hand side still iterating
        int left = std::min(p->maxit, inner_cap);
        for (int r = 0; r < R; ++r)
            if (!done[r]) left = std::min(left, p->maxit - total[r]);
        const int rc = gmres_batched(A, A->far_low, W.r, W.d, R, p->restart, left, inner_tol, in.data(), W, stream,
                                     p->precond != 0);
        if (rc != BEM_OK) return rc;
        int progress = 0;
        for (int r = 0; r < R; ++r)
            if (!done[r]) {
                total[r] += in[r].iterations;
                outer[r] += 1;
                progress += in[r].iterations;
            }
        if (progress == 0) break;
        if (k == W.hist) k = 0;  // history full: restart the outer loop from x
        // u = A d (FP64) orthonormalised per column against U_0..U_{k-1}; d alike
        if (bapply(A, 0, W.d, W.w, R, stream) != BEM_OK) return BEM_EDEVICE;
        if (k > 0) {
            HIP_CHECK(bsolve_dots(cp, N, R, k, W.U, W.w, W.gpart, W.gh1, stream));
            HIP_CHECK(bsolve_update(cp, N, R, k, W.D, W.gh1, W.d, W.npart, 0, stream));
            HIP_CHECK(bsolve_update(cp, N, R, k, W.U, W.gh1, W.w, W.npart, 0, stream));
            HIP_CHECK(bsolve_dots(cp, N, R, k, W.U, W.w, W.gpart, W.gh2, stream));
            HIP_CHECK(bsolve_update(cp, N, R, k, W.D, W.gh2, W.d, W.npart, 0, stream));
        }
        HIP_CHECK(bsolve_update(cp, N, R, k, W.U, W.gh2, W.w, W.npart, 1, stream));  // k = 0: ||u|| only
        HIP_CHECK(bsolve_scale2(cp, N, R, W.npart, W.w, W.d, Uj(k), Dj(k), stream));
        // alpha_r = U_k[:, r]^H r_r; x += alpha D_k
        HIP_CHECK(bsolve_dots(cp, N, R, 1, Uj(k), W.r, W.gpart, W.gh1, stream));
        HIP_CHECK(bsolve_xupdate(cp, N, R, 1, Dj(k), W.gh1, x, stream));
        ++k;
        // the FP64 residual of the new iterates
        if (bapply(A, 0, x, W.r, R, stream) != BEM_OK) return BEM_EDEVICE;
        HIP_CHECK(bsolve_residual(cp, N, R, b, W.r, W.npart, 0, stream));
        if (norms(rnorm) != BEM_OK) return BEM_EDEVICE;
    }
    for (int r = 0; r < R; ++r) {
        out[r].iterations = total[r];
        out[r].outer = outer[r];
        out[r].relres = bnorm[r] > 0.0 ? rnorm[r] / bnorm[r] : 0.0;
        out[r].converged = out[r].relres <= p->tol ? 1 : 0;
    }
    return BEM_OK;
}

extern "C" {

const char* bem_last_error(void) { return g_err.c_str(); }

int bem_geometry_analytic(int kind, const double* params, int nparams, bem_geometry* out) {
    if (!out) return fail(BEM_EINVAL, "out is NULL");
    GeomDesc g{};
    g.kind = kind;
    g.a = g.b = g.c = 1.0;
    switch (kind) {
        case GEOM_SPHERE6:
            g.npatch = 6;
            break;
        case GEOM_ELLIPSOID6:
            if (nparams < 3 || !params) return fail(BEM_EINVAL, "ellipsoid needs 3 semi-axes");
            if (!(params[0] > 0 && params[1] > 0 && params[2] > 0)) return fail(BEM_EINVAL, "semi-axes must be > 0");
            g.npatch = 6;
            g.a = params[0];
            g.b = params[1];
            g.c = params[2];
            break;
        case GEOM_TORUS16:
            if (nparams < 2 || !params) return fail(BEM_EINVAL, "torus needs R and r");
            if (!(params[1] > 0 && params[0] > params[1])) return fail(BEM_EINVAL, "torus needs R > r > 0");
            g.npatch = 16;
            g.a = params[0];
            g.b = params[1];
            break;
        case GEOM_FLAT1:
            if (nparams < 1 || !params || !(params[0] > 0)) return fail(BEM_EINVAL, "flat square needs a side > 0");
            g.npatch = 1;
            g.a = params[0];
            break;
        default:
            return fail(BEM_EINVAL, "unknown geometry kind");
    }
    bem_geometry_s* G = new (std::nothrow) bem_geometry_s;
    if (!G) return fail(BEM_ENOMEM, "host allocation failed");
    G->g = g;
    *out = G;
    return BEM_OK;
}

void bem_geometry_destroy(bem_geometry g) { delete g; }

}  // extern "C"

// Kernels evaluate NURBS maps from the device copy of the tables.
static int need_device_geometry(const SpaceDesc& S) {
    if (S.geom.kind == GEOM_NURBS && !S.geom.tab_dev)
        return fail(BEM_EDEVICE, "NURBS geometry created without a GPU: no device copy of its tables");
    if (S.form == 0 && !S.glue)
        return fail(BEM_EDEVICE, "S^0 space created without a GPU: no device copy of its gluing");
    return BEM_OK;
}

// S^0 gluing (App. E: continuity across patch boundaries): every local B-spline is anchored
// at the image of its Greville point; with clamped knots the functions that do not vanish
// on a patch boundary have their anchors on it, and by the matching condition the functions
// of neighbouring patches that coincide on a shared edge or vertex share their anchor.
// Boundary anchors are sorted by their first coordinate; anchors that agree in all three
// coordinates within 1e-10 of the largest coordinate are one global function (first local
// occurrence numbers it).
static bool build_glue(const SpaceDesc& S, GlueTab& T, int64_t& nglob) {
    const int nb = S.nb, d = S.d;
    std::vector<double> knots;
    for (int i = 0; i <= d; ++i) knots.push_back(0.0);
    for (int k = 1; k < S.nel; ++k)
        for (int m = 0; m < S.r; ++m) knots.push_back((double)k / S.nel);
    for (int i = 0; i <= d; ++i) knots.push_back(1.0);
    std::vector<double> gr(nb);
    for (int j = 0; j < nb; ++j) {
        double a = 0.0;
        for (int k = 1; k <= d; ++k) a += knots[j + k];
        gr[j] = a / d;
    }
    struct Anchor {
        double x[3];
        int64_t g;
    };
    std::vector<Anchor> an;
    double scale = 0.0;
    for (int f = 0; f < S.geom.npatch; ++f)
        for (int j1 = 0; j1 < nb; ++j1)
            for (int j2 = 0; j2 < nb; ++j2) {
                if (j1 != 0 && j1 != nb - 1 && j2 != 0 && j2 != nb - 1) continue;
                Anchor a;
                patch_point(S.geom, f, gr[j1], gr[j2], a.x);
                a.g = dof_id(S, f, j1, j2);
                for (double v : a.x) scale = std::max(scale, std::fabs(v));
                an.push_back(a);
            }
    const double tol = 1e-10 * std::max(scale, 1e-300);
    std::sort(an.begin(), an.end(), [](const Anchor& u, const Anchor& v) { return u.x[0] < v.x[0]; });
    std::vector<int64_t> parent(S.ndof);
    for (int64_t g = 0; g < S.ndof; ++g) parent[g] = g;
    auto root = [&](int64_t g) {
        while (parent[g] != g) g = parent[g] = parent[parent[g]];
        return g;
    };
    for (size_t a = 0; a < an.size(); ++a)
        for (size_t b = a + 1; b < an.size() && an[b].x[0] - an[a].x[0] <= tol; ++b)
            if (std::fabs(an[a].x[1] - an[b].x[1]) <= tol && std::fabs(an[a].x[2] - an[b].x[2]) <= tol) {
                const int64_t ra = root(an[a].g), rb = root(an[b].g);
                if (ra != rb) parent[std::max(ra, rb)] = std::min(ra, rb);
            }
    std::vector<int64_t> gid(S.ndof, -1);
    T.glue.resize(S.ndof);
    nglob = 0;
    for (int64_t g = 0; g < S.ndof; ++g) {
        const int64_t r = root(g);
        if (gid[r] < 0) gid[r] = nglob++;
        T.glue[g] = (int32_t)gid[r];
    }
    T.ginv_ptr.assign(nglob + 1, 0);
    for (int64_t g = 0; g < S.ndof; ++g) ++T.ginv_ptr[T.glue[g] + 1];
    for (int64_t k = 0; k < nglob; ++k) T.ginv_ptr[k + 1] += T.ginv_ptr[k];
    T.ginv_idx.resize(S.ndof);
    std::vector<int64_t> fill(T.ginv_ptr.begin(), T.ginv_ptr.end() - 1);
    for (int64_t g = 0; g < S.ndof; ++g) T.ginv_idx[fill[T.glue[g]]++] = (int32_t)g;  // ascending per global
    return true;
}

// S^1 spaces (App. E): component 0 = b^p_j1(s) b^{p-1}_j2(t) e_s (j1 < nbp, j2 < nbq),
// component 1 = b^{p-1}_j1(s) b^p_j2(t) e_t (j1 < nbq, j2 < nbp), local index
// ((f * 2 + c) * nbp * nbq) + (c == 0 ? j1 * nbq + j2 : j1 * nbp + j2).
static int64_t mx_local(const MxTab& T, int f, int c, int j1, int j2) {
    const int64_t per = (int64_t)T.nbp * T.nbq;
    return ((int64_t)f * 2 + c) * per + (c == 0 ? (int64_t)j1 * T.nbq + j2 : (int64_t)j1 * T.nbp + j2);
}

// Normal continuity across patch edges (App. E).  The functions whose degree-p index is first
// or last carry a normal component on that edge, their flux being the tangential B-spline.
// Each such edge function is anchored at the image of (edge coordinate, a), a the mean of
// the Greville abscissa of its tangential factor and the centre of that factor's support
// (distinct for distinct functions, strictly inside the edge, invariant under reversal of
// the edge parameter); by the matching condition (App. D) the function of the neighbour
// with the same anchor is its partner.  Partners form one global function, the second with
// sign -o1 o2 (o = +1 where the reference direction leaves the patch, at coordinate 1, -1 at
// coordinate 0), so that the flux leaving one patch enters the other; an edge function
// without partner (open surface) is dropped.  Globals are numbered in local order.
static bool build_mx(const SpaceDesc& S, int p, MxTab& T, std::string& err) {
    const int nel = S.nel;
    T.p = p;
    T.nbp = nel + p;
    T.nbq = nel + p - 1;
    T.nl = 2 * p * (p + 1);
    const int npatch = S.geom.npatch;
    T.nloc = (int64_t)npatch * 2 * T.nbp * T.nbq;
    // degree p - 1 knots: clamped, 2^L equal elements
    std::vector<double> kq;
    for (int i = 0; i < p; ++i) kq.push_back(0.0);
    for (int k = 1; k < nel; ++k) kq.push_back((double)k / nel);
    for (int i = 0; i < p; ++i) kq.push_back(1.0);
    auto anchor = [&](int j) {
        const int d = p - 1;
        double gr;
        if (d == 0) {
            gr = 0.5 * (kq[j] + kq[j + 1]);
        } else {
            gr = 0.0;
            for (int k = 1; k <= d; ++k) gr += kq[j + k];
            gr /= d;
        }
        return 0.5 * (gr + 0.5 * (kq[j] + kq[j + d + 1]));
    };
    struct Anc {
        double x[3];
        int64_t lid;
    };
    std::vector<Anc> an;
    std::vector<int8_t> orient(T.nloc, 0);  // 0: interior function
    double scale = 0.0;
    for (int f = 0; f < npatch; ++f)
        for (int c = 0; c < 2; ++c)
            for (int e = 0; e < 2; ++e) {
                const int jn = e == 0 ? 0 : T.nbp - 1;
                const double en = e == 0 ? 0.0 : 1.0;
                for (int jt = 0; jt < T.nbq; ++jt) {
                    Anc a;
                    const double at = anchor(jt);
                    if (c == 0) {
                        patch_point(S.geom, f, en, at, a.x);
                        a.lid = mx_local(T, f, 0, jn, jt);
                    } else {
                        patch_point(S.geom, f, at, en, a.x);
                        a.lid = mx_local(T, f, 1, jt, jn);
                    }
                    orient[a.lid] = e == 0 ? -1 : 1;
                    for (double v : a.x) scale = std::max(scale, std::fabs(v));
                    an.push_back(a);
                }
            }
    const double tol = 1e-10 * std::max(scale, 1e-300);
    std::sort(an.begin(), an.end(), [](const Anc& u, const Anc& v) { return u.x[0] < v.x[0]; });
    std::vector<int64_t> partner(T.nloc, -1);
    for (size_t a = 0; a < an.size(); ++a)
        for (size_t b = a + 1; b < an.size() && an[b].x[0] - an[a].x[0] <= tol; ++b)
            if (std::fabs(an[a].x[1] - an[b].x[1]) <= tol && std::fabs(an[a].x[2] - an[b].x[2]) <= tol) {
                if (partner[an[a].lid] >= 0 || partner[an[b].lid] >= 0) {
                    err = "an S^1 edge function matches more than one neighbour (matching condition)";
                    return false;
                }
                partner[an[a].lid] = an[b].lid;
                partner[an[b].lid] = an[a].lid;
            }
    T.glob.assign(T.nloc, -2);
    T.sgn.assign(T.nloc, 1);
    int64_t n = 0;
    for (int64_t l = 0; l < T.nloc; ++l) {
        if (T.glob[l] != -2) continue;
        if (orient[l] == 0) {
            T.glob[l] = (int32_t)n++;
        } else if (partner[l] < 0) {
            T.glob[l] = -1;
            T.sgn[l] = 0;
        } else {
            const int64_t m = partner[l];
            T.glob[l] = T.glob[m] = (int32_t)n++;
            T.sgn[m] = -orient[l] * orient[m];
        }
    }
    T.nglob = n;
    // per element position, in the order of the device evaluation (component 0 with l1 outer,
    // then component 1), and the pieces of every global function in element order
    T.eglob.assign((size_t)S.nelem * T.nl, -1);
    T.esgn.assign((size_t)S.nelem * T.nl, 0);
    std::vector<int64_t> cnt(T.nglob + 1, 0);
    for (int64_t e = 0; e < S.nelem; ++e) {
        const int i2 = (int)(e % nel), i1 = (int)((e / nel) % nel), f = (int)(e / ((int64_t)nel * nel));
        int k = 0;
        for (int l1 = 0; l1 <= p; ++l1)
            for (int l2 = 0; l2 < p; ++l2, ++k) {
                const int64_t l = mx_local(T, f, 0, i1 + l1, i2 + l2);
                T.eglob[e * T.nl + k] = T.glob[l];
                T.esgn[e * T.nl + k] = T.sgn[l];
            }
        for (int l1 = 0; l1 < p; ++l1)
            for (int l2 = 0; l2 <= p; ++l2, ++k) {
                const int64_t l = mx_local(T, f, 1, i1 + l1, i2 + l2);
                T.eglob[e * T.nl + k] = T.glob[l];
                T.esgn[e * T.nl + k] = T.sgn[l];
            }
    }
    for (size_t q = 0; q < T.eglob.size(); ++q)
        if (T.eglob[q] >= 0) ++cnt[T.eglob[q] + 1];
    for (int64_t g = 0; g < T.nglob; ++g) cnt[g + 1] += cnt[g];
    T.gptr = cnt;
    T.gpos.assign(cnt[T.nglob], 0);
    T.gsgn.assign(cnt[T.nglob], 0);
    std::vector<int64_t> fill(cnt.begin(), cnt.end() - 1);
    for (size_t q = 0; q < T.eglob.size(); ++q)
        if (T.eglob[q] >= 0) {
            const int64_t at = fill[T.eglob[q]]++;
            T.gpos[at] = (int32_t)q;
            T.gsgn[at] = T.esgn[q];
        }
    bspline_local_polys(p, 1, S.L, T.polp);
    bspline_local_polys(p - 1, 1, S.L, T.polq);
    return true;
}

static hipError_t mx_upload(MxTab& T) {
    auto put = [](auto** dst, const auto& v) -> hipError_t {
        const size_t bytes = sizeof(v[0]) * std::max<size_t>(v.size(), 1);
        hipError_t e = hipMalloc((void**)dst, bytes);
        if (e != hipSuccess) return e;
        return v.empty() ? hipSuccess : hipMemcpy(*dst, v.data(), sizeof(v[0]) * v.size(), hipMemcpyHostToDevice);
    };
    hipError_t e;
    if ((e = put(&T.d_polp, T.polp)) != hipSuccess) return e;
    if ((e = put(&T.d_polq, T.polq)) != hipSuccess) return e;
    if ((e = put(&T.d_eglob, T.eglob)) != hipSuccess) return e;
    if ((e = put(&T.d_esgn, T.esgn)) != hipSuccess) return e;
    if ((e = put(&T.d_gptr, T.gptr)) != hipSuccess) return e;
    if ((e = put(&T.d_gpos, T.gpos)) != hipSuccess) return e;
    return put(&T.d_gsgn, T.gsgn);
}

// device description of an S^1 space (no operator parts)
static MxDev mx_dev_of(const bem_space_s* s) {
    const MxTab& T = *s->mx;
    MxDev d{};
    d.geom = s->S.geom;
    d.ker = s->S.ker;
    d.p = T.p;
    d.nel = s->S.nel;
    d.nl = T.nl;
    d.h = s->S.h;
    d.nelem = s->S.nelem;
    d.nglob = T.nglob;
    d.polp = T.d_polp;
    d.polq = T.d_polq;
    d.eglob = T.d_eglob;
    d.esgn = T.d_esgn;
    d.gptr = T.d_gptr;
    d.gpos = T.d_gpos;
    d.gsgn = T.d_gsgn;
    return d;
}

// Checks and packs NURBS patches into a geometry (table in host and device memory).
static int make_nurbs_geometry(int npatch, const int* meta, const double* knots, const double* cw,
                               bem_geometry* out) {
    if (!meta || !knots || !cw || !out) return fail(BEM_EINVAL, "NULL argument");
    if (npatch < 1 || npatch > 1 << 20) return fail(BEM_EINVAL, "npatch must lie in [1, 2^20]");
    auto tab = std::make_shared<GeomTab>();
    std::vector<double>& T = tab->host;
    T.assign(1 + 6 * (size_t)npatch, 0.0);
    T[0] = npatch;
    size_t ko = 0, co = 0;
    for (int f = 0; f < npatch; ++f) {
        const int p1 = meta[4 * f], p2 = meta[4 * f + 1], k1 = meta[4 * f + 2], k2 = meta[4 * f + 3];
        const std::string pf = "patch " + std::to_string(f) + ": ";
        if (p1 < 0 || p2 < 0 || p1 > kNurbsMaxDeg || p2 > kNurbsMaxDeg)
            return fail(BEM_EINVAL, pf + "degrees must lie in [0, " + std::to_string(kNurbsMaxDeg) + "]");
        if (k1 <= p1 || k2 <= p2 || k1 > 4096 || k2 > 4096)
            return fail(BEM_EINVAL, pf + "basis counts must exceed the degrees (and be <= 4096)");
        const int pd[2] = {p1, p2}, kd[2] = {k1, k2};
        double* hdr = &T[1 + 6 * (size_t)f];
        hdr[0] = p1;
        hdr[1] = p2;
        hdr[2] = k1;
        hdr[3] = k2;
        hdr[4] = (double)T.size();
        for (int d = 0; d < 2; ++d) {
            const int nk = kd[d] + pd[d] + 1;
            const double* xi = knots + ko;
            ko += nk;
            for (int i = 0; i < nk; ++i) {
                if (!std::isfinite(xi[i])) return fail(BEM_EINVAL, pf + "knots must be finite");
                if (i > 0 && xi[i] < xi[i - 1]) return fail(BEM_EINVAL, pf + "knots must not decrease");
            }
            for (int i = 0; i <= pd[d]; ++i)
                if (xi[i] != 0.0 || xi[nk - 1 - i] != 1.0)
                    return fail(BEM_EINVAL, pf + "knot vectors must be clamped to [0, 1] (degree + 1 end knots)");
            T.insert(T.end(), xi, xi + nk);
        }
        hdr = &T[1 + 6 * (size_t)f];
        hdr[5] = (double)T.size();
        const size_t n = (size_t)k1 * k2 * 4;
        for (size_t i = 0; i < n; ++i) {
            const double v = cw[co + i];
            if (!std::isfinite(v)) return fail(BEM_EINVAL, pf + "control points must be finite");
            if (i % 4 == 3 && !(v > 0.0)) return fail(BEM_EINVAL, pf + "weights must be positive");
        }
        T.insert(T.end(), cw + co, cw + co + n);
        co += n;
    }
    // the device copy; on a host without a GPU the geometry still serves host planning, and
    // every call that would launch a kernel on it fails with EDEVICE
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) == hipSuccess && ndev > 0) {
        HIP_CHECK(hipMalloc((void**)&tab->dev, sizeof(double) * T.size()));
        HIP_CHECK(hipMemcpy(tab->dev, T.data(), sizeof(double) * T.size(), hipMemcpyHostToDevice));
    } else {
        (void)hipGetLastError();
    }
    bem_geometry_s* G = new (std::nothrow) bem_geometry_s;
    if (!G) return fail(BEM_ENOMEM, "host allocation failed");
    G->g = GeomDesc{};
    G->g.kind = GEOM_NURBS;
    G->g.npatch = npatch;
    G->g.a = G->g.b = G->g.c = 1.0;
    G->g.tab_host = tab->host.data();
    G->g.tab_dev = tab->dev;
    G->tab = tab;
    *out = G;
    return BEM_OK;
}

// Dense LU with partial pivoting (row-major n x n, in place) and the solve of one
// right-hand side: the collocation systems of user maps (n <= 4096 + 8).
static bool lu_factor(std::vector<double>& A, int n, std::vector<int>& piv) {
    piv.resize(n);
    for (int c = 0; c < n; ++c) {
        int pr = c;
        for (int r = c + 1; r < n; ++r)
            if (std::fabs(A[(size_t)r * n + c]) > std::fabs(A[(size_t)pr * n + c])) pr = r;
        if (A[(size_t)pr * n + c] == 0.0) return false;
        piv[c] = pr;
        if (pr != c)
            for (int k = 0; k < n; ++k) std::swap(A[(size_t)c * n + k], A[(size_t)pr * n + k]);
        for (int r = c + 1; r < n; ++r) {
            const double m = A[(size_t)r * n + c] / A[(size_t)c * n + c];
            A[(size_t)r * n + c] = m;
            for (int k = c + 1; k < n; ++k) A[(size_t)r * n + k] -= m * A[(size_t)c * n + k];
        }
    }
    return true;
}
static void lu_solve(const std::vector<double>& A, int n, const std::vector<int>& piv, double* b, int stride) {
    for (int c = 0; c < n; ++c) {
        if (piv[c] != c) std::swap(b[(size_t)c * stride], b[(size_t)piv[c] * stride]);
        for (int r = c + 1; r < n; ++r) b[(size_t)r * stride] -= A[(size_t)r * n + c] * b[(size_t)c * stride];
    }
    for (int c = n - 1; c >= 0; --c) {
        double v = b[(size_t)c * stride];
        for (int k = c + 1; k < n; ++k) v -= A[(size_t)c * n + k] * b[(size_t)k * stride];
        b[(size_t)c * stride] = v / A[(size_t)c * n + c];
    }
}

extern "C" {

int bem_geometry_nurbs(int npatch, const int* meta, const double* knots, const double* cw, bem_geometry* out) {
    return make_nurbs_geometry(npatch, meta, knots, cw, out);
}

// File layout (plain text, '#' starts a comment running to the end of its line): the word
// BEMNURBS and the format version 1, the number of patches, then per patch the degrees p1 p2
// and basis counts k1 k2, the k1 + p1 + 1 knots of the first direction, the k2 + p2 + 1
// knots of the second, and k1 * k2 control points "x y z w" (j1 outer).
int bem_geometry_load(const char* path, bem_geometry* out) {
    if (!path || !out) return fail(BEM_EINVAL, "NULL argument");
    std::ifstream in(path);
    if (!in) return fail(BEM_EINVAL, std::string("cannot open ") + path);
    std::stringstream body;
    std::string line;
    while (std::getline(in, line)) {
        const size_t h = line.find('#');
        body << (h == std::string::npos ? line : line.substr(0, h)) << '\n';
    }
    std::string tag;
    int version = 0, npatch = 0;
    if (!(body >> tag >> version) || tag != "BEMNURBS" || version != 1)
        return fail(BEM_EINVAL, "not a BEMNURBS 1 file");
    if (!(body >> npatch) || npatch < 1 || npatch > 1 << 20) return fail(BEM_EINVAL, "bad patch count");
    std::vector<int> meta;
    std::vector<double> knots, cw;
    for (int f = 0; f < npatch; ++f) {
        int m[4];
        if (!(body >> m[0] >> m[1] >> m[2] >> m[3])) return fail(BEM_EINVAL, "truncated patch header");
        if (m[0] < 0 || m[1] < 0 || m[0] > kNurbsMaxDeg || m[1] > kNurbsMaxDeg || m[2] <= m[0] || m[3] <= m[1] ||
            m[2] > 4096 || m[3] > 4096)
            return fail(BEM_EINVAL, "patch " + std::to_string(f) + ": bad degrees or basis counts");
        meta.insert(meta.end(), m, m + 4);
        const size_t nk = (size_t)(m[2] + m[0] + 1) + (size_t)(m[3] + m[1] + 1);
        for (size_t i = 0; i < nk; ++i) {
            double v;
            if (!(body >> v)) return fail(BEM_EINVAL, "truncated knot vector");
            knots.push_back(v);
        }
        const size_t nc = (size_t)m[2] * m[3] * 4;
        for (size_t i = 0; i < nc; ++i) {
            double v;
            if (!(body >> v)) return fail(BEM_EINVAL, "truncated control points");
            cw.push_back(v);
        }
    }
    return make_nurbs_geometry(npatch, meta.data(), knots.data(), cw.data(), out);
}

int bem_geometry_save(bem_geometry g, const char* path) {
    if (!g || !path) return fail(BEM_EINVAL, "NULL argument");
    if (g->g.kind != GEOM_NURBS || !g->tab) return fail(BEM_EINVAL, "only NURBS geometries are written");
    FILE* fp = std::fopen(path, "w");
    if (!fp) return fail(BEM_EINVAL, std::string("cannot create ") + path);
    const std::vector<double>& T = g->tab->host;
    std::fprintf(fp, "BEMNURBS 1\n%d\n", g->g.npatch);
    for (int f = 0; f < g->g.npatch; ++f) {
        const double* h = &T[1 + 6 * (size_t)f];
        const int p1 = (int)h[0], p2 = (int)h[1], k1 = (int)h[2], k2 = (int)h[3];
        std::fprintf(fp, "# patch %d\n%d %d %d %d\n", f, p1, p2, k1, k2);
        const double* xi = &T[(size_t)h[4]];
        for (int i = 0; i < k1 + p1 + 1; ++i) std::fprintf(fp, "%.17g%c", xi[i], i + 1 < k1 + p1 + 1 ? ' ' : '\n');
        xi += k1 + p1 + 1;
        for (int i = 0; i < k2 + p2 + 1; ++i) std::fprintf(fp, "%.17g%c", xi[i], i + 1 < k2 + p2 + 1 ? ' ' : '\n');
        const double* c = &T[(size_t)h[5]];
        for (int i = 0; i < k1 * k2; ++i)
            std::fprintf(fp, "%.17g %.17g %.17g %.17g\n", c[4 * i], c[4 * i + 1], c[4 * i + 2], c[4 * i + 3]);
    }
    const bool ok = std::fclose(fp) == 0;
    return ok ? BEM_OK : fail(BEM_EINVAL, std::string("write failed: ") + path);
}

int bem_geometry_user(int npatch, bem_user_map gamma, void* user, int degree, int intervals, bem_geometry* out) {
    if (!gamma || !out) return fail(BEM_EINVAL, "NULL argument");
    if (npatch < 1 || npatch > 1 << 20) return fail(BEM_EINVAL, "npatch must lie in [1, 2^20]");
    if (degree < 1 || degree > kNurbsMaxDeg) return fail(BEM_EINVAL, "degree must lie in [1, 8]");
    if (intervals < 1 || intervals > 1024) return fail(BEM_EINVAL, "intervals must lie in [1, 1024]");
    const int p = degree, k = intervals + degree;
    // clamped uniform knots, Greville abscissae and the collocation matrix B[i][j] = b_j(x_i)
    std::vector<double> xi;
    for (int i = 0; i <= p; ++i) xi.push_back(0.0);
    for (int i = 1; i < intervals; ++i) xi.push_back((double)i / intervals);
    for (int i = 0; i <= p; ++i) xi.push_back(1.0);
    std::vector<double> gx(k), Bm((size_t)k * k, 0.0);
    for (int j = 0; j < k; ++j) {
        double sum = 0.0;
        for (int m = 1; m <= p; ++m) sum += xi[j + m];
        gx[j] = sum / p;
    }
    for (int i = 0; i < k; ++i) {
        double N[kNurbsMaxDeg + 1];
        const int mu = nurbs_span(xi.data(), p, k, gx[i]);
        nurbs_funs(xi.data(), p, mu, gx[i], N);
        for (int r = 0; r <= p; ++r) Bm[(size_t)i * k + mu - p + r] = N[r];
    }
    std::vector<int> piv;
    if (!lu_factor(Bm, k, piv)) return fail(BEM_EINVAL, "singular collocation matrix");
    std::vector<double> st((size_t)k * k * 2), xyz((size_t)k * k * 3), jac((size_t)k * k * 6);
    for (int i = 0; i < k; ++i)
        for (int j = 0; j < k; ++j) {
            st[2 * ((size_t)i * k + j)] = gx[i];
            st[2 * ((size_t)i * k + j) + 1] = gx[j];
        }
    std::vector<int> meta;
    std::vector<double> knots, cw;
    for (int f = 0; f < npatch; ++f) {
        std::fill(xyz.begin(), xyz.end(), std::nan(""));
        gamma(f, st.data(), (int64_t)k * k, xyz.data(), jac.data(), user);
        for (double v : xyz)
            if (!std::isfinite(v)) return fail(BEM_EINVAL, "the user map returned a non-finite point");
        // B C B^T = F per coordinate: solve along the first index, then along the second
        for (int d = 0; d < 3; ++d) {
            std::vector<double> F((size_t)k * k);
            for (size_t i = 0; i < F.size(); ++i) F[i] = xyz[3 * i + d];
            for (int j = 0; j < k; ++j) lu_solve(Bm, k, piv, &F[j], k);           // columns
            for (int i = 0; i < k; ++i) lu_solve(Bm, k, piv, &F[(size_t)i * k], 1);  // rows
            if (d == 0) cw.resize(cw.size() + (size_t)k * k * 4);
            double* C = &cw[cw.size() - (size_t)k * k * 4];
            for (size_t i = 0; i < F.size(); ++i) {
                C[4 * i + d] = F[i];
                C[4 * i + 3] = 1.0;
            }
        }
        meta.insert(meta.end(), {p, p, k, k});
        knots.insert(knots.end(), xi.begin(), xi.end());
        knots.insert(knots.end(), xi.begin(), xi.end());
    }
    return make_nurbs_geometry(npatch, meta.data(), knots.data(), cw.data(), out);
}

}  // extern "C"

// S^1 space (App. E) for the Maxwell single layer (MS): degree p in the normal direction of
// each component, p - 1 along it, simple interior knots.
static int create_s1(bem_geometry g, double kappa_re, double kappa_im, int p, int knot_repetition, int level,
                     bem_space* out) {
    if (p < 1) return fail(BEM_EINVAL, "S^1 spaces need degree >= 1");
    if (level < 0 || level > 12) return fail(BEM_EINVAL, "level must lie in [0, 12]");
    if (!std::isfinite(kappa_re) || !std::isfinite(kappa_im)) return fail(BEM_EINVAL, "wavenumber must be finite");
    if (kappa_re == 0.0 && kappa_im == 0.0) return fail(BEM_EINVAL, "the Maxwell single layer needs a non-zero wavenumber");
    if (p > kMxMaxP) return fail(BEM_EUNSUPPORTED, "S^1 spaces: this build supports degree <= 2");
    if (knot_repetition != 1) return fail(BEM_EUNSUPPORTED, "S^1 spaces: simple interior knots only (knot repetition 1)");
    SpaceDesc S{};
    S.geom = g->g;
    S.ker.pde = PDE_HELMHOLTZ;  // the fundamental solution of (MS)
    S.ker.kre = kappa_re;
    S.ker.kim = kappa_im;
    S.d = p;
    S.r = 1;
    S.L = level;
    S.nel = 1 << level;
    S.nb = S.nel + p;
    S.nelem = (int64_t)S.geom.npatch * S.nel * S.nel;
    S.h = 1.0 / S.nel;
    S.form = 1;
    auto T = std::make_shared<MxTab>();
    std::string err;
    try {
        if (!build_mx(S, p, *T, err)) return fail(BEM_EINVAL, err);
    } catch (const std::bad_alloc&) {
        return fail(BEM_ENOMEM, "host allocation failed");
    }
    if (T->nloc > 0x7fffffff || S.nelem * T->nl > 0x7fffffff) return fail(BEM_EINVAL, "too many functions for an S^1 space");
    S.ndof = T->nloc;
    S.nglob = T->nglob;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) == hipSuccess && ndev > 0)
        HIP_CHECK(mx_upload(*T));
    else
        (void)hipGetLastError();
    bem_space_s* sp = new (std::nothrow) bem_space_s;
    if (!sp) return fail(BEM_ENOMEM, "host allocation failed");
    sp->S = S;
    sp->tab = g->tab;
    sp->mx = T;
    *out = sp;
    return BEM_OK;
}

// S^1 kernels read the gluing tables from device memory.
static int need_mx_device(const bem_space_s* s) {
    if (s->S.geom.kind == GEOM_NURBS && !s->S.geom.tab_dev)
        return fail(BEM_EDEVICE, "NURBS geometry created without a GPU: no device copy of its tables");
    if (!s->mx->d_eglob) return fail(BEM_EDEVICE, "S^1 space created without a GPU: no device copy of its tables");
    return BEM_OK;
}

// Workspace of a dense S^1 operator: the Galerkin matrix (op), and for the assembly the
// element-pair blocks, the pair types and the two Gauss rules (tmp).
static size_t mx_layout(const bem_operator_s& A, char* ob, char* tb, MxDev* d) {
    const int64_t ne = A.mxd.nelem, nl = A.mxd.nl;
    auto al = [](size_t b) { return (b + 255) / 256 * 256; };
    if (ob) d->M = ob;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        char* q = tb ? tb + off : nullptr;
        off += al(bytes);
        return q;
    };
    char* B = take((size_t)ne * ne * nl * nl * 16);
    char* ti = take((size_t)ne * ne * 4);
    char* bl = take((size_t)ne * ne * 8);
    char* r = take(sizeof(double) * (2 * A.mxd.qg + 2 * A.mxd.qs));
    if (tb) {
        d->B = B;
        d->tinfo = (const int32_t*)ti;
        d->blist = (const int64_t*)bl;
        d->gx = (const double*)r;
        d->gw = d->gx + A.mxd.qg;
        d->sx = d->gw + A.mxd.qg;
        d->sw = d->sx + A.mxd.qs;
    }
    return off + 256;  // + base alignment
}

// Plan of the dense Maxwell operator: every element pair, touching ones classified as for the
// scalar near field (App. C: Duffy rules of the identical, edge and vertex cases).
static int mxh_plan(bem_space_s* s, const bem_h2_params* p, bem_operator* out, bem_operator_info* info);

// pair blocks grouped by kind (the regular ones first, each group in block order)
static int64_t mx_block_list(const std::vector<int32_t>& tinfo, std::vector<int64_t>& bl) {
    bl.clear();
    bl.reserve(tinfo.size());
    for (size_t k = 0; k < tinfo.size(); ++k)
        if (tinfo[k] == 0) bl.push_back((int64_t)k);
    const int64_t nreg = (int64_t)bl.size();
    for (size_t k = 0; k < tinfo.size(); ++k)
        if (tinfo[k] != 0) bl.push_back((int64_t)k);
    return nreg;
}

static int mx_plan(bem_space_s* s, const bem_h2_params* p, bem_operator* out, bem_operator_info* info) {
    if (p->far_low != 0 || p->batch_rhs > 1 || p->far_eval != 0)
        return fail(BEM_EUNSUPPORTED, "S^1 operators: FP64, one column per pass (far_low = 0, batch_rhs <= 1, far_eval = 0)");
    if (p->qg < 1 || p->qg > 8 || p->qs < 1 || p->qs > 16)
        return fail(BEM_EINVAL, "S^1 operators: qg must lie in [1, 8] and qs in [1, 16]");
    if (!(p->eta >= 0.0) || !std::isfinite(p->eta)) return fail(BEM_EINVAL, "eta must be finite and >= 0");
    if (p->eta > 0.0) return mxh_plan(s, p, out, info);
    const SpaceDesc& S = s->S;
    if (S.nelem > 32768) return fail(BEM_EUNSUPPORTED, "S^1 operators: at most 32768 elements (dense pair table)");
    std::vector<int64_t> pairs;
    std::vector<int32_t> tinfo;
    std::string err;
    bem_operator_s* A = new (std::nothrow) bem_operator_s;
    if (!A) return fail(BEM_ENOMEM, "host allocation failed");
    try {
        if (!element_touch_pairs(S, pairs, tinfo, err)) {
            delete A;
            return fail(BEM_EINVAL, err);
        }
        A->mx_tinfo.assign((size_t)(S.nelem * S.nelem), 0);
        for (size_t k = 0; k < tinfo.size(); ++k) A->mx_tinfo[pairs[2 * k] * S.nelem + pairs[2 * k + 1]] = tinfo[k];
        mx_block_list(A->mx_tinfo, A->mx_blist);
        gauss_legendre01(p->qg, A->plan.gx, A->plan.gw);
        gauss_legendre01(p->qs, A->plan.sx, A->plan.sw);
        A->mx_rules.clear();
        for (auto* v : {&A->plan.gx, &A->plan.gw, &A->plan.sx, &A->plan.sw})
            A->mx_rules.insert(A->mx_rules.end(), v->begin(), v->end());
    } catch (const std::bad_alloc&) {
        delete A;
        return fail(BEM_ENOMEM, "host allocation failed while planning");
    }
    A->sp = s;
    A->mx = true;
    A->cplx = true;
    A->scal = 16;
    A->plan.S = S;
    A->plan.leaf = S.L;
    A->dev.S = S;
    MxDev& d = A->mxd;
    d = MxDev{};
    d.p = s->mx->p;
    d.nl = s->mx->nl;
    d.nelem = S.nelem;
    d.nglob = S.nglob;
    d.qg = p->qg;
    d.qs = p->qs;
    d.npairs = S.nelem * S.nelem;
    d.nreg = (int64_t)std::count(A->mx_tinfo.begin(), A->mx_tinfo.end(), 0);
    const int64_t N = S.nglob;
    bem_operator_info& I = A->info;
    I.ndof = N;
    I.nlocal = S.ndof;
    I.nnear = S.nelem * S.nelem;
    I.ntouch = (int64_t)tinfo.size();
    I.near_nnz = N * N;
    I.leaf_level = S.L;
    I.op_bytes = (size_t)N * N * 16 + 256;
    I.tmp_bytes = mx_layout(*A, nullptr, nullptr, nullptr);
    I.near_bytes = (double)N * N * 16;
    if (info) *info = I;
    *out = A;
    return BEM_OK;
}

static int mxh_assemble(bem_operator_s* A, void* op_ws, void* tmp_ws, hipStream_t stream);

static int mx_assemble(bem_operator_s* A, void* op_ws, void* tmp_ws, hipStream_t stream) {
    if (need_mx_device(A->sp) != BEM_OK) return BEM_EDEVICE;
    if (A->mxh) return mxh_assemble(A, op_ws, tmp_ws, stream);
    char* ob = (char*)(((uintptr_t)op_ws + 255) / 256 * 256);
    char* tb = (char*)(((uintptr_t)tmp_ws + 255) / 256 * 256);
    MxDev d = mx_dev_of(A->sp);
    d.qg = A->mxd.qg;
    d.qs = A->mxd.qs;
    d.npairs = A->mxd.npairs;
    d.nreg = A->mxd.nreg;
    mx_layout(*A, ob, tb, &d);
    HIP_CHECK(hipMemcpyAsync((void*)d.tinfo, A->mx_tinfo.data(), A->mx_tinfo.size() * 4, hipMemcpyHostToDevice, stream));
    HIP_CHECK(hipMemcpyAsync((void*)d.blist, A->mx_blist.data(), A->mx_blist.size() * 8, hipMemcpyHostToDevice, stream));
    HIP_CHECK(hipMemcpyAsync((void*)d.gx, A->mx_rules.data(), A->mx_rules.size() * 8, hipMemcpyHostToDevice, stream));
    HIP_CHECK(launch_mx_pairs(d, stream));
    HIP_CHECK(launch_mx_gather(d, stream));
    // the pair blocks, pair types and rules live in the temporary workspace
    d.B = nullptr;
    d.tinfo = nullptr;
    d.blist = nullptr;
    d.gx = d.gw = d.sx = d.sw = nullptr;
    A->mxd = d;
    A->assembled = true;
    return BEM_OK;
}

// Workspace of the compressed S^1 operator.  op: kernel blocks, near element-pair blocks,
// channel moments, the matvec scratch and the tree tables; tmp: the near pair list and
// types, the cluster points and the quadrature tables of the assembly.
static size_t mxh_layout(const bem_operator_s& A, char* ob, char* tb, MxhDev* d, size_t* tmp_bytes) {
    const Plan& pl = A.plan;
    const MxhDev& h = A.mxhd;
    const int64_t q2 = h.q2, nl = h.s.nl, ne = h.s.nelem, npairs = h.s.npairs;
    auto al = [](size_t b) { return (b + 255) / 256 * 256; };
    size_t off = 0;
    auto take = [&](size_t bytes) {
        char* q = ob ? ob + off : nullptr;
        off += al(bytes);
        return q;
    };
    char* K = take((size_t)h.nstored * q2 * q2 * 16);
    char* NB = take((size_t)npairs * nl * nl * 16);
    char* Mt = take((size_t)ne * nl * 4 * q2 * 8);
    char* mom = take((size_t)h.ncl * 4 * q2 * 16);
    char* lv = take((size_t)h.ncl * 4 * q2 * 16);
    char* lev = take(pl.lev_off.size() * 8);
    char* ot = take(pl.own_t.size() * 4);
    char* os = take(pl.own_src.size() * 4);
    char* trp = take(A.mxh_tr_ptr.size() * 8);
    char* trb = take(A.mxh_tr_blk.size() * 4);
    char* tpr = take((size_t)h.nstored * 4 * q2 * 16);
    char* nrp = take(pl.near_rowptr.size() * 4);
    char* ns = take(pl.near_s.size() * 4);
    char* cheb = take(pl.cheb.size() * 8);
    char* E = take(pl.E.size() * 8);
    char* chp0 = take(A.mxh_ch_p0.size() * 4);
    char* chp1 = take(A.mxh_ch_p1.size() * 4);
    char* clch = take(A.mxh_cl_chunk.size() * 8);
    char* part = take(A.mxh_ch_p0.size() * 4 * q2 * 16);
    char* nrow = take(A.mxh_nrowptr.size() * 8);
    char* ncol = take(A.mxh_ncol.size() * 4);
    char* nval = take(A.mxh_ncol.size() * 16);
    const size_t op_total = off + 256;
    size_t toff = 0;
    auto ttake = [&](size_t bytes) {
        char* q = tb ? tb + toff : nullptr;
        toff += al(bytes);
        return q;
    };
    char* plist = ttake((size_t)npairs * 8);
    char* tinfo = ttake((size_t)npairs * 4);
    char* blist = ttake((size_t)npairs * 8);
    char* xc = ttake((size_t)h.ncl * q2 * 3 * 8);
    char* rules = ttake(sizeof(double) * (2 * h.s.qg + 2 * h.s.qs));
    char* lg = ttake(A.mxh_lg.size() * 8);
    if (tmp_bytes) *tmp_bytes = toff + 256;
    if (ob && tb && d) {
        d->K = K;
        d->s.B = NB;
        d->Mt = (double*)Mt;
        d->mom = mom;
        d->lv = lv;
        d->lev_off = (const int64_t*)lev;
        d->own_t = (const int32_t*)ot;
        d->own_s = (const int32_t*)os;
        d->tr_ptr = (const int64_t*)trp;
        d->tr_blk = (const int32_t*)trb;
        d->tprod = tpr;
        d->near_rowptr = (const int32_t*)nrp;
        d->near_s = (const int32_t*)ns;
        d->cheb = (const double*)cheb;
        d->E = (const double*)E;
        d->ch_p0 = (const int32_t*)chp0;
        d->ch_p1 = (const int32_t*)chp1;
        d->cl_chunk = (const int64_t*)clch;
        d->partial = part;
        d->nrowptr = (const int64_t*)nrow;
        d->ncol = (const int32_t*)ncol;
        d->nval = nval;
        d->s.plist = (const int64_t*)plist;
        d->s.tinfo = (const int32_t*)tinfo;
        d->s.blist = (const int64_t*)blist;
        d->xc = (double*)xc;
        d->s.gx = (const double*)rules;
        d->s.gw = d->s.gx + h.s.qg;
        d->s.sx = d->s.gw + h.s.qg;
        d->s.sw = d->s.sx + h.s.qs;
        d->Lg = (const double*)lg;
    }
    return op_total;
}

// Plan of the compressed S^1 operator: the block partition of the scalar operators on the
// same patches (cluster tree, admissibility, near leaf pairs with their touching element
// pairs), from the element space of the same surface and wavenumber.
static int mxh_plan(bem_space_s* s, const bem_h2_params* p, bem_operator* out, bem_operator_info* info) {
    if (p->q < 1 || p->q > 8) return fail(BEM_EINVAL, "q must lie in [1, 8]");
    if (!(p->kappa_adm >= 0.0) || !std::isfinite(p->kappa_adm)) return fail(BEM_EINVAL, "kappa_adm must be finite and >= 0");
    const SpaceDesc& S = s->S;
    if (p->leaf_level > S.L) return fail(BEM_EINVAL, "leaf level must lie in [0, L]");
    SpaceDesc Sc = S;  // element space (degree 0) of the same surface and wavenumber
    Sc.form = 2;
    Sc.d = 0;
    Sc.r = 1;
    Sc.nb = Sc.nel;
    Sc.ndof = Sc.nglob = S.nelem;
    H2Params P;
    P.q = p->q;
    P.eta = p->eta;
    P.leaf = p->leaf_level < 0 ? std::max(S.L - 1, 0) : p->leaf_level;
    P.qg = p->qg;
    P.qs = p->qs;
    P.kadm = p->kappa_adm;
    bem_operator_s* A = new (std::nothrow) bem_operator_s;
    if (!A) return fail(BEM_ENOMEM, "host allocation failed");
    std::string err;
    try {
        if (!build_plan(Sc, P, A->plan, err)) {
            delete A;
            return fail(BEM_EINVAL, err);
        }
        const Plan& pl = A->plan;
        const int m = pl.m, m2 = m * m;
        const int64_t nnear = (int64_t)pl.near_t.size(), npairs = nnear * m2 * m2;
        if (npairs > 0x7fffffff) {
            delete A;
            return fail(BEM_EUNSUPPORTED, "too many near element pairs (lower the leaf level's element count)");
        }
        auto elem = [&](int64_t l, int v) {
            const int n1 = pl.nleaf1;
            const int64_t f = l / ((int64_t)n1 * n1);
            const int li = (int)((l / n1) % n1), lj = (int)(l % n1);
            return (f * S.nel + li * m + v / m) * S.nel + lj * m + v % m;
        };
        A->mxh_plist.resize(npairs);
        A->mx_tinfo.assign(npairs, 0);
        for (int64_t lp = 0; lp < nnear; ++lp) {
            for (int u = 0; u < m2; ++u)
                for (int v = 0; v < m2; ++v)
                    A->mxh_plist[(lp * m2 + u) * m2 + v] = elem(pl.near_t[lp], u) * S.nelem + elem(pl.near_s[lp], v);
            for (int32_t k = pl.touch_rowptr[lp]; k < pl.touch_rowptr[lp + 1]; ++k) {
                const int32_t* t5 = &pl.touch[5 * (size_t)k];
                A->mx_tinfo[(lp * m2 + t5[0]) * m2 + t5[1]] = t5[2] | t5[3] << 4 | t5[4] << 8;
            }
        }
        // glued near field: row g holds every global function h with a piece on an element
        // that forms a near pair with an element of a piece of g (ascending columns).  Per
        // leaf the functions with a piece on it; per row the near leaves of its pieces' leaves,
        // each visited once.
        {
            const MxTab& T = *s->mx;
            const int nl = T.nl;
            const int64_t N = T.nglob, nlv = pl.nleaves;
            std::vector<int64_t> stamp(N, -1), lptr(nlv + 1, 0);
            std::vector<int32_t> ldof, cols;
            for (int64_t l = 0; l < nlv; ++l) {
                for (int v = 0; v < m2; ++v) {
                    const int32_t* eg = &T.eglob[(size_t)elem(l, v) * nl];
                    for (int k = 0; k < nl; ++k)
                        if (eg[k] >= 0 && stamp[eg[k]] != l) {
                            stamp[eg[k]] = l;
                            ldof.push_back(eg[k]);
                        }
                }
                lptr[l + 1] = (int64_t)ldof.size();
            }
            std::fill(stamp.begin(), stamp.end(), -1);
            std::vector<int64_t> seen_src(nlv, -1), seen_near(nlv, -1);
            A->mxh_nrowptr.assign(N + 1, 0);
            A->mxh_ncol.clear();
            for (int64_t g = 0; g < N; ++g) {
                cols.clear();
                for (int64_t t = T.gptr[g]; t < T.gptr[g + 1]; ++t) {
                    const int64_t e1 = T.gpos[t] / nl;
                    const int64_t f = e1 / ((int64_t)S.nel * S.nel);
                    const int i = (int)((e1 / S.nel) % S.nel), j = (int)(e1 % S.nel);
                    const int64_t l1 = (f * pl.nleaf1 + i / m) * pl.nleaf1 + j / m;
                    if (seen_src[l1] == g) continue;
                    seen_src[l1] = g;
                    for (int32_t lp = pl.near_rowptr[l1]; lp < pl.near_rowptr[l1 + 1]; ++lp) {
                        const int32_t l2 = pl.near_s[lp];
                        if (seen_near[l2] == g) continue;
                        seen_near[l2] = g;
                        for (int64_t r = lptr[l2]; r < lptr[l2 + 1]; ++r)
                            if (stamp[ldof[r]] != g) {
                                stamp[ldof[r]] = g;
                                cols.push_back(ldof[r]);
                            }
                    }
                }
                std::sort(cols.begin(), cols.end());
                A->mxh_ncol.insert(A->mxh_ncol.end(), cols.begin(), cols.end());
                A->mxh_nrowptr[g + 1] = (int64_t)A->mxh_ncol.size();
            }
        }
        A->mx_rules.clear();
        for (auto* v : {&pl.gx, &pl.gw, &pl.sx, &pl.sw}) A->mx_rules.insert(A->mx_rules.end(), v->begin(), v->end());
        if (pl.own_src.size() > 0x7fffffff) {
            delete A;
            return fail(BEM_EUNSUPPORTED, "too many admissible pairs");
        }
        mx_block_list(A->mx_tinfo, A->mx_blist);
        // coupling work chunks: up to kMxhChunk consecutive stored blocks of one owner;
        // per cluster the stored blocks in which it is the partner (ascending)
        A->mxh_cl_chunk.assign(pl.ncl + 1, 0);
        for (int64_t c = 0; c < pl.ncl; ++c) {
            for (int64_t q0 = pl.own_rowptr[c]; q0 < pl.own_rowptr[c + 1]; q0 += kMxhChunk) {
                A->mxh_ch_p0.push_back((int32_t)q0);
                A->mxh_ch_p1.push_back((int32_t)std::min<int64_t>(q0 + kMxhChunk, pl.own_rowptr[c + 1]));
            }
            A->mxh_cl_chunk[c + 1] = (int64_t)A->mxh_ch_p0.size();
        }
        A->mxh_tr_ptr.assign(pl.ncl + 1, 0);
        for (int32_t v : pl.own_src) ++A->mxh_tr_ptr[v + 1];
        for (int64_t c = 0; c < pl.ncl; ++c) A->mxh_tr_ptr[c + 1] += A->mxh_tr_ptr[c];
        A->mxh_tr_blk.assign(pl.own_src.size(), 0);
        std::vector<int64_t> fill(A->mxh_tr_ptr.begin(), A->mxh_tr_ptr.end() - 1);
        for (size_t sb = 0; sb < pl.own_src.size(); ++sb) A->mxh_tr_blk[fill[pl.own_src[sb]]++] = (int32_t)sb;
        A->mxh_lg.assign((size_t)m * P.qg * P.q, 0.0);
        for (int i = 0; i < m; ++i)
            for (int k = 0; k < P.qg; ++k)
                for (int a = 0; a < P.q; ++a)
                    A->mxh_lg[((size_t)i * P.qg + k) * P.q + a] = lagrange_bary(pl.cheb, a, (i + pl.gx[k]) / m);
    } catch (const std::bad_alloc&) {
        delete A;
        return fail(BEM_ENOMEM, "host allocation failed while planning");
    }
    const Plan& pl = A->plan;
    A->sp = s;
    A->mx = true;
    A->mxh = true;
    A->cplx = true;
    A->scal = 16;
    A->dev.S = S;
    MxhDev& d = A->mxhd;
    d = MxhDev{};
    d.s.p = s->mx->p;
    d.s.nl = s->mx->nl;
    d.s.nel = S.nel;
    d.s.nelem = S.nelem;
    d.s.nglob = S.nglob;
    d.s.qg = P.qg;
    d.s.qs = P.qs;
    d.s.npairs = (int64_t)A->mxh_plist.size();
    d.s.nreg = (int64_t)std::count(A->mx_tinfo.begin(), A->mx_tinfo.end(), 0);
    d.q = P.q;
    d.q2 = P.q * P.q;
    d.leaf = pl.leaf;
    d.m = pl.m;
    d.nleaf1 = pl.nleaf1;
    d.ncl = pl.ncl;
    d.nleaves = pl.nleaves;
    d.nfar = (int64_t)pl.far_t.size();
    d.nnear = (int64_t)pl.near_t.size();
    d.nchunks = (int64_t)A->mxh_ch_p0.size();
    d.nstored = (int64_t)pl.own_src.size();
    d.nnzg = (int64_t)A->mxh_ncol.size();
    const int64_t N = S.nglob;
    bem_operator_info& I = A->info;
    I.ndof = N;
    I.nlocal = S.ndof;
    I.nclusters = pl.ncl;
    I.nchunks = d.nchunks;
    I.nfar = d.nfar;
    I.nnear = d.nnear;
    I.ntouch = (int64_t)(pl.touch.size() / 5);
    I.near_nnz = d.s.npairs * d.s.nl * d.s.nl;
    I.leaf_level = pl.leaf;
    size_t tmpb = 0;
    I.op_bytes = mxh_layout(*A, nullptr, nullptr, nullptr, &tmpb);
    I.tmp_bytes = tmpb;
    I.nstored = d.nstored;
    I.far_bytes = (double)d.nstored * d.q2 * d.q2 * 16;
    // per apply the glued near field is read: values, columns and row pointers
    I.near_bytes = (double)d.nnzg * 20 + (double)(N + 1) * 8;
    // the plan's own arrays (they stay with the operator) are the scalar element space's;
    // the operator is reported on S^1
    A->plan.S.form = 1;
    if (info) *info = I;
    *out = A;
    return BEM_OK;
}

static int mxh_assemble(bem_operator_s* A, void* op_ws, void* tmp_ws, hipStream_t stream) {
    char* ob = (char*)(((uintptr_t)op_ws + 255) / 256 * 256);
    char* tb = (char*)(((uintptr_t)tmp_ws + 255) / 256 * 256);
    const Plan& pl = A->plan;
    MxhDev d = A->mxhd;
    const MxDev sd = mx_dev_of(A->sp);
    d.s.geom = sd.geom;
    d.s.ker = sd.ker;
    d.s.h = sd.h;
    d.s.polp = sd.polp;
    d.s.polq = sd.polq;
    d.s.eglob = sd.eglob;
    d.s.esgn = sd.esgn;
    d.s.gptr = sd.gptr;
    d.s.gpos = sd.gpos;
    d.s.gsgn = sd.gsgn;
    mxh_layout(*A, ob, tb, &d, nullptr);
    auto up = [&](const void* dst, const void* src, size_t bytes) -> hipError_t {
        if (bytes == 0) return hipSuccess;
        return hipMemcpyAsync((void*)dst, src, bytes, hipMemcpyHostToDevice, stream);
    };
    HIP_CHECK(up(d.lev_off, pl.lev_off.data(), pl.lev_off.size() * 8));
    HIP_CHECK(up(d.own_t, pl.own_t.data(), pl.own_t.size() * 4));
    HIP_CHECK(up(d.own_s, pl.own_src.data(), pl.own_src.size() * 4));
    HIP_CHECK(up(d.tr_ptr, A->mxh_tr_ptr.data(), A->mxh_tr_ptr.size() * 8));
    HIP_CHECK(up(d.tr_blk, A->mxh_tr_blk.data(), A->mxh_tr_blk.size() * 4));
    HIP_CHECK(up(d.near_rowptr, pl.near_rowptr.data(), pl.near_rowptr.size() * 4));
    HIP_CHECK(up(d.near_s, pl.near_s.data(), pl.near_s.size() * 4));
    HIP_CHECK(up(d.cheb, pl.cheb.data(), pl.cheb.size() * 8));
    HIP_CHECK(up(d.E, pl.E.data(), pl.E.size() * 8));
    HIP_CHECK(up(d.ch_p0, A->mxh_ch_p0.data(), A->mxh_ch_p0.size() * 4));
    HIP_CHECK(up(d.ch_p1, A->mxh_ch_p1.data(), A->mxh_ch_p1.size() * 4));
    HIP_CHECK(up(d.cl_chunk, A->mxh_cl_chunk.data(), A->mxh_cl_chunk.size() * 8));
    HIP_CHECK(up(d.s.plist, A->mxh_plist.data(), A->mxh_plist.size() * 8));
    HIP_CHECK(up(d.s.tinfo, A->mx_tinfo.data(), A->mx_tinfo.size() * 4));
    HIP_CHECK(up(d.s.blist, A->mx_blist.data(), A->mx_blist.size() * 8));
    HIP_CHECK(up(d.s.gx, A->mx_rules.data(), A->mx_rules.size() * 8));
    HIP_CHECK(up(d.Lg, A->mxh_lg.data(), A->mxh_lg.size() * 8));
    HIP_CHECK(up(d.nrowptr, A->mxh_nrowptr.data(), A->mxh_nrowptr.size() * 8));
    HIP_CHECK(up(d.ncol, A->mxh_ncol.data(), A->mxh_ncol.size() * 4));
    HIP_CHECK(launch_mxh_assemble(d, stream));
    // tables of the temporary workspace
    d.s.plist = nullptr;
    d.s.tinfo = nullptr;
    d.s.blist = nullptr;
    d.s.gx = d.s.gw = d.s.sx = d.s.sw = nullptr;
    d.xc = nullptr;
    d.Lg = nullptr;
    A->mxhd = d;
    A->assembled = true;
    return BEM_OK;
}

extern "C" {

int bem_space_create(bem_geometry g, int kernel, double kappa_re, double kappa_im, int degree, int knot_repetition,
                     int level, bem_space* out) {
    return bem_space_create_ex(g, kernel, kappa_re, kappa_im, degree, knot_repetition, level, BEM_SPACE_S2, out);
}

int bem_space_create_ex(bem_geometry g, int kernel, double kappa_re, double kappa_im, int degree, int knot_repetition,
                        int level, int space_kind, bem_space* out) {
    if (!g || !out) return fail(BEM_EINVAL, "NULL argument");
    if (space_kind != BEM_SPACE_S2 && space_kind != BEM_SPACE_S0 && space_kind != BEM_SPACE_S1)
        return fail(BEM_EINVAL, "unknown space kind");
    if ((kernel == BEM_MAXWELL_SINGLE) != (space_kind == BEM_SPACE_S1))
        return fail(BEM_EINVAL, "the Maxwell single layer lives on S^1 spaces, the scalar kernels on S^0 and S^2");
    if (space_kind == BEM_SPACE_S1)
        return create_s1(g, kappa_re, kappa_im, degree, knot_repetition, level, out);
    if (space_kind == BEM_SPACE_S0 && degree < 1) return fail(BEM_EINVAL, "continuous spaces need degree >= 1");
    if (kernel != BEM_LAPLACE_SINGLE && kernel != BEM_HELMHOLTZ_SINGLE) return fail(BEM_EINVAL, "unknown kernel");
    if (degree < 0) return fail(BEM_EINVAL, "degree must be >= 0");
    if (level < 0 || level > 12) return fail(BEM_EINVAL, "level must lie in [0, 12]");
    if (knot_repetition < 1 || knot_repetition > degree + 1)
        return fail(BEM_EINVAL, "knot repetition must lie in [1, degree+1]");
    if (kernel == BEM_HELMHOLTZ_SINGLE && kappa_re == 0.0 && kappa_im == 0.0)
        return fail(BEM_EINVAL, "Helmholtz needs a non-zero wavenumber");
    if (!std::isfinite(kappa_re) || !std::isfinite(kappa_im)) return fail(BEM_EINVAL, "wavenumber must be finite");
    if (degree > 2) return fail(BEM_EUNSUPPORTED, "this build supports degree <= 2");
    SpaceDesc S{};
    S.geom = g->g;
    S.ker.pde = kernel;
    S.ker.kre = kernel == BEM_HELMHOLTZ_SINGLE ? kappa_re : 0.0;
    S.ker.kim = kernel == BEM_HELMHOLTZ_SINGLE ? kappa_im : 0.0;
    S.d = degree;
    S.r = knot_repetition;
    S.L = level;
    S.nel = 1 << level;
    S.nb = degree + 1 + (S.nel - 1) * knot_repetition;
    S.nelem = (int64_t)S.geom.npatch * S.nel * S.nel;
    S.ndof = (int64_t)S.geom.npatch * S.nb * S.nb;
    S.h = 1.0 / S.nel;
    S.form = space_kind == BEM_SPACE_S0 ? 0 : 2;
    S.nglob = S.ndof;
    std::shared_ptr<GlueTab> glue;
    if (space_kind == BEM_SPACE_S0) {
        if (S.ndof > 0x7fffffff) return fail(BEM_EINVAL, "too many functions for an S^0 space");
        glue = std::make_shared<GlueTab>();
        build_glue(S, *glue, S.nglob);
        int ndev = 0;
        if (hipGetDeviceCount(&ndev) == hipSuccess && ndev > 0) {
            HIP_CHECK(hipMalloc((void**)&glue->d_glue, sizeof(int32_t) * glue->glue.size()));
            HIP_CHECK(hipMalloc((void**)&glue->d_ptr, sizeof(int64_t) * glue->ginv_ptr.size()));
            HIP_CHECK(hipMalloc((void**)&glue->d_idx, sizeof(int32_t) * glue->ginv_idx.size()));
            HIP_CHECK(hipMemcpy(glue->d_glue, glue->glue.data(), sizeof(int32_t) * glue->glue.size(),
                                hipMemcpyHostToDevice));
            HIP_CHECK(hipMemcpy(glue->d_ptr, glue->ginv_ptr.data(), sizeof(int64_t) * glue->ginv_ptr.size(),
                                hipMemcpyHostToDevice));
            HIP_CHECK(hipMemcpy(glue->d_idx, glue->ginv_idx.data(), sizeof(int32_t) * glue->ginv_idx.size(),
                                hipMemcpyHostToDevice));
            S.glue = glue->d_glue;
            S.ginv_ptr = glue->d_ptr;
            S.ginv_idx = glue->d_idx;
        } else {
            (void)hipGetLastError();
        }
    }
    bem_space_s* sp = new (std::nothrow) bem_space_s;
    if (!sp) return fail(BEM_ENOMEM, "host allocation failed");
    sp->S = S;
    sp->tab = g->tab;
    sp->glue = glue;
    if (!make_basis_tab(S, sp->bt)) {
        delete sp;
        return fail(BEM_EUNSUPPORTED, "element basis classes do not repeat for this knot vector");
    }
    *out = sp;
    return BEM_OK;
}

int bem_space_ndof(bem_space s, int64_t* n) {
    if (!s || !n) return fail(BEM_EINVAL, "NULL argument");
    *n = s->S.nglob;
    return BEM_OK;
}

int bem_space_glue(bem_space s, int64_t* nlocal, int32_t* glue_host) {
    if (!s || !nlocal) return fail(BEM_EINVAL, "NULL argument");
    *nlocal = s->S.ndof;
    if (glue_host && s->mx) {
        std::copy(s->mx->glob.begin(), s->mx->glob.end(), glue_host);
    } else if (glue_host) {
        if (s->glue)
            std::copy(s->glue->glue.begin(), s->glue->glue.end(), glue_host);
        else
            for (int64_t g = 0; g < s->S.ndof; ++g) glue_host[g] = (int32_t)g;
    }
    return BEM_OK;
}

int bem_space_glue_sign(bem_space s, int32_t* sign_host) {
    if (!s || !sign_host) return fail(BEM_EINVAL, "NULL argument");
    if (s->mx)
        std::copy(s->mx->sgn.begin(), s->mx->sgn.end(), sign_host);
    else
        std::fill(sign_host, sign_host + s->S.ndof, 1);
    return BEM_OK;
}

void bem_space_destroy(bem_space s) { delete s; }

int bem_rhs(bem_space s, int data_kind, const double* data_params, int nrhs, void* b_dev, int64_t ldb,
            hipStream_t stream) {
    if (!s || !data_params || !b_dev) return fail(BEM_EINVAL, "NULL argument");
    if (nrhs < 1) return fail(BEM_EINVAL, "nrhs must be >= 1");
    if (need_device_geometry(s->S) != BEM_OK) return BEM_EDEVICE;
    if (ldb < s->S.nglob) return fail(BEM_EINVAL, "ldb must be >= N");
    if (s->mx) {
        if (data_kind != BEM_DATA_DIPOLE && data_kind != BEM_DATA_PLANE_WAVE_E)
            return fail(BEM_EINVAL, "S^1 spaces take BEM_DATA_DIPOLE or BEM_DATA_PLANE_WAVE_E");
        if (need_mx_device(s) != BEM_OK) return BEM_EDEVICE;
        const MxDev d = mx_dev_of(s);
        const Gauss8 g8 = gauss8();
        for (int r = 0; r < nrhs; ++r)
            HIP_CHECK(launch_mx_rhs(d, g8, data_kind - BEM_DATA_DIPOLE, data_params + 6 * r, (char*)b_dev + r * ldb * 16,
                                    stream));
        return BEM_OK;
    }
    if (data_kind != BEM_DATA_POINT_SOURCE && data_kind != BEM_DATA_PLANE_WAVE)
        return fail(BEM_EINVAL, "unknown data kind");
    if (data_kind == BEM_DATA_PLANE_WAVE && s->S.ker.pde != PDE_HELMHOLTZ)
        return fail(BEM_EINVAL, "plane waves need the Helmholtz kernel");
    const Gauss8 g8 = gauss8();
    const size_t sc = s->S.ker.pde == PDE_HELMHOLTZ ? 16 : 8;
    for (int r = 0; r < nrhs; ++r)
        HIP_CHECK(launch_rhs(s->S, s->bt, g8, data_kind, data_params + 3 * r, (char*)b_dev + r * ldb * sc, stream));
    return BEM_OK;
}

int bem_rhs_quadpoints(bem_space s, double* xyz_dev, int64_t* npts, hipStream_t stream) {
    if (!s || !npts) return fail(BEM_EINVAL, "NULL argument");
    if (s->mx) return fail(BEM_EUNSUPPORTED, "sampled data: scalar spaces only");
    *npts = s->S.nelem * 64;
    if (xyz_dev && need_device_geometry(s->S) != BEM_OK) return BEM_EDEVICE;
    if (xyz_dev) HIP_CHECK(launch_quadpoints(s->S, gauss8(), xyz_dev, stream));
    return BEM_OK;
}

int bem_rhs_from_samples(bem_space s, const void* g_dev, int64_t ldg, int nrhs, void* b_dev, int64_t ldb,
                         hipStream_t stream) {
    if (!s || !g_dev || !b_dev) return fail(BEM_EINVAL, "NULL argument");
    if (s->mx) return fail(BEM_EUNSUPPORTED, "sampled data: scalar spaces only");
    if (need_device_geometry(s->S) != BEM_OK) return BEM_EDEVICE;
    if (nrhs < 1) return fail(BEM_EINVAL, "nrhs must be >= 1");
    if (ldb < s->S.nglob) return fail(BEM_EINVAL, "ldb must be >= N");
    if (ldg < s->S.nelem * 64) return fail(BEM_EINVAL, "ldg must be >= the number of quadrature points");
    const Gauss8 g8 = gauss8();
    const size_t sc = s->S.ker.pde == PDE_HELMHOLTZ ? 16 : 8;
    for (int r = 0; r < nrhs; ++r)
        HIP_CHECK(launch_rhs_samples(s->S, s->bt, g8, (const char*)g_dev + r * ldg * sc, (char*)b_dev + r * ldb * sc,
                                     stream));
    return BEM_OK;
}

int bem_eval_potential(bem_space s, const double* pts_dev, int64_t npts, const void* rho_dev, int64_t ldr, int nrhs,
                       void* u_dev, int64_t ldu, hipStream_t stream) {
    if (!s || !rho_dev || (npts > 0 && (!pts_dev || !u_dev))) return fail(BEM_EINVAL, "NULL argument");
    if (nrhs < 1 || npts < 0) return fail(BEM_EINVAL, "nrhs must be >= 1 and npts >= 0");
    if (npts == 0) return BEM_OK;
    if (npts > 0x7fffffff) return fail(BEM_EINVAL, "too many points");
    if (s->mx) {
        if (ldr < s->S.nglob || ldu < 3 * npts) return fail(BEM_EINVAL, "leading dimension too small (S^1: ldu >= 3 npts)");
        if (need_mx_device(s) != BEM_OK) return BEM_EDEVICE;
        const MxDev d = mx_dev_of(s);
        const Gauss8 g8 = gauss8();
        for (int r = 0; r < nrhs; ++r)
            HIP_CHECK(launch_mx_field(d, g8, pts_dev, npts, (const char*)rho_dev + r * ldr * 16,
                                      (char*)u_dev + r * ldu * 16, stream));
        return BEM_OK;
    }
    if (ldr < s->S.nglob || ldu < npts) return fail(BEM_EINVAL, "leading dimension too small");
    if (need_device_geometry(s->S) != BEM_OK) return BEM_EDEVICE;
    if (npts > 0x7fffffff) return fail(BEM_EINVAL, "too many points");
    const Gauss8 g8 = gauss8();
    const size_t sc = s->S.ker.pde == PDE_HELMHOLTZ ? 16 : 8;
    for (int r = 0; r < nrhs; ++r)
        HIP_CHECK(launch_potential(s->S, s->bt, g8, pts_dev, npts, (const char*)rho_dev + r * ldr * sc,
                                   (char*)u_dev + r * ldu * sc, stream));
    return BEM_OK;
}

int bem_assemble_plan(bem_space s, const bem_h2_params* p, bem_operator* out, bem_operator_info* info) {
    if (!s || !p || !out) return fail(BEM_EINVAL, "NULL argument");
    if (s->mx) return mx_plan(s, p, out, info);
    if (p->far_eval != 0 && p->far_eval != 1) return fail(BEM_EINVAL, "far_eval must be 0 or 1");
    if (p->far_eval && (p->far_low != 0 || p->batch_rhs > 1))
        return fail(BEM_EUNSUPPORTED, "far_eval needs far_low = 0 and batch_rhs <= 1");
    if (p->far_eval && s->S.ker.pde == PDE_HELMHOLTZ) {
        // the on-the-fly sine and cosine take arguments Re(kappa) r below 2^20
        const GeomDesc& gd = s->S.geom;
        const double diam = 2.0 * (std::fabs(gd.a) + std::fabs(gd.b) + std::fabs(gd.c) + 1.0);
        if (std::fabs(s->S.ker.kre) * diam >= 1048576.0)
            return fail(BEM_EUNSUPPORTED, "far_eval: Re(kappa) times the surface diameter must stay below 2^20");
    }
    if (p->far_low < 0 || p->far_low > 2) return fail(BEM_EINVAL, "far_low must be 0, BEM_PREC_FP32 or BEM_PREC_BF16");
    if (p->batch_rhs < 0 || p->batch_rhs > 4096) return fail(BEM_EINVAL, "batch_rhs must lie in [0, 4096]");
    if (p->batch_rhs > 1 && p->q > 6) return fail(BEM_EUNSUPPORTED, "many-RHS kernels need q <= 6");
    if (s->S.form == 0 && (p->far_low != 0 || p->batch_rhs > 1))
        return fail(BEM_EUNSUPPORTED, "S^0 spaces: one column at a time in FP64 (far_low = 0, batch_rhs <= 1)");
    H2Params P;
    P.chunk = p->chunk_cols != 0 ? p->chunk_cols : (p->far_eval ? 256 : 128);
    P.q = p->q;
    P.eta = p->eta;
    P.leaf = p->leaf_level;
    P.qg = p->qg;
    P.qs = p->qs;
    if (!(p->kappa_adm >= 0.0) || !std::isfinite(p->kappa_adm)) return fail(BEM_EINVAL, "kappa_adm must be finite and >= 0");
    P.kadm = p->kappa_adm;
    bem_operator_s* A = new (std::nothrow) bem_operator_s;
    if (!A) return fail(BEM_ENOMEM, "host allocation failed");
    std::string err;
    try {
        if (!build_plan(s->S, P, A->plan, err)) {
            delete A;
            return fail(BEM_EINVAL, err);
        }
    } catch (const std::bad_alloc&) {
        delete A;
        return fail(BEM_ENOMEM, "host allocation failed while planning");
    }
    A->sp = s;
    A->cplx = s->S.ker.pde == PDE_HELMHOLTZ;
    A->scal = A->cplx ? 16 : 8;
    A->far_low = p->far_low;
    A->batch_rhs = p->batch_rhs > 1 ? p->batch_rhs : 0;
    A->far_eval = p->far_eval == 1;
    const Plan& pl = A->plan;
    if (A->batch_rhs > 1) {
        // dense near-field tiles: rows of 4 x 4 blocks of B-spline indices, columns the union
        // of their patterns, values padded to whole steps of 4 columns (64 per step)
        const int nb = pl.S.nb, nbt = (nb + 3) / 4;
        A->tile_rowptr.assign(1, 0);
        A->tile_colptr.assign(1, 0);
        A->tile_voff.assign(1, 0);
        std::vector<int32_t> uni, tmp;
        for (int f = 0; f < pl.S.geom.npatch; ++f)
            for (int a1 = 0; a1 < nbt; ++a1)
                for (int a2 = 0; a2 < nbt; ++a2) {
                    uni.clear();
                    for (int j1 = 4 * a1; j1 < std::min(4 * a1 + 4, nb); ++j1)
                        for (int j2 = 4 * a2; j2 < std::min(4 * a2 + 4, nb); ++j2) {
                            const int64_t g = dof_id(pl.S, f, j1, j2);
                            A->tile_rows.push_back((int32_t)g);
                            tmp.clear();
                            std::set_union(uni.begin(), uni.end(), pl.col.begin() + pl.rowptr[g],
                                           pl.col.begin() + pl.rowptr[g + 1], std::back_inserter(tmp));
                            uni.swap(tmp);
                        }
                    A->tile_cols.insert(A->tile_cols.end(), uni.begin(), uni.end());
                    A->tile_rowptr.push_back((int64_t)A->tile_rows.size());
                    A->tile_colptr.push_back((int64_t)A->tile_cols.size());
                    A->tile_voff.push_back(A->tile_voff.back() + (int64_t)((uni.size() + 3) / 4) * 64);
                }
    }
    for (size_t lp = 0; lp + 1 < pl.touch_rowptr.size(); ++lp)
        if (pl.touch_rowptr[lp + 1] > pl.touch_rowptr[lp]) A->touch_lp.push_back((int32_t)lp);
    bem_operator_info& I = A->info;
    I.ndof = s->S.nglob;
    I.nlocal = s->S.ndof;
    I.nclusters = pl.ncl;
    I.nfar = (int64_t)pl.far_t.size();
    I.nnear = (int64_t)pl.near_t.size();
    I.ntouch = (int64_t)(pl.touch.size() / 5);
    I.near_nnz = (int64_t)pl.col.size();
    I.leaf_level = pl.leaf;
    I.op_bytes = op_layout(*A, nullptr, nullptr);
    I.tmp_bytes = tmp_layout(*A, nullptr, nullptr);
    I.far_bytes = A->far_eval ? 0.0 : (double)pl.ktotal * A->scal;
    I.near_bytes = (double)pl.col.size() * (A->scal + 4) + (double)pl.rowptr.size() * 8;
    I.nstored = (int64_t)pl.own_src.size();
    I.nchunks = (int64_t)pl.ch_t.size();
    I.transposed_bytes = (double)pl.ptotal * A->scal;
    if (info) *info = I;
    *out = A;
    return BEM_OK;
}

int bem_operator_info_get(bem_operator A, bem_operator_info* info) {
    if (!A || !info) return fail(BEM_EINVAL, "NULL argument");
    *info = A->info;
    return BEM_OK;
}

int bem_operator_dims(bem_operator A, int64_t* rows, int64_t* cols) {
    if (!A || !rows || !cols) return fail(BEM_EINVAL, "NULL argument");
    *rows = *cols = A->info.ndof;
    return BEM_OK;
}

int bem_assemble(bem_operator A, void* op_ws, size_t op_bytes, void* tmp_ws, size_t tmp_bytes, hipStream_t stream) {
    if (!A || !op_ws || !tmp_ws) return fail(BEM_EINVAL, "NULL argument");
    if (op_bytes < A->info.op_bytes || tmp_bytes < A->info.tmp_bytes)
        return fail(BEM_ENOMEM, "workspace smaller than bem_assemble_plan reported");
    if (A->mx) return mx_assemble(A, op_ws, tmp_ws, stream);
    if (need_device_geometry(A->sp->S) != BEM_OK) return BEM_EDEVICE;
    const Plan& p = A->plan;
    // align the workspaces' bases to 256 bytes
    char* ob = (char*)(((uintptr_t)op_ws + 255) / 256 * 256);
    char* tb = (char*)(((uintptr_t)tmp_ws + 255) / 256 * 256);
    OpDev d;
    AsmDev as;
    BatchDev bd{};
    op_layout(*A, ob, &d, &bd);
    tmp_layout(*A, tb, &as);
    as.xc = const_cast<double*>(d.xc);  // the cluster points stay with the operator
    d.S = p.S;
    d.bt = A->sp->bt;
    d.q = p.P.q;
    d.q2 = p.q2;
    d.leaf = p.leaf;
    d.m = p.m;
    d.nloc = p.nloc;
    d.nleaf1 = p.nleaf1;
    d.qg = p.P.qg;
    d.qs = p.P.qs;
    d.ncl = p.ncl;
    d.nleaves = p.nleaves;
    d.nfar = (int64_t)p.far_t.size();
    d.nstored = (int64_t)p.own_src.size();
    d.up_root = up_root_of(p);
    d.up_depth = p.leaf - d.up_root;
    d.tile = std::min(p.nleaf1, 2);
    d.nchunks = (int64_t)p.ch_t.size();
    d.nnear = (int64_t)p.near_t.size();
    d.ntouch = (int64_t)(p.touch.size() / 5);
    d.nnz = (int64_t)p.col.size();
    d.ngroups = (int64_t)p.grp_rowptr.size() - 1;
    d.cplx = A->cplx ? 1 : 0;
    auto up = [&](const void* dst, const void* src, size_t bytes) -> hipError_t {
        if (bytes == 0) return hipSuccess;
        return hipMemcpyAsync((void*)dst, src, bytes, hipMemcpyHostToDevice, stream);
    };
    HIP_CHECK(up(d.lev_off, p.lev_off.data(), p.lev_off.size() * 8));
    HIP_CHECK(up(d.ball, p.ball.data(), p.ball.size() * 8));
    HIP_CHECK(hipMemsetAsync(d.up_count, 0, sizeof(int) * p.S.geom.npatch, stream));
    HIP_CHECK(up(d.rowptr, p.rowptr.data(), p.rowptr.size() * 8));
    HIP_CHECK(up(d.col, p.col.data(), p.col.size() * 4));
    HIP_CHECK(up(d.grp_rowptr, p.grp_rowptr.data(), p.grp_rowptr.size() * 8));
    HIP_CHECK(up(d.grp_rows, p.grp_rows.data(), p.grp_rows.size() * 4));
    HIP_CHECK(up(d.grp_voff, p.grp_voff.data(), p.grp_voff.size() * 8));
    HIP_CHECK(up(as.row_grp, p.row_grp.data(), p.row_grp.size() * 4));
    HIP_CHECK(up(as.row_pos, p.row_pos.data(), p.row_pos.size() * 4));
    HIP_CHECK(up(d.own_rowptr, p.own_rowptr.data(), p.own_rowptr.size() * 8));
    HIP_CHECK(up(d.own_src, p.own_src.data(), p.own_src.size() * 4));
    HIP_CHECK(up(d.koff, p.koff.data(), p.koff.size() * 8));
    HIP_CHECK(up(d.krs, p.krs.data(), p.krs.size() * 4));
    HIP_CHECK(up(d.pcol, p.pcol.data(), p.pcol.size() * 8));
    HIP_CHECK(up(d.tr_rowptr, p.tr_rowptr.data(), p.tr_rowptr.size() * 8));
    HIP_CHECK(up(d.tr_off, p.tr_off.data(), p.tr_off.size() * 8));
    HIP_CHECK(up(d.ch_t, p.ch_t.data(), p.ch_t.size() * 4));
    HIP_CHECK(up(d.ch_k0, p.ch_k0.data(), p.ch_k0.size() * 4));
    HIP_CHECK(up(d.ch_k1, p.ch_k1.data(), p.ch_k1.size() * 4));
    HIP_CHECK(up(d.cl_chunk, p.cl_chunk.data(), p.cl_chunk.size() * 8));
    HIP_CHECK(up(d.V1, p.V1.data(), p.V1.size() * 8));
    HIP_CHECK(up(d.E, p.E.data(), p.E.size() * 8));
    HIP_CHECK(up(as.near_t, p.near_t.data(), p.near_t.size() * 4));
    HIP_CHECK(up(as.near_s, p.near_s.data(), p.near_s.size() * 4));
    HIP_CHECK(up(as.near_rowptr, p.near_rowptr.data(), p.near_rowptr.size() * 4));
    HIP_CHECK(up(as.touch_rowptr, p.touch_rowptr.data(), p.touch_rowptr.size() * 4));
    HIP_CHECK(up(as.touch, p.touch.data(), p.touch.size() * 4));
    HIP_CHECK(up(as.touch_lp, A->touch_lp.data(), A->touch_lp.size() * 4));
    HIP_CHECK(up(as.vid, p.vid.data(), p.vid.size() * 4));
    HIP_CHECK(up(as.gx, p.gx.data(), p.gx.size() * 8));
    HIP_CHECK(up(as.gw, p.gw.data(), p.gw.size() * 8));
    HIP_CHECK(up(as.psi, p.psi.data(), p.psi.size() * 8));
    HIP_CHECK(up(as.psiw, p.psiw.data(), p.psiw.size() * 8));
    HIP_CHECK(up(as.sx, p.sx.data(), p.sx.size() * 8));
    HIP_CHECK(up(as.sw, p.sw.data(), p.sw.size() * 8));
    HIP_CHECK(up(as.cheb, p.cheb.data(), p.cheb.size() * 8));
    HIP_CHECK(up(as.own_t, p.own_t.data(), p.own_t.size() * 4));
    // coupling rows are padded to even length: clear them before the blocks are written
    if (p.ktotal > 0 && d.K) HIP_CHECK(hipMemsetAsync(d.K, 0, (size_t)p.ktotal * A->scal, stream));
    HIP_CHECK(launch_gauss_points(d, as, stream));
    HIP_CHECK(launch_leaf_tables0(d, as, stream));
    HIP_CHECK(launch_near_regular(d, as, stream));
    HIP_CHECK(launch_near_singular(d, as, stream));
    HIP_CHECK(launch_near_gather(d, as, stream));
    HIP_CHECK(launch_far_assemble(d, as, stream));
    HIP_CHECK(launch_cast_low(d, stream));
    if (A->batch_rhs > 1) {
        // where each ordered far block sits in the stored rows (row 0 of the block, the
        // owner's row stride, negative when the block is stored as its transpose)
        const size_t np = p.far_t.size();
        A->fb_off.resize(np);
        A->fb_rs.resize(np);
        for (size_t i = 0; i < np; ++i) {
            const int t = p.far_t[i], s = p.far_s[i];
            const int lo = std::min(t, s), hi = std::max(t, s);
            const int owner = ((lo + hi) & 1) ? lo : hi, other = owner == t ? s : t;
            auto first = p.own_src.begin() + p.own_rowptr[owner], last = p.own_src.begin() + p.own_rowptr[owner + 1];
            const int64_t slot = std::lower_bound(first, last, other) - first;
            A->fb_off[i] = p.koff[owner] + slot * p.q2;
            A->fb_rs[i] = owner == t ? p.krs[owner] : -p.krs[owner];
        }
        HIP_CHECK(up(bd.tile_rowptr, A->tile_rowptr.data(), A->tile_rowptr.size() * 8));
        HIP_CHECK(up(bd.tile_rows, A->tile_rows.data(), A->tile_rows.size() * 4));
        HIP_CHECK(up(bd.tile_colptr, A->tile_colptr.data(), A->tile_colptr.size() * 8));
        HIP_CHECK(up(bd.tile_cols, A->tile_cols.data(), A->tile_cols.size() * 4));
        HIP_CHECK(up(bd.tile_voff, A->tile_voff.data(), A->tile_voff.size() * 8));
        HIP_CHECK(up(bd.row_grp, p.row_grp.data(), p.row_grp.size() * 4));
        HIP_CHECK(up(bd.row_pos, p.row_pos.data(), p.row_pos.size() * 4));
        HIP_CHECK(launch_tile_fill(d, bd, stream));
        HIP_CHECK(up(bd.far_rowptr, p.far_rowptr.data(), p.far_rowptr.size() * 8));
        HIP_CHECK(up(bd.far_s, p.far_s.data(), np * 4));
        HIP_CHECK(up(bd.fb_off, A->fb_off.data(), np * 8));
        HIP_CHECK(up(bd.fb_rs, A->fb_rs.data(), np * 4));
        if (A->far_low == 2 && p.P.q <= 5) HIP_CHECK(launch_build_bf_blocks(d, bd, (int64_t)np, stream));
        // leaf-to-ancestor transfers: E^(1)_b = E_b; E^(k)_b = E_(b mod 2) E^(k-1)_(b div 2)
        const int Q = p.P.q, q2 = p.q2;
        A->ec.assign((size_t)q2 * ((size_t(2) << p.P.leaf) - 2) + 1, 0.0);
        for (int k = 1; k <= p.P.leaf; ++k) {
            double* Ek = A->ec.data() + (size_t)q2 * ((size_t(1) << k) - 2);
            const double* Ep = A->ec.data() + (size_t)q2 * ((size_t(1) << (k - 1)) - 2);
            for (int b = 0; b < (1 << k); ++b)
                for (int pp = 0; pp < Q; ++pp)
                    for (int a = 0; a < Q; ++a) {
                        double v = 0.0;
                        if (k == 1) {
                            v = p.E[((size_t)b * Q + pp) * Q + a];
                        } else {
                            for (int mid = 0; mid < Q; ++mid)
                                v += p.E[((size_t)(b & 1) * Q + pp) * Q + mid] * Ep[((size_t)(b >> 1) * Q + mid) * Q + a];
                        }
                        Ek[((size_t)b * Q + pp) * Q + a] = v;
                    }
        }
        HIP_CHECK(up(bd.Ec, A->ec.data(), A->ec.size() * 8));
    }
    A->bdev = bd;
    // the host tables above are copied from pageable memory; make sure they have been read
    // before the caller may free the temporary workspace (the plan itself stays alive)
    A->dev = d;
    A->assembled = true;
    return BEM_OK;
}

int bem_apply(bem_operator A, const void* x_dev, int64_t ldx, void* y_dev, int64_t ldy, int nrhs, hipStream_t stream) {
    return bem_apply_ex(A, BEM_PREC_FP64, x_dev, ldx, y_dev, ldy, nrhs, stream);
}

int bem_apply_ex(bem_operator A, int prec, const void* x_dev, int64_t ldx, void* y_dev, int64_t ldy, int nrhs,
                 hipStream_t stream) {
    if (!A || !x_dev || !y_dev) return fail(BEM_EINVAL, "NULL argument");
    if (prec != BEM_PREC_FP64 && prec != A->far_low)
        return fail(BEM_EINVAL, "precision not available (assemble with far_low set to it)");
    if (!A->assembled) return fail(BEM_EINVAL, "operator not assembled");
    if (nrhs < 1) return fail(BEM_EINVAL, "nrhs must be >= 1");
    const int64_t N = A->info.ndof;
    if (ldx < N || ldy < N) return fail(BEM_EINVAL, "leading dimension too small");
    const char* xb = (const char*)x_dev;
    char* yb = (char*)y_dev;
    const size_t span_x = ((size_t)(nrhs - 1) * ldx + N) * A->scal, span_y = ((size_t)(nrhs - 1) * ldy + N) * A->scal;
    if (!(xb + span_x <= yb || yb + span_y <= xb)) return fail(BEM_EINVAL, "x and y overlap");
    if (nrhs > 1 && A->batch_rhs > 1) {
        if (prec == BEM_PREC_BF16 && A->plan.P.q > 5) return fail(BEM_EUNSUPPORTED, "BF16 many-RHS coupling needs q <= 5");
        for (int r0 = 0; r0 < nrhs; r0 += A->batch_rhs) {
            BatchDev bd = A->bdev;
            bd.R = std::min(A->batch_rhs, nrhs - r0);
            const void* xr = xb + (size_t)r0 * ldx * A->scal;
            void* yr = yb + (size_t)r0 * ldy * A->scal;
            if (!A->prof) {
                HIP_CHECK(launch_apply_batched(A->dev, bd, xr, ldx, yr, ldy, prec, stream));
                continue;
            }
            const size_t need = A->ev_used + kBatchStages + 1;
            while (A->ev.size() < need) {
                hipEvent_t e;
                HIP_CHECK(hipEventCreate(&e));
                A->ev.push_back(e);
            }
            HIP_CHECK(hipEventRecord(A->ev[A->ev_used], stream));
            for (int s = 0; s < kBatchStages; ++s) {
                HIP_CHECK(launch_apply_batched_stage(A->dev, bd, s, xr, ldx, yr, ldy, prec, stream));
                HIP_CHECK(hipEventRecord(A->ev[A->ev_used + 1 + s], stream));
            }
            A->ev_used = need;
        }
        return BEM_OK;
    }
    for (int r = 0; r < nrhs; ++r) {
        const void* xr = xb + (size_t)r * ldx * A->scal;
        void* yr = yb + (size_t)r * ldy * A->scal;
        if (!A->prof) {
            HIP_CHECK(op_apply(A, prec, xr, yr, stream));
            continue;
        }
        const size_t need = A->ev_used + kApplyStages + 1;
        while (A->ev.size() < need) {
            hipEvent_t e;
            HIP_CHECK(hipEventCreate(&e));
            A->ev.push_back(e);
        }
        HIP_CHECK(hipEventRecord(A->ev[A->ev_used], stream));
        for (int s = 0; s < kApplyStages; ++s) {
            HIP_CHECK(launch_apply_stage(A->dev, s, xr, yr, prec, stream));
            HIP_CHECK(hipEventRecord(A->ev[A->ev_used + 1 + s], stream));
        }
        A->ev_used = need;
    }
    return BEM_OK;
}

int bem_apply_stage(bem_operator A, int prec, int stage, const void* x_dev, void* y_dev, hipStream_t stream) {
    if (!A || !x_dev || !y_dev) return fail(BEM_EINVAL, "NULL argument");
    if (!A->assembled) return fail(BEM_EINVAL, "operator not assembled");
    if (prec != BEM_PREC_FP64 && prec != A->far_low)
        return fail(BEM_EINVAL, "precision not available (assemble with far_low set to it)");
    if (stage < 0 || stage >= kApplyStages) return fail(BEM_EINVAL, "stage must lie in [0, 4)");
    if (A->plan.S.form != 2) return fail(BEM_EUNSUPPORTED, "single stages need an S^2 space");
    HIP_CHECK(launch_apply_stage(A->dev, stage, x_dev, y_dev, prec, stream));
    return BEM_OK;
}

int bem_profile_enable(bem_operator A, int on) {
    if (A && A->plan.S.form != 2 && on) return fail(BEM_EUNSUPPORTED, "stage timing needs an S^2 space");
    if (!A) return fail(BEM_EINVAL, "NULL argument");
    A->prof = on != 0;
    A->ev_used = 0;
    return BEM_OK;
}

int bem_profile_read(bem_operator A, double* stage_ms, int nstages, int* napplies) {
    if (!A || !stage_ms || !napplies) return fail(BEM_EINVAL, "NULL argument");
    if (nstages < kApplyStages) return fail(BEM_EINVAL, "nstages must be >= 4");
    const size_t per = kApplyStages + 1;
    const size_t n = A->ev_used / per;
    for (int s = 0; s < nstages; ++s) stage_ms[s] = 0.0;
    if (n > 0) HIP_CHECK(hipEventSynchronize(A->ev[A->ev_used - 1]));
    for (size_t k = 0; k < n; ++k)
        for (int s = 0; s < kApplyStages; ++s) {
            float ms = 0.0f;
            HIP_CHECK(hipEventElapsedTime(&ms, A->ev[k * per + s], A->ev[k * per + s + 1]));
            stage_ms[s] += ms;
        }
    if (n > 0)
        for (int s = 0; s < kApplyStages; ++s) stage_ms[s] /= (double)n;
    *napplies = (int)n;
    A->ev_used = 0;
    return BEM_OK;
}

void bem_operator_destroy(bem_operator A) { delete A; }

// ------------------------------------------------------------------------------ preconditioner
static int64_t prec_tiles(const bem_operator_s& A, int* nt) {
    const int t = (A.plan.S.nb + kTile - 1) / kTile;
    if (nt) *nt = t;
    return (int64_t)A.plan.S.geom.npatch * t * t;
}

int bem_precond_info(bem_operator A, int64_t* ntiles, size_t* ws_bytes) {
    if (A && A->plan.S.form != 2) return fail(BEM_EUNSUPPORTED, "the block preconditioner needs an S^2 space");
    if (!A || !ntiles || !ws_bytes) return fail(BEM_EINVAL, "NULL argument");
    *ntiles = prec_tiles(*A, nullptr);
    OpDev d{};
    d.S = A->plan.S;
    d.cplx = A->cplx ? 1 : 0;
    *ws_bytes = prec_layout(d, *ntiles, nullptr, nullptr);
    return BEM_OK;
}

int bem_precond_build(bem_operator A, void* ws, size_t ws_bytes, hipStream_t stream) {
    if (A && A->plan.S.form != 2) return fail(BEM_EUNSUPPORTED, "the block preconditioner needs an S^2 space");
    if (!A || !ws) return fail(BEM_EINVAL, "NULL argument");
    if (!A->assembled) return fail(BEM_EINVAL, "operator not assembled");
    int nt = 0;
    const int64_t ntl = prec_tiles(*A, &nt);
    if (ws_bytes < prec_layout(A->dev, ntl, nullptr, nullptr)) return fail(BEM_ENOMEM, "workspace too small");
    char* base = (char*)(((uintptr_t)ws + 255) / 256 * 256);
    PrecDev pc{};
    prec_layout(A->dev, ntl, base, &pc);
    pc.nt = nt;
    HIP_CHECK(hipMemsetAsync(pc.status, 0, sizeof(int), stream));
    HIP_CHECK(launch_prec_build(A->dev, pc, stream));
    int st = 0;
    HIP_CHECK(hipMemcpyAsync(&st, pc.status, sizeof(int), hipMemcpyDeviceToHost, stream));
    HIP_CHECK(hipStreamSynchronize(stream));
    if (st != 0) return fail(BEM_EDEVICE, "a diagonal block of the near field is singular");
    A->pdev = pc;
    A->prec_built = true;
    return BEM_OK;
}

int bem_precond_apply(bem_operator A, const void* r, int64_t ldr, void* z, int64_t ldz, int nrhs, hipStream_t stream) {
    if (!A || !r || !z) return fail(BEM_EINVAL, "NULL argument");
    if (!A->prec_built) return fail(BEM_EINVAL, "preconditioner not built");
    const int64_t N = A->info.ndof;
    if (nrhs < 1 || ldr < N || ldz < N) return fail(BEM_EINVAL, "nrhs >= 1 and leading dimensions >= N");
    for (int c = 0; c < nrhs; ++c)
        HIP_CHECK(launch_prec_apply(A->dev, A->pdev, 1, (const char*)r + (size_t)c * ldr * A->scal,
                                    (char*)z + (size_t)c * ldz * A->scal, stream));
    return BEM_OK;
}

int bem_precond_export(bem_operator A, int which, double* inv_host, hipStream_t stream) {
    if (!A || !inv_host) return fail(BEM_EINVAL, "NULL argument");
    if (!A->prec_built) return fail(BEM_EINVAL, "preconditioner not built");
    const size_t bytes = (size_t)A->pdev.ntiles * kTileN * kTileN * A->scal;
    HIP_CHECK(hipMemcpyAsync(inv_host, which ? A->pdev.D0inv : A->pdev.Dinv, bytes, hipMemcpyDeviceToHost, stream));
    HIP_CHECK(hipStreamSynchronize(stream));
    return BEM_OK;
}

int bem_precond_features(bem_operator A, float* feats_dev, hipStream_t stream) {
    if (!A || !feats_dev) return fail(BEM_EINVAL, "NULL argument");
    if (!A->prec_built) return fail(BEM_EINVAL, "preconditioner not built");
    HIP_CHECK(launch_prec_features(A->dev, A->pdev, feats_dev, stream));
    return BEM_OK;
}

int bem_precond_target_bytes(bem_operator A, int ring, int64_t nt, size_t* bytes) {
    if (!A || !bytes) return fail(BEM_EINVAL, "NULL argument");
    if (A->plan.S.form != 2) return fail(BEM_EUNSUPPORTED, "the block preconditioner needs an S^2 space");
    if (ring < 0 || ring > 8 || nt < 1) return fail(BEM_EINVAL, "ring in [0, 8] and nt >= 1");
    OpDev d{};
    d.S = A->plan.S;
    d.cplx = A->cplx ? 1 : 0;
    *bytes = prec_target_bytes(d, ring, nt) + 256;
    return BEM_OK;
}

int bem_precond_targets(bem_operator A, int ring, int64_t t0, int64_t nt, void* work, size_t work_bytes,
                        float* delta_dev, hipStream_t stream) {
    if (!A || !work || !delta_dev) return fail(BEM_EINVAL, "NULL argument");
    if (!A->prec_built) return fail(BEM_EINVAL, "preconditioner not built");
    if (ring < 0 || ring > 8 || nt < 1 || t0 < 0 || t0 + nt > A->pdev.ntiles)
        return fail(BEM_EINVAL, "ring in [0, 8] and tiles inside [0, ntiles)");
    if (work_bytes < prec_target_bytes(A->dev, ring, nt) + 256) return fail(BEM_ENOMEM, "work too small");
    char* base = (char*)(((uintptr_t)work + 255) / 256 * 256);
    HIP_CHECK(hipMemsetAsync(A->pdev.status, 0, sizeof(int), stream));
    HIP_CHECK(launch_prec_targets(A->dev, A->pdev, ring, t0, nt, base, delta_dev, stream));
    int st = 0;
    HIP_CHECK(hipMemcpyAsync(&st, A->pdev.status, sizeof(int), hipMemcpyDeviceToHost, stream));
    HIP_CHECK(hipStreamSynchronize(stream));
    if (st != 0) return fail(BEM_EDEVICE, "a neighbourhood system of the near field is singular");
    return BEM_OK;
}

int bem_precond_correct(bem_operator A, const float* uv_dev, int mode, int ring, int* accepted_host,
                        hipStream_t stream) {
    if (!A || (!uv_dev && mode != 0)) return fail(BEM_EINVAL, "NULL argument");
    if (!A->prec_built) return fail(BEM_EINVAL, "preconditioner not built");
    if (mode < 0 || mode > 2 || ring < 0 || ring > 8) return fail(BEM_EINVAL, "mode in {0,1,2}, ring in [0, 8]");
    const int64_t nt = A->pdev.ntiles;
    if (mode == 0) {
        HIP_CHECK(hipMemcpyAsync(A->pdev.Dinv, A->pdev.D0inv, (size_t)nt * kTileN * kTileN * A->scal,
                                 hipMemcpyDeviceToDevice, stream));
        HIP_CHECK(hipStreamSynchronize(stream));
        if (accepted_host) std::memset(accepted_host, 0, sizeof(int) * nt);
        return BEM_OK;
    }
    HIP_CHECK(launch_prec_correct(A->dev, A->pdev, uv_dev, mode, ring, A->pdev.accepted, stream));
    if (accepted_host)
        HIP_CHECK(hipMemcpyAsync(accepted_host, A->pdev.accepted, sizeof(int) * nt, hipMemcpyDeviceToHost, stream));
    HIP_CHECK(hipStreamSynchronize(stream));
    return BEM_OK;
}

int bem_solve_plan(bem_operator A, int nrhs, const bem_solve_params* p, size_t* bytes) {
    if (!A || !p || !bytes) return fail(BEM_EINVAL, "NULL argument");
    if (nrhs < 1 || p->restart < 1 || p->restart > kMaxRestart)
        return fail(BEM_EINVAL, "nrhs must be >= 1 and restart in [1, 64]");
    const int hist = refine_hist(p);
    *bytes = solve_layout(A->info.ndof, p->restart, A->scal, nullptr, nullptr, hist);
    if (nrhs > 1 && A->batch_rhs > 1)
        *bytes = std::max(*bytes, bsolve_layout(A->info.ndof, p->restart, std::min(nrhs, A->batch_rhs), A->scal,
                                                nullptr, nullptr, hist));
    return BEM_OK;
}

int bem_solve(bem_operator A, const void* b_dev, int64_t ldb, void* x_dev, int64_t ldx, int nrhs,
              const bem_solve_params* p, bem_solve_stats* stats, void* ws, size_t ws_bytes, hipStream_t stream) {
    if (!A || !b_dev || !x_dev || !p || !stats || !ws) return fail(BEM_EINVAL, "NULL argument");
    if (!A->assembled) return fail(BEM_EINVAL, "operator not assembled");
    if (nrhs < 1 || p->restart < 1 || p->restart > kMaxRestart || p->maxit < 1 || !(p->tol > 0.0))
        return fail(BEM_EINVAL, "bad solver parameters (restart must lie in [1, 64])");
    for (int i = 0; i < 2; ++i)
        if (p->reserved[i] != 0) return fail(BEM_EINVAL, "reserved fields must be zero");
    if (p->inner_maxit < 0) return fail(BEM_EINVAL, "inner_maxit must be >= 0");
    if (p->precond != BEM_PRECOND_NONE && p->precond != BEM_PRECOND_BLOCK)
        return fail(BEM_EINVAL, "precond must be BEM_PRECOND_NONE or BEM_PRECOND_BLOCK");
    if (p->precond == BEM_PRECOND_BLOCK && !A->prec_built) return fail(BEM_EINVAL, "preconditioner not built");
    const int64_t N = A->info.ndof;
    if (ldb < N || ldx < N) return fail(BEM_EINVAL, "leading dimension too small");
    if (p->refine != 0 && p->refine != 1) return fail(BEM_EINVAL, "refine must be 0 or 1");
    if (p->refine && A->far_low == 0) return fail(BEM_EINVAL, "refinement needs far_low set at assembly");
    if (p->max_outer < 0 || p->inner_tol < 0.0) return fail(BEM_EINVAL, "max_outer and inner_tol must be >= 0");
    if (!A->pinned) HIP_CHECK(hipHostMalloc((void**)&A->pinned, sizeof(double) * (kMaxRestart + 2 + kSolveBlocks)));
    char* base = (char*)(((uintptr_t)ws + 255) / 256 * 256);
    const int hist = refine_hist(p);
    if (nrhs > 1 && A->batch_rhs > 1) {
        // many right-hand sides in lockstep, up to batch_rhs per pass
        const int Rb = std::min(nrhs, A->batch_rhs);
        if (ws_bytes < bsolve_layout(N, p->restart, Rb, A->scal, nullptr, nullptr, hist))
            return fail(BEM_ENOMEM, "solver workspace too small");
        BSolveWs W;
        bsolve_layout(N, p->restart, Rb, A->scal, base, &W, hist);
        bool all = true;
        for (int r0 = 0; r0 < nrhs; r0 += Rb) {
            const int R = std::min(Rb, nrhs - r0);
            HIP_CHECK(launch_to_slab(A->cplx, N, R, (const char*)b_dev + (size_t)r0 * ldb * A->scal, ldb, W.bs,
                                     stream));
            const int rc = p->refine ? refine_batched(A, W.bs, W.xs, R, p, stats + r0, W, stream)
                                     : gmres_batched(A, 0, W.bs, W.xs, R, p->restart, p->maxit, p->tol, stats + r0,
                                                     W, stream, p->precond != 0);
            if (rc != BEM_OK) return rc;
            HIP_CHECK(launch_from_slab(A->cplx, N, R, W.xs, (char*)x_dev + (size_t)r0 * ldx * A->scal, ldx, stream));
            for (int r = 0; r < R; ++r) all = all && stats[r0 + r].converged;
        }
        HIP_CHECK(hipStreamSynchronize(stream));
        if (!all) return fail(BEM_ENOCONV, "GMRES did not reach the tolerance for every right-hand side");
        return BEM_OK;
    }
    const size_t need = solve_layout(N, p->restart, A->scal, nullptr, nullptr, hist);
    if (ws_bytes < need) return fail(BEM_ENOMEM, "solver workspace too small");
    SolveWs W;
    solve_layout(N, p->restart, A->scal, base, &W, hist);
    bool all = true;
    for (int r = 0; r < nrhs; ++r) {
        const void* b = (const char*)b_dev + (size_t)r * ldb * A->scal;
        void* x = (char*)x_dev + (size_t)r * ldx * A->scal;
        const int rc = p->refine ? refine_one(A, b, x, p, &stats[r], W, stream)
                                 : gmres_one(A, 0, b, x, p->restart, p->maxit, p->tol, &stats[r], W, stream,
                                             p->precond != 0);
        if (rc != BEM_OK) return rc;
        all = all && stats[r].converged;
    }
    if (!all) return fail(BEM_ENOCONV, "GMRES did not reach the tolerance for every right-hand side");
    return BEM_OK;
}

int bem_precond_select(bem_operator A, const float* uv_dev, const void* b_dev, int restart, void* ws,
                       size_t ws_bytes, int* kept, double* relres2, hipStream_t stream) {
    if (!A || !uv_dev || !b_dev || !ws || !kept) return fail(BEM_EINVAL, "NULL argument");
    if (!A->prec_built) return fail(BEM_EINVAL, "preconditioner not built");
    if (restart < 1 || restart > kMaxRestart) return fail(BEM_EINVAL, "restart in [1, 64]");
    const int64_t N = A->info.ndof;
    const size_t need = solve_layout(N, restart, A->scal, nullptr, nullptr);
    if (ws_bytes < need + (size_t)N * A->scal + 512) return fail(BEM_ENOMEM, "workspace too small");
    if (!A->pinned) HIP_CHECK(hipHostMalloc((void**)&A->pinned, sizeof(double) * (kMaxRestart + 2 + kSolveBlocks)));
    char* base = (char*)(((uintptr_t)ws + 255) / 256 * 256);
    SolveWs W;
    solve_layout(N, restart, A->scal, base, &W);
    char* x = base + (need + 255) / 256 * 256;
    double rr[2] = {0.0, 0.0};
    for (int c = 0; c < 2; ++c) {
        const int rc = bem_precond_correct(A, c ? uv_dev : nullptr, c ? 1 : 0, 0, nullptr, stream);
        if (rc != BEM_OK) return rc;
        bem_solve_stats st{};
        const int g = gmres_one(A, 0, b_dev, x, restart, restart, 1e-300, &st, W, stream, true);
        if (g != BEM_OK) return g;
        rr[c] = st.relres;
    }
    *kept = rr[1] < rr[0] ? 1 : 0;
    if (!*kept) {
        const int rc = bem_precond_correct(A, nullptr, 0, 0, nullptr, stream);
        if (rc != BEM_OK) return rc;
    }
    if (relres2) {
        relres2[0] = rr[0];
        relres2[1] = rr[1];
    }
    return BEM_OK;
}

// ------------------------------------------------------------------------------ network
int bem_mlp_sizes(int in, int hidden, int out, int batch, int64_t* nparams, size_t* ws_bytes) {
    if (!nparams || !ws_bytes) return fail(BEM_EINVAL, "NULL argument");
    if (in < 1 || hidden < 1 || out < 1 || batch < 1) return fail(BEM_EINVAL, "sizes must be >= 1");
    *nparams = mlp_nparams(in, hidden, out);
    *ws_bytes = mlp_ws_bytes(hidden, out, batch);
    return BEM_OK;
}

int bem_mlp_init(int in, int hidden, int out, uint64_t seed, float* params_dev, hipStream_t stream) {
    if (!params_dev) return fail(BEM_EINVAL, "NULL argument");
    if (in < 1 || hidden < 1 || out < 1) return fail(BEM_EINVAL, "sizes must be >= 1");
    HIP_CHECK(mlp_init(in, hidden, out, seed, params_dev, stream));
    return BEM_OK;
}

int bem_mlp_forward(int in, int hidden, int out, int batch, const float* params_dev, const float* X_dev, float* Y_dev,
                    int precision, void* ws, size_t ws_bytes, hipStream_t stream) {
    if (!params_dev || !X_dev || !Y_dev || !ws) return fail(BEM_EINVAL, "NULL argument");
    if (in < 1 || hidden < 1 || out < 1 || batch < 1 || (precision != 0 && precision != 1))
        return fail(BEM_EINVAL, "sizes >= 1, precision 0 or 1");
    if (batch > kMlpMaxBatch) return fail(BEM_EINVAL, "batch above " + std::to_string(kMlpMaxBatch));
    if (ws_bytes < mlp_ws_bytes(hidden, out, batch)) return fail(BEM_ENOMEM, "workspace too small");
    HIP_CHECK(mlp_forward(in, hidden, out, batch, params_dev, X_dev, Y_dev, precision, ws, stream));
    return BEM_OK;
}

int bem_mlp_forward_noalloc(int in, int hidden, int out, int batch, const float* params_dev, const float* X_dev,
                            float* Y_dev, int precision, hipStream_t stream) {
    if (!params_dev || !X_dev || !Y_dev) return fail(BEM_EINVAL, "NULL argument");
    if (in < 1 || hidden < 1 || out < 1 || batch < 1 || (precision != 0 && precision != 1))
        return fail(BEM_EINVAL, "sizes >= 1, precision 0 or 1");
    if (batch > kMlpMaxBatch) return fail(BEM_EINVAL, "batch above " + std::to_string(kMlpMaxBatch));
    const size_t need = mlp_forward_scratch_bytes(hidden, batch);
    if (need > kMlpScratchBytes)
        return fail(BEM_EINVAL, "batch * hidden too large for the fixed scratch: needs " + std::to_string(need) +
                                    " bytes, the limit is " + std::to_string(kMlpScratchBytes));
    void* scr = nullptr;
    HIP_CHECK(mlp_scratch(&scr));
    HIP_CHECK(mlp_forward_noalloc(in, hidden, out, batch, params_dev, X_dev, Y_dev, precision, scr, stream));
    return BEM_OK;
}

int bem_mlp_loss_grad(int in, int hidden, int out, int batch, int is_complex, const float* params_dev,
                      const float* X_dev, const float* T_dev, float* grad_dev, float* loss_dev, int precision,
                      void* ws, size_t ws_bytes, hipStream_t stream) {
    if (!params_dev || !X_dev || !T_dev || !grad_dev || !loss_dev || !ws) return fail(BEM_EINVAL, "NULL argument");
    if (in < 1 || hidden < 1 || batch < 1 || (precision != 0 && precision != 1))
        return fail(BEM_EINVAL, "sizes >= 1, precision 0 or 1");
    if (out != (is_complex ? 4 : 2) * kMlpSlots * kMlpRank) return fail(BEM_EINVAL, "out must be 1024 (real) or 2048");
    if (ws_bytes < mlp_ws_bytes(hidden, out, batch)) return fail(BEM_ENOMEM, "workspace too small");
    HIP_CHECK(mlp_loss_grad(in, hidden, out, batch, is_complex ? 1 : 0, params_dev, X_dev, T_dev, grad_dev, loss_dev,
                            precision, ws, stream));
    return BEM_OK;
}

int bem_mlp_adam(int64_t n, float* params_dev, const float* grad_dev, float* m_dev, float* v_dev, int step, float lr,
                 float beta1, float beta2, float eps, hipStream_t stream) {
    if (!params_dev || !grad_dev || !m_dev || !v_dev) return fail(BEM_EINVAL, "NULL argument");
    if (n < 1 || step < 1) return fail(BEM_EINVAL, "n >= 1 and step >= 1");
    HIP_CHECK(mlp_adam(n, params_dev, grad_dev, m_dev, v_dev, step, lr, beta1, beta2, eps, stream));
    return BEM_OK;
}

// ------------------------------------------------------------------------------ groups
}  // extern "C"

struct bem_group_s {
    std::vector<bem_operator> ops;
    std::vector<int> ncols;
    int cplx = 0, q = 0;
    int64_t napply = 0;
    size_t ws_bytes = 0;
    std::vector<OpDev> host_ops;
    std::vector<int64_t> prefix, first;
    std::vector<int32_t> ncol32;
    std::vector<const void*> xs;
    std::vector<void*> ys;
    GroupDev dev{};
    bool bound = false;
};

// group workspace: tables (OpDev per apply, x and y pointers, stage prefixes), then per
// apply the one-column scratch (moments, local expansions, chunk sums, transposed products)
static size_t group_layout(bem_group_s& G, char* base, std::vector<OpDev>* ops) {
    Bump b(base);
    const size_t n = (size_t)G.napply;
    OpDev* d_ops = b.take<OpDev>(n);
    const void** d_x = b.take<const void*>(n);
    void** d_y = b.take<void*>(n);
    const size_t nop = G.ops.size();
    int64_t* d_pre = b.take<int64_t>((size_t)kGroupStages * (nop + 1));
    int64_t* d_first = b.take<int64_t>(nop);
    int32_t* d_ncol = b.take<int32_t>(nop);
    if (ops) ops->clear();
    for (size_t i = 0; i < G.ops.size(); ++i) {
        const bem_operator_s& A = *G.ops[i];
        const Plan& p = A.plan;
        for (int c = 0; c < G.ncols[i]; ++c) {
            OpDev o = A.dev;
            o.mom = b.take<char>((size_t)p.ncl * p.q2 * A.scal);
            o.lv = b.take<char>((size_t)p.ncl * p.q2 * A.scal);
            o.partial = b.take<char>(p.ch_t.size() * p.q2 * A.scal);
            o.P = b.take<char>((size_t)p.ptotal * A.scal);
            if (ops) ops->push_back(o);
        }
    }
    if (base) {
        G.dev.ops = d_ops;
        G.dev.x = d_x;
        G.dev.y = d_y;
        G.dev.prefix = d_pre;
        G.dev.first = d_first;
        G.dev.ncol = d_ncol;
    }
    return b.off + 256;
}

extern "C" {

int bem_group_create(int nops, const bem_operator* ops, const int* ncols, bem_group* out, size_t* ws_bytes) {
    if (!ops || !ncols || !out || !ws_bytes || nops < 1) return fail(BEM_EINVAL, "NULL argument or nops < 1");
    bem_group_s* G = new (std::nothrow) bem_group_s;
    if (!G) return fail(BEM_ENOMEM, "host allocation failed");
    for (int i = 0; i < nops; ++i) {
        if (!ops[i] || !ops[i]->assembled || ncols[i] < 1) {
            delete G;
            return fail(BEM_EINVAL, "every operator must be assembled and have >= 1 column");
        }
        if (ops[i]->plan.S.form != 2) {
            delete G;
            return fail(BEM_EUNSUPPORTED, "grouped launches need S^2 spaces");
        }
        const int c = ops[i]->cplx ? 1 : 0, q = ops[i]->plan.P.q;
        if (i == 0) {
            G->cplx = c;
            G->q = q;
        } else if (c != G->cplx || q != G->q) {
            delete G;
            return fail(BEM_EINVAL, "a group's operators share the PDE kind and q");
        }
        G->ops.push_back(ops[i]);
        G->ncols.push_back(ncols[i]);
        G->napply += ncols[i];
    }
    G->ws_bytes = group_layout(*G, nullptr, nullptr);
    *ws_bytes = G->ws_bytes;
    *out = G;
    return BEM_OK;
}

int bem_group_bind(bem_group G, void* ws, size_t ws_bytes, const void* const* x_cols, void* const* y_cols,
                   hipStream_t stream) {
    if (!G || !ws || !x_cols || !y_cols) return fail(BEM_EINVAL, "NULL argument");
    if (ws_bytes < G->ws_bytes) return fail(BEM_ENOMEM, "workspace too small");
    char* base = (char*)(((uintptr_t)ws + 255) / 256 * 256);
    group_layout(*G, base, &G->host_ops);
    const size_t n = (size_t)G->napply;
    G->xs.assign(x_cols, x_cols + n);
    G->ys.assign(y_cols, y_cols + n);
    for (size_t a = 0; a < n; ++a)
        if (!G->xs[a] || !G->ys[a]) return fail(BEM_EINVAL, "NULL column pointer");
    // per operator: the blocks of all its columns in each stage (see group_stage_blocks;
    // every column of an operator has the block counts of the operator's first apply)
    const size_t nop = G->ops.size();
    G->prefix.assign((size_t)kGroupStages * (nop + 1), 0);
    G->first.assign(nop, 0);
    G->ncol32.assign(nop, 0);
    for (size_t i = 0, a = 0; i < nop; a += (size_t)G->ncols[i], ++i) {
        G->first[i] = (int64_t)a;
        G->ncol32[i] = G->ncols[i];
        int64_t nb[kGroupStages];
        group_stage_blocks(G->host_ops[a], G->ncols[i], nb);
        for (int s = 0; s < kGroupStages; ++s) G->prefix[s * (nop + 1) + i + 1] = G->prefix[s * (nop + 1) + i] + nb[s];
    }
    G->dev.napply = G->napply;
    G->dev.nop = (int64_t)nop;
    for (int s = 0; s < kGroupStages; ++s) {
        G->dev.nblocks[s] = G->prefix[s * (nop + 1) + nop];
        if (G->dev.nblocks[s] > 0x7fffffff) return fail(BEM_EUNSUPPORTED, "too many blocks in one launch");
    }
    HIP_CHECK(hipMemcpyAsync((void*)G->dev.ops, G->host_ops.data(), n * sizeof(OpDev), hipMemcpyHostToDevice, stream));
    HIP_CHECK(hipMemcpyAsync((void*)G->dev.x, G->xs.data(), n * sizeof(void*), hipMemcpyHostToDevice, stream));
    HIP_CHECK(hipMemcpyAsync((void*)G->dev.y, G->ys.data(), n * sizeof(void*), hipMemcpyHostToDevice, stream));
    HIP_CHECK(hipMemcpyAsync((void*)G->dev.prefix, G->prefix.data(), G->prefix.size() * 8, hipMemcpyHostToDevice,
                             stream));
    HIP_CHECK(hipMemcpyAsync((void*)G->dev.first, G->first.data(), nop * 8, hipMemcpyHostToDevice, stream));
    HIP_CHECK(hipMemcpyAsync((void*)G->dev.ncol, G->ncol32.data(), nop * 4, hipMemcpyHostToDevice, stream));
    HIP_CHECK(hipStreamSynchronize(stream));
    G->bound = true;
    return BEM_OK;
}

int bem_group_apply(bem_group G, hipStream_t stream) {
    if (!G) return fail(BEM_EINVAL, "NULL argument");
    if (!G->bound) return fail(BEM_EINVAL, "group not bound");
    HIP_CHECK(launch_group_apply(G->dev, G->cplx, G->q, stream));
    return BEM_OK;
}

void bem_group_destroy(bem_group G) { delete G; }

// ------------------------------------------------------------------------------ graphs
}  // extern "C"

struct bem_graph_s {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    ~bem_graph_s() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
    }
};

extern "C" {

int bem_capture_begin(hipStream_t stream) {
    HIP_CHECK(hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal));
    return BEM_OK;
}

int bem_capture_end(hipStream_t stream, bem_graph* out) {
    if (!out) return fail(BEM_EINVAL, "NULL argument");
    bem_graph_s* g = new (std::nothrow) bem_graph_s;
    if (!g) return fail(BEM_ENOMEM, "host allocation failed");
    hipError_t e = hipStreamEndCapture(stream, &g->graph);
    if (e == hipSuccess) e = hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        delete g;
        return fail(BEM_EDEVICE, std::string("graph capture: ") + hipGetErrorString(e));
    }
    *out = g;
    return BEM_OK;
}

int bem_graph_launch(bem_graph g, hipStream_t stream) {
    if (!g || !g->exec) return fail(BEM_EINVAL, "NULL graph");
    HIP_CHECK(hipGraphLaunch(g->exec, stream));
    return BEM_OK;
}

void bem_graph_destroy(bem_graph g) { delete g; }

// ------------------------------------------------------------------------------ exports
int bem_export_near(bem_operator A, int64_t* rowptr, int32_t* col, double* val, hipStream_t stream) {
    if (!A) return fail(BEM_EINVAL, "NULL argument");
    if (A->mx) return fail(BEM_EUNSUPPORTED, "S^1 operators are dense: no near/far split to export");
    if (val && !A->assembled) return fail(BEM_EINVAL, "operator not assembled");
    const Plan& p = A->plan;
    if (rowptr) std::memcpy(rowptr, p.rowptr.data(), p.rowptr.size() * 8);
    if (col) std::memcpy(col, p.col.data(), p.col.size() * 4);
    if (val) {
        // values are stored by row groups; return them in CSR order
        std::vector<char> gv(p.col.size() * A->scal);
        HIP_CHECK(hipMemcpyAsync(gv.data(), A->dev.val, gv.size(), hipMemcpyDeviceToHost, stream));
        HIP_CHECK(hipStreamSynchronize(stream));
        const size_t sc = A->scal;
        for (size_t g = 0; g + 1 < p.rowptr.size(); ++g) {
            const int64_t nc = p.rowptr[g + 1] - p.rowptr[g];
            const int64_t src = p.grp_voff[p.row_grp[g]] + (int64_t)p.row_pos[g] * nc;
            std::memcpy((char*)val + p.rowptr[g] * sc, gv.data() + src * sc, nc * sc);
        }
    }
    return BEM_OK;
}

int bem_export_far(bem_operator A, int64_t* pairs, double* blocks, hipStream_t stream) {
    if (!A) return fail(BEM_EINVAL, "NULL argument");
    if (A->mx) return fail(BEM_EUNSUPPORTED, "S^1 operators are dense: no near/far split to export");
    if (blocks && !A->assembled) return fail(BEM_EINVAL, "operator not assembled");
    const Plan& p = A->plan;
    const size_t nf = p.far_t.size();
    if (pairs)
        for (size_t i = 0; i < nf; ++i) {
            pairs[2 * i] = p.far_t[i];
            pairs[2 * i + 1] = p.far_s[i];
        }
    if (blocks && A->far_eval) return fail(BEM_EUNSUPPORTED, "no stored coupling blocks (far_eval)");
    if (blocks && nf > 0) {
        std::vector<char> K((size_t)p.ktotal * A->scal);
        HIP_CHECK(hipMemcpyAsync(K.data(), A->dev.K, K.size(), hipMemcpyDeviceToHost, stream));
        HIP_CHECK(hipStreamSynchronize(stream));
        const int q2 = p.q2;
        const size_t sc = A->scal;
        for (size_t i = 0; i < nf; ++i) {
            const int t = p.far_t[i], s = p.far_s[i];
            // the pair is stored in the row of its owner; the partner sees the transpose
            const int lo = std::min(t, s), hi = std::max(t, s);
            const int owner = ((lo + hi) & 1) ? lo : hi, other = owner == t ? s : t;
            auto first = p.own_src.begin() + p.own_rowptr[owner], last = p.own_src.begin() + p.own_rowptr[owner + 1];
            const int64_t slot = std::lower_bound(first, last, other) - first;
            const char* rows = K.data() + p.koff[owner] * sc;
            for (int a = 0; a < q2; ++a)
                for (int b = 0; b < q2; ++b) {
                    const int ra = owner == t ? a : b, cb = owner == t ? b : a;
                    std::memcpy((char*)blocks + ((i * q2 + a) * q2 + b) * sc,
                                rows + ((int64_t)ra * p.krs[owner] + slot * q2 + cb) * sc, sc);
                }
        }
    }
    return BEM_OK;
}

int bem_write_vtk(bem_space s, const void* rho_host, int64_t ldr, int nrhs, int nsub, const char* path) {
    if (!s || !path || (nrhs > 0 && !rho_host)) return fail(BEM_EINVAL, "NULL argument");
    if (s->mx) return fail(BEM_EUNSUPPORTED, "VTK output: scalar spaces only");
    if (nrhs < 0 || nrhs > 64) return fail(BEM_EINVAL, "nrhs must lie in [0, 64]");
    if (nsub < 1 || nsub > 64) return fail(BEM_EINVAL, "nsub must lie in [1, 64]");
    const SpaceDesc& S = s->S;
    if (nrhs > 0 && ldr < S.nglob) return fail(BEM_EINVAL, "ldr must be >= N");
    const bool cplx = S.ker.pde == PDE_HELMHOLTZ;
    const int32_t* glue = s->glue ? s->glue->glue.data() : nullptr;  // S^0: local -> global
    const int np1 = nsub + 1;
    const int64_t npe = (int64_t)np1 * np1;
    const int64_t npts = S.nelem * npe, ncell = S.nelem * nsub * nsub;
    if (npts > ((int64_t)1 << 31)) return fail(BEM_EINVAL, "too many output points");
    FILE* fp = std::fopen(path, "w");
    if (!fp) return fail(BEM_EINVAL, std::string("cannot create ") + path);
    std::vector<double> kap((size_t)npts);
    std::vector<double> val((size_t)npts * (cplx ? 2 : 1) * (size_t)std::max(nrhs, 1));
    std::fprintf(fp, "# vtk DataFile Version 3.0\nboundary density\nASCII\nDATASET UNSTRUCTURED_GRID\n");
    std::fprintf(fp, "POINTS %lld double\n", (long long)npts);
    const double fd = 1e-6;  // parameter step of the central differences of the surface element
    int64_t k = 0;
    for (int64_t e = 0; e < S.nelem; ++e) {
        const int i2 = (int)(e % S.nel), i1 = (int)((e / S.nel) % S.nel), f = (int)(e / ((int64_t)S.nel * S.nel));
        const int ca = basis_class(s->bt, i1), cb = basis_class(s->bt, i2);
        for (int a = 0; a <= nsub; ++a)
            for (int b = 0; b <= nsub; ++b, ++k) {
                const double u1 = (double)a / nsub, u2 = (double)b / nsub;
                const double ps = (i1 + u1) * S.h, pt = (i2 + u2) * S.h;
                double x[3], xp[3], xm[3], yp[3], ym[3];
                patch_point(S.geom, f, ps, pt, x);
                patch_point(S.geom, f, ps + fd, pt, xp);
                patch_point(S.geom, f, ps - fd, pt, xm);
                patch_point(S.geom, f, ps, pt + fd, yp);
                patch_point(S.geom, f, ps, pt - fd, ym);
                double ds[3], dt[3];
                for (int c = 0; c < 3; ++c) {
                    ds[c] = (xp[c] - xm[c]) / (2 * fd);
                    dt[c] = (yp[c] - ym[c]) / (2 * fd);
                }
                const double nx = ds[1] * dt[2] - ds[2] * dt[1], ny = ds[2] * dt[0] - ds[0] * dt[2],
                             nz = ds[0] * dt[1] - ds[1] * dt[0];
                kap[k] = std::sqrt(nx * nx + ny * ny + nz * nz);
                std::fprintf(fp, "%.17g %.17g %.17g\n", x[0], x[1], x[2]);
                for (int r = 0; r < nrhs; ++r) {
                    double re = 0.0, im = 0.0;
                    for (int l1 = 0; l1 <= S.d; ++l1)
                        for (int l2 = 0; l2 <= S.d; ++l2) {
                            const double phi = basis_eval(s->bt, ca, l1, u1) * basis_eval(s->bt, cb, l2, u2);
                            const int64_t loc = dof_id(S, f, i1 * S.r + l1, i2 * S.r + l2);
                            const int64_t g = (glue ? glue[loc] : loc) + (int64_t)r * ldr;
                            if (cplx) {
                                re += phi * ((const double*)rho_host)[2 * g];
                                im += phi * ((const double*)rho_host)[2 * g + 1];
                            } else {
                                re += phi * ((const double*)rho_host)[g];
                            }
                        }
                    // 2-form lifting: the density on the surface is rho_hat / kappa; 0-form: rho_hat
                    const double sc = S.form == 0 ? 1.0 : 1.0 / kap[k];
                    const size_t o = ((size_t)r * npts + k) * (cplx ? 2 : 1);
                    val[o] = re * sc;
                    if (cplx) val[o + 1] = im * sc;
                }
            }
    }
    std::fprintf(fp, "CELLS %lld %lld\n", (long long)ncell, (long long)ncell * 5);
    for (int64_t e = 0; e < S.nelem; ++e)
        for (int a = 0; a < nsub; ++a)
            for (int b = 0; b < nsub; ++b) {
                const int64_t p0 = e * npe + (int64_t)a * np1 + b;
                std::fprintf(fp, "4 %lld %lld %lld %lld\n", (long long)p0, (long long)(p0 + np1),
                             (long long)(p0 + np1 + 1), (long long)(p0 + 1));
            }
    std::fprintf(fp, "CELL_TYPES %lld\n", (long long)ncell);
    for (int64_t c = 0; c < ncell; ++c) std::fprintf(fp, "9\n");
    std::fprintf(fp, "POINT_DATA %lld\nSCALARS kappa double 1\nLOOKUP_TABLE default\n", (long long)npts);
    for (int64_t p = 0; p < npts; ++p) std::fprintf(fp, "%.17g\n", kap[p]);
    for (int r = 0; r < nrhs; ++r)
        for (int part = 0; part < (cplx ? 2 : 1); ++part) {
            std::fprintf(fp, "SCALARS rho%s_%d double 1\nLOOKUP_TABLE default\n", cplx ? (part ? "_im" : "_re") : "", r);
            for (int64_t p = 0; p < npts; ++p)
                std::fprintf(fp, "%.17g\n", val[((size_t)r * npts + p) * (cplx ? 2 : 1) + part]);
        }
    const bool ok = std::fclose(fp) == 0;
    return ok ? BEM_OK : fail(BEM_EINVAL, std::string("write failed: ") + path);
}

int bem_eval_potential_h2(bem_operator A, const double* pts_dev, int64_t npts, const void* rho_dev, int64_t ldr,
                          int nrhs, void* u_dev, int64_t ldu, double eta, hipStream_t stream) {
    if (!A || !rho_dev || (npts > 0 && (!pts_dev || !u_dev))) return fail(BEM_EINVAL, "NULL argument");
    if (A->mx) return fail(BEM_EUNSUPPORTED, "S^1 operators have no cluster tree: use bem_eval_potential");
    if (!A->assembled) return fail(BEM_EINVAL, "operator not assembled");
    if (nrhs < 1 || npts < 0) return fail(BEM_EINVAL, "nrhs must be >= 1 and npts >= 0");
    if (!(eta >= 0.0) || !std::isfinite(eta)) return fail(BEM_EINVAL, "eta must be finite and >= 0");
    if (npts == 0) return BEM_OK;
    const int64_t N = A->info.ndof;
    if (ldr < N || ldu < npts) return fail(BEM_EINVAL, "leading dimension too small");
    if (npts > ((int64_t)1 << 33)) return fail(BEM_EINVAL, "too many points");
    const Gauss8 g8 = gauss8();
    for (int r = 0; r < nrhs; ++r) {
        const char* rho = (const char*)rho_dev + (size_t)r * ldr * A->scal;
        if (A->dev.S.form == 0) {  // the moments of the local functions
            HIP_CHECK(launch_glue_gather(A->dev.S, A->cplx ? 1 : 0, rho, A->dev.xl, stream));
            HIP_CHECK(launch_moments(A->dev, A->dev.xl, stream));
        } else {
            HIP_CHECK(launch_moments(A->dev, rho, stream));
        }
        HIP_CHECK(launch_potential_tree(A->dev, g8, eta, pts_dev, npts, rho, (char*)u_dev + (size_t)r * ldu * A->scal,
                                        stream));
    }
    return BEM_OK;
}

int bem_export_moments(bem_operator A, const void* x_dev, double* mom_host, hipStream_t stream) {
    if (!A || !x_dev || !mom_host) return fail(BEM_EINVAL, "NULL argument");
    if (A->mx) return fail(BEM_EUNSUPPORTED, "S^1 operators have no cluster tree");
    if (!A->assembled) return fail(BEM_EINVAL, "operator not assembled");
    if (A->dev.S.form == 0) {
        HIP_CHECK(launch_glue_gather(A->dev.S, A->cplx ? 1 : 0, x_dev, A->dev.xl, stream));
        HIP_CHECK(launch_moments(A->dev, A->dev.xl, stream));
    } else {
        HIP_CHECK(launch_moments(A->dev, x_dev, stream));
    }
    HIP_CHECK(hipMemcpyAsync(mom_host, A->dev.mom, (size_t)A->plan.ncl * A->plan.q2 * A->scal, hipMemcpyDeviceToHost,
                             stream));
    HIP_CHECK(hipStreamSynchronize(stream));
    return BEM_OK;
}

}  // extern "C"
