// Driver of the oracle's C API for the sanitizer build (address + undefined behaviour):
// small dense and H^2 operators on analytic and NURBS geometries, Laplace and Helmholtz,
// products, GMRES, block-Jacobi, the tree potential.  Exit status 0 when every call succeeds.
#include <cstdint>
#include <cstdio>
#include <vector>

extern "C" {
const char* orc_last_error();
int orc_space_new(int, const double*, int, int, double, double, int, int, int, void**);
int orc_space_new_nurbs(int, const int*, const double*, const double*, int, double, double, int, int, int, void**);
void orc_space_free(void*);
int64_t orc_space_ndof(void*);
int orc_dense(void*, int, int, double*);
int orc_rhs(void*, int, const double*, int, int, double*);
int orc_potential(void*, int, const double*, int64_t, const double*, double*);
int orc_h2_new(void*, int, double, int, int, int, int, double, void**);
void orc_h2_free(void*);
int orc_h2_apply(void*, const double*, double*, int);
int orc_h2_potential(void*, const double*, int64_t, const double*, double, double*);
int orc_h2_gmres(void*, const double*, double*, double, int, int, double*);
int orc_bj_new(void*, int, void**);
void orc_bj_free(void*);
int orc_bj_apply(void*, const double*, double*);
}

static int check(int rc, const char* what) {
    if (rc != 0) std::fprintf(stderr, "%s failed: %s\n", what, orc_last_error());
    return rc;
}

static int run_space(void* S, int cplx, int leaf) {
    const int64_t N = orc_space_ndof(S);
    const int sc = cplx ? 2 : 1;
    std::vector<double> A((size_t)N * N * sc), b((size_t)N * sc), x((size_t)N * sc), y((size_t)N * sc);
    if (check(orc_dense(S, 4, 4, A.data()), "dense")) return 1;
    const double x0[3] = {0.1, -0.2, 0.15};
    if (check(orc_rhs(S, 0, x0, 1, 4, b.data()), "rhs")) return 1;
    void* H = nullptr;
    if (check(orc_h2_new(S, 3, 1.6, leaf, 4, 4, 1, 0.0, &H), "h2_new")) return 1;
    int rc = check(orc_h2_apply(H, b.data(), y.data(), 1), "h2_apply");
    double st[3] = {0, 0, 0};
    rc |= check(orc_h2_gmres(H, b.data(), x.data(), 1e-8, 10, 200, st), "h2_gmres");
    void* BJ = nullptr;
    rc |= check(orc_bj_new(H, 8, &BJ), "bj_new");
    if (BJ) {
        rc |= check(orc_bj_apply(BJ, b.data(), y.data()), "bj_apply");
        orc_bj_free(BJ);
    }
    const double pts[6] = {2.0, 0.1, 0.3, -0.4, 3.0, 0.5};
    std::vector<double> u(2 * sc);
    rc |= check(orc_h2_potential(H, x.data(), 2, pts, 1.6, u.data()), "h2_potential");
    rc |= check(orc_potential(S, 4, x.data(), 2, pts, u.data()), "potential");
    orc_h2_free(H);
    return rc;
}

int main() {
    int rc = 0;
    for (int pde = 0; pde < 2; ++pde) {
        void* S = nullptr;
        if (check(orc_space_new(0, nullptr, 0, pde, pde ? 2.0 : 0.0, 0.0, 1, 1, 1, &S), "space")) return 1;
        rc |= run_space(S, pde, 1);
        orc_space_free(S);
        const double tor[2] = {1.0, 0.4};
        if (check(orc_space_new(2, tor, 2, pde, pde ? 1.5 : 0.0, 0.2, 2, 1, 0, &S), "space torus")) return 1;
        rc |= run_space(S, pde, 0);
        orc_space_free(S);
    }
    // one biquadratic rational patch (a quarter of a cylinder-like surface) and a flat one
    const int meta[8] = {2, 2, 3, 3, 1, 1, 2, 2};
    const double knots[6 + 6 + 4 + 4] = {0, 0, 0, 1, 1, 1, 0, 0, 0, 1, 1, 1, 0, 0, 1, 1, 0, 0, 1, 1};
    std::vector<double> cw;
    const double w[3] = {1.0, 0.7071067811865476, 1.0};
    const double px[3] = {1, 1, 0}, py[3] = {0, 1, 1};
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) cw.insert(cw.end(), {px[i], py[i], 0.5 * j, w[i]});
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j) cw.insert(cw.end(), {3.0 + i, 0.0 + j, 0.0, 1.0});
    void* S = nullptr;
    if (check(orc_space_new_nurbs(2, meta, knots, cw.data(), 0, 0.0, 0.0, 1, 1, 1, &S), "space nurbs")) return 1;
    rc |= run_space(S, 0, 1);
    orc_space_free(S);
    std::printf("oracle driver: %s\n", rc ? "FAILED" : "ok");
    return rc;
}
