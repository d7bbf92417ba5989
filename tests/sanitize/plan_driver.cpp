// Driver of the library's host planning code (cluster tree, admissibility, block partition,
// near pattern, row groups, touching pairs) for the sanitizer build: plans of analytic and
// NURBS geometries at several levels, degrees, leaf levels and admissibility parameters.
#include <cstdio>
#include <string>
#include <vector>

#include "../../paper_1906_00785_amd/csrc/bem_plan.h"

using namespace bem;

static SpaceDesc space(const GeomDesc& g, int pde, int d, int L) {
    SpaceDesc S{};
    S.geom = g;
    S.ker.pde = pde;
    S.ker.kre = pde ? 3.0 : 0.0;
    S.d = d;
    S.r = 1;
    S.L = L;
    S.nel = 1 << L;
    S.nb = d + 1 + (S.nel - 1);
    S.nelem = (int64_t)g.npatch * S.nel * S.nel;
    S.ndof = (int64_t)g.npatch * S.nb * S.nb;
    S.h = 1.0 / S.nel;
    return S;
}

int main() {
    int bad = 0;
    std::vector<GeomDesc> geoms;
    GeomDesc g{};
    g.kind = GEOM_SPHERE6; g.npatch = 6; g.a = g.b = g.c = 1.0;
    geoms.push_back(g);
    g.kind = GEOM_ELLIPSOID6; g.a = 0.7; g.b = 1.2; g.c = 1.6;
    geoms.push_back(g);
    g.kind = GEOM_TORUS16; g.npatch = 16; g.a = 1.0; g.b = 0.4;
    geoms.push_back(g);
    g.kind = GEOM_FLAT1; g.npatch = 1; g.a = 2.0;
    geoms.push_back(g);
    // a flat NURBS patch: degrees 1, 1, four control points, unit weights
    static const double tab[] = {1, 1, 1, 2, 2, 7, 15, 0, 0, 1, 1, 0, 0, 1, 1,
                                 0, 0, 0, 1, 0, 1, 0, 1, 1, 0, 0, 1, 1, 1, 0, 1};
    g = GeomDesc{};
    g.kind = GEOM_NURBS; g.npatch = 1; g.a = g.b = g.c = 1.0; g.tab_host = tab;
    geoms.push_back(g);
    for (const GeomDesc& G : geoms)
        for (int L = 0; L <= 3; ++L)
            for (int d = 0; d <= 2; ++d)
                for (int leaf = 0; leaf <= L; ++leaf)
                    for (double eta : {0.0, 1.6}) {
                        H2Params P;
                        P.q = 3 + (L + d) % 3;
                        P.eta = eta;
                        P.leaf = leaf;
                        P.kadm = (L & 1) ? 4.0 : 0.0;
                        Plan plan;
                        std::string err;
                        if (!build_plan(space(G, L & 1, d, L), P, plan, err)) {
                            std::fprintf(stderr, "plan failed (kind %d L %d d %d leaf %d): %s\n", G.kind, L, d, leaf,
                                         err.c_str());
                            bad = 1;
                        }
                    }
    std::printf("plan driver: %s\n", bad ? "FAILED" : "ok");
    return bad;
}
