// Host plan of the H^2 operator (see bem_plan.h).
#include "bem_plan.h"

#include <algorithm>
#include <cmath>
#include <array>
#include <map>
#include <unordered_map>

namespace bem {

// Legendre P_n and its derivative at z by the three-term recurrence
static void legendre_pd(int n, double z, double& p, double& dp) {
    double pm1 = 1.0, pc = z;
    if (n == 0) {
        p = 1.0;
        dp = 0.0;
        return;
    }
    for (int k = 1; k < n; ++k) {
        const double pn = ((2 * k + 1) * z * pc - k * pm1) / (k + 1);
        pm1 = pc;
        pc = pn;
    }
    p = pc;
    dp = n * (pm1 - z * pc) / (1.0 - z * z);
}

void gauss_legendre01(int n, std::vector<double>& x, std::vector<double>& w) {
    x.assign(n, 0.0);
    w.assign(n, 0.0);
    for (int k = 0; k < n; ++k) {
        // k-th root from the largest down, initial guess from the asymptotic formula
        double z = std::cos(kPi * (4.0 * k + 3.0) / (4.0 * n + 2.0));
        double p, dp;
        for (int it = 0; it < 100; ++it) {
            legendre_pd(n, z, p, dp);
            const double step = p / dp;
            z -= step;
            if (std::fabs(step) <= 1e-17) break;
        }
        legendre_pd(n, z, p, dp);
        // node on [0,1] ascending: the k-th largest root maps to position n-1-k
        x[n - 1 - k] = 0.5 + 0.5 * z;
        w[n - 1 - k] = 1.0 / ((1.0 - z * z) * dp * dp);
    }
}

// Cox-de Boor recursion carried out on polynomials of the element-local coordinate.
void bspline_local_polys(int d, int r, int L, std::vector<double>& out) {
    const int nel = 1 << L;
    std::vector<double> kn;
    for (int i = 0; i <= d; ++i) kn.push_back(0.0);
    for (int k = 1; k < nel; ++k)
        for (int t = 0; t < r; ++t) kn.push_back((double)k / nel);
    for (int i = 0; i <= d; ++i) kn.push_back(1.0);
    const double h = 1.0 / nel;
    out.assign((size_t)nel * (d + 1) * (d + 1), 0.0);
    for (int i = 0; i < nel; ++i) {
        const int span = d + i * r;
        const double x0 = (double)i / nel;  // x = x0 + h * xhat
        // N[j - (span - p)] holds the polynomial of N_j^p for j = span-p .. span
        std::vector<std::vector<double>> N(1, std::vector<double>(d + 1, 0.0));
        N[0][0] = 1.0;
        for (int p = 1; p <= d; ++p) {
            std::vector<std::vector<double>> M(p + 1, std::vector<double>(d + 1, 0.0));
            for (int jj = 0; jj <= p; ++jj) {
                const int j = span - p + jj;
                // left term: (x - kn[j]) / (kn[j+p] - kn[j]) * N_j^{p-1}
                if (jj >= 1) {
                    const double den = kn[j + p] - kn[j];
                    if (den > 0.0) {
                        const std::vector<double>& a = N[jj - 1];
                        const double c0 = (x0 - kn[j]) / den, c1 = h / den;
                        for (int k = 0; k <= d; ++k) {
                            M[jj][k] += c0 * a[k];
                            if (k + 1 <= d) M[jj][k + 1] += c1 * a[k];
                        }
                    }
                }
                // right term: (kn[j+p+1] - x) / (kn[j+p+1] - kn[j+1]) * N_{j+1}^{p-1}
                if (jj <= p - 1) {
                    const double den = kn[j + p + 1] - kn[j + 1];
                    if (den > 0.0) {
                        const std::vector<double>& a = N[jj];
                        const double c0 = (kn[j + p + 1] - x0) / den, c1 = -h / den;
                        for (int k = 0; k <= d; ++k) {
                            M[jj][k] += c0 * a[k];
                            if (k + 1 <= d) M[jj][k + 1] += c1 * a[k];
                        }
                    }
                }
            }
            N.swap(M);
        }
        // local basis l is B-spline i*r + l = span - d + l
        for (int l = 0; l <= d; ++l)
            for (int k = 0; k <= d; ++k) out[((size_t)i * (d + 1) + l) * (d + 1) + k] = N[l][k];
    }
}

static double poly_eval(const double* c, int d, double x) {
    double v = c[d];
    for (int k = d - 1; k >= 0; --k) v = v * x + c[k];
    return v;
}

double lagrange_bary(const std::vector<double>& xs, int a, double y) {
    const int q = (int)xs.size();
    for (int b = 0; b < q; ++b)
        if (y == xs[b]) return b == a ? 1.0 : 0.0;
    // barycentric weights of arbitrary nodes: w_b = 1 / prod_{c != b} (x_b - x_c)
    double num = 0.0, den = 0.0;
    for (int b = 0; b < q; ++b) {
        double wb = 1.0;
        for (int c = 0; c < q; ++c)
            if (c != b) wb /= (xs[b] - xs[c]);
        const double t = wb / (y - xs[b]);
        den += t;
        if (b == a) num = t;
    }
    return num / den;
}

static double dist(const double* a, const double* b) {
    const double dx = a[0] - b[0], dy = a[1] - b[1], dz = a[2] - b[2];
    return std::sqrt(dx * dx + dy * dy + dz * dz);
}

namespace {

struct ClusterId {
    int lev, f, i, j;
};

struct Builder {
    Plan& p;
    explicit Builder(Plan& pl) : p(pl) {}

    int64_t cidx(int lev, int f, int i, int j) const {
        const int64_t n = (int64_t)1 << lev;
        return p.lev_off[lev] + ((int64_t)f * n + i) * n + j;
    }
    ClusterId cid(int64_t c) const {
        int lev = 0;
        while (c >= p.lev_off[lev + 1]) ++lev;
        const int64_t loc = c - p.lev_off[lev];
        const int n = 1 << lev;
        ClusterId r;
        r.lev = lev;
        r.j = (int)(loc % n);
        r.i = (int)((loc / n) % n);
        r.f = (int)(loc / ((int64_t)n * n));
        return r;
    }

    // ball around gamma(midpoint) covering gamma on a 9x9 grid of the cluster square
    void balls() {
        p.ball.assign(4 * p.ncl, 0.0);
        for (int64_t c = 0; c < p.ncl; ++c) {
            const ClusterId C = cid(c);
            const double w = 1.0 / (double)(1 << C.lev);
            double* B = &p.ball[4 * c];
            patch_point(p.S.geom, C.f, (C.i + 0.5) * w, (C.j + 0.5) * w, B);
            double rad = 0.0;
            for (int a = 0; a <= 8; ++a)
                for (int b = 0; b <= 8; ++b) {
                    double x[3];
                    patch_point(p.S.geom, C.f, (C.i + a / 8.0) * w, (C.j + b / 8.0) * w, x);
                    rad = std::max(rad, dist(x, B));
                }
            B[3] = rad;
        }
    }

    bool admissible(int64_t t, int64_t s) const {
        const double* A = &p.ball[4 * t];
        const double* B = &p.ball[4 * s];
        const double gap = dist(A, B) - A[3] - B[3];
        if (!(gap > 0.0)) return false;
        const double lhs = 2.0 * std::max(A[3], B[3]);
        const double rhs = p.P.eta * gap;
        if (std::fabs(lhs - rhs) <= 1e-12 * gap) return false;  // ties are inadmissible
        if (!(lhs <= rhs)) return false;
        // the interpolation resolves the oscillating kernel only while |kappa| times the
        // larger diameter stays below kadm (ties inadmissible)
        if (p.P.kadm > 0.0 && p.S.ker.pde == PDE_HELMHOLTZ) {
            const double kd = std::hypot(p.S.ker.kre, p.S.ker.kim) * lhs;
            if (std::fabs(kd - p.P.kadm) <= 1e-12 * p.P.kadm || kd > p.P.kadm) return false;
        }
        return true;
    }

    void partition(std::vector<std::pair<int32_t, int32_t>>& far,
                   std::vector<std::pair<int32_t, int32_t>>& nearp) {
        std::vector<std::pair<int64_t, int64_t>> stack;
        for (int f = p.S.geom.npatch - 1; f >= 0; --f)
            for (int g = p.S.geom.npatch - 1; g >= 0; --g) stack.push_back({cidx(0, f, 0, 0), cidx(0, g, 0, 0)});
        while (!stack.empty()) {
            auto pr = stack.back();
            stack.pop_back();
            if (admissible(pr.first, pr.second)) {
                far.push_back({(int32_t)pr.first, (int32_t)pr.second});
                continue;
            }
            const ClusterId A = cid(pr.first), B = cid(pr.second);
            if (A.lev == p.leaf) {
                nearp.push_back({(int32_t)(pr.first - p.lev_off[p.leaf]), (int32_t)(pr.second - p.lev_off[p.leaf])});
                continue;
            }
            for (int a = 0; a < 4; ++a)
                for (int b = 0; b < 4; ++b)
                    stack.push_back({cidx(A.lev + 1, A.f, 2 * A.i + (a >> 1), 2 * A.j + (a & 1)),
                                     cidx(B.lev + 1, B.f, 2 * B.i + (b >> 1), 2 * B.j + (b & 1))});
        }
        std::sort(far.begin(), far.end());
        std::sort(nearp.begin(), nearp.end());
    }

    // leaf-local index of the leaf containing element (f, i1, i2)
    int32_t leaf_of_elem(int f, int i1, int i2) const {
        return (int32_t)(((int64_t)f * p.nleaf1 + i1 / p.m) * p.nleaf1 + i2 / p.m);
    }

    // corner vertex ids by merging coincident physical points
    void vertex_ids() {
        const SpaceDesc& S = p.S;
        p.vid.assign(4 * S.nelem, -1);
        const double cell = 1e-7 * S.h;
        const double tol = 1e-10 * S.h;
        std::unordered_map<uint64_t, std::vector<int32_t>> grid;
        std::vector<double> pts;
        auto key = [&](int64_t a, int64_t b, int64_t c) {
            return ((uint64_t)(a & 0x1FFFFF) << 42) | ((uint64_t)(b & 0x1FFFFF) << 21) | (uint64_t)(c & 0x1FFFFF);
        };
        for (int64_t e = 0; e < S.nelem; ++e) {
            const int i2 = (int)(e % S.nel), i1 = (int)((e / S.nel) % S.nel), f = (int)(e / ((int64_t)S.nel * S.nel));
            for (int c = 0; c < 4; ++c) {
                const int c1 = c >> 1, c2 = c & 1;
                double x[3];
                patch_point(S.geom, f, (i1 + c1) * S.h, (i2 + c2) * S.h, x);
                const int64_t q0 = (int64_t)std::floor(x[0] / cell), q1 = (int64_t)std::floor(x[1] / cell),
                              q2 = (int64_t)std::floor(x[2] / cell);
                int32_t found = -1;
                for (int da = -1; da <= 1 && found < 0; ++da)
                    for (int db = -1; db <= 1 && found < 0; ++db)
                        for (int dc = -1; dc <= 1 && found < 0; ++dc) {
                            auto it = grid.find(key(q0 + da, q1 + db, q2 + dc));
                            if (it == grid.end()) continue;
                            for (int32_t id : it->second)
                                if (dist(&pts[3 * id], x) <= tol) {
                                    found = id;
                                    break;
                                }
                        }
                if (found < 0) {
                    found = (int32_t)(pts.size() / 3);
                    pts.insert(pts.end(), x, x + 3);
                    grid[key(q0, q1, q2)].push_back(found);
                }
                p.vid[4 * e + c] = found;
            }
        }
    }

    int corner_vid(int64_t e, int k, double a, double b) const {
        double o1, o2;
        d4_apply(k, a, b, o1, o2);
        return p.vid[4 * e + ((int)o1) * 2 + (int)o2];
    }

    // kind of the touching pair (e, e2) (elements sharing a vertex) and the symmetries of the
    // unit square that move the common vertex (and edge) to the origin (and the edge t = 0)
    bool classify(int64_t e, int64_t e2, int& type, int& k1, int& k2, std::string& err) const {
        int shared = 0;
        for (int a = 0; a < 4; ++a)
            for (int b = 0; b < 4; ++b)
                if (p.vid[4 * e + a] == p.vid[4 * e2 + b]) ++shared;
        k1 = k2 = 0;
        if (e == e2) {
            type = PT_IDENTICAL;
            return true;
        }
        if (shared != 2 && shared != 1) {
            err = "distinct elements share more than an edge";
            return false;
        }
        type = shared == 2 ? PT_EDGE : PT_VERTEX;
        for (int a = 0; a < 8; ++a)
            for (int b = 0; b < 8; ++b) {
                if (corner_vid(e, a, 0, 0) != corner_vid(e2, b, 0, 0)) continue;
                if (type == PT_EDGE && corner_vid(e, a, 0, 1) != corner_vid(e2, b, 0, 1)) continue;
                k1 = a;
                k2 = b;
                return true;
            }
        err = "no symmetry aligns a shared edge/vertex (matching condition)";
        return false;
    }

    // every touching element pair (both orders, e1 == e2 included), sorted
    bool touching_elements(std::vector<int64_t>& pairs, std::vector<int32_t>& info, std::string& err) const {
        const SpaceDesc& S = p.S;
        int32_t nv = 0;
        for (int32_t v : p.vid) nv = std::max(nv, v + 1);
        std::vector<std::vector<int64_t>> vel(nv);
        for (int64_t e = 0; e < S.nelem; ++e)
            for (int c = 0; c < 4; ++c) {
                auto& L = vel[p.vid[4 * e + c]];
                if (L.empty() || L.back() != e) L.push_back(e);
            }
        std::vector<int64_t> nb;
        pairs.clear();
        info.clear();
        for (int64_t e = 0; e < S.nelem; ++e) {
            nb.clear();
            for (int c = 0; c < 4; ++c)
                for (int64_t e2 : vel[p.vid[4 * e + c]]) nb.push_back(e2);
            std::sort(nb.begin(), nb.end());
            nb.erase(std::unique(nb.begin(), nb.end()), nb.end());
            for (int64_t e2 : nb) {
                int type, k1, k2;
                if (!classify(e, e2, type, k1, k2, err)) return false;
                pairs.push_back(e);
                pairs.push_back(e2);
                info.push_back(type | k1 << 4 | k2 << 8);
            }
        }
        return true;
    }

    bool touching(bool& ok, std::string& err) {
        const SpaceDesc& S = p.S;
        // vertex -> elements
        int32_t nv = 0;
        for (int32_t v : p.vid) nv = std::max(nv, v + 1);
        std::vector<std::vector<int64_t>> vel(nv);
        for (int64_t e = 0; e < S.nelem; ++e)
            for (int c = 0; c < 4; ++c) {
                auto& L = vel[p.vid[4 * e + c]];
                if (L.empty() || L.back() != e) L.push_back(e);
            }
        const int64_t nnear = (int64_t)p.near_t.size();
        std::vector<std::vector<std::array<int32_t, 5>>> lists(nnear);
        std::vector<int64_t> nb;
        for (int64_t e = 0; e < S.nelem; ++e) {
            nb.clear();
            for (int c = 0; c < 4; ++c)
                for (int64_t e2 : vel[p.vid[4 * e + c]]) nb.push_back(e2);
            std::sort(nb.begin(), nb.end());
            nb.erase(std::unique(nb.begin(), nb.end()), nb.end());
            const int i2 = (int)(e % S.nel), i1 = (int)((e / S.nel) % S.nel), f = (int)(e / ((int64_t)S.nel * S.nel));
            const int32_t lt = leaf_of_elem(f, i1, i2);
            for (int64_t e2 : nb) {
                const int j2 = (int)(e2 % S.nel), j1 = (int)((e2 / S.nel) % S.nel), g = (int)(e2 / ((int64_t)S.nel * S.nel));
                const int32_t ls = leaf_of_elem(g, j1, j2);
                // locate the near leaf pair (lt, ls)
                auto lo = p.near_s.begin() + p.near_rowptr[lt], hi = p.near_s.begin() + p.near_rowptr[lt + 1];
                auto it = std::lower_bound(lo, hi, ls);
                if (it == hi || *it != ls) {
                    err = "touching elements in an admissible block (geometry violates the matching condition?)";
                    ok = false;
                    return false;
                }
                const int64_t lp = it - p.near_s.begin();
                int type, k1, k2;
                if (!classify(e, e2, type, k1, k2, err)) {
                    ok = false;
                    return false;
                }
                const int et = (i1 % p.m) * p.m + (i2 % p.m);
                const int es = (j1 % p.m) * p.m + (j2 % p.m);
                lists[lp].push_back({et, es, type, k1, k2});
            }
        }
        p.touch_rowptr.assign(nnear + 1, 0);
        p.touch.clear();
        for (int64_t lp = 0; lp < nnear; ++lp) {
            std::sort(lists[lp].begin(), lists[lp].end());
            for (auto& t : lists[lp]) p.touch.insert(p.touch.end(), t.begin(), t.end());
            p.touch_rowptr[lp + 1] = (int32_t)(p.touch.size() / 5);
        }
        ok = true;
        return true;
    }

    // union over near leaf pairs (tau, sigma) of dofs(tau) x dofs(sigma)
    void near_pattern() {
        const SpaceDesc& S = p.S;
        const int64_t N = S.ndof;
        p.rowptr.assign(N + 1, 0);
        p.col.clear();
        std::vector<int64_t> mark(N, -1);
        std::vector<int32_t> cols;
        const int stride = p.m * S.r;
        for (int64_t g = 0; g < N; ++g) {
            const int j2 = (int)(g % S.nb), j1 = (int)((g / S.nb) % S.nb), f = (int)(g / ((int64_t)S.nb * S.nb));
            int lo1, hi1, lo2, hi2;
            leaves_of_basis(p, j1, lo1, hi1);
            leaves_of_basis(p, j2, lo2, hi2);
            cols.clear();
            for (int a = lo1; a <= hi1; ++a)
                for (int b = lo2; b <= hi2; ++b) {
                    const int32_t lt = (int32_t)(((int64_t)f * p.nleaf1 + a) * p.nleaf1 + b);
                    for (int32_t k = p.near_rowptr[lt]; k < p.near_rowptr[lt + 1]; ++k) {
                        const int32_t ls = p.near_s[k];
                        const int sb = ls % p.nleaf1, sa = (ls / p.nleaf1) % p.nleaf1, sf = ls / (p.nleaf1 * p.nleaf1);
                        for (int u = 0; u < p.nloc; ++u)
                            for (int v = 0; v < p.nloc; ++v) {
                                const int64_t h = dof_id(S, sf, sa * stride + u, sb * stride + v);
                                if (mark[h] != g) {
                                    mark[h] = g;
                                    cols.push_back((int32_t)h);
                                }
                            }
                    }
                }
            std::sort(cols.begin(), cols.end());
            p.col.insert(p.col.end(), cols.begin(), cols.end());
            p.rowptr[g + 1] = (int64_t)p.col.size();
        }
    }

    // rows with the same patch and leaf ranges share their columns
    void near_groups() {
        const SpaceDesc& S = p.S;
        const int64_t N = S.ndof;
        std::map<std::array<int, 5>, int32_t> open;  // key -> open group
        std::vector<std::vector<int32_t>> rows;
        p.row_grp.assign(N, 0);
        p.row_pos.assign(N, 0);
        for (int64_t g = 0; g < N; ++g) {
            const int j2 = (int)(g % S.nb), j1 = (int)((g / S.nb) % S.nb), f = (int)(g / ((int64_t)S.nb * S.nb));
            std::array<int, 5> key;
            key[0] = f;
            leaves_of_basis(p, j1, key[1], key[2]);
            leaves_of_basis(p, j2, key[3], key[4]);
            auto it = open.find(key);
            if (it == open.end() || (int)rows[it->second].size() >= kGroupRows) {
                rows.emplace_back();
                open[key] = (int32_t)(rows.size() - 1);
                it = open.find(key);
            }
            p.row_grp[g] = it->second;
            p.row_pos[g] = (int32_t)rows[it->second].size();
            rows[it->second].push_back((int32_t)g);
        }
        const size_t ng = rows.size();
        p.grp_rowptr.assign(ng + 1, 0);
        p.grp_voff.assign(ng + 1, 0);
        p.grp_rows.clear();
        for (size_t G = 0; G < ng; ++G) {
            p.grp_rows.insert(p.grp_rows.end(), rows[G].begin(), rows[G].end());
            p.grp_rowptr[G + 1] = (int64_t)p.grp_rows.size();
            const int64_t first = rows[G][0];
            const int64_t nc = p.rowptr[first + 1] - p.rowptr[first];
            p.grp_voff[G + 1] = p.grp_voff[G] + nc * (int64_t)rows[G].size();
        }
    }
};

}  // namespace

bool element_touch_pairs(const SpaceDesc& S, std::vector<int64_t>& pairs, std::vector<int32_t>& info,
                         std::string& err) {
    Plan p;
    p.S = S;
    Builder B(p);
    B.vertex_ids();
    return B.touching_elements(pairs, info, err);
}

bool build_plan(const SpaceDesc& S, const H2Params& P, Plan& p, std::string& err) {
    p = Plan();
    p.S = S;
    p.P = P;
    if (P.q < 1 || P.q > 8) {
        err = "q must lie in [1, 8]";
        return false;
    }
    if (!(P.eta >= 0.0) || !std::isfinite(P.eta)) {
        err = "eta must be finite and >= 0";
        return false;
    }
    if (P.chunk < 128 || P.chunk % 128 != 0 || P.chunk > (1 << 20)) {
        err = "chunk_cols must be a positive multiple of 128";
        return false;
    }
    if (P.qg < 1 || P.qg > 16 || P.qs < 1 || P.qs > 16) {
        err = "qg and qs must lie in [1, 16]";
        return false;
    }
    p.leaf = P.leaf < 0 ? std::max(S.L - 2, 0) : P.leaf;
    if (p.leaf > S.L) {
        err = "leaf level must not exceed the refinement level";
        return false;
    }
    p.m = 1 << (S.L - p.leaf);
    p.nloc = (p.m - 1) * S.r + S.d + 1;
    p.nleaf1 = 1 << p.leaf;
    p.q2 = P.q * P.q;
    p.lev_off.assign(p.leaf + 2, 0);
    for (int l = 0; l <= p.leaf; ++l)
        p.lev_off[l + 1] = p.lev_off[l] + (int64_t)S.geom.npatch * ((int64_t)1 << (2 * l));
    p.ncl = p.lev_off[p.leaf + 1];
    p.nleaves = p.ncl - p.lev_off[p.leaf];

    Builder B(p);
    B.balls();
    std::vector<std::pair<int32_t, int32_t>> far, nearp;
    B.partition(far, nearp);
    p.far_t.resize(far.size());
    p.far_s.resize(far.size());
    for (size_t i = 0; i < far.size(); ++i) {
        p.far_t[i] = far[i].first;
        p.far_s[i] = far[i].second;
    }
    p.far_rowptr.assign(p.ncl + 1, 0);
    for (auto& f : far) p.far_rowptr[f.first + 1]++;
    for (int64_t c = 0; c < p.ncl; ++c) p.far_rowptr[c + 1] += p.far_rowptr[c];
    // stored blocks: each unordered pair once, in its owner's rows
    std::vector<std::vector<int32_t>> own(p.ncl), tr(p.ncl);
    for (auto& f : far) {
        const int32_t a = std::min(f.first, f.second), b = std::max(f.first, f.second);
        if (f.first != a) continue;  // visit each unordered pair once
        const int32_t owner = ((a + b) & 1) ? a : b, other = owner == a ? b : a;
        own[owner].push_back(other);
    }
    p.own_rowptr.assign(p.ncl + 1, 0);
    p.koff.assign(p.ncl, 0);
    p.krs.assign(p.ncl, 0);
    p.pcol.assign(p.ncl, 0);
    p.cl_chunk.assign(p.ncl + 1, 0);
    int64_t off = 0, poff = 0;
    for (int64_t c = 0; c < p.ncl; ++c) {
        std::sort(own[c].begin(), own[c].end());
        const int64_t n = (int64_t)own[c].size();
        const int64_t rs = ((n * p.q2) + 1) / 2 * 2;  // even row length for paired loads
        p.koff[c] = off;
        p.krs[c] = (int32_t)rs;
        p.pcol[c] = poff;
        for (int64_t s = 0; s < n; ++s) {
            p.own_src.push_back(own[c][s]);
            p.own_t.push_back((int32_t)c);
            tr[own[c][s]].push_back(0);  // counted below
        }
        p.own_rowptr[c + 1] = p.own_rowptr[c] + n;
        for (int64_t k0 = 0; k0 < rs; k0 += P.chunk) {
            p.ch_t.push_back((int32_t)c);
            p.ch_k0.push_back((int32_t)k0);
            p.ch_k1.push_back((int32_t)std::min<int64_t>(rs, k0 + P.chunk));
        }
        p.cl_chunk[c + 1] = (int64_t)p.ch_t.size();
        off += rs * p.q2;
        poff += rs;
    }
    p.ktotal = off;
    p.ptotal = poff;
    // transposed lists: for each partner, the offsets of its columns in the owners' rows
    p.tr_rowptr.assign(p.ncl + 1, 0);
    for (int64_t c = 0; c < p.ncl; ++c) p.tr_rowptr[c + 1] = p.tr_rowptr[c] + (int64_t)tr[c].size();
    p.tr_off.assign(p.tr_rowptr[p.ncl], 0);
    std::vector<int64_t> fill(p.tr_rowptr.begin(), p.tr_rowptr.end() - 1);
    for (int64_t c = 0; c < p.ncl; ++c)
        for (int64_t s = p.own_rowptr[c]; s < p.own_rowptr[c + 1]; ++s)
            p.tr_off[fill[p.own_src[s]]++] = p.pcol[c] + (s - p.own_rowptr[c]) * p.q2;

    p.near_t.resize(nearp.size());
    p.near_s.resize(nearp.size());
    p.near_rowptr.assign(p.nleaves + 1, 0);
    for (size_t i = 0; i < nearp.size(); ++i) {
        p.near_t[i] = nearp[i].first;
        p.near_s[i] = nearp[i].second;
        p.near_rowptr[nearp[i].first + 1]++;
    }
    for (int64_t c = 0; c < p.nleaves; ++c) p.near_rowptr[c + 1] += p.near_rowptr[c];

    B.vertex_ids();
    bool ok = true;
    B.touching(ok, err);
    if (!ok) return false;
    B.near_pattern();
    B.near_groups();

    // tables
    gauss_legendre01(P.qg, p.gx, p.gw);
    gauss_legendre01(P.qs, p.sx, p.sw);
    bspline_local_polys(S.d, S.r, S.L, p.bpoly);
    const int d1 = S.d + 1;
    p.psi.assign((size_t)S.nel * P.qg * d1, 0.0);
    for (int i = 0; i < S.nel; ++i)
        for (int a = 0; a < P.qg; ++a)
            for (int l = 0; l < d1; ++l)
                p.psi[((size_t)i * P.qg + a) * d1 + l] = poly_eval(&p.bpoly[((size_t)i * d1 + l) * d1], S.d, p.gx[a]);
    p.psiw.resize(p.psi.size());
    for (size_t k = 0; k < p.psi.size(); ++k) p.psiw[k] = p.gw[(k / d1) % P.qg] * p.psi[k];
    p.cheb.resize(P.q);
    for (int a = 0; a < P.q; ++a) p.cheb[a] = 0.5 + 0.5 * std::cos((2.0 * a + 1.0) * kPi / (2.0 * P.q));
    p.E.assign(2 * p.q2, 0.0);
    for (int b = 0; b < 2; ++b)
        for (int ap = 0; ap < P.q; ++ap)
            for (int a = 0; a < P.q; ++a) p.E[(b * P.q + ap) * P.q + a] = lagrange_bary(p.cheb, a, 0.5 * (b + p.cheb[ap]));
    // 1-D leaf moments: exact Gauss with ceil((q+d)/2) points per element
    const int qm = (P.q + S.d + 1) / 2;
    std::vector<double> mx, mw;
    gauss_legendre01(qm, mx, mw);
    p.V1.assign((size_t)p.nleaf1 * P.q * p.nloc, 0.0);
    for (int i = 0; i < p.nleaf1; ++i)
        for (int el = i * p.m; el < (i + 1) * p.m; ++el) {
            const int off_b = (el - i * p.m) * S.r;  // first local basis of el within the leaf
            for (int k = 0; k < qm; ++k) {
                const double xl = ((el - i * p.m) + mx[k]) / p.m;  // leaf-local coordinate
                for (int a = 0; a < P.q; ++a) {
                    const double La = lagrange_bary(p.cheb, a, xl);
                    for (int l = 0; l < d1; ++l) {
                        const double bv = poly_eval(&p.bpoly[((size_t)el * d1 + l) * d1], S.d, mx[k]);
                        p.V1[((size_t)i * P.q + a) * p.nloc + off_b + l] += mw[k] * S.h * La * bv;
                    }
                }
            }
        }
    return true;
}

}  // namespace bem
