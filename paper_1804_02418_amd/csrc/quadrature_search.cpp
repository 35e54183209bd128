// Quadrature search on prescribed nodes (Sec. 2.3), host side of the C ABI
// in include/rlbm_quadrature.h.  Long double throughout: the massive systems
// reach condition numbers near 1e10 where non-negative solutions exist.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>

#include "../../include/rlbm_quadrature.h"
#include "rlbm_internal.h"

namespace rlbm {
rlbm_status set_error(rlbm_status st, const char *msg);
}

namespace {

typedef long double LD;

rlbm_status bad(const char *msg) { return rlbm::set_error(RLBM_EINVAL, msg); }

// (b-1)!! (c-1)!! / (b+c)!!: the angular mean of cos^b sin^c (b, c even).
LD angular_mean(int b, int c)
{
    auto dfact = [](int n) {
        LD r = 1;
        for (int k = n; k > 1; k -= 2) r *= k;
        return r;
    };
    return dfact(b - 1) * dfact(c - 1) / dfact(b + c);
}

// <p0^a px^b py^c> of the rest Maxwell-Juttner weight (T0 = 1), closed form.
LD mj_moment(LD m, int a, int b, int c)
{
    if ((b & 1) || (c & 1)) return 0;
    const int k = (b + c) / 2;
    // polynomial in u of (u + m)^a u^k (u + 2m)^k, then int e^-u u^n du = n!
    std::vector<LD> poly(1, 1.0L);
    auto mul = [&poly](LD shift) {  // poly *= (u + shift)
        std::vector<LD> out(poly.size() + 1, 0.0L);
        for (size_t n = 0; n < poly.size(); ++n) {
            out[n + 1] += poly[n];
            out[n] += shift * poly[n];
        }
        poly.swap(out);
    };
    for (int i = 0; i < a; ++i) mul(m);
    for (int i = 0; i < k; ++i) mul(0);
    for (int i = 0; i < k; ++i) mul(2 * m);
    LD sum = 0, fact = 1;
    for (size_t n = 0; n < poly.size(); ++n) {
        if (n > 0) fact *= (LD)n;
        sum += poly[n] * fact;
    }
    return angular_mean(b, c) * sum;
}

struct Cond {
    int a, b, c;
    LD target, scale;
};

// Monomial conditions that symmetric weights do not satisfy by symmetry:
// a + b + c <= 2 * order, b and c even.
std::vector<Cond> conditions(LD m, int order)
{
    std::vector<Cond> out;
    const int top = 2 * order;
    for (int a = 0; a <= top; ++a)
        for (int b = 0; a + b <= top; b += 2)
            for (int c = 0; a + b + c <= top; c += 2) {
                const LD t = mj_moment(m, a, b, c);
                out.push_back(Cond{a, b, c, t, std::max(std::fabs(t), (LD)1)});
            }
    return out;
}

// Orbits of the symmetries of the square; false if the set is not closed.
bool make_orbits(const int *v, int n, std::vector<std::vector<int>> &orbits)
{
    std::vector<int> orbit_of(n, -1);
    for (int i = 0; i < n; ++i) {
        if (orbit_of[i] >= 0) continue;
        const int x = v[2 * i], y = v[2 * i + 1];
        const int img[8][2] = {{x, y}, {-x, y}, {x, -y}, {-x, -y}, {y, x}, {-y, x}, {y, -x}, {-y, -x}};
        std::vector<int> members;
        for (auto &p : img) {
            int found = -1;
            for (int k = 0; k < n; ++k)
                if (v[2 * k] == p[0] && v[2 * k + 1] == p[1]) found = k;
            if (found < 0) return false;
            if (std::find(members.begin(), members.end(), found) == members.end()) members.push_back(found);
        }
        for (int k : members) {
            if (orbit_of[k] >= 0 && orbit_of[k] != (int)orbits.size()) return false;
            orbit_of[k] = (int)orbits.size();
        }
        orbits.push_back(members);
    }
    // duplicated vectors would sit in no orbit twice; reject them
    for (int i = 0; i < n; ++i)
        for (int k = i + 1; k < n; ++k)
            if (v[2 * i] == v[2 * k] && v[2 * i + 1] == v[2 * k + 1]) return false;
    return true;
}

// Least squares min |A x - r| (rows x cols, rows >= cols) by Householder QR
// (A and r are overwritten).  Returns false if a column is (numerically) null.
bool least_squares(std::vector<LD> &A, std::vector<LD> &r, int rows, int cols, std::vector<LD> &x)
{
    for (int k = 0; k < cols; ++k) {
        LD norm = 0;
        for (int i = k; i < rows; ++i) norm += A[i * cols + k] * A[i * cols + k];
        norm = std::sqrt(norm);
        if (!(norm > 0)) return false;
        const LD alpha = A[k * cols + k] > 0 ? -norm : norm;
        std::vector<LD> u(rows - k);
        for (int i = k; i < rows; ++i) u[i - k] = A[i * cols + k];
        u[0] -= alpha;
        LD un = 0;
        for (LD e : u) un += e * e;
        if (un > 0) {
            for (int j = k; j < cols; ++j) {
                LD d = 0;
                for (int i = k; i < rows; ++i) d += u[i - k] * A[i * cols + j];
                d = 2 * d / un;
                for (int i = k; i < rows; ++i) A[i * cols + j] -= d * u[i - k];
            }
            LD d = 0;
            for (int i = k; i < rows; ++i) d += u[i - k] * r[i];
            d = 2 * d / un;
            for (int i = k; i < rows; ++i) r[i] -= d * u[i - k];
        }
    }
    x.assign(cols, 0);
    for (int k = cols - 1; k >= 0; --k) {
        LD s = r[k];
        for (int j = k + 1; j < cols; ++j) s -= A[k * cols + j] * x[j];
        if (!(std::fabs(A[k * cols + k]) > 0)) return false;
        x[k] = s / A[k * cols + k];
    }
    return true;
}

struct MassiveResult {
    std::vector<LD> w;  // per orbit
    LD min_w = -INFINITY, residual = INFINITY;
    bool ok = false;
};

MassiveResult solve_massive(LD m, LD v0, const int *vec, const std::vector<std::vector<int>> &orbits,
                            const std::vector<Cond> &conds)
{
    const int rows = (int)conds.size(), cols = (int)orbits.size();
    std::vector<LD> A((size_t)rows * cols), r(rows);
    for (int q = 0; q < rows; ++q) {
        const Cond &cd = conds[q];
        r[q] = cd.target / cd.scale;
        for (int o = 0; o < cols; ++o) {
            LD s = 0;
            for (int i : orbits[o]) {
                const LD nx = vec[2 * i], ny = vec[2 * i + 1];
                const LD v = v0 * std::sqrt(nx * nx + ny * ny);
                const LD p0 = m / std::sqrt(1 - v * v);
                s += std::pow(p0, cd.a) * std::pow(p0 * v0 * nx, cd.b) * std::pow(p0 * v0 * ny, cd.c);
            }
            A[(size_t)q * cols + o] = s / cd.scale;
        }
    }
    const std::vector<LD> A0 = A, r0 = r;
    MassiveResult res;
    if (!least_squares(A, r, rows, cols, res.w)) return res;
    res.residual = 0;
    for (int q = 0; q < rows; ++q) {
        LD s = -r0[q];
        for (int o = 0; o < cols; ++o) s += A0[(size_t)q * cols + o] * res.w[o];
        res.residual = std::max(res.residual, std::fabs(s));
    }
    res.min_w = *std::min_element(res.w.begin(), res.w.end());
    res.ok = std::isfinite((double)res.residual) && std::isfinite((double)res.min_w);
    return res;
}

// ---------------------------------------------------------------- massless

struct MasslessProblem {
    int nsh = 0;
    std::vector<std::vector<int>> orbits;
    std::vector<Cond> conds;
    std::vector<std::vector<LD>> S;  // S[q][o] = sum over orbit of nhat_x^b nhat_y^c
};

// Residuals (scaled) and Jacobian at parameters x = [s (orbits x shells, orbit-major), q (shells)].
void massless_eval(const MasslessProblem &P, const std::vector<LD> &x, std::vector<LD> &res, std::vector<LD> *jac)
{
    const int no = (int)P.orbits.size(), ns = P.nsh, nu = no * ns + ns, rows = (int)P.conds.size();
    res.assign(rows, 0);
    if (jac) jac->assign((size_t)rows * nu, 0);
    for (int q = 0; q < rows; ++q) {
        const Cond &cd = P.conds[q];
        const int d = cd.a + cd.b + cd.c;
        LD val = 0;
        for (int j = 0; j < ns; ++j) {
            const LD qj = x[no * ns + j], p0 = qj * qj;
            const LD pd = std::pow(p0, d);
            LD ang = 0;
            for (int o = 0; o < no; ++o) {
                const LD s = x[o * ns + j];
                ang += s * s * P.S[q][o];
                if (jac) (*jac)[(size_t)q * nu + o * ns + j] = 2 * s * pd * P.S[q][o] / cd.scale;
            }
            val += pd * ang;
            if (jac && d > 0) (*jac)[(size_t)q * nu + no * ns + j] = 2 * qj * d * std::pow(p0, d - 1) * ang / cd.scale;
        }
        res[q] = (val - cd.target) / cd.scale;
    }
}

LD max_abs(const std::vector<LD> &v)
{
    LD m = 0;
    for (LD e : v) m = std::max(m, std::fabs(e));
    return m;
}

// Solve the symmetric positive (semi-)definite n x n system M d = g by
// Cholesky; false if it breaks down.
bool cholesky_solve(std::vector<LD> M, std::vector<LD> g, int n, std::vector<LD> &d)
{
    for (int j = 0; j < n; ++j) {
        LD s = M[j * n + j];
        for (int k = 0; k < j; ++k) s -= M[j * n + k] * M[j * n + k];
        if (!(s > 0)) return false;
        M[j * n + j] = std::sqrt(s);
        for (int i = j + 1; i < n; ++i) {
            LD t = M[i * n + j];
            for (int k = 0; k < j; ++k) t -= M[i * n + k] * M[j * n + k];
            M[i * n + j] = t / M[j * n + j];
        }
    }
    for (int i = 0; i < n; ++i) {
        LD t = g[i];
        for (int k = 0; k < i; ++k) t -= M[i * n + k] * g[k];
        g[i] = t / M[i * n + i];
    }
    for (int i = n - 1; i >= 0; --i) {
        LD t = g[i];
        for (int k = i + 1; k < n; ++k) t -= M[k * n + i] * g[k];
        g[i] = t / M[i * n + i];
    }
    d = g;
    return true;
}

// Levenberg-Marquardt from x; returns the final largest scaled residual.
LD levenberg_marquardt(const MasslessProblem &P, std::vector<LD> &x, int max_iter)
{
    const int nu = (int)x.size(), rows = (int)P.conds.size();
    std::vector<LD> r, J;
    massless_eval(P, x, r, &J);
    LD cost = 0;
    for (LD e : r) cost += e * e;
    LD lambda = 1e-3L;
    for (int it = 0; it < max_iter && max_abs(r) > 1e-16L; ++it) {
        std::vector<LD> JTJ((size_t)nu * nu, 0), g(nu, 0);
        for (int q = 0; q < rows; ++q)
            for (int a = 0; a < nu; ++a) {
                const LD ja = J[(size_t)q * nu + a];
                if (ja == 0) continue;
                g[a] -= ja * r[q];
                for (int b = 0; b < nu; ++b) JTJ[(size_t)a * nu + b] += ja * J[(size_t)q * nu + b];
            }
        bool improved = false;
        for (int tries = 0; tries < 30 && !improved; ++tries) {
            std::vector<LD> M = JTJ, d;
            for (int a = 0; a < nu; ++a) M[(size_t)a * nu + a] += lambda * (JTJ[(size_t)a * nu + a] + 1e-30L);
            if (!cholesky_solve(M, g, nu, d)) {
                lambda *= 10;
                continue;
            }
            std::vector<LD> xn(nu), rn;
            for (int a = 0; a < nu; ++a) xn[a] = x[a] + d[a];
            massless_eval(P, xn, rn, nullptr);
            LD cn = 0;
            for (LD e : rn) cn += e * e;
            if (std::isfinite((double)cn) && cn < cost) {
                x = xn;
                cost = cn;
                lambda = std::max(lambda / 3, (LD)1e-12L);
                improved = true;
            } else {
                lambda *= 4;
            }
        }
        if (!improved) break;
        massless_eval(P, x, r, &J);
    }
    return max_abs(r);
}

uint64_t splitmix(uint64_t &s)
{
    uint64_t z = (s += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

}  // namespace

namespace rlbm {
double massless_stencil_residual(const Quadrature &qd)
{
    const std::vector<Cond> conds = conditions(0, 3);
    LD worst = 0;
    for (const Cond &cd : conds) {
        LD s = 0;
        for (int d = 0; d < kDirs; ++d)
            for (int j = 0; j < kShells; ++j) {
                const LD w = kGroup[d] ? qd.w2[j] : qd.w1[j];
                const LD p0 = qd.p0[j];
                s += w * std::pow(p0, cd.a) * std::pow(p0 * kCx[d] / 5.0L, cd.b) * std::pow(p0 * kCy[d] / 5.0L, cd.c);
            }
        worst = std::max(worst, std::fabs(s - cd.target) / cd.scale);
    }
    return (double)worst;
}
}  // namespace rlbm

extern "C" {

rlbm_status rlbm_mj_moment(double mbar, int a, int b, int c, double *value)
{
    if (!value || !(mbar >= 0) || !std::isfinite(mbar) || a < 0 || b < 0 || c < 0 || a + b + c > 24)
        return bad("rlbm_mj_moment: invalid argument");
    *value = (double)mj_moment(mbar, a, b, c);
    return RLBM_OK;
}

rlbm_status rlbm_quadrature_massive(double mbar, int order, const int *vectors, int nvec, int nscan, double *v0_out,
                                    double *weights, double *min_weight, double *residual)
{
    if (!vectors || nvec < 1 || !v0_out || !weights || !min_weight || !residual)
        return bad("rlbm_quadrature_massive: NULL or empty argument");
    if (!(mbar > 0) || !std::isfinite(mbar)) return bad("rlbm_quadrature_massive: mbar must be positive");
    if (order < 1 || order > 4) return bad("rlbm_quadrature_massive: order must be 1..4");
    std::vector<std::vector<int>> orbits;
    if (!make_orbits(vectors, nvec, orbits))
        return bad("rlbm_quadrature_massive: the stencil is not closed under the symmetries of the square");
    LD rmax = 0;
    for (int i = 0; i < nvec; ++i)
        rmax = std::max(rmax, std::sqrt((LD)vectors[2 * i] * vectors[2 * i] + (LD)vectors[2 * i + 1] * vectors[2 * i + 1]));
    if (!(rmax > 0)) return bad("rlbm_quadrature_massive: the stencil has no moving node");
    const std::vector<Cond> conds = conditions(mbar, order);
    if ((int)conds.size() < (int)orbits.size())
        return bad("rlbm_quadrature_massive: more orbits than conditions (the weights are not determined)");
    const int n = nscan > 0 ? nscan : 20000;
    const LD lo = 1e-3L / rmax, hi = (1 - 1e-9L) / rmax;
    auto margin = [&](LD v0) {
        const MassiveResult r = solve_massive(mbar, v0, vectors, orbits, conds);
        return (r.ok && r.residual < 1e-10L) ? r.min_w : -INFINITY;
    };
    LD best_v = lo, best = -INFINITY;
    for (int k = 0; k < n; ++k) {
        const LD v0 = lo + (hi - lo) * k / (n - 1);
        const LD g = margin(v0);
        if (g > best) {
            best = g;
            best_v = v0;
        }
    }
    // golden-section refinement of the smallest weight around the best grid point
    const LD h = (hi - lo) / (n - 1);
    LD a = std::max(lo, best_v - h), b = std::min(hi, best_v + h);
    const LD gr = (std::sqrt((LD)5) - 1) / 2;
    LD c = b - gr * (b - a), d = a + gr * (b - a);
    LD fc = margin(c), fd = margin(d);
    for (int it = 0; it < 120; ++it) {
        if (fc > fd) {
            b = d;
            d = c;
            fd = fc;
            c = b - gr * (b - a);
            fc = margin(c);
        } else {
            a = c;
            c = d;
            fc = fd;
            d = a + gr * (b - a);
            fd = margin(d);
        }
    }
    LD v0 = (a + b) / 2;
    if (!(margin(v0) >= best)) v0 = best_v;
    const MassiveResult r = solve_massive(mbar, v0, vectors, orbits, conds);
    *v0_out = (double)v0;
    for (size_t o = 0; o < orbits.size(); ++o)
        for (int i : orbits[o]) weights[i] = r.ok ? (double)r.w[o] : NAN;
    *min_weight = (double)r.min_w;
    *residual = (double)r.residual;
    if (!r.ok || !(r.min_w >= 0) || !(r.residual < 1e-10L))
        return rlbm::set_error(RLBM_ENOTFOUND, "rlbm_quadrature_massive: no v0 gives non-negative weights");
    return RLBM_OK;
}

rlbm_status rlbm_quadrature_massless(int order, const int *directions, int ndir, int nshells, const double *start_p0,
                                     const double *start_w, uint64_t seed, int max_starts, double *p0_out,
                                     double *weights, double *min_weight, double *residual)
{
    if (!directions || ndir < 1 || nshells < 1 || nshells > 16 || !p0_out || !weights || !min_weight || !residual)
        return bad("rlbm_quadrature_massless: NULL or empty argument");
    if (order < 1 || order > 4) return bad("rlbm_quadrature_massless: order must be 1..4");
    if ((start_p0 == nullptr) != (start_w == nullptr))
        return bad("rlbm_quadrature_massless: give both start_p0 and start_w, or neither");
    MasslessProblem P;
    P.nsh = nshells;
    if (!make_orbits(directions, ndir, P.orbits))
        return bad("rlbm_quadrature_massless: the directions are not closed under the symmetries of the square");
    const long long r2 = (long long)directions[0] * directions[0] + (long long)directions[1] * directions[1];
    for (int i = 0; i < ndir; ++i)
        if ((long long)directions[2 * i] * directions[2 * i] + (long long)directions[2 * i + 1] * directions[2 * i + 1] !=
                r2 ||
            r2 == 0)
            return bad("rlbm_quadrature_massless: directions must be non-zero and of one length");
    const LD R = std::sqrt((LD)r2);
    P.conds = conditions(0, order);
    for (const Cond &cd : P.conds) {
        std::vector<LD> row;
        for (const auto &orb : P.orbits) {
            LD s = 0;
            for (int i : orb) s += std::pow(directions[2 * i] / R, cd.b) * std::pow(directions[2 * i + 1] / R, cd.c);
            row.push_back(s);
        }
        P.S.push_back(row);
    }
    const int no = (int)P.orbits.size(), ns = nshells;
    std::vector<LD> best_x;
    LD best_res = INFINITY;
    auto accept = [&](const std::vector<LD> &x, LD res) {
        std::vector<LD> p(ns);
        for (int j = 0; j < ns; ++j) p[j] = x[no * ns + j] * x[no * ns + j];
        std::vector<LD> sp = p;
        std::sort(sp.begin(), sp.end());
        for (int j = 1; j < ns; ++j)
            if (!(sp[j] - sp[j - 1] > 1e-6L * sp[ns - 1])) return false;
        return res < 1e-13L;
    };
    uint64_t st = seed;
    const int starts = start_p0 ? 1 : std::max(1, max_starts);
    for (int k = 0; k < starts; ++k) {
        std::vector<LD> x(no * ns + ns);
        if (start_p0) {
            for (int j = 0; j < ns; ++j) {
                x[no * ns + j] = std::sqrt(std::max((LD)start_p0[j], (LD)0));
                for (int o = 0; o < no; ++o)
                    x[o * ns + j] = std::sqrt(std::max((LD)start_w[(size_t)j * ndir + P.orbits[o][0]], (LD)0));
            }
        } else {
            auto uni = [&st]() { return (LD)((splitmix(st) >> 11) * (1.0 / 9007199254740992.0)); };
            for (int j = 0; j < ns; ++j) x[no * ns + j] = std::sqrt(0.05L + 10 * uni());
            for (int o = 0; o < no; ++o)
                for (int j = 0; j < ns; ++j) x[o * ns + j] = std::sqrt(0.001L + 0.05L * uni());
        }
        const LD res = levenberg_marquardt(P, x, 400);
        const bool good = accept(x, res);
        if (good || (best_x.empty() || res < best_res)) {
            best_x = x;
            best_res = res;
        }
        if (good) break;
    }
    // outputs, shells sorted ascending
    std::vector<int> order_j(ns);
    for (int j = 0; j < ns; ++j) order_j[j] = j;
    std::sort(order_j.begin(), order_j.end(), [&](int u, int v) { return best_x[no * ns + u] * best_x[no * ns + u] < best_x[no * ns + v] * best_x[no * ns + v]; });
    LD mw = INFINITY;
    for (int jj = 0; jj < ns; ++jj) {
        const int j = order_j[jj];
        p0_out[jj] = (double)(best_x[no * ns + j] * best_x[no * ns + j]);
        for (int o = 0; o < no; ++o) {
            const LD w = best_x[o * ns + j] * best_x[o * ns + j];
            mw = std::min(mw, w);
            for (int i : P.orbits[o]) weights[(size_t)jj * ndir + i] = (double)w;
        }
    }
    *min_weight = (double)mw;
    *residual = (double)best_res;
    if (!accept(best_x, best_res))
        return rlbm::set_error(RLBM_ENOTFOUND, "rlbm_quadrature_massless: no start converged to a solution");
    return RLBM_OK;
}

}  // extern "C"
