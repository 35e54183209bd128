// Host-side constants of the library: the polished quadrature, the force
// projection matrices and a start-up self-check of the harmonic form of
// Appendix A used by the kernels.  Computed once per process in long double.
#include "rlbm_internal.h"

#include <cmath>
#include <cstring>
#include <mutex>

namespace rlbm {
namespace {

using LD = long double;

// ---- Appendix A as monomials c * p0^a px^b py^c (third order, m = 0) ----
struct Mono {
    LD coef;
    int a, b, c;
};
struct Poly {
    int n;
    Mono m[4];
};

const Poly *appendix_a_monomials()
{
    static Poly P[kK];
    static std::once_flag once;
    std::call_once(once, [] {
        const LD r3 = sqrtl(3.0L), r15 = sqrtl(15.0L), r6 = sqrtl(6.0L), r10 = sqrtl(10.0L);
        const LD r53 = sqrtl(5.0L / 3.0L), r23 = sqrtl(2.0L / 3.0L), r25 = sqrtl(2.0L / 5.0L);
        const Poly table[kK] = {
            {1, {{1, 0, 0, 0}}},                                                     // J0
            {2, {{1, 1, 0, 0}, {-1, 0, 0, 0}}},                                      // J1_0
            {1, {{1, 0, 1, 0}}},                                                     // J1_x
            {1, {{1, 0, 0, 1}}},                                                     // J1_y
            {3, {{0.5L, 2, 0, 0}, {-2, 1, 0, 0}, {1, 0, 0, 0}}},                     // J2_00
            {2, {{1 / r3, 1, 1, 0}, {-r3, 0, 1, 0}}},                                // J2_0x
            {2, {{1 / r3, 1, 0, 1}, {-r3, 0, 0, 1}}},                                // J2_0y
            {2, {{1 / r3, 0, 2, 0}, {-1 / (2 * r3), 2, 0, 0}}},                      // J2_xx
            {1, {{1 / r3, 0, 1, 1}}},                                                // J2_xy
            {4, {{1.0L / 6, 3, 0, 0}, {-1.5L, 2, 0, 0}, {3, 1, 0, 0}, {-1, 0, 0, 0}}},  // J3_000
            {3, {{-1, 1, 1, 0}, {1.0L / 6, 0, 3, 0}, {1.5L, 0, 1, 0}}},              // J3_xxx
            {4, {{1 / r15, 2, 1, 0}, {-r53, 1, 1, 0}, {-1 / (2 * r15), 0, 3, 0}, {r15 / 2, 0, 1, 0}}},  // J3_00x
            {4, {{-1 / (2 * r15), 3, 0, 0}, {r53 / 2, 2, 0, 0}, {1 / r15, 1, 2, 0}, {-r53, 0, 2, 0}}},  // J3_0xx
            {3, {{1 / (2 * r6), 2, 0, 1}, {-2 * r23, 1, 0, 1}, {r6, 0, 0, 1}}},      // J3_00y
            {2, {{r25 / 3, 0, 2, 1}, {-1 / (6 * r10), 2, 0, 1}}},                    // J3_xxy
            {2, {{1 / r15, 1, 1, 1}, {-r53, 0, 1, 1}}},                              // J3_0xy
        };
        for (int k = 0; k < kK; ++k) P[k] = table[k];
    });
    return P;
}

// J_k at p = p0 (1, c, s) and its derivative along the ray (d/dp0 at fixed angle).
void eval_on_ray(LD p0, LD c, LD s, LD J[kK], LD dJ[kK])
{
    const Poly *P = appendix_a_monomials();
    for (int k = 0; k < kK; ++k) {
        LD v = 0, d = 0;
        for (int t = 0; t < P[k].n; ++t) {
            const Mono &m = P[k].m[t];
            const int e = m.a + m.b + m.c;
            const LD ang = powl(c, m.b) * powl(s, m.c);
            v += m.coef * powl(p0, e) * ang;
            if (e > 0) d += m.coef * e * powl(p0, e - 1) * ang;
        }
        J[k] = v;
        dJ[k] = d;
    }
}

// Printed values (Sec. 2.3, the m = 0 order-3 stencil, 12 decimals, truncated).
const LD kPrintedW1[4] = {0.003930503244L, 0.008026424774L, 0.000175706060L, 0.042659667266L};
const LD kPrintedW2[4] = {0.054642060984L, 0.013535762740L, 0.000296310700L, 0.071941262878L};
const LD kPrintedP0[4] = {0.000016359462L, 3.305423649330L, 7.758786843141L, 0.935838587521L};

constexpr int kNeq = kK * (kK + 1) / 2;  // Gram entries l <= k
constexpr int kNx = 12;                  // unknowns: w1[4], w2[4], p0[4]

// Residual G_lk - delta_lk of Eq. orthonormal and its Jacobian.
void gram_system(const LD x[kNx], LD r[kNeq], LD jac[kNeq][kNx])
{
    for (int q = 0; q < kNeq; ++q) {
        r[q] = 0;
        for (int u = 0; u < kNx; ++u) jac[q][u] = 0;
    }
    for (int d = 0; d < kDirs; ++d) {
        const int g = kGroup[d];
        const LD c = kCx[d] / 5.0L, s = kCy[d] / 5.0L;
        for (int j = 0; j < kShells; ++j) {
            const LD w = x[4 * g + j], p0 = x[8 + j];
            LD J[kK], dJ[kK];
            eval_on_ray(p0, c, s, J, dJ);
            int q = 0;
            for (int l = 0; l < kK; ++l)
                for (int k = l; k < kK; ++k, ++q) {
                    r[q] += w * J[l] * J[k];
                    jac[q][4 * g + j] += J[l] * J[k];
                    jac[q][8 + j] += w * (dJ[l] * J[k] + J[l] * dJ[k]);
                }
        }
    }
    int q = 0;
    for (int l = 0; l < kK; ++l)
        for (int k = l; k < kK; ++k, ++q)
            if (k == l) r[q] -= 1;
}

// Minimum-norm least-squares step dx = -pinv(A) r by one-sided Jacobi SVD.
void min_norm_step(LD A[kNeq][kNx], const LD r[kNeq], LD dx[kNx], int *rank)
{
    static LD U[kNeq][kNx];
    LD V[kNx][kNx];
    for (int q = 0; q < kNeq; ++q)
        for (int u = 0; u < kNx; ++u) U[q][u] = A[q][u];
    for (int a = 0; a < kNx; ++a)
        for (int b = 0; b < kNx; ++b) V[a][b] = (a == b);
    for (int sweep = 0; sweep < 60; ++sweep) {
        LD off = 0;
        for (int p = 0; p < kNx; ++p)
            for (int q = p + 1; q < kNx; ++q) {
                LD alpha = 0, beta = 0, gamma = 0;
                for (int i = 0; i < kNeq; ++i) {
                    alpha += U[i][p] * U[i][p];
                    beta += U[i][q] * U[i][q];
                    gamma += U[i][p] * U[i][q];
                }
                if (gamma == 0) continue;
                off = fmaxl(off, fabsl(gamma) / sqrtl(alpha * beta));
                const LD zeta = (beta - alpha) / (2 * gamma);
                const LD t = (zeta >= 0 ? 1 : -1) / (fabsl(zeta) + sqrtl(1 + zeta * zeta));
                const LD cs = 1 / sqrtl(1 + t * t), sn = cs * t;
                for (int i = 0; i < kNeq; ++i) {
                    const LD up = U[i][p], uq = U[i][q];
                    U[i][p] = cs * up - sn * uq;
                    U[i][q] = sn * up + cs * uq;
                }
                for (int i = 0; i < kNx; ++i) {
                    const LD vp = V[i][p], vq = V[i][q];
                    V[i][p] = cs * vp - sn * vq;
                    V[i][q] = sn * vp + cs * vq;
                }
            }
        if (off < 1e-18L) break;
    }
    LD sig[kNx], smax = 0;
    for (int u = 0; u < kNx; ++u) {
        LD nn = 0;
        for (int i = 0; i < kNeq; ++i) nn += U[i][u] * U[i][u];
        sig[u] = sqrtl(nn);
        smax = fmaxl(smax, sig[u]);
    }
    for (int u = 0; u < kNx; ++u) dx[u] = 0;
    *rank = 0;
    for (int u = 0; u < kNx; ++u) {
        if (sig[u] <= 1e-10L * smax) continue;
        ++*rank;
        LD proj = 0;  // (U_u / sig)^T r
        for (int i = 0; i < kNeq; ++i) proj += U[i][u] * r[i];
        proj /= sig[u] * sig[u];
        for (int v = 0; v < kNx; ++v) dx[v] -= V[v][u] * proj;
    }
}

struct Constants {
    Quadrature q;
    double Cx[kK][kK], Cy[kK][kK];
    int rank;
    double gram_residual;
    bool ok;
    char err[256];
};

LD angular_mean(int b, int c)
{
    // (1/2pi) integral of cos^b sin^c over a period
    if ((b & 1) || (c & 1)) return 0;
    const int k = b / 2, l = c / 2;
    return tgammal(k + 0.5L) * tgammal(l + 0.5L) / (3.14159265358979323846264338327950288L * tgammal(k + l + 1));
}

// C_j[k][m] = -< J_m ( d_j J_k - J_k p^j / p0^2 ) > with d_j the on-shell
// derivative, integrated exactly term by term: a term c p0^e cos^b sin^c has
// mean e! * angular_mean(b, c); terms with e = -1 must have zero angular mean.
bool force_matrices_exact(double Cx[kK][kK], double Cy[kK][kK], char *err)
{
    const Poly *P = appendix_a_monomials();
    for (int axis = 0; axis < 2; ++axis) {
        for (int k = 0; k < kK; ++k)
            for (int m = 0; m < kK; ++m) {
                LD acc = 0;
                for (int t1 = 0; t1 < P[m].n; ++t1)
                    for (int t2 = 0; t2 < P[k].n; ++t2) {
                        const Mono &A = P[m].m[t1], &B = P[k].m[t2];
                        const int e = A.a + A.b + A.c + B.a + B.b + B.c - 1;
                        // d_x (p0^a px^b py^c) - (p0^a px^b py^c) px/p0^2 on the shell:
                        //   p0^(a+b+c-1) [ b cos^(b-1) sin^c + (a-1) cos^(b+1) sin^c ]   (x)
                        //   p0^(a+b+c-1) [ c cos^b sin^(c-1) + (a-1) cos^b sin^(c+1) ]   (y)
                        LD ang;
                        if (axis == 0) {
                            ang = (B.b ? B.b * angular_mean(A.b + B.b - 1, A.c + B.c) : 0) +
                                  (B.a - 1) * angular_mean(A.b + B.b + 1, A.c + B.c);
                        } else {
                            ang = (B.c ? B.c * angular_mean(A.b + B.b, A.c + B.c - 1) : 0) +
                                  (B.a - 1) * angular_mean(A.b + B.b, A.c + B.c + 1);
                        }
                        if (ang == 0) continue;
                        if (e < 0) {
                            if (fabsl(ang) > 1e-15L) {
                                snprintf(err, 256, "force matrix: non-integrable term survives (k=%d m=%d)", k, m);
                                return false;
                            }
                            continue;
                        }
                        acc += A.coef * B.coef * tgammal(e + 1) * ang;
                    }
                (axis == 0 ? Cx : Cy)[k][m] = (double)(-acc);
            }
    }
    return true;
}

// The harmonic form used by the kernels must equal the monomial transcription.
bool check_harmonic_form(char *err)
{
    double a[kK], H[kK];
    unsigned s = 12345u;
    auto rnd = [&s]() {
        s = s * 1664525u + 1013904223u;
        return (double)(s >> 8) / 16777216.0 - 0.5;
    };
    for (int trial = 0; trial < 64; ++trial) {
        for (int k = 0; k < kK; ++k) a[k] = rnd();
        appendix_a_to_harmonics(a, H);
        const double p0 = 8.0 * (rnd() + 0.5), t = 6.283185307179586 * rnd();
        LD J[kK], dJ[kK];
        eval_on_ray(p0, cosl(t), sinl(t), J, dJ);
        LD ref = 0, mag = 0;
        for (int k = 0; k < kK; ++k) {
            ref += a[k] * J[k];
            mag += fabsl(a[k] * J[k]);
        }
        const double got = harmonics_eval(H, p0, std::cos(t), std::sin(t));
        if (fabsl(got - ref) > 1e-13L * (mag + 1)) {
            snprintf(err, 256, "harmonic form of Appendix A disagrees with the monomial form (trial %d)", trial);
            return false;
        }
    }
    return true;
}

// The combined relaxation polynomial (omega_harmonics / omega_pair) against
// omega(t) Qa(t) - Qb(t) evaluated directly, at a direction and its opposite.
bool check_omega_form(char *err)
{
    unsigned s = 54321u;
    auto rnd = [&s]() {
        s = s * 1664525u + 1013904223u;
        return (double)(s >> 8) / 16777216.0 - 0.5;
    };
    for (int trial = 0; trial < 64; ++trial) {
        double Ha[kK], Hb[kK], Wc[4][5], Ws[4][5], E[4], O[4];
        for (int k = 0; k < kK; ++k) {
            Ha[k] = rnd();
            Hb[k] = rnd();
        }
        const double U0 = 1.0 + rnd(), Ux = rnd(), Uy = rnd();
        omega_harmonics(Ha, Hb, U0, Ux, Uy, Wc, Ws);
        const double t = 6.283185307179586 * rnd(), p0 = 8.0 * (rnd() + 0.5);
        const DirTrig tg = trig_of(std::cos(t), std::sin(t));
        omega_pair(Wc, Ws, tg, E, O);
        for (int side = 0; side < 2; ++side) {
            const double c = side ? -std::cos(t) : std::cos(t), sn = side ? -std::sin(t) : std::sin(t);
            const double ref = (U0 - Ux * c - Uy * sn) * harmonics_eval(Ha, p0, c, sn) - harmonics_eval(Hb, p0, c, sn);
            const double sg = side ? -1.0 : 1.0;
            const double got = (((E[3] + sg * O[3]) * p0 + (E[2] + sg * O[2])) * p0 + (E[1] + sg * O[1])) * p0 +
                               (E[0] + sg * O[0]);
            if (std::fabs(got - ref) > 1e-12 * (1.0 + std::fabs(ref)) * p0 * p0 * p0) {
                snprintf(err, 256, "combined relaxation polynomial disagrees with its definition (trial %d)", trial);
                return false;
            }
        }
    }
    return true;
}

const Constants &constants()
{
    static Constants C;
    static std::once_flag once;
    std::call_once(once, [] {
        C.ok = false;
        C.err[0] = 0;
        LD x[kNx];
        for (int j = 0; j < 4; ++j) {
            x[j] = kPrintedW1[j];
            x[4 + j] = kPrintedW2[j];
            x[8 + j] = kPrintedP0[j];
        }
        static LD r[kNeq], jac[kNeq][kNx];
        LD dx[kNx];
        for (int it = 0; it < 12; ++it) {
            gram_system(x, r, jac);
            min_norm_step(jac, r, dx, &C.rank);
            LD step = 0;
            for (int u = 0; u < kNx; ++u) {
                x[u] += dx[u];
                step = fmaxl(step, fabsl(dx[u]));
            }
            if (step < 1e-21L) break;
        }
        gram_system(x, r, jac);
        LD res = 0;
        for (int q = 0; q < kNeq; ++q) res = fmaxl(res, fabsl(r[q]));
        C.gram_residual = (double)res;
        for (int j = 0; j < 4; ++j) {
            C.q.w1[j] = (double)x[j];
            C.q.w2[j] = (double)x[4 + j];
            C.q.p0[j] = (double)x[8 + j];
        }
        if (res > 1e-16L) {
            snprintf(C.err, sizeof C.err, "quadrature polish did not converge (residual %.3Le)", res);
            return;
        }
        for (int u = 0; u < kNx; ++u) {
            const LD printed = u < 4 ? kPrintedW1[u] : u < 8 ? kPrintedW2[u - 4] : kPrintedP0[u - 8];
            if (fabsl(x[u] - printed) > 2e-12L) {
                snprintf(C.err, sizeof C.err, "polished quadrature moved %.3Le from the printed value", fabsl(x[u] - printed));
                return;
            }
        }
        if (!force_matrices_exact(C.Cx, C.Cy, C.err)) return;
        if (!check_harmonic_form(C.err)) return;
        if (!check_omega_form(C.err)) return;
        C.ok = true;
    });
    return C;
}

}  // namespace

bool host_constants(Quadrature *q, double Cx[kK][kK], double Cy[kK][kK], const char **err)
{
    const Constants &C = constants();
    if (!C.ok) {
        if (err) *err = C.err;
        return false;
    }
    if (q) *q = C.q;
    if (Cx) std::memcpy(Cx, C.Cx, sizeof C.Cx);
    if (Cy) std::memcpy(Cy, C.Cy, sizeof C.Cy);
    return true;
}

}  // namespace rlbm
