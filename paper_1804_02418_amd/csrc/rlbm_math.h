// Per-site arithmetic of the relativistic LB step, shared by the host
// (set-up and self-checks) and the gfx950 kernels.  Everything here is the
// library's own formulation of the paper's Sec. 2:
//
//  * On the massless shell a node momentum is p = p0 (1, cos t, sin t).  A
//    polynomial of degree <= 3 in (p0, px, py) restricted to the shell is
//    sum_e p0^e H_e(t) with H_e a trigonometric polynomial of degree <= e, so
//    it is held as 16 "harmonic" coefficients:
//        e=0: [1]   e=1: [1, cos, sin]   e=2: [1, cos, sin, cos2, sin2]
//        e=3: [1, cos, sin, cos2, sin2, cos3, sin3]
//    appendix_a_to_harmonics() maps the 16 expansion coefficients of the
//    Appendix A basis to these (derived by hand from Appendix A with
//    product-to-sum identities; the host checks it against a monomial
//    transcription of Appendix A at start-up).
//  * Opposite directions differ by t -> t + pi, which flips the sign of the
//    odd harmonics; the kernels evaluate each pair of directions at once.
//  * appendix_b() is Appendix B (projections of the Maxwell-Juttner
//    equilibrium), with the density factor n/T (the prefactor of
//    Appendix C).
#pragma once

#include <cmath>

#ifndef __HIPCC__
#define __host__
#define __device__
#endif

#define RLBM_HD __host__ __device__ inline

namespace rlbm {

constexpr int kQ = 48;      // populations per site (Sec. 2.3)
constexpr int kDirs = 12;   // directions of G = {(+-3,+-4)_FS, (+-5,0)_FS}
constexpr int kShells = 4;  // energy shells
constexpr int kK = 16;      // polynomials up to third order (Appendix A)
constexpr int kReach = 5;   // stencil radius ||n_i|| in sites

// Directions sorted by angle; opposite of d is (d + 6) % 12.
constexpr int kCx[kDirs] = {5, 4, 3, 0, -3, -4, -5, -4, -3, 0, 3, 4};
constexpr int kCy[kDirs] = {0, 3, 4, 5, 4, 3, 0, -3, -4, -5, -4, -3};
// 0 for the (+-3,+-4)_FS family (weights w_1j), 1 for (+-5,0)_FS (w_2j).
constexpr int kGroup[kDirs] = {1, 0, 0, 1, 0, 0, 1, 0, 0, 1, 0, 0};

// Angular constants of a direction t: cos kt, sin kt for k = 1..4; for the
// lattice, (cos t, sin t) = n_d / 5 for the first six directions (the other
// six are their opposites).
struct DirTrig {
    double c, s, c2, s2, c3, s3, c4, s4;
};
RLBM_HD constexpr DirTrig trig_of(double c, double s)
{
    return DirTrig{c, s, c * c - s * s, 2.0 * c * s, c * (c * c - 3.0 * s * s), s * (3.0 * c * c - s * s),
                   (c * c - s * s) * (c * c - s * s) - 4.0 * c * c * s * s, 4.0 * c * s * (c * c - s * s)};
}
RLBM_HD constexpr DirTrig dir_trig(int d) { return trig_of(kCx[d] / 5.0, kCy[d] / 5.0); }

// Appendix A (third order, m = 0) in harmonic form: H = sum_k a_k * harm(J_k).
template <class R>
RLBM_HD void appendix_a_to_harmonics(const R a[kK], R H[kK])
{
    // constants of Appendix A, as products (no divisions in the kernels)
    const R r3 = R(1.7320508075688772935274463);       // sqrt(3)
    const R i3 = R(0.5773502691896257645091488);       // 1/sqrt(3)
    const R i23 = R(0.2886751345948128822545744);      // 1/(2 sqrt(3))
    const R h15 = R(1.9364916731037084425896327);      // sqrt(15)/2
    const R r6 = R(2.4494897427831780981972840);       // sqrt(6)
    const R r53 = R(1.2909944487358056283930885);      // sqrt(5/3)
    const R h53 = R(0.6454972243679028141965442);      // sqrt(5/3)/2
    const R r83 = R(1.6329931618554520654648560);      // 2 sqrt(2/3)
    const R c11 = R(0.1613743060919757035491361);      // 5/(8 sqrt(15))
    const R i26 = R(0.2041241452319315136032131);      // 1/(2 sqrt(6))
    const R i215 = R(0.1290994448735805628393088);     // 1/(2 sqrt(15))
    const R c14 = R(0.0322748612183951407098272);      // 1/(8 sqrt(15))
    const R i610 = R(0.0527046276694729988666482);     // 1/(6 sqrt(10))
    // a index: 0:J0 1:J1_0 2:J1_x 3:J1_y 4:J2_00 5:J2_0x 6:J2_0y 7:J2_xx 8:J2_xy
    //          9:J3_000 10:J3_xxx 11:J3_00x 12:J3_0xx 13:J3_00y 14:J3_xxy 15:J3_0xy
    // e = 0
    H[0] = a[0] - a[1] + a[4] - a[9];
    // e = 1: [1, cos, sin]
    H[1] = a[1] - R(2) * a[4] + R(3) * a[9];
    H[2] = a[2] - r3 * a[5] + R(1.5) * a[10] + h15 * a[11];
    H[3] = a[3] - r3 * a[6] + r6 * a[13];
    // e = 2: [1, cos, sin, cos2, sin2]
    H[4] = R(0.5) * a[4] - R(1.5) * a[9];
    H[5] = i3 * a[5] - a[10] - r53 * a[11];
    H[6] = i3 * a[6] - r83 * a[13];
    H[7] = i23 * a[7] - h53 * a[12];
    H[8] = i23 * a[8] - h53 * a[15];
    // e = 3: [1, cos, sin, cos2, sin2, cos3, sin3]
    H[9] = R(0.16666666666666666666666667) * a[9];
    H[10] = R(0.125) * a[10] + c11 * a[11];
    H[11] = i26 * a[13];
    H[12] = i215 * a[12];
    H[13] = i215 * a[15];
    H[14] = R(0.04166666666666666666666667) * a[10] - c14 * a[11];
    H[15] = i610 * a[14];
}

// Even / odd (in t -> t + pi) parts of the four radial coefficients
// Q_e(t) = H_e(t) for one direction with angular constants tg.
template <class R>
RLBM_HD void harmonics_pair(const R H[kK], const DirTrig &tg, R E[4], R O[4])
{
    const R c = R(tg.c), s = R(tg.s), c2 = R(tg.c2), s2 = R(tg.s2), c3 = R(tg.c3), s3 = R(tg.s3);
    E[0] = H[0];
    O[0] = R(0);
    E[1] = H[1];
    O[1] = H[2] * c + H[3] * s;
    E[2] = H[4] + H[7] * c2 + H[8] * s2;
    O[2] = H[5] * c + H[6] * s;
    E[3] = H[9] + H[12] * c2 + H[13] * s2;
    O[3] = H[10] * c + H[11] * s + H[14] * c3 + H[15] * s3;
}

// Relaxation-and-force polynomial in harmonic form.  With
// omega(t) = U0 - Ux cos t - Uy sin t (the relaxation rate of a direction,
// times tau), the per-direction update needs omega(t) Qa_e(t) - Qb_e(t) for
// the radial powers e = 0..3, Qa / Qb having harmonic coefficients Ha / Hb.
// The product raises the trigonometric degree by one (product-to-sum), so
// W_e has degree e + 1: cosine coefficients Wc[e][0..e+1], sine
// coefficients Ws[e][1..e+1] (24 numbers instead of the 32 of Ha and Hb).
template <class R>
RLBM_HD void omega_harmonics(const R Ha[kK], const R Hb[kK], R U0, R Ux, R Uy, R Wc[4][5], R Ws[4][5])
{
    // harmonic layout of Ha / Hb per power e: cosine and sine coefficients
    constexpr int kC[4][4] = {{0, -1, -1, -1}, {1, 2, -1, -1}, {4, 5, 7, -1}, {9, 10, 12, 14}};
    constexpr int kS[4][4] = {{-1, -1, -1, -1}, {-1, 3, -1, -1}, {-1, 6, 8, -1}, {-1, 11, 13, 15}};
    const R hx = R(0.5) * Ux, hy = R(0.5) * Uy;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
#pragma unroll
        for (int k = 0; k < 5; ++k) Wc[e][k] = Ws[e][k] = R(0);
#pragma unroll
        for (int k = 0; k <= e; ++k) {
            const R C = Ha[kC[e][k]];
            const R S = k >= 1 ? Ha[kS[e][k]] : R(0);
            Wc[e][k] += U0 * C - Hb[kC[e][k]];
            if (k >= 1) Ws[e][k] += U0 * S - Hb[kS[e][k]];
            if (k == 0) {
                Wc[e][1] -= Ux * C;  // cos t * 1
                Ws[e][1] -= Uy * C;  // sin t * 1
            } else {
                // cos t cos kt = (cos(k+1)t + cos(k-1)t) / 2, cos t sin kt = (sin(k+1)t + sin(k-1)t) / 2
                Wc[e][k + 1] -= hx * C;
                Wc[e][k - 1] -= hx * C;
                Ws[e][k + 1] -= hx * S;
                if (k >= 2) Ws[e][k - 1] -= hx * S;
                // sin t cos kt = (sin(k+1)t - sin(k-1)t) / 2, sin t sin kt = (cos(k-1)t - cos(k+1)t) / 2
                Ws[e][k + 1] -= hy * C;
                if (k >= 2) Ws[e][k - 1] += hy * C;
                Wc[e][k - 1] -= hy * S;
                Wc[e][k + 1] += hy * S;
            }
        }
    }
}

// Even / odd (in t -> t + pi) parts of W_e at direction tg.
template <class R>
RLBM_HD void omega_pair(const R Wc[4][5], const R Ws[4][5], const DirTrig &tg, R E[4], R O[4])
{
    const R c = R(tg.c), s = R(tg.s), c2 = R(tg.c2), s2 = R(tg.s2), c3 = R(tg.c3), s3 = R(tg.s3);
    const R c4 = R(tg.c4), s4 = R(tg.s4);
    E[0] = Wc[0][0];
    O[0] = Wc[0][1] * c + Ws[0][1] * s;
    E[1] = Wc[1][0] + Wc[1][2] * c2 + Ws[1][2] * s2;
    O[1] = Wc[1][1] * c + Ws[1][1] * s;
    E[2] = Wc[2][0] + Wc[2][2] * c2 + Ws[2][2] * s2;
    O[2] = Wc[2][1] * c + Ws[2][1] * s + Wc[2][3] * c3 + Ws[2][3] * s3;
    E[3] = Wc[3][0] + Wc[3][2] * c2 + Ws[3][2] * s2 + Wc[3][4] * c4 + Ws[3][4] * s4;
    O[3] = Wc[3][1] * c + Ws[3][1] * s + Wc[3][3] * c3 + Ws[3][3] * s3;
}

// Value of the polynomial with harmonic coefficients H at p = p0 (1, cos t, sin t).
template <class R>
RLBM_HD R harmonics_eval(const R H[kK], R p0, R t_cos, R t_sin)
{
    const R c = t_cos, s = t_sin;
    const R c2 = c * c - s * s, s2 = R(2) * c * s;
    const R c3 = c * (c * c - R(3) * s * s), s3 = s * (R(3) * c * c - s * s);
    const R q0 = H[0];
    const R q1 = H[1] + H[2] * c + H[3] * s;
    const R q2 = H[4] + H[5] * c + H[6] * s + H[7] * c2 + H[8] * s2;
    const R q3 = H[9] + H[10] * c + H[11] * s + H[12] * c2 + H[13] * s2 + H[14] * c3 + H[15] * s3;
    return ((q3 * p0 + q2) * p0 + q1) * p0 + q0;
}

// Appendix B: a^(k) for temperature T and 4-velocity U, times the density
// factor sc = n/T, handed to sink(k, a_k) one coefficient at a time (so that
// a kernel can convert each one as it is formed instead of holding all
// sixteen).
template <class Sink>
RLBM_HD void appendix_b_each_sc(double sc, double T, double u0, double ux, double uy, Sink &&sink)
{
#pragma clang fp contract(on)
    const double s3 = 1.7320508075688772935274463;
    const double s15 = 3.8729833462074168851792654;
    const double s32 = 1.2247448713915890490986420;  // sqrt(3/2)
    const double s52 = 1.5811388300841896659994467;  // sqrt(5/2)
    const double Tu = T * u0 - 1.0;
    const double T2 = T * T;
    const double ux2 = ux * ux, u02 = u0 * u0;
    sink(0, sc);
    sink(1, sc * Tu);
    sink(2, sc * T * ux);
    sink(3, sc * T * uy);
    sink(4, sc * (0.5 * T2 * (3.0 * u02 - 1.0) - 2.0 * T * u0 + 1.0));
    sink(5, sc * s3 * T * ux * Tu);
    sink(6, sc * s3 * T * uy * Tu);
    sink(7, sc * (-0.5 * s3 * T2 * (u02 - 2.0 * ux2 - 1.0)));
    sink(8, sc * s3 * T2 * ux * uy);
    sink(9, sc * 0.5 * Tu * (T2 * (5.0 * u02 - 3.0) - 4.0 * T * u0 + 2.0));
    sink(10, sc * 0.5 * T * ux * (T2 * (5.0 * ux2 + 3.0) - 6.0 * T * u0 + 3.0));
    sink(11, sc * (-0.5 * s15 * T * ux * (T2 * (-2.0 * u02 + ux2 + 1.0) + 2.0 * T * u0 - 1.0)));
    sink(12, sc * (-0.5 * s15 * T2 * Tu * (u02 - 2.0 * ux2 - 1.0)));
    sink(13, sc * 0.5 * s32 * T * uy * (T2 * (5.0 * u02 - 1.0) - 8.0 * T * u0 + 4.0));
    sink(14, sc * (-0.5 * s52 * T2 * T * uy * (u02 - 4.0 * ux2 - 1.0)));
    sink(15, sc * s15 * T2 * ux * uy * Tu);
}

RLBM_HD void appendix_b(double n, double T, double u0, double ux, double uy, double a[kK])
{
    appendix_b_each_sc(n / T, T, u0, ux, uy, [&](int k, double v) { a[k] = v; });
}

// Exact reciprocal and reciprocal square root (host callers; the kernels
// pass hardware estimates refined by Newton steps).
struct ExactRecip {
    RLBM_HD double rcp(double x) const { return 1.0 / x; }
    RLBM_HD double rsqrt(double x) const { return 1.0 / std::sqrt(x); }
};

// Landau frame of the contravariant stress-energy tensor (symmetric, entries
// t00, t0x, t0y, txx, txy, tyy): eps U^a = T^ab U_b with U the timelike
// eigenvector, U^0 > 0, U.U = 1.  eps is the largest real root of the
// characteristic polynomial of M = T eta (eta = diag(1,-1,-1)), reached by
// Newton's method from T^00 less its flow part (for a perfect fluid that
// start lies between eps and T^00, so the iteration comes down to eps
// monotonically, two steps near rest).  U is the cross product of the two
// spatial rows of M - eps I, which carries no cancellation when the velocity
// is small.  Returns false when no timelike eigenvector is found.
template <class Ops = ExactRecip>
RLBM_HD bool landau_frame(double t00, double t0x, double t0y, double txx, double txy, double tyy, double &eps,
                          double &u0, double &ux, double &uy, const Ops &ops = Ops())
{
    // products fused within a statement only: the rounding is then fixed by
    // the source, identical in every kernel that inlines this
#pragma clang fp contract(on)
    const double c2 = t00 - txx - tyy;
    const double c1 = -t00 * txx + t0x * t0x - t00 * tyy + t0y * t0y + txx * tyy - txy * txy;
    // det of [[t00,-t0x,-t0y],[t0x,-txx,-txy],[t0y,-txy,-tyy]]
    const double c0 = t00 * (txx * tyy - txy * txy) + t0x * (txy * t0y - t0x * tyy) - t0y * (txx * t0y - t0x * txy);
    // start: a perfect fluid has t00 = (eps + P) g^2 - P and |t0| = (eps + P) g^2 v,
    // so eps = t00 - |t0|^2 / (t00 + P) exactly; (txx + tyy) / 2 in place of P
    // leaves an O(v^4) error on the high side
    double l = t00 - fma(t0x, t0x, t0y * t0y) * ops.rcp(t00 + 0.5 * (txx + tyy));
    for (int it = 0; it < 64; ++it) {
        const double pl = ((l - c2) * l + c1) * l - c0;
        const double dp = (3.0 * l - 2.0 * c2) * l + c1;
        const double step = pl * ops.rcp(dp);
        l -= step;
        if (!(std::fabs(step) > 4.0 * 2.220446049250313e-16 * std::fabs(l))) break;
    }
    eps = l;
    const double ax = txx + l, ay = tyy + l;
    const double v0 = ax * ay - txy * txy;
    const double vx = t0x * ay - txy * t0y;
    const double vy = t0y * ax - t0x * txy;
    const double nn = v0 * v0 - vx * vx - vy * vy;
    if (!(v0 > 0.0) || !(nn > 0.0)) {
        u0 = ux = uy = NAN;
        return false;
    }
    const double inv = ops.rsqrt(nn);
    u0 = v0 * inv;
    ux = vx * inv;
    uy = vy * inv;
    return true;
}

}  // namespace rlbm
