/*
 * Quadrature search on prescribed nodes (Sec. 2.3): the host-side tool that
 * finds the weights (and, for massless particles, the energy shells) of a
 * Gaussian-type quadrature whose nodes sit on lattice vectors, so that the
 * orthonormality conditions of Eq. `orthonormal` hold up to a chosen order
 * with non-negative weights.  Host code only: no call here touches a device.
 *
 * Conditions.  The products J_l J_k of the polynomials up to order N span the
 * polynomials of degree <= 2N on the mass shell, so Eq. `orthonormal` is the
 * exactness of sum_i w_i M(p_i) = <M> for every monomial M = p0^a px^b py^c
 * with a + b + c <= 2N, <M> being the moment of the rest Maxwell-Juttner
 * weight omega ~ exp(-p0 / T0) (T0 = 1) normalised to <1> = 1 over d^2p / p0
 * (Eq. `mj-poly-weighting-factor`).  Stencils must be closed under the eight
 * symmetries of the square ("full symmetric", FS); weights are then taken
 * equal on each symmetry orbit (averaging any solution over the symmetries
 * gives such a one), and the monomials odd in px or py hold by symmetry.
 *
 * Errors: RLBM_EINVAL for bad arguments (NULL outputs, order outside 1..4,
 * a stencil that is not closed under the symmetries, v0 |n| >= 1 ranges that
 * are empty, massless directions of unequal length), RLBM_ENOTFOUND when no
 * non-negative solution was found (the outputs then hold the best attempt).
 */
#pragma once

#include <stdint.h>

#include "rlbm.h"

#ifdef __cplusplus
extern "C" {
#endif

/* <p0^a px^b py^c> of the rest Maxwell-Juttner weight of particles of mass
 * mbar >= 0 (in units of T0), in closed form: zero unless b and c are even;
 * else (b-1)!!(c-1)!!/(b+c)!! times int_0^inf e^-u (u + m)^a u^k (u + 2m)^k du
 * with k = (b + c)/2 (the substitution u = p0 - m keeps every term positive). */
rlbm_status rlbm_mj_moment(double mbar, int a, int b, int c, double *value);

/* Massive particles (Sec. 2.3, Eqs. `discrete-quadri-momentum`,
 * `discrete-p0`): nodes p_i = p0_i (1, v0 n_i), p0_i = mbar / sqrt(1 - v0^2 |n_i|^2)
 * on the nvec integer vectors `vectors` (nvec pairs x, y; the zero vector is
 * the rest node).  For each v0 the orbit weights solve the conditions of
 * order `order` by least squares (Householder QR in long double); the search
 * scans nscan values of v0 over (0, 1/max|n|) (nscan <= 0: 20000), keeps the
 * one with the largest smallest weight and refines it by golden section.
 * Outputs (caller-owned): *v0, weights[nvec] (per node, in the order of
 * `vectors`), *min_weight, *residual (largest violation of a condition
 * divided by max(|<M>|, 1)).  RLBM_ENOTFOUND if the smallest weight stays
 * negative or the residual above 1e-10. */
rlbm_status rlbm_quadrature_massive(double mbar, int order, const int *vectors, int nvec, int nscan, double *v0,
                                    double *weights, double *min_weight, double *residual);

/* Massless particles (Sec. 2.3): nodes p_{i,j} = p0_j (1, n_i / |n_i|) on
 * ndir integer directions of one length and nshells energy shells p0_j,
 * both the shells and the orbit weights unknown (a nonlinear system whose
 * solutions form a family).  Levenberg-Marquardt on w = s^2, p0 = q^2 (so
 * every solution is non-negative) from start_p0[nshells] and
 * start_w[nshells * ndir] when given (per node, shell-major: index
 * j * ndir + i), else from up to max_starts seeded random starts
 * (splitmix64 seeded with `seed`).  A start succeeds when the residual
 * falls below 1e-13 and the shells are distinct.  Outputs: p0[nshells]
 * sorted ascending, weights[nshells * ndir] (shell-major, per node, in the
 * order of `directions`), *min_weight, *residual. */
rlbm_status rlbm_quadrature_massless(int order, const int *directions, int ndir, int nshells, const double *start_p0,
                                     const double *start_w, uint64_t seed, int max_starts, double *p0,
                                     double *weights, double *min_weight, double *residual);

#ifdef __cplusplus
}
#endif
