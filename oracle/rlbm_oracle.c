/*
 * FP64 CPU oracle of the (2+1)-D relativistic lattice Boltzmann step
 * (m = 0, third order, 48 populations).
 *
 * TEST INFRASTRUCTURE ONLY.  Only tests, the smoke check and the CPU
 * baseline of the benchmark may load this library; the product path never
 * does.  It shares no code with the GPU library.
 *
 * It is written to be checked by eye against the paper, not to be fast:
 * every site runs the steps of the per-site algorithm of Sec. 2 in order
 *   1. moments N^a = sum f_i p_i^a, T^ab = sum f_i p_i^a p_i^b
 *   2. Landau frame: eps U^a = T^ab U_b (largest real eigenvalue, U.U = 1)
 *   3. n = U_a N^a
 *   4. T from the massless 2-D equation of state eps = 2 n T
 *   5. f^eq_i = w_i sum_k a^(k) J^(k)(p_i)    (Eq. feq-expansion-discrete)
 *   6. forcing term (Sec. 2.4)
 *   7. f*_i = f_i - (p_i^mu U_mu)/(p^0_i tau) (f_i - f^eq_i) + F_i
 *      (Eq. discrete-rbe, relaxing sign), then streaming.
 *
 * The caller supplies the quadrature (weights, node momenta), the 48x16
 * table of Appendix A polynomials at the nodes and the two 16x16 force
 * matrices; Appendix B (the projections a^(k)) is transcribed here.
 *
 * The external force of step 6 is the uniform drive, plus, when switched
 * on, the local-capacitance term of Sec. 3 (Eq. lca) taken from the density
 * of the previous state (orc_lattice_set_lca).
 *
 * Storage: populations are SoA, f[i * ny * nx + y * nx + x], i = 4*d + j.
 * The state kept between steps is the pre-collision f(t).
 *
 * Arithmetic type: `real` is double.  Built with -DORC_LONG_DOUBLE, every
 * state array and every operation is long double (x87 extended, 64-bit
 * significand) instead, with the same stencil constants (given as double):
 * the same discrete problem evaluated with about 2^-11 of the rounding
 * error, which measures the FP64 rounding floor of this implementation.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <float.h>
#include <omp.h>

#define Q 48
#define K 16
#define MAXC 16

#ifdef ORC_LONG_DOUBLE
typedef long double real;
#define R_SQRT sqrtl
#define R_FABS fabsl
#define R_EPS LDBL_EPSILON
#define R_NAN ((real)NAN)
#else
typedef double real;
#define R_SQRT sqrt
#define R_FABS fabs
#define R_EPS DBL_EPSILON
#define R_NAN NAN
#endif

/* Size of the arithmetic type, so that a caller can check which build it loaded. */
int orc_real_bytes(void) { return (int)sizeof(real); }

typedef struct {
    real w[Q], p0[Q], px[Q], py[Q];
    int cx[Q], cy[Q], opp[Q];
    real J[Q][K];
    real Cx[K][K], Cy[K][K];
} orc_stencil;

typedef struct {
    int edge;          /* 0: bottom (y < 0), 1: top (y >= ny), 2: left (x < 0), 3: right (x >= nx) */
    int start, width;  /* span along the edge: x in [start, start+width) for bottom/top, y for left/right */
    double n, T, vx, vy;
} orc_contact;

typedef struct {
    const orc_stencil *st;
    int nx, ny, periodic_x, periodic_y;
    int ncontacts;
    orc_contact c[MAXC];
    real feq_c[MAXC][Q];
    unsigned char *solid;   /* NULL or nx*ny, 1 = solid */
    double tau, Fx, Fy;
    double inv_cg;          /* 1/C_g of the local-capacitance force (0: off) */
    real *n_prev;         /* density of the previous state (for the LCA force) */
} orc_lattice;

/* ---------------------------------------------------------------- stencil */

orc_stencil *orc_stencil_new(const double *w, const double *p0, const double *px, const double *py,
                             const int *cx, const int *cy, const int *opp,
                             const double *Jtab, const double *Cx, const double *Cy)
{
    orc_stencil *s = (orc_stencil *)calloc(1, sizeof(orc_stencil));
    if (!s) return NULL;
    for (int i = 0; i < Q; ++i) {
        s->w[i] = w[i]; s->p0[i] = p0[i]; s->px[i] = px[i]; s->py[i] = py[i];
        s->cx[i] = cx[i]; s->cy[i] = cy[i]; s->opp[i] = opp[i];
        for (int k = 0; k < K; ++k) s->J[i][k] = Jtab[i * K + k];
    }
    for (int k = 0; k < K; ++k)
        for (int m = 0; m < K; ++m) { s->Cx[k][m] = Cx[k * K + m]; s->Cy[k][m] = Cy[k * K + m]; }
    return s;
}

void orc_stencil_free(orc_stencil *s) { free(s); }

/* Worker threads of the lattice loops (timing of the CPU baseline only; the
 * sums do not depend on it: each site is computed by one thread). */
void orc_set_threads(int n) { omp_set_num_threads(n > 0 ? n : 1); }
int orc_get_threads(void) { return omp_get_max_threads(); }

/* ------------------------------------------------------------ Appendix B */

/* Projections a^(k) of the Maxwell-Juttner equilibrium (Appendix B), in the
 * order of Appendix A, for 4-velocity U = (u0, ux, uy).  The appendix lists
 * them divided by the density scale; the factor that makes f^eq carry the
 * right density is n/T (the prefactor w_i n / T of Appendix C). */
void orc_projections(real n, real T, const real U[3], real a[K])
{
    const real u0 = U[0], ux = U[1], uy = U[2];
    const real s3 = R_SQRT(3.0), s15 = R_SQRT(15.0);
    a[0] = 1.0;
    a[1] = T * u0 - 1.0;
    a[2] = T * ux;
    a[3] = T * uy;
    a[4] = 0.5 * T * T * (3.0 * u0 * u0 - 1.0) - 2.0 * T * u0 + 1.0;
    a[5] = s3 * T * ux * (T * u0 - 1.0);
    a[6] = s3 * T * uy * (T * u0 - 1.0);
    a[7] = -0.5 * s3 * T * T * (u0 * u0 - 2.0 * ux * ux - 1.0);
    a[8] = s3 * T * T * ux * uy;
    a[9] = 0.5 * (T * u0 - 1.0) * (T * T * (5.0 * u0 * u0 - 3.0) - 4.0 * T * u0 + 2.0);
    a[10] = 0.5 * T * ux * (T * T * (5.0 * ux * ux + 3.0) - 6.0 * T * u0 + 3.0);
    a[11] = -0.5 * s15 * T * ux * (T * T * (-2.0 * u0 * u0 + ux * ux + 1.0) + 2.0 * T * u0 - 1.0);
    a[12] = -0.5 * s15 * T * T * (T * u0 - 1.0) * (u0 * u0 - 2.0 * ux * ux - 1.0);
    a[13] = 0.5 * R_SQRT(1.5) * T * uy * (T * T * (5.0 * u0 * u0 - 1.0) - 8.0 * T * u0 + 4.0);
    a[14] = -0.5 * R_SQRT(2.5) * T * T * T * uy * (u0 * u0 - 4.0 * ux * ux - 1.0);
    a[15] = s15 * T * T * ux * uy * (T * u0 - 1.0);
    const real scale = n / T;
    for (int k = 0; k < K; ++k) a[k] *= scale;
}

/* --------------------------------------------------------------- moments */

/* Compensated (Neumaier) accumulation: the sum is the same sum, evaluated to
 * about one rounding of the result instead of a rounding of every partial
 * sum, so that the oracle's own round-off does not grow with the size of the
 * populations when the moment itself (e.g. T^0x of a slow flow) is small. */
typedef struct { real s, c; } orc_acc;

static void acc_add(orc_acc *a, real v)
{
    const real t = a->s + v;
    if (R_FABS(a->s) >= R_FABS(v)) a->c += (a->s - t) + v;
    else a->c += (v - t) + a->s;
    a->s = t;
}

void orc_moments(const orc_stencil *s, const real *f, real N[3], real Tm[9])
{
    orc_acc n[3] = {{0, 0}}, t[9] = {{0, 0}};
    for (int i = 0; i < Q; ++i) {
        const real p[3] = {s->p0[i], s->px[i], s->py[i]};
        for (int a = 0; a < 3; ++a) {
            acc_add(&n[a], f[i] * p[a]);
            for (int b = 0; b < 3; ++b) acc_add(&t[3 * a + b], f[i] * p[a] * p[b]);
        }
    }
    for (int a = 0; a < 3; ++a) N[a] = n[a].s + n[a].c;
    for (int a = 0; a < 9; ++a) Tm[a] = t[a].s + t[a].c;
}

/* Landau frame: the timelike eigenvector of M^a_b = T^ac eta_cb,
 * eta = diag(1, -1, -1).  eps is the largest real root of the characteristic
 * polynomial, found by Newton's method from lambda = T^00; U is a cross
 * product of two rows of (M - eps I), scaled to U^0 > 0 and U.U = 1.
 * Returns 0 on success, -1 if no timelike eigenvector was found. */
int orc_landau(const real Tm[9], real *eps, real U[3])
{
    real M[3][3];
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) M[a][b] = Tm[3 * a + b] * (b == 0 ? 1.0 : -1.0);
    const real c2 = M[0][0] + M[1][1] + M[2][2];
    const real c1 = M[0][0] * M[1][1] - M[0][1] * M[1][0]
                    + M[0][0] * M[2][2] - M[0][2] * M[2][0]
                    + M[1][1] * M[2][2] - M[1][2] * M[2][1];
    const real c0 = M[0][0] * (M[1][1] * M[2][2] - M[1][2] * M[2][1])
                    - M[0][1] * (M[1][0] * M[2][2] - M[1][2] * M[2][0])
                    + M[0][2] * (M[1][0] * M[2][1] - M[1][1] * M[2][0]);
    real l = Tm[0];
    for (int it = 0; it < 200; ++it) {
        const real pl = ((l - c2) * l + c1) * l - c0;
        const real dp = (3.0 * l - 2.0 * c2) * l + c1;
        if (dp == 0.0) break;
        const real step = pl / dp;
        l -= step;
        if (R_FABS(step) <= 4.0 * R_EPS * R_FABS(l)) break;
    }
    *eps = l;
    real A[3][3];
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) A[a][b] = M[a][b] - (a == b ? l : 0.0);
    real best[3] = {0, 0, 0}, bestn = -1.0;
    const int pairs[3][2] = {{0, 1}, {0, 2}, {1, 2}};
    for (int q = 0; q < 3; ++q) {
        const real *r = A[pairs[q][0]], *t = A[pairs[q][1]];
        const real v[3] = {r[1] * t[2] - r[2] * t[1], r[2] * t[0] - r[0] * t[2], r[0] * t[1] - r[1] * t[0]};
        const real nn = v[0] * v[0] + v[1] * v[1] + v[2] * v[2];
        if (nn > bestn) { bestn = nn; best[0] = v[0]; best[1] = v[1]; best[2] = v[2]; }
    }
    if (best[0] < 0.0) { best[0] = -best[0]; best[1] = -best[1]; best[2] = -best[2]; }
    const real norm2 = best[0] * best[0] - best[1] * best[1] - best[2] * best[2];
    if (!(norm2 > 0.0)) return -1;
    const real inv = 1.0 / R_SQRT(norm2);
    U[0] = best[0] * inv; U[1] = best[1] * inv; U[2] = best[2] * inv;
    return 0;
}

/* Macroscopic fields of one site: n, T, eps and the 4-velocity U. */
int orc_macro(const orc_stencil *s, const real *f, real *n, real *T, real *eps, real U[3])
{
    real N[3], Tm[9];
    orc_moments(s, f, N, Tm);
    if (orc_landau(Tm, eps, U)) return -1;
    *n = U[0] * N[0] - U[1] * N[1] - U[2] * N[2];
    *T = *eps / (2.0 * *n);
    return 0;
}

/* f^eq_i = w_i sum_k a^(k) J^(k)(p_i) (Eq. feq-expansion-discrete, N = 3). */
void orc_feq(const orc_stencil *s, real n, real T, const real U[3], real *feq)
{
    real a[K];
    orc_projections(n, T, U, a);
    for (int i = 0; i < Q; ++i) {
        real acc = 0.0;
        for (int k = 0; k < K; ++k) acc += a[k] * s->J[i][k];
        feq[i] = s->w[i] * acc;
    }
}

/* Forcing term (Sec. 2.4): b_j = C_j a, F_i = -w_i sum_j F^j sum_k J^(k)(p_i) b^(k)_j. */
void orc_force_term(const orc_stencil *s, real n, real T, const real U[3],
                    real Fx, real Fy, real *F)
{
    real a[K], bx[K], by[K];
    orc_projections(n, T, U, a);
    for (int k = 0; k < K; ++k) {
        bx[k] = 0.0; by[k] = 0.0;
        for (int m = 0; m < K; ++m) { bx[k] += s->Cx[k][m] * a[m]; by[k] += s->Cy[k][m] * a[m]; }
    }
    for (int i = 0; i < Q; ++i) {
        real acc = 0.0;
        for (int k = 0; k < K; ++k) acc += s->J[i][k] * (Fx * bx[k] + Fy * by[k]);
        F[i] = -s->w[i] * acc;
    }
}

/* Post-collision populations of one site (right-hand side of Eq. discrete-rbe). */
int orc_collide(const orc_stencil *s, const real *f, real tau, real Fx, real Fy, real *out)
{
    real n, T, eps, U[3], feq[Q], F[Q];
    if (orc_macro(s, f, &n, &T, &eps, U)) return -1;
    orc_feq(s, n, T, U, feq);
    orc_force_term(s, n, T, U, Fx, Fy, F);
    for (int i = 0; i < Q; ++i) {
        const real pU = s->p0[i] * U[0] - s->px[i] * U[1] - s->py[i] * U[2];
        const real omega = pU / (s->p0[i] * tau);
        out[i] = f[i] - omega * (f[i] - feq[i]) + F[i];
    }
    return 0;
}

/* --------------------------------------------------------------- lattice */

orc_lattice *orc_lattice_new(const orc_stencil *st, int nx, int ny, int periodic_x, int periodic_y,
                             int ncontacts, const int *edge, const int *start, const int *width,
                             const double *state /* 4 per contact: n, T, vx, vy */,
                             const unsigned char *solid, double tau, double Fx, double Fy)
{
    if (ncontacts > MAXC || nx <= 0 || ny <= 0) return NULL;
    orc_lattice *L = (orc_lattice *)calloc(1, sizeof(orc_lattice));
    if (!L) return NULL;
    L->st = st; L->nx = nx; L->ny = ny; L->periodic_x = periodic_x; L->periodic_y = periodic_y;
    L->tau = tau; L->Fx = Fx; L->Fy = Fy; L->ncontacts = ncontacts;
    for (int c = 0; c < ncontacts; ++c) {
        orc_contact *C = &L->c[c];
        C->edge = edge[c]; C->start = start[c]; C->width = width[c];
        C->n = state[4 * c]; C->T = state[4 * c + 1]; C->vx = state[4 * c + 2]; C->vy = state[4 * c + 3];
        const real cvx = C->vx, cvy = C->vy;
        const real g = 1.0 / R_SQRT(1.0 - cvx * cvx - cvy * cvy);
        const real U[3] = {g, g * cvx, g * cvy};
        orc_feq(st, C->n, C->T, U, L->feq_c[c]);
    }
    if (solid) {
        L->solid = (unsigned char *)malloc((size_t)nx * ny);
        memcpy(L->solid, solid, (size_t)nx * ny);
    }
    return L;
}

void orc_lattice_free(orc_lattice *L)
{
    if (!L) return;
    free(L->solid);
    free(L->n_prev);
    free(L);
}

/* Local-capacitance electrostatics (Sec. 3, Eq. lca): phi = -e n / C_g.  The
 * force per particle is taken as F = -(e^2 / C_g) grad n (Coulomb repulsion
 * pushes carriers out of denser regions), with e = 1 in lattice units, so the
 * total force on a site is the uniform drive plus -(1/C_g) grad n.  grad n is
 * the central difference of the density of the previous state; a neighbour
 * that is off the lattice (no periodic wrap) or solid takes the site's own
 * density.  inv_cg = 0 switches the term off (C_g = infinity). */
void orc_lattice_set_lca(orc_lattice *L, double inv_cg)
{
    L->inv_cg = inv_cg;
    free(L->n_prev);
    L->n_prev = NULL;
}

int orc_lattice_fields(const orc_lattice *L, const real *f, real *n, real *vx, real *vy,
                       real *eps, real *T);

/* Density of the state f into n (nx*ny). */
static int density_of(const orc_lattice *L, const real *f, real *n)
{
    const size_t P = (size_t)L->nx * L->ny;
    real *tmp = (real *)malloc(4 * P * sizeof(real));
    if (!tmp) return -2;
    orc_lattice_fields(L, f, n, tmp, tmp + P, tmp + 2 * P, tmp + 3 * P);
    free(tmp);
    return 0;
}

/* With the force on and no previous density yet, the first collision takes
 * the density of the state it collides. */
static int ensure_n_prev(orc_lattice *L, const real *f)
{
    if (L->inv_cg == 0.0 || L->n_prev) return 0;
    L->n_prev = (real *)malloc((size_t)L->nx * L->ny * sizeof(real));
    if (!L->n_prev) return -2;
    return density_of(L, f, L->n_prev);
}

static real n_at(const orc_lattice *L, const real *n, int x, int y, int x0, int y0)
{
    if (L->periodic_x) x = ((x % L->nx) + L->nx) % L->nx;
    if (L->periodic_y) y = ((y % L->ny) + L->ny) % L->ny;
    if (x < 0 || x >= L->nx || y < 0 || y >= L->ny) return n[(size_t)y0 * L->nx + x0];
    if (L->solid && L->solid[(size_t)y * L->nx + x]) return n[(size_t)y0 * L->nx + x0];
    return n[(size_t)y * L->nx + x];
}

static void site_force(const orc_lattice *L, int x, int y, real *Fx, real *Fy)
{
    *Fx = L->Fx;
    *Fy = L->Fy;
    if (L->inv_cg == 0.0 || !L->n_prev) return;
    const real *n = L->n_prev;
    const real gx = 0.5 * (n_at(L, n, x + 1, y, x, y) - n_at(L, n, x - 1, y, x, y));
    const real gy = 0.5 * (n_at(L, n, x, y + 1, x, y) - n_at(L, n, x, y - 1, x, y));
    *Fx -= L->inv_cg * gx;
    *Fy -= L->inv_cg * gy;
}

static int is_solid(const orc_lattice *L, int x, int y)
{
    return L->solid ? L->solid[(size_t)y * L->nx + x] : 0;
}

/* Index of the contact whose ghost span holds off-lattice point (x, y), or -1. */
static int contact_at(const orc_lattice *L, int x, int y)
{
    for (int c = 0; c < L->ncontacts; ++c) {
        const orc_contact *C = &L->c[c];
        int along, off;
        switch (C->edge) {
        case 0: off = (y < 0); along = x; if (x < 0 || x >= L->nx) off = 0; break;
        case 1: off = (y >= L->ny); along = x; if (x < 0 || x >= L->nx) off = 0; break;
        case 2: off = (x < 0); along = y; if (y < 0 || y >= L->ny) off = 0; break;
        default: off = (x >= L->nx); along = y; if (y < 0 || y >= L->ny) off = 0; break;
        }
        if (off && along >= C->start && along < C->start + C->width) return c;
    }
    return -1;
}

static void get_site(const orc_lattice *L, const real *f, size_t site, real *out)
{
    const size_t plane = (size_t)L->nx * L->ny;
    for (int i = 0; i < Q; ++i) out[i] = f[i * plane + site];
}

/* Post-collision populations at every fluid site (solid sites copied). */
int orc_lattice_collide(orc_lattice *L, const real *f, real *fstar)
{
    if (ensure_n_prev(L, f)) return -2;
    const size_t plane = (size_t)L->nx * L->ny;
    int bad = 0;
#pragma omp parallel for schedule(static) reduction(+ : bad)
    for (int y = 0; y < L->ny; ++y) {
        real in[Q], out[Q];
        for (int x = 0; x < L->nx; ++x) {
            const size_t site = (size_t)y * L->nx + x;
            get_site(L, f, site, in);
            real Fx, Fy;
            site_force(L, x, y, &Fx, &Fy);
            if (is_solid(L, x, y)) {
                for (int i = 0; i < Q; ++i) out[i] = in[i];
            } else if (orc_collide(L->st, in, L->tau, Fx, Fy, out)) {
                bad += 1;
                for (int i = 0; i < Q; ++i) out[i] = R_NAN;
            }
            for (int i = 0; i < Q; ++i) fstar[i * plane + site] = out[i];
        }
    }
    return bad;
}

/* Streaming with boundary resolution (pull form of Eq. discrete-rbe):
 * f_i(x, t+1) = f*_i(x - c_i) if the source is a fluid site (after wrapping
 * periodic axes); the fixed contact equilibrium if it lies in a contact's
 * ghost span; otherwise bounce-back, f_i(x, t+1) = f*_opp(i)(x). */
void orc_lattice_stream(const orc_lattice *L, const real *fstar, real *fnew)
{
    const orc_stencil *s = L->st;
    const size_t plane = (size_t)L->nx * L->ny;
#pragma omp parallel for schedule(static)
    for (int y = 0; y < L->ny; ++y) {
        for (int x = 0; x < L->nx; ++x) {
            const size_t site = (size_t)y * L->nx + x;
            if (is_solid(L, x, y)) {
                for (int i = 0; i < Q; ++i) fnew[i * plane + site] = fstar[i * plane + site];
                continue;
            }
            for (int i = 0; i < Q; ++i) {
                int sx = x - s->cx[i], sy = y - s->cy[i];
                if (L->periodic_x) sx = ((sx % L->nx) + L->nx) % L->nx;
                if (L->periodic_y) sy = ((sy % L->ny) + L->ny) % L->ny;
                real v;
                if (sx >= 0 && sx < L->nx && sy >= 0 && sy < L->ny) {
                    if (is_solid(L, sx, sy)) v = fstar[s->opp[i] * plane + site];
                    else v = fstar[i * plane + (size_t)sy * L->nx + sx];
                } else {
                    const int c = contact_at(L, sx, sy);
                    v = (c >= 0) ? L->feq_c[c][i] : fstar[s->opp[i] * plane + site];
                }
                fnew[i * plane + site] = v;
            }
        }
    }
}

/* Advance the pre-collision state f by nsteps steps in place.  With the LCA
 * force on, the collision of f(t) uses grad n of f(t-1) (of f(0) itself at
 * t = 0), which the lattice keeps between calls in n_prev. */
int orc_lattice_run(orc_lattice *L, real *f, int64_t nsteps)
{
    const size_t n = (size_t)Q * L->nx * L->ny;
    const size_t P = (size_t)L->nx * L->ny;
    real *fstar = (real *)malloc(n * sizeof(real));
    if (!fstar) return -2;
    real *ncur = NULL;
    if (L->inv_cg != 0.0) {
        ncur = (real *)malloc(P * sizeof(real));
        if (!ncur || ensure_n_prev(L, f)) { free(fstar); free(ncur); return -2; }
    }
    int bad = 0;
    for (int64_t t = 0; t < nsteps; ++t) {
        if (ncur) density_of(L, f, ncur);
        bad += orc_lattice_collide(L, f, fstar);
        orc_lattice_stream(L, fstar, f);
        if (ncur) memcpy(L->n_prev, ncur, P * sizeof(real));
    }
    free(fstar);
    free(ncur);
    return bad;
}

/* Fields of the pre-collision state: n, vx, vy (3-velocity), eps, T per site. */
int orc_lattice_fields(const orc_lattice *L, const real *f, real *n, real *vx, real *vy,
                       real *eps, real *T)
{
    int bad = 0;
#pragma omp parallel for schedule(static) reduction(+ : bad)
    for (int y = 0; y < L->ny; ++y) {
        real in[Q];
        for (int x = 0; x < L->nx; ++x) {
            const size_t site = (size_t)y * L->nx + x;
            real nn = 0, TT = 0, ee = 0, U[3] = {1, 0, 0};
            if (!is_solid(L, x, y)) {
                get_site(L, f, site, in);
                if (orc_macro(L->st, in, &nn, &TT, &ee, U)) { bad += 1; nn = TT = ee = R_NAN; }
            }
            n[site] = nn; vx[site] = U[1] / U[0]; vy[site] = U[2] / U[0]; eps[site] = ee; T[site] = TT;
        }
    }
    return bad;
}

/* f = f^eq(n, T, v) at every site (initial state). */
void orc_lattice_init(orc_lattice *L, const double *n, const double *T, const double *vx,
                      const double *vy, real *f)
{
    free(L->n_prev);  /* the next collision takes the density of f(0) */
    L->n_prev = NULL;
    const size_t plane = (size_t)L->nx * L->ny;
#pragma omp parallel for schedule(static)
    for (int y = 0; y < L->ny; ++y) {
        real feq[Q];
        for (int x = 0; x < L->nx; ++x) {
            const size_t site = (size_t)y * L->nx + x;
            const real sx = vx[site], sy = vy[site];
            const real g = 1.0 / R_SQRT(1.0 - sx * sx - sy * sy);
            const real U[3] = {g, g * sx, g * sy};
            orc_feq(L->st, n[site], T[site], U, feq);
            for (int i = 0; i < Q; ++i) f[i * plane + site] = feq[i];
        }
    }
}
