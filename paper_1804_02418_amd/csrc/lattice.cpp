// Host runtime of the rlbm C ABI: one lattice = two population buffers, the
// fields, the boundary tables and the per-lattice constants, all on one HIP
// device and ordered on one stream.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/rlbm.h"
#include "rlbm_internal.h"
#include "rlbm_kernels.h"

using namespace rlbm;

namespace {

thread_local std::string g_error;

rlbm_status fail(rlbm_status st, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_error = buf;
    return st;
}

#define HIP_TRY(expr)                                                                              \
    do {                                                                                           \
        hipError_t e_ = (expr);                                                                    \
        if (e_ != hipSuccess) return fail(RLBM_EDEVICE, "%s: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

struct Consts {
    Quadrature q;
    double Cx[kK][kK], Cy[kK][kK];
};

rlbm_status load_constants(Consts *c)
{
    const char *err = nullptr;
    if (!host_constants(&c->q, c->Cx, c->Cy, &err)) return fail(RLBM_EDEVICE, "constants: %s", err ? err : "?");
    // the kernels carry the non-zero entries of C_x, C_y as constants: they
    // must equal this exact computation, and every other entry must vanish
    double tx[kK][kK] = {}, ty[kK][kK] = {};
    for (int q = 0; q < kForceNx; ++q) tx[kForceX[q].k][kForceX[q].m] = kForceX[q].v;
    for (int q = 0; q < kForceNy; ++q) ty[kForceY[q].k][kForceY[q].m] = kForceY[q].v;
    for (int k = 0; k < kK; ++k)
        for (int m = 0; m < kK; ++m)
            if (std::fabs(c->Cx[k][m] - tx[k][m]) > 1e-15 || std::fabs(c->Cy[k][m] - ty[k][m]) > 1e-15)
                return fail(RLBM_EDEVICE, "force matrix entry (%d,%d) differs from the kernel constant", k, m);
    // the reference rest frame has projections only at kRestK
    double a[kK];
    appendix_b(1.3, 0.7, 1.0, 0.0, 0.0, a);
    for (int k = 0; k < kK; ++k) {
        const bool rest = k == kRestK[0] || k == kRestK[1] || k == kRestK[2] || k == kRestK[3];
        if (!rest && a[k] != 0.0) return fail(RLBM_EDEVICE, "rest-frame projection %d is not zero", k);
    }
    return RLBM_OK;
}

size_t store_bytes(rlbm_storage st) { return st == RLBM_F64 ? 8 : st == RLBM_F32 ? 4 : 2; }

// Population value of the equilibrium f^eq_i(n, T, v) (Eq. feq-expansion-discrete) on the host.
void host_feq(const Quadrature &q, double n, double T, double vx, double vy, double out[kQ])
{
    const double g = 1.0 / std::sqrt(1.0 - vx * vx - vy * vy);
    double a[kK], H[kK];
    appendix_b(n, T, g, g * vx, g * vy, a);
    appendix_a_to_harmonics(a, H);
    for (int d = 0; d < kDirs; ++d) {
        for (int j = 0; j < kShells; ++j) {
            const double wj = kGroup[d] ? q.w2[j] : q.w1[j];
            out[4 * d + j] = wj * harmonics_eval(H, q.p0[j], kCx[d] / 5.0, kCy[d] / 5.0);
        }
    }
}

}  // namespace

struct rlbm_lattice {
    int nx = 0, ny = 0;
    rlbm_storage storage = RLBM_F64;
    hipStream_t stream = nullptr;
    Consts C{};
    // parameters
    int periodic_x = 0, periodic_y = 0;
    std::vector<rlbm_contact> contacts;
    std::vector<uint8_t> mask_host;
    double tau = 1.0, Fx = 0.0, Fy = 0.0;
    double n_ref = 1.0, T_ref = 1.0, scale = 1.0;
    // state
    bool initialized = false;
    bool fields_valid = false;
    int64_t t = 0;
    int64_t last_K = 0;
    int cur = 0;
    LaunchShape shape{256, 1};
    // device buffers
    void *pop[2] = {nullptr, nullptr};
    double *fld = nullptr;   // 4 planes: n, vx, vy, eps
    double *prev = nullptr;  // 2 planes: vx, vy of the previous rlbm_step call
    unsigned char *mask = nullptr;
    signed char *edge = nullptr;
    void *contact_eta = nullptr;
    double *part = nullptr;
    int part_blocks = 0;
    double *fref = nullptr, *wscale = nullptr;
    unsigned *gtab = nullptr;  // boundary gather table
    long long gtab_rows = 0;
    // argument blocks (one is used, by storage)
    StepArgs<double> args_d{};
    StepArgs<float> args_f{};

    long long plane() const { return (long long)nx * ny; }
    Store store() const { return storage == RLBM_F64 ? Store::F64 : storage == RLBM_F32 ? Store::F32 : Store::F16; }
    const void *args() const { return storage == RLBM_F64 ? (const void *)&args_d : (const void *)&args_f; }
};

namespace {

template <class R>
void fill_args(rlbm_lattice *L, StepArgs<R> &A)
{
    const Quadrature &q = L->C.q;
    A.nx = L->nx;
    A.ny = L->ny;
    A.periodic_x = L->periodic_x;
    A.periodic_y = L->periodic_y;
    A.has_mask = L->mask != nullptr;
    A.has_force = (L->Fx != 0.0 || L->Fy != 0.0);
    A.write_fields = 0;
    A.plane = L->plane();
    for (int j = 0; j < kShells; ++j) {
        A.wp0[0][j] = R(L->scale * q.w1[j] * q.p0[j]);
        A.wp0[1][j] = R(L->scale * q.w2[j] * q.p0[j]);
        A.wp0sq[0][j] = R(L->scale * q.w1[j] * q.p0[j] * q.p0[j]);
        A.wp0sq[1][j] = R(L->scale * q.w2[j] * q.p0[j] * q.p0[j]);
        A.p0[j] = R(q.p0[j]);
    }
    A.n_ref = L->n_ref;
    A.T_ref = L->T_ref;
    appendix_b(L->n_ref, L->T_ref, 1.0, 0.0, 0.0, A.a_ref);
    A.inv_scale = 1.0 / L->scale;
    A.tau_inv = 1.0 / L->tau;
    A.fx = R(L->Fx);
    A.fy = R(L->Fy);
    for (int r = 0; r < 4; ++r) A.aref_s[r] = R(A.a_ref[kRestK[r]] / L->scale);
    A.mask = L->mask;
    A.edge_contact = L->edge;
    A.gather_tab = L->gtab;
    A.nbnd = L->gtab_rows;
    A.contact_eta = static_cast<const R *>(L->contact_eta);
    A.fn = L->fld;
    A.fvx = L->fld + L->plane();
    A.fvy = L->fld + 2 * L->plane();
    A.feps = L->fld + 3 * L->plane();
}

// Boundary rules of the pull (periodic wrap, then contact span, then
// bounce-back, a solid source also bouncing back) resolved on the host for
// every boundary site: the source element of each population, or a contact
// equilibrium.  Used while 48 * nx * ny fits in 31 bits.
rlbm_status build_gather_table(rlbm_lattice *L, const std::vector<signed char> &edge)
{
    hipFree(L->gtab);
    L->gtab = nullptr;
    L->gtab_rows = 0;
    const long long P = L->plane();
    if (P * kQ >= (1LL << 31)) return RLBM_OK;  // computed gather for huge lattices
    const int nx = L->nx, ny = L->ny;
    const bool all = !has_interior(nx, ny, L->mask != nullptr);
    const long long nb = boundary_count(nx, ny, all);
    std::vector<unsigned> tab((size_t)nb * kQ);
    for (long long b = 0; b < nb; ++b) {
        int x, y;
        boundary_site(b, nx, ny, all, x, y);
        const long long site = (long long)y * nx + x;
        for (int i = 0; i < kQ; ++i) {
            const int d = i / kShells;
            const int o = kShells * ((d + kDirs / 2) % kDirs) + (i % kShells);
            long long sx = x - kCx[d], sy = y - kCy[d];
            if (L->periodic_x) sx = ((sx % nx) + nx) % nx;
            if (L->periodic_y) sy = ((sy % ny) + ny) % ny;
            const bool inside = sx >= 0 && sx < nx && sy >= 0 && sy < ny;
            unsigned code;
            if (inside && !(L->mask && L->mask_host[(size_t)(sy * nx + sx)])) {
                code = (unsigned)(i * P + sy * nx + sx);
            } else {
                int c = -1;
                if (!inside) {
                    if (sy < 0 && sx >= 0 && sx < nx) c = edge[sx];
                    else if (sy >= ny && sx >= 0 && sx < nx) c = edge[nx + sx];
                    else if (sx < 0 && sy >= 0 && sy < ny) c = edge[2 * nx + sy];
                    else if (sx >= nx && sy >= 0 && sy < ny) c = edge[2 * nx + ny + sy];
                }
                code = c >= 0 ? (kContactFlag | (unsigned)(c * kQ + i)) : (unsigned)(o * P + site);
            }
            tab[(size_t)i * nb + b] = code;
        }
    }
    HIP_TRY(hipMalloc((void **)&L->gtab, tab.size() * sizeof(unsigned)));
    HIP_TRY(hipMemcpyAsync(L->gtab, tab.data(), tab.size() * sizeof(unsigned), hipMemcpyHostToDevice, L->stream));
    HIP_TRY(hipStreamSynchronize(L->stream));
    L->gtab_rows = nb;
    return RLBM_OK;
}

// Upload boundary tables (when the geometry changed) and rebuild the kernel
// argument blocks.
rlbm_status refresh(rlbm_lattice *L, bool geometry)
{
    const int nedge = 2 * L->nx + 2 * L->ny;
    std::vector<signed char> edge(nedge, -1);
    for (size_t c = 0; c < L->contacts.size(); ++c) {
        const rlbm_contact &k = L->contacts[c];
        const int base = k.edge == RLBM_EDGE_BOTTOM ? 0 : k.edge == RLBM_EDGE_TOP ? L->nx
                                                      : k.edge == RLBM_EDGE_LEFT ? 2 * L->nx
                                                                                 : 2 * L->nx + L->ny;
        for (int p = k.start; p < k.start + k.width; ++p) edge[base + p] = (signed char)c;
    }
    HIP_TRY(hipMemcpyAsync(L->edge, edge.data(), nedge, hipMemcpyHostToDevice, L->stream));
    if (geometry) {
        rlbm_status gst = build_gather_table(L, edge);
        if (gst) return gst;
    }
    // contact equilibria in storage (eta) units
    double fref[kQ], wsc[kQ];
    host_feq(L->C.q, L->n_ref, L->T_ref, 0.0, 0.0, fref);
    for (int i = 0; i < kQ; ++i) {
        const int d = i / kShells, j = i % kShells;
        wsc[i] = (kGroup[d] ? L->C.q.w2[j] : L->C.q.w1[j]) * L->scale;
    }
    std::vector<double> eta_d(kMaxContacts * kQ, 0.0);
    std::vector<float> eta_f(kMaxContacts * kQ, 0.0f);
    for (size_t c = 0; c < L->contacts.size(); ++c) {
        const rlbm_contact &k = L->contacts[c];
        double feq[kQ];
        host_feq(L->C.q, k.n, k.T, k.vx, k.vy, feq);
        for (int i = 0; i < kQ; ++i) {
            eta_d[c * kQ + i] = (feq[i] - fref[i]) / wsc[i];
            eta_f[c * kQ + i] = (float)eta_d[c * kQ + i];
        }
    }
    if (L->storage == RLBM_F64)
        HIP_TRY(hipMemcpyAsync(L->contact_eta, eta_d.data(), eta_d.size() * 8, hipMemcpyHostToDevice, L->stream));
    else
        HIP_TRY(hipMemcpyAsync(L->contact_eta, eta_f.data(), eta_f.size() * 4, hipMemcpyHostToDevice, L->stream));
    HIP_TRY(hipMemcpyAsync(L->fref, fref, sizeof fref, hipMemcpyHostToDevice, L->stream));
    HIP_TRY(hipMemcpyAsync(L->wscale, wsc, sizeof wsc, hipMemcpyHostToDevice, L->stream));
    // these host arrays go out of scope: finish the copies now
    HIP_TRY(hipStreamSynchronize(L->stream));
    if (L->storage == RLBM_F64)
        fill_args(L, L->args_d);
    else
        fill_args(L, L->args_f);
    return RLBM_OK;
}

void set_write_fields(rlbm_lattice *L, int on)
{
    L->args_d.write_fields = on;
    L->args_f.write_fields = on;
}

LaunchShape default_shape(int nx)
{
    int tx = ((nx - 2 * kReach + 63) / 64) * 64;
    if (tx > 256) tx = 256;
    if (tx < 64) tx = 64;
    if (tx == 192) tx = 128;
    return LaunchShape{tx, 256 / tx};
}

}  // namespace

extern "C" {

const char *rlbm_last_error(void) { return g_error.c_str(); }

int rlbm_version(void) { return 1; }

rlbm_status rlbm_quadrature(double w1[4], double w2[4], double p0[4])
{
    Consts c;
    rlbm_status st = load_constants(&c);
    if (st) return st;
    for (int j = 0; j < 4; ++j) {
        if (w1) w1[j] = c.q.w1[j];
        if (w2) w2[j] = c.q.w2[j];
        if (p0) p0[j] = c.q.p0[j];
    }
    return RLBM_OK;
}

rlbm_status rlbm_force_matrices(double Cx[256], double Cy[256])
{
    Consts c;
    rlbm_status st = load_constants(&c);
    if (st) return st;
    for (int k = 0; k < kK; ++k)
        for (int m = 0; m < kK; ++m) {
            if (Cx) Cx[k * kK + m] = c.Cx[k][m];
            if (Cy) Cy[k * kK + m] = c.Cy[k][m];
        }
    return RLBM_OK;
}

void rlbm_destroy(rlbm_lattice *L)
{
    if (!L) return;
    (void)hipStreamSynchronize(L->stream);
    hipFree(L->pop[0]);
    hipFree(L->pop[1]);
    hipFree(L->fld);
    hipFree(L->prev);
    hipFree(L->mask);
    hipFree(L->edge);
    hipFree(L->contact_eta);
    hipFree(L->part);
    hipFree(L->fref);
    hipFree(L->wscale);
    hipFree(L->gtab);
    delete L;
}

rlbm_status rlbm_create(int nx, int ny, rlbm_storage storage, void *hip_stream, rlbm_lattice **out)
{
    if (!out) return fail(RLBM_EINVAL, "rlbm_create: out is NULL");
    *out = nullptr;
    if (nx < 1 || ny < 1 || (long long)nx * ny > (1LL << 31) - 1)
        return fail(RLBM_EINVAL, "rlbm_create: invalid size %d x %d", nx, ny);
    if (storage != RLBM_F64 && storage != RLBM_F32 && storage != RLBM_F16DEV)
        return fail(RLBM_EINVAL, "rlbm_create: unknown storage %d", (int)storage);
    rlbm_lattice *L = new (std::nothrow) rlbm_lattice();
    if (!L) return fail(RLBM_ENOMEM, "rlbm_create: host allocation failed");
    rlbm_status st = load_constants(&L->C);
    if (st) {
        delete L;
        return st;
    }
    L->nx = nx;
    L->ny = ny;
    L->storage = storage;
    L->stream = static_cast<hipStream_t>(hip_stream);
    L->scale = storage == RLBM_F16DEV ? 1.0 / 4096.0 : 1.0;
    L->shape = default_shape(nx);
    const size_t P = (size_t)nx * ny;
    const size_t pop_bytes = P * kQ * store_bytes(storage);
    L->part_blocks = (int)std::min<size_t>(1024, (P + 255) / 256);
    hipError_t e = hipSuccess;
    auto alloc = [&](void **p, size_t b) {
        if (e == hipSuccess) e = hipMalloc(p, b);
    };
    alloc(&L->pop[0], pop_bytes);
    alloc(&L->pop[1], pop_bytes);
    alloc((void **)&L->fld, 4 * P * sizeof(double));
    alloc((void **)&L->prev, 2 * P * sizeof(double));
    alloc((void **)&L->edge, 2 * nx + 2 * ny);
    alloc(&L->contact_eta, kMaxContacts * kQ * sizeof(double));
    alloc((void **)&L->part, 3 * L->part_blocks * sizeof(double));
    alloc((void **)&L->fref, kQ * sizeof(double));
    alloc((void **)&L->wscale, kQ * sizeof(double));
    if (e == hipSuccess) e = hipMemsetAsync(L->pop[0], 0, pop_bytes, L->stream);
    if (e == hipSuccess) e = hipMemsetAsync(L->pop[1], 0, pop_bytes, L->stream);
    if (e == hipSuccess) e = hipMemsetAsync(L->fld, 0, 4 * P * sizeof(double), L->stream);
    if (e != hipSuccess) {
        rlbm_destroy(L);
        return fail(e == hipErrorOutOfMemory ? RLBM_ENOMEM : RLBM_EDEVICE, "rlbm_create: %s",
                    hipGetErrorString(e));
    }
    st = refresh(L, true);
    if (st) {
        rlbm_destroy(L);
        return st;
    }
    *out = L;
    return RLBM_OK;
}

#define CHECK_L(L)                                                         \
    do {                                                                   \
        if (!(L)) return fail(RLBM_EINVAL, "%s: NULL lattice", __func__); \
    } while (0)

rlbm_status rlbm_set_boundaries(rlbm_lattice *L, int periodic_x, int periodic_y, const rlbm_contact *contacts,
                                int ncontacts)
{
    CHECK_L(L);
    if (ncontacts < 0 || ncontacts > kMaxContacts || (ncontacts > 0 && !contacts))
        return fail(RLBM_EINVAL, "rlbm_set_boundaries: invalid contact count %d", ncontacts);
    for (int c = 0; c < ncontacts; ++c) {
        const rlbm_contact &k = contacts[c];
        if (k.edge < 0 || k.edge > 3) return fail(RLBM_EINVAL, "contact %d: bad edge %d", c, k.edge);
        const bool horiz = k.edge == RLBM_EDGE_BOTTOM || k.edge == RLBM_EDGE_TOP;
        const int len = horiz ? L->nx : L->ny;
        if (k.width < 1 || k.start < 0 || k.start + k.width > len)
            return fail(RLBM_EINVAL, "contact %d: span [%d, %d) outside the edge (length %d)", c, k.start,
                        k.start + k.width, len);
        if ((horiz && periodic_y) || (!horiz && periodic_x))
            return fail(RLBM_EINVAL, "contact %d lies on a periodic edge", c);
        if (!(k.n > 0) || !(k.T > 0) || !(k.vx * k.vx + k.vy * k.vy < 1.0))
            return fail(RLBM_EINVAL, "contact %d: invalid state", c);
        for (int o = 0; o < c; ++o) {
            const rlbm_contact &m = contacts[o];
            if (m.edge == k.edge && m.start < k.start + k.width && k.start < m.start + m.width)
                return fail(RLBM_EINVAL, "contacts %d and %d overlap", o, c);
        }
    }
    L->periodic_x = periodic_x != 0;
    L->periodic_y = periodic_y != 0;
    L->contacts.assign(contacts, contacts + ncontacts);
    return refresh(L, true);
}

rlbm_status rlbm_set_mask(rlbm_lattice *L, const uint8_t *mask)
{
    CHECK_L(L);
    const size_t P = (size_t)L->plane();
    if (!mask) {
        hipFree(L->mask);
        L->mask = nullptr;
        L->mask_host.clear();
        return refresh(L, true);
    }
    if (!L->mask) HIP_TRY(hipMalloc((void **)&L->mask, P));
    L->mask_host.assign(mask, mask + P);
    for (auto &v : L->mask_host) v = v ? 1 : 0;
    HIP_TRY(hipMemcpyAsync(L->mask, L->mask_host.data(), P, hipMemcpyHostToDevice, L->stream));
    return refresh(L, true);
}

rlbm_status rlbm_set_tau(rlbm_lattice *L, double tau)
{
    CHECK_L(L);
    if (!(tau > 0.5) || !std::isfinite(tau)) return fail(RLBM_EINVAL, "rlbm_set_tau: tau must exceed 1/2 (got %g)", tau);
    L->tau = tau;
    return refresh(L, false);
}

rlbm_status rlbm_set_drive(rlbm_lattice *L, double Fx, double Fy)
{
    CHECK_L(L);
    if (!std::isfinite(Fx) || !std::isfinite(Fy)) return fail(RLBM_EINVAL, "rlbm_set_drive: non-finite force");
    L->Fx = Fx;
    L->Fy = Fy;
    return refresh(L, false);
}

rlbm_status rlbm_set_reference(rlbm_lattice *L, double n_ref, double T_ref, double scale)
{
    CHECK_L(L);
    if (!(n_ref > 0) || !(T_ref > 0) || !(scale > 0) || !std::isfinite(n_ref + T_ref + scale))
        return fail(RLBM_EINVAL, "rlbm_set_reference: invalid reference");
    L->n_ref = n_ref;
    L->T_ref = T_ref;
    L->scale = scale;
    L->initialized = false;
    L->fields_valid = false;
    return refresh(L, false);
}

static rlbm_status do_init(rlbm_lattice *L, const double *n, const double *T, const double *vx, const double *vy,
                           const double u[4])
{
    L->cur = 0;
    HIP_TRY(launch_init(L->store(), L->args(), n, T, vx, vy, u, L->pop[0], L->stream));
    // the state after init holds f*(0); its fields are those of f(0)
    HIP_TRY(hipMemcpyAsync(L->prev, L->fld + L->plane(), 2 * L->plane() * sizeof(double), hipMemcpyDeviceToDevice,
                           L->stream));
    L->initialized = true;
    L->fields_valid = true;
    L->t = 0;
    L->last_K = 0;
    return RLBM_OK;
}

rlbm_status rlbm_init_uniform(rlbm_lattice *L, double n, double T, double vx, double vy)
{
    CHECK_L(L);
    if (!(n > 0) || !(T > 0) || !(vx * vx + vy * vy < 1.0)) return fail(RLBM_EINVAL, "rlbm_init_uniform: invalid state");
    const double u[4] = {n, T, vx, vy};
    return do_init(L, nullptr, nullptr, nullptr, nullptr, u);
}

rlbm_status rlbm_init_fields(rlbm_lattice *L, const double *n, const double *T, const double *vx, const double *vy,
                             int on_device)
{
    CHECK_L(L);
    if (!n || !T || !vx || !vy) return fail(RLBM_EINVAL, "rlbm_init_fields: NULL field");
    const size_t bytes = (size_t)L->plane() * sizeof(double);
    const double u[4] = {1, 1, 0, 0};
    if (on_device) return do_init(L, n, T, vx, vy, u);
    // stage the host fields through the field planes (each init thread reads its own site before writing it)
    double *dn = L->fld, *dvx = L->fld + L->plane(), *dvy = L->fld + 2 * L->plane(), *dT = L->fld + 3 * L->plane();
    HIP_TRY(hipMemcpyAsync(dn, n, bytes, hipMemcpyHostToDevice, L->stream));
    HIP_TRY(hipMemcpyAsync(dvx, vx, bytes, hipMemcpyHostToDevice, L->stream));
    HIP_TRY(hipMemcpyAsync(dvy, vy, bytes, hipMemcpyHostToDevice, L->stream));
    HIP_TRY(hipMemcpyAsync(dT, T, bytes, hipMemcpyHostToDevice, L->stream));
    rlbm_status st = do_init(L, dn, dT, dvx, dvy, u);
    if (st) return st;
    HIP_TRY(hipStreamSynchronize(L->stream));
    return RLBM_OK;
}

rlbm_status rlbm_step(rlbm_lattice *L, int64_t nsteps)
{
    CHECK_L(L);
    if (!L->initialized) return fail(RLBM_ESTATE, "rlbm_step: lattice not initialised");
    if (nsteps < 0) return fail(RLBM_EINVAL, "rlbm_step: negative step count");
    if (nsteps == 0) return RLBM_OK;
    HIP_TRY(hipMemcpyAsync(L->prev, L->fld + L->plane(), 2 * L->plane() * sizeof(double), hipMemcpyDeviceToDevice,
                           L->stream));
    for (int64_t k = 0; k < nsteps; ++k) {
        set_write_fields(L, k == nsteps - 1);
        HIP_TRY(launch_step(L->store(), L->args(), L->pop[L->cur], L->pop[1 - L->cur], L->shape, L->stream));
        L->cur ^= 1;
    }
    set_write_fields(L, 0);
    L->t += nsteps;
    L->last_K = nsteps;
    L->fields_valid = true;
    return RLBM_OK;
}

rlbm_status rlbm_get_time(rlbm_lattice *L, int64_t *t)
{
    CHECK_L(L);
    if (!t) return fail(RLBM_EINVAL, "rlbm_get_time: NULL");
    *t = L->t;
    return RLBM_OK;
}

rlbm_status rlbm_read_fields(rlbm_lattice *L, double *n, double *vx, double *vy, double *eps, int on_device)
{
    CHECK_L(L);
    if (!L->fields_valid) return fail(RLBM_ESTATE, "rlbm_read_fields: no fields yet (initialise or step first)");
    const size_t P = (size_t)L->plane();
    double *dst[4] = {n, vx, vy, eps};
    const hipMemcpyKind kind = on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
    for (int f = 0; f < 4; ++f)
        if (dst[f]) HIP_TRY(hipMemcpyAsync(dst[f], L->fld + f * P, P * sizeof(double), kind, L->stream));
    if (!on_device) HIP_TRY(hipStreamSynchronize(L->stream));
    return RLBM_OK;
}

static rlbm_status residual_sums(rlbm_lattice *L, double *dv, double *vv, double *bad)
{
    const size_t P = (size_t)L->plane();
    HIP_TRY(launch_residual((int)P, L->mask, L->fld, L->fld + P, L->fld + 2 * P, L->prev, L->prev + P, L->part,
                            L->part_blocks, L->stream));
    std::vector<double> h(3 * L->part_blocks);
    HIP_TRY(hipMemcpyAsync(h.data(), L->part, h.size() * sizeof(double), hipMemcpyDeviceToHost, L->stream));
    HIP_TRY(hipStreamSynchronize(L->stream));
    *dv = *vv = *bad = 0;
    for (int b = 0; b < L->part_blocks; ++b) {
        *dv += h[3 * b];
        *vv += h[3 * b + 1];
        *bad += h[3 * b + 2];
    }
    return RLBM_OK;
}

rlbm_status rlbm_residual(rlbm_lattice *L, double *r)
{
    CHECK_L(L);
    if (!r) return fail(RLBM_EINVAL, "rlbm_residual: NULL");
    if (!L->fields_valid) return fail(RLBM_ESTATE, "rlbm_residual: no fields");
    double dv, vv, bad;
    rlbm_status st = residual_sums(L, &dv, &vv, &bad);
    if (st) return st;
    const double K = L->last_K > 0 ? (double)L->last_K : 1.0;
    *r = vv > 0 ? std::sqrt(dv) / (K * std::sqrt(vv)) : 0.0;
    if (bad > 0 || !std::isfinite(*r))
        return fail(RLBM_EUNSTABLE, "health check: %.0f unhealthy sites at step %lld", bad, (long long)L->t);
    return RLBM_OK;
}

rlbm_status rlbm_step_until(rlbm_lattice *L, int64_t max_steps, int64_t check_every, double tol, int64_t *steps_taken,
                            double *residual)
{
    CHECK_L(L);
    if (check_every < 1 || max_steps < 0) return fail(RLBM_EINVAL, "rlbm_step_until: invalid counts");
    int64_t done = 0;
    double r = INFINITY;
    while (done < max_steps) {
        const int64_t k = std::min<int64_t>(check_every, max_steps - done);
        rlbm_status st = rlbm_step(L, k);
        if (st) return st;
        done += k;
        st = rlbm_residual(L, &r);
        if (st) {
            if (steps_taken) *steps_taken = done;
            if (residual) *residual = r;
            return st;
        }
        if (k == check_every && r < tol) break;
    }
    if (steps_taken) *steps_taken = done;
    if (residual) *residual = r;
    return RLBM_OK;
}

rlbm_status rlbm_read_populations(rlbm_lattice *L, double *f, int on_device)
{
    CHECK_L(L);
    if (!f) return fail(RLBM_EINVAL, "rlbm_read_populations: NULL");
    if (!L->initialized) return fail(RLBM_ESTATE, "rlbm_read_populations: not initialised");
    const size_t bytes = (size_t)L->plane() * kQ * sizeof(double);
    if (on_device) {
        HIP_TRY(launch_decode(L->store(), L->nx, L->ny, L->pop[L->cur], L->fref, L->wscale, f, L->stream));
        return RLBM_OK;
    }
    double *tmp = nullptr;
    HIP_TRY(hipMalloc((void **)&tmp, bytes));
    hipError_t e = launch_decode(L->store(), L->nx, L->ny, L->pop[L->cur], L->fref, L->wscale, tmp, L->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(f, tmp, bytes, hipMemcpyDeviceToHost, L->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(L->stream);
    hipFree(tmp);
    if (e != hipSuccess) return fail(RLBM_EDEVICE, "rlbm_read_populations: %s", hipGetErrorString(e));
    return RLBM_OK;
}

namespace {
struct StateHeader {
    uint64_t magic;
    int32_t version, nx, ny, storage;
    int64_t t, last_K;
    double n_ref, T_ref, scale;
    int32_t fields_valid, pad;
};
constexpr uint64_t kMagic = 0x524c424d53544154ull;  // "RLBMSTAT"
}  // namespace

rlbm_status rlbm_state_bytes(rlbm_lattice *L, size_t *bytes)
{
    CHECK_L(L);
    if (!bytes) return fail(RLBM_EINVAL, "rlbm_state_bytes: NULL");
    const size_t P = (size_t)L->plane();
    *bytes = sizeof(StateHeader) + P * kQ * store_bytes(L->storage) + 6 * P * sizeof(double);
    return RLBM_OK;
}

rlbm_status rlbm_get_state(rlbm_lattice *L, void *dst, size_t bytes)
{
    CHECK_L(L);
    size_t need;
    rlbm_state_bytes(L, &need);
    if (!dst || bytes < need) return fail(RLBM_EINVAL, "rlbm_get_state: buffer too small (%zu < %zu)", bytes, need);
    if (!L->initialized) return fail(RLBM_ESTATE, "rlbm_get_state: not initialised");
    const size_t P = (size_t)L->plane();
    StateHeader h{kMagic, 1, L->nx, L->ny, (int32_t)L->storage, L->t, L->last_K, L->n_ref, L->T_ref, L->scale,
                  L->fields_valid ? 1 : 0, 0};
    char *p = static_cast<char *>(dst);
    std::memcpy(p, &h, sizeof h);
    p += sizeof h;
    const size_t pb = P * kQ * store_bytes(L->storage);
    HIP_TRY(hipMemcpyAsync(p, L->pop[L->cur], pb, hipMemcpyDeviceToHost, L->stream));
    p += pb;
    HIP_TRY(hipMemcpyAsync(p, L->fld, 4 * P * sizeof(double), hipMemcpyDeviceToHost, L->stream));
    p += 4 * P * sizeof(double);
    HIP_TRY(hipMemcpyAsync(p, L->prev, 2 * P * sizeof(double), hipMemcpyDeviceToHost, L->stream));
    HIP_TRY(hipStreamSynchronize(L->stream));
    return RLBM_OK;
}

rlbm_status rlbm_set_state(rlbm_lattice *L, const void *src, size_t bytes)
{
    CHECK_L(L);
    size_t need;
    rlbm_state_bytes(L, &need);
    if (!src || bytes < need) return fail(RLBM_EINVAL, "rlbm_set_state: buffer too small");
    StateHeader h;
    std::memcpy(&h, src, sizeof h);
    if (h.magic != kMagic || h.version != 1 || h.nx != L->nx || h.ny != L->ny || h.storage != (int32_t)L->storage)
        return fail(RLBM_EINVAL, "rlbm_set_state: state does not match this lattice");
    if (h.n_ref != L->n_ref || h.T_ref != L->T_ref || h.scale != L->scale) {
        L->n_ref = h.n_ref;
        L->T_ref = h.T_ref;
        L->scale = h.scale;
        rlbm_status st = refresh(L, false);
        if (st) return st;
    }
    const size_t P = (size_t)L->plane();
    const char *p = static_cast<const char *>(src) + sizeof h;
    const size_t pb = P * kQ * store_bytes(L->storage);
    L->cur = 0;
    HIP_TRY(hipMemcpyAsync(L->pop[0], p, pb, hipMemcpyHostToDevice, L->stream));
    p += pb;
    HIP_TRY(hipMemcpyAsync(L->fld, p, 4 * P * sizeof(double), hipMemcpyHostToDevice, L->stream));
    p += 4 * P * sizeof(double);
    HIP_TRY(hipMemcpyAsync(L->prev, p, 2 * P * sizeof(double), hipMemcpyHostToDevice, L->stream));
    HIP_TRY(hipStreamSynchronize(L->stream));
    L->t = h.t;
    L->last_K = h.last_K;
    L->initialized = true;
    L->fields_valid = h.fields_valid != 0;
    return RLBM_OK;
}

rlbm_status rlbm_set_launch_shape(rlbm_lattice *L, int tile_x, int rows)
{
    CHECK_L(L);
    if (tile_x < 64 || tile_x % 64 || rows < 1 || tile_x * rows != 256)
        return fail(RLBM_EINVAL, "rlbm_set_launch_shape: invalid shape %d x %d", tile_x, rows);
    L->shape = LaunchShape{tile_x, rows};
    return RLBM_OK;
}

rlbm_status rlbm_synchronize(rlbm_lattice *L)
{
    CHECK_L(L);
    HIP_TRY(hipStreamSynchronize(L->stream));
    return RLBM_OK;
}

}  // extern "C"
