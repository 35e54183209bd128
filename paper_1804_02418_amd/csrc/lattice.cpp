// Host runtime of the rlbm C ABI: one lattice = two population buffers, the
// fields, the boundary tables and the per-lattice constants, all on one HIP
// device and ordered on one stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <tuple>
#include <string>
#include <vector>

#include "../../include/rlbm.h"
#include "rlbm_internal.h"
#include "rlbm_kernels.h"

using namespace rlbm;

namespace {

thread_local std::string g_error;

// release paths ignore HIP errors on purpose (nothing useful can be done)
inline void dfree(void *p) { (void)hipFree(p); }

}  // namespace

namespace rlbm {
// Error reporting shared by the other translation units of the library.
rlbm_status set_error(rlbm_status st, const char *msg)
{
    g_error = msg ? msg : "";
    return st;
}
}  // namespace rlbm

namespace {

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
        if (e_ != hipSuccess)                                                                      \
            return fail(e_ == hipErrorOutOfMemory ? RLBM_ENOMEM : RLBM_EDEVICE, "%s: %s", #expr,   \
                        hipGetErrorString(e_));                                                    \
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
    int device = 0;  // the HIP device current at rlbm_create
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
    int nt_store = 0;  // streaming (non-temporal) population stores
    int nt_load = 0;   // non-temporal interior population loads
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
    bool table_off = false;    // rlbm_set_gather_table(0): never build one
    // local-capacitance force: 1/C_g (0: off) and the density ping-pong,
    // nlca[ncur] holding the density of the current state
    double inv_cg = 0.0;
    double *nlca[2] = {nullptr, nullptr};
    int ncur = 0;
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
    A.nt_store = L->nt_store;
    A.nt_load = L->nt_load;
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
    A.side_contacts = 0;
    for (const rlbm_contact &k : L->contacts)
        A.side_contacts |= k.edge == RLBM_EDGE_LEFT ? 1 : k.edge == RLBM_EDGE_RIGHT ? 2 : 0;
    A.gather_tab = L->gtab;
    A.nbnd = L->gtab_rows;
    A.contact_eta = static_cast<const R *>(L->contact_eta);
    A.fn = L->fld;
    A.fvx = L->fld + L->plane();
    A.fvy = L->fld + 2 * L->plane();
    A.feps = L->fld + 3 * L->plane();
    A.inv_cg = L->inv_cg;
    A.n_prev = L->inv_cg != 0.0 ? L->nlca[L->ncur] : nullptr;
    A.n_next = L->inv_cg != 0.0 ? L->nlca[L->ncur ^ 1] : nullptr;
}

// Point the local-capacitance density buffers of both argument blocks at
// (n_prev, n_next).
void set_lca_buffers(rlbm_lattice *L, const double *n_prev, double *n_next)
{
    L->args_d.n_prev = L->args_f.n_prev = n_prev;
    L->args_d.n_next = L->args_f.n_next = n_next;
}

// Boundary rules of the pull (periodic wrap, then contact span, then
// bounce-back, a solid source also bouncing back) resolved on the host for
// every boundary site: the source element of each population, or a contact
// equilibrium.  Used while 48 * nx * ny fits in 31 bits.
rlbm_status build_gather_table(rlbm_lattice *L, const std::vector<signed char> &edge)
{
    dfree(L->gtab);
    L->gtab = nullptr;
    L->gtab_rows = 0;
    const long long P = L->plane();
    // computed gather for huge lattices: table codes are 31-bit element
    // indices, and the kernels that read a table address every population
    // as a 32-bit byte offset from the array
    if (L->table_off || P * kQ >= (1LL << 31) || P * kQ * (long long)store_bytes(L->storage) >= (1LL << 32))
        return RLBM_OK;
    const int nx = L->nx, ny = L->ny;
    const int w = tuple_width((int)store_bytes(L->storage));
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
                code = (unsigned)pop_elem(w, i, sy * nx + sx, P);
            } else {
                int c = -1;
                if (!inside) {
                    if (sy < 0 && sx >= 0 && sx < nx) c = edge[sx];
                    else if (sy >= ny && sx >= 0 && sx < nx) c = edge[nx + sx];
                    else if (sx < 0 && sy >= 0 && sy < ny) c = edge[2 * nx + sy];
                    else if (sx >= nx && sy >= 0 && sy < ny) c = edge[2 * nx + ny + sy];
                }
                code = c >= 0 ? (kContactFlag | (unsigned)(c * kQ + i)) : (unsigned)pop_elem(w, o, site, P);
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

// bit 0: streaming stores, bit 1: non-temporal interior loads
void set_memory_form(rlbm_lattice *L, int form)
{
    L->nt_store = form & 1;
    L->nt_load = (form >> 1) & 1;
    L->args_d.nt_store = L->args_f.nt_store = L->nt_store;
    L->args_d.nt_load = L->args_f.nt_load = L->nt_load;
}

void set_write_fields(rlbm_lattice *L, int on)
{
    L->args_d.write_fields = on;
    L->args_f.write_fields = on;
}

// ---- autotune cache: (arch, storage, nx, ny, mask) -> tile_x and memory
// form (bit 0: streaming stores, bit 1: non-temporal loads) ----
using TuneKey = std::tuple<std::string, int, int, int, int>;
struct TuneVal {
    int tile_x, form;
};
std::mutex g_tune_mu;
std::map<TuneKey, TuneVal> g_tune;
bool g_tune_loaded = false;

std::string device_arch()
{
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) return "unknown";
    std::string a = prop.gcnArchName;
    const size_t colon = a.find(':');
    return colon == std::string::npos ? a : a.substr(0, colon);
}

void tune_cache_load()
{
    if (g_tune_loaded) return;
    g_tune_loaded = true;
    const char *path = std::getenv("RLBM_TUNE_CACHE");
    if (!path) return;
    FILE *f = std::fopen(path, "r");
    if (!f) return;
    // one entry per line: arch storage nx ny mask tile_x form; lines of
    // another shape or with values out of range are skipped
    char line[256], arch[64];
    int st, nx, ny, mask, tile, form;
    while (std::fgets(line, sizeof line, f)) {
        if (std::sscanf(line, "%63s %d %d %d %d %d %d", arch, &st, &nx, &ny, &mask, &tile, &form) != 7) continue;
        if ((tile != 64 && tile != 128 && tile != 256) || form < 0 || form > 3) continue;
        g_tune[TuneKey(arch, st, nx, ny, mask)] = TuneVal{tile, form};
    }
    std::fclose(f);
}

void tune_cache_store(const TuneKey &k, TuneVal v)
{
    g_tune[k] = v;
    const char *path = std::getenv("RLBM_TUNE_CACHE");
    if (!path) return;
    FILE *f = std::fopen(path, "a");
    if (!f) return;
    std::fprintf(f, "%s %d %d %d %d %d %d\n", std::get<0>(k).c_str(), std::get<1>(k), std::get<2>(k), std::get<3>(k),
                 std::get<4>(k), v.tile_x, v.form);
    std::fclose(f);
}

LaunchShape default_shape(int nx)
{
    int tx = ((nx + 63) / 64) * 64;  // interior tiles span whole rows
    if (tx > 256) tx = 256;
    if (tx < 64) tx = 64;
    if (tx == 192) tx = 128;
    return LaunchShape{tx, 256 / tx};
}

}  // namespace

extern "C" {

const char *rlbm_last_error(void) { return g_error.c_str(); }

int rlbm_version(void) { return 2; }

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
    dfree(L->pop[0]);
    dfree(L->pop[1]);
    dfree(L->fld);
    dfree(L->prev);
    dfree(L->mask);
    dfree(L->edge);
    dfree(L->contact_eta);
    dfree(L->part);
    dfree(L->fref);
    dfree(L->wscale);
    dfree(L->gtab);
    dfree(L->nlca[0]);
    dfree(L->nlca[1]);
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
    if ((long long)nx * ny * (long long)store_bytes(storage) * tuple_width((int)store_bytes(storage)) >= (1LL << 32))
        return fail(RLBM_EINVAL, "rlbm_create: one population plane (tuple array) of %d x %d exceeds 4 GiB", nx, ny);
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
    if (hipGetDevice(&L->device) != hipSuccess) {
        delete L;
        return fail(RLBM_EDEVICE, "rlbm_create: no current HIP device");
    }
    L->scale = storage == RLBM_F16DEV ? 1.0 / 4096.0 : 1.0;
    L->shape = default_shape(nx);
    // populations that outgrow the 256 MB Infinity Cache are streamed
    L->nt_store = 2.0 * (double)nx * ny * kQ * store_bytes(storage) > 256.0 * 1024 * 1024 ? 1 : 0;
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        tune_cache_load();
        auto it = g_tune.find(TuneKey(device_arch(), (int)storage, nx, ny, 0));
        if (it != g_tune.end()) {
            L->shape = LaunchShape{it->second.tile_x, 256 / it->second.tile_x};
            L->nt_store = it->second.form & 1;
            L->nt_load = (it->second.form >> 1) & 1;
        }
    }
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
        if (k.width < 1 || k.start < 0 || (long long)k.start + k.width > len)
            return fail(RLBM_EINVAL, "contact %d: span [%d, %d) outside the edge (length %d)", c, k.start,
                        k.start + k.width, len);
        if ((horiz && periodic_y) || (!horiz && periodic_x))
            return fail(RLBM_EINVAL, "contact %d lies on a periodic edge", c);
        if (!(k.n > 0) || !(k.T > 0) || !(k.vx * k.vx + k.vy * k.vy < 1.0) || !std::isfinite(k.n + k.T))
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
        dfree(L->mask);
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

rlbm_status rlbm_set_lca(rlbm_lattice *L, double inv_cg)
{
    CHECK_L(L);
    if (!std::isfinite(inv_cg) || inv_cg < 0.0)
        return fail(RLBM_EINVAL, "rlbm_set_lca: 1/C_g must be finite and >= 0 (got %g)", inv_cg);
    if (inv_cg != 0.0 && !L->nlca[0]) {
        const size_t b = (size_t)L->plane() * sizeof(double);
        HIP_TRY(hipMalloc((void **)&L->nlca[0], b));
        HIP_TRY(hipMalloc((void **)&L->nlca[1], b));
    }
    if (inv_cg != 0.0 && L->inv_cg == 0.0 && L->initialized) {
        // switched on mid-run: the previous density is that of the current state
        if (!L->fields_valid) return fail(RLBM_ESTATE, "rlbm_set_lca: the current state has no fields");
        L->ncur = 0;
        HIP_TRY(hipMemcpyAsync(L->nlca[0], L->fld, (size_t)L->plane() * sizeof(double), hipMemcpyDeviceToDevice,
                               L->stream));
    }
    L->inv_cg = inv_cg;
    return refresh(L, false);
}

rlbm_status rlbm_set_quadrature(rlbm_lattice *L, const double w1[4], const double w2[4], const double p0[4])
{
    CHECK_L(L);
    if (!w1 || !w2 || !p0) return fail(RLBM_EINVAL, "rlbm_set_quadrature: NULL table");
    Quadrature q;
    for (int j = 0; j < 4; ++j) {
        if (!(w1[j] >= 0) || !(w2[j] >= 0) || !(p0[j] > 0) || !std::isfinite(w1[j] + w2[j] + p0[j]))
            return fail(RLBM_EINVAL, "rlbm_set_quadrature: weights must be >= 0 and energies > 0");
        q.w1[j] = w1[j];
        q.w2[j] = w2[j];
        q.p0[j] = p0[j];
    }
    const double res = massless_stencil_residual(q);
    if (!(res < 1e-12))
        return fail(RLBM_EINVAL, "rlbm_set_quadrature: the orthonormality conditions fail by %.3g", res);
    L->C.q = q;
    L->initialized = false;
    L->fields_valid = false;
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
    if (L->inv_cg != 0.0) {
        // the collision of f(0) takes grad n of f(0) itself: its density first
        L->ncur = 0;
        set_lca_buffers(L, nullptr, L->nlca[0]);
        HIP_TRY(launch_init(L->store(), L->args(), n, T, vx, vy, u, L->pop[0], kInitDensity, L->stream));
        set_lca_buffers(L, L->nlca[0], L->nlca[1]);
        HIP_TRY(launch_init(L->store(), L->args(), n, T, vx, vy, u, L->pop[0], kInitLca, L->stream));
    } else {
        HIP_TRY(launch_init(L->store(), L->args(), n, T, vx, vy, u, L->pop[0], kInitPlain, L->stream));
    }
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
    if (!(n > 0) || !(T > 0) || !(vx * vx + vy * vy < 1.0) || !std::isfinite(n + T))
        return fail(RLBM_EINVAL, "rlbm_init_uniform: invalid state");
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
    const bool lca = L->inv_cg != 0.0;
    for (int64_t k = 0; k < nsteps; ++k) {
        set_write_fields(L, k == nsteps - 1);
        if (lca) set_lca_buffers(L, L->nlca[L->ncur], L->nlca[L->ncur ^ 1]);
        const hipError_t e = launch_step(L->store(), L->args(), L->pop[L->cur], L->pop[1 - L->cur], L->shape, L->stream);
        if (e != hipSuccess) {
            // the k steps launched before stand; the fields are not those of the state
            set_write_fields(L, 0);
            L->t += k;
            L->last_K = k;
            L->fields_valid = false;
            return fail(RLBM_EDEVICE, "rlbm_step: step %lld of %lld: %s", (long long)k, (long long)nsteps,
                        hipGetErrorString(e));
        }
        L->cur ^= 1;
        if (lca) L->ncur ^= 1;
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

rlbm_status rlbm_residual_noalloc(rlbm_lattice *L, double *r)
{
    CHECK_L(L);
    if (!r) return fail(RLBM_EINVAL, "rlbm_residual_noalloc: NULL");
    if (!L->fields_valid) return fail(RLBM_ESTATE, "rlbm_residual_noalloc: no fields");
    if (L->part_blocks > kNoAllocResidualBlocks)
        return fail(RLBM_EINVAL, "rlbm_residual_noalloc: %d partial sums exceed the scratch of %d", L->part_blocks,
                    kNoAllocResidualBlocks);
    int dev = -1;
    HIP_TRY(hipGetDevice(&dev));
    if (dev != L->device)
        return fail(RLBM_ESTATE, "rlbm_residual_noalloc: the lattice lives on device %d but device %d is current",
                    L->device, dev);
    const size_t P = (size_t)L->plane();
    double tot[3];
    HIP_TRY(launch_residual_noalloc((int)P, L->mask, L->fld, L->fld + P, L->fld + 2 * P, L->prev, L->prev + P,
                                    L->part_blocks, tot, L->stream));
    const double K = L->last_K > 0 ? (double)L->last_K : 1.0;
    *r = tot[1] > 0 ? std::sqrt(tot[0]) / (K * std::sqrt(tot[1])) : 0.0;
    if (tot[2] > 0 || !std::isfinite(*r))
        return fail(RLBM_EUNSTABLE, "health check: %.0f unhealthy sites at step %lld", tot[2], (long long)L->t);
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
    dfree(tmp);
    if (e != hipSuccess) return fail(RLBM_EDEVICE, "rlbm_read_populations: %s", hipGetErrorString(e));
    return RLBM_OK;
}

namespace {
struct StateHeader {
    uint64_t magic;
    int32_t version, nx, ny, storage;
    int64_t t, last_K;
    double n_ref, T_ref, scale;
    int32_t fields_valid, lca;  // lca: the density of the current state follows the fields
};
constexpr uint64_t kMagic = 0x524c424d53544154ull;  // "RLBMSTAT"
}  // namespace

rlbm_status rlbm_state_bytes(rlbm_lattice *L, size_t *bytes)
{
    CHECK_L(L);
    if (!bytes) return fail(RLBM_EINVAL, "rlbm_state_bytes: NULL");
    const size_t P = (size_t)L->plane();
    *bytes = sizeof(StateHeader) + P * kQ * store_bytes(L->storage) + (L->inv_cg != 0.0 ? 7 : 6) * P * sizeof(double);
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
    const int lca = L->inv_cg != 0.0 ? 1 : 0;
    StateHeader h{kMagic, 1, L->nx, L->ny, (int32_t)L->storage, L->t, L->last_K, L->n_ref, L->T_ref, L->scale,
                  L->fields_valid ? 1 : 0, lca};
    char *p = static_cast<char *>(dst);
    std::memcpy(p, &h, sizeof h);
    p += sizeof h;
    const size_t pb = P * kQ * store_bytes(L->storage);
    HIP_TRY(hipMemcpyAsync(p, L->pop[L->cur], pb, hipMemcpyDeviceToHost, L->stream));
    p += pb;
    HIP_TRY(hipMemcpyAsync(p, L->fld, 4 * P * sizeof(double), hipMemcpyDeviceToHost, L->stream));
    p += 4 * P * sizeof(double);
    HIP_TRY(hipMemcpyAsync(p, L->prev, 2 * P * sizeof(double), hipMemcpyDeviceToHost, L->stream));
    p += 2 * P * sizeof(double);
    if (lca) HIP_TRY(hipMemcpyAsync(p, L->nlca[L->ncur], P * sizeof(double), hipMemcpyDeviceToHost, L->stream));
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
    if (h.lca != (L->inv_cg != 0.0 ? 1 : 0))
        return fail(RLBM_EINVAL, "rlbm_set_state: the state was saved with the local-capacitance force %s",
                    h.lca ? "on" : "off");
    if (!(h.n_ref > 0) || !(h.T_ref > 0) || !(h.scale > 0) || !std::isfinite(h.n_ref + h.T_ref + h.scale) || h.t < 0 ||
        h.last_K < 0)
        return fail(RLBM_EINVAL, "rlbm_set_state: corrupt header");
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
    p += 2 * P * sizeof(double);
    if (h.lca) {
        L->ncur = 0;
        HIP_TRY(hipMemcpyAsync(L->nlca[0], p, P * sizeof(double), hipMemcpyHostToDevice, L->stream));
    }
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
    L->shape = LaunchShape{tile_x, rows, L->shape.xcd};
    return RLBM_OK;
}

rlbm_status rlbm_get_launch_shape(rlbm_lattice *L, int *tile_x, int *rows)
{
    CHECK_L(L);
    if (tile_x) *tile_x = L->shape.tile_x;
    if (rows) *rows = L->shape.rows;
    return RLBM_OK;
}

rlbm_status rlbm_autotune(rlbm_lattice *L, int trial_steps, double *ms_per_step)
{
    CHECK_L(L);
    if (!L->initialized) return fail(RLBM_ESTATE, "rlbm_autotune: lattice not initialised");
    if (trial_steps < 1) return fail(RLBM_EINVAL, "rlbm_autotune: trial_steps must be >= 1");
    const size_t P = (size_t)L->plane();
    const size_t pb = P * kQ * store_bytes(L->storage);
    // save the state (current populations, fields, previous velocities)
    void *save = nullptr;
    HIP_TRY(hipMalloc(&save, pb + 7 * P * sizeof(double)));
    char *sv = static_cast<char *>(save);
    const int cur0 = L->cur, ncur0 = L->ncur;
    const bool lca = L->inv_cg != 0.0;
    const int64_t t0 = L->t, k0 = L->last_K;
    const bool fv0 = L->fields_valid;
    const LaunchShape shape0 = L->shape;
    hipError_t e = hipMemcpyAsync(sv, L->pop[cur0], pb, hipMemcpyDeviceToDevice, L->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(sv + pb, L->fld, 4 * P * sizeof(double), hipMemcpyDeviceToDevice, L->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(sv + pb + 4 * P * sizeof(double), L->prev, 2 * P * sizeof(double), hipMemcpyDeviceToDevice,
                           L->stream);
    if (e == hipSuccess && lca)
        e = hipMemcpyAsync(sv + pb + 6 * P * sizeof(double), L->nlca[ncur0], P * sizeof(double),
                           hipMemcpyDeviceToDevice, L->stream);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (e == hipSuccess) e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    const int tiles[3] = {64, 128, 256};
    double best = INFINITY;
    const int form0 = L->nt_store | (L->nt_load << 1);
    int best_tile = shape0.tile_x, best_form = form0;
    const int interior_w = L->nx;  // interior tiles span whole rows
    // candidate c: tile tiles[c % 3], memory form c / 3 (bit 0: streaming
    // stores, bit 1: non-temporal loads).  Two rounds, the second in the
    // reverse order, each candidate keeping the faster of its two runs: one
    // slow run (or the position in the sequence) does not decide.
    double per_c[12];
    for (int c = 0; c < 12; ++c) per_c[c] = INFINITY;
    for (int k = 0; k < 24 && e == hipSuccess; ++k) {
        const int c = k < 12 ? k : 23 - k;
        const int tc = c % 3, form = c / 3;
        if (tc > 0 && tiles[tc - 1] >= interior_w) continue;  // wider tiles only add idle lanes
        L->shape = LaunchShape{tiles[tc], 256 / tiles[tc], shape0.xcd};
        set_memory_form(L, form);
        rlbm_status st = rlbm_step(L, 2);
        if (st == RLBM_OK) e = hipEventRecord(e0, L->stream);
        if (st == RLBM_OK && e == hipSuccess) st = rlbm_step(L, trial_steps);
        if (st == RLBM_OK && e == hipSuccess) e = hipEventRecord(e1, L->stream);
        if (st == RLBM_OK && e == hipSuccess) e = hipEventSynchronize(e1);
        float ms = 0;
        if (st == RLBM_OK && e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
        if (st != RLBM_OK) {
            e = hipErrorUnknown;
            break;
        }
        per_c[c] = std::min(per_c[c], (double)ms / trial_steps);
    }
    for (int c = 0; c < 12; ++c) {
        if (ms_per_step) ms_per_step[c] = std::isfinite(per_c[c]) ? per_c[c] : 0.0;
        if (per_c[c] < best) {
            best = per_c[c];
            best_tile = tiles[c % 3];
            best_form = c / 3;
        }
    }
    // the setting on entry stays unless the fastest candidate beats it by
    // more than 1%: closer than that, short trials do not rank two settings
    // reliably (they run at other clocks than a long run does)
    for (int tc = 0; tc < 3; ++tc) {
        const int c0 = form0 * 3 + tc;
        if (tiles[tc] == shape0.tile_x && std::isfinite(per_c[c0]) && best >= 0.99 * per_c[c0]) {
            best_tile = shape0.tile_x;
            best_form = form0;
        }
    }
    // restore
    L->cur = cur0;
    if (e == hipSuccess) e = hipMemcpyAsync(L->pop[cur0], sv, pb, hipMemcpyDeviceToDevice, L->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(L->fld, sv + pb, 4 * P * sizeof(double), hipMemcpyDeviceToDevice, L->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(L->prev, sv + pb + 4 * P * sizeof(double), 2 * P * sizeof(double), hipMemcpyDeviceToDevice,
                           L->stream);
    L->ncur = ncur0;
    if (e == hipSuccess && lca)
        e = hipMemcpyAsync(L->nlca[ncur0], sv + pb + 6 * P * sizeof(double), P * sizeof(double),
                           hipMemcpyDeviceToDevice, L->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(L->stream);
    dfree(save);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    L->t = t0;
    L->last_K = k0;
    L->fields_valid = fv0;
    if (e != hipSuccess) {
        L->shape = shape0;
        set_memory_form(L, form0);
        return fail(RLBM_EDEVICE, "rlbm_autotune: %s", hipGetErrorString(e));
    }
    L->shape = LaunchShape{best_tile, 256 / best_tile, shape0.xcd};
    set_memory_form(L, best_form);
    std::lock_guard<std::mutex> lk(g_tune_mu);
    tune_cache_store(TuneKey(device_arch(), (int)L->storage, L->nx, L->ny, L->mask ? 1 : 0),
                     TuneVal{best_tile, best_form});
    return RLBM_OK;
}

rlbm_status rlbm_set_block_order(rlbm_lattice *L, int xcd_contiguous)
{
    CHECK_L(L);
    if (xcd_contiguous != 0 && xcd_contiguous != 1) return fail(RLBM_EINVAL, "rlbm_set_block_order: 0 or 1");
    L->shape.xcd = xcd_contiguous;
    return RLBM_OK;
}

rlbm_status rlbm_set_gather_table(rlbm_lattice *L, int enabled)
{
    CHECK_L(L);
    if (enabled != 0 && enabled != 1) return fail(RLBM_EINVAL, "rlbm_set_gather_table: 0 or 1");
    L->table_off = enabled == 0;
    return refresh(L, true);
}

rlbm_status rlbm_set_streaming_stores(rlbm_lattice *L, int on)
{
    CHECK_L(L);
    set_memory_form(L, (on ? 1 : 0) | (L->nt_load << 1));
    return RLBM_OK;
}

rlbm_status rlbm_set_streaming_loads(rlbm_lattice *L, int on)
{
    CHECK_L(L);
    set_memory_form(L, L->nt_store | ((on ? 1 : 0) << 1));
    return RLBM_OK;
}

rlbm_status rlbm_get_memory_form(rlbm_lattice *L, int *streaming_stores, int *nontemporal_loads)
{
    CHECK_L(L);
    if (streaming_stores) *streaming_stores = L->nt_store;
    if (nontemporal_loads) *nontemporal_loads = L->nt_load;
    return RLBM_OK;
}

rlbm_status rlbm_synchronize(rlbm_lattice *L)
{
    CHECK_L(L);
    HIP_TRY(hipStreamSynchronize(L->stream));
    return RLBM_OK;
}


}  // extern "C"

// ---------------------------------------------------------------- batch

struct rlbm_batch {
    std::vector<rlbm_lattice *> lat;
    std::vector<uint8_t> active;
    rlbm_storage storage = RLBM_F64;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    void *descs = nullptr;      // BatchDesc<R>[n]
    unsigned *items = nullptr;  // work list
    size_t items_cap = 0;
    int *n_items = nullptr;
    int n_items_host = 0;
    int xcd = 0;  // XCD-contiguous item order
    int nt = 0;   // streaming stores (every active sample has them on)
    double *part = nullptr;
    int part_blocks = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    static constexpr int kGraphSteps = 32;
};

namespace {

int step_blocks(const rlbm_lattice *L, int *nbnd, int *tiles_x, int *all)
{
    const bool interior = has_interior(L->nx, L->ny, L->mask != nullptr);
    *all = interior ? 0 : 1;
    const long long nb = boundary_count(L->nx, L->ny, !interior);
    *nbnd = (int)((nb + 255) / 256);
    *tiles_x = 0;
    int tiles = 0;
    if (interior) {
        const int rows = 256 / L->shape.tile_x;
        *tiles_x = (L->nx + L->shape.tile_x - 1) / L->shape.tile_x;
        tiles = *tiles_x * ((L->ny - 2 * kReach + rows - 1) / rows);
    }
    return *nbnd + tiles;
}

void drop_graph(rlbm_batch *B)
{
    if (B->exec) (void)hipGraphExecDestroy(B->exec);
    if (B->graph) (void)hipGraphDestroy(B->graph);
    B->exec = nullptr;
    B->graph = nullptr;
}

template <class R>
rlbm_status upload_descs_t(rlbm_batch *B)
{
    const int n = (int)B->lat.size();
    std::vector<BatchDesc<R>> d(n);
    std::vector<unsigned> items;
    bool nt_all = true;
    for (int s = 0; s < n; ++s) {
        rlbm_lattice *L = B->lat[s];
        BatchDesc<R> &D = d[s];
        D.a = *static_cast<const StepArgs<R> *>(L->args());
        D.a.write_fields = 0;
        D.pop[0] = L->pop[0];
        D.pop[1] = L->pop[1];
        D.pvx = L->prev;
        D.pvy = L->prev + L->plane();
        const int nblk = step_blocks(L, &D.nbnd, &D.tiles_x, &D.all);
        D.tile_x = L->shape.tile_x;
        D.parity_xor = L->cur;  // launches start at parity 0
        D.pad_ = 0;
        if (!B->active[s]) continue;
        nt_all = nt_all && L->nt_store;
        for (int b = 0; b < nblk; ++b) items.push_back(((unsigned)s << kItemBlockBits) | (unsigned)b);
    }
    if ((nt_all ? 1 : 0) != B->nt) {
        drop_graph(B);  // the captured graph holds the other store form
        B->nt = nt_all ? 1 : 0;
    }
    HIP_TRY(hipMemcpyAsync(B->descs, d.data(), n * sizeof(BatchDesc<R>), hipMemcpyHostToDevice, B->stream));
    if (items.size() > B->items_cap) {
        // the launch grid is the capacity: a captured graph holds the old one
        drop_graph(B);
        dfree(B->items);
        B->items = nullptr;
        HIP_TRY(hipMalloc((void **)&B->items, items.size() * sizeof(unsigned)));
        B->items_cap = items.size();
    }
    if (!items.empty())
        HIP_TRY(hipMemcpyAsync(B->items, items.data(), items.size() * sizeof(unsigned), hipMemcpyHostToDevice,
                               B->stream));
    B->n_items_host = (int)items.size();
    HIP_TRY(hipMemcpyAsync(B->n_items, &B->n_items_host, sizeof(int), hipMemcpyHostToDevice, B->stream));
    HIP_TRY(hipStreamSynchronize(B->stream));  // host vectors go out of scope
    return RLBM_OK;
}

rlbm_status upload_descs(rlbm_batch *B)
{
    return B->storage == RLBM_F64 ? upload_descs_t<double>(B) : upload_descs_t<float>(B);
}

Store store_of(rlbm_storage st) { return st == RLBM_F64 ? Store::F64 : st == RLBM_F32 ? Store::F32 : Store::F16; }

rlbm_status batch_launch(rlbm_batch *B, int parity, int wf)
{
    HIP_TRY(launch_batch_step(store_of(B->storage), B->descs, B->items, B->n_items, (int)B->items_cap, parity, wf,
                              B->xcd, B->nt, B->stream));
    return RLBM_OK;
}

rlbm_status ensure_graph(rlbm_batch *B)
{
    if (B->exec) return RLBM_OK;
    HIP_TRY(hipStreamBeginCapture(B->stream, hipStreamCaptureModeThreadLocal));
    rlbm_status st = RLBM_OK;
    for (int k = 0; k < rlbm_batch::kGraphSteps && st == RLBM_OK; ++k) st = batch_launch(B, k & 1, 0);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(B->stream, &g);
    if (st) {
        if (g) (void)hipGraphDestroy(g);
        return st;
    }
    if (e != hipSuccess) return fail(RLBM_EDEVICE, "graph capture: %s", hipGetErrorString(e));
    B->graph = g;
    e = hipGraphInstantiate(&B->exec, B->graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        // keep no half-built graph: the next call captures afresh
        (void)hipGraphDestroy(B->graph);
        B->graph = nullptr;
        B->exec = nullptr;
        return fail(RLBM_EDEVICE, "graph instantiation: %s", hipGetErrorString(e));
    }
    return RLBM_OK;
}

}  // namespace

extern "C" {

void rlbm_batch_destroy(rlbm_batch *B)
{
    if (!B) return;
    if (B->stream) (void)hipStreamSynchronize(B->stream);
    if (B->exec) (void)hipGraphExecDestroy(B->exec);
    if (B->graph) (void)hipGraphDestroy(B->graph);
    for (rlbm_lattice *L : B->lat) rlbm_destroy(L);
    dfree(B->descs);
    dfree(B->items);
    dfree(B->n_items);
    dfree(B->part);
    if (B->own_stream && B->stream) (void)hipStreamDestroy(B->stream);
    delete B;
}

rlbm_status rlbm_batch_create(const rlbm_sample *samples, int nsamples, rlbm_storage storage, void *hip_stream,
                              rlbm_batch **out)
{
    if (!out) return fail(RLBM_EINVAL, "rlbm_batch_create: out is NULL");
    *out = nullptr;
    if (!samples || nsamples < 1 || nsamples >= (1 << (32 - kItemBlockBits)))
        return fail(RLBM_EINVAL, "rlbm_batch_create: invalid sample count %d", nsamples);
    rlbm_batch *B = new (std::nothrow) rlbm_batch();
    if (!B) return fail(RLBM_ENOMEM, "rlbm_batch_create: host allocation failed");
    B->storage = storage;
    if (hip_stream) {
        B->stream = static_cast<hipStream_t>(hip_stream);
    } else {
        hipError_t e = hipStreamCreateWithFlags(&B->stream, hipStreamNonBlocking);
        if (e != hipSuccess) {
            delete B;
            return fail(RLBM_EDEVICE, "rlbm_batch_create: %s", hipGetErrorString(e));
        }
        B->own_stream = true;
    }
    rlbm_status st = RLBM_OK;
    for (int s = 0; s < nsamples && st == RLBM_OK; ++s) {
        const rlbm_sample &q = samples[s];
        if (q.ncontacts < 0 || q.ncontacts > 4) {
            st = fail(RLBM_EINVAL, "sample %d: at most 4 contacts", s);
            break;
        }
        rlbm_lattice *L = nullptr;
        st = rlbm_create(q.nx, q.ny, storage, B->stream, &L);
        if (st) break;
        B->lat.push_back(L);
        // default tiles: 256 x 1 where the width is a whole number of them,
        // else 64 x 4 (no idle wave at the end of a row, and a block's four
        // waves pull from four adjacent rows that share source lines in L1)
        L->shape = q.nx % 256 == 0 ? LaunchShape{256, 1} : LaunchShape{64, 4};
        int nblk_dummy[3];
        if (step_blocks(L, &nblk_dummy[0], &nblk_dummy[1], &nblk_dummy[2]) >= (1 << kItemBlockBits)) {
            st = fail(RLBM_EINVAL, "sample %d is too large for the batched work list", s);
            break;
        }
        st = rlbm_set_boundaries(L, q.periodic_x, q.periodic_y, q.contacts, q.ncontacts);
        if (!st) st = rlbm_set_tau(L, q.tau);
        if (!st) st = rlbm_set_drive(L, q.Fx, q.Fy);
        if (!st) st = rlbm_init_uniform(L, q.n0, q.T0, q.vx0, q.vy0);
        if (st) g_error = "sample " + std::to_string(s) + ": " + g_error;
    }
    B->active.assign(nsamples, 1);
    if (!st) {
        // the batch streams all its samples each step: once their populations
        // together outgrow the 256 MB Infinity Cache, streaming stores by default
        double bytes = 0.0;
        for (rlbm_lattice *L : B->lat) bytes += 2.0 * (double)L->plane() * kQ * store_bytes(storage);
        if (bytes > 256.0 * 1024 * 1024)
            for (rlbm_lattice *L : B->lat) rlbm_set_streaming_stores(L, 1);
    }
    const size_t desc_bytes = nsamples * (storage == RLBM_F64 ? sizeof(BatchDesc<double>) : sizeof(BatchDesc<float>));
    hipError_t e = hipSuccess;
    if (!st) e = hipMalloc(&B->descs, desc_bytes);
    if (!st && e == hipSuccess) e = hipMalloc((void **)&B->n_items, sizeof(int));
    B->part_blocks = 8;
    if (!st && e == hipSuccess) e = hipMalloc((void **)&B->part, (size_t)nsamples * B->part_blocks * 3 * sizeof(double));
    if (!st && e != hipSuccess) st = fail(RLBM_EDEVICE, "rlbm_batch_create: %s", hipGetErrorString(e));
    if (!st) st = upload_descs(B);
    if (st) {
        rlbm_batch_destroy(B);
        return st;
    }
    *out = B;
    return RLBM_OK;
}

rlbm_status rlbm_batch_lattice(rlbm_batch *B, int i, rlbm_lattice **lat)
{
    if (!B || !lat || i < 0 || i >= (int)B->lat.size()) return fail(RLBM_EINVAL, "rlbm_batch_lattice: bad argument");
    *lat = B->lat[i];
    return RLBM_OK;
}

rlbm_status rlbm_batch_set_block_order(rlbm_batch *B, int xcd_contiguous)
{
    if (!B || (xcd_contiguous != 0 && xcd_contiguous != 1))
        return fail(RLBM_EINVAL, "rlbm_batch_set_block_order: bad argument");
    if (B->xcd != xcd_contiguous) drop_graph(B);  // the captured graph holds the old order
    B->xcd = xcd_contiguous;
    return RLBM_OK;
}

rlbm_status rlbm_batch_sites(rlbm_batch *B, int64_t *sites)
{
    if (!B || !sites) return fail(RLBM_EINVAL, "rlbm_batch_sites: bad argument");
    int64_t n = 0;
    for (size_t s = 0; s < B->lat.size(); ++s)
        if (B->active[s]) n += B->lat[s]->plane();
    *sites = n;
    return RLBM_OK;
}

rlbm_status rlbm_batch_set_active(rlbm_batch *B, const uint8_t *active)
{
    if (!B || !active) return fail(RLBM_EINVAL, "rlbm_batch_set_active: bad argument");
    for (size_t s = 0; s < B->lat.size(); ++s) B->active[s] = active[s] ? 1 : 0;
    return RLBM_OK;
}

rlbm_status rlbm_batch_step(rlbm_batch *B, int64_t nsteps, int use_graph)
{
    if (!B) return fail(RLBM_EINVAL, "rlbm_batch_step: NULL batch");
    if (nsteps < 0) return fail(RLBM_EINVAL, "rlbm_batch_step: negative step count");
    if (nsteps == 0) return RLBM_OK;
    for (size_t s = 0; s < B->lat.size(); ++s)
        if (B->active[s] && B->lat[s]->inv_cg != 0.0)
            return fail(RLBM_EINVAL, "rlbm_batch_step: sample %zu has the local-capacitance force on (step it alone)", s);
    // descriptors reflect each sample's current buffer, shape and parameters
    rlbm_status st = upload_descs(B);
    if (st) return st;
    for (size_t s = 0; s < B->lat.size(); ++s) {
        rlbm_lattice *L = B->lat[s];
        if (!B->active[s]) continue;
        if (!L->initialized) return fail(RLBM_ESTATE, "rlbm_batch_step: sample %zu not initialised", s);
        HIP_TRY(hipMemcpyAsync(L->prev, L->fld + L->plane(), 2 * L->plane() * sizeof(double), hipMemcpyDeviceToDevice,
                               B->stream));
    }
    if (B->n_items_host > 0) {
        int64_t done = 0;
        const int64_t body = nsteps - 1;  // the last step writes fields
        if (use_graph && body >= rlbm_batch::kGraphSteps) {
            st = ensure_graph(B);
            if (st) return st;
            for (; done + rlbm_batch::kGraphSteps <= body; done += rlbm_batch::kGraphSteps)
                HIP_TRY(hipGraphLaunch(B->exec, B->stream));
        }
        for (; done < body; ++done) {
            st = batch_launch(B, (int)(done & 1), 0);
            if (st) return st;
        }
        st = batch_launch(B, (int)(done & 1), 1);
        if (st) return st;
    }
    for (size_t s = 0; s < B->lat.size(); ++s) {
        if (!B->active[s]) continue;
        rlbm_lattice *L = B->lat[s];
        L->cur ^= (int)(nsteps & 1);
        L->t += nsteps;
        L->last_K = nsteps;
        L->fields_valid = true;
    }
    return RLBM_OK;
}

rlbm_status rlbm_batch_residual(rlbm_batch *B, double *r)
{
    if (!B || !r) return fail(RLBM_EINVAL, "rlbm_batch_residual: bad argument");
    const int n = (int)B->lat.size();
    HIP_TRY(launch_batch_residual(store_of(B->storage), B->descs, n, B->part_blocks, B->part, B->stream));
    std::vector<double> h((size_t)n * B->part_blocks * 3);
    HIP_TRY(hipMemcpyAsync(h.data(), B->part, h.size() * sizeof(double), hipMemcpyDeviceToHost, B->stream));
    HIP_TRY(hipStreamSynchronize(B->stream));
    double bad_total = 0;
    for (int s = 0; s < n; ++s) {
        double dv = 0, vv = 0, bad = 0;
        for (int j = 0; j < B->part_blocks; ++j) {
            const double *p = &h[((size_t)s * B->part_blocks + j) * 3];
            dv += p[0];
            vv += p[1];
            bad += p[2];
        }
        const double K = B->lat[s]->last_K > 0 ? (double)B->lat[s]->last_K : 1.0;
        r[s] = vv > 0 ? std::sqrt(dv) / (K * std::sqrt(vv)) : 0.0;
        bad_total += bad;
    }
    if (bad_total > 0) return fail(RLBM_EUNSTABLE, "health check: %.0f unhealthy sites in the batch", bad_total);
    return RLBM_OK;
}

rlbm_status rlbm_batch_step_until(rlbm_batch *B, int64_t max_steps, int64_t check_every, double tol, int64_t *steps,
                                  double *r)
{
    if (!B || check_every < 1 || max_steps < 0) return fail(RLBM_EINVAL, "rlbm_batch_step_until: bad argument");
    const int n = (int)B->lat.size();
    std::vector<int64_t> taken(n, 0);
    std::vector<double> res(n, INFINITY), cur(n);
    std::vector<uint8_t> act = B->active;
    int64_t done = 0;
    rlbm_status st = RLBM_OK;
    while (done < max_steps) {
        bool any = false;
        for (int s = 0; s < n; ++s) any = any || act[s];
        if (!any) break;
        const int64_t k = std::min<int64_t>(check_every, max_steps - done);
        rlbm_batch_set_active(B, act.data());
        st = rlbm_batch_step(B, k, 1);
        if (st) break;
        done += k;
        st = rlbm_batch_residual(B, cur.data());
        for (int s = 0; s < n; ++s) {
            if (!act[s]) continue;
            taken[s] += k;
            res[s] = cur[s];
            if (k == check_every && cur[s] < tol) act[s] = 0;
        }
        if (st) break;
    }
    std::vector<uint8_t> all(n, 1);
    rlbm_batch_set_active(B, all.data());
    for (int s = 0; s < n; ++s) {
        if (steps) steps[s] = taken[s];
        if (r) r[s] = res[s];
    }
    return st;
}

rlbm_status rlbm_batch_autotune(rlbm_batch *B, int trial_steps, double *ms_per_step)
{
    if (!B || trial_steps < 1) return fail(RLBM_EINVAL, "rlbm_batch_autotune: bad argument");
    const int n = (int)B->lat.size();
    // save every sample's state on the device: current populations, fields, previous velocities
    std::vector<size_t> off(n + 1, 0);
    for (int s = 0; s < n; ++s) {
        const rlbm_lattice *L = B->lat[s];
        off[s + 1] = off[s] + (size_t)L->plane() * (kQ * store_bytes(L->storage) + 6 * sizeof(double));
    }
    char *save = nullptr;
    HIP_TRY(hipMalloc((void **)&save, off[n]));
    std::vector<int> cur0(n);
    std::vector<int64_t> t0(n), k0(n);
    for (int s = 0; s < n; ++s) {
        rlbm_lattice *L = B->lat[s];
        const size_t P = (size_t)L->plane(), pb = P * kQ * store_bytes(L->storage);
        cur0[s] = L->cur;
        t0[s] = L->t;
        k0[s] = L->last_K;
        HIP_TRY(hipMemcpyAsync(save + off[s], L->pop[L->cur], pb, hipMemcpyDeviceToDevice, B->stream));
        HIP_TRY(hipMemcpyAsync(save + off[s] + pb, L->fld, 4 * P * 8, hipMemcpyDeviceToDevice, B->stream));
        HIP_TRY(hipMemcpyAsync(save + off[s] + pb + 4 * P * 8, L->prev, 2 * P * 8, hipMemcpyDeviceToDevice, B->stream));
    }
    std::vector<LaunchShape> shape0(n);
    for (int s = 0; s < n; ++s) shape0[s] = B->lat[s]->shape;
    const int tiles[3] = {64, 128, 256};
    hipEvent_t e0 = nullptr, e1 = nullptr;
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    rlbm_status st = RLBM_OK;
    std::vector<int> nt0(n);
    for (int s = 0; s < n; ++s) nt0[s] = B->lat[s]->nt_store;
    // ms per step of the current setting: the faster of two timed runs
    // (each after two untimed steps), so that one slow run does not decide
    auto trial = [&](double &per) {
        per = INFINITY;
        for (int rep = 0; rep < 2 && st == RLBM_OK; ++rep) {
            st = rlbm_batch_step(B, 2, 0);
            if (st) break;
            (void)hipEventRecord(e0, B->stream);
            st = rlbm_batch_step(B, trial_steps, 0);
            if (st) break;
            (void)hipEventRecord(e1, B->stream);
            (void)hipEventSynchronize(e1);
            float ms = 0;
            (void)hipEventElapsedTime(&ms, e0, e1);
            per = std::min(per, (double)ms / trial_steps);
        }
    };
    auto capped = [](int t, int w) {
        while (t > 64 && t / 2 >= w) t /= 2;
        return t;
    };
    // stage 1: one tile width (capped at each sample's width) and store form
    // for every sample; the entry setting is left only for a candidate more
    // than 1% faster
    double best = INFINITY;
    int best_c = -1;  // -1: the shapes and store forms the samples had on entry
    for (int c = -1; c < 6 && st == RLBM_OK; ++c) {
        if (c >= 0) {
            for (int s = 0; s < n; ++s) {
                B->lat[s]->shape = LaunchShape{capped(tiles[c % 3], B->lat[s]->nx), 256 / capped(tiles[c % 3], B->lat[s]->nx)};
                rlbm_set_streaming_stores(B->lat[s], c / 3);
            }
        }
        double per = INFINITY;
        trial(per);
        if (st) break;
        if (ms_per_step && c >= 0) ms_per_step[c] = per;
        if (per < (best_c == -1 ? 0.99 * best : best)) {
            best = per;
            best_c = c;
        }
    }
    std::vector<LaunchShape> shape1(n);
    std::vector<int> nt1(n);
    for (int s = 0; s < n; ++s) {
        if (best_c >= 0) {
            const int t = capped(tiles[best_c % 3], B->lat[s]->nx);
            shape1[s] = LaunchShape{t, 256 / t};
            nt1[s] = best_c / 3;
        } else {
            shape1[s] = shape0[s];
            nt1[s] = nt0[s];
        }
    }
    // stage 2: per width class (a multiple of 256; of 128 only; anything
    // else), each width that tiles the class's rows exactly, the other
    // classes held at their best; a change needs more than 1% to be kept
    auto cls = [](int w) { return w % 256 == 0 ? 0 : w % 128 == 0 ? 1 : 2; };
    for (int k = 0; k < 3 && st == RLBM_OK; ++k) {
        bool present = false;
        for (int s = 0; s < n; ++s) present = present || cls(B->lat[s]->nx) == k;
        if (!present) continue;
        for (int ti = 0; ti < 3 && st == RLBM_OK; ++ti) {
            const int t = tiles[ti];
            if ((k == 1 && t == 256) || (k == 2 && t != 64)) continue;
            bool same = true;
            for (int s = 0; s < n; ++s) {
                const bool mine = cls(B->lat[s]->nx) == k;
                const int ts = mine ? capped(t, B->lat[s]->nx) : shape1[s].tile_x;
                same = same && (!mine || ts == shape1[s].tile_x);
                B->lat[s]->shape = mine ? LaunchShape{ts, 256 / ts} : shape1[s];
                rlbm_set_streaming_stores(B->lat[s], nt1[s]);
            }
            if (same) continue;
            double per = INFINITY;
            trial(per);
            if (st) break;
            if (per < 0.99 * best) {
                best = per;
                for (int s = 0; s < n; ++s) shape1[s] = B->lat[s]->shape;
            }
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    for (int s = 0; s < n; ++s) {
        rlbm_lattice *L = B->lat[s];
        const size_t P = (size_t)L->plane(), pb = P * kQ * store_bytes(L->storage);
        L->cur = cur0[s];
        L->t = t0[s];
        L->last_K = k0[s];
        hipError_t e = hipMemcpyAsync(L->pop[L->cur], save + off[s], pb, hipMemcpyDeviceToDevice, B->stream);
        if (e == hipSuccess) e = hipMemcpyAsync(L->fld, save + off[s] + pb, 4 * P * 8, hipMemcpyDeviceToDevice, B->stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync(L->prev, save + off[s] + pb + 4 * P * 8, 2 * P * 8, hipMemcpyDeviceToDevice, B->stream);
        if (e != hipSuccess && !st) st = fail(RLBM_EDEVICE, "rlbm_batch_autotune: restore: %s", hipGetErrorString(e));
        L->shape = st ? shape0[s] : shape1[s];
        rlbm_set_streaming_stores(L, st ? nt0[s] : nt1[s]);
    }
    {
        hipError_t e = hipStreamSynchronize(B->stream);
        if (e != hipSuccess && !st) st = fail(RLBM_EDEVICE, "rlbm_batch_autotune: %s", hipGetErrorString(e));
    }
    dfree(save);
    drop_graph(B);
    return st;
}

}  // extern "C"
