// gfx950 kernels of the fused relativistic LB step (templates; each
// storage is instantiated in a translation unit of its own).
//
// Storage: 48 SoA planes of nx*ny values, plane i = population i = 4*d + j
// (float16: 12 arrays of four-shell direction tuples, see tuple_width),
// holding the post-collision state f*(t) as the scaled deviation eta_i from
// the reference rest equilibrium.  One step reads f*(t) from src and writes
// f*(t+1) to dst (ping-pong), so every stored value is read exactly once
// and written exactly once per step: the step is bound by HBM bandwidth.
//
// Work mapping: one thread per site; a block covers tile_x consecutive
// sites of `rows` rows, so each wavefront reads 64 consecutive values of a
// plane row (shifted by the hop) and writes 64 aligned values.  Waves whose
// 5-site halo lies inside the lattice (and without a solid mask) take a
// branch-free gather; the others resolve periodic wrap, contact ghost spans
// and bounce-back per lane (side columns and the top and bottom bands), or
// through a host-built table (lattices with a solid mask).
#pragma once

#include "rlbm_kernels.h"

namespace rlbm {
namespace {

template <class S>
struct StoreIO;
template <>
struct StoreIO<double> {
    template <class R, class P>
    __device__ static R load(P p) { return R(*p); }
    template <class R, class P>
    __device__ static void store(P p, R v) { *p = double(v); }
    template <class R, class P>
    __device__ static void store_nt(P p, R v) { __builtin_nontemporal_store(double(v), p); }
};
template <>
struct StoreIO<float> {
    template <class R, class P>
    __device__ static R load(P p) { return R(*p); }
    template <class R, class P>
    __device__ static void store(P p, R v) { *p = float(v); }
    template <class R, class P>
    __device__ static void store_nt(P p, R v) { __builtin_nontemporal_store(float(v), p); }
};
template <>
struct StoreIO<_Float16> {
    template <class R, class P>
    __device__ static R load(P p) { return R(float(*p)); }
    template <class R, class P>
    __device__ static void store(P p, R v) { *p = _Float16(float(v)); }
    template <class R, class P>
    __device__ static void store_nt(P p, R v) { __builtin_nontemporal_store(_Float16(float(v)), p); }
};

// Tuple of the four shells of one direction (float16 storage).
typedef _Float16 half4 __attribute__((ext_vector_type(4)));
template <class S>
constexpr int kTup = tuple_width((int)sizeof(S));

struct SiteFields {
    double n, u0, ux, uy, eps;  // density, Landau 4-velocity, energy density
};

// Element `site` of a plane given by a uniform base pointer, addressed as
// that base (held in scalar registers) plus a 32-bit byte offset, in the
// global address space: one vector offset then serves every plane, instead
// of a 64-bit address per lane and plane.  The empty asm only pins the base
// to scalar registers (it keeps the compiler from folding the per-plane
// bases into per-lane addresses).  Planes stay below 4 GiB (the library
// rejects larger lattices).
template <class T>
__device__ __forceinline__ __attribute__((address_space(1))) T *plane_at(T *base, unsigned site)
{
    asm("" : "+s"(base));
    typedef __attribute__((address_space(1))) T GT;
    typedef __attribute__((address_space(1))) const char GC;
    return (GT *)((GC *)base + site * (unsigned)sizeof(T));
}

// The same from a byte offset held in a register.  The stores of the step
// come after the Landau solve's branches, in other basic blocks than the
// one that formed the site's offset, and there the compiler sees only a
// 64-bit value and forms a 64-bit address per lane and store (48 vector
// instructions per site).  The caller passes the offset through an empty
// asm in the store's own block, so that it is a fresh 32-bit value there and
// the store takes the scalar-base plus 32-bit-offset form.
template <class T>
__device__ __forceinline__ __attribute__((address_space(1))) T *plane_at_bytes(T *base, unsigned byte_offset)
{
    asm("" : "+s"(base));
    typedef __attribute__((address_space(1))) T GT;
    typedef __attribute__((address_space(1))) const char GC;
    return (GT *)((GC *)base + byte_offset);
}

// Reciprocal and reciprocal square root in float64 from the hardware
// estimates (about 23 correct bits) and two Newton steps each, which leave
// a few units in the last place: the Landau solve and the density factors
// need no correctly rounded division.
struct DeviceRecip {
    __device__ double rcp(double x) const
    {
        double r = __builtin_amdgcn_rcp(x);
        r = fma(fma(-x, r, 1.0), r, r);
        return fma(fma(-x, r, 1.0), r, r);
    }
    __device__ double rsqrt(double x) const
    {
        const double h = 0.5 * x;
        double r = __builtin_amdgcn_rsq(x);
        r *= fma(-h * r, r, 1.5);
        return r * fma(-h * r, r, 1.5);
    }
};

// Discards the post-collision values (callers that read h afterwards).
struct NoEmit {
    template <class R>
    __device__ void operator()(int, R, const R *, const R *) const {}
};

// Two float16 values a * h0 + q0 and a * h1 + q1, each rounded once from
// the exact a * h + q (mixed-precision FMA), packed low / high in 32 bits.
// Written out so that every kernel rounds alike: left to the compiler,
// some values became an FMA rounded to float32 and then converted (two
// roundings), differently in different kernels.
__device__ __forceinline__ unsigned fma_pack_f16(float a, float h0, float q0, float h1, float q1)
{
    // the low half is written first (the high half it leaves is overwritten next)
    unsigned r;
    asm("v_fma_mixlo_f16 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(h0), "v"(q0));
    asm("v_fma_mixhi_f16 %0, %1, %2, %3" : "+v"(r) : "v"(a), "v"(h1), "v"(q1));
    return r;
}

// Stores the four post-collision values v of direction d of one site into
// the population array dst (P sites per plane or tuple array): four plane
// elements, or one tuple in float16 storage.  site_bytes is the site's
// offset in bytes within one plane, or within one tuple array (site times
// sizeof(S) times the tuple width).
template <class S, class R, bool NT>
__device__ __forceinline__ void store_dir(S *__restrict__ dst, long long P, int d, unsigned site_bytes, R a,
                                          const R *h, const R *q)
{
    if constexpr (kTup<S> == kShells) {
        typedef unsigned u32x2 __attribute__((ext_vector_type(2)));
        const u32x2 t = {fma_pack_f16(a, h[0], q[0], h[1], q[1]), fma_pack_f16(a, h[2], q[2], h[3], q[3])};
        auto p = plane_at_bytes(reinterpret_cast<u32x2 *>(dst) + (long long)d * P, site_bytes);
        if constexpr (NT)
            __builtin_nontemporal_store(t, p);
        else
            *p = t;
    } else {
#pragma unroll
        for (int j = 0; j < kShells; ++j) {
            auto p = plane_at_bytes(dst + (long long)(kShells * d + j) * P, site_bytes);
            const R v = a * h[j] + q[j];
            if constexpr (NT)
                StoreIO<S>::template store_nt<R>(p, v);
            else
                StoreIO<S>::template store<R>(p, v);
        }
    }
}
// Discards the site's fields.
struct NoFields {
    __device__ void operator()(const SiteFields &, bool) const {}
};

// Collision of one site, in place on the 48 scaled deviations h.
// Steps: moments -> Landau frame -> n, T -> Appendix B projections ->
// equilibrium and forcing polynomials -> relaxation with
// omega_d = p_i.U / (p0_i tau) = (U^0 - nhat_d . U_s) / tau.
// fields(f, ok) receives the site's fields right after the Landau frame and
// emit(d, a, h, q) the four post-collision values of direction d,
// a * h[j] + q[j] for shell j (a = 1 - omega_d, h the pre-collision values),
// as soon as their terms are formed, so a caller that stores them lets their
// registers die early; h itself is left as it was.
template <class R, class Emit = NoEmit, class Fields = NoFields>
__device__ __forceinline__ bool collide_site(R (&h)[kQ], const StepArgs<R> &A, R fx, R fy, bool has_force,
                                             const Emit &emit = Emit(), const Fields &fields = Fields())
{
    // ---- moments of the deviation, one pair of opposite directions at a time ----
    R N0 = 0, Nx = 0, Ny = 0, T00 = 0, T0x = 0, T0y = 0, Txx = 0, Txy = 0, Tyy = 0;
#pragma unroll
    for (int d = 0; d < kDirs / 2; ++d) {
        const int g = kGroup[d];
        R a1 = 0, a2 = 0, b1 = 0, b2 = 0;
#pragma unroll
        for (int j = 0; j < kShells; ++j) {
            a1 += A.wp0[g][j] * h[4 * d + j];
            a2 += A.wp0[g][j] * h[4 * (d + 6) + j];
            b1 += A.wp0sq[g][j] * h[4 * d + j];
            b2 += A.wp0sq[g][j] * h[4 * (d + 6) + j];
        }
        const DirTrig tg = dir_trig(d);
        const R c = R(tg.c), s = R(tg.s);
        const R Ae = a1 + a2, Ao = a1 - a2, Be = b1 + b2, Bo = b1 - b2;
        N0 += Ae;
        Nx += Ao * c;
        Ny += Ao * s;
        T00 += Be;
        T0x += Bo * c;
        T0y += Bo * s;
        Txx += Be * (c * c);
        Txy += Be * (c * s);
        Tyy += Be * (s * s);
    }
    // ---- Landau frame in float64, reference moments added back ----
    const double nT = A.n_ref * A.T_ref;
    const double dN0 = A.n_ref + double(N0), dNx = double(Nx), dNy = double(Ny);
    double eps, u0, ux, uy;
    const DeviceRecip rc;
    const bool ok = landau_frame(2.0 * nT + double(T00), double(T0x), double(T0y), nT + double(Txx), double(Txy),
                                 nT + double(Tyy), eps, u0, ux, uy, rc);
    const double n = fma(u0, dN0, -fma(ux, dNx, uy * dNy));
    // T = eps / (2 n) and the density factor n / T = 2 n^2 / eps
    const double T = (0.5 * eps) * rc.rcp(n);
    const double sc = (2.0 * n) * n * rc.rcp(eps);
    fields(SiteFields{n, u0, ux, uy, eps}, ok);
    const R U0 = R(u0 * A.tau_inv), Ux = R(ux * A.tau_inv), Uy = R(uy * A.tau_inv);
    // ---- equilibrium and force coefficients (deviation from the reference, / scale) ----
    R ad[kK];
    // the reference rest state projects only onto kRestK (checked on the host
    // at set-up), so the other coefficients need no subtraction
    appendix_b_each_sc(sc, T, u0, ux, uy, [&](int k, double v) {
        const bool rest = k == kRestK[0] || k == kRestK[1] || k == kRestK[2] || k == kRestK[3];
        ad[k] = R((rest ? v - A.a_ref[k] : v) * A.inv_scale);
    });
    R Hb[kK];
    if (has_force) {
        // b = (Fx C_x + Fy C_y) a / scale with a / scale = ad + a_ref / scale,
        // row by row: the row's terms of C_x and of C_y with their constant
        // coefficients, then the two force components once per row
        R arest[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) arest[r] = ad[kRestK[r]] + A.aref_s[r];
        auto coef = [&](int m) -> R {
            const int r = m == kRestK[0] ? 0 : m == kRestK[1] ? 1 : m == kRestK[2] ? 2 : m == kRestK[3] ? 3 : -1;
            return r >= 0 ? arest[r] : ad[m];
        };
        R b[kK];
#pragma unroll
        for (int k = 0; k < kK; ++k) {
            // -0 is the additive identity, so the first term is a plain product
            R tx = R(-0.0), ty = R(-0.0);
#pragma unroll
            for (int q = 0; q < kForceNx; ++q)
                if (kForceX[q].k == k) tx += R(kForceX[q].v) * coef(kForceX[q].m);
#pragma unroll
            for (int q = 0; q < kForceNy; ++q)
                if (kForceY[q].k == k) ty += R(kForceY[q].v) * coef(kForceY[q].m);
            b[k] = fx * tx + fy * ty;
        }
        appendix_a_to_harmonics(b, Hb);
    } else {
#pragma unroll
        for (int k = 0; k < kK; ++k) Hb[k] = R(0);
    }
    R Wc[4][5], Ws[4][5];
    {
        R Ha[kK];
        appendix_a_to_harmonics(ad, Ha);
        omega_harmonics(Ha, Hb, U0, Ux, Uy, Wc, Ws);
    }
    // ---- relaxation plus forcing, one pair of opposite directions at a time ----
    // f*_i = f_i - omega_d f_i + (omega_d f^eq - force)(p_i), the bracket being
    // the radial polynomial sum_e p0^e W_e(t_d) (odd harmonics flip for d + 6)
#pragma unroll
    for (int d = 0; d < kDirs / 2; ++d) {
        const DirTrig tg = dir_trig(d);
        R E[4], O[4];
        omega_pair(Wc, Ws, tg, E, O);
        const R proj = Ux * R(tg.c) + Uy * R(tg.s);
        const R wp = U0 - proj, wm = U0 + proj;  // omega of d and of d + 6
        R Qp[kShells], Qm[kShells];
#pragma unroll
        for (int j = 0; j < kShells; ++j) {
            const R p = A.p0[j];
            const R qp = (((E[3] + O[3]) * p + (E[2] + O[2])) * p + (E[1] + O[1])) * p + (E[0] + O[0]);
            const R qm = (((E[3] - O[3]) * p + (E[2] - O[2])) * p + (E[1] - O[1])) * p + (E[0] - O[0]);
            Qp[j] = qp;
            Qm[j] = qm;
        }
        emit(d, R(1) - wp, &h[4 * d], Qp);
        emit(d + 6, R(1) - wm, &h[4 * (d + 6)], Qm);
    }
    return ok;
}

template <class R>
__device__ __forceinline__ void write_fields(const StepArgs<R> &A, long long site, const SiteFields &f, bool ok)
{
    if (!ok) {
        A.fn[site] = NAN;
        A.fvx[site] = NAN;
        A.fvy[site] = NAN;
        A.feps[site] = NAN;
        return;
    }
    A.fn[site] = f.n;
    A.fvx[site] = f.ux / f.u0;
    A.fvy[site] = f.uy / f.u0;
    A.feps[site] = f.eps;
}

// Density of the previous state at (x, y) for the local-capacitance gradient
// at (x0, y0): periodic wrap, else an off-lattice or solid neighbour takes
// the density of the site itself.
template <class R>
__device__ __forceinline__ double lca_density(const StepArgs<R> &A, int x, int y, long long site0)
{
    if (A.periodic_x) x = x < 0 ? x + A.nx : (x >= A.nx ? x - A.nx : x);
    if (A.periodic_y) y = y < 0 ? y + A.ny : (y >= A.ny ? y - A.ny : y);
    if ((unsigned)x >= (unsigned)A.nx || (unsigned)y >= (unsigned)A.ny) return A.n_prev[site0];
    const long long s = (long long)y * A.nx + x;
    if (A.has_mask && A.mask[s]) return A.n_prev[site0];
    return A.n_prev[s];
}

// Total force on a site with the local-capacitance term: drive minus
// inv_cg times the central-difference gradient of the previous density.
// `inner`: the four neighbours lie on the lattice and none is solid.
template <class R>
__device__ __forceinline__ void lca_force(const StepArgs<R> &A, int x, int y, long long site, bool inner, R &fx,
                                          R &fy)
{
    double ge, gw, gn, gs;
    if (inner) {
        ge = A.n_prev[site + 1];
        gw = A.n_prev[site - 1];
        gn = A.n_prev[site + A.nx];
        gs = A.n_prev[site - A.nx];
    } else {
        ge = lca_density(A, x + 1, y, site);
        gw = lca_density(A, x - 1, y, site);
        gn = lca_density(A, x, y + 1, site);
        gs = lca_density(A, x, y - 1, site);
    }
    const double gx = 0.5 * (ge - gw), gy = 0.5 * (gn - gs);
    fx = R(double(A.fx) - A.inv_cg * gx);
    fy = R(double(A.fy) - A.inv_cg * gy);
}

// Gather of one site with the boundary rules: periodic wrap, then a contact's
// ghost span (fixed equilibrium), otherwise bounce-back from the site itself
// (also for a solid source site).
template <class S, class R>
__device__ __forceinline__ void gather_general(const StepArgs<R> &A, const S *__restrict__ src, int x, int y,
                                               long long site, R (&h)[kQ])
{
    const int nx = A.nx, ny = A.ny;
    const long long P = A.plane;
#pragma unroll
    for (int i = 0; i < kQ; ++i) {
        const int d = i / kShells;
        const int o = kShells * ((d + kDirs / 2) % kDirs) + (i % kShells);
        int sx = x - kCx[d], sy = y - kCy[d];
        if (A.periodic_x) {
            while (sx < 0) sx += nx;
            while (sx >= nx) sx -= nx;
        }
        if (A.periodic_y) {
            while (sy < 0) sy += ny;
            while (sy >= ny) sy -= ny;
        }
        const bool inside = (unsigned)sx < (unsigned)nx && (unsigned)sy < (unsigned)ny;
        const long long s2 = (long long)sy * nx + sx;
        const bool pull = inside && !(A.has_mask && A.mask[s2]);
        R v;
        if (pull) {
            v = StoreIO<S>::template load<R>(src + pop_elem(kTup<S>, i, s2, P));
        } else {
            int c = -1;
            if (!inside) {
                if (sy < 0 && (unsigned)sx < (unsigned)nx)
                    c = A.edge_contact[sx];
                else if (sy >= ny && (unsigned)sx < (unsigned)nx)
                    c = A.edge_contact[nx + sx];
                else if (sx < 0 && (unsigned)sy < (unsigned)ny)
                    c = A.edge_contact[2 * nx + sy];
                else if (sx >= nx && (unsigned)sy < (unsigned)ny)
                    c = A.edge_contact[2 * nx + ny + sy];
            }
            v = c >= 0 ? A.contact_eta[c * kQ + i] : StoreIO<S>::template load<R>(src + pop_elem(kTup<S>, o, site, P));
        }
        h[i] = v;
    }
}

// Loads of a wave of the top or bottom boundary band of a lattice with an
// interior (no solid mask, nx and ny above twice the stencil's reach, so
// one wrap brings any source back onto a periodic axis).  Per direction:
// the source site after the periodic wraps, or, for a source off the
// lattice, bounce-back from the site itself (the opposite direction's
// value there); then a source in a contact's ghost span (off the lattice
// beyond exactly one edge) takes the span's equilibrium.  The rules and
// their precedence are gather_general's; here every lane loads every
// direction at a selected 32-bit offset (no branch around a load, no table
// codes to read: the population array is below 4 GiB whenever the lattice
// has a gather table, the only case that calls this).
template <class S, class R>
__device__ __forceinline__ void band_wave_gather(const StepArgs<R> &A, const S *__restrict__ src, int x, int y,
                                                 unsigned site, R (&h)[kQ])
{
    const int nx = A.nx, ny = A.ny;
    const unsigned Pu = (unsigned)A.plane;
    int cdir[kDirs];
    bool any = false;
#pragma unroll
    for (int d = 0; d < kDirs; ++d) {
        int sx = x - kCx[d], sy = y - kCy[d];
        if (A.periodic_x) sx = sx < 0 ? sx + nx : (sx >= nx ? sx - nx : sx);
        if (A.periodic_y) sy = sy < 0 ? sy + ny : (sy >= ny ? sy - ny : sy);
        const bool xin = (unsigned)sx < (unsigned)nx, yin = (unsigned)sy < (unsigned)ny;
        const bool pull = xin & yin;
        const unsigned dd = pull ? (unsigned)d : (unsigned)((d + kDirs / 2) % kDirs);
        const unsigned ss = pull ? (unsigned)(sy * nx + sx) : site;
        if constexpr (kTup<S> == kShells) {
            const half4 v = *plane_at_bytes(reinterpret_cast<const half4 *>(src), (dd * Pu + ss) * (unsigned)sizeof(half4));
#pragma unroll
            for (int j = 0; j < kShells; ++j) h[kShells * d + j] = R(float(v[j]));
        } else {
            const unsigned e0 = kShells * dd * Pu + ss;
#pragma unroll
            for (int j = 0; j < kShells; ++j)
                h[kShells * d + j] =
                    StoreIO<S>::template load<R>(plane_at_bytes(src, (e0 + (unsigned)j * Pu) * (unsigned)sizeof(S)));
        }
        // edge table entry of a source beyond exactly one edge, else none
        const int ei = (xin & !yin) ? (sy < 0 ? sx : nx + sx) : (!xin & yin) ? (sx < 0 ? 2 * nx : 2 * nx + ny) + sy : -1;
        const int c = A.edge_contact[ei < 0 ? 0 : ei];
        cdir[d] = ei < 0 ? -1 : c;
        any = any || cdir[d] >= 0;
    }
    if (__ballot(any)) {
#pragma unroll
        for (int d = 0; d < kDirs; ++d) {
            const int cc = cdir[d] < 0 ? 0 : cdir[d];
#pragma unroll
            for (int j = 0; j < kShells; ++j) {
                const R v = A.contact_eta[cc * kQ + kShells * d + j];
                h[kShells * d + j] = cdir[d] >= 0 ? v : h[kShells * d + j];
            }
        }
    }
}

// Loads of a wave that holds side columns of an interior row (x < reach or
// x >= nx - reach).  For a side lane, the populations whose source lies
// beyond the left or right edge follow the boundary rules of the pull:
// periodic wrap, else the edge's contact span, else bounce-back from the
// site itself; every other lane and population pulls as in the interior.
// The source row is always inside the lattice here.  Each load picks its
// address per lane (no lane skips a load), and the contact equilibria, when
// the side has contact spans at all, replace values afterwards.
// OFF32: the whole population array is below 4 GiB (every lattice that has
// a boundary gather table), so every element is a 32-bit byte offset from
// src: the loads take the scalar-base plus 32-bit-offset form and the
// address arithmetic stays in 32 bits (instead of a 64-bit address per lane
// and population).
template <class S, class R, bool OFF32>
__device__ __forceinline__ void side_wave_gather(const StepArgs<R> &A, const S *__restrict__ src, int x, int y,
                                                 unsigned site, R (&h)[kQ])
{
    const int nx = A.nx;
    const long long P = A.plane;
    if constexpr (kTup<S> == kShells) {
        // one tuple (all four shells) per direction; e indexes tuples
#pragma unroll
        for (int d = 0; d < kDirs; ++d) {
            const int sx = x - kCx[d];
            half4 v;
            if constexpr (OFF32) {
                const unsigned Pu = (unsigned)P;
                unsigned e = (unsigned)d * Pu + (unsigned)((y - kCy[d]) * nx + sx);  // plain pull
                if (kCx[d] != 0) {
                    const bool out = (unsigned)sx >= (unsigned)nx;
                    const unsigned wrapped = e + (unsigned)(sx < 0 ? nx : -nx);
                    const unsigned bounce = (unsigned)((d + kDirs / 2) % kDirs) * Pu + site;
                    e = out ? (A.periodic_x ? wrapped : bounce) : e;
                }
                v = *plane_at_bytes(reinterpret_cast<const half4 *>(src), e * (unsigned)sizeof(half4));
            } else {
                long long e = (long long)d * P + (long long)(y - kCy[d]) * nx + sx;  // plain pull
                if (kCx[d] != 0) {
                    const bool out = (unsigned)sx >= (unsigned)nx;
                    const long long wrapped = e + (sx < 0 ? nx : -nx);
                    const long long bounce = (long long)((d + kDirs / 2) % kDirs) * P + site;
                    e = out ? (A.periodic_x ? wrapped : bounce) : e;
                }
                v = reinterpret_cast<const half4 *>(src)[e];
            }
#pragma unroll
            for (int j = 0; j < kShells; ++j) h[kShells * d + j] = R(float(v[j]));
        }
    } else if constexpr (OFF32) {
        const unsigned Pu = (unsigned)P;
#pragma unroll
        for (int i = 0; i < kQ; ++i) {
            const int d = i / kShells;
            const int sx = x - kCx[d];
            unsigned e = (unsigned)i * Pu + (unsigned)((y - kCy[d]) * nx + sx);  // plain pull
            if (kCx[d] != 0) {
                const bool out = (unsigned)sx >= (unsigned)nx;
                const unsigned wrapped = e + (unsigned)(sx < 0 ? nx : -nx);
                const unsigned bounce = (unsigned)(kShells * ((d + kDirs / 2) % kDirs) + (i % kShells)) * Pu + site;
                e = out ? (A.periodic_x ? wrapped : bounce) : e;
            }
            h[i] = StoreIO<S>::template load<R>(plane_at_bytes(src, e * (unsigned)sizeof(S)));
        }
    } else {
#pragma unroll
        for (int i = 0; i < kQ; ++i) {
            const int d = i / kShells;
            const int sx = x - kCx[d];
            long long e = (long long)i * P + (long long)(y - kCy[d]) * nx + sx;  // plain pull
            if (kCx[d] != 0) {
                const bool out = (unsigned)sx >= (unsigned)nx;
                const long long wrapped = e + (sx < 0 ? nx : -nx);
                const long long bounce = (long long)(kShells * ((d + kDirs / 2) % kDirs) + (i % kShells)) * P + site;
                e = out ? (A.periodic_x ? wrapped : bounce) : e;
            }
            h[i] = StoreIO<S>::template load<R>(src + e);
        }
    }
    if (!A.periodic_x && A.side_contacts) {
#pragma unroll
        for (int d = 0; d < kDirs; ++d) {
            if (kCx[d] == 0) continue;
            const int sx = x - kCx[d];
            const bool out = (unsigned)sx >= (unsigned)nx;
            const int c = out ? A.edge_contact[(sx < 0 ? 2 * nx : 2 * nx + A.ny) + (y - kCy[d])] : -1;
            const int cc = c < 0 ? 0 : c;
#pragma unroll
            for (int j = 0; j < kShells; ++j) {
                const R v = A.contact_eta[cc * kQ + kShells * d + j];
                h[kShells * d + j] = c >= 0 ? v : h[kShells * d + j];
            }
        }
    }
}

// One block of a time step.  The step's 1-D grid of 256-thread blocks: the
// first nbnd blocks take the boundary sites (the top and bottom bands,
// band_wave_gather; every site through the gather table, or the computed
// gather without one, when the lattice has a mask or no interior), the rest
// tile the rows y in [5, ny - 5) over their whole width with tile_x * rows
// sites per block, tiles aligned to tile_x so every wavefront stores 64
// aligned values; the side columns of those rows patch their boundary
// populations in place (side_wave_gather).
// Force mode of a step kernel, fixed at compile time so that no runtime
// branch splits the register allocation: no force, the uniform drive, or
// the drive plus the local-capacitance term.
enum ForceMode { kNoForce = 0, kDrive = 1, kLca = 2 };

// GATHER: kGatherTable (the lattice has a gather table: its population
// array is below 4 GiB), kGatherComputed (it has none: 4 GiB and more, or
// dropped with rlbm_set_gather_table) or kGatherEither (decided per launch
// from the arguments; the batched kernel).  The computed gather
// is long code, kept out of the kernels that do not need it.
enum GatherMode { kGatherTable = 0, kGatherComputed = 1, kGatherEither = 2 };

// NT: streaming (non-temporal) population stores.  A compile-time choice:
// with a runtime flag the compiler merges the two store forms of each value
// into one ordinary store.
template <class S, class R, int MODE, int GATHER, bool NT, bool NTL = false>
__device__ __forceinline__ void step_block(const StepArgs<R> &A, const S *__restrict__ src, S *__restrict__ dst,
                                           int b, int nbnd, int tile_x, int tiles_x, int all, int wf)
{
    const int t = threadIdx.x;
    const int nx = A.nx;
    const long long P = A.plane;
    // ---- locate the site: boundary band (table row idx) or interior tile ----
    int x, y;
    unsigned idx = 0;  // boundary band row (the band holds far fewer than 2^31 sites)
    const bool bnd = b < nbnd;
    if (bnd) {
        idx = (unsigned)b * blockDim.x + t;
        if ((long long)idx >= boundary_count(nx, A.ny, all)) return;
        boundary_site(idx, nx, A.ny, all, x, y);
    } else {
        const int tb = b - nbnd;
        const int by = tb / tiles_x, bx = tb - by * tiles_x;
        // tile_x is 64, 128 or 256 (tile_x * rows = 256): shifts, not divisions
        const int lg = 31 - __builtin_clz(tile_x);
        const int rows = (int)blockDim.x >> lg;
        const int ty = t >> lg;
        x = bx * tile_x + (t & (tile_x - 1));
        y = kReach + by * rows + ty;
        if (x >= nx || y >= A.ny - kReach) return;
    }
    const bool side = !bnd && (x < kReach || x >= nx - kReach);
    // a wave's 64 lanes are consecutive sites of one row (tile_x is a
    // multiple of 64): whether it touches a side column is uniform
    const int x0 = x - (int)(threadIdx.x & 63);
    const bool side_wave = !bnd && (x0 < kReach || x0 + 63 >= nx - kReach);
    const unsigned site = (unsigned)y * (unsigned)nx + (unsigned)x;
    if (bnd && A.has_mask && A.mask[site]) {
        if (wf) {
            A.fn[site] = 0.0;
            A.fvx[site] = 0.0;
            A.fvy[site] = 0.0;
            A.feps[site] = 0.0;
        }
        return;
    }
    // ---- force (before the gather: its temporaries die before h is loaded) ----
    R fx = A.fx, fy = A.fy;
    if constexpr (MODE == kLca) lca_force(A, x, y, site, !bnd && !side, fx, fy);
    // ---- gather ----
    R h[kQ];
    if (bnd) {
        const bool table = GATHER == kGatherTable || (GATHER == kGatherEither && A.gather_tab);
        if (table && !all) {
            band_wave_gather<S, R>(A, src, x, y, site, h);
        } else if (table) {
            // eight table codes, then their eight values, at a time, the
            // codes of the next eight already in flight: the band's path then
            // waits for about four memory round trips instead of twelve, and
            // holds at most sixteen codes (all 48 at once would set the
            // kernel's register budget)
            const unsigned *__restrict__ tab = A.gather_tab;
            unsigned c[2][8];
#pragma unroll
            for (int i = 0; i < 8; ++i) c[0][i] = tab[(long long)i * A.nbnd + idx];
#pragma unroll
            for (int i0 = 0; i0 < kQ; i0 += 8) {
                const int cur = (i0 / 8) & 1;
                if (i0 + 8 < kQ) {
#pragma unroll
                    for (int i = 0; i < 8; ++i) c[cur ^ 1][i] = tab[(long long)(i0 + 8 + i) * A.nbnd + idx];
                }
                // every lane loads a population (code 0 stands in for a
                // contact, an always valid element) and the contact
                // equilibria are patched in only by waves that have one:
                // a branch per value would make every 16-bit load wait for
                // the one before it
                bool any = false;
#pragma unroll
                for (int i = 0; i < 8; ++i) {
                    const unsigned code = c[cur][i];
                    const bool contact = (code & kContactFlag) != 0;
                    h[i0 + i] = StoreIO<S>::template load<R>(
                        plane_at_bytes(src, (contact ? 0u : code) * (unsigned)sizeof(S)));
                    any = any || contact;
                }
                if (__ballot(any)) {
#pragma unroll
                    for (int i = 0; i < 8; ++i) {
                        const unsigned code = c[cur][i];
                        if (code & kContactFlag) h[i0 + i] = A.contact_eta[code & ~kContactFlag];
                    }
                }
                asm volatile("" ::: "memory");
            }
        } else if constexpr (GATHER != kGatherTable) {
            gather_general<S, R>(A, src, x, y, site, h);
        }
    } else if (side_wave) {
        if constexpr (GATHER == kGatherTable) {
            side_wave_gather<S, R, true>(A, src, x, y, site, h);
        } else if constexpr (GATHER == kGatherEither) {
            if (A.gather_tab)
                side_wave_gather<S, R, true>(A, src, x, y, site, h);
            else
                side_wave_gather<S, R, false>(A, src, x, y, site, h);
        } else {
            side_wave_gather<S, R, false>(A, src, x, y, site, h);
        }
    } else {
        // uniform plane base pointers + one 32-bit site offset; NTL: loads
        // that do not allocate in the caches, which leaves the Infinity Cache
        // to the step's own stores (read by the next step)
        if constexpr (kTup<S> == kShells) {
#pragma unroll
            for (int d = 0; d < kDirs; ++d) {
                const half4 *__restrict__ arr =
                    reinterpret_cast<const half4 *>(src) + ((long long)d * P - ((long long)kCy[d] * nx + kCx[d]));
                half4 v;
                if constexpr (NTL)
                    v = __builtin_nontemporal_load(plane_at(arr, site));
                else
                    v = *plane_at(arr, site);
#pragma unroll
                for (int j = 0; j < kShells; ++j) h[kShells * d + j] = R(float(v[j]));
            }
        } else {
#pragma unroll
            for (int i = 0; i < kQ; ++i) {
                const int d = i / kShells;
                const S *__restrict__ plane = src + ((long long)i * P - ((long long)kCy[d] * nx + kCx[d]));
                if constexpr (NTL)
                    h[i] = R(__builtin_nontemporal_load(plane_at(plane, site)));
                else
                    h[i] = StoreIO<S>::template load<R>(plane_at(plane, site));
            }
        }
    }
    // ---- collide; each post-collision value is stored as soon as it is
    // formed (streaming stores bypass the caches: the next step reads every
    // value once) ----
    unsigned site_bytes = site * (unsigned)(sizeof(S) * kTup<S>);
    auto store = [&](int d, R a, const R *hv, const R *q) {
        asm volatile("" : "+v"(site_bytes));
        store_dir<S, R, NT>(dst, P, d, site_bytes, a, hv, q);
    };
    auto fields = [&](const SiteFields &f, bool ok) {
        if (wf) write_fields(A, site, f, ok);
        if constexpr (MODE == kLca) A.n_next[site] = ok ? f.n : NAN;
    };
    collide_site<R>(h, A, fx, fy, MODE != kNoForce, store, fields);
}

// At most four waves per SIMD for FP32 and FP64 storage, five for FP16:
// measured on MI355X, five waves (93-95 VGPRs, no spills) make FP16 3-4%
// faster and FP32 1.3% slower than four.
template <class S, class R, int MODE, int GATHER, bool NT, bool NTL>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(1, sizeof(S) == 2 ? 5 : 4))) void step_kernel(const StepArgs<R> A, const S *__restrict__ src,
                                                   S *__restrict__ dst, int nbnd, int tile_x, int tiles_x, int all,
                                                   int xcd)
{
    const int b = xcd ? xcd_block((int)blockIdx.x, (int)gridDim.x) : (int)blockIdx.x;
    step_block<S, R, MODE, GATHER, NT, NTL>(A, src, dst, b, nbnd, tile_x, tiles_x, all, A.write_fields);
}

// Batched step: one block per work item of the list of (sample, block)
// items, each item being one block of that sample's step grid; the grid is
// the list's capacity and blocks past the current item count leave at once.
// (A persistent grid looping over the items keeps each item's descriptor
// live across iterations and needs every register of the SIMD, one wave
// per SIMD; one item per block keeps the single-lattice kernel's budget.)
template <class S, class R, bool NT>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(1, sizeof(S) == 2 ? 5 : 4))) void batch_step_kernel(const BatchDesc<R> *__restrict__ descs,
                                                         const unsigned *__restrict__ items,
                                                         const int *__restrict__ n_items_p, int parity, int wf,
                                                         int xcd)
{
    const unsigned n_items = (unsigned)*n_items_p;
    const unsigned k = xcd ? (unsigned)xcd_block((int)blockIdx.x, (int)gridDim.x) : blockIdx.x;
    if (k >= n_items) return;
    const unsigned it = __builtin_amdgcn_readfirstlane(items[k]);
    const int smp = (int)(it >> kItemBlockBits), b = (int)(it & ((1u << kItemBlockBits) - 1));
    const BatchDesc<R> &D = descs[smp];
    const int par = parity ^ D.parity_xor;
    // the drive variant serves every sample: a zero drive adds exactly zero
    step_block<S, R, kDrive, kGatherEither, NT>(D.a, static_cast<const S *>(D.pop[par]), static_cast<S *>(D.pop[par ^ 1]),
                                            b, D.nbnd, D.tile_x, D.tiles_x, D.all, wf);
}

// Per-sample residual partial sums: block (s, j) covers sites j, j + B*256,
// ... of sample s; part[(s * B + j) * 3 + {0,1,2}] = |u - u_prev|^2, |u|^2,
// unhealthy count.
template <class R>
__global__ __launch_bounds__(256) void batch_residual_kernel(const BatchDesc<R> *__restrict__ descs,
                                                             double *__restrict__ part)
{
    const int smp = blockIdx.y, B = gridDim.x;
    const BatchDesc<R> &D = descs[smp];
    const long long n = D.a.plane;
    double dv = 0.0, vv = 0.0, bad = 0.0;
    for (long long s = (long long)blockIdx.x * blockDim.x + threadIdx.x; s < n; s += (long long)B * blockDim.x) {
        if (D.a.has_mask && D.a.mask[s]) continue;
        const double a = D.a.fvx[s], b = D.a.fvy[s], dn = D.a.fn[s];
        const double ex = a - D.pvx[s], ey = b - D.pvy[s];
        const double v2 = a * a + b * b;
        if (!(dn > 0.0) || !(v2 < 1.0) || !isfinite(a) || !isfinite(b) || !isfinite(dn)) bad += 1.0;
        dv += ex * ex + ey * ey;
        vv += v2;
    }
    for (int off = 32; off > 0; off >>= 1) {
        dv += __shfl_down(dv, off, 64);
        vv += __shfl_down(vv, off, 64);
        bad += __shfl_down(bad, off, 64);
    }
    __shared__ double red[3][256 / 64];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) {
        red[0][wid] = dv;
        red[1][wid] = vv;
        red[2][wid] = bad;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double s0 = 0, s1 = 0, s2 = 0;
        for (int w = 0; w < (int)(blockDim.x / 64); ++w) {
            s0 += red[0][w];
            s1 += red[1][w];
            s2 += red[2][w];
        }
        double *o = part + ((long long)smp * B + blockIdx.x) * 3;
        o[0] = s0;
        o[1] = s1;
        o[2] = s2;
    }
}

template <class S, class R>
__global__ __launch_bounds__(256) void init_kernel(const StepArgs<R> A, const double *__restrict__ n_in,
                                                   const double *__restrict__ T_in, const double *__restrict__ vx_in,
                                                   const double *__restrict__ vy_in, double un, double uT, double uvx,
                                                   double uvy, S *__restrict__ dst, int mode)
{
    const long long site = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (site >= A.plane) return;
    if (A.has_mask && A.mask[site]) {
        if (mode == kInitDensity) return;
        for (int i = 0; i < kQ; ++i) StoreIO<S>::template store<R>(dst + pop_elem(kTup<S>, i, site, A.plane), R(0));
        A.fn[site] = 0.0;
        A.fvx[site] = 0.0;
        A.fvy[site] = 0.0;
        A.feps[site] = 0.0;
        return;
    }
    const double n = n_in ? n_in[site] : un;
    const double T = T_in ? T_in[site] : uT;
    const double vx = vx_in ? vx_in[site] : uvx;
    const double vy = vy_in ? vy_in[site] : uvy;
    const double g = 1.0 / sqrt(1.0 - vx * vx - vy * vy);
    double a[kK];
    appendix_b(n, T, g, g * vx, g * vy, a);
    R ad[kK], H[kK];
    for (int k = 0; k < kK; ++k) ad[k] = R((a[k] - A.a_ref[k]) * A.inv_scale);
    appendix_a_to_harmonics(ad, H);
    R h[kQ];
#pragma unroll
    for (int d = 0; d < kDirs / 2; ++d) {
        R E[4], O[4];
        harmonics_pair(H, dir_trig(d), E, O);
#pragma unroll
        for (int j = 0; j < kShells; ++j) {
            const R p = A.p0[j];
            h[4 * d + j] = (((E[3] + O[3]) * p + (E[2] + O[2])) * p + (E[1] + O[1])) * p + (E[0] + O[0]);
            h[4 * (d + 6) + j] = (((E[3] - O[3]) * p + (E[2] - O[2])) * p + (E[1] - O[1])) * p + (E[0] - O[0]);
        }
    }
    R fx = A.fx, fy = A.fy;
    bool force = A.has_force != 0;
    if (mode == kInitLca) {
        const int y = (int)(site / A.nx), x = (int)(site - (long long)y * A.nx);
        lca_force(A, x, y, site, false, fx, fy);
        force = true;
    }
    if (mode == kInitDensity) {
        collide_site<R>(h, A, fx, fy, force, NoEmit(),
                        [&](const SiteFields &f, bool ok) { A.n_next[site] = ok ? f.n : NAN; });
        return;
    }
    collide_site<R>(h, A, fx, fy, force,
                    [&](int d, R a, const R *hv, const R *q) {
                        if constexpr (kTup<S> == kShells) {
                            store_dir<S, R, false>(dst, A.plane, d, (unsigned)site * (unsigned)sizeof(half4), a, hv, q);
                        } else {
#pragma unroll
                            for (int j = 0; j < kShells; ++j)
                                StoreIO<S>::template store<R>(dst + pop_elem(1, kShells * d + j, site, A.plane),
                                                              a * hv[j] + q[j]);
                        }
                    },
                    [&](const SiteFields &f, bool ok) { write_fields(A, site, f, ok); });
}

template <class S>
__global__ __launch_bounds__(256) void decode_kernel(long long plane, const S *__restrict__ src,
                                                     const double *__restrict__ fref,
                                                     const double *__restrict__ wscale, double *__restrict__ f)
{
    const long long site = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (site >= plane) return;
    for (int i = 0; i < kQ; ++i) {
        const double e = StoreIO<S>::template load<double>(src + pop_elem(kTup<S>, i, site, plane));
        f[(long long)i * plane + site] = fref[i] + wscale[i] * e;
    }
}

template <class S, class R>
hipError_t launch_step_t(const void *args, const void *src, void *dst, LaunchShape sh, hipStream_t s)
{
    const StepArgs<R> &A = *static_cast<const StepArgs<R> *>(args);
    const bool interior = !A.has_mask && A.nx > 2 * kReach && A.ny > 2 * kReach;
    const int block = 256;
    const long long nb = boundary_count(A.nx, A.ny, !interior);
    const int nbnd = (int)((nb + block - 1) / block);
    int tiles_x = 0, tiles = 0;
    if (interior) {
        const int rows = block / sh.tile_x;
        tiles_x = (A.nx + sh.tile_x - 1) / sh.tile_x;
        tiles = tiles_x * ((A.ny - 2 * kReach + rows - 1) / rows);
    }
    const dim3 grid((unsigned)(nbnd + tiles));
    const S *in = static_cast<const S *>(src);
    S *out = static_cast<S *>(dst);
    const int all = interior ? 0 : 1;
    const int mode = A.n_prev ? kLca : A.has_force ? kDrive : kNoForce;
    const int gather = A.gather_tab ? kGatherTable : kGatherComputed;
#define RLBM_LAUNCH_STEP_MEM(M, G, NT, NTL)                                                                        \
    hipLaunchKernelGGL((step_kernel<S, R, M, G, NT, NTL>), grid, dim3(block), 0, s, A, in, out, nbnd, sh.tile_x,  \
                       tiles_x, all, sh.xcd)
#define RLBM_LAUNCH_STEP(M, G)                                                                                     \
    do {                                                                                                           \
        if (A.nt_store && A.nt_load) RLBM_LAUNCH_STEP_MEM(M, G, true, true);                                     \
        else if (A.nt_store) RLBM_LAUNCH_STEP_MEM(M, G, true, false);                                            \
        else if (A.nt_load) RLBM_LAUNCH_STEP_MEM(M, G, false, true);                                             \
        else RLBM_LAUNCH_STEP_MEM(M, G, false, false);                                                           \
    } while (0)
    if (gather == kGatherTable) {
        if (mode == kLca) RLBM_LAUNCH_STEP(kLca, kGatherTable);
        else if (mode == kDrive) RLBM_LAUNCH_STEP(kDrive, kGatherTable);
        else RLBM_LAUNCH_STEP(kNoForce, kGatherTable);
    } else {
        if (mode == kLca) RLBM_LAUNCH_STEP(kLca, kGatherComputed);
        else if (mode == kDrive) RLBM_LAUNCH_STEP(kDrive, kGatherComputed);
        else RLBM_LAUNCH_STEP(kNoForce, kGatherComputed);
    }
#undef RLBM_LAUNCH_STEP
#undef RLBM_LAUNCH_STEP_MEM
    return hipGetLastError();
}

template <class S, class R>
hipError_t launch_init_t(const void *args, const double *n, const double *T, const double *vx, const double *vy,
                         const double u[4], void *dst, int mode, hipStream_t s)
{
    const StepArgs<R> &A = *static_cast<const StepArgs<R> *>(args);
    if ((mode == kInitDensity && !A.n_next) || (mode == kInitLca && !A.n_prev) || mode < 0 || mode > 2)
        return hipErrorInvalidValue;
    const int block = 256;
    const long long grid = (A.plane + block - 1) / block;
    hipLaunchKernelGGL((init_kernel<S, R>), dim3((unsigned)grid), dim3(block), 0, s, A, n, T, vx, vy, u[0], u[1], u[2],
                       u[3], static_cast<S *>(dst), mode);
    return hipGetLastError();
}

template <class S, class R>
hipError_t launch_batch_t(const void *descs, const unsigned *items, const int *n_items, int grid, int parity, int wf,
                          int xcd, int nt, hipStream_t s)
{
    if (nt)
        hipLaunchKernelGGL((batch_step_kernel<S, R, true>), dim3(grid), dim3(256), 0, s,
                           static_cast<const BatchDesc<R> *>(descs), items, n_items, parity, wf, xcd);
    else
        hipLaunchKernelGGL((batch_step_kernel<S, R, false>), dim3(grid), dim3(256), 0, s,
                           static_cast<const BatchDesc<R> *>(descs), items, n_items, parity, wf, xcd);
    return hipGetLastError();
}

}  // namespace

// The launchers of one storage S (arithmetic R), defined by the translation
// unit of that storage.
#define RLBM_DEFINE_STORAGE_LAUNCHERS(S, R, SUFFIX)                                                              \
    hipError_t launch_step_##SUFFIX(const void *args, const void *src, void *dst, LaunchShape sh, hipStream_t s) \
    {                                                                                                            \
        return launch_step_t<S, R>(args, src, dst, sh, s);                                                       \
    }                                                                                                            \
    hipError_t launch_init_##SUFFIX(const void *args, const double *n, const double *T, const double *vx,        \
                                    const double *vy, const double u[4], void *dst, int mode, hipStream_t s)     \
    {                                                                                                            \
        return launch_init_t<S, R>(args, n, T, vx, vy, u, dst, mode, s);                                         \
    }                                                                                                            \
    hipError_t launch_batch_##SUFFIX(const void *descs, const unsigned *items, const int *n_items, int grid,     \
                                     int parity, int wf, int xcd, int nt, hipStream_t s)                         \
    {                                                                                                            \
        return launch_batch_t<S, R>(descs, items, n_items, grid, parity, wf, xcd, nt, s);                        \
    }                                                                                                            \
    hipError_t launch_batch_residual_##SUFFIX(const void *descs, int nsamples, int blocks_per_sample,            \
                                              double *part, hipStream_t s)                                       \
    {                                                                                                            \
        hipLaunchKernelGGL(batch_residual_kernel<R>, dim3(blocks_per_sample, nsamples), dim3(256), 0, s,         \
                           static_cast<const BatchDesc<R> *>(descs), part);                                      \
        return hipGetLastError();                                                                                \
    }                                                                                                            \
    hipError_t launch_decode_##SUFFIX(long long plane, const void *src, const double *fref, const double *wscale, \
                                      double *f, hipStream_t s)                                                  \
    {                                                                                                            \
        const dim3 grid((unsigned)((plane + 255) / 256));                                                        \
        hipLaunchKernelGGL(decode_kernel<S>, grid, dim3(256), 0, s, plane, static_cast<const S *>(src), fref,    \
                           wscale, f);                                                                           \
        return hipGetLastError();                                                                                \
    }

}  // namespace rlbm
