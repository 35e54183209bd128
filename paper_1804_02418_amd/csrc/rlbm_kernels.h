// Kernel-side data layout and launch interface of the rlbm library.
#pragma once

#include <hip/hip_runtime.h>

#include "rlbm_math.h"

namespace rlbm {

// Non-zero entries {k, m, value} of the force projection matrices C_x and
// C_y (Sec. 2.4: b_j = C_j a in the Appendix A basis).  They are fixed
// numbers (rationals times square roots); the host recomputes both matrices
// exactly at set-up and refuses to run if any entry differs from these or
// if an entry outside these lists is non-zero.
struct ForceEntry {
    unsigned char k, m;
    double v;
};
constexpr int kForceNx = 48;
constexpr ForceEntry kForceX[kForceNx] = {
    {0, 2, 0.5}, {0, 5, -0.57735026918962573}, {0, 10, 0.375},
    {0, 11, 0.48412291827592713}, {1, 2, -0.5}, {1, 5, 0.57735026918962573},
    {1, 10, -0.375}, {1, 11, -0.48412291827592713}, {2, 0, -0.5},
    {2, 7, 0.14433756729740643}, {2, 12, -0.12909944487358058}, {3, 8, 0.14433756729740643},
    {3, 15, -0.12909944487358058}, {4, 5, -0.57735026918962573}, {4, 10, 0.375},
    {4, 11, 0.48412291827592713}, {5, 0, 0.28867513459481287}, {5, 1, -0.57735026918962573},
    {5, 7, -0.25}, {5, 12, 0.22360679774997896}, {6, 8, -0.25},
    {6, 15, 0.22360679774997896}, {7, 2, -0.4330127018922193}, {7, 10, 0.072168783648703216},
    {7, 11, -0.055901699437494741}, {8, 3, -0.4330127018922193}, {8, 14, 0.091287092917527679},
    {9, 10, -0.375}, {9, 11, -0.48412291827592713}, {10, 0, -0.125},
    {10, 1, 0.25}, {10, 4, -0.375}, {10, 7, -0.36084391824351608},
    {10, 12, -0.19364916731037085}, {11, 0, -0.1613743060919757}, {11, 1, 0.3227486121839514},
    {11, 4, -0.48412291827592713}, {11, 7, 0.27950849718747373}, {11, 12, -0.25},
    {12, 2, 0.19364916731037085}, {12, 5, -0.44721359549995793}, {12, 10, -0.1613743060919757},
    {12, 11, 0.125}, {13, 15, -0.31622776601683794}, {14, 8, -0.45643546458763845},
    {15, 3, 0.19364916731037085}, {15, 6, -0.44721359549995793}, {15, 14, -0.20412414523193151}};
constexpr int kForceNy = 41;
constexpr ForceEntry kForceY[kForceNy] = {
    {0, 3, 0.5}, {0, 6, -0.57735026918962573}, {0, 13, 0.61237243569579447},
    {1, 3, -0.5}, {1, 6, 0.57735026918962573}, {1, 13, -0.61237243569579447},
    {2, 8, 0.14433756729740643}, {2, 15, -0.12909944487358058}, {3, 0, -0.5},
    {3, 7, -0.14433756729740643}, {3, 12, 0.12909944487358058}, {4, 6, -0.57735026918962573},
    {4, 13, 0.61237243569579447}, {5, 8, -0.25}, {5, 15, 0.22360679774997896},
    {6, 0, 0.28867513459481287}, {6, 1, -0.57735026918962573}, {6, 7, 0.25},
    {6, 12, -0.22360679774997896}, {7, 3, 0.4330127018922193}, {7, 14, 0.091287092917527679},
    {8, 2, -0.4330127018922193}, {8, 10, -0.072168783648703216}, {8, 11, 0.055901699437494741},
    {9, 13, -0.61237243569579447}, {10, 8, 0.36084391824351608}, {10, 15, -0.19364916731037085},
    {11, 8, -0.27950849718747373}, {11, 15, -0.25}, {12, 3, -0.19364916731037085},
    {12, 6, 0.44721359549995793}, {12, 14, -0.20412414523193151}, {13, 0, -0.20412414523193151},
    {13, 1, 0.40824829046386302}, {13, 4, -0.61237243569579447}, {13, 12, 0.31622776601683794},
    {14, 7, -0.45643546458763845}, {15, 2, 0.19364916731037085}, {15, 5, -0.44721359549995793},
    {15, 10, 0.1613743060919757}, {15, 11, -0.125}};

// The rest-frame projections of the reference state are non-zero only for
// these Appendix A indices (J0, J1_0, J2_00, J3_000).
constexpr int kRestK[4] = {0, 1, 4, 9};

constexpr int kMaxContacts = 16;
constexpr unsigned kContactFlag = 0x80000000u;

// Population layout of a storage: 48 / W arrays of nx*ny tuples, a tuple
// holding W consecutive populations, i.e. W shells of one direction (the
// four shells of a direction hop alike).  W = 1 is the plain layout of 48
// planes (float64 and float32 storage); float16 storage keeps the four
// shells of a direction in one 8-byte tuple, so that a pull reads each
// direction as one 8-byte load per site (2-byte loads cap the pull well
// below the bandwidth that 4- and 8-byte loads reach).
__host__ __device__ constexpr int tuple_width(int store_bytes) { return store_bytes == 2 ? kShells : 1; }
// Element index of population i at site s, P = nx*ny sites, tuples of w.
__host__ __device__ constexpr long long pop_elem(int w, int i, long long s, long long P)
{
    return ((long long)(i / w) * P + s) * w + (i % w);
}

// Boundary part of the step grid: with an interior (nx, ny > 2 * reach, no
// mask) the bottom and top bands of `reach` rows (the side columns of the
// rows in between belong to the interior tiles, which resolve their few
// boundary populations in place); without one, every site.
__host__ __device__ inline long long boundary_count(int nx, int ny, bool all)
{
    if (all) return (long long)nx * ny;
    return 2LL * kReach * nx;
}

__host__ __device__ inline void boundary_site(long long idx, int nx, int ny, bool all, int &x, int &y)
{
    const long long band = (long long)kReach * nx;
    if (all || idx < band) {
        y = (int)(idx / nx);
        x = (int)(idx - (long long)y * nx);
    } else {
        const long long r = idx - band;
        const int ry = (int)(r / nx);
        y = ny - kReach + ry;
        x = (int)(r - (long long)ry * nx);
    }
}

__host__ __device__ inline bool has_interior(int nx, int ny, bool mask)
{
    return !mask && nx > 2 * kReach && ny > 2 * kReach;
}

// Everything a step, init or decode kernel needs, passed by value.  R is the
// arithmetic type of the population update (double for F64 storage, float
// for F32 and F16DEV).  Populations are stored as the scaled deviation
//   eta_i = (f_i - f_ref_i) / (w_i * scale),  f_ref = f^eq(n_ref, T_ref, 0).
template <class R>
struct StepArgs {
    int nx, ny;
    int periodic_x, periodic_y;
    int has_mask;
    int has_force;
    int write_fields;
    int nt_store;     // 1: stores bypass the caches (streaming), 0: ordinary stores
    int nt_load;      // 1: interior population loads are non-temporal (no cache allocation)
    long long plane;  // nx * ny
    // moments of eta: N^a = N_ref^a + sum_i wp0 * eta_i * (1, nhat), T likewise with wp0sq
    R wp0[2][kShells];    // scale * w_gj * p0_j
    R wp0sq[2][kShells];  // scale * w_gj * p0_j^2
    R p0[kShells];
    double n_ref, T_ref;
    double a_ref[kK];  // Appendix B projections of the reference state
    double inv_scale;
    double tau_inv;
    R fx, fy;           // drive F (force term b = Fx C_x a + Fy C_y a, in units of scale)
    R aref_s[4];        // a_ref[kRestK] / scale
    // boundaries
    const unsigned char *mask;        // nx*ny, 1 = solid (or null)
    const signed char *edge_contact;  // [bottom: nx][top: nx][left: ny][right: ny] -> contact or -1
    int side_contacts;                // bit 0: the left edge has a contact span, bit 1: the right edge
    const R *contact_eta;             // [contact][48], eta units
    // boundary gather table [48][nbnd]: source element of population i of
    // boundary site b (its index in the population array, pop_elem), or
    // kContactFlag | (c*48 + i)
    // for a contact equilibrium; null -> the gather is computed in place
    const unsigned *gather_tab;
    long long nbnd;
    // fields (float64 SoA), written when write_fields != 0
    double *fn, *fvx, *fvy, *feps;
    // local-capacitance force F = drive - inv_cg * grad n (Sec. 3, Eq. lca):
    // n_prev holds the density of the previous state (central differences,
    // an off-lattice or solid neighbour taking the site's own density);
    // every step writes its own density to n_next.  n_prev == null: off.
    double inv_cg;
    const double *n_prev;
    double *n_next;
};

enum class Store { F64 = 0, F32 = 1, F16 = 2 };

// One sample of a batch: its step arguments (fields pointers included), its
// two population buffers and its step-grid geometry.  The buffer holding the
// current state is pop[parity ^ parity_xor] for the batch-wide step parity.
template <class R>
struct BatchDesc {
    StepArgs<R> a;
    void *pop[2];
    const double *pvx, *pvy;  // velocities at the end of the previous batch step call
    int nbnd, tile_x, tiles_x, all;
    int parity_xor, pad_;
};

// Work item = (sample << kItemBlockBits) | block of that sample's step grid.
constexpr int kItemBlockBits = 20;

struct LaunchShape {
    int tile_x;   // sites per block along x (multiple of 64)
    int rows;     // rows per block
    int xcd = 0;  // 1: consecutive tiles go to the same XCD (its own L2)
};

// Workgroups of a launch are dealt to the 8 XCDs in turn (block b runs on
// XCD b % 8).  With `xcd` on, block b takes logical block xcd_block(b, G) so
// that each XCD gets one contiguous range of the G logical blocks: tiles
// that share cache lines (horizontal neighbours) then share an L2.  A
// bijection of [0, G) for any G.
__device__ __forceinline__ int xcd_block(int b, int G)
{
    const int x = b & 7, q = G >> 3, r = G & 7;
    return x * q + (x < r ? x : r) + (b >> 3);
}

// One time step src -> dst (post-collision storage, pull streaming): an
// interior kernel for the sites whose whole stencil lies on the lattice
// (none when there is a mask) and a boundary kernel for the rest.
hipError_t launch_step(Store st, const void *args, const void *src, void *dst, LaunchShape shape, hipStream_t s);

// Batched step: `grid` blocks (at least *n_items), block b taking work item
// b, or xcd_block(b, grid) when `xcd` is set; blocks past *n_items leave.
// nt: streaming population stores for every sample.
hipError_t launch_batch_step(Store st, const void *descs, const unsigned *items, const int *n_items, int grid,
                             int parity, int write_fields, int xcd, int nt, hipStream_t s);
// Per-sample residual partial sums (3 doubles per block, blocks_per_sample per sample).
hipError_t launch_batch_residual(Store st, const void *descs, int nsamples, int blocks_per_sample, double *part,
                                 hipStream_t s);

// Initial post-collision state from fields (n, T, vx, vy; null pointers ->
// the uniform values u[4]).  mode kInitPlain: writes dst and the fields of
// the initial state; kInitDensity: writes only the density of f(0) to
// n_next; kInitLca: as plain, the collision taking the local-capacitance
// force from n_prev (the density written by a kInitDensity pass).
enum InitMode { kInitPlain = 0, kInitDensity = 1, kInitLca = 2 };
hipError_t launch_init(Store st, const void *args, const double *n, const double *T, const double *vx,
                       const double *vy, const double u[4], void *dst, int mode, hipStream_t s);

// Decode storage to float64 populations f_i = f_ref_i + w_i * scale * eta_i.
hipError_t launch_decode(Store st, int nx, int ny, const void *src, const double *fref, const double *wscale,
                         double *f, hipStream_t s);

// Per-block partial sums over fluid sites: |u - u_prev|^2, |u|^2 and the
// count of unhealthy sites (non-finite, n <= 0, |u| >= 1).  part has 3 * nblocks doubles.
hipError_t launch_residual(int nsites, const unsigned char *mask, const double *n, const double *vx,
                           const double *vy, const double *pvx, const double *pvy, double *part, int nblocks,
                           hipStream_t s);

// The same residual sums without any buffer from the caller or the library:
// the partial sums (nblocks <= kNoAllocResidualBlocks) and their totals go
// through a file-scope device array of the current device; totals[3] (host)
// receives sum |u - u_prev|^2, sum |u|^2 and the unhealthy count, added in
// the order launch_residual's caller adds them.  Synchronises the stream.
constexpr int kNoAllocResidualBlocks = 1024;
hipError_t launch_residual_noalloc(int nsites, const unsigned char *mask, const double *n, const double *vx,
                                   const double *vy, const double *pvx, const double *pvy, int nblocks,
                                   double totals[3], hipStream_t s);

}  // namespace rlbm
