// Kernel-side data layout and launch interface of the rlbm library.
#pragma once

#include <hip/hip_runtime.h>

#include "rlbm_math.h"

namespace rlbm {

// Non-zero positions (k, m) of C_x and C_y (Sec. 2.4 force projection,
// b_j = C_j a): the two patterns are disjoint and together have 89 entries.
// The host verifies at set-up that every other entry of its own C_x, C_y is
// zero.
constexpr int kForceNnz = 89;
constexpr unsigned char kForceK[kForceNnz] = {
    0, 0, 0, 0, 0, 0, 0, 1, 1, 1, 1, 1, 1, 1, 2, 2, 2, 2, 2, 3, 3, 3, 3, 3, 4, 4, 4, 4, 4, 5, 5, 5, 5, 5, 5,
    6, 6, 6, 6, 6, 6, 7, 7, 7, 7, 7, 8, 8, 8, 8, 8, 9, 9, 9, 10, 10, 10, 10, 10, 10, 10, 11, 11, 11, 11, 11, 11,
    11, 12, 12, 12, 12, 12, 12, 12, 13, 13, 13, 13, 13, 14, 14, 15, 15, 15, 15, 15, 15, 15};
constexpr unsigned char kForceM[kForceNnz] = {
    2, 3, 5, 6, 10, 11, 13, 2, 3, 5, 6, 10, 11, 13, 0, 7, 8, 12, 15, 0, 7, 8, 12, 15, 5, 6, 10, 11, 13, 0, 1, 7, 8,
    12, 15, 0, 1, 7, 8, 12, 15, 2, 3, 10, 11, 14, 2, 3, 10, 11, 14, 10, 11, 13, 0, 1, 4, 7, 8, 12, 15, 0, 1, 4, 7,
    8, 12, 15, 2, 3, 5, 6, 10, 11, 14, 0, 1, 4, 12, 15, 7, 8, 2, 3, 5, 6, 10, 11, 14};

constexpr int kMaxContacts = 16;

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
    int pad_;
    long long plane;  // nx * ny
    // moments of eta: N^a = N_ref^a + sum_i wp0 * eta_i * (1, nhat), T likewise with wp0sq
    R wp0[2][kShells];    // scale * w_gj * p0_j
    R wp0sq[2][kShells];  // scale * w_gj * p0_j^2
    R p0[kShells];
    double n_ref, T_ref;
    double a_ref[kK];  // Appendix B projections of the reference state
    double inv_scale;
    double tau_inv;
    R cf[kForceNnz];  // (Fx C_x + Fy C_y) on the pattern
    R cf_aref[kK];    // (Fx C_x + Fy C_y) a_ref / scale
    // boundaries
    const unsigned char *mask;        // nx*ny, 1 = solid (or null)
    const signed char *edge_contact;  // [bottom: nx][top: nx][left: ny][right: ny] -> contact or -1
    const R *contact_eta;             // [contact][48], eta units
    // fields (float64 SoA), written when write_fields != 0
    double *fn, *fvx, *fvy, *feps;
};

enum class Store { F64 = 0, F32 = 1, F16 = 2 };

struct LaunchShape {
    int tile_x;  // sites per block along x (multiple of 64)
    int rows;    // rows per block
};

// One time step src -> dst (post-collision storage, pull streaming).
hipError_t launch_step(Store st, const void *args, const void *src, void *dst, LaunchShape shape, hipStream_t s);

// Initial post-collision state from fields (n, T, vx, vy; null pointers ->
// the uniform values u[4]).  Writes dst and the fields of the initial state.
hipError_t launch_init(Store st, const void *args, const double *n, const double *T, const double *vx,
                       const double *vy, const double u[4], void *dst, hipStream_t s);

// Decode storage to float64 populations f_i = f_ref_i + w_i * scale * eta_i.
hipError_t launch_decode(Store st, int nx, int ny, const void *src, const double *fref, const double *wscale,
                         double *f, hipStream_t s);

// Per-block partial sums over fluid sites: |u - u_prev|^2, |u|^2 and the
// count of unhealthy sites (non-finite, n <= 0, |u| >= 1).  part has 3 * nblocks doubles.
hipError_t launch_residual(int nsites, const unsigned char *mask, const double *n, const double *vx,
                           const double *vy, const double *pvx, const double *pvy, double *part, int nblocks,
                           hipStream_t s);

}  // namespace rlbm
