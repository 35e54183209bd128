/*
 * rlbm.h -- C ABI of the MI355X (gfx950) library for the (2+1)-dimensional
 * relativistic lattice Boltzmann method on a Gaussian quadrature
 * (massless particles, third-order equilibrium, 48 populations per site).
 *
 * The problem the calls follow is the one of the paper's Sec. 2-3: a 2-D
 * lattice carrying the m = 0, order-3 stencil G = {(+-3,+-4)_FS, (+-5,0)_FS}
 * with four energy shells (Sec. 2.3), relaxed with time tau by the discrete
 * Anderson-Witting equation (Eq. discrete-rbe), driven by an external force
 * (Sec. 2.4), bounded by bounce-back walls and by inlet/outlet sites that do
 * not evolve in time (Sec. 3), advanced N steps, and observed through the
 * density n, the velocity u and the energy density eps.
 *
 * Conventions shared by every call:
 *  - Lattice units: one site per unit length, one step per unit time; every
 *    population hops ||n_i|| = 5 sites per step, so the speed of light (the
 *    Fermi velocity of the paper's graphene application) is 5 sites/step.
 *  - Velocities are 3-velocities u = U_s / U^0 (|u| < 1 in units of c).
 *  - Field arrays are nx*ny float64, row-major with y the slow index:
 *    a[y * nx + x].  on_device = 0: host pointers; 1: device pointers on the
 *    lattice's device (e.g. torch tensor data_ptr()); the copy is ordered on
 *    the lattice's stream.
 *  - Population index i = 4*d + j: direction d in 0..11 sorted by angle,
 *    (5,0),(4,3),(3,4),(0,5),(-3,4),(-4,3),(-5,0),(-4,-3),(-3,-4),(0,-5),
 *    (3,-4),(4,-3) (opposite of d is (d+6)%12), shell j in 0..3 in the order
 *    the paper prints the energies p0_j.
 *  - Every call returns an rlbm_status; on failure rlbm_last_error() holds a
 *    thread-local message.  No C++ exception crosses this boundary.
 *  - Ownership: the library owns every device buffer it allocates (the two
 *    population arrays, fields, constants); it never frees caller memory.
 *    Calls on one lattice are not thread-safe; different lattices are
 *    independent.
 */
#ifndef RLBM_H
#define RLBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct rlbm_lattice rlbm_lattice;

typedef enum {
    RLBM_OK = 0,
    RLBM_EINVAL = -1,    /* bad argument (sizes, tau <= 1/2, contact outside an edge, NULL handle) */
    RLBM_ENOMEM = -2,    /* device or host allocation failed */
    RLBM_EDEVICE = -3,   /* a HIP call failed */
    RLBM_ESTATE = -4,    /* call out of order (e.g. step before init) */
    RLBM_EUNSTABLE = -5, /* health check: non-finite value, n <= 0 or |u| >= 1 somewhere */
    RLBM_ENOTFOUND = -6  /* a search (rlbm_quadrature.h) found no admissible solution */
} rlbm_status;

/* Storage of the populations.  All three store the deviation
 * (f_i - f_ref_i) / (w_i * scale) from the rest equilibrium f_ref of a
 * reference state (n_ref, T_ref) (see rlbm_set_reference).
 *   RLBM_F64:    float64 storage, float64 arithmetic (the parity path).
 *   RLBM_F32:    float32 storage, float32 arithmetic; moments are turned
 *                into the Landau frame in float64.
 *   RLBM_F16DEV: float16 storage of the scaled deviation, float32
 *                arithmetic, float64 Landau frame.
 * Device layout (seen only in the raw population part of a checkpoint):
 * F64 and F32 hold 48 planes of nx*ny values, plane i = population i;
 * F16DEV holds 12 arrays of nx*ny tuples, array d holding at each site the
 * four shells of direction d (populations 4d .. 4d+3) in 8 bytes.  Every
 * other call that takes or returns populations uses the 48-plane layout. */
typedef enum { RLBM_F64 = 0, RLBM_F32 = 1, RLBM_F16DEV = 2 } rlbm_storage;

typedef enum { RLBM_EDGE_BOTTOM = 0, RLBM_EDGE_TOP = 1, RLBM_EDGE_LEFT = 2, RLBM_EDGE_RIGHT = 3 } rlbm_edge;

/* Inlet/outlet ("sites that do not evolve in time", Sec. 3): a ghost span of
 * the five rows (columns) just outside an edge, at positions
 * [start, start + width) along that edge (x for bottom/top, y for
 * left/right), held at the equilibrium f^eq(n, T, u = (vx, vy)).  A
 * population pulled from the span takes that equilibrium value; one that
 * streams into it is absorbed. */
typedef struct {
    int edge;
    int start;
    int width;
    double n, T, vx, vy;
} rlbm_contact;

/* ---- library-wide ---- */

/* Message of the last failed call on this thread ("" if none). */
const char *rlbm_last_error(void);

/* ABI version (incremented on incompatible changes): 2 (the autotuner
 * reports 12 timings). */
int rlbm_version(void);

/* The quadrature the library uses (Sec. 2.3): the printed weights w_1j
 * (directions (+-3,+-4)_FS), w_2j ((+-5,0)_FS) and energies p0_j, polished on
 * the host onto an exact solution of the orthonormality conditions
 * (Eq. orthonormal): the solution closest to the printed values.  Host-only;
 * needs no device.  Arrays of 4, caller-owned. */
rlbm_status rlbm_quadrature(double w1[4], double w2[4], double p0[4]);

/* The force projection matrices C_x, C_y (row-major 16x16, caller-owned),
 * b_j = C_j a in the polynomial basis of Appendix A (Sec. 2.4), computed on
 * the host.  Host-only. */
rlbm_status rlbm_force_matrices(double Cx[256], double Cy[256]);

/* ---- one lattice ---- */

/* Create an nx x ny lattice (nx, ny >= 1, nx*ny < 2^31, one plane or
 * tuple array below 4 GiB; RLBM_EINVAL otherwise) on the current HIP device.
 * hip_stream: a hipStream_t to order all work on (NULL = the null stream).
 * Defaults: all edges are walls, no contacts, no mask, tau = 1, no drive,
 * reference (n_ref, T_ref) = (1, 1), scale 1 (F64/F32) or 2^-12 (F16DEV).
 * The lattice must be initialised (rlbm_init_*) before stepping. */
rlbm_status rlbm_create(int nx, int ny, rlbm_storage storage, void *hip_stream, rlbm_lattice **out);

/* Release every device buffer of the lattice (after its stream drains).  NULL is a no-op. */
void rlbm_destroy(rlbm_lattice *lat);

/* Geometry (Sec. 3): periodic_x / periodic_y wrap that axis; every other edge
 * is a bounce-back wall (on-site reversal, f_i(x, t+1) = f*_opp(i)(x, t))
 * except where a contact's ghost span lies.  Precedence for a pull source
 * outside the lattice: periodic wrap, then contact, then wall.  Contacts on a
 * periodic edge, overlapping contacts or spans outside [0, edge length) give
 * RLBM_EINVAL.  At most 16 contacts.  Takes effect at the next init or step. */
rlbm_status rlbm_set_boundaries(rlbm_lattice *lat, int periodic_x, int periodic_y,
                                const rlbm_contact *contacts, int ncontacts);

/* Optional solid sites (host array nx*ny, 1 = solid, 0 = fluid; NULL clears
 * the mask).  A pull from a solid site bounces back like a wall; solid sites
 * are not updated and report n = u = eps = 0. */
rlbm_status rlbm_set_mask(rlbm_lattice *lat, const uint8_t *mask);

/* Relaxation (proper) time tau in steps (Eq. discrete-rbe); tau <= 1/2 gives
 * RLBM_EINVAL.  The shear diffusivity is 6.25 (tau - 1/2) sites^2/step. */
rlbm_status rlbm_set_tau(rlbm_lattice *lat, double tau);

/* Constant external 3-force per particle F = (Fx, Fy) on every fluid site
 * (Sec. 2.4 forcing scheme; the electrostatic drive of Sec. 3 held uniform). */
rlbm_status rlbm_set_drive(rlbm_lattice *lat, double Fx, double Fy);

/* Local-capacitance electrostatics (Sec. 3, Eq. lca): the potential
 * phi = -e n / C_g adds the per-particle force -(e^2 / C_g) grad n (carriers
 * repel; e = 1 in lattice units) to the drive: F = (Fx, Fy) - inv_cg grad n.
 * grad n is the central difference of the density of the previous state (of
 * f(0) itself for the first collision); a neighbour off the lattice (no
 * periodic wrap) or solid takes the site's own density.  inv_cg = 1/C_g must
 * be finite and >= 0 (RLBM_EINVAL otherwise); 0 switches the term off
 * (C_g = infinity).  Best set before rlbm_init_*; switched on later, the
 * previous density is taken from the current fields (RLBM_ESTATE if there
 * are none).  Costs one extra 8-byte density read and write per site and
 * step.  Lattices with the term on cannot be stepped in a batch. */
rlbm_status rlbm_set_lca(rlbm_lattice *lat, double inv_cg);

/* Use another member of the family of massless third-order quadratures on
 * the 48-node stencil (Sec. 2.3; the solutions form a two-parameter family,
 * see rlbm_quadrature_massless in rlbm_quadrature.h): w1[4] are the weights
 * of the (+-3,+-4)_FS directions, w2[4] of (+-5,0)_FS, p0[4] the shell
 * energies (host arrays).  Checked on the host: weights >= 0, energies > 0,
 * and Eq. `orthonormal` (every monomial condition of degree <= 6, each
 * relative to max(|moment|, 1)) to 1e-12, else RLBM_EINVAL.  The lattice
 * becomes uninitialised: call rlbm_init_* next. */
rlbm_status rlbm_set_quadrature(rlbm_lattice *lat, const double w1[4], const double w2[4], const double p0[4]);

/* Reference state of the deviation storage: f_ref_i = f^eq_i(n_ref, T_ref, 0)
 * and the stored value is (f_i - f_ref_i) / (w_i * scale).  Must be called
 * before rlbm_init_*; n_ref > 0, T_ref > 0, scale > 0. */
rlbm_status rlbm_set_reference(rlbm_lattice *lat, double n_ref, double T_ref, double scale);

/* Initial state f_i = f^eq_i(n, T, u) (Eq. feq-expansion-discrete) at every
 * fluid site, uniform or from nx*ny fields.  Resets the step counter to 0;
 * afterwards rlbm_read_fields returns the fields of this state. */
rlbm_status rlbm_init_uniform(rlbm_lattice *lat, double n, double T, double vx, double vy);
rlbm_status rlbm_init_fields(rlbm_lattice *lat, const double *n, const double *T,
                             const double *vx, const double *vy, int on_device);

/* Advance nsteps >= 0 time steps (asynchronous on the lattice's stream).  One
 * step is, at every fluid site: pull the 48 populations along the stencil
 * with the boundary rules, form N^a and T^ab, solve eps U^a = T^ab U_b for the
 * Landau frame, n = U_a N^a, T = eps / (2 n), build the order-3 equilibrium and
 * the forcing term, relax with p_i.U / (p0_i tau) and store.  The fields of the
 * last step are kept for rlbm_read_fields. */
rlbm_status rlbm_step(rlbm_lattice *lat, int64_t nsteps);

/* Number of steps taken since the last init. */
rlbm_status rlbm_get_time(rlbm_lattice *lat, int64_t *t);

/* Fields of the current state (time t): density n, 3-velocity (vx, vy) and
 * energy density eps.  Any pointer may be NULL.  Synchronises the stream when
 * on_device = 0. */
rlbm_status rlbm_read_fields(rlbm_lattice *lat, double *n, double *vx, double *vy, double *eps,
                             int on_device);

/* Residual of the last rlbm_step call of K steps, over fluid sites:
 * r = ||u(t) - u(t-K)||_2 / (K ||u(t)||_2), in float64 (0 if ||u(t)|| = 0).
 * Also runs the health check: RLBM_EUNSTABLE if any fluid site has a
 * non-finite field, n <= 0 or |u| >= 1 (r is still written).  Synchronises. */
rlbm_status rlbm_residual(rlbm_lattice *lat, double *r);

/* For callers that cannot allocate (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): rlbm_residual without any
 * allocation.  Same result as rlbm_residual, bit for bit (the per-block
 * partial sums are added in the same order), and the same health check
 * (RLBM_EUNSTABLE).  Its kernels keep their partial sums in a file-scope
 * device array of the library (3 x 1024 + 3 doubles, 24.6 KB per device,
 * held until the process ends) instead of the lattice's buffer; every
 * lattice qualifies (its kernel covers any size with at most 1024 blocks),
 * and a larger partial-sum count would give RLBM_EINVAL.  The array is
 * shared by every call on one device: calls that overlap on one device
 * (several threads, or lattices on several streams) race and must be
 * serialised by the caller.  The lattice's device must be current
 * (RLBM_ESTATE otherwise).  Synchronises the lattice's stream. */
rlbm_status rlbm_residual_noalloc(rlbm_lattice *lat, double *r);

/* Step until the residual over check_every steps falls below tol or
 * max_steps have been taken; writes the steps taken and the last residual.
 * Returns RLBM_EUNSTABLE from the health check. */
rlbm_status rlbm_step_until(rlbm_lattice *lat, int64_t max_steps, int64_t check_every, double tol,
                            int64_t *steps_taken, double *residual);

/* Post-collision populations f*_i(x, t) of the current state as float64
 * (48 planes of nx*ny, plane i = population i), decoded from the storage. */
rlbm_status rlbm_read_populations(rlbm_lattice *lat, double *f, int on_device);

/* Checkpoint: size of, copy out and restore the whole state (a header, the
 * raw population storage, the fields and, with the local-capacitance force
 * on, the previous density).  rlbm_set_state requires a lattice created with
 * the same nx, ny and storage and with the force on or off as when saved
 * (RLBM_EINVAL otherwise); continuing from a restored state is bit-identical
 * to continuing from the saved one.  Host buffers. */
rlbm_status rlbm_state_bytes(rlbm_lattice *lat, size_t *bytes);
rlbm_status rlbm_get_state(rlbm_lattice *lat, void *dst, size_t bytes);
rlbm_status rlbm_set_state(rlbm_lattice *lat, const void *src, size_t bytes);

/* Work decomposition of the step kernel: each 256-thread block of the
 * lattice interior (the rows 5 .. ny-6 at full width, when the lattice has
 * no solid mask and nx, ny > 10) covers tile_x consecutive sites (64, 128 or
 * 256: a multiple of the 64-wide wavefront) of rows = 256 / tile_x rows; the
 * top and bottom 5-row bands (every site, with a mask) run through a
 * host-built gather table.  Results do not depend on it (every site is
 * computed independently); only speed does.  Default: the largest of
 * 64/128/256 not above the width rounded up to 64. */
rlbm_status rlbm_set_launch_shape(rlbm_lattice *lat, int tile_x, int rows);
/* The lattice's current work decomposition (set, defaulted or chosen by an
 * autotuner, also for a sample of a batch); *tile_x, *rows: caller-owned,
 * either may be NULL. */
rlbm_status rlbm_get_launch_shape(rlbm_lattice *lat, int *tile_x, int *rows);

/* Block order of the step kernel: xcd_contiguous = 1 deals each of the 8
 * XCDs (with its own L2) one contiguous range of the launch's blocks, so
 * horizontally adjacent tiles, which share cache lines at their edges, run
 * under one L2; 0 (default) keeps the launch order, in which consecutive
 * blocks alternate between XCDs.  Results are identical either way. */
rlbm_status rlbm_set_block_order(rlbm_lattice *lat, int xcd_contiguous);

/* Boundary gather table: enabled = 1 (default) lets the lattice build its
 * host-side table of boundary sources (every site of a lattice with a solid
 * mask or no interior) whenever its population array is below 4 GiB;
 * enabled = 0 drops it, and the kernels then resolve every boundary source
 * in place with 64-bit addressing, as they do for lattices of 4 GiB and
 * more, which never have a table: the way to exercise that path at small
 * sizes.  Results are identical either way.  RLBM_EINVAL for other values;
 * takes effect for the next step (the table is rebuilt or freed at once,
 * synchronising the lattice's stream). */
rlbm_status rlbm_set_gather_table(rlbm_lattice *lat, int enabled);

/* Streaming (non-temporal) stores of the populations: on = 1 launches the
 * form of the step kernel whose stores bypass the caches.  Pays off once the
 * two population arrays outgrow the 256 MB Infinity Cache (the default
 * there; 12% faster at 4096 x 2048 in FP32); below it the next step's reads
 * hit the cache and ordinary stores are faster (25% at 1024 x 512).  Results
 * are identical either way.  Batches use the streaming form when every
 * active sample has it on. */
rlbm_status rlbm_set_streaming_stores(rlbm_lattice *lat, int on);

/* Non-temporal population loads: on = 1 launches the form of the step
 * kernel whose interior loads do not allocate in the caches, which leaves
 * the Infinity Cache to the populations the step stores (the next step's
 * input).  Pays off where one population array fits the 256 MB cache but
 * the two do not (FP64 at 1024 x 512: 4-5% faster than the best form
 * with ordinary loads); elsewhere it is slower (3-12% on the graphene
 * sample).  Off by default; the autotuner decides.  Results are identical either way.  Batches always use
 * ordinary loads.  Any nonzero on counts as 1. */
rlbm_status rlbm_set_streaming_loads(rlbm_lattice *lat, int on);

/* The memory form the next step launches with (as set, autotuned or read
 * from the tune cache at rlbm_create): *streaming_stores and
 * *nontemporal_loads receive 0 or 1; either pointer may be NULL. */
rlbm_status rlbm_get_memory_form(rlbm_lattice *lat, int *streaming_stores, int *nontemporal_loads);

/* Autotuner: time every candidate launch shape of the step kernel on this
 * lattice -- tile_x 64, 128, 256, each in four memory forms: ordinary
 * loads and stores, streaming stores, non-temporal loads, both --
 * (two rounds, the second in the reverse order, each candidate timed over
 * trial_steps steps after 2 warm-up steps with HIP events on the lattice's
 * stream and keeping the faster of its two runs), keep the fastest (the
 * setting on entry stays unless the fastest beats it by more than 1%), and
 * remember it for lattices of the same device architecture, storage, size
 * and mask use in this process (and in the text file named by the environment variable
 * RLBM_TUNE_CACHE, if set, which later processes read at rlbm_create).  The
 * lattice state, time and fields are restored afterwards.  ms_per_step
 * (optional, 12 entries since ABI version 2, caller-owned) receives those
 * timings for tile_x = 64, 128, 256 in the ordinary form, then the same with
 * streaming stores, with non-temporal loads, and with both (0 for a shape
 * that does not apply).  Synchronises. */
rlbm_status rlbm_autotune(rlbm_lattice *lat, int trial_steps, double *ms_per_step);

/* Block until all work queued on the lattice's stream is done. */
rlbm_status rlbm_synchronize(rlbm_lattice *lat);

/* ---- many lattices in one launch ---- */

typedef struct rlbm_batch rlbm_batch;

/* One sample of a batch: its own lattice size, boundaries (up to 4
 * contacts), tau, drive and uniform initial state. */
typedef struct {
    int nx, ny;
    int periodic_x, periodic_y;
    double tau, Fx, Fy;
    int ncontacts;
    rlbm_contact contacts[4];
    double n0, T0, vx0, vy0;
} rlbm_sample;

/* Create a batch of nsamples (>= 1) lattices with one storage, all ordered
 * on one stream (hip_stream, or a stream the batch creates when NULL), and
 * initialise each to its uniform equilibrium.  The samples may differ in
 * size and parameters.  Each sample starts with 256 x 1 tiles when its width
 * is a multiple of 256, else 64 x 4 (measured on a 256-sample batch of
 * widths 128..1024: 10% faster than 256 x 1 everywhere).  When their
 * populations together outgrow the 256 MB Infinity Cache, every sample
 * starts with streaming stores on. */
rlbm_status rlbm_batch_create(const rlbm_sample *samples, int nsamples, rlbm_storage storage, void *hip_stream,
                              rlbm_batch **out);

/* Release the batch and all its lattices.  NULL is a no-op. */
void rlbm_batch_destroy(rlbm_batch *b);

/* The lattice of sample i (owned by the batch): every single-lattice call
 * (fields, residual, init for warm starts, checkpoints, ...) works on it. */
rlbm_status rlbm_batch_lattice(rlbm_batch *b, int i, rlbm_lattice **lat);

/* Advance every active sample by nsteps.  Each step is ONE launch over the
 * list of (sample, block) work items of all active samples, in sample
 * order, one 256-thread block per item (each item is one block of that
 * sample's own step grid: boundary band or row tile); the grid is the
 * list's capacity and blocks past the current item count leave at once, so
 * freezing samples needs no new graph.  With use_graph the launches are
 * replayed from a captured HIP graph.  Fields are kept for the last step.  RLBM_EINVAL if an
 * active sample has the local-capacitance force on. */
rlbm_status rlbm_batch_step(rlbm_batch *b, int64_t nsteps, int use_graph);

/* Mark samples active (1) or frozen (0); frozen samples keep their state
 * and take no work.  active: nsamples bytes, caller-owned. */
rlbm_status rlbm_batch_set_active(rlbm_batch *b, const uint8_t *active);

/* Residual of every sample over its last rlbm_batch_step call (as
 * rlbm_residual), in one batched reduction; r has nsamples entries
 * (caller-owned).  RLBM_EUNSTABLE if any sample fails the health check. */
rlbm_status rlbm_batch_residual(rlbm_batch *b, double *r);

/* Step until every sample's residual over check_every steps is below tol or
 * max_steps have been taken; converged samples are frozen as they converge.
 * steps[i] receives the steps sample i took, r[i] its last residual (both
 * caller-owned, nsamples entries, may be NULL). */
rlbm_status rlbm_batch_step_until(rlbm_batch *b, int64_t max_steps, int64_t check_every, double tol,
                                  int64_t *steps, double *r);

/* Autotuner for the batch, in two stages, every time the faster of two runs
 * of trial_steps steps.  Stage 1: the samples' shapes and store forms as
 * they are, then every sample's tile width set to each candidate (64, 128,
 * 256, capped at the sample's width) with ordinary and with streaming
 * stores; the entry setting is kept unless a candidate is more than 1%
 * faster.  Stage 2: per width class (widths that are multiples of 256, of
 * 128 only, or neither), each tile width that divides the class's widths,
 * the other classes held at their best; a change is kept when more than 1%
 * faster.  Restores every sample's state and keeps the fastest setting.
 * ms_per_step: NULL or 6 entries, stage 1's candidates in that order. */
rlbm_status rlbm_batch_autotune(rlbm_batch *b, int trial_steps, double *ms_per_step);

/* Item order of the batched kernel, as rlbm_set_block_order: 1 deals each
 * XCD one contiguous range of the items in flight, 0 (default) interleaves
 * them.  Results are identical either way. */
rlbm_status rlbm_batch_set_block_order(rlbm_batch *b, int xcd_contiguous);

/* Total lattice sites of the active samples. */
rlbm_status rlbm_batch_sites(rlbm_batch *b, int64_t *sites);

#ifdef __cplusplus
}
#endif

#endif /* RLBM_H */
