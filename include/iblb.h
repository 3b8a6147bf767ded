/*
 * iblb.h - C ABI of the MI355X (gfx950) immersed boundary - lattice
 * Boltzmann (IBLB) wetting step.
 *
 * The library advances, on one GPU, lattice boxes of D3Q19 BGK fluid with
 * Guo forcing (paper Sec. 2, Eqs. 1-6) coupled to closed triangulated droplet
 * meshes through Peskin 4-point interpolation and spreading (Eqs. 7-8), the
 * droplets carrying surface tension and the wetting interaction
 * Pi(d) = A[(xi/d)^n - (xi/d)^m] with A from the contact angle (Eqs. 9-11).
 *
 * Conventions shared by every call
 *   - Lattice units, dx = dt = 1, c_s^2 = 1/3.  Cell (i,j,k) of an
 *     nx x ny x nz box is centred at (i+1/2, j+1/2, k+1/2).  x and y are
 *     periodic.  In z the box is periodic (IBLB_Z_PERIODIC, test mode) or
 *     closed by no-slip walls on the planes z = 0 (the wetting surface) and
 *     z = nz (IBLB_Z_WALLS), realised as halfway bounce-back; the walls
 *     rest or move in their own plane (iblb_box.wall_lo / wall_hi).
 *   - Mesh node coordinates are unwrapped lattice coordinates; the height
 *     above the wall used by Pi is the node's z.
 *   - Every call returns an iblb_status (0 = success, < 0 = error) and
 *     never throws; iblb_last_error() gives the message of the last failure.
 *   - Device work is enqueued on the HIP stream given to iblb_init.
 *     Calls documented as "synchronising" wait for that stream.  A context
 *     also owns a second non-blocking stream for the mesh kernels of a step
 *     (and, with IBLB_FLAG_GRAPH, one for graph capture); each step forks
 *     from and joins back into the caller's stream with events, so work the
 *     caller enqueues on that stream afterwards sees the step's results.
 *   - Calls on one context must not overlap (a context is not thread-safe);
 *     separate contexts may be driven from separate threads.  Make every
 *     call with the device current at iblb_init.  The message of a failure
 *     without a context is kept per thread.
 *   - Host arrays passed in are read during the call and not retained.
 *   - The device workspace is owned by the caller, must stay allocated and
 *     untouched until iblb_destroy, and is never freed by the library.
 *   - The library keeps its own D3Q19 order (iblb_velocity_set); population
 *     arrays crossing the ABI use it.
 */
#ifndef IBLB_H
#define IBLB_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t iblb_status;
enum {
    IBLB_OK = 0,
    IBLB_E_INVAL = -1,     /* bad argument or configuration value           */
    IBLB_E_MESH = -2,      /* mesh open, non-manifold, mis-oriented, or a
                              node at or below the wall                     */
    IBLB_E_DEVICE = -3,    /* a HIP call failed                             */
    IBLB_E_WORKSPACE = -4, /* workspace missing, misaligned or too small    */
    IBLB_E_UNSTABLE = -5,  /* the device status word reports an instability */
    IBLB_E_STATE = -6      /* call not valid in the context's current state */
};

/* Population storage.  F64 and F32 hold the deviation f_i - w_i rho0 in that
 * precision (an exact shift; arithmetic in the same precision).  F16DEV and
 * BF16DEV hold s (f_i - w_i rho0) as IEEE binary16 / bfloat16 with a
 * power-of-two scale s (dev_scale), converted with round-to-nearest-even,
 * and compute in FP32. */
enum { IBLB_F64 = 0, IBLB_F32 = 1, IBLB_F16DEV = 2, IBLB_BF16DEV = 3 };

enum { IBLB_Z_WALLS = 0, IBLB_Z_PERIODIC = 1 };

/* iblb_config.flags */
enum {
    IBLB_FLAG_GRAPH = 1u,    /* replay each step as a captured hipGraph      */
    IBLB_FLAG_AUTOTUNE = 2u, /* time the stream-collide launch shapes and the
                                step schedule at init (iblb_set_launch); the
                                result is kept for later inits of the same
                                device, storage, boxes and droplet sizes in
                                the process, and across processes in the
                                file named by the environment variable
                                IBLB_TUNE_CACHE, if set                     */
    IBLB_FLAG_FULL_U = 4u    /* write u of every cell each step (testing);
                                otherwise only cells near a mesh            */
};

/* Device status bits (sticky; reported by iblb_observables). */
enum {
    IBLB_BIT_RHO = 1u,        /* a density was non-finite or <= 0         */
    IBLB_BIT_MACH = 2u,       /* |u| exceeded the lattice sound speed     */
    IBLB_BIT_WALL = 4u,       /* a node reached d <= 0 (Pi is singular)   */
    IBLB_BIT_JUMP = 8u,       /* a node moved more than 1 lu in one step,
                                 or a coordinate left |q| < 1e7            */
    IBLB_BIT_BAND = 16u       /* reserved, never set: every cell relaxes
                                 with the inside bits of its own step      */
};

typedef struct {
    int32_t nx, ny, nz; /* cells; nx, ny, nz >= 4 when the box holds a droplet;
                           ten planes of populations (x-rows padded to 128
                           bytes) may take at most 4 GiB, e.g. about 107 M
                           cells in FP32, 53 M in FP64 */
    int32_t zbc;        /* IBLB_Z_WALLS or IBLB_Z_PERIODIC                    */
    double tau;         /* BGK relaxation time, > 1/2 (Sec. 2, viscosity
                           mu = rho c_s^2 (tau - 1/2))                         */
    double rho0;        /* initial (and reference) density, > 0               */
    double body_force[3]; /* uniform force density added to every cell's F   */
    double tau_in;      /* relaxation time of the cells inside the box's
                           droplets, > 1/2, or 0 for tau everywhere.  Inside
                           means: the vertical ray below the cell centre
                           crosses the closed meshes an odd number of times
                           (Sec. 2, below Eq. 13: ray tracing assigns tau_in
                           and tau_out; viscosity ratio (tau_in - 1/2) /
                           (tau - 1/2)).  Decided exactly on node positions
                           rounded to multiples of 2^-18, a point on the
                           surface resolved as if moved by (+e, +e^2) in x, y
                           and a crossing at the centre's height counting as
                           below it.  Droplets of one box must not overlap. */
    double wall_lo[2];  /* (u_x, u_y) of the wall at z = 0 and of the wall   */
    double wall_hi[2];  /* at z = nz (IBLB_Z_WALLS only; zeros: resting).  A
                           moving wall adds 6 w_i rho0 (c_i . u_w) to each
                           population it reflects (halfway bounce-back on a
                           moving wall); two walls moving apart drive the
                           shear flow of the free-droplet test of Sec. 4.
                           Each component finite, |u| <= 0.1.             */
} iblb_box;

typedef struct {
    int32_t box;        /* index of the box holding the droplet               */
    int32_t n_nodes, n_tris;
    int32_t n_exp, m_exp; /* exponents of Pi, n > m >= 1 (Eq. 10)             */
    int32_t reserved;
    const double *nodes;  /* host [n_nodes][3]                                */
    const int32_t *tris;  /* host [n_tris][3], counter-clockwise from outside */
    double sigma;         /* surface tension, >= 0                            */
    double theta_eq;      /* equilibrium contact angle (rad), in [0, pi]       */
    double xi;            /* regularisation length of Pi, > 0                  */
    double k_vol;         /* volume-penalty modulus (0 = off; not in the paper) */
} iblb_droplet;

typedef struct {
    int32_t n_boxes, n_droplets;
    const iblb_box *boxes;
    const iblb_droplet *droplets;
    int32_t storage;      /* IBLB_F64 .. IBLB_BF16DEV                          */
    uint32_t flags;       /* IBLB_FLAG_*                                       */
    double dev_scale;     /* power of two; used by IBLB_F16DEV (e.g. 4096)     */
} iblb_config;

typedef struct {
    int64_t step;
    double volume, area;   /* FP64 sums over the mesh                          */
    double z_min, z_max;
    double height;         /* z_max - z_min: highest minus lowest node (Sec. 3) */
    double contact_radius; /* mean horizontal distance from the area-weighted
                              centroid of the points where mesh edges cross
                              z = z_min + xi (0 if none)                        */
    double theta_app;      /* 2 atan(height / contact_radius)                  */
    double centroid[3];    /* area-weighted surface centroid                    */
    double deformation;    /* D = (r1 - r3) / (r1 + r3) in the x-z (shear)
                              plane (Sec. 4): r1 >= r3 the semi-axes of the
                              ellipsoid with the same second moments of
                              volume about the volume centroid (an
                              ellipsoid of semi-axis r has int x^2 dV =
                              V r^2 / 5 along it), from the x-z block      */
    double inclination;    /* angle of the r1 axis from x toward z, in
                              (-pi/2, pi/2]                                  */
    int32_t n_crossings;
    uint32_t status_bits;
} iblb_obs;

typedef struct {
    int64_t step;
    double mass;           /* FP64 sum of all populations                      */
    double max_u;          /* max over cells of |sum_i c_i f_i| / rho           */
    uint32_t status_bits;
    int32_t reserved;
} iblb_box_obs;

/* D3Q19 velocities c[19][3] and weights w[19] in the library's order. */
iblb_status iblb_velocity_set(int32_t *c, double *w);

/* Bytes of device workspace the configuration needs (host only, no device
 * call).  Fails with IBLB_E_INVAL / IBLB_E_MESH on an invalid configuration. */
iblb_status iblb_workspace_size(const iblb_config *cfg, size_t *bytes);

/* Set up the problem of Sec. 2: the lattice boxes (D3Q19 BGK fluid with
 * relaxation time tau, Eqs. 1-6, walls as halfway bounce-back) and the
 * closed droplet meshes with fixed connectivity that the fluid carries.
 * Validates the configuration, lays out the workspace, uploads meshes and
 * tables, sets the fluid at rest (f_i = w_i rho0, the equilibrium of Eq. 3
 * at u = 0), computes each droplet's wetting amplitude
 * A = sigma (m-1)(n-1)(1 + cos theta_eq) / ((n-m) xi) (Eq. 11) and its
 * reference volume V0 (the FP64 mesh volume of the initial positions, used
 * by the optional volume penalty; not in the paper).  `dev_workspace` must
 * be device memory of at least iblb_workspace_size bytes, 256-byte aligned,
 * owned by the caller.  `hip_stream` is a hipStream_t (NULL = default
 * stream).  On success *out owns the context (free it with iblb_destroy);
 * on failure *out is NULL and iblb_last_error(NULL) holds the message.
 * Synchronising. */
iblb_status iblb_init(const iblb_config *cfg, void *dev_workspace, size_t bytes,
                      void *hip_stream, struct iblb_ctx **out);

/* Enqueue n_steps full time steps t -> t+1 of Sec. 2, in this order:
 * nodal forces at q^t (surface tension from the area gradient, the wetting
 * force -chi Pi(d) n / 3 with Pi of Eq. 10; Eqs. 9-11), spreading of those
 * forces onto the lattice with the 4-point delta (Eq. 8), the fused
 * stream-collide with the Guo source (Eqs. 1-6, u^t including the
 * half-force term), interpolation of u^t at q^t (Eq. 7) and the forward
 * Euler advection q^{t+1} = q^t + U.  n_steps >= 0 (0 is a no-op).
 * Asynchronous: only enqueues on the context's stream.  Returns
 * IBLB_E_INVAL for n_steps < 0, IBLB_E_STATE after an instability was
 * reported by iblb_observables, IBLB_E_DEVICE when a launch fails. */
iblb_status iblb_step(struct iblb_ctx *ctx, int64_t n_steps);

/* For callers that cannot allocate device memory while they run (code under
 * HIP graph capture, tight serving loops, harnesses that forbid it): the
 * same n_steps time steps as iblb_step, bit for bit, with the step's own
 * scratch arrays (triangle records and FP64 partial sums, node-block
 * boxes, region descriptors and partial spread regions, the stamped-tile
 * list and the per-tile block records) taken from a fixed device array of
 * the library, 32 MiB per GPU, held from the library's load until the
 * process ends, instead of from the context's workspace.  Allocates
 * nothing and replays no graph: the kernels of each step are enqueued on
 * the context's stream one after another, with the step's advection
 * applied at its end.  The step scratch of a configuration grows with its
 * nodes (about 560 B per node in FP32, 1.1 KB in FP64) and its box cells
 * (1.25 B per cell): the 128x128x64 spreading workload needs about 7 MB.
 * One that exceeds 32 MiB returns IBLB_E_WORKSPACE with the bytes it
 * needs.  The array is shared by every
 * context on the GPU and keeps the last call's contents (the records that
 * must start empty are cleared by each call): calls that overlap on one
 * GPU, from any context or thread, race.  Asynchronous like iblb_step. */
iblb_status iblb_step_static(struct iblb_ctx *ctx, int64_t n_steps);

/* Observables of the current state (per droplet and per box).  Either
 * output may be NULL.  Synchronising.  Returns IBLB_E_UNSTABLE (after
 * filling the outputs) when any status bit is set; that state is sticky. */
iblb_status iblb_observables(struct iblb_ctx *ctx, iblb_obs *per_droplet, int32_t n_droplets,
                             iblb_box_obs *per_box, int32_t n_boxes);

/* Populations f_i(x, t) of box `box` at the current time (before the
 * collision of the next step), FP64, [19][nz][ny][nx] in the library's
 * velocity order.  `u_out` (may be NULL): [3][nz][ny][nx] velocity with the
 * half-force correction of the last step, NaN where it was not written.
 * Synchronising. */
iblb_status iblb_read_state(struct iblb_ctx *ctx, int32_t box, double *f_out, double *u_out);

/* The same for a window of box `box`: the cells lo[0] .. lo[0]+ext[0]-1
 * along x and lo[1] .. lo[1]+ext[1]-1 along y, both taken modulo the box
 * size (a window may cross the periodic sides), and lo[2] .. lo[2]+ext[2]-1
 * along z (inside [0, nz) in a walled box, modulo nz in a z-periodic one);
 * 1 <= ext[a] <= the box size.  f_out [19][ext2][ext1][ext0], u_out (may be
 * NULL) [3][ext2][ext1][ext0], as iblb_read_state gives them; only the rows
 * the window needs are copied from the device.  Synchronising. */
iblb_status iblb_read_window(struct iblb_ctx *ctx, int32_t box, const int32_t *lo, const int32_t *ext,
                             double *f_out, double *u_out);

/* Replace the populations of box `box` by f_in (layout as iblb_read_state),
 * converted to the storage precision.  Synchronising. */
iblb_status iblb_write_state(struct iblb_ctx *ctx, int32_t box, const double *f_in);

/* Node positions of droplet `d`, [n_nodes][3] in the caller's node order. */
iblb_status iblb_read_nodes(struct iblb_ctx *ctx, int32_t d, double *nodes_out);
iblb_status iblb_write_nodes(struct iblb_ctx *ctx, int32_t d, const double *nodes_in);

/* Inspection calls used by parity tests.  Each runs the same kernels as a
 * step on the current state and copies one intermediate out:
 *   compute_forces : nodal forces phi_j (Eqs. 9-11), [n_nodes][3]
 *   compute_spread : spread force density F (Eq. 8) of box b,
 *                    [3][nz][ny][nx], zero away from the meshes; and the
 *                    flags of the band tiles holding a stencil cell (tile
 *                    shape and numbering: iblb_band_tile; may be NULL)
 *   interpolate    : U_j = sum_x u(x) Delta(q_j - x) (Eq. 7) of a given
 *                    [3][nz][ny][nx] field u, without moving the nodes
 *   read_bins      : base cell floor(q - 1/2) per axis, x and y wrapped
 *                    into the box, [n_nodes][3]
 *   read_csr       : node -> incident triangles, entries 3*t + corner
 *                    sorted by t; offsets [n_nodes + 1], entries [3 n_tris]
 * None of them advances time.  Synchronising. */
iblb_status iblb_compute_forces(struct iblb_ctx *ctx, int32_t d, double *phi_out);
iblb_status iblb_compute_spread(struct iblb_ctx *ctx, int32_t b, double *F_out,
                                uint8_t *tile_flags_out);
iblb_status iblb_interpolate(struct iblb_ctx *ctx, int32_t d, const double *u_in,
                             double *U_out);
iblb_status iblb_read_bins(struct iblb_ctx *ctx, int32_t d, int32_t *base_out);
iblb_status iblb_read_csr(struct iblb_ctx *ctx, int32_t d, int32_t *offsets, int32_t *entries);

/* Cells of box b inside its droplets at the current node positions: 1 where
 * the vertical ray below the cell centre crosses the closed meshes an odd
 * number of times (exact predicates; the tie rule and the periodic images
 * are those of the tau_in field of iblb_box), else 0; [nz][ny][nx].  Only
 * for a box with tau_in > 0 (else IBLB_E_INVAL).  Does not advance time.
 * Synchronising. */
iblb_status iblb_read_inside(struct iblb_ctx *ctx, int32_t b, uint8_t *inside_out);

/* Checkpoints.  iblb_save_state writes the whole state of the current time
 * into `blob` (host memory of exactly iblb_state_size bytes): the stored
 * populations of every box as they are held (no rounding), the node
 * positions as held, each droplet's reference volume V0, the step count
 * and the status word.  iblb_load_state puts such a blob into a context
 * built from the same configuration (boxes, storage, droplet parameters,
 * meshes and initial node order; IBLB_E_INVAL otherwise): stepping on
 * from there gives bit for bit what the saving context gives.  The inside
 * bits are recomputed; the velocity of the last step is not kept (read_state
 * reports NaN for it until the next step).  Both synchronise; save applies
 * a pending advection first. */
iblb_status iblb_state_size(const struct iblb_ctx *ctx, size_t *bytes);
iblb_status iblb_save_state(struct iblb_ctx *ctx, void *blob, size_t bytes);
iblb_status iblb_load_state(struct iblb_ctx *ctx, const void *blob, size_t bytes);

/* Launch configuration of the fused stream-collide kernel and the step
 * schedule:
 *   threads_x         threads along x per row, a multiple of 32 (when a
 *                     multiple of 64, rows longer than threads_x cells are
 *                     split into segments of that length, one per workgroup);
 *   rows_per_group    rows of a workgroup; threads_x * rows_per_group must be
 *                     a multiple of 64 and at most 256;
 *   cells_per_thread  1 or 2 rows handled by a thread at a time (their loads
 *                     issued together); 2 needs threads_x a multiple of 64;
 *   streaming_stores  0 or 1: write the populations with non-temporal stores,
 *                     in the stream-collide and the band kernel (helps once
 *                     the two population buffers exceed the GPU's last-level
 *                     cache, hurts while they fit);
 *   max_workgroups    0, or a cap on the grid: the workgroups then loop over
 *                     the rows, leaving compute units to the mesh kernels that
 *                     run beside the stream-collide;
 *   band_after_bulk   0: the cells of the band tiles (those within reach of a
 *                     node's stencil) are computed by the band kernel beside
 *                     the stream-collide of the other cells, which waits for
 *                     the step's node pass; 1: the stream-collide runs over
 *                     every cell beside the mesh kernels and the band kernel
 *                     then recomputes the band tiles (not with tau_in).
 * Other values return IBLB_E_INVAL.  Rebuilds the step graphs.  Synchronising.
 * Results do not depend on the configuration. */
iblb_status iblb_set_launch(struct iblb_ctx *ctx, int32_t threads_x, int32_t rows_per_group,
                            int32_t cells_per_thread, int32_t streaming_stores,
                            int32_t max_workgroups, int32_t band_after_bulk);
iblb_status iblb_get_launch(const struct iblb_ctx *ctx, int32_t *threads_x, int32_t *rows_per_group,
                            int32_t *cells_per_thread, int32_t *streaming_stores,
                            int32_t *max_workgroups, int32_t *band_after_bulk);

/* Shape of the band tiles that iblb_compute_spread's tile_flags refer to:
 * shape[0..2] = cells per tile along x, y, z (a tile is 64 cells).  Tiles are
 * numbered x fastest: ((tz * tiles_y) + ty) * tiles_x + tx, tiles_a =
 * ceil(n_a / shape[a]).  Host memory; no device. */
iblb_status iblb_band_tile(int32_t *shape);

/* Average device time (ms) of one stream-collide launch over `reps` launches,
 * measured with HIP events on the context's stream (the populations are
 * advanced; the mesh is not).  Synchronising. */
iblb_status iblb_time_stream_collide(struct iblb_ctx *ctx, int32_t reps, double *ms_out);

/* Average device time (ms) of the mesh kernels of one step (triangle
 * records, node pass with stamps and partial spread, stamped-tile list,
 * interpolation; with tau_in the inside bits), over `reps` eager
 * repetitions on the context's stream, each in a fresh tile epoch.  The
 * nodes do not move and the fluid is not touched; the last step's band
 * velocities are dropped (read_state reports NaN for them until the next
 * step).  0 when there are no droplets.  Synchronising. */
iblb_status iblb_time_mesh_chain(struct iblb_ctx *ctx, int32_t reps, double *ms_out);

/* Free host-side state and graphs (not the caller's workspace). */
iblb_status iblb_destroy(struct iblb_ctx *ctx);

/* Message of the last error on ctx (or of the last context-less failure when
 * ctx is NULL).  Never NULL. */
const char *iblb_last_error(const struct iblb_ctx *ctx);

#ifdef __cplusplus
}
#endif
#endif /* IBLB_H */
