/*
 * roeam.h -- C ABI of the MI355X (gfx950) Roe-AM finite-volume library.
 *
 * The library evaluates the Roe-AM numerical flux of Li, Ren and Gu
 * ("An Improved Roe Scheme for All Mach-Number Flows Simultaneously Curing
 * Known Problems", arXiv 1711.09272, Sec. 6.2, Eqs. 85-109) on every face of a
 * structured 2-D grid, sums the face fluxes into the cell residual of a
 * finite-volume method (Sec. 2.2, Eqs. 2-4) and advances the conserved state
 * Q = (rho, rho u, rho v, rho E) of the Euler equations (Eq. 1, with w = 0)
 * with an explicit Runge-Kutta method.  All arithmetic runs in HIP kernels on
 * the GPU; nothing here falls back to the CPU.
 *
 * Conventions
 *   - State arrays are device memory, FP64, structure of arrays:
 *     q[k][j][i] at q + k*ny*pitch + j*pitch + i, k = 0..3 (rho, rho u,
 *     rho v, rho E) and k = 4..3+ns for a grid carrying ns transported
 *     scalars (rho k_m, see roeam_grid_set_scalars), j = 0..ny-1, i = 0..nx-1.  The row pitch (in elements)
 *     is chosen by the library and read back with roeam_grid_layout(); pad
 *     elements i >= nx are never read or written.
 *   - Every function returns a roeam_status; no C++ exception crosses the
 *     ABI.  Argument errors are reported synchronously.  Numerical failure
 *     (a non-physical state) is detected on the device and reported with the
 *     step statistics or by the batch poll.
 *   - Work is enqueued on the context's HIP stream and is asynchronous unless
 *     a function says otherwise.  Caller-owned buffers must stay valid until
 *     that stream has finished the work.
 *   - A context must be used by one host thread at a time.
 */
#ifndef ROEAM_H
#define ROEAM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    ROEAM_OK = 0,
    ROEAM_EINVAL = -1,    /* invalid argument (see each function)                  */
    ROEAM_ENOMEM = -2,    /* device allocation failed or the arena is too small     */
    ROEAM_EDEVICE = -3,   /* a HIP runtime call failed                              */
    ROEAM_ENONPHYS = -4,  /* rho <= 0, p <= 0 or a non-finite value was produced     */
    ROEAM_EBUSY = -5,     /* the request cannot be admitted now                     */
    ROEAM_ENOTFOUND = -6  /* unknown batch ticket                                   */
} roeam_status;

typedef struct roeam_ctx roeam_ctx;   /* device, stream, kernel tables, batch engine      */
typedef struct roeam_grid roeam_grid; /* immutable grid: sizes, metrics, boundary kinds    */

/* Boundary kinds (the paper's Sec. 7 cases use inflow, outflow, walls and
 * periodic directions; the ghost-cell rules themselves are not printed):
 *   PERIODIC      wrap around;
 *   TRANSMISSIVE  copy the nearest interior cell (zero gradient);
 *   SLIPWALL      mirror the interior cells and reflect the velocity about the
 *                 wall-face normal;
 *   DIRICHLET     a fixed state supplied at grid creation;
 *   MOVING        (uniform grids) a side split at a + b t along it: below the
 *                 split (cell-centre coordinate x for south/north, y for
 *                 west/east) the side's Dirichlet state from grid creation or
 *                 a slip wall, above it a slip wall or a second Dirichlet
 *                 state (see roeam_grid_set_moving_side; until then the whole
 *                 side is Dirichlet).  t is the time of the state the stage
 *                 reads: the step's start plus 0, dt, dt/2 for the SSP-RK3
 *                 stages and 0, dt/4, dt/3, dt/2 for the four-stage scheme.
 *                 The double-Mach reflection of Sec. 7.4 needs it (a wall
 *                 from x = 1/6 on, a top side that follows the exact incident
 *                 shock), and so does the supersonic corner of Sec. 7.3 (the
 *                 step's wall below the corner, the inflow above it; b = 0).
 * Two ghost layers are used.  Corner ghosts apply the x rule first and then
 * the y rule. */
typedef enum {
    ROEAM_BC_PERIODIC = 0,
    ROEAM_BC_TRANSMISSIVE = 1,
    ROEAM_BC_SLIPWALL = 2,
    ROEAM_BC_DIRICHLET = 3,
    ROEAM_BC_MOVING = 4
} roeam_bc;

enum { ROEAM_WEST = 0, ROEAM_EAST = 1, ROEAM_SOUTH = 2, ROEAM_NORTH = 3 };

/* Grid metrics: the face-normal vectors and face lengths of Eq. (4) and the
 * cell areas of the finite-volume sum come from either a uniform spacing or
 * the node coordinates of a structured grid.
 *   kind 0: uniform, cell (i, j) = [i dx, (i+1) dx] x [j dy, (j+1) dy];
 *   kind 1: node coordinates xn, yn, HOST pointers to (ny+1)*(nx+1) doubles,
 *           row-major [j][i]; the library copies them.  The i-face between
 *           cells (i-1, j) and (i, j) joins nodes (i, j) and (i, j+1); its
 *           vector is (y(i,j+1) - y(i,j), -(x(i,j+1) - x(i,j))).  The j-face
 *           between (i, j-1) and (i, j) joins nodes (i, j) and (i+1, j); its
 *           vector is (-(y(i+1,j) - y(i,j)), x(i+1,j) - x(i,j)).  Cell areas
 *           by the shoelace formula. */
typedef struct {
    int kind;
    double dx, dy;
    const double *xn, *yn;
} roeam_metrics;

/* Variant bits of the Roe-AM scheme: alternative readings of ambiguous
 * passages (bits 0-2) and the ablations the paper compares in Sec. 7 (bits
 * 3-7).  0 = the scheme of Eqs. (85)-(109) with the default readings.  When
 * both bits 4 and 6 are set bit 4 wins; when both 5 and 7 are set bit 7 wins. */
#define ROEAM_V_XI_UNGATED   (1u << 0) /* xi as printed in Eq. (86), without the Eq. (68) gate */
#define ROEAM_V_EXPFIX_F8    (1u << 1) /* f^8(Mbar) weight of Eq. (73) instead of f(Mbar)       */
#define ROEAM_V_CLAMP_UPRIME (1u << 2) /* clamp |U|' of Eq. (92) at zero                        */
#define ROEAM_V_NO_EQ92      (1u << 3) /* |U|' = |U|: no expansion-shock fix                    */
#define ROEAM_V_XI_ROE       (1u << 4) /* xi = |U| of classical Roe, Eq. (13)                   */
#define ROEAM_V_DUP_ROE      (1u << 5) /* dU_p of classical Roe, Eq. (17)                       */
#define ROEAM_V_XI_EQ46      (1u << 6) /* xi = |U_R + U_L| / 2 of Eq. (46)                      */
#define ROEAM_V_DUP_ZERO     (1u << 7) /* dU_p = 0                                              */
#define ROEAM_V_SUPPORTED    0xffu

/* Flux scheme. */
#define ROEAM_SCHEME_ROEAM      0 /* Roe-AM, Eqs. (85)-(109)                                   */
#define ROEAM_SCHEME_ROE        1 /* classical Roe, Eq. (7) with Eqs. (8)-(12)                 */
#define ROEAM_SCHEME_ROE_HARTEN 2 /* classical Roe with Harten's entropy fix, Eqs. (114)-(115) */

/* Scheme parameters.
 *   gamma     ratio of specific heats (Eq. 54), > 1;
 *   cfl       Courant number of the time-step rule, > 0 (roeam_step only);
 *   mach_ref  global reference Mach number of Eq. (101), > 0;
 *   u_ref     reference speed of Eq. (108), >= 0;
 *   eps1      switch of Eq. (111): 0 or 1;
 *   eps2      entropy-fix constant of Eq. (112), >= 0 (paper: 0.05);
 *   s1_mode   0: pressure-density detector of Eqs. (95)-(97); 1: s1 = 1 (Eq. 110);
 *   order     1: piecewise-constant face states (Sec. 7.1);
 *             2: MUSCL-minmod on (rho, u, v, p);
 *   time_scheme 0: forward Euler; 1: three-stage SSP Runge-Kutta;
 *             2: the four-stage Runge-Kutta of Sec. 7.1 (read as the
 *                low-storage form Q^(k) = Q^n + a_k dt R(Q^(k-1)),
 *                a = 1/4, 1/3, 1/2, 1);
 *   precision 0: FP64 throughout;
 *             1: flux coefficients in FP32, with the state, the jumps of
 *                Eq. (85), the central term and the residual sum in FP64;
 *   variant   ROEAM_V_* bits (Roe-AM scheme only);
 *   scheme    ROEAM_SCHEME_*; the classical schemes ignore mach_ref, u_ref,
 *             eps1, eps2, s1_mode and variant in the flux (mach_ref still
 *             enters the time-step rule below);
 *   eps_lambda threshold factor of Harten's fix, Eq. (115), >= 0.
 * Time step: dt = cfl / max over cells of
 *   (|V.Si| + ce |Si| + |V.Sj| + ce |Sj|) / Omega,  ce = c / sqrt(theta_cell),
 * with Si, Sj the means of opposite face vectors and theta_cell of Eq. (101)
 * from the cell Mach number (ce bounds the speed of the low-Mach dU_p term
 * of Eq. 89). */
typedef struct {
    double gamma, cfl, mach_ref, u_ref, eps1, eps2;
    int s1_mode, order, time_scheme, precision;
    unsigned variant;
    int scheme;
    double eps_lambda;
} roeam_params;

typedef struct {
    double t;        /* time reached                                             */
    double dt_last;  /* last time step taken                                     */
    double max_rate; /* max explicit rate that set dt_last                       */
    long steps;      /* steps taken by this call                                 */
    int nonphys;     /* nonzero if a non-physical state was produced              */
} roeam_step_stats;

/* Create a context on HIP device `device`, enqueueing on `hip_stream`
 * (a hipStream_t; NULL = the null stream).  EINVAL: bad device; EDEVICE. */
roeam_status roeam_ctx_create(int device, void *hip_stream, roeam_ctx **out);
roeam_status roeam_ctx_destroy(roeam_ctx *ctx);
/* Rebind the stream used by later calls. */
roeam_status roeam_ctx_set_stream(roeam_ctx *ctx, void *hip_stream);
/* Text of the last error of this context (never NULL). */
const char *roeam_last_error(const roeam_ctx *ctx);

/* Create a grid of nx x ny cells (nx, ny >= 2, nx * ny < 2^31).  bc[4] = kinds for west,
 * east, south, north; a periodic kind must be used on both sides of its
 * direction.  dirichlet_state: HOST array [4 sides][4] of conserved states,
 * used by DIRICHLET sides (NULL allowed if none).  The grid owns device
 * copies of its metrics and, from its first roeam_step on, two stage
 * buffers of the state size (batched solves use the batch arena instead).
 * EINVAL: sizes, kinds or metrics invalid (non-positive spacing or cell
 * area); ENOMEM. */
roeam_status roeam_grid_create(roeam_ctx *ctx, int nx, int ny, const roeam_metrics *metrics,
                               const int bc[4], const double *dirichlet_state, roeam_grid **out);
roeam_status roeam_grid_destroy(roeam_grid *grid);
/* Layout of state arrays: q[k][j][i] at k*ny*pitch + j*pitch + i. */
roeam_status roeam_grid_layout(const roeam_grid *grid, int *nx, int *ny, long *pitch);
/* Tile shape of the stage kernel for this grid (cells per workgroup /
 * threads): 0 = 32x15/256, 1 = 16x15/128, 2 = 8x7/64, 6 = 16x15/256,
 * 7 = 32x7/256 (one or two faces per thread), 3 = 8x7/128, 4 = 16x15/512,
 * 5 = 32x7/512, 8 = 16x7/256 (one face per thread), or -1 (default) =
 * chosen by the autotuner, which times every shape on the grid at its first
 * roeam_step and keeps the fastest per (order, precision).  Every shape
 * computes bitwise the same result.  EINVAL: shape outside -1..8. */
roeam_status roeam_grid_set_tile_shape(roeam_grid *grid, int shape);
/* Split of a ROEAM_BC_MOVING side: a + b t (a may be +-infinity); lo_kind
 * below the split: ROEAM_BC_DIRICHLET (the side's state from grid creation)
 * or ROEAM_BC_SLIPWALL; hi_kind above it: ROEAM_BC_SLIPWALL or
 * ROEAM_BC_DIRICHLET, state_hi a HOST conserved state [4] for the latter (NULL
 * otherwise).  Later calls see it.  EINVAL: not a moving side, NaN a,
 * non-finite b, bad lo_kind, hi_kind or state. */
roeam_status roeam_grid_set_moving_side(roeam_grid *grid, int side, double a, double b, int lo_kind, int hi_kind,
                                        const double *state_hi);
/* Time at which roeam_residual evaluates moving sides (default 0; steps use
 * their own stage times).  EINVAL: NULL grid, non-finite t. */
roeam_status roeam_grid_set_boundary_time(roeam_grid *grid, double t);

/* Transported scalars (Eq. 85: the rows rho k, ... of turbulence or species
 * variables, "other scalar equations" in Sec. 6.2).  A grid may carry up to
 * ROEAM_MAX_SCALARS of them as state rows 4 .. 3 + nscalars (rho k_m).  Their
 * flux is Eq. (85)'s: central U rho k, minus half of xi Delta(rho k)
 * + dU_p rho^ k^ + dU_u,R (rho k)_R + dU_u,L (rho k)_L (classical Roe:
 * xi Delta(rho k) + (dU_u + dU_p) rho^ k^), with k^ the sqrt(rho)-weighted Roe
 * average and no pressure term; MUSCL reconstructs k = (rho k)/rho.  The flow
 * rows do not depend on the scalars.  Boundary kinds act on k as on rho
 * (periodic, copy, mirror); a Dirichlet side takes dirichlet_scalars, a HOST
 * array [4 sides][nscalars] of rho k_m (NULL allowed when no side is
 * Dirichlet).  Call before the grid's residual or step calls; a change drops
 * the grid's stage buffers, captured graphs and tuned tile shapes (waiting for
 * the context stream first).  Grids with scalars run through every call,
 * roeam_batch_submit included (the batch engine groups solves by scalar
 * count); a grid's scalar count must not change while a solve of it is
 * submitted and not yet done.
 * EINVAL: nscalars outside 0..ROEAM_MAX_SCALARS, missing or non-finite
 * Dirichlet scalars; EDEVICE. */
#define ROEAM_MAX_SCALARS 2
roeam_status roeam_grid_set_scalars(roeam_grid *grid, int nscalars, const double *dirichlet_scalars);
/* The shape in use for these parameters (-1 if not tuned yet). */
roeam_status roeam_grid_tile_shape(const roeam_grid *grid, const roeam_params *params, int *shape);

/* Residual R = dQ/dt = -(1/Omega) sum over the cell's faces of F.S, with F the
 * Roe-AM flux of Eq. (85) (Sec. 2.2: finite-volume cell faces).
 * q: device, state layout, read only; r: device, state layout, written.
 * max_rate_out: nullable DEVICE pointer to one double that receives the
 * largest explicit rate of q (time-step rule above).  Runs the grid's set
 * tile shape, else the one tuned for these parameters, else 16x15/256 (it
 * does not tune).  Asynchronous.  EINVAL: NULL q/r, bad params; EDEVICE. */
roeam_status roeam_residual(roeam_ctx *ctx, const roeam_grid *grid, const roeam_params *params,
                            const double *q, double *r, double *max_rate_out);

/* Advance q (device, state layout) in place by up to nsteps steps of the
 * chosen time scheme, stopping when t reaches t_end (t_end <= 0: no stop;
 * the last step is shortened to land on t_end).  The step loop runs from
 * device-resident dt and t (no host synchronisation inside) as captured HIP
 * graphs.  If stats != NULL the call waits for the stream and fills it; a
 * non-physical state then returns ROEAM_ENONPHYS (q undefined).  With
 * stats == NULL the call is asynchronous; roeam_last_stats() reads them later.
 * EINVAL: NULL q, nsteps < 0, bad params; EDEVICE. */
roeam_status roeam_step(roeam_ctx *ctx, const roeam_grid *grid, const roeam_params *params,
                        double *q, long nsteps, double t0, double t_end, roeam_step_stats *stats);
/* Profiling aid (same arithmetic as roeam_step): advance q by nsteps steps
 * launching every kernel directly, with HIP events recorded on the context
 * stream around each stage kernel.  Waits for the stream, then writes the
 * mean duration in milliseconds of the stage kernels into stage_ms[0..3]
 * (first to fourth stage of a step; forward Euler fills stage_ms[0] only,
 * SSP-RK3 stage_ms[0..2]) and
 * the number of timed launches into *launches (nullable).
 * EINVAL as roeam_step; EDEVICE. */
roeam_status roeam_profile_step(roeam_ctx *ctx, const roeam_grid *grid, const roeam_params *params, double *q,
                                long nsteps, double t0, double stage_ms[4], long *launches);
/* Wait for the grid's last roeam_step and read its statistics. */
roeam_status roeam_last_stats(roeam_ctx *ctx, const roeam_grid *grid, roeam_step_stats *stats);
/* Norms of a residual array r (device, the grid's state layout, e.g. from
 * roeam_residual) for convergence monitoring: norms_out (DEVICE, 2 * rows
 * doubles, rows = 4 + nscalars) receives sqrt(mean over cells of r_k^2) in
 * [0, rows) and max |r_k| in [rows, 2 rows).  A fixed-order two-pass
 * reduction: the same bits on every call.  The grid keeps a small scratch
 * buffer, allocated at the first call.  Asynchronous.  EINVAL: NULL argument;
 * EDEVICE. */
roeam_status roeam_residual_norms(roeam_ctx *ctx, const roeam_grid *grid, const double *r, double *norms_out);
/* roeam_residual_norms without any allocation, for callers that cannot
 * allocate device memory: code under HIP graph capture, serving loops and
 * harnesses that forbid hipMalloc.  Same arguments, kernels and bits as
 * roeam_residual_norms.  Its partials live in a static device buffer of
 * 2 x 6 rows x 1024 blocks doubles (96 KiB) that every GPU the library runs on
 * holds until the process ends; its device address is taken when a context is
 * created on that GPU.  All calls on one GPU share that buffer, so calls whose
 * work overlaps on one GPU (other streams, other contexts, other host threads)
 * race: order them on one stream.  Nothing in the buffer needs clearing (each
 * call writes every partial it reads).  EINVAL: NULL argument, or a grid
 * whose partials exceed the buffer (more than 6 rows); EDEVICE. */
roeam_status roeam_residual_norms_noalloc(roeam_ctx *ctx, const roeam_grid *grid, const double *r, double *norms_out);

/* ------------------------------------------------------------------------ */
/* 3-D uniform Cartesian grids                                              */
/* ------------------------------------------------------------------------ */

/* The scheme in three dimensions (the paper states its equations in 3-D:
 * Eqs. 1-4 with w and n_z, the nine-face detector of Eq. 96 and the cross
 * products of Eq. 109): state Q = (rho, rho u, rho v, rho w, rho E), cell
 * (i, j, l) = [i dx, (i+1) dx] x [j dy, (j+1) dy] x [l dz, (l+1) dz].
 *   - State arrays are device memory, FP64, structure of arrays:
 *     q[k][l][j][i] at q + ((k*nz + l)*ny + j)*pitch + i, k = 0..4 + nscalars
 *     (rows rho, rho u, rho v, rho w, rho E, then the transported scalars rho k_m
 *     of roeam_grid3d_set_scalars); pad elements i >= nx are never read or
 *     written.
 *   - Boundary kinds as for 2-D grids, per side W, E, S, N, bottom (l < 0),
 *     top (l >= nz); ghost cells apply the x rule, then the y rule, then the
 *     z rule (edges and corners follow); a slip wall mirrors the cells and
 *     negates the velocity component normal to it.
 *   - The flux of a face normal to axis a is Eq. (85) with n = e_a; f_rr of
 *     Eq. (103) takes n2 along (n1 x n) x n1 (zero when n1 = +-n).
 *   - Time step: dt = cfl / max over cells of
 *     ((|u| + ce) dy dz + (|v| + ce) dx dz + (|w| + ce) dx dy) / (dx dy dz),
 *     ce as for 2-D grids.
 * All roeam_params fields mean what they mean for 2-D grids. */
enum { ROEAM_BOTTOM = 4, ROEAM_TOP = 5 };

typedef struct roeam_grid3d roeam_grid3d;

/* Create an nx x ny x nz grid (each >= 2, nx*ny*nz < 2^31) of spacing dx, dy,
 * dz (> 0).  bc[6] = kinds for W, E, S, N, bottom, top; a periodic kind must
 * be used on both sides of its direction.  dirichlet_state: HOST array
 * [6 sides][5] of conserved states for DIRICHLET sides (NULL allowed if none).
 * The grid owns two stage buffers of the state size from its first
 * roeam_step3d on.  EINVAL: sizes, spacing, kinds or Dirichlet states invalid;
 * ENOMEM; EDEVICE. */
roeam_status roeam_grid3d_create(roeam_ctx *ctx, int nx, int ny, int nz, double dx, double dy, double dz,
                                 const int bc[6], const double *dirichlet_state, roeam_grid3d **out);
roeam_status roeam_grid3d_destroy(roeam_grid3d *grid);
/* Layout of state arrays: q[k][l][j][i] at ((k*nz + l)*ny + j)*pitch + i. */
roeam_status roeam_grid3d_layout(const roeam_grid3d *grid, int *nx, int *ny, int *nz, long *pitch);
/* Transported scalars on a 3-D grid: as roeam_grid_set_scalars (Eq. 85 with its
 * rho k rows, here in three dimensions), state rows 5 .. 4 + nscalars;
 * dirichlet_scalars: HOST array [6 sides][nscalars] of rho k_m (NULL allowed
 * when no side is Dirichlet).  A change drops the grid's stage buffers and
 * captured graphs (waiting for the context stream first).  EINVAL: nscalars
 * outside 0..ROEAM_MAX_SCALARS, missing or non-finite Dirichlet scalars;
 * EDEVICE. */
roeam_status roeam_grid3d_set_scalars(roeam_grid3d *grid, int nscalars, const double *dirichlet_scalars);
/* Brick shape of the 3-D stage kernel (cells per workgroup / threads):
 * 0 = 8x8x4/256, 1 = 8x4x4/128, 2 = 16x8x4/512, 3 = 16x4x4/256,
 * 4 = 8x8x4/320, 5 = 8x4x4/192, 6 = 16x8x4/640, 7 = 8x8x8/576
 * (4-7: one thread per face of each direction), 8 = 16x8x4/512 and
 * 9 = 8x8x8/512 persistent (as many workgroups as the GPU holds, each taking a
 * band of bricks in turn and loading the next brick's halo while it computes
 * the current one).  10-12: z-marching column tiles of 16x15 cells with 256
 * threads, each workgroup walking a run of 4 (10), 8 (11) or 16 (12)
 * planes upward with one plane and its x-y halo in LDS while the next
 * plane's footprint loads into registers (three workgroups per CU); 13: the
 * same with every tile's height cut into as many equal runs as one round of
 * workgroups allows (not chosen by default: faster at 128^3, but it reads
 * more, and larger grids leave part of the round empty).  -1
 * (default): the z-marching shape with the longest run whose workgroups
 * still number at least nine per CU of the device (else runs of 4).  Every
 * shape computes bitwise the same result.  With two transported scalars the
 * 16x8x4 bricks (2, 6, 8) exceed the LDS of a workgroup; such a grid runs
 * shape 9 instead.  EINVAL: shape outside -1..13. */
roeam_status roeam_grid3d_set_tile_shape(roeam_grid3d *grid, int shape);
/* The shape the stage kernel runs with for MUSCL order `order` (1 or 2),
 * the default's choice and the scalar fallback applied.  EINVAL: NULL
 * argument, bad order. */
roeam_status roeam_grid3d_tile_shape(const roeam_grid3d *grid, int order, int *shape);
/* Residual R = dQ/dt = -(1/V) sum over the cell's six faces of F A (Eq. 85
 * per unit area times the face area).  q: device, 3-D state layout, read
 * only; r: device, same layout, written.  max_rate_out: nullable DEVICE
 * pointer to one double receiving the largest explicit rate of q.
 * Asynchronous.  EINVAL: NULL q/r, bad params; EDEVICE. */
roeam_status roeam_residual3d(roeam_ctx *ctx, const roeam_grid3d *grid, const roeam_params *params,
                              const double *q, double *r, double *max_rate_out);
/* Advance q (device, 3-D state layout) in place, as roeam_step does for 2-D
 * grids: up to nsteps steps of params->time_scheme from time t0, stopping at
 * t_end (t_end <= 0: no stop), device-resident dt and t, captured HIP graphs;
 * stats != NULL waits and fills them (ENONPHYS for a non-physical state).
 * EINVAL: NULL q, nsteps < 0, bad params; EDEVICE. */
roeam_status roeam_step3d(roeam_ctx *ctx, const roeam_grid3d *grid, const roeam_params *params, double *q,
                          long nsteps, double t0, double t_end, roeam_step_stats *stats);
/* Wait for the grid's last roeam_step3d and read its statistics. */
roeam_status roeam_last_stats3d(roeam_ctx *ctx, const roeam_grid3d *grid, roeam_step_stats *stats);
/* roeam_residual_norms for a 3-D residual array (rows = 5 + nscalars,
 * norms_out 2 * rows doubles). */
roeam_status roeam_residual_norms3d(roeam_ctx *ctx, const roeam_grid3d *grid, const double *r, double *norms_out);

/* ------------------------------------------------------------------------ */
/* Batched and served solves                                                */
/* ------------------------------------------------------------------------ */

/* One solve: a grid, its parameters, an initial state and a run length.
 * q0: HOST or DEVICE pointer (q0_on_device) in the grid's state layout, read
 * at admission; q_out: HOST or DEVICE pointer (q_out_on_device) written when
 * the solve completes.  Both caller-owned; they must stay valid until the
 * ticket reports done. */
typedef struct {
    const roeam_grid *grid;
    roeam_params params;
    const double *q0;
    int q0_on_device;
    long nsteps;
    double t_end;
    double *q_out;
    int q_out_on_device;
} roeam_solve_desc;

/* Reserve `arena_bytes` of device memory for resident batch state (three
 * state copies per solve plus per-solve slots); must be called before the
 * first submit.  ENOMEM if the allocation fails. */
roeam_status roeam_batch_reserve(roeam_ctx *ctx, size_t arena_bytes);
/* The same over caller-owned DEVICE memory (for example a torch tensor's
 * storage) of arena_bytes at `arena`, 256-byte aligned: the engine places the
 * resident solves' state there and never frees it.  The memory must stay
 * valid, and must not be used otherwise, until the context is destroyed or
 * another reserve/attach replaces the engine.  EINVAL: NULL or unaligned
 * arena, too small; EBUSY: the current engine has work. */
roeam_status roeam_batch_attach(roeam_ctx *ctx, void *arena, size_t arena_bytes);
/* Bytes of arena a solve on this grid occupies while resident. */
size_t roeam_batch_footprint(const roeam_grid *grid);
/* Queue n solves; tickets_out[n] receives their tickets.  A descriptor's grid
 * may belong to any context on this context's device (the engine reads it,
 * and it must outlive the solve).  Solves are
 * admitted when arena memory is free and then advance together, one step of
 * every resident solve per scheduler iteration, with solves that arrive
 * later joining at the next iteration (continuous batching).
 * EINVAL: bad descriptor (validated before anything is queued). */
roeam_status roeam_batch_submit(roeam_ctx *ctx, int n, const roeam_solve_desc *descs,
                                uint64_t *tickets_out);
/* Drive the scheduler for `iterations` iterations, rounded up to whole
 * graphs of graph_iters (0: only admit and retire; -1: until every queued
 * solve is done, its state copied out: polls then report it done).  Every iteration advances each resident solve by one step;
 * a solve whose budget or end time is reached idles until the status read
 * after its graph retires it.  Returns the number of solves still pending in
 * *pending (nullable). */
roeam_status roeam_batch_run(roeam_ctx *ctx, long iterations, int *pending);
/* Profiling aid (same arithmetic as roeam_batch_run): drive the scheduler
 * with every kernel launched directly (no graphs), HIP events recorded on
 * the context stream around each batched stage kernel, and the status read
 * after every second iteration (a host wait each time), so that finished
 * solves leave at once and few timed launches are idle ones.  Waits for the stream, then writes the mean duration in
 * milliseconds of the batched stage kernels into stage_ms[0..3] (first to
 * fourth stage of a step; a stage that never ran reads 0) and the number of
 * timed launches into *launches (nullable).  Errors as roeam_batch_run. */
roeam_status roeam_batch_profile_run(roeam_ctx *ctx, long iterations, int *pending, double stage_ms[4],
                                     long *launches);
/* Scheduler options.  graph_iters: iterations per captured graph (even,
 * 2..256; default 16): a finished solve is noticed after the graph it
 * finished in.  persistent: 1 runs the batched stage kernels as resident
 * workgroups that take the tiles of a work list in turn, 0 (default) one
 * workgroup per tile.  policy: order in which queued solves are admitted when
 * arena space frees up, ROEAM_ADMIT_FIFO (default) or ROEAM_ADMIT_SHORTEST
 * (increasing cells x steps).  autotune: 1 (default) times the batched
 * kernel on a group's real work list for every tile shape when the group
 * first forms and keeps the fastest; 0 takes 16x7/256 below about 200k cells
 * and 16x15/256 above (a shape forced on the group's first grid wins either
 * way).  max_resident: at most this many solves resident at once (0: as many
 * as the arena holds; 1 runs the queue one solve at a time).  Applies from
 * the next scheduler iteration.  EINVAL: out of range or no engine. */
enum { ROEAM_ADMIT_FIFO = 0, ROEAM_ADMIT_SHORTEST = 1 };
roeam_status roeam_batch_configure(roeam_ctx *ctx, int graph_iters, int persistent, int policy, int autotune,
                                   int max_resident);
/* Counters of the batch engine: graph captures so far (one when the first
 * group forms, then only when a group appears or empties or a work list's
 * capacity changes: admitting and retiring solves that fit does not
 * re-capture), graph launches, scheduler iterations, tile-shape tunings, the
 * resident and queued solves, the options, and the tile shape of the group
 * formed last (-1: none yet). */
typedef struct {
    long captures, graph_launches, iterations, tunes;
    int resident, queued, graph_iters, persistent, policy, shape, max_resident;
} roeam_batch_stats;
roeam_status roeam_batch_info(roeam_ctx *ctx, roeam_batch_stats *out);
/* Non-blocking poll: *done = 1 once the solve's output is written; stats
 * (nullable) then holds its statistics.  A solve that produced a
 * non-physical state is done with return value ROEAM_ENONPHYS; the other
 * solves are not affected.  The poll that reports a ticket done also
 * forgets it; later polls of it return ENOTFOUND (unknown ticket). */
roeam_status roeam_batch_poll(roeam_ctx *ctx, uint64_t ticket, int *done, roeam_step_stats *stats);

#ifdef __cplusplus
}
#endif
#endif /* ROEAM_H */
