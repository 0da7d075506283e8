/*
 * hlbm.h -- C ABI of the MI355X (gfx950) homogenized lattice Boltzmann sweep.
 *
 * The library advances a lattice BGK discretization of the homogenized BGK
 * Boltzmann equation (HBGKBE) of Simonis et al., "Homogenized lattice Boltzmann
 * methods for fluid flow through porous media -- part I" (Sec. 3.2,
 * eq:HBGKBE): the BGK collision relaxes toward the homogenized Maxwellian
 * M^eq = f^eq(n, varpi*u, T) whose velocity argument is scaled by the porosity
 * control varpi = 1 - nu*tau/K (eq:porousVeloMaxwellian, eq:d-definition).
 * Per cell the caller supplies d = 1 - varpi in [0, 1]: d = 0 is free fluid
 * (plain BGK, varpi = 1), d = 1 drives the equilibrium velocity to zero.  The
 * resulting per-step momentum loss (1/tau)(1 - varpi) rho u is the Darcy /
 * Brinkman drag of the target equations (Sec. 3.3 Step 1, eq:momentumHLBM).
 *
 * One step is a fused pull-stream + collide sweep over every cell:
 *   g*_i(x) = g_i(x - c_i)                        (pull streaming)
 *   rho = rho0 + sum g*_i, j = sum c_i g*_i, u = (j + F/2)/rho
 *   u_eq = (1 - d(x)) u                           (porosity shift)
 *   g_i <- g*_i - (g*_i - g^eq_i(rho, u_eq))/tau + S_i(u, F)   (BGK + Guo)
 * with shifted populations g_i = f_i - w_i rho0, the second-order Maxwellian
 * (c_s^2 = 1/3, from the covariance 1/(3 eps^2) I of Sec. 3.3 Step 2 at
 * eps = 1) and lattice viscosity nu = (tau - 1/2)/3.
 *
 * Conventions
 *   * Every call returns an int status: HLBM_OK (0) or a negative code; no
 *     call aborts or throws.  hlbm_last_error() returns a message for the
 *     last failure on the calling thread.
 *   * Lattice units (dx = dt = 1).  Cell index = x + nx*(y + ny*z).
 *   * Device pointers are HIP device addresses on the current device; host
 *     pointers belong to the caller and are only read or written during the
 *     call.
 *   * Work is enqueued on the stream named in the config (NULL = default
 *     stream).  hlbm_step only enqueues; hlbm_moments, hlbm_get_state and
 *     hlbm_sync wait for the stream, and an asynchronous device fault
 *     surfaces there as HLBM_EDEVICE.
 *   * A context is not thread-safe; distinct contexts may be used from
 *     distinct threads.
 */
#ifndef HLBM_H
#define HLBM_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

#define HLBM_ABI_VERSION 3

typedef struct hlbm_ctx hlbm_ctx;

/* Status codes. */
enum {
    HLBM_OK = 0,
    HLBM_EINVAL = -1,       /* invalid argument (NULL, range, NaN, tau <= 1/2, ...) */
    HLBM_ENOMEM = -2,       /* device or host allocation failed */
    HLBM_EDEVICE = -3,      /* HIP runtime or kernel error */
    HLBM_EUNSUPPORTED = -4, /* combination of options not provided */
    HLBM_ESTATE = -5,       /* call out of order (e.g. step before porosity) */
    HLBM_ENUMERIC = -6      /* non-finite value in a result */
};

/* Velocity sets (textbook lattices; c_s^2 = 1/3). */
enum { HLBM_D2Q9 = 9, HLBM_D3Q19 = 19 };

/* Population storage in HBM.  All forms store shifted populations
 * g = f - w*rho0.  F64: f64 storage and arithmetic.  F32: f32 storage and
 * arithmetic.  F16S / BF16S: 16-bit storage of s*g (s = store_scale, a power of
 * two) with f32 arithmetic, round to nearest even on store. */
enum { HLBM_F64 = 0, HLBM_F32 = 1, HLBM_F16S = 2, HLBM_BF16S = 3 };

/* Buffer pattern.  HLBM_AB: two population buffers swapped every step.
 * HLBM_AA: one buffer updated in place (the AA pattern), half the population
 * memory.  Its steps alternate between two forms: one reads the cell's own
 * slots and writes post-collision population i to the cell's slot opp(i); the
 * other reads population i from slot opp(i) of x - c_i and writes
 * post-collision population i to slot i of x + c_i.  With wall faces the
 * second form reads a population whose source is solid from the cell's own
 * slot i and writes one whose target is solid to its own slot opp(i)
 * (halfway bounce-back).  Every slot is read and written by one cell per step,
 * and each cell does the arithmetic of the AB sweep, so both patterns give the
 * same results bit for bit.  hlbm_get_state / hlbm_set_state use the AB
 * layout for both.  HLBM_AA takes periodic and wall faces only: an open face
 * needs the cell's own post-collision state, whose slots its neighbours write
 * in the same step (EUNSUPPORTED).  It takes block_x <= 256 (EUNSUPPORTED
 * otherwise). */
enum { HLBM_AB = 0, HLBM_AA = 1 };

/* Face kinds, per axis and side.  HLBM_PERIODIC must be used on both sides of
 * an axis or on neither.  HLBM_WALL makes the first (lo) or last (hi) layer of
 * cells solid, with halfway bounce-back at the fluid-solid link (no-slip,
 * u = 0 on the boundary, Sec. 2.4 eq:targetEBTL). */
enum { HLBM_PERIODIC = 0, HLBM_WALL = 1, HLBM_INLET_U = 2, HLBM_OUTLET_RHO = 3 };

/* Element types of caller arrays. */
enum { HLBM_DT_F64 = 0, HLBM_DT_F32 = 1, HLBM_DT_F16 = 2 };

/* Porosity control kinds.  HLBM_POROSITY_SCALAR: one value d = 1 - varpi per
 * cell, u_eq = (1 - d) u (isotropic permeability, Sec. 3.2).
 * HLBM_POROSITY_TENSOR (D3Q19): a symmetric 3x3 matrix D = nu tau K^{-1} per
 * cell for a tensor permeability K, u_eq = (I - D) u -- the anisotropic
 * extension the paper leaves to future work; D = d I is the scalar case. */
enum { HLBM_POROSITY_SCALAR = 0, HLBM_POROSITY_TENSOR = 1 };

typedef struct {
    int lattice;         /* HLBM_D2Q9 or HLBM_D3Q19 */
    int storage;         /* HLBM_F64, HLBM_F32, HLBM_F16S, HLBM_BF16S */
    int pattern;         /* HLBM_AB or HLBM_AA */
    int nx, ny, nz;      /* cells per axis; nz = 1 for D2Q9; nx*ny*nz < 2^32 */
    double tau;          /* BGK relaxation time, > 1/2; nu = (tau - 1/2)/3 */
    double force[3];     /* body-force density F (lattice units) */
    int bc_lo[3];        /* face kind of the lo side of x, y, z */
    int bc_hi[3];        /* face kind of the hi side of x, y, z */
    double inlet_u[3];   /* velocity of HLBM_INLET_U faces */
    double outlet_rho;   /* density of HLBM_OUTLET_RHO faces */
    double rho0;         /* reference density of the shifted populations (1) */
    double store_scale;  /* power of two s for F16S/BF16S; ignored otherwise */
    int external_memory; /* 1: caller binds population/porosity memory */
    int block_x;         /* threads per block along x (multiple of 64, <= 1024; <= 256 for HLBM_AA;
                            for a batch, items[0].block_x is the tile, <= 512); 0 = auto */
    void *hip_stream;    /* hipStream_t for all work of this context, NULL = default */
    int porosity_kind;   /* HLBM_POROSITY_SCALAR (default) or HLBM_POROSITY_TENSOR */
    int row_pad_bytes;   /* bytes of padding after each population row: 0 (dense, default) or a
                            multiple of 256 up to 2^24; for a batch, items[0] pads the packed
                            rows and the other items must give 0 */
} hlbm_config;

/* Library ABI version (HLBM_ABI_VERSION). */
int hlbm_version(void);

/* Message for the last failing call on this thread ("" if none). */
const char *hlbm_last_error(void);

/* Fill *cfg with defaults: D3Q19, F32, AB, 32^3 periodic, tau = 0.6, F = 0,
 * rho0 = 1, store_scale = 1, library-owned memory, default stream. */
int hlbm_config_default(hlbm_config *cfg);

/* Velocity set of `lattice` in the library's population order: c[3*i + a]
 * (integer components) and w[i].  Arrays hold at least 3*Q and Q entries.
 * Used to map states between orderings; the populations in
 * hlbm_get_state/hlbm_set_state follow this order. */
int hlbm_lattice_info(int lattice, int *c, double *w);

/* Bytes of one population buffer and of the porosity field for *cfg (six
 * rows for a tensor control).  HLBM_AB uses two such buffers, HLBM_AA one.
 * A population buffer holds Q rows; each row stores the N = nx*ny*nz cells
 * followed by row_pad_bytes of padding.  The pad shifts the rows against
 * each other modulo every power of two, which changes how the 19 read and 19
 * write streams of a sweep fall on the HBM channels: where N * element size
 * is a large power of two (512^3 FP32: 512 MiB rows) an 8448-byte pad makes
 * the sweep about 6% faster, at 256^3 any pad makes it slower, so the value is
 * chosen per shape by measurement.  The six rows of a tensor control take the
 * same pitch (porosity_bytes = 6 * (N * element size + row_pad_bytes)); a
 * scalar control is one dense row.  State snapshots are dense whatever the
 * pad. */
int hlbm_required_bytes(const hlbm_config *cfg, size_t *pop_bytes, size_t *porosity_bytes);

/* Validate *cfg and create a context.  Unless cfg->external_memory is set the
 * library allocates the population buffers (two for HLBM_AB, one for HLBM_AA)
 * and the porosity field in device memory.  The state starts at rest (g = 0: rho = rho0, u = 0 before the
 * half-force shift), step counter 0.  EINVAL on a bad field, EUNSUPPORTED on an
 * unsupported combination, ENOMEM if allocation fails. */
int hlbm_create(const hlbm_config *cfg, hlbm_ctx **out);

/* Use caller-owned device memory (e.g. torch tensors) for the two population
 * buffers and the porosity field, each of hlbm_required_bytes() size and at
 * least 256-byte aligned.  The memory must outlive the context.  Resets the
 * state to rest and the step counter to 0; the porosity must be set again. */
int hlbm_bind_buffers(hlbm_ctx *ctx, void *pop_a, void *pop_b, void *porosity);
/* (HLBM_AA: one population buffer; pop_b must be NULL, else EINVAL.) */

/* Wait for outstanding work, free library-owned memory, destroy the context.
 * NULL is accepted.  Returns EDEVICE if outstanding work had failed (the
 * context is still destroyed). */
int hlbm_destroy(hlbm_ctx *ctx);

/* Set the porosity control d = 1 - varpi per cell (eq:d-definition; varpi > 1
 * is excluded by the paper, Sec. 3.2, and varpi < 0 lies outside the model),
 * N = nx*ny*nz values, x fastest, of type `dtype` (HLBM_DT_*), on the device
 * if on_device else on the host.  Values are rounded to nearest even into the
 * storage's porosity type (f64, f32, or f16 for the 16-bit forms).  Any NaN or
 * value outside [0, 1] -> EINVAL and the field is left unset.  Synchronous.
 * With HLBM_POROSITY_TENSOR, d holds 6 rows of N values, D[r*N + cell] for
 * r = xx, yy, zz, xy, xz, yz; D must have eigenvalues in [0, 1] (D and I - D
 * positive semidefinite, checked through their principal minors with a
 * rounding allowance of 1e-12), else EINVAL. */
int hlbm_set_porosity(hlbm_ctx *ctx, const void *d, int dtype, int on_device);

/* Enqueue `nsteps` >= 0 fused stream-collide sweeps.  ESTATE if the porosity
 * was never set.  Asynchronous. */
int hlbm_step(hlbm_ctx *ctx, int nsteps);

/* Number of completed (enqueued) steps. */
int hlbm_get_step(const hlbm_ctx *ctx, long long *step);

/* Moments at the current time level n: those of the post-streaming,
 * pre-collision populations (Sec. 3.1 moment definitions):
 *   drho[cell]   = rho - rho0 = sum_i g*_i
 *   u[a*N+cell]  = (sum_i c_ia g*_i + F_a/2) / rho,   a = 0, 1, 2
 * (u[2*N..] = 0 for D2Q9).  Solid cells report 0.  dtype HLBM_DT_F64 or
 * HLBM_DT_F32; on_device selects device or host arrays.  Either array may be
 * NULL.  If totals != NULL it receives FP64 sums over fluid cells:
 * totals[0] = sum (rho - rho0), totals[1..3] = sum rho*u_a (computed on the
 * device in FP64: wavefront reduction, per-block partials, one fixed-order
 * second pass).  Waits for the stream; EDEVICE on a device fault, ENUMERIC if
 * a total is not finite. */
int hlbm_moments(hlbm_ctx *ctx, void *drho, void *u, int dtype, int on_device, double *totals);

/* hlbm_moments for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same moments kernel and fixed-order FP64 reduction, with the block
 * partials in a static device array of the library instead of memory
 * allocated on first use, and nothing else allocated, copied or awaited.
 * drho, u: device arrays as for hlbm_moments with on_device = 1 (either may
 * be NULL); totals: a device array of 4 doubles (or NULL), written with the
 * same values hlbm_moments returns.  Only enqueues work on the context's
 * stream: results are there once the stream reaches this point (hlbm_sync or
 * a wait on the stream), and a non-finite total is not reported.  The static
 * array holds the partials of at most 2^19 blocks (16 MiB per GPU the library
 * runs on, held until the process ends): totals of a box with more blocks of
 * block_x cells -> EINVAL (512^3 cells at block_x 256 fit).  Every call on a
 * GPU shares that GPU's array, so calls whose work overlaps on one GPU (two
 * streams, two threads) race on it; serialize them.  ESTATE if buffers are
 * not bound, EUNSUPPORTED for a batch. */
int hlbm_moments_noalloc(hlbm_ctx *ctx, void *drho, void *u, int dtype, double *totals);

/* Size in bytes of a raw state snapshot: Q dense rows of N stored values
 * (smaller than a population buffer, whose rows are padded). */
int hlbm_state_bytes(const hlbm_ctx *ctx, size_t *bytes);

/* Copy the current post-collision populations (storage element type, library
 * population order, g[i*N + cell]) to `dst` (device if on_device) and the step
 * counter to *step (may be NULL).  A device dst must not overlap the buffer
 * that holds the current state, else EINVAL.  Waits for the stream. */
int hlbm_get_state(hlbm_ctx *ctx, void *dst, int on_device, long long *step);
/* (HLBM_AA: the state is converted to the AB layout by a copy kernel; a device
 * dst must not overlap the population buffer, else EINVAL; a host dst may take
 * a temporary device buffer of one population buffer's size.  hlbm_set_state
 * copies row i of the snapshot into row opp(i); a device src must not overlap
 * the population buffer either.) */

/* Replace the current state by a snapshot taken with hlbm_get_state and set
 * the step counter.  Resuming from a snapshot reproduces the original run
 * bit for bit.  A device src must not overlap the buffer that holds the
 * current state, else EINVAL.  Waits for the stream. */
int hlbm_set_state(hlbm_ctx *ctx, const void *src, int on_device, long long step);

/* Reset to rest (g = 0) and step 0; the porosity field is kept. */
int hlbm_reset(hlbm_ctx *ctx);

/* Wait for all work of the context; EDEVICE on a device fault (and, for a
 * batch, if a grid barrier of the persistent kernel timed out). */
int hlbm_sync(hlbm_ctx *ctx);

/* Resolved obstacles in a fully periodic box (the geometry of the periodic
 * unit-cell Stokes problem the homogenized control stands in for, Sec. 2.2):
 * mask[cell] != 0 marks a solid cell (N bytes, x fastest; device memory if
 * on_device, else host).  No-slip u = 0 on the obstacle surface (Sec. 2.4,
 * eq:targetEBTL) by halfway bounce-back at every fluid-solid link: a
 * population whose pull source is solid is the cell's own opposite one.
 * Solid cells hold zeros and report zero moments; the porosity control still
 * applies in fluid cells.  mask = NULL removes the obstacles.  The link mask
 * (4 bytes per cell) is built on the device.  EUNSUPPORTED unless every face
 * is periodic, for HLBM_AA or for a batch (hlbm_batch_set_solid_mask sets an
 * item's obstacles); ESTATE while an adjoint tape is set.
 * Synchronous. */
int hlbm_set_solid_mask(hlbm_ctx *ctx, const unsigned char *mask, int on_device);

/* Diagnostics taken inside the sweep.  With every > 0, each hlbm_step sweep
 * that starts from a time level n with n % every == 0 also reduces the moments
 * it forms (those of time level n, as hlbm_moments would report them) to FP64
 * totals over fluid cells -- sum (rho - rho0), sum rho u_x, sum rho u_y,
 * sum rho u_z -- by a wavefront reduction, per-block partials and a
 * fixed-order two-pass sum, and appends them to a device log of `capacity`
 * records; further records are dropped (and counted) until the log is read.
 * The totals equal those hlbm_moments returns at that time level, bit for
 * bit.  every = 0 switches this off and frees the log.  Waits for the stream. */
int hlbm_set_diagnostics(hlbm_ctx *ctx, int every, int capacity);

/* Move up to max_records records, oldest first, into out[5*k ...]:
 * (n, sum (rho - rho0), sum rho u_x, sum rho u_y, sum rho u_z), n stored as a
 * double.  *count receives the records written; *dropped (may be NULL) the
 * records lost since the last read (log full, or beyond max_records).  The log
 * is emptied.  ENUMERIC if a total is not finite (records are still written).
 * Waits for the stream. */
int hlbm_read_diagnostics(hlbm_ctx *ctx, double *out, int max_records, int *count,
                          long long *dropped);

/* ------------------------------------------------------------------------
 * Discrete adjoint (reverse mode) for gradients with respect to the porosity
 * control d (the optimization variable of the homogenized model: varpi is a
 * design field, Sec. 3.2).
 *
 * The gradient is that of the discrete scheme itself: one step is pull
 * streaming S followed by the cell-local collision C(., d), and an objective
 * J observes the moments (drho, u) of the current time level (definitions as
 * for hlbm_moments).  Given dJ/d(drho) and dJ/du at the current time level,
 * hlbm_adjoint_step applies the transposed Jacobians of the last `nsteps`
 * steps in reverse order, carrying adjoint populations (FP64 storage and
 * arithmetic for HLBM_F64, FP32 for the other forms; each step's contribution
 * to dJ_dd is added in FP64), and adds
 *   sum over those steps of (dJ/dx_t) . dC(y_t, d)/dd
 * to dJ_dd: the derivative of J with respect to d through those steps (the
 * state before them held fixed).  Explicit dependences of J on d are the
 * caller's to add.  With HLBM_POROSITY_TENSOR the control is the six rows
 * xx, yy, zz, xy, xz, yz of the symmetric D in u_eq = (I - D) u, and dJ_dd
 * holds one row of N derivatives per control row; an off-diagonal row is one
 * variable standing at (a, b) and (b, a), so its derivative counts both
 * places.  At D = d I the three diagonal rows sum to the scalar dJ/dd.
 *
 * A reverse step needs only the pre-collision moments (rho - rho0, j) of
 * every cell at its forward step: the collision is linearized at them.  The
 * forward sweep sums them in FP64; a moment record keeps them in the
 * adjoint's precision (FP64 for HLBM_F64, FP32 for the other forms: 4
 * values, R = 32 or 16 bytes, per cell and step).  They come from a tape: with a tape set, hlbm_step stores the state every `every`
 * steps (checkpoints); the reverse sweep recomputes each segment of `every`
 * steps from its checkpoint with a sweep that also writes those moments (a
 * moment record of the segment), and the reverse steps read the record.  The
 * replay of the segment below runs on a second stream of the library's own
 * (default priority) while the reverse steps of the current segment run on
 * the context's stream; events order the two, and hlbm_adjoint_step waits
 * for both before it returns.  The forward steps of the tape's top two
 * segments (the one that holds step max_steps and the one below it) write
 * those segments' records themselves, so that a reverse sweep replays only
 * the segments below them.  A call that replays into a kept record's set
 * overwrites it; a later call replays that segment too.  (HLBM_TAPE_MOMENTS
 * records the moments of every forward step instead.)  The tape
 * records from the state current when it is set and restarts at the current
 * state whenever the state or the porosity changes otherwise (hlbm_set_state,
 * hlbm_reset, hlbm_set_porosity, hlbm_bind_buffers).
 *
 * Single HLBM_AB contexts only (a batch or HLBM_AA returns EUNSUPPORTED).
 * ------------------------------------------------------------------------ */

/* Allocate a tape for up to `max_steps` forward steps with a checkpoint every
 * `every` >= 1 steps, and start recording at the current state.  Device memory:
 * (max_steps/every + 1) checkpoints and 4 replay states (two segments,
 * replayed alternately, whose sweeps alternate between two buffers), each one
 * population buffer, two moment records of `every` steps (every * R * N
 * bytes each, R as above), plus two adjoint buffers of Q rows of P values (P = N +
 * row_pad_bytes divided by the storage's element size, the population row
 * pitch; 8 bytes each for HLBM_F64, else 4).  every = 0
 * frees the tape.  EUNSUPPORTED if one adjoint population row (N values of
 * 8 bytes for HLBM_F64, else 4) would reach 4 GiB.  hlbm_step returns EINVAL
 * (and does nothing) if it would take the recorded steps past max_steps.
 * Called again with the tape's own every and max_steps (and kind), it keeps
 * the tape's memory and only restarts recording at the current state.
 * Waits for the stream. */
int hlbm_set_tape(hlbm_ctx *ctx, int every, int max_steps);

/* What the tape keeps for the reverse sweep.
 *   HLBM_TAPE_REPLAY  (default) checkpoints every `every` steps; the reverse
 *                     sweep replays each segment from its checkpoint into a
 *                     moment record of the segment, as described above.
 *   HLBM_TAPE_MOMENTS the same checkpoints, and every recorded forward step
 *                     also writes the moments of every cell to a record of
 *                     R bytes per cell and step (max_steps * R * N bytes of
 *                     device memory, no replay states or segment records).
 *                     The reverse sweep reads that record and replays
 *                     nothing; the gradients are the same bit for bit.  This
 *                     trades memory (at the 288 GB of one MI355X, plenty for
 *                     the sizes here) for the replay's forward sweeps.
 * Takes effect at once: a tape already set is rebuilt in the new kind and
 * restarts at the current state.  EINVAL for another kind. */
enum { HLBM_TAPE_REPLAY = 0, HLBM_TAPE_MOMENTS = 1 };
int hlbm_set_tape_kind(hlbm_ctx *ctx, int kind);

/* The tape's every and max_steps (0 when none), the steps recorded since its
 * origin, and its device bytes.  Any output may be NULL. */
int hlbm_tape_info(const hlbm_ctx *ctx, int *every, int *max_steps, long long *recorded,
                   size_t *device_bytes);

/* Reverse sweep over the last nsteps recorded steps (0 <= nsteps <= recorded).
 * dJ_drho[N] and dJ_du[3][N] (x fastest, u component-major as in
 * hlbm_moments; entries of solid cells are ignored) are FP64 cotangents of the
 * moments at the current time level; dJ_dd (FP64) is accumulated (+=): N
 * values for a scalar control, 6 rows of N for a tensor one.
 * All three arrays are device memory if on_device, else host memory.  The
 * current state and the step counter are unchanged.  ESTATE without a tape;
 * EINVAL for nsteps outside the recorded range or a NULL array.  Waits for
 * the stream. */
int hlbm_adjoint_step(hlbm_ctx *ctx, int nsteps, const double *dJ_drho, const double *dJ_du,
                      double *dJ_dd, int on_device);

/* ------------------------------------------------------------------------
 * Batched periodic boxes.
 *
 * Many independent fully periodic D3Q19 boxes -- for instance porous unit
 * cells of uneven sizes and porosities, each with its own tau and force --
 * held in one context and advanced together.  Every item evolves exactly as a
 * single context of the same configuration would (bit for bit); items do not
 * interact.  The cells of all items are packed one after another (x fastest
 * inside an item) and each population row spans all items.
 *
 * hlbm_step advances every item.  Modes:
 *   HLBM_BATCH_GRAPH      (default) one executable HIP graph per call that
 *                         holds one node of the per-step kernel per step, each
 *                         node depending on the one before: the whole call is
 *                         one graph launch;
 *   HLBM_BATCH_PERSISTENT one persistent kernel that runs all steps with a
 *                         grid-wide barrier between them, launched directly;
 *   HLBM_BATCH_PER_STEP   one kernel launch per step;
 *   HLBM_BATCH_GRAPH_PERSISTENT one executable HIP graph per call holding a
 *                         reset node and the persistent kernel.
 * A graph is built on the first call with a given step count and starting
 * buffer and reused by later calls with the same ones.
 * Schedule: the packed cells are cut into tiles of `tile` cells that never
 * straddle two items; a tile is one block of `tile` threads in every mode.
 * The persistent kernel keeps blocks_per_cu blocks resident on each CU (at
 * most what fits at once) and blocks draw `chunk` tiles at a time from a
 * device-wide counter.  The state does not depend on the schedule (bit for
 * bit); hlbm_batch_moments' totals sum per-tile partials, so their rounding
 * follows the tile size.
 * Its barrier waits with a bounded spin; if the bound is hit, every block
 * leaves and the next syncing call returns HLBM_EDEVICE.
 * Items may hold resolved obstacles (hlbm_batch_set_solid_mask), with the
 * rule of hlbm_set_solid_mask inside each item's periodic box.
 * hlbm_get_state / hlbm_set_state / hlbm_reset / hlbm_get_step work on the
 * packed state; hlbm_set_porosity, hlbm_moments and hlbm_set_solid_mask
 * return HLBM_EUNSUPPORTED for a batch (use the calls below).
 * ------------------------------------------------------------------------ */
enum { HLBM_BATCH_GRAPH = 0, HLBM_BATCH_PERSISTENT = 1, HLBM_BATCH_PER_STEP = 2, HLBM_BATCH_GRAPH_PERSISTENT = 3 };

/* Create a batch of n_items >= 1 boxes.  items[k] gives box k's nx, ny, nz
 * (each in [2, 1024], with nx*ny*nz*max(nx, ny) < 2^32), tau and force; all
 * items must use HLBM_D3Q19, the same storage, HLBM_AB and periodic faces on
 * every axis.  rho0, store_scale, block_x and hip_stream are taken from
 * items[0]; items[0].block_x is the tile (0 = 256 cells; else a multiple of 64
 * up to 512, EINVAL above).  external_memory must be 0 (the library allocates).  The packed
 * cell count times the element size must stay below 4 GiB.  State at rest.
 * EUNSUPPORTED if no block of `tile` threads of the batched kernel fits on a
 * CU.  The schedule starts at blocks_per_cu = max(1, 512 / tile) (capped at
 * what fits) and chunk = 2. */
int hlbm_create_batch(const hlbm_config *items, int n_items, hlbm_ctx **out);

/* Number of items and total packed cells of a batch (EINVAL if not a batch). */
int hlbm_batch_info(const hlbm_ctx *ctx, int *n_items, size_t *total_cells);

/* Select how hlbm_step advances a batch (HLBM_BATCH_*). */
int hlbm_batch_set_mode(hlbm_ctx *ctx, int mode);

/* Schedule of the persistent kernel: resident blocks per CU, in
 * [1, max_blocks_per_cu] (0 = the default), and tiles per draw, in [1, 64]
 * (0 = 2).  EINVAL outside those ranges.  Waits for the stream. */
int hlbm_batch_set_schedule(hlbm_ctx *ctx, int blocks_per_cu, int chunk);

/* Bound on the wait of the persistent kernel's grid barrier, in polls of
 * about 0.1 us each (default 2^20).  When a block's wait exceeds it, every
 * block leaves the kernel at its next barrier (the kernel always ends) and the
 * next syncing call (hlbm_sync, hlbm_batch_moments) returns HLBM_EDEVICE; the
 * state is then undefined until hlbm_reset or hlbm_set_state.  0 makes any
 * wait fail, which exercises that path.  EINVAL for polls < 0 or if not a
 * batch.  Waits for the stream. */
int hlbm_batch_set_barrier_limit(hlbm_ctx *ctx, int polls);

/* The batch's tile, resident blocks per CU, the most blocks that fit per CU,
 * and chunk.  Any output may be NULL.  EINVAL if not a batch. */
int hlbm_batch_get_schedule(const hlbm_ctx *ctx, int *tile, int *blocks_per_cu, int *max_blocks_per_cu,
                            int *chunk);

/* Porosity control d = 1 - varpi of one item (nx*ny*nz values, x fastest),
 * same rules as hlbm_set_porosity.  Every item must be set before stepping. */
int hlbm_batch_set_porosity(hlbm_ctx *ctx, int item, const void *d, int dtype, int on_device);

/* Resolved obstacles in item `item` (the periodic unit-cell Stokes problem
 * behind the permeability, Sec. 2.2, with no-slip on the obstacle, Sec. 2.4
 * eq:targetEBTL): mask[cell] != 0 marks a solid cell of that item
 * (nx*ny*nz bytes, x fastest; device memory if on_device, else host).  Within
 * the item's periodic box the rule is that of hlbm_set_solid_mask: halfway
 * bounce-back at every fluid-solid link, zeros in solid cells, which report
 * zero moments and add nothing to the totals; the porosity control still
 * applies in fluid cells.  mask = NULL removes the item's obstacles.  While
 * any item holds obstacles every item runs the masked kernels (4 more bytes
 * per cell: a link mask over all packed cells, allocated on first use); an
 * item without obstacles then evolves bit for bit as without them.  The
 * state is left as it is (a solid cell's populations become zeros at the next
 * step).  Synchronous. */
int hlbm_batch_set_solid_mask(hlbm_ctx *ctx, int item, const unsigned char *mask, int on_device);

/* Moments of a batch at the current time level (definitions as for
 * hlbm_moments), FP64.  If drho or u is not NULL they receive the fields of
 * `item` (drho[nx*ny*nz], u[3][nx*ny*nz]); on_device selects device or host
 * arrays.  If totals is not NULL it receives, for every item k,
 * totals[4k] = sum (rho - rho0), totals[4k+1..4k+3] = sum rho u_a, in FP64
 * (block partials per tile, then one fixed-order pass per item).  Waits for
 * the stream. */
int hlbm_batch_moments(hlbm_ctx *ctx, int item, double *drho, double *u, int on_device,
                       double *totals);

#ifdef __cplusplus
}
#endif

#endif /* HLBM_H */
