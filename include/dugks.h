/*
 * dugks.h -- C ABI of the MI355X (gfx950) DUGKS library: one D2Q9 discrete
 * unified gas-kinetic scheme time step for the conservative Allen-Cahn
 * equation (Yang, Zhong & Zhuo, arXiv 2007.07760, Sec. II).
 *
 * The problem statement follows the paper: a periodic grid of unit cells
 * (Sec. III), a prescribed velocity field (Sec. III, Eqs. 43-45), the mobility
 * M_phi and interface width W of Eqs. (1)-(4), the CFL number C of Eq. (39)
 * (dt = C since dx = sqrt(3RT) = 1) and the face reconstruction (central,
 * Eq. 25, or upwind, Eq. 26).
 *
 * Conventions
 *  - Every call returns a dugks_status; nothing is thrown and nothing aborts.
 *    dugks_strerror() gives a static text for each code.
 *  - The library owns the plan (host memory, and a small pinned host copy of
 *    the state's constant head made by the first dugks_init).  Device memory
 *    for states is owned by the caller: it allocates dugks_state_bytes() bytes
 *    (256-byte aligned) and passes the pointer.  Batches (below) own a small
 *    device allocation of their own for slot descriptors and the work list.
 *  - Streams are the caller's (hipStream_t passed as void*; NULL = default
 *    stream).  Calls that launch work are asynchronous on that stream; device
 *    faults surface at the caller's next synchronisation.
 *  - The step counter is the caller's: step n of the state is passed to each
 *    call that depends on it (which of the two ping-pong buffers is current,
 *    the time t_n = n dt of the velocity field, and the zero d(phi u)/dt of the
 *    first step).
 *  - Layout in the state: a 256-byte header, the face-stencil and velocity
 *    tables, two ping-pong buffers and mass scratch (T3S3 states: also a
 *    second stencil table and two stage buffers, f~ at t + dt/3 and Q of
 *    Eq. 32).  A buffer holds the grid
 *    in strips of 58 columns (the columns one 64-lane wavefront owns); row y
 *    of a strip is one chunk of 10 planes of 58 elements -- f~_0..f~_8 and the
 *    phi of the previous step -- padded to whole 128-byte lines.  Callers read
 *    the state only through dugks_phi / dugks_distributions / dugks_mass.
 *  - Plans are immutable after creation and may be shared between threads;
 *    calls on distinct states may run concurrently on distinct streams.
 *    Calls on one state must be ordered by the caller.
 *  - Blow-up (Eq. 39's scheme is only conditionally stable): every state
 *    carries a sticky status word, DUGKS_OK until a total mass computed for
 *    it is non-finite -- its phi0 at dugks_init, a dugks_mass call, or the
 *    per-step sum of plans with DUGKS_FLAG_MASS_FIX -- and DUGKS_ENUMERIC from
 *    then on.  Launches are asynchronous, so the status is read back with
 *    dugks_state_status (dugks_batch_status for the slots of a batch).
 *  - Reading of Eq. (2) where grad(phi) vanishes: n = g / max(|g|, 1e-12), g
 *    the isotropic gradient.
 */
#ifndef DUGKS_H
#define DUGKS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  DUGKS_OK = 0,
  DUGKS_EINVAL = 1,       /* invalid argument (sizes, ranges, NULL, alignment) */
  DUGKS_ENOMEM = 2,       /* host allocation failed                            */
  DUGKS_EDEVICE = 3,      /* a HIP launch or runtime call failed               */
  DUGKS_ENUMERIC = 4,     /* non-finite total mass                             */
  DUGKS_EUNSUPPORTED = 5  /* valid request the library does not provide        */
} dugks_status;

typedef enum { DUGKS_F64 = 0, DUGKS_F32 = 1 } dugks_precision;

/* Face reconstruction of fbar(x_b, t+h) = fbar+(x_b - xi h, t), Eq. (24):
 *  CENTRAL2  Eq. (25): value and gradient at the face from the neighbouring
 *            cells (mean of the two cells; normal difference; tangential
 *            mean of central differences).                       (T2S2CD)
 *  UPWIND3   Eq. (26): second-order Taylor expansion, with the factor 1/2,
 *            about the upstream cell centre, isotropic D2Q9-weighted gradient
 *            and Hessian; mean of the two sides when xi_i is parallel to the
 *            face.                                                (T2S3)
 *  CENTRAL4  Eq. (25) with fourth-order central estimates of the face value
 *            and of both gradient components.
 *  UPWIND5   the fifth-order, non-isotropic reconstruction of DUGKS-T2S5
 *            (Sec. III names it, gives no stencil): fbar+ at the foot
 *            x_b - xi_i h by a tensor product of one-dimensional Lagrange
 *            interpolations through the cell centres -- along the face
 *            normal the five cells centred on the upstream cell (the six
 *            centred on the face when xi_i is parallel to it), along the
 *            tangent the five cells centred on the face's row (one when
 *            xi_i is normal to the face).  T2 plans of the analytic velocity
 *            kinds only (T3S3 or ARRAYS: DUGKS_EUNSUPPORTED); single grids
 *            (batches refuse it). */
typedef enum {
  DUGKS_CENTRAL2 = 0,
  DUGKS_UPWIND3 = 1,
  DUGKS_CENTRAL4 = 2,
  DUGKS_UPWIND5 = 3
} dugks_recon;

/* Prescribed velocity u(x, y, t); cell centres at (i + 1/2, j + 1/2):
 *  UNIFORM        u = p0, v = p1
 *  ROTATION       u = -p0 (y - p2), v = p0 (x - p1)           (Eq. 43 form)
 *  SINGLE_VORTEX  u = -p0 sin^2(pi X) sin(2 pi Y) cos(pi t / p1)
 *                 v =  p0 sin(2 pi X) sin^2(pi Y) cos(pi t / p1),
 *                 X = x / nx, Y = y / ny
 *  DEFORMATION    u = -p0 sin(4 pi x/nx) sin(4 pi y/ny) cos(pi t / p1)
 *                 v = -p0 cos(4 pi x/nx) cos(4 pi y/ny) cos(pi t / p1)  (Eq. 45)
 *  ARRAYS         a steady field given at the cell centres by the caller
 *                 (the general prescribed field of Sec. III): u and v arrays
 *                 passed to dugks_init; the velocity of a face is the mean
 *                 of its two cells'.  vel_param is unused.  Single grids only
 *                 (batches refuse such plans: DUGKS_EUNSUPPORTED). */
typedef enum {
  DUGKS_VEL_UNIFORM = 0,
  DUGKS_VEL_ROTATION = 1,
  DUGKS_VEL_SINGLE_VORTEX = 2,
  DUGKS_VEL_DEFORMATION = 3,
  DUGKS_VEL_ARRAYS = 4
} dugks_vel_kind;

/* Time discretisation:
 *  T2    the original two-level DUGKS (Sec. II.B.1): the state stores
 *        f~ = f - (dt/2)(Omega + S); one face reconstruction per step at
 *        t + dt/2.
 *  T3S3  the third-order DUGKS of Sec. II.B.2: the state stores
 *        f^ = f - (dt/4)(Omega + S); two reconstructions per step, at
 *        t + dt/6 from fbar+ at t (Eq. 31) and at t + 3dt/4 from fbar+ at
 *        t + dt/3 (Eq. 34), combined by Eq. 16.  Needs dt < 12 tau (the
 *        coefficient of f^ in Eq. 31 must stay positive); d(phi u)/dt at
 *        t + dt/3 is the difference quotient over [t, t + dt/3]. */
typedef enum { DUGKS_T2 = 0, DUGKS_T3S3 = 1 } dugks_scheme;

/* flags */
#define DUGKS_FLAG_DTPHIU_ZERO 1u /* drop d(phi u)/dt from the source (test hook) */
/* Fused mass correction (meant for FP32 plans): every step also sums
 * phi^{n+1} in FP64 (per 8-row group of each strip, then a fixed-order
 * Neumaier reduction) and counts the cells whose new f~_0 is below 1e-3 (the
 * phase with phi near 0, where a small correction is not lost to rounding).
 * It records delta = (M0 - M^{n+1}) / count (or / (nx ny), and every cell,
 * when fewer than 1 % of the cells qualify); the next step adds w_i delta to
 * each f~_i of those cells as it loads it.  dugks_phi, dugks_distributions
 * and dugks_mass include the pending correction.  Segments of such plans are
 * whole 8-row groups (tile_rows is rounded up), so results stay independent
 * of the tiling.  T3S3 plans take it in the same way on their stored f^:
 * stage A applies the pending correction as it reads f^^n, stage B sums
 * f^^{n+1}. */
#define DUGKS_FLAG_MASS_FIX 2u

typedef struct {
  int32_t nx, ny;          /* cells per side, periodic; each in [8, 65536]         */
  double mobility;         /* M_phi > 0, finite; tau = M_phi / RT = 3 M_phi       */
  double width;            /* W > 0 cells; +INFINITY switches the theta term off  */
  double cfl;              /* C in (0, 1]; dt = C, h = dt / 2                     */
  int32_t recon;           /* dugks_recon                                        */
  int32_t precision;       /* dugks_precision of the stored f~ and phi            */
  int32_t vel_kind;        /* dugks_vel_kind                                     */
  int32_t flags;           /* DUGKS_FLAG_*                                       */
  double vel_param[6];     /* p0.. of the velocity kind; finite                  */
  int32_t tile_rows;       /* rows one wavefront marches; 0 = library default    */
  int32_t scheme;          /* dugks_scheme                                       */
} dugks_params;

typedef struct dugks_plan dugks_plan;

/* Validate p and build an immutable plan (stencil coefficients of the chosen
 * reconstruction, collision coefficients, launch geometry).  Host-only: no HIP
 * call is made.  Errors: EINVAL (p or out NULL, a field out of range, T3S3
 * with dt >= 12 tau), ENOMEM. */
int dugks_plan_create(const dugks_params *p, dugks_plan **out);
void dugks_plan_destroy(dugks_plan *plan);

/* Bytes of device memory one state needs (caller allocates, 256-B aligned);
 * ARRAYS plans include a copy of the two velocity planes. */
size_t dugks_state_bytes(const dugks_plan *plan);

/* Write the first state (step 0) from phi0 (device, FP64, [ny][nx] dense):
 * f~^0 = feq(phi0, u(x, 0)) - (dt/2) S^0 with d(phi u)/dt = 0 (T2; T3S3
 * stores f^0 = feq - (dt/4) S^0), i.e. f = feq at t = 0, and the
 * coefficient and velocity tables of the plan, and record M0 = sum phi0 (FP64;
 * a non-finite M0 sets the status to DUGKS_ENUMERIC).
 * uv_dev: ARRAYS plans only (ignored otherwise, may be NULL): the cell
 * velocities, device, FP64, [2][ny][nx] dense (u plane, then v plane); they
 * are copied into the state (in the plan's precision) on `stream`, so the
 * caller may release them once that copy has run.
 * Asynchronous on `stream`.  The first call on a plan stages the tables in
 * pinned host memory the plan keeps until dugks_plan_destroy, which must not
 * run before the copy has executed.  Errors: EINVAL (NULL, misaligned state,
 * uv_dev NULL for an ARRAYS plan), EDEVICE. */
int dugks_init(const dugks_plan *plan, void *state, const double *phi0_dev,
               const double *uv_dev, void *stream);

/* Advance the state from step `step` by `nsteps` steps of the plan's scheme:
 * T2 (Eqs. 21-28 with the Eq. 15 update form) is one fused
 * face-reconstruction + flux + update kernel per step; T3S3 two such kernels
 * (stages at t + dt/6 and t + 3 dt/4).  Asynchronous on `stream`.  Errors:
 * EINVAL (NULL, step < 0, nsteps < 0), EDEVICE. */
int dugks_step(const dugks_plan *plan, void *state, int64_t step,
               int64_t nsteps, void *stream);

/* Autotuner of the tile height (rows one wavefront marches; results do not
 * depend on it).  For the library default and every height 16..256 (steps of
 * 8, at most ny), times `reps` launches of the step's kernels on `state` at
 * `step` (the state of the plan built from `params`, any tile_rows) -- after
 * 20 warm-up launches, twice per height, the better kept -- and writes the
 * fastest height to rows_out; the caller builds its plan with it.
 * The timed launches read the state at `step` and write only what the step
 * itself overwrites before it reads it (the next-step buffer, T3S3's stage
 * buffers, the mass partials); the fused correction's reduction does not run,
 * so the state at `step` and its header are unchanged.  Blocks until done.
 * Errors: EINVAL (NULL, misaligned state, step < 0, reps outside 1..1000,
 * params invalid), EUNSUPPORTED, EDEVICE. */
int dugks_tune(const dugks_params *params, void *state, int64_t step, int32_t reps,
               int32_t *rows_out, void *stream);

/* phi = sum_i of the stored distributions (Eq. 30; Eq. 30a for T3S3) of the
 * state at `step`, written to phi_out_dev as [ny][nx] dense elements of the
 * plan's precision.  Asynchronous. */
int dugks_phi(const dugks_plan *plan, const void *state, int64_t step,
              void *phi_out_dev, void *stream);

/* The 9 stored distributions (f~_i for T2, f^_i for T3S3) of the state at
 * `step`, written to out_dev as
 * [9][ny][nx] dense elements of the plan's precision (velocity-major, paper
 * order of Sec. II.B.2).  Asynchronous.  Errors: EINVAL, EDEVICE. */
int dugks_distributions(const dugks_plan *plan, const void *state, int64_t step,
                        void *out_dev, void *stream);

/* The phi history plane of the state at `step` -- phi^{n-1} = sum_i of the
 * stored distributions one step earlier, the earlier phi of d(phi u)/dt in
 * Eq. (14b) -- as stored, [ny][nx] dense elements of the plan's precision.
 * With dugks_distributions it gives the complete input of the next step.
 * Asynchronous.  Errors: EINVAL, EDEVICE. */
int dugks_history(const dugks_plan *plan, const void *state, int64_t step,
                  void *out_dev, void *stream);

/* The state's sticky status word (DUGKS_OK, or DUGKS_ENUMERIC once a total
 * mass computed for it was non-finite), copied to *status_out (device or
 * pinned host memory), asynchronously on `stream`.  Errors: EINVAL, EDEVICE. */
int dugks_state_status(const dugks_plan *plan, const void *state, int32_t *status_out,
                       void *stream);

/* Total mass sum(phi) of the state at `step`, FP64, Neumaier-compensated, with
 * a fixed reduction order (deterministic), written to *mass_out_dev (device).
 * Uses the state's scratch.  Asynchronous; a non-finite total (the state has
 * blown up) also sets the state's status to DUGKS_ENUMERIC (dugks_state_status).
 * Errors: EINVAL, EDEVICE. */
int dugks_mass(const dugks_plan *plan, void *state, int64_t step,
               double *mass_out_dev, void *stream);

/* FP32 plans: measure the mass of the state at `step` as dugks_mass does and
 * add w_i * (M0 - M) / (nx ny) to every f~_i, M0 being the mass of phi0 in
 * FP64 recorded by dugks_init.  The correction's own rounding is measured and
 * corrected once more.  FP64 plans and plans with DUGKS_FLAG_MASS_FIX (which
 * correct every step): no-op.  Asynchronous. */
int dugks_mass_correct(const dugks_plan *plan, void *state, int64_t step,
                       void *stream);

/* Initial mass M0 (FP64) recorded by dugks_init, copied to *out_dev. */
int dugks_mass0(const dugks_plan *plan, const void *state, double *out_dev,
                void *stream);

/* ------------------------------------------------------------------ batches
 * Many independent grids advanced together, as the serving and batched forms
 * need them: a batch has `capacity` slots, each holding a (plan, state) pair
 * of the batch's precision and reconstruction, the step the state is at and
 * the step to stop at.  One persistent kernel takes the tiles of every active
 * grid from a work list in device memory, cut into one queue per XCD (whole
 * small grids or bands of a large one, taller tiles first) -- for
 * DUGKS_BATCH_T3S3 batches one such kernel per stage; a last, tiny kernel then
 * advances each active slot's step counter (and applies the fused mass
 * correction of DUGKS_FLAG_MASS_FIX batches).  Results are bitwise those of
 * dugks_step on the same plan and state.
 *  - The batch allocates a small amount of device memory of its own (slot
 *    descriptors, step counters, work list) on the device current at
 *    dugks_batch_create; every later call expects that device to be current.
 *  - set / clear change the host copy; dugks_batch_commit uploads it
 *    (asynchronously, ordered on `stream`) and must come before the next
 *    dugks_batch_step.  States must stay allocated while a slot holds them.
 *  - The step counters are the batch's while a state is attached: read them
 *    with dugks_batch_steps.
 *  - A slot whose state reports DUGKS_ENUMERIC at the end of a batch step
 *    (non-finite phi0, or a non-finite total in the fused correction of
 *    DUGKS_FLAG_MASS_FIX batches) stops: its target becomes the step it has
 *    reached, and dugks_batch_status reports it; other slots go on.
 *  - A batch is not thread-safe; calls on one batch must be serialised. */
typedef struct dugks_batch dugks_batch;

/* Batch flag: the batch advances DUGKS-T3S3 plans (two stage kernels per
 * batch step); without it, T2 plans. */
#define DUGKS_BATCH_T3S3 4u

/* Create a batch of `capacity` slots (1..65536), all empty.  flags: 0,
 * DUGKS_FLAG_MASS_FIX (then every attached plan must carry it, else none may)
 * or DUGKS_BATCH_T3S3 (then every attached plan is a T3S3 plan).  Errors:
 * EINVAL, ENOMEM, EDEVICE. */
int dugks_batch_create(int32_t capacity, int32_t precision, int32_t recon,
                       uint32_t flags, dugks_batch **out);
/* Wait for the device, then free the batch and its device memory. */
void dugks_batch_destroy(dugks_batch *batch);

/* Attach `state` (initialised by dugks_init for `plan`, currently at `step`)
 * to `slot`; the grid advances until its counter reaches `target` (>= step).
 * Replaces whatever the slot held.  Errors: EINVAL (range, NULL, misaligned
 * state, plan of another precision / reconstruction / mass-fix flag / time
 * scheme than the batch's), EUNSUPPORTED (an ARRAYS plan). */
int dugks_batch_set(dugks_batch *batch, int32_t slot, const dugks_plan *plan,
                    void *state, int64_t step, int64_t target);
/* Empty `slot`.  Errors: EINVAL. */
int dugks_batch_clear(dugks_batch *batch, int32_t slot);
/* Upload slot descriptors, changed step counters and the work list.
 * Asynchronous on `stream` (pinned staging; may wait for an older upload).
 * Errors: EINVAL, EDEVICE. */
int dugks_batch_commit(dugks_batch *batch, void *stream);
/* Run `nsteps` batch steps on `stream`: each active slot advances by one step
 * per batch step until it reaches its target.  With graph_steps > 1, whole
 * groups of graph_steps steps replay one captured hipGraph (captured on first
 * use for that group size); the rest are launched directly.  Asynchronous.
 * Errors: EINVAL (nsteps < 0, graph_steps outside 0..4096), EDEVICE. */
int dugks_batch_step(dugks_batch *batch, int64_t nsteps, int32_t graph_steps,
                     void *stream);
/* Copy the per-slot (step, target) pairs, int64[2 * capacity], to `out`
 * (host or device memory; asynchronous on `stream` when `out` is pinned or on
 * the device).  Errors: EINVAL, EDEVICE. */
int dugks_batch_steps(const dugks_batch *batch, int64_t *out, void *stream);
/* The status of each slot's state at its last batch step, int32[capacity]
 * (DUGKS_OK or DUGKS_ENUMERIC; DUGKS_OK for a slot not stepped since it was
 * set or cleared), copied to `out` (host or device memory; asynchronous on
 * `stream` when `out` is pinned or on the device).  Errors: EINVAL, EDEVICE. */
int dugks_batch_status(const dugks_batch *batch, int32_t *out, void *stream);

/* Rows per tile of every grid (a multiple of 8; grids shorter than that are
 * one tile high).  Default 64.  set: EINVAL unless 8 <= rows <= 65536 and
 * rows % 8 == 0; takes effect at the next commit. */
int dugks_batch_tile_rows(const dugks_batch *batch);
int dugks_batch_set_tile_rows(dugks_batch *batch, int32_t rows);
/* Autotuner: time the persistent step kernel over the attached, active grids
 * (`reps` launches per candidate tile height from 16 to 256 rows, HIP events
 * on `stream`), keep the fastest and commit it.  The timed launches write only
 * each grid's next-step buffer and mass partials, which the next real step
 * overwrites, so the states and results are unchanged.  Blocks until done.
 * Errors: EINVAL, EDEVICE. */
int dugks_batch_tune(dugks_batch *batch, int32_t reps, int32_t *rows_out,
                     void *stream);

/* ------------------------------------------------- allocation-free variant
 * For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.
 * dugks_step_many_noalloc is the batch step (dugks_batch_step) of many
 * independent grids without a batch: grid j (plans[j], states[j], initialised
 * by dugks_init, currently at step steps[j]) advances by nsteps steps, each
 * step one persistent launch of the batch step kernel over every grid's tiles
 * (two for T3S3; each grid whole in one of the per-XCD work queues) and the
 * finish kernel; results are bitwise those of
 * dugks_step and of a batch.  Nothing is allocated: descriptors, step
 * counters, slot status and the work list live in one fixed 1 MiB device
 * array of the library per GPU, filled by small set-up kernels whose inputs
 * travel as kernel arguments; no hipMalloc, hipFree, pinned staging or graph.
 *  - plans, states, steps: host arrays of n entries.  Every plan of one
 *    precision, reconstruction, DUGKS_FLAG_MASS_FIX setting and time scheme;
 *    each grid is tiled at its own plan's tile height.
 *  - Limits: 1 <= n <= 256 grids and at most 116192 tiles (strips x row
 *    segments) over all grids; beyond them DUGKS_EINVAL, before anything is
 *    launched.
 *  - Every call on one GPU shares that GPU's array, which keeps the last
 *    call's contents (each call rewrites what it reads first).  Calls that
 *    overlap on one GPU -- other streams, other threads -- race: the caller
 *    orders them.
 *  - The step counters stay the caller's: grid j ends at steps[j] + nsteps,
 *    unless its state turns non-finite (status DUGKS_ENUMERIC, see
 *    dugks_state_status), which stops it early.
 * Asynchronous on `stream`.  Errors: EINVAL (NULL arrays, a NULL or
 * misaligned state, mixed plans, the limits), EUNSUPPORTED (ARRAYS velocity or
 * the upwind-5 reconstruction, which the batch kernels do not provide),
 * EDEVICE. */
int dugks_step_many_noalloc(const dugks_plan *const *plans, void *const *states,
                            const int64_t *steps, int32_t n, int64_t nsteps, void *stream);

const char *dugks_strerror(int status);

/* Library version string. */
const char *dugks_version(void);

#ifdef __cplusplus
}
#endif
#endif
