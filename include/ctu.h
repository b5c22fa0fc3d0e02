/*
 * ctu.h -- C ABI of the MI355X (gfx950) CTU library: one unsplit Corner Transport Upwind
 * timestep of the 3D Euler equations on a static Cartesian mesh (Schneider & Robertson,
 * "Cholla", arXiv:1410.4194): PPMC or PPMP reconstruction with half-step tracing (Sec. 2.2,
 * App. A.3, A.4), interface fluxes from the exact Riemann solver or the Roe solver with the
 * HLLE fallback and the optional H correction (Sec. 2.3, App. B.1, B.2, C), the CTU
 * transverse corrections and conservative update (Sec. 2.1), the CFL time step, and
 * periodic, outflow or reflecting boundaries (Sec. 3.1); one grid at a time or batches of
 * independent grids.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Return value: ctu_status; 0 is success, negative values are errors.  A short message for
 *   the last error of the calling thread is available from ctu_last_error().
 * Memory ownership: device memory belongs to the caller.  A grid uses two caller-allocated
 *   device buffers (state and workspace) whose sizes ctu_workspace_bytes() reports; the
 *   library allocates only small host-side handles.  Host arrays passed in are copied;
 *   host arrays passed out are filled.
 * Streams: every grid is bound to the HIP stream given at creation (NULL = the default
 *   stream).  Entry points marked "async" only enqueue work; entry points marked "syncs"
 *   wait for that stream.
 * State layout (Sec. 3.2, memory structure: one contiguous array per conserved field,
 *   fields one after another, ghost cells included): structure of arrays.  Field q in
 *   {0: rho, 1: rho*u, 2: rho*v, 3: rho*w, 4: E} (total energy per volume,
 *   E = p/(gamma-1) + rho V^2/2, Sec. 2) occupies a
 *   contiguous array of the allocated box (nx+2g)(ny+2g)(nz+2g), x fastest: real cell
 *   (i, j, k), 0 <= i < nx, is element (i+g) + NX*((j+g) + NY*(k+g)), NX = nx+2g,
 *   NY = ny+2g.  Consecutive fields start `field_stride` elements apart
 *   (ctu_grid_info).  g ghost layers per side: g = 3 with PPMC (its stencil needs two, the
 *   CTU transverse correction one more), g = 4 with PPMP (three-cell stencil), one more
 *   with the H correction.  Element type is double (CTU_FP64) or float (CTU_FP32).
 * Host arrays for set/get are the real cells only, packed, x fastest, one array per field.
 * Errors found on the device (non-finite or non-positive density / energy in an updated
 *   state) are reported at the next syncing call of that grid as CTU_ENONPHYS.
 */
#ifndef CTU_H
#define CTU_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  CTU_OK = 0,
  CTU_EINVAL = -1,    /* invalid argument or configuration; nothing was launched */
  CTU_ENOMEM = -2,    /* caller buffer too small */
  CTU_EDEVICE = -3,   /* HIP runtime error (message in ctu_last_error) */
  CTU_ENONPHYS = -4,  /* device found a non-physical state (see ctu_check flags) */
  CTU_ENOCONV = -5,   /* Newton iteration reached its cap (counted, see ctu_check) */
  CTU_EAGAIN = -6     /* batch has no free slot */
} ctu_status;

/* Boundary types, Sec. 3.1 (ghost cells and boundary conditions).
 * Periodic: a ghost copies the real cell one period away.
 * Outflow (transmissive): every ghost layer copies the edge real cell.
 * Reflect: a ghost copies its mirror-image real cell across the wall (ghost layer m outside
 * takes real layer m-1 inside) and negates the momentum normal to the wall; the axis needs
 * at least as many real cells as there are ghost layers (3 with PPMC, 4 with PPMP, one
 * more with the H correction) so that every mirror image is a real cell. */
typedef enum { CTU_BC_PERIODIC = 0, CTU_BC_OUTFLOW = 1, CTU_BC_REFLECT = 2 } ctu_bc;
typedef enum { CTU_FP64 = 0, CTU_FP32 = 1 } ctu_prec;

/* Riemann solvers, Sec. 2.3.  Exact: Newton iteration for the star pressure (App. B.1).
 * Roe: the linearized solver of App. B.2, which substitutes the HLLE flux where an
 * intermediate state would have a non-positive density or pressure (counted in
 * ctu_check counters[3]). */
typedef enum { CTU_RIEMANN_EXACT = 0, CTU_RIEMANN_ROE = 1 } ctu_riemann;

/* Interface reconstructions, Sec. 2.2.  PPMC: piecewise parabolic with characteristic
 * limiting and tracing (App. A.3), three ghost layers.  PPMP: piecewise parabolic in the
 * primitive variables with contact steepening, shock flattening and CW84 tracing
 * (App. A.4); its three-cell stencil needs four ghost layers. */
typedef enum { CTU_RECON_PPMC = 0, CTU_RECON_PPMP = 1 } ctu_recon;
typedef enum {
  CTU_SCHEDULE_AUTO = 0,
  CTU_SCHEDULE_IN_ORDER = 1,
  CTU_SCHEDULE_OVERLAP = 2,
  CTU_SCHEDULE_FUSED_Z = 3
} ctu_schedule;
/* CTU_SCHEDULE_AUTO overlaps the sweeps of grids of at most this many real cells and fuses
 * the z sweeps above (measured crossover on MI355X: between 256^3 and 288^3 in both
 * precisions) */
#define CTU_OVERLAP_MAX_CELLS ((int64_t)20 << 20)
/* with the H correction (no fused z) CTU_SCHEDULE_AUTO overlaps while each field array takes
 * at most this many bytes (elem_bytes x field_stride of ctu_grid_info), in order above */
#define CTU_OVERLAP_MAX_FIELD_BYTES ((size_t)192 << 20)

/* Device error-word bits reported by ctu_check. */
enum {
  CTU_FLAG_NONFINITE = 1u << 0, /* an updated conserved value is NaN or infinite */
  CTU_FLAG_DENSITY = 1u << 1,   /* an updated density is <= 0 */
  CTU_FLAG_PFLOOR = 1u << 2,    /* a pressure was raised to p_floor (count in counters[0]) */
  CTU_FLAG_NEWTON_CAP = 1u << 3 /* a Newton solve hit newton_max_iter (counters[1]) */
};

/* Grid configuration.  Sec. 2.1 (CTU), eq. calc_dt_3D (CFL), App. B.1 (Newton tolerance,
 * pressure floor of Sec. 2.3.1). */
typedef struct {
  int32_t nx, ny, nz;      /* real cells per axis, each >= 1 */
  double dx, dy, dz;       /* cell widths, > 0 */
  double gamma;            /* ratio of specific heats, > 1 */
  int32_t bc[6];           /* x-, x+, y-, y+, z-, z+ : ctu_bc; periodic must pair;
                              reflect needs as many cells on its axis as there are
                              ghost layers */
  int32_t prec;            /* ctu_prec.  CTU_FP32 stores state, reconstruction and fluxes
                              in float and keeps the Newton star-pressure solve in double */
  double cfl;              /* Courant number C0, 0 < cfl < 0.5 (six-solve CTU limit) */
  double newton_tol;       /* relative change that stops the Newton loop (1e-6) */
  int32_t newton_max_iter; /* Newton iteration cap (50) */
  double p_floor;          /* pressure floor on every primitive conversion (1e-20) */
  int32_t march_seg[2];    /* tile shape: target cells per thread of the y and z sweeps, which
                              march along their axis; 0 = the library default (32).  The
                              n cells of an axis are split into round(n/target) equal
                              segments.  Changes the launch shape; results change only by
                              rounding (last-bit differences in a segment's first trace). */
  int32_t riemann;         /* ctu_riemann; both stages use the same solver */
  int32_t recon;           /* ctu_recon */
  int32_t h_correction;    /* 1: H correction of the second-stage Roe fluxes (App. C): |lambda|
                              is floored at the largest eta = |(u+a)_R - (u+a)_L|/2 of the
                              face and of the transverse faces around its two cells, taken
                              from the second-stage states; needs CTU_RIEMANN_ROE and one
                              ghost layer more */
  int32_t x_rows;          /* tile shape: x-rows of real cells per wavefront of the x sweep
                              fused with the update, 1..8 (capped at ny); 0 = the library's
                              choice (the fewest idle lanes, one row unless more cut idle lanes
                              by 20%).  Changes the launch shape only: results are bitwise
                              the same */
  int32_t x_chunks;        /* tile shape: consecutive 58-cell chunks per wavefront of the
                              first-stage x sweep, 1..16; 0 = the library default (4).
                              Changes the launch shape only: results are bitwise the same */
  int32_t schedule;        /* ctu_schedule: the order of the passes of a step taken by
                              ctu_step / ctu_advance.  CTU_SCHEDULE_OVERLAP runs the
                              first-stage y sweep and then the second-stage z sweep (with
                              the H correction: the eta pass along z) on a stream of the
                              grid's own (created with the grid, default priority), beside
                              the other sweeps, ordered with events, and the PPMP
                              coefficient passes beside the first-stage sweeps; the
                              caller's stream still sees each step as one ordered unit.
                              CTU_SCHEDULE_FUSED_Z runs the first-stage y sweep on that
                              stream beside the x sweep and then both z stages in one march
                              (with the H correction: as OVERLAP).  CTU_SCHEDULE_IN_ORDER
                              runs every pass in order on the grid's stream.
                              CTU_SCHEDULE_AUTO (0) overlaps grids of at most
                              CTU_OVERLAP_MAX_CELLS real cells and fuses the z sweeps above;
                              with the H correction it overlaps while one field array takes
                              at most CTU_OVERLAP_MAX_FIELD_BYTES and runs in order above
                              (measured on MI355X: the overlap gains 3-4% at 256^3 and
                              10-25% on small grids, fused z 1.4-4% on 288^3-512^3 grids
                              where overlapped sweeps no longer fit the last-level cache).
                              In order and overlapped give bitwise the same results; fused z
                              agrees with them to rounding (a separately compiled copy of the
                              same formulas).  ctu_step_noalloc always runs in order; batches
                              overlap on a stream of their own. */
} ctu_config;

typedef struct ctu_grid ctu_grid;
typedef struct ctu_batch ctu_batch;

typedef struct {
  int64_t alloc_cells;   /* (nx+2g)(ny+2g)(nz+2g) */
  int64_t field_stride;  /* elements between consecutive fields of the state buffer */
  int32_t elem_bytes;    /* 8 (FP64) or 4 (FP32) */
  double t;              /* simulation time accumulated by step/advance (syncs) */
  int64_t steps;         /* steps taken (syncs) */
  int32_t ghost;         /* g, ghost layers per side */
  int32_t schedule;      /* the schedule steps use: CTU_SCHEDULE_IN_ORDER, _OVERLAP or
                            _FUSED_Z */
} ctu_grid_info;

/* Fill *cfg with the defaults: cfl 0.3, newton_tol 1e-6, newton_max_iter 50,
 * p_floor 1e-20, FP64, periodic, gamma 5/3, unit cells, 1x1x1. */
ctu_status ctu_config_default(ctu_config* cfg);

/* Bytes of the two device buffers a grid with this configuration needs.  Either output
 * pointer may be NULL.  No device work. */
ctu_status ctu_workspace_bytes(const ctu_config* cfg, size_t* state_bytes, size_t* work_bytes);

/* Create a grid over caller-owned device buffers d_state (>= state_bytes) and d_work
 * (>= work_bytes, 256-byte aligned), bound to hip_stream (hipStream_t, NULL = default).
 * This is the set-up half of Sec. 3.1 (simulation overview: the grid, its ghost cells and
 * boundary types, the header values of domain size and time), with the device memory of
 * Sec. 3.2 resident for the grid's lifetime instead of copied every step.
 * Validates cfg (CTU_EINVAL) and sizes (CTU_ENOMEM); launches nothing.  A grid of more
 * than 2^31 real cells, or one whose largest pass would exceed 2^32 - 1 work-items in one
 * dispatch, is refused with CTU_EINVAL (memory runs out first on one MI355X: 1024^3 takes
 * 153 GB in FP32 and 306 GB in FP64). */
ctu_status ctu_grid_create(const ctu_config* cfg, void* d_state, void* d_work, size_t work_bytes,
                           void* hip_stream, ctu_grid** out);
ctu_status ctu_grid_destroy(ctu_grid* g);
ctu_status ctu_grid_info_get(ctu_grid* g, ctu_grid_info* info); /* syncs */

/* Upload conserved real-cell values: h_fields[5] host arrays of nx*ny*nz elements of the
 * grid's element type, scattered into the field arrays of the layout above (Sec. 3.2; the
 * initial conditions of Sec. 3.1 are the caller's).  Resets t and the step count.  Syncs. */
ctu_status ctu_set_state(ctu_grid* g, const void* const h_fields[5]);

/* Upload primitive real-cell values (rho, u, v, w, p) as host double arrays and convert
 * them to conserved variables on the device with the ideal-gas EOS (Sec. 2).  Syncs. */
ctu_status ctu_set_primitive(ctu_grid* g, const double* const h_fields[5]);

/* Download conserved real-cell values into h_fields[5] (grid element type), gathered from
 * the field arrays of the layout above (Sec. 3.2).  Syncs;
 * returns CTU_ENONPHYS if the device error word is set (the data is still copied). */
ctu_status ctu_get_state(ctu_grid* g, void* const h_fields[5]);

/* CFL time step of the current state (eq. calc_dt_3D over the real cells:
 * cfl * min(dx/(|u|+a), dy/(|v|+a), dz/(|w|+a))).  Syncs. */
ctu_status ctu_compute_dt(ctu_grid* g, double* dt);

/* One CTU step with time step dt > 0 (Sec. 2.1, steps 1-5): ghost fill, reconstruction +
 * tracing and first Riemann solve per direction, transverse correction and second Riemann
 * solve per direction, conservative update (eq. conserved_update), and the reduction that
 * yields the next CFL time step (Sec. 3.5).  The kernel sequence follows Sec. 3.4 (one
 * kernel per stage and direction, intermediates in device memory), with reconstruction and
 * Riemann solve fused per direction and the last second-stage sweep fused with the update;
 * with the overlapped schedule (ctu_config.schedule) the kernels whose inputs allow it run on
 * the grid's second stream beside the others.  Async on the grid's stream, which sees the
 * whole step as one ordered unit. */
ctu_status ctu_step(ctu_grid* g, double dt);

/* nsteps CTU steps with the time step computed on the device from the state each step
 * starts with, the last one clipped so that t does not pass t_end (steps after t_end, and
 * steps after an update was flagged non-physical, are no-ops): the main loop of Sec. 3.1
 * (boundaries, CTU step, time update), with the time step of Sec. 3.5 kept on the device
 * so that no step waits for the host.  No host synchronization.  Async. */
ctu_status ctu_advance(ctu_grid* g, int32_t nsteps, double t_end);

/* Sums over the real cells of the five conserved fields, accumulated in double in a fixed
 * order (bitwise reproducible).  Syncs. */
ctu_status ctu_totals(ctu_grid* g, double out[5]);

/* Read and clear the device error word and counters: counters[0] pressure-floor hits,
 * [1] Newton solves that hit the cap, [2] non-physical updated cells, [3] Roe solves that
 * substituted the HLLE flux (informational; sets no flag).
 * Returns CTU_ENONPHYS if non-physical bits are set, CTU_ENOCONV if only the Newton cap
 * was hit, else CTU_OK.  Syncs. */
ctu_status ctu_check(ctu_grid* g, uint32_t* flags, uint64_t counters[4]);

/* Debug access to the fluxes of the last step as the step keeps them: per-cell differences
 * dF(c) = F(c - 1/2) - F(c + 1/2) along the flux's own axis (host double arrays over the
 * allocated box, x fastest), the only form that the transverse correction and the update
 * consume.  which = 0: first-stage F*, G*, H*; which = 1: CTU F^{n+1/2}, G^{n+1/2},
 * H^{n+1/2}; dir 0/1/2 = x/y/z; h_fields[5] arrays of alloc_cells doubles.  Only values on
 * the cells the step covers are meaningful.  The x CTU difference feeds the update in
 * registers and is stored only while ctu_debug_keep_fluxes(g, 1) is in effect (which = 1,
 * dir = 0 fails with CTU_EINVAL otherwise).  Both sync. */
ctu_status ctu_debug_keep_fluxes(ctu_grid* g, int32_t keep);
ctu_status ctu_debug_fluxes(ctu_grid* g, int32_t which, int32_t dir, double* const h_fields[5]);

/* ---- Measurement -------------------------------------------------------------------------
 * ctu_profile_enable(g, mode) starts a fresh accumulation (syncs); mode 0 stops and frees it.
 *   CTU_PROFILE_TIMING: every kernel a step launches is bracketed by HIP events recorded on
 *     the grid's stream, and elapsed times accumulate per kernel class.
 *   CTU_PROFILE_NEWTON: the sweeps run instrumented copies that count, for every exact
 *     Riemann solve (App. B.1), the Newton iterations it took, in 8 bins: 0 or 1 (equal
 *     face states have the constant state as their exact solution and take none), 2, 3, 4,
 *     5-8, 9-16, more than 16, and the cap (newton_max_iter reached).  The copies are
 *     slower; time with CTU_PROFILE_TIMING alone.
 * ctu_profile_read fills up to max_classes entries of ms[] (total milliseconds) and
 *   launches[] (launch counts) in the order of ctu_profile_name(i), and sets *count to the
 *   number of classes (syncs).  ctu_profile_name returns "" past the last class.
 * ctu_newton_histogram fills hist[8] with the bins accumulated since the histogram was
 *   enabled (syncs). */
enum { CTU_PROFILE_TIMING = 1, CTU_PROFILE_NEWTON = 2 };
ctu_status ctu_profile_enable(ctu_grid* g, int32_t mode);
ctu_status ctu_profile_read(ctu_grid* g, int32_t max_classes, double* ms, int64_t* launches,
                            int32_t* count);
const char* ctu_profile_name(int32_t k);
ctu_status ctu_newton_histogram(ctu_grid* g, uint64_t hist[8]);

/* Plain streaming kernels, not part of the method: what this GPU's HBM delivers to accesses
 * shaped like the sweeps' (one 8-byte element per lane, 64 consecutive elements per
 * wavefront, four independent loads per lane): the achievable ceiling beside the published
 * 8 TB/s peak when the cell-update rate of Sec. 3.7.3 is set against HBM bandwidth.  kind:
 *   CTU_STREAM_READ      c[b] = sum of block b's elements of a (every element read once;
 *                        c needs ctu_stream_probe_blocks(n) doubles);
 *   CTU_STREAM_COPY      c[i] = a[i];
 *   CTU_STREAM_ADD       c[i] = a[i] + b[i];
 *   CTU_STREAM_COMBINE5  c[i] = a[i] + a[n+i] + a[2n+i] + a[3n+i] + a[4n+i] (a holds 5n).
 * a, b, c: device arrays of doubles (b only for ADD); n >= 1 elements.  Async on hip_stream
 * (NULL = default).  CTU_EINVAL for an unknown kind, a missing array or n = 0;
 * CTU_EDEVICE if the launch fails. */
enum { CTU_STREAM_READ = 0, CTU_STREAM_COPY = 1, CTU_STREAM_ADD = 2, CTU_STREAM_COMBINE5 = 3 };
size_t ctu_stream_probe_blocks(size_t n);
ctu_status ctu_stream_probe(int32_t kind, const double* a, const double* b, double* c, size_t n,
                            void* hip_stream);

/* ---- Batches: many independent grids advanced together ----------------------------------
 * Continuous batching of independent grids (each created as above, any sizes, boundary
 * types and precisions).  Every pass of a step is one launch over all running grids of a
 * precision, each grid taking its own device-side time step as in ctu_advance, so small
 * grids share the GPU instead of running one after another.
 *
 * ctu_batch_workspace_bytes: device bytes a batch of max_slots slots needs (1..65536).
 * ctu_batch_create: a batch over a caller-owned device buffer d_work (>= those bytes,
 *   256-byte aligned), ordered after and before the work of hip_stream (NULL = default
 *   stream); batch work itself runs on a stream of the batch's own, of default priority,
 *   with the overlapped sweep schedule (CTU_SCHEDULE_OVERLAP) on a second stream of the
 *   batch's, whatever the grids' own schedule (many small grids gain from it at any total
 *   size).
 *   flags: CTU_BATCH_GRAPH captures one step of the current set of grids in a HIP graph and
 *   replays it (recaptured whenever the set changes; the overlap becomes parallel branches
 *   of the graph).  Creates two streams and six events.
 * ctu_batch_submit: places grid g in a free slot (CTU_EAGAIN when none is free) with a step
 *   budget nsteps >= 0 and an end time t_end; enqueues its CFL reduction on the grid's
 *   stream and orders the batch after it.  Until its ticket ends, every other call on g
 *   fails with CTU_EINVAL.  Async.
 * ctu_batch_run: enqueues `steps` steps of every running grid; grids that used their budget,
 *   reached t_end or were found non-physical take no-op steps.  Async.
 * ctu_batch_poll: state of a ticket (CTU_TICKET_RUNNING, DONE, FAILED = non-physical state,
 *   UNKNOWN = no such ticket) and its simulation time.  A DONE or FAILED ticket releases its
 *   slot and its grid, whose state can then be read with ctu_get_state.  Syncs the batch
 *   stream (one read-back for all slots until the next submit or run).
 * ctu_batch_destroy: waits for the batch stream and releases every grid. */
enum { CTU_TICKET_QUEUED = 0, CTU_TICKET_RUNNING = 1, CTU_TICKET_DONE = 2, CTU_TICKET_FAILED = 3,
       CTU_TICKET_UNKNOWN = -1 };
enum { CTU_BATCH_GRAPH = 1 };
ctu_status ctu_batch_workspace_bytes(int32_t max_slots, size_t* work_bytes);
ctu_status ctu_batch_create(int32_t max_slots, void* d_work, size_t work_bytes, void* hip_stream,
                            int32_t flags, ctu_batch** out);
ctu_status ctu_batch_submit(ctu_batch* b, ctu_grid* g, int32_t nsteps, double t_end,
                            uint64_t* ticket); /* async */
ctu_status ctu_batch_run(ctu_batch* b, int32_t steps); /* async */
ctu_status ctu_batch_poll(ctu_batch* b, uint64_t ticket, int32_t* state, double* t_now); /* syncs */
ctu_status ctu_batch_destroy(ctu_batch* b);

/* ---- A step that allocates nothing -------------------------------------------------------
 * For callers that cannot allocate device memory: code under HIP graph capture, serving
 * loops that must not allocate, harnesses that forbid hipMalloc.  ctu_step_noalloc takes one
 * CTU step exactly as ctu_step does (same kernels, same results; the state's ghost cells are
 * filled by the step) of the state in d_state (the layout above, state_bytes of
 * ctu_workspace_bytes, 256-byte aligned, caller-owned), with the step's workspace taken from a
 * fixed array in the library's own device memory instead of a caller buffer:
 * CTU_NOALLOC_SCRATCH_BYTES (128 MiB) per GPU, which every GPU the library runs on holds
 * until the process ends.  A configuration whose work_bytes (ctu_workspace_bytes) exceeds it
 * is refused with CTU_EINVAL before anything is launched (PPMC + exact: up to about 76^3 real
 * cells in FP64, 97^3 in FP32).  cfg is validated as by ctu_workspace_bytes; dt must be finite
 * and > 0.  Uses the current device (hip_stream, NULL = default, must belong to it); calls no
 * hipMalloc, hipFree or other allocating routine, on the device or the host.  Async.
 * Every call on one GPU shares that GPU's array, which keeps the last call's contents (each
 * call rewrites all it reads): calls whose work overlaps on one GPU race, so order them (one
 * stream).  The step's device error word is not reported (there is no grid to query it). */
#define CTU_NOALLOC_SCRATCH_BYTES ((size_t)128 << 20)
ctu_status ctu_step_noalloc(const ctu_config* cfg, void* d_state, double dt, void* hip_stream);

/* Message for the last failing call on this thread (valid until the next call). */
const char* ctu_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
