/*
 * pi.h -- C ABI of the MI355X photoionisation source-term library.
 *
 * The library advances non-equilibrium hydrogen photoionisation on a uniform
 * 3D Cartesian grid around a point source by the second-order explicit,
 * operator-split step of Mackey, "Accuracy and efficiency of raytracing
 * photoionisation algorithms" (A&A 2012), algorithm 3 of Sect. 2.2:
 * raytrace at t_n (which also sets the timestep, eq. 4 and Table 1),
 * micro-physics over dt/2 on those columns, raytrace of the half-step state,
 * micro-physics over dt from t_n on the time-centred columns.  The paper's
 * statement of the problem gives the module two interfaces, one for the
 * timestep and one for the micro-physical update (Sect. 2.1); pi_timestep and
 * pi_chem_step are those two, pi_raytrace is the short-characteristics tracer
 * they depend on (Sect. 2, Sect. 5), and pi_step_o2 composes them.
 *
 * Conventions
 *  - Units are CGS.  Fields are structure-of-arrays of nx*ny*nz cells with x
 *    varying fastest: cell (i,j,k) is element i + nx*(j + ny*k).
 *  - Field pointers are DEVICE pointers owned by the caller (e.g. torch
 *    tensors); they must stay valid until pi_grid_destroy.  Element type is
 *    double for PI_FP64 and float for PI_FP32 / PI_MIXED / PI_MIXED_FRONT.
 *  - Every call that takes a stream enqueues asynchronous work on that HIP
 *    stream (hipStream_t passed as void*; NULL = the null stream) and returns
 *    without waiting, except the calls documented as synchronising.
 *  - Every call returns a pi_status; nothing throws across the ABI.  On error
 *    pi_last_error() returns a message (thread-local, valid until the next call
 *    on the same thread).
 */
#ifndef PI_H
#define PI_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    PI_OK = 0,
    PI_PENDING = 1,      /* served request queued or running                  */
    PI_EINVAL = -1,      /* invalid argument or descriptor                    */
    PI_ENOMEM = -2,      /* device allocation failed                          */
    PI_EDEVICE = -3,     /* HIP runtime error                                 */
    PI_EREJECTED = -4,   /* served request larger than the server's budget    */
    PI_ENAN = -5,        /* a non-finite value was found in the grid's state  */
    PI_ECANCELLED = -6   /* served request cancelled                          */
} pi_status;

/* PI_MIXED: float fields and float bulk arithmetic.  A cell is re-solved in
 * double from the same float inputs when its float integration took a
 * decision that the precision can flip: a substep-control decision within a
 * relative 1e-3 of its threshold (initial substep count, rejection of a
 * substep), a stage solve that needed the bracketed fallback, or a neutral
 * fraction held at 1 on an unstable equilibrium.
 * PI_MIXED_FRONT: PI_MIXED, and the ionisation-front cells in double: a cell
 * whose neutral fraction at the start of a micro-physics update lies in
 * [1e-3, 0.5] (the front's transition layer between ionised and mostly
 * neutral gas) is integrated in double only.
 * Both store results in float.  Reductions (timestep, diagnostics) are double
 * in every precision. */
typedef enum { PI_FP64 = 0, PI_FP32 = 1, PI_MIXED = 2, PI_MIXED_FRONT = 3 } pi_precision;
enum { PI_SPEC_MONO = 0, PI_SPEC_TABLE = 1 };
enum { PI_T_FIXED = 0, PI_T_EVOLVE = 1 };
enum { PI_ALPHA_CONST = 0, PI_ALPHA_POWER = 1 };
enum { PI_W_GEOMETRIC = 0, PI_W_MELLEMA = 1 };
/* PI_SRC_POINT: point source at the vertex src (Sect. 2, Sect. 5);
 * PI_SRC_PLANE: plane-parallel source at x = -infinity (the slab test of
 * Sect. 3.1 on a 3D grid): each row of cells along x is traced from the x = 0
 * face, and Q is the photon flux entering that face. */
enum { PI_SRC_POINT = 0, PI_SRC_PLANE = 1 };
/* which state / column buffer an operation reads or writes */
enum { PI_BUF_N = 0, PI_BUF_HALF = 1 };
/* number of FP64 diagnostics returned by pi_diagnostics */
#define PI_NDIAG 8
/* number of work counters returned by pi_work_counters */
#define PI_NWORK 5
#define PI_NTAB 64
/* most point sources of one grid */
#define PI_MAX_SRC 4

/* Problem description (copied by pi_grid_create). */
typedef struct {
    int32_t n[3];             /* cells per axis, each >= 1                            */
    int32_t src[3];           /* source vertex, 0 <= src[d] <= n[d] (Sect. 5: the     */
                              /* source sits on the nearest cell vertex); unused for  */
                              /* PI_SRC_PLANE                                         */
    double  dx;               /* cell size [cm], > 0                                  */
    double  Q;                /* ionising photons per second, >= 0; PI_SRC_PLANE:     */
                              /* photons per cm^2 per second into the x = 0 face      */
    double  sigma0;           /* photoionisation cross-section at 13.6 eV [cm^2] > 0  */
    int32_t spectrum;         /* PI_SPEC_MONO, or PI_SPEC_TABLE: blackbody of T_bb    */
                              /* with rates tabulated against optical depth (Sect. 2) */
    double  e_excess;         /* MONO: heating per photoionisation [erg], >= 0        */
    double  T_bb;             /* TABLE: blackbody temperature [K], > 0                */
    int32_t thermal;          /* PI_T_FIXED (T = T_fixed) or PI_T_EVOLVE (eq. 2 for E)*/
    double  T_fixed;          /* [K]                                                  */
    int32_t recomb;           /* PI_ALPHA_CONST: alpha_B; PI_ALPHA_POWER:             */
                              /* alpha_B (T / 1e4 K)^-0.7                             */
    double  alpha_B;          /* case-B coefficient [cm^3/s], >= 0                    */
    int32_t collisional;      /* 1: collisional ionisation rate and its cooling       */
    int32_t cooling;          /* 1: radiative cooling (PI_T_EVOLVE only)              */
    int32_t weights;          /* PI_W_MELLEMA (default) or PI_W_GEOMETRIC             */
    int32_t source_cell_rule; /* 1: each octant's corner cell takes Q/8 (default)     */
    int32_t n_sub;            /* micro-integration substeps, 1..64                    */
    double  K[4];             /* eq. (4) factors K1..K4; +inf disables a criterion    */
                              /* (dt02 of Table 1: {inf, inf, inf, 0.25})             */
    int32_t precision;        /* pi_precision                                         */
    int32_t source;           /* PI_SRC_POINT or PI_SRC_PLANE                         */
    /* Several point sources (PI_SRC_POINT; grids, batches and served requests;
     * not algorithm 1).  nsrc 0 or 1: the source at src with Q alone.  nsrc = m in 2..PI_MAX_SRC:
     * source 0 at src with Q, source s = 1..m-1 at vertex src_more[s-1] with
     * Q_more[s-1] photons per second (>= 0); all share the spectrum.  Each
     * source is traced on its own and the photoionisation and heating rates of
     * the sources add in every cell.  tau and tau_half then hold m consecutive
     * arrays of nx*ny*nz cells, source s at element offset s*nx*ny*nz. */
    int32_t nsrc;
    int32_t src_more[PI_MAX_SRC - 1][3];
    double  Q_more[PI_MAX_SRC - 1];
} pi_grid_desc;

/* Caller-owned device fields (see Conventions).  E and E_half may be NULL when
 * thermal == PI_T_FIXED.  x_half / E_half / tau_half hold the half-step state
 * and its columns. */
typedef struct {
    void* nH;        /* hydrogen number density [cm^-3], > 0                  */
    void* x;         /* neutral fraction 1 - y in [0, 1] (Sect. 2.1)          */
    void* E;         /* internal energy density [erg cm^-3]                   */
    void* tau;       /* threshold optical depth from the source to each       */
                     /* cell's entry face, for (x, E); nsrc > 1: one array of */
                     /* cells per source, source after source                 */
    void* x_half;
    void* E_half;
    void* tau_half;
    void* nH_half;   /* optional, may be NULL: the density at t + dt/2 that the */
                     /* raytrace of the half-step state uses (Sect. 2.2: the    */
                     /* time-centred density of a hydrodynamics code); NULL:    */
                     /* nH.  Read at every raytrace of PI_BUF_HALF.             */
} pi_fields;

typedef struct pi_grid pi_grid;

/* Validate the descriptor (n >= 1, 0 <= src <= n, dx > 0, Q >= 0, sigma0 > 0,
 * n_sub in 1..64, K > 0 (inf disables), known enums), build the rate table (TABLE mode), upload
 * the constants and bind the fields.  Allocates the grid's small private device
 * buffers (reduction partials, timestep scalars, tile schedule, table).
 * Returns PI_EINVAL, PI_ENOMEM or PI_EDEVICE on failure (nothing is leaked). */
pi_status pi_grid_create(const pi_grid_desc* desc, const pi_fields* fields, pi_grid** out);

/* Free the grid's private buffers (synchronises the device first).  The
 * caller's fields are not touched.  NULL is accepted. */
pi_status pi_grid_destroy(pi_grid* grid);

/* Memory a grid of this description needs (host-only, no device call):
 * *field_bytes = bytes of the caller-owned fields pi_fields points to, i.e.
 *   nx*ny*nz*w * (3 + 2 m + (PI_T_EVOLVE ? 2 : 0)) with w = 8 (PI_FP64) or 4
 *   and m sources (n_H, x, x_half, m arrays each of tau and tau_half, E and
 *   E_half; nH_half not counted);
 * *work_bytes = device bytes pi_grid_create allocates privately (clock,
 *   reduction partials, tile schedules of every tile edge, launch tables,
 *   work counters, the mixed-precision re-solve list of one entry per cell,
 *   the rate table), before the allocator's rounding.
 * Either pointer may be NULL.  PI_EINVAL for an invalid descriptor.  (The
 * paper states the problem's inputs per cell, Sect. 2.1; this sizes them.) */
pi_status pi_grid_required_bytes(const pi_grid_desc* desc, size_t* field_bytes,
                                 size_t* work_bytes);

/* Checkpoint of a grid's state (SYNCHRONISES the stream): a header with the
 * layout and the clock (t, dt, t_end, last dt, step count), then n_H, x, E
 * (PI_T_EVOLVE only) and the columns of every source, each nx*ny*nz values of
 * the grid's word size in the field layout.  The half-step buffers are not
 * saved (a step does not read them before writing them).  *needed (if not
 * NULL) receives the size; host_buf NULL is a size query.  host_buf is host
 * memory owned by the caller, at least *needed bytes (PI_EINVAL otherwise).
 * A grid loaded from it continues bit for bit as the saved grid would have. */
pi_status pi_grid_save(pi_grid* grid, void* host_buf, size_t bytes, size_t* needed,
                       void* stream);
/* Loads a checkpoint written by pi_grid_save (or pi_checkpoint) into the
 * grid's fields and clock (SYNCHRONISES the stream).  PI_EINVAL unless the
 * checkpoint has the grid's layout: cells per axis, precision, thermal mode
 * and number of sources; the other parameters are the loading grid's own. */
pi_status pi_grid_load(pi_grid* grid, const void* host_buf, size_t bytes, void* stream);

/* Short-characteristics raytrace (Sect. 2; Sect. 5): columns tau of the
 * neutral fractions of state `state` (PI_BUF_N: x, PI_BUF_HALF: x_half) into
 * `tau_buf` (PI_BUF_N: tau, PI_BUF_HALF: tau_half).  Octants around the
 * source vertex are traced independently in tile-wavefront order. */
pi_status pi_raytrace(pi_grid* grid, int state, int tau_buf, void* stream);

/* Micro-physics update (eq. 2 for the neutral fraction and, with PI_T_EVOLVE,
 * the internal energy) of every cell from state `from_state` over an interval
 * h with the entering columns `tau_buf` frozen, written to `to_state`
 * (from == to updates in place).  h = h_value seconds when use_device_dt == 0,
 * else h = h_value * (the timestep last computed by pi_timestep/pi_step_o2,
 * held on the device). */
pi_status pi_chem_step(pi_grid* grid, int use_device_dt, double h_value, int tau_buf,
                       int from_state, int to_state, void* stream);

/* pi_chem_step followed by pi_raytrace(grid, to_state, tau_out): the
 * micro-physics of the cells and then the columns of the new state, the pair
 * each half of the step of Sect. 2.2 runs.  With the persistent raytrace
 * (PI_TILE_PERSISTENT) on a grid of float storage with one point source
 * (not PI_MIXED_FRONT; with PI_MIXED, tau_buf != tau_out), the two run as one
 * launch in which every tile integrates its cells and then sweeps them;
 * otherwise as the two calls.  The results are the same either way, bit for
 * bit.  Arguments as for the two calls. */
pi_status pi_chem_raytrace(pi_grid* grid, int use_device_dt, double h_value, int tau_buf,
                           int from_state, int to_state, int tau_out, void* stream);

/* Timestep (eq. 4 with the grid's K1..K4): min over cells of the limit
 * evaluated at state PI_BUF_N with columns tau, reduced in FP64, capped at
 * t_end - t (a remainder below 1e-12 t_end is absorbed).  The result stays on
 * the device for pi_chem_step / pi_step_o2; pi_grid_state reads it. */
pi_status pi_timestep(pi_grid* grid, double t_end, void* stream);

/* One step of algorithm 3 (Sect. 2.2): pi_timestep; predictor over dt/2 on
 * tau into the half state; raytrace of the half state into tau_half; corrector
 * over dt from (x, E) on tau_half in place; raytrace of the new state into
 * tau; t += dt.  Requires tau to hold the columns of (x, E) on entry (call
 * pi_raytrace(grid, PI_BUF_N, PI_BUF_N, s) once after loading a state).  Does
 * nothing useful once t >= t_end (dt = 0).  The step's kernels are replayed
 * from a HIP graph the grid captures on its first step (the clock carries
 * t_end into it); on a stream that is itself being captured they are launched
 * directly, so they become part of the caller's graph. */
pi_status pi_step_o2(pi_grid* grid, double t_end, void* stream);

/* One step of algorithm 2 (Sect. 2.2), the first-order variant: timestep,
 * micro-physics over dt on tau, raytrace of the new state. */
pi_status pi_step_o1(pi_grid* grid, double t_end, void* stream);

/* One step of algorithm 1 (Sect. 2.1), the implicit scheme with time-averaged
 * attenuation: timestep (eq. 4 with the grid's K; Table 1's implicit columns
 * limit it by K1 t_rec), then one pass over the cells in raytrace order in
 * which each cell is integrated over dt on the time-averaged column entering
 * it while its attenuation exp(-Delta tau) is averaged over the step; the
 * cell's time-averaged optical depth -ln <exp(-Delta tau)> then enters the
 * columns of the cells behind it.  Afterwards x_half holds each cell's
 * time-averaged optical depth per cell length (sigma0 dx units), tau_half the
 * time-averaged entering columns, and tau the columns of the new state (a
 * raytrace, for the next timestep).  One point source only (PI_EINVAL for
 * PI_SRC_PLANE or nsrc > 1); the pass runs on 8^3 tiles whatever the raytrace
 * tile. */
pi_status pi_step_a1(pi_grid* grid, double t_end, void* stream);

/* Energy density of state `state` from a uniform temperature T0 [K] for pure
 * hydrogen with gamma = 5/3 (Sect. 2): E = 3/2 n_H (2 - x) k_B T0. */
pi_status pi_init_energy(pi_grid* grid, double T0, int state, void* stream);

/* Set the grid clock (t, step count, last dt) on the device. */
pi_status pi_set_time(pi_grid* grid, double t, int64_t nsteps, void* stream);

/* Read the grid clock.  SYNCHRONISES the stream. */
pi_status pi_grid_state(pi_grid* grid, double* t, int64_t* nsteps, double* last_dt,
                        void* stream);

/* FP64 diagnostics of state PI_BUF_N with columns tau (SYNCHRONISES):
 * out[0] ions sum n_H (1-x) V, out[1] ionised volume sum (1-x) V,
 * out[2] volume-equivalent ionised radius (3 V_ion 8 / (4 pi n_octants))^1/3
 * (PI_SRC_PLANE: ionised depth, V_ion over the area of the lit face; several
 * sources: n_octants counts the octants of every source),
 * out[3] photoionisations per second, out[4] recombinations per second,
 * out[5] number of non-finite cells, out[6] number of octants (0 for
 * PI_SRC_PLANE), out[7] time t. */
pi_status pi_diagnostics(pi_grid* grid, double* out, void* stream);

/* Work of the micro-physics updates since the last reset (SYNCHRONISES):
 * out[0] accepted substeps, out[1] rejected substeps, out[2] stage solves that
 * needed the bracketed fallback, out[3] Newton iterations of the stage solves,
 * out[4] cells re-solved in double by PI_MIXED / PI_MIXED_FRONT grids (out has PI_NWORK
 * elements).  reset != 0 zeroes the counters after reading.
 * Counters are summed over all pi_chem_step / step calls of the grid. */
pi_status pi_work_counters(pi_grid* grid, int64_t* out, int reset, void* stream);

/* ------------------------------------------------------------- batches
 * A batch advances many grids together: every kernel of a step is one launch
 * over the cells (or raytrace tiles) of all grids, and the step is replayed
 * from a captured HIP graph.  Each grid keeps its own descriptor, fields,
 * clock, timestep (eq. 4 reduced over its own cells) and t_end; a grid at its
 * t_end takes dt = 0 while the others go on.  A grid advanced in a batch goes
 * through the same per-cell arithmetic as the same grid advanced alone with
 * pi_step_o2, so its results do not depend on the composition of the batch
 * (up to the summation order of the diagnostics). */
typedef struct pi_batch pi_batch;

/* ngrids descriptors and fields (arrays of ngrids, copied; the fields stay
 * owned by the caller and valid until pi_batch_destroy).  All descriptors
 * share one precision; grids with one and with several sources may be mixed.
 * Errors as pi_grid_create, prefixed with the grid. */
pi_status pi_batch_create(int ngrids, const pi_grid_desc* descs, const pi_fields* fields,
                          pi_batch** out);
/* Synchronises the device and frees the batch; NULL is accepted. */
pi_status pi_batch_destroy(pi_batch* batch);
/* Per grid (host arrays of ngrids): clock t, step count (NULL: 0) and t_end
 * of the steps to come.  SYNCHRONISES the stream. */
pi_status pi_batch_set_time(pi_batch* batch, const double* t, const int64_t* nsteps,
                            const double* t_end, void* stream);
/* pi_init_energy for every grid, T0 a host array of ngrids. */
pi_status pi_batch_init_energy(pi_batch* batch, const double* T0, int state, void* stream);
/* pi_raytrace of every grid. */
pi_status pi_batch_raytrace(pi_batch* batch, int state, int tau_buf, void* stream);
/* One algorithm-3 step of every grid toward its own t_end (pi_step_o2 with the
 * t_end set by pi_batch_set_time), enqueued as one graph launch on stream. */
pi_status pi_batch_step_o2(pi_batch* batch, void* stream);
/* One algorithm-1 step (pi_step_a1) of every grid, each to its own t_end;
 * launched directly (not from a captured graph).  PI_EINVAL if a grid has a
 * plane-parallel source or several sources. */
pi_status pi_batch_step_a1(pi_batch* batch, void* stream);
/* Per grid clock (host arrays of ngrids; NULL skips).  SYNCHRONISES. */
pi_status pi_batch_state(pi_batch* batch, double* t, int64_t* nsteps, double* last_dt,
                         void* stream);
/* pi_diagnostics of every grid: out[ngrids * PI_NDIAG], grid-major.  SYNCHRONISES. */
pi_status pi_batch_diagnostics(pi_batch* batch, double* out, void* stream);
/* pi_work_counters summed over the grids of the batch.  SYNCHRONISES. */
pi_status pi_batch_work_counters(pi_batch* batch, int64_t* out, int reset, void* stream);

/* -------------------------------------------------------------- serving
 * A server owns a worker thread, a HIP stream and one device allocation of
 * hbm_budget bytes (an arena for the fields of the requests it holds).
 * Submitted requests are admitted in arrival order while fewer than max_active
 * grids are running and their fields fit in the arena; all admitted grids are
 * advanced together as one batch (steps_per_tick algorithm-3 steps between
 * admission checks) until each reaches its t_end, then their results are
 * copied to host memory and their arena space is reused.  Calls that overlap
 * on one server are safe (a mutex guards its queues). */
typedef struct pi_server pi_server;

typedef struct {
    size_t  hbm_budget;       /* arena bytes; 0: 80% of the free device memory    */
    int32_t max_active;       /* grids advanced together at most, >= 1           */
    int32_t precision;        /* pi_precision of every request                   */
    int32_t steps_per_tick;   /* batch steps between admission checks, >= 1      */
} pi_server_desc;

typedef struct {
    pi_grid_desc  desc;       /* precision must be the server's                  */
    const double* nH;         /* host, n[0]*n[1]*n[2] cells, > 0 (copied)         */
    const double* x0;         /* host initial neutral fraction, or NULL: 1       */
    double        T0;         /* initial temperature [K] (T evolving)            */
    double        t_end;      /* time to advance to from t = 0 [s]               */
    /* Optional (NULL: start from nH, x0, T0 at t = 0): a checkpoint written by
     * pi_grid_save or pi_checkpoint for this desc's layout (copied).  The
     * request then resumes from its state and clock (density included; nH,
     * x0 and T0 are ignored) and runs to t_end. */
    const void*   checkpoint;
    size_t        checkpoint_bytes;
} pi_request;

typedef struct {
    int32_t status;           /* PI_OK, PI_PENDING or the failure status         */
    double  t;                /* time reached                                    */
    int64_t nsteps;           /* steps taken                                     */
    double  latency_s;        /* submission to completion (or to now)            */
    double  queue_s;          /* submission to admission (or to now)             */
} pi_result;

/* Starts the worker thread on the current device.  PI_ENOMEM if the arena
 * cannot be allocated.  A running request whose clock does not advance over a
 * whole tick before its t_end fails with PI_EDEVICE.  Finished requests' x and
 * E are copied to pinned host memory on a second stream while the other
 * grids go on; their arena space is reused once the copy is complete. */
pi_status pi_server_create(const pi_server_desc* desc, pi_server** out);
/* Validates and copies the request (host arrays); returns a ticket.
 * PI_EREJECTED if its fields can never fit in the arena. */
pi_status pi_submit(pi_server* server, const pi_request* request, uint64_t* ticket);
/* Status of a ticket.  PI_PENDING while queued or running; once finished,
 * returns PI_OK and copies the final neutral fraction and temperature into
 * x_out and T_out (host arrays of the grid's cells, either may be NULL), or
 * returns the failure status; the ticket is released in both cases. */
pi_status pi_poll(pi_server* server, uint64_t ticket, pi_result* out, double* x_out,
                  double* T_out);
/* Asks for a ticket to be dropped (queued: at once; running: at the next tick).
 * Its poll then returns PI_ECANCELLED. */
pi_status pi_cancel(pi_server* server, uint64_t ticket);
/* Checkpoint of a running request (the pi_grid_save format), taken by the
 * worker at the end of its current tick of steps; the call BLOCKS until then.
 * host_buf NULL is a size query (*needed).  Returns PI_PENDING if the request
 * is still queued (nothing to save yet), PI_EINVAL if it has finished (poll
 * it) or the buffer is too small, PI_EDEVICE if the tick failed.  Submitting
 * the checkpoint (pi_request.checkpoint) continues the request bit for bit. */
pi_status pi_checkpoint(pi_server* server, uint64_t ticket, void* host_buf, size_t bytes,
                        size_t* needed);
/* out[8]: completed requests, cell-updates done, busy seconds of the worker,
 * batch steps, running grids, queued requests, arena bytes in use, batch
 * rebuilds. */
pi_status pi_server_stats(pi_server* server, double* out);
/* Stops the worker (running requests are dropped) and frees everything. */
pi_status pi_server_destroy(pi_server* server);

/* Host-only: blackbody rate table of the TABLE spectrum (Sect. 2, rates
 * tabulated against optical depth): out[5*PI_NTAB] = node optical depths, P
 * (photons/s surviving a threshold column tau), -dP/dtau, H (excess energy
 * carried, erg/s), -dH/dtau, for a T_bb blackbody of Q photons/s with
 * cross-section sigma0 (nu0/nu)^3.  Nodes: 0, then 63 log-spaced in [1e-4, 1e4]. */
pi_status pi_table_build(double T_bb, double Q, double* out);

/* The raytrace of pi_raytrace for a grid given only by its description and
 * fields, without a pi_grid and without allocating anything: for callers that
 * cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid allocation).  The grid table and the tile
 * schedule the sweep reads live in a static device array of the library
 * (4 MiB + 16 KiB on every device it runs on, held until the process ends),
 * written by a set-up kernel on the stream before the sweep.  Limits: at most
 * 262144 raytrace tiles of edge 8 over all sources and octants (e.g. 512^3
 * cells with one source, 256^3 with four) and 4096 tile diagonals;
 * PI_EINVAL beyond them, before anything is launched.  Validation, arguments
 * and columns as pi_raytrace (bit for bit).  Every call on a device shares
 * that device's array: calls that overlap on one device (another stream,
 * another thread) race and must not overlap. */
pi_status pi_raytrace_static(const pi_grid_desc* desc, const pi_fields* fields, int state,
                             int tau_buf, void* stream);

/* Raytrace tile edge: 4, 8 or 16 (cells of the cubic tile one workgroup
 * sweeps, one launch per tile diagonal), PI_TILE_PERSISTENT (8^3 tiles, the
 * whole raytrace in one launch of persistent workgroups that claim tiles in
 * wavefront order and wait until their upstream tiles have published the
 * halo they need, each wait bounded by pi_set_raytrace_wait_limit), or 0 to
 * time them all on the next
 * raytrace outside graph capture and keep the fastest (the default; that
 * first raytrace then SYNCHRONISES its stream).  The choice does not change
 * any result: every cell's interpolation is the same.  pi_get_raytrace_tile
 * returns 0 while untuned.  PI_EINVAL for other values. */
#define PI_TILE_PERSISTENT 0x108
pi_status pi_set_raytrace_tile(pi_grid* grid, int edge);
pi_status pi_get_raytrace_tile(pi_grid* grid, int* edge);
pi_status pi_batch_set_raytrace_tile(pi_batch* batch, int edge);
pi_status pi_batch_get_raytrace_tile(pi_batch* batch, int* edge);

/* Longest wait, in seconds, of a tile of the persistent raytrace
 * (PI_TILE_PERSISTENT) for its upstream tiles; 0.02 by default.  A wait that
 * runs out lets the workgroup go on with the columns as they stand, so the
 * launch always ends; the raytrace is then invalid and the next
 * synchronising call on the grid or batch returns PI_EDEVICE (once).  Any
 * value in [0, PI_WAIT_LIMIT_MAX]; 0 fails every wait that is not met at its
 * first look (a way to exercise that path).  Drops a captured step graph.
 * PI_EINVAL outside the range.  The staged raytraces do not wait. */
#define PI_WAIT_LIMIT_MAX 10.0
pi_status pi_set_raytrace_wait_limit(pi_grid* grid, double seconds);
pi_status pi_batch_set_raytrace_wait_limit(pi_batch* batch, double seconds);

/* Thread-local message of the last failing call on this thread ("" if none). */
const char* pi_last_error(void);

/* ABI version of this header (major * 100 + minor); the library returns the
 * value it was built with. */
#define PI_ABI_VERSION 111
int pi_abi_version(void);

#ifdef __cplusplus
}
#endif
#endif
