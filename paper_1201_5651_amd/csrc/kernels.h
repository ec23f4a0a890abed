// kernels.h -- launch interface between the C-ABI runtime and the kernels.
//
// Every kernel works on a batch of grids described by an array of GridDev in
// device memory; a single grid is a batch of one, so one grid advanced alone
// and the same grid advanced inside a batch run the same per-cell arithmetic.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "physics.h"

namespace pi {

// Edges of the cubic tiles of the raytrace wavefront (octant-local cells swept
// by one workgroup); an engine uses one of them, chosen by timing them all on
// its first raytrace.
constexpr int NSWEEP = 3;
constexpr int SWEEP_TILES[NSWEEP] = { 4, 8, 16 };
constexpr int SWEEP_T_LARGEST = 16;
// Threads per workgroup of the micro-physics kernel.  Each wavefront
// integrates one brick of CHEM_BX x CHEM_BY x CHEM_BZ = 64 neighbouring cells
// (bricks in x, then y, then z order; bricks that overhang the grid leave
// lanes idle): cells that need many Newton iterations cluster in space, so a
// compact brick wastes fewer lanes than a 64-cell row.  The four bricks of a
// workgroup lie side by side along x (16 cells); pairs of consecutive
// workgroups, which share 128-byte lines, are kept on one XCD (xcd_block).
constexpr int CHEM_BLOCK = 256, CHEM_BX = 4, CHEM_BY = 4, CHEM_BZ = 4;
// XCDs of the device: the hardware hands workgroup ids to them in turn.
constexpr int NXCD = 8;
// Logical block of hardware workgroup id w in a launch of n workgroups: the two
// logical blocks 2m and 2m + 1, which share 128-byte lines, go to the same XCD
// (m % NXCD), and successive pairs go round the XCDs so that every XCD still
// samples the whole grid (work per cell varies in space).  A bijection of
// [0, n): the last n % (2 NXCD) blocks keep their ids.
__host__ __device__ constexpr int xcd_block(int w, int n)
{
    const int full = n - n % (2 * NXCD);
    if (w >= full) return w;
    const int x = w % NXCD, slot = w / NXCD;
    return 2 * NXCD * (slot / 2) + 2 * x + slot % 2;
}
static_assert(CHEM_BX * CHEM_BY * CHEM_BZ == 64, "one brick per wavefront");
// Bricks of a grid and micro-physics workgroups that cover them.
__host__ __device__ constexpr int64_t chem_bricks(int nx, int ny, int nz)
{
    return (int64_t)((nx + CHEM_BX - 1) / CHEM_BX) * ((ny + CHEM_BY - 1) / CHEM_BY) *
           ((nz + CHEM_BZ - 1) / CHEM_BZ);
}
__host__ __device__ constexpr int64_t chem_workgroups(int nx, int ny, int nz)
{
    return (chem_bricks(nx, ny, nz) + CHEM_BLOCK / 64 - 1) / (CHEM_BLOCK / 64);
}
// Threads per workgroup and largest number of workgroups per grid of the
// timestep/diagnostics reduction.
constexpr int DT_BLOCK = 256, DT_MAX_BLOCKS = 4096;
// Per-block partials of the timestep/diagnostics reduction:
// [0] min dt limit, [1] sum n(1-x), [2] sum (1-x), [3] sum A, [4] sum recomb, [5] non-finite cells
constexpr int NPART = 6;

// Grid clock and last reduction results, resident in device memory.
struct DevState {
    double t;
    double dt;        // timestep of the step in flight (0 once t >= t_end)
    double t_end;
    double last_dt;
    long long nsteps;
    long long pad;
    double diag[8];   // see pi_diagnostics
};

// Micro-integration work counters (accepted, rejected substeps, fallback
// solves, Newton iterations, cells re-solved in double), each spread over
// WORK_SLOTS slots so that the per-workgroup atomic additions do not all meet
// on one address; a reader sums the slots.  Layout: counter c, slot s at
// [c * WORK_SLOTS + s].
constexpr int WORK_COUNTERS = 5, WORK_SLOTS = 64;

// Device view of one grid.  Field arrays are indexed by the buffer selectors
// of include/pi.h (0: state n, 1: half-step state).
template <typename R> struct GridDev {
    Params<R> p;          // parameters in the grid's arithmetic
    Params<double> pd;    // double parameters (mixed-precision re-solve)
    Sources<R> src;       // the sources beyond source 0 (read only when several)
    Sources<double> srcd;
    const R* nH;
    const R* nHr[2];      // density a raytrace of state 0 / 1 uses (1: time-centred, or nH)
    R* x[2];
    R* E[2];              // null when the temperature is fixed
    R* tau[2];
    DevState* st;
    double* part;         // timestep partials of the grid's blocks
    double cell_vol;
    double face_area;     // plane-parallel source: area of the lit face [cm^2]; else 0
    int noct;
};

// Launch geometry of a batch: grid g owns the workgroups [first[g], first[g+1])
// of a launch over all grids.
struct BatchDev {
    int ngrids;
    const int* chem_first;   // micro-physics workgroups (CHEM_BLOCK / 64 bricks each)
    const int* dt_first;     // timestep workgroups
    const int* row_first;    // rows along x of plane-parallel grids (0 for point sources)
    // Mixed precision: fix_n[0] is the length of fix_list, fix_n[1] counts the
    // finished workgroups of launch_chem_fix (both zero between launches);
    // fix_n[2] asks for the conditional raytrace after a fused launch.
    unsigned int* fix_n;
    long long* fix_list;     // (grid << 32) | cell, for the double re-solve
    unsigned int fix_cap;    // entries fix_list holds
    // Grid kinds present: bit 0 grids with one source, bit 1 grids with
    // several.  The micro-physics and timestep kernels come in one variant per
    // kind; with both kinds each launch skips the workgroups of the other.
    int kinds;
};

// Control block of the persistent raytrace and of the fused micro-physics
// (zeroed once when allocated): the workgroups that have left, the epoch of
// the last completed call (the face entries and done-flags of the current
// call carry epoch + 1), an error flag set when a wait exceeded its limit,
// and the tickets of the tile lists.
struct SweepCtl {
    unsigned exited, epoch, err;
    unsigned lticket[NXCD];   // tickets of the tile lists (TileLists)
};
// Tile lists of a persistent launch: list l holds tiles[first[l] ..
// first[l + 1]) in schedule order; with n = NXCD, workgroup w takes from list
// w % NXCD, the list of the XCD the hardware deals it to.
struct TileLists {
    int n;
    int first[NXCD + 1];
};
// Tile edge of the persistent raytrace, and the index of its variant after
// the one-launch-per-stage variants of SWEEP_TILES.
constexpr int PERSIST_TILE = 8;
constexpr int SWEEP_PERSIST = 3;
constexpr int PERSIST_SCHEDULE = 1;   // SWEEP_TILES[1] == PERSIST_TILE
// Entries of the face buffer per tile of the persistent raytrace (for its
// three downstream faces, sigma0 n_H x dx and the centre column of every
// cell), FACE_BYTES each: a double, or a float with the epoch of the launch
// that wrote it.
constexpr int FACE_WORDS = 6 * PERSIST_TILE * PERSIST_TILE;
constexpr int FACE_BYTES = 8;
// Threads per workgroup of the micro-physics fused with the persistent sweep
// (two wavefronts, four 4^3 bricks of a tile each).
constexpr int FUSED_THREADS = 128;

// One tile-diagonal stage of the raytrace of every grid with tiles of edge
// `tile` (one of SWEEP_TILES): tiles[first .. first + count) are
// (grid << 3 | octant, tx, ty, tz).
template <typename R>
hipError_t launch_sweep_stage(const GridDev<R>* grids, int state, int tau_buf, const int4* tiles,
                              int first, int count, int tile, hipStream_t s);
// The whole raytrace of every grid in one launch of nwg persistent workgroups
// over the schedule of edge PERSIST_TILE (stage after stage) in `lists` of
// tiles (one list, or one per XCD when nwg >= NXCD); octs[grid << 3 | octant] = (first flag/slot index, tiles along x,
// y, z); fbuf: the face buffer, FACE_WORDS entries per tile, zeroed when
// allocated; flags: one done-flag per tile (used by double grids, whose face
// entries carry no epoch).  spin_ticks bounds each wait (100 MHz ticks).
// cond: null, or a word that must be non-zero for the raytrace to run
// (cleared by it).
template <typename R>
hipError_t launch_sweep_persist(const GridDev<R>* grids, int state, int tau_buf, const int4* tiles,
                                const TileLists& lists, const int4* octs, unsigned* flags,
                                void* fbuf, SweepCtl* ctl, int nwg, long long spin_ticks,
                                unsigned* cond, hipStream_t s);
// One half of an A3 step (or an A2 step) of every grid in one launch of nwg
// persistent workgroups, for batches of grids with one point source each:
// the micro-physics of launch_chem over h = hscale (x dt when dev_dt) from
// `from` to `to` on the columns tau_chem, then the raytrace of state `to`
// into tau_sweep, over the schedule and face buffer of launch_sweep_persist.
// With mixed, precision-sensitive cells are listed as by launch_chem (and
// swept with their float values): launch_chem_fix with mark, then
// launch_sweep_persist with cond = b.fix_n + 2, must follow.  Float storage
// only (hipErrorNotSupported for double).
template <typename R>
hipError_t launch_chem_sweep(const GridDev<R>* grids, const BatchDev& b, int from, int to,
                             int tau_chem, int tau_sweep, bool dev_dt, double hscale,
                             unsigned long long* ctr, bool mixed, const int4* tiles,
                             const TileLists& lists, const int4* octs, void* fbuf, SweepCtl* ctl,
                             int nwg, long long spin_ticks, hipStream_t s);
// Workgroups of k_chem_sweep one compute unit holds at once.
template <typename R> int chem_sweep_occupancy(bool mixed);
// Resident workgroups of the persistent raytrace kernel on one CU.
template <typename R> int sweep_persist_occupancy();
// Micro-physics of every cell of every grid from state `from` on columns
// `tau_buf` into state `to`, over h = hscale * (st->dt if dev_dt else 1).
// With mixed, precision-sensitive cells are listed for launch_chem_fix.
// Raytrace of the plane-parallel grids: one wavefront per row along x of
// every such grid (`rows` in all), a running column from the x = 0 face.
template <typename R>
hipError_t launch_plane_scan(const GridDev<R>* grids, const BatchDev& b, int rows, int state,
                             int tau_buf, hipStream_t s);
// Algorithm 1's pass (Sect. 2.1) over one stage of the 4^3 tile schedule
// (tiles[first .. first + count)): state n advanced in place over st->dt,
// time-averaged entering columns into tau[1], time-averaged optical depth per
// cell length into x[1].
template <typename R>
hipError_t launch_sweep_a1(const GridDev<R>* grids, const int4* tiles, int first, int count,
                           unsigned long long* ctr, int mixed, hipStream_t s);
// mixed: 0 none, 1 precision-sensitive cells to the double pass, 2 those and
// the ionisation-front cells.
template <typename R>
hipError_t launch_chem(const GridDev<R>* grids, const BatchDev& b, int nblocks, int from, int to,
                       int tau_buf, bool dev_dt, double hscale, unsigned long long* ctr,
                       int mixed, hipStream_t s);
// Mixed precision: double re-solve of the cells listed by launch_chem, from the
// unmodified float inputs; its last workgroup empties the list, so every
// launch_chem with mixed must be followed by one launch_chem_fix.  With mark,
// b.fix_n[2] is set when cells were re-solved (the condition word of a second
// raytrace after launch_chem_sweep).
hipError_t launch_chem_fix(const GridDev<float>* grids, const BatchDev& b, int nblk, int from,
                           int to, int tau_buf, bool dev_dt, double hscale,
                           unsigned long long* ctr, bool mark, hipStream_t s);
// Timestep limit (eq. 4) and diagnostics of state n of every grid, reduced per
// grid; t_end_arg finite: the t_end of every grid, else each grid's st->t_end.
template <typename R>
hipError_t launch_dtdiag(const GridDev<R>* grids, const BatchDev& b, int nblocks, double t_end_arg,
                         hipStream_t s);
template <typename R>
hipError_t launch_advance(const GridDev<R>* grids, int ngrids, hipStream_t s);
template <typename R>
hipError_t launch_energy(int64_t n, const R* nH, const R* x, R* E, double T0, hipStream_t s);
// Sets the t_end of a grid clock (a step replayed from a captured graph reads
// it there).
hipError_t launch_set_t_end(DevState* st, double t_end, hipStream_t s);

}  // namespace pi
