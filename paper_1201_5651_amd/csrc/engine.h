// engine.h -- host side of a batch of grids advanced together.
//
// A GridHost holds one grid: its descriptor, the caller's field pointers, and
// the small device buffers that belong to the grid alone (clock, reduction
// partials).  An Engine advances a set of GridHost of one precision with one
// launch per kernel for the whole set: it owns the device descriptor array,
// the launch geometry, the combined raytrace tile schedule, the mixed-precision
// re-solve list, the work counters and the rate tables (shared between grids
// with the same spectrum).  A single grid is an Engine over one GridHost.
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "../../include/pi.h"
#include "kernels.h"

namespace pi {

// Sets the thread-local message returned by pi_last_error.
pi_status fail(pi_status s, const std::string& msg);
const std::string& last_error();
pi_status validate_desc(const pi_grid_desc* d);
pi_status validate_fields(const pi_grid_desc* d, const pi_fields* f);

struct GridHost {
    pi_grid_desc d{};
    pi_fields f{};
    DevState* st = nullptr;   // device clock and diagnostics
    double* part = nullptr;   // device timestep partials (nblk_dt * NPART)
    int nblk_dt = 0;
    int noct = 0;
    double cell_vol = 0.0;
    int64_t ncell = 0;
    // per source, per tile edge (SWEEP_TILES), per tile diagonal:
    // (octant, tx, ty, tz)
    std::vector<std::vector<int4>> tiles[MAX_SRC][NSWEEP];
};

pi_status grid_host_init(GridHost& h, const pi_grid_desc& d, const pi_fields& f);
void grid_host_free(GridHost& h);

struct Engine {
    int precision = PI_FP64;
    std::vector<GridHost*> grids;
    void* gdev = nullptr;            // GridDev<R>[ngrids]
    size_t gdev_cap = 0;
    int* first = nullptr;            // chem_first[ngrids+1], then dt_first[ngrids+1]
    size_t first_cap = 0;
    int chem_blocks = 0, dt_blocks = 0;
    int plane_rows = 0;   // rows along x of the plane-parallel grids
    // (grid, source) of the raytrace entries past the grids: the further
    // sources of the grids with several; kinds as BatchDev::kinds
    std::vector<int2> extra;
    int kinds = 1;
    // raytrace schedules, one per tile edge of SWEEP_TILES
    int4* tiles[NSWEEP] = {};
    size_t tiles_cap[NSWEEP] = {};
    std::vector<int> stage_first[NSWEEP], stage_count[NSWEEP];
    // raytrace variant: 0..NSWEEP-1 one launch per tile diagonal with tiles
    // of edge SWEEP_TILES[sweep]; SWEEP_PERSIST one persistent launch over
    // the schedule of edge PERSIST_TILE; -1 until tuned
    int sweep = -1;
    // persistent raytrace: per raytrace entry and octant (first flag and slot
    // index, tiles along x, y, z), one done-flag per tile (double grids), the
    // face buffer, the control block, and the workgroups of a launch
    int4* octs = nullptr;
    size_t octs_cap = 0;
    unsigned* flags = nullptr;
    size_t flags_cap = 0;
    void* fbuf = nullptr;        // face buffer: FACE_WORDS entries of FACE_BYTES per tile
    size_t fbuf_cap = 0;
    // the persistent schedule dealt into one list per XCD (TileLists), for
    // the fused launches
    int4* xtiles = nullptr;
    size_t xtiles_cap = 0;
    TileLists xlists{};
    SweepCtl* ctl = nullptr;
    int persist_wg = 0;
    // longest wait of a persistent tile for its upstream tiles (ticks of the
    // 100 MHz real-time counter); 2e6 = 20 ms unless the caller sets it
    long long persist_spin = 2000000LL;
    // workgroups of a launch of the micro-physics fused with the persistent
    // sweep (float storage; 0 until built)
    int fused_wg = 0;
    // whether a step runs the micro-physics and the raytrace that follows
    // it as one fused launch: float storage (not the front-in-double form,
    // whose front cells all go to the double pass), the persistent raytrace,
    // and only grids with one point source
    bool fused() const;
    unsigned int* fix_n = nullptr;
    long long* fix_list = nullptr;
    size_t fix_cap = 0;
    int fix_blocks = 0;
    unsigned long long* work = nullptr;
    struct Table {
        int spectrum;
        double T_bb;
        void* d;   // DevTable<double>
        void* f;   // DevTable<float>
    };
    std::vector<Table> tables;
    // When set, tables are looked up in and added to this cache instead, which
    // outlives the engine (engine_free then leaves them alone).
    std::vector<Table>* table_cache = nullptr;
    hipStream_t cap = nullptr;       // capture stream of the step graph
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;

    bool fp64() const { return precision == PI_FP64; }
    bool mixed() const { return precision == PI_MIXED || precision == PI_MIXED_FRONT; }
    // the double pass also takes the ionisation-front cells
    bool front() const { return precision == PI_MIXED_FRONT; }
    int ngrids() const { return (int)grids.size(); }
    BatchDev bd() const;
};

// (Re)builds the device structures of e for `grids` (all of e.precision);
// keeps allocations whose capacity suffices and drops a captured step graph.
pi_status engine_build(Engine& e, const std::vector<GridHost*>& grids);
void engine_free(Engine& e);
// Destroys a captured step graph (the next step captures a new one).
void engine_drop_graph(Engine& e);
// Whether the engine's steps would fuse the micro-physics with the persistent
// raytrace if that raytrace were chosen.
bool fused_eligible(const Engine& e);
void free_tables(std::vector<Engine::Table>& tables);

// Raytrace with the tuned tile edge; the first call outside graph capture times
// both tile edges on s (synchronising it) and keeps the faster.  Tiling does
// not change the arithmetic of any cell, so every edge gives the same columns.
pi_status engine_raytrace(Engine& e, int state, int tau_buf, hipStream_t s);
// The timing itself: raytraces of (state -> tau_buf) with each tile edge.
pi_status engine_autotune(Engine& e, int state, int tau_buf, hipStream_t s);
// Micro-physics, then the raytrace of state `to` into tau_out: fused when
// the engine's steps fuse and the buffers allow it, else the two in turn.
pi_status engine_chem_raytrace(Engine& e, bool dev_dt, double h, int tau_buf, int from, int to,
                               int tau_out, hipStream_t s);
pi_status engine_chem(Engine& e, bool dev_dt, double h, int tau_buf, int from, int to,
                      hipStream_t s);
// t_end_arg finite: the common t_end, else each grid's stored t_end.
pi_status engine_timestep(Engine& e, double t_end_arg, hipStream_t s);
pi_status engine_step(Engine& e, double t_end_arg, int order, hipStream_t s);
// One step of algorithm 1 (Sect. 2.1) for every grid (point sources only).
pi_status engine_step_a1(Engine& e, double t_end_arg, hipStream_t s);
// One A3 step of every grid toward its stored t_end, as a captured graph
// (captured on first use, replayed on s).
pi_status engine_step_graph(Engine& e, hipStream_t s);
pi_status engine_init_energy(Engine& e, int grid, double T0, int state, hipStream_t s);
// Clock and diagnostics of every grid (synchronise s).
pi_status engine_read_states(Engine& e, std::vector<DevState>& out, hipStream_t s);
pi_status engine_write_states(Engine& e, const std::vector<DevState>& in, hipStream_t s);
// Recomputed diagnostics of state n of every grid (ngrids * PI_NDIAG), leaving
// the clocks and the stored timesteps as they were (synchronises s).
pi_status engine_diagnostics(Engine& e, std::vector<double>& out, hipStream_t s);
pi_status engine_work(Engine& e, int64_t* out, int reset, hipStream_t s);

// Device bytes the library allocates for one grid created alone
// (pi_grid_required_bytes); also the bytes of its caller-owned fields.
size_t grid_private_bytes(const pi_grid_desc& d);
size_t grid_field_bytes(const pi_grid_desc& d);

// Checkpoint of one grid's state (pi_grid_save / pi_grid_load, and served
// requests): a header with the layout and the clock, then n_H, x, E (T
// evolving only) and the columns of every source, each nx*ny*nz values of
// the grid's word size in the field layout.
size_t checkpoint_bytes(const pi_grid_desc& d);
size_t checkpoint_header_bytes();
// Writes the checkpoint of h into buf (bytes >= checkpoint_bytes); the fields
// are read on s, which is synchronised.
pi_status grid_save(const GridHost& h, void* buf, size_t bytes, hipStream_t s);
// Checks that buf holds a checkpoint of h's layout (cells, precision,
// thermal mode, sources) and writes it into h's fields and clock on s
// (synchronised).
pi_status grid_load(GridHost& h, const void* buf, size_t bytes, hipStream_t s);
// Layout check of a checkpoint against a descriptor, without loading it.
pi_status checkpoint_check(const pi_grid_desc& d, const void* buf, size_t bytes);

// The raytrace entries of one grid (source 0, then one per further source)
// as an engine builds them, without rate tables or clock: out holds
// MAX_SRC entries; returns how many are used.
template <typename R> int raytrace_entries(const pi_grid_desc& d, const pi_fields& f, GridDev<R>* out);

}  // namespace pi
