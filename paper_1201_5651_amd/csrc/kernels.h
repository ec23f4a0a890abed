// kernels.h -- launch interface between the C-ABI runtime and the kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "physics.h"

namespace pi {

// Edge of the cubic tile of the raytrace wavefront (octant-local cells swept by
// one workgroup, one thread per cell).
constexpr int SWEEP_T = 8;
// Threads per workgroup of the micro-physics kernel.
constexpr int CHEM_BLOCK = 256;
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
    unsigned int fix_n;   // mixed precision: cells listed for the double re-solve
    unsigned int pad;
    double diag[8];   // see pi_diagnostics
};

// Micro-integration work counters (accepted, rejected substeps, fallback
// solves, Newton iterations), each spread over WORK_SLOTS slots so that the
// per-workgroup atomic additions do not all meet on one address; a reader sums
// the slots.  Layout: counter c, slot s at [c * WORK_SLOTS + s].
constexpr int WORK_COUNTERS = 5, WORK_SLOTS = 64;

template <typename R>
hipError_t launch_sweep_stage(const Params<R>& p, const R* nH, const R* x, R* tau,
                              const int4* tiles, int first, int count, hipStream_t s);
template <typename R>
hipError_t launch_chem(const Params<R>& p, const R* nH, const R* x0, const R* E0, const R* tau,
                       R* x1, R* E1, DevState* st, bool dev_dt, double hscale,
                       unsigned long long* ctr, int* fix_list, hipStream_t s);
// Mixed precision: double re-solve of the float cells listed by launch_chem
// (fix_list, count in st->fix_n), from the unmodified float inputs.
hipError_t launch_chem_fix(const Params<double>& p, const float* nH, const float* x0,
                           const float* E0, const float* tau, float* x1, float* E1,
                           DevState* st, bool dev_dt, double hscale, unsigned long long* ctr,
                           const int* fix_list, int nblk, hipStream_t s);
template <typename R>
hipError_t launch_dtdiag(const Params<R>& p, const R* nH, const R* x, const R* E, const R* tau,
                         double* part, int nblk, DevState* st, double t_end, double cell_vol,
                         int noct, hipStream_t s);
hipError_t launch_advance(DevState* st, hipStream_t s);
template <typename R>
hipError_t launch_energy(int64_t n, const R* nH, const R* x, R* E, double T0, hipStream_t s);

}  // namespace pi
