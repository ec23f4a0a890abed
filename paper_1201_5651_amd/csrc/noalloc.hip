// noalloc.hip -- pi_raytrace_static: the short-characteristics raytrace of a
// grid given only by its description and fields, allocating nothing.
//
// The raytrace kernels read a small device table (one entry per source) and
// a tile schedule (the tiles of every stage of the tile wavefront).  A grid
// made by pi_grid_create keeps both in buffers it allocates; here they live in
// `scratch`, a file-scope device array of fixed size that every call on a
// device shares.  A one-workgroup set-up kernel writes the table (passed to
// it by value) and builds the schedule into it, so no host-to-device copy and
// no allocation take place; then the same sweep kernels as pi_raytrace run,
// stage by stage, with tiles of edge 8.  Every cell's arithmetic is that of
// pi_raytrace, so the columns are bit for bit the same.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>
#include <string>

#include "../../include/pi.h"
#include "engine.h"
#include "kernels.h"

namespace pi {
namespace {

constexpr int STATIC_TILE = 8;                     // tile edge of the schedule
constexpr int STATIC_SWEEP = 1;                    // its index in SWEEP_TILES
static_assert(SWEEP_TILES[STATIC_SWEEP] == STATIC_TILE, "tile edge of the static raytrace");
constexpr int STATIC_MAX_TILES = 262144;           // e.g. 512^3 cells, one source
constexpr int STATIC_MAX_STAGES = 4096;            // tile diagonals of the schedule
constexpr size_t STATIC_TABLE_BYTES = 16384;       // grid table and row offsets
constexpr size_t STATIC_BYTES = STATIC_TABLE_BYTES + sizeof(int4) * (size_t)STATIC_MAX_TILES;
constexpr size_t ROWS_OFFSET = STATIC_TABLE_BYTES - 256;
static_assert(sizeof(GridDev<double>) * MAX_SRC <= ROWS_OFFSET, "grid table fits its part");

// The scratch of every device the library runs on (each holds its own copy
// until the process ends).  Host code must not use this name as an address:
// it takes the device address from hipGetSymbolAddress (scratch_of).
static __device__ __align__(256) unsigned char scratch[STATIC_BYTES];

constexpr int MAX_DEVICES = 64;
std::mutex g_mu;
unsigned char* g_scratch[MAX_DEVICES] = {};

// Device address of `scratch` on the current device, taken once per device.
pi_status scratch_of(unsigned char** out)
{
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0) return fail(PI_EDEVICE, "no current device");
    if (dev >= MAX_DEVICES) return fail(PI_EDEVICE, "device index beyond the static scratch table");
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_scratch[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(PI_EDEVICE, std::string("static scratch address: ") + hipGetErrorString(e));
        g_scratch[dev] = static_cast<unsigned char*>(p);
    }
    *out = g_scratch[dev];
    return PI_OK;
}

// Tiles of edge T of one raytrace entry whose octant-local indices sum to k
// (stage k); emit(octant, tx, ty, tz) is called for each, in a fixed order.
template <typename R, typename F>
__device__ int stage_tiles(const Params<R>& p, int T, int k, F emit)
{
    int count = 0;
    for (int o = 0; o < 8; ++o) {
        const int ex = (o & 1) ? p.nx - p.sx : p.sx;
        const int ey = (o & 2) ? p.ny - p.sy : p.sy;
        const int ez = (o & 4) ? p.nz - p.sz : p.sz;
        if (ex <= 0 || ey <= 0 || ez <= 0) continue;
        const int ntx = (ex + T - 1) / T, nty = (ey + T - 1) / T, ntz = (ez + T - 1) / T;
        for (int tx = 0; tx < ntx && tx <= k; ++tx)
            for (int ty = 0; ty < nty && tx + ty <= k; ++ty) {
                const int tz = k - tx - ty;
                if (tz < ntz) {
                    emit(o, tx, ty, tz);
                    ++count;
                }
            }
    }
    return count;
}

template <typename R> struct SetupArgs {
    GridDev<R> g[MAX_SRC];
    int nentries;   // raytrace entries (sources)
    int nstage;     // stages of the schedule
    int rows;       // rows along x of a plane-parallel grid (0 for point sources)
};
// passed by value: within the kernel-argument limit
static_assert(sizeof(SetupArgs<double>) + sizeof(void*) <= 4096, "set-up arguments too large");

// One workgroup: copies the grid table into the scratch, the row offsets of
// a plane-parallel grid, and builds the schedule -- stage by stage, the
// tiles of every entry with that tile diagonal -- by the enumeration the host
// uses for the launches.
template <typename R>
__global__ void __launch_bounds__(256) k_static_setup(SetupArgs<R> a, unsigned char* base)
{
    __shared__ int s_first[STATIC_MAX_STAGES];
    GridDev<R>* gd = reinterpret_cast<GridDev<R>*>(base);
    for (int i = threadIdx.x; i < a.nentries; i += blockDim.x) gd[i] = a.g[i];
    int* rowf = reinterpret_cast<int*>(base + ROWS_OFFSET);
    if (threadIdx.x == 0) {
        rowf[0] = 0;
        rowf[1] = a.rows;
    }
    for (int k = threadIdx.x; k < a.nstage; k += blockDim.x) {
        int c = 0;
        for (int r = 0; r < a.nentries; ++r)
            c += stage_tiles(a.g[r].p, STATIC_TILE, k, [](int, int, int, int) {});
        s_first[k] = c;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        int run = 0;
        for (int k = 0; k < a.nstage; ++k) {
            const int c = s_first[k];
            s_first[k] = run;
            run += c;
        }
    }
    __syncthreads();
    int4* tiles = reinterpret_cast<int4*>(base + STATIC_TABLE_BYTES);
    for (int k = threadIdx.x; k < a.nstage; k += blockDim.x) {
        int at = s_first[k];
        for (int r = 0; r < a.nentries; ++r)
            stage_tiles(a.g[r].p, STATIC_TILE, k, [&](int o, int tx, int ty, int tz) {
                tiles[at++] = make_int4((r << 3) | o, tx, ty, tz);
            });
    }
}

template <typename R>
pi_status raytrace_static_t(const pi_grid_desc& d, const pi_fields& f, int state, int tau_buf,
                            hipStream_t s)
{
    SetupArgs<R> a{};
    a.nentries = raytrace_entries<R>(d, f, a.g);
    const bool plane = d.source == PI_SRC_PLANE;
    a.rows = plane ? d.n[1] * d.n[2] : 0;
    // the schedule's stages and their sizes, as the set-up kernel builds it
    int nstage = 0;
    if (!plane)
        for (int r = 0; r < a.nentries; ++r) {
            const Params<R>& p = a.g[r].p;
            for (int o = 0; o < 8; ++o) {
                const int ex = (o & 1) ? p.nx - p.sx : p.sx;
                const int ey = (o & 2) ? p.ny - p.sy : p.sy;
                const int ez = (o & 4) ? p.nz - p.sz : p.sz;
                if (ex <= 0 || ey <= 0 || ez <= 0) continue;
                const int T = STATIC_TILE;
                const int64_t st = (int64_t)(ex + T - 1) / T + (ey + T - 1) / T + (ez + T - 1) / T - 2;
                if (st > STATIC_MAX_STAGES)
                    return fail(PI_EINVAL, "pi_raytrace_static: " + std::to_string(st) +
                                               " tile stages exceed the static limit of " +
                                               std::to_string(STATIC_MAX_STAGES));
                nstage = std::max(nstage, (int)st);
            }
        }
    a.nstage = nstage;
    // tiles in all, then per stage (tile diagonal tx + ty + tz)
    const int T = STATIC_TILE;
    int64_t total = 0;
    int count[STATIC_MAX_STAGES] = {};
    for (int pass = 0; pass < 2 && !plane; ++pass)
        for (int r = 0; r < a.nentries; ++r) {
            const Params<R>& p = a.g[r].p;
            for (int o = 0; o < 8; ++o) {
                const int ex = (o & 1) ? p.nx - p.sx : p.sx;
                const int ey = (o & 2) ? p.ny - p.sy : p.sy;
                const int ez = (o & 4) ? p.nz - p.sz : p.sz;
                if (ex <= 0 || ey <= 0 || ez <= 0) continue;
                const int ntx = (ex + T - 1) / T, nty = (ey + T - 1) / T, ntz = (ez + T - 1) / T;
                if (pass == 0) {
                    total += (int64_t)ntx * nty * ntz;
                    continue;
                }
                for (int tx = 0; tx < ntx; ++tx)
                    for (int ty = 0; ty < nty; ++ty)
                        for (int tz = 0; tz < ntz; ++tz) ++count[tx + ty + tz];
            }
            if (pass == 0 && total > STATIC_MAX_TILES)
                return fail(PI_EINVAL, "pi_raytrace_static: " + std::to_string(total) +
                                           "+ tiles of edge 8 exceed the static limit of " +
                                           std::to_string(STATIC_MAX_TILES));
        }
    unsigned char* base = nullptr;
    pi_status r = scratch_of(&base);
    if (r != PI_OK) return r;
    hipLaunchKernelGGL((k_static_setup<R>), dim3(1), dim3(256), 0, s, a, base);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(PI_EDEVICE, std::string("set-up launch: ") + hipGetErrorString(e));
    const GridDev<R>* gd = reinterpret_cast<const GridDev<R>*>(base);
    if (plane) {
        BatchDev b{};
        b.ngrids = 1;
        b.row_first = reinterpret_cast<const int*>(base + ROWS_OFFSET);
        e = launch_plane_scan<R>(gd, b, a.rows, state, tau_buf, s);
    } else {
        const int4* tiles = reinterpret_cast<const int4*>(base + STATIC_TABLE_BYTES);
        int first = 0;
        for (int k = 0; k < nstage && e == hipSuccess; ++k) {
            e = launch_sweep_stage<R>(gd, state, tau_buf, tiles, first, count[k], STATIC_TILE, s);
            first += count[k];
        }
    }
    if (e != hipSuccess) return fail(PI_EDEVICE, std::string("raytrace launch: ") + hipGetErrorString(e));
    return PI_OK;
}

}  // namespace
}  // namespace pi

using namespace pi;

extern "C" pi_status pi_raytrace_static(const pi_grid_desc* desc, const pi_fields* fields,
                                        int state, int tau_buf, void* stream)
{
    pi_status v = validate_desc(desc);
    if (v != PI_OK) return v;
    if ((v = validate_fields(desc, fields)) != PI_OK) return v;
    if ((state != PI_BUF_N && state != PI_BUF_HALF) || (tau_buf != PI_BUF_N && tau_buf != PI_BUF_HALF))
        return fail(PI_EINVAL, "buffer selector");
    hipStream_t s = static_cast<hipStream_t>(stream);
    return desc->precision == PI_FP64
               ? raytrace_static_t<double>(*desc, *fields, state, tau_buf, s)
               : raytrace_static_t<float>(*desc, *fields, state, tau_buf, s);
}
