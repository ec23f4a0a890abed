// kernels.hip -- gfx950 kernels of the photoionisation source-term step and
// their launchers.
//
//  k_sweep     short-characteristics raytrace of one tile-wavefront stage
//              (all octants at once), Sect. 2 and Sect. 5 of Mackey (A&A 2012)
//  k_chem      micro-physics of every cell over h on frozen columns (eq. 2)
//  k_dtdiag    per-cell timestep limit (eq. 4) and FP64 diagnostics,
//              reduced to per-block partials
//  k_finalize  fixed-order reduction of the partials; dt capped at t_end
//  k_advance   clock update at the end of a step
//  k_energy    internal energy from a uniform temperature
#include "kernels.h"

#include <hip/hip_runtime.h>

#include <type_traits>

namespace pi {

// ------------------------------------------------------------------ raytrace
// Thread -> cell map of a T^3 tile in diagonal-plane order (lx + ly + lz
// ascending), built at compile time: the cells of one plane are consecutive
// threads, so a plane occupies one or two wavefronts instead of one lane in
// each of T wavefronts.  Packed as lx | ly << 5 | lz << 10.
template <int T> struct PlaneOrder {
    unsigned short cell[T * T * T];
};

template <int T> constexpr PlaneOrder<T> make_plane_order()
{
    PlaneOrder<T> o{};
    int q = 0;
    for (int s = 0; s < 3 * T - 2; ++s)
        for (int lz = 0; lz < T; ++lz)
            for (int ly = 0; ly < T; ++ly) {
                const int lx = s - ly - lz;
                if (lx >= 0 && lx < T) o.cell[q++] = (unsigned short)(lx | ly << 5 | lz << 10);
            }
    return o;
}
static_assert(SWEEP_T_LARGEST <= 32, "tile coordinates are packed in 5 bits");

__constant__ PlaneOrder<SWEEP_TILES[0]> c_plane_order_0 = make_plane_order<SWEEP_TILES[0]>();
__constant__ PlaneOrder<SWEEP_TILES[1]> c_plane_order_1 = make_plane_order<SWEEP_TILES[1]>();
__constant__ PlaneOrder<SWEEP_TILES[2]> c_plane_order_2 = make_plane_order<SWEEP_TILES[2]>();

// Level order of a tile of edge PERSIST_TILE by its class.  Only the cells of
// one layer back along a cell's major axis feed it, so a cell's level -- one
// more than the highest level it reads inside the tile -- depends on which
// axes can be major in the tile, which the tile indices (tx, ty, tz) in the
// octant decide:
//   one index largest: every cell's major axis is that axis a, level = l_a
//     (PERSIST_TILE levels of T^2 cells);
//   two indices tie for largest: the major axis is one of those two, p and q,
//     and level = l_p + l_q (2T - 1 levels);
//   all three equal: the diagonal planes, level = lx + ly + lz (3T - 2).
// Cells of one level are independent, so a sweep by levels computes the same
// columns as one by diagonal planes, in fewer steps.  Classes 0-2: a = x, y,
// z; 3-5: the tied pair xy, yz, xz; 6: diagonal.  Every level lies in one
// group of 64 consecutive slots (a wavefront's lanes for the sweep kernels):
// single levels for the first classes, pairs of levels whose sizes add up to
// 64 for the second (sizes 8 min(l + 1, 15 - l) for T = 8).  Packed as
// lx | ly << 5 | lz << 10 | level << 15.
constexpr int LEVEL_CLASSES = 7;
struct LevelOrder {
    unsigned cell[LEVEL_CLASSES][PERSIST_TILE * PERSIST_TILE * PERSIST_TILE];
};
constexpr LevelOrder make_level_order()
{
    constexpr int T = PERSIST_TILE;
    static_assert(T == 8, "the level pairing below is that of 8^3 tiles");
    LevelOrder o{};
    for (int a = 0; a < 3; ++a) {
        // one major axis: level la, lanes over the two other axes (lower one fastest)
        const int b = a == 0 ? 1 : 0, c = a == 2 ? 1 : 2;
        int q = 0;
        for (int la = 0; la < T; ++la)
            for (int lc = 0; lc < T; ++lc)
                for (int lb = 0; lb < T; ++lb) {
                    int L[3] = { 0, 0, 0 };
                    L[a] = la;
                    L[b] = lb;
                    L[c] = lc;
                    o.cell[a][q++] = (unsigned)(L[0] | L[1] << 5 | L[2] << 10 | la << 15);
                }
    }
    const int groups[8][2] = { { 7, -1 }, { 0, 6 }, { 1, 5 }, { 2, 4 },
                               { 3, 11 }, { 8, 14 }, { 9, 13 }, { 10, 12 } };
    for (int t = 0; t < 3; ++t) {
        // tied pair (p, q), the third axis r
        const int p = t == 2 ? 0 : t, qx = t == 2 ? 2 : t + 1, r = 3 - p - qx;
        int n = 0;
        for (int g = 0; g < 8; ++g)
            for (int h = 0; h < 2; ++h) {
                const int lev = groups[g][h];
                if (lev < 0) continue;
                for (int lr = 0; lr < T; ++lr)
                    for (int lp = 0; lp < T; ++lp) {
                        const int lq = lev - lp;
                        if (lq < 0 || lq >= T) continue;
                        int L[3] = { 0, 0, 0 };
                        L[p] = lp;
                        L[qx] = lq;
                        L[r] = lr;
                        o.cell[3 + t][n++] = (unsigned)(L[0] | L[1] << 5 | L[2] << 10 | lev << 15);
                    }
            }
    }
    int n = 0;
    for (int sd = 0; sd < 3 * T - 2; ++sd)
        for (int lz = 0; lz < T; ++lz)
            for (int ly = 0; ly < T; ++ly) {
                const int lx = sd - ly - lz;
                if (lx >= 0 && lx < T)
                    o.cell[6][n++] = (unsigned)(lx | ly << 5 | lz << 10 | sd << 15);
            }
    return o;
}
// First slot of every level in the level order of each class: the level's
// cells lie in the 64 slots from there (-1 for a level the class lacks).
struct LevelStart {
    short first[LEVEL_CLASSES][3 * PERSIST_TILE - 2];
};
constexpr LevelStart make_level_start()
{
    constexpr int N = PERSIST_TILE * PERSIST_TILE * PERSIST_TILE;
    const LevelOrder o = make_level_order();
    LevelStart w{};
    for (int c = 0; c < LEVEL_CLASSES; ++c) {
        for (int l = 0; l < 3 * PERSIST_TILE - 2; ++l) w.first[c][l] = -1;
        for (int i = 0; i < N; ++i) {
            const int l = (int)(o.cell[c][i] >> 15);
            if (w.first[c][l] < 0) w.first[c][l] = (short)i;
        }
    }
    return w;
}
__constant__ LevelOrder c_level_order = make_level_order();
__constant__ LevelStart c_level_start = make_level_start();

// Class of a tile for c_level_order from its indices in the octant, and its
// number of levels.
__device__ __forceinline__ int level_class(int tx, int ty, int tz, int& nlev)
{
    const int m = max(tx, max(ty, tz));
    const int top = (tx == m) + (ty == m) + (tz == m);
    nlev = top == 1 ? PERSIST_TILE : (top == 2 ? 2 * PERSIST_TILE - 1 : 3 * PERSIST_TILE - 2);
    if (top == 1) return tx == m ? 0 : (ty == m ? 1 : 2);
    if (top == 2) return tz != m ? 3 : (tx != m ? 4 : 5);
    return 6;
}

// Entries of the (T+1)^3 halo buffer of a T^3 tile that lie on its upstream
// faces (local index -1 along some axis), in buffer order: the halo cells a
// tile reads from earlier tiles, one per thread of every sweep kernel.
template <int T> struct FaceList {
    static constexpr int N = (T + 1) * (T + 1) * (T + 1) - T * T * T;
    unsigned short q[N];
};
template <int T> constexpr FaceList<T> make_face_list()
{
    FaceList<T> o{};
    int n = 0;
    for (int q = 0; q < (T + 1) * (T + 1) * (T + 1); ++q) {
        const int hx = q % (T + 1), hy = (q / (T + 1)) % (T + 1), hz = q / ((T + 1) * (T + 1));
        if (hx == 0 || hy == 0 || hz == 0) o.q[n++] = (unsigned short)q;
    }
    return o;
}
__constant__ FaceList<SWEEP_TILES[0]> c_faces_0 = make_face_list<SWEEP_TILES[0]>();
__constant__ FaceList<SWEEP_TILES[1]> c_faces_1 = make_face_list<SWEEP_TILES[1]>();
__constant__ FaceList<SWEEP_TILES[2]> c_faces_2 = make_face_list<SWEEP_TILES[2]>();
template <int T> __device__ __forceinline__ int face_entry(int f);
template <> __device__ __forceinline__ int face_entry<SWEEP_TILES[0]>(int f)
{
    return c_faces_0.q[f];
}
template <> __device__ __forceinline__ int face_entry<SWEEP_TILES[1]>(int f)
{
    return c_faces_1.q[f];
}
template <> __device__ __forceinline__ int face_entry<SWEEP_TILES[2]>(int f)
{
    return c_faces_2.q[f];
}

template <int T> __device__ __forceinline__ int plane_cell(int t);
template <> __device__ __forceinline__ int plane_cell<SWEEP_TILES[0]>(int t)
{
    return c_plane_order_0.cell[t];
}
template <> __device__ __forceinline__ int plane_cell<SWEEP_TILES[1]>(int t)
{
    return c_plane_order_1.cell[t];
}
template <> __device__ __forceinline__ int plane_cell<SWEEP_TILES[2]>(int t)
{
    return c_plane_order_2.cell[t];
}

// Weighted upstream average of the short-characteristics interpolation:
// sum w_i T_i / sum w_i with w_i = g_i (Mellema: divided by max(0.6, T_i)).
template <typename R>
__device__ __forceinline__ R sc_average(bool mellema, R g00, R g10, R g01, R g11, R T00, R T10,
                                        R T01, R T11)
{
    R w00 = g00, w10 = g10, w01 = g01, w11 = g11;
    if (mellema) {
        w00 = g00 * r_rcp(r_max(R(W_FLOOR), T00));
        w10 = g10 * r_rcp(r_max(R(W_FLOOR), T10));
        w01 = g01 * r_rcp(r_max(R(W_FLOOR), T01));
        w11 = g11 * r_rcp(r_max(R(W_FLOOR), T11));
    }
    return (w00 * T00 + w10 * T10 + w01 * T01 + w11 * T11) * r_rcp(w00 + w10 + w01 + w11);
}
// double keeps the divisions of the definition
template <>
__device__ __forceinline__ double sc_average<double>(bool mellema, double g00, double g10,
                                                     double g01, double g11, double T00,
                                                     double T10, double T01, double T11)
{
    double w00 = g00, w10 = g10, w01 = g01, w11 = g11;
    if (mellema) {
        w00 /= fmax(W_FLOOR, T00);
        w10 /= fmax(W_FLOOR, T10);
        w01 /= fmax(W_FLOOR, T01);
        w11 /= fmax(W_FLOOR, T11);
    }
    return (w00 * T00 + w10 * T10 + w01 * T01 + w11 * T11) / (w00 + w10 + w01 + w11);
}

// One tile-diagonal stage of the octant sweeps of every grid of a batch.  Each
// workgroup owns one TX*TY*TZ tile of one octant of one grid (one thread per
// cell) and needs only the tiles of earlier stages, so a stage is one launch.  The tile's cells and its
// upstream halo (octant-local index -1 on any axis) are staged in LDS as
//   s_kap: sigma0 n_H x dx (optical depth per cell length),
//   s_tc : optical depth from the source to the cell centre (halo only, from
//          the stored entering depth of the earlier stage);
// the tile is then swept level by level: a tile of edge PERSIST_TILE in the
// level order of its class (c_level_order), other edges diagonal plane by
// diagonal plane, lx+ly+lz = s.
//
// A cell C with dominant axis a interpolates, on the plane through the centres
// of the layer one step back along a, the four upstream centres around the
// point where the ray to C crosses that plane (offsets ad_b/ad_a in (0, 1]);
// each carries T = tau_centre + (ds_C/2) kap, its depth at C's entry face, with
// bilinear weights divided by max(0.6, T) (Mellema weighting).  Neighbours
// across a source plane (octant-local index -1) get weight 0.
// Threads of the sweep workgroup for tile edge TT: one per cell up to 1024,
// then several cells per thread (consecutive planes or levels are whole thread
// ranges, and none exceeds the thread count, so a thread owns at most one cell
// of any of them).
template <int TT> struct SweepShape {
    static constexpr int CELLS = TT * TT * TT;
    static constexpr int THREADS = CELLS < 1024 ? CELLS : 1024;
    static constexpr int CPT = CELLS / THREADS;
};

// Quotient num / den of the sweep geometry.  Float: the hardware reciprocal
// and one correction by a fused multiply-add, within rounding of the divided
// quotient and exactly 1 when num == den (the residual num - q den is then
// exact); double: the division.
template <typename R> __device__ __forceinline__ R geom_quot(R num, R den);
template <> __device__ __forceinline__ double geom_quot<double>(double num, double den)
{
    return num / den;
}
template <> __device__ __forceinline__ float geom_quot<float>(float num, float den)
{
    const float r = __builtin_amdgcn_rcpf(den);
    const float q = num * r;
    return __builtin_fmaf(__builtin_fmaf(-q, den, num), r, q);
}

// Half path length per cell length through the cell whose centre sits at
// offsets (ax, ay, az) from the source vertex, da the largest of them:
// sqrt(ax^2 + ay^2 + az^2) / (2 da), with the same operations (no
// contraction) wherever a sweep needs it.
template <typename R> __device__ __forceinline__ R half_path(R ax, R ay, R az, R da)
{
#pragma clang fp contract(off)
    return geom_quot<R>(R(0.5) * r_sqrt(ax * ax + ay * ay + az * az), da);
}

// Short-characteristics geometry of a cell at octant-local coordinates L
// (Sect. 2.1): the major axis a of the ray from the source vertex to the cell
// centre and the two others (b, c); the bilinear weights of the four upstream
// centres on the plane one step back along a (zero across a source plane);
// the half path length per cell length, hds; and whether the cell lies on the
// source plane normal to a (corner: no upstream cells).  Every sweep kernel
// takes it from here, so all of them compute it with the same operations.
template <typename R> struct ScGeom {
    int a, b, c;
    R g00, g10, g01, g11, hds;
    bool corner;
};
template <typename R> __device__ __forceinline__ ScGeom<R> sc_geom(const int L[3])
{
    ScGeom<R> o;
    const R ad[3] = { R(L[0]) + R(0.5), R(L[1]) + R(0.5), R(L[2]) + R(0.5) };
    o.a = (ad[2] >= ad[0] && ad[2] >= ad[1]) ? 2 : (ad[1] >= ad[0] ? 1 : 0);
    o.b = o.a == 2 ? 0 : o.a + 1;
    o.c = o.a == 0 ? 2 : o.a - 1;
    // a tie of axes gives a quotient of exactly 1 (zero weights stay zero)
    const R fb = geom_quot<R>(ad[o.b], ad[o.a]), fc = geom_quot<R>(ad[o.c], ad[o.a]);
    const bool vb = L[o.b] >= 1, vc = L[o.c] >= 1;
    o.g00 = (R(1) - fb) * (R(1) - fc);
    o.g10 = vb ? fb * (R(1) - fc) : R(0);
    o.g01 = vc ? (R(1) - fb) * fc : R(0);
    o.g11 = (vb && vc) ? fb * fc : R(0);
    o.hds = half_path<R>(ad[0], ad[1], ad[2], ad[o.a]);
    o.corner = L[o.a] == 0;
    return o;
}

// Depth of an upstream centre column tc at the entry face of the cell, tc +
// hds kap, with the product rounded on its own (no contraction), as in every
// sweep kernel.
template <typename R> __device__ __forceinline__ R upstream_T(R tc, R hds, R kap)
{
#pragma clang fp contract(off)
    return tc + hds * kap;
}

// Half path length per cell length of the halo cell at octant-local L (its
// centre column from its entering one: tc = tin + hh kap).
template <typename R> __device__ __forceinline__ R halo_hds(int Lx, int Ly, int Lz)
{
    const R ax = R(Lx) + R(0.5), ay = R(Ly) + R(0.5), az = R(Lz) + R(0.5);
    const R da = (az >= ax && az >= ay) ? az : (ay >= ax ? ay : ax);
    return half_path<R>(ax, ay, az, da);
}

// Kinds of tile sweep.  TILE_STAGED: every upstream tile belongs to an
// earlier launch; the halo's sigma0 n_H x dx and columns are read from the
// grid.  TILE_COHERENT: upstream tiles run in the same launch.  A finished
// tile publishes sigma0 n_H x dx and the centre column of the cells on its
// three downstream faces in its slot of a face buffer (FACE_WORDS entries per
// tile), written and read as relaxed atomics at agent scope (loads and stores
// that reach the device-wide point of coherence, past the caches of the
// compute unit and of its XCD); a tile takes its halo from the slots of the
// up to seven upstream tiles that own it -- contiguous rows instead of
// scattered cells -- and writes its columns to the grid with plain stores.
// The published values are those a halo read from the grid would form.  A
// float entry carries the epoch of the launch that wrote it (FaceWord), so
// the reader polls the entries themselves; double tiles wait for the
// upstream tiles' done-flags first.
// TILE_FUSED: as TILE_COHERENT, after the tile's own micro-physics in the
// same workgroup, which has put sigma0 n_H x dx of the tile's own cells in
// s_kap.
enum { TILE_STAGED = 0, TILE_COHERENT = 1, TILE_FUSED = 2 };

// Entry of the face buffer: for float, one 64-bit word holding the value's
// bits in its lower half and the epoch of the launch that wrote it in its
// upper half, written and read whole, so that a reader tells a current entry
// from one of an earlier launch without a flag; for double, the value (its
// sweeps order the entries with done-flags).  Eight bytes either way.
template <typename R> struct FaceWord {
    using type = double;
    static constexpr bool tagged = false;
};
template <> struct FaceWord<float> {
    using type = unsigned long long;
    static constexpr bool tagged = true;
};
template <typename R> using face_t = typename FaceWord<R>::type;
static_assert(sizeof(face_t<float>) == FACE_BYTES && sizeof(face_t<double>) == FACE_BYTES,
              "face buffer entries are FACE_BYTES wide");

// Face buffer slot of a tile of edge T: for the faces at local x, y, z =
// T - 1 in turn, T^2 values of sigma0 n_H x dx and then T^2 centre columns,
// the face's cells in order (ly, lz), (lx, lz), (lx, ly) with the first index
// fastest.
template <int T> struct FaceSlot {
    static constexpr int WORDS = 6 * T * T;
    __host__ __device__ static constexpr int kap(int face, int i, int j) { return (2 * face) * T * T + j * T + i; }
    __host__ __device__ static constexpr int col(int face, int i, int j) { return (2 * face + 1) * T * T + j * T + i; }
};

// The sweep of one tile by NT threads (the body of the tiled raytrace
// kernels), with the LDS arrays of the workgroup.  wait() runs between the
// work that does not depend on earlier tiles (sigma0 n_H x dx of the tile --
// and for TILE_STAGED of its halo -- and the cells' geometry) and the loads
// that do (the halo); every thread calls it, and the caller's
// synchronisation follows it.  For the coherent kinds, fbuf is the face
// buffer, idx the tile's flag (and slot) index and oc its octant's (first
// flag, tiles along x, y, z); done is the launch's epoch, which float entries
// are tagged with and polled for, at most spin_ticks of the 100 MHz clock
// before ctl->err is set.
template <typename R, int TT, int NT, int Kind, typename Wait>
__device__ __forceinline__ void sweep_tile(const GridDev<R>* __restrict__ grids, int state,
                                           int tau_buf, int4 tl, R* s_tc, R* s_kap, Wait wait,
                                           face_t<R>* fbuf = nullptr, int idx = 0,
                                           int4 oc = int4{}, unsigned done = 0u,
                                           long long spin_ticks = 0, SweepCtl* ctl = nullptr)
{
    constexpr int TX = TT, TY = TT, TZ = TT;
    constexpr int CPT = TT * TT * TT / NT;
    static_assert(CPT * NT == TT * TT * TT, "whole cells per thread");
    constexpr int HX = TX + 1, HY = TY + 1, HZ = TZ + 1, NHALO = HX * HY * HZ;
    const GridDev<R>& G = grids[tl.x >> 3];
    const Params<R> p = G.p;
    const R* __restrict__ nH = G.nHr[state];
    const R* __restrict__ xs = G.x[state];
    R* __restrict__ tau = G.tau[tau_buf];
    const int oct = tl.x & 7;
    const bool px = oct & 1, py = oct & 2, pz = oct & 4;
    const int ex = px ? p.nx - p.sx : p.sx;
    const int ey = py ? p.ny - p.sy : p.sy;
    const int ez = pz ? p.nz - p.sz : p.sz;
    const int X0 = tl.y * TX, Y0 = tl.z * TY, Z0 = tl.w * TZ;

    if constexpr (Kind == TILE_STAGED) {
        // the tile and its halo (a fixed trip count, so that every
        // iteration's loads are in flight together)
#pragma unroll
        for (int k = 0; k < (NHALO + NT - 1) / NT; ++k) {
            const int q = threadIdx.x + k * NT;
            if (q >= NHALO) break;
            const int hx = q % HX, hy = (q / HX) % HY, hz = q / (HX * HY);
            const int Lx = X0 + hx - 1, Ly = Y0 + hy - 1, Lz = Z0 + hz - 1;
            R kap = R(0);
            if (Lx >= 0 && Ly >= 0 && Lz >= 0 && Lx < ex && Ly < ey && Lz < ez) {
                const int gi = px ? p.sx + Lx : p.sx - 1 - Lx;
                const int gj = py ? p.sy + Ly : p.sy - 1 - Ly;
                const int gk = pz ? p.sz + Lz : p.sz - 1 - Lz;
                const int64_t g = gi + (int64_t)p.nx * (gj + (int64_t)p.ny * gk);
                kap = p.sdx * nH[g] * xs[g];
            }
            s_kap[q] = kap;
        }
    } else if constexpr (Kind == TILE_COHERENT) {
        // the tile's own cells (its halo comes from the face buffer)
#pragma unroll
        for (int k = 0; k < TX * TY * TZ / NT; ++k) {
            const int t = threadIdx.x + k * NT;
            const int ox = t % TX, oy = (t / TX) % TY, oz = t / (TX * TY);
            const int Lx = X0 + ox, Ly = Y0 + oy, Lz = Z0 + oz;
            R kap = R(0);
            if (Lx < ex && Ly < ey && Lz < ez) {
                const int gi = px ? p.sx + Lx : p.sx - 1 - Lx;
                const int gj = py ? p.sy + Ly : p.sy - 1 - Ly;
                const int gk = pz ? p.sz + Lz : p.sz - 1 - Lz;
                const int64_t g = gi + (int64_t)p.nx * (gj + (int64_t)p.ny * gk);
                kap = p.sdx * nH[g] * xs[g];
            }
            s_kap[(oz + 1) * HX * HY + (oy + 1) * HX + (ox + 1)] = kap;
        }
    }

    // the halo entries of the coherent kinds: every halo entry of the thread
    // comes from the slot of its owner -- the upstream tile across every face
    // the entry lies on -- at the owner's local coordinates and on the owner's
    // face that holds it; all loads in flight together.  Tagged entries tell a
    // current value from a stale one themselves, so after a tile's own
    // micro-physics (whose upstream tiles have mostly finished by then) their
    // loads are issued before the geometry below and arrive while it is
    // formed; a bare sweep, which mostly finds its upstream tiles still
    // running, and untagged entries (read only after wait() has seen the
    // owners' done-flags) load them after it.
    constexpr int NFACE = FaceList<TT>::N, KF = (NFACE + NT - 1) / NT;
    constexpr bool early = Kind == TILE_FUSED && FaceWord<R>::tagged;
    int qf[KF];
    const face_t<R>* pk[KF];
    const face_t<R>* pc[KF];
    face_t<R> wk[KF], wc[KF];
    auto face_loads = [&]() {
#pragma unroll
        for (int k = 0; k < KF; ++k) {
            const int f = threadIdx.x + k * NT;
            qf[k] = -1;
            pk[k] = pc[k] = nullptr;
            wk[k] = wc[k] = face_t<R>(0);
            if (f < NFACE) {
                const int q = face_entry<TT>(f);
                qf[k] = q;
                const int hx = q % HX, hy = (q / HX) % HY, hz = q / (HX * HY);
                const int Lx = X0 + hx - 1, Ly = Y0 + hy - 1, Lz = Z0 + hz - 1;
                if (Lx >= 0 && Ly >= 0 && Lz >= 0 && Lx < ex && Ly < ey && Lz < ez) {
                    const int ux = hx == 0, uy = hy == 0, uz = hz == 0;
                    const int owner = idx - ux - uy * oc.y - uz * oc.y * oc.z;
                    const int ox = ux ? TT - 1 : hx - 1, oy = uy ? TT - 1 : hy - 1;
                    const int oz = uz ? TT - 1 : hz - 1;
                    const int face = ux ? 0 : (uy ? 1 : 2);
                    const int i = face == 0 ? oy : ox, j = face == 2 ? oy : oz;
                    const face_t<R>* slot = fbuf + (int64_t)owner * FaceSlot<TT>::WORDS;
                    pk[k] = &slot[FaceSlot<TT>::kap(face, i, j)];
                    pc[k] = &slot[FaceSlot<TT>::col(face, i, j)];
                    wk[k] = __hip_atomic_load(pk[k], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    wc[k] = __hip_atomic_load(pc[k], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                }
            }
        }
    };
    if constexpr (early) face_loads();

    // geometry of the thread's cells (cell k: index threadIdx.x + k NT of the
    // tile's level order, or of the diagonal-plane order for other edges)
    const bool mellema = p.weights == 1;
    int nlev = TX + TY + TZ - 2;
    int cls = 0;
    if constexpr (TT == PERSIST_TILE) cls = level_class(tl.y, tl.z, tl.w, nlev);
    int self[CPT], n00[CPT], n10[CPT], n01[CPT], n11[CPT], lev[CPT], nat[CPT];
    bool active[CPT], corner[CPT];
    R g00[CPT], g10[CPT], g01[CPT], g11[CPT], hds[CPT], tin[CPT];
#pragma unroll
    for (int k = 0; k < CPT; ++k) {
        int cl;
        if constexpr (TT == PERSIST_TILE) {
            cl = (int)c_level_order.cell[cls][threadIdx.x + k * NT];
        } else {
            cl = plane_cell<TT>(threadIdx.x + k * NT);
        }
        const int lx = cl & 31, ly = (cl >> 5) & 31, lz = (cl >> 10) & 31;
        const int L[3] = { X0 + lx, Y0 + ly, Z0 + lz };
        active[k] = L[0] < ex && L[1] < ey && L[2] < ez;
        const ScGeom<R> sg = sc_geom<R>(L);
        const int st[3] = { 1, HX, HX * HY };
        self[k] = (lz + 1) * HX * HY + (ly + 1) * HX + (lx + 1);
        n00[k] = self[k] - st[sg.a];
        n10[k] = n00[k] - st[sg.b];
        n01[k] = n00[k] - st[sg.c];
        n11[k] = n10[k] - st[sg.c];
        g00[k] = sg.g00;
        g10[k] = sg.g10;
        g01[k] = sg.g01;
        g11[k] = sg.g11;
        hds[k] = sg.hds;
        corner[k] = sg.corner;
        lev[k] = TT == PERSIST_TILE ? cl >> 15 : lx + ly + lz;
        nat[k] = lx + TX * (ly + TY * lz);
        tin[k] = R(0);
    }
    if constexpr (early) {
        // the geometry is formed here, while the halo loads are in flight (the
        // compiler would otherwise defer it past the halo's arrival)
#pragma unroll
        for (int k = 0; k < CPT; ++k)
            asm volatile("" ::"v"(g00[k]), "v"(g10[k]), "v"(g01[k]), "v"(g11[k]), "v"(hds[k]));
    }

    wait();
    __syncthreads();
    // the upstream halo (the faces at local index -1): centre columns and,
    // for the coherent kinds, sigma0 n_H x dx; the tile's own entries of s_tc
    // are written by their cells before any cell reads them
    if constexpr (Kind == TILE_STAGED) {
#pragma unroll
        for (int k = 0; k < KF; ++k) {
            const int f = threadIdx.x + k * NT;
            if (f >= NFACE) break;
            const int q = face_entry<TT>(f);
            const int hx = q % HX, hy = (q / HX) % HY, hz = q / (HX * HY);
            const int Lx = X0 + hx - 1, Ly = Y0 + hy - 1, Lz = Z0 + hz - 1;
            R tc = R(0);
            if (Lx >= 0 && Ly >= 0 && Lz >= 0 && Lx < ex && Ly < ey && Lz < ez) {
                const int gi = px ? p.sx + Lx : p.sx - 1 - Lx;
                const int gj = py ? p.sy + Ly : p.sy - 1 - Ly;
                const int gk = pz ? p.sz + Lz : p.sz - 1 - Lz;
                const int64_t g = gi + (int64_t)p.nx * (gj + (int64_t)p.ny * gk);
                // the centre column exactly as the cell's own tile formed it
                tc = r_fma(halo_hds<R>(Lx, Ly, Lz), s_kap[q], tau[g]);
            }
            s_tc[q] = tc;
        }
    } else {
        if constexpr (!early) face_loads();
        if constexpr (FaceWord<R>::tagged) {
            // an entry still of an earlier launch is polled until its owner
            // writes it (each lane for its own entries; the owners are held by
            // running workgroups)
            auto stale = [&](face_t<R> w) { return (unsigned)(w >> 32) != done; };
            bool pending = false;
#pragma unroll
            for (int k = 0; k < KF; ++k)
                pending |= pk[k] != nullptr && (stale(wk[k]) || stale(wc[k]));
            if (pending) {
                const long long t0 = (long long)__builtin_amdgcn_s_memrealtime();
                while (pending) {
                    if ((long long)__builtin_amdgcn_s_memrealtime() - t0 > spin_ticks) {
                        __hip_atomic_store(&ctl->err, 1u, __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_AGENT);
                        break;
                    }
                    __builtin_amdgcn_s_sleep(1);
                    pending = false;
#pragma unroll
                    for (int k = 0; k < KF; ++k) {
                        if (pk[k] == nullptr) continue;
                        if (stale(wk[k]))
                            wk[k] = __hip_atomic_load(pk[k], __ATOMIC_RELAXED,
                                                      __HIP_MEMORY_SCOPE_AGENT);
                        if (stale(wc[k]))
                            wc[k] = __hip_atomic_load(pc[k], __ATOMIC_RELAXED,
                                                      __HIP_MEMORY_SCOPE_AGENT);
                        pending |= stale(wk[k]) || stale(wc[k]);
                    }
                }
            }
        }
#pragma unroll
        for (int k = 0; k < KF; ++k) {
            if (qf[k] < 0) continue;
            if constexpr (FaceWord<R>::tagged) {
                s_kap[qf[k]] = __uint_as_float((unsigned)wk[k]);
                s_tc[qf[k]] = __uint_as_float((unsigned)wc[k]);
            } else {
                s_kap[qf[k]] = wk[k];
                s_tc[qf[k]] = wc[k];
            }
        }
    }
    __syncthreads();

    for (int s = 0; s < nlev; ++s) {
#pragma unroll
        for (int k = 0; k < CPT; ++k) {
            if (active[k] && lev[k] == s) {
                // every LDS value of the cell is read before any arithmetic, so
                // the reads share one round trip (the neighbour entries of a
                // corner cell lie in the halo buffer too; it discards them)
                const R c00 = s_tc[n00[k]], c10 = s_tc[n10[k]];
                const R c01 = s_tc[n01[k]], c11 = s_tc[n11[k]];
                const R k00 = s_kap[n00[k]], k10 = s_kap[n10[k]];
                const R k01 = s_kap[n01[k]], k11 = s_kap[n11[k]];
                const R kself = s_kap[self[k]];
                const R T00 = upstream_T(c00, hds[k], k00);
                const R T10 = upstream_T(c10, hds[k], k10);
                const R T01 = upstream_T(c01, hds[k], k01);
                const R T11 = upstream_T(c11, hds[k], k11);
                const R avg = sc_average<R>(mellema, g00[k], g10[k], g01[k], g11[k], T00, T10,
                                            T01, T11);
                tin[k] = corner[k] ? R(0) : avg;
                // entry face to centre
                s_tc[self[k]] = r_fma(hds[k], kself, tin[k]);
            }
        }
        __syncthreads();
    }
    if constexpr (Kind != TILE_STAGED) {
        // publish the downstream faces: entry (face, i, j) is the cell at local
        // TT - 1 along the face's axis (cells outside the octant give 0)
        face_t<R>* slot = fbuf + (int64_t)idx * FaceSlot<TT>::WORDS;
        for (int e = threadIdx.x; e < 3 * TT * TT; e += NT) {
            const int face = e / (TT * TT), i = e % TT, j = (e / TT) % TT;
            const int lx = face == 0 ? TT - 1 : i;
            const int ly = face == 0 ? i : (face == 1 ? TT - 1 : j);
            const int lz = face == 2 ? TT - 1 : j;
            const bool in = X0 + lx < ex && Y0 + ly < ey && Z0 + lz < ez;
            const int c = (lz + 1) * HX * HY + (ly + 1) * HX + (lx + 1);
            const R kv = in ? s_kap[c] : R(0), cv = in ? s_tc[c] : R(0);
            face_t<R> wk, wc;
            if constexpr (FaceWord<R>::tagged) {
                const face_t<R> tag = (face_t<R>)done << 32;
                wk = tag | __float_as_uint(kv);
                wc = tag | __float_as_uint(cv);
            } else {
                wk = kv;
                wc = cv;
            }
            __hip_atomic_store(&slot[FaceSlot<TT>::kap(face, i, j)], wk, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(&slot[FaceSlot<TT>::col(face, i, j)], wc, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
        }
        __syncthreads();   // (s_kap becomes the output buffer)
    }
    // entering columns back to natural order (in the halo buffer, no longer
    // read) for a coalesced store
    R* s_out = s_kap;
#pragma unroll
    for (int k = 0; k < CPT; ++k) s_out[nat[k]] = tin[k];
    __syncthreads();
    for (int t = threadIdx.x; t < TX * TY * TZ; t += NT) {
        const int ox = t % TX, oy = (t / TX) % TY, oz = t / (TX * TY);
        const int Lx = X0 + ox, Ly = Y0 + oy, Lz = Z0 + oz;
        if (Lx < ex && Ly < ey && Lz < ez) {
            const int gi = px ? p.sx + Lx : p.sx - 1 - Lx;
            const int gj = py ? p.sy + Ly : p.sy - 1 - Ly;
            const int gk = pz ? p.sz + Lz : p.sz - 1 - Lz;
            tau[gi + (int64_t)p.nx * (gj + (int64_t)p.ny * gk)] = s_out[t];
        }
    }
}

// One tile-diagonal stage of the octant sweeps of every grid of a batch: one
// workgroup per tile of the stage, all of whose upstream tiles belong to
// earlier launches.
template <typename R, int TT>
__global__ void __launch_bounds__(SweepShape<TT>::THREADS)
k_sweep(const GridDev<R>* __restrict__ grids, int state, int tau_buf,
        const int4* __restrict__ tiles, int first)
{
    constexpr int NHALO = (TT + 1) * (TT + 1) * (TT + 1);
    static_assert(NHALO >= TT * TT * TT, "the output reuses the halo buffer");
    __shared__ R s_tc[NHALO];
    __shared__ R s_kap[NHALO];
    sweep_tile<R, TT, SweepShape<TT>::THREADS, TILE_STAGED>(
        grids, state, tau_buf, tiles[first + blockIdx.x], s_tc, s_kap, [] {});
}

// Wait of a persistent tile (its first wavefront) for the flags of its upstream
// tiles to read `done`: lanes 0, 1 and 2 poll the tiles upstream along x, y
// and z (where there is one), so one round trip reads all three, and the loop
// is uniform over the wavefront.  After spin_ticks of the 100 MHz clock the
// error word is set and the wait gives up.
__device__ __forceinline__ void wait_upstream(const unsigned* __restrict__ flags, int idx, int4 tl,
                                              int4 oc, unsigned done, long long spin_ticks,
                                              SweepCtl* ctl)
{
    const int lane = threadIdx.x & 63;
    int up = -1;
    if (lane == 0 && tl.y > 0) up = idx - 1;
    if (lane == 1 && tl.z > 0) up = idx - oc.y;
    if (lane == 2 && tl.w > 0) up = idx - oc.y * oc.z;
    const long long t0 = (long long)__builtin_amdgcn_s_memrealtime();
    for (;;) {
        unsigned f = done;
        if (up >= 0) f = __hip_atomic_load(&flags[up], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (__ballot(f != done) == 0ull) break;
        __builtin_amdgcn_s_sleep(2);
        if ((long long)__builtin_amdgcn_s_memrealtime() - t0 > spin_ticks) {
            __hip_atomic_store(&ctl->err, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            break;
        }
    }
}

// The whole raytrace in one launch: persistent workgroups claim tiles in the
// order of the schedule (stage by stage) from a ticket -- of one list per XCD
// (TileLists, as k_chem_sweep), into which the tiles are dealt by the 128-byte
// lines their rows lie in, each list in schedule order -- and read a tile's
// upstream halo only once the tiles across its three upstream faces have
// published it (those tiles waited in turn for theirs).  Every list being in
// schedule order, the lowest unfinished tile is always held by a running
// workgroup or next in its list, so the sweep cannot deadlock.  On float
// grids the halo entries carry the epoch of the call (ctl->epoch + 1) and are
// polled until current; on double grids the tile waits for the upstream
// tiles' done-flags, which carry the epoch, and sets its own once its stores
// have completed.  The last workgroup to leave resets the tickets and
// advances the epoch, so replays of a captured graph need no reset.  A wait
// longer than spin_ticks (of the 100 MHz real-time counter) sets ctl->err and
// goes on, so every workgroup exits; the result is then reported invalid.
// With a condition word (cond), the raytrace runs only if the word is
// non-zero, and the last workgroup to leave clears it.  The exit count, the
// resets and the epoch are relaxed atomics: a workgroup counts itself only
// after its last claim has returned, and the next launch that reads them
// follows this one's end (an agent-scope release per workgroup would write
// back the XCD's L2 a thousand times per launch).
//
// Columns pass between tiles without cache maintenance: a tile writes its
// face entries, and reads its upstream halo, as relaxed atomics at agent
// scope, which go to the device-wide point of coherence instead of the caches
// of one compute unit or one XCD.  With done-flags, every wave waits for its
// stores to complete (vmcnt 0) before the workgroup barrier that precedes the
// flag store, so a flag is seen only after the entries it covers are in
// place.  (An agent-scope release and acquire per tile would write back and
// invalidate the L2 of the XCD on every tile instead.)
//
// The claims, waits and flag stores are made by the whole of wave 0, under
// branches on values made uniform with readfirstlane, never under a branch
// on the lane (threadIdx.x == 0): the compiler may merge the lane-0 flag
// store at the end of one tile with the lane-0 claim at the start of the
// next, and a branch on the lane then splits wave 0 into lane 0 (store and
// claim) and the other lanes (straight back to the next tile), which loop
// on the old ticket forever while lane 0 waits for them to rejoin.  Wave-
// uniform branches keep every wave whole; all lanes of wave 0 store the same
// value, and only lane 0 adds 1 to a counter (the others add 0).
template <typename R, int TT>
__global__ void __launch_bounds__(SweepShape<TT>::THREADS)
k_sweep_persist(const GridDev<R>* __restrict__ grids, int state, int tau_buf,
                const int4* __restrict__ tiles, TileLists lists, const int4* __restrict__ octs,
                unsigned* __restrict__ flags, face_t<R>* fbuf, SweepCtl* ctl, long long spin_ticks,
                unsigned* cond)
{
    constexpr int NHALO = (TT + 1) * (TT + 1) * (TT + 1);
    __shared__ R s_tc[NHALO];
    __shared__ R s_kap[NHALO];
    __shared__ int s_ticket;
    const bool lead = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6)) == 0;
    const unsigned done =
        __builtin_amdgcn_readfirstlane(
            __hip_atomic_load(&ctl->epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) + 1u;
    // with a condition word that reads 0, every workgroup leaves at once and
    // nothing is counted or reset (all of them read the same value: the word
    // is cleared only after every workgroup of a running launch has counted
    // itself)
    if (cond && __builtin_amdgcn_readfirstlane(__hip_atomic_load(
                    cond, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) == 0u)
        return;
    // the tile list of this workgroup's XCD
    const int list = lists.n > 1 ? (int)(blockIdx.x % NXCD) : 0;
    const int lfirst = lists.first[list], lcount = lists.first[list + 1] - lfirst;
    // thread 0 claims the tickets: the first here, each later one before the
    // sweep of the tile before it, so that it arrives while that tile sweeps
    // (a held tile waits for the tile its workgroup sweeps, which is earlier
    // in schedule order, as every upstream tile is: a chain of waits always
    // ends at a tile that runs)
    unsigned claim = 0u;
    if (threadIdx.x == 0)
        claim = __hip_atomic_fetch_add(&ctl->lticket[list], 1u, __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
    for (;;) {
        if (threadIdx.x == 0) s_ticket = (int)claim;
        __syncthreads();
        const int t = __builtin_amdgcn_readfirstlane(s_ticket);
        __syncthreads();   // (s_ticket is rewritten by the next claim)
        if (t >= lcount) break;
        const int4 tl = tiles[lfirst + t];
        const int4 oc = octs[tl.x];                         // flag base, tiles per axis
        const int idx = oc.x + (tl.w * oc.z + tl.z) * oc.y + tl.y;
        if (threadIdx.x == 0)
            claim = __hip_atomic_fetch_add(&ctl->lticket[list], 1u, __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_AGENT);
        sweep_tile<R, TT, SweepShape<TT>::THREADS, TILE_COHERENT>(
            grids, state, tau_buf, tl, s_tc, s_kap, [&] {
            if constexpr (!FaceWord<R>::tagged)
                if (lead) wait_upstream(flags, idx, tl, oc, done, spin_ticks, ctl);
        }, fbuf, idx, oc, done, spin_ticks, ctl);
        if constexpr (!FaceWord<R>::tagged) {
            // every wave's column stores complete, then the flag
            asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
            __syncthreads();
            if (lead)
                __hip_atomic_store(&flags[idx], done, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        // (tagged entries need no flag; the claim's barrier keeps the next
        // tile's LDS writes behind this tile's last reads)
    }
    if (threadIdx.x == 0) {
        const unsigned left = __hip_atomic_fetch_add(&ctl->exited, 1u, __ATOMIC_RELAXED,
                                                      __HIP_MEMORY_SCOPE_AGENT);
        if (left == gridDim.x - 1) {
            // every workgroup read the condition before it left
            if (cond) __hip_atomic_store(cond, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            for (int l = 0; l < NXCD; ++l)
                __hip_atomic_store(&ctl->lticket[l], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(&ctl->exited, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(&ctl->epoch, done, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
}

// ---------------------------------------------------------------- chemistry
// Grid of workgroup b of a launch over a batch (first[g] <= b < first[g+1]).
__device__ __forceinline__ int find_grid(const int* __restrict__ first, int ngrids, int b)
{
    int lo = 0, hi = ngrids - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (first[mid] <= b) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// Work counters: summed over the workgroup (wavefront shuffles, then LDS) and
// added with one atomic per counter per workgroup, into the slot of the
// workgroup.
__device__ __forceinline__ void add_work(unsigned long long* ctr, const Work& w)
{
    __shared__ unsigned long long s_w[WORK_COUNTERS];
    if (threadIdx.x < WORK_COUNTERS) s_w[threadIdx.x] = 0;
    __syncthreads();
    unsigned long long v[WORK_COUNTERS] = {
        (unsigned long long)w.accepted, (unsigned long long)w.rejected,
        (unsigned long long)w.fallbacks, (unsigned long long)w.newton,
        (unsigned long long)w.fixed };
#pragma unroll
    for (int c = 0; c < WORK_COUNTERS; ++c)
        for (int o = 32; o > 0; o >>= 1) v[c] += __shfl_xor(v[c], o, 64);
    if ((threadIdx.x & 63) == 0) {
#pragma unroll
        for (int c = 0; c < WORK_COUNTERS; ++c) atomicAdd(&s_w[c], v[c]);
    }
    __syncthreads();
    if (threadIdx.x < WORK_COUNTERS)
        atomicAdd(&ctr[threadIdx.x * WORK_SLOTS + blockIdx.x % WORK_SLOTS], s_w[threadIdx.x]);
}

// Waves per SIMD the register allocation of k_chem aims at: the double
// kernel otherwise needs more than the 256 registers that two waves share,
// and so does the variant for several sources (one environment per source,
// unrolled); it takes the double kernel's two.
template <typename R> struct ChemWaves { static constexpr int value = 3; };
template <> struct ChemWaves<double> { static constexpr int value = 2; };

// Copy of the rate table in LDS (it is read at every rate evaluation); the
// returned parameters point at it.  Every thread of the block must call it.
template <typename R>
__device__ __forceinline__ Params<R> table_to_lds(const Params<R>& p, DevTable<R>& s_tab)
{
    if (p.spectrum == 1) {
        constexpr int NW = (int)(sizeof(DevTable<R>) / sizeof(R));
        const R* src = reinterpret_cast<const R*>(p.tab);
        R* dst = reinterpret_cast<R*>(&s_tab);
        for (int i = threadIdx.x; i < NW; i += blockDim.x) dst[i] = src[i];
    }
    __syncthreads();
    Params<R> pl = p;
    pl.tab = &s_tab;   // (not read with the monochromatic spectrum)
    return pl;
}

// Environment of cell q = (i, j, k) of a grid with several sources: source s
// has its own geometry and its own columns, tau[s * ncell + q].  ok turns false
// when one of the columns is not finite.
template <int MS, typename C, typename S>
__device__ __forceinline__ EnvM<C, MS> multi_env(const Params<C>& p, const Sources<C>& src, C n,
                                                 const S* __restrict__ tau, int q, int i, int j,
                                                 int k, C tq, bool& ok)
{
    EnvM<C, MS> e{};
    e.s[0] = make_env(p, n, cell_geom(p, i, j, k), tq);
    e.n = e.s[0].n;
    e.inv_n = e.s[0].inv_n;
    e.c3 = e.s[0].c3;
    e.ns = src.n;
#pragma unroll
    for (int s = 1; s < MS; ++s) {
        if (s < src.n) {
            const C ts = C(tau[(int64_t)s * p.ncell + q]);
            ok = ok && isfinite(ts);
            const CellGeom<C> cg =
                cell_geom_at(p, src.v[s - 1][0], src.v[s - 1][1], src.v[s - 1][2], i, j, k);
            e.s[s] = make_env_q(p, src.QV[s - 1], n, cg, ts);
        }
    }
    return e;
}

// With grids of both kinds in a batch, whether grid G belongs to the launch of
// the kernel variant for MS sources.
template <int MS, typename R>
__device__ __forceinline__ bool other_kind(const BatchDev& bd, const GridDev<R>& G)
{
    return bd.kinds == 3 && ((G.src.n > 1) != (MS > 1));
}

// Micro-integration of cell q in arithmetic C from storage S.  A non-finite
// input stays non-finite (the bound projections of the solver would otherwise
// turn it into a valid-looking state), so the grid's diagnostics report it.
// (i, j, k) are the cell's coordinates, q = i + nx (j + ny k).
// Micro-integration of a cell lit by one point source from its loaded
// values: (x, E) at t_n in, at t_n + hd out (NaN for a non-finite input).
template <typename C>
__device__ __forceinline__ void chem_cell_at(const Params<C>& p, C n, C tq, int i, int j, int k,
                                             double hd, C& x, C& E, Work& w)
{
    if (!(isfinite(x) && isfinite(E) && isfinite(n) && isfinite(tq))) {
        x = E = C(__builtin_nan(""));
        return;
    }
    const CellGeom<C> cg = cell_geom(p, i, j, k);
    const Env<C> e = make_env(p, n, cg, tq);
    micro(p, e, C(hd), x, E, w);
}

template <typename C, typename S, int MS>
__device__ __forceinline__ void chem_cell(const Params<C>& p, const Sources<C>& src, int q, int i,
                                          int j, int k, const S* __restrict__ nH, const S* x0,
                                          const S* E0, const S* __restrict__ tau, double hd, C& x,
                                          C& E, Work& w)
{
    x = C(x0[q]);
    E = E0 ? C(E0[q]) : C(0);
    const C n = C(nH[q]), tq = C(tau[q]);
    if constexpr (MS == 1) {
        chem_cell_at(p, n, tq, i, j, k, hd, x, E, w);
    } else {
        if (!(isfinite(x) && isfinite(E) && isfinite(n) && isfinite(tq))) {
            x = E = C(__builtin_nan(""));
            return;
        }
        bool ok = true;
        const EnvM<C, MS> e = multi_env<MS>(p, src, n, tau, q, i, j, k, tq, ok);
        if (!ok) {
            x = E = C(__builtin_nan(""));
            return;
        }
        micro(p, e, C(hd), x, E, w);
    }
}

// Micro-physics of every cell of every grid.  With mixed precision a cell
// whose float integration took a precision-sensitive decision is not
// written, and with mixed == 2 an ionisation-front cell (front_cell of its
// starting neutral fraction) is not integrated in float at all; both are
// appended to the batch's re-solve list for the double pass.
template <typename R, int MS>
__global__ void __launch_bounds__(CHEM_BLOCK)
__attribute__((amdgpu_waves_per_eu(MS > 1 ? ChemWaves<double>::value : ChemWaves<R>::value)))
k_chem(const GridDev<R>* __restrict__ grids, BatchDev bd, int from, int to, int tau_buf,
       int dev_dt, double hscale, unsigned long long* ctr, int mixed)
{
    __shared__ DevTable<R> s_tab;
    const int lb = xcd_block((int)blockIdx.x, (int)gridDim.x);
    const int g = find_grid(bd.chem_first, bd.ngrids, lb);
    const GridDev<R>& G = grids[g];
    if (other_kind<MS>(bd, G)) return;   // uniform over the workgroup
    const Params<R> pl = table_to_lds(G.p, s_tab);
    // the brick is the same for the whole wavefront: its decomposition runs on
    // the scalar unit
    const int brick = __builtin_amdgcn_readfirstlane(
        (lb - bd.chem_first[g]) * (CHEM_BLOCK / 64) + (int)(threadIdx.x >> 6));
    const int lane = threadIdx.x & 63;
    const int nbx = (pl.nx + CHEM_BX - 1) / CHEM_BX, nby = (pl.ny + CHEM_BY - 1) / CHEM_BY;
    const int i = CHEM_BX * (brick % nbx) + (lane & 3);
    const int j = CHEM_BY * ((brick / nbx) % nby) + ((lane >> 2) & 3);
    const int k = CHEM_BZ * (brick / (nbx * nby)) + (lane >> 4);
    const bool inside = i < pl.nx && j < pl.ny && k < pl.nz;
    const int q = inside ? i + pl.nx * (j + pl.ny * k) : 0;
    static_assert(CHEM_BX == 4 && CHEM_BY == 4 && CHEM_BZ == 4 && CHEM_BLOCK % 64 == 0,
                  "lane -> cell map assumes 4^3 bricks");
    Work w{};
    bool flag = false;
    if (inside) {
        const double hd = dev_dt ? hscale * G.st->dt : hscale;
        R x, E;
        // with the front in double, an ionisation-front cell goes straight
        // to the double pass
        flag = mixed == 2 && front_cell(G.x[from][q]);
        if (!flag) {
            chem_cell<R, R, MS>(pl, G.src, q, i, j, k, G.nH, G.x[from], G.E[from],
                                G.tau[tau_buf], hd, x, E, w);
            flag = mixed && w.close > 0;
        }
        if (!flag) {
            G.x[to][q] = x;
            if (G.E[to]) G.E[to][q] = E;
        }
    }
    if (mixed) {
        // one atomic per wavefront for the flagged cells of the wavefront
        const unsigned long long m = __ballot(flag);
        if (m) {
            const int lane = threadIdx.x & 63;
            const int lead = __ffsll((long long)m) - 1;
            unsigned base = 0;
            if (lane == lead) base = atomicAdd(bd.fix_n, (unsigned)__popcll(m));
            base = __shfl(base, lead, 64);
            const unsigned slot = base + __popcll(m & ((1ull << lane) - 1ull));
            if (flag && slot < bd.fix_cap)
                bd.fix_list[slot] = ((long long)g << 32) | (long long)q;
        }
    }
    add_work(ctr, w);
}

// Double re-solve of the listed cells (mixed precision): each entry names its
// grid, so the rate table is read from global memory here.  Workgroups beyond
// the list return at once; the last workgroup to finish clears the list length
// and the finish count for the next micro-physics launch.
template <int MS>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(ChemWaves<double>::value)))
k_chem_fix(const GridDev<float>* __restrict__ grids, BatchDev bd, int from, int to, int tau_buf,
           int dev_dt, double hscale, unsigned long long* ctr, int clear, int mark)
{
    const unsigned n = min(bd.fix_n[0], bd.fix_cap);
    // an empty list: nothing to re-solve, mark or clear (every workgroup reads
    // the same length, which only the last workgroup of a non-empty launch
    // resets)
    if (n == 0) return;
    if (blockIdx.x * blockDim.x < n) {   // uniform over the workgroup
        Work w{};
        for (unsigned i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
            const long long e = bd.fix_list[i];
            const GridDev<float>& G = grids[(int)(e >> 32)];
            if (other_kind<MS>(bd, G)) continue;
            const int q = (int)(e & 0xffffffffll);
            const int ci = q % G.pd.nx, cj = (q / G.pd.nx) % G.pd.ny, ck = q / (G.pd.nx * G.pd.ny);
            const double hd = dev_dt ? hscale * G.st->dt : hscale;
            double x, E;
            chem_cell<double, float, MS>(G.pd, G.srcd, q, ci, cj, ck, G.nH, G.x[from], G.E[from],
                                         G.tau[tau_buf], hd, x, E, w);
            G.x[to][q] = (float)x;
            if (G.E[to]) G.E[to][q] = (float)E;
            ++w.fixed;
        }
        add_work(ctr, w);
    }
    // With grids of both kinds the first of the two launches leaves the list
    // to the second.
    if (!clear) return;
    // Every wave has its value of the list length (its branch above waited for
    // the load), so once all workgroups have counted themselves no read of the
    // length is outstanding and the last one may clear it; no fence is needed.
    __syncthreads();
    if (threadIdx.x == 0) {
        if (atomicAdd(&bd.fix_n[1], 1u) == gridDim.x - 1) {
            // cells were re-solved after a fused raytrace: it is run again
            if (mark) bd.fix_n[2] = 1u;
            bd.fix_n[0] = 0u;
            bd.fix_n[1] = 0u;
        }
    }
}

// ------------------------------------------- micro-physics fused with the sweep
// One half of an A3 step (or an A2 step) in one launch for grids with one
// point source: the micro-physics over h of every cell (from -> to, on the
// columns tau_chem), then the raytrace of the new state into tau_sweep.  The
// persistent workgroups take the tiles of edge PERSIST_TILE of the raytrace
// schedule in order (a ticket), as k_sweep_persist does -- from one list per
// XCD (TileLists), each in schedule order, into which the tiles are dealt by
// the 128-byte lines their rows lie in, so that the tiles sharing a line are
// integrated and swept behind one L2.  Every list being in schedule order,
// the lowest unfinished tile is always held or next in its list, so the
// sweep cannot deadlock.  A workgroup first
// integrates its tile's cells (each wavefront four 4^3 bricks, with the
// per-cell arithmetic of k_chem), writes the new state (plain stores: no
// other tile of the launch reads it) and puts sigma0 n_H x dx of every cell
// in LDS; then it sweeps the tile (TILE_FUSED), polling its halo entries in
// the face buffer until the upstream tiles have written them (the entries
// carry the launch's epoch, so no done-flag is stored).  A tile's micro-physics
// needs nothing from other tiles, so while some workgroups of a compute unit
// sweep or wait, the others integrate.  The register budget is that of three
// wavefronts per SIMD (168 registers), which the integrator and the sweep fit
// without spilling: at four (128) the spills' scratch traffic, with many
// workgroups resident, went past the L2s and exceeded the fields' own bytes
// for no gain in time.  With Mixed (mixed
// precision) a cell whose float integration took a precision-sensitive
// decision is listed for launch_chem_fix and not written, as in k_chem, and
// the sweep uses its float result; launch_chem_fix then re-solves it and
// marks the columns for a second, conditional raytrace.  Polls are bounded
// as in k_sweep_persist.  The rate table is copied to LDS when a tile's grid
// differs from the workgroup's previous one.
template <typename R, bool Mixed>
__global__ void __launch_bounds__(FUSED_THREADS) __attribute__((amdgpu_waves_per_eu(3)))
k_chem_sweep(const GridDev<R>* __restrict__ grids, BatchDev bd, int from, int to, int tau_chem,
             int tau_sweep, int dev_dt, double hscale, unsigned long long* ctr,
             const int4* __restrict__ tiles, TileLists lists, const int4* __restrict__ octs,
             face_t<R>* fbuf, SweepCtl* ctl, long long spin_ticks)
{
    constexpr int TT = PERSIST_TILE, NT = FUSED_THREADS;
    constexpr int HX = TT + 1, HY = TT + 1, NHALO = HX * HY * (TT + 1);
    constexpr int BRICKS = (TT / 4) * (TT / 4) * (TT / 4), BPW = BRICKS / (NT / 64);
    static_assert(TT % 4 == 0 && BPW * (NT / 64) == BRICKS, "whole bricks per wavefront");
    __shared__ DevTable<R> s_tab;
    __shared__ R s_tc[NHALO];
    __shared__ R s_kap[NHALO];
    // inputs of the tile's cells: x, E, n_H and the column at t_n, and n_H
    // of the state swept (each thread's own slots)
    __shared__ R s_in[5][BRICKS * 64];
    __shared__ int s_ticket;
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int lane = threadIdx.x & 63;
    const unsigned done =
        __builtin_amdgcn_readfirstlane(
            __hip_atomic_load(&ctl->epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) + 1u;
    int table_of = -1;   // grid whose rate table s_tab holds
    // the tile list of this workgroup's XCD
    const int list = lists.n > 1 ? (int)(blockIdx.x % NXCD) : 0;
    const int lfirst = lists.first[list], lcount = lists.first[list + 1] - lfirst;
    Work w{};
    // thread 0 claims the tickets: the first here, each later one before the
    // sweep of the tile before it, so that it arrives while that tile sweeps
    // (a held tile waits for the tile its workgroup sweeps, which is earlier
    // in schedule order, as every upstream tile is: a chain of waits always
    // ends at a tile that runs)
    unsigned claim = 0u;
    if (threadIdx.x == 0)
        claim = __hip_atomic_fetch_add(&ctl->lticket[list], 1u, __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
    for (;;) {
        if (threadIdx.x == 0) s_ticket = (int)claim;
        __syncthreads();
        const int t = __builtin_amdgcn_readfirstlane(s_ticket);
        __syncthreads();   // (s_ticket is rewritten by the next claim)
        if (t >= lcount) break;
        const int4 tl = tiles[lfirst + t];
        const int4 oc = octs[tl.x];                         // flag base, tiles per axis
        const int idx = oc.x + (tl.w * oc.z + tl.z) * oc.y + tl.y;
        const int gidx = tl.x >> 3;
        const GridDev<R>& G = grids[gidx];
        if (gidx != table_of) {   // uniform
            table_to_lds(G.p, s_tab);
            table_of = gidx;
        }
        Params<R> pl = G.p;
        pl.tab = &s_tab;
        const int oct = tl.x & 7;
        const bool px = oct & 1, py = oct & 2, pz = oct & 4;
        const int ex = px ? pl.nx - pl.sx : pl.sx;
        const int ey = py ? pl.ny - pl.sy : pl.sy;
        const int ez = pz ? pl.nz - pl.sz : pl.sz;
        const double hd = dev_dt ? hscale * G.st->dt : hscale;
        const R* __restrict__ nHs = G.nHr[to];
        // the inputs of the thread's cells of the tile, every load in flight
        // at once, parked in LDS until their brick is integrated (one wait for
        // memory per tile instead of one per brick)
#pragma unroll
        for (int b = 0; b < BPW; ++b) {
            const int brick = wave * BPW + b;
            const int lx = 4 * (brick % (TT / 4)) + (lane & 3);
            const int ly = 4 * ((brick / (TT / 4)) % (TT / 4)) + ((lane >> 2) & 3);
            const int lz = 4 * (brick / ((TT / 4) * (TT / 4))) + (lane >> 4);
            const int Lx = tl.y * TT + lx, Ly = tl.z * TT + ly, Lz = tl.w * TT + lz;
            R vx = R(0), vE = R(0), vn = R(0), vt = R(0), vs = R(0);
            if (Lx < ex && Ly < ey && Lz < ez) {
                const int gi = px ? pl.sx + Lx : pl.sx - 1 - Lx;
                const int gj = py ? pl.sy + Ly : pl.sy - 1 - Ly;
                const int gk = pz ? pl.sz + Lz : pl.sz - 1 - Lz;
                const int q = gi + pl.nx * (gj + pl.ny * gk);
                vx = G.x[from][q];
                vE = G.E[from] ? G.E[from][q] : R(0);
                vn = G.nH[q];
                vt = G.tau[tau_chem][q];
                vs = nHs[q];
            }
            const int slot = b * NT + threadIdx.x;
            s_in[0][slot] = vx;
            s_in[1][slot] = vE;
            s_in[2][slot] = vn;
            s_in[3][slot] = vt;
            s_in[4][slot] = vs;
        }
        // micro-physics of the tile's cells; sigma0 n_H x dx of each into LDS
        for (int b = 0; b < BPW; ++b) {
            const int brick = wave * BPW + b;
            const int lx = 4 * (brick % (TT / 4)) + (lane & 3);
            const int ly = 4 * ((brick / (TT / 4)) % (TT / 4)) + ((lane >> 2) & 3);
            const int lz = 4 * (brick / ((TT / 4) * (TT / 4))) + (lane >> 4);
            const int Lx = tl.y * TT + lx, Ly = tl.z * TT + ly, Lz = tl.w * TT + lz;
            R kap = R(0);
            bool flag = false;
            int q = 0;
            if (Lx < ex && Ly < ey && Lz < ez) {
                const int gi = px ? pl.sx + Lx : pl.sx - 1 - Lx;
                const int gj = py ? pl.sy + Ly : pl.sy - 1 - Ly;
                const int gk = pz ? pl.sz + Lz : pl.sz - 1 - Lz;
                q = gi + pl.nx * (gj + pl.ny * gk);
                const int slot = b * NT + threadIdx.x;
                R x = s_in[0][slot], E = s_in[1][slot];
                const int close0 = w.close;
                chem_cell_at<R>(pl, s_in[2][slot], s_in[3][slot], gi, gj, gk, hd, x, E, w);
                flag = Mixed && w.close > close0;
                if (!flag) {
                    G.x[to][q] = x;
                    if (G.E[to]) G.E[to][q] = E;
                }
                kap = pl.sdx * s_in[4][slot] * x;
            }
            s_kap[(lz + 1) * HX * HY + (ly + 1) * HX + (lx + 1)] = kap;
            if (Mixed) {
                // one atomic per wavefront for the listed cells of the brick
                const unsigned long long m = __ballot(flag);
                if (m) {
                    const int first = __ffsll((long long)m) - 1;
                    unsigned base = 0;
                    if (lane == first) base = atomicAdd(bd.fix_n, (unsigned)__popcll(m));
                    base = __shfl(base, first, 64);
                    const unsigned slot = base + __popcll(m & ((1ull << lane) - 1ull));
                    if (flag && slot < bd.fix_cap)
                        bd.fix_list[slot] = ((long long)gidx << 32) | (long long)q;
                }
            }
        }
        if (threadIdx.x == 0)
            claim = __hip_atomic_fetch_add(&ctl->lticket[list], 1u, __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_AGENT);
        // the sweep is on the launch's critical path (later tiles wait for it):
        // its instructions go before those of the integrating wavefronts of
        // the compute unit
        __builtin_amdgcn_s_setprio(3);
        sweep_tile<R, TT, NT, TILE_FUSED>(grids, to, tau_sweep, tl, s_tc, s_kap, [] {}, fbuf,
                                          idx, oc, done, spin_ticks, ctl);
        __builtin_amdgcn_s_setprio(0);
    }
    if (threadIdx.x == 0) {
        const unsigned left = __hip_atomic_fetch_add(&ctl->exited, 1u, __ATOMIC_RELAXED,
                                                      __HIP_MEMORY_SCOPE_AGENT);
        if (left == gridDim.x - 1) {
            for (int l = 0; l < NXCD; ++l)
                __hip_atomic_store(&ctl->lticket[l], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(&ctl->exited, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(&ctl->epoch, done, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
    add_work(ctr, w);
}

// ------------------------------------------------------------- algorithm 1
// Double integration of one cell of a float grid's algorithm-1 pass (mixed
// precision) over hd on the entering column tin, out of line: it is rarely
// taken, and inline its registers would spill into the float path.
__device__ __attribute__((noinline)) void a1_cell_double(const GridDev<float>& G, int gi, int gj,
                                                         int gk, double n, double tin, double hd,
                                                         double& x, double& E, double& tb, Work& w)
{
    const Params<double>& pd = G.pd;
    const CellGeom<double> cgd = cell_geom(pd, gi, gj, gk);
    const Env<double> ed = make_env(pd, n, cgd, tin);
    micro_t<double, true>(pd, ed, hd, x, E, w, &tb);
}

// Algorithm 1's pass (Sect. 2.1): the raytrace on tiles of edge PERSIST_TILE,
// one wavefront per tile and one launch per tile diagonal, in which every
// cell, when its level comes (c_level_order, as in sweep_tile), is integrated
// over dt on the time-averaged column entering it and then passes on its own
// time-averaged optical depth per cell length, kbar = tau_avg / ell, in place
// of sigma0 n_H x dx.  At level s lane t takes the slot of the level's 64
// slots (from c_level_start) that is t modulo 64, so one copy of the
// integrator serves every level and a level of 64 cells fills the wavefront.
// The state n is advanced in place; the half-step buffers receive the pass's
// time-averaged entering columns (tau[1]) and kbar (x[1]), which the tiles of
// later stages read as their halo.  With mixed precision an ionisation-front
// cell is integrated in double, and a cell whose float integration took a
// precision-sensitive decision is integrated again in double at once (later
// cells depend on it), both out of line.
// (A stage has at most a few thousand tiles, one wavefront each: two
// wavefronts per SIMD are all a launch fills, so the kernel takes their
// register budget.)
template <typename R>
__global__ void __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(2)))
k_sweep_a1(const GridDev<R>* __restrict__ grids, const int4* __restrict__ tiles, int first,
           unsigned long long* ctr, int mixed)
{
    constexpr int TT = PERSIST_TILE, NC = TT * TT * TT;
    constexpr int HX = TT + 1, HY = TT + 1, NHALO = HX * HY * (TT + 1);
    __shared__ R s_tc[NHALO];
    __shared__ R s_kap[NHALO];
    __shared__ DevTable<R> s_tab;

    const int4 tl = tiles[first + blockIdx.x];
    const GridDev<R>& G = grids[tl.x >> 3];
    // the rate table in LDS: every rate evaluation of the integrations reads it
    const Params<R> p = table_to_lds(G.p, s_tab);
    const R* __restrict__ kbar_in = G.x[1];
    const R* __restrict__ tavg_in = G.tau[1];
    const int oct = tl.x & 7;
    const bool px = oct & 1, py = oct & 2, pz = oct & 4;
    const int ex = px ? p.nx - p.sx : p.sx;
    const int ey = py ? p.ny - p.sy : p.sy;
    const int ez = pz ? p.nz - p.sz : p.sz;
    const int X0 = tl.y * TT, Y0 = tl.z * TT, Z0 = tl.w * TT;

    // the upstream halo from the earlier stages of this pass (time-averaged
    // centre columns as the owner formed them); the tile's own cells are
    // written when their levels come
    for (int f = threadIdx.x; f < FaceList<TT>::N; f += 64) {
        const int q = face_entry<TT>(f);
        const int hx = q % HX, hy = (q / HX) % HY, hz = q / (HX * HY);
        const int Lx = X0 + hx - 1, Ly = Y0 + hy - 1, Lz = Z0 + hz - 1;
        R kap = R(0), tc = R(0);
        if (Lx >= 0 && Ly >= 0 && Lz >= 0 && Lx < ex && Ly < ey && Lz < ez) {
            const int gi = px ? p.sx + Lx : p.sx - 1 - Lx;
            const int gj = py ? p.sy + Ly : p.sy - 1 - Ly;
            const int gk = pz ? p.sz + Lz : p.sz - 1 - Lz;
            const int64_t g = gi + (int64_t)p.nx * (gj + (int64_t)p.ny * gk);
            kap = kbar_in[g];
            tc = r_fma(halo_hds<R>(Lx, Ly, Lz), kap, tavg_in[g]);
        }
        s_kap[q] = kap;
        s_tc[q] = tc;
    }
    int nlev = 0;
    const int cls = level_class(tl.y, tl.z, tl.w, nlev);
    const bool mellema = p.weights == 1;
    const double hd = G.st->dt;
    Work w{};
    __syncthreads();

    // the lane's cell at level s (the level's slot that is the lane modulo
    // 64), if the level has one there inside the grid
    struct LaneCell {
        int cl, gi, gj, gk;
        int64_t q;
        bool on;
    };
    auto lane_cell = [&](int s) {
        LaneCell c{ -1, 0, 0, 0, 0, false };
        const int w0 = c_level_start.first[cls][s];
        const int slot = w0 + (((int)threadIdx.x - w0) & 63);
        c.cl = slot < NC ? (int)c_level_order.cell[cls][slot] : -1;
        if (c.cl >= 0 && (c.cl >> 15) == s) {
            const int Lx = X0 + (c.cl & 31), Ly = Y0 + ((c.cl >> 5) & 31);
            const int Lz = Z0 + ((c.cl >> 10) & 31);
            if (Lx < ex && Ly < ey && Lz < ez) {
                c.gi = px ? p.sx + Lx : p.sx - 1 - Lx;
                c.gj = py ? p.sy + Ly : p.sy - 1 - Ly;
                c.gk = pz ? p.sz + Lz : p.sz - 1 - Lz;
                c.q = c.gi + (int64_t)p.nx * (c.gj + (int64_t)p.ny * c.gk);
                c.on = true;
            }
        }
        return c;
    };
    // a level's inputs are loaded while the level before it integrates (no
    // cell of a level is written before its own level)
    LaneCell cur = lane_cell(0);
    R n = R(1), x = R(1), E = R(0);
    if (cur.on) {
        n = G.nH[cur.q];
        x = G.x[0][cur.q];
        E = G.E[0] ? G.E[0][cur.q] : R(0);
    }
    for (int s = 0; s < nlev; ++s) {
        LaneCell nxt{ -1, 0, 0, 0, 0, false };
        R n1 = R(1), x1 = R(1), E1 = R(0);
        if (s + 1 < nlev) {
            nxt = lane_cell(s + 1);
            if (nxt.on) {
                n1 = G.nH[nxt.q];
                x1 = G.x[0][nxt.q];
                E1 = G.E[0] ? G.E[0][nxt.q] : R(0);
            }
        }
        if (cur.on) {
            const int lx = cur.cl & 31, ly = (cur.cl >> 5) & 31, lz = (cur.cl >> 10) & 31;
            const int L[3] = { X0 + lx, Y0 + ly, Z0 + lz };
            const ScGeom<R> sg = sc_geom<R>(L);
            const int st[3] = { 1, HX, HX * HY };
            const int self = (lz + 1) * HX * HY + (ly + 1) * HX + (lx + 1);
            R tin = R(0);
            if (!sg.corner) {
                const int n00 = self - st[sg.a], n10 = n00 - st[sg.b];
                const int n01 = n00 - st[sg.c], n11 = n10 - st[sg.c];
                const R T00 = upstream_T(s_tc[n00], sg.hds, s_kap[n00]);
                const R T10 = upstream_T(s_tc[n10], sg.hds, s_kap[n10]);
                const R T01 = upstream_T(s_tc[n01], sg.hds, s_kap[n01]);
                const R T11 = upstream_T(s_tc[n11], sg.hds, s_kap[n11]);
                tin = sc_average<R>(mellema, sg.g00, sg.g10, sg.g01, sg.g11, T00, T10, T01, T11);
            }
            const int64_t q = cur.q;
            const CellGeom<R> cg = cell_geom(p, cur.gi, cur.gj, cur.gk);
            R xo = x, Eo = E, tb;
            if (!(isfinite(n) && isfinite(x) && isfinite(E) && isfinite(tin))) {
                xo = Eo = tb = R(__builtin_nan(""));
            } else {
                Work wc{};
                // mixed: an ionisation-front cell is integrated in double only
                const bool front = mixed == 2 && front_cell(x);
                if (!front) {
                    const Env<R> env = make_env(p, n, cg, tin);
                    if constexpr (std::is_same<R, float>::value) {
                        // inline: a call here would save and restore the
                        // wavefront's registers around every cell (the
                        // double integrator spills more inline than called)
                        [[clang::always_inline]] micro_t<R, true>(p, env, R(hd), xo, Eo, wc,
                                                                  &tb);
                    } else {
                        micro_t<R, true>(p, env, R(hd), xo, Eo, wc, &tb);
                    }
                }
                if constexpr (std::is_same<R, float>::value) {
                    if (front || (mixed && wc.close > 0)) {
                        // precision-sensitive: the same cell in double, from the same inputs
                        double xd = (double)x, Ed = (double)E, tbd;
                        a1_cell_double(G, cur.gi, cur.gj, cur.gk, (double)n, (double)tin, hd, xd,
                                       Ed, tbd, wc);
                        xo = R(xd);
                        Eo = R(Ed);
                        tb = R(tbd);
                        ++wc.fixed;
                    }
                }
                w.accepted += wc.accepted;
                w.rejected += wc.rejected;
                w.fallbacks += wc.fallbacks;
                w.newton += wc.newton;
                w.fixed += wc.fixed;
            }
            const R kbar = tb / cg.ell;
            s_kap[self] = kbar;
            s_tc[self] = r_fma(sg.hds, kbar, tin);   // entry face to centre
            G.x[0][q] = xo;
            if (G.E[0]) G.E[0][q] = Eo;
            G.tau[1][q] = tin;
            G.x[1][q] = kbar;
        }
        __syncthreads();
        cur = nxt;
        n = n1;
        x = x1;
        E = E1;
    }
    add_work(ctr, w);
}

// ---------------------------------------------------- plane-parallel raytrace
// One wavefront per row: the cells' optical depths sigma0 n_H x dx are summed
// along x in chunks of 64 (a shuffle scan within the wavefront plus the carry
// of the chunks before), and each cell gets the column before it.  No barrier:
// a wavefront past the last row returns whole.
template <typename R>
__global__ void __launch_bounds__(256)
k_plane_scan(const GridDev<R>* __restrict__ grids, BatchDev bd, int rows, int state, int tau_buf)
{
    const int row = (int)(blockIdx.x * 4 + (threadIdx.x >> 6));
    if (row >= rows) return;
    const int lane = threadIdx.x & 63;
    const int g = find_grid(bd.row_first, bd.ngrids, row);
    const GridDev<R>& G = grids[g];
    const int nx = G.p.nx;
    const int64_t base = (int64_t)(row - bd.row_first[g]) * nx;
    const R* __restrict__ nH = G.nHr[state] + base;
    const R* __restrict__ x = G.x[state] + base;
    R* __restrict__ tau = G.tau[tau_buf] + base;
    const R sdx = G.p.sdx;
    R carry = R(0);
    for (int i0 = 0; i0 < nx; i0 += 64) {
        const int i = i0 + lane;
        const R d = i < nx ? sdx * nH[i] * x[i] : R(0);
        R v = d;   // inclusive scan over the wavefront
        for (int o = 1; o < 64; o <<= 1) {
            const R u = __shfl_up(v, o, 64);
            if (lane >= o) v += u;
        }
        R before = __shfl_up(v, 1, 64);
        if (lane == 0) before = R(0);
        if (i < nx) tau[i] = carry + before;
        carry += __shfl(v, 63, 64);
    }
}

// ------------------------------------------------------ timestep + diagnostics
template <typename T> __device__ __forceinline__ T wave_sum(T v)
{
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
template <typename T> __device__ __forceinline__ T wave_min(T v)
{
    for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o, 64));
    return v;
}

// Per-workgroup partials of the timestep limit and diagnostics of state n; the
// workgroups of grid g stride over its cells, with the rate table in LDS.
template <typename R, int MS>
__global__ void __launch_bounds__(DT_BLOCK)
k_dtdiag(const GridDev<R>* __restrict__ grids, BatchDev bd)
{
    __shared__ DevTable<R> s_tab;
    const int g = find_grid(bd.dt_first, bd.ngrids, blockIdx.x);
    const GridDev<R>& G = grids[g];
    if (other_kind<MS>(bd, G)) return;   // uniform over the workgroup
    const Params<R> p = table_to_lds(G.p, s_tab);
    const int lb = blockIdx.x - bd.dt_first[g], nb = bd.dt_first[g + 1] - bd.dt_first[g];
    const R* __restrict__ nH = G.nH;
    const R* __restrict__ x = G.x[0];
    const R* __restrict__ E = G.E[0];
    const R* __restrict__ tau = G.tau[0];
    // the energy criterion reads dE/dt; without it the cooling terms are not
    // formed (uniform over the grid)
    const bool energy = p.K[1] < R(1e30) && p.thermal == 1;
    double v[NPART] = { __builtin_huge_val(), 0.0, 0.0, 0.0, 0.0, 0.0 };
    // (i, j, k) of the thread's first cell and of the stride, divided once;
    // each step adds them with carries
    const int q0 = lb * DT_BLOCK + threadIdx.x, stride = nb * DT_BLOCK;
    int i = q0 % p.nx, j = (q0 / p.nx) % p.ny, k = q0 / (p.nx * p.ny);
    const int si = stride % p.nx, sj = (stride / p.nx) % p.ny, sk = stride / (p.nx * p.ny);
    for (int q = q0; q < p.ncell; q += stride) {
        const CellGeom<R> cg = cell_geom(p, i, j, k);
        const R n = nH[q], xq = x[q], tq = tau[q];
        const R Eq = E ? E[q] : R(0);
        Rhs<R> r;
        bool ok = true;
        if constexpr (MS == 1) {
            const Env<R> e = make_env(p, n, cg, tq);
            if (energy) rhs_full(p, e, xq, Eq, r);
            else rhs_full<R, Env<R>, false>(p, e, xq, Eq, r);
        } else {
            const EnvM<R, MS> e = multi_env<MS>(p, G.src, n, tau, q, i, j, k, tq, ok);
            if (energy) rhs_full(p, e, xq, Eq, r);
            else rhs_full<R, EnvM<R, MS>, false>(p, e, xq, Eq, r);
        }
        v[0] = fmin(v[0], cell_dt(p, r, n, xq, Eq));
        v[1] += (double)n * (1.0 - (double)xq);
        v[2] += 1.0 - (double)xq;
        v[3] += (double)r.A;
        v[4] += (double)r.rec;
        const bool bad = !isfinite((double)xq) || !isfinite((double)tq) || !ok ||
                         (E && !isfinite((double)Eq));
        v[5] += bad ? 1.0 : 0.0;
        i += si;
        const int ci = i >= p.nx;
        i -= ci ? p.nx : 0;
        j += sj + ci;
        const int cj = j >= p.ny;
        j -= cj ? p.ny : 0;
        k += sk + cj;
    }
    __shared__ double sm[NPART][DT_BLOCK / 64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    v[0] = wave_min(v[0]);
    for (int m = 1; m < NPART; ++m) v[m] = wave_sum(v[m]);
    if (lane == 0)
        for (int m = 0; m < NPART; ++m) sm[m][w] = v[m];
    __syncthreads();
    if (threadIdx.x == 0) {
        double o[NPART];
        o[0] = fmin(fmin(sm[0][0], sm[0][1]), fmin(sm[0][2], sm[0][3]));
        for (int m = 1; m < NPART; ++m) o[m] = ((sm[m][0] + sm[m][1]) + sm[m][2]) + sm[m][3];
        for (int m = 0; m < NPART; ++m) G.part[lb * NPART + m] = o[m];
    }
}

// One workgroup per grid: fixed-order reduction of the grid's partials
// (deterministic for a given grid), then dt = min(limit, t_end - t) with a
// remainder below 1e-12 t_end absorbed into the step.
template <typename R>
__global__ void __launch_bounds__(256)
k_finalize(const GridDev<R>* __restrict__ grids, BatchDev bd, double t_end_arg)
{
    const GridDev<R>& G = grids[blockIdx.x];
    const int nblk = bd.dt_first[blockIdx.x + 1] - bd.dt_first[blockIdx.x];
    const double* __restrict__ part = G.part;
    DevState* st = G.st;
    __shared__ double sm[NPART][256];
    double v[NPART] = { __builtin_huge_val(), 0.0, 0.0, 0.0, 0.0, 0.0 };
    for (int b = threadIdx.x; b < nblk; b += 256) {
        v[0] = fmin(v[0], part[b * NPART]);
        for (int m = 1; m < NPART; ++m) v[m] += part[b * NPART + m];
    }
    for (int m = 0; m < NPART; ++m) sm[m][threadIdx.x] = v[m];
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) {
            sm[0][threadIdx.x] = fmin(sm[0][threadIdx.x], sm[0][threadIdx.x + w]);
            for (int m = 1; m < NPART; ++m) sm[m][threadIdx.x] += sm[m][threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double t_end = isfinite(t_end_arg) ? t_end_arg : st->t_end;
        double dt = sm[0][0];
        const double rem = t_end - st->t;
        if (!(rem > 0.0)) {
            dt = 0.0;
        } else {
            if (dt > rem) dt = rem;
            if (rem - dt <= 1e-12 * t_end) dt = rem;
        }
        const double cv = G.cell_vol;
        st->dt = dt;
        st->t_end = t_end;
        st->diag[0] = sm[1][0] * cv;
        st->diag[1] = sm[2][0] * cv;
        st->diag[2] = G.face_area > 0.0
                          ? sm[2][0] * cv / G.face_area
                          : cbrt(3.0 * sm[2][0] * cv * 8.0 / (4.0 * 3.14159265358979323846 * G.noct));
        st->diag[3] = sm[3][0] * cv;
        st->diag[4] = sm[4][0] * cv;
        st->diag[5] = sm[5][0];
        st->diag[6] = G.noct;
        st->diag[7] = st->t;
    }
}

template <typename R>
__global__ void k_advance(const GridDev<R>* __restrict__ grids, int ngrids)
{
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g < ngrids) {
        DevState* st = grids[g].st;
        const double dt = st->dt;
        if (dt > 0.0) {
            st->t = (st->t_end - st->t - dt <= 0.0) ? st->t_end : st->t + dt;
            st->nsteps += 1;
            st->last_dt = dt;
        }
    }
}

template <typename R>
__global__ void __launch_bounds__(256)
k_energy(int64_t n, const R* __restrict__ nH, const R* __restrict__ x, R* __restrict__ E, double T0)
{
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q < n) E[q] = R(1.5 * KB * T0) * nH[q] * (R(2) - x[q]);
}

__global__ void k_set_t_end(DevState* st, double t_end)
{
    if (threadIdx.x == 0) st->t_end = t_end;
}

// ---------------------------------------------------------------- launchers
hipError_t launch_set_t_end(DevState* st, double t_end, hipStream_t s)
{
    hipLaunchKernelGGL(k_set_t_end, dim3(1), dim3(64), 0, s, st, t_end);
    return hipGetLastError();
}

template <typename R, int TT>
void launch_sweep_t(const GridDev<R>* grids, int state, int tau_buf, const int4* tiles, int first,
                    int count, hipStream_t s)
{
    hipLaunchKernelGGL((k_sweep<R, TT>), dim3(count), dim3(SweepShape<TT>::THREADS), 0, s, grids,
                       state, tau_buf, tiles, first);
}

template <typename R>
hipError_t launch_sweep_stage(const GridDev<R>* grids, int state, int tau_buf, const int4* tiles,
                              int first, int count, int tile, hipStream_t s)
{
    if (count <= 0) return hipSuccess;
    if (tile == SWEEP_TILES[0])
        launch_sweep_t<R, SWEEP_TILES[0]>(grids, state, tau_buf, tiles, first, count, s);
    else if (tile == SWEEP_TILES[1])
        launch_sweep_t<R, SWEEP_TILES[1]>(grids, state, tau_buf, tiles, first, count, s);
    else if (tile == SWEEP_TILES[2])
        launch_sweep_t<R, SWEEP_TILES[2]>(grids, state, tau_buf, tiles, first, count, s);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

template <typename R>
hipError_t launch_sweep_persist(const GridDev<R>* grids, int state, int tau_buf, const int4* tiles,
                                const TileLists& lists, const int4* octs, unsigned* flags,
                                void* fbuf, SweepCtl* ctl, int nwg, long long spin_ticks,
                                unsigned* cond, hipStream_t s)
{
    if (lists.first[lists.n] <= 0 || nwg <= 0) return hipSuccess;
    // every list needs a workgroup
    if (lists.n > 1 && nwg < NXCD) return hipErrorInvalidValue;
    hipLaunchKernelGGL((k_sweep_persist<R, PERSIST_TILE>), dim3(nwg),
                       dim3(SweepShape<PERSIST_TILE>::THREADS), 0, s, grids, state, tau_buf, tiles,
                       lists, octs, flags, static_cast<face_t<R>*>(fbuf), ctl, spin_ticks, cond);
    return hipGetLastError();
}

template <typename R> int sweep_persist_occupancy()
{
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_sweep_persist<R, PERSIST_TILE>,
                                                     SweepShape<PERSIST_TILE>::THREADS, 0) !=
        hipSuccess)
        return 1;
    return n > 0 ? n : 1;
}

template <typename R>
hipError_t launch_chem_sweep(const GridDev<R>* grids, const BatchDev& b, int from, int to,
                             int tau_chem, int tau_sweep, bool dev_dt, double hscale,
                             unsigned long long* ctr, bool mixed, const int4* tiles,
                             const TileLists& lists, const int4* octs, void* fbuf, SweepCtl* ctl,
                             int nwg, long long spin_ticks, hipStream_t s)
{
    if constexpr (std::is_same<R, float>::value) {
        if (lists.first[lists.n] <= 0 || nwg <= 0) return hipSuccess;
        // every list needs a workgroup
        if (lists.n > 1 && nwg < NXCD) return hipErrorInvalidValue;
        if (mixed)
            hipLaunchKernelGGL((k_chem_sweep<R, true>), dim3(nwg), dim3(FUSED_THREADS), 0, s,
                               grids, b, from, to, tau_chem, tau_sweep, (int)dev_dt, hscale, ctr,
                               tiles, lists, octs, static_cast<face_t<R>*>(fbuf), ctl,
                               spin_ticks);
        else
            hipLaunchKernelGGL((k_chem_sweep<R, false>), dim3(nwg), dim3(FUSED_THREADS), 0, s,
                               grids, b, from, to, tau_chem, tau_sweep, (int)dev_dt, hscale, ctr,
                               tiles, lists, octs, static_cast<face_t<R>*>(fbuf), ctl,
                               spin_ticks);
        return hipGetLastError();
    } else {
        // double storage keeps the separate kernels (its integrator does not
        // fit the fused kernel's registers)
        return hipErrorNotSupported;
    }
}

template <typename R> int chem_sweep_occupancy(bool mixed)
{
    int n = 0;
    hipError_t e = hipErrorNotSupported;
    if constexpr (std::is_same<R, float>::value) {
        if (mixed)
            e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_chem_sweep<R, true>,
                                                             FUSED_THREADS, 0);
        else
            e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_chem_sweep<R, false>,
                                                             FUSED_THREADS, 0);
    }
    if (e != hipSuccess) return 1;
    return n > 0 ? n : 1;
}

template <typename R>
hipError_t launch_sweep_a1(const GridDev<R>* grids, const int4* tiles, int first, int count,
                           unsigned long long* ctr, int mixed, hipStream_t s)
{
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL((k_sweep_a1<R>), dim3(count), dim3(64), 0, s, grids, tiles, first, ctr,
                       mixed);
    return hipGetLastError();
}

template <typename R>
hipError_t launch_plane_scan(const GridDev<R>* grids, const BatchDev& b, int rows, int state,
                             int tau_buf, hipStream_t s)
{
    if (rows <= 0) return hipSuccess;
    hipLaunchKernelGGL((k_plane_scan<R>), dim3((rows + 3) / 4), dim3(256), 0, s, grids, b, rows,
                       state, tau_buf);
    return hipGetLastError();
}

template <typename R>
hipError_t launch_chem(const GridDev<R>* grids, const BatchDev& b, int nblocks, int from, int to,
                       int tau_buf, bool dev_dt, double hscale, unsigned long long* ctr,
                       int mixed, hipStream_t s)
{
    if (nblocks <= 0) return hipSuccess;
    if (b.kinds & 1)
        hipLaunchKernelGGL((k_chem<R, 1>), dim3(nblocks), dim3(CHEM_BLOCK), 0, s, grids, b, from,
                           to, tau_buf, (int)dev_dt, hscale, ctr, mixed);
    if (b.kinds & 2)
        hipLaunchKernelGGL((k_chem<R, MAX_SRC>), dim3(nblocks), dim3(CHEM_BLOCK), 0, s, grids, b,
                           from, to, tau_buf, (int)dev_dt, hscale, ctr, mixed);
    return hipGetLastError();
}

hipError_t launch_chem_fix(const GridDev<float>* grids, const BatchDev& b, int nblk, int from,
                           int to, int tau_buf, bool dev_dt, double hscale,
                           unsigned long long* ctr, bool mark, hipStream_t s)
{
    if (nblk <= 0) return hipSuccess;
    if (b.kinds & 1)
        hipLaunchKernelGGL(k_chem_fix<1>, dim3(nblk), dim3(256), 0, s, grids, b, from, to,
                           tau_buf, (int)dev_dt, hscale, ctr, (b.kinds & 2) ? 0 : 1, (int)mark);
    if (b.kinds & 2)
        hipLaunchKernelGGL(k_chem_fix<MAX_SRC>, dim3(nblk), dim3(256), 0, s, grids, b, from, to,
                           tau_buf, (int)dev_dt, hscale, ctr, 1, (int)mark);
    return hipGetLastError();
}

template <typename R>
hipError_t launch_dtdiag(const GridDev<R>* grids, const BatchDev& b, int nblocks, double t_end_arg,
                         hipStream_t s)
{
    if (nblocks <= 0 || b.ngrids <= 0) return hipSuccess;
    if (b.kinds & 1)
        hipLaunchKernelGGL((k_dtdiag<R, 1>), dim3(nblocks), dim3(DT_BLOCK), 0, s, grids, b);
    if (b.kinds & 2)
        hipLaunchKernelGGL((k_dtdiag<R, MAX_SRC>), dim3(nblocks), dim3(DT_BLOCK), 0, s, grids, b);
    hipLaunchKernelGGL((k_finalize<R>), dim3(b.ngrids), dim3(256), 0, s, grids, b, t_end_arg);
    return hipGetLastError();
}

template <typename R>
hipError_t launch_advance(const GridDev<R>* grids, int ngrids, hipStream_t s)
{
    if (ngrids <= 0) return hipSuccess;
    hipLaunchKernelGGL((k_advance<R>), dim3((ngrids + 63) / 64), dim3(64), 0, s, grids, ngrids);
    return hipGetLastError();
}

template <typename R>
hipError_t launch_energy(int64_t n, const R* nH, const R* x, R* E, double T0, hipStream_t s)
{
    hipLaunchKernelGGL((k_energy<R>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, nH, x,
                       E, T0);
    return hipGetLastError();
}

#define PI_INSTANTIATE(R)                                                                          \
    template hipError_t launch_sweep_stage<R>(const GridDev<R>*, int, int, const int4*, int, int,  \
                                              int, hipStream_t);                                   \
    template hipError_t launch_sweep_persist<R>(const GridDev<R>*, int, int, const int4*,          \
                                                const TileLists&, const int4*, unsigned*, void*,   \
                                                SweepCtl*, int, long long, unsigned*,              \
                                                hipStream_t);                                      \
    template int sweep_persist_occupancy<R>();                                                     \
    template hipError_t launch_chem_sweep<R>(const GridDev<R>*, const BatchDev&, int, int, int,     \
                                             int, bool, double, unsigned long long*, bool,         \
                                             const int4*, const TileLists&, const int4*,           \
                                             void*, SweepCtl*, int, long long, hipStream_t);       \
    template int chem_sweep_occupancy<R>(bool);                                                    \
    template hipError_t launch_chem<R>(const GridDev<R>*, const BatchDev&, int, int, int, int,    \
                                       bool, double, unsigned long long*, int, hipStream_t);       \
    template hipError_t launch_dtdiag<R>(const GridDev<R>*, const BatchDev&, int, double,         \
                                         hipStream_t);                                             \
    template hipError_t launch_advance<R>(const GridDev<R>*, int, hipStream_t);                   \
    template hipError_t launch_plane_scan<R>(const GridDev<R>*, const BatchDev&, int, int, int,   \
                                             hipStream_t);                                         \
    template hipError_t launch_sweep_a1<R>(const GridDev<R>*, const int4*, int, int,              \
                                           unsigned long long*, int, hipStream_t);                 \
    template hipError_t launch_energy<R>(int64_t, const R*, const R*, R*, double, hipStream_t);
PI_INSTANTIATE(double)
PI_INSTANTIATE(float)

}  // namespace pi
