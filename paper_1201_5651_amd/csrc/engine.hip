// engine.hip -- batch engine: device structures of a set of grids and the
// composition of the kernels into the operations of the C ABI (raytrace,
// micro-physics update, timestep, and the second-order (algorithm 3) and
// first-order (algorithm 2) steps of Sect. 2.2 of Mackey (A&A 2012)).
#include "engine.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>

namespace pi {

#define HIP_OR(expr, msg)                                                                          \
    do {                                                                                           \
        hipError_t e_ = (expr);                                                                    \
        if (e_ != hipSuccess)                                                                      \
            return fail(PI_EDEVICE, std::string(msg) + ": " + hipGetErrorString(e_));              \
    } while (0)

namespace {

static_assert(MAX_SRC == PI_MAX_SRC, "the kernels and the ABI agree on the most sources");

// Point sources of a grid and the vertex of source s.
int nsources(const pi_grid_desc& d)
{
    return (d.source == PI_SRC_POINT && d.nsrc > 1) ? d.nsrc : 1;
}

const int32_t* source_vertex(const pi_grid_desc& d, int s)
{
    return s == 0 ? d.src : d.src_more[s - 1];
}

// Octants around every source that hold cells.
int octant_count(const pi_grid_desc& d)
{
    if (d.source == PI_SRC_PLANE) return 0;
    int noct = 0;
    for (int s = 0; s < nsources(d); ++s) {
        const int32_t* v = source_vertex(d, s);
        for (int o = 0; o < 8; ++o) {
            bool ok = true;
            for (int a = 0; a < 3; ++a) {
                const int ext = ((o >> a) & 1) ? d.n[a] - v[a] : v[a];
                ok = ok && ext > 0;
            }
            noct += ok;
        }
    }
    return noct;
}

// Rate table in the form the kernels use: values normalised by Q, logarithms
// of the values relative to tau = 0 and logarithmic slopes at the nodes.
template <typename R> void fill_table(DevTable<R>& T, const double* tab, double Q)
{
    const double* tn = tab;
    const double* P = tab + PI_NTAB;
    const double* P1 = tab + 2 * PI_NTAB;
    const double* H = tab + 3 * PI_NTAB;
    const double* H1 = tab + 4 * PI_NTAB;
    const double q = Q > 0 ? Q : 1.0;
    T.p0 = R(P[0] / q);
    T.p1_0 = R(P1[0] / q);
    T.h0 = R(H[0] / q);
    T.h1_0 = R(H1[0] / q);
    const double s1 = std::log(tn[1]);
    const double delta = std::log(tn[2]) - std::log(tn[1]);
    T.s1 = R(s1);
    T.delta = R(delta);
    T.inv_delta = R(1.0 / delta);
    T.tau1 = R(tn[1]);
    T.tau_last = R(tn[PI_NTAB - 1]);
    // ln V/V_0 and d ln V / d ln tau at node n (zero where a value vanishes)
    auto node = [&](const double* V, const double* V1, int n, double& L, double& m) {
        if (n == 0 || P[n] <= 0 || H[n] <= 0) {
            L = m = 0.0;
            return;
        }
        L = std::log(V[n] / V[0]);
        m = -tn[n] * V1[n] / V[n];
    };
    for (int j = 0; j < PI_NTAB; ++j)
        for (int c = 0; c < 8; ++c) T.cp[j][c] = T.ch[j][c] = R(0);
    // the cubic Hermite interpolant on interval j (nodes j + 1, j + 2) in
    // powers of the local coordinate t = (ln tau - ln tau_{j+1}) / Delta
    for (int j = 0; j + 2 < PI_NTAB; ++j) {
        for (int which = 0; which < 2; ++which) {
            const double* V = which ? H : P;
            const double* V1 = which ? H1 : P1;
            double L0, m0, L1, m1;
            node(V, V1, j + 1, L0, m0);
            node(V, V1, j + 2, L1, m1);
            m0 *= delta;
            m1 *= delta;
            const double a[4] = { L0, m0, 3.0 * (L1 - L0) - 2.0 * m0 - m1,
                                  2.0 * (L0 - L1) + m0 + m1 };
            R* c = which ? T.ch[j] : T.cp[j];
            for (int k = 0; k < 4; ++k) c[k] = R(a[k]);
            c[4] = R(a[1] / delta);
            c[5] = R(2.0 * a[2] / delta);
            c[6] = R(3.0 * a[3] / delta);
        }
    }
}

template <typename R> Params<R> make_params(const pi_grid_desc& d)
{
    Params<R> p;
    p.nx = d.n[0];
    p.ny = d.n[1];
    p.nz = d.n[2];
    p.sx = d.src[0];
    p.sy = d.src[1];
    p.sz = d.src[2];
    p.ncell = (int64_t)d.n[0] * d.n[1] * d.n[2];
    const bool plane = d.source == PI_SRC_PLANE;
    p.QV = R(plane ? d.Q / d.dx : d.Q / (d.dx * d.dx * d.dx));
    p.plane = plane ? 1 : 0;
    p.sdx = R(d.sigma0 * d.dx);
    p.eps = R(d.e_excess);
    p.T_fixed = R(d.T_fixed);
    p.alpha_B = R(d.alpha_B);
    for (int i = 0; i < 4; ++i) p.K[i] = std::isfinite(d.K[i]) ? R(d.K[i]) : R(INFINITY);
    p.spectrum = d.spectrum;
    p.thermal = d.thermal;
    p.recomb = d.recomb;
    p.collisional = d.collisional;
    p.cooling = d.cooling;
    p.weights = d.weights;
    p.src_rule = d.source_cell_rule;
    p.n_sub = d.n_sub;
    p.tab = nullptr;
    return p;
}

template <typename R> Sources<R> make_sources(const pi_grid_desc& d)
{
    Sources<R> m;
    m.n = nsources(d);
    for (int s = 1; s < MAX_SRC; ++s) {
        const bool on = s < m.n;
        for (int a = 0; a < 3; ++a) m.v[s - 1][a] = on ? d.src_more[s - 1][a] : 0;
        m.QV[s - 1] = R(on ? d.Q_more[s - 1] / (d.dx * d.dx * d.dx) : 0.0);
    }
    return m;
}

// Device copies of the rate table of (spectrum, T_bb), shared by the grids of
// the engine that use it.  The table is normalised by Q, so Q does not enter.
pi_status table_for(Engine& e, const pi_grid_desc& d, void** td, void** tf)
{
    *td = *tf = nullptr;
    if (d.spectrum != PI_SPEC_TABLE) return PI_OK;
    std::vector<Engine::Table>& tables = e.table_cache ? *e.table_cache : e.tables;
    for (const Engine::Table& t : tables)
        if (t.spectrum == d.spectrum && t.T_bb == d.T_bb) {
            *td = t.d;
            *tf = t.f;
            return PI_OK;
        }
    // the host quadrature is shared by every engine of the process
    static std::mutex mu;
    static std::map<double, std::vector<double>> cache;   // T_bb -> table for Q = 1
    std::vector<double> raw;
    {
        std::lock_guard<std::mutex> lk(mu);
        auto it = cache.find(d.T_bb);
        if (it != cache.end()) raw = it->second;
    }
    if (raw.empty()) {
        raw.assign(5 * PI_NTAB, 0.0);
        pi_status r = pi_table_build(d.T_bb, 1.0, raw.data());
        if (r != PI_OK) return r;
        std::lock_guard<std::mutex> lk(mu);
        cache[d.T_bb] = raw;
    }
    Engine::Table t{ d.spectrum, d.T_bb, nullptr, nullptr };
    DevTable<double> Td{};
    fill_table(Td, raw.data(), 1.0);
    DevTable<float> Tf{};
    fill_table(Tf, raw.data(), 1.0);
    HIP_OR(hipMalloc(&t.d, sizeof(Td)), "table allocation");
    if (hipMalloc(&t.f, sizeof(Tf)) != hipSuccess) {
        (void)hipFree(t.d);
        return fail(PI_ENOMEM, "table allocation");
    }
    tables.push_back(t);
    HIP_OR(hipMemcpy(t.d, &Td, sizeof(Td), hipMemcpyHostToDevice), "table upload");
    HIP_OR(hipMemcpy(t.f, &Tf, sizeof(Tf), hipMemcpyHostToDevice), "table upload");
    *td = t.d;
    *tf = t.f;
    return PI_OK;
}

template <typename R> R* fld(void* v) { return static_cast<R*>(v); }

// Device view of a grid without its tables and clock (set by the caller).
template <typename R> GridDev<R> base_entry(const pi_grid_desc& d, const pi_fields& f)
{
    GridDev<R> D{};
    D.p = make_params<R>(d);
    D.pd = make_params<double>(d);
    D.src = make_sources<R>(d);
    D.srcd = make_sources<double>(d);
    D.nH = fld<R>(f.nH);
    D.nHr[0] = D.nH;
    D.nHr[1] = f.nH_half ? fld<R>(f.nH_half) : D.nH;
    D.x[0] = fld<R>(f.x);
    D.x[1] = fld<R>(f.x_half);
    const bool ev = d.thermal == PI_T_EVOLVE;
    D.E[0] = ev ? fld<R>(f.E) : nullptr;
    D.E[1] = ev ? fld<R>(f.E_half) : nullptr;
    D.tau[0] = fld<R>(f.tau);
    D.tau[1] = fld<R>(f.tau_half);
    D.cell_vol = d.dx * d.dx * d.dx;
    D.face_area = d.source == PI_SRC_PLANE ? (double)d.n[1] * d.n[2] * d.dx * d.dx : 0.0;
    D.noct = octant_count(d);
    return D;
}

// The raytrace entry of further source s: the grid seen from that source,
// whose columns follow the grid's columns at s arrays of cells.
template <typename R> GridDev<R> source_entry(const GridDev<R>& base, const pi_grid_desc& d, int s)
{
    GridDev<R> D = base;
    const int32_t* v = source_vertex(d, s);
    D.p.sx = D.pd.sx = v[0];
    D.p.sy = D.pd.sy = v[1];
    D.p.sz = D.pd.sz = v[2];
    const int64_t n = (int64_t)d.n[0] * d.n[1] * d.n[2];
    D.tau[0] += (int64_t)s * n;
    D.tau[1] += (int64_t)s * n;
    return D;
}

template <typename R> pi_status upload_grids(Engine& e)
{
    std::vector<GridDev<R>> h(e.grids.size() + e.extra.size());
    for (size_t g = 0; g < e.grids.size(); ++g) {
        const GridHost& G = *e.grids[g];
        void *td, *tf;
        pi_status r = table_for(e, G.d, &td, &tf);
        if (r != PI_OK) return r;
        GridDev<R>& D = h[g];
        D = base_entry<R>(G.d, G.f);
        D.pd.tab = static_cast<const DevTable<double>*>(td);
        D.p.tab = static_cast<const DevTable<R>*>(sizeof(R) == sizeof(double) ? td : tf);
        D.st = G.st;
        D.part = G.part;
    }
    for (size_t m = 0; m < e.extra.size(); ++m) {
        const int g = e.extra[m].x, src = e.extra[m].y;
        h[e.grids.size() + m] = source_entry(h[g], e.grids[g]->d, src);
    }
    const size_t bytes = sizeof(GridDev<R>) * std::max<size_t>(1, h.size());
    if (bytes > e.gdev_cap) {
        if (e.gdev) (void)hipFree(e.gdev);
        e.gdev = nullptr;
        e.gdev_cap = 0;
        HIP_OR(hipMalloc(&e.gdev, bytes), "grid table allocation");
        e.gdev_cap = bytes;
    }
    if (!h.empty())
        HIP_OR(hipMemcpy(e.gdev, h.data(), sizeof(GridDev<R>) * h.size(), hipMemcpyHostToDevice),
               "grid table upload");
    return PI_OK;
}

void drop_graph(Engine& e)
{
    if (e.exec) (void)hipGraphExecDestroy(e.exec);
    if (e.graph) (void)hipGraphDestroy(e.graph);
    e.exec = nullptr;
    e.graph = nullptr;
}

template <typename R> const GridDev<R>* gd(const Engine& e)
{
    return static_cast<const GridDev<R>*>(e.gdev);
}

// Tiles of the persistent schedule, and the lists a launch of nwg persistent
// workgroups takes them from: one per XCD (tiles dealt by their 128-byte
// lines, so that the tiles sharing a line go through one L2) when every list
// gets a workgroup, else the schedule as one list.
int persist_tiles(const Engine& e)
{
    const int w = PERSIST_SCHEDULE;
    return e.stage_first[w].empty() ? 0 : e.stage_first[w].back() + e.stage_count[w].back();
}
const int4* persist_tiles_of(const Engine& e, int nwg)
{
    return nwg >= NXCD ? e.xtiles : e.tiles[PERSIST_SCHEDULE];
}
TileLists persist_lists(const Engine& e, int nwg)
{
    if (nwg >= NXCD) return e.xlists;
    TileLists one{};
    one.n = 1;
    one.first[1] = persist_tiles(e);
    return one;
}

template <typename R>
pi_status raytrace_t(Engine& e, int state, int tau_buf, int which, hipStream_t s)
{
    static_assert(SWEEP_TILES[PERSIST_SCHEDULE] == PERSIST_TILE, "schedule of the persistent sweep");
    HIP_OR(launch_plane_scan<R>(gd<R>(e), e.bd(), e.plane_rows, state, tau_buf, s),
           "plane-parallel raytrace launch");
    if (which == SWEEP_PERSIST) {
        const int nwg = std::min(persist_tiles(e), e.persist_wg);
        HIP_OR(launch_sweep_persist<R>(gd<R>(e), state, tau_buf, persist_tiles_of(e, nwg),
                                       persist_lists(e, nwg), e.octs, e.flags, e.fbuf, e.ctl, nwg,
                                       e.persist_spin, nullptr, s),
               "persistent raytrace launch");
        return PI_OK;
    }
    for (size_t k = 0; k < e.stage_first[which].size(); ++k)
        HIP_OR(launch_sweep_stage<R>(gd<R>(e), state, tau_buf, e.tiles[which],
                                     e.stage_first[which][k], e.stage_count[which][k],
                                     SWEEP_TILES[which], s),
               "raytrace launch");
    return PI_OK;
}

pi_status raytrace_any(Engine& e, int state, int tau_buf, int which, hipStream_t s)
{
    return e.fp64() ? raytrace_t<double>(e, state, tau_buf, which, s)
                    : raytrace_t<float>(e, state, tau_buf, which, s);
}

// Tile edge used inside graph capture before any tuning.
constexpr int SWEEP_DEFAULT = 1;

template <typename R>
pi_status chem_t(Engine& e, bool dev_dt, double h, int tau_buf, int from, int to, hipStream_t s)
{
    const BatchDev b = e.bd();
    HIP_OR(launch_chem<R>(gd<R>(e), b, e.chem_blocks, from, to, tau_buf, dev_dt, h, e.work,
                          e.mixed() ? (e.front() ? 2 : 1) : 0, s),
           "chemistry launch");
    if (e.mixed())
        HIP_OR(launch_chem_fix(gd<float>(e), b, e.fix_blocks, from, to, tau_buf, dev_dt, h, e.work,
                               false, s),
               "double re-solve launch");
    return PI_OK;
}

// Micro-physics over h x dt (from -> to, on the columns tau_chem) and the
// raytrace of state `to` into tau_sweep, fused in one persistent launch; with
// mixed precision, the double re-solve of the cells the fused launch listed
// and, if there were any, the raytrace again (a persistent launch that leaves
// at once otherwise: the decision is the device's, so a captured graph
// replays it).
pi_status chem_sweep_fused(Engine& e, bool dev_dt, double h, int tau_chem, int from, int to,
                           int tau_sweep, hipStream_t s)
{
    const int ntiles = persist_tiles(e);
    const BatchDev b = e.bd();
    const int nwg = std::min(ntiles, e.fused_wg);
    HIP_OR(launch_chem_sweep<float>(gd<float>(e), b, from, to, tau_chem, tau_sweep, dev_dt, h,
                                    e.work, e.mixed(), persist_tiles_of(e, nwg),
                                    persist_lists(e, nwg), e.octs, e.fbuf, e.ctl, nwg,
                                    e.persist_spin, s),
           "fused micro-physics and raytrace launch");
    if (e.mixed()) {
        HIP_OR(launch_chem_fix(gd<float>(e), b, e.fix_blocks, from, to, tau_chem, dev_dt, h,
                               e.work, true, s),
               "double re-solve launch");
        const int nwr = std::min(ntiles, e.persist_wg);
        HIP_OR(launch_sweep_persist<float>(gd<float>(e), to, tau_sweep, persist_tiles_of(e, nwr),
                                           persist_lists(e, nwr), e.octs, e.flags, e.fbuf, e.ctl,
                                           nwr, e.persist_spin, e.fix_n + 2, s),
               "conditional raytrace launch");
    }
    return PI_OK;
}

template <typename R> pi_status timestep_t(Engine& e, double t_end_arg, hipStream_t s)
{
    HIP_OR(launch_dtdiag<R>(gd<R>(e), e.bd(), e.dt_blocks, t_end_arg, s), "timestep launch");
    return PI_OK;
}

template <typename R> pi_status step_t(Engine& e, double t_end_arg, int order, hipStream_t s)
{
    pi_status r = timestep_t<R>(e, t_end_arg, s);
    if (r != PI_OK) return r;
    // (A2 with mixed precision keeps the separate kernels: its raytrace
    // overwrites the columns its micro-physics read, which the double
    // re-solve after the fused launch would still need)
    if (e.fused() && (order == 2 || !e.mixed())) {
        // predictor to the half step with the raytrace of x*, corrector with
        // the raytrace of the new state (A3); or the one step of A2
        if (order == 2 && (r = chem_sweep_fused(e, true, 0.5, PI_BUF_N, PI_BUF_N, PI_BUF_HALF,
                                                PI_BUF_HALF, s)) != PI_OK)
            return r;
        if ((r = chem_sweep_fused(e, true, 1.0, order == 2 ? PI_BUF_HALF : PI_BUF_N, PI_BUF_N,
                                  PI_BUF_N, PI_BUF_N, s)) != PI_OK)
            return r;
        HIP_OR(launch_advance<R>(gd<R>(e), e.ngrids(), s), "advance launch");
        return PI_OK;
    }
    if (order == 2) {
        if ((r = chem_t<R>(e, true, 0.5, PI_BUF_N, PI_BUF_N, PI_BUF_HALF, s)) != PI_OK) return r;
        const int w = e.sweep >= 0 ? e.sweep : SWEEP_DEFAULT;
    if ((r = raytrace_t<R>(e, PI_BUF_HALF, PI_BUF_HALF, w, s)) != PI_OK) return r;
        if ((r = chem_t<R>(e, true, 1.0, PI_BUF_HALF, PI_BUF_N, PI_BUF_N, s)) != PI_OK) return r;
    } else {
        if ((r = chem_t<R>(e, true, 1.0, PI_BUF_N, PI_BUF_N, PI_BUF_N, s)) != PI_OK) return r;
    }
    if ((r = raytrace_t<R>(e, PI_BUF_N, PI_BUF_N, e.sweep >= 0 ? e.sweep : SWEEP_DEFAULT, s)) != PI_OK)
        return r;
    HIP_OR(launch_advance<R>(gd<R>(e), e.ngrids(), s), "advance launch");
    return PI_OK;
}

// Algorithm 1 (Sect. 2.1): timestep, the combined pass (stages of the
// schedule of edge PERSIST_TILE), the raytrace of the new state for the next
// timestep, clock.
template <typename R> pi_status step_a1_t(Engine& e, double t_end_arg, hipStream_t s)
{
    for (GridHost* h : e.grids)
        if (h->d.source != PI_SRC_POINT || nsources(h->d) > 1)
            return fail(PI_EINVAL, "algorithm 1 needs grids with one point source");
    pi_status r = timestep_t<R>(e, t_end_arg, s);
    if (r != PI_OK) return r;
    const int w = PERSIST_SCHEDULE;
    for (size_t k = 0; k < e.stage_first[w].size(); ++k)
        HIP_OR(launch_sweep_a1<R>(gd<R>(e), e.tiles[w], e.stage_first[w][k], e.stage_count[w][k],
                                  e.work, e.mixed() ? (e.front() ? 2 : 1) : 0, s),
               "algorithm 1 pass launch");
    if ((r = raytrace_t<R>(e, PI_BUF_N, PI_BUF_N, e.sweep >= 0 ? e.sweep : SWEEP_DEFAULT, s)) != PI_OK)
        return r;
    HIP_OR(launch_advance<R>(gd<R>(e), e.ngrids(), s), "advance launch");
    return PI_OK;
}

}  // namespace

bool fused_eligible(const Engine& e)
{
    return !e.fp64() && !e.front() && e.kinds == 1 && e.plane_rows == 0 && e.extra.empty() &&
           e.fused_wg > 0;
}

bool Engine::fused() const { return sweep == SWEEP_PERSIST && fused_eligible(*this); }

BatchDev Engine::bd() const
{
    BatchDev b;
    b.ngrids = ngrids();
    b.chem_first = first;
    b.dt_first = first ? first + ngrids() + 1 : nullptr;
    b.row_first = first ? first + 2 * (ngrids() + 1) : nullptr;
    b.fix_n = fix_n;
    b.fix_list = fix_list;
    b.fix_cap = (unsigned int)fix_cap;
    b.kinds = kinds;
    return b;
}

pi_status grid_host_init(GridHost& h, const pi_grid_desc& d, const pi_fields& f)
{
    h.d = d;
    h.f = f;
    h.ncell = (int64_t)d.n[0] * d.n[1] * d.n[2];
    h.noct = octant_count(d);
    h.cell_vol = d.dx * d.dx * d.dx;
    h.nblk_dt = (int)std::min<int64_t>((h.ncell + DT_BLOCK - 1) / DT_BLOCK, DT_MAX_BLOCKS);
    if (hipMalloc(&h.st, sizeof(DevState)) != hipSuccess) return fail(PI_ENOMEM, "state allocation");
    DevState s0{};
    if (hipMemcpy(h.st, &s0, sizeof(s0), hipMemcpyHostToDevice) != hipSuccess) {
        grid_host_free(h);
        return fail(PI_EDEVICE, "state upload");
    }
    if (hipMalloc(&h.part, sizeof(double) * NPART * h.nblk_dt) != hipSuccess) {
        grid_host_free(h);
        return fail(PI_ENOMEM, "partials allocation");
    }
    // tile schedules of every source: every octant's tiles, grouped by tile
    // diagonal tx+ty+tz (none for a plane-parallel source, which is traced row
    // by row)
    for (int s = 0; s < MAX_SRC; ++s)
        for (int w = 0; w < NSWEEP; ++w) {
            const int T = SWEEP_TILES[w];
            std::vector<std::vector<int4>>& tl = h.tiles[s][w];
            tl.clear();
            if (d.source == PI_SRC_PLANE || s >= nsources(d)) continue;
            const int32_t* v = source_vertex(d, s);
            for (int o = 0; o < 8; ++o) {
                int ext[3];
                for (int a = 0; a < 3; ++a) ext[a] = ((o >> a) & 1) ? d.n[a] - v[a] : v[a];
                if (ext[0] <= 0 || ext[1] <= 0 || ext[2] <= 0) continue;
                const int ntx = (ext[0] + T - 1) / T;
                const int nty = (ext[1] + T - 1) / T;
                const int ntz = (ext[2] + T - 1) / T;
                for (int tz = 0; tz < ntz; ++tz)
                    for (int ty = 0; ty < nty; ++ty)
                        for (int tx = 0; tx < ntx; ++tx) {
                            const int D = tx + ty + tz;
                            if ((int)tl.size() <= D) tl.resize(D + 1);
                            tl[D].push_back(make_int4(o, tx, ty, tz));
                        }
            }
        }
    return PI_OK;
}

void grid_host_free(GridHost& h)
{
    if (h.st) (void)hipFree(h.st);
    if (h.part) (void)hipFree(h.part);
    h.st = nullptr;
    h.part = nullptr;
}

pi_status engine_build(Engine& e, const std::vector<GridHost*>& grids)
{
    drop_graph(e);
    e.grids = grids;
    const int G = e.ngrids();
    // further sources of each grid: raytrace entries G, G + 1, ...
    e.extra.clear();
    bool one = false;
    for (int g = 0; g < G; ++g) {
        const int ns = nsources(e.grids[g]->d);
        one = one || ns == 1;
        for (int s = 1; s < ns; ++s) e.extra.push_back(make_int2(g, s));
    }
    e.kinds = e.extra.empty() ? 1 : (one ? 3 : 2);
    // a tile names its raytrace entry in the bits above its octant
    if ((int64_t)G + (int64_t)e.extra.size() > (1 << 27))
        return fail(PI_EINVAL, "too many grids and sources in one batch");
    // launch geometry
    // three prefix tables of G + 1 entries: micro-physics workgroups,
    // timestep workgroups, rows of plane-parallel grids
    std::vector<int> first(3 * (G + 1), 0);
    int64_t cells = 0;
    int* rowf = first.data() + 2 * (G + 1);
    for (int g = 0; g < G; ++g) {
        const int64_t n = e.grids[g]->ncell;
        const pi_grid_desc& d = e.grids[g]->d;
        const int64_t cb = chem_workgroups(d.n[0], d.n[1], d.n[2]);
        const int64_t rows = d.source == PI_SRC_PLANE ? (int64_t)d.n[1] * d.n[2] : 0;
        if ((int64_t)first[g] + cb > 2147483647LL || (int64_t)rowf[g] + rows > 2147483647LL)
            return fail(PI_EINVAL, "batch too large");
        first[g + 1] = first[g] + (int)cb;
        first[G + 1 + g + 1] = first[G + 1 + g] + e.grids[g]->nblk_dt;
        rowf[g + 1] = rowf[g] + (int)rows;
        cells += n;
    }
    e.chem_blocks = first[G];
    e.dt_blocks = first[2 * G + 1];
    e.plane_rows = rowf[G];
    const size_t fb = sizeof(int) * first.size();
    if (fb > e.first_cap) {
        if (e.first) (void)hipFree(e.first);
        e.first = nullptr;
        e.first_cap = 0;
        HIP_OR(hipMalloc(&e.first, fb), "launch table allocation");
        e.first_cap = fb;
    }
    HIP_OR(hipMemcpy(e.first, first.data(), fb, hipMemcpyHostToDevice), "launch table upload");
    // combined tile schedules: stage k holds tile diagonal k of every grid
    for (int w = 0; w < NSWEEP; ++w) {
        e.stage_first[w].clear();
        e.stage_count[w].clear();
        std::vector<int4> flat;
        size_t nst = 0;
        for (GridHost* h : e.grids)
            for (int s = 0; s < MAX_SRC; ++s) nst = std::max(nst, h->tiles[s][w].size());
        // entry r of the grid table traces grid g from source s
        const int R = G + (int)e.extra.size();
        const int T = SWEEP_TILES[w];
        const int line_shift = e.fp64() ? 4 : 5;   // cells per 128-byte line: 16 or 32
        std::vector<int4> bucket[NXCD];
        for (size_t k = 0; k < nst; ++k) {
            e.stage_first[w].push_back((int)flat.size());
            // The hardware deals the workgroups of a launch to the XCDs in
            // turn.  Tiles are given slots by a hash of the 128-byte line
            // their rows start in, so neighbours along x (swept by successive
            // launches) and the same cells seen from another source share an
            // XCD, while the tiles of one octant spread over all of them.  On
            // the 256^3 medium this order makes the large middle stages
            // shorter (raytrace 0.607 -> 0.584 ms), though the bytes fetched
            // per raytrace do not change.
            for (int r = 0; r < R; ++r) {
                const int g = r < G ? r : e.extra[r - G].x;
                const int src = r < G ? 0 : e.extra[r - G].y;
                const std::vector<std::vector<int4>>& tl = e.grids[g]->tiles[src][w];
                if (k >= tl.size()) continue;
                const int32_t* v = source_vertex(e.grids[g]->d, src);
                for (const int4& t : tl[k]) {
                    const int o = t.x;
                    const int gx = (o & 1) ? v[0] + T * t.y : std::max(v[0] - T * (t.y + 1), 0);
                    const int gy = (o & 2) ? v[1] + T * t.z : v[1] - T * (t.z + 1);
                    const int gz = (o & 4) ? v[2] + T * t.w : v[2] - T * (t.w + 1);
                    const uint64_t key = (uint64_t)g * 0x9E3779B97F4A7C15ull ^
                                         (uint64_t)(gx >> line_shift) * 0xC2B2AE3D27D4EB4Full ^
                                         (uint64_t)(int64_t)gy * 0x165667B19E3779F9ull ^
                                         (uint64_t)(int64_t)gz * 0xD6E8FEB86659FD93ull;
                    bucket[(key ^ (key >> 29)) % NXCD].push_back(
                        make_int4((r << 3) | o, t.y, t.z, t.w));
                }
            }
            // slot p runs on XCD p % NXCD: take from that XCD's bucket, or
            // from the fullest one when it is empty
            size_t left = 0;
            for (int b = 0; b < NXCD; ++b) left += bucket[b].size();
            size_t pos[NXCD] = {};
            for (size_t p = 0; left > 0; ++p, --left) {
                int b = (int)(p % NXCD);
                if (pos[b] == bucket[b].size()) {
                    size_t most = 0;
                    for (int c = 0; c < NXCD; ++c)
                        if (bucket[c].size() - pos[c] > most) {
                            most = bucket[c].size() - pos[c];
                            b = c;
                        }
                }
                flat.push_back(bucket[b][pos[b]++]);
            }
            for (int b = 0; b < NXCD; ++b) bucket[b].clear();
            e.stage_count[w].push_back((int)flat.size() - e.stage_first[w].back());
        }
        if (flat.size() > e.tiles_cap[w]) {
            if (e.tiles[w]) (void)hipFree(e.tiles[w]);
            e.tiles[w] = nullptr;
            e.tiles_cap[w] = 0;
            HIP_OR(hipMalloc(&e.tiles[w], sizeof(int4) * flat.size()), "tile schedule allocation");
            e.tiles_cap[w] = flat.size();
        }
        if (!flat.empty())
            HIP_OR(hipMemcpy(e.tiles[w], flat.data(), sizeof(int4) * flat.size(),
                             hipMemcpyHostToDevice),
                   "tile schedule upload");
        if (w == PERSIST_SCHEDULE) {
            // the persistent schedule in one list per XCD: slot p of a stage
            // (dealt above to XCD p % NXCD) goes to list p % NXCD, stage after
            // stage, so every list keeps the schedule's order
            std::vector<int4> xl;
            xl.reserve(flat.size());
            e.xlists.n = NXCD;
            for (int b = 0; b < NXCD; ++b) {
                e.xlists.first[b] = (int)xl.size();
                for (size_t k = 0; k < e.stage_first[w].size(); ++k)
                    for (int q = b; q < e.stage_count[w][k]; q += NXCD)
                        xl.push_back(flat[e.stage_first[w][k] + q]);
            }
            e.xlists.first[NXCD] = (int)xl.size();
            if (xl.size() > e.xtiles_cap) {
                if (e.xtiles) (void)hipFree(e.xtiles);
                e.xtiles = nullptr;
                e.xtiles_cap = 0;
                HIP_OR(hipMalloc(&e.xtiles, sizeof(int4) * xl.size()), "tile list allocation");
                e.xtiles_cap = xl.size();
            }
            if (!xl.empty())
                HIP_OR(hipMemcpy(e.xtiles, xl.data(), sizeof(int4) * xl.size(),
                                 hipMemcpyHostToDevice),
                       "tile list upload");
        }
    }
    // persistent raytrace: flag bases per raytrace entry and octant (edge
    // PERSIST_TILE), one flag per tile, the control block
    {
        const int R = G + (int)e.extra.size();
        std::vector<int4> oct(8 * (size_t)std::max(R, 1), make_int4(0, 0, 0, 0));
        int64_t nflag = 0;
        for (int r = 0; r < R; ++r) {
            const int g = r < G ? r : e.extra[r - G].x;
            const int src = r < G ? 0 : e.extra[r - G].y;
            const pi_grid_desc& d = e.grids[g]->d;
            if (d.source == PI_SRC_PLANE) continue;
            const int32_t* v = source_vertex(d, src);
            for (int o = 0; o < 8; ++o) {
                int nt[3];
                for (int a = 0; a < 3; ++a) {
                    const int ext = ((o >> a) & 1) ? d.n[a] - v[a] : v[a];
                    nt[a] = ext > 0 ? (ext + PERSIST_TILE - 1) / PERSIST_TILE : 0;
                }
                oct[8 * r + o] = make_int4((int)nflag, nt[0], nt[1], nt[2]);
                nflag += (int64_t)nt[0] * nt[1] * nt[2];
            }
        }
        if (nflag > 2147483647LL) return fail(PI_EINVAL, "batch too large for the raytrace flags");
        const size_t ob = sizeof(int4) * oct.size();
        if (ob > e.octs_cap) {
            if (e.octs) (void)hipFree(e.octs);
            e.octs = nullptr;
            e.octs_cap = 0;
            HIP_OR(hipMalloc(&e.octs, ob), "octant table allocation");
            e.octs_cap = ob;
        }
        HIP_OR(hipMemcpy(e.octs, oct.data(), ob, hipMemcpyHostToDevice), "octant table upload");
        const size_t fb = sizeof(unsigned) * (size_t)std::max<int64_t>(nflag, 1);
        if (fb > e.flags_cap) {
            // fresh flags are zero: below the done value of every call, so a
            // flag left from another layout or an earlier call never reads done
            if (e.flags) (void)hipFree(e.flags);
            e.flags = nullptr;
            e.flags_cap = 0;
            HIP_OR(hipMalloc(&e.flags, fb), "raytrace flag allocation");
            HIP_OR(hipMemset(e.flags, 0, fb), "raytrace flag clear");
            e.flags_cap = fb;
        }
        const size_t bb = (size_t)FACE_BYTES * FACE_WORDS * (size_t)std::max<int64_t>(nflag, 1);
        if (bb > e.fbuf_cap) {
            // zero: float entries then carry epoch 0, below the epoch of every
            // call (double entries are never read before a tile of the same
            // call has written them)
            if (e.fbuf) (void)hipFree(e.fbuf);
            e.fbuf = nullptr;
            e.fbuf_cap = 0;
            HIP_OR(hipMalloc(&e.fbuf, bb), "raytrace face buffer allocation");
            HIP_OR(hipMemset(e.fbuf, 0, bb), "raytrace face buffer clear");
            e.fbuf_cap = bb;
        }
        if (!e.ctl) {
            HIP_OR(hipMalloc(&e.ctl, sizeof(SweepCtl)), "raytrace control allocation");
            HIP_OR(hipMemset(e.ctl, 0, sizeof(SweepCtl)), "raytrace control clear");
        }
        if (e.persist_wg == 0) {
            int dev = 0, cus = 0;
            HIP_OR(hipGetDevice(&dev), "device query");
            HIP_OR(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev),
                   "device query");
            const int per = e.fp64() ? sweep_persist_occupancy<double>()
                                     : sweep_persist_occupancy<float>();
            e.persist_wg = std::max(1, per * cus);
            if (!e.fp64()) e.fused_wg = std::max(1, chem_sweep_occupancy<float>(e.mixed()) * cus);
        }
    }
    // work counters
    if (!e.work) {
        const size_t wb = sizeof(unsigned long long) * WORK_COUNTERS * WORK_SLOTS;
        HIP_OR(hipMalloc(&e.work, wb), "counter allocation");
        HIP_OR(hipMemset(e.work, 0, wb), "counter clear");
    }
    // mixed precision: re-solve list for every cell of the batch
    if (e.mixed()) {
        if (!e.fix_n) {
            HIP_OR(hipMalloc(&e.fix_n, 3 * sizeof(unsigned int)), "re-solve count allocation");
            HIP_OR(hipMemset(e.fix_n, 0, 3 * sizeof(unsigned int)), "re-solve count clear");
        }
        if ((size_t)cells > e.fix_cap) {
            if (e.fix_list) (void)hipFree(e.fix_list);
            e.fix_list = nullptr;
            e.fix_cap = 0;
            HIP_OR(hipMalloc(&e.fix_list, sizeof(long long) * std::max<int64_t>(cells, 1)),
                   "re-solve list allocation");
            e.fix_cap = (size_t)cells;
        }
        // 512 workgroups of four waves fill every SIMD at the two waves the
        // double kernel's registers allow
        e.fix_blocks = (int)std::min<int64_t>((cells + 255) / 256, 512);
    }
    return e.fp64() ? upload_grids<double>(e) : upload_grids<float>(e);
}

void engine_drop_graph(Engine& e) { drop_graph(e); }

void engine_free(Engine& e)
{
    drop_graph(e);
    if (e.cap) (void)hipStreamDestroy(e.cap);
    e.cap = nullptr;
    for (void* p : { e.gdev, (void*)e.first, (void*)e.fix_n, (void*)e.fix_list, (void*)e.work,
                     (void*)e.octs, (void*)e.flags, e.fbuf, (void*)e.xtiles, (void*)e.ctl })
        if (p) (void)hipFree(p);
    e.fbuf = nullptr;
    e.fbuf_cap = 0;
    e.xtiles = nullptr;
    e.xtiles_cap = 0;
    e.octs = nullptr;
    e.flags = nullptr;
    e.ctl = nullptr;
    e.octs_cap = e.flags_cap = 0;
    e.persist_wg = 0;
    e.fused_wg = 0;
    for (int w = 0; w < NSWEEP; ++w) {
        if (e.tiles[w]) (void)hipFree(e.tiles[w]);
        e.tiles[w] = nullptr;
        e.tiles_cap[w] = 0;
    }
    free_tables(e.tables);
    e.gdev = nullptr;
    e.first = nullptr;
    e.fix_n = nullptr;
    e.fix_list = nullptr;
    e.work = nullptr;
    e.gdev_cap = e.first_cap = e.fix_cap = 0;
}

void free_tables(std::vector<Engine::Table>& tables)
{
    for (const Engine::Table& t : tables) {
        if (t.d) (void)hipFree(t.d);
        if (t.f) (void)hipFree(t.f);
    }
    tables.clear();
}

pi_status engine_autotune(Engine& e, int state, int tau_buf, hipStream_t s)
{
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    HIP_OR(hipStreamIsCapturing(s, &cs), "capture query");
    if (cs != hipStreamCaptureStatusNone) return PI_OK;   // tuned later, outside capture
    hipEvent_t ev[3];
    for (int i = 0; i < 3; ++i) HIP_OR(hipEventCreate(&ev[i]), "event creation");
    float best = 0.0f;
    int pick = SWEEP_DEFAULT;
    pi_status r = PI_OK;
    for (int w = 0; w <= SWEEP_PERSIST && r == PI_OK; ++w) {
        if (w >= NSWEEP && w != SWEEP_PERSIST) continue;
        // the second of two runs (the first warms the caches)
        r = raytrace_any(e, state, tau_buf, w, s);
        if (r == PI_OK && hipEventRecord(ev[0], s) != hipSuccess) r = fail(PI_EDEVICE, "event record");
        if (r == PI_OK) r = raytrace_any(e, state, tau_buf, w, s);
        if (r == PI_OK && hipEventRecord(ev[1], s) != hipSuccess) r = fail(PI_EDEVICE, "event record");
        if (r == PI_OK && hipEventSynchronize(ev[1]) != hipSuccess) r = fail(PI_EDEVICE, "event sync");
        float ms = 0.0f;
        if (r == PI_OK && hipEventElapsedTime(&ms, ev[0], ev[1]) != hipSuccess)
            r = fail(PI_EDEVICE, "event time");
        // a grid whose step fuses the micro-physics with the persistent
        // raytrace hides most of that raytrace's time in the step: the
        // persistent variant is taken unless it is 1.5x slower than the best
        if (r == PI_OK && w == SWEEP_PERSIST && fused_eligible(e)) ms /= 1.5f;
        if (r == PI_OK && (w == 0 || ms < best)) {
            best = ms;
            pick = w;
        }
    }
    for (int i = 0; i < 3; ++i) (void)hipEventDestroy(ev[i]);
    if (r != PI_OK) return r;
    e.sweep = pick;
    drop_graph(e);   // a graph captured before tuning holds the default tiles
    return PI_OK;
}

pi_status engine_raytrace(Engine& e, int state, int tau_buf, hipStream_t s)
{
    if (e.sweep < 0) {
        pi_status r = engine_autotune(e, state, tau_buf, s);
        if (r != PI_OK) return r;
    }
    return raytrace_any(e, state, tau_buf, e.sweep >= 0 ? e.sweep : SWEEP_DEFAULT, s);
}

pi_status engine_chem_raytrace(Engine& e, bool dev_dt, double h, int tau_buf, int from, int to,
                               int tau_out, hipStream_t s)
{
    if (e.sweep < 0) {
        pi_status r = engine_autotune(e, PI_BUF_N, PI_BUF_N, s);
        if (r != PI_OK) return r;
    }
    // (with mixed precision the double re-solve after a fused launch reads
    // the columns tau_buf, which the fused raytrace must not overwrite)
    if (e.fused() && !(e.mixed() && tau_buf == tau_out))
        return chem_sweep_fused(e, dev_dt, h, tau_buf, from, to, tau_out, s);
    pi_status r = engine_chem(e, dev_dt, h, tau_buf, from, to, s);
    if (r != PI_OK) return r;
    return raytrace_any(e, to, tau_out, e.sweep >= 0 ? e.sweep : SWEEP_DEFAULT, s);
}

pi_status engine_chem(Engine& e, bool dev_dt, double h, int tau_buf, int from, int to, hipStream_t s)
{
    return e.fp64() ? chem_t<double>(e, dev_dt, h, tau_buf, from, to, s)
                    : chem_t<float>(e, dev_dt, h, tau_buf, from, to, s);
}

pi_status engine_timestep(Engine& e, double t_end_arg, hipStream_t s)
{
    return e.fp64() ? timestep_t<double>(e, t_end_arg, s) : timestep_t<float>(e, t_end_arg, s);
}

pi_status engine_step(Engine& e, double t_end_arg, int order, hipStream_t s)
{
    return e.fp64() ? step_t<double>(e, t_end_arg, order, s) : step_t<float>(e, t_end_arg, order, s);
}

pi_status engine_step_a1(Engine& e, double t_end_arg, hipStream_t s)
{
    return e.fp64() ? step_a1_t<double>(e, t_end_arg, s) : step_a1_t<float>(e, t_end_arg, s);
}

pi_status engine_step_graph(Engine& e, hipStream_t s)
{
    if (e.ngrids() == 0) return PI_OK;
    if (!e.exec) {
        if (!e.cap) HIP_OR(hipStreamCreateWithFlags(&e.cap, hipStreamNonBlocking), "capture stream");
        HIP_OR(hipStreamBeginCapture(e.cap, hipStreamCaptureModeThreadLocal), "begin capture");
        pi_status r = engine_step(e, NAN, 2, e.cap);
        hipGraph_t g = nullptr;
        const hipError_t ce = hipStreamEndCapture(e.cap, &g);
        if (r != PI_OK) {
            if (g) (void)hipGraphDestroy(g);
            return r;
        }
        HIP_OR(ce, "end capture");
        e.graph = g;
        HIP_OR(hipGraphInstantiate(&e.exec, e.graph, nullptr, nullptr, 0), "graph instantiation");
    }
    HIP_OR(hipGraphLaunch(e.exec, s), "graph launch");
    return PI_OK;
}

pi_status engine_init_energy(Engine& e, int grid, double T0, int state, hipStream_t s)
{
    const GridHost& G = *e.grids[grid];
    if (G.d.thermal != PI_T_EVOLVE) return PI_OK;
    void* E = state == PI_BUF_HALF ? G.f.E_half : G.f.E;
    const void* x = state == PI_BUF_HALF ? G.f.x_half : G.f.x;
    if (e.fp64())
        HIP_OR(launch_energy<double>(G.ncell, static_cast<const double*>(G.f.nH),
                                     static_cast<const double*>(x), static_cast<double*>(E), T0, s),
               "energy launch");
    else
        HIP_OR(launch_energy<float>(G.ncell, static_cast<const float*>(G.f.nH),
                                    static_cast<const float*>(x), static_cast<float*>(E), T0, s),
               "energy launch");
    return PI_OK;
}

pi_status engine_read_states(Engine& e, std::vector<DevState>& out, hipStream_t s)
{
    out.assign(e.grids.size(), DevState{});
    for (size_t g = 0; g < e.grids.size(); ++g)
        HIP_OR(hipMemcpyAsync(&out[g], e.grids[g]->st, sizeof(DevState), hipMemcpyDeviceToHost, s),
               "state read");
    SweepCtl c{};
    if (e.ctl) HIP_OR(hipMemcpyAsync(&c, e.ctl, sizeof(c), hipMemcpyDeviceToHost, s), "state read");
    HIP_OR(hipStreamSynchronize(s), "state read sync");
    if (c.err) {
        // reported once; the columns of that raytrace are not valid
        const unsigned zero = 0;
        HIP_OR(hipMemcpy(&e.ctl->err, &zero, sizeof(zero), hipMemcpyHostToDevice), "state write");
        return fail(PI_EDEVICE, "a persistent raytrace tile waited longer than its limit for its "
                                "upstream tiles; the columns are not valid");
    }
    return PI_OK;
}

pi_status engine_write_states(Engine& e, const std::vector<DevState>& in, hipStream_t s)
{
    for (size_t g = 0; g < e.grids.size(); ++g)
        HIP_OR(hipMemcpyAsync(e.grids[g]->st, &in[g], sizeof(DevState), hipMemcpyHostToDevice, s),
               "state write");
    HIP_OR(hipStreamSynchronize(s), "state write sync");
    return PI_OK;
}

pi_status engine_diagnostics(Engine& e, std::vector<double>& out, hipStream_t s)
{
    std::vector<DevState> keep, now;
    pi_status r = engine_read_states(e, keep, s);
    if (r != PI_OK) return r;
    if ((r = engine_timestep(e, NAN, s)) != PI_OK) return r;
    if ((r = engine_read_states(e, now, s)) != PI_OK) return r;
    out.assign(e.grids.size() * PI_NDIAG, 0.0);
    bool bad = false;
    for (size_t g = 0; g < e.grids.size(); ++g) {
        for (int i = 0; i < PI_NDIAG; ++i) out[g * PI_NDIAG + i] = now[g].diag[i];
        bad = bad || now[g].diag[5] > 0;
        for (int i = 0; i < 8; ++i) keep[g].diag[i] = now[g].diag[i];
    }
    if ((r = engine_write_states(e, keep, s)) != PI_OK) return r;
    if (bad) return fail(PI_ENAN, "non-finite values in the grid state");
    return PI_OK;
}

pi_status engine_work(Engine& e, int64_t* out, int reset, hipStream_t s)
{
    unsigned long long h[WORK_COUNTERS * WORK_SLOTS];
    HIP_OR(hipMemcpyAsync(h, e.work, sizeof(h), hipMemcpyDeviceToHost, s), "counter read");
    HIP_OR(hipStreamSynchronize(s), "counter read sync");
    for (int c = 0; c < WORK_COUNTERS; ++c) {
        unsigned long long v = 0;
        for (int k = 0; k < WORK_SLOTS; ++k) v += h[c * WORK_SLOTS + k];
        out[c] = (int64_t)v;
    }
    if (reset) {
        HIP_OR(hipMemsetAsync(e.work, 0, sizeof(h), s), "counter clear");
        HIP_OR(hipStreamSynchronize(s), "counter clear sync");
    }
    return PI_OK;
}

// ------------------------------------------------------------ memory sizes
namespace {
size_t word_of(const pi_grid_desc& d) { return d.precision == PI_FP64 ? 8 : 4; }
int64_t cells_of(const pi_grid_desc& d) { return (int64_t)d.n[0] * d.n[1] * d.n[2]; }

// tiles of every source's octants for tile edge T (as grid_host_init lists them)
int64_t tile_count(const pi_grid_desc& d, int T)
{
    if (d.source == PI_SRC_PLANE) return 0;
    int64_t k = 0;
    for (int s = 0; s < nsources(d); ++s) {
        const int32_t* v = source_vertex(d, s);
        for (int o = 0; o < 8; ++o) {
            int64_t c = 1;
            for (int a = 0; a < 3; ++a) {
                const int ext = ((o >> a) & 1) ? d.n[a] - v[a] : v[a];
                c *= ext > 0 ? (ext + T - 1) / T : 0;
            }
            k += c;
        }
    }
    return k;
}
}  // namespace

size_t grid_field_bytes(const pi_grid_desc& d)
{
    const size_t f = (size_t)cells_of(d) * word_of(d);
    const size_t ncol = (size_t)nsources(d);
    const size_t evolve = d.thermal == PI_T_EVOLVE ? 2 : 0;
    // nH, x, x_half, E, E_half; tau and tau_half one array per source
    return f * (3 + evolve + 2 * ncol);
}

size_t grid_private_bytes(const pi_grid_desc& d)
{
    const int64_t n = cells_of(d);
    const int64_t nblk = std::min<int64_t>((n + DT_BLOCK - 1) / DT_BLOCK, DT_MAX_BLOCKS);
    size_t b = sizeof(DevState) + sizeof(double) * NPART * (size_t)nblk;
    const size_t gd = d.precision == PI_FP64 ? sizeof(GridDev<double>) : sizeof(GridDev<float>);
    b += gd * (size_t)nsources(d);                 // grid table (one entry per source)
    b += sizeof(int) * 3 * 2;                      // launch prefix tables of one grid
    for (int w = 0; w < NSWEEP; ++w) b += sizeof(int4) * (size_t)tile_count(d, SWEEP_TILES[w]);
    b += sizeof(unsigned long long) * WORK_COUNTERS * WORK_SLOTS;
    if (d.precision == PI_MIXED || d.precision == PI_MIXED_FRONT)
        b += 3 * sizeof(unsigned int) + sizeof(long long) * (size_t)n;
    // persistent raytrace: octant table, a done-flag, a face-buffer slot and a
    // per-XCD list entry per tile, control block
    b += sizeof(int4) * 8 * (size_t)nsources(d) +
         (sizeof(unsigned) + sizeof(int4) +
          (size_t)FACE_BYTES * FACE_WORDS) *
             (size_t)tile_count(d, PERSIST_TILE) +
         sizeof(SweepCtl);
    if (d.spectrum == PI_SPEC_TABLE) b += sizeof(DevTable<double>) + sizeof(DevTable<float>);
    return b;
}

// -------------------------------------------------------------- checkpoints
namespace {
constexpr uint64_t CKPT_MAGIC = 0x31544b4350434950ull;   // "PICPCKT1"
struct CkptHeader {
    uint64_t magic;
    int32_t precision, thermal, nsrc, word;
    int32_t n[3], pad;
    int64_t ncell, nsteps;
    double t, dt, t_end, last_dt;
    int64_t payload;   // bytes after the header
};

int64_t ckpt_arrays(const pi_grid_desc& d)
{
    return 2 + (d.thermal == PI_T_EVOLVE ? 1 : 0) + nsources(d);
}

CkptHeader header_of(const pi_grid_desc& d)
{
    CkptHeader h{};
    h.magic = CKPT_MAGIC;
    h.precision = d.precision;
    h.thermal = d.thermal;
    h.nsrc = nsources(d);
    h.word = (int32_t)word_of(d);
    for (int a = 0; a < 3; ++a) h.n[a] = d.n[a];
    h.ncell = cells_of(d);
    h.payload = ckpt_arrays(d) * h.ncell * h.word;
    return h;
}
}  // namespace

size_t checkpoint_header_bytes() { return sizeof(CkptHeader); }

size_t checkpoint_bytes(const pi_grid_desc& d)
{
    return sizeof(CkptHeader) + (size_t)header_of(d).payload;
}

pi_status checkpoint_check(const pi_grid_desc& d, const void* buf, size_t bytes)
{
    if (!buf || bytes < sizeof(CkptHeader)) return fail(PI_EINVAL, "checkpoint too short");
    CkptHeader h;
    std::memcpy(&h, buf, sizeof(h));
    const CkptHeader w = header_of(d);
    if (h.magic != CKPT_MAGIC) return fail(PI_EINVAL, "not a checkpoint of this library");
    if (h.precision != w.precision || h.thermal != w.thermal || h.nsrc != w.nsrc ||
        h.word != w.word || h.n[0] != w.n[0] || h.n[1] != w.n[1] || h.n[2] != w.n[2])
        return fail(PI_EINVAL, "checkpoint layout (cells, precision, thermal mode or sources) "
                               "differs from the grid's");
    if (h.payload != w.payload || bytes < sizeof(CkptHeader) + (size_t)h.payload)
        return fail(PI_EINVAL, "checkpoint truncated");
    if (!std::isfinite(h.t) || !std::isfinite(h.t_end) || h.nsteps < 0)
        return fail(PI_EINVAL, "checkpoint clock is not valid");
    return PI_OK;
}

pi_status grid_save(const GridHost& g, void* buf, size_t bytes, hipStream_t s)
{
    const pi_grid_desc& d = g.d;
    if (!buf || bytes < checkpoint_bytes(d)) return fail(PI_EINVAL, "checkpoint buffer too small");
    CkptHeader h = header_of(d);
    DevState st{};
    HIP_OR(hipMemcpyAsync(&st, g.st, sizeof(st), hipMemcpyDeviceToHost, s), "clock read");
    char* p = static_cast<char*>(buf) + sizeof(CkptHeader);
    const size_t fb = (size_t)h.ncell * h.word;
    HIP_OR(hipMemcpyAsync(p, g.f.nH, fb, hipMemcpyDeviceToHost, s), "checkpoint read");
    p += fb;
    HIP_OR(hipMemcpyAsync(p, g.f.x, fb, hipMemcpyDeviceToHost, s), "checkpoint read");
    p += fb;
    if (d.thermal == PI_T_EVOLVE) {
        HIP_OR(hipMemcpyAsync(p, g.f.E, fb, hipMemcpyDeviceToHost, s), "checkpoint read");
        p += fb;
    }
    HIP_OR(hipMemcpyAsync(p, g.f.tau, fb * h.nsrc, hipMemcpyDeviceToHost, s), "checkpoint read");
    HIP_OR(hipStreamSynchronize(s), "checkpoint sync");
    h.t = st.t;
    h.dt = st.dt;
    h.t_end = st.t_end;
    h.last_dt = st.last_dt;
    h.nsteps = st.nsteps;
    std::memcpy(buf, &h, sizeof(h));
    return PI_OK;
}

pi_status grid_load(GridHost& g, const void* buf, size_t bytes, hipStream_t s)
{
    const pi_grid_desc& d = g.d;
    pi_status r = checkpoint_check(d, buf, bytes);
    if (r != PI_OK) return r;
    CkptHeader h;
    std::memcpy(&h, buf, sizeof(h));
    const char* p = static_cast<const char*>(buf) + sizeof(CkptHeader);
    const size_t fb = (size_t)h.ncell * h.word;
    HIP_OR(hipMemcpyAsync(g.f.nH, p, fb, hipMemcpyHostToDevice, s), "checkpoint write");
    p += fb;
    HIP_OR(hipMemcpyAsync(g.f.x, p, fb, hipMemcpyHostToDevice, s), "checkpoint write");
    p += fb;
    if (d.thermal == PI_T_EVOLVE) {
        HIP_OR(hipMemcpyAsync(g.f.E, p, fb, hipMemcpyHostToDevice, s), "checkpoint write");
        p += fb;
    }
    HIP_OR(hipMemcpyAsync(g.f.tau, p, fb * h.nsrc, hipMemcpyHostToDevice, s), "checkpoint write");
    DevState st{};
    HIP_OR(hipMemcpyAsync(&st, g.st, sizeof(st), hipMemcpyDeviceToHost, s), "clock read");
    HIP_OR(hipStreamSynchronize(s), "checkpoint sync");
    st.t = h.t;
    st.dt = h.dt;
    st.t_end = h.t_end;
    st.last_dt = h.last_dt;
    st.nsteps = h.nsteps;
    HIP_OR(hipMemcpyAsync(g.st, &st, sizeof(st), hipMemcpyHostToDevice, s), "clock write");
    HIP_OR(hipStreamSynchronize(s), "checkpoint sync");
    return PI_OK;
}

// ------------------------------------------------- entries of a lone grid
template <typename R> int raytrace_entries(const pi_grid_desc& d, const pi_fields& f, GridDev<R>* out)
{
    out[0] = base_entry<R>(d, f);
    const int ns = nsources(d);
    for (int s = 1; s < ns; ++s) out[s] = source_entry(out[0], d, s);
    return ns;
}
template int raytrace_entries<double>(const pi_grid_desc&, const pi_fields&, GridDev<double>*);
template int raytrace_entries<float>(const pi_grid_desc&, const pi_fields&, GridDev<float>*);

}  // namespace pi
