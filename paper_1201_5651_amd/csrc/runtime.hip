// runtime.hip -- C-ABI runtime of the photoionisation library (include/pi.h).
//
// Owns the per-grid device state (constants, rate table, tile schedule,
// reduction partials, clock) and composes the kernels into the operations of
// the ABI: the raytrace, the micro-physics update, the timestep, and the
// second-order (algorithm 3) and first-order (algorithm 2) steps of Sect. 2.2
// of Mackey (A&A 2012).  All device work is enqueued on the caller's stream.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstddef>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/pi.h"
#include "kernels.h"

using namespace pi;

namespace {

thread_local std::string g_err;

pi_status fail(pi_status s, const std::string& msg)
{
    g_err = msg;
    return s;
}

#define HIP_OR(expr, msg)                                                                          \
    do {                                                                                           \
        hipError_t e_ = (expr);                                                                    \
        if (e_ != hipSuccess)                                                                      \
            return fail(PI_EDEVICE, std::string(msg) + ": " + hipGetErrorString(e_));              \
    } while (0)

// --------------------------------------------------------- blackbody table
// Photon number spectrum of a blackbody above the threshold, u = h nu / k T:
// dN/du ~ u^2 / (e^u - 1).  Integrals by Richardson-extrapolated composite
// Simpson on [u0, u0 + 150].
struct BBIntegrand {
    double u0, tau;
    int moment;      // 0: photons, 1: excess energy (u - u0)
    bool weighted;   // multiply by sigma_nu / sigma0 = (u0/u)^3
    double operator()(double u) const
    {
        const double s = (u0 / u) * (u0 / u) * (u0 / u);
        double v = u * u / std::expm1(u) * std::exp(-tau * s);
        if (moment == 1) v *= (u - u0);
        if (weighted) v *= s;
        return v;
    }
};

// Composite Simpson with a compensated (Neumaier) sum.
double simpson(const BBIntegrand& f, double a, double b, int n)
{
    const double h = (b - a) / n;
    double s = f(a) + f(b), c = 0.0;
    for (int i = 1; i < n; ++i) {
        const double v = (i & 1 ? 4.0 : 2.0) * f(a + i * h);
        const double t = s + v;
        c += std::fabs(s) >= std::fabs(v) ? (s - t) + v : (v - t) + s;
        s = t;
    }
    return (s + c) * h / 3.0;
}

// Composite Simpson on n and 2n intervals with one Richardson step (error h^6).
double quad(const BBIntegrand& f, double a, double b, int n)
{
    const double s1 = simpson(f, a, b, n), s2 = simpson(f, a, b, 2 * n);
    return s2 + (s2 - s1) / 15.0;
}

int octant_count(const pi_grid_desc& d)
{
    int noct = 0;
    for (int o = 0; o < 8; ++o) {
        bool ok = true;
        for (int a = 0; a < 3; ++a) {
            const int ext = ((o >> a) & 1) ? d.n[a] - d.src[a] : d.src[a];
            ok = ok && ext > 0;
        }
        noct += ok;
    }
    return noct;
}

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
    for (int j = 0; j < PI_NTAB; ++j) {
        if (j == 0 || P[j] <= 0 || H[j] <= 0) {
            T.lp[j] = T.mp[j] = T.lh[j] = T.mh[j] = R(0);
            continue;
        }
        T.lp[j] = R(std::log(P[j] / P[0]));
        T.mp[j] = R(-tn[j] * P1[j] / P[j]);
        T.lh[j] = R(std::log(H[j] / H[0]));
        T.mh[j] = R(-tn[j] * H1[j] / H[j]);
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
    p.QV = R(d.Q / (d.dx * d.dx * d.dx));
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

}  // namespace

struct pi_grid {
    pi_grid_desc d;
    pi_fields f;
    bool fp64;
    bool mixed;                  // float bulk pass + double re-solve of listed cells
    Params<double> pd;
    Params<float> pf;
    DevTable<double>* table_d = nullptr;   // FP64 and MIXED
    DevTable<float>* table_f = nullptr;    // FP32 and MIXED
    int* fix_list = nullptr;               // MIXED: cells for the double re-solve (ncell)
    int fix_blocks = 0;
    DevState* st = nullptr;
    unsigned long long* work = nullptr;   // WORK_COUNTERS x WORK_SLOTS
    double* part = nullptr;
    int nblk = 0;
    int4* tiles = nullptr;
    std::vector<int> stage_first, stage_count;
    int noct = 0;
    double cell_vol = 0;
};

namespace {

pi_status validate(const pi_grid_desc* d, const pi_fields* f)
{
    if (!d || !f) return fail(PI_EINVAL, "null descriptor or fields");
    for (int a = 0; a < 3; ++a) {
        if (d->n[a] < 1) return fail(PI_EINVAL, "n[d] must be >= 1");
        if (d->src[a] < 0 || d->src[a] > d->n[a]) return fail(PI_EINVAL, "source vertex outside [0, n]");
    }
    const double N = (double)d->n[0] * d->n[1] * d->n[2];
    if (N >= 2147483647.0) return fail(PI_EINVAL, "grid larger than 2^31 - 1 cells");
    if (!(d->dx > 0) || !std::isfinite(d->dx)) return fail(PI_EINVAL, "dx must be > 0");
    if (!(d->Q >= 0) || !std::isfinite(d->Q)) return fail(PI_EINVAL, "Q must be >= 0");
    if (!(d->sigma0 > 0)) return fail(PI_EINVAL, "sigma0 must be > 0");
    if (d->spectrum != PI_SPEC_MONO && d->spectrum != PI_SPEC_TABLE) return fail(PI_EINVAL, "spectrum");
    if (d->spectrum == PI_SPEC_TABLE && !(d->T_bb > 0)) return fail(PI_EINVAL, "T_bb must be > 0");
    if (!(d->e_excess >= 0)) return fail(PI_EINVAL, "e_excess must be >= 0");
    if (d->thermal != PI_T_FIXED && d->thermal != PI_T_EVOLVE) return fail(PI_EINVAL, "thermal");
    if (d->thermal == PI_T_FIXED && !(d->T_fixed > 0)) return fail(PI_EINVAL, "T_fixed must be > 0");
    if (d->recomb != PI_ALPHA_CONST && d->recomb != PI_ALPHA_POWER) return fail(PI_EINVAL, "recomb");
    if (!(d->alpha_B >= 0)) return fail(PI_EINVAL, "alpha_B must be >= 0");
    if (d->weights != PI_W_GEOMETRIC && d->weights != PI_W_MELLEMA) return fail(PI_EINVAL, "weights");
    if (d->n_sub < 1 || d->n_sub > 64) return fail(PI_EINVAL, "n_sub must be in 1..64");
    for (int i = 0; i < 4; ++i)
        if (!(d->K[i] >= 0)) return fail(PI_EINVAL, "K factors must be >= 0 (inf disables)");
    if (d->precision != PI_FP64 && d->precision != PI_FP32 && d->precision != PI_MIXED)
        return fail(PI_EINVAL, "precision");
    if (!f->nH || !f->x || !f->tau || !f->x_half || !f->tau_half)
        return fail(PI_EINVAL, "nH, x, tau, x_half and tau_half are required");
    if (d->thermal == PI_T_EVOLVE && (!f->E || !f->E_half))
        return fail(PI_EINVAL, "E and E_half are required when the temperature evolves");
    return PI_OK;
}

void free_grid(pi_grid* g)
{
    if (!g) return;
    if (g->table_d) (void)hipFree(g->table_d);
    if (g->table_f) (void)hipFree(g->table_f);
    if (g->fix_list) (void)hipFree(g->fix_list);
    if (g->st) (void)hipFree(g->st);
    if (g->work) (void)hipFree(g->work);
    if (g->part) (void)hipFree(g->part);
    if (g->tiles) (void)hipFree(g->tiles);
    delete g;
}

template <typename R> const R* cp(const void* v) { return static_cast<const R*>(v); }
template <typename R> R* mp(void* v) { return static_cast<R*>(v); }

template <typename R> const Params<R>& params(const pi_grid* g);
template <> const Params<double>& params<double>(const pi_grid* g) { return g->pd; }
template <> const Params<float>& params<float>(const pi_grid* g) { return g->pf; }

template <typename R> pi_status raytrace_t(pi_grid* g, int state, int tau_buf, hipStream_t s)
{
    const R* x = cp<R>(state == PI_BUF_HALF ? g->f.x_half : g->f.x);
    R* tau = mp<R>(tau_buf == PI_BUF_HALF ? g->f.tau_half : g->f.tau);
    const R* nH = cp<R>(g->f.nH);
    for (size_t k = 0; k < g->stage_first.size(); ++k)
        HIP_OR(launch_sweep_stage<R>(params<R>(g), nH, x, tau, g->tiles, g->stage_first[k],
                                     g->stage_count[k], s),
               "raytrace launch");
    return PI_OK;
}

template <typename R>
pi_status chem_t(pi_grid* g, bool dev_dt, double h, int tau_buf, int from, int to, hipStream_t s)
{
    const R* nH = cp<R>(g->f.nH);
    const R* x0 = cp<R>(from == PI_BUF_HALF ? g->f.x_half : g->f.x);
    const R* E0 = cp<R>(from == PI_BUF_HALF ? g->f.E_half : g->f.E);
    R* x1 = mp<R>(to == PI_BUF_HALF ? g->f.x_half : g->f.x);
    R* E1 = mp<R>(to == PI_BUF_HALF ? g->f.E_half : g->f.E);
    const R* tau = cp<R>(tau_buf == PI_BUF_HALF ? g->f.tau_half : g->f.tau);
    if (g->d.thermal == PI_T_FIXED) {
        E0 = nullptr;
        E1 = nullptr;
    }
    HIP_OR(launch_chem<R>(params<R>(g), nH, x0, E0, tau, x1, E1, g->st, dev_dt, h, g->work,
                          g->mixed ? g->fix_list : nullptr, s),
           "chemistry launch");
    if (g->mixed)
        HIP_OR(launch_chem_fix(g->pd, cp<float>(nH), cp<float>(x0), cp<float>(E0), cp<float>(tau),
                               mp<float>(x1), mp<float>(E1), g->st, dev_dt, h, g->work,
                               g->fix_list, g->fix_blocks, s),
               "double re-solve launch");
    return PI_OK;
}

template <typename R> pi_status timestep_t(pi_grid* g, double t_end, hipStream_t s)
{
    const R* E = g->d.thermal == PI_T_EVOLVE ? cp<R>(g->f.E) : nullptr;
    HIP_OR(launch_dtdiag<R>(params<R>(g), cp<R>(g->f.nH), cp<R>(g->f.x), E, cp<R>(g->f.tau),
                            g->part, g->nblk, g->st, t_end, g->cell_vol, g->noct, s),
           "timestep launch");
    return PI_OK;
}

template <typename R> pi_status step_t(pi_grid* g, double t_end, int order, hipStream_t s)
{
    pi_status r = timestep_t<R>(g, t_end, s);
    if (r != PI_OK) return r;
    if (order == 2) {
        if ((r = chem_t<R>(g, true, 0.5, PI_BUF_N, PI_BUF_N, PI_BUF_HALF, s)) != PI_OK) return r;
        if ((r = raytrace_t<R>(g, PI_BUF_HALF, PI_BUF_HALF, s)) != PI_OK) return r;
        if ((r = chem_t<R>(g, true, 1.0, PI_BUF_HALF, PI_BUF_N, PI_BUF_N, s)) != PI_OK) return r;
    } else {
        if ((r = chem_t<R>(g, true, 1.0, PI_BUF_N, PI_BUF_N, PI_BUF_N, s)) != PI_OK) return r;
    }
    if ((r = raytrace_t<R>(g, PI_BUF_N, PI_BUF_N, s)) != PI_OK) return r;
    HIP_OR(launch_advance(g->st, s), "advance launch");
    return PI_OK;
}

}  // namespace

extern "C" {

int pi_abi_version(void) { return PI_ABI_VERSION; }

const char* pi_last_error(void) { return g_err.c_str(); }

pi_status pi_table_build(double T_bb, double Q, double* out)
{
    if (!out || !(T_bb > 0) || !(Q >= 0)) return fail(PI_EINVAL, "pi_table_build: bad argument");
    const double kB = 1.380649e-16, eV = 1.602176634e-12;
    const double kT = kB * T_bb;
    const double u0 = 13.6 * eV / kT;
    const double ub = u0 + 150.0;
    const int nint = 40000;
    BBIntegrand f{ u0, 0.0, 0, false };
    const double norm = quad(f, u0, ub, nint);
    out[0] = 0.0;
    for (int j = 1; j < PI_NTAB; ++j) out[j] = 1e-4 * std::pow(10.0, 8.0 * (j - 1) / 62.0);
    for (int j = 0; j < PI_NTAB; ++j) {
        const double tau = out[j];
        out[PI_NTAB + j] = Q * quad({ u0, tau, 0, false }, u0, ub, nint) / norm;
        out[2 * PI_NTAB + j] = Q * quad({ u0, tau, 0, true }, u0, ub, nint) / norm;
        out[3 * PI_NTAB + j] = Q * kT * quad({ u0, tau, 1, false }, u0, ub, nint) / norm;
        out[4 * PI_NTAB + j] = Q * kT * quad({ u0, tau, 1, true }, u0, ub, nint) / norm;
    }
    return PI_OK;
}

pi_status pi_grid_create(const pi_grid_desc* desc, const pi_fields* fields, pi_grid** out)
{
    if (!out) return fail(PI_EINVAL, "null output pointer");
    *out = nullptr;
    pi_status v = validate(desc, fields);
    if (v != PI_OK) return v;
    pi_grid* g = new pi_grid();
    g->d = *desc;
    g->f = *fields;
    g->fp64 = desc->precision == PI_FP64;
    g->mixed = desc->precision == PI_MIXED;
    g->pd = make_params<double>(*desc);
    g->pf = make_params<float>(*desc);
    g->noct = octant_count(*desc);
    g->cell_vol = desc->dx * desc->dx * desc->dx;

    auto bail = [&](pi_status s, const std::string& m) {
        free_grid(g);
        return fail(s, m);
    };
    // rate table (normalised, log-Hermite form) for the kernels
    {
        std::vector<double> raw(5 * PI_NTAB, 0.0);
        if (desc->spectrum == PI_SPEC_TABLE) pi_table_build(desc->T_bb, desc->Q > 0 ? desc->Q : 1.0, raw.data());
        const double Qn = desc->Q > 0 ? desc->Q : 1.0;
        if (g->fp64 || g->mixed) {
            DevTable<double> T{};
            if (desc->spectrum == PI_SPEC_TABLE) fill_table(T, raw.data(), Qn);
            if (hipMalloc(&g->table_d, sizeof(T)) != hipSuccess) return bail(PI_ENOMEM, "table allocation");
            if (hipMemcpy(g->table_d, &T, sizeof(T), hipMemcpyHostToDevice) != hipSuccess)
                return bail(PI_EDEVICE, "table upload");
        }
        if (!g->fp64) {
            DevTable<float> T{};
            if (desc->spectrum == PI_SPEC_TABLE) fill_table(T, raw.data(), Qn);
            if (hipMalloc(&g->table_f, sizeof(T)) != hipSuccess) return bail(PI_ENOMEM, "table allocation");
            if (hipMemcpy(g->table_f, &T, sizeof(T), hipMemcpyHostToDevice) != hipSuccess)
                return bail(PI_EDEVICE, "table upload");
        }
        g->pd.tab = g->table_d;
        g->pf.tab = g->table_f;
    }
    // clock
    if (hipMalloc(&g->st, sizeof(DevState)) != hipSuccess) return bail(PI_ENOMEM, "state allocation");
    {
        DevState s0{};
        if (hipMemcpy(g->st, &s0, sizeof(s0), hipMemcpyHostToDevice) != hipSuccess)
            return bail(PI_EDEVICE, "state upload");
    }
    // work counters
    {
        const size_t wb = sizeof(unsigned long long) * WORK_COUNTERS * WORK_SLOTS;
        if (hipMalloc(&g->work, wb) != hipSuccess) return bail(PI_ENOMEM, "counter allocation");
        if (hipMemset(g->work, 0, wb) != hipSuccess) return bail(PI_EDEVICE, "counter clear");
    }
    // reduction partials
    const int64_t N = (int64_t)desc->n[0] * desc->n[1] * desc->n[2];
    // mixed precision: list of cells for the double re-solve
    if (g->mixed) {
        if (hipMalloc(&g->fix_list, sizeof(int) * N) != hipSuccess)
            return bail(PI_ENOMEM, "re-solve list allocation");
        g->fix_blocks = (int)std::min<int64_t>((N + 255) / 256, 2048);
    }
    g->nblk = (int)std::min<int64_t>((N + 255) / 256, 1024);
    if (hipMalloc(&g->part, sizeof(double) * NPART * g->nblk) != hipSuccess)
        return bail(PI_ENOMEM, "partials allocation");
    // tile schedule: every octant's tiles, grouped by tile diagonal tx+ty+tz
    {
        std::vector<std::vector<int4>> by_stage;
        for (int o = 0; o < 8; ++o) {
            int ext[3];
            for (int a = 0; a < 3; ++a) ext[a] = ((o >> a) & 1) ? desc->n[a] - desc->src[a] : desc->src[a];
            if (ext[0] <= 0 || ext[1] <= 0 || ext[2] <= 0) continue;
            const int ntx = (ext[0] + SWEEP_T - 1) / SWEEP_T;
            const int nty = (ext[1] + SWEEP_T - 1) / SWEEP_T;
            const int ntz = (ext[2] + SWEEP_T - 1) / SWEEP_T;
            for (int tz = 0; tz < ntz; ++tz)
                for (int ty = 0; ty < nty; ++ty)
                    for (int tx = 0; tx < ntx; ++tx) {
                        const int D = tx + ty + tz;
                        if ((int)by_stage.size() <= D) by_stage.resize(D + 1);
                        by_stage[D].push_back(make_int4(o, tx, ty, tz));
                    }
        }
        std::vector<int4> flat;
        for (auto& v : by_stage) {
            g->stage_first.push_back((int)flat.size());
            g->stage_count.push_back((int)v.size());
            flat.insert(flat.end(), v.begin(), v.end());
        }
        if (!flat.empty()) {
            if (hipMalloc(&g->tiles, sizeof(int4) * flat.size()) != hipSuccess)
                return bail(PI_ENOMEM, "tile schedule allocation");
            if (hipMemcpy(g->tiles, flat.data(), sizeof(int4) * flat.size(), hipMemcpyHostToDevice) !=
                hipSuccess)
                return bail(PI_EDEVICE, "tile schedule upload");
        }
    }
    *out = g;
    return PI_OK;
}

pi_status pi_grid_destroy(pi_grid* g)
{
    if (!g) return PI_OK;
    (void)hipDeviceSynchronize();
    free_grid(g);
    return PI_OK;
}

pi_status pi_raytrace(pi_grid* g, int state, int tau_buf, void* stream)
{
    if (!g) return fail(PI_EINVAL, "null grid");
    if ((state != PI_BUF_N && state != PI_BUF_HALF) || (tau_buf != PI_BUF_N && tau_buf != PI_BUF_HALF))
        return fail(PI_EINVAL, "buffer selector");
    hipStream_t s = static_cast<hipStream_t>(stream);
    return g->fp64 ? raytrace_t<double>(g, state, tau_buf, s) : raytrace_t<float>(g, state, tau_buf, s);
}

pi_status pi_chem_step(pi_grid* g, int use_device_dt, double h_value, int tau_buf, int from_state,
                       int to_state, void* stream)
{
    if (!g) return fail(PI_EINVAL, "null grid");
    if (!(h_value >= 0) || !std::isfinite(h_value)) return fail(PI_EINVAL, "h must be finite and >= 0");
    for (int b : { tau_buf, from_state, to_state })
        if (b != PI_BUF_N && b != PI_BUF_HALF) return fail(PI_EINVAL, "buffer selector");
    hipStream_t s = static_cast<hipStream_t>(stream);
    return g->fp64 ? chem_t<double>(g, use_device_dt != 0, h_value, tau_buf, from_state, to_state, s)
                   : chem_t<float>(g, use_device_dt != 0, h_value, tau_buf, from_state, to_state, s);
}

pi_status pi_timestep(pi_grid* g, double t_end, void* stream)
{
    if (!g) return fail(PI_EINVAL, "null grid");
    if (!std::isfinite(t_end)) return fail(PI_EINVAL, "t_end must be finite");
    hipStream_t s = static_cast<hipStream_t>(stream);
    return g->fp64 ? timestep_t<double>(g, t_end, s) : timestep_t<float>(g, t_end, s);
}

pi_status pi_step_o2(pi_grid* g, double t_end, void* stream)
{
    if (!g) return fail(PI_EINVAL, "null grid");
    if (!std::isfinite(t_end)) return fail(PI_EINVAL, "t_end must be finite");
    hipStream_t s = static_cast<hipStream_t>(stream);
    return g->fp64 ? step_t<double>(g, t_end, 2, s) : step_t<float>(g, t_end, 2, s);
}

pi_status pi_step_o1(pi_grid* g, double t_end, void* stream)
{
    if (!g) return fail(PI_EINVAL, "null grid");
    if (!std::isfinite(t_end)) return fail(PI_EINVAL, "t_end must be finite");
    hipStream_t s = static_cast<hipStream_t>(stream);
    return g->fp64 ? step_t<double>(g, t_end, 1, s) : step_t<float>(g, t_end, 1, s);
}

pi_status pi_init_energy(pi_grid* g, double T0, int state, void* stream)
{
    if (!g) return fail(PI_EINVAL, "null grid");
    if (!(T0 > 0)) return fail(PI_EINVAL, "T0 must be > 0");
    if (g->d.thermal != PI_T_EVOLVE) return PI_OK;
    hipStream_t s = static_cast<hipStream_t>(stream);
    void* E = state == PI_BUF_HALF ? g->f.E_half : g->f.E;
    const void* x = state == PI_BUF_HALF ? g->f.x_half : g->f.x;
    const int64_t n = g->pd.ncell;
    if (g->fp64)
        HIP_OR(launch_energy<double>(n, cp<double>(g->f.nH), cp<double>(x), mp<double>(E), T0, s),
               "energy launch");
    else
        HIP_OR(launch_energy<float>(n, cp<float>(g->f.nH), cp<float>(x), mp<float>(E), T0, s),
               "energy launch");
    return PI_OK;
}

pi_status pi_set_time(pi_grid* g, double t, int64_t nsteps, void* stream)
{
    if (!g) return fail(PI_EINVAL, "null grid");
    if (!std::isfinite(t)) return fail(PI_EINVAL, "t must be finite");
    hipStream_t s = static_cast<hipStream_t>(stream);
    // copied from a stack buffer: wait before returning
    DevState h{};
    HIP_OR(hipMemcpyAsync(&h, g->st, sizeof(h), hipMemcpyDeviceToHost, s), "state read");
    HIP_OR(hipStreamSynchronize(s), "state read sync");
    h.t = t;
    h.nsteps = nsteps;
    h.dt = 0;
    HIP_OR(hipMemcpyAsync(g->st, &h, sizeof(h), hipMemcpyHostToDevice, s), "state write");
    HIP_OR(hipStreamSynchronize(s), "state write sync");
    return PI_OK;
}

pi_status pi_grid_state(pi_grid* g, double* t, int64_t* nsteps, double* last_dt, void* stream)
{
    if (!g) return fail(PI_EINVAL, "null grid");
    hipStream_t s = static_cast<hipStream_t>(stream);
    DevState h{};
    HIP_OR(hipMemcpyAsync(&h, g->st, sizeof(h), hipMemcpyDeviceToHost, s), "state read");
    HIP_OR(hipStreamSynchronize(s), "state read sync");
    if (t) *t = h.t;
    if (nsteps) *nsteps = h.nsteps;
    if (last_dt) *last_dt = h.last_dt;
    return PI_OK;
}

pi_status pi_work_counters(pi_grid* g, int64_t* out, int reset, void* stream)
{
    if (!g || !out) return fail(PI_EINVAL, "null argument");
    hipStream_t s = static_cast<hipStream_t>(stream);
    unsigned long long h[WORK_COUNTERS * WORK_SLOTS];
    HIP_OR(hipMemcpyAsync(h, g->work, sizeof(h), hipMemcpyDeviceToHost, s), "counter read");
    HIP_OR(hipStreamSynchronize(s), "counter read sync");
    for (int c = 0; c < WORK_COUNTERS; ++c) {
        unsigned long long v = 0;
        for (int k = 0; k < WORK_SLOTS; ++k) v += h[c * WORK_SLOTS + k];
        out[c] = (int64_t)v;
    }
    if (reset) {
        HIP_OR(hipMemsetAsync(g->work, 0, sizeof(h), s), "counter clear");
        HIP_OR(hipStreamSynchronize(s), "counter clear sync");
    }
    return PI_OK;
}

pi_status pi_diagnostics(pi_grid* g, double* out, void* stream)
{
    if (!g || !out) return fail(PI_EINVAL, "null argument");
    hipStream_t s = static_cast<hipStream_t>(stream);
    DevState h{};
    HIP_OR(hipMemcpyAsync(&h, g->st, sizeof(h), hipMemcpyDeviceToHost, s), "state read");
    HIP_OR(hipStreamSynchronize(s), "state read sync");
    // recompute on the current state without disturbing the clock or dt
    const double t_end_keep = h.t_end, dt_keep = h.dt;
    pi_status r = g->fp64 ? timestep_t<double>(g, h.t + 1.0, s) : timestep_t<float>(g, h.t + 1.0, s);
    if (r != PI_OK) return r;
    DevState h2{};
    HIP_OR(hipMemcpyAsync(&h2, g->st, sizeof(h2), hipMemcpyDeviceToHost, s), "state read");
    HIP_OR(hipStreamSynchronize(s), "state read sync");
    for (int i = 0; i < PI_NDIAG; ++i) out[i] = h2.diag[i];
    h2.t_end = t_end_keep;
    h2.dt = dt_keep;
    HIP_OR(hipMemcpyAsync(g->st, &h2, sizeof(h2), hipMemcpyHostToDevice, s), "state restore");
    HIP_OR(hipStreamSynchronize(s), "state restore sync");
    if (h2.diag[5] > 0) return fail(PI_ENAN, "non-finite values in the grid state");
    return PI_OK;
}

}  // extern "C"
