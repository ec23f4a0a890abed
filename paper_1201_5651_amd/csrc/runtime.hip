// runtime.hip -- C-ABI entry points of the photoionisation library
// (include/pi.h): descriptor validation, the host-built blackbody rate table,
// the single-grid calls (an engine over one grid) and the batch calls (an
// engine over many grids, one launch per kernel for all of them).  All device
// work is enqueued on the caller's stream.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstddef>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/pi.h"
#include "engine.h"
#include "kernels.h"

namespace pi {

namespace {
thread_local std::string g_err;
}

pi_status fail(pi_status s, const std::string& msg)
{
    g_err = msg;
    return s;
}

const std::string& last_error() { return g_err; }

pi_status validate_desc(const pi_grid_desc* d)
{
    if (!d) return fail(PI_EINVAL, "null descriptor");
    if (d->source != PI_SRC_POINT && d->source != PI_SRC_PLANE) return fail(PI_EINVAL, "source");
    for (int a = 0; a < 3; ++a) {
        if (d->n[a] < 1) return fail(PI_EINVAL, "n[d] must be >= 1");
        if (d->source == PI_SRC_POINT && (d->src[a] < 0 || d->src[a] > d->n[a]))
            return fail(PI_EINVAL, "source vertex outside [0, n]");
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
    // a zero factor would make eq. (4) give dt = 0 and the clock could never
    // advance
    for (int i = 0; i < 4; ++i)
        if (!(d->K[i] > 0)) return fail(PI_EINVAL, "K factors must be > 0 (inf disables)");
    if (d->precision != PI_FP64 && d->precision != PI_FP32 && d->precision != PI_MIXED &&
        d->precision != PI_MIXED_FRONT)
        return fail(PI_EINVAL, "precision");
    if (d->nsrc < 0 || d->nsrc > PI_MAX_SRC) return fail(PI_EINVAL, "nsrc must be in 0..PI_MAX_SRC");
    if (d->nsrc > 1) {
        if (d->source != PI_SRC_POINT) return fail(PI_EINVAL, "several sources must be point sources");
        for (int s = 0; s < d->nsrc - 1; ++s) {
            for (int a = 0; a < 3; ++a)
                if (d->src_more[s][a] < 0 || d->src_more[s][a] > d->n[a])
                    return fail(PI_EINVAL, "source vertex outside [0, n]");
            if (!(d->Q_more[s] >= 0) || !std::isfinite(d->Q_more[s]))
                return fail(PI_EINVAL, "Q of every source must be >= 0");
        }
    }
    return PI_OK;
}

pi_status validate_fields(const pi_grid_desc* d, const pi_fields* f)
{
    if (!f) return fail(PI_EINVAL, "null fields");
    if (!f->nH || !f->x || !f->tau || !f->x_half || !f->tau_half)
        return fail(PI_EINVAL, "nH, x, tau, x_half and tau_half are required");
    if (d->thermal == PI_T_EVOLVE && (!f->E || !f->E_half))
        return fail(PI_EINVAL, "E and E_half are required when the temperature evolves");
    return PI_OK;
}

}  // namespace pi

using namespace pi;

namespace {

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

bool buf_ok(int b) { return b == PI_BUF_N || b == PI_BUF_HALF; }

}  // namespace

// A single grid: an engine over one grid.
struct pi_grid {
    GridHost h;
    Engine e;
};

// A batch: an engine over the grids of the batch.
struct pi_batch {
    std::vector<GridHost> h;
    Engine e;
};

extern "C" {

int pi_abi_version(void) { return PI_ABI_VERSION; }

const char* pi_last_error(void) { return last_error().c_str(); }

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

// ------------------------------------------------------------------- grid
pi_status pi_grid_create(const pi_grid_desc* desc, const pi_fields* fields, pi_grid** out)
{
    if (!out) return fail(PI_EINVAL, "null output pointer");
    *out = nullptr;
    pi_status v = validate_desc(desc);
    if (v != PI_OK) return v;
    if ((v = validate_fields(desc, fields)) != PI_OK) return v;
    pi_grid* g = new pi_grid();
    g->e.precision = desc->precision;
    if ((v = grid_host_init(g->h, *desc, *fields)) != PI_OK) {
        delete g;
        return v;
    }
    if ((v = engine_build(g->e, { &g->h })) != PI_OK) {
        engine_free(g->e);
        grid_host_free(g->h);
        delete g;
        return v;
    }
    *out = g;
    return PI_OK;
}

pi_status pi_grid_destroy(pi_grid* g)
{
    if (!g) return PI_OK;
    (void)hipDeviceSynchronize();
    engine_free(g->e);
    grid_host_free(g->h);
    delete g;
    return PI_OK;
}

pi_status pi_raytrace(pi_grid* g, int state, int tau_buf, void* stream)
{
    if (!g) return fail(PI_EINVAL, "null grid");
    if (!buf_ok(state) || !buf_ok(tau_buf)) return fail(PI_EINVAL, "buffer selector");
    return engine_raytrace(g->e, state, tau_buf, static_cast<hipStream_t>(stream));
}

pi_status pi_chem_step(pi_grid* g, int use_device_dt, double h_value, int tau_buf, int from_state,
                       int to_state, void* stream)
{
    if (!g) return fail(PI_EINVAL, "null grid");
    if (!(h_value >= 0) || !std::isfinite(h_value)) return fail(PI_EINVAL, "h must be finite and >= 0");
    if (!buf_ok(tau_buf) || !buf_ok(from_state) || !buf_ok(to_state))
        return fail(PI_EINVAL, "buffer selector");
    return engine_chem(g->e, use_device_dt != 0, h_value, tau_buf, from_state, to_state,
                       static_cast<hipStream_t>(stream));
}

pi_status pi_chem_raytrace(pi_grid* g, int use_device_dt, double h_value, int tau_buf,
                           int from_state, int to_state, int tau_out, void* stream)
{
    if (!g) return fail(PI_EINVAL, "null grid");
    if (!(h_value >= 0) || !std::isfinite(h_value)) return fail(PI_EINVAL, "h must be finite and >= 0");
    if (!buf_ok(tau_buf) || !buf_ok(from_state) || !buf_ok(to_state) || !buf_ok(tau_out))
        return fail(PI_EINVAL, "buffer selector");
    return engine_chem_raytrace(g->e, use_device_dt != 0, h_value, tau_buf, from_state, to_state,
                                tau_out, static_cast<hipStream_t>(stream));
}

pi_status pi_timestep(pi_grid* g, double t_end, void* stream)
{
    if (!g) return fail(PI_EINVAL, "null grid");
    if (!std::isfinite(t_end)) return fail(PI_EINVAL, "t_end must be finite");
    return engine_timestep(g->e, t_end, static_cast<hipStream_t>(stream));
}

pi_status pi_step_o2(pi_grid* g, double t_end, void* stream)
{
    if (!g) return fail(PI_EINVAL, "null grid");
    if (!std::isfinite(t_end)) return fail(PI_EINVAL, "t_end must be finite");
    hipStream_t s = static_cast<hipStream_t>(stream);
    // Inside a caller's capture the kernels are launched directly (they become
    // nodes of the caller's graph); otherwise the step is replayed from the
    // grid's own captured graph, which reads t_end from the clock.
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(s, &cs) != hipSuccess) return fail(PI_EDEVICE, "capture query");
    if (cs != hipStreamCaptureStatusNone) return engine_step(g->e, t_end, 2, s);
    if (launch_set_t_end(g->h.st, t_end, s) != hipSuccess) return fail(PI_EDEVICE, "clock launch");
    return engine_step_graph(g->e, s);
}

pi_status pi_step_o1(pi_grid* g, double t_end, void* stream)
{
    if (!g) return fail(PI_EINVAL, "null grid");
    if (!std::isfinite(t_end)) return fail(PI_EINVAL, "t_end must be finite");
    return engine_step(g->e, t_end, 1, static_cast<hipStream_t>(stream));
}

pi_status pi_step_a1(pi_grid* g, double t_end, void* stream)
{
    if (!g) return fail(PI_EINVAL, "null grid");
    if (!std::isfinite(t_end)) return fail(PI_EINVAL, "t_end must be finite");
    return engine_step_a1(g->e, t_end, static_cast<hipStream_t>(stream));
}

pi_status pi_init_energy(pi_grid* g, double T0, int state, void* stream)
{
    if (!g) return fail(PI_EINVAL, "null grid");
    if (!(T0 > 0)) return fail(PI_EINVAL, "T0 must be > 0");
    if (!buf_ok(state)) return fail(PI_EINVAL, "buffer selector");
    return engine_init_energy(g->e, 0, T0, state, static_cast<hipStream_t>(stream));
}

pi_status pi_set_time(pi_grid* g, double t, int64_t nsteps, void* stream)
{
    if (!g) return fail(PI_EINVAL, "null grid");
    if (!std::isfinite(t)) return fail(PI_EINVAL, "t must be finite");
    hipStream_t s = static_cast<hipStream_t>(stream);
    std::vector<DevState> st;
    pi_status r = engine_read_states(g->e, st, s);
    if (r != PI_OK) return r;
    st[0].t = t;
    st[0].nsteps = nsteps;
    st[0].dt = 0;
    return engine_write_states(g->e, st, s);
}

pi_status pi_grid_state(pi_grid* g, double* t, int64_t* nsteps, double* last_dt, void* stream)
{
    if (!g) return fail(PI_EINVAL, "null grid");
    std::vector<DevState> st;
    pi_status r = engine_read_states(g->e, st, static_cast<hipStream_t>(stream));
    if (r != PI_OK) return r;
    if (t) *t = st[0].t;
    if (nsteps) *nsteps = st[0].nsteps;
    if (last_dt) *last_dt = st[0].last_dt;
    return PI_OK;
}

pi_status pi_grid_required_bytes(const pi_grid_desc* desc, size_t* field_bytes,
                                 size_t* work_bytes)
{
    pi_status v = validate_desc(desc);
    if (v != PI_OK) return v;
    if (field_bytes) *field_bytes = grid_field_bytes(*desc);
    if (work_bytes) *work_bytes = grid_private_bytes(*desc);
    return PI_OK;
}

pi_status pi_grid_save(pi_grid* g, void* host_buf, size_t bytes, size_t* needed, void* stream)
{
    if (!g) return fail(PI_EINVAL, "null grid");
    const size_t need = checkpoint_bytes(g->h.d);
    if (needed) *needed = need;
    if (!host_buf) return PI_OK;   // size query
    if (bytes < need) return fail(PI_EINVAL, "checkpoint buffer too small");
    return grid_save(g->h, host_buf, bytes, static_cast<hipStream_t>(stream));
}

pi_status pi_grid_load(pi_grid* g, const void* host_buf, size_t bytes, void* stream)
{
    if (!g || !host_buf) return fail(PI_EINVAL, "null argument");
    return grid_load(g->h, host_buf, bytes, static_cast<hipStream_t>(stream));
}

pi_status pi_work_counters(pi_grid* g, int64_t* out, int reset, void* stream)
{
    if (!g || !out) return fail(PI_EINVAL, "null argument");
    return engine_work(g->e, out, reset, static_cast<hipStream_t>(stream));
}

pi_status pi_diagnostics(pi_grid* g, double* out, void* stream)
{
    if (!g || !out) return fail(PI_EINVAL, "null argument");
    std::vector<double> d;
    pi_status r = engine_diagnostics(g->e, d, static_cast<hipStream_t>(stream));
    if (!d.empty())
        for (int i = 0; i < PI_NDIAG; ++i) out[i] = d[i];
    return r;
}

namespace {
pi_status set_tile(Engine& e, int edge)
{
    if (edge == 0) {
        e.sweep = -1;
    } else if (edge == PI_TILE_PERSISTENT) {
        e.sweep = SWEEP_PERSIST;
    } else {
        int w = -1;
        for (int k = 0; k < NSWEEP; ++k)
            if (SWEEP_TILES[k] == edge) w = k;
        if (w < 0)
            return fail(PI_EINVAL, "raytrace tile edge must be 0, 4, 8, 16 or PI_TILE_PERSISTENT");
        e.sweep = w;
    }
    engine_build(e, e.grids);   // drops a graph captured with the old tiles
    return PI_OK;
}
int get_tile(const Engine& e)
{
    if (e.sweep == SWEEP_PERSIST) return PI_TILE_PERSISTENT;
    return e.sweep >= 0 ? SWEEP_TILES[e.sweep] : 0;
}
}  // namespace

pi_status pi_set_raytrace_tile(pi_grid* g, int edge)
{
    if (!g) return fail(PI_EINVAL, "null grid");
    return set_tile(g->e, edge);
}

pi_status pi_get_raytrace_tile(pi_grid* g, int* edge)
{
    if (!g || !edge) return fail(PI_EINVAL, "null argument");
    *edge = get_tile(g->e);
    return PI_OK;
}

pi_status pi_batch_set_raytrace_tile(pi_batch* b, int edge)
{
    if (!b) return fail(PI_EINVAL, "null batch");
    return set_tile(b->e, edge);
}

pi_status pi_batch_get_raytrace_tile(pi_batch* b, int* edge)
{
    if (!b || !edge) return fail(PI_EINVAL, "null argument");
    *edge = get_tile(b->e);
    return PI_OK;
}

namespace {
pi_status set_wait_limit(Engine& e, double seconds)
{
    if (!(seconds >= 0.0 && seconds <= PI_WAIT_LIMIT_MAX))
        return fail(PI_EINVAL, "raytrace wait limit must lie in [0, PI_WAIT_LIMIT_MAX] seconds");
    e.persist_spin = (long long)(seconds * 1e8);
    engine_drop_graph(e);   // a captured graph holds the old limit
    return PI_OK;
}
}  // namespace

pi_status pi_set_raytrace_wait_limit(pi_grid* g, double seconds)
{
    if (!g) return fail(PI_EINVAL, "null grid");
    return set_wait_limit(g->e, seconds);
}

pi_status pi_batch_set_raytrace_wait_limit(pi_batch* b, double seconds)
{
    if (!b) return fail(PI_EINVAL, "null batch");
    return set_wait_limit(b->e, seconds);
}

// ------------------------------------------------------------------ batch
pi_status pi_batch_create(int ngrids, const pi_grid_desc* descs, const pi_fields* fields,
                          pi_batch** out)
{
    if (!out) return fail(PI_EINVAL, "null output pointer");
    *out = nullptr;
    if (ngrids < 1 || !descs || !fields) return fail(PI_EINVAL, "need ngrids >= 1, descriptors and fields");
    if (ngrids > (1 << 27)) return fail(PI_EINVAL, "too many grids");
    for (int g = 0; g < ngrids; ++g) {
        pi_status v = validate_desc(&descs[g]);
        if (v == PI_OK) v = validate_fields(&descs[g], &fields[g]);
        if (v != PI_OK) return fail(v, "grid " + std::to_string(g) + ": " + last_error());
        if (descs[g].precision != descs[0].precision)
            return fail(PI_EINVAL, "all grids of a batch share one precision");
    }
    pi_batch* b = new pi_batch();
    b->e.precision = descs[0].precision;
    b->h.resize(ngrids);
    std::vector<GridHost*> ptrs;
    pi_status v = PI_OK;
    for (int g = 0; g < ngrids && v == PI_OK; ++g) {
        v = grid_host_init(b->h[g], descs[g], fields[g]);
        ptrs.push_back(&b->h[g]);
    }
    if (v == PI_OK) v = engine_build(b->e, ptrs);
    if (v != PI_OK) {
        engine_free(b->e);
        for (GridHost& h : b->h) grid_host_free(h);
        delete b;
        return v;
    }
    *out = b;
    return PI_OK;
}

pi_status pi_batch_destroy(pi_batch* b)
{
    if (!b) return PI_OK;
    (void)hipDeviceSynchronize();
    engine_free(b->e);
    for (GridHost& h : b->h) grid_host_free(h);
    delete b;
    return PI_OK;
}

pi_status pi_batch_set_time(pi_batch* b, const double* t, const int64_t* nsteps,
                            const double* t_end, void* stream)
{
    if (!b || !t || !t_end) return fail(PI_EINVAL, "null argument");
    for (size_t g = 0; g < b->h.size(); ++g)
        if (!std::isfinite(t[g]) || !std::isfinite(t_end[g]))
            return fail(PI_EINVAL, "t and t_end must be finite");
    hipStream_t s = static_cast<hipStream_t>(stream);
    std::vector<DevState> st;
    pi_status r = engine_read_states(b->e, st, s);
    if (r != PI_OK) return r;
    for (size_t g = 0; g < st.size(); ++g) {
        st[g].t = t[g];
        st[g].nsteps = nsteps ? nsteps[g] : 0;
        st[g].t_end = t_end[g];
        st[g].dt = 0;
    }
    return engine_write_states(b->e, st, s);
}

pi_status pi_batch_init_energy(pi_batch* b, const double* T0, int state, void* stream)
{
    if (!b || !T0) return fail(PI_EINVAL, "null argument");
    if (!buf_ok(state)) return fail(PI_EINVAL, "buffer selector");
    for (size_t g = 0; g < b->h.size(); ++g)
        if (!(T0[g] > 0)) return fail(PI_EINVAL, "T0 must be > 0");
    for (size_t g = 0; g < b->h.size(); ++g) {
        pi_status r = engine_init_energy(b->e, (int)g, T0[g], state, static_cast<hipStream_t>(stream));
        if (r != PI_OK) return r;
    }
    return PI_OK;
}

pi_status pi_batch_raytrace(pi_batch* b, int state, int tau_buf, void* stream)
{
    if (!b) return fail(PI_EINVAL, "null batch");
    if (!buf_ok(state) || !buf_ok(tau_buf)) return fail(PI_EINVAL, "buffer selector");
    return engine_raytrace(b->e, state, tau_buf, static_cast<hipStream_t>(stream));
}

pi_status pi_batch_step_o2(pi_batch* b, void* stream)
{
    if (!b) return fail(PI_EINVAL, "null batch");
    return engine_step_graph(b->e, static_cast<hipStream_t>(stream));
}

pi_status pi_batch_step_a1(pi_batch* b, void* stream)
{
    if (!b) return fail(PI_EINVAL, "null batch");
    return engine_step_a1(b->e, NAN, static_cast<hipStream_t>(stream));
}

pi_status pi_batch_state(pi_batch* b, double* t, int64_t* nsteps, double* last_dt, void* stream)
{
    if (!b) return fail(PI_EINVAL, "null batch");
    std::vector<DevState> st;
    pi_status r = engine_read_states(b->e, st, static_cast<hipStream_t>(stream));
    if (r != PI_OK) return r;
    for (size_t g = 0; g < st.size(); ++g) {
        if (t) t[g] = st[g].t;
        if (nsteps) nsteps[g] = st[g].nsteps;
        if (last_dt) last_dt[g] = st[g].last_dt;
    }
    return PI_OK;
}

pi_status pi_batch_diagnostics(pi_batch* b, double* out, void* stream)
{
    if (!b || !out) return fail(PI_EINVAL, "null argument");
    std::vector<double> d;
    pi_status r = engine_diagnostics(b->e, d, static_cast<hipStream_t>(stream));
    for (size_t i = 0; i < d.size(); ++i) out[i] = d[i];
    return r;
}

pi_status pi_batch_work_counters(pi_batch* b, int64_t* out, int reset, void* stream)
{
    if (!b || !out) return fail(PI_EINVAL, "null argument");
    return engine_work(b->e, out, reset, static_cast<hipStream_t>(stream));
}

}  // extern "C"
