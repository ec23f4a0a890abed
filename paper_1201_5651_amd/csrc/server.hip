// server.hip -- served form of the library: a worker thread that admits
// requests (one grid each) into a device-memory arena as room frees up and
// advances every admitted grid together with the batch engine, one A3 step of
// all of them per graph replay, until each reaches its own t_end.  Results
// are copied out on a second stream into pinned host buffers while the next
// steps of the other grids run.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "../../include/pi.h"
#include "arena.h"
#include "engine.h"

using namespace pi;

namespace {

using Clock = std::chrono::steady_clock;

double seconds(Clock::time_point a, Clock::time_point b)
{
    return std::chrono::duration<double>(b - a).count();
}

// One device allocation carved by an ArenaMap.
struct Arena {
    char* base = nullptr;
    size_t size = 0;
    ArenaMap map;

    static size_t round(size_t n) { return ArenaMap::round(n); }
    bool init(size_t bytes)
    {
        map.init(bytes);
        size = map.size;
        if (size == 0 || hipMalloc(reinterpret_cast<void**>(&base), size) != hipSuccess) return false;
        return true;
    }
    void release()
    {
        if (base) (void)hipFree(base);
        base = nullptr;
    }
    void* alloc(size_t n)
    {
        size_t off = 0;
        return map.alloc(n, &off) ? base + off : nullptr;
    }
    void free(void* p, size_t n) { map.release(static_cast<char*>(p) - base, n); }
};

// Pinned host buffers for result downloads, reused between requests.
struct PinnedPool {
    std::vector<std::pair<void*, size_t>> idle;
    void* take(size_t n, size_t* got)
    {
        size_t best = idle.size();
        for (size_t i = 0; i < idle.size(); ++i)
            if (idle[i].second >= n && (best == idle.size() || idle[i].second < idle[best].second))
                best = i;
        if (best < idle.size()) {
            void* p = idle[best].first;
            *got = idle[best].second;
            idle.erase(idle.begin() + (long)best);
            return p;
        }
        void* p = nullptr;
        if (hipHostMalloc(&p, n, hipHostMallocDefault) != hipSuccess) return nullptr;
        *got = n;
        return p;
    }
    void give(void* p, size_t n)
    {
        if (p) idle.emplace_back(p, n);
    }
    void release()
    {
        for (auto& b : idle) (void)hipHostFree(b.first);
        idle.clear();
    }
};

enum CkptState { CK_NONE = 0, CK_ASKED = 1, CK_DONE = 2, CK_FAILED = 3 };

struct Request {
    uint64_t ticket = 0;
    pi_grid_desc d{};
    std::vector<double> nH, x0;
    std::vector<char> resume;   // checkpoint to start from (empty: nH, x0, T0)
    double T0 = 0, t_end = 0;
    int status = PI_PENDING;
    std::string error;
    Clock::time_point submitted, admitted, completed;
    // while active
    GridHost grid;
    void* block = nullptr;
    size_t bytes = 0;
    bool active = false;
    bool was_admitted = false;
    bool cancel = false;
    bool nonfinite = false;
    // result download in flight: pinned copy of x (and E), its event
    void* pinned = nullptr;
    size_t pinned_bytes = 0;
    hipEvent_t copied = nullptr;
    // checkpoint asked for by pi_checkpoint (worker fills ck_buf)
    int ck_state = CK_NONE;
    void* ck_buf = nullptr;
    size_t ck_bytes = 0;
    std::string ck_error;
    // results
    std::vector<double> x_out, T_out;
    double t = 0;
    int64_t nsteps = 0;
    double start_t = 0;        // clock at admission (a resumed request's checkpoint)
    int64_t start_nsteps = 0;
};

size_t word_bytes(int precision) { return precision == PI_FP64 ? 8 : 4; }

int nfields(const pi_grid_desc& d) { return d.thermal == PI_T_EVOLVE ? 7 : 5; }

// columns per cell: one per point source
int ncolumns(const pi_grid_desc& d)
{
    return (d.source == PI_SRC_POINT && d.nsrc > 1) ? d.nsrc : 1;
}

// fields of a request in the arena: tau and tau_half carry one array per source
size_t footprint(const pi_grid_desc& d)
{
    const size_t n = (size_t)d.n[0] * d.n[1] * d.n[2];
    return (size_t)(nfields(d) + 2 * (ncolumns(d) - 1)) * Arena::round(n * word_bytes(d.precision));
}

}  // namespace

struct pi_server {
    pi_server_desc desc{};
    int device = 0;
    Arena arena;
    hipStream_t stream = nullptr;   // the steps
    hipStream_t copy = nullptr;     // result downloads
    Engine engine;
    std::vector<Engine::Table> tables;   // rate tables shared by every engine of the server
    PinnedPool pinned;
    std::mutex mu;
    std::condition_variable cv;      // wakes the worker
    std::condition_variable ck_cv;   // wakes pi_checkpoint callers
    std::deque<std::shared_ptr<Request>> queue;               // submitted, not admitted
    std::map<uint64_t, std::shared_ptr<Request>> requests;    // every live ticket
    std::vector<std::shared_ptr<Request>> active;
    std::vector<std::shared_ptr<Request>> draining;           // results being copied out
    uint64_t next_ticket = 1;
    bool stop = false;
    std::thread worker;
    // statistics
    double cell_updates = 0, busy_s = 0;
    uint64_t done = 0, steps = 0, rebuilds = 0;
    std::string worker_error;

    void run();
    bool admit_locked(std::shared_ptr<Request>& r);
    pi_status start(Request& r);
    void retire(Request& r, bool ok, const std::string& why);
    bool finish_download(Request& r, bool wait);
    void checkpoints();
};

// Places a request's fields in the arena (mutex held); false if it does not fit now.
bool pi_server::admit_locked(std::shared_ptr<Request>& r)
{
    r->bytes = footprint(r->d);
    r->block = arena.alloc(r->bytes);
    return r->block != nullptr;
}

// Uploads the request's state and prepares its grid (worker thread, no lock).
pi_status pi_server::start(Request& r)
{
    const pi_grid_desc& d = r.d;
    const size_t n = (size_t)d.n[0] * d.n[1] * d.n[2];
    const size_t fb = Arena::round(n * word_bytes(d.precision));
    char* p = static_cast<char*>(r.block);
    pi_fields f{};
    void** slots[7] = { &f.nH, &f.x, &f.tau, &f.x_half, &f.tau_half, &f.E, &f.E_half };
    for (int k = 0; k < nfields(d); ++k) {
        *slots[k] = p;
        p += (k == 2 || k == 4) ? ncolumns(d) * fb : fb;   // tau, tau_half
    }
    pi_status s = grid_host_init(r.grid, d, f);
    if (s != PI_OK) return s;
    if (!r.resume.empty()) {
        // state, columns and clock from the checkpoint; t_end is the request's
        s = grid_load(r.grid, r.resume.data(), r.resume.size(), stream);
        if (s != PI_OK) return s;
        r.resume.clear();
        r.resume.shrink_to_fit();
        DevState st{};
        if (hipMemcpyAsync(&st, r.grid.st, sizeof(st), hipMemcpyDeviceToHost, stream) != hipSuccess ||
            hipStreamSynchronize(stream) != hipSuccess)
            return fail(PI_EDEVICE, "clock read");
        st.t_end = r.t_end;
        st.dt = 0.0;
        if (hipMemcpyAsync(r.grid.st, &st, sizeof(st), hipMemcpyHostToDevice, stream) != hipSuccess ||
            hipStreamSynchronize(stream) != hipSuccess)
            return fail(PI_EDEVICE, "clock write");
        r.start_t = st.t;
        r.start_nsteps = st.nsteps;
        return PI_OK;
    }
    // initial state, converted to the field precision on the host
    std::vector<double> x(n, 1.0);
    if (!r.x0.empty()) x = r.x0;
    if (d.precision == PI_FP64) {
        if (hipMemcpyAsync(f.nH, r.nH.data(), n * 8, hipMemcpyHostToDevice, stream) != hipSuccess ||
            hipMemcpyAsync(f.x, x.data(), n * 8, hipMemcpyHostToDevice, stream) != hipSuccess)
            return fail(PI_EDEVICE, "request upload");
        if (hipStreamSynchronize(stream) != hipSuccess) return fail(PI_EDEVICE, "request upload sync");
    } else {
        std::vector<float> a(r.nH.begin(), r.nH.end()), b(x.begin(), x.end());
        if (hipMemcpyAsync(f.nH, a.data(), n * 4, hipMemcpyHostToDevice, stream) != hipSuccess ||
            hipMemcpyAsync(f.x, b.data(), n * 4, hipMemcpyHostToDevice, stream) != hipSuccess)
            return fail(PI_EDEVICE, "request upload");
        if (hipStreamSynchronize(stream) != hipSuccess) return fail(PI_EDEVICE, "request upload sync");
    }
    // energy, initial columns and clock through a one-grid engine on the same fields
    Engine one;
    one.precision = d.precision;
    one.table_cache = &tables;
    one.sweep = engine.sweep >= 0 ? engine.sweep : 1;   // no tuning for a one-off raytrace
    s = engine_build(one, { &r.grid });
    if (s == PI_OK) s = engine_init_energy(one, 0, r.T0, PI_BUF_N, stream);
    if (s == PI_OK) s = engine_raytrace(one, PI_BUF_N, PI_BUF_N, stream);
    std::vector<DevState> st;
    if (s == PI_OK) s = engine_read_states(one, st, stream);
    if (s == PI_OK) {
        st[0].t = 0.0;
        st[0].nsteps = 0;
        st[0].t_end = r.t_end;
        st[0].dt = 0.0;
        s = engine_write_states(one, st, stream);
    }
    engine_free(one);
    return s;
}

// Ends a request (worker thread, mutex held).  A finished request's x and E
// are copied out on the copy stream into a pinned buffer; the request stays in
// `draining` until the copy is complete (finish_download), and its arena space
// is released only then.  Failed requests are released at once.  The step
// stream is idle here (the tick ended with a synchronising clock read), so the
// fields hold the final state.
void pi_server::retire(Request& r, bool ok, const std::string& why)
{
    r.active = false;
    if (r.ck_state == CK_ASKED) {
        // a checkpoint asked for but not served (the tick failed)
        r.ck_state = CK_FAILED;
        r.ck_error = why;
        ck_cv.notify_all();
    }
    if (ok) {
        const size_t n = (size_t)r.d.n[0] * r.d.n[1] * r.d.n[2];
        const size_t fb = n * word_bytes(r.d.precision);
        const size_t need = (r.d.thermal == PI_T_EVOLVE ? 2 : 1) * fb;
        bool good = (r.pinned = pinned.take(need, &r.pinned_bytes)) != nullptr;
        if (good) good = hipEventCreateWithFlags(&r.copied, hipEventDisableTiming) == hipSuccess;
        if (good)
            good = hipMemcpyAsync(r.pinned, r.grid.f.x, fb, hipMemcpyDeviceToHost, copy) == hipSuccess;
        if (good && r.d.thermal == PI_T_EVOLVE)
            good = hipMemcpyAsync(static_cast<char*>(r.pinned) + fb, r.grid.f.E, fb,
                                  hipMemcpyDeviceToHost, copy) == hipSuccess;
        if (good) good = hipEventRecord(r.copied, copy) == hipSuccess;
        auto it = requests.find(r.ticket);
        if (good && it != requests.end()) {
            grid_host_free(r.grid);
            draining.push_back(it->second);
            return;
        }
        r.status = PI_EDEVICE;
        r.error = "result download";
    } else {
        r.status = r.cancel ? PI_ECANCELLED : (r.nonfinite ? PI_ENAN : PI_EDEVICE);
        r.error = why;
    }
    r.completed = Clock::now();
    grid_host_free(r.grid);
    if (r.block) arena.free(r.block, r.bytes);
    r.block = nullptr;
    if (r.copied) (void)hipEventDestroy(r.copied);
    r.copied = nullptr;
    pinned.give(r.pinned, r.pinned_bytes);
    r.pinned = nullptr;
}

// Completes a download once its copy has finished (wait: block until it has);
// mutex held.  Returns false while the copy is still in flight.
bool pi_server::finish_download(Request& r, bool wait)
{
    const hipError_t q = wait ? hipEventSynchronize(r.copied) : hipEventQuery(r.copied);
    if (q == hipErrorNotReady) return false;
    const size_t n = (size_t)r.d.n[0] * r.d.n[1] * r.d.n[2];
    if (q != hipSuccess) {
        r.status = PI_EDEVICE;
        r.error = "result download";
    } else {
        r.x_out.assign(n, 0.0);
        r.T_out.assign(n, r.d.T_fixed);
        const bool f32 = r.d.precision != PI_FP64;
        const char* p = static_cast<const char*>(r.pinned);
        if (f32) {
            const float* a = reinterpret_cast<const float*>(p);
            for (size_t q2 = 0; q2 < n; ++q2) r.x_out[q2] = a[q2];
        } else {
            std::memcpy(r.x_out.data(), p, n * 8);
        }
        if (r.d.thermal == PI_T_EVOLVE) {
            // T from the stored state (the density as the grid holds it)
            const double kB = 1.380649e-16;
            for (size_t q2 = 0; q2 < n; ++q2) {
                const double E = f32 ? (double)reinterpret_cast<const float*>(p)[n + q2]
                                     : reinterpret_cast<const double*>(p)[n + q2];
                const double nq = f32 ? (double)(float)r.nH[q2] : r.nH[q2];
                r.T_out[q2] = 2.0 * E / (3.0 * kB * nq * (2.0 - r.x_out[q2]));
            }
        }
        r.status = PI_OK;
        done++;
    }
    r.completed = Clock::now();
    if (r.block) arena.free(r.block, r.bytes);
    r.block = nullptr;
    (void)hipEventDestroy(r.copied);
    r.copied = nullptr;
    pinned.give(r.pinned, r.pinned_bytes);
    r.pinned = nullptr;
    return true;
}

// Serves the checkpoints asked for by pi_checkpoint (worker thread, no lock
// held while the state is read; the step stream is idle).
void pi_server::checkpoints()
{
    std::vector<std::shared_ptr<Request>> ask;
    {
        std::lock_guard<std::mutex> lk(mu);
        for (auto& r : active)
            if (r->ck_state == CK_ASKED) ask.push_back(r);
    }
    if (ask.empty()) return;
    for (auto& r : ask) {
        const pi_status s = grid_save(r->grid, r->ck_buf, r->ck_bytes, stream);
        std::lock_guard<std::mutex> lk(mu);
        r->ck_state = s == PI_OK ? CK_DONE : CK_FAILED;
        if (s != PI_OK) r->ck_error = last_error();
    }
    ck_cv.notify_all();
}

void pi_server::run()
{
    (void)hipSetDevice(device);
    // The batch is rebuilt once per change of the active set (at the next tick
    // after admissions or retirements).  A HIP graph of the step costs a
    // capture (several ms of host time while the GPU waits), so steps are
    // launched directly until the set has been the same for two ticks, and
    // replayed from a graph after that; the kernels and their order are the
    // same either way.
    bool dirty = false;
    int stable = 0;
    for (;;) {
        std::vector<std::shared_ptr<Request>> admitted;
        {
            std::unique_lock<std::mutex> lk(mu);
            cv.wait(lk, [&] {
                return stop || !queue.empty() || !active.empty() || !draining.empty();
            });
            if (stop) break;
            // downloads that have finished free their arena space first
            for (auto it = draining.begin(); it != draining.end();)
                it = finish_download(**it, active.empty() && queue.empty()) ? draining.erase(it)
                                                                             : it + 1;
            // cancelled requests leave the queue; the rest are admitted in order
            // while a slot and room in the arena are free
            for (auto it = queue.begin(); it != queue.end();) {
                if ((*it)->cancel) {
                    (*it)->status = PI_ECANCELLED;
                    (*it)->completed = Clock::now();
                    it = queue.erase(it);
                } else {
                    ++it;
                }
            }
            while (!queue.empty() && (int)(active.size() + admitted.size()) < desc.max_active) {
                std::shared_ptr<Request>& r = queue.front();
                if (!admit_locked(r)) break;   // head-of-line: keep arrival order
                r->admitted = Clock::now();
                r->was_admitted = true;
                admitted.push_back(r);
                queue.pop_front();
            }
            // nothing to step while the head of the queue waits for space that
            // draining downloads still hold: wait for one of them
            if (active.empty() && admitted.empty() && !draining.empty()) {
                if (finish_download(*draining.front(), true)) draining.erase(draining.begin());
                continue;
            }
        }
        bool changed = !admitted.empty();
        for (auto& r : admitted) {
            const pi_status s = start(*r);
            std::lock_guard<std::mutex> lk(mu);
            if (s != PI_OK) {
                retire(*r, false, last_error());
            } else {
                r->active = true;
                r->t = r->start_t;
                r->nsteps = r->start_nsteps;
                active.push_back(r);
            }
        }
        const Clock::time_point t0 = Clock::now();
        std::vector<GridHost*> grids;
        std::vector<int64_t> before;
        {
            std::lock_guard<std::mutex> lk(mu);
            for (auto& r : active) {
                grids.push_back(&r->grid);
                before.push_back(r->nsteps);
            }
        }
        if (grids.empty()) continue;
        pi_status s = PI_OK;
        if (changed || dirty || engine.ngrids() != (int)grids.size()) {
            s = engine_build(engine, grids);
            rebuilds++;
            dirty = false;
            stable = 0;
            // first batch: choose the raytrace tiles (recomputes the current columns)
            if (s == PI_OK && engine.sweep < 0) s = engine_autotune(engine, PI_BUF_N, PI_BUF_N, stream);
        }
        std::vector<DevState> st;
        if (s == PI_OK) {
            for (int k = 0; k < desc.steps_per_tick && s == PI_OK; ++k)
                s = stable >= 2 ? engine_step_graph(engine, stream) : engine_step(engine, NAN, 2, stream);
            ++stable;
            if (s == PI_OK) s = engine_read_states(engine, st, stream);
        }
        if (s == PI_OK) checkpoints();
        std::lock_guard<std::mutex> lk(mu);
        busy_s += seconds(t0, Clock::now());
        if (s != PI_OK) {
            // a device error ends every active request
            worker_error = last_error();
            for (auto& r : active) retire(*r, false, worker_error);
            active.clear();
            engine_build(engine, {});
            continue;
        }
        steps += desc.steps_per_tick;
        std::vector<std::shared_ptr<Request>> keep;
        for (size_t g = 0; g < active.size(); ++g) {
            Request& r = *active[g];
            cell_updates += (double)r.grid.ncell * (double)(st[g].nsteps - r.nsteps);
            r.t = st[g].t;
            r.nsteps = st[g].nsteps;
            if (r.cancel) {
                retire(r, false, "cancelled");
            } else if (st[g].diag[5] > 0) {
                r.nonfinite = true;
                retire(r, false, "non-finite values in the grid state");
            } else if (st[g].t >= r.t_end) {
                retire(r, true, "");
            } else if (st[g].nsteps == before[g]) {
                // a whole tick without a step before t_end: the timestep is zero
                retire(r, false, "no progress: the timestep of eq. (4) is zero");
            } else {
                keep.push_back(active[g]);
            }
        }
        if (keep.size() != active.size()) {
            active = keep;
            dirty = true;   // retired grids' memory is free: rebuilt before the next step
        }
    }
    // a checkpoint still asked for when the worker stops cannot be served
    std::lock_guard<std::mutex> lk(mu);
    for (auto& r : active)
        if (r->ck_state == CK_ASKED) {
            r->ck_state = CK_FAILED;
            r->ck_error = "server stopped";
        }
    ck_cv.notify_all();
}

extern "C" {

pi_status pi_server_create(const pi_server_desc* desc, pi_server** out)
{
    if (!out || !desc) return fail(PI_EINVAL, "null argument");
    *out = nullptr;
    if (desc->max_active < 1 || desc->steps_per_tick < 1)
        return fail(PI_EINVAL, "max_active and steps_per_tick must be >= 1");
    if (desc->precision != PI_FP64 && desc->precision != PI_FP32 && desc->precision != PI_MIXED &&
        desc->precision != PI_MIXED_FRONT)
        return fail(PI_EINVAL, "precision");
    std::unique_ptr<pi_server> s(new pi_server());
    s->desc = *desc;
    if (hipGetDevice(&s->device) != hipSuccess) return fail(PI_EDEVICE, "no device");
    size_t budget = desc->hbm_budget;
    if (budget == 0) {
        size_t fr = 0, tot = 0;
        if (hipMemGetInfo(&fr, &tot) != hipSuccess) return fail(PI_EDEVICE, "memory query");
        budget = (size_t)(0.8 * (double)fr);
    }
    if (!s->arena.init(budget)) return fail(PI_ENOMEM, "arena allocation of the HBM budget");
    s->engine.precision = desc->precision;
    s->engine.table_cache = &s->tables;
    if (hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking) != hipSuccess) {
        s->arena.release();
        return fail(PI_EDEVICE, "stream creation");
    }
    if (hipStreamCreateWithFlags(&s->copy, hipStreamNonBlocking) != hipSuccess) {
        (void)hipStreamDestroy(s->stream);
        s->arena.release();
        return fail(PI_EDEVICE, "stream creation");
    }
    pi_server* p = s.release();
    p->worker = std::thread([p] { p->run(); });
    *out = p;
    return PI_OK;
}

pi_status pi_submit(pi_server* s, const pi_request* req, uint64_t* ticket)
{
    if (!s || !req || !ticket) return fail(PI_EINVAL, "null argument");
    pi_status v = validate_desc(&req->desc);
    if (v != PI_OK) return v;
    if (req->desc.precision != s->desc.precision) return fail(PI_EINVAL, "precision differs from the server's");
    if (!std::isfinite(req->t_end) || !(req->t_end >= 0)) return fail(PI_EINVAL, "t_end must be finite and >= 0");
    if (footprint(req->desc) > s->arena.size)
        return fail(PI_EREJECTED, "request larger than the server's device-memory budget");
    auto r = std::make_shared<Request>();
    const size_t n = (size_t)req->desc.n[0] * req->desc.n[1] * req->desc.n[2];
    r->d = req->desc;
    if (req->checkpoint) {
        // resumed: the state (density included) comes from the checkpoint
        if ((v = checkpoint_check(req->desc, req->checkpoint, req->checkpoint_bytes)) != PI_OK)
            return v;
        const char* c = static_cast<const char*>(req->checkpoint);
        r->resume.assign(c, c + checkpoint_bytes(req->desc));
        // the density as the grid holds it, for the temperatures of the result
        const size_t wb = word_bytes(req->desc.precision);
        const char* nh = c + checkpoint_header_bytes();   // n_H is the first array
        r->nH.resize(n);
        for (size_t q = 0; q < n; ++q)
            r->nH[q] = wb == 8 ? reinterpret_cast<const double*>(nh)[q]
                               : (double)reinterpret_cast<const float*>(nh)[q];
    } else {
        if (!req->nH) return fail(PI_EINVAL, "nH is required");
        if (req->desc.thermal == PI_T_EVOLVE && !(req->T0 > 0)) return fail(PI_EINVAL, "T0 must be > 0");
        r->nH.assign(req->nH, req->nH + n);
        for (double v2 : r->nH)
            if (!(v2 > 0) || !std::isfinite(v2)) return fail(PI_EINVAL, "nH must be finite and > 0");
        if (req->x0) {
            r->x0.assign(req->x0, req->x0 + n);
            for (double v2 : r->x0)
                if (!(v2 >= 0 && v2 <= 1)) return fail(PI_EINVAL, "x0 must lie in [0, 1]");
        }
    }
    r->T0 = req->desc.thermal == PI_T_EVOLVE ? req->T0 : 1.0;
    r->t_end = req->t_end;
    r->submitted = Clock::now();
    {
        std::lock_guard<std::mutex> lk(s->mu);
        r->ticket = s->next_ticket++;
        s->requests[r->ticket] = r;
        s->queue.push_back(r);
    }
    s->cv.notify_one();
    *ticket = r->ticket;
    return PI_OK;
}

pi_status pi_poll(pi_server* s, uint64_t ticket, pi_result* out, double* x_out, double* T_out)
{
    if (!s || !out) return fail(PI_EINVAL, "null argument");
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->requests.find(ticket);
    if (it == s->requests.end()) return fail(PI_EINVAL, "unknown ticket");
    Request& r = *it->second;
    out->status = r.status;
    out->t = r.t;
    out->nsteps = r.nsteps;
    out->queue_s = r.was_admitted ? seconds(r.submitted, r.admitted) : seconds(r.submitted, Clock::now());
    out->latency_s = r.status == PI_PENDING ? seconds(r.submitted, Clock::now())
                                            : seconds(r.submitted, r.completed);
    if (r.status == PI_PENDING) return PI_PENDING;
    if (r.status != PI_OK) {
        const pi_status st = (pi_status)r.status;
        const std::string e = r.error;
        s->requests.erase(it);
        return fail(st, e);
    }
    if (x_out) std::copy(r.x_out.begin(), r.x_out.end(), x_out);
    if (T_out) std::copy(r.T_out.begin(), r.T_out.end(), T_out);
    s->requests.erase(it);
    return PI_OK;
}

pi_status pi_cancel(pi_server* s, uint64_t ticket)
{
    if (!s) return fail(PI_EINVAL, "null server");
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->requests.find(ticket);
    if (it == s->requests.end()) return fail(PI_EINVAL, "unknown ticket");
    it->second->cancel = true;
    s->cv.notify_one();
    return PI_OK;
}

pi_status pi_checkpoint(pi_server* s, uint64_t ticket, void* host_buf, size_t bytes, size_t* needed)
{
    if (!s) return fail(PI_EINVAL, "null server");
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->requests.find(ticket);
    if (it == s->requests.end()) return fail(PI_EINVAL, "unknown ticket");
    std::shared_ptr<Request> r = it->second;
    const size_t need = checkpoint_bytes(r->d);
    if (needed) *needed = need;
    if (!host_buf) return PI_OK;   // size query
    if (bytes < need) return fail(PI_EINVAL, "checkpoint buffer too small");
    if (r->status != PI_PENDING || r->pinned)
        return fail(PI_EINVAL, "request has finished: poll it for its result");
    if (!r->active) return fail(PI_PENDING, "request not started yet: nothing to save");
    if (r->ck_state == CK_ASKED) return fail(PI_EINVAL, "a checkpoint of this request is in progress");
    r->ck_buf = host_buf;
    r->ck_bytes = bytes;
    r->ck_state = CK_ASKED;
    s->cv.notify_one();
    s->ck_cv.wait(lk, [&] { return r->ck_state != CK_ASKED; });
    const bool ok = r->ck_state == CK_DONE;
    r->ck_state = CK_NONE;
    r->ck_buf = nullptr;
    return ok ? PI_OK : fail(PI_EDEVICE, "checkpoint: " + r->ck_error);
}

pi_status pi_server_stats(pi_server* s, double* out)
{
    if (!s || !out) return fail(PI_EINVAL, "null argument");
    std::lock_guard<std::mutex> lk(s->mu);
    out[0] = (double)s->done;
    out[1] = s->cell_updates;
    out[2] = s->busy_s;
    out[3] = (double)s->steps;
    out[4] = (double)s->active.size();
    out[5] = (double)s->queue.size();
    out[6] = (double)s->arena.map.used;
    out[7] = (double)s->rebuilds;
    return PI_OK;
}

pi_status pi_server_destroy(pi_server* s)
{
    if (!s) return PI_OK;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
    }
    s->cv.notify_one();
    if (s->worker.joinable()) s->worker.join();
    (void)hipStreamSynchronize(s->stream);
    (void)hipStreamSynchronize(s->copy);
    for (auto& r : s->active) grid_host_free(r->grid);
    for (auto& r : s->draining) {
        if (r->copied) (void)hipEventDestroy(r->copied);
        s->pinned.give(r->pinned, r->pinned_bytes);
        r->pinned = nullptr;
    }
    engine_free(s->engine);
    free_tables(s->tables);
    s->pinned.release();
    (void)hipStreamDestroy(s->stream);
    (void)hipStreamDestroy(s->copy);
    s->arena.release();
    delete s;
    return PI_OK;
}

}  // extern "C"
