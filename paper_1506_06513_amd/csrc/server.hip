// Request loop with continuous batching (flusi_server_*), built on the public
// C ABI: plans, states and one ensemble that all admitted requests join.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <thread>
#include <vector>

#include "../../include/flusi.h"

namespace flusi {
int set_error(int code, const char* fmt, ...);
int insect_error(const flusi_insect* ins);
}
using flusi::insect_error;
using flusi::set_error;

namespace {
using clk = std::chrono::steady_clock;

struct Req {
    long long id = 0;
    flusi_request r{};               // copy; r.u0 cleared
    std::vector<unsigned char> u0;   // host copy of the initial field (empty: at rest)
    size_t bytes = 0;                // footprint while admitted
    clk::time_point t_submit;
    // while admitted (worker thread only)
    flusi_plan plan = nullptr;
    void* state = nullptr;
    void* ubuf = nullptr;            // device field: initial velocity, later the result
    int member = -1;
    int remaining = 0;
    // result (under the server mutex once done)
    bool done = false;
    int status = FLUSI_OK;
    std::vector<unsigned char> u;
    double diag[FLUSI_NDIAG] = {0};
    double latency_ms = 0.0;
};

size_t real_bytes(int dtype) { return dtype == FLUSI_F32 ? 4 : 8; }
size_t field_bytes(int n, int dtype) { return 3ul * n * n * n * real_bytes(dtype); }
}  // namespace

struct flusi_server_s {
    int dtype = 0;
    size_t budget = 0;
    int max_chunk = 1;
    int device = 0;
    hipStream_t stream = nullptr;
    flusi_ensemble ens = nullptr;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<Req*> waiting;           // arrival order
    std::vector<Req*> active;           // worker thread only
    std::map<long long, Req*> reqs;     // every request not yet collected by flusi_server_wait
    long long next_id = 1;
    bool stop = false;
    std::thread worker;
    // statistics (under mu)
    long long submitted = 0, completed = 0, failed = 0;
    std::vector<double> lat;
    double point_steps = 0.0;
    bool have_first = false;
    clk::time_point first_submit, last_done;
    size_t used = 0, peak_bytes = 0;
    int n_active = 0, peak_active = 0;
};

namespace {

void free_device(Req* q) {
    if (q->plan) flusi_plan_destroy(q->plan);
    if (q->state) (void)hipFree(q->state);
    if (q->ubuf) (void)hipFree(q->ubuf);
    q->plan = nullptr;
    q->state = nullptr;
    q->ubuf = nullptr;
}

// Plan, state and initial field of an admitted request; joins the ensemble.
int setup(flusi_server s, Req* q) {
    const int n = q->r.n;
    int rc = flusi_plan_create(n, n, n, q->r.L, q->r.nu, q->r.eta, s->dtype, &q->plan);
    if (rc) return rc;
    flusi_set_stream(q->plan, s->stream);
    size_t ws = 0, sb = 0;
    flusi_sizes(n, s->dtype, &ws, &sb);
    if (hipMalloc(&q->state, sb) != hipSuccess) return set_error(FLUSI_ENOMEM, "server: state");
    const size_t fb = field_bytes(n, s->dtype);
    if (hipMalloc(&q->ubuf, fb) != hipSuccess) return set_error(FLUSI_ENOMEM, "server: field");
    hipError_t e;
    if (q->u0.empty()) e = hipMemsetAsync(q->ubuf, 0, fb, s->stream);
    else e = hipMemcpyAsync(q->ubuf, q->u0.data(), fb, hipMemcpyHostToDevice, s->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
    if (e != hipSuccess) return set_error(FLUSI_EDEVICE, "server: %s", hipGetErrorString(e));
    std::vector<unsigned char>().swap(q->u0);
    rc = flusi_state_init(q->plan, q->state, q->ubuf, 0.0);
    if (rc) return rc;
    flusi_step_params p = q->r.p;
    p.history = nullptr;
    rc = flusi_ensemble_add(s->ens, q->plan, q->state, q->r.has_insect ? &q->r.ins : nullptr, &p, &q->member);
    if (rc) return rc;
    q->remaining = q->r.p.nsteps;
    return FLUSI_OK;
}

// Result of a request whose steps are done; frees its device memory.
void finish(flusi_server s, Req* q) {
    int status = q->status;
    if (q->member >= 0) {
        flusi_ensemble_remove(s->ens, q->member);
        q->member = -1;
    }
    if (!status) {
        const size_t fb = field_bytes(q->r.n, s->dtype);
        status = flusi_state_velocity(q->plan, q->state, q->ubuf);
        if (!status) {
            q->u.resize(fb);
            hipError_t e = hipMemcpyAsync(q->u.data(), q->ubuf, fb, hipMemcpyDeviceToHost, s->stream);
            if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
            if (e != hipSuccess) status = set_error(FLUSI_EDEVICE, "server: %s", hipGetErrorString(e));
        }
        const int frc = flusi_forces(q->plan, q->state, q->diag);
        if (!status) status = frc;
    }
    free_device(q);
    const clk::time_point now = clk::now();
    std::lock_guard<std::mutex> lk(s->mu);
    q->status = status;
    q->latency_ms = std::chrono::duration<double, std::milli>(now - q->t_submit).count();
    q->done = true;
    s->used -= q->bytes;
    s->n_active -= 1;
    s->last_done = now;
    if (status == FLUSI_OK) {
        s->completed += 1;
        s->lat.push_back(q->latency_ms);
        s->point_steps += std::pow((double)q->r.n, 3) * q->r.p.nsteps;
    } else {
        s->failed += 1;
    }
}

void worker_main(flusi_server s) {
    (void)hipSetDevice(s->device);
    for (;;) {
        std::vector<Req*> admit;
        {
            std::unique_lock<std::mutex> lk(s->mu);
            s->cv_work.wait(lk, [&] { return s->stop || !s->waiting.empty() || !s->active.empty(); });
            if (s->stop) return;
            // admission in arrival order while the footprints fit
            while (!s->waiting.empty() && s->used + s->waiting.front()->bytes <= s->budget) {
                Req* q = s->waiting.front();
                s->waiting.pop_front();
                s->used += q->bytes;
                s->n_active += 1;
                s->peak_bytes = std::max(s->peak_bytes, s->used);
                s->peak_active = std::max(s->peak_active, s->n_active);
                admit.push_back(q);
            }
        }
        for (Req* q : admit) {
            q->status = setup(s, q);
            if (q->status || q->remaining == 0) finish(s, q);
            else s->active.push_back(q);
        }
        if (!admit.empty()) s->cv_done.notify_all();
        if (s->active.empty()) continue;
        int k = s->max_chunk;
        for (Req* q : s->active) k = std::min(k, q->remaining);
        int rc = flusi_ensemble_step(s->ens, k, 0);
        hipError_t e = hipStreamSynchronize(s->stream);
        if (!rc && e != hipSuccess) rc = set_error(FLUSI_EDEVICE, "server: %s", hipGetErrorString(e));
        std::vector<Req*> keep;
        for (Req* q : s->active) {
            q->remaining -= k;
            if (rc) q->status = rc;
            if (rc || q->remaining <= 0) finish(s, q);
            else keep.push_back(q);
        }
        if (keep.size() != s->active.size()) s->cv_done.notify_all();
        s->active.swap(keep);
    }
}

}  // namespace

extern "C" {

size_t flusi_request_bytes(int n, int dtype) {
    size_t ws = 0, sb = 0;
    if (flusi_sizes(n, dtype, &ws, &sb)) return 0;
    const size_t cxb = 2 * real_bytes(dtype);
    // workspace + state + velocity-export scratch (3 full-layout spectra) + field
    return ws + sb + 3ul * n * n * (n / 2 + 1) * cxb + field_bytes(n, dtype);
}

int flusi_server_create(int dtype, size_t hbm_budget, int max_chunk, flusi_server* out) {
    if (!out) return set_error(FLUSI_EINVAL, "out is NULL");
    *out = nullptr;
    if (dtype != FLUSI_F32 && dtype != FLUSI_F64) return set_error(FLUSI_EINVAL, "dtype must be FLUSI_F32 or FLUSI_F64");
    if (max_chunk < 1 || hbm_budget == 0) return set_error(FLUSI_EINVAL, "server: need max_chunk >= 1 and a budget");
    flusi_server s = new (std::nothrow) flusi_server_s();
    if (!s) return set_error(FLUSI_ENOMEM, "host allocation");
    s->dtype = dtype;
    s->budget = hbm_budget;
    s->max_chunk = max_chunk;
    hipError_t e = hipGetDevice(&s->device);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking);
    if (e != hipSuccess) {
        delete s;
        return set_error(FLUSI_EDEVICE, "server_create: %s", hipGetErrorString(e));
    }
    int rc = flusi_ensemble_create(dtype, &s->ens);
    if (!rc) rc = flusi_ensemble_set_stream(s->ens, s->stream);
    if (rc) {
        if (s->ens) flusi_ensemble_destroy(s->ens);
        (void)hipStreamDestroy(s->stream);
        delete s;
        return rc;
    }
    s->worker = std::thread(worker_main, s);
    *out = s;
    return FLUSI_OK;
}

int flusi_server_destroy(flusi_server s) {
    if (!s) return FLUSI_OK;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
    }
    s->cv_work.notify_all();
    if (s->worker.joinable()) s->worker.join();
    (void)hipStreamSynchronize(s->stream);
    for (Req* q : s->active) {
        if (q->member >= 0) flusi_ensemble_remove(s->ens, q->member);
        free_device(q);
    }
    flusi_ensemble_destroy(s->ens);
    for (auto& kv : s->reqs) delete kv.second;
    (void)hipStreamDestroy(s->stream);
    delete s;
    return FLUSI_OK;
}

int flusi_server_submit(flusi_server s, const flusi_request* r, long long* id) {
    if (!s || !r) return set_error(FLUSI_EINVAL, "server_submit: null pointer");
    if (!(r->L > 0.0) || !(r->nu >= 0.0) || !(r->eta > 0.0) || r->p.nsteps < 0)
        return set_error(FLUSI_EINVAL, "server_submit: need L > 0, nu >= 0, eta > 0, nsteps >= 0");
    if (!(r->p.dt_fixed > 0.0) && !(r->p.cfl > 0.0)) return set_error(FLUSI_EINVAL, "server_submit: need dt_fixed > 0 or cfl > 0");
    if (r->has_insect)
        if (int rc = insect_error(&r->ins)) return rc;
    const size_t bytes = flusi_request_bytes(r->n, s->dtype);
    if (!bytes) return set_error(FLUSI_EUNSUPPORTED, "server_submit: grid size %d not supported", r->n);
    if (bytes > s->budget)
        return set_error(FLUSI_ENOMEM, "server_submit: request needs %zu bytes, budget is %zu", bytes, s->budget);
    Req* q = new (std::nothrow) Req();
    if (!q) return set_error(FLUSI_ENOMEM, "host allocation");
    q->r = *r;
    q->r.u0 = nullptr;
    q->r.p.history = nullptr;
    q->bytes = bytes;
    if (r->u0) {
        const size_t fb = field_bytes(r->n, s->dtype);
        q->u0.resize(fb);
        std::memcpy(q->u0.data(), r->u0, fb);
    }
    {
        std::lock_guard<std::mutex> lk(s->mu);
        q->id = s->next_id++;
        q->t_submit = clk::now();
        if (!s->have_first) {
            s->have_first = true;
            s->first_submit = q->t_submit;
        }
        s->submitted += 1;
        s->reqs[q->id] = q;
        s->waiting.push_back(q);
    }
    s->cv_work.notify_all();
    if (id) *id = q->id;
    return FLUSI_OK;
}

int flusi_server_wait(flusi_server s, long long id, double timeout_ms, void* u_host, double* diag,
                      double* latency_ms) {
    if (!s) return set_error(FLUSI_EINVAL, "null server");
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->reqs.find(id);
    if (it == s->reqs.end()) return set_error(FLUSI_EINVAL, "server_wait: unknown request %lld", id);
    Req* q = it->second;
    auto ready = [&] { return q->done; };
    if (timeout_ms < 0) {
        s->cv_done.wait(lk, ready);
    } else if (!s->cv_done.wait_for(lk, std::chrono::duration<double, std::milli>(timeout_ms), ready)) {
        return 1;
    }
    if (u_host && !q->u.empty()) std::memcpy(u_host, q->u.data(), q->u.size());
    if (diag) std::memcpy(diag, q->diag, sizeof q->diag);
    if (latency_ms) *latency_ms = q->latency_ms;
    const int status = q->status;
    s->reqs.erase(it);
    delete q;
    if (status) return set_error(status, "request %lld ended with status %d", id, status);
    return FLUSI_OK;
}

int flusi_server_stats_get(flusi_server s, flusi_server_stats* out) {
    if (!s || !out) return set_error(FLUSI_EINVAL, "server_stats: null pointer");
    std::lock_guard<std::mutex> lk(s->mu);
    flusi_server_stats st{};
    st.submitted = s->submitted;
    st.completed = s->completed;
    st.failed = s->failed;
    st.waiting = (long long)s->waiting.size();
    st.active = s->n_active;
    std::vector<double> l = s->lat;
    std::sort(l.begin(), l.end());
    // nearest-rank percentiles
    auto pct = [&](double p) {
        if (l.empty()) return 0.0;
        size_t k = (size_t)std::ceil(p / 100.0 * l.size());
        return l[std::min(l.size(), std::max<size_t>(k, 1)) - 1];
    };
    st.p50_ms = pct(50.0);
    st.p99_ms = pct(99.0);
    st.max_ms = l.empty() ? 0.0 : l.back();
    st.point_steps = s->point_steps;
    st.busy_s = s->have_first && s->completed ? std::chrono::duration<double>(s->last_done - s->first_submit).count() : 0.0;
    st.mpoint_steps_per_s = st.busy_s > 0 ? st.point_steps / st.busy_s / 1e6 : 0.0;
    st.peak_bytes = s->peak_bytes;
    st.peak_active = s->peak_active;
    *out = st;
    return FLUSI_OK;
}

}  // extern "C"
