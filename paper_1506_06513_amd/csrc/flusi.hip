// C ABI of the pseudo-spectral penalized Navier-Stokes library (see include/flusi.h).
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <vector>

#include "impl.hpp"

namespace flusi {

#define FLUSI_SIZE(s) ImplBase* make_impl_##s(int);
#include "sizes.def"
#undef FLUSI_SIZE

static thread_local char g_err[512] = "no error";

int set_error(int code, const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
    return code;
}

int ensure_scratch(void** ptr, size_t* cur, size_t need, PlanData& p) {
    if (*cur >= need) return FLUSI_OK;
    if (*ptr) {
        (void)hipStreamSynchronize(p.stream);
        (void)hipFree(*ptr);
        p.workspace -= *cur;
        *ptr = nullptr;
        *cur = 0;
    }
    if (hipMalloc(ptr, need) != hipSuccess) {
        *ptr = nullptr;
        return set_error(FLUSI_ENOMEM, "cannot allocate %zu bytes of scratch", need);
    }
    *cur = need;
    p.workspace += need;
    return FLUSI_OK;
}

static ImplBase* make_impl(int n, int dtype) {
    switch (n) {
#define FLUSI_SIZE(s) \
    case s:           \
        return make_impl_##s(dtype);
#include "sizes.def"
#undef FLUSI_SIZE
        default:
            return nullptr;
    }
}

// cos and sin of 2 pi m / n (n a multiple of 8), reduced to the first octant and
// evaluated in extended precision so that the doubles are correctly rounded.
static void sincos_2pi(long m, long n, double* c, double* s) {
    m %= n;
    if (m < 0) m += n;
    double sgn_s = 1.0, sgn_c = 1.0;
    bool swap = false;
    if (2 * m > n) {  // theta -> 2 pi - theta
        m = n - m;
        sgn_s = -1.0;
    }
    if (4 * m > n) {  // theta -> pi - theta
        m = n / 2 - m;
        sgn_c = -1.0;
    }
    if (8 * m > n) {  // theta -> pi/2 - theta
        m = n / 4 - m;
        swap = true;
    }
    const long double th = 2.0L * 3.14159265358979323846264338327950288L * (long double)m / (long double)n;
    long double cc = cosl(th), ss = sinl(th);
    if (m == 0) {
        cc = 1.0L;
        ss = 0.0L;
    }
    if (swap) {
        const long double t = cc;
        cc = ss;
        ss = t;
    }
    *c = sgn_c * (double)cc;
    *s = sgn_s * (double)ss;
}

static int check_plan(flusi_plan p);

}  // namespace flusi

struct flusi_plan_s {
    flusi::PlanData d;
};

namespace flusi {
static int check_plan(flusi_plan p) {
    if (!p || !p->d.impl) return set_error(FLUSI_EINVAL, "null plan");
    return FLUSI_OK;
}
static void free_plan(PlanData& d) {
    void* ptrs[] = {d.tw, d.bufA, d.bufB, d.partial, d.partial2, d.kin, d.ins_dev, d.member_dev, d.pmax, d.spec, d.phys};
    for (void* q : ptrs)
        if (q) (void)hipFree(q);
    for (hipEvent_t e : d.events) (void)hipEventDestroy(e);
    d.events.clear();
    delete d.impl;
    d.impl = nullptr;
}
}  // namespace flusi

using namespace flusi;

static_assert(sizeof(flusi_insect) == 16 + 8 * 36, "flusi_insect layout");
static_assert(sizeof(flusi_step_params) == 8 + 5 * 8 + 8, "flusi_step_params layout");

extern "C" {

const char* flusi_last_error(void) { return g_err; }

int flusi_plan_create(int nx, int ny, int nz, double L, double nu, double eta, int dtype, flusi_plan* out) {
    if (!out) return set_error(FLUSI_EINVAL, "out is NULL");
    *out = nullptr;
    if (nx != ny || ny != nz) return set_error(FLUSI_EUNSUPPORTED, "only cubic grids are supported (%d x %d x %d)", nx, ny, nz);
    if (!(L > 0.0) || !(nu >= 0.0) || !(eta > 0.0)) return set_error(FLUSI_EINVAL, "need L > 0, nu >= 0, eta > 0");
    if (dtype != FLUSI_F32 && dtype != FLUSI_F64) return set_error(FLUSI_EINVAL, "dtype must be FLUSI_F32 or FLUSI_F64");
    ImplBase* impl = make_impl(nx, dtype);
    if (!impl) return set_error(FLUSI_EUNSUPPORTED, "grid size %d not supported", nx);
    flusi_plan p = new (std::nothrow) flusi_plan_s();
    if (!p) {
        delete impl;
        return set_error(FLUSI_ENOMEM, "host allocation");
    }
    PlanData& d = p->d;
    d.impl = impl;
    d.n = nx;
    d.dtype = dtype;
    d.L = L;
    d.nu = nu;
    d.eta = eta;
    d.K = kmax_of(nx);
    d.KP = d.K + 1;
    d.M = 2 * d.K + 1;
    d.Q = d.M * d.KP;
    const size_t cxb = dtype == FLUSI_F32 ? 8 : 16;
    d.szA = impl->bufA_elems() * cxb;
    d.szB = impl->bufB_elems() * cxb;
    d.nwg_x = impl->nwg_x();
    bool ok = hipMalloc(&d.tw, nx * cxb) == hipSuccess;
    ok = ok && hipMalloc(&d.bufA, d.szA) == hipSuccess;
    ok = ok && hipMalloc(&d.bufB, d.szB) == hipSuccess;
    ok = ok && hipMalloc(&d.partial, (size_t)d.nwg_x * NV * sizeof(double)) == hipSuccess;
    ok = ok && hipMalloc(&d.partial2, (size_t)NRED_BLOCKS * NV * sizeof(double)) == hipSuccess;
    ok = ok && hipMalloc(&d.kin, sizeof(Kin)) == hipSuccess;
    ok = ok && hipMalloc(&d.ins_dev, sizeof(flusi_insect)) == hipSuccess;
    ok = ok && hipMalloc(&d.member_dev, sizeof(Member)) == hipSuccess;
    d.split_z = impl->split_z_default();
    if (!ok) {
        free_plan(d);
        delete p;
        return set_error(FLUSI_ENOMEM, "device allocation for a %d^3 plan", nx);
    }
    d.workspace = nx * cxb + d.szA + d.szB + (size_t)d.nwg_x * NV * 8 + NRED_BLOCKS * NV * 8 + sizeof(Kin) + sizeof(flusi_insect) + sizeof(Member);
    // FP64 twiddles exp(-2 pi i m / n); the FP32 table is rounded from them.
    std::vector<double> w(2 * nx);
    for (int m = 0; m < nx; ++m) {
        double c, s;
        sincos_2pi(m, nx, &c, &s);
        w[2 * m] = c;
        w[2 * m + 1] = -s;
    }
    hipError_t e;
    if (dtype == FLUSI_F64) {
        e = hipMemcpy(d.tw, w.data(), nx * cxb, hipMemcpyHostToDevice);
    } else {
        std::vector<float> wf(2 * nx);
        for (int i = 0; i < 2 * nx; ++i) wf[i] = (float)w[i];
        e = hipMemcpy(d.tw, wf.data(), nx * cxb, hipMemcpyHostToDevice);
    }
    if (e != hipSuccess) {
        free_plan(d);
        delete p;
        return set_error(FLUSI_EDEVICE, "plan setup: %s", hipGetErrorString(e));
    }
    *out = p;
    return FLUSI_OK;
}

int flusi_plan_destroy(flusi_plan plan) {
    if (!plan) return FLUSI_OK;
    if (plan->d.stream) (void)hipStreamSynchronize(plan->d.stream);
    else (void)hipDeviceSynchronize();
    free_plan(plan->d);
    delete plan;
    return FLUSI_OK;
}

int flusi_set_stream(flusi_plan plan, void* stream) {
    if (int rc = check_plan(plan)) return rc;
    plan->d.stream = static_cast<hipStream_t>(stream);
    return FLUSI_OK;
}

size_t flusi_plan_workspace_bytes(flusi_plan plan) { return plan ? plan->d.workspace : 0; }

size_t flusi_state_bytes(flusi_plan plan) { return (plan && plan->d.impl) ? plan->d.impl->state_bytes() : 0; }

int flusi_tables(flusi_plan plan, int* j_signed, int* keep_signed) {
    if (int rc = check_plan(plan)) return rc;
    const int n = plan->d.n;
    for (int i = 0; i < n; ++i) {
        const int j = i < n / 2 ? i : i - n;
        if (j_signed) j_signed[i] = j;
        if (keep_signed) keep_signed[i] = (3 * (j < 0 ? -j : j) < n) ? 1 : 0;
    }
    return FLUSI_OK;
}

int flusi_fft_r2c(flusi_plan plan, const void* in, void* out, int nf) {
    if (int rc = check_plan(plan)) return rc;
    if (!in || !out || nf < 1) return set_error(FLUSI_EINVAL, "fft_r2c: null pointer or nf < 1");
    return plan->d.impl->fft_r2c(plan->d, in, out, nf);
}

int flusi_fft_c2r(flusi_plan plan, const void* in, void* out, int nf) {
    if (int rc = check_plan(plan)) return rc;
    if (!in || !out || nf < 1) return set_error(FLUSI_EINVAL, "fft_c2r: null pointer or nf < 1");
    return plan->d.impl->fft_c2r(plan->d, in, out, nf);
}

int flusi_mask_insect(flusi_plan plan, const flusi_insect* ins, double t, void* chi, void* us, int16_t* colour) {
    if (int rc = check_plan(plan)) return rc;
    if (!ins) return set_error(FLUSI_EINVAL, "mask_insect: insect is NULL");
    return plan->d.impl->mask(plan->d, *ins, t, chi, us, colour);
}

int flusi_rhs(flusi_plan plan, const void* uhat, const void* chi, const void* us, void* rhs_hat, int mean_mode,
              double* umax_host) {
    if (int rc = check_plan(plan)) return rc;
    if (!uhat || !rhs_hat) return set_error(FLUSI_EINVAL, "rhs: null pointer");
    return plan->d.impl->rhs(plan->d, uhat, chi, us, rhs_hat, mean_mode, umax_host);
}

int flusi_state_init(flusi_plan plan, void* state, const void* u0, double t0) {
    if (int rc = check_plan(plan)) return rc;
    if (!state || !u0) return set_error(FLUSI_EINVAL, "state_init: null pointer");
    return plan->d.impl->state_init(plan->d, state, u0, t0);
}

int flusi_state_export_uhat(flusi_plan plan, const void* state, void* uhat) {
    if (int rc = check_plan(plan)) return rc;
    if (!state || !uhat) return set_error(FLUSI_EINVAL, "state_export_uhat: null pointer");
    return plan->d.impl->export_uhat(plan->d, state, uhat);
}

int flusi_state_velocity(flusi_plan plan, const void* state, void* u) {
    if (int rc = check_plan(plan)) return rc;
    if (!state || !u) return set_error(FLUSI_EINVAL, "state_velocity: null pointer");
    return plan->d.impl->velocity(plan->d, state, u);
}

int flusi_state_time(flusi_plan plan, const void* state, double* t, long long* n) {
    if (int rc = check_plan(plan)) return rc;
    if (!state) return set_error(FLUSI_EINVAL, "state_time: null pointer");
    StateHdr h;
    hipError_t e = hipMemcpyAsync(&h, state, sizeof(StateHdr), hipMemcpyDeviceToHost, plan->d.stream);
    if (e == hipSuccess) e = hipStreamSynchronize(plan->d.stream);
    if (e != hipSuccess) return set_error(FLUSI_EDEVICE, "state_time: %s", hipGetErrorString(e));
    if (t) *t = h.slot[h.cur].t;
    if (n) *n = h.slot[h.cur].n;
    return FLUSI_OK;
}

int flusi_step(flusi_plan plan, void* state, const flusi_insect* ins, const flusi_step_params* p) {
    if (int rc = check_plan(plan)) return rc;
    if (!state || !p) return set_error(FLUSI_EINVAL, "step: null pointer");
    if (p->nsteps < 0) return set_error(FLUSI_EINVAL, "step: nsteps < 0");
    if (!(p->dt_fixed > 0.0) && !(p->cfl > 0.0)) return set_error(FLUSI_EINVAL, "step: need dt_fixed > 0 or cfl > 0");
    if (p->nsteps == 0) return FLUSI_OK;
    return plan->d.impl->step(plan->d, state, ins, *p);
}

int flusi_forces(flusi_plan plan, const void* state, double* out) {
    if (int rc = check_plan(plan)) return rc;
    if (!state || !out) return set_error(FLUSI_EINVAL, "forces: null pointer");
    StateHdr h;
    hipError_t e = hipMemcpyAsync(&h, state, sizeof(StateHdr), hipMemcpyDeviceToHost, plan->d.stream);
    if (e == hipSuccess) e = hipStreamSynchronize(plan->d.stream);
    if (e != hipSuccess) return set_error(FLUSI_EDEVICE, "forces: %s", hipGetErrorString(e));
    std::memcpy(out, h.diag, sizeof(h.diag));
    if (h.status == FLUSI_ENONFINITE) return set_error(FLUSI_ENONFINITE, "velocity became non-finite");
    if (h.status != 0) return set_error(h.status, "state stopped (status %d)", h.status);
    return FLUSI_OK;
}

int flusi_profile(flusi_plan plan, int enable) {
    if (int rc = check_plan(plan)) return rc;
    PlanData& d = plan->d;
    if (enable) {
        d.prof_recs.clear();
        d.ev_used = 0;
    }
    d.prof = enable != 0;
    return FLUSI_OK;
}

int flusi_pass_times(flusi_plan plan, double* ms, long long* launches) {
    if (int rc = check_plan(plan)) return rc;
    PlanData& d = plan->d;
    hipError_t e = hipStreamSynchronize(d.stream);
    if (e != hipSuccess) return set_error(FLUSI_EDEVICE, "pass_times: %s", hipGetErrorString(e));
    double acc[FLUSI_NPASS] = {0};
    long long cnt[FLUSI_NPASS] = {0};
    for (const auto& r : d.prof_recs) {
        float t = 0.0f;
        e = hipEventElapsedTime(&t, d.events[r.second], d.events[r.second + 1]);
        if (e != hipSuccess) return set_error(FLUSI_EDEVICE, "pass_times: %s", hipGetErrorString(e));
        acc[r.first] += t;
        cnt[r.first] += 1;
    }
    for (int i = 0; i < FLUSI_NPASS; ++i) {
        if (ms) ms[i] = acc[i];
        if (launches) launches[i] = cnt[i];
    }
    return FLUSI_OK;
}

}  // extern "C"
