// C ABI of the pseudo-spectral penalized Navier-Stokes library (see include/flusi.h).
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <vector>

#include "impl.hpp"

namespace flusi {

#define FLUSI_SIZE(s) ImplBase* make_impl_##s(int);
#define FLUSI_BOX(x, s) ImplBase* make_impl_##x##_##s(int);
#include "sizes.def"
#undef FLUSI_SIZE
#undef FLUSI_BOX

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

// Instantiated grids: cubic n^3 (FLUSI_SIZE) and nx x n x n boxes (FLUSI_BOX).
static ImplBase* make_impl(int nx, int n, int dtype) {
#define FLUSI_SIZE(s) \
    if (nx == s && n == s) return make_impl_##s(dtype);
#define FLUSI_BOX(x, s) \
    if (nx == x && n == s) return make_impl_##x##_##s(dtype);
#include "sizes.def"
#undef FLUSI_SIZE
#undef FLUSI_BOX
    return nullptr;
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

// Scratch of the allocation-free inverse transform (flusi_fft_c2r_noalloc): a
// fixed array in the code object, one copy per GPU, held until the process
// ends.  Host code never uses the array's name as an address: its device
// address on each GPU comes from hipGetSymbolAddress (noalloc_scratch_of).
constexpr size_t NOALLOC_SCRATCH_BYTES = 64ull << 20;
static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];

// Device address of `scratch` on the current device, resolved once per device
// (null when the runtime cannot give it; the entry point then reports it).
static void* noalloc_scratch_of_current_device() {
    static std::mutex mu;
    static std::map<int, void*> addr;
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) return nullptr;
    std::lock_guard<std::mutex> lk(mu);
    auto it = addr.find(dev);
    if (it != addr.end()) return it->second;
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess) {
        (void)hipGetLastError();
        ptr = nullptr;
    }
    addr[dev] = ptr;
    return ptr;
}

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
    void* ptrs[] = {d.tw, d.twx != d.tw ? d.twx : nullptr, d.bufA, d.bufB, d.partial, d.partial2, d.kin, d.ins_dev, d.member_dev, d.pmax, d.spec, d.phys,
                    d.rtab, d.rtab32, d.ustage};
    for (void* q : ptrs)
        if (q) (void)hipFree(q);
    for (hipEvent_t e : d.events) (void)hipEventDestroy(e);
    d.events.clear();
    if (d.ev_z) (void)hipEventDestroy(d.ev_z);
    if (d.ev_k) (void)hipEventDestroy(d.ev_k);
    if (d.side) (void)hipStreamDestroy(d.side);
    d.ev_z = d.ev_k = nullptr;
    d.side = nullptr;
    delete d.impl;
    d.impl = nullptr;
}
static int sched_check(const flusi_schedule& s) {
    const int v[4] = {s.y_inverse, s.x_pass, s.y_forward, s.z_pass};
    for (int x : v)
        if (x < 0 || x >= NVARIANT) return set_error(FLUSI_EINVAL, "tile variants must be in [0, %d)", NVARIANT);
    if (s.split_z != 0 && s.split_z != 1) return set_error(FLUSI_EINVAL, "split_z must be 0 or 1");
    return FLUSI_OK;
}
static Sched sched_from(const flusi_schedule& s) {
    Sched d;
    d.y_inverse = s.y_inverse;
    d.x_pass = s.x_pass;
    d.y_forward = s.y_forward;
    d.z_pass = s.z_pass;
    d.split_z = s.split_z;
    return d;
}
static flusi_schedule sched_to(const Sched& d) {
    flusi_schedule s{};
    s.y_inverse = d.y_inverse;
    s.x_pass = d.x_pass;
    s.y_forward = d.y_forward;
    s.z_pass = d.z_pass;
    s.split_z = d.split_z;
    return s;
}

// Average time per launch of each stepping pass over reps steps of g with
// schedule sc (prof: plan whose event pool records the passes).
static int time_passes(ImplBase* impl, GroupRun g, const Sched& sc, PlanData& prof, int reps, double* avg_ms) {
    g.sched = sc;
    g.prof = nullptr;
    if (int rc = impl->run_steps(g, 2)) return rc;
    const bool was = prof.prof;
    prof.prof = true;
    prof.prof_recs.clear();
    prof.ev_used = 0;
    g.prof = &prof;
    int rc = impl->run_steps(g, reps);
    prof.prof = was;
    if (rc) return rc;
    hipError_t e = hipStreamSynchronize(g.stream);
    if (e != hipSuccess) return set_error(FLUSI_EDEVICE, "autotune: %s", hipGetErrorString(e));
    double acc[FLUSI_NPASS] = {0};
    int cnt[FLUSI_NPASS] = {0};
    for (const auto& r : prof.prof_recs) {
        float t = 0.0f;
        e = hipEventElapsedTime(&t, prof.events[r.second], prof.events[r.second + 1]);
        if (e != hipSuccess) return set_error(FLUSI_EDEVICE, "autotune: %s", hipGetErrorString(e));
        acc[r.first] += t;
        cnt[r.first] += 1;
    }
    prof.prof_recs.clear();
    prof.ev_used = 0;
    for (int i = 0; i < FLUSI_NPASS; ++i) avg_ms[i] = cnt[i] ? acc[i] / cnt[i] : 0.0;
    return FLUSI_OK;
}

// Whole-step time (ms per step) of g with schedule sc.
static int time_steps(ImplBase* impl, GroupRun g, const Sched& sc, int reps, double* ms_per_step) {
    g.sched = sc;
    g.prof = nullptr;
    if (int rc = impl->run_steps(g, 2)) return rc;
    hipEvent_t a, b;
    if (hipEventCreate(&a) != hipSuccess) return set_error(FLUSI_EDEVICE, "autotune: event");
    if (hipEventCreate(&b) != hipSuccess) {
        (void)hipEventDestroy(a);
        return set_error(FLUSI_EDEVICE, "autotune: event");
    }
    hipError_t e = hipEventRecord(a, g.stream);
    int rc = e == hipSuccess ? impl->run_steps(g, reps) : FLUSI_OK;
    if (e == hipSuccess && !rc) e = hipEventRecord(b, g.stream);
    if (e == hipSuccess && !rc) e = hipEventSynchronize(b);
    float t = 0.0f;
    if (e == hipSuccess && !rc) e = hipEventElapsedTime(&t, a, b);
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    if (rc) return rc;
    if (e != hipSuccess) return set_error(FLUSI_EDEVICE, "autotune: %s", hipGetErrorString(e));
    *ms_per_step = t / reps;
    return FLUSI_OK;
}

// Chooses the fastest variant per pass, then one- or two-launch z-pass.
static int tune_group(ImplBase* impl, const GroupRun& g, PlanData& prof, int reps, Sched* out) {
    double t[NVARIANT][FLUSI_NPASS];
    Sched base = impl->default_sched();
    for (int v = 0; v < NVARIANT; ++v) {
        Sched sc = base;
        sc.y_inverse = sc.x_pass = sc.y_forward = sc.z_pass = v;
        if (int rc = time_passes(impl, g, sc, prof, reps, t[v])) return rc;
    }
    // fastest variant per pass (the z-pass with its inverse launch when split)
    auto pick = [&](auto cost) {
        int b = 0;
        for (int v = 1; v < NVARIANT; ++v)
            if (cost(v) < cost(b)) b = v;
        return b;
    };
    Sched best = base;
    best.y_inverse = pick([&](int v) { return t[v][PASS_YINV]; });
    best.x_pass = pick([&](int v) { return t[v][PASS_X]; });
    best.y_forward = pick([&](int v) { return t[v][PASS_YFWD]; });
    best.z_pass = pick([&](int v) { return t[v][PASS_Z] + t[v][PASS_ZINV]; });
    double ms[2];
    for (int sp = 0; sp < 2; ++sp) {
        Sched sc = best;
        sc.split_z = sp;
        if (int rc = time_steps(impl, g, sc, reps, &ms[sp])) return rc;
    }
    best.split_z = ms[1] < ms[0] ? 1 : 0;
    *out = best;
    return FLUSI_OK;
}

}  // namespace flusi

using namespace flusi;

static_assert(sizeof(flusi_insect) == 16 + 8 * 47 + 16 + 8 * (3 * 2 * (FLUSI_KIN_MAX + 1) + 2 + 2 * (FLUSI_WING_MAX + 1) + 8 + 4 + 6), "flusi_insect layout");
static_assert(sizeof(flusi_step_params) == 8 + 5 * 8 + 8, "flusi_step_params layout");

extern "C" {

const char* flusi_last_error(void) { return g_err; }

int flusi_plan_create(int nx, int ny, int nz, double L, double nu, double eta, int dtype, flusi_plan* out) {
    if (!out) return set_error(FLUSI_EINVAL, "out is NULL");
    *out = nullptr;
    if (ny != nz) return set_error(FLUSI_EUNSUPPORTED, "need ny = nz (%d x %d x %d)", nx, ny, nz);
    if (!(L > 0.0) || !(nu >= 0.0) || !(eta > 0.0)) return set_error(FLUSI_EINVAL, "need L > 0, nu >= 0, eta > 0");
    if (dtype != FLUSI_F32 && dtype != FLUSI_F64) return set_error(FLUSI_EINVAL, "dtype must be FLUSI_F32 or FLUSI_F64");
    ImplBase* impl = make_impl(nx, ny, dtype);
    if (!impl) return set_error(FLUSI_EUNSUPPORTED, "grid %d x %d x %d not supported", nx, ny, nz);
    flusi_plan p = new (std::nothrow) flusi_plan_s();
    if (!p) {
        delete impl;
        return set_error(FLUSI_ENOMEM, "host allocation");
    }
    PlanData& d = p->d;
    d.impl = impl;
    d.n = ny;
    d.nx = nx;
    d.dtype = dtype;
    d.L = L;
    d.Lx = nx == ny ? L : L * nx / ny;
    d.nu = nu;
    d.eta = eta;
    d.K = kmax_of(ny);
    d.KP = kmax_of(nx) + 1;
    d.M = 2 * d.K + 1;
    d.Q = d.M * d.KP;
    const size_t cxb = dtype == FLUSI_F32 ? 8 : 16;
    d.szA = impl->bufA_elems() * cxb;
    d.szB = impl->bufB_elems() * cxb;
    d.nwg_x = impl->nwg_x();
    const int n = ny;
    bool ok = hipMalloc(&d.tw, n * cxb) == hipSuccess;
    if (nx != n) ok = ok && hipMalloc(&d.twx, nx * cxb) == hipSuccess;
    else d.twx = d.tw;
    ok = ok && hipMalloc(&d.bufA, d.szA) == hipSuccess;
    ok = ok && hipMalloc(&d.bufB, d.szB) == hipSuccess;
    ok = ok && hipMalloc(&d.partial, (size_t)d.nwg_x * NV * sizeof(double)) == hipSuccess;
    ok = ok && hipMalloc(&d.partial2, (size_t)NRED_MAX * NV * sizeof(double)) == hipSuccess;
    ok = ok && hipMalloc(&d.kin, sizeof(Kin)) == hipSuccess;
    ok = ok && hipMalloc(&d.ins_dev, sizeof(flusi_insect)) == hipSuccess;
    ok = ok && hipMalloc(&d.member_dev, sizeof(Member)) == hipSuccess;
    ok = ok && hipMalloc(&d.rtab, RTAB_BYTES64) == hipSuccess;
    ok = ok && hipMalloc(&d.rtab32, RTAB_BYTES32) == hipSuccess;
    ok = ok && hipStreamCreateWithFlags(&d.side, hipStreamNonBlocking) == hipSuccess;
    ok = ok && hipEventCreateWithFlags(&d.ev_z, hipEventDisableTiming) == hipSuccess;
    ok = ok && hipEventCreateWithFlags(&d.ev_k, hipEventDisableTiming) == hipSuccess;
    d.sched = impl->default_sched();
    d.noalloc_scratch = noalloc_scratch_of_current_device();
    if (!ok) {
        free_plan(d);
        delete p;
        return set_error(FLUSI_ENOMEM, "device allocation for a %d x %d x %d plan", nx, ny, nz);
    }
    d.workspace = (n + (nx != n ? nx : 0)) * cxb + d.szA + d.szB + (size_t)d.nwg_x * NV * 8 + NRED_MAX * NV * 8 + sizeof(Kin) + sizeof(flusi_insect) +
                  sizeof(Member) + RTAB_BYTES64 + RTAB_BYTES32;
    // FP64 twiddles exp(-2 pi i m / len); the FP32 tables are rounded from them.
    const auto upload = [&](void* dst, int len) {
        std::vector<double> w(2 * len);
        for (int m = 0; m < len; ++m) {
            double c, s;
            sincos_2pi(m, len, &c, &s);
            w[2 * m] = c;
            w[2 * m + 1] = -s;
        }
        if (dtype == FLUSI_F64) return hipMemcpy(dst, w.data(), len * cxb, hipMemcpyHostToDevice);
        std::vector<float> wf(2 * len);
        for (int i = 0; i < 2 * len; ++i) wf[i] = (float)w[i];
        return hipMemcpy(dst, wf.data(), len * cxb, hipMemcpyHostToDevice);
    };
    hipError_t e = upload(d.tw, n);
    if (e == hipSuccess && nx != n) e = upload(d.twx, nx);
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

int flusi_sizes(int n, int dtype, size_t* workspace_bytes, size_t* state_bytes) {
    if (dtype != FLUSI_F32 && dtype != FLUSI_F64) return set_error(FLUSI_EINVAL, "dtype must be FLUSI_F32 or FLUSI_F64");
    ImplBase* impl = make_impl(n, n, dtype);
    if (!impl) return set_error(FLUSI_EUNSUPPORTED, "grid size %d not supported", n);
    const size_t cxb = dtype == FLUSI_F32 ? 8 : 16;
    if (workspace_bytes)
        *workspace_bytes = n * cxb + impl->bufA_elems() * cxb + impl->bufB_elems() * cxb +
                           (size_t)impl->nwg_x() * NV * 8 + NRED_MAX * NV * 8 + sizeof(Kin) + sizeof(flusi_insect) +
                           sizeof(Member) + RTAB_BYTES64 + RTAB_BYTES32;
    if (state_bytes) *state_bytes = impl->state_bytes();
    delete impl;
    return FLUSI_OK;
}

int flusi_plan_set_walls(flusi_plan plan, const double* thickness, const double* u_wall) {
    if (int rc = check_plan(plan)) return rc;
    PlanData& d = plan->d;
    double th[3] = {0.0, 0.0, 0.0}, uw[3] = {0.0, 0.0, 0.0};
    for (int a = 0; a < 3; ++a) {
        if (thickness) th[a] = thickness[a];
        if (u_wall) uw[a] = u_wall[a];
        if (!(th[a] >= 0.0) || !(th[a] <= (a == 0 ? d.Lx : d.L)) || !std::isfinite(uw[a]))
            return set_error(FLUSI_EINVAL, "set_walls: thickness in [0, side] and finite velocity");
    }
    for (int a = 0; a < 3; ++a) {
        d.wall_th[a] = th[a];
        d.u_wall[a] = uw[a];
    }
    d.gen += 1;
    return FLUSI_OK;
}

int flusi_plan_set_sponge(flusi_plan plan, double c_sp, const double* thickness) {
    if (int rc = check_plan(plan)) return rc;
    PlanData& d = plan->d;
    double th[3] = {0.0, 0.0, 0.0};
    if (thickness)
        for (int a = 0; a < 3; ++a) {
            if (!(thickness[a] >= 0.0) || thickness[a] > (a == 0 ? d.Lx : d.L))
                return set_error(FLUSI_EINVAL, "set_sponge: thickness must be in [0, side]");
            th[a] = thickness[a];
        }
    const bool on = c_sp > 0.0 && (th[0] > 0.0 || th[1] > 0.0 || th[2] > 0.0);
    if (on) {
        const size_t cxb = d.dtype == FLUSI_F32 ? 8 : 16;
        const size_t need = d.impl->bufA_elems_sponge() * cxb;
        if (need > d.szA) {
            void* nb = nullptr;
            // the old buffer may still be in use on any stream (the plan's own, or
            // the streams of an ensemble that holds the plan)
            (void)hipDeviceSynchronize();
            if (hipMalloc(&nb, need) != hipSuccess) return set_error(FLUSI_ENOMEM, "set_sponge: scratch");
            (void)hipFree(d.bufA);
            d.workspace += need - d.szA;
            d.bufA = nb;
            d.szA = need;
        }
    }
    d.c_sp = on ? c_sp : 0.0;
    for (int a = 0; a < 3; ++a) d.sp_thick[a] = on ? th[a] : 0.0;
    d.gen += 1;
    return FLUSI_OK;
}

int flusi_plan_set_integrator(flusi_plan plan, int integrator) {
    if (int rc = check_plan(plan)) return rc;
    if (integrator != FLUSI_INT_AB2 && integrator != FLUSI_INT_RK4)
        return set_error(FLUSI_EINVAL, "set_integrator: FLUSI_INT_AB2 or FLUSI_INT_RK4");
    PlanData& d = plan->d;
    if (integrator == FLUSI_INT_RK4 && !d.ustage) {
        const size_t need = d.impl->field3_bytes();
        if (hipMalloc(&d.ustage, need) != hipSuccess) {
            d.ustage = nullptr;
            return set_error(FLUSI_ENOMEM, "set_integrator: stage velocity");
        }
        d.ustage_sz = need;
        d.workspace += need;
    }
    d.integrator = integrator;
    d.gen += 1;
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

int flusi_fft_c2r_noalloc(flusi_plan plan, const void* in, void* out, int nf) {
    if (int rc = check_plan(plan)) return rc;
    if (!in || !out || nf <= 0) return set_error(FLUSI_EINVAL, "fft_c2r_noalloc: bad arguments");
    PlanData& d = plan->d;
    const size_t need = (size_t)nf * d.impl->spec_bytes();
    if (need > NOALLOC_SCRATCH_BYTES)
        return set_error(FLUSI_EINVAL,
                         "fft_c2r_noalloc: %d field(s) of %d x %d x %d need %zu bytes of scratch, above the "
                         "fixed %zu-byte array (use flusi_fft_c2r)",
                         nf, d.nx, d.n, d.n, need, (size_t)NOALLOC_SCRATCH_BYTES);
    if (!d.noalloc_scratch) return set_error(FLUSI_EDEVICE, "fft_c2r_noalloc: no device address for the scratch array");
    return d.impl->fft_c2r_into(d, in, out, nf, d.noalloc_scratch);
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

int flusi_state_solid(flusi_plan plan, const void* state, double* out) {
    if (int rc = check_plan(plan)) return rc;
    if (!state || !out) return set_error(FLUSI_EINVAL, "state_solid: null pointer");
    StateHdr h;
    hipError_t e = hipMemcpyAsync(&h, state, sizeof(StateHdr), hipMemcpyDeviceToHost, plan->d.stream);
    if (e == hipSuccess) e = hipStreamSynchronize(plan->d.stream);
    if (e != hipSuccess) return set_error(FLUSI_EDEVICE, "state_solid: %s", hipGetErrorString(e));
    if (h.status == FLUSI_ENONFINITE) return set_error(FLUSI_ENONFINITE, "velocity became non-finite");
    if (h.status != 0) return set_error(h.status, "state stopped (status %d)", h.status);
    const Slot& sl = h.slot[h.cur];
    if (sl.ff_state != 1) return set_error(FLUSI_EINVAL, "state_solid: the state has no free-flight body");
    std::memcpy(out, sl.ff, sizeof(sl.ff));
    return FLUSI_OK;
}

int flusi_state_set_solid(flusi_plan plan, void* state, const double* y) {
    if (int rc = check_plan(plan)) return rc;
    if (!state || !y) return set_error(FLUSI_EINVAL, "state_set_solid: null pointer");
    Solid13 v;
    double q = 0.0;
    for (int i = 0; i < 13; ++i) {
        if (!std::isfinite(y[i])) return set_error(FLUSI_EINVAL, "state_set_solid: value %d not finite", i);
        v.v[i] = y[i];
    }
    for (int i = 6; i < 10; ++i) q += y[i] * y[i];
    if (std::fabs(q - 1.0) > 1e-12) return set_error(FLUSI_EINVAL, "state_set_solid: quaternion not of unit length");
    k_solid_set<<<1, 64, 0, plan->d.stream>>>(static_cast<StateHdr*>(state), v);
    return launch_check("state_set_solid");
}

int flusi_step(flusi_plan plan, void* state, const flusi_insect* ins, const flusi_step_params* p) {
    if (int rc = check_plan(plan)) return rc;
    if (!state || !p) return set_error(FLUSI_EINVAL, "step: null pointer");
    if (int rc = check_insect(ins)) return rc;
    if (p->nsteps < 0) return set_error(FLUSI_EINVAL, "step: nsteps < 0");
    if (!(p->dt_fixed > 0.0) && !(p->cfl > 0.0)) return set_error(FLUSI_EINVAL, "step: need dt_fixed > 0 or cfl > 0");
    if (plan->d.integrator == FLUSI_INT_RK4 && free_flight_on(ins))
        return set_error(FLUSI_EUNSUPPORTED, "step: free flight is stepped with AB2 only");
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

int flusi_plan_get_schedule(flusi_plan plan, flusi_schedule* out) {
    if (int rc = check_plan(plan)) return rc;
    if (!out) return set_error(FLUSI_EINVAL, "get_schedule: out is NULL");
    *out = sched_to(plan->d.sched);
    return FLUSI_OK;
}

int flusi_plan_set_schedule(flusi_plan plan, const flusi_schedule* s) {
    if (int rc = check_plan(plan)) return rc;
    if (!s) return set_error(FLUSI_EINVAL, "set_schedule: schedule is NULL");
    if (int rc = sched_check(*s)) return rc;
    plan->d.sched = sched_from(*s);
    plan->d.gen += 1;
    return FLUSI_OK;
}

int flusi_autotune(flusi_plan plan, const void* state, const flusi_insect* ins, const flusi_step_params* p, int reps,
                   flusi_schedule* out) {
    if (int rc = check_plan(plan)) return rc;
    if (!state || !p) return set_error(FLUSI_EINVAL, "autotune: null pointer");
    if (reps < 1) return set_error(FLUSI_EINVAL, "autotune: reps < 1");
    if (int rc = check_insect(ins)) return rc;
    if (!(p->dt_fixed > 0.0) && !(p->cfl > 0.0)) return set_error(FLUSI_EINVAL, "autotune: need dt_fixed > 0 or cfl > 0");
    PlanData& d = plan->d;
    const size_t sb = d.impl->state_bytes();
    void* tmp = nullptr;
    if (hipMalloc(&tmp, sb) != hipSuccess) return set_error(FLUSI_ENOMEM, "autotune: scratch state");
    hipError_t e = hipMemcpyAsync(tmp, state, sb, hipMemcpyDeviceToDevice, d.stream);
    flusi_step_params sp = *p;
    sp.history = nullptr;
    const Member m = make_member(d, tmp, ins, sp);
    if (e == hipSuccess) {
        k_member_set<<<1, 64, 0, d.stream>>>(d.member_dev, m, m.nc > 0 ? *ins : flusi_insect{});
        e = hipGetLastError();
    }
    int rc = FLUSI_OK;
    if (e == hipSuccess && m.nc > 0) rc = prepare_wing_table(d, ins, d.stream);
    if (e != hipSuccess) rc = set_error(FLUSI_EDEVICE, "autotune: %s", hipGetErrorString(e));
    Sched best;
    if (!rc) {
        GroupRun g;
        g.mt = d.member_dev;
        g.nmem = 1;
        g.n_nc[m.sponge][colour_slot(m.nc)] = 1;
        g.any_dyn = m.dyn != 0;
        g.any_ff = m.ff != 0;
        g.rk = m.rk != 0;
        g.tw = d.tw;
        g.twx = d.twx;
        g.stream = d.stream;
        rc = tune_group(d.impl, g, d, reps, &best);
    }
    (void)hipStreamSynchronize(d.stream);
    (void)hipFree(tmp);
    if (rc) return rc;
    d.sched = best;
    d.gen += 1;
    if (out) *out = sched_to(best);
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

// ---------------------------------------------------------------------------
// Ensembles
// ---------------------------------------------------------------------------
namespace flusi {
int insect_error(const flusi_insect* ins) { return check_insect(ins); }

struct EnsMember {
    flusi_plan plan = nullptr;
    void* state = nullptr;
    bool has_ins = false;
    flusi_insect ins{};
    flusi_step_params sp{};
    bool used = false;
    unsigned long gen = 0;  // the plan's option generation the launch tables were built from
};
struct EnsGroup {
    int n = 0;
    ImplBase* impl = nullptr;
    flusi_plan p0 = nullptr;  // member plan that holds the group's schedule
    Member* dev = nullptr;  // device member table
    GroupRun run;
    hipEvent_t done = nullptr;
};
}  // namespace flusi

struct flusi_ensemble_s {
    int dtype = 0;
    hipStream_t ext = nullptr;   // caller's stream
    hipStream_t own = nullptr;   // ordering/capture stream of the ensemble
    hipEvent_t ev_in = nullptr, ev_out = nullptr, fork = nullptr;
    std::vector<flusi::EnsMember> members;
    std::vector<flusi::EnsGroup> groups;
    std::vector<hipStream_t> pool;  // one stream per size group
    std::map<int, hipGraphExec_t> graphs;
    bool dirty = true;
};

namespace flusi {
static void ens_clear_groups(flusi_ensemble e) {
    for (auto& g : e->groups) {
        if (g.dev) (void)hipFree(g.dev);
        if (g.done) (void)hipEventDestroy(g.done);
    }
    e->groups.clear();
    for (auto& kv : e->graphs) (void)hipGraphExecDestroy(kv.second);
    e->graphs.clear();
}

// A member plan whose options changed since the tables were built (sponge,
// walls, integrator, schedule) makes the ensemble rebuild them: the records
// carry the plan's buffers and flags, and the captured graphs their pointers.
static void ens_check_plans(flusi_ensemble e) {
    for (const auto& m : e->members)
        if (m.used && m.plan->d.gen != m.gen) e->dirty = true;
}

// Groups the members by grid size, orders each group by colour count and
// uploads the launch tables (synchronous; outside the stepping hot path).
static int ens_rebuild(flusi_ensemble e) {
    ens_check_plans(e);
    if (!e->dirty) return FLUSI_OK;
    hipError_t err = hipStreamSynchronize(e->own);
    if (err != hipSuccess) return set_error(FLUSI_EDEVICE, "ensemble: %s", hipGetErrorString(err));
    ens_clear_groups(e);
    // key: grid shape (nx, n) and integrator (the RK4 and AB2 pass sequences differ)
    std::map<long, std::vector<int>> by_n;
    for (int i = 0; i < (int)e->members.size(); ++i)
        if (e->members[i].used) {
            const PlanData& pd = e->members[i].plan->d;
            by_n[((long)pd.nx * 65536 + pd.n) * 2 + (pd.integrator == FLUSI_INT_RK4 ? 1 : 0)].push_back(i);
        }
    for (auto& kv : by_n) {
        std::vector<int>& ids = kv.second;
        // order: without sponge, then with; within each, by colour count
        auto key = [&](int i) {
            const int nc = colour_count(e->members[i].has_ins ? &e->members[i].ins : nullptr);
            return (sponge_on(e->members[i].plan->d) ? 8 : 0) + nc;
        };
        std::stable_sort(ids.begin(), ids.end(), [&](int a, int b) { return key(a) < key(b); });
        EnsGroup g;
        g.n = (int)(kv.first / 2 % 65536);
        g.run.rk = (kv.first & 1) != 0;
        g.p0 = e->members[ids[0]].plan;
        const PlanData& p0 = g.p0->d;
        g.impl = p0.impl;
        std::vector<Member> host;
        for (int i : ids) {
            EnsMember& m = e->members[i];
            PlanData& pd = m.plan->d;
            m.gen = pd.gen;
            const flusi_insect* ins = m.has_ins ? &m.ins : nullptr;
            if (ins) {
                err = hipMemcpy(pd.ins_dev, ins, sizeof(flusi_insect), hipMemcpyHostToDevice);
                if (err != hipSuccess) return set_error(FLUSI_EDEVICE, "ensemble: %s", hipGetErrorString(err));
                if (int rc = prepare_wing_table(pd, ins, pd.stream)) return rc;
                err = hipStreamSynchronize(pd.stream);
                if (err != hipSuccess) return set_error(FLUSI_EDEVICE, "ensemble: %s", hipGetErrorString(err));
            }
            const Member rec = make_member(pd, m.state, ins, m.sp);
            host.push_back(rec);
            g.run.n_nc[rec.sponge][colour_slot(rec.nc)] += 1;
            g.run.any_dyn = g.run.any_dyn || rec.dyn;
            g.run.any_ff = g.run.any_ff || rec.ff;
        }
        if (hipMalloc(&g.dev, host.size() * sizeof(Member)) != hipSuccess)
            return set_error(FLUSI_ENOMEM, "ensemble: member table");
        err = hipMemcpy(g.dev, host.data(), host.size() * sizeof(Member), hipMemcpyHostToDevice);
        if (err == hipSuccess) err = hipEventCreateWithFlags(&g.done, hipEventDisableTiming);
        if (err != hipSuccess) {
            (void)hipFree(g.dev);
            return set_error(FLUSI_EDEVICE, "ensemble: %s", hipGetErrorString(err));
        }
        g.run.mt = g.dev;
        g.run.nmem = (int)host.size();
        g.run.tw = p0.tw;
        g.run.twx = p0.twx;
        g.run.sched = p0.sched;
        e->groups.push_back(g);
    }
    while (e->pool.size() < e->groups.size()) {
        hipStream_t st;
        err = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
        if (err != hipSuccess) return set_error(FLUSI_EDEVICE, "ensemble: %s", hipGetErrorString(err));
        e->pool.push_back(st);
    }
    e->dirty = false;
    return FLUSI_OK;
}

// Enqueues nsteps of every group on e->own (forking one stream per group).
static int ens_launch(flusi_ensemble e, int nsteps) {
    if (e->groups.size() == 1) {
        GroupRun r = e->groups[0].run;
        r.stream = e->own;
        return e->groups[0].impl->run_steps(r, nsteps);
    }
    hipError_t err = hipEventRecord(e->fork, e->own);
    for (size_t i = 0; i < e->groups.size() && err == hipSuccess; ++i) {
        EnsGroup& g = e->groups[i];
        err = hipStreamWaitEvent(e->pool[i], e->fork, 0);
        if (err != hipSuccess) break;
        GroupRun r = g.run;
        r.stream = e->pool[i];
        if (int rc = g.impl->run_steps(r, nsteps)) return rc;
        err = hipEventRecord(g.done, e->pool[i]);
        if (err == hipSuccess) err = hipStreamWaitEvent(e->own, g.done, 0);
    }
    if (err != hipSuccess) return set_error(FLUSI_EDEVICE, "ensemble step: %s", hipGetErrorString(err));
    return FLUSI_OK;
}
}  // namespace flusi

extern "C" {

int flusi_ensemble_create(int dtype, flusi_ensemble* out) {
    if (!out) return set_error(FLUSI_EINVAL, "out is NULL");
    *out = nullptr;
    if (dtype != FLUSI_F32 && dtype != FLUSI_F64) return set_error(FLUSI_EINVAL, "dtype must be FLUSI_F32 or FLUSI_F64");
    flusi_ensemble e = new (std::nothrow) flusi_ensemble_s();
    if (!e) return set_error(FLUSI_ENOMEM, "host allocation");
    e->dtype = dtype;
    hipError_t err = hipStreamCreateWithFlags(&e->own, hipStreamNonBlocking);
    if (err == hipSuccess) err = hipEventCreateWithFlags(&e->ev_in, hipEventDisableTiming);
    if (err == hipSuccess) err = hipEventCreateWithFlags(&e->ev_out, hipEventDisableTiming);
    if (err == hipSuccess) err = hipEventCreateWithFlags(&e->fork, hipEventDisableTiming);
    if (err != hipSuccess) {
        flusi_ensemble_destroy(e);
        return set_error(FLUSI_EDEVICE, "ensemble_create: %s", hipGetErrorString(err));
    }
    *out = e;
    return FLUSI_OK;
}

int flusi_ensemble_destroy(flusi_ensemble e) {
    if (!e) return FLUSI_OK;
    if (e->own) (void)hipStreamSynchronize(e->own);
    ens_clear_groups(e);
    for (hipStream_t s : e->pool) (void)hipStreamDestroy(s);
    if (e->ev_in) (void)hipEventDestroy(e->ev_in);
    if (e->ev_out) (void)hipEventDestroy(e->ev_out);
    if (e->fork) (void)hipEventDestroy(e->fork);
    if (e->own) (void)hipStreamDestroy(e->own);
    delete e;
    return FLUSI_OK;
}

int flusi_ensemble_set_stream(flusi_ensemble e, void* stream) {
    if (!e) return set_error(FLUSI_EINVAL, "null ensemble");
    e->ext = static_cast<hipStream_t>(stream);
    return FLUSI_OK;
}

int flusi_ensemble_add(flusi_ensemble e, flusi_plan plan, void* state, const flusi_insect* ins,
                       const flusi_step_params* p, int* id) {
    if (!e) return set_error(FLUSI_EINVAL, "null ensemble");
    if (int rc = check_plan(plan)) return rc;
    if (!state || !p) return set_error(FLUSI_EINVAL, "ensemble_add: null pointer");
    if (int rc = check_insect(ins)) return rc;
    if (plan->d.dtype != e->dtype) return set_error(FLUSI_EINVAL, "ensemble_add: plan dtype differs from the ensemble's");
    if (plan->d.integrator == FLUSI_INT_RK4 && free_flight_on(ins))
        return set_error(FLUSI_EUNSUPPORTED, "ensemble_add: free flight is stepped with AB2 only");
    if (!(p->dt_fixed > 0.0) && !(p->cfl > 0.0)) return set_error(FLUSI_EINVAL, "ensemble_add: need dt_fixed > 0 or cfl > 0");
    for (const auto& m : e->members)
        if (m.used && m.plan == plan) return set_error(FLUSI_EINVAL, "ensemble_add: plan is already a member");
    EnsMember m;
    m.plan = plan;
    m.state = state;
    m.has_ins = colour_count(ins) > 0;
    if (m.has_ins) m.ins = *ins;
    m.sp = *p;
    m.sp.nsteps = 0;
    m.used = true;
    int slot = -1;
    for (int i = 0; i < (int)e->members.size(); ++i)
        if (!e->members[i].used) {
            slot = i;
            break;
        }
    if (slot < 0) {
        slot = (int)e->members.size();
        e->members.push_back(m);
    } else {
        e->members[slot] = m;
    }
    e->dirty = true;
    if (id) *id = slot;
    return FLUSI_OK;
}

int flusi_ensemble_remove(flusi_ensemble e, int id) {
    if (!e) return set_error(FLUSI_EINVAL, "null ensemble");
    if (id < 0 || id >= (int)e->members.size() || !e->members[id].used)
        return set_error(FLUSI_EINVAL, "ensemble_remove: no member %d", id);
    e->members[id].used = false;
    e->dirty = true;
    return FLUSI_OK;
}

int flusi_ensemble_size(flusi_ensemble e, int* members, int* groups) {
    if (!e) return set_error(FLUSI_EINVAL, "null ensemble");
    if (int rc = ens_rebuild(e)) return rc;
    int n = 0;
    for (const auto& m : e->members) n += m.used ? 1 : 0;
    if (members) *members = n;
    if (groups) *groups = (int)e->groups.size();
    return FLUSI_OK;
}

int flusi_ensemble_step(flusi_ensemble e, int nsteps, int use_graph) {
    if (!e) return set_error(FLUSI_EINVAL, "null ensemble");
    if (nsteps < 0) return set_error(FLUSI_EINVAL, "ensemble_step: nsteps < 0");
    if (int rc = ens_rebuild(e)) return rc;
    if (nsteps == 0 || e->groups.empty()) return FLUSI_OK;
    hipError_t err = hipEventRecord(e->ev_in, e->ext);
    if (err == hipSuccess) err = hipStreamWaitEvent(e->own, e->ev_in, 0);
    if (err != hipSuccess) return set_error(FLUSI_EDEVICE, "ensemble_step: %s", hipGetErrorString(err));
    if (use_graph) {
        auto it = e->graphs.find(nsteps);
        if (it == e->graphs.end()) {
            err = hipStreamBeginCapture(e->own, hipStreamCaptureModeThreadLocal);
            if (err != hipSuccess) return set_error(FLUSI_EDEVICE, "ensemble capture: %s", hipGetErrorString(err));
            const int rc = ens_launch(e, nsteps);
            hipGraph_t graph = nullptr;
            err = hipStreamEndCapture(e->own, &graph);
            if (rc) {
                if (graph) (void)hipGraphDestroy(graph);
                return rc;
            }
            if (err != hipSuccess) return set_error(FLUSI_EDEVICE, "ensemble capture: %s", hipGetErrorString(err));
            hipGraphExec_t exec = nullptr;
            err = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
            (void)hipGraphDestroy(graph);
            if (err != hipSuccess) return set_error(FLUSI_EDEVICE, "ensemble graph: %s", hipGetErrorString(err));
            it = e->graphs.emplace(nsteps, exec).first;
        }
        err = hipGraphLaunch(it->second, e->own);
        if (err != hipSuccess) return set_error(FLUSI_EDEVICE, "ensemble graph launch: %s", hipGetErrorString(err));
    } else {
        if (int rc = ens_launch(e, nsteps)) return rc;
    }
    err = hipEventRecord(e->ev_out, e->own);
    if (err == hipSuccess) err = hipStreamWaitEvent(e->ext, e->ev_out, 0);
    if (err != hipSuccess) return set_error(FLUSI_EDEVICE, "ensemble_step: %s", hipGetErrorString(err));
    return FLUSI_OK;
}

int flusi_ensemble_autotune(flusi_ensemble e, int reps) {
    if (!e) return set_error(FLUSI_EINVAL, "null ensemble");
    if (reps < 1) return set_error(FLUSI_EINVAL, "ensemble_autotune: reps < 1");
    if (int rc = ens_rebuild(e)) return rc;
    hipError_t err = hipStreamSynchronize(e->own);
    if (err != hipSuccess) return set_error(FLUSI_EDEVICE, "ensemble_autotune: %s", hipGetErrorString(err));
    for (auto& g : e->groups) {
        // member records of the group, pointing at scratch copies of the states
        std::vector<Member> host(g.run.nmem);
        err = hipMemcpy(host.data(), g.dev, host.size() * sizeof(Member), hipMemcpyDeviceToHost);
        if (err != hipSuccess) return set_error(FLUSI_EDEVICE, "ensemble_autotune: %s", hipGetErrorString(err));
        std::vector<void*> copies;
        Member* dev = nullptr;
        int rc = FLUSI_OK;
        const size_t sb = g.impl->state_bytes();
        for (auto& m : host) {
            void* c = nullptr;
            if (hipMalloc(&c, sb) != hipSuccess) {
                rc = set_error(FLUSI_ENOMEM, "ensemble_autotune: scratch states");
                break;
            }
            copies.push_back(c);
            err = hipMemcpy(c, m.hdr, sb, hipMemcpyDeviceToDevice);
            if (err != hipSuccess) {
                rc = set_error(FLUSI_EDEVICE, "ensemble_autotune: %s", hipGetErrorString(err));
                break;
            }
            m.hdr = static_cast<StateHdr*>(c);
            m.history = nullptr;
        }
        if (!rc && hipMalloc(&dev, host.size() * sizeof(Member)) != hipSuccess)
            rc = set_error(FLUSI_ENOMEM, "ensemble_autotune: member table");
        if (!rc) {
            err = hipMemcpy(dev, host.data(), host.size() * sizeof(Member), hipMemcpyHostToDevice);
            if (err != hipSuccess) rc = set_error(FLUSI_EDEVICE, "ensemble_autotune: %s", hipGetErrorString(err));
        }
        Sched best;
        if (!rc) {
            GroupRun r = g.run;
            r.mt = dev;
            r.stream = e->own;
            // the group's first plan holds the schedule and lends its event pool
            rc = tune_group(g.impl, r, g.p0->d, reps, &best);
            if (!rc) {
                g.p0->d.sched = best;
                g.run.sched = best;
            }
        }
        (void)hipStreamSynchronize(e->own);
        for (void* c : copies) (void)hipFree(c);
        if (dev) (void)hipFree(dev);
        if (rc) return rc;
    }
    for (auto& kv : e->graphs) (void)hipGraphExecDestroy(kv.second);
    e->graphs.clear();
    return FLUSI_OK;
}

}  // extern "C"
