// Host-side launch logic of one (real type, grid size) instantiation.
#pragma once
#include <cstddef>
#include <cstdint>
#include <vector>

#include "kernels.hpp"

namespace flusi {

struct ImplBase;

// Plan contents shared with the launchers.
struct PlanData {
    int n = 0, dtype = 0;
    double L = 0, nu = 0, eta = 0;
    int K = 0, KP = 0, M = 0, Q = 0;
    hipStream_t stream = nullptr;
    void* tw = nullptr;  // n twiddles exp(-2 pi i m/n) of the plan's real type
    void* bufA = nullptr;
    void* bufB = nullptr;
    size_t szA = 0, szB = 0;
    double* partial = nullptr;
    int nwg_x = 0;
    double* partial2 = nullptr;
    Kin* kin = nullptr;
    flusi_insect* ins_dev = nullptr;  // device copy of the insect of the current stepping call
    double* pmax = nullptr;
    int npmax = 0;
    void* spec = nullptr;  // lazily allocated full-layout scratch
    size_t spec_sz = 0;
    void* phys = nullptr;
    size_t phys_sz = 0;
    size_t workspace = 0;
    ImplBase* impl = nullptr;
    // instrumentation (flusi_profile)
    bool prof = false;
    std::vector<hipEvent_t> events;
    size_t ev_used = 0;
    std::vector<std::pair<int, size_t>> prof_recs;
};

// Brackets one launch with a pair of events when profiling is on.
struct PassScope {
    PlanData& p;
    int pass;
    size_t idx = 0;
    PassScope(PlanData& pd, int ps) : p(pd), pass(ps) {
        if (!p.prof) return;
        while (p.events.size() < p.ev_used + 2) {
            hipEvent_t e;
            if (hipEventCreate(&e) != hipSuccess) {
                p.prof = false;
                return;
            }
            p.events.push_back(e);
        }
        idx = p.ev_used;
        p.ev_used += 2;
        (void)hipEventRecord(p.events[idx], p.stream);
    }
    ~PassScope() {
        if (!p.prof) return;
        (void)hipEventRecord(p.events[idx + 1], p.stream);
        p.prof_recs.emplace_back(pass, idx);
    }
};
enum { PASS_ZINV = 0, PASS_YINV = 1, PASS_X = 2, PASS_SCALAR = 3, PASS_YFWD = 4, PASS_Z = 5 };

int set_error(int code, const char* fmt, ...);
int ensure_scratch(void** ptr, size_t* cur, size_t need, PlanData& p);

struct ImplBase {
    virtual ~ImplBase() {}
    virtual size_t bufA_elems() const = 0;
    virtual size_t bufB_elems() const = 0;
    virtual int nwg_x() const = 0;
    virtual size_t state_bytes() const = 0;
    virtual int fft_r2c(PlanData&, const void*, void*, int) = 0;
    virtual int fft_c2r(PlanData&, const void*, void*, int) = 0;
    virtual int mask(PlanData&, const flusi_insect&, double, void*, void*, int16_t*) = 0;
    virtual int rhs(PlanData&, const void*, const void*, const void*, void*, int, double*) = 0;
    virtual int state_init(PlanData&, void*, const void*, double) = 0;
    virtual int export_uhat(PlanData&, const void*, void*) = 0;
    virtual int velocity(PlanData&, const void*, void*) = 0;
    virtual int step(PlanData&, void*, const flusi_insect*, const flusi_step_params&) = 0;
};

inline int launch_check(const char* what) {
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return set_error(FLUSI_EDEVICE, "%s: %s", what, hipGetErrorString(e));
    return FLUSI_OK;
}

template <typename T, int N>
struct Impl final : ImplBase {
    using CX = cx<T>;
    static constexpr int K = kmax_of(N), KP = K + 1, M = 2 * K + 1, Q = M * KP;
    static constexpr int KPp = Geo<T, N>::KPp, Qp = Geo<T, N>::Qp;
    static constexpr int C = cols_of(N), RW = rows_x(N, sizeof(cx<T>)), NKX = N / 2 + 1;
    static constexpr int CZ = cols_z(N), NTZ = nt_z(N);
    static constexpr long N2 = (long)N * N, N3 = (long)N * N * N;
    static constexpr long FULL = N2 * NKX;  // full-layout spectrum per field

    size_t bufA_elems() const override {
        const size_t a = 6ul * N * Qp, b = 3ul * N2 * KPp;
        return a > b ? a : b;
    }
    size_t bufB_elems() const override {
        const size_t a = 6ul * N2 * KPp, b = 3ul * N * Qp;
        return a > b ? a : b;
    }
    int nwg_x() const override { return (int)(N2 / RW); }
    static size_t field_bytes() { return (size_t)M * Qp * sizeof(CX); }
    size_t state_bytes() const override { return STATE_HDR_BYTES + 6 * ((field_bytes() + 255) / 256 * 256); }

    static CX* st_uhat(void* st) { return reinterpret_cast<CX*>(static_cast<char*>(st) + STATE_HDR_BYTES); }
    static long st_fs() { return (long)((field_bytes() + 255) / 256 * 256 / sizeof(CX)); }
    static CX* st_nold(void* st) { return st_uhat(st) + 3 * st_fs(); }

    const CX* tw(const PlanData& p) const { return static_cast<const CX*>(p.tw); }
    // The z-pass runs as two launches (forward + update, then curl + inverse)
    // when one fused launch would hold too many registers per thread.
    static constexpr bool split_z() { return N >= 192; }

    // --- full-layout column passes ------------------------------------------------
    // column launch over nf fields, 1D grid of nbx*nf (+ extra) workgroups
    template <int DIR, bool PIN, bool POUT, int EXTRA>
    void colfft(PlanData& p, const CX* in, CX* out, int cols, int KX, long blk_in, long s_in, long blk_out,
                long s_out, long fs_in, long fs_out, int nf, const int* status, const ColExtra& ex, int nextra) {
        const int nbx = (cols + C - 1) / C;
        k_colfft<T, N, DIR, PIN, POUT, EXTRA><<<(unsigned)(nbx * nf + nextra), NT, 0, p.stream>>>(
            in, out, cols, KX, blk_in, s_in, blk_out, s_out, fs_in, fs_out, tw(p), status, nbx, nf, ex);
    }
    void y_full(PlanData& p, const CX* in, CX* out, int nf, int dir) {
        const int cols = N * NKX;
        if (dir < 0)
            colfft<-1, false, false, 0>(p, in, out, cols, NKX, N * NKX, NKX, N * NKX, NKX, FULL, FULL, nf, nullptr, {}, 0);
        else
            colfft<+1, false, false, 0>(p, in, out, cols, NKX, N * NKX, NKX, N * NKX, NKX, FULL, FULL, nf, nullptr, {}, 0);
    }
    void z_full(PlanData& p, const CX* in, CX* out, int nf, int dir) {
        const int cols = N * NKX;
        if (dir < 0)
            colfft<-1, false, false, 0>(p, in, out, cols, cols, 0, cols, 0, cols, FULL, FULL, nf, nullptr, {}, 0);
        else
            colfft<+1, false, false, 0>(p, in, out, cols, cols, 0, cols, 0, cols, FULL, FULL, nf, nullptr, {}, 0);
    }
    void x_r2c(PlanData& p, const T* in, CX* out, long nrows, int nkx, int pitch) {
        constexpr int RR = 2 * RW;
        k_x_r2c<T, N><<<(unsigned)((nrows + RR - 1) / RR), NT, 0, p.stream>>>(in, out, nrows, nkx, pitch, tw(p));
    }
    void x_c2r(PlanData& p, const CX* in, T* out, long nrows, int nkx) {
        constexpr int RR = 2 * RW;
        k_x_c2r<T, N><<<(unsigned)((nrows + RR - 1) / RR), NT, 0, p.stream>>>(in, out, nrows, nkx,
                                                                              T(1.0 / (double)N3), tw(p));
    }

    int fft_r2c(PlanData& p, const void* in, void* out, int nf) override {
        CX* o = static_cast<CX*>(out);
        x_r2c(p, static_cast<const T*>(in), o, (long)nf * N2, NKX, NKX);
        y_full(p, o, o, nf, -1);
        z_full(p, o, o, nf, -1);
        return launch_check("fft_r2c");
    }
    // inverse of nf full-layout fields held in `spec` (destroyed) into out
    void c2r_inplace(PlanData& p, CX* spec, T* out, int nf) {
        z_full(p, spec, spec, nf, +1);
        y_full(p, spec, spec, nf, +1);
        x_c2r(p, spec, out, (long)nf * N2, NKX);
    }
    int fft_c2r(PlanData& p, const void* in, void* out, int nf) override {
        int rc = ensure_scratch(&p.spec, &p.spec_sz, (size_t)nf * FULL * sizeof(CX), p);
        if (rc) return rc;
        CX* s = static_cast<CX*>(p.spec);
        z_full(p, static_cast<const CX*>(in), s, nf, +1);
        y_full(p, s, s, nf, +1);
        x_c2r(p, s, static_cast<T*>(out), (long)nf * N2, NKX);
        return launch_check("fft_c2r");
    }

    int mask(PlanData& p, const flusi_insect& ins, double t, void* chi, void* us, int16_t* col) override {
        const double dx = p.L / N;
        k_kin<<<1, 64, 0, p.stream>>>(p.kin, ins, t, dx);
        k_mask<T><<<(unsigned)((N3 + 255) / 256), 256, 0, p.stream>>>(p.kin, N, dx, static_cast<T*>(chi),
                                                                       static_cast<T*>(us), col);
        return launch_check("mask_insect");
    }

    int rhs(PlanData& p, const void* uhat, const void* chi, const void* us, void* rhs_hat, int mean_mode,
            double* umax_host) override {
        int rc = ensure_scratch(&p.spec, &p.spec_sz, 6ul * FULL * sizeof(CX), p);
        if (rc) return rc;
        rc = ensure_scratch(&p.phys, &p.phys_sz, 6ul * N3 * sizeof(T), p);
        if (rc) return rc;
        const double ks = 2.0 * M_PI / p.L;
        CX* s = static_cast<CX*>(p.spec);
        T* ph = static_cast<T*>(p.phys);
        k_curl_full<T><<<(unsigned)((FULL + 255) / 256), 256, 0, p.stream>>>(static_cast<const CX*>(uhat), s, N, ks);
        c2r_inplace(p, s, ph, 6);
        const int nb = (int)((N3 + NT - 1) / NT);
        if (nb > p.npmax) {
            if (p.pmax) (void)hipFree(p.pmax);
            p.pmax = nullptr;
            if (hipMalloc(&p.pmax, nb * sizeof(double)) != hipSuccess) return set_error(FLUSI_ENOMEM, "rhs scratch");
            p.npmax = nb;
        }
        k_source_full<T><<<nb, NT, 0, p.stream>>>(ph, static_cast<const T*>(chi), static_cast<const T*>(us), N3,
                                                  1.0 / p.eta, p.pmax);
        CX* o = static_cast<CX*>(rhs_hat);
        x_r2c(p, ph, o, 3 * N2, NKX, NKX);
        y_full(p, o, o, 3, -1);
        z_full(p, o, o, 3, -1);
        k_project_full<T><<<(unsigned)((FULL + 255) / 256), 256, 0, p.stream>>>(o, N, ks, mean_mode);
        rc = launch_check("rhs");
        if (rc) return rc;
        if (umax_host) {
            double* h = new double[nb];
            hipError_t e = hipMemcpyAsync(h, p.pmax, nb * sizeof(double), hipMemcpyDeviceToHost, p.stream);
            if (e == hipSuccess) e = hipStreamSynchronize(p.stream);
            if (e != hipSuccess) {
                delete[] h;
                return set_error(FLUSI_EDEVICE, "rhs: %s", hipGetErrorString(e));
            }
            double m = 0.0;
            for (int i = 0; i < nb; ++i) m = h[i] > m || h[i] != h[i] ? h[i] : m;
            delete[] h;
            *umax_host = sqrt(m);
        }
        return FLUSI_OK;
    }

    // --- pruned stepping schedule ------------------------------------------------
    // y-inverse of the 6 z-partial fields; with kin set, one extra workgroup
    // evaluates the kinematics of time level `par`
    void y_inverse(PlanData& p, const int* status, const ColExtra* kin) {
        const int cols = N * KP;
        const CX* a = static_cast<const CX*>(p.bufA);
        CX* b = static_cast<CX*>(p.bufB);
        if (kin)
            colfft<+1, true, false, 2>(p, a, b, cols, KP, Qp, KP, (long)N * KPp, KPp, (long)N * Qp, N2 * KPp, 6, status,
                                       *kin, 1);
        else
            colfft<+1, true, false, 0>(p, a, b, cols, KP, Qp, KP, (long)N * KPp, KPp, (long)N * Qp, N2 * KPp, 6, status,
                                       {}, 0);
    }
    // y-forward of nf fields; with red set, NRED_BLOCKS extra workgroups do the
    // first-level reduction of the x-pass partial sums
    void y_forward(PlanData& p, const int* status, int nf, const ColExtra* red) {
        const int cols = N * KP;
        const CX* a = static_cast<const CX*>(p.bufA);
        CX* b = static_cast<CX*>(p.bufB);
        if (red)
            colfft<-1, false, true, 1>(p, a, b, cols, KP, (long)N * KPp, KPp, Qp, KP, N2 * KPp, (long)N * Qp, nf, status,
                                       *red, NRED_BLOCKS);
        else
            colfft<-1, false, true, 0>(p, a, b, cols, KP, (long)N * KPp, KPp, Qp, KP, N2 * KPp, (long)N * Qp, nf, status,
                                       {}, 0);
    }
    template <int MODE>
    void zpass(PlanData& p, void* st, int mean_mode, int par = 0, const StepCtl* ctl = nullptr,
               double* history = nullptr) {
        const unsigned nb = (Q + CZ - 1) / CZ;
        StepCtl c{};
        if (ctl) c = *ctl;
        k_zpass<T, N, MODE><<<nb, NTZ, 0, p.stream>>>(static_cast<const CX*>(p.bufB), (long)N * Qp, st_uhat(st),
                                                      st_nold(st), st_fs(), static_cast<CX*>(p.bufA), (long)N * Qp,
                                                      tw(p), static_cast<StateHdr*>(st), 2.0 * M_PI / p.L, p.nu,
                                                      mean_mode, p.partial2, par, c, p.L / N, p.eta, history);
    }

    int state_init(PlanData& p, void* st, const void* u0, double t0) override {
        k_hdr_init<<<1, 64, 0, p.stream>>>(static_cast<StateHdr*>(st), t0);
        x_r2c(p, static_cast<const T*>(u0), static_cast<CX*>(p.bufA), 3 * N2, KP, KPp);
        y_forward(p, nullptr, 3, nullptr);
        zpass<MODE_IMPORT>(p, st, FLUSI_MEAN_FREE);
        return launch_check("state_init");
    }

    int export_uhat(PlanData& p, const void* st, void* out) override {
        k_export_full<T><<<(unsigned)((FULL + 255) / 256), 256, 0, p.stream>>>(
            st_uhat(const_cast<void*>(st)), static_cast<CX*>(out), N, st_fs(), (long)Qp);
        return launch_check("export_uhat");
    }

    int velocity(PlanData& p, const void* st, void* u) override {
        int rc = ensure_scratch(&p.spec, &p.spec_sz, 3ul * FULL * sizeof(CX), p);
        if (rc) return rc;
        rc = export_uhat(p, st, p.spec);
        if (rc) return rc;
        c2r_inplace(p, static_cast<CX*>(p.spec), static_cast<T*>(u), 3);
        return launch_check("state_velocity");
    }

    int step(PlanData& p, void* st, const flusi_insect* ins, const flusi_step_params& sp) override {
        StateHdr* hdr = static_cast<StateHdr*>(st);
        const int* status = &hdr->status;
        flusi_insect in{};
        const bool masked = ins && (ins->body != FLUSI_BODY_NONE || ins->wings);
        if (masked) in = *ins;
        const int nc = masked ? (in.wings ? 3 : 1) : 0;
        const double dx = p.L / N;
        const bool dyn = masked && (in.wings || in.psi_dot != 0.0 || in.beta_dot != 0.0 || in.gamma_dot != 0.0);
        StepCtl ctl{sp.dt_fixed, sp.cfl, sp.dt_max, sp.eta_cap, sp.t_end, masked ? 1 : 0, sp.mean_mode, dyn ? 1 : 0, 0};
        k_prologue<<<1, 64, 0, p.stream>>>(hdr, in, p.ins_dev, dx, masked ? 1 : 0);
        {
            PassScope ps(p, PASS_ZINV);
            zpass<MODE_INVERSE>(p, st, sp.mean_mode);
        }
        const unsigned nwg = (unsigned)nwg_x();
        ColExtra red{p.partial, p.partial2, (int)nwg, 0, hdr, p.ins_dev, dx};
        for (int s = 0; s < sp.nsteps; ++s) {
            const int par = s & 1;
            {
                PassScope ps(p, PASS_YINV);
                ColExtra kin{nullptr, nullptr, 0, par, hdr, p.ins_dev, dx};
                y_inverse(p, status, dyn ? &kin : nullptr);
            }
            {
                PassScope ps(p, PASS_X);
                const CX* yin = static_cast<const CX*>(p.bufB);
                CX* xo = static_cast<CX*>(p.bufA);
                if (nc == 0)
                    k_xpass<T, N, 0><<<nwg, NT, 0, p.stream>>>(yin, xo, N2 * KPp, N2 * KPp, tw(p), hdr, dx, 1.0 / p.eta, p.partial);
                else if (nc == 1)
                    k_xpass<T, N, 1><<<nwg, NT, 0, p.stream>>>(yin, xo, N2 * KPp, N2 * KPp, tw(p), hdr, dx, 1.0 / p.eta, p.partial);
                else
                    k_xpass<T, N, 3><<<nwg, NT, 0, p.stream>>>(yin, xo, N2 * KPp, N2 * KPp, tw(p), hdr, dx, 1.0 / p.eta, p.partial);
            }
            {
                PassScope ps(p, PASS_YFWD);
                y_forward(p, status, 3, &red);
            }
            double* hist = sp.history ? sp.history + (long)s * FLUSI_NDIAG : nullptr;
            {
                PassScope ps(p, PASS_Z);
                if (s + 1 < sp.nsteps && !split_z()) zpass<MODE_STEP>(p, st, sp.mean_mode, par, &ctl, hist);
                else zpass<MODE_STEP_LAST>(p, st, sp.mean_mode, par, &ctl, hist);
            }
            if (s + 1 < sp.nsteps && split_z()) {
                PassScope ps(p, PASS_ZINV);
                zpass<MODE_INVERSE>(p, st, sp.mean_mode);
            }
        }
        return launch_check("step");
    }
};

}  // namespace flusi
