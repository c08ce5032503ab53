// Host-side launch logic of one (real type, grid size) instantiation.
#pragma once
#include <cstddef>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>

#include "kernels.hpp"

namespace flusi {

struct ImplBase;

// Schedule of the stepping passes: tile variant (0 .. NVARIANT-1) of each pass and
// whether the z-pass runs as one launch or as update + inverse launches.
struct Sched {
    int y_inverse = 0, x_pass = 0, y_forward = 0, z_pass = 0;
    int split_z = 0;
};

constexpr size_t RTAB_BYTES64 = (FLUSI_RTABLE + 1) * sizeof(double);
constexpr size_t RTAB_BYTES32 = (FLUSI_RTABLE + 1) * sizeof(float);

// Plan contents shared with the launchers.
struct PlanData {
    int n = 0, nx = 0, dtype = 0;  // n points on y and z, nx on x
    double L = 0, Lx = 0, nu = 0, eta = 0;  // box side on y and z, on x (one spacing L/n)
    int K = 0, KP = 0, M = 0, Q = 0;  // K: largest kept |j| on y, z; KP: kept kx
    hipStream_t stream = nullptr;
    void* tw = nullptr;   // n twiddles exp(-2 pi i m/n) of the plan's real type (y and z)
    void* twx = nullptr;  // nx twiddles of the x axis (the same table when nx = n)
    void* bufA = nullptr;
    void* bufB = nullptr;
    size_t szA = 0, szB = 0;
    double* partial = nullptr;
    int nwg_x = 0;
    double* partial2 = nullptr;
    Kin* kin = nullptr;
    flusi_insect* ins_dev = nullptr;  // device copy of the insect of the current stepping call
    int integrator = FLUSI_INT_AB2;   // FLUSI_INT_*
    hipStream_t side = nullptr;       // kinematics side stream of the plan's own calls
    hipEvent_t ev_z = nullptr, ev_k = nullptr;
    void* ustage = nullptr;           // RK4 stage velocity (3 state fields), allocated when RK4 is chosen
    size_t ustage_sz = 0;
    double* rtab = nullptr;           // Fourier wing radius table (FLUSI_RTABLE + 1 samples) ...
    float* rtab32 = nullptr;          // ... and its FP32 copy
    WingCoef rtab_key{};              // coefficients the table holds
    bool rtab_valid = false;
    Member* member_dev = nullptr;     // launch record of the plan's own calls
    Sched sched;                      // schedule of the plan's own stepping calls
    unsigned long gen = 0;            // bumped by every option change (ensembles rebuild on a change)
    void* noalloc_scratch = nullptr;  // device address of the static scratch array on the plan's GPU
    double wall_th[3] = {0.0, 0.0, 0.0};  // Dirichlet layer thickness per axis (0: none)
    double u_wall[3] = {0.0, 0.0, 0.0};   // velocity imposed in the layers
    double c_sp = 0.0;                // vorticity sponge constant (0: off)
    double sp_thick[3] = {0.0, 0.0, 0.0};  // sponge layer thickness per axis
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

// Brackets one launch on stream st with a pair of events when profiling is on
// (records kept in the plan).
struct PassScope {
    PlanData* pp;
    int pass;
    hipStream_t st;
    size_t idx = 0;
    PassScope(PlanData* pd, int ps, hipStream_t s) : pp(pd && pd->prof ? pd : nullptr), pass(ps), st(s) {
        if (!pp) return;
        PlanData& p = *pp;
        while (p.events.size() < p.ev_used + 2) {
            hipEvent_t e;
            if (hipEventCreate(&e) != hipSuccess) {
                p.prof = false;
                pp = nullptr;
                return;
            }
            p.events.push_back(e);
        }
        idx = p.ev_used;
        p.ev_used += 2;
        (void)hipEventRecord(p.events[idx], st);
    }
    ~PassScope() {
        if (!pp) return;
        (void)hipEventRecord(pp->events[idx + 1], st);
        pp->prof_recs.emplace_back(pass, idx);
    }
};

// One batched stepping launch sequence: members of one (real type, size) that
// advance together.  The device table is ordered by sponge flag, then colour
// count (nc = 0, then 1, then 3), so that each x-pass variant runs over a
// contiguous range.
struct GroupRun {
    const Member* mt = nullptr;
    int nmem = 0;
    int n_nc[2][3] = {{0, 0, 0}, {0, 0, 0}};  // members [without, with sponge][nc = 0, 1, 3]
    bool any_dyn = false;
    bool any_ff = false;      // some member is in free flight
    bool rk = false;          // RK4 integrator (single-plan runs)
    // side stream for the kinematics kernel of the RK4 stages (null: they run
    // on `stream`): forked after the z-pass, joined before the x-pass, so they
    // overlap the y-inverse, which does not read them (the AB2 steps evaluate
    // the kinematics inside the y-inverse launch instead)
    hipStream_t side = nullptr;
    hipEvent_t ev_z = nullptr, ev_k = nullptr;
    const void* tw = nullptr;   // y and z twiddles
    const void* twx = nullptr;  // x twiddles
    Sched sched;
    hipStream_t stream = nullptr;
    PlanData* prof = nullptr; // pass timing events, or null
};

inline int colour_count(const flusi_insect* ins) {
    const bool masked = ins && (ins->body != FLUSI_BODY_NONE || ins->wings);
    return masked ? (ins->wings ? 3 : 1) : 0;
}
inline int colour_slot(int nc) { return nc == 0 ? 0 : (nc == 1 ? 1 : 2); }
inline bool sponge_on(const PlanData& p) {
    return p.c_sp > 0.0 && (p.sp_thick[0] > 0.0 || p.sp_thick[1] > 0.0 || p.sp_thick[2] > 0.0);
}
inline int free_flight_on(const flusi_insect* ins) { return colour_count(ins) > 0 && ins->free_flight ? 1 : 0; }
inline int kin_dynamic(const flusi_insect* ins) {
    return colour_count(ins) > 0 && (ins->wings || ins->free_flight || ins->psi_dot != 0.0 ||
                                     ins->beta_dot != 0.0 || ins->gamma_dot != 0.0);
}

// Launch record of (plan, state) for a stepping call with parameters sp.
inline Member make_member(const PlanData& p, void* st, const flusi_insect* ins, const flusi_step_params& sp) {
    Member m{};
    const int nc = colour_count(ins);
    m.hdr = static_cast<StateHdr*>(st);
    m.bufA = p.bufA;
    m.bufB = p.bufB;
    m.partial = p.partial;
    m.partial2 = p.partial2;
    m.ins = p.ins_dev;
    m.rtab = p.rtab;
    m.rtab32 = p.rtab32;
    m.history = sp.history;
    m.dx = p.L / p.n;
    m.ks = 2.0 * M_PI / p.L;
    m.ksx = p.nx == p.n ? m.ks : 2.0 * M_PI / p.Lx;
    m.nu = p.nu;
    m.eta = p.eta;
    m.inv_eta = 1.0 / p.eta;
    const bool walls = p.wall_th[0] > 0.0 || p.wall_th[1] > 0.0 || p.wall_th[2] > 0.0;
    m.ctl = StepCtl{sp.dt_fixed, sp.cfl, sp.dt_max, sp.eta_cap, sp.t_end, (nc > 0 || walls) ? 1 : 0, sp.mean_mode,
                    kin_dynamic(ins), nc > 0 ? 1 : 0};
    m.wall = walls ? 1 : 0;
    for (int a = 0; a < 3; ++a) {
        m.wall_lo[a] = p.wall_th[a] > 0.0 ? (a == 0 ? p.Lx : p.L) - p.wall_th[a] : 1e300;
        m.u_wall[a] = p.u_wall[a];
    }
    m.mean_mode = sp.mean_mode;
    m.nc = nc;
    m.dyn = kin_dynamic(ins);
    m.sponge = sponge_on(p) ? 1 : 0;
    m.ff = free_flight_on(ins);
    m.rk = p.integrator == FLUSI_INT_RK4 ? 1 : 0;
    m.ustage = p.ustage;
    if (m.rk && p.nu > 0.0 && p.K > 0) {
        // explicit diffusion: dt * nu * max|k|^2 <= 2.5 (RK4 is stable to about 2.785)
        const double kx = (p.KP - 1) * m.ksx, ky = p.K * m.ks;
        m.ctl.visc_cap = 2.5 / (p.nu * (kx * kx + ky * ky + ky * ky));
    }
    m.inv_csp = m.sponge ? 1.0 / p.c_sp : 0.0;
    for (int a = 0; a < 3; ++a)
        m.sp_lo[a] = (m.sponge && p.sp_thick[a] > 0.0) ? (a == 0 ? p.Lx : p.L) - p.sp_thick[a] : 1e300;
    return m;
}
enum { PASS_ZINV = 0, PASS_YINV = 1, PASS_X = 2, PASS_KIN = 3, PASS_YFWD = 4, PASS_Z = 5 };

int set_error(int code, const char* fmt, ...);
int ensure_scratch(void** ptr, size_t* cur, size_t need, PlanData& p);

// Checks the free-flight parameters of a body description (Sec. 3.6);
// FLUSI_OK or FLUSI_EINVAL with a message.
inline int check_insect(const flusi_insect* ins) {
    if (!ins) return FLUSI_OK;
    if (ins->kin_type < FLUSI_KIN_SINE || ins->kin_type > FLUSI_KIN_HERMITE)
        return set_error(FLUSI_EINVAL, "insect: kin_type must be FLUSI_KIN_SINE, _FOURIER or _HERMITE");
    if (ins->kin_type == FLUSI_KIN_FOURIER && (ins->kin_n < 0 || ins->kin_n > FLUSI_KIN_MAX))
        return set_error(FLUSI_EINVAL, "insect: Fourier kinematics need 0 <= kin_n <= %d", FLUSI_KIN_MAX);
    if (ins->kin_type == FLUSI_KIN_HERMITE && (ins->kin_n < 2 || ins->kin_n > FLUSI_KIN_MAX || !(ins->freq > 0.0)))
        return set_error(FLUSI_EINVAL, "insect: Hermite kinematics need 2 <= kin_n <= %d and freq > 0", FLUSI_KIN_MAX);
    if (ins->wing_shape != FLUSI_WING_ELLIPSE && ins->wing_shape != FLUSI_WING_FOURIER &&
        ins->wing_shape != FLUSI_WING_RECT)
        return set_error(FLUSI_EINVAL, "insect: wing_shape must be FLUSI_WING_ELLIPSE, _FOURIER or _RECT");
    if (ins->wing_shape == FLUSI_WING_RECT && !(ins->wing_rect[3] > 0.0 && ins->wing_rect[1] > ins->wing_rect[0]))
        return set_error(FLUSI_EINVAL, "insect: rectangular wing needs B > 0 and tip > a");
    if (ins->wing_shape == FLUSI_WING_FOURIER && (ins->wing_n < 0 || ins->wing_n > FLUSI_WING_MAX))
        return set_error(FLUSI_EINVAL, "insect: Fourier wing needs 0 <= wing_n <= %d", FLUSI_WING_MAX);
    if (!(ins->head_r >= 0.0) || !(ins->eye_r >= 0.0) || !std::isfinite(ins->head_r) || !std::isfinite(ins->eye_r))
        return set_error(FLUSI_EINVAL, "insect: head_r and eye_r must be finite and >= 0");
    for (int i = 0; i < 6; ++i)
        if (!std::isfinite(ins->wing_J[i])) return set_error(FLUSI_EINVAL, "insect: wing_J not finite");
    if (!ins->free_flight) return FLUSI_OK;
    if (ins->free_flight != 1) return set_error(FLUSI_EINVAL, "insect: free_flight must be 0 or 1");
    if (colour_count(ins) == 0) return set_error(FLUSI_EINVAL, "insect: free flight needs a body or wings");
    if (!(ins->mass > 0.0) || !std::isfinite(ins->mass)) return set_error(FLUSI_EINVAL, "insect: free flight needs mass > 0");
    for (int i = 0; i < 3; ++i)
        if (!(ins->inertia[i] > 0.0) || !std::isfinite(ins->inertia[i]))
            return set_error(FLUSI_EINVAL, "insect: free flight needs inertia > 0");
    if (!std::isfinite(ins->gravity)) return set_error(FLUSI_EINVAL, "insect: gravity not finite");
    for (int i = 0; i < 6; ++i)
        if (ins->dof[i] != 0.0 && ins->dof[i] != 1.0) return set_error(FLUSI_EINVAL, "insect: dof entries must be 0 or 1");
    return FLUSI_OK;
}



struct ImplBase {
    virtual ~ImplBase() {}
    virtual size_t bufA_elems() const = 0;
    virtual size_t bufA_elems_sponge() const = 0;
    virtual size_t bufB_elems() const = 0;
    virtual int nwg_x() const = 0;
    virtual size_t state_bytes() const = 0;
    virtual size_t field3_bytes() const = 0;  // three state fields (the RK4 stage velocity)
    virtual int fft_r2c(PlanData&, const void*, void*, int) = 0;
    virtual int fft_c2r(PlanData&, const void*, void*, int) = 0;
    virtual int fft_c2r_into(PlanData&, const void*, void*, int, void* scratch) = 0;
    virtual size_t spec_bytes() const = 0;  // one full-layout spectrum field
    virtual int mask(PlanData&, const flusi_insect&, double, void*, void*, int16_t*) = 0;
    virtual int rhs(PlanData&, const void*, const void*, const void*, void*, int, double*) = 0;
    virtual int state_init(PlanData&, void*, const void*, double) = 0;
    virtual int export_uhat(PlanData&, const void*, void*) = 0;
    virtual int velocity(PlanData&, const void*, void*) = 0;
    virtual int step(PlanData&, void*, const flusi_insect*, const flusi_step_params&) = 0;
    virtual int run_steps(const GroupRun&, int nsteps) = 0;
    virtual Sched default_sched() const = 0;
};

inline int launch_check(const char* what) {
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return set_error(FLUSI_EDEVICE, "%s: %s", what, hipGetErrorString(e));
    return FLUSI_OK;
}

// Radius table of a Fourier wing: rebuilt on the stream (graph-capturable, no
// allocation) when the coefficients differ from those it holds.
inline int prepare_wing_table(PlanData& p, const flusi_insect* ins, hipStream_t stream) {
    if (!ins || !ins->wings || ins->wing_shape != FLUSI_WING_FOURIER) return FLUSI_OK;
    WingCoef c{};
    c.n = ins->wing_n;
    for (int i = 0; i <= ins->wing_n; ++i) {
        c.a[i] = ins->wing_coef[0][i];
        c.b[i] = ins->wing_coef[1][i];
    }
    if (p.rtab_valid && std::memcmp(&c, &p.rtab_key, sizeof(c)) == 0) return FLUSI_OK;
    k_rtab_build<<<(unsigned)((FLUSI_RTABLE + 1 + 255) / 256), 256, 0, stream>>>(c, p.rtab, p.rtab32);
    p.rtab_key = c;
    p.rtab_valid = true;
    return launch_check("wing radius table");
}

// Stepping and utilities of an NX x N x N grid (x, y, z).
template <typename T, int NX, int N>
struct Impl final : ImplBase {
    using CX = cx<T>;
    using G = Geo<T, NX, N>;
    static constexpr int K = G::K, KP = G::KP, M = G::M, Q = G::Q;
    static constexpr int KPp = G::KPp, Qp = G::Qp;
    static constexpr int C = cols_of(N), RW = rows_x(NX, sizeof(cx<T>)), NKX = NX / 2 + 1;
    static constexpr int CZ = cols_z(N);
    static constexpr long N2 = (long)N * N, N3 = (long)NX * N * N;  // rows along x, points
    static constexpr long FULL = N2 * NKX;  // full-layout spectrum per field

    size_t bufA_elems() const override {
        const size_t a = 6ul * N * Qp, b = 3ul * N2 * KPp;
        return a > b ? a : b;
    }
    // the x-pass writes 6 fields (N and chi_sp w) with the sponge
    size_t bufA_elems_sponge() const override {
        const size_t a = bufA_elems(), b = 6ul * N2 * KPp;
        return a > b ? a : b;
    }
    size_t bufB_elems() const override {
        const size_t a = 6ul * N2 * KPp, b = 3ul * N * Qp;
        return a > b ? a : b;
    }
    // x-pass workgroups per member, largest over the tile variants (sizes the
    // partial-sum buffer)
    int nwg_x() const override { return (int)(N2 / rows_x(NX, sizeof(cx<T>), NVARIANT - 1)); }
    static size_t field_bytes() { return (size_t)M * Qp * sizeof(CX); }
    size_t state_bytes() const override { return STATE_HDR_BYTES + 6 * ((field_bytes() + 255) / 256 * 256); }

    static CX* st_uhat(void* st) { return reinterpret_cast<CX*>(static_cast<char*>(st) + STATE_HDR_BYTES); }
    static long st_fs() { return (long)((field_bytes() + 255) / 256 * 256 / sizeof(CX)); }
    size_t field3_bytes() const override { return 3 * ((field_bytes() + 255) / 256 * 256); }
    static CX* st_nold(void* st) { return st_uhat(st) + 3 * st_fs(); }

    const CX* tw(const PlanData& p) const { return static_cast<const CX*>(p.tw); }
    const CX* twx(const PlanData& p) const { return static_cast<const CX*>(p.twx); }
    // The z-pass runs as two launches (forward + update, then curl + inverse)
    // when one fused launch would hold too many registers per thread.
    static constexpr bool split_z() { return N >= 192; }

    // --- full-layout column passes ------------------------------------------------
    // column transforms of nf fields, 1D grid of nbx*nf workgroups
    template <int DIR, bool PIN, bool POUT>
    void colfft(PlanData& p, const CX* in, CX* out, int cols, int KX, long blk_in, long s_in, long blk_out,
                long s_out, long fs_in, long fs_out, int nf) {
        const int nbx = (cols + C - 1) / C;
        k_colfft<T, N, DIR, PIN, POUT><<<(unsigned)(nbx * nf), NT, 0, p.stream>>>(
            in, out, cols, KX, blk_in, s_in, blk_out, s_out, fs_in, fs_out, tw(p), nbx);
    }
    void y_full(PlanData& p, const CX* in, CX* out, int nf, int dir) {
        const int cols = N * NKX;
        if (dir < 0)
            colfft<-1, false, false>(p, in, out, cols, NKX, N * NKX, NKX, N * NKX, NKX, FULL, FULL, nf);
        else
            colfft<+1, false, false>(p, in, out, cols, NKX, N * NKX, NKX, N * NKX, NKX, FULL, FULL, nf);
    }
    void z_full(PlanData& p, const CX* in, CX* out, int nf, int dir) {
        const int cols = N * NKX;
        if (dir < 0)
            colfft<-1, false, false>(p, in, out, cols, cols, 0, cols, 0, cols, FULL, FULL, nf);
        else
            colfft<+1, false, false>(p, in, out, cols, cols, 0, cols, 0, cols, FULL, FULL, nf);
    }
    void x_r2c(PlanData& p, const T* in, CX* out, long nrows, int nkx, int pitch) {
        constexpr int RR = 2 * RW;
        k_x_r2c<T, NX><<<(unsigned)((nrows + RR - 1) / RR), NT, 0, p.stream>>>(in, out, nrows, nkx, pitch, twx(p));
    }
    void x_c2r(PlanData& p, const CX* in, T* out, long nrows, int nkx) {
        constexpr int RR = 2 * RW;
        k_x_c2r<T, NX><<<(unsigned)((nrows + RR - 1) / RR), NT, 0, p.stream>>>(in, out, nrows, nkx,
                                                                               T(1.0 / (double)N3), twx(p));
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
        return fft_c2r_into(p, in, out, nf, p.spec);
    }
    // inverse through caller-provided scratch of nf full-layout spectra (every
    // element is written by the z pass before any later pass reads it)
    int fft_c2r_into(PlanData& p, const void* in, void* out, int nf, void* scratch) override {
        CX* s = static_cast<CX*>(scratch);
        z_full(p, static_cast<const CX*>(in), s, nf, +1);
        y_full(p, s, s, nf, +1);
        x_c2r(p, s, static_cast<T*>(out), (long)nf * N2, NKX);
        return launch_check("fft_c2r");
    }
    size_t spec_bytes() const override { return (size_t)FULL * sizeof(CX); }

    int mask(PlanData& p, const flusi_insect& ins, double t, void* chi, void* us, int16_t* col) override {
        const double dx = p.L / N;
        if (int rc = prepare_wing_table(p, &ins, p.stream)) return rc;
        k_kin<<<1, 64, 0, p.stream>>>(p.kin, ins, t, dx, p.rtab, p.rtab32);
        k_mask<T><<<(unsigned)((N3 + 255) / 256), 256, 0, p.stream>>>(p.kin, NX, N, dx, static_cast<T*>(chi),
                                                                       static_cast<T*>(us), col);
        return launch_check("mask_insect");
    }

    int rhs(PlanData& p, const void* uhat, const void* chi, const void* us, void* rhs_hat, int mean_mode,
            double* umax_host) override {
        if (NX != N) return set_error(FLUSI_EUNSUPPORTED, "rhs: the unfused path takes cubic grids only");
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

    // --- pruned stepping schedule over a member table ------------------------------
    template <int V>
    static constexpr int nby(int nf) { return (N * KP + cols_of(N, V) - 1) / cols_of(N, V) * nf; }
    template <int V>
    static constexpr int nwg(int) { return (int)(N2 / rows_x(NX, sizeof(cx<T>), V)); }
    static constexpr int NBZ = (Q + CZ - 1) / CZ;  // z-pass tiles per member
    static int nwg_of(int v) { return v == 2 ? nwg<2>(0) : (v == 1 ? nwg<1>(0) : nwg<0>(0)); }

    // y-inverse of the 6 z-partial fields
    // kin_par >= 0: the launch also evaluates the kinematics of time level
    // kin_par (one extra workgroup per member, at the start of the grid)
    template <int V>
    static void y_inverse_v(const GroupRun& g, int kin_par) {
        const CX* w = static_cast<const CX*>(g.tw);
        constexpr int nb = nby<V>(6);
        if (kin_par >= 0)
            k_ypass<T, NX, N, +1, 2, V><<<(unsigned)((nb + 1) * g.nmem), NT, 0, g.stream>>>(g.mt, nb, w, 6, kin_par);
        else
            k_ypass<T, NX, N, +1, 0, V><<<(unsigned)(nb * g.nmem), NT, 0, g.stream>>>(g.mt, nb, w, 6, 0);
    }
    static void y_inverse(const GroupRun& g, int kin_par = -1) {
        if (g.sched.y_inverse == 2) y_inverse_v<2>(g, kin_par);
        else if (g.sched.y_inverse == 1) y_inverse_v<1>(g, kin_par);
        else y_inverse_v<0>(g, kin_par);
    }
    // y-forward of 3 fields; with red set, nred_of(NX, N) extra workgroups per member
    // do the first-level reduction of the x-pass sums
    template <int V>
    static void y_forward_v(const GroupRun& g, bool red) {
        const CX* w = static_cast<const CX*>(g.tw);
        const int nfwd = (g.n_nc[1][0] + g.n_nc[1][1] + g.n_nc[1][2]) ? 6 : 3;
        const int nb = nby<V>(nfwd);
        if (red)
            k_ypass<T, NX, N, -1, 1, V><<<(unsigned)((nb + nred_of(NX, N)) * g.nmem), NT, 0, g.stream>>>(
                g.mt, nb + nred_of(NX, N), w, nfwd, nwg_of(g.sched.x_pass));
        else
            k_ypass<T, NX, N, -1, 0, V><<<(unsigned)(nb * g.nmem), NT, 0, g.stream>>>(g.mt, nb, w, nfwd, 0);
    }
    static void y_forward(const GroupRun& g, bool red) {
        if (g.sched.y_forward == 2) y_forward_v<2>(g, red);
        else if (g.sched.y_forward == 1) y_forward_v<1>(g, red);
        else y_forward_v<0>(g, red);
    }
    template <int V, bool SP>
    static const Member* xpass_range(const GroupRun& g, const Member* mt) {
        const CX* w = static_cast<const CX*>(g.twx);
        constexpr int nw = nwg<V>(0);
        const int* n = g.n_nc[SP ? 1 : 0];
        if (n[0]) k_xpass<T, NX, N, 0, V, SP><<<(unsigned)(nw * n[0]), xpass_threads<T, NX, V, SP>(), 0, g.stream>>>(mt, w);
        mt += n[0];
        if (n[1]) k_xpass<T, NX, N, 1, V, SP><<<(unsigned)(nw * n[1]), xpass_threads<T, NX, V, SP>(), 0, g.stream>>>(mt, w);
        mt += n[1];
        if (n[2]) k_xpass<T, NX, N, 3, V, SP><<<(unsigned)(nw * n[2]), xpass_threads<T, NX, V, SP>(), 0, g.stream>>>(mt, w);
        return mt + n[2];
    }
    template <int V>
    static void xpass_v(const GroupRun& g) {
        const Member* mt = xpass_range<V, false>(g, g.mt);
        xpass_range<V, true>(g, mt);
    }
    static void xpass(const GroupRun& g) {
        if (g.sched.x_pass == 2) xpass_v<2>(g);
        else if (g.sched.x_pass == 1) xpass_v<1>(g);
        else xpass_v<0>(g);
    }
    template <int MODE, int V, bool SP>
    static void zpass_launch(const GroupRun& g, const Member* mt, int nmem, int par, int s, int rk) {
        // modes with the reduction: one more workgroup per member (diagnostics, next level)
        constexpr int nb = NBZ + ((MODE == MODE_STEP || MODE == MODE_STEP_LAST || MODE == MODE_RK1) ? 1 : 0);
        if (nmem > 0)
            k_zpass<T, NX, N, MODE, V, SP><<<(unsigned)(nb * nmem), nt_z(N, V), 0, g.stream>>>(
                mt, static_cast<const CX*>(g.tw), par, s, rk);
    }
    // update modes: members without the sponge, then those with it (the table
    // is ordered that way); other modes: all members in one launch
    template <int MODE, int V>
    static void zpass_v(const GroupRun& g, int par, int s, int rk) {
        constexpr bool update = MODE == MODE_STEP || MODE == MODE_STEP_LAST || MODE == MODE_RK1 || MODE == MODE_RKS;
        const int nsp = g.n_nc[1][0] + g.n_nc[1][1] + g.n_nc[1][2];
        if (update && nsp) {
            zpass_launch<MODE, V, false>(g, g.mt, g.nmem - nsp, par, s, rk);
            zpass_launch<MODE, V, update>(g, g.mt + (g.nmem - nsp), nsp, par, s, rk);
        } else {
            zpass_launch<MODE, V, false>(g, g.mt, g.nmem, par, s, rk);
        }
    }
    template <int MODE>
    static void zpass(const GroupRun& g, int par = 0, int s = 0, int rk = 0) {
        if (g.sched.z_pass == 2) zpass_v<MODE, 2>(g, par, s, rk);
        else if (g.sched.z_pass == 1) zpass_v<MODE, 1>(g, par, s, rk);
        else zpass_v<MODE, 0>(g, par, s, rk);
    }

    Sched default_sched() const override {
        Sched d;
        d.split_z = split_z() ? 1 : 0;
        return d;
    }

    // Launches the kinematics kernel of a time level (c < 0) or of an RK4 stage
    // time (c >= 0); on the side stream when the group has one.  Returns
    // whether the caller must join the side stream before the x-pass.
    static bool kin_launch(const GroupRun& g, int par, double c, hipError_t& err) {
        const unsigned nbk = (unsigned)g.nmem;
        hipStream_t st = g.stream;
        if (g.side) {
            if (err == hipSuccess) err = hipEventRecord(g.ev_z, g.stream);
            if (err == hipSuccess) err = hipStreamWaitEvent(g.side, g.ev_z, 0);
            st = g.side;
        }
        {
            PassScope ps(g.prof, PASS_KIN, st);
            if (c < 0.0) k_kin_level<T><<<nbk, NT_KIN, 0, st>>>(g.mt, g.nmem, par);
            else k_kin_stage<T><<<nbk, NT_KIN, 0, st>>>(g.mt, g.nmem, par, c);
        }
        if (g.side && err == hipSuccess) err = hipEventRecord(g.ev_k, g.side);
        return g.side != nullptr;
    }
    static void kin_join(const GroupRun& g, bool pending, hipError_t& err) {
        if (pending && err == hipSuccess) err = hipStreamWaitEvent(g.stream, g.ev_k, 0);
    }

    // RK4 (Sec. 2.4): four pipeline passes per step.  The first stage reduces
    // the x-pass sums, picks dt and writes the diagnostics and the next time
    // level; the others use that dt, the kinematics of their own time and no
    // reduction.  The z-pass is always the fused form here.
    int run_steps_rk(const GroupRun& g, int nsteps) {
        {
            PassScope ps(g.prof, PASS_KIN, g.stream);
            k_prologue<T><<<(unsigned)g.nmem, NT_KIN, 0, g.stream>>>(g.mt, g.nmem);
        }
        {
            PassScope ps(g.prof, PASS_ZINV, g.stream);
            zpass<MODE_INVERSE>(g);
        }
        hipError_t err = hipSuccess;
        for (int s = 0; s < nsteps; ++s) {
            const int par = s & 1;
            for (int stage = 1; stage <= 4; ++stage) {
                bool pend = false;
                if (g.any_dyn && (stage > 1 || s > 0))
                    pend = kin_launch(g, par, stage == 1 ? -1.0 : (stage == 4 ? 1.0 : 0.5), err);
                {
                    PassScope ps(g.prof, PASS_YINV, g.stream);
                    y_inverse(g);
                }
                kin_join(g, pend, err);
                {
                    PassScope ps(g.prof, PASS_X, g.stream);
                    xpass(g);
                }
                {
                    PassScope ps(g.prof, PASS_YFWD, g.stream);
                    y_forward(g, stage == 1);
                }
                {
                    PassScope ps(g.prof, PASS_Z, g.stream);
                    const int inv = (stage < 4 || s + 1 < nsteps) ? 16 : 0;
                    if (stage == 1) zpass<MODE_RK1>(g, par, s, inv);
                    else zpass<MODE_RKS>(g, par, s, stage | inv);
                }
            }
        }
        if (err != hipSuccess) return set_error(FLUSI_EDEVICE, "step: %s", hipGetErrorString(err));
        return launch_check("step");
    }

    int run_steps(const GroupRun& g, int nsteps) override {
        if (g.nmem <= 0 || nsteps <= 0) return FLUSI_OK;
        if (g.rk) return run_steps_rk(g, nsteps);
        {
            PassScope ps(g.prof, PASS_KIN, g.stream);
            k_prologue<T><<<(unsigned)g.nmem, NT_KIN, 0, g.stream>>>(g.mt, g.nmem);
        }
        {
            PassScope ps(g.prof, PASS_ZINV, g.stream);
            zpass<MODE_INVERSE>(g);
        }
        hipError_t err = hipSuccess;
        for (int s = 0; s < nsteps; ++s) {
            const int par = s & 1;
            // kinematics of this time level (the prologue covers the first),
            // evaluated by extra workgroups of the y-inverse
            {
                PassScope ps(g.prof, PASS_YINV, g.stream);
                y_inverse(g, (g.any_dyn && s > 0) ? par : -1);
            }
            {
                PassScope ps(g.prof, PASS_X, g.stream);
                xpass(g);
            }
            {
                PassScope ps(g.prof, PASS_YFWD, g.stream);
                y_forward(g, true);
            }
            {
                PassScope ps(g.prof, PASS_Z, g.stream);
                if (s + 1 < nsteps && !g.sched.split_z) zpass<MODE_STEP>(g, par, s);
                else zpass<MODE_STEP_LAST>(g, par, s);
            }
            if (s + 1 < nsteps && g.sched.split_z) {
                PassScope ps(g.prof, PASS_ZINV, g.stream);
                zpass<MODE_INVERSE>(g);
            }
        }
        // free flight: advance the body to the new current level
        if (g.any_ff) {
            PassScope ps(g.prof, PASS_KIN, g.stream);
            k_kin_level<T><<<(unsigned)g.nmem, NT_KIN, 0, g.stream>>>(g.mt, g.nmem, nsteps & 1);
        }
        if (err != hipSuccess) return set_error(FLUSI_EDEVICE, "step: %s", hipGetErrorString(err));
        return launch_check("step");
    }

    int state_init(PlanData& p, void* st, const void* u0, double t0) override {
        flusi_step_params sp{};
        sp.mean_mode = FLUSI_MEAN_FREE;
        const Member m = make_member(p, st, nullptr, sp);
        k_member_set<<<1, 64, 0, p.stream>>>(p.member_dev, m, flusi_insect{});
        k_hdr_init<<<1, 64, 0, p.stream>>>(static_cast<StateHdr*>(st), t0);
        x_r2c(p, static_cast<const T*>(u0), static_cast<CX*>(p.bufA), 3 * N2, KP, KPp);
        GroupRun g;
        g.mt = p.member_dev;
        g.nmem = 1;
        g.tw = p.tw;
        g.twx = p.twx;
        g.stream = p.stream;
        y_forward(g, false);
        zpass<MODE_IMPORT>(g);
        return launch_check("state_init");
    }

    int export_uhat(PlanData& p, const void* st, void* out) override {
        k_export_full<T><<<(unsigned)((FULL + 255) / 256), 256, 0, p.stream>>>(
            st_uhat(const_cast<void*>(st)), static_cast<CX*>(out), NX, N, st_fs(), (long)Qp);
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
        const Member m = make_member(p, st, ins, sp);
        k_member_set<<<1, 64, 0, p.stream>>>(p.member_dev, m, m.nc > 0 ? *ins : flusi_insect{});
        if (m.nc > 0)
            if (int rc = prepare_wing_table(p, ins, p.stream)) return rc;
        GroupRun g;
        g.mt = p.member_dev;
        g.nmem = 1;
        g.n_nc[m.sponge][colour_slot(m.nc)] = 1;
        g.any_dyn = m.dyn != 0;
        g.any_ff = m.ff != 0;
        g.rk = m.rk != 0;
        g.tw = p.tw;
        g.twx = p.twx;
        g.sched = p.sched;
        g.stream = p.stream;
        // RK4 stage kinematics on the side stream: the fork/join costs a few
        // microseconds of event latency, worth it only where the y-inverse it
        // overlaps is long
        if (N >= 192) {
            g.side = p.side;
            g.ev_z = p.ev_z;
            g.ev_k = p.ev_k;
        }
        g.prof = &p;
        return run_steps(g, sp.nsteps);
    }
};

}  // namespace flusi
