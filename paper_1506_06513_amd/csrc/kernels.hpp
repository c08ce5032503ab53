// HIP kernels of the pseudo-spectral penalized Navier-Stokes step (gfx950).
//
// Stepping schedule, four HBM passes per time step over 2/3-pruned spectra
// of an nx x n x n grid (K = (n-1)/3 is the largest kept |j| on y and z,
// KX = (nx-1)/3 on x; KP = KX+1 kept kx; M = 2K+1 kept ky,kz):
//   y-inverse   : z-partials [6][z][ky'][kx]  -> y-partials [6][z][y][kx]
//   x-pass      : y-partials -> c2r along x -> u, w -> mask/u_s on the fly ->
//                 N = u x w - (chi/C_eta)(u - u_s), FP64 partial sums ->
//                 r2c along x -> [3][z][y][kx]
//   scalar      : FP64 reduction -> dt, force, torque, energy, AB2 weights,
//                 time advance, kinematics of the next time level
//   y-forward   : [3][z][y][kx] -> [3][z][ky'][kx]
//   z-pass      : forward z -> projection -> IF-AB2 -> state; curl ->
//                 inverse z of u and w -> z-partials of the next step
// Reference: Sec. 2.1 (eq. PNST_org_momentum, force_with_unst_corrections,
// moment_of_love), Sec. 2.4 (Fourier discretization, 2/3 rule, AB2 with
// integrating factor), Algorithm 1.
#pragma once
#include <type_traits>

#include "common.hpp"
#include "fft.hpp"
#include "insect.hpp"

namespace flusi {

constexpr int NT = 256;   // threads per workgroup of the y passes and the x-pass
constexpr int NV = 39;    // reduction values per workgroup (see xpass)
constexpr int NRED_MAX = 64;  // most first-level reduction workgroups per member

// Tile shapes.  Each stepping pass has NVARIANT shapes that compute the same
// values (V = 0 the default); a schedule picks one per pass (see the
// autotuner).
constexpr int NVARIANT = 3;
// Columns per workgroup of the y passes: C*N ~ 4096 elements in LDS (V = 0),
// a half (V = 1) or a quarter (V = 2) of that.
__host__ __device__ constexpr int cols_of(int N, int V = 0) {
    int c = 4096 / N, p = 8;
    while (p * 2 <= c) p *= 2;
    return p >> V;
}
// Columns and threads per workgroup of the z-pass (more, narrower workgroups:
// the z-pass has only (2K+1)(K+1) columns).  V = 1 and 2 use more threads per
// column (fewer rows per thread): the smallest multiple of the V = 0 count
// among {2, 3} (V = 1) or {4, 6} (V = 2) whose rows per sweep divide the
// column, at most 1024 threads; otherwise the previous variant's count.
__host__ __device__ constexpr int cols_z(int N) { return N <= 24 ? 16 : 8; }
__host__ __device__ constexpr int nt_z(int N, int V = 0) {
    const int t0 = N <= 192 ? 128 : 256;
    const int C = cols_z(N);
    const auto fits = [&](int t) { return t <= 1024 && N % (t / C) == 0; };
    const int t1 = fits(2 * t0) ? 2 * t0 : 3 * t0;
    if (V == 0) return t0;
    if (V == 1) return t1;
    return fits(4 * t0) ? 4 * t0 : (fits(6 * t0) ? 6 * t0 : t1);
}
// Rows per workgroup of the x-pass: 3*RW*N ~ 3072 elements in LDS (V = 0), a
// half (V = 1) or a quarter (V = 2) of that, at least 2 rows (an even count
// pairs the rows' N_z in one forward transform); a single row where two rows
// of complex values (nine columns) would not fit the LDS (long FP64 rows),
// and as the smaller variants of rows of 1024 points or more, whose two-row
// tile leaves room for one workgroup per CU only.
__host__ __device__ constexpr int rows_x(int N, int cbytes = 8, int V = 0) {
    int c = 1024 / N, p = 2;
    while (p * 2 <= c) p *= 2;
    p >>= V;
    if (p < 2) p = (V > 0 && N >= 1024) ? 1 : 2;
    if (p == 2 && 9 * cm_stride(N) * cbytes > 150 * 1024) p = 1;
    return p;
}
__host__ __device__ constexpr int round_up(int a, int b) { return (a + b - 1) / b * b; }
// First-level reduction workgroups per member: every z-pass workgroup reads
// their NV-value records, so small grids use few; large grids (many x-pass
// records) use more so that the first level stays shorter than the y-forward.
__host__ __device__ constexpr int nred_of(int NX, int N) {
    const int n = N * N / rows_x(NX) / 128;
    return n < 16 ? 16 : (n > NRED_MAX ? NRED_MAX : n);
}

// Pruned-spectrum geometry of an NX x N x N grid (x, y, z): K is the largest
// kept |j| on y and z, KX on x; KP = KX + 1 kept kx.  Row pitches are padded to
// 128 bytes so that every row of a pass starts on a cache line.
template <typename T, int NX, int N>
struct Geo {
    static constexpr int K = kmax_of(N), KX = kmax_of(NX), KP = KX + 1, M = 2 * K + 1, Q = M * KP;
    static constexpr int AL = 128 / (int)sizeof(cx<T>);
    static constexpr int KPp = round_up(KP, AL);  // pitch of [z][y][kx] rows
    static constexpr int Qp = round_up(Q, AL);    // pitch of [z][ky'][kx] planes
};

// Workgroups are dispatched round-robin over the 8 XCDs (each with its own
// L2).  Remap so that consecutive logical tiles, which share cache lines, run
// on the same XCD.
__device__ __forceinline__ int xcd_tile(int bid, int nb) {
    const int x = bid & 7, s = bid >> 3;
    const int per = nb >> 3, rem = nb & 7;
    return x < rem ? x * (per + 1) + s : rem * (per + 1) + (x - rem) * per + s;
}

// Twiddle table of a workgroup's FFTs staged in LDS (every butterfly stage
// reads it; LDS latency instead of cache latency).  Visible after the barrier
// that opens the first column transform.
template <typename T, int N>
__device__ __forceinline__ void stage_twiddles(cx<T>* tws, const cx<T>* __restrict__ tw, int nthreads) {
    for (int e = threadIdx.x; e < N; e += nthreads) tws[e] = tw[e];
}

struct Solid13 {
    double v[13];
};

struct StepCtl {
    double dt_fixed, cfl, dt_max, eta_cap, t_end;
    int masked, mean_mode, kin_dynamic, body;  // body: a body or wings (kinematics exist)
    double visc_cap;  // RK4: adaptive dt <= visc_cap (explicit diffusion); 0: none
};

// Per-time-level scalars of a state.
struct Slot {
    double t;        // time of the coefficients
    double dt_prev;  // previous step size
    long long n;     // steps taken
    int have_prev;   // previous right-hand side stored
    int have_I;      // previous solid-momentum integral stored
    double I_prev[3][6];
    double J_prev[3];  // moment of the solid momentum about the body centre (with have_I)
    // Free flight (Sec. 3.6).  ff_state: 0 none; 1 ff is the state at t;
    // 2 ff is the state of the previous level and still has to be advanced
    // by ff_w[0]*f(ff; ff_F, ff_m) + ff_w[1]*ff_f (done before the level's
    // kinematics are evaluated).
    int ff_state;
    int ff_have_prev;  // ff_f holds the right-hand side of the previous step
    double ff[13];     // x_cntr, u_cntr, eps, Omega^(b)
    double ff_f[13];
    double ff_F[3], ff_m[3];  // total force and torque about x_cntr (global frame)
    double ff_w[2];           // dt*b1, dt*b2
    double rk_dt;             // RK4: step size of the step that produced this level (0: no step)
    double rk_pad[3];
};

// Device-resident per-state scalars (first 4 KiB of a state buffer).  The time
// level is double-buffered: during a step every workgroup reads slot[p] and a
// single thread writes the next level into slot[1-p], so readers and the
// writer never touch the same bytes.  `cur` names the current slot between
// steps.
struct StateHdr {
    int status;      // 0, FLUSI_ENONFINITE or FLUSI_EINVAL
    int cur;
    int pad[2];
    Slot slot[2];
    double diag[FLUSI_NDIAG];
    Kin kin;         // kinematics at the current time level
    KinT<float> kf;  // the same, prepared for the FP32 mask evaluation
    KinT<double> kd; // ... and for the FP64 one
};
static_assert(sizeof(StateHdr) <= 4096, "state header too large");
constexpr size_t STATE_HDR_BYTES = 4096;

// Launch record of one simulation (device memory).  The stepping kernels take
// a table of these and work on every member of the table in one launch: the
// 1D grid holds `per` workgroups per member, member = tile / per.  A single
// plan is a table of one.
struct Member {
    StateHdr* hdr;              // state: header, then the fields (pruned layout)
    void* bufA;                 // z-partials (inverse) / x-pass output
    void* bufB;                 // y-partials (inverse) / y-forward output
    double* partial;            // NV sums per x-pass workgroup
    double* partial2;           // NV sums per first-level reduction workgroup
    const flusi_insect* ins;    // device copy of the body description
    const double* rtab;         // Fourier wing radius table of the plan (or null)
    const float* rtab32;
    double* history;            // FLUSI_NDIAG values per step of a call, or null
    double dx, ks, ksx, nu, eta, inv_eta;  // ks = 2 pi / L on y and z, ksx on x
    StepCtl ctl;
    int mean_mode;
    int nc;                     // colours of the mask: 0 (none), 1 (body), 3 (body + wings)
    int dyn;                    // kinematics change with time
    int sponge;                 // vorticity sponge on: 3 more forward fields (chi_sp w)
    int ff;                     // free flight: the body pose is integrated
    int rk;                     // RK4 integrator (stage velocity in ustage)
    void* ustage;               // RK4 stage velocity [3] (state field layout)
    double inv_csp;             // 1/C_sp
    double sp_lo[3];            // chi_sp = 1 where x_a >= sp_lo[a] for some axis a
    int wall, pad_w;            // Dirichlet layers on
    double wall_lo[3];          // layer where x_a >= wall_lo[a] for some axis a ...
    double u_wall[3];           // ... with the velocity u_wall imposed
};

template <int NRED>
__device__ inline void reduce_level1(const double* __restrict__ partial, int nwg, double* __restrict__ partial2,
                                     int b, double (*red)[NV]);

// ---------------------------------------------------------------------------
// Column FFT along y or z of one tile of C columns.
// Column q (q < Q) of a field starts at (q / KX) * blk + q % KX; element e of
// the column sits at stride s.  PIN: the input holds only the 2K+1 kept
// signed modes (pruned storage); POUT: only those are written.
// ---------------------------------------------------------------------------
template <typename T, int N, int DIR, bool PIN, bool POUT, int C>
__device__ __forceinline__ void colfft_tile(const glb<cx<T>>* __restrict__ in, glb<cx<T>>* __restrict__ out, int Q, int KX,
                                            long blk_in, long s_in, long blk_out, long s_out, int tile,
                                            const cx<T>* __restrict__ tw, cx<T>* buf) {
    constexpr int K = kmax_of(N);
    constexpr int SC = cm_stride(N);
    constexpr int RS = NT / C;      // rows handled per sweep
    constexpr int RPT = N / RS;     // rows per thread
    static_assert(NT % C == 0 && N % RS == 0, "column mapping");
    const int tid = threadIdx.x;
    const int c = tid % C, r0 = tid / C;
    const int q = tile * C + c;
    const bool ok = q < Q;
    const long bin = ok ? (long)(q / KX) * blk_in + q % KX : 0;
    const long bout = ok ? (long)(q / KX) * blk_out + q % KX : 0;
    cx<T> v[RPT];
#pragma unroll
    for (int i = 0; i < RPT; ++i) {
        const int n = r0 + i * RS;
        v[i] = cx<T>{T(0), T(0)};
        if (ok) {
            if constexpr (PIN) {
                const int m = m_of_bin(n, N, K);
                if (m >= 0) v[i] = gld(in, bin + m * s_in);
            } else {
                v[i] = gld(in, bin + n * s_in);
            }
        }
    }
#pragma unroll
    for (int i = 0; i < RPT; ++i) buf[c * SC + cpad(r0 + i * RS)] = v[i];
    fft_cols<T, N, DIR, C, NT, SC>(buf, tw);
    if (ok) {
        constexpr int NOUT = POUT ? 2 * K + 1 : N;
#pragma unroll
        for (int i = 0; i < (NOUT + RS - 1) / RS; ++i) {
            const int o = r0 + i * RS;
            if (o < NOUT) {
                const int n = POUT ? bin_of_m(o, N, K) : o;
                gst(out, bout + o * s_out, buf[c * SC + cpad(n)]);
            }
        }
    }
}

// Column transforms of nf fields given by pointers (full-layout utilities):
// 1D grid of nbx * nf workgroups.
template <typename T, int N, int DIR, bool PIN, bool POUT>
__global__ __launch_bounds__(NT) void k_colfft(const cx<T>* in, cx<T>* out, int Q, int KX, long blk_in, long s_in,
                                               long blk_out, long s_out, long fs_in, long fs_out,
                                               const cx<T>* __restrict__ tw, int nbx) {
    __shared__ cx<T> buf[cols_of(N) * cm_stride(N)];
    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    const int f = tile / nbx;
    colfft_tile<T, N, DIR, PIN, POUT, cols_of(N)>(gview(in) + f * fs_in, gview(out) + f * fs_out, Q, KX, blk_in, s_in, blk_out, s_out,
                                      tile % nbx, tw, buf);
}

// Kinematics of member m and the mask-evaluation blocks its passes read, by one
// workgroup (one wave or more).  The threads stage the body description in
// LDS (one round trip instead of a chain of dependent loads) and evaluate the
// sines and cosines in parallel, in two rounds: the angle series and fixed
// angles, then the wing angles that the series give.  From those values one
// thread assembles the body part of the kinematics in LDS and two lanes the
// two wings (kin_body, kin_wing); the FP64 and FP32 blocks are then converted,
// their arrays on all lanes of a wave, by two waves at once where the
// workgroup has them, and only the ones the plan's passes read (FP32: the
// FP32 block, and the FP64 one for the part decision where parts overlap;
// FP64: the FP64 block); all threads store.
// Time: slot p's time (at == false), or t_at (RK4 stages; no free flight).
// In free flight the body pose is the free-flight state of the level: taken
// from the tethered kinematics on the first free-flight step, or advanced by
// the AB2 step that the previous step's diagnostics left pending (Alg. 1 step
// (f); the quaternion is renormalized).
struct KinShared {
    flusi_insect in;
    Kin k;
    KinT<float> kf;
    KinT<double> kd;
    double arg[KIN_TRIG_MAX];
    SinCos val[KIN_TRIG_MAX];
    unsigned char dep[KIN_TRIG_MAX];
    double y[13], f[13];
    double rall[3];  // cull radii of the body parts and of each wing (kin_body, kin_wing)
    double t;
    int n, st;
};
static_assert(sizeof(flusi_insect) % 8 == 0 && sizeof(Kin) % 8 == 0 && sizeof(KinT<float>) % 8 == 0 &&
                  sizeof(KinT<double>) % 8 == 0 && offsetof(StateHdr, kin) % 8 == 0 &&
                  offsetof(StateHdr, kf) % 8 == 0 && offsetof(StateHdr, kd) % 8 == 0,
              "kinematics blocks are copied in 8-byte words");

// nbytes (a multiple of 8; both ends 8-byte aligned) copied by the workgroup.
__device__ __forceinline__ void wg_copy8(void* dst, const void* src, int nbytes) {
    auto* d = static_cast<unsigned long long*>(dst);
    const auto* q = static_cast<const unsigned long long*>(src);
    for (int i = threadIdx.x; i < nbytes / 8; i += blockDim.x) d[i] = q[i];
}

template <typename T>
__device__ __forceinline__ void kin_update(const Member& m, int p, bool at, double t_at, KinShared& s) {
    const int tid = threadIdx.x, nth = blockDim.x;
    StateHdr* h = m.hdr;
    Slot& sl = h->slot[p];
    // the level's time is loaded alongside the description
    const double t_lvl = at ? t_at : sl.t;
    wg_copy8(&s.in, m.ins, (int)sizeof(flusi_insect));
    __syncthreads();
    const flusi_insect& in = s.in;
    if (tid == 0) {
        int st = 0;
        if (!at && in.free_flight) {
            st = sl.ff_state;
            if (st != 0) {
                for (int i = 0; i < 13; ++i) s.y[i] = sl.ff[i];
                if (st == 2) {
                    double F[3], mm[3], fp[13];
                    for (int i = 0; i < 3; ++i) {
                        F[i] = sl.ff_F[i];
                        mm[i] = sl.ff_m[i];
                    }
                    const double w0 = sl.ff_w[0], w1 = sl.ff_w[1];
                    const int hp = sl.ff_have_prev;
                    for (int i = 0; i < 13; ++i) fp[i] = sl.ff_f[i];
                    solid_rhs(in, s.y, F, mm, s.f);
                    for (int i = 0; i < 13; ++i) s.y[i] += hp ? w0 * s.f[i] + w1 * fp[i] : w0 * s.f[i];
                    const double q = 1.0 / sqrt(s.y[6] * s.y[6] + s.y[7] * s.y[7] + s.y[8] * s.y[8] + s.y[9] * s.y[9]);
                    for (int i = 6; i < 10; ++i) s.y[i] *= q;
                }
            }
        }
        s.t = t_lvl;
        s.st = st;
        s.n = kin_trig_args(in, s.t, st != 0, 0, nullptr, s.arg, s.dep);
    }
    __syncthreads();
    const int n = s.n;
    for (int j = tid; j < n; j += nth)
        if (!s.dep[j]) s.val[j] = sin_cos(s.arg[j]);
    __syncthreads();
    if (in.wings) {
        if (tid == 0) {
            double ang[3], rate[3];
            wing_angle_values(in, s.t, ang, rate, TrigTable{s.arg, s.val, n, s.st != 0 ? 0 : 6});
            kin_trig_args(in, s.t, s.st != 0, 1, ang, s.arg, s.dep);
        }
        __syncthreads();
        for (int j = tid; j < n; j += nth)
            if (s.dep[j]) s.val[j] = sin_cos(s.arg[j]);
        __syncthreads();
    }
    // assembled in LDS: the block never occupies registers
    Kin& k = s.k;
    const int st = s.st;
    if (tid == 0) {
        const double rb = kin_body(in, s.t, m.dx, k, st != 0 ? s.y : nullptr, TrigTable{s.arg, s.val, n, 0});
        s.rall[0] = rb;
        if (!in.wings) {
            kin_nowings(k);
            k.r2all = rb * rb;
        }
        k.rtab = m.rtab;
        k.rtab32 = m.rtab32;
    }
    __syncthreads();
    if (in.wings) {
        // the two wings on lanes 0 and 1 (one instruction stream for both);
        // each reads its sines and cosines at its own place in the table
        if (tid < 2) {
            TrigTable tt{s.arg, s.val, n, st != 0 ? 0 : 6};
            double ang[3], rate[3], acc[3];
            wing_angle_values(in, s.t, ang, rate, tt, acc);
            if (tid == 1) tt.i += 4;  // past the left wing's four
            s.rall[1 + tid] = kin_wing(in, k, tid, ang, rate, acc, wings_inert(in), tt);
        }
        __syncthreads();
        if (tid == 0) {
            const double r = fmax(fmax(s.rall[0], s.rall[1]), s.rall[2]);
            k.r2all = r * r;
        }
    }
    if (tid == 0 && in.free_flight && !at) {
        if (st == 0) {
            for (int i = 0; i < 3; ++i) {
                s.y[i] = k.xc[i];
                s.y[3 + i] = k.uc[i];
                s.y[10 + i] = k.omb[i];
            }
            for (int i = 0; i < 4; ++i) s.y[6 + i] = k.eps[i];
        }
        if (st != 1)
            for (int i = 0; i < 13; ++i) sl.ff[i] = s.y[i];
        if (st == 2)
            for (int i = 0; i < 13; ++i) sl.ff_f[i] = s.f[i];
        if (st == 0) sl.ff_have_prev = 0;
        if (st == 2) sl.ff_have_prev = 1;
        sl.ff_state = 1;
    }
    __syncthreads();
    // the blocks' arrays on all lanes of a wave, the rest on its first lane;
    // FP64 on the first wave and FP32 on the second where there is one
    constexpr bool F64 = sizeof(T) == 8;
    const bool need_kd = F64 || m.nc > 1, need_kf = !F64;
    const int wv = tid >> 6, ln = tid & 63, wkf = nth > 64 ? 1 : 0;
    if (need_kd && wv == 0) {
        kin_cast_arrays<double>(k, s.kd, ln, 64);
        if (ln == 0) kin_cast_rest<double>(k, s.kd);
    }
    if (need_kf && wv == wkf) {
        kin_cast_arrays<float>(k, s.kf, ln, 64);
        if (ln == 0) kin_cast_rest<float>(k, s.kf);
    }
    __syncthreads();
    wg_copy8(&h->kin, &s.k, (int)sizeof(Kin));
    if (need_kf) wg_copy8(&h->kf, &s.kf, (int)sizeof(KinT<float>));
    if (need_kd) wg_copy8(&h->kd, &s.kd, (int)sizeof(KinT<double>));
}

// y passes of the stepping schedule over a member table.
//   DIR = +1 (y-inverse): 6 z-partial fields bufA [f][z][ky'][kx] (pitch Qp per
//            z) -> bufB [f][z][y][kx] (pitch KPp per y)
//   DIR = -1 (y-forward): 3 fields bufA [f][z][y][kx] -> bufB [f][z][ky'][kx]
// Each member has nbx*nf column tiles followed by the extra workgroups:
//   EXTRA 1: nred_of(NX, N) workgroups reduce the x-pass sums (first level)
// nwg: x-pass workgroups per member (records of the first-level reduction).
// EXTRA 2 (y-inverse): the grid starts with one workgroup per member that
// evaluates the member's kinematics of time level nwg (members whose
// kinematics change with time), beside the column tiles: the y-inverse does
// not read them, the x-pass after it does.  That path is held to the
// register budget of four waves per SIMD, which the column tiles' LDS allows
// at most anyway for the larger tiles.
// nfwd: forward fields per member (3, or 6 when a member of the launch has the
// vorticity sponge; members without it skip fields 3..5).
template <typename T, int NX, int N, int DIR, int EXTRA, int V>
__global__ __launch_bounds__(NT, EXTRA == 2 ? 4 : 1) void k_ypass(const Member* __restrict__ mt, int per,
                                                                  const cx<T>* __restrict__ tw, int nfwd, int nwg) {
    using G = Geo<T, NX, N>;
    constexpr int KP = G::KP, KPp = G::KPp, Qp = G::Qp;
    constexpr int C = cols_of(N, V);
    constexpr int nbx = (N * KP + C - 1) / C;
    constexpr size_t BUF = sizeof(cx<T>) * C * cm_stride(N);
    constexpr size_t LDS = EXTRA == 2 && sizeof(KinShared) > BUF ? sizeof(KinShared) : BUF;
    const int nf = DIR > 0 ? 6 : nfwd;
    __shared__ __align__(16) unsigned char lds[LDS];
    cx<T>* buf = reinterpret_cast<cx<T>*>(lds);
    int bid = blockIdx.x, nb = gridDim.x;
    if constexpr (EXTRA == 2) {
        const int nmem = nb / (per + 1);
        if (bid < nmem) {
            const Member& m = mt[bid];
            if (m.dyn && !*gview(&m.hdr->status))
                kin_update<T>(m, nwg, false, 0.0, *reinterpret_cast<KinShared*>(lds));
            return;
        }
        bid -= nmem;
        nb -= nmem;
    }
    const int lin = xcd_tile(bid, nb);
    const Member& m = mt[lin / per];
    const int tile = lin % per;
    if (*gview(&m.hdr->status)) return;
    const int f = tile / nbx;
    if (f >= nf) {
        if constexpr (EXTRA == 1) {
            __shared__ double red[NT / 64][NV];
            if (tile - nf * nbx < nred_of(NX, N))
                reduce_level1<nred_of(NX, N)>(m.partial, nwg, m.partial2, tile - nf * nbx, red);
        }
        return;
    }
    if (DIR < 0 && f >= 3 && !m.sponge) return;
    __shared__ cx<T> tws[N];
    stage_twiddles<T, N>(tws, tw, NT);
    const glb<cx<T>>* A = gview(static_cast<const cx<T>*>(m.bufA));
    glb<cx<T>>* B = gview(static_cast<cx<T>*>(m.bufB));
    if constexpr (DIR > 0)
        colfft_tile<T, N, +1, true, false, C>(A + f * (long)N * Qp, B + f * (long)N * N * KPp, N * KP, KP, Qp, KP,
                                           (long)N * KPp, KPp, tile % nbx, tws, buf);
    else
        colfft_tile<T, N, -1, false, true, C>(A + f * (long)N * N * KPp, B + f * (long)N * Qp, N * KP, KP,
                                           (long)N * KPp, KPp, Qp, KP, tile % nbx, tws, buf);
}

// ---------------------------------------------------------------------------
// Deterministic workgroup reductions
// ---------------------------------------------------------------------------
// Wave-wide FP64 reductions with DPP lane moves (no LDS traffic).  The result
// is complete in lane 63; lanes whose DPP source is out of range add 0, which
// is the identity for the sums and for the maxima of non-negative values used
// here.  The combination order is fixed, so results are deterministic.
template <int CTRL, int ROWM, int BANKM>
__device__ __forceinline__ double dpp_move(double v) {
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, ROWM, BANKM, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, ROWM, BANKM, false);
    return __hiloint2double(hi, lo);
}
template <bool MAX>
__device__ __forceinline__ double wave_reduce63(double v) {
    auto op = [](double a, double b) { return MAX ? fmax(a, b) : a + b; };
    v = op(v, dpp_move<0xb1, 0xf, 0xf>(v));   // quad_perm [1,0,3,2]
    v = op(v, dpp_move<0x4e, 0xf, 0xf>(v));   // quad_perm [2,3,0,1]
    v = op(v, dpp_move<0x114, 0xf, 0xe>(v));  // row_shr:4
    v = op(v, dpp_move<0x118, 0xf, 0xc>(v));  // row_shr:8
    v = op(v, dpp_move<0x142, 0xa, 0xf>(v));  // row_bcast:15
    v = op(v, dpp_move<0x143, 0xc, 0xf>(v));  // row_bcast:31
    return v;
}
__device__ __forceinline__ double wave_sum(double v) {
    v = wave_reduce63<false>(v);
    return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), 63),
                            __builtin_amdgcn_readlane(__double2loint(v), 63));
}

// Wave sums of twelve FP64 values per lane at once, in a fixed order.  The
// values are halved over lanes twice with the gfx950 half-wave and row swaps
// (lanes 0-31 go on with values 0-5 summed over lanes l and l + 32, lanes 32-63
// with values 6-11; then row r of 16 lanes with values 3r .. 3r + 2), and the
// three left in each row are summed within the row by DPP.  Lane 16r + 15
// returns the totals of values 3r, 3r + 1, 3r + 2 in s[0..2].  About a quarter
// of the instructions of twelve separate wave sums.
__device__ __forceinline__ double swap_add32(double x, double y) {
    const auto lo = __builtin_amdgcn_permlane32_swap((unsigned)__double2loint(x), (unsigned)__double2loint(y), false, false);
    const auto hi = __builtin_amdgcn_permlane32_swap((unsigned)__double2hiint(x), (unsigned)__double2hiint(y), false, false);
    // first: x on lanes 0-31, y's lanes 0-31 on 32-63; second: x's lanes 32-63
    // on 0-31, y on 32-63
    return __hiloint2double((int)hi[0], (int)lo[0]) + __hiloint2double((int)hi[1], (int)lo[1]);
}
__device__ __forceinline__ double swap_add16(double x, double y) {
    const auto lo = __builtin_amdgcn_permlane16_swap((unsigned)__double2loint(x), (unsigned)__double2loint(y), false, false);
    const auto hi = __builtin_amdgcn_permlane16_swap((unsigned)__double2hiint(x), (unsigned)__double2hiint(y), false, false);
    // first: rows 0 and 2 of x, rows 0 and 2 of y in rows 1 and 3; second:
    // rows 1 and 3 of x in rows 0 and 2, rows 1 and 3 of y
    return __hiloint2double((int)hi[0], (int)lo[0]) + __hiloint2double((int)hi[1], (int)lo[1]);
}
__device__ __forceinline__ void wave_sum12(const double (&v)[12], double (&s)[3]) {
    double a[6];
#pragma unroll
    for (int j = 0; j < 6; ++j) a[j] = swap_add32(v[j], v[j + 6]);
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        double b = swap_add16(a[j], a[j + 3]);
        b += dpp_move<0xb1, 0xf, 0xf>(b);   // quad_perm [1,0,3,2]
        b += dpp_move<0x4e, 0xf, 0xf>(b);   // quad_perm [2,3,0,1]
        b += dpp_move<0x114, 0xf, 0xe>(b);  // row_shr:4
        b += dpp_move<0x118, 0xf, 0xc>(b);  // row_shr:8
        s[j] = b;
    }
}
__device__ __forceinline__ double wave_max(double v) {
    v = wave_reduce63<true>(v);
    return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), 63),
                            __builtin_amdgcn_readlane(__double2loint(v), 63));
}

// Reduce NV per-thread values (value 0 and 2 by max, the rest by sum) over the
// workgroup; the result lands in out[0..NV) (global) from thread v.
template <int NVAL>
__device__ __forceinline__ void block_reduce_store(const double (&acc)[NVAL], double (*red)[NV], double* out) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int v = 0; v < NVAL; ++v) {
        double r = 0.0;
        if (__any(acc[v] != 0.0)) r = (v == 0 || v == 2) ? wave_max(acc[v]) : wave_sum(acc[v]);
        if (lane == 0) red[wv][v] = r;
    }
    __syncthreads();
    const int t = threadIdx.x;
    if (t < NV) {
        double r = 0.0;
        if (t < NVAL) {
            r = red[0][t];
            for (int w = 1; w < NT / 64; ++w) r = (t == 0 || t == 2) ? fmax(r, red[w][t]) : r + red[w][t];
        }
        gview(out)[t] = r;
    }
}

// ---------------------------------------------------------------------------
// x-pass: inverse x, pointwise source with the mask, FP64 partial sums,
// forward x.  Reduction values per workgroup:
//   [0] max |u|^2, [1] sum |u|^2 (non-finite values propagate into it), [2] 0,
//   [3 + 12 c + 0..2]  sum chi (u - u_s)            (colour c+1)
//   [3 + 12 c + 3..5]  sum (x - x_ref) x chi (u - u_s)
//   [3 + 12 c + 6..8]  sum chi u_s
//   [3 + 12 c + 9..11] sum (x - x_ref) x chi u_s
// NC: number of colours accumulated (0 no mask, 1 single body, 3 insect).
// ---------------------------------------------------------------------------
// Member table: N*N/RW workgroups per member, y-partials in bufB, output in bufA.
// SP: members with the vorticity sponge; chi_sp * w is transformed beside N
// and stored as fields 3..5.
// Workgroups per CU the x-pass asks the compiler to fit (registers), where
// its LDS allows: the FP32 full-size tile without the sponge (its twiddles are
// then read from the table in memory, and the three-colour tile also drops the
// column pad, keeping the tile under 40 KiB); not at nx = 512, where the
// 128-register budget spills.
template <typename T, int NX, int NC, int V, bool SP>
__host__ __device__ constexpr int xpass_min_blocks() {
    return (sizeof(T) < 8 && V == 0 && !SP && NX < 512) ? 4 : 1;
}
// Column stride of the x-pass tile: the FFT layout's (cm_stride), without its
// one-element pad for the three-colour tile at 4 workgroups per CU (the pad
// spreads the column starts over the LDS banks; without it 256^3 and 128^3
// measured no slower, and the tile fits in 40 KiB).
template <typename T, int NX, int NC, int V, bool SP>
__host__ __device__ constexpr int xpass_stride() {
    return (NC > 1 && xpass_min_blocks<T, NX, NC, V, SP>() == 4) ? NX + NX / 16 : cm_stride(NX);
}
// Threads per x-pass workgroup: NT, except for one-row tiles of rows of 1024
// points or more, whose columns take 32 lanes each (36 values per lane at
// 1152): there the row's 3 inverse and 2 forward column transforms would leave
// most of 8 lane groups idle, so the tile gets 4 groups.  Not for FP64 with the
// sponge, whose tile holds one workgroup per CU by its LDS alone.
template <typename T, int NX, int V, bool SP>
__host__ __device__ constexpr int xpass_threads() {
    return (NX >= 1024 && rows_x(NX, sizeof(cx<T>), V) == 1 && (sizeof(T) < 8 || !SP)) ? 128 : NT;
}

template <typename T, int NX, int N, int NC, int V, bool SP>
__global__ __launch_bounds__((xpass_threads<T, NX, V, SP>()), (xpass_min_blocks<T, NX, NC, V, SP>())) void k_xpass(
    const Member* __restrict__ mt, const cx<T>* __restrict__ tw) {
    constexpr int NT = xpass_threads<T, NX, V, SP>();  // this kernel's workgroup size
    using G = Geo<T, NX, N>;
    constexpr int K = G::KX, KP = G::KP, KPp = G::KPp;  // the x axis' cut
    constexpr int RW = rows_x(NX, sizeof(cx<T>), V);
    constexpr int NWG = N * N / RW;
    constexpr long fs_in = (long)N * N * KPp, fs_out = (long)N * N * KPp;
    const Member& m = mt[blockIdx.x / NWG];
    const StateHdr* __restrict__ hdr = m.hdr;
    const glb<cx<T>>* __restrict__ yin = gview(static_cast<const cx<T>*>(m.bufB));
    glb<cx<T>>* __restrict__ xout = gview(static_cast<cx<T>*>(m.bufA));
    const double dx = m.dx, inv_eta = m.inv_eta;
    glb<double>* __restrict__ partial = gview(m.partial);
    const int wg = blockIdx.x % NWG;
    constexpr int SC = xpass_stride<T, NX, NC, V, SP>();
    // forward columns: (N_x, N_y) of each row, N_z of row pairs (one row:
    // N_z alone, with a zero imaginary part)
    constexpr int CI = 3 * RW, CF = RW == 1 ? 2 : 3 * RW / 2;
    constexpr int CFT = SP ? 2 * CF : CF;  // forward columns (N, then chi_sp w)
    constexpr int NVAL = 3 + 12 * NC;

    constexpr int LP = (RW * KP + NT - 1) / NT;
    // FP64 kinematics for the part choice where parts overlap (FP32 runs)
    constexpr bool K64 = NC > 1 && sizeof(T) < 8;
    // inverse columns [0, CI), forward columns [CI, CI + CF).  A one-row tile
    // writes its forward columns over its first two inverse columns instead:
    // each point's thread reads its three inverse values before it writes its
    // N values at the same element.  Points flagged for the second sweep (K64)
    // write nothing in the first, so their inverse values are still there when
    // the second sweep reads them; lanes of that sweep without a flagged point
    // read aliased values but only add zeros to the wave sums.  Not with the
    // sponge's extra forward columns.  (1152-point rows: FP64 60 instead of
    // 98 KB, FP32 with flagged points 29 instead of 49 KB.)
    constexpr bool ALIAS = RW == 1 && !SP;
    __shared__ cx<T> buf[(ALIAS ? CI : CI + CFT) * SC];
    cx<T>* fbuf = ALIAS ? buf : buf + CI * SC;
    // per-wave sums: with three colours the wave rows wred also take the three
    // lane-reduced values (slots 0..2 are free there), which saves the LDS of red
    constexpr bool WAVE_ACC = NC > 1;
    __shared__ double red[WAVE_ACC ? 1 : NT / 64][WAVE_ACC ? 1 : NVAL];
    __shared__ double wred[WAVE_ACC ? NT / 64 : 1][WAVE_ACC ? NV : 1];
    __shared__ KinT<T> kin;
    // point flagged for the FP64 part decision (one bit per point); the FP64
    // kinematics of those few points are read from the state header
    __shared__ unsigned amb[K64 ? (RW * NX + 31) / 32 : 1];
    __shared__ int amb_any;
    // twiddles from LDS unless the table would cost a workgroup per CU (FP64,
    // full-size tile: the tile alone is just under half of the 160 KiB), and
    // not for rows of 1024 points or more, where staging the table for every
    // workgroup costs more than the LDS reads save (1152 points, FP32: one-row
    // tile 35.4 ms with LDS twiddles, 18.6 ms without)
    constexpr bool TWL = !(sizeof(T) == 8 && V == 0) && xpass_min_blocks<T, NX, NC, V, SP>() == 1 && NX < 1024;
    __shared__ cx<T> tws[TWL ? NX : 1];
    if (*gview(&hdr->status)) return;
    const int tid = threadIdx.x;
    const int row0 = wg * RW;
    const cx<T>* twx = tw;
    if constexpr (TWL) {
        stage_twiddles<T, NX>(tws, tw, NT);
        twx = tws;
    }
    // kinematics blocks prepared once per time level (state header) -> LDS
    const auto lds_copy = [&](const void* src, void* dst, int bytes) {
        const glb<unsigned>* a = gview(static_cast<const unsigned*>(src));
        unsigned* b = static_cast<unsigned*>(dst);
        for (int e = tid; e < bytes / 4; e += NT) b[e] = a[e];
    };
    if constexpr (NC > 0) {
        if constexpr (sizeof(T) < 8) lds_copy(&hdr->kf, &kin, (int)sizeof(KinT<T>));
        else lds_copy(&hdr->kd, &kin, (int)sizeof(KinT<T>));
    }

    if constexpr (K64) {
        for (int e = tid; e < (RW * NX + 31) / 32; e += NT) amb[e] = 0u;
        if (tid == 0) amb_any = 0;
    }
    // the wave rows of the sums start at zero; each wave clears its own row
    // (its lane 0 adds to it later, and one wave's LDS accesses stay in order)
    if constexpr (WAVE_ACC) {
        if ((tid & 63) < NV) wred[tid >> 6][(tid & 63)] = 0.0;
    }
    // 1. pack three Hermitian pairs per row: Z = X + iY over the full x axis
    cx<T> la[3][LP], lb[3][LP];
#pragma unroll
    for (int p = 0; p < 3; ++p) {
        const glb<cx<T>>* A = yin + (2 * p) * fs_in + (long)row0 * KPp;
        const glb<cx<T>>* B = yin + (2 * p + 1) * fs_in + (long)row0 * KPp;
#pragma unroll
        for (int i = 0; i < LP; ++i) {
            const int idx = tid + i * NT;
            if (idx < RW * KP) {
                const int r = idx / KP, k = idx % KP;
                la[p][i] = gld(A, r * KPp + k);
                lb[p][i] = gld(B, r * KPp + k);
            }
        }
    }
    for (int idx = tid; idx < CI * (NX - 2 * K - 1); idx += NT) {
        const int c = idx / (NX - 2 * K - 1), n = K + 1 + idx % (NX - 2 * K - 1);
        buf[lds_at<true, 1, SC>(n, c)] = cx<T>{T(0), T(0)};
    }
#pragma unroll
    for (int p = 0; p < 3; ++p) {
#pragma unroll
        for (int i = 0; i < LP; ++i) {
            const int idx = tid + i * NT;
            if (idx < RW * KP) {
                const int r = idx / KP, k = idx % KP;
                const cx<T> a = la[p][i], b = lb[p][i];
                const int cc = 3 * r + p;
                if (k == 0) {
                    buf[lds_at<true, 1, SC>(0, cc)] = cx<T>{a.x, b.x};
                } else {
                    buf[lds_at<true, 1, SC>(k, cc)] = cx<T>{a.x - b.y, a.y + b.x};
                    buf[lds_at<true, 1, SC>(NX - k, cc)] = cx<T>{a.x + b.y, b.x - a.y};
                }
            }
        }
    }
    fft_cols<T, NX, +1, CI, NT, SC>(buf, twx);
    // Whether any point of this workgroup's rows can lie inside the body's
    // cull sphere (radius^2 r2all about xc, beyond which chi == 0 exactly).
    // The rows span the whole x axis, so only their (y, z) distance counts; it
    // is taken in FP64 with a relative margin far above the rounding of the
    // per-point test, so a skipped workgroup has no point with chi > 0.
    bool wg_mask = NC > 0;
    if constexpr (NC > 0) {
        const double cy = (double)kin.xc[1], cz = (double)kin.xc[2];
        const double r2 = (double)kin.r2all * (1.0 + 1e-5);
        bool any = false;
        for (int r = 0; r < RW; ++r) {
            const int row = row0 + r;
            const double dy = dx * (row % N) - cy, dz = dx * (row / N) - cz;
            any = any || (dy * dy + dz * dz <= r2);
        }
        wg_mask = any;
    }

    // 2. pointwise source and partial sums, one point per iteration (the mask
    //    code is large; a rolled loop keeps the register count down).  The
    //    forward input goes to separate columns: column r holds (Nx, Ny) of row
    //    r, column RW + r/2 holds Nz of rows (2q, 2q+1).
    // per-lane: max |u|^2, sum |u|^2, non-finite flag, and for a single body its
    // 12 force/torque terms.  With three colours the 36 terms are rare (chi > 0
    // on few points) and are wave-reduced per iteration into wred[wave][.]
    // instead, which keeps them out of the registers.
    constexpr int NLANE = WAVE_ACC ? 3 : NVAL;
    const int lane = tid & 63, wv = tid >> 6;
    double acc[NLANE];
#pragma unroll
    for (int v = 0; v < NLANE; ++v) acc[v] = 0.0;
    const T s = T(1.0 / ((double)NX * (double)N * (double)N));
    const KinT<double>* k64p = nullptr;
    if constexpr (K64) k64p = &hdr->kd;
    // One grid point.  PH = 0: main sweep (with K64, points where two parts
    // overlap are only flagged); PH = 1: the flagged points again, with the
    // part decided in FP64 (the grid-sum terms of u were taken in the sweep).
    // act = false: the lane only takes part in the wave sums.
    // Sweep index g -> (row r, x index i).  Each wave takes a compact patch of
    // PR rows x PX points (PR*PX = 64) rather than 64 points of one row, so the
    // lanes that need the mask's geometry tend to share waves.
    constexpr int PR = (RW >= 4 && NX % 16 == 0) ? 4 : ((RW >= 2 && NX % 32 == 0) ? 2 : 1);
    constexpr int PX = 64 / PR;
    const auto decode = [](int g, int& r, int& i) {
        if constexpr (PR == 1) {
            r = g / NX;
            i = g % NX;
        } else {
            const int lane_ = g & 63, p = g >> 6;
            constexpr int NPX = NX / PX;
            r = (p / NPX) * PR + lane_ / PX;
            i = (p % NPX) * PX + lane_ % PX;
        }
    };
    const auto point = [&](int idx, bool act, auto phase) {
        constexpr int PH = decltype(phase)::value;
        // keep the kinematics block in LDS: without this compiler barrier the
        // loop-invariant values would be hoisted into registers
        __asm__ volatile("" ::: "memory");
        int r, i;
        decode(idx, r, i);
        const int row = row0 + r;
        const cx<T> z0 = buf[lds_at<true, 1, SC>(i, 3 * r)];
        const cx<T> z1 = buf[lds_at<true, 1, SC>(i, 3 * r + 1)];
        const cx<T> z2 = buf[lds_at<true, 1, SC>(i, 3 * r + 2)];
        const T ux = z0.x * s, uy = z0.y * s, uz = z1.x * s;
        const T wx = z1.y * s, wy = z2.x * s, wz = z2.y * s;
        T nx = uy * wz - uz * wy;
        T ny = uz * wx - ux * wz;
        T nz = ux * wy - uy * wx;
        if constexpr (PH == 0) {
            const double u2 = (double)ux * ux + (double)uy * uy + (double)uz * uz;
            // a non-finite value reaches the FP64 sum acc[1] (NaN and Inf
            // propagate through additions), which the step checks; slot 2 stays 0
            acc[0] = fmax(acc[0], u2);
            acc[1] += u2;
        }
        // Dirichlet layer (Sec. 2.3): penalized to u_wall below, with no body
        // terms at its points
        bool deferred = false;  // flagged for the second sweep (set in the first)
        const bool inwall = m.wall && (dx * i >= m.wall_lo[0] || dx * (row % N) >= m.wall_lo[1] ||
                                       dx * (row / N) >= m.wall_lo[2]);
        if constexpr (NC > 0) {
          if (wg_mask) {
            const double xg = dx * i, yg = dx * (row % N), zg = dx * (row / N);
            MaskPt<T> mp;
            mp.chi = T(0);
            mp.us[0] = mp.us[1] = mp.us[2] = T(0);
            mp.colour = 0;
            if (act && !inwall) {
                if constexpr (PH == 1) {
                    mp = eval_mask<T>(kin, xg, yg, zg, k64p);
                } else if constexpr (K64) {
                    bool defer = false;
                    mp = eval_mask<T>(kin, xg, yg, zg, nullptr, &defer);
                    if (defer) {
                        atomicOr(&amb[idx >> 5], 1u << (idx & 31));
                        amb_any = 1;
                        deferred = true;
                    }
                } else {
                    mp = eval_mask<T>(kin, xg, yg, zg, nullptr);
                }
            }
            const bool has = mp.chi > T(0);
            // FP64 force and torque terms from the working-precision mask values
            const auto terms = [&](double* val) {
                const double ch = mp.chi, s0 = mp.us[0], s1 = mp.us[1], s2 = mp.us[2];
                const double p0 = ch * ((double)ux - s0);
                const double p1 = ch * ((double)uy - s1);
                const double p2 = ch * ((double)uz - s2);
                const double i0 = ch * s0, i1 = ch * s1, i2 = ch * s2;
                // moments about the reference point of this part's colour (static
                // selects, no dynamic index into an array)
                const int ci = mp.colour - 1;
                const double xr0 = ci == 0 ? kin.xref[0][0] : (ci == 1 ? kin.xref[1][0] : kin.xref[2][0]);
                const double xr1 = ci == 0 ? kin.xref[0][1] : (ci == 1 ? kin.xref[1][1] : kin.xref[2][1]);
                const double xr2 = ci == 0 ? kin.xref[0][2] : (ci == 1 ? kin.xref[1][2] : kin.xref[2][2]);
                const double rx = xg - xr0, ry = yg - xr1, rz = zg - xr2;
                val[0] = p0; val[1] = p1; val[2] = p2;
                val[3] = ry * p2 - rz * p1; val[4] = rz * p0 - rx * p2; val[5] = rx * p1 - ry * p0;
                val[6] = i0; val[7] = i1; val[8] = i2;
                val[9] = ry * i2 - rz * i1; val[10] = rz * i0 - rx * i2; val[11] = rx * i1 - ry * i0;
            };
            const auto penalize = [&]() {
                const T pen = mp.chi * T(inv_eta);
                nx -= pen * (ux - mp.us[0]);
                ny -= pen * (uy - mp.us[1]);
                nz -= pen * (uz - mp.us[2]);
            };
            if constexpr (!WAVE_ACC) {
                if (has) {
                    penalize();
                    double val[12];
                    terms(val);
#pragma unroll
                    for (int e = 0; e < 12; ++e) acc[3 + e] += val[e];
                }
            } else {
                // every lane takes part in the wave sums (lanes of other colours
                // add 0); the twelve terms of a colour are formed only in waves
                // where it is present and summed together (wave_sum12)
                if (has) penalize();
                const int ci = has ? mp.colour - 1 : -1;
                static_for<NC>([&](auto cc) {
                    constexpr int col = decltype(cc)::value;
                    const bool mine = ci == col;
                    if (__any(mine)) {  // wave-uniform: only colours present in this wave
                        const double ch = mp.chi, s0 = mp.us[0], s1 = mp.us[1], s2 = mp.us[2];
                        const double p[3] = {ch * ((double)ux - s0), ch * ((double)uy - s1), ch * ((double)uz - s2)};
                        const double q[3] = {ch * s0, ch * s1, ch * s2};
                        const double rx = xg - kin.xref[col][0], ry = yg - kin.xref[col][1],
                                     rz = zg - kin.xref[col][2];
                        const double t[12] = {p[0], p[1], p[2],
                                              ry * p[2] - rz * p[1], rz * p[0] - rx * p[2], rx * p[1] - ry * p[0],
                                              q[0], q[1], q[2],
                                              ry * q[2] - rz * q[1], rz * q[0] - rx * q[2], rx * q[1] - ry * q[0]};
                        double v[12], sr[3];
#pragma unroll
                        for (int e = 0; e < 12; ++e) v[e] = mine ? t[e] : 0.0;
                        wave_sum12(v, sr);
                        if ((lane & 15) == 15) {
#pragma unroll
                            for (int j = 0; j < 3; ++j) wred[wv][3 + 12 * col + 3 * (lane >> 4) + j] += sr[j];
                        }
                    }
                });
            }
          }
        }
        if (inwall) {
            const T pen = T(inv_eta);
            nx -= pen * (ux - T(m.u_wall[0]));
            ny -= pen * (uy - T(m.u_wall[1]));
            nz -= pen * (uz - T(m.u_wall[2]));
        }
        if (act && !(ALIAS && deferred)) {
            fbuf[lds_at<true, 1, SC>(i, r)] = cx<T>{nx, ny};
            if constexpr (RW == 1) fbuf[lds_at<true, 1, SC>(i, 1)] = cx<T>{nz, T(0)};
            else reinterpret_cast<T*>(fbuf + lds_at<true, 1, SC>(i, RW + r / 2))[r & 1] = nz;
            if constexpr (SP) {
                // vorticity sponge: chi_sp * w, same column scheme after the N columns
                const double xs = dx * i, ys = dx * (row % N), zs = dx * (row / N);
                const bool in = xs >= m.sp_lo[0] || ys >= m.sp_lo[1] || zs >= m.sp_lo[2];
                const T c = in ? T(1) : T(0);
                fbuf[lds_at<true, 1, SC>(i, CF + r)] = cx<T>{c * wx, c * wy};
                if constexpr (RW == 1) fbuf[lds_at<true, 1, SC>(i, CF + 1)] = cx<T>{c * wz, T(0)};
                else reinterpret_cast<T*>(fbuf + lds_at<true, 1, SC>(i, CF + RW + r / 2))[r & 1] = c * wz;
            }
        }
    };
#pragma unroll 1
    for (int idx = tid; idx < RW * NX; idx += NT) point(idx, true, std::integral_constant<int, 0>{});
    if constexpr (K64) {
        // points where two parts overlap, in a fixed order (deterministic sums);
        // every lane runs the same number of iterations for the wave sums
        __syncthreads();
        if (wg_mask && amb_any) {
#pragma unroll 1
            for (int idx = tid; idx < RW * NX; idx += NT) point(idx, ((amb[idx >> 5] >> (idx & 31)) & 1u) != 0, std::integral_constant<int, 1>{});
        }
    }
    // workgroup partial sums: lane values of the first three by DPP, the wave rows
    // of the rest, combined over waves in a fixed order
    {
#pragma unroll
        for (int v = 0; v < NLANE; ++v) {
            double r = 0.0;
            if (__any(acc[v] != 0.0)) r = (v == 0 || v == 2) ? wave_max(acc[v]) : wave_sum(acc[v]);
            if (lane == 0) {
                if constexpr (WAVE_ACC) wred[wv][v] = r;
                else red[wv][v] = r;
            }
        }
        __syncthreads();
        if (tid < NV) {
            double r = 0.0;
            for (int w = 0; w < NT / 64; ++w) {
                double x = 0.0;
                if (tid < NVAL) {
                    if constexpr (WAVE_ACC) x = wred[w][tid];
                    else x = red[w][tid];
                }
                r = w == 0 ? x : ((tid == 0 || tid == 2) ? fmax(r, x) : r + x);
            }
            partial[(long)wg * NV + tid] = r;
        }
    }
    fft_cols<T, NX, -1, CFT, NT, SC>(fbuf, twx);

    // 3. split the packed spectra and store kx = 0..K
#pragma unroll
    for (int f = 0; f < (SP ? 6 : 3); ++f) {
        glb<cx<T>>* O = xout + f * fs_out + (long)row0 * KPp;
        const int fb = f % 3, c0 = f < 3 ? 0 : CF;
        for (int idx = tid; idx < RW * KP; idx += NT) {
            const int r = idx / KP, k = idx % KP;
            const int colx = c0 + ((fb < 2) ? r : RW + r / 2);
            const bool second = (fb == 1) || (fb == 2 && (r & 1));
            const cx<T> zk = fbuf[lds_at<true, 1, SC>(k, colx)];
            const cx<T> zm = fbuf[lds_at<true, 1, SC>((NX - k) % NX, colx)];
            cx<T> v;
            if (!second) {
                v = cx<T>{T(0.5) * (zk.x + zm.x), T(0.5) * (zk.y - zm.y)};
            } else {
                const T dxr = zk.x - zm.x, dyi = zk.y + zm.y;  // zk - conj(zm)
                v = cx<T>{T(0.5) * dyi, T(-0.5) * dxr};
            }
            gst(O, r * KPp + k, v);
        }
    }
}

// ---------------------------------------------------------------------------
// Scalar work of a step.  The x-pass leaves NV partial sums per workgroup;
// nred_of(NX, N) extra workgroups of the y-forward launch reduce fixed
// contiguous chunks of them (first level); every z-pass workgroup reduces the
// nred_of(NX, N) results in a fixed order (second level) and derives dt and the
// AB2 weights itself, so all workgroups agree bit for bit.  Workgroup 0 of the
// z-pass then writes the diagnostics and the next time level.
// ---------------------------------------------------------------------------
struct Coef {
    double dt, dtp, b1, b2;
    double umax, E;
    int first, active, bad, pad;
};

__device__ inline Coef step_coef(const double* tot, const Slot& sl, StepCtl ctl, double dx, double eta) {
    Coef c{};
    const double dV = dx * dx * dx;
    c.umax = sqrt(tot[0]);
    c.E = 0.5 * tot[1] * dV;
    if (tot[2] != 0.0 || !isfinite(c.E) || !isfinite(c.umax)) {
        c.bad = FLUSI_ENONFINITE;
        return c;
    }
    double dt;
    if (ctl.dt_fixed > 0.0) {
        dt = ctl.dt_fixed;
    } else {
        dt = c.umax > 0.0 ? ctl.cfl * dx / c.umax : INFINITY;
        if (ctl.masked) dt = fmin(dt, ctl.eta_cap * eta);
        if (ctl.dt_max > 0.0) dt = fmin(dt, ctl.dt_max);
        if (ctl.visc_cap > 0.0) dt = fmin(dt, ctl.visc_cap);
    }
    if (ctl.t_end > 0.0 && sl.t + dt > ctl.t_end) dt = ctl.t_end - sl.t;
    if (!isfinite(dt)) {
        c.bad = FLUSI_EINVAL;
        return c;
    }
    c.dt = dt;
    c.active = dt > 0.0;  // end time reached: leave the state as it is
    c.first = sl.have_prev ? 0 : 1;
    c.dtp = sl.dt_prev;
    if (sl.have_prev) {
        const double r = dt / sl.dt_prev;
        c.b1 = 1.0 + 0.5 * r;
        c.b2 = -0.5 * r;
    } else {
        c.b1 = 1.0;
        c.b2 = 0.0;
    }
    return c;
}

// Diagnostics of time level p and the next time level (one thread).  With a
// mask: the body's state at t^n (Sec. 3.6) and the wings' aerodynamic power (Sec. 3.5),
// the moment of the solid momentum about the body centre for the next step's
// unsteady torque term, and in free flight the total force and torque about
// x_cntr that advance the body (the advance itself runs with the next
// level's kinematics).  Values go to memory as they are formed and the loops
// over parts stay rolled: this code shares the z-pass kernel's registers.
__device__ inline void write_step(StateHdr* h, int p, const double* tot, const Coef& c, StepCtl ctl, double dx,
                                  double eta, double* history, int ff, int rk) {
    const Slot& sl = h->slot[p];
    Slot& nx = h->slot[1 - p];
    if (c.bad) {
        h->status = c.bad;
        return;
    }
    const double dV = dx * dx * dx;
    double* dg = h->diag;
    const auto put = [&](int i, double v) {
        dg[i] = v;
        if (history) history[i] = v;
    };
    put(0, sl.t);
    put(1, c.dt);
    put(2, c.umax);
    put(3, c.E);
    const bool corr = sl.have_I && sl.dt_prev > 0.0;
    // force (i < 3) or torque (i >= 3) on part k, with the unsteady term
    const auto part = [&](int k, int i) {
        const double* a = tot + 3 + 12 * k;
        double v = a[i] * dV / eta;
        if (corr) v += (a[6 + i] * dV - sl.I_prev[k][i]) / sl.dt_prev;
        return v;
    };
#pragma unroll 1
    for (int k = 0; k < 3; ++k)
#pragma unroll 1
        for (int i = 0; i < 6; ++i) put(4 + 6 * k + i, part(k, i));
#pragma unroll 1
    for (int i = 22; i < FLUSI_NDIAG; ++i) put(i, 0.0);
    double J[3] = {0.0, 0.0, 0.0}, Ft[3] = {0.0, 0.0, 0.0}, mt[3] = {0.0, 0.0, 0.0};
    if (ctl.body) {
        const Kin& K = h->kin;
#pragma unroll 1
        for (int i = 0; i < 3; ++i) {
            put(22 + i, K.xc[i]);
            put(25 + i, K.uc[i]);
            put(32 + i, K.omb[i]);
        }
#pragma unroll 1
        for (int i = 0; i < 4; ++i) put(28 + i, K.eps[i]);
        if (K.wings) {
#pragma unroll 1
            for (int s = 0; s < 2; ++s) {
                double wg[3];
                mat_tvec(K.Mb, K.omw[s], wg);
                const double pa = -(part(1 + s, 3) * wg[0] + part(1 + s, 4) * wg[1] + part(1 + s, 5) * wg[2]);
                put(35 + s, pa);
                put(37 + s, K.pinert[s]);               // inertial power (Sec. 3.5)
                put(39 + s, fmax(K.pinert[s] + pa, 0.0));  // total power, no energy storage
            }
        }
        // moments about x_cntr: part sums moved from each part's reference point
#pragma unroll 1
        for (int k = 0; k < 3; ++k) {
            const double* a = tot + 3 + 12 * k;
            double r[3], F[3], IF[3], t1[3], t2[3];
            for (int i = 0; i < 3; ++i) {
                r[i] = K.xref[k][i] - K.xc[i];
                F[i] = a[i] * dV / eta;
                IF[i] = a[6 + i] * dV;
                Ft[i] += part(k, i);
            }
            cross3(r, F, t1);
            cross3(r, IF, t2);
            for (int i = 0; i < 3; ++i) {
                mt[i] += a[3 + i] * dV / eta + t1[i];
                J[i] += a[9 + i] * dV + t2[i];
            }
        }
        if (corr)
            for (int i = 0; i < 3; ++i) mt[i] += (J[i] - sl.J_prev[i]) / sl.dt_prev;
    }
    {
        static_assert(sizeof(Slot) % 8 == 0, "slot copy by words");
        const double* src = reinterpret_cast<const double*>(&sl);
        double* dst = reinterpret_cast<double*>(&nx);
        constexpr int W = (int)(sizeof(Slot) / 8), B = 8;
        static_assert(W % B == 0, "slot copy batches");
#pragma unroll 1
        for (int i = 0; i < W; i += B) {
            double v[B];
#pragma unroll
            for (int j = 0; j < B; ++j) v[j] = src[i + j];
#pragma unroll
            for (int j = 0; j < B; ++j) dst[i + j] = v[j];
        }
    }
    if (c.active) {
        if (ctl.masked) {
#pragma unroll 1
            for (int k = 0; k < 3; ++k)
#pragma unroll 1
                for (int i = 0; i < 6; ++i) nx.I_prev[k][i] = tot[3 + 12 * k + 6 + i] * dV;
            for (int i = 0; i < 3; ++i) nx.J_prev[i] = J[i];
            nx.have_I = 1;
        } else {
            nx.have_I = 0;
        }
        if (ff) {
            // AB2 weights of the body (Euler on its first step)
            double b1 = 1.0, b2 = 0.0;
            if (sl.ff_have_prev) {
                const double r = c.dt / sl.dt_prev;
                b1 = 1.0 + 0.5 * r;
                b2 = -0.5 * r;
            }
            nx.ff_w[0] = c.dt * b1;
            nx.ff_w[1] = c.dt * b2;
            for (int i = 0; i < 3; ++i) {
                nx.ff_F[i] = Ft[i];
                nx.ff_m[i] = mt[i];
            }
            nx.ff_state = 2;
        } else {
            nx.ff_state = 0;
            nx.ff_have_prev = 0;
        }
        nx.have_prev = rk ? 0 : 1;  // RK4 leaves no AB2 history (its stages use that storage)
        nx.dt_prev = c.dt;
        nx.t = sl.t + c.dt;
        nx.n = sl.n + 1;
    }
    nx.rk_dt = c.active ? c.dt : 0.0;
    h->cur = 1 - p;
}

// First level: workgroup b (< NRED) reduces the x-pass records
// [b*chunk, (b+1)*chunk) ([workgroup][NV]).  Each wave reads whole records
// (one coalesced load of NV doubles) and lane v accumulates value v; the four
// waves take every fourth record and are combined in a fixed order.
template <int NRED>
__device__ inline void reduce_level1(const double* __restrict__ partial, int nwg, double* __restrict__ partial2,
                                     int b, double (*red)[NV]) {
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    constexpr int NW = NT / 64;
    const int chunk = (nwg + NRED - 1) / NRED;
    const int lo = b * chunk, hi = min(nwg, lo + chunk);
    const bool is_max = lane == 0 || lane == 2;
    const glb<double>* P = gview(partial);
    double acc = 0.0;
    if (lane < NV) {
        int w = lo + wv;
        constexpr int UN = 8;  // records in flight per wave
#pragma unroll 1
        for (; w + (UN - 1) * NW < hi; w += UN * NW) {
            double x[UN];
#pragma unroll
            for (int u = 0; u < UN; ++u) x[u] = P[(long)(w + u * NW) * NV + lane];
#pragma unroll
            for (int u = 0; u < UN; ++u) acc = is_max ? fmax(acc, x[u]) : acc + x[u];
        }
        for (; w < hi; w += NW) {
            const double x = P[(long)w * NV + lane];
            acc = is_max ? fmax(acc, x) : acc + x;
        }
        red[wv][lane] = acc;
    }
    __syncthreads();
    if (tid < NV) {
        double r = red[0][tid];
        for (int k = 1; k < NW; ++k) r = (tid == 0 || tid == 2) ? fmax(r, red[k][tid]) : r + red[k][tid];
        gview(partial2)[(long)b * NV + tid] = r;
    }
}

// Second level (whole workgroup, NTH threads): totals of the NRED records.
template <int NTH, int NRED>
__device__ inline void reduce_level2(const double* __restrict__ partial2, double* p2s, double* tot) {
    const int tid = threadIdx.x;
    constexpr int L2N = (NRED * NV + NTH - 1) / NTH;
    double tmp[L2N];
#pragma unroll
    for (int i = 0; i < L2N; ++i) {
        const int e = tid + i * NTH;
        tmp[i] = e < NRED * NV ? gview(partial2)[e] : 0.0;
    }
#pragma unroll
    for (int i = 0; i < L2N; ++i) {
        const int e = tid + i * NTH;
        if (e < NRED * NV) p2s[e] = tmp[i];
    }
    __syncthreads();
    // fixed order: value v is summed in 4 chains of NRED/4 records, then
    // the 4 chain results in order
    constexpr int CH = 4, PER = NRED / CH;
    __shared__ double chain[CH * NV];
    for (int w = tid; w < CH * NV; w += NTH) {
        const int v = w % NV, k = w / NV;
        double r = p2s[(k * PER) * NV + v];
        for (int b = 1; b < PER; ++b) {
            const double x = p2s[(k * PER + b) * NV + v];
            r = (v == 0 || v == 2) ? fmax(r, x) : r + x;
        }
        chain[k * NV + v] = r;
    }
    __syncthreads();
    for (int v = tid; v < NV; v += NTH) {
        double r = chain[v];
        for (int k = 1; k < CH; ++k) r = (v == 0 || v == 2) ? fmax(r, chain[k * NV + v]) : r + chain[k * NV + v];
        tot[v] = r;
    }
    __syncthreads();
}

// Values 0..2 of the NRED first-level records (max |u|^2, sum |u|^2, the
// non-finite flag) by one wave: lane b takes record b.  The maximum does not
// depend on the order; the sum is only tested for finiteness here (the writer
// workgroup forms every sum in the fixed order of reduce_level2).
template <int NRED>
__device__ inline void reduce_scalars(const double* __restrict__ partial2, double* tot) {
    static_assert(NRED <= 64, "one record per lane");
    const int lane = threadIdx.x & 63;
    const glb<double>* P = gview(partial2);
    double v0 = 0.0, v1 = 0.0, v2 = 0.0;
    if (lane < NRED) {
        v0 = P[(long)lane * NV + 0];
        v1 = P[(long)lane * NV + 1];
        v2 = P[(long)lane * NV + 2];
    }
    v0 = wave_max(v0);
    v1 = wave_sum(v1);
    v2 = wave_max(v2);
    if (lane == 0) {
        tot[0] = v0;
        tot[1] = v1;
        tot[2] = v2;
    }
}

// Threads of the stand-alone kinematics kernels (two waves: the two
// mask-block conversions run at once).
constexpr int NT_KIN = 128;

// Start of a stepping call, one workgroup per member: make slot 0 current and
// evaluate the kinematics of the current time level.
template <typename T>
static __global__ __launch_bounds__(NT_KIN) void k_prologue(const Member* __restrict__ mt, int nmem) {
    if ((int)blockIdx.x >= nmem) return;
    const Member& m = mt[blockIdx.x];
    StateHdr* hdr = m.hdr;
    if (threadIdx.x == 0 && hdr->cur == 1) {
        hdr->slot[0] = hdr->slot[1];
        hdr->cur = 0;
    }
    __syncthreads();
    __shared__ KinShared ks;
    if (m.nc > 0 && !hdr->status) kin_update<T>(m, 0, false, 0.0, ks);
}

// Kinematics of time level p of every member whose kinematics change with
// time (one workgroup per member); after the last step of a call it
// completes the pending free-flight advance.
template <typename T>
static __global__ __launch_bounds__(NT_KIN) void k_kin_level(const Member* __restrict__ mt, int nmem, int p) {
    if ((int)blockIdx.x >= nmem) return;
    const Member& m = mt[blockIdx.x];
    __shared__ KinShared ks;
    if (m.dyn && !m.hdr->status) kin_update<T>(m, p, false, 0.0, ks);
}

// RK4 stage kinematics (one workgroup per moving member): time t^n + c*dt,
// with t^n in slot p and dt in the slot the step's first stage wrote.
template <typename T>
static __global__ __launch_bounds__(NT_KIN) void k_kin_stage(const Member* __restrict__ mt, int nmem, int p, double c) {
    if ((int)blockIdx.x >= nmem) return;
    const Member& m = mt[blockIdx.x];
    __shared__ KinShared ks;
    if (m.dyn && !m.hdr->status) kin_update<T>(m, p, true, m.hdr->slot[p].t + c * m.hdr->slot[1 - p].rk_dt, ks);
}

// Free-flight state of the current time level of a state (one thread).
static __global__ void k_solid_set(StateHdr* h, Solid13 y) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        Slot& sl = h->slot[h->cur];
        for (int i = 0; i < 13; ++i) sl.ff[i] = y.v[i];
        sl.ff_state = 1;
        sl.ff_have_prev = 0;
    }
}

// Writes the launch record of a single plan (and the device copy of its body
// description) ahead of the kernels that read it, in stream order.
static __global__ void k_member_set(Member* dst, Member v, flusi_insect ins) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        *dst = v;
        if (v.nc > 0) *const_cast<flusi_insect*>(v.ins) = ins;
    }
}

static __global__ void k_hdr_init(StateHdr* hdr, double t0) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        unsigned char* b = reinterpret_cast<unsigned char*>(hdr);
        for (size_t i = 0; i < sizeof(StateHdr); ++i) b[i] = 0;
        hdr->slot[0].t = t0;
        hdr->cur = 0;
    }
}

// ---------------------------------------------------------------------------
// z-pass.  Columns are the kept (ky, kx) pairs, q = my*KP + kx < Q = M*KP.
// MODE_IMPORT : forward z of the imported field, projection -> state uhat
// MODE_STEP   : forward z of N, projection, IF-AB2 -> state; curl and inverse
//               z of u and w -> z-partials
// MODE_STEP_LAST : as MODE_STEP without the inverse part
// MODE_INVERSE   : curl and inverse z from the state uhat
// ---------------------------------------------------------------------------
enum { MODE_IMPORT = 0, MODE_STEP = 1, MODE_STEP_LAST = 2, MODE_INVERSE = 3, MODE_RK1 = 4, MODE_RKS = 5 };
// RK4 (MODE_RK1: first stage, with the reduction, dt and the step writer;
// MODE_RKS: stages 2-4): k_s = P N_hat - nu |k|^2 u_s; the sum k1 + 2 k2 + 2 k3
// is kept in the state's second field set, the stage velocity in ustage;
// stage 4 writes u^{n+1} = u^n + dt/6 (sum + k4).  rk = stage (2..4) | 16 when
// the curl and inverse z of the new velocity follow.

// Member table: ceil(Q/C) workgroups per member.  par: slot of the current
// time level; s: step index within the call (row of the history).
// SP: the members have the vorticity sponge (fields 3..5 of the forward input).
// Fields the z-pass transforms together (one column transform over FB*C
// columns, so that more lanes work at once): 3 where three column tiles fit
// in 64 KiB of LDS, else 1.
template <typename T, int N>
__host__ __device__ constexpr int zpass_fb() {
    return 3 * cols_z(N) * cm_stride(N) * (int)sizeof(cx<T>) <= 65536 ? 3 : 1;
}

template <typename T, int NX, int N, int MODE, int V, bool SP = false>
__global__ __launch_bounds__(nt_z(N, V)) void k_zpass(const Member* __restrict__ mt, const cx<T>* __restrict__ tw,
                                                      int par, int s, int rk) {
    using G = Geo<T, NX, N>;
    constexpr int K = G::K, KP = G::KP, M = G::M, Q = G::Q, Qp = G::Qp;
    constexpr int C = cols_z(N), NTZ = nt_z(N, V);
    constexpr int NBZ = (Q + C - 1) / C;
    // update modes: one more workgroup per member writes the diagnostics and
    // the next time level, beside the column workgroups
    constexpr bool STEPM = (MODE == MODE_STEP || MODE == MODE_STEP_LAST || MODE == MODE_RK1);
    constexpr bool RKM = (MODE == MODE_RK1 || MODE == MODE_RKS);
    constexpr int NBZ1 = NBZ + (STEPM ? 1 : 0);
    // state fields: [uhat 3][nold 3], each padded to 256 bytes
    constexpr long fs_s = (((long)M * Qp * (long)sizeof(cx<T>) + 255) / 256 * 256) / (long)sizeof(cx<T>);
    constexpr long fs_y = (long)N * Qp, fs_z = (long)N * Qp;
    const int lin = xcd_tile(blockIdx.x, gridDim.x);
    const Member& mb = mt[lin / NBZ1];
    const int tile = lin % NBZ1;
    StateHdr* hdr = mb.hdr;
    glb<cx<T>>* uhat = gview(reinterpret_cast<cx<T>*>(reinterpret_cast<char*>(hdr) + STATE_HDR_BYTES));
    glb<cx<T>>* nold = uhat + 3 * fs_s;
    const glb<cx<T>>* __restrict__ yin = gview(static_cast<const cx<T>*>(mb.bufB));
    glb<cx<T>>* __restrict__ zout = gview(static_cast<cx<T>*>(mb.bufA));
    const double kscale = mb.ks, nu = mb.nu, dx = mb.dx, eta = mb.eta;
    const int mean_mode = mb.mean_mode;
    const double* __restrict__ partial2 = mb.partial2;
    constexpr int RS = NTZ / C;   // rows per sweep
    constexpr int RPT = N / RS;   // rows per thread
    static_assert(NTZ % C == 0 && N % RS == 0, "column mapping");
    constexpr int PERM = (M + RS - 1) / RS;
    constexpr int SC = cm_stride(N);
    constexpr int FB = zpass_fb<T, N>();
    constexpr int BUFB = FB * C * SC * (int)sizeof(cx<T>);
    constexpr int REDB = nred_of(NX, N) * NV * 8;
    __shared__ __align__(16) unsigned char smem[BUFB > REDB ? BUFB : REDB];
    __shared__ double tot[NV];
    __shared__ Coef cf;
    __shared__ cx<T> tws[N];
    // AB2 steps: the integrating factors exp(-nu |k|^2 dt) split into the
    // column's exp(-nu (kx^2 + ky^2) dt) and a table of exp(-nu kz^2 dt) over
    // the kept kz (and the same for the previous step size)
    constexpr bool AB2M = (MODE == MODE_STEP || MODE == MODE_STEP_LAST);
    __shared__ double exz[AB2M ? 2 : 1][AB2M ? M : 1];
    cx<T>* buf = reinterpret_cast<cx<T>*>(smem);
    if (*gview(&hdr->status)) return;
    const int tid = threadIdx.x;
    stage_twiddles<T, N>(tws, tw, NTZ);
    const int c = tid % C, r0 = tid / C;
    const int q = tile * C + c;
    const bool okq = q < Q;
    const int kxi = q % KP, myi = q / KP;
    const double kxv = mb.ksx * kxi;
    const double kyv = kscale * j_of_m(myi, K);

    const bool step_mode = (MODE == MODE_STEP || MODE == MODE_STEP_LAST || RKM);
    // forward input: the next FB fields are loaded while the current FB are
    // transformed; the first FB are in flight together with the reduction loads
    constexpr bool FWD = (MODE == MODE_IMPORT) || step_mode;
    cx<T> vn[FWD ? FB : 1][RPT];
    const auto load_field = [&](int f, int slot) {
#pragma unroll
        for (int i = 0; i < RPT; ++i)
            vn[slot][i] = okq ? gld(yin, f * fs_y + (long)(r0 + i * RS) * Qp + q) : cx<T>{T(0), T(0)};
    };
    if constexpr (FWD) {
#pragma unroll
        for (int f = 0; f < FB; ++f) load_field(f, f);
    }
    if constexpr (STEPM) {
        if (tile == NBZ) {
            // the writer: every sum in the fixed order (diagnostics, forces)
            reduce_level2<NTZ, nred_of(NX, N)>(partial2, reinterpret_cast<double*>(smem), tot);
            if (tid == 0)
                write_step(hdr, par, tot, step_coef(tot, hdr->slot[par], mb.ctl, dx, eta), mb.ctl, dx, eta,
                           mb.history ? mb.history + (long)s * FLUSI_NDIAG : nullptr, mb.ff, mb.rk);
            return;
        }
        // column workgroups need max|u|^2 (order-free), the finiteness of the
        // |u|^2 sum and the non-finite flag: one wave, no LDS round trips
        if (tid < 64) reduce_scalars<nred_of(NX, N)>(partial2, tot);
        __syncthreads();
        if (tid == 0) cf = step_coef(tot, hdr->slot[par], mb.ctl, dx, eta);
        __syncthreads();
        if (cf.bad) return;
        if constexpr (AB2M) {
            // visible after the barriers of the forward transforms
            for (int m = tid; m < M; m += NTZ) {
                const double kz = kscale * j_of_m(m, K);
                exz[0][m] = exp(-nu * (kz * kz) * cf.dt);
                exz[1][m] = cf.first ? 0.0 : exp(-nu * (kz * kz) * cf.dtp);
            }
        }
    }
    // RK stages 2-4: the step size the first stage chose (0: no step)
    const double rdt = MODE == MODE_RKS ? *gview(&hdr->slot[1 - par].rk_dt) : 0.0;
    if (MODE == MODE_RKS && !(rdt > 0.0)) return;
    const bool active = STEPM ? (cf.active != 0) : true;
    const bool do_fwd = (MODE == MODE_IMPORT) || (step_mode && active);
    const bool do_inv = (MODE == MODE_STEP) || (MODE == MODE_INVERSE) || (RKM && (rk & 16));

    // kept kz of this thread: m = r0 + i*RS, i < PERM
    cx<T> U[3][PERM];
    if (do_fwd) {
        // vorticity sponge: fields 3..5 hold chi_sp * w
        constexpr bool sp = SP && (MODE == MODE_STEP || MODE == MODE_STEP_LAST || RKM);
        cx<T> Nh[3][PERM];
        // column c of field f0 + b of a batch sits in LDS column b*C + c
        const auto put_batch = [&](int f0) {
#pragma unroll
            for (int b = 0; b < FB; ++b) {
#pragma unroll
                for (int i = 0; i < RPT; ++i) buf[(b * C + c) * SC + cpad(r0 + i * RS)] = vn[b][i];
            }
            if (f0 + FB < (sp ? 6 : 3)) {
#pragma unroll
                for (int b = 0; b < FB; ++b) load_field(f0 + FB + b, b);
            }
            fft_cols<T, N, -1, FB * C, NTZ, SC>(buf, tws);
        };
#pragma unroll
        for (int f0 = 0; f0 < 3; f0 += FB) {
            put_batch(f0);
#pragma unroll
            for (int b = 0; b < FB; ++b) {
#pragma unroll
                for (int i = 0; i < PERM; ++i) {
                    const int m = r0 + i * RS;
                    if (m < M) Nh[f0 + b][i] = buf[(b * C + c) * SC + cpad(bin_of_m(m, N, K))];
                }
            }
            __syncthreads();
        }
        if constexpr (sp) {
            // N_hat += -(1/C_sp) (i k x W_hat)/|k|^2, one W component at a time
            // (eq. PNST_org_momentum, sponge term; zero at k = 0)
#pragma unroll
            for (int f0 = 3; f0 < 6; f0 += FB) {
                put_batch(f0);
#pragma unroll
                for (int b = 0; b < FB; ++b) {
                const int f = f0 + b;
#pragma unroll
                for (int i = 0; i < PERM; ++i) {
                    const int m = r0 + i * RS;
                    if (m < M && okq) {
                        const cx<T> w = buf[(b * C + c) * SC + cpad(bin_of_m(m, N, K))];
                        const double kzv = kscale * j_of_m(m, K);
                        const double k2 = kxv * kxv + kyv * kyv + kzv * kzv;
                        const double a = k2 > 0.0 ? -mb.inv_csp / k2 : 0.0;
                        // i * w = (-w.y, w.x)
                        const double pr = -a * (double)w.y, pi = a * (double)w.x;
                        const auto add = [&](cx<T>& t, double coef) {
                            t = cx<T>{T((double)t.x + coef * pr), T((double)t.y + coef * pi)};
                        };
                        if (f == 3) {         // W_x: (k x W)_y += kz Wx, (k x W)_z -= ky Wx
                            add(Nh[1][i], kzv);
                            add(Nh[2][i], -kyv);
                        } else if (f == 4) {  // W_y: (k x W)_x -= kz Wy, (k x W)_z += kx Wy
                            add(Nh[0][i], -kzv);
                            add(Nh[2][i], kxv);
                        } else {              // W_z: (k x W)_x += ky Wz, (k x W)_y -= kx Wz
                            add(Nh[0][i], kyv);
                            add(Nh[1][i], -kxv);
                        }
                    }
                }
                }
                __syncthreads();
            }
        }
        double dt = 0, b1 = 0, b2 = 0, dtp = 0;
        int first = 1;
        if (STEPM) {
            dt = cf.dt;
            b1 = cf.b1;
            b2 = cf.b2;
            dtp = cf.dtp;
            first = cf.first;
        }
        if (MODE == MODE_RKS) dt = rdt;
        double exy[2] = {0.0, 0.0};
        if (AB2M) {
            const double kxy2 = kxv * kxv + kyv * kyv;
            exy[0] = exp(-nu * kxy2 * dt);
            exy[1] = first ? 0.0 : exp(-nu * kxy2 * dtp);
        }
        const int stage = MODE == MODE_RK1 ? 1 : (rk & 15);
        glb<cx<T>>* ust = gview(static_cast<cx<T>*>(mb.ustage));
#pragma unroll
        for (int i = 0; i < PERM; ++i) {
            const int m = r0 + i * RS;
            if (m < M && okq) {
                const double kzv = kscale * j_of_m(m, K);
                const double k2 = kxv * kxv + kyv * kyv + kzv * kzv;
                double nr[3], ni[3];
#pragma unroll
                for (int f = 0; f < 3; ++f) {
                    nr[f] = (double)Nh[f][i].x;
                    ni[f] = (double)Nh[f][i].y;
                }
                if (k2 > 0.0) {
                    const double ik2 = 1.0 / k2;
                    const double sr = (kxv * nr[0] + kyv * nr[1] + kzv * nr[2]) * ik2;
                    const double si = (kxv * ni[0] + kyv * ni[1] + kzv * ni[2]) * ik2;
                    nr[0] -= kxv * sr; nr[1] -= kyv * sr; nr[2] -= kzv * sr;
                    ni[0] -= kxv * si; ni[1] -= kyv * si; ni[2] -= kzv * si;
                } else if (step_mode && mean_mode == FLUSI_MEAN_FIXED) {
                    nr[0] = nr[1] = nr[2] = 0.0;
                    ni[0] = ni[1] = ni[2] = 0.0;
                }
                const long e = (long)m * Qp + q;
                if (MODE == MODE_IMPORT) {
#pragma unroll
                    for (int f = 0; f < 3; ++f) {
                        U[f][i] = cx<T>{T(nr[f]), T(ni[f])};
                        gst(uhat, f * fs_s + e, U[f][i]);
                    }
                } else if constexpr (RKM) {
                    const double nk2 = nu * k2;
#pragma unroll
                    for (int f = 0; f < 3; ++f) {
                        const cx<T> un = gld(uhat, f * fs_s + e);
                        const cx<T> us = stage == 1 ? un : gld(ust, f * fs_s + e);
                        const double kr = nr[f] - nk2 * (double)us.x, ki = ni[f] - nk2 * (double)us.y;
                        double vr, vi;
                        if (stage == 4) {
                            const cx<T> a = gld(nold, f * fs_s + e);
                            vr = (double)un.x + dt / 6.0 * ((double)a.x + kr);
                            vi = (double)un.y + dt / 6.0 * ((double)a.y + ki);
                            U[f][i] = cx<T>{T(vr), T(vi)};
                            gst(uhat, f * fs_s + e, U[f][i]);
                        } else {
                            double ar = kr, ai = ki;
                            if (stage > 1) {
                                const cx<T> a = gld(nold, f * fs_s + e);
                                ar = (double)a.x + 2.0 * kr;
                                ai = (double)a.y + 2.0 * ki;
                            }
                            gst(nold, f * fs_s + e, cx<T>{T(ar), T(ai)});
                            const double cs = stage == 3 ? dt : 0.5 * dt;
                            vr = (double)un.x + cs * kr;
                            vi = (double)un.y + cs * ki;
                            U[f][i] = cx<T>{T(vr), T(vi)};
                            gst(ust, f * fs_s + e, U[f][i]);
                        }
                    }
                } else {
                    const double e1 = exy[0] * exz[AB2M ? 0 : 0][AB2M ? m : 0];
                    const double c2 = first ? 0.0 : b2 * (exy[1] * exz[AB2M ? 1 : 0][AB2M ? m : 0]);
                    // the six loads of this mode are issued before its first
                    // store, so that they are in flight together (interleaved
                    // with the stores, which may alias them as far as the
                    // compiler knows, each would wait one memory round trip)
                    cx<T> uo[3], no[3];
#pragma unroll
                    for (int f = 0; f < 3; ++f) {
                        uo[f] = gld(uhat, f * fs_s + e);
                        if (!first) no[f] = gld(nold, f * fs_s + e);
                    }
#pragma unroll
                    for (int f = 0; f < 3; ++f) {
                        double ar = nr[f], ai = ni[f];
                        if (!first) {
                            ar = b1 * nr[f] + c2 * (double)no[f].x;
                            ai = b1 * ni[f] + c2 * (double)no[f].y;
                        }
                        const double vr = e1 * ((double)uo[f].x + dt * ar);
                        const double vi = e1 * ((double)uo[f].y + dt * ai);
                        U[f][i] = cx<T>{T(vr), T(vi)};
                        gst(uhat, f * fs_s + e, U[f][i]);
                        gst(nold, f * fs_s + e, cx<T>{T(nr[f]), T(ni[f])});
                    }
                }
            }
        }
    } else if (do_inv) {
#pragma unroll
        for (int i = 0; i < PERM; ++i) {
            const int m = r0 + i * RS;
            if (m < M && okq) {
                const long e = (long)m * Qp + q;
#pragma unroll
                for (int f = 0; f < 3; ++f) U[f][i] = gld(uhat, f * fs_s + e);
            }
        }
    }
    if (!do_inv) return;

    const T kx = T(kxv), ky = T(kyv);
    // u and w = i k x u, FB fields per column transform (field g0 + b in LDS
    // columns b*C ..)
#pragma unroll
    for (int g0 = 0; g0 < 6; g0 += FB) {
        for (int idx = tid; idx < FB * C * (N - M); idx += NTZ) {
            const int b = idx / (C * (N - M)), e = idx % (C * (N - M));
            buf[(b * C + e % C) * SC + cpad(K + 1 + e / C)] = cx<T>{T(0), T(0)};
        }
#pragma unroll
        for (int b = 0; b < FB; ++b) {
            const int g = g0 + b;
#pragma unroll
            for (int i = 0; i < PERM; ++i) {
                const int m = r0 + i * RS;
                if (m < M) {
                    cx<T> v = {T(0), T(0)};
                    if (okq) {
                        if (g < 3) {
                            v = U[g][i];
                        } else {
                            const T kz = T(kscale * j_of_m(m, K));
                            cx<T> a;
                            if (g == 3) a = U[2][i] * ky - U[1][i] * kz;
                            else if (g == 4) a = U[0][i] * kz - U[2][i] * kx;
                            else a = U[1][i] * kx - U[0][i] * ky;
                            v = mul_pi(a);
                        }
                    }
                    buf[(b * C + c) * SC + cpad(bin_of_m(m, N, K))] = v;
                }
            }
        }
        fft_cols<T, N, +1, FB * C, NTZ, SC>(buf, tws);
        if (okq) {
#pragma unroll
            for (int b = 0; b < FB; ++b) {
                cx<T> o[RPT];
#pragma unroll
                for (int i = 0; i < RPT; ++i) o[i] = buf[(b * C + c) * SC + cpad(r0 + i * RS)];
#pragma unroll
                for (int i = 0; i < RPT; ++i) gst(zout, (g0 + b) * fs_z + (long)(r0 + i * RS) * Qp + q, o[i]);
            }
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Real transforms along x for the full-layout utilities.  Two real rows are
// packed into one complex transform.  nkx: number of kx written/read
// (n/2+1 for the full layout, K+1 for the pruned import).
// ---------------------------------------------------------------------------
template <typename T, int N>
__global__ __launch_bounds__(NT) void k_x_r2c(const T* __restrict__ in, cx<T>* __restrict__ out, long nrows, int nkx,
                                              int pitch, const cx<T>* __restrict__ tw) {
    constexpr int RW = 2 * rows_x(N);  // real rows per workgroup
    constexpr int SC = cm_stride(N);
    constexpr int CP = RW / 2;
    __shared__ cx<T> buf[CP * SC];
    const int tid = threadIdx.x;
    const long row0 = (long)blockIdx.x * RW;
    for (int idx = tid; idx < RW * N; idx += NT) {
        const int r = idx / N, i = idx % N;
        const T v = (row0 + r < nrows) ? in[row0 * N + idx] : T(0);
        reinterpret_cast<T*>(buf + lds_at<true, 1, SC>(i, r / 2))[r & 1] = v;
    }
    fft_cols<T, N, -1, CP, NT, SC>(buf, tw);
    for (int idx = tid; idx < RW * nkx; idx += NT) {
        const int r = idx / nkx, k = idx % nkx;
        if (row0 + r >= nrows) continue;
        const cx<T> zk = buf[lds_at<true, 1, SC>(k, r / 2)];
        const cx<T> zm = buf[lds_at<true, 1, SC>((N - k) % N, r / 2)];
        cx<T> v;
        if (!(r & 1)) {
            v = cx<T>{T(0.5) * (zk.x + zm.x), T(0.5) * (zk.y - zm.y)};
        } else {
            v = cx<T>{T(0.5) * (zk.y + zm.y), T(-0.5) * (zk.x - zm.x)};
        }
        out[(row0 + r) * pitch + k] = v;
    }
}

template <typename T, int N>
__global__ __launch_bounds__(NT) void k_x_c2r(const cx<T>* __restrict__ in, T* __restrict__ out, long nrows, int nkx,
                                              T scale, const cx<T>* __restrict__ tw) {
    constexpr int RW = 2 * rows_x(N);
    constexpr int SC = cm_stride(N);
    constexpr int CP = RW / 2;
    __shared__ cx<T> buf[CP * SC];
    const int tid = threadIdx.x;
    const long row0 = (long)blockIdx.x * RW;
    for (int idx = tid; idx < CP * N; idx += NT) buf[lds_at<true, 1, SC>(idx % N, idx / N)] = cx<T>{T(0), T(0)};
    __syncthreads();
    for (int idx = tid; idx < CP * nkx; idx += NT) {
        const int p = idx / nkx, k = idx % nkx;
        const long ra = row0 + 2 * p, rb = ra + 1;
        const cx<T> a = ra < nrows ? in[ra * nkx + k] : cx<T>{T(0), T(0)};
        const cx<T> b = rb < nrows ? in[rb * nkx + k] : cx<T>{T(0), T(0)};
        if (k == 0 || 2 * k == N) {
            buf[lds_at<true, 1, SC>(k, p)] = cx<T>{a.x, b.x};
        } else {
            buf[lds_at<true, 1, SC>(k, p)] = cx<T>{a.x - b.y, a.y + b.x};
            buf[lds_at<true, 1, SC>(N - k, p)] = cx<T>{a.x + b.y, b.x - a.y};
        }
    }
    fft_cols<T, N, +1, CP, NT, SC>(buf, tw);
    for (int idx = tid; idx < RW * N; idx += NT) {
        const int r = idx / N, i = idx % N;
        if (row0 + r >= nrows) continue;
        const cx<T> z = buf[lds_at<true, 1, SC>(i, r / 2)];
        out[row0 * N + idx] = ((r & 1) ? z.y : z.x) * scale;
    }
}

// ---------------------------------------------------------------------------
// Full-layout helpers of the unfused right-hand side
// ---------------------------------------------------------------------------
__device__ __forceinline__ int jsigned(int i, int n) { return i < n / 2 ? i : i - n; }

// w_hat = i k x u_hat and a copy of u_hat: out [6] = (u0,u1,u2,w0,w1,w2)
template <typename T>
__global__ void k_curl_full(const cx<T>* __restrict__ uh, cx<T>* __restrict__ out, int n, double kscale) {
    const int nkx = n / 2 + 1;
    const long tot = (long)n * n * nkx;
    const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= tot) return;
    const int ix = e % nkx, iy = (e / nkx) % n, iz = e / ((long)nkx * n);
    // derivative of a Nyquist mode is zero
    const T kx = ix == n / 2 ? T(0) : T(kscale * ix);
    const T ky = iy == n / 2 ? T(0) : T(kscale * jsigned(iy, n));
    const T kz = iz == n / 2 ? T(0) : T(kscale * jsigned(iz, n));
    const cx<T> u0 = uh[e], u1 = uh[tot + e], u2 = uh[2 * tot + e];
    out[e] = u0;
    out[tot + e] = u1;
    out[2 * tot + e] = u2;
    out[3 * tot + e] = mul_pi(u2 * ky - u1 * kz);
    out[4 * tot + e] = mul_pi(u0 * kz - u2 * kx);
    out[5 * tot + e] = mul_pi(u1 * kx - u0 * ky);
}

// N = u x w - (chi/C_eta)(u - u_s) in place over the first three fields; max|u|^2 partials
template <typename T>
__global__ __launch_bounds__(NT) void k_source_full(T* __restrict__ f6, const T* __restrict__ chi,
                                                    const T* __restrict__ us, long npts, double inv_eta,
                                                    double* __restrict__ pmax) {
    __shared__ double red[NT / 64];
    const long p = (long)blockIdx.x * NT + threadIdx.x;
    double u2 = 0.0;
    if (p < npts) {
        const T ux = f6[p], uy = f6[npts + p], uz = f6[2 * npts + p];
        const T wx = f6[3 * npts + p], wy = f6[4 * npts + p], wz = f6[5 * npts + p];
        T nx = uy * wz - uz * wy, ny = uz * wx - ux * wz, nz = ux * wy - uy * wx;
        if (chi) {
            const T pen = T((double)chi[p] * inv_eta);
            const T s0 = us ? us[p] : T(0), s1 = us ? us[npts + p] : T(0), s2 = us ? us[2 * npts + p] : T(0);
            nx -= pen * (ux - s0);
            ny -= pen * (uy - s1);
            nz -= pen * (uz - s2);
        }
        f6[p] = nx;
        f6[npts + p] = ny;
        f6[2 * npts + p] = nz;
        u2 = (double)ux * ux + (double)uy * uy + (double)uz * uz;
        if (!isfinite(u2)) u2 = INFINITY;
    }
    u2 = wave_max(u2);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = u2;
    __syncthreads();
    if (threadIdx.x == 0) {
        double r = red[0];
        for (int w = 1; w < NT / 64; ++w) r = fmax(r, red[w]);
        pmax[blockIdx.x] = r;
    }
}

// 2/3 rule and projection of a full-layout right-hand side, in place.
template <typename T>
__global__ void k_project_full(cx<T>* __restrict__ f3, int n, double kscale, int mean_mode) {
    const int nkx = n / 2 + 1;
    const long tot = (long)n * n * nkx;
    const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= tot) return;
    const int ix = e % nkx, iy = (e / nkx) % n, iz = e / ((long)nkx * n);
    const int jx = ix, jy = jsigned(iy, n), jz = jsigned(iz, n);
    if (3 * abs(jx) >= n || 3 * abs(jy) >= n || 3 * abs(jz) >= n) {
        f3[e] = f3[tot + e] = f3[2 * tot + e] = cx<T>{T(0), T(0)};
        return;
    }
    const double kx = kscale * jx, ky = kscale * jy, kz = kscale * jz;
    const double k2 = kx * kx + ky * ky + kz * kz;
    const cx<T> a = f3[e], b = f3[tot + e], c = f3[2 * tot + e];
    if (k2 > 0.0) {
        const double sr = (kx * a.x + ky * b.x + kz * c.x) / k2;
        const double si = (kx * a.y + ky * b.y + kz * c.y) / k2;
        f3[e] = cx<T>{T(a.x - kx * sr), T(a.y - kx * si)};
        f3[tot + e] = cx<T>{T(b.x - ky * sr), T(b.y - ky * si)};
        f3[2 * tot + e] = cx<T>{T(c.x - kz * sr), T(c.y - kz * si)};
    } else if (mean_mode == FLUSI_MEAN_FIXED) {
        f3[e] = f3[tot + e] = f3[2 * tot + e] = cx<T>{T(0), T(0)};
    }
}

// Materialized mask (flusi_mask_insect).
template <typename T>
__global__ void k_mask(const Kin* __restrict__ kin, int nx, int n, double dx, T* __restrict__ chi,
                       T* __restrict__ us, int16_t* __restrict__ colour) {
    __shared__ KinT<T> kt;
    constexpr bool K64 = sizeof(T) < 8;
    __shared__ typename std::conditional<K64, KinT<double>, char>::type k64s;
    if (threadIdx.x == 0) kin_cast<T>(*kin, kt);
    if constexpr (K64) {
        if (threadIdx.x == 64) kin_cast<double>(*kin, k64s);
    }
    __syncthreads();
    const long npts = (long)nx * n * n;
    const long p = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= npts) return;
    const int i = p % nx, j = (p / nx) % n, k = p / ((long)nx * n);
    const KinT<double>* k64 = nullptr;
    if constexpr (K64) k64 = &k64s;
    const MaskPt<T> mp = eval_mask<T>(kt, dx * i, dx * j, dx * k, k64);
    if (chi) chi[p] = T(mp.chi);
    if (us) {
        us[p] = T(mp.us[0]);
        us[npts + p] = T(mp.us[1]);
        us[2 * npts + p] = T(mp.us[2]);
    }
    if (colour) colour[p] = (int16_t)mp.colour;
}

static __global__ void k_kin(Kin* kin, flusi_insect ins, double t, double dx, const double* rtab,
                             const float* rtab32) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        compute_kin(ins, t, dx, *kin);
        kin->rtab = rtab;
        kin->rtab32 = rtab32;
    }
}

// Radius table of a Fourier wing (Sec. 3.4): R at the FLUSI_RTABLE angles
// v_j = j / FLUSI_RTABLE in turns, plus a copy of the first sample at the end
// for the interpolation across v = 1; FP32 copies rounded from the FP64 ones.
static __global__ __launch_bounds__(256) void k_rtab_build(WingCoef c, double* __restrict__ tab,
                                                           float* __restrict__ tab32) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j > FLUSI_RTABLE) return;
    const double v = (double)(j % FLUSI_RTABLE) / FLUSI_RTABLE;
    double r = 0.5 * c.a[0];
    for (int i = 1; i <= c.n; ++i) r += c.a[i] * cos(2.0 * M_PI * i * v) + c.b[i] * sin(2.0 * M_PI * i * v);
    tab[j] = r;
    tab32[j] = float(r);
}

// Pruned state spectrum [3][M][Qp] (q = my*KP + kx) -> full layout [3][n][n][nx/2+1] (zeros elsewhere).
template <typename T>
__global__ void k_export_full(const cx<T>* __restrict__ st, cx<T>* __restrict__ out, int nx, int n, long fs_s,
                              long Qp) {
    const int nkx = nx / 2 + 1;
    const int K = kmax_of(n), KX = kmax_of(nx), KP = KX + 1;
    const long tot = (long)n * n * nkx;
    const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= tot) return;
    const int ix = e % nkx, iy = (e / nkx) % n, iz = e / ((long)nkx * n);
    const int my = m_of_bin(iy, n, K), mz = m_of_bin(iz, n, K);
    const bool kept = ix <= KX && my >= 0 && mz >= 0;
    for (int f = 0; f < 3; ++f)
        out[f * tot + e] = kept ? st[f * fs_s + (long)mz * Qp + (long)my * KP + ix] : cx<T>{T(0), T(0)};
}

}  // namespace flusi
