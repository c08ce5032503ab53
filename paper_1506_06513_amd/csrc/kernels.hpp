// HIP kernels of the pseudo-spectral penalized Navier-Stokes step (gfx950).
//
// Stepping schedule, four HBM passes per time step over 2/3-pruned spectra
// (K = (n-1)/3 is the largest kept |j|; KP = K+1 kept kx; M = 2K+1 kept ky,kz):
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
#include "common.hpp"
#include "fft.hpp"
#include "insect.hpp"

namespace flusi {

constexpr int NT = 256;   // threads per workgroup of every pass
constexpr int NV = 39;    // reduction values per workgroup (see xpass)
constexpr int NRED_BLOCKS = 64;

// Columns per workgroup of the column passes: C*N ~ 4096 elements in LDS.
__host__ __device__ constexpr int cols_of(int N) {
    int c = 4096 / N, p = 8;
    while (p * 2 <= c) p *= 2;
    return p;
}
// Rows per workgroup of the x-pass (even): 3*RW*N ~ 3072 elements in LDS.
__host__ __device__ constexpr int rows_x(int N) {
    int c = 1024 / N, p = 2;
    while (p * 2 <= c) p *= 2;
    return p;
}

struct StepCtl {
    double dt_fixed, cfl, dt_max, eta_cap, t_end;
    int masked, mean_mode;
};

// Device-resident per-state scalars (first 4 KiB of a state buffer).
struct StateHdr {
    double t;        // time of the current coefficients
    double dt_prev;  // previous step size
    long long n;     // steps taken
    int have_prev;   // previous right-hand side stored
    int status;      // 0 or FLUSI_ENONFINITE / FLUSI_EINVAL
    int have_I;      // previous solid-momentum integral stored
    int active;      // coefficient block below is valid for this step
    int first;       // this step is the first (Euler) step
    int pad0;
    double dt, dtp, b1, b2;  // coefficients of the current update
    double I_prev[3][6];
    double diag[FLUSI_NDIAG];
    Kin kin;         // kinematics at time t
};
static_assert(sizeof(StateHdr) <= 4096, "state header too large");
constexpr size_t STATE_HDR_BYTES = 4096;

// ---------------------------------------------------------------------------
// Generic column FFT along y or z.
// Column q (q < Q) of a field starts at (q / KX) * blk + q % KX; element e of
// the column sits at stride s.  PIN: the input holds only the 2K+1 kept
// signed modes (pruned storage); POUT: only those are written.
// ---------------------------------------------------------------------------
template <typename T, int N, int DIR, bool PIN, bool POUT>
__global__ __launch_bounds__(NT) void k_colfft(const cx<T>* in, cx<T>* out, int K, int Q, int KX,
                                               long blk_in, long s_in, long blk_out, long s_out,
                                               long fs_in, long fs_out, const cx<T>* __restrict__ tw,
                                               const int* status) {
    constexpr int C = cols_of(N);
    static_assert(NT % C == 0 || C % NT == 0, "column mapping");
    __shared__ cx<T> buf[C * N];
    if (status && *status) return;
    const int tid = threadIdx.x;
    const int f = blockIdx.y;
    in += f * fs_in;
    out += f * fs_out;
    const int c = tid % C;
    const int q = blockIdx.x * C + c;
    const bool ok = q < Q;
    const long bin = ok ? (long)(q / KX) * blk_in + q % KX : 0;
    const long bout = ok ? (long)(q / KX) * blk_out + q % KX : 0;
    for (int n = tid / C; n < N; n += NT / C) {
        cx<T> v = {T(0), T(0)};
        if (ok) {
            if constexpr (PIN) {
                const int m = m_of_bin(n, N, K);
                if (m >= 0) v = in[bin + m * s_in];
            } else {
                v = in[bin + n * s_in];
            }
        }
        buf[n * C + c] = v;
    }
    fft_lds<T, N, DIR, C, NT, C, 1>(buf, tw);
    const int nout = POUT ? 2 * K + 1 : N;
    if (ok) {
        for (int o = tid / C; o < nout; o += NT / C) {
            const int n = POUT ? bin_of_m(o, N, K) : o;
            out[bout + o * s_out] = buf[n * C + c];
        }
    }
}

// ---------------------------------------------------------------------------
// Deterministic workgroup reductions
// ---------------------------------------------------------------------------
__device__ __forceinline__ double wave_sum(double v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
__device__ __forceinline__ double wave_max(double v) {
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}

// Reduce NV per-thread values (value 0 and 2 by max, the rest by sum) over the
// workgroup; the result lands in out[0..NV) (global) from thread v.
template <int NVAL>
__device__ __forceinline__ void block_reduce_store(const double (&acc)[NVAL], double (*red)[NV], double* out) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int v = 0; v < NVAL; ++v) {
        const double r = (v == 0 || v == 2) ? wave_max(acc[v]) : wave_sum(acc[v]);
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
        out[t] = r;
    }
}

// ---------------------------------------------------------------------------
// x-pass: inverse x, pointwise source with the mask, FP64 partial sums,
// forward x.  Reduction values per workgroup:
//   [0] max |u|^2, [1] sum |u|^2, [2] non-finite flag,
//   [3 + 12 c + 0..2]  sum chi (u - u_s)            (colour c+1)
//   [3 + 12 c + 3..5]  sum (x - x_ref) x chi (u - u_s)
//   [3 + 12 c + 6..8]  sum chi u_s
//   [3 + 12 c + 9..11] sum (x - x_ref) x chi u_s
// NC: number of colours accumulated (0 no mask, 1 single body, 3 insect).
// ---------------------------------------------------------------------------
template <typename T, int N, int NC>
__global__ __launch_bounds__(NT) void k_xpass(const cx<T>* __restrict__ yin, cx<T>* __restrict__ xout,
                                              long fs_in, long fs_out, const cx<T>* __restrict__ tw,
                                              const StateHdr* __restrict__ hdr, flusi_insect ins, double dx,
                                              double inv_eta, double* __restrict__ partial) {
    constexpr int K = kmax_of(N), KP = K + 1;
    constexpr int RW = rows_x(N);
    constexpr int SC = N + 1;
    constexpr int CI = 3 * RW, CF = 3 * RW / 2;
    constexpr int NVAL = 3 + 12 * NC;
    constexpr int PP = (RW * N + NT - 1) / NT;
    __shared__ cx<T> buf[CI * SC];
    __shared__ double red[NT / 64][NV];
    __shared__ Kin kin;
    if (hdr->status) return;
    const int tid = threadIdx.x;
    const int row0 = blockIdx.x * RW;
    if constexpr (NC > 0) {
        if (tid == 0) kin = hdr->kin;
    }

    // 1. pack three Hermitian pairs per row: Z = X + iY over the full x axis
    for (int idx = tid; idx < CI * (N - 2 * K - 1); idx += NT) {
        const int c = idx / (N - 2 * K - 1), n = K + 1 + idx % (N - 2 * K - 1);
        buf[c * SC + n] = cx<T>{T(0), T(0)};
    }
#pragma unroll
    for (int p = 0; p < 3; ++p) {
        const cx<T>* A = yin + (2 * p) * fs_in + (long)row0 * KP;
        const cx<T>* B = yin + (2 * p + 1) * fs_in + (long)row0 * KP;
        for (int idx = tid; idx < RW * KP; idx += NT) {
            const int r = idx / KP, k = idx % KP;
            const cx<T> a = A[idx], b = B[idx];
            cx<T>* col = buf + (3 * r + p) * SC;
            if (k == 0) {
                col[0] = cx<T>{a.x, b.x};
            } else {
                col[k] = cx<T>{a.x - b.y, a.y + b.x};
                col[N - k] = cx<T>{a.x + b.y, b.x - a.y};
            }
        }
    }
    fft_lds<T, N, +1, CI, NT, 1, SC>(buf, tw);

    // 2. pointwise source and partial sums
    double acc[NVAL];
#pragma unroll
    for (int v = 0; v < NVAL; ++v) acc[v] = 0.0;
    const T s = T(1.0 / ((double)N * (double)N * (double)N));
    T res[PP][3];
#pragma unroll
    for (int j = 0; j < PP; ++j) {
        const int idx = tid + j * NT;
        if (idx < RW * N) {
            const int r = idx / N, i = idx % N;
            const int row = row0 + r;
            const cx<T> z0 = buf[(3 * r) * SC + i], z1 = buf[(3 * r + 1) * SC + i], z2 = buf[(3 * r + 2) * SC + i];
            const T ux = z0.x * s, uy = z0.y * s, uz = z1.x * s;
            const T wx = z1.y * s, wy = z2.x * s, wz = z2.y * s;
            T nx = uy * wz - uz * wy;
            T ny = uz * wx - ux * wz;
            T nz = ux * wy - uy * wx;
            const double u2 = (double)ux * ux + (double)uy * uy + (double)uz * uz;
            acc[0] = fmax(acc[0], u2);
            acc[1] += u2;
            if (!isfinite(u2)) acc[2] = 1.0;
            if constexpr (NC > 0) {
                const double xg = dx * i, yg = dx * (row % N), zg = dx * (row / N);
                const MaskPt mp = eval_mask(kin, ins, xg, yg, zg);
                if (mp.chi > 0.0) {
                    const T pen = T(mp.chi * inv_eta);
                    nx -= pen * (ux - T(mp.us[0]));
                    ny -= pen * (uy - T(mp.us[1]));
                    nz -= pen * (uz - T(mp.us[2]));
                    const double p0 = mp.chi * ((double)ux - mp.us[0]);
                    const double p1 = mp.chi * ((double)uy - mp.us[1]);
                    const double p2 = mp.chi * ((double)uz - mp.us[2]);
                    const double i0 = mp.chi * mp.us[0], i1 = mp.chi * mp.us[1], i2 = mp.chi * mp.us[2];
                    static_for<NC>([&](auto cc) {
                        constexpr int col = decltype(cc)::value;
                        if (mp.colour == col + 1) {
                            const double rx = xg - kin.xref[col][0], ry = yg - kin.xref[col][1], rz = zg - kin.xref[col][2];
                            double* a = acc + 3 + 12 * col;
                            a[0] += p0; a[1] += p1; a[2] += p2;
                            a[3] += ry * p2 - rz * p1; a[4] += rz * p0 - rx * p2; a[5] += rx * p1 - ry * p0;
                            a[6] += i0; a[7] += i1; a[8] += i2;
                            a[9] += ry * i2 - rz * i1; a[10] += rz * i0 - rx * i2; a[11] += rx * i1 - ry * i0;
                        }
                    });
                }
            }
            res[j][0] = nx;
            res[j][1] = ny;
            res[j][2] = nz;
        }
    }
    __syncthreads();
    // forward input: column r holds (Nx, Ny) of row r; column RW + r/2 holds Nz of rows (2q, 2q+1)
#pragma unroll
    for (int j = 0; j < PP; ++j) {
        const int idx = tid + j * NT;
        if (idx < RW * N) {
            const int r = idx / N, i = idx % N;
            buf[r * SC + i] = cx<T>{res[j][0], res[j][1]};
            T* zc = reinterpret_cast<T*>(buf + (RW + r / 2) * SC + i);
            zc[r & 1] = res[j][2];
        }
    }
    fft_lds<T, N, -1, CF, NT, 1, SC>(buf, tw);

    // 3. split the packed spectra and store kx = 0..K
#pragma unroll
    for (int f = 0; f < 3; ++f) {
        cx<T>* O = xout + f * fs_out + (long)row0 * KP;
        for (int idx = tid; idx < RW * KP; idx += NT) {
            const int r = idx / KP, k = idx % KP;
            const int colx = (f < 2) ? r : RW + r / 2;
            const bool second = (f == 1) || (f == 2 && (r & 1));
            const cx<T> zk = buf[colx * SC + k];
            const cx<T> zm = buf[colx * SC + ((N - k) % N)];
            cx<T> v;
            if (!second) {
                v = cx<T>{T(0.5) * (zk.x + zm.x), T(0.5) * (zk.y - zm.y)};
            } else {
                const T dxr = zk.x - zm.x, dyi = zk.y + zm.y;  // zk - conj(zm)
                v = cx<T>{T(0.5) * dyi, T(-0.5) * dxr};
            }
            O[idx] = v;
        }
    }
    block_reduce_store<NVAL>(acc, red, partial + (long)blockIdx.x * NV);
}

// ---------------------------------------------------------------------------
// Scalar step: reduction of the x-pass partial sums (two fixed-order levels,
// the last workgroup to finish does the second level), then dt, force,
// torque, energy, AB2 weights, time advance and the kinematics of the new
// time level.
// ---------------------------------------------------------------------------
__device__ inline void finish_step(const double* tot, StateHdr* h, const flusi_insect& ins, const StepCtl& ctl,
                                   double dx, double eta, double* history) {
    const double dV = dx * dx * dx;
    const double umax = sqrt(tot[0]);
    const double E = 0.5 * tot[1] * dV;
    if (tot[2] != 0.0 || !isfinite(E) || !isfinite(umax)) {
        h->status = FLUSI_ENONFINITE;
        h->active = 0;
        return;
    }
    const double t = h->t;
    double dt;
    if (ctl.dt_fixed > 0.0) {
        dt = ctl.dt_fixed;
    } else {
        dt = umax > 0.0 ? ctl.cfl * dx / umax : INFINITY;
        if (ctl.masked) dt = fmin(dt, ctl.eta_cap * eta);
        if (ctl.dt_max > 0.0) dt = fmin(dt, ctl.dt_max);
    }
    if (ctl.t_end > 0.0 && t + dt > ctl.t_end) dt = ctl.t_end - t;
    if (!isfinite(dt)) {
        h->status = FLUSI_EINVAL;
        h->active = 0;
        return;
    }
    double* d = h->diag;
    d[0] = t;
    d[1] = dt;
    d[2] = umax;
    d[3] = E;
    for (int c = 0; c < 3; ++c) {
        const double* a = tot + 3 + 12 * c;
        for (int i = 0; i < 6; ++i) {
            double v = a[i] * dV / eta;
            if (h->have_I && h->dt_prev > 0.0) v += (a[6 + i] * dV - h->I_prev[c][i]) / h->dt_prev;
            d[4 + 6 * c + i] = v;
        }
    }
    if (history)
        for (int i = 0; i < FLUSI_NDIAG; ++i) history[i] = d[i];
    if (!(dt > 0.0)) {  // end time reached: leave the state as it is
        h->active = 0;
        return;
    }
    h->active = 1;
    h->first = h->have_prev ? 0 : 1;
    h->dt = dt;
    h->dtp = h->dt_prev;
    if (h->have_prev) {
        const double r = dt / h->dt_prev;
        h->b1 = 1.0 + 0.5 * r;
        h->b2 = -0.5 * r;
    } else {
        h->b1 = 1.0;
        h->b2 = 0.0;
    }
    if (ctl.masked) {
        for (int c = 0; c < 3; ++c)
            for (int i = 0; i < 6; ++i) h->I_prev[c][i] = tot[3 + 12 * c + 6 + i] * dV;
        h->have_I = 1;
    }
    h->have_prev = 1;
    h->dt_prev = dt;
    h->t = t + dt;
    h->n += 1;
    if (ctl.masked) compute_kin(ins, h->t, dx, h->kin);
}

static __global__ __launch_bounds__(NT) void k_scalar(const double* __restrict__ partial, int nwg, double* partial2,
                                               unsigned* counter, StateHdr* hdr, flusi_insect ins, StepCtl ctl,
                                               double dx, double eta, double* history) {
    __shared__ double red[NT / 64][NV];
    __shared__ double tot[NV];
    __shared__ unsigned ticket;
    if (hdr->status) return;
    const int tid = threadIdx.x;
    const int chunk = (nwg + NRED_BLOCKS - 1) / NRED_BLOCKS;
    const int lo = blockIdx.x * chunk, hi = min(nwg, lo + chunk);
    double acc[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) acc[v] = 0.0;
    for (int w = lo + tid; w < hi; w += NT) {
        const double* p = partial + (long)w * NV;
#pragma unroll
        for (int v = 0; v < NV; ++v) acc[v] = (v == 0 || v == 2) ? fmax(acc[v], p[v]) : acc[v] + p[v];
    }
    block_reduce_store<NV>(acc, red, partial2 + (long)blockIdx.x * NV);
    __threadfence();
    __syncthreads();
    if (tid == 0) ticket = atomicAdd(counter, 1u);
    __syncthreads();
    if (ticket != NRED_BLOCKS - 1) return;
    __threadfence();
    if (tid < NV) {
        double r = __hip_atomic_load(partial2 + tid, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        for (int b = 1; b < NRED_BLOCKS; ++b) {
            const double x = __hip_atomic_load(partial2 + (long)b * NV + tid, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            r = (tid == 0 || tid == 2) ? fmax(r, x) : r + x;
        }
        tot[tid] = r;
    }
    __syncthreads();
    if (tid == 0) {
        finish_step(tot, hdr, ins, ctl, dx, eta, history);
        atomicExch(counter, 0u);
    }
}

// Kinematics of the current time level of a state (start of each stepping call).
static __global__ void k_prologue(StateHdr* hdr, flusi_insect ins, double dx) {
    if (threadIdx.x == 0 && blockIdx.x == 0) compute_kin(ins, hdr->t, dx, hdr->kin);
}

static __global__ void k_hdr_init(StateHdr* hdr, double t0) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        StateHdr h;
        unsigned char* b = reinterpret_cast<unsigned char*>(&h);
        for (size_t i = 0; i < sizeof(StateHdr); ++i) b[i] = 0;
        h.t = t0;
        *hdr = h;
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
enum { MODE_IMPORT = 0, MODE_STEP = 1, MODE_STEP_LAST = 2, MODE_INVERSE = 3 };

template <typename T, int N, int MODE>
__global__ __launch_bounds__(NT) void k_zpass(const cx<T>* __restrict__ yin, long fs_y, cx<T>* uhat, cx<T>* nold,
                                              long fs_s, cx<T>* __restrict__ zout, long fs_z,
                                              const cx<T>* __restrict__ tw, const StateHdr* __restrict__ hdr,
                                              double kscale, double nu, int mean_mode) {
    constexpr int K = kmax_of(N), KP = K + 1, M = 2 * K + 1, Q = M * KP;
    constexpr int C = cols_of(N);
    static_assert(NT % C == 0, "column mapping");
    constexpr int PERM = (M * C + NT - 1) / NT;
    __shared__ cx<T> buf[C * N];
    if (hdr->status) return;
    const int tid = threadIdx.x;
    const int c = tid % C;
    const int q = blockIdx.x * C + c;
    const bool okq = q < Q;
    const int kxi = q % KP, myi = q / KP;
    const double kxv = kscale * kxi;
    const double kyv = kscale * j_of_m(myi, K);

    const bool step_mode = (MODE == MODE_STEP || MODE == MODE_STEP_LAST);
    const bool active = step_mode ? (hdr->active != 0) : true;
    const bool do_fwd = (MODE == MODE_IMPORT) || (step_mode && active);
    const bool do_inv = (MODE == MODE_STEP) || (MODE == MODE_INVERSE);

    cx<T> U[3][PERM];
    if (do_fwd) {
        cx<T> Nh[3][PERM];
#pragma unroll
        for (int f = 0; f < 3; ++f) {
            for (int n = tid / C; n < N; n += NT / C)
                buf[n * C + c] = okq ? yin[f * fs_y + (long)n * Q + q] : cx<T>{T(0), T(0)};
            fft_lds<T, N, -1, C, NT, C, 1>(buf, tw);
#pragma unroll
            for (int i = 0; i < PERM; ++i) {
                const int m = tid / C + i * (NT / C);
                if (m < M) Nh[f][i] = buf[bin_of_m(m, N, K) * C + c];
            }
            __syncthreads();
        }
        double dt = 0, b1 = 0, b2 = 0, dtp = 0;
        int first = 1;
        if (step_mode) {
            dt = hdr->dt;
            b1 = hdr->b1;
            b2 = hdr->b2;
            dtp = hdr->dtp;
            first = hdr->first;
        }
#pragma unroll
        for (int i = 0; i < PERM; ++i) {
            const int m = tid / C + i * (NT / C);
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
                    const double sr = (kxv * nr[0] + kyv * nr[1] + kzv * nr[2]) / k2;
                    const double si = (kxv * ni[0] + kyv * ni[1] + kzv * ni[2]) / k2;
                    nr[0] -= kxv * sr; nr[1] -= kyv * sr; nr[2] -= kzv * sr;
                    ni[0] -= kxv * si; ni[1] -= kyv * si; ni[2] -= kzv * si;
                } else if (step_mode && mean_mode == FLUSI_MEAN_FIXED) {
                    nr[0] = nr[1] = nr[2] = 0.0;
                    ni[0] = ni[1] = ni[2] = 0.0;
                }
                const long e = (long)m * Q + q;
                if (MODE == MODE_IMPORT) {
#pragma unroll
                    for (int f = 0; f < 3; ++f) {
                        U[f][i] = cx<T>{T(nr[f]), T(ni[f])};
                        uhat[f * fs_s + e] = U[f][i];
                    }
                } else {
                    const double e1 = exp(-nu * k2 * dt);
                    const double e0 = first ? 0.0 : exp(-nu * k2 * dtp);
#pragma unroll
                    for (int f = 0; f < 3; ++f) {
                        const cx<T> uh = uhat[f * fs_s + e];
                        double ar, ai;
                        if (first) {
                            ar = nr[f];
                            ai = ni[f];
                        } else {
                            const cx<T> no = nold[f * fs_s + e];
                            const double c2 = b2 * e0;
                            ar = b1 * nr[f] + c2 * (double)no.x;
                            ai = b1 * ni[f] + c2 * (double)no.y;
                        }
                        const double vr = e1 * ((double)uh.x + dt * ar);
                        const double vi = e1 * ((double)uh.y + dt * ai);
                        U[f][i] = cx<T>{T(vr), T(vi)};
                        uhat[f * fs_s + e] = U[f][i];
                        nold[f * fs_s + e] = cx<T>{T(nr[f]), T(ni[f])};
                    }
                }
            }
        }
    } else if (do_inv) {
#pragma unroll
        for (int i = 0; i < PERM; ++i) {
            const int m = tid / C + i * (NT / C);
            if (m < M && okq) {
                const long e = (long)m * Q + q;
#pragma unroll
                for (int f = 0; f < 3; ++f) U[f][i] = uhat[f * fs_s + e];
            }
        }
    }
    if (!do_inv) return;

    const T kx = T(kxv), ky = T(kyv);
#pragma unroll
    for (int g = 0; g < 6; ++g) {
        for (int idx = tid; idx < C * (N - M); idx += NT) buf[(K + 1 + idx / C) * C + idx % C] = cx<T>{T(0), T(0)};
#pragma unroll
        for (int i = 0; i < PERM; ++i) {
            const int m = tid / C + i * (NT / C);
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
                buf[bin_of_m(m, N, K) * C + c] = v;
            }
        }
        fft_lds<T, N, +1, C, NT, C, 1>(buf, tw);
        if (okq)
            for (int n = tid / C; n < N; n += NT / C) zout[g * fs_z + (long)n * Q + q] = buf[n * C + c];
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
                                              const cx<T>* __restrict__ tw) {
    constexpr int RW = 2 * rows_x(N);  // real rows per workgroup
    constexpr int SC = N + 1;
    constexpr int CP = RW / 2;
    __shared__ cx<T> buf[CP * SC];
    const int tid = threadIdx.x;
    const long row0 = (long)blockIdx.x * RW;
    for (int idx = tid; idx < RW * N; idx += NT) {
        const int r = idx / N, i = idx % N;
        const T v = (row0 + r < nrows) ? in[row0 * N + idx] : T(0);
        reinterpret_cast<T*>(buf + (r / 2) * SC + i)[r & 1] = v;
    }
    fft_lds<T, N, -1, CP, NT, 1, SC>(buf, tw);
    for (int idx = tid; idx < RW * nkx; idx += NT) {
        const int r = idx / nkx, k = idx % nkx;
        if (row0 + r >= nrows) continue;
        const cx<T> zk = buf[(r / 2) * SC + k];
        const cx<T> zm = buf[(r / 2) * SC + ((N - k) % N)];
        cx<T> v;
        if (!(r & 1)) {
            v = cx<T>{T(0.5) * (zk.x + zm.x), T(0.5) * (zk.y - zm.y)};
        } else {
            v = cx<T>{T(0.5) * (zk.y + zm.y), T(-0.5) * (zk.x - zm.x)};
        }
        out[(row0 + r) * nkx + k] = v;
    }
}

template <typename T, int N>
__global__ __launch_bounds__(NT) void k_x_c2r(const cx<T>* __restrict__ in, T* __restrict__ out, long nrows, int nkx,
                                              T scale, const cx<T>* __restrict__ tw) {
    constexpr int RW = 2 * rows_x(N);
    constexpr int SC = N + 1;
    constexpr int CP = RW / 2;
    __shared__ cx<T> buf[CP * SC];
    const int tid = threadIdx.x;
    const long row0 = (long)blockIdx.x * RW;
    for (int idx = tid; idx < CP * N; idx += NT) buf[(idx / N) * SC + idx % N] = cx<T>{T(0), T(0)};
    __syncthreads();
    for (int idx = tid; idx < CP * nkx; idx += NT) {
        const int p = idx / nkx, k = idx % nkx;
        const long ra = row0 + 2 * p, rb = ra + 1;
        const cx<T> a = ra < nrows ? in[ra * nkx + k] : cx<T>{T(0), T(0)};
        const cx<T> b = rb < nrows ? in[rb * nkx + k] : cx<T>{T(0), T(0)};
        cx<T>* col = buf + p * SC;
        if (k == 0 || 2 * k == N) {
            col[k] = cx<T>{a.x, b.x};
        } else {
            col[k] = cx<T>{a.x - b.y, a.y + b.x};
            col[N - k] = cx<T>{a.x + b.y, b.x - a.y};
        }
    }
    fft_lds<T, N, +1, CP, NT, 1, SC>(buf, tw);
    for (int idx = tid; idx < RW * N; idx += NT) {
        const int r = idx / N, i = idx % N;
        if (row0 + r >= nrows) continue;
        const cx<T> z = buf[(r / 2) * SC + i];
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
__global__ void k_mask(const Kin* __restrict__ kin, flusi_insect ins, int n, double dx, T* __restrict__ chi,
                       T* __restrict__ us, int16_t* __restrict__ colour) {
    const long npts = (long)n * n * n;
    const long p = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= npts) return;
    const int i = p % n, j = (p / n) % n, k = p / ((long)n * n);
    const MaskPt mp = eval_mask(*kin, ins, dx * i, dx * j, dx * k);
    if (chi) chi[p] = T(mp.chi);
    if (us) {
        us[p] = T(mp.us[0]);
        us[npts + p] = T(mp.us[1]);
        us[2 * npts + p] = T(mp.us[2]);
    }
    if (colour) colour[p] = (int16_t)mp.colour;
}

static __global__ void k_kin(Kin* kin, flusi_insect ins, double t, double dx) {
    if (threadIdx.x == 0 && blockIdx.x == 0) compute_kin(ins, t, dx, *kin);
}

// Pruned state spectrum [3][M][M][KP] -> full layout [3][n][n][n/2+1] (zeros elsewhere).
template <typename T>
__global__ void k_export_full(const cx<T>* __restrict__ st, cx<T>* __restrict__ out, int n, long fs_s) {
    const int nkx = n / 2 + 1;
    const int K = kmax_of(n), KP = K + 1, M = 2 * K + 1;
    const long tot = (long)n * n * nkx;
    const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= tot) return;
    const int ix = e % nkx, iy = (e / nkx) % n, iz = e / ((long)nkx * n);
    const int my = m_of_bin(iy, n, K), mz = m_of_bin(iz, n, K);
    const bool kept = ix <= K && my >= 0 && mz >= 0;
    for (int f = 0; f < 3; ++f)
        out[f * tot + e] = kept ? st[f * fs_s + ((long)mz * M + my) * KP + ix] : cx<T>{T(0), T(0)};
}

}  // namespace flusi
