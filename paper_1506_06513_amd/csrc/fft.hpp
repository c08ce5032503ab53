// Register/LDS mixed-radix FFT machinery for gfx950.
//
// A workgroup transforms columns of length N held in padded column-major LDS.
// Each stage of radix R (Stockham, decimation in time, auto-sorting) reads R
// elements with stride N/R into registers, applies the inter-stage twiddles
// from an FP64-accurate table, performs an R-point DFT in registers (R in
// {2,3,4,6,8,12,16}) and writes the R results back in place.  A column is
// owned by one group of lanes of one wavefront for all stages, so the stages
// synchronize at wavefront level only.  The output is in natural order.  The forward transform uses exp(-2 pi i nk/N), the inverse
// exp(+2 pi i nk/N), both unnormalized.
#pragma once
#include "common.hpp"

namespace flusi {

// ---------------------------------------------------------------------------
// Radix plans (product = N).  Every radix of a plan divides E = fft_E(N), the
// number of elements a lane holds, so that a column is always owned by the
// same G = N/E lanes of one wavefront.
// ---------------------------------------------------------------------------
__host__ __device__ constexpr int fft_nstages(int N) {
    switch (N) {
        case 16: return 1;
        case 24: case 32: case 64: case 96: case 128: case 256: return 2;
        case 48: case 192: case 384: case 512: case 768: case 1024: return 3;
        case 1152: return 4;
        default: return 0;
    }
}
__host__ __device__ constexpr int fft_radix(int N, int s) {
    switch (N) {
        case 16: return 16;
        case 24: return s == 0 ? 8 : 3;
        case 32: return s == 0 ? 8 : 4;
        case 48: return s == 2 ? 3 : 4;
        case 64: return 8;
        case 96: return s == 0 ? 8 : 12;
        case 128: return s == 0 ? 8 : 16;
        case 192: return s == 2 ? 3 : 8;
        case 256: return 16;
        case 384: return s == 2 ? 6 : 8;
        case 512: return 8;
        case 768: return s == 2 ? 12 : 8;
        case 1024: return s == 2 ? 4 : 16;
        case 1152: return s < 2 ? 12 : (s == 2 ? 4 : 2);
        default: return 1;
    }
}
// elements per lane: a multiple of every radix (their least common multiple,
// or a multiple of it where that leaves more than 64 lanes per column)
__host__ __device__ constexpr int fft_E(int N) {
    switch (N) {
        case 16: return 16;
        case 24: return 24;
        case 32: return 8;
        case 48: return 12;
        case 64: return 8;
        case 96: return 24;
        case 128: return 16;
        case 192: return 24;
        case 256: return 16;
        case 384: return 24;
        case 512: return 8;
        case 768: return 24;
        case 1024: return 16;
        case 1152: return 36;  // a multiple of 12 whose lane count divides 64
        default: return 1;
    }
}
// lanes per column
__host__ __device__ constexpr int fft_G(int N) { return N / fft_E(N); }
__host__ __device__ constexpr int fft_prefix(int N, int s) {
    int p = 1;
    for (int i = 0; i < s; ++i) p *= fft_radix(N, i);
    return p;
}
__host__ __device__ constexpr bool fft_supported(int N) {
    if (fft_nstages(N) == 0 || fft_prefix(N, fft_nstages(N)) != N) return false;
    for (int i = 0; i < fft_nstages(N); ++i)
        if (fft_E(N) % fft_radix(N, i) != 0) return false;
    return 64 % fft_G(N) == 0;
}

// ---------------------------------------------------------------------------
// Exact small-radix twiddles: cos/sin of multiples of 2 pi / 48 (R | 48)
// ---------------------------------------------------------------------------
// cos(r * 7.5 deg) for the r that radices 2,3,4,6,8,12,16 need (r in 0..12)
__host__ __device__ constexpr double cos_q(int r) {
    switch (r) {
        case 0: return 1.0;
        case 3: return 0.92387953251128675612818318939678828682;   // 22.5 deg
        case 4: return 0.86602540378443864676372317075293618347;   // 30 deg
        case 6: return 0.70710678118654752440084436210484903928;   // 45 deg
        case 8: return 0.5;                                        // 60 deg
        case 9: return 0.38268343236508977172845998403039886676;   // 67.5 deg
        case 12: return 0.0;                                       // 90 deg
        default: return 2.0;  // not needed by any supported radix
    }
}
// cos and sin of a * 7.5 deg, a in [0, 48)
__host__ __device__ constexpr double cos48(int a) {
    const int q = a / 12, r = a % 12;
    return q == 0 ? cos_q(r) : q == 1 ? -cos_q(12 - r) : q == 2 ? -cos_q(r) : cos_q(12 - r);
}
__host__ __device__ constexpr double sin48(int a) {
    const int q = a / 12, r = a % 12;
    return q == 0 ? cos_q(12 - r) : q == 1 ? cos_q(r) : q == 2 ? -cos_q(12 - r) : -cos_q(r);
}

// v * exp(DIR * 2 pi i M / R) with DIR = -1 forward, +1 inverse; trivial angles
// are applied as sign changes / swaps.
template <int R, int M, int DIR, typename T>
__device__ __forceinline__ cx<T> twc(cx<T> v) {
    constexpr int a = ((M % R) * (48 / R)) % 48;
    if constexpr (a == 0) {
        return v;
    } else if constexpr (a == 24) {
        return {-v.x, -v.y};
    } else if constexpr (a == 12) {
        return DIR < 0 ? mul_mi(v) : mul_pi(v);
    } else if constexpr (a == 36) {
        return DIR < 0 ? mul_pi(v) : mul_mi(v);
    } else {
        constexpr double c = cos48(a);
        constexpr double s = DIR < 0 ? -sin48(a) : sin48(a);
        return cmul(v, cx<T>{T(c), T(s)});
    }
}

// ---------------------------------------------------------------------------
// R-point DFTs in registers
// ---------------------------------------------------------------------------
template <int R, int DIR, typename T>
struct Dft;

template <int DIR, typename T>
struct Dft<1, DIR, T> {
    __device__ __forceinline__ static void run(cx<T>*) {}
};

template <int DIR, typename T>
struct Dft<2, DIR, T> {
    __device__ __forceinline__ static void run(cx<T>* v) {
        const cx<T> a = v[0], b = v[1];
        v[0] = a + b;
        v[1] = a - b;
    }
};

template <int DIR, typename T>
struct Dft<3, DIR, T> {
    __device__ __forceinline__ static void run(cx<T>* v) {
        constexpr T h = T(0.5);
        constexpr T s3 = T(0.86602540378443864676372317075293618347);
        const cx<T> s = v[1] + v[2];
        const cx<T> d = v[1] - v[2];
        const cx<T> m = v[0] - s * h;
        // forward: X1 = m - i s3 d, X2 = m + i s3 d
        const cx<T> r = (DIR < 0) ? mul_mi(d * s3) : mul_pi(d * s3);
        v[0] = v[0] + s;
        v[1] = m + r;
        v[2] = m - r;
    }
};

template <int DIR, typename T>
struct Dft<4, DIR, T> {
    __device__ __forceinline__ static void run(cx<T>* v) {
        const cx<T> a = v[0] + v[2], b = v[0] - v[2];
        const cx<T> c = v[1] + v[3], d = v[1] - v[3];
        const cx<T> e = (DIR < 0) ? mul_mi(d) : mul_pi(d);
        v[0] = a + c;
        v[2] = a - c;
        v[1] = b + e;
        v[3] = b - e;
    }
};

// R = P*Q: n = Q n1 + n2, k = k1 + P k2.
template <int P, int Q, int DIR, typename T>
struct DftPQ {
    __device__ __forceinline__ static void run(cx<T>* v) {
        constexpr int R = P * Q;
        cx<T> y[Q][P];
        static_for<Q>([&](auto n2c) {
            constexpr int n2 = decltype(n2c)::value;
            cx<T> a[P];
            static_for<P>([&](auto n1c) { a[decltype(n1c)::value] = v[Q * decltype(n1c)::value + n2]; });
            Dft<P, DIR, T>::run(a);
            static_for<P>([&](auto k1c) {
                constexpr int k1 = decltype(k1c)::value;
                y[n2][k1] = twc<R, n2 * k1, DIR>(a[k1]);
            });
        });
        static_for<P>([&](auto k1c) {
            constexpr int k1 = decltype(k1c)::value;
            cx<T> b[Q];
            static_for<Q>([&](auto n2c) { b[decltype(n2c)::value] = y[decltype(n2c)::value][k1]; });
            Dft<Q, DIR, T>::run(b);
            static_for<Q>([&](auto k2c) { v[k1 + P * decltype(k2c)::value] = b[decltype(k2c)::value]; });
        });
    }
};

template <int DIR, typename T>
struct Dft<6, DIR, T> : DftPQ<2, 3, DIR, T> {};
template <int DIR, typename T>
struct Dft<8, DIR, T> : DftPQ<2, 4, DIR, T> {};
template <int DIR, typename T>
struct Dft<12, DIR, T> : DftPQ<4, 3, DIR, T> {};
template <int DIR, typename T>
struct Dft<16, DIR, T> : DftPQ<4, 4, DIR, T> {};

// Padded column-major LDS: element n of column c at c*SC + n + n/16 (one pad
// slot every 16 elements keeps the stride-R Stockham writes off a single bank).
template <bool CM, int SN, int SC>
__device__ __forceinline__ int lds_at(int n, int c) {
    static_assert(CM, "only the column-major layout is used");
    return c * SC + n + (n >> 4);
}
// column stride of a padded column-major buffer
__host__ __device__ constexpr int cm_stride(int N) { return N + N / 16 + 1; }

// ---------------------------------------------------------------------------
// One column per group of G = N/E lanes of a wavefront, in padded column-major
// LDS (element n at col[n + n/16]).  Lane l of the group handles butterflies
// b = l + j*G of every stage, so a column never leaves its wavefront and the
// stages only need wavefront-level ordering: LDS operations of one wavefront
// complete in program order.  Callers stage data and block-synchronize before
// and after.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}
__device__ __forceinline__ int cpad(int n) { return n + (n >> 4); }

template <typename T, int N, int DIR, int S>
__device__ __forceinline__ void fft_col_stage(cx<T>* col, int l, const cx<T>* __restrict__ tw) {
    constexpr int E = fft_E(N), G = N / E;
    constexpr int R = fft_radix(N, S);
    constexpr int Ns = fft_prefix(N, S);
    constexpr int NBC = N / R;
    constexpr int J = E / R;  // butterflies per lane
    constexpr int TWS = N / (Ns * R);
    cx<T> v[J][R];
    static_for<J>([&](auto jc) {
        constexpr int j = decltype(jc)::value;
        const int b = l + j * G;
        static_for<R>([&](auto rc) {
            constexpr int r = decltype(rc)::value;
            v[j][r] = col[cpad(b + r * NBC)];
        });
        if constexpr (Ns > 1) {
            const int k = b % Ns;
            static_for<R - 1>([&](auto rc) {
                constexpr int r = decltype(rc)::value + 1;
                const cx<T> wv = tw[k * r * TWS];
                v[j][r] = (DIR < 0) ? cmul(v[j][r], wv) : cmulc(v[j][r], wv);
            });
        }
        Dft<R, DIR, T>::run(v[j]);
    });
    wave_sync();
    static_for<J>([&](auto jc) {
        constexpr int j = decltype(jc)::value;
        const int b = l + j * G;
        const int ob = (b / Ns) * Ns * R + b % Ns;
        static_for<R>([&](auto rc) {
            constexpr int r = decltype(rc)::value;
            col[cpad(ob + r * Ns)] = v[j][r];
        });
    });
    wave_sync();
}

template <typename T, int N, int DIR>
__device__ __forceinline__ void fft_col(cx<T>* col, int l, const cx<T>* __restrict__ tw) {
    static_assert(fft_supported(N), "unsupported FFT length");
    static_for<fft_nstages(N)>([&](auto sc) { fft_col_stage<T, N, DIR, decltype(sc)::value>(col, l, tw); });
}

// Transform columns 0..C-1 of a padded column-major buffer (column stride SC)
// with NT threads; every lane group loops over its columns.
template <typename T, int N, int DIR, int C, int NT, int SC>
__device__ __forceinline__ void fft_cols(cx<T>* buf, const cx<T>* __restrict__ tw) {
    constexpr int G = fft_G(N);
    static_assert(NT % 64 == 0, "whole wavefronts");
    const int l = threadIdx.x % G;
    __syncthreads();
    // all lanes of a wavefront run the same number of iterations
    for (int c0 = 0; c0 < C; c0 += NT / G) {
        const int c = c0 + threadIdx.x / G;
        if (c < C) fft_col<T, N, DIR>(buf + c * SC, l, tw);
    }
    __syncthreads();
}

}  // namespace flusi
