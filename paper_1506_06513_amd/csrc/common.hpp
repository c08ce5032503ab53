// Shared device-side types for the pseudo-spectral penalized Navier-Stokes path.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <type_traits>
#include <utility>

namespace flusi {

template <typename T>
struct cx {
    T x, y;
};

// Global-memory views.  A pointer read from memory (a launch table) is
// generic, and generic accesses compile to flat instructions; these typed views
// keep bulk accesses on global instructions.
template <typename T>
using glb = __attribute__((address_space(1))) T;
template <typename T>
__device__ __forceinline__ glb<T>* gview(T* p) { return (glb<T>*)p; }
template <typename T>
__device__ __forceinline__ const glb<T>* gview(const T* p) { return (const glb<T>*)p; }
template <typename T>
__device__ __forceinline__ cx<T> gld(const glb<cx<T>>* p, long i) { return cx<T>{p[i].x, p[i].y}; }
template <typename T>
__device__ __forceinline__ void gst(glb<cx<T>>* p, long i, cx<T> v) {
    p[i].x = v.x;
    p[i].y = v.y;
}

template <typename T>
__device__ __forceinline__ cx<T> mk(T a, T b) { return cx<T>{a, b}; }
template <typename T>
__device__ __forceinline__ cx<T> operator+(cx<T> a, cx<T> b) { return {a.x + b.x, a.y + b.y}; }
template <typename T>
__device__ __forceinline__ cx<T> operator-(cx<T> a, cx<T> b) { return {a.x - b.x, a.y - b.y}; }
template <typename T>
__device__ __forceinline__ cx<T> operator*(cx<T> a, T s) { return {a.x * s, a.y * s}; }
template <typename T>
__device__ __forceinline__ cx<T> cmul(cx<T> a, cx<T> b) {
    return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
// a * conj(b)
template <typename T>
__device__ __forceinline__ cx<T> cmulc(cx<T> a, cx<T> b) {
    return {a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y};
}
template <typename T>
__device__ __forceinline__ cx<T> conj(cx<T> a) { return {a.x, -a.y}; }
// multiply by -i
template <typename T>
__device__ __forceinline__ cx<T> mul_mi(cx<T> a) { return {a.y, -a.x}; }
// multiply by +i
template <typename T>
__device__ __forceinline__ cx<T> mul_pi(cx<T> a) { return {-a.y, a.x}; }

// compile-time loop: f(std::integral_constant<int, I>{}) for I in [0, N)
template <int N, typename F, int... I>
__device__ __forceinline__ void static_for_impl(F&& f, std::integer_sequence<int, I...>) {
    (f(std::integral_constant<int, I>{}), ...);
}
template <int N, typename F>
__device__ __forceinline__ void static_for(F&& f) {
    static_for_impl<N>(f, std::make_integer_sequence<int, N>{});
}

// Number of kept modes per signed axis and on the half axis under the 2/3 rule
// (keep iff 3|j| < n): |j| <= K with K = (n - 1) / 3.
__host__ __device__ constexpr int kmax_of(int n) { return (n - 1) / 3; }

// Signed storage index m in [0, 2K] <-> wavenumber j in [-K, K].
__host__ __device__ constexpr int j_of_m(int m, int K) { return m <= K ? m : m - (2 * K + 1); }
// FFT bin n in [0, N) of a signed axis -> pruned index, or -1 when the bin is dealiased away.
__host__ __device__ constexpr int m_of_bin(int n, int N, int K) {
    return n <= K ? n : (n >= N - K ? n - N + 2 * K + 1 : -1);
}
// pruned index m -> FFT bin
__host__ __device__ constexpr int bin_of_m(int m, int N, int K) { return m <= K ? m : m - (2 * K + 1) + N; }

}  // namespace flusi
