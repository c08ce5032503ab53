// One grid per translation unit: compiled with -DFLUSI_N=<n> for the cubic
// n^3 grid, and with -DFLUSI_NX=<nx> as well for an nx x n x n box.
#include "impl.hpp"

#ifndef FLUSI_N
#error "FLUSI_N must be defined"
#endif

#define FLUSI_CAT2(a, b) a##b
#define FLUSI_CAT(a, b) FLUSI_CAT2(a, b)

namespace flusi {
#ifdef FLUSI_NX
ImplBase* FLUSI_CAT(FLUSI_CAT(FLUSI_CAT(make_impl_, FLUSI_NX), _), FLUSI_N)(int dtype) {
    if (dtype == FLUSI_F32) return new Impl<float, FLUSI_NX, FLUSI_N>();
    return new Impl<double, FLUSI_NX, FLUSI_N>();
}
#else
ImplBase* FLUSI_CAT(make_impl_, FLUSI_N)(int dtype) {
    if (dtype == FLUSI_F32) return new Impl<float, FLUSI_N, FLUSI_N>();
    return new Impl<double, FLUSI_N, FLUSI_N>();
}
#endif
}  // namespace flusi
