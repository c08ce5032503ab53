// One grid size per translation unit: compiled with -DFLUSI_N=<n>.
#include "impl.hpp"

#ifndef FLUSI_N
#error "FLUSI_N must be defined"
#endif

#define FLUSI_CAT2(a, b) a##b
#define FLUSI_CAT(a, b) FLUSI_CAT2(a, b)

namespace flusi {
ImplBase* FLUSI_CAT(make_impl_, FLUSI_N)(int dtype) {
    if (dtype == FLUSI_F32) return new Impl<float, FLUSI_N>();
    return new Impl<double, FLUSI_N>();
}
}  // namespace flusi
