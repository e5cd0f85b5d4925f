// Strict AFMM entry points: configuration lookup over the instantiation units,
// and the direct-load variant.
#include "strict_kernels.hpp"

namespace afmm {

bool rep_part_a(const StrictArgs* a, int R, int C, int W, int U, int KP, hipStream_t s,
                hipError_t* err);
bool rep_part_b(const StrictArgs* a, int R, int C, int W, int U, int KP, hipStream_t s,
                hipError_t* err);
bool rep_part_c(const StrictArgs* a, int R, int C, int W, int U, int KP, hipStream_t s,
                hipError_t* err);

bool rep_uniform_supported(int R, int C, int W, int U, int KP) {
    return rep_part_a(nullptr, R, C, W, U, KP, nullptr, nullptr) ||
           rep_part_b(nullptr, R, C, W, U, KP, nullptr, nullptr) ||
           rep_part_c(nullptr, R, C, W, U, KP, nullptr, nullptr);
}

hipError_t launch_rep_uniform(const StrictArgs& a, int R, int C, int W, int U, int KP,
                              hipStream_t s) {
    hipError_t e = hipErrorInvalidValue;
    if (rep_part_a(&a, R, C, W, U, KP, s, &e) || rep_part_b(&a, R, C, W, U, KP, s, &e) ||
        rep_part_c(&a, R, C, W, U, KP, s, &e))
        return e;
    return hipErrorInvalidValue;
}

#define AFMM_DIRECT_CONFIGS(X) \
    X(8, 8, 4)                 \
    X(4, 8, 8)                 \
    X(16, 4, 4)

bool rep_direct_supported(int R, int C, int W) {
#define AFMM_CASE(r, c, w) \
    if (R == r && C == c && W == w) return true;
    AFMM_DIRECT_CONFIGS(AFMM_CASE)
#undef AFMM_CASE
    return false;
}

bool rep_direct_usable(const StrictArgs& a) {
    return (a.ldq % 4 == 0) && (a.n_c % 4 == 0 || a.q_padded) &&
           (reinterpret_cast<uintptr_t>(a.Q) % 16 == 0);
}

hipError_t launch_rep_direct(const StrictArgs& a, int R, int C, int W, hipStream_t s) {
#define AFMM_CASE(r, c, w) \
    if (R == r && C == c && W == w) return launch_direct<r, c, w>(a, s);
    AFMM_DIRECT_CONFIGS(AFMM_CASE)
#undef AFMM_CASE
    return hipErrorInvalidValue;
}

}  // namespace afmm
