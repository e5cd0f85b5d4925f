// Instantiations of the strict LDS-panel kernel: 16 columns per lane.
#include "strict_kernels.hpp"

namespace afmm {

// (R, C, W, U, KP)
#define AFMM_PART_CONFIGS(X) \
    X(4, 16, 8, 1, 8)       \
    X(4, 16, 8, 2, 8)       \
    X(6, 16, 4, 1, 8)       \
    X(4, 16, 16, 1, 16)     \
    X(4, 16, 16, 2, 16)

// With a == nullptr: is (R, C, W, U, KP) compiled here?  Otherwise launch it.
bool rep_part_a(const StrictArgs* a, int R, int C, int W, int U, int KP, hipStream_t s,
                 hipError_t* err) {
#define AFMM_CASE(r, c, w, u, kp)                                            \
    if (R == r && C == c && W == w && U == u && KP == kp) {                   \
        if (a) *err = launch_rep<r, c, w, u, kp>(*a, s);                     \
        return true;                                                         \
    }
    AFMM_PART_CONFIGS(AFMM_CASE)
#undef AFMM_CASE
    return false;
}

}  // namespace afmm
