// Instantiations of the strict LDS-panel kernel: 4 or fewer columns per lane.
#include "strict_kernels.hpp"

namespace afmm {

// (R, C, W, U, KP)
#define AFMM_PART_CONFIGS(X) \
    X(8, 4, 8, 1, 16)       \
    X(8, 4, 8, 2, 16)       \
    X(4, 4, 8, 1, 16)       \
    X(8, 4, 4, 1, 16)       \
    X(8, 4, 4, 2, 16)       \
    X(4, 4, 4, 1, 16)       \
    X(4, 2, 4, 1, 16)       \
    X(4, 2, 4, 2, 16)       \
    X(2, 1, 4, 1, 16)

// With a == nullptr: is (R, C, W, U, KP) compiled here?  Otherwise launch it.
bool rep_part_c(const StrictArgs* a, int R, int C, int W, int U, int KP, hipStream_t s,
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
