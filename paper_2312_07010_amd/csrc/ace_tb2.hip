// Dispatch to the instantiated variants of the register-resident 2D blocked
// kernel (ace_tb2.h; each variant is compiled in its own translation unit,
// ace_tb2_v<i>.hip, in the order of TB2_TABLE).
#include "ace_internal.h"

namespace ace {

// ---- the register-resident variants (ace_tb2.h, one translation unit each) ----

hipError_t launch_tb2_v0(const Shape &, const StepCoef &, const double *, double *, double *, int64_t *, int,
                         int64_t, hipStream_t);
hipError_t launch_tb2_v1(const Shape &, const StepCoef &, const double *, double *, double *, int64_t *, int,
                         int64_t, hipStream_t);
hipError_t launch_tb2_v2(const Shape &, const StepCoef &, const double *, double *, double *, int64_t *, int,
                         int64_t, hipStream_t);
hipError_t launch_tb2_v3(const Shape &, const StepCoef &, const double *, double *, double *, int64_t *, int,
                         int64_t, hipStream_t);
int64_t tb2_blocks_v0(const Shape &, int);
int64_t tb2_blocks_v1(const Shape &, int);
int64_t tb2_blocks_v2(const Shape &, int);
int64_t tb2_blocks_v3(const Shape &, int);

bool tb2_supported(const Shape &s) { return tblock2d_supported(s) && s.M1 * s.M2 < ((int64_t)1 << 31); }

int tb2_find(int rows, int rpt)
{
    for (int v = 0; v < TB2_VARIANTS; ++v)
        if (TB2_TABLE[v].rows == rows && TB2_TABLE[v].rpt == rpt) return v;
    return -1;
}

hipError_t launch_step_tb2(int v, const Shape &s, const StepCoef &c, const double *in, double *out,
                           double *partials, int64_t *nparts, int K, int64_t level_stride, hipStream_t st)
{
    if (!tb2_supported(s) || v < 0 || v >= TB2_VARIANTS || K < 1 || K > tb2_max_depth(v))
        return hipErrorInvalidValue;
    switch (v) {
    case 0: return launch_tb2_v0(s, c, in, out, partials, nparts, K, level_stride, st);
    case 1: return launch_tb2_v1(s, c, in, out, partials, nparts, K, level_stride, st);
    case 2: return launch_tb2_v2(s, c, in, out, partials, nparts, K, level_stride, st);
    case 3: return launch_tb2_v3(s, c, in, out, partials, nparts, K, level_stride, st);
    default: return hipErrorInvalidValue;
    }
}

int64_t tb2_blocks(int v, const Shape &s, int K)
{
    switch (v) {
    case 0: return tb2_blocks_v0(s, K);
    case 1: return tb2_blocks_v1(s, K);
    case 2: return tb2_blocks_v2(s, K);
    case 3: return tb2_blocks_v3(s, K);
    default: return 0;
    }
}

}  // namespace ace
