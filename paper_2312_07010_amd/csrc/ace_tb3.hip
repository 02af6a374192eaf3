// Dispatch to the instantiated variants of the configurable 3D blocked kernel
// (ace_tb3.h; each variant is compiled in its own translation unit,
// ace_tb3_v<i>.hip, in the order of TB3_TABLE).
#include "ace_internal.h"

namespace ace {

// ---- the configurable variants (ace_tb3.h, one translation unit each) ------

hipError_t launch_tb3_v0(const Shape &, const StepCoef &, const double *, double *, double *, int64_t *,
                         int, hipStream_t);
hipError_t launch_tb3_v1(const Shape &, const StepCoef &, const double *, double *, double *, int64_t *,
                         int, hipStream_t);
hipError_t launch_tb3_v2(const Shape &, const StepCoef &, const double *, double *, double *, int64_t *,
                         int, hipStream_t);
hipError_t launch_tb3_v3(const Shape &, const StepCoef &, const double *, double *, double *, int64_t *,
                         int, hipStream_t);
hipError_t launch_tb3_v4(const Shape &, const StepCoef &, const double *, double *, double *, int64_t *,
                         int, hipStream_t);
hipError_t launch_tb3_v5(const Shape &, const StepCoef &, const double *, double *, double *, int64_t *,
                         int, hipStream_t);
int64_t tb3_partials_v0(const Shape &, int);
int64_t tb3_partials_v1(const Shape &, int);
int64_t tb3_partials_v2(const Shape &, int);
int64_t tb3_partials_v3(const Shape &, int);
int64_t tb3_partials_v4(const Shape &, int);
int64_t tb3_partials_v5(const Shape &, int);

bool tb3_supported(const Shape &s)
{
    // (in-plane byte offsets and the output buffers are 32-bit: planes below 2^31 bytes)
    return s.d == 3 && s.M0 >= 1 && s.M1 >= 1 && s.M2 >= 1 && s.M1 * s.M2 < ((int64_t)1 << 28);
}

int tb3_find(int depth, int rows, int rpt)
{
    for (int v = 0; v < TB3_VARIANTS; ++v)
        if (TB3_TABLE[v].depth == depth && TB3_TABLE[v].rows == rows && TB3_TABLE[v].rpt == rpt) return v;
    return -1;
}

hipError_t launch_step_tb3(int v, const Shape &s, const StepCoef &c, const double *in, double *out,
                           double *partials, int64_t *nparts, int zchunk, hipStream_t st)
{
    if (!tb3_supported(s) || zchunk < 0) return hipErrorInvalidValue;
    switch (v) {
    case 0: return launch_tb3_v0(s, c, in, out, partials, nparts, zchunk, st);
    case 1: return launch_tb3_v1(s, c, in, out, partials, nparts, zchunk, st);
    case 2: return launch_tb3_v2(s, c, in, out, partials, nparts, zchunk, st);
    case 3: return launch_tb3_v3(s, c, in, out, partials, nparts, zchunk, st);
    case 4: return launch_tb3_v4(s, c, in, out, partials, nparts, zchunk, st);
    case 5: return launch_tb3_v5(s, c, in, out, partials, nparts, zchunk, st);
    default: return hipErrorInvalidValue;
    }
}

int64_t tb3_partials_needed(int v, const Shape &s, int zchunk)
{
    switch (v) {
    case 0: return tb3_partials_v0(s, zchunk);
    case 1: return tb3_partials_v1(s, zchunk);
    case 2: return tb3_partials_v2(s, zchunk);
    case 3: return tb3_partials_v3(s, zchunk);
    case 4: return tb3_partials_v4(s, zchunk);
    case 5: return tb3_partials_v5(s, zchunk);
    default: return 0;
    }
}

}  // namespace ace
