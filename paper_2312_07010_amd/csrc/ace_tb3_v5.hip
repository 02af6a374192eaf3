// Instantiation of the configurable 3D blocked kernel (ace_tb3.h): depth
// 4, a 32 x 64 region on 16 wavefronts of 2 rows each.
#include <algorithm>
#include <type_traits>

#include "ace_tb3.h"

namespace ace {

hipError_t launch_tb3_v5(const Shape &s, const StepCoef &c, const double *in, double *out,
                        double *partials, int64_t *nparts, int zchunk, hipStream_t st)
{
    return tb3::launch_any<4, 16, 2, 4>(s, c, in, out, partials, nparts, zchunk, st);
}

int64_t tb3_partials_v5(const Shape &s, int zchunk)
{
    return tb3::partials_needed<4, 16, 2>(s, zchunk);
}

}  // namespace ace
