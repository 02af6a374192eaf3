// Instantiation of the configurable 3D blocked kernel (ace_tb3.h): depth
// 3, a 48 x 64 region on 12 wavefronts of 4 rows each.
#include <algorithm>
#include <type_traits>

#include "ace_tb3.h"

namespace ace {

hipError_t launch_tb3_v2(const Shape &s, const StepCoef &c, const double *in, double *out,
                        double *partials, int64_t *nparts, int zchunk, hipStream_t st)
{
    return tb3::launch_any<3, 12, 4, 3>(s, c, in, out, partials, nparts, zchunk, st);
}

int64_t tb3_partials_v2(const Shape &s, int zchunk)
{
    return tb3::partials_needed<3, 12, 4>(s, zchunk);
}

}  // namespace ace
