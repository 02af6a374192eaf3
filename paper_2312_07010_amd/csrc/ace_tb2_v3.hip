// Instantiation of the register-resident 2D blocked kernel (ace_tb2.h): a
// 16 x 64 region on 8 wavefronts of 2 rows each.
#include <type_traits>

#include "ace_tb2.h"

namespace ace {

hipError_t launch_tb2_v3(const Shape &s, const StepCoef &c, const double *in, double *out,
                        double *partials, int64_t *nparts, int K, int64_t level_stride, hipStream_t st)
{
    return tb2::launch_any<8, 2>(s, c, in, out, partials, nparts, K, level_stride, st);
}

int64_t tb2_blocks_v3(const Shape &s, int K)
{
    int tx, n;
    tb2::tiles<8, 2>(s, K, tx, n);
    return n;
}

}  // namespace ace
