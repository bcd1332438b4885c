// 2D acoustic leapfrog, two time steps per launch, for plans with a point
// source or receivers (Sec. 3): the kernels of acoustic2d_tb.h with the
// forcing code compiled in, in a translation unit of their own.
#include "acoustic2d_tb.h"

namespace hw {

hipError_t launch_ac2d_step2_forcing(const Ac2dBatch &a, const Ac2dDesc *one, int storage,
                                     int comp, int order, int tile, hipStream_t s)
{
    return step2_launch<true>(a, one, storage, comp, order, tile, s);
}

}  // namespace hw
