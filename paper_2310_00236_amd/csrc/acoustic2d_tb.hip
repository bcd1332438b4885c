// 2D acoustic leapfrog, two time steps per launch: the launches of plans
// without a point source or receivers (the kernels are in acoustic2d_tb.h;
// acoustic2d_tb_var.hip compiles them with the forcing code).
#include "acoustic2d_tb.h"

namespace hw {

hipError_t launch_ac2d_step2(const Ac2dBatch &a, const Ac2dDesc *one, int storage,
                             int comp, int order, int tile, bool forced, hipStream_t s)
{
    if (forced)
        return launch_ac2d_step2_forcing(a, one, storage, comp, order, tile, s);
    return step2_launch<false>(a, one, storage, comp, order, tile, s);
}

}  // namespace hw
