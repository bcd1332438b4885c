// Variants of the 2D acoustic step kernel with a point source and receivers
// compiled in (Sec. 3) and with the stencil in the storage format or in
// fp64 (the all-fp16 step of Alg. 1 read literally; App. B).  They run on
// tile shape 0 only; plans without these features use the kernels of
// acoustic2d.hip, which carry none of this code.
#include "acoustic2d_kernels.h"

#pragma clang fp contract(off)

namespace hw {

template <class S, int COMP, int ORDER, int SP>
static hipError_t variant_launch(const Ac2dBatch &a, const Ac2dDesc *one,
                                 hipStream_t s)
{
    static_assert(kTiles2D[0].kind == 0 && kTiles2D[0].tx == 64, "tile 0");
    constexpr int T = kTiles2D[0].ty;
    const dim3 grid(a.total_tiles), block(kThreads);
    if (one) {
        Ac2dOne o;
        o.d = *one;
        o.parity = a.parity[0];
        o.tiles_x = a.tiles_x[0];
        o.total_tiles = a.total_tiles;
        hipLaunchKernelGGL((ac2d_step1_kernel<S, COMP, ORDER, 1, T, true, SP>), grid,
                           block, 0, s, o);
    } else {
        hipLaunchKernelGGL((ac2d_step_kernel<S, COMP, ORDER, 1, T, true, SP>), grid,
                           block, 0, s, a);
    }
    return hipGetLastError();
}

template <class S, int COMP, int ORDER>
static hipError_t variant_sp(const Ac2dBatch &a, const Ac2dDesc *one, int stencil,
                             hipStream_t s)
{
    switch (stencil) {
    case HW_STENCIL_F32: return variant_launch<S, COMP, ORDER, 0>(a, one, s);
    case HW_STENCIL_STORAGE: return variant_launch<S, COMP, ORDER, 1>(a, one, s);
    case HW_STENCIL_F64: return variant_launch<S, COMP, ORDER, 2>(a, one, s);
    }
    return hipErrorInvalidValue;
}

template <class S, int COMP>
static hipError_t variant_order(const Ac2dBatch &a, const Ac2dDesc *one, int order,
                                int stencil, hipStream_t s)
{
    return order == 4 ? variant_sp<S, COMP, 4>(a, one, stencil, s)
                      : variant_sp<S, COMP, 2>(a, one, stencil, s);
}

template <class S>
static hipError_t variant_comp(const Ac2dBatch &a, const Ac2dDesc *one, int comp,
                               int order, int stencil, hipStream_t s)
{
    switch (comp) {
    case COMP_NONE: return variant_order<S, COMP_NONE>(a, one, order, stencil, s);
    case COMP_FAST2SUM: return variant_order<S, COMP_FAST2SUM>(a, one, order, stencil, s);
    case COMP_TWOSUM: return variant_order<S, COMP_TWOSUM>(a, one, order, stencil, s);
    case COMP_TWOSUM8:
        if constexpr (S::id != F32::id)
            return variant_order<S, COMP_TWOSUM8>(a, one, order, stencil, s);
        break;
    }
    return hipErrorInvalidValue;
}

hipError_t launch_ac2d_variant(const Ac2dBatch &a, const Ac2dDesc *one, int format,
                               int comp, int order, int tile, int stencil,
                               hipStream_t s)
{
    if (tile != 0)
        return hipErrorInvalidValue;
    switch (format) {
    case F32::id: return variant_comp<F32>(a, one, comp, order, stencil, s);
    case F16::id: return variant_comp<F16>(a, one, comp, order, stencil, s);
    case BF16::id: return variant_comp<BF16>(a, one, comp, order, stencil, s);
    }
    return hipErrorInvalidValue;
}

}  // namespace hw
