// 2D acoustic leapfrog step and energy kernels for gfx950.
//
// One launch advances every shot of a batch by one full leapfrog step
// (Sec. 3; Alg. 1 or Alg. 2 of Sec. 4) in a single pass over HBM.  Two
// kernel shapes are compiled (the autotuner picks per problem):
//   tile:  a workgroup owns a TX x TY tile; it issues every global load of
//          the tile at once (old pressure with a halo of 2R-1 cells and
//          buoyancy with a halo of R into LDS, velocity words of the tile
//          plus the R-cell halo, kappa), computes the new velocities of its
//          cells and of the halo its pressure stencil needs (recomputed
//          redundantly from old values, so no grid-wide barrier), keeps them
//          in LDS, then computes the new pressure;
//   march: a workgroup walks down a strip with LDS ring buffers, prefetching
//          the next rows while computing the current ones.
// Fields ping-pong between two sets; with compensation each field value
// sits next to its compensation term in one word.  Every arithmetic
// operation matches the op-by-op definition the CPU reference uses, so
// results are bit-identical to it and independent of the kernel shape and
// of the batch a shot runs in.
#include "acoustic2d_kernels.h"

#pragma clang fp contract(off)

namespace hw {

// One-thread kernels that advance the device step counters of the plans of
// a launch (after their step) and set one counter.
__global__ void tick_kernel(const StepCounters c)
{
    const int i = threadIdx.x;
    if (i < c.n)
        c.c[i][0] += c.by;
}

__global__ void set_counter_kernel(int64_t *c, int64_t v)
{
    if (threadIdx.x == 0)
        *c = v;
}

__device__ __forceinline__ double block_sum(double v, double *red)
{
    return block_sum_f64<kThreads>(v, red);
}

// Energy of the state, one workgroup per grid row (each XCD takes a
// contiguous band of rows): per-cell terms in fp64
// (v^{n+1/2} recomputed in fp64 from the stored state), summed in an order
// that depends only on the grid size.
template <class S, int ORDER>
__global__ __launch_bounds__(kThreads) void ac2d_energy_kernel(
    const Ac2dDesc *__restrict__ dd, int par, int st, double *__restrict__ partial)
{
    using T = typename S::store_t;
    __shared__ double red[kThreads];
    const Ac2dDesc &d = *dd;
    const int64_t nx = d.nx, ny = d.ny, pitch = d.pitch;
    const int64_t j = xcd_band<kNumXcd>(blockIdx.x, gridDim.x);
    const int64_t j1 = wrap1(j + 1, ny);
    const int64_t j2 = wrapn(j + 2, ny);
    const int64_t jm = wrap1(j - 1, ny);
    const T *__restrict__ p = (const T *)d.p[par];   // element stride st
    const T *__restrict__ vx = (const T *)d.vx[par];
    const T *__restrict__ vy = (const T *)d.vy[par];
    const double w1 = d.w1, w2 = d.w2;
    double acc = 0.0;
    for (int64_t i = threadIdx.x; i < nx; i += kThreads) {
        const int64_t i1 = wrap1(i + 1, nx);
        const int64_t q = j * pitch + i;
        const double pc = S::load(p[(q) * st]);
        double gx = w1 * ((double)S::load(p[(j * pitch + i1) * st]) - pc);
        double gy = w1 * ((double)S::load(p[(j1 * pitch + i) * st]) - pc);
        if constexpr (ORDER == 4) {
            const int64_t i2 = wrapn(i + 2, nx), im = wrap1(i - 1, nx);
            gx = gx + w2 * ((double)S::load(p[(j * pitch + i2) * st]) -
                            (double)S::load(p[(j * pitch + im) * st]));
            gy = gy + w2 * ((double)S::load(p[(j2 * pitch + i) * st]) -
                            (double)S::load(p[(jm * pitch + i) * st]));
        }
        const double bc = d.b[q];
        const double bx = 0.5 * (bc + (double)d.b[j * pitch + i1]);
        const double by = 0.5 * (bc + (double)d.b[j1 * pitch + i]);
        const double vxm = S::load(vx[(q) * st]);
        const double vym = S::load(vy[(q) * st]);
        const double vxp = vxm + bx * gx;
        const double vyp = vym + by * gy;
        double e = (pc * pc) / (double)d.k[q] + (vxm * vxp) / bx;
        e = e + (vym * vyp) / by;
        acc += e;
    }
    const double s = block_sum(acc, red);
    if (threadIdx.x == 0)
        partial[j] = s;
}

__global__ __launch_bounds__(kThreads) void energy_finish_kernel(
    const double *__restrict__ partial, int64_t n, double factor,
    double *__restrict__ out, int32_t *__restrict__ flag)
{
    __shared__ double red[kThreads];
    // four independent chains per thread (element i goes to chain
    // (i / kThreads) % 4), joined in a fixed order
    double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
    int64_t i = threadIdx.x;
    for (; i + 3 * kThreads < n; i += 4 * kThreads) {
        a0 += partial[i];
        a1 += partial[i + kThreads];
        a2 += partial[i + 2 * kThreads];
        a3 += partial[i + 3 * kThreads];
    }
    if (i < n)
        a0 += partial[i];
    if (i + kThreads < n)
        a1 += partial[i + kThreads];
    if (i + 2 * kThreads < n)
        a2 += partial[i + 2 * kThreads];
    const double s = block_sum((a0 + a1) + (a2 + a3), red);
    if (threadIdx.x == 0) {
        const double e = s * factor;
        *out = e;
        if (!isfinite(e))
            *flag = 1;
    }
}

// ------------------------------------------------------------- dispatch --

template <class S, int COMP, int ORDER>
static hipError_t step_tile(const Ac2dBatch &a, const Ac2dDesc *one, int tile,
                            bool forced, int stencil, hipStream_t s)
{
    const dim3 grid(a.total_tiles), block(kThreads), block8(8 * 64);
    Ac2dOne o;
    if (one) {
        o.d = *one;
        o.parity = a.parity[0];
        o.tiles_x = a.tiles_x[0];
        o.total_tiles = a.total_tiles;
    }
    if (forced || stencil != 0)
        return launch_ac2d_variant(a, one, S::id, COMP, ORDER, tile, stencil, s);
    switch (tile) {
#define HW_TILE(n)                                                                \
    case n: {                                                                     \
        constexpr int V = kTiles2D[n].tx / 64, T = kTiles2D[n].ty;                \
        if constexpr (kTiles2D[n].kind == 0) {                                    \
            if (one)                                                              \
                hipLaunchKernelGGL((ac2d_step1_kernel<S, COMP, ORDER, V, T>),     \
                                   grid, block, 0, s, o);                         \
            else                                                                  \
                hipLaunchKernelGGL((ac2d_step_kernel<S, COMP, ORDER, V, T>),      \
                                   grid, block, 0, s, a);                         \
        } else if constexpr (kTiles2D[n].kind == 3) {                             \
            if (one)                                                              \
                hipLaunchKernelGGL((ac2d_step1_kernel<S, COMP, ORDER, V, T,       \
                                                      false, 0, 8>),              \
                                   grid, block8, 0, s, o);                        \
            else                                                                  \
                hipLaunchKernelGGL((ac2d_step_kernel<S, COMP, ORDER, V, T,        \
                                                     false, 0, 8>),               \
                                   grid, block8, 0, s, a);                        \
        } else if constexpr (COMP == COMP_TWOSUM8 ||                              \
                             steps_per_launch2d(kTiles2D[n]) != 1) {              \
            return hipErrorInvalidValue;   /* not a one-step shape here */        \
        } else {                                                                  \
            if (one)                                                              \
                hipLaunchKernelGGL((ac2d_march1_kernel<S, COMP, ORDER, V, T>),    \
                                   grid, block, 0, s, o);                         \
            else                                                                  \
                hipLaunchKernelGGL((ac2d_march_kernel<S, COMP, ORDER, V, T>),     \
                                   grid, block, 0, s, a);                         \
        }                                                                         \
        break;                                                                    \
    }
        HW_TILE(0) HW_TILE(1) HW_TILE(2) HW_TILE(3) HW_TILE(4) HW_TILE(5) HW_TILE(6)
        HW_TILE(7) HW_TILE(8)
#undef HW_TILE
    default:
        return hipErrorInvalidValue;   // two-step shapes: launch_ac2d_step2
    }
    static_assert(kNumTiles2D == 12, "update the tile dispatch");
    return hipGetLastError();
}

template <class S, int COMP>
static hipError_t step_order(const Ac2dBatch &a, const Ac2dDesc *one, int order,
                             int tile, bool forced, int stencil, hipStream_t s)
{
    return order == 4 ? step_tile<S, COMP, 4>(a, one, tile, forced, stencil, s)
                      : step_tile<S, COMP, 2>(a, one, tile, forced, stencil, s);
}

template <class S>
static hipError_t step_comp(const Ac2dBatch &a, const Ac2dDesc *one, int comp,
                            int order, int tile, bool forced, int stencil,
                            hipStream_t s)
{
    switch (comp) {
    case COMP_NONE:
        return step_order<S, COMP_NONE>(a, one, order, tile, forced, stencil, s);
    case COMP_FAST2SUM:
        return step_order<S, COMP_FAST2SUM>(a, one, order, tile, forced, stencil, s);
    case COMP_TWOSUM:
        return step_order<S, COMP_TWOSUM>(a, one, order, tile, forced, stencil, s);
    case COMP_TWOSUM8:
        if constexpr (S::id != F32::id)
            return step_order<S, COMP_TWOSUM8>(a, one, order, tile, forced, stencil, s);
        break;
    }
    return hipErrorInvalidValue;
}

hipError_t launch_ac2d_step(const Ac2dBatch &a, const Ac2dDesc *one, int storage,
                            int comp, int order, int tile, bool forced, int stencil,
                            hipStream_t s)
{
    if (a.total_tiles <= 0)
        return hipSuccess;
    if (one && a.nshots != 1)
        return hipErrorInvalidValue;
    switch (storage) {
    case HW_F32: return step_comp<F32>(a, one, comp, order, tile, forced, stencil, s);
    case HW_F16: return step_comp<F16>(a, one, comp, order, tile, forced, stencil, s);
    case HW_BF16: return step_comp<BF16>(a, one, comp, order, tile, forced, stencil, s);
    }
    return hipErrorInvalidValue;
}

template <class S>
static hipError_t energy_order(const Ac2dDesc *d, int par, int64_t ny,
                               int order, int st, double *partial, hipStream_t s)
{
    if (order == 4)
        hipLaunchKernelGGL((ac2d_energy_kernel<S, 4>), dim3(ny), dim3(kThreads),
                           0, s, d, par, st, partial);
    else
        hipLaunchKernelGGL((ac2d_energy_kernel<S, 2>), dim3(ny), dim3(kThreads),
                           0, s, d, par, st, partial);
    return hipGetLastError();
}

hipError_t launch_ac2d_energy(const Ac2dDesc *d_desc, int parity, int64_t ny,
                              int storage, int order, int stride,
                              double *partial, hipStream_t s)
{
    switch (storage) {
    case HW_F32: return energy_order<F32>(d_desc, parity, ny, order, stride, partial, s);
    case HW_F16: return energy_order<F16>(d_desc, parity, ny, order, stride, partial, s);
    case HW_BF16: return energy_order<BF16>(d_desc, parity, ny, order, stride, partial, s);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_tick(const StepCounters &c, hipStream_t s)
{
    hipLaunchKernelGGL(tick_kernel, dim3(1), dim3(kMaxBatch), 0, s, c);
    return hipGetLastError();
}

hipError_t launch_set_counter(int64_t *c, int64_t value, hipStream_t s)
{
    hipLaunchKernelGGL(set_counter_kernel, dim3(1), dim3(64), 0, s, c, value);
    return hipGetLastError();
}

hipError_t launch_energy_finish(const double *partial, int64_t n,
                                double factor, double *out, int32_t *flag,
                                hipStream_t s)
{
    hipLaunchKernelGGL(energy_finish_kernel, dim3(1), dim3(kThreads), 0, s,
                       partial, n, factor, out, flag);
    return hipGetLastError();
}

}  // namespace hw
