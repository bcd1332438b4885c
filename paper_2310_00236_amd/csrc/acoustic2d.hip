// 2D acoustic leapfrog step and energy kernels for gfx950.
//
// One launch advances every shot of a batch by one full leapfrog step
// (Sec. 3; Alg. 1 or Alg. 2 of Sec. 4): a workgroup owns a TX x TY tile of
// cells and, in a single pass over HBM,
//   1. stages the old pressure tile plus a halo of 2R-1 cells in LDS,
//   2. computes the new velocities v^{n+1/2} for its cells plus the R-cell
//      halo its pressure stencil needs (the halo values are recomputed
//      redundantly from old values, so no grid-wide barrier is needed),
//      keeping them in LDS and writing its own cells to the other field set,
//   3. computes the new pressure p^{n+1} from the LDS velocities.
// Fields and velocity compensation terms ping-pong between two sets; the
// pressure compensation is private to its cell and updated in place.  Every
// arithmetic operation matches the op-by-op definition the CPU reference
// uses, so results are bit-identical to it and independent of the tile
// shape and of the batch a shot runs in.
#include "hw_device.h"
#include "hw_internal.h"

#pragma clang fp contract(off)

namespace hw {

// Workgroups are dealt to the 8 XCDs round-robin; give each XCD a
// contiguous range of tiles so that tiles sharing halos share an L2.
__device__ __forceinline__ int32_t xcd_tile(int32_t b, int32_t n)
{
    int32_t per = n / kNumXcd, rem = n % kNumXcd;
    int32_t x = b % kNumXcd, r = b / kNumXcd;
    return x * per + (x < rem ? x : rem) + r;
}

template <class A>
__device__ __forceinline__ int find_shot(const A &a, int32_t t)
{
    int lo = 0, hi = a.nshots - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (a.tile_start[mid] <= t)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

constexpr int cdiv(int a, int b) { return (a + b - 1) / b; }

// Periodic wrap of a 32-bit index (any offset).
__device__ __forceinline__ int wrapi(int i, int n)
{
    const int r = i % n;
    return r < 0 ? r + n : r;
}

template <class S, int COMP, int ORDER, int TX, int TY>
__global__ __launch_bounds__(kThreads) void ac2d_step_kernel(const Ac2dBatch a)
{
    using T = typename S::store_t;
    using WD = Word<S, COMP>;
    using W = typename WD::type;
    constexpr int R = ORDER / 2;              // velocity halo
    constexpr int H = 2 * R - 1;              // pressure halo
    constexpr int PW = TX + 2 * H, PH = TY + 2 * H, NPT = PW * PH;
    constexpr int BW = TX + 2 * R, BH = TY + 2 * R, NBT = BW * BH;
    constexpr int VXW = TX + 2 * R - 1, NVX = TY * VXW;   // lx in [-R, TX+R-1)
    constexpr int VYH = TY + 2 * R - 1, NVY = VYH * TX;   // ly in [-R, TY+R-1)
    constexpr int NC = TX * TY;
    constexpr int KP = cdiv(NPT, kThreads), KB = cdiv(NBT, kThreads);
    constexpr int KVX = cdiv(NVX, kThreads), KVY = cdiv(NVY, kThreads);
    constexpr int KC = cdiv(NC, kThreads);
    __shared__ float ps[NPT];     // old p,   x in [x0-H, x0+TX+H), y likewise
    __shared__ float bs[NBT];     // 1/rho,   x in [x0-R, x0+TX+R), y likewise
    __shared__ float vxs[NVX];    // new vx on the tile rows
    __shared__ float vys[NVY];    // new vy on the tile columns
    const int tid = threadIdx.x;

    int32_t tile = xcd_tile(blockIdx.x, a.total_tiles);
    const int shot = find_shot(a, tile);
    const Ac2dDesc &d = *a.desc[shot];
    const int par = a.parity[shot];
    tile -= a.tile_start[shot];
    const int nx = (int)d.nx, ny = (int)d.ny, pitch = (int)d.pitch;
    const int ntx = a.tiles_x[shot];
    const int x0 = (tile % ntx) * TX;
    const int y0 = (tile / ntx) * TY;
    const float w1 = d.w1, w2 = d.w2;
    const float HW_GLOBAL *__restrict__ b = gmem(d.b);
    const float HW_GLOBAL *__restrict__ kap = gmem(d.k);
    const W HW_GLOBAL *__restrict__ p_in = gmem((const W *)d.p[par]);
    const W HW_GLOBAL *__restrict__ vx_in = gmem((const W *)d.vx[par]);
    const W HW_GLOBAL *__restrict__ vy_in = gmem((const W *)d.vy[par]);
    W HW_GLOBAL *__restrict__ p_out = gmem((W *)d.p[par ^ 1]);
    W HW_GLOBAL *__restrict__ vx_out = gmem((W *)d.vx[par ^ 1]);
    W HW_GLOBAL *__restrict__ vy_out = gmem((W *)d.vy[par ^ 1]);
    // No index of this tile (halos included) leaves the grid: no wrapping.
    const bool interior = x0 >= H && x0 + TX + H <= nx && y0 >= H &&
                          y0 + TY + H <= ny;

    // ---- 1. issue every global load of the tile before using any of them
    float pr[KP], br[KB], kr[KC];
    W vxo[KVX], vyo[KVY], po[KC];
#pragma unroll
    for (int k = 0; k < KP; ++k) {
        const int e = tid + k * kThreads;
        if (e < NPT) {
            int gy = y0 + e / PW - H, gx = x0 + e % PW - H;
            if (!interior) {
                gy = wrapi(gy, ny);
                gx = wrapi(gx, nx);
            }
            pr[k] = S::load(WD::v(p_in[gy * pitch + gx]));
        }
    }
#pragma unroll
    for (int k = 0; k < KB; ++k) {
        const int e = tid + k * kThreads;
        if (e < NBT) {
            int gy = y0 + e / BW - R, gx = x0 + e % BW - R;
            if (!interior) {
                gy = wrapi(gy, ny);
                gx = wrapi(gx, nx);
            }
            br[k] = b[gy * pitch + gx];
        }
    }
#pragma unroll
    for (int k = 0; k < KVX; ++k) {
        const int e = tid + k * kThreads;
        const int gy = y0 + e / VXW;
        if (e < NVX && gy < ny) {
            int gx = x0 + e % VXW - R;
            if (!interior)
                gx = wrapi(gx, nx);
            vxo[k] = vx_in[gy * pitch + gx];
        }
    }
#pragma unroll
    for (int k = 0; k < KVY; ++k) {
        const int e = tid + k * kThreads;
        const int gx = x0 + e % TX;
        if (e < NVY && gx < nx) {
            int gy = y0 + e / TX - R;
            if (!interior)
                gy = wrapi(gy, ny);
            vyo[k] = vy_in[gy * pitch + gx];
        }
    }
#pragma unroll
    for (int k = 0; k < KC; ++k) {
        const int e = tid + k * kThreads;
        const int gx = x0 + e % TX, gy = y0 + e / TX;
        if (e < NC && gx < nx && gy < ny) {
            const int q = gy * pitch + gx;
            kr[k] = kap[q];
            po[k] = p_in[q];
        }
    }

    // ---- 2. stage old pressure and buoyancy in LDS
#pragma unroll
    for (int k = 0; k < KP; ++k) {
        const int e = tid + k * kThreads;
        if (e < NPT)
            ps[e] = pr[k];
    }
#pragma unroll
    for (int k = 0; k < KB; ++k) {
        const int e = tid + k * kThreads;
        if (e < NBT)
            bs[e] = br[k];
    }
    __syncthreads();

    // ---- 3a. new vx on the tile rows, x in [x0-R, x0+TX+R-1)
#pragma unroll
    for (int k = 0; k < KVX; ++k) {
        const int e = tid + k * kThreads;
        const int ly = e / VXW, lx = e % VXW - R;
        if (e < NVX && y0 + ly < ny) {
            const float *pp = &ps[(ly + H) * PW + (lx + H)];
            const float a0 = pp[1] - pp[0];
            float g;
            if constexpr (ORDER == 4) {
                const float a1 = pp[2] - pp[-1];
                g = w1 * a0 + w2 * a1;
            } else {
                g = w1 * a0;
            }
            const float *bb = &bs[(ly + R) * BW + (lx + R)];
            const float bx = 0.5f * (bb[0] + bb[1]);
            const float inc = bx * g;
            T v = WD::v(vxo[k]), c = WD::c(vxo[k]);
            update_store<S, COMP>(v, c, inc);
            vxs[e] = S::load(v);
            if (lx >= 0 && lx < TX && x0 + lx < nx)
                __builtin_nontemporal_store(WD::make(v, c), &vx_out[(y0 + ly) * pitch + x0 + lx]);
        }
    }

    // ---- 3b. new vy on the tile columns, y in [y0-R, y0+TY+R-1)
#pragma unroll
    for (int k = 0; k < KVY; ++k) {
        const int e = tid + k * kThreads;
        const int ly = e / TX - R, lx = e % TX;
        if (e < NVY && x0 + lx < nx) {
            const float *pp = &ps[(ly + H) * PW + (lx + H)];
            const float a0 = pp[PW] - pp[0];
            float g;
            if constexpr (ORDER == 4) {
                const float a1 = pp[2 * PW] - pp[-PW];
                g = w1 * a0 + w2 * a1;
            } else {
                g = w1 * a0;
            }
            const float *bb = &bs[(ly + R) * BW + (lx + R)];
            const float by = 0.5f * (bb[0] + bb[BW]);
            const float inc = by * g;
            T v = WD::v(vyo[k]), c = WD::c(vyo[k]);
            update_store<S, COMP>(v, c, inc);
            vys[e] = S::load(v);
            if (ly >= 0 && ly < TY && y0 + ly < ny)
                __builtin_nontemporal_store(WD::make(v, c), &vy_out[(y0 + ly) * pitch + x0 + lx]);
        }
    }
    __syncthreads();

    // ---- 4. new pressure on the tile
#pragma unroll
    for (int k = 0; k < KC; ++k) {
        const int e = tid + k * kThreads;
        const int ly = e / TX, lx = e % TX;
        if (e < NC && x0 + lx < nx && y0 + ly < ny) {
            const float *vr = &vxs[ly * VXW + lx + R];
            const float *vc = &vys[(ly + R) * TX + lx];
            const float ax0 = vr[0] - vr[-1];
            const float ay0 = vc[0] - vc[-TX];
            float gxv, gyv;
            if constexpr (ORDER == 4) {
                const float ax1 = vr[1] - vr[-2];
                const float ay1 = vc[TX] - vc[-2 * TX];
                gxv = w1 * ax0 + w2 * ax1;
                gyv = w1 * ay0 + w2 * ay1;
            } else {
                gxv = w1 * ax0;
                gyv = w1 * ay0;
            }
            const float dv = gxv + gyv;
            const float inc = kr[k] * dv;
            T pv = WD::v(po[k]), c = WD::c(po[k]);
            update_store<S, COMP>(pv, c, inc);
            __builtin_nontemporal_store(WD::make(pv, c), &p_out[(y0 + ly) * pitch + x0 + lx]);
        }
    }
}

// Fixed-order block sum of one fp64 value per thread (thread 0 returns it).
__device__ __forceinline__ double block_sum(double v, double *red)
{
    red[threadIdx.x] = v;
    __syncthreads();
    for (int s = kThreads / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s)
            red[threadIdx.x] = red[threadIdx.x] + red[threadIdx.x + s];
        __syncthreads();
    }
    return red[0];
}

// Energy of the state, one workgroup per grid row: per-cell terms in fp64
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
    const int64_t j = blockIdx.x;
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
    double acc = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += kThreads)
        acc += partial[i];
    const double s = block_sum(acc, red);
    if (threadIdx.x == 0) {
        const double e = s * factor;
        *out = e;
        if (!isfinite(e))
            *flag = 1;
    }
}

// ------------------------------------------------------------- dispatch --

template <class S, int COMP, int ORDER>
static hipError_t step_tile(const Ac2dBatch &a, int tile, hipStream_t s)
{
    const dim3 grid(a.total_tiles), block(kThreads);
    switch (tile) {
#define HW_TILE(n)                                                              \
    case n:                                                                     \
        hipLaunchKernelGGL((ac2d_step_kernel<S, COMP, ORDER, kTiles2D[n].tx,    \
                                             kTiles2D[n].ty>),                  \
                           grid, block, 0, s, a);                               \
        break;
        HW_TILE(0) HW_TILE(1) HW_TILE(2) HW_TILE(3) HW_TILE(4)
#undef HW_TILE
    default:
        return hipErrorInvalidValue;
    }
    static_assert(kNumTiles2D == 5, "update the tile dispatch");
    return hipGetLastError();
}

template <class S, int COMP>
static hipError_t step_order(const Ac2dBatch &a, int order, int tile,
                             hipStream_t s)
{
    return order == 4 ? step_tile<S, COMP, 4>(a, tile, s)
                      : step_tile<S, COMP, 2>(a, tile, s);
}

template <class S>
static hipError_t step_comp(const Ac2dBatch &a, int comp, int order, int tile,
                            hipStream_t s)
{
    switch (comp) {
    case COMP_NONE: return step_order<S, COMP_NONE>(a, order, tile, s);
    case COMP_FAST2SUM: return step_order<S, COMP_FAST2SUM>(a, order, tile, s);
    case COMP_TWOSUM: return step_order<S, COMP_TWOSUM>(a, order, tile, s);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_ac2d_step(const Ac2dBatch &a, int storage, int comp,
                            int order, int tile, hipStream_t s)
{
    if (a.total_tiles <= 0)
        return hipSuccess;
    switch (storage) {
    case HW_F32: return step_comp<F32>(a, comp, order, tile, s);
    case HW_F16: return step_comp<F16>(a, comp, order, tile, s);
    case HW_BF16: return step_comp<BF16>(a, comp, order, tile, s);
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

hipError_t launch_energy_finish(const double *partial, int64_t n,
                                double factor, double *out, int32_t *flag,
                                hipStream_t s)
{
    hipLaunchKernelGGL(energy_finish_kernel, dim3(1), dim3(kThreads), 0, s,
                       partial, n, factor, out, flag);
    return hipGetLastError();
}

}  // namespace hw
