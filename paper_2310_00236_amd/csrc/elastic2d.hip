// 2D elastic (velocity-stress) leapfrog step and energy kernels for gfx950:
// Eq. (A1) of App. A, 2nd-order staggered differences, periodic in x, free
// surfaces on the normal-stress rows 0 and ny-1.
//
// Two kernel shapes, one thread per cell of 64 x 4 tiles: the fused shape
// computes a step in one pass (each thread recomputes the four neighbouring
// new velocities its stresses read); the two-pass shape runs a velocity
// pass (old stresses and velocities of field set par -> new velocities in
// set par^1) and then a stress pass (new velocities and old stresses -> new
// stresses in set par^1).  At the
// surfaces sxy is odd (the value half a cell outside is minus the value half
// a cell inside), syy stays zero, and sxx moves with the plate modulus
// carried by the per-cell coefficient tables.  Rows that lie outside the
// body (vy and sxy on row ny-1) and the surface rows of syy are copied
// through unchanged, so both field sets always hold a whole state.  Every
// arithmetic operation follows the same op-by-op definition as the CPU
// reference, so the results are bit-identical to it.
#include "hw_device.h"
#include "hw_internal.h"

#pragma clang fp contract(off)

namespace hw {

namespace {

constexpr int kTx = kTilesEl2D[0].tx;
constexpr int kTy = kTilesEl2D[0].ty;
static_assert(kTx * kTy == kThreads, "one thread per cell of a tile");

struct Where {
    int i, j;
    bool valid;
};

__device__ __forceinline__ Where where(const El2dDesc &d)
{
    const int tiles_x = (int)((d.nx + kTx - 1) / kTx);
    Where w;
    w.i = (int)(blockIdx.x % tiles_x) * kTx + (int)threadIdx.x % kTx;
    w.j = (int)(blockIdx.x / tiles_x) * kTy + (int)threadIdx.x / kTx;
    w.valid = w.i < (int)d.nx && w.j < (int)d.ny;
    return w;
}

__device__ __forceinline__ int wrapx(int i, int n)
{
    return i < 0 ? i + n : (i >= n ? i - n : i);
}

// Load of a word that this pass reads once: non-temporal in the two-pass
// kernels (at 4096^2 the passes run 12-21% faster), through the caches in
// the one-pass kernel, whose threads re-read their neighbours' words.
template <bool NT, class T>
__device__ __forceinline__ T once(const T *base, int q)
{
    if constexpr (NT)
        return __builtin_nontemporal_load(gmem(base) + q);
    else
        return gmem(base)[q];
}

// Store of one field word to the new set: non-temporal for words of 4 bytes
// and more (a value with its compensation term, or fp32), plain for 2-byte
// words -- the choice that measured fastest for the 2D acoustic step.
template <class W>
__device__ __forceinline__ void put(W *base, int q, W v)
{
    if constexpr (sizeof(W) >= 4)
        __builtin_nontemporal_store(v, gmem(base) + q);
    else
        gmem(base)[q] = v;
}

}  // namespace

// The new velocity words of one cell (from the old stresses and velocities
// of set par): vx at (i+1/2, j), and vy at (i, j+1/2) -- on row ny-1, which
// lies outside the body, the old word.  FRC: the plan has a point source
// (on vy) or receivers; the source sample of this step joins the vy
// increment after the multiplication by the staggered buoyancy.  Shared by
// the two-pass velocity kernel and the fused kernel, which recomputes its
// neighbours' new velocities with them.
template <class S, int COMP, bool NT>
__device__ __forceinline__ typename Word<S, COMP>::type new_vx(const El2dDesc &d, int par,
                                                                int i, int j)
{
    using WD = Word<S, COMP>;
    using W = typename WD::type;
    using GW = const W HW_GLOBAL *;
    const int nx = (int)d.nx, ny = (int)d.ny, pitch = (int)d.pitch;
    const int ip = wrapx(i + 1, nx);
    const int row = j * pitch, q = row + i;
    // the row below, clamped so that the load address lies in the grid
    const int qdn = j > 0 ? q - pitch : q;
    const float HW_GLOBAL *__restrict__ B = gmem(d.b);
    GW sxx = gmem((const W *)d.f[par][2]);
    GW sxy = gmem((const W *)d.f[par][4]);
    auto L = [](GW p, int idx) { return S::load(WD::v(p[idx])); };
    // sxy below and above the point, imaged across the surfaces
    const float s_dn = L(sxy, qdn), s_q = L(sxy, q);
    const float lo = j == 0 ? -s_q : s_dn;
    const float hi = j == ny - 1 ? -s_dn : s_q;
    const float d1 = L(sxx, row + ip) - L(sxx, q);
    const float d2 = hi - lo;
    const float g = d.w * (d1 + d2);
    const float bb = 0.5f * (B[q] + B[row + ip]);
    const W old = once<NT>((const W *)d.f[par][0], q);
    auto v = WD::v(old), cc = WD::c(old);
    update_store<S, COMP>(v, cc, bb * g);
    return WD::make(v, cc);
}

template <class S, int COMP, bool FRC, bool NT>
__device__ __forceinline__ typename Word<S, COMP>::type new_vy(const El2dDesc &d, int par,
                                                                int i, int j)
{
    using WD = Word<S, COMP>;
    using W = typename WD::type;
    using GW = const W HW_GLOBAL *;
    const int nx = (int)d.nx, ny = (int)d.ny, pitch = (int)d.pitch;
    const int im = wrapx(i - 1, nx);
    const int row = j * pitch, q = row + i;
    const W old = once<NT>((const W *)d.f[par][1], q);
    if (j >= ny - 1)
        return old;
    const float HW_GLOBAL *__restrict__ B = gmem(d.b);
    GW syy = gmem((const W *)d.f[par][3]);
    GW sxy = gmem((const W *)d.f[par][4]);
    auto L = [](GW p, int idx) { return S::load(WD::v(p[idx])); };
    const float d1 = L(sxy, q) - L(sxy, row + im);
    const float d2 = L(syy, q + pitch) - L(syy, q);
    const float g = d.w * (d1 + d2);
    const float bb = 0.5f * (B[q] + B[q + pitch]);
    float inc = bb * g;
    if constexpr (FRC) {
        if (d.src_n > 0 && i == d.src_x && j == d.src_y) {
            const int64_t n = *gmem(d.step);
            if (n < d.src_n)
                inc = inc + gmem(d.src)[n];
        }
    }
    auto v = WD::v(old), cc = WD::c(old);
    update_store<S, COMP>(v, cc, inc);
    return WD::make(v, cc);
}

// Two-pass step, first pass: the new velocities of one cell to set par^1.
template <class S, int COMP, bool FRC>
__global__ __launch_bounds__(kThreads) void el2d_velocity_kernel(const El2dDesc d,
                                                                 int par)
{
    using W = typename Word<S, COMP>::type;
    const Where c = where(d);
    if (!c.valid)
        return;
    const int q = c.j * (int)d.pitch + c.i;
    put((W *)d.f[par ^ 1][0], q, new_vx<S, COMP, true>(d, par, c.i, c.j));
    put((W *)d.f[par ^ 1][1], q, new_vy<S, COMP, FRC, true>(d, par, c.i, c.j));
}

// The new stresses of cell (i, j) from the new velocities it needs (vx at
// (i, j), (i-1, j), (i, j+1); vy at (i, j), (i, j-1), (i+1, j)) given as
// values, old stresses from set par, written to set par^1.
template <class S, int COMP, bool NT>
__device__ __forceinline__ void stress_update(const El2dDesc &d, int par, int i, int j,
                                              float vx_q, float vx_im, float vx_jp,
                                              float vy_q, float vy_dn, float vy_ip)
{
    using WD = Word<S, COMP>;
    using W = typename WD::type;
    const int ny = (int)d.ny;
    const int q = j * (int)d.pitch + i;
    const float w = d.w;
    const bool surface = j == 0 || j == ny - 1;
    const float ex = w * (vx_q - vx_im);
    const float ey = surface ? 0.0f : w * (vy_q - vy_dn);
    const float l2m = once<NT>(d.l2m, q), lam = once<NT>(d.lam, q);
    auto upd = [&](int f, float inc) {
        const W old = once<NT>((const W *)d.f[par][f], q);
        auto v = WD::v(old), cc = WD::c(old);
        update_store<S, COMP>(v, cc, inc);
        put((W *)d.f[par ^ 1][f], q, WD::make(v, cc));
    };
    auto keep = [&](int f) { put((W *)d.f[par ^ 1][f], q, once<NT>((const W *)d.f[par][f], q)); };
    upd(2, l2m * ex + lam * ey);
    if (!surface)
        upd(3, l2m * ey + lam * ex);
    else
        keep(3);
    if (j < ny - 1) {   // sxy at (i+1/2, j+1/2)
        const float a1 = vy_ip - vy_q;
        const float a2 = vx_jp - vx_q;
        const float g = w * (a1 + a2);
        upd(4, once<NT>(d.mxy, q) * g);
    } else {
        keep(4);
    }
}

// One-pass step: each thread computes its cell's new velocities (stored)
// and the four neighbouring new velocities its stresses read, recomputed
// from old values with the same operations, so new velocities never pass
// through memory within a step; then its new stresses.  Every word of the
// state is read from set par and written to set par^1 once per step (the
// neighbours' old words are re-read from the caches).
template <class S, int COMP, bool FRC>
__global__ __launch_bounds__(kThreads) void el2d_fused_kernel(const El2dDesc d, int par)
{
    using WD = Word<S, COMP>;
    using W = typename WD::type;
    const Where c = where(d);
    if (!c.valid)
        return;
    const int nx = (int)d.nx, ny = (int)d.ny;
    const int i = c.i, j = c.j;
    const int q = j * (int)d.pitch + i;
    const W wx = new_vx<S, COMP, false>(d, par, i, j);
    const W wy = new_vy<S, COMP, FRC, false>(d, par, i, j);
    put((W *)d.f[par ^ 1][0], q, wx);
    put((W *)d.f[par ^ 1][1], q, wy);
    auto V = [](W x) { return S::load(WD::v(x)); };
    const float vx_q = V(wx), vy_q = V(wy);
    const float vx_im = V(new_vx<S, COMP, false>(d, par, wrapx(i - 1, nx), j));
    // the rows above and below are read only off the surfaces (ey) and
    // above the last row (sxy); rows stay uniform across a wavefront
    float vy_dn = 0.0f, vx_jp = 0.0f, vy_ip = 0.0f;
    if (j > 0 && j < ny - 1)
        vy_dn = V(new_vy<S, COMP, FRC, false>(d, par, i, j - 1));
    if (j < ny - 1) {
        vx_jp = V(new_vx<S, COMP, false>(d, par, i, j + 1));
        vy_ip = V(new_vy<S, COMP, FRC, false>(d, par, wrapx(i + 1, nx), j));
    }
    stress_update<S, COMP, false>(d, par, i, j, vx_q, vx_im, vx_jp, vy_q, vy_dn, vy_ip);
}

// Two-pass step, second pass: the new stresses of one cell from the new
// velocities in set par^1.
template <class S, int COMP>
__global__ __launch_bounds__(kThreads) void el2d_stress_kernel(const El2dDesc d,
                                                               int par)
{
    using WD = Word<S, COMP>;
    using W = typename WD::type;
    using GW = const W HW_GLOBAL *;
    const Where c = where(d);
    if (!c.valid)
        return;
    const int nx = (int)d.nx, ny = (int)d.ny, pitch = (int)d.pitch;
    const int i = c.i, j = c.j;
    const int ip = wrapx(i + 1, nx), im = wrapx(i - 1, nx);
    const int row = j * pitch, q = row + i;
    // neighbour rows, clamped so that every load address lies in the grid
    const int qdn = j > 0 ? q - pitch : q, qup = j < ny - 1 ? q + pitch : q;
    GW vx = gmem((const W *)d.f[par ^ 1][0]);
    GW vy = gmem((const W *)d.f[par ^ 1][1]);
    auto L = [](GW p, int idx) { return S::load(WD::v(p[idx])); };
    stress_update<S, COMP, true>(d, par, i, j, L(vx, q), L(vx, row + im), L(vx, qup),
                           L(vy, q), L(vy, qdn), L(vy, row + ip));
}

// Receivers after the step: the five new fields at each receiver cell, as
// fp64 (exact widening, unscaled), in trace row n = the plan's step count.
template <class S, int COMP>
__global__ __launch_bounds__(64) void el2d_record_kernel(const El2dDesc d, int par)
{
    using WD = Word<S, COMP>;
    using W = typename WD::type;
    const int r = (int)threadIdx.x;
    if (r >= d.rec_n)
        return;
    const int64_t n = *gmem(d.step);
    if (n >= d.rec_rows)
        return;
    const int32_t HW_GLOBAL *xy = gmem(d.rec_xy);
    const int64_t q = (int64_t)xy[2 * r + 1] * d.pitch + xy[2 * r];
    for (int f = 0; f < 5; ++f) {
        const float v = S::load(WD::v(gmem((const W *)d.f[par][f])[q]));
        gmem(d.rec)[(n * d.rec_n + r) * 5 + f] = (double)v * d.rec_scale;
    }
}

__device__ __forceinline__ double block_sum2(double v, double *red)
{
    return block_sum_f64<kThreads>(v, red);
}

// Energy of the state, one workgroup per row, fp64 per cell: h_j (vx^- vx^+
// / bx + s^T C^-1 s) plus, below the last row, vy^- vy^+ / by + sxy^2 / mxy,
// with v^+ recomputed in fp64 and h_j = 1/2 on the surface rows.
template <class S>
__global__ __launch_bounds__(kThreads) void el2d_energy_kernel(
    const El2dDesc *__restrict__ dd, int par, int st, double *__restrict__ partial)
{
    using T = typename S::store_t;
    __shared__ double red[kThreads];
    const El2dDesc &d = *dd;
    const int64_t nx = d.nx, ny = d.ny, pitch = d.pitch;
    const int64_t j = xcd_band<kNumXcd>(blockIdx.x, gridDim.x);
    const double w = d.w;
    const T *f[5];
    for (int n = 0; n < 5; ++n)
        f[n] = (const T *)d.f[par][n];
    auto L = [&](int n, int64_t idx) { return (double)S::load(f[n][idx * st]); };
    const float *B = d.b;
    const double h = (j == 0 || j == ny - 1) ? 0.5 : 1.0;
    double acc = 0.0;
    for (int64_t i = threadIdx.x; i < nx; i += kThreads) {
        const int64_t ip = wrap1(i + 1, nx), im = wrap1(i - 1, nx);
        const int64_t row = j * pitch, q = row + i;
        const int64_t qdn = j > 0 ? q - pitch : q, qup = j < ny - 1 ? q + pitch : q;
        const double sxx = L(2, q), syy = L(3, q);
        const double s_dn = L(4, qdn), s_q = L(4, q);
        const double lo = j == 0 ? -s_q : s_dn;
        const double hi = j == ny - 1 ? -s_dn : s_q;
        const double gx = w * ((L(2, row + ip) - sxx) + (hi - lo));
        const double bx = 0.5 * ((double)B[q] + (double)B[row + ip]);
        const double vx = L(0, q);
        const double vxp = vx + bx * gx;
        const double l2m = d.l2m[q], lam = d.lam[q];
        const double en = (l2m * (sxx * sxx + syy * syy) - 2.0 * lam * (sxx * syy)) /
                          (l2m * l2m - lam * lam);
        double e = h * ((vx * vxp) / bx + en);
        if (j < ny - 1) {
            const double sxy = L(4, q);
            const double gy = w * ((sxy - L(4, row + im)) + (L(3, qup) - syy));
            const double by = 0.5 * ((double)B[q] + (double)B[qup]);
            const double vy = L(1, q);
            const double vyp = vy + by * gy;
            e = e + ((vy * vyp) / by + (sxy * sxy) / (double)d.mxy[q]);
        }
        acc += e;
    }
    const double s = block_sum2(acc, red);
    if (threadIdx.x == 0)
        partial[j] = s;
}

// ------------------------------------------------------------- dispatch --

template <class S, int COMP>
static hipError_t el2d_launch(const El2dDesc &d, int parity, bool forced, int tile,
                              hipStream_t s)
{
    const int64_t tiles = ((d.nx + kTx - 1) / kTx) * ((d.ny + kTy - 1) / kTy);
    const dim3 grid((unsigned)tiles), block(kThreads);
    if (kTilesEl2D[tile].kind == 1) {
        if (forced)
            hipLaunchKernelGGL((el2d_fused_kernel<S, COMP, true>), grid, block, 0, s, d,
                               parity);
        else
            hipLaunchKernelGGL((el2d_fused_kernel<S, COMP, false>), grid, block, 0, s, d,
                               parity);
    } else {
        if (forced)
            hipLaunchKernelGGL((el2d_velocity_kernel<S, COMP, true>), grid, block, 0, s, d,
                               parity);
        else
            hipLaunchKernelGGL((el2d_velocity_kernel<S, COMP, false>), grid, block, 0, s, d,
                               parity);
        hipLaunchKernelGGL((el2d_stress_kernel<S, COMP>), grid, block, 0, s, d, parity);
    }
    if (forced && d.rec_n > 0)
        hipLaunchKernelGGL((el2d_record_kernel<S, COMP>), dim3(1), dim3(64), 0, s, d,
                           parity ^ 1);
    return hipGetLastError();
}

template <class S>
static hipError_t el2d_comp(const El2dDesc &d, int parity, int comp, bool forced,
                            int tile, hipStream_t s)
{
    switch (comp) {
    case COMP_NONE: return el2d_launch<S, COMP_NONE>(d, parity, forced, tile, s);
    case COMP_FAST2SUM: return el2d_launch<S, COMP_FAST2SUM>(d, parity, forced, tile, s);
    case COMP_TWOSUM: return el2d_launch<S, COMP_TWOSUM>(d, parity, forced, tile, s);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_el2d_step(const El2dDesc &d, int parity, int storage, int comp,
                            bool forced, int tile, hipStream_t s)
{
    if (d.nx <= 0 || d.ny <= 0)
        return hipSuccess;
    if (tile < 0 || tile >= kNumTilesEl2D)
        return hipErrorInvalidValue;
    switch (storage) {
    case HW_F32: return el2d_comp<F32>(d, parity, comp, forced, tile, s);
    case HW_F16: return el2d_comp<F16>(d, parity, comp, forced, tile, s);
    case HW_BF16: return el2d_comp<BF16>(d, parity, comp, forced, tile, s);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_el2d_energy(const El2dDesc *d_desc, int parity, int64_t ny,
                              int storage, int stride, double *partial,
                              hipStream_t s)
{
    switch (storage) {
    case HW_F32:
        hipLaunchKernelGGL(el2d_energy_kernel<F32>, dim3(ny), dim3(kThreads), 0, s,
                           d_desc, parity, stride, partial);
        break;
    case HW_F16:
        hipLaunchKernelGGL(el2d_energy_kernel<F16>, dim3(ny), dim3(kThreads), 0, s,
                           d_desc, parity, stride, partial);
        break;
    case HW_BF16:
        hipLaunchKernelGGL(el2d_energy_kernel<BF16>, dim3(ny), dim3(kThreads), 0, s,
                           d_desc, parity, stride, partial);
        break;
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace hw
