// 3D elastic (velocity-stress) leapfrog step and energy kernels for gfx950.
//
// A step is two passes over the grid, both in place: the velocity pass
// updates vx, vy, vz from the divergence of the old stresses, then the
// stress pass updates the six stresses from the new velocities (the 3D form
// of Eq. A1, App. A, 2nd-order staggered differences).  Each pass reads
// only fields the other pass writes, plus the cell's own field, so updating
// in place is race free.  Every arithmetic operation follows the same
// op-by-op definition as the CPU reference (bit-identical results).
#include "hw_device.h"
#include "hw_internal.h"

#pragma clang fp contract(off)

namespace hw {

__device__ __forceinline__ int32_t xcd_tile3(int32_t b, int32_t n)
{
    int32_t per = n / kNumXcd, rem = n % kNumXcd;
    int32_t x = b % kNumXcd, r = b / kNumXcd;
    return x * per + (x < rem ? x : rem) + r;
}

__device__ __forceinline__ int find_shot3(const El3dBatch &a, int32_t t)
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

struct Cell {
    int i, j, k;
    bool valid;
};

__device__ __forceinline__ int wrapu(int i, int n)
{
    return i < 0 ? i + n : (i >= n ? i - n : i);
}

template <int TX, int TY>
__device__ __forceinline__ Cell locate(const El3dBatch &a, const El3dDesc *&dp)
{
    int32_t tile = xcd_tile3(blockIdx.x, a.total_tiles);
    const int shot = find_shot3(a, tile);
    dp = a.desc[shot];
    const El3dDesc &d = *dp;
    tile -= a.tile_start[shot];
    const int ntx = a.tiles_x[shot];
    const int per_slice = ntx * a.tiles_y[shot];
    const int r = tile % per_slice;
    Cell c;
    c.k = tile / per_slice;
    c.i = (r % ntx) * TX + (int)threadIdx.x % TX;
    c.j = (r / ntx) * TY + (int)threadIdx.x / TX;
    c.valid = c.i < (int)d.nx && c.j < (int)d.ny;
    return c;
}

template <class S, int COMP, int TX, int TY>
__global__ __launch_bounds__(kThreads) void el3d_velocity_kernel(const El3dBatch a)
{
    using WD = Word<S, COMP>;
    using W = typename WD::type;
    const El3dDesc *dp;
    const Cell cl = locate<TX, TY>(a, dp);
    if (!cl.valid)
        return;
    const El3dDesc &d = *dp;
    const int nx = (int)d.nx, ny = (int)d.ny, nz = (int)d.nz;
    const int pitch = (int)d.pitch, slab = (int)d.slab;
    const int i = cl.i, j = cl.j, k = cl.k;
    const int ip = wrapu(i + 1, nx), im = wrapu(i - 1, nx);
    const int jp = wrapu(j + 1, ny), jm = wrapu(j - 1, ny);
    const int kp = wrapu(k + 1, nz), km = wrapu(k - 1, nz);
    const int row = k * slab + j * pitch;
    const int q = row + i;
    const float w = d.w;
    using GW = const W HW_GLOBAL *;
    const float HW_GLOBAL *__restrict__ B = gmem(d.b);
    GW sxx = gmem((const W *)d.f[3]), syy = gmem((const W *)d.f[4]);
    GW szz = gmem((const W *)d.f[5]), sxy = gmem((const W *)d.f[6]);
    GW sxz = gmem((const W *)d.f[7]), syz = gmem((const W *)d.f[8]);
    auto L = [](GW p, int idx) { return S::load(WD::v(p[idx])); };
    const float sxy_q = L(sxy, q), sxz_q = L(sxz, q), syz_q = L(syz, q);
    const float bq = B[q];
    float inc[3];
    {   // vx at (i+1/2, j, k)
        const float d1 = L(sxx, row + ip) - L(sxx, q);
        const float d2 = sxy_q - L(sxy, k * slab + jm * pitch + i);
        const float d3 = sxz_q - L(sxz, km * slab + j * pitch + i);
        const float g = w * ((d1 + d2) + d3);
        const float bb = 0.5f * (bq + B[row + ip]);
        inc[0] = bb * g;
    }
    {   // vy at (i, j+1/2, k)
        const float d1 = sxy_q - L(sxy, row + im);
        const float d2 = L(syy, k * slab + jp * pitch + i) - L(syy, q);
        const float d3 = syz_q - L(syz, km * slab + j * pitch + i);
        const float g = w * ((d1 + d2) + d3);
        const float bb = 0.5f * (bq + B[k * slab + jp * pitch + i]);
        inc[1] = bb * g;
    }
    {   // vz at (i, j, k+1/2)
        const float d1 = sxz_q - L(sxz, row + im);
        const float d2 = syz_q - L(syz, k * slab + jm * pitch + i);
        const float d3 = L(szz, kp * slab + j * pitch + i) - L(szz, q);
        const float g = w * ((d1 + d2) + d3);
        const float bb = 0.5f * (bq + B[kp * slab + j * pitch + i]);
        inc[2] = bb * g;
    }
#pragma unroll
    for (int f = 0; f < 3; ++f) {
        W HW_GLOBAL *vf = gmem((W *)d.f[f]);
        const W old = vf[q];
        auto v = WD::v(old), c = WD::c(old);
        update_store<S, COMP>(v, c, inc[f]);
        vf[q] = WD::make(v, c);
    }
}

template <class S, int COMP, int TX, int TY>
__global__ __launch_bounds__(kThreads) void el3d_stress_kernel(const El3dBatch a)
{
    using WD = Word<S, COMP>;
    using W = typename WD::type;
    const El3dDesc *dp;
    const Cell cl = locate<TX, TY>(a, dp);
    if (!cl.valid)
        return;
    const El3dDesc &d = *dp;
    const int nx = (int)d.nx, ny = (int)d.ny, nz = (int)d.nz;
    const int pitch = (int)d.pitch, slab = (int)d.slab;
    const int i = cl.i, j = cl.j, k = cl.k;
    const int ip = wrapu(i + 1, nx), im = wrapu(i - 1, nx);
    const int jp = wrapu(j + 1, ny), jm = wrapu(j - 1, ny);
    const int kp = wrapu(k + 1, nz), km = wrapu(k - 1, nz);
    const int row = k * slab + j * pitch;
    const int q = row + i;
    const float w = d.w;
    using GW = const W HW_GLOBAL *;
    GW vx = gmem((const W *)d.f[0]), vy = gmem((const W *)d.f[1]);
    GW vz = gmem((const W *)d.f[2]);
    auto L = [](GW p, int idx) { return S::load(WD::v(p[idx])); };
    const float HW_GLOBAL *__restrict__ M = gmem(d.mu);
    const float HW_GLOBAL *__restrict__ LM = gmem(d.lam);
    const float vx_q = L(vx, q), vy_q = L(vy, q), vz_q = L(vz, q);
    const float ex = w * (vx_q - L(vx, row + im));
    const float ey = w * (vy_q - L(vy, k * slab + jm * pitch + i));
    const float ez = w * (vz_q - L(vz, km * slab + j * pitch + i));
    const float lam = LM[q];
    const float mq = M[q];
    const float l2m = lam + 2.0f * mq;
    float inc[6];
    inc[0] = l2m * ex + lam * (ey + ez);
    inc[1] = l2m * ey + lam * (ex + ez);
    inc[2] = l2m * ez + lam * (ex + ey);
    const int q_ip = row + ip;
    const int q_jp = k * slab + jp * pitch + i;
    const int q_kp = kp * slab + j * pitch + i;
    {   // sxy at (i+1/2, j+1/2, k)
        const float a1 = L(vy, q_ip) - vy_q;
        const float a2 = L(vx, q_jp) - vx_q;
        const float g = w * (a1 + a2);
        const float m = 0.25f * ((mq + M[q_ip]) +
                                 (M[q_jp] + M[k * slab + jp * pitch + ip]));
        inc[3] = m * g;
    }
    {   // sxz at (i+1/2, j, k+1/2)
        const float a1 = L(vz, q_ip) - vz_q;
        const float a2 = L(vx, q_kp) - vx_q;
        const float g = w * (a1 + a2);
        const float m = 0.25f * ((mq + M[q_ip]) +
                                 (M[q_kp] + M[kp * slab + j * pitch + ip]));
        inc[4] = m * g;
    }
    {   // syz at (i, j+1/2, k+1/2)
        const float a1 = L(vz, q_jp) - vz_q;
        const float a2 = L(vy, q_kp) - vy_q;
        const float g = w * (a1 + a2);
        const float m = 0.25f * ((mq + M[q_jp]) +
                                 (M[q_kp] + M[kp * slab + jp * pitch + i]));
        inc[5] = m * g;
    }
#pragma unroll
    for (int f = 0; f < 6; ++f) {
        W HW_GLOBAL *sf = gmem((W *)d.f[3 + f]);
        const W old = sf[q];
        auto v = WD::v(old), c = WD::c(old);
        update_store<S, COMP>(v, c, inc[f]);
        sf[q] = WD::make(v, c);
    }
}

__device__ __forceinline__ double block_sum3(double v, double *red)
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

// Energy of the elastic state, one workgroup per (j, k) row, fp64.
template <class S>
__global__ __launch_bounds__(kThreads) void el3d_energy_kernel(
    const El3dDesc *__restrict__ dd, int st, double *__restrict__ partial)
{
    using T = typename S::store_t;
    __shared__ double red[kThreads];
    const El3dDesc &d = *dd;
    const int64_t nx = d.nx, ny = d.ny, nz = d.nz, pitch = d.pitch, slab = d.slab;
    const int64_t r = blockIdx.x;
    const int64_t k = r / ny, j = r % ny;
    const int64_t jp = wrap1(j + 1, ny), jm = wrap1(j - 1, ny);
    const int64_t kp = wrap1(k + 1, nz), km = wrap1(k - 1, nz);
    const double w = d.w;
    const T *f[9];
    for (int n = 0; n < 9; ++n)
        f[n] = (const T *)d.f[n];
    auto L = [&](int n, int64_t idx) { return (double)S::load(f[n][idx * st]); };
    const float *B = d.b, *LM = d.lam, *M = d.mu;
    double acc = 0.0;
    for (int64_t i = threadIdx.x; i < nx; i += kThreads) {
        const int64_t ip = wrap1(i + 1, nx), im = wrap1(i - 1, nx);
        const int64_t row = k * slab + j * pitch;
        const int64_t q = row + i;
        const int64_t q_ip = row + ip, q_im = row + im;
        const int64_t q_jp = k * slab + jp * pitch + i;
        const int64_t q_jm = k * slab + jm * pitch + i;
        const int64_t q_kp = kp * slab + j * pitch + i;
        const int64_t q_km = km * slab + j * pitch + i;
        const double sxx = L(3, q), syy = L(4, q), szz = L(5, q);
        const double sxy = L(6, q), sxz = L(7, q), syz = L(8, q);
        const double gx = w * ((L(3, q_ip) - sxx) + (sxy - L(6, q_jm)) +
                               (sxz - L(7, q_km)));
        const double gy = w * ((sxy - L(6, q_im)) + (L(4, q_jp) - syy) +
                               (syz - L(8, q_km)));
        const double gz = w * ((sxz - L(7, q_im)) + (syz - L(8, q_jm)) +
                               (L(5, q_kp) - szz));
        const double bq = B[q];
        const double bx = 0.5 * (bq + (double)B[q_ip]);
        const double by = 0.5 * (bq + (double)B[q_jp]);
        const double bz = 0.5 * (bq + (double)B[q_kp]);
        const double vx = L(0, q), vy = L(1, q), vz = L(2, q);
        const double vxp = vx + bx * gx;
        const double vyp = vy + by * gy;
        const double vzp = vz + bz * gz;
        double ev = (vx * vxp) / bx + (vy * vyp) / by;
        ev = ev + (vz * vzp) / bz;
        const double lam = LM[q], mu = M[q];
        const double tr = (sxx + syy) + szz;
        const double sq = (sxx * sxx + syy * syy) + szz * szz;
        const double en = (sq - (lam / (3.0 * lam + 2.0 * mu)) * (tr * tr)) /
                          (2.0 * mu);
        const double mxy = 0.25 * (((double)M[q] + (double)M[q_ip]) +
                                   ((double)M[q_jp] + (double)M[k * slab + jp * pitch + ip]));
        const double mxz = 0.25 * (((double)M[q] + (double)M[q_ip]) +
                                   ((double)M[q_kp] + (double)M[kp * slab + j * pitch + ip]));
        const double myz = 0.25 * (((double)M[q] + (double)M[q_jp]) +
                                   ((double)M[q_kp] + (double)M[kp * slab + jp * pitch + i]));
        double es = (sxy * sxy) / mxy + (sxz * sxz) / mxz;
        es = es + (syz * syz) / myz;
        acc += (ev + en) + es;
    }
    const double s = block_sum3(acc, red);
    if (threadIdx.x == 0)
        partial[r] = s;
}

// ------------------------------------------------------------- dispatch --

template <class S, int COMP>
static hipError_t el3d_tile(const El3dBatch &a, int tile, hipStream_t s)
{
    const dim3 grid(a.total_tiles), block(kThreads);
    switch (tile) {
#define HW_TILE(n)                                                              \
    case n:                                                                     \
        hipLaunchKernelGGL((el3d_velocity_kernel<S, COMP, kTiles3D[n].tx,       \
                                                 kTiles3D[n].ty>),              \
                           grid, block, 0, s, a);                               \
        hipLaunchKernelGGL((el3d_stress_kernel<S, COMP, kTiles3D[n].tx,         \
                                               kTiles3D[n].ty>),                \
                           grid, block, 0, s, a);                               \
        break;
        HW_TILE(0) HW_TILE(1) HW_TILE(2) HW_TILE(3)
#undef HW_TILE
    default:
        return hipErrorInvalidValue;
    }
    static_assert(kNumTiles3D == 4, "update the tile dispatch");
    return hipGetLastError();
}

template <class S>
static hipError_t el3d_comp(const El3dBatch &a, int comp, int tile, hipStream_t s)
{
    switch (comp) {
    case COMP_NONE: return el3d_tile<S, COMP_NONE>(a, tile, s);
    case COMP_FAST2SUM: return el3d_tile<S, COMP_FAST2SUM>(a, tile, s);
    case COMP_TWOSUM: return el3d_tile<S, COMP_TWOSUM>(a, tile, s);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_el3d_step(const El3dBatch &a, int storage, int comp,
                            int tile, hipStream_t s)
{
    if (a.total_tiles <= 0)
        return hipSuccess;
    switch (storage) {
    case HW_F32: return el3d_comp<F32>(a, comp, tile, s);
    case HW_F16: return el3d_comp<F16>(a, comp, tile, s);
    case HW_BF16: return el3d_comp<BF16>(a, comp, tile, s);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_el3d_energy(const El3dDesc *d_desc, int64_t rows,
                              int storage, int stride, double *partial,
                              hipStream_t s)
{
    switch (storage) {
    case HW_F32:
        hipLaunchKernelGGL(el3d_energy_kernel<F32>, dim3(rows), dim3(kThreads),
                           0, s, d_desc, stride, partial);
        break;
    case HW_F16:
        hipLaunchKernelGGL(el3d_energy_kernel<F16>, dim3(rows), dim3(kThreads),
                           0, s, d_desc, stride, partial);
        break;
    case HW_BF16:
        hipLaunchKernelGGL(el3d_energy_kernel<BF16>, dim3(rows), dim3(kThreads),
                           0, s, d_desc, stride, partial);
        break;
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace hw
