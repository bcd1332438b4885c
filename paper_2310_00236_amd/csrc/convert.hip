// Conversions between fp64 arrays in the caller's layout (row-major, no
// padding) and the device layout (padded row pitch), and material
// preprocessing.
#include "hw_device.h"
#include "hw_internal.h"

#pragma clang fp contract(off)

namespace hw {

// Round a double to the nearest value with `prec` significand bits and
// smallest normal exponent `emin` (subnormal spacing 2^(emin-prec+1)), ties
// to even, by integer arithmetic on the binary64 encoding.  Results beyond
// maxfin become infinity.  The result is exactly representable in fp32.
__device__ double round_double(double x, int prec, int emin, double maxfin)
{
    const uint64_t u = (uint64_t)__double_as_longlong(x);
    const uint64_t sign = u & 0x8000000000000000ull;
    const uint64_t mag = u ^ sign;
    if (mag >= 0x7ff0000000000000ull || mag == 0)
        return x;                                   // inf, nan, zero
    const int ebits = (int)(mag >> 52);
    if (ebits == 0)                                 // below 2^-1022: tiny
        return __longlong_as_double((long long)sign);
    const int e = ebits - 1023;                     // exponent of leading bit
    const uint64_t m = (mag & 0x000fffffffffffffull) | 0x0010000000000000ull;
    const int lead = e < emin ? emin : e;
    // value = m * 2^(e-52); quantum = 2^(lead-prec+1); drop the low bits
    const int drop = 52 - (prec - 1) + (lead - e);
    if (drop > 60)
        return __longlong_as_double((long long)sign);
    uint64_t kept = m >> drop;
    const uint64_t rem = m & ((1ull << drop) - 1);
    const uint64_t half = 1ull << (drop - 1);
    if (rem > half || (rem == half && (kept & 1)))
        ++kept;
    double r = ldexp((double)kept, lead - prec + 1);
    if (r > maxfin)
        r = __longlong_as_double(0x7ff0000000000000ll);
    return sign ? -r : r;
}

template <class S>
__device__ __forceinline__ typename S::store_t from_double(double x);
template <>
__device__ __forceinline__ float from_double<F32>(double x)
{
    return (float)x;   // fp64 -> fp32 conversion rounds to nearest even
}
template <>
__device__ __forceinline__ _Float16 from_double<F16>(double x)
{
    return F16::store((float)round_double(x, 11, -14, 65504.0));
}
template <>
__device__ __forceinline__ uint16_t from_double<BF16>(double x)
{
    return BF16::store((float)round_double(x, 8, -126, 0x1.fep127));
}

template <class S>
__global__ __launch_bounds__(kThreads) void to_storage_kernel(
    const double *__restrict__ src, typename S::store_t *__restrict__ dst,
    int64_t nx, int64_t rows, int64_t pitch, int stride, int offset,
    double scale)
{
    const int64_t n = nx * rows;
    for (int64_t t = blockIdx.x * (int64_t)kThreads + threadIdx.x; t < n;
         t += (int64_t)gridDim.x * kThreads) {
        const int64_t r = t / nx, i = t % nx;
        dst[(r * pitch + i) * stride + offset] = from_double<S>(src[t] * scale);
    }
}

template <class S>
__global__ __launch_bounds__(kThreads) void from_storage_kernel(
    const typename S::store_t *__restrict__ src, double *__restrict__ dst,
    int64_t nx, int64_t rows, int64_t pitch, int stride, int offset,
    double scale)
{
    const int64_t n = nx * rows;
    for (int64_t t = blockIdx.x * (int64_t)kThreads + threadIdx.x; t < n;
         t += (int64_t)gridDim.x * kThreads) {
        const int64_t r = t / nx, i = t % nx;
        dst[t] = (double)S::load(src[(r * pitch + i) * stride + offset]) * scale;
    }
}

__global__ __launch_bounds__(kThreads) void fill_zero_kernel(uint32_t *dst,
                                                             int64_t n)
{
    for (int64_t t = blockIdx.x * (int64_t)kThreads + threadIdx.x; t < n;
         t += (int64_t)gridDim.x * kThreads)
        dst[t] = 0u;
}

// Material value in fp32: v itself, or its reciprocal (buoyancy 1/rho),
// each formed in fp64 and rounded once to fp32.
__global__ __launch_bounds__(kThreads) void material_kernel(
    const double *__restrict__ src, float *__restrict__ dst, int reciprocal,
    int64_t nx, int64_t rows, int64_t pitch)
{
    const int64_t n = nx * rows;
    for (int64_t t = blockIdx.x * (int64_t)kThreads + threadIdx.x; t < n;
         t += (int64_t)gridDim.x * kThreads) {
        const int64_t r = t / nx, i = t % nx;
        const double v = reciprocal ? 1.0 / src[t] : src[t];
        dst[r * pitch + i] = (float)v;
    }
}

static dim3 grid_for(int64_t n)
{
    int64_t g = (n + kThreads - 1) / kThreads;
    if (g > 65536)
        g = 65536;
    if (g < 1)
        g = 1;
    return dim3((unsigned)g);
}

hipError_t launch_to_storage(const double *src, void *dst, int storage,
                             int64_t nx, int64_t rows, int64_t pitch,
                             int stride, int offset, double scale,
                             hipStream_t s)
{
    const dim3 g = grid_for(nx * rows), b(kThreads);
    switch (storage) {
    case HW_F32:
        hipLaunchKernelGGL(to_storage_kernel<F32>, g, b, 0, s, src,
                           (float *)dst, nx, rows, pitch, stride, offset, scale);
        break;
    case HW_F16:
        hipLaunchKernelGGL(to_storage_kernel<F16>, g, b, 0, s, src,
                           (_Float16 *)dst, nx, rows, pitch, stride, offset, scale);
        break;
    case HW_BF16:
        hipLaunchKernelGGL(to_storage_kernel<BF16>, g, b, 0, s, src,
                           (uint16_t *)dst, nx, rows, pitch, stride, offset, scale);
        break;
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_from_storage(const void *src, double *dst, int storage,
                               int64_t nx, int64_t rows, int64_t pitch,
                               int stride, int offset, double scale,
                               hipStream_t s)
{
    const dim3 g = grid_for(nx * rows), b(kThreads);
    switch (storage) {
    case HW_F32:
        hipLaunchKernelGGL(from_storage_kernel<F32>, g, b, 0, s,
                           (const float *)src, dst, nx, rows, pitch, stride, offset, scale);
        break;
    case HW_F16:
        hipLaunchKernelGGL(from_storage_kernel<F16>, g, b, 0, s,
                           (const _Float16 *)src, dst, nx, rows, pitch, stride, offset, scale);
        break;
    case HW_BF16:
        hipLaunchKernelGGL(from_storage_kernel<BF16>, g, b, 0, s,
                           (const uint16_t *)src, dst, nx, rows, pitch, stride, offset, scale);
        break;
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_fill_zero(void *dst, size_t bytes, hipStream_t s)
{
    const int64_t n = (int64_t)(bytes / 4);
    hipLaunchKernelGGL(fill_zero_kernel, grid_for(n), dim3(kThreads), 0, s,
                       (uint32_t *)dst, n);
    return hipGetLastError();
}

hipError_t launch_material(const double *src, float *dst, int reciprocal,
                           int64_t nx, int64_t rows, int64_t pitch,
                           hipStream_t s)
{
    hipLaunchKernelGGL(material_kernel, grid_for(nx * rows), dim3(kThreads), 0,
                       s, src, dst, reciprocal, nx, rows, pitch);
    return hipGetLastError();
}

}  // namespace hw
