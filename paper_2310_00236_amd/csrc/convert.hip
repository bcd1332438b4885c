// Conversions between fp64 arrays in the caller's layout (row-major, no
// padding) and the device layout (padded row pitch), and material
// preprocessing.
#include "hw_device.h"
#include "hw_internal.h"

#pragma clang fp contract(off)

namespace hw {

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

template <class S>
__global__ __launch_bounds__(kThreads) void comp8_kernel(
    const typename S::store_t *__restrict__ v, const int8_t *__restrict__ q,
    double *__restrict__ dst, int64_t nx, int64_t rows, int64_t pitch,
    double scale)
{
    const int64_t n = nx * rows;
    for (int64_t t = blockIdx.x * (int64_t)kThreads + threadIdx.x; t < n;
         t += (int64_t)gridDim.x * kThreads) {
        const int64_t r = t / nx, i = t % nx;
        const int64_t e = r * pitch + i;
        dst[t] = (double)comp8_decode<S>(q[e], v[e]) * scale;
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

hipError_t launch_comp8_to_double(const void *values, size_t comp_off, double *dst,
                                  int storage, int64_t nx, int64_t rows,
                                  int64_t pitch, double scale, hipStream_t s)
{
    const dim3 g = grid_for(nx * rows), b(kThreads);
    const int8_t *q = (const int8_t *)((const char *)values + comp_off);
    switch (storage) {
    case HW_F16:
        hipLaunchKernelGGL(comp8_kernel<F16>, g, b, 0, s, (const _Float16 *)values, q,
                           dst, nx, rows, pitch, scale);
        break;
    case HW_BF16:
        hipLaunchKernelGGL(comp8_kernel<BF16>, g, b, 0, s, (const uint16_t *)values, q,
                           dst, nx, rows, pitch, scale);
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
