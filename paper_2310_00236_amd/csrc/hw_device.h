// Device-side numeric primitives: storage formats, round-to-nearest-even
// conversions and the solution updates of Alg. 1 and Alg. 2 (Sec. 4).
//
// Values of a storage format are carried in fp32 registers (every fp16 and
// bf16 value is exactly an fp32 value).  An operation of the storage format
// is an fp32 operation followed by rounding to the format: for operands with
// p <= 11 significand bits the fp32 result (24 bits >= 2p + 2) rounded once
// more equals the correctly rounded p-bit result, so this is IEEE fp16/bf16
// arithmetic.  The whole library is compiled without floating-point
// contraction, so every a*b+c below is two rounded operations.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#pragma clang fp contract(off)

namespace hw {

enum Comp { COMP_NONE = 0, COMP_FAST2SUM = 1, COMP_TWOSUM = 2, COMP_TWOSUM8 = 3 };

// ---------------------------------------------------------------- formats

struct F32 {
    using store_t = float;
    static constexpr int id = 0;
    __device__ __forceinline__ static float load(store_t x) { return x; }
    __device__ __forceinline__ static store_t store(float x) { return x; }
    __device__ __forceinline__ static float rn(float x) { return x; }
};

// Opaque copy of an fp32 value: the compiler may not fold the operation
// that produced it into the consumer.  Without it the backend merges
// "fp32 multiply, then convert to fp16" into one mixed-precision fma that
// rounds the exact product once (and turns a -0 product into +0), which is
// a different operation from the two roundings the method defines.
__device__ __forceinline__ float opaque(float x)
{
    __asm__("" : "+v"(x));
    return x;
}

struct F16 {
    using store_t = _Float16;
    static constexpr int id = 1;
    __device__ __forceinline__ static float load(store_t x) { return (float)x; }
    // fp32 -> fp16 conversion rounds to nearest even, keeps subnormals and
    // overflows to infinity.
    __device__ __forceinline__ static store_t store(float x)
    {
        return (_Float16)opaque(x);
    }
    __device__ __forceinline__ static float rn(float x)
    {
        return (float)(_Float16)opaque(x);
    }
};

struct BF16 {
    using store_t = uint16_t;
    static constexpr int id = 2;
    __device__ __forceinline__ static float load(store_t x) {
        return __uint_as_float((uint32_t)x << 16);
    }
    // fp32 -> bf16 by the hardware conversion (one instruction on gfx950):
    // round to nearest even under the default rounding mode, subnormals kept
    // (fp32 denormals are enabled in these kernels), values past the largest
    // finite bf16 become infinity, NaNs stay NaNs (payload unspecified).
    // For every non-NaN input this equals the bit-pattern rounding "add
    // 0x7fff plus the lowest kept bit, keep the top 16 bits".
    __device__ __forceinline__ static store_t store(float x) {
        return __builtin_bit_cast(store_t, (__bf16)opaque(x));
    }
    __device__ __forceinline__ static float rn(float x) { return load(store(x)); }
};

template <int ID> struct FormatOf;
template <> struct FormatOf<0> { using type = F32; };
template <> struct FormatOf<1> { using type = F16; };
template <> struct FormatOf<2> { using type = BF16; };

// ------------------------------------------------------- solution updates

// v and c hold values of format S.  inc is the fp32 increment R of the
// paper's algorithms after scaling by the material.
//   plain (Alg. 1):     v <- v (+) RN(inc)
//   compensated (Alg. 2, compensation added after scaling):
//                       y = RN(inc + c);  (v, c) <- sum(v, y)
// with sum the 3-operation form (Code 1) or the 6-operation form (Code 2).
template <class S, int COMP>
__device__ __forceinline__ void update(float &v, float &c, float inc)
{
    if constexpr (COMP == COMP_NONE) {
        float r = S::rn(inc);
        v = S::rn(v + r);
    } else {
        float y = S::rn(inc + c);
        float s = S::rn(v + y);
        if constexpr (COMP == COMP_FAST2SUM) {
            float z = S::rn(s - v);
            c = S::rn(y - z);
        } else {
            float pa = S::rn(s - y);
            float pb = S::rn(s - pa);
            float da = S::rn(v - pa);
            float db = S::rn(y - pb);
            c = S::rn(da + db);
        }
        v = s;
    }
}

// The same updates on values held in the storage type.  For fp16 the
// compensated sum runs on native half-precision instructions: each of its
// operations has fp16 operands, so the half-precision instruction's result
// is the correctly rounded fp16 result the definition asks for.  Only the
// narrowing of the fp32 increment goes through an explicit rounding.
template <class S, int COMP>
__device__ __forceinline__ void update_store(typename S::store_t &v,
                                             typename S::store_t &c, float inc)
{
    if constexpr (S::id == F16::id) {
        if constexpr (COMP == COMP_NONE) {
            const _Float16 r = (_Float16)opaque(inc);
            v = v + r;
        } else {
            const _Float16 y = (_Float16)opaque(inc + (float)c);
            const _Float16 s = v + y;
            if constexpr (COMP == COMP_FAST2SUM) {
                const _Float16 z = s - v;
                c = y - z;
            } else {
                const _Float16 pa = s - y;
                const _Float16 pb = s - pa;
                const _Float16 da = v - pa;
                const _Float16 db = y - pb;
                c = da + db;
            }
            v = s;
        }
    } else {
        float vf = S::load(v), cf = COMP ? S::load(c) : 0.0f;
        update<S, COMP>(vf, cf, inc);
        v = S::store(vf);
        if (COMP)
            c = S::store(cf);
    }
}

// Round a double to the nearest value with `prec` significand bits and
// smallest normal exponent `emin` (subnormal spacing 2^(emin-prec+1)), ties
// to even, by integer arithmetic on the binary64 encoding (a double to
// float to half conversion would round twice).  Results beyond maxfin become
// infinity.  The result is exactly representable in fp32.
__device__ inline double round_double(double x, int prec, int emin, double maxfin)
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

// A double rounded once to the storage format.
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

// v <- v (+) y and, unless COMP_NONE, c <- the error (Fast2Sum or TwoSum),
// all in format S; y is already a value of the format.
template <class S, int COMP = COMP_TWOSUM>
__device__ __forceinline__ void update_sum_store(typename S::store_t &v,
                                                 typename S::store_t &c,
                                                 typename S::store_t y)
{
    if constexpr (S::id == F16::id) {
        const _Float16 s = v + y;
        if constexpr (COMP == COMP_FAST2SUM) {
            const _Float16 z = s - v;
            c = y - z;
        } else if constexpr (COMP != COMP_NONE) {
            const _Float16 pa = s - y;
            const _Float16 pb = s - pa;
            const _Float16 da = v - pa;
            const _Float16 db = y - pb;
            c = da + db;
        }
        v = s;
    } else {
        const float vf = S::load(v), yf = S::load(y);
        const float s = S::rn(vf + yf);
        if constexpr (COMP == COMP_FAST2SUM) {
            const float z = S::rn(s - vf);
            c = S::store(S::rn(yf - z));
        } else if constexpr (COMP != COMP_NONE) {
            const float pa = S::rn(s - yf);
            const float pb = S::rn(s - pa);
            const float da = S::rn(vf - pa);
            const float db = S::rn(yf - pb);
            c = S::store(S::rn(da + db));
        }
        v = S::store(s);
    }
}

// The updates with an fp64 increment (the stencil evaluated in fp64): the
// increment, or increment plus compensation, is rounded once to the storage
// format; the sum that follows is the same as above.
template <class S, int COMP>
__device__ __forceinline__ void update_store_d(typename S::store_t &v,
                                               typename S::store_t &c, double inc)
{
    using T = typename S::store_t;
    const T y = COMP == COMP_NONE ? from_double<S>(inc)
                                  : from_double<S>(inc + (double)S::load(c));
    update_sum_store<S, COMP>(v, c, y);
}

// Workgroup b of n renumbered so that each of NXCD dies, which receive the
// workgroups of a launch round-robin, works through one contiguous range
// (neighbouring rows or tiles then share that die's L2).
template <int NXCD>
__device__ __forceinline__ int32_t xcd_band(int32_t b, int32_t n)
{
    const int32_t per = n / NXCD, rem = n % NXCD;
    const int32_t x = b % NXCD, r = b / NXCD;
    return x * per + (x < rem ? x : rem) + r;
}

// ------------------------------------------------- fp64 workgroup sum
//
// Sum of one fp64 value per thread over a workgroup of NT threads, in an
// order fixed by NT alone: a butterfly across each wavefront's 64 lanes
// (lane 0 keeps its result), then the wavefront sums added in wavefront
// order.  Every thread returns the total; red holds NT / 64 doubles and is
// written once, so a kernel calls this at most once.
template <int NT>
__device__ __forceinline__ double block_sum_f64(double v, double *red)
{
    static_assert(NT % 64 == 0 && NT >= 64, "whole wavefronts");
    for (int m = 32; m > 0; m >>= 1)
        v = v + __shfl_xor(v, m, 64);
    if ((threadIdx.x & 63u) == 0)
        red[threadIdx.x >> 6] = v;
    __syncthreads();
    double s = red[0];
    for (int w = 1; w < NT / 64; ++w)
        s = s + red[w];
    return s;
}

// ------------------------------------------ 8-bit compensation word
//
// With COMP_TWOSUM8 the TwoSum error t of a sum s (|t| <= ulp(s)/2, ulp the
// spacing of s's binade, the subnormal spacing for zero and subnormal s) is
// kept as the integer q = round(t / ulp(s) * 2^7), ties to even, |q| <= 64,
// one byte per cell next to the value array, and read back as
// q * ulp(s) / 2^7.  Both scalings are exact powers of two.

// Biased exponent field of s, and whether s is finite.
__device__ __forceinline__ uint32_t exp_field(_Float16 s)
{
    return __builtin_amdgcn_ubfe((uint32_t)__builtin_bit_cast(uint16_t, s), 10, 5);
}
__device__ __forceinline__ uint32_t exp_field_bf16(uint16_t s)
{
    return __builtin_amdgcn_ubfe((uint32_t)s, 7, 8);
}

// One step of q is ulp(s) / 2^7, with ulp(s) = 2^(max(E,1) - 25) for fp16
// (E the exponent field; E = 0 gives the subnormal spacing 2^-24) and
// 2^(max(E,1) - 134) for bf16.  For fp16 the power of two is a normal fp32
// number, built from its exponent field; for bf16 it can leave the fp32
// range, so the scaling goes through ldexpf.  Either way it is exact.
template <class S>
__device__ __forceinline__ float comp8_decode(int8_t q, typename S::store_t s)
{
    if constexpr (S::id == F16::id) {
        const uint32_t e = max(exp_field(s), 1u);
        return (float)q * __uint_as_float((e + 95u) << 23);   // q 2^(e - 32)
    } else {
        const int e = (int)max(exp_field_bf16(s), 1u);
        return ldexpf((float)q, e - 141);
    }
}

// q = round(t / ulp(s) * 2^7), ties to even; 0 when s or t is not finite
// (an operation of the sum overflowed).  |t| <= ulp(s)/2 keeps |q| <= 64.
//
// t is the error of the six-operation sum s = v + y, and only t is tested:
// when s is not finite t is NaN (s is NaN, or s - y or s - pa subtracts two
// infinities of one sign), so a finite t implies a finite s.
//
// x = t / ulp(s) * 2^7 is rounded by one addition of 1.5 * 2^m, m the
// fraction bits of the format the addition is done in: the spacing there
// is 1, so the round-to-nearest-even sum is round(x) + 1.5 * 2^m exactly,
// and its low byte is round(x) in two's complement.  For fp16 the scaling
// and the addition are fp16 operations: x has at most 11 significant bits,
// |x| <= 64 and no bit below 2^-22, so it is exact in fp16.  For bf16 they
// are fp32 operations (an x below the fp32 range rounds to 0 either way).
// No branch either way.
__device__ __forceinline__ _Float16 comp8_scaled_f16(_Float16 t, _Float16 s)
{
    const int e = (int)max(exp_field(s), 1u);
    return __builtin_amdgcn_ldexph(t, 32 - e);                     // t 2^(32 - e)
}
__device__ __forceinline__ int8_t comp8_pick_f16(_Float16 r, _Float16 t)
{
    const int8_t q = (int8_t)(__builtin_bit_cast(uint16_t, r) & 0xffu);
    return __builtin_isfinite(t) ? q : (int8_t)0;
}
constexpr float kRound16 = 1536.0f;          // 1.5 * 2^10
constexpr float kRound32 = 12582912.0f;      // 1.5 * 2^23

template <class S>
__device__ __forceinline__ int8_t comp8_encode(float t, typename S::store_t s)
{
    if constexpr (S::id == F16::id) {
        const _Float16 th = (_Float16)t;                            // t is an fp16 value
        return comp8_pick_f16(comp8_scaled_f16(th, s) + (_Float16)kRound16, th);
    } else {
        const int e = (int)max(exp_field_bf16(s), 1u);
        const float r = ldexpf(t, 141 - e) + kRound32;
        const int8_t q = (int8_t)(__float_as_uint(r) & 0xffu);
        return __builtin_isfinite(t) ? q : (int8_t)0;
    }
}

// The compensated update with the 8-bit word: y = RN(inc + t_old), the
// 6-operation sum of v and y in format S, the new error re-quantised.
template <class S>
__device__ __forceinline__ void update_store8(typename S::store_t &v, int8_t &q, float inc)
{
    const float told = comp8_decode<S>(q, v);
    if constexpr (S::id == F16::id) {
        const _Float16 y = (_Float16)opaque(inc + told);
        const _Float16 s = v + y;
        const _Float16 pa = s - y;
        const _Float16 pb = s - pa;
        const _Float16 da = v - pa;
        const _Float16 db = y - pb;
        const _Float16 t = da + db;
        q = comp8_pick_f16(comp8_scaled_f16(t, s) + (_Float16)kRound16, t);
        v = s;
    } else {
        const float vf = S::load(v);
        const float y = S::rn(inc + told);
        const float s = S::rn(vf + y);
        const float pa = S::rn(s - y);
        const float pb = S::rn(s - pa);
        const float da = S::rn(vf - pa);
        const float db = S::rn(y - pb);
        const float t = S::rn(da + db);
        v = S::store(s);
        q = comp8_encode<S>(t, v);
    }
}

// Two independent fp16 cells at once: the two narrowings of the right-hand
// sides are one packed conversion, the two six-operation sums and the two
// rounding additions packed half-precision instructions.  Lane by lane these
// are the operations of update_store8, each correctly rounded, so the bits
// are those of two single updates.
__device__ __forceinline__ void update_pair8_f16(_Float16 &v0, int8_t &q0, _Float16 &v1,
                                                 int8_t &q1, float inc0, float inc1)
{
    typedef _Float16 h2 __attribute__((ext_vector_type(2)));
    typedef float f2 __attribute__((ext_vector_type(2)));
    f2 a = {inc0 + comp8_decode<F16>(q0, v0), inc1 + comp8_decode<F16>(q1, v1)};
    __asm__("" : "+v"(a));        // no fusing into the narrowing (see opaque)
    const h2 y = __builtin_convertvector(a, h2);
    const h2 v = {v0, v1};
    const h2 s = v + y;
    const h2 pa = s - y;
    const h2 pb = s - pa;
    const h2 da = v - pa;
    const h2 db = y - pb;
    const h2 t = da + db;
    const h2 x = {comp8_scaled_f16(t[0], s[0]), comp8_scaled_f16(t[1], s[1])};
    const h2 r = x + h2{(_Float16)kRound16, (_Float16)kRound16};
    q0 = comp8_pick_f16(r[0], t[0]);
    q1 = comp8_pick_f16(r[1], t[1]);
    v0 = s[0];
    v1 = s[1];
}

// The same with an fp64 increment (stencil in fp64).
template <class S>
__device__ __forceinline__ void update_store8_d(typename S::store_t &v, int8_t &q, double inc)
{
    using T = typename S::store_t;
    const T y = from_double<S>(inc + (double)comp8_decode<S>(q, v));
    T c = T(0);
    update_sum_store<S>(v, c, y);
    q = comp8_encode<S>(S::load(c), v);
}

// Memory word of one field at one cell: the value alone, or the value and
// its compensation term side by side.
template <class S, int COMP>
struct Word {
    using T = typename S::store_t;
    typedef T type __attribute__((ext_vector_type(2)));   // (value, comp)
    __device__ __forceinline__ static T v(type w) { return w[0]; }
    __device__ __forceinline__ static T c(type w) { return w[1]; }
    __device__ __forceinline__ static type make(T v, T c) { return type{v, c}; }
};

template <class S>
struct Word<S, COMP_NONE> {
    using T = typename S::store_t;
    using type = T;
    __device__ __forceinline__ static T v(type w) { return w; }
    __device__ __forceinline__ static T c(type) { return T(0); }
    __device__ __forceinline__ static type make(T v, T) { return v; }
};

// Pointers into device memory in the global address space.  The buffers
// reach the kernels through descriptors as generic pointers; without the
// cast every access would be a flat instruction, which the hardware counts
// against both the vector-memory and the LDS counters, so each wait for an
// LDS read would also wait for outstanding global stores.
#define HW_GLOBAL __attribute__((address_space(1)))
template <class T>
__device__ __forceinline__ T HW_GLOBAL *gmem(T *p)
{
    return (T HW_GLOBAL *)p;
}
template <class T>
__device__ __forceinline__ const T HW_GLOBAL *gmem(const T *p)
{
    return (const T HW_GLOBAL *)p;
}

// Periodic index for offsets of at most one period beyond [0, n).
__device__ __forceinline__ int64_t wrap1(int64_t i, int64_t n)
{
    return i < 0 ? i + n : (i >= n ? i - n : i);
}

// Periodic index for any offset (tiny grids where a halo spans several
// periods).
__device__ __forceinline__ int64_t wrapn(int64_t i, int64_t n)
{
    int64_t r = i % n;
    return r < 0 ? r + n : r;
}

}  // namespace hw
