// gpu_checks.hip - device checks of two exactness facts the simulation kernel
// relies on, run against the kernel's own device functions (the template is
// included as it is).
//
//  * The SR conversions read only the top B bits of their random operand
//    (B = 13 for fp16: bits 31..19; B = 16 for bf16: bits 31..16), so a
//    B-bit random field shifted to the top may carry the neighbouring
//    fields below it.
//  * the short fma divisions return the IEEE quotient: div_rn_log for every
//    log argument, div_rn_inrange for -ln(u1) / a0 over the fp16 ranges,
//    div_rn_log64 for binary64 log arguments (a hashed sample and the edges).
//
// Test infrastructure: built next to the tests, loaded by them only.
#include <hip/hip_runtime.h>

#include <cstdint>

#define SSA_N_ITEMS 1
#include "../paper_2605_00479_amd/csrc/ssa_device.hip"

namespace {

__device__ __forceinline__ uint32_t mix64(uint64_t x)
{
    x ^= x >> 33;
    x *= 0xff51afd7ed558ccdull;
    x ^= x >> 33;
    x *= 0xc4ceb9fe1a85ec53ull;
    x ^= x >> 33;
    return (uint32_t)x;
}

__global__ void check_sr_lowbits(unsigned long long n, unsigned long long *cnt)
{
    const unsigned long long stride = (unsigned long long)gridDim.x * blockDim.x;
    for (unsigned long long i = blockIdx.x * (unsigned long long)blockDim.x + threadIdx.x; i < n; i += stride) {
        uint32_t vb = mix64(2 * i), w = mix64(2 * i + 1);
        // magnitudes 2^-37 .. 2^33: fp16 subnormals, normals and overflow, bf16 normals
        vb = (vb & 0x807FFFFFu) | ((90u + (vb >> 23) % 71u) << 23);
        const float v = __uint_as_float(vb);
        if (__float_as_uint(sr_f16(v, w)) != __float_as_uint(sr_f16(v, w & 0xFFF80000u)))
            atomicAdd(&cnt[0], 1ull);
        if (__float_as_uint(sr_bf16(v, w)) != __float_as_uint(sr_bf16(v, w & 0xFFFF0000u)))
            atomicAdd(&cnt[1], 1ull);
    }
}

// every binary32 f in [1/2, 2): s = (f - 1) / (f + 1), the log's argument
__global__ void check_div_log(unsigned long long *cnt)
{
    const uint32_t lo = 0x3F000000u, hi = 0x40000000u;
    for (uint32_t b = lo + blockIdx.x * blockDim.x + threadIdx.x; b < hi; b += gridDim.x * blockDim.x) {
        const float f = __uint_as_float(b);
        const float num = f - 1.0f, den = f + 1.0f;
        if (__float_as_uint(div_rn_log(num, den)) != __float_as_uint(num / den))
            atomicAdd(&cnt[0], 1ull);
    }
}

// numerators: zero and every `step`-th binary32 in [2^-26, 32); per numerator
// n_den denominators in [2^-24, 2^27) drawn by a hash
__global__ void check_div_tau(uint32_t step, int n_den, unsigned long long *cnt)
{
    const uint32_t lo = 0x32800000u, hi = 0x42000000u;
    const uint32_t count = (hi - lo) / step + 1;
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < count; i += gridDim.x * blockDim.x) {
        const float L = i == count - 1 ? 0.0f : __uint_as_float(lo + i * step);
        for (int j = 0; j < n_den; ++j) {
            const uint32_t h = mix64(((uint64_t)i << 8) | (uint32_t)j);
            const uint32_t e = 103u + h % 51u;
            const float a0 = __uint_as_float((e << 23) | (h >> 9));
            if (__float_as_uint(div_rn_inrange(L, a0)) != __float_as_uint(L / a0))
                atomicAdd(&cnt[0], 1ull);
        }
    }
}

// binary64 f in [1/2, 2): n hashed mantissas per exponent (f in [1/2, 1) and
// [1, 2)), plus the 64 mantissas at each end of both binades
__global__ void check_div_log64(unsigned long long n, unsigned long long *cnt)
{
    const unsigned long long total = 2 * (n + 128);
    for (unsigned long long i = blockIdx.x * (unsigned long long)blockDim.x + threadIdx.x; i < total;
         i += (unsigned long long)gridDim.x * blockDim.x) {
        const unsigned long long j = i >> 1;
        const uint64_t ex = (i & 1) ? 0x3FE0000000000000ull : 0x3FF0000000000000ull;
        uint64_t m;
        if (j < 64)
            m = j;
        else if (j < 128)
            m = 0x000FFFFFFFFFFFFFull - (j - 64);
        else
            m = (((uint64_t)mix64(j) << 32) | mix64(j ^ 0x9E3779B97F4A7C15ull)) & 0x000FFFFFFFFFFFFFull;
        const double f = __longlong_as_double((long long)(ex | m));
        const double num = f - 1.0, den = f + 1.0;
        if (__double_as_longlong(div_rn_log64(num, den)) != __double_as_longlong(num / den))
            atomicAdd(&cnt[0], 1ull);
    }
}

int finish(unsigned long long *d, unsigned long long *h, int n)
{
    if (hipDeviceSynchronize() != hipSuccess)
        return 3;
    if (hipMemcpy(h, d, n * sizeof(unsigned long long), hipMemcpyDeviceToHost) != hipSuccess)
        return 3;
    return hipFree(d) == hipSuccess ? 0 : 3;
}

int alloc_counters(unsigned long long **d, int n)
{
    if (hipMalloc(d, n * sizeof(unsigned long long)) != hipSuccess)
        return 2;
    return hipMemset(*d, 0, n * sizeof(unsigned long long)) == hipSuccess ? 0 : 3;
}

}  // namespace

extern "C" {

// Mismatches of the SR conversions with and without the operand's bits below
// the top B, over n random (value, word) pairs: out[0] fp16, out[1] bf16.
int gpu_check_sr_lowbits(unsigned long long n, unsigned long long *out)
{
    unsigned long long *d = nullptr;
    int rc = alloc_counters(&d, 2);
    if (rc)
        return rc;
    check_sr_lowbits<<<4096, 256>>>(n, d);
    return finish(d, out, 2);
}

// Mismatches against the IEEE division: out[0] div_rn_log over every log
// argument, out[1] div_rn_inrange over the -ln(u1) / a0 sweep (see check_div_tau).
int gpu_check_division(unsigned int step, int n_den, unsigned long long *out)
{
    if (step == 0 || n_den < 1)
        return 4;
    unsigned long long *d = nullptr;
    int rc = alloc_counters(&d, 2);
    if (rc)
        return rc;
    check_div_log<<<4096, 256>>>(d);
    check_div_tau<<<4096, 256>>>(step, n_den, d + 1);
    return finish(d, out, 2);
}

// Mismatches of div_rn_log64 against the IEEE binary64 division over
// 2 (n + 128) log arguments (see check_div_log64): out[0].
int gpu_check_division64(unsigned long long n, unsigned long long *out)
{
    unsigned long long *d = nullptr;
    int rc = alloc_counters(&d, 1);
    if (rc)
        return rc;
    check_div_log64<<<4096, 256>>>(n, d);
    return finish(d, out, 1);
}

}  // extern "C"
