// valu_peak.hip - measured VALU issue cost per instruction class on gfx950.
//
// Each kernel gives every lane CH independent dependency chains of a single
// instruction class; the loop body holds STEPS x CH copies of that instruction
// and no other VALU work, so the loop's own branch is amortised over 16 steps
// of every chain. Classes written as inline asm (plain adds and round trips
// would fold) carry one s_nop 0 between dependent asm blocks, which the
// compiler adds because it cannot see what the asm is; in the one-chain shape
// this adds a wait state per step. Three shapes are measured per class:
//   8 waves per SIMD, 8 chains : the SIMD's issue throughput for the class;
//   1 wave per SIMD,  8 chains : what one wave alone can issue;
//   1 wave per SIMD,  1 chain  : the dependent-issue latency of the class.
// valu_peak_run_shape() reports lane-steps per second; the SIMD cycles per
// wave64 step follow as cycles = SIMDs x clock x 64 / rate. In the one-wave
// shapes that is the time between two issues of the same wave.
//
// hbm_copy_run() launches hbm_copy_kernel, a plain 16-byte-per-lane copy of a
// known size: the memory counters a profiler reads for it calibrate the same
// counters read for other kernels (bytes counted per byte moved).
#include <hip/hip_runtime.h>

#include <cstdint>

#define STEPS 16

typedef _Float16 half_v2 __attribute__((ext_vector_type(2)));

enum {
    OP_ADD_U32 = 0,       // v_add_u32
    OP_BITOP3 = 1,        // v_bitop3_b32
    OP_MAD_U64 = 2,       // v_mad_u64_u32
    OP_MUL_F32 = 3,       // v_mul_f32
    OP_FMA_F32 = 4,       // v_fma_f32 (as v_fmamk_f32)
    OP_MUL_F64 = 5,       // v_mul_f64
    OP_FMA_F64 = 6,       // v_fma_f64
    OP_RCP_F32 = 7,       // v_rcp_f32
    OP_RCP_F64 = 8,       // v_rcp_f64
    OP_CVT_SR_F16 = 9,    // v_cvt_sr_f16_f32 + v_cvt_f32_f16 (pair)
    OP_CVT_F16 = 10,      // v_cvt_f16_f32 + v_cvt_f32_f16 (pair)
    OP_ADD_F32 = 11,      // v_add_f32
    OP_ADD_F64 = 12,      // v_add_f64
    OP_CVT_F32_I32 = 13,  // v_cvt_f32_i32 + v_cvt_i32_f32 (pair)
    OP_MUL_HI_U32 = 14,   // v_mul_hi_u32 + v_or_b32 (pair)
    OP_CNDMASK = 15,      // v_cndmask_b32 with an SGPR-pair mask written once
    OP_ADD_F32_VV = 16,   // v_add_f32 with two VGPR operands
    OP_COUNT = 17
};

template <int OP, int CH>
__global__ void __launch_bounds__(256) valu_kernel(uint32_t *out, int iters, uint32_t seed)
{
    const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    uint32_t u[CH];
    double d[CH];
    float f[CH];
    int32_t s[CH];
#pragma unroll
    for (int c = 0; c < CH; ++c) {
        u[c] = t * 2654435761u + (uint32_t)c * 40503u + seed;
        d[c] = 1.0 + (double)(u[c] & 0xFFFF) * 1e-9;
        f[c] = 1.0f + (float)(u[c] & 0xFFFF) * 1e-7f;
        s[c] = (int32_t)(u[c] & 0xFFFFF);
    }
    const uint32_t k = seed | 1u;
    const uint32_t k2 = seed * 3u + 5u;
    const uint64_t mask = ~(uint64_t)(seed >> 31);   // every lane, not known at compile time
    const uint32_t alt = k2 ^ t;
    const float fv = __uint_as_float(0x33800000u | (t & 0xFFFFu));   // lane-varying, in a VGPR
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int st = 0; st < STEPS; ++st)
#pragma unroll
        for (int c = 0; c < CH; ++c) {
            if constexpr (OP == OP_ADD_U32) {
                // register-only VALU instruction; a plain add chain would fold into one multiply
                __asm__ volatile("v_add_u32_e32 %0, %1, %0" : "+v"(u[c]) : "v"(alt));
            } else if constexpr (OP == OP_BITOP3) {
                u[c] = __builtin_amdgcn_bitop3_b32(u[c], k2, k, 0x96);
            } else if constexpr (OP == OP_MAD_U64) {
                u[c] = (uint32_t)(((uint64_t)u[c] * (uint64_t)0xD2511F53u + k) >> 32);
            } else if constexpr (OP == OP_MUL_F32) {
                f[c] = f[c] * 0.9999999f;
            } else if constexpr (OP == OP_FMA_F32) {
                f[c] = __builtin_fmaf(f[c], 0.9999999f, __uint_as_float(k2 & 0x007FFFFF));
            } else if constexpr (OP == OP_MUL_F64) {
                d[c] = d[c] * 0.9999999999;
            } else if constexpr (OP == OP_FMA_F64) {
                d[c] = __builtin_fma(d[c], 0.9999999999, 1e-300);
            } else if constexpr (OP == OP_RCP_F32) {
                f[c] = __builtin_amdgcn_rcpf(f[c]);
            } else if constexpr (OP == OP_RCP_F64) {
                d[c] = __builtin_amdgcn_rcp(d[c]);
            } else if constexpr (OP == OP_CVT_SR_F16) {
                f[c] = (float)__builtin_amdgcn_cvt_sr_f16_f32(__builtin_bit_cast(half_v2, f[c]), f[c], k, false)[0];
            } else if constexpr (OP == OP_CVT_F16) {
                // register-only VALU instructions; the round trip is idempotent and would fold
                __asm__ volatile("v_cvt_f16_f32_e32 %0, %0\n\tv_cvt_f32_f16_e32 %0, %0" : "+v"(f[c]));
            } else if constexpr (OP == OP_ADD_F32) {
                f[c] = f[c] + __uint_as_float(k2 & 0x007FFFFF);
            } else if constexpr (OP == OP_ADD_F64) {
                d[c] = d[c] + 1e-300;
            } else if constexpr (OP == OP_CVT_F32_I32) {
                // register-only VALU instructions; the round trip is idempotent and would fold
                __asm__ volatile("v_cvt_f32_i32_e32 %0, %0\n\tv_cvt_i32_f32_e32 %0, %0" : "+v"(s[c]));
            } else if constexpr (OP == OP_MUL_HI_U32) {
                u[c] = __umulhi(u[c], 0xD2511F53u) | k;
            } else if constexpr (OP == OP_ADD_F32_VV) {
                f[c] = f[c] + fv;
            } else if constexpr (OP == OP_CNDMASK) {
                // register-only VALU instruction (no memory access)
                __asm__ volatile("v_cndmask_b32_e64 %0, %1, %0, %2" : "+v"(u[c]) : "v"(alt), "s"(mask));
            }
        }
    }
    uint32_t acc = 0;
#pragma unroll
    for (int c = 0; c < CH; ++c)
        acc ^= u[c] ^ (uint32_t)(d[c] * 1e6) ^ __float_as_uint(f[c]) ^ (uint32_t)s[c];
    out[t] = acc;
}

template <int OP, int CH>
static void launch_op(int grid, int block, uint32_t *out, int iters)
{
    valu_kernel<OP, CH><<<grid, block>>>(out, iters, 7u);
}

typedef void (*launch_fn)(int, int, uint32_t *, int);

template <int CH>
struct Table {
    static constexpr launch_fn fn[OP_COUNT] = {
        launch_op<0, CH>,  launch_op<1, CH>,  launch_op<2, CH>,  launch_op<3, CH>,
        launch_op<4, CH>,  launch_op<5, CH>,  launch_op<6, CH>,  launch_op<7, CH>,
        launch_op<8, CH>,  launch_op<9, CH>,  launch_op<10, CH>, launch_op<11, CH>,
        launch_op<12, CH>, launch_op<13, CH>, launch_op<14, CH>, launch_op<15, CH>,
        launch_op<16, CH>};
};

__global__ void __launch_bounds__(256) hbm_copy_kernel(const uint4 *__restrict__ src, uint4 *__restrict__ dst,
                                                       size_t n)
{
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
        dst[i] = src[i];
}

extern "C" {

// Copies `bytes` (a multiple of 16) between two device buffers it allocates,
// once untimed and once timed; reports the timed copy's duration. Returns 0 on
// success, 4 for a bad size, 2 if allocation fails, 3 on a HIP error.
int hbm_copy_run(size_t bytes, double *ms_out)
{
    if (bytes == 0 || bytes % 16 != 0)
        return 4;
    const size_t n = bytes / 16;
    uint4 *src = nullptr, *dst = nullptr;
    if (hipMalloc(&src, bytes) != hipSuccess)
        return 2;
    if (hipMalloc(&dst, bytes) != hipSuccess) {
        (void)hipFree(src);
        return 2;
    }
    (void)hipMemset(src, 0x5a, bytes);
    const int block = 256;
    const size_t want = (n + block - 1) / block;
    const int grid = (int)(want < 65536 ? want : 65536);
    hipEvent_t a, b;
    (void)hipEventCreate(&a);
    (void)hipEventCreate(&b);
    hbm_copy_kernel<<<grid, block>>>(src, dst, n);
    (void)hipEventRecord(a, nullptr);
    hbm_copy_kernel<<<grid, block>>>(src, dst, n);
    (void)hipEventRecord(b, nullptr);
    hipError_t e = hipEventSynchronize(b);
    float ms = 0.0f;
    if (e == hipSuccess)
        e = hipEventElapsedTime(&ms, a, b);
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    (void)hipFree(src);
    (void)hipFree(dst);
    if (e != hipSuccess)
        return 3;
    *ms_out = ms;
    return 0;
}

int valu_peak_count(void) { return OP_COUNT; }

// Lane-steps per second for one instruction class (one step = one link of one
// chain on one lane; the pair classes execute two instructions per step), at
// `waves_per_simd` waves on every SIMD (1..8) and `chains` independent chains
// per lane (1, 2, 4 or 8). Returns 0 on success, 4 for bad arguments, 1-3 on
// HIP errors.
int valu_peak_run_shape(int op, int iters, int waves_per_simd, int chains, double *steps_per_s, double *ms_out)
{
    if (op < 0 || op >= OP_COUNT || iters < 1 || waves_per_simd < 1 || waves_per_simd > 8)
        return 4;
    const launch_fn *tab = chains == 1   ? Table<1>::fn
                           : chains == 2 ? Table<2>::fn
                           : chains == 4 ? Table<4>::fn
                           : chains == 8 ? Table<8>::fn
                                         : nullptr;
    if (!tab)
        return 4;
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return 1;
    const int block = 256;                 // 4 waves: one on each SIMD of a CU
    const int grid = cus * waves_per_simd;
    uint32_t *out = nullptr;
    if (hipMalloc(&out, (size_t)grid * block * sizeof(uint32_t)) != hipSuccess)
        return 2;
    hipEvent_t a, b;
    (void)hipEventCreate(&a);
    (void)hipEventCreate(&b);
    tab[op](grid, block, out, 64);
    (void)hipEventRecord(a, nullptr);
    tab[op](grid, block, out, iters);
    (void)hipEventRecord(b, nullptr);
    hipError_t e = hipEventSynchronize(b);
    float ms = 0.0f;
    if (e == hipSuccess)
        e = hipEventElapsedTime(&ms, a, b);
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    (void)hipFree(out);
    if (e != hipSuccess)
        return 3;
    *steps_per_s = (double)grid * block * (double)iters * STEPS * chains / (ms * 1e-3);
    *ms_out = ms;
    return 0;
}

// The throughput shape: 8 waves per SIMD, 8 chains.
int valu_peak_run(int op, int iters, double *steps_per_s, double *ms_out)
{
    return valu_peak_run_shape(op, iters, 8, 8, steps_per_s, ms_out);
}

}  // extern "C"
