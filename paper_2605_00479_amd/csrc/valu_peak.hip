// valu_peak.hip - measured VALU issue rates per instruction class on gfx950.
//
// Each kernel gives every lane 8 independent dependency chains of one
// instruction class, so the rate is set by issue throughput, not latency.
// valu_peak_run() times a launch that fills the chip (blocks of 256 threads,
// 8 waves per SIMD) and reports lane-operations per second. bench.py uses the
// rates to check the roofline's weights (full-rate ops 1 slot, quarter-rate
// ops 4 slots) and the 39.3 T slots/s peak.
#include <hip/hip_runtime.h>

#include <cstdint>

#define CHAINS 8

typedef _Float16 half2_t __attribute__((ext_vector_type(2)));
typedef _Float16 half_v2 __attribute__((ext_vector_type(2)));

template <int OP>
__global__ void __launch_bounds__(256) valu_kernel(uint32_t *out, int iters, uint32_t seed)
{
    const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    uint32_t u[CHAINS];
    double d[CHAINS];
    float f[CHAINS];
    half2_t h[CHAINS];
#pragma unroll
    for (int c = 0; c < CHAINS; ++c) {
        u[c] = t * 2654435761u + (uint32_t)c * 40503u + seed;
        d[c] = (double)u[c] * 1e-9;
        f[c] = (float)u[c] * 1e-9f;
        h[c] = half2_t{(_Float16)(f[c] * 1e-3f), (_Float16)(f[c] * 2e-3f)};
    }
    const uint32_t k = seed | 1u;
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int c = 0; c < CHAINS; ++c) {
            if constexpr (OP == 0) {          // v_fma_f64
                d[c] = __builtin_fma(d[c], 0.999999, 1e-7);
            } else if constexpr (OP == 1) {   // v_fma_f32
                f[c] = __builtin_fmaf(f[c], 0.999999f, 1e-7f);
            } else if constexpr (OP == 2) {   // v_pk_fma_f16 (two lanes of fp16 per op)
                h[c] = __builtin_elementwise_fma(h[c], half2_t{(_Float16)0.999f, (_Float16)0.999f},
                                                 half2_t{(_Float16)1e-3f, (_Float16)1e-3f});
            } else if constexpr (OP == 3) {   // v_mad_u64_u32
                uint64_t p = (uint64_t)u[c] * (uint64_t)0xD2511F53u + k;
                u[c] = (uint32_t)(p >> 32) ^ (uint32_t)p;
            } else if constexpr (OP == 4) {   // v_bitop3_b32 (xor3)
                u[c] = __builtin_amdgcn_bitop3_b32(u[c], u[(c + 1) % CHAINS], k, 0x96);
            } else if constexpr (OP == 5) {   // v_cvt_sr_f16_f32 + v_cvt_f32_f16
                half_v2 z = {};
                half_v2 r = __builtin_amdgcn_cvt_sr_f16_f32(z, f[c], u[c], false);
                f[c] = (float)r[0] + 1.0f;
            } else if constexpr (OP == 6) {   // v_rcp_f32
                f[c] = __builtin_amdgcn_rcpf(f[c] + 1.0f);
            }
        }
    }
    uint32_t acc = 0;
#pragma unroll
    for (int c = 0; c < CHAINS; ++c)
        acc ^= u[c] ^ (uint32_t)(d[c] * 1e6) ^ __float_as_uint(f[c]) ^ (uint32_t)(float)h[c][0];
    out[t] = acc;
}

extern "C" {

// op: 0 f64 fma, 1 f32 fma, 2 packed fp16 fma, 3 u64 mad (+ xor), 4 xor3,
// 5 SR cvt (+ widen + add), 6 f32 rcp (+ add). Returns 0 and the rate of chain
// steps (one step of one chain on one lane) per second.
int valu_peak_run(int op, int iters, double *ops_per_s, double *ms_out)
{
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return 1;
    const int block = 256;
    const int grid = cus * 8;   // 8 waves per SIMD
    uint32_t *out = nullptr;
    if (hipMalloc(&out, (size_t)grid * block * sizeof(uint32_t)) != hipSuccess)
        return 2;
    hipEvent_t a, b;
    (void)hipEventCreate(&a);
    (void)hipEventCreate(&b);
    auto launch = [&](int it) {
        switch (op) {
        case 0: valu_kernel<0><<<grid, block>>>(out, it, 7u); break;
        case 1: valu_kernel<1><<<grid, block>>>(out, it, 7u); break;
        case 2: valu_kernel<2><<<grid, block>>>(out, it, 7u); break;
        case 3: valu_kernel<3><<<grid, block>>>(out, it, 7u); break;
        case 4: valu_kernel<4><<<grid, block>>>(out, it, 7u); break;
        case 5: valu_kernel<5><<<grid, block>>>(out, it, 7u); break;
        default: valu_kernel<6><<<grid, block>>>(out, it, 7u); break;
        }
    };
    launch(16);
    (void)hipEventRecord(a, nullptr);
    launch(iters);
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
    const double steps = (double)grid * block * (double)iters * CHAINS;
    *ops_per_s = steps / (ms * 1e-3);
    *ms_out = ms;
    return 0;
}

}  // extern "C"
