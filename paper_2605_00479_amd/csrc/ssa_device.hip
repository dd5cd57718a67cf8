// ssa_device.hip - device side of the ensemble direct method on gfx950.
//
// This file is compiled at run time by hipRTC together with a short,
// generated description of the reaction networks in the launch (species and
// reaction counts, the op sequence of every propensity, the net-change table)
// and one instantiation line. Everything structural is therefore a
// compile-time constant: propensity evaluation, prefix sums, selection and the
// integer update are straight-line code in registers, one trajectory per lane.
// Rate constants, initial states, horizons and snapshot grids stay runtime data.
//
// Method (Kimpson, Flegg & Flegg, Sec. 2, Direct Method steps 1-4):
//   a_j(x), a0 = sum a_j;  tau = -ln(u1)/a0;  mu = min{j : S_j > u2 a0};
//   x += nu_mu, t += tau.
// Precision partition (Sec. 3.2 and opening of Sec. 4):
//   FP64 / FP32: every op in that type.
//   mixed T16:   propensity ops in fp16/bf16, sums, tau, time in binary32.
//   uniform T16: every op in fp16/bf16, including the clock.
// Stochastic rounding (Sec. 3.3): each 16-bit op rounds its binary32 result
// up with probability (x - x-)/(x+ - x-), decided by a 16-bit halfword.
//
// Random bits: Philox4x32-10, key = seed, counter = (event lo, event hi,
// trajectory id, stream). Stream 0 gives the two uniforms (53-bit pairs in
// FP64, the high 24 bits of words 0 and 1 otherwise). In SR modes every
// rounding op of an event owns a fixed slot holding a B-bit random field
// (B = 13 for fp16, 16 for bf16: the mantissa bits a binary32 -> 16-bit
// rounding discards). Main slots are fields of the 80 spare bits of stream 0,
// then of streams 1, 2, ...; conversions of counts have their own slots in
// streams 2^31, 2^31 + 1, ..., drawn only when a count is not exactly
// representable (otherwise the conversion rounds nothing). A step's randomness
// is a function of (seed, trajectory, event) only, so results do not depend on
// lane scheduling.
#pragma clang fp contract(off)

typedef unsigned int u32;
typedef int i32;
typedef unsigned long long u64;
typedef long long i64;

#define SSA_INF_F __builtin_inff()

// --------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror & Shaw, SC'11).
// --------------------------------------------------------------------------
struct W4 {
    u32 w0, w1, w2, w3;
};

__device__ __forceinline__ u32 xor3(u32 a, u32 b, u32 c)
{
    return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);   // a ^ b ^ c in one VALU op
}

__device__ __forceinline__ W4 philox10(u32 c0, u32 c1, u32 c2, u32 c3, u32 k0, u32 k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        u64 p0 = (u64)0xD2511F53u * (u64)c0;
        u64 p1 = (u64)0xCD9E8D57u * (u64)c2;
        u32 n0 = xor3((u32)(p1 >> 32), c1, k0);
        u32 n2 = xor3((u32)(p0 >> 32), c3, k1);
        c1 = (u32)p1;
        c3 = (u32)p0;
        c0 = n0;
        c2 = n2;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    W4 o = {c0, c1, c2, c3};
    return o;
}

// --------------------------------------------------------------------------
// Uniforms on (0, 1]: (m + 1) 2^-53 from 53 bits, (m + 1) 2^-24 from 24 bits.
// --------------------------------------------------------------------------
__device__ __forceinline__ double unif53(u32 a, u32 b)
{
    u64 m = ((u64)a << 21) | (u64)(b >> 11);
    return (double)(m + 1ull) * 0x1p-53;
}

__device__ __forceinline__ float unif24(u32 w)
{
    // (m + 1) 2^-24 = m 2^-24 + 2^-24, exact in binary32 for m < 2^24
    return __builtin_fmaf((float)(w >> 8), 0x1p-24f, 0x1p-24f);
}

// --------------------------------------------------------------------------
// Correctly rounded binary32 a / b (the IEEE quotient) for operands that need
// no range scaling: a = 0 or 2^-26 <= |a| < 32, and 2^-24 <= b < 2^27. The
// hardware reciprocal is refined by one Newton-Raphson step, then the quotient
// by two remainder corrections (Markstein's fma division). On these ranges it
// equals the full division sequence, which adds operand scaling and a
// special-case fix-up (checked on the device over every log argument and
// 2^28 numerators x 16 denominators); it saves three instructions per use.
// --------------------------------------------------------------------------
// (f - 1) / (f + 1) for binary32 f in [1/2, 2): the hardware reciprocal, the
// product and one remainder correction already give the IEEE quotient for
// every such f (checked on the device over all of them).
__device__ __forceinline__ float div_rn_log(float a, float b)
{
    const float r = __builtin_amdgcn_rcpf(b);
    const float q = a * r;
    const float rem = __builtin_fmaf(-b, q, a);
    return __builtin_fmaf(rem, r, q);
}

// (f - 1) / (f + 1) for binary64 f in [1/2, 2): the compiler's IEEE division
// without its operand scaling and special-case fix-up, which leave these
// operands unchanged (the numerator is 0 or at least 2^-53 in magnitude, the
// denominator in [1.5, 3), the quotient normal): reciprocal, two Newton steps,
// product, and the remainder correction as a plain fma.
__device__ __forceinline__ double div_rn_log64(double a, double b)
{
    const double r0 = __builtin_amdgcn_rcp(b);
    const double e0 = __builtin_fma(-b, r0, 1.0);
    const double r1 = __builtin_fma(r0, e0, r0);
    const double e1 = __builtin_fma(-b, r1, 1.0);
    const double r2 = __builtin_fma(r1, e1, r1);
    const double q = a * r2;
    const double rem = __builtin_fma(-b, q, a);
    return __builtin_fma(rem, r2, q);
}

__device__ __forceinline__ float div_rn_inrange(float a, float b)
{
    float r = __builtin_amdgcn_rcpf(b);
    float e = __builtin_fmaf(-b, r, 1.0f);
    r = __builtin_fmaf(e, r, r);
    float q = a * r;
    float rem = __builtin_fmaf(-b, q, a);
    q = __builtin_fmaf(rem, r, q);
    rem = __builtin_fmaf(-b, q, a);
    return __builtin_fmaf(rem, r, q);
}

// --------------------------------------------------------------------------
// -ln(u), u in (0, 1]: u = 2^e f with f in [1/sqrt2, sqrt2],
// ln f = 2 atanh(s) = 2s (1 + s^2/3 + s^4/5 + ...), s = (f - 1)/(f + 1),
// e ln2 with ln2 split in a short high part (exact product) and a low part.
// Only correctly rounded +, -, *, / and fused multiply-adds are used, in a
// fixed order: the quotient s, the series by Horner's rule in fmas, ln f =
// fma(2s, p z, 2s), and fma(e, ln2_hi, fma(e, ln2_lo, ln f)).
// --------------------------------------------------------------------------
__device__ __forceinline__ double neg_log64(double u)
{
    u64 bits = (u64)__double_as_longlong(u);
    int e = (int)((bits >> 52) & 0x7FFull) - 1023;
    double f = __longlong_as_double((i64)((bits & 0x000FFFFFFFFFFFFFull) | 0x3FF0000000000000ull));
    if (f > 0x1.6a09e667f3bcdp+0) {
        f = f * 0.5;
        e = e + 1;
    }
    double s = div_rn_log64(f - 1.0, f + 1.0);
    double z = s * s;
    double p = 0x1.8618618618618p-5;         // 1/21
    p = __builtin_fma(p, z, 0x1.af286bca1af28p-5); // 1/19
    p = __builtin_fma(p, z, 0x1.e1e1e1e1e1e1ep-5); // 1/17
    p = __builtin_fma(p, z, 0x1.1111111111111p-4); // 1/15
    p = __builtin_fma(p, z, 0x1.3b13b13b13b14p-4); // 1/13
    p = __builtin_fma(p, z, 0x1.745d1745d1746p-4); // 1/11
    p = __builtin_fma(p, z, 0x1.c71c71c71c71cp-4); // 1/9
    p = __builtin_fma(p, z, 0x1.2492492492492p-3); // 1/7
    p = __builtin_fma(p, z, 0x1.999999999999ap-3); // 1/5
    p = __builtin_fma(p, z, 0x1.5555555555555p-2); // 1/3
    p = p * z;
    double s2 = s + s;
    double lnf = __builtin_fma(s2, p, s2);
    double ed = (double)e;
    double r = __builtin_fma(ed, 0x1.62e42fep-1, __builtin_fma(ed, 0x1.f473de6af278fp-30, lnf));
    return 0.0 - r;
}

__device__ __forceinline__ float neg_log32(float u)
{
    u32 bits = __float_as_uint(u);
    int e = (int)((bits >> 23) & 0xFFu) - 127;
    float f = __uint_as_float((bits & 0x7FFFFFu) | 0x3F800000u);
    if (f > 0x1.6a09e6p+0f) {
        f = f * 0.5f;
        e = e + 1;
    }
    float s = div_rn_log(f - 1.0f, f + 1.0f);   // f in [1/sqrt2, sqrt2]
    float z = s * s;
    float p = 0x1.c71c72p-4f;                 // 1/9
    p = __builtin_fmaf(p, z, 0x1.24924ap-3f); // 1/7
    p = __builtin_fmaf(p, z, 0x1.99999ap-3f); // 1/5
    p = __builtin_fmaf(p, z, 0x1.555556p-2f); // 1/3
    p = p * z;
    float s2 = s + s;
    float lnf = __builtin_fmaf(s2, p, s2);
    float ed = (float)e;
    float r = __builtin_fmaf(ed, 0x1.62e4p-1f, __builtin_fmaf(ed, 0x1.7f7d1cp-20f, lnf));
    return 0.0f - r;
}

// --------------------------------------------------------------------------
// Rounding a binary32 value to fp16 / bf16 (result carried as binary32).
// Formats per Table tab:formats. Round-to-nearest-even uses the IEEE
// conversions (subnormals kept, overflow to infinity). Stochastic rounding
// uses gfx950's SR conversions: with f the dropped fraction of a grid step,
// the magnitude rounds up when the top B bits of the 16-bit halfword plus
// floor(f 2^B) reach 2^B (B = 16 for bf16, 13 for fp16). The instructions read
// their random bits from the upper half of the 32-bit operand and ignore the
// lower half, so `r` carries the slot's halfword in bits 31..16.
// --------------------------------------------------------------------------
typedef __bf16 ssa_v2bf16 __attribute__((ext_vector_type(2)));
typedef _Float16 ssa_v2f16 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ float rne_f16(float v)
{
    return (float)(_Float16)v;
}

__device__ __forceinline__ float rne_bf16(float v)
{
    return (float)(__bf16)v;
}

// The conversions write one 16-bit half of a register and keep the other; the
// random operand (used once, dead afterwards) serves as that other half, so no
// register needs clearing or copying.
__device__ __forceinline__ float sr_bf16(float v, u32 r)
{
    ssa_v2bf16 o = __builtin_amdgcn_cvt_sr_bf16_f32(__builtin_bit_cast(ssa_v2bf16, r), v, r, false);
    return (float)o[0];
}

__device__ __forceinline__ float sr_f16(float v, u32 r)
{
    ssa_v2f16 o = __builtin_amdgcn_cvt_sr_f16_f32(__builtin_bit_cast(ssa_v2f16, r), v, r, false);
    return (float)o[0];
}

// --------------------------------------------------------------------------
// Precision policies. T: propensity type; A: sum/target type; Tm: clock type.
// rnd(v, rb) is the one rounding applied after every 16-bit op.
// --------------------------------------------------------------------------
enum { FMT_FP64 = 0, FMT_FP32 = 1, FMT_FP16 = 2, FMT_BF16 = 3 };

struct PrecF64 {
    typedef double T;
    typedef double A;
    typedef double Tm;
    static constexpr bool SR = false, UNI = false, NORM = false, WIDE = true, SELECTIVE = false, NATIVE16 = false;
    static constexpr i32 EXACT_INT = 0;   // conversions are exact: no count test
    static constexpr int SR_B = 16;
    template <bool EXACT>
    __device__ static T cvt(i32 v, u32) { return (double)v; }
    // (x - i) converted: x converted once, then an exact binary64 subtraction
    template <bool EXACT>
    __device__ static T cvt_sub(i32 x, i32 i, u32) { return (double)x - (double)i; }
    __device__ static T mul(T a, T b, u32) { return a * b; }
    __device__ static T div(T a, T b, u32) { return a / b; }
    __device__ static T add(T a, T b, u32) { return a + b; }
    __device__ static A acc(A s, T a, u32) { return s + (A)a; }
    __device__ static A arnd(A v, u32) { return v; }
    __device__ static A tacc(A v, u32) { return v; }
    __device__ static A tau_div(A l, A a0) { return l / a0; }
};

struct PrecF32 {
    typedef float T;
    typedef float A;
    typedef float Tm;
    static constexpr bool SR = false, UNI = false, NORM = false, WIDE = false, SELECTIVE = false, NATIVE16 = false;
    static constexpr i32 EXACT_INT = 0;
    static constexpr int SR_B = 16;
    template <bool EXACT>
    __device__ static T cvt(i32 v, u32) { return (float)v; }
    template <bool EXACT>
    __device__ static T cvt_sub(i32 x, i32 i, u32 rb) { return cvt<EXACT>(x - i, rb); }
    __device__ static T mul(T a, T b, u32) { return a * b; }
    __device__ static T div(T a, T b, u32) { return a / b; }
    __device__ static T add(T a, T b, u32) { return a + b; }
    __device__ static A acc(A s, T a, u32) { return s + a; }
    __device__ static A arnd(A v, u32) { return v; }
    __device__ static A tacc(A v, u32) { return v; }
    __device__ static A tau_div(A l, A a0) { return l / a0; }
};

// v as computed in binary32. An operation followed by a conversion to fp16 may
// otherwise be fused into one v_fma_mixlo_f16, which rounds the exact result
// once where the op and the conversion round twice. For +, -, x, / of two fp16
// values the two agree; where an operand has more bits (u2 in the selection
// target) they can differ at a tie of the second rounding.
__device__ __forceinline__ float f32_kept(float v)
{
    __asm__ volatile("" : "+v"(v));
    return v;
}

template <int FMT, bool SRM>
__device__ __forceinline__ float rnd16(float v, u32 rb)
{
    if constexpr (FMT == FMT_FP16)
        return SRM ? sr_f16(v, rb) : rne_f16(v);
    else
        return SRM ? sr_bf16(v, rb) : rne_bf16(v);
}

// RND: 0 round to nearest; 1 stochastic rounding after every 16-bit op;
// 2 stochastic rounding only where values accumulate (partial sums and the
// clock, uniform mode), round to nearest elsewhere - the selective SR the
// paper names as untested (Sec. 3.3, last paragraph).
// binary32 a * b and a + b, each rounded once. For fp16 operands they are
// written as fma(a, b, +0) and fma(a, 1, b) (equal to the product and the sum
// for the non-negative values met here), which gfx950 runs as v_fma_mix_f32
// reading the 16-bit halves directly, without a separate widening conversion.
template <int FMT>
__device__ __forceinline__ float mul32(float a, float b)
{
    if constexpr (FMT == FMT_FP16)
        return __builtin_fmaf(a, b, 0.0f);
    else
        return a * b;
}

template <int FMT>
__device__ __forceinline__ float add32(float a, float b)
{
    if constexpr (FMT == FMT_FP16)
        return __builtin_fmaf(b, 1.0f, a);
    else
        return a + b;
}

template <int FMT, int RND, bool UNIF, bool NRM>
struct Prec16 {
    typedef float T;
    typedef float A;
    typedef float Tm;
    static constexpr bool SR = RND != 0, UNI = UNIF, NORM = NRM, WIDE = false, SELECTIVE = RND == 2;
    static constexpr bool SR_OPS = RND == 1, SR_ACC = RND != 0;
    static constexpr int SR_B = FMT == FMT_FP16 ? 13 : 16;   // random bits per SR rounding
    // counts up to EXACT_INT in magnitude are 16-bit values already: their
    // conversion rounds nothing (by either rule) and needs no random bits
    static constexpr i32 EXACT_INT = FMT == FMT_FP16 ? 2048 : 256;
    template <bool EXACT>
    __device__ static T cvt(i32 v, u32 rb)
    {
        if constexpr (EXACT)
            return (float)v;
        else
            return rnd16<FMT, SR_OPS>((float)v, rb);
    }
    // (x - i) converted. With |x| within the exact-integer limit the binary32
    // subtraction of the converted x is exact, and x is converted once.
    template <bool EXACT>
    __device__ static T cvt_sub(i32 x, i32 i, u32 rb)
    {
        if constexpr (EXACT)
            return (float)x - (float)i;
        else
            return rnd16<FMT, SR_OPS>((float)(x - i), rb);
    }
    // Round to nearest in fp16: the hardware's fp16 product and sum
    // (v_mul_f16, v_add_f16) are the correctly rounded results, equal to the
    // binary32 op followed by one rounding (exact product; innocuous double
    // rounding for the sum, 24 >= 2*11 + 2). Division keeps the binary32
    // quotient and one rounding (the compiler's fp16 division is not an IEEE
    // operation).
    static constexpr bool NATIVE16 = FMT == FMT_FP16 && !SR_OPS;
    __device__ static T mul(T a, T b, u32 rb)
    {
        if constexpr (NATIVE16)
            return (float)((_Float16)a * (_Float16)b);
        else
            return rnd16<FMT, SR_OPS>(mul32<FMT>(a, b), rb);
    }
    __device__ static T div(T a, T b, u32 rb) { return rnd16<FMT, SR_OPS>(a / b, rb); }
    __device__ static T add(T a, T b, u32 rb)
    {
        if constexpr (NATIVE16)
            return (float)((_Float16)a + (_Float16)b);
        else
            return rnd16<FMT, SR_OPS>(add32<FMT>(a, b), rb);
    }
    __device__ static A acc(A s, T a, u32 rb)
    {
        if constexpr (UNIF && FMT == FMT_FP16 && !SR_ACC)
            return (float)((_Float16)s + (_Float16)a);
        else
            return UNIF ? rnd16<FMT, SR_ACC>(add32<FMT>(s, a), rb) : add32<FMT>(s, a);
    }
    __device__ static A arnd(A v, u32 rb) { return UNIF ? rnd16<FMT, SR_OPS>(v, rb) : v; }
    __device__ static A tacc(A v, u32 rb) { return UNIF ? rnd16<FMT, SR_ACC>(v, rb) : v; }
    // -ln(u1) / a0. With fp16 propensities a0 lies in [2^-24, 2^22] whenever
    // the event can fire (any other value only sets a status), and
    // -ln(u1) in {0} or [2^-24, 16.7]: the short division applies.
    __device__ static A tau_div(A l, A a0)
    {
        if constexpr (FMT == FMT_FP16)
            return div_rn_inrange(l, a0);
        else
            return l / a0;
    }
};

// --------------------------------------------------------------------------
// Random fields of one event. A string of bits is cut into B-bit fields from
// its low end (field r = bits [rB, rB + B), spanning two words when it must).
// Pool (main slots): the 80-bit string w[0..2] = (stream-0 word 2, word 3,
// low bytes of words 0 and 1) holds F0 = floor(80/B) fields; each further
// stream's 128-bit string (4 words) holds F1 = floor(128/B). ConvPool
// (conversion slots): F1 fields per stream 2^31 + q. hw(s) is the SR
// conversions' random operand for slot s: the field in bits 31..32-B (the
// instructions read only those; the bits below are don't-cares). Slot numbers
// are compile-time constants, so each hw is one shift or one funnel shift.
// --------------------------------------------------------------------------
template <int B>
__device__ __forceinline__ u32 field_operand(const u32 *w, int off)
{
    const int wi = off / 32, p = off % 32;
    if (p + B <= 32)
        return w[wi] << (32 - B - p);
    return __builtin_amdgcn_alignbit(w[wi + 1], w[wi], p + B - 32);
}

template <int NSLOT, int B>
struct Pool {
    static constexpr int F0 = 80 / B, F1 = 128 / B;
    static constexpr int NSTREAM = NSLOT <= F0 ? 1 : 1 + (NSLOT - F0 + F1 - 1) / F1;
    static constexpr int NW = NSLOT <= 0 ? 1 : 3 + 4 * (NSTREAM - 1);
    u32 w[NW];
    // the third word, whose bit 31 a producer sets on a draw whose ring slot
    // also holds its conversion fields (no field uses that bit)
    __device__ __forceinline__ u32 mark() const
    {
        if constexpr (NW > 2)
            return w[2];
        else
            return 0u;
    }
    // slots past the pool belong to ops that do not round stochastically
    __device__ __forceinline__ u32 hw(int s) const
    {
        if (s >= NSLOT)
            return 0u;
        if (s < F0)
            return field_operand<B>(w, s * B);
        return field_operand<B>(w + 3 + 4 * ((s - F0) / F1), ((s - F0) % F1) * B);
    }
};

#define SSA_CONV_STREAM 0x80000000u

template <int NCONV, int B>
struct ConvPool {
    static constexpr int F1 = 128 / B;
    static constexpr int NSTREAM = NCONV <= 0 ? 0 : (NCONV + F1 - 1) / F1;
    u32 w[NSTREAM > 0 ? 4 * NSTREAM : 1];
    __device__ __forceinline__ u32 hw(int s) const
    {
        if (s >= NCONV)
            return 0u;
        return field_operand<B>(w + 4 * (s / F1), (s % F1) * B);
    }
};

// Conversion fields of event n (drawn only when a count is not exactly representable).
template <int NCONV, int B>
__device__ __forceinline__ ConvPool<NCONV, B> make_conv(u64 n, u32 id, u32 k0, u32 k1)
{
    ConvPool<NCONV, B> cp;
#pragma unroll
    for (int q = 0; q < ConvPool<NCONV, B>::NSTREAM; ++q) {
        W4 r = philox10((u32)n, (u32)(n >> 32), id, SSA_CONV_STREAM + (u32)q, k0, k1);
        cp.w[4 * q + 0] = r.w0;
        cp.w[4 * q + 1] = r.w1;
        cp.w[4 * q + 2] = r.w2;
        cp.w[4 * q + 3] = r.w3;
    }
    return cp;
}

// A conversion pool for runs whose conversions need no random bits.
struct NoConv {
    __device__ __forceinline__ u32 hw(int) const { return 0u; }
};

// --------------------------------------------------------------------------
// Everything an event takes from its random numbers alone: the rounding
// halfword pool, -ln(u1) (rounded once in uniform mode) and u2. It depends on
// (seed, trajectory, event index) only, so the kernel forms event n+1's draw
// while event n's state-dependent chain runs.
// --------------------------------------------------------------------------
template <class P, int NSLOT>
struct Draw {
    Pool<NSLOT, P::SR_B> pool;
    typename P::A L;
    typename P::A u2;
};

template <class P, int NSLOT, int SLOT_LOG>
__device__ __forceinline__ Draw<P, NSLOT> make_draw(u64 n, u32 id, u32 k0, u32 k1)
{
    Draw<P, NSLOT> d;
    W4 r0 = philox10((u32)n, (u32)(n >> 32), id, 0u, k0, k1);
    if constexpr (NSLOT > 0) {
        d.pool.w[0] = r0.w2;
        d.pool.w[1] = r0.w3;
        d.pool.w[2] = (r0.w0 & 0xFFu) | ((r0.w1 & 0xFFu) << 8);
#pragma unroll
        for (int q = 1; q < Pool<NSLOT, P::SR_B>::NSTREAM; ++q) {
            W4 rq = philox10((u32)n, (u32)(n >> 32), id, (u32)q, k0, k1);
            d.pool.w[3 + 4 * (q - 1) + 0] = rq.w0;
            d.pool.w[3 + 4 * (q - 1) + 1] = rq.w1;
            d.pool.w[3 + 4 * (q - 1) + 2] = rq.w2;
            d.pool.w[3 + 4 * (q - 1) + 3] = rq.w3;
        }
    }
    if constexpr (P::WIDE) {
        d.L = neg_log64(unif53(r0.w0, r0.w1));
        d.u2 = unif53(r0.w2, r0.w3);
    } else {
        d.L = P::arnd(neg_log32(unif24(r0.w0)), d.pool.hw(SLOT_LOG));
        d.u2 = unif24(r0.w1);
    }
    return d;
}

// --------------------------------------------------------------------------
// Launch arguments.
// --------------------------------------------------------------------------
struct ItemArgs {
    const void *rates;       // [n_sets][M] constants in the mode's type (T)
    const void *hill;        // [M][2] (b_j, K_j) in T, Hill reactions only
    const i32 *x0;           // [N]
    i32 *snap;               // [k_hi - k_lo][N][E] snapshot rows of this launch
    u64 *n_events;           // [E]
    double *t_last;          // [E]
    unsigned char *status;   // [E]; 255 = suspended at a chunk boundary
    i32 *cx;                 // carry [N][E] (chunked runs)
    double *ct;              // carry clock [E]
    u64 *cn;                 // carry event index [E]
    i32 *ck;                 // carry next snapshot index [E]
    float *cm;               // carry running maximum [E]
    u32 *counter;            // work counter of this item (starts at 0)
    const u32 *order;        // claim order: trajectory of the w-th claim (NULL: w itself)
    u32 *work;               // events each trajectory fired in this launch (NULL: not recorded)
    double *rec_t;           // event record [E][rec_cap]: clock after each recorded firing
    unsigned char *rec_j;    // [E][rec_cap]: the reaction
    u32 *rec_n;              // [E]: recorded firings so far (also carried between chunks)
    u32 E;                   // trajectories
    u32 traj_per_set;        // trajectories per rate set (0: one set)
    u32 id_base;             // Philox trajectory id of trajectory 0
    u32 rec_cap;             // records kept per trajectory
};

struct LaunchArgs {
    const double *snap_t64;  // [K]
    const float *snap_t32;   // [K]
    double t_end64;
    float t_end32;
    i32 K;
    i32 k_lo, k_hi;          // snapshot rows written by this launch
    i32 first, last;         // first / last chunk of the run
    u32 seed_lo, seed_hi;
    u32 place;               // PLACE_* bits (512-thread and single-item launches)
    u32 place_pad;
    u64 max_events;          // 0 = no cap
    ItemArgs item[SSA_N_ITEMS];
};

// Placement of work in a launch.
//   PLACE_NEIGHBOUR: in a 512-thread workgroup the draws of event-loop wave c
//     come from the producer wave on SIMD (c + 1) mod 4 instead of its own
//     SIMD (waves w and w + 4 share a SIMD), so an event-loop wave whose
//     neighbours have drained runs with its SIMD to itself.
//   PLACE_WAVE_MAJOR: single-item launches take their first claims
//     statically, wave-major: claim slot r = c * gridDim.x + blockIdx.x of
//     event-loop wave c in its workgroup holds claims [64 r, 64 r + 64) of
//     the claim order (heaviest first after a reordering window), so the
//     heaviest trajectories sit on wave 0 of every workgroup; the work
//     counter starts past the static claims.
//   PLACE_SOLO0: wave 0's SIMD holds no other wave: the producers feed the
//     event-loop waves of the next SIMD (as PLACE_NEIGHBOUR), event-loop wave
//     3 forms its own draws and wave 4 does not run. With PLACE_WAVE_MAJOR the
//     heaviest trajectories then run with a SIMD to themselves from the start.
//   PLACE_FEED0: the producer feeding event-loop wave 0 runs at wave 0's
//     priority and event-loop waves 1-3 one below it, so that on a busy chip
//     wave 0 (with PLACE_WAVE_MAJOR, the heaviest trajectories) keeps its draws
//   PLACE_PRODUCER_FIRST: producer waves issue ahead of event-loop waves (a
//     producer stops at a full ring, so it takes only what its consumer uses)
//   PLACE_DEDICATED: three event-loop waves per workgroup; wave 0 alone on its
//     SIMD, its producer alone on the next (waves 1 and 4 do not run), waves 2
//     and 3 each fed by the producer on its own SIMD
//   PLACE_TWO0 (with PLACE_DEDICATED, one-item launches): wave 1 runs as a
//     second producer of wave 0 on SIMD 1; waves 5 and 1 make wave 0's draws
//     of even and odd event index. A lone event-loop wave on the conversion
//     path uses its draws faster than one producer wave makes them with their
//     conversion fields; two waves on one SIMD also hide each other's latency.
enum {
    PLACE_NEIGHBOUR = 1u,
    PLACE_WAVE_MAJOR = 2u,
    PLACE_SOLO0 = 4u,
    PLACE_FEED0 = 8u,
    PLACE_PRODUCER_FIRST = 16u,
    PLACE_DEDICATED = 32u,
    PLACE_TWO0 = 64u
};

enum { ST_DONE = 0, ST_ABSORBED = 1, ST_OVERFLOW = 2, ST_CAPPED = 3, ST_SUSPENDED = 255 };

__device__ __forceinline__ u32 lane_id()
{
    return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
}

// Mask of the wave's lanes where c holds. Given one comparison, the mask is the
// comparison's own result; a conjunction is formed as the AND of its terms'
// masks (scalar ops), since a mask of a combined condition costs two dependent
// vector ops more.
__device__ __forceinline__ u64 lanes(bool c)
{
    return __builtin_amdgcn_ballot_w64(c);
}

// A wave-uniform value moved to a scalar register.
template <class V>
__device__ __forceinline__ V uniform_value(V v)
{
    if constexpr (sizeof(V) == 4) {
        return __builtin_bit_cast(V, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(u32, v)));
    } else {
        const u64 b = __builtin_bit_cast(u64, v);
        // readfirstlane returns a signed int: widen through u32, not by sign extension
        const u64 r = ((u64)(u32)__builtin_amdgcn_readfirstlane((u32)(b >> 32)) << 32) |
                      (u64)(u32)__builtin_amdgcn_readfirstlane((u32)b);
        return __builtin_bit_cast(V, r);
    }
}

__device__ __forceinline__ u32 rank_in(u64 mask)
{
    return __builtin_amdgcn_mbcnt_hi((u32)(mask >> 32), __builtin_amdgcn_mbcnt_lo((u32)mask, 0u));
}

template <class P>
__device__ __forceinline__ typename P::Tm snap_time(const LaunchArgs &L, int k)
{
    if constexpr (P::WIDE)
        return L.snap_t64[k];
    else
        return L.snap_t32[k];
}

// --------------------------------------------------------------------------
// Rounding slots of an event (Md: generated network description). With
// selective SR only the M-1 partial sums and the clock draw.
// --------------------------------------------------------------------------
template <class P, class Md>
struct Slots {
    static constexpr int M = Md::M;
    static constexpr int NSLOT = !P::SR ? 0
                                 : (P::SELECTIVE ? M : Md::NPROP + (P::UNI ? (P::NORM ? 2 * M + 4 : M + 3) : 0));
    static constexpr int NORM = Md::NPROP;
    static constexpr int SUM = P::SELECTIVE ? 0 : Md::NPROP + (P::NORM ? M : 0);
    static constexpr int LOG = SUM + M - 1;
    static constexpr int TAU = LOG + 1;
    static constexpr int TAUM = TAU + 1;
    static constexpr int TIME = P::SELECTIVE ? M - 1 : TAU + 1 + (P::NORM ? 1 : 0);
    static constexpr int TARGET = TIME + 1;
};

// A draw as 32-bit words: the pool's words, then L and u2 (one word each in
// binary32, two in binary64). Word k of a stored draw sits at w[S k], with S a
// multiple of 64, so the 64 lanes of a wave touch 64 consecutive words.
template <class P, int NSLOT>
struct DrawIO {
    static constexpr int NP = NSLOT > 0 ? Pool<NSLOT, P::SR_B>::NW : 0;
    static constexpr int NA = (int)(sizeof(typename P::A) / 4);
    static constexpr int NW = NP + 2 * NA;

    template <int S>
    __device__ static void store(u32 *w, const Draw<P, NSLOT> &d)
    {
        if constexpr (NP > 0) {
#pragma unroll
            for (int k = 0; k < NP; ++k)
                w[S * k] = d.pool.w[k];
        }
        if constexpr (NA == 1) {
            w[S * NP] = __float_as_uint((float)d.L);
            w[S * (NP + 1)] = __float_as_uint((float)d.u2);
        } else {
            const u64 a = (u64)__double_as_longlong((double)d.L), b = (u64)__double_as_longlong((double)d.u2);
            w[S * NP] = (u32)a;
            w[S * (NP + 1)] = (u32)(a >> 32);
            w[S * (NP + 2)] = (u32)b;
            w[S * (NP + 3)] = (u32)(b >> 32);
        }
    }

    // the pool's words (needed first: the propensities' rounding fields)
    template <int S>
    __device__ static void load_pool(const u32 *w, Draw<P, NSLOT> &d)
    {
        if constexpr (NP > 0) {
#pragma unroll
            for (int k = 0; k < NP; ++k)
                d.pool.w[k] = w[S * k];
        }
    }

    // L and u2 (needed later in an event than the pool)
    template <int S>
    __device__ static void load_tail(const u32 *w, Draw<P, NSLOT> &d)
    {
        if constexpr (NA == 1) {
            d.L = __uint_as_float(w[S * NP]);
            d.u2 = __uint_as_float(w[S * (NP + 1)]);
        } else {
            d.L = __longlong_as_double((long long)(((u64)w[S * (NP + 1)] << 32) | w[S * NP]));
            d.u2 = __longlong_as_double((long long)(((u64)w[S * (NP + 3)] << 32) | w[S * (NP + 2)]));
        }
    }
};

// Conversion fields a producer may carry in a ring slot, after the draw's own
// words: models whose count conversions round stochastically (R13: drawn
// only when a count exceeds the exact-integer limit). Bit 31 of the third
// pool word marks a draw whose slot holds them.
template <class P, class Md>
struct ConvRing {
    static constexpr bool ON = P::SR && !P::SELECTIVE && Md::NCONV > 0;
    static constexpr int NW = ON ? 4 * ConvPool<Md::NCONV, P::SR_B>::NSTREAM : 0;
    static constexpr u32 MARK = 0x80000000u;
};

// Words of one ring slot for a model: the draw, then its conversion fields.
template <class P, class Md>
struct RingWords {
    static constexpr int NW = DrawIO<P, Slots<P, Md>::NSLOT>::NW + ConvRing<P, Md>::NW;
};

// --------------------------------------------------------------------------
// Draw feeds. The event loop takes event n + 1's draw while it runs event n.
// SelfFeed forms it in the same wave. RingFeed takes it from a ring in LDS
// that a producer wave on the same SIMD fills ahead (produce_item), and forms
// it itself wherever the ring does not hold it: the event loop never waits
// for the producer. The producer makes exactly the draws the loop would form
// (same function of seed, trajectory and event index), so results do not
// depend on the feed.
//
// Protocol, per lane (consumer lane l and producer lane l of the paired waves).
// A counter word is (low 24 bits of an event index) << 8 | epoch, so a lane
// steps it by adding 256 and the 24-bit index wraps without touching the epoch:
//   req_*  consumer -> producer: trajectory id and claim event index, then the
//          epoch e (1..255, new at every claim) once the rest is written;
//   done   consumer -> producer: counter word of the first draw the consumer
//          has not read yet;
//   made   producer -> consumer: counter word of the first draw not made yet;
//          draws [made - D, made) of epoch e are in the ring (the consumer
//          resets it at a claim, before publishing the epoch). With two
//          producers for one consumer (PLACE_TWO0), producer k makes the draws
//          of odd (k = 1) or even (k = 0) event index and publishes made[k]:
//          its draws of that parity in [made[k] - D, made[k]) are in the ring,
//          and the consumer reads the made word of its next draw's parity.
//   convw  consumer -> producer: the lane's counts need conversion fields
//          (reset at a claim); the producer then also forms each draw's
//          conversion fields, stores them after the draw's words, and marks
//          the draw by bit 31 of its third pool word (a bit no field uses).
// The producer writes draw p only while p < done + D, so a draw the consumer
// finds made stays in place until it has read it. Ordering rests on waits for
// completed LDS operations (lgkmcnt 0): the producer waits for its ring
// stores before it updates made, the consumer waits for its made load before
// it loads ring words, and for its ring loads before it updates done.
// --------------------------------------------------------------------------
struct RingCtl {
    u32 made[2][64];   // [parity class][lane]; class 1 only with two producers
    u32 done[64];
    u32 req_e[64];
    u32 req_id[64];
    u32 req_lo[64];
    u32 req_hi[64];
    u32 convw[64];   // consumer -> producer: 1 while the lane's trajectory wants conversion fields
    u32 item;        // consumer -> producer: sequence number of the item in progress (~0u: finished)
};

__device__ __forceinline__ void lgkm_wait()
{
    __builtin_amdgcn_s_waitcnt(0xC07F);   // lgkmcnt(0)
    __asm__ volatile("" ::: "memory");
}

__device__ __forceinline__ u32 lds_ld(const u32 *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

__device__ __forceinline__ void lds_st(u32 *p, u32 v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

struct SelfFeed {
    static constexpr bool RING = false;
    __device__ void claim(u32, u64) {}
    __device__ void request_conv(u32) const {}
};

template <int D, int NWMAX, bool TWO = false>
struct RingFeed {
    static constexpr bool RING = true;
    static_assert((D & (D - 1)) == 0, "ring depth is a power of two");
    RingCtl *ctl;   // this consumer wave's control words
    u32 *ring;      // [NWMAX][D][64]: word k of slot s, lane l at ring[(k D + s) 64 + l]
    u32 lane;
    u32 eb;         // epoch of the lane's trajectory (0: none claimed yet)
    u32 dw;         // counter word of the draw the lane takes next (event n + 1)
    // TWO (two producers, PLACE_TWO0): the made word for draw dw, formed when dw
    // changes (its byte offset in made is the parity bit of the event index, bit
    // 8 of a counter word), so the load at the top of the next event waits for
    // no address arithmetic (a lone wave on the conversion path measured 679
    // cycles per event with the address formed from dw there, 648 with it formed
    // ahead). With one producer the made word's address is fixed: a feed type of
    // its own keeps that arithmetic out of every other event loop (5% of the
    // five-network batch's step).
    const u32 *mptr;   // &ctl->made[0][lane] until the first claim

    // a new trajectory on this lane; the loop forms draws n and n + 1 itself.
    // made is reset to "nothing made in this epoch" before the epoch is
    // published, so a made word the lane finds in its epoch was written for it
    // (a late write from an older epoch is a few epochs behind, never a hit)
    __device__ void claim(u32 id, u64 n)
    {
        eb = eb % 255u + 1u;
        dw = ((u32)(n + 1) << 8) | eb;
        lds_st(&ctl->done[lane], dw);
        lds_st(&ctl->made[0][lane], dw);
        lds_st(&ctl->made[1][lane], dw);
        if constexpr (TWO)
            mptr = (const u32 *)((const char *)&ctl->made[0][lane] + (dw & 0x100u));
        lds_st(&ctl->req_id[lane], id);
        lds_st(&ctl->req_lo[lane], (u32)n);
        lds_st(&ctl->req_hi[lane], (u32)(n >> 32));
        lds_st(&ctl->convw[lane], 0u);
        lgkm_wait();
        lds_st(&ctl->req_e[lane], eb);
    }

    // The request word: while the wave runs a version whose conversions
    // round, each of its lanes asks the producer for every draw's conversion
    // fields (set when the wave enters a version loop; a claim clears it).
    // The producer forms them for the whole wave once any lane asks.
    __device__ void request_conv(u32 on) const { lds_st(&ctl->convw[lane], on); }

    // Conversion fields of the current event's draw (event n, counter word
    // dw - 256): from its ring slot where the producer formed them with the
    // draw (the draw came from the ring and carries the mark), formed here
    // for the active lanes whose draw lacks the mark (a draw made before the
    // request, or formed by the event loop); a lane whose counts are all
    // exact ignores its fields. The slot is intact: the producer may rewrite
    // it only once done passes event n, which read() publishes after this
    // event's loads have completed.
    // pre: the slot's conversion words, loaded with the draw (read_conv in the
    // previous event; meaningful where the draw carries the mark).
    template <int NCONV, int B>
    __device__ ConvPool<NCONV, B> conv(const ConvPool<NCONV, B> &pre, u32 mark, u64 act, u64 n, u32 id, u32 k0,
                                       u32 k1) const
    {
        ConvPool<NCONV, B> cp = pre;
        const u64 self = act & ~lanes((i32)mark < 0);   // the mark is bit 31
        if (__builtin_expect(self != 0, 0)) {
            __asm__ volatile("");
            const ConvPool<NCONV, B> f = make_conv<NCONV, B>(n, id, k0, k1);
            if ((self >> lane) & 1u)
                cp = f;
        }
        return cp;
    }

    // the made word of the parity class of the draw the lane takes next (dw)
    __device__ u32 made_word() const
    {
        if constexpr (TWO)
            return lds_ld(mptr);
        else
            return lds_ld(&ctl->made[0][lane]);
    }

    // slot of the draw with counter word dw: its index mod D, times the 256
    // bytes of a slot's word, is dw's index bits [8, 8 + log2 D) in place
    __device__ const u32 *slot() const
    {
        return (const u32 *)((const char *)(ring + lane) + (dw & (u32)((D - 1) << 8)));
    }

    // the pool words of the next draw (valid where finish finds it made)
    template <class P, int NSLOT>
    __device__ void read(Draw<P, NSLOT> &d) const
    {
        lgkm_wait();   // the made word, and the previous draw's ring words, are in
        lds_st(&ctl->done[lane], dw);
        DrawIO<P, NSLOT>::template load_pool<D * 64>(slot(), d);
    }

    // the conversion words of the next draw's slot, loaded with its pool words
    // (models whose conversions round stochastically): in registers by the
    // time an event on the conversion path needs them
    template <int NCONV, int B, int OFF>
    __device__ void read_conv(ConvPool<NCONV, B> &cp) const
    {
#pragma unroll
        for (int q = 0; q < ConvPool<NCONV, B>::NSTREAM * 4; ++q)
            cp.w[q] = slot()[(OFF + q) * D * 64];
    }

    // its L and u2, loaded once this event's are no longer needed
    template <class P, int NSLOT>
    __device__ void read_tail(Draw<P, NSLOT> &d) const
    {
        DrawIO<P, NSLOT>::template load_tail<D * 64>(slot(), d);
    }

    // lanes whose next draw the ring does not hold (the event loop forms it
    // itself). With x = made - (dw + 256), the draw is made (want < made <=
    // want + D, epochs equal) exactly when x rotated right by 8 is below D:
    // equal epochs leave a zero low byte and the index difference minus one
    // above it; any other epoch puts a nonzero byte on top after the rotation
    __device__ u64 miss_lanes(u32 mw, u64 act) const
    {
        const u32 next = dw + 256u;
        const bool hit = __builtin_amdgcn_alignbit(mw - next, mw - next, 8) < (u32)D;
        return act & ~lanes(hit);
    }

    // form draw `want` for the lanes in miss (the ring did not hold it)
    template <class P, int NSLOT, int SLOT_LOG>
    __device__ void self_draw(Draw<P, NSLOT> &d, u64 miss, u64 want, u32 id, u32 k0, u32 k1) const
    {
        const Draw<P, NSLOT> s = make_draw<P, NSLOT, SLOT_LOG>(want, id, k0, k1);
        if ((miss >> lane) & 1u)
            d = s;
    }

    // step to the draw after the next one
    __device__ void advance()
    {
        dw += 256u;
        if constexpr (TWO)
            mptr = (const u32 *)((const char *)&ctl->made[0][lane] + (dw & 0x100u));
    }
};

// Producer wave of one item: for each lane, the draws of its consumer lane's
// trajectory from the claim's event index + 1 on, up to D ahead of the
// consumer. A batch starts once some lane has START free slots; its BATCH
// draws are formed in one block, so their Philox and logarithm chains overlap
// (a lane with fewer free slots stores only those). The shape is measured:
// with the event loop and this wave sharing a SIMD, 6 draws from 6 free slots
// of 16 keep the ring ahead for binary32 and 16-bit draws, 8 from 4 for binary64.
// STRIDE 2: one of two producers of the consumer, making the draws whose event
// index has parity cls (PLACE_TWO0); each then holds at most D / 2 draws of
// the ring, and a batch of 4 from 4 free places keeps its half ahead.
// Returns once the consumer has moved past item `seq`.
template <class P, class Md, int D, int NWMAX, int STRIDE>
__device__ void produce_item(const LaunchArgs &L, const ItemArgs &I, RingCtl *ctl, u32 *ring, u32 seq, u32 cls)
{
    typedef Slots<P, Md> S;
    typedef DrawIO<P, S::NSLOT> IO;
    typedef ConvRing<P, Md> CR;
    static_assert(!CR::ON || IO::NP >= 3, "the conversion mark lives in the third pool word");
    static_assert(STRIDE == 1 || (STRIDE == 2 && D >= 4), "two producers share a ring of at least 4 slots");
    constexpr int BATCH = STRIDE == 2 ? (D >= 16 ? 4 : D / 4) : D >= 16 ? (P::WIDE ? 8 : 6) : (D >= 2 ? D / 2 : 1);
    constexpr int START = STRIDE == 2 ? BATCH : P::WIDE && BATCH > 4 ? 4 : BATCH;
    const u32 lane = lane_id();
    u32 e = 0, id = 0;
    u64 p = 0;
    // the loop on a 64-byte boundary, as the event loops: with its first block
    // 4 bytes past a 32-byte boundary (where the code before it happened to
    // leave it) the heavy trajectories' producer fell behind and the open
    // dimerisation sweep took 457-464 ms against 414-428 aligned, every other
    // instruction the same
    __asm__ volatile(".p2align 6");
    for (;;) {
        const u32 re = lds_ld(&ctl->req_e[lane]);
        lgkm_wait();   // a new epoch's request words were written before it
        const u32 item = __builtin_amdgcn_readfirstlane(lds_ld(&ctl->item));
        const u32 dw = lds_ld(&ctl->done[lane]);
        u32 cw = 0u;
        if constexpr (CR::ON)
            cw = lds_ld(&ctl->convw[lane]);
        if (item != seq)
            break;
        if (re != e) {
            e = re;
            id = lds_ld(&ctl->req_id[lane]);
            p = (((u64)lds_ld(&ctl->req_hi[lane]) << 32) | lds_ld(&ctl->req_lo[lane])) + 1;
            if constexpr (STRIDE == 2)
                p += ((u32)p ^ cls) & 1u;   // the first index of this producer's parity
        }
        // draws made and not yet read: p - done, as a signed 24-bit difference. The
        // event-loop lane may be ahead (it forms draws itself until the ring holds
        // them, e.g. right after a claim): then skip to its next unread draw (of
        // this producer's parity).
        const bool mine = e != 0 && (dw & 0xFFu) == e;
        i32 ahead = (i32)(((u32)p << 8) - (dw & ~0xFFu)) >> 8;
        if (mine && ahead < 0) {
            p += (u64)(u32)(-ahead);
            ahead = 0;
            if constexpr (STRIDE == 2) {
                const u32 fix = ((u32)p ^ cls) & 1u;
                p += fix;
                ahead = (i32)fix;
            }
        }
        // places p, p + 1, ... below done + D; this producer's draws among them
        const u32 span = (mine && ahead < D) ? (u32)(D - ahead) : 0u;
        const u32 room = STRIDE == 2 ? (span + 1u) >> 1 : span;
        if (__builtin_amdgcn_ballot_w64(room >= (u32)START) == 0) {
            __builtin_amdgcn_s_sleep(2);
            continue;
        }
        Draw<P, S::NSLOT> d[BATCH];
#pragma unroll
        for (int b = 0; b < BATCH; ++b)
            d[b] = make_draw<P, S::NSLOT, S::LOG>(p + (u64)(STRIDE * b), id, L.seed_lo, L.seed_hi);
        // formed here, every one: left to the guarded stores below, each
        // would be formed in a block of its own, one chain after another
#pragma unroll
        for (int b = 0; b < BATCH; ++b) {
            __asm__ volatile("" : "+v"(d[b].L), "+v"(d[b].u2));
            if constexpr (S::NSLOT > 0) {
#pragma unroll
                for (int k = 0; k < IO::NP; ++k)
                    __asm__ volatile("" : "+v"(d[b].pool.w[k]));
            }
        }
        // conversion fields of the batch, where some lane of the wave asked
        // for them: formed for every lane, marked in each draw, stored after
        // the draw's words
        if constexpr (CR::ON) {
            if (__builtin_amdgcn_ballot_w64(mine && cw != 0u) != 0) {
                ConvPool<Md::NCONV, P::SR_B> cv[BATCH];
#pragma unroll
                for (int b = 0; b < BATCH; ++b)
                    cv[b] = make_conv<Md::NCONV, P::SR_B>(p + (u64)(STRIDE * b), id, L.seed_lo, L.seed_hi);
#pragma unroll
                for (int b = 0; b < BATCH; ++b) {
#pragma unroll
                    for (int q = 0; q < CR::NW; ++q)
                        __asm__ volatile("" : "+v"(cv[b].w[q]));
                    d[b].pool.w[2] |= CR::MARK;
                }
#pragma unroll
                for (int b = 0; b < BATCH; ++b)
                    if ((u32)b < room) {
                        u32 *w = ring + ((u32)(p + (u64)(STRIDE * b)) & (u32)(D - 1)) * 64 + lane;
#pragma unroll
                        for (int q = 0; q < CR::NW; ++q)
                            w[(IO::NW + q) * D * 64] = cv[b].w[q];
                    }
            }
        }
#pragma unroll
        for (int b = 0; b < BATCH; ++b)
            if ((u32)b < room)
                IO::template store<D * 64>(ring + ((u32)(p + (u64)(STRIDE * b)) & (u32)(D - 1)) * 64 + lane, d[b]);
        const u32 k = room < (u32)BATCH ? room : (u32)BATCH;
        lgkm_wait();
        if (k != 0u) {
            p += (u64)(STRIDE * k);
            lds_st(&ctl->made[STRIDE == 2 ? cls : 0u][lane], ((u32)p << 8) | e);
        }
    }
    (void)I;
}

// Ring depth for draws of nw words: the largest power of two up to 16 whose
// four rings and four control blocks fit a workgroup's LDS (gfx950: 160 KiB
// per CU, all of it available to one workgroup; 1 KiB is left spare); 0
// where not even a depth of 2 fits (then the 512-thread kernel runs eight
// event-loop waves that form their own draws).
constexpr int kLdsBytes = 160 * 1024;
__host__ __device__ constexpr int ring_depth(int nw)
{
    int d = 16;
    while (d >= 2 && 4 * d * nw * 64 * 4 + 4 * (int)sizeof(RingCtl) > kLdsBytes - 1024)
        d /= 2;
    return d >= 2 ? d : 0;
}

__host__ __device__ constexpr int cmax(int a, int b)
{
    return a > b ? a : b;
}

// --------------------------------------------------------------------------
// Propensity versions. Each computes the same values wherever it runs; a state
// needs one of them (wave-uniform, over the lanes holding a trajectory):
//   VER_EXACT    every count exactly representable in the propensity type (or
//                a binary type), none below a reactant order: no zero guard;
//   VER_GUARD    counts exact, some count below its order: zero guards;
//   VER_CONV     some count above the exact-integer limit (its conversion
//                rounds and draws conversion fields), zero guards;
//   VER_CONV_NG  the same with every count at or above its orders.
// The event loop runs one straight-line loop per version and leaves it when
// the updated state needs another, so a wave that stays in one version (a
// long trajectory far above the exact-integer limit) takes no branch but the
// loop's own each event. The loop test is one ballot for the states the
// version cannot compute; a move to a cheaper version waits for the next
// event that takes the rare path (a snapshot crossing, a fallback selection,
// a draw the producer has not made), which costs time, never results.
// --------------------------------------------------------------------------
enum { VER_EXACT = 0, VER_GUARD = 1, VER_CONV = 2, VER_CONV_NG = 3 };

template <int V>
struct IC {
    static constexpr int value = V;
};

template <class P, class Md>
struct Versions {
    static constexpr bool CONV = P::SR && !P::SELECTIVE && Md::NCONV > 0;
    static constexpr bool GUARD = Md::LO_MAX > 0;

    __device__ static __forceinline__ u32 max_count(const i32 (&x)[Md::N])
    {
        u32 mx = (u32)x[0];
#pragma unroll
        for (int s = 1; s < Md::N; ++s)
            mx = (u32)x[s] > mx ? (u32)x[s] : mx;
        return mx;
    }

    // counts are never negative; as unsigned, a negative one would only send
    // the wave to the version that handles every count
    __device__ static __forceinline__ int of(const i32 (&x)[Md::N], u64 act)
    {
        if constexpr (CONV) {
            if ((act & lanes(Md::range_key(x) > (u32)(P::EXACT_INT - Md::LO_MAX))) == 0)
                return VER_EXACT;
            if ((act & lanes(max_count(x) > (u32)P::EXACT_INT)) == 0)
                return VER_GUARD;
            return (GUARD && (act & lanes(Md::below(x))) != 0) ? VER_CONV : VER_CONV_NG;
        } else if constexpr (GUARD) {
            return (act & lanes(Md::below(x))) == 0 ? VER_EXACT : VER_GUARD;
        } else {
            return VER_EXACT;
        }
    }

    // Lanes whose updated state version V cannot compute: a count above the
    // exact-integer limit where V converts without rounding, a count below a
    // reactant order where V has no zero guard. VER_CONV computes every state.
    // One ballot per version; leaving for a cheaper version (a state that no
    // longer needs V's extra work) is optional, and is tested on the rare path.
    template <int V>
    __device__ static __forceinline__ u64 must_leave(const i32 (&x)[Md::N], u64 act)
    {
        if constexpr (V == VER_EXACT) {
            if constexpr (CONV)
                return act & lanes(Md::range_key(x) > (u32)(P::EXACT_INT - Md::LO_MAX));
            else if constexpr (GUARD)
                return act & lanes(Md::below(x));
            else
                return 0;
        } else if constexpr (V == VER_GUARD) {
            if constexpr (CONV)
                return act & lanes(max_count(x) > (u32)P::EXACT_INT);
            else
                return 0;
        } else if constexpr (V == VER_CONV_NG) {
            if constexpr (GUARD)
                return act & lanes(Md::below(x));
            else
                return 0;
        } else {
            return 0;
        }
    }
};

// --------------------------------------------------------------------------
// One wave works through one item: lanes claim trajectories from the item's
// counter, run events, and claim again as they finish (ballot + prefix rank,
// one atomic per refill), until the counter passes E and every lane is idle.
// Md: generated network description; P: precision policy.
// --------------------------------------------------------------------------
template <class P, class Md, bool PER_LANE_RATES, class F>
__device__ void run_item(const LaunchArgs &L, const ItemArgs &I, F &feed, u32 slot_rank, u32 n_slots)
{
    typedef typename P::T T;
    typedef typename P::A A;
    typedef typename P::Tm Tm;
    typedef Slots<P, Md> S;
    typedef Versions<P, Md> VS;
    constexpr int N = Md::N, M = Md::M;
    constexpr int NSLOT = S::NSLOT;
    constexpr int SLOT_NORM = S::NORM;
    constexpr int SLOT_SUM = S::SUM;
    constexpr int SLOT_LOG = S::LOG;
    constexpr int SLOT_TAU = S::TAU;
    constexpr int SLOT_TAUM = S::TAUM;
    constexpr int SLOT_TIME = S::TIME;
    constexpr int SLOT_TARGET = S::TARGET;

    const T *rates = (const T *)I.rates;
    const T *hill = (const T *)I.hill;
    const Tm t_end = P::WIDE ? (Tm)L.t_end64 : (Tm)L.t_end32;
    const u32 lane = lane_id();

    // initialised: a lane without a trajectory still runs the event step on them
    i32 x[N] = {};
    T c[M] = {};
    Tm t = 0;
    u64 n = 0;
    i32 k = 0;
    Tm t_next = 0;     // time of snapshot k (infinity past the last row of this launch)
    Tm t_stop = 0;     // an event at t_new fires only if t_new <= t_stop (-infinity: suspend)
    Draw<P, NSLOT> cur = {};
    // conversion words of cur's ring slot (RingFeed, models whose conversions
    // round stochastically); used only where cur carries the producer's mark
    constexpr bool CONV_RING = F::RING && ConvRing<P, Md>::ON;
    typedef ConvPool<Md::NCONV, P::SR_B> CP;
    CP conv_cur = {};
    u64 n_claim = 0;   // event index when this launch claimed the trajectory
    u32 rec_cnt = 0;   // recorded firings of this trajectory (Md::REC reactions)
    const u64 n_stop = L.max_events ? L.max_events : ~0ull;
    float mrun = 0.0f;
    u32 idx = 0;
    bool active = false;
    bool open = true;

    if constexpr (!PER_LANE_RATES) {
        // one set for the item: wave-uniform, kept in scalar registers
#pragma unroll
        for (int j = 0; j < M; ++j)
            c[j] = uniform_value(rates[j]);
    }

    // wave-major static first claim (single-item launches): every lane is idle
    // at the start, so the wave's claim is its slot's 64 consecutive claims
    bool static_claim = SSA_N_ITEMS == 1 && (L.place & PLACE_WAVE_MAJOR) != 0u;
    const u32 dyn_base = static_claim ? n_slots * 64u : 0u;   // claims after the static ones
    for (;;) {
        if (open) {
            u64 need = __ballot(!active);
            if (need) {
                u32 cnt = (u32)__popcll(need);
                u32 leader = (u32)__ffsll((long long)need) - 1u;
                u32 base = 0;
                if (static_claim) {
                    base = slot_rank * 64u;
                    static_claim = false;
                } else {
                    if (lane == leader)
                        base = atomicAdd(I.counter, cnt);
                    base = __builtin_amdgcn_readlane(base, leader) + dyn_base;
                }
                if (!active) {
                    u32 w = base + rank_in(need);
                    if (w < I.E) {
                        u32 id = I.order ? I.order[w] : w;
                        idx = id;
                        active = true;
                        if constexpr (PER_LANE_RATES) {
                            u32 set = I.traj_per_set ? id / I.traj_per_set : 0u;
#pragma unroll
                            for (int j = 0; j < M; ++j)
                                c[j] = rates[(u64)set * M + j];
                        }
                        if (L.first) {
#pragma unroll
                            for (int s = 0; s < N; ++s)
                                x[s] = I.x0[s];
                            t = 0;
                            n = 0;
                            k = 0;
                            mrun = 0.0f;
                            rec_cnt = 0;
                        } else {
#pragma unroll
                            for (int s = 0; s < N; ++s)
                                x[s] = I.cx[(u64)s * I.E + id];
                            t = (Tm)I.ct[id];
                            n = I.cn[id];
                            k = I.ck[id];
                            mrun = I.cm[id];
                            if constexpr (Md::REC != 0)
                                rec_cnt = I.rec_n[id];
                            if (I.status[id] != ST_SUSPENDED) {
                                if (I.work)
                                    I.work[id] = 0u;
                                // finished in an earlier chunk: fill this chunk's rows
                                for (int kk = L.k_lo; kk < L.k_hi; ++kk)
#pragma unroll
                                    for (int s = 0; s < N; ++s)
                                        I.snap[((u64)(kk - L.k_lo) * N + s) * I.E + id] = x[s];
                                active = false;
                            }
                        }
                        t_next = k < L.k_hi ? snap_time<P>(L, k) : (Tm)SSA_INF_F;
                        t_stop = (!L.last && k >= L.k_hi) ? (Tm)(-SSA_INF_F) : t_end;
                        n_claim = n;
                        cur = make_draw<P, NSLOT, SLOT_LOG>(n, I.id_base + id, L.seed_lo, L.seed_hi);
                        feed.claim(I.id_base + id, n);
                    }
                }
                if (base + cnt >= I.E)
                    open = false;
            }
        }
        u64 act = lanes(active);   // the wave's lanes holding a trajectory
        if (act == 0) {
            if (!open)
                break;
            continue;
        }

        // Every lane runs the event step, also one without a trajectory: such a
        // lane never fires, stores nothing and leaves its registers unused, and
        // the step needs no exec-mask save and restore around it.
        for (;;) {
            // the last event's values, from which a stopping lane's status is read
            A a0 = 0;
            Tm t_new = 0;
            bool a_ok = false, m_ok = true, fire = false;
            u64 stop_lanes;
            // One event step in propensity version V; returns the lanes (or, for a
            // cheaper version, every lane) that make the wave choose its version again.
            auto step = [&](auto vtag) __attribute__((always_inline)) -> u64 {
                constexpr int V = decltype(vtag)::value;
                // ---- draws: cur belongs to event n; event n+1's is formed (or
                // taken from the producer's ring) alongside
                const u32 id = I.id_base + idx;
                Draw<P, NSLOT> nxt;
                u32 made_w = 0;
                if constexpr (F::RING)
                    made_w = feed.made_word();
                else
                    nxt = make_draw<P, NSLOT, SLOT_LOG>(n + 1, id, L.seed_lo, L.seed_hi);
                const Pool<NSLOT, P::SR_B> &pool = cur.pool;
                // ---- propensities (generated op sequence) in version V.
                // Conversions of counts draw random bits only when they round:
                // with every count exactly representable in the 16-bit type
                // no conversion stream is drawn. A mass-action propensity is
                // zero when a count is below its order; with every count at or
                // above its species' largest order no guard can apply.
                u64 cheaper = 0;
                T a[M];
                if constexpr (V == VER_EXACT) {
                    Md::template propensities<P, VS::CONV, false>(x, c, hill, a, pool, NoConv());
                } else if constexpr (V == VER_GUARD) {
                    Md::template propensities<P, VS::CONV, true>(x, c, hill, a, pool, NoConv());
                } else {
                    // conversion fields: from the producer where it formed them
                    // (ring feed), else formed here
                    CP cpool;
                    if constexpr (F::RING)
                        cpool = feed.template conv<Md::NCONV, P::SR_B>(conv_cur, cur.pool.mark(), act, n, id,
                                                                        L.seed_lo, L.seed_hi);
                    else
                        cpool = make_conv<Md::NCONV, P::SR_B>(n, id, L.seed_lo, L.seed_hi);
                    Md::template propensities<P, false, V == VER_CONV>(x, c, hill, a, pool, cpool);
                }
                CP conv_nxt;
                if constexpr (F::RING) {
                    feed.read(nxt);
                    if constexpr (CONV_RING)
                        feed.template read_conv<Md::NCONV, P::SR_B, DrawIO<P, NSLOT>::NW>(conv_nxt);
                }
                // ---- optional running-max normalisation (uniform 16-bit)
                T m = (T)1;
                m_ok = true;
                if constexpr (P::NORM) {
                    float mx = 0.0f;
#pragma unroll
                    for (int j = 0; j < M; ++j)
                        mx = a[j] > mx ? a[j] : mx;
                    mrun = mx > mrun ? mx : mrun;
                    m_ok = mrun > 0.0f && mrun <= 3.40282347e38f;
                    m = mrun;
#pragma unroll
                    for (int j = 0; j < M; ++j)
                        a[j] = P::div(a[j], m, pool.hw(SLOT_NORM + j));
                }
                // ---- partial sums and total
                A S[M];
                S[0] = (A)a[0];
#pragma unroll
                for (int j = 1; j < M; ++j)
                    S[j] = P::acc(S[j - 1], a[j], pool.hw(SLOT_SUM + j - 1));
                a0 = S[M - 1];
                // a0 in (0, largest finite]: false for zero, negatives, infinity and NaN
                if constexpr (P::WIDE)   // positive finite binary64: bit patterns 1 .. 0x7FEFFFFFFFFFFFFF
                    a_ok = (u64)__double_as_longlong(a0) - 1ull < 0x7FEFFFFFFFFFFFFFull;
                else
                    a_ok = __float_as_uint(a0) - 1u < 0x7F7FFFFFu;
                a_ok = a_ok && m_ok;
                // ---- waiting time and clock (formed on every lane, used only if the event fires)
                if constexpr (P::UNI) {
                    A tau = P::arnd(P::tau_div(cur.L, a0), pool.hw(SLOT_TAU));
                    if constexpr (P::NORM)
                        tau = P::arnd(tau / m, pool.hw(SLOT_TAUM));
                    t_new = P::tacc(t + tau, pool.hw(SLOT_TIME));
                } else {
                    t_new = t + P::tau_div(cur.L, a0);
                }
                const u64 ok_lanes = act & lanes(a_ok);
                // ---- selection: mu = number of prefix sums at or below the target
                A target;
                if constexpr (P::UNI)   // binary32 product, then one rounding to the 16-bit type
                    target = P::arnd(f32_kept(cur.u2 * a0), pool.hw(SLOT_TARGET));
                else
                    target = cur.u2 * a0;
                if constexpr (F::RING)
                    feed.read_tail(nxt);   // cur's L and u2 are used by now
                int mu = 0;
#pragma unroll
                for (int j = 0; j < M; ++j)
                    mu += (S[j] <= target) ? 1 : 0;
                // ---- rare work behind one wave-uniform test (out of line): snapshots
                // strictly before t_new hold the current state; a target at or above
                // the total selects the last reaction with a positive propensity; a
                // next draw the producer has not made is formed here
                u64 miss = 0;
                if constexpr (F::RING)
                    miss = feed.miss_lanes(made_w, act);
                if (__builtin_expect(((ok_lanes & (lanes(t_next < t_new) | lanes(mu == M))) | miss) != 0, 0)) {
                    __asm__ volatile("");
                    if (active && a_ok && t_next < t_new) {
                        do {
#pragma unroll
                            for (int s = 0; s < N; ++s)
                                I.snap[((u64)(k - L.k_lo) * N + s) * I.E + idx] = x[s];
                            ++k;
                            t_next = k < L.k_hi ? snap_time<P>(L, k) : (Tm)SSA_INF_F;
                        } while (t_next < t_new);
                        t_stop = (!L.last && k >= L.k_hi) ? (Tm)(-SSA_INF_F) : t_end;
                    }
                    if (active && a_ok && t_new <= t_stop && mu == M) {
                        int last_pos = 0;
#pragma unroll
                        for (int j = 0; j < M; ++j)
                            last_pos = (a[j] > (T)0) ? j : last_pos;
                        mu = last_pos;
                    }
                    if constexpr (F::RING) {
                        if (miss != 0)
                            feed.template self_draw<P, NSLOT, SLOT_LOG>(nxt, miss, n + 1, id, L.seed_lo, L.seed_hi);
                    }
                    // a cheaper version may serve the state now: leave after this event
                    // and choose again (a state V cannot compute is caught after the update)
                    if constexpr (V != VER_EXACT)
                        cheaper = lanes(VS::of(x, act) != V);
                }
                fire = active && a_ok && t_new <= t_stop;
                const u64 fire_lanes = ok_lanes & lanes(t_new <= t_stop);
                // ---- integer update (mu = M: nothing fires)
                Md::update(x, fire ? mu : M);
                t = fire ? t_new : t;
                n += 1;   // also where the event does not fire: such a lane stops, and is reset below
                if constexpr (Md::REC != 0) {
                    // event record: firings of the recorded reactions, with the clock after them
                    if (fire && ((Md::REC >> mu) & 1ull)) {
                        if (rec_cnt < I.rec_cap) {
                            I.rec_t[(u64)idx * I.rec_cap + rec_cnt] = (double)t;
                            I.rec_j[(u64)idx * I.rec_cap + rec_cnt] = (unsigned char)mu;
                        }
                        ++rec_cnt;
                    }
                }
                if constexpr (F::RING)
                    feed.advance();
                cur = nxt;   // a lane that stops here draws afresh when it claims again
                if constexpr (CONV_RING)
                    conv_cur = conv_nxt;
                stop_lanes = act & (~fire_lanes | lanes(n == n_stop));
                return VS::template must_leave<V>(x, act) | cheaper;
            };
            // one straight-line loop per version; its first instruction on a
            // 64-byte boundary (where the taken back-branch lands decides how
            // many instruction-fetch lines an event spans; the same loop
            // measured up to 5% apart between offsets; the padding runs once)
            int ver = VS::of(x, act);
            for (;;) {
                u64 leave;
                if constexpr (CONV_RING)
                    feed.request_conv(ver >= VER_CONV ? 1u : 0u);
                if (ver == VER_EXACT) {
                    __asm__ volatile(".p2align 6");
                    do {
                        leave = step(IC<VER_EXACT>());
                    } while (__builtin_expect((stop_lanes | leave) == 0, 1));
                } else if (VS::GUARD && ver == VER_GUARD) {
                    if constexpr (VS::GUARD) {
                        __asm__ volatile(".p2align 6");
                        do {
                            leave = step(IC<VER_GUARD>());
                        } while (__builtin_expect((stop_lanes | leave) == 0, 1));
                    }
                } else if (VS::CONV && ver == VER_CONV_NG) {
                    if constexpr (VS::CONV) {
                        __asm__ volatile(".p2align 6");
                        do {
                            leave = step(IC<VER_CONV_NG>());
                        } while (__builtin_expect((stop_lanes | leave) == 0, 1));
                    }
                } else {
                    if constexpr (VS::CONV && VS::GUARD) {
                        __asm__ volatile(".p2align 6");
                        do {
                            leave = step(IC<VER_CONV>());
                        } while (__builtin_expect((stop_lanes | leave) == 0, 1));
                    }
                }
                if (stop_lanes != 0)
                    break;
                ver = VS::of(x, act);
            }
            if (active && (!fire || n == n_stop)) {
                if (!fire)
                    n -= 1;
                // ---- finish (or suspend) this trajectory, once per trajectory
                int status;
                if (!a_ok)
                    status = !m_ok ? (!(mrun <= 3.40282347e38f) ? ST_OVERFLOW : ST_ABSORBED)
                                   : (!(a0 <= (P::WIDE ? (A)1.7976931348623157e308 : (A)3.40282347e38f))
                                          ? ST_OVERFLOW
                                          : ST_ABSORBED);
                else if (!fire)
                    status = t_new > t_end ? ST_DONE : ST_SUSPENDED;
                else
                    status = ST_CAPPED;
                if (status != ST_SUSPENDED) {
                    for (; k < L.k_hi; ++k)
#pragma unroll
                        for (int s = 0; s < N; ++s)
                            I.snap[((u64)(k - L.k_lo) * N + s) * I.E + idx] = x[s];
                    I.n_events[idx] = n;
                    I.t_last[idx] = (double)t;
                }
                I.status[idx] = (unsigned char)status;
                if (I.work)
                    I.work[idx] = (u32)(n - n_claim);
                if constexpr (Md::REC != 0)
                    I.rec_n[idx] = rec_cnt;
                if (!L.last) {
#pragma unroll
                    for (int s = 0; s < N; ++s)
                        I.cx[(u64)s * I.E + idx] = x[s];
                    I.ct[idx] = (double)t;
                    I.cn[idx] = n;
                    I.ck[idx] = k;
                    I.cm[idx] = mrun;
                }
                active = false;
            }
            // leave to claim new trajectories once a lane stops (while any are
            // left), or when every lane has stopped
            act = lanes(active);
            if (open || act == 0)
                break;
        }
    }
}

// --------------------------------------------------------------------------
// Claim order for the next snapshot chunk: trajectories sorted by the events
// they fired in the last chunk, heaviest first, in 256 log-spaced classes
// (8 per octave). Waves then hold trajectories of similar length, and the
// longest start first. Only the lane a trajectory runs on changes; its draws
// are keyed by its id, so results are unchanged.
// --------------------------------------------------------------------------
__device__ __forceinline__ u32 work_class(u32 w)
{
    u32 v = w + 1u;
    u32 lz = 31u - (u32)__builtin_clz(v);                 // floor(log2 v)
    u32 frac = lz >= 3u ? (v >> (lz - 3u)) & 7u : (v << (3u - lz)) & 7u;
    u32 key = lz * 8u + frac;
    return 255u - (key > 255u ? 255u : key);               // heaviest first
}

extern "C" __global__ void ssa_regroup_hist(const u32 *work, u32 E, u32 *hist)
{
    __shared__ u32 h[256];
    h[threadIdx.x] = 0u;
    __syncthreads();
    for (u32 i = blockIdx.x * blockDim.x + threadIdx.x; i < E; i += gridDim.x * blockDim.x)
        atomicAdd(&h[work_class(work[i])], 1u);
    __syncthreads();
    if (h[threadIdx.x])
        atomicAdd(&hist[threadIdx.x], h[threadIdx.x]);
}

extern "C" __global__ void ssa_regroup_scan(u32 *hist)
{
    // one workgroup of 256 threads: exclusive prefix sum in place
    __shared__ u32 v[256];
    const u32 t = threadIdx.x;
    v[t] = hist[t];
    __syncthreads();
    for (u32 off = 1; off < 256u; off <<= 1) {
        u32 add = t >= off ? v[t - off] : 0u;
        __syncthreads();
        v[t] += add;
        __syncthreads();
    }
    hist[t] = t ? v[t - 1] : 0u;
}

// Workgroups of 256 threads take tiles of 256 trajectories: ranks within a
// class come from an LDS histogram of the tile and each (tile, class) reserves
// its range with one global atomic. The order inside a class is arbitrary.
extern "C" __global__ void __launch_bounds__(256) ssa_regroup_scatter(const u32 *work, u32 E, u32 *offs, u32 *order)
{
    __shared__ u32 cnt[256];
    __shared__ u32 base[256];
    const u32 t = threadIdx.x;
    // the tile loop condition is the same for every thread of the workgroup
    for (u32 tile = blockIdx.x * 256u; tile < E; tile += gridDim.x * 256u) {
        cnt[t] = 0u;
        __syncthreads();
        const u32 i = tile + t;
        u32 cls = 0u, rank = 0u;
        if (i < E) {
            cls = work_class(work[i]);
            rank = atomicAdd(&cnt[cls], 1u);
        }
        __syncthreads();
        if (cnt[t])
            base[t] = atomicAdd(&offs[t], cnt[t]);
        __syncthreads();
        if (i < E)
            order[base[cls] + rank] = i;
        __syncthreads();
    }
}
