/*
 * ssa_oracle.c - CPU oracle for the ensemble Gillespie direct method in FP64,
 * FP32, mixed 16-bit and uniform 16-bit precision (with stochastic rounding and
 * optional running-max propensity normalisation).
 *
 * TEST INFRASTRUCTURE. This file is the plain, slow, obviously-correct
 * statement of what the GPU path must compute. Only the test suite, the smoke
 * check and the CPU-baseline leg of the benchmark may load it. It shares no code
 * with the GPU library: every routine here is written out on its own.
 *
 * Where each step comes from (Kimpson, Flegg & Flegg, "Reduced-Precision
 * Stochastic Simulation for Mathematical Biology"):
 *   - Direct Method steps 1-4 (propensities and their sum a0, tau = -ln(u1)/a0,
 *     smallest mu with partial sum > u2*a0, x += nu_mu, t += tau):  Sec. 2.
 *   - Mixed partition (16-bit propensities, 32-bit sum/time accumulators,
 *     integer state) and the "uniform" all-16-bit mode:  Sec. 3.2 and the
 *     opening of Sec. 4.
 *   - Stochastic rounding, SR(x) = x- w.p. (x+ - x)/(x+ - x-), else x+:
 *     Sec. 3.3 (the SR equation); applied at every arithmetic op (Sec. 3.3).
 *   - fp16/bf16 format parameters: Table "tab:formats" (Sec. 3.1).
 *   - Propensity normalisation: named in the abstract only; read here as
 *     dividing every propensity by the running maximum of the largest
 *     propensity over the steps so far (current step included).
 * Pins: the tests hold each part to closed forms, exhaustive checks or
 * brute force. The repressilator as a whole has none (parity unpinned); its
 * Hill and first-order laws are pinned separately.
 * The paper does not fix the random number generator, the uniform interval,
 * the op order inside a propensity, or how SR bits are drawn. The readings
 * implemented here are:
 *   - RNG: Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11), key = seed,
 *     counter = (event lo, event hi, trajectory id, stream).
 *   - FP64 uniforms: u = (m53 + 1) * 2^-53 in (0,1]; other modes: 24 bits.
 *   - -ln(u): argument reduction by powers of two (Cody & Waite split of ln 2)
 *     and the atanh series ln f = 2 atanh((f-1)/(f+1)), in the working type.
 *   - Mass action: a_j = c_j * prod_s (x_s)(x_s-1)...(x_s-o_s+1), with
 *     c_j = k_j / prod_s o_s!, factors multiplied left to right starting from
 *     the constant; a_j = 0 (no ops) when some x_s < o_s.
 *   - Hill: a = b + v / (1 + (x/K)^h) (repression) or b + v (x/K)^h / (1 + (x/K)^h).
 *   - Every 16-bit op = exact or correctly rounded FP32 op, then one rounding
 *     to the 16-bit format (RNE or SR). SR halfwords come from a static slot
 *     schedule per event (see sr_bits below).
 *
 * Build: gcc -O2 -std=c11 -ffp-contract=off -fno-fast-math -fopenmp -shared -fPIC
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------------- */
/* Philox4x32-10 (Salmon et al., SC'11): 10 rounds of the 4x32 Philox S-box.  */
/* Each round multiplies counter words 0 and 2 by fixed odd constants, takes  */
/* the 64-bit products' high and low halves, and mixes them with words 1, 3   */
/* and the round key; the key is advanced by two Weyl increments per round.   */
/* ------------------------------------------------------------------------- */
#define PHILOX_MUL0 0xD2511F53u
#define PHILOX_MUL1 0xCD9E8D57u
#define PHILOX_WEYL0 0x9E3779B9u
#define PHILOX_WEYL1 0xBB67AE85u

void or_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += PHILOX_WEYL0;
            k1 += PHILOX_WEYL1;
        }
        uint64_t p0 = (uint64_t)PHILOX_MUL0 * (uint64_t)c0;
        uint64_t p1 = (uint64_t)PHILOX_MUL1 * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* Draw for (seed, trajectory id, event index, stream). */
static void draw(uint64_t seed, uint32_t id, uint64_t n, uint32_t stream, uint32_t out[4])
{
    uint32_t ctr[4] = {(uint32_t)n, (uint32_t)(n >> 32), id, stream};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    or_philox4x32_10(ctr, key, out);
}

/* ------------------------------------------------------------------------- */
/* Uniforms on (0, 1].                                                        */
/* ------------------------------------------------------------------------- */
double or_u53(uint32_t a, uint32_t b)
{
    uint64_t m = ((uint64_t)a << 21) | (uint64_t)(b >> 11); /* 53 random bits */
    return (double)(m + 1u) * 0x1p-53;
}

float or_u24(uint32_t w)
{
    uint32_t m = w >> 8; /* 24 random bits */
    return (float)(m + 1u) * 0x1p-24f;
}

/* ------------------------------------------------------------------------- */
/* -ln(u) for u in (0, 1].                                                    */
/* u = 2^e * f with f in [1/sqrt2, sqrt2]; ln u = e ln2 + ln f;               */
/* ln f = 2 atanh(s), s = (f-1)/(f+1): 2s (1 + s^2/3 + s^4/5 + ...).          */
/* ln 2 is split (Cody & Waite) so that e*LN2_HI is exact.                    */
/* The paper does not fix the logarithm; this is the project's definition,   */
/* with every step a correctly rounded IEEE operation: s is the correctly    */
/* rounded quotient, the series is evaluated by Horner's rule with fused     */
/* multiply-adds (one rounding per step), ln f = fma(2s, p z, 2s), and       */
/* r = fma(e, LN2_HI, fma(e, LN2_LO, ln f)) (e * LN2_HI is exact).            */
/* ------------------------------------------------------------------------- */
static const double LN2_HI_D = 0x1.62e42fep-1;         /* ln 2 truncated to 29 bits */
static const double LN2_LO_D = 0x1.f473de6af278fp-30;  /* ln 2 - LN2_HI_D */
static const double SQRT2_D = 0x1.6a09e667f3bcdp+0;
/* 1/(2k+1), k = 1..10 */
static const double ATANH_D[10] = {
    0x1.5555555555555p-2, 0x1.999999999999ap-3, 0x1.2492492492492p-3,
    0x1.c71c71c71c71cp-4, 0x1.745d1745d1746p-4, 0x1.3b13b13b13b14p-4,
    0x1.1111111111111p-4, 0x1.e1e1e1e1e1e1ep-5, 0x1.af286bca1af28p-5,
    0x1.8618618618618p-5};

double or_nlog64(double u)
{
    uint64_t bits;
    memcpy(&bits, &u, sizeof bits);
    int e = (int)((bits >> 52) & 0x7FF) - 1023;
    uint64_t fbits = (bits & 0x000FFFFFFFFFFFFFull) | 0x3FF0000000000000ull;
    double f;
    memcpy(&f, &fbits, sizeof f);
    if (f > SQRT2_D) {
        f = f * 0.5;
        e = e + 1;
    }
    double s = (f - 1.0) / (f + 1.0);
    double z = s * s;
    double p = ATANH_D[9];
    for (int i = 8; i >= 0; --i)
        p = fma(p, z, ATANH_D[i]);
    p = p * z;
    double s2 = s + s;
    double lnf = fma(s2, p, s2);
    double ed = (double)e;
    double r = fma(ed, LN2_HI_D, fma(ed, LN2_LO_D, lnf));
    return 0.0 - r;
}

static const float LN2_HI_F = 0x1.62e4p-1f;          /* ln 2 truncated to 17 bits */
static const float LN2_LO_F = 0x1.7f7d1cp-20f;       /* ln 2 - LN2_HI_F */
static const float SQRT2_F = 0x1.6a09e6p+0f;
static const float ATANH_F[4] = {0x1.555556p-2f, 0x1.99999ap-3f, 0x1.24924ap-3f,
                                 0x1.c71c72p-4f};

float or_nlog32(float u)
{
    uint32_t bits;
    memcpy(&bits, &u, sizeof bits);
    int e = (int)((bits >> 23) & 0xFF) - 127;
    uint32_t fbits = (bits & 0x7FFFFFu) | 0x3F800000u;
    float f;
    memcpy(&f, &fbits, sizeof f);
    if (f > SQRT2_F) {
        f = f * 0.5f;
        e = e + 1;
    }
    float s = (f - 1.0f) / (f + 1.0f);
    float z = s * s;
    float p = ATANH_F[3];
    for (int i = 2; i >= 0; --i)
        p = fmaf(p, z, ATANH_F[i]);
    p = p * z;
    float s2 = s + s;
    float lnf = fmaf(s2, p, s2);
    float ed = (float)e;
    float r = fmaf(ed, LN2_HI_F, fmaf(ed, LN2_LO_F, lnf));
    return 0.0f - r;
}

/* ------------------------------------------------------------------------- */
/* Rounding to a 16-bit format (Table tab:formats):                          */
/*   fp16: 11 significand bits, min normal exponent -14, overflow at 2^16;   */
/*   bf16:  8 significand bits, min normal exponent -126, overflow at 2^128. */
/* v is any double; the result is the rounded value (exact in float).        */
/* rb < 0: round to nearest, ties to even.                                   */
/* rb in [0, 65535]: stochastic rounding (Sec. 3.3). With x- <= |v| < x+ the */
/* neighbours on the format's grid and f = (|v| - x-)/(x+ - x-), the         */
/* magnitude goes to x+ when the top B bits of the halfword rb, read as an   */
/* integer, plus floor(f * 2^B) reach 2^B; B = 16 for bf16 and 13 for fp16.  */
/* For uniform rb this happens with probability floor(f 2^B)/2^B, i.e. the   */
/* SR probability f to within 2^-B. x+ beyond the largest finite value is    */
/* infinity.                                                                  */
/* ------------------------------------------------------------------------- */
enum { OR_FP64 = 0, OR_FP32 = 1, OR_FP16 = 2, OR_BF16 = 3 };

double or_round16(int fmt, double v, int rb)
{
    int p, emin;
    double ovf;
    if (fmt == OR_FP16) {
        p = 11; emin = -14; ovf = 65536.0;
    } else {
        p = 8; emin = -126; ovf = ldexp(1.0, 128);
    }
    if (isnan(v) || isinf(v) || v == 0.0)
        return v;
    double sign = v < 0.0 ? -1.0 : 1.0;
    double av = fabs(v);
    int e2;
    (void)frexp(av, &e2);          /* av = f * 2^e2, f in [0.5, 1) */
    int E = e2 - 1;                /* floor(log2 av) */
    if (E < emin)
        E = emin;                  /* subnormal range: fixed spacing */
    double ulp = ldexp(1.0, E - (p - 1));
    double q = av / ulp;           /* exact: scaling by a power of two */
    double fl = floor(q);
    double frac = q - fl;          /* exact */
    int up;
    if (rb < 0) {
        up = frac > 0.5 || (frac == 0.5 && fmod(fl, 2.0) == 1.0);
    } else {
        int B = fmt == OR_FP16 ? 13 : 16;
        double scale = ldexp(1.0, B);
        double rtop = (double)(rb >> (16 - B));  /* top B bits of the halfword */
        up = rtop + floor(frac * scale) >= scale;
    }
    double r = (fl + (double)up) * ulp;
    if (r >= ovf)
        r = INFINITY;
    return sign * r;
}

/* ------------------------------------------------------------------------- */
/* Model and run descriptions.                                               */
/* ------------------------------------------------------------------------- */
enum { LAW_MASS_ACTION = 0, LAW_HILL_REPRESS = 1, LAW_HILL_ACTIVATE = 2 };
enum { ST_DONE = 0, ST_ABSORBED = 1, ST_OVERFLOW = 2, ST_CAPPED = 3 };

typedef struct {
    int32_t n_species;
    int32_t n_reactions;
    const int32_t *order;    /* [M][N] reactant orders (mass action) */
    const int32_t *nu;       /* [M][N] net change of each species */
    const int32_t *law;      /* [M] */
    const double *rate;      /* [M] mass action: k_j; Hill: v_j */
    const int32_t *hill_reg; /* [M] regulator species */
    const int32_t *hill_h;   /* [M] Hill exponent (>= 1) */
    const double *hill_b;    /* [M] basal rate */
    const double *hill_K;    /* [M] half-saturation constant */
} or_model;

typedef struct {
    int32_t fmt;     /* OR_FP64, OR_FP32, OR_FP16, OR_BF16 */
    int32_t uniform; /* 16-bit formats: 0 = mixed, 1 = uniform */
    int32_t sr;      /* 16-bit formats: 0 = round to nearest, 1 = stochastic rounding
                        at every op, 2 = stochastic rounding only where values
                        accumulate (partial sums and the clock; uniform mode) */
    int32_t norm;    /* uniform 16-bit: running-max normalisation */
} or_mode;

typedef struct {
    const int32_t *x0;       /* [N] */
    double t_end;
    const double *snap_t;    /* [K], ascending, each <= t_end */
    int32_t n_snap;
    uint64_t seed;
    uint32_t traj_id_base;
    uint64_t max_events;     /* 0 = no cap */
    const double *set_rate;  /* optional [n_sets][M] rates replacing model->rate */
    int64_t n_sets;
    int64_t traj_per_set;
} or_run;

/* Event record: every firing of a reaction in `mask` is logged with the clock
 * after it (widened to binary64) and the reaction index, up to `cap` records
 * per trajectory; `n` counts all such firings, also those past `cap`. The
 * switching times of a gene (Sec. 4.3 dwell times) are such a record. */
typedef struct {
    uint64_t mask;
    int32_t cap;
    double *t;               /* [count][cap] */
    uint8_t *j;              /* [count][cap] */
    uint32_t *n;             /* [count] */
} or_rec;

typedef struct {
    int32_t *snap;           /* [K][N][stride] */
    int64_t stride;
    int64_t col;
    const or_rec *rec;       /* NULL: no record */
} or_out;

#define MAXM 64
#define MAXN 64

static int64_t factorial(int n)
{
    int64_t f = 1;
    for (int i = 2; i <= n; ++i)
        f *= i;
    return f;
}

/* Number of rounding slots each reaction's propensity uses (static schedule). */
/* Rounding ops of reaction j's propensity: count conversions (conversion    */
/* slots) and the other ops (main slots).                                     */
static int reaction_conv_ops(const or_model *md, int j)
{
    const int N = md->n_species;
    if (md->law[j] == LAW_MASS_ACTION) {
        int total = 0;
        for (int s = 0; s < N; ++s)
            total += md->order[j * N + s];
        return total;      /* one conversion per factor */
    }
    return 1;              /* the regulator's count */
}

static int reaction_main_ops(const or_model *md, int j)
{
    if (md->law[j] == LAW_MASS_ACTION)
        return reaction_conv_ops(md, j);   /* one multiply per factor */
    /* q = x/K, h-1 powers, d = 1 + q^h, f = v/d (activation: g = v q^h, f = g/d), a = b + f */
    if (md->law[j] == LAW_HILL_REPRESS)
        return md->hill_h[j] + 3;
    return md->hill_h[j] + 4;
}

static void record(const or_out *o, uint32_t *cnt, int mu, double t)
{
    if (!o->rec || !((o->rec->mask >> mu) & 1u))
        return;
    if (*cnt < (uint32_t)o->rec->cap) {
        o->rec->t[o->col * o->rec->cap + *cnt] = t;
        o->rec->j[o->col * o->rec->cap + *cnt] = (uint8_t)mu;
    }
    ++*cnt;
}

static void finish_record(const or_out *o, uint32_t cnt)
{
    if (o->rec && o->rec->n)
        o->rec->n[o->col] = cnt;
}

static void write_snap(const or_out *o, int k, int N, const int32_t *x)
{
    for (int s = 0; s < N; ++s)
        o->snap[((int64_t)k * N + s) * o->stride + o->col] = x[s];
}

static double primary_rate(const or_model *md, const or_run *run, int64_t idx, int j)
{
    if (run->set_rate) {
        int64_t set = idx / run->traj_per_set;
        return run->set_rate[set * md->n_reactions + j];
    }
    return md->rate[j];
}

/* Mass-action constant c_j = k_j / prod_s o_s! (one FP64 division). */
static double folded_constant(const or_model *md, int j, double k)
{
    const int N = md->n_species;
    int64_t d = 1;
    for (int s = 0; s < N; ++s)
        d *= factorial(md->order[j * N + s]);
    return k / (double)d;
}

/* Selection (Sec. 2, step 3): smallest mu with S_mu > target; S is
 * non-decreasing, so mu = #{j : S_j <= target}. If none exceeds target, the
 * last reaction with a positive summand is taken. */
static int select_mu(int M, const double *S, const double *summand, double target)
{
    for (int j = 0; j < M; ++j)
        if (S[j] > target)
            return j;
    int mu = M - 1;
    while (mu > 0 && !(summand[mu] > 0.0))
        --mu;
    return mu;
}

/* ------------------------------------------------------------------------- */
/* FP64 direct method.                                                        */
/* ------------------------------------------------------------------------- */
static void traj_fp64(const or_model *md, const or_run *run, int64_t idx, const or_out *o,
                      uint64_t *n_out, double *t_out, uint8_t *st_out)
{
    const int N = md->n_species, M = md->n_reactions, K = run->n_snap;
    const uint32_t id = run->traj_id_base + (uint32_t)idx;
    int32_t x[MAXN];
    double c[MAXM], hb[MAXM], hK[MAXM];
    for (int s = 0; s < N; ++s)
        x[s] = run->x0[s];
    for (int j = 0; j < M; ++j) {
        double k = primary_rate(md, run, idx, j);
        c[j] = md->law[j] == LAW_MASS_ACTION ? folded_constant(md, j, k) : k;
        hb[j] = md->hill_b ? md->hill_b[j] : 0.0;
        hK[j] = md->hill_K ? md->hill_K[j] : 1.0;
    }
    double t = 0.0;
    uint64_t n = 0;
    int k = 0, status;
    uint32_t rec_cnt = 0;
    for (;;) {
        uint32_t w[4];
        draw(run->seed, id, n, 0, w);
        double u1 = or_u53(w[0], w[1]);
        double u2 = or_u53(w[2], w[3]);
        double a[MAXM], S[MAXM];
        for (int j = 0; j < M; ++j) {
            if (md->law[j] == LAW_MASS_ACTION) {
                double acc = c[j];
                int zero = 0;
                for (int s = 0; s < N; ++s) {
                    int o_s = md->order[j * N + s];
                    if (x[s] < o_s)
                        zero = 1;
                }
                if (zero) {
                    a[j] = 0.0;
                    continue;
                }
                for (int s = 0; s < N; ++s)
                    for (int i = 0; i < md->order[j * N + s]; ++i)
                        acc = acc * (double)(x[s] - i);
                a[j] = acc;
            } else {
                double q = (double)x[md->hill_reg[j]] / hK[j];
                double qh = q;
                for (int i = 1; i < md->hill_h[j]; ++i)
                    qh = qh * q;
                double d = 1.0 + qh;
                double f;
                if (md->law[j] == LAW_HILL_REPRESS)
                    f = c[j] / d;
                else
                    f = (c[j] * qh) / d;
                a[j] = hb[j] + f;
            }
        }
        S[0] = a[0];
        for (int j = 1; j < M; ++j)
            S[j] = S[j - 1] + a[j];
        double a0 = S[M - 1];
        if (!(a0 <= 1.7976931348623157e308)) { status = ST_OVERFLOW; break; }
        if (!(a0 > 0.0)) { status = ST_ABSORBED; break; }
        double tau = or_nlog64(u1) / a0;
        double t_new = t + tau;
        while (k < K && run->snap_t[k] < t_new) {
            write_snap(o, k, N, x);
            ++k;
        }
        if (t_new > run->t_end) { status = ST_DONE; break; }
        double target = u2 * a0;
        int mu = select_mu(M, S, a, target);
        for (int s = 0; s < N; ++s)
            x[s] += md->nu[mu * N + s];
        t = t_new;
        ++n;
        record(o, &rec_cnt, mu, (double)t);
        if (run->max_events && n == run->max_events) { status = ST_CAPPED; break; }
    }
    for (; k < K; ++k)
        write_snap(o, k, N, x);
    finish_record(o, rec_cnt);
    *n_out = n;
    *t_out = t;
    *st_out = (uint8_t)status;
}

/* ------------------------------------------------------------------------- */
/* FP32 direct method (every op in binary32, 24-bit uniforms).               */
/* ------------------------------------------------------------------------- */
static void traj_fp32(const or_model *md, const or_run *run, int64_t idx, const or_out *o,
                      uint64_t *n_out, double *t_out, uint8_t *st_out)
{
    const int N = md->n_species, M = md->n_reactions, K = run->n_snap;
    const uint32_t id = run->traj_id_base + (uint32_t)idx;
    int32_t x[MAXN];
    float c[MAXM], hb[MAXM], hK[MAXM];
    for (int s = 0; s < N; ++s)
        x[s] = run->x0[s];
    for (int j = 0; j < M; ++j) {
        double k = primary_rate(md, run, idx, j);
        c[j] = (float)(md->law[j] == LAW_MASS_ACTION ? folded_constant(md, j, k) : k);
        hb[j] = (float)(md->hill_b ? md->hill_b[j] : 0.0);
        hK[j] = (float)(md->hill_K ? md->hill_K[j] : 1.0);
    }
    const float t_end = (float)run->t_end;
    float t = 0.0f;
    uint64_t n = 0;
    int k = 0, status;
    uint32_t rec_cnt = 0;
    for (;;) {
        uint32_t w[4];
        draw(run->seed, id, n, 0, w);
        float u1 = or_u24(w[0]);
        float u2 = or_u24(w[1]);
        float a[MAXM], S[MAXM];
        double Sd[MAXM], ad[MAXM];
        for (int j = 0; j < M; ++j) {
            if (md->law[j] == LAW_MASS_ACTION) {
                float acc = c[j];
                int zero = 0;
                for (int s = 0; s < N; ++s)
                    if (x[s] < md->order[j * N + s])
                        zero = 1;
                if (zero) {
                    a[j] = 0.0f;
                    continue;
                }
                for (int s = 0; s < N; ++s)
                    for (int i = 0; i < md->order[j * N + s]; ++i)
                        acc = acc * (float)(x[s] - i);
                a[j] = acc;
            } else {
                float q = (float)x[md->hill_reg[j]] / hK[j];
                float qh = q;
                for (int i = 1; i < md->hill_h[j]; ++i)
                    qh = qh * q;
                float d = 1.0f + qh;
                float f;
                if (md->law[j] == LAW_HILL_REPRESS)
                    f = c[j] / d;
                else
                    f = (c[j] * qh) / d;
                a[j] = hb[j] + f;
            }
        }
        S[0] = a[0];
        for (int j = 1; j < M; ++j)
            S[j] = S[j - 1] + a[j];
        float a0 = S[M - 1];
        if (!(a0 <= 3.40282347e38f)) { status = ST_OVERFLOW; break; }
        if (!(a0 > 0.0f)) { status = ST_ABSORBED; break; }
        float tau = or_nlog32(u1) / a0;
        float t_new = t + tau;
        while (k < K && (float)run->snap_t[k] < t_new) {
            write_snap(o, k, N, x);
            ++k;
        }
        if (t_new > t_end) { status = ST_DONE; break; }
        float target = u2 * a0;
        for (int j = 0; j < M; ++j) {
            Sd[j] = S[j];
            ad[j] = a[j];
        }
        int mu = select_mu(M, Sd, ad, (double)target);
        for (int s = 0; s < N; ++s)
            x[s] += md->nu[mu * N + s];
        t = t_new;
        ++n;
        record(o, &rec_cnt, mu, (double)t);
        if (run->max_events && n == run->max_events) { status = ST_CAPPED; break; }
    }
    for (; k < K; ++k)
        write_snap(o, k, N, x);
    finish_record(o, rec_cnt);
    *n_out = n;
    *t_out = (double)t;
    *st_out = (uint8_t)status;
}

/* ------------------------------------------------------------------------- */
/* 16-bit modes.                                                              */
/* Each op on 16-bit values is the binary32 op (exact or correctly rounded),  */
/* then one rounding to the 16-bit format: RNE, or SR with the halfword of    */
/* its static slot.                                                           */
/*                                                                            */
/* Slot schedule per event (slot numbers are fixed by the model, so skipped   */
/* ops leave their slots unused). Two kinds of slots:                        */
/*   main slots - propensity ops other than count conversions, reaction by   */
/*     reaction, op by op [0, P); then, uniform mode, in order: M            */
/*     normalisations (if norm), M-1 partial sums, -ln(u1), tau, tau/m (if   */
/*     norm), t + tau, u2 * a0;                                              */
/*   conversion slots - the int -> 16-bit conversions of counts, in the same */
/*     op order [0, C).                                                      */
/* With SR only at accumulation points (the paper's "selective SR", Sec. 3.3  */
/* last paragraph) the partial sums take main slots 0..M-2 and the clock      */
/* update slot M-1; every other op rounds to nearest and takes no slot.       */
/*                                                                            */
/* Random field of a slot (Sec. 3.3: SR to fp16 discards 13 mantissa bits of  */
/* a binary32 result, to bf16 16, and needs that many random bits; B = 13 or  */
/* 16). A string of bits is cut into B-bit fields from its low end: field r   */
/* is bits [rB, rB + B), bit 0 being bit 0 of the string's first word, and    */
/* fields may span two words. Main slots: the first F0 = floor(80/B) are the  */
/* fields of the 80-bit string (word 2, word 3, then the low bytes of words 0 */
/* and 1) of the event's stream-0 draw, whose words 0 and 1 give the two      */
/* 24-bit uniforms from their high bits; main slot F0 + F1 q + r is field r   */
/* of the 128-bit string of the stream-(q+1) draw (F1 = floor(128/B)).        */
/* Conversion slot F1 q + r is field r of the stream-(2^31 + q) draw. A       */
/* conversion's bits matter only when the count is not exactly representable */
/* (|count| > 2^11 fp16, 2^8 bf16). The field f is passed to or_round16 as   */
/* the halfword f << (16 - B).                                               */
/* ------------------------------------------------------------------------- */
#define SR_CONV_STREAM 0x80000000u

typedef struct {
    uint64_t seed;
    uint32_t id;
    uint64_t n;
    int B;             /* field width */
    uint32_t w0[4];
    int have;          /* main extra streams drawn so far */
    uint32_t ws[64][4];
    int have_cv;       /* conversion streams drawn so far */
    uint32_t wc[64][4];
} sr_ctx;

/* bits [off, off + B) of a little-endian string of 32-bit words */
static uint32_t bit_field(const uint32_t *w, int off, int B)
{
    uint64_t pair = (uint64_t)w[off / 32];
    if (off % 32 + B > 32)
        pair |= (uint64_t)w[off / 32 + 1] << 32;
    return (uint32_t)((pair >> (off % 32)) & ((1u << B) - 1u));
}

static int sr_bits(sr_ctx *c, int slot)
{
    const int B = c->B, F0 = 80 / B, F1 = 128 / B;
    uint32_t f;
    if (slot < F0) {
        uint32_t s0[3] = {c->w0[2], c->w0[3], (c->w0[0] & 0xFFu) | ((c->w0[1] & 0xFFu) << 8)};
        f = bit_field(s0, slot * B, B);
    } else {
        int q = (slot - F0) / F1, r = (slot - F0) % F1;
        while (c->have <= q) {
            draw(c->seed, c->id, c->n, (uint32_t)(c->have + 1), c->ws[c->have]);
            c->have++;
        }
        f = bit_field(c->ws[q], r * B, B);
    }
    return (int)(f << (16 - B));
}

static int sr_conv_bits(sr_ctx *c, int slot)
{
    const int B = c->B, F1 = 128 / B;
    int q = slot / F1, r = slot % F1;
    while (c->have_cv <= q) {
        draw(c->seed, c->id, c->n, SR_CONV_STREAM + (uint32_t)c->have_cv, c->wc[c->have_cv]);
        c->have_cv++;
    }
    return (int)(bit_field(c->wc[q], r * B, B) << (16 - B));
}

typedef struct {
    int fmt;
    int sr;
    sr_ctx *ctx;
} rounder;

/* Round the float result of one op; 'slot' is that op's static main slot. */
static float rnd(const rounder *R, float v, int slot)
{
    int rb = R->sr ? sr_bits(R->ctx, slot) : -1;
    return (float)or_round16(R->fmt, (double)v, rb);
}

/* Round a converted count; 'slot' is its conversion slot. */
static float rnd_conv(const rounder *R, float v, int slot)
{
    int rb = R->sr ? sr_conv_bits(R->ctx, slot) : -1;
    return (float)or_round16(R->fmt, (double)v, rb);
}

static void traj_16(const or_model *md, or_mode mode, const or_run *run, int64_t idx,
                    const or_out *o, uint64_t *n_out, double *t_out, uint8_t *st_out)
{
    const int N = md->n_species, M = md->n_reactions, K = run->n_snap;
    const uint32_t id = run->traj_id_base + (uint32_t)idx;
    const int uni = mode.uniform, norm = mode.uniform && mode.norm;
    const int selective = mode.sr == 2;
    int32_t x[MAXN];
    float c[MAXM], hb[MAXM], hK[MAXM];
    int base[MAXM], cbase[MAXM];
    int P = 0, C = 0;
    for (int s = 0; s < N; ++s)
        x[s] = run->x0[s];
    for (int j = 0; j < M; ++j) {
        double k = primary_rate(md, run, idx, j);
        double cj = md->law[j] == LAW_MASS_ACTION ? folded_constant(md, j, k) : k;
        /* constants: one round-to-nearest from FP64, also in SR modes */
        c[j] = (float)or_round16(mode.fmt, cj, -1);
        hb[j] = (float)or_round16(mode.fmt, md->hill_b ? md->hill_b[j] : 0.0, -1);
        hK[j] = (float)or_round16(mode.fmt, md->hill_K ? md->hill_K[j] : 1.0, -1);
        base[j] = P;
        P += reaction_main_ops(md, j);
        cbase[j] = C;
        C += reaction_conv_ops(md, j);
    }
    /* accumulation-phase slots (uniform mode) */
    const int slot_norm = P;
    const int slot_sum = selective ? 0 : P + (norm ? M : 0);  /* S_j uses slot_sum + j - 1 */
    const int slot_log = slot_sum + (M - 1);
    const int slot_tau = slot_log + 1;
    const int slot_taum = slot_tau + 1;           /* norm only */
    const int slot_time = selective ? M - 1 : slot_tau + 1 + (norm ? 1 : 0);
    const int slot_target = slot_time + 1;

    const float t_end = (float)run->t_end;
    float t = 0.0f;     /* FP32 (mixed) or a 16-bit value (uniform) */
    float mx_run = 0.0f;
    uint64_t n = 0;
    int k = 0, status;
    uint32_t rec_cnt = 0;
    sr_ctx ctx;
    rounder R = {mode.fmt, mode.sr == 1, &ctx};    /* propensity and other ops */
    rounder RA = {mode.fmt, mode.sr >= 1, &ctx};   /* partial sums and the clock */
    for (;;) {
        ctx.seed = run->seed;
        ctx.id = id;
        ctx.n = n;
        ctx.have = 0;
        ctx.have_cv = 0;
        ctx.B = mode.fmt == OR_FP16 ? 13 : 16;
        draw(run->seed, id, n, 0, ctx.w0);
        float u1 = or_u24(ctx.w0[0]);
        float u2 = or_u24(ctx.w0[1]);
        float a[MAXM], S[MAXM];
        double Sd[MAXM], ad[MAXM];
        for (int j = 0; j < M; ++j) {
            int sl = base[j], cs = cbase[j];
            if (md->law[j] == LAW_MASS_ACTION) {
                int zero = 0;
                for (int s = 0; s < N; ++s)
                    if (x[s] < md->order[j * N + s])
                        zero = 1;
                if (zero) {
                    a[j] = 0.0f;
                    continue;
                }
                float acc = c[j];
                for (int s = 0; s < N; ++s)
                    for (int i = 0; i < md->order[j * N + s]; ++i) {
                        float fv = rnd_conv(&R, (float)(x[s] - i), cs++);
                        acc = rnd(&R, acc * fv, sl++);
                    }
                a[j] = acc;
            } else {
                float xr = rnd_conv(&R, (float)x[md->hill_reg[j]], cs++);
                float q = rnd(&R, xr / hK[j], sl++);
                float qh = q;
                for (int i = 1; i < md->hill_h[j]; ++i)
                    qh = rnd(&R, qh * q, sl++);
                float d = rnd(&R, 1.0f + qh, sl++);
                float f;
                if (md->law[j] == LAW_HILL_REPRESS) {
                    f = rnd(&R, c[j] / d, sl++);
                } else {
                    float g = rnd(&R, c[j] * qh, sl++);
                    f = rnd(&R, g / d, sl++);
                }
                a[j] = rnd(&R, hb[j] + f, sl++);
            }
        }
        /* summands: a_j, or a_j / m with m the running maximum (norm) */
        float m = 1.0f;
        if (norm) {
            float mx = 0.0f;
            for (int j = 0; j < M; ++j)
                if (a[j] > mx)
                    mx = a[j];
            if (mx > mx_run)
                mx_run = mx;
            if (!(mx_run <= 3.40282347e38f)) { status = ST_OVERFLOW; break; }
            if (!(mx_run > 0.0f)) { status = ST_ABSORBED; break; }
            m = mx_run;
            for (int j = 0; j < M; ++j)
                a[j] = rnd(&R, a[j] / m, slot_norm + j);
        }
        S[0] = a[0];
        for (int j = 1; j < M; ++j)
            S[j] = uni ? rnd(&RA, S[j - 1] + a[j], slot_sum + j - 1) : S[j - 1] + a[j];
        float a0 = S[M - 1];
        if (!(a0 <= 3.40282347e38f)) { status = ST_OVERFLOW; break; }
        if (!(a0 > 0.0f)) { status = ST_ABSORBED; break; }
        float L = or_nlog32(u1);
        float tau, t_new;
        if (uni) {
            L = rnd(&R, L, slot_log);
            tau = rnd(&R, L / a0, slot_tau);
            if (norm)
                tau = rnd(&R, tau / m, slot_taum);
            t_new = rnd(&RA, t + tau, slot_time);
        } else {
            tau = L / a0;
            t_new = t + tau;
        }
        while (k < K && (float)run->snap_t[k] < t_new) {
            write_snap(o, k, N, x);
            ++k;
        }
        if (t_new > t_end) { status = ST_DONE; break; }
        float target = uni ? rnd(&R, u2 * a0, slot_target) : u2 * a0;
        for (int j = 0; j < M; ++j) {
            Sd[j] = S[j];
            ad[j] = a[j];
        }
        int mu = select_mu(M, Sd, ad, (double)target);
        for (int s = 0; s < N; ++s)
            x[s] += md->nu[mu * N + s];
        t = t_new;
        ++n;
        record(o, &rec_cnt, mu, (double)t);
        if (run->max_events && n == run->max_events) { status = ST_CAPPED; break; }
    }
    for (; k < K; ++k)
        write_snap(o, k, N, x);
    finish_record(o, rec_cnt);
    *n_out = n;
    *t_out = (double)t;
    *st_out = (uint8_t)status;
}

/* ------------------------------------------------------------------------- */
/* Ensemble driver over a list of trajectory indices.                        */
/* Outputs: snap [K][N][count], n_events/t_last/status [count], and with rec */
/* the event record ([count][cap] times and reactions, [count] counts).      */
/* Returns 0, or -1 for an argument the oracle does not handle.              */
/* ------------------------------------------------------------------------- */
int or_simulate(const or_model *md, or_mode mode, const or_run *run, const int64_t *idx,
                int64_t count, int32_t *snap, uint64_t *n_events, double *t_last,
                uint8_t *status, const or_rec *rec, int32_t n_threads)
{
    if (md->n_species < 1 || md->n_species > MAXN || md->n_reactions < 1 ||
        md->n_reactions > MAXM || run->n_snap < 0)
        return -1;
    if (mode.fmt < OR_FP64 || mode.fmt > OR_BF16 || mode.sr < 0 || mode.sr > 2)
        return -1;
    if (mode.sr == 2 && !mode.uniform)
        return -1;
    if (run->set_rate && run->traj_per_set < 1)
        return -1;
    if (rec && (rec->cap < 0 || (rec->cap > 0 && (!rec->t || !rec->j)) || !rec->n))
        return -1;
    if (mode.fmt >= OR_FP16) {
        /* the random-field streams an event may draw must fit sr_ctx */
        int P = 0, C = 0, M = md->n_reactions;
        for (int j = 0; j < M; ++j) {
            P += reaction_main_ops(md, j);
            C += reaction_conv_ops(md, j);
        }
        const int B = mode.fmt == OR_FP16 ? 13 : 16;
        if (P + 2 * M + 4 > 80 / B + 64 * (128 / B) || C > 64 * (128 / B))
            return -1;
    }
    if (n_threads < 1)
        n_threads = 1;
    int64_t i;
#pragma omp parallel for schedule(dynamic, 4) num_threads(n_threads)
    for (i = 0; i < count; ++i) {
        or_out o = {snap, count, i, rec};
        if (mode.fmt == OR_FP64)
            traj_fp64(md, run, idx[i], &o, &n_events[i], &t_last[i], &status[i]);
        else if (mode.fmt == OR_FP32)
            traj_fp32(md, run, idx[i], &o, &n_events[i], &t_last[i], &status[i]);
        else
            traj_16(md, mode, run, idx[i], &o, &n_events[i], &t_last[i], &status[i]);
    }
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Vectorised numerics entry points used by the pin tests.                    */
/* ------------------------------------------------------------------------- */
/* SR random fields as the trajectory code reads them: for each i, the       */
/* halfword (field << (16 - B)) of main slot (conv[i] == 0) or conversion    */
/* slot (conv[i] != 0) slot[i] of event n[i] of trajectory id[i].            */
void or_sr_field_batch(int fmt, uint64_t seed, const uint32_t *id, const uint64_t *n, const int32_t *slot,
                       const int32_t *conv, int32_t *out, int64_t count)
{
    for (int64_t i = 0; i < count; ++i) {
        sr_ctx c;
        c.seed = seed;
        c.id = id[i];
        c.n = n[i];
        c.B = fmt == OR_FP16 ? 13 : 16;
        c.have = 0;
        c.have_cv = 0;
        draw(seed, id[i], n[i], 0, c.w0);
        out[i] = conv[i] ? sr_conv_bits(&c, slot[i]) : sr_bits(&c, slot[i]);
    }
}

void or_philox_batch(const uint32_t *ctr, const uint32_t *key, uint32_t *out, int64_t n)
{
    for (int64_t i = 0; i < n; ++i)
        or_philox4x32_10(ctr + 4 * i, key + 2 * i, out + 4 * i);
}

void or_nlog64_batch(const double *u, double *out, int64_t n)
{
    for (int64_t i = 0; i < n; ++i)
        out[i] = or_nlog64(u[i]);
}

void or_nlog32_batch(const float *u, float *out, int64_t n)
{
    for (int64_t i = 0; i < n; ++i)
        out[i] = or_nlog32(u[i]);
}

void or_round16_batch(int fmt, const double *v, const int32_t *rb, double *out, int64_t n)
{
    for (int64_t i = 0; i < n; ++i)
        out[i] = or_round16(fmt, v[i], rb ? rb[i] : -1);
}

void or_uniform_batch(const uint32_t *w, double *u53, float *u24, int64_t n)
{
    for (int64_t i = 0; i < n; ++i) {
        u53[i] = or_u53(w[2 * i], w[2 * i + 1]);
        u24[i] = or_u24(w[2 * i]);
    }
}
