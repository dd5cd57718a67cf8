// ssa_capi.cpp - host side of libssa_rp.so: the C ABI declared in ssa_rp.h.
//
//  * ssa_model_create validates a reaction network and keeps a copy.
//  * ssa_ensemble_run rounds the rate constants once to the run's precision,
//    generates the network description for the device template
//    (ssa_device.hip), compiles it for gfx950 with ROCm's offline clang
//    (hipRTC where there is none; cached in memory and on disk), uploads
//    tables and launches the persistent kernel, in one launch or in
//    snapshot-window chunks (direct launches, or beyond kGraphMinChunks
//    windows one hipGraph captured and launched per run).
//  * getters copy results out; ssa_run_info_get reports HIP-event timings.
#include "ssa_rp.h"

#include <hip/hip_runtime.h>
#include <hip/hiprtc.h>

#include <dlfcn.h>
#include <fcntl.h>
#include <spawn.h>
#include <sys/stat.h>
#include <sys/wait.h>
#include <unistd.h>

#include <cerrno>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <map>
#include <memory>
#include <mutex>
#include <sstream>
#include <string>
#include <unordered_map>
#include <vector>

#include "ssa_device_src.inc"  // const char kDeviceSource[] (ssa_device.hip)

namespace {

// ------------------------------------------------------------------ errors
thread_local std::string g_err;

int fail(int code, const std::string &msg)
{
    g_err = msg;
    return code;
}

#define HIP_TRY(expr)                                                                          \
    do {                                                                                       \
        hipError_t e_ = (expr);                                                                \
        if (e_ != hipSuccess)                                                                  \
            return fail(SSA_E_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_));      \
    } while (0)

// ------------------------------------------------------------------ models
struct Model {
    int N = 0, M = 0;
    std::vector<int32_t> order;  // [M][N]
    std::vector<int32_t> nu;     // [M][N]
    std::vector<ssa_law> law;    // [M]
};

constexpr int kMaxSpecies = 32;
constexpr int kMaxReactions = 64;
constexpr int kMaxOrder = 4;
constexpr int kMaxSnap = 65536;
constexpr int kGraphMinChunks = 16;

int64_t factorial(int n)
{
    int64_t f = 1;
    for (int i = 2; i <= n; ++i)
        f *= i;
    return f;
}

// Propensity constant of reaction j from its k: mass action divides by
// prod_s o_s! (one binary64 division), Hill uses vmax as given.
double primary_constant(const Model &md, int j, double k)
{
    if (md.law[j].kind != SSA_LAW_MASS_ACTION)
        return k;
    int64_t d = 1;
    for (int s = 0; s < md.N; ++s)
        d *= factorial(md.order[(size_t)j * md.N + s]);
    return k / (double)d;
}

// Round-to-nearest-even of a binary64 value onto a floating grid with p
// significand bits, smallest normal exponent emin and overflow threshold ovf.
double round_to_grid(double v, int p, int emin, double ovf)
{
    if (std::isnan(v) || std::isinf(v) || v == 0.0)
        return v;
    double a = std::fabs(v);
    int e = std::ilogb(a);
    if (e < emin)
        e = emin;
    double step = std::ldexp(1.0, e - (p - 1));
    double r = std::nearbyint(a / step) * step;  // default rounding: ties to even
    if (r >= ovf)
        r = INFINITY;
    return std::copysign(r, v);
}

// Value of constant v in the run's propensity type, widened to double.
double to_prop_type(int fmt, double v)
{
    switch (fmt) {
    case SSA_FMT_FP64: return v;
    case SSA_FMT_FP32: return (double)(float)v;
    case SSA_FMT_FP16: return round_to_grid(v, 11, -14, 65536.0);
    default: return round_to_grid(v, 8, -126, std::ldexp(1.0, 128));
    }
}

}  // namespace

struct ssa_model {
    Model m;
};

namespace {

// ------------------------------------------------------------------ codegen
int mass_action_total_order(const Model &md, int j)
{
    int t = 0;
    for (int s = 0; s < md.N; ++s)
        t += md.order[(size_t)j * md.N + s];
    return t;
}

// Rounding ops of reaction j: count conversions (conversion slots) and the
// other ops (main slots): mass action one of each per factor; Hill one
// conversion and q = x/K, h-1 powers, 1 + q^h, v/d (activation also v q^h),
// b + f.
int reaction_conv_slots(const Model &md, int j)
{
    return md.law[j].kind == SSA_LAW_MASS_ACTION ? mass_action_total_order(md, j) : 1;
}

int reaction_main_slots(const Model &md, int j)
{
    const ssa_law &L = md.law[j];
    if (L.kind == SSA_LAW_MASS_ACTION)
        return mass_action_total_order(md, j);
    return L.h + (L.kind == SSA_LAW_HILL_REPRESS ? 3 : 4);
}

// Propensities for round-to-nearest fp16 (P::NATIVE16): the same op sequence
// per reaction (a_j = c_j times its falling-factorial factors, left to right),
// with the mass-action chains of two reactions advanced together: their k-th
// products form one packed fp16 multiply (v_pk_mul_f16, two IEEE fp16
// products). Reactions are paired longest chain first, so paired chains
// share most of their steps. Hill laws are computed as in the other modes.
std::string gen_propensities_packed(const Model &md)
{
    std::ostringstream o;
    std::vector<int> ma;   // mass-action reactions with at least one factor
    std::vector<std::vector<std::pair<int, int>>> fac((size_t)md.M);
    for (int j = 0; j < md.M; ++j) {
        if (md.law[j].kind != SSA_LAW_MASS_ACTION)
            continue;
        for (int s = 0; s < md.N; ++s)
            for (int i = 0; i < md.order[(size_t)j * md.N + s]; ++i)
                fac[(size_t)j].push_back({s, i});
        if (!fac[(size_t)j].empty())
            ma.push_back(j);
    }
    std::stable_sort(ma.begin(), ma.end(),
                     [&](int a, int b) { return fac[(size_t)a].size() > fac[(size_t)b].size(); });
    o << "      typedef _Float16 h2 __attribute__((ext_vector_type(2)));\n";
    auto f16 = [](const std::pair<int, int> &f) {
        return "(_Float16)P::template cvt_sub<EXACT>(x[" + std::to_string(f.first) + "], " +
               std::to_string(f.second) + ", 0u)";
    };
    for (size_t p = 0; p < ma.size(); p += 2) {
        const int j0 = ma[p];
        if (p + 1 == ma.size()) {
            o << "      { _Float16 r = (_Float16)c[" << j0 << "];\n";
            for (const auto &f : fac[(size_t)j0])
                o << "        r = r * " << f16(f) << ";\n";
            o << "        a[" << j0 << "] = (float)r; }\n";
            continue;
        }
        const int j1 = ma[p + 1];
        const size_t n0 = fac[(size_t)j0].size(), n1 = fac[(size_t)j1].size();   // n0 >= n1
        o << "      { h2 r = {(_Float16)c[" << j0 << "], (_Float16)c[" << j1 << "]};\n";
        for (size_t k = 0; k < n1; ++k)
            o << "        r = r * (h2){" << f16(fac[(size_t)j0][k]) << ", " << f16(fac[(size_t)j1][k]) << "};\n";
        o << "        _Float16 r0 = r.x;\n";
        for (size_t k = n1; k < n0; ++k)
            o << "        r0 = r0 * " << f16(fac[(size_t)j0][k]) << ";\n";
        o << "        a[" << j0 << "] = (float)r0; a[" << j1 << "] = (float)r.y; }\n";
    }
    for (int j = 0; j < md.M; ++j) {
        const ssa_law &L = md.law[j];
        if (L.kind == SSA_LAW_MASS_ACTION) {
            if (fac[(size_t)j].empty()) {
                o << "      a[" << j << "] = c[" << j << "];\n";
                continue;
            }
            std::string zero;
            for (int s = 0; s < md.N; ++s) {
                int os = md.order[(size_t)j * md.N + s];
                if (os > 0)
                    zero += (zero.empty() ? "" : " || ") + std::string("x[") + std::to_string(s) + "] < " +
                            std::to_string(os);
            }
            o << "      if (GUARD && (" << zero << ")) a[" << j << "] = (T)0;\n";
        } else {
            o << "      { T xr = P::template cvt<EXACT>(x[" << L.regulator << "], 0u);\n"
              << "        T q = P::div(xr, hill[" << 2 * j + 1 << "], 0u);\n"
              << "        T qh = q;\n";
            for (int i = 1; i < L.h; ++i)
                o << "        qh = P::mul(qh, q, 0u);\n";
            o << "        T d = P::add((T)1, qh, 0u);\n";
            if (L.kind == SSA_LAW_HILL_REPRESS) {
                o << "        T f = P::div(c[" << j << "], d, 0u);\n";
            } else {
                o << "        T g = P::mul(c[" << j << "], qh, 0u);\n"
                  << "        T f = P::div(g, d, 0u);\n";
            }
            o << "        a[" << j << "] = P::add(hill[" << 2 * j << "], f, 0u); }\n";
        }
    }
    return o.str();
}

// Device description of one network: propensity op sequence with its static
// rounding slots (main and conversion), and the integer update x += nu_mu.
std::string gen_model(const Model &md, int idx, uint64_t record_mask)
{
    int nprop = 0, nconv = 0;
    for (int j = 0; j < md.M; ++j) {
        nprop += reaction_main_slots(md, j);
        nconv += reaction_conv_slots(md, j);
    }
    // lo[s]: the largest order of species s in a mass-action reactant list.
    // With every count at or above it, no mass-action propensity needs its
    // zero guard (a count below the order makes the falling factorial zero).
    std::vector<int> lo((size_t)md.N, 0);
    for (int j = 0; j < md.M; ++j)
        if (md.law[j].kind == SSA_LAW_MASS_ACTION)
            for (int s = 0; s < md.N; ++s)
                lo[(size_t)s] = std::max(lo[(size_t)s], md.order[(size_t)j * md.N + s]);
    int lo_max = 0;
    for (int s = 0; s < md.N; ++s)
        lo_max = std::max(lo_max, lo[(size_t)s]);
    std::ostringstream o;
    o << "struct Md" << idx << " {\n"
      << "  static constexpr int N = " << md.N << ", M = " << md.M << ", NPROP = " << nprop << ", NCONV = " << nconv
      << ";\n"
      << "  static constexpr u64 REC = " << record_mask << "ull;  // reactions whose firings are recorded\n"
      << "  static constexpr int LO_MAX = " << lo_max << ";  // largest reactant order of a species\n"
      << "  // some count below its species' largest reactant order (a zero guard may apply);\n"
      << "  // counts are never negative, so x - lo < 0 exactly when x < lo, and the OR of\n"
      << "  // the differences is negative when one of them is (one compare for the wave)\n"
      << "  __device__ static __forceinline__ bool below(const i32 (&x)[N]) {\n"
      << "    (void)x;\n"
      << "    return (0";
    for (int s = 0; s < md.N; ++s)
        if (lo[(size_t)s] > 0)
            o << " | (x[" << s << "] - " << lo[(size_t)s] << ")";
    o << ") < 0;\n  }\n"
      << "  // max over species of count - largest order, as unsigned (a count below\n"
      << "  // its order wraps to a large value)\n"
      << "  __device__ static __forceinline__ u32 range_key(const i32 (&x)[N]) {\n"
      << "    u32 r = (u32)(x[0] - " << lo[0] << ");\n";
    for (int s = 1; s < md.N; ++s)
        o << "    r = (u32)(x[" << s << "] - " << lo[(size_t)s] << ") > r ? (u32)(x[" << s << "] - " << lo[(size_t)s]
          << ") : r;\n";
    o << "    return r;\n  }\n"
      << "  // GUARD = false: every count is at or above its species' largest order\n"
      << "  template <class P, bool EXACT, bool GUARD, class PoolT, class CPoolT>\n"
      << "  __device__ static __forceinline__ void propensities(const i32 (&x)[N], const typename P::T (&c)[M],"
      << " const typename P::T *hill, typename P::T (&a)[M], const PoolT &pool, const CPoolT &cpool) {\n"
      << "    typedef typename P::T T;\n"
      << "    (void)hill; (void)pool; (void)cpool;\n"
      << "    if constexpr (P::NATIVE16) {\n"
      << gen_propensities_packed(md)
      << "    } else {\n";
    int slot = 0, cslot = 0;
    for (int j = 0; j < md.M; ++j) {
        const ssa_law &L = md.law[j];
        if (L.kind == SSA_LAW_MASS_ACTION) {
            if (mass_action_total_order(md, j) == 0) {
                o << "    a[" << j << "] = c[" << j << "];\n";
                continue;
            }
            o << "    { T acc = c[" << j << "];\n";
            std::string zero;
            for (int s = 0; s < md.N; ++s) {
                int os = md.order[(size_t)j * md.N + s];
                for (int i = 0; i < os; ++i) {
                    o << "      acc = P::mul(acc, P::template cvt_sub<EXACT>(x[" << s << "], " << i << ", cpool.hw("
                      << cslot << ")), pool.hw(" << slot << "));\n";
                    slot += 1;
                    cslot += 1;
                }
                if (os > 0) {
                    if (!zero.empty())
                        zero += " || ";
                    zero += "x[" + std::to_string(s) + "] < " + std::to_string(os);
                }
            }
            o << "      a[" << j << "] = (GUARD && (" << zero << ")) ? (T)0 : acc; }\n";
        } else {
            int b = slot;
            o << "    { T xr = P::template cvt<EXACT>(x[" << L.regulator << "], cpool.hw(" << cslot++ << "));\n"
              << "      T q = P::div(xr, hill[" << 2 * j + 1 << "], pool.hw(" << b << "));\n"
              << "      T qh = q;\n";
            int sl = b + 1;
            for (int i = 1; i < L.h; ++i)
                o << "      qh = P::mul(qh, q, pool.hw(" << sl++ << "));\n";
            o << "      T d = P::add((T)1, qh, pool.hw(" << sl++ << "));\n";
            if (L.kind == SSA_LAW_HILL_REPRESS) {
                o << "      T f = P::div(c[" << j << "], d, pool.hw(" << sl++ << "));\n";
            } else {
                o << "      T g = P::mul(c[" << j << "], qh, pool.hw(" << sl++ << "));\n"
                  << "      T f = P::div(g, d, pool.hw(" << sl++ << "));\n";
            }
            o << "      a[" << j << "] = P::add(hill[" << 2 * j << "], f, pool.hw(" << sl++ << ")); }\n";
            slot = sl;
        }
    }
    o << "    }\n";
    // x += nu_mu, mu in [0, M] (mu = M: nothing fires). A species whose net
    // changes fit W-bit signed fields for all M + 1 values of mu reads its
    // change from one packed constant with a single bitfield extract; any other
    // species sums one select per reaction.
    o << "  }\n"
      << "  __device__ static __forceinline__ void update(i32 (&x)[N], int mu) {\n";
    for (int s = 0; s < md.N; ++s) {
        int lo = 0, hi = 0;
        for (int j = 0; j < md.M; ++j) {
            int d = md.nu[(size_t)j * md.N + s];
            lo = d < lo ? d : lo;
            hi = d > hi ? d : hi;
        }
        if (lo == 0 && hi == 0)
            continue;
        int width = 0;
        for (int w = 2; w <= 16; ++w) {
            if (lo >= -(1 << (w - 1)) && hi <= (1 << (w - 1)) - 1 && (md.M + 1) * w <= 32) {
                width = w;
                break;
            }
        }
        if (width) {
            uint32_t pack = 0;
            for (int j = 0; j < md.M; ++j) {
                uint32_t field = (uint32_t)md.nu[(size_t)j * md.N + s] & ((1u << width) - 1u);
                pack |= field << (j * width);
            }
            o << "    x[" << s << "] += __builtin_amdgcn_sbfe((i32)" << pack << "u, (u32)mu * " << width << "u, "
              << width << "u);\n";
            continue;
        }
        std::string terms;
        for (int j = 0; j < md.M; ++j) {
            int d = md.nu[(size_t)j * md.N + s];
            if (d == 0)
                continue;
            if (!terms.empty())
                terms += " + ";
            terms += "(mu == " + std::to_string(j) + " ? " + std::to_string(d) + " : 0)";
        }
        o << "    x[" << s << "] += " << terms << ";\n";
    }
    o << "  }\n};\n";
    return o.str();
}

struct ModeSpec {
    int fmt, accum, rnd, norm;
    std::string policy() const
    {
        if (fmt == SSA_FMT_FP64)
            return "PrecF64";
        if (fmt == SSA_FMT_FP32)
            return "PrecF32";
        std::string f = fmt == SSA_FMT_FP16 ? "FMT_FP16" : "FMT_BF16";
        return "Prec16<" + f + ", " + std::to_string(rnd) + ", " +
               (accum == SSA_ACC_UNIFORM ? "true" : "false") + ", " +
               (norm == SSA_NORM_RUNNING_MAX ? "true" : "false") + ">";
    }
};

std::string gen_source(const std::vector<const Model *> &models, const ModeSpec &ms,
                       const std::vector<bool> &per_lane_rates, const std::vector<uint64_t> &record_masks)
{
    std::ostringstream o;
    o << "#define SSA_N_ITEMS " << models.size() << "\n" << kDeviceSource << "\n";
    for (size_t i = 0; i < models.size(); ++i)
        o << gen_model(*models[i], (int)i, record_masks[i]);
    o << "typedef " << ms.policy() << " PrecRun;\n"
      << "extern \"C\" __global__ void __launch_bounds__(256) ssa_kernel(LaunchArgs L) {\n"
      << "  const u32 wave = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;\n"
      << "  const u32 slot_rank = (threadIdx.x >> 6) * gridDim.x + blockIdx.x, n_slots = gridDim.x * (blockDim.x >> 6);\n"
      << "  SelfFeed feed;\n"
      << "  u32 it = wave % SSA_N_ITEMS;\n"
      << "  for (u32 i = 0; i < SSA_N_ITEMS; ++i) {\n"
      << "    switch (it) {\n";
    for (size_t i = 0; i < models.size(); ++i)
        o << "    case " << i << ": run_item<PrecRun, Md" << i << ", " << (per_lane_rates[i] ? "true" : "false")
          << ">(L, L.item[" << i << "], feed, slot_rank, n_slots); break;\n";
    o << "    default: break;\n"
      << "    }\n"
      << "    it = it + 1 == SSA_N_ITEMS ? 0 : it + 1;\n"
      << "  }\n"
      << "}\n";
    // 512-thread workgroups: waves 0-3 run the event loop, wave w + 4 (on the
    // same SIMD as wave w) forms wave w's draws ahead into an LDS ring
    o << "constexpr int SSA_RING_NW = ";
    for (size_t i = 0; i < models.size(); ++i)
        o << (i ? ", " : "") << (i + 1 < models.size() ? "cmax(" : "")
          << "RingWords<PrecRun, Md" << i << ">::NW";
    for (size_t i = 1; i < models.size(); ++i)
        o << ")";
    o << ";\n"
      << "constexpr int SSA_RING_D = ring_depth(SSA_RING_NW);\n"
      << "// 512 threads are two waves per SIMD: at most 256 registers (VGPRs and AGPRs\n"
      << "// together) per wave, which the waves-per-EU bound makes the compiler keep\n"
      << "extern \"C\" __global__ void __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(2, 2)))\n"
      << "ssa_kernel_pc(LaunchArgs L) {\n"
      << "  // wave index made wave-uniform: role branches are scalar branches, so the\n"
      << "  // SALU work of one role (priorities, sleeps) never runs in another role's wave\n"
      << "  const u32 w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = lane_id();\n"
      << "  // event-loop wave c (= w for w < 4) is fed by the producer wave on its own\n"
      << "  // SIMD (w = c + 4) or, with PLACE_NEIGHBOUR, on the next one (w = 4 + (c + 1) % 4).\n"
      << "  // PLACE_DEDICATED: event-loop waves 0, 2, 3; wave 0 alone on SIMD 0 and its\n"
      << "  // producer (wave 5) alone on SIMD 1; waves 2 and 3 fed from their own SIMDs\n"
      << "  const bool ded = (L.place & PLACE_DEDICATED) != 0u;\n"
      << "  const u32 c = w < 4u ? w\n"
      << "              : ded ? (w == 5u ? 0u : w == 4u ? 1u : w - 4u)\n"
      << "                    : ((w + ((L.place & (PLACE_NEIGHBOUR | PLACE_SOLO0)) ? 3u : 0u)) & 3u);\n"
      << "  if constexpr (SSA_RING_D == 0) {\n"
      << "    SelfFeed feed;\n"
      << "    const u32 slot_rank = w * gridDim.x + blockIdx.x, n_slots = gridDim.x * 8u;\n"
      << "    u32 it = (blockIdx.x * 8u + w) % SSA_N_ITEMS;\n"
      << "    for (u32 i = 0; i < SSA_N_ITEMS; ++i) {\n"
      << "      switch (it) {\n";
    for (size_t i = 0; i < models.size(); ++i)
        o << "      case " << i << ": run_item<PrecRun, Md" << i << ", " << (per_lane_rates[i] ? "true" : "false")
          << ">(L, L.item[" << i << "], feed, slot_rank, n_slots); break;\n";
    o << "      default: break;\n"
      << "      }\n"
      << "      it = it + 1 == SSA_N_ITEMS ? 0 : it + 1;\n"
      << "    }\n"
      << "    return;\n"
      << "  } else {\n"
      << "  __shared__ RingCtl ctl[4];\n"
      << "  __shared__ u32 ring[4 * (SSA_RING_D > 0 ? SSA_RING_D : 1) * SSA_RING_NW * 64];\n"
      << "  if (w < 4) {\n"
      << "    ctl[c].convw[lane] = 0u;\n"
      << "    ctl[c].req_e[lane] = 0u;\n"
      << "    ctl[c].done[lane] = 0u;\n"
      << "    ctl[c].item = 0u;\n"
      << "  } else {\n"
      << "    ctl[c].made[0][lane] = 0u;\n"
      << "    ctl[c].made[1][lane] = 0u;\n"
      << "  }\n"
      << "  __syncthreads();\n"
      << "  u32 *my_ring = ring + c * (SSA_RING_D * SSA_RING_NW * 64);\n"
      << "  u32 it = (blockIdx.x * 4u + c) % SSA_N_ITEMS;\n"
      << "  const bool solo0 = SSA_N_ITEMS == 1 && (L.place & PLACE_SOLO0) != 0u && !ded;\n"
      << "  // PLACE_TWO0 (with PLACE_DEDICATED, one-item launches): wave 1 is a second\n"
      << "  // producer of wave 0; waves 5 and 1 make its draws of even and odd index\n"
      << "  // (a ring of fewer than 4 slots, for the largest networks, keeps one producer)\n"
      << "  const bool two = SSA_N_ITEMS == 1 && SSA_RING_D >= 4 && ded && (L.place & PLACE_TWO0) != 0u;\n"
      << "  // event-loop slots (the wave-major static claims go in slot order, heaviest\n"
      << "  // first): with PLACE_DEDICATED three per workgroup (waves 0, 2, 3); with\n"
      << "  // PLACE_FEED0 wave 1, which shares its SIMD with wave 0's producer, comes last\n"
      << "  const bool feed0 = (L.place & PLACE_FEED0) != 0u;\n"
      << "  const u32 ev_rank = ded ? (c == 0u ? 0u : c - 1u) : feed0 ? (c == 0u ? 0u : c == 1u ? 3u : c - 1u) : c;\n"
      << "  const u32 ev_per_wg = ded ? 3u : 4u;\n"
      << "  // wave priorities: event-loop waves 3, producers 0; PLACE_PRODUCER_FIRST:\n"
      << "  // producers 3, event-loop waves 2; PLACE_FEED0: wave 0 and its producer 3,\n"
      << "  // event-loop waves 1-3 2, the other producers 0\n"
      << "  const bool pfirst = (L.place & PLACE_PRODUCER_FIRST) != 0u;\n"
      << "  const bool ev_low = pfirst || ((L.place & PLACE_FEED0) != 0u && c != 0u);\n"
      << "  const bool pr_high = pfirst || ((L.place & PLACE_FEED0) != 0u && c == 0u);\n"
      << "  // PLACE_SOLO0 (one-item launches): event-loop wave 3 forms its own draws; a\n"
      << "  // second copy of the event loop per network, so it is compiled only for one\n"
      << "  // network (several networks' copies would crowd the instruction cache)\n"
      << "#if SSA_N_ITEMS == 1\n"
      << "  if (w < 4 && solo0 && c == 3u) {\n"
      << "    if (ev_low) __builtin_amdgcn_s_setprio(2); else __builtin_amdgcn_s_setprio(3);\n"
      << "    SelfFeed feed;\n"
      << "    const u32 slot_rank = ev_rank * gridDim.x + blockIdx.x, n_slots = gridDim.x * 4u;\n"
      << "    for (u32 i = 0; i < SSA_N_ITEMS; ++i) {\n"
      << "      switch (it) {\n";
    for (size_t i = 0; i < models.size(); ++i)
        o << "      case " << i << ": run_item<PrecRun, Md" << i << ", " << (per_lane_rates[i] ? "true" : "false")
          << ">(L, L.item[" << i << "], feed, slot_rank, n_slots); break;\n";
    o << "      default: break;\n"
      << "      }\n"
      << "      it = it + 1 == SSA_N_ITEMS ? 0 : it + 1;\n"
      << "    }\n"
      << "  } else if (two && (w == 1u || w == 5u)) {\n"
      << "    if constexpr (SSA_RING_D >= 4) {\n"
      << "      if (pfirst || feed0) __builtin_amdgcn_s_setprio(3);\n"
      << "      produce_item<PrecRun, Md0, SSA_RING_D, SSA_RING_NW, 2>(L, L.item[0], &ctl[0], ring, 0u, w == 1u ? 1u : 0u);\n"
      << "    }\n"
      << "  } else if (two && w == 0u) {   // the event loop fed by both\n"
      << "    if constexpr (SSA_RING_D >= 4) {\n"
      << "      if (ev_low) __builtin_amdgcn_s_setprio(2); else __builtin_amdgcn_s_setprio(3);\n"
      << "      RingFeed<SSA_RING_D, SSA_RING_NW, true> feed{&ctl[0], ring, lane, 0u, 0u, &ctl[0].made[0][lane]};\n"
      << "      lds_st(&ctl[0].item, 0u);\n"
      << "      lgkm_wait();\n"
      << "      run_item<PrecRun, Md0, " << (per_lane_rates[0] ? "true" : "false")
      << ">(L, L.item[0], feed, blockIdx.x, gridDim.x * ev_per_wg);\n"
      << "      lds_st(&ctl[0].item, ~0u);\n"
      << "    }\n"
      << "  } else\n"
      << "#endif\n"
      << "  if (w < 4 && !(ded && w == 1u)) {   // PLACE_DEDICATED: wave 1 leaves SIMD 1 to wave 5\n"
      << "    if (ev_low) __builtin_amdgcn_s_setprio(2); else __builtin_amdgcn_s_setprio(3);\n"
      << "    RingFeed<SSA_RING_D, SSA_RING_NW> feed{&ctl[c], my_ring, lane, 0u, 0u, &ctl[c].made[0][lane]};\n"
      << "    const u32 slot_rank = ev_rank * gridDim.x + blockIdx.x, n_slots = gridDim.x * ev_per_wg;\n"
      << "    for (u32 i = 0; i < SSA_N_ITEMS; ++i) {\n"
      << "      lds_st(&ctl[c].item, i);\n"
      << "      lgkm_wait();\n"
      << "      switch (it) {\n";
    for (size_t i = 0; i < models.size(); ++i)
        o << "      case " << i << ": run_item<PrecRun, Md" << i << ", " << (per_lane_rates[i] ? "true" : "false")
          << ">(L, L.item[" << i << "], feed, slot_rank, n_slots); break;\n";
    o << "      default: break;\n"
      << "      }\n"
      << "      it = it + 1 == SSA_N_ITEMS ? 0 : it + 1;\n"
      << "    }\n"
      << "    lds_st(&ctl[c].item, ~0u);\n"
      << "  } else if (w >= 4u && !((solo0 || ded) && w == 4u)) {   // PLACE_SOLO0, PLACE_DEDICATED: wave 4 leaves SIMD 0 to wave 0\n"
      << "    if (pr_high) __builtin_amdgcn_s_setprio(3);\n"
      << "    for (u32 i = 0; i < SSA_N_ITEMS; ++i) {\n"
      << "      switch (it) {\n";
    for (size_t i = 0; i < models.size(); ++i)
        o << "      case " << i << ": produce_item<PrecRun, Md" << i
          << ", SSA_RING_D, SSA_RING_NW, 1>(L, L.item[" << i << "], &ctl[c], my_ring, i, 0u); break;\n";
    o << "      default: break;\n"
      << "      }\n"
      << "      it = it + 1 == SSA_N_ITEMS ? 0 : it + 1;\n"
      << "    }\n"
      << "  }\n"
      << "  }\n"
      << "}\n"
      << "extern \"C\" __global__ void ssa_fill_u32(u32 *p, u32 n, u32 v) {\n"
      << "  u32 i = blockIdx.x * blockDim.x + threadIdx.x;\n"
      << "  if (i < n) p[i] = v;\n"
      << "}\n";
    return o.str();
}

// ------------------------------------------------------------------ JIT
// The event loop runs one wave per SIMD, so the instruction schedule should
// hide latency rather than save registers for occupancy: AMDGPU's max-ILP
// scheduling strategy (measured on the Schloegl benchmark: FP64 5% and
// MIX_F16_SR 1% faster per step than the default strategy).
// Spills of a very large network go to scratch, not to AGPRs: some compilers
// (the hipRTC that the PyTorch wheel bundles) add AGPRs beyond the 256
// registers per wave that two waves per SIMD (512-thread workgroups) allow,
// and such a kernel cannot be dispatched at that size.
const char *const kJitOptions[] = {"-O3", "-std=c++17", "-ffp-contract=off", "-Xclang", "-target-feature",
                                   "-Xclang", "-packed-fp32-ops", "-mllvm", "-amdgpu-sched-strategy=max-ilp",
                                   "-mllvm", "-amdgpu-spill-vgpr-to-agpr=0"};

uint64_t fnv1a(const std::string &s, uint64_t h = 1469598103934665603ull)
{
    for (unsigned char ch : s) {
        h ^= ch;
        h *= 1099511628211ull;
    }
    return h;
}

std::string cache_dir()
{
    if (const char *e = std::getenv("SSA_RP_CACHE_DIR"))
        return e;
    Dl_info info;
    if (dladdr((void *)&cache_dir, &info) && info.dli_fname) {
        std::string p = info.dli_fname;
        size_t sl = p.find_last_of('/');
        if (sl != std::string::npos)
            return p.substr(0, sl) + "/_kcache";
    }
    return "_kcache";
}

struct CompiledKernel {
    std::vector<char> code;
};

// ROCm's offline clang, run as a child process, compiles the kernels: the
// in-process hipRTC resolves to whichever comgr the host process loaded first
// (inside PyTorch, the one its wheel bundles), and that compiler gives the
// largest networks' 512-thread kernels more registers than two waves per SIMD
// can hold. SSA_RP_CLANG names another clang; set to an empty string it selects
// hipRTC. Without an offline clang, hipRTC compiles.
std::string offline_compiler()
{
    if (const char *e = std::getenv("SSA_RP_CLANG"))
        return e;
    const char *rp = std::getenv("ROCM_PATH");
    const std::string p = std::string(rp && *rp ? rp : "/opt/rocm") + "/llvm/bin/clang++";
    return ::access(p.c_str(), X_OK) == 0 ? p : std::string();
}

bool read_file(const std::string &path, std::vector<char> &out)
{
    std::ifstream in(path, std::ios::binary);
    if (!in)
        return false;
    out.assign(std::istreambuf_iterator<char>(in), std::istreambuf_iterator<char>());
    return true;
}

// compile src into a gfx950 code object with the clang at cc (child process;
// its messages go to a log file that an error reports)
int compile_offline(const std::string &cc, const std::string &src, const std::string &arch,
                    std::vector<char> &code)
{
    const char *td = std::getenv("TMPDIR");
    char tmpl[512];
    std::snprintf(tmpl, sizeof tmpl, "%s/ssa_rp_jit_XXXXXX", td && *td ? td : "/tmp");
    if (!::mkdtemp(tmpl))
        return fail(SSA_E_COMPILE, std::string("cannot create a directory for the kernel build: ") + tmpl);
    const std::string dir = tmpl, in = dir + "/k.hip", out = dir + "/k.co", log = dir + "/k.log";
    auto cleanup = [&] {
        std::remove(in.c_str());
        std::remove(out.c_str());
        std::remove(log.c_str());
        ::rmdir(dir.c_str());
    };
    {
        std::ofstream f(in, std::ios::binary);
        f.write(src.data(), (std::streamsize)src.size());
        if (!f) {
            cleanup();
            return fail(SSA_E_COMPILE, "cannot write the kernel source to " + in);
        }
    }
    std::vector<std::string> args = {cc, "-x", "hip", "--offload-arch=" + arch, "--offload-device-only",
                                     "--no-gpu-bundle-output", "-include", "hip/hip_runtime.h"};
    for (const char *opt : kJitOptions)
        args.push_back(opt);
    args.insert(args.end(), {"-o", out, in});
    std::vector<char *> argv;
    for (auto &a : args)
        argv.push_back(&a[0]);
    argv.push_back(nullptr);
    posix_spawn_file_actions_t fa;
    posix_spawn_file_actions_init(&fa);
    posix_spawn_file_actions_addopen(&fa, 0, "/dev/null", O_RDONLY, 0);
    posix_spawn_file_actions_addopen(&fa, 1, log.c_str(), O_WRONLY | O_CREAT | O_TRUNC, 0644);
    posix_spawn_file_actions_adddup2(&fa, 1, 2);
    pid_t pid = 0;
    const int se = posix_spawn(&pid, cc.c_str(), &fa, nullptr, argv.data(), environ);
    posix_spawn_file_actions_destroy(&fa);
    if (se != 0) {
        cleanup();
        return fail(SSA_E_COMPILE, "cannot start " + cc + ": " + std::strerror(se));
    }
    int status = 0;
    while (::waitpid(pid, &status, 0) < 0 && errno == EINTR) {
    }
    const bool ok = WIFEXITED(status) && WEXITSTATUS(status) == 0 && read_file(out, code) && !code.empty();
    if (!ok) {
        std::vector<char> msg;
        read_file(log, msg);
        cleanup();
        return fail(SSA_E_COMPILE, "kernel compilation (" + cc + ") failed: " +
                                       std::string(msg.begin(), msg.end()).substr(0, 4000));
    }
    cleanup();
    return SSA_OK;
}

int compile_hiprtc(const std::string &src, const std::string &arch, std::vector<char> &code)
{
    hiprtcProgram prog;
    if (hiprtcCreateProgram(&prog, src.c_str(), "ssa_jit.hip", 0, nullptr, nullptr) != HIPRTC_SUCCESS)
        return fail(SSA_E_COMPILE, "hiprtcCreateProgram failed");
    std::vector<const char *> opts;
    std::string archopt = "--offload-arch=" + arch;
    opts.push_back(archopt.c_str());
    for (const char *opt : kJitOptions)
        opts.push_back(opt);
    hiprtcResult rc = hiprtcCompileProgram(prog, (int)opts.size(), opts.data());
    if (rc != HIPRTC_SUCCESS) {
        size_t ls = 0;
        hiprtcGetProgramLogSize(prog, &ls);
        std::string log(ls, '\0');
        if (ls)
            hiprtcGetProgramLog(prog, &log[0]);
        hiprtcDestroyProgram(&prog);
        return fail(SSA_E_COMPILE, "hipRTC compilation failed: " + log.substr(0, 4000));
    }
    size_t cs = 0;
    hiprtcGetCodeSize(prog, &cs);
    code.resize(cs);
    hiprtcGetCode(prog, code.data());
    hiprtcDestroyProgram(&prog);
    return SSA_OK;
}

// the code object for src: from the disk cache (keyed by source, target,
// options and compiler) or freshly compiled and cached
int compile_source(const std::string &src, const std::string &arch, std::vector<char> &code,
                   std::string *path_out = nullptr)
{
    const std::string cc = offline_compiler();
    uint64_t h = fnv1a(arch + "\n" + src);
    for (const char *opt : kJitOptions)
        h = fnv1a(opt, h);
    h = fnv1a(cc.empty() ? std::string("hiprtc") : "clang:" + cc, h);
    char name[64];
    std::snprintf(name, sizeof name, "%016llx.co", (unsigned long long)h);
    const std::string dir = cache_dir();
    const std::string path = dir + "/" + name;
    if (path_out)
        *path_out = path;
    if (read_file(path, code) && !code.empty())
        return SSA_OK;
    const int rc = cc.empty() ? compile_hiprtc(src, arch, code) : compile_offline(cc, src, arch, code);
    if (rc != SSA_OK)
        return rc;
    // best-effort disk cache (write to a temporary name, then rename)
    ::mkdir(dir.c_str(), 0755);
    std::string tmp = path + ".tmp" + std::to_string((long long)getpid());
    {
        std::ofstream out(tmp, std::ios::binary);
        if (out)
            out.write(code.data(), (std::streamsize)code.size());
    }
    std::rename(tmp.c_str(), path.c_str());
    return SSA_OK;
}

struct Loaded {
    hipModule_t mod = nullptr;
    hipFunction_t kernel = nullptr;
    hipFunction_t kernel_pc = nullptr;   // 512-thread workgroups: event-loop waves paired with draw producers
    hipFunction_t fill = nullptr;
    hipFunction_t rg_hist = nullptr, rg_scan = nullptr, rg_scatter = nullptr;
    int vgprs = -1, vgprs_pc = -1;
    // dynamic LDS added to each ssa_kernel_pc workgroup (unused by the kernel) so
    // that it holds more than half of a CU's LDS: one workgroup, i.e. one
    // event-loop wave per SIMD, per CU, whatever the dispatcher would pack
    unsigned pc_lds_pad = 0;
};

std::mutex g_jit_mu;
std::unordered_map<std::string, Loaded> g_loaded;  // key: device + source hash

// load_if_missing = false: only a kernel an earlier run loaded on this
// device (no compilation, no module load: they allocate)
int get_kernel(const std::string &src, Loaded &out, bool load_if_missing = true)
{
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    const std::string key = std::to_string(dev) + ":" + std::to_string(fnv1a(src)) + ":" +
                            std::to_string(src.size());
    std::lock_guard<std::mutex> lk(g_jit_mu);
    auto it = g_loaded.find(key);
    if (it != g_loaded.end()) {
        out = it->second;
        return SSA_OK;
    }
    if (!load_if_missing)
        return fail(SSA_E_INVALID, "ssa_ensemble_run_noalloc: the kernel for these networks and this precision is "
                                   "not loaded on this device; run ssa_ensemble_run (or ssa_autotune) with them "
                                   "once first");
    std::vector<char> code;
    int rc = compile_source(src, "gfx950", code);
    if (rc != SSA_OK)
        return rc;
    Loaded ld;
    HIP_TRY(hipModuleLoadData(&ld.mod, code.data()));
    HIP_TRY(hipModuleGetFunction(&ld.kernel, ld.mod, "ssa_kernel"));
    HIP_TRY(hipModuleGetFunction(&ld.kernel_pc, ld.mod, "ssa_kernel_pc"));
    HIP_TRY(hipModuleGetFunction(&ld.fill, ld.mod, "ssa_fill_u32"));
    HIP_TRY(hipModuleGetFunction(&ld.rg_hist, ld.mod, "ssa_regroup_hist"));
    HIP_TRY(hipModuleGetFunction(&ld.rg_scan, ld.mod, "ssa_regroup_scan"));
    HIP_TRY(hipModuleGetFunction(&ld.rg_scatter, ld.mod, "ssa_regroup_scatter"));
    int regs = -1;
    if (hipFuncGetAttribute(&regs, HIP_FUNC_ATTRIBUTE_NUM_REGS, ld.kernel) == hipSuccess)
        ld.vgprs = regs;
    regs = -1;
    if (hipFuncGetAttribute(&regs, HIP_FUNC_ATTRIBUTE_NUM_REGS, ld.kernel_pc) == hipSuccess)
        ld.vgprs_pc = regs;
    int lds_cu = 0, lds_block = 0, lds_static = 0;
    if (hipDeviceGetAttribute(&lds_cu, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, dev) == hipSuccess &&
        hipDeviceGetAttribute(&lds_block, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess &&
        hipFuncGetAttribute(&lds_static, HIP_FUNC_ATTRIBUTE_SHARED_SIZE_BYTES, ld.kernel_pc) == hipSuccess) {
        const int want = lds_cu / 2 + 1024;
        if (want > lds_static && want <= lds_block)
            ld.pc_lds_pad = (unsigned)(want - lds_static);
    }
    g_loaded[key] = ld;
    out = ld;
    return SSA_OK;
}

// ------------------------------------------------------------------ tuning cache
// Launch shapes chosen by ssa_autotune, keyed by the kernel source and the
// workload's shape, kept in memory and appended to <cache dir>/tune.txt.
struct Tuned {
    int block = 0, grid = 0, chunks = 0, window = 0, place = 0;
    double ms = 0.0;
};

std::mutex g_tune_mu;
std::unordered_map<std::string, Tuned> g_tuned;
bool g_tune_loaded = false;

std::string tune_key(const ssa_run_desc *d, const std::string &src)
{
    std::ostringstream k;
    k << std::hex << fnv1a(src) << std::dec << ":" << d->n_snap << ":" << d->t_end << ":" << d->max_events;
    for (int i = 0; i < d->n_items; ++i)
        k << ":" << d->items[i].n_traj;
    return k.str();
}

void tune_load_locked()
{
    if (g_tune_loaded)
        return;
    g_tune_loaded = true;
    std::ifstream in(cache_dir() + "/tune.txt");
    std::string line;
    while (std::getline(in, line)) {
        std::istringstream ls(line);
        std::string key;
        Tuned t;
        if (ls >> key >> t.block >> t.grid >> t.chunks >> t.window >> t.ms >> t.place)
            g_tuned[key] = t;
    }
}

bool tune_lookup(const std::string &key, Tuned &t)
{
    std::lock_guard<std::mutex> lk(g_tune_mu);
    tune_load_locked();
    auto it = g_tuned.find(key);
    if (it == g_tuned.end())
        return false;
    t = it->second;
    return true;
}

void tune_store(const std::string &key, const Tuned &t)
{
    std::lock_guard<std::mutex> lk(g_tune_mu);
    tune_load_locked();
    g_tuned[key] = t;
    ::mkdir(cache_dir().c_str(), 0755);
    std::ofstream out(cache_dir() + "/tune.txt", std::ios::app);
    if (out)
        out << key << " " << t.block << " " << t.grid << " " << t.chunks << " " << t.window << " " << t.ms << " "
            << t.place << "\n";
}

// ------------------------------------------------------------------ launch arguments
// Must match LaunchArgs / ItemArgs in ssa_device.hip (same field order and types).
struct ItemArgsH {
    const void *rates;
    const void *hill;
    const int32_t *x0;
    int32_t *snap;
    uint64_t *n_events;
    double *t_last;
    unsigned char *status;
    int32_t *cx;
    double *ct;
    uint64_t *cn;
    int32_t *ck;
    float *cm;
    uint32_t *counter;
    const uint32_t *order;
    uint32_t *work;
    double *rec_t;
    unsigned char *rec_j;
    uint32_t *rec_n;
    uint32_t E;
    uint32_t traj_per_set;
    uint32_t id_base;
    uint32_t rec_cap;
};

constexpr int kMaxItems = 8;

struct LaunchArgsHead {
    const double *snap_t64;
    const float *snap_t32;
    double t_end64;
    float t_end32;
    int32_t K;
    int32_t k_lo, k_hi;
    int32_t first, last;
    uint32_t seed_lo, seed_hi;
    uint32_t place, place_pad;
    uint64_t max_events;
};

template <int NI>
struct LaunchArgsH {
    LaunchArgsHead h;
    ItemArgsH item[NI];
};

// ------------------------------------------------------------------ validation
int validate_mode(const ssa_run_desc *d)
{
    if (d->format < SSA_FMT_FP64 || d->format > SSA_FMT_BF16)
        return fail(SSA_E_INVALID, "format must be one of SSA_FMT_*");
    if (d->accum != SSA_ACC_MIXED && d->accum != SSA_ACC_UNIFORM)
        return fail(SSA_E_INVALID, "accum must be SSA_ACC_MIXED or SSA_ACC_UNIFORM");
    if (d->rounding != SSA_RND_RTN && d->rounding != SSA_RND_SR && d->rounding != SSA_RND_SR_ACC)
        return fail(SSA_E_INVALID, "rounding must be SSA_RND_RTN, SSA_RND_SR or SSA_RND_SR_ACC");
    if (d->norm != SSA_NORM_NONE && d->norm != SSA_NORM_RUNNING_MAX)
        return fail(SSA_E_INVALID, "norm must be SSA_NORM_NONE or SSA_NORM_RUNNING_MAX");
    if (d->format <= SSA_FMT_FP32 &&
        (d->accum != SSA_ACC_MIXED || d->rounding != SSA_RND_RTN || d->norm != SSA_NORM_NONE))
        return fail(SSA_E_INVALID, "FP64/FP32 take accum=MIXED, rounding=RTN, norm=NONE");
    if (d->rounding == SSA_RND_SR_ACC && d->accum != SSA_ACC_UNIFORM)
        return fail(SSA_E_UNSUPPORTED, "SR at accumulation points is defined for uniform 16-bit mode only "
                                       "(mixed mode accumulates in binary32)");
    if (d->norm == SSA_NORM_RUNNING_MAX && d->accum != SSA_ACC_UNIFORM)
        return fail(SSA_E_UNSUPPORTED, "propensity normalisation is defined for uniform 16-bit mode only");
    return SSA_OK;
}

int validate_desc(const ssa_run_desc *d)
{
    if (!d)
        return fail(SSA_E_INVALID, "desc is NULL");
    if (!d->items || d->n_items < 1 || d->n_items > kMaxItems)
        return fail(SSA_E_INVALID, "n_items must be in [1, 8] with a non-NULL items array");
    if (!(d->t_end > 0.0) || !std::isfinite(d->t_end))
        return fail(SSA_E_INVALID, "t_end must be finite and > 0");
    if (d->n_snap < 0 || d->n_snap > kMaxSnap)
        return fail(SSA_E_INVALID, "n_snap must be in [0, 65536]");
    if (d->n_snap > 0 && !d->snap_t)
        return fail(SSA_E_INVALID, "snap_t is NULL");
    for (int k = 0; k < d->n_snap; ++k) {
        double tk = d->snap_t[k];
        if (!(tk >= 0.0) || !(tk <= d->t_end))
            return fail(SSA_E_INVALID, "snapshot times must lie in [0, t_end]");
        if (k > 0 && !(tk >= d->snap_t[k - 1]))
            return fail(SSA_E_INVALID, "snapshot times must be ascending");
    }
    int rc = validate_mode(d);
    if (rc != SSA_OK)
        return rc;
    // A binary32 or 16-bit clock stops advancing once the waiting time falls
    // below half its spacing at t (round to nearest; Sec. 4 reports the stall
    // for uniform round-to-nearest runs): such a trajectory fires events
    // forever, so these clocks need a finite cap.
    if (d->format != SSA_FMT_FP64 && d->max_events == 0)
        return fail(SSA_E_INVALID, "max_events must be > 0 unless format is FP64: a binary32 or 16-bit clock "
                                   "can stop advancing, and the trajectory would then never end");
    if (d->n_chunks < 0 || d->n_chunks > 4096)
        return fail(SSA_E_INVALID, "n_chunks must be in [0, 4096]");
    if (d->block_size != 0 && d->block_size != 512 &&
        (d->block_size < 64 || d->block_size > 256 || d->block_size % 64 != 0))
        return fail(SSA_E_INVALID, "block_size must be 0, a multiple of 64 in [64, 256], or 512");
    if (d->grid_size < 0)
        return fail(SSA_E_INVALID, "grid_size must be >= 0");
    if (d->reorder < -1 || d->reorder > 1)
        return fail(SSA_E_INVALID, "reorder must be -1, 0 or 1");
    if (d->first_window < 0)
        return fail(SSA_E_INVALID, "first_window must be >= 0");
    if (d->placement != 0 && (!(d->placement & SSA_PLACE_EXPLICIT) ||
                              (d->placement & ~(SSA_PLACE_EXPLICIT | SSA_PLACE_NEIGHBOUR_PRODUCER |
                                                SSA_PLACE_WAVE_MAJOR | SSA_PLACE_SOLO_WAVE0 |
                                                SSA_PLACE_FEED_WAVE0 | SSA_PLACE_PRODUCER_FIRST |
                                                SSA_PLACE_DEDICATED_FEED0 | SSA_PLACE_TWO_FEED0)) != 0))
        return fail(SSA_E_INVALID, "placement must be 0 or SSA_PLACE_EXPLICIT with SSA_PLACE_* flags");
    if ((d->placement & SSA_PLACE_SOLO_WAVE0) && d->n_items > 1)
        return fail(SSA_E_INVALID, "SSA_PLACE_SOLO_WAVE0 needs a one-item launch");
    if ((d->placement & SSA_PLACE_TWO_FEED0) && (d->n_items > 1 || !(d->placement & SSA_PLACE_DEDICATED_FEED0)))
        return fail(SSA_E_INVALID, "SSA_PLACE_TWO_FEED0 needs a one-item launch and SSA_PLACE_DEDICATED_FEED0");
    if (d->n_chunks > 1 && d->first_window > 0 && d->first_window > d->n_snap - (d->n_chunks - 1))
        return fail(SSA_E_INVALID, "first_window leaves no snapshot row for a later chunk");
    uint64_t total = 0;
    for (int i = 0; i < d->n_items; ++i) {
        const ssa_item &it = d->items[i];
        if (!it.model)
            return fail(SSA_E_INVALID, "item model is NULL");
        if (!it.x0)
            return fail(SSA_E_INVALID, "item x0 is NULL");
        if (it.n_traj < 0 || it.n_traj >= (int64_t)1 << 31)
            return fail(SSA_E_INVALID, "n_traj must be in [0, 2^31)");
        for (int s = 0; s < it.model->m.N; ++s)
            if (it.x0[s] < 0)
                return fail(SSA_E_INVALID, "initial counts must be >= 0");
        if (it.set_rates) {
            if (it.n_sets < 1 || it.traj_per_set < 1 || it.traj_per_set >= ((int64_t)1 << 31) ||
                it.n_traj > it.n_sets * it.traj_per_set)
                return fail(SSA_E_INVALID, "set_rates needs n_sets >= 1, traj_per_set >= 1 and "
                                           "n_traj <= n_sets * traj_per_set");
            const int M = it.model->m.M;
            for (int64_t r = 0; r < it.n_sets * M; ++r)
                if (!(it.set_rates[r] >= 0.0) || !std::isfinite(it.set_rates[r]))
                    return fail(SSA_E_INVALID, "set_rates must be finite and >= 0");
        }
        if (it.record_mask) {
            if (it.record_cap < 0 || it.record_cap > (1 << 20) ||
                (uint64_t)it.record_cap * (uint64_t)it.n_traj > ((uint64_t)1 << 31))
                return fail(SSA_E_INVALID, "record_cap must be in [0, 2^20] with record_cap * n_traj <= 2^31");
            if (it.model->m.M < 64 && (it.record_mask >> it.model->m.M) != 0)
                return fail(SSA_E_INVALID, "record_mask names a reaction the model does not have");
        }
        total += (uint64_t)it.n_traj;
    }
    if ((uint64_t)d->traj_id_base + total > 0xFFFFFFFFull)
        return fail(SSA_E_INVALID, "traj_id_base + total trajectories must be < 2^32");
    return SSA_OK;
}

// Kernel source and flags for a descriptor (no device needed).
int build_source(const ssa_run_desc *d, std::string &src)
{
    std::vector<const Model *> models;
    std::vector<bool> per_lane;
    std::vector<uint64_t> rec;
    for (int i = 0; i < d->n_items; ++i) {
        models.push_back(&d->items[i].model->m);
        per_lane.push_back(d->items[i].set_rates != nullptr && d->items[i].n_sets > 1);
        rec.push_back(d->items[i].record_cap > 0 ? d->items[i].record_mask : 0ull);
    }
    ModeSpec ms{d->format, d->accum, d->rounding, d->norm};
    src = gen_source(models, ms, per_lane, rec);
    return SSA_OK;
}

}  // namespace

// ------------------------------------------------------------------ run object
struct ItemBuf {
    int N = 0, M = 0;
    int64_t E = 0;
    int32_t *snap = nullptr;
    uint64_t *nev = nullptr;
    double *tlast = nullptr;
    uint8_t *status = nullptr;
    int32_t *cx = nullptr;
    double *ct = nullptr;
    uint64_t *cn = nullptr;
    int32_t *ck = nullptr;
    float *cm = nullptr;
    void *rates = nullptr;
    void *hill = nullptr;
    int32_t *x0 = nullptr;
    uint32_t *order = nullptr;   // claim order for the next chunk (chunked runs)
    uint32_t *work = nullptr;    // events per trajectory in the last chunk
    uint32_t *hist = nullptr;    // 256 work classes
    double *rec_t = nullptr;     // event record [E][rec_cap]
    uint8_t *rec_j = nullptr;
    uint32_t *rec_n = nullptr;   // [E]; also the carry of the record count between chunks
    uint32_t rec_cap = 0;
    uint32_t traj_per_set = 0;
    uint32_t id_base = 0;
};

struct ssa_run {
    int device = 0;
    hipStream_t stream = nullptr;
    int K = 0;
    int n_launch = 0;
    int first_window = 0;  // snapshot rows of the first chunk (0: even windows)
    int block = 0, grid = 0, vgprs = -1;
    int place = 0;        // PLACE_* bits of the launches
    bool graph = false;
    std::vector<ItemBuf> items;
    std::vector<std::pair<void *, size_t>> owned;  // library-owned device buffers (returned to the cache)
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    bool ev1_recorded = false;    // ev1 marks the end of all queued work
    bool queued = false;          // some work was queued on the streams
    std::vector<hipEvent_t> kev;  // start/stop per launch (non-graph runs)
    hipGraph_t g = nullptr;
    hipGraphExec_t gx = nullptr;
    hipStream_t cap = nullptr;
    double *t64 = nullptr;
    float *t32 = nullptr;
    uint32_t *counters = nullptr;
    // runs of ssa_ensemble_run_noalloc: device buffers come from the scratch
    // array (bump allocation), no events, no graph, no kernel compilation
    bool noalloc = false;
    char *scratch = nullptr;
    size_t scratch_used = 0, scratch_cap = 0;
};

namespace {

// ------------------------------------------------------------------ buffer cache
// The library's own device buffers (tables, carry state, claim order, counters
// and outputs the caller does not provide) go back to a per-device free list
// when a run is destroyed (after its work has finished) and are handed out
// again to later runs, so repeated runs of one workload allocate nothing. At
// most kCacheCap bytes are kept per device; the rest is freed.
constexpr int kMaxDevices = 64;
constexpr size_t kCacheCap = (size_t)1 << 30;

struct BufCache {
    std::mutex mu;
    std::multimap<size_t, void *> free;
    size_t bytes = 0;
};
BufCache g_cache[kMaxDevices];

size_t cache_size_class(size_t bytes)
{
    return (bytes + 4095) & ~(size_t)4095;
}

// A cached block of at least `bytes` (and at most twice that), or NULL; its
// size goes to *size.
void *cache_take(int dev, size_t bytes, size_t *size)
{
    if (dev < 0 || dev >= kMaxDevices)
        return nullptr;
    BufCache &c = g_cache[dev];
    std::lock_guard<std::mutex> lk(c.mu);
    auto it = c.free.lower_bound(bytes);
    if (it == c.free.end() || it->first > 2 * bytes)
        return nullptr;
    void *p = it->second;
    *size = it->first;
    c.bytes -= it->first;
    c.free.erase(it);
    return p;
}

void cache_give(int dev, void *p, size_t bytes)
{
    if (dev >= 0 && dev < kMaxDevices) {
        BufCache &c = g_cache[dev];
        std::lock_guard<std::mutex> lk(c.mu);
        if (c.bytes + bytes <= kCacheCap) {
            c.free.emplace(bytes, p);
            c.bytes += bytes;
            return;
        }
    }
    (void)hipFree(p);
}

template <class T>
int dalloc(ssa_run *r, T **p, size_t n)
{
    *p = nullptr;
    if (n == 0)
        return SSA_OK;
    if (r->noalloc) {
        const size_t off = (r->scratch_used + 255) & ~(size_t)255;
        const size_t bytes = n * sizeof(T);
        if (bytes > r->scratch_cap || off > r->scratch_cap - bytes)
            return fail(SSA_E_INVALID, "the run needs more than the " + std::to_string(r->scratch_cap >> 20) +
                                           " MiB scratch array of ssa_ensemble_run_noalloc (fewer snapshot "
                                           "windows or trajectories, or use ssa_ensemble_run)");
        r->scratch_used = off + bytes;
        *p = (T *)(r->scratch + off);
        return SSA_OK;
    }
    const size_t want = cache_size_class(n * sizeof(T));
    size_t got = want;
    void *q = cache_take(r->device, want, &got);
    if (!q) {
        hipError_t e = hipMalloc(&q, want);
        if (e != hipSuccess)
            return fail(e == hipErrorOutOfMemory ? SSA_E_NOMEM : SSA_E_DEVICE,
                        std::string("hipMalloc: ") + hipGetErrorString(e));
    }
    r->owned.emplace_back(q, got);
    *p = (T *)q;
    return SSA_OK;
}

// Snapshot rows [k_lo, k_hi) of chunk c: with first_window w > 0 the first
// chunk holds rows [0, w) and the others split [w, K) evenly; else all split
// [0, K) evenly.
void chunk_rows(int K, int n_chunks, int w, int c, int &k_lo, int &k_hi)
{
    if (w > 0 && n_chunks > 1) {
        if (c == 0) {
            k_lo = 0;
            k_hi = w;
            return;
        }
        const int64_t rest = K - w, m = n_chunks - 1;
        k_lo = w + (int)((int64_t)(c - 1) * rest / m);
        k_hi = c == n_chunks - 1 ? K : w + (int)((int64_t)c * rest / m);
        return;
    }
    k_lo = (int)((int64_t)c * K / n_chunks);
    k_hi = c == n_chunks - 1 ? K : (int)((int64_t)(c + 1) * K / n_chunks);
}

template <int NI>
int launch_all(ssa_run *r, const ssa_run_desc *d, const Loaded &ld, int n_chunks)
{
    LaunchArgsH<NI> A;
    std::memset(&A, 0, sizeof A);
    A.h.snap_t64 = r->t64;
    A.h.snap_t32 = r->t32;
    A.h.t_end64 = d->t_end;
    A.h.t_end32 = (float)d->t_end;
    A.h.K = r->K;
    A.h.seed_lo = (uint32_t)d->seed;
    A.h.seed_hi = (uint32_t)(d->seed >> 32);
    A.h.max_events = d->max_events;
    A.h.place = (uint32_t)r->place;
    const int nI = d->n_items;
    hipStream_t s = r->graph ? r->cap : r->stream;
    // one zeroed counter per (chunk, item)
    {
        uint32_t n = (uint32_t)(n_chunks * nI);
        uint32_t v = 0;
        void *args[] = {&r->counters, &n, &v};
        HIP_TRY(hipModuleLaunchKernel(ld.fill, (n + 255) / 256, 1, 1, 256, 1, 1, 0, s, args, nullptr));
    }
    for (int c = 0; c < n_chunks; ++c) {
        int k_lo, k_hi;
        chunk_rows(r->K, n_chunks, r->first_window, c, k_lo, k_hi);
        A.h.k_lo = k_lo;
        A.h.k_hi = k_hi;
        A.h.first = c == 0;
        A.h.last = c == n_chunks - 1;
        for (int i = 0; i < nI; ++i) {
            const ItemBuf &b = r->items[i];
            ItemArgsH &ia = A.item[i];
            ia.rates = b.rates;
            ia.hill = b.hill;
            ia.x0 = b.x0;
            ia.snap = b.snap ? b.snap + (size_t)k_lo * b.N * b.E : nullptr;
            ia.n_events = b.nev;
            ia.t_last = b.tlast;
            ia.status = b.status;
            ia.cx = b.cx;
            ia.ct = b.ct;
            ia.cn = b.cn;
            ia.ck = b.ck;
            ia.cm = b.cm;
            ia.counter = r->counters + (size_t)c * nI + i;
            ia.order = (c > 0 && b.order) ? b.order : nullptr;
            ia.work = b.work;
            ia.rec_t = b.rec_t;
            ia.rec_j = b.rec_j;
            ia.rec_n = b.rec_n;
            ia.rec_cap = b.rec_cap;
            ia.E = (uint32_t)b.E;
            ia.traj_per_set = b.traj_per_set;
            ia.id_base = b.id_base;
        }
        void *args[] = {&A};
        if (!r->kev.empty())
            HIP_TRY(hipEventRecord(r->kev[2 * c], s));
        HIP_TRY(hipModuleLaunchKernel(r->block == 512 ? ld.kernel_pc : ld.kernel, r->grid, 1, 1, r->block, 1, 1,
                                      r->block == 512 ? ld.pc_lds_pad : 0u, s, args, nullptr));
        if (!r->kev.empty())
            HIP_TRY(hipEventRecord(r->kev[2 * c + 1], s));
        // claim order for the next chunk: heaviest trajectories of this chunk first
        if (c + 1 < n_chunks) {
            for (int i = 0; i < nI; ++i) {
                ItemBuf &b = r->items[i];
                if (!b.order || b.E == 0)
                    continue;
                uint32_t nb = 256, zero = 0, E = (uint32_t)b.E;
                uint32_t blocks = (uint32_t)std::min<int64_t>((b.E + 255) / 256, 1024);
                void *fa[] = {&b.hist, &nb, &zero};
                HIP_TRY(hipModuleLaunchKernel(ld.fill, 1, 1, 1, 256, 1, 1, 0, s, fa, nullptr));
                void *ha[] = {&b.work, &E, &b.hist};
                HIP_TRY(hipModuleLaunchKernel(ld.rg_hist, blocks, 1, 1, 256, 1, 1, 0, s, ha, nullptr));
                void *sa[] = {&b.hist};
                HIP_TRY(hipModuleLaunchKernel(ld.rg_scan, 1, 1, 1, 256, 1, 1, 0, s, sa, nullptr));
                void *xa[] = {&b.work, &E, &b.hist, &b.order};
                HIP_TRY(hipModuleLaunchKernel(ld.rg_scatter, blocks, 1, 1, 256, 1, 1, 0, s, xa, nullptr));
            }
        }
    }
    return SSA_OK;
}

int dispatch_launch(ssa_run *r, const ssa_run_desc *d, const Loaded &ld, int n_chunks)
{
    switch (d->n_items) {
    case 1: return launch_all<1>(r, d, ld, n_chunks);
    case 2: return launch_all<2>(r, d, ld, n_chunks);
    case 3: return launch_all<3>(r, d, ld, n_chunks);
    case 4: return launch_all<4>(r, d, ld, n_chunks);
    case 5: return launch_all<5>(r, d, ld, n_chunks);
    case 6: return launch_all<6>(r, d, ld, n_chunks);
    case 7: return launch_all<7>(r, d, ld, n_chunks);
    default: return launch_all<8>(r, d, ld, n_chunks);
    }
}

int run_impl(const ssa_run_desc *d, ssa_run *r)
{
    HIP_TRY(hipGetDevice(&r->device));
    r->stream = (hipStream_t)d->hip_stream;
    r->K = d->n_snap;
    std::string src;
    build_source(d, src);
    Loaded ld;
    int rc = get_kernel(src, ld, !r->noalloc);
    if (rc != SSA_OK)
        return rc;
    r->vgprs = ld.vgprs;

    // launch shape chosen by ssa_autotune for this kernel and workload, if any
    Tuned tuned;
    const bool have_tuned = (d->block_size == 0 || d->grid_size == 0 || d->n_chunks == 0 || d->placement == 0) &&
                            tune_lookup(tune_key(d, src), tuned);
    const bool wide = d->format == SSA_FMT_FP64;
    int n_chunks = d->n_chunks == 0 ? (have_tuned ? tuned.chunks : 1) : d->n_chunks;
    int window = d->n_chunks == 0 ? (have_tuned ? tuned.window : 0) : d->first_window;
    if (n_chunks < 1)
        n_chunks = 1;
    if (n_chunks > std::max(r->K, 1))
        n_chunks = std::max(r->K, 1);
    // the first window must leave at least one row for every later chunk
    if (n_chunks < 2 || window < 0 || window > r->K - (n_chunks - 1))
        window = 0;
    r->first_window = window;

    // All small tables (snapshot times in both clock types, and per item the
    // rate table, Hill constants and x0) go to one device block in one copy.
    std::vector<char> blob;
    auto put = [&blob](const void *src, size_t n) {
        size_t off = (blob.size() + 255) & ~(size_t)255;
        blob.resize(off + n);
        if (n)
            std::memcpy(blob.data() + off, src, n);
        return off;
    };
    std::vector<float> t32(r->K);
    for (int k = 0; k < r->K; ++k)
        t32[k] = (float)d->snap_t[k];
    const size_t off_t64 = put(d->snap_t, sizeof(double) * r->K);
    const size_t off_t32 = put(t32.data(), sizeof(float) * r->K);
    struct ItemOffsets {
        size_t rates, hill, x0;
    };
    std::vector<ItemOffsets> item_off;
    if ((rc = dalloc(r, &r->counters, (size_t)n_chunks * d->n_items)))
        return rc;

    uint64_t id_base = d->traj_id_base;
    int64_t total = 0;
    for (int i = 0; i < d->n_items; ++i) {
        const ssa_item &it = d->items[i];
        const Model &md = it.model->m;
        ItemBuf b;
        b.N = md.N;
        b.M = md.M;
        b.E = it.n_traj;
        b.id_base = (uint32_t)id_base;
        id_base += (uint64_t)it.n_traj;
        total += it.n_traj;
        const bool per_lane = it.set_rates != nullptr && it.n_sets > 1;
        b.traj_per_set = per_lane ? (uint32_t)it.traj_per_set : 0u;
        // rate table in the propensity type
        const int64_t n_sets = it.set_rates ? (per_lane ? it.n_sets : 1) : 1;
        const size_t tsz = wide ? sizeof(double) : sizeof(float);
        std::vector<char> rtab((size_t)n_sets * md.M * tsz);
        char *rt = rtab.data();
        for (int64_t sidx = 0; sidx < n_sets; ++sidx)
            for (int j = 0; j < md.M; ++j) {
                double k = it.set_rates ? it.set_rates[sidx * md.M + j] : md.law[j].k;
                double v = to_prop_type(d->format, primary_constant(md, j, k));
                if (wide)
                    ((double *)rt)[sidx * md.M + j] = v;
                else
                    ((float *)rt)[sidx * md.M + j] = (float)v;
            }
        std::vector<char> htab((size_t)2 * md.M * tsz);
        char *ht = htab.data();
        for (int j = 0; j < md.M; ++j) {
            bool hill = md.law[j].kind != SSA_LAW_MASS_ACTION;
            double bv = to_prop_type(d->format, hill ? md.law[j].basal : 0.0);
            double kv = to_prop_type(d->format, hill ? md.law[j].K : 1.0);
            if (wide) {
                ((double *)ht)[2 * j] = bv;
                ((double *)ht)[2 * j + 1] = kv;
            } else {
                ((float *)ht)[2 * j] = (float)bv;
                ((float *)ht)[2 * j + 1] = (float)kv;
            }
        }
        ItemOffsets io;
        io.rates = put(rtab.data(), rtab.size());
        io.hill = put(htab.data(), htab.size());
        io.x0 = put(it.x0, sizeof(int32_t) * md.N);
        item_off.push_back(io);
        // outputs
        const size_t E = (size_t)it.n_traj;
        b.snap = it.d_snap;
        if (!b.snap && (rc = dalloc(r, &b.snap, (size_t)r->K * md.N * E)))
            return rc;
        b.nev = it.d_n_events;
        if (!b.nev && (rc = dalloc(r, &b.nev, E)))
            return rc;
        b.tlast = it.d_t_last;
        if (!b.tlast && (rc = dalloc(r, &b.tlast, E)))
            return rc;
        b.status = it.d_status;
        if (!b.status && (rc = dalloc(r, &b.status, E)))
            return rc;
        if (it.record_mask && it.record_cap > 0) {
            b.rec_cap = (uint32_t)it.record_cap;
            b.rec_t = it.d_rec_t;
            b.rec_j = it.d_rec_j;
            b.rec_n = it.d_rec_n;
            const size_t cells = E * (size_t)it.record_cap;
            if ((!b.rec_t && (rc = dalloc(r, &b.rec_t, cells))) || (!b.rec_j && (rc = dalloc(r, &b.rec_j, cells))) ||
                (!b.rec_n && (rc = dalloc(r, &b.rec_n, E))))
                return rc;
        }
        if (n_chunks > 1) {
            if ((rc = dalloc(r, &b.cx, (size_t)md.N * E)) || (rc = dalloc(r, &b.ct, E)) ||
                (rc = dalloc(r, &b.cn, E)) || (rc = dalloc(r, &b.ck, E)) || (rc = dalloc(r, &b.cm, E)))
                return rc;
            if (d->reorder >= 0 && E > 0 &&
                ((rc = dalloc(r, &b.order, E)) || (rc = dalloc(r, &b.work, E)) || (rc = dalloc(r, &b.hist, 256))))
                return rc;
        }
        r->items.push_back(b);
    }
    {
        char *base = nullptr;
        if ((rc = dalloc(r, &base, blob.size())))
            return rc;
        if (!blob.empty()) {
            if (r->noalloc)   // ordered on the run's stream after earlier work there
                HIP_TRY(hipMemcpyAsync(base, blob.data(), blob.size(), hipMemcpyHostToDevice, r->stream));
            else
                HIP_TRY(hipMemcpy(base, blob.data(), blob.size(), hipMemcpyHostToDevice));
        }
        r->t64 = (double *)(base + off_t64);
        r->t32 = (float *)(base + off_t32);
        for (int i = 0; i < d->n_items; ++i) {
            r->items[i].rates = base + item_off[i].rates;
            r->items[i].hill = base + item_off[i].hill;
            r->items[i].x0 = (int32_t *)(base + item_off[i].x0);
        }
    }

    // launch shape: enough waves to cover the ensemble, at most what stays resident
    int cus = 0;
    HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, r->device));
    r->block = d->block_size ? d->block_size : (have_tuned ? tuned.block : 256);
    if (r->block == 512)
        r->vgprs = ld.vgprs_pc;
    int per_cu = 0;
    HIP_TRY(hipModuleOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, r->block == 512 ? ld.kernel_pc : ld.kernel,
                                                              r->block, r->block == 512 ? ld.pc_lds_pad : 0u));
    // a workgroup that cannot be resident at all (registers or LDS beyond a
    // CU's) would fail at dispatch: refuse it here
    if (per_cu < 1)
        return fail(SSA_E_UNSUPPORTED, "the kernel for these networks needs more registers or LDS than one " +
                                           std::to_string(r->block) + "-thread workgroup per CU allows; use a smaller "
                                           "block_size (or 0)");
    // lanes running the event loop per workgroup (half of a 512-thread one)
    const int loop_lanes = r->block == 512 ? 256 : r->block;
    int64_t need = (total + loop_lanes - 1) / loop_lanes;
    int64_t resident = (int64_t)per_cu * cus;
    int64_t grid = d->grid_size ? d->grid_size
                                : (have_tuned && tuned.block == r->block ? tuned.grid
                                                                          : std::max<int64_t>(1, std::min(need, resident)));
    r->grid = (int)grid;
    // placement bits: explicit (placement = SSA_PLACE_EXPLICIT | flags), else
    // the autotuned choice where the tuned block size is the one launched
    if (d->placement != 0)
        r->place = d->placement & (SSA_PLACE_NEIGHBOUR_PRODUCER | SSA_PLACE_WAVE_MAJOR | SSA_PLACE_SOLO_WAVE0 |
                                   SSA_PLACE_FEED_WAVE0 | SSA_PLACE_PRODUCER_FIRST | SSA_PLACE_DEDICATED_FEED0 |
                                   SSA_PLACE_TWO_FEED0);
    else if (have_tuned && tuned.block == r->block)
        r->place = tuned.place;
    r->place = (r->place & SSA_PLACE_NEIGHBOUR_PRODUCER ? 1 : 0) | (r->place & SSA_PLACE_WAVE_MAJOR ? 2 : 0) |
               (r->place & SSA_PLACE_SOLO_WAVE0 ? 4 : 0) | (r->place & SSA_PLACE_FEED_WAVE0 ? 8 : 0) |
               (r->place & SSA_PLACE_PRODUCER_FIRST ? 16 : 0) | (r->place & SSA_PLACE_DEDICATED_FEED0 ? 32 : 0) |
               (r->place & SSA_PLACE_TWO_FEED0 ? 64 : 0);

    r->n_launch = n_chunks;
    if (r->noalloc) {   // direct launches, no events
        r->graph = false;
        r->queued = true;
        return dispatch_launch(r, d, ld, n_chunks);
    }
    HIP_TRY(hipEventCreate(&r->ev0));
    HIP_TRY(hipEventCreate(&r->ev1));
    // A captured graph pays off only over long chunk sequences: capture and
    // instantiation cost more than a few direct launches.
    r->graph = n_chunks > kGraphMinChunks;
    if (!r->graph) {
        r->kev.resize(2 * n_chunks);
        for (auto &e : r->kev)
            HIP_TRY(hipEventCreate(&e));
    }
    HIP_TRY(hipEventRecord(r->ev0, r->stream));
    r->queued = true;
    if (r->graph) {
        HIP_TRY(hipStreamCreateWithFlags(&r->cap, hipStreamNonBlocking));
        HIP_TRY(hipStreamBeginCapture(r->cap, hipStreamCaptureModeThreadLocal));
        rc = dispatch_launch(r, d, ld, n_chunks);
        hipGraph_t g = nullptr;
        hipError_t ec = hipStreamEndCapture(r->cap, &g);
        if (rc != SSA_OK)
            return rc;
        if (ec != hipSuccess)
            return fail(SSA_E_DEVICE, std::string("hipStreamEndCapture: ") + hipGetErrorString(ec));
        r->g = g;
        HIP_TRY(hipGraphInstantiate(&r->gx, r->g, nullptr, nullptr, 0));
        HIP_TRY(hipGraphLaunch(r->gx, r->stream));
    } else {
        rc = dispatch_launch(r, d, ld, n_chunks);
        if (rc != SSA_OK)
            return rc;
    }
    HIP_TRY(hipEventRecord(r->ev1, r->stream));
    r->ev1_recorded = true;
    return SSA_OK;
}

void release(ssa_run *r)
{
    if (!r)
        return;
    // The buffers go back to the cache only once no queued kernel can still
    // write them: after ev1, or, where a failure came before ev1 was
    // recorded, after everything queued on the run's streams.
    if (r->ev1_recorded) {
        (void)hipEventSynchronize(r->ev1);
    } else if (r->queued) {
        if (r->cap)
            (void)hipStreamSynchronize(r->cap);
        (void)hipStreamSynchronize(r->stream);
    }
    if (r->gx)
        (void)hipGraphExecDestroy(r->gx);
    if (r->g)
        (void)hipGraphDestroy(r->g);
    if (r->cap)
        (void)hipStreamDestroy(r->cap);
    for (auto e : r->kev)
        if (e)
            (void)hipEventDestroy(e);
    if (r->ev0)
        (void)hipEventDestroy(r->ev0);
    if (r->ev1)
        (void)hipEventDestroy(r->ev1);
    for (auto &o : r->owned)
        cache_give(r->device, o.first, o.second);
    delete r;
}

// ------------------------------------------------------------------ scratch array
// Device memory of ssa_ensemble_run_noalloc: tables, work counters, carry state
// and claim order of its runs. Each device holds its own copy (from the first
// call on it until the process ends). In host code `scratch` names a host-side
// stand-in, never the device memory: the device address comes from
// hipGetSymbolAddress, once per device, and only that address is used.
constexpr size_t kScratchBytes = (size_t)64 << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

int scratch_address(int dev, char **out)
{
    if (dev < 0 || dev >= kMaxDevices)
        return fail(SSA_E_UNSUPPORTED, "device index beyond the library's limit");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(SSA_E_DEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        g_scratch_ptr[dev] = p;
    }
    *out = (char *)g_scratch_ptr[dev];
    return SSA_OK;
}

}  // namespace

// ------------------------------------------------------------------ C ABI
extern "C" {

int ssa_model_create(int32_t n_species, int32_t n_reactions, const int32_t *reactant_order,
                     const int32_t *stoich, const ssa_law *laws, ssa_model **out)
{
    if (!out)
        return fail(SSA_E_INVALID, "out is NULL");
    *out = nullptr;
    if (n_species < 1 || n_species > kMaxSpecies)
        return fail(SSA_E_INVALID, "n_species must be in [1, 32]");
    if (n_reactions < 1 || n_reactions > kMaxReactions)
        return fail(SSA_E_INVALID, "n_reactions must be in [1, 64]");
    if (!reactant_order || !stoich || !laws)
        return fail(SSA_E_INVALID, "reactant_order, stoich and laws must be non-NULL");
    const int N = n_species, M = n_reactions;
    for (int j = 0; j < M; ++j) {
        const ssa_law &L = laws[j];
        if (!(L.k >= 0.0) || !std::isfinite(L.k))
            return fail(SSA_E_INVALID, "rate constant k must be finite and >= 0 (reaction " + std::to_string(j) + ")");
        if (L.kind == SSA_LAW_MASS_ACTION) {
            int tot = 0;
            for (int s = 0; s < N; ++s) {
                int o = reactant_order[(size_t)j * N + s];
                if (o < 0)
                    return fail(SSA_E_INVALID, "reactant orders must be >= 0");
                tot += o;
            }
            if (tot > kMaxOrder)
                return fail(SSA_E_UNSUPPORTED, "total reaction order above 4");
        } else if (L.kind == SSA_LAW_HILL_REPRESS || L.kind == SSA_LAW_HILL_ACTIVATE) {
            if (L.regulator < 0 || L.regulator >= N)
                return fail(SSA_E_INVALID, "Hill regulator out of range");
            if (L.h < 1 || L.h > 8)
                return fail(SSA_E_INVALID, "Hill exponent must be in [1, 8]");
            if (!(L.K > 0.0) || !std::isfinite(L.K))
                return fail(SSA_E_INVALID, "Hill K must be finite and > 0");
            if (!(L.basal >= 0.0) || !std::isfinite(L.basal))
                return fail(SSA_E_INVALID, "Hill basal rate must be finite and >= 0");
        } else {
            return fail(SSA_E_INVALID, "unknown law kind");
        }
        for (int s = 0; s < N; ++s) {
            int v = stoich[(size_t)j * N + s];
            if (v < -1024 || v > 1024)
                return fail(SSA_E_INVALID, "stoichiometric entries must be in [-1024, 1024]");
        }
    }
    ssa_model *m = new (std::nothrow) ssa_model;
    if (!m)
        return fail(SSA_E_NOMEM, "out of host memory");
    m->m.N = N;
    m->m.M = M;
    m->m.order.assign(reactant_order, reactant_order + (size_t)M * N);
    m->m.nu.assign(stoich, stoich + (size_t)M * N);
    m->m.law.assign(laws, laws + M);
    for (int j = 0; j < M; ++j)
        if (m->m.law[j].kind != SSA_LAW_MASS_ACTION)
            for (int s = 0; s < N; ++s)
                m->m.order[(size_t)j * N + s] = 0;
    *out = m;
    return SSA_OK;
}

void ssa_model_destroy(ssa_model *model) { delete model; }

int ssa_ensemble_run(const ssa_run_desc *desc, ssa_run **out)
{
    if (!out)
        return fail(SSA_E_INVALID, "out is NULL");
    *out = nullptr;
    int rc = validate_desc(desc);
    if (rc != SSA_OK)
        return rc;
    ssa_run *r = new (std::nothrow) ssa_run;
    if (!r)
        return fail(SSA_E_NOMEM, "out of host memory");
    rc = run_impl(desc, r);
    if (rc != SSA_OK) {
        std::string keep = g_err;
        release(r);
        g_err = keep;
        return rc;
    }
    *out = r;
    return SSA_OK;
}

// The allocation-free variant of ssa_ensemble_run (declared in ssa_rp.h).
int ssa_ensemble_run_noalloc(const ssa_run_desc *desc)
{
    int rc = validate_desc(desc);
    if (rc != SSA_OK)
        return rc;
    for (int i = 0; i < desc->n_items; ++i) {
        const ssa_item &it = desc->items[i];
        const size_t E = (size_t)it.n_traj;
        const size_t cells = (size_t)desc->n_snap * it.model->m.N * E;
        if ((cells && !it.d_snap) || (E && (!it.d_n_events || !it.d_t_last || !it.d_status)))
            return fail(SSA_E_INVALID, "ssa_ensemble_run_noalloc: every item needs its device outputs "
                                       "(d_snap, d_n_events, d_t_last, d_status)");
        if (it.record_mask && it.record_cap > 0 && E && (!it.d_rec_t || !it.d_rec_j || !it.d_rec_n))
            return fail(SSA_E_INVALID, "ssa_ensemble_run_noalloc: a recording item needs d_rec_t, d_rec_j "
                                       "and d_rec_n");
    }
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    ssa_run r;
    r.noalloc = true;
    r.scratch_cap = kScratchBytes;
    if ((rc = scratch_address(dev, &r.scratch)) != SSA_OK)
        return rc;
    return run_impl(desc, &r);
}

int ssa_run_wait(ssa_run *run)
{
    if (!run)
        return fail(SSA_E_INVALID, "run is NULL");
    HIP_TRY(hipEventSynchronize(run->ev1));
    return SSA_OK;
}

int ssa_snapshots_get(const ssa_run *run, int32_t item, int32_t *dst, size_t dst_elems, int dst_is_device)
{
    if (!run || item < 0 || item >= (int)run->items.size())
        return fail(SSA_E_INVALID, "run is NULL or item out of range");
    const ItemBuf &b = run->items[item];
    size_t n = (size_t)run->K * b.N * b.E;
    if (dst_elems != n)
        return fail(SSA_E_INVALID, "dst_elems must equal n_snap * n_species * n_traj");
    if (n == 0)
        return SSA_OK;
    if (!dst)
        return fail(SSA_E_INVALID, "dst is NULL");
    HIP_TRY(hipEventSynchronize(run->ev1));
    HIP_TRY(hipMemcpy(dst, b.snap, n * sizeof(int32_t), dst_is_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost));
    return SSA_OK;
}

int ssa_run_stats_get(const ssa_run *run, int32_t item, uint64_t *n_events, double *t_last, uint8_t *status,
                      int dst_is_device)
{
    if (!run || item < 0 || item >= (int)run->items.size())
        return fail(SSA_E_INVALID, "run is NULL or item out of range");
    const ItemBuf &b = run->items[item];
    const size_t E = (size_t)b.E;
    if (E == 0)
        return SSA_OK;
    HIP_TRY(hipEventSynchronize(run->ev1));
    hipMemcpyKind kind = dst_is_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
    if (n_events)
        HIP_TRY(hipMemcpy(n_events, b.nev, E * sizeof(uint64_t), kind));
    if (t_last)
        HIP_TRY(hipMemcpy(t_last, b.tlast, E * sizeof(double), kind));
    if (status)
        HIP_TRY(hipMemcpy(status, b.status, E * sizeof(uint8_t), kind));
    return SSA_OK;
}

int ssa_records_get(const ssa_run *run, int32_t item, double *t, uint8_t *j, uint32_t *n, int dst_is_device)
{
    if (!run || item < 0 || item >= (int)run->items.size())
        return fail(SSA_E_INVALID, "run is NULL or item out of range");
    const ItemBuf &b = run->items[item];
    if (!b.rec_n)
        return fail(SSA_E_INVALID, "the item has no event record");
    const size_t E = (size_t)b.E, cells = E * b.rec_cap;
    if (E == 0)
        return SSA_OK;
    HIP_TRY(hipEventSynchronize(run->ev1));
    hipMemcpyKind kind = dst_is_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
    if (t && cells)
        HIP_TRY(hipMemcpy(t, b.rec_t, cells * sizeof(double), kind));
    if (j && cells)
        HIP_TRY(hipMemcpy(j, b.rec_j, cells * sizeof(uint8_t), kind));
    if (n)
        HIP_TRY(hipMemcpy(n, b.rec_n, E * sizeof(uint32_t), kind));
    return SSA_OK;
}

int ssa_run_info_get(const ssa_run *run, ssa_run_info *info)
{
    if (!run || !info)
        return fail(SSA_E_INVALID, "run and info must be non-NULL");
    HIP_TRY(hipEventSynchronize(run->ev1));
    float ms = 0.0f;
    HIP_TRY(hipEventElapsedTime(&ms, run->ev0, run->ev1));
    info->elapsed_ms = ms;
    double kms = 0.0;
    if (!run->graph) {
        for (int c = 0; c < run->n_launch; ++c) {
            float m = 0.0f;
            HIP_TRY(hipEventElapsedTime(&m, run->kev[2 * c], run->kev[2 * c + 1]));
            kms += m;
        }
    } else {
        kms = ms;
    }
    info->kernel_ms = kms;
    info->n_launches = run->n_launch;
    info->block_size = run->block;
    info->grid_size = run->grid;
    info->vgprs = run->vgprs;
    uint64_t tot = 0;
    for (const ItemBuf &b : run->items) {
        if (b.E == 0)
            continue;
        std::vector<uint64_t> h((size_t)b.E);
        HIP_TRY(hipMemcpy(h.data(), b.nev, h.size() * sizeof(uint64_t), hipMemcpyDeviceToHost));
        for (uint64_t v : h)
            tot += v;
    }
    info->total_events = tot;
    info->first_window = run->n_launch > 1 ? run->first_window : 0;
    info->graph = run->graph ? 1 : 0;
    info->placement = SSA_PLACE_EXPLICIT | (run->place & 1 ? SSA_PLACE_NEIGHBOUR_PRODUCER : 0) |
                      (run->place & 2 ? SSA_PLACE_WAVE_MAJOR : 0) | (run->place & 4 ? SSA_PLACE_SOLO_WAVE0 : 0) |
                      (run->place & 8 ? SSA_PLACE_FEED_WAVE0 : 0) | (run->place & 16 ? SSA_PLACE_PRODUCER_FIRST : 0) |
                      (run->place & 32 ? SSA_PLACE_DEDICATED_FEED0 : 0) | (run->place & 64 ? SSA_PLACE_TWO_FEED0 : 0);
    return SSA_OK;
}

void ssa_run_destroy(ssa_run *run) { release(run); }

const char *ssa_last_error(void) { return g_err.c_str(); }

const char *ssa_version(void) { return "ssa_rp 0.1 (gfx950)"; }

// Time candidate launch shapes on the workload itself and remember the best.
int ssa_autotune(const ssa_run_desc *desc, ssa_tune_result *res)
{
    int rc = validate_desc(desc);
    if (rc != SSA_OK)
        return rc;
    std::string src;
    build_source(desc, src);
    Loaded ld;
    if ((rc = get_kernel(src, ld)) != SSA_OK)
        return rc;
    int dev = 0, cus = 0;
    HIP_TRY(hipGetDevice(&dev));
    HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    int64_t total = 0;
    for (int i = 0; i < desc->n_items; ++i)
        total += desc->items[i].n_traj;
    struct Cand {
        int block, grid, chunks, window, place;
    };
    std::vector<Cand> cands;
    // one launch; 4 even windows; a first window of about a tenth of the rows
    // (it measures every trajectory's event rate, so the longest start first)
    // followed by one or two windows, or of about 15% or 20% of the rows
    // followed by one (a longer first look sorts later state switches in too)
    struct ChunkOpt {
        int chunks, window;
    };
    std::vector<ChunkOpt> chunk_opts = {{1, 0}};
    if (desc->n_snap >= 8)
        chunk_opts.push_back({4, 0});
    if (desc->n_snap >= 10) {
        const int w = std::max(1, desc->n_snap / 10);
        chunk_opts.push_back({2, w});
        chunk_opts.push_back({3, w});
        for (int pct : {15, 20}) {
            const int wl = std::max(1, desc->n_snap * pct / 100);
            if (wl != w && wl <= desc->n_snap - 1)
                chunk_opts.push_back({2, wl});
        }
    }
    for (int block : {64, 256}) {
        int per_cu = 0;
        HIP_TRY(hipModuleOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, ld.kernel, block, 0));
        per_cu = std::max(per_cu, 1);
        const int64_t need = std::max<int64_t>(1, (total + block - 1) / block);
        const int64_t resident = (int64_t)per_cu * cus;
        const int waves_per_block = block / 64;
        // waves per SIMD: 1, 2, 4, and enough lanes for one trajectory each
        std::vector<int64_t> grids = {std::min(need, resident)};
        for (int wps : {1, 2, 4}) {
            int64_t g = (int64_t)cus * 4 * wps / waves_per_block;
            if (g < need && g <= resident)
                grids.push_back(g);
        }
        std::sort(grids.begin(), grids.end());
        grids.erase(std::unique(grids.begin(), grids.end()), grids.end());
        for (int64_t g : grids)
            for (const ChunkOpt &ch : chunk_opts)
                cands.push_back({block, (int)g, ch.chunks, ch.window, SSA_PLACE_EXPLICIT});
    }
    // 512-thread workgroups: one event-loop wave per SIMD, each paired with
    // the wave that forms its draws
    {
        int per_cu = 0;
        HIP_TRY(hipModuleOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, ld.kernel_pc, 512, ld.pc_lds_pad));
        if (per_cu >= 1) {
            const int64_t need = std::max<int64_t>(1, (total + 255) / 256);
            const int64_t g = std::min<int64_t>(need, cus);
            // producers on their own or the next SIMD; claims as they come, or
            // the first ones wave-major (one launch per item only), with wave
            // priorities that favour wave 0's draws
            std::vector<int> places = {SSA_PLACE_EXPLICIT, SSA_PLACE_EXPLICIT | SSA_PLACE_NEIGHBOUR_PRODUCER};
            if (desc->n_items == 1) {
                places.push_back(SSA_PLACE_EXPLICIT | SSA_PLACE_WAVE_MAJOR);
                places.push_back(SSA_PLACE_EXPLICIT | SSA_PLACE_NEIGHBOUR_PRODUCER | SSA_PLACE_WAVE_MAJOR);
                places.push_back(SSA_PLACE_EXPLICIT | SSA_PLACE_SOLO_WAVE0 | SSA_PLACE_WAVE_MAJOR);
                // the heaviest trajectories alone on a SIMD, fed ahead of the rest
                places.push_back(SSA_PLACE_EXPLICIT | SSA_PLACE_SOLO_WAVE0 | SSA_PLACE_WAVE_MAJOR |
                                 SSA_PLACE_FEED_WAVE0);
                places.push_back(SSA_PLACE_EXPLICIT | SSA_PLACE_SOLO_WAVE0 | SSA_PLACE_WAVE_MAJOR |
                                 SSA_PLACE_PRODUCER_FIRST);
                // three event-loop waves, wave 0 and its producer on SIMDs of their own
                places.push_back(SSA_PLACE_EXPLICIT | SSA_PLACE_DEDICATED_FEED0 | SSA_PLACE_WAVE_MAJOR);
                // the same with two producers for wave 0
                places.push_back(SSA_PLACE_EXPLICIT | SSA_PLACE_DEDICATED_FEED0 | SSA_PLACE_WAVE_MAJOR |
                                 SSA_PLACE_TWO_FEED0);
            }
            for (int pl : places)
                for (const ChunkOpt &ch : chunk_opts)
                    cands.push_back({512, (int)g, ch.chunks, ch.window, pl});
        }
    }
    cands.erase(std::unique(cands.begin(), cands.end(),
                            [](const Cand &a, const Cand &b) {
                                return a.block == b.block && a.grid == b.grid && a.chunks == b.chunks &&
                                       a.window == b.window && a.place == b.place;
                            }),
                cands.end());
    Tuned best;
    best.ms = 1e300;
    for (const Cand &c : cands) {
        ssa_run_desc d2 = *desc;
        std::vector<ssa_item> items(desc->items, desc->items + desc->n_items);
        for (auto &it : items) {
            it.d_snap = nullptr;
            it.d_n_events = nullptr;
            it.d_t_last = nullptr;
            it.d_status = nullptr;
            it.d_rec_t = nullptr;
            it.d_rec_j = nullptr;
            it.d_rec_n = nullptr;
        }
        d2.items = items.data();
        d2.block_size = c.block;
        d2.grid_size = c.grid;
        d2.n_chunks = c.chunks;
        d2.first_window = c.window;
        d2.placement = c.place;
        ssa_run *r = new (std::nothrow) ssa_run;
        if (!r)
            return fail(SSA_E_NOMEM, "out of host memory");
        rc = run_impl(&d2, r);
        float ms = 0.0f;
        if (rc == SSA_OK) {
            hipError_t e = hipEventSynchronize(r->ev1);
            if (e == hipSuccess)
                e = hipEventElapsedTime(&ms, r->ev0, r->ev1);
            if (e != hipSuccess)
                rc = fail(SSA_E_DEVICE, std::string("autotune trial: ") + hipGetErrorString(e));
        }
        std::string keep = g_err;
        release(r);
        g_err = keep;
        if (rc != SSA_OK)
            return rc;
        if (ms < best.ms) {
            best.block = c.block;
            best.grid = c.grid;
            best.chunks = c.chunks;
            best.window = c.window;
            best.place = c.place & ~SSA_PLACE_EXPLICIT;
            best.ms = ms;
        }
    }
    tune_store(tune_key(desc, src), best);
    if (res) {
        res->block_size = best.block;
        res->grid_size = best.grid;
        res->n_chunks = best.chunks;
        res->first_window = best.window;
        res->placement = SSA_PLACE_EXPLICIT | best.place;
        res->best_ms = best.ms;
        res->n_candidates = (int32_t)cands.size();
    }
    return SSA_OK;
}

// Compile (and cache on disk) the kernel a run with this descriptor would use,
// without touching a GPU. Used by the build step to fill the kernel cache.
int ssa_prepare(const ssa_run_desc *desc)
{
    int rc = validate_desc(desc);
    if (rc != SSA_OK)
        return rc;
    std::string src;
    build_source(desc, src);
    std::vector<char> code;
    return compile_source(src, "gfx950", code);
}

// Compile (if needed) and report the on-disk code object of a descriptor.
int ssa_kernel_file(const ssa_run_desc *desc, char *path, size_t len)
{
    int rc = validate_desc(desc);
    if (rc != SSA_OK)
        return rc;
    if (!path || len == 0)
        return fail(SSA_E_INVALID, "path buffer is NULL or empty");
    std::string src, file;
    build_source(desc, src);
    std::vector<char> code;
    rc = compile_source(src, "gfx950", code, &file);
    if (rc != SSA_OK)
        return rc;
    if (file.size() + 1 > len)
        return fail(SSA_E_INVALID, "path buffer too small");
    std::memcpy(path, file.c_str(), file.size() + 1);
    return SSA_OK;
}

// Write the generated kernel source for a descriptor to `path` (inspection).
int ssa_dump_source(const ssa_run_desc *desc, const char *path)
{
    int rc = validate_desc(desc);
    if (rc != SSA_OK)
        return rc;
    std::string src;
    build_source(desc, src);
    std::ofstream out(path);
    if (!out)
        return fail(SSA_E_INVALID, "cannot open path");
    out << src;
    return SSA_OK;
}

}  // extern "C"
