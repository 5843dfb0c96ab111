// fill.hip -- bulk-fill kernels for gfx950 (Tables 4-5, Section 3).
//
// Output layout: substream-major, value t of substream i at out[i * P + t].
// Every substream's values equal the serial definition (consecutive calls of
// one scalar generator on that substream), whatever the launch shape.
//
// Two kernel families:
//
//  * k_fill_wave ("one wavefront per substream"), for engines whose word at
//    any position is cheap to reach: Philox4x32-10 and Philox-4x64 (counter
//    based) and PCG64 (lane l steps with the stride-64 LCG multiplier A^64).
//    The 64 lanes of a wavefront generate consecutive words of one substream
//    (R words per lane, a "chunk" of 64 R words per iteration), classify every
//    word as if a sample started there, and then resolve which words really
//    start samples with a short scalar walk over the rare multi-word cases
//    (ziggurat wedge/tail).  Accepted samples are compacted with ballot +
//    popcount so each chunk is written as one contiguous, coalesced run.
//
//  * k_fill_lane ("one lane per substream"), for engines that can only step
//    serially (xoshiro256++, sfc64, ranlux++); each lane runs the serial
//    sampler directly.
//
// Device code is compiled with -ffp-contract=off: every floating-point
// expression is rounded exactly as written, as in the serial definition.
#include <hip/hip_runtime.h>

#include <mutex>

#include "rp_internal.h"

#define RP_TBL __device__ const
#include "zig_tables.inc"
#include "crmath.h"

namespace rp {

// ---------------------------------------------------------------------------
// constant tables uploaded once per device
struct PcgAffineDev {
    uint64_t mlo, mhi, plo, phi;
};
__constant__ PcgAffineDev c_pcg_lane[65];  // A^(8l), G_(8l) for l = 0..64 (8 words per lane)
__constant__ PcgAffineDev c_pcg_pow2[64];  // A^(2^k), G_(2^k)
__constant__ PcgAffineDev c_pcg_s127;      // A^127, G_127 (direct order: pair to pair)
__constant__ uint32_t c_rl_B[kRlL * kRlL];  // ranlux++ folded step table (rl_mul_tab)

static PcgAffineDev to_dev(const PcgAffine &p) { return {p.mult.lo, p.mult.hi, p.plus.lo, p.plus.hi}; }

static PcgAffine compose(const PcgAffine &outer, const PcgAffine &inner)
{
    // s -> outer.m (inner.m s + inner.p inc) + outer.p inc
    return {mul128(outer.mult, inner.mult), add128(mul128(outer.mult, inner.plus), outer.plus)};
}

int ensure_device_tables()
{
    static std::mutex mu;
    static bool done[64] = {false};
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail(RP_EDEVICE, "hipGetDevice: %s", hipGetErrorString(e));
    if (dev < 0 || dev >= 64) return fail(RP_EDEVICE, "device index %d out of range", dev);
    std::lock_guard<std::mutex> lk(mu);
    if (done[dev]) return RP_OK;
    PcgAffineDev lane[65], pow2[64];
    const PcgAffine step{{kPcgMult, 0}, {1, 0}};
    PcgAffine step8{{1, 0}, {0, 0}};
    for (int k = 0; k < 8; k++) step8 = compose(step, step8);
    PcgAffine cur{{1, 0}, {0, 0}};
    for (int l = 0; l <= 64; l++) {
        lane[l] = to_dev(cur);
        cur = compose(step8, cur);
    }
    PcgAffine p = step;
    for (int k = 0; k < 64; k++) {
        pow2[k] = to_dev(p);
        p = compose(p, p);
    }
    PcgAffine s127{{1, 0}, {0, 0}};
    for (int k = 0; k < 127; k++) s127 = compose(step, s127);
    const PcgAffineDev s127d = to_dev(s127);
    e = hipMemcpyToSymbol(HIP_SYMBOL(c_pcg_lane), lane, sizeof lane);
    if (e == hipSuccess) e = hipMemcpyToSymbol(HIP_SYMBOL(c_pcg_pow2), pow2, sizeof pow2);
    if (e == hipSuccess) e = hipMemcpyToSymbol(HIP_SYMBOL(c_pcg_s127), &s127d, sizeof s127d);
    if (e == hipSuccess) e = hipMemcpyToSymbol(HIP_SYMBOL(c_rl_B), ranlux_B(), sizeof c_rl_B);
    if (e != hipSuccess) return fail(RP_EDEVICE, "uploading constant tables: %s", hipGetErrorString(e));
    done[dev] = true;
    return RP_OK;
}

// ---------------------------------------------------------------------------
// small device helpers
__device__ __forceinline__ uint64_t readlane64(uint64_t v, int l)
{
    uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, l);
    uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), l);
    return (uint64_t)lo | ((uint64_t)hi << 32);
}

__device__ __forceinline__ double u01_53(uint64_t w) { return (double)(w >> 11) * 0x1.0p-53; }
__device__ __forceinline__ double u01_52(uint64_t w)
{
    return __longlong_as_double((long long)((w >> 12) | 0x3ff0000000000000ull)) - 1.0;
}
__device__ __forceinline__ float u01f_24(uint32_t u) { return (float)(u >> 8) * 0x1.0p-24f; }
// float ziggurat: the wedge / tail uniform of a 32-bit item, exact in binary64
__device__ __forceinline__ double u01_24d(uint64_t it) { return (double)((uint32_t)it >> 8) * 0x1.0p-24; }
// The float ziggurat reads 32-bit items: strip = low byte, normal sign = bit
// 8, magnitude = the remaining 23 (normal) or 24 (exponential) bits.  It is
// the binary64 ziggurat run on the magnitude m 2^29, i.e. on the word with
// the same low byte (and sign) and m 2^29 in the magnitude field.
template <int DIST>
__device__ __forceinline__ uint64_t item_word(uint64_t it)
{
    const uint32_t u = (uint32_t)it;
    if (DIST == RP_NORM) return (uint64_t)(u & 0x1ffu) | ((uint64_t)(u >> 9) << 38);
    return (uint64_t)(u & 0xffu) | ((uint64_t)(u >> 8) << 37);
}
// the uniform of a follow-up word (binary64 draws) or item (float draws)
template <bool HALF>
__device__ __forceinline__ double zig_u(uint64_t w)
{
    if constexpr (HALF) return u01_24d(w);
    else return (double)(w >> 11) * 0x1.0p-53;
}
__device__ __forceinline__ float u01f_23(uint32_t u) { return __uint_as_float((u >> 9) | 0x3f800000u) - 1.0f; }

__device__ __forceinline__ u128 pcg_apply(const PcgAffineDev &m, u128 s, u128 inc)
{
    u128 a = mul128(u128{m.mlo, m.mhi}, s);
    u128 b = mul128(u128{m.plo, m.phi}, inc);
    return add128(a, b);
}

// state advanced by n steps: binary composition of the A^(2^k) maps
__device__ __forceinline__ u128 pcg_jump(u128 s, u128 inc, uint64_t n)
{
    for (int k = 0; n; k++, n >>= 1)
        if (n & 1) s = pcg_apply(c_pcg_pow2[k], s, inc);
    return s;
}

// The tail loop accepts with probability above 0.9 per iteration; this cap
// (never reached: 0.1^4096) only bounds the loop.
static constexpr int kMaxTailIters = 4096;

// ---------------------------------------------------------------------------
// ziggurat tables in LDS
struct WKe {
    double w;    // strip width factor W[j]
    uint64_t k;  // fast-accept bound K[j]
};
struct ZigLds {
    __align__(16) WKe WK[256];  // W and K of a strip in one 16-byte read
    double F[256];
    double X[256];
    double S[256];
    double DP[256];
    double DM[256];
};

// The elementary functions of the bitexact setting (correctly rounded, the
// same on every platform), out of line.  Kernels take the setting as a
// template parameter (BX): the ordinary instantiations call none of these,
// so their registers and occupancy are those of the platform functions.
__device__ __noinline__ double bx_exp(double x) { return crm::cr_exp(x); }
__device__ __noinline__ double bx_log(double x) { return crm::cr_log(x); }
__device__ __noinline__ double bx_log1p(double x) { return crm::cr_log1p(x); }
__device__ __noinline__ double bx_pow(double x, double y) { return crm::cr_pow(x, y); }
__device__ __noinline__ double bx_powinv(double u, double a) { return crm::cr_powinv(u, a); }
template <bool BX>
__device__ __forceinline__ double f_exp(double x)
{
    if constexpr (BX) return bx_exp(x);
    else return exp(x);
}
template <bool BX>
__device__ __forceinline__ double f_log(double x)
{
    if constexpr (BX) return bx_log(x);
    else return log(x);
}
template <bool BX>
__device__ __forceinline__ double f_log1p(double x)
{
    if constexpr (BX) return bx_log1p(x);
    else return log1p(x);
}
template <bool BX>
__device__ __forceinline__ double f_pow(double x, double y)
{
    if constexpr (BX) return bx_pow(x, y);
    else return pow(x, y);
}

// The transform code XF of the fill kernels: the law (bits 0..5) and the
// bitexact setting (kXfBx).
constexpr int kXfBx = 64;
constexpr int xf_law(int xf) { return xf & (kXfBx - 1); }
constexpr bool xf_bx(int xf) { return (xf & kXfBx) != 0; }

// flags: the FillArgs flags of the call.  With the squeeze switched off the
// bands are infinite, so neither squeeze test decides and every wedge test
// evaluates f(x) (the decisions, and so the values, are the same).
template <int DIST>
__device__ __forceinline__ void load_zig(ZigLds *t, int flags)
{
    const bool nrm = DIST == RP_NORM;
    const bool sq = !(flags & kFlagNoSqueeze);
    for (int k = threadIdx.x; k < 256; k += blockDim.x) {
        t->WK[k].w = nrm ? RP_ZN_W[k] : RP_ZE_W[k];
        t->WK[k].k = nrm ? RP_ZN_K[k] : RP_ZE_K[k];
        t->F[k] = nrm ? RP_ZN_F[k] : RP_ZE_F[k];
        t->X[k] = nrm ? RP_ZN_X[k] : RP_ZE_X[k];
        t->S[k] = nrm ? RP_ZN_S[k] : RP_ZE_S[k];
        t->DP[k] = sq ? (nrm ? RP_ZN_DP[k] : RP_ZE_DP[k]) : __builtin_huge_val();
        t->DM[k] = sq ? (nrm ? RP_ZN_DM[k] : RP_ZE_DM[k]) : __builtin_huge_val();
    }
}

// Wedge test of strip j >= 1 (Section 3.1, ziggurat figure): y drawn in
// [f_j, f_{j-1}) is accepted iff y < f(x).  The secant/tangent squeeze
// decides most cases without exp(); its bounds carry a margin far above the
// rounding of the secant and of exp, so a squeeze decision always equals the
// plain test evaluated in binary64.
template <int DIST, bool HALF = false, bool BX = false>
__device__ __forceinline__ bool wedge_accept(const ZigLds *t, int j, double x, uint64_t uword)
{
    double U = zig_u<HALF>(uword);
    double fj = t->F[j], fj1 = t->F[j - 1];
    double y = fj + U * (fj1 - fj);
    double l = fj1 + t->S[j] * (x - t->X[j - 1]);
    if (y < l - t->DM[j]) return true;
    if (y > l + t->DP[j]) return false;
    if (DIST == RP_NORM) return y < f_exp<BX>(-0.5 * x * x);
    return y < f_exp<BX>(-x);
}

// ---------------------------------------------------------------------------
// wavefront-per-substream engines.  A chunk is 64 * R consecutive words of
// one substream; lane l holds words R l .. R l + R - 1 of the chunk.  Word
// positions are counted from the start of the block (or state) the substream
// pointed at when the call began.  Per-substream values (keys, increments) are
// wave-uniform and live in scalar registers.
//
// Direct order (fills of one item per word or half, which need no parse):
// the same chunk, but lane l holds groups of G consecutive words at positions
// 64 G k + G l .. 64 G k + G l + G - 1, k = 0 .. R/G - 1, so that one store
// instruction per group covers 64 G consecutive words with no transpose
// through LDS.  G is the engine's block size (2 for Philox4x32-10 and PCG64,
// 4 for Philox-4x64).  load_direct / gen_direct replace load / gen /
// next_chunk; gen_direct also moves to the next chunk.
static constexpr int kWaveR = 8;

__device__ __forceinline__ uint64_t uni64(uint64_t v)
{
    uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    return (uint64_t)lo | ((uint64_t)hi << 32);
}

struct WavePhilox32 {
    static constexpr bool kDirect = true;  // raw / uniform fills in store order
    static constexpr int R = kWaveR;  // 4 blocks of 2 words per lane
    uint64_t key, b0lo, b0hi;         // uniform: key, counter of the first block
    uint64_t clo, chi;                // this lane's first block in the chunk
    uint32_t phase0;

    __device__ void load(const FillArgs &a, uint64_t i, int lane)
    {
        b0lo = uni64(a.words[i]);
        b0hi = uni64(a.words[a.n + i]);
        key = uni64(a.words[2 * a.n + i]);
        phase0 = __builtin_amdgcn_readfirstlane(a.phase[i]);
        clo = b0lo + (uint64_t)(lane * (R / 2));
        chi = b0hi + (clo < b0lo ? 1u : 0u);
    }
    // float draws: R / 2 words per lane (R / 4 blocks), 32 R words per chunk
    __device__ void load_half(const FillArgs &a, uint64_t i, int lane)
    {
        load(a, i, lane);
        clo = b0lo + (uint64_t)(lane * (R / 4));
        chi = b0hi + (clo < b0lo ? 1u : 0u);
    }
    __device__ void gen_half(uint64_t w[R / 2])
    {
        uint64_t kk = key;
        asm volatile("" : "+s"(kk));
#pragma unroll
        for (int k = 0; k < R / 4; k++) {
            uint64_t lo = clo + (uint64_t)k;
            uint64_t hi = chi + (lo < clo ? 1u : 0u);
            philox4x32(lo, hi, kk, w[2 * k], w[2 * k + 1]);
        }
        const uint64_t o = clo;
        clo += 64 * (R / 4);
        chi += (clo < o) ? 1u : 0u;
    }
    static constexpr int G = 2;
    __device__ void load_direct(const FillArgs &a, uint64_t i, int lane)
    {
        load(a, i, lane);
        clo = b0lo + (uint64_t)lane;  // block 64 k + lane of the chunk
        chi = b0hi + (clo < b0lo ? 1u : 0u);
    }
    __device__ void gen_direct(uint64_t w[R])
    {
        uint64_t kk = key;
        asm volatile("" : "+s"(kk));
#pragma unroll
        for (int k = 0; k < R / 2; k++) {
            uint64_t lo = clo + (uint64_t)(64 * k);
            uint64_t hi = chi + (lo < clo ? 1u : 0u);
            philox4x32(lo, hi, kk, w[2 * k], w[2 * k + 1]);
        }
        next_chunk();
    }
    __device__ void gen(uint64_t w[R]) const
    {
        // an opaque copy of the key: its ten round keys are then formed here,
        // once per chunk, instead of hoisted out of the chunk loop where they
        // would hold twenty scalar registers for the whole kernel
        uint64_t kk = key;
        asm volatile("" : "+s"(kk));
#pragma unroll
        for (int k = 0; k < R / 2; k++) {
            uint64_t lo = clo + (uint64_t)k;
            uint64_t hi = chi + (lo < clo ? 1u : 0u);
            philox4x32(lo, hi, kk, w[2 * k], w[2 * k + 1]);
        }
    }
    __device__ void next_chunk()
    {
        uint64_t o = clo;
        clo += 64 * (R / 2);
        chi += (clo < o) ? 1u : 0u;
    }
    __device__ uint64_t far_word(uint64_t pos) const
    {
        uint64_t lo = b0lo + pos / 2, hi = b0hi + (lo < b0lo ? 1u : 0u);
        uint64_t w0, w1;
        philox4x32(lo, hi, key, w0, w1);
        return (pos & 1) ? w1 : w0;
    }
    __device__ void store(const FillArgs &a, uint64_t i, uint64_t pos) const
    {
        uint64_t lo = b0lo + pos / 2, hi = b0hi + (lo < b0lo ? 1u : 0u);
        a.words[i] = lo;
        a.words[a.n + i] = hi;
        a.phase[i] = (uint32_t)(pos & 1);
    }
};

struct WavePhilox64 {
    static constexpr bool kDirect = true;  // raw / uniform fills in store order
    static constexpr int R = kWaveR;  // 2 blocks of 4 words per lane
    uint64_t b0[4], k0, k1;          // uniform
    uint64_t c[4];                   // this lane's first block in the chunk
    uint32_t phase0;

    __device__ static void add256(const uint64_t in[4], uint64_t add, uint64_t out[4])
    {
        uint64_t carry = add;
#pragma unroll
        for (int k = 0; k < 4; k++) {
            uint64_t v = in[k] + carry;
            carry = (v < carry) ? 1u : 0u;
            out[k] = v;
        }
    }
    __device__ void load(const FillArgs &a, uint64_t i, int lane)
    {
#pragma unroll
        for (int k = 0; k < 4; k++) b0[k] = uni64(a.words[(uint64_t)k * a.n + i]);
        k0 = uni64(a.words[4 * a.n + i]);
        k1 = uni64(a.words[5 * a.n + i]);
        phase0 = __builtin_amdgcn_readfirstlane(a.phase[i]);
        add256(b0, (uint64_t)(lane * (R / 4)), c);
    }
    // float draws: R / 2 = 4 words (one block) per lane, 64 blocks per chunk
    static_assert(R == 8, "one block per lane for float draws");
    __device__ void load_half(const FillArgs &a, uint64_t i, int lane)
    {
        load(a, i, lane);
        add256(b0, (uint64_t)lane, c);
    }
    __device__ void gen_half(uint64_t w[R / 2])
    {
        philox4x64(c, k0, k1, w);
        add256(c, 64, c);
    }
    static constexpr int G = 4;
    __device__ void load_direct(const FillArgs &a, uint64_t i, int lane)
    {
        load(a, i, lane);
        add256(b0, (uint64_t)lane, c);  // block 64 k + lane of the chunk
    }
    __device__ void gen_direct(uint64_t w[R])
    {
#pragma unroll
        for (int k = 0; k < R / 4; k++) {
            uint64_t blk[4];
            add256(c, (uint64_t)(64 * k), blk);
            philox4x64(blk, k0, k1, &w[4 * k]);
        }
        next_chunk();
    }
    __device__ void gen(uint64_t w[R]) const
    {
#pragma unroll
        for (int k = 0; k < R / 4; k++) {
            uint64_t blk[4];
            add256(c, (uint64_t)k, blk);
            philox4x64(blk, k0, k1, &w[4 * k]);
        }
    }
    __device__ void next_chunk() { add256(c, 64 * (R / 4), c); }
    __device__ uint64_t far_word(uint64_t pos) const
    {
        uint64_t blk[4], w[4];
        add256(b0, pos / 4, blk);
        philox4x64(blk, k0, k1, w);
        uint64_t r = w[0];
        r = ((pos & 3) == 1) ? w[1] : r;
        r = ((pos & 3) == 2) ? w[2] : r;
        r = ((pos & 3) == 3) ? w[3] : r;
        return r;
    }
    __device__ void store(const FillArgs &a, uint64_t i, uint64_t pos) const
    {
        uint64_t blk[4];
        add256(b0, pos / 4, blk);
#pragma unroll
        for (int k = 0; k < 4; k++) a.words[(uint64_t)k * a.n + i] = blk[k];
        a.phase[i] = (uint32_t)(pos & 3);
    }
};

// squares64: word p of the substream is squares64(c0 + p, key); any
// position is one evaluation away.  No block phase (one word per counter).
struct WaveSquares {
    static constexpr bool kDirect = true;  // raw / uniform fills in store order
    static constexpr int R = kWaveR;
    static constexpr int G = 1;
    uint64_t c0, key;  // uniform
    uint64_t c;        // this lane's first counter in the chunk
    uint32_t phase0;

    __device__ void load(const FillArgs &a, uint64_t i, int lane)
    {
        c0 = uni64(a.words[i]);
        key = uni64(a.words[a.n + i]);
        phase0 = 0;
        c = c0 + (uint64_t)(lane * R);
    }
    __device__ void gen(uint64_t w[R]) const
    {
#pragma unroll
        for (int k = 0; k < R; k++) w[k] = squares64(c + (uint64_t)k, key);
    }
    __device__ void next_chunk() { c += 64 * R; }
    __device__ void load_direct(const FillArgs &a, uint64_t i, int lane)
    {
        load(a, i, lane);
        c = c0 + (uint64_t)lane;  // positions 64 k + lane
    }
    __device__ void gen_direct(uint64_t w[R])
    {
#pragma unroll
        for (int k = 0; k < R; k++) w[k] = squares64(c + (uint64_t)(64 * k), key);
        c += 64 * R;
    }
    __device__ void load_half(const FillArgs &a, uint64_t i, int lane)
    {
        load(a, i, lane);
        c = c0 + (uint64_t)(lane * (R / 2));
    }
    __device__ void gen_half(uint64_t w[R / 2])
    {
#pragma unroll
        for (int k = 0; k < R / 2; k++) w[k] = squares64(c + (uint64_t)k, key);
        c += 32 * R;
    }
    __device__ void store(const FillArgs &a, uint64_t i, uint64_t pos) const { a.words[i] = c0 + pos; }
};

// ChaCha20: one 8-word block per lane per chunk (block counter c0 + 64 k +
// lane in chunk k); the 32-bit counter wraps modulo 2^32.  Raw fills use the
// LDS transpose: lane-private 64-byte stores of whole blocks measured slow.
struct WaveChacha {
    static constexpr bool kDirect = false;
    static constexpr int R = kWaveR;  // one block
    static constexpr int G = 8;
    uint32_t key[8], n0, n1, n2;  // uniform
    uint32_t c0, c;               // counter at the call's first block; this lane's block
    uint32_t phase0;
    __device__ void load(const FillArgs &a, uint64_t i, int lane)
    {
#pragma unroll
        for (int k = 0; k < 4; k++) {
            const uint64_t w = uni64(a.words[(uint64_t)k * a.n + i]);
            key[2 * k] = (uint32_t)w;
            key[2 * k + 1] = (uint32_t)(w >> 32);
        }
        const uint64_t w4 = uni64(a.words[4 * a.n + i]), w5 = uni64(a.words[5 * a.n + i]);
        n0 = (uint32_t)w4;
        n1 = (uint32_t)(w4 >> 32);
        n2 = (uint32_t)w5;
        c0 = (uint32_t)(w5 >> 32);
        phase0 = __builtin_amdgcn_readfirstlane(a.phase[i]);
        c = c0 + (uint32_t)lane;
    }
    __device__ void gen(uint64_t w[R]) const { chacha20_block(key, n0, n1, n2, c, w); }
    __device__ void next_chunk() { c += 64; }
    // float draws: 4 words per lane, two lanes per block
    bool upper = false;
    __device__ void load_half(const FillArgs &a, uint64_t i, int lane)
    {
        load(a, i, lane);
        c = c0 + (uint32_t)(lane >> 1);
        upper = lane & 1;
    }
    __device__ void gen_half(uint64_t w[R / 2])
    {
        uint64_t b[8];
        chacha20_block(key, n0, n1, n2, c, b);
#pragma unroll
        for (int k = 0; k < 4; k++) w[k] = upper ? b[4 + k] : b[k];
        c += 32;
    }
    __device__ void store(const FillArgs &a, uint64_t i, uint64_t pos) const
    {
        const uint32_t blk = c0 + (uint32_t)(pos / 8);
        a.words[5 * a.n + i] = (uint64_t)n2 | ((uint64_t)blk << 32);
        a.phase[i] = (uint32_t)(pos & 7);
    }
};

// PCG64: lane l starts each chunk at word R l (state A^(R l) s + G_(R l) inc),
// takes R - 1 ordinary steps inside the chunk, and moves to the next chunk
// with the stride-64R map from the constant table.
struct WavePcg {
    static constexpr bool kDirect = true;  // raw / uniform fills in store order
    static constexpr int R = kWaveR;
    u128 s;        // this lane's state at its first word of the chunk
    u128 inc, s0;  // uniform
    uint32_t phase0;

    __device__ void load(const FillArgs &a, uint64_t i, int lane)
    {
        s0 = u128{uni64(a.words[i]), uni64(a.words[a.n + i])};
        inc = u128{uni64(a.words[2 * a.n + i]), uni64(a.words[3 * a.n + i])};
        phase0 = 0;
        s = pcg_apply(c_pcg_lane[lane], s0, inc);
    }
    // float draws: words (R / 2) l .. (R / 2) l + R / 2 - 1 of a 32 R-word
    // chunk; the next chunk is A^(32 R) = A^256 away
    static_assert(R == 8, "A^256 advances a float-draw chunk");
    __device__ void load_half(const FillArgs &a, uint64_t i, int lane)
    {
        s0 = u128{uni64(a.words[i]), uni64(a.words[a.n + i])};
        inc = u128{uni64(a.words[2 * a.n + i]), uni64(a.words[3 * a.n + i])};
        phase0 = 0;
        s = pcg_jump(s0, inc, (uint64_t)(R / 2) * (uint64_t)lane);
    }
    __device__ void gen_half(uint64_t w[R / 2])
    {
        u128 t = s;
#pragma unroll
        for (int k = 0; k < R / 2; k++) {
            w[k] = pcg_dxsm(t);
            if (k + 1 < R / 2) t = pcg_step(t, inc);
        }
        s = pcg_apply(c_pcg_pow2[8], s, inc);
    }
    // direct order: words 128 k + 2 l and 128 k + 2 l + 1; from the second
    // of a pair to the first of the next pair is 127 steps (A^127 s + c127,
    // c127 = G_127 inc formed once)
    static constexpr int G = 2;
    u128 c127;
    __device__ void load_direct(const FillArgs &a, uint64_t i, int lane)
    {
        s0 = u128{uni64(a.words[i]), uni64(a.words[a.n + i])};
        inc = u128{uni64(a.words[2 * a.n + i]), uni64(a.words[3 * a.n + i])};
        phase0 = 0;
        s = pcg_jump(s0, inc, 2 * (uint64_t)lane);
        c127 = mul128(u128{c_pcg_s127.plo, c_pcg_s127.phi}, inc);
    }
    __device__ void gen_direct(uint64_t w[R])
    {
        const u128 m{c_pcg_s127.mlo, c_pcg_s127.mhi};
        u128 t = s;
#pragma unroll
        for (int k = 0; k < R / 2; k++) {
            w[2 * k] = pcg_dxsm(t);
            t = pcg_step(t, inc);
            w[2 * k + 1] = pcg_dxsm(t);
            t = add128(mul128(m, t), c127);
        }
        s = t;
    }
    __device__ void gen(uint64_t w[R]) const
    {
        u128 t = s;
#pragma unroll
        for (int k = 0; k < R; k++) {
            w[k] = pcg_dxsm(t);
            if (k + 1 < R) t = pcg_step(t, inc);
        }
    }
    __device__ void next_chunk() { s = pcg_apply(c_pcg_lane[64], s, inc); }
    __device__ uint64_t far_word(uint64_t pos) const { return pcg_dxsm(pcg_jump(s0, inc, pos)); }
    __device__ void store(const FillArgs &a, uint64_t i, uint64_t pos) const
    {
        u128 f = pcg_jump(s0, inc, pos);
        a.words[i] = f.lo;
        a.words[a.n + i] = f.hi;
    }
};

template <int DIST, int OT>
struct OutType;
template <int D> struct OutType<D, RP_U64> { using T = uint64_t; };
template <int D> struct OutType<D, RP_U32> { using T = uint32_t; };
template <int D> struct OutType<D, RP_F64> { using T = double; };
template <int D> struct OutType<D, RP_F32> { using T = float; };

// value of a fixed-consumption or Lemire item.  'it' is a 64-bit word or a
// 32-bit half (in the low bits).  Returns whether the item is accepted.
template <int DIST, int OT>
__device__ __forceinline__ bool item_value(uint64_t it, const FillArgs &a, typename OutType<DIST, OT>::T &v)
{
    if constexpr (DIST == RP_RAW) {
        v = (typename OutType<DIST, OT>::T)it;
        return true;
    } else if constexpr (DIST == RP_U01 && OT == RP_F64) {
        v = (a.flags & RP_FLAG_52BIT) ? u01_52(it) : u01_53(it);
        return true;
    } else if constexpr (DIST == RP_U01 && OT == RP_F32) {
        v = (a.flags & RP_FLAG_52BIT) ? u01f_23((uint32_t)it) : u01f_24((uint32_t)it);
        return true;
    } else if constexpr (DIST == RP_BOUNDED && OT == RP_U64) {
        // Lemire: w b = hi 2^64 + lo; reject iff lo < (2^64 - b) mod b
        if (a.bound == 0) {
            v = it;
            return true;
        }
        v = mulhi64(it, a.bound);
        return it * a.bound >= a.thresh;
    } else {  // RP_BOUNDED, RP_U32
        const uint32_t b = (uint32_t)a.bound;
        if (b == 0) {
            v = (uint32_t)it;
            return true;
        }
        uint64_t p = (uint64_t)(uint32_t)it * b;
        v = (uint32_t)(p >> 32);
        return (uint32_t)p >= (uint32_t)a.thresh;
    }
}

// number of set bits of mask in lanes below this one
__device__ __forceinline__ uint32_t mbcnt64(uint64_t mask)
{
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

// Fast ziggurat test of one word as the first word of a sample.  Returns true
// when the sample is accepted from this word alone (value in val); otherwise
// the word starts a wedge test or the tail and needs the next word(s).
template <int DIST, bool HALF = false>
__device__ __forceinline__ bool zig_fast(const WKe *wk, uint64_t w_or_item, double &val)
{
    const uint64_t w = HALF ? item_word<DIST>(w_or_item) : w_or_item;
    const int j = (int)(w & 0xff);
    const WKe e = wk[j];
    if (DIST == RP_NORM) {
        const uint64_t m = (w >> 9) & ((1ull << 52) - 1);
        // m < 2^52: (2^52 + m) - 2^52 is exact; the sign comes from bit 8
        const double md = __longlong_as_double((long long)(m | 0x4330000000000000ull)) - 0x1.0p52;
        const double x = md * e.w;
        const uint64_t sgn = (w & 0x100) << 55;
        val = __longlong_as_double(__double_as_longlong(x) ^ (long long)sgn);
        return m < e.k;
    } else {
        const uint64_t m = (w >> 8) & ((1ull << 53) - 1);
        // m < 2^53: hi 2^32 + lo formed exactly with one fused operation
        const double md = __fma_rn((double)(uint32_t)(m >> 32), 0x1.0p32, (double)(uint32_t)m);
        val = md * e.w;
        return m < e.k;
    }
}

// Orders a wavefront's LDS accesses: writes before the barrier are visible
// to reads after it (all lanes of one wavefront).
__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Slow part of a sample whose first word w0 failed the fast test.  The
// following words are word(1), word(2), ...; only `avail` of them exist in
// the current chunk.  Returns the words used including w0 (2 for a wedge test
// or the exponential tail, 3 + 2 t for the normal tail), or 0 if the sample
// needs words past the chunk; then, for the normal tail, *u1 receives an
// unused first word of a pair when one is left (has_u1).
// exp and log1p kept out of line on the rare paths of the wavefront kernel,
// so that their constants do not occupy registers across its chunk loop
__device__ __noinline__ double exp_ool(double x) { return exp(x); }
__device__ __noinline__ double log1p_ool(double x) { return log1p(x); }
// one pair of the normal tail test: accepted iff e2 + e2 > e1 e1; t = r + e1
template <bool HALF, bool BX>
__device__ __noinline__ bool normal_tail_pair(uint64_t a, uint64_t b, double &t)
{
    const double e1 = -f_log1p<BX>(-zig_u<HALF>(a)) / RP_ZN_R;
    const double e2 = -f_log1p<BX>(-zig_u<HALF>(b));
    t = RP_ZN_R + e1;
    return e2 + e2 > e1 * e1;
}

// wedge-test tables in global memory (read only on the rare wedge path)
template <int DIST>
struct ZigG {
    // Each table address passes through an opaque copy where it is used: the
    // wedge test is a rare path, and five table addresses hoisted out of the
    // chunk loop would hold ten scalar registers for the whole kernel.  The
    // copy is an integer, turned back into a global pointer, so that the
    // loads stay global loads, issued together.
    using GP = const __attribute__((address_space(1))) double *;
    static __device__ __forceinline__ double ld(const double *p, int j)
    {
        uint64_t a = (uint64_t)p;
        asm volatile("" : "+s"(a));
        return ((GP)a)[j];
    }
    static __device__ __forceinline__ double F(int j) { return ld(DIST == RP_NORM ? RP_ZN_F : RP_ZE_F, j); }
    static __device__ __forceinline__ double X(int j) { return ld(DIST == RP_NORM ? RP_ZN_X : RP_ZE_X, j); }
    static __device__ __forceinline__ double S(int j) { return ld(DIST == RP_NORM ? RP_ZN_S : RP_ZE_S, j); }
    static __device__ __forceinline__ double DP(int j) { return ld(DIST == RP_NORM ? RP_ZN_DP : RP_ZE_DP, j); }
    static __device__ __forceinline__ double DM(int j) { return ld(DIST == RP_NORM ? RP_ZN_DM : RP_ZE_DM, j); }
};

// INL: exp and log1p inline (no calls, so no registers saved around them).
// BX: the bitexact setting.  zflags: the FillArgs flags (the squeeze switch).
template <int DIST, bool HALF, bool INL = false, bool BX = false, class Word>
__device__ __forceinline__ int zig_resolve(const WKe *t, uint64_t w0, Word word, int avail, int zflags,
                                           bool &accepted, double &val, bool &has_u1, uint64_t &u1)
{
    const bool squeeze = !(zflags & kFlagNoSqueeze);
    auto EXP = [](double x) { return BX ? bx_exp(x) : (INL ? exp(x) : exp_ool(x)); };
    auto LOG1P = [](double x) { return BX ? bx_log1p(x) : (INL ? log1p(x) : log1p_ool(x)); };
    const int j = (int)(w0 & 0xff);
    accepted = false;
    has_u1 = false;
    if (j != 0 || DIST == RP_EXP) {
        if (avail < 1) return 0;
        const uint64_t u = word(1);
        if (j != 0) {
            double x;
            zig_fast<DIST, HALF>(t, w0, x);
            val = x;
            // the wedge test of wedge_accept, with the exp out of line
            const double ax = DIST == RP_NORM ? fabs(x) : x;
            const double U = zig_u<HALF>(u);
            using G = ZigG<DIST>;
            // every table value loaded up front: one memory round trip
            const double fj = G::F(j), fj1 = G::F(j - 1), sj = G::S(j), xj1 = G::X(j - 1);
            const double dm = G::DM(j), dp = G::DP(j);
            const double y = fj + U * (fj1 - fj);
            const double l = fj1 + sj * (ax - xj1);
            if (squeeze && y < l - dm) accepted = true;
            else if (squeeze && y > l + dp) accepted = false;
            else accepted = y < EXP(DIST == RP_NORM ? -0.5 * ax * ax : -ax);
        } else {
            val = RP_ZE_R - LOG1P(-zig_u<HALF>(u));
            accepted = true;
        }
        return 2;
    }
    // normal tail (Marsaglia 1964): pairs of uniforms until e2 + e2 > e1 e1
    for (int it = 0; it < kMaxTailIters; it++) {
        if (2 + 2 * it > avail) {
            if (1 + 2 * it <= avail) {
                has_u1 = true;
                u1 = word(1 + 2 * it);
            }
            return 0;
        }
        double tt;
        bool ok;
        if constexpr (INL) {
            const double e1 = -f_log1p<BX>(-zig_u<HALF>(word(1 + 2 * it))) / RP_ZN_R;
            const double e2 = -f_log1p<BX>(-zig_u<HALF>(word(2 + 2 * it)));
            tt = RP_ZN_R + e1;
            ok = e2 + e2 > e1 * e1;
        } else {
            ok = normal_tail_pair<HALF, BX>(word(1 + 2 * it), word(2 + 2 * it), tt);
        }
        if (ok) {
            val = ((w0 >> 8) & 1) ? -tt : tt;
            accepted = true;
            return 3 + 2 * it;
        }
    }
    return 2;  // unreachable in practice (see kMaxTailIters)
}

// A chunk's words live in LDS in stream order with two spare words after
// every eight: the generating lanes' 16-byte writes (eight consecutive words
// per lane) and the transposed reads (consecutive positions on consecutive
// lanes) then spread over the banks.
__device__ __forceinline__ int wpos(int p) { return p + 2 * (p >> 3); }

// Mask of the chunk positions [lo, hi) that fall in ballot word r
// (positions 64 r .. 64 r + 63).
__device__ __forceinline__ uint64_t range_mask(int r, int lo, int hi)
{
    const int a = lo > 64 * r ? lo - 64 * r : 0;
    const int b = hi < 64 * r + 64 ? hi - 64 * r : 64;
    if (a >= b) return 0;
    const uint64_t top = b == 64 ? ~0ull : ((1ull << b) - 1);
    return top & ~((1ull << a) - 1);
}

// The base value a derived law transforms: the binary64 draw, or for the
// binary32 laws (float draws) the binary32 value the float sampler returns
template <bool HALF>
__device__ __forceinline__ double zbase(double v)
{
    if constexpr (HALF) return (double)(float)v;
    else return v;
}

// The derived laws of rp_fill_law: one transform of one base draw (U, Z or
// E), in binary64, in the order the boundary documents, fused into the store
// of the base fill.  Law 0 is the base value itself.  Under the bitexact
// setting (xf_bx) the exp, log and pow are the correctly rounded ones.
template <int XFC>
__device__ __forceinline__ double xform(double v, const FillArgs &a)
{
    constexpr int XF = xf_law(XFC);
    constexpr bool BX = xf_bx(XFC);
    if constexpr (XF == RP_LAW_UNIF) {
        return a.xp[0] + a.xp[1] * v;  // a + (b - a) U, b - a formed on the host
    } else if constexpr (XF == RP_LAW_NORMAL) {
        return a.xp[0] + a.xp[1] * v;
    } else if constexpr (XF == RP_LAW_LOGNORMAL) {
        return f_exp<BX>(a.xp[0] + a.xp[1] * v);
    } else if constexpr (XF == RP_LAW_EXP) {
        return a.xp[0] * v;
    } else if constexpr (XF == RP_LAW_GUMBEL) {
        return a.xp[0] - a.xp[1] * f_log<BX>(-f_log<BX>(v));
    } else if constexpr (XF == RP_LAW_PARETO) {
        return a.xp[0] * f_exp<BX>(v / a.xp[1]);
    } else if constexpr (XF == RP_LAW_GPARETO) {
        const double mu = a.xp[0], sg = a.xp[1], xi = a.xp[2];
        if (xi == 0.0) return mu + sg * v;
        const double P = f_exp<BX>(v / a.xp[3]);
        if (xi > 0.0) return mu + (sg * (P - 1.0)) / xi;
        return mu - (sg * (1.0 - 1.0 / P)) / xi;
    } else if constexpr (XF == RP_LAW_WEIBULL) {
        return a.xp[1] * f_pow<BX>(v, a.xp[2]);
    } else {
        return v;
    }
}

template <class E, int DIST, int OT, int XF = 0>
__global__ __launch_bounds__(256, (DIST == RP_NORM || (DIST == RP_EXP && OT == RP_F32)) ? 5 : 1) void k_fill_wave(FillArgs a)
{
    using T = typename OutType<DIST, OT>::T;
    constexpr int R = E::R;              // words per lane per chunk
    constexpr int CHW = 64 * R;          // words per chunk
    constexpr int CHWP = CHW + CHW / 4;  // with the spare words
    constexpr bool ZIG = DIST == RP_NORM || DIST == RP_EXP;
    constexpr bool FIXED = DIST == RP_RAW || DIST == RP_U01;
    constexpr int IPW = (OT == RP_U32 || OT == RP_F32) ? 2 : 1;  // items per word
    // float ziggurat: the chunk holds 64 R 32-bit items (32 R words), and
    // every position below counts items; the state store converts back
    constexpr bool ZH = ZIG && IPW == 2;
    // raw / uniform fills in store order (engines with small blocks); the
    // others go through the LDS transpose like the ziggurat
    constexpr bool DIRECT = FIXED && E::kDirect;

    const int wib = threadIdx.x >> 6;
    const int lane = threadIdx.x & 63;
    __shared__ __align__(16) uint64_t wbuf_all[4][CHWP];
    uint64_t *const wbuf = wbuf_all[wib];
    const WKe *zt = nullptr;
    uint32_t *slot_pos = nullptr;
    uint16_t *linfo = nullptr;             // long item at a position: length | 0x8000 if it yields a value
    unsigned long long *covl = nullptr;    // per ballot word r: [2r] positions inside other samples,
                                           // [2r + 1] accepted long starts
    unsigned long long *omem = nullptr;    // per ballot word r: positions that yield a value
    uint32_t *pmem = nullptr;              //   and the values before word r
    if constexpr (ZIG) {
        __shared__ __align__(16) WKe zbuf[256];
        __shared__ uint32_t spos[4][64];
        __shared__ uint16_t linf[4][CHW];
        __shared__ __align__(16) unsigned long long cov[4][2 * R];
        __shared__ unsigned long long omv[4][R];
        __shared__ uint32_t pcv[4][R];
        for (int k = threadIdx.x; k < 256; k += blockDim.x) {
            zbuf[k].w = DIST == RP_NORM ? RP_ZN_W[k] : RP_ZE_W[k];
            zbuf[k].k = DIST == RP_NORM ? RP_ZN_K[k] : RP_ZE_K[k];
        }
        __syncthreads();
        zt = zbuf;
        slot_pos = spos[wib];
        linfo = linf[wib];
        covl = cov[wib];
        omem = omv[wib];
        pmem = pcv[wib];
    }
    const uint64_t sub = (uint64_t)__builtin_amdgcn_readfirstlane(blockIdx.x * (blockDim.x >> 6) + wib);
    if (sub >= a.n) return;
    const uint64_t P = a.per_stream;
    T *const out = (T *)a.out + sub * P;

    E eng;
    if constexpr (DIRECT) eng.load_direct(a, sub, lane);
    else if constexpr (ZH) eng.load_half(a, sub, lane);
    else eng.load(a, sub, lane);
    int e = (int)eng.phase0 * IPW;  // items of this chunk already used
    uint64_t produced = 0;
    uint64_t final_pos = 0;         // words from the start, after the last value
    bool pending = false;           // a sample that started in the previous chunk still needs words
    uint64_t pend_w = 0;            // its first word
    bool pend_hu = false;           // it holds an unused first word of a tail pair:
    uint64_t pend_u1 = 0;           //   this one
    // Each chunk yields well over half of CHW values, so this bound is never
    // reached; it only guarantees that the wavefront exits.
    const uint64_t max_chunks = 2 * (P / CHW) + 1024;
    for (uint64_t chunk = 0; chunk < max_chunks; chunk++) {
        const uint64_t base_pos = chunk * CHW;
        uint64_t w[R];
        if constexpr (DIRECT) {
            // direct order: w[j] is the word at chunk position
            // 64 G (j / G) + G lane + j % G
            eng.gen_direct(w);
        } else {
            // ---- generate R consecutive words per lane, transpose through
            //      LDS: afterwards w[r] is the word at chunk position
            //      64 r + lane ----
            if constexpr (ZH) {
                // R / 2 words per lane: items R lane .. R lane + R - 1, the
                // low half of each word first
                uint64_t g[R / 2];
                eng.gen_half(g);
#pragma unroll
                for (int k = 0; k < R / 2; k++) {
                    ulonglong2 q;
                    q.x = g[k] & 0xffffffffull;
                    q.y = g[k] >> 32;
                    *(ulonglong2 *)(wbuf + wpos(R * lane + 2 * k)) = q;
                }
            } else {
                uint64_t g[R];
                eng.gen(g);
#pragma unroll
                for (int k = 0; k < R; k += 2) {
                    ulonglong2 q;
                    q.x = g[k];
                    q.y = g[k + 1];
                    *(ulonglong2 *)(wbuf + wpos(R * lane + k)) = q;
                }
                eng.next_chunk();
            }
            wave_sync();
#pragma unroll
            for (int r = 0; r < R; r++) w[r] = wbuf[wpos(64 * r + lane)];
        }

        if constexpr (FIXED) {
            constexpr int G = DIRECT ? E::G : 1;  // after the transpose: position 64 j + lane
            const uint64_t need = P - produced;
            const uint64_t got = (uint64_t)(IPW * CHW - e);
            T *dst = out + produced - e;  // item q of the chunk goes to dst[q]
            // a whole chunk in range: unpredicated stores, which the compiler
            // merges into one 16-byte store per pair of u64 / f64 or per four
            // u32 / f32 (dword alignment suffices on gfx950)
            T v[IPW * R];
#pragma unroll
            for (int j = 0; j < R; j++) {
                if constexpr (IPW == 1) {
                    item_value<DIST, OT>(w[j], a, v[j]);
                    if constexpr (XF != 0) v[j] = xform<XF>(v[j], a);
                } else {
                    item_value<DIST, OT>(w[j] & 0xffffffffull, a, v[2 * j]);
                    item_value<DIST, OT>(w[j] >> 32, a, v[2 * j + 1]);
                    if constexpr (XF != 0) {
                        v[2 * j] = (T)xform<XF>(v[2 * j], a);
                        v[2 * j + 1] = (T)xform<XF>(v[2 * j + 1], a);
                    }
                }
            }
            // item i of this lane sits at chunk item q(i)
            auto qof = [&](int i) { return IPW * (64 * G * ((i / IPW) / G) + G * lane + (i / IPW) % G) + i % IPW; };
            if (e == 0 && need >= (uint64_t)(IPW * CHW)) {
                T *d = dst + qof(0);
#pragma unroll
                for (int i = 0; i < IPW * R; i++) d[qof(i) - qof(0)] = v[i];
            } else {
#pragma unroll
                for (int i = 0; i < IPW * R; i++) {
                    const int q = qof(i);
                    if (q >= e && (uint64_t)(q - e) < need) dst[q] = v[i];
                }
            }
            if (got >= need) {
                const uint64_t items = (uint64_t)e + need;
                final_pos = base_pos + (items + IPW - 1) / IPW;
                break;
            }
            produced += got;
            e = 0;
        } else if constexpr (!ZIG) {
            // Lemire: every item is a candidate of its own; items in stream
            // order are (r, lane, half)
            constexpr int H = IPW;
            T val[R][H];
            uint64_t okm[R][H];
#pragma unroll
            for (int r = 0; r < R; r++) {
#pragma unroll
                for (int h = 0; h < H; h++) {
                    const uint64_t it = (H == 2) ? (h ? (w[r] >> 32) : (w[r] & 0xffffffffull)) : w[r];
                    const bool ok = item_value<DIST, OT>(it, a, val[r][h]);
                    const int q = H * (64 * r + lane) + h;
                    okm[r][h] = __ballot(ok && q >= e);
                }
            }
            const uint64_t need = P - produced;
            uint64_t basec = 0;
            int endq = -1;
#pragma unroll
            for (int r = 0; r < R; r++) {
                uint32_t idx = (uint32_t)basec;
#pragma unroll
                for (int h = 0; h < H; h++) idx += mbcnt64(okm[r][h]);
#pragma unroll
                for (int h = 0; h < H; h++) {
                    if ((okm[r][h] >> lane) & 1) {
                        if (idx < need) out[produced + idx] = val[r][h];
                        if (idx == need - 1) endq = H * (64 * r + lane) + h + 1;
                        idx++;
                    }
                }
#pragma unroll
                for (int h = 0; h < H; h++) basec += (uint64_t)__popcll(okm[r][h]);
            }
            if (basec >= need) {
                const uint64_t who = __ballot(endq >= 0);
                const int src = __ffsll((long long)who) - 1;
                const int eq = __shfl(endq, src);
                final_pos = base_pos + (uint64_t)((eq + H - 1) / H);
                break;
            }
            produced += basec;
            e = 0;
        } else {
            // ---- ziggurat.  (1) A sample carried over from the previous
            //      chunk: its words are [a spare tail uniform,] then this
            //      chunk from position 0. ----
            bool whole = false;  // the carried sample uses the whole chunk
            {
                uint32_t fb = 0, lb = 0;  // per lane: bit r set if position 64 r + lane is a fast / long start
#pragma unroll
                for (int r = 0; r < R; r++) {
                    double v0;
                    const bool f = zig_fast<DIST, ZH>(zt, w[r], v0);
                    fb |= (f ? 1u : 0u) << r;
                    lb |= (f ? 0u : 1u) << r;
                }
                // keep the flags as bits of a vector register: otherwise each
                // row's compare result stays live as a scalar lane mask (two
                // scalar registers per row) until the stores
                asm volatile("" : "+v"(fb), "+v"(lb));
                // number of long items (plus the carried sample as slot 0):
                // each lane's count (<= R < 16) summed bitwise
                const int npre = pending ? 1 : 0;
                int K = npre;
                {
                    const int cnt = __popc(lb);
#pragma unroll
                    for (int bit = 0; bit < 4; bit++) K += __popcll(__ballot((cnt >> bit) & 1)) << bit;
                }
                if (lane < 2 * R) covl[lane] = 0;
                if (e > 0 && lane < R) {  // words of the chunk used before its first start
                    const uint64_t m = range_mask(lane, 0, e);
                    if (m) atomicOr(&covl[2 * lane], (unsigned long long)m);
                }
                // ---- (3) long items, 64 at a time in position order: one
                //      lane each resolves its wedge / tail test, then a scalar
                //      walk decides which of them start a sample (one inside
                //      an earlier long sample does not) ----
                int cover_end = e;
                int pend_slot = -1;
                uint64_t pw = 0, pu1 = 0;
                int phu = 0;
                // the resolving lane of a long value keeps it for the store
                int yq = -1;
                double yv = 0.0;
                uint32_t first = 0;    // values before position 0 (the carried sample's)
                for (int base = 0; base < K; base += 64) {
                    int rk0 = npre;  // slots before ballot word r
#pragma unroll
                    for (int r = 0; r < R; r++) {
                        const uint64_t lm = __ballot((lb >> r) & 1);
                        if ((lb >> r) & 1) {
                            const int rk = rk0 + (int)mbcnt64(lm) - base;
                            if (rk >= 0 && rk < 64) slot_pos[rk] = (uint32_t)(64 * r + lane);
                        }
                        rk0 += __popcll(lm);
                    }
                    if (npre && base == 0 && lane == 0) slot_pos[0] = 0xffffffffu;
                    wave_sync();
                    const int ns = K - base < 64 ? K - base : 64;
                    int q = 0, L = 0;
                    bool acc = false, hu_out = false;
                    double v = 0.0;
                    uint64_t u1o = 0, w0 = 0;
                    if (lane < ns) {
                        const uint32_t sp = slot_pos[lane];
                        const bool cp = sp == 0xffffffffu;  // the carried sample: its words are
                        const int hu = (cp && pend_hu) ? 1 : 0;  // [spare,] then position 0 on
                        q = cp ? -1 : (int)sp;
                        const int off = cp ? -1 - hu : q;
                        w0 = cp ? pend_w : wbuf[wpos(q)];
                        L = zig_resolve<DIST, ZH, false, xf_bx(XF)>(
                            zt, w0, [&](int kk) { return (hu && kk == 1) ? pend_u1 : wbuf[wpos(off + kk)]; },
                            cp ? CHW + hu : CHW - 1 - q, a.flags, acc, v, hu_out, u1o);
                    }
                    int i0 = 0;
                    if (npre && base == 0) {
                        // the carried sample decides where this chunk's first start is
                        i0 = 1;
                        const int L0 = __builtin_amdgcn_readlane(L, 0);
                        if (L0 <= 0) {
                            pend_hu = __builtin_amdgcn_readlane(hu_out ? 1 : 0, 0) != 0;
                            pend_u1 = readlane64(u1o, 0);
                            whole = true;
                            break;
                        }
                        e = L0 - 1 - (pend_hu ? 1 : 0);
                        cover_end = e;
                        pending = false;
                        if (lane < R) {
                            const uint64_t m = range_mask(lane, 0, e);
                            if (m) atomicOr(&covl[2 * lane], (unsigned long long)m);
                        }
                        if (__builtin_amdgcn_readlane(acc ? 1 : 0, 0)) {
                            first = 1;
                            if (lane == 0) {
                                yq = -2;  // stored first, before every position
                                yv = v;
                            }
                        }
                    }
                    uint64_t stm = 0;
                    for (int i = i0; i < ns; i++) {
                        const int qi = __builtin_amdgcn_readlane(q, i);
                        if (qi < cover_end) continue;
                        const int Li = __builtin_amdgcn_readlane(L, i);
                        stm |= 1ull << i;
                        if (Li <= 0) {
                            pend_slot = i;
                            cover_end = CHW;
                            break;
                        }
                        cover_end = qi + Li;
                    }
                    if (pend_slot >= 0) {
                        pw = readlane64(w0, pend_slot);
                        pu1 = readlane64(u1o, pend_slot);
                        phu = __builtin_amdgcn_readlane(hu_out ? 1 : 0, pend_slot);
                    }
                    if (lane < ns && q >= 0) {
                        const bool st = (stm >> lane) & 1;
                        const bool yields = st && L > 0 && acc;
                        if (st && L == 2) {
                            const int c = q + 1;  // c < CHW: the sample fits in the chunk
                            atomicOr(&covl[2 * (c >> 6)], 1ull << (c & 63));
                        } else if (st) {
                            const int end = L > 0 ? q + L : CHW;
#pragma unroll
                            for (int r = 0; r < R; r++) {
                                const uint64_t m = range_mask(r, q + 1, end);
                                if (m) atomicOr(&covl[2 * r], (unsigned long long)m);
                            }
                        }
                        if (yields) {
                            atomicOr(&covl[2 * (q >> 6) + 1], 1ull << (q & 63));
                            linfo[q] = (uint16_t)L;
                            yq = q;
                            yv = v;
                        }
                    }
                    wave_sync();
                    if (pend_slot >= 0) break;
                }
                if (whole) {
                    wave_sync();
                } else {
                wave_sync();
                // ---- (4) values in stream order: position p yields a value
                //      if it is a fast start not inside another sample, or a
                //      long start that was accepted.  Fast values are stored
                //      by their own lanes, one ballot word at a time; the
                //      resolving lanes store the long ones. ----
                const uint64_t need = P - produced;
                T *const dst = out + produced;
                uint32_t total = first;
                if (yq == -2) dst[0] = xform<XF>(zbase<ZH>(yv), a);  // need >= 1 here
                if (first && need == 1) {
                    final_pos = base_pos + (uint64_t)e;
                    break;
                }
                if (need >= (uint64_t)CHW + 1) {
#pragma unroll
                    for (int r = 0; r < R; r++) {
                        const ulonglong2 c = *(const ulonglong2 *)&covl[2 * r];
                        const uint64_t cv = uni64(c.x), ol = uni64(c.y);
                        const uint64_t fo = __ballot((fb >> r) & 1) & ~cv;
                        const uint64_t om = fo | ol;
                        if ((fo >> lane) & 1) {
                            // the value again from the word (cheaper than keeping R values live)
                            double v0;
                            zig_fast<DIST, ZH>(zt, wbuf[wpos(64 * r + lane)], v0);
                            dst[total + mbcnt64(om)] = xform<XF>(zbase<ZH>(v0), a);
                        }
                        if (lane == 0) {
                            omem[r] = om;
                            pmem[r] = total;
                        }
                        total += (uint32_t)__popcll(om);
                    }
                    wave_sync();
                    if (yq >= 0) {
                        const int r = yq >> 6, b = yq & 63;
                        dst[pmem[r] + (uint32_t)__popcll(omem[r] & ((1ull << b) - 1))] = xform<XF>(zbase<ZH>(yv), a);
                    }
                } else {
                    // the last chunk of this call: only need values, and the
                    // position after the last one
                    bool done = false;
#pragma unroll
                    for (int r = 0; r < R; r++) {
                        const ulonglong2 c = *(const ulonglong2 *)&covl[2 * r];
                        const uint64_t cv = uni64(c.x), ol = uni64(c.y);
                        const uint64_t fo = __ballot((fb >> r) & 1) & ~cv;
                        const uint64_t om = fo | ol;
                        if ((fo >> lane) & 1) {
                            const uint32_t idx = total + mbcnt64(om);
                            double v0;
                            zig_fast<DIST, ZH>(zt, wbuf[wpos(64 * r + lane)], v0);
                            if (idx < need) dst[idx] = xform<XF>(zbase<ZH>(v0), a);
                        }
                        if (lane == 0) {
                            omem[r] = om;
                            pmem[r] = total;
                        }
                        const uint32_t cnt = (uint32_t)__popcll(om);
                        if (!done && (uint64_t)(total + cnt) >= need) {
                            uint64_t m = om;
                            for (uint64_t k = need - 1 - total; k > 0; k--) m &= m - 1;
                            const int bit = __ffsll((long long)m) - 1;
                            const int qe = 64 * r + bit;
                            const int len = ((ol >> bit) & 1) ? (int)linfo[qe] : 1;
                            final_pos = base_pos + (uint64_t)(qe + len);
                            done = true;
                        }
                        total += cnt;
                    }
                    wave_sync();
                    if (yq >= 0) {
                        const int r = yq >> 6, b = yq & 63;
                        const uint32_t idx = pmem[r] + (uint32_t)__popcll(omem[r] & ((1ull << b) - 1));
                        if (idx < need) dst[idx] = xform<XF>(zbase<ZH>(yv), a);
                    }
                    if (done) break;
                }
                produced += (uint64_t)total;
                e = 0;
                if (pend_slot >= 0) {
                    pending = true;
                    pend_w = pw;
                    pend_hu = phu != 0;
                    pend_u1 = pu1;
                }
                }
            }
        }
        wave_sync();  // the next chunk overwrites wbuf
    }
    // float draws: a high half left over at the end of the call is dropped
    if (lane == 0) eng.store(a, sub, ZH ? (final_pos + 1) / 2 : final_pos);
}

// ---------------------------------------------------------------------------
// lane-per-substream engines (serial word streams)
// xoshiro256++ (SS = false) and xoshiro256** (SS = true): one state, two outputs
template <bool SS>
struct LaneX256T {
    X256 s;
    __device__ void load(const FillArgs &a, uint64_t i)
    {
        s = X256{a.words[i], a.words[a.n + i], a.words[2 * a.n + i], a.words[3 * a.n + i]};
    }
    __device__ uint64_t next() { return SS ? s.next_ss() : s.next(); }
    __device__ void reserve(int) {}
    __device__ void store(const FillArgs &a, uint64_t i) const
    {
        a.words[i] = s.s0;
        a.words[a.n + i] = s.s1;
        a.words[2 * a.n + i] = s.s2;
        a.words[3 * a.n + i] = s.s3;
    }
};
using LaneX256 = LaneX256T<false>;
using LaneX256SS = LaneX256T<true>;

// xoroshiro128++ and xorshift128+ (two state words each)
template <class S>
struct Lane2 {
    S s;
    __device__ void load(const FillArgs &a, uint64_t i) { s = S{a.words[i], a.words[a.n + i]}; }
    __device__ uint64_t next() { return s.next(); }
    __device__ void reserve(int) {}
    __device__ void store(const FillArgs &a, uint64_t i) const
    {
        a.words[i] = s.s0;
        a.words[a.n + i] = s.s1;
    }
};
using LaneXoro128 = Lane2<Xoro128>;
using LaneXs128 = Lane2<Xs128>;

// ChaCha20 on one lane: the current block buffered, words handed out in order
struct LaneChacha {
    uint32_t key[8], n0, n1, n2, ctr;
    uint64_t blk[8];
    int used;  // words of blk already returned (0..8)
    __device__ void start(int phase)
    {
        chacha20_block(key, n0, n1, n2, ctr, blk);
        used = phase;
    }
    __device__ void load(const FillArgs &a, uint64_t i)
    {
#pragma unroll
        for (int k = 0; k < 4; k++) {
            const uint64_t w = a.words[(uint64_t)k * a.n + i];
            key[2 * k] = (uint32_t)w;
            key[2 * k + 1] = (uint32_t)(w >> 32);
        }
        const uint64_t w4 = a.words[4 * a.n + i], w5 = a.words[5 * a.n + i];
        n0 = (uint32_t)w4;
        n1 = (uint32_t)(w4 >> 32);
        n2 = (uint32_t)w5;
        ctr = (uint32_t)(w5 >> 32);
        start((int)a.phase[i]);
    }
    __device__ uint64_t next()
    {
        if (used == 8) {
            ctr++;
            chacha20_block(key, n0, n1, n2, ctr, blk);
            used = 0;
        }
        uint64_t w = blk[0];
#pragma unroll
        for (int k = 1; k < 8; k++) w = (used == k) ? blk[k] : w;
        used++;
        return w;
    }
    __device__ void reserve(int) {}
    __device__ void store(const FillArgs &a, uint64_t i) const
    {
        const bool done = used == 8;
        a.words[5 * a.n + i] = (uint64_t)n2 | ((uint64_t)(done ? ctr + 1u : ctr) << 32);
        a.phase[i] = done ? 0u : (uint32_t)used;
    }
};

struct LaneSquares {
    uint64_t c, key;
    __device__ void load(const FillArgs &a, uint64_t i)
    {
        c = a.words[i];
        key = a.words[a.n + i];
    }
    __device__ uint64_t next() { return squares64(c++, key); }
    __device__ void reserve(int) {}
    __device__ void store(const FillArgs &a, uint64_t i) const { a.words[i] = c; }
};

struct LaneSfc64 {
    Sfc64 s;
    __device__ void load(const FillArgs &a, uint64_t i)
    {
        s = Sfc64{a.words[i], a.words[a.n + i], a.words[2 * a.n + i], a.words[3 * a.n + i]};
    }
    __device__ uint64_t next() { return s.next(); }
    __device__ void reserve(int) {}
    __device__ void store(const FillArgs &a, uint64_t i) const
    {
        a.words[i] = s.a;
        a.words[a.n + i] = s.b;
        a.words[2 * a.n + i] = s.c;
        a.words[3 * a.n + i] = s.ctr;
    }
};

// cwg128: x, a, Weyl sequence and increment, two words each
struct LaneCwg128 {
    Cwg128 g;
    __device__ void load(const FillArgs &a, uint64_t i)
    {
        const uint64_t n = a.n;
        g = Cwg128{{a.words[i], a.words[n + i]},
                   {a.words[2 * n + i], a.words[3 * n + i]},
                   {a.words[4 * n + i], a.words[5 * n + i]},
                   {a.words[6 * n + i], a.words[7 * n + i]}};
    }
    __device__ uint64_t next() { return g.next(); }
    __device__ void reserve(int) {}
    __device__ void store(const FillArgs &a, uint64_t i) const
    {
        const uint64_t n = a.n;
        a.words[i] = g.x.lo;
        a.words[n + i] = g.x.hi;
        a.words[2 * n + i] = g.a.lo;
        a.words[3 * n + i] = g.a.hi;
        a.words[4 * n + i] = g.w.lo;
        a.words[5 * n + i] = g.w.hi;
    }
};

// SIMD engines (Section 4.1): eight sub-streams per substream.  A round is one
// word of each sub-stream, in sub-stream order, formed together; the
// sub-streams move one step when the round is used.  `used` is the phase
// (words of the round already returned); the round's words are picked with a
// select chain.
template <int KIND>  // RP_X256PPS, RP_X256SSS or RP_SFC64S
struct LaneSimd {
    uint64_t s[32];   // sub-stream k at s[4 k .. 4 k + 3]
    uint64_t cur[8];  // the round formed from s
    int used;
    __device__ void round()
    {
#pragma unroll
        for (int k = 0; k < 8; k++) {
            if constexpr (KIND == RP_SFC64S) {
                cur[k] = s[4 * k] + s[4 * k + 1] + s[4 * k + 3];
            } else {
                X256 c{s[4 * k], s[4 * k + 1], s[4 * k + 2], s[4 * k + 3]};
                cur[k] = KIND == RP_X256SSS ? c.next_ss() : c.next();
            }
        }
    }
    __device__ void step()
    {
#pragma unroll
        for (int k = 0; k < 8; k++) {
            if constexpr (KIND == RP_SFC64S) {
                Sfc64 c{s[4 * k], s[4 * k + 1], s[4 * k + 2], s[4 * k + 3]};
                (void)c.next();
                s[4 * k] = c.a;
                s[4 * k + 1] = c.b;
                s[4 * k + 2] = c.c;
                s[4 * k + 3] = c.ctr;
            } else {
                X256 c{s[4 * k], s[4 * k + 1], s[4 * k + 2], s[4 * k + 3]};
                c.linear();
                s[4 * k] = c.s0;
                s[4 * k + 1] = c.s1;
                s[4 * k + 2] = c.s2;
                s[4 * k + 3] = c.s3;
            }
        }
    }
    __device__ void load(const FillArgs &a, uint64_t i)
    {
#pragma unroll
        for (int w = 0; w < 32; w++) s[w] = a.words[(uint64_t)w * a.n + i];
        used = (int)a.phase[i];
        round();
    }
    __device__ uint64_t next()
    {
        if (used == 8) {
            step();
            round();
            used = 0;
        }
        uint64_t w = cur[0];
#pragma unroll
        for (int k = 1; k < 8; k++) w = (used == k) ? cur[k] : w;
        used++;
        return w;
    }
    __device__ void reserve(int) {}
    __device__ void store(const FillArgs &a, uint64_t i)
    {
        if (used == 8) {
            step();
            used = 0;
        }
#pragma unroll
        for (int w = 0; w < 32; w++) a.words[(uint64_t)w * a.n + i] = s[w];
        a.phase[i] = (uint32_t)used;
    }
};
using LaneX256Simd = LaneSimd<RP_X256PPS>;
using LaneX256SSSimd = LaneSimd<RP_X256SSS>;
using LaneSfc64Simd = LaneSimd<RP_SFC64S>;

// Lanes of a wavefront that run serial streams drift apart in how many words
// they have used, so a per-lane "make a block when the current one is used
// up" branch would run the block computation for the whole wavefront on
// almost every word.  Block engines therefore keep a second block: when some
// lane has used both, every lane without a next block makes one, so the
// wavefront computes about one block per block's worth of words.
__device__ __forceinline__ bool wave_any(bool p) { return __ballot(p) != 0; }

// ranlux++: state (x, phase); the current block is the nine limbs of A x, of
// which `phase` words are used.  Here: cur = A xp, nxt = A cur when hn.
//
// The step is computed in two places.  reserve(k), called by the kernels at
// points every active lane reaches, gives each lane at least k words: as
// soon as one lane is short, every lane without a next block computes it
// (inline, one copy per call site), so a wavefront pays about one step per
// nine words.  next() only falls back to an out-of-line step when a caller
// took more words than it reserved (rejection loops that run long).
typedef const __attribute__((address_space(4))) uint32_t RlTab;

__device__ __forceinline__ void rl_step_inline(const uint64_t *in, uint64_t *out)
{
    // an opaque copy of the table address keeps its scalar loads here
    // instead of hoisted (and spilled) across the kernel's loops
    RlTab *B = (RlTab *)c_rl_B;
    asm volatile("" : "+s"(B));
    rl_mul_tab(in, B, out);
}

struct Rl9 {
    uint64_t w[9];
};
__device__ __noinline__ Rl9 rl_step_call(Rl9 x)
{
    Rl9 y;
    rl_step_inline(x.w, y.w);
    return y;
}

struct LaneRanlux {
    uint64_t xp[9], cur[9], nxt[9];
    int used;  // words of cur already returned (0..9)
    bool hn;   // nxt holds A cur
    __device__ void start(int phase)
    {
        Rl9 x;
#pragma unroll
        for (int k = 0; k < 9; k++) x.w[k] = xp[k];
        const Rl9 y = rl_step_call(x);
#pragma unroll
        for (int k = 0; k < 9; k++) cur[k] = y.w[k];
        used = phase;
        hn = false;
    }
    __device__ void load(const FillArgs &a, uint64_t i)
    {
#pragma unroll
        for (int k = 0; k < 9; k++) xp[k] = a.words[(uint64_t)k * a.n + i];
        start((int)a.phase[i]);
    }
    __device__ void reserve(int k)
    {
        if (wave_any(!hn && used > 9 - k)) {
            if (!hn) {
                rl_step_inline(cur, nxt);
                hn = true;
            }
        }
    }
    __device__ uint64_t next()
    {
        if (used == 9) {
            if (!hn) {
                Rl9 x;
#pragma unroll
                for (int k = 0; k < 9; k++) x.w[k] = cur[k];
                const Rl9 y = rl_step_call(x);
#pragma unroll
                for (int k = 0; k < 9; k++) nxt[k] = y.w[k];
            }
#pragma unroll
            for (int k = 0; k < 9; k++) {
                xp[k] = cur[k];
                cur[k] = nxt[k];
            }
            hn = false;
            used = 0;
        }
        uint64_t w = cur[0];
#pragma unroll
        for (int k = 1; k < 9; k++) w = (used == k) ? cur[k] : w;
        used++;
        return w;
    }
    __device__ void store(const FillArgs &a, uint64_t i) const
    {
        const bool done = used == 9;
#pragma unroll
        for (int k = 0; k < 9; k++) a.words[(uint64_t)k * a.n + i] = done ? cur[k] : xp[k];
        a.phase[i] = done ? 0u : (uint32_t)used;
    }
};

// serial ziggurat (identical decisions to the wavefront classifier)
// One serial ziggurat draw.  next() yields the next 64-bit word (binary64
// draws) or 32-bit item (float draws, HALF).
template <int DIST, bool HALF, bool BX = false, class Next>
__device__ __forceinline__ double zig_serial_g(const ZigLds *t, Next next)
{
    for (;;) {
        const uint64_t it = next();
        const uint64_t w = HALF ? item_word<DIST>(it) : it;
        const int j = (int)(w & 0xff);
        if (DIST == RP_NORM) {
            const uint64_t m = (w >> 9) & ((1ull << 52) - 1);
            const bool neg = (w >> 8) & 1;
            const WKe e = t->WK[j];
            const double x = (double)m * e.w;
            if (m < e.k) return neg ? -x : x;
            if (j == 0) {
                for (int k = 0; k < kMaxTailIters; k++) {
                    const double e1 = -f_log1p<BX>(-zig_u<HALF>(next())) / RP_ZN_R;
                    const double e2 = -f_log1p<BX>(-zig_u<HALF>(next()));
                    if (e2 + e2 > e1 * e1) {
                        const double tt = RP_ZN_R + e1;
                        return neg ? -tt : tt;
                    }
                }
                continue;  // unreachable in practice (see kMaxTailIters)
            }
            if (wedge_accept<DIST, HALF, BX>(t, j, x, next())) return neg ? -x : x;
        } else {
            const uint64_t m = (w >> 8) & ((1ull << 53) - 1);
            const WKe e = t->WK[j];
            const double x = (double)m * e.w;
            if (m < e.k) return x;
            if (j == 0) return RP_ZE_R - f_log1p<BX>(-zig_u<HALF>(next()));
            if (wedge_accept<DIST, HALF, BX>(t, j, x, next())) return x;
        }
    }
}

// the binary64 draw, written out with the engine's next() (no callable
// wrapper, so an engine's out-of-line step sees only its own live values)
template <int DIST, bool BX = false, class E>
__device__ double zig_serial(const ZigLds *t, E &eng)
{
    for (;;) {
        const uint64_t w = eng.next();
        const int j = (int)(w & 0xff);
        if (DIST == RP_NORM) {
            const uint64_t m = (w >> 9) & ((1ull << 52) - 1);
            const bool neg = (w >> 8) & 1;
            const WKe e = t->WK[j];
            const double x = (double)m * e.w;
            if (m < e.k) return neg ? -x : x;
            if (j == 0) {
                for (int k = 0; k < kMaxTailIters; k++) {
                    const double e1 = -f_log1p<BX>(-u01_53(eng.next())) / RP_ZN_R;
                    const double e2 = -f_log1p<BX>(-u01_53(eng.next()));
                    if (e2 + e2 > e1 * e1) {
                        const double tt = RP_ZN_R + e1;
                        return neg ? -tt : tt;
                    }
                }
                continue;  // unreachable in practice (see kMaxTailIters)
            }
            if (wedge_accept<DIST, false, BX>(t, j, x, eng.next())) return neg ? -x : x;
        } else {
            const uint64_t m = (w >> 8) & ((1ull << 53) - 1);
            const WKe e = t->WK[j];
            const double x = (double)m * e.w;
            if (m < e.k) return x;
            if (j == 0) return RP_ZE_R - f_log1p<BX>(-u01_53(eng.next()));
            if (wedge_accept<DIST, false, BX>(t, j, x, eng.next())) return x;
        }
    }
}

// Lane engines whose rows go through the LDS stage.  ranlux++ keeps the
// per-lane body: compiled into the staged body, its 27-word state and
// out-of-line block step took 392-552 bytes of scratch per lane (168 in the
// per-lane body) and its fills ran about 2.5 times slower.
template <class E>
struct LaneStaged {
    static constexpr bool value = true;
};
template <>
struct LaneStaged<LaneRanlux> {
    static constexpr bool value = false;
};

// One lane per substream: lane i produces the values of row i in order.
// Rows are P values apart, so per-lane stores would touch 64 lines per
// instruction; a wavefront whose 64 substreams all exist instead produces V
// values per lane per round (V = 128 bytes of output), stages them in LDS
// and writes 64 / V whole rows runs of 128 bytes per store instruction.  The
// last P mod V values of each row, and wavefronts past the last full one,
// use per-lane stores.
template <class E, int DIST, int OT, int XF = 0>
__global__ __launch_bounds__(256) void k_fill_lane(FillArgs a)
{
    using T = typename OutType<DIST, OT>::T;
    constexpr bool ZIG = DIST == RP_NORM || DIST == RP_EXP;
    constexpr bool HALF = OT == RP_U32 || OT == RP_F32;
    constexpr int V = 128 / (int)sizeof(T);  // values per lane per round
    constexpr int VP = V + 16 / (int)sizeof(T);  // padded row: 16-byte aligned, banks spread
    ZigLds *zt = nullptr;
    if constexpr (ZIG) {
        __shared__ ZigLds zbuf;
        load_zig<DIST>(&zbuf, a.flags);
        __syncthreads();
        zt = &zbuf;
    }
    __shared__ __align__(16) T stage_all[4][64 * VP];
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int lane = (int)(threadIdx.x & 63);
    const uint64_t id0 = i - (uint64_t)lane;
    if (i >= a.n) return;
    const uint64_t P = a.per_stream;
    T *out = (T *)a.out + i * P;
    if constexpr (!LaneStaged<E>::value) {
        // per-lane stores (see LaneStaged)
        E eng;
        eng.load(a, i);
        bool have = false;
        uint32_t hi = 0;
        for (uint64_t t = 0; t < P;) {
            if constexpr (ZIG && HALF) {
                eng.reserve(2);
                out[t++] = (T)xform<XF>(zbase<true>(zig_serial_g<DIST, true, xf_bx(XF)>(zt,
                                                               [&]() -> uint64_t {
                                                                   if (have) {
                                                                       have = false;
                                                                       return hi;
                                                                   }
                                                                   const uint64_t w = eng.next();
                                                                   hi = (uint32_t)(w >> 32);
                                                                   have = true;
                                                                   return w & 0xffffffffull;
                                                               })),
                                        a);
            } else if constexpr (ZIG) {
                eng.reserve(3);
                out[t++] = (T)xform<XF>(zig_serial<DIST, xf_bx(XF)>(zt, eng), a);
            } else {
                eng.reserve(1);
                uint64_t it;
                if constexpr (HALF) {
                    if (have) {
                        it = hi;
                        have = false;
                    } else {
                        const uint64_t w = eng.next();
                        it = w & 0xffffffffull;
                        hi = (uint32_t)(w >> 32);
                        have = true;
                    }
                } else {
                    it = eng.next();
                }
                T v;
                if (item_value<DIST, OT>(it, a, v)) {
                    if constexpr (XF != 0) v = xform<XF>(v, a);
                    out[t++] = v;
                }
            }
        }
        eng.store(a, i);
        return;
    } else {
        E eng;
        eng.load(a, i);
        bool have = false;
        uint32_t hi = 0;
        auto next32 = [&]() __attribute__((always_inline)) -> uint64_t {
            if (have) {
                have = false;
                return hi;
            }
            const uint64_t w = eng.next();
            hi = (uint32_t)(w >> 32);
            have = true;
            return w & 0xffffffffull;
        };
        // the next value of this lane's row
        auto produce = [&]() __attribute__((always_inline)) -> T {
            if constexpr (ZIG && HALF) {
                eng.reserve(2);
                return (T)xform<XF>(zbase<true>(zig_serial_g<DIST, true, xf_bx(XF)>(zt, next32)), a);
            } else if constexpr (ZIG) {
                eng.reserve(3);
                return (T)xform<XF>(zig_serial<DIST, xf_bx(XF)>(zt, eng), a);
            } else {
                T v;
                for (;;) {
                    eng.reserve(1);
                    uint64_t it;
                    if constexpr (HALF) it = next32();
                    else it = eng.next();
                    if (item_value<DIST, OT>(it, a, v)) break;
                }
                if constexpr (XF != 0) v = xform<XF>(v, a);
                return v;
            }
        };
        uint64_t t = 0;
        if (blockDim.x <= 256 && id0 + 64 <= a.n) {  // wave-uniform: all 64 rows exist
            T *const stage = stage_all[(threadIdx.x >> 6) & 3];
            constexpr int RPI = 64 / V;  // rows per store instruction
            for (; t + V <= P; t += V) {
#pragma unroll 1
                for (int k = 0; k < V; k++) stage[lane * VP + k] = produce();
                wave_sync();
                // instruction j: rows RPI j .. RPI j + RPI - 1, this lane's
                // row lane / V of them at element t + lane mod V
                T *p = (T *)a.out + (id0 + (uint64_t)(lane / V)) * P + t + (uint64_t)(lane % V);
                const T *q = stage + (lane / V) * VP + lane % V;
                const uint64_t step = (uint64_t)RPI * P;
#pragma unroll
                for (int j = 0; j < V; j++) {
                    *p = q[j * RPI * VP];
                    p += step;
                }
                wave_sync();
            }
        }
        for (; t < P; t++) out[t] = produce();
        eng.store(a, i);
    }
}

#include "k_zig.h"

// wavefront engines that generate in store order take k_zig for binary64
// ziggurat draws
template <bool WAVE, class E>
struct StoreOrder {
    static constexpr bool value = false;
};
template <class E>
struct StoreOrder<true, E> {
    static constexpr bool value = E::kDirect;
};

// ---------------------------------------------------------------------------
// whether a fill kernel evaluates exp, log, log1p or pow (the ziggurat's
// rare paths, or the law's transform): those have a bitexact instantiation
template <int DIST, int XF>
constexpr bool uses_elementary()
{
    return DIST == RP_NORM || DIST == RP_EXP || XF == RP_LAW_LOGNORMAL || XF == RP_LAW_GUMBEL ||
           XF == RP_LAW_PARETO || XF == RP_LAW_GPARETO || XF == RP_LAW_WEIBULL;
}

template <bool WAVE, class E, int DIST, int OT, int XF>
static int launch_kernel(const FillArgs &a, hipStream_t st)
{
    const unsigned threads = 256;
    const unsigned per_block = WAVE ? threads / 64 : threads;
    const uint64_t blocks = (a.n + per_block - 1) / per_block;
    if constexpr (StoreOrder<WAVE, E>::value && (DIST == RP_NORM || DIST == RP_EXP) && OT == RP_F64)
        hipLaunchKernelGGL((k_zig<E, DIST, XF>), dim3((unsigned)blocks), dim3(threads), 0, st, a);
    else if constexpr (WAVE)
        hipLaunchKernelGGL((k_fill_wave<E, DIST, OT, XF>), dim3((unsigned)blocks), dim3(threads), 0, st, a);
    else
        hipLaunchKernelGGL((k_fill_lane<E, DIST, OT, XF>), dim3((unsigned)blocks), dim3(threads), 0, st, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(RP_EDEVICE, "fill kernel launch: %s", hipGetErrorString(e));
    return RP_OK;
}

template <bool WAVE, class E, int DIST, int OT, int XF = 0>
static int launch_one(const FillArgs &a, hipStream_t st)
{
    if constexpr (uses_elementary<DIST, XF>())
        if (a.flags & kFlagBitexact) return launch_kernel<WAVE, E, DIST, OT, XF | kXfBx>(a, st);
    return launch_kernel<WAVE, E, DIST, OT, XF>(a, st);
}

template <bool WAVE, class E>
static int dispatch_dist(int dist, int dtype, const FillArgs &a, hipStream_t st)
{
    switch (dist) {
    case RP_RAW:
        return dtype == RP_U64 ? launch_one<WAVE, E, RP_RAW, RP_U64>(a, st)
                               : launch_one<WAVE, E, RP_RAW, RP_U32>(a, st);
    case RP_U01:
        return dtype == RP_F64 ? launch_one<WAVE, E, RP_U01, RP_F64>(a, st)
                               : launch_one<WAVE, E, RP_U01, RP_F32>(a, st);
    case RP_BOUNDED:
        return dtype == RP_U64 ? launch_one<WAVE, E, RP_BOUNDED, RP_U64>(a, st)
                               : launch_one<WAVE, E, RP_BOUNDED, RP_U32>(a, st);
    case RP_NORM:
        return dtype == RP_F64 ? launch_one<WAVE, E, RP_NORM, RP_F64>(a, st)
                               : launch_one<WAVE, E, RP_NORM, RP_F32>(a, st);
    case RP_EXP:
        return dtype == RP_F64 ? launch_one<WAVE, E, RP_EXP, RP_F64>(a, st)
                               : launch_one<WAVE, E, RP_EXP, RP_F32>(a, st);
    }
    return fail(RP_EINVAL, "unknown distribution");
}

int launch_fill(int engine, int dist, int dtype, const FillArgs &a, hipStream_t st)
{
    if (a.n > (uint64_t)UINT32_MAX * 4) return fail(RP_EINVAL, "too many substreams for one launch");
    switch (engine) {
    case RP_PHILOX4X32: return dispatch_dist<true, WavePhilox32>(dist, dtype, a, st);
    case RP_PHILOX: return dispatch_dist<true, WavePhilox64>(dist, dtype, a, st);
    case RP_PCG64: return dispatch_dist<true, WavePcg>(dist, dtype, a, st);
    case RP_X256PP: return dispatch_dist<false, LaneX256>(dist, dtype, a, st);
    case RP_X256SS: return dispatch_dist<false, LaneX256SS>(dist, dtype, a, st);
    case RP_SQUARES: return dispatch_dist<true, WaveSquares>(dist, dtype, a, st);
    case RP_CHACHA20: return dispatch_dist<true, WaveChacha>(dist, dtype, a, st);
    case RP_XORO128: return dispatch_dist<false, LaneXoro128>(dist, dtype, a, st);
    case RP_XS128: return dispatch_dist<false, LaneXs128>(dist, dtype, a, st);
    case RP_SFC64: return dispatch_dist<false, LaneSfc64>(dist, dtype, a, st);
    case RP_CWG128: return dispatch_dist<false, LaneCwg128>(dist, dtype, a, st);
    case RP_X256PPS: return dispatch_dist<false, LaneX256Simd>(dist, dtype, a, st);
    case RP_X256SSS: return dispatch_dist<false, LaneX256SSSimd>(dist, dtype, a, st);
    case RP_SFC64S: return dispatch_dist<false, LaneSfc64Simd>(dist, dtype, a, st);
    case RP_RANLUX: return dispatch_dist<false, LaneRanlux>(dist, dtype, a, st);
    }
    return fail(RP_EINVAL, "unknown engine");
}

template <bool WAVE, class E, int OT>
static int dispatch_law_t(int law, const FillArgs &a, hipStream_t st)
{
    switch (law) {
    case RP_LAW_UNIF: return launch_one<WAVE, E, RP_U01, OT, RP_LAW_UNIF>(a, st);
    case RP_LAW_NORMAL: return launch_one<WAVE, E, RP_NORM, OT, RP_LAW_NORMAL>(a, st);
    case RP_LAW_LOGNORMAL: return launch_one<WAVE, E, RP_NORM, OT, RP_LAW_LOGNORMAL>(a, st);
    case RP_LAW_EXP: return launch_one<WAVE, E, RP_EXP, OT, RP_LAW_EXP>(a, st);
    case RP_LAW_GUMBEL: return launch_one<WAVE, E, RP_U01, OT, RP_LAW_GUMBEL>(a, st);
    case RP_LAW_PARETO: return launch_one<WAVE, E, RP_EXP, OT, RP_LAW_PARETO>(a, st);
    case RP_LAW_GPARETO: return launch_one<WAVE, E, RP_EXP, OT, RP_LAW_GPARETO>(a, st);
    case RP_LAW_WEIBULL: return launch_one<WAVE, E, RP_EXP, OT, RP_LAW_WEIBULL>(a, st);
    }
    return fail(RP_EINVAL, "unknown law");
}

template <bool WAVE, class E>
static int dispatch_law(int law, bool f32, const FillArgs &a, hipStream_t st)
{
    return f32 ? dispatch_law_t<WAVE, E, RP_F32>(law, a, st) : dispatch_law_t<WAVE, E, RP_F64>(law, a, st);
}

int launch_fill_law(int engine, int law, bool f32, const FillArgs &a, hipStream_t st)
{
    if (a.n > (uint64_t)UINT32_MAX * 4) return fail(RP_EINVAL, "too many substreams for one launch");
    switch (engine) {
    case RP_PHILOX4X32: return dispatch_law<true, WavePhilox32>(law, f32, a, st);
    case RP_PHILOX: return dispatch_law<true, WavePhilox64>(law, f32, a, st);
    case RP_PCG64: return dispatch_law<true, WavePcg>(law, f32, a, st);
    case RP_X256PP: return dispatch_law<false, LaneX256>(law, f32, a, st);
    case RP_X256SS: return dispatch_law<false, LaneX256SS>(law, f32, a, st);
    case RP_SQUARES: return dispatch_law<true, WaveSquares>(law, f32, a, st);
    case RP_CHACHA20: return dispatch_law<true, WaveChacha>(law, f32, a, st);
    case RP_XORO128: return dispatch_law<false, LaneXoro128>(law, f32, a, st);
    case RP_XS128: return dispatch_law<false, LaneXs128>(law, f32, a, st);
    case RP_SFC64: return dispatch_law<false, LaneSfc64>(law, f32, a, st);
    case RP_CWG128: return dispatch_law<false, LaneCwg128>(law, f32, a, st);
    case RP_X256PPS: return dispatch_law<false, LaneX256Simd>(law, f32, a, st);
    case RP_X256SSS: return dispatch_law<false, LaneX256SSSimd>(law, f32, a, st);
    case RP_SFC64S: return dispatch_law<false, LaneSfc64Simd>(law, f32, a, st);
    case RP_RANLUX: return dispatch_law<false, LaneRanlux>(law, f32, a, st);
    }
    return fail(RP_EINVAL, "unknown engine");
}

#include "k_samplers.h"
#include "k_discrete.h"
#include "k_batched.h"
#include "k_serial.h"

}  // namespace rp
