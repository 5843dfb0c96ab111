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

namespace rp {

// ---------------------------------------------------------------------------
// constant tables uploaded once per device
struct PcgAffineDev {
    uint64_t mlo, mhi, plo, phi;
};
__constant__ PcgAffineDev c_pcg_lane[65];  // A^l, G_l for l = 0..64
__constant__ PcgAffineDev c_pcg_pow2[64];  // A^(2^k), G_(2^k)
__constant__ uint64_t c_rl_A[9];           // ranlux++ step multiplier a^2048 mod m

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
    PcgAffine cur{{1, 0}, {0, 0}};
    for (int l = 0; l <= 64; l++) {
        lane[l] = to_dev(cur);
        cur = compose(step, cur);
    }
    PcgAffine p = step;
    for (int k = 0; k < 64; k++) {
        pow2[k] = to_dev(p);
        p = compose(p, p);
    }
    e = hipMemcpyToSymbol(HIP_SYMBOL(c_pcg_lane), lane, sizeof lane);
    if (e == hipSuccess) e = hipMemcpyToSymbol(HIP_SYMBOL(c_pcg_pow2), pow2, sizeof pow2);
    if (e == hipSuccess) e = hipMemcpyToSymbol(HIP_SYMBOL(c_rl_A), ranlux_A(), 9 * 8);
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
struct ZigLds {
    double W[256];
    uint64_t K[256];
    double F[256];
    double X[256];
    double S[256];
    double DP[256];
    double DM[256];
};

template <int DIST>
__device__ __forceinline__ void load_zig(ZigLds *t)
{
    const bool nrm = DIST == RP_NORM;
    for (int k = threadIdx.x; k < 256; k += blockDim.x) {
        t->W[k] = nrm ? RP_ZN_W[k] : RP_ZE_W[k];
        t->K[k] = nrm ? RP_ZN_K[k] : RP_ZE_K[k];
        t->F[k] = nrm ? RP_ZN_F[k] : RP_ZE_F[k];
        t->X[k] = nrm ? RP_ZN_X[k] : RP_ZE_X[k];
        t->S[k] = nrm ? RP_ZN_S[k] : RP_ZE_S[k];
        t->DP[k] = nrm ? RP_ZN_DP[k] : RP_ZE_DP[k];
        t->DM[k] = nrm ? RP_ZN_DM[k] : RP_ZE_DM[k];
    }
}

// Wedge test of strip j >= 1 (Section 3.1, ziggurat figure): y drawn in
// [f_j, f_{j-1}) is accepted iff y < f(x).  The secant/tangent squeeze
// decides most cases without exp(); its bounds carry a margin far above the
// rounding of the secant and of exp, so a squeeze decision always equals the
// plain test evaluated in binary64.
template <int DIST>
__device__ __forceinline__ bool wedge_accept(const ZigLds *t, int j, double x, uint64_t uword)
{
    double U = u01_53(uword);
    double fj = t->F[j], fj1 = t->F[j - 1];
    double y = fj + U * (fj1 - fj);
    double l = fj1 + t->S[j] * (x - t->X[j - 1]);
    if (y < l - t->DM[j]) return true;
    if (y > l + t->DP[j]) return false;
    if (DIST == RP_NORM) return y < exp(-0.5 * x * x);
    return y < exp(-x);
}

// Classify a word as the first word of a sample.
//   kind 0: fast accept (1 word), 1: accept using the next word (2 words),
//   2: reject after the wedge test (2 words), 3: normal tail (resolved later)
template <int DIST>
__device__ __forceinline__ int zig_classify(const ZigLds *t, uint64_t w, uint64_t next_w, double &val)
{
    const int j = (int)(w & 0xff);
    if (DIST == RP_NORM) {
        const uint64_t m = (w >> 9) & ((1ull << 52) - 1);
        const bool neg = (w >> 8) & 1;
        const double x = (double)m * t->W[j];
        val = neg ? -x : x;
        if (m < t->K[j]) return 0;
        if (j == 0) return 3;
        return wedge_accept<DIST>(t, j, x, next_w) ? 1 : 2;
    } else {
        const uint64_t m = (w >> 8) & ((1ull << 53) - 1);
        const double x = (double)m * t->W[j];
        val = x;
        if (m < t->K[j]) return 0;
        if (j == 0) {
            val = RP_ZE_R - log1p(-u01_53(next_w));
            return 1;
        }
        return wedge_accept<DIST>(t, j, x, next_w) ? 1 : 2;
    }
}

// ---------------------------------------------------------------------------
// wavefront-per-substream engines.  Word positions are counted from the
// start of the block (or state) the substream pointed at when the call began.
struct WavePhilox32 {
    static constexpr int R = 2;  // words per lane per chunk (one block)
    uint64_t key, clo, chi, b0lo, b0hi;
    uint32_t phase0;

    __device__ void load(const FillArgs &a, uint64_t i, int lane)
    {
        b0lo = a.words[i];
        b0hi = a.words[a.n + i];
        key = a.words[2 * a.n + i];
        phase0 = a.phase[i];
        clo = b0lo + (uint64_t)lane;
        chi = b0hi + (clo < b0lo ? 1u : 0u);
    }
    __device__ void gen(uint64_t w[R]) { philox4x32(clo, chi, key, w[0], w[1]); }
    __device__ void next_chunk()
    {
        uint64_t o = clo;
        clo += 64;
        chi += (clo < o) ? 1u : 0u;
    }
    __device__ uint64_t far_word(uint64_t pos) const  // pos: words from the start
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
    static constexpr int R = 4;
    uint64_t c[4], b0[4], k0, k1;
    uint32_t phase0;

    __device__ static void add256(const uint64_t in[4], uint64_t add, uint64_t out[4])
    {
        uint64_t carry = add;
#pragma unroll
        for (int k = 0; k < 4; k++) {
            uint64_t s = in[k] + carry;
            carry = (s < carry) ? 1u : 0u;
            out[k] = s;
        }
    }
    __device__ void load(const FillArgs &a, uint64_t i, int lane)
    {
#pragma unroll
        for (int k = 0; k < 4; k++) b0[k] = a.words[(uint64_t)k * a.n + i];
        k0 = a.words[4 * a.n + i];
        k1 = a.words[5 * a.n + i];
        phase0 = a.phase[i];
        add256(b0, (uint64_t)lane, c);
    }
    __device__ void gen(uint64_t w[R]) { philox4x64(c, k0, k1, w); }
    __device__ void next_chunk() { add256(c, 64, c); }
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

struct WavePcg {
    static constexpr int R = 1;
    u128 s, inc, s0;
    uint32_t phase0;

    __device__ void load(const FillArgs &a, uint64_t i, int lane)
    {
        s0 = u128{a.words[i], a.words[a.n + i]};
        inc = u128{a.words[2 * a.n + i], a.words[3 * a.n + i]};
        phase0 = 0;
        s = pcg_apply(c_pcg_lane[lane], s0, inc);
    }
    __device__ void gen(uint64_t w[R]) { w[0] = pcg_dxsm(s); }
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

template <class E, int DIST, int OT>
__global__ __launch_bounds__(256) void k_fill_wave(FillArgs a)
{
    using T = typename OutType<DIST, OT>::T;
    constexpr int R = E::R;
    constexpr bool ZIG = DIST == RP_NORM || DIST == RP_EXP;
    constexpr bool FIXED = DIST == RP_RAW || DIST == RP_U01;
    constexpr int IPW = (OT == RP_U32 || OT == RP_F32) ? 2 : 1;  // items per word
    constexpr int RI = R * IPW;                                  // items per lane
    constexpr int CH = 64 * RI;                                  // items per chunk
    constexpr int CHW = 64 * R;                                  // words per chunk

    ZigLds *zt = nullptr;
    if constexpr (ZIG) {
        __shared__ ZigLds zbuf;
        load_zig<DIST>(&zbuf);
        __syncthreads();
        zt = &zbuf;
    }
    const int lane = threadIdx.x & 63;
    const uint64_t sub = (uint64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (sub >= a.n) return;
    const uint64_t P = a.per_stream;
    T *out = (T *)a.out + sub * P;
    const uint64_t ltmask = (1ull << lane) - 1;

    E eng;
    eng.load(a, sub, lane);
    int e = (int)eng.phase0 * IPW;  // items of chunk 0 already used
    uint64_t produced = 0;
    uint64_t cur[R], nxt[R];
    eng.gen(cur);
    if constexpr (ZIG) {
        eng.next_chunk();
        eng.gen(nxt);
    }
    uint64_t final_pos = 0;  // words from the start, after the last value
    // Every chunk yields about CH values (at least half of them for the
    // samplers here), so this bound is never reached by a correct kernel; it
    // only guarantees that the wavefront exits.
    const uint64_t max_chunks = 2 * (P / CH) + 1024;
    for (uint64_t chunk = 0; chunk < max_chunks; chunk++) {
        const uint64_t need = P - produced;
        if constexpr (FIXED) {
            // every item is a value: item q -> value produced + q - e
#pragma unroll
            for (int r = 0; r < RI; r++) {
                const int q = RI * lane + r;
                const uint64_t w = cur[r / IPW];
                const uint64_t it = (IPW == 2) ? ((r & 1) ? (w >> 32) : (w & 0xffffffffull)) : w;
                T v;
                item_value<DIST, OT>(it, a, v);
                const uint64_t idx = (uint64_t)(q - e);
                if (q >= e && idx < need) out[produced + idx] = v;
            }
            const uint64_t got = (uint64_t)(CH - e);
            if (got >= need) {
                const uint64_t items = (uint64_t)e + need;
                final_pos = chunk * CHW + (items + IPW - 1) / IPW;
                break;
            }
            produced += got;
            e = 0;
        } else {
            T val[RI];
            bool acc[RI];
            int len[RI];
            uint64_t lmask[RI], tmask[RI];
#pragma unroll
            for (int r = 0; r < RI; r++) {
                len[r] = 1;
                lmask[r] = 0;
                tmask[r] = 0;
            }
            if constexpr (ZIG) {
                // the word after item q: same lane, next lane, or next chunk
                const uint64_t up = __shfl(cur[0], (lane + 1) & 63);
                const uint64_t nx0 = __shfl(nxt[0], 0);
                const uint64_t after_last = (lane == 63) ? nx0 : up;
#pragma unroll
                for (int r = 0; r < R; r++) {
                    const uint64_t nw = (r + 1 < R) ? cur[(r + 1) % R] : after_last;
                    double v;
                    const int kind = zig_classify<DIST>(zt, cur[r], nw, v);
                    val[r] = v;
                    acc[r] = kind <= 1;
                    len[r] = kind == 0 ? 1 : 2;
                    lmask[r] = __ballot(kind != 0);
                    tmask[r] = __ballot(kind == 3);
                }
            } else {
#pragma unroll
                for (int r = 0; r < RI; r++) {
                    const uint64_t w = cur[r / IPW];
                    const uint64_t it = (IPW == 2) ? ((r & 1) ? (w >> 32) : (w & 0xffffffffull)) : w;
                    acc[r] = item_value<DIST, OT>(it, a, val[r]);
                }
            }
            // items before the entry point e belong to the previous sample
            uint64_t skip[RI];
#pragma unroll
            for (int r = 0; r < RI; r++) {
                const int lim = (e - r + RI - 1) / RI;  // lanes l with RI l + r < e
                skip[r] = lim <= 0 ? 0ull : (lim >= 64 ? ~0ull : ((1ull << lim) - 1));
            }
            int c = e;  // next sample start (relative to this chunk)
            if constexpr (ZIG) {
                uint64_t cand = 0;
#pragma unroll
                for (int r = 0; r < R; r++) cand |= lmask[r];
                while (cand) {
                    const int l = __ffsll((long long)cand) - 1;
                    cand &= cand - 1;
#pragma unroll
                    for (int r = 0; r < R; r++) {
                        if (!((lmask[r] >> l) & 1)) continue;
                        const int q = R * l + r;
                        if (q < c) continue;  // used by an earlier sample
                        int L = 2;
                        if constexpr (DIST == RP_NORM) {
                            if ((tmask[r] >> l) & 1) {
                                // Marsaglia's tail: pairs of uniforms from the
                                // words after q until e2 + e2 > e1 e1
                                const uint64_t w0 = readlane64(cur[r], l);
                                auto word_at = [&](int p) -> uint64_t {
                                    if (p < CHW) {
                                        uint64_t v = cur[0];
#pragma unroll
                                        for (int rr = 1; rr < R; rr++) v = (p % R == rr) ? cur[rr] : v;
                                        return readlane64(v, p / R);
                                    }
                                    if (p < 2 * CHW) {
                                        const int pp = p - CHW;
                                        uint64_t v = nxt[0];
#pragma unroll
                                        for (int rr = 1; rr < R; rr++) v = (pp % R == rr) ? nxt[rr] : v;
                                        return readlane64(v, pp / R);
                                    }
                                    return eng.far_word(chunk * CHW + (uint64_t)p);
                                };
                                double tv = 0.0;
                                for (int it = 0; it < kMaxTailIters; it++) {
                                    const double U1 = u01_53(word_at(q + 1 + 2 * it));
                                    const double U2 = u01_53(word_at(q + 2 + 2 * it));
                                    const double e1 = -log1p(-U1) / RP_ZN_R;
                                    const double e2 = -log1p(-U2);
                                    if (e2 + e2 > e1 * e1) {
                                        const double tt = RP_ZN_R + e1;
                                        tv = ((w0 >> 8) & 1) ? -tt : tt;
                                        L = 3 + 2 * it;
                                        break;
                                    }
                                }
                                if (lane == l) {
                                    val[r] = tv;
                                    acc[r] = true;
                                    len[r] = L;
                                }
                            }
                        }
                        c = q + L;
                        for (int p = q + 1; p < c && p < CH; p++) {
#pragma unroll
                            for (int rr = 0; rr < R; rr++)
                                if (p % R == rr) skip[rr] |= 1ull << (p / R);
                        }
                    }
                }
            }
            // compaction: prefix count of accepted starts in stream order
            bool outp[RI];
            uint64_t bal[RI];
            uint64_t before = 0, total = 0;
#pragma unroll
            for (int r = 0; r < RI; r++) {
                outp[r] = acc[r] && !((skip[r] >> lane) & 1);
                bal[r] = __ballot(outp[r]);
                before += (uint64_t)__popcll(bal[r] & ltmask);
                total += (uint64_t)__popcll(bal[r]);
            }
            uint64_t idx = before;
            int endp = -1;
#pragma unroll
            for (int r = 0; r < RI; r++) {
                if (outp[r]) {
                    if (idx < need) out[produced + idx] = val[r];
                    if (idx == need - 1) endp = RI * lane + r + len[r];
                    idx++;
                }
            }
            if (total >= need) {
                const uint64_t who = __ballot(endp >= 0);
                const int src = __ffsll((long long)who) - 1;
                const int endq = __shfl(endp, src);
                final_pos = chunk * CHW + (uint64_t)((endq + IPW - 1) / IPW);
                break;
            }
            produced += total;
            if constexpr (ZIG) e = c > CH ? c - CH : 0;
            else e = 0;
        }
        if constexpr (ZIG) {
#pragma unroll
            for (int r = 0; r < R; r++) cur[r] = nxt[r];
            eng.next_chunk();
            eng.gen(nxt);
        } else {
            eng.next_chunk();
            eng.gen(cur);
        }
    }
    if (lane == 0) eng.store(a, sub, final_pos);
}

// ---------------------------------------------------------------------------
// lane-per-substream engines (serial word streams)
struct LaneX256 {
    X256 s;
    __device__ void load(const FillArgs &a, uint64_t i)
    {
        s = X256{a.words[i], a.words[a.n + i], a.words[2 * a.n + i], a.words[3 * a.n + i]};
    }
    __device__ uint64_t next() { return s.next(); }
    __device__ void store(const FillArgs &a, uint64_t i) const
    {
        a.words[i] = s.s0;
        a.words[a.n + i] = s.s1;
        a.words[2 * a.n + i] = s.s2;
        a.words[3 * a.n + i] = s.s3;
    }
};

struct LaneSfc64 {
    Sfc64 s;
    __device__ void load(const FillArgs &a, uint64_t i)
    {
        s = Sfc64{a.words[i], a.words[a.n + i], a.words[2 * a.n + i], a.words[3 * a.n + i]};
    }
    __device__ uint64_t next() { return s.next(); }
    __device__ void store(const FillArgs &a, uint64_t i) const
    {
        a.words[i] = s.a;
        a.words[a.n + i] = s.b;
        a.words[2 * a.n + i] = s.c;
        a.words[3 * a.n + i] = s.ctr;
    }
};

// ranlux++: state (x, phase); the current block is the nine limbs of y = A x,
// of which `phase` words are used.  When the block is used up, x <- y.
struct LaneRanlux {
    uint64_t x[9], y[9];
    int used;     // words of y already returned (0..9)
    bool have;    // y holds A x
    __device__ void load(const FillArgs &a, uint64_t i)
    {
#pragma unroll
        for (int k = 0; k < 9; k++) x[k] = a.words[(uint64_t)k * a.n + i];
        used = (int)a.phase[i];
        have = false;
    }
    __device__ uint64_t next()
    {
        if (!have) {
            uint64_t A[9];
#pragma unroll
            for (int k = 0; k < 9; k++) A[k] = c_rl_A[k];
            rl_mulmod(x, A, y);
            have = true;
        }
        uint64_t w = y[0];
#pragma unroll
        for (int k = 1; k < 9; k++) w = (used == k) ? y[k] : w;
        if (++used == 9) {
#pragma unroll
            for (int k = 0; k < 9; k++) x[k] = y[k];
            used = 0;
            have = false;
        }
        return w;
    }
    __device__ void store(const FillArgs &a, uint64_t i) const
    {
#pragma unroll
        for (int k = 0; k < 9; k++) a.words[(uint64_t)k * a.n + i] = x[k];
        a.phase[i] = (uint32_t)used;
    }
};

// serial ziggurat (identical decisions to the wavefront classifier)
template <int DIST, class E>
__device__ double zig_serial(const ZigLds *t, E &eng)
{
    for (;;) {
        const uint64_t w = eng.next();
        const int j = (int)(w & 0xff);
        if (DIST == RP_NORM) {
            const uint64_t m = (w >> 9) & ((1ull << 52) - 1);
            const bool neg = (w >> 8) & 1;
            const double x = (double)m * t->W[j];
            if (m < t->K[j]) return neg ? -x : x;
            if (j == 0) {
                for (int it = 0; it < kMaxTailIters; it++) {
                    const double e1 = -log1p(-u01_53(eng.next())) / RP_ZN_R;
                    const double e2 = -log1p(-u01_53(eng.next()));
                    if (e2 + e2 > e1 * e1) {
                        const double tt = RP_ZN_R + e1;
                        return neg ? -tt : tt;
                    }
                }
                continue;  // unreachable in practice (see kMaxTailIters)
            }
            if (wedge_accept<DIST>(t, j, x, eng.next())) return neg ? -x : x;
        } else {
            const uint64_t m = (w >> 8) & ((1ull << 53) - 1);
            const double x = (double)m * t->W[j];
            if (m < t->K[j]) return x;
            if (j == 0) return RP_ZE_R - log1p(-u01_53(eng.next()));
            if (wedge_accept<DIST>(t, j, x, eng.next())) return x;
        }
    }
}

template <class E, int DIST, int OT>
__global__ __launch_bounds__(256) void k_fill_lane(FillArgs a)
{
    using T = typename OutType<DIST, OT>::T;
    constexpr bool ZIG = DIST == RP_NORM || DIST == RP_EXP;
    constexpr bool HALF = OT == RP_U32 || OT == RP_F32;
    ZigLds *zt = nullptr;
    if constexpr (ZIG) {
        __shared__ ZigLds zbuf;
        load_zig<DIST>(&zbuf);
        __syncthreads();
        zt = &zbuf;
    }
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.n) return;
    const uint64_t P = a.per_stream;
    T *out = (T *)a.out + i * P;
    E eng;
    eng.load(a, i);
    bool have = false;
    uint32_t hi = 0;
    for (uint64_t t = 0; t < P;) {
        if constexpr (ZIG) {
            out[t++] = zig_serial<DIST>(zt, eng);
        } else {
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
            if (item_value<DIST, OT>(it, a, v)) out[t++] = v;
        }
    }
    eng.store(a, i);
}

// ---------------------------------------------------------------------------
template <bool WAVE, class E, int DIST, int OT>
static int launch_one(const FillArgs &a, hipStream_t st)
{
    const unsigned threads = 256;
    const unsigned per_block = WAVE ? threads / 64 : threads;
    const uint64_t blocks = (a.n + per_block - 1) / per_block;
    if constexpr (WAVE)
        hipLaunchKernelGGL((k_fill_wave<E, DIST, OT>), dim3((unsigned)blocks), dim3(threads), 0, st, a);
    else
        hipLaunchKernelGGL((k_fill_lane<E, DIST, OT>), dim3((unsigned)blocks), dim3(threads), 0, st, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(RP_EDEVICE, "fill kernel launch: %s", hipGetErrorString(e));
    return RP_OK;
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
        return launch_one<WAVE, E, RP_NORM, RP_F64>(a, st);
    case RP_EXP:
        return launch_one<WAVE, E, RP_EXP, RP_F64>(a, st);
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
    case RP_SFC64: return dispatch_dist<false, LaneSfc64>(dist, dtype, a, st);
    case RP_RANLUX: return dispatch_dist<false, LaneRanlux>(dist, dtype, a, st);
    }
    return fail(RP_EINVAL, "unknown engine");
}

}  // namespace rp
