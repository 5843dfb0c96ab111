// k_serial.h -- one stream split over many lanes by jump-ahead, with the
// output order equal to the serial definition (Section 4.4: jumps through
// the characteristic polynomial for the xor family; counter and LCG
// advances for the others).  Included by fill.hip after k_batched.h.
//
// Lane l starts at word l C of the stream.  Outputs that take a fixed number
// of words (raw bits, uniforms, unbounded integers) go straight to their
// place.  For rejection samplers (ziggurat, bounded integers) the lanes first
// store the words; the serial order is then recovered in three steps:
//   k_ser_map     for each chunk of kS units and each entry offset e < kE
//                 (where the first attempt of the chunk starts), the exit
//                 offset into the next chunk and the number of accepted
//                 samples; an inclusive scan composes these maps in a block
//   k_ser_blocks  one block composes the block maps from entry 0
//   k_ser_emit    each chunk walks its attempts from its true entry and
//                 writes its samples at their serial positions
// An entry or exit of kE or more units (a normal tail spilling far into the
// next chunk) cannot be composed; it is flagged and the caller falls back to
// the one-lane serial fill.

namespace ser {
constexpr int kS = 32;          // units per chunk
constexpr int kE = 8;           // entry offsets tracked per chunk
constexpr int kBlk = 256;       // chunks per block
constexpr uint8_t kOver = 0xff; // entry/exit of kE or more
}  // namespace ser

int serial_chunk_units() { return ser::kS; }
int serial_entries() { return ser::kE; }
int serial_chunks_per_block() { return ser::kBlk; }

// ---------------------------------------------------------------------------
// generator lanes: start state of lane `id` = base advanced by id * C words
template <int ENG>
struct SerLane;

// xoshiro256++ and xoshiro256** (one linear core): the wave's base by the
// jump polynomials x^(64 C 2^k) for the set bits k of the wave index
// (uniform in the wave), then lane l applies x^(l C) mod P.  All lanes of a wave share one orbit T^i b, i < 256, and
// each accumulates the terms its own polynomial selects.
template <bool SS>
struct SerLaneX256 : LaneX256T<SS> {
    __device__ static X256 jump(X256 cur, uint64_t q0, uint64_t q1, uint64_t q2, uint64_t q3)
    {
        uint64_t a0 = 0, a1 = 0, a2 = 0, a3 = 0;
        for (int k = 0; k < 256; k++) {
            const uint64_t q = k < 64 ? q0 : k < 128 ? q1 : k < 192 ? q2 : q3;
            const uint64_t m = 0 - ((q >> (k & 63)) & 1);
            a0 ^= cur.s0 & m;
            a1 ^= cur.s1 & m;
            a2 ^= cur.s2 & m;
            a3 ^= cur.s3 & m;
            cur.linear();
        }
        return X256{a0, a1, a2, a3};
    }
    __device__ void init(const SerialArgs &a, uint64_t id)
    {
        X256 b{a.base[0], a.base[1], a.base[2], a.base[3]};
        const uint64_t w = id >> 6;
        for (int k = 0; k < 12; k++)
            if ((w >> k) & 1) {
                const uint64_t *q = &a.jt[256 + 4 * k];
                b = jump(b, q[0], q[1], q[2], q[3]);
            }
        const uint64_t *q = &a.jt[4 * (id & 63)];
        this->s = jump(b, q[0], q[1], q[2], q[3]);
    }
};

template <>
struct SerLane<RP_X256PP> : SerLaneX256<false> {};
template <>
struct SerLane<RP_X256SS> : SerLaneX256<true> {};

// PCG64: affine maps (A^(C 2^k), G_(C 2^k)) for the set bits of the lane id.
template <>
struct SerLane<RP_PCG64> : LanePcg {
    __device__ void init(const SerialArgs &a, uint64_t id)
    {
        s = u128{a.base[0], a.base[1]};
        inc = u128{a.base[2], a.base[3]};
        for (int k = 0; k < 18; k++)
            if ((id >> k) & 1) {
                const uint64_t *m = &a.jt[4 * k];
                s = add128(mul128(u128{m[0], m[1]}, s), mul128(u128{m[2], m[3]}, inc));
            }
    }
};

// Philox: counter plus id C / (words per block); the phase is unchanged.
template <>
struct SerLane<RP_PHILOX4X32> : LanePhilox32 {
    __device__ void init(const SerialArgs &a, uint64_t id)
    {
        const uint64_t add = id * (a.C / 2);
        const uint64_t lo = a.base[0] + add;
        start(lo, a.base[1] + (lo < add ? 1u : 0u), a.base[2], a.phase);
    }
};

template <>
struct SerLane<RP_PHILOX> : LanePhilox64 {
    __device__ void init(const SerialArgs &a, uint64_t id)
    {
        uint64_t add = id * (a.C / 4), carry = 0;
#pragma unroll
        for (int k = 0; k < 4; k++) {
            const uint64_t s1 = a.base[k] + add;
            const uint64_t c1 = s1 < add ? 1u : 0u;
            const uint64_t s2 = s1 + carry;
            carry = c1 + (s2 < s1 ? 1u : 0u);
            c[k] = s2;
            add = 0;
        }
        k0 = a.base[4];
        k1 = a.base[5];
        start(a.phase);
    }
};

// ChaCha20: block counter plus id C / 8 (mod 2^32); the phase is unchanged.
template <>
struct SerLane<RP_CHACHA20> : LaneChacha {
    __device__ void init(const SerialArgs &a, uint64_t id)
    {
#pragma unroll
        for (int k = 0; k < 4; k++) {
            key[2 * k] = (uint32_t)a.base[k];
            key[2 * k + 1] = (uint32_t)(a.base[k] >> 32);
        }
        n0 = (uint32_t)a.base[4];
        n1 = (uint32_t)(a.base[4] >> 32);
        n2 = (uint32_t)a.base[5];
        ctr = (uint32_t)(a.base[5] >> 32) + (uint32_t)(id * (a.C / 8));
        start((int)a.phase);
    }
};

// squares64: counter plus id C.
template <>
struct SerLane<RP_SQUARES> : LaneSquares {
    __device__ void init(const SerialArgs &a, uint64_t id)
    {
        c = a.base[0] + id * a.C;
        key = a.base[1];
    }
};

// ranlux++: x times A^((C/9) 2^k) mod m for the set bits of the lane id.
template <>
struct SerLane<RP_RANLUX> : LaneRanlux {
    __device__ void init(const SerialArgs &a, uint64_t id)
    {
#pragma unroll
        for (int k = 0; k < 9; k++) xp[k] = a.base[k];
        for (int k = 0; k < 18; k++)
            if ((id >> k) & 1) {
                uint64_t m[9];
#pragma unroll
                for (int t = 0; t < 9; t++) m[t] = a.jt[9 * k + t];
                rl_mulmod(xp, m, xp);
            }
        start((int)a.phase);
    }
};

// Fixed consumption: word w gives output w (or outputs 2w, 2w+1 from its
// halves, low half first); outputs at or past n are not written.
template <int ENG, int DIST, int OT, bool FIXED>
__global__ __launch_bounds__(256) void k_ser_gen(SerialArgs a)
{
    using T = typename OutType<DIST, OT>::T;
    constexpr bool HALF = OT == RP_U32 || OT == RP_F32;
    const uint64_t id = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    SerLane<ENG> g;
    g.init(a, id);  // every lane of the wave takes part (shared orbit)
    if (id >= a.lanes) return;
    const uint64_t w0 = id * a.C;
    uint64_t w1 = w0 + a.C;
    if (w1 > a.words) w1 = a.words;
    T *out = (T *)a.fa.out;
    uint64_t w = w0;
    if constexpr (!HALF) {
        // Wavefront-cooperative runs.  A lane's chunk is contiguous in the
        // output, so per-lane stores touch 64 cache lines per instruction and
        // leave lines half written.  When every lane of the wavefront has a
        // whole chunk of C words inside the output, each lane stages its next
        // 16 values in LDS and the wavefront writes them as 4 runs of 16
        // consecutive values (4 whole 128-byte lines) per store instruction.
        constexpr int kRow = 18;  // 16 values + padding, 16-byte aligned rows
        __shared__ __align__(16) uint64_t stage_all[4][64 * kRow];
        uint64_t *const stage = stage_all[(threadIdx.x >> 6) & 3];
        const int lane = (int)(threadIdx.x & 63);
        const uint64_t id0 = id - (uint64_t)lane;
        const uint64_t lim = FIXED ? (a.words < a.n ? a.words : a.n) : a.words;
        if (blockDim.x <= 256 && id0 + 64 <= (uint64_t)a.lanes && (id0 + 64) * a.C <= lim) {
            uint64_t *const dst = FIXED ? (uint64_t *)out : a.wbuf;
            const uint64_t nrun = a.C / 16;
            for (uint64_t it = 0; it < nrun; it++) {
                uint64_t v[16];
#pragma unroll
                for (int k = 0; k < 16; k++) {
                    if (k % 8 == 0) g.reserve(8);
                    const uint64_t word = g.next();
                    if constexpr (FIXED) {
                        T t;
                        item_value<DIST, OT>(word, a.fa, t);
                        v[k] = __builtin_bit_cast(uint64_t, t);
                    } else {
                        v[k] = word;
                    }
                }
#pragma unroll
                for (int k = 0; k < 16; k += 2) {
                    ulonglong2 q;
                    q.x = v[k];
                    q.y = v[k + 1];
                    *(ulonglong2 *)(stage + lane * kRow + k) = q;
                }
                wave_sync();
                const int e = lane & 15;
#pragma unroll
                for (int k = 0; k < 16; k++) {
                    const int r = 4 * k + (lane >> 4);
                    dst[(id0 + (uint64_t)r) * a.C + it * 16 + (uint64_t)e] = stage[r * kRow + e];
                }
                wave_sync();
            }
            w = w0 + nrun * 16;
        }
    }
    if constexpr (FIXED && !HALF) {
        // whole 128-byte runs (16 values) per store burst where they fit
        if ((((uintptr_t)(out + w)) & 15) == 0) {
            for (; w + 16 <= w1 && w + 16 <= a.n; w += 16) {
                T v[16];
#pragma unroll
                for (int k = 0; k < 16; k++) {
                    if (k % 8 == 0) g.reserve(8);
                    item_value<DIST, OT>(g.next(), a.fa, v[k]);
                }
#pragma unroll
                for (int k = 0; k < 16; k += 2) {
                    ulonglong2 q;
                    q.x = __builtin_bit_cast(uint64_t, v[k]);
                    q.y = __builtin_bit_cast(uint64_t, v[k + 1]);
                    *(ulonglong2 *)(out + w + k) = q;
                }
            }
        }
    }
    for (; w < w1; w++) {
        g.reserve(1);
        const uint64_t word = g.next();
        if constexpr (!FIXED) {
            a.wbuf[w] = word;
        } else if constexpr (HALF) {
            T v;
            item_value<DIST, OT>(word & 0xffffffffull, a.fa, v);
            if (2 * w < a.n) out[2 * w] = v;
            item_value<DIST, OT>(word >> 32, a.fa, v);
            if (2 * w + 1 < a.n) out[2 * w + 1] = v;
        } else {
            T v;
            item_value<DIST, OT>(word, a.fa, v);
            if (w < a.n) out[w] = v;
        }
    }
}

// ---------------------------------------------------------------------------
// One attempt starting at unit P: its length in units, whether it yields a
// sample, and the sample.  The decisions are those of the serial ziggurat
// (zig_serial; the float ziggurat on 32-bit items for binary32 output) and
// of Lemire's method.
template <int DIST, int OT, bool BX = false>
__device__ __forceinline__ uint32_t ser_attempt(const SerialArgs &a, const ZigLds *zt, uint64_t P, bool &acc,
                                                typename OutType<DIST, OT>::T &val)
{
    constexpr bool HALF = OT == RP_U32 || OT == RP_F32;
    if constexpr (DIST == RP_BOUNDED) {
        const uint64_t it = HALF ? ((a.wbuf[P >> 1] >> (32 * (P & 1))) & 0xffffffffull) : a.wbuf[P];
        acc = item_value<DIST, OT>(it, a.fa, val);
        return 1;
    } else {
        // unit q: a word, or (float draws) the 32-bit item q of the word stream
        auto unit = [&](uint64_t q) -> uint64_t {
            if constexpr (HALF) return (a.wbuf[q >> 1] >> (32 * (q & 1))) & 0xffffffffull;
            else return a.wbuf[q];
        };
        const uint64_t w = HALF ? item_word<DIST>(unit(P)) : unit(P);
        const int j = (int)(w & 0xff);
        if constexpr (DIST == RP_NORM) {
            const uint64_t m = (w >> 9) & ((1ull << 52) - 1);
            const bool neg = (w >> 8) & 1;
            const WKe e = zt->WK[j];
            const double x = (double)m * e.w;
            if (m < e.k) {
                acc = true;
                val = (typename OutType<DIST, OT>::T)(neg ? -x : x);
                return 1;
            }
            if (j == 0) {
                for (int it = 0; it < kMaxTailIters; it++) {
                    const double e1 = -f_log1p<BX>(-zig_u<HALF>(unit(P + 1 + 2 * it))) / RP_ZN_R;
                    const double e2 = -f_log1p<BX>(-zig_u<HALF>(unit(P + 2 + 2 * it)));
                    if (e2 + e2 > e1 * e1) {
                        const double t = RP_ZN_R + e1;
                        acc = true;
                        val = (typename OutType<DIST, OT>::T)(neg ? -t : t);
                        return 1 + 2 * (it + 1);
                    }
                }
                acc = false;
                return 1 + 2 * kMaxTailIters;
            }
            acc = wedge_accept<DIST, HALF, BX>(zt, j, x, unit(P + 1));
            val = (typename OutType<DIST, OT>::T)(neg ? -x : x);
            return 2;
        } else {
            const uint64_t m = (w >> 8) & ((1ull << 53) - 1);
            const WKe e = zt->WK[j];
            const double x = (double)m * e.w;
            if (m < e.k) {
                acc = true;
                val = (typename OutType<DIST, OT>::T)x;
                return 1;
            }
            if (j == 0) {
                acc = true;
                val = (typename OutType<DIST, OT>::T)(RP_ZE_R - f_log1p<BX>(-zig_u<HALF>(unit(P + 1))));
                return 2;
            }
            acc = wedge_accept<DIST, HALF, BX>(zt, j, x, unit(P + 1));
            val = (typename OutType<DIST, OT>::T)x;
            return 2;
        }
    }
}

struct SerMap {
    uint8_t ex[ser::kE];
    uint32_t ct[ser::kE];
};

// a then b (entries index a)
__device__ __forceinline__ void ser_compose(const SerMap &a, const SerMap &b, SerMap &o)
{
#pragma unroll
    for (int e = 0; e < ser::kE; e++) {
        const uint8_t x = a.ex[e];
        if (x >= ser::kE) {
            o.ex[e] = ser::kOver;
            o.ct[e] = 0;
        } else {
            o.ex[e] = b.ex[x];
            o.ct[e] = a.ct[e] + b.ct[x];
        }
    }
}

__device__ __forceinline__ void ser_identity(SerMap &m)
{
#pragma unroll
    for (int e = 0; e < ser::kE; e++) {
        m.ex[e] = (uint8_t)e;
        m.ct[e] = 0;
    }
}

// Inclusive scan of the block's maps (one per thread) in LDS; on return
// buf[t] holds the inclusive result of thread t.
__device__ __forceinline__ void ser_block_scan(SerMap *buf, SerMap &cur)
{
    const int t = threadIdx.x;
    buf[t] = cur;
    __syncthreads();
    for (int off = 1; off < (int)blockDim.x; off <<= 1) {
        SerMap nxt = buf[t];
        if (t >= off) ser_compose(buf[t - off], buf[t], nxt);
        __syncthreads();
        buf[t] = nxt;
        __syncthreads();
    }
    cur = buf[t];
}

template <int DIST, int OT, bool BX = false>
__global__ __launch_bounds__(ser::kBlk) void k_ser_map(SerialArgs a)
{
    constexpr bool ZIG = DIST == RP_NORM || DIST == RP_EXP;
    __shared__ ZigLds zt;
    __shared__ uint16_t lens[ser::kBlk][ser::kS];
    __shared__ SerMap buf[ser::kBlk];
    if constexpr (ZIG) load_zig<DIST>(&zt, a.fa.flags);
    __syncthreads();
    const int t = threadIdx.x;
    const uint64_t c = (uint64_t)blockIdx.x * ser::kBlk + t;
    SerMap m;
    ser_identity(m);
    if (c < a.nchunks) {
        const uint64_t c0 = c * ser::kS;
        const int seff = (int)((a.units - c0) < (uint64_t)ser::kS ? (a.units - c0) : (uint64_t)ser::kS);
        for (int p = 0; p < seff; p++) {
            bool acc;
            typename OutType<DIST, OT>::T v;
            const uint32_t len = ser_attempt<DIST, OT, BX>(a, &zt, c0 + p, acc, v);
            lens[t][p] = (uint16_t)(len | (acc ? 0x8000u : 0u));
        }
#pragma unroll
        for (int e = 0; e < ser::kE; e++) {
            int pos = e;
            uint32_t cnt = 0;
            while (pos < seff) {
                const uint32_t l = lens[t][pos];
                cnt += l >> 15;
                pos += (int)(l & 0x7fff);
            }
            const int ex = pos - seff;
            m.ex[e] = ex < ser::kE ? (uint8_t)ex : ser::kOver;
            m.ct[e] = cnt;
        }
    }
    ser_block_scan(buf, m);
    SerMap ex;
    if (t == 0) ser_identity(ex);
    else ex = buf[t - 1];
    if (c < a.nchunks) {
#pragma unroll
        for (int e = 0; e < ser::kE; e++) {
            a.cexit[c * ser::kE + e] = ex.ex[e];
            a.ccount[c * ser::kE + e] = ex.ct[e];
        }
    }
    if (t == ser::kBlk - 1) {
#pragma unroll
        for (int e = 0; e < ser::kE; e++) {
            a.bexit[(uint64_t)blockIdx.x * ser::kE + e] = m.ex[e];
            a.bcount[(uint64_t)blockIdx.x * ser::kE + e] = m.ct[e];
        }
    }
}

// One block of 1024 threads walks the block maps from entry 0, 1024 at a time.
__global__ __launch_bounds__(1024) void k_ser_blocks(SerialArgs a)
{
    __shared__ SerMap buf[1024];
    const int t = threadIdx.x;
    uint32_t ce = 0;   // entry of the next block (kOver once lost)
    uint64_t cb = 0;   // outputs before it
    for (uint64_t s0 = 0; s0 < a.nblocks; s0 += 1024) {
        const uint64_t i = s0 + t;
        SerMap m;
        if (i < a.nblocks) {
#pragma unroll
            for (int e = 0; e < ser::kE; e++) {
                m.ex[e] = a.bexit[i * ser::kE + e];
                m.ct[e] = a.bcount[i * ser::kE + e];
            }
        } else {
            ser_identity(m);
        }
        ser_block_scan(buf, m);
        // exclusive prefix of block i applied to the running entry (read in LDS)
        if (i < a.nblocks) {
            if (ce < (uint32_t)ser::kE) {
                a.bentry[i] = t == 0 ? (uint8_t)ce : buf[t - 1].ex[ce];
                a.bbase[i] = cb + (t == 0 ? 0u : buf[t - 1].ct[ce]);
            } else {
                a.bentry[i] = ser::kOver;
                a.bbase[i] = 0;
            }
        }
        uint32_t nce = ce;
        uint64_t ncb = cb;
        if (ce < (uint32_t)ser::kE) {
            ncb = cb + buf[1023].ct[ce];
            nce = buf[1023].ex[ce];
        }
        __syncthreads();
        ce = nce;
        cb = ncb;
    }
    if (t == 0) {
        a.result[0] = a.units + (ce < (uint32_t)ser::kE ? ce : 0);
        a.result[1] = cb;
        a.result[2] = ce < (uint32_t)ser::kE ? 0 : 1;
    }
}

template <int DIST, int OT, bool BX = false>
__global__ __launch_bounds__(ser::kBlk) void k_ser_emit(SerialArgs a)
{
    constexpr bool ZIG = DIST == RP_NORM || DIST == RP_EXP;
    using T = typename OutType<DIST, OT>::T;
    __shared__ ZigLds zt;
    if constexpr (ZIG) load_zig<DIST>(&zt, a.fa.flags);
    __syncthreads();
    const uint64_t c = (uint64_t)blockIdx.x * ser::kBlk + threadIdx.x;
    if (c >= a.nchunks) return;
    const uint8_t be = a.bentry[blockIdx.x];
    if (be >= ser::kE) {
        a.result[2] = 1;
        return;
    }
    const uint8_t e = a.cexit[c * ser::kE + be];
    if (e >= ser::kE) {
        a.result[2] = 1;
        return;
    }
    uint64_t base = a.bbase[blockIdx.x] + a.ccount[c * ser::kE + be];
    if (base >= a.n) return;
    const uint64_t c0 = c * ser::kS;
    const int seff = (int)((a.units - c0) < (uint64_t)ser::kS ? (a.units - c0) : (uint64_t)ser::kS);
    T *out = (T *)a.fa.out;
    int pos = e;
    while (pos < seff && base < a.n) {
        bool acc;
        T v;
        const uint64_t P = c0 + pos;
        const uint32_t len = ser_attempt<DIST, OT, BX>(a, &zt, P, acc, v);
        if (acc) {
            out[base] = v;
            if (base == a.n - 1) a.result[0] = P + len;
            base++;
        }
        pos += (int)len;
    }
}

// ---------------------------------------------------------------------------
template <int ENG>
static int ser_fixed_eng(int dist, int dtype, const SerialArgs &a, hipStream_t st)
{
    const dim3 grid((a.lanes + 255) / 256), block(256);
    switch (dist) {
    case RP_RAW:
        if (dtype == RP_U64) hipLaunchKernelGGL((k_ser_gen<ENG, RP_RAW, RP_U64, true>), grid, block, 0, st, a);
        else hipLaunchKernelGGL((k_ser_gen<ENG, RP_RAW, RP_U32, true>), grid, block, 0, st, a);
        break;
    case RP_U01:
        if (dtype == RP_F64) hipLaunchKernelGGL((k_ser_gen<ENG, RP_U01, RP_F64, true>), grid, block, 0, st, a);
        else hipLaunchKernelGGL((k_ser_gen<ENG, RP_U01, RP_F32, true>), grid, block, 0, st, a);
        break;
    case RP_BOUNDED:  // bound 0: the full range, one item per output
        if (dtype == RP_U64) hipLaunchKernelGGL((k_ser_gen<ENG, RP_BOUNDED, RP_U64, true>), grid, block, 0, st, a);
        else hipLaunchKernelGGL((k_ser_gen<ENG, RP_BOUNDED, RP_U32, true>), grid, block, 0, st, a);
        break;
    default: return fail(RP_EINVAL, "serial fill: distribution %d has no fixed form", dist);
    }
    return RP_OK;
}

int launch_serial_fixed(int engine, int dist, int dtype, const SerialArgs &a, hipStream_t st)
{
    int rc;
    switch (engine) {
    case RP_X256PP: rc = ser_fixed_eng<RP_X256PP>(dist, dtype, a, st); break;
    case RP_X256SS: rc = ser_fixed_eng<RP_X256SS>(dist, dtype, a, st); break;
    case RP_SQUARES: rc = ser_fixed_eng<RP_SQUARES>(dist, dtype, a, st); break;
    case RP_CHACHA20: rc = ser_fixed_eng<RP_CHACHA20>(dist, dtype, a, st); break;
    case RP_PCG64: rc = ser_fixed_eng<RP_PCG64>(dist, dtype, a, st); break;
    case RP_PHILOX4X32: rc = ser_fixed_eng<RP_PHILOX4X32>(dist, dtype, a, st); break;
    case RP_PHILOX: rc = ser_fixed_eng<RP_PHILOX>(dist, dtype, a, st); break;
    case RP_RANLUX: rc = ser_fixed_eng<RP_RANLUX>(dist, dtype, a, st); break;
    default: return fail(RP_EUNSUPPORTED, "serial fill: engine has no jump");
    }
    if (rc) return rc;
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? RP_OK : fail(RP_EDEVICE, "serial fill launch: %s", hipGetErrorString(e));
}

template <int DIST, int OT, bool BX = false>
static void ser_stitch_bx(const SerialArgs &a, hipStream_t st)
{
    const dim3 grid((unsigned)a.nblocks);
    hipLaunchKernelGGL((k_ser_map<DIST, OT, BX>), grid, dim3(ser::kBlk), 0, st, a);
    hipLaunchKernelGGL(k_ser_blocks, dim3(1), dim3(1024), 0, st, a);
    hipLaunchKernelGGL((k_ser_emit<DIST, OT, BX>), grid, dim3(ser::kBlk), 0, st, a);
}

// the ziggurat's rare paths take exp / log1p: a bitexact instantiation
template <int DIST, int OT>
static void ser_stitch_kernels(const SerialArgs &a, hipStream_t st)
{
    if constexpr (DIST == RP_NORM || DIST == RP_EXP)
        if (a.fa.flags & kFlagBitexact) return ser_stitch_bx<DIST, OT, true>(a, st);
    ser_stitch_bx<DIST, OT, false>(a, st);
}

int launch_serial_stitch(int engine, int dist, int dtype, const SerialArgs &a, hipStream_t st)
{
    const dim3 grid((a.lanes + 255) / 256), block(256);
    switch (engine) {
    case RP_X256PP: hipLaunchKernelGGL((k_ser_gen<RP_X256PP, RP_RAW, RP_U64, false>), grid, block, 0, st, a); break;
    case RP_X256SS: hipLaunchKernelGGL((k_ser_gen<RP_X256SS, RP_RAW, RP_U64, false>), grid, block, 0, st, a); break;
    case RP_SQUARES: hipLaunchKernelGGL((k_ser_gen<RP_SQUARES, RP_RAW, RP_U64, false>), grid, block, 0, st, a); break;
    case RP_CHACHA20: hipLaunchKernelGGL((k_ser_gen<RP_CHACHA20, RP_RAW, RP_U64, false>), grid, block, 0, st, a); break;
    case RP_PCG64: hipLaunchKernelGGL((k_ser_gen<RP_PCG64, RP_RAW, RP_U64, false>), grid, block, 0, st, a); break;
    case RP_PHILOX4X32:
        hipLaunchKernelGGL((k_ser_gen<RP_PHILOX4X32, RP_RAW, RP_U64, false>), grid, block, 0, st, a);
        break;
    case RP_PHILOX: hipLaunchKernelGGL((k_ser_gen<RP_PHILOX, RP_RAW, RP_U64, false>), grid, block, 0, st, a); break;
    case RP_RANLUX: hipLaunchKernelGGL((k_ser_gen<RP_RANLUX, RP_RAW, RP_U64, false>), grid, block, 0, st, a); break;
    default: return fail(RP_EUNSUPPORTED, "serial fill: engine has no jump");
    }
    switch (dist) {
    case RP_NORM:
        if (dtype == RP_F64) ser_stitch_kernels<RP_NORM, RP_F64>(a, st);
        else ser_stitch_kernels<RP_NORM, RP_F32>(a, st);
        break;
    case RP_EXP:
        if (dtype == RP_F64) ser_stitch_kernels<RP_EXP, RP_F64>(a, st);
        else ser_stitch_kernels<RP_EXP, RP_F32>(a, st);
        break;
    case RP_BOUNDED:
        if (dtype == RP_U64) ser_stitch_kernels<RP_BOUNDED, RP_U64>(a, st);
        else ser_stitch_kernels<RP_BOUNDED, RP_U32>(a, st);
        break;
    default: return fail(RP_EINVAL, "serial fill: distribution %d has no rejection form", dist);
    }
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? RP_OK : fail(RP_EDEVICE, "serial fill launch: %s", hipGetErrorString(e));
}
