// k_zig.h -- binary64 ziggurat fills (Section 3.1, ziggurat figure) for the
// wavefront engines that generate in store order: Philox4x32-10, PCG64
// (groups of G = 2 words), Philox-4x64-10 (G = 4) and squares64 (G = 1).
// Included by fill.hip.
//
// One wavefront per substream.  A chunk is 64 R consecutive words; lane l
// holds the G words at chunk positions 64 G g + G l + j (group g < R / G,
// j < G), as the engines' raw fills produce them, so the common path needs
// no transpose.  Per chunk:
//
//  1. the words go to LDS in stream order, and every word is classified as
//     if a sample started there (strip, fast test against K[j]);
//  2. each lane resolves its own long items (wedge test, exponential tail,
//     normal tail), one per pass, from the words in LDS: words used, and
//     whether the attempt yields a value;
//  3. group by group, the samples are found: when no long item lies inside
//     another and none is a normal tail, every long item starts a two-word
//     sample and a few mask operations give the group's values; otherwise a
//     scalar walk over the long items in stream order decides which start
//     samples (one inside an earlier long sample does not) and which fast
//     words they cover.  Only a group where a normal tail starts takes the
//     walk on its account.  The values are stored at their ranks in stream
//     order (ballot + mbcnt); a wedge accept has the fast candidate's value.
//     A tail that yields is resolved once more from the words in LDS: the
//     exponential one where it is stored, the normal one (its own loop of
//     pairs) after the walk, written by the same lane over the candidate
//     stored at its rank.
//
// A sample that needs words past the chunk is carried into the next chunk
// (its first word, and for the normal tail an unused first word of a
// pair), resolved there before anything else.

template <class E>
struct ZigConsecutive {
    static constexpr bool value = false;
};
template <>
struct ZigConsecutive<WavePcg> {
    static constexpr bool value = true;
};

// Six wavefronts per SIMD (at most 85 VGPRs; the LDS of a block allows six
// blocks per compute unit) measured fastest: 3.2 ms for 2^30 Philox4x32-10
// normals against 3.6 ms at four and 4.3 ms at eight (spills).  Transforms
// with exp, log or pow in the store need more registers and take four.
template <int XFC>
struct ZigWaves {
    static constexpr int XF = xf_law(XFC);
    static constexpr int value = (XF == 0 || XF == RP_LAW_NORMAL || XF == RP_LAW_EXP) ? 6 : 4;
};

template <class E, int DIST, int XF>
__global__ __launch_bounds__(256, ZigWaves<XF>::value) void k_zig(FillArgs a)
{
    constexpr int R = E::R;       // words per lane per chunk
    constexpr int G = E::G;       // consecutive words per lane per group
    constexpr int NG = R / G;     // groups per chunk
    constexpr int GW = 64 * G;    // words per group
    constexpr int CHW = 64 * R;   // words per chunk
    static_assert(R % G == 0 && (G == 1 || G == 2 || G == 4), "group layout");

    const int wib = threadIdx.x >> 6;
    const int lane = threadIdx.x & 63;
    __shared__ __align__(16) WKe zt[256];
    __shared__ __align__(16) uint64_t wb_all[4][CHW];
    __shared__ uint16_t rinf_all[4][CHW];  // long item at a position: words used | 0x8000 if it yields
    // normal tails with a value: each walked group's final masks and first
    // rank, for the fix-up after the walk
    constexpr bool TFIX = DIST == RP_NORM;
    __shared__ uint64_t fy_all[4][TFIX ? R : 1];
    __shared__ uint32_t fnv_all[4][TFIX ? NG : 1];
    for (int k = threadIdx.x; k < 256; k += blockDim.x) {
        zt[k].w = DIST == RP_NORM ? RP_ZN_W[k] : RP_ZE_W[k];
        zt[k].k = DIST == RP_NORM ? RP_ZN_K[k] : RP_ZE_K[k];
    }
    __syncthreads();
    const uint64_t sub = (uint64_t)__builtin_amdgcn_readfirstlane(blockIdx.x * (blockDim.x >> 6) + wib);
    if (sub >= a.n) return;
    const uint64_t P = a.per_stream;
    if (P == 0) return;
    uint64_t *const wb = wb_all[wib];
    uint16_t *const rinf = rinf_all[wib];
    double *const out = (double *)a.out + sub * P;
    const int zflags = a.flags;  // squeeze switch and bitexact setting

    // Engines whose consecutive words are cheaper than the store-order ones
    // (PCG64: ordinary steps instead of stride-127 jumps) generate R
    // consecutive words per lane and take their store-order words back
    // from LDS.
    constexpr bool CONSEC = ZigConsecutive<E>::value;
    E eng;
    if constexpr (CONSEC) eng.load(a, sub, lane);
    else eng.load_direct(a, sub, lane);
    // chunk position of this lane's item i
    auto posof = [&](int i) { return GW * (i / G) + G * lane + i % G; };
    // lanes whose position 64 G g + G l + j is at least p
    auto lanes_from = [](int p, int g, int j) -> uint64_t {
        const int d = p - GW * g - j;
        if (d <= 0) return ~0ull;
        const int lo = (d + G - 1) / G;
        return lo >= 64 ? 0ull : (~0ull << lo);
    };

    int s0 = (int)eng.phase0;       // first position of the chunk that may start a sample
    uint64_t produced = 0;
    uint64_t final_pos = 0;         // words from the start, after the last value
    bool carry = false;             // a sample from the previous chunk still needs words:
    bool c_hu = false;              //   it holds an unused first word of a tail pair
    uint64_t c_w0 = 0, c_u1 = 0;    //   its first word and that spare word
    // every chunk yields well over half of its words as values: the bound
    // is never reached and only guarantees that the wavefront exits
    const uint64_t max_chunks = 2 * (P / CHW) + 1024;
    for (uint64_t chunk = 0; chunk < max_chunks; chunk++) {
        const uint64_t base_pos = chunk * CHW;
        double v[R];      // candidate value of every word as a fast or wedge sample
        uint32_t lb = 0;  // bit i: item i fails the fast test
        {
            uint64_t w[R];
            if constexpr (CONSEC) {
                static_assert(G == 2 && R % 2 == 0, "consecutive generation layout");
                eng.gen(w);
                eng.next_chunk();
#pragma unroll
                for (int k = 0; k < R; k += 2) {
                    ulonglong2 q;
                    q.x = w[k];
                    q.y = w[k + 1];
                    *(ulonglong2 *)(wb + R * lane + k) = q;
                }
                wave_sync();
#pragma unroll
                for (int g = 0; g < NG; g++) {
                    const ulonglong2 q = *(const ulonglong2 *)(wb + GW * g + G * lane);
                    w[G * g] = q.x;
                    w[G * g + 1] = q.y;
                }
            } else {
                eng.gen_direct(w);
#pragma unroll
                for (int g = 0; g < NG; g++) {
                    const int p0 = GW * g + G * lane;
                    if constexpr (G == 1) {
                        wb[p0] = w[g];
                    } else {
#pragma unroll
                        for (int k = 0; k < G; k += 2) {
                            ulonglong2 q;
                            q.x = w[G * g + k];
                            q.y = w[G * g + k + 1];
                            *(ulonglong2 *)(wb + p0 + k) = q;
                        }
                    }
                }
            }
#pragma unroll
            for (int i = 0; i < R; i++) {
                lb |= (zig_fast<DIST>(zt, w[i], v[i]) ? 0u : 1u) << i;
                // formed here, so that neither the word nor its table entry
                // stays live until the store
                asm volatile("" : "+v"(v[i]));
            }
        }
        asm volatile("" : "+v"(lb));
        wave_sync();

        // ---- the sample carried over from the previous chunk: its words are
        //      [the spare tail word,] then this chunk from position 0 ----
        bool have_first = false;
        double first_v = 0.0;
        if (carry) {
            const int hu = c_hu ? 1 : 0;
            bool acc = false, hu_o = false;
            double cv = 0.0;
            uint64_t u1o = 0;
            int L = zig_resolve<DIST, false, false, xf_bx(XF)>(
                zt, c_w0, [&](int k) { return (hu && k == 1) ? c_u1 : wb[k - 1 - hu]; }, CHW + hu, zflags, acc, cv,
                hu_o, u1o);
            L = __builtin_amdgcn_readfirstlane(L);
            if (L == 0) {  // it uses the whole chunk
                c_hu = __builtin_amdgcn_readfirstlane(hu_o ? 1 : 0) != 0;
                c_u1 = uni64(u1o);
                wave_sync();
                continue;
            }
            carry = false;
            s0 = L - 1 - hu;
            if (__builtin_amdgcn_readfirstlane(acc ? 1 : 0)) {
                have_first = true;
                first_v = cv;
            }
        }

        // ---- (2) each lane resolves its long items at positions >= s0 ----
        uint32_t live = (1u << R) - 1;
        if (s0 > 0) {
#pragma unroll
            for (int i = 0; i < R; i++)
                if (posof(i) < s0) live &= ~(1u << i);
        }
        uint32_t rem = lb & live;
        uint32_t accb = 0;       // bit i: long item i yields a value if it starts a sample
        uint32_t tlb = 0;        // bit i: long item i starts a normal tail
        bool tails = false;      // a normal tail (words used vary) among the long items
        bool tail_vals = false;  // a tail (strip 0) that yields a value
        while (__ballot(rem != 0)) {
            if (rem) {
                const int i = __builtin_ctz(rem);
                rem &= rem - 1;
                const int p = posof(i);
                const uint64_t w0 = wb[p];
                bool acc, hu_o;
                double val;
                uint64_t u1o;
                const int L = zig_resolve<DIST, false, false, xf_bx(XF)>(
                    zt, w0, [&](int k) { return wb[p + k]; }, CHW - 1 - p, zflags, acc, val, hu_o, u1o);
                rinf[p] = (uint16_t)(L | (acc ? 0x8000 : 0));
                accb |= (acc ? 1u : 0u) << i;
                if ((w0 & 0xff) == 0) {
                    tails = tails || DIST == RP_NORM;
                    tail_vals = tail_vals || acc;
                    if (DIST == RP_NORM) tlb |= 1u << i;
                }
            }
        }
        const bool any_tail = DIST == RP_NORM && __ballot(tails) != 0;
        const bool any_tail_val = __ballot(tail_vals) != 0;
        wave_sync();  // rinf visible to the walk
        // words a long item at q uses (0: more than the chunk holds)
        auto long_len = [&](int q) -> int {
            if (any_tail) return __builtin_amdgcn_readfirstlane((int)rinf[q]) & 0x7fff;
            return q + 1 < CHW ? 2 : 0;
        };

        // ---- (3) walk and store, group by group ----
        const uint64_t need = P - produced;  // >= 1
        double *const dst = out + produced;
        uint32_t nv = 0;                     // values of this chunk so far
        bool done = false;
        int walked = 0;                      // groups walked (tail fix-up)
        if (have_first) {
            if (lane == 0) dst[0] = xform<XF>(first_v, a);
            nv = 1;
            if (need == 1) {
                final_pos = base_pos + (uint64_t)s0;
                done = true;
            }
        }
        int cover_end = s0;  // positions below are used by earlier samples
        int pend_q = -1;     // a sample starting here needs words past the chunk
        // unrolled: v[] is then indexed by constants and stays in registers
#pragma unroll
        for (int g = 0; g < NG; g++) {
            if (done || pend_q >= 0) break;
            const int g0 = GW * g;
            // positions below cover_end belong to earlier samples (or precede
            // the call's first word)
            uint64_t Lm[G], Fm[G], Am[G], Y[G];
#pragma unroll
            for (int j = 0; j < G; j++) {
                const uint64_t lmask = __ballot((lb >> (G * g + j)) & 1);
                const uint64_t lv = cover_end > g0 ? lanes_from(cover_end, g, j) : ~0ull;
                Lm[j] = lmask & lv;
                Fm[j] = ~lmask & lv;
                Am[j] = __ballot((accb >> (G * g + j)) & 1);
            }
            // The position after each long item, in the same layout: the
            // words such an item covers when it starts a two-word sample.
            uint64_t Cn[G];
            Cn[0] = Lm[G - 1] << 1;
#pragma unroll
            for (int j = 1; j < G; j++) Cn[j] = Lm[j - 1];
            uint64_t chain = 0;
#pragma unroll
            for (int j = 0; j < G; j++) chain |= Cn[j] & Lm[j];
            const bool last_long = g == NG - 1 && (Lm[G - 1] >> 63) != 0;
            // only a group where a normal tail starts needs the walk for its
            // sake (a tail before it is seen through cover_end)
            bool gtail = false;
            if (any_tail) {
                uint64_t tm = 0;
#pragma unroll
                for (int j = 0; j < G; j++) tm |= __ballot((tlb >> (G * g + j)) & 1);
                gtail = tm != 0;
            }
            if (!gtail && !chain && !last_long) {
                // common case: every long item starts a two-word sample and
                // covers only the word after it
#pragma unroll
                for (int j = 0; j < G; j++) Y[j] = (Fm[j] & ~Cn[j]) | (Lm[j] & Am[j]);
                const int ge = g0 + GW;
                cover_end = (Lm[G - 1] >> 63) ? ge + 1 : (cover_end > ge ? cover_end : ge);
            } else {
                // a long item inside another, a tail, or a sample running past
                // the chunk: walk the long items in stream order
                uint64_t C[G], Sa[G], rm[G];
#pragma unroll
                for (int j = 0; j < G; j++) {
                    C[j] = 0;
                    Sa[j] = 0;
                    rm[j] = Lm[j];
                }
                for (;;) {
                    int best = 1 << 30, bj = 0;
#pragma unroll
                    for (int j = 0; j < G; j++) {
                        if (rm[j]) {
                            const int c = G * (int)__builtin_ctzll(rm[j]) + j;
                            if (c < best) {
                                best = c;
                                bj = j;
                            }
                        }
                    }
                    if (best == 1 << 30) break;
#pragma unroll
                    for (int j = 0; j < G; j++)
                        if (j == bj) rm[j] &= rm[j] - 1;
                    const int q = g0 + best;
                    if (q < cover_end) continue;  // inside an earlier sample
                    const int L = long_len(q);
                    if (L == 0) {
                        pend_q = q;
                        break;
                    }
                    const int l = best / G;
#pragma unroll
                    for (int j = 0; j < G; j++)
                        if (j == bj) Sa[j] |= Am[j] & (1ull << l);
                    cover_end = q + L;
                    // fast words inside this sample, in this group (later
                    // groups see cover_end)
                    const int cend = cover_end < g0 + GW ? cover_end : g0 + GW;
                    for (int c = q + 1; c < cend; c++) {
                        const int cin = c - g0;
#pragma unroll
                        for (int j = 0; j < G; j++)
                            if (j == cin % G) C[j] |= 1ull << (cin / G);
                    }
                }
#pragma unroll
                for (int j = 0; j < G; j++) {
                    Y[j] = (Fm[j] & ~C[j]) | Sa[j];
                    if (pend_q >= 0) Y[j] &= ~lanes_from(pend_q, g, j);
                }
            }
            uint32_t cnt = 0;
#pragma unroll
            for (int j = 0; j < G; j++) cnt += (uint32_t)__popcll(Y[j]);
            if ((uint64_t)nv + cnt >= need) {
                // the last values of the call: keep the first need - nv in
                // stream order, and find where the last one's words end
                uint32_t k = (uint32_t)(need - nv);
                uint64_t keep[G], ym[G];
#pragma unroll
                for (int j = 0; j < G; j++) {
                    keep[j] = 0;
                    ym[j] = Y[j];
                }
                int lastq = 0;
                for (; k > 0; k--) {
                    int best = 1 << 30, bj = 0;
#pragma unroll
                    for (int j = 0; j < G; j++) {
                        if (ym[j]) {
                            const int c = G * (int)__builtin_ctzll(ym[j]) + j;
                            if (c < best) {
                                best = c;
                                bj = j;
                            }
                        }
                    }
#pragma unroll
                    for (int j = 0; j < G; j++) {
                        if (j == bj) {
                            keep[j] |= ym[j] & (0 - ym[j]);
                            ym[j] &= ym[j] - 1;
                        }
                    }
                    lastq = GW * g + best;
                }
                bool lastlong = false;
#pragma unroll
                for (int j = 0; j < G; j++)
                    if (j == (lastq - GW * g) % G) lastlong = (Lm[j] >> ((lastq - GW * g) / G)) & 1;
                int L = 1;
                if (lastlong) L = long_len(lastq);
                final_pos = base_pos + (uint64_t)(lastq + L);
#pragma unroll
                for (int j = 0; j < G; j++) Y[j] = keep[j];
                cnt = (uint32_t)(need - nv);
                done = true;
            }
            if (TFIX && any_tail_val) {
                if (lane == 0) {
#pragma unroll
                    for (int j = 0; j < G; j++) fy_all[wib][G * g + j] = Y[j];
                    fnv_all[wib][g] = nv;
                }
                walked = g + 1;
            }
            // values at their ranks in stream order
            uint32_t idx = nv;
#pragma unroll
            for (int j = 0; j < G; j++) idx += mbcnt64(Y[j]);
#pragma unroll
            for (int j = 0; j < G; j++) {
                const bool mine = (Y[j] >> lane) & 1;
                if (mine) {
                    double x = v[G * g + j];
                    if (!TFIX && any_tail_val && ((Lm[j] >> lane) & 1)) {
                        // a tail (strip 0) that starts a sample: its value
                        // from the tail draw, resolved again
                        const int p = g0 + G * lane + j;
                        const uint64_t w0 = wb[p];
                        if ((w0 & 0xff) == 0) {
                            bool acc, hu_o;
                            uint64_t u1o;
                            (void)zig_resolve<DIST, false, false, xf_bx(XF)>(
                                zt, w0, [&](int k) { return wb[p + k]; }, CHW - 1 - p, zflags, acc, x, hu_o, u1o);
                        }
                    }
                    dst[idx] = xform<XF>(x, a);
                }
                idx += mine ? 1u : 0u;
            }
            nv += cnt;
        }
        if (TFIX && any_tail_val) {
            // A normal tail that starts a sample was stored above with its
            // fast candidate; the same lane stores its value over it, resolved
            // again from the words in LDS.  Kept out of the unrolled walk:
            // inline there, the rare resolution costs the common path.
            wave_sync();
#pragma unroll 1
            for (int g = 0; g < walked; g++) {
                uint64_t Yg[G];
#pragma unroll
                for (int j = 0; j < G; j++) Yg[j] = uni64(fy_all[wib][G * g + j]);
                uint32_t idx = (uint32_t)__builtin_amdgcn_readfirstlane((int)fnv_all[wib][g]);
#pragma unroll
                for (int j = 0; j < G; j++) idx += mbcnt64(Yg[j]);
#pragma unroll
                for (int j = 0; j < G; j++) {
                    const bool mine = (Yg[j] >> lane) & 1;
                    if (mine && ((tlb >> (G * g + j)) & 1)) {
                        const int p = GW * g + G * lane + j;
                        bool acc, hu_o;
                        uint64_t u1o;
                        double x;
                        (void)zig_resolve<DIST, false, false, xf_bx(XF)>(
                            zt, wb[p], [&](int k) { return wb[p + k]; }, CHW - 1 - p, zflags, acc, x, hu_o, u1o);
                        dst[idx] = xform<XF>(x, a);
                    }
                    idx += mine ? 1u : 0u;
                }
            }
        }
        produced += nv;
        if (done) break;
        if (pend_q >= 0) {
            // the sample at pend_q continues in the next chunk: its first
            // word and, for a normal tail, a spare first word of a pair
            carry = true;
            c_w0 = uni64(wb[pend_q]);
            c_hu = false;
            c_u1 = 0;
            if (DIST == RP_NORM && (c_w0 & 0xff) == 0) {
                bool acc, hu_o;
                double cv;
                uint64_t u1o = 0;
                const int p = pend_q;
                (void)zig_resolve<DIST, false, false, xf_bx(XF)>(
                    zt, c_w0, [&](int k) { return wb[p + k]; }, CHW - 1 - p, zflags, acc, cv, hu_o, u1o);
                c_hu = __builtin_amdgcn_readfirstlane(hu_o ? 1 : 0) != 0;
                c_u1 = uni64(u1o);
            }
        }
        s0 = 0;
        wave_sync();  // the next chunk overwrites wb and rinf
    }
    if (lane == 0) eng.store(a, sub, final_pos);
}
