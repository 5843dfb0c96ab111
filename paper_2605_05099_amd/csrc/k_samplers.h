// k_samplers.h -- lane-per-substream samplers: fused moments, gamma, beta.
// Included by fill.hip (one translation unit shares the constant tables).
//
// Each lane runs the serial definition of its substream: normals by the
// ziggurat (zig_serial), uniforms from the top 53 bits, Marsaglia-Tsang gamma
// (Section 3.1, "Gamma and related distributions") with the shape < 1 boost,
// beta as X / (X + Y).  Floating point is evaluated exactly as written
// (-ffp-contract=off), so the decisions and values match the serial
// definition; only log/exp may differ from another library by an ulp.
#pragma once

// ---------------------------------------------------------------------------
// serial word streams for the counter / LCG engines (lane-per-substream use)
// Philox4x32-10: counter of the current block, its two words, and the next
// block (counter + 1) when hn (the two-block scheme of wave_any in fill.hip).
struct LanePhilox32 {
    uint64_t clo, chi, key;
    uint64_t c0, c1, n0, n1;
    uint32_t ph;  // words of the current block used (0..2)
    bool hn;
    __device__ void start(uint64_t lo, uint64_t hi, uint64_t k, uint32_t phase)
    {
        clo = lo;
        chi = hi;
        key = k;
        ph = phase;
        philox4x32(clo, chi, key, c0, c1);
        hn = false;
    }
    __device__ void reserve(int) {}
    __device__ void load(const FillArgs &a, uint64_t i)
    {
        start(a.words[i], a.words[a.n + i], a.words[2 * a.n + i], a.phase[i]);
    }
    __device__ uint64_t next()
    {
        if (wave_any(ph == 2 && !hn)) {
            if (!hn) {
                const uint64_t lo = clo + 1;
                philox4x32(lo, chi + (lo == 0 ? 1u : 0u), key, n0, n1);
                hn = true;
            }
        }
        if (ph == 2) {
            clo += 1;
            chi += (clo == 0) ? 1u : 0u;
            c0 = n0;
            c1 = n1;
            hn = false;
            ph = 0;
        }
        const uint64_t w = ph ? c1 : c0;
        ph++;
        return w;
    }
    __device__ void store(const FillArgs &a, uint64_t i) const
    {
        const bool done = ph == 2;
        const uint64_t lo = clo + (done ? 1u : 0u);
        a.words[i] = lo;
        a.words[a.n + i] = chi + ((done && lo == 0) ? 1u : 0u);
        a.phase[i] = done ? 0u : ph;
    }
};

// Philox-4x64-10: 256-bit counter of the current block, its four words, and
// the next block when hn.
struct LanePhilox64 {
    uint64_t c[4], k0, k1, b[4], nb[4];
    uint32_t ph;  // 0..4
    bool hn;
    __device__ static void inc(const uint64_t *in, uint64_t *out)
    {
        uint64_t carry = 1;
#pragma unroll
        for (int k = 0; k < 4; k++) {
            out[k] = in[k] + carry;
            carry = (carry && out[k] == 0) ? 1u : 0u;
        }
    }
    __device__ void start(uint32_t phase)
    {
        ph = phase;
        philox4x64(c, k0, k1, b);
        hn = false;
    }
    __device__ void reserve(int) {}
    __device__ void load(const FillArgs &a, uint64_t i)
    {
#pragma unroll
        for (int k = 0; k < 4; k++) c[k] = a.words[(uint64_t)k * a.n + i];
        k0 = a.words[4 * a.n + i];
        k1 = a.words[5 * a.n + i];
        start(a.phase[i]);
    }
    __device__ uint64_t next()
    {
        if (wave_any(ph == 4 && !hn)) {
            if (!hn) {
                uint64_t cn[4];
                inc(c, cn);
                philox4x64(cn, k0, k1, nb);
                hn = true;
            }
        }
        if (ph == 4) {
            inc(c, c);
#pragma unroll
            for (int k = 0; k < 4; k++) b[k] = nb[k];
            hn = false;
            ph = 0;
        }
        uint64_t w = b[0];
        w = (ph == 1) ? b[1] : w;
        w = (ph == 2) ? b[2] : w;
        w = (ph == 3) ? b[3] : w;
        ph++;
        return w;
    }
    __device__ void store(const FillArgs &a, uint64_t i) const
    {
        uint64_t cn[4];
        inc(c, cn);
        const bool done = ph == 4;
#pragma unroll
        for (int k = 0; k < 4; k++) a.words[(uint64_t)k * a.n + i] = done ? cn[k] : c[k];
        a.phase[i] = done ? 0u : ph;
    }
};

struct LanePcg {
    u128 s, inc;
    __device__ void reserve(int) {}
    __device__ void load(const FillArgs &a, uint64_t i)
    {
        s = u128{a.words[i], a.words[a.n + i]};
        inc = u128{a.words[2 * a.n + i], a.words[3 * a.n + i]};
    }
    __device__ uint64_t next()
    {
        const uint64_t w = pcg_dxsm(s);
        s = pcg_step(s, inc);
        return w;
    }
    __device__ void store(const FillArgs &a, uint64_t i) const
    {
        a.words[i] = s.lo;
        a.words[a.n + i] = s.hi;
    }
};

// ---------------------------------------------------------------------------
// U^(1/a) for the gamma boost (a < 1), U = k 2^-53.  log U is formed to about
// 2^-70 absolute with the table log: U = 2^e m, m in [1, 2), c = table point
// near m, log U = e ln2 + log c + log1p((m - c)/c); then t = log(U)/a as a
// pair of doubles and the result exp(t_hi) (1 + t_lo).  Its error is about an
// ulp whatever the size of |t|, where a plain exp(log(U)/a) would lose
// |t| ulps.
__device__ __forceinline__ void two_sum(double a, double b, double &s, double &e)
{
    s = a + b;
    const double bb = s - a;
    e = (a - (s - bb)) + (b - bb);
}

// The log table of log_dd, one 32-byte entry per point, staged in LDS by the
// kernels that draw boosted gammas: the lookup sits on every boosted draw,
// where a global-memory load stalls the whole wavefront.
struct LogE {
    double c, inv, hi, lo;
};
struct LogLds {
    LogE e[256];
};
__device__ __forceinline__ void load_logt(LogLds *t)
{
    for (int k = threadIdx.x; k < 256; k += blockDim.x) t->e[k] = LogE{RP_LOG_C[k], RP_LOG_INV[k], RP_LOG_HI[k], RP_LOG_LO[k]};
}

// log u as a pair (lh, ll), u > 0 finite, from the 256-entry table: u = 2^e m,
// m in [1, 2), c the table point of m's top fraction bits, log u =
// e ln2 + log c + log1p((m - c)/c) with a degree-7 series.
__device__ __forceinline__ void log_dd(double u, double &lh, double &ll, const LogLds *lt)
{
    int ex;
    double m = frexp(u, &ex);  // u = m 2^ex, m in [0.5, 1)
    m = m * 2.0;
    ex -= 1;
    const int i = (int)(((uint64_t)__double_as_longlong(m) >> 44) & 0xff);
    const LogE te = lt->e[i];
    const double c = te.c, ic = te.inv;
    const double num = m - c;  // exact: m and c are within a factor of 2
    const double rh = num * ic;
    const double rl = __fma_rn(-rh, c, num) * ic;
    const double p = (rh * rh) * (-0.5 + rh * (1.0 / 3.0 + rh * (-0.25 + rh * (0.2 + rh * (-1.0 / 6.0 + rh * (1.0 / 7.0))))));
    double sh, sl, t;
    two_sum((double)ex * RP_LN2_HI, te.hi, sh, sl);
    two_sum(sh, rh, sh, t);
    sl = sl + t + (((double)ex * RP_LN2_LO + te.lo) + (rl + p));
    lh = sh + sl;
    ll = sl - (lh - sh);
}

template <bool BX>
__device__ double boost_pow(double u, double a, double ia, const LogLds *lt)
{
    if constexpr (BX) return bx_powinv(u, a);  // correctly rounded u^(1/a)
    if (u == 0.0) return 0.0;
    double lh, ll;
    log_dd(u, lh, ll, lt);
    // t = log(u) / a as th + tl; th need not be the rounded quotient
    const double th = lh * ia;
    const double tl = (__fma_rn(-th, a, lh) + ll) * ia;
    const double eh = exp(th);
    if (eh == 0.0) return 0.0;  // also keeps 0 * inf away when a is tiny
    return eh + eh * tl;
}

// One ziggurat normal candidate (the serial ziggurat's decisions): true with
// the value when it is accepted, false when rejected (the caller starts a
// new candidate, exactly where the serial sampler would).
// HALF: the float ziggurat on 32-bit items (the binary32 value it returns).
template <class E, bool HALF = false, bool BX = false>
__device__ __forceinline__ bool zig_candidate(E &eng, const ZigLds *zt, double &x)
{
    const uint64_t w = HALF ? item_word<RP_NORM>(eng.next()) : eng.next();
    const int j = (int)(w & 0xff);
    const uint64_t m = (w >> 9) & ((1ull << 52) - 1);
    const bool neg = (w >> 8) & 1;
    const WKe e = zt->WK[j];
    const double xx = (double)m * e.w;
    if (m < e.k) {
        x = zbase<HALF>(neg ? -xx : xx);
        return true;
    }
    if (j == 0) {
        for (int it = 0; it < kMaxTailIters; it++) {
            const double e1 = -f_log1p<BX>(-zig_u<HALF>(eng.next())) / RP_ZN_R;
            const double e2 = -f_log1p<BX>(-zig_u<HALF>(eng.next()));
            if (e2 + e2 > e1 * e1) {
                const double t = RP_ZN_R + e1;
                x = zbase<HALF>(neg ? -t : t);
                return true;
            }
        }
        return false;
    }
    if (wedge_accept<RP_NORM, HALF, BX>(zt, j, xx, eng.next())) {
        x = zbase<HALF>(neg ? -xx : xx);
        return true;
    }
    return false;
}

// 32-bit items of a lane engine, low half first (a half left over when the
// caller stops is dropped: the engine's state is after the last word)
template <class E>
struct ItemEng {
    E &e;
    bool have = false;
    uint32_t hi = 0;
    __device__ explicit ItemEng(E &x) : e(x) {}
    __device__ uint64_t next()
    {
        if (have) {
            have = false;
            return hi;
        }
        const uint64_t w = e.next();
        hi = (uint32_t)(w >> 32);
        have = true;
        return (uint32_t)w;
    }
    __device__ void reserve(int k) { e.reserve((k + 1) / 2); }
};

// The normal ziggurat as a step machine: a step takes at most two words (a
// candidate and its wedge word, or one tail pair) and either yields a value
// or leaves the machine where the serial sampler would continue.  Kernels
// that loop over steps can therefore reserve two words per step.
struct NormMachine {
    int tail;  // tail pairs taken for the current candidate, -1 outside the tail
    bool neg;
    __device__ void reset() { tail = -1; }
    template <bool BX = false, class E>
    __device__ __forceinline__ bool step(E &eng, const ZigLds *zt, double &x)
    {
        if (tail >= 0) {
            const double e1 = -f_log1p<BX>(-u01_53(eng.next())) / RP_ZN_R;
            const double e2 = -f_log1p<BX>(-u01_53(eng.next()));
            if (e2 + e2 > e1 * e1) {
                tail = -1;
                const double t = RP_ZN_R + e1;
                x = neg ? -t : t;
                return true;
            }
            if (++tail == kMaxTailIters) tail = -1;
            return false;
        }
        const uint64_t w = eng.next();
        const int j = (int)(w & 0xff);
        const uint64_t m = (w >> 9) & ((1ull << 52) - 1);
        neg = (w >> 8) & 1;
        const WKe e = zt->WK[j];
        const double xx = (double)m * e.w;
        if (m < e.k) {
            x = neg ? -xx : xx;
            return true;
        }
        if (j == 0) {
            tail = 0;
            return false;
        }
        if (wedge_accept<RP_NORM, false, BX>(zt, j, xx, eng.next())) {
            x = neg ? -xx : xx;
            return true;
        }
        return false;
    }
};

// The Marsaglia-Tsang test log u < x^2/2 + d (1 - v + log v), decided first
// with the binary32 hardware logarithm (log2, an ulp or two) of u and v.  Its
// error, with that of rounding u and v to binary32, is below 2^-16 (1 + |log|)
// for either logarithm, and the binary64 evaluation of the right-hand side
// errs by far less than 1e-13 (x^2 + d (1 + v)).  When the two sides are
// further apart than the sum of these bounds the binary64 test can only
// agree; otherwise (a few attempts in 10^5) the binary64 logarithms decide,
// exactly as written.  About one attempt in twelve reaches this test, so a
// wavefront meets it at almost every step: the bound saves the two binary64
// logarithms there.
template <bool BX>
__device__ __forceinline__ bool mt_log_test(double u, double x2, double v, double d)
{
    constexpr double kLn2 = 0x1.62e42fefa39efp-1;
    const double lu = (double)__builtin_amdgcn_logf((float)u) * kLn2;
    const double lv = (double)__builtin_amdgcn_logf((float)v) * kLn2;
    const double r = 0.5 * x2 + d * ((1.0 - v) + lv);
    const double e = 0x1p-16 * (1.0 + fabs(lu) + d * (1.0 + fabs(lv))) + 1e-13 * (x2 + d * (1.0 + v));
    if (lu < r - e) return true;
    if (lu > r + e) return false;
    return f_log<BX>(u) < 0.5 * x2 + d * ((1.0 - v) + f_log<BX>(v));
}

// Marsaglia-Tsang constants of one shape: d = s - 1/3, c = 1/sqrt(9 d) for
// s = a (a >= 1) or s = a + 1 followed by the boost U^(1/a) (a < 1).
struct GamParam {
    double a, d, c, ia;
    bool boost;
};

__device__ __forceinline__ GamParam gam_param(double a)
{
    GamParam p;
    p.a = a;
    p.boost = a < 1.0;
    const double s = p.boost ? a + 1.0 : a;
    p.d = s - 1.0 / 3.0;
    p.c = 1.0 / sqrt(9.0 * p.d);
    p.ia = 1.0 / a;
    return p;
}

// Gamma or beta draws as a sequence of single attempts, so the lanes of a
// wavefront move on independently: each step() takes one ziggurat candidate
// and, if it is accepted and v > 0, one uniform for the squeeze / log test
// (and one more for the boost when the attempt is accepted and a < 1).  The
// words used and the decisions are those of the serial sampler: a rejected
// candidate or attempt is followed by a fresh one, as in its loops.  Beta
// draws X ~ Gamma(a), then Y ~ Gamma(b), then returns X / (X + Y).
// MODE 0: Gamma(a) draws; 1: Beta(a, b) = X / (X + Y); 2: the F ratio
// (X / nu1) / (Y / nu2) of X ~ Gamma(a), Y ~ Gamma(b), nu1 = 2a, nu2 = 2b (both
// doublings exact).  X is drawn before Y.
// HALF: the float gamma (32-bit items: the float ziggurat's binary32 normal,
// 24-bit uniforms for the test and the boost; binary64 arithmetic)
template <int MODE, bool HALF = false, bool BX = false>
struct GamMachine {
    static constexpr bool BETA = MODE != 0;
    GamParam pa, pb;
    bool second;
    double X;
    __device__ void set(double a, double b)
    {
        pa = gam_param(a);
        if (BETA) pb = gam_param(b);
        second = false;
    }
    template <class E>
    __device__ __forceinline__ bool step(E &eng, const ZigLds *zt, const LogLds *lt, double &val)
    {
        eng.reserve(4);  // candidate, wedge word, uniform, boost uniform
        const bool sb = BETA && second;
        const double d = sb ? pb.d : pa.d, c = sb ? pb.c : pa.c;
        double x;
        if (!zig_candidate<E, HALF, BX>(eng, zt, x)) return false;
        double v = 1.0 + c * x;
        if (v <= 0.0) return false;
        v = v * v * v;
        const double u = zig_u<HALF>(eng.next());
        const double x2 = x * x;
        bool acc = u < 1.0 - 0.0331 * (x2 * x2);
        if (!acc) acc = mt_log_test<BX>(u, x2, v, d);
        if (!acc) return false;
        double g = d * v;
        if (sb ? pb.boost : pa.boost) {
            const double a = sb ? pb.a : pa.a, ia = sb ? pb.ia : pa.ia;
            g = g * boost_pow<BX>(zig_u<HALF>(eng.next()), a, ia, lt);
        }
        if (!BETA) {
            val = g;
            return true;
        }
        if (!second) {
            X = g;
            second = true;
            return false;
        }
        second = false;
        if constexpr (MODE == 2) {
            val = (X / (2.0 * pa.a)) / (g / (2.0 * pb.a));
            return true;
        }
        const double t = X + g;
        val = (t == 0.0) ? pa.a / (pa.a + pb.a) : X / t;
        return true;
    }
};

template <class E, bool BX = false>
__global__ __launch_bounds__(256) void k_norm_moments(SampArgs s)
{
    __shared__ ZigLds zt;
    load_zig<RP_NORM>(&zt, s.f.flags);
    __syncthreads();
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= s.count) return;
    E eng;
    eng.load(s.f, i);
    NormMachine nm;
    nm.reset();
    double a = 0.0, q = 0.0;
    for (uint64_t t = 0; t < s.f.per_stream;) {
        eng.reserve(2);
        double x;
        if (nm.template step<BX>(eng, &zt, x)) {
            a = a + x;
            q = q + x * x;
            t++;
        }
    }
    s.sum[i] = a;
    s.sumsq[i] = q;
    eng.store(s.f, i);
}

// Element e draws from substream e.  Lanes take elements e, e + stride, ...
// and move to their next element as soon as the current one is accepted.
template <class E, bool BETA, bool BX = false>
__global__ __launch_bounds__(256) void k_gamma_elem(SampArgs s)
{
    __shared__ ZigLds zt;
    __shared__ LogLds lt;
    load_zig<RP_NORM>(&zt, s.f.flags);
    load_logt(&lt);
    __syncthreads();
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    E eng;
    GamMachine<BETA, false, BX> gm;
    bool open = false;
    for (;;) {
        if (!open) {
            if (i >= s.count) break;
            const double pa = (double)s.pa[i];
            const double pb = BETA ? (double)s.pb[i] : 1.0;
            if (!(pa > 0.0) || !(pb > 0.0)) {
                s.z[i] = __builtin_nanf("");
                i += stride;
                continue;
            }
            eng.load(s.f, i);
            gm.set(pa, pb);
            open = true;
        }
        double v;
        if (gm.step(eng, &zt, &lt, v)) {
            s.z[i] = (float)v;
            eng.store(s.f, i);
            open = false;
            i += stride;
        }
    }
}

// Row i of z (count rows of per_stream = d values) holds the next d normals
// of substream i rounded to binary32.  With d a multiple of 4 each lane
// writes its row as 16-byte pieces.
template <class E, bool BX = false>
__global__ __launch_bounds__(256) void k_norm_rows(SampArgs s)
{
    __shared__ ZigLds zt;
    load_zig<RP_NORM>(&zt, s.f.flags);
    __syncthreads();
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= s.count) return;
    E eng;
    eng.load(s.f, i);
    const uint64_t d = s.f.per_stream;
    float *row = s.z + i * d;
    if ((d & 3) == 0) {
        for (uint64_t t = 0; t < d; t += 4) {
            float4 v;
            eng.reserve(9);  // four normals rarely take more than nine words
            v.x = (float)zig_serial<RP_NORM, BX>(&zt, eng);
            v.y = (float)zig_serial<RP_NORM, BX>(&zt, eng);
            v.z = (float)zig_serial<RP_NORM, BX>(&zt, eng);
            v.w = (float)zig_serial<RP_NORM, BX>(&zt, eng);
            *(float4 *)(row + t) = v;
        }
    } else {
        for (uint64_t t = 0; t < d; t++) {
            eng.reserve(3);
            row[t] = (float)zig_serial<RP_NORM, BX>(&zt, eng);
        }
    }
    if (s.advance) eng.store(s.f, i);
}

// Derived laws that need more than one base draw per value (Table 4):
// chi-square, Student t, F, skew-normal, and gamma / beta with scalar
// parameters, one lane per substream writing its own run of per_stream
// values, each a state machine that takes at most four words per step:
//   GAMMA   theta G,  G ~ Gamma(alpha)              xp = {alpha, theta}
//   BETA    X / (X + Y), X ~ Gamma(a), Y ~ Gamma(b) xp = {a, b}
//   CHI2    2 G, G ~ Gamma(nu / 2)                  xp = {nu / 2}
//   T       Z / sqrt(V / nu), Z normal, then V = 2 G, G ~ Gamma(nu / 2)
//                                                   xp = {nu / 2, nu}
//   F       (X / nu1) / (Y / nu2), X ~ Gamma(nu1 / 2), Y ~ Gamma(nu2 / 2)
//                                                   xp = {nu1 / 2, nu2 / 2}
//   SKEW    mu + sigma (delta |U0| + c U1), U0 then U1 normal,
//           delta = alpha / sqrt(1 + alpha^2), c = sqrt(1 - delta^2)
//                                                   xp = {mu, sigma, delta, c}
// LAWC: the law, with kXfBx for the bitexact setting
template <class E, int LAWC>
__global__ __launch_bounds__(256) void k_fill_mix(FillArgs f)
{
    constexpr int LAW = xf_law(LAWC);
    constexpr bool BX = xf_bx(LAWC);
    __shared__ ZigLds zt;
    __shared__ LogLds lt;
    load_zig<RP_NORM>(&zt, f.flags);
    load_logt(&lt);
    __syncthreads();
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= f.n) return;
    E eng;
    eng.load(f, i);
    const uint64_t P = f.per_stream;
    double *out = (double *)f.out + i * P;
    constexpr int GM = LAW == RP_LAW_BETA ? 1 : (LAW == RP_LAW_F ? 2 : 0);
    GamMachine<GM, false, BX> gm;
    NormMachine nm;
    nm.reset();
    if constexpr (LAW == RP_LAW_GAMMA) gm.set(f.xp[0], 1.0);
    else if constexpr (LAW == RP_LAW_BETA) gm.set(f.xp[0], f.xp[1]);
    else if constexpr (LAW == RP_LAW_F) gm.set(f.xp[0], f.xp[1]);
    else gm.set(f.xp[0], 1.0);
    int phase = 0;  // t and skew-normal: which draw of the value is being made
    double z0 = 0.0;
    for (uint64_t t = 0; t < P;) {
        eng.reserve(4);
        double v;
        if constexpr (LAW == RP_LAW_GAMMA || LAW == RP_LAW_BETA || LAW == RP_LAW_F || LAW == RP_LAW_CHI2) {
            if (gm.step(eng, &zt, &lt, v)) {
                if constexpr (LAW == RP_LAW_GAMMA) v = f.xp[1] * v;
                if constexpr (LAW == RP_LAW_CHI2) v = 2.0 * v;
                out[t++] = v;
            }
        } else if constexpr (LAW == RP_LAW_T) {
            if (phase == 0) {
                if (nm.template step<BX>(eng, &zt, z0)) phase = 1;
            } else if (gm.step(eng, &zt, &lt, v)) {
                out[t++] = z0 / sqrt((2.0 * v) / f.xp[1]);
                phase = 0;
            }
        } else {  // skew-normal
            if (nm.template step<BX>(eng, &zt, v)) {
                if (phase == 0) {
                    z0 = v;
                    phase = 1;
                } else {
                    out[t++] = f.xp[0] + f.xp[1] * (f.xp[2] * fabs(z0) + f.xp[3] * v);
                    phase = 0;
                }
            }
        }
    }
    eng.store(f, i);
}

template <class E, bool BX>
static int launch_mix_e(int law, const FillArgs &f, hipStream_t st)
{
    const dim3 grid((unsigned)((f.n + 255) / 256)), block(256);
    constexpr int B = BX ? kXfBx : 0;
    switch (law) {
    case RP_LAW_GAMMA: hipLaunchKernelGGL((k_fill_mix<E, RP_LAW_GAMMA | B>), grid, block, 0, st, f); break;
    case RP_LAW_BETA: hipLaunchKernelGGL((k_fill_mix<E, RP_LAW_BETA | B>), grid, block, 0, st, f); break;
    case RP_LAW_CHI2: hipLaunchKernelGGL((k_fill_mix<E, RP_LAW_CHI2 | B>), grid, block, 0, st, f); break;
    case RP_LAW_T: hipLaunchKernelGGL((k_fill_mix<E, RP_LAW_T | B>), grid, block, 0, st, f); break;
    case RP_LAW_F: hipLaunchKernelGGL((k_fill_mix<E, RP_LAW_F | B>), grid, block, 0, st, f); break;
    case RP_LAW_SKEWNORMAL: hipLaunchKernelGGL((k_fill_mix<E, RP_LAW_SKEWNORMAL | B>), grid, block, 0, st, f); break;
    default: return fail(RP_EINVAL, "unknown law");
    }
    return RP_OK;
}

// Float gamma (rp_fill_lawf with RP_LAW_GAMMA): theta G rounded to
// binary32, G the float Marsaglia-Tsang draw on the substream's items.
template <class E, bool BX = false>
__global__ __launch_bounds__(256) void k_fill_gammaf(FillArgs f)
{
    __shared__ ZigLds zt;
    __shared__ LogLds lt;
    load_zig<RP_NORM>(&zt, f.flags);
    load_logt(&lt);
    __syncthreads();
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= f.n) return;
    E eng;
    eng.load(f, i);
    ItemEng<E> it(eng);
    const uint64_t P = f.per_stream;
    float *out = (float *)f.out + i * P;
    GamMachine<0, true, BX> gm;
    gm.set(f.xp[0], 1.0);
    for (uint64_t t = 0; t < P;) {
        double v;
        if (gm.step(it, &zt, &lt, v)) out[t++] = (float)(f.xp[1] * v);
    }
    eng.store(f, i);
}

// Float versions of the laws of several draws (rp_fill_lawf): the float
// gamma (GamMachine on 32-bit items, binary64, unrounded) and the binary32
// normal of the float ziggurat, combined as in k_fill_mix, in binary64, and
// rounded once to binary32.  xp as for k_fill_mix.
template <class E, int LAWC>
__global__ __launch_bounds__(256) void k_fill_mixf(FillArgs f)
{
    constexpr int LAW = xf_law(LAWC);
    constexpr bool BX = xf_bx(LAWC);
    __shared__ ZigLds zt;
    __shared__ LogLds lt;
    load_zig<RP_NORM>(&zt, f.flags);
    load_logt(&lt);
    __syncthreads();
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= f.n) return;
    E eng;
    eng.load(f, i);
    ItemEng<E> it(eng);
    const uint64_t P = f.per_stream;
    float *out = (float *)f.out + i * P;
    constexpr int GM = LAW == RP_LAW_BETA ? 1 : (LAW == RP_LAW_F ? 2 : 0);
    GamMachine<GM, true, BX> gm;
    if constexpr (LAW == RP_LAW_BETA || LAW == RP_LAW_F) gm.set(f.xp[0], f.xp[1]);
    else gm.set(f.xp[0], 1.0);
    for (uint64_t t = 0; t < P;) {
        double v;
        if constexpr (LAW == RP_LAW_BETA || LAW == RP_LAW_F || LAW == RP_LAW_CHI2) {
            if (gm.step(it, &zt, &lt, v)) {
                if constexpr (LAW == RP_LAW_CHI2) v = 2.0 * v;
                out[t++] = (float)v;
            }
        } else if constexpr (LAW == RP_LAW_T) {
            double z;
            while (!zig_candidate<ItemEng<E>, true, BX>(it, &zt, z)) {
            }
            while (!gm.step(it, &zt, &lt, v)) {
            }
            out[t++] = (float)(z / sqrt((2.0 * v) / f.xp[1]));
        } else {  // skew-normal
            double z0, z1;
            while (!zig_candidate<ItemEng<E>, true, BX>(it, &zt, z0)) {
            }
            while (!zig_candidate<ItemEng<E>, true, BX>(it, &zt, z1)) {
            }
            out[t++] = (float)(f.xp[0] + f.xp[1] * (f.xp[2] * fabs(z0) + f.xp[3] * z1));
        }
    }
    eng.store(f, i);
}

template <class E, bool BX>
static int launch_mix_bx(int law, bool f32, const FillArgs &f, hipStream_t st)
{
    if (!f32) return launch_mix_e<E, BX>(law, f, st);
    const dim3 grid((unsigned)((f.n + 255) / 256)), block(256);
    constexpr int B = BX ? kXfBx : 0;
    switch (law) {
    case RP_LAW_GAMMA: hipLaunchKernelGGL((k_fill_gammaf<E, BX>), grid, block, 0, st, f); break;
    case RP_LAW_BETA: hipLaunchKernelGGL((k_fill_mixf<E, RP_LAW_BETA | B>), grid, block, 0, st, f); break;
    case RP_LAW_CHI2: hipLaunchKernelGGL((k_fill_mixf<E, RP_LAW_CHI2 | B>), grid, block, 0, st, f); break;
    case RP_LAW_T: hipLaunchKernelGGL((k_fill_mixf<E, RP_LAW_T | B>), grid, block, 0, st, f); break;
    case RP_LAW_F: hipLaunchKernelGGL((k_fill_mixf<E, RP_LAW_F | B>), grid, block, 0, st, f); break;
    case RP_LAW_SKEWNORMAL: hipLaunchKernelGGL((k_fill_mixf<E, RP_LAW_SKEWNORMAL | B>), grid, block, 0, st, f); break;
    default: return fail(RP_EINVAL, "unknown law");
    }
    return RP_OK;
}

template <class E>
static int launch_mix_any(int law, bool f32, const FillArgs &f, hipStream_t st)
{
    return (f.flags & kFlagBitexact) ? launch_mix_bx<E, true>(law, f32, f, st) : launch_mix_bx<E, false>(law, f32, f, st);
}

int launch_fill_mix(int engine, int law, bool f32, const FillArgs &f, hipStream_t st)
{
    int rc;
    switch (engine) {
    case RP_X256PP: rc = launch_mix_any<LaneX256>(law, f32, f, st); break;
    case RP_X256SS: rc = launch_mix_any<LaneX256SS>(law, f32, f, st); break;
    case RP_SQUARES: rc = launch_mix_any<LaneSquares>(law, f32, f, st); break;
    case RP_XORO128: rc = launch_mix_any<LaneXoro128>(law, f32, f, st); break;
    case RP_XS128: rc = launch_mix_any<LaneXs128>(law, f32, f, st); break;
    case RP_CHACHA20: rc = launch_mix_any<LaneChacha>(law, f32, f, st); break;
    case RP_PCG64: rc = launch_mix_any<LanePcg>(law, f32, f, st); break;
    case RP_PHILOX4X32: rc = launch_mix_any<LanePhilox32>(law, f32, f, st); break;
    case RP_PHILOX: rc = launch_mix_any<LanePhilox64>(law, f32, f, st); break;
    case RP_SFC64: rc = launch_mix_any<LaneSfc64>(law, f32, f, st); break;
    case RP_CWG128: rc = launch_mix_any<LaneCwg128>(law, f32, f, st); break;
    case RP_X256PPS: rc = launch_mix_any<LaneX256Simd>(law, f32, f, st); break;
    case RP_X256SSS: rc = launch_mix_any<LaneX256SSSimd>(law, f32, f, st); break;
    case RP_SFC64S: rc = launch_mix_any<LaneSfc64Simd>(law, f32, f, st); break;
    case RP_RANLUX: rc = launch_mix_any<LaneRanlux>(law, f32, f, st); break;
    default: return fail(RP_EINVAL, "unknown engine");
    }
    if (rc) return rc;
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? RP_OK : fail(RP_EDEVICE, "law fill launch: %s", hipGetErrorString(e));
}

template <class E>
static int launch_moments_e(const SampArgs &s, hipStream_t st)
{
    const uint64_t blocks = (s.count + 255) / 256;
    if (s.f.flags & kFlagBitexact)
        hipLaunchKernelGGL((k_norm_moments<E, true>), dim3((unsigned)blocks), dim3(256), 0, st, s);
    else
        hipLaunchKernelGGL((k_norm_moments<E, false>), dim3((unsigned)blocks), dim3(256), 0, st, s);
    return RP_OK;
}

template <class E>
static int launch_elem_e(const SampArgs &s, bool beta, hipStream_t st)
{
    uint64_t blocks = (s.count + 255) / 256;
    if (blocks > 4096) blocks = 4096;  // lanes then take several elements each
    const bool bx = (s.f.flags & kFlagBitexact) != 0;
    if (beta && bx)
        hipLaunchKernelGGL((k_gamma_elem<E, true, true>), dim3((unsigned)blocks), dim3(256), 0, st, s);
    else if (beta)
        hipLaunchKernelGGL((k_gamma_elem<E, true, false>), dim3((unsigned)blocks), dim3(256), 0, st, s);
    else if (bx)
        hipLaunchKernelGGL((k_gamma_elem<E, false, true>), dim3((unsigned)blocks), dim3(256), 0, st, s);
    else
        hipLaunchKernelGGL((k_gamma_elem<E, false, false>), dim3((unsigned)blocks), dim3(256), 0, st, s);
    return RP_OK;
}

int launch_moments(int engine, const SampArgs &s, hipStream_t st)
{
    switch (engine) {
    case RP_X256PP: launch_moments_e<LaneX256>(s, st); break;
    case RP_X256SS: launch_moments_e<LaneX256SS>(s, st); break;
    case RP_SQUARES: launch_moments_e<LaneSquares>(s, st); break;
    case RP_XORO128: launch_moments_e<LaneXoro128>(s, st); break;
    case RP_XS128: launch_moments_e<LaneXs128>(s, st); break;
    case RP_CHACHA20: launch_moments_e<LaneChacha>(s, st); break;
    case RP_PCG64: launch_moments_e<LanePcg>(s, st); break;
    case RP_PHILOX4X32: launch_moments_e<LanePhilox32>(s, st); break;
    case RP_PHILOX: launch_moments_e<LanePhilox64>(s, st); break;
    case RP_SFC64: launch_moments_e<LaneSfc64>(s, st); break;
    case RP_CWG128: launch_moments_e<LaneCwg128>(s, st); break;
    case RP_X256PPS: launch_moments_e<LaneX256Simd>(s, st); break;
    case RP_X256SSS: launch_moments_e<LaneX256SSSimd>(s, st); break;
    case RP_SFC64S: launch_moments_e<LaneSfc64Simd>(s, st); break;
    case RP_RANLUX: launch_moments_e<LaneRanlux>(s, st); break;
    default: return fail(RP_EINVAL, "unknown engine");
    }
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? RP_OK : fail(RP_EDEVICE, "moments launch: %s", hipGetErrorString(e));
}

template <class E>
static void launch_rows_e(const SampArgs &s, dim3 grid, dim3 block, hipStream_t st)
{
    if (s.f.flags & kFlagBitexact) hipLaunchKernelGGL((k_norm_rows<E, true>), grid, block, 0, st, s);
    else hipLaunchKernelGGL((k_norm_rows<E, false>), grid, block, 0, st, s);
}

int launch_norm_rows(int engine, const SampArgs &s, hipStream_t st)
{
    const dim3 grid((unsigned)((s.count + 255) / 256)), block(256);
    switch (engine) {
    case RP_X256PP: launch_rows_e<LaneX256>(s, grid, block, st); break;
    case RP_X256SS: launch_rows_e<LaneX256SS>(s, grid, block, st); break;
    case RP_SQUARES: launch_rows_e<LaneSquares>(s, grid, block, st); break;
    case RP_XORO128: launch_rows_e<LaneXoro128>(s, grid, block, st); break;
    case RP_XS128: launch_rows_e<LaneXs128>(s, grid, block, st); break;
    case RP_CHACHA20: launch_rows_e<LaneChacha>(s, grid, block, st); break;
    case RP_PCG64: launch_rows_e<LanePcg>(s, grid, block, st); break;
    case RP_PHILOX4X32: launch_rows_e<LanePhilox32>(s, grid, block, st); break;
    case RP_PHILOX: launch_rows_e<LanePhilox64>(s, grid, block, st); break;
    case RP_SFC64: launch_rows_e<LaneSfc64>(s, grid, block, st); break;
    case RP_CWG128: launch_rows_e<LaneCwg128>(s, grid, block, st); break;
    case RP_X256PPS: launch_rows_e<LaneX256Simd>(s, grid, block, st); break;
    case RP_X256SSS: launch_rows_e<LaneX256SSSimd>(s, grid, block, st); break;
    case RP_SFC64S: launch_rows_e<LaneSfc64Simd>(s, grid, block, st); break;
    case RP_RANLUX: launch_rows_e<LaneRanlux>(s, grid, block, st); break;
    default: return fail(RP_EINVAL, "unknown engine");
    }
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? RP_OK : fail(RP_EDEVICE, "normal rows launch: %s", hipGetErrorString(e));
}

int launch_gamma_elem(int engine, const SampArgs &s, bool beta, hipStream_t st)
{
    switch (engine) {
    case RP_X256PP: launch_elem_e<LaneX256>(s, beta, st); break;
    case RP_X256SS: launch_elem_e<LaneX256SS>(s, beta, st); break;
    case RP_SQUARES: launch_elem_e<LaneSquares>(s, beta, st); break;
    case RP_XORO128: launch_elem_e<LaneXoro128>(s, beta, st); break;
    case RP_XS128: launch_elem_e<LaneXs128>(s, beta, st); break;
    case RP_CHACHA20: launch_elem_e<LaneChacha>(s, beta, st); break;
    case RP_PCG64: launch_elem_e<LanePcg>(s, beta, st); break;
    case RP_PHILOX4X32: launch_elem_e<LanePhilox32>(s, beta, st); break;
    case RP_PHILOX: launch_elem_e<LanePhilox64>(s, beta, st); break;
    case RP_SFC64: launch_elem_e<LaneSfc64>(s, beta, st); break;
    case RP_CWG128: launch_elem_e<LaneCwg128>(s, beta, st); break;
    case RP_X256PPS: launch_elem_e<LaneX256Simd>(s, beta, st); break;
    case RP_X256SSS: launch_elem_e<LaneX256SSSimd>(s, beta, st); break;
    case RP_SFC64S: launch_elem_e<LaneSfc64Simd>(s, beta, st); break;
    case RP_RANLUX: launch_elem_e<LaneRanlux>(s, beta, st); break;
    default: return fail(RP_EINVAL, "unknown engine");
    }
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? RP_OK : fail(RP_EDEVICE, "gamma launch: %s", hipGetErrorString(e));
}
