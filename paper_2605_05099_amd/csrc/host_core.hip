// host_core.hip -- host side of the C ABI: handles, errors, seeding, stream
// control (jump / advance / setters), substream construction and dispatch.
//
// Section 2.1 (interface), Section 2.3 (seeding, substreams, Table 3),
// Section 4.4 (thread safety, serialization, engine query, jumping).
#include <hip/hip_runtime.h>

#include <sys/random.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cctype>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>

#include "rp_internal.h"

using namespace rp;

// ---------------------------------------------------------------------------
// errors (per thread for handle-less calls, per handle otherwise)
static thread_local std::string t_err;

namespace rp {

static void vformat(std::string &dst, const char *fmt, va_list ap)
{
    char buf[512];
    vsnprintf(buf, sizeof buf, fmt, ap);
    dst = buf;
}

void set_error(const char *fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vformat(t_err, fmt, ap);
    va_end(ap);
}

void set_error_rng(rp_rng *rng, const char *fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vformat(t_err, fmt, ap);
    va_end(ap);
    if (rng) rng->err = t_err;
}

int fail(int code, const char *fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vformat(t_err, fmt, ap);
    va_end(ap);
    return code;
}

}  // namespace rp

static int fail_rng(const rp_rng *rng, int code, const char *fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vformat(t_err, fmt, ap);
    va_end(ap);
    if (rng) const_cast<rp_rng *>(rng)->err = t_err;
    return code;
}

// ---------------------------------------------------------------------------
// engine table (Table 2)
struct EngineInfo {
    const char *id;
    const char *desc;
    int words;  // state words (Table 2 "State words"; philox4x32: counter 2 + key 1)
    int block;  // 64-bit words per output block
};

static const EngineInfo kEngines[RP_NENGINES] = {
    {"x256++", "xoshiro256++ (Vigna and Blackman, 2019), 4 state words, period 2^256-1", 4, 1},
    {"pcg64", "PCG64 DXSM (O'Neill, 2019), 4 state words, period 2^128 per increment", 4, 1},
    {"philox4x32", "Philox4x32-10 (Salmon and Moraes, 2011), 3 state words, period 2^129 per key", 3, 2},
    {"philox", "Philox-4x64-10 (Salmon and Moraes, 2011), 6 state words, period 2^258 per key", 6, 4},
    {"sfc64", "sfc64 (Chris Doty-Humphrey, 2010), 4 state words, average period >= 2^64", 4, 1},
    {"ranlux++", "ranlux++ (Sibidanov, 2017), 9 state words, period about 2^570", 9, 9},
    {"x256**", "xoshiro256** (Blackman and Vigna, 2018), 4 state words, period 2^256-1", 4, 1},
    {"squares", "squares64 (Widynski, 2021), 2 state words, period 2^64 per key", 2, 1},
    {"xoro++", "xoroshiro128++ (Blackman and Vigna, 2019), 2 state words, period 2^128-1", 2, 1},
    {"x128+", "xorshift128+ (Vigna, 2014), 2 state words, period 2^128-1", 2, 1},
    {"chacha20", "ChaCha20 (Bernstein, 2008), 6 state words, period 2^35 per nonce", 6, 8},
    {"cwg128", "cwg128 (Dziala, 2022), 8 state words, period 2^128 per Weyl increment", 8, 1},
    {"x256++simd", "xoshiro256++ x 8 interleaved (Vigna and Blackman, 2019), 32 state words", 32, 8},
    {"x256**simd", "xoshiro256** x 8 interleaved (Blackman and Vigna, 2018), 32 state words", 32, 8},
    {"sfc64simd", "sfc64 x 8 interleaved (Chris Doty-Humphrey, 2010), 32 state words", 32, 8},
};

namespace {
bool is_simd(int e) { return e == RP_X256PPS || e == RP_X256SSS || e == RP_SFC64S; }
bool is_x256(int e) { return e == RP_X256PP || e == RP_X256SS || e == RP_X256PPS || e == RP_X256SSS; }
}  // namespace

namespace rp {
int state_words(int e) { return kEngines[e].words; }
int block_words(int e) { return kEngines[e].block; }
}  // namespace rp

extern "C" const char *rp_errmsg(void) { return t_err.c_str(); }

extern "C" const char *rp_last_error(const rp_rng *rng)
{
    if (!rng) return t_err.c_str();
    return rng->err.c_str();
}

extern "C" int rp_engines(char *buf, size_t len)
{
    std::string s;
    for (const auto &e : kEngines) {
        s += e.id;
        s += ": ";
        s += e.desc;
        s += "\n";
    }
    if (buf && len > 0) {
        size_t n = std::min(len - 1, s.size());
        memcpy(buf, s.data(), n);
        buf[n] = 0;
    }
    return (int)s.size();
}

extern "C" int rp_engine_id(const char *name)
{
    if (!name) return fail(RP_ENULL, "rp_engine_id: NULL name");
    for (int e = 0; e < RP_NENGINES; e++) {
        const char *a = kEngines[e].id;
        const char *b = name;
        while (*a && *b && std::tolower((unsigned char)*a) == std::tolower((unsigned char)*b)) {
            a++;
            b++;
        }
        if (!*a && !*b) return e;
    }
    return fail(RP_EINVAL, "unknown engine identifier '%s'", name);
}

// ---------------------------------------------------------------------------
// seed_seq_fe128 mixer (Section 2.3): a 128-bit entropy pool of four 32-bit
// words.  Input words are hashed into the pool (short inputs padded with
// hashed zeros), every pool word is mixed with a hash of every other, any
// further input words are mixed into all pool words, and output words are
// produced by hashing the pool words round-robin with a second hash sequence.
namespace {
class SeedMixer {
  public:
    explicit SeedMixer(const std::vector<uint32_t> &in)
    {
        uint32_t mult = kInitA;
        auto hash = [&mult](uint32_t v) {
            v ^= mult;
            mult *= kMultA;
            v *= mult;
            return v ^ (v >> 16);
        };
        auto mix = [](uint32_t x, uint32_t y) {
            uint32_t r = kMixL * x - kMixR * y;
            return r ^ (r >> 16);
        };
        for (size_t i = 0; i < 4; i++) pool_[i] = hash(i < in.size() ? in[i] : 0u);
        for (size_t s = 0; s < 4; s++)
            for (size_t d = 0; d < 4; d++)
                if (s != d) pool_[d] = mix(pool_[d], hash(pool_[s]));
        for (size_t i = 4; i < in.size(); i++)
            for (size_t d = 0; d < 4; d++) pool_[d] = mix(pool_[d], hash(in[i]));
    }
    void generate(uint32_t *out, size_t n) const
    {
        uint32_t mult = kInitB;
        for (size_t i = 0; i < n; i++) {
            uint32_t v = pool_[i & 3] ^ mult;
            mult *= kMultB;
            v *= mult;
            out[i] = v ^ (v >> 16);
        }
    }

  private:
    static constexpr uint32_t kInitA = 0x43b0d7e5u, kMultA = 0x931e8875u;
    static constexpr uint32_t kInitB = 0x8b51f9ddu, kMultB = 0x58f38dedu;
    static constexpr uint32_t kMixL = 0xca01f9ddu, kMixR = 0x4973f715u;
    uint32_t pool_[4];
};
}  // namespace

// ---------------------------------------------------------------------------
// ranlux++ constants: m = 2^576 - 2^240 + 1, a = m - (m - 1) / 2^24 (the LCG
// equivalent of RANLUX with base 2^24, lags 24 and 10), A = a^2048 (the luxury
// taken: 2048 subtract-with-borrow steps per engine step).
static void ranlux_base(uint64_t a[9])
{
    // m - 1 = 2^576 - 2^240;  (m - 1) / 2^24 = 2^552 - 2^216
    // a = m - (2^552 - 2^216) = 2^576 - 2^552 - 2^240 + 2^216 + 1
    // limbs: 2^576 - 2^552 = (2^24 - 1) 2^552 -> limb 8 bits 40..63 set
    uint64_t v[9] = {0};
    v[8] = 0xFFFFFF0000000000ull;             // 2^576 - 2^552
    // subtract 2^240 (limb 3, bit 48), add 2^216 (limb 3, bit 24), add 1
    // 2^216 - 2^240 = -(2^240 - 2^216) = -(2^24 - 1) 2^216
    // v - (2^24-1) 2^216: borrow from limb 8 through limbs 4..7
    uint64_t sub = ((1ull << 24) - 1) << 24;  // (2^24 - 1) 2^216 in limb 3
    // v[3] = 0 - sub with borrow propagating to limb 8
    v[3] = 0 - sub;
    for (int k = 4; k < 8; k++) v[k] = ~0ull;  // borrow chain 0 - 1
    v[8] -= 1;
    v[0] = 1;
    memcpy(a, v, sizeof v);
}

static uint64_t g_rl_A[9];
static std::once_flag g_rl_once;

namespace rp {
const uint64_t *ranlux_A()
{
    std::call_once(g_rl_once, [] {
        uint64_t a[9], acc[9] = {1}, base[9];
        ranlux_base(a);
        memcpy(base, a, sizeof a);
        for (uint32_t e = 2048; e; e >>= 1) {
            if (e & 1) rl_mulmod(acc, base, acc);
            rl_mulmod(base, base, base);
        }
        memcpy(g_rl_A, acc, sizeof acc);
    });
    return g_rl_A;
}

// B[j * 20 + i] = limb j (29 bits) of 2^(29 i) A mod m, the table of the
// folded generator step (engines.h)
const uint32_t *ranlux_B()
{
    static uint32_t B[kRlL * kRlL];
    static std::once_flag once;
    std::call_once(once, [] {
        const uint64_t *A = ranlux_A();
        for (int i = 0; i < kRlL; i++) {
            uint64_t t[9] = {0}, y[9];
            t[(29 * i) / 64] = 1ull << ((29 * i) % 64);
            rl_mulmod(A, t, y);
            for (int j = 0; j < kRlL; j++) {
                const int p = 29 * j, w = p / 64, off = p % 64;
                uint64_t v = y[w] >> off;
                if (off > 35 && w + 1 < 9) v |= y[w + 1] << (64 - off);
                B[j * kRlL + i] = (uint32_t)(v & kRlM29);
            }
        }
    });
    return B;
}
}  // namespace rp

// base^e (e given as 64-bit limbs, little-endian) mod m
static void ranlux_pow(const uint64_t base_in[9], const uint64_t *e, int ne, uint64_t out[9])
{
    uint64_t acc[9] = {1}, b[9];
    memcpy(b, base_in, sizeof b);
    for (int i = 0; i < ne; i++)
        for (int bit = 0; bit < 64; bit++) {
            if ((e[i] >> bit) & 1) rl_mulmod(acc, b, acc);
            rl_mulmod(b, b, b);
        }
    memcpy(out, acc, sizeof acc);
}

static void ranlux_fixup(uint64_t x[9])
{
    uint64_t p[18] = {0};
    memcpy(p, x, 9 * 8);
    rl_reduce(p, x);
    bool zero = true;
    for (int k = 0; k < 9; k++) zero = zero && x[k] == 0;
    if (zero) x[0] = 1;
}

// ---------------------------------------------------------------------------
// xoshiro256 jump polynomials (Section 4.4 "Jumping"): T^N = p(T) with
// p(x) = x^N mod P(x), P the characteristic polynomial of the linear core.
// P is found with the Berlekamp-Massey algorithm from 512 output bits of
// one state bit; polynomials over GF(2) are 5 x 64-bit bitsets.
namespace {
struct Poly {
    uint64_t w[5] = {0, 0, 0, 0, 0};
    bool bit(int i) const { return (w[i >> 6] >> (i & 63)) & 1; }
    void flip(int i) { w[i >> 6] ^= 1ull << (i & 63); }
};

Poly g_charpoly;
std::once_flag g_charpoly_once;

const Poly &x256_charpoly()
{
    std::call_once(g_charpoly_once, [] {
        X256 s{0x9E3779B97F4A7C15ull, 0x3C6EF372FE94F82Aull, 0xDAA66D2C7DDF743Full, 1};
        std::vector<int> bits(512);
        for (int i = 0; i < 512; i++) {
            bits[i] = (int)(s.s0 & 1);
            s.linear();
        }
        // Berlekamp-Massey over GF(2): connection polynomial C (degree L)
        std::vector<int> C(513, 0), B(513, 0), T;
        C[0] = B[0] = 1;
        int L = 0, m = 1;
        for (int n = 0; n < 512; n++) {
            int d = bits[n];
            for (int i = 1; i <= L; i++) d ^= C[i] & bits[n - i];
            if (!d) {
                m++;
                continue;
            }
            T = C;
            for (int i = 0; i + m <= 512; i++) C[i + m] ^= B[i];
            if (2 * L <= n) {
                L = n + 1 - L;
                B = T;
                m = 1;
            } else {
                m++;
            }
        }
        // characteristic polynomial = reciprocal of C: P(x) = x^L C(1/x)
        Poly p;
        for (int i = 0; i <= L; i++)
            if (C[i]) p.flip(L - i);
        g_charpoly = p;  // L is 256 (primitive polynomial of degree 256)
    });
    return g_charpoly;
}

// a * x mod P (deg P = 256)
void poly_mulx(Poly &a, const Poly &P)
{
    uint64_t carry = 0;
    for (int k = 0; k < 5; k++) {
        uint64_t nc = a.w[k] >> 63;
        a.w[k] = (a.w[k] << 1) | carry;
        carry = nc;
    }
    if (a.bit(256))
        for (int k = 0; k < 5; k++) a.w[k] ^= P.w[k];
}

Poly poly_mulmod(const Poly &a, const Poly &b, const Poly &P)
{
    Poly r;
    for (int i = 255; i >= 0; i--) {
        poly_mulx(r, P);
        if (b.bit(i))
            for (int k = 0; k < 5; k++) r.w[k] ^= a.w[k];
    }
    return r;
}

// x^N mod P for N = lo + hi 2^64
Poly poly_xpow(uint64_t lo, uint64_t hi, const Poly &P)
{
    Poly r, base;
    r.flip(0);
    base.flip(1);
    for (int half = 0; half < 2; half++) {
        uint64_t e = half ? hi : lo;
        for (int bit = 0; bit < 64; bit++) {
            if ((e >> bit) & 1) r = poly_mulmod(r, base, P);
            base = poly_mulmod(base, base, P);
        }
    }
    return r;
}

// degree-D versions for the 128-bit xor engines (D = 128)
template <int D>
void poly_mulx_d(Poly &a, const Poly &P)
{
    uint64_t carry = 0;
    for (int k = 0; k < 5; k++) {
        uint64_t nc = a.w[k] >> 63;
        a.w[k] = (a.w[k] << 1) | carry;
        carry = nc;
    }
    if (a.bit(D))
        for (int k = 0; k < 5; k++) a.w[k] ^= P.w[k];
}

template <int D>
Poly poly_mulmod_d(const Poly &a, const Poly &b, const Poly &P)
{
    Poly r;
    for (int i = D - 1; i >= 0; i--) {
        poly_mulx_d<D>(r, P);
        if (b.bit(i))
            for (int k = 0; k < 5; k++) r.w[k] ^= a.w[k];
    }
    return r;
}

template <int D>
Poly poly_xpow_d(uint64_t lo, uint64_t hi, const Poly &P)
{
    Poly r, base;
    r.flip(0);
    base.flip(1);
    for (int half = 0; half < 2; half++) {
        uint64_t e = half ? hi : lo;
        for (int bit = 0; bit < 64; bit++) {
            if ((e >> bit) & 1) r = poly_mulmod_d<D>(r, base, P);
            base = poly_mulmod_d<D>(base, base, P);
        }
    }
    return r;
}

// characteristic polynomial of a 2-word linear core from 256 output bits
// (Berlekamp-Massey over GF(2); the reciprocal of the connection polynomial)
template <class S>
Poly x128_charpoly_of()
{
    S s{0x0123456789ABCDEFull, 0x0F1E2D3C4B5A6978ull};
    std::vector<int> bits(256);
    for (int i = 0; i < 256; i++) {
        bits[i] = (int)(s.s0 & 1);
        s.linear();
    }
    std::vector<int> C(257, 0), B(257, 0), T;
    C[0] = B[0] = 1;
    int L = 0, m = 1;
    for (int n = 0; n < 256; n++) {
        int d = bits[n];
        for (int i = 1; i <= L; i++) d ^= C[i] & bits[n - i];
        if (!d) {
            m++;
            continue;
        }
        T = C;
        for (int i = 0; i + m <= 256; i++) C[i + m] ^= B[i];
        if (2 * L <= n) {
            L = n + 1 - L;
            B = T;
            m = 1;
        } else {
            m++;
        }
    }
    Poly p;
    for (int i = 0; i <= L; i++)
        if (C[i]) p.flip(L - i);
    return p;  // L is 128 (primitive of degree 128)
}

const Poly &x128_charpoly(int engine)
{
    static const Poly xoro = x128_charpoly_of<Xoro128>();
    static const Poly xs = x128_charpoly_of<Xs128>();
    return engine == RP_XORO128 ? xoro : xs;
}

template <class S>
void x128_apply_s(uint64_t st[2], const Poly &p)
{
    S cur{st[0], st[1]};
    uint64_t a0 = 0, a1 = 0;
    for (int k = 0; k < 128; k++) {
        if (p.bit(k)) {
            a0 ^= cur.s0;
            a1 ^= cur.s1;
        }
        cur.linear();
    }
    st[0] = a0;
    st[1] = a1;
}

void x128_apply(int engine, uint64_t st[2], const Poly &p)
{
    if (engine == RP_XORO128) x128_apply_s<Xoro128>(st, p);
    else x128_apply_s<Xs128>(st, p);
}

void x256_apply(uint64_t st[4], const Poly &p)
{
    X256 cur{st[0], st[1], st[2], st[3]};
    uint64_t acc[4] = {0, 0, 0, 0};
    for (int k = 0; k < 256; k++) {
        if (p.bit(k)) {
            acc[0] ^= cur.s0;
            acc[1] ^= cur.s1;
            acc[2] ^= cur.s2;
            acc[3] ^= cur.s3;
        }
        cur.linear();
    }
    memcpy(st, acc, sizeof acc);
}
}  // namespace

// ---------------------------------------------------------------------------
// PCG64 affine powering: stepping N times maps s to A^N s + G_N inc with
// G_N = 1 + A + ... + A^(N-1); binary powering composes the maps for 2^k.
static PcgAffine pcg_power(uint64_t lo, uint64_t hi)
{
    PcgAffine acc{{1, 0}, {0, 0}};
    PcgAffine cur{{kPcgMult, 0}, {1, 0}};
    for (int half = 0; half < 2; half++) {
        uint64_t e = half ? hi : lo;
        for (int bit = 0; bit < 64; bit++) {
            if ((e >> bit) & 1) {
                // acc <- cur o acc : s -> cur.m (acc.m s + acc.p inc) + cur.p inc
                acc.plus = add128(mul128(cur.mult, acc.plus), cur.plus);
                acc.mult = mul128(cur.mult, acc.mult);
            }
            // cur <- cur o cur
            cur.plus = add128(mul128(cur.mult, cur.plus), cur.plus);
            cur.mult = mul128(cur.mult, cur.mult);
        }
    }
    return acc;
}

// ---------------------------------------------------------------------------
// stepping on the host (state checks, sfc64 warm-up)
static uint64_t host_next(rp_rng *r)
{
    uint64_t *st = r->st;
    switch (r->engine) {
    case RP_X256PP:
    case RP_X256SS: {
        X256 s{st[0], st[1], st[2], st[3]};
        uint64_t w = r->engine == RP_X256SS ? s.next_ss() : s.next();
        st[0] = s.s0; st[1] = s.s1; st[2] = s.s2; st[3] = s.s3;
        return w;
    }
    case RP_PCG64: {
        u128 s{st[0], st[1]}, inc{st[2], st[3]};
        uint64_t w = pcg_dxsm(s);
        s = pcg_step(s, inc);
        st[0] = s.lo;
        st[1] = s.hi;
        return w;
    }
    case RP_SQUARES:
        return squares64(st[0]++, st[1]);
    case RP_XORO128: {
        Xoro128 s{st[0], st[1]};
        const uint64_t w = s.next();
        st[0] = s.s0;
        st[1] = s.s1;
        return w;
    }
    case RP_XS128: {
        Xs128 s{st[0], st[1]};
        const uint64_t w = s.next();
        st[0] = s.s0;
        st[1] = s.s1;
        return w;
    }
    case RP_SFC64: {
        Sfc64 s{st[0], st[1], st[2], st[3]};
        uint64_t w = s.next();
        st[0] = s.a; st[1] = s.b; st[2] = s.c; st[3] = s.ctr;
        return w;
    }
    case RP_X256PPS:
    case RP_X256SSS:
    case RP_SFC64S: {
        // word `phase` of the round: sub-stream `phase`'s next word, taken
        // from a copy; all eight sub-streams move once the round is used
        uint64_t *l = st + 4 * r->phase;
        uint64_t w;
        if (r->engine == RP_SFC64S) {
            Sfc64 c{l[0], l[1], l[2], l[3]};
            w = c.next();
        } else {
            X256 c{l[0], l[1], l[2], l[3]};
            w = r->engine == RP_X256SSS ? c.next_ss() : c.next();
        }
        if (++r->phase == 8) {
            r->phase = 0;
            for (int k = 0; k < 8; k++) {
                uint64_t *m = st + 4 * k;
                if (r->engine == RP_SFC64S) {
                    Sfc64 c{m[0], m[1], m[2], m[3]};
                    (void)c.next();
                    m[0] = c.a; m[1] = c.b; m[2] = c.c; m[3] = c.ctr;
                } else {
                    X256 c{m[0], m[1], m[2], m[3]};
                    c.linear();
                    m[0] = c.s0; m[1] = c.s1; m[2] = c.s2; m[3] = c.s3;
                }
            }
        }
        return w;
    }
    case RP_CWG128: {
        Cwg128 g{{st[0], st[1]}, {st[2], st[3]}, {st[4], st[5]}, {st[6], st[7]}};
        const uint64_t w = g.next();
        st[0] = g.x.lo; st[1] = g.x.hi; st[2] = g.a.lo; st[3] = g.a.hi;
        st[4] = g.w.lo; st[5] = g.w.hi;
        return w;
    }
    case RP_PHILOX4X32: {
        uint64_t w0, w1;
        philox4x32(st[0], st[1], st[2], w0, w1);
        uint64_t w = r->phase ? w1 : w0;
        if (++r->phase == 2) {
            r->phase = 0;
            st[0] += 1;
            if (st[0] == 0) st[1] += 1;
        }
        return w;
    }
    case RP_CHACHA20: {
        uint32_t key[8];
        for (int k = 0; k < 4; k++) {
            key[2 * k] = (uint32_t)st[k];
            key[2 * k + 1] = (uint32_t)(st[k] >> 32);
        }
        uint64_t o[8];
        chacha20_block(key, (uint32_t)st[4], (uint32_t)(st[4] >> 32), (uint32_t)st[5], (uint32_t)(st[5] >> 32), o);
        uint64_t w = o[r->phase];
        if (++r->phase == 8) {
            r->phase = 0;
            st[5] = (st[5] & 0xffffffffull) | ((uint64_t)(uint32_t)((st[5] >> 32) + 1u) << 32);
        }
        return w;
    }
    case RP_PHILOX: {
        uint64_t o[4];
        philox4x64(st, st[4], st[5], o);
        uint64_t w = o[r->phase];
        if (++r->phase == 4) {
            r->phase = 0;
            for (int k = 0; k < 4; k++)
                if (++st[k] != 0) break;
        }
        return w;
    }
    case RP_RANLUX: {
        uint64_t y[9];
        rl_mul_tab(st, ranlux_B(), y);
        uint64_t w = y[r->phase];
        if (++r->phase == 9) {
            r->phase = 0;
            memcpy(st, y, sizeof y);
        }
        return w;
    }
    }
    return 0;
}

static void sfc64_setabc(rp_rng *r, uint64_t a, uint64_t b, uint64_t c)
{
    r->st[0] = a;
    r->st[1] = b;
    r->st[2] = c;
    r->st[3] = 1;
    r->phase = 0;
    for (int i = 0; i < 18; i++) host_next(r);
}

// SIMD engines (Section 4.1): the eight sub-streams from the scalar base
// state: xoshiro sub-stream k is the base jumped by k 2^253 steps (x^(2^253)
// mod P applied k times), sfc64 sub-stream k has k 2^61 added to the counter.
static const Poly &x256_lane_jump()
{
    static const Poly J = [] {
        Poly x;
        x.flip(1);
        const Poly &P = x256_charpoly();
        for (int i = 0; i < 253; i++) x = poly_mulmod(x, x, P);
        return x;
    }();
    return J;
}

static void simd_from_base(rp_rng *r, const uint64_t base[4])
{
    uint64_t cur[4];
    memcpy(cur, base, sizeof cur);
    for (int k = 0; k < 8; k++) {
        if (r->engine == RP_SFC64S) {
            memcpy(r->st + 4 * k, base, 24);
            r->st[4 * k + 3] = base[3] + ((uint64_t)k << 61);
        } else {
            memcpy(r->st + 4 * k, cur, sizeof cur);
            x256_apply(cur, x256_lane_jump());
        }
    }
    r->phase = 0;
}

// the scalar engine a SIMD engine interleaves
static int simd_base_engine(int e)
{
    return e == RP_X256PPS ? RP_X256PP : e == RP_X256SSS ? RP_X256SS : RP_SFC64;
}

// cwg128 stream setter: the Weyl increment made odd, then 96 warm-up steps
// (Table 3 caption); x, a and the Weyl sequence are kept.
static void cwg128_setweyl(rp_rng *r, uint64_t lo, uint64_t hi)
{
    r->st[6] = lo | 1u;
    r->st[7] = hi;
    r->phase = 0;
    for (int i = 0; i < 96; i++) host_next(r);
}

static void seed_state(rp_rng *r, uint64_t seed, const uint32_t *key, size_t n_key)
{
    if (is_simd(r->engine)) {  // seeded as the scalar engine, then the sub-streams
        rp_rng b;
        b.engine = simd_base_engine(r->engine);
        seed_state(&b, seed, key, n_key);
        memset(r->st, 0, sizeof r->st);
        simd_from_base(r, b.st);
        return;
    }
    std::vector<uint32_t> in = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    if (n_key) {
        in.resize(4, 0u);  // keep "no key" and "key [0]" distinct
        in.insert(in.end(), key, key + n_key);
    }
    int nw = (r->engine == RP_SFC64) ? 3 : kEngines[r->engine].words;
    uint32_t o[18];
    SeedMixer(in).generate(o, (size_t)(2 * nw));
    uint64_t w[9];
    for (int i = 0; i < nw; i++) w[i] = (uint64_t)o[2 * i] | ((uint64_t)o[2 * i + 1] << 32);
    memset(r->st, 0, sizeof r->st);
    r->phase = 0;
    switch (r->engine) {
    case RP_X256PP:
    case RP_X256SS:
        memcpy(r->st, w, 32);
        if (!(w[0] | w[1] | w[2] | w[3])) r->st[0] = 1;
        break;
    case RP_PCG64:
        memcpy(r->st, w, 32);
        r->st[2] |= 1u;
        break;
    case RP_XORO128:
    case RP_XS128:
        memcpy(r->st, w, 16);
        if (!(w[0] | w[1])) r->st[0] = 1;  // the excluded all-zero state
        break;
    case RP_SQUARES:
        // reading: the key is made odd (key 0 gives a constant stream)
        r->st[0] = w[0];
        r->st[1] = w[1] | 1u;
        break;
    case RP_PHILOX4X32:
    case RP_PHILOX:
    case RP_CHACHA20:
        memcpy(r->st, w, (size_t)nw * 8);
        break;
    case RP_SFC64:
        sfc64_setabc(r, w[0], w[1], w[2]);
        break;
    case RP_RANLUX:
        memcpy(r->st, w, 72);
        ranlux_fixup(r->st);
        break;
    case RP_CWG128:  // x, a, Weyl from the mixer, the increment through the setter
        memcpy(r->st, w, 48);
        cwg128_setweyl(r, w[6], w[7]);
        break;
    }
}

// ---------------------------------------------------------------------------
// serial streams
// 64 bits from the operating system's entropy source (Section 2.3): getrandom,
// then /dev/urandom; if neither answers, the clock mixed with addresses and a
// counter through a splitmix64 step (an emergency fallback, not secure).
static uint64_t system_entropy64()
{
    uint64_t v = 0;
    size_t got = 0;
    while (got < sizeof v) {
        const ssize_t r = getrandom((char *)&v + got, sizeof v - got, 0);
        if (r <= 0) break;
        got += (size_t)r;
    }
    if (got == sizeof v) return v;
    if (FILE *f = std::fopen("/dev/urandom", "rb")) {
        const size_t n = std::fread(&v, 1, sizeof v, f);
        std::fclose(f);
        if (n == sizeof v) return v;
    }
    static uint64_t counter = 0;
    uint64_t z = (uint64_t)std::chrono::high_resolution_clock::now().time_since_epoch().count() ^
                 (uint64_t)(uintptr_t)&v ^ (++counter * 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

extern "C" int rp_randomize(rp_rng *rng)
{
    if (!rng) return fail(RP_ENULL, "rp_randomize: NULL rng");
    return rp_seed(rng, system_entropy64(), nullptr, 0);
}

extern "C" rp_rng *rp_create(const char *engine)
{
    int e = RP_X256PP;
    if (engine && *engine) {
        e = rp_engine_id(engine);
        if (e < 0) return nullptr;
    }
    rp_rng *r = new (std::nothrow) rp_rng;
    if (!r) {
        set_error("rp_create: out of memory");
        return nullptr;
    }
    r->engine = e;
    // a new engine is randomized from system entropy (Section 2.1)
    rp_randomize(r);
    return r;
}

extern "C" void rp_free(rp_rng *rng) { delete rng; }

extern "C" rp_rng *rp_duplicate(const rp_rng *rng)
{
    if (!rng) {
        set_error("rp_duplicate: NULL rng");
        return nullptr;
    }
    rp_rng *r = new (std::nothrow) rp_rng(*rng);
    if (!r) set_error("rp_duplicate: out of memory");
    return r;
}

extern "C" int rp_set_full_mantissa(rp_rng *rng, int on)
{
    if (!rng) return fail(RP_ENULL, "rp_set_full_mantissa: NULL rng");
    if (on != 0 && on != 1) return fail(RP_EINVAL, "rp_set_full_mantissa: on must be 0 or 1, not %d", on);
    rng->full_mantissa = on == 1;
    return RP_OK;
}

extern "C" int rp_get_full_mantissa(const rp_rng *rng)
{
    if (!rng) return fail(RP_ENULL, "rp_get_full_mantissa: NULL rng");
    return rng->full_mantissa ? 1 : 0;
}

// Settings of a stream or substream set (RP_FULL_MANTISSA, RP_SQUEEZE,
// RP_BITEXACT).
static bool *setting_slot(bool *full_mantissa, bool *squeeze, bool *bitexact, int flag)
{
    switch (flag) {
    case RP_FULL_MANTISSA:
        return full_mantissa;
    case RP_SQUEEZE:
        return squeeze;
    case RP_BITEXACT:
        return bitexact;
    default:
        return nullptr;
    }
}

extern "C" int rp_set_flag(rp_rng *rng, int flag, int value)
{
    if (!rng) return fail(RP_ENULL, "rp_set_flag: NULL rng");
    bool *slot = setting_slot(&rng->full_mantissa, &rng->squeeze, &rng->bitexact, flag);
    if (!slot) return fail_rng(rng, RP_EINVAL, "rp_set_flag: unknown setting %d", flag);
    if (value != 0 && value != 1) return fail_rng(rng, RP_EINVAL, "rp_set_flag: value must be 0 or 1, not %d", value);
    *slot = value == 1;
    return RP_OK;
}

extern "C" int rp_get_flag(const rp_rng *rng, int flag)
{
    if (!rng) return fail(RP_ENULL, "rp_get_flag: NULL rng");
    rp_rng *r = const_cast<rp_rng *>(rng);
    bool *slot = setting_slot(&r->full_mantissa, &r->squeeze, &r->bitexact, flag);
    if (!slot) return fail_rng(rng, RP_EINVAL, "rp_get_flag: unknown setting %d", flag);
    return *slot ? 1 : 0;
}

extern "C" int rp_seed(rp_rng *rng, uint64_t seed, const uint32_t *spawn_key, size_t n_key)
{
    if (!rng) return fail(RP_ENULL, "rp_seed: NULL rng");
    if (n_key && !spawn_key) return fail_rng(rng, RP_ENULL, "rp_seed: NULL spawn key");
    if (n_key > 1024) return fail_rng(rng, RP_EINVAL, "rp_seed: spawn key longer than 1024 words");
    rng->seed = seed;
    rng->key.assign(spawn_key, spawn_key + n_key);
    seed_state(rng, seed, spawn_key, n_key);
    return RP_OK;
}

extern "C" int rp_state_words(const rp_rng *rng)
{
    if (!rng) return fail(RP_ENULL, "rp_state_words: NULL rng");
    return kEngines[rng->engine].words;
}

// Why the words w (Table 3 order, `stride` apart) are not a state the engine
// can reach, or nullptr.  The excluded states are those the seeding fix-ups
// replace: the all-zero state of the xor family (a fixed point that outputs
// zeros for ever), an even PCG64 increment, an even squares64 key, and a
// ranlux++ value outside [1, m).
static const char *state_defect(int e, const uint64_t *w, size_t stride)
{
    auto W = [&](int k) { return w[(size_t)k * stride]; };
    switch (e) {
    case RP_X256PP:
    case RP_X256SS:
        if (!(W(0) | W(1) | W(2) | W(3))) return "the all-zero xoshiro256 state (a fixed point)";
        break;
    case RP_XORO128:
    case RP_XS128:
        if (!(W(0) | W(1))) return "the all-zero state (a fixed point)";
        break;
    case RP_PCG64:
        if (!(W(2) & 1)) return "an even PCG64 increment";
        break;
    case RP_SQUARES:
        if (!(W(1) & 1)) return "an even squares64 key";
        break;
    case RP_CWG128:
        if (!(W(6) & 1)) return "an even cwg128 Weyl increment";
        break;
    case RP_X256PPS:
    case RP_X256SSS:
        for (int k = 0; k < 8; k++)
            if (!(W(4 * k) | W(4 * k + 1) | W(4 * k + 2) | W(4 * k + 3)))
                return "an all-zero xoshiro256 sub-stream (a fixed point)";
        break;
    case RP_RANLUX: {
        // m = 2^576 - 2^240 + 1: limbs 4..8 all ones, limb 3 bits 48..63, limb 0 = 1
        static const uint64_t m[9] = {1, 0, 0, 0xFFFF000000000000ull, ~0ull, ~0ull, ~0ull, ~0ull, ~0ull};
        bool zero = true;
        for (int k = 0; k < 9; k++) zero = zero && W(k) == 0;
        if (zero) return "the ranlux++ value 0";
        for (int k = 8; k >= 0; k--) {
            if (W(k) < m[k]) return nullptr;
            if (W(k) > m[k]) return "a ranlux++ value not below m = 2^576 - 2^240 + 1";
        }
        return "the ranlux++ value m";
    }
    default:
        break;
    }
    return nullptr;
}

// Exclusive bound on k for jumps by 2^k engine steps: 2^k must stay below the
// period of one stream (one key, increment or nonce).  0: the engine has no
// jump (sfc64 is not linear).
static int jump_limit(int e)
{
    switch (e) {
    case RP_X256PP:
    case RP_X256SS:
    case RP_PHILOX:  // 256-bit block counter
    case RP_RANLUX:  // period about 2^570; exponents up to 2^256 are formed
        return 256;
    case RP_PCG64:
    case RP_PHILOX4X32:  // 128-bit block counter
    case RP_XORO128:
    case RP_XS128:
        return 128;
    case RP_SQUARES:
        return 64;
    case RP_CHACHA20:  // 32-bit block counter per nonce
        return 32;
    case RP_X256PPS:  // every sub-stream moves; they are 2^253 steps apart
    case RP_X256SSS:
        return 253;
    default:
        return 0;
    }
}

// Whether n substreams of 2^k engine steps each fit in one period without
// overlap: n * 2^k <= period.  The counter engines and pcg64 have periods of
// exactly 2^jump_limit steps (blocks for the block engines), the xor engines
// 2^jump_limit - 1; ranlux++'s period (about 2^570) holds every family; the
// sub-streams of the SIMD engines are 2^253 steps apart, each substream
// taking 2^k steps of every sub-stream.
static bool jump_family_fits(int e, int k, uint64_t n)
{
    if (e == RP_RANLUX) return true;
    const int room = jump_limit(e) - k;  // >= 1
    if (room >= 64) return true;         // n <= 2^32 already
    uint64_t cap = 1ull << room;
    if (e == RP_X256PP || e == RP_X256SS || e == RP_XORO128 || e == RP_XS128) cap -= 1;
    return n <= cap;
}

extern "C" int rp_get_state(const rp_rng *rng, uint64_t *words, size_t n, uint32_t *phase)
{
    if (!rng || !words) return fail(RP_ENULL, "rp_get_state: NULL argument");
    int nw = kEngines[rng->engine].words;
    if (n < (size_t)nw) return fail_rng(rng, RP_EINVAL, "rp_get_state: need %d words", nw);
    memcpy(words, rng->st, (size_t)nw * 8);
    if (phase) *phase = rng->phase;
    return RP_OK;
}

extern "C" int rp_set_state(rp_rng *rng, const uint64_t *words, size_t n, uint32_t phase)
{
    if (!rng || !words) return fail(RP_ENULL, "rp_set_state: NULL argument");
    int nw = kEngines[rng->engine].words;
    if (n != (size_t)nw) return fail_rng(rng, RP_EINVAL, "rp_set_state: expected %d words", nw);
    if (phase >= (uint32_t)kEngines[rng->engine].block)
        return fail_rng(rng, RP_EINVAL, "rp_set_state: phase %u out of range", phase);
    if (const char *why = state_defect(rng->engine, words, 1))
        return fail_rng(rng, RP_EINVAL, "rp_set_state: %s is not a state of '%s'", why, kEngines[rng->engine].id);
    memset(rng->st, 0, sizeof rng->st);
    memcpy(rng->st, words, n * 8);
    rng->phase = phase;
    return RP_OK;
}

static int advance_impl(rp_rng *rng, uint64_t lo, uint64_t hi)
{
    uint64_t *st = rng->st;
    switch (rng->engine) {
    case RP_X256PP:
    case RP_X256SS:
        x256_apply(st, poly_xpow(lo, hi, x256_charpoly()));
        return RP_OK;
    case RP_X256PPS:  // every sub-stream moves n steps; the phase is kept
    case RP_X256SSS: {
        const Poly p = poly_xpow(lo, hi, x256_charpoly());
        for (int k = 0; k < 8; k++) x256_apply(st + 4 * k, p);
        return RP_OK;
    }
    case RP_SQUARES:  // period 2^64: hi 2^64 steps are a full period
        st[0] += lo;
        return RP_OK;
    case RP_CHACHA20:  // blocks: the 32-bit counter, modulo 2^32
        st[5] = (st[5] & 0xffffffffull) | ((uint64_t)(uint32_t)((st[5] >> 32) + (uint32_t)lo) << 32);
        return RP_OK;
    case RP_XORO128:
    case RP_XS128:
        x128_apply(rng->engine, st, poly_xpow_d<128>(lo, hi, x128_charpoly(rng->engine)));
        return RP_OK;
    case RP_PCG64: {
        PcgAffine m = pcg_power(lo, hi);
        u128 s{st[0], st[1]}, inc{st[2], st[3]};
        s = add128(mul128(m.mult, s), mul128(m.plus, inc));
        st[0] = s.lo;
        st[1] = s.hi;
        return RP_OK;
    }
    case RP_PHILOX4X32: {
        u128 c{st[0], st[1]};
        c = add128(c, u128{lo, hi});
        st[0] = c.lo;
        st[1] = c.hi;
        return RP_OK;
    }
    case RP_PHILOX: {
        uint64_t add[4] = {lo, hi, 0, 0}, carry = 0;
        for (int k = 0; k < 4; k++) {
            uint64_t s1 = st[k] + add[k];
            uint64_t c = s1 < st[k];
            uint64_t s2 = s1 + carry;
            c += s2 < s1;
            st[k] = s2;
            carry = c;
        }
        return RP_OK;
    }
    case RP_RANLUX: {
        uint64_t e[2] = {lo, hi}, An[9];
        ranlux_pow(ranlux_A(), e, 2, An);
        rl_mulmod(st, An, st);
        return RP_OK;
    }
    default:
        return fail_rng(rng, RP_EUNSUPPORTED, "advance: engine '%s' has no jump", kEngines[rng->engine].id);
    }
}

extern "C" int rp_advance(rp_rng *rng, uint64_t lo, uint64_t hi)
{
    if (!rng) return fail(RP_ENULL, "rp_advance: NULL rng");
    return advance_impl(rng, lo, hi);
}

// Advances the stream by 2^k engine steps, 0 <= k < jump_limit(engine).
static int jump_pow2(rp_rng *rng, int k)
{
    if (k < 128) return advance_impl(rng, k < 64 ? (1ull << k) : 0, k >= 64 ? (1ull << (k - 64)) : 0);
    switch (rng->engine) {
    case RP_X256PP:
    case RP_X256SS:
    case RP_X256PPS:
    case RP_X256SSS: {
        Poly x;
        x.flip(1);
        const Poly &P = x256_charpoly();
        for (int i = 0; i < k; i++) x = poly_mulmod(x, x, P);  // x^(2^k)
        const int lanes = is_simd(rng->engine) ? 8 : 1;
        for (int l = 0; l < lanes; l++) x256_apply(rng->st + 4 * l, x);
        return RP_OK;
    }
    case RP_PHILOX: {  // add 2^k to the 256-bit block counter
        uint64_t add = 1ull << (k % 64);
        for (int j = k / 64; j < 4; j++) {
            uint64_t s1 = rng->st[j] + add;
            bool c = s1 < rng->st[j];
            rng->st[j] = s1;
            if (!c) break;
            add = 1;
        }
        return RP_OK;
    }
    case RP_RANLUX: {
        uint64_t e[4] = {0, 0, 0, 0}, An[9];
        e[k / 64] = 1ull << (k % 64);
        ranlux_pow(ranlux_A(), e, 4, An);
        rl_mulmod(rng->st, An, rng->st);
        return RP_OK;
    }
    default:
        return fail_rng(rng, RP_EINVAL, "jump: 2^%d is not below the period of '%s'", k, kEngines[rng->engine].id);
    }
}

extern "C" int rp_jump(rp_rng *rng, int k)
{
    if (!rng) return fail(RP_ENULL, "rp_jump: NULL rng");
    if (k != 32 && k != 64 && k != 96 && k != 128 && k != 192)
        return fail_rng(rng, RP_EINVAL, "rp_jump: k must be 32, 64, 96, 128 or 192 (got %d)", k);
    const int lim = jump_limit(rng->engine);
    if (lim == 0) return fail_rng(rng, RP_EUNSUPPORTED, "rp_jump: '%s' has no jump", kEngines[rng->engine].id);
    if (k >= lim)
        return fail_rng(rng, RP_EINVAL, "rp_jump: 2^%d is not below the period of '%s'%s", k,
                        kEngines[rng->engine].id, rng->engine == RP_CHACHA20 ? " (use the nonce)" : "");
    return jump_pow2(rng, k);
}

extern "C" int rp_pcg64_set_inc(rp_rng *rng, uint64_t lo, uint64_t hi)
{
    if (!rng) return fail(RP_ENULL, "rp_pcg64_set_inc: NULL rng");
    if (rng->engine != RP_PCG64) return fail_rng(rng, RP_EUNSUPPORTED, "pcg64_set_inc: engine is not pcg64");
    rng->st[2] = lo | 1u;
    rng->st[3] = hi;
    return RP_OK;
}

extern "C" int rp_philox_set_key(rp_rng *rng, uint64_t k0, uint64_t k1)
{
    if (!rng) return fail(RP_ENULL, "rp_philox_set_key: NULL rng");
    if (rng->engine == RP_PHILOX4X32) {
        rng->st[2] = k0;
    } else if (rng->engine == RP_PHILOX) {
        rng->st[4] = k0;
        rng->st[5] = k1;
    } else {
        return fail_rng(rng, RP_EUNSUPPORTED, "philox_set_key: engine is not philox");
    }
    return RP_OK;
}

extern "C" int rp_sfc64_set_abc(rp_rng *rng, uint64_t a, uint64_t b, uint64_t c)
{
    if (!rng) return fail(RP_ENULL, "rp_sfc64_set_abc: NULL rng");
    if (rng->engine == RP_SFC64S) {  // the base as the scalar setter makes it, then the counters
        rp_rng t;
        t.engine = RP_SFC64;
        sfc64_setabc(&t, a, b, c);
        memset(rng->st, 0, sizeof rng->st);
        simd_from_base(rng, t.st);
        return RP_OK;
    }
    if (rng->engine != RP_SFC64) return fail_rng(rng, RP_EUNSUPPORTED, "sfc64_set_abc: engine is not sfc64");
    sfc64_setabc(rng, a, b, c);
    return RP_OK;
}

extern "C" int rp_chacha20_set_nonce(rp_rng *rng, uint64_t lo, uint64_t hi)
{
    if (!rng) return fail(RP_ENULL, "rp_chacha20_set_nonce: NULL rng");
    if (rng->engine != RP_CHACHA20)
        return fail_rng(rng, RP_EUNSUPPORTED, "chacha20_set_nonce: engine is not chacha20");
    if (hi >> 32) return fail_rng(rng, RP_EINVAL, "chacha20_set_nonce: the nonce has 96 bits");
    rng->st[4] = lo;
    rng->st[5] = (rng->st[5] & 0xffffffff00000000ull) | hi;
    return RP_OK;
}

extern "C" int rp_cwg128_set_weyl(rp_rng *rng, uint64_t lo, uint64_t hi)
{
    if (!rng) return fail(RP_ENULL, "rp_cwg128_set_weyl: NULL rng");
    if (rng->engine != RP_CWG128) return fail_rng(rng, RP_EUNSUPPORTED, "cwg128_set_weyl: engine is not cwg128");
    cwg128_setweyl(rng, lo, hi);
    return RP_OK;
}

extern "C" int rp_squares_set_key(rp_rng *rng, uint64_t key)
{
    if (!rng) return fail(RP_ENULL, "rp_squares_set_key: NULL rng");
    if (rng->engine != RP_SQUARES) return fail_rng(rng, RP_EUNSUPPORTED, "squares_set_key: engine is not squares");
    rng->st[1] = key | 1u;
    return RP_OK;
}

// serialized image: magic, engine, phase, key length, 32 state words, seed,
// key (version 2: 32 state words, for the SIMD engines)
static constexpr uint32_t kMagic = 0x52503032u;  // "RP02"
static constexpr size_t kImgWords = 32;
static constexpr size_t kImgSeed = 16 + 8 * kImgWords;  // offset of the seed
static constexpr size_t kImgKey = kImgSeed + 8;         // offset of the key

extern "C" int rp_serialize(const rp_rng *rng, void *buf, size_t len, size_t *needed)
{
    if (!rng) return fail(RP_ENULL, "rp_serialize: NULL rng");
    size_t need = kImgKey + rng->key.size() * 4;
    if (needed) *needed = need;
    if (!buf) return RP_OK;
    if (len < need) return fail_rng(rng, RP_EINVAL, "rp_serialize: buffer too small (%zu < %zu)", len, need);
    uint8_t *p = (uint8_t *)buf;
    uint32_t hdr[4] = {kMagic, (uint32_t)rng->engine, rng->phase, (uint32_t)rng->key.size()};
    memcpy(p, hdr, 16);
    memcpy(p + 16, rng->st, 8 * kImgWords);
    memcpy(p + kImgSeed, &rng->seed, 8);
    if (!rng->key.empty()) memcpy(p + kImgKey, rng->key.data(), rng->key.size() * 4);
    return RP_OK;
}

extern "C" int rp_deserialize(rp_rng *rng, const void *buf, size_t len)
{
    if (!rng || !buf) return fail(RP_ENULL, "rp_deserialize: NULL argument");
    if (len < kImgKey) return fail_rng(rng, RP_EINVAL, "rp_deserialize: buffer too small");
    const uint8_t *p = (const uint8_t *)buf;
    uint32_t hdr[4];
    memcpy(hdr, p, 16);
    if (hdr[0] != kMagic || hdr[1] >= RP_NENGINES || hdr[2] >= (uint32_t)kEngines[hdr[1]].block || hdr[3] > 1024 ||
        len < kImgKey + (size_t)hdr[3] * 4)
        return fail_rng(rng, RP_EINVAL, "rp_deserialize: not a serialized stream");
    uint64_t st[kImgWords];
    memcpy(st, p + 16, sizeof st);
    for (int k = kEngines[hdr[1]].words; k < (int)kImgWords; k++)
        if (st[k]) return fail_rng(rng, RP_EINVAL, "rp_deserialize: not a serialized stream");
    if (const char *why = state_defect((int)hdr[1], st, 1))
        return fail_rng(rng, RP_EINVAL, "rp_deserialize: %s is not a state of '%s'", why, kEngines[hdr[1]].id);
    rng->engine = (int)hdr[1];
    rng->phase = hdr[2];
    memcpy(rng->st, st, sizeof st);
    memcpy(&rng->seed, p + kImgSeed, 8);
    rng->key.assign((const uint32_t *)(p + kImgKey), (const uint32_t *)(p + kImgKey) + hdr[3]);
    return RP_OK;
}

extern "C" int rp_raw_host(rp_rng *rng, uint64_t *out, size_t n)
{
    if (!rng || (!out && n)) return fail(RP_ENULL, "rp_raw_host: NULL argument");
    for (size_t i = 0; i < n; i++) out[i] = host_next(rng);
    return RP_OK;
}

// ---------------------------------------------------------------------------
// device substreams
static int hip_fail(hipError_t e, const char *what)
{
    return fail(RP_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

extern "C" int rp_streams_create(const rp_rng *base, int kind, uint64_t n, int jump_log2, rp_streams **out)
{
    if (!base || !out) return fail(RP_ENULL, "rp_streams_create: NULL argument");
    *out = nullptr;
    if (n == 0) return fail(RP_EINVAL, "rp_streams_create: n must be positive");
    if (n > (1ull << 32)) return fail(RP_EINVAL, "rp_streams_create: at most 2^32 substreams");
    const int e = base->engine;
    const int nw = kEngines[e].words;
    switch (kind) {
    case RP_SUB_KEY:
        if (e != RP_PHILOX4X32 && e != RP_PHILOX && e != RP_CHACHA20)
            return fail(RP_EUNSUPPORTED, "RP_SUB_KEY needs a philox or chacha20 engine");
        break;
    case RP_SUB_INC:
        if (e != RP_PCG64 && e != RP_CWG128) return fail(RP_EUNSUPPORTED, "RP_SUB_INC needs pcg64 or cwg128");
        break;
    case RP_SUB_SPAWN:
        break;
    case RP_SUB_JUMP:
        if (jump_limit(e) == 0) return fail(RP_EUNSUPPORTED, "'%s' has no jump", kEngines[e].id);
        if (jump_log2 < 0 || jump_log2 >= jump_limit(e))
            return fail(RP_EINVAL, "rp_streams_create: jump_log2 %d: 2^k steps must be below the period of '%s' "
                                   "(k < %d)", jump_log2, kEngines[e].id, jump_limit(e));
        if (!jump_family_fits(e, jump_log2, n))
            return fail(RP_EINVAL, "rp_streams_create: %llu substreams of 2^%d steps overlap within the period of '%s'",
                        (unsigned long long)n, jump_log2, kEngines[e].id);
        break;
    default:
        return fail(RP_EINVAL, "rp_streams_create: unknown kind %d", kind);
    }
    std::vector<uint64_t> words((size_t)nw * n);
    std::vector<uint32_t> phase(n, 0);
    rp_rng cur = *base;
    rp_rng jumped = *base;  // JUMP: running state advanced by 2^jump_log2 per substream
    const uint64_t jl = (jump_log2 >= 0 && jump_log2 < 64) ? (1ull << jump_log2) : 0;
    const uint64_t jh = (jump_log2 >= 64 && jump_log2 < 128) ? (1ull << (jump_log2 - 64)) : 0;
    // precomputed per-step transforms for JUMP
    Poly jpoly;
    uint64_t jmul[9];
    PcgAffine jpcg{};
    if (kind == RP_SUB_JUMP && n > 1) {
        if (is_x256(e)) {
            Poly base_x;
            base_x.flip(1);
            const Poly &P = x256_charpoly();
            for (int i = 0; i < jump_log2; i++) base_x = poly_mulmod(base_x, base_x, P);
            jpoly = base_x;
        } else if (e == RP_XORO128 || e == RP_XS128) {
            Poly base_x;
            base_x.flip(1);
            const Poly &P = x128_charpoly(e);
            for (int i = 0; i < jump_log2; i++) base_x = poly_mulmod_d<128>(base_x, base_x, P);
            jpoly = base_x;
        } else if (e == RP_RANLUX) {
            uint64_t ex[4] = {0, 0, 0, 0};
            ex[jump_log2 / 64] = 1ull << (jump_log2 % 64);
            ranlux_pow(ranlux_A(), ex, 4, jmul);
        } else if (e == RP_PCG64) {
            jpcg = pcg_power(jl, jh);
        }
    }
    for (uint64_t i = 0; i < n; i++) {
        switch (kind) {
        case RP_SUB_KEY:
            cur = *base;
            if (e == RP_PHILOX4X32) cur.st[2] = i;
            else if (e == RP_CHACHA20) {  // nonce := i, key and counter from the base
                cur.st[4] = i;
                cur.st[5] &= 0xffffffff00000000ull;
            } else {
                cur.st[4] = i;
                cur.st[5] = 0;
            }
            break;
        case RP_SUB_INC:
            cur = *base;
            if (e == RP_CWG128) {
                cwg128_setweyl(&cur, 2 * i + 1, 0);
            } else {
                cur.st[2] = 2 * i + 1;
                cur.st[3] = 0;
            }
            break;
        case RP_SUB_SPAWN: {
            cur.engine = e;
            uint32_t k = (uint32_t)i;
            seed_state(&cur, base->seed, &k, 1);
            break;
        }
        case RP_SUB_JUMP:
            if (i > 0) {
                if (is_x256(e)) {
                    const int lanes = is_simd(e) ? 8 : 1;  // SIMD engines: every sub-stream
                    for (int l = 0; l < lanes; l++) x256_apply(jumped.st + 4 * l, jpoly);
                }
                else if (e == RP_XORO128 || e == RP_XS128) x128_apply(e, jumped.st, jpoly);
                else if (e == RP_RANLUX) rl_mulmod(jumped.st, jmul, jumped.st);
                else if (e == RP_PCG64) {
                    u128 s{jumped.st[0], jumped.st[1]}, inc{jumped.st[2], jumped.st[3]};
                    s = add128(mul128(jpcg.mult, s), mul128(jpcg.plus, inc));
                    jumped.st[0] = s.lo;
                    jumped.st[1] = s.hi;
                } else {  // counters: philox (any k below 256), philox4x32, squares64, chacha20
                    int rc = jump_pow2(&jumped, jump_log2);
                    if (rc) return rc;
                }
            }
            cur = jumped;
            break;
        }
        for (int k = 0; k < nw; k++) words[(size_t)k * n + i] = cur.st[k];
        phase[i] = cur.phase;
    }
    rp_streams *s = new (std::nothrow) rp_streams;
    if (!s) return fail(RP_ENOMEM, "rp_streams_create: out of memory");
    s->engine = e;
    s->n = n;
    s->nwords = nw;
    s->full_mantissa = base->full_mantissa;
    s->squeeze = base->squeeze;
    s->bitexact = base->bitexact;
    hipError_t err = hipGetDevice(&s->device);
    if (err != hipSuccess) {
        delete s;
        return hip_fail(err, "hipGetDevice");
    }
    err = hipMalloc(&s->d_words, words.size() * 8);
    if (err == hipSuccess) err = hipMalloc(&s->d_phase, n * 4);
    if (err == hipSuccess) err = hipMemcpy(s->d_words, words.data(), words.size() * 8, hipMemcpyHostToDevice);
    if (err == hipSuccess) err = hipMemcpy(s->d_phase, phase.data(), n * 4, hipMemcpyHostToDevice);
    if (err != hipSuccess) {
        (void)hipFree(s->d_words);
        (void)hipFree(s->d_phase);
        delete s;
        return fail(RP_ENOMEM, "rp_streams_create: device allocation/copy failed: %s", hipGetErrorString(err));
    }
    *out = s;
    return RP_OK;
}

extern "C" void rp_streams_free(rp_streams *s)
{
    if (!s) return;
    (void)hipFree(s->d_words);
    (void)hipFree(s->d_phase);
    delete s;
}

extern "C" uint64_t rp_streams_count(const rp_streams *s) { return s ? s->n : 0; }

extern "C" int rp_streams_engine(const rp_streams *s)
{
    if (!s) return fail(RP_ENULL, "rp_streams_engine: NULL streams");
    return s->engine;
}

extern "C" int rp_streams_get(const rp_streams *s, uint64_t *words, uint32_t *phase)
{
    if (!s || !words || !phase) return fail(RP_ENULL, "rp_streams_get: NULL argument");
    hipError_t e = hipDeviceSynchronize();
    if (e == hipSuccess) e = hipMemcpy(words, s->d_words, (size_t)s->nwords * s->n * 8, hipMemcpyDeviceToHost);
    if (e == hipSuccess) e = hipMemcpy(phase, s->d_phase, s->n * 4, hipMemcpyDeviceToHost);
    return e == hipSuccess ? RP_OK : hip_fail(e, "rp_streams_get");
}

extern "C" int rp_streams_set(rp_streams *s, const uint64_t *words, const uint32_t *phase)
{
    if (!s || !words || !phase) return fail(RP_ENULL, "rp_streams_set: NULL argument");
    for (uint64_t i = 0; i < s->n; i++) {
        if (phase[i] >= (uint32_t)kEngines[s->engine].block) return fail(RP_EINVAL, "rp_streams_set: bad phase");
        if (const char *why = state_defect(s->engine, words + i, s->n))
            return fail(RP_EINVAL, "rp_streams_set: substream %llu: %s is not a state of '%s'", (unsigned long long)i,
                        why, kEngines[s->engine].id);
    }
    hipError_t e = hipDeviceSynchronize();
    if (e == hipSuccess) e = hipMemcpy(s->d_words, words, (size_t)s->nwords * s->n * 8, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(s->d_phase, phase, s->n * 4, hipMemcpyHostToDevice);
    return e == hipSuccess ? RP_OK : hip_fail(e, "rp_streams_set");
}

extern "C" int rp_streams_set_flag(rp_streams *s, int flag, int value)
{
    if (!s) return fail(RP_ENULL, "rp_streams_set_flag: NULL streams");
    bool *slot = setting_slot(&s->full_mantissa, &s->squeeze, &s->bitexact, flag);
    if (!slot) return fail(RP_EINVAL, "rp_streams_set_flag: unknown setting %d", flag);
    if (value != 0 && value != 1) return fail(RP_EINVAL, "rp_streams_set_flag: value must be 0 or 1, not %d", value);
    *slot = value == 1;
    return RP_OK;
}

extern "C" int rp_streams_get_flag(const rp_streams *s, int flag)
{
    if (!s) return fail(RP_ENULL, "rp_streams_get_flag: NULL streams");
    rp_streams *m = const_cast<rp_streams *>(s);
    bool *slot = setting_slot(&m->full_mantissa, &m->squeeze, &m->bitexact, flag);
    if (!slot) return fail(RP_EINVAL, "rp_streams_get_flag: unknown setting %d", flag);
    return *slot ? 1 : 0;
}

extern "C" int rp_streams_duplicate(const rp_streams *s, rp_streams **out)
{
    if (!s || !out) return fail(RP_ENULL, "rp_streams_duplicate: NULL argument");
    rp_streams *d = new (std::nothrow) rp_streams(*s);
    if (!d) return fail(RP_ENOMEM, "rp_streams_duplicate: out of memory");
    d->d_words = nullptr;
    d->d_phase = nullptr;
    hipError_t e = hipMalloc(&d->d_words, (size_t)s->nwords * s->n * 8);
    if (e == hipSuccess) e = hipMalloc(&d->d_phase, s->n * 4);
    if (e == hipSuccess) e = hipMemcpy(d->d_words, s->d_words, (size_t)s->nwords * s->n * 8, hipMemcpyDeviceToDevice);
    if (e == hipSuccess) e = hipMemcpy(d->d_phase, s->d_phase, s->n * 4, hipMemcpyDeviceToDevice);
    if (e != hipSuccess) {
        (void)hipFree(d->d_words);
        (void)hipFree(d->d_phase);
        delete d;
        return hip_fail(e, "rp_streams_duplicate");
    }
    *out = d;
    return RP_OK;
}

// serialized image of a substream set: magic, engine, state words per
// substream, settings (4 x u32; bit 0 the full-mantissa setting, bit 1 the
// squeeze switched off, bit 2 bitexact), n (u64), then the state words (SoA, word k of
// substream i at k n + i) and the n phases
static constexpr uint32_t kStreamsMagic = 0x31535052u;  // "RPS1"

extern "C" int rp_streams_serialize(const rp_streams *s, void *buf, size_t len, size_t *needed)
{
    if (!s) return fail(RP_ENULL, "rp_streams_serialize: NULL streams");
    const size_t nw = (size_t)s->nwords * s->n;
    const size_t need = 24 + nw * 8 + s->n * 4;
    if (needed) *needed = need;
    if (!buf) return RP_OK;
    if (len < need) return fail(RP_EINVAL, "rp_streams_serialize: buffer too small (%zu < %zu)", len, need);
    std::vector<uint64_t> words(nw);
    std::vector<uint32_t> phase(s->n);
    const int rc = rp_streams_get(s, words.data(), phase.data());
    if (rc) return rc;
    uint8_t *p = (uint8_t *)buf;
    const uint32_t hdr[4] = {kStreamsMagic, (uint32_t)s->engine, (uint32_t)s->nwords,
                             (s->full_mantissa ? 1u : 0u) | (s->squeeze ? 0u : 2u) | (s->bitexact ? 4u : 0u)};
    memcpy(p, hdr, 16);
    memcpy(p + 16, &s->n, 8);
    memcpy(p + 24, words.data(), nw * 8);
    memcpy(p + 24 + nw * 8, phase.data(), s->n * 4);
    return RP_OK;
}

extern "C" int rp_streams_deserialize(const void *buf, size_t len, rp_streams **out)
{
    if (!buf || !out) return fail(RP_ENULL, "rp_streams_deserialize: NULL argument");
    *out = nullptr;
    if (len < 24) return fail(RP_EINVAL, "rp_streams_deserialize: buffer too small");
    const uint8_t *p = (const uint8_t *)buf;
    uint32_t hdr[4];
    uint64_t n;
    memcpy(hdr, p, 16);
    memcpy(&n, p + 16, 8);
    if (hdr[0] != kStreamsMagic || hdr[1] >= RP_NENGINES || hdr[2] != (uint32_t)kEngines[hdr[1]].words ||
        hdr[3] > 7 || n == 0 || n > (1ull << 32))
        return fail(RP_EINVAL, "rp_streams_deserialize: not a serialized substream set");
    const size_t nw = (size_t)hdr[2] * n;
    if (len < 24 + nw * 8 + n * 4) return fail(RP_EINVAL, "rp_streams_deserialize: image truncated");
    std::vector<uint64_t> words(nw);
    std::vector<uint32_t> phase(n);
    memcpy(words.data(), p + 24, nw * 8);
    memcpy(phase.data(), p + 24 + nw * 8, n * 4);
    for (uint64_t i = 0; i < n; i++) {
        if (phase[i] >= (uint32_t)kEngines[hdr[1]].block)
            return fail(RP_EINVAL, "rp_streams_deserialize: bad phase of substream %llu", (unsigned long long)i);
        if (const char *why = state_defect((int)hdr[1], words.data() + i, n))
            return fail(RP_EINVAL, "rp_streams_deserialize: substream %llu: %s is not a state of '%s'",
                        (unsigned long long)i, why, kEngines[hdr[1]].id);
    }
    rp_streams *s = new (std::nothrow) rp_streams;
    if (!s) return fail(RP_ENOMEM, "rp_streams_deserialize: out of memory");
    s->engine = (int)hdr[1];
    s->n = n;
    s->nwords = (int)hdr[2];
    s->full_mantissa = (hdr[3] & 1) != 0;
    s->squeeze = (hdr[3] & 2) == 0;
    s->bitexact = (hdr[3] & 4) != 0;
    hipError_t e = hipGetDevice(&s->device);
    if (e == hipSuccess) e = hipMalloc(&s->d_words, nw * 8);
    if (e == hipSuccess) e = hipMalloc(&s->d_phase, n * 4);
    if (e == hipSuccess) e = hipMemcpy(s->d_words, words.data(), nw * 8, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(s->d_phase, phase.data(), n * 4, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        (void)hipFree(s->d_words);
        (void)hipFree(s->d_phase);
        delete s;
        return hip_fail(e, "rp_streams_deserialize");
    }
    *out = s;
    return RP_OK;
}

// ---------------------------------------------------------------------------
// bulk fill dispatch
extern "C" int rp_fill(rp_streams *s, int dist, int dtype, uint64_t bound, int flags, void *d_out,
                       uint64_t per_stream, void *hip_stream)
{
    if (!s) return fail(RP_ENULL, "rp_fill: NULL streams");
    if (per_stream == 0) return RP_OK;
    if (!d_out) return fail(RP_ENULL, "rp_fill: NULL output");
    bool ok = false;
    switch (dist) {
    case RP_RAW: ok = dtype == RP_U64 || dtype == RP_U32; break;
    case RP_U01: ok = dtype == RP_F64 || dtype == RP_F32; break;
    case RP_BOUNDED: ok = dtype == RP_U64 || (dtype == RP_U32 && bound <= 0xFFFFFFFFull); break;
    case RP_NORM:
    case RP_EXP: ok = dtype == RP_F64 || dtype == RP_F32; break;
    default: return fail(RP_EINVAL, "rp_fill: unknown distribution %d", dist);
    }
    if (!ok) return fail(RP_EUNSUPPORTED, "rp_fill: distribution %d has no dtype %d form (or bound too large)", dist, dtype);
    if (flags & ~RP_FLAG_52BIT) return fail(RP_EINVAL, "rp_fill: unknown flags 0x%x", flags);
    if (!s->full_mantissa) flags |= RP_FLAG_52BIT;
    size_t esz = (dtype == RP_U64 || dtype == RP_F64) ? 8 : 4;
    if ((uintptr_t)d_out % esz) return fail(RP_EINVAL, "rp_fill: output not aligned to %zu bytes", esz);
    if (s->n > UINT64_MAX / per_stream) return fail(RP_EINVAL, "rp_fill: size overflow");
    int rc = ensure_device_tables();
    if (rc) return rc;
    FillArgs a{};
    a.words = s->d_words;
    a.phase = s->d_phase;
    a.n = s->n;
    a.per_stream = per_stream;
    a.out = d_out;
    a.bound = bound;
    a.thresh = 0;
    if (dist == RP_BOUNDED && bound) {
        if (dtype == RP_U64) a.thresh = (0 - bound) % bound;
        else a.thresh = (uint32_t)(0u - (uint32_t)bound) % (uint32_t)bound;
    }
    a.flags = flags | settings_flags(s);
    return launch_fill(s->engine, dist, dtype, a, (hipStream_t)hip_stream);
}

extern "C" int rp_permutations(rp_streams *s, uint32_t n, uint32_t *d_out, void *hip_stream)
{
    if (!s) return fail(RP_ENULL, "rp_permutations: NULL streams");
    if (n == 0) return RP_OK;
    if (!d_out) return fail(RP_ENULL, "rp_permutations: NULL output");
    if ((uintptr_t)d_out % 4) return fail(RP_EINVAL, "rp_permutations: output not aligned to 4 bytes");
    int rc = ensure_device_tables();
    if (rc) return rc;
    FillArgs a{};
    a.words = s->d_words;
    a.phase = s->d_phase;
    a.n = s->n;
    a.per_stream = n;
    a.out = d_out;
    return launch_discrete(s->engine, true, a, nullptr, 0, (hipStream_t)hip_stream);
}

// Samples without allocation: Floyd's membership tables live in a file-scope
// device array of kSampleScratchBytes, one copy per GPU held until the
// process ends.  Its host-side name is not a device address: the address
// comes from hipGetSymbolAddress, taken once per device with that device
// current, and only that address is handed to kernels.
static constexpr uint64_t kSampleScratchBytes = 64ull << 20;
static __device__ __align__(256) uint32_t scratch[kSampleScratchBytes / 4];

static int sample_scratch(uint32_t **out)
{
    static std::mutex mu;
    static uint32_t *ptr[64] = {};
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail(RP_EDEVICE, "hipGetDevice: %s", hipGetErrorString(e));
    if (dev < 0 || dev >= 64) return fail(RP_EDEVICE, "device index %d out of range", dev);
    std::lock_guard<std::mutex> lk(mu);
    if (!ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(RP_EDEVICE, "rp_sample_noalloc: scratch address on device %d: %s", dev,
                        hipGetErrorString(e));
        ptr[dev] = (uint32_t *)p;
    }
    *out = ptr[dev];
    return RP_OK;
}

static int sample_impl(const char *who, rp_streams *s, uint32_t n, uint32_t k, uint32_t *d_out, void *hip_stream,
                       bool noalloc)
{
    if (!s) return fail(RP_ENULL, "%s: NULL streams", who);
    if (k > n) return fail(RP_EINVAL, "%s: k = %u exceeds n = %u", who, k, n);
    if (k >= (1u << 30)) return fail(RP_EINVAL, "%s: k = %u too large", who, k);
    if (k == 0) return RP_OK;
    if (!d_out) return fail(RP_ENULL, "%s: NULL output", who);
    if ((uintptr_t)d_out % 4) return fail(RP_EINVAL, "%s: output not aligned to 4 bytes", who);
    int rc = ensure_device_tables();
    if (rc) return rc;
    FillArgs a{};
    a.words = s->d_words;
    a.phase = s->d_phase;
    a.n = s->n;
    a.per_stream = k;
    a.bound = n;
    a.out = d_out;
    const hipStream_t st = (hipStream_t)hip_stream;
    if (2 * (uint64_t)k > n) return launch_discrete(s->engine, false, a, nullptr, 0, st);
    int tbits = 1;
    while ((1ull << tbits) < 2 * (uint64_t)k) tbits++;
    const uint64_t cap = 1ull << tbits;
    if (s->n > UINT64_MAX / (cap * 4)) return fail(RP_EINVAL, "%s: workspace size overflow", who);
    const uint64_t bytes = s->n * cap * 4;
    if (noalloc) {
        if (bytes > kSampleScratchBytes)
            return fail(RP_EINVAL,
                        "%s: Floyd tables of %llu substreams x %llu entries need %llu bytes, above the fixed "
                        "scratch of %llu bytes (use rp_sample)",
                        who, (unsigned long long)s->n, (unsigned long long)cap, (unsigned long long)bytes,
                        (unsigned long long)kSampleScratchBytes);
        uint32_t *tab = nullptr;
        rc = sample_scratch(&tab);
        if (rc) return rc;
        return launch_discrete(s->engine, false, a, tab, tbits, st);
    }
    uint32_t *tab = nullptr;
    hipError_t e = hipMallocAsync((void **)&tab, bytes, st);
    if (e != hipSuccess) return fail(RP_ENOMEM, "%s: workspace: %s", who, hipGetErrorString(e));
    rc = launch_discrete(s->engine, false, a, tab, tbits, st);
    (void)hipFreeAsync(tab, st);
    return rc;
}

extern "C" int rp_sample(rp_streams *s, uint32_t n, uint32_t k, uint32_t *d_out, void *hip_stream)
{
    return sample_impl("rp_sample", s, n, k, d_out, hip_stream, false);
}

extern "C" int rp_sample_noalloc(rp_streams *s, uint32_t n, uint32_t k, uint32_t *d_out, void *hip_stream)
{
    return sample_impl("rp_sample_noalloc", s, n, k, d_out, hip_stream, true);
}

// rp_fill_law (binary64 output) and rp_fill_lawf (binary32: the float base
// draws, the transform in binary64, one rounding)
static int fill_law_impl(rp_streams *s, int law, const double *p, int np, void *d_out, uint64_t per_stream,
                         void *hip_stream, bool f32)
{
    if (!s) return fail(RP_ENULL, "rp_fill_law: NULL streams");
    static const int kParams[15] = {0, 2, 2, 2, 1, 2, 2, 3, 2, 2, 2, 1, 1, 2, 3};
    if (law < RP_LAW_UNIF || law > RP_LAW_SKEWNORMAL) return fail(RP_EINVAL, "rp_fill_law: unknown law %d", law);
    if (np != kParams[law]) return fail(RP_EINVAL, "rp_fill_law: law %d takes %d parameters, not %d", law, kParams[law], np);
    if (!p) return fail(RP_ENULL, "rp_fill_law: NULL parameters");
    for (int k = 0; k < np; k++)
        if (!std::isfinite(p[k])) return fail(RP_EINVAL, "rp_fill_law: parameter %d is not finite", k);
    FillArgs a{};
    bool ok = true;
    switch (law) {
    case RP_LAW_UNIF:
        ok = p[0] < p[1];
        a.xp[0] = p[0];
        a.xp[1] = p[1] - p[0];
        ok = ok && std::isfinite(a.xp[1]);
        break;
    case RP_LAW_NORMAL:
    case RP_LAW_LOGNORMAL:
        ok = p[1] >= 0.0;
        a.xp[0] = p[0];
        a.xp[1] = p[1];
        break;
    case RP_LAW_EXP:
        ok = p[0] > 0.0;
        a.xp[0] = p[0];
        break;
    case RP_LAW_GUMBEL:
        ok = p[1] > 0.0;
        a.xp[0] = p[0];
        a.xp[1] = p[1];
        break;
    case RP_LAW_PARETO:
        ok = p[0] > 0.0 && p[1] > 0.0;
        a.xp[0] = p[0];
        a.xp[1] = p[1];
        break;
    case RP_LAW_GPARETO:
        ok = p[1] > 0.0;
        a.xp[0] = p[0];
        a.xp[1] = p[1];
        a.xp[2] = p[2];
        a.xp[3] = p[2] != 0.0 ? 1.0 / std::fabs(p[2]) : 0.0;
        ok = ok && std::isfinite(a.xp[3]);
        break;
    case RP_LAW_WEIBULL:
        ok = p[0] > 0.0 && p[1] > 0.0;
        a.xp[0] = p[0];
        a.xp[1] = p[1];
        a.xp[2] = 1.0 / p[0];
        ok = ok && std::isfinite(a.xp[2]);
        break;
    case RP_LAW_GAMMA:
    case RP_LAW_BETA:
        ok = p[0] > 0.0 && p[1] > 0.0;
        a.xp[0] = p[0];
        a.xp[1] = p[1];
        break;
    case RP_LAW_CHI2:
    case RP_LAW_T:
        ok = p[0] > 0.0 && p[0] / 2.0 > 0.0;
        a.xp[0] = p[0] / 2.0;
        a.xp[1] = p[0];
        break;
    case RP_LAW_F:
        ok = p[0] / 2.0 > 0.0 && p[1] / 2.0 > 0.0;
        a.xp[0] = p[0] / 2.0;
        a.xp[1] = p[1] / 2.0;
        break;
    case RP_LAW_SKEWNORMAL: {
        ok = p[1] >= 0.0;
        const double dl = p[2] / std::sqrt(1.0 + p[2] * p[2]);
        a.xp[0] = p[0];
        a.xp[1] = p[1];
        a.xp[2] = dl;
        a.xp[3] = std::sqrt(1.0 - dl * dl);
        ok = ok && std::isfinite(dl);
        break;
    }
    }
    if (!ok) return fail(RP_EINVAL, "rp_fill_law: parameters outside the law's domain");
    if (per_stream == 0) return RP_OK;
    if (!d_out) return fail(RP_ENULL, "rp_fill_law: NULL output");
    if ((uintptr_t)d_out % (f32 ? 4 : 8)) return fail(RP_EINVAL, "rp_fill_law: output not aligned to its element size");
    if (s->n > UINT64_MAX / per_stream) return fail(RP_EINVAL, "rp_fill_law: size overflow");
    int rc = ensure_device_tables();
    if (rc) return rc;
    a.words = s->d_words;
    a.phase = s->d_phase;
    a.n = s->n;
    a.per_stream = per_stream;
    a.out = d_out;
    a.flags = settings_flags(s);
    if (law >= RP_LAW_GAMMA) return launch_fill_mix(s->engine, law, f32, a, (hipStream_t)hip_stream);
    return launch_fill_law(s->engine, law, f32, a, (hipStream_t)hip_stream);
}

extern "C" int rp_fill_law(rp_streams *s, int law, const double *p, int np, double *d_out, uint64_t per_stream,
                           void *hip_stream)
{
    return fill_law_impl(s, law, p, np, d_out, per_stream, hip_stream, false);
}

extern "C" int rp_fill_lawf(rp_streams *s, int law, const double *p, int np, float *d_out, uint64_t per_stream,
                            void *hip_stream)
{
    return fill_law_impl(s, law, p, np, d_out, per_stream, hip_stream, true);
}

// ---------------------------------------------------------------------------
// lane-per-substream samplers
static FillArgs state_args(rp_streams *s, uint64_t per_stream)
{
    FillArgs a{};
    a.words = s->d_words;
    a.phase = s->d_phase;
    a.n = s->n;
    a.per_stream = per_stream;
    a.flags = settings_flags(s);
    return a;
}

extern "C" int rp_norm_moments(rp_streams *s, uint64_t per_stream, double *d_sum, double *d_sumsq,
                               void *hip_stream)
{
    if (!s) return fail(RP_ENULL, "rp_norm_moments: NULL streams");
    if (s->n == 0) return RP_OK;
    if (!d_sum || !d_sumsq) return fail(RP_ENULL, "rp_norm_moments: NULL output");
    if ((uintptr_t)d_sum % 8 || (uintptr_t)d_sumsq % 8)
        return fail(RP_EINVAL, "rp_norm_moments: outputs not aligned to 8 bytes");
    int rc = ensure_device_tables();
    if (rc) return rc;
    SampArgs a{};
    a.f = state_args(s, per_stream);
    a.count = s->n;
    a.sum = d_sum;
    a.sumsq = d_sumsq;
    return launch_moments(s->engine, a, (hipStream_t)hip_stream);
}

static int elem_common(const char *who, rp_streams *s, const float *pa, const float *pb, bool beta, float *z,
                       uint64_t n, void *hip_stream)
{
    if (!s) return fail(RP_ENULL, "%s: NULL streams", who);
    if (n == 0) return RP_OK;
    if (!pa || !z || (beta && !pb)) return fail(RP_ENULL, "%s: NULL device pointer", who);
    if (n > s->n) return fail(RP_EINVAL, "%s: %llu elements but only %llu substreams", who,
                              (unsigned long long)n, (unsigned long long)s->n);
    if ((uintptr_t)pa % 4 || (uintptr_t)z % 4 || (beta && (uintptr_t)pb % 4))
        return fail(RP_EINVAL, "%s: pointers not aligned to 4 bytes", who);
    int rc = ensure_device_tables();
    if (rc) return rc;
    SampArgs a{};
    a.f = state_args(s, 1);
    a.count = n;
    a.pa = pa;
    a.pb = pb;
    a.z = z;
    return launch_gamma_elem(s->engine, a, beta, (hipStream_t)hip_stream);
}

extern "C" int rp_gamma_elem(rp_streams *s, const float *d_alpha, float *d_z, uint64_t n, void *hip_stream)
{
    return elem_common("rp_gamma_elem", s, d_alpha, nullptr, false, d_z, n, hip_stream);
}

extern "C" int rp_beta_elem(rp_streams *s, const float *d_a, const float *d_b, float *d_z, uint64_t n,
                            void *hip_stream)
{
    return elem_common("rp_beta_elem", s, d_a, d_b, true, d_z, n, hip_stream);
}

// ---------------------------------------------------------------------------
// serial split of one stream
namespace {

// Words consumed from (state, phase): block engines move the counter by whole
// blocks and keep the remainder as the phase.
int advance_words(rp_rng *r, uint64_t w)
{
    const int B = block_words(r->engine);
    if (B <= 1) return advance_impl(r, w, 0);
    const uint64_t p = (uint64_t)r->phase + w;
    r->phase = (uint32_t)(p % (uint64_t)B);
    return advance_impl(r, p / (uint64_t)B, 0);
}

// Jump data for lanes C words apart (cached for the last C of each engine).
struct SerialTables {
    std::mutex mu;
    uint64_t c_x256 = 0, c_pcg = 0, c_rl = 0;
    uint64_t x256[304], pcg[72], rl[162];
} g_ser;

void serial_tables(int engine, uint64_t C, uint64_t *jt)
{
    std::lock_guard<std::mutex> lock(g_ser.mu);
    switch (engine) {
    case RP_X256PP:
    case RP_X256SS:
        if (g_ser.c_x256 != C) {
            // lanes l < 64: x^(l C) mod P; waves: x^(64 C 2^k), k < 12
            const Poly &P = x256_charpoly();
            const Poly q = poly_xpow(C, 0, P);
            Poly cur;
            cur.flip(0);
            for (int l = 0; l < 64; l++) {
                memcpy(&g_ser.x256[4 * l], cur.w, 32);
                cur = poly_mulmod(cur, q, P);
            }
            for (int k = 0; k < 12; k++) {
                memcpy(&g_ser.x256[256 + 4 * k], cur.w, 32);
                cur = poly_mulmod(cur, cur, P);
            }
            g_ser.c_x256 = C;
        }
        memcpy(jt, g_ser.x256, sizeof g_ser.x256);
        break;
    case RP_PCG64:
        if (g_ser.c_pcg != C) {
            for (int k = 0; k < 18; k++) {
                const PcgAffine m = pcg_power(C << k, k ? C >> (64 - k) : 0);
                g_ser.pcg[4 * k] = m.mult.lo;
                g_ser.pcg[4 * k + 1] = m.mult.hi;
                g_ser.pcg[4 * k + 2] = m.plus.lo;
                g_ser.pcg[4 * k + 3] = m.plus.hi;
            }
            g_ser.c_pcg = C;
        }
        memcpy(jt, g_ser.pcg, sizeof g_ser.pcg);
        break;
    case RP_RANLUX:
        if (g_ser.c_rl != C) {
            uint64_t e = C / 9, a[9];
            ranlux_pow(ranlux_A(), &e, 1, a);
            for (int k = 0; k < 18; k++) {
                memcpy(&g_ser.rl[9 * k], a, 72);
                rl_mulmod(a, a, a);
            }
            g_ser.c_rl = C;
        }
        memcpy(jt, g_ser.rl, sizeof g_ser.rl);
        break;
    default: break;
    }
}

void plan_lanes(SerialArgs &a, uint64_t words, int B)
{
    // about 256 words per lane for short requests; at most 2^16 lanes (1024
    // wavefronts) for long ones: with the wavefront writing whole lines that
    // already keeps the stores near the fill bandwidth (2^18 lanes measured
    // no faster), and fewer lanes need fewer jumps
    uint64_t L = (words + 255) / 256;
    if (L < 1) L = 1;
    if (L > (1u << 16)) L = 1u << 16;
    uint64_t C = (words + L - 1) / L;
    C = (C + B - 1) / B * B;
    if (C == 0) C = B;
    a.C = C;
    a.lanes = (uint32_t)((words + C - 1) / C);
    a.words = words;
}

int serial_family(int engine)
{
    switch (engine) {
    case RP_PHILOX4X32:
    case RP_PHILOX:
    case RP_CHACHA20: return RP_SUB_KEY;
    case RP_PCG64: return RP_SUB_INC;
    case RP_SFC64:
    case RP_CWG128:
    case RP_X256PPS:
    case RP_X256SSS:
    case RP_SFC64S: return RP_SUB_SPAWN;
    default: return RP_SUB_JUMP;
    }
}

// The whole request on one substream holding the stream's state (one lane
// or one wavefront), then the state copied back.
int serial_fallback(rp_rng *rng, int dist, int dtype, uint64_t bound, int flags, void *d_out, uint64_t n,
                    hipStream_t st)
{
    rp_streams *s = nullptr;
    int rc = rp_streams_create(rng, serial_family(rng->engine), 1, 64, &s);
    if (rc) return rc;
    uint64_t words[32];
    uint32_t ph = rng->phase;
    memcpy(words, rng->st, sizeof words);
    rc = rp_streams_set(s, words, &ph);
    if (rc == RP_OK) rc = rp_fill(s, dist, dtype, bound, flags, d_out, n, st);
    if (rc == RP_OK) {
        const hipError_t e = hipStreamSynchronize(st);
        if (e != hipSuccess) rc = hip_fail(e, "rp_fill_serial");
    }
    if (rc == RP_OK) rc = rp_streams_get(s, words, &ph);
    if (rc == RP_OK) {
        memcpy(rng->st, words, (size_t)state_words(rng->engine) * 8);
        rng->phase = ph;
    }
    rp_streams_free(s);
    return rc;
}

}  // namespace

extern "C" int rp_fill_serial(rp_rng *rng, int dist, int dtype, uint64_t bound, int flags, void *d_out, uint64_t n,
                              void *hip_stream)
{
    if (!rng) return fail(RP_ENULL, "rp_fill_serial: NULL rng");
    if (n == 0) return RP_OK;
    if (!d_out) return fail(RP_ENULL, "rp_fill_serial: NULL output");
    bool ok = false;
    switch (dist) {
    case RP_RAW: ok = dtype == RP_U64 || dtype == RP_U32; break;
    case RP_U01: ok = dtype == RP_F64 || dtype == RP_F32; break;
    case RP_BOUNDED: ok = dtype == RP_U64 || (dtype == RP_U32 && bound <= 0xFFFFFFFFull); break;
    case RP_NORM:
    case RP_EXP: ok = dtype == RP_F64 || dtype == RP_F32; break;
    default: return fail(RP_EINVAL, "rp_fill_serial: unknown distribution %d", dist);
    }
    if (!ok) return fail(RP_EUNSUPPORTED, "rp_fill_serial: distribution %d has no dtype %d form", dist, dtype);
    if (flags & ~RP_FLAG_52BIT) return fail(RP_EINVAL, "rp_fill_serial: unknown flags 0x%x", flags);
    if (!rng->full_mantissa) flags |= RP_FLAG_52BIT;
    const bool half = dtype == RP_U32 || dtype == RP_F32;
    if ((uintptr_t)d_out % (half ? 4 : 8)) return fail(RP_EINVAL, "rp_fill_serial: output not aligned");
    if (n > (1ull << 40)) return fail(RP_EINVAL, "rp_fill_serial: n above 2^40");
    int rc = ensure_device_tables();
    if (rc) return rc;
    hipStream_t st = (hipStream_t)hip_stream;
    // sfc64 and cwg128 have no jump; the 128-bit xor and SIMD engines have no lane jump tables
    if (rng->engine == RP_SFC64 || rng->engine == RP_XORO128 || rng->engine == RP_XS128 ||
        rng->engine == RP_CWG128 || is_simd(rng->engine))
        return serial_fallback(rng, dist, dtype, bound, flags, d_out, n, st);
    SerialArgs a{};
    memcpy(a.base, rng->st, sizeof a.base);
    a.phase = rng->phase;
    a.fa.out = d_out;
    a.fa.bound = bound;
    a.fa.flags = flags | (rng->squeeze ? 0 : kFlagNoSqueeze) | (rng->bitexact ? kFlagBitexact : 0);
    if (dist == RP_BOUNDED && bound) {
        if (dtype == RP_U64) a.fa.thresh = (0 - bound) % bound;
        else a.fa.thresh = (uint32_t)(0u - (uint32_t)bound) % (uint32_t)bound;
    }
    a.n = n;
    const int B = block_words(rng->engine);
    const bool fixed = dist == RP_RAW || dist == RP_U01 || (dist == RP_BOUNDED && bound == 0);
    if (fixed) {
        const uint64_t words = half ? (n + 1) / 2 : n;
        plan_lanes(a, words, B);
        serial_tables(rng->engine, a.C, a.jt);
        rc = launch_serial_fixed(rng->engine, dist, dtype, a, st);
        if (rc) return rc;
        return advance_words(rng, words);
    }
    // rejection samplers: enough units that n samples are found in all but
    // astronomically rare cases (then the one-lane fill takes over)
    uint64_t units;
    if (dist == RP_BOUNDED) {
        const double rej = dtype == RP_U64 ? (double)a.fa.thresh * 0x1.0p-64 : (double)a.fa.thresh * 0x1.0p-32;
        units = (uint64_t)((double)n / (1.0 - rej) * 1.03) + 64;
    } else {
        units = n + n / 16 + 64;
    }
    const uint64_t margin = 2 * (uint64_t)8192 + 16;  // longest attempt: a normal tail at its iteration cap
    const uint64_t gen_units = units + margin;
    plan_lanes(a, half ? (gen_units + 1) / 2 : gen_units, B);
    serial_tables(rng->engine, a.C, a.jt);
    a.units = units;
    const int S = serial_chunk_units(), E = serial_entries(), CB = serial_chunks_per_block();
    a.nchunks = (units + S - 1) / S;
    a.nblocks = (a.nchunks + CB - 1) / CB;
    auto al = [](uint64_t x) { return (x + 255) & ~255ull; };
    const uint64_t o_wbuf = 0, o_cexit = al(o_wbuf + a.words * 8), o_ccount = al(o_cexit + a.nchunks * E),
                   o_bexit = al(o_ccount + a.nchunks * E * 4), o_bcount = al(o_bexit + a.nblocks * E),
                   o_bentry = al(o_bcount + a.nblocks * E * 4), o_bbase = al(o_bentry + a.nblocks),
                   o_res = al(o_bbase + a.nblocks * 8), total = al(o_res + 64);
    char *ws = nullptr;
    hipError_t e = hipMallocAsync((void **)&ws, total, st);
    if (e != hipSuccess) return fail(RP_ENOMEM, "rp_fill_serial: workspace: %s", hipGetErrorString(e));
    a.wbuf = (uint64_t *)(ws + o_wbuf);
    a.cexit = (uint8_t *)(ws + o_cexit);
    a.ccount = (uint32_t *)(ws + o_ccount);
    a.bexit = (uint8_t *)(ws + o_bexit);
    a.bcount = (uint32_t *)(ws + o_bcount);
    a.bentry = (uint8_t *)(ws + o_bentry);
    a.bbase = (uint64_t *)(ws + o_bbase);
    a.result = (uint64_t *)(ws + o_res);
    static thread_local uint64_t *h_res = nullptr;
    if (!h_res) {
        e = hipHostMalloc((void **)&h_res, 64, hipHostMallocDefault);
        if (e != hipSuccess) {
            h_res = nullptr;
            (void)hipFreeAsync(ws, st);
            return fail(RP_ENOMEM, "rp_fill_serial: pinned result buffer: %s", hipGetErrorString(e));
        }
    }
    rc = launch_serial_stitch(rng->engine, dist, dtype, a, st);
    if (rc == RP_OK) {
        e = hipMemcpyAsync(h_res, a.result, 3 * sizeof(uint64_t), hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) rc = hip_fail(e, "rp_fill_serial");
    }
    (void)hipFreeAsync(ws, st);
    if (rc) return rc;
    if (h_res[2] != 0 || h_res[1] < n) return serial_fallback(rng, dist, dtype, bound, flags, d_out, n, st);
    const uint64_t end = h_res[0];
    return advance_words(rng, half ? (end + 1) / 2 : end);
}
