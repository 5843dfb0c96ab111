/*
 * oracle.c -- reference oracle for the Randompack hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  A plain, slow, scalar C implementation of the
 * engines, seeding, stream control and samplers that the GPU library computes.
 * Only the test suite, the smoke check and the CPU-baseline leg of the
 * benchmark load it.  It shares no source, header, table or generator with the
 * GPU library (paper_2605_05099_amd/csrc), and it never calls it.
 *
 * Every routine follows the *serial definition*: the outputs of a stream are
 * what consecutive calls of one scalar generator produce.  Floating point is
 * IEEE binary64 (binary32 for the float outputs) with round-to-nearest; the
 * file is compiled with -ffp-contract=off -fno-fast-math so that every
 * expression is evaluated exactly as written (no fused multiply-add).
 *
 * Citations name the paper's sections, tables and figures (Randompack,
 * arXiv 2605.05099).  Where the paper is silent, the reading taken is stated
 * next to the code.
 *
 * Parity status of each part (pins live in tests/test_oracle_*.py):
 *   pcg64, philox4x64, sfc64 engines       pinned: NumPy bit generators
 *   philox4x32-10                          pinned: rocRAND host engine + derived Weyl constants
 *   xoshiro256++ linear core               pinned: primitive characteristic polynomial
 *   xoshiro256++ output scrambler          parity unpinned (no external implementation here)
 *   xoshiro256** output scrambler          parity unpinned (no external implementation here)
 *   squares64 output function              parity unpinned (no external implementation here)
 *   xoroshiro128++, xorshift128+ cores     pinned: primitive characteristic polynomials (period 2^128-1)
 *   their output scramblers                parity unpinned (no external implementation here)
 *   chacha20 block function                pinned: RFC 8439 quarter-round and block examples
 *   cwg128 step and output                 parity unpinned (the paper names the engine but does
 *                                          not define it; reading below; Weyl-part invariants only)
 *   x256++simd, x256**simd, sfc64simd      interleave of eight scalar sub-streams: pinned to the
 *                                          scalar engines (each sub-stream equals its jumped or
 *                                          counter-offset scalar stream); the order of the eight
 *                                          words of a round is a reading (parity unpinned)
 *   ranlux++                               pinned: modulus/multiplier/period, big-integer arithmetic
 *   seeding mixer (seed_seq_fe128)         pinned: NumPy SeedSequence
 *   u01 / u01f / bounded ints              pinned: NumPy Generator
 *   ziggurat normal                        pinned: NumPy layout/ratio test, geometry, rates, KS
 *   ziggurat exponential                   pinned: geometry, paper's rejection rate, KS
 *   float ziggurat (normf, expf)           pinned: KS, fast-accept rates, strip boundaries, tails
 *   permutations, Floyd / reservoir samples pinned: exact laws on small cases (enumeration), validity
 *   float gamma (gammaf)                   pinned: KS against the gamma law, moments
 *   gamma (alpha >= 1)                     pinned: NumPy Marsaglia-Tsang, moments, KS
 *   gamma boost (alpha < 1), beta          pinned: mpmath power, moments, KS
 */
#include <math.h>
#include <quadmath.h>
#include <stddef.h>
#include <stdint.h>
#include <string.h>

#include "zig_tables.h"

typedef unsigned __int128 u128;

/* ------------------------------------------------------------------------ */
/* Engine identifiers (Table 2; philox4x32 is the 32-bit sibling of the     */
/* paper's Philox-4x64 from the same Random123 family).                     */
/* ------------------------------------------------------------------------ */
enum {
    OR_X256PP = 0,
    OR_PCG64 = 1,
    OR_PHILOX4X32 = 2,
    OR_PHILOX4X64 = 3,
    OR_SFC64 = 4,
    OR_RANLUX = 5,
    OR_X256SS = 6,
    OR_SQUARES = 7,
    OR_XORO128PP = 8,
    OR_XS128P = 9,
    OR_CHACHA20 = 10,
    OR_CWG128 = 11,
    OR_X256PPS = 12, /* x256++simd: eight interleaved xoshiro256++ sub-streams */
    OR_X256SSS = 13, /* x256**simd */
    OR_SFC64S = 14,  /* sfc64simd: eight interleaved sfc64 sub-streams */
    OR_NENGINE = 15
};

/*
 * One serial stream.  'phase' counts the 64-bit words already taken from the
 * current output block of a block engine (Philox-4x32: 2 words per block,
 * Philox-4x64: 4, ranlux++: 9; Section 4.3 describes 9-word ranlux++ chunks).
 * For one-word engines phase is always 0.
 *
 * State words (Table 3 order):
 *   x256++      st[0..3] = s0..s3
 *   pcg64       st[0..1] = state (lo, hi), st[2..3] = increment (lo, hi)
 *   philox4x32  st[0..1] = 128-bit counter (lo, hi), st[2] = key (k0 | k1 << 32)
 *   philox4x64  st[0..3] = 256-bit counter, st[4..5] = key
 *   sfc64       st[0..3] = a, b, c, counter
 *   ranlux++    st[0..8] = x (576 bits, little-endian limbs), 0 < x < m
 *   cwg128      st[0..1] = x, st[2..3] = a, st[4..5] = Weyl sequence,
 *               st[6..7] = Weyl increment (odd); 128-bit words, low first
 *   *simd       st[4k .. 4k+3] = sub-stream k (k < 8) as the scalar engine's
 *               four words; a block is one word of each sub-stream, in
 *               sub-stream order (Section 4.1: eight disjoint scalar streams,
 *               buffers filled in 8-word chunks)
 * For block engines the current block is the one computed from st; after its
 * last word is consumed st advances (counter + 1, or x <- A x mod m).
 */
typedef struct {
    uint64_t engine;
    uint64_t phase;
    uint64_t st[32];
    uint64_t blk[9];
    uint64_t blk_ok;
} or_stream;

/* Event counts used by the rate pins (all optional). */
typedef struct {
    uint64_t words;       /* 64-bit words consumed                           */
    uint64_t candidates;  /* ziggurat candidates (leading words)             */
    uint64_t pdf_evals;   /* exp() evaluations in wedge tests                */
    uint64_t tail_entries;/* candidates that fell in the base-strip tail     */
    uint64_t tail_logs;   /* log1p() evaluations in tail sampling            */
    uint64_t rejections;  /* ziggurat candidates rejected                    */
    uint64_t mt_attempts; /* Marsaglia-Tsang attempts                        */
    uint64_t mt_logtests; /* Marsaglia-Tsang attempts needing the log test   */
} or_counts;

size_t or_stream_words(void) { return sizeof(or_stream) / 8; }
size_t or_counts_words(void) { return sizeof(or_counts) / 8; }

static inline uint64_t rotl64(uint64_t x, int k) { return (x << k) | (x >> (64 - k)); }

/* ------------------------------------------------------------------------ */
/* xoshiro256++ (Blackman and Vigna; Table 2 "x256++").                      */
/* The linear map T on F_2^256 and the "++" output rotl(s0 + s3, 23) + s0,   */
/* the output being taken from the state before the update.                  */
/* ------------------------------------------------------------------------ */
static void x256_linear(uint64_t s[4])
{
    uint64_t t = s[1] << 17;
    s[2] ^= s[0];
    s[3] ^= s[1];
    s[1] ^= s[2];
    s[0] ^= s[3];
    s[2] ^= t;
    s[3] = rotl64(s[3], 45);
}

static uint64_t x256pp_word(uint64_t s[4])
{
    uint64_t out = rotl64(s[0] + s[3], 23) + s[0];
    x256_linear(s);
    return out;
}

/* xoshiro256** (Blackman and Vigna 2018; Table 2 "x256**"): the same linear
 * map T, with the "**" output rotl(5 s1, 7) 9 of the state before the
 * update.  Seeding, jumps and substreams are those of xoshiro256++. */
static uint64_t x256ss_word(uint64_t s[4])
{
    uint64_t out = rotl64(s[1] * 5u, 7) * 9u;
    x256_linear(s);
    return out;
}

/* ------------------------------------------------------------------------ */
/* xoroshiro128++ (Blackman and Vigna 2019; Table 2 "xoro++") and           */
/* xorshift128+ (Vigna; Table 2 "x128+"), two state words each.  The ++     */
/* output is rotl(s0 + s1, 17) + s0 and the + output s0 + s1, both of the   */
/* state before the update.  xorshift128+ uses the shift triple (23, 18, 5) */
/* of the current reference code (the 2014 paper's constants were           */
/* (23, 17, 26)).                                                            */
/* ------------------------------------------------------------------------ */
static void xoro128_linear(uint64_t s[2])
{
    uint64_t s0 = s[0], s1 = s[1];
    s1 ^= s0;
    s[0] = rotl64(s0, 49) ^ s1 ^ (s1 << 21);
    s[1] = rotl64(s1, 28);
}

static uint64_t xoro128pp_word(uint64_t s[2])
{
    uint64_t out = rotl64(s[0] + s[1], 17) + s[0];
    xoro128_linear(s);
    return out;
}

static void xs128_linear(uint64_t s[2])
{
    uint64_t a = s[0];
    const uint64_t b = s[1];
    s[0] = b;
    a ^= a << 23;
    s[1] = a ^ b ^ (a >> 18) ^ (b >> 5);
}

static uint64_t xs128p_word(uint64_t s[2])
{
    uint64_t out = s[0] + s[1];
    xs128_linear(s);
    return out;
}

/* one step of a 128-bit linear core (characteristic polynomials) */
int or_x128_linear_steps(uint64_t engine, uint64_t st[2], uint64_t *bit0_out, size_t n)
{
    if (engine != OR_XORO128PP && engine != OR_XS128P) return -1;
    for (size_t i = 0; i < n; i++) {
        bit0_out[i] = st[0] & 1u;
        if (engine == OR_XORO128PP) xoro128_linear(st);
        else xs128_linear(st);
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* ChaCha20 (Bernstein; Table 2 "chacha20"; Table 3: key (4) + nonce (1.5) + */
/* counter (0.5)).  Reading: st[0..3] hold the 256-bit key (32-bit words     */
/* low half first), st[4] and the low half of st[5] the 96-bit nonce, the    */
/* high half of st[5] the 32-bit block counter.  A block is the 20-round     */
/* ChaCha permutation (ten column-and-diagonal double rounds) of the input   */
/* words (the four "expand 32-byte k" constants, key, counter, nonce), the   */
/* input added back; its 16 words give 8 64-bit words, the earlier word in  */
/* the low half.  The counter advances by one per block (period 2^35 words). */
/* ------------------------------------------------------------------------ */
static uint32_t rotl32(uint32_t x, int k) { return (x << k) | (x >> (32 - k)); }

static void chacha_qr(uint32_t x[16], int a, int b, int c, int d)
{
    x[a] += x[b]; x[d] ^= x[a]; x[d] = rotl32(x[d], 16);
    x[c] += x[d]; x[b] ^= x[c]; x[b] = rotl32(x[b], 12);
    x[a] += x[b]; x[d] ^= x[a]; x[d] = rotl32(x[d], 8);
    x[c] += x[d]; x[b] ^= x[c]; x[b] = rotl32(x[b], 7);
}

/* one quarter round on four words (exposed for the tests) */
void or_chacha_qr(uint32_t q[4])
{
    uint32_t x[16] = {0};
    x[0] = q[0];
    x[1] = q[1];
    x[2] = q[2];
    x[3] = q[3];
    chacha_qr(x, 0, 1, 2, 3);
    memcpy(q, x, 16);
}

static void or_chacha20_block(const uint64_t st[6], uint64_t out[8])
{
    uint32_t in[16] = {0x61707865u, 0x3320646eu, 0x79622d32u, 0x6b206574u};
    for (int i = 0; i < 4; i++) {
        in[4 + 2 * i] = (uint32_t)st[i];
        in[5 + 2 * i] = (uint32_t)(st[i] >> 32);
    }
    in[12] = (uint32_t)(st[5] >> 32);
    in[13] = (uint32_t)st[4];
    in[14] = (uint32_t)(st[4] >> 32);
    in[15] = (uint32_t)st[5];
    uint32_t x[16];
    memcpy(x, in, sizeof x);
    for (int r = 0; r < 10; r++) {
        chacha_qr(x, 0, 4, 8, 12);
        chacha_qr(x, 1, 5, 9, 13);
        chacha_qr(x, 2, 6, 10, 14);
        chacha_qr(x, 3, 7, 11, 15);
        chacha_qr(x, 0, 5, 10, 15);
        chacha_qr(x, 1, 6, 11, 12);
        chacha_qr(x, 2, 7, 8, 13);
        chacha_qr(x, 3, 4, 9, 14);
    }
    for (int k = 0; k < 8; k++)
        out[k] = (uint64_t)(x[2 * k] + in[2 * k]) | ((uint64_t)(x[2 * k + 1] + in[2 * k + 1]) << 32);
}

/* ------------------------------------------------------------------------ */
/* squares64 (Widynski; Table 2 "squares", Table 3: counter (1) + key (1)).  */
/* Word = five rounds on x = counter * key: square, add y = x0 or            */
/* z = x0 + key alternately, swap the 32-bit halves; the fourth round's      */
/* value t is kept and the fifth returns t ^ ((x^2 + y) >> 32).  The counter */
/* then increases by one (period 2^64 per key).                              */
/* ------------------------------------------------------------------------ */
static uint64_t swap32(uint64_t x) { return (x >> 32) | (x << 32); }

static uint64_t squares_word(uint64_t st[2])
{
    uint64_t x = st[0] * st[1];
    uint64_t y = x, z = y + st[1];
    x = swap32(x * x + y);
    x = swap32(x * x + z);
    x = swap32(x * x + y);
    uint64_t t = x * x + z;
    x = swap32(t);
    st[0] += 1u;
    return t ^ ((x * x + y) >> 32);
}

/* ------------------------------------------------------------------------ */
/* PCG64 DXSM (O'Neill 2019; Table 2 "pcg64").  128-bit LCG with the 64-bit  */
/* "cheap" multiplier; output is the DXSM permutation of the state before    */
/* the step (this is the form NumPy ships, which the paper validates         */
/* against).                                                                 */
/* ------------------------------------------------------------------------ */
#define OR_PCG_MULT 0xda942042e4dd58b5ULL

static uint64_t pcg64_word(uint64_t st[4])
{
    u128 s = ((u128)st[1] << 64) | st[0];
    u128 inc = ((u128)st[3] << 64) | st[2];
    uint64_t hi = (uint64_t)(s >> 64);
    uint64_t lo = (uint64_t)s | 1u;
    hi ^= hi >> 32;
    hi *= OR_PCG_MULT;
    hi ^= hi >> 48;
    hi *= lo;
    s = s * (u128)OR_PCG_MULT + inc;
    st[0] = (uint64_t)s;
    st[1] = (uint64_t)(s >> 64);
    return hi;
}

/* ------------------------------------------------------------------------ */
/* Philox (Salmon, Moraes, Dror, Shaw 2011).  Ten rounds; the key is bumped  */
/* by the Weyl constants before every round but the first.                   */
/* ------------------------------------------------------------------------ */
#define OR_PH32_M0 0xD2511F53u
#define OR_PH32_M1 0xCD9E8D57u
#define OR_PH32_W0 0x9E3779B9u /* floor(2^32 (golden ratio - 1)) */
#define OR_PH32_W1 0xBB67AE85u /* floor(2^32 (sqrt(3) - 1))       */
#define OR_PH64_M0 0xD2E7470EE14C6C93ULL
#define OR_PH64_M1 0xCA5A826395121157ULL
#define OR_PH64_W0 0x9E3779B97F4A7C15ULL /* floor(2^64 (golden ratio - 1)) */
#define OR_PH64_W1 0xBB67AE8584CAA73BULL /* floor(2^64 (sqrt(3) - 1))       */

void or_philox4x32_block(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; round++) {
        if (round > 0) {
            k0 += OR_PH32_W0;
            k1 += OR_PH32_W1;
        }
        uint64_t p0 = (uint64_t)OR_PH32_M0 * c0;
        uint64_t p1 = (uint64_t)OR_PH32_M1 * c2;
        uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
        uint32_t n1 = (uint32_t)p1;
        uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
        uint32_t n3 = (uint32_t)p0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

void or_philox4x64_block(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4])
{
    uint64_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint64_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; round++) {
        if (round > 0) {
            k0 += OR_PH64_W0;
            k1 += OR_PH64_W1;
        }
        u128 p0 = (u128)OR_PH64_M0 * c0;
        u128 p1 = (u128)OR_PH64_M1 * c2;
        uint64_t n0 = (uint64_t)(p1 >> 64) ^ c1 ^ k0;
        uint64_t n1 = (uint64_t)p1;
        uint64_t n2 = (uint64_t)(p0 >> 64) ^ c3 ^ k1;
        uint64_t n3 = (uint64_t)p0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

void or_philox_constants(uint64_t out[8])
{
    out[0] = OR_PH32_M0; out[1] = OR_PH32_M1; out[2] = OR_PH32_W0; out[3] = OR_PH32_W1;
    out[4] = OR_PH64_M0; out[5] = OR_PH64_M1; out[6] = OR_PH64_W0; out[7] = OR_PH64_W1;
}

/* ------------------------------------------------------------------------ */
/* sfc64 (Doty-Humphrey, PractRand; Table 2 "sfc64").                        */
/* ------------------------------------------------------------------------ */
static uint64_t sfc64_word(uint64_t st[4])
{
    uint64_t a = st[0], b = st[1], c = st[2], ctr = st[3];
    uint64_t out = a + b + ctr;
    st[0] = b ^ (b >> 11);
    st[1] = c + (c << 3);
    st[2] = rotl64(c, 24) + out;
    st[3] = ctr + 1;
    return out;
}

/* ------------------------------------------------------------------------ */
/* cwg128 (Dziala's Collatz-Weyl generator; Table 2 "cwg128", Table 3: state */
/* of six words plus a two-word Weyl increment).  The paper names the engine */
/* but does not give its step; the reading here is the generator's published */
/* 128-bit form: the Weyl sequence grows by the odd increment s each step,   */
/* a accumulates x, and x becomes (x >> 1) (a | 1) xor weyl, all modulo      */
/* 2^128; the 128-bit output is (a >> 96) xor x, of which the 64-bit word is */
/* the low half (the half that every term of the output reaches).            */
/* ------------------------------------------------------------------------ */
static uint64_t cwg128_word(uint64_t st[8])
{
    u128 x = ((u128)st[1] << 64) | st[0];
    u128 a = ((u128)st[3] << 64) | st[2];
    u128 weyl = ((u128)st[5] << 64) | st[4];
    const u128 inc = ((u128)st[7] << 64) | st[6];
    a += x;
    weyl += inc;
    x = ((x >> 1) * (a | 1)) ^ weyl;
    st[0] = (uint64_t)x;
    st[1] = (uint64_t)(x >> 64);
    st[2] = (uint64_t)a;
    st[3] = (uint64_t)(a >> 64);
    st[4] = (uint64_t)weyl;
    st[5] = (uint64_t)(weyl >> 64);
    return (uint64_t)((a >> 96) ^ x);
}

/* ------------------------------------------------------------------------ */
/* ranlux++ (Sibidanov 2017; Table 2 "ranlux++").  The LCG form of the       */
/* RANLUX subtract-with-borrow generator with base b = 2^24, lags r = 24,    */
/* s = 10:  m = b^r - b^s + 1 = 2^576 - 2^240 + 1,  a = m - (m - 1)/b.       */
/* One engine step is x <- A x mod m with A = a^p; p = 2048 is the luxury    */
/* taken here (the paper does not state p).  Each step outputs the nine      */
/* 64-bit limbs of the new x, least significant first (Section 4.3).         */
/* Multi-limb arithmetic below is schoolbook, on little-endian 64-bit limbs. */
/* ------------------------------------------------------------------------ */
#define RL_N 9   /* limbs of a residue            */
#define RL_W 20  /* limbs of a working integer    */
#define OR_RANLUX_P 2048

/* r = a + b over n limbs, returns carry */
static uint64_t mp_add(uint64_t *r, const uint64_t *a, const uint64_t *b, int n)
{
    uint64_t carry = 0;
    for (int i = 0; i < n; i++) {
        u128 t = (u128)a[i] + b[i] + carry;
        r[i] = (uint64_t)t;
        carry = (uint64_t)(t >> 64);
    }
    return carry;
}

/* r = a - b over n limbs, returns borrow */
static uint64_t mp_sub(uint64_t *r, const uint64_t *a, const uint64_t *b, int n)
{
    uint64_t borrow = 0;
    for (int i = 0; i < n; i++) {
        uint64_t ai = a[i], bi = b[i];
        uint64_t d = ai - bi - borrow;
        borrow = (ai < bi) || (ai == bi && borrow) ? 1 : 0;
        r[i] = d;
    }
    return borrow;
}

static int mp_cmp(const uint64_t *a, const uint64_t *b, int n)
{
    for (int i = n - 1; i >= 0; i--) {
        if (a[i] != b[i]) return a[i] < b[i] ? -1 : 1;
    }
    return 0;
}

static int mp_is_zero(const uint64_t *a, int n)
{
    for (int i = 0; i < n; i++)
        if (a[i]) return 0;
    return 1;
}

/* r = a << sh (bits) over n limbs (bits shifted out are lost) */
static void mp_shl(uint64_t *r, const uint64_t *a, int sh, int n)
{
    uint64_t tmp[RL_W * 2];
    int limbs = sh / 64, bits = sh % 64;
    for (int i = 0; i < n; i++) tmp[i] = 0;
    for (int i = n - 1; i >= 0; i--) {
        int src = i - limbs;
        if (src < 0) continue;
        uint64_t v = a[src] << bits;
        if (bits && src - 1 >= 0) v |= a[src - 1] >> (64 - bits);
        tmp[i] = v;
    }
    memcpy(r, tmp, (size_t)n * 8);
}

/* r = a >> sh (bits) over n limbs */
static void mp_shr(uint64_t *r, const uint64_t *a, int sh, int n)
{
    uint64_t tmp[RL_W * 2];
    int limbs = sh / 64, bits = sh % 64;
    for (int i = 0; i < n; i++) {
        int src = i + limbs;
        uint64_t v = 0;
        if (src < n) {
            v = a[src] >> bits;
            if (bits && src + 1 < n) v |= a[src + 1] << (64 - bits);
        }
        tmp[i] = v;
    }
    memcpy(r, tmp, (size_t)n * 8);
}

/* the modulus m = 2^576 - 2^240 + 1 as RL_W limbs */
static void rl_modulus(uint64_t m[RL_W])
{
    uint64_t one[RL_W] = {1}, p576[RL_W] = {0}, p240[RL_W] = {0};
    p576[9] = 1;            /* 2^576 */
    p240[3] = 1ULL << 48;   /* 2^240 = 2^(3*64 + 48) */
    mp_sub(m, p576, p240, RL_W);
    mp_add(m, m, one, RL_W);
}

/* x mod m for a working integer x (RL_W limbs); result in r[0..8].
 * Folding identity: 2^576 = 2^240 - 1 (mod m).  With x = H 2^576 + L,
 * x = L + H 2^240 - H (mod m), which is >= 0 and smaller; repeat, then
 * subtract m while the value is >= m. */
static void rl_reduce(uint64_t r[RL_N], const uint64_t x_in[RL_W])
{
    uint64_t m[RL_W], x[RL_W], L[RL_W], H[RL_W], t[RL_W];
    rl_modulus(m);
    memcpy(x, x_in, sizeof x);
    for (;;) {
        memset(H, 0, sizeof H);
        mp_shr(H, x, 576, RL_W);
        if (mp_is_zero(H, RL_W)) break;
        memset(L, 0, sizeof L);
        memcpy(L, x, RL_N * 8);
        mp_shl(t, H, 240, RL_W);
        mp_add(x, L, t, RL_W);
        mp_sub(x, x, H, RL_W);
    }
    while (mp_cmp(x, m, RL_W) >= 0) mp_sub(x, x, m, RL_W);
    memcpy(r, x, RL_N * 8);
}

/* r = a * b mod m for residues a, b (RL_N limbs each) */
static void rl_mulmod(uint64_t r[RL_N], const uint64_t a[RL_N], const uint64_t b[RL_N])
{
    uint64_t prod[RL_W];
    memset(prod, 0, sizeof prod);
    for (int i = 0; i < RL_N; i++) {
        uint64_t carry = 0;
        for (int j = 0; j < RL_N; j++) {
            u128 t = (u128)a[i] * b[j] + prod[i + j] + carry;
            prod[i + j] = (uint64_t)t;
            carry = (uint64_t)(t >> 64);
        }
        prod[i + RL_N] = carry;
    }
    rl_reduce(r, prod);
}

/* r = base^e mod m, e given as 64-bit limbs (ne of them) */
static void rl_powmod(uint64_t r[RL_N], const uint64_t base[RL_N], const uint64_t *e, int ne)
{
    uint64_t acc[RL_N] = {1}, b[RL_N];
    memcpy(b, base, sizeof b);
    for (int i = 0; i < ne; i++) {
        for (int bit = 0; bit < 64; bit++) {
            if ((e[i] >> bit) & 1) rl_mulmod(acc, acc, b);
            rl_mulmod(b, b, b);
        }
    }
    memcpy(r, acc, sizeof acc);
}

/* a = m - (m - 1) / 2^24 */
static void rl_base_multiplier(uint64_t a[RL_N])
{
    uint64_t m[RL_W], one[RL_W] = {1}, q[RL_W], t[RL_W];
    rl_modulus(m);
    mp_sub(t, m, one, RL_W);
    mp_shr(q, t, 24, RL_W);
    mp_sub(t, m, q, RL_W);
    memcpy(a, t, RL_N * 8);
}

static uint64_t rl_A[RL_N];
static int rl_A_ready = 0;

static const uint64_t *rl_step_multiplier(void)
{
    if (!rl_A_ready) {
        uint64_t a[RL_N], e[1] = {OR_RANLUX_P};
        rl_base_multiplier(a);
        rl_powmod(rl_A, a, e, 1);
        rl_A_ready = 1;
    }
    return rl_A;
}

void or_ranlux_constants(uint64_t m_out[10], uint64_t a_out[9], uint64_t A_out[9])
{
    uint64_t m[RL_W];
    rl_modulus(m);
    memcpy(m_out, m, 10 * 8);
    rl_base_multiplier(a_out);
    memcpy(A_out, rl_step_multiplier(), RL_N * 8);
}

/* Exposed for the big-integer pin: r = a * b mod m. */
void or_ranlux_mulmod(uint64_t r[9], const uint64_t a[9], const uint64_t b[9])
{
    rl_mulmod(r, a, b);
}

/* x mod m for a 576-bit value, mapping 0 to 1 (seeding fix-up). */
static void rl_seed_fixup(uint64_t x[RL_N])
{
    uint64_t w[RL_W];
    memset(w, 0, sizeof w);
    memcpy(w, x, RL_N * 8);
    rl_reduce(x, w);
    if (mp_is_zero(x, RL_N)) x[0] = 1;
}

/* ------------------------------------------------------------------------ */
/* Word stream.                                                             */
/* ------------------------------------------------------------------------ */
static int block_words(uint64_t engine)
{
    switch (engine) {
    case OR_PHILOX4X32: return 2;
    case OR_PHILOX4X64: return 4;
    case OR_RANLUX: return 9;
    case OR_CHACHA20: return 8;
    case OR_X256PPS:
    case OR_X256SSS:
    case OR_SFC64S: return 8;
    default: return 1;
    }
}

/* One word of sub-stream k of a SIMD engine, from a copy (the sub-stream
 * itself moves only when the whole block has been used). */
static uint64_t simd_peek(const or_stream *s, int k)
{
    uint64_t t[4];
    memcpy(t, &s->st[4 * k], sizeof t);
    if (s->engine == OR_X256PPS) return x256pp_word(t);
    if (s->engine == OR_X256SSS) return x256ss_word(t);
    return sfc64_word(t);
}

static void make_block(or_stream *s)
{
    switch (s->engine) {
    case OR_X256PPS:
    case OR_X256SSS:
    case OR_SFC64S:
        for (int k = 0; k < 8; k++) s->blk[k] = simd_peek(s, k);
        break;
    case OR_PHILOX4X32: {
        uint32_t ctr[4] = {(uint32_t)s->st[0], (uint32_t)(s->st[0] >> 32),
                           (uint32_t)s->st[1], (uint32_t)(s->st[1] >> 32)};
        uint32_t key[2] = {(uint32_t)s->st[2], (uint32_t)(s->st[2] >> 32)};
        uint32_t y[4];
        or_philox4x32_block(ctr, key, y);
        /* a 64-bit word takes the earlier 32-bit output in its low half */
        s->blk[0] = (uint64_t)y[0] | ((uint64_t)y[1] << 32);
        s->blk[1] = (uint64_t)y[2] | ((uint64_t)y[3] << 32);
        break;
    }
    case OR_PHILOX4X64:
        or_philox4x64_block(&s->st[0], &s->st[4], s->blk);
        break;
    case OR_CHACHA20:
        or_chacha20_block(s->st, s->blk);
        break;
    case OR_RANLUX:
        rl_mulmod(s->blk, s->st, rl_step_multiplier());
        break;
    }
    s->blk_ok = 1;
}

static void advance_block_state(or_stream *s)
{
    switch (s->engine) {
    case OR_PHILOX4X32: {
        u128 c = ((u128)s->st[1] << 64) | s->st[0];
        c += 1;
        s->st[0] = (uint64_t)c;
        s->st[1] = (uint64_t)(c >> 64);
        break;
    }
    case OR_PHILOX4X64:
        for (int i = 0; i < 4; i++) {
            s->st[i] += 1;
            if (s->st[i] != 0) break;
        }
        break;
    case OR_RANLUX:
        memcpy(s->st, s->blk, RL_N * 8);
        break;
    case OR_CHACHA20: /* 32-bit block counter in the high half of st[5] */
        s->st[5] = (s->st[5] & 0xffffffffu) | ((uint64_t)(uint32_t)((s->st[5] >> 32) + 1u) << 32);
        break;
    case OR_X256PPS:
    case OR_X256SSS:
    case OR_SFC64S: /* every sub-stream moves one step */
        for (int k = 0; k < 8; k++) {
            uint64_t *t = &s->st[4 * k];
            if (s->engine == OR_SFC64S) (void)sfc64_word(t);
            else x256_linear(t);
        }
        break;
    }
    s->blk_ok = 0;
}

static uint64_t next_word(or_stream *s)
{
    switch (s->engine) {
    case OR_X256PP: return x256pp_word(s->st);
    case OR_X256SS: return x256ss_word(s->st);
    case OR_SQUARES: return squares_word(s->st);
    case OR_XORO128PP: return xoro128pp_word(s->st);
    case OR_XS128P: return xs128p_word(s->st);
    case OR_PCG64: return pcg64_word(s->st);
    case OR_SFC64: return sfc64_word(s->st);
    case OR_CWG128: return cwg128_word(s->st);
    default: {
        int nb = block_words(s->engine);
        if (!s->blk_ok) make_block(s);
        uint64_t w = s->blk[s->phase];
        s->phase++;
        if ((int)s->phase == nb) {
            s->phase = 0;
            advance_block_state(s);
        }
        return w;
    }
    }
}

static inline uint64_t nx(or_stream *s, or_counts *c)
{
    if (c) c->words++;
    return next_word(s);
}

void or_raw64(or_stream *s, uint64_t *out, size_t n)
{
    for (size_t i = 0; i < n; i++) out[i] = next_word(s);
}

/* ------------------------------------------------------------------------ */
/* Seeding mixer: O'Neill's seed_seq_fe with a 128-bit pool (Section 2.3).   */
/* Input words are hashed into four 32-bit pool words, every pool word is    */
/* mixed into every other, surplus input words are mixed into all of them,   */
/* and output words are hashed out of the pool round-robin.                  */
/* ------------------------------------------------------------------------ */
#define SSQ_INIT_A 0x43b0d7e5u
#define SSQ_MULT_A 0x931e8875u
#define SSQ_INIT_B 0x8b51f9ddu
#define SSQ_MULT_B 0x58f38dedu
#define SSQ_MIX_MULT_L 0xca01f9ddu
#define SSQ_MIX_MULT_R 0x4973f715u
#define SSQ_XSHIFT 16

static uint32_t ssq_hash(uint32_t value, uint32_t *hash_const)
{
    value ^= *hash_const;
    *hash_const *= SSQ_MULT_A;
    value *= *hash_const;
    value ^= value >> SSQ_XSHIFT;
    return value;
}

static uint32_t ssq_mix(uint32_t x, uint32_t y)
{
    uint32_t result = SSQ_MIX_MULT_L * x - SSQ_MIX_MULT_R * y;
    result ^= result >> SSQ_XSHIFT;
    return result;
}

void or_seed_seq(const uint32_t *in, size_t n_in, uint32_t *out, size_t n_out)
{
    uint32_t pool[4];
    uint32_t hc = SSQ_INIT_A;
    for (size_t i = 0; i < 4; i++) pool[i] = ssq_hash(i < n_in ? in[i] : 0u, &hc);
    for (size_t src = 0; src < 4; src++)
        for (size_t dst = 0; dst < 4; dst++)
            if (src != dst) pool[dst] = ssq_mix(pool[dst], ssq_hash(pool[src], &hc));
    for (size_t i = 4; i < n_in; i++)
        for (size_t dst = 0; dst < 4; dst++) pool[dst] = ssq_mix(pool[dst], ssq_hash(in[i], &hc));
    uint32_t hb = SSQ_INIT_B;
    for (size_t i = 0; i < n_out; i++) {
        uint32_t v = pool[i % 4];
        v ^= hb;
        hb *= SSQ_MULT_B;
        v *= hb;
        v ^= v >> SSQ_XSHIFT;
        out[i] = v;
    }
}

/* Words of engine state filled by seeding (Table 2/3 state composition). */
static int seeded_words(uint64_t engine)
{
    switch (engine) {
    case OR_X256PP: return 4;
    case OR_X256SS: return 4;
    case OR_SQUARES: return 2;
    case OR_XORO128PP: return 2;
    case OR_XS128P: return 2;
    case OR_CHACHA20: return 6;
    case OR_PCG64: return 4;
    case OR_PHILOX4X32: return 3;
    case OR_PHILOX4X64: return 6;
    case OR_SFC64: return 3;
    case OR_RANLUX: return 9;
    case OR_CWG128: return 8;
    default: return 0;
    }
}

void or_sfc64_set_abc(or_stream *s, uint64_t a, uint64_t b, uint64_t c);
int or_cwg128_set_weyl(or_stream *s, uint64_t lo, uint64_t hi);

/*
 * Seeding (Section 2.3): the mixer input is the 64-bit seed as two 32-bit
 * words (low first) followed by the spawn-key words.  When a spawn key is
 * given, the seed words are first padded with zeros to the pool size (four
 * words); without this, a key of [0] would reproduce the unkeyed stream,
 * because the mixer pads short inputs with hashed zeros.  The mixer emits two
 * 32-bit words per 64-bit state word (low half first), filled in Table 3
 * order.  Fix-ups: pcg64 increment made odd; an all-zero xoshiro state (the
 * one excluded state) replaced by s0 = 1; ranlux++ x reduced into [1, m);
 * sfc64 goes through its stream setter (counter 1, 18 warm-up steps).
 */
int or_seed(or_stream *s, uint64_t engine, uint64_t seed, const uint32_t *key, size_t n_key)
{
    /* the SIMD engines are assembled from their seeded scalar engine by the
     * Python layer (their sub-streams need jump polynomials) */
    if (engine >= OR_NENGINE || engine >= OR_X256PPS) return -1;
    uint32_t in[64 + 4];
    if (n_key > 64) return -1;
    size_t n_in = 0;
    in[n_in++] = (uint32_t)seed;
    in[n_in++] = (uint32_t)(seed >> 32);
    if (n_key > 0) {
        while (n_in < 4) in[n_in++] = 0;
        for (size_t i = 0; i < n_key; i++) in[n_in++] = key[i];
    }
    int nw = seeded_words(engine);
    uint32_t o[18];
    or_seed_seq(in, n_in, o, (size_t)(2 * nw));
    uint64_t w[9];
    for (int i = 0; i < nw; i++) w[i] = (uint64_t)o[2 * i] | ((uint64_t)o[2 * i + 1] << 32);
    memset(s, 0, sizeof *s);
    s->engine = engine;
    switch (engine) {
    case OR_X256PP:
    case OR_X256SS:
        memcpy(s->st, w, 4 * 8);
        if (!(w[0] | w[1] | w[2] | w[3])) s->st[0] = 1;
        break;
    case OR_PCG64:
        memcpy(s->st, w, 4 * 8);
        s->st[2] |= 1u;
        break;
    case OR_PHILOX4X32:
    case OR_PHILOX4X64:
    case OR_CHACHA20:
        memcpy(s->st, w, (size_t)nw * 8);
        break;
    case OR_SFC64:
        or_sfc64_set_abc(s, w[0], w[1], w[2]);
        break;
    case OR_XORO128PP:
    case OR_XS128P:
        memcpy(s->st, w, 2 * 8);
        if (!(w[0] | w[1])) s->st[0] = 1; /* the excluded all-zero state */
        break;
    case OR_SQUARES:
        /* reading: the key is made odd (the key 0 would give a constant
         * stream); the counter is the first mixer word */
        s->st[0] = w[0];
        s->st[1] = w[1] | 1u;
        break;
    case OR_RANLUX:
        memcpy(s->st, w, 9 * 8);
        rl_seed_fixup(s->st);
        break;
    case OR_CWG128:
        /* x, a and the Weyl sequence from the mixer; the increment goes
         * through the stream setter (made odd, 96 warm-up steps), as sfc64's
         * (a, b, c) go through its setter */
        memcpy(s->st, w, 6 * 8);
        or_cwg128_set_weyl(s, w[6], w[7]);
        break;
    }
    return 0;
}

/* Exact state assignment (Section 2.3, set_state). */
int or_set_state(or_stream *s, uint64_t engine, const uint64_t *st, size_t n, uint64_t phase)
{
    if (engine >= OR_NENGINE || n > 32) return -1;
    memset(s, 0, sizeof *s);
    s->engine = engine;
    memcpy(s->st, st, n * 8);
    s->phase = phase;
    return 0;
}

/* ---- stream setters (Table 3) ------------------------------------------ */
int or_pcg64_set_inc(or_stream *s, uint64_t lo, uint64_t hi)
{
    if (s->engine != OR_PCG64) return -1;
    s->st[2] = lo | 1u;   /* the increment must be odd */
    s->st[3] = hi;
    return 0;
}

int or_philox_set_key(or_stream *s, uint64_t k0, uint64_t k1)
{
    if (s->engine == OR_PHILOX4X32) {
        s->st[2] = k0;    /* 2 x 32-bit key words packed, k0 low */
    } else if (s->engine == OR_PHILOX4X64) {
        s->st[4] = k0;
        s->st[5] = k1;
    } else {
        return -1;
    }
    s->blk_ok = 0;
    return 0;
}

/* squares stream setter (Table 3): the key, made odd as in seeding. */
int or_squares_set_key(or_stream *s, uint64_t key)
{
    if (s->engine != OR_SQUARES) return -1;
    s->st[1] = key | 1u;
    return 0;
}

/* chacha20 stream setter (Table 3): the 96-bit nonce; key and counter kept. */
int or_chacha20_set_nonce(or_stream *s, uint64_t lo, uint64_t hi)
{
    if (s->engine != OR_CHACHA20) return -1;
    s->st[4] = lo;
    s->st[5] = (s->st[5] & 0xffffffff00000000ull) | (uint32_t)hi;
    s->blk_ok = 0;
    return 0;
}

/* cwg128 stream setter (Table 3): the Weyl increment, made odd (an even one
 * would not give the full period of the Weyl sequence), then the 96 warm-up
 * steps of the Table 3 caption; x, a and the Weyl sequence are kept. */
int or_cwg128_set_weyl(or_stream *s, uint64_t lo, uint64_t hi)
{
    if (s->engine != OR_CWG128) return -1;
    s->st[6] = lo | 1u;
    s->st[7] = hi;
    s->phase = 0;
    for (int i = 0; i < 96; i++) (void)cwg128_word(s->st);
    return 0;
}

/* sfc64 stream setter: (a, b, c) chosen, counter = 1, 18 warm-up steps. */
void or_sfc64_set_abc(or_stream *s, uint64_t a, uint64_t b, uint64_t c)
{
    s->engine = OR_SFC64;
    s->phase = 0;
    s->st[0] = a;
    s->st[1] = b;
    s->st[2] = c;
    s->st[3] = 1;
    for (int i = 0; i < 18; i++) (void)sfc64_word(s->st);
}

/* ---- jumps and advances (Section 2.3, Section 4.4 "Jumping") ------------ */

/* xor family: apply p(T) for a jump polynomial p of degree < 256 given by
 * its coefficient bits (bit k of poly = coefficient of x^k):
 *   s' = sum_k p_k T^k s. */
int or_x256_apply_poly(or_stream *s, const uint64_t poly[4])
{
    if (s->engine != OR_X256PP && s->engine != OR_X256SS) return -1;
    uint64_t acc[4] = {0, 0, 0, 0}, cur[4];
    memcpy(cur, s->st, sizeof cur);
    for (int k = 0; k < 256; k++) {
        if ((poly[k / 64] >> (k % 64)) & 1) {
            for (int i = 0; i < 4; i++) acc[i] ^= cur[i];
        }
        x256_linear(cur);
    }
    memcpy(s->st, acc, sizeof acc);
    return 0;
}

/* 128-bit xor engines: s' = sum_k p_k T^k s for a polynomial of degree < 128 */
int or_x128_apply_poly(or_stream *s, const uint64_t poly[2])
{
    if (s->engine != OR_XORO128PP && s->engine != OR_XS128P) return -1;
    uint64_t acc[2] = {0, 0}, cur[2] = {s->st[0], s->st[1]};
    for (int k = 0; k < 128; k++) {
        if ((poly[k / 64] >> (k % 64)) & 1) {
            acc[0] ^= cur[0];
            acc[1] ^= cur[1];
        }
        if (s->engine == OR_XORO128PP) xoro128_linear(cur);
        else xs128_linear(cur);
    }
    s->st[0] = acc[0];
    s->st[1] = acc[1];
    return 0;
}

/* one step of the linear core, for computing the characteristic polynomial */
void or_x256_linear_steps(uint64_t st[4], uint64_t *bit0_out, size_t n)
{
    for (size_t i = 0; i < n; i++) {
        bit0_out[i] = st[0] & 1u;
        x256_linear(st);
    }
}

/* pcg64: advance by delta steps (delta = lo + hi 2^64) by binary powering of
 * the affine map s -> M s + c (mod 2^128). */
int or_pcg64_advance(or_stream *s, uint64_t dlo, uint64_t dhi)
{
    if (s->engine != OR_PCG64) return -1;
    u128 delta = ((u128)dhi << 64) | dlo;
    u128 cur_mult = OR_PCG_MULT, cur_plus = ((u128)s->st[3] << 64) | s->st[2];
    u128 acc_mult = 1, acc_plus = 0;
    while (delta > 0) {
        if (delta & 1) {
            acc_mult *= cur_mult;
            acc_plus = acc_plus * cur_mult + cur_plus;
        }
        cur_plus = (cur_mult + 1) * cur_plus;
        cur_mult *= cur_mult;
        delta >>= 1;
    }
    u128 st = ((u128)s->st[1] << 64) | s->st[0];
    st = acc_mult * st + acc_plus;
    s->st[0] = (uint64_t)st;
    s->st[1] = (uint64_t)(st >> 64);
    return 0;
}

/* philox: advance the block counter by delta blocks; delta is given as four
 * 64-bit limbs (the 4x64 counter is 256 bits, the 4x32 counter 128 bits,
 * both wrapping). */
int or_philox_advance(or_stream *s, const uint64_t d[4])
{
    if (s->engine == OR_PHILOX4X32) {
        u128 c = ((u128)s->st[1] << 64) | s->st[0];
        c += ((u128)d[1] << 64) | d[0];
        s->st[0] = (uint64_t)c;
        s->st[1] = (uint64_t)(c >> 64);
    } else if (s->engine == OR_PHILOX4X64) {
        mp_add(&s->st[0], &s->st[0], d, 4);
    } else {
        return -1;
    }
    s->blk_ok = 0;
    return 0;
}

/* ranlux++: jump by N engine steps, N given as four 64-bit limbs:
 * x <- A^N x mod m. */
int or_ranlux_advance(or_stream *s, const uint64_t e[4])
{
    if (s->engine != OR_RANLUX) return -1;
    uint64_t An[RL_N];
    rl_powmod(An, rl_step_multiplier(), e, 4);
    rl_mulmod(s->st, s->st, An);
    s->blk_ok = 0;
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Uniform conversions (Section 3.1, "Uniform distribution").               */
/* ------------------------------------------------------------------------ */
/* method 1: 53-bit, x = floor(u / 2^11) 2^-53 (the full-mantissa option)   */
static inline double u01_53(uint64_t w) { return (double)(w >> 11) * 0x1.0p-53; }

/* method 2: 52-bit, fraction field from u / 2^12 with exponent of 1, minus 1 */
static inline double u01_52(uint64_t w)
{
    uint64_t bits = (w >> 12) | 0x3ff0000000000000ULL;
    double x;
    memcpy(&x, &bits, 8);
    return x - 1.0;
}

/* float analogues on 32-bit words: 24-bit and 23-bit */
static inline float u01f_24(uint32_t u) { return (float)(u >> 8) * 0x1.0p-24f; }
static inline float u01f_23(uint32_t u)
{
    uint32_t bits = (u >> 9) | 0x3f800000u;
    float x;
    memcpy(&x, &bits, 4);
    return x - 1.0f;
}

/* 32-bit consumption of the word stream (Section 4.3): the low half of each
 * 64-bit word first, then its high half.  A high half left over at the end
 * of a call is discarded. */
typedef struct {
    or_stream *s;
    int have;
    uint32_t hi;
} half_reader;

static uint32_t next32(half_reader *h)
{
    if (h->have) {
        h->have = 0;
        return h->hi;
    }
    uint64_t w = next_word(h->s);
    h->hi = (uint32_t)(w >> 32);
    h->have = 1;
    return (uint32_t)w;
}

void or_u01(or_stream *s, double *out, size_t n, int full_mantissa)
{
    for (size_t i = 0; i < n; i++) {
        uint64_t w = next_word(s);
        out[i] = full_mantissa ? u01_53(w) : u01_52(w);
    }
}

void or_u01f(or_stream *s, float *out, size_t n, int full_mantissa)
{
    half_reader h = {s, 0, 0};
    for (size_t i = 0; i < n; i++) {
        uint32_t u = next32(&h);
        out[i] = full_mantissa ? u01f_24(u) : u01f_23(u);
    }
}

void or_raw32(or_stream *s, uint32_t *out, size_t n)
{
    half_reader h = {s, 0, 0};
    for (size_t i = 0; i < n; i++) out[i] = next32(&h);
}

/* ------------------------------------------------------------------------ */
/* Bounded integers: Lemire's 2019 nearly-divisionless rejection method      */
/* (Section 3.2).  b = 0 means the full range (Table 5).                     */
/* ------------------------------------------------------------------------ */
void or_bounded64(or_stream *s, uint64_t b, uint64_t *out, size_t n)
{
    for (size_t i = 0; i < n; i++) {
        uint64_t w = next_word(s);
        if (b == 0) {
            out[i] = w;
            continue;
        }
        u128 p = (u128)w * b;
        uint64_t low = (uint64_t)p;
        if (low < b) {
            uint64_t threshold = (0 - b) % b; /* (2^64 - b) mod b */
            while (low < threshold) {
                w = next_word(s);
                p = (u128)w * b;
                low = (uint64_t)p;
            }
        }
        out[i] = (uint64_t)(p >> 64);
    }
}

void or_bounded32(or_stream *s, uint32_t b, uint32_t *out, size_t n)
{
    half_reader h = {s, 0, 0};
    for (size_t i = 0; i < n; i++) {
        uint32_t u = next32(&h);
        if (b == 0) {
            out[i] = u;
            continue;
        }
        uint64_t p = (uint64_t)u * b;
        uint32_t low = (uint32_t)p;
        if (low < b) {
            uint32_t threshold = (0u - b) % b;
            while (low < threshold) {
                u = next32(&h);
                p = (uint64_t)u * b;
                low = (uint32_t)p;
            }
        }
        out[i] = (uint32_t)(p >> 32);
    }
}

/* ------------------------------------------------------------------------ */
/* Permutations and sampling (Section 3.2).  Every draw is a 32-bit bounded */
/* integer by Lemire's method on the 32-bit item stream (low half first),   */
/* one item reader per call.                                                 */
/* ------------------------------------------------------------------------ */
static uint32_t bounded_item(half_reader *h, uint32_t b)
{
    uint32_t u = next32(h);
    uint64_t p = (uint64_t)u * b;
    uint32_t low = (uint32_t)p;
    if (low < b) {
        uint32_t threshold = (0u - b) % b;
        while (low < threshold) {
            u = next32(h);
            p = (uint64_t)u * b;
            low = (uint32_t)p;
        }
    }
    return (uint32_t)(p >> 32);
}

/* Fisher-Yates (Durstenfeld's form): start from the identity; for j from  */
/* n-1 down to 1 swap entry j with entry r, r uniform on {0..j}.            */
void or_permutation(or_stream *s, uint32_t n, uint32_t *out)
{
    half_reader h = {s, 0, 0};
    for (uint32_t i = 0; i < n; i++) out[i] = i;
    for (uint32_t j = n; j-- > 1;) {
        uint32_t r = bounded_item(&h, j + 1);
        uint32_t t = out[j];
        out[j] = out[r];
        out[r] = t;
    }
}

/* k distinct elements of {0..n-1}.  k <= n/2: Floyd's algorithm -- for j   */
/* from n-k to n-1 draw t uniform on {0..j}; append t if it is not yet in   */
/* the sample, else append j (the sample in the order of insertion).        */
/* k > n/2: reservoir sampling (Vitter's algorithm R) -- start from         */
/* 0..k-1; for i from k to n-1 draw j uniform on {0..i} and replace entry j */
/* by i when j < k.  The membership test is a plain scan.                   */
void or_sample(or_stream *s, uint32_t n, uint32_t k, uint32_t *out)
{
    half_reader h = {s, 0, 0};
    if (2 * (uint64_t)k <= n) {
        for (uint32_t c = 0; c < k; c++) {
            uint32_t j = n - k + c;
            uint32_t t = bounded_item(&h, j + 1);
            int seen = 0;
            for (uint32_t q = 0; q < c; q++) seen |= out[q] == t;
            out[c] = seen ? j : t;
        }
    } else {
        for (uint32_t i = 0; i < k; i++) out[i] = i;
        for (uint32_t i = k; i < n; i++) {
            uint32_t j = bounded_item(&h, i + 1);
            if (j < k) out[j] = i;
        }
    }
}

/* ------------------------------------------------------------------------ */
/* The bitexact setting (Section 4.2: library function calls made the same  */
/* on every platform).  Reading taken here: with the setting on, every exp, */
/* log and log1p of a sampler is the correctly rounded binary64 value,      */
/* taken as the binary128 value of libquadmath (about 2^-112 relative)      */
/* rounded once to binary64; pow and the gamma boost the same way.  Off,    */
/* they are the C library's.  The setting is global to the oracle (test     */
/* infrastructure, one caller at a time): or_set_bitexact.                  */
/* ------------------------------------------------------------------------ */
static int or_bx = 0;

void or_set_bitexact(int on) { or_bx = on != 0; }
int or_get_bitexact(void) { return or_bx; }

static double q_exp(double x) { return (double)expq((__float128)x); }
static double q_log(double x) { return (double)logq((__float128)x); }
static double q_log1p(double x) { return (double)log1pq((__float128)x); }
static double q_pow(double x, double y) { return (double)powq((__float128)x, (__float128)y); }
/* u^(1/a) with the quotient log(u)/a in binary128 (1/a not rounded) */
static double q_powinv(double u, double a)
{
    if (u != u || a != a) return u + a;
    if (u < 0.0 || a <= 0.0) return NAN;
    if (u == 0.0 || u == 1.0 || a == 1.0 || isinf(u)) return u;
    if (isinf(a)) return 1.0;
    return (double)expq(logq((__float128)u) / (__float128)a);
}

static double OR_EXP(double x) { return or_bx ? q_exp(x) : exp(x); }
static double OR_LOG(double x) { return or_bx ? q_log(x) : log(x); }
static double OR_LOG1P(double x) { return or_bx ? q_log1p(x) : log1p(x); }

/* out[i] = f(x[i], y[i]) for f = 0 exp, 1 log, 2 log1p, 3 pow, 4 u^(1/a), */
/* each the binary128 value rounded once to binary64 (y read for 3 and 4)   */
void or_crmath(int fn, const double *x, const double *y, double *out, size_t n)
{
    for (size_t i = 0; i < n; i++) {
        switch (fn) {
        case 0: out[i] = q_exp(x[i]); break;
        case 1: out[i] = q_log(x[i]); break;
        case 2: out[i] = q_log1p(x[i]); break;
        case 3: out[i] = q_pow(x[i], y[i]); break;
        default: out[i] = q_powinv(x[i], y[i]); break;
        }
    }
}

/* ------------------------------------------------------------------------ */
/* Ziggurat normal and exponential (Section 3.1 and the ziggurat figure).   */
/* Strip j = low byte of a 64-bit word.  Normal: bit 8 = sign, bits 9..60 =  */
/* 52-bit magnitude m.  Exponential: bits 8..60 = 53-bit magnitude m.  The   */
/* top three bits are unused.  Candidate x = m w_j; fast accept if m < k_j.  */
/* Otherwise, strip 0 samples the tail and strips j >= 1 run the wedge test  */
/*   y = f_j + U (f_{j-1} - f_j),  accept iff y < f(x),                      */
/* drawing a fresh word on rejection.  This is the plain test that always    */
/* evaluates f; the paper's secant/tangent squeeze only skips exp() calls    */
/* and cannot change which candidates are accepted.                          */
/* Tail readings (the paper names Marsaglia's 1964 method but prints no      */
/* formula): normal  e1 = -log1p(-U1)/r, e2 = -log1p(-U2), accept when       */
/* e2 + e2 > e1 e1, return +-(r + e1) with the sign from bit 8;              */
/* exponential  r - log1p(-U) (memorylessness).  U are 53-bit uniforms.      */
/* ------------------------------------------------------------------------ */
static double norm_one(or_stream *s, or_counts *c)
{
    for (;;) {
        uint64_t w = nx(s, c);
        if (c) c->candidates++;
        int j = (int)(w & 0xff);
        int neg = (int)((w >> 8) & 1);
        uint64_t m = (w >> 9) & ((1ULL << 52) - 1);
        double x = (double)m * OR_NORM_W[j];
        if (m < OR_NORM_K[j]) return neg ? -x : x;
        if (j == 0) {
            if (c) c->tail_entries++;
            for (;;) {
                double e1 = -OR_LOG1P(-u01_53(nx(s, c))) / OR_NORM_R;
                double e2 = -OR_LOG1P(-u01_53(nx(s, c)));
                if (c) c->tail_logs += 2;
                if (e2 + e2 > e1 * e1) {
                    double t = OR_NORM_R + e1;
                    return neg ? -t : t;
                }
            }
        }
        double y = OR_NORM_F[j] + u01_53(nx(s, c)) * (OR_NORM_F[j - 1] - OR_NORM_F[j]);
        if (c) c->pdf_evals++;
        if (y < OR_EXP(-0.5 * x * x)) return neg ? -x : x;
        if (c) c->rejections++;
    }
}

static double exp_one(or_stream *s, or_counts *c)
{
    for (;;) {
        uint64_t w = nx(s, c);
        if (c) c->candidates++;
        int j = (int)(w & 0xff);
        uint64_t m = (w >> 8) & ((1ULL << 53) - 1);
        double x = (double)m * OR_EXP_W[j];
        if (m < OR_EXP_K[j]) return x;
        if (j == 0) {
            if (c) {
                c->tail_entries++;
                c->tail_logs++;
            }
            return OR_EXP_R - OR_LOG1P(-u01_53(nx(s, c)));
        }
        double y = OR_EXP_F[j] + u01_53(nx(s, c)) * (OR_EXP_F[j - 1] - OR_EXP_F[j]);
        if (c) c->pdf_evals++;
        if (y < OR_EXP(-x)) return x;
        if (c) c->rejections++;
    }
}

/* ------------------------------------------------------------------------ */
/* Float ziggurat (the paper's float versions: a binary32 function for each  */
/* continuous law; it states only that the float case is analogous to the   */
/* double one).  Reading taken here: a float draw consumes 32-bit items of    */
/* the word stream (low half first, as every 32-bit consumer).  Strip j =     */
/* low byte; normal: bit 8 = sign, bits 9..31 = 23-bit magnitude m;           */
/* exponential: bits 8..31 = 24-bit magnitude m.  The candidate and every     */
/* test are those of the double ziggurat for the magnitude m 2^29 (the same  */
/* geometry and tables), in binary64; wedge and tail uniforms are 24-bit     */
/* float uniforms of the following items.  The returned value is the        */
/* binary64 result rounded once to binary32.                                  */
/* ------------------------------------------------------------------------ */
static double u01_24(uint32_t u) { return (double)(u >> 8) * 0x1.0p-24; }

static float normf_one(half_reader *h)
{
    for (;;) {
        uint32_t u = next32(h);
        int j = (int)(u & 0xff);
        int neg = (int)((u >> 8) & 1);
        uint64_t m = (uint64_t)(u >> 9) << 29;
        double x = (double)m * OR_NORM_W[j];
        if (m < OR_NORM_K[j]) return (float)(neg ? -x : x);
        if (j == 0) {
            for (;;) {
                double e1 = -OR_LOG1P(-u01_24(next32(h))) / OR_NORM_R;
                double e2 = -OR_LOG1P(-u01_24(next32(h)));
                if (e2 + e2 > e1 * e1) {
                    double t = OR_NORM_R + e1;
                    return (float)(neg ? -t : t);
                }
            }
        }
        double y = OR_NORM_F[j] + u01_24(next32(h)) * (OR_NORM_F[j - 1] - OR_NORM_F[j]);
        if (y < OR_EXP(-0.5 * x * x)) return (float)(neg ? -x : x);
    }
}

static float expf_one(half_reader *h)
{
    for (;;) {
        uint32_t u = next32(h);
        int j = (int)(u & 0xff);
        uint64_t m = (uint64_t)(u >> 8) << 29;
        double x = (double)m * OR_EXP_W[j];
        if (m < OR_EXP_K[j]) return (float)x;
        if (j == 0) return (float)(OR_EXP_R - OR_LOG1P(-u01_24(next32(h))));
        double y = OR_EXP_F[j] + u01_24(next32(h)) * (OR_EXP_F[j - 1] - OR_EXP_F[j]);
        if (y < OR_EXP(-x)) return (float)x;
    }
}

void or_normf(or_stream *s, float *out, size_t n)
{
    half_reader h = {s, 0, 0};
    for (size_t i = 0; i < n; i++) out[i] = normf_one(&h);
}

void or_expf(or_stream *s, float *out, size_t n)
{
    half_reader h = {s, 0, 0};
    for (size_t i = 0; i < n; i++) out[i] = expf_one(&h);
}

void or_norm(or_stream *s, double *out, size_t n, or_counts *c)
{
    for (size_t i = 0; i < n; i++) out[i] = norm_one(s, c);
}

void or_exp(or_stream *s, double *out, size_t n, or_counts *c)
{
    for (size_t i = 0; i < n; i++) out[i] = exp_one(s, c);
}

/* Fused generate-and-reduce: per-stream sum and sum of squares of n
 * standard normals, accumulated in draw order in binary64. */
void or_norm_moments(or_stream *s, size_t n, double *sum, double *sumsq)
{
    double a = 0.0, q = 0.0;
    for (size_t i = 0; i < n; i++) {
        double x = norm_one(s, NULL);
        a = a + x;
        q = q + x * x;
    }
    *sum = a;
    *sumsq = q;
}

/* ------------------------------------------------------------------------ */
/* Gamma: Marsaglia and Tsang (2000), Section 3.1 "Gamma and related        */
/* distributions".  For shape a >= 1:                                        */
/*   d = a - 1/3, c = 1/sqrt(9 d); repeat: draw normals x until             */
/*   v = 1 + c x > 0; v = v^3; draw U; accept d v if                         */
/*   U < 1 - 0.0331 x^4, or if log U < x^2/2 + d (1 - v + log v).            */
/* Shape a < 1 uses the boost Gamma(a) = Gamma(a + 1) U^(1/a), the gamma     */
/* draw first, then U.  The power U^(1/a) is taken correctly rounded: it is  */
/* formed in binary128 (libquadmath), so the only rounding that matters is   */
/* the final one to binary64.                                                */
/* ------------------------------------------------------------------------ */
static double mt_gamma(or_stream *s, double a, or_counts *cn)
{
    double d = a - 1.0 / 3.0;
    double c = 1.0 / sqrt(9.0 * d);
    for (;;) {
        double x, v;
        do {
            x = norm_one(s, NULL);
            v = 1.0 + c * x;
        } while (v <= 0.0);
        v = v * v * v;
        double u = u01_53(next_word(s));
        double x2 = x * x;
        if (cn) cn->mt_attempts++;
        if (u < 1.0 - 0.0331 * (x2 * x2)) return d * v;
        if (cn) cn->mt_logtests++;
        if (OR_LOG(u) < 0.5 * x2 + d * ((1.0 - v) + OR_LOG(v))) return d * v;
    }
}

double or_boost_pow(double u, double a)
{
    __float128 t = logq((__float128)u) / (__float128)a;
    return (double)expq(t);
}

static double gamma_one(or_stream *s, double a, or_counts *cn)
{
    if (a < 1.0) {
        double g = mt_gamma(s, a + 1.0, cn);
        double u = u01_53(next_word(s));
        return g * or_boost_pow(u, a);
    }
    return mt_gamma(s, a, cn);
}

/* Float gamma (the paper's gammaf; reading as for the float ziggurat):
 * Marsaglia-Tsang with the binary32 normal of the float ziggurat, the
 * 24-bit uniform of the next 32-bit item for the test and for the shape < 1
 * boost, binary64 arithmetic throughout, theta g rounded once to binary32. */
static double mt_gammaf(half_reader *h, double a)
{
    double d = a - 1.0 / 3.0;
    double c = 1.0 / sqrt(9.0 * d);
    for (;;) {
        double x, v;
        do {
            x = (double)normf_one(h);
            v = 1.0 + c * x;
        } while (v <= 0.0);
        v = v * v * v;
        double u = u01_24(next32(h));
        double x2 = x * x;
        if (u < 1.0 - 0.0331 * (x2 * x2)) return d * v;
        if (OR_LOG(u) < 0.5 * x2 + d * ((1.0 - v) + OR_LOG(v))) return d * v;
    }
}

/* The float gamma draw in binary64 (shape < 1: Gamma(a + 1), then the
 * U^(1/a) boost on the next item's 24-bit uniform). */
static double gammaf_draw(half_reader *h, double a)
{
    if (a < 1.0) {
        double g = mt_gammaf(h, a + 1.0);
        return g * or_boost_pow(u01_24(next32(h)), a);
    }
    return mt_gammaf(h, a);
}

void or_gammaf(or_stream *s, double a, double theta, float *out, size_t n)
{
    half_reader h = {s, 0, 0};
    for (size_t i = 0; i < n; i++) out[i] = (float)(theta * gammaf_draw(&h, a));
}

/* Float versions (Section 4.4) of the laws of several draws (Table 4), law
 * numbers as rp_fill_lawf's: 10 beta(a, b), 11 chi2(nu), 12 t(nu),
 * 13 F(nu1, nu2), 14 skew-normal(mu, sigma, alpha).  The base draws are the
 * float gamma (binary64, unrounded) and the binary32 normal of the float
 * ziggurat, all on the 32-bit items of one call (a half left over at the end
 * is dropped); the combination is as for the binary64 laws, in binary64,
 * rounded once to binary32. */
void or_mixf(or_stream *s, int law, const double *p, float *out, size_t n)
{
    half_reader h = {s, 0, 0};
    for (size_t i = 0; i < n; i++) {
        double v = 0.0;
        switch (law) {
        case 10: {
            double x = gammaf_draw(&h, p[0]);
            double y = gammaf_draw(&h, p[1]);
            double t = x + y;
            v = (t == 0.0) ? p[0] / (p[0] + p[1]) : x / t;
            break;
        }
        case 11:
            v = 2.0 * gammaf_draw(&h, p[0] / 2.0);
            break;
        case 12: {
            double z = (double)normf_one(&h);
            double w = 2.0 * gammaf_draw(&h, p[0] / 2.0);
            v = z / sqrt(w / p[0]);
            break;
        }
        case 13: {
            double x = gammaf_draw(&h, p[0] / 2.0);
            double y = gammaf_draw(&h, p[1] / 2.0);
            v = (x / p[0]) / (y / p[1]);
            break;
        }
        case 14: {
            double d = p[2] / sqrt(1.0 + p[2] * p[2]);
            double c = sqrt(1.0 - d * d);
            double z0 = (double)normf_one(&h);
            double z1 = (double)normf_one(&h);
            v = p[0] + p[1] * (d * fabs(z0) + c * z1);
            break;
        }
        }
        out[i] = (float)v;
    }
}

void or_gamma(or_stream *s, double a, double *out, size_t n, or_counts *cn)
{
    for (size_t i = 0; i < n; i++) out[i] = gamma_one(s, a, cn);
}

/* Beta(a, b) = X / (X + Y), X ~ Gamma(a) drawn before Y ~ Gamma(b) on the
 * same stream (Table 4).  X + Y = 0 (both draws underflowed) returns the
 * mean a / (a + b); the paper is silent on this measure-zero case. */
static double beta_one(or_stream *s, double a, double b)
{
    double x = gamma_one(s, a, NULL);
    double y = gamma_one(s, b, NULL);
    double t = x + y;
    if (t == 0.0) return a / (a + b);
    return x / t;
}

void or_beta(or_stream *s, double a, double b, double *out, size_t n)
{
    for (size_t i = 0; i < n; i++) out[i] = beta_one(s, a, b);
}

/* Batched gamma: set j draws count[j] values from stream j into
 * out[offset_j ...], offset_j = count[0] + ... + count[j-1]. */
void or_gamma_batched(or_stream *streams, const double *alpha, const int64_t *count, size_t n_sets,
                      double *out)
{
    size_t off = 0;
    for (size_t j = 0; j < n_sets; j++) {
        for (int64_t t = 0; t < count[j]; t++) out[off + (size_t)t] = gamma_one(&streams[j], alpha[j], NULL);
        off += (size_t)count[j];
    }
}

void or_beta_batched(or_stream *streams, const double *a, const double *b, const int64_t *count,
                     size_t n_sets, double *out)
{
    size_t off = 0;
    for (size_t j = 0; j < n_sets; j++) {
        for (int64_t t = 0; t < count[j]; t++) out[off + (size_t)t] = beta_one(&streams[j], a[j], b[j]);
        off += (size_t)count[j];
    }
}

/* Per-element forms: element e draws one value from stream e; parameters
 * and results are binary32, the draw itself is computed in binary64 and
 * rounded once. */
void or_gamma_elem(or_stream *streams, const float *alpha, float *z, size_t n)
{
    for (size_t e = 0; e < n; e++) z[e] = (float)gamma_one(&streams[e], (double)alpha[e], NULL);
}

void or_beta_elem(or_stream *streams, const float *a, const float *b, float *z, size_t n)
{
    for (size_t e = 0; e < n; e++) z[e] = (float)beta_one(&streams[e], (double)a[e], (double)b[e]);
}

/* Multivariate normal rows: row j takes the first d normals of stream j,
 * each rounded to binary32 (Z is n x d, row-major). */
void or_mvn_z(or_stream *streams, int d, size_t n, float *z)
{
    for (size_t j = 0; j < n; j++)
        for (int i = 0; i < d; i++) z[j * (size_t)d + (size_t)i] = (float)norm_one(&streams[j], NULL);
}

/* ---- timing harness for the CPU baseline of the benchmark ---------------
 * Not part of the method: it runs the plain routines above, unchanged, over
 * many streams at once so that the benchmark can time the oracle on all host
 * cores.  Each of `threads` POSIX threads takes a contiguous range of the n
 * streams (stored back to back) and draws `per` values from each, in place,
 * into a private buffer.  what: 0 raw 64-bit words, 1 U(0,1) binary32, 2
 * U(0,1) binary64, 3 standard normal, 4 standard exponential.  Returns the
 * wall time in seconds (CLOCK_MONOTONIC around thread start and join), or a
 * negative value if a thread could not be started or a buffer allocated. */
#include <pthread.h>
#include <stdlib.h>
#include <time.h>

typedef struct {
    or_stream *streams;
    size_t first, count, per;
    int what, failed;
} or_timing_job;

static void *or_timing_worker(void *arg)
{
    or_timing_job *j = (or_timing_job *)arg;
    void *buf = malloc(j->per * 8 + 8);
    if (!buf) {
        j->failed = 1;
        return NULL;
    }
    for (size_t i = j->first; i < j->first + j->count; i++) {
        or_stream *s = &j->streams[i];
        switch (j->what) {
        case 0: or_raw64(s, (uint64_t *)buf, j->per); break;
        case 1: or_u01f(s, (float *)buf, j->per, 1); break;
        case 2: or_u01(s, (double *)buf, j->per, 1); break;
        case 3: or_norm(s, (double *)buf, j->per, NULL); break;
        default: or_exp(s, (double *)buf, j->per, NULL); break;
        }
    }
    free(buf);
    return NULL;
}

double or_time_fills(or_stream *streams, size_t n, int what, size_t per, int threads)
{
    if (threads < 1) threads = 1;
    if ((size_t)threads > n) threads = (int)n;
    or_timing_job *jobs = (or_timing_job *)calloc((size_t)threads, sizeof *jobs);
    pthread_t *tid = (pthread_t *)calloc((size_t)threads, sizeof *tid);
    if (!jobs || !tid) {
        free(jobs);
        free(tid);
        return -1.0;
    }
    struct timespec t0, t1;
    clock_gettime(CLOCK_MONOTONIC, &t0);
    int started = 0, failed = 0;
    for (int t = 0; t < threads; t++) {
        const size_t lo = n * (size_t)t / (size_t)threads, hi = n * (size_t)(t + 1) / (size_t)threads;
        jobs[t] = (or_timing_job){streams, lo, hi - lo, per, what, 0};
        if (pthread_create(&tid[t], NULL, or_timing_worker, &jobs[t]) != 0) {
            failed = 1;
            break;
        }
        started++;
    }
    for (int t = 0; t < started; t++) {
        pthread_join(tid[t], NULL);
        failed |= jobs[t].failed;
    }
    clock_gettime(CLOCK_MONOTONIC, &t1);
    free(jobs);
    free(tid);
    if (failed) return -1.0;
    return (double)(t1.tv_sec - t0.tv_sec) + 1e-9 * (double)(t1.tv_nsec - t0.tv_nsec);
}
