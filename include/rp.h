/*
 * rp.h -- C ABI of the MI355X (gfx950) implementation of the Randompack hot
 * path: bulk generation from the paper's engines on many independent
 * substreams, fed through its distribution layer (Randompack, arXiv
 * 2605.05099).
 *
 * Conventions (Section 2.1, Section 4.4 "Thread safety"):
 *   - Every call returns int: RP_OK (0) or a negative RP_E* code.  No
 *     exception crosses the ABI.  A message describing the last failure is
 *     kept per handle (rp_last_error) and per thread (rp_errmsg) for calls
 *     without a handle.
 *   - Handles (rp_rng, rp_streams) are opaque, created and freed by the
 *     library.  One handle must not be used by two threads at once; distinct
 *     handles are independent (no global mutable state except the per-thread
 *     error slot and read-only tables).
 *   - NULL pointers where an object is required give RP_ENULL.  A count of
 *     zero is valid and does nothing.
 *   - Device pointers ("d_" prefix) point to GPU memory the caller owns;
 *     host pointers point to host memory.  Launches are asynchronous on the
 *     given HIP stream (a hipStream_t passed as void*; NULL = default
 *     stream).  Errors found before launch are reported synchronously; a
 *     launch failure is reported as RP_EDEVICE.
 *
 * Engines (Table 2; philox4x32 is the 32-bit member of the paper's Philox
 * family).  Identifiers are matched case-insensitively with no aliases
 * (Section 4.4, "Engine query").
 */
#ifndef RP_H
#define RP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------- */
enum {
    RP_OK = 0,
    RP_EINVAL = -1,       /* invalid argument value                          */
    RP_ENOMEM = -2,       /* host or device allocation failed                */
    RP_EUNSUPPORTED = -3, /* operation not defined for this engine / dtype   */
    RP_EDEVICE = -4,      /* HIP runtime or kernel launch error              */
    RP_ENOTSPD = -5,      /* matrix is not symmetric positive definite       */
    RP_ENULL = -6         /* required pointer was NULL                       */
};

/* ---- engines (Table 2) -------------------------------------------------- */
enum {
    RP_X256PP = 0,     /* "x256++"     xoshiro256++, 4 state words          */
    RP_PCG64 = 1,      /* "pcg64"      PCG64 DXSM, state 2 + increment 2    */
    RP_PHILOX4X32 = 2, /* "philox4x32" Philox4x32-10, counter 2 + key 1     */
    RP_PHILOX = 3,     /* "philox"     Philox-4x64-10, counter 4 + key 2    */
    RP_SFC64 = 4,      /* "sfc64"      sfc64, (a, b, c) + counter           */
    RP_RANLUX = 5,     /* "ranlux++"   ranlux++, 9 words (576-bit LCG)      */
    RP_X256SS = 6,     /* "x256**"     xoshiro256**, 4 state words; seeding, */
                       /*              jumps and substreams as x256++       */
    RP_SQUARES = 7,    /* "squares"    squares64, counter 1 + key 1         */
    RP_XORO128 = 8,    /* "xoro++"     xoroshiro128++, 2 state words        */
    RP_XS128 = 9,      /* "x128+"      xorshift128+, 2 state words; jumps   */
                       /*              2^k only for k < 128 (both engines)  */
    RP_CHACHA20 = 10,  /* "chacha20"   ChaCha20, key 4 + nonce 1.5 + block  */
                       /*              counter 0.5 (high half of word 5)    */
    RP_CWG128 = 11,    /* "cwg128"     Collatz-Weyl, x 2 + a 2 + Weyl 2 +   */
                       /*              odd Weyl increment 2 (128-bit words) */
    /* SIMD engines (Section 4.1): eight interleaved scalar sub-streams, 32
     * state words (sub-stream k at words 4k .. 4k+3), blocks of 8 words
     * (word 8 t + k is sub-stream k's t-th word; phase counts the words of
     * the current round already used, the sub-streams moving one step when
     * all eight are used).  xoshiro sub-stream k is the seeded base jumped by
     * k 2^253 steps; sfc64 sub-stream k has k 2^61 added to the seeded base's
     * counter.  Jumps and advances move every sub-stream (k < 253). */
    RP_X256PPS = 12,   /* "x256++simd" the paper's default engine          */
    RP_X256SSS = 13,   /* "x256**simd"                                     */
    RP_SFC64S = 14,    /* "sfc64simd"  (no jump; rp_sfc64_set_abc sets the */
                       /*              base, then the counter offsets)     */
    RP_NENGINES = 15
};

typedef struct rp_rng rp_rng;         /* one serial stream, host resident  */
typedef struct rp_streams rp_streams; /* n substreams, device resident     */

/* ---- errors and engine query -------------------------------------------- */
/* Message of the last failed call on this thread ("" if none). */
const char *rp_errmsg(void);
/* Message of the last failed call on this handle; NULL handle = rp_errmsg. */
const char *rp_last_error(const rp_rng *rng);
/* Writes "id: description" lines for all engines into buf (NUL-terminated,
 * truncated to len).  Returns the length needed (excluding NUL). */
int rp_engines(char *buf, size_t len);
/* Engine number of an identifier (case-insensitive), or RP_EINVAL. */
int rp_engine_id(const char *name);

/* ---- serial streams (Section 2.1, Section 2.3) -------------------------- */
/* Creates a stream; NULL or "" selects x256++.  The new stream is
 * randomized (rp_randomize); call rp_seed for a reproducible one.  Returns
 * NULL on failure (see rp_errmsg). */
rp_rng *rp_create(const char *engine);
/* Seeds the stream from system entropy (Section 2.3): a 64-bit seed from
 * getrandom (then /dev/urandom; if neither answers, the clock mixed with a
 * counter), used as rp_seed(rng, seed, NULL, 0) would, so spawn-key
 * substreams derive from it as from any seed.  Not reproducible. */
int rp_randomize(rp_rng *rng);
void rp_free(rp_rng *rng);
/* Exact copy (Section 2.3 "duplicate"). */
rp_rng *rp_duplicate(const rp_rng *rng);
/* Deterministic seeding (Section 2.3): the seed (two 32-bit words, low
 * first), zero-padded to four words when a spawn key follows, then the
 * spawn-key words, go through the seed_seq_fe128 mixer, which is asked for
 * two 32-bit words per 64-bit state word.  n_key = 0 means no key. */
int rp_seed(rp_rng *rng, uint64_t seed, const uint32_t *spawn_key, size_t n_key);
/* Number of 64-bit state words of the engine (Table 2 "State words"). */
int rp_state_words(const rp_rng *rng);
/* Exact state get/set (Section 2.3 "set_state").  words has
 * rp_state_words() entries in Table 3 order; phase is the number of 64-bit
 * words already used from the current output block (always 0 except for
 * philox4x32 (< 2), philox (< 4) and ranlux++ (< 9)).  rp_set_state (and
 * rp_deserialize, rp_streams_set, rp_streams_deserialize) reject with
 * RP_EINVAL the states that seeding never produces because they are not
 * proper states of the engine: the all-zero state of xoshiro256,
 * xoroshiro128++ and xorshift128+ (a fixed point), an even PCG64 increment,
 * an even squares64 key, an even cwg128 Weyl increment, and a ranlux++
 * value outside [1, m). */
int rp_get_state(const rp_rng *rng, uint64_t *words, size_t n, uint32_t *phase);
int rp_set_state(rp_rng *rng, const uint64_t *words, size_t n, uint32_t phase);
/* Jump by 2^k engine steps, k in {32, 64, 96, 128, 192} (Section 2.3).
 * RP_EINVAL when 2^k is not below the period of one stream (squares64:
 * k >= 64; ChaCha20: every k, its block counter has 32 bits; pcg64,
 * philox4x32, xoroshiro128++, xorshift128+: k >= 128); RP_EUNSUPPORTED for
 * sfc64, which has no jump. */
int rp_jump(rp_rng *rng, int k);
/* Advance by n = lo + hi 2^64 engine steps (a block for block engines):
 * PCG64 affine powering, Philox and squares64 counter addition (squares64:
 * modulo its period 2^64), xoshiro jump polynomial x^n mod P(x) (Section
 * 4.4 "Jumping"), ranlux++ A^n mod m.  sfc64 has no jump: RP_EUNSUPPORTED.
 * rp_jump rejects 2^k at or beyond the engine's period (RP_EINVAL). */
int rp_advance(rp_rng *rng, uint64_t lo, uint64_t hi);
/* Stream setters (Table 3). */
int rp_pcg64_set_inc(rp_rng *rng, uint64_t lo, uint64_t hi);       /* inc |= 1 */
int rp_philox_set_key(rp_rng *rng, uint64_t k0, uint64_t k1);      /* 4x32: key = k0 */
int rp_sfc64_set_abc(rp_rng *rng, uint64_t a, uint64_t b, uint64_t c); /* +18 steps */
int rp_squares_set_key(rp_rng *rng, uint64_t key);                  /* key |= 1 */
int rp_chacha20_set_nonce(rp_rng *rng, uint64_t lo, uint64_t hi);   /* 96-bit nonce */
/* cwg128 (Table 3): the Weyl increment s = lo + hi 2^64 made odd; x, a and
 * the Weyl sequence are kept; then 96 warm-up steps (the setter's mixing
 * warm-up, Table 3 caption).  The engine itself (Table 2, Dziala's
 * Collatz-Weyl generator on 128-bit words) is, per step,
 *   a += x;  weyl += s;  x = (x >> 1) * (a | 1) ^ weyl;
 * and the 64-bit word is the low half of (a >> 96) ^ x.  The paper does not
 * spell the step out; this reading is marked unpinned in the oracle. */
int rp_cwg128_set_weyl(rp_rng *rng, uint64_t lo, uint64_t hi);      /* inc |= 1, +96 steps */
/* Checkpointing (Section 4.4): opaque byte image of the stream.  With
 * buf == NULL only *needed is set. */
int rp_serialize(const rp_rng *rng, void *buf, size_t len, size_t *needed);
int rp_deserialize(rp_rng *rng, const void *buf, size_t len);
/* Host reference draw of raw 64-bit words (used for state checks). */
int rp_raw_host(rp_rng *rng, uint64_t *out, size_t n);

/* ---- device substreams (Section 2.3: duplicate, then set stream or jump) - */
enum {
    RP_SUB_KEY = 0,   /* philox*: substream i has key i (k1 = 0)             */
    RP_SUB_INC = 1,   /* pcg64: substream i has increment 2 i + 1; cwg128:   */
                      /*   Weyl increment 2 i + 1 through its setter        */
    RP_SUB_SPAWN = 2, /* any engine: seeded with (seed, spawn key [i])       */
    RP_SUB_JUMP = 3   /* every engine but sfc64: base advanced by           */
                      /*   i * 2^jump_log2 engine steps                      */
};
/* Builds n substreams from `base` (its seed is remembered by rp_seed) and
 * copies them to device memory owned by the returned handle.  The state
 * layout in device memory is structure-of-arrays: state word k of substream
 * i at words[k * n + i], phase[i] separately.  RP_SUB_JUMP takes jump_log2
 * from 0 up to (not including) the bound rp_jump applies: 256 for x256++,
 * x256**, philox and ranlux++, 128 for pcg64, philox4x32, xoro++ and x128+,
 * 64 for squares and 32 for chacha20 (RP_EINVAL otherwise; RP_EUNSUPPORTED
 * for sfc64); the family must also fit in one period, n * 2^jump_log2 <=
 * the period (2^bound steps, blocks for the block engines, or 2^bound - 1
 * for the xor engines; RP_EINVAL otherwise), so the substreams never overlap. */
int rp_streams_create(const rp_rng *base, int kind, uint64_t n, int jump_log2, rp_streams **out);
void rp_streams_free(rp_streams *s);
uint64_t rp_streams_count(const rp_streams *s);
int rp_streams_engine(const rp_streams *s);
/* Copies substream states to / from host memory: words is
 * state_words * n (SoA as above), phase is n entries. */
int rp_streams_get(const rp_streams *s, uint64_t *words, uint32_t *phase);
int rp_streams_set(rp_streams *s, const uint64_t *words, const uint32_t *phase);
/* New handle holding a device copy of the current states. */
int rp_streams_duplicate(const rp_streams *s, rp_streams **out);
/* Checkpointing of a substream set (Section 4.4, serialization, for the
 * device-resident states): an opaque byte image of the engine, the
 * full-mantissa setting and every substream's state and phase, host memory
 * of *needed bytes (24 + 8 state_words n + 4 n).  With buf == NULL only
 * *needed is set; len below it is RP_EINVAL.  Waits for the device.
 * rp_streams_deserialize builds a new set on the current device from such
 * an image; fills from it continue exactly where the serialized set stood.
 * Errors: RP_ENULL, RP_EINVAL for an image that is not one (magic, engine,
 * word count, setting, n, phases, length), RP_EDEVICE. */
int rp_streams_serialize(const rp_streams *s, void *buf, size_t len, size_t *needed);
int rp_streams_deserialize(const void *buf, size_t len, rp_streams **out);

/* ---- bulk fills (Tables 4 and 5, Section 3) ------------------------------ */
enum {
    RP_RAW = 0,     /* raw bits: U64 words, or U32 halves (low half first)   */
    RP_U01 = 1,     /* uniform [0,1): F64 from the top 53 bits (or 52, flag),*/
                    /*   F32 from the top 24 bits of a 32-bit half (or 23)   */
    RP_BOUNDED = 2, /* {0..b-1} by Lemire's method, U64 or U32; b = 0: full  */
    RP_NORM = 3,    /* standard normal, ziggurat, F64 (or F32, see below)    */
    RP_EXP = 4      /* standard exponential, ziggurat, F64 (or F32)          */
};
enum { RP_U64 = 0, RP_U32 = 1, RP_F64 = 2, RP_F32 = 3 };
enum { RP_FLAG_52BIT = 1 }; /* uniform method 2 (mantissa fill, 52/23 bits) */

/* Full-mantissa setting of a stream (Section 3.1, uniform distribution: the
 * switch between the two conversions).  on = 1 (the default of a new
 * stream) keeps method 1, x = (u >> 11) 2^-53 (binary32: 24 bits of a
 * 32-bit half); on = 0 selects method 2 for every U(0,1) fill from this
 * stream (rp_fill_serial) and from substream sets created from it
 * afterwards (rp_streams_create copies the setting; a set keeps it for
 * life), exactly as if RP_FLAG_52BIT were passed.  RP_FLAG_52BIT in a call
 * still selects method 2 when the setting is on.  Only RP_U01 fills read
 * it: the laws, samplers and ziggurat keep their own uniforms.  The setting
 * is copied by rp_duplicate, is not part of rp_serialize's state, and
 * survives rp_seed / rp_randomize.  Errors: RP_ENULL, RP_EINVAL for on not
 * 0 or 1.  rp_get_full_mantissa returns 1 or 0 (or RP_ENULL). */
int rp_set_full_mantissa(rp_rng *rng, int on);
int rp_get_full_mantissa(const rp_rng *rng);

/* Settings of a stream (rp_set_flag) or of a substream set
 * (rp_streams_set_flag), value 0 or 1.  A set takes its stream's settings
 * when it is created (rp_streams_create) and keeps them in its image
 * (rp_streams_serialize); rp_duplicate and rp_streams_duplicate copy them.
 *   RP_FULL_MANTISSA  the full-mantissa setting above (default 1).
 *   RP_SQUEEZE        the ziggurat's squeeze (Section 3.1: the secant and
 *                     tangent bands of each strip decide most wedge tests
 *                     without evaluating f(x)); default 1.  The bands carry
 *                     margins far above the rounding of the secant and of
 *                     exp, so the decisions, and therefore every value and
 *                     every state, are bit-identical with the squeeze on or
 *                     off; off evaluates f(x) for every wedge test.  Read by
 *                     every sampler built on the ziggurat (normal,
 *                     exponential, the laws, gamma, beta, moments, rows of
 *                     the multivariate normal, the one-stream split).
 *   RP_BITEXACT       (Section 4.2, exact reproducibility across platforms)
 *                     every exp, log, log1p and pow a sampler evaluates is
 *                     the correctly rounded one (rp_crmath below): the
 *                     ziggurat's wedge tests and tails, the gamma's log test
 *                     and its U^(1/a) boost (taken as the correctly rounded
 *                     u^(1/a), 1/a unrounded), and the transforms of
 *                     lognormal, Gumbel, Pareto, generalized Pareto and
 *                     Weibull.  A correctly rounded function has one
 *                     admissible result, so every value and every state is
 *                     then the same on any platform that evaluates the same
 *                     formulas; the affine parts are plain binary64
 *                     operations in the documented order here in every
 *                     mode.  Default 0 (the platform's exp / log, faithful
 *                     to an ulp; values can then differ in the last bit
 *                     where a result lands next to a rounding boundary).
 *                     Read by every sampler that calls those functions
 *                     (not by rp_mvn's matrix product, nor by the gradients).
 * rp_get_flag / rp_streams_get_flag return 1 or 0.  Errors: RP_ENULL;
 * RP_EINVAL for an unknown setting or a value other than 0 and 1. */
enum { RP_FULL_MANTISSA = 1, RP_SQUEEZE = 2, RP_BITEXACT = 3 };
int rp_set_flag(rp_rng *rng, int flag, int value);
int rp_get_flag(const rp_rng *rng, int flag);
int rp_streams_set_flag(rp_streams *s, int flag, int value);
int rp_streams_get_flag(const rp_streams *s, int flag);

/* Fills d_out[i * per_stream + t] (substream-major) with the next per_stream
 * values of substream i, for every substream, and advances each substream
 * past the words it used, so a second call continues the streams.  32-bit
 * outputs use the two halves of each word, low first; a half left over at
 * the end of a call is dropped.  d_out must hold n * per_stream elements of
 * dtype and be aligned to the element size.
 *
 * RP_NORM / RP_EXP with RP_F32 are the float versions of the two samplers
 * (Section 4.4, float versions): each draw reads 32-bit items; strip = low
 * byte, normal sign = bit 8, magnitude = the remaining 23 (normal) or 24
 * (exponential) bits; candidate and tests are the binary64 ziggurat's for
 * the magnitude m 2^29 (same tables); wedge and tail uniforms are 24-bit
 * uniforms of the following items; the value is rounded once to binary32.
 * rp_fill_serial gives the same float draws for one stream. */
int rp_fill(rp_streams *s, int dist, int dtype, uint64_t bound, int flags, void *d_out,
            uint64_t per_stream, void *hip_stream);

/* ---- derived continuous laws by transform (Table 4, Section 3.1) ------- */
/* rp_fill_law fills d_out[i * per_stream + t] (binary64, substream-major) with
 * per_stream draws of a derived law per substream, each draw one transform of
 * one base draw, the base draws being exactly those rp_fill would return
 * (U(0,1) with 53 bits, or the ziggurat N(0,1) or Exp(1)), so the streams
 * advance exactly as rp_fill advances them.  The transforms are evaluated in
 * binary64 in the order written (no contraction); "inv" values are formed
 * once on the host.  Parameters p[] (host memory):
 *   RP_LAW_UNIF      U(a,b),        p = {a, b}, a < b:       a + (b - a) U
 *   RP_LAW_NORMAL    N(mu,sigma^2), p = {mu, sigma}, s >= 0: mu + sigma Z
 *   RP_LAW_LOGNORMAL log N,         p = {mu, sigma}, s >= 0: exp(mu + sigma Z)
 *   RP_LAW_EXP       Exp(beta),     p = {beta}, beta > 0 (the scale): beta E
 *   RP_LAW_GUMBEL    Gumbel(mu,b),  p = {mu, b}, b > 0:      mu - b log(-log U)
 *   RP_LAW_PARETO    Pareto(xm,a),  p = {xm, a}, both > 0:   xm exp(E / a)
 *   RP_LAW_GPARETO   GPD(mu,s,xi),  p = {mu, s, xi}, s > 0:  with P =
 *                    exp(E / inv), inv = 1/|xi| (P is Pareto(1, 1/|xi|)):
 *                    xi > 0: mu + s (P - 1) / xi; xi < 0: mu - s (1 - 1/P) / xi;
 *                    xi = 0: mu + s E
 *   RP_LAW_WEIBULL   Weibull(k,l),  p = {k, l}, both > 0:    l pow(E, inv), inv = 1/k
 * Laws of several base draws per value (Marsaglia-Tsang gamma draws G with
 * the shape < 1 boost, ziggurat normals Z, drawn in the order listed):
 *   RP_LAW_GAMMA     Gamma(al,th),  p = {alpha, theta}, both > 0: theta G(alpha)
 *   RP_LAW_BETA      Beta(a,b),     p = {a, b}, both > 0: X / (X + Y), X = G(a) then Y = G(b)
 *   RP_LAW_CHI2      chi2(nu),      p = {nu}, nu > 0:   2 G(nu / 2)
 *   RP_LAW_T         t(nu),         p = {nu}, nu > 0:   Z / sqrt(V / nu), Z then V = 2 G(nu / 2)
 *   RP_LAW_F         F(nu1,nu2),    p = {nu1, nu2} > 0: (X / nu1) / (Y / nu2), X = G(nu1 / 2) then
 *                                                      Y = G(nu2 / 2)
 *   RP_LAW_SKEWNORMAL SN(mu,s,al),  p = {mu, s, alpha}, s >= 0: mu + s (d |Z0| + c Z1), Z0 then Z1,
 *                    d = alpha / sqrt(1 + alpha^2), c = sqrt(1 - d^2) (Azzalini's construction)
 * These run one lane per substream.  Parameters must be finite; others give
 * RP_EINVAL.  d_out must be 8-byte aligned device memory of n * per_stream
 * doubles owned by the caller.  Asynchronous on hip_stream; per_stream = 0
 * does nothing.
 * rp_fill_lawf is the binary32 form of laws 1-8 (the paper's float
 * versions): the base draw is the binary32 one rp_fill(..., RP_F32) returns
 * (24-bit uniform of a 32-bit item, or the float ziggurat's value), the
 * transform is evaluated in binary64 on that value and rounded once to
 * binary32; d_out holds n * per_stream floats (4-byte aligned).  Law 9 is
 * the float gamma: Marsaglia-Tsang on 32-bit items (the float ziggurat's
 * binary32 normal, 24-bit uniforms for the test and the shape < 1 boost),
 * binary64 arithmetic, theta G rounded once.  Laws 10-14 combine, on one
 * item stream per call, float gammas (the law 9 draw in binary64, before any
 * rounding) and binary32 normals of the float ziggurat as their binary64
 * forms above do, in binary64, rounded once to binary32. */
enum {
    RP_LAW_UNIF = 1,
    RP_LAW_NORMAL = 2,
    RP_LAW_LOGNORMAL = 3,
    RP_LAW_EXP = 4,
    RP_LAW_GUMBEL = 5,
    RP_LAW_PARETO = 6,
    RP_LAW_GPARETO = 7,
    RP_LAW_WEIBULL = 8,
    RP_LAW_GAMMA = 9,
    RP_LAW_BETA = 10,
    RP_LAW_CHI2 = 11,
    RP_LAW_T = 12,
    RP_LAW_F = 13,
    RP_LAW_SKEWNORMAL = 14
};
int rp_fill_law(rp_streams *s, int law, const double *p, int np, double *d_out, uint64_t per_stream,
                void *hip_stream);
int rp_fill_lawf(rp_streams *s, int law, const double *p, int np, float *d_out, uint64_t per_stream,
                 void *hip_stream);

/* ---- one stream split over many lanes (Section 4.4 jumps) -------------- */
/* Fills d_out[0 .. n-1] with the next n values of the single stream `rng`,
 * exactly as n serial calls would (same values, same order), and advances
 * rng past the words those values used (a 32-bit half left over at the end
 * is dropped, as in rp_fill).  The work is split over GPU lanes that start
 * at word offsets l C found by jump-ahead: the characteristic-polynomial
 * jump for x256++, affine powers for pcg64, counter arithmetic for Philox,
 * A^k for ranlux++.  Rejection samplers (normal, exponential, bounded) are
 * put back in serial order from per-chunk entry/exit maps; these forms wait
 * for the device (the consumed word count decides the new state), the
 * fixed-consumption forms (raw, uniform, bound 0) do not.  sfc64 has no
 * jump and runs on one lane.  dist, dtype, bound and flags as for rp_fill;
 * d_out is device memory of n elements owned by the caller. */
int rp_fill_serial(rp_rng *rng, int dist, int dtype, uint64_t bound, int flags, void *d_out, uint64_t n,
                   void *hip_stream);

/* ---- fused generate-and-reduce (Section 3.1 normals) -------------------- */
/* For every substream i draws per_stream standard normals (the same values
 * rp_fill(RP_NORM) would return) and stores only their sum and sum of
 * squares, accumulated in draw order in binary64: d_sum[i], d_sumsq[i].
 * The substreams are advanced as by that fill.  per_stream = 0 stores
 * zeros.  Device buffers of n doubles each, owned by the caller. */
int rp_norm_moments(rp_streams *s, uint64_t per_stream, double *d_sum, double *d_sumsq, void *hip_stream);

/* ---- gamma and beta, one draw per element (Section 3.1, "Gamma and ------ */
/* related distributions"; Table 4) ----------------------------------------- */
/* Element e (0 <= e < n <= number of substreams) draws one Gamma(alpha[e], 1)
 * value from substream e by Marsaglia and Tsang's method; shape < 1 draws
 * Gamma(alpha + 1) and then a uniform U and scales by U^(1/alpha).  The draw
 * is computed in binary64 from the binary32 shape and rounded once to
 * binary32 into z[e].  A shape that is not > 0 (or NaN) gives NaN and uses
 * no words.  Substreams e >= n are untouched.  All pointers are device
 * memory owned by the caller; n = 0 does nothing. */
int rp_gamma_elem(rp_streams *s, const float *d_alpha, float *d_z, uint64_t n, void *hip_stream);
/* Beta(a[e], b[e]) = X / (X + Y), X ~ Gamma(a) drawn before Y ~ Gamma(b) on
 * substream e; X + Y = 0 (both underflow) gives a / (a + b).  Invalid
 * parameters as for rp_gamma_elem. */
int rp_beta_elem(rp_streams *s, const float *d_a, const float *d_b, float *d_z, uint64_t n, void *hip_stream);

/* ---- batched gamma and beta (Section 3.1; Table 4) ---------------------- */
/* Set j (0 <= j < n_sets <= number of substreams) draws count[j] values from
 * substream j: Gamma(alpha[j], 1) by Marsaglia and Tsang's method (shape < 1:
 * Gamma(alpha + 1) then the U^(1/alpha) boost), or Beta(a[j], b[j]) as
 * X / (X + Y) with X ~ Gamma(a) drawn before Y ~ Gamma(b).  The values go to
 * d_out[offset_j ...], offset_j = count[0] + ... + count[j-1] (set-major), in
 * binary64, each set's values in its stream's serial order; the substreams
 * are advanced as by those serial draws.  Negative counts count as 0.  A set
 * whose parameter is not > 0 (or NaN) gets NaN values and its substream is
 * untouched.  d_out must hold sum(count) doubles; all arrays are device
 * memory owned by the caller.
 *
 * The plan holds scratch memory (about 12 bytes per set), the generator's
 * launch configuration, and a HIP graph recording the whole sequence (count
 * scan, sort of the sets longest first, persistent generator fed by an
 * atomic work queue).  A call with the same streams, pointers, n_sets and
 * configuration as the previous call on the plan replays that graph; other
 * calls record it again (and may allocate scratch).  A plan serves one call
 * at a time: calls on different HIP streams that may overlap need separate
 * plans.  n_sets = 0 does nothing. */
typedef struct rp_plan rp_plan;
int rp_plan_create(rp_plan **out);
void rp_plan_free(rp_plan *p);
/* block: threads per block (64, 128, 192 or 256); blocks_per_cu: resident
 * blocks asked for per compute unit (grid = CUs x blocks_per_cu, 1..64);
 * sets_per_lane: sets each lane takes from one popped group (1..16). */
int rp_plan_set_config(rp_plan *p, int block, int blocks_per_cu, int sets_per_lane);
/* Returns 1 if the configuration came from rp_plan_autotune, else 0. */
int rp_plan_get_config(const rp_plan *p, int *block, int *blocks_per_cu, int *sets_per_lane);
/* Times the generator over a grid of configurations on a copy of the
 * substreams (the caller's are not advanced) with the given inputs and keeps
 * the fastest.  beta = 0: gamma with d_pa = alpha (d_pb unused); beta = 1:
 * Beta(d_pa, d_pb).  d_out is overwritten.  Synchronizes the device. */
int rp_plan_autotune(rp_plan *p, rp_streams *s, int beta, const double *d_pa, const double *d_pb,
                     const int64_t *d_count, uint64_t n_sets, double *d_out);
int rp_gamma_batched(rp_streams *s, const double *d_alpha, const int64_t *d_count, uint64_t n_sets, double *d_out,
                     rp_plan *plan, void *hip_stream);
int rp_beta_batched(rp_streams *s, const double *d_a, const double *d_b, const int64_t *d_count, uint64_t n_sets,
                    double *d_out, rp_plan *plan, void *hip_stream);

/* ---- implicit-reparameterization backward (gamma and beta draws) -------- */
/* A draw z = F^{-1}(u; theta) is differentiated with u held fixed:
 * dz/dtheta = -(dF/dtheta)(z; theta) / f(z; theta), F the distribution
 * function and f the density of the Gamma(alpha, 1) or Beta(a, b) law
 * sampled by rp_gamma_elem / rp_beta_elem (Section 3.1 defines the laws; the
 * paper has no derivatives).  Each element returns g_theta = g_z dz/dtheta.
 * Inputs and outputs are binary32 device arrays of n elements owned by the
 * caller.  The derivative is evaluated in binary32 (the bulk) with an
 * estimate of its rounding error; where the estimate exceeds a fixed bound
 * (small z with large shapes, the tails of the series, cancellation in the
 * digamma combinations) the element is evaluated again in binary64 at the
 * same binary32 values.  On 2^20 elements of the [4096, 1024] workload
 * (shapes log-uniform over [0.05, 50]) the results are within 5e-6
 * (gamma) and 8e-6 (beta) relative of the all-binary64 evaluation
 * (rp_*_grad_host), with about 1 % (gamma) and 6 % (beta) of the elements
 * taking binary64.
 * z = 0 (or z = 1 for beta) gives 0; a parameter not > 0 or z outside the
 * support gives NaN.  Each result depends only on its own element, and an
 * output array may be the same as an input array (results overwrite their
 * inputs in place).  Stateless; n = 0 does nothing; pointers must be 4-byte
 * aligned (RP_EINVAL otherwise). */
int rp_gamma_grad(const float *d_z, const float *d_alpha, const float *d_gz, float *d_galpha, uint64_t n,
                  void *hip_stream);
int rp_beta_grad(const float *d_z, const float *d_a, const float *d_b, const float *d_gz, float *d_ga, float *d_gb,
                 uint64_t n, void *hip_stream);
/* The same results evaluated entirely in binary64 on the host (host arrays;
 * the reference precision the device's binary32 bulk is measured against).
 * Errors: RP_ENULL. */
int rp_gamma_grad_host(const float *z, const float *alpha, const float *gz, float *galpha, uint64_t n);
int rp_beta_grad_host(const float *z, const float *a, const float *b, const float *gz, float *ga, float *gb,
                      uint64_t n);

/* ---- permutations and samples (Section 3.2) ------------------------------ */
/* One instance per substream; every draw is a 32-bit bounded integer by
 * Lemire's method on the substream's 32-bit items (low half first; a half
 * left over at the end of the call is dropped), and each substream advances
 * past the items it used.
 * rp_permutations: d_out[i * n + q] (uint32, device) is the Fisher-Yates
 * permutation of 0..n-1 of substream i: start from the identity, for j from
 * n-1 down to 1 swap entries j and r, r uniform on {0..j}.  n = 0 does
 * nothing.
 * rp_sample: d_out[i * k + c] is a sample of k distinct elements of 0..n-1
 * (k <= n, k < 2^30): for k <= n/2 Floyd's algorithm (for j from n-k to n-1
 * draw t on {0..j}, append t, or j when t is already in the sample; entries
 * in the order appended), otherwise reservoir sampling (Vitter's algorithm
 * R: start from 0..k-1, for v from k to n-1 draw j on {0..v} and replace
 * entry j by v when j < k).  Floyd's membership test takes a workspace of
 * 2^ceil(log2(2k)) uint32 per substream from the stream-ordered pool.
 * k = 0 does nothing; k > n gives RP_EINVAL.  Asynchronous on hip_stream. */
int rp_permutations(rp_streams *s, uint32_t n, uint32_t *d_out, void *hip_stream);
int rp_sample(rp_streams *s, uint32_t n, uint32_t k, uint32_t *d_out, void *hip_stream);
/* rp_sample for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * identical results and stream advance, but Floyd's membership tables
 * (k <= n/2) live in a fixed 64 MiB device array inside the library (one per
 * GPU, held until the process ends) instead of the stream-ordered pool; the
 * call performs no allocation of any kind.  RP_EINVAL when the tables,
 * n_substreams x 2^ceil(log2(2k)) x 4 bytes, exceed 64 MiB.  The kernel
 * clears the tables it uses before reading them.  Every call on one GPU
 * shares that array: calls that may overlap on one GPU (different HIP
 * streams, host threads) race and must be serialized by the caller. */
int rp_sample_noalloc(rp_streams *s, uint32_t n, uint32_t k, uint32_t *d_out, void *hip_stream);

/* ---- multivariate normal (Section 3.1, "Multivariate normal distribution") */
/* Cholesky factor of a covariance matrix, on the host in binary64: reads the
 * lower triangle of Sigma (row-major d x d, host memory), writes L (row-major,
 * zeros above the diagonal) with Sigma = L L^T.  RP_ENOTSPD when a leading
 * minor is not positive definite (or not finite); L is then incomplete. */
int rp_cholesky(const double *Sigma, int d, double *L);
/* The factor A with Sigma = A A^T that rp_mvn takes (host, binary64; Section
 * 3.1): the Cholesky factor when Sigma (lower triangle read) is positive
 * definite, otherwise A = P L from a pivoted Cholesky factorization (LAPACK
 * dpstrf's rule: the largest remaining diagonal entry as pivot, stop at
 * tol = d eps max_i Sigma_ii), so A is not triangular and its columns from
 * *rank on are zero.  *rank = d in the definite case.  RP_ENOTSPD when a
 * trailing diagonal entry is below -tol (Sigma not semidefinite);
 * RP_EINVAL for non-finite entries.  A is d x d row-major host memory.
 * rp_mvn accepts this A unchanged (it reads the whole matrix); rp_mvn_backward
 * returns the gradient's lower triangle, the parameters of a Cholesky factor. */
int rp_mvn_factor(const double *Sigma, int d, double *A, int *rank);
/* Row i < n of X (n x d, row-major, binary32) is mu + L z_i, where z_i is the
 * next d standard normals of substream i (ziggurat in binary64, rounded to
 * binary32); that is X = mu + Z L^T.  The contraction runs on the matrix
 * cores in binary32 with binary32 accumulation.  L is the d x d factor
 * (row-major binary32), the Cholesky factor or any A from rp_mvn_factor:
 * the whole matrix is read, and when every entry above the diagonal is +0
 * the contraction skips the products with them (exact zeros; the check runs
 * on the device).  mu has d entries.  Substreams i < n are advanced by
 * their d normals.  Device pointers owned by the caller; a workspace of
 * n x d floats (plus 256 bytes) is taken from the device's stream-ordered
 * pool. */
int rp_mvn(rp_streams *s, const float *d_mu, const float *d_L, int d, uint64_t n, float *d_X, void *hip_stream);
/* Backward of rp_mvn for upstream gradient G (n x d): gmu = sum of the rows
 * of G, gL = tril(G^T Z) (d x d row-major, zeros above the diagonal).  Z is
 * regenerated from s, which must hold the substream states the forward
 * started from (for example an rp_streams_duplicate taken before it); s is
 * not advanced.  Partial sums over row slices are binary32 (matrix cores),
 * combined in binary64.  Uses a workspace of n x d floats plus the slice
 * partials from the stream-ordered pool. */
int rp_mvn_backward(rp_streams *s, const float *d_G, int d, uint64_t n, float *d_gmu, float *d_gL,
                    void *hip_stream);

/* ---- correctly rounded elementary functions (Section 4.2) ---------------- */
/* The functions the samplers call under the RP_BITEXACT setting, correctly
 * rounded to binary64 (round to nearest, ties to even) for every argument:
 *   RP_CR_EXP     exp(x)
 *   RP_CR_LOG     log(x)
 *   RP_CR_LOG1P   log(1 + x)
 *   RP_CR_POW     x^y, with the special values of C99 Annex F (F.9.4.4)
 *   RP_CR_POWINV  x^(1/y) for x >= 0, y > 0, the exponent 1/y exact (not
 *                 rounded), as exp(log(x)/y); NaN outside that domain.
 * Evaluation is in triple-double arithmetic (relative error below about
 * 2^-135) with one final correctly rounded three-term sum; for pow and
 * powinv a result that is itself exactly a binary64 midpoint is rounded
 * from that evaluation.  rp_crmath_host evaluates out[i] = f(x[i], y[i]) for
 * i < n on the host (host memory); rp_crmath does the same on the device
 * (device memory, queued on hip_stream, no allocation).  y is read only for
 * RP_CR_POW and RP_CR_POWINV (else it may be NULL).  The two give identical
 * bits.  Errors: RP_EINVAL for an unknown fn, RP_ENULL for a NULL x, out or
 * (when read) y, RP_EDEVICE for a failed launch. */
enum { RP_CR_EXP = 0, RP_CR_LOG = 1, RP_CR_LOG1P = 2, RP_CR_POW = 3, RP_CR_POWINV = 4 };
int rp_crmath_host(int fn, const double *x, const double *y, double *out, uint64_t n);
int rp_crmath(int fn, const double *d_x, const double *d_y, double *d_out, uint64_t n, void *hip_stream);

#ifdef __cplusplus
}
#endif
#endif /* RP_H */
