// engines.h -- engine arithmetic shared by the host core and the kernels.
//
// All functions are __host__ __device__ so the host core (substream setup,
// jumps, rp_raw_host) and the gfx950 kernels run the same arithmetic.
// Engine definitions follow Table 2 of the paper and the publications it
// cites for each engine.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

#define RP_HD __host__ __device__ __forceinline__

namespace rp {

RP_HD uint64_t rotl(uint64_t x, int k) { return (x << k) | (x >> (64 - k)); }

RP_HD uint64_t mulhi64(uint64_t a, uint64_t b)
{
#if defined(__HIP_DEVICE_COMPILE__)
    return __umul64hi(a, b);
#else
    return (uint64_t)(((unsigned __int128)a * b) >> 64);
#endif
}

// a ^ b ^ c: on the device one three-input bitwise instruction of gfx950
// (truth table 0x96), where the compiler would otherwise issue two xors
RP_HD uint32_t xor3_32(uint32_t a, uint32_t b, uint32_t c)
{
#if defined(__HIP_DEVICE_COMPILE__)
    return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);
#else
    return a ^ b ^ c;
#endif
}

RP_HD uint64_t xor3_64(uint64_t a, uint64_t b, uint64_t c)
{
    return (uint64_t)xor3_32((uint32_t)a, (uint32_t)b, (uint32_t)c) |
           ((uint64_t)xor3_32((uint32_t)(a >> 32), (uint32_t)(b >> 32), (uint32_t)(c >> 32)) << 32);
}

// ---------------------------------------------------------------------------
// 128-bit unsigned arithmetic (PCG64 state, Philox4x32 counter).
struct u128 {
    uint64_t lo, hi;
};

RP_HD u128 add128(u128 a, u128 b)
{
    u128 r;
    r.lo = a.lo + b.lo;
    r.hi = a.hi + b.hi + (r.lo < a.lo ? 1u : 0u);
    return r;
}

// low 128 bits of a * b
RP_HD u128 mul128(u128 a, u128 b)
{
    u128 r;
    r.lo = a.lo * b.lo;
    r.hi = mulhi64(a.lo, b.lo) + a.lo * b.hi + a.hi * b.lo;
    return r;
}

// ---------------------------------------------------------------------------
// xoshiro256++: linear map T on F_2^256 and the "++" scrambler applied to
// the state before the update.
struct X256 {
    uint64_t s0, s1, s2, s3;

    RP_HD void linear()
    {
        uint64_t t = s1 << 17;
        s2 ^= s0;
        s3 ^= s1;
        s1 ^= s2;
        s0 ^= s3;
        s2 ^= t;
        s3 = rotl(s3, 45);
    }
    RP_HD uint64_t next()
    {
        uint64_t r = rotl(s0 + s3, 23) + s0;
        linear();
        return r;
    }
    // xoshiro256** (Table 2 "x256**"): the same linear map, output
    // rotl(5 s1, 7) 9 of the state before the update
    RP_HD uint64_t next_ss()
    {
        uint64_t r = rotl(s1 * 5u, 7) * 9u;
        linear();
        return r;
    }
};

// xoroshiro128++ (Table 2 "xoro++"): linear map s1 ^= s0;
// s0 = rotl(s0, 49) ^ s1 ^ (s1 << 21); s1 = rotl(s1, 28); output
// rotl(s0 + s1, 17) + s0 of the state before the update.
struct Xoro128 {
    uint64_t s0, s1;
    RP_HD void linear()
    {
        const uint64_t t = s1 ^ s0;
        s0 = rotl(s0, 49) ^ t ^ (t << 21);
        s1 = rotl(t, 28);
    }
    RP_HD uint64_t next()
    {
        const uint64_t r = rotl(s0 + s1, 17) + s0;
        linear();
        return r;
    }
};

// xorshift128+ (Table 2 "x128+"), with the shift triple (23, 18, 5) of the
// current reference code: t = s0 ^ (s0 << 23); (s0, s1) <- (s1, t ^ s1 ^
// (t >> 18) ^ (s1 >> 5)); output s0 + s1 of the state before the update.
struct Xs128 {
    uint64_t s0, s1;
    RP_HD void linear()
    {
        uint64_t t = s0 ^ (s0 << 23);
        s0 = s1;
        s1 = t ^ s1 ^ (t >> 18) ^ (s1 >> 5);
    }
    RP_HD uint64_t next()
    {
        const uint64_t r = s0 + s1;
        linear();
        return r;
    }
};

// ---------------------------------------------------------------------------
// PCG64 DXSM: s <- s * M + inc (mod 2^128) with the 64-bit multiplier M;
// the output permutes the state before the step.
static constexpr uint64_t kPcgMult = 0xda942042e4dd58b5ull;

RP_HD uint64_t pcg_dxsm(u128 s)
{
    uint64_t hi = s.hi;
    uint64_t lo = s.lo | 1u;
    hi ^= hi >> 32;
    hi *= kPcgMult;
    hi ^= hi >> 48;
    hi *= lo;
    return hi;
}

RP_HD u128 pcg_step(u128 s, u128 inc)
{
    u128 r;
    r.lo = s.lo * kPcgMult;
    r.hi = mulhi64(s.lo, kPcgMult) + s.hi * kPcgMult;
    return add128(r, inc);
}

// ---------------------------------------------------------------------------
// Philox (Salmon et al. 2011), ten rounds, key bumped after every round.
static constexpr uint32_t kPh32M0 = 0xD2511F53u, kPh32M1 = 0xCD9E8D57u;
static constexpr uint32_t kPh32W0 = 0x9E3779B9u, kPh32W1 = 0xBB67AE85u;
static constexpr uint64_t kPh64M0 = 0xD2E7470EE14C6C93ull, kPh64M1 = 0xCA5A826395121157ull;
static constexpr uint64_t kPh64W0 = 0x9E3779B97F4A7C15ull, kPh64W1 = 0xBB67AE8584CAA73Bull;

// Block for 128-bit counter (c_lo, c_hi) and key (k0 | k1 << 32); returns the
// two 64-bit words (earlier 32-bit output in the low half).
// ChaCha20 (Table 2 "chacha20"): the block of counter ctr under the 256-bit
// key (eight 32-bit words) and the 96-bit nonce (n0, n1, n2): twenty rounds
// (ten column-and-diagonal double rounds) of the quarter round on the input
// words (constants "expand 32-byte k", key, counter, nonce), the input added
// back; word k of the output is x[2k] | x[2k+1] << 32.
RP_HD uint32_t rotl32(uint32_t x, int k) { return (x << k) | (x >> (32 - k)); }
#define RP_CHACHA_QR(a, b, c, d)                                                   \
    do {                                                                           \
        x[a] += x[b]; x[d] ^= x[a]; x[d] = rotl32(x[d], 16);                       \
        x[c] += x[d]; x[b] ^= x[c]; x[b] = rotl32(x[b], 12);                       \
        x[a] += x[b]; x[d] ^= x[a]; x[d] = rotl32(x[d], 8);                        \
        x[c] += x[d]; x[b] ^= x[c]; x[b] = rotl32(x[b], 7);                        \
    } while (0)
RP_HD void chacha20_block(const uint32_t key[8], uint32_t n0, uint32_t n1, uint32_t n2, uint32_t ctr,
                          uint64_t out[8])
{
    uint32_t in[16] = {0x61707865u, 0x3320646eu, 0x79622d32u, 0x6b206574u, key[0], key[1], key[2], key[3],
                       key[4],      key[5],      key[6],      key[7],      ctr,    n0,     n1,     n2};
    uint32_t x[16];
#pragma unroll
    for (int i = 0; i < 16; i++) x[i] = in[i];
#pragma unroll 1
    for (int r = 0; r < 10; r++) {
        RP_CHACHA_QR(0, 4, 8, 12);
        RP_CHACHA_QR(1, 5, 9, 13);
        RP_CHACHA_QR(2, 6, 10, 14);
        RP_CHACHA_QR(3, 7, 11, 15);
        RP_CHACHA_QR(0, 5, 10, 15);
        RP_CHACHA_QR(1, 6, 11, 12);
        RP_CHACHA_QR(2, 7, 8, 13);
        RP_CHACHA_QR(3, 4, 9, 14);
    }
#pragma unroll
    for (int k = 0; k < 8; k++) out[k] = (uint64_t)(x[2 * k] + in[2 * k]) | ((uint64_t)(x[2 * k + 1] + in[2 * k + 1]) << 32);
}
#undef RP_CHACHA_QR

// squares64 (Widynski; Table 2 "squares"): the word of counter c under key k.
// Five rounds on x = c k: square, add y = c k or z = y + k alternately and
// swap the 32-bit halves; the fourth round's square-plus-z t is kept, and
// the word is t xor the high half of the fifth round's x^2 + y.
RP_HD uint64_t squares64(uint64_t c, uint64_t k)
{
    uint64_t x = c * k;
    const uint64_t y = x, z = y + k;
    x = x * x + y;
    x = (x >> 32) | (x << 32);
    x = x * x + z;
    x = (x >> 32) | (x << 32);
    x = x * x + y;
    x = (x >> 32) | (x << 32);
    const uint64_t t = x * x + z;
    x = (t >> 32) | (t << 32);
    return t ^ ((x * x + y) >> 32);
}

RP_HD void philox4x32(uint64_t c_lo, uint64_t c_hi, uint64_t key, uint64_t &w0, uint64_t &w1)
{
    uint32_t x0 = (uint32_t)c_lo, x1 = (uint32_t)(c_lo >> 32);
    uint32_t x2 = (uint32_t)c_hi, x3 = (uint32_t)(c_hi >> 32);
    uint32_t k0 = (uint32_t)key, k1 = (uint32_t)(key >> 32);
#pragma unroll
    for (int r = 0; r < 10; r++) {
        uint64_t p0 = (uint64_t)kPh32M0 * x0;
        uint64_t p1 = (uint64_t)kPh32M1 * x2;
        uint32_t y0 = xor3_32((uint32_t)(p1 >> 32), x1, k0);
        uint32_t y2 = xor3_32((uint32_t)(p0 >> 32), x3, k1);
        x1 = (uint32_t)p1;
        x3 = (uint32_t)p0;
        x0 = y0;
        x2 = y2;
        k0 += kPh32W0;
        k1 += kPh32W1;
    }
    w0 = (uint64_t)x0 | ((uint64_t)x1 << 32);
    w1 = (uint64_t)x2 | ((uint64_t)x3 << 32);
}

RP_HD void philox4x64(const uint64_t c[4], uint64_t k0, uint64_t k1, uint64_t out[4])
{
    uint64_t x0 = c[0], x1 = c[1], x2 = c[2], x3 = c[3];
#pragma unroll
    for (int r = 0; r < 10; r++) {
        uint64_t h0 = mulhi64(kPh64M0, x0), l0 = kPh64M0 * x0;
        uint64_t h1 = mulhi64(kPh64M1, x2), l1 = kPh64M1 * x2;
        uint64_t y0 = xor3_64(h1, x1, k0);
        uint64_t y2 = xor3_64(h0, x3, k1);
        x1 = l1;
        x3 = l0;
        x0 = y0;
        x2 = y2;
        k0 += kPh64W0;
        k1 += kPh64W1;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

// ---------------------------------------------------------------------------
// sfc64: state (a, b, c, counter); output a + b + counter.
struct Sfc64 {
    uint64_t a, b, c, ctr;
    RP_HD uint64_t next()
    {
        uint64_t r = a + b + ctr;
        ctr += 1;
        a = b ^ (b >> 11);
        b = c + (c << 3);
        c = rotl(c, 24) + r;
        return r;
    }
};

// ---------------------------------------------------------------------------
// cwg128 (Dziala's Collatz-Weyl generator, 128-bit words): per step
// a += x, weyl += s, x = (x >> 1) * (a | 1) ^ weyl; the word is the low half
// of (a >> 96) ^ x.  s (the Weyl increment, the stream selector) is odd.
struct Cwg128 {
    u128 x, a, w, s;
    RP_HD uint64_t next()
    {
        a = add128(a, x);
        w = add128(w, s);
        const u128 xh{(x.lo >> 1) | (x.hi << 63), x.hi >> 1};
        const u128 p = mul128(xh, u128{a.lo | 1u, a.hi});
        x = u128{p.lo ^ w.lo, p.hi ^ w.hi};
        return (a.hi >> 32) ^ x.lo;
    }
};

// ---------------------------------------------------------------------------
// ranlux++: x <- A x mod m, m = 2^576 - 2^240 + 1, on nine 64-bit limbs
// (little-endian).
//
// A product of two residues has 18 limbs, P = H 2^576 + L.  Since
// 2^576 = 2^240 - 1 (mod m), P = L + (H << 240) - H (mod m) ("fold").
// Fold 1 (H: 9 limbs) leaves a value below 2^817 (13 limbs); fold 2 (H: the
// top 241 bits, 4 limbs) leaves a value below 2^576 + 2^481 (10 limbs);
// fold 3 (H: 0 or 1) leaves a value below 2^576.  Every fold result is
// non-negative because (H << 240) >= H.  Finally m is subtracted once if the
// value is >= m, tested as "value + 2^240 - 1 carries out of 2^576".
static constexpr int kRlLimbs = 9;

// out[0..NOUT) = L + (H << 240) - H, with L = in[0..9) and H = in[9..9+NH)
template <int NH, int NOUT>
RP_HD void rl_fold(const uint64_t *in, uint64_t *out)
{
    const uint64_t *H = in + 9;
    uint64_t carry = 0;
#pragma unroll
    for (int k = 0; k < NOUT; k++) {
        uint64_t l = (k < 9) ? in[k] : 0;
        uint64_t sh = 0;
        if (k - 3 >= 0 && k - 3 < NH) sh |= H[k - 3] << 48;
        if (k - 4 >= 0 && k - 4 < NH) sh |= H[k - 4] >> 16;
        uint64_t t = l + sh;
        uint64_t c = (t < l) ? 1u : 0u;
        uint64_t t2 = t + carry;
        c += (t2 < t) ? 1u : 0u;
        out[k] = t2;
        carry = c;
    }
    uint64_t borrow = 0;
#pragma unroll
    for (int k = 0; k < NOUT; k++) {
        uint64_t h = (k < NH) ? H[k] : 0;
        uint64_t v = out[k];
        uint64_t d = v - h;
        uint64_t b = (v < h) ? 1u : 0u;
        uint64_t d2 = d - borrow;
        b += (d < borrow) ? 1u : 0u;
        out[k] = d2;
        borrow = b;
    }
}

// out[0..9) = r3 mod m for r3 < 2^576: subtract m once if r3 >= m, tested as
// "r3 + 2^240 - 1 carries out of 2^576".
RP_HD void rl_final(const uint64_t r3[9], uint64_t x[9])
{
    uint64_t t[9];
    uint64_t carry = 0;
#pragma unroll
    for (int k = 0; k < 9; k++) {
        uint64_t add = (k < 3) ? ~0ull : (k == 3 ? ((1ull << 48) - 1) : 0ull);
        uint64_t s1 = r3[k] + add;
        uint64_t c = (s1 < add) ? 1u : 0u;
        uint64_t s2 = s1 + carry;
        c += (s2 < s1) ? 1u : 0u;
        t[k] = s2;
        carry = c;
    }
#pragma unroll
    for (int k = 0; k < 9; k++) x[k] = carry ? t[k] : r3[k];
}

// x = p mod m for an 18-limb product p
RP_HD void rl_reduce(const uint64_t p[18], uint64_t x[9])
{
    uint64_t r1[13], r2[10], r3[9];
    rl_fold<9, 13>(p, r1);
    rl_fold<4, 10>(r1, r2);
    rl_fold<1, 9>(r2, r3);
    rl_final(r3, x);
}

RP_HD void rl_mul_full(const uint64_t a[9], const uint64_t b[9], uint64_t p[18])
{
#pragma unroll
    for (int i = 0; i < 18; i++) p[i] = 0;
#pragma unroll
    for (int i = 0; i < 9; i++) {
        uint64_t carry = 0;
#pragma unroll
        for (int j = 0; j < 9; j++) {
            uint64_t lo = a[i] * b[j];
            uint64_t hi = mulhi64(a[i], b[j]);
            uint64_t t = p[i + j] + lo;
            hi += (t < lo) ? 1u : 0u;
            uint64_t t2 = t + carry;
            hi += (t2 < t) ? 1u : 0u;
            p[i + j] = t2;
            carry = hi;
        }
        p[i + 9] = carry;
    }
}

RP_HD void rl_mulmod(const uint64_t a[9], const uint64_t b[9], uint64_t x[9])
{
    uint64_t p[18];
    rl_mul_full(a, b, p);
    rl_reduce(p, x);
}

// ---------------------------------------------------------------------------
// The generator step x <- A x mod m with the reduction folded into a table.
// Write x = sum_i x_i 2^(29 i) with 20 limbs x_i of 29 bits (580 >= 576) and
// let B_i = 2^(29 i) A mod m, itself in 29-bit limbs B_i,j.  Then
//     A x = sum_j y_j 2^(29 j)  (mod m),   y_j = sum_i x_i B_i,j,
// and each column sum y_j of 20 products below 2^58 stays below 2^64, so a
// column is a chain of 32x32->64 multiply-adds with no carry handling.
// After the carries are propagated the value is below 20 2^29 m < 2^610;
// one fold of its top word and one of the 0/1 overflow bring it below 2^576
// and a conditional subtraction of m finishes.  B is stored row-major by
// output limb: B[j * 20 + i] = B_i,j.
static constexpr int kRlL = 20;
static constexpr uint32_t kRlM29 = (1u << 29) - 1;

template <class TAB>
RP_HD void rl_mul_tab(const uint64_t in[9], TAB *B, uint64_t out[9])
{
    uint32_t d[18];
#pragma unroll
    for (int k = 0; k < 9; k++) {
        d[2 * k] = (uint32_t)in[k];
        d[2 * k + 1] = (uint32_t)(in[k] >> 32);
    }
    uint32_t x[kRlL];
#pragma unroll
    for (int i = 0; i < kRlL; i++) {
        const int p = 29 * i, k = p >> 5, off = p & 31;
        uint32_t v = d[k] >> off;
        if (off > 3 && k + 1 < 18) v |= d[k + 1] << (32 - off);
        x[i] = v & kRlM29;
    }
    uint32_t D[20];
#pragma unroll
    for (int k = 0; k < 20; k++) D[k] = 0;
    uint64_t carry = 0;
#pragma unroll
    for (int j = 0; j < kRlL; j++) {
        uint64_t s0 = 0, s1 = 0;
#pragma unroll
        for (int i = 0; i < kRlL; i += 2) {
            s0 += (uint64_t)x[i] * B[j * kRlL + i];
            s1 += (uint64_t)x[i + 1] * B[j * kRlL + i + 1];
        }
        const uint64_t z = s0 + s1 + carry;
        const uint32_t limb = (uint32_t)z & kRlM29;
        carry = z >> 29;
        const int p = 29 * j, k = p >> 5, off = p & 31;
        D[k] |= limb << off;
        if (off > 3) D[k + 1] |= limb >> (32 - off);
    }
    // carry has weight 2^580 = bit 4 of dword 18
    D[18] |= (uint32_t)carry << 4;
    D[19] |= (uint32_t)(carry >> 28);
    uint64_t p[10], r2[10], r3[9];
#pragma unroll
    for (int q = 0; q < 10; q++) p[q] = D[2 * q] | ((uint64_t)D[2 * q + 1] << 32);
    rl_fold<1, 10>(p, r2);
    rl_fold<1, 9>(r2, r3);
    rl_final(r3, out);
}

}  // namespace rp
