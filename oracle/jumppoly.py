"""Jump polynomials for the xor-family engines (test infrastructure).

Section 4.4 ("Jumping"): T is linear on F_2^n, so by Cayley--Hamilton
T^N = p(T) for a polynomial p of degree < n, namely p(x) = x^N mod P(x)
where P is the characteristic polynomial of T.  Here P is obtained with the
Berlekamp--Massey algorithm from one state bit over 2n steps of the linear
core, and x^N mod P by square-and-multiply.  Polynomials over GF(2) are
Python integers (bit k = coefficient of x^k).
"""
import ctypes

import numpy as np


def berlekamp_massey(bits):
    """Shortest LFSR (connection polynomial C, length L) generating bits."""
    c, b = 1, 1
    length, m = 0, 1
    for n, s in enumerate(bits):
        d = s
        for i in range(1, length + 1):
            d ^= ((c >> i) & 1) & bits[n - i]
        if d == 0:
            m += 1
        elif 2 * length <= n:
            t = c
            c ^= b << m
            length, b, m = n + 1 - length, t, 1
        else:
            c ^= b << m
            m += 1
    return c, length


def char_poly_from_bits(bits):
    """Characteristic polynomial from an output-bit sequence.

    The connection polynomial C(z) = 1 + c_1 z + ... + c_L z^L corresponds to
    the recurrence s_n = sum c_i s_{n-i}; its reciprocal
    P(x) = x^L + c_1 x^{L-1} + ... + c_L is the minimal polynomial of T on
    that sequence."""
    c, length = berlekamp_massey(bits)
    p = 0
    for i in range(length + 1):
        if (c >> i) & 1:
            p |= 1 << (length - i)
    return p, length


def pmulmod(a, b, p):
    """a * b mod p over GF(2)."""
    deg = p.bit_length() - 1
    r = 0
    while b:
        if b & 1:
            r ^= a
        b >>= 1
        a <<= 1
        if (a >> deg) & 1:
            a ^= p
    return r


def pmod(a, p):
    deg = p.bit_length() - 1
    while a.bit_length() - 1 >= deg:
        a ^= p << (a.bit_length() - 1 - deg)
    return a


def xpow_mod(n, p):
    """x^n mod p over GF(2) by square-and-multiply."""
    result, base = 1, pmod(2, p)
    while n:
        if n & 1:
            result = pmulmod(result, base, p)
        base = pmulmod(base, base, p)
        n >>= 1
    return result


def poly_words(poly, nwords=4):
    return np.array([(poly >> (64 * i)) & ((1 << 64) - 1) for i in range(nwords)], dtype=np.uint64)


_X256_P = None


def x256_char_poly(lib):
    """Characteristic polynomial of the xoshiro256 linear core (degree 256)."""
    global _X256_P
    if _X256_P is None:
        st = np.array([0x0123456789ABCDEF, 0x0F1E2D3C4B5A6978, 0x1, 0xDEADBEEF], dtype=np.uint64)
        bits = np.zeros(512, dtype=np.uint64)
        lib.or_x256_linear_steps(st.ctypes.data_as(ctypes.c_void_p),
                                 bits.ctypes.data_as(ctypes.c_void_p), ctypes.c_size_t(512))
        p, length = char_poly_from_bits([int(b) for b in bits])
        assert length == 256, length
        _X256_P = p
    return _X256_P


_X128_P = {}


def x128_char_poly(lib, engine):
    """Characteristic polynomial of a 128-bit xor engine's linear core
    (xoroshiro128 or xorshift128; degree 128)."""
    if engine not in _X128_P:
        st = np.array([0x0123456789ABCDEF, 0x0F1E2D3C4B5A6978], dtype=np.uint64)
        bits = np.zeros(256, dtype=np.uint64)
        rc = lib.or_x128_linear_steps(ctypes.c_uint64(engine), st.ctypes.data_as(ctypes.c_void_p),
                                      bits.ctypes.data_as(ctypes.c_void_p), ctypes.c_size_t(256))
        assert rc == 0
        p, length = char_poly_from_bits([int(b) for b in bits])
        assert length == 128, length
        _X128_P[engine] = p
    return _X128_P[engine]
