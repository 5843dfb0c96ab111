"""Generate csrc/zig_tables.inc: ziggurat, squeeze and log tables for the kernels.

Geometry (Section 3.1 and the ziggurat figure): 256 strips of equal area v
under f (normal: exp(-x^2/2), exponential: exp(-x)); edges
0 = x_0 < x_1 < ... < x_255 = r; strip j >= 1 is the rectangle
[0, x_j] x [f(x_j), f(x_{j-1})]; strip 0 is [0, r] x [0, f(r)] plus the tail.

This generator solves the geometry TOP-DOWN: for a trial area v it places
the rectangles from the peak of f downwards (each edge x_{j+1} solves
x_{j+1} (f(x_j) - f(x_{j+1})) = v by Newton's method) and then adjusts v by
the secant method until the base strip also has area v.  (The test oracle
solves the same geometry bottom-up by bisection on r; the two sets of doubles
are compared bit for bit by the test suite.)

Per strip the kernels get
  W[j] = x_j 2^-B (j >= 1), W[0] = (v / f(r)) 2^-B      magnitude scale
  K[j] = floor(2^B x_{j-1} / x_j), K[0] = floor(2^B r f(r) / v)   fast-accept bound
  F[j] = f(x_j), F[0] = 1                               strip heights
and, for the squeeze that skips exp() in the wedge test (the paper's
McFarland-type saving), with the secant l_j(x) = F[j-1] + S[j] (x - X[j-1]):
  X[j]  = x_j                                           edges
  S[j]  = slope of the secant through (x_{j-1}, f(x_{j-1})) and (x_j, f(x_j))
  DP[j] = max(f - l_j) over the strip, plus a safety margin
  DM[j] = max(l_j - f) over the strip, plus a safety margin
The maxima sit where f'(x) equals the secant slope: for the normal
x* = sqrt(-W_k(-s^2)) (Lambert W, k = 0 when x* < 1, k = -1 when x* > 1); for
the exponential x* = -ln(-s).  The margin (1e-13, far above the few-ulp
rounding of l_j and of exp) makes a squeeze decision agree with the plain
test y < f(x) evaluated in binary64.

B = 52 for the normal (52-bit magnitude), 53 for the exponential.

The log table (c_i, 1/c_i, log c_i as hi + lo) lets the gamma boost form
log(U) to about 2^-70 absolute, so that U^(1/alpha) = exp(log(U)/alpha) stays
within an ulp even when |log(U)/alpha| is in the hundreds.
Run: python paper_2605_05099_amd/csrc/gen_tables.py
"""
import os

import mpmath as mp

mp.mp.dps = 60
N = 256
MARGIN = mp.mpf("1e-13")


class Normal:
    name, B = "ZN", 52

    @staticmethod
    def f(x):
        return mp.exp(-x * x / 2)

    @staticmethod
    def df(x):
        return -x * mp.exp(-x * x / 2)

    @staticmethod
    def tail(r):
        return mp.sqrt(mp.pi / 2) * mp.erfc(r / mp.sqrt(2))

    @staticmethod
    def tangent_points(s, a, b):
        pts = []
        for k in (0, -1):
            w = mp.lambertw(-s * s, k)
            if abs(mp.im(w)) < mp.mpf(10) ** -40:
                x = mp.sqrt(-mp.re(w))
                if a <= x <= b:
                    pts.append(x)
        return pts


class Exponential:
    name, B = "ZE", 53

    @staticmethod
    def f(x):
        return mp.exp(-x)

    @staticmethod
    def df(x):
        return -mp.exp(-x)

    @staticmethod
    def tail(r):
        return mp.exp(-r)

    @staticmethod
    def tangent_points(s, a, b):
        x = -mp.log(-s)
        return [x] if a <= x <= b else []


def _place(D, v):
    """Top-down placement for area v; returns edges x_0..x_255."""
    x = [mp.mpf(0)]
    top = mp.mpf(1)  # f(x_0)
    guess = mp.mpf("0.2")
    for j in range(1, N):
        # solve g(t) = t (top - f(t)) - v = 0, t > x_{j-1}
        t = max(guess, x[-1] * (1 + mp.mpf("1e-3")))
        for _ in range(200):
            g = t * (top - D.f(t)) - v
            dg = (top - D.f(t)) - t * D.df(t)
            step = g / dg
            t = t - step
            if abs(step) < mp.mpf(10) ** -55 * max(1, abs(t)):
                break
        x.append(t)
        top = D.f(t)
        guess = t + (t - x[-2])
    return x


def solve(D):
    def base_residual(v):
        x = _place(D, v)
        r = x[-1]
        return r * D.f(r) + D.tail(r) - v

    v0, v1 = mp.mpf("0.0049") if D is Normal else mp.mpf("0.0039"), None
    v1 = v0 * (1 + mp.mpf("1e-3"))
    r0, r1 = base_residual(v0), base_residual(v1)
    for _ in range(100):
        v2 = v1 - r1 * (v1 - v0) / (r1 - r0)
        v0, r0 = v1, r1
        v1, r1 = v2, base_residual(v2)
        if abs(v1 - v0) < mp.mpf(10) ** -55:
            break
    return _place(D, v1), v1


def tables(D):
    x, v = solve(D)
    r = x[-1]
    two_b = mp.mpf(2) ** D.B
    W = [float(v / D.f(r) / two_b)] + [float(x[j] / two_b) for j in range(1, N)]
    K = [int(mp.floor(two_b * r * D.f(r) / v))] + [int(mp.floor(two_b * x[j - 1] / x[j])) for j in range(1, N)]
    F = [1.0] + [float(D.f(x[j])) for j in range(1, N)]
    X = [float(x[j]) for j in range(N)]
    S = [0.0] * N
    DP = [0.0] * N
    DM = [0.0] * N
    for j in range(1, N):
        a, b = x[j - 1], x[j]
        fa = D.f(a) if j > 1 else mp.mpf(1)
        s = (D.f(b) - fa) / (b - a)
        line = lambda t: fa + s * (t - a)
        dev = [D.f(t) - line(t) for t in D.tangent_points(s, a, b)]
        dp = max([mp.mpf(0)] + [d for d in dev if d > 0])
        dm = max([mp.mpf(0)] + [-d for d in dev if d < 0])
        S[j] = float(s)
        DP[j] = float(dp + MARGIN)
        DM[j] = float(dm + MARGIN)
    return dict(r=float(r), v=float(v), W=W, K=K, F=F, X=X, S=S, DP=DP, DM=DM)


def _arr(ctype, name, vals, fmt):
    body = ",\n".join("  " + ", ".join(fmt(v) for v in vals[i:i + 4]) for i in range(0, len(vals), 4))
    return f"RP_TBL {ctype} {name}[256] = {{\n{body}\n}};"


def log_table():
    """Table for an accurate log on [1, 2): c_i = 1 + (i + 1/2)/256, with
    1/c_i rounded and log(c_i) as a pair of doubles (hi + lo)."""
    C, INV, HI, LO = [], [], [], []
    for i in range(256):
        c = 1 + (mp.mpf(i) + mp.mpf(1) / 2) / 256
        C.append(float(c))
        INV.append(float(1 / c))
        lg = mp.log(c)
        hi = float(lg)
        HI.append(hi)
        LO.append(float(lg - mp.mpf(hi)))
    ln2 = mp.log(2)
    # ln2 split so that e * LN2_HI is exact for |e| < 2^11
    ln2_hi = float(mp.floor(ln2 * 2**42) / 2**42)
    ln2_lo = float(ln2 - mp.mpf(ln2_hi))
    return C, INV, HI, LO, ln2_hi, ln2_lo


def main():
    out = ["// Generated by csrc/gen_tables.py (mpmath, 60 digits, top-down solve). Do not edit.",
           "// Define RP_TBL (e.g. as `__device__ const`) before including.",
           "#pragma once", "#include <cstdint>", "#ifndef RP_TBL", "#define RP_TBL static const", "#endif"]
    for D in (Normal, Exponential):
        t = tables(D)
        p = "RP_" + D.name
        out.append(f"static constexpr double {p}_R = {float.hex(t['r'])};  // {t['r']!r}")
        out.append(f"static constexpr double {p}_V = {float.hex(t['v'])};  // {t['v']!r}")
        hx = lambda v: float.hex(v)
        out.append(_arr("double", p + "_W", t["W"], hx))
        out.append(_arr("uint64_t", p + "_K", t["K"], lambda v: f"{v}ull"))
        out.append(_arr("double", p + "_F", t["F"], hx))
        out.append(_arr("double", p + "_X", t["X"], hx))
        out.append(_arr("double", p + "_S", t["S"], hx))
        out.append(_arr("double", p + "_DP", t["DP"], hx))
        out.append(_arr("double", p + "_DM", t["DM"], hx))
    C, INV, HI, LO, l2h, l2l = log_table()
    hx = lambda v: float.hex(v)
    out.append(f"static constexpr double RP_LN2_HI = {hx(l2h)};")
    out.append(f"static constexpr double RP_LN2_LO = {hx(l2l)};")
    out.append(_arr("double", "RP_LOG_C", C, hx))
    out.append(_arr("double", "RP_LOG_INV", INV, hx))
    out.append(_arr("double", "RP_LOG_HI", HI, hx))
    out.append(_arr("double", "RP_LOG_LO", LO, hx))
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "zig_tables.inc")
    with open(path, "w") as fh:
        fh.write("\n".join(out) + "\n")
    return path


if __name__ == "__main__":
    print(main())
