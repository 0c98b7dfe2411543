"""Generate ``csrc/generated/consts.inc``: split constants for the kernels.

* Cody-Waite pieces of pi/2 and pi (Section 5, sin/cos and tan), all
  doubles.  binary64 (|q| < 2^14): the two leading pieces carry 39
  significant bits, so q times either is an exact double, the first one
  truncated towards zero (the head subtraction x - q*C0 is then exact by
  Sterbenz's lemma); the other two are the nearest doubles to what is left.
  binary32 (reduced in binary64, |q| < 2^16): a 37-bit truncated head and
  the nearest double to the rest.
* ln 2 for exp/pow reductions: a leading part with 11 (float: 8) trailing zero
  bits, so k * LN2_HI is exact for every reduction integer k that occurs,
  plus the rounded rest.
* double-double (float-float) values of pi/2, pi, 1/ln2, 1/3, 2/3, 1/6,
  ln 10, 1/ln 10, 2/sqrt(pi) and -2/(3 sqrt(pi)).
* the binary64 accurate path's constants (see accurate_path_constants).

mpmath at 600 bits; this is a build step of the GPU library, independent of
the test oracle.   Run:  python -m paper_2001_09258_amd.gen.make_consts
"""
import os

import mpmath as mp
import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
OUT = os.path.join(HERE, "..", "csrc", "generated", "consts.inc")

mp.mp.prec = 600


def rnd(v, fmt):
    return mp.mpf(float(v)) if fmt == "f64" else mp.mpf(float(np.float32(float(v))))


def split(v, n, fmt):
    out = []
    rest = v
    for _ in range(n):
        h = rnd(rest, fmt)
        out.append(h)
        rest -= h
    return out


def short_pieces(v, bits, n):
    """n pieces of v: a head of ``bits`` significant bits truncated towards
    zero (at least 2^-50 below v, which Sterbenz's lemma needs at q = 1),
    for n = 4 a second rounded piece of ``bits`` bits, then nearest doubles."""
    e = int(mp.floor(mp.log(abs(v), 2)))
    scale = mp.mpf(2) ** (bits - 1 - e)
    c0 = mp.floor(v * scale) / scale
    assert (v - c0) / v >= mp.mpf(2) ** -50
    out = [c0]
    if n == 4:
        out.append(trailing_zero_head(v - c0, bits))
    while len(out) < n:
        out.append(rnd(v - sum(out), "f64"))
    for c in out:
        assert mp.mpf(float(c)) == c
    return out


def trailing_zero_head(v, bits):
    """v rounded to ``bits`` significant bits."""
    e = int(mp.floor(mp.log(abs(v), 2)))
    scale = mp.mpf(2) ** (bits - 1 - e)
    return mp.nint(v * scale) / scale


def cw_float_pieces(v):
    """Four binary32 pieces of v for the float-float Cody-Waite reduction:
    c0 the nearest float, c1 the rest rounded to 8 significant bits (q*c1
    exact for |q| < 2^16), c2 and c3 the nearest floats to what is left."""
    c0 = rnd(v, "f32")
    c1 = trailing_zero_head(v - c0, 8)
    c2 = rnd(v - c0 - c1, "f32")
    c3 = rnd(v - c0 - c1 - c2, "f32")
    out = [c0, c1, c2, c3]
    for c in out:
        assert mp.mpf(float(np.float32(float(c)))) == c
    assert abs(v - sum(out)) < abs(v) * mp.mpf(2) ** -78
    return out


def accurate_path_constants(lines, ln2, head):
    """Constants of the binary64 accurate path (results in the subnormal
    range, where the last bit needs about 2^-100 relative accuracy):
    ln 2 in three pieces, the first two of 42 significant bits (k times
    either is exact for |k| <= 2048); ln 10 in three doubles; 1/n! for
    n = 0..13 as pairs and n = 14..23 as doubles (the Taylor series of e^r);
    1/(2n+1) for n = 0..11 as pairs and n = 12..23 as doubles (the series of
    atanh, log m = 2 atanh t); the coefficients of erfc's asymptotic series."""
    P = "__device__ constexpr double "
    b = trailing_zero_head(ln2 - head, 42)
    c = rnd(ln2 - head - b, "f64")
    lines.append(P + "LN2_A_D = %s;  // 42 significant bits" % hx(head, "f64"))
    lines.append(P + "LN2_B_D = %s;  // 42 significant bits" % hx(b, "f64"))
    lines.append(P + "LN2_C_D = %s;" % hx(c, "f64"))
    for i, t in enumerate(split(mp.log(10), 3, "f64")):
        lines.append(P + "LN10_T%d_D = %s;" % (i, hx(t, "f64")))

    def table(name, vals):
        lines.append(P + "%s[%d] = {%s};" % (name, len(vals), ", ".join(hx(v, "f64") for v in vals)))

    fact = [1 / mp.factorial(n) for n in range(24)]
    pairs = [split(v, 2, "f64") for v in fact[:14]]
    table("INVFACT_D_H", [h for h, _ in pairs])
    table("INVFACT_D_L", [l for _, l in pairs])
    table("INVFACT_TAIL_D", [rnd(v, "f64") for v in fact[14:]])
    odd = [mp.mpf(1) / (2 * n + 1) for n in range(24)]
    pairs = [split(v, 2, "f64") for v in odd[:12]]
    table("INVODD_D_H", [h for h, _ in pairs])
    table("INVODD_D_L", [l for _, l in pairs])
    table("INVODD_TAIL_D", [rnd(v, "f64") for v in odd[12:]])
    # erfc's asymptotic series in z = 1/a^2: (-1)^n (2n-1)!!/2^n, exact doubles
    asym = []
    for n in range(16):
        df = mp.mpf(1)
        for j in range(1, 2 * n, 2):
            df *= j
        c = (-1) ** n * df / mp.mpf(2) ** n
        assert mp.mpf(float(c)) == c
        asym.append(c)
    table("ERFC_ASYM_D", asym)


def gamma_constants(lines):
    """lgamma/tgamma: Euler's gamma, 1 - gamma, log(2 pi)/2 and log pi as
    pairs; Stirling's coefficients B_2k / (2k (2k - 1)), k = 1..10, from
    exact Bernoulli numbers."""
    from fractions import Fraction
    P = "__device__ constexpr double "
    for name, v in (("EULER", mp.euler), ("ONE_M_EULER", 1 - mp.euler),
                    ("HALF_LN2PI", mp.log(2 * mp.pi) / 2), ("LNPI", mp.log(mp.pi))):
        h, l = split(v, 2, "f64")
        lines.append(P + "%s_D_H = %s;" % (name, hx(h, "f64")))
        lines.append(P + "%s_D_L = %s;" % (name, hx(l, "f64")))
    bern = [Fraction(1)]
    for m in range(1, 22):
        acc, c = Fraction(0), 1
        for j in range(m):
            acc += c * bern[j]
            c = c * (m + 1 - j) // (j + 1)
        bern.append(-acc / (m + 1))
    coef = [bern[2 * k] / (2 * k * (2 * k - 1)) for k in range(1, 11)]
    lines.append(P + "LGAM_STIRLING_D[10] = {%s};" % ", ".join(
        hx(rnd(mp.mpf(c.numerator) / c.denominator, "f64"), "f64") for c in coef))
    lines.append(P + "LGAM_STIRLING_TAIL_D[9] = {%s};" % ", ".join(
        hx(rnd(mp.mpf(c.numerator) / c.denominator, "f64"), "f64") for c in coef[1:]))
    # sine's Taylor series for the accurate reflection: 1/7! and 1/9! as
    # pairs, the terms from r^11 on as doubles
    for name, n in (("INV5040", 7), ("INV362880", 9)):
        h, l = split(mp.mpf(1) / mp.factorial(n), 2, "f64")
        lines.append(P + "%s_D_H = %s;" % (name, hx(h, "f64")))
        lines.append(P + "%s_D_L = %s;" % (name, hx(l, "f64")))
    tail = [(-1) ** (k + 1) / mp.factorial(11 + 2 * k) for k in range(8)]
    lines.append(P + "SIN_TAYLOR11_D[8] = {%s};" % ", ".join(hx(rnd(v, "f64"), "f64") for v in tail))


def hx(v, fmt):
    return float(v).hex() + ("f" if fmt == "f32" else "")


def main():
    lines = ["// Generated by paper_2001_09258_amd/gen/make_consts.py -- do not edit.",
             "#pragma once", ""]
    for fmt, ctype, sfx, hbits in (("f64", "double", "D", 42), ("f32", "float", "F", 16)):
        P = "__device__ constexpr %s " % ctype
        for name, v in (("PIH", mp.pi / 2), ("PI", mp.pi)):
            if fmt == "f64":
                parts, tag = short_pieces(v, 39, 4), "D"
                for i, p in enumerate(parts):
                    lines.append("__device__ constexpr double %s_%s_%d = %s;"
                                 % (name, tag, i, hx(p, "f64")))
            else:
                for i, p in enumerate(cw_float_pieces(v)):
                    lines.append(P + "%s_F_C%d = %s;" % (name, i, hx(p, "f32")))
        ln2 = mp.log(2)
        head = trailing_zero_head(ln2, hbits)
        lines.append(P + "LN2_HI_%s = %s;  // %d significant bits" % (sfx, hx(head, fmt), hbits))
        lines.append(P + "LN2_LO_%s = %s;" % (sfx, hx(rnd(ln2 - head, fmt), fmt)))
        for name, v in (("LN2", ln2), ("INVLN2", 1 / ln2), ("THIRD", mp.mpf(1) / 3),
                        ("TWOTHIRD", mp.mpf(2) / 3), ("SIXTH", mp.mpf(1) / 6), ("INV120", mp.mpf(1) / 120),
                        ("PIH2", mp.pi / 2), ("PI2", mp.pi), ("LN10", mp.log(10)),
                        ("INVLN10", 1 / mp.log(10)), ("TWO_OVER_SQRTPI", 2 / mp.sqrt(mp.pi)),
                        ("ERF_C1", -2 / (3 * mp.sqrt(mp.pi)))):
            h, l = split(v, 2, fmt)
            lines.append(P + "%s_%s_H = %s;" % (name, sfx, hx(h, fmt)))
            lines.append(P + "%s_%s_L = %s;" % (name, sfx, hx(l, fmt)))
        if fmt == "f64":
            accurate_path_constants(lines, ln2, head)
            gamma_constants(lines)
        for name, v in (("LOG2E", 1 / mp.log(2)), ("INV_PI", 1 / mp.pi),
                        ("TWO_OVER_PI", 2 / mp.pi), ("LOG2_10", mp.log(10, 2))):
            lines.append(P + "%s_%s = %s;" % (name, sfx, hx(rnd(v, fmt), fmt)))
        lines.append("")
    with open(OUT, "w") as fh:
        fh.write("\n".join(lines) + "\n")


if __name__ == "__main__":
    main()
