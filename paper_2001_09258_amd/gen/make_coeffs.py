"""Generate ``csrc/generated/poly_coeffs.inc`` and ``gen/poly_report.txt``.

Every polynomial the kernels evaluate is listed in SPECS: the function it
approximates (written so that the exactly known leading terms are split off,
as the paper does when it keeps the lowest terms in double-double; Section 5,
overview), the interval of the reduced argument, the weight (relative error
of the final function), the target format and the error goal.  The degree is
the smallest that reaches the goal after the coefficients are rounded.

Run:  python -m paper_2001_09258_amd.gen.make_coeffs
"""
import os
import sys
import time

import mpmath as mp

from .remez import remez, remez_rounded

mp.mp.prec = 320
ZERO_EPS = mp.mpf(10) ** -40

HERE = os.path.dirname(os.path.abspath(__file__))
OUT_INC = os.path.join(HERE, "..", "csrc", "generated", "poly_coeffs.inc")
OUT_REPORT = os.path.join(HERE, "poly_report.txt")


def _series_guard(f, series):
    """Evaluate f(z), or its series near z = 0 where f cancels."""
    def g(z):
        if abs(z) < mp.mpf(10) ** -24:
            return series(z)
        return f(z)
    return g


# ---- target functions (z is the polynomial variable) ---------------------

def exp_p():
    f = _series_guard(lambda r: (mp.exp(r) - 1 - r) / r ** 2,
                      lambda r: mp.mpf(1) / 2 + r / 6 + r ** 2 / 24)
    w = lambda r: r ** 2 / mp.exp(r)
    L = mp.log(2) / 2 * mp.mpf("1.002")
    return f, w, -L, L


def log_q():
    # log m = 2t + t^3 Q(t^2), t = (m-1)/(m+1), m in [0.75, 1.5)
    f = _series_guard(lambda z: (2 * mp.atanh(mp.sqrt(z)) - 2 * mp.sqrt(z)) / z ** mp.mpf(1.5),
                      lambda z: mp.mpf(2) / 3 + 2 * z / 5 + 2 * z ** 2 / 7)
    w = lambda z: z ** mp.mpf(1.5) / (2 * mp.atanh(mp.sqrt(z))) if z > 0 else mp.mpf(0)
    return f, w, mp.mpf(0), mp.mpf(1) / 25 * mp.mpf("1.01")


def log_r():
    # log m = 2t + (2/3) t^3 + t^5 R(t^2)
    f = _series_guard(lambda z: (2 * mp.atanh(mp.sqrt(z)) - 2 * mp.sqrt(z)
                                 - mp.mpf(2) / 3 * z ** mp.mpf(1.5)) / z ** mp.mpf(2.5),
                      lambda z: mp.mpf(2) / 5 + 2 * z / 7 + 2 * z ** 2 / 9)
    w = lambda z: z ** mp.mpf(2.5) / (2 * mp.atanh(mp.sqrt(z))) if z > 0 else mp.mpf(0)
    return f, w, mp.mpf(0), mp.mpf(1) / 25 * mp.mpf("1.01")


def log_r7():
    # log m = 2t + (2/3) t^3 + (2/5) t^5 + t^7 R7(t^2): pow's logarithm, whose
    # relative error is multiplied by |y log x| (up to ~745) in the result
    f = _series_guard(lambda z: (2 * mp.atanh(mp.sqrt(z)) - 2 * mp.sqrt(z)
                                 - mp.mpf(2) / 3 * z ** mp.mpf(1.5)
                                 - mp.mpf(2) / 5 * z ** mp.mpf(2.5)) / z ** mp.mpf(3.5),
                      lambda z: mp.mpf(2) / 7 + 2 * z / 9 + 2 * z ** 2 / 11)
    w = lambda z: z ** mp.mpf(3.5) / (2 * mp.atanh(mp.sqrt(z))) if z > 0 else mp.mpf(0)
    return f, w, mp.mpf(0), mp.mpf(1) / 25 * mp.mpf("1.01")


LGAM_T = mp.mpf("0.0625")


def lgam1():
    # log Gamma(1 + t) = -gamma t + t^2 L1(t), |t| <= 1/16
    f = _series_guard(lambda t: (mp.loggamma(1 + t) + mp.euler * t) / t ** 2,
                      lambda t: mp.zeta(2) / 2 - mp.zeta(3) / 3 * t + mp.zeta(4) / 4 * t ** 2)
    # relative weight t^2 / |log Gamma(1 + t)| = |t| / |-gamma + t L1(t)|
    w = lambda t: abs(t) / abs(-mp.euler + t * f(t))
    return f, w, -LGAM_T * mp.mpf("1.001"), LGAM_T * mp.mpf("1.001")


def lgam2():
    # log Gamma(2 + t) = (1 - gamma) t + t^2 L2(t), |t| <= 1/16
    f = _series_guard(lambda t: (mp.loggamma(2 + t) - (1 - mp.euler) * t) / t ** 2,
                      lambda t: (mp.zeta(2) - 1) / 2 - (mp.zeta(3) - 1) / 3 * t
                      + (mp.zeta(4) - 1) / 4 * t ** 2)
    w = lambda t: abs(t) / abs((1 - mp.euler) + t * f(t))
    return f, w, -LGAM_T * mp.mpf("1.001"), LGAM_T * mp.mpf("1.001")


def sin_s():
    # sin r = r + r^3 S(r^2), |r| <= pi/2
    f = _series_guard(lambda z: (mp.sin(mp.sqrt(z)) - mp.sqrt(z)) / z ** mp.mpf(1.5),
                      lambda z: -mp.mpf(1) / 6 + z / 120 - z ** 2 / 5040)
    w = lambda z: z ** mp.mpf(1.5) / mp.sin(mp.sqrt(z)) if z > 0 else mp.mpf(0)
    return f, w, mp.mpf(0), (mp.pi / 2) ** 2 * mp.mpf("1.0005")


def sin_s2():
    # sin r = r - r^3/6 + r^5 S2(r^2)
    f = _series_guard(lambda z: (mp.sin(mp.sqrt(z)) - mp.sqrt(z) + z ** mp.mpf(1.5) / 6)
                      / z ** mp.mpf(2.5),
                      lambda z: mp.mpf(1) / 120 - z / 5040 + z ** 2 / 362880)
    w = lambda z: z ** mp.mpf(2.5) / mp.sin(mp.sqrt(z)) if z > 0 else mp.mpf(0)
    return f, w, mp.mpf(0), (mp.pi / 2) ** 2 * mp.mpf("1.0005")


def sin_s3():
    # sin r = r - r^3/6 + r^5/120 + r^7 S3(r^2)
    f = _series_guard(lambda z: (mp.sin(mp.sqrt(z)) - mp.sqrt(z) + z ** mp.mpf(1.5) / 6
                                 - z ** mp.mpf(2.5) / 120) / z ** mp.mpf(3.5),
                      lambda z: -mp.mpf(1) / 5040 + z / 362880 - z ** 2 / 39916800)
    w = lambda z: z ** mp.mpf(3.5) / mp.sin(mp.sqrt(z)) if z > 0 else mp.mpf(0)
    return f, w, mp.mpf(0), (mp.pi / 2) ** 2 * mp.mpf("1.0005")


def tan_t():
    # tan y = y + y^3 T(y^2), |y| <= pi/8
    f = _series_guard(lambda z: (mp.tan(mp.sqrt(z)) - mp.sqrt(z)) / z ** mp.mpf(1.5),
                      lambda z: mp.mpf(1) / 3 + 2 * z / 15 + 17 * z ** 2 / 315)
    w = lambda z: z ** mp.mpf(1.5) / mp.tan(mp.sqrt(z)) if z > 0 else mp.mpf(0)
    return f, w, mp.mpf(0), (mp.pi / 8) ** 2 * mp.mpf("1.002")


def atan_a():
    # atan t = t + t^3 A(t^2), 0 <= t <= 1
    f = _series_guard(lambda z: (mp.atan(mp.sqrt(z)) - mp.sqrt(z)) / z ** mp.mpf(1.5),
                      lambda z: -mp.mpf(1) / 3 + z / 5 - z ** 2 / 7)
    w = lambda z: z ** mp.mpf(1.5) / mp.atan(mp.sqrt(z)) if z > 0 else mp.mpf(0)
    return f, w, mp.mpf(0), mp.mpf(1)


def atan_a2():
    # atan t = t - t^3/3 + t^5 A2(t^2)
    f = _series_guard(lambda z: (mp.atan(mp.sqrt(z)) - mp.sqrt(z) + z ** mp.mpf(1.5) / 3)
                      / z ** mp.mpf(2.5),
                      lambda z: mp.mpf(1) / 5 - z / 7 + z ** 2 / 9)
    w = lambda z: z ** mp.mpf(2.5) / mp.atan(mp.sqrt(z)) if z > 0 else mp.mpf(0)
    return f, w, mp.mpf(0), mp.mpf(1)


def atan_b2():
    # atan v = v - v^3/3 + v^5 B2(v^2), 0 <= v <= tan(pi/8): the argument
    # after atan t = pi/4 + atan((t - 1)/(t + 1)) for t > tan(pi/8)
    f = _series_guard(lambda z: (mp.atan(mp.sqrt(z)) - mp.sqrt(z) + z ** mp.mpf(1.5) / 3)
                      / z ** mp.mpf(2.5),
                      lambda z: mp.mpf(1) / 5 - z / 7 + z ** 2 / 9)
    w = lambda z: z ** mp.mpf(2.5) / mp.atan(mp.sqrt(z)) if z > 0 else mp.mpf(0)
    return f, w, mp.mpf(0), mp.tan(mp.pi / 8) ** 2 * mp.mpf("1.001")


def asin_s():
    # asin x = x + x^3 S(x^2), |x| <= 1/2 (Section 5, asin/acos: the
    # reduced argument lies in [0, 0.5])
    f = _series_guard(lambda z: (mp.asin(mp.sqrt(z)) - mp.sqrt(z)) / z ** mp.mpf(1.5),
                      lambda z: mp.mpf(1) / 6 + 3 * z / 40 + 15 * z ** 2 / 336)
    w = lambda z: z ** mp.mpf(1.5) / mp.asin(mp.sqrt(z)) if z > 0 else mp.mpf(0)
    return f, w, mp.mpf(0), mp.mpf(1) / 4 * mp.mpf("1.0001")


def sinh_h():
    # sinh x = x + x^3 H(x^2), |x| <= 1
    f = _series_guard(lambda z: (mp.sinh(mp.sqrt(z)) - mp.sqrt(z)) / z ** mp.mpf(1.5),
                      lambda z: mp.mpf(1) / 6 + z / 120 + z ** 2 / 5040)
    w = lambda z: z ** mp.mpf(1.5) / mp.sinh(mp.sqrt(z)) if z > 0 else mp.mpf(0)
    return f, w, mp.mpf(0), mp.mpf("1.0001")


def tanh_g():
    # tanh x = x + x^3 G(x^2), |x| <= 0.625
    f = _series_guard(lambda z: (mp.tanh(mp.sqrt(z)) - mp.sqrt(z)) / z ** mp.mpf(1.5),
                      lambda z: -mp.mpf(1) / 3 + 2 * z / 15 - 17 * z ** 2 / 315)
    w = lambda z: z ** mp.mpf(1.5) / mp.tanh(mp.sqrt(z)) if z > 0 else mp.mpf(0)
    return f, w, mp.mpf(0), mp.mpf("0.625") ** 2 * mp.mpf("1.0001")


def erf_p():
    # erf x = c0 x + c1 x^3 + x^5 P(z), z = x^2 <= 0.75^2, c0 = 2/sqrt(pi),
    # c1 = -c0/3 (both kept as pairs in the kernel)
    c0 = 2 / mp.sqrt(mp.pi)
    c1 = -c0 / 3
    f = _series_guard(lambda z: ((mp.erf(mp.sqrt(z)) / mp.sqrt(z) - c0) / z - c1) / z,
                      lambda z: c0 * (mp.mpf(1) / 10 - z / 42 + z ** 2 / 216))
    w = lambda z: z ** 2 * mp.sqrt(z) / mp.erf(mp.sqrt(z)) if z > 0 else mp.mpf(0)
    return f, w, mp.mpf(0), mp.mpf("0.5626")


# name, target builder, format, error goal (log2), first degree tried
SPECS = [
    ("EXP_P_F64", exp_p, "f64", -63, 10),
    ("LOG_Q_F64", log_q, "f64", -62, 6),
    ("LOG_R_F64", log_r, "f64", -60, 7),
    ("LOG_R7_F64", log_r7, "f64", -67, 5),
    ("LGAM1_F64", lgam1, "f64", -60, 8),
    ("LGAM2_F64", lgam2, "f64", -60, 8),
    ("SIN_S_F64", sin_s, "f64", -60, 7),
    ("SIN_S2_F64", sin_s2, "f64", -62, 6),
    ("SIN_S3_F64", sin_s3, "f64", -62, 5),
    ("TAN_T_F64", tan_t, "f64", -62, 8),
    ("ATAN_A_F64", atan_a, "f64", -58, 16),
    ("ATAN_A2_F64", atan_a2, "f64", -61, 16),
    ("ATAN_B2_F64", atan_b2, "f64", -62, 6),
    ("SINH_H_F64", sinh_h, "f64", -62, 5),
    ("ASIN_S_F64", asin_s, "f64", -58, 8),
    ("TANH_G_F64", tanh_g, "f64", -62, 9),
    ("ERF_P_F64", erf_p, "f64", -60, 5),
    ("EXP_P_F32", exp_p, "f32", -32, 4),
    ("LOG_Q_F32", log_q, "f32", -31, 2),
    ("LOG_R_F32", log_r, "f32", -36, 2),
    ("SIN_S_F32", sin_s, "f32", -30, 4),
    ("SIN_S2_F32", sin_s2, "f32", -31, 3),
    ("SIN_S3_F32", sin_s3, "f32", -31, 2),
    ("TAN_T_F32", tan_t, "f32", -31, 3),
    ("ATAN_A_F32", atan_a, "f32", -28, 6),
    ("ATAN_A2_F32", atan_a2, "f32", -31, 6),
    ("ATAN_B2_F32", atan_b2, "f32", -32, 2),
    ("SINH_H_F32", sinh_h, "f32", -31, 2),
    ("ASIN_S_F32", asin_s, "f32", -29, 3),
    ("ERF_P_F32", erf_p, "f32", -28, 2),
    ("ATAN_N_F32", atan_a, "f32", -19, 3),
    ("TANH_G_F32", tanh_g, "f32", -31, 4),
]


def _hex(v, fmt):
    if fmt == "f64":
        return float(v).hex()
    return float(v).hex() + "f"


def _existing():
    """name -> (comment line, definition line) of the current output file."""
    out = {}
    if os.path.exists(OUT_INC):
        lines = open(OUT_INC).read().splitlines()
        for i, ln in enumerate(lines):
            if ln.startswith("__device__ constexpr"):
                name = ln.split()[3].split("[")[0]
                out[name] = (lines[i - 1], ln)
    rep = {}
    if os.path.exists(OUT_REPORT):
        for ln in open(OUT_REPORT).read().splitlines():
            if ln.strip():
                rep[ln.split()[0]] = ln
    return out, rep


def build(names=None, verbose=True):
    lines = ["// Generated by paper_2001_09258_amd/gen/make_coeffs.py -- do not edit.",
             "// Minimax coefficients (own Remez tool, relative-error weight); lowest",
             "// degree first.  Errors of the rounded polynomials: gen/poly_report.txt.",
             "#pragma once", ""]
    report = []
    old, old_rep = _existing()
    for name, builder, fmt, goal, n0 in SPECS:
        if names and name not in names:
            if name in old:
                lines.extend([old[name][0], old[name][1], ""])
                report.append(old_rep.get(name, name))
            continue
        f, w, a, b = builder()
        n = n0
        t0 = time.time()
        # smallest degree whose exact minimax error is a bit below the goal,
        # then the greedy rounding (one more coefficient if rounding hurts)
        while n < 24:
            _, e_exact = remez(f, w, a, b, n, iters=12, grid=500)
            if float(mp.log(e_exact, 2)) <= goal - 1:
                break
            n += 1
        while True:
            vals, err = remez_rounded(f, w, a, b, n, fmt, iters=8, grid=600)
            e2 = float(mp.log(err, 2)) if err > 0 else -999
            if e2 <= goal or n >= 24:
                break
            n += 1
        ctype = "double" if fmt == "f64" else "float"
        body = ", ".join(_hex(v, fmt) for v in vals)
        lines.append("// %s: %d coefficients on [%s, %s], max weighted error 2^%.2f"
                     % (name, n, mp.nstr(a, 6), mp.nstr(b, 6), e2))
        lines.append("__device__ constexpr %s %s[%d] = {%s};" % (ctype, name, n, body))
        lines.append("")
        report.append("%-12s %s  n=%2d  [%s, %s]  err=2^%.2f  (goal 2^%d)"
                      % (name, fmt, n, mp.nstr(a, 8), mp.nstr(b, 8), e2, goal))
        if verbose:
            print(report[-1], "%.0fs" % (time.time() - t0), flush=True)
    with open(OUT_INC, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    with open(OUT_REPORT, "w") as fh:
        fh.write("\n".join(report) + "\n")


if __name__ == "__main__":
    build(sys.argv[1:] or None)
