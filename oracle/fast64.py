"""ctypes binding of the oracle's fast binary64 stage (``oracle/fast/fast64.c``)
for sin, cos, tan, exp, exp2, log, log2, sinh, cosh, tanh, asin, acos, atan, log10,
log1p, exp10, expm1, cbrt, asinh, acosh, atanh, erf, erfc, lgamma, tgamma, pow and
atan2.

TEST INFRASTRUCTURE ONLY (see the package docstring).  The C stage gives the
value within 2^-90 relative (lgamma and tgamma: a bound of its own per input)
and the correctly rounded binary64 result where
that bound decides it; ``evaluate`` and ``check_all`` send the inputs it
cannot decide to the ball oracle.  Pinned against mpmath and the ball oracle
in ``tests/test_oracle_fast.py``.
"""
import concurrent.futures as cf
import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "fast", "fast64.c")
DEPS = [SRC, os.path.join(HERE, "fast", "common.h"), os.path.join(HERE, "fast", "binary.h"),
        os.path.join(HERE, "fast", "tables.h")]
LIB = os.path.join(HERE, "liboracle_fast64.so")
FNS = {"sin": 0, "exp": 1, "log": 2, "cos": 3, "tan": 4, "exp2": 5, "log2": 6, "sinh": 7,
       "cosh": 8, "tanh": 9, "asin": 10, "acos": 11, "atan": 12, "log10": 13, "log1p": 14,
       "exp10": 15, "expm1": 16, "cbrt": 17, "asinh": 18, "acosh": 19, "atanh": 20, "erf": 21,
       "erfc": 22, "lgamma": 23, "tgamma": 24}
FNS2 = {"pow": 0, "atan2": 1}          # two operands (oracle/fast/binary.h)

_lib = None


def build():
    """Compile the C stage (gcc, IEEE binary64, no contraction; fma() as the
    x86-64 fused multiply-add)."""
    tmp = "%s.tmp%d" % (LIB, os.getpid())
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-mfma", "-ffp-contract=off",
           "-fno-fast-math", "-o", tmp, SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


class CheckStats(ctypes.Structure):
    _fields_ = [("n", ctypes.c_long), ("undecided", ctypes.c_long),
                ("special_mismatch", ctypes.c_long), ("violations", ctypes.c_long),
                ("max_ulp", ctypes.c_double), ("sum_ulp", ctypes.c_double),
                ("n_reg", ctypes.c_long), ("worst", ctypes.c_long)]


def load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < max(os.path.getmtime(d) for d in DEPS):
            build()
        lib = ctypes.CDLL(LIB)
        P = ctypes.c_void_p
        lib.oracle_fast64_eval.restype = None
        lib.oracle_fast64_rel.restype = None
        lib.oracle_fast64_rel.argtypes = [ctypes.c_int, P, ctypes.c_long, P]
        lib.oracle_fast64_eval.argtypes = [ctypes.c_int, P, ctypes.c_long, P, P, P, P]
        lib.oracle_fast64_check.restype = None
        lib.oracle_fast64_check.argtypes = [ctypes.c_int, P, P, ctypes.c_long, ctypes.c_double,
                                            ctypes.POINTER(CheckStats), P, ctypes.c_long, P,
                                            ctypes.c_long]
        lib.oracle_fast64_eval2.restype = None
        lib.oracle_fast64_eval2.argtypes = [ctypes.c_int, P, P, ctypes.c_long, P, P, P, P]
        lib.oracle_fast64_check2.restype = None
        lib.oracle_fast64_check2.argtypes = [ctypes.c_int, P, P, P, ctypes.c_long, ctypes.c_double,
                                             ctypes.POINTER(CheckStats), P, ctypes.c_long, P,
                                             ctypes.c_long]
        _lib = lib
    return _lib


def fast_eval(fn, x, z=None):
    """The C stage alone: (rn, hi, lo, undecided) for binary64 inputs x (and
    second operands z for pow and atan2)."""
    lib = load()
    x = np.ascontiguousarray(x, dtype=np.float64)
    n = x.size
    hi, lo, rn = (np.empty(n, np.float64) for _ in range(3))
    und = np.empty(n, np.uint8)
    if fn in FNS2:
        z = np.ascontiguousarray(z, dtype=np.float64)
        assert z.size == n
        lib.oracle_fast64_eval2(FNS2[fn], x.ctypes.data, z.ctypes.data, n, hi.ctypes.data,
                                lo.ctypes.data, rn.ctypes.data, und.ctypes.data)
    else:
        lib.oracle_fast64_eval(FNS[fn], x.ctypes.data, n, hi.ctypes.data, lo.ctypes.data,
                               rn.ctypes.data, und.ctypes.data)
    return rn, hi, lo, und.astype(bool)


def fast_rel(fn, x):
    """The relative error bound the C stage claims for each input's pair
    (0 where its result is exact), one-operand functions."""
    lib = load()
    x = np.ascontiguousarray(x, dtype=np.float64)
    rel = np.empty(x.size, np.float64)
    lib.oracle_fast64_rel(FNS[fn], x.ctypes.data, x.size, rel.ctypes.data)
    return rel


def evaluate(fn, x, z=None):
    """(rn, hi, lo) as oracle.evaluate(fn, "f64", x[, z]), undecided inputs
    by the ball oracle."""
    from . import evaluate as ball_evaluate
    rn, hi, lo, und = fast_eval(fn, x, z)
    if und.any():
        zz = None if z is None else np.asarray(z, np.float64)[und]
        r2, h2, l2 = ball_evaluate(fn, "f64", np.asarray(x, np.float64)[und], zz)
        rn[und], hi[und], lo[und] = r2, h2, l2
    return rn, hi, lo


def check(fn, x, y, bound, cap=1 << 10, z=None):
    """Results y for inputs x (and second operands z) against the C stage
    (tests/ulp.py's metric): (stats, failing indices, undecided indices)."""
    lib = load()
    x = np.ascontiguousarray(x, dtype=np.float64)
    y = np.ascontiguousarray(y, dtype=np.float64)
    st = CheckStats()
    bad = np.empty(cap, np.int64)
    und = np.empty(cap, np.int64)
    if fn in FNS2:
        z = np.ascontiguousarray(z, dtype=np.float64)
        lib.oracle_fast64_check2(FNS2[fn], x.ctypes.data, z.ctypes.data, y.ctypes.data, x.size,
                                 bound, ctypes.byref(st), bad.ctypes.data, cap, und.ctypes.data,
                                 cap)
    else:
        lib.oracle_fast64_check(FNS[fn], x.ctypes.data, y.ctypes.data, x.size, bound,
                                ctypes.byref(st), bad.ctypes.data, cap, und.ctypes.data, cap)
    return st, bad[:min(st.special_mismatch + st.violations, cap)], und[:min(st.undecided, cap)]


def check_all(fn, x, y, bound, threads=16, chunk=1 << 20, z=None):
    """check() over chunks on a thread pool; returns a dict of totals with
    the failing and undecided indices (up to 1024 each)."""
    load()
    tot = dict(n=0, undecided=0, special_mismatch=0, violations=0, n_reg=0, max_ulp=0.0,
               sum_ulp=0.0)
    bad, und = [], []
    with cf.ThreadPoolExecutor(threads) as ex:
        futs = [(s, ex.submit(check, fn, x[s:s + chunk], y[s:s + chunk], bound,
                              z=None if z is None else z[s:s + chunk]))
                for s in range(0, x.size, chunk)]
        for s, f in futs:
            st, b, u = f.result()
            for k in ("n", "undecided", "special_mismatch", "violations", "n_reg"):
                tot[k] += getattr(st, k)
            tot["sum_ulp"] += st.sum_ulp
            tot["max_ulp"] = max(tot["max_ulp"], st.max_ulp)
            bad.append(b + s)
            und.append(u + s)
    tot["bad"] = np.concatenate(bad)[:1024] if bad else np.zeros(0, np.int64)
    tot["undecided_idx"] = np.concatenate(und)[:1024] if und else np.zeros(0, np.int64)
    return tot
