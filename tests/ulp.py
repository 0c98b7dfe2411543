"""ULP error of library results against the oracle (test-side helper).

The metric: ulp(v) = 2^(max(floor(log2|v|), emin) - p + 1) for the exact value
v of the output format; the error of a result y is |y - v| / ulp(v).  An
infinite y against a finite v counts as 2^(emax+1).  Results whose correctly
rounded value is NaN, +-inf or +-0 must match it bit for bit (NaN as a class);
these are reported separately from the ULP statistics.

Subnormal results: in binary64 and binary32 a result whose correctly rounded
value is subnormal must match it bit for bit (the strict reading of the
paper's special-number handling, Section 5, "Handling of Special Numbers",
which itself only promises the error bound there).  For bf16, f16 and the
binary32-through-binary64 form, whose last step rounds an already rounded
value (or a binary32 one) into a narrow format, subnormal mismatches are
counted and reported ("subnormal_mismatch") while the ULP bound still holds;
pass subnormal="exact" or "report" to choose explicitly.
"""
import numpy as np

FMT = {"f64": (53, -1022, 1023), "f32": (24, -126, 127),
       "bf16": (8, -126, 127), "f16": (11, -14, 15)}


def _floor_log2(hi, lo):
    m, e = np.frexp(np.abs(hi))          # |hi| = m 2^e, m in [0.5, 1)
    e = e.astype(np.int64) - 1
    # v = hi + lo lies just below a power of two when hi is one and lo
    # has the opposite sign
    pow2 = m == 0.5
    below = pow2 & (np.sign(lo) == -np.sign(hi)) & (lo != 0)
    return np.where(below, e - 1, e)


def compare(y, rn, hi, lo, fmt, bound, subnormal=None):
    """Returns a dict with max/mean ULP error, the number of bound
    violations, special-class mismatches (subnormal results included when
    they are held bit-exact), subnormal-result mismatches and the indices of
    failures."""
    if subnormal is None:
        subnormal = "exact" if fmt in ("f64", "f32") else "report"
    assert subnormal in ("exact", "report")
    p, emin, emax = FMT[fmt]
    y = np.asarray(y, dtype=np.float64)
    rn = np.asarray(rn, dtype=np.float64)
    hi = np.asarray(hi, dtype=np.float64)
    lo = np.asarray(lo, dtype=np.float64)
    special = np.isnan(rn) | np.isinf(rn) | (rn == 0)
    same = (y == rn) & (np.signbit(y) == np.signbit(rn))
    same |= np.isnan(y) & np.isnan(rn)
    with np.errstate(invalid="ignore"):
        sub = ~special & (np.abs(rn) < 2.0 ** emin)
    sub_bad = sub & ~same
    if subnormal == "exact":
        special = special | sub
    special_bad = special & ~same
    reg = ~special
    with np.errstate(invalid="ignore", over="ignore", divide="ignore"):
        e = np.maximum(_floor_log2(hi, lo), emin)
        ulp = np.ldexp(1.0, (e - p + 1).astype(np.int32))
        # an infinite result against a finite value counts as 2^(emax+1);
        # scale by 1/2 first so that 2^(emax+1) stays finite for binary64
        yy = np.where(np.isinf(y), np.sign(y) * 2.0 ** emax * 2.0 if emax < 1023 else 0.0, y)
        err = np.abs((yy - hi) - lo) / ulp
        inf_err = np.abs((np.sign(y) * 2.0 ** emax - hi * 0.5) - lo * 0.5) / (ulp * 0.5)
        err = np.where(np.isinf(y), inf_err, err)
    err = np.where(np.isnan(y), np.inf, err)
    # a result equal to the correctly rounded value is within half an ulp by
    # definition (next to 2^emin the pair's low word can lose that fraction)
    err = np.where(same & reg, np.minimum(err, 0.5), err)
    err = np.where(reg, err, 0.0)
    viol = reg & (err > bound)
    res = {
        "n": int(y.size),
        "max_ulp": float(err.max()) if y.size else 0.0,
        "mean_ulp": float(err[reg].mean()) if reg.any() else 0.0,
        "violations": int(viol.sum()),
        "special_mismatch": int(special_bad.sum()),
        "subnormal_results": int(sub.sum()),
        "subnormal_mismatch": int(sub_bad.sum()),
        "bad_idx": np.nonzero(viol | special_bad)[0][:20],
    }
    return res


def exact_compare(y, rn):
    """Bit-exact comparison (NaN as a class): number of mismatches."""
    y = np.asarray(y, dtype=np.float64)
    rn = np.asarray(rn, dtype=np.float64)
    same = (y == rn) & (np.signbit(y) == np.signbit(rn))
    same |= np.isnan(y) & np.isnan(rn)
    return int((~same).sum()), np.nonzero(~same)[0][:20]
