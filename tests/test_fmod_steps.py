"""Step counts of the exact remainder (Section 5, "FP Remainder", Algorithm 1;
Appendix C), from the host build of the same evaluator source
(libm_hip_host_fmod_steps), on the CPU.

* The paper's worked example: 1e40 mod 0.75 = 0.25 in three long-division
  steps (the figure of Section 5).
* The paper's n/d sweep (Section 7, the fmod figure: d ~ U[1, 100], n =
  r d U[0.95, 1.05], r = 10^0, 10^0.5, ..., 10^25): every result equals the
  host C library's fmod (exact by definition), and the steps grow as the
  step function the paper describes: at most ceil(log2(n/d) / 50) + 1 (a
  digit covers at least 50 bits of the quotient; the last step may be a
  (1, 3) correction) and at least ceil(log2(n/d) / 53).
* Over the whole binary64 range (quotients up to 2^2098): at most 42 steps,
  and at most 21 — the loop bound of the paper's listing — while the
  quotient stays below 2^1024; binary32: at most 14 and 7.
"""
import math

import numpy as np
import pytest

import workloads as W
import paper_2001_09258_amd as L


@pytest.fixture(scope="module", autouse=True)
def _lib():
    try:
        L.load_host()
    except L.LibmHipError as e:
        pytest.fail(str(e))


def test_worked_example_three_steps():
    r, s = L.host_fmod_steps(np.array([1e40]), np.array([0.75]))
    assert r[0] == 0.25 and s[0] == 3


@pytest.mark.parametrize("e2", range(0, 51))
def test_paper_ratio_sweep(e2):
    e = e2 / 2.0
    rng = np.random.default_rng(1000 + e2)
    n = 4000
    d = rng.uniform(1.0, 100.0, n)
    x = 10.0 ** e * d * rng.uniform(0.95, 1.05, n)
    r, s = L.host_fmod_steps(x, d)
    assert np.array_equal(r, np.fmod(x, d))
    q = np.log2(x / d)
    big = q > 0
    assert (s[big] <= np.ceil(q[big] / 50.0) + 1).all(), (e, s.max())
    assert (s[big] >= np.ceil(q[big] / 53.0)).all(), (e, s.min())
    assert (s[~big] == 0).all()


@pytest.mark.parametrize("dt,cap,cap_in_range,emax", [("f64", 42, 21, 1024), ("f32", 14, 7, 128)])
def test_whole_range_step_bounds(dt, cap, cap_in_range, emax):
    npd = np.float64 if dt == "f64" else np.float32
    x = W.large_args("fmod", dt, 1 << 18, 0).astype(npd)
    y = W.large_args("fmod", dt, 1 << 18, 1).astype(npd)
    r, s = L.host_fmod_steps(x, y)
    assert np.array_equal(r.view(np.uint64 if dt == "f64" else np.uint32),
                          np.fmod(x, y).view(np.uint64 if dt == "f64" else np.uint32))
    q = np.log2(np.abs(x.astype(np.float64))) - np.log2(np.abs(y.astype(np.float64)))
    assert s.max() <= cap
    assert s[q < emax].max() <= cap_in_range
    p = 50.0 if dt == "f64" else 21.0
    big = q > 0
    assert (s[big] <= np.ceil(q[big] / p) + 1).all()
