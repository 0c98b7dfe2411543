"""Arguments that stress the binary64 trig reductions.

* For every k with |k pi/2| < 2^14: the double nearest to k pi/2 and its two
  neighbours, with both signs.  These are the smallest reduced arguments the
  Cody-Waite reduction meets below 2^14 (the smallest, about 2^-60.5, at the
  double nearest to 29 pi/2), so they expose any piece of pi/2 or pi that is
  short of bits.  The binary32 set does the same below 65536 (smallest
  about 2^-27.8, at the float nearest to 161 pi/2).
* Log-uniform magnitudes in [2^14, 1e14] with random signs: the Payne-Hanek
  range whose table rows start with leading zeros, plus the boundaries.

pi/2 comes from mpmath at 200 bits (input generation only; the expected
values come from the oracle).
"""
import math

import numpy as np


def near_multiples(dt="f64"):
    """binary64: below 2^14 (the binary64 Cody-Waite range); binary32: below
    65536 (the binary32 one), neighbours taken in binary32."""
    import mpmath as mp
    limit = 2.0 ** 14 if dt == "f64" else 65536.0
    with mp.workprec(200):
        pih = mp.pi / 2
        pts = []
        for k in range(1, int(limit / float(pih)) + 2):
            if dt == "f64":
                x = float(k * pih)
                near = (math.nextafter(x, 0.0), x, math.nextafter(x, math.inf))
            else:
                x = np.float32(float(k * pih))
                near = [float(v) for v in (np.nextafter(x, np.float32(0)), x,
                                           np.nextafter(x, np.float32(np.inf)))]
            for v in near:
                if v < limit:
                    pts += [v, -v]
    return np.array(pts)


def mid_range(n, seed=2014):
    rng = np.random.default_rng(seed)
    mag = np.exp(rng.uniform(math.log(2.0 ** 14), math.log(1e14), n))
    edges = [2.0 ** 14, math.nextafter(2.0 ** 14, 0.0), 1e14, math.nextafter(1e14, 0.0),
             2.0 ** 52, 2.0 ** 52 + 0.5, 2.0 ** 53]
    x = np.concatenate([mag * np.where(rng.random(n) < 0.5, -1.0, 1.0), edges,
                        [-e for e in edges]])
    return x
