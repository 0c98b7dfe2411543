"""Array front end of the oracle: elementwise evaluation over a process pool.

Test infrastructure only.  Workers are started with the 'spawn' method (a
fresh interpreter, never a fork of a process that may hold GPU state) and
touch no GPU.
"""
import multiprocessing as mp
import os
import sys

import numpy as np

from .functions import evaluate1

__all__ = ["evaluate", "default_workers", "shutdown"]

_pool = None
_pool_size = 0


def default_workers():
    """Worker processes: the CPUs this process may run on, at most 16."""
    try:
        n = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def shutdown():
    """Terminate and join the worker pool (if one was started)."""
    global _pool, _pool_size
    if _pool is not None:
        _pool.terminate()
        _pool.join()
    _pool = None
    _pool_size = 0


def _chunk(args):
    fn, fmt, a, b = args
    out = np.empty((3, len(a)), dtype=np.float64)
    if b is None:
        for i, x in enumerate(a.tolist()):
            out[:, i] = evaluate1(fn, fmt, x)
    else:
        for i, (x, y) in enumerate(zip(a.tolist(), b.tolist())):
            out[:, i] = evaluate1(fn, fmt, x, y)
    return out


def _get_pool(workers):
    global _pool, _pool_size
    if _pool is None or _pool_size != workers:
        if _pool is not None:
            _pool.terminate()
        # The workers only need this module.  Hide the main script from the
        # spawn bootstrap so that scripts without a __main__ guard are not
        # re-executed in every worker.
        main = sys.modules.get("__main__")
        saved = {}
        for attr in ("__file__", "__spec__"):
            if main is not None and hasattr(main, attr):
                saved[attr] = getattr(main, attr)
                setattr(main, attr, None)
        try:
            _pool = mp.get_context("spawn").Pool(workers)
        finally:
            for attr, v in saved.items():
                setattr(main, attr, v)
        _pool_size = workers
    return _pool


def evaluate(fn, fmt, a, b=None, workers=None, serial_below=256):
    """Correctly rounded fn over numpy arrays ``a`` (and ``b``).

    Inputs may be float64/float32/float16 arrays or bfloat16 values already
    widened to float32; every value is converted exactly to a Python float.
    Returns three float64 arrays (rn, hi, lo)."""
    a = np.asarray(a).astype(np.float64).ravel()
    if b is not None:
        b = np.asarray(b).astype(np.float64).ravel()
        assert b.shape == a.shape
    n = a.shape[0]
    if workers is None:
        workers = default_workers()
    if n < serial_below or workers <= 1:
        out = _chunk((fn, fmt, a, b))
    else:
        nchunks = min(n, workers * 8)
        bounds = np.linspace(0, n, nchunks + 1).astype(np.int64)
        jobs = [(fn, fmt, a[s:e], None if b is None else b[s:e])
                for s, e in zip(bounds[:-1], bounds[1:]) if e > s]
        parts = _get_pool(workers).map(_chunk, jobs)
        out = np.concatenate(parts, axis=1)
    return out[0], out[1], out[2]


def _grad_chunk(args):
    fn, fmt, a, b, g = args
    from .derivatives import grad1, grad_pow, grad_atan2
    k = 1 if b is None else 2
    out = np.empty((k, 3, len(a)), dtype=np.float64)
    for i in range(len(a)):
        if b is None:
            out[0, :, i] = grad1(fn, fmt, float(a[i]), float(g[i]))
        else:
            f = grad_pow if fn == "pow" else grad_atan2
            r0, r1 = f(fmt, float(a[i]), float(b[i]), float(g[i]))
            out[0, :, i] = r0
            out[1, :, i] = r1
    return out


def evaluate_grad(fn, fmt, a, g, b=None, workers=None):
    """Correctly rounded g * f'(x) (unary) or both partials of pow(a, b) /
    atan2(a, b) times g.  Returns a list of (rn, hi, lo) triples."""
    a = np.asarray(a, dtype=np.float64).ravel()
    g = np.asarray(g, dtype=np.float64).ravel()
    b = None if b is None else np.asarray(b, dtype=np.float64).ravel()
    n = a.shape[0]
    workers = workers or default_workers()
    nchunks = max(1, min(n, workers * 8))
    bounds = np.linspace(0, n, nchunks + 1).astype(np.int64)
    jobs = [(fn, fmt, a[s:e], None if b is None else b[s:e], g[s:e])
            for s, e in zip(bounds[:-1], bounds[1:]) if e > s]
    if n < 256 or workers <= 1:
        parts = [_grad_chunk(j) for j in jobs]
    else:
        parts = _get_pool(workers).map(_grad_chunk, jobs)
    out = np.concatenate(parts, axis=2)
    return [(out[k, 0], out[k, 1], out[k, 2]) for k in range(out.shape[0])]
