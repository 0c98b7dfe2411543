"""Correctly rounded CPU oracle for the elementwise math functions.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import, call or run anything in this
package.  The GPU library never uses it, and it uses nothing of the GPU
library: the two share no code, headers, tables or constant generators.

``evaluate(fn, fmt, a, b=None)`` maps numpy arrays elementwise to
``(rn, hi, lo)``: the correctly rounded result in the output format and a
binary64 pair approximating the exact value (see ``functions.evaluate1``).

Parity status of every function is listed in the module docstring of
``functions``; the pins live in ``tests/test_oracle_*.py``.

``fast32`` is a first stage in C for binary32 sin, exp and log over every
binary32 input (double-double within 2^-90, the ball code for what that
cannot decide), pinned against mpmath, the ball oracle and the host libm.
"""
from .functions import UNARY, BINARY, evaluate1, OracleError
from .batch import evaluate

__all__ = ["UNARY", "BINARY", "evaluate1", "evaluate", "OracleError"]
