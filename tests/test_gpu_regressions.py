"""Every input of tests/golden/regressions.txt, on the GPU entry point it
names, against the oracle (same bounds as the parity tests)."""
import os

import numpy as np
import pytest

from tests.gpu_common import check

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_2001_09258_amd as L  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))


def _cases():
    out = []
    with open(os.path.join(HERE, "golden", "regressions.txt")) as fh:
        for line in fh:
            line = line.split("#", 1)[0].strip()
            if not line:
                continue
            fn, v, dt, *vals = line.split()
            out.append((fn, v, dt, [float.fromhex(x) for x in vals]))
    return out


CASES = _cases()


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    L.load()


@pytest.mark.parametrize("fn,v,dt,vals", CASES,
                         ids=["%s-%s-%s-%d" % (c[0], c[1], c[2], i) for i, c in enumerate(CASES)])
def test_regression_input(fn, v, dt, vals):
    # a few copies so the value also lands on the vector path
    a = np.full(33, vals[0])
    b = np.full(33, vals[1]) if len(vals) > 1 else None
    check(fn, v, dt, a, b, label="regression")
