"""Autotuner on the GPU: a tuned launch shape is returned, recorded and used,
and results are bit-identical to the default shape."""
import numpy as np
import pytest

import workloads as W
from tests.gpu_common import to_device

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
import paper_2001_09258_amd as L  # noqa: E402


@pytest.fixture(scope="session", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    L.load()


@pytest.mark.parametrize("fn,dt", [("exp", "f64"), ("log", "f32"), ("pow", "f64"),
                                    ("tanh", "bf16")])
def test_tune_then_results_unchanged(fn, dt, tmp_path):
    n = (1 << 20) + 123
    mk = W.narrow_mixture if dt in ("bf16", "f16") else W.mixture
    a = to_device(mk(fn, dt, n, 0), dt)
    b = to_device(mk(fn, dt, n, 1), dt) if fn == "pow" else None
    L.tune_reset()
    ref = L.evaluate(fn, a, b)
    blk, pk = L.tune(fn, a, b)
    assert blk in (64, 128, 256, 512, 1024) and pk in (1, 2, 4)
    got = L.evaluate(fn, a, b)
    torch.cuda.synchronize()
    x, y = (t.float() if t.dtype in (torch.bfloat16, torch.float16) else t for t in (ref, got))
    assert torch.equal(torch.nan_to_num(x, nan=3.0), torch.nan_to_num(y, nan=3.0))
    path = tmp_path / "tune.txt"
    L.tune_save(str(path))
    text = path.read_text().strip()
    # a shape is stored only when it beat the default (256, 1) by 2%
    assert (text == "") == ((blk, pk) == (256, 1)), (blk, pk, text)
    L.tune_reset()


@pytest.mark.parametrize("fn", ["sin", "cos", "tan"])
def test_trig_shape_is_fixed(fn):
    """The gathering trig kernels keep their one launch shape."""
    a = to_device(W.mixture(fn, "f64", 4096, 0), "f64")
    assert L.tune(fn, a) == (256, 1)
