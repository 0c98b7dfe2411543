"""The Python binding rejects operands that would hand a kernel a host
pointer or an undersized buffer: every check raises before any launch.

The CPU tests cover host tensors given as the first operand; the GPU tests
mix one device tensor with a wrong second operand, upstream gradient or
output (each raises on the host, so no kernel ever runs on them)."""
import pytest
import torch

import paper_2001_09258_amd as L


CPU_CALLS = [
    ("evaluate", lambda x: L.evaluate("sin", x)),
    ("pow", lambda x: L.pow(x, x)),
    ("sincos", lambda x: L.sincos(x)),
    ("ldexp", lambda x: L.ldexp(x, torch.zeros(x.shape, dtype=torch.int32))),
    ("ilogb", lambda x: L.ilogb(x)),
    ("frexp", lambda x: L.frexp(x)),
    ("modf", lambda x: L.modf(x)),
    ("fma", lambda x: L.fma(x, x, x)),
    ("lrint", lambda x: L.lrint(x)),
    ("remquo", lambda x: L.remquo(x, x)),
    ("backward", lambda x: L.backward("sin", (x,), x)),
    ("consistent", lambda x: L.consistent("sin", x)),
]


@pytest.mark.parametrize("name,call", CPU_CALLS, ids=[c[0] for c in CPU_CALLS])
def test_host_tensor_is_rejected(name, call):
    x = torch.linspace(0.5, 2.0, 16, dtype=torch.float64)
    with pytest.raises(ValueError):
        call(x)


def _mixed_cases():
    dev = torch.device("cuda")
    x = torch.linspace(0.5, 2.0, 64, dtype=torch.float64, device=dev)
    cpu = x.cpu()
    f32 = x.float()
    short = x[:32].clone()
    i32 = torch.zeros(64, dtype=torch.int32, device=dev)
    strided = torch.empty(128, dtype=torch.float64, device=dev)[::2]
    return [
        ("pow second operand on host", lambda: L.pow(x, cpu)),
        ("pow second operand float32", lambda: L.pow(x, f32)),
        ("pow second operand shorter", lambda: L.pow(x, short)),
        ("out float32", lambda: L.sin(x, out=torch.empty_like(f32))),
        ("out on host", lambda: L.sin(x, out=torch.empty_like(cpu))),
        ("out shorter", lambda: L.sin(x, out=torch.empty_like(short))),
        ("out not contiguous", lambda: L.sin(x, out=strided)),
        ("ldexp exponent on host", lambda: L.ldexp(x, i32.cpu())),
        ("ldexp exponent int64", lambda: L.ldexp(x, i32.long())),
        ("ldexp exponent shorter", lambda: L.ldexp(x, i32[:32])),
        ("ldexp out float32", lambda: L.ldexp(x, i32, out=torch.empty_like(f32))),
        ("ldexp out on host", lambda: L.ldexp(x, i32, out=torch.empty_like(cpu))),
        ("fma b on host", lambda: L.fma(x, cpu, x)),
        ("fma c float32", lambda: L.fma(x, x, f32)),
        ("fma c shorter", lambda: L.fma(x, x, short)),
        ("remquo y on host", lambda: L.remquo(x, cpu)),
        ("remquo y float32", lambda: L.remquo(x, f32)),
        ("sincos out float32", lambda: L.sincos(x, outs=(torch.empty_like(f32),
                                                          torch.empty_like(x)))),
        ("backward gradient on host", lambda: L.backward("sin", (x,), cpu)),
        ("backward gradient shorter", lambda: L.backward("sin", (x,), short)),
        ("backward pow second input on host", lambda: L.backward("pow", (x, cpu), x)),
        ("backward out float32", lambda: L.backward("exp", (x,), x,
                                                    outs=(torch.empty_like(f32),))),
        ("consistent second operand on host", lambda: L.consistent("pow", x, cpu)),
        ("consistent out shorter", lambda: L.consistent("sin", x, out=short)),
    ]


@pytest.mark.gpu
def test_mixed_operands_are_rejected_before_launch():
    for label, call in _mixed_cases():
        with pytest.raises(ValueError):
            call()
        print("rejected:", label, flush=True)
