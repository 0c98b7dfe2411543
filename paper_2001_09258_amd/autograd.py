"""torch.autograd.Function wrappers: forward and backward both run libm_hip
kernels (the backward ones compute g * f'(x) elementwise on the device).

    from paper_2001_09258_amd import autograd as A
    y = A.Sin.apply(x); y.sum().backward()

Inputs must be float64 or float32 device tensors (the backward kernels
exist for those); the functions save their inputs, not their outputs.
"""
import torch

from . import evaluate, backward

__all__ = ["Sin", "Cos", "Tan", "Exp", "Log", "Tanh", "Pow", "Atan2",
           "sin", "cos", "tan", "exp", "log", "tanh", "pow", "atan2"]


def _unary(fn_name):
    class F(torch.autograd.Function):
        @staticmethod
        def forward(ctx, x):
            ctx.save_for_backward(x)
            return evaluate(fn_name, x, None, "u10")

        @staticmethod
        def backward(ctx, g):
            (x,) = ctx.saved_tensors
            return backward(fn_name, (x,), g)[0]

    F.__name__ = fn_name.capitalize()
    F.__qualname__ = F.__name__
    return F


Sin = _unary("sin")
Cos = _unary("cos")
Tan = _unary("tan")
Exp = _unary("exp")
Log = _unary("log")
Tanh = _unary("tanh")


class Pow(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x, y):
        ctx.save_for_backward(x, y)
        return evaluate("pow", x, y, "u10")

    @staticmethod
    def backward(ctx, g):
        x, y = ctx.saved_tensors
        gx, gy = backward("pow", (x, y), g)
        return gx, gy


class Atan2(torch.autograd.Function):
    @staticmethod
    def forward(ctx, y, x):
        ctx.save_for_backward(y, x)
        return evaluate("atan2", y, x, "u10")

    @staticmethod
    def backward(ctx, g):
        y, x = ctx.saved_tensors
        gy, gx = backward("atan2", (y, x), g)
        return gy, gx


sin, cos, tan, exp, log, tanh = (Sin.apply, Cos.apply, Tan.apply, Exp.apply, Log.apply,
                                 Tanh.apply)
pow, atan2 = Pow.apply, Atan2.apply
