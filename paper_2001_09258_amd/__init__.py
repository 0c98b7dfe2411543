"""Python binding of libm_hip (argument marshalling only).

Every computation runs in the HIP kernels of ``libm_hip.so`` (built from
``csrc/`` by ``paper_2001_09258_amd.build``).  PyTorch supplies device memory
and the current stream; nothing here evaluates a math function, and there is
no CPU fallback: if the shared library is missing, every call raises.

Two layers:

* ``libm_hip_<fn>_<variant>_<dtype>(a_ptr, [b_ptr,] out_ptr, n, stream)`` --
  one Python callable per C-ABI entry point, same name and argument order
  (pointers and the stream as integers), returning the status code;
* ``sin(x, variant="u10")``, ``pow(x, y)``, ``atan2(y, x)``, ... -- torch
  front ends: contiguous device tensors of float64 / float32 / bfloat16 /
  float16 in, a new tensor (or ``out=``) back, enqueued on the current stream.
"""
import ctypes
import os

__all__ = ["load", "library_path", "UNARY", "BINARY", "VARIANTS", "entry_name",
           "call", "evaluate", "sin", "cos", "tan", "exp", "exp2", "log", "log2",
           "sinh", "cosh", "tanh", "asin", "acos", "atan", "log10", "log1p", "exp10",
           "expm1", "cbrt", "asinh", "acosh", "atanh", "erf", "erfc", "lgamma", "tgamma",
           "sincos", "pow", "atan2",
           "hypot", "fmod", "remainder", "fdim", "fmax", "fmin", "copysign", "nextafter",
           "sqrt", "trunc", "floor", "ceil", "rint", "fabs", "logb",
           "consistent", "host_consistent", "LibmHipError"]

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIBNAME = "libm_hip.so"

UNARY = ("sin", "cos", "tan", "exp", "exp2", "log", "log2", "sinh", "cosh", "tanh",
         "asin", "acos", "atan", "log10", "log1p", "exp10", "expm1", "cbrt", "asinh",
         "acosh", "atanh", "erf", "erfc", "lgamma", "tgamma", "sqrt", "trunc", "floor", "ceil",
         "round", "rint",
         "fabs", "logb")
BINARY = ("pow", "atan2", "hypot", "fmod", "remainder", "fdim", "fmax", "fmin", "copysign",
          "nextafter")
EXACT = ("fmod", "remainder", "fdim", "fmax", "fmin", "copysign", "nextafter", "sqrt", "trunc",
         "floor", "ceil", "round", "rint", "fabs", "logb")
# accuracy variants served per function
VARIANTS = {fn: ("exact",) if fn in EXACT else ("u10",) for fn in UNARY + BINARY}
VARIANTS.update({"sin": ("u10", "u35"), "cos": ("u10", "u35"), "tan": ("u10", "u35"),
                 "asin": ("u10", "u35"), "acos": ("u10", "u35"), "atan": ("u10", "u35"),
                 "log": ("u10", "u35"), "atan2": ("u10", "u35"), "sinh": ("u10", "u35"),
                 "pow": ("u10", "u35"),
                 "cosh": ("u10", "u35"), "tanh": ("u10", "u35"),
                 "fmod": ("exact",), "remainder": ("exact",), "fdim": ("exact",),
                 "fmax": ("exact",), "fmin": ("exact",)})
DTYPES = ("f64", "f32", "bf16", "f16", "f32_via_f64")


class LibmHipError(RuntimeError):
    pass


def library_path():
    return os.path.join(_HERE, _LIBNAME)


def entry_name(fn, variant, dtype):
    if fn in EXACT:
        return "libm_hip_%s_%s" % (fn, dtype)
    return "libm_hip_%s_%s_%s" % (fn, variant, dtype)


def served(fn, variant, dtype):
    """True if the library exports this combination."""
    if variant not in VARIANTS.get(fn, ()):
        return False
    if fn in EXACT:
        return dtype in ("f64", "f32")
    if variant == "u35":
        return dtype in ("f64", "f32")
    return dtype in DTYPES


BWD_UNARY = ("sin", "cos", "tan", "exp", "log", "tanh")
BWD_BINARY = ("pow", "atan2")


def bwd_entry_points():
    """(fn, dtype, name) of every backward entry point."""
    return [(fn, dt, "libm_hip_%s_u10_%s_bwd" % (fn, dt))
            for fn in BWD_UNARY + BWD_BINARY for dt in ("f64", "f32")]


def sincos_entry_points():
    """(variant, dtype, symbol) of every sincos entry point."""
    return [(v, dt, "libm_hip_sincos_%s_%s" % (v, dt))
            for v in ("u10", "u35") for dt in DTYPES if served("sin", v, dt)]


def all_entry_points():
    out = []
    for fn in UNARY + BINARY:
        for v in VARIANTS[fn]:
            for dt in DTYPES:
                if served(fn, v, dt):
                    out.append((fn, v, dt, entry_name(fn, v, dt)))
    return out


_lib = None


def load():
    """Load libm_hip.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    path = library_path()
    if not os.path.exists(path):
        raise LibmHipError("libm_hip.so not found at %s; run "
                           "python -m paper_2001_09258_amd.build" % path)
    lib = ctypes.CDLL(path)
    lib.libm_hip_last_error.restype = ctypes.c_char_p
    lib.libm_hip_version.restype = ctypes.c_char_p
    vp, sz = ctypes.c_void_p, ctypes.c_size_t
    for fn, v, dt, name in all_entry_points():
        f = getattr(lib, name)
        f.restype = ctypes.c_int
        if fn in UNARY:
            f.argtypes = [vp, vp, sz, vp]
        else:
            f.argtypes = [vp, vp, vp, sz, vp]
    for v, dt, name in sincos_entry_points():
        f = getattr(lib, name)
        f.restype = ctypes.c_int
        f.argtypes = [vp, vp, vp, sz, vp]
    for fn, dt, name in bwd_entry_points():
        f = getattr(lib, name)
        f.restype = ctypes.c_int
        f.argtypes = [vp, vp, vp, sz, vp] if fn in BWD_UNARY else [vp, vp, vp, vp, vp, sz, vp]
    lib.libm_hip_eval.restype = ctypes.c_int
    for nm in ("libm_hip_ldexp_f64", "libm_hip_ldexp_f32", "libm_hip_frexp_f64",
               "libm_hip_frexp_f32"):
        getattr(lib, nm).restype = ctypes.c_int
        getattr(lib, nm).argtypes = [vp, vp, vp, sz, vp]
    for nm in ("libm_hip_ilogb_f64", "libm_hip_ilogb_f32"):
        getattr(lib, nm).restype = ctypes.c_int
        getattr(lib, nm).argtypes = [vp, vp, sz, vp]
    lib.libm_hip_consistent_eval.restype = ctypes.c_int
    lib.libm_hip_consistent_eval.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, vp, vp,
                                             vp, sz, vp]
    lib.libm_hip_eval.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, vp, vp, vp, sz, vp]
    _lib = lib
    return lib


def _check(status, name):
    if status != 0:
        msg = load().libm_hip_last_error().decode()
        raise LibmHipError("%s failed with status %d: %s" % (name, status, msg))


def _make_raw(name):
    def raw(*args):
        return getattr(load(), name)(*args)
    raw.__name__ = name
    raw.__doc__ = "Direct call of the C-ABI entry point %s (pointers as ints)." % name
    return raw


for _fn, _v, _dt, _name in all_entry_points():
    globals()[_name] = _make_raw(_name)
    __all__.append(_name)
for _fn, _dt, _name in bwd_entry_points():
    globals()[_name] = _make_raw(_name)
    __all__.append(_name)


def call(fn, variant, dtype, a_ptr, b_ptr, out_ptr, n, stream=0):
    """Call one entry point with raw device pointers; raises on error."""
    name = entry_name(fn, variant, dtype)
    f = getattr(load(), name)
    if fn in UNARY:
        st = f(a_ptr, out_ptr, n, stream)
    else:
        st = f(a_ptr, b_ptr, out_ptr, n, stream)
    _check(st, name)


# ---------------------------------------------------------------------------
# torch front ends
# ---------------------------------------------------------------------------
def _dtype_tag(t, via_f64):
    import torch
    tag = {torch.float64: "f64", torch.float32: "f32", torch.bfloat16: "bf16",
           torch.float16: "f16"}.get(t.dtype)
    if tag is None:
        raise TypeError("unsupported dtype %s" % t.dtype)
    if via_f64:
        if tag != "f32":
            raise TypeError("via_f64 applies to float32 tensors only")
        tag = "f32_via_f64"
    return tag


def _stream_handle():
    import torch
    return torch.cuda.current_stream().cuda_stream


def _operand(t, ref, what, dtype=None):
    """Check that ``t`` is a device tensor on ``ref``'s device with ``ref``'s
    shape and the given dtype (``ref``'s by default); returns it contiguous.
    Raises before anything reaches a kernel."""
    import torch
    if not isinstance(t, torch.Tensor):
        raise TypeError("%s must be a tensor" % what)
    if not t.is_cuda or t.device != ref.device:
        raise ValueError("%s must be a device tensor on %s" % (what, ref.device))
    if t.shape != ref.shape:
        raise ValueError("%s has shape %s, expected %s" % (what, tuple(t.shape),
                                                            tuple(ref.shape)))
    want = ref.dtype if dtype is None else dtype
    if t.dtype != want:
        raise ValueError("%s has dtype %s, expected %s" % (what, t.dtype, want))
    return t.contiguous()


def _output(t, ref, what, dtype=None):
    """As ``_operand`` for a caller-supplied output, which must already be
    contiguous (a copy would not be written back); None allocates one."""
    import torch
    if t is None:
        return torch.empty(ref.shape, dtype=ref.dtype if dtype is None else dtype,
                           device=ref.device)
    _operand(t, ref, what, dtype)
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % what)
    return t


def _device_input(a):
    import torch
    if not isinstance(a, torch.Tensor) or not a.is_cuda:
        raise ValueError("libm_hip evaluates device tensors only")
    return a.contiguous()


def evaluate(fn, a, b=None, variant=None, out=None, via_f64=False):
    """fn over device tensors (C argument order for binary functions)."""
    import torch
    load()
    if variant is None:
        variant = VARIANTS[fn][0]
    a = _device_input(a)
    if fn in BINARY:
        if b is None:
            raise ValueError("%s needs two tensors" % fn)
        b = _operand(b, a, "second operand")
    tag = _dtype_tag(a, via_f64)
    if not served(fn, variant, tag):
        raise ValueError("%s %s is not served for %s" % (fn, variant, tag))
    out = _output(out, a, "out")
    with torch.cuda.device(a.device):
        call(fn, variant, tag, a.data_ptr(), 0 if b is None else b.data_ptr(),
             out.data_ptr(), a.numel(), _stream_handle())
    return out


def _unary(fn):
    def f(x, variant="u10", out=None, via_f64=False):
        return evaluate(fn, x, None, variant, out, via_f64)
    f.__name__ = fn
    f.__doc__ = "Elementwise %s on a device tensor (variant 'u10' or 'u35')." % fn
    return f


sin, cos, tan = _unary("sin"), _unary("cos"), _unary("tan")
exp, exp2, log, log2 = _unary("exp"), _unary("exp2"), _unary("log"), _unary("log2")
sinh, cosh, tanh = _unary("sinh"), _unary("cosh"), _unary("tanh")
asin, acos, atan = _unary("asin"), _unary("acos"), _unary("atan")
log10, log1p, exp10 = _unary("log10"), _unary("log1p"), _unary("exp10")
expm1, cbrt = _unary("expm1"), _unary("cbrt")
asinh, acosh, atanh = _unary("asinh"), _unary("acosh"), _unary("atanh")
erf, erfc = _unary("erf"), _unary("erfc")
lgamma, tgamma = _unary("lgamma"), _unary("tgamma")


def _exact1(fn):
    def f(x, out=None):
        return evaluate(fn, x, None, "exact", out)
    f.__name__ = fn
    f.__doc__ = "Elementwise C %s on a float64/float32 device tensor (exact result)." % fn
    return f


sqrt, trunc, floor, ceil = _exact1("sqrt"), _exact1("trunc"), _exact1("floor"), _exact1("ceil")
round, rint, fabs, logb = _exact1("round"), _exact1("rint"), _exact1("fabs"), _exact1("logb")


def sincos(x, variant="u10", outs=None, via_f64=False):
    """(sin x, cos x) elementwise in one pass, each bit-identical to sin and
    cos of the same variant."""
    import torch
    x = _device_input(x)
    tag = _dtype_tag(x, via_f64)
    if not served("sin", variant, tag):
        raise LibmHipError("sincos: %s %s is not served" % (variant, tag))
    s, c = (None, None) if outs is None else outs
    s, c = _output(s, x, "sin output"), _output(c, x, "cos output")
    name = "libm_hip_sincos_%s_%s" % (variant, tag)
    lib = load()
    with torch.cuda.device(x.device):
        _check(getattr(lib, name)(x.data_ptr(), s.data_ptr(), c.data_ptr(), x.numel(),
                                  _stream_handle()), name)
    return s, c


def pow(x, y, out=None, via_f64=False):
    """x ** y elementwise (C pow semantics, 1-ULP)."""
    return evaluate("pow", x, y, "u10", out, via_f64)


def atan2(y, x, variant="u10", out=None, via_f64=False):
    """atan2(y, x) elementwise (C semantics; variant 'u10' or 'u35')."""
    return evaluate("atan2", y, x, variant, out, via_f64)


def hypot(x, y, out=None, via_f64=False):
    """sqrt(x^2 + y^2) elementwise without spurious overflow (C semantics, 1-ULP)."""
    return evaluate("hypot", x, y, "u10", out, via_f64)


def fmod(x, y, out=None):
    """Exact C fmod(x, y) elementwise."""
    return evaluate("fmod", x, y, "exact", out)


def remainder(x, y, out=None):
    """Exact IEEE remainder(x, y) elementwise."""
    return evaluate("remainder", x, y, "exact", out)


def fdim(x, y, out=None):
    """C fdim(x, y) elementwise: x - y if x > y, else +0."""
    return evaluate("fdim", x, y, "exact", out)


def fmax(x, y, out=None):
    """C fmax(x, y) elementwise (NaN-ignoring; -0 below +0)."""
    return evaluate("fmax", x, y, "exact", out)


def fmin(x, y, out=None):
    """C fmin(x, y) elementwise (NaN-ignoring; -0 below +0)."""
    return evaluate("fmin", x, y, "exact", out)


def copysign(x, y, out=None):
    """C copysign(x, y) elementwise."""
    return evaluate("copysign", x, y, "exact", out)


def nextafter(x, y, out=None):
    """C nextafter(x, y) elementwise."""
    return evaluate("nextafter", x, y, "exact", out)


def backward(fn, inputs, gout, outs=None):
    """Raw backward call: ``inputs`` are the saved forward inputs (C order),
    ``gout`` the upstream gradient; returns the input gradient(s)."""
    import torch
    load()
    x0 = _device_input(inputs[0])
    tag = _dtype_tag(x0, False)
    if tag not in ("f64", "f32"):
        raise TypeError("backward kernels take float64 or float32")
    name = "libm_hip_%s_u10_%s_bwd" % (fn, tag)
    f = getattr(load(), name)
    k = 1 if fn in BWD_UNARY else 2
    if len(inputs) != k:
        raise ValueError("%s backward takes %d saved input(s)" % (fn, k))
    ins = [x0] + [_operand(t, x0, "saved input %d" % i) for i, t in enumerate(inputs[1:], 1)]
    g = _operand(gout, x0, "upstream gradient")
    n = ins[0].numel()
    outs = (None,) * k if outs is None else tuple(outs)
    if len(outs) != k:
        raise ValueError("%s backward writes %d gradient(s)" % (fn, k))
    with torch.cuda.device(ins[0].device):
        if fn in BWD_UNARY:
            gx = _output(outs[0], x0, "gradient output")
            _check(f(ins[0].data_ptr(), g.data_ptr(), gx.data_ptr(), n, _stream_handle()), name)
            return (gx,)
        g0 = _output(outs[0], x0, "gradient output 0")
        g1 = _output(outs[1], x0, "gradient output 1")
        _check(f(ins[0].data_ptr(), ins[1].data_ptr(), g.data_ptr(), g0.data_ptr(),
                 g1.data_ptr(), n, _stream_handle()), name)
        return (g0, g1)


# ---------------------------------------------------------------------------
# batched evaluation (one persistent kernel per run, hip-graph replayed)
# ---------------------------------------------------------------------------
FN_CODES = {"sin": 0, "cos": 1, "tan": 2, "exp": 3, "exp2": 4, "log": 5, "log2": 6,
            "pow": 7, "atan2": 8, "sinh": 9, "cosh": 10, "tanh": 11, "fmod": 12,
            "remainder": 13, "asin": 14, "acos": 15, "atan": 16, "log10": 17,
            "log1p": 18, "exp10": 19, "expm1": 20, "cbrt": 21, "hypot": 22, "asinh": 23,
            "acosh": 24, "atanh": 25, "erf": 26, "erfc": 27, "fdim": 28, "fmax": 29,
            "fmin": 30, "sqrt": 31, "trunc": 32, "floor": 33, "ceil": 34, "round": 35,
            "rint": 36, "fabs": 37, "logb": 38, "copysign": 39, "nextafter": 40,
            "lgamma": 41, "tgamma": 42}
VARIANT_CODES = {"u10": 0, "u35": 1, "exact": 2}
DTYPE_CODES = {"f64": 0, "f32": 1, "bf16": 2, "f16": 3, "f32_via_f64": 4}


class Request(ctypes.Structure):
    """Mirror of the C struct libm_hip_request."""
    _fields_ = [("fn", ctypes.c_int), ("variant", ctypes.c_int), ("dtype", ctypes.c_int),
                ("reserved", ctypes.c_int), ("a", ctypes.c_void_p), ("b", ctypes.c_void_p),
                ("out", ctypes.c_void_p), ("n", ctypes.c_size_t)]


def _batch_lib():
    lib = load()
    if not getattr(lib, "_batch_ready", False):
        lib.libm_hip_batch_plan_create.restype = ctypes.c_int
        lib.libm_hip_batch_plan_create.argtypes = [ctypes.POINTER(ctypes.c_void_p), ctypes.c_int,
                                                   ctypes.c_int]
        lib.libm_hip_batch_run.restype = ctypes.c_int
        lib.libm_hip_batch_run.argtypes = [ctypes.c_void_p, ctypes.POINTER(Request), ctypes.c_int,
                                           ctypes.c_void_p]
        lib.libm_hip_batch_run_noalloc.restype = ctypes.c_int
        lib.libm_hip_batch_run_noalloc.argtypes = [ctypes.POINTER(Request), ctypes.c_int,
                                                   ctypes.c_void_p]
        lib.libm_hip_batch_plan_set_graph.restype = ctypes.c_int
        lib.libm_hip_batch_plan_set_graph.argtypes = [ctypes.c_void_p, ctypes.c_int]
        lib.libm_hip_batch_plan_destroy.restype = None
        lib.libm_hip_batch_plan_destroy.argtypes = [ctypes.c_void_p]
        lib.libm_hip_batch_last_error.restype = ctypes.c_char_p
        lib._batch_ready = True
    return lib


class BatchPlan:
    """A libm_hip batch plan: ``run([(fn, variant, dtype, a, b, out), ...])``
    with device tensors (``b`` None for unary functions); enqueued on the
    current stream."""

    def __init__(self, max_requests=64, use_graph=True, device=-1):
        lib = _batch_lib()
        h = ctypes.c_void_p()
        st = lib.libm_hip_batch_plan_create(ctypes.byref(h), max_requests, device)
        if st != 0:
            raise LibmHipError("batch_plan_create failed (%d): %s"
                               % (st, lib.libm_hip_last_error().decode()))
        self._h = h
        if not use_graph:
            _check(lib.libm_hip_batch_plan_set_graph(h, 0), "libm_hip_batch_plan_set_graph")
        self.max_requests = max_requests

    def run(self, requests, stream=None):
        lib = _batch_lib()
        arr = (Request * max(1, len(requests)))()
        for i, (fn, v, dt, a, b, out) in enumerate(requests):
            arr[i] = Request(FN_CODES[fn], VARIANT_CODES[v], DTYPE_CODES[dt], 0,
                             a.data_ptr(), 0 if b is None else b.data_ptr(), out.data_ptr(),
                             a.numel())
        st = lib.libm_hip_batch_run(self._h, arr, len(requests),
                                    _stream_handle() if stream is None else stream)
        if st != 0:
            raise LibmHipError("batch_run failed (%d): %s"
                               % (st, lib.libm_hip_last_error().decode()))

    def run_raw(self, arr, k, stream):
        """Run a prepared ctypes Request array (no Python-side marshalling)."""
        return _batch_lib().libm_hip_batch_run(self._h, arr, k, stream)

    def close(self):
        if self._h:
            _batch_lib().libm_hip_batch_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def request_array(requests):
    """A ctypes libm_hip_request array from (fn, variant, dtype, a, b, out)
    tuples of device tensors (b None for unary functions)."""
    arr = (Request * max(1, len(requests)))()
    for i, (fn, v, dt, a, b, out) in enumerate(requests):
        arr[i] = Request(FN_CODES[fn], VARIANT_CODES[v], DTYPE_CODES[dt], 0, a.data_ptr(),
                         0 if b is None else b.data_ptr(), out.data_ptr(), a.numel())
    return arr


def batch_run_noalloc(requests, stream=None):
    """libm_hip_batch_run_noalloc over (fn, variant, dtype, a, b, out) tuples
    of device tensors, on the current stream; allocates nothing on the
    device."""
    lib = _batch_lib()
    st = lib.libm_hip_batch_run_noalloc(request_array(requests), len(requests),
                                        _stream_handle() if stream is None else stream)
    if st != 0:
        raise LibmHipError("batch_run_noalloc failed (%d): %s"
                           % (st, lib.libm_hip_last_error().decode()))


# ---------------------------------------------------------------------------
# launch-shape autotuner
# ---------------------------------------------------------------------------
def _tune_lib():
    lib = load()
    if not getattr(lib, "_tune_ready", False):
        vp = ctypes.c_void_p
        lib.libm_hip_tune.restype = ctypes.c_int
        lib.libm_hip_tune.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, vp, vp, vp,
                                      ctypes.c_size_t, vp, ctypes.POINTER(ctypes.c_int),
                                      ctypes.POINTER(ctypes.c_int)]
        lib.libm_hip_tune_save.restype = ctypes.c_int
        lib.libm_hip_tune_save.argtypes = [ctypes.c_char_p]
        lib.libm_hip_tune_load.restype = ctypes.c_int
        lib.libm_hip_tune_load.argtypes = [ctypes.c_char_p]
        lib.libm_hip_tune_reset.restype = None
        lib.libm_hip_tune_reset.argtypes = []
        lib._tune_ready = True
    return lib


def tune(fn, a, b=None, variant=None, out=None, via_f64=False):
    """Autotune the launch shape of ``fn`` for tensors like ``a`` (the
    buffers are used for timing); returns (workgroup size, packs per lane)."""
    import torch
    lib = _tune_lib()
    variant = variant or VARIANTS[fn][0]
    a = _device_input(a)
    if fn in BINARY:
        if b is None:
            raise ValueError("%s needs two tensors" % fn)
        b = _operand(b, a, "second operand")
    tag = _dtype_tag(a, via_f64)
    out = _output(out, a, "out")
    blk, pk = ctypes.c_int(0), ctypes.c_int(0)
    st = lib.libm_hip_tune(FN_CODES[fn], VARIANT_CODES[variant], DTYPE_CODES[tag], a.data_ptr(),
                           None if b is None else b.data_ptr(), out.data_ptr(), a.numel(),
                           _stream_handle(), ctypes.byref(blk), ctypes.byref(pk))
    _check(st, "libm_hip_tune")
    return blk.value, pk.value


def tune_save(path):
    _check(_tune_lib().libm_hip_tune_save(os.fsencode(path)), "libm_hip_tune_save")


def tune_load(path):
    _check(_tune_lib().libm_hip_tune_load(os.fsencode(path)), "libm_hip_tune_load")


def tune_reset():
    _tune_lib().libm_hip_tune_reset()


# ---------------------------------------------------------------------------
# bit-consistent form: libm_hip_consistent_eval on the GPU and the host build
# of the same evaluators (libm_hip_host.so), whose results are bit-identical
# ---------------------------------------------------------------------------
_HOSTLIB = "libm_hip_host.so"
_host = None


def host_library_path():
    return os.path.join(_HERE, _HOSTLIB)


def load_host():
    """Load libm_hip_host.so (raises if it has not been built)."""
    global _host
    if _host is not None:
        return _host
    path = host_library_path()
    if not os.path.exists(path):
        raise LibmHipError("libm_hip_host.so not found at %s; run "
                           "python -m paper_2001_09258_amd.build" % path)
    lib = ctypes.CDLL(path)
    vp = ctypes.c_void_p
    lib.libm_hip_host_eval.restype = ctypes.c_int
    lib.libm_hip_host_eval.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, vp, vp, vp,
                                       ctypes.c_size_t]
    lib.libm_hip_host_fmod_steps.restype = ctypes.c_int
    lib.libm_hip_host_fmod_steps.argtypes = [ctypes.c_int, vp, vp, vp, vp, ctypes.c_size_t]
    _host = lib
    return lib


def host_fmod_steps(x, y):
    """fmod over float64/float32 numpy arrays on the host (the bit-consistent
    build) and the number of long-division digit steps of each element."""
    import numpy as np
    lib = load_host()
    x = np.ascontiguousarray(x)
    tag = {np.dtype(np.float64): "f64", np.dtype(np.float32): "f32"}.get(x.dtype)
    if tag is None:
        raise TypeError("fmod steps take float64 or float32")
    y = np.ascontiguousarray(y, dtype=x.dtype)
    if y.shape != x.shape:
        raise ValueError("fmod needs two arrays of equal shape")
    out = np.empty_like(x)
    steps = np.empty(x.shape, dtype=np.int32)
    st = lib.libm_hip_host_fmod_steps(DTYPE_CODES[tag], x.ctypes.data, y.ctypes.data,
                                      out.ctypes.data, steps.ctypes.data, x.size)
    if st != 0:
        raise LibmHipError("libm_hip_host_fmod_steps failed with status %d" % st)
    return out, steps


def _consistent_args(fn, variant):
    if fn not in FN_CODES or fn in ("sincos",):
        raise ValueError("unknown function %s" % fn)
    if variant is None:
        variant = VARIANTS[fn][0]
    if variant not in VARIANTS[fn]:
        raise ValueError("%s has no variant %s" % (fn, variant))
    return FN_CODES[fn], VARIANT_CODES[variant]


def consistent(fn, a, b=None, variant=None, out=None):
    """fn over float64/float32 device tensors in the bit-consistent form (the
    same bits as ``host_consistent`` on the host)."""
    import torch
    lib = load()
    f, v = _consistent_args(fn, variant)
    a = _device_input(a)
    tag = {torch.float64: "f64", torch.float32: "f32"}.get(a.dtype)
    if tag is None:
        raise TypeError("the bit-consistent form takes float64 or float32")
    if fn in BINARY:
        if b is None:
            raise ValueError("%s needs two tensors" % fn)
        b = _operand(b, a, "second operand")
    out = _output(out, a, "out")
    with torch.cuda.device(a.device):
        st = lib.libm_hip_consistent_eval(f, v, DTYPE_CODES[tag], a.data_ptr(),
                                          None if b is None else b.data_ptr(), out.data_ptr(),
                                          a.numel(), _stream_handle())
    _check(st, "libm_hip_consistent_eval")
    return out


def host_consistent(fn, a, b=None, variant=None):
    """fn over float64/float32 numpy arrays on the host, bit-identical to
    ``consistent`` on the GPU (the host build of the same evaluators)."""
    import numpy as np
    lib = load_host()
    f, v = _consistent_args(fn, variant)
    a = np.ascontiguousarray(a)
    tag = {np.dtype(np.float64): "f64", np.dtype(np.float32): "f32"}.get(a.dtype)
    if tag is None:
        raise TypeError("the bit-consistent form takes float64 or float32")
    if fn in BINARY:
        b = np.ascontiguousarray(b, dtype=a.dtype)
        if b.shape != a.shape:
            raise ValueError("binary functions need two arrays of equal shape")
    out = np.empty_like(a)
    st = lib.libm_hip_host_eval(f, v, DTYPE_CODES[tag], a.ctypes.data,
                                None if b is None else b.ctypes.data, out.ctypes.data, a.size)
    if st != 0:
        raise LibmHipError("libm_hip_host_eval failed with status %d" % st)
    return out


# ---------------------------------------------------------------------------
# integer-operand functions (C99 7.12.6): ldexp, ilogb, frexp
# ---------------------------------------------------------------------------
def _fp_tag(a):
    import torch
    if not isinstance(a, torch.Tensor) or not a.is_cuda:
        raise ValueError("expects a float64 or float32 device tensor")
    tag = {torch.float64: "f64", torch.float32: "f32"}.get(a.dtype)
    if tag is None:
        raise TypeError("expects a float64 or float32 device tensor")
    return tag


def ldexp(x, e, out=None):
    """x * 2^e elementwise (e an int32 device tensor of x's shape)."""
    import torch
    lib = load()
    tag = _fp_tag(x)
    x = x.contiguous()
    e = _operand(e, x, "exponent tensor", torch.int32)
    out = _output(out, x, "out")
    with torch.cuda.device(x.device):
        st = getattr(lib, "libm_hip_ldexp_" + tag)(x.data_ptr(), e.data_ptr(), out.data_ptr(),
                                                   x.numel(), _stream_handle())
    _check(st, "libm_hip_ldexp_" + tag)
    return out


def ilogb(x):
    """The exponent of x as if normalized, as an int32 tensor."""
    import torch
    lib = load()
    tag = _fp_tag(x)
    x = x.contiguous()
    e = torch.empty(x.shape, dtype=torch.int32, device=x.device)
    with torch.cuda.device(x.device):
        st = getattr(lib, "libm_hip_ilogb_" + tag)(x.data_ptr(), e.data_ptr(), x.numel(),
                                                   _stream_handle())
    _check(st, "libm_hip_ilogb_" + tag)
    return e


def frexp(x):
    """(m, e): m in [0.5, 1) of x's dtype and e int32 with x = m * 2^e."""
    import torch
    lib = load()
    tag = _fp_tag(x)
    x = x.contiguous()
    m = torch.empty_like(x)
    e = torch.empty(x.shape, dtype=torch.int32, device=x.device)
    with torch.cuda.device(x.device):
        st = getattr(lib, "libm_hip_frexp_" + tag)(x.data_ptr(), m.data_ptr(), e.data_ptr(),
                                                   x.numel(), _stream_handle())
    _check(st, "libm_hip_frexp_" + tag)
    return m, e


def modf(x):
    """(fraction, integral part) of x elementwise, both with x's sign."""
    import torch
    lib = load()
    tag = _fp_tag(x)
    x = x.contiguous()
    f, ip = torch.empty_like(x), torch.empty_like(x)
    nm = "libm_hip_modf_" + tag
    with torch.cuda.device(x.device):
        st = getattr(lib, nm)(ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(f.data_ptr()),
                              ctypes.c_void_p(ip.data_ptr()), ctypes.c_size_t(x.numel()),
                              ctypes.c_void_p(_stream_handle()))
    _check(st, nm)
    return f, ip


def fma(a, b, c):
    """a * b + c rounded once, elementwise."""
    import torch
    lib = load()
    tag = _fp_tag(a)
    a = a.contiguous()
    b, c = _operand(b, a, "second operand"), _operand(c, a, "third operand")
    y = torch.empty_like(a)
    nm = "libm_hip_fma_" + tag
    with torch.cuda.device(a.device):
        st = getattr(lib, nm)(*[ctypes.c_void_p(t.data_ptr()) for t in (a, b, c, y)],
                              ctypes.c_size_t(a.numel()), ctypes.c_void_p(_stream_handle()))
    _check(st, nm)
    return y


def _to_int64(kind, x):
    import torch
    lib = load()
    tag = _fp_tag(x)
    x = x.contiguous()
    y = torch.empty(x.shape, dtype=torch.int64, device=x.device)
    nm = "libm_hip_%s_%s" % (kind, tag)
    with torch.cuda.device(x.device):
        st = getattr(lib, nm)(ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(y.data_ptr()),
                              ctypes.c_size_t(x.numel()), ctypes.c_void_p(_stream_handle()))
    _check(st, nm)
    return y


def lrint(x):
    """Nearest integer (ties to even) as int64; INT64_MIN where it does not fit."""
    return _to_int64("lrint", x)


def lround(x):
    """Nearest integer (ties away from zero) as int64; INT64_MIN where it does not fit."""
    return _to_int64("lround", x)


def remquo(x, y):
    """(remainder(x, y), quo) elementwise; quo int32 with the sign of x/y and
    the quotient's low three bits."""
    import torch
    lib = load()
    tag = _fp_tag(x)
    x = x.contiguous()
    y = _operand(y, x, "second operand")
    r = torch.empty_like(x)
    q = torch.empty(x.shape, dtype=torch.int32, device=x.device)
    nm = "libm_hip_remquo_" + tag
    with torch.cuda.device(x.device):
        st = getattr(lib, nm)(*[ctypes.c_void_p(t.data_ptr()) for t in (x, y, r, q)],
                              ctypes.c_size_t(x.numel()), ctypes.c_void_p(_stream_handle()))
    _check(st, nm)
    return r, q
