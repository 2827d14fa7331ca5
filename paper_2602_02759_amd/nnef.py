"""Python binding of libnnef (C ABI in ``include/nnef.h``).

Argument marshalling only: every step of a sweep runs in the library's HIP
kernels.  The functions keep the C names (``nnef_plan``, ``nnef_step``,
``nnef_loss``, ...); ``Plan`` is a small owner object around them.  Tensors are
torch tensors on the GPU: Y float32, mask uint8 (1 = observed) or None, factors
float32, all contiguous, in the layouts the header documents.

There is no fallback: if ``libnnef.so`` is missing or fails to load, every call
raises.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("NNEF_LIB") or os.path.join(_HERE, "libnnef.so")
_lib = None

STATUS = {0: "NNEF_OK", 1: "NNEF_E_PARSE", 2: "NNEF_E_SHAPE", 3: "NNEF_E_LOSS_UNSUPPORTED",
          4: "NNEF_E_ARG", 5: "NNEF_E_DEVICE", 6: "NNEF_E_NOMEM", 7: "NNEF_E_UNSUPPORTED"}
PREC = {"fp32": 0, "bf16": 1, "fp16": 2, "bf16_all": 3, "fp16_all": 4}
FAMILY = {"ab": 0, "negbin": 1, "binomial": 2, "js": 3}


class NnefError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class Options(ctypes.Structure):
    _fields_ = [("eps", ctypes.c_double), ("prec", ctypes.c_int), ("deterministic", ctypes.c_int),
                ("family", ctypes.c_int), ("reserved", ctypes.c_int * 5),
                ("family_param", ctypes.c_double)]


class Problem(ctypes.Structure):
    _fields_ = [("model_str", ctypes.c_char_p), ("mode_sizes", ctypes.POINTER(ctypes.c_int64)),
                ("n_modes", ctypes.c_int), ("ranks", ctypes.POINTER(ctypes.c_int64)),
                ("n_ranks", ctypes.c_int), ("alpha", ctypes.c_double), ("beta", ctypes.c_double),
                ("n_restarts", ctypes.c_int), ("masked", ctypes.c_int)]


class FitOptions(ctypes.Structure):
    _fields_ = [("max_sweeps", ctypes.c_int), ("patience", ctypes.c_int), ("rel_tol", ctypes.c_double),
                ("check_every", ctypes.c_int), ("train_value", ctypes.c_int), ("val_value", ctypes.c_int)]


class FitResult(ctypes.Structure):
    _fields_ = [("stop_sweep", ctypes.c_int), ("sweeps_run", ctypes.c_int), ("reason", ctypes.c_int),
                ("train_loss", ctypes.c_double), ("val_loss", ctypes.c_double)]


EXPORTS = {
    "nnef_default_options": (None, [ctypes.POINTER(Options)]),
    "nnef_plan": (ctypes.c_int, [ctypes.c_char_p, ctypes.POINTER(ctypes.c_int64), ctypes.c_int,
                                 ctypes.POINTER(ctypes.c_int64), ctypes.c_int, ctypes.c_double,
                                 ctypes.c_double, ctypes.POINTER(Options),
                                 ctypes.POINTER(ctypes.c_void_p)]),
    "nnef_plan_destroy": (None, [ctypes.c_void_p]),
    "nnef_plan_dry": (ctypes.c_size_t, [ctypes.c_char_p, ctypes.POINTER(ctypes.c_int64), ctypes.c_int,
                                        ctypes.POINTER(ctypes.c_int64), ctypes.c_int, ctypes.c_double,
                                        ctypes.c_double, ctypes.POINTER(Options), ctypes.POINTER(ctypes.c_int),
                                        ctypes.c_char_p, ctypes.c_size_t]),
    "nnef_plan_num_factors": (ctypes.c_int, [ctypes.c_void_p]),
    "nnef_plan_factor_numel": (ctypes.c_int64, [ctypes.c_void_p, ctypes.c_int]),
    "nnef_plan_describe": (ctypes.c_size_t, [ctypes.c_void_p, ctypes.c_char_p, ctypes.c_size_t]),
    "nnef_step": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                 ctypes.POINTER(ctypes.c_void_p), ctypes.c_int, ctypes.c_void_p,
                                 ctypes.c_void_p]),
    "nnef_loss": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                 ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(ctypes.c_double),
                                 ctypes.c_void_p]),
    "nnef_loss_device": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                        ctypes.POINTER(ctypes.c_void_p), ctypes.c_void_p,
                                        ctypes.c_void_p]),
    "nnef_plan_set_timing": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int]),
    "nnef_plan_timing": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int),
                                        ctypes.POINTER(ctypes.c_double)]),
    "nnef_last_error": (ctypes.c_char_p, []),
    "nnef_batch_plan": (ctypes.c_int, [ctypes.POINTER(Problem), ctypes.c_int, ctypes.POINTER(Options),
                                       ctypes.POINTER(ctypes.c_void_p)]),
    "nnef_batch_destroy": (None, [ctypes.c_void_p]),
    "nnef_batch_num_runs": (ctypes.c_int, [ctypes.c_void_p]),
    "nnef_batch_step": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p),
                                       ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(ctypes.c_void_p),
                                       ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p]),
    "nnef_batch_autotune": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p),
                                           ctypes.POINTER(ctypes.c_void_p),
                                           ctypes.POINTER(ctypes.c_void_p), ctypes.c_void_p]),
    "nnef_batch_describe": (ctypes.c_size_t, [ctypes.c_void_p, ctypes.c_char_p, ctypes.c_size_t]),
    "nnef_loss_split": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int,
                                       ctypes.POINTER(ctypes.c_void_p), ctypes.c_void_p, ctypes.c_void_p]),
    "nnef_default_fit_options": (None, [ctypes.POINTER(FitOptions)]),
    "nnef_fit": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(FitOptions),
                                ctypes.POINTER(FitResult), ctypes.c_void_p, ctypes.c_void_p,
                                ctypes.c_void_p]),
    "nnef_mlp_num_params": (ctypes.c_int, []),
    "nnef_mlp_create": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p)]),
    "nnef_mlp_destroy": (None, [ctypes.c_void_p]),
    "nnef_mlp_params": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "nnef_mlp_forward": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                                        ctypes.c_void_p, ctypes.c_void_p]),
    "nnef_mlp_gradient": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                         ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p,
                                         ctypes.c_void_p, ctypes.c_void_p]),
    "nnef_mlp_gradient_noalloc": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                                 ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p,
                                                 ctypes.c_void_p, ctypes.c_void_p]),
    "nnef_mlp_train_step": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                           ctypes.c_void_p, ctypes.c_int64, ctypes.c_double,
                                           ctypes.c_void_p, ctypes.c_void_p]),
    "nnef_learned_rows": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p),
                                         ctypes.POINTER(ctypes.c_void_p),
                                         ctypes.POINTER(ctypes.c_void_p),
                                         ctypes.POINTER(ctypes.c_void_p), ctypes.c_double,
                                         ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "nnef_step_learned": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                         ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p),
                                         ctypes.c_int, ctypes.c_int, ctypes.c_void_p,
                                         ctypes.c_void_p, ctypes.c_void_p]),
}


def lib():
    """Load libnnef.so (raises if it is not built)."""
    global _lib
    if _lib is None:
        # torch bundles its own libamdhip64.so.7; load it first so that the
        # library binds to the same HIP runtime instead of a second copy.
        import torch  # noqa: F401
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build()")
        h = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in EXPORTS.items():
            f = getattr(h, name)
            f.restype = res
            f.argtypes = args
        _lib = h
    return _lib


def _check(st):
    if st != 0:
        raise NnefError(st, lib().nnef_last_error().decode())


def _ptr(t, dtype, what):
    import torch
    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{what} must be a CUDA (HIP) torch tensor")
    if t.dtype != dtype:
        raise TypeError(f"{what} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{what} must be contiguous")
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream))


def _factor_array(factors, numels=None):
    import torch
    arr = (ctypes.c_void_p * len(factors))()
    for i, f in enumerate(factors):
        arr[i] = _ptr(f, torch.float32, f"factor {i}")
        if numels is not None and f.numel() != numels[i]:
            raise ValueError(f"factor {i} has {f.numel()} elements, the plan expects {numels[i]}")
    return arr


# ------------------------------------------------------------------ C-named calls
def nnef_plan(model_str, mode_sizes, ranks, alpha, beta, eps=1e-10, prec="fp32", family="ab",
              family_param=0.0):
    opt = Options()
    lib().nnef_default_options(ctypes.byref(opt))
    opt.eps = eps
    opt.prec = PREC[prec]
    opt.family = FAMILY[family]
    opt.family_param = float(family_param)
    ms = (ctypes.c_int64 * len(mode_sizes))(*mode_sizes)
    rk = (ctypes.c_int64 * max(1, len(ranks)))(*ranks)
    h = ctypes.c_void_p()
    _check(lib().nnef_plan(model_str.encode(), ms, len(mode_sizes), rk, len(ranks),
                           float(alpha), float(beta), ctypes.byref(opt), ctypes.byref(h)))
    return h


def nnef_plan_dry(model_str, mode_sizes, ranks, alpha=1.0, beta=0.0, eps=1e-10, prec="fp32", family="ab",
                  family_param=0.0):
    """Lowering description of a plan, computed without a GPU."""
    opt = Options()
    lib().nnef_default_options(ctypes.byref(opt))
    opt.eps = eps
    opt.prec = PREC[prec]
    opt.family = FAMILY[family]
    opt.family_param = float(family_param)
    ms = (ctypes.c_int64 * max(1, len(mode_sizes)))(*mode_sizes)
    rk = (ctypes.c_int64 * max(1, len(ranks)))(*ranks)
    st = ctypes.c_int()
    args = (model_str.encode(), ms, len(mode_sizes), rk, len(ranks), float(alpha), float(beta),
            ctypes.byref(opt), ctypes.byref(st))
    n = lib().nnef_plan_dry(*args, None, 0)
    _check(st.value)
    buf = ctypes.create_string_buffer(n + 1)
    lib().nnef_plan_dry(*args, buf, n + 1)
    return buf.value.decode()


def nnef_plan_destroy(h):
    lib().nnef_plan_destroy(h)


def nnef_plan_describe(h):
    n = lib().nnef_plan_describe(h, None, 0)
    buf = ctypes.create_string_buffer(n + 1)
    lib().nnef_plan_describe(h, buf, n + 1)
    return buf.value.decode()


def nnef_plan_set_timing(h, enable):
    _check(lib().nnef_plan_set_timing(h, int(bool(enable))))


def nnef_plan_timing(h):
    n = ctypes.c_int()
    ms = ctypes.c_double()
    _check(lib().nnef_plan_timing(h, ctypes.byref(n), ctypes.byref(ms)))
    return n.value, ms.value


def nnef_step(h, Y, M, factors, n_sweeps, loss_trace=None, stream=None):
    import torch
    _check(lib().nnef_step(h, _ptr(Y, torch.float32, "Y"), _ptr(M, torch.uint8, "mask"),
                           _factor_array(factors), int(n_sweeps),
                           _ptr(loss_trace, torch.float64, "loss_trace"), _stream(stream)))


def nnef_loss(h, Y, M, factors, stream=None):
    import torch
    out = ctypes.c_double()
    _check(lib().nnef_loss(h, _ptr(Y, torch.float32, "Y"), _ptr(M, torch.uint8, "mask"),
                           _factor_array(factors), ctypes.byref(out), _stream(stream)))
    return out.value


def nnef_loss_device(h, Y, M, factors, d_out, stream=None):
    import torch
    _check(lib().nnef_loss_device(h, _ptr(Y, torch.float32, "Y"), _ptr(M, torch.uint8, "mask"),
                                  _factor_array(factors), _ptr(d_out, torch.float64, "d_out"),
                                  _stream(stream)))


def nnef_mlp_num_params():
    return lib().nnef_mlp_num_params()


def nnef_mlp_create(init_params):
    import torch
    h = ctypes.c_void_p()
    if init_params.numel() != nnef_mlp_num_params():
        raise ValueError(f"expected {nnef_mlp_num_params()} parameters, got {init_params.numel()}")
    _check(lib().nnef_mlp_create(_ptr(init_params, torch.float32, "init_params"), ctypes.byref(h)))
    return h


def nnef_mlp_destroy(h):
    lib().nnef_mlp_destroy(h)


def nnef_mlp_params(h, d_out, stream=None):
    import torch
    _check(lib().nnef_mlp_params(h, _ptr(d_out, torch.float32, "d_out"), _stream(stream)))


def nnef_mlp_forward(h, X, s_out, stream=None):
    import torch
    _check(lib().nnef_mlp_forward(h, _ptr(X, torch.float32, "X"), X.shape[0],
                                  _ptr(s_out, torch.float32, "s_out"), _stream(stream)))


def nnef_mlp_gradient(h, X, tau, idx, n_rows, d_grad, d_loss=None, stream=None):
    import torch
    _check(lib().nnef_mlp_gradient(h, _ptr(X, torch.float32, "X"), _ptr(tau, torch.float32, "tau"),
                                   _ptr(idx, torch.int32, "idx"), int(n_rows),
                                   _ptr(d_grad, torch.float32, "d_grad"),
                                   _ptr(d_loss, torch.float64, "d_loss"), _stream(stream)))


def nnef_mlp_gradient_noalloc(params, X, tau, idx, n_rows, d_grad, d_loss=None, stream=None):
    import torch
    _check(lib().nnef_mlp_gradient_noalloc(_ptr(params, torch.float32, "params"),
                                           _ptr(X, torch.float32, "X"), _ptr(tau, torch.float32, "tau"),
                                           _ptr(idx, torch.int32, "idx"), int(n_rows),
                                           _ptr(d_grad, torch.float32, "d_grad"),
                                           _ptr(d_loss, torch.float64, "d_loss"), _stream(stream)))


def nnef_mlp_train_step(h, X, tau, idx, n_rows, lr, d_loss=None, stream=None):
    import torch
    _check(lib().nnef_mlp_train_step(h, _ptr(X, torch.float32, "X"), _ptr(tau, torch.float32, "tau"),
                                     _ptr(idx, torch.int32, "idx"), int(n_rows), float(lr),
                                     _ptr(d_loss, torch.float64, "d_loss"), _stream(stream)))


def nnef_learned_rows(h, th_t, th_tm1, th_tm2, th_target, rel_dec, X, tau=None, stream=None):
    import torch
    _check(lib().nnef_learned_rows(h, _factor_array(th_t), _factor_array(th_tm1),
                                   _factor_array(th_tm2),
                                   _factor_array(th_target) if th_target is not None else None,
                                   float(rel_dec), _ptr(X, torch.float32, "X"),
                                   _ptr(tau, torch.float32, "tau"), _stream(stream)))


def nnef_step_learned(h, mlp, Y, M, factors, n_sweeps, propose_every, loss_trace=None,
                      n_accepted=None, stream=None):
    import torch
    _check(lib().nnef_step_learned(h, mlp, _ptr(Y, torch.float32, "Y"), _ptr(M, torch.uint8, "mask"),
                                   _factor_array(factors), int(n_sweeps), int(propose_every),
                                   _ptr(loss_trace, torch.float64, "loss_trace"),
                                   _ptr(n_accepted, torch.int32, "n_accepted"), _stream(stream)))


def _ptr_array(ts, dtype, what, allow_none=False):
    arr = (ctypes.c_void_p * len(ts))()
    for i, t in enumerate(ts):
        if t is None and allow_none:
            arr[i] = None
        else:
            arr[i] = _ptr(t, dtype, f"{what} {i}")
    return arr


def nnef_batch_plan(problems, eps=1e-10, prec="fp32"):
    """problems: list of dicts with model_str, mode_sizes, ranks, alpha, beta,
    n_restarts and masked."""
    opt = Options()
    lib().nnef_default_options(ctypes.byref(opt))
    opt.eps = eps
    opt.prec = PREC[prec]
    arr = (Problem * len(problems))()
    keep = []
    for i, d in enumerate(problems):
        ms = (ctypes.c_int64 * len(d["mode_sizes"]))(*d["mode_sizes"])
        rk = (ctypes.c_int64 * max(1, len(d["ranks"])))(*d["ranks"])
        name = d["model_str"].encode()
        keep += [ms, rk, name]
        arr[i] = Problem(name, ms, len(d["mode_sizes"]), rk, len(d["ranks"]), float(d["alpha"]),
                         float(d["beta"]), int(d.get("n_restarts", 1)), int(bool(d.get("masked", 0))))
    h = ctypes.c_void_p()
    _check(lib().nnef_batch_plan(arr, len(problems), ctypes.byref(opt), ctypes.byref(h)))
    return h


def _batch_args(Ys, Ms, factors):
    import torch
    y = _ptr_array(Ys, torch.float32, "Y")
    m = _ptr_array(Ms, torch.uint8, "mask", allow_none=True) if Ms is not None else None
    flat = [f for run in factors for f in run]
    return y, m, _factor_array(flat)


def nnef_batch_step(h, Ys, Ms, factors, n_sweeps, loss_trace=None, stream=None):
    import torch
    y, m, f = _batch_args(Ys, Ms, factors)
    _check(lib().nnef_batch_step(h, y, m, f, int(n_sweeps), _ptr(loss_trace, torch.float64, "loss_trace"),
                                 _stream(stream)))


def nnef_batch_autotune(h, Ys, Ms, factors, stream=None):
    y, m, f = _batch_args(Ys, Ms, factors)
    _check(lib().nnef_batch_autotune(h, y, m, f, _stream(stream)))


def nnef_batch_describe(h):
    n = lib().nnef_batch_describe(h, None, 0)
    buf = ctypes.create_string_buffer(n + 1)
    lib().nnef_batch_describe(h, buf, n + 1)
    return buf.value.decode()


class Batch:
    """Owner of an ``nnef_batch_t``: many problems x restarts swept together.
    ``factors`` arguments are lists (one per run, problem-major) of factor lists."""

    def __init__(self, problems, eps=1e-10, prec="fp32"):
        self.h = nnef_batch_plan(problems, eps, prec)
        self.n_runs = lib().nnef_batch_num_runs(self.h)

    def step(self, Ys, Ms, factors, n_sweeps=1, loss_trace=None, stream=None):
        if len(factors) != self.n_runs:
            raise ValueError(f"expected {self.n_runs} runs, got {len(factors)}")
        nnef_batch_step(self.h, Ys, Ms, factors, n_sweeps, loss_trace, stream)

    def autotune(self, Ys, Ms, factors, stream=None):
        nnef_batch_autotune(self.h, Ys, Ms, factors, stream)

    def describe(self):
        return nnef_batch_describe(self.h)

    def close(self):
        if self.h:
            lib().nnef_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def nnef_loss_split(h, Y, M, value, factors, d_out, stream=None):
    import torch
    _check(lib().nnef_loss_split(h, _ptr(Y, torch.float32, "Y"), _ptr(M, torch.uint8, "mask"), int(value),
                                 _factor_array(factors), _ptr(d_out, torch.float64, "d_out"),
                                 _stream(stream)))


def nnef_fit(h, Y, M, factors, train_trace=None, val_trace=None, stream=None, **options):
    """Options: max_sweeps, patience, rel_tol, check_every, train_value, val_value."""
    import torch
    opt = FitOptions()
    lib().nnef_default_fit_options(ctypes.byref(opt))
    for k, v in options.items():
        if not hasattr(opt, k):
            raise TypeError(f"unknown fit option {k}")
        setattr(opt, k, v)
    res = FitResult()
    _check(lib().nnef_fit(h, _ptr(Y, torch.float32, "Y"), _ptr(M, torch.uint8, "mask"),
                          _factor_array(factors), ctypes.byref(opt), ctypes.byref(res),
                          _ptr(train_trace, torch.float64, "train_trace"),
                          _ptr(val_trace, torch.float64, "val_trace"), _stream(stream)))
    return {"stop_sweep": res.stop_sweep, "sweeps_run": res.sweeps_run,
            "reason": {0: "max_sweeps", 1: "train_tol", 2: "validation"}[res.reason],
            "train_loss": res.train_loss, "val_loss": res.val_loss}


class Mlp:
    """Owner of an ``nnef_mlp_t`` (the extrapolation network)."""

    def __init__(self, init_params):
        self.h = nnef_mlp_create(init_params)

    def params(self):
        import torch
        out = torch.empty(nnef_mlp_num_params(), dtype=torch.float32, device="cuda")
        nnef_mlp_params(self.h, out)
        return out

    def forward(self, X):
        import torch
        s = torch.empty(X.shape[0], dtype=torch.float32, device=X.device)
        nnef_mlp_forward(self.h, X, s)
        return s

    def gradient(self, X, tau, idx=None):
        import torch
        n = idx.numel() if idx is not None else X.shape[0]
        g = torch.empty(nnef_mlp_num_params(), dtype=torch.float32, device=X.device)
        l = torch.empty(1, dtype=torch.float64, device=X.device)
        nnef_mlp_gradient(self.h, X, tau, idx, n, g, l)
        return g, l

    def train_step(self, X, tau, lr, idx=None, d_loss=None):
        n = idx.numel() if idx is not None else X.shape[0]
        nnef_mlp_train_step(self.h, X, tau, idx, n, lr, d_loss)

    def close(self):
        if self.h:
            nnef_mlp_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Plan:
    """Owner of an ``nnef_plan_t``; the methods call the C entry points."""

    def __init__(self, model_str, mode_sizes, ranks, alpha=1.0, beta=0.0, eps=1e-10, prec="fp32",
                 family="ab", family_param=0.0):
        self.model_str = model_str
        self.h = nnef_plan(model_str, list(mode_sizes), list(ranks), alpha, beta, eps, prec, family,
                           family_param)
        n = lib().nnef_plan_num_factors(self.h)
        self.numels = [lib().nnef_plan_factor_numel(self.h, i) for i in range(n)]

    def describe(self):
        return nnef_plan_describe(self.h)

    def _check_factors(self, factors):
        if len(factors) != len(self.numels):
            raise ValueError(f"expected {len(self.numels)} factors, got {len(factors)}")
        _factor_array(factors, self.numels)

    def step(self, Y, M, factors, n_sweeps=1, loss_trace=None, stream=None):
        self._check_factors(factors)
        nnef_step(self.h, Y, M, factors, n_sweeps, loss_trace, stream)

    def loss(self, Y, M, factors, stream=None):
        self._check_factors(factors)
        return nnef_loss(self.h, Y, M, factors, stream)

    def loss_device(self, Y, M, factors, d_out, stream=None):
        self._check_factors(factors)
        nnef_loss_device(self.h, Y, M, factors, d_out, stream)

    def rows(self, th_t, th_tm1, th_tm2, th_target, rel_dec, X, tau=None):
        for f in (th_t, th_tm1, th_tm2) + ((th_target,) if th_target is not None else ()):
            self._check_factors(f)
        nnef_learned_rows(self.h, th_t, th_tm1, th_tm2, th_target, rel_dec, X, tau)

    def step_learned(self, mlp, Y, M, factors, n_sweeps, propose_every, loss_trace=None,
                     n_accepted=None, stream=None):
        self._check_factors(factors)
        nnef_step_learned(self.h, mlp.h, Y, M, factors, n_sweeps, propose_every, loss_trace,
                          n_accepted, stream)

    def loss_split(self, Y, M, value, factors):
        """Loss over the entries whose mask byte equals ``value`` (syncs)."""
        import torch
        self._check_factors(factors)
        out = torch.empty(1, dtype=torch.float64, device=Y.device)
        nnef_loss_split(self.h, Y, M, value, factors, out)
        return out.item()

    def fit(self, Y, M, factors, train_trace=None, val_trace=None, **options):
        self._check_factors(factors)
        return nnef_fit(self.h, Y, M, factors, train_trace, val_trace, **options)

    def set_timing(self, enable=True):
        nnef_plan_set_timing(self.h, enable)

    def timing(self):
        """(number of fused passes timed, their total milliseconds)."""
        return nnef_plan_timing(self.h)

    def close(self):
        if self.h:
            nnef_plan_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
