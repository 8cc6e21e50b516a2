"""Python binding of libdl.so, the gfx950 library for linear-algebraic Datalog
evaluation (least models of transitive closure, same generation and the
epsilon-scaled linear form, Sato's method).

Argument marshalling only: every step runs in the library's HIP kernels.
torch supplies device memory and the stream.  The functions keep the C names
(``dl_tc``, ``dl_sg``, ``dl_solve_eps`` ...) and take uint8 CUDA/HIP tensors.

The library must be built beforehand (``python -m paper_1608_00139_amd.build``
or ``__graft_entry__.build()``); importing this module never compiles and
never falls back to another implementation: a missing library raises.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import torch

__all__ = [
    "DL_TC_PLAIN", "DL_TC_SQUARE", "DL_I8", "DL_F32", "DL_BF16", "DL_FP8", "DL_FP4",
    "DLError", "Context", "lib_path", "load",
    "dl_tc", "dl_tc_steps", "dl_tc_batch", "dl_tc_noalloc", "dl_sg", "dl_sg_steps", "dl_solve_eps", "dl_eps_bound", "dl_sg_eps",
    "dl_padded_size", "Batch", "DL_EAGAIN", "dl_solve_linear", "dl_solve_two_sided", "Program",
    "DL_EVAL_ITERATION", "DL_EVAL_MATRIX", "dl_measure_peak",
]

DL_EAGAIN = 6
DL_EVAL_ITERATION, DL_EVAL_MATRIX = 0, 1
FORMS = ("nonrecursive", "right_tail", "left_tail", "two_sided", "general")

DL_TC_PLAIN, DL_TC_SQUARE = 0, 1
DL_I8, DL_F32, DL_BF16, DL_FP8, DL_FP4 = 0, 1, 2, 3, 4
PRECISIONS = {"i8": DL_I8, "f32": DL_F32, "bf16": DL_BF16, "fp8": DL_FP8, "fp4": DL_FP4}

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None


def lib_path() -> str:
    return os.path.join(_HERE, "libdl.so")


class DLError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"status {status}: {msg}")
        self.status = status


def load() -> ctypes.CDLL:
    """Load libdl.so; raises if it has not been built."""
    global _LIB
    if _LIB is not None:
        return _LIB
    path = lib_path()
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with `python -m paper_1608_00139_amd.build`")
    lib = ctypes.CDLL(path)
    i64, i32, vp, dbl = ctypes.c_int64, ctypes.c_int32, ctypes.c_void_p, ctypes.c_double
    pi32 = ctypes.POINTER(ctypes.c_int32)
    pi64 = ctypes.POINTER(ctypes.c_int64)
    sig = {
        "dl_create": ([ctypes.POINTER(vp), ctypes.c_int, ctypes.c_size_t], ctypes.c_int),
        "dl_destroy": ([vp], ctypes.c_int),
        "dl_tc": ([vp, i64, vp, i64, vp, i64, ctypes.c_int, ctypes.c_int, pi32, vp], ctypes.c_int),
        "dl_tc_steps": ([vp, i64, vp, i64, vp, i64, ctypes.c_int, ctypes.c_int, i32, pi64, pi32, pi32, vp],
                        ctypes.c_int),
        "dl_tc_batch": ([vp, i32, i64, ctypes.POINTER(vp), i64, ctypes.POINTER(vp), i64, ctypes.c_int, ctypes.c_int,
                         pi32, vp], ctypes.c_int),
        "dl_sg": ([vp, i64, vp, i64, vp, i64, ctypes.c_int, pi32, vp], ctypes.c_int),
        "dl_sg_steps": ([vp, i64, vp, i64, vp, i64, ctypes.c_int, i32, pi64, pi32, pi32, vp], ctypes.c_int),
        "dl_solve_eps": ([vp, i64, vp, i64, dbl, vp, i64, vp, i64, pi32, pi32, vp], ctypes.c_int),
        "dl_tc_noalloc": ([i64, vp, i64, vp, i64, ctypes.c_int, pi32, vp], ctypes.c_int),
        "dl_eps_bound": ([vp, i64, vp, i64, ctypes.POINTER(dbl), vp], ctypes.c_int),
        "dl_sg_eps": ([vp, i64, vp, i64, dbl, vp, i64, vp, i64, pi32, vp], ctypes.c_int),
        "dl_set_timing": ([vp, ctypes.c_int], ctypes.c_int),
        "dl_tune": ([vp, ctypes.c_int, i64, pi32, ctypes.POINTER(dbl), ctypes.POINTER(dbl), vp], ctypes.c_int),
        "dl_tune_set": ([vp, ctypes.c_int, i64, i32], ctypes.c_int),
        "dl_tune_get": ([vp, pi32, pi64, pi32, ctypes.POINTER(dbl), i32, pi32], ctypes.c_int),
        "dl_kernel_stats": ([vp, ctypes.c_int, pi64, ctypes.POINTER(dbl), ctypes.c_int], ctypes.c_int),
        "dl_padded_size": ([i64, ctypes.c_int, ctypes.c_int], i64),
        "dl_batch_create": ([vp, ctypes.c_int, ctypes.c_size_t, ctypes.c_int, ctypes.POINTER(vp)], ctypes.c_int),
        "dl_batch_destroy": ([vp], ctypes.c_int),
        "dl_batch_submit": ([vp, ctypes.c_int, i64, vp, i64, i64, pi32, vp], ctypes.c_int),
        "dl_batch_submit_edges": ([vp, ctypes.c_int, i64, vp, i64, i64, pi32, vp], ctypes.c_int),
        "dl_batch_step": ([vp, pi32, pi32, vp], ctypes.c_int),
        "dl_batch_set_lookahead": ([vp, i32], ctypes.c_int),
        "dl_batch_tune": ([vp, pi64, i32, pi32, ctypes.POINTER(dbl), vp], ctypes.c_int),
        "dl_batch_set_tiles": ([vp, pi64, pi32, i32], ctypes.c_int),
        "dl_batch_poll": ([vp, pi64, pi32, pi32, i32, pi32], ctypes.c_int),
        "dl_batch_fetch": ([vp, i32, vp, i64, pi64, vp], ctypes.c_int),
        "dl_batch_submit_edges_n": ([vp, i32, pi32, pi64, ctypes.POINTER(vp), pi64, pi64, pi32, pi32, vp],
                                    ctypes.c_int),
        "dl_batch_release_n": ([vp, i32, pi32, pi64], ctypes.c_int),
        "dl_batch_info": ([vp, pi32, pi32, ctypes.POINTER(ctypes.c_size_t)], ctypes.c_int),
        "dl_solve_linear": ([vp, i64, vp, i64, vp, i64, dbl, vp, i64, vp, i64, vp], ctypes.c_int),
        "dl_solve_two_sided": ([vp, i64, vp, i64, vp, i64, vp, i64, dbl, vp, i64, vp, i64, pi32, vp],
                               ctypes.c_int),
        "dl_program_create": ([vp, ctypes.c_char_p, ctypes.POINTER(vp)], ctypes.c_int),
        "dl_program_destroy": ([vp], ctypes.c_int),
        "dl_program_counts": ([vp, pi32, pi32], ctypes.c_int),
        "dl_program_predicate": ([vp, i32, ctypes.POINTER(ctypes.c_char_p), pi32, pi32], ctypes.c_int),
        "dl_program_bind": ([vp, ctypes.c_char_p, i64, vp, i64], ctypes.c_int),
        "dl_program_run": ([vp, ctypes.c_int, vp], ctypes.c_int),
        "dl_program_layer": ([vp, i32, pi32, pi32, i32, pi32, pi32, pi32], ctypes.c_int),
        "dl_program_fetch": ([vp, ctypes.c_char_p, vp, i64, pi64, vp], ctypes.c_int),
        "dl_measure_peak": ([vp, ctypes.c_int, ctypes.POINTER(dbl), vp], ctypes.c_int),
        "dl_status_str": ([ctypes.c_int], ctypes.c_char_p),
        "dl_last_error": ([], ctypes.c_char_p),
    }
    for name, (args, res) in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = res
    _LIB = lib
    return lib


def _check(rc: int) -> None:
    if rc != 0:
        lib = load()
        raise DLError(rc, f"{lib.dl_status_str(rc).decode()} -- {lib.dl_last_error().decode()}")


def _stream_ptr(stream) -> ctypes.c_void_p:
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _mat(t: torch.Tensor, name: str, dtype=torch.uint8) -> tuple[int, int]:
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a device tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}")
    if t.dim() != 2 or t.shape[0] != t.shape[1]:
        raise ValueError(f"{name} must be square")
    if t.stride(1) != 1 or (t.shape[0] > 1 and t.stride(0) < t.shape[1]):
        raise ValueError(f"{name} must be row-major with unit column stride")
    return t.shape[0], max(t.stride(0), t.shape[1]) if t.shape[0] > 0 else 1


class Context:
    """Owns a dl_ctx (workspace, counters) on one device."""

    def __init__(self, device: int | None = None, workspace_budget: int = 0):
        lib = load()
        if device is None:
            device = torch.cuda.current_device()
        self.device = device
        self._h = ctypes.c_void_p()
        _check(lib.dl_create(ctypes.byref(self._h), device, workspace_budget))

    @property
    def handle(self) -> ctypes.c_void_p:
        if not self._h:
            raise RuntimeError("context destroyed")
        return self._h

    def close(self) -> None:
        if self._h:
            load().dl_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_timing(self, on: bool) -> None:
        _check(load().dl_set_timing(self.handle, int(bool(on))))

    def kernel_stats(self, kernel_class: int, reset: bool = False) -> tuple[int, float]:
        n = ctypes.c_int64()
        ms = ctypes.c_double()
        _check(load().dl_kernel_stats(self.handle, kernel_class, ctypes.byref(n), ctypes.byref(ms), int(reset)))
        return int(n.value), float(ms.value)

    # -- tile autotuner (dl_tune*) --
    def tune(self, prec, n: int, stream=None, candidates: bool = False):
        """Time every tile configuration for (prec, n) and keep the fastest:
        (configuration, ms per product launch), plus the list of every
        candidate's ms when ``candidates`` is true."""
        cfg = ctypes.c_int32()
        ms = ctypes.c_double()
        cand = (ctypes.c_double * 5)()
        _check(load().dl_tune(self.handle, _prec(prec), int(n), ctypes.byref(cfg), ctypes.byref(ms), cand,
                              _stream_ptr(stream)))
        if candidates:
            return int(cfg.value), float(ms.value), [float(cand[i]) for i in range(5)]
        return int(cfg.value), float(ms.value)

    def set_tuning(self, prec, n: int, cfg: int) -> None:
        """Fix the tile configuration for (prec, n); cfg = -1 removes it."""
        _check(load().dl_tune_set(self.handle, _prec(prec), int(n), int(cfg)))

    def tuning(self) -> list[dict]:
        """The context's tuned entries: precision name, padded size, cfg, ms."""
        count = ctypes.c_int32()
        _check(load().dl_tune_get(self.handle, None, None, None, None, 0, ctypes.byref(count)))
        k = count.value
        pr, npad = (ctypes.c_int32 * max(k, 1))(), (ctypes.c_int64 * max(k, 1))()
        cf, ms = (ctypes.c_int32 * max(k, 1))(), (ctypes.c_double * max(k, 1))()
        _check(load().dl_tune_get(self.handle, pr, npad, cf, ms, k, ctypes.byref(count)))
        names = {v: key for key, v in PRECISIONS.items()}
        return [{"prec": names[pr[i]], "np": int(npad[i]), "cfg": int(cf[i]), "ms": float(ms[i])}
                for i in range(k)]

    def save_tuning(self, path: str) -> None:
        with open(path, "w") as f:
            f.write(tuning_to_json(self.tuning(), torch.cuda.get_device_name(self.device)))

    def load_tuning(self, path: str) -> list[dict]:
        """Apply the entries of a file written by save_tuning; returns them."""
        with open(path) as f:
            entries = tuning_from_json(f.read())
        for e in entries:
            self.set_tuning(e["prec"], e["np"], e["cfg"])
        return entries


TUNING_FORMAT = "dl-tuning-1"


def tuning_to_json(entries: list, device: str) -> str:
    """Tuning entries as a JSON document (format, device name, entries)."""
    import json

    rows = [{"prec": e["prec"], "np": int(e["np"]), "cfg": int(e["cfg"]), "ms": float(e.get("ms", 0.0))}
            for e in entries]
    return json.dumps({"format": TUNING_FORMAT, "device": device, "entries": rows}, indent=1)


def tuning_from_json(text: str) -> list:
    """Entries of a document written by tuning_to_json, validated."""
    import json

    doc = json.loads(text)
    if doc.get("format") != TUNING_FORMAT:
        raise ValueError("not a tuning document")
    out = []
    for e in doc["entries"]:
        if e["prec"] not in PRECISIONS or int(e["np"]) <= 0 or int(e["cfg"]) < 0:
            raise ValueError(f"bad tuning entry {e}")
        out.append({"prec": e["prec"], "np": int(e["np"]), "cfg": int(e["cfg"]), "ms": float(e.get("ms", 0.0))})
    return out


_DEFAULT: dict[int, Context] = {}


def _ctx(ctx: Context | None) -> Context:
    if ctx is not None:
        return ctx
    dev = torch.cuda.current_device()
    if dev not in _DEFAULT:
        _DEFAULT[dev] = Context(dev)
    return _DEFAULT[dev]


def _prec(p) -> int:
    return PRECISIONS[p] if isinstance(p, str) else int(p)


def dl_tc(A: torch.Tensor, method: int = DL_TC_SQUARE, prec=DL_I8, out: torch.Tensor | None = None,
          ctx: Context | None = None, stream=None) -> tuple[torch.Tensor, int]:
    """Transitive closure of A (uint8 n x n on the device): (R, iters)."""
    n, lda = _mat(A, "A")
    R = out if out is not None else torch.empty((n, n), dtype=torch.uint8, device=A.device)
    _, ldr = _mat(R, "R")
    it = ctypes.c_int32()
    c = _ctx(ctx)
    _check(load().dl_tc(c.handle, n, ctypes.c_void_p(A.data_ptr()), lda, ctypes.c_void_p(R.data_ptr()), ldr,
                        int(method), _prec(prec), ctypes.byref(it), _stream_ptr(stream)))
    return R, int(it.value)


def dl_tc_noalloc(A: torch.Tensor, prec=DL_I8, out: torch.Tensor | None = None,
                  stream=None) -> tuple[torch.Tensor, int]:
    """Plain closure of A (n <= 512) without any device allocation by the
    library (its buffers live in a static device array): (R, iters)."""
    n, lda = _mat(A, "A")
    R = out if out is not None else torch.empty((n, n), dtype=torch.uint8, device=A.device)
    _, ldr = _mat(R, "R")
    it = ctypes.c_int32()
    _check(load().dl_tc_noalloc(n, ctypes.c_void_p(A.data_ptr()), lda, ctypes.c_void_p(R.data_ptr()), ldr,
                                _prec(prec), ctypes.byref(it), _stream_ptr(stream)))
    return R, int(it.value)


def dl_tc_batch(As: list, method: int = DL_TC_SQUARE, prec=DL_I8, outs: list | None = None,
                ctx: Context | None = None, stream=None) -> tuple[list, list]:
    """Transitive closures of several relations of one size (uint8 n x n on
    the device, one common row stride), two fixpoints in flight:
    (list of R, list of iters)."""
    if not As:
        return [], []
    dims = [_mat(a, "A") for a in As]
    n, lda = dims[0]
    if any(d != (n, lda) for d in dims):
        raise ValueError("every relation must have the same size and row stride")
    Rs = outs if outs is not None else [torch.empty((n, n), dtype=torch.uint8, device=a.device) for a in As]
    if len(Rs) != len(As):
        raise ValueError("one output per input")
    rdims = [_mat(r, "R") for r in Rs]
    ldr = rdims[0][1]
    if any(d != (n, ldr) for d in rdims):
        raise ValueError("every output must be n x n with one common row stride")
    k = len(As)
    a_arr = (ctypes.c_void_p * k)(*[a.data_ptr() for a in As])
    r_arr = (ctypes.c_void_p * k)(*[r.data_ptr() for r in Rs])
    its = (ctypes.c_int32 * k)()
    c = _ctx(ctx)
    _check(load().dl_tc_batch(c.handle, k, n, a_arr, lda, r_arr, ldr, int(method), _prec(prec), its,
                              _stream_ptr(stream)))
    return Rs, [int(its[g]) for g in range(k)]


@dataclass
class StepResult:
    R: torch.Tensor
    ones: list
    steps: int
    converged: bool


def dl_tc_steps(A: torch.Tensor, max_steps: int, method: int = DL_TC_SQUARE, prec=DL_I8,
                out: torch.Tensor | None = None, ctx: Context | None = None, stream=None) -> StepResult:
    n, lda = _mat(A, "A")
    R = out if out is not None else torch.empty((n, n), dtype=torch.uint8, device=A.device)
    _, ldr = _mat(R, "R")
    ones = (ctypes.c_int64 * (max_steps + 1))()
    steps = ctypes.c_int32()
    conv = ctypes.c_int32()
    c = _ctx(ctx)
    _check(load().dl_tc_steps(c.handle, n, ctypes.c_void_p(A.data_ptr()), lda, ctypes.c_void_p(R.data_ptr()),
                              ldr, int(method), _prec(prec), int(max_steps), ones, ctypes.byref(steps),
                              ctypes.byref(conv), _stream_ptr(stream)))
    return StepResult(R, [int(ones[k]) for k in range(steps.value + 1)], int(steps.value), bool(conv.value))


def dl_sg(P: torch.Tensor, prec=DL_I8, out: torch.Tensor | None = None, ctx: Context | None = None,
          stream=None) -> tuple[torch.Tensor, int]:
    """Same-generation model of the parent relation P: (S, iters)."""
    n, ldp = _mat(P, "P")
    S = out if out is not None else torch.empty((n, n), dtype=torch.uint8, device=P.device)
    _, lds = _mat(S, "S")
    it = ctypes.c_int32()
    c = _ctx(ctx)
    _check(load().dl_sg(c.handle, n, ctypes.c_void_p(P.data_ptr()), ldp, ctypes.c_void_p(S.data_ptr()), lds,
                        _prec(prec), ctypes.byref(it), _stream_ptr(stream)))
    return S, int(it.value)


def dl_sg_steps(P: torch.Tensor, max_steps: int, prec=DL_I8, out: torch.Tensor | None = None,
                ctx: Context | None = None, stream=None) -> StepResult:
    n, ldp = _mat(P, "P")
    S = out if out is not None else torch.empty((n, n), dtype=torch.uint8, device=P.device)
    _, lds = _mat(S, "S")
    ones = (ctypes.c_int64 * (max_steps + 1))()
    steps = ctypes.c_int32()
    conv = ctypes.c_int32()
    c = _ctx(ctx)
    _check(load().dl_sg_steps(c.handle, n, ctypes.c_void_p(P.data_ptr()), ldp, ctypes.c_void_p(S.data_ptr()),
                              lds, _prec(prec), int(max_steps), ones, ctypes.byref(steps), ctypes.byref(conv),
                              _stream_ptr(stream)))
    return StepResult(S, [int(ones[k]) for k in range(steps.value + 1)], int(steps.value), bool(conv.value))


def dl_eps_bound(A: torch.Tensor, ctx: Context | None = None, stream=None) -> float:
    n, lda = _mat(A, "A")
    out = ctypes.c_double()
    c = _ctx(ctx)
    _check(load().dl_eps_bound(c.handle, n, ctypes.c_void_p(A.data_ptr()), lda, ctypes.byref(out),
                               _stream_ptr(stream)))
    return float(out.value)


def dl_solve_eps(A: torch.Tensor, eps: float, want_x: bool = False, out: torch.Tensor | None = None,
                 ctx: Context | None = None, stream=None, underflow: bool = False):
    """Epsilon form: returns (R, X or None); R = [(I - eps A)^-1 eps A > 0].
    With underflow=True returns (R, X or None, flag), flag = 1 when an entry
    of R may have been lost to fp64 underflow (see include/dl.h)."""
    n, lda = _mat(A, "A")
    R = out if out is not None else torch.empty((n, n), dtype=torch.uint8, device=A.device)
    _, ldr = _mat(R, "R")
    X = torch.empty((n, n), dtype=torch.float64, device=A.device) if want_x else None
    ldx = max(n, 1)
    it = ctypes.c_int32()
    uf = ctypes.c_int32()
    c = _ctx(ctx)
    _check(load().dl_solve_eps(c.handle, n, ctypes.c_void_p(A.data_ptr()), lda, float(eps),
                               ctypes.c_void_p(R.data_ptr()), ldr,
                               ctypes.c_void_p(X.data_ptr()) if X is not None else None, ldx,
                               ctypes.byref(it), ctypes.byref(uf), _stream_ptr(stream)))
    return (R, X, int(uf.value)) if underflow else (R, X)


def dl_sg_eps(P: torch.Tensor, eps: float, want_x: bool = False, out: torch.Tensor | None = None,
              ctx: Context | None = None, stream=None):
    """Same-generation epsilon form: returns (S, X or None, doublings)."""
    n, ldp = _mat(P, "P")
    S = out if out is not None else torch.empty((n, n), dtype=torch.uint8, device=P.device)
    _, lds = _mat(S, "S")
    X = torch.empty((n, n), dtype=torch.float64, device=P.device) if want_x else None
    d = ctypes.c_int32()
    c = _ctx(ctx)
    _check(load().dl_sg_eps(c.handle, n, ctypes.c_void_p(P.data_ptr()), ldp, float(eps),
                            ctypes.c_void_p(S.data_ptr()), lds,
                            ctypes.c_void_p(X.data_ptr()) if X is not None else None, max(n, 1),
                            ctypes.byref(d), _stream_ptr(stream)))
    return S, X, int(d.value)


def dl_solve_linear(B: torch.Tensor, C: torch.Tensor, eps: float, want_x: bool = False,
                    out: torch.Tensor | None = None, ctx: Context | None = None, stream=None):
    """Tail-recursive equation X = eps (C + B X): returns (R, X or None), R = [X > 0]."""
    n, ldb = _mat(B, "B")
    nc, ldc = _mat(C, "C")
    if nc != n:
        raise ValueError("B and C differ in size")
    R = out if out is not None else torch.empty((n, n), dtype=torch.uint8, device=B.device)
    _, ldr = _mat(R, "R")
    X = torch.empty((n, n), dtype=torch.float64, device=B.device) if want_x else None
    c = _ctx(ctx)
    _check(load().dl_solve_linear(c.handle, n, ctypes.c_void_p(B.data_ptr()), ldb, ctypes.c_void_p(C.data_ptr()),
                                  ldc, float(eps), ctypes.c_void_p(R.data_ptr()), ldr,
                                  ctypes.c_void_p(X.data_ptr()) if X is not None else None, max(n, 1),
                                  _stream_ptr(stream)))
    return R, X


def dl_solve_two_sided(Q: torch.Tensor, B: torch.Tensor, C: torch.Tensor, eps: float, want_x: bool = False,
                       out: torch.Tensor | None = None, ctx: Context | None = None, stream=None):
    """Two-sided equation X = eps (Q + B X C): returns (R, X or None, doublings)."""
    n, ldq = _mat(Q, "Q")
    nb, ldb = _mat(B, "B")
    nc, ldc = _mat(C, "C")
    if not n == nb == nc:
        raise ValueError("Q, B and C differ in size")
    R = out if out is not None else torch.empty((n, n), dtype=torch.uint8, device=Q.device)
    _, ldr = _mat(R, "R")
    X = torch.empty((n, n), dtype=torch.float64, device=Q.device) if want_x else None
    d = ctypes.c_int32()
    c = _ctx(ctx)
    _check(load().dl_solve_two_sided(c.handle, n, ctypes.c_void_p(Q.data_ptr()), ldq, ctypes.c_void_p(B.data_ptr()),
                                     ldb, ctypes.c_void_p(C.data_ptr()), ldc, float(eps),
                                     ctypes.c_void_p(R.data_ptr()), ldr,
                                     ctypes.c_void_p(X.data_ptr()) if X is not None else None, max(n, 1),
                                     ctypes.byref(d), _stream_ptr(stream)))
    return R, X, int(d.value)


class Program:
    """A linear binary Datalog program evaluated layer by layer (dl_program_*).

    ``Program(text)`` parses and layers the program; ``bind(name, M)`` gives a
    relation (uint8 device matrix); ``run(method)`` evaluates; ``fetch(name)``
    returns a defined relation; ``layers()`` describes the layers of the last
    run.  Bound tensors must stay alive until ``run`` returns."""

    def __init__(self, text: str, ctx: Context | None = None):
        lib = load()
        self.ctx = _ctx(ctx)
        self._h = ctypes.c_void_p()
        self._bound = {}
        _check(lib.dl_program_create(self.ctx.handle, text.encode(), ctypes.byref(self._h)))

    def close(self) -> None:
        if self._h:
            load().dl_program_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def predicates(self) -> list[tuple[str, int, int]]:
        lib = load()
        npred, nl = ctypes.c_int32(), ctypes.c_int32()
        _check(lib.dl_program_counts(self._h, ctypes.byref(npred), ctypes.byref(nl)))
        out = []
        for i in range(npred.value):
            name, kind, layer = ctypes.c_char_p(), ctypes.c_int32(), ctypes.c_int32()
            _check(lib.dl_program_predicate(self._h, i, ctypes.byref(name), ctypes.byref(kind), ctypes.byref(layer)))
            out.append((name.value.decode(), kind.value, layer.value))
        return out

    def bind(self, name: str, M: torch.Tensor) -> None:
        n, ld = _mat(M, name)
        _check(load().dl_program_bind(self._h, name.encode(), n, ctypes.c_void_p(M.data_ptr()), ld))
        self._bound[name] = M

    def run(self, method: int = DL_EVAL_ITERATION, stream=None) -> None:
        _check(load().dl_program_run(self._h, int(method), _stream_ptr(stream)))

    def layers(self) -> list[dict]:
        lib = load()
        names = [p[0] for p in self.predicates()]
        npred, nl = ctypes.c_int32(), ctypes.c_int32()
        _check(lib.dl_program_counts(self._h, ctypes.byref(npred), ctypes.byref(nl)))
        out = []
        for L in range(nl.value):
            nh, form, meth, it = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
            heads = (ctypes.c_int32 * max(1, npred.value))()
            _check(lib.dl_program_layer(self._h, L, ctypes.byref(nh), heads, npred.value, ctypes.byref(form),
                                        ctypes.byref(meth), ctypes.byref(it)))
            out.append({"heads": sorted(names[heads[i]] for i in range(nh.value)),
                        "form": FORMS[form.value] if form.value >= 0 else None,
                        "method": meth.value, "iters": it.value})
        return out

    def fetch(self, name: str, out: torch.Tensor | None = None, n: int | None = None, stream=None):
        """Returns (model, ones)."""
        if out is None:
            if n is None:
                n = next(iter(self._bound.values())).shape[0] if self._bound else 0
            out = torch.empty((n, n), dtype=torch.uint8, device=f"cuda:{self.ctx.device}")
        nn, ld = _mat(out, "out")
        ones = ctypes.c_int64()
        _check(load().dl_program_fetch(self._h, name.encode(), ctypes.c_void_p(out.data_ptr()), ld,
                                       ctypes.byref(ones), _stream_ptr(stream)))
        return out, int(ones.value)


PEAK_KINDS = {"i8": 0, "f32": 1, "bf16": 2, "fp8": 3, "fp4": 4, "f64": 5, "lds_read": 6, "lds_fill": 7,
              "f64_agpr": 8}


def dl_measure_peak(kind: str, ctx: Context | None = None, stream=None) -> float:
    """Measured MFMA throughput of the device in operations per second
    (kinds "lds_read" and "lds_fill": bytes per second of the LDS data paths)."""
    out = ctypes.c_double()
    c = _ctx(ctx)
    _check(load().dl_measure_peak(c.handle, PEAK_KINDS[kind], ctypes.byref(out), _stream_ptr(stream)))
    return float(out.value)


def dl_padded_size(n: int, kind: int, prec=DL_I8) -> int:
    return int(load().dl_padded_size(n, kind, _prec(prec)))


class Batch:
    """Continuous-batching handle (dl_batch_*): requests resident in one pool,
    advanced together one product per dl_batch_step."""

    TC, SG = 0, 1

    def __init__(self, pool_bytes: int, max_active: int = 256, ctx: Context | None = None, stream=None,
                 lookahead: int = 0):
        lib = load()
        self.ctx = _ctx(ctx)
        self.stream = stream
        self._h = ctypes.c_void_p()
        _check(lib.dl_batch_create(self.ctx.handle, self.ctx.device, int(pool_bytes), int(max_active),
                                   ctypes.byref(self._h)))
        if lookahead:
            _check(lib.dl_batch_set_lookahead(self._h, int(lookahead)))
        self._cap = int(max_active)
        self._tags = (ctypes.c_int64 * self._cap)()
        self._slots = (ctypes.c_int32 * self._cap)()
        self._iters = (ctypes.c_int32 * self._cap)()
        self._pending_edges: list = []
        # edge lists admitted in bulk: kept referenced until the round that
        # scatters them has completed (two dl_batch_step calls later at most)
        self._bulk_edges: list = []
        self._bulk_held: list = [[], []]

    def close(self) -> None:
        if self._h:
            load().dl_batch_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def dl_batch_submit(self, kind: int, A: torch.Tensor, tag: int) -> int | None:
        """Admit a request; returns its slot, or None when the pool is full."""
        n, lda = _mat(A, "A")
        slot = ctypes.c_int32()
        rc = load().dl_batch_submit(self._h, int(kind), n, ctypes.c_void_p(A.data_ptr()), lda, int(tag),
                                    ctypes.byref(slot), _stream_ptr(self.stream))
        if rc == DL_EAGAIN:
            return None
        _check(rc)
        return int(slot.value)

    def dl_batch_submit_edges(self, kind: int, n: int, edges: torch.Tensor, tag: int) -> int | None:
        """Admit a request given as a device int32 [m, 2] edge list over n
        constants; returns its slot, or None when the pool is full."""
        if not isinstance(edges, torch.Tensor) or not edges.is_cuda or edges.dtype != torch.int32:
            raise TypeError("edges must be a device int32 tensor")
        if edges.numel() and (edges.dim() != 2 or edges.shape[1] != 2 or not edges.is_contiguous()):
            raise ValueError("edges must be a contiguous [m, 2] tensor")
        m = edges.shape[0] if edges.numel() else 0
        slot = ctypes.c_int32()
        rc = load().dl_batch_submit_edges(self._h, int(kind), int(n),
                                          ctypes.c_void_p(edges.data_ptr()) if m else None, m, int(tag),
                                          ctypes.byref(slot), _stream_ptr(self.stream))
        if rc == DL_EAGAIN:
            return None
        _check(rc)
        # the library reads the edges in the next dl_batch_step, whose scatter
        # may still be in flight on the batch's stream when that call returns
        # (look-ahead): keep a reference until then, and tell the caching
        # allocator the memory is in use on that stream, so it is not handed
        # to a new tensor before the scatter has read it
        self._pending_edges.append(edges)
        if m:
            edges.record_stream(self.stream if self.stream is not None else torch.cuda.current_stream(edges.device))
        return int(slot.value)

    def dl_batch_submit_edges_n(self, kinds, ns, edges: list, tags) -> list[int]:
        """Admit requests given as device int32 [m, 2] edge lists, in order,
        until one does not fit; returns the slots of those admitted (a prefix
        of the requests)."""
        k = len(edges)
        if not (len(kinds) == len(ns) == len(tags) == k):
            raise ValueError("one kind, size and tag per edge list")
        if k == 0:
            return []
        ptrs = (ctypes.c_void_p * k)()
        ms = (ctypes.c_int64 * k)()
        for i, e in enumerate(edges):
            if not isinstance(e, torch.Tensor) or not e.is_cuda or e.dtype != torch.int32:
                raise TypeError("edges must be device int32 tensors")
            if e.numel() and (e.dim() != 2 or e.shape[1] != 2 or not e.is_contiguous()):
                raise ValueError("edges must be contiguous [m, 2] tensors")
            ms[i] = e.shape[0] if e.numel() else 0
            ptrs[i] = e.data_ptr() if ms[i] else None
        kk = (ctypes.c_int32 * k)(*[int(x) for x in kinds])
        nn = (ctypes.c_int64 * k)(*[int(x) for x in ns])
        tt = (ctypes.c_int64 * k)(*[int(x) for x in tags])
        slots = (ctypes.c_int32 * k)()
        got = ctypes.c_int32()
        rc = load().dl_batch_submit_edges_n(self._h, k, kk, nn, ptrs, ms, tt, slots, ctypes.byref(got),
                                            _stream_ptr(self.stream))
        self._bulk_edges.extend(edges[:got.value])
        _check(rc)
        return [int(slots[i]) for i in range(got.value)]

    def dl_batch_release_n(self, slots) -> list[int]:
        """Free finished requests without copying their models; returns their
        numbers of true entries."""
        k = len(slots)
        if k == 0:
            return []
        ss = (ctypes.c_int32 * k)(*[int(x) for x in slots])
        ones = (ctypes.c_int64 * k)()
        _check(load().dl_batch_release_n(self._h, k, ss, ones))
        return [int(ones[i]) for i in range(k)]

    def tune(self, sizes: list | None = None) -> list[dict]:
        """Time the grouped step at each tile size for each request size and
        keep the fastest per size (dl_batch_tune); returns one entry per
        size: n, tile, ms per request-product for tiles 64 / 128 / 256."""
        k = len(sizes) if sizes else 10
        arr = (ctypes.c_int64 * k)(*sizes) if sizes else None
        tiles = (ctypes.c_int32 * k)()
        ms = (ctypes.c_double * (3 * k))()
        _check(load().dl_batch_tune(self._h, arr, len(sizes) if sizes else 0, tiles, ms, _stream_ptr(self.stream)))
        got = list(sizes) if sizes else [96, 128, 192, 256, 384, 512, 768, 1024, 1536, 2048]
        return [{"n": got[i], "tile": int(tiles[i]), "ms": [float(ms[3 * i + j]) for j in range(3)]}
                for i in range(k)]

    def set_tiles(self, table: list) -> None:
        """Tile table as from tune(): entries with "n" (ascending) and "tile"."""
        k = len(table)
        ns = (ctypes.c_int64 * max(k, 1))(*[int(e["n"]) for e in table])
        ts = (ctypes.c_int32 * max(k, 1))(*[int(e["tile"]) for e in table])
        _check(load().dl_batch_set_tiles(self._h, ns, ts, k))

    def dl_batch_step(self) -> tuple[int, int]:
        active = ctypes.c_int32()
        fin = ctypes.c_int32()
        try:
            _check(load().dl_batch_step(self._h, ctypes.byref(active), ctypes.byref(fin), _stream_ptr(self.stream)))
        finally:
            self._pending_edges.clear()
            # the round issued now scatters the bulk-admitted edges; it has
            # completed once the next call returns
            self._bulk_held = [self._bulk_held[1], self._bulk_edges]
            self._bulk_edges = []
        return int(active.value), int(fin.value)

    def dl_batch_poll(self) -> list[tuple[int, int, int]]:
        count = ctypes.c_int32()
        _check(load().dl_batch_poll(self._h, self._tags, self._slots, self._iters, self._cap, ctypes.byref(count)))
        return [(int(self._tags[i]), int(self._slots[i]), int(self._iters[i])) for i in range(count.value)]

    def dl_batch_fetch(self, slot: int, out: torch.Tensor | None = None) -> int:
        """Write the model of a finished request into `out` (or discard it);
        returns its number of true entries and frees the slot."""
        ones = ctypes.c_int64()
        if out is None:
            _check(load().dl_batch_fetch(self._h, int(slot), None, 0, ctypes.byref(ones), _stream_ptr(self.stream)))
        else:
            _, ldr = _mat(out, "R")
            _check(load().dl_batch_fetch(self._h, int(slot), ctypes.c_void_p(out.data_ptr()), ldr,
                                         ctypes.byref(ones), _stream_ptr(self.stream)))
        return int(ones.value)

    def dl_batch_info(self) -> tuple[int, int, int]:
        a = ctypes.c_int32()
        u = ctypes.c_int32()
        f = ctypes.c_size_t()
        _check(load().dl_batch_info(self._h, ctypes.byref(a), ctypes.byref(u), ctypes.byref(f)))
        return int(a.value), int(u.value), int(f.value)
