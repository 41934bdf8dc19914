"""MI355X (gfx950) Monte Carlo estimator of exp(tA) v (Acebron, arXiv:1904.12759).

Thin Python binding over the C ABI in include/mc_expmv.h (libmcexpmv.so, built
in-tree by ``paper_1904_12759_amd.build``).  The functions here only marshal
arguments: device memory and streams come from PyTorch tensors, and every step
of the computation runs in the library's HIP kernels.  If the library is not
built, or no GPU is present, calls raise instead of falling back to anything.
"""
from __future__ import annotations

import ctypes
import os

__all__ = ["MCExpmv", "MCBatch", "MLP", "MCError", "EXACT", "STRANG", "LIE", "FP64", "FP32", "lib",
           "load"]

HERE = os.path.dirname(os.path.abspath(__file__))
# MC_EXPMV_LIB may name another build of the library (the host-code sanitizer build,
# for CPU checks); by default the in-tree libmcexpmv.so
LIB_PATH = os.environ.get("MC_EXPMV_LIB") or os.path.join(HERE, "libmcexpmv.so")

EXACT, STRANG, LIE = 0, 1, 2
FP64, FP32 = 0, 1

MC_OK = 0
STATUS_NAMES = {
    0: "MC_OK", 1: "MC_ERR_INVALID_ARG", 2: "MC_ERR_NOT_METZLER", 3: "MC_ERR_NONFINITE",
    4: "MC_ERR_OUT_OF_RANGE", 5: "MC_ERR_NOT_SYMMETRIC", 6: "MC_ERR_NO_MEMORY",
    7: "MC_ERR_DEVICE", 8: "MC_ERR_WALK_LIMIT", 9: "MC_ERR_OVERFLOW", 10: "MC_ERR_TOO_LARGE",
}


class MCError(RuntimeError):
    def __init__(self, code: int, where: str = ""):
        msg = STATUS_NAMES.get(code, str(code))
        if _lib is not None:
            msg += ": " + _lib.mc_expmv_status_string(code).decode()
        super().__init__(f"{where}: {msg}" if where else msg)
        self.code = code


class mc_expmv_opts(ctypes.Structure):
    _fields_ = [
        ("struct_size", ctypes.c_uint32),
        ("mode", ctypes.c_int32),
        ("dt", ctypes.c_double),
        ("weight_prec", ctypes.c_int32),
        ("relabel", ctypes.c_int32),
        ("lds_budget", ctypes.c_uint32),
        ("resort_period", ctypes.c_uint32),
        ("walkers_per_block", ctypes.c_uint32),
        ("instance_id", ctypes.c_uint32),
        ("max_events", ctypes.c_uint32),
        ("stream", ctypes.c_void_p),
        ("cond_first_jump", ctypes.c_int32),
        ("cond_max_rt", ctypes.c_double),
        ("task_walkers", ctypes.c_uint32),
        ("slot_rows", ctypes.c_int32),
        ("qmc_first", ctypes.c_int32),
    ]


class mc_expmv_run_stats(ctypes.Structure):
    _fields_ = [
        ("walkers", ctypes.c_uint64),
        ("events", ctypes.c_uint64),
        ("jumps", ctypes.c_uint64),
        ("ms", ctypes.c_double),
        ("alg_bytes", ctypes.c_double),
    ]


class mc_instance_desc(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int64), ("nnz", ctypes.c_int64),
        ("rowptr", ctypes.c_void_p), ("col", ctypes.c_void_p), ("val", ctypes.c_void_p),
        ("t", ctypes.c_double), ("mode", ctypes.c_int32), ("dt", ctypes.c_double),
        ("weight_prec", ctypes.c_int32), ("instance_id", ctypes.c_uint32),
        ("v", ctypes.c_void_p), ("idx", ctypes.c_void_p), ("k", ctypes.c_int64),
        ("n_walkers", ctypes.c_int64), ("est", ctypes.c_void_p), ("stderr_", ctypes.c_void_p),
    ]


class mc_batch_opts(ctypes.Structure):
    _fields_ = [
        ("struct_size", ctypes.c_uint32), ("walkers_per_block", ctypes.c_uint32),
        ("blocks_per_cu", ctypes.c_uint32), ("group", ctypes.c_uint32),
        ("use_graph", ctypes.c_int32), ("max_events", ctypes.c_uint32),
        ("stream", ctypes.c_void_p), ("slot_rows", ctypes.c_int32),
    ]


class mc_batch_schedule(ctypes.Structure):
    _fields_ = [
        ("walkers_per_block", ctypes.c_uint32), ("blocks_per_cu", ctypes.c_uint32),
        ("group", ctypes.c_uint32), ("tasks", ctypes.c_int64),
    ]


class mc_learn_opts(ctypes.Structure):
    _fields_ = [
        ("struct_size", ctypes.c_uint32), ("pilot_walkers", ctypes.c_int64),
        ("steps", ctypes.c_int32), ("batch", ctypes.c_int64), ("lr", ctypes.c_float),
        ("seed", ctypes.c_uint64), ("params_out", ctypes.c_void_p),
    ]


class mc_learn_report(ctypes.Structure):
    _fields_ = [
        ("initial_loss", ctypes.c_float), ("final_loss", ctypes.c_float),
        ("steps", ctypes.c_int32), ("pilot_ms", ctypes.c_double), ("train_ms", ctypes.c_double),
    ]


NPARAM = 4801

_lib = None

# exported C symbols and their signatures (also checked by the CPU tests)
_SIGS = {
    "mc_expmv_default_opts": (None, [ctypes.c_void_p]),
    "mc_expmv_status_string": (ctypes.c_char_p, [ctypes.c_int]),
    "mc_expmv_create": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int64,
                                       ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                       ctypes.c_double, ctypes.c_uint64, ctypes.c_void_p]),
    "mc_expmv_create_stencil7": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int64,
                                                ctypes.c_int64] + [ctypes.c_void_p] * 4 +
                                 [ctypes.c_double, ctypes.c_uint64, ctypes.c_void_p]),
    "mc_expmv_entries": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                        ctypes.c_int64, ctypes.c_int64, ctypes.c_void_p,
                                        ctypes.c_void_p]),
    "mc_expmv_entries_noalloc": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                                ctypes.c_int64, ctypes.c_int64, ctypes.c_void_p,
                                                ctypes.c_void_p]),
    "mc_expmv_full": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                                     ctypes.c_void_p, ctypes.c_void_p]),
    "mc_expmv_entries_multi": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                              ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p,
                                              ctypes.c_void_p]),
    "mc_expmv_entries_to_target": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                                  ctypes.c_int64, ctypes.c_int64, ctypes.c_double,
                                                  ctypes.c_double, ctypes.c_int64, ctypes.c_int64,
                                                  ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "mc_expmv_forward": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                                        ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "mc_expmv_forward_trace": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                                              ctypes.c_int64] + [ctypes.c_void_p] * 5),
    "mc_expmv_set_proposal": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    "mc_expmv_get_proposal": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    "mc_expmv_sync": (ctypes.c_int, [ctypes.c_void_p]),
    "mc_expmv_stats": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    "mc_expmv_trace": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                                      ctypes.c_int64, ctypes.c_int64, ctypes.c_int32,
                                      ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                      ctypes.c_void_p]),
    "mc_expmv_get_tables": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32] + [ctypes.c_void_p] * 8),
    "mc_expmv_get_stencil": (ctypes.c_int, [ctypes.c_void_p] * 5),
    "mc_expmv_info": (ctypes.c_int, [ctypes.c_void_p] * 5),
    "mc_expmv_set_stream": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    "mc_expmv_destroy": (None, [ctypes.c_void_p]),
    "mc_batch_default_opts": (None, [ctypes.c_void_p]),
    "mc_expmv_batch_create": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p,
                                             ctypes.c_uint64, ctypes.c_void_p]),
    "mc_expmv_batch_run": (ctypes.c_int, [ctypes.c_void_p]),
    "mc_expmv_batch_sync": (ctypes.c_int, [ctypes.c_void_p]),
    "mc_expmv_batch_stats": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "mc_expmv_batch_set_schedule": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    "mc_expmv_batch_destroy": (None, [ctypes.c_void_p]),
    "mc_mlp_create": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_void_p]),
    "mc_mlp_destroy": (None, [ctypes.c_void_p]),
    "mc_mlp_get_params": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    "mc_mlp_set_params": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    "mc_mlp_features": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "mc_mlp_log_h": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                    ctypes.c_int64, ctypes.c_void_p]),
    "mc_mlp_forward": (ctypes.c_int, [ctypes.c_void_p] * 4),
    "mc_mlp_gradient": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                       ctypes.c_void_p, ctypes.c_int64, ctypes.c_int64,
                                       ctypes.c_void_p, ctypes.c_void_p]),
    "mc_mlp_adam_step": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_float]),
    "mc_mlp_train": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                    ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64,
                                    ctypes.c_float, ctypes.c_void_p]),
    "mc_learn_default_opts": (None, [ctypes.c_void_p]),
    "mc_expmv_learn_proposal": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p,
                                               ctypes.c_void_p, ctypes.c_void_p]),
    "mc_math_eval": (ctypes.c_int, [ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p,
                                    ctypes.c_int64, ctypes.c_void_p]),
    "mc_isim": (ctypes.c_int, [ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                               ctypes.c_void_p, ctypes.c_void_p]),
}


def load() -> ctypes.CDLL:
    """Load libmcexpmv.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run python -m paper_1904_12759_amd.build")
        lib = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def lib() -> ctypes.CDLL:
    return load()


def _check(code: int, where: str):
    if code != MC_OK:
        raise MCError(code, where)


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _require_cuda(*tensors):
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("libmcexpmv needs a HIP device; none is available")
    for t in tensors:
        if t is not None and not t.is_cuda:
            raise ValueError("all arrays must be device tensors")


def default_opts(**kw) -> mc_expmv_opts:
    o = mc_expmv_opts()
    load().mc_expmv_default_opts(ctypes.byref(o))
    for k, v in kw.items():
        if k == "stream":
            v = ctypes.c_void_p(v)
        setattr(o, k, v)
    return o


def isim(x, y, k: int | None = None, stream=None) -> float:
    """Intersection similarity isim_K of the rankings of x and y (``mc_isim``); x and
    y are device tensors (or arrays, copied to the device) of one length n, K = k or n."""
    import torch
    dev = torch.device("cuda", torch.cuda.current_device())
    xs = torch.as_tensor(x).to(device=dev, dtype=torch.float64).contiguous()
    ys = torch.as_tensor(y).to(device=dev, dtype=torch.float64).contiguous()
    if xs.shape != ys.shape or xs.dim() != 1:
        raise ValueError("x and y must be vectors of one length")
    n = xs.numel()
    k = n if k is None else int(k)
    if stream is None:
        stream = torch.cuda.current_stream().cuda_stream
    out = ctypes.c_double()
    _check(load().mc_isim(n, _ptr(xs), _ptr(ys), k, ctypes.byref(out), ctypes.c_void_p(stream)),
           "mc_isim")
    return out.value


MATH_FNS = {"log": 0, "exp": 1, "one_minus_exp_neg": 2, "exp_f32": 3}


def math_eval(fn: str, x):
    """The walk kernels' own FP64 log / exp / 1 - e^{-x} and FP32 exp on a vector (``mc_math_eval``),
    returned as a device tensor."""
    import torch
    dev = torch.device("cuda", torch.cuda.current_device())
    xs = torch.as_tensor(x).to(device=dev, dtype=torch.float64).contiguous()
    ys = torch.empty_like(xs)
    stream = torch.cuda.current_stream().cuda_stream
    _check(load().mc_math_eval(MATH_FNS[fn], _ptr(xs), _ptr(ys), xs.numel(),
                               ctypes.c_void_p(stream)), "mc_math_eval")
    return ys


class MCExpmv:
    """Handle over ``mc_expmv_create`` for one matrix A, horizon t and seed.

    rowptr/col/val may be numpy arrays or torch tensors; they are copied to the
    device.  Every call runs on the current torch stream at creation time
    (change it with :meth:`set_stream`)."""

    def __init__(self, rowptr, col, val, t: float, seed: int, mode: int = EXACT,
                 dt: float = 0.03125, fp32: bool = False, instance: int = 0,
                 max_events: int = 0, walkers_per_block: int = 64, relabel: int = 0,
                 lds_budget: int = 0, stream=None, cond: bool = False,
                 cond_max_rt: float = float("inf"), task_walkers: int = 0,
                 resort_period: int = 0, slot_rows: int = 0, qmc: bool = False):
        import torch
        lib_ = load()
        dev = torch.device("cuda", torch.cuda.current_device())
        rp = torch.as_tensor(rowptr, dtype=torch.int64).to(dev).contiguous()
        cl = torch.as_tensor(col, dtype=torch.int32).to(dev).contiguous()
        vl = torch.as_tensor(val, dtype=torch.float64).to(dev).contiguous()
        _require_cuda(rp, cl, vl)
        if stream is None:
            stream = torch.cuda.current_stream().cuda_stream
        self.stream = stream
        opts = default_opts(mode=mode, dt=dt, weight_prec=FP32 if fp32 else FP64,
                            instance_id=instance, max_events=max_events,
                            walkers_per_block=walkers_per_block, relabel=relabel,
                            lds_budget=lds_budget, stream=stream, cond_first_jump=int(cond),
                            cond_max_rt=float(cond_max_rt), task_walkers=int(task_walkers),
                            resort_period=int(resort_period), slot_rows=int(slot_rows),
                            qmc_first=int(qmc))
        h = ctypes.c_void_p()
        torch.cuda.current_stream().synchronize()
        _check(lib_.mc_expmv_create(ctypes.byref(h), rp.numel() - 1, cl.numel(), _ptr(rp),
                                    _ptr(cl), _ptr(vl), float(t), int(seed) & (2**64 - 1),
                                    ctypes.byref(opts)), "mc_expmv_create")
        self._h = h
        self.n = rp.numel() - 1
        self.nnz = cl.numel()
        self.t = float(t)
        self.mode = mode
        self.fp32 = fp32
        self.device = dev
        n, ns, ng, dtv = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64(), ctypes.c_double()
        _check(lib_.mc_expmv_info(h, ctypes.byref(n), ctypes.byref(ns), ctypes.byref(ng),
                                  ctypes.byref(dtv)), "mc_expmv_info")
        self.nslots, self.ngrid, self.dt = ns.value, ng.value, dtv.value

    @classmethod
    def stencil7(cls, nx, ny, nz, fx, fy, fz, diag, t: float, seed: int, mode: int = EXACT,
                 dt: float = 0.03125, fp32: bool = False, instance: int = 0,
                 max_events: int = 0, walkers_per_block: int = 64, stream=None,
                 task_walkers: int = 0):
        """Handle over ``mc_expmv_create_stencil7``: the matrix-free walk on a 7-point
        stencil given by its face rates fx, fy, fz (rate to the +x / +y / +z neighbour,
        0 on the last plane) and diagonal."""
        import torch
        lib_ = load()
        dev = torch.device("cuda", torch.cuda.current_device())
        arrs = [torch.as_tensor(a, dtype=torch.float64).to(dev).contiguous()
                for a in (fx, fy, fz, diag)]
        _require_cuda(*arrs)
        if stream is None:
            stream = torch.cuda.current_stream().cuda_stream
        self = cls.__new__(cls)
        self.stream = stream
        opts = default_opts(mode=mode, dt=dt, weight_prec=FP32 if fp32 else FP64,
                            instance_id=instance, max_events=max_events,
                            walkers_per_block=walkers_per_block, stream=stream,
                            task_walkers=int(task_walkers))
        h = ctypes.c_void_p()
        torch.cuda.current_stream().synchronize()
        _check(lib_.mc_expmv_create_stencil7(ctypes.byref(h), int(nx), int(ny), int(nz),
                                             *[_ptr(a) for a in arrs], float(t),
                                             int(seed) & (2**64 - 1), ctypes.byref(opts)),
               "mc_expmv_create_stencil7")
        self._h = h
        self.n = int(nx) * int(ny) * int(nz)
        self.nnz = 0
        self.t = float(t)
        self.mode = mode
        self.fp32 = fp32
        self.device = dev
        n, ns, ng, dtv = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64(), ctypes.c_double()
        _check(lib_.mc_expmv_info(h, ctypes.byref(n), ctypes.byref(ns), ctypes.byref(ng),
                                  ctypes.byref(dtv)), "mc_expmv_info")
        self.nslots, self.ngrid, self.dt = ns.value, ng.value, dtv.value
        return self

    # -- plumbing
    def close(self):
        if getattr(self, "_h", None):
            load().mc_expmv_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_stream(self, stream):
        _check(load().mc_expmv_set_stream(self._h, ctypes.c_void_p(stream)), "mc_expmv_set_stream")
        self.stream = stream

    def _v(self, v):
        import torch
        dt = torch.float32 if self.fp32 else torch.float64
        v = torch.as_tensor(v)
        v = v.to(device=self.device, dtype=dt).contiguous()
        if v.numel() != self.n:
            raise ValueError("v must have n entries")
        return v

    # -- estimator
    def entries(self, v, idx, n_walkers: int, est=None, stderr=None, sync: bool = True):
        import torch
        v = self._v(v)
        idx = torch.as_tensor(idx).to(device=self.device, dtype=torch.int64).contiguous()
        k = idx.numel()
        if est is None:
            est = torch.empty(k, dtype=torch.float64, device=self.device)
        if stderr is None:
            stderr = torch.empty(k, dtype=torch.float64, device=self.device)
        _require_cuda(v, idx, est, stderr)
        _check(load().mc_expmv_entries(self._h, _ptr(v), _ptr(idx), k, int(n_walkers),
                                       _ptr(est), _ptr(stderr)), "mc_expmv_entries")
        if sync:
            self.sync()
        return est, stderr

    def entries_noalloc(self, v, idx, n_walkers: int, est, stderr=None, sync: bool = True):
        """mc_expmv_entries_noalloc: as entries(), the library allocating nothing (its
        partials in a fixed static device array).  v, idx, est (and stderr) must be
        device tensors already."""
        _require_cuda(v, idx, est, *([stderr] if stderr is not None else []))
        _check(load().mc_expmv_entries_noalloc(self._h, _ptr(v), _ptr(idx), idx.numel(),
                                               int(n_walkers), _ptr(est), _ptr(stderr)),
               "mc_expmv_entries_noalloc")
        if sync:
            self.sync()
        return est, stderr

    def entries_multi(self, v, idx, n_walkers, est=None, stderr=None, sync: bool = True):
        """Entries idx with their own walker counts n_walkers (one launch)."""
        import numpy as np
        import torch
        v = self._v(v)
        idx = torch.as_tensor(idx).to(device=self.device, dtype=torch.int64).contiguous()
        k = idx.numel()
        counts = np.ascontiguousarray(n_walkers, dtype=np.int64)
        if counts.shape != (k,):
            raise ValueError("n_walkers must have one count per entry")
        if est is None:
            est = torch.empty(k, dtype=torch.float64, device=self.device)
        if stderr is None:
            stderr = torch.empty(k, dtype=torch.float64, device=self.device)
        _require_cuda(v, idx, est, stderr)
        _check(load().mc_expmv_entries_multi(self._h, _ptr(v), _ptr(idx), k,
                                             counts.ctypes.data_as(ctypes.c_void_p), _ptr(est),
                                             _ptr(stderr)), "mc_expmv_entries_multi")
        if sync:
            self.sync()
        return est, stderr

    def entries_to_target(self, v, idx, pilot_walkers: int, target: float = 1e-3,
                          margin: float = 1.2, min_walkers: int = 2, max_walkers: int = 1 << 26,
                          est=None, stderr=None, walkers=None, sync: bool = True):
        """Entries to a relative standard error target, pilot and production on the
        device (mc_expmv_entries_to_target): returns (est, stderr, walkers per entry)."""
        import torch
        v = self._v(v)
        idx = torch.as_tensor(idx).to(device=self.device, dtype=torch.int64).contiguous()
        k = idx.numel()
        if est is None:
            est = torch.empty(k, dtype=torch.float64, device=self.device)
        if stderr is None:
            stderr = torch.empty(k, dtype=torch.float64, device=self.device)
        if walkers is None:
            walkers = torch.empty(k, dtype=torch.int64, device=self.device)
        _require_cuda(v, idx, est, stderr, walkers)
        _check(load().mc_expmv_entries_to_target(self._h, _ptr(v), _ptr(idx), k, int(pilot_walkers),
                                                 float(target), float(margin), int(min_walkers),
                                                 int(max_walkers), _ptr(est), _ptr(stderr),
                                                 _ptr(walkers)), "mc_expmv_entries_to_target")
        if sync:
            self.sync()
        return est, stderr, walkers

    def full(self, v, n_per_node: int, est=None, stderr=None, sync: bool = True):
        import torch
        v = self._v(v)
        if est is None:
            est = torch.empty(self.n, dtype=torch.float64, device=self.device)
        if stderr is None:
            stderr = torch.empty(self.n, dtype=torch.float64, device=self.device)
        _require_cuda(v, est, stderr)
        _check(load().mc_expmv_full(self._h, _ptr(v), int(n_per_node), _ptr(est), _ptr(stderr)),
               "mc_expmv_full")
        if sync:
            self.sync()
        return est, stderr

    def forward(self, v, n_walkers: int, est=None, stderr=None, total=None, sync: bool = True,
                total_only: bool = False):
        """Forward estimator (Lemma 2, Theorem 2, Algorithm 2; A must be symmetric):
        per-node mean and standard error, and a device double[2] with the mean of the
        walker values (an estimate of sum_i x_i) and its standard error.  With
        total_only=True only the latter is computed (est and stderr are None)."""
        import torch
        v = self._v(v)
        if est is None and not total_only:
            est = torch.empty(self.n, dtype=torch.float64, device=self.device)
        if stderr is None and not total_only:
            stderr = torch.empty(self.n, dtype=torch.float64, device=self.device)
        if total is None:
            total = torch.empty(2, dtype=torch.float64, device=self.device)
        _require_cuda(*[x for x in (v, est, stderr, total) if x is not None])
        _check(load().mc_expmv_forward(self._h, _ptr(v), int(n_walkers), _ptr(est), _ptr(stderr),
                                       _ptr(total)), "mc_expmv_forward")
        if sync:
            self.sync()
        return est, stderr, total

    def forward_trace(self, v, w0: int, count: int):
        """Per-walker (start, end, events, jumps, Y) of forward walkers w0..w0+count-1."""
        import torch
        v = self._v(v)
        d = self.device
        st = torch.empty(count, dtype=torch.int32, device=d)
        en = torch.empty(count, dtype=torch.int32, device=d)
        ev = torch.empty(count, dtype=torch.int32, device=d)
        ju = torch.empty(count, dtype=torch.int32, device=d)
        y = torch.empty(count, dtype=torch.float64, device=d)
        _check(load().mc_expmv_forward_trace(self._h, _ptr(v), int(w0), int(count), _ptr(st),
                                             _ptr(en), _ptr(ev), _ptr(ju), _ptr(y)),
               "mc_expmv_forward_trace")
        self.sync()
        return (st.cpu().numpy(), en.cpu().numpy(), ev.cpu().numpy().view("uint32"),
                ju.cpu().numpy().view("uint32"), y.cpu().numpy())

    def set_proposal(self, edge_bias):
        import torch
        if edge_bias is None:
            _check(load().mc_expmv_set_proposal(self._h, None), "mc_expmv_set_proposal")
            return
        b = torch.as_tensor(edge_bias).to(device=self.device, dtype=torch.float32).contiguous()
        if b.numel() != self.nnz:
            raise ValueError("edge_bias must have nnz entries (CSR order)")
        _check(load().mc_expmv_set_proposal(self._h, _ptr(b)), "mc_expmv_set_proposal")

    def get_proposal(self):
        import torch
        b = torch.empty(self.nnz, dtype=torch.float32, device=self.device)
        _check(load().mc_expmv_get_proposal(self._h, _ptr(b)), "mc_expmv_get_proposal")
        return b

    def sync(self):
        _check(load().mc_expmv_sync(self._h), "mc_expmv_sync")

    def learn_proposal(self, v, pilot_walkers: int = 256, steps: int = 400, batch: int = 1 << 16,
                       lr: float = 3e-3, seed: int = 1) -> dict:
        """Train the proposal network on the GPU and install the tilted walk.  The
        returned dict holds the trained FP32 parameters under "params"."""
        import numpy as np
        v = self._v(v)
        o = mc_learn_opts()
        load().mc_learn_default_opts(ctypes.byref(o))
        o.pilot_walkers, o.steps, o.batch, o.lr, o.seed = pilot_walkers, steps, batch, lr, seed
        params = np.zeros(NPARAM, np.float32)
        o.params_out = params.ctypes.data_as(ctypes.c_void_p)
        rep = mc_learn_report()
        _check(load().mc_expmv_learn_proposal(self._h, _ptr(v), ctypes.byref(o), ctypes.byref(rep)),
               "mc_expmv_learn_proposal")
        return dict(initial_loss=rep.initial_loss, final_loss=rep.final_loss, steps=rep.steps,
                    pilot_ms=rep.pilot_ms, train_ms=rep.train_ms, params=params)

    def features(self, v):
        import torch
        v = self._v(v)
        f = torch.empty(self.n, 4, dtype=torch.float32, device=self.device)
        _check(load().mc_mlp_features(self._h, _ptr(v), _ptr(f)), "mc_mlp_features")
        return f

    def log_h(self, est, stderr, n_walkers: int):
        import torch
        lh = torch.empty(self.n, dtype=torch.float32, device=self.device)
        _check(load().mc_mlp_log_h(self._h, _ptr(est), _ptr(stderr), int(n_walkers), _ptr(lh)),
               "mc_mlp_log_h")
        self.sync()
        return lh

    def stats(self) -> dict:
        s = mc_expmv_run_stats()
        _check(load().mc_expmv_stats(self._h, ctypes.byref(s)), "mc_expmv_stats")
        return dict(walkers=s.walkers, events=s.events, jumps=s.jumps, ms=s.ms,
                    alg_bytes=s.alg_bytes)

    def trace(self, v, start: int, w0: int, count: int, proposal: bool = False):
        import torch
        v = self._v(v)
        d = self.device
        x = torch.empty(count, dtype=torch.int32, device=d)
        ev = torch.empty(count, dtype=torch.int32, device=d)
        ju = torch.empty(count, dtype=torch.int32, device=d)
        f = torch.empty(count, dtype=torch.float64, device=d)
        _check(load().mc_expmv_trace(self._h, _ptr(v), int(start), int(w0), int(count),
                                     int(proposal), _ptr(x), _ptr(ev), _ptr(ju), _ptr(f)),
               "mc_expmv_trace")
        return x.cpu().numpy(), ev.cpu().numpy().view("uint32"), ju.cpu().numpy().view("uint32"), \
            f.cpu().numpy()

    def tables(self, proposal: bool = False) -> dict:
        import numpy as np
        n, ns = self.n, self.nslots
        out = dict(r=np.zeros(n), d=np.zeros(n), inv_r=np.zeros(n), deg=np.zeros(n, np.int64),
                   begin=np.zeros(n, np.int64), col=np.zeros(max(ns, 1), np.int32),
                   thr=np.zeros(max(ns, 1), np.uint32), alias=np.zeros(max(ns, 1), np.int32))
        p = lambda a: a.ctypes.data_as(ctypes.c_void_p)  # noqa: E731
        _check(load().mc_expmv_get_tables(self._h, int(proposal), *[p(out[k]) for k in (
            "r", "d", "inv_r", "deg", "begin", "col", "thr", "alias")]), "mc_expmv_get_tables")
        for k in ("col", "thr", "alias"):
            out[k] = out[k][:ns]
        return out

    def stencil_records(self) -> dict:
        """A stencil handle's state records (host copies): d, inv_r, the face word
        and the five jump thresholds per node (shape (n, 5))."""
        import numpy as np
        n = self.n
        out = dict(d=np.zeros(n), inv_r=np.zeros(n), faces=np.zeros(n, np.uint32),
                   thr=np.zeros((n, 5), np.uint32))
        p = lambda a: a.ctypes.data_as(ctypes.c_void_p)  # noqa: E731
        _check(load().mc_expmv_get_stencil(self._h, *[p(out[k]) for k in (
            "d", "inv_r", "faces", "thr")]), "mc_expmv_get_stencil")
        return out


class MCBatch:
    """Many instances in one persistent, graph-captured launch (``mc_expmv_batch_*``).

    ``instances`` is a list of dicts with keys: rowptr, col, val (CSR, host or
    device), t, v, and optionally idx (entries; None for the full vector),
    n_walkers, mode, dt, fp32, instance_id.  Device copies of every buffer are
    owned by this object; results land in ``est[i]`` / ``stderr[i]``."""

    def __init__(self, instances, seed: int, walkers_per_block: int = 0,
                 blocks_per_cu: int = 0, group: int = 0, use_graph: bool = True,
                 max_events: int = 0, stream=None, slot_rows: int = 0):
        import torch
        lib_ = load()
        dev = torch.device("cuda", torch.cuda.current_device())
        self.device = dev
        self._keep = []
        self.est, self.stderr = [], []
        descs = (mc_instance_desc * len(instances))()
        for i, inst in enumerate(instances):
            rp = torch.as_tensor(inst["rowptr"], dtype=torch.int64).to(dev).contiguous()
            cl = torch.as_tensor(inst["col"], dtype=torch.int32).to(dev).contiguous()
            vl = torch.as_tensor(inst["val"], dtype=torch.float64).to(dev).contiguous()
            fp32 = bool(inst.get("fp32", False))
            v = torch.as_tensor(inst["v"]).to(device=dev, dtype=torch.float32 if fp32 else
                                               torch.float64).contiguous()
            n = rp.numel() - 1
            idx = inst.get("idx")
            if idx is not None:
                idx = torch.as_tensor(idx).to(device=dev, dtype=torch.int64).contiguous()
                k = idx.numel()
            else:
                k = n
            est = torch.empty(k, dtype=torch.float64, device=dev)
            se = torch.empty(k, dtype=torch.float64, device=dev)
            self._keep += [rp, cl, vl, v, idx]
            self.est.append(est)
            self.stderr.append(se)
            d = descs[i]
            d.n, d.nnz = n, cl.numel()
            d.rowptr, d.col, d.val = rp.data_ptr(), cl.data_ptr(), vl.data_ptr()
            d.t = float(inst["t"])
            d.mode = int(inst.get("mode", EXACT))
            d.dt = float(inst.get("dt", 0.03125))
            d.weight_prec = FP32 if fp32 else FP64
            d.instance_id = int(inst.get("instance_id", i))
            d.v = v.data_ptr()
            d.idx = idx.data_ptr() if idx is not None else None
            d.k = k if idx is not None else 0
            d.n_walkers = int(inst["n_walkers"])
            d.est, d.stderr_ = est.data_ptr(), se.data_ptr()
        o = mc_batch_opts()
        lib_.mc_batch_default_opts(ctypes.byref(o))
        o.walkers_per_block, o.blocks_per_cu, o.group = walkers_per_block, blocks_per_cu, group
        o.use_graph = 1 if use_graph else 0
        o.max_events = max_events
        o.slot_rows = int(slot_rows)
        if stream is None:
            stream = torch.cuda.current_stream().cuda_stream
        o.stream = stream
        torch.cuda.current_stream().synchronize()
        h = ctypes.c_void_p()
        _check(lib_.mc_expmv_batch_create(ctypes.byref(h), len(instances), descs,
                                          int(seed) & (2**64 - 1), ctypes.byref(o)),
               "mc_expmv_batch_create")
        self._h = h

    def run(self, sync: bool = True):
        _check(load().mc_expmv_batch_run(self._h), "mc_expmv_batch_run")
        if sync:
            self.sync()
        return self.est, self.stderr

    def sync(self):
        _check(load().mc_expmv_batch_sync(self._h), "mc_expmv_batch_sync")

    def schedule(self) -> dict:
        sc = mc_batch_schedule()
        _check(load().mc_expmv_batch_stats(self._h, None, ctypes.byref(sc)), "mc_expmv_batch_stats")
        return dict(walkers_per_block=sc.walkers_per_block, blocks_per_cu=sc.blocks_per_cu,
                    group=sc.group, tasks=sc.tasks)

    def set_schedule(self, walkers_per_block: int, blocks_per_cu: int, group: int):
        sc = mc_batch_schedule(walkers_per_block, blocks_per_cu, group, 0)
        _check(load().mc_expmv_batch_set_schedule(self._h, ctypes.byref(sc)),
               "mc_expmv_batch_set_schedule")

    def stats(self) -> dict:
        s = mc_expmv_run_stats()
        _check(load().mc_expmv_batch_stats(self._h, ctypes.byref(s), None), "mc_expmv_batch_stats")
        return dict(walkers=s.walkers, events=s.events, jumps=s.jumps, ms=s.ms,
                    alg_bytes=s.alg_bytes)

    def close(self):
        if getattr(self, "_h", None):
            load().mc_expmv_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class MLP:
    """The proposal network (``mc_mlp_*``), bound to one MCExpmv handle's matrix."""

    def __init__(self, handle: MCExpmv, seed: int = 1):
        import torch
        self.h = handle
        m = ctypes.c_void_p()
        _check(load().mc_mlp_create(ctypes.byref(m), int(seed), ctypes.c_void_p(handle.stream)),
               "mc_mlp_create")
        self._m = m
        self.device = handle.device
        self._grad = torch.empty(NPARAM, dtype=torch.float32, device=self.device)
        self._loss = torch.empty(1, dtype=torch.float32, device=self.device)

    def close(self):
        if getattr(self, "_m", None):
            load().mc_mlp_destroy(self._m)
            self._m = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def params(self):
        import numpy as np
        out = np.zeros(NPARAM, np.float32)
        _check(load().mc_mlp_get_params(self._m, out.ctypes.data_as(ctypes.c_void_p)),
               "mc_mlp_get_params")
        return out

    def set_params(self, p):
        import numpy as np
        p = np.ascontiguousarray(p, dtype=np.float32)
        assert p.shape == (NPARAM,)
        _check(load().mc_mlp_set_params(self._m, p.ctypes.data_as(ctypes.c_void_p)),
               "mc_mlp_set_params")

    def forward(self, feats, handle: "MCExpmv | None" = None):
        """Tilts for every CSR position of `handle`'s matrix (default: the bound one),
        from that matrix's node features."""
        import torch
        h = handle or self.h
        b = torch.empty(h.nnz, dtype=torch.float32, device=h.device)
        _check(load().mc_mlp_forward(self._m, h._h, _ptr(feats), _ptr(b)), "mc_mlp_forward")
        h.sync()
        return b

    def gradient(self, feats, lh, p0: int, p1: int):
        _check(load().mc_mlp_gradient(self._m, self.h._h, _ptr(feats), _ptr(lh), int(p0), int(p1),
                                      _ptr(self._grad), _ptr(self._loss)), "mc_mlp_gradient")
        self.h.sync()
        return self._grad.clone(), float(self._loss.item())

    def adam_step(self, grad, lr: float):
        _check(load().mc_mlp_adam_step(self._m, _ptr(grad), float(lr)), "mc_mlp_adam_step")
        self.h.sync()

    def train(self, feats, lh, steps: int, batch: int, lr: float):
        import numpy as np
        loss = np.zeros(steps, np.float32)
        _check(load().mc_mlp_train(self._m, self.h._h, _ptr(feats), _ptr(lh), int(steps),
                                   int(batch), float(lr), loss.ctypes.data_as(ctypes.c_void_p)),
               "mc_mlp_train")
        return loss
