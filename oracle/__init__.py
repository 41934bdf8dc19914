"""CPU FP64 oracle for the Monte Carlo estimator of exp(tA) v (arXiv:1904.12759).

TEST INFRASTRUCTURE ONLY: imported by the tests, by the smoke check and by the
CPU-baseline leg of the benchmark.  The HIP library never loads it and it never
loads the HIP library; the two share no code.

`Oracle` wraps the plain C implementation in ``oracle.c`` (built with gcc by
:func:`build`).  The dense and closed-form references that pin it live with the
tests (``tests/refs.py``); the FP64 MLP used to check the learned-proposal
kernels lives in ``oracle.mlp`` and the ranking measure in ``oracle.rank``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

EXACT, STRANG, LIE = 0, 1, 2

STATUS = {
    0: "ok",
    1: "invalid argument",
    2: "negative off-diagonal entry",
    3: "non-finite value",
    4: "index out of range",
    6: "out of memory",
    8: "walk-length cap reached",
    9: "weight overflow",
}


class OracleError(RuntimeError):
    def __init__(self, code: int):
        super().__init__(f"oracle error {code}: {STATUS.get(code, '?')}")
        self.code = code


def build(force: bool = False) -> str:
    """Compile oracle.c into liboracle.so with gcc (plain C11, no FP contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call([
            "gcc", "-std=c11", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
            "-pthread", _SRC, "-o", tmp, "-lm",
        ])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        # ORACLE_LIB names another build of oracle.c to load instead (the
        # planted-mistake tests load deliberately broken builds this way)
        path = os.environ.get("ORACLE_LIB") or build()
        lib = ctypes.CDLL(path)
        vp, i64, u64, u32, i32, dbl = (ctypes.c_void_p, ctypes.c_int64, ctypes.c_uint64,
                                       ctypes.c_uint32, ctypes.c_int, ctypes.c_double)
        lib.oracle_create.argtypes = [ctypes.POINTER(vp), i64, i64, vp, vp, vp, dbl, u64, i32,
                                      dbl, u32, u32]
        lib.oracle_create.restype = i32
        lib.oracle_destroy.argtypes = [vp]
        lib.oracle_destroy.restype = None
        lib.oracle_set_proposal.argtypes = [vp, vp, vp, vp, vp]
        lib.oracle_set_proposal.restype = i32
        lib.oracle_trace.argtypes = [vp, vp, i64, u32, i64, i32, vp, vp, vp, vp, vp]
        lib.oracle_trace.restype = i32
        lib.oracle_estimate.argtypes = [vp, vp, vp, i64, i64, i32, i32, vp, vp, vp, vp]
        lib.oracle_estimate.restype = i32
        lib.oracle_nslots.argtypes = [vp]
        lib.oracle_nslots.restype = i64
        lib.oracle_ngrid.argtypes = [vp]
        lib.oracle_ngrid.restype = i64
        lib.oracle_dt.argtypes = [vp]
        lib.oracle_dt.restype = dbl
        lib.oracle_get_tables.argtypes = [vp, i32] + [vp] * 9
        lib.oracle_get_tables.restype = i32
        lib.oracle_set_conditioning.argtypes = [vp, i32, dbl]
        lib.oracle_set_conditioning.restype = i32
        lib.oracle_set_qmc.argtypes = [vp, i32, i32]
        lib.oracle_set_qmc.restype = i32
        lib.oracle_set_jump_rule.argtypes = [vp, i32]
        lib.oracle_set_jump_rule.restype = i32
        lib.oracle_forward.argtypes = [vp, vp, i64, i32, vp, vp, vp, vp, vp, vp, vp, vp, vp]
        lib.oracle_forward.restype = i32
        lib.oracle_philox4x32_10.argtypes = [vp, vp, vp]
        lib.oracle_philox4x32_10.restype = None
        _lib = lib
    return _lib


def _p(a: np.ndarray | None):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def philox4x32_10(counter, key) -> np.ndarray:
    """Philox4x32-10 of one 128-bit counter (4 words) under a 64-bit key (2 words)."""
    lib = _load()
    c = np.ascontiguousarray(counter, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib.oracle_philox4x32_10(_p(c), _p(k), _p(out))
    return out


class Oracle:
    """The oracle for one matrix A (CSR), horizon t, seed and weight mode."""

    def __init__(self, rowptr, col, val, t: float, seed: int, mode: int = EXACT,
                 dt: float = 0.03125, instance: int = 0, max_events: int = 0,
                 cond: bool = False, cond_max_rt: float = float("inf"), qmc: bool = False,
                 qmc_bits: int = 9, cdf_jump: bool = False):
        lib = _load()
        self._rowptr = np.ascontiguousarray(rowptr, dtype=np.int64)
        self._col = np.ascontiguousarray(col, dtype=np.int32)
        self._val = np.ascontiguousarray(val, dtype=np.float64)
        self.n = len(self._rowptr) - 1
        self.nnz = len(self._col)
        self.t = float(t)
        self.mode = mode
        h = ctypes.c_void_p()
        st = lib.oracle_create(ctypes.byref(h), self.n, self.nnz, _p(self._rowptr),
                               _p(self._col), _p(self._val), float(t), int(seed) & (2**64 - 1),
                               int(mode), float(dt), int(instance), int(max_events))
        if st != 0:
            raise OracleError(st)
        self._h = h
        self.nslots = int(lib.oracle_nslots(h))
        self.ngrid = int(lib.oracle_ngrid(h))
        self.dt = float(lib.oracle_dt(h))
        self.has_proposal = False
        self.cond = bool(cond)
        lib.oracle_set_conditioning(h, int(self.cond), float(cond_max_rt))
        self.qmc = bool(qmc)
        st = lib.oracle_set_qmc(h, int(self.qmc), int(qmc_bits))
        if st == 0:
            st = lib.oracle_set_jump_rule(h, int(bool(cdf_jump)))
        if st != 0:
            raise OracleError(st)

    def close(self):
        if getattr(self, "_h", None):
            _load().oracle_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_proposal(self, bias):
        """Tilted jump rates a_ij*exp(b_ij); bias has one float32 per CSR position."""
        if bias is None:
            st = _load().oracle_set_proposal(self._h, None, None, None, None)
            self.has_proposal = False
        else:
            b = np.ascontiguousarray(bias, dtype=np.float32)
            assert b.shape == (self.nnz,)
            st = _load().oracle_set_proposal(self._h, _p(self._rowptr), _p(self._col),
                                             _p(self._val), _p(b))
            self.has_proposal = st == 0
        if st != 0:
            raise OracleError(st)

    def trace(self, v, start: int, w0: int, count: int, proposal: bool = False):
        """Per-walker (x_end, events, jumps, f, logw) for walkers w0..w0+count-1 of `start`."""
        v = np.ascontiguousarray(v, dtype=np.float64)
        x = np.zeros(count, np.int32)
        ev = np.zeros(count, np.uint32)
        ju = np.zeros(count, np.uint32)
        f = np.zeros(count, np.float64)
        lw = np.zeros(count, np.float64)
        st = _load().oracle_trace(self._h, _p(v), int(start), int(w0), int(count),
                                  int(proposal), _p(x), _p(ev), _p(ju), _p(f), _p(lw))
        if st != 0:
            raise OracleError(st)
        return x, ev, ju, f, lw

    def estimate(self, v, idx=None, nwalk: int = 1000, proposal: bool = False,
                 threads: int = 1, counts: bool = False):
        """Mean and standard error of entries idx (all nodes if None) of exp(tA) v."""
        v = np.ascontiguousarray(v, dtype=np.float64)
        if idx is None:
            k = self.n
            ip = None
        else:
            ip = np.ascontiguousarray(idx, dtype=np.int64)
            k = len(ip)
        est = np.zeros(k, np.float64)
        se = np.zeros(k, np.float64)
        ev = np.zeros(k, np.uint64)
        ju = np.zeros(k, np.uint64)
        st = _load().oracle_estimate(self._h, _p(v), _p(ip), k, int(nwalk), int(proposal),
                                     int(threads), _p(est), _p(se), _p(ev), _p(ju))
        if st != 0:
            raise OracleError(st)
        if counts:
            return est, se, ev, ju
        return est, se

    def forward(self, v, nwalk: int, walkers: bool = False):
        """Forward estimator (Lemma 2, Theorem 2): per-node mean and standard error, the
        mean of the walker values Y and its standard error, and with walkers=True the
        per-walker (start, end, events, jumps, Y)."""
        v = np.ascontiguousarray(v, dtype=np.float64)
        n = self.n
        est = np.zeros(n)
        se = np.zeros(n)
        tot = np.zeros(2)
        per = (np.zeros(nwalk, np.int32), np.zeros(nwalk, np.int32), np.zeros(nwalk, np.uint32),
               np.zeros(nwalk, np.uint32), np.zeros(nwalk)) if walkers else (None,) * 5
        st = _load().oracle_forward(self._h, _p(v), int(nwalk), 0, _p(est), _p(se), _p(tot[0:1]),
                                    _p(tot[1:2]), *[_p(a) for a in per])
        if st != 0:
            raise OracleError(st)
        out = (est, se, float(tot[0]), float(tot[1]))
        return out + (per,) if walkers else out

    def tables(self, proposal: bool = False) -> dict:
        n, ns = self.n, self.nslots
        out = dict(r=np.zeros(n), d=np.zeros(n), inv_r=np.zeros(n),
                   deg=np.zeros(n, np.int64), begin=np.zeros(n, np.int64),
                   col=np.zeros(max(ns, 1), np.int32), thr=np.zeros(max(ns, 1), np.uint32),
                   alias=np.zeros(max(ns, 1), np.int32), logcorr=np.zeros(max(ns, 1)))
        st = _load().oracle_get_tables(self._h, int(proposal), *[_p(out[k]) for k in (
            "r", "d", "inv_r", "deg", "begin", "col", "thr", "alias", "logcorr")])
        if st != 0:
            raise OracleError(st)
        for k in ("col", "thr", "alias", "logcorr"):
            out[k] = out[k][:ns]
        return out
