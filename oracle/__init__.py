"""CPU oracle for Metropolis-family resampling (test infrastructure).

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package. The product path (the HIP library and
its Python binding) never imports, links or calls it.

``mgp_oracle.c`` holds the arithmetic; this module builds it with gcc and wraps
it with ctypes. See the C file for the definitions and their sources in the
paper (Algorithms 2-5, eq. (proposition)).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "mgp_oracle.c")
LIB = os.path.join(HERE, "libmgp_oracle.so")

METROPOLIS, C1, C2, MEGOPOLIS = 0, 1, 2, 3
VARIANTS = {"metropolis": METROPOLIS, "c1": C1, "c2": C2, "megopolis": MEGOPOLIS}

OK, EINVAL, ERANGE, EWEIGHTS = 0, -1, -2, -6

CFLAGS = ["-std=c11", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared"]


def build(force: bool = True) -> str:
    """Compile ``mgp_oracle.c`` into ``libmgp_oracle.so`` (single-threaded, no fast-math)."""
    if not force and os.path.exists(LIB) and os.path.getmtime(LIB) >= os.path.getmtime(SRC):
        return LIB
    tmp = LIB + ".tmp%d" % os.getpid()
    subprocess.run(["gcc", *CFLAGS, "-o", tmp, SRC, "-lm"], check=True)
    os.replace(tmp, LIB)
    return LIB


_lib = None

_u32p = ctypes.POINTER(ctypes.c_uint32)
_i32p = ctypes.POINTER(ctypes.c_int32)
_f32p = ctypes.POINTER(ctypes.c_float)
_f64p = ctypes.POINTER(ctypes.c_double)
_u64p = ctypes.POINTER(ctypes.c_uint64)


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            build()
        L = ctypes.CDLL(LIB)
        L.mgp_oracle_philox4x32_10.argtypes = [_u32p, _u32p, _u32p]
        L.mgp_oracle_philox4x32_10.restype = None
        L.mgp_oracle_draw_u.argtypes = [ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32]
        L.mgp_oracle_draw_u.restype = ctypes.c_float
        L.mgp_oracle_offset.argtypes = [ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32]
        L.mgp_oracle_offset.restype = ctypes.c_uint32
        L.mgp_oracle_offsets.argtypes = [ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32, _u32p]
        L.mgp_oracle_offsets.restype = None
        L.mgp_oracle_megopolis_index.argtypes = [ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32]
        L.mgp_oracle_megopolis_index.restype = ctypes.c_uint32
        L.mgp_oracle_resample.argtypes = [_f32p, ctypes.c_int32, ctypes.c_int, ctypes.c_uint32, ctypes.c_uint64,
                                          ctypes.c_uint32, ctypes.c_uint32, _u32p, _i32p, _u64p]
        L.mgp_oracle_resample.restype = ctypes.c_int
        L.mgp_oracle_resample_m.argtypes = [_f32p, ctypes.c_int32, ctypes.c_int32, ctypes.c_int, ctypes.c_uint32,
                                            ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32, _u32p,
                                            _i32p]
        L.mgp_oracle_megopolis_index_s.argtypes = [ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32,
                                                   ctypes.c_uint32]
        L.mgp_oracle_megopolis_index_s.restype = ctypes.c_uint32
        L.mgp_oracle_resample_m.restype = ctypes.c_int
        L.mgp_oracle_resample_subset.argtypes = [_f32p, ctypes.c_int32, ctypes.c_int, ctypes.c_uint32,
                                                 ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32,
                                                 _u32p, _i32p, ctypes.c_int32, _i32p,
                                                 ctypes.POINTER(ctypes.c_uint64)]
        L.mgp_oracle_resample_subset.restype = ctypes.c_int
        L.mgp_oracle_trace.argtypes = [ctypes.c_int32, ctypes.c_int, ctypes.c_uint32, ctypes.c_uint64,
                                       ctypes.c_uint32, ctypes.c_uint32, _u32p, ctypes.c_int32, _u32p, _f32p]
        L.mgp_oracle_trace.restype = ctypes.c_int
        L.mgp_oracle_reduce.argtypes = [_f32p, ctypes.c_int32, _f32p, _f64p]
        L.mgp_oracle_reduce.restype = ctypes.c_int
        L.mgp_oracle_choose_B.argtypes = [ctypes.c_double, ctypes.c_float, ctypes.c_int32, ctypes.c_double,
                                          ctypes.c_uint32, _u32p, _f64p, ctypes.POINTER(ctypes.c_int)]
        L.mgp_oracle_choose_B.restype = ctypes.c_int
        L.mgp_oracle_gather.argtypes = [_f32p, ctypes.c_int32, ctypes.c_int32, _i32p, ctypes.c_int32, _f32p]
        L.mgp_oracle_gather.restype = ctypes.c_int
        L.mgp_oracle_sir_normal.argtypes = [ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32]
        L.mgp_oracle_sir_normal.restype = ctypes.c_double
        L.mgp_oracle_sir_predict_update.argtypes = [_f32p, ctypes.c_int32, ctypes.c_uint32, ctypes.c_double,
                                                    ctypes.c_uint64, ctypes.c_uint32, _f32p, _f32p]
        L.mgp_oracle_sir_predict_update.restype = None
        L.mgp_oracle_mean.argtypes = [_f32p, ctypes.c_int32]
        L.mgp_oracle_mean.restype = ctypes.c_double
        L.mgp_oracle_prefix_scale.argtypes = [ctypes.c_float, ctypes.c_int32]
        L.mgp_oracle_prefix_scale.restype = ctypes.c_int
        L.mgp_oracle_prefix_fixed.argtypes = [ctypes.c_float, ctypes.c_int]
        L.mgp_oracle_prefix_fixed.restype = ctypes.c_uint64
        L.mgp_oracle_prefix_sum.argtypes = [_f32p, ctypes.c_int32, _u64p, ctypes.POINTER(ctypes.c_int)]
        L.mgp_oracle_prefix_sum.restype = ctypes.c_int
        L.mgp_oracle_prefix_threshold.argtypes = [ctypes.c_int, ctypes.c_uint64, ctypes.c_int32, ctypes.c_uint64,
                                                  ctypes.c_uint32, ctypes.c_uint32]
        L.mgp_oracle_prefix_threshold.restype = ctypes.c_uint64
        L.mgp_oracle_resample_prefix.argtypes = [_f32p, ctypes.c_int32, ctypes.c_int, ctypes.c_uint64,
                                                 ctypes.c_uint32, _u64p, _i32p]
        L.mgp_oracle_resample_prefix.restype = ctypes.c_int
        _lib = L
    return _lib


def _ptr(a: np.ndarray, t):
    return a.ctypes.data_as(t)


class OracleError(RuntimeError):
    def __init__(self, code: int, what: str):
        super().__init__(f"{what} returned {code}")
        self.code = code


def _variant(v) -> int:
    return VARIANTS[v] if isinstance(v, str) else int(v)


def philox4x32_10(counter, key) -> np.ndarray:
    c = np.ascontiguousarray(counter, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib().mgp_oracle_philox4x32_10(_ptr(c, _u32p), _ptr(k, _u32p), _ptr(out, _u32p))
    return out


def draw_u(seed: int, stream_id: int, i: int, b: int) -> np.float32:
    return np.float32(lib().mgp_oracle_draw_u(seed, stream_id, i, b))


def offsets(seed: int, stream_id: int, n: int, B: int) -> np.ndarray:
    o = np.zeros(max(B, 1), dtype=np.uint32)
    lib().mgp_oracle_offsets(seed, stream_id, n, B, _ptr(o, _u32p))
    return o[:B]


def megopolis_index(i: int, o: int, n: int, segment: int = 32) -> int:
    if segment == 32:
        return int(lib().mgp_oracle_megopolis_index(i, o, n))
    return int(lib().mgp_oracle_megopolis_index_s(i, o, n, segment))


@dataclass
class Stats:
    w_max: float
    w_sum: float
    status: int


def reduce(w: np.ndarray) -> Stats:
    w = np.ascontiguousarray(w, dtype=np.float32)
    mx = ctypes.c_float()
    s = ctypes.c_double()
    rc = lib().mgp_oracle_reduce(_ptr(w, _f32p), w.size, ctypes.byref(mx), ctypes.byref(s))
    if rc == EINVAL:
        raise OracleError(rc, "mgp_oracle_reduce")
    return Stats(float(mx.value), float(s.value), rc)


def choose_B(w_sum: float, w_max: float, n: int, eps: float, b_max: int = 65536):
    """Returns (B, raw, clamped)."""
    B = ctypes.c_uint32()
    raw = ctypes.c_double()
    cl = ctypes.c_int()
    rc = lib().mgp_oracle_choose_B(w_sum, w_max, n, eps, b_max, ctypes.byref(B), ctypes.byref(raw),
                                   ctypes.byref(cl))
    if rc:
        raise OracleError(rc, "mgp_oracle_choose_B")
    return int(B.value), float(raw.value), bool(cl.value)


def B_from_weights(w: np.ndarray, eps: float, b_max: int = 65536):
    st = reduce(w)
    if st.status:
        raise OracleError(st.status, "mgp_oracle_reduce")
    return choose_B(st.w_sum, st.w_max, w.size, eps, b_max)


def resample(w: np.ndarray, variant, B: int, seed: int, stream_id: int = 0, partition_bytes: int = 128,
             return_accepts: bool = False):
    w = np.ascontiguousarray(w, dtype=np.float32)
    n = w.size
    v = _variant(variant)
    anc = np.empty(n, dtype=np.int32)
    scratch = np.zeros(max(B, 1), dtype=np.uint32)
    acc = ctypes.c_uint64()
    rc = lib().mgp_oracle_resample(_ptr(w, _f32p), n, v, B, seed, stream_id, partition_bytes,
                                   _ptr(scratch, _u32p), _ptr(anc, _i32p), ctypes.byref(acc))
    if rc:
        raise OracleError(rc, "mgp_oracle_resample")
    if return_accepts:
        return anc, int(acc.value)
    return anc


def resample_m(w: np.ndarray, m: int, variant, B: int, seed: int, stream_id: int = 0,
               partition_bytes: int = 128, segment: int = 32) -> np.ndarray:
    """M != N: m ancestors from the n = len(w) weighted inputs (m = n: the
    usual resample); `segment` is the Megopolis segment width, 32 or 64."""
    w = np.ascontiguousarray(w, dtype=np.float32)
    anc = np.empty(m, dtype=np.int32)
    scratch = np.zeros(max(B, 1), dtype=np.uint32)
    rc = lib().mgp_oracle_resample_m(_ptr(w, _f32p), w.size, m, _variant(variant), B, seed, stream_id,
                                     partition_bytes, segment, _ptr(scratch, _u32p), _ptr(anc, _i32p))
    if rc:
        raise OracleError(rc, "mgp_oracle_resample_m")
    return anc


def resample_subset(w: np.ndarray, variant, B: int, seed: int, idx, stream_id: int = 0,
                    partition_bytes: int = 128, segment: int = 32, return_accepts: bool = False):
    """Ancestors of the particles idx only (the chains of resample(), each
    computed alone); `segment` is the Megopolis segment width, 32 or 64.
    With return_accepts, also the number of accepted steps of these chains."""
    w = np.ascontiguousarray(w, dtype=np.float32)
    idx = np.ascontiguousarray(idx, dtype=np.int32)
    out = np.empty(idx.size, dtype=np.int32)
    scratch = np.zeros(max(B, 1), dtype=np.uint32)
    acc = ctypes.c_uint64()
    rc = lib().mgp_oracle_resample_subset(_ptr(w, _f32p), w.size, _variant(variant), B, seed, stream_id,
                                          partition_bytes, segment, _ptr(scratch, _u32p), _ptr(idx, _i32p), idx.size,
                                          _ptr(out, _i32p), ctypes.byref(acc))
    if rc:
        raise OracleError(rc, "mgp_oracle_resample_subset")
    if return_accepts:
        return out, int(acc.value)
    return out


def trace(n: int, variant, B: int, seed: int, i: int, stream_id: int = 0, partition_bytes: int = 128):
    """Candidate indices j_b and draws u_b of particle i, b = 0..B-1."""
    j = np.zeros(max(B, 1), dtype=np.uint32)
    u = np.zeros(max(B, 1), dtype=np.float32)
    scratch = np.zeros(max(B, 1), dtype=np.uint32)
    rc = lib().mgp_oracle_trace(n, _variant(variant), B, seed, stream_id, partition_bytes,
                                _ptr(scratch, _u32p), i, _ptr(j, _u32p), _ptr(u, _f32p))
    if rc:
        raise OracleError(rc, "mgp_oracle_trace")
    return j[:B].astype(np.int64), u[:B]


def gather(states: np.ndarray, anc: np.ndarray) -> np.ndarray:
    states = np.ascontiguousarray(states, dtype=np.float32)
    if states.ndim == 1:
        states = states.reshape(-1, 1)
    anc = np.ascontiguousarray(anc, dtype=np.int32)
    n_states, d = states.shape
    out = np.empty((anc.size, d), dtype=np.float32)
    rc = lib().mgp_oracle_gather(_ptr(states, _f32p), n_states, d, _ptr(anc, _i32p), anc.size,
                                 _ptr(out, _f32p))
    if rc:
        raise OracleError(rc, "mgp_oracle_gather")
    return out


# ---------------------------------------------------------------------------
# The SIR application of Section 7 (Algorithm 6)
# ---------------------------------------------------------------------------

def sir_normal(seed: int, run: int, i: int, t: int) -> float:
    return float(lib().mgp_oracle_sir_normal(seed, run, i, t))


def sir_predict_update(xbar: np.ndarray, t: int, z: float, seed: int, run: int):
    xbar = np.ascontiguousarray(xbar, dtype=np.float32)
    x = np.empty_like(xbar)
    w = np.empty_like(xbar)
    lib().mgp_oracle_sir_predict_update(_ptr(xbar, _f32p), xbar.size, t, z, seed, run, _ptr(x, _f32p),
                                        _ptr(w, _f32p))
    return x, w


def mean(x: np.ndarray) -> float:
    x = np.ascontiguousarray(x, dtype=np.float32)
    return float(lib().mgp_oracle_mean(_ptr(x, _f32p), x.size))


def sir_step_seed(seed: int, t: int) -> int:
    """Philox key of the resample at step t: the seed plus t * 2^32 (mod 2^64)."""
    return (seed + (t << 32)) & 0xFFFFFFFFFFFFFFFF


def sir_filter(x0: np.ndarray, z: np.ndarray, variant, B: int, seed: int, run: int, partition_bytes: int = 128,
               epsilon: float = 0.1, steps=None):
    """The modified SIR filter of Algorithm 6 for one run, over steps
    t = 1..T (T = len(z) - 1 unless `steps` is given):
      stage 1: predict + update (sir_predict_update);
      stage 2: resample with B iterations (B = 0: B from eq. (bcalc) with
               `epsilon`, per step), Philox key sir_step_seed(seed, t), stream
               `run`, then x_bar = x[ancestors]; variant "multinomial" or
               "systematic" resamples by resample_prefix instead (B recorded
               as 1);
      stage 3: the estimate, the mean of x_bar.
    A step whose weights are all zero (fp32 underflow) keeps the predicted
    particles unresampled (x_bar = x) and reports MGP_EWEIGHTS.
    Returns (estimates[T], B[T], status[T], last x_bar)."""
    xbar = np.ascontiguousarray(x0, dtype=np.float32)
    T = len(z) - 1 if steps is None else steps
    est, bs, sts = [], [], []
    for t in range(1, T + 1):
        x, w = sir_predict_update(xbar, t, float(z[t]), seed, run)
        st = reduce(w)
        if st.status:
            xbar, b = x, 0
        elif isinstance(variant, str) and variant in PREFIX_METHODS:
            # stage 2 by a prefix-sum method (Algorithms 7 and 8): no iterations
            b = 1
            anc = resample_prefix(w, variant, sir_step_seed(seed, t), stream_id=run)
            xbar = gather(x, anc).reshape(-1)
        else:
            b = B if B > 0 else choose_B(st.w_sum, st.w_max, w.size, epsilon)[0]
            anc = resample(w, variant, b, sir_step_seed(seed, t), stream_id=run, partition_bytes=partition_bytes)
            xbar = gather(x, anc).reshape(-1)
        est.append(mean(xbar))
        bs.append(b)
        sts.append(st.status)
    return np.array(est), np.array(bs, dtype=np.int64), np.array(sts, dtype=np.int64), xbar


# ---------------------------------------------------------------------------
# Prefix-sum resamplers (Algorithms 7 and 8)
# ---------------------------------------------------------------------------
PREFIX_METHODS = {"multinomial": 0, "systematic": 1}


def _method(m) -> int:
    return PREFIX_METHODS[m] if isinstance(m, str) else int(m)


def prefix_scale(w_max: float, n: int) -> int:
    """The fixed-point exponent K of n weights with maximum w_max."""
    return int(lib().mgp_oracle_prefix_scale(float(np.float32(w_max)), int(n)))


def prefix_fixed(w: float, K: int) -> int:
    """q = floor(w 2^K) of one fp32 weight."""
    return int(lib().mgp_oracle_prefix_fixed(float(np.float32(w)), int(K)))


def prefix_sum(w: np.ndarray):
    """(inclusive fixed-point prefix sums as uint64, K)."""
    w = np.ascontiguousarray(w, dtype=np.float32)
    incl = np.empty(w.size, dtype=np.uint64)
    K = ctypes.c_int()
    rc = lib().mgp_oracle_prefix_sum(_ptr(w, _f32p), w.size, _ptr(incl, _u64p), ctypes.byref(K))
    if rc:
        raise OracleError(rc, "mgp_oracle_prefix_sum")
    return incl, K.value


def prefix_threshold(method, S: int, n: int, seed: int, stream_id: int, i: int) -> int:
    return int(lib().mgp_oracle_prefix_threshold(_method(method), int(S), int(n), int(seed) & (2**64 - 1),
                                                 int(stream_id), int(i)))


def resample_prefix(w: np.ndarray, method, seed: int, stream_id: int = 0) -> np.ndarray:
    """Multinomial ("multinomial", Algorithm 7) or systematic ("systematic",
    Algorithm 8) resampling through the fixed-point prefix sum."""
    w = np.ascontiguousarray(w, dtype=np.float32)
    incl = np.empty(w.size, dtype=np.uint64)
    anc = np.empty(w.size, dtype=np.int32)
    rc = lib().mgp_oracle_resample_prefix(_ptr(w, _f32p), w.size, _method(method), int(seed) & (2**64 - 1),
                                          int(stream_id), _ptr(incl, _u64p), _ptr(anc, _i32p))
    if rc:
        raise OracleError(rc, "mgp_oracle_resample_prefix")
    return anc
