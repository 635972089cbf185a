"""Independent checks used by the tests: a second Philox, exact Markov-chain
distributions of tiny resampling problems, and closed forms from the paper.

Nothing here imports the oracle or the HIP library.
"""
from __future__ import annotations

import ctypes
import math
import os
import shutil
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
_ref = None


def philox_reference():
    """rocRAND's open-source Philox4x32-10 engine, built for the host (None if
    hipcc is unavailable)."""
    global _ref
    if _ref is not None:
        return _ref
    src = os.path.join(HERE, "philox_rocrand.cpp")
    out = os.path.join(HERE, "libphilox_rocrand.so")
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(out) or os.path.getmtime(out) < os.path.getmtime(src):
        if not os.path.exists(hipcc):
            return None
        tmp = out + ".tmp%d" % os.getpid()
        subprocess.run([hipcc, "-x", "hip", "--offload-host-only", "-O1", "-fPIC", "-shared", "-o", tmp, src],
                       check=True, cwd="/tmp")
        os.replace(tmp, out)
    L = ctypes.CDLL(out)
    p = ctypes.POINTER(ctypes.c_uint32)
    L.rocrand_philox_block.argtypes = [p, p, p]
    L.rocrand_philox_block.restype = None

    def f(counter, key):
        c = np.ascontiguousarray(counter, dtype=np.uint32)
        k = np.ascontiguousarray(key, dtype=np.uint32)
        o = np.zeros(4, dtype=np.uint32)
        L.rocrand_philox_block(c.ctypes.data_as(p), k.ctypes.data_as(p), o.ctypes.data_as(p))
        return o

    _ref = f
    return f


# ---------------------------------------------------------------------------
# Exact distributions for tiny problems
# ---------------------------------------------------------------------------
U_LEVELS = 1 << 24


def accept_count(wk, wj):
    """Number of u levels m in [1, 2^24] (u = m 2^-24) with fl32(u * wk) <= wj.

    The test is monotone in m, so a vectorised binary search finds the
    largest accepted m. Works elementwise on broadcast arrays."""
    wk = np.asarray(wk, dtype=np.float32)
    wj = np.asarray(wj, dtype=np.float32)
    wk, wj = np.broadcast_arrays(wk, wj)
    lo = np.zeros(wk.shape, dtype=np.int64)            # lo always accepted (m=0 -> p=0)
    hi = np.full(wk.shape, U_LEVELS + 1, dtype=np.int64)  # hi never accepted (sentinel)
    while True:
        active = hi - lo > 1
        if not active.any():
            break
        mid = (lo + hi) // 2
        u = (mid.astype(np.float64) * 2.0 ** -24).astype(np.float32)  # exact
        ok = (u * wk) <= wj                                           # fp32 product, RNE
        ok |= mid == 0
        take = active & ok
        drop = active & ~ok
        lo = np.where(take, mid, lo)
        hi = np.where(drop, mid, hi)
    return lo


def accept_prob(wk, wj):
    return accept_count(wk, wj).astype(np.float64) / U_LEVELS


def transition_matrix(w, support=None):
    """One Metropolis step with the candidate uniform over `support` (default:
    all indices): T[k, j] = P(move from k to j)."""
    w = np.asarray(w, dtype=np.float32)
    n = w.size
    if support is None:
        support = np.arange(n)
    support = np.asarray(support)
    A = accept_prob(w[:, None], w[None, support])  # [n, |support|]
    T = np.zeros((n, n))
    T[:, support] = A / support.size
    np.fill_diagonal(T, 0.0)
    T[np.arange(n), np.arange(n)] = 1.0 - T.sum(axis=1)
    return T


def chain_marginal(T, i, B):
    v = np.zeros(T.shape[0])
    v[i] = 1.0
    for _ in range(B):
        v = v @ T
    return v


_accept_cache = {}


def accept_matrix(w):
    """A[k, j] = P(accept candidate j from ancestor k)."""
    w = np.asarray(w, dtype=np.float32)
    key = w.tobytes()
    if key not in _accept_cache:
        _accept_cache[key] = accept_prob(w[:, None], w[None, :])
    return _accept_cache[key]


def fixed_candidate_step(v, w, j):
    """Distribution after one step in which the candidate is the fixed index j."""
    a = accept_matrix(w)[:, j]
    out = v * (1.0 - a)
    out[j] += float(np.dot(v, a))
    return out


def megopolis_index_small(i, o, n):
    """Candidate index for n <= 16, where the 32-wide segment covers the whole
    array and the map is the plain cyclic shift (i + o) mod n."""
    assert n <= 16
    return (i + o) % n


# ---------------------------------------------------------------------------
# Closed forms from the paper
# ---------------------------------------------------------------------------

def gaussian_B_closed_form(y: float, eps: float = 0.01) -> int:
    """Population B for eq. (distribution) weights: Section 6.3 gives
    max w = 1/sqrt(2 pi) and E(w) = exp(-y^2/4)/sqrt(4 pi), so
    E(w)/max w = exp(-y^2/4)/sqrt(2), put into eq. (proposition)."""
    r = math.exp(-y * y / 4.0) / math.sqrt(2.0)
    return int(math.ceil(math.log(eps) / math.log(1.0 - r)))


def recurrence_P(n: int, ratio: float, B: int) -> float:
    """P_B from the recurrence P_B = 1/N + P_{B-1} (1 - E(w)/w_p), P_0 = 0
    (proof of the proposition in Section 4.1)."""
    P = 0.0
    for _ in range(B):
        P = 1.0 / n + P * (1.0 - ratio)
    return P


def build_c_client() -> str:
    """Compiles helpers/c_client.c, a plain C program that calls libmgp
    through include/mgp.h and the HIP runtime's C API only, with gcc (the
    library itself must already be built). Returns the executable's path."""
    root = os.path.dirname(os.path.dirname(HERE))
    src = os.path.join(HERE, "c_client.c")
    exe = os.path.join(HERE, "c_client")
    lib_dir = os.path.join(root, "paper_2109_13504_amd")
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    if os.path.exists(exe) and os.path.getmtime(exe) >= max(os.path.getmtime(src),
                                                            os.path.getmtime(os.path.join(lib_dir, "libmgp.so"))):
        return exe
    tmp = exe + ".tmp%d" % os.getpid()
    subprocess.run(["gcc", "-std=c11", "-Wall", "-Werror", "-D__HIP_PLATFORM_AMD__",
                    "-I", os.path.join(root, "include"), "-I", os.path.join(rocm, "include"), "-o", tmp, src,
                    "-L", lib_dir, "-lmgp", "-L", os.path.join(rocm, "lib"), "-lamdhip64",
                    "-Wl,-rpath," + lib_dir, "-Wl,-rpath," + os.path.join(rocm, "lib")], check=True)
    os.replace(tmp, exe)
    return exe
