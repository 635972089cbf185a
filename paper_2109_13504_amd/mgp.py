"""ctypes binding of libmgp (include/mgp.h).

The mgp_* functions mirror the C entry points one to one and take raw device
pointers (ints); they only marshal arguments and turn negative return codes
into MgpError. The helpers below them (Resampler, resample, gather) allocate
the device tensors with torch and call the same entry points; every step of
the computation runs in the HIP kernels of libmgp.so.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libmgp.so")

MGP_OK, MGP_EINVAL, MGP_ERANGE, MGP_ENOMEM, MGP_EHIP, MGP_EBUSY, MGP_EWEIGHTS = 0, -1, -2, -3, -4, -5, -6
MGP_METROPOLIS, MGP_C1, MGP_C2, MGP_MEGOPOLIS = 0, 1, 2, 3
MGP_MULTINOMIAL, MGP_SYSTEMATIC = 0, 1
PREFIX_METHODS = {"multinomial": MGP_MULTINOMIAL, "systematic": MGP_SYSTEMATIC}
MGP_SIR_MULTINOMIAL, MGP_SIR_SYSTEMATIC = 4, 5
MGP_NOALLOC_SCRATCH_BYTES = 64 << 20
VARIANTS = {"metropolis": MGP_METROPOLIS, "c1": MGP_C1, "c2": MGP_C2, "megopolis": MGP_MEGOPOLIS}
SIR_VARIANTS = {**VARIANTS, "multinomial": MGP_SIR_MULTINOMIAL, "systematic": MGP_SIR_SYSTEMATIC}


class MgpError(RuntimeError):
    def __init__(self, code: int, func: str, message: str):
        super().__init__(f"{func} failed ({code}): {message}")
        self.code = code


class mgp_params(ctypes.Structure):
    _fields_ = [("variant", ctypes.c_int32), ("B", ctypes.c_uint32), ("epsilon", ctypes.c_double),
                ("seed", ctypes.c_uint64), ("stream_id", ctypes.c_uint32), ("partition_bytes", ctypes.c_uint32),
                ("b_max", ctypes.c_uint32), ("segment", ctypes.c_uint32)]


class mgp_stats(ctypes.Structure):
    _fields_ = [("w_sum", ctypes.c_double), ("ratio", ctypes.c_double), ("b_raw", ctypes.c_double),
                ("w_max", ctypes.c_float), ("B", ctypes.c_uint32), ("clamped", ctypes.c_uint32),
                ("status", ctypes.c_int32), ("n", ctypes.c_uint32), ("tag", ctypes.c_uint32)]


class mgp_filter_desc(ctypes.Structure):
    _fields_ = [("w_dev", ctypes.c_void_p), ("n", ctypes.c_int32), ("B", ctypes.c_uint32),
                ("epsilon", ctypes.c_double), ("seed", ctypes.c_uint64), ("stream_id", ctypes.c_uint32),
                ("reserved", ctypes.c_uint32), ("ancestors_dev", ctypes.c_void_p), ("states_dev", ctypes.c_void_p),
                ("out_states_dev", ctypes.c_void_p), ("stats_dev", ctypes.c_void_p)]


class mgp_batch_config(ctypes.Structure):
    _fields_ = [("variant", ctypes.c_int32), ("d", ctypes.c_int32), ("partition_bytes", ctypes.c_uint32),
                ("b_max", ctypes.c_uint32), ("block_threads", ctypes.c_int32),
                ("particles_per_thread", ctypes.c_int32), ("schedule", ctypes.c_int32), ("use_graph", ctypes.c_int32),
                ("tune_cache", ctypes.c_char_p)]


class mgp_batch_info(ctypes.Structure):
    _fields_ = [("filters", ctypes.c_int32), ("block_threads", ctypes.c_int32),
                ("particles_per_thread", ctypes.c_int32), ("schedule", ctypes.c_int32),
                ("from_cache", ctypes.c_int32), ("xcds", ctypes.c_int32), ("particles", ctypes.c_int64),
                ("tiles", ctypes.c_int64), ("device_bytes", ctypes.c_int64), ("est_particle_steps", ctypes.c_double),
                ("grid", ctypes.c_int64)]


class mgp_server_config(ctypes.Structure):
    _fields_ = [("variant", ctypes.c_int32), ("d", ctypes.c_int32), ("partition_bytes", ctypes.c_uint32),
                ("b_max", ctypes.c_uint32), ("hbm_budget", ctypes.c_uint64), ("streams", ctypes.c_int32),
                ("max_batch", ctypes.c_int32), ("max_batch_particles", ctypes.c_int64), ("max_n", ctypes.c_int32),
                ("simulate", ctypes.c_int32), ("sim_us_fixed", ctypes.c_double),
                ("sim_ns_per_particle", ctypes.c_double), ("sim_fail_every", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


class mgp_request(ctypes.Structure):
    _fields_ = [("w_dev", ctypes.c_void_p), ("n", ctypes.c_int32), ("B", ctypes.c_uint32),
                ("epsilon", ctypes.c_double), ("seed", ctypes.c_uint64), ("stream_id", ctypes.c_uint32),
                ("reserved", ctypes.c_uint32), ("states_dev", ctypes.c_void_p)]


class mgp_request_result(ctypes.Structure):
    _fields_ = [("state", ctypes.c_int32), ("status", ctypes.c_int32), ("B", ctypes.c_uint32), ("n", ctypes.c_int32),
                ("ancestors_dev", ctypes.c_void_p), ("out_states_dev", ctypes.c_void_p),
                ("t_submit", ctypes.c_double), ("t_admit", ctypes.c_double), ("t_dispatch", ctypes.c_double),
                ("t_done", ctypes.c_double)]


class mgp_server_stats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_int64), ("admitted", ctypes.c_int64), ("completed", ctypes.c_int64),
                ("failed", ctypes.c_int64), ("cancelled", ctypes.c_int64), ("released", ctypes.c_int64),
                ("micro_batches", ctypes.c_int64), ("queued", ctypes.c_int64), ("in_flight", ctypes.c_int64),
                ("pool_bytes", ctypes.c_uint64), ("pool_in_use", ctypes.c_uint64), ("pool_peak", ctypes.c_uint64),
                ("max_concurrent_batches", ctypes.c_int64)]


class mgp_sir_config(ctypes.Structure):
    _fields_ = [("variant", ctypes.c_int32), ("runs", ctypes.c_int32), ("n", ctypes.c_int32),
                ("steps", ctypes.c_int32), ("B", ctypes.c_uint32), ("partition_bytes", ctypes.c_uint32),
                ("epsilon", ctypes.c_double), ("seed", ctypes.c_uint64), ("b_max", ctypes.c_uint32),
                ("use_graph", ctypes.c_int32), ("block_threads", ctypes.c_int32),
                ("particles_per_thread", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("reserved2", ctypes.c_int32)]


class mgp_sir_buffers(ctypes.Structure):
    _fields_ = [("x_dev", ctypes.c_void_p), ("w_dev", ctypes.c_void_p), ("xbar_dev", ctypes.c_void_p),
                ("ancestors_dev", ctypes.c_void_p), ("ld", ctypes.c_int64), ("device_bytes", ctypes.c_int64),
                ("accept_grid", ctypes.c_int64), ("block_threads", ctypes.c_int32),
                ("particles_per_thread", ctypes.c_int32)]


MGP_REQ_QUEUED, MGP_REQ_RUNNING, MGP_REQ_DONE, MGP_REQ_FAILED, MGP_REQ_CANCELLED = 0, 1, 2, 3, 4

STATS_BYTES = ctypes.sizeof(mgp_stats)
STATS_DTYPE = np.dtype([("w_sum", "<f8"), ("ratio", "<f8"), ("b_raw", "<f8"), ("w_max", "<f4"), ("B", "<u4"),
                        ("clamped", "<u4"), ("status", "<i4"), ("n", "<u4"), ("tag", "<u4")])
assert STATS_DTYPE.itemsize == STATS_BYTES == 48

_lib = None
_vp = ctypes.c_void_p


def lib():
    """The loaded libmgp.so. Raises if the HIP library has not been built:
    there is no fallback path."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"HIP library {LIB_PATH} is not built; run __graft_entry__.build()")
        L = ctypes.CDLL(LIB_PATH)
        P = ctypes.POINTER(mgp_params)
        L.mgp_workspace_size.argtypes = [ctypes.c_int32, P, ctypes.POINTER(ctypes.c_size_t)]
        L.mgp_resample.argtypes = [_vp, ctypes.c_int32, P, _vp, _vp, _vp, ctypes.c_size_t, _vp]
        L.mgp_compute_B.argtypes = [_vp, ctypes.c_int32, P, _vp, _vp, ctypes.c_size_t, _vp]
        L.mgp_resample_m.argtypes = [_vp, ctypes.c_int32, ctypes.c_int32, P, _vp, _vp, _vp, ctypes.c_size_t, _vp]
        L.mgp_resample_noalloc.argtypes = [_vp, ctypes.c_int32, P, _vp, _vp, _vp]
        L.mgp_resample_prepared.argtypes = [_vp, ctypes.c_int32, P, _vp, _vp, ctypes.c_size_t, _vp]
        L.mgp_gather.argtypes = [_vp, ctypes.c_int32, ctypes.c_int32, _vp, ctypes.c_int32, _vp, _vp]
        L.mgp_resample_gather.argtypes = [_vp, ctypes.c_int32, P, _vp, ctypes.c_int32, _vp, _vp, _vp, _vp,
                                          ctypes.c_size_t, _vp]
        L.mgp_resample_gather_prepared.argtypes = [_vp, ctypes.c_int32, P, _vp, ctypes.c_int32, _vp, _vp, _vp,
                                                   ctypes.c_size_t, _vp]
        L.mgp_batch_plan_create.argtypes = [ctypes.POINTER(mgp_filter_desc), ctypes.c_int32,
                                            ctypes.POINTER(mgp_batch_config), _vp, ctypes.POINTER(_vp)]
        L.mgp_batch_set_seeds.argtypes = [_vp, ctypes.POINTER(ctypes.c_uint64), _vp]
        L.mgp_batch_run.argtypes = [_vp, _vp]
        L.mgp_batch_run_separate.argtypes = [_vp, _vp]
        L.mgp_batch_plan_info.argtypes = [_vp, ctypes.POINTER(mgp_batch_info)]
        L.mgp_batch_plan_destroy.argtypes = [_vp]
        for f in ("mgp_batch_plan_create", "mgp_batch_set_seeds", "mgp_batch_run", "mgp_batch_run_separate",
                  "mgp_batch_plan_info", "mgp_batch_plan_destroy"):
            getattr(L, f).restype = ctypes.c_int
        L.mgp_server_create.argtypes = [ctypes.POINTER(mgp_server_config), ctypes.POINTER(_vp)]
        L.mgp_server_submit.argtypes = [_vp, ctypes.POINTER(mgp_request), ctypes.POINTER(ctypes.c_uint64)]
        L.mgp_server_poll.argtypes = [_vp, ctypes.c_uint64, ctypes.POINTER(mgp_request_result)]
        L.mgp_server_wait.argtypes = [_vp, ctypes.c_uint64, ctypes.c_double, ctypes.POINTER(mgp_request_result)]
        L.mgp_server_cancel.argtypes = [_vp, ctypes.c_uint64]
        L.mgp_server_copy_outputs.argtypes = [_vp, ctypes.c_uint64, _vp, _vp, _vp]
        L.mgp_server_release.argtypes = [_vp, ctypes.c_uint64]
        L.mgp_server_get_stats.argtypes = [_vp, ctypes.POINTER(mgp_server_stats)]
        L.mgp_server_destroy.argtypes = [_vp]
        for f in ("mgp_server_create", "mgp_server_submit", "mgp_server_poll", "mgp_server_wait", "mgp_server_cancel",
                  "mgp_server_copy_outputs", "mgp_server_release", "mgp_server_get_stats", "mgp_server_destroy"):
            getattr(L, f).restype = ctypes.c_int
        L.mgp_sir_create.argtypes = [ctypes.POINTER(mgp_sir_config), _vp, ctypes.POINTER(_vp)]
        L.mgp_sir_set_measurements.argtypes = [_vp, ctypes.POINTER(ctypes.c_double), _vp]
        L.mgp_sir_reset.argtypes = [_vp, _vp, _vp]
        L.mgp_sir_predict_update.argtypes = [_vp, ctypes.c_int32, _vp]
        L.mgp_sir_resample.argtypes = [_vp, ctypes.c_int32, _vp]
        L.mgp_sir_estimate.argtypes = [_vp, ctypes.c_int32, _vp]
        L.mgp_sir_run.argtypes = [_vp, _vp]
        L.mgp_sir_results.argtypes = [_vp, _vp, _vp, _vp, _vp]
        L.mgp_sir_get_buffers.argtypes = [_vp, ctypes.POINTER(mgp_sir_buffers)]
        L.mgp_sir_destroy.argtypes = [_vp]
        L.mgp_sir_copy_buffer.argtypes = [_vp, ctypes.c_int32, _vp, _vp]
        for f in ("mgp_sir_copy_buffer", "mgp_sir_create", "mgp_sir_set_measurements", "mgp_sir_reset", "mgp_sir_predict_update",
                  "mgp_sir_resample", "mgp_sir_estimate", "mgp_sir_run", "mgp_sir_results", "mgp_sir_get_buffers",
                  "mgp_sir_destroy"):
            getattr(L, f).restype = ctypes.c_int
        L.mgp_prefix_workspace_size.argtypes = [ctypes.c_int32, ctypes.POINTER(ctypes.c_size_t)]
        L.mgp_prefix_workspace_size.restype = ctypes.c_int
        L.mgp_resample_prefix.argtypes = [_vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_uint64, ctypes.c_uint32, _vp,
                                          _vp, _vp, ctypes.c_size_t, _vp]
        L.mgp_resample_prefix.restype = ctypes.c_int
        L.mgp_probe_stream_read.argtypes = [_vp, ctypes.c_size_t, ctypes.c_int32, ctypes.c_int32, _vp, _vp]
        L.mgp_probe_stream_read.restype = ctypes.c_int
        L.mgp_probe_pattern_read.argtypes = [_vp, ctypes.c_size_t, ctypes.c_uint32, _vp, ctypes.c_int32, _vp, _vp]
        L.mgp_probe_pattern_read.restype = ctypes.c_int
        L.mgp_last_error.argtypes = []
        L.mgp_last_error.restype = ctypes.c_char_p
        L.mgp_version.argtypes = []
        for f in ("mgp_workspace_size", "mgp_resample", "mgp_resample_m", "mgp_resample_noalloc", "mgp_compute_B",
                  "mgp_resample_prepared", "mgp_gather", "mgp_resample_gather", "mgp_resample_gather_prepared",
                  "mgp_version"):
            getattr(L, f).restype = ctypes.c_int
        _lib = L
    return _lib


def _check(rc: int, func: str) -> int:
    if rc < 0:
        raise MgpError(rc, func, (lib().mgp_last_error() or b"").decode())
    return rc


def make_params(variant="megopolis", B: int = 0, epsilon: float = 0.01, seed: int = 0, stream_id: int = 0,
                partition_bytes: int = 128, b_max: int = 0, segment: int = 32) -> mgp_params:
    v = VARIANTS[variant] if isinstance(variant, str) else int(variant)
    return mgp_params(v, int(B), float(epsilon), int(seed) & (2**64 - 1), int(stream_id), int(partition_bytes),
                      int(b_max), int(segment))


# ---------------------------------------------------------------------------
# C entry points, same names
# ---------------------------------------------------------------------------

def mgp_version() -> int:
    return lib().mgp_version()


def mgp_last_error() -> str:
    return (lib().mgp_last_error() or b"").decode()


def mgp_workspace_size(n: int, params: mgp_params) -> int:
    out = ctypes.c_size_t()
    _check(lib().mgp_workspace_size(n, ctypes.byref(params), ctypes.byref(out)), "mgp_workspace_size")
    return out.value


def mgp_resample(w_dev: int, n: int, params: mgp_params, ancestors_dev: int, stats_dev: int, workspace_dev: int,
                 workspace_bytes: int, stream: int) -> None:
    _check(lib().mgp_resample(w_dev, n, ctypes.byref(params), ancestors_dev, stats_dev or None, workspace_dev,
                              workspace_bytes, stream or None), "mgp_resample")


def mgp_resample_noalloc(w_dev: int, n: int, params: mgp_params, ancestors_dev: int, stats_dev: int,
                         stream: int) -> None:
    _check(lib().mgp_resample_noalloc(w_dev, n, ctypes.byref(params), ancestors_dev, stats_dev or None,
                                      stream or None), "mgp_resample_noalloc")


def mgp_resample_m(w_dev: int, n: int, m: int, params: mgp_params, ancestors_dev: int, stats_dev: int,
                   workspace_dev: int, workspace_bytes: int, stream: int) -> None:
    _check(lib().mgp_resample_m(w_dev, n, m, ctypes.byref(params), ancestors_dev, stats_dev or None, workspace_dev,
                                workspace_bytes, stream or None), "mgp_resample_m")


def mgp_compute_B(w_dev: int, n: int, params: mgp_params, stats_dev: int, workspace_dev: int,
                  workspace_bytes: int, stream: int) -> None:
    _check(lib().mgp_compute_B(w_dev, n, ctypes.byref(params), stats_dev or None, workspace_dev, workspace_bytes,
                               stream or None), "mgp_compute_B")


def mgp_resample_prepared(w_dev: int, n: int, params: mgp_params, ancestors_dev: int, workspace_dev: int,
                          workspace_bytes: int, stream: int) -> None:
    _check(lib().mgp_resample_prepared(w_dev, n, ctypes.byref(params), ancestors_dev, workspace_dev,
                                       workspace_bytes, stream or None), "mgp_resample_prepared")


def mgp_gather(states_dev: int, n_states: int, d: int, ancestors_dev: int, n_out: int, out_dev: int,
               stream: int) -> None:
    _check(lib().mgp_gather(states_dev, n_states, d, ancestors_dev, n_out, out_dev, stream or None), "mgp_gather")


def mgp_resample_gather(w_dev: int, n: int, params: mgp_params, states_dev: int, d: int, ancestors_dev: int,
                        out_dev: int, stats_dev: int, workspace_dev: int, workspace_bytes: int, stream: int) -> None:
    _check(lib().mgp_resample_gather(w_dev, n, ctypes.byref(params), states_dev, d, ancestors_dev or None, out_dev,
                                     stats_dev or None, workspace_dev, workspace_bytes, stream or None),
           "mgp_resample_gather")


def mgp_resample_gather_prepared(w_dev: int, n: int, params: mgp_params, states_dev: int, d: int,
                                 ancestors_dev: int, out_dev: int, workspace_dev: int, workspace_bytes: int,
                                 stream: int) -> None:
    _check(lib().mgp_resample_gather_prepared(w_dev, n, ctypes.byref(params), states_dev, d, ancestors_dev or None,
                                              out_dev, workspace_dev, workspace_bytes, stream or None),
           "mgp_resample_gather_prepared")


def mgp_batch_plan_create(filters, config: mgp_batch_config, stream: int) -> int:
    arr = (mgp_filter_desc * len(filters))(*filters)
    plan = _vp()
    _check(lib().mgp_batch_plan_create(arr, len(filters), ctypes.byref(config), stream or None, ctypes.byref(plan)),
           "mgp_batch_plan_create")
    return plan.value


def mgp_batch_set_seeds(plan: int, seeds, stream: int) -> None:
    arr = (ctypes.c_uint64 * len(seeds))(*[int(x) & (2**64 - 1) for x in seeds])
    _check(lib().mgp_batch_set_seeds(plan, arr, stream or None), "mgp_batch_set_seeds")


def mgp_batch_run(plan: int, stream: int) -> None:
    _check(lib().mgp_batch_run(plan, stream or None), "mgp_batch_run")


def mgp_batch_run_separate(plan: int, stream: int) -> None:
    _check(lib().mgp_batch_run_separate(plan, stream or None), "mgp_batch_run_separate")


def mgp_batch_plan_info(plan: int) -> dict:
    info = mgp_batch_info()
    _check(lib().mgp_batch_plan_info(plan, ctypes.byref(info)), "mgp_batch_plan_info")
    return {k: getattr(info, k) for k, _ in mgp_batch_info._fields_}


def mgp_batch_plan_destroy(plan: int) -> None:
    _check(lib().mgp_batch_plan_destroy(plan), "mgp_batch_plan_destroy")


def mgp_server_create(config: mgp_server_config) -> int:
    h = _vp()
    _check(lib().mgp_server_create(ctypes.byref(config), ctypes.byref(h)), "mgp_server_create")
    return h.value


def mgp_server_submit(server: int, request: mgp_request) -> int:
    t = ctypes.c_uint64()
    _check(lib().mgp_server_submit(server, ctypes.byref(request), ctypes.byref(t)), "mgp_server_submit")
    return t.value


def _result_dict(r: mgp_request_result) -> dict:
    return {k: getattr(r, k) for k, _ in mgp_request_result._fields_}


def mgp_server_poll(server: int, ticket: int) -> dict:
    r = mgp_request_result()
    _check(lib().mgp_server_poll(server, ticket, ctypes.byref(r)), "mgp_server_poll")
    return _result_dict(r)


def mgp_server_wait(server: int, ticket: int, timeout_ms: float = -1.0) -> dict:
    r = mgp_request_result()
    _check(lib().mgp_server_wait(server, ticket, timeout_ms, ctypes.byref(r)), "mgp_server_wait")
    return _result_dict(r)


def mgp_server_cancel(server: int, ticket: int) -> None:
    _check(lib().mgp_server_cancel(server, ticket), "mgp_server_cancel")


def mgp_server_copy_outputs(server: int, ticket: int, ancestors_dev: int, out_states_dev: int, stream: int) -> None:
    _check(lib().mgp_server_copy_outputs(server, ticket, ancestors_dev, out_states_dev or None, stream or None),
           "mgp_server_copy_outputs")


def mgp_server_release(server: int, ticket: int) -> None:
    _check(lib().mgp_server_release(server, ticket), "mgp_server_release")


def mgp_server_get_stats(server: int) -> dict:
    st = mgp_server_stats()
    _check(lib().mgp_server_get_stats(server, ctypes.byref(st)), "mgp_server_get_stats")
    return {k: getattr(st, k) for k, _ in mgp_server_stats._fields_}


def mgp_server_destroy(server: int) -> None:
    _check(lib().mgp_server_destroy(server), "mgp_server_destroy")


def mgp_sir_create(config: mgp_sir_config, stream: int) -> int:
    h = _vp()
    _check(lib().mgp_sir_create(ctypes.byref(config), stream or None, ctypes.byref(h)), "mgp_sir_create")
    return h.value


def mgp_sir_set_measurements(filt: int, z: np.ndarray, stream: int) -> None:
    z = np.ascontiguousarray(z, dtype=np.float64)
    _check(lib().mgp_sir_set_measurements(filt, z.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), stream or None),
           "mgp_sir_set_measurements")


def mgp_sir_reset(filt: int, x0_dev: int, stream: int) -> None:
    _check(lib().mgp_sir_reset(filt, x0_dev, stream or None), "mgp_sir_reset")


def mgp_sir_predict_update(filt: int, t: int, stream: int) -> None:
    _check(lib().mgp_sir_predict_update(filt, t, stream or None), "mgp_sir_predict_update")


def mgp_sir_resample(filt: int, t: int, stream: int) -> None:
    _check(lib().mgp_sir_resample(filt, t, stream or None), "mgp_sir_resample")


def mgp_sir_estimate(filt: int, t: int, stream: int) -> None:
    _check(lib().mgp_sir_estimate(filt, t, stream or None), "mgp_sir_estimate")


def mgp_sir_run(filt: int, stream: int) -> None:
    _check(lib().mgp_sir_run(filt, stream or None), "mgp_sir_run")


def mgp_sir_results(filt: int, est: np.ndarray | None, B: np.ndarray | None, status: np.ndarray | None,
                    stream: int) -> None:
    def ptr(a):
        return None if a is None else a.ctypes.data
    _check(lib().mgp_sir_results(filt, ptr(est), ptr(B), ptr(status), stream or None), "mgp_sir_results")


def mgp_sir_get_buffers(filt: int) -> dict:
    b = mgp_sir_buffers()
    _check(lib().mgp_sir_get_buffers(filt, ctypes.byref(b)), "mgp_sir_get_buffers")
    return {k: getattr(b, k) for k, _ in mgp_sir_buffers._fields_}


MGP_SIR_X, MGP_SIR_W, MGP_SIR_XBAR, MGP_SIR_ANCESTORS = 0, 1, 2, 3


def mgp_sir_copy_buffer(filt: int, which: int, dst_dev: int, stream: int) -> None:
    _check(lib().mgp_sir_copy_buffer(filt, which, dst_dev, stream or None), "mgp_sir_copy_buffer")


def mgp_sir_destroy(filt: int) -> None:
    _check(lib().mgp_sir_destroy(filt), "mgp_sir_destroy")


def mgp_prefix_workspace_size(n: int) -> int:
    out = ctypes.c_size_t()
    _check(lib().mgp_prefix_workspace_size(n, ctypes.byref(out)), "mgp_prefix_workspace_size")
    return out.value


def mgp_resample_prefix(w_dev: int, n: int, method: int, seed: int, stream_id: int, ancestors_dev: int,
                        stats_dev: int, workspace_dev: int, workspace_bytes: int, stream: int) -> None:
    _check(lib().mgp_resample_prefix(w_dev, n, method, int(seed) & (2**64 - 1), stream_id, ancestors_dev,
                                     stats_dev or None, workspace_dev, workspace_bytes, stream or None),
           "mgp_resample_prefix")


def mgp_probe_stream_read(buf_dev: int, nbytes: int, passes: int, blocks: int, sink_dev: int, stream: int) -> None:
    _check(lib().mgp_probe_stream_read(buf_dev, nbytes, passes, blocks, sink_dev, stream or None),
           "mgp_probe_stream_read")


def mgp_probe_pattern_read(mirror_dev: int, mirror_bytes: int, n: int, offsets_dev: int, steps: int, sink_dev: int,
                           stream: int) -> None:
    _check(lib().mgp_probe_pattern_read(mirror_dev, mirror_bytes, n, offsets_dev, steps, sink_dev, stream or None),
           "mgp_probe_pattern_read")


# ---------------------------------------------------------------------------
# torch helpers
# ---------------------------------------------------------------------------

def _torch():
    import torch
    return torch


def current_stream() -> int:
    return _torch().cuda.current_stream().cuda_stream


def decode_stats(stats_tensor) -> dict:
    raw = stats_tensor.detach().cpu().numpy().tobytes()
    rec = np.frombuffer(raw[:STATS_BYTES], dtype=STATS_DTYPE)[0]
    return {k: rec[k].item() for k in STATS_DTYPE.names}


def _require_weights(w) -> None:
    torch = _torch()
    if w.dtype != torch.float32 or not w.is_cuda or not w.is_contiguous() or w.dim() != 1:
        raise ValueError("weights must be a contiguous 1-D fp32 device tensor")


def _require_buffer(t, numel: int, dtype, name: str, device=None) -> None:
    """The kernels write (or read) `numel` elements through a plain pointer:
    the tensor must be a contiguous device tensor of that dtype holding at
    least that many, on the expected device."""
    if (t.dtype != dtype or not t.is_cuda or not t.is_contiguous() or t.numel() < numel
            or (device is not None and t.device != device)):
        raise ValueError(f"{name} must be a contiguous {dtype} device tensor of at least {numel} elements"
                         + (f" on {device}" if device is not None else ""))


class Resampler:
    """Holds a device workspace sized for (n_max, b_max) and calls mgp_resample."""

    def __init__(self, n_max: int, b_max: int = 0, device="cuda"):
        torch = _torch()
        self.device = torch.device(device)
        self.b_max = b_max
        self.ws_bytes = mgp_workspace_size(max(1, n_max), make_params(b_max=b_max))
        self.workspace = torch.empty(self.ws_bytes, dtype=torch.uint8, device=self.device)
        self.stats = torch.zeros(STATS_BYTES, dtype=torch.uint8, device=self.device)

    def resample(self, w, variant="megopolis", B: int = 0, epsilon: float = 0.01, seed: int = 0,
                 stream_id: int = 0, partition_bytes: int = 128, out=None, stream: int | None = None,
                 segment: int = 32):
        self._check_weights(w)
        torch = _torch()
        n = w.numel()
        if out is None:
            out = torch.empty(n, dtype=torch.int32, device=w.device)
        _require_buffer(out, n, torch.int32, "out (ancestors)", w.device)
        p = make_params(variant, B, epsilon, seed, stream_id, partition_bytes, self.b_max, segment)
        mgp_resample(w.data_ptr(), n, p, out.data_ptr(), self.stats.data_ptr(), self.workspace.data_ptr(),
                     self.ws_bytes, current_stream() if stream is None else stream)
        return out

    def resample_m(self, w, m: int, variant="megopolis", B: int = 0, epsilon: float = 0.01, seed: int = 0,
                   stream_id: int = 0, partition_bytes: int = 128, out=None, stream: int | None = None,
                 segment: int = 32):
        """m ancestors from the n = w.numel() weighted inputs (M != N)."""
        self._check_weights(w)
        torch = _torch()
        if out is None:
            out = torch.empty(int(m), dtype=torch.int32, device=w.device)
        _require_buffer(out, int(m), torch.int32, "out (ancestors)", w.device)
        p = make_params(variant, B, epsilon, seed, stream_id, partition_bytes, self.b_max, segment)
        mgp_resample_m(w.data_ptr(), w.numel(), int(m), p, out.data_ptr(), self.stats.data_ptr(),
                       self.workspace.data_ptr(), self.ws_bytes, current_stream() if stream is None else stream)
        return out

    def compute_B(self, w, variant="megopolis", B: int = 0, epsilon: float = 0.01, seed: int = 0,
                  stream_id: int = 0, partition_bytes: int = 128, stream: int | None = None,
                  segment: int = 32) -> None:
        """Reduction, B and offsets only (asynchronous; read last_stats() after a sync)."""
        self._check_weights(w)
        p = make_params(variant, B, epsilon, seed, stream_id, partition_bytes, self.b_max, segment)
        mgp_compute_B(w.data_ptr(), w.numel(), p, self.stats.data_ptr(), self.workspace.data_ptr(), self.ws_bytes,
                      current_stream() if stream is None else stream)

    def resample_prepared(self, w, variant="megopolis", B: int = 0, epsilon: float = 0.01, seed: int = 0,
                          stream_id: int = 0, partition_bytes: int = 128, out=None, stream: int | None = None,
                 segment: int = 32):
        """The accept loop only, after compute_B with the same arguments."""
        self._check_weights(w)
        torch = _torch()
        n = w.numel()
        if out is None:
            out = torch.empty(n, dtype=torch.int32, device=w.device)
        _require_buffer(out, n, torch.int32, "out (ancestors)", w.device)
        p = make_params(variant, B, epsilon, seed, stream_id, partition_bytes, self.b_max, segment)
        mgp_resample_prepared(w.data_ptr(), n, p, out.data_ptr(), self.workspace.data_ptr(), self.ws_bytes,
                              current_stream() if stream is None else stream)
        return out

    def _rows(self, w, states, out, anc, with_anc: bool):
        """Checks the states [n, d] and allocates the outputs of a fused call."""
        torch = _torch()
        n = w.numel()
        if states.dtype != torch.float32 or not states.is_cuda or not states.is_contiguous() or states.dim() < 1:
            raise ValueError("states must be a contiguous fp32 device tensor [n, d]")
        st2 = states.view(states.shape[0], -1)
        if st2.shape[0] != n or st2.device != w.device:
            raise ValueError(f"states must hold {n} rows on {w.device}")
        d = st2.shape[1]
        if out is None:
            out = torch.empty((n, d), dtype=torch.float32, device=w.device)
        _require_buffer(out, n * d, torch.float32, "out (x_bar)", w.device)
        if anc is None and with_anc:
            anc = torch.empty(n, dtype=torch.int32, device=w.device)
        if anc is not None:
            _require_buffer(anc, n, torch.int32, "anc (ancestors)", w.device)
        return st2, d, out, anc

    def resample_gather(self, w, states, variant="megopolis", B: int = 0, epsilon: float = 0.01, seed: int = 0,
                        stream_id: int = 0, partition_bytes: int = 128, out=None, anc=None, with_anc: bool = True,
                        stream: int | None = None, segment: int = 32):
        """mgp_resample_gather: returns (x_bar [n, d], ancestors or None)."""
        self._check_weights(w)
        st2, d, out, anc = self._rows(w, states, out, anc, with_anc)
        p = make_params(variant, B, epsilon, seed, stream_id, partition_bytes, self.b_max, segment)
        mgp_resample_gather(w.data_ptr(), w.numel(), p, st2.data_ptr(), d, anc.data_ptr() if anc is not None else 0,
                            out.data_ptr(), self.stats.data_ptr(), self.workspace.data_ptr(), self.ws_bytes,
                            current_stream() if stream is None else stream)
        return out, anc

    def resample_gather_prepared(self, w, states, variant="megopolis", B: int = 0, epsilon: float = 0.01,
                                 seed: int = 0, stream_id: int = 0, partition_bytes: int = 128, out=None, anc=None,
                                 with_anc: bool = True, stream: int | None = None, segment: int = 32):
        """The accept loop with the particle copy only, after compute_B with the same arguments."""
        self._check_weights(w)
        st2, d, out, anc = self._rows(w, states, out, anc, with_anc)
        p = make_params(variant, B, epsilon, seed, stream_id, partition_bytes, self.b_max, segment)
        mgp_resample_gather_prepared(w.data_ptr(), w.numel(), p, st2.data_ptr(), d,
                                     anc.data_ptr() if anc is not None else 0, out.data_ptr(),
                                     self.workspace.data_ptr(), self.ws_bytes,
                                     current_stream() if stream is None else stream)
        return out, anc

    def last_stats(self) -> dict:
        return decode_stats(self.stats)

    def _check_weights(self, w) -> None:
        _require_weights(w)
        if w.device != self.workspace.device:
            raise ValueError(f"weights are on {w.device}, the workspace on {self.workspace.device}")


class PrefixResampler:
    """Holds a workspace for mgp_resample_prefix (multinomial or systematic
    resampling, Algorithms 7 and 8) up to n_max particles."""

    def __init__(self, n_max: int, device="cuda"):
        torch = _torch()
        self.device = torch.device(device)
        self.ws_bytes = mgp_prefix_workspace_size(max(1, n_max))
        self.workspace = torch.empty(self.ws_bytes, dtype=torch.uint8, device=self.device)
        self.stats = torch.zeros(STATS_BYTES, dtype=torch.uint8, device=self.device)

    def resample(self, w, method="systematic", seed: int = 0, stream_id: int = 0, out=None,
                 stream: int | None = None):
        torch = _torch()
        _require_weights(w)
        if w.device != self.workspace.device:
            raise ValueError(f"weights are on {w.device}, the workspace on {self.workspace.device}")
        n = w.numel()
        if out is None:
            out = torch.empty(n, dtype=torch.int32, device=w.device)
        _require_buffer(out, n, torch.int32, "out (ancestors)", w.device)
        m = PREFIX_METHODS[method] if isinstance(method, str) else int(method)
        mgp_resample_prefix(w.data_ptr(), n, m, seed, stream_id, out.data_ptr(), self.stats.data_ptr(),
                            self.workspace.data_ptr(), self.ws_bytes, current_stream() if stream is None else stream)
        return out

    def last_stats(self) -> dict:
        return decode_stats(self.stats)


def resample(w, variant="megopolis", B: int = 0, epsilon: float = 0.01, seed: int = 0, stream_id: int = 0,
             partition_bytes: int = 128, b_max: int = 0, segment: int = 32):
    """One-shot resample of a device weight vector; returns (ancestors, stats dict)."""
    r = Resampler(w.numel(), b_max, w.device)
    anc = r.resample(w, variant, B, epsilon, seed, stream_id, partition_bytes, segment=segment)
    return anc, r.last_stats()


def gather(states, anc, out=None, stream: int | None = None):
    """out[i] = states[anc[i]] for fp32 states [n_states, d] on the device."""
    torch = _torch()
    if states.dtype != torch.float32 or not states.is_cuda or not states.is_contiguous() or states.dim() < 1:
        raise ValueError("states must be a contiguous fp32 device tensor [n_states, d]")
    if anc.dtype != torch.int32 or not anc.is_cuda or not anc.is_contiguous():
        raise ValueError("ancestors must be a contiguous int32 device tensor")
    st2 = states.view(states.shape[0], -1)
    n_states, d = st2.shape
    n_out = anc.numel()
    if anc.device != states.device:
        raise ValueError("ancestors and states must be on the same device")
    if out is None:
        out = torch.empty((n_out, d), dtype=torch.float32, device=states.device)
    _require_buffer(out, n_out * d, torch.float32, "out (gathered states)", states.device)
    mgp_gather(st2.data_ptr(), n_states, d, anc.data_ptr(), n_out, out.data_ptr(),
               current_stream() if stream is None else stream)
    return out


class BatchPlan:
    """Owns an mgp_batch_plan over device tensors.

    filters: list of dicts with keys w (device fp32 [n]), anc (device int32
    [n]), and optionally B, epsilon, seed, stream_id, states ([n, d]) and out
    ([n, d]). The tensors must stay alive as long as the plan."""

    def __init__(self, filters, variant="megopolis", d: int = 0, partition_bytes: int = 128, b_max: int = 0,
                 block_threads: int = 0, particles_per_thread: int = 0, schedule: int = 0, use_graph: bool = True,
                 tune_cache: str | None = None, stream: int | None = None):
        torch = _torch()
        self.filters = filters
        descs = []
        for k, f in enumerate(filters):
            st = f.get("states")
            _require_weights(f["w"])
            n = f["w"].numel()
            dev = f["w"].device
            _require_buffer(f["anc"], n, torch.int32, f"filter {k}: anc", dev)
            if st is not None:
                _require_buffer(st, n * max(int(d), 1), torch.float32, f"filter {k}: states", dev)
                _require_buffer(f["out"], n * max(int(d), 1), torch.float32, f"filter {k}: out", dev)
            if f.get("stats") is not None:
                _require_buffer(f["stats"], STATS_BYTES, torch.uint8, f"filter {k}: stats", dev)
            descs.append(mgp_filter_desc(f["w"].data_ptr(), f["w"].numel(), int(f.get("B", 0)),
                                         float(f.get("epsilon", 0.01)), int(f.get("seed", 0)) & (2**64 - 1),
                                         int(f.get("stream_id", 0)), 0, f["anc"].data_ptr(),
                                         st.data_ptr() if st is not None else None,
                                         f["out"].data_ptr() if st is not None else None,
                                         f["stats"].data_ptr() if f.get("stats") is not None else None))
        v = VARIANTS[variant] if isinstance(variant, str) else int(variant)
        self._cache = tune_cache.encode() if tune_cache else None
        cfg = mgp_batch_config(v, int(d), int(partition_bytes), int(b_max), int(block_threads),
                               int(particles_per_thread), int(schedule), 1 if use_graph else 0, self._cache)
        self.plan = mgp_batch_plan_create(descs, cfg, current_stream() if stream is None else stream)

    def info(self) -> dict:
        return mgp_batch_plan_info(self.plan)

    def set_seeds(self, seeds, stream: int | None = None) -> None:
        mgp_batch_set_seeds(self.plan, seeds, current_stream() if stream is None else stream)

    def run(self, stream: int | None = None) -> None:
        mgp_batch_run(self.plan, current_stream() if stream is None else stream)

    def run_separate(self, stream: int | None = None) -> None:
        mgp_batch_run_separate(self.plan, current_stream() if stream is None else stream)

    def close(self) -> None:
        if self.plan:
            mgp_batch_plan_destroy(self.plan)
            self.plan = 0

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """A resample server (mgp_server_*). Requests name device tensors (or raw
    device addresses) for weights and states; outputs are owned by the
    server until release()."""

    def __init__(self, variant="megopolis", d: int = 0, hbm_budget: int = 16 << 30, streams: int = 4,
                 max_batch: int = 64, max_batch_particles: int = 0, max_n: int = 0, b_max: int = 0,
                 partition_bytes: int = 128, simulate: bool = False, sim_us_fixed: float = 0.0,
                 sim_ns_per_particle: float = 0.0, sim_fail_every: int = 0):
        v = VARIANTS[variant] if isinstance(variant, str) else int(variant)
        cfg = mgp_server_config(v, int(d), int(partition_bytes), int(b_max), int(hbm_budget), int(streams),
                                int(max_batch), int(max_batch_particles), int(max_n), 1 if simulate else 0,
                                float(sim_us_fixed), float(sim_ns_per_particle), int(sim_fail_every), 0)
        self.handle = mgp_server_create(cfg)
        self.d = d

    def submit(self, w, n: int | None = None, B: int = 0, epsilon: float = 0.01, seed: int = 0, stream_id: int = 0,
               states=None) -> int:
        if not isinstance(w, int):
            _require_weights(w)
            if n is not None and int(n) > w.numel():
                raise ValueError(f"n = {n} exceeds the {w.numel()} weights given")
        if states is not None and not isinstance(states, int):
            nn = n if n is not None else w.numel()
            _require_buffer(states, int(nn) * max(int(self.d), 1), _torch().float32, "states")
        wp = w if isinstance(w, int) else w.data_ptr()
        n = n if n is not None else w.numel()
        sp = None if states is None else (states if isinstance(states, int) else states.data_ptr())
        req = mgp_request(wp, int(n), int(B), float(epsilon), int(seed) & (2**64 - 1), int(stream_id), 0, sp)
        return mgp_server_submit(self.handle, req)

    def poll(self, ticket: int) -> dict:
        return mgp_server_poll(self.handle, ticket)

    def wait(self, ticket: int, timeout_ms: float = -1.0) -> dict:
        return mgp_server_wait(self.handle, ticket, timeout_ms)

    def cancel(self, ticket: int) -> None:
        mgp_server_cancel(self.handle, ticket)

    def release(self, ticket: int) -> None:
        mgp_server_release(self.handle, ticket)

    def stats(self) -> dict:
        return mgp_server_get_stats(self.handle)

    def outputs(self, ticket: int, result: dict):
        """Copies a finished request's ancestors (and gathered states) into new
        device tensors with mgp_server_copy_outputs; returns host numpy arrays."""
        torch = _torch()
        n = result["n"]
        anc = torch.empty(n, dtype=torch.int32, device="cuda")
        out = torch.empty((n, self.d), dtype=torch.float32, device="cuda") if result["out_states_dev"] else None
        mgp_server_copy_outputs(self.handle, ticket, anc.data_ptr(), out.data_ptr() if out is not None else 0,
                                current_stream())
        torch.cuda.synchronize()
        return anc.cpu().numpy(), (out.cpu().numpy() if out is not None else None)

    def close(self) -> None:
        if self.handle:
            mgp_server_destroy(self.handle)
            self.handle = 0

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class SirFilter:
    """Owns an mgp_sir_filter: R runs of the SIR filter of Algorithm 6, n
    particles each, T steps, stage 2 done by `variant` with B iterations (or B
    from epsilon per step when B is 0), or by the prefix-sum method
    "multinomial" or "systematic" (Algorithms 7 and 8; B unused)."""

    def __init__(self, runs: int, n: int, steps: int, variant="megopolis", B: int = 16, epsilon: float = 0.1,
                 seed: int = 0, partition_bytes: int = 128, b_max: int = 0, use_graph: bool = True,
                 block_threads: int = 0, particles_per_thread: int = 0, stream: int | None = None):
        v = SIR_VARIANTS[variant] if isinstance(variant, str) else int(variant)
        cfg = mgp_sir_config(v, int(runs), int(n), int(steps), int(B), int(partition_bytes), float(epsilon),
                             int(seed) & (2**64 - 1), int(b_max), 1 if use_graph else 0, int(block_threads),
                             int(particles_per_thread), 0, 0)
        self.runs, self.n, self.steps = int(runs), int(n), int(steps)
        self.filt = mgp_sir_create(cfg, current_stream() if stream is None else stream)

    def _s(self, stream):
        return current_stream() if stream is None else stream

    def set_measurements(self, z, stream: int | None = None) -> None:
        z = np.ascontiguousarray(z, dtype=np.float64)
        if z.shape != (self.runs, self.steps + 1):
            raise ValueError(f"measurements must have shape ({self.runs}, {self.steps + 1})")
        mgp_sir_set_measurements(self.filt, z, self._s(stream))

    def reset(self, x0, stream: int | None = None) -> None:
        torch = _torch()
        if (x0.dtype != torch.float32 or not x0.is_cuda or not x0.is_contiguous()
                or tuple(x0.shape) != (self.runs, self.n)):
            raise ValueError(f"initial particles must be a contiguous fp32 device tensor of shape "
                             f"({self.runs}, {self.n})")
        mgp_sir_reset(self.filt, x0.data_ptr(), self._s(stream))

    def predict_update(self, t: int, stream: int | None = None) -> None:
        mgp_sir_predict_update(self.filt, t, self._s(stream))

    def resample(self, t: int, stream: int | None = None) -> None:
        mgp_sir_resample(self.filt, t, self._s(stream))

    def estimate(self, t: int, stream: int | None = None) -> None:
        mgp_sir_estimate(self.filt, t, self._s(stream))

    def step(self, t: int, stream: int | None = None) -> None:
        self.predict_update(t, stream)
        self.resample(t, stream)
        self.estimate(t, stream)

    def run(self, stream: int | None = None) -> None:
        mgp_sir_run(self.filt, self._s(stream))

    def results(self, stream: int | None = None):
        """(estimates [R, T] fp64, B [R, T] uint32, status [R, T] int32)."""
        est = np.zeros((self.runs, self.steps), dtype=np.float64)
        B = np.zeros((self.runs, self.steps), dtype=np.uint32)
        st = np.zeros((self.runs, self.steps), dtype=np.int32)
        mgp_sir_results(self.filt, est, B, st, self._s(stream))
        return est, B, st

    def buffers(self) -> dict:
        return mgp_sir_get_buffers(self.filt)

    def copy(self, name: str, stream: int | None = None):
        """A new device tensor [R, n] holding 'x', 'w', 'xbar' (fp32) or 'ancestors' (int32)."""
        torch = _torch()
        which = {"x": MGP_SIR_X, "w": MGP_SIR_W, "xbar": MGP_SIR_XBAR, "ancestors": MGP_SIR_ANCESTORS}[name]
        out = torch.empty((self.runs, self.n), dtype=torch.int32 if name == "ancestors" else torch.float32,
                          device="cuda")
        mgp_sir_copy_buffer(self.filt, which, out.data_ptr(), self._s(stream))
        return out

    def close(self) -> None:
        if self.filt:
            mgp_sir_destroy(self.filt)
            self.filt = 0

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
