"""CPU-only checks of the HIP library's C ABI: it loads, exports every entry
point include/mgp.h declares, and answers the host-only calls (no device
work is launched here)."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mgp.h")


@pytest.fixture(scope="module")
def mgp():
    from paper_2109_13504_amd import mgp as m
    from paper_2109_13504_amd.csrc import build as b
    if b.needs_build():
        b.build()
    m.lib()
    return m


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\s*\*?\s*(mgp_[A-Za-z_0-9]+)\s*\(", text, flags=re.M)
    return sorted(set(names))


def test_header_declares_entry_points():
    names = declared_functions()
    for required in ("mgp_resample", "mgp_gather", "mgp_compute_B", "mgp_workspace_size", "mgp_last_error"):
        assert required in names


def test_library_exports_every_declared_symbol(mgp):
    out = subprocess.run(["nm", "-D", "--defined-only", mgp.LIB_PATH], capture_output=True, text=True,
                         check=True).stdout
    exported = {ln.split()[-1] for ln in out.splitlines() if ln.strip()}
    missing = [f for f in declared_functions() if f not in exported]
    assert not missing, missing
    lib = ctypes.CDLL(mgp.LIB_PATH)
    for f in declared_functions():
        assert hasattr(lib, f)


def test_struct_layouts_match_header(mgp, tmp_path):
    """sizeof / offsetof of every ABI struct, from a C program built against
    include/mgp.h, equal the ctypes mirrors in the binding."""
    import json
    exe = tmp_path / "abi_layout"
    subprocess.run(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), "-o", str(exe),
                    os.path.join(ROOT, "tests", "helpers", "abi_layout.c")], check=True)
    layout = json.loads(subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout)
    for name in ("mgp_params", "mgp_stats", "mgp_filter_desc", "mgp_batch_config", "mgp_batch_info",
                 "mgp_server_config", "mgp_request", "mgp_request_result", "mgp_server_stats", "mgp_sir_config",
                 "mgp_sir_buffers"):
        cls = getattr(mgp, name)
        assert ctypes.sizeof(cls) == layout[name], name
        for field, _ in cls._fields_:
            assert getattr(cls, field).offset == layout[f"{name}.{field}"], (name, field)


def test_workspace_size_host_only(mgp):
    small = mgp.mgp_workspace_size(100, mgp.make_params(b_max=16))
    big = mgp.mgp_workspace_size(100, mgp.make_params(b_max=65536))
    assert big >= small + 4 * (65536 - 16) - 256
    assert small % 256 == 0


def test_argument_errors_before_any_device_call(mgp):
    with pytest.raises(mgp.MgpError) as e:
        mgp.mgp_workspace_size(0, mgp.make_params())
    assert e.value.code == mgp.MGP_EINVAL
    with pytest.raises(mgp.MgpError) as e:
        mgp.mgp_workspace_size(10, mgp.make_params(variant=7))
    assert e.value.code == mgp.MGP_EINVAL
    with pytest.raises(mgp.MgpError) as e:
        mgp.mgp_workspace_size(10, mgp.make_params(B=100, b_max=50))
    assert e.value.code == mgp.MGP_ERANGE
    with pytest.raises(mgp.MgpError) as e:
        mgp.mgp_resample(0, 10, mgp.make_params(), 0, 0, 0, 0, 0)
    assert e.value.code == mgp.MGP_EINVAL
    assert "NULL" in mgp.mgp_last_error()
    with pytest.raises(mgp.MgpError) as e:
        mgp.mgp_gather(0, 10, 4, 0, 10, 0, 0)
    assert e.value.code == mgp.MGP_EINVAL
    # the fused entry points check the row arguments before any device work
    with pytest.raises(mgp.MgpError) as e:
        mgp.mgp_resample_gather(16, 10, mgp.make_params(B=3), 0, 4, 0, 16, 0, 0, 0, 0)
    assert e.value.code == mgp.MGP_EINVAL
    with pytest.raises(mgp.MgpError) as e:
        mgp.mgp_resample_gather_prepared(16, 10, mgp.make_params(B=3), 256, 0, 0, 4096, 0, 0, 0)
    assert e.value.code == mgp.MGP_EINVAL
    assert "d must be" in mgp.mgp_last_error()
    with pytest.raises(mgp.MgpError) as e:
        mgp.mgp_prefix_workspace_size(0)
    assert e.value.code == mgp.MGP_EINVAL
    with pytest.raises(mgp.MgpError) as e:  # unknown method, before any device call
        mgp.mgp_resample_prefix(16, 10, 5, 1, 0, 16, 0, 256, 1 << 20, 0)
    assert e.value.code == mgp.MGP_EINVAL
    assert mgp.mgp_prefix_workspace_size(1 << 20) >= 8 << 20


def test_noalloc_size_limit_checked_on_the_host(mgp):
    """mgp_resample_noalloc rejects a size whose workspace exceeds its static
    scratch before any device call (the pointers are never dereferenced)."""
    p = mgp.make_params("megopolis")
    n = 9_000_000
    assert mgp.mgp_workspace_size(n, p) > mgp.MGP_NOALLOC_SCRATCH_BYTES
    with pytest.raises(mgp.MgpError) as e:
        mgp.mgp_resample_noalloc(16, n, p, 16, 0, 0)
    assert e.value.code == mgp.MGP_ERANGE
    assert "scratch" in mgp.mgp_last_error()
    with pytest.raises(mgp.MgpError) as e:
        mgp.mgp_resample_noalloc(0, 100, p, 16, 0, 0)
    assert e.value.code == mgp.MGP_EINVAL


def test_probe_argument_errors_before_any_device_call(mgp):
    """The memory probes check their arguments on the host (the pointers are
    never dereferenced when a check fails)."""
    n = 1 << 20
    ok = 4 * (2 * n + 1024)
    for args, code in [((0, ok, n, 16, 10, 16), mgp.MGP_EINVAL),        # NULL mirror
                       ((16, ok, n + 5, 16, 10, 16), mgp.MGP_EINVAL),   # n not a multiple of 1024
                       ((16, ok, n, 16, 7, 16), mgp.MGP_EINVAL),        # steps not a multiple of 5
                       ((16, ok - 4, n, 16, 10, 16), mgp.MGP_EINVAL),   # mirror too small
                       ((16, 1 << 33, 1 << 30, 16, 10, 16), mgp.MGP_ERANGE)]:  # n above 2^29
        with pytest.raises(mgp.MgpError) as e:
            mgp.mgp_probe_pattern_read(*args, 0)
        assert e.value.code == code, (args, mgp.mgp_last_error())
    with pytest.raises(mgp.MgpError) as e:
        mgp.mgp_probe_stream_read(16, 24, 1, 1, 16, 0)  # bytes not a multiple of 16
    assert e.value.code == mgp.MGP_EINVAL


def test_version(mgp):
    assert mgp.mgp_version() >= 100


def test_plain_c_client_builds_against_the_header_and_library():
    """A C program using only include/mgp.h and the HIP runtime's C API
    compiles without warnings and links against libmgp.so (it runs in the
    GPU tests)."""
    from helpers import build_c_client
    exe = build_c_client()
    assert os.access(exe, os.X_OK)
