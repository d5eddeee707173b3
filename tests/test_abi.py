"""The C ABI library loads and exports everything include/gcpush.h declares;
struct layouts seen from Python match the C compiler's; host-side argument
checks work without a GPU."""
import ctypes as C
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gcpush.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?[\w\s\*]+?\b(gc_\w+)\s*\(", text, flags=re.M)))


def test_library_exports_every_declared_symbol():
    from paper_2403_06706_amd import _abi
    lib = C.CDLL(_abi.LIB_PATH)
    names = _declared()
    assert len(names) >= 15
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing
    assert sorted(_abi.DECLARED) == names


def test_struct_layouts_match_c(tmp_path):
    from paper_2403_06706_amd import _abi
    structs = ["gc_options", "gc_field_desc", "gc_inject_desc", "gc_moment_spec", "gc_state_view", "gc_counters",
               "gc_tune_space", "gc_tune_result", "gc_mlp_desc", "gc_mlp_train_opts"]
    src = tmp_path / "sz.c"
    body = "".join(f'printf("{s} %zu\\n", sizeof({s}));' for s in structs)
    src.write_text(f'#include <stdio.h>\n#include "gcpush.h"\nint main(void){{{body}return 0;}}\n')
    exe = tmp_path / "sz"
    subprocess.check_call(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)])
    out = subprocess.check_output([str(exe)]).decode().split()
    sizes = dict(zip(out[0::2], map(int, out[1::2])))
    for s in structs:
        assert C.sizeof(getattr(_abi, s)) == sizes[s], s


def test_host_side_errors_without_device():
    from paper_2403_06706_amd import _abi
    lib = _abi.load()
    # null context / arguments are rejected before any device work
    assert lib.gc_advance(None, 1.0, 10) == _abi.GC_EINVAL
    assert lib.gc_inject(None, None) == _abi.GC_EINVAL
    assert lib.gc_moments_size(None) == -1
    o = _abi.gc_options()
    lib.gc_default_options(C.byref(o))
    # the defaults gcpush.h documents for gc_default_options
    assert o.precision == _abi.GC_PREC_F64 and o.order == _abi.GC_ORDER_BIN
    assert o.chunk_steps == 64 and o.bin_coarsen == 0 and o.block_size == 64
    assert o.persistent == 0 and o.tile == 1024 and o.log_depth == 0 and o.timing == 0
    assert o.field_source == _abi.GC_SOURCE_GRID and o.tail_threshold == 131072
    assert not o.dev_alloc and not o.dev_free and not o.hip_stream and o.device == 0
    # invalid options are reported with a message, on a context that must be destroyed
    o.block_size = 100
    h = C.c_void_p()
    st = lib.gc_create(C.byref(h), C.byref(o))
    assert st == _abi.GC_EINVAL
    assert b"block_size" in lib.gc_last_error(h)
    lib.gc_destroy(h)
    o.block_size = 256
    o.timing = 3
    st = lib.gc_create(C.byref(h), C.byref(o))
    assert st == _abi.GC_EINVAL
    assert b"timing" in lib.gc_last_error(h)
    lib.gc_destroy(h)
    o.timing = 0
    o.field_source = 7
    st = lib.gc_create(C.byref(h), C.byref(o))
    assert st == _abi.GC_EINVAL
    assert b"field_source" in lib.gc_last_error(h)
    lib.gc_destroy(h)
    # an allocator needs both callbacks
    o.field_source = 0
    keep = _abi.DEV_ALLOC_FN(lambda n, user: None)
    o.dev_alloc = keep
    st = lib.gc_create(C.byref(h), C.byref(o))
    assert st == _abi.GC_EINVAL
    assert b"dev_alloc" in lib.gc_last_error(h)
    lib.gc_destroy(h)
    assert lib.gc_mlp_eval(None, None, 0, None) == _abi.GC_EINVAL
    assert lib.gc_mlp_train_step(None, None, None, 1, None, None) == _abi.GC_EINVAL


def test_create_reports_missing_device():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    from paper_2403_06706_amd import _abi
    lib = _abi.load()
    o = _abi.gc_options()
    lib.gc_default_options(C.byref(o))
    h = C.c_void_p()
    st = lib.gc_create(C.byref(h), C.byref(o))
    assert st == _abi.GC_EDEVICE
    lib.gc_destroy(h)
