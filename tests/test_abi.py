"""The C-ABI library loads and exports every entry point of include/zfpx.h;
argument errors are reported before anything reaches a GPU."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "zfpx.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    text = re.sub(r"^\s*#.*$", "", text, flags=re.M)  # preprocessor lines
    return sorted(set(re.findall(r"\b([A-Za-z_][A-Za-z0-9_]*)\s*\(", text)) -
                  {"sizeof", "defined"})


def test_header_declares_the_hot_path():
    names = _declared()
    for n in ("zfpx_encode_fixed_rate", "zfpx_decode_fixed_rate", "zfpx_pack_encode",
              "zfpx_decode_unpack", "f16_truncate", "f16_restore"):
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_2609_24294_amd import zfpx
    lib = zfpx.library()
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_argument_errors_without_gpu():
    from paper_2609_24294_amd import zfpx
    L = zfpx.library()
    fake = 4096  # never dereferenced: every call below fails its checks first
    # bad rates
    for r in (0, -1, 33):
        assert L.zfpx_encode_fixed_rate(fake, 4, 4, 4, 1, 4, 16, r, fake, 1 << 20, None) == zfpx.EINVAL
        assert L.zfpx_fixed_rate_bytes(4, 4, 4, r) == zfpx.EINVAL
    # output too small, misaligned output, null input
    assert L.zfpx_encode_fixed_rate(fake, 4, 4, 4, 1, 4, 16, 8, fake, 63, None) == zfpx.ENOSPC
    assert L.zfpx_encode_fixed_rate(fake, 4, 4, 4, 1, 4, 16, 8, fake + 4, 64, None) == zfpx.EINVAL
    assert L.zfpx_encode_fixed_rate(None, 4, 4, 4, 1, 4, 16, 8, fake, 64, None) == zfpx.EINVAL
    assert L.zfpx_decode_fixed_rate(fake, 10, 4, 4, 4, 1, 4, 16, 8, fake, None) == zfpx.ENOSPC
    assert L.zfpx_decode_fixed_rate(fake, 64, -1, 4, 4, 1, 4, 16, 8, fake, None) == zfpx.EINVAL
    # empty arrays and empty f16 buffers are no-ops
    assert L.zfpx_encode_fixed_rate(None, 0, 4, 4, 1, 4, 16, 8, None, 0, None) == zfpx.OK
    assert L.f16_truncate(None, 0, None, None) == zfpx.OK
    assert L.f16_restore(fake, 8, fake + 1, None) == zfpx.EINVAL
    # sizes
    assert L.zfpx_fixed_rate_bytes(128, 64, 8, 16) == 1024 * 8 * 16
    assert L.zfpx_fixed_rate_bytes(5, 1, 1, 1) == 2 * 8
    assert L.zfpx_status_string(zfpx.ENOSPC) == b"output buffer too small"


def test_plan_table_checks_without_gpu():
    from paper_2609_24294_amd import zfpx
    import numpy as np
    # zero chunks: valid and empty (no device tables needed)
    p = zfpx.Plan([], [], [], [0], [], [])
    assert p.nblocks == 0 and p.sizes(8)[2] == 0
    p.close()
    # a row of length 0 is rejected
    with pytest.raises(zfpx.ZfpxError):
        zfpx.Plan([0], [16], [1], [0, 1], [0], [0])
    # row_start must start at 0 and not decrease
    with pytest.raises(zfpx.ZfpxError):
        zfpx.Plan([0], [16], [1], [1, 2], [0, 0], [4, 4])


def test_variable_mode_host_checks_without_gpu():
    from paper_2609_24294_amd import zfpx
    L = zfpx.library()
    # minexp of accuracy mode: the largest e with 2^e <= tolerance
    assert L.zfpx_accuracy_minexp(1.0) == 0
    assert L.zfpx_accuracy_minexp(0.75) == -1
    assert L.zfpx_accuracy_minexp(2.0 ** -20) == -20
    assert L.zfpx_accuracy_minexp(1000.0) == 9
    assert L.zfpx_accuracy_minexp(0.0) == zfpx.MINEXP_NONE
    assert L.zfpx_accuracy_minexp(-1.0) == zfpx.MINEXP_NONE
    fake = 4096
    assert L.zfpx_plan_var_sizes(None, 16, None, None, None) == zfpx.EINVAL
    p = zfpx.Plan([], [], [], [0], [], [])  # empty plan: no device tables
    assert zfpx.zfpx_plan_var_sizes(p, 16) == (0, 0, 0)
    for mp, me, cap in ((0, 0, 16), (33, 0, 16), (32, -1075, 16), (32, 1025, 16), (32, 0, 0),
                        (32, 0, 33)):
        assert L.zfpx_plan_encode_var(p.handle, fake, 0, mp, me, cap, fake, 64, fake, fake,
                                      fake, 64, None) == zfpx.EINVAL
        assert L.zfpx_plan_decode_var(p.handle, fake, 64, fake, fake, mp, me, cap, fake, 0,
                                      None) == zfpx.EINVAL
    # nothing to code: no launch
    assert L.zfpx_plan_encode_var(p.handle, None, 0, 16, zfpx.MINEXP_NONE, 16, None, 0, None,
                                  None, None, 0, None) == zfpx.OK
    assert L.zfpx_plan_decode_var(p.handle, None, 0, None, None, 32, -10, 8, None, 0,
                                  None) == zfpx.OK
    p.close()



def test_pipeline_host_checks_without_gpu():
    from paper_2609_24294_amd import zfpx
    L = zfpx.library()
    import ctypes
    h = ctypes.c_void_p()
    assert L.zfpx_pipeline_create(None, 16, 4, ctypes.byref(h)) == zfpx.EINVAL
    p = zfpx.Plan([], [], [], [0], [], [])
    assert L.zfpx_pipeline_create(p.handle, 0, 4, ctypes.byref(h)) == zfpx.EINVAL
    assert L.zfpx_pipeline_create(p.handle, 16, 0, ctypes.byref(h)) == zfpx.EINVAL
    assert L.zfpx_pipeline_send(None, None, 0, None, 0, None, 0, None, None) == zfpx.EINVAL
    assert L.zfpx_pipeline_recv(None, None, 0, None, 0, None, 0, None, None) == zfpx.EINVAL
    assert L.zfpx_pipeline_destroy(None) == zfpx.EINVAL
    p.close()
