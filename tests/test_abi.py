"""C-ABI checks that need no GPU: the library loads, exports every function
that include/juqcs_gpu.h declares, and rejects bad arguments on the host
before anything is launched."""
import ctypes as ct
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "juqcs_gpu.h")).read()
    return sorted(set(re.findall(r"^\s*(?:juqcs_status|const char\*)\s+(juqcs_\w+)\s*\(", text, re.M)))


@pytest.fixture(scope="module")
def J():
    from paper_1912_03243_amd import juqcs
    return juqcs


def test_every_declared_symbol_is_exported(J):
    names = declared_functions()
    assert len(names) >= 25
    lib = ct.CDLL(J.LIB_PATH)
    for name in names:
        assert hasattr(lib, name), name
    assert sorted(J.EXPORTED) == names


def test_version(J):
    assert "gfx950" in J.juqcs_version()


def test_state_bytes(J):
    assert J.juqcs_state_bytes(30, J.C128) [0] == 16 << 30
    assert J.juqcs_state_bytes(34, J.C64)[0] == 8 << 34
    a, s, w = J.juqcs_state_bytes(36, J.ENC2, 8)
    assert a == 2 << 36 and s == 4 << 28 and w > 0
    a, s, _ = J.juqcs_state_bytes(20, J.ENC2, 10)
    assert s == 4 << 10


@pytest.mark.parametrize("n, dt, bb, status", [
    (0, 0, 0, -1), (41, 0, 0, -1), (10, 7, 0, -3), (10, 2, 2, -1), (10, 2, 13, -1), (5, 2, 8, -1)])
def test_state_bytes_errors(J, n, dt, bb, status):
    with pytest.raises(J.JuqcsError) as e:
        J.juqcs_state_bytes(n, dt, bb)
    assert e.value.status == status
    assert J.juqcs_last_error()


def test_create_rejects_bad_buffers_before_any_device_call(J):
    h = ct.c_void_p()
    lib = J._lib
    assert lib.juqcs_state_create(None, 4, 0, 0, 16, 1 << 8, None, 0, None, 0, None) == J.ERR_ARG
    assert lib.juqcs_state_create(ct.byref(h), 4, 0, 0, None, 1 << 8, None, 0, None, 0, None) == J.ERR_ARG
    # misaligned amplitude pointer
    assert lib.juqcs_state_create(ct.byref(h), 4, 0, 0, 8, 1 << 8, None, 0, None, 0, None) == J.ERR_ARG
    # too small
    assert lib.juqcs_state_create(ct.byref(h), 4, 0, 0, 16, 255, None, 0, None, 0, None) == J.ERR_SIZE
    # ENC2 without scales
    assert lib.juqcs_state_create(ct.byref(h), 8, 2, 0, 16, 512, None, 0, None, 0, None) == J.ERR_ARG
    # workspace too small
    assert lib.juqcs_state_create(ct.byref(h), 4, 0, 0, 16, 256, None, 0, 32, 16, None) == J.ERR_SIZE
    assert h.value is None


def test_null_handle_and_codec_errors(J):
    lib = J._lib
    u = (ct.c_double * 8)()
    assert lib.juqcs_apply_1q(None, 0, u) == J.ERR_ARG
    assert lib.juqcs_state_init(None, 0) == J.ERR_ARG
    assert lib.juqcs_norm(None, None) == J.ERR_ARG
    assert lib.juqcs_state_destroy(None) == J.OK
    assert lib.juqcs_encode2(16, 2, 8, 8, 16, 16, None) == J.ERR_DTYPE
    assert lib.juqcs_encode2(16, 0, 8, 2, 16, 16, None) == J.ERR_ARG
    assert lib.juqcs_decode2(16, 16, 8, 8, 16, 2, None) == J.ERR_DTYPE
    assert lib.juqcs_copy(16, 16, 15, None) == J.ERR_ARG
    assert lib.juqcs_copy(None, 16, 16, None) == J.ERR_ARG
