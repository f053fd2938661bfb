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
    # workspace: required (the library never allocates), 256-byte aligned, large enough
    assert lib.juqcs_state_create(ct.byref(h), 4, 0, 0, 16, 256, None, 0, None, 0, None) == J.ERR_ARG
    assert lib.juqcs_state_create(ct.byref(h), 4, 0, 0, 16, 256, None, 0, 32, 1 << 30, None) == J.ERR_ARG
    assert lib.juqcs_state_create(ct.byref(h), 4, 0, 0, 16, 256, None, 0, 256, 16, None) == J.ERR_SIZE
    assert h.value is None


def test_global_factor_rejects_bad_arguments(J):
    lib = J._lib
    g = (ct.c_double * 2)(1.0, 0.0)
    assert lib.juqcs_set_global_factor(None, g) == J.ERR_ARG
    assert lib.juqcs_mul_global_factor(None, g) == J.ERR_ARG
    assert lib.juqcs_get_global_factor(None, g) == J.ERR_ARG
    assert lib.juqcs_renormalize(None, None) == J.ERR_ARG


def _batch_args(J, ns, soff):
    import numpy as np
    from paper_1912_03243_amd import workloads as W
    circs = [W.layered_brick(n, 2, seed=n) for n in ns]
    offs = np.zeros(len(ns) + 1, dtype=np.int64)
    offs[1:] = np.cumsum([len(c) for c in circs])
    g = np.ascontiguousarray(np.concatenate(circs))
    nn = np.array(ns, dtype=np.int32)
    so = np.array(soff, dtype=np.uint64)
    keep = (g, nn, offs, so)
    return keep, (len(ns), nn.ctypes.data_as(ct.POINTER(ct.c_int)), g.ctypes.data,
                  offs.ctypes.data_as(ct.POINTER(ct.c_int64)))


def test_batch_create_checks_the_state_buffer_on_the_host(J):
    # states past the end of the buffer, overlapping regions and misaligned
    # buffers are rejected before any device work (the pointer is never used)
    lib = J._lib
    h = ct.c_void_p()
    keep, a = _batch_args(J, [4, 5], [0, 256])
    so = keep[3].ctypes.data_as(ct.POINTER(ct.c_uint64))
    need = 256 + (8 << 5)
    assert lib.juqcs_batch_create(ct.byref(h), *a, 256, need - 1, so, None) == J.ERR_SIZE
    assert lib.juqcs_batch_create(ct.byref(h), *a, 8, need, so, None) == J.ERR_ARG
    keep2, a2 = _batch_args(J, [4, 5], [0, 64])      # 8 * 2^4 = 128 bytes: overlaps
    so2 = keep2[3].ctypes.data_as(ct.POINTER(ct.c_uint64))
    assert lib.juqcs_batch_create(ct.byref(h), *a2, 256, 1 << 20, so2, None) == J.ERR_ARG
    assert h.value is None


def test_batch_workspace_is_sized_and_required(J):
    lib = J._lib
    h = ct.c_void_p()
    keep, a = _batch_args(J, [4, 5], [0, 256])
    so = keep[3].ctypes.data_as(ct.POINTER(ct.c_uint64))
    assert lib.juqcs_batch_create(ct.byref(h), *a, 256, 1 << 20, so, None) == J.OK
    try:
        b = ct.c_size_t()
        assert lib.juqcs_batch_bytes(h, ct.byref(b)) == J.OK
        assert b.value >= 4 << 20
        # no workspace bound yet: nothing runs or reads
        assert lib.juqcs_batch_run(h, None) == J.ERR_ARG
        assert lib.juqcs_batch_norms(h, (ct.c_double * 2)(), None) == J.ERR_ARG
        assert lib.juqcs_batch_autotune(h, None) == J.ERR_ARG
        # too small, misaligned, null
        assert lib.juqcs_batch_bind(h, 256, b.value - 1, None) == J.ERR_SIZE
        assert lib.juqcs_batch_bind(h, 16, b.value, None) == J.ERR_ARG
        assert lib.juqcs_batch_bind(h, None, b.value, None) == J.ERR_ARG
    finally:
        assert lib.juqcs_batch_destroy(h) == J.OK


def test_branch_workspace_is_sized_and_required(J):
    import numpy as np
    from paper_1912_03243_amd import workloads as W
    lib = J._lib
    circ, side = W.grid_circuit(2, 4, 4, 3, max_cross=None)
    n = 8
    z = np.arange(16, dtype=np.uint64)
    mn, full = J.juqcs_branch_bytes(n, circ, side, 1, z.size, 0, True)
    assert 0 < mn <= full
    mn1, g1 = J.juqcs_branch_bytes(n, circ, side, 1, z.size, 1, True)
    assert mn1 == mn and g1 == mn
    dmn, _ = J.juqcs_branch_bytes(n, circ, side, 1, z.size, 1, False)
    assert dmn < mn                       # no staged bitstrings or result
    out = np.zeros(2 * z.size)
    sp = side.ctypes.data_as(ct.POINTER(ct.c_uint8))
    zp = z.ctypes.data_as(ct.POINTER(ct.c_uint64))
    args = (n, circ.ctypes.data, circ.size, sp, zp, z.size)
    dp = out.ctypes.data_as(ct.POINTER(ct.c_double))
    # null, misaligned, or too small for one branch / for the group size
    assert lib.juqcs_branch_amplitudes(*args, 0, dp, None, 1 << 30, None) == J.ERR_ARG
    assert lib.juqcs_branch_amplitudes(*args, 0, dp, 16, 1 << 30, None) == J.ERR_ARG
    assert lib.juqcs_branch_amplitudes(*args, 0, dp, 256, mn - 1, None) == J.ERR_SIZE
    assert lib.juqcs_branch_amplitudes(*args, 1 << 20, dp, 256, mn, None) == J.ERR_SIZE
    # no bitstrings: nothing to do, no workspace needed
    assert lib.juqcs_branch_amplitudes(n, circ.ctypes.data, circ.size, sp, zp, 0, 0, dp, None, 0,
                                       None) == J.OK


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


def test_tuning_table_round_trip(J, tmp_path):
    # an empty table saves and loads; a written table is read back entry by
    # entry; malformed files are rejected
    J.juqcs_tune_clear()
    p = tmp_path / "tune.json"
    J.juqcs_tune_save(str(p))
    J.juqcs_tune_load(str(p))
    p.write_text('{"juqcs_tune": 1, "entries": [\n'
                 ' {"key": "00000000000000ab", "n": 30, "dtype": 0, "mode": 2, "fuse_k": 5, "mma": 4, '
                 '"tile_bits": 0, "low_bits": 0, "pass_gates": 0, "relabel": 0, "ms": 500.5, '
                 '"default_ms": 600.25, "trials": 17}]}\n')
    J.juqcs_tune_load(str(p))
    q = tmp_path / "tune2.json"
    J.juqcs_tune_save(str(q))
    text = q.read_text()
    assert '"key": "00000000000000ab"' in text and '"mode": 2' in text and '"fuse_k": 5' in text
    assert '"ms": 500.500000' in text and '"trials": 17' in text
    bad = tmp_path / "bad.json"
    bad.write_text('{"entries": []}')
    with pytest.raises(J.JuqcsError) as e:
        J.juqcs_tune_load(str(bad))
    assert e.value.status == J.ERR_ARG
    bad.write_text('{"juqcs_tune": 1, "entries": [{"key": "1", "n": 3}]}')
    with pytest.raises(J.JuqcsError):
        J.juqcs_tune_load(str(bad))
    with pytest.raises(J.JuqcsError):
        J.juqcs_tune_load(str(tmp_path / "missing.json"))
    J.juqcs_tune_clear()


def test_noalloc_rejects_beyond_the_scratch_before_any_device_call(J):
    # two 24-qubit halves: one part state alone is 128 MiB, beyond the static
    # 32 MiB scratch; the pointers are never used
    import numpy as np
    from paper_1912_03243_amd import workloads as W
    lib = J._lib
    circ, side = W.grid_circuit(6, 8, 2, 5, max_cross=2)
    rc = lib.juqcs_branch_amplitudes_noalloc(48, circ.ctypes.data, circ.size,
                                             side.ctypes.data_as(ct.POINTER(ct.c_uint8)), 256, 1, 4, 0,
                                             256, None)
    assert rc == J.ERR_SIZE
    assert "scratch" in J.juqcs_last_error()
    # no bitstrings: nothing to do
    assert lib.juqcs_branch_amplitudes_noalloc(48, circ.ctypes.data, circ.size,
                                               side.ctypes.data_as(ct.POINTER(ct.c_uint8)), 256, 1, 0, 0,
                                               256, None) == J.OK


def test_library_sources_never_allocate_device_memory():
    # every device buffer is the caller's: no allocation or release calls in
    # the library's sources (host vectors and the static scratch array aside)
    import glob
    calls = re.compile(r"\bhip(Malloc|MallocAsync|MallocManaged|ExtMallocWithFlags|Free|FreeAsync|HostMalloc)\s*\(")
    for path in glob.glob(os.path.join(ROOT, "paper_1912_03243_amd", "csrc", "*")):
        text = open(path).read()
        assert not calls.search(text), f"{os.path.basename(path)} allocates device memory"


def test_committed_tuning_record_loads(J):
    # the record bench.py reads: every entry well formed, choices that the
    # planner accepts (a tile or fused mode), times not worse than defaults
    import json
    path = os.path.join(ROOT, "paper_1912_03243_amd", "tuning_mi355x.json")
    rec = json.load(open(path))
    assert rec["juqcs_tune"] == 1 and rec["entries"]
    for e in rec["entries"]:
        assert e["mode"] in (J.PLAN_PLAIN, J.PLAN_TILE, J.PLAN_FUSED)
        assert e["ms"] <= e["default_ms"] and e["trials"] > 0
    J.juqcs_tune_clear()
    J.juqcs_tune_load(path)
    J.juqcs_tune_clear()
