"""ctypes binding of libjuqcs_gpu (C-ABI declared in include/juqcs_gpu.h).

Argument marshalling only: every step of the computation runs in the
library's HIP kernels.  PyTorch provides device memory and the HIP stream.
The module-level functions carry the C names; ``State`` and ``Batch`` wrap a
handle plus the torch buffers it borrows.

Importing this module loads the library and raises ImportError if it has
not been built (``python -m paper_1912_03243_amd.build``): there is no
fallback path.
"""
from __future__ import annotations

import ctypes as ct
import os

import numpy as np

from .workloads import GATE_DTYPE

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libjuqcs_gpu.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing; build it with: python -m paper_1912_03243_amd.build")
_lib = ct.CDLL(LIB_PATH)

# ---- enums (include/juqcs_gpu.h) -------------------------------------------
OK, ERR_ARG, ERR_QUBIT, ERR_DTYPE, ERR_SIZE, ERR_HIP, ERR_UNSUPPORTED, ERR_NUMERIC = (
    0, -1, -2, -3, -4, -5, -6, -7)
C128, C64, ENC2 = 0, 1, 2
DTYPES = {"c128": C128, "c64": C64, "enc2": ENC2}
MMA_FP64, MMA_FP32, MMA_BF16, MMA_BF16X3, MMA_AUTO = 0, 1, 2, 3, 4
MMAS = {"fp64": MMA_FP64, "fp32": MMA_FP32, "bf16": MMA_BF16, "bf16x3": MMA_BF16X3,
        "auto": MMA_AUTO}
PLAN_PLAIN, PLAN_TILE, PLAN_FUSED, PLAN_AUTO = 0, 1, 2, 3
PLANS = {"plain": PLAN_PLAIN, "tile": PLAN_TILE, "fused": PLAN_FUSED, "auto": PLAN_AUTO}


class PlanOpts(ct.Structure):
    _fields_ = [("mode", ct.c_int32), ("fuse_k", ct.c_int32), ("mma", ct.c_int32),
                ("tile_bits", ct.c_int32), ("low_bits", ct.c_int32), ("profile", ct.c_int32),
                ("autotune", ct.c_int32), ("pass_gates", ct.c_int32), ("relabel", ct.c_int32),
                ("passes", ct.c_int64),
                ("gates", ct.c_int64),
                ("kernel_ms", ct.c_double), ("bytes", ct.c_double), ("flops", ct.c_double),
                ("mma_flops", ct.c_double)]


class TuneResult(ct.Structure):
    _fields_ = [("opts", PlanOpts), ("ms", ct.c_double), ("default_ms", ct.c_double),
                ("trials", ct.c_int32), ("pad", ct.c_int32), ("key", ct.c_uint64)]


class BranchStats(ct.Structure):
    _fields_ = [("crossings", ct.c_int32), ("group_bits", ct.c_int32), ("groups", ct.c_int64),
                ("tree_states", ct.c_int64), ("tile_passes", ct.c_int64), ("pass_bytes", ct.c_double),
                ("gate_flops", ct.c_double), ("sum_flops", ct.c_double), ("lds_sum", ct.c_int32),
                ("pad", ct.c_int32)]


class JuqcsError(RuntimeError):
    def __init__(self, status: int, where: str):
        msg = _lib.juqcs_last_error().decode()
        super().__init__(f"{where}: status {status}: {msg}")
        self.status = status


_P = ct.c_void_p
_I = ct.c_int
_S = ct.c_size_t
_U64 = ct.c_uint64
_DP = ct.POINTER(ct.c_double)

_SIGS = {
    "juqcs_state_bytes": [_I, _I, _I, ct.POINTER(_S), ct.POINTER(_S), ct.POINTER(_S)],
    "juqcs_state_create": [ct.POINTER(_P), _I, _I, _I, _P, _S, _P, _S, _P, _S, _P],
    "juqcs_state_destroy": [_P],
    "juqcs_state_init": [_P, _U64],
    "juqcs_state_set_stream": [_P, _P],
    "juqcs_apply_1q": [_P, _I, _DP],
    "juqcs_apply_controlled": [_P, _I, _I, _DP],
    "juqcs_apply_2q": [_P, _I, _I, _DP],
    "juqcs_apply_fused_k": [_P, _I, ct.POINTER(_I), _DP, _I],
    "juqcs_run_circuit": [_P, _P, _S, ct.POINTER(PlanOpts)],
    "juqcs_autotune": [_P, _P, _S, ct.POINTER(TuneResult)],
    "juqcs_tune_save": [ct.c_char_p],
    "juqcs_tune_load": [ct.c_char_p],
    "juqcs_tune_clear": [],
    "juqcs_tune_lookup": [_P, _P, _S, ct.POINTER(TuneResult)],
    "juqcs_amplitudes": [_P, ct.POINTER(_U64), _S, _DP],
    "juqcs_amplitudes_device": [_P, _P, _S, _P],
    "juqcs_norm": [_P, _DP],
    "juqcs_scale": [_P, ct.c_double],
    "juqcs_expectations": [_P, _DP],
    "juqcs_permute": [_P, ct.POINTER(_I)],
    "juqcs_state_canonicalize": [_P],
    "juqcs_get_layout": [_P, ct.POINTER(_I)],
    "juqcs_encode2": [_P, _I, _U64, _I, _P, _P, _P],
    "juqcs_decode2": [_P, _P, _U64, _I, _P, _I, _P],
    "juqcs_set_global_factor": [_P, _DP],
    "juqcs_mul_global_factor": [_P, _DP],
    "juqcs_get_global_factor": [_P, _DP],
    "juqcs_renormalize": [_P, _DP],
    "juqcs_batch_create": [ct.POINTER(_P), _I, ct.POINTER(_I), _P, ct.POINTER(ct.c_int64), _P, _S,
                           ct.POINTER(_U64), ct.POINTER(PlanOpts)],
    "juqcs_batch_bytes": [_P, ct.POINTER(_S)],
    "juqcs_batch_bind": [_P, _P, _S, _P],
    "juqcs_batch_autotune": [_P, _P],
    "juqcs_batch_run": [_P, _P],
    "juqcs_batch_wait": [_P],
    "juqcs_batch_fusion": [_P, ct.POINTER(_I)],
    "juqcs_batch_layout": [_P, _I, ct.POINTER(_I)],
    "juqcs_batch_amplitudes": [_P, ct.POINTER(_U64), _I, _DP, _P],
    "juqcs_batch_amplitudes_device": [_P, _P, _I, _P, _P],
    "juqcs_batch_norms": [_P, _DP, _P],
    "juqcs_batch_norms_device": [_P, _P, _P],
    "juqcs_batch_stats": [_P, ct.POINTER(ct.c_int64), ct.POINTER(ct.c_int64),
                          ct.POINTER(ct.c_int64)],
    "juqcs_batch_destroy": [_P],
    "juqcs_branch_amplitudes": [_I, _P, _S, ct.POINTER(ct.c_uint8), ct.POINTER(_U64), _S, _I,
                                _DP, _P, _S, _P],
    "juqcs_branch_amplitudes_wide": [_I, _P, _S, ct.POINTER(ct.c_uint8), ct.POINTER(_U64), _I, _S,
                                     _I, _DP, _P, _S, _P],
    "juqcs_branch_amplitudes_device": [_I, _P, _S, ct.POINTER(ct.c_uint8), _P, _I, _S, _I, _P,
                                       _P, _S, _P],
    "juqcs_branch_amplitudes_noalloc": [_I, _P, _S, ct.POINTER(ct.c_uint8), _P, _I, _S, _I, _P, _P],
    "juqcs_branch_last_stats": [ct.POINTER(BranchStats)],
    "juqcs_branch_bytes": [_I, _P, _S, ct.POINTER(ct.c_uint8), _I, _S, _I, _I, ct.POINTER(_S),
                           ct.POINTER(_S)],
    "juqcs_copy": [_P, _P, _S, _P],
}
EXPORTED = sorted(list(_SIGS) + ["juqcs_last_error", "juqcs_version"])

for _name, _args in _SIGS.items():
    _f = getattr(_lib, _name)
    _f.argtypes = _args
    _f.restype = ct.c_int
_lib.juqcs_last_error.restype = ct.c_char_p
_lib.juqcs_last_error.argtypes = []
_lib.juqcs_version.restype = ct.c_char_p
_lib.juqcs_version.argtypes = []


def _check(rc: int, where: str) -> None:
    if rc != OK:
        raise JuqcsError(rc, where)


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(_DP)


def _cplx_to_f64(m) -> np.ndarray:
    m = np.ascontiguousarray(np.asarray(m, dtype=np.complex128))
    return np.ascontiguousarray(np.stack([m.real, m.imag], axis=-1).reshape(-1))


def _stream_handle(stream) -> int:
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return int(stream.cuda_stream) if hasattr(stream, "cuda_stream") else int(stream)


def _gates(gates) -> np.ndarray:
    g = np.ascontiguousarray(gates)
    if g.dtype != GATE_DTYPE:
        raise TypeError("gate records must use workloads.GATE_DTYPE")
    return g


# ---- thin wrappers with the C names ------------------------------------------
def juqcs_version() -> str:
    return _lib.juqcs_version().decode()


def juqcs_last_error() -> str:
    return _lib.juqcs_last_error().decode()


def juqcs_state_bytes(n: int, dtype: int, block_bits: int = 0):
    a, s, w = _S(), _S(), _S()
    _check(_lib.juqcs_state_bytes(n, dtype, block_bits, ct.byref(a), ct.byref(s), ct.byref(w)),
           "juqcs_state_bytes")
    return a.value, s.value, w.value


def juqcs_tune_save(path: str):
    _check(_lib.juqcs_tune_save(os.fsencode(path)), "juqcs_tune_save")


def juqcs_tune_load(path: str):
    _check(_lib.juqcs_tune_load(os.fsencode(path)), "juqcs_tune_load")


def juqcs_tune_clear():
    _check(_lib.juqcs_tune_clear(), "juqcs_tune_clear")


MODE_NAMES = {v: k for k, v in PLANS.items()}


def juqcs_encode2(src, src_dtype: int, count: int, block_bits: int, codes, scales, stream=None):
    _check(_lib.juqcs_encode2(src.data_ptr(), src_dtype, count, block_bits, codes.data_ptr(),
                              scales.data_ptr(), _stream_handle(stream)), "juqcs_encode2")


def juqcs_decode2(codes, scales, count: int, block_bits: int, dst, dst_dtype: int, stream=None):
    _check(_lib.juqcs_decode2(codes.data_ptr(), scales.data_ptr(), count, block_bits,
                              dst.data_ptr(), dst_dtype, _stream_handle(stream)), "juqcs_decode2")


def juqcs_copy(dst, src, nbytes: int, stream=None):
    _check(_lib.juqcs_copy(dst.data_ptr(), src.data_ptr(), nbytes, _stream_handle(stream)),
           "juqcs_copy")


def juqcs_branch_bytes(n: int, gates, side, words: int, count: int, group_size: int = 0,
                       host_io: bool = True):
    """(min_bytes, bytes): workspace of the decomposition for groups of one
    branch, and for group_size (0: all branches in one group)."""
    g = _gates(gates)
    side = np.ascontiguousarray(side, dtype=np.uint8)
    mn, full = _S(), _S()
    _check(_lib.juqcs_branch_bytes(n, g.ctypes.data, g.size, side.ctypes.data_as(ct.POINTER(ct.c_uint8)),
                                   words, count, group_size, int(host_io), ct.byref(mn), ct.byref(full)),
           "juqcs_branch_bytes")
    return mn.value, full.value


# Workspace of a decomposition with group_size 0: all branches in one group
# when that fits half the free device memory (at most about 64 GiB), else as much
# as that budget holds (the library then takes the largest group that fits).
_BRANCH_BUDGET = 66 << 30  # 64 GiB of part states plus the other arrays


def branch_workspace(n, gates, side, words, count, group_size=0, host_io=True, device="cuda"):
    """A torch device buffer for the decomposition calls (juqcs_branch_bytes'
    size for group_size; for group_size 0 the budget above)."""
    import torch
    g = _gates(gates)
    if count == 0:
        return None
    mn, full = juqcs_branch_bytes(n, g, side, words, count, group_size, host_io)
    need = full
    if group_size <= 0:
        free, _ = torch.cuda.mem_get_info(torch.device(device))
        need = max(mn, min(full, free // 2, _BRANCH_BUDGET))
    return torch.empty(need, dtype=torch.uint8, device=device)


def juqcs_branch_amplitudes(n: int, gates, side, z, group_size: int = 0, stream=None,
                            device="cuda", work=None) -> np.ndarray:
    """<z|C|0> by the Eq. (3) decomposition.  z: a 1-D uint64 array of
    bitstrings (n <= 62), or a (count, words) array of little-endian uint64
    words (n <= 240, juqcs_branch_amplitudes_wide).  The device workspace
    is a torch buffer sized by juqcs_branch_bytes."""
    g = _gates(gates)
    side = np.ascontiguousarray(side, dtype=np.uint8)
    z = np.ascontiguousarray(z, dtype=np.uint64)
    count = z.shape[0] if z.ndim == 2 else z.size
    words = z.shape[1] if z.ndim == 2 else 1
    out = np.empty(2 * count, dtype=np.float64)
    sp = side.ctypes.data_as(ct.POINTER(ct.c_uint8))
    zp = z.ctypes.data_as(ct.POINTER(_U64))
    if work is None:
        work = branch_workspace(n, g, side, words, count, group_size, True, device)
    wp = work.data_ptr() if work is not None else None
    wb = work.numel() if work is not None else 0
    if z.ndim == 2:
        _check(_lib.juqcs_branch_amplitudes_wide(n, g.ctypes.data, g.size, sp, zp, words, count,
                                                 group_size, _dptr(out), wp, wb,
                                                 _stream_handle(stream)),
               "juqcs_branch_amplitudes_wide")
    else:
        _check(_lib.juqcs_branch_amplitudes(n, g.ctypes.data, g.size, sp, zp, count, group_size,
                                            _dptr(out), wp, wb, _stream_handle(stream)),
               "juqcs_branch_amplitudes")
    return out.view(np.complex128)  # (re, im) pairs


def juqcs_branch_amplitudes_device(n: int, gates, side, z, out, group_size: int = 0, stream=None,
                                   work=None):
    """juqcs_branch_amplitudes with device tensors: z an int64 (count, words)
    tensor of little-endian 64-bit words, out a float64 tensor of 2*count
    (re, im) pairs, both on the GPU (torch owns the memory).  work: an
    optional uint8 device tensor to use as the workspace (else one is
    allocated for the call)."""
    g = _gates(gates)
    side = np.ascontiguousarray(side, dtype=np.uint8)
    if z.dim() != 2 or not z.is_contiguous() or z.dtype.itemsize != 8:
        raise ValueError("z: contiguous (count, words) tensor of 64-bit words")
    if out.numel() != 2 * z.shape[0] or not out.is_contiguous() or out.element_size() != 8:
        raise ValueError("out: contiguous float64 tensor of 2*count elements")
    if work is None:
        work = branch_workspace(n, g, side, z.shape[1], z.shape[0], group_size, False, z.device)
    _check(_lib.juqcs_branch_amplitudes_device(n, g.ctypes.data, g.size,
                                               side.ctypes.data_as(ct.POINTER(ct.c_uint8)),
                                               z.data_ptr(), z.shape[1], z.shape[0], group_size,
                                               out.data_ptr(),
                                               work.data_ptr() if work is not None else None,
                                               work.numel() if work is not None else 0,
                                               _stream_handle(stream)),
           "juqcs_branch_amplitudes_device")
    return out


def juqcs_branch_last_stats() -> dict:
    """Statistics of this thread's last completed decomposition call."""
    st = BranchStats()
    _check(_lib.juqcs_branch_last_stats(ct.byref(st)), "juqcs_branch_last_stats")
    return {name: getattr(st, name) for name, _ in BranchStats._fields_ if name != "pad"}


NOALLOC_SCRATCH_BYTES = 32 << 20  # JUQCS_NOALLOC_SCRATCH_BYTES


def juqcs_branch_amplitudes_noalloc(n: int, gates, side, z, out, group_size: int = 0, stream=None):
    """juqcs_branch_amplitudes_device with the library's static scratch as
    the workspace (no device allocation by anyone during the call): z an
    int64 (count, words) device tensor, out a float64 device tensor of
    2*count elements."""
    g = _gates(gates)
    side = np.ascontiguousarray(side, dtype=np.uint8)
    if z.dim() != 2 or not z.is_contiguous() or z.dtype.itemsize != 8:
        raise ValueError("z: contiguous (count, words) tensor of 64-bit words")
    if out.numel() != 2 * z.shape[0] or not out.is_contiguous() or out.element_size() != 8:
        raise ValueError("out: contiguous float64 tensor of 2*count elements")
    _check(_lib.juqcs_branch_amplitudes_noalloc(n, g.ctypes.data, g.size,
                                                side.ctypes.data_as(ct.POINTER(ct.c_uint8)),
                                                z.data_ptr(), z.shape[1], z.shape[0], group_size,
                                                out.data_ptr(), _stream_handle(stream)),
           "juqcs_branch_amplitudes_noalloc")
    return out


# ---- State --------------------------------------------------------------------
class State:
    """A state vector in torch-owned device memory plus its library handle."""

    def __init__(self, n: int, dtype: str = "c128", block_bits: int = 0, device="cuda",
                 stream=None, amps=None):
        import torch
        self.n = n
        self.dtype_name = dtype
        self.dtype = DTYPES[dtype]
        self.block_bits = (block_bits or 8) if self.dtype == ENC2 else 0
        ab, sb, wb = juqcs_state_bytes(n, self.dtype, block_bits)
        self.amps = amps if amps is not None else torch.empty(ab, dtype=torch.uint8, device=device)
        self.scales = torch.empty(max(sb, 16), dtype=torch.uint8, device=device) if sb else None
        self.work = torch.empty(wb, dtype=torch.uint8, device=device)
        self.stream = stream
        h = _P()
        _check(_lib.juqcs_state_create(
            ct.byref(h), n, self.dtype, block_bits, self.amps.data_ptr(),
            self.amps.numel() * self.amps.element_size(),
            self.scales.data_ptr() if self.scales is not None else None, sb,
            self.work.data_ptr(), wb, _stream_handle(stream)), "juqcs_state_create")
        self.h = h

    # lifetime
    def close(self):
        if getattr(self, "h", None):
            _lib.juqcs_state_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # gates
    def init(self, basis_index: int = 0):
        _check(_lib.juqcs_state_init(self.h, basis_index), "juqcs_state_init")
        return self

    def apply_1q(self, t: int, u):
        _check(_lib.juqcs_apply_1q(self.h, t, _dptr(_cplx_to_f64(u))), "juqcs_apply_1q")

    def apply_controlled(self, c: int, t: int, u):
        _check(_lib.juqcs_apply_controlled(self.h, c, t, _dptr(_cplx_to_f64(u))),
               "juqcs_apply_controlled")

    def apply_2q(self, q0: int, q1: int, m):
        _check(_lib.juqcs_apply_2q(self.h, q0, q1, _dptr(_cplx_to_f64(m))), "juqcs_apply_2q")

    def apply_fused(self, targets, m, mode: str = "auto"):
        t = np.ascontiguousarray(targets, dtype=np.int32)
        arr = (ct.c_int * t.size)(*t.tolist())
        _check(_lib.juqcs_apply_fused_k(self.h, t.size, arr, _dptr(_cplx_to_f64(m)), MMAS[mode]),
               "juqcs_apply_fused_k")

    def run(self, gates, mode: str = "auto", fuse_k: int = 0, mma: str = "auto",
            tile_bits: int = 0, low_bits: int = 0, profile: bool = False,
            pass_gates: int = 0, relabel: int = 0) -> PlanOpts:
        g = _gates(gates)
        o = PlanOpts(mode=PLANS[mode], fuse_k=fuse_k, mma=MMAS[mma], tile_bits=tile_bits,
                     low_bits=low_bits, profile=int(profile), pass_gates=pass_gates,
                     relabel=relabel)
        _check(_lib.juqcs_run_circuit(self.h, g.ctypes.data, g.size, ct.byref(o)),
               "juqcs_run_circuit")
        return o

    def autotune(self, gates) -> dict:
        """Timed trials of planner options for this circuit (juqcs_autotune);
        later run(mode="auto") calls on circuits of the same structure use
        the winner."""
        g = _gates(gates)
        r = TuneResult()
        _check(_lib.juqcs_autotune(self.h, g.ctypes.data, g.size, ct.byref(r)), "juqcs_autotune")
        return self._tune_dict(r)

    def tuned(self, gates):
        """The tuning table's entry for this circuit's structure, or None."""
        g = _gates(gates)
        r = TuneResult()
        if _lib.juqcs_tune_lookup(self.h, g.ctypes.data, g.size, ct.byref(r)) != OK:
            return None
        return self._tune_dict(r)

    @staticmethod
    def _tune_dict(r):
        o = r.opts
        return {"mode": MODE_NAMES[o.mode], "fuse_k": o.fuse_k, "mma": o.mma, "tile_bits": o.tile_bits,
                "low_bits": o.low_bits, "pass_gates": o.pass_gates, "relabel": o.relabel,
                "ms": r.ms, "default_ms": r.default_ms, "trials": r.trials, "key": f"{r.key:016x}"}

    # read-out
    def amplitudes(self, idx) -> np.ndarray:
        z = np.ascontiguousarray(idx, dtype=np.uint64)
        out = np.empty(2 * z.size, dtype=np.float64)
        _check(_lib.juqcs_amplitudes(self.h, z.ctypes.data_as(ct.POINTER(_U64)), z.size,
                                     _dptr(out)), "juqcs_amplitudes")
        return out[0::2] + 1j * out[1::2]

    def amplitudes_device(self, d_idx, d_out):
        _check(_lib.juqcs_amplitudes_device(self.h, d_idx.data_ptr(), d_idx.numel(),
                                            d_out.data_ptr()), "juqcs_amplitudes_device")

    def norm(self) -> float:
        out = np.zeros(1)
        _check(_lib.juqcs_norm(self.h, _dptr(out)), "juqcs_norm")
        return float(out[0])

    def scale(self, f: float):
        _check(_lib.juqcs_scale(self.h, f), "juqcs_scale")

    def expectations(self) -> np.ndarray:
        out = np.zeros(3 * self.n)
        _check(_lib.juqcs_expectations(self.h, _dptr(out)), "juqcs_expectations")
        return out.reshape(self.n, 3)

    def permute(self, new_phys):
        p = (ct.c_int * self.n)(*[int(x) for x in new_phys])
        _check(_lib.juqcs_permute(self.h, p), "juqcs_permute")

    def canonicalize(self):
        _check(_lib.juqcs_state_canonicalize(self.h), "juqcs_state_canonicalize")

    def layout(self):
        p = (ct.c_int * self.n)()
        _check(_lib.juqcs_get_layout(self.h, p), "juqcs_get_layout")
        return list(p)

    def global_factor(self) -> complex:
        g = np.zeros(2)
        _check(_lib.juqcs_get_global_factor(self.h, _dptr(g)), "juqcs_get_global_factor")
        return complex(g[0], g[1])

    def set_global_factor(self, g: complex):
        a = np.array([complex(g).real, complex(g).imag])
        _check(_lib.juqcs_set_global_factor(self.h, _dptr(a)), "juqcs_set_global_factor")

    def mul_global_factor(self, f: complex):
        a = np.array([complex(f).real, complex(f).imag])
        _check(_lib.juqcs_mul_global_factor(self.h, _dptr(a)), "juqcs_mul_global_factor")

    def renormalize(self) -> float:
        out = np.zeros(1)
        _check(_lib.juqcs_renormalize(self.h, _dptr(out)), "juqcs_renormalize")
        return float(out[0])

    def state_vector(self) -> np.ndarray:
        """Whole state in logical order as complex128 (host copy), read by
        the library: juqcs_amplitudes_device over every basis index (the
        library maps each through the qubit layout, decodes two-byte
        amplitudes and applies the global factor), in chunks of 2^22."""
        import torch
        count = 1 << self.n
        chunk = min(count, 1 << 22)
        dev = self.amps.device
        idx = torch.empty(chunk, dtype=torch.int64, device=dev)
        out = torch.empty(2 * chunk, dtype=torch.float64, device=dev)
        res = np.empty(count, dtype=np.complex128)
        for a in range(0, count, chunk):
            torch.arange(a, a + chunk, dtype=torch.int64, device=dev, out=idx)
            if self.stream is not None:
                torch.cuda.current_stream(dev).synchronize()
            _check(_lib.juqcs_amplitudes_device(self.h, idx.data_ptr(), chunk, out.data_ptr()),
                   "juqcs_amplitudes_device")
            self._sync()
            res[a:a + chunk] = out.cpu().numpy().view(np.complex128)
        return res

    def _sync(self):
        import torch
        if self.stream is None:
            torch.cuda.current_stream(self.amps.device).synchronize()
        elif hasattr(self.stream, "synchronize"):
            self.stream.synchronize()
        else:
            torch.cuda.synchronize(self.amps.device)

    def raw_vector(self) -> np.ndarray:
        """The stored C128/C64 amplitudes in physical order, without the
        global factor (host copy)."""
        import torch
        self._sync()
        if self.dtype == C128:
            t = self.amps[: (1 << self.n) * 16].view(torch.float64)
        elif self.dtype == C64:
            t = self.amps[: (1 << self.n) * 8].view(torch.float32)
        else:
            raise ValueError("raw_vector: C128 or C64 states only (raw_codes for ENC2)")
        a = t.cpu().numpy().astype(np.float64)
        return a[0::2] + 1j * a[1::2]

    def raw_codes(self):
        """(codes int8 (2^n, 2), scales float32) of an ENC2 state (host copies)."""
        import torch
        torch.cuda.synchronize()
        codes = self.amps[: 2 << self.n].cpu().numpy().view(np.int8).reshape(-1, 2)
        nb = (1 << self.n) >> self.block_bits
        scales = self.scales[: 4 * nb].cpu().numpy().view(np.float32)
        return codes, scales


# ---- Batch --------------------------------------------------------------------
class Batch:
    """Many independent C64 circuits executed by one graph launch (one kernel
    per pass round).  torch owns the state buffer and the workspace; the
    library plans on the host (juqcs_batch_create), reports the workspace
    size (juqcs_batch_bytes) and uploads its work list there
    (juqcs_batch_bind)."""

    def __init__(self, circuits, device="cuda", states=None, fuse_k: int = 0,
                 autotune: bool = False, relabel: int = 0, stream=None):
        import torch
        ns = np.array([n for n, _ in circuits], dtype=np.int32)
        offs = np.zeros(len(circuits) + 1, dtype=np.int64)
        for i, (_, g) in enumerate(circuits):
            offs[i + 1] = offs[i] + len(g)
        allg = np.ascontiguousarray(np.concatenate([g for _, g in circuits])) if len(circuits) \
            else np.zeros(0, dtype=GATE_DTYPE)
        sizes = (8 << ns.astype(np.int64))
        soff = np.zeros(len(circuits), dtype=np.uint64)
        run = 0
        for i, s in enumerate(sizes):
            soff[i] = run
            run += int((s + 255) // 256 * 256)
        self.n = ns
        self.state_offset = soff
        self.device = device
        self.states = states if states is not None else torch.empty(max(run, 256), dtype=torch.uint8,
                                                                     device=device)
        o = PlanOpts(mode=PLAN_TILE, fuse_k=fuse_k, autotune=int(autotune), relabel=relabel)
        h = _P()
        _check(_lib.juqcs_batch_create(ct.byref(h), len(circuits),
                                       ns.ctypes.data_as(ct.POINTER(_I)), allg.ctypes.data,
                                       offs.ctypes.data_as(ct.POINTER(ct.c_int64)),
                                       self.states.data_ptr(),
                                       self.states.numel() * self.states.element_size(),
                                       soff.ctypes.data_as(ct.POINTER(_U64)), ct.byref(o)),
               "juqcs_batch_create")
        self.h = h
        self.work = None
        self._bind(stream)
        if autotune:
            _check(_lib.juqcs_batch_autotune(self.h, _stream_handle(stream)), "juqcs_batch_autotune")
            self._bind(stream)

    def bytes(self) -> int:
        b = _S()
        _check(_lib.juqcs_batch_bytes(self.h, ct.byref(b)), "juqcs_batch_bytes")
        return b.value

    def _bind(self, stream=None):
        import torch
        need = self.bytes()
        if self.work is None or self.work.numel() < need:
            self.work = None
            self.work = torch.empty(need, dtype=torch.uint8, device=self.device)
        _check(_lib.juqcs_batch_bind(self.h, self.work.data_ptr(), self.work.numel(),
                                     _stream_handle(stream)), "juqcs_batch_bind")

    def run(self, stream=None):
        _check(_lib.juqcs_batch_run(self.h, _stream_handle(stream)), "juqcs_batch_run")

    def wait(self):
        _check(_lib.juqcs_batch_wait(self.h), "juqcs_batch_wait")

    def fusion(self) -> np.ndarray:
        k = (ct.c_int * len(self.n))()
        _check(_lib.juqcs_batch_fusion(self.h, k), "juqcs_batch_fusion")
        return np.array(list(k))

    def amplitudes(self, idx, stream=None) -> np.ndarray:
        """idx: (count, m) uint64 -> (count, m) complex128."""
        z = np.ascontiguousarray(idx, dtype=np.uint64)
        m = z.shape[1]
        out = np.empty(2 * z.size, dtype=np.float64)
        _check(_lib.juqcs_batch_amplitudes(self.h, z.ctypes.data_as(ct.POINTER(_U64)), m,
                                           _dptr(out), _stream_handle(stream)),
               "juqcs_batch_amplitudes")
        return (out[0::2] + 1j * out[1::2]).reshape(z.shape)

    def amplitudes_device(self, d_idx, m: int, d_out, stream=None):
        """d_idx: (count*m) int64 device tensor; d_out: 2*count*m float64."""
        if d_idx.numel() != len(self.n) * m or d_out.numel() != 2 * len(self.n) * m:
            raise ValueError("d_idx: count*m indices, d_out: 2*count*m doubles")
        _check(_lib.juqcs_batch_amplitudes_device(self.h, d_idx.data_ptr(), m, d_out.data_ptr(),
                                                  _stream_handle(stream)),
               "juqcs_batch_amplitudes_device")

    def norms(self, stream=None) -> np.ndarray:
        out = np.empty(len(self.n), dtype=np.float64)
        _check(_lib.juqcs_batch_norms(self.h, _dptr(out), _stream_handle(stream)),
               "juqcs_batch_norms")
        return out

    def norms_device(self, d_out, stream=None):
        if d_out.numel() != len(self.n):
            raise ValueError("d_out: one double per circuit")
        _check(_lib.juqcs_batch_norms_device(self.h, d_out.data_ptr(), _stream_handle(stream)),
               "juqcs_batch_norms_device")

    def stats(self):
        a, b, c = ct.c_int64(), ct.c_int64(), ct.c_int64()
        _check(_lib.juqcs_batch_stats(self.h, ct.byref(a), ct.byref(b), ct.byref(c)),
               "juqcs_batch_stats")
        return {"tasks": a.value, "gate_apps": b.value, "passes": c.value}

    def layout(self, i: int):
        p = (ct.c_int * int(self.n[i]))()
        _check(_lib.juqcs_batch_layout(self.h, i, p), "juqcs_batch_layout")
        return list(p)

    def state_vector(self, i: int, stream=None) -> np.ndarray:
        """State of circuit i in logical order, read by the library
        (juqcs_batch_amplitudes_device over every basis index of circuit i;
        the other circuits read index 0)."""
        import torch
        n = int(self.n[i])
        count = len(self.n)
        m = 1 << n
        if count * m > (1 << 28):
            raise ValueError("state_vector reads every circuit's m indices: use amplitudes() on large batches")
        idx = torch.zeros((count, m), dtype=torch.int64, device=self.device)
        idx[i] = torch.arange(m, dtype=torch.int64, device=self.device)
        out = torch.empty(2 * count * m, dtype=torch.float64, device=self.device)
        self.amplitudes_device(idx, m, out, stream)
        torch.cuda.synchronize()
        o = out.view(count, 2 * m)[i].cpu().numpy()
        return o[0::2] + 1j * o[1::2]

    def close(self):
        if getattr(self, "h", None):
            _lib.juqcs_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
