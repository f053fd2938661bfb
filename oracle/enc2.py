"""Reference two-byte amplitude codec.  Test infrastructure only.

The paper stores each amplitude in two bytes with an adaptive coding
(Section 1: 8x less memory than FP64 complex, about three digits) but does
not give the format.  This project defines one, and this module is its
bit-exact definition:

* amplitudes are grouped in blocks of 2^B consecutive indices (the last block
  may be shorter);
* per block, s = max over the block of max(|Re|, |Im|) after rounding every
  component to FP32 (round to nearest even);
* if s < 2^-100 the block is stored as scale 0 and all-zero codes;
* otherwise r = fl32(127 / s) and each component is coded as
  q = clamp(rint(fl32(x * r)), -127, 127) (int8, ties to even);
  one amplitude = (q_re, q_im) = 2 bytes;
* decoding: d = fl32(s / 127), x = fl32(q * d).

All arithmetic below is FP32 with one rounding per operation.
"""
import numpy as np

TINY = np.float32(2.0 ** -100)
F127 = np.float32(127.0)


def _components(amps: np.ndarray) -> np.ndarray:
    a = np.asarray(amps)
    comp = np.stack([a.real, a.imag], axis=-1).astype(np.float32)
    return comp  # (count, 2) float32


def encode(amps: np.ndarray, block_bits: int):
    """Returns (codes int8 (count, 2), scales float32 (nblocks,))."""
    x = _components(amps)
    count = x.shape[0]
    bs = 1 << block_bits
    nblocks = (count + bs - 1) // bs
    codes = np.zeros((count, 2), dtype=np.int8)
    scales = np.zeros(nblocks, dtype=np.float32)
    for b in range(nblocks):
        blk = x[b * bs:(b + 1) * bs]
        s = np.float32(np.max(np.abs(blk))) if blk.size else np.float32(0)
        if not (s >= TINY):
            continue
        r = np.float32(F127 / s)
        prod = blk * r                       # float32 x float32 -> float32
        assert prod.dtype == np.float32
        q = np.clip(np.rint(prod), -127, 127)
        codes[b * bs:(b + 1) * bs] = q.astype(np.int8)
        scales[b] = s
    return codes, scales


def decode(codes: np.ndarray, scales: np.ndarray, block_bits: int) -> np.ndarray:
    """Returns complex64 amplitudes."""
    count = codes.shape[0]
    bs = 1 << block_bits
    out = np.zeros((count, 2), dtype=np.float32)
    for b in range(scales.size):
        d = np.float32(scales[b] / F127)
        out[b * bs:(b + 1) * bs] = codes[b * bs:(b + 1) * bs].astype(np.float32) * d
    return (out[:, 0] + 1j * out[:, 1]).astype(np.complex64)
