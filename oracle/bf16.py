"""FP32 -> BF16 rounding to nearest, ties to even (test infrastructure).

BF16 keeps the FP32 sign, the 8-bit exponent and the top 7 stored mantissa
bits (8-bit significand).  Rounding to nearest even on the 16 discarded bits:
add 0x7FFF plus the lowest kept bit, then truncate; every NaN maps to the
canonical quiet NaN 0x7FC0.  Pinned by torch's
``Tensor.to(torch.bfloat16)`` (a library routine) on random and special values.
"""
import numpy as np


def round_to_bf16_bits(a):
    a = np.ascontiguousarray(a, dtype=np.float32)
    bits = a.view(np.uint32).astype(np.uint64)
    lsb = (bits >> 16) & 1
    rounded = ((bits + 0x7FFF + lsb) >> 16).astype(np.uint16)
    nan = np.isnan(a)
    if nan.any():
        rounded[nan] = np.uint16(0x7FC0)
    return rounded


def bf16_bits_to_f32(h):
    h = np.ascontiguousarray(h, dtype=np.uint16)
    return (h.astype(np.uint32) << 16).view(np.float32)


def round_to_bf16(a):
    """The FP32 values of RNE(a) in BF16."""
    return bf16_bits_to_f32(round_to_bf16_bits(a))
