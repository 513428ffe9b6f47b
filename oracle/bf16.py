"""bfloat16 rounding emulation (oracle, test infrastructure).

The anchor decoder (Sec. 3.2, Eq. 4) runs its first layer on bfloat16
operands.  The anchor feature F (float32) is rounded to bfloat16 with
round-to-nearest, ties-to-even before the product; the decoder weights are
given as bfloat16 bit patterns.
"""
import numpy as np


def round_to_bf16(x) -> np.ndarray:
    """Round float32 values to the nearest bfloat16 (ties to even); returns
    float64 holding the exact bfloat16 values.  NaN/Inf are not expected."""
    f = np.ascontiguousarray(np.asarray(x, np.float32))
    bits = f.view(np.uint32).astype(np.uint64)
    lsb = (bits >> np.uint64(16)) & np.uint64(1)
    rounded = ((bits + np.uint64(0x7FFF) + lsb) >> np.uint64(16)) << np.uint64(16)
    return rounded.astype(np.uint32).view(np.float32).astype(np.float64)


def from_bits(bits) -> np.ndarray:
    """bfloat16 bit patterns (uint16) -> float64 values."""
    b = np.asarray(bits, np.uint16).astype(np.uint32) << np.uint32(16)
    return b.view(np.float32).astype(np.float64)
