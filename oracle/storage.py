"""Rounding of values to a narrow storage format (TEST INFRASTRUCTURE ONLY).

The paper computes in FP64 throughout (Numerical experiments section); storing
the fields and the geometric factors in FP32, BF16 or FP16 is this project's
addition.  A narrow-storage apply computes the operator of the *rounded*
inputs, so the oracle's reference for it is its own FP64 operator applied to
inputs rounded here.  The rounding is defined in two steps, FP64 -> FP32
(round to nearest even) and then FP32 -> the 16-bit format (round to nearest
even), each written out below from the formats' definitions:

* FP32: IEEE binary32, 24-bit significand.
* BF16: the upper 16 bits of a binary32 (8-bit exponent, 8-bit significand);
  rounding adds half an ulp of the dropped 16 bits, ties to even.
* FP16: IEEE binary16 (5-bit exponent, 11-bit significand), via NumPy's
  float32 -> float16 conversion (round to nearest even).

FP16 storage multiplies by a power of two ``scale`` before rounding (the raw
geometric factors of fine meshes underflow binary16); the value the operator
sees is the rounded number divided by ``scale`` (exact, a power of two).
"""
from __future__ import annotations

import numpy as np


def to_f32(x: np.ndarray) -> np.ndarray:
    """Round FP64 values to binary32 and return them as FP64."""
    return np.asarray(x, dtype=np.float64).astype(np.float32).astype(np.float64)


def to_bf16(x: np.ndarray) -> np.ndarray:
    """Round FP64 values to bfloat16 (through binary32) and return them as FP64."""
    f = np.ascontiguousarray(np.asarray(x, dtype=np.float64).astype(np.float32))
    bits = f.view(np.uint32).astype(np.uint64)
    # round to nearest even on the 16 dropped bits (finite values only)
    bits = (bits + 0x7FFF + ((bits >> 16) & 1)) >> 16 << 16
    return bits.astype(np.uint32).view(np.float32).astype(np.float64)


def to_f16(x: np.ndarray) -> np.ndarray:
    """Round FP64 values to binary16 (through binary32) and return them as FP64."""
    return np.asarray(x, dtype=np.float64).astype(np.float32).astype(np.float16).astype(np.float64)


ROUND = {"f64": lambda x: np.asarray(x, dtype=np.float64), "f32": to_f32, "bf16": to_bf16, "f16": to_f16}


def stored(x: np.ndarray, fmt: str, scale: float = 1.0) -> np.ndarray:
    """The value an operator sees for x stored in ``fmt`` with storage scale
    ``scale`` (a power of two; FP16 storage only): round(x * scale) / scale."""
    if scale != 1.0:
        m, e = np.frexp(scale)
        assert m == 0.5, "the storage scale must be a power of two"
    return ROUND[fmt](np.asarray(x, dtype=np.float64) * scale) / scale
