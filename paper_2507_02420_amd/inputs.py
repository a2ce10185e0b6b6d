"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle checks.

This module holds no arithmetic of the transform itself: it only draws
vectors and base matrices W from fixed seeds (numpy PCG64 via
``default_rng``), always in float64 / complex128 first, so that the GPU path
and the FP64 oracle see identical values after the cast to a storage dtype.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "gaussian", "uniform", "int_uniform", "haar_unitary", "u3", "hadamard2",
    "dft_matrix", "ragged_shapes", "RAGGED_VALID_N", "to_bf16_f64",
]


def gaussian(shape, seed: int, complex_: bool = False) -> np.ndarray:
    """x ~ N(0, 1) (real) or standard complex normal (re, im i.i.d. N(0, 1/2))."""
    rng = np.random.default_rng(seed)
    if complex_:
        re = rng.standard_normal(shape)
        im = rng.standard_normal(shape)
        return (re + 1j * im) / np.sqrt(2.0)
    return rng.standard_normal(shape)


def uniform(shape, seed: int, lo: float = -1.0, hi: float = 1.0) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return rng.uniform(lo, hi, size=shape)


def int_uniform(shape, seed: int, lo: int, hi: int) -> np.ndarray:
    """Integers uniform on [lo, hi] inclusive, as int64."""
    rng = np.random.default_rng(seed)
    return rng.integers(lo, hi + 1, size=shape, dtype=np.int64)


def haar_unitary(b: int, seed: int, complex_: bool = True) -> np.ndarray:
    """Random b x b unitary (complex) or orthogonal (real) matrix: QR of a
    Gaussian matrix with the phases of diag(R) moved into Q (Haar measure)."""
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((b, b))
    if complex_:
        A = (A + 1j * rng.standard_normal((b, b))) / np.sqrt(2.0)
    Q, R = np.linalg.qr(A)
    d = np.diagonal(R)
    ph = d / np.abs(d)
    return Q * ph[np.newaxis, :]


def u3(theta: float, phi: float, lam: float) -> np.ndarray:
    """The 2 x 2 U3(theta, phi, lambda) gate used as W in the paper's examples."""
    c, s = np.cos(theta / 2), np.sin(theta / 2)
    return np.array([[c, -np.exp(1j * lam) * s],
                     [np.exp(1j * phi) * s, np.exp(1j * (phi + lam)) * c]])


def hadamard2(normalized: bool = True) -> np.ndarray:
    H = np.array([[1.0, 1.0], [1.0, -1.0]])
    return H / np.sqrt(2.0) if normalized else H


def dft_matrix(b: int) -> np.ndarray:
    """Unitary DFT of order b: F[j, k] = exp(-2 pi i j k / b) / sqrt(b)."""
    j = np.arange(b)
    return np.exp(-2j * np.pi * np.outer(j, j) / b) / np.sqrt(b)


# n ranges per radix for the ragged batch: N = b**n spans 2^10 .. 2^20
RAGGED_VALID_N = {2: list(range(10, 21)), 4: list(range(5, 11)),
                  16: list(range(3, 6)), 32: list(range(2, 5))}


def ragged_shapes(count: int = 1024, seed: int = 52):
    """(b, n) per instance for the ragged batch: b uniform over {2, 4, 16, 32},
    then n uniform over that radix's valid range (N from 2^10 to 2^20)."""
    rng = np.random.default_rng(seed)
    radices = [2, 4, 16, 32]
    out = []
    for _ in range(count):
        b = radices[int(rng.integers(4))]
        valid = RAGGED_VALID_N[b]
        n = valid[int(rng.integers(len(valid)))]
        out.append((b, n))
    return out


def to_bf16_f64(a: np.ndarray) -> np.ndarray:
    """Round float64 values to bfloat16 (round to nearest even) and return them
    as float64, i.e. the exact values a bf16 buffer holds."""
    a32 = np.asarray(a, dtype=np.float32)
    u = a32.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    u = (u + 0x7FFF + lsb) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)
