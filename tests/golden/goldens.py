"""Helpers for the stored oracle results (test infrastructure)."""
from __future__ import annotations

import hashlib
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))


def row_digests(bits: np.ndarray, counts: np.ndarray) -> np.ndarray:
    """64-bit BLAKE2b digest of each row's packed words followed by its count."""
    bits = np.ascontiguousarray(bits, dtype=np.uint32)
    counts = np.ascontiguousarray(counts, dtype=np.uint32)
    out = np.zeros(len(counts), dtype=np.uint64)
    for i in range(len(counts)):
        h = hashlib.blake2b(bits[i].tobytes() + counts[i:i + 1].tobytes(), digest_size=8)
        out[i] = np.frombuffer(h.digest(), dtype=np.uint64)[0]
    return out


def load(name: str):
    return np.load(os.path.join(HERE, name), allow_pickle=False)
