"""Pure-Python literal oracle for small cases (test infrastructure only).

The definitions, written out with Python integers:
  K = P#/d  (deficient primorial, Section 2 "Primorials" and Section 3),
  rows    m in [m_start, m_start + m_inc) with gcd(m, d) = 1  (Section 3, M_c),
  columns X in [-sl, sl] with gcd(X, K) = 1                     (interval S = 2X + 1, Section 3.2),
  for each row, N = m*K and for every prime p <= limit: r = N mod p, mark N - r + i*p
  (the traditional sieve of Section 2.1), i.e. every X = -r (mod p) in the window.
Loops are plain Python; use it only where rows x primes is at most a few million.
"""
from __future__ import annotations

import math

import numpy as np


def primes_upto(n: int) -> list[int]:
    """Sieve of Eratosthenes (plain, one byte per integer)."""
    if n < 2:
        return []
    comp = bytearray(n + 1)
    out = []
    for i in range(2, n + 1):
        if not comp[i]:
            out.append(i)
            for j in range(i * i, n + 1, i):
                comp[j] = 1
    return out


def primorial(P: int) -> int:
    k = 1
    for q in primes_upto(P):
        k *= q
    return k


def K_of(P: int, d: int) -> int:
    pp = primorial(P)
    if d <= 0 or pp % d:
        raise ValueError("d must divide P#")
    for q in primes_upto(P):
        if d % (q * q) == 0:
            raise ValueError("d must be squarefree")
    return pp // d


def columns(P: int, d: int, sl: int) -> list[int]:
    K = K_of(P, d)
    return [X for X in range(-sl, sl + 1) if math.gcd(X, K) == 1]


def rows(d: int, m_start: int, m_inc: int) -> list[int]:
    return [m for m in range(m_start, m_start + m_inc) if math.gcd(m, d) == 1]


def sieve(job, p_lo: int = 2, p_hi: int | None = None, m_rows=None, witness: bool = False):
    """Unpacked result: bits[row][col] (uint8), counts[row], and the smallest marking prime.

    m_rows overrides the row list (e.g. a sample of rows)."""
    P, d, m_start, m_inc, sl, limit = job.as_tuple()
    if p_hi is None:
        p_hi = limit
    K = K_of(P, d)
    cols = columns(P, d, sl)
    col_of = {X: c for c, X in enumerate(cols)}
    ms = rows(d, m_start, m_inc) if m_rows is None else list(m_rows)
    ps = [p for p in primes_upto(p_hi) if p >= p_lo]
    bits = np.zeros((len(ms), len(cols)), dtype=np.uint8)
    counts = np.zeros(len(ms), dtype=np.uint32)
    wit = np.zeros((len(ms), len(cols)), dtype=np.uint64)
    for i, m in enumerate(ms):
        N = m * K
        for p in ps:
            r = N % p
            # smallest X >= -sl with X = -r (mod p)
            X = -sl + ((-r + sl) % p)
            while X <= sl:
                c = col_of.get(X)
                if c is not None:
                    bits[i, c] = 1
                    counts[i] += 1
                    if wit[i, c] == 0:
                        wit[i, c] = p
                X += p
    if witness:
        return bits, counts, wit
    return bits, counts


def pack(bits: np.ndarray) -> np.ndarray:
    """One uint8 per (row, column) -> uint32 words, column c at word c//32, bit c%32."""
    n, nx = bits.shape
    rw = (nx + 31) // 32
    padded = np.zeros((n, rw * 32), dtype=np.uint8)
    padded[:, :nx] = bits
    words = np.zeros((n, rw), dtype=np.uint64)
    for b in range(32):
        words |= padded[:, b::32].astype(np.uint64) << np.uint64(b)
    return words.astype(np.uint32)


def unpack(words: np.ndarray, n_x: int) -> np.ndarray:
    words = np.asarray(words, dtype=np.uint32)
    n, rw = words.shape
    out = np.zeros((n, rw * 32), dtype=np.uint8)
    for b in range(32):
        out[:, b::32] = ((words >> np.uint32(b)) & np.uint32(1)).astype(np.uint8)
    return out[:, :n_x]
