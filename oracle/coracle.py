"""ctypes wrapper of the C oracle (csieve_oracle.c).  Test infrastructure only.

Every routine computes the plain definition of the sieve (Section 2.1 traditional sieve over the
intervals of Section 3.2); see the header of csieve_oracle.c.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from . import build as _build

DIRECT = 0   # r = N mod p from the bignum N = m*K (literal traditional sieve, Section 2.1)
CACHED = 1   # r = ((m mod p)(K mod p)) mod p, the identity of Eq. 1 (Section 3.1)

_lib = None


def lib():
    global _lib
    if _lib is None:
        path = _build.LIB
        if not os.path.exists(path):
            _build.build()
        L = C.CDLL(path)
        u64, i64, u32, i32 = C.c_uint64, C.c_int64, C.c_uint32, C.c_int
        L.orc_prime_stats.argtypes = [u64, u64, C.POINTER(u64), C.POINTER(C.c_double), i32]
        L.orc_prime_stats.restype = i32
        L.orc_primes_range.argtypes = [u64, u64, C.c_void_p, u64]
        L.orc_primes_range.restype = i64
        L.orc_columns.argtypes = [u32, u64, u32, C.c_void_p, u64]
        L.orc_columns.restype = i64
        L.orc_rows.argtypes = [u64, u64, u64, C.c_void_p, u64]
        L.orc_rows.restype = i64
        L.orc_sieve_rows.argtypes = [u32, u64, u32, C.c_void_p, u64, u64, u64, i32,
                                     C.c_void_p, C.c_void_p, C.c_void_p, i32]
        L.orc_sieve_rows.restype = i32
        L.orc_window_hit_primes.argtypes = [u32, u64, u64, u32, u64, u64, i32]
        L.orc_window_hit_primes.restype = i64
        L.orc_n_mod.argtypes = [u32, u64, u64, C.c_void_p, u64, C.c_void_p]
        L.orc_n_mod.restype = i32
        _lib = L
    return _lib


def _ptr(a):
    return a.ctypes.data_as(C.c_void_p)


def prime_stats(lo: int, hi: int, threads: int = 0):
    """(pi(hi) - pi(lo - 1), sum of log(1 - 1/p)) over primes in [lo, hi] (Section 4.1 table)."""
    cnt = C.c_uint64(0)
    s = C.c_double(0.0)
    st = lib().orc_prime_stats(lo, hi, C.byref(cnt), C.byref(s), threads)
    if st:
        raise RuntimeError(f"orc_prime_stats failed: {st}")
    return int(cnt.value), float(s.value)


def primes_range(lo: int, hi: int) -> np.ndarray:
    n = lib().orc_primes_range(lo, hi, None, 0)
    if n < 0:
        raise RuntimeError(f"orc_primes_range failed: {n}")
    out = np.zeros(max(n, 1), dtype=np.uint64)
    lib().orc_primes_range(lo, hi, _ptr(out), n)
    return out[:n]


def columns(P: int, d: int, sl: int) -> np.ndarray:
    n = lib().orc_columns(P, d, sl, None, 0)
    if n < 0:
        raise ValueError(f"invalid (P, d) = ({P}, {d})")
    out = np.zeros(max(n, 1), dtype=np.int32)
    lib().orc_columns(P, d, sl, _ptr(out), n)
    return out[:n]


def rows(d: int, m_start: int, m_inc: int) -> np.ndarray:
    n = lib().orc_rows(d, m_start, m_inc, None, 0)
    out = np.zeros(max(n, 1), dtype=np.uint64)
    lib().orc_rows(d, m_start, m_inc, _ptr(out), n)
    return out[:n]


def sieve_rows(P: int, d: int, sl: int, m_rows, p_lo: int, p_hi: int, mode: int = DIRECT,
               witness: bool = False, threads: int = 0):
    """Bitmap (n_rows x row_words uint32, LSB-first columns), counts (uint32) and optionally the
    smallest marking prime per (row, column) for the listed multipliers and primes in [p_lo, p_hi]."""
    m = np.ascontiguousarray(np.asarray(m_rows, dtype=np.uint64))
    n_x = lib().orc_columns(P, d, sl, None, 0)
    if n_x < 0:
        raise ValueError(f"invalid (P, d) = ({P}, {d})")
    row_words = (n_x + 31) // 32
    n = len(m)
    bits = np.zeros((max(n, 1), max(row_words, 1)), dtype=np.uint32)
    counts = np.zeros(max(n, 1), dtype=np.uint32)
    wit = np.zeros((max(n, 1), max(n_x, 1)), dtype=np.uint64) if witness else None
    st = lib().orc_sieve_rows(P, d, sl, _ptr(m) if n else None, n, p_lo, p_hi, mode,
                              _ptr(bits), _ptr(counts), _ptr(wit) if witness else None, threads)
    if st:
        raise RuntimeError(f"orc_sieve_rows failed: {st}")
    bits = bits[:n, :row_words]
    counts = counts[:n]
    if witness:
        return bits, counts, wit[:n, :n_x]
    return bits, counts


def sieve_job(job, mode: int = CACHED, witness: bool = False, threads: int = 0, p_lo: int = 2,
              p_hi: int | None = None):
    """Every row of a job: the plain definition over all primes <= job.limit."""
    m = rows(job.d, job.m_start, job.m_inc)
    return sieve_rows(job.P, job.d, job.sl, m, p_lo, job.limit if p_hi is None else p_hi,
                      mode=mode, witness=witness, threads=threads)


def window_hit_primes(P: int, d: int, m: int, sl: int, p_lo: int, p_hi: int, threads: int = 0) -> int:
    """How many primes in [p_lo, p_hi] divide some N + X, |X| <= sl, N = m*P#/d (Section 3.2)."""
    n = lib().orc_window_hit_primes(P, d, m, sl, p_lo, p_hi, threads)
    if n < 0:
        raise RuntimeError(f"orc_window_hit_primes failed: {n}")
    return int(n)


def n_mod(P: int, d: int, m: int, ps) -> np.ndarray:
    ps = np.ascontiguousarray(np.asarray(ps, dtype=np.uint64))
    out = np.zeros(max(len(ps), 1), dtype=np.uint64)
    st = lib().orc_n_mod(P, d, m, _ptr(ps), len(ps), _ptr(out))
    if st:
        raise RuntimeError(f"orc_n_mod failed: {st}")
    return out[:len(ps)]
