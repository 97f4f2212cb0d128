"""ctypes binding of libcsieve.so.  Mirrors include/csieve.h name for name."""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(HERE, "_lib", "libcsieve.so")

LARGE_G = 0
LARGE_THREE_GAP = 1
BRANCH_ALL = 0
BRANCH_SMALL = 1
BRANCH_LARGE = 2
SCATTER_AUTO = 0
SCATTER_ATOMIC = 1
SCATTER_BYTES = 2
SCATTER_LIST = 3
WALK_CLASSES = 0
WALK_ALL = 1
KMOD_AUTO, KMOD_TABLE = 0, 1
DECADES = 20

_ERRORS = {0: "CS_OK", -1: "CS_EINVAL", -2: "CS_ERANGE", -3: "CS_ENOMEM", -4: "CS_EDEVICE", -5: "CS_EBUSY"}


class CsError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        super().__init__(f"{where}: {_ERRORS.get(status, status)}")


class cs_job(C.Structure):
    _fields_ = [("P", C.c_uint32), ("sl", C.c_uint32), ("d", C.c_uint64), ("m_start", C.c_uint64),
                ("m_inc", C.c_uint64), ("limit", C.c_uint64)]


class cs_tune(C.Structure):
    _fields_ = [("thr", C.c_uint64), ("tile_rows", C.c_uint32), ("hits_per_item", C.c_uint32),
                ("large_mode", C.c_uint32), ("large_blocks", C.c_uint32), ("small_slices", C.c_uint32),
                ("branches", C.c_uint32), ("scatter", C.c_uint32), ("list_chunks", C.c_uint32),
                ("walk", C.c_uint32), ("wide_log2", C.c_uint32), ("kmod", C.c_uint32)]


class cs_layout(C.Structure):
    _fields_ = [("n_m", C.c_uint64), ("n_x", C.c_uint32), ("row_words", C.c_uint32),
                ("bitmap_bytes", C.c_uint64), ("counts_bytes", C.c_uint64), ("ws_bytes", C.c_uint64),
                ("prime_cap", C.c_uint64), ("thr", C.c_uint64), ("scatter", C.c_uint32), ("reserved", C.c_uint32)]


_DEC_FIELDS = ("dec_primes", "dec_raw_hits", "dec_hits", "dec_solves", "dec_levels")


class cs_diag(C.Structure):
    _fields_ = ([(n, C.c_uint64) for n in ("n_primes", "small_primes", "large_primes", "small_pairs",
                                           "small_marks", "large_raw_hits", "large_hits", "g_calls",
                                           "g_levels", "error_flags")] + [("large_kernel_ms", C.c_double)]
                + [(n, C.c_uint64 * DECADES) for n in _DEC_FIELDS])


class cs_batch_opts(C.Structure):
    _fields_ = [("path", C.c_uint32), ("items_per_task", C.c_uint32), ("blocks_per_cu", C.c_uint32),
                ("order", C.c_uint32)]


class cs_server_config(C.Structure):
    _fields_ = [("budget_bytes", C.c_uint64), ("max_limit", C.c_uint64), ("max_active", C.c_uint32),
                ("chunks", C.c_uint32), ("tune", cs_tune), ("long_ms", C.c_double)]


class cs_ticket_info(C.Structure):
    _fields_ = [("state", C.c_int32), ("n_x", C.c_uint32), ("row_words", C.c_uint32), ("pad", C.c_uint32),
                ("n_m", C.c_uint64), ("queued_s", C.c_double), ("latency_s", C.c_double)]


class cs_server_counters(C.Structure):
    _fields_ = [(n, C.c_uint64) for n in ("submitted", "admitted", "completed", "failed", "iterations",
                                          "kmod_builds", "kmod_hits", "kmod_evictions", "bytes_in_use",
                                          "active", "queued", "bytes_iterations")]


@dataclass
class Tune:
    thr: int = 0
    tile_rows: int = 0
    hits_per_item: int = 0
    large_mode: int = LARGE_G
    large_blocks: int = 0
    small_slices: int = 0
    branches: int = 0
    scatter: int = 0
    list_chunks: int = 0
    walk: int = WALK_CLASSES
    wide_log2: int = 0
    kmod: int = KMOD_AUTO

    def c(self):
        return cs_tune(self.thr, self.tile_rows, self.hits_per_item, self.large_mode, self.large_blocks,
                       self.small_slices, self.branches, self.scatter, self.list_chunks, self.walk, self.wide_log2,
                       self.kmod)


@dataclass
class Layout:
    n_m: int
    n_x: int
    row_words: int
    bitmap_bytes: int
    counts_bytes: int
    ws_bytes: int
    prime_cap: int
    thr: int
    scatter: int


@dataclass
class Diag:
    n_primes: int
    small_primes: int
    large_primes: int
    small_pairs: int
    small_marks: int
    large_raw_hits: int
    large_hits: int
    g_calls: int
    g_levels: int
    error_flags: int
    large_kernel_ms: float = 0.0
    dec_primes: tuple = ()      # large-branch counters per prime decade 10^i <= p < 10^(i+1)
    dec_raw_hits: tuple = ()
    dec_hits: tuple = ()
    dec_solves: tuple = ()
    dec_levels: tuple = ()


def _diag_of(out) -> Diag:
    vals = []
    for f in cs_diag._fields_:
        v = getattr(out, f[0])
        vals.append(tuple(int(x) for x in v) if f[0] in _DEC_FIELDS else v)
    return Diag(*vals)


class cs_surround_stats(C.Structure):
    _fields_ = [("rounds", C.c_uint64), ("tests", C.c_uint64), ("limbs", C.c_uint64), ("bits", C.c_uint64),
                ("test_ms", C.c_double), ("lucas_tests", C.c_uint64), ("lucas_passes", C.c_uint64),
                ("lucas_ms", C.c_double)]


@dataclass
class SurroundStats:
    rounds: int
    tests: int
    limbs: int
    bits: int
    test_ms: float
    lucas_tests: int = 0
    lucas_passes: int = 0
    lucas_ms: float = 0.0


_lib = None


def lib_path() -> str:
    return _LIB_PATH


def lib():
    """Loads libcsieve.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        raise RuntimeError(f"{_LIB_PATH} is missing: build it with `python -c 'import __graft_entry__ as g; g.build()'`")
    L = C.CDLL(_LIB_PATH)
    P, u64, u32, i32, vp = C.POINTER, C.c_uint64, C.c_uint32, C.c_int32, C.c_void_p
    sig = {
        "cs_strerror": ([i32], C.c_char_p),
        "cs_last_error": ([], C.c_char_p),
        "cs_plan": ([P(cs_job), P(cs_tune), P(cs_layout)], i32),
        "cs_columns": ([P(cs_job), vp, u64], i32),
        "cs_rows": ([P(cs_job), vp, u64], i32),
        "cs_sieve": ([P(cs_job), P(cs_tune), vp, vp, vp, u64, vp], i32),
        "cs_prepare": ([P(cs_job), P(cs_tune), vp, u64, vp], i32),
        "cs_sieve_range": ([P(cs_job), P(cs_tune), u64, u64, vp, vp, vp, u64, vp], i32),
        "cs_plan_chunked": ([P(cs_job), P(cs_tune), u64, P(cs_layout)], i32),
        "cs_sieve_chunked": ([P(cs_job), P(cs_tune), u64, vp, vp, vp, u64, vp], i32),
        "cs_sieve_chunked_range": ([P(cs_job), P(cs_tune), u64, u64, u64, vp, vp, vp, u64, vp], i32),
        "cs_diag_read": ([vp, P(cs_diag), vp], i32),
        "cs_primes_ws": ([u64, P(u64), P(u64)], i32),
        "cs_primes": ([u64, vp, u64, vp, vp, u64, vp], i32),
        "cs_kmod_ws": ([u32, u64, P(u64)], i32),
        "cs_kmod": ([u32, u64, vp, u64, vp, vp, u64, vp], i32),
        "cs_batch_create": ([P(cs_job), u32, P(cs_tune), P(vp)], i32),
        "cs_batch_create_ex": ([P(cs_job), u32, P(cs_tune), P(cs_batch_opts), P(vp)], i32),
        "cs_batch_path": ([vp], u32),
        "cs_batch_ws": ([P(cs_job), u32, P(cs_tune), P(u64)], i32),
        "cs_sieve_batch": ([P(cs_job), u32, P(cs_tune), P(cs_batch_opts), P(vp), P(vp), vp, u64, vp], i32),
        "cs_batch_layout": ([vp, u32, P(cs_layout)], i32),
        "cs_batch_run": ([vp, P(vp), P(vp), i32, vp], i32),
        "cs_batch_diag": ([vp, P(cs_diag), vp], i32),
        "cs_batch_destroy": ([vp], i32),
        "cs_server_create": ([P(cs_server_config), P(vp)], i32),
        "cs_server_submit": ([vp, P(cs_job), P(u64)], i32),
        "cs_server_poll": ([vp, u64, P(cs_ticket_info)], i32),
        "cs_server_wait": ([vp, u64, C.c_double, P(cs_ticket_info)], i32),
        "cs_server_copy_outputs": ([vp, u64, vp, vp, vp], i32),
        "cs_server_release": ([vp, u64], i32),
        "cs_server_stats": ([vp, P(cs_server_counters)], i32),
        "cs_server_destroy": ([vp], i32),
        "cs_prp_numbers": ([vp, u32, u64, vp, vp], i32),
        "cs_prp_test": ([vp, u32, u64, u32, vp, vp], i32),
        "cs_surround_ws": ([P(cs_job), u64, P(u64)], i32),
        "cs_surround": ([P(cs_job), vp, vp, u64, vp, vp, u64, P(cs_surround_stats), vp], i32),
        "cs_probe_scatter": ([vp, u64, u64, u32, u32, u64, vp], i32),
        "cs_sieve_noalloc": ([P(cs_job), P(cs_tune), vp, vp, vp], i32),
        "cs_scratch_bytes": ([], u64),
    }
    for name, (args, res) in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = res
    _lib = L
    return L


def _check(st: int, where: str):
    if st != 0:
        detail = lib().cs_last_error().decode() if st == -4 else ""
        raise CsError(st, where + (f" [{detail}]" if detail else ""))


def job_tuple(job):
    if hasattr(job, "as_tuple"):
        return job.as_tuple()
    return tuple(job)


def _cjob(job) -> cs_job:
    P, d, m_start, m_inc, sl, limit = job_tuple(job)
    return cs_job(P, sl, d, m_start, m_inc, limit)


def _ctune(tune):
    if tune is None:
        return None
    return C.byref(tune.c())


def _stream(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


def plan(job, tune: Tune | None = None) -> Layout:
    out = cs_layout()
    _check(lib().cs_plan(C.byref(_cjob(job)), _ctune(tune), C.byref(out)), "cs_plan")
    return Layout(out.n_m, out.n_x, out.row_words, out.bitmap_bytes, out.counts_bytes, out.ws_bytes,
                  out.prime_cap, out.thr, out.scatter)


def plan_chunked(job, span: int, tune: Tune | None = None) -> Layout:
    """Layout of cs_sieve_chunked with chunks of `span` integers of the prime range."""
    out = cs_layout()
    _check(lib().cs_plan_chunked(C.byref(_cjob(job)), _ctune(tune), span, C.byref(out)), "cs_plan_chunked")
    return Layout(out.n_m, out.n_x, out.row_words, out.bitmap_bytes, out.counts_bytes, out.ws_bytes,
                  out.prime_cap, out.thr, out.scatter)


def columns(job):
    import numpy as np
    lay = plan(job)
    out = np.zeros(max(lay.n_x, 1), dtype=np.int32)
    _check(lib().cs_columns(C.byref(_cjob(job)), out.ctypes.data_as(C.c_void_p), lay.n_x), "cs_columns")
    return out[:lay.n_x]


def rows(job):
    import numpy as np
    lay = plan(job)
    out = np.zeros(max(lay.n_m, 1), dtype=np.uint64)
    _check(lib().cs_rows(C.byref(_cjob(job)), out.ctypes.data_as(C.c_void_p), lay.n_m), "cs_rows")
    return out[:lay.n_m]


def alloc_outputs(job, tune=None, device="cuda"):
    import torch
    lay = plan(job, tune)
    bitmap = torch.empty((lay.n_m, lay.row_words), dtype=torch.int32, device=device)
    counts = torch.empty((lay.n_m,), dtype=torch.int32, device=device)
    ws = torch.empty((lay.ws_bytes,), dtype=torch.uint8, device=device)
    return lay, bitmap, counts, ws


def sieve_into(job, bitmap, counts, ws, tune: Tune | None = None, stream=None):
    _check(lib().cs_sieve(C.byref(_cjob(job)), _ctune(tune), _ptr(bitmap), _ptr(counts), _ptr(ws),
                          ws.numel(), _stream(stream)), "cs_sieve")


def sieve_noalloc_into(job, bitmap, counts, tune: Tune | None = None, stream=None):
    """cs_sieve_noalloc: the whole sieve with the library's own device workspace (no allocation)."""
    _check(lib().cs_sieve_noalloc(C.byref(_cjob(job)), _ctune(tune), _ptr(bitmap), _ptr(counts), _stream(stream)),
           "cs_sieve_noalloc")


def scratch_bytes() -> int:
    return int(lib().cs_scratch_bytes())


def sieve(job, tune: Tune | None = None, stream=None):
    """Runs cs_sieve on freshly allocated device tensors.  Returns (bitmap int32 [n_m, row_words]
    holding the uint32 words, counts int32 [n_m], workspace)."""
    lay, bitmap, counts, ws = alloc_outputs(job, tune)
    sieve_into(job, bitmap, counts, ws, tune, stream)
    return bitmap, counts, ws


def sieve_chunked_into(job, span: int, bitmap, counts, ws, tune: Tune | None = None, stream=None):
    _check(lib().cs_sieve_chunked(C.byref(_cjob(job)), _ctune(tune), span, _ptr(bitmap), _ptr(counts), _ptr(ws),
                                  ws.numel(), _stream(stream)), "cs_sieve_chunked")


def sieve_chunked_range(job, span: int, p_lo: int, p_hi: int, bitmap, counts, ws, tune: Tune | None = None,
                        stream=None):
    _check(lib().cs_sieve_chunked_range(C.byref(_cjob(job)), _ctune(tune), span, p_lo, p_hi, _ptr(bitmap),
                                        _ptr(counts), _ptr(ws), ws.numel(), _stream(stream)), "cs_sieve_chunked_range")


def sieve_chunked(job, span: int, tune: Tune | None = None, stream=None):
    """cs_sieve_chunked on freshly allocated device tensors: (bitmap, counts, workspace)."""
    import torch
    lay = plan_chunked(job, span, tune)
    bitmap = torch.empty((lay.n_m, lay.row_words), dtype=torch.int32, device="cuda")
    counts = torch.empty((lay.n_m,), dtype=torch.int32, device="cuda")
    ws = torch.empty((lay.ws_bytes,), dtype=torch.uint8, device="cuda")
    sieve_chunked_into(job, span, bitmap, counts, ws, tune, stream)
    return bitmap, counts, ws


def prepare(job, ws, tune: Tune | None = None, stream=None):
    _check(lib().cs_prepare(C.byref(_cjob(job)), _ctune(tune), _ptr(ws), ws.numel(), _stream(stream)),
           "cs_prepare")


def sieve_range(job, p_lo, p_hi, bitmap, counts, ws, tune: Tune | None = None, stream=None):
    _check(lib().cs_sieve_range(C.byref(_cjob(job)), _ctune(tune), p_lo, p_hi, _ptr(bitmap), _ptr(counts),
                                _ptr(ws), ws.numel(), _stream(stream)), "cs_sieve_range")


def diag_read(ws, stream=None, check: bool = True) -> Diag:
    out = cs_diag()
    st = lib().cs_diag_read(_ptr(ws), C.byref(out), _stream(stream))
    d = _diag_of(out)
    if check:
        _check(st, f"cs_diag_read (error_flags={d.error_flags})")
    return d


def primes(limit: int, stream=None):
    """Device prime table (uint64 values in an int64 tensor) and its length."""
    import torch
    cap = C.c_uint64()
    wsb = C.c_uint64()
    _check(lib().cs_primes_ws(limit, C.byref(cap), C.byref(wsb)), "cs_primes_ws")
    out = torch.empty((cap.value,), dtype=torch.int64, device="cuda")
    cnt = torch.zeros((1,), dtype=torch.int64, device="cuda")
    ws = torch.empty((wsb.value,), dtype=torch.uint8, device="cuda")
    _check(lib().cs_primes(limit, _ptr(out), cap.value, _ptr(cnt), _ptr(ws), wsb.value, _stream(stream)),
           "cs_primes")
    torch.cuda.current_stream().synchronize() if stream is None else stream.synchronize()
    n = int(cnt.item())
    return out[:n], n


def kmod(P: int, d: int, primes_dev, stream=None):
    """K mod p for each prime of a device int64 tensor (K = P#/d)."""
    import torch
    wsb = C.c_uint64()
    _check(lib().cs_kmod_ws(P, d, C.byref(wsb)), "cs_kmod_ws")
    ws = torch.empty((max(wsb.value, 8),), dtype=torch.uint8, device="cuda")
    out = torch.empty_like(primes_dev)
    _check(lib().cs_kmod(P, d, _ptr(primes_dev), primes_dev.numel(), _ptr(out), _ptr(ws), ws.numel(),
                         _stream(stream)), "cs_kmod")
    return out


def unpack_bits(words, n_x: int):
    """int32/uint32 words [n, row_words] (numpy) -> uint8 [n, n_x], column c = bit c%32 of word c//32."""
    import numpy as np
    w = np.asarray(words).view(np.uint32)
    n, rw = w.shape
    out = np.zeros((n, rw * 32), dtype=np.uint8)
    for b in range(32):
        out[:, b::32] = ((w >> np.uint32(b)) & np.uint32(1)).astype(np.uint8)
    return out[:, :n_x]


BATCH_AUTO = 0
BATCH_PERSISTENT = 1
BATCH_LANES = 2


def _job_arrays(jobs, tunes):
    arr = (cs_job * len(jobs))(*[_cjob(j) for j in jobs])
    tarr = None
    if tunes is not None:
        tarr = (cs_tune * len(jobs))(*[t.c() if t is not None else Tune().c() for t in tunes])
    return arr, tarr


def batch_ws_bytes(jobs, tunes=None) -> int:
    jobs = list(jobs)
    arr, tarr = _job_arrays(jobs, tunes)
    out = C.c_uint64()
    _check(lib().cs_batch_ws(arr, len(jobs), tarr, C.byref(out)), "cs_batch_ws")
    return out.value


ORDER_AUTO = 0
ORDER_LARGE_FIRST = 1
ORDER_SMALL_FIRST = 2
ORDER_BY_JOB = 3


def _opts(path=BATCH_AUTO, items_per_task=0, blocks_per_cu=0, order=ORDER_AUTO):
    return cs_batch_opts(path, items_per_task, blocks_per_cu, order)


def sieve_batch(jobs, bitmaps, counts, ws, tunes=None, stream=None, **opts):
    """cs_sieve_batch: every job in one call on the caller's stream and workspace."""
    jobs = list(jobs)
    arr, tarr = _job_arrays(jobs, tunes)
    n = len(jobs)
    bp = (C.c_void_p * n)(*[t.data_ptr() if t.numel() else None for t in bitmaps])
    cp = (C.c_void_p * n)(*[t.data_ptr() if t.numel() else None for t in counts])
    _check(lib().cs_sieve_batch(arr, n, tarr, C.byref(_opts(**opts)), bp, cp, _ptr(ws), ws.numel(), _stream(stream)),
           "cs_sieve_batch")


class Batch:
    """Many jobs sieved by one fused launch sequence (replayed from a hipGraph).  Keyword options
    are cs_batch_opts' fields (path, items_per_task, blocks_per_cu, order)."""

    def __init__(self, jobs, tunes=None, path=BATCH_AUTO, **opts):
        jobs = list(jobs)
        self.n = len(jobs)
        arr, tarr = _job_arrays(jobs, tunes)
        h = C.c_void_p()
        _check(lib().cs_batch_create_ex(arr, self.n, tarr, C.byref(_opts(path, **opts)), C.byref(h)),
               "cs_batch_create_ex")
        self.h = h
        self.path = int(lib().cs_batch_path(self.h))
        self.layouts = []
        for i in range(self.n):
            out = cs_layout()
            _check(lib().cs_batch_layout(self.h, i, C.byref(out)), "cs_batch_layout")
            self.layouts.append(Layout(out.n_m, out.n_x, out.row_words, out.bitmap_bytes, out.counts_bytes,
                                       out.ws_bytes, out.prime_cap, out.thr, out.scatter))

    def alloc_outputs(self):
        import torch
        bm = [torch.empty((L.n_m, L.row_words), dtype=torch.int32, device="cuda") for L in self.layouts]
        ct = [torch.empty((L.n_m,), dtype=torch.int32, device="cuda") for L in self.layouts]
        return bm, ct

    def run(self, bitmaps, counts, use_graph=True, stream=None):
        bp = (C.c_void_p * self.n)(*[t.data_ptr() if t.numel() else None for t in bitmaps])
        cp = (C.c_void_p * self.n)(*[t.data_ptr() if t.numel() else None for t in counts])
        _check(lib().cs_batch_run(self.h, bp, cp, 1 if use_graph else 0, _stream(stream)), "cs_batch_run")

    def diag(self, stream=None) -> Diag:
        out = cs_diag()
        st = lib().cs_batch_diag(self.h, C.byref(out), _stream(stream))
        d = _diag_of(out)
        _check(st, f"cs_batch_diag (error_flags={d.error_flags})")
        return d

    def close(self):
        if self.h:
            lib().cs_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """Continuous-batching sieve server (native loop in libcsieve; this class only marshals)."""

    def __init__(self, budget_bytes: int, max_limit: int, max_active: int = 16, chunks: int = 1,
                 tune: Tune | None = None, long_ms: float = 0.0):
        """long_ms > 0: jobs estimated to take longer than that alone run in a second lane."""
        cfg = cs_server_config(budget_bytes, max_limit, max_active, chunks, (tune or Tune()).c(), long_ms)
        h = C.c_void_p()
        _check(lib().cs_server_create(C.byref(cfg), C.byref(h)), "cs_server_create")
        self.h = h

    def submit(self, job) -> int:
        t = C.c_uint64()
        _check(lib().cs_server_submit(self.h, C.byref(_cjob(job)), C.byref(t)), "cs_server_submit")
        return t.value

    def poll(self, ticket: int):
        info = cs_ticket_info()
        st = lib().cs_server_poll(self.h, ticket, C.byref(info))
        _check(st, "cs_server_poll")
        return info

    def wait(self, ticket: int, timeout_s: float = 120.0):
        info = cs_ticket_info()
        st = lib().cs_server_wait(self.h, ticket, timeout_s, C.byref(info))
        _check(st, "cs_server_wait")
        return info

    def fetch(self, ticket: int, stream=None):
        """Copies a finished ticket's outputs into new device tensors."""
        import torch
        info = self.poll(ticket)
        bm = torch.empty((info.n_m, info.row_words), dtype=torch.int32, device="cuda")
        ct = torch.empty((info.n_m,), dtype=torch.int32, device="cuda")
        _check(lib().cs_server_copy_outputs(self.h, ticket, _ptr(bm) if bm.numel() else None,
                                            _ptr(ct) if ct.numel() else None, _stream(stream)),
               "cs_server_copy_outputs")
        return bm, ct

    def release(self, ticket: int):
        _check(lib().cs_server_release(self.h, ticket), "cs_server_release")

    def stats(self) -> dict:
        out = cs_server_counters()
        _check(lib().cs_server_stats(self.h, C.byref(out)), "cs_server_stats")
        return {f[0]: getattr(out, f[0]) for f in cs_server_counters._fields_}

    def close(self):
        if self.h:
            lib().cs_server_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def prp_numbers(limbs, stream=None):
    """Strong probable-prime test to base 2 (cs_prp_numbers) of the numbers in a device int32
    tensor [n, n_limbs] of little-endian 32-bit limbs.  Returns a device uint8 tensor [n]."""
    import torch
    n, nl = limbs.shape
    out = torch.empty((n,), dtype=torch.uint8, device=limbs.device)
    _check(lib().cs_prp_numbers(_ptr(limbs.contiguous()), nl, n, _ptr(out), _stream(stream)), "cs_prp_numbers")
    return out


PRP_SPRP2 = 0
PRP_LUCAS = 1
PRP_BPSW = 2


def prp_test(limbs, test: int = PRP_BPSW, stream=None):
    """cs_prp_test: the strong test to base 2, the strong Lucas test or BPSW (PRP_*) of the numbers
    in a device int32 tensor [n, n_limbs] of little-endian 32-bit limbs.  Returns a device uint8
    tensor [n]."""
    import torch
    n, nl = limbs.shape
    out = torch.empty((n,), dtype=torch.uint8, device=limbs.device)
    _check(lib().cs_prp_test(_ptr(limbs.contiguous()), nl, n, test, _ptr(out), _stream(stream)), "cs_prp_test")
    return out


def surround_ws_bytes(job, n_rows: int) -> int:
    out = C.c_uint64()
    _check(lib().cs_surround_ws(C.byref(_cjob(job)), n_rows, C.byref(out)), "cs_surround_ws")
    return out.value


def surround(job, bitmap, m_rows, ws=None, stream=None):
    """Nearest BPSW probable primes below and above N = m*K for each row (cs_surround).  bitmap: device
    int32 [n_rows, row_words] (sieved rows); m_rows: device int64 [n_rows] (the m of each row).
    Returns (device int32 tensor [n_rows, 4] = prev, next, tests_prev, tests_next; SurroundStats).
    The call returns after the work has completed."""
    import torch
    n = int(m_rows.numel())
    out = torch.empty((max(n, 1), 4), dtype=torch.int32, device=m_rows.device)
    if ws is None:
        ws = torch.empty((max(surround_ws_bytes(job, n), 1),), dtype=torch.uint8, device=m_rows.device)
    st = cs_surround_stats()
    _check(lib().cs_surround(C.byref(_cjob(job)), _ptr(bitmap), _ptr(m_rows), n, _ptr(out), _ptr(ws), ws.numel(),
                             C.byref(st), _stream(stream)), "cs_surround")
    return out[:n], SurroundStats(st.rounds, st.tests, st.limbs, st.bits, st.test_ms, st.lucas_tests,
                                  st.lucas_passes, st.lucas_ms)


PROBE_ATOMIC = 0
PROBE_STORE = 1
PROBE_LDS_ATOMIC = 2


def probe_scatter(buf, n_ops: int, slices: int = 1, op: int = PROBE_ATOMIC, seed: int = 1, stream=None):
    """cs_probe_scatter on a device int32 tensor (its words): n_ops random-word operations."""
    _check(lib().cs_probe_scatter(_ptr(buf), buf.numel(), n_ops, slices, op, seed, _stream(stream)),
           "cs_probe_scatter")
