"""MI355X Combined Sieve: Python binding of libcsieve.so (argument marshalling only).

Every computation runs in the HIP library; PyTorch only provides device memory and streams.
Importing this package does not load the library; the first call does, and raises if the
library was not built (there is no fallback path).
"""
from .binding import (  # noqa: F401
    CsError, Tune, Layout, Diag, LARGE_G, LARGE_THREE_GAP, BRANCH_ALL, BRANCH_SMALL, BRANCH_LARGE, SCATTER_AUTO, SCATTER_ATOMIC, SCATTER_BYTES, SCATTER_LIST, lib, lib_path, plan, columns, rows,
    sieve, sieve_into, prepare, sieve_range, diag_read, primes, kmod, job_tuple, unpack_bits, Batch, Server,
    prp_numbers, prp_test, PRP_SPRP2, PRP_LUCAS, PRP_BPSW, surround, surround_ws_bytes, SurroundStats, plan_chunked, sieve_chunked, sieve_chunked_into, sieve_chunked_range,
    WALK_CLASSES, WALK_ALL, DECADES, probe_scatter, PROBE_ATOMIC, PROBE_STORE, PROBE_LDS_ATOMIC,
    sieve_noalloc_into, scratch_bytes, BATCH_AUTO, BATCH_PERSISTENT, BATCH_LANES, batch_ws_bytes, sieve_batch,
    ORDER_AUTO, ORDER_LARGE_FIRST, ORDER_SMALL_FIRST, ORDER_BY_JOB, KMOD_AUTO, KMOD_TABLE,
)
