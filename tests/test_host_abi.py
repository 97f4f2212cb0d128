"""CPU checks of the C-ABI library: it loads, exports every symbol the headers declare, and its
host-only planning (rows, columns, layout, validation) agrees with the oracle.  No GPU work."""
import os
import re

import numpy as np
import pytest

import workloads as W
from oracle import coracle
import paper_2012_03771_amd as cs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    names = []
    inc = os.path.join(ROOT, "include")
    for fn in sorted(os.listdir(inc)):
        if not fn.endswith(".h"):
            continue
        text = open(os.path.join(inc, fn)).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        names += re.findall(r"\b(cs_[a-z_0-9]+)\s*\(", text)
    return sorted(set(names))


def test_library_exports_every_declared_symbol():
    L = cs.lib()
    names = _declared_functions()
    assert "cs_sieve" in names and "cs_plan" in names
    for n in names:
        assert hasattr(L, n), n


def test_strerror():
    L = cs.lib()
    assert L.cs_strerror(0) == b"ok"
    assert L.cs_strerror(-1) == b"invalid argument"


@pytest.mark.parametrize("job", [W.SMALL, W.MEDIUM, W.PAPER_SCALE] + W.tiny_jobs(11, 20),
                         ids=lambda j: "P%d_d%d_m%d+%d_sl%d_L%d" % j.as_tuple())
def test_rows_and_columns_match_oracle(job):
    lay = cs.plan(job)
    xs = coracle.columns(job.P, job.d, job.sl)
    assert lay.n_x == len(xs)
    assert lay.row_words == (len(xs) + 31) // 32
    assert np.array_equal(cs.columns(job), xs)
    if job.m_inc <= 10**5:
        ms = coracle.rows(job.d, job.m_start, job.m_inc)
        assert lay.n_m == len(ms)
        assert np.array_equal(cs.rows(job), ms)
    assert lay.bitmap_bytes == lay.n_m * lay.row_words * 4
    assert lay.counts_bytes == lay.n_m * 4


def test_paper_scale_layout():
    """953#/210 over m in [1e8, 1e8 + 1e6): 228,573 rows, 13,102 columns, a 375 MB bitmap."""
    lay = cs.plan(W.PAPER_SCALE)
    assert lay.n_m == len(coracle.rows(210, 10**8, 10**6)) == 228573
    assert lay.n_x == 13102
    assert lay.bitmap_bytes == 228573 * 410 * 4
    assert lay.prime_cap >= 455052511


def test_coprime_m_count_13_primorial(paper_values):
    c = paper_values["coprime_m_count"]
    lay = cs.plan(W.Job(8887, c["d"], 1, c["M"], 1000, 10**6))
    assert lay.n_m == c["M_c"]


@pytest.mark.parametrize("bad,code", [
    (W.Job(1, 1, 1, 10, 10, 100), -1),               # P < 2
    (W.Job(11, 4, 1, 10, 10, 100), -1),              # d not squarefree
    (W.Job(11, 13, 1, 10, 10, 100), -1),             # d has a factor above P
    (W.Job(11, 0, 1, 10, 10, 100), -1),              # d = 0
    (W.Job(11, 1, 0, 10, 10, 100), -1),              # m_start = 0
    (W.Job(11, 1, 1, 0, 10, 100), -1),               # m_inc = 0
    (W.Job(11, 1, 1, 2**32, 10, 100), -1),           # m_inc too large
    (W.Job(11, 1, 1, 10, 0, 100), -1),               # sl = 0
    (W.Job(11, 1, 1, 10, 2**17, 100), -1),           # sl too large
    (W.Job(11, 1, 1, 10, 10, 1), -1),                # limit < 2
    (W.Job(11, 1, 1, 10, 10, 2**63), -2),            # limit too large (primes below 2^63)
    (W.Job(5, 30, 1, 10, 1, 100), -1),               # K = 1, sl >= m_start*K
    (W.Job(7, 6, 1, 10, 35, 100), -1),               # K = 35, sl = 35 >= 1*35
])
def test_validation(bad, code):
    with pytest.raises(cs.CsError) as e:
        cs.plan(bad)
    assert e.value.status == code


def test_three_gap_threshold_floor():
    lay = cs.plan(W.SMALL, cs.Tune(thr=1, large_mode=cs.LARGE_THREE_GAP))
    assert lay.thr >= 4 * W.SMALL.sl
    lay = cs.plan(W.SMALL, cs.Tune(thr=1))
    assert lay.thr == max(W.SMALL.P, 2 * W.SMALL.sl)


def test_zero_row_job_is_valid():
    lay = cs.plan(W.Job(11, 2, 4, 1, 5, 100))     # m = 4 only, even, d = 2
    assert lay.n_m == 0 and lay.bitmap_bytes == 0


def _cell_bound(job, thr):
    """Distinct prime factors above thr that a number m K + X of the interval can have."""
    import math
    ps = [q for q in range(2, job.P + 1) if all(q % r for r in range(2, int(q ** 0.5) + 1))]
    log2_n = math.log2(job.m_start + job.m_inc + 1) + sum(math.log2(q) for q in ps if job.d % q)
    return math.floor(log2_n / math.log2(thr + 1))


@pytest.mark.parametrize("job", [W.SMALL, W.MEDIUM, W.PAPER_SCALE, W.Job(4001, 1, 1, 100, 1000, 10**6),
                                 W.Job(1511, 30, 10, 2000, 300, 10**7)],
                         ids=["small", "medium", "paper", "p4001", "p1511"])
@pytest.mark.parametrize("mode", [cs.LARGE_G, cs.LARGE_THREE_GAP], ids=["g", "three_gap"])
def test_scatter_choice_follows_the_counter_bound(job, mode):
    lay = cs.plan(job, cs.Tune(large_mode=mode))
    fits = _cell_bound(job, lay.thr) < 256
    lb = 0
    while lb < 6 and (2 << lb) * (lay.row_words * 4 + 4) <= 60 * 1024:
        lb += 1
    shift = max(lay.n_x - 1, 0).bit_length()
    list_ok = lay.n_m > 0 and (lay.n_m << shift) <= 2**32 and -(-lay.n_m // (1 << lb)) <= 8192
    auto_list = False                      # the list is taken only on request
    assert lay.scatter == (cs.SCATTER_LIST if auto_list else cs.SCATTER_BYTES if fits else cs.SCATTER_ATOMIC)
    assert cs.plan(job, cs.Tune(large_mode=mode, scatter=cs.SCATTER_ATOMIC)).scatter == cs.SCATTER_ATOMIC
    if list_ok:
        ll = cs.plan(job, cs.Tune(large_mode=mode, scatter=cs.SCATTER_LIST))
        assert ll.scatter == cs.SCATTER_LIST and (ll.ws_bytes == lay.ws_bytes or not auto_list)
    if fits:
        lb = cs.plan(job, cs.Tune(large_mode=mode, scatter=cs.SCATTER_BYTES))
        assert lb.scatter == cs.SCATTER_BYTES
        la = cs.plan(job, cs.Tune(large_mode=mode, scatter=cs.SCATTER_ATOMIC))
        assert lb.ws_bytes + 256 >= la.ws_bytes + lay.n_m * lay.row_words * 32   # 256-byte aligned regions
    else:
        with pytest.raises(cs.CsError) as e:
            cs.plan(job, cs.Tune(large_mode=mode, scatter=cs.SCATTER_BYTES))
        assert e.value.status == -1


def test_paper_scale_scatter_modes():
    assert cs.plan(W.PAPER_SCALE, cs.Tune(large_mode=cs.LARGE_THREE_GAP)).scatter == cs.SCATTER_BYTES
    assert cs.plan(W.PAPER_SCALE, cs.Tune(large_mode=cs.LARGE_G)).scatter == cs.SCATTER_BYTES
    for mode in (cs.LARGE_G, cs.LARGE_THREE_GAP):
        assert cs.plan(W.PAPER_SCALE, cs.Tune(large_mode=mode, scatter=cs.SCATTER_LIST)).scatter == cs.SCATTER_LIST
        assert cs.plan(W.PAPER_SCALE, cs.Tune(large_mode=mode, scatter=cs.SCATTER_BYTES)).scatter == cs.SCATTER_BYTES
    # the list pool holds ~1.15x the expected large hits (n_m n_x (log log limit - log log thr))
    import math
    lay = cs.plan(W.PAPER_SCALE, cs.Tune(large_mode=cs.LARGE_THREE_GAP, scatter=cs.SCATTER_LIST))
    atom = cs.plan(W.PAPER_SCALE, cs.Tune(large_mode=cs.LARGE_THREE_GAP, scatter=cs.SCATTER_ATOMIC))
    expect = lay.n_m * lay.n_x * (math.log(math.log(1e10)) - math.log(math.log(lay.thr + 1)))
    assert 2 * 4 * 1.15 * expect < lay.ws_bytes - atom.ws_bytes < 2 * 4 * 1.2 * expect + 2**30
    # a job with 228,573 rows of 13,102 columns fits 32-bit cells; a wider one does not
    assert cs.plan(W.Job(953, 210, 10**8, 4 * 10**6, 20000, 10**9)).scatter != cs.SCATTER_LIST
    with pytest.raises(cs.CsError):
        cs.plan(W.Job(953, 210, 10**8, 4 * 10**6, 20000, 10**9), cs.Tune(scatter=cs.SCATTER_LIST))
    assert cs.plan(W.Job(4001, 1, 1, 100, 1000, 10**6), cs.Tune(scatter=cs.SCATTER_LIST)).scatter == cs.SCATTER_LIST


def test_chunked_plan():
    """cs_plan_chunked: spans must be segment-aligned, at least 2^25 and above P; a span above
    the limit is the whole sieve; smaller spans hold one chunk's tables."""
    job = W.PAPER_SCALE
    whole = cs.plan(job, cs.Tune(kmod=cs.KMOD_TABLE))     # chunks always read K mod p from tables
    for bad in (0, (1 << 25) + 1, 1 << 24, 3 << 19):
        with pytest.raises(cs.CsError):
            cs.plan_chunked(job, bad)
    assert cs.plan_chunked(job, 1 << 34).ws_bytes == whole.ws_bytes
    lay = cs.plan_chunked(job, 1 << 31)
    assert lay.ws_bytes < whole.ws_bytes / 2
    assert 105_000_000 < lay.prime_cap < 106_000_000          # pi(2^31) = 105,097,565, plus a margin
    assert (lay.n_m, lay.n_x, lay.row_words) == (whole.n_m, whole.n_x, whole.row_words)


def test_chunked_range_validation():
    """cs_sieve_chunked_range rejects a zero span and a missing workspace before any device work;
    chunked plans take limits below 2^63 and reject 2^63."""
    import ctypes as C
    L = cs.binding.lib()
    job = cs.binding._cjob(W.Job(61, 6, 1000, 100, 500, 10**8))
    assert L.cs_sieve_chunked_range(C.byref(job), None, 0, 2, 100, None, None, None, 0, None) == -1
    assert L.cs_sieve_chunked_range(C.byref(job), None, 1 << 25, 2, 100, None, None, None, 0, None) == -1
    lay = cs.plan_chunked(W.Job(61, 6, 1000, 100, 500, 2**42 - 1), 1 << 36)
    assert lay.prime_cap < 3 * 10**9                         # one chunk's table, not pi(2^42)
    assert cs.plan_chunked(W.Job(61, 6, 1000, 100, 500, 2**42), 1 << 36).prime_cap < 3 * 10**9
    with pytest.raises(cs.CsError) as e:
        cs.plan_chunked(W.Job(61, 6, 1000, 100, 500, 2**63), 1 << 36)
    assert e.value.status == -2


def test_struct_layouts_match_the_header(tmp_path):
    """The ctypes mirrors of the header's structs have the C compiler's sizes and field offsets."""
    import ctypes
    import subprocess
    B = cs.binding
    structs = {"cs_job": B.cs_job, "cs_tune": B.cs_tune, "cs_layout": B.cs_layout, "cs_diag": B.cs_diag,
               "cs_server_config": B.cs_server_config, "cs_ticket_info": B.cs_ticket_info,
               "cs_batch_opts": B.cs_batch_opts,
               "cs_surround_stats": B.cs_surround_stats}
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "csieve.h"', "int main(void) {"]
    for name, ct in structs.items():
        lines.append(f'  printf("{name} %zu\\n", sizeof({name}));')
        for f in ct._fields_:
            lines.append(f'  printf("{name}.{f[0]} %zu\\n", offsetof({name}, {f[0]}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "sizes.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "sizes"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = dict(line.split() for line in out if line)
    for name, ct in structs.items():
        assert int(got[name]) == ctypes.sizeof(ct), name
        for f in ct._fields_:
            assert int(got[f"{name}.{f[0]}"]) == getattr(ct, f[0]).offset, f"{name}.{f[0]}"


def test_limits_up_to_2_63_are_planned():
    """Limits from 2^42 to 2^63 - 1 take the 64-bit residue path; planning accepts them, with the
    level-2 base primes (up to the square root of the limit) in the chunked workspace."""
    job = W.Job(7, 1, 10**12, 1000, 4000, 2**63 - 1)
    lay = cs.plan_chunked(job, 1 << 25)
    assert lay.n_m == 1000 and lay.ws_bytes > 8 * 140_000_000      # base primes up to 3.04e9
    assert cs.plan(W.Job(7, 1, 10**12, 1000, 4000, 2**42)).n_m == 1000
    with pytest.raises(cs.CsError):
        cs.plan(W.SMALL, cs.Tune(wide_log2=19))


def test_kmod_formed_in_the_large_branch_by_default():
    """A single job below 2^42 forms K mod p in the large-branch kernel, so its K mod p tables stop
    at the threshold; CS_KMOD_TABLE keeps them for every prime, and other values are rejected."""
    job = W.PAPER_SCALE
    fused = cs.plan(job, cs.Tune(large_mode=cs.LARGE_THREE_GAP))
    table = cs.plan(job, cs.Tune(large_mode=cs.LARGE_THREE_GAP, kmod=cs.KMOD_TABLE))
    # two tables of 8 bytes per prime up to the limit, against up to thr
    assert 2 * 8 * 454_000_000 < table.ws_bytes - fused.ws_bytes < 2 * 8 * 456_000_000
    with pytest.raises(cs.CsError):
        cs.plan(job, cs.Tune(kmod=2))
