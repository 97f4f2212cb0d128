// Host-side launch wrappers of the kernels (defined in kernels.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "device.h"

namespace cs {

// Scratch of the segmented prime sieve.
struct PrimeWs {
  uint32_t* base;       // odd primes <= 2^20
  uint32_t* n_base;     // device scalar
  uint32_t* flags;      // n_seg * kSegWords prime flags
  uint32_t* seg_count;  // n_seg
  uint64_t* seg_off;    // n_seg
  uint64_t* primes;     // output table
  uint64_t* n_primes;   // device scalar
  uint64_t cap;
  // level-2 base primes for limits from 2^42 (null otherwise): the primes up to isq, sieved with
  // their own segment scratch, then the base of the limit's segments
  uint64_t* base2 = nullptr;
  uint64_t* n_base2 = nullptr;
  uint32_t* flags2 = nullptr;
  uint32_t* seg_count2 = nullptr;
  uint64_t* seg_off2 = nullptr;
  uint64_t cap2 = 0, isq = 0;
};

// Name and message of the last failed launch in this thread (empty if none).
const char* last_error_detail();
// Checks the last launch and records "what: message" for cs_last_error if it failed.
hipError_t record_launch(const char* what);

hipError_t launch_write_job(const JobDev& jd, JobDev* dst, hipStream_t s);
// Copies a small host table to device memory through kernel arguments (2 KB per launch):
// no pinned staging buffer and nothing that a graph capture would reject.
hipError_t launch_upload(void* dst, const void* src, uint64_t bytes, hipStream_t s);
hipError_t launch_fill_u32(uint32_t* p, uint64_t n, uint32_t v, hipStream_t s);
hipError_t launch_zero_ctrl(JobCtrl* c, hipStream_t s);
hipError_t launch_primes(uint64_t lim, const PrimeWs& pw, hipStream_t s);
// The primes of segments seg0 .. lim >> kSegLog (integers seg0 * 2^kSegLog .. lim) into pw.primes.
hipError_t launch_primes_range(uint64_t seg0, uint64_t lim, const PrimeWs& pw, hipStream_t s);
// Table bounds of a later chunk of the prime range (chunked sieve).
hipError_t launch_chunk_bounds(JobDev* jobs, hipStream_t s);
// Kernels over a job array take the job from blockIdx.y (grid.y = n_jobs).
hipError_t launch_prep_tables(JobDev* jobs, uint32_t n_jobs, hipStream_t s);
// lim_base: n_jobs + 1 device words; total_cap: an upper bound of all jobs' primes <= limit.
hipError_t launch_kmod(const JobDev* jobs, uint32_t n_jobs, uint64_t* lim_base, uint64_t total_cap, int n_cu,
                       hipStream_t s);
hipError_t launch_fill_jobs(const JobDev* jobs, uint32_t n_jobs, uint64_t max_words, hipStream_t s);
hipError_t launch_zero_ctrls(const JobDev* jobs, uint32_t n_jobs, hipStream_t s);
hipError_t launch_kmod_list(const uint64_t* primes, uint64_t n, const uint64_t* groups, uint32_t ng,
                            uint64_t* out, int n_cu, hipStream_t s);
hipError_t launch_rows_cols(const JobDev* jobs, uint32_t n_jobs, uint64_t max_m_inc, uint32_t max_sl, int n_cu,
                            hipStream_t s);
// Per-class patterns of the primes dividing d (jobs with dpat_on); LDS of max_row_words words.
hipError_t launch_dpattern(const JobDev* jobs, uint32_t n_jobs, uint32_t max_phi, uint32_t max_row_words,
                           hipStream_t s);
// Byte-counter scatter: clear the counters (once, after allocation; max_words = the largest
// n_m * row_words over the jobs) / fold them into the bitmaps and counts and clear them again
// (max_rows = the largest n_m).
hipError_t launch_zero_bytes(const JobDev* jobs, uint32_t n_jobs, uint64_t max_words, int n_cu, hipStream_t s);
hipError_t launch_fold_bytes(const JobDev* jobs, uint32_t n_jobs, uint64_t max_rows, int n_cu, hipStream_t s);
hipError_t launch_prep_bounds(JobDev* jobs, uint32_t n_jobs, hipStream_t s);
hipError_t launch_items_scan(const JobDev* jobs, uint32_t n_jobs, uint64_t* base, hipStream_t s);
// hit_rows: the instance with the hit-row pass for small primes far above w (see k_small)
hipError_t launch_small(const JobDev* jobs, uint32_t n_jobs, uint64_t total_units, uint32_t lds_bytes,
                        uint32_t lds_ct_words, uint32_t blocks, hipStream_t s, bool hit_rows = false);
// lds_bytes = 0: tables read from global memory (any number of jobs); otherwise n_jobs must be 1
// and the column table (lds_ct_words uint2, 0 = global) and residue table (dpre_n entries) of
// that job are staged in LDS.  scatter_kind: 0 = atomic OR/add into the bitmaps and counts,
// 1 = every job's byte counters (all jobs must have them), 2 = the job's list pool (single-job
// launches only; 0 otherwise).
// diag: D_COUNT totals; dec: DC_COUNT x kDecades counters per prime decade (or null).
// large_mode: CS_LARGE_G (0) or CS_LARGE_THREE_GAP (1), the same for every job of the launch.
// wide: the primes of the launch are at least 2^42 (single-job launches): exact 64-bit residues.
hipError_t launch_large(const JobDev* jobs, uint32_t n_jobs, const uint64_t* job_item_base,
                        unsigned long long* diag, unsigned long long* dec, uint32_t blocks, uint32_t lds_bytes,
                        uint32_t lds_ct_words, uint32_t dpre_n, uint32_t scatter_kind, uint32_t large_mode,
                        hipStream_t s, bool wide = false);
// Groups the list pool of one job by row bucket and applies it to the bitmap and counts.  The
// caller cleared the pool cursor and the bucket counts before the k_large launch.
hipError_t launch_list_group(const JobDev* job, uint64_t list_chunks, uint32_t n_bkt, uint32_t bkt_rows,
                             uint32_t super_shift, uint32_t row_words, hipStream_t s);

// The persistent batch kernel over n_jobs jobs (see k_batch): tbase holds 2 n_jobs + 1 device words
// and next one; every job's column table fits lds_ct_words (and its residue table after it);
// scatter_kind 0 (atomic) or 1 (byte counters) and large_mode are common to the jobs.
// items_per_task: a multiple of 256; order: 0 large tasks first, 1 small tasks first, 2 by job.
// kg_off_words: LDS word offset (8-byte aligned) where a large task of a job that forms K mod p
// itself stages K's groups; 0 when no job does.
hipError_t launch_batch_persistent(const JobDev* jobs, uint32_t n_jobs, uint64_t* tbase, unsigned long long* next,
                                   uint32_t blocks, uint32_t lds_bytes, uint32_t lds_ct_words, uint32_t kg_off_words,
                                   uint32_t scatter_kind, uint32_t large_mode, uint32_t items_per_task, uint32_t order,
                                   hipStream_t s);

// Scatter-rate probe (see k_probe_scatter).
hipError_t launch_probe_scatter(uint32_t* buf, uint64_t words, uint64_t n_ops, uint32_t slices, uint32_t op,
                                uint64_t seed, int n_cu, hipStream_t s);

}  // namespace cs
