// Fused multi-job launches shared by the batch graph and the server.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

#include "device.h"
#include "launch.h"
#include "plan.h"

namespace cs {

struct MultiJob {
  uint32_t n = 0;
  int n_cu = 256;
  std::vector<Plan> plans;
  uint64_t Lp = 0, n_seg = 0, cap = 0;
  // device memory (one allocation) and offsets inside it
  uint8_t* mem = nullptr;
  uint64_t mem_bytes = 0;
  uint64_t o_nbase = 0, o_np = 0, o_base = 0, o_flags = 0, o_cnt = 0, o_off = 0, o_primes = 0;
  uint64_t o_jobs = 0, o_lim = 0, o_items = 0;
  std::vector<uint64_t> job_off;
  PrimeWs pw{};
  JobDev* jobs_dev = nullptr;
  uint64_t* lim_base = nullptr;
  uint64_t* items_base = nullptr;
  std::vector<JobDev> jds;
  // launch shapes
  uint64_t units = 0, max_words = 0, max_m_inc = 0, kmod_cap = 0, max_rows = 0;
  bool bytes = false;                  // large hits through every job's byte counters
  uint32_t lds_bytes = 0, lds_ct_words = 0, max_sl = 0;
  uint32_t max_phi = 0, max_rw = 0;   // class-pattern launch shape
  // lanes: streams that run the jobs' branches side by side (forked from and joined back into
  // the launch stream by events, so a captured graph holds them as parallel branches)
  std::vector<hipStream_t> lanes;
  hipEvent_t ev_fork = nullptr;
  std::vector<hipEvent_t> ev_done;
  // persistent path: every job's branches in one launch of k_batch popping tasks from a queue
  bool persistent = false;
  uint32_t large_mode = 0;
  uint32_t items_per_task = 256, order = 0;
  uint32_t persist_lds = 0, persist_blocks = 0;
  uint32_t kg_off_words = 0;        // LDS word offset of K's groups in k_batch (0: no job forms K mod p)
  uint64_t o_tbase = 0, o_next = 0;
  uint64_t* tbase = nullptr;
  unsigned long long* task_next = nullptr;
};

constexpr uint32_t kBatchLanes = 4;
// Dynamic LDS of one workgroup of the persistent kernel: with its static LDS (about 1.1 KB) four
// workgroups (sixteen wavefronts) fit the 160 KB of a CU.
constexpr uint32_t kPersistLds = 38 * 1024;
constexpr uint32_t kPersistBlocksPerCu = 4;

// Re-derives the small-branch tiles of a plan for a shared LDS column-table size and an LDS budget.
void retile_small(Plan& pl, uint32_t lds_ct_words, int n_cu, const cs_tune* tune, uint32_t lds_budget = kLdsBudget);
// Plans every job (tables without a prime table) and lays out one device allocation whose
// shared prime table reaches at least prime_extent.  want_persistent: 1 = the persistent kernel
// (CS_EINVAL when the jobs do not admit it), 0 = per-job launches over lane streams, -1 = the
// persistent kernel when the jobs admit it.
cs_status multi_build(MultiJob& b, const cs_job* jobs, const cs_tune* tunes, uint32_t n, int n_cu,
                      uint64_t prime_extent, int want_persistent = 0);
// Applies the batch-level knobs (CS_EINVAL when out of range); want_persistent as multi_build's.
cs_status batch_opts_of(const cs_batch_opts* opts, int* want_persistent);
void apply_batch_opts(MultiJob& b, const cs_batch_opts* opts);
// Allocates the device memory (hipMalloc) and uploads the per-job residue tables on s.
cs_status multi_alloc(MultiJob& b, hipStream_t s);
// Points every job's descriptor at its outputs and writes the descriptors on s.
cs_status multi_bind(MultiJob& b, uint32_t* const* bitmaps, uint32_t* const* counts, hipStream_t s);
// Enqueues the whole sieve of all jobs on s (the lane path forks the jobs' branches onto the lane
// streams and joins them back; with no lanes they run on s in turn).
cs_status multi_enqueue(MultiJob& b, hipStream_t s);
// Binds a caller-provided device allocation of b.mem_bytes instead of multi_alloc's own (no lane
// streams, everything on s): uploads the residue tables and clears the byte counters.
cs_status multi_use_memory(MultiJob& b, uint8_t* mem, hipStream_t s);
// Reads the counters of all jobs (the caller has synchronised).
cs_status multi_diag(const MultiJob& b, cs_diag* out);

}  // namespace cs
