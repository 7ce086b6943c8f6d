// Launch interface of the sparse detection-event kernel (host side).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "circuit.h"

namespace stimgpu {

struct SparseParams {
  const DevOp *ops;
  const uint32_t *targets;
  const uint64_t *thresholds;   // [rows][64]
  const uint32_t *inst_pc;      // [instances] pc of each noise execution
  const uint64_t *inst_instr;   // [instances] its flat instruction index
  const uint64_t *gen_base;     // [instances] first error-set generator
  const uint32_t *set_off;      // [generators + 1]
  const uint32_t *set_lanes;    // lane d < num_det: detector d; else observable d - num_det
  uint64_t seed, word0, num_words, num_shots;
  uint64_t *det;                // [num_det][num_words], zeroed by the caller
  uint64_t *obs;                // [observables][num_words], zeroed by the caller, or NULL
  uint32_t num_det;
};

// Candidates -- (32-slot group, word) pairs -- per workgroup.
constexpr uint32_t kSparseChunk = 2048;

// Draws every error of every noise execution (the frame sampler's own draws)
// and XORs the detector / observable sets of its Pauli into det / obs; grid
// (ceil(max_candidates / kSparseChunk), instances).  max_candidates is the
// largest number of (32-slot group, word) pairs of one noise execution.
hipError_t launch_sparse_events(const SparseParams &p, uint32_t instances, uint64_t max_candidates,
                                hipStream_t stream);

// Windowed variant: one workgroup per tile of T words (T = 1 or 2) walks
// the noise executions in circuit order, in batches, and accumulates its
// detection events in an LDS window of `win` detector rows (a ring), writing
// each row to det once it can no longer change (plain stores, no atomics, no
// zeroing of det).  Batch b covers executions [batch_e0[b], batch_e1[b]); all
// rows below batch_base[b] are final before it starts, and every row its
// errors touch lies in [batch_base[b], batch_base[b] + win).  Observables
// (at most kWindowMaxObs) are accumulated in LDS too.
constexpr uint32_t kWindowThreads = 1024;
constexpr uint32_t kWindowMaxExec = 32;      // executions per batch
constexpr uint32_t kWindowMaxObs = 256;

struct SparseWindowParams {
  SparseParams s;
  const uint32_t *batch_e0, *batch_e1, *batch_base;
  uint32_t num_batches;
  uint32_t win;
  uint32_t num_obs;
};

// Dynamic LDS bytes of one windowed workgroup, and the most window rows that
// fit next to the static part.
size_t sparse_window_lds_bytes(int T, uint32_t win, uint32_t num_obs);
uint32_t sparse_window_max_rows(int T, uint32_t num_obs);
hipError_t launch_sparse_window(const SparseWindowParams &p, int T, hipStream_t stream);

}  // namespace stimgpu
