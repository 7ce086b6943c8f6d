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

}  // namespace stimgpu
