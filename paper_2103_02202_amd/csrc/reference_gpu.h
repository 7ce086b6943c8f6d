// Canonical reference sample computed on the GPU (host entry point).
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "circuit.h"

namespace stimgpu {

// Same result as reference_sample (Sec. 4, every random result 0), with the
// inverse tableau in device memory; runs on `s` and waits for it.  Returns a
// STIM_* code (message in err).
int gpu_reference_sample(const std::vector<Node> &tree, uint64_t num_qubits, uint64_t num_measurements,
                         std::vector<uint64_t> &bits, hipStream_t s, std::string &err);

}  // namespace stimgpu
