// C ABI of the sampler (declared in include/stim_gpu.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "stim_gpu.h"
#include "circuit.h"
#include "frame_kernels.h"

using namespace stimgpu;

namespace {

thread_local std::string g_last_error;

int set_error(int code, const std::string &msg) {
  g_last_error = msg;
  return code;
}

int hip_error(hipError_t e, const char *what) {
  return set_error(STIM_E_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

// Device-resident copy of a compiled circuit.
struct DeviceCopy {
  DevOp *ops = nullptr;
  uint32_t *targets = nullptr;
  uint64_t *thresholds = nullptr;
  uint64_t *ref = nullptr;
  uint32_t *det_off = nullptr, *det_idx = nullptr, *obs_off = nullptr, *obs_idx = nullptr;
};

}  // namespace

struct stim_circuit {
  std::vector<Node> tree;
  Program prog;
  std::mutex mu;
  bool have_ref = false;
  std::vector<uint64_t> ref;
  std::map<int, DeviceCopy> dev;
};

namespace {

template <typename V>
hipError_t upload(const V &host, typename V::value_type **dst, hipStream_t s) {
  size_t bytes = std::max<size_t>(host.size(), 1) * sizeof(typename V::value_type);
  hipError_t e = hipMalloc((void **)dst, bytes);
  if (e != hipSuccess) return e;
  if (!host.empty()) e = hipMemcpyAsync(*dst, host.data(), host.size() * sizeof(typename V::value_type),
                                        hipMemcpyHostToDevice, s);
  return e;
}

int ensure_reference(stim_circuit *c) {
  if (c->have_ref) return STIM_OK;
  try {
    c->ref = reference_sample(c->tree, c->prog.num_qubits, c->prog.num_measurements);
  } catch (const std::bad_alloc &) {
    return set_error(STIM_E_OOM, "out of host memory computing the reference sample");
  }
  c->have_ref = true;
  return STIM_OK;
}

// Uploads the program and reference to the current device (first use only).
int ensure_device(stim_circuit *c, hipStream_t s, DeviceCopy **out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_error(e, "hipGetDevice");
  auto it = c->dev.find(dev);
  if (it != c->dev.end()) {
    *out = &it->second;
    return STIM_OK;
  }
  DeviceCopy d;
  const Program &P = c->prog;
  if ((e = upload(P.ops, &d.ops, s)) != hipSuccess || (e = upload(P.targets, &d.targets, s)) != hipSuccess ||
      (e = upload(P.thresholds, &d.thresholds, s)) != hipSuccess || (e = upload(c->ref, &d.ref, s)) != hipSuccess ||
      (e = upload(P.det_offsets, &d.det_off, s)) != hipSuccess ||
      (e = upload(P.det_indices, &d.det_idx, s)) != hipSuccess ||
      (e = upload(P.obs_offsets, &d.obs_off, s)) != hipSuccess ||
      (e = upload(P.obs_indices, &d.obs_idx, s)) != hipSuccess) {
    return e == hipErrorOutOfMemory ? set_error(STIM_E_OOM, "device allocation failed") : hip_error(e, "upload");
  }
  // Other streams may use this copy next: make sure the upload has landed.
  if ((e = hipStreamSynchronize(s)) != hipSuccess) return hip_error(e, "hipStreamSynchronize");
  c->dev[dev] = d;
  *out = &c->dev[dev];
  return STIM_OK;
}

bool is_device_pointer(const void *p) {
  if (!p) return false;
  hipPointerAttribute_t a;
  if (hipPointerGetAttributes(&a, p) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  return a.type == hipMemoryTypeDevice || a.type == hipMemoryTypeManaged || a.type == hipMemoryTypeUnified;
}

uint32_t threads_for(size_t frame_bytes) {
  return frame_bytes > 80 * 1024 ? 1024 : frame_bytes > 40 * 1024 ? 512 : 256;
}

bool fits_lds(uint64_t n, int T) {
  size_t fb = (size_t)16 * n * T;
  return frame_lds_bytes(n, T, true, threads_for(fb)) <= kMaxLdsBytes;
}

// Picks the shot-tile width and frame placement: the widest tile whose frame
// slice fits in LDS while still giving enough tiles to occupy the GPU.
// STIM_TILE_WORDS (1..32, power of two) and STIM_FRAME_PLACEMENT (lds|global)
// override the choice; results do not depend on it.
FrameConfig choose_config(uint64_t n, uint64_t W) {
  FrameConfig cfg{1, true, 256};
  const char *tw = std::getenv("STIM_TILE_WORDS"), *pl = std::getenv("STIM_FRAME_PLACEMENT");
  if (tw || pl) {
    int T = tw ? std::atoi(tw) : 1;
    if (T != 1 && T != 2 && T != 4 && T != 8 && T != 16 && T != 32) T = 1;
    bool lds = pl ? std::strcmp(pl, "global") != 0 : true;
    if (lds && !fits_lds(n, T)) lds = false;
    cfg.tile_words = T;
    cfg.in_lds = lds;
    cfg.threads = lds ? threads_for((size_t)16 * n * T) : 256;
    return cfg;
  }
  const int widths[] = {32, 16, 8, 4, 2, 1};
  for (int T : widths) {
    uint64_t tiles = (W + T - 1) / T;
    if (fits_lds(n, T) && (tiles >= 512 || T == 1)) {
      cfg.tile_words = T;
      cfg.in_lds = true;
      cfg.threads = threads_for((size_t)16 * n * T);
      return cfg;
    }
  }
  if (fits_lds(n, 1)) return cfg;
  // Frame slice too large for LDS even for one word: global scratch.
  cfg.in_lds = false;
  cfg.threads = 256;
  cfg.tile_words = 1;
  for (int T : widths) {
    if ((W + T - 1) / T >= 512) { cfg.tile_words = T; break; }
  }
  return cfg;
}

int check_sample_args(stim_circuit *c, uint64_t shot_offset, uint64_t num_shots) {
  if (!c) return set_error(STIM_E_INVALID_ARG, "null circuit handle");
  if (num_shots == 0) return set_error(STIM_E_INVALID_ARG, "num_shots must be positive");
  if (shot_offset % 64) return set_error(STIM_E_INVALID_ARG, "shot_offset must be a multiple of 64");
  if (c->prog.max_loop_depth > 8) return set_error(STIM_E_UNSUPPORTED, "REPEAT nesting deeper than 8");
  if (c->prog.num_qubits >= (1ull << 31)) return set_error(STIM_E_UNSUPPORTED, "too many qubits");
  return STIM_OK;
}

// Runs the frame kernel; ref == nullptr writes raw flips.
int run_frame(stim_circuit *c, DeviceCopy *d, uint64_t seed, uint64_t shot_offset, uint64_t num_shots,
              const uint64_t *ref, uint64_t *out, hipStream_t s) {
  const uint64_t W = (num_shots + 63) / 64;
  FrameConfig cfg = choose_config(c->prog.num_qubits, W);
  FrameParams p{};
  p.ops = d->ops;
  p.num_ops = (uint32_t)c->prog.ops.size();
  p.num_qubits = (uint32_t)c->prog.num_qubits;
  p.targets = d->targets;
  p.thresholds = d->thresholds;
  p.ref = ref;
  p.seed = seed;
  p.word0 = shot_offset / 64;
  p.num_words = W;
  uint64_t rem = num_shots % 64;
  p.tail_mask = rem ? ((1ull << rem) - 1) : ~0ull;
  p.out = out;
  p.out_stride = W;
  p.scratch = nullptr;
  hipError_t e;
  if (!cfg.in_lds) {
    uint64_t tiles = (W + cfg.tile_words - 1) / cfg.tile_words;
    size_t bytes = (size_t)tiles * cfg.tile_words * 16 * std::max<uint64_t>(c->prog.num_qubits, 1);
    if ((e = hipMallocAsync((void **)&p.scratch, bytes, s)) != hipSuccess)
      return set_error(STIM_E_OOM, "frame scratch allocation failed");
  }
  if (c->prog.num_measurements > 0 || c->prog.num_qubits > 0) {
    if ((e = launch_frame(p, cfg, s)) != hipSuccess) {
      if (p.scratch) (void)hipFreeAsync(p.scratch, s);
      return hip_error(e, "frame kernel launch");
    }
  }
  if (p.scratch && (e = hipFreeAsync(p.scratch, s)) != hipSuccess) return hip_error(e, "hipFreeAsync");
  return STIM_OK;
}

}  // namespace

extern "C" {

const char *stim_last_error(void) { return g_last_error.c_str(); }

int stim_compile(const char *text, size_t len, stim_circuit **out) {
  if (!out || (!text && len)) return set_error(STIM_E_INVALID_ARG, "null argument");
  *out = nullptr;
  try {
    std::unique_ptr<stim_circuit> c(new stim_circuit());
    c->tree = parse_circuit(std::string(text ? text : "", len));
    c->prog = compile_program(c->tree);
    *out = c.release();
    g_last_error.clear();
    return STIM_OK;
  } catch (const CompileError &e) {
    return set_error(e.code, e.msg);
  } catch (const std::bad_alloc &) {
    return set_error(STIM_E_OOM, "out of host memory");
  } catch (const std::exception &e) {
    return set_error(STIM_E_PARSE, e.what());
  }
}

void stim_circuit_free(stim_circuit *c) {
  if (!c) return;
  int cur = 0;
  (void)hipGetDevice(&cur);
  for (auto &kv : c->dev) {
    (void)hipSetDevice(kv.first);
    DeviceCopy &d = kv.second;
    void *ptrs[] = {d.ops, d.targets, d.thresholds, d.ref, d.det_off, d.det_idx, d.obs_off, d.obs_idx};
    for (void *p : ptrs) if (p) (void)hipFree(p);
  }
  if (!c->dev.empty()) (void)hipSetDevice(cur);
  delete c;
}

int stim_circuit_shape(const stim_circuit *c, uint64_t *num_qubits, uint64_t *num_measurements,
                       uint64_t *num_detectors, uint64_t *num_observables, uint64_t *num_gate_targets) {
  if (!c) return set_error(STIM_E_INVALID_ARG, "null circuit handle");
  if (num_qubits) *num_qubits = c->prog.num_qubits;
  if (num_measurements) *num_measurements = c->prog.num_measurements;
  if (num_detectors) *num_detectors = c->prog.num_detectors;
  if (num_observables) *num_observables = c->prog.num_observables;
  if (num_gate_targets) *num_gate_targets = c->prog.num_gate_targets;
  return STIM_OK;
}

int stim_reference_sample(stim_circuit *c, uint64_t *ref_out) {
  if (!c) return set_error(STIM_E_INVALID_ARG, "null circuit handle");
  std::lock_guard<std::mutex> lock(c->mu);
  int rc = ensure_reference(c);
  if (rc) return rc;
  if (ref_out && !c->ref.empty()) std::memcpy(ref_out, c->ref.data(), c->ref.size() * sizeof(uint64_t));
  return STIM_OK;
}

int stim_frame_sample(stim_circuit *c, uint64_t seed, uint64_t shot_offset, uint64_t num_shots,
                      uint64_t *out_meas, void *hip_stream) {
  int rc = check_sample_args(c, shot_offset, num_shots);
  if (rc) return rc;
  if (c->prog.num_measurements > 0 && !is_device_pointer(out_meas))
    return set_error(STIM_E_INVALID_ARG, "out_meas is not a device pointer");
  hipStream_t s = (hipStream_t)hip_stream;
  DeviceCopy *d = nullptr;
  {
    std::lock_guard<std::mutex> lock(c->mu);
    if ((rc = ensure_reference(c))) return rc;
    if ((rc = ensure_device(c, s, &d))) return rc;
  }
  return run_frame(c, d, seed, shot_offset, num_shots, d->ref, out_meas, s);
}

int stim_detector_sample(stim_circuit *c, uint64_t seed, uint64_t shot_offset, uint64_t num_shots,
                         uint64_t *out_det, uint64_t *out_obs, void *hip_stream) {
  int rc = check_sample_args(c, shot_offset, num_shots);
  if (rc) return rc;
  if (c->prog.num_detectors > 0 && !is_device_pointer(out_det))
    return set_error(STIM_E_INVALID_ARG, "out_det is not a device pointer");
  if (out_obs && c->prog.num_observables > 0 && !is_device_pointer(out_obs))
    return set_error(STIM_E_INVALID_ARG, "out_obs is not a device pointer");
  hipStream_t s = (hipStream_t)hip_stream;
  DeviceCopy *d = nullptr;
  {
    std::lock_guard<std::mutex> lock(c->mu);
    if ((rc = ensure_reference(c))) return rc;
    if ((rc = ensure_device(c, s, &d))) return rc;
  }
  const uint64_t W = (num_shots + 63) / 64;
  uint64_t *flips = nullptr;
  size_t bytes = (size_t)std::max<uint64_t>(c->prog.num_measurements, 1) * W * sizeof(uint64_t);
  hipError_t e = hipMallocAsync((void **)&flips, bytes, s);
  if (e != hipSuccess) return set_error(STIM_E_OOM, "flip scratch allocation failed");
  rc = run_frame(c, d, seed, shot_offset, num_shots, nullptr, flips, s);
  if (!rc && (e = launch_parity(flips, W, d->det_off, d->det_idx, (uint32_t)c->prog.num_detectors, out_det, s)) !=
                 hipSuccess)
    rc = hip_error(e, "detector kernel launch");
  if (!rc && out_obs &&
      (e = launch_parity(flips, W, d->obs_off, d->obs_idx, (uint32_t)c->prog.num_observables, out_obs, s)) !=
          hipSuccess)
    rc = hip_error(e, "observable kernel launch");
  hipError_t fe = hipFreeAsync(flips, s);
  if (!rc && fe != hipSuccess) rc = hip_error(fe, "hipFreeAsync");
  return rc;
}

int stim_batch_sample(const stim_request *reqs, size_t n, void *hip_stream) {
  if (!reqs && n) return set_error(STIM_E_INVALID_ARG, "null request array");
  for (size_t i = 0; i < n; i++) {
    const stim_request &r = reqs[i];
    int rc = r.mode == 0 ? stim_frame_sample(r.c, r.seed, r.shot_offset, r.num_shots, r.out0, hip_stream)
             : r.mode == 1 ? stim_detector_sample(r.c, r.seed, r.shot_offset, r.num_shots, r.out0, r.out1, hip_stream)
                           : set_error(STIM_E_INVALID_ARG, "bad request mode");
    if (rc) return rc;
  }
  return STIM_OK;
}

}  // extern "C"
