// Raises a kernel's dynamic-LDS limit once per (device, kernel).  Safe to call
// from several host threads: launches from different threads (one stream
// each) share the record of what has been set.
#pragma once

#include <hip/hip_runtime.h>

#include <mutex>
#include <set>
#include <utility>

namespace stimgpu {

inline hipError_t allow_dynamic_lds(const void *kernel, int bytes) {
  static std::mutex mu;
  static std::set<std::pair<int, const void *>> done;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  std::lock_guard<std::mutex> lock(mu);
  if (done.count({dev, kernel})) return hipSuccess;
  e = hipFuncSetAttribute(kernel, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
  if (e == hipSuccess) done.insert({dev, kernel});
  return e;
}

}  // namespace stimgpu
