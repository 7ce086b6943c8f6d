// Sparse detection-event sampling for gfx950 (Sec. 5.6).
//
// Instead of propagating a frame through every gate, draw the errors and XOR
// into the outputs the detectors and observables each error flips (sets
// computed once per circuit on the host).  The errors are exactly the frame
// sampler's: the same keyed generator calls, the same 8-bit prefix test per
// (noise site, 64-shot word) and the same geometric gaps (Sec. 5.5), so on a
// circuit whose detectors are deterministic the events equal the frame
// sampler's bit for bit, at a cost of one generator call per 32 sites and
// word plus the errors themselves.
//
// One workgroup takes a contiguous range of (32-slot group, word)
// candidates of one noise execution, words fastest, so that the lanes of a
// wave draw independent calls and their hits land on neighbouring words of
// the same output rows.  Per wave: prefix test, compaction of the surviving
// (slot, word) pairs in LDS, one pair per lane for the gap walk, and an
// atomic XOR per (error, flipped lane).  Atomics are needed because two
// errors of one word can flip the same output.
#include <hip/hip_runtime.h>

#include "rng.h"
#include "sparse_kernels.h"

namespace stimgpu {

namespace {

struct SparsePhilox {
  __device__ U64x4 operator()(uint64_t c0, uint64_t c1, uint64_t c2, uint64_t c3, uint64_t seed) const {
    return philox4x64_10(c0, c1, c2, c3, seed, KEY_HI);
  }
};

__device__ __forceinline__ uint32_t wave_exclusive_scan(uint32_t v, uint32_t lane, uint32_t *total) {
  uint32_t x = v;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    uint32_t y = __shfl_up(x, d, 64);
    if (lane >= (uint32_t)d) x += y;
  }
  *total = __shfl(x, 63, 64);
  return x - v;
}

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

constexpr uint32_t kThreads = 256;

__global__ void __launch_bounds__(kThreads) k_sparse_events(SparseParams p) {
  __shared__ uint64_t thr[64];
  __shared__ uint64_t queue[kThreads];           // 64 entries per wave
  const uint32_t inst = blockIdx.y;
  const DevOp op = p.ops[p.inst_pc[inst]];
  const uint32_t code = op.code & 0xFFFFu;
  const int K = code == OP_NOISE_DEP1 ? 3 : code == OP_NOISE_DEP2 ? 15 : 0;
  const uint32_t Q = code == OP_NOISE_DEP2 ? 2 : 1;
  const uint64_t instr = p.inst_instr[inst];
  const uint64_t gbase = p.gen_base[inst];
  const uint32_t s_lo = op.slot0, s_hi = op.slot0 + op.n;
  const uint32_t g_lo = s_lo >> 5, ngroups = ((s_hi - 1) >> 5) - g_lo + 1;
  const uint64_t W = p.num_words;
  const uint64_t cand = (uint64_t)ngroups * W;
  const uint64_t c_begin = (uint64_t)blockIdx.x * kSparseChunk;
  if (c_begin >= cand) return;                   // uniform
  const uint64_t c_end = c_begin + kSparseChunk < cand ? c_begin + kSparseChunk : cand;
  if (threadIdx.x < 64) thr[threadIdx.x] = p.thresholds[(size_t)op.aux * 64 + threadIdx.x];
  __syncthreads();
  const uint64_t cut = thr[63] >> 56;            // prefix below cut: no error in the word
  const float p_est = (float)(0ull - thr[0]) * 0x1p-64f + (thr[0] == 0 ? 1.0f : 0.0f);
  const float inv_log2_keep = 1.0f / (log1pf(-p_est) * 1.44269504088896340736f);
  const uint32_t lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  uint64_t *q = queue + wave * 64;
  for (uint64_t b = c_begin + wave * 64; b < c_end; b += kThreads) {
    const uint64_t c = b + lane;
    uint32_t mask = 0, grp = 0;
    uint64_t w = 0;
    U64x4 r{{0, 0, 0, 0}};
    if (c < c_end) {
      grp = g_lo + (uint32_t)(c / W);
      w = c % W;
      r = philox4x64_10(instr, grp, p.word0 + w, PURPOSE_NOISE_PREFIX << 32, p.seed, KEY_HI);
#pragma unroll
      for (uint32_t k = 0; k < 32; k++) {
        const uint32_t s = grp * 32 + k;
        const uint64_t vp = (r.v[k >> 3] >> (8 * (k & 7))) & 0xFF;
        if (s >= s_lo && s < s_hi && vp >= cut) mask |= 1u << k;
      }
    }
    uint32_t total;
    const uint32_t first = wave_exclusive_scan((uint32_t)__builtin_popcount(mask), lane, &total);
    for (uint32_t r0 = 0; r0 < total; r0 += 64) {
      // Entries [r0, r0 + 64) of the wave's compacted list: (slot - s_lo, word, prefix).
      uint32_t idx = first;
      uint32_t m = mask;
      while (m) {
        const uint32_t k = (uint32_t)__builtin_ctz(m);
        m &= m - 1;
        if (idx >= r0 && idx < r0 + 64) {
          const uint64_t vp = (r.v[k >> 3] >> (8 * (k & 7))) & 0xFF;
          q[idx - r0] = ((uint64_t)(grp * 32 + k - s_lo) << 40) | (w << 8) | vp;
        }
        idx++;
      }
      wave_sync();
      if (r0 + lane < total) {
        const uint64_t e = q[lane];
        const uint32_t k = (uint32_t)(e >> 40);
        const uint64_t ww = (e >> 8) & 0xFFFFFFFFull;
        const uint64_t shots_left = p.num_shots - 64 * ww;      // > 0
        const uint64_t gk = gbase + 2ull * Q * k;
        noise_walk(K, p.seed, instr, (uint64_t)s_lo + k, p.word0 + ww, thr, inv_log2_keep, e & 0xFF, SparsePhilox(),
                   [&](int pos, uint32_t ch) {
                     if ((uint64_t)pos >= shots_left) return;   // past the last shot
                     // Generator bits X_a, Z_a, X_b, Z_b of the error's Pauli.
                     uint32_t gens;
                     if (K == 15) gens = ch + 1;
                     else if (K == 3) gens = (ch <= 1 ? 1u : 0u) | (ch >= 1 ? 2u : 0u);
                     else gens = code == OP_NOISE_X ? 1u : code == OP_NOISE_Z ? 2u : 3u;
                     const uint64_t bit = 1ull << pos;
                     for (uint32_t gb = 0; gb < 2 * Q; gb++) {
                       if (!((gens >> gb) & 1)) continue;
                       const uint64_t gid = gk + gb;
                       for (uint32_t a = p.set_off[gid]; a < p.set_off[gid + 1]; a++) {
                         const uint32_t l = p.set_lanes[a];
                         uint64_t *dst = l < p.num_det ? p.det + (uint64_t)l * W + ww
                                                       : p.obs + (uint64_t)(l - p.num_det) * W + ww;
                         if (l < p.num_det || p.obs != nullptr)
                           __hip_atomic_fetch_xor(dst, bit, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                       }
                     }
                   });
      }
      wave_sync();
    }
  }
}

}  // namespace

hipError_t launch_sparse_events(const SparseParams &p, uint32_t instances, uint64_t max_candidates,
                                hipStream_t stream) {
  if (instances == 0 || max_candidates == 0) return hipSuccess;
  const uint64_t gx = (max_candidates + kSparseChunk - 1) / kSparseChunk;
  if (instances > 65535 || gx > 0x7FFFFFFFull || p.num_words >= (1ull << 32)) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_sparse_events, dim3((uint32_t)gx, instances), dim3(kThreads), 0, stream, p);
  return hipGetLastError();
}

}  // namespace stimgpu
