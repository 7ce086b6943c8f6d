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

#include "lds_attr.h"
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
  __shared__ uint64_t queue[2 * kThreads];       // 128 entries per wave
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
  uint64_t *q = queue + wave * 128;              // up to 63 carried + 64 new entries
  uint32_t pending = 0;                          // entries waiting in q (same in every lane)
  // Expands one queued (slot, word) into its errors and XORs their sets.  The
  // slot's generator offsets are loaded before the walk's generator calls.
  auto walk = [&](uint64_t e, bool active) {
    if (!active) return;
    const uint32_t k = (uint32_t)(e >> 40);
    const uint64_t ww = (e >> 8) & 0xFFFFFFFFull;
    const uint64_t shots_left = p.num_shots - 64 * ww;      // > 0
    const uint64_t gk = gbase + 2ull * Q * k;
    uint32_t so[5];
#pragma unroll
    for (int i = 0; i < 5; i++) so[i] = p.set_off[gk + (i <= (int)(2 * Q) ? i : 0)];
    // The walk collects, per generator (X_a, Z_a, X_b, Z_b), the shots whose
    // error contains it; each generator's set is then XORed once.
    uint64_t m[4] = {0, 0, 0, 0};
    noise_walk(K, p.seed, instr, (uint64_t)s_lo + k, p.word0 + ww, thr, inv_log2_keep, e & 0xFF, SparsePhilox(),
               [&](int pos, uint32_t ch) { add_error(K, pos, ch, m); });
    if (shots_left < 64) {                       // past the last shot
#pragma unroll
      for (int g = 0; g < 4; g++) m[g] &= (1ull << shots_left) - 1;
    }
    if (K == 0) {                                // one Pauli: X (x), Z (z) or Y (both)
      const uint64_t v = m[0];
      m[0] = code != OP_NOISE_Z ? v : 0;
      m[1] = code != OP_NOISE_X ? v : 0;
    }
#pragma unroll
    for (uint32_t gb = 0; gb < 4; gb++) {
      if (gb >= 2 * Q || !m[gb]) continue;
      for (uint32_t a = so[gb]; a < so[gb + 1]; a++) {
        const uint32_t l = p.set_lanes[a];
        uint64_t *dst = l < p.num_det ? p.det + (uint64_t)l * W + ww : p.obs + (uint64_t)(l - p.num_det) * W + ww;
        if (l < p.num_det || p.obs != nullptr)
          __hip_atomic_fetch_xor(dst, m[gb], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
    }
  };
  for (uint64_t b = c_begin + wave * 64; b < c_end; b += kThreads) {
    const uint64_t c = b + lane;
    uint32_t mask = 0, grp = 0;
    uint64_t w = 0;
    U64x4 r{{0, 0, 0, 0}};
    if (c < c_end) {
      grp = g_lo + (uint32_t)(c / W);
      w = c % W;
      r = philox4x64_10(instr, grp, p.word0 + w, PURPOSE_NOISE_PREFIX << 32, p.seed, KEY_HI);
      mask = prefix_pass_mask(r, cut) & group_slot_mask(grp, s_lo, s_hi);
    }
    uint32_t total;
    const uint32_t first = wave_exclusive_scan((uint32_t)__builtin_popcount(mask), lane, &total);
    for (uint32_t r0 = 0; r0 < total; r0 += 64) {
      // Append entries [r0, r0 + 64) of this batch's compacted list --
      // (slot - s_lo, word, prefix) -- behind the `pending` carried over.
      const uint32_t take = total - r0 < 64 ? total - r0 : 64;
      uint32_t idx = first;
      uint32_t m = mask;
      while (m) {
        const uint32_t k = (uint32_t)__builtin_ctz(m);
        m &= m - 1;
        if (idx >= r0 && idx < r0 + 64) {
          const uint64_t vp = (r.v[k >> 3] >> (8 * (k & 7))) & 0xFF;
          q[pending + idx - r0] = ((uint64_t)(grp * 32 + k - s_lo) << 40) | (w << 8) | vp;
        }
        idx++;
      }
      pending += take;
      wave_sync();
      if (pending >= 64) {                         // a full round for the lanes
        walk(q[lane], true);
        wave_sync();
        pending -= 64;
        if (lane < pending) q[lane] = q[64 + lane];
        wave_sync();
      }
    }
  }
  walk(q[lane], lane < pending);
}

// Windowed kernel (see sparse_kernels.h).  Dynamic LDS: window [win][T],
// observables [num_obs][T], per-wave queues [waves][128], threshold rows
// [kWindowMaxExec][64].
template <int T>
__global__ void __launch_bounds__(kWindowThreads) k_sparse_window(SparseWindowParams P) {
  extern __shared__ uint64_t lds[];
  __shared__ uint64_t s_instr[kWindowMaxExec], s_gbase[kWindowMaxExec], s_cut[kWindowMaxExec];
  __shared__ float s_inv[kWindowMaxExec];
  __shared__ uint32_t s_code[kWindowMaxExec], s_slo[kWindowMaxExec], s_shi[kWindowMaxExec],
      s_cstart[kWindowMaxExec + 1];
  const SparseParams &p = P.s;
  const uint32_t WIN = P.win;
  uint64_t *win = lds;
  uint64_t *obs_acc = win + (size_t)WIN * T;
  uint64_t *queues = obs_acc + (size_t)P.num_obs * T;
  uint64_t *thr_all = queues + (kWindowThreads / 64) * 128;
  const uint32_t lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  uint64_t *q = queues + wave * 128;
  const uint64_t W = p.num_words;
  // Tiles of one XCD are contiguous (the hardware deals workgroups round-robin
  // over the 8 XCDs), so the 16-byte row pieces that neighbouring tiles write
  // meet in the same L2 and leave it as whole lines.
  const uint32_t X = 8, xcd = blockIdx.x % X, per = gridDim.x / X, rem = gridDim.x % X;
  const uint32_t tile = xcd * per + (xcd < rem ? xcd : rem) + blockIdx.x / X;
  const uint64_t tw0 = (uint64_t)tile * T;
  const int valid = (int)(W - tw0 < (uint64_t)T ? W - tw0 : (uint64_t)T);
  const uint64_t D = p.num_det;
  for (uint32_t i = threadIdx.x; i < (WIN + P.num_obs) * T; i += blockDim.x) win[i] = 0;
  uint64_t cur_base = 0;     // rows below are written out
  uint32_t ring0 = 0;        // window slot of row cur_base

  auto slot_of = [&](uint64_t row) -> uint32_t {
    uint32_t s = (uint32_t)(row - cur_base) + ring0;
    return s >= WIN ? s - WIN : s;
  };
  // Writes rows [cur_base, upto) and clears their slots.
  auto flush = [&](uint64_t upto) {
    const uint64_t rows = upto - cur_base;
    for (uint64_t i = threadIdx.x; i < rows * T; i += blockDim.x) {
      const uint64_t r = cur_base + i / T;
      const int j = (int)(i % T);
      uint64_t v = 0;
      if (r - cur_base < WIN) {
        const uint32_t sl = slot_of(r);
        v = win[sl * T + j];
        win[sl * T + j] = 0;
      }
      if (j < valid) p.det[r * W + tw0 + j] = v;
    }
    ring0 = (uint32_t)((ring0 + rows) % WIN);
    cur_base = upto;
  };

  uint32_t ne = 0;           // executions of the current batch
  uint32_t pending = 0;      // queued entries of this wave
  auto walk = [&](uint64_t e, bool active) {
    if (!active) return;
    const uint32_t i = (uint32_t)(e >> 56);
    const uint32_t k = (uint32_t)((e >> 32) & 0xFFFFFFu);
    const int j = (int)((e >> 8) & 0xFF);
    const uint32_t code = s_code[i];
    const int K = code == OP_NOISE_DEP1 ? 3 : code == OP_NOISE_DEP2 ? 15 : 0;
    const uint32_t Q = code == OP_NOISE_DEP2 ? 2 : 1;
    const uint64_t gk = s_gbase[i] + 2ull * Q * k;
    uint32_t so[5];
#pragma unroll
    for (int a = 0; a < 5; a++) so[a] = p.set_off[gk + (a <= (int)(2 * Q) ? a : 0)];
    const uint64_t shots_left = p.num_shots - 64 * (tw0 + j);
    uint64_t m[4] = {0, 0, 0, 0};               // shots per generator, as in the global kernel
    noise_walk(K, p.seed, s_instr[i], (uint64_t)s_slo[i] + k, p.word0 + tw0 + j, thr_all + i * 64, s_inv[i],
               e & 0xFF, SparsePhilox(), [&](int pos, uint32_t ch) { add_error(K, pos, ch, m); });
    if (shots_left < 64) {
#pragma unroll
      for (int g = 0; g < 4; g++) m[g] &= (1ull << shots_left) - 1;
    }
    if (K == 0) {
      const uint64_t v = m[0];
      m[0] = code != OP_NOISE_Z ? v : 0;
      m[1] = code != OP_NOISE_X ? v : 0;
    }
    const uint32_t base32 = (uint32_t)cur_base;
#pragma unroll
    for (uint32_t gb = 0; gb < 4; gb++) {
      if (gb >= 2 * Q || !m[gb]) continue;
      for (uint32_t a = so[gb]; a < so[gb + 1]; a++) {
        const uint32_t l = p.set_lanes[a];
        uint64_t *dst;
        if (l < (uint32_t)D) {
          // The batch plan keeps every detector row it touches inside the
          // window; the test only guards the LDS.
          const uint32_t off = l - base32;
          if (off >= WIN) continue;
          const uint32_t sl = off + ring0 >= WIN ? off + ring0 - WIN : off + ring0;
          dst = win + sl * T + j;
        } else {
          dst = obs_acc + (l - (uint32_t)D) * T + j;
        }
        __hip_atomic_fetch_xor(dst, m[gb], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
      }
    }
  };

  __syncthreads();
  for (uint32_t b = 0; b < P.num_batches; b++) {
    const uint32_t e0 = P.batch_e0[b];
    ne = P.batch_e1[b] - e0;
    flush(P.batch_base[b]);
    // Stage the batch's executions.
    if (threadIdx.x < ne) {
      const uint32_t e = e0 + threadIdx.x;
      const DevOp op = p.ops[p.inst_pc[e]];
      s_code[threadIdx.x] = op.code & 0xFFFFu;
      s_slo[threadIdx.x] = op.slot0;
      s_shi[threadIdx.x] = op.slot0 + op.n;
      s_instr[threadIdx.x] = p.inst_instr[e];
      s_gbase[threadIdx.x] = p.gen_base[e];
    }
    for (uint32_t t = threadIdx.x; t < ne * 64; t += blockDim.x) {
      const uint32_t e = e0 + t / 64;
      thr_all[t] = p.thresholds[(size_t)p.ops[p.inst_pc[e]].aux * 64 + (t % 64)];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      uint32_t c = 0;
      for (uint32_t i = 0; i < ne; i++) {
        s_cstart[i] = c;
        c += ((((s_shi[i] - 1) >> 5) - (s_slo[i] >> 5) + 1) * T);
        const uint64_t *t = thr_all + i * 64;
        s_cut[i] = t[63] >> 56;
        const float p_est = (float)(0ull - t[0]) * 0x1p-64f + (t[0] == 0 ? 1.0f : 0.0f);
        s_inv[i] = 1.0f / (log1pf(-p_est) * 1.44269504088896340736f);
      }
      s_cstart[ne] = c;
    }
    __syncthreads();
    const uint32_t ctotal = s_cstart[ne];
    for (uint32_t b0 = wave * 64; b0 < ctotal; b0 += kWindowThreads) {
      const uint32_t c = b0 + lane;
      uint32_t mask = 0, grp = 0, i = 0;
      int j = 0;
      U64x4 r{{0, 0, 0, 0}};
      if (c < ctotal) {
        while (c >= s_cstart[i + 1]) i++;
        const uint32_t local = c - s_cstart[i];
        grp = (s_slo[i] >> 5) + local / T;
        j = (int)(local % T);
        if (j < valid) {
          r = philox4x64_10(s_instr[i], grp, p.word0 + tw0 + j, PURPOSE_NOISE_PREFIX << 32, p.seed, KEY_HI);
          mask = prefix_pass_mask(r, s_cut[i]) & group_slot_mask(grp, s_slo[i], s_shi[i]);
        }
      }
      uint32_t total;
      const uint32_t first = wave_exclusive_scan((uint32_t)__builtin_popcount(mask), lane, &total);
      for (uint32_t r0 = 0; r0 < total; r0 += 64) {
        const uint32_t take = total - r0 < 64 ? total - r0 : 64;
        uint32_t idx = first;
        uint32_t m = mask;
        while (m) {
          const uint32_t k = (uint32_t)__builtin_ctz(m);
          m &= m - 1;
          if (idx >= r0 && idx < r0 + 64) {
            const uint64_t vp = (r.v[k >> 3] >> (8 * (k & 7))) & 0xFF;
            q[pending + idx - r0] = ((uint64_t)i << 56) | ((uint64_t)(grp * 32 + k - s_slo[i]) << 32) |
                                    ((uint64_t)j << 8) | vp;
          }
          idx++;
        }
        pending += take;
        wave_sync();
        if (pending >= 64) {
          walk(q[lane], true);
          wave_sync();
          pending -= 64;
          if (lane < pending) q[lane] = q[64 + lane];
          wave_sync();
        }
      }
    }
    walk(q[lane], lane < pending);                 // the batch's last partial round
    pending = 0;
    __syncthreads();
  }
  flush(D);
  if (p.obs != nullptr)
    for (uint32_t i = threadIdx.x; i < P.num_obs * T; i += blockDim.x)
      if ((int)(i % T) < valid) p.obs[(uint64_t)(i / T) * W + tw0 + i % T] = obs_acc[i];
}

}  // namespace

size_t sparse_window_lds_bytes(int T, uint32_t win, uint32_t num_obs) {
  return ((size_t)(win + num_obs) * T + (kWindowThreads / 64) * 128 + kWindowMaxExec * 64) * sizeof(uint64_t);
}

// Static LDS of the windowed kernel (per-execution fields), kept out of the
// dynamic budget.
constexpr size_t kWindowStaticLds = 2048;

uint32_t sparse_window_max_rows(int T, uint32_t num_obs) {
  const size_t fixed = sparse_window_lds_bytes(T, 0, num_obs) + kWindowStaticLds;
  return fixed >= 160 * 1024 ? 0u : (uint32_t)((160 * 1024 - fixed) / (T * sizeof(uint64_t)));
}

template <int T>
static hipError_t launch_window_t(const SparseWindowParams &p, hipStream_t stream) {
  hipError_t e = allow_dynamic_lds((const void *)k_sparse_window<T>, (int)(160 * 1024 - kWindowStaticLds));
  if (e != hipSuccess) return e;
  const uint64_t tiles = (p.s.num_words + T - 1) / T;
  hipLaunchKernelGGL(k_sparse_window<T>, dim3((uint32_t)tiles), dim3(kWindowThreads),
                     sparse_window_lds_bytes(T, p.win, p.num_obs), stream, p);
  return hipGetLastError();
}

hipError_t launch_sparse_window(const SparseWindowParams &p, int T, hipStream_t stream) {
  if (sparse_window_lds_bytes(T, p.win, p.num_obs) + kWindowStaticLds > 160 * 1024 || p.win == 0 ||
      p.num_obs > kWindowMaxObs || p.s.num_words >= (1ull << 31))
    return hipErrorInvalidValue;
  if (p.num_batches == 0 && p.s.num_det == 0 && p.num_obs == 0) return hipSuccess;
  return T == 1 ? launch_window_t<1>(p, stream) : T == 2 ? launch_window_t<2>(p, stream) : hipErrorInvalidValue;
}

hipError_t launch_sparse_events(const SparseParams &p, uint32_t instances, uint64_t max_candidates,
                                hipStream_t stream) {
  if (instances == 0 || max_candidates == 0) return hipSuccess;
  const uint64_t gx = (max_candidates + kSparseChunk - 1) / kSparseChunk;
  if (instances > 65535 || gx > 0x7FFFFFFFull || p.num_words >= (1ull << 32)) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_sparse_events, dim3((uint32_t)gx, instances), dim3(kThreads), 0, stream, p);
  return hipGetLastError();
}

}  // namespace stimgpu
