// Pauli-frame propagation kernels for gfx950 (Sec. 3, data layout of Sec. 5.1).
//
// One workgroup owns a tile of T consecutive 64-shot words and walks the whole
// device program over it.  Shots are independent, so tiles never communicate.
// Inside a workgroup the work of one op is spread over its targets and the
// tile's words; an op's targets touch pairwise distinct qubits (the compiler
// splits instructions where a qubit repeats), so they run in parallel, and a
// barrier separates consecutive ops.
//
// The frame slice of a tile holds T X words and T Z words per qubit (bit j of
// word w = shot 64 (tile word w) + j), plus one dummy row past the last qubit
// that absorbs the writes of idle lanes.  It lives in LDS when 16 (n + 1) T
// bytes fit, as two planes X then Z, each [n + 1][T]; otherwise in a global
// scratch buffer as [n + 1][2][T] (a qubit's X and Z words adjacent).
//
// Random bits are drawn cooperatively: a lane evaluates one Philox call for a
// group of slots on one word -- four slots for Z randomisation, thirty-two
// 8-bit noise prefixes -- and only the few (slot, word) pairs whose prefix
// admits an error are queued, compacted per wave in LDS, and expanded by all
// lanes together (geometric gaps, Sec. 5.5).
#include <hip/hip_runtime.h>

#include <type_traits>

#include "bit_transpose.h"
#include "circuit.h"
#include "frame_kernels.h"
#include "lds_attr.h"
#include "rng.h"

namespace stimgpu {

// Maps a workgroup index to a tile so that the tiles of one XCD are
// contiguous: the hardware deals workgroups round-robin over the 8 XCDs, and
// neighbouring tiles share output cache lines.
__device__ __forceinline__ uint32_t xcd_tile(uint32_t bid, uint32_t nblocks) {
  const uint32_t X = 8;
  uint32_t xcd = bid % X, local = bid / X;
  uint32_t per = nblocks / X, rem = nblocks % X;
  return xcd * per + (xcd < rem ? xcd : rem) + local;
}

// Orders LDS traffic of one wave (all lanes of a wave run in lockstep).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Barrier between ops.  With the frame in LDS only LDS traffic must be
// visible to the other waves, so global stores (records, outputs) and
// prefetched loads stay in flight across it; a global frame needs the full
// fence.
template <bool IN_LDS>
__device__ __forceinline__ void tile_barrier() {
  if constexpr (IN_LDS) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
  } else {
    __syncthreads();
  }
}

// The threads that walk one tile: the whole workgroup, or (WAVE) one wave of
// it that walks its own tile with wave-level synchronisation only.
template <bool WAVE>
__device__ __forceinline__ uint32_t team_tid() { return WAVE ? (threadIdx.x & 63u) : threadIdx.x; }
template <bool WAVE>
__device__ __forceinline__ uint32_t team_size() { return WAVE ? 64u : blockDim.x; }
template <bool IN_LDS, bool WAVE>
__device__ __forceinline__ void team_barrier() {
  if constexpr (WAVE) wave_sync();
  else tile_barrier<IN_LDS>();
}
// Barrier over all memory: the team then reads global words it wrote.
template <bool WAVE>
__device__ __forceinline__ void team_barrier_all() {
  if constexpr (WAVE) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
  } else {
    __syncthreads();
  }
}

// Exclusive prefix sum over the 64 lanes of a wave; *total gets the sum.
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

// Raw buffer resource over `bytes` bytes at `base`.  Buffer loads past the end
// return zero without touching memory, so such loads can be issued
// unconditionally (no branch around them).
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buffer_rsrc(const void *base, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), (short)0, (int)bytes, 0x00020000);
}

template <int T, bool IN_LDS>
struct Tile {
  // Word index inside a plane: 32 bits suffice for an LDS-resident slice.
  typedef typename std::conditional<IN_LDS, uint32_t, size_t>::type Index;
  uint64_t *FX, *FZ;          // frame planes
  uint64_t *queue;            // this wave's 64-entry LDS queue
  uint64_t tw0;               // first local word of the tile
  int valid;                  // words of the tile inside [0, W)
  uint32_t dummy;             // row past the last qubit: a sink for writes of idle items

  __device__ __forceinline__ Index at(uint32_t q, int j) const {
    if constexpr (IN_LDS) return q * (uint32_t)T + (uint32_t)j;
    else return (size_t)q * (2 * T) + j;
  }
};

// One out-of-line copy of the generator keeps the walker's code small enough
// for the instruction cache.
__device__ __forceinline__ U64x4 philox_call(uint64_t c0, uint64_t c1, uint64_t c2, uint64_t c3, uint64_t seed) {
  return philox4x64_10(c0, c1, c2, c3, seed, KEY_HI);
}

struct PhiloxCall {
  __device__ U64x4 operator()(uint64_t c0, uint64_t c1, uint64_t c2, uint64_t c3, uint64_t seed) const {
    return philox_call(c0, c1, c2, c3, seed);
  }
};

// Applies a noise op: prefix test per (32-slot group, word), wave-compacted
// expansion of the surviving (slot, word) pairs.
template <int T, bool IN_LDS, bool WAVE>
__device__ __forceinline__ void noise_op(const FrameParams &p, const Tile<T, IN_LDS> &tl, const DevOp &op,
                                      uint32_t code, uint64_t instr, const uint64_t *thr) {
  const int K = code == OP_NOISE_DEP1 ? 3 : code == OP_NOISE_DEP2 ? 15 : 0;
  const uint32_t lane = threadIdx.x & 63, wave = WAVE ? 0u : threadIdx.x >> 6, nwaves = WAVE ? 1u : blockDim.x >> 6;
  const uint64_t cut = thr[63] >> 56;            // prefix below cut: no error in the word
  // 1 / log2(1 - p) from the exact value 2^64 - t[0] ~ p 2^64; seeds the gap search.
  const float p_est = (float)(0ull - thr[0]) * 0x1p-64f + (thr[0] == 0 ? 1.0f : 0.0f);
  const float inv_log2_keep = 1.0f / (log1pf(-p_est) * 1.44269504088896340736f);
  const uint32_t s_lo = op.slot0, s_hi = op.slot0 + op.n;
  const uint32_t g_lo = s_lo >> 5, ngroups = ((s_hi - 1) >> 5) - g_lo + 1;
  const uint32_t cand = ngroups * T;
  const uint32_t *tg = p.targets + op.toff;
  for (uint32_t base = wave * 64; base < cand; base += nwaves * 64) {
    const uint32_t c = base + lane;
    uint32_t mask = 0;
    U64x4 r{{0, 0, 0, 0}};
    uint32_t g = 0;
    int j = 0;
    if (c < cand) {
      g = g_lo + c / T;
      j = (int)(c % T);
      if (j < tl.valid) {
        r = philox_call(instr, g, p.word0 + tl.tw0 + j, PURPOSE_NOISE_PREFIX << 32, p.seed);
        mask = prefix_pass_mask(r, cut) & group_slot_mask(g, s_lo, s_hi);
      }
    }
    uint32_t total;
    const uint32_t first = wave_exclusive_scan((uint32_t)__builtin_popcount(mask), lane, &total);
    for (uint32_t r0 = 0; r0 < total; r0 += 64) {
      // Publish entries [r0, r0 + 64) of the wave's compacted list.
      uint32_t idx = first;
      uint32_t m = mask;
      while (m) {
        uint32_t b = (uint32_t)__builtin_ctz(m);
        m &= m - 1;
        if (idx >= r0 && idx < r0 + 64) {
          uint64_t vp = (r.v[b >> 3] >> (8 * (b & 7))) & 0xFF;
          tl.queue[idx - r0] = ((uint64_t)(g * 32 + b) << 24) | ((uint64_t)j << 16) | vp;
        }
        idx++;
      }
      wave_sync();
      if (r0 + lane < total) {
        const uint64_t e = tl.queue[lane];
        const uint32_t s = (uint32_t)(e >> 24);
        const int jj = (int)((e >> 16) & 0xFF);
        const uint64_t vp = e & 0xFFFF;
        uint64_t mk[4] = {0, 0, 0, 0};
        noise_masks(K, p.seed, instr, s, p.word0 + tl.tw0 + jj, thr, inv_log2_keep, vp, mk, PhiloxCall());
        const uint32_t k = s - s_lo;
        if (code == OP_NOISE_DEP2) {
          const uint32_t a = tg[2 * k], b = tg[2 * k + 1];
          tl.FX[tl.at(a, jj)] ^= mk[0];
          tl.FZ[tl.at(a, jj)] ^= mk[1];
          tl.FX[tl.at(b, jj)] ^= mk[2];
          tl.FZ[tl.at(b, jj)] ^= mk[3];
        } else {
          const uint32_t q = tg[k];
          const uint64_t mx = code == OP_NOISE_DEP1 ? mk[0] : code != OP_NOISE_Z ? mk[0] : 0;
          const uint64_t mz = code == OP_NOISE_DEP1 ? mk[1] : code != OP_NOISE_X ? mk[0] : 0;
          tl.FX[tl.at(q, jj)] ^= mx;
          tl.FZ[tl.at(q, jj)] ^= mz;
        }
      }
      wave_sync();
    }
  }
}

// Collapse ops (INIT, R, M, MR): one lane per (4-slot group, word), sharing the
// Z-randomisation call of the group.  Each thread takes two groups at a time
// and loads both groups' targets (and reference words) before doing either.
// Every thread runs at least one pass, and every load of a pass is issued
// unconditionally (clamped indices), then `after_loads` runs: loads complete in issue order, so the loads it
// issues stay in flight while the pass waits only for its own.
template <int T, bool IN_LDS, bool WAVE, bool EVENTS, typename AfterLoads>
__device__ __forceinline__ void collapse_op(const FrameParams &p, const Tile<T, IN_LDS> &tl, const DevOp &op,
                                            uint32_t code, uint64_t instr, uint64_t meas, uint64_t *ring,
                                            uint32_t ring_pos, AfterLoads after_loads) {
  constexpr int V = WAVE ? 1 : 2;               // one-wave teams: fewer registers, more waves in flight
  const uint32_t s_lo = op.slot0, s_hi = op.slot0 + op.n;
  const uint32_t g_lo = s_lo >> 2, ngroups = ((s_hi - 1) >> 2) - g_lo + 1;
  const uint32_t cand = ngroups * T;
  const uint32_t *tg = p.targets + op.toff;
  const bool measures = code == OP_M || code == OP_MR;
  const bool use_ref = !EVENTS && measures && p.ref != nullptr;      // events: raw flips
  const bool all_live = (op.code & OPF_ZRAND_LIVE) != 0;       // uniform
  const uint32_t stride = team_size<WAVE>();
  uint32_t base = team_tid<WAVE>();
  do {
    uint32_t tv[V][4];
    bool ok[V];
    uint64_t rw[V][2];           // reference words of the group's measurements
#pragma unroll
    for (int v = 0; v < V; v++) {
      const uint32_t c = base + v * stride;
      const uint32_t g = g_lo + c / T;
      const int j = (int)(c % T);
      ok[v] = c < cand && j < tl.valid;
#pragma unroll
      for (uint32_t u = 0; u < 4; u++) {
        const uint32_t s = g * 4 + u;
        const bool in = ok[v] && s >= s_lo && s < s_hi;
        const uint32_t t = tg[in ? s - s_lo : 0];
        tv[v][u] = in ? t : (TGT_DEAD_ZRAND | 0x7FFFFFFFu);
      }
      rw[v][0] = rw[v][1] = 0;
      if (use_ref) {             // uniform; the loads after it are issued on both paths
        const uint64_t m0 = meas + ((g * 4 > s_lo ? g * 4 : s_lo) - s_lo);
        const uint64_t m1 = meas + ((g * 4 + 3 < s_hi - 1 ? g * 4 + 3 : s_hi - 1) - s_lo);
        rw[v][0] = p.ref[ok[v] ? m0 >> 6 : 0];
        rw[v][1] = p.ref[ok[v] ? m1 >> 6 : 0];
      }
    }
    after_loads();
#pragma unroll
    for (int v = 0; v < V; v++) {
      if (!ok[v]) continue;
      const uint32_t c = base + v * stride;
      const uint32_t g = g_lo + c / T;
      const int j = (int)(c % T);
      const uint64_t word = p.word0 + tl.tw0 + j;
      U64x4 r{{0, 0, 0, 0}};
      if (all_live) {
        // No dependence on the targets: the draw overlaps their loads (and
        // the stores of the previous op, which complete before them).
        r = philox_call(instr, g, word, PURPOSE_ZRAND << 32, p.seed);
      } else {
        bool need = false;
#pragma unroll
        for (uint32_t u = 0; u < 4; u++) need |= !(tv[v][u] & TGT_DEAD_ZRAND);
        if (need) r = philox_call(instr, g, word, PURPOSE_ZRAND << 32, p.seed);
      }
      const uint64_t m0 = meas + ((g * 4 > s_lo ? g * 4 : s_lo) - s_lo);
#pragma unroll
      for (uint32_t u = 0; u < 4; u++) {
        const uint32_t s = g * 4 + u;
        if (s < s_lo || s >= s_hi) continue;
        const uint32_t k = s - s_lo, q = tv[v][u] & TGT_QUBIT_MASK;
        const bool dead = (tv[v][u] & TGT_DEAD_ZRAND) != 0;
        const uint64_t zr = dead ? 0 : r.v[u];
        const auto ix = tl.at(q, j);
        if (measures) {
          const uint64_t m = meas + k;
          uint64_t x = tl.FX[ix];
          const uint64_t refw = (m >> 6) == (m0 >> 6) ? rw[v][0] : rw[v][1];
          if (use_ref && ((refw >> (m & 63)) & 1)) x = ~x;
          if (tl.tw0 + j == p.num_words - 1) x &= p.tail_mask;
          if constexpr (EVENTS) {
            const uint32_t row = ring_pos + k < p.ring_rows ? ring_pos + k : ring_pos + k - p.ring_rows;
            ring[(size_t)row * T + j] = x;
          } else {
            p.out[m * p.out_stride + tl.tw0 + j] = x;
          }
        }
        if (code == OP_M) {
          if (!dead) tl.FZ[ix] ^= zr;
        } else {
          tl.FX[ix] = 0;
          tl.FZ[ix] = zr;
        }
      }
    }
    base += V * stride;
  } while (base < cand);
}

// Clifford ops: one item per (target, pair of words) -- a thread moves two
// adjacent words of a qubit with one 16-byte LDS access (one word when T = 1).
// One instantiation per opcode, so that nothing inside the item loop depends
// on the opcode at run time: a thread takes up to U items at once, issues
// every target load of the pass (a pair as one 8-byte load: the compiler
// starts every two-qubit op's targets on an even index), then every frame
// read, then the writes.  The items of one op touch distinct (qubit, word)
// cells, so this is safe.  Words of the tile past the end of the shot range
// are updated too (they belong to no shot and are never written out).  Every
// thread runs at least one pass; loads use clamped indices, so they are issued
// on every path and the compiler waits only for the loads it needs.
template <int T, bool IN_LDS, bool WAVE, uint32_t CODE, typename AfterLoads>
__device__ __forceinline__ void clifford_op(const FrameParams &p, const Tile<T, IN_LDS> &tl, const DevOp &op,
                                            AfterLoads after_loads) {
  constexpr int U = WAVE ? 1 : 3;               // one-wave teams: fewer registers, more waves in flight
  constexpr uint32_t C = T >= 2 ? 2 : 1;          // words per item
  constexpr uint32_t CPT = T / C;                 // items per target
  constexpr bool TWO = CODE == OP_CX || CODE == OP_CY || CODE == OP_CZ || CODE == OP_SWAP;
  typedef uint64_t U64x2v __attribute__((ext_vector_type(2)));
  typedef typename std::conditional<C == 2, U64x2v, uint64_t>::type Vec;
  typedef typename Tile<T, IN_LDS>::Index Index;
  const uint32_t items = op.n * CPT;
  const uint32_t *tg = p.targets + op.toff;
  const uint32_t tsize = team_size<WAVE>();
  const uint32_t per_pass = U * tsize;
  const uint32_t passes = items > per_pass ? (items + per_pass - 1) / per_pass : 1u;     // uniform
  auto X = [&](Index i) -> Vec & { return *reinterpret_cast<Vec *>(tl.FX + i); };
  auto Z = [&](Index i) -> Vec & { return *reinterpret_cast<Vec *>(tl.FZ + i); };
  for (uint32_t pass = 0; pass < passes; pass++) {
    const uint32_t base = team_tid<WAVE>() + pass * per_pass;
    uint32_t qa[U], qb[U];
    bool ok[U];
#pragma unroll
    for (int u = 0; u < U; u++) {
      const uint32_t it = base + u * tsize;
      ok[u] = it < items;
      const uint32_t k = ok[u] ? it / CPT : 0u;
      if constexpr (TWO) {
        const uint2 pr = *reinterpret_cast<const uint2 *>(tg + 2 * k);
        qa[u] = pr.x;
        qb[u] = pr.y;
      } else {
        qa[u] = tg[k];
        qb[u] = 0;
      }
    }
    after_loads();
    // Idle items (past the op's last target) read a real row and write the
    // dummy row, so that no access is predicated.
    Index ra[U], rb[U], wa[U], wb[U];
    Vec xa[U], za[U], xb[U], zb[U];
#pragma unroll
    for (int u = 0; u < U; u++) {
      const int j = (int)(((base + u * tsize) % CPT) * C);
      ra[u] = tl.at(qa[u], j);
      rb[u] = tl.at(qb[u], j);
      wa[u] = ok[u] ? ra[u] : tl.at(tl.dummy, j);
      wb[u] = ok[u] ? rb[u] : tl.at(tl.dummy, j);
      xa[u] = X(ra[u]);
      za[u] = Z(ra[u]);
      if constexpr (TWO) {
        xb[u] = X(rb[u]);
        zb[u] = Z(rb[u]);
      }
    }
#pragma unroll
    for (int u = 0; u < U; u++) {
      if constexpr (CODE == OP_SWAP_XZ) {
        X(wa[u]) = za[u];
        Z(wa[u]) = xa[u];
      } else if constexpr (CODE == OP_Z_XOR_X) {
        Z(wa[u]) = za[u] ^ xa[u];
      } else if constexpr (CODE == OP_X_XOR_Z) {
        X(wa[u]) = xa[u] ^ za[u];
      } else if constexpr (CODE == OP_CX) {
        X(wb[u]) = xb[u] ^ xa[u];
        Z(wa[u]) = za[u] ^ zb[u];
      } else if constexpr (CODE == OP_CZ) {
        Z(wa[u]) = za[u] ^ xb[u];
        Z(wb[u]) = zb[u] ^ xa[u];
      } else if constexpr (CODE == OP_CY) {
        X(wb[u]) = xb[u] ^ xa[u];
        Z(wb[u]) = zb[u] ^ xa[u];
        Z(wa[u]) = za[u] ^ xb[u] ^ zb[u];
      } else {   // SWAP
        X(wa[u]) = xb[u];
        Z(wa[u]) = zb[u];
        X(wb[u]) = xa[u];
        Z(wb[u]) = za[u];
      }
    }
  }
}

// Ring row of the measurement `back` measurements before the one at ring row
// `pos` (1 <= back < rows).
__device__ __forceinline__ uint32_t ring_back(uint32_t pos, uint32_t back, uint32_t rows) {
  return pos >= back ? pos - back : pos + rows - back;
}

// Detection events formed in the walk (Sec. 5.6): detector i of the op is the
// XOR of the flips its lookbacks name, read from the ring (written before the
// last full barrier), and goes straight to its row of det_out.  An item is a
// (detector, C words) pair; a thread takes up to U items at once and issues
// their loads together.  The op ends with no barrier: it writes nothing the
// team reads, and the ring rows it reads are not rewritten before the next
// measurement op's own barrier (the ring holds the longest lookback plus the
// largest measurement op).
template <int T, bool IN_LDS, bool WAVE>
__device__ __forceinline__ void detector_op(const FrameParams &p, const Tile<T, IN_LDS> &tl, const DevOp &op,
                                            const uint64_t *ring, uint32_t ring_pos, uint32_t det) {
  constexpr int U = 3;
  constexpr uint32_t C = T >= 2 ? 2 : 1;
  constexpr uint32_t CPT = T / C;
  typedef uint64_t U64x2v __attribute__((ext_vector_type(2)));
  typedef typename std::conditional<C == 2, U64x2v, uint64_t>::type Vec;
  const uint32_t c = op.aux;                       // lookbacks per detector, even
  const uint32_t items = op.n * CPT;
  const uint32_t *tg = p.targets + op.toff;
  const uint32_t R = p.ring_rows;
  const uint32_t tsize = team_size<WAVE>();
  for (uint32_t base = team_tid<WAVE>(); base < items; base += U * tsize) {
    uint32_t k[U], j[U];
    Vec acc[U];
#pragma unroll
    for (int u = 0; u < U; u++) {
      const uint32_t it = base + u * tsize;
      k[u] = it < items ? it / CPT : 0u;
      j[u] = (it % CPT) * C;
      acc[u] = Vec(0);
    }
    for (uint32_t r = 0; r < c; r += 2) {
      uint2 lb[U];
#pragma unroll
      for (int u = 0; u < U; u++) lb[u] = *reinterpret_cast<const uint2 *>(tg + (size_t)k[u] * c + r);
      // Every load is issued (a padding entry reads the row one back and its
      // value is dropped), so that they are all in flight at once.
      Vec va[U], vb[U];
#pragma unroll
      for (int u = 0; u < U; u++) {
        const uint32_t ra = ring_back(ring_pos, lb[u].x ? lb[u].x : 1u, R);
        const uint32_t rb = ring_back(ring_pos, lb[u].y ? lb[u].y : 1u, R);
        va[u] = *reinterpret_cast<const Vec *>(ring + ra * T + j[u]);
        vb[u] = *reinterpret_cast<const Vec *>(ring + rb * T + j[u]);
      }
#pragma unroll
      for (int u = 0; u < U; u++) {
        acc[u] ^= lb[u].x ? va[u] : Vec(0);
        acc[u] ^= lb[u].y ? vb[u] : Vec(0);
      }
    }
    // A whole pair goes out as one 16-byte store when rows start 16-byte
    // aligned (even row stride) and both words are in range: one memory
    // request per item.
    const bool whole = (p.out_stride & 1) == 0 && ((uintptr_t)p.det_out & 15) == 0;       // uniform
#pragma unroll
    for (int u = 0; u < U; u++) {
      const uint32_t it = base + u * tsize;
      if (it >= items) continue;
      uint64_t *dst = p.det_out + (uint64_t)(det + k[u]) * p.out_stride + tl.tw0 + j[u];
      if constexpr (C == 2) {
        if (whole && (int)j[u] + 1 < tl.valid) {
          *reinterpret_cast<Vec *>(dst) = acc[u];
        } else {
          if ((int)j[u] < tl.valid) dst[0] = acc[u][0];
          if ((int)j[u] + 1 < tl.valid) dst[1] = acc[u][1];
        }
      } else {
        if ((int)j[u] < tl.valid) dst[0] = acc[u];
      }
    }
  }
}

// Observable op: row op.aux of obs_out takes the XOR of the op's lookbacks.
// Item = (lookback, word); each wave XORs its items per word across lanes
// (lane l holds word l mod T, and T divides 64) and lanes 0 .. T-1 fold the
// result into the row with one atomic XOR per word: several waves, and later
// ops of the same observable, add to one word.
template <int T, bool IN_LDS, bool WAVE>
__device__ __forceinline__ void observable_op(const FrameParams &p, const Tile<T, IN_LDS> &tl, const DevOp &op,
                                              const uint64_t *ring, uint32_t ring_pos) {
  const uint32_t items = op.n * T;
  const uint32_t *tg = p.targets + op.toff;
  const uint32_t lane = threadIdx.x & 63;
  uint64_t *dst = p.obs_out + (size_t)op.aux * p.out_stride + tl.tw0;
  for (uint32_t base = team_tid<WAVE>() - lane; base < items; base += team_size<WAVE>()) {   // uniform per wave
    const uint32_t it = base + lane;
    uint64_t v = 0;
    if (it < items) v = ring[(size_t)ring_back(ring_pos, tg[it / T], p.ring_rows) * T + it % T];
#pragma unroll
    for (uint32_t d = T; d < 64; d <<= 1) v ^= shfl_xor64(v, (int)d);
    if (lane < (uint32_t)T && (int)lane < tl.valid) atomicXor((unsigned long long *)(dst + lane), (unsigned long long)v);
  }
}

// Classically controlled Pauli (Sec. 3, tracking corrections): for each pair
// (qubit, lookback k) and word of the tile, the shots whose result k
// measurements back differs from the reference's take the Pauli into their
// frame.  That difference is read back from the record this workgroup wrote
// (stored result XOR the reference bit): only this workgroup wrote those
// words, so a workgroup-scope barrier (release and acquire over all memory)
// and workgroup-scope loads make the stores of every wave visible.  A pair
// marked local (its result is a plain M of the same qubit, and nothing has
// acted on the qubit since) takes the difference from the qubit's own frame
// x bit instead: no barrier over memory and no load; an op whose pairs are
// all local needs neither.
template <int T, bool IN_LDS, bool WAVE, bool EVENTS>
__device__ __forceinline__ void feedback_op(const FrameParams &p, const Tile<T, IN_LDS> &tl, const DevOp &op,
                                            uint32_t code, uint64_t meas, const uint64_t *ring, uint32_t ring_pos) {
  if (!(op.code & OPF_FB_LOCAL)) team_barrier_all<WAVE>();
  const uint32_t items = op.n * T;
  const uint32_t *tg = p.targets + op.toff;
  for (uint32_t it = team_tid<WAVE>(); it < items; it += team_size<WAVE>()) {
    const uint32_t k = it / T;
    const int j = (int)(it % T);
    if (j >= tl.valid) continue;
    const uint32_t qw = tg[2 * k];
    const uint32_t q = qw & ~TGT_FB_LOCAL;
    const auto ix = tl.at(q, j);
    uint64_t f;
    if (qw & TGT_FB_LOCAL) {
      f = tl.FX[ix];                            // this item's own cell
    } else {
      const uint32_t back = tg[2 * k + 1];
      if constexpr (EVENTS) {      // raw flips
        f = __hip_atomic_load(ring + (size_t)ring_back(ring_pos, back, p.ring_rows) * T + j, __ATOMIC_RELAXED,
                              __HIP_MEMORY_SCOPE_WORKGROUP);
      } else {
        const uint64_t m = meas - back;
        f = __hip_atomic_load(p.out + m * p.out_stride + tl.tw0 + j, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        if (p.ref != nullptr && ((p.ref[m >> 6] >> (m & 63)) & 1)) f = ~f;
      }
    }
    if (code != OP_FB_Z) tl.FX[ix] ^= f;
    if (code != OP_FB_X) tl.FZ[ix] ^= f;
  }
}

// Applies precomputed noise records: each names a qubit (and partner), a word
// of the tile and up to five errors (6-bit position, 4-bit choice).
template <int T, bool IN_LDS>
__device__ __forceinline__ void apply_record(const Tile<T, IN_LDS> &tl, uint32_t code, int K, const uint4 r) {
  {
    const uint32_t qa = r.x & 0x7FFFFFFu, qb = r.y;
    const int j = (int)(r.x >> 27);
    const uint64_t h = (uint64_t)r.z | ((uint64_t)r.w << 32);
    uint64_t mk[4] = {0, 0, 0, 0};
    const int nh = (int)(h & 7);
    for (int i = 0; i < nh; i++)
      add_error(K, (int)((h >> (3 + 11 * i)) & 63), (uint32_t)((h >> (9 + 11 * i)) & 15), mk);
    // In LDS the XORs are atomics without return: no read-wait-write round
    // trip.
    auto flip = [&](uint64_t *w, uint64_t m) {
      if constexpr (IN_LDS) __hip_atomic_fetch_xor(w, m, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
      else *w ^= m;
    };
    if (code == OP_NOISE_DEP2) {
      flip(tl.FX + tl.at(qa, j), mk[0]);
      flip(tl.FZ + tl.at(qa, j), mk[1]);
      flip(tl.FX + tl.at(qb, j), mk[2]);
      flip(tl.FZ + tl.at(qb, j), mk[3]);
    } else {
      const uint64_t mx = code == OP_NOISE_DEP1 ? mk[0] : code != OP_NOISE_Z ? mk[0] : 0;
      const uint64_t mz = code == OP_NOISE_DEP1 ? mk[1] : code != OP_NOISE_X ? mk[0] : 0;
      flip(tl.FX + tl.at(qa, j), mx);
      flip(tl.FZ + tl.at(qa, j), mz);
    }
  }
}

// Records of one noise execution for this tile; the first two per thread may
// already be in registers (loaded one op earlier).
template <int T, bool IN_LDS, bool WAVE>
__device__ __forceinline__ void apply_records(const Tile<T, IN_LDS> &tl, uint32_t code, const uint4 *rec,
                                              uint32_t count, bool have, const uint4 &r0, const uint4 &r1) {
  const int K = code == OP_NOISE_DEP1 ? 3 : code == OP_NOISE_DEP2 ? 15 : 0;
  const uint32_t tsize = team_size<WAVE>();
  uint32_t e = team_tid<WAVE>();
  if (have) {
    if (e < count) apply_record(tl, code, K, r0);
    e += tsize;
    if (e < count) apply_record(tl, code, K, r1);
    e += tsize;
  }
  for (; e < count; e += tsize) apply_record(tl, code, K, rec[e]);
}

// Noise pre-pass: one workgroup per (noise execution, group of up to
// kGenTiles tiles).  The prefix test runs over all (32-slot group, word)
// candidates of the group's tiles, flattened so that the lanes stay busy;
// surviving (slot, word) pairs are queued in LDS per tile and then expanded
// into records, again flattened over the tiles.  If a tile's queue would
// exceed its reserved records (or its LDS queue), or one of its words holds
// more than five errors, its count is set to kNoRecords and the walker draws
// that op inline for that tile instead.
template <int T>
__global__ void __launch_bounds__(512) k_noise_gen(NoiseGenParams g) {
  extern __shared__ uint64_t queue[];            // [tiles of the group][g.queue_per_tile]
  __shared__ uint64_t thr[64];
  __shared__ uint32_t s_cnt[kGenTiles], s_bad[kGenTiles], s_off[kGenTiles + 1];
  const uint32_t inst = blockIdx.y;
  const uint32_t t0 = blockIdx.x * g.tiles_per_group;
  const uint32_t S = g.tiles - t0 < g.tiles_per_group ? g.tiles - t0 : g.tiles_per_group;
  uint2 *meta = g.meta + (size_t)t0 * g.tile_stride + (size_t)inst * g.inst_stride;   // entry t at meta[t * tile_stride]
  const uint32_t cap = g.cap[inst];
  const uint64_t base = g.base[inst];
  if (cap == 0) {
    if (threadIdx.x < S) meta[(size_t)threadIdx.x * g.tile_stride] = make_uint2(kNoRecords, 0u);
    return;
  }
  const DevOp op = g.ops[g.inst_pc[inst]];
  const uint32_t code = op.code & 0xFFFFu;
  const int K = code == OP_NOISE_DEP1 ? 3 : code == OP_NOISE_DEP2 ? 15 : 0;
  const uint64_t instr = g.inst_instr[inst];
  if (threadIdx.x < 64) thr[threadIdx.x] = g.thresholds[(size_t)op.aux * 64 + threadIdx.x];
  if (threadIdx.x < S) { s_cnt[threadIdx.x] = 0; s_bad[threadIdx.x] = 0; }
  __syncthreads();
  const uint64_t cut = thr[63] >> 56;
  const float p_est = (float)(0ull - thr[0]) * 0x1p-64f + (thr[0] == 0 ? 1.0f : 0.0f);
  const float inv_log2_keep = 1.0f / (log1pf(-p_est) * 1.44269504088896340736f);
  const uint32_t s_lo = op.slot0, s_hi = op.slot0 + op.n;
  const uint32_t g_lo = s_lo >> 5, ngroups = ((s_hi - 1) >> 5) - g_lo + 1;
  const uint32_t cand = ngroups * T;                 // candidates per tile
  const uint32_t qcap = cap < g.queue_per_tile ? cap : g.queue_per_tile;
  const uint32_t lane = threadIdx.x & 63;
  const uint32_t all_cand = S * cand;
  for (uint32_t c0 = 0; c0 < all_cand; c0 += blockDim.x) {       // uniform trip count
    const uint32_t c = c0 + threadIdx.x;
    const uint32_t ts = c / cand, cc = c % cand;
    const uint32_t grp = g_lo + cc / T;
    const int j = (int)(cc % T);
    const uint64_t tw0 = (uint64_t)(t0 + ts) * T;
    uint32_t mask = 0;
    U64x4 r{{0, 0, 0, 0}};
    if (c < all_cand && tw0 + j < g.num_words) {
      r = philox_call(instr, grp, g.word0 + tw0 + j, PURPOSE_NOISE_PREFIX << 32, g.seed);
      mask = prefix_pass_mask(r, cut) & group_slot_mask(grp, s_lo, s_hi);
    }
    // Queue positions: one LDS atomic per (wave, tile) present in the wave.
    bool pending = mask != 0;
    uint32_t idx = 0;
    while (true) {
      const uint64_t act = __ballot(pending);
      if (!act) break;
      const uint32_t s0 = __shfl(ts, __ffsll((unsigned long long)act) - 1, 64);
      const bool mine = pending && ts == s0;
      uint32_t wtotal;
      const uint32_t first = wave_exclusive_scan(mine ? (uint32_t)__builtin_popcount(mask) : 0u, lane, &wtotal);
      uint32_t wbase = 0;
      if (lane == 0) wbase = atomicAdd(&s_cnt[s0], wtotal);
      wbase = __shfl(wbase, 0, 64);
      if (mine) {
        idx = wbase + first;
        pending = false;
      }
    }
    uint64_t *q = queue + (size_t)ts * g.queue_per_tile;
    while (mask) {
      const uint32_t b = (uint32_t)__builtin_ctz(mask);
      mask &= mask - 1;
      if (idx < qcap) {
        const uint64_t vp = (r.v[b >> 3] >> (8 * (b & 7))) & 0xFF;
        q[idx] = ((uint64_t)(grp * 32 + b - s_lo) << 24) | ((uint64_t)j << 16) | vp;
      }
      idx++;
    }
  }
  __syncthreads();
  // Flatten the queues of the tiles that fit (a tile that overflows draws inline).
  if (threadIdx.x == 0) {
    uint32_t off = 0;
    for (uint32_t t = 0; t < S; t++) {
      s_off[t] = off;
      off += s_cnt[t] <= qcap ? s_cnt[t] : 0u;
    }
    s_off[S] = off;
  }
  __syncthreads();
  const uint32_t total = s_off[S];
  const uint32_t *tg = g.targets + op.toff;
  for (uint32_t e = threadIdx.x; e < total; e += blockDim.x) {
    uint32_t ts = 0;
    while (ts + 1 < S && s_off[ts + 1] <= e) ts++;
    const uint32_t le = e - s_off[ts];
    const uint64_t qe = queue[(size_t)ts * g.queue_per_tile + le];
    const uint32_t k = (uint32_t)(qe >> 24);
    const int j = (int)((qe >> 16) & 0xFF);
    const uint64_t tw0 = (uint64_t)(t0 + ts) * T;
    uint64_t packed = 0;
    int nh = 0;
    noise_walk(K, g.seed, instr, (uint64_t)s_lo + k, g.word0 + tw0 + j, thr, inv_log2_keep, qe & 0xFFFF,
               PhiloxCall(), [&](int pos, uint32_t ch) {
                 if (nh < 5) packed |= ((uint64_t)pos | ((uint64_t)ch << 6)) << (3 + 11 * nh);
                 nh++;
               });
    if (nh > 5) s_bad[ts] = 1;
    packed |= (uint64_t)(nh < 5 ? nh : 5);
    uint4 rec;
    rec.x = (code == OP_NOISE_DEP2 ? tg[2 * k] : tg[k]) | ((uint32_t)j << 27);
    rec.y = code == OP_NOISE_DEP2 ? tg[2 * k + 1] : 0u;
    rec.z = (uint32_t)packed;
    rec.w = (uint32_t)(packed >> 32);
    g.rec[base + (uint64_t)(t0 + ts) * cap + le] = rec;
  }
  __syncthreads();
  if (threadIdx.x < S) {
    const uint32_t t = threadIdx.x;
    const bool ok = s_cnt[t] <= qcap && !s_bad[t];
    meta[(size_t)t * g.tile_stride] = make_uint2(ok ? s_cnt[t] : kNoRecords, (uint32_t)(base + (uint64_t)(t0 + t) * cap));
  }
}

// One program entry, read through the constant address space: the kernel
// never writes the program, so these uniform loads become scalar loads.  A
// vector load would first wait (the vector memory counter completes in issue
// order) for every store and record prefetch still in flight.
__device__ __forceinline__ DevOp load_op(const DevOp *ops, uint32_t pc) {
  typedef __attribute__((address_space(4))) const uint32_t ConstU32;
  ConstU32 *w = (ConstU32 *)(ops + pc);
  DevOp op;
  op.code = w[0];
  op.lead = w[1];
  op.n = w[2];
  op.toff = w[3];
  op.slot0 = w[4];
  op.aux = w[5];
  op.aux2 = w[6];
  op.pad = w[7];
  return op;
}

// {count, first record} of a noise execution that has no records.
__device__ const uint32_t kNoMeta[2] = {kNoRecords, 0u};

// A meta entry, read as uniform scalar loads (the walk never writes it).
__device__ __forceinline__ uint2 load_meta(const uint32_t *w) {
  typedef __attribute__((address_space(4))) const uint32_t ConstU32;
  ConstU32 *c = (ConstU32 *)w;
  return make_uint2(c[0], c[1]);
}

// Walks the whole program over one tile.  `lds` is the workgroup's dynamic
// LDS: per-wave queues, one threshold row, then (IN_LDS) the frame slice.
// NOZ: the walk may run the program without Z randomisations, whose flags
// (an M that resets, an R it makes redundant, Cliffords on zero qubits) it
// then honours; the measurement-mode walk leaves that state out.
template <int T, bool IN_LDS, bool WAVE = false, bool EVENTS = false, bool NOZ = true>
__device__ __forceinline__ void walk_tile(const FrameParams &p, uint32_t tile, uint32_t slot, uint64_t *lds) {
  const uint32_t nwaves = WAVE ? 1u : blockDim.x >> 6;
  const uint32_t n = p.num_qubits;
  Tile<T, IN_LDS> tl;
  tl.queue = lds + (WAVE ? 0u : (threadIdx.x >> 6) * 64);
  uint64_t *thr_lds = lds + nwaves * 64;         // threshold row of the current noise op
  uint32_t thr_row = 0xFFFFFFFFu;
  uint64_t *F;
  if constexpr (IN_LDS) F = lds + nwaves * 64 + 64;
  else F = p.scratch + (size_t)slot * 2 * (n + 1) * T;
  tl.FX = F;
  // In LDS the X and Z planes are separate (fewer bank conflicts on the
  // strided target patterns); in global memory each qubit's X and Z words
  // are adjacent, so one cache line serves both.
  tl.FZ = IN_LDS ? F + (size_t)(n + 1) * T : F + T;
  tl.dummy = n;
  tl.tw0 = (uint64_t)tile * T;
  tl.valid = (int)((p.num_words - tl.tw0) < (uint64_t)T ? (p.num_words - tl.tw0) : (uint64_t)T);

  uint64_t flat = 0, meas = 0;
  // EVENTS: ring of recent flips (detection events formed in the walk);
  // ring_pos is the ring row of measurement `meas`, det the next detector.
  uint64_t *ring = EVENTS ? p.ring + (size_t)slot * p.ring_rows * T : nullptr;
  uint32_t ring_pos = 0, det = 0;
  if (EVENTS && p.obs_out && p.num_obs) {
    // Observable words start at zero; observable ops XOR into them atomically,
    // after the full barrier below.
    for (uint32_t i = team_tid<WAVE>(); i < p.num_obs * (uint32_t)T; i += team_size<WAVE>())
      if ((int)(i % T) < tl.valid) p.obs_out[(size_t)(i / T) * p.out_stride + tl.tw0 + i % T] = 0;
    team_barrier_all<WAVE>();
  }
  uint32_t loop_left[8];
  int depth = 0;
  uint32_t noise_seq = 0;
  uint32_t inner_left = 0;       // passes left of the innermost loop, this one included
  bool reset_done = false;       // the last collapse was an M that also did the next R
  // Two-stage prefetch of the next noise execution's records.  Stage A (at a
  // noise op) loads the next execution's {count, first record}: the same for
  // the whole workgroup, and never written by the walk, so a scalar load
  // through the constant address space (it then does not wait behind the
  // vector loads and stores in flight).  Stage B (in each following op, right
  // after that op's own loads) loads this thread's first two records with
  // vector loads issued on every path: a load issued on one path only makes
  // later waits conservative.
  const bool recs = p.noise_meta != nullptr;
  uint32_t a_inst = 0;
  uint2 a_meta = make_uint2(kNoRecords, 0u);
  auto stage_a = [&](uint32_t inst) {
    const bool ok = recs && inst < p.noise_instances;
    // Tile-major table for walks of the program without Z randomisations
    // (consecutive executions share scalar-cache lines), execution-major
    // otherwise: each layout measured faster for its walk.
    const size_t at = NOZ ? (size_t)tile * p.noise_instances + inst : (size_t)inst * p.noise_tiles + tile;
    const uint32_t *src = ok ? (const uint32_t *)(p.noise_meta + at) : kNoMeta;
    a_meta = load_meta(src);
    a_inst = ok ? inst : 0xFFFFFFFFu;
  };
  uint32_t pf_inst = 0xFFFFFFFFu, pf_count = kNoRecords;
  const uint4 *pf_rec = p.noise_rec;
  uint4 pf_r0 = make_uint4(0, 0, 0, 0), pf_r1 = make_uint4(0, 0, 0, 0);
  auto stage_b = [&]() {
    const uint32_t count = __builtin_amdgcn_readfirstlane(a_meta.x);
    const uint32_t first = __builtin_amdgcn_readfirstlane(a_meta.y);
    const bool ok = a_inst != 0xFFFFFFFFu && count != kNoRecords;
    pf_inst = a_inst;
    pf_count = ok ? count : kNoRecords;
    pf_rec = p.noise_rec + (ok ? first : 0u);
    const auto rs = buffer_rsrc(pf_rec, ok ? count * 16u : 0u);
    const auto v0 = __builtin_amdgcn_raw_buffer_load_b128(rs, team_tid<WAVE>() * 16u, 0, 0);
    const auto v1 = __builtin_amdgcn_raw_buffer_load_b128(rs, (team_tid<WAVE>() + team_size<WAVE>()) * 16u, 0, 0);
    pf_r0 = make_uint4(v0[0], v0[1], v0[2], v0[3]);
    pf_r1 = make_uint4(v1[0], v1[1], v1[2], v1[3]);
  };
  stage_a(0);
  for (uint32_t pc = 0; pc < p.num_ops; pc++) {
    const DevOp op = load_op(p.ops, pc);
    const uint32_t code = op.code & 0xFFFFu;

    if (code == OP_LOOP_BEGIN) {
      flat += op.lead;
      loop_left[depth++] = op.aux;
      if constexpr (NOZ) inner_left = op.aux;
      continue;
    }
    if (code == OP_LOOP_END) {
      flat += op.lead;
      if (--loop_left[depth - 1] > 0) pc = op.aux;    // back to the loop begin; body follows
      else depth--;
      if constexpr (NOZ) inner_left = depth > 0 ? loop_left[depth - 1] : 0u;
      continue;
    }
    if constexpr (EVENTS) {      // event ops (only in the events program): no flat index, no barrier
      if (code == OP_DET) {
        detector_op<T, IN_LDS, WAVE>(p, tl, op, ring, ring_pos, det);
        det += op.n;
        continue;
      }
      if (code == OP_OBS) {
        if (p.obs_out) observable_op<T, IN_LDS, WAVE>(p, tl, op, ring, ring_pos);
        continue;
      }
    }
    uint64_t instr;
    if (code == OP_INIT) {
      instr = INIT_INSTRUCTION;
    } else if (op.code & OPF_NEW_INSTR) {
      flat += op.lead;
      instr = flat++;
    } else {
      instr = flat - 1;
    }
    if (code == OP_INIT || code == OP_R || code == OP_M || code == OP_MR) {
      uint32_t eff = code;
      if constexpr (NOZ) {
        // An R that a reset M already did (uniform): nothing to do, no barrier.
        if (code == OP_R && reset_done && (op.code & OPF_R_AFTER_M)) {
          reset_done = false;
          continue;
        }
        reset_done = false;
        const bool resets =
            code == OP_M && ((op.code & OPF_M_RESETS) || ((op.code & OPF_M_RESETS_IN_LOOP) && inner_left > 1));
        if (resets) {
          reset_done = true;
          eff = OP_MR;
        }
      }
      collapse_op<T, IN_LDS, WAVE, EVENTS>(p, tl, op, eff, instr, meas, ring, ring_pos, stage_b);
    } else if (code >= OP_NOISE_X && code <= OP_NOISE_DEP2) {
      const uint32_t inst = noise_seq++;
      uint32_t count = kNoRecords;                 // same value in every thread
      const uint4 *rec = p.noise_rec;
      bool have = false;
      if (pf_inst == inst) {                       // records already in flight
        count = pf_count;
        rec = pf_rec;
        have = true;
      } else if (a_inst == inst) {                 // e.g. two noise ops in a row
        count = __builtin_amdgcn_readfirstlane(a_meta.x);
        rec = p.noise_rec + __builtin_amdgcn_readfirstlane(a_meta.y);
      }
      pf_inst = 0xFFFFFFFFu;
      stage_a(inst + 1);
      if (count != kNoRecords) {
        apply_records<T, IN_LDS, WAVE>(tl, code, rec, count, have, pf_r0, pf_r1);
      } else {
        if (op.aux != thr_row) {
          thr_row = op.aux;
          const uint32_t tt = team_tid<WAVE>();
          if (tt < 64) thr_lds[tt] = p.thresholds[(size_t)thr_row * 64 + tt];
          team_barrier<IN_LDS, WAVE>();
        }
        noise_op<T, IN_LDS, WAVE>(p, tl, op, code, instr, thr_lds);
      }
    } else if (code >= OP_FB_X) {
      feedback_op<T, IN_LDS, WAVE, EVENTS>(p, tl, op, code, meas, ring, ring_pos);
    } else {
      if constexpr (NOZ)
        if (op.code & OPF_ZERO_SKIP) continue;    // its qubits are zero in every shot: nothing changes
      switch (code) {
        case OP_SWAP_XZ: clifford_op<T, IN_LDS, WAVE, OP_SWAP_XZ>(p, tl, op, stage_b); break;
        case OP_Z_XOR_X: clifford_op<T, IN_LDS, WAVE, OP_Z_XOR_X>(p, tl, op, stage_b); break;
        case OP_X_XOR_Z: clifford_op<T, IN_LDS, WAVE, OP_X_XOR_Z>(p, tl, op, stage_b); break;
        case OP_CX: clifford_op<T, IN_LDS, WAVE, OP_CX>(p, tl, op, stage_b); break;
        case OP_CY: clifford_op<T, IN_LDS, WAVE, OP_CY>(p, tl, op, stage_b); break;
        case OP_CZ: clifford_op<T, IN_LDS, WAVE, OP_CZ>(p, tl, op, stage_b); break;
        default: clifford_op<T, IN_LDS, WAVE, OP_SWAP>(p, tl, op, stage_b); break;
      }
    }
    if (code == OP_M || code == OP_MR) {
      meas += op.n;
      if constexpr (EVENTS)
        ring_pos = ring_pos + op.n < p.ring_rows ? ring_pos + op.n : ring_pos + op.n - p.ring_rows;
    }
    // Flips in the ring are read back by other waves: a measurement's barrier
    // then covers global memory too.
    if (EVENTS && (code == OP_M || code == OP_MR)) team_barrier_all<WAVE>();
    else team_barrier<IN_LDS, WAVE>();
  }
}

// One workgroup per tile, or (a global frame) a smaller grid of workgroups
// that take tiles in turn, each reusing its own scratch slot, so that the
// frames in flight stay within the caches.
template <int T, bool IN_LDS, bool EVENTS, bool NOZ>
__global__ void __launch_bounds__(1024) k_frame(FrameParams p) {
  extern __shared__ uint64_t lds[];
  const uint32_t ntiles = (uint32_t)((p.num_words + T - 1) / T);
  const uint32_t first = xcd_tile(blockIdx.x, gridDim.x);
  for (uint32_t t = first; t < ntiles; t += gridDim.x)
    walk_tile<T, IN_LDS, false, EVENTS, NOZ>(p, t, blockIdx.x, lds);
}

// Persistent multi-circuit kernel: every workgroup pops (request, tile) items
// from a global counter until the list is exhausted, then exits.  Frames are
// LDS-resident; all requests of a launch share one tile width.
template <int T>
__global__ void __launch_bounds__(1024) k_batch(const FrameParams *__restrict__ reqs,
                                                const BatchItem *__restrict__ items, uint32_t num_items,
                                                uint32_t *counter) {
  extern __shared__ uint64_t lds[];
  __shared__ uint32_t s_item;
  while (true) {
    if (threadIdx.x == 0) s_item = atomicAdd(counter, 1u);
    tile_barrier<true>();
    const uint32_t it = __builtin_amdgcn_readfirstlane(s_item);
    tile_barrier<true>();
    if (it >= num_items) break;                  // uniform: every wave leaves together
    // The item and its request's parameters are uniform and never written
    // by the kernel: scalar loads through the constant address space keep
    // them in scalar registers (so the walk's own loads through them are
    // scalar too).
    typedef __attribute__((address_space(4))) const uint32_t ConstU32;
    static_assert(sizeof(BatchItem) % 4 == 0 && sizeof(FrameParams) % 4 == 0, "word copies");
    BatchItem bi;
    {
      ConstU32 *src = (ConstU32 *)(items + it);
      uint32_t w[sizeof(BatchItem) / 4];
#pragma unroll
      for (size_t k = 0; k < sizeof(BatchItem) / 4; k++) w[k] = src[k];
      __builtin_memcpy(&bi, w, sizeof bi);
    }
    FrameParams p;
    {
      ConstU32 *src = (ConstU32 *)(reqs + bi.req);
      uint32_t w[sizeof(FrameParams) / 4];
#pragma unroll
      for (size_t k = 0; k < sizeof(FrameParams) / 4; k++) w[k] = src[k];
      __builtin_memcpy(&p, w, sizeof p);
    }
    walk_tile<T, true>(p, bi.tile, 0, lds);
  }
}

// The same persistent walk with one wave per tile: each wave pops (request,
// tile) items on its own and walks them in its own LDS region (queue,
// threshold row, frame slice of `wave_words` words in all), synchronising with
// wave barriers only.  For small circuits, whose ops have few items, this
// keeps many tiles in flight per CU instead of idling most of a workgroup.
template <int T>
__global__ void __launch_bounds__(1024) k_batch_wave(const FrameParams *__restrict__ reqs,
                                                     const BatchItem *__restrict__ items, uint32_t num_items,
                                                     uint32_t *counter, uint32_t wave_words) {
  extern __shared__ uint64_t lds[];
  uint64_t *mine = lds + (size_t)(threadIdx.x >> 6) * wave_words;
  while (true) {
    uint32_t it = 0;
    if ((threadIdx.x & 63) == 0) it = atomicAdd(counter, 1u);
    it = __builtin_amdgcn_readfirstlane(it);       // lane 0's item for the whole wave
    if (it >= num_items) break;                    // uniform within the wave
    typedef __attribute__((address_space(4))) const uint32_t ConstU32;
    BatchItem bi;
    {
      ConstU32 *src = (ConstU32 *)(items + it);
      uint32_t w[sizeof(BatchItem) / 4];
#pragma unroll
      for (size_t k = 0; k < sizeof(BatchItem) / 4; k++) w[k] = src[k];
      __builtin_memcpy(&bi, w, sizeof bi);
    }
    FrameParams p;
    {
      ConstU32 *src = (ConstU32 *)(reqs + bi.req);
      uint32_t w[sizeof(FrameParams) / 4];
#pragma unroll
      for (size_t k = 0; k < sizeof(FrameParams) / 4; k++) w[k] = src[k];
      __builtin_memcpy(&p, w, sizeof p);
    }
    walk_tile<T, true, true>(p, bi.tile, 0, mine);
  }
}

__global__ void k_fill_u32(uint32_t *ptr, uint32_t value) { *ptr = value; }

// Detection events / observable flips: row r of `out` is the XOR of the flip
// rows listed in idx[off[r] .. off[r+1]) (Sec. 5.6).  A thread owns VEC
// adjacent words and walks `rows_per_block` rows in visiting order; the last
// two flip rows it loaded stay in registers, so a row shared by consecutive
// detectors of a chain is read from memory once.
template <int VEC>
__global__ void __launch_bounds__(256) k_parity(const uint64_t *__restrict__ flips, uint64_t W,
                                                 const uint32_t *__restrict__ off, const uint32_t *__restrict__ idx,
                                                 const uint32_t *__restrict__ order, uint32_t rows,
                                                 uint32_t rows_per_block, uint64_t *__restrict__ out) {
  typedef uint64_t V2 __attribute__((ext_vector_type(2)));
  typedef typename std::conditional<VEC == 2, V2, uint64_t>::type V;
  const uint64_t w = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) * VEC;
  if (w >= W) return;
  const uint32_t r0 = blockIdx.y * rows_per_block;
  const uint32_t r1 = rows - r0 < rows_per_block ? rows : r0 + rows_per_block;
  uint32_t ci0 = 0xFFFFFFFFu, ci1 = 0xFFFFFFFFu;
  V cv0 = V(0), cv1 = V(0);
  for (uint32_t i = r0; i < r1; i++) {
    const uint32_t r = order ? order[i] : i;
    V acc = V(0);
    for (uint32_t k = off[r]; k < off[r + 1]; k++) {
      const uint32_t m = idx[k];
      V v;
      if (m == ci0) {
        v = cv0;
      } else if (m == ci1) {
        v = cv1;
      } else {
        v = *reinterpret_cast<const V *>(flips + (uint64_t)m * W + w);
        ci1 = ci0;
        cv1 = cv0;
        ci0 = m;
        cv0 = v;
      }
      acc ^= v;
    }
    *reinterpret_cast<V *>(out + (uint64_t)r * W + w) = acc;
  }
}

// Detection events by blocks of the chained detector order (Sec. 5.6): a
// workgroup takes one block and VEC adjacent words per thread, issues the
// loads of all the block's flip rows (at most kDetBlockRows) before using any,
// then XORs each detector's rows from registers.  The block descriptor is
// uniform and never written, so it is read with scalar loads.  A block that is
// one detector with more rows goes through the CSR lists.
template <int VEC>
__global__ void __launch_bounds__(256) k_parity_blocks(const uint64_t *__restrict__ flips, uint64_t W,
                                                       const uint32_t *__restrict__ blocks, uint32_t xb,
                                                       const uint32_t *__restrict__ off,
                                                       const uint32_t *__restrict__ idx, uint64_t *__restrict__ out) {
  typedef uint64_t V2 __attribute__((ext_vector_type(2)));
  typedef typename std::conditional<VEC == 2, V2, uint64_t>::type V;
  typedef __attribute__((address_space(4))) const uint32_t ConstU32;
  const uint32_t blk = blockIdx.x / xb, xpart = blockIdx.x % xb;
  const uint64_t w = ((uint64_t)xpart * blockDim.x + threadIdx.x) * VEC;
  if (w >= W) return;
  ConstU32 *dsc = (ConstU32 *)(blocks + (size_t)blk * kDetBlockWords);
  const uint32_t head = dsc[0];
  if (head & kDetBlockCsr) {
    const uint32_t d = dsc[1];
    V acc = V(0);
    for (uint32_t k = off[d]; k < off[d + 1]; k++) acc ^= *reinterpret_cast<const V *>(flips + (uint64_t)idx[k] * W + w);
    *reinterpret_cast<V *>(out + (uint64_t)d * W + w) = acc;
    return;
  }
  const uint32_t ndet = head & 0xFFu, nrows = (head >> 8) & 0xFFu;
  V row[kDetBlockRows];
#pragma unroll
  for (uint32_t r = 0; r < kDetBlockRows; r++)
    row[r] = r < nrows ? *reinterpret_cast<const V *>(flips + (uint64_t)dsc[1 + r] * W + w) : V(0);
#pragma unroll
  for (uint32_t i = 0; i < kDetBlockDets; i++) {
    if (i >= ndet) break;
    const uint32_t mask = dsc[1 + kDetBlockRows + kDetBlockDets + i];
    V acc = V(0);
#pragma unroll
    for (uint32_t r = 0; r < kDetBlockRows; r++)
      if ((mask >> r) & 1u) acc ^= row[r];
    *reinterpret_cast<V *>(out + (uint64_t)dsc[1 + kDetBlockRows + i] * W + w) = acc;
  }
}

// ---------------------------------------------------------------------------
// Launchers.
// ---------------------------------------------------------------------------
size_t frame_lds_bytes(uint64_t n, int T, bool in_lds, uint32_t threads) {
  return ((size_t)(threads / 64) * 64 + 64) * sizeof(uint64_t) + (in_lds ? (size_t)16 * (n + 1) * T : 0);
}

template <int T, bool IN_LDS>
static hipError_t launch_frame_t(const FrameParams &p, uint32_t tiles, uint32_t threads, size_t lds_bytes,
                                 hipStream_t stream) {
  // One instantiation per mode, so that the measurement-mode walk carries
  // none of the ring's state, nor that of the program without Z
  // randomisations.
  const void *k = p.ring  ? (const void *)k_frame<T, IN_LDS, true, false>
                  : p.noz ? (const void *)k_frame<T, IN_LDS, false, true>
                          : (const void *)k_frame<T, IN_LDS, false, false>;
  hipError_t e = allow_dynamic_lds(k, (int)kMaxLdsBytes);
  if (e != hipSuccess) return e;
  if (p.ring)
    hipLaunchKernelGGL((k_frame<T, IN_LDS, true, false>), dim3(tiles), dim3(threads), lds_bytes, stream, p);
  else if (p.noz)
    hipLaunchKernelGGL((k_frame<T, IN_LDS, false, true>), dim3(tiles), dim3(threads), lds_bytes, stream, p);
  else
    hipLaunchKernelGGL((k_frame<T, IN_LDS, false, false>), dim3(tiles), dim3(threads), lds_bytes, stream, p);
  return hipGetLastError();
}

hipError_t launch_frame(const FrameParams &p, const FrameConfig &cfg, hipStream_t stream) {
  size_t lds = frame_lds_bytes(p.num_qubits, cfg.tile_words, cfg.in_lds, cfg.threads);
  if (lds > kMaxLdsBytes || cfg.threads % 64 || cfg.threads == 0 || cfg.threads > 1024) return hipErrorInvalidValue;
  uint32_t tiles = (uint32_t)((p.num_words + cfg.tile_words - 1) / cfg.tile_words);
  if (cfg.slots && cfg.slots < tiles) tiles = cfg.slots;      // workgroups of a global frame, or ring slots
#define STIM_CASE(TT)                                                                        \
  case TT:                                                                                   \
    return cfg.in_lds ? launch_frame_t<TT, true>(p, tiles, cfg.threads, lds, stream)         \
                      : launch_frame_t<TT, false>(p, tiles, cfg.threads, lds, stream);
  switch (cfg.tile_words) {
    STIM_CASE(1)
    STIM_CASE(2)
    STIM_CASE(4)
    STIM_CASE(8)
    STIM_CASE(16)
    STIM_CASE(32)
    default:
      return hipErrorInvalidValue;
  }
#undef STIM_CASE
}

template <int T>
static hipError_t launch_batch_t(const FrameParams *reqs, const BatchItem *items, uint32_t num_items,
                                 uint32_t *counter, uint32_t blocks, uint32_t threads, size_t lds, hipStream_t stream) {
  hipError_t e = allow_dynamic_lds((const void *)k_batch<T>, (int)(kMaxLdsBytes - kBatchStaticLds));
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(1), 0, stream, counter, 0u);
  hipLaunchKernelGGL((k_batch<T>), dim3(blocks), dim3(threads), lds, stream, reqs, items, num_items, counter);
  return hipGetLastError();
}

size_t wave_lds_bytes(uint64_t n, int T) { return ((size_t)64 + 64) * sizeof(uint64_t) + (size_t)16 * (n + 1) * T; }

uint32_t batch_waves_per_block(uint64_t n, int T) {
  const size_t per = wave_lds_bytes(n, T);
  const size_t w = per > kMaxLdsBytes ? 0 : kMaxLdsBytes / per;
  return (uint32_t)(w < 16 ? w : 16);
}

template <int T>
static hipError_t launch_batch_wave_t(const FrameParams *reqs, const BatchItem *items, uint32_t num_items,
                                      uint32_t *counter, uint32_t blocks, uint32_t waves, uint64_t n,
                                      hipStream_t stream) {
  hipError_t e = allow_dynamic_lds((const void *)k_batch_wave<T>, (int)kMaxLdsBytes);
  if (e != hipSuccess) return e;
  const uint32_t words = (uint32_t)(wave_lds_bytes(n, T) / sizeof(uint64_t));
  hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(1), 0, stream, counter, 0u);
  hipLaunchKernelGGL((k_batch_wave<T>), dim3(blocks), dim3(64 * waves), (size_t)waves * words * sizeof(uint64_t),
                     stream, reqs, items, num_items, counter, words);
  return hipGetLastError();
}

hipError_t launch_batch(const FrameParams *reqs, const BatchItem *items, uint32_t num_items, uint32_t *counter,
                        const FrameConfig &cfg, uint64_t max_qubits, uint32_t blocks, hipStream_t stream) {
  if (cfg.wave) {
    const uint32_t waves = batch_waves_per_block(max_qubits, cfg.tile_words);
    if (waves == 0 || wave_lds_bytes(max_qubits, cfg.tile_words) % 16) return hipErrorInvalidValue;
    switch (cfg.tile_words) {
      case 1: return launch_batch_wave_t<1>(reqs, items, num_items, counter, blocks, waves, max_qubits, stream);
      case 2: return launch_batch_wave_t<2>(reqs, items, num_items, counter, blocks, waves, max_qubits, stream);
      case 4: return launch_batch_wave_t<4>(reqs, items, num_items, counter, blocks, waves, max_qubits, stream);
      case 8: return launch_batch_wave_t<8>(reqs, items, num_items, counter, blocks, waves, max_qubits, stream);
      default: return hipErrorInvalidValue;
    }
  }
  size_t lds = frame_lds_bytes(max_qubits, cfg.tile_words, true, cfg.threads);
  if (lds + kBatchStaticLds > kMaxLdsBytes || cfg.threads % 64 || cfg.threads == 0 || cfg.threads > 1024)
    return hipErrorInvalidValue;
  switch (cfg.tile_words) {
    case 1: return launch_batch_t<1>(reqs, items, num_items, counter, blocks, cfg.threads, lds, stream);
    case 2: return launch_batch_t<2>(reqs, items, num_items, counter, blocks, cfg.threads, lds, stream);
    case 4: return launch_batch_t<4>(reqs, items, num_items, counter, blocks, cfg.threads, lds, stream);
    case 8: return launch_batch_t<8>(reqs, items, num_items, counter, blocks, cfg.threads, lds, stream);
    default: return hipErrorInvalidValue;
  }
}

int batch_blocks_per_cu(const FrameConfig &cfg, uint64_t max_qubits) {
  if (cfg.wave) return 1;                  // one block of up to 16 waves fills the LDS
  size_t lds = frame_lds_bytes(max_qubits, cfg.tile_words, true, cfg.threads) + kBatchStaticLds;
  int by_lds = (int)(kMaxLdsBytes / lds);
  int by_threads = 2048 / (int)cfg.threads;
  int b = by_lds < by_threads ? by_lds : by_threads;
  return b < 1 ? 1 : b;
}

hipError_t launch_noise_gen(const NoiseGenParams &g, int tile_words, uint32_t instances, uint32_t threads,
                            hipStream_t stream) {
  if (instances == 0 || g.tiles == 0) return hipSuccess;
  if (instances > 65535 || threads == 0 || threads % 64 || threads > 512 || g.tiles_per_group == 0 ||
      !((g.inst_stride == 1 && g.tile_stride >= instances) || (g.tile_stride == 1 && g.inst_stride >= g.tiles)) ||
      g.tiles_per_group > kGenTiles || g.queue_per_tile == 0 ||
      (size_t)g.tiles_per_group * g.queue_per_tile > kGenQueue)
    return hipErrorInvalidValue;
  dim3 grid((g.tiles + g.tiles_per_group - 1) / g.tiles_per_group, instances), block(threads);
  const size_t lds = (size_t)g.tiles_per_group * g.queue_per_tile * sizeof(uint64_t);
  switch (tile_words) {
    case 1: hipLaunchKernelGGL(k_noise_gen<1>, grid, block, lds, stream, g); break;
    case 2: hipLaunchKernelGGL(k_noise_gen<2>, grid, block, lds, stream, g); break;
    case 4: hipLaunchKernelGGL(k_noise_gen<4>, grid, block, lds, stream, g); break;
    case 8: hipLaunchKernelGGL(k_noise_gen<8>, grid, block, lds, stream, g); break;
    case 16: hipLaunchKernelGGL(k_noise_gen<16>, grid, block, lds, stream, g); break;
    case 32: hipLaunchKernelGGL(k_noise_gen<32>, grid, block, lds, stream, g); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_parity_blocks(const uint64_t *flips, uint64_t W, const uint32_t *blocks, uint64_t nblocks,
                                const uint32_t *off, const uint32_t *idx, uint64_t *out, hipStream_t stream) {
  if (nblocks == 0 || W == 0) return hipSuccess;
  const uint32_t threads = 256;
  const int vec = W % 2 == 0 && (uintptr_t)out % 16 == 0 && (uintptr_t)flips % 16 == 0 ? 2 : 1;
  const uint64_t xb = (W / vec + threads - 1) / threads;
  if (xb * nblocks > 0x7FFFFFFFull) return hipErrorInvalidValue;
  const dim3 grid((uint32_t)(xb * nblocks));
  if (vec == 2)
    hipLaunchKernelGGL(k_parity_blocks<2>, grid, dim3(threads), 0, stream, flips, W, blocks, (uint32_t)xb, off, idx,
                       out);
  else
    hipLaunchKernelGGL(k_parity_blocks<1>, grid, dim3(threads), 0, stream, flips, W, blocks, (uint32_t)xb, off, idx,
                       out);
  return hipGetLastError();
}

hipError_t launch_parity(const uint64_t *flips, uint64_t W, const uint32_t *off, const uint32_t *idx,
                         const uint32_t *order, uint32_t rows, uint64_t *out, hipStream_t stream) {
  if (rows == 0 || W == 0) return hipSuccess;
  const uint32_t threads = 256;
  const uint32_t rows_per_block = 8;
  // 16-byte accesses when every row of both arrays starts 16-byte aligned.
  const int vec = W % 2 == 0 && (uintptr_t)out % 16 == 0 && (uintptr_t)flips % 16 == 0 ? 2 : 1;
  const uint64_t xb = (W / vec + threads - 1) / threads;
  const uint64_t yb = (rows + rows_per_block - 1) / rows_per_block;
  if (xb > 0x7FFFFFFFull || yb > 65535) {
    // Very many rows: widen the row groups so that the grid's y extent fits.
    const uint64_t rpb = (rows + 65534) / 65535;
    if (xb > 0x7FFFFFFFull || rpb > 0xFFFFFFFFull) return hipErrorInvalidValue;
    const dim3 grid((uint32_t)xb, (uint32_t)((rows + rpb - 1) / rpb));
    if (vec == 2)
      hipLaunchKernelGGL(k_parity<2>, grid, dim3(threads), 0, stream, flips, W, off, idx, order, rows, (uint32_t)rpb, out);
    else
      hipLaunchKernelGGL(k_parity<1>, grid, dim3(threads), 0, stream, flips, W, off, idx, order, rows, (uint32_t)rpb, out);
    return hipGetLastError();
  }
  const dim3 grid((uint32_t)xb, (uint32_t)yb);
  if (vec == 2)
    hipLaunchKernelGGL(k_parity<2>, grid, dim3(threads), 0, stream, flips, W, off, idx, order, rows, rows_per_block, out);
  else
    hipLaunchKernelGGL(k_parity<1>, grid, dim3(threads), 0, stream, flips, W, off, idx, order, rows, rows_per_block, out);
  return hipGetLastError();
}

}  // namespace stimgpu
