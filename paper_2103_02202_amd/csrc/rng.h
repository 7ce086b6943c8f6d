// Counter-based random bits for the frame kernels.
//
// Generator: Philox4x64-10 (Salmon, Moraes, Dror, Shaw, "Parallel random
// numbers: as easy as 1, 2, 3", SC'11).  Key = (seed, KEY_HI).  Each call maps
// a 256-bit counter to four 64-bit outputs ("lanes").
//
// Counter layout for one random quantity:
//   c0 = flat instruction index (all ones for the initial frame randomisation)
//   c1 = target slot, or slot / 4 (Z randomisation), or slot / 32 (noise prefix)
//   c2 = absolute 64-shot word index (shot / 64)
//   c3 = purpose << 32 | call number
//
// Z randomisation after a collapse (Sec. 3): the 64 bits for (instr, slot,
// word) are lane slot % 4 of call (instr, slot / 4, word, 1 << 32).
//
// Pauli noise by geometric gaps (Sec. 5.5), per (instr, slot, word): a
// sequence of 64-bit draws d_0, d_1, ...; d_0's top 8 bits are byte slot % 32
// (bits 8 (k % 8) .. of lane k / 8) of call (instr, slot / 32, word, 2 << 32)
// and its low 56 bits come from lane 0 of call (instr, slot, word, 3 << 32);
// d_j (j >= 1) is lane j % 4 of call (instr, slot, word, 3 << 32 | j / 4).
// Starting at position 0, each gap draw u advances the position by
// G = #{g in 1..64 : u < t[g]}; a position below 64 is an error, followed (for
// depolarizing channels) by a choice draw c = floor(u K / 2^64), then the
// position steps past it.  Because the first draw's high bits come from a call
// shared by 32 slots, most words are proved error-free without evaluating the
// slot's own call.
#pragma once

#include <cstdint>

#if defined(__HIPCC__)
#define STIM_HD __host__ __device__ __forceinline__
#else
#define STIM_HD inline
#endif

namespace stimgpu {

constexpr uint64_t KEY_HI = 0x5354494D5F465241ull;
constexpr uint64_t PURPOSE_ZRAND = 1, PURPOSE_NOISE_PREFIX = 2, PURPOSE_NOISE_DETAIL = 3;
constexpr uint64_t INIT_INSTRUCTION = ~0ull;
constexpr uint64_t MASK56 = (1ull << 56) - 1;
// Slots sharing one noise-prefix call, and the width of each slot's prefix.
constexpr uint32_t PREFIX_SLOTS = 32, PREFIX_BITS = 8;

struct U64x4 { uint64_t v[4]; };

STIM_HD uint64_t mul_hi64(uint64_t a, uint64_t b) {
#if defined(__HIP_DEVICE_COMPILE__)
  return __umul64hi(a, b);
#else
  return (uint64_t)(((unsigned __int128)a * b) >> 64);
#endif
}

// Full 64 x 64 -> 128-bit product.  On the device it is built from four
// 32 x 32 + 64 multiply-adds (v_mad_u64_u32): the cross terms are folded into
// the running sums so that no intermediate overflows.
STIM_HD void mul_wide64(uint64_t m, uint64_t a, uint64_t &hi, uint64_t &lo) {
#if defined(__HIP_DEVICE_COMPILE__)
  const uint32_t ml = (uint32_t)m, mh = (uint32_t)(m >> 32);
  const uint32_t al = (uint32_t)a, ah = (uint32_t)(a >> 32);
  const uint64_t t0 = (uint64_t)al * ml;
  const uint64_t t1 = (uint64_t)al * mh + (t0 >> 32);
  const uint64_t t2 = (uint64_t)ah * ml + (uint32_t)t1;
  hi = (uint64_t)ah * mh + (t1 >> 32) + (t2 >> 32);
  lo = (t2 << 32) | (uint32_t)t0;
#else
  unsigned __int128 p = (unsigned __int128)m * a;
  hi = (uint64_t)(p >> 64);
  lo = (uint64_t)p;
#endif
}

STIM_HD U64x4 philox4x64_10(uint64_t c0, uint64_t c1, uint64_t c2, uint64_t c3, uint64_t k0, uint64_t k1) {
  const uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
  const uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
  for (int r = 0; r < 10; r++) {
    uint64_t lo0, hi0, lo1, hi1;
    mul_wide64(M0, c0, hi0, lo0);
    mul_wide64(M1, c2, hi1, lo1);
    uint64_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
    c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
    k0 += W0; k1 += W1;
  }
  return U64x4{{c0, c1, c2, c3}};
}

STIM_HD uint64_t lane_of(const U64x4 &r, uint32_t lane) {
  return lane == 0 ? r.v[0] : lane == 1 ? r.v[1] : lane == 2 ? r.v[2] : r.v[3];
}

STIM_HD uint64_t zrand_word(uint64_t seed, uint64_t instr, uint64_t slot, uint64_t word) {
  U64x4 r = philox4x64_10(instr, slot >> 2, word, PURPOSE_ZRAND << 32, seed, KEY_HI);
  return lane_of(r, (uint32_t)(slot & 3));
}

STIM_HD uint64_t noise_prefix(uint64_t seed, uint64_t instr, uint64_t slot, uint64_t word) {
  U64x4 r = philox4x64_10(instr, slot >> 5, word, PURPOSE_NOISE_PREFIX << 32, seed, KEY_HI);
  uint32_t k = (uint32_t)(slot & 31);
  return (lane_of(r, k >> 3) >> (8 * (k & 7))) & 0xFF;
}

// The 8-bit prefixes of one prefix call: bit k of the result is set when
// prefix k (byte k % 8 of lane k / 8, least significant byte first) is at
// least `cut` (0..255), i.e. when slot group position k may hold an error.
// Bytewise unsigned compare without per-byte loops: the low seven bits are
// compared with the byte's top bit forced on (no borrow leaves the byte),
// then the top bits decide where they differ.
STIM_HD uint32_t prefix_pass_mask(const U64x4 &r, uint64_t cut) {
  const uint64_t H = 0x8080808080808080ull, L = 0x7F7F7F7F7F7F7F7Full;
  const uint64_t y = cut * 0x0101010101010101ull;
  const uint64_t yh = y & H, yl = y & L;
  uint32_t out = 0;
#pragma unroll
  for (int i = 0; i < 4; i++) {
    const uint64_t x = r.v[i];
    const uint64_t xh = x & H;
    const uint64_t lo_ge = ((x & L) | H) - yl;                // bit 7 of a byte: low 7 bits x >= y
    const uint64_t ge = ((xh & ~yh) | (~(xh ^ yh) & lo_ge)) & H;
    // Gather the eight top bits into one byte.
    out |= (uint32_t)(((ge >> 7) * 0x0102040810204080ull) >> 56) << (8 * i);
  }
  return out;
}

// Bits [lo - 32 g, hi - 32 g) of a 32-slot group g: the group's slots that
// belong to the slot range [lo, hi).
STIM_HD uint32_t group_slot_mask(uint32_t g, uint32_t lo, uint32_t hi) {
  const int64_t a = (int64_t)lo - 32 * (int64_t)g, b = (int64_t)hi - 32 * (int64_t)g;
  const int64_t a0 = a < 0 ? 0 : a, b0 = b > 32 ? 32 : b;
  if (b0 <= a0) return 0u;
  const uint64_t bits = ((1ull << (b0 - a0)) - 1) << a0;
  return (uint32_t)bits;
}

// G = #{g in 1..64 : u < t[g-1]} for non-increasing t.
STIM_HD int gap_length(uint64_t u, const uint64_t *t) {
  int lo = 0, hi = 64;
  while (lo < hi) {
    int mid = (lo + hi) >> 1;
    if (u < t[mid]) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}

// The same G, starting from the estimate floor(log(u / 2^64) / log(1 - p))
// (inv_log2_keep = 1 / log2(1 - p)) and then moving to the exact answer with
// integer comparisons, so the result never depends on floating-point rounding.
STIM_HD int gap_length_from_guess(uint64_t u, const uint64_t *t, float inv_log2_keep) {
  float x = (float)(u >> 40) * 0x1p-24f + 0x1p-25f;      // u / 2^64, never 0
  float est = log2f(x) * inv_log2_keep;
  int g = est >= 64.0f ? 64 : est <= 0.0f ? 0 : (int)est;
  while (g > 0 && u >= t[g - 1]) g--;
  while (g < 64 && u < t[g]) g++;
  return g;
}

// Walks the errors of one noise site on one word (geometric gaps, Sec. 5.5):
// calls on_hit(position, choice) for each error in increasing position
// (choice = floor(u K / 2^64) from the draw after the gap, K = 0: no choice).
// philox(c0, c1, c2, c3, seed) evaluates one generator call; vp is the
// site's 8-bit prefix; inv_log2_keep = 1 / log2(1 - p) seeds the gap search.
// With max_draws set, the walk stops (returning false) instead of taking draw
// number max_draws; errors reported before that point are then incomplete.
template <typename Philox, typename OnHit>
STIM_HD bool noise_walk(int K, uint64_t seed, uint64_t instr, uint64_t slot, uint64_t word, const uint64_t *t,
                        float inv_log2_keep, uint64_t vp, Philox philox, OnHit on_hit,
                        uint32_t max_draws = 0xFFFFFFFFu) {
  // Four draws per call, kept in named registers (no indexed local array).
  uint64_t b0 = 0, b1 = 0, b2 = 0, b3 = 0;
  uint32_t j = 0;
  auto draw = [&]() -> uint64_t {
    uint32_t lane = j & 3;
    if (lane == 0) {
      U64x4 r = philox(instr, slot, word, (PURPOSE_NOISE_DETAIL << 32) | (j >> 2), seed);
      b0 = r.v[0]; b1 = r.v[1]; b2 = r.v[2]; b3 = r.v[3];
    }
    j++;
    return lane == 0 ? b0 : lane == 1 ? b1 : lane == 2 ? b2 : b3;
  };
  uint64_t u = (vp << 56) | (draw() & MASK56);
  int pos = 0;
  while (true) {
    pos += gap_length_from_guess(u, t, inv_log2_keep);
    if (pos >= 64) break;
    if (K && j >= max_draws) return false;
    uint32_t c = K ? (uint32_t)mul_hi64(draw(), (uint64_t)K) : 0u;
    on_hit(pos, c);
    if (++pos >= 64) break;
    if (j >= max_draws) return false;
    u = draw();
  }
  return true;
}

// Flip masks of one error: K = 0 single mask in m[0]; K = 3 (DEPOLARIZE1)
// m[0] = x, m[1] = z for choice 0 X, 1 Y, 2 Z; K = 15 (DEPOLARIZE2) m[0..3] =
// x_a, z_a, x_b, z_b from the bits of choice + 1.
STIM_HD void add_error(int K, int pos, uint32_t c, uint64_t m[4]) {
  uint64_t bit = 1ull << pos;
  if (K == 0) {
    m[0] |= bit;
  } else if (K == 3) {
    if (c <= 1) m[0] |= bit;
    if (c >= 1) m[1] |= bit;
  } else {
    uint32_t v = c + 1;
    if (v & 1) m[0] |= bit;
    if (v & 2) m[1] |= bit;
    if (v & 4) m[2] |= bit;
    if (v & 8) m[3] |= bit;
  }
}

// Error masks of one noise site on one word (see add_error for m).
template <typename Philox>
STIM_HD void noise_masks(int K, uint64_t seed, uint64_t instr, uint64_t slot, uint64_t word, const uint64_t *t,
                         float inv_log2_keep, uint64_t vp, uint64_t m[4], Philox philox) {
  noise_walk(K, seed, instr, slot, word, t, inv_log2_keep, vp, philox,
             [&](int pos, uint32_t c) { add_error(K, pos, c, m); });
}

}  // namespace stimgpu
