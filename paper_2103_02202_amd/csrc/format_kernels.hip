// Shot-major output formats (Sec. 5.11) from the sampler's measurement-major
// tables.
//
// A table is [rows][W] uint64 with bit j of word w = shot 64 w + j.  The
// formats are written per shot, so the first step transposes the table in
// 64 x 64 bit blocks into a shot-major scratch table
// T[shot][nchunks] (bit i of T[s][c] = row 64 c + i of shot s).  Dense formats
// (01, b8) then map T to the output byte by byte; sparse formats (hits, r8)
// take one wave per shot twice: once to measure each shot's output, and,
// after a prefix sum over the shots, once to write it.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

#include "bit_transpose.h"
#include "format_kernels.h"
#include "lds_attr.h"

namespace stimgpu {

namespace {

// Maps a workgroup index so that the workgroups of one XCD take consecutive
// blocks (the hardware deals workgroups round-robin over the 8 XCDs).
__device__ __forceinline__ uint32_t xcd_block(uint32_t bid, uint32_t nblocks) {
  const uint32_t X = 8;
  const uint32_t xcd = bid % X, local = bid / X;
  const uint32_t per = nblocks / X, rem = nblocks % X;
  return xcd * per + (xcd < rem ? xcd : rem) + local;
}

// One workgroup (1024 threads) per block of kTransposeChunks x 64 rows x 16
// words: coalesced 128-byte row segments into LDS, then each wave transposes
// the kTransposeChunks 64 x 64 blocks of one word column; each of the 1024
// shots' chunks form one contiguous piece of 8 kTransposeChunks bytes (T rows
// are padded to a multiple of kTransposeChunks chunks), staged in LDS and
// written by four consecutive lanes, so that a shot's piece covers whole
// 64-byte lines and a store instruction 16 of them.
// B8: instead of T, write the b8 bytes directly -- bytes [64 cg, 64 cg + 64)
// of shot s's row, clipped to its nbytes, at out + s nbytes (nbytes a
// multiple of 4, so every piece starts on a 4-byte boundary; other widths go
// through T and k_b8, since byte stores at unaligned piece ends cost more
// than the second pass).
constexpr uint32_t kTransposeChunks = 8;
constexpr size_t kTransposeLds = (size_t)kTransposeChunks * 64 * 17 * sizeof(uint64_t);

template <bool B8>
__global__ void __launch_bounds__(1024) k_transpose(const uint64_t *__restrict__ table, uint64_t rows, uint64_t W,
                                                    uint64_t shots, uint32_t nchunks, uint32_t tstride,
                                                    uint64_t *__restrict__ T, uint8_t *__restrict__ out,
                                                    uint64_t nbytes) {
  constexpr uint32_t NB = kTransposeChunks;
  extern __shared__ uint64_t tile_mem[];
  uint64_t(*tile)[17] = reinterpret_cast<uint64_t(*)[17]>(tile_mem);    // [NB * 64][17]
  const uint32_t ngroups = (nchunks + NB - 1) / NB;
  // Chunk-group-fastest order: workgroups on one XCD at the same time fill
  // neighbouring pieces of the same T rows.
  const uint32_t b = xcd_block(blockIdx.x, gridDim.x);
  const uint32_t cg = b % ngroups, wb = b / ngroups;
  const uint64_t w0 = (uint64_t)wb * 16;
  {
    const uint32_t rr = threadIdx.x >> 4, ww = threadIdx.x & 15;
    const uint64_t w = w0 + ww;
#pragma unroll
    for (uint32_t h = 0; h < NB; h++) {
      const uint64_t r = (uint64_t)cg * NB * 64 + h * 64 + rr;
      tile[h * 64 + rr][ww] = (r < rows && w < W) ? table[r * W + w] : 0;
    }
  }
  __syncthreads();
  const uint32_t lane = threadIdx.x & 63, k = threadIdx.x >> 6;
  typedef uint64_t V2 __attribute__((ext_vector_type(2)));
  uint64_t y[NB];
#pragma unroll
  for (uint32_t h = 0; h < NB; h++) y[h] = bit_transpose64(tile[h * 64 + lane][k], lane);
  // Stage each shot's 8 NB bytes shot-major in LDS (the input tile is no
  // longer needed; word h of local shot ls sits at ls NB + (h ^ (ls & 7)), a
  // swizzle that spreads a wave's writes over the banks), then write them
  // with four consecutive lanes per shot: a store instruction covers 16
  // whole 64-byte pieces instead of 64 scattered 16-byte ones.
  static_assert(NB == 8, "staging assumes 64-byte pieces");
  __syncthreads();
  uint64_t *stage = tile_mem;                                       // [1024 local shots][NB]
  {
    const uint32_t ls = k * 64 + lane;
#pragma unroll
    for (uint32_t h = 0; h < NB; h++) stage[ls * NB + (h ^ (ls & 7))] = y[h];
  }
  __syncthreads();
#pragma unroll
  for (uint32_t i = 0; i < 4; i++) {
    const uint32_t q = threadIdx.x + i * 1024, ls = q >> 2, part = q & 3;
    const uint64_t s = w0 * 64 + ls;
    if (s >= shots) continue;
    const uint64_t a = stage[ls * NB + ((2 * part) ^ (ls & 7))];
    const uint64_t b = stage[ls * NB + ((2 * part + 1) ^ (ls & 7))];
    if constexpr (B8) {
      typedef uint32_t U32x4a __attribute__((ext_vector_type(4), aligned(4)));
      const uint64_t off = (uint64_t)cg * NB * 8 + 16 * part;      // byte offset of the piece in row s
      if (off >= nbytes) continue;
      uint8_t *piece = out + s * nbytes + off;
      if (nbytes - off >= 16) {
        *reinterpret_cast<U32x4a *>(piece) = U32x4a{(uint32_t)a, (uint32_t)(a >> 32), (uint32_t)b, (uint32_t)(b >> 32)};
      } else {
        const uint32_t nw = (uint32_t)(nbytes - off) / 4;       // nbytes is a multiple of 4
        const uint32_t w[4] = {(uint32_t)a, (uint32_t)(a >> 32), (uint32_t)b, (uint32_t)(b >> 32)};
#pragma unroll
        for (uint32_t t = 0; t < 3; t++)
          if (t < nw) reinterpret_cast<uint32_t *>(piece)[t] = w[t];
      }
    } else {
      *reinterpret_cast<V2 *>(T + s * tstride + (uint64_t)cg * NB + 2 * part) = V2{a, b};
    }
  }
}

// b8: shot s's bytes are the first nbytes bytes of T[s] (T rows are
// little-endian bit strings), packed back to back.  A thread writes one
// aligned 16-byte piece of the output that lies inside row s, funnel-shifted
// out of five aligned 4-byte words of T (every word it reads starts inside
// the row's bytes, and T rows are padded to whole 64-byte chunks); the at
// most fifteen bytes at either end of a row that share a piece with the
// neighbouring row are written singly.
__global__ void __launch_bounds__(256) k_b8(const uint64_t *__restrict__ T, uint32_t tstride, uint64_t shots,
                                            uint64_t nbytes, uint8_t *__restrict__ out) {
  typedef uint32_t U32x4 __attribute__((ext_vector_type(4), aligned(4)));   // `out` is 4-byte aligned
  const uint32_t *src32 = reinterpret_cast<const uint32_t *>(T);
  const uint8_t *src8 = reinterpret_cast<const uint8_t *>(T);
  const uint64_t q = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;   // output piece within the row's span
  for (uint64_t s = blockIdx.y; s < shots; s += gridDim.y) {
    const uint64_t a0 = s * nbytes, a1 = a0 + nbytes;                    // row s occupies [a0, a1)
    const uint64_t first = (a0 + 15) / 16, last = a1 / 16;              // whole output pieces [first, last)
    const uint64_t tw = (uint64_t)s * tstride * 2;                       // row s in 32-bit words of T
    const uint64_t op = first + q;
    if (op < last) {
      const uint64_t b = op * 16 - a0;                                   // byte offset inside row s
      const uint32_t sh = (uint32_t)(b & 3) * 8;
      const uint32_t *w = src32 + tw + (b >> 2);
      const uint32_t w0 = w[0], w1 = w[1], w2 = w[2], w3 = w[3];
      U32x4 v;
      if (sh) {
        const uint32_t w4 = w[4];
        v = U32x4{(uint32_t)((((uint64_t)w1 << 32) | w0) >> sh), (uint32_t)((((uint64_t)w2 << 32) | w1) >> sh),
                  (uint32_t)((((uint64_t)w3 << 32) | w2) >> sh), (uint32_t)((((uint64_t)w4 << 32) | w3) >> sh)};
      } else {
        v = U32x4{w0, w1, w2, w3};
      }
      reinterpret_cast<U32x4 *>(out)[op] = v;
    }
    if (q < 16) {                                                        // ragged ends of the row
      const uint64_t head = first * 16 - a0 < nbytes ? first * 16 - a0 : nbytes;
      if (q < head) out[a0 + q] = src8[s * tstride * 8 + q];
      const uint64_t tail_start = last * 16 > a0 + head ? last * 16 : a0 + head;
      if (tail_start + q < a1) out[tail_start + q] = src8[s * tstride * 8 + (tail_start + q - a0)];
    }
  }
}

// 01: one character per row and a newline per shot.  A wave writes 512
// aligned 16-byte pieces of the output lying inside shot s's line, lane l the
// pieces l, l + 64, ..., l + 448 (each store instruction of the wave covers
// 1 KB in one run); a lane's eight pieces start 1,024 rows = sixteen words
// apart in the row, so they share one shift and one address computation.
// The pieces go out as non-temporal stores (7.7 GB of text at d = 49 and
// 65,536 shots, written once): measured 15 % faster than plain stores here,
// while the same hint slowed the b8 and transpose writers.  Each piece is sixteen characters from sixteen result bits;
// the piece holding the newline is written character by character, and the
// ragged ends -- at most fifteen bytes at each end of a line, which share a
// 16-byte piece with the neighbouring line -- are written singly.
__device__ __forceinline__ uint8_t char01(const uint64_t *row, uint64_t r, uint64_t rows) {
  return r < rows ? (uint8_t)('0' + ((row[r >> 6] >> (r & 63)) & 1)) : (uint8_t)'\n';
}

// Four result bits (bit k = character k) as four '0'/'1' bytes.
__device__ __forceinline__ uint32_t chars4(uint32_t b) {
  return 0x30303030u | (b & 1u) | (b & 2u) << 7 | (b & 4u) << 14 | (b & 8u) << 21;
}

__global__ void __launch_bounds__(256) k_01(const uint64_t *__restrict__ T, uint32_t tstride, uint64_t shots,
                                            uint64_t rows, uint8_t *__restrict__ out) {
  // Pieces are 16-byte aligned relative to `out`, which is 4-byte aligned.
  typedef uint32_t U32x4 __attribute__((ext_vector_type(4), aligned(4)));
  constexpr int S = 2;                                 // shots per iteration: their loads go out together
  constexpr int K = 8;                                 // pieces per lane, 64 pieces apart
  const uint64_t width = rows + 1;
  const uint64_t q = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const uint64_t p0 = (q >> 6) * (64 * K) + (q & 63);  // this lane's first piece, from the line's first
  for (uint64_t s0 = blockIdx.y; s0 < shots; s0 += (uint64_t)gridDim.y * S) {
    uint64_t lo[S][K], hi[S][K];
#pragma unroll
    for (int i = 0; i < S; i++) {
      const uint64_t s = s0 + (uint64_t)i * gridDim.y;
      const uint64_t a0 = s * width;
      const uint64_t r = ((a0 + 15) / 16 + p0) * 16 - a0;         // first row of piece k = 0
      const uint64_t *row = T + (s < shots ? s : 0) * tstride;
#pragma unroll
      for (int k = 0; k < K; k++) {
        const uint64_t rk = r + 1024 * k;
        const bool full = s < shots && rk + 16 <= rows;
        const uint64_t c = full ? rk >> 6 : 0;
        lo[i][k] = row[c];
        hi[i][k] = (full && (rk & 63) > 48) ? row[c + 1] : 0;
      }
    }
#pragma unroll
    for (int i = 0; i < S; i++) {
      const uint64_t s = s0 + (uint64_t)i * gridDim.y;
      if (s >= shots) break;
      const uint64_t *row = T + s * tstride;
      const uint64_t a0 = s * width, a1 = a0 + width;
      const uint64_t first = (a0 + 15) / 16, last = a1 / 16;     // whole 16-byte pieces [first, last)
      const uint64_t r = (first + p0) * 16 - a0;
      const uint32_t sh = (uint32_t)(r & 63);                    // the same for all K pieces
#pragma unroll
      for (int k = 0; k < K; k++) {
        const uint64_t ow = first + p0 + 64 * k;
        if (ow >= last) break;
        const uint64_t rk = r + 1024 * k;
        U32x4 v;
        if (rk + 16 <= rows) {
          uint64_t bits = lo[i][k] >> sh;
          if (sh > 48) bits |= hi[i][k] << (64 - sh);
          const uint32_t b = (uint32_t)bits;
          v = U32x4{chars4(b & 15u), chars4((b >> 4) & 15u), chars4((b >> 8) & 15u), chars4((b >> 12) & 15u)};
        } else {                                       // the piece holding the newline
          uint32_t w[4];
          for (uint32_t j = 0; j < 4; j++) {
            w[j] = 0;
            for (uint32_t b = 0; b < 4; b++) w[j] |= (uint32_t)char01(row, rk + 4 * j + b, rows) << (8 * b);
          }
          v = U32x4{w[0], w[1], w[2], w[3]};
        }
        __builtin_nontemporal_store(v, reinterpret_cast<U32x4 *>(out) + ow);
      }
      if (q < 16) {                                    // ragged ends of the line
        const uint64_t head = first * 16 - a0 < width ? first * 16 - a0 : width;
        if (q < head) out[a0 + q] = char01(row, q, rows);
        const uint64_t tail_start = last * 16 > a0 + head ? last * 16 : a0 + head;
        if (tail_start + q < a1) out[tail_start + q] = char01(row, tail_start + q - a0, rows);
      }
    }
  }
}

__device__ __forceinline__ uint32_t decimal_digits(uint32_t v) {
  return v < 10u ? 1 : v < 100u ? 2 : v < 1000u ? 3 : v < 10000u ? 4 : v < 100000u ? 5 : v < 1000000u ? 6
       : v < 10000000u ? 7 : v < 100000000u ? 8 : v < 1000000000u ? 9 : 10;
}

// Bytes of an r8 run of n zeros (n / 255 continuation bytes and the rest).
__device__ __forceinline__ uint64_t r8_bytes(uint64_t n) { return n / 255 + 1; }

// Exclusive sum over the lanes of a wave (32-bit); *total = the wave's sum.
__device__ __forceinline__ uint32_t wave_exclusive_sum(uint32_t v, uint32_t lane, uint32_t *total) {
  uint32_t x = v;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const uint32_t y = __shfl_up(x, d, 64);
    if (lane >= (uint32_t)d) x += y;
  }
  *total = __shfl(x, 63, 64);
  return x - v;
}

// Inclusive max over lanes 0..lane.
__device__ __forceinline__ uint32_t wave_inclusive_max(uint32_t v, uint32_t lane) {
  uint32_t x = v;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const uint32_t y = __shfl_up(x, d, 64);
    if (lane >= (uint32_t)d && y > x) x = y;
  }
  return x;
}

// Sparse formats, one wave per shot; chunk c of the shot goes to lane c % 64
// in round c / 64, so that each round's output is a contiguous, in-order
// piece.  WRITE = false: lens[s] = the shot's byte count; WRITE = true: the
// bytes, at out + offs[s].
// Set results of one round (64 chunks) a wave formats balanced over its lanes.
constexpr uint32_t kHitsBuffered = 1024;

template <bool R8, bool WRITE>
__global__ void __launch_bounds__(256) k_sparse(const uint64_t *__restrict__ T, uint32_t nchunks, uint32_t tstride,
                                                uint64_t shots, uint64_t rows, uint64_t *__restrict__ lens,
                                                const uint64_t *__restrict__ offs, uint8_t *__restrict__ out) {
  __shared__ uint32_t hit_list[R8 ? 1 : 4][R8 ? 1 : kHitsBuffered];   // hits: per wave, one round's results
  const uint32_t lane = threadIdx.x & 63;
  const uint64_t s = (uint64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (s >= shots) return;                          // whole waves leave together
  const uint64_t *row = T + s * tstride;
  uint64_t base = WRITE ? offs[s] : 0;             // output bytes so far
  // Set results are handled as index + 1 (0: none), in 32 bits (rows < 2^32).
  uint32_t prev1 = 0;                              // last set result before this round, + 1
  uint32_t nhits_before = 0;
  for (uint32_t c0 = 0; c0 < nchunks; c0 += 64) {
    const uint32_t c = c0 + lane;
    const uint64_t x = c < nchunks ? row[c] : 0;
    const uint32_t hit0 = c * 64;
    // The last set result before this lane's chunk (r8) or the number of set
    // results before it (hits: all but the first get a comma).
    uint32_t p1 = prev1, k = 0, hits_total = 0;
    if (R8) {
      const uint32_t last1 = x ? hit0 + 64 - (uint32_t)__builtin_clzll(x) : 0u;
      const uint32_t incl = wave_inclusive_max(last1 > prev1 ? last1 : prev1, lane);
      const uint32_t up = __shfl_up(incl, 1, 64);
      p1 = lane == 0 ? prev1 : up;
      prev1 = __shfl(incl, 63, 64);
    } else {
      k = wave_exclusive_sum((uint32_t)__builtin_popcountll(x), lane, &hits_total) + nhits_before;
      nhits_before += hits_total;
    }
    if (!R8 && hits_total <= kHitsBuffered) {        // uniform
      // hits, balanced over the lanes: the round's set results go to the
      // wave's LDS list in order, then lane l formats results l, l + 64, ...
      // (comma and decimal digits), so that no lane loops over a dense chunk
      // while the others wait.  (The same for r8, whose results mostly take
      // one byte each, was slower than its per-lane loop.)
      uint32_t *list = hit_list[threadIdx.x >> 6];
      {
        uint32_t r = k - (nhits_before - hits_total);     // this lane's first rank in the round
        for (uint64_t m = x; m; m &= m - 1) list[r++] = hit0 + (uint32_t)__builtin_ctzll(m);
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      const uint32_t first_rank = nhits_before - hits_total;   // results of the shot before this round
      for (uint32_t h0 = 0; h0 < hits_total; h0 += 64) {       // uniform
        const uint32_t h = h0 + lane;
        const bool valid = h < hits_total;
        const uint32_t i = valid ? list[h] : 0u;
        const bool comma = first_rank + h > 0;
        const uint32_t d = decimal_digits(i);
        uint32_t run;
        const uint32_t off = wave_exclusive_sum(valid ? d + (comma ? 1u : 0u) : 0u, lane, &run);
        if (WRITE && valid) {
          uint8_t *o = out + base + off;
          if (comma) *o++ = ',';
          uint32_t v = i;
          for (uint32_t q = d; q > 0; q--) {
            o[q - 1] = (uint8_t)('0' + v % 10u);
            v /= 10u;
          }
        }
        base += run;
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");   // the next round reuses the list
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      continue;
    }
    uint32_t n = 0;
    {
      uint32_t q1 = p1, kk = k;
      for (uint64_t m = x; m; m &= m - 1) {
        const uint32_t i = hit0 + (uint32_t)__builtin_ctzll(m);
        n += R8 ? (uint32_t)r8_bytes(i - q1) : decimal_digits(i) + (kk > 0 ? 1u : 0u);
        q1 = i + 1;
        kk++;
      }
    }
    uint32_t total;
    const uint32_t before = wave_exclusive_sum(n, lane, &total);
    if (WRITE && x) {
      uint8_t *o = out + base + before;
      uint32_t q1 = p1, kk = k;
      for (uint64_t m = x; m; m &= m - 1) {
        const uint32_t i = hit0 + (uint32_t)__builtin_ctzll(m);
        if (R8) {
          uint32_t run = i - q1;
          for (; run >= 255; run -= 255) *o++ = 255;
          *o++ = (uint8_t)run;
        } else {
          if (kk > 0) *o++ = ',';
          const uint32_t d = decimal_digits(i);
          uint32_t v = i;
          for (uint32_t q = d; q > 0; q--) {
            o[q - 1] = (uint8_t)('0' + v % 10u);
            v /= 10u;
          }
          o += d;
        }
        q1 = i + 1;
        kk++;
      }
    }
    base += total;
  }
  const int64_t prev = (int64_t)prev1 - 1;
  // Closing bytes: r8's run to the end of the shot; hits' newline.
  const uint64_t tail = R8 ? r8_bytes(rows - (uint64_t)(prev + 1)) : 1;
  (void)nhits_before;
  if (!WRITE) {
    if (lane == 0) lens[s] = base + tail;
  } else if (lane == 0) {
    if (R8) {
      uint64_t run = rows - (uint64_t)(prev + 1);
      uint8_t *o = out + base;
      for (; run >= 255; run -= 255) *o++ = 255;
      *o = (uint8_t)run;
    } else {
      out[base] = '\n';
    }
  }
}

// Exclusive prefix sum of n values in three steps: each block sums its
// contiguous segment; one block scans the block sums; each block scans its
// segment from its offset.  *total = the sum of all.
__device__ __forceinline__ uint64_t block_exclusive_scan(uint64_t v, uint64_t *tmp, uint64_t *total) {
  tmp[threadIdx.x] = v;
  __syncthreads();
  for (uint32_t d = 1; d < blockDim.x; d <<= 1) {
    const uint64_t y = threadIdx.x >= d ? tmp[threadIdx.x - d] : 0;
    __syncthreads();
    tmp[threadIdx.x] += y;
    __syncthreads();
  }
  const uint64_t incl = tmp[threadIdx.x];
  *total = tmp[blockDim.x - 1];
  __syncthreads();
  return incl - v;
}

__global__ void __launch_bounds__(256) k_scan_partial(const uint64_t *__restrict__ in, uint64_t n, uint64_t seg,
                                                      uint64_t *__restrict__ sums) {
  __shared__ uint64_t tmp[256];
  const uint64_t lo = blockIdx.x * seg, hi = lo + seg < n ? lo + seg : n;
  uint64_t v = 0;
  for (uint64_t i = lo + threadIdx.x; i < hi; i += blockDim.x) v += in[i];
  uint64_t total;
  block_exclusive_scan(v, tmp, &total);
  if (threadIdx.x == 0) sums[blockIdx.x] = total;
}

__global__ void __launch_bounds__(1024) k_scan_top(uint64_t *__restrict__ sums, uint32_t nblocks,
                                                   uint64_t *__restrict__ total) {
  __shared__ uint64_t tmp[1024];
  const uint64_t v = threadIdx.x < nblocks ? sums[threadIdx.x] : 0;
  uint64_t t;
  const uint64_t ex = block_exclusive_scan(v, tmp, &t);
  if (threadIdx.x < nblocks) sums[threadIdx.x] = ex;
  if (threadIdx.x == 0) *total = t;
}

__global__ void __launch_bounds__(256) k_scan_apply(const uint64_t *__restrict__ in, uint64_t n, uint64_t seg,
                                                    const uint64_t *__restrict__ sums, uint64_t *__restrict__ out) {
  __shared__ uint64_t tmp[256];
  const uint64_t lo = blockIdx.x * seg, hi = lo + seg < n ? lo + seg : n;
  uint64_t carry = sums[blockIdx.x];
  for (uint64_t b = lo; b < hi; b += blockDim.x) {
    const uint64_t i = b + threadIdx.x;
    const uint64_t v = i < hi ? in[i] : 0;
    uint64_t t;
    const uint64_t ex = block_exclusive_scan(v, tmp, &t);
    if (i < hi) out[i] = carry + ex;
    carry += t;
  }
}

}  // namespace

hipError_t launch_transpose(const uint64_t *table, uint64_t rows, uint64_t W, uint64_t shots, uint64_t *T,
                            hipStream_t stream) {
  const uint64_t nchunks = (rows + 63) / 64, ngroups = (nchunks + kTransposeChunks - 1) / kTransposeChunks;
  const uint64_t wblocks = (W + 15) / 16, blocks = ngroups * wblocks;
  if (blocks == 0) return hipSuccess;
  if (blocks > 0x7FFFFFFFull || nchunks > 0x3FFFFFFFull) return hipErrorInvalidValue;
  hipError_t e = allow_dynamic_lds((const void *)k_transpose<false>, (int)kTransposeLds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_transpose<false>, dim3((uint32_t)blocks), dim3(1024), kTransposeLds, stream, table, rows, W,
                     shots, (uint32_t)nchunks, (uint32_t)transpose_stride(rows), T, (uint8_t *)nullptr, (uint64_t)0);
  return hipGetLastError();
}

hipError_t launch_transpose_b8(const uint64_t *table, uint64_t rows, uint64_t W, uint64_t shots, uint8_t *out,
                               hipStream_t stream) {
  const uint64_t nchunks = (rows + 63) / 64, ngroups = (nchunks + kTransposeChunks - 1) / kTransposeChunks;
  const uint64_t wblocks = (W + 15) / 16, blocks = ngroups * wblocks, nbytes = (rows + 7) / 8;
  if (blocks == 0) return hipSuccess;
  if (blocks > 0x7FFFFFFFull || nchunks > 0x3FFFFFFFull || nbytes % 4 || (uintptr_t)out % 4)
    return hipErrorInvalidValue;
  hipError_t e = allow_dynamic_lds((const void *)k_transpose<true>, (int)kTransposeLds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_transpose<true>, dim3((uint32_t)blocks), dim3(1024), kTransposeLds, stream, table, rows, W,
                     shots, (uint32_t)nchunks, (uint32_t)transpose_stride(rows), (uint64_t *)nullptr, out, nbytes);
  return hipGetLastError();
}

hipError_t launch_dense_format(const uint64_t *T, uint64_t rows, uint64_t shots, int b8, uint8_t *out,
                               hipStream_t stream) {
  const uint64_t width = b8 ? (rows + 7) / 8 : rows + 1;
  // b8: a thread per 16-byte piece; 01: a wave per 512 16-byte pieces.
  const uint64_t xb = b8 ? (width / 16 + 1 + 255) / 256 : (((width / 16 + 1) + 511) / 512 * 64 + 255) / 256;
  if (shots == 0) return hipSuccess;
  if (xb > 0x7FFFFFFFull) return hipErrorInvalidValue;
  const uint32_t tstride = (uint32_t)transpose_stride(rows);
  // Each block walks many shots, so that a few thousand blocks cover the output.
  const uint64_t yb = std::max<uint64_t>(1, std::min<uint64_t>(shots, std::max<uint64_t>(1, 16384 / xb)));
  const dim3 grid((uint32_t)xb, (uint32_t)yb);
  if (b8)
    hipLaunchKernelGGL(k_b8, grid, dim3(256), 0, stream, T, tstride, shots, width, out);
  else
    hipLaunchKernelGGL(k_01, grid, dim3(256), 0, stream, T, tstride, shots, rows, out);
  return hipGetLastError();
}

hipError_t launch_sparse_format(const uint64_t *T, uint64_t rows, uint64_t shots, int r8, uint64_t *lens,
                                const uint64_t *offs, uint8_t *out, hipStream_t stream) {
  const uint64_t nchunks = (rows + 63) / 64;
  const uint64_t blocks = (shots + 3) / 4;
  if (blocks == 0) return hipSuccess;
  if (blocks > 0x7FFFFFFFull || nchunks > 0x3FFFFFFFull) return hipErrorInvalidValue;
  const uint32_t tstride = (uint32_t)transpose_stride(rows);
  const bool write = offs != nullptr;
  const dim3 grid((uint32_t)blocks), block(256);
  if (r8 && write)
    hipLaunchKernelGGL((k_sparse<true, true>), grid, block, 0, stream, T, (uint32_t)nchunks, tstride, shots, rows,
                       lens, offs, out);
  else if (r8)
    hipLaunchKernelGGL((k_sparse<true, false>), grid, block, 0, stream, T, (uint32_t)nchunks, tstride, shots, rows,
                       lens, offs, out);
  else if (write)
    hipLaunchKernelGGL((k_sparse<false, true>), grid, block, 0, stream, T, (uint32_t)nchunks, tstride, shots, rows,
                       lens, offs, out);
  else
    hipLaunchKernelGGL((k_sparse<false, false>), grid, block, 0, stream, T, (uint32_t)nchunks, tstride, shots, rows,
                       lens, offs, out);
  return hipGetLastError();
}

hipError_t launch_scan(const uint64_t *in, uint64_t n, uint64_t *out, uint64_t *sums, uint64_t *total,
                       hipStream_t stream) {
  if (n == 0) return hipSuccess;
  const uint32_t nblocks = (uint32_t)(n < kScanBlocks * 256ull ? (n + 255) / 256 : kScanBlocks);
  const uint64_t seg = (n + nblocks - 1) / nblocks;
  hipLaunchKernelGGL(k_scan_partial, dim3(nblocks), dim3(256), 0, stream, in, n, seg, sums);
  hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(1024), 0, stream, sums, nblocks, total);
  hipLaunchKernelGGL(k_scan_apply, dim3(nblocks), dim3(256), 0, stream, in, n, seg, sums, out);
  return hipGetLastError();
}

}  // namespace stimgpu
