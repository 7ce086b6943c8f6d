// Pauli-frame propagation kernels for gfx950 (Sec. 3, data layout of Sec. 5.1).
//
// One workgroup owns a tile of T consecutive 64-shot words and walks the whole
// device program over it.  Shots are independent, so tiles never communicate.
// Inside a workgroup the work of one op is spread over (target, word) items;
// an op's targets touch pairwise distinct qubits (the compiler splits
// instructions where a qubit repeats), so its items run in parallel and a
// barrier separates consecutive ops.
//
// The frame slice of a tile is two bit planes, X then Z, each [n][T] uint64
// (bit j of word w = shot 64 (tile word w) + j).  It lives in LDS when
// 16 n T bytes fit, otherwise in a global scratch buffer.
#include <hip/hip_runtime.h>

#include "circuit.h"
#include "frame_kernels.h"
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

template <int T, bool IN_LDS>
__global__ void __launch_bounds__(1024) k_frame(FrameParams p) {
  extern __shared__ uint64_t lds_frame[];
  const uint32_t tile = xcd_tile(blockIdx.x, gridDim.x);
  const uint64_t tw0 = (uint64_t)tile * T;                 // first local word of the tile
  const uint32_t n = p.num_qubits;
  uint64_t *F;
  if constexpr (IN_LDS) F = lds_frame;
  else F = p.scratch + (size_t)tile * 2 * n * T;
  uint64_t *FX = F, *FZ = F + (size_t)n * T;
  // Index of (qubit, word j) in a plane; 32-bit arithmetic suffices in LDS.
#define FI(q) (IN_LDS ? (size_t)((uint32_t)(q) * (uint32_t)T + (uint32_t)j) : (size_t)(q) * T + j)
  const int valid = (int)((p.num_words - tw0) < (uint64_t)T ? (p.num_words - tw0) : (uint64_t)T);

  uint64_t flat = 0, meas = 0;
  uint32_t loop_left[8];
  int depth = 0;
  for (uint32_t pc = 0; pc < p.num_ops; pc++) {
    const DevOp op = p.ops[pc];
    const uint32_t code = op.code & 0xFFFFu;
    if (code == OP_LOOP_BEGIN) {
      flat += op.lead;
      loop_left[depth++] = op.aux;
      continue;
    }
    if (code == OP_LOOP_END) {
      flat += op.lead;
      if (--loop_left[depth - 1] > 0) pc = op.aux;    // back to the loop begin; body follows
      else depth--;
      continue;
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
    const uint32_t *tg = p.targets + op.toff;
    const uint32_t items = op.n * T;
    for (uint32_t it = threadIdx.x; it < items; it += blockDim.x) {
      const uint32_t k = it / T;
      const int j = (int)(it % T);
      if (j >= valid) continue;
      const uint64_t word = p.word0 + tw0 + j;               // absolute 64-shot word
      const uint64_t slot = (uint64_t)op.slot0 + k;
      switch (code) {
        case OP_INIT: {
          uint32_t t = tg[k], q = t & TGT_QUBIT_MASK;
          FX[FI(q)] = 0;
          FZ[FI(q)] = (t & TGT_DEAD_ZRAND) ? 0 : zrand_word(p.seed, instr, q, word);
          break;
        }
        case OP_SWAP_XZ: {
          uint32_t q = tg[k];
          uint64_t x = FX[FI(q)];
          FX[FI(q)] = FZ[FI(q)];
          FZ[FI(q)] = x;
          break;
        }
        case OP_Z_XOR_X: {
          uint32_t q = tg[k];
          FZ[FI(q)] ^= FX[FI(q)];
          break;
        }
        case OP_X_XOR_Z: {
          uint32_t q = tg[k];
          FX[FI(q)] ^= FZ[FI(q)];
          break;
        }
        case OP_CX: {
          uint32_t c = tg[2 * k], t = tg[2 * k + 1];
          FX[FI(t)] ^= FX[FI(c)];
          FZ[FI(c)] ^= FZ[FI(t)];
          break;
        }
        case OP_CZ: {
          uint32_t a = tg[2 * k], b = tg[2 * k + 1];
          uint64_t xa = FX[FI(a)], xb = FX[FI(b)];
          FZ[FI(a)] ^= xb;
          FZ[FI(b)] ^= xa;
          break;
        }
        case OP_CY: {
          uint32_t c = tg[2 * k], t = tg[2 * k + 1];
          uint64_t xc = FX[FI(c)], xt = FX[FI(t)], zt = FZ[FI(t)];
          FX[FI(t)] = xt ^ xc;
          FZ[FI(t)] = zt ^ xc;
          FZ[FI(c)] ^= xt ^ zt;
          break;
        }
        case OP_SWAP: {
          uint32_t a = tg[2 * k], b = tg[2 * k + 1];
          uint64_t xa = FX[FI(a)], za = FZ[FI(a)];
          FX[FI(a)] = FX[FI(b)];
          FZ[FI(a)] = FZ[FI(b)];
          FX[FI(b)] = xa;
          FZ[FI(b)] = za;
          break;
        }
        case OP_R: {
          uint32_t t = tg[k], q = t & TGT_QUBIT_MASK;
          FX[FI(q)] = 0;
          FZ[FI(q)] = (t & TGT_DEAD_ZRAND) ? 0 : zrand_word(p.seed, instr, slot, word);
          break;
        }
        case OP_M:
        case OP_MR: {
          uint32_t t = tg[k], q = t & TGT_QUBIT_MASK;
          const uint64_t m = meas + k;
          uint64_t v = FX[FI(q)];
          if (p.ref && ((p.ref[m >> 6] >> (m & 63)) & 1)) v = ~v;
          if (tw0 + j == p.num_words - 1) v &= p.tail_mask;
          p.out[m * p.out_stride + tw0 + j] = v;
          if (code == OP_MR) {
            FX[FI(q)] = 0;
            FZ[FI(q)] = (t & TGT_DEAD_ZRAND) ? 0 : zrand_word(p.seed, instr, slot, word);
          } else if (!(t & TGT_DEAD_ZRAND)) {
            FZ[FI(q)] ^= zrand_word(p.seed, instr, slot, word);
          }
          break;
        }
        case OP_NOISE_X:
        case OP_NOISE_Y:
        case OP_NOISE_Z: {
          const uint64_t *thr = p.thresholds + (size_t)op.aux * 64;
          uint64_t v16 = noise_prefix16(p.seed, instr, slot, word);
          if (v16 < (thr[63] >> 48)) break;                   // no error in these 64 shots
          uint64_t m[4] = {0, 0, 0, 0};
          noise_masks<0>(p.seed, instr, slot, word, thr, v16, m);
          uint32_t q = tg[k];
          if (code != OP_NOISE_Z) FX[FI(q)] ^= m[0];
          if (code != OP_NOISE_X) FZ[FI(q)] ^= m[0];
          break;
        }
        case OP_NOISE_DEP1: {
          const uint64_t *thr = p.thresholds + (size_t)op.aux * 64;
          uint64_t v16 = noise_prefix16(p.seed, instr, slot, word);
          if (v16 < (thr[63] >> 48)) break;
          uint64_t m[4] = {0, 0, 0, 0};
          noise_masks<3>(p.seed, instr, slot, word, thr, v16, m);
          uint32_t q = tg[k];
          FX[FI(q)] ^= m[0];
          FZ[FI(q)] ^= m[1];
          break;
        }
        case OP_NOISE_DEP2: {
          const uint64_t *thr = p.thresholds + (size_t)op.aux * 64;
          uint64_t v16 = noise_prefix16(p.seed, instr, slot, word);
          if (v16 < (thr[63] >> 48)) break;
          uint64_t m[4] = {0, 0, 0, 0};
          noise_masks<15>(p.seed, instr, slot, word, thr, v16, m);
          uint32_t a = tg[2 * k], b = tg[2 * k + 1];
          FX[FI(a)] ^= m[0];
          FZ[FI(a)] ^= m[1];
          FX[FI(b)] ^= m[2];
          FZ[FI(b)] ^= m[3];
          break;
        }
        default:
          break;
      }
    }
    if (code == OP_M || code == OP_MR) meas += op.n;
    __syncthreads();
  }
}

#undef FI

// Detection events / observable flips: row r of `out` is the XOR of the flip
// rows listed in idx[off[r] .. off[r+1]) (Sec. 5.6).
__global__ void __launch_bounds__(256) k_parity(const uint64_t *__restrict__ flips, uint64_t W,
                                                 const uint32_t *__restrict__ off, const uint32_t *__restrict__ idx,
                                                 uint32_t rows, uint32_t blocks_per_row, uint64_t *__restrict__ out) {
  const uint32_t r = blockIdx.x / blocks_per_row;
  const uint64_t w = (uint64_t)(blockIdx.x % blocks_per_row) * blockDim.x + threadIdx.x;
  if (r >= rows || w >= W) return;
  uint64_t acc = 0;
  for (uint32_t k = off[r]; k < off[r + 1]; k++) acc ^= flips[(uint64_t)idx[k] * W + w];
  out[(uint64_t)r * W + w] = acc;
}

// ---------------------------------------------------------------------------
// Launchers.
// ---------------------------------------------------------------------------
template <int T, bool IN_LDS>
static hipError_t launch_frame_t(const FrameParams &p, uint32_t tiles, uint32_t threads, size_t lds_bytes,
                                 hipStream_t stream) {
  static bool attr_set = false;
  if (IN_LDS && !attr_set) {
    hipError_t e = hipFuncSetAttribute((const void *)k_frame<T, IN_LDS>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    if (e != hipSuccess) return e;
    attr_set = true;
  }
  hipLaunchKernelGGL((k_frame<T, IN_LDS>), dim3(tiles), dim3(threads), IN_LDS ? lds_bytes : 0, stream, p);
  return hipGetLastError();
}

hipError_t launch_frame(const FrameParams &p, const FrameConfig &cfg, hipStream_t stream) {
  size_t lds = (size_t)2 * p.num_qubits * cfg.tile_words * sizeof(uint64_t);
  uint32_t tiles = (uint32_t)((p.num_words + cfg.tile_words - 1) / cfg.tile_words);
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

hipError_t launch_parity(const uint64_t *flips, uint64_t W, const uint32_t *off, const uint32_t *idx,
                         uint32_t rows, uint64_t *out, hipStream_t stream) {
  if (rows == 0) return hipSuccess;
  const uint32_t threads = 256;
  uint32_t bpr = (uint32_t)((W + threads - 1) / threads);
  uint64_t blocks = (uint64_t)bpr * rows;
  if (blocks > 0x7FFFFFFFull) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_parity, dim3((uint32_t)blocks), dim3(threads), 0, stream, flips, W, off, idx, rows, bpr, out);
  return hipGetLastError();
}

}  // namespace stimgpu
