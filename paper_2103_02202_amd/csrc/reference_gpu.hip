// Canonical reference sample on the GPU: the inverse-tableau simulation of
// Sec. 4 with the tableau resident in device memory.
//
// The tableau T maps an observable at the current time to the equivalent one
// at the start of time (all qubits |0>).  It is stored by columns (Sec. 5.1):
// column c < n is T(X_c), column n + q is T(Z_q); each column holds n x bits
// and n z bits in 64-bit words, plus a sign.  The work is organised so that
// the parallel parts run wide and only the inherently ordered part runs in
// one workgroup:
//
//   * a Clifford layer (the targets of one instruction, split where a qubit
//     repeats) prepends its gate's inverse to the columns of each target's
//     qubits: one wave per target, word-parallel column products whose phase
//     is reduced across the wave (Sec. 2.3.2);
//   * a measurement layer first reads, one wave per target, every result that
//     is already deterministic (the Z column has no X or Y term; its sign is
//     the result) -- measuring a deterministic observable commutes with the
//     other collapses of the layer, and a deterministic observable stays
//     deterministic;
//   * then one workgroup walks the layer's remaining targets in order: a
//     target that is still random is collapsed to 0 by inserting operations
//     at the start of time ("appends": CNOTs from a pivot onto the column's
//     other X/Y terms, H or H_YZ on the pivot, X when the sign must flip),
//     each of which touches every column, spread over the workgroup's
//     threads.
//
// Classically controlled Paulis are prepended when the reference's own
// result is 1.  The canonical rule (every random result is 0) makes the
// sample unique, so it is identical to the host computation's.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <string>
#include <unordered_map>
#include <vector>

#include "bit_transpose.h"
#include "circuit.h"
#include "format_kernels.h"
#include "reference_gpu.h"
#include "stim_gpu.h"

namespace stimgpu {

namespace {

struct Tab {
  uint64_t *xb, *zb;     // by columns: [2n][nwp]
  uint32_t *sb;          // signs, one bit per column (also read as 64-bit words)
  uint32_t n, nw, nwp;   // qubits, words per column, column stride
};

enum StepKind : uint8_t { STEP_PREPEND, STEP_MEASURE, STEP_FEEDBACK };

struct Step {
  StepKind kind;
  Gate gate;             // Clifford / R / M / MR; feedback: the controlled gate (CX, CY, CZ)
  uint32_t toff, count;  // targets (pairs for two-qubit gates and feedback)
  uint64_t meas0;        // measurements before the step
};

__device__ __forceinline__ int wave_sum(int v) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
  return v;
}

__device__ __forceinline__ uint32_t sign_of(const Tab &t, uint32_t c) { return (t.sb[c >> 5] >> (c & 31)) & 1u; }

// Sign bits of different columns share words: updates are atomic.
__device__ __forceinline__ void sign_xor(const Tab &t, uint32_t c, uint32_t v) {
  if (v) atomicXor(t.sb + (c >> 5), 1u << (c & 31));
}

__device__ __forceinline__ void wave_swap_cols(const Tab &t, uint32_t a, uint32_t b, uint32_t lane) {
  uint64_t *xa = t.xb + (size_t)a * t.nwp, *xb = t.xb + (size_t)b * t.nwp;
  uint64_t *za = t.zb + (size_t)a * t.nwp, *zb = t.zb + (size_t)b * t.nwp;
  for (uint32_t w = lane; w < t.nw; w += 64) {
    const uint64_t x = xa[w], z = za[w];
    xa[w] = xb[w];
    za[w] = zb[w];
    xb[w] = x;
    zb[w] = z;
  }
  if (lane == 0) {
    const uint32_t d = sign_of(t, a) ^ sign_of(t, b);
    sign_xor(t, a, d);
    sign_xor(t, b, d);
  }
}

// Column dst <- i^e * dst * src.  For Hermitian single-qubit Paulis written
// as i^(x z) X^x Z^z, the product's phase exponent is the sum over qubits of
// x1 z1 + x2 z2 + 2 z1 x2 - x3 z3; it must be even (a real sign).
__device__ __forceinline__ void wave_mul_cols(const Tab &t, uint32_t dst, uint32_t src, int e, uint32_t lane) {
  uint64_t *x1 = t.xb + (size_t)dst * t.nwp, *z1 = t.zb + (size_t)dst * t.nwp;
  const uint64_t *x2 = t.xb + (size_t)src * t.nwp, *z2 = t.zb + (size_t)src * t.nwp;
  int acc = 0;
  for (uint32_t w = lane; w < t.nw; w += 64) {
    const uint64_t a = x1[w], b = z1[w], c = x2[w], d = z2[w];
    const uint64_t x3 = a ^ c, z3 = b ^ d;
    acc += __popcll(a & b) + __popcll(c & d) + 2 * __popcll(b & c) - __popcll(x3 & z3);
    x1[w] = x3;
    z1[w] = z3;
  }
  acc = wave_sum(acc) + e;
  if (lane == 0) sign_xor(t, dst, sign_of(t, src) ^ (uint32_t)((acc >> 1) & 1));
}

__device__ __forceinline__ void flip_sign(const Tab &t, uint32_t col, uint32_t lane) {
  if (lane == 0) sign_xor(t, col, 1u);
}

// Prepends the inverse of `gate` (T'(g) = T(G^dagger g G)), one wave per
// target; the targets of a step touch distinct qubits.
__global__ void __launch_bounds__(256) k_ref_prepend(Tab t, Gate gate, const uint32_t *tg, uint32_t count) {
  const uint32_t lane = threadIdx.x & 63;
  const uint32_t k = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  if (k >= count) return;
  const bool two = gate == G_CX || gate == G_CY || gate == G_CZ || gate == G_SWAP;
  const uint32_t a = two ? tg[2 * k] : tg[k], b = two ? tg[2 * k + 1] : a;
  const uint32_t n = t.n, Xa = a, Za = n + a, Xb = b, Zb = n + b;
  switch (gate) {
    case G_X: flip_sign(t, Za, lane); break;
    case G_Y: flip_sign(t, Xa, lane); flip_sign(t, Za, lane); break;
    case G_Z: flip_sign(t, Xa, lane); break;
    case G_H: wave_swap_cols(t, Xa, Za, lane); break;
    case G_S: wave_mul_cols(t, Xa, Za, 3, lane); break;
    case G_S_DAG: wave_mul_cols(t, Xa, Za, 1, lane); break;
    case G_SQRT_X: wave_mul_cols(t, Za, Xa, 3, lane); break;
    case G_SQRT_X_DAG: wave_mul_cols(t, Za, Xa, 1, lane); break;
    case G_SQRT_Y: wave_swap_cols(t, Xa, Za, lane); flip_sign(t, Za, lane); break;
    case G_SQRT_Y_DAG: wave_swap_cols(t, Xa, Za, lane); flip_sign(t, Xa, lane); break;
    case G_H_XY: wave_mul_cols(t, Xa, Za, 1, lane); flip_sign(t, Za, lane); break;
    case G_H_YZ: wave_mul_cols(t, Za, Xa, 3, lane); flip_sign(t, Xa, lane); break;
    case G_CX: wave_mul_cols(t, Xa, Xb, 0, lane); wave_mul_cols(t, Zb, Za, 0, lane); break;
    case G_CZ: wave_mul_cols(t, Xa, Zb, 0, lane); wave_mul_cols(t, Xb, Za, 0, lane); break;
    case G_CY:
      wave_mul_cols(t, Xa, Xb, 0, lane);
      wave_mul_cols(t, Xa, Zb, 1, lane);
      wave_mul_cols(t, Xb, Za, 0, lane);
      wave_mul_cols(t, Zb, Za, 0, lane);
      break;
    case G_SWAP: wave_swap_cols(t, Xa, Xb, lane); wave_swap_cols(t, Za, Zb, lane); break;
    default: break;
  }
}

__device__ __forceinline__ void set_ref_bit(uint64_t *ref, uint64_t m) {
  __hip_atomic_fetch_or(ref + (m >> 6), 1ull << (m & 63), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Deterministic results of a measurement step, one wave per target; random
// targets are flagged for the ordered pass and counted in *random.
__global__ void __launch_bounds__(256) k_ref_measure_det(Tab t, Gate gate, const uint32_t *tg, uint32_t count,
                                                         uint64_t meas0, uint64_t *ref, uint32_t *flag,
                                                         uint32_t *random) {
  const uint32_t lane = threadIdx.x & 63;
  const uint32_t k = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  if (k >= count) return;
  const uint32_t c = t.n + (tg[k] & TGT_QUBIT_MASK);
  bool any = false;
  for (uint32_t w = lane; w < t.nw; w += 64) any |= t.xb[(size_t)c * t.nwp + w] != 0;
  any = __any(any);
  if (lane == 0) {
    flag[k] = any ? 1u : 0u;
    if (any) {
      atomicAdd(random, 1u);
    } else {
      const uint32_t r = sign_of(t, c);
      if (gate != G_R && r) set_ref_bit(ref, meas0 + k);
      if (gate != G_M) sign_xor(t, c, r);      // reset: force the sign to +
    }
  }
}

constexpr uint32_t kRefThreads = 1024;
constexpr uint32_t kRefList = 8192;          // support rows gathered per round

// The ordered pass over a measurement step's random targets, one workgroup,
// on the transposed tableau: XR[cw * n + j] / ZR[cw * n + j] hold, for qubit
// j, the x / z bits of columns 64 cw .. 64 cw + 63, and SB the column signs.
// Appending a gate at the start of time is then a few word-parallel row
// operations (the reason the paper transposes for bursts of random
// measurements).  Words of one column group are contiguous over the qubits,
// so the scan of a column for its pivot and support reads consecutive words;
// a row operation touches one word per column group.
__global__ void __launch_bounds__(kRefThreads) k_ref_collapse_rows(uint64_t *XR, uint64_t *ZR, uint64_t *SB,
                                                                    uint32_t n, Gate gate,
                                                                    const uint32_t *tg, uint32_t count, uint64_t meas0,
                                                                    uint64_t *ref, const uint32_t *flag) {
  __shared__ uint32_t list[kRefList];
  __shared__ uint32_t s_flag[kRefThreads * 4];
  __shared__ uint32_t s_pivot, s_cnt, s_bit, s_more;
  const uint32_t tid = threadIdx.x, words = (2 * n + 63) / 64;
  for (uint32_t k = 0; k < count; k++) {
    if (k % (kRefThreads * 4) == 0) {        // next chunk of flags, loaded in parallel
      __syncthreads();
      for (uint32_t i = tid; i < kRefThreads * 4 && k + i < count; i += blockDim.x) s_flag[i] = flag[k + i];
      __syncthreads();
    }
    if (!s_flag[k % (kRefThreads * 4)]) continue;   // uniform
    const uint32_t c = n + (tg[k] & TGT_QUBIT_MASK);
    const uint32_t cw = c >> 6;
    const uint64_t cm = 1ull << (c & 63);
    // One scan finds the pivot (lowest row with an X/Y term in column c)
    // and gathers the first rows of the support.
    if (tid == 0) {
      s_pivot = 0xFFFFFFFFu;
      s_cnt = 0;
      s_more = 0;
    }
    __syncthreads();
    for (uint32_t j0 = tid; j0 < n; j0 += 4 * blockDim.x) {
      uint64_t v[4];
#pragma unroll
      for (int u = 0; u < 4; u++) {
        const uint32_t j = j0 + u * blockDim.x;
        v[u] = j < n ? XR[(size_t)cw * n + j] : 0;
      }
#pragma unroll
      for (int u = 0; u < 4; u++) {
        if (!(v[u] & cm)) continue;
        const uint32_t j = j0 + u * blockDim.x;
        atomicMin(&s_pivot, j);
        const uint32_t i = atomicAdd(&s_cnt, 1u);
        if (i < kRefList) list[i] = j;
        else s_more = 1;
      }
    }
    __syncthreads();
    const uint32_t p = s_pivot;
    if (p == 0xFFFFFFFFu) {                  // made deterministic by an earlier collapse
      if (tid == 0) {
        const bool r = (SB[cw] & cm) != 0;
        if (gate != G_R && r) set_ref_bit(ref, meas0 + k);
        if (gate != G_M && r) SB[cw] ^= cm;
      }
      __syncthreads();
      continue;
    }
    // Word w of the pivot row: xp_row[w * n] (the row's words are n apart).
    uint64_t *xp_row = XR + p, *zp_row = ZR + p;
    // CNOT appends from the pivot onto every other row with an X/Y term in
    // column c (the pivot's own entry in the list is skipped).  A support
    // larger than the list is handled in rounds: an append clears the row's
    // bit in column c, so a rescan finds the rest.
    bool first_round = true;
    while (true) {
      if (!first_round) {
        if (tid == 0) {
          s_cnt = 0;
          s_more = 0;
        }
        __syncthreads();
        for (uint32_t j = tid; j < n; j += blockDim.x) {
          if (j == p || !(XR[(size_t)cw * n + j] & cm)) continue;
          const uint32_t i = atomicAdd(&s_cnt, 1u);
          if (i < kRefList) list[i] = j;
          else s_more = 1;
        }
        __syncthreads();
      }
      first_round = false;
      const uint32_t cnt = s_cnt < kRefList ? s_cnt : kRefList;
      const bool more = s_more != 0;           // read before the next reset
      for (uint32_t w = tid; w < words; w += blockDim.x) {
        const uint64_t xp = xp_row[(size_t)w * n];
        uint64_t zp = zp_row[(size_t)w * n], sb = SB[w];
        for (uint32_t i = 0; i < cnt; i++) {
          const uint32_t r = list[i];
          if (r == p) continue;
          uint64_t *xt_p = XR + (size_t)w * n + r;
          const uint64_t xt = *xt_p, zt = ZR[(size_t)w * n + r];
          sb ^= xp & zt & ~(xt ^ zp);
          *xt_p = xt ^ xp;
          zp ^= zt;
        }
        zp_row[(size_t)w * n] = zp;
        SB[w] = sb;
      }
      __syncthreads();
      if (!more) break;
    }
    // H (X term at the pivot) or H_YZ (Y term) turns the column into +-Z_p.
    if (tid == 0) s_bit = (zp_row[(size_t)cw * n] & cm) ? 1u : 0u;
    __syncthreads();
    const bool yz = s_bit != 0;
    for (uint32_t w = tid; w < words; w += blockDim.x) {
      const uint64_t x = xp_row[(size_t)w * n], z = zp_row[(size_t)w * n];
      if (yz) {                                // X -> -X, Y -> Z, Z -> Y
        SB[w] ^= x & ~z;
        xp_row[(size_t)w * n] = x ^ z;
      } else {                                 // X <-> Z, Y -> -Y
        SB[w] ^= x & z;
        xp_row[(size_t)w * n] = z;
        zp_row[(size_t)w * n] = x;
      }
    }
    __syncthreads();
    if (tid == 0) s_bit = (SB[cw] & cm) ? 1u : 0u;
    __syncthreads();
    if (s_bit)                                 // X on the pivot: the result becomes 0
      for (uint32_t w = tid; w < words; w += blockDim.x) SB[w] ^= zp_row[(size_t)w * n];
    __syncthreads();
  }
}

// The tableau by columns (c[col][w]: bits of qubits 64 w .. 64 w + 63 of
// column col, column stride nwp words) <-> by column groups (r[cw * n + j]:
// bits of columns 64 cw .. 64 cw + 63 for qubit j): one wave per 64 x 64 bit
// block, transposed in registers.
__global__ void __launch_bounds__(256) k_ref_to_rows(const uint64_t *__restrict__ c, uint64_t *__restrict__ r,
                                                     uint32_t n, uint32_t nwp, uint32_t groups) {
  const uint32_t lane = threadIdx.x & 63;
  const uint64_t b = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;     // block (cw, w)
  const uint32_t nw = (n + 63) / 64;
  if (b >= (uint64_t)groups * nw) return;                                        // whole waves leave
  const uint32_t cw = (uint32_t)(b / nw), w = (uint32_t)(b % nw);
  const uint32_t col = cw * 64 + lane;
  const uint64_t v = col < 2 * n ? c[(size_t)col * nwp + w] : 0;
  const uint64_t y = bit_transpose64(v, lane);
  const uint32_t j = w * 64 + lane;
  if (j < n) r[(size_t)cw * n + j] = y;
}

__global__ void __launch_bounds__(256) k_ref_from_rows(const uint64_t *__restrict__ r, uint64_t *__restrict__ c,
                                                       uint32_t n, uint32_t nwp, uint32_t groups) {
  const uint32_t lane = threadIdx.x & 63;
  const uint64_t b = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const uint32_t nw = (n + 63) / 64;
  if (b >= (uint64_t)groups * nw) return;
  const uint32_t cw = (uint32_t)(b / nw), w = (uint32_t)(b % nw);
  const uint32_t j = w * 64 + lane;
  const uint64_t v = j < n ? r[(size_t)cw * n + j] : 0;
  const uint64_t y = bit_transpose64(v, lane);
  const uint32_t col = cw * 64 + lane;
  if (col < 2 * n) c[(size_t)col * nwp + w] = y;
}

// Classically controlled Paulis: pairs (qubit, lookback); the Pauli is
// prepended where the reference's own result is 1.
__global__ void k_ref_feedback(Tab t, Gate gate, const uint32_t *tg, uint32_t count, uint64_t meas0,
                               const uint64_t *ref) {
  const uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= count) return;
  const uint32_t q = tg[2 * k];
  const uint64_t m = meas0 - tg[2 * k + 1];
  if (!((ref[m >> 6] >> (m & 63)) & 1)) return;
  if (gate != G_CZ) sign_xor(t, t.n + q, 1u);  // X part flips T(Z_q)
  if (gate != G_CX) sign_xor(t, q, 1u);        // Z part flips T(X_q)
}

__global__ void k_ref_identity(Tab t) {
  const uint32_t q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= t.n) return;
  t.xb[(size_t)q * t.nwp + q / 64] = 1ull << (q % 64);
  t.zb[(size_t)(t.n + q) * t.nwp + q / 64] = 1ull << (q % 64);
}

__global__ void k_ref_zero(uint64_t *p, size_t n) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) p[i] = 0;
}

// Host-side plan: the unrolled circuit as kernel steps.
constexpr size_t kMaxSteps = 20000000;
struct Planner {
  std::vector<Step> steps;
  std::vector<uint32_t> targets;
  uint64_t meas = 0;
  // Run in which each value was last used (values: qubits, and lookbacks of
  // feedback pairs, which at worst split a run more often than needed).
  std::unordered_map<uint32_t, uint64_t> big_stamp;
  std::vector<uint64_t> stamp;
  uint64_t run_id = 0;

  explicit Planner(uint64_t n) : stamp(n, ~0ull) {}

  bool seen(uint32_t v) {
    if (v < stamp.size()) return stamp[v] == run_id;
    auto it = big_stamp.find(v);
    return it != big_stamp.end() && it->second == run_id;
  }
  void mark(uint32_t v) {
    if (v < stamp.size()) stamp[v] = run_id;
    else big_stamp[v] = run_id;
  }

  // Splits a target list (k per item) into runs of items with distinct qubits.
  void add_runs(StepKind kind, Gate gate, const std::vector<uint32_t> &t, size_t k) {
    size_t i = 0;
    while (i < t.size() / k) {
      run_id++;
      Step s{kind, gate, (uint32_t)targets.size(), 0, meas};
      while (i < t.size() / k) {
        bool clash = false;
        for (size_t j = 0; j < k; j++) clash |= seen(t[i * k + j] & TGT_QUBIT_MASK);
        if (clash) break;
        for (size_t j = 0; j < k; j++) {
          mark(t[i * k + j] & TGT_QUBIT_MASK);
          targets.push_back(t[i * k + j]);
        }
        s.count++;
        i++;
        if (kind == STEP_MEASURE && gate != G_R) meas++;
      }
      steps.push_back(s);
    }
  }

  bool too_long = false;

  void walk(const std::vector<Node> &nodes) {
    for (const Node &n : nodes) {
      if (too_long) return;
      if (steps.size() > kMaxSteps) {          // e.g. a huge REPEAT count: leave it to the host
        too_long = true;
        return;
      }
      if (n.repeat) {
        for (uint64_t r = 0; r < n.reps && !too_long; r++) walk(n.body);
        continue;
      }
      if (n.gate == G_M || n.gate == G_MR || n.gate == G_R) {
        add_runs(STEP_MEASURE, n.gate, n.targets, 1);
      } else if (gate_is_clifford(n.gate) && !n.targets.empty()) {
        if (!gate_is_two_qubit(n.gate)) {
          add_runs(STEP_PREPEND, n.gate, n.targets, 1);
          continue;
        }
        // Runs of ordinary pairs and of classically controlled pairs, in order.
        size_t i = 0;
        const size_t pairs = n.targets.size() / 2;
        while (i < pairs) {
          const bool fb = ((n.targets[2 * i] | n.targets[2 * i + 1]) & TGT_REC) != 0;
          std::vector<uint32_t> run;
          while (i < pairs && (((n.targets[2 * i] | n.targets[2 * i + 1]) & TGT_REC) != 0) == fb) {
            uint32_t a = n.targets[2 * i], b = n.targets[2 * i + 1];
            if (fb && (a & TGT_REC)) std::swap(a, b);
            run.push_back(a);
            run.push_back(fb ? (b & ~TGT_REC) : b);
            i++;
          }
          if (fb) {
            // Feedback pairs only flip signs of their own qubit's columns;
            // runs with a repeated qubit are split like gates.
            add_runs(STEP_FEEDBACK, n.gate, run, 2);
          } else {
            add_runs(STEP_PREPEND, n.gate, run, 2);
          }
        }
      }
    }
  }
};

// add_runs treats the lookback of a feedback pair as a qubit when checking
// for repeats; splitting more often than needed is harmless.

}  // namespace

int gpu_reference_sample(const std::vector<Node> &tree, uint64_t num_qubits, uint64_t num_measurements,
                         std::vector<uint64_t> &bits, hipStream_t s, std::string &err) {
  bits.assign((num_measurements + 63) / 64, 0);
  if (num_measurements == 0) return STIM_OK;
  const uint64_t n = num_qubits;
  if (n >= (1ull << 30)) {
    err = "too many qubits for the GPU reference sampler";
    return STIM_E_UNSUPPORTED;
  }
  Planner P(n);
  P.walk(tree);
  if (P.too_long) {
    err = "circuit too long for the GPU reference sampler";
    return STIM_E_UNSUPPORTED;
  }
  const uint64_t nw = (n + 63) / 64, nwp = transpose_stride(n);          // column stride
  const uint64_t s2 = transpose_stride(2 * n);                           // row stride (transposed)
  Tab t{nullptr, nullptr, nullptr, (uint32_t)n, (uint32_t)nw, (uint32_t)nwp};
  uint64_t *ref = nullptr, *XR = nullptr, *ZR = nullptr;
  uint32_t *dtg = nullptr, *flag = nullptr, *random = nullptr;
  uint32_t max_meas_count = 1, nmeas_steps = 0;
  for (const Step &st : P.steps)
    if (st.kind == STEP_MEASURE) {
      max_meas_count = std::max(max_meas_count, st.count);
      nmeas_steps++;
    }
  const size_t cwords = (size_t)2 * n * nwp, rwords = (size_t)n * s2;
  hipError_t e = hipSuccess;
  auto fail = [&](hipError_t code, const char *what) {
    err = std::string(what) + ": " + hipGetErrorString(code);
    return code == hipErrorOutOfMemory ? STIM_E_OOM : STIM_E_DEVICE;
  };
  auto alloc = [&](void **ptr, size_t bytes) { return hipMallocAsync(ptr, std::max<size_t>(bytes, 8), s); };
  int rc = STIM_OK;
  do {
    if ((e = alloc((void **)&t.xb, cwords * 8)) != hipSuccess || (e = alloc((void **)&t.zb, cwords * 8)) != hipSuccess ||
        (e = alloc((void **)&t.sb, s2 * 8)) != hipSuccess || (e = alloc((void **)&XR, rwords * 8)) != hipSuccess ||
        (e = alloc((void **)&ZR, rwords * 8)) != hipSuccess || (e = alloc((void **)&ref, bits.size() * 8)) != hipSuccess ||
        (e = alloc((void **)&flag, (size_t)max_meas_count * 4)) != hipSuccess ||
        (e = alloc((void **)&random, (size_t)(std::max<uint32_t>(nmeas_steps, 1) + 1) / 2 * 8)) != hipSuccess ||
        (e = alloc((void **)&dtg, P.targets.size() * 4)) != hipSuccess) {
      rc = fail(e, "reference allocation");
      break;
    }
    if (!P.targets.empty() &&
        (e = hipMemcpyAsync(dtg, P.targets.data(), P.targets.size() * 4, hipMemcpyHostToDevice, s)) != hipSuccess) {
      rc = fail(e, "target upload");
      break;
    }
    hipLaunchKernelGGL(k_ref_zero, dim3(1024), dim3(256), 0, s, t.xb, cwords);
    hipLaunchKernelGGL(k_ref_zero, dim3(1024), dim3(256), 0, s, t.zb, cwords);
    hipLaunchKernelGGL(k_ref_zero, dim3(64), dim3(256), 0, s, (uint64_t *)t.sb, (size_t)s2);
    hipLaunchKernelGGL(k_ref_zero, dim3(64), dim3(256), 0, s, ref, bits.size());
    hipLaunchKernelGGL(k_ref_zero, dim3(64), dim3(256), 0, s, (uint64_t *)random,
                       (size_t)(std::max<uint32_t>(nmeas_steps, 1) + 1) / 2);
    hipLaunchKernelGGL(k_ref_identity, dim3((uint32_t)((n + 255) / 256)), dim3(256), 0, s, t);
    uint32_t mstep = 0;
    for (const Step &st : P.steps) {
      if (st.count == 0) continue;
      const uint32_t *tg = dtg + st.toff;
      const dim3 waves((st.count + 3) / 4);
      if (st.kind == STEP_PREPEND) {
        hipLaunchKernelGGL(k_ref_prepend, waves, dim3(256), 0, s, t, st.gate, tg, st.count);
      } else if (st.kind == STEP_FEEDBACK) {
        hipLaunchKernelGGL(k_ref_feedback, dim3((st.count + 255) / 256), dim3(256), 0, s, t, st.gate, tg, st.count,
                           st.meas0, (const uint64_t *)ref);
      } else {
        uint32_t *rnd = random + mstep++;
        hipLaunchKernelGGL(k_ref_measure_det, waves, dim3(256), 0, s, t, st.gate, tg, st.count, st.meas0, ref, flag,
                           rnd);
        uint32_t h_rnd = 0;
        if ((e = hipMemcpyAsync(&h_rnd, rnd, 4, hipMemcpyDeviceToHost, s)) != hipSuccess ||
            (e = hipStreamSynchronize(s)) != hipSuccess) {
          rc = fail(e, "reference measurement step");
          break;
        }
        if (h_rnd == 0) continue;
        // Random results: transpose, collapse them in order, transpose back.
        const uint32_t groups = (uint32_t)((2 * n + 63) / 64);
        const dim3 tgrid((uint32_t)(((uint64_t)groups * nw * 64 + 255) / 256));
        hipLaunchKernelGGL(k_ref_to_rows, tgrid, dim3(256), 0, s, t.xb, XR, (uint32_t)n, (uint32_t)nwp, groups);
        hipLaunchKernelGGL(k_ref_to_rows, tgrid, dim3(256), 0, s, t.zb, ZR, (uint32_t)n, (uint32_t)nwp, groups);
        hipLaunchKernelGGL(k_ref_collapse_rows, dim3(1), dim3(kRefThreads), 0, s, XR, ZR, (uint64_t *)t.sb,
                           (uint32_t)n, st.gate, tg, st.count, st.meas0, ref, (const uint32_t *)flag);
        hipLaunchKernelGGL(k_ref_from_rows, tgrid, dim3(256), 0, s, XR, t.xb, (uint32_t)n, (uint32_t)nwp, groups);
        hipLaunchKernelGGL(k_ref_from_rows, tgrid, dim3(256), 0, s, ZR, t.zb, (uint32_t)n, (uint32_t)nwp, groups);
      }
    }
    if (rc) break;
    if ((e = hipGetLastError()) != hipSuccess) { rc = fail(e, "reference kernel launch"); break; }
    if ((e = hipMemcpyAsync(bits.data(), ref, bits.size() * 8, hipMemcpyDeviceToHost, s)) != hipSuccess) {
      rc = fail(e, "reference download");
      break;
    }
    if ((e = hipStreamSynchronize(s)) != hipSuccess) { rc = fail(e, "reference kernels"); break; }
  } while (false);
  void *ptrs[] = {t.xb, t.zb, t.sb, XR, ZR, ref, flag, random, dtg};
  for (void *p : ptrs)
    if (p) (void)hipFreeAsync(p, s);
  return rc;
}

}  // namespace stimgpu
