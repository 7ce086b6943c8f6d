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

#include "circuit.h"
#include "reference_gpu.h"
#include "stim_gpu.h"

namespace stimgpu {

namespace {

struct Tab {
  uint64_t *xb, *zb;     // [2n][nw]
  uint32_t *sign;        // [2n]
  uint32_t n, nw;
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

__device__ __forceinline__ void wave_swap_cols(const Tab &t, uint32_t a, uint32_t b, uint32_t lane) {
  uint64_t *xa = t.xb + (size_t)a * t.nw, *xb = t.xb + (size_t)b * t.nw;
  uint64_t *za = t.zb + (size_t)a * t.nw, *zb = t.zb + (size_t)b * t.nw;
  for (uint32_t w = lane; w < t.nw; w += 64) {
    const uint64_t x = xa[w], z = za[w];
    xa[w] = xb[w];
    za[w] = zb[w];
    xb[w] = x;
    zb[w] = z;
  }
  if (lane == 0) {
    const uint32_t s = t.sign[a];
    t.sign[a] = t.sign[b];
    t.sign[b] = s;
  }
}

// Column dst <- i^e * dst * src.  For Hermitian single-qubit Paulis written
// as i^(x z) X^x Z^z, the product's phase exponent is the sum over qubits of
// x1 z1 + x2 z2 + 2 z1 x2 - x3 z3; it must be even (a real sign).
__device__ __forceinline__ void wave_mul_cols(const Tab &t, uint32_t dst, uint32_t src, int e, uint32_t lane) {
  uint64_t *x1 = t.xb + (size_t)dst * t.nw, *z1 = t.zb + (size_t)dst * t.nw;
  const uint64_t *x2 = t.xb + (size_t)src * t.nw, *z2 = t.zb + (size_t)src * t.nw;
  int acc = 0;
  for (uint32_t w = lane; w < t.nw; w += 64) {
    const uint64_t a = x1[w], b = z1[w], c = x2[w], d = z2[w];
    const uint64_t x3 = a ^ c, z3 = b ^ d;
    acc += __popcll(a & b) + __popcll(c & d) + 2 * __popcll(b & c) - __popcll(x3 & z3);
    x1[w] = x3;
    z1[w] = z3;
  }
  acc = wave_sum(acc) + e;
  if (lane == 0) t.sign[dst] ^= t.sign[src] ^ (uint32_t)((acc >> 1) & 1);
}

__device__ __forceinline__ void flip_sign(const Tab &t, uint32_t col, uint32_t lane) {
  if (lane == 0) t.sign[col] ^= 1u;
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
// targets are flagged for the ordered pass.
__global__ void __launch_bounds__(256) k_ref_measure_det(Tab t, Gate gate, const uint32_t *tg, uint32_t count,
                                                         uint64_t meas0, uint64_t *ref, uint32_t *flag) {
  const uint32_t lane = threadIdx.x & 63;
  const uint32_t k = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  if (k >= count) return;
  const uint32_t c = t.n + (tg[k] & TGT_QUBIT_MASK);
  bool any = false;
  for (uint32_t w = lane; w < t.nw; w += 64) any |= t.xb[(size_t)c * t.nw + w] != 0;
  any = __any(any);
  if (lane == 0) {
    flag[k] = any ? 1u : 0u;
    if (!any) {
      if (gate != G_R && t.sign[c]) set_ref_bit(ref, meas0 + k);
      if (gate != G_M) t.sign[c] = 0;
    }
  }
}

constexpr uint32_t kRefThreads = 1024;
constexpr uint32_t kRefMaxWords = 4096;     // n up to 262,144 qubits

// The ordered pass over a measurement step's random targets (one workgroup).
__global__ void __launch_bounds__(kRefThreads) k_ref_measure_rand(Tab t, Gate gate, const uint32_t *tg,
                                                                   uint32_t count, uint64_t meas0, uint64_t *ref,
                                                                   const uint32_t *flag) {
  __shared__ uint64_t snap[kRefMaxWords];      // X part of the measured column
  __shared__ uint32_t words[kRefMaxWords];     // indices of its non-zero words
  __shared__ uint32_t s_pivot, s_bit, s_nwords;
  const uint32_t tid = threadIdx.x, nw = t.nw, ncols = 2 * t.n;
  for (uint32_t k = 0; k < count; k++) {
    if (!flag[k]) continue;                    // uniform
    const uint32_t c = t.n + (tg[k] & TGT_QUBIT_MASK);
    if (tid == 0) {
      s_pivot = 0xFFFFFFFFu;
      s_nwords = 0;
    }
    __syncthreads();
    for (uint32_t w = tid; w < nw; w += blockDim.x) {
      const uint64_t v = t.xb[(size_t)c * nw + w];
      snap[w] = v;
      if (v) {
        atomicMin(&s_pivot, w * 64 + (uint32_t)__builtin_ctzll(v));
        words[atomicAdd(&s_nwords, 1u)] = w;
      }
    }
    __syncthreads();
    const uint32_t nwords = s_nwords;
    const uint32_t pivot = s_pivot;
    if (pivot == 0xFFFFFFFFu) {                // made deterministic by an earlier collapse
      if (tid == 0) {
        if (gate != G_R && t.sign[c]) set_ref_bit(ref, meas0 + k);
        if (gate != G_M) t.sign[c] = 0;
      }
      __syncthreads();
      continue;
    }
    const uint32_t pw = pivot >> 6;
    const uint64_t pm = 1ull << (pivot & 63);
    // CNOT appends from the pivot onto every other X/Y term, all columns
    // (appends with a common control commute, so their order is free).
    for (uint32_t col = tid; col < ncols; col += blockDim.x) {
      uint64_t *X = t.xb + (size_t)col * nw, *Z = t.zb + (size_t)col * nw;
      const uint64_t xp = (X[pw] & pm) ? 1 : 0;
      uint64_t zp = (Z[pw] & pm) ? 1 : 0;
      uint32_t s = 0;
      for (uint32_t i = 0; i < nwords; i++) {
        const uint32_t w = words[i];
        uint64_t v = snap[w];
        if (w == pw) v &= ~pm;
        if (!v) continue;
        uint64_t xw = X[w], zw = Z[w];
        const uint64_t x0 = xw;
        while (v) {
          const uint32_t b = (uint32_t)__builtin_ctzll(v);
          v &= v - 1;
          const uint64_t xt = (xw >> b) & 1, zt = (zw >> b) & 1;
          s ^= (uint32_t)(xp & zt & (xt ^ zp ^ 1));
          xw ^= xp << b;
          zp ^= zt;
        }
        if (xw != x0) X[w] = xw;
      }
      const uint64_t zcur = (Z[pw] & pm) ? 1 : 0;
      if (zcur != zp) Z[pw] ^= pm;
      if (s) t.sign[col] ^= 1u;
    }
    __syncthreads();
    if (tid == 0) s_bit = (t.zb[(size_t)c * nw + pw] & pm) ? 1u : 0u;
    __syncthreads();
    const bool yz = s_bit != 0;                // Y term at the pivot: H_YZ, else H
    for (uint32_t col = tid; col < ncols; col += blockDim.x) {
      uint64_t *X = t.xb + (size_t)col * nw + pw, *Z = t.zb + (size_t)col * nw + pw;
      const uint64_t x = (*X & pm) ? 1 : 0, z = (*Z & pm) ? 1 : 0;
      if (yz) {                                // X -> -X, Y -> Z, Z -> Y
        if (x & (z ^ 1)) t.sign[col] ^= 1u;
        if (z) *X ^= pm;
      } else {                                 // X <-> Z, Y -> -Y
        if (x & z) t.sign[col] ^= 1u;
        if (x ^ z) {
          *X ^= pm;
          *Z ^= pm;
        }
      }
    }
    __syncthreads();
    if (tid == 0) s_bit = t.sign[c];
    __syncthreads();
    if (s_bit)                                 // X on the pivot makes the result 0
      for (uint32_t col = tid; col < ncols; col += blockDim.x)
        if (t.zb[(size_t)col * nw + pw] & pm) t.sign[col] ^= 1u;
    __syncthreads();
    if (tid == 0 && gate != G_M) t.sign[c] = 0;
    __syncthreads();
  }
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
  if (gate != G_CZ) t.sign[t.n + q] ^= 1u;     // X part flips T(Z_q)
  if (gate != G_CX) t.sign[q] ^= 1u;           // Z part flips T(X_q)
}

__global__ void k_ref_identity(Tab t) {
  const uint32_t q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= t.n) return;
  t.xb[(size_t)q * t.nw + q / 64] = 1ull << (q % 64);
  t.zb[(size_t)(t.n + q) * t.nw + q / 64] = 1ull << (q % 64);
}

__global__ void k_ref_zero(uint64_t *p, size_t n) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) p[i] = 0;
}

// Host-side plan: the unrolled circuit as kernel steps.
struct Planner {
  std::vector<Step> steps;
  std::vector<uint32_t> targets;
  uint64_t meas = 0;

  // Splits a target list (k per item) into runs of items with distinct qubits.
  void add_runs(StepKind kind, Gate gate, const std::vector<uint32_t> &t, size_t k) {
    std::unordered_map<uint32_t, int> used;
    size_t i = 0;
    while (i < t.size() / k) {
      used.clear();
      Step s{kind, gate, (uint32_t)targets.size(), 0, meas};
      while (i < t.size() / k) {
        bool clash = false;
        for (size_t j = 0; j < k; j++) clash |= used.count(t[i * k + j] & TGT_QUBIT_MASK) > 0;
        if (clash) break;
        for (size_t j = 0; j < k; j++) {
          used[t[i * k + j] & TGT_QUBIT_MASK] = 1;
          targets.push_back(t[i * k + j]);
        }
        s.count++;
        i++;
        if (kind == STEP_MEASURE && gate != G_R) meas++;
      }
      steps.push_back(s);
    }
  }

  void walk(const std::vector<Node> &nodes) {
    for (const Node &n : nodes) {
      if (n.repeat) {
        for (uint64_t r = 0; r < n.reps; r++) walk(n.body);
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
  const uint64_t n = num_qubits, nw = (n + 63) / 64;
  if (nw > kRefMaxWords) {
    err = "too many qubits for the GPU reference sampler";
    return STIM_E_UNSUPPORTED;
  }
  Planner P;
  P.walk(tree);
  Tab t{nullptr, nullptr, nullptr, (uint32_t)n, (uint32_t)nw};
  uint64_t *ref = nullptr;
  uint32_t *dtg = nullptr, *flag = nullptr;
  uint32_t max_meas_count = 1;
  for (const Step &st : P.steps)
    if (st.kind == STEP_MEASURE) max_meas_count = std::max(max_meas_count, st.count);
  const size_t words = (size_t)2 * n * nw;
  hipError_t e = hipSuccess;
  auto fail = [&](hipError_t code, const char *what) {
    err = std::string(what) + ": " + hipGetErrorString(code);
    return code == hipErrorOutOfMemory ? STIM_E_OOM : STIM_E_DEVICE;
  };
  int rc = STIM_OK;
  do {
    if ((e = hipMallocAsync((void **)&t.xb, words * 8, s)) != hipSuccess) { rc = fail(e, "tableau allocation"); break; }
    if ((e = hipMallocAsync((void **)&t.zb, words * 8, s)) != hipSuccess) { rc = fail(e, "tableau allocation"); break; }
    if ((e = hipMallocAsync((void **)&t.sign, 2 * n * 4 + 4, s)) != hipSuccess) { rc = fail(e, "tableau allocation"); break; }
    if ((e = hipMallocAsync((void **)&ref, bits.size() * 8, s)) != hipSuccess) { rc = fail(e, "reference allocation"); break; }
    if ((e = hipMallocAsync((void **)&flag, (size_t)max_meas_count * 4, s)) != hipSuccess) { rc = fail(e, "flag allocation"); break; }
    if ((e = hipMallocAsync((void **)&dtg, std::max<size_t>(P.targets.size(), 1) * 4, s)) != hipSuccess) {
      rc = fail(e, "target allocation");
      break;
    }
    if (!P.targets.empty() &&
        (e = hipMemcpyAsync(dtg, P.targets.data(), P.targets.size() * 4, hipMemcpyHostToDevice, s)) != hipSuccess) {
      rc = fail(e, "target upload");
      break;
    }
    hipLaunchKernelGGL(k_ref_zero, dim3(1024), dim3(256), 0, s, t.xb, words);
    hipLaunchKernelGGL(k_ref_zero, dim3(1024), dim3(256), 0, s, t.zb, words);
    hipLaunchKernelGGL(k_ref_zero, dim3(64), dim3(256), 0, s, (uint64_t *)t.sign, (size_t)(2 * n * 4 + 4) / 8);
    hipLaunchKernelGGL(k_ref_zero, dim3(64), dim3(256), 0, s, ref, bits.size());
    hipLaunchKernelGGL(k_ref_identity, dim3((uint32_t)((n + 255) / 256)), dim3(256), 0, s, t);
    for (const Step &st : P.steps) {
      if (st.count == 0) continue;
      const uint32_t *tg = dtg + st.toff;
      const dim3 waves((st.count + 3) / 4);
      if (st.kind == STEP_PREPEND) {
        hipLaunchKernelGGL(k_ref_prepend, waves, dim3(256), 0, s, t, st.gate, tg, st.count);
      } else if (st.kind == STEP_MEASURE) {
        hipLaunchKernelGGL(k_ref_measure_det, waves, dim3(256), 0, s, t, st.gate, tg, st.count, st.meas0, ref, flag);
        hipLaunchKernelGGL(k_ref_measure_rand, dim3(1), dim3(kRefThreads), 0, s, t, st.gate, tg, st.count, st.meas0,
                           ref, (const uint32_t *)flag);
      } else {
        hipLaunchKernelGGL(k_ref_feedback, dim3((st.count + 255) / 256), dim3(256), 0, s, t, st.gate, tg, st.count,
                           st.meas0, (const uint64_t *)ref);
      }
    }
    if ((e = hipGetLastError()) != hipSuccess) { rc = fail(e, "reference kernel launch"); break; }
    if ((e = hipMemcpyAsync(bits.data(), ref, bits.size() * 8, hipMemcpyDeviceToHost, s)) != hipSuccess) {
      rc = fail(e, "reference download");
      break;
    }
    if ((e = hipStreamSynchronize(s)) != hipSuccess) { rc = fail(e, "reference kernels"); break; }
  } while (false);
  void *ptrs[] = {t.xb, t.zb, t.sign, ref, flag, dtg};
  for (void *p : ptrs)
    if (p) (void)hipFreeAsync(p, s);
  return rc;
}

}  // namespace stimgpu
