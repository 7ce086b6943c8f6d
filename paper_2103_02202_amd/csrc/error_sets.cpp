// Error sets for sparse detection-event sampling (Sec. 5.6).
//
// For every noise site the sampler needs the detectors and observables that
// each of its single-qubit Pauli generators flips.  They are found for all
// sites at once by running the circuit backwards with one "lane" per
// detector and observable: lane l carries the Pauli S_l(t) such that an
// error E inserted at time t flips output l exactly when E anticommutes with
// S_l(t).  Going backwards, a Z measurement that output l reads adds Z on the
// measured qubit to S_l; a Clifford U maps S to U^dagger S U, whose unsigned
// xz map equals U's own (every frame map of the gate set is an involution);
// a reset clears the qubit, since errors before it cannot reach later
// outputs.  An X error on q then flips the lanes whose S has a Z part on q,
// a Z error those with an X part.
//
// The frame simulation adds a random Z after every collapse (Sec. 3).  An
// output is deterministic only if none of those can reach it, i.e. if no
// lane has an X part on the collapsed qubit right after the collapse; the
// walk checks this and refuses circuits that fail it, because the sparse
// method cannot reproduce a random detector.
//
// Lanes are processed in independent chunks of 64-lane words on a few host
// threads.  Storage per chunk is an X row and a Z row per qubit.
#include <algorithm>
#include <atomic>
#include <thread>

#include "circuit.h"
#include "stim_gpu.h"

namespace stimgpu {

namespace {

constexpr size_t kChunkWords = 32;     // lanes per chunk = 2048

struct Exec {
  uint32_t pc;
  uint64_t meas;     // measurements before this op
  uint32_t noise;    // noise execution index, or ~0u
};

struct ChunkOut {
  std::vector<std::pair<uint64_t, uint32_t>> entries;   // (generator, lane)
  uint64_t random_lane = ~0ull;                         // a lane that depends on a random outcome
};

// Walks the program backwards for lanes [lane0, lane_end), whose outputs
// read measurements m_lo .. m_hi only: ops after m_hi see all-zero rows and
// are skipped, and once m_lo is passed the walk stops as soon as every row
// is zero again (nothing earlier can then reach these outputs).
void walk_chunk(const Program &P, const std::vector<Exec> &exec, const std::vector<uint64_t> &gen_base,
                const std::vector<uint32_t> &moff, const std::vector<uint32_t> &mlanes, uint64_t lane0,
                uint64_t lane_end, uint64_t m_lo, uint64_t m_hi, ChunkOut &out) {
  const size_t CW = kChunkWords;
  const size_t n = P.num_qubits;
  std::vector<uint64_t> X(n * CW, 0), Z(n * CW, 0);
  // live[q] = 0 guarantees all-zero rows for qubit q (1 means "maybe"), so
  // the many ops away from a chunk's outputs cost a flag test each.
  std::vector<uint8_t> live(n, 0);
  auto xr = [&](uint32_t q) { return &X[(size_t)q * CW]; };
  auto zr = [&](uint32_t q) { return &Z[(size_t)q * CW]; };
  auto any = [&](const uint64_t *r) -> uint64_t {
    for (size_t w = 0; w < CW; w++) if (r[w]) return lane0 + 64 * w + (uint64_t)__builtin_ctzll(r[w]);
    return ~0ull;
  };
  auto check_collapse = [&](uint32_t q) {
    if (!live[q]) return;
    uint64_t l = any(xr(q));
    if (l != ~0ull && out.random_lane == ~0ull) out.random_lane = l;
  };
  auto clear = [&](uint32_t q) {
    if (!live[q]) return;
    std::fill(xr(q), xr(q) + CW, 0);
    std::fill(zr(q), zr(q) + CW, 0);
    live[q] = 0;
  };
  auto add_measurement = [&](uint32_t q, uint64_t m) {
    uint64_t *z = zr(q);
    for (uint32_t a = moff[m]; a < moff[m + 1]; a++) {
      uint64_t l = mlanes[a];
      if (l >= lane0 && l < lane_end) {
        z[(l - lane0) / 64] ^= 1ull << ((l - lane0) % 64);
        live[q] = 1;
      }
    }
  };
  auto emit = [&](const uint64_t *r, uint64_t gid) {
    for (size_t w = 0; w < CW; w++) {
      uint64_t v = r[w];
      while (v) {
        out.entries.push_back({gid, (uint32_t)(lane0 + 64 * w + (uint64_t)__builtin_ctzll(v))});
        v &= v - 1;
      }
    }
  };
  // Refreshes the live flags; true when no row is non-zero.
  auto all_zero = [&]() {
    bool none = true;
    for (size_t q = 0; q < n; q++) {
      if (!live[q]) continue;
      const uint64_t *x = xr((uint32_t)q), *z = zr((uint32_t)q);
      bool nz = false;
      for (size_t w = 0; w < CW && !nz; w++) nz = (x[w] | z[w]) != 0;
      live[q] = nz;
      none &= !nz;
    }
    return none;
  };
  uint32_t since_check = 0;
  for (size_t i = exec.size(); i-- > 0;) {
    if (exec[i].meas > m_hi) continue;         // after the last measurement the lanes read
    if (exec[i].meas <= m_lo && ++since_check >= 8) {
      since_check = 0;
      if (all_zero()) break;
    }
    const DevOp &op = P.ops[exec[i].pc];
    const uint32_t code = op.code & 0xFFFFu;
    const uint32_t *tg = &P.targets[op.toff];
    switch (code) {
      case OP_INIT:
        for (uint32_t q = 0; q < n; q++) check_collapse(q);
        break;
      case OP_R:
      case OP_M:
      case OP_MR:
        for (uint32_t k = 0; k < op.n; k++) {
          const uint32_t q = tg[k] & TGT_QUBIT_MASK;
          check_collapse(q);
          if (code != OP_M) clear(q);
          if (code != OP_R) add_measurement(q, exec[i].meas + k);
        }
        break;
      case OP_SWAP_XZ:
        for (uint32_t k = 0; k < op.n; k++)
          if (live[tg[k]]) std::swap_ranges(xr(tg[k]), xr(tg[k]) + CW, zr(tg[k]));
        break;
      case OP_Z_XOR_X:
        for (uint32_t k = 0; k < op.n; k++) {
          if (!live[tg[k]]) continue;
          uint64_t *x = xr(tg[k]), *z = zr(tg[k]);
          for (size_t w = 0; w < CW; w++) z[w] ^= x[w];
        }
        break;
      case OP_X_XOR_Z:
        for (uint32_t k = 0; k < op.n; k++) {
          if (!live[tg[k]]) continue;
          uint64_t *x = xr(tg[k]), *z = zr(tg[k]);
          for (size_t w = 0; w < CW; w++) x[w] ^= z[w];
        }
        break;
      case OP_CX: case OP_CY: case OP_CZ: case OP_SWAP:
        for (uint32_t k = 0; k < op.n; k++) {
          const uint32_t qa = tg[2 * k], qb = tg[2 * k + 1];
          if (!live[qa] && !live[qb]) continue;
          live[qa] = live[qb] = 1;
          uint64_t *xa = xr(qa), *za = zr(qa), *xb = xr(qb), *zb = zr(qb);
          for (size_t w = 0; w < CW; w++) {
            const uint64_t a = xa[w], b = za[w], c = xb[w], d = zb[w];
            switch (code) {
              case OP_CX: xb[w] = c ^ a; za[w] = b ^ d; break;
              case OP_CZ: za[w] = b ^ c; zb[w] = d ^ a; break;
              case OP_CY: xb[w] = c ^ a; zb[w] = d ^ a; za[w] = b ^ c ^ d; break;
              default: xa[w] = c; za[w] = d; xb[w] = a; zb[w] = b; break;
            }
          }
        }
        break;
      case OP_NOISE_X: case OP_NOISE_Y: case OP_NOISE_Z: case OP_NOISE_DEP1: case OP_NOISE_DEP2: {
        const uint32_t Q = code == OP_NOISE_DEP2 ? 2 : 1;
        const uint64_t base = gen_base[exec[i].noise];
        for (uint32_t k = 0; k < op.n; k++)
          for (uint32_t j = 0; j < Q; j++) {
            const uint32_t q = tg[Q * k + j];
            if (!live[q]) continue;
            const uint64_t gid = base + 2 * (Q * (uint64_t)k + j);
            emit(zr(q), gid);          // X error: lanes with a Z part on q
            emit(xr(q), gid + 1);      // Z error: lanes with an X part on q
          }
        break;
      }
      default:
        break;
    }
  }
}

}  // namespace

ErrorModel build_error_model(const Program &P) {
  ErrorModel em;
  // Forward walk: every op execution with its measurement count, and the
  // first generator of every noise execution (slot order within it).
  std::vector<Exec> exec;
  {
    std::vector<uint32_t> left;
    uint64_t meas = 0, steps = 0;
    uint32_t noise = 0;
    for (uint32_t pc = 0; pc < P.ops.size(); pc++) {
      const DevOp &op = P.ops[pc];
      const uint32_t code = op.code & 0xFFFFu;
      if (code == OP_LOOP_BEGIN) { left.push_back(op.aux); continue; }
      if (code == OP_LOOP_END) {
        if (--left.back() > 0) pc = op.aux;
        else left.pop_back();
        continue;
      }
      if (++steps > 20000000ull)
        throw CompileError{STIM_E_UNSUPPORTED, "circuit too long for sparse detection sampling"};
      if (code >= OP_FB_X && code <= OP_FB_Z)
        throw CompileError{STIM_E_UNSUPPORTED, "sparse detection sampling does not take classically controlled Paulis"};
      Exec e{pc, meas, ~0u};
      if (code >= OP_NOISE_X && code <= OP_NOISE_DEP2) {
        e.noise = noise++;
        em.gen_base.push_back(em.num_generators);
        em.num_generators += (uint64_t)op.n * (code == OP_NOISE_DEP2 ? 4 : 2);
      }
      if (code == OP_M || code == OP_MR) meas += op.n;
      exec.push_back(e);
    }
    if (noise != P.noise_pc.size())
      throw CompileError{STIM_E_UNSUPPORTED, "too many noise executions for sparse detection sampling"};
  }
  // Measurement -> lanes (detector d: lane d, observable o: lane D + o).
  const uint64_t D = P.num_detectors, L = P.num_observables, M = P.num_measurements;
  std::vector<uint32_t> moff(M + 1, 0), mlanes;
  {
    for (uint32_t m : P.det_indices) moff[m + 1]++;
    for (uint32_t m : P.obs_indices) moff[m + 1]++;
    for (uint64_t m = 0; m < M; m++) moff[m + 1] += moff[m];
    mlanes.resize(moff[M]);
    std::vector<uint32_t> fill(moff.begin(), moff.end() - 1);
    for (uint64_t d = 0; d < D; d++)
      for (uint32_t a = P.det_offsets[d]; a < P.det_offsets[d + 1]; a++) mlanes[fill[P.det_indices[a]]++] = (uint32_t)d;
    for (uint64_t o = 0; o < L; o++)
      for (uint32_t a = P.obs_offsets[o]; a < P.obs_offsets[o + 1]; a++)
        mlanes[fill[P.obs_indices[a]]++] = (uint32_t)(D + o);
  }
  const uint64_t lanes = D + L;
  if (lanes >= 0xFFFFFFFFull) throw CompileError{STIM_E_UNSUPPORTED, "too many detectors for sparse detection sampling"};
  const size_t nchunks = (size_t)((lanes + 64 * kChunkWords - 1) / (64 * kChunkWords));
  std::vector<ChunkOut> outs(nchunks);
  std::atomic<size_t> next{0};
  // Measurement range read by each chunk's lanes.
  std::vector<uint64_t> c_lo(nchunks, ~0ull), c_hi(nchunks, 0);
  auto note = [&](uint64_t lane, uint64_t m) {
    const size_t ch = (size_t)(lane / (64 * kChunkWords));
    c_lo[ch] = std::min(c_lo[ch], m);
    c_hi[ch] = std::max(c_hi[ch], m);
  };
  for (uint64_t d = 0; d < D; d++)
    for (uint32_t a = P.det_offsets[d]; a < P.det_offsets[d + 1]; a++) note(d, P.det_indices[a]);
  for (uint64_t o = 0; o < L; o++)
    for (uint32_t a = P.obs_offsets[o]; a < P.obs_offsets[o + 1]; a++) note(D + o, P.obs_indices[a]);
  auto worker = [&]() {
    for (size_t ch; (ch = next.fetch_add(1)) < nchunks;) {
      const uint64_t l0 = (uint64_t)ch * 64 * kChunkWords;
      if (c_lo[ch] == ~0ull) {
        // Lanes that read no measurement are never flipped; the walk still
        // checks them for dependence on random outcomes (there is none).
        continue;
      }
      walk_chunk(P, exec, em.gen_base, moff, mlanes, l0, std::min<uint64_t>(lanes, l0 + 64 * kChunkWords),
                 c_lo[ch], c_hi[ch], outs[ch]);
    }
  };
  const size_t nthreads = std::min<size_t>({nchunks, 16, std::max(1u, std::thread::hardware_concurrency())});
  std::vector<std::thread> pool;
  for (size_t t = 1; t < nthreads; t++) pool.emplace_back(worker);
  worker();
  for (auto &t : pool) t.join();
  for (const ChunkOut &o : outs)
    if (o.random_lane != ~0ull) {
      const bool det = o.random_lane < D;
      throw CompileError{STIM_E_UNSUPPORTED,
                         std::string(det ? "detector " : "observable ") +
                             std::to_string(det ? o.random_lane : o.random_lane - D) +
                             " depends on a random measurement outcome"};
    }
  // CSR over generators; within a generator, lanes ascend (chunks in order).
  uint64_t total = 0;
  for (const ChunkOut &o : outs) total += o.entries.size();
  if (total >= 0xFFFFFFFFull)
    throw CompileError{STIM_E_UNSUPPORTED, "too many error-set entries for sparse detection sampling"};
  em.set_off.assign(em.num_generators + 1, 0);
  for (const ChunkOut &o : outs)
    for (const auto &e : o.entries) em.set_off[e.first + 1]++;
  for (uint64_t g = 0; g < em.num_generators; g++) em.set_off[g + 1] += em.set_off[g];
  em.set_lanes.resize(total);
  std::vector<uint32_t> fill(em.set_off.begin(), em.set_off.end() - 1);
  for (const ChunkOut &o : outs) {
    // Entries of one chunk were appended walking backwards: generators in
    // descending order, lanes ascending within each.
    for (const auto &e : o.entries) em.set_lanes[fill[e.first]++] = e.second;
  }
  return em;
}

}  // namespace stimgpu
