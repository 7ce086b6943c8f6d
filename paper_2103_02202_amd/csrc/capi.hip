// C ABI of the sampler (declared in include/stim_gpu.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "stim_gpu.h"
#include "circuit.h"
#include "format_kernels.h"
#include "frame_kernels.h"
#include "reference_gpu.h"
#include "sparse_kernels.h"

using namespace stimgpu;

// Device scratch of stim_detector_sample_noalloc: the flip table (and the
// frame slots of circuits too large for LDS) of one call, in a file-scope
// device array instead of the stream-ordered pool.  Each device that loads
// the library holds its own copy until the process ends.  Host code reaches
// it only through the address hipGetSymbolAddress returns on each device (the
// array's name on the host is a stand-in, not a device address).
constexpr size_t kNoAllocScratchBytes = 256ull << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace {

thread_local std::string g_last_error;

int set_error(int code, const std::string &msg) {
  g_last_error = msg;
  return code;
}

int hip_error(hipError_t e, const char *what) {
  return set_error(STIM_E_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

// Device-resident copy of a compiled circuit.
struct DeviceCopy {
  DevOp *ops = nullptr;
  DevOp *event_ops = nullptr;       // the program with event ops
  // Detector mode of a circuit whose detectors and observables are all
  // deterministic: the program with every collapse's Z randomisation marked
  // unread (see ensure_noz_program); NULL when not built or not applicable.
  DevOp *noz_ops = nullptr;
  uint32_t *noz_targets = nullptr;
  bool noz_checked = false;
  uint32_t *targets = nullptr;
  uint64_t *thresholds = nullptr;
  uint64_t *ref = nullptr;
  uint32_t *det_off = nullptr, *det_idx = nullptr, *obs_off = nullptr, *obs_idx = nullptr, *det_order = nullptr;
  uint32_t *det_blocks = nullptr;   // Program::det_blocks
  uint32_t *noise_pc = nullptr;
  uint64_t *noise_instr = nullptr;
  // Error sets of sparse detection sampling (uploaded on its first use).
  uint64_t *gen_base = nullptr;
  uint32_t *set_off = nullptr, *set_lanes = nullptr;
  uint32_t *wb_e0 = nullptr, *wb_e1 = nullptr, *wb_base = nullptr;   // window batches
};

}  // namespace

struct stim_circuit {
  std::vector<Node> tree;
  Program prog;
  std::mutex mu;
  bool have_ref = false;
  std::vector<uint64_t> ref;
  std::map<int, DeviceCopy> dev;
  // Error sets (sparse detection sampling): built on first use; a circuit
  // they cannot serve keeps its error.
  bool have_em = false;
  int em_code = 0;
  std::string em_msg;
  ErrorModel em;
  uint32_t em_max_groups = 0;     // most 32-slot groups of one noise execution
  // Windowed sparse kernel: tile width (0: use the global-atomic kernel),
  // window rows and the batches of noise executions.
  int win_T = 0;
  uint32_t win_rows = 0;
  std::vector<uint32_t> wb_e0, wb_e1, wb_base;
};

namespace {

template <typename V>
hipError_t upload(const V &host, typename V::value_type **dst, hipStream_t s) {
  size_t bytes = std::max<size_t>(host.size(), 1) * sizeof(typename V::value_type);
  hipError_t e = hipMalloc((void **)dst, bytes);
  if (e != hipSuccess) return e;
  if (!host.empty()) e = hipMemcpyAsync(*dst, host.data(), host.size() * sizeof(typename V::value_type),
                                        hipMemcpyHostToDevice, s);
  return e;
}

// Circuits with at least this many qubits compute their reference sample on
// the GPU when a sampling call first needs it (STIM_GPU_REFERENCE = 0 / 1
// forces the host / the GPU).
constexpr uint64_t kGpuReferenceMinQubits = 1024;

int ensure_reference(stim_circuit *c, hipStream_t s = nullptr, bool allow_gpu = false) {
  if (c->have_ref) return STIM_OK;
  bool gpu = allow_gpu && c->prog.num_qubits >= kGpuReferenceMinQubits;
  if (const char *env = std::getenv("STIM_GPU_REFERENCE")) gpu = allow_gpu && std::atoi(env) != 0;
  if (gpu) {
    std::string err;
    std::vector<uint64_t> bits;
    int rc;
    try {
      rc = gpu_reference_sample(c->tree, c->prog.num_qubits, c->prog.num_measurements, bits, s, err);
    } catch (const std::bad_alloc &) {
      return set_error(STIM_E_OOM, "out of host memory planning the GPU reference sample");
    }
    if (rc == STIM_OK) {
      c->ref = std::move(bits);
      c->have_ref = true;
      return STIM_OK;
    }
    // A circuit the GPU planner does not take (too many unrolled steps) is
    // left to the host tableau, which walks it without unrolling it.
    if (rc != STIM_E_UNSUPPORTED) return set_error(rc, err);
  }
  try {
    c->ref = reference_sample(c->tree, c->prog.num_qubits, c->prog.num_measurements);
  } catch (const std::bad_alloc &) {
    return set_error(STIM_E_OOM, "out of host memory computing the reference sample");
  }
  c->have_ref = true;
  return STIM_OK;
}

// Uploads the program and reference to the current device (first use only).
// The per-call scratch (flip record, noise records, frame slots) comes from
// the device's stream-ordered pool.  Its memory is kept reserved between
// calls instead of being returned at every synchronisation, so that a steady
// stream of calls does not map and unmap gigabytes each time.
std::mutex g_pool_mu;
std::vector<int> g_pool_ready;

void keep_pool_reserved(int dev) {
  std::lock_guard<std::mutex> lock(g_pool_mu);
  if (std::find(g_pool_ready.begin(), g_pool_ready.end(), dev) != g_pool_ready.end()) return;
  g_pool_ready.push_back(dev);
  hipMemPool_t pool;
  if (hipDeviceGetDefaultMemPool(&pool, dev) == hipSuccess) {
    uint64_t keep = ~0ull;
    (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &keep);
  }
}

int ensure_device(stim_circuit *c, hipStream_t s, DeviceCopy **out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_error(e, "hipGetDevice");
  keep_pool_reserved(dev);
  auto it = c->dev.find(dev);
  if (it != c->dev.end()) {
    *out = &it->second;
    return STIM_OK;
  }
  DeviceCopy d;
  const Program &P = c->prog;
  if ((e = upload(P.ops, &d.ops, s)) != hipSuccess || (e = upload(P.event_ops, &d.event_ops, s)) != hipSuccess ||
      (e = upload(P.targets, &d.targets, s)) != hipSuccess ||
      (e = upload(P.thresholds, &d.thresholds, s)) != hipSuccess || (e = upload(c->ref, &d.ref, s)) != hipSuccess ||
      (e = upload(P.det_offsets, &d.det_off, s)) != hipSuccess ||
      (e = upload(P.det_indices, &d.det_idx, s)) != hipSuccess ||
      (e = upload(P.det_order, &d.det_order, s)) != hipSuccess ||
      (e = upload(P.det_blocks, &d.det_blocks, s)) != hipSuccess ||
      (e = upload(P.obs_offsets, &d.obs_off, s)) != hipSuccess ||
      (e = upload(P.obs_indices, &d.obs_idx, s)) != hipSuccess ||
      (e = upload(P.noise_pc, &d.noise_pc, s)) != hipSuccess ||
      (e = upload(P.noise_instr, &d.noise_instr, s)) != hipSuccess) {
    return e == hipErrorOutOfMemory ? set_error(STIM_E_OOM, "device allocation failed") : hip_error(e, "upload");
  }
  // Other streams may use this copy next: make sure the upload has landed.
  if ((e = hipStreamSynchronize(s)) != hipSuccess) return hip_error(e, "hipStreamSynchronize");
  c->dev[dev] = d;
  *out = &c->dev[dev];
  return STIM_OK;
}

void plan_window(stim_circuit *c);

void build_error_model_once(stim_circuit *c) {
  if (!c->have_em) {
    c->have_em = true;
    try {
      c->em = build_error_model(c->prog);
      for (uint32_t pc : c->prog.noise_pc) {
        const DevOp &op = c->prog.ops[pc];
        if (op.n >= (1u << 24)) throw CompileError{STIM_E_UNSUPPORTED, "noise instruction with 2^24 or more sites"};
        const uint32_t groups = ((op.slot0 + op.n - 1) >> 5) - (op.slot0 >> 5) + 1;
        c->em_max_groups = std::max(c->em_max_groups, groups);
      }
      plan_window(c);
    } catch (const CompileError &e) {
      c->em_code = e.code;
      c->em_msg = e.msg;
    } catch (const std::bad_alloc &) {
      c->em_code = STIM_E_OOM;
      c->em_msg = "out of host memory building the error sets";
    } catch (const std::exception &e) {
      c->em_code = STIM_E_UNSUPPORTED;
      c->em_msg = std::string("building the error sets failed: ") + e.what();
    }
  }
}

int ensure_error_model(stim_circuit *c) {
  build_error_model_once(c);
  return c->em_code ? set_error(c->em_code, c->em_msg) : STIM_OK;
}

// In the program without Z randomisations a reset leaves x = z = 0, and a
// Clifford maps a zero frame to zero, so a Clifford op all of whose qubits
// are zero for every shot changes nothing (for example H right after the
// reset of an ancilla): flags it OPF_ZERO_SKIP.  A forward pass over the
// program tracks which qubits are zero at each op: resets (R, MR, INIT)
// zero their targets, noise ops and classically controlled ops make theirs
// nonzero, M keeps the frame, and a Clifford's qubits stay zero only when
// all the qubits it couples are.  A loop body is analysed from the meet
// (qubit zero on every entry) of the state before the loop and at the end of
// the body, until the state at the body's start stops changing.
static void zero_pass(std::vector<DevOp> &ops, const std::vector<uint32_t> &tg, size_t lo, size_t hi,
                      std::vector<uint8_t> &zero, bool mark) {
  for (size_t pc = lo; pc < hi; pc++) {
    DevOp &op = ops[pc];
    const uint32_t code = op.code & 0xFFFFu;
    const uint32_t *t = tg.data() + op.toff;
    if (code == OP_LOOP_BEGIN) {
      const size_t end = op.aux2;                  // pc of the matching loop end
      std::vector<uint8_t> in = zero;
      for (int it = 0; it < 64; it++) {
        std::vector<uint8_t> st = in;
        zero_pass(ops, tg, pc + 1, end, st, false);
        bool changed = false;
        for (size_t q = 0; q < in.size(); q++) {
          const uint8_t m = in[q] & st[q];
          changed |= m != in[q];
          in[q] = m;
        }
        if (!changed) break;
      }
      zero = in;
      zero_pass(ops, tg, pc + 1, end, zero, mark);  // the state after the loop: the last pass's end
      pc = end;
      continue;
    }
    if (code == OP_INIT || code == OP_R || code == OP_MR) {
      for (uint32_t k = 0; k < op.n; k++) zero[t[k] & TGT_QUBIT_MASK] = 1;
    } else if (code == OP_M) {
      // M keeps the frame; one that always resets zeroes it (one that resets
      // only when its loop goes round again leaves zero qubits zero).
      if (op.code & OPF_M_RESETS)
        for (uint32_t k = 0; k < op.n; k++) zero[t[k] & TGT_QUBIT_MASK] = 1;
    } else if (code >= OP_SWAP_XZ && code <= OP_SWAP) {
      const bool two = code >= OP_CX;
      bool all = true;
      for (uint32_t k = 0; k < op.n * (two ? 2u : 1u); k++) all &= zero[t[k]] != 0;
      if (two)
        for (uint32_t k = 0; k < op.n; k++) {
          const bool z = zero[t[2 * k]] && zero[t[2 * k + 1]];
          zero[t[2 * k]] = zero[t[2 * k + 1]] = z;
        }
      if (mark && all) op.code |= OPF_ZERO_SKIP;
    } else if ((code >= OP_NOISE_X && code <= OP_NOISE_DEP2) || (code >= OP_FB_X && code <= OP_FB_Z)) {
      const uint32_t per = code == OP_NOISE_DEP2 ? 2u : 1u, stride = code >= OP_FB_X ? 2u : 1u;
      for (uint32_t k = 0; k < op.n * per; k++) zero[t[k * stride] & TGT_QUBIT_MASK] = 0;
    }
  }
}

static void mark_zero_frame_ops(std::vector<DevOp> &ops, const std::vector<uint32_t> &tg, uint64_t n) {
  std::vector<uint8_t> zero(n, 0);
  zero_pass(ops, tg, 0, ops.size(), zero, true);
}

// Detection events without the collapses' Z randomisations (Sec. 3, 5.6).
// The frame is linear over GF(2) in its random bits, so the Z randomisation
// drawn after a collapse adds to the events exactly the detector set of a Z
// error at that point.  When every detector and observable is deterministic
// -- the condition the error-set walk checks: no output is sensitive to an X
// component on a qubit right after its collapse -- all those sets are empty,
// and a detector-mode walk may skip every such draw: the events are the same
// bits, only the intermediate flips of random measurements differ.  Built
// once per device, with the caller holding c->mu; not for circuits the walk
// refuses (random outputs, classically controlled Paulis, circuits too long
// to walk), nor with STIM_EVENT_ZRAND=1.
int ensure_noz_program(stim_circuit *c, DeviceCopy *d, hipStream_t s) {
  if (d->noz_checked) return STIM_OK;
  const char *env = std::getenv("STIM_EVENT_ZRAND");
  if (env && std::strcmp(env, "1") == 0) return STIM_OK;     // not recorded: the switch may change
  d->noz_checked = true;
  const Program &P = c->prog;
  if (P.num_detectors + P.num_observables == 0) return STIM_OK;
  build_error_model_once(c);
  if (c->em_code) return STIM_OK;
  std::vector<DevOp> ops = P.ops;
  std::vector<uint32_t> tg = P.targets;
  for (DevOp &op : ops) {
    const uint32_t code = op.code & 0xFFFFu;
    if (code != OP_INIT && code != OP_R && code != OP_M && code != OP_MR) continue;
    op.code &= ~OPF_ZRAND_LIVE;
    for (uint32_t k = 0; k < op.n; k++) tg[(size_t)op.toff + k] |= TGT_DEAD_ZRAND;
  }
  // M followed by an R of the same qubits: the M resets them (see OPF_M_RESETS).
  auto same_qubits = [&](const DevOp &a, const DevOp &b) {
    if (a.n != b.n) return false;
    std::vector<uint32_t> x(tg.begin() + a.toff, tg.begin() + a.toff + a.n);
    std::vector<uint32_t> y(tg.begin() + b.toff, tg.begin() + b.toff + b.n);
    std::sort(x.begin(), x.end());
    std::sort(y.begin(), y.end());
    return x == y;
  };
  auto is_r = [&](size_t pc) { return pc < ops.size() && (ops[pc].code & 0xFFFFu) == OP_R; };
  for (size_t pc = 0; pc + 1 < ops.size(); pc++) {
    if ((ops[pc].code & 0xFFFFu) != OP_M) continue;
    const uint32_t next = ops[pc + 1].code & 0xFFFFu;
    size_t r = 0;
    uint32_t flag = 0;
    if (is_r(pc + 1)) {
      r = pc + 1;
      flag = OPF_M_RESETS;
    } else if (next == OP_LOOP_BEGIN && is_r(pc + 2)) {
      r = pc + 2;
      flag = OPF_M_RESETS;
    } else if (next == OP_LOOP_END && is_r((size_t)ops[pc + 1].aux + 1)) {
      r = (size_t)ops[pc + 1].aux + 1;
      flag = OPF_M_RESETS_IN_LOOP;
    }
    if (flag && same_qubits(ops[pc], ops[r])) {
      ops[pc].code |= flag;
      ops[r].code |= OPF_R_AFTER_M;
    }
  }
  mark_zero_frame_ops(ops, tg, P.num_qubits);
  hipError_t e;
  DevOp *dops = nullptr;
  uint32_t *dtg = nullptr;
  if ((e = upload(ops, &dops, s)) != hipSuccess || (e = upload(tg, &dtg, s)) != hipSuccess) {
    if (dops) (void)hipFree(dops);
    return e == hipErrorOutOfMemory ? set_error(STIM_E_OOM, "device allocation failed") : hip_error(e, "upload");
  }
  if ((e = hipStreamSynchronize(s)) != hipSuccess) return hip_error(e, "hipStreamSynchronize");
  d->noz_ops = dops;
  d->noz_targets = dtg;
  return STIM_OK;
}

// Plans the windowed sparse kernel: batches of consecutive noise executions
// such that, before a batch, every detector row below its base is final (no
// later execution touches it) and every row touched so far but not final
// fits in the window.  Tries T = 2, then T = 1; leaves win_T = 0 when the
// window does not fit (the global-atomic kernel is used instead).
//
// Choice between the two kernels: the windowed one writes every output word
// once from LDS but pays per-batch barriers and 16-byte row pieces; the
// global one zeroes the outputs at full bandwidth and then pays one global
// atomic per (error, flipped output).  The second wins when the expected
// flipped outputs per shot are a small fraction of the detectors: below
// kWindowMinDensity the global kernel is used.  STIM_SPARSE_WINDOW = 0 / 1
// forces either kernel.
constexpr double kWindowMinDensity = 0.005;

void plan_window(stim_circuit *c) {
  c->win_T = 0;
  const char *env = std::getenv("STIM_SPARSE_WINDOW");
  if (env && std::atoi(env) == 0) return;
  const bool forced = env && std::atoi(env) == 1;
  const Program &P = c->prog;
  const ErrorModel &em = c->em;
  const uint64_t D = P.num_detectors, L = P.num_observables;
  if (L > kWindowMaxObs || D >= (1ull << 31)) return;
  const size_t E = em.gen_base.size();
  std::vector<int64_t> lo(E, (int64_t)D), hi(E, -1);
  double flips_per_shot = 0;
  for (size_t e = 0; e < E; e++) {
    const uint64_t g1 = e + 1 < E ? em.gen_base[e + 1] : em.num_generators;
    const DevOp &op = P.ops[P.noise_pc[e]];
    const double pe = (double)(0ull - P.thresholds[(size_t)op.aux * 64]) * 0x1p-64;
    // An error activates about half of its site's generators.
    flips_per_shot += pe * 0.5 * (double)(em.set_off[g1] - em.set_off[em.gen_base[e]]);
    for (uint64_t a = em.set_off[em.gen_base[e]]; a < em.set_off[g1]; a++) {
      const int64_t l = em.set_lanes[a];
      if (l >= (int64_t)D) continue;
      lo[e] = std::min(lo[e], l);
      hi[e] = std::max(hi[e], l);
    }
  }
  if (!forced && flips_per_shot < kWindowMinDensity * (double)std::max<uint64_t>(D, 1)) return;
  std::vector<int64_t> suf(E + 1, (int64_t)D);
  for (size_t e = E; e-- > 0;) suf[e] = std::min(suf[e + 1], lo[e]);
  int order[2] = {2, 1};
  if (const char *t = std::getenv("STIM_SPARSE_T")) {
    const int v = std::atoi(t);
    if (v == 1 || v == 2) order[0] = order[1] = v;
  }
  for (int T : order) {
    const int64_t cap = sparse_window_max_rows(T, (uint32_t)L);
    if (cap <= 0) continue;
    std::vector<uint32_t> e0s, e1s, bases;
    int64_t H = -1, need = 1;
    bool ok = true;
    for (size_t e = 0; e < E && ok;) {
      const int64_t base = suf[e];
      size_t e1 = e;
      int64_t Hb = H;
      while (e1 < E && e1 - e < kWindowMaxExec) {
        const int64_t h = std::max(Hb, hi[e1]);
        if (h >= base && h - base + 1 > cap) break;
        Hb = h;
        e1++;
      }
      if (e1 == e) ok = false;
      else {
        if (Hb >= base) need = std::max(need, Hb - base + 1);
        e0s.push_back((uint32_t)e);
        e1s.push_back((uint32_t)e1);
        bases.push_back((uint32_t)base);
        H = Hb;
        e = e1;
      }
    }
    if (!ok) continue;
    c->win_T = T;
    c->win_rows = (uint32_t)need;
    c->wb_e0 = std::move(e0s);
    c->wb_e1 = std::move(e1s);
    c->wb_base = std::move(bases);
    return;
  }
}

int ensure_sparse_device(stim_circuit *c, DeviceCopy *d, hipStream_t s) {
  if (d->set_off) return STIM_OK;
  hipError_t e;
  if ((e = upload(c->em.gen_base, &d->gen_base, s)) != hipSuccess ||
      (e = upload(c->em.set_off, &d->set_off, s)) != hipSuccess ||
      (e = upload(c->em.set_lanes, &d->set_lanes, s)) != hipSuccess ||
      (e = upload(c->wb_e0, &d->wb_e0, s)) != hipSuccess || (e = upload(c->wb_e1, &d->wb_e1, s)) != hipSuccess ||
      (e = upload(c->wb_base, &d->wb_base, s)) != hipSuccess)
    return e == hipErrorOutOfMemory ? set_error(STIM_E_OOM, "device allocation failed") : hip_error(e, "upload");
  if ((e = hipStreamSynchronize(s)) != hipSuccess) return hip_error(e, "hipStreamSynchronize");
  return STIM_OK;
}

bool is_device_pointer(const void *p) {
  if (!p) return false;
  hipPointerAttribute_t a;
  if (hipPointerGetAttributes(&a, p) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  return a.type == hipMemoryTypeDevice || a.type == hipMemoryTypeManaged || a.type == hipMemoryTypeUnified;
}

uint32_t threads_for(size_t frame_bytes) {
  return frame_bytes > 80 * 1024 ? 1024 : frame_bytes > 40 * 1024 ? 512 : 256;
}

bool fits_lds(uint64_t n, int T) {
  size_t fb = (size_t)16 * n * T;
  return frame_lds_bytes(n, T, true, threads_for(fb)) <= kMaxLdsBytes;
}

// Picks the shot-tile width and frame placement: the widest tile whose frame
// slice fits in LDS while still giving enough tiles to occupy the GPU.
// STIM_TILE_WORDS (1..32, power of two), STIM_FRAME_PLACEMENT (lds|global)
// and STIM_FRAME_THREADS override the choice; results do not depend on it.
FrameConfig choose_config(uint64_t n, uint64_t W) {
  FrameConfig cfg{1, true, 256};
  const char *tw = std::getenv("STIM_TILE_WORDS"), *pl = std::getenv("STIM_FRAME_PLACEMENT");
  if (tw || pl) {
    int T = tw ? std::atoi(tw) : 1;
    if (T != 1 && T != 2 && T != 4 && T != 8 && T != 16 && T != 32) T = 1;
    bool lds = pl ? std::strcmp(pl, "global") != 0 : true;
    if (lds && !fits_lds(n, T)) lds = false;
    cfg.tile_words = T;
    cfg.in_lds = lds;
    cfg.threads = lds ? threads_for((size_t)16 * n * T) : 256;
    if (const char *th = std::getenv("STIM_FRAME_THREADS")) {
      const int t = std::atoi(th);
      if (t >= 64 && t <= 1024 && t % 64 == 0 && frame_lds_bytes(n, T, lds, (uint32_t)t) <= kMaxLdsBytes)
        cfg.threads = (uint32_t)t;
    }
    return cfg;
  }
  const int widths[] = {32, 16, 8, 4, 2, 1};
  for (int T : widths) {
    uint64_t tiles = (W + T - 1) / T;
    if (fits_lds(n, T) && (tiles >= 512 || T == 1)) {
      cfg.tile_words = T;
      cfg.in_lds = true;
      cfg.threads = threads_for((size_t)16 * n * T);
      return cfg;
    }
  }
  if (fits_lds(n, 1)) return cfg;
  // Frame slice too large for LDS even for one word: global scratch.  Wider
  // tiles make each frame access a longer contiguous piece; measured at
  // d = 101: 8 words per tile once there are at least 256 tiles of them, else
  // 4, else 2 (512 threads; about one workgroup per CU in flight).
  cfg.in_lds = false;
  cfg.threads = 512;
  cfg.tile_words = W >= 2048 ? 8 : W >= 1024 ? 4 : W >= 128 ? 2 : 1;
  return cfg;
}

// Pinned host buffers for uploading per-launch tables without blocking the
// host: a buffer is reused only after the copy that read it has completed.
// Sampling calls may come from several host threads at once (one stream
// each), so the pool is taken under a lock for the whole pick-copy-record
// sequence.
struct StagingBuffer {
  void *ptr = nullptr;
  size_t cap = 0;
  hipEvent_t done = nullptr;
  bool busy = false;
};
std::mutex g_staging_mu;
std::vector<StagingBuffer> g_staging;

int stage_upload(const void *src, size_t bytes, void *dst, hipStream_t s) {
  std::lock_guard<std::mutex> lock(g_staging_mu);
  StagingBuffer *buf = nullptr;
  for (StagingBuffer &b : g_staging) {
    if (b.busy && hipEventQuery(b.done) == hipSuccess) b.busy = false;
    if (!b.busy && b.cap >= bytes && !buf) buf = &b;
  }
  if (!buf) {
    for (StagingBuffer &b : g_staging)
      if (!b.busy && !buf) buf = &b;
    if (!buf) {
      g_staging.emplace_back();
      buf = &g_staging.back();
      if (hipEventCreateWithFlags(&buf->done, hipEventDisableTiming) != hipSuccess) {
        g_staging.pop_back();
        return set_error(STIM_E_DEVICE, "hipEventCreate failed");
      }
    }
    if (buf->cap < bytes) {
      if (buf->ptr) (void)hipHostFree(buf->ptr);
      buf->ptr = nullptr;
      buf->cap = 0;
      size_t cap = std::max<size_t>(bytes, 1 << 16);
      if (hipHostMalloc(&buf->ptr, cap, hipHostMallocDefault) != hipSuccess)
        return set_error(STIM_E_OOM, "pinned staging allocation failed");
      buf->cap = cap;
    }
  }
  std::memcpy(buf->ptr, src, bytes);
  hipError_t e = hipMemcpyAsync(dst, buf->ptr, bytes, hipMemcpyHostToDevice, s);
  if (e != hipSuccess) return hip_error(e, "table upload");
  if ((e = hipEventRecord(buf->done, s)) != hipSuccess) return hip_error(e, "hipEventRecord");
  buf->busy = true;
  return STIM_OK;
}

int check_sample_args(stim_circuit *c, uint64_t shot_offset, uint64_t num_shots) {
  if (!c) return set_error(STIM_E_INVALID_ARG, "null circuit handle");
  if (num_shots == 0) return set_error(STIM_E_INVALID_ARG, "num_shots must be positive");
  if (shot_offset % 64) return set_error(STIM_E_INVALID_ARG, "shot_offset must be a multiple of 64");
  if (c->prog.max_loop_depth > 8) return set_error(STIM_E_UNSUPPORTED, "REPEAT nesting deeper than 8");
  if (c->prog.num_qubits >= (1ull << 31)) return set_error(STIM_E_UNSUPPORTED, "too many qubits");
  return STIM_OK;
}

// Optional per-kernel timing: HIP events recorded on the launch stream around
// the noise pre-pass and the frame kernel of every sampling pass.
struct PassEvents {
  hipEvent_t start, mid, end;
  bool prepass;
};
std::mutex g_timing_mu;
bool g_timing_on = false;
std::vector<PassEvents> g_timing;

void release_timing() {
  for (PassEvents &t : g_timing) {
    (void)hipEventDestroy(t.start);
    (void)hipEventDestroy(t.mid);
    (void)hipEventDestroy(t.end);
  }
  g_timing.clear();
}

// Compute units of a device (cached; callers may be on several host threads).
std::mutex g_cu_mu;
std::map<int, int> g_cu_count;
int cu_count(int dev) {
  std::lock_guard<std::mutex> lock(g_cu_mu);
  auto it = g_cu_count.find(dev);
  if (it != g_cu_count.end()) return it->second;
  hipDeviceProp_t prop;
  int n = 256;
  if (hipGetDeviceProperties(&prop, dev) == hipSuccess && prop.multiProcessorCount > 0) n = prop.multiProcessorCount;
  g_cu_count[dev] = n;
  return n;
}

// Noise pre-pass reservations at tile width T over `ntiles` tiles: for each
// noise execution, mean + 6 sigma + 16 records per tile for the expected
// number of words whose prefix admits an error (0 = too many for one
// workgroup's queue: that execution stays inline), and its first record.
// Returns the total number of records.
constexpr uint64_t kMaxRecordBytes = 8ull << 30;
constexpr size_t kMaxGenInstances = 65535;          // noise executions per pre-pass launch (grid rows)

uint64_t noise_reservations(const Program &P, int T, uint64_t ntiles, std::vector<uint32_t> &cap,
                            std::vector<uint64_t> &base, uint32_t &max_cap) {
  const size_t ninst = P.noise_pc.size();
  cap.assign(ninst, 0);
  base.assign(ninst, 0);
  max_cap = 1;
  uint64_t nrec = 0;
  for (size_t i = 0; i < ninst; i++) {
    const DevOp &op = P.ops[P.noise_pc[i]];
    const uint64_t cut = P.thresholds[(size_t)op.aux * 64 + 63] >> 56;
    const double q = (256.0 - (double)cut) / 256.0;
    const double mu = (double)op.n * T * q;
    const double capd = std::ceil(mu + 6.0 * std::sqrt(mu) + 16.0);
    cap[i] = capd > (double)kGenQueue ? 0u : (uint32_t)capd;
    max_cap = std::max(max_cap, cap[i]);
    base[i] = nrec;
    nrec += (uint64_t)cap[i] * ntiles;
  }
  return nrec;
}

// Whether a pass over `ntiles` tiles precomputes its noise (records hold
// 27-bit qubit indices; one pre-pass launch covers 65,535 noise executions).
bool prepass_enabled(const Program &P, uint64_t ntiles) {
  const size_t ninst = P.noise_pc.size();
  const char *pre_env = std::getenv("STIM_NOISE_PREPASS");
  return ninst > 0 && ninst <= kMaxGenInstances && !(pre_env && std::strcmp(pre_env, "0") == 0) &&
         ntiles <= 0x7FFFFFFFull && P.num_qubits < (1ull << 27);
}

// Workgroups in flight (each with its own scratch slot) for a frame kept in
// global memory: about one per CU, so that the frames stay in the caches.
uint64_t global_frame_slots(int dev, uint64_t ntiles) {
  uint64_t slots = (uint64_t)cu_count(dev);
  if (const char *v = std::getenv("STIM_FRAME_SLOTS")) slots = std::max<long>(1, atol(v));
  return std::min<uint64_t>(slots, ntiles);
}

// Device scratch one sampling pass of num_shots allocates: noise records and
// their tables, and the global frame slots of circuits too large for LDS.
uint64_t pass_scratch_bytes(const Program &P, uint64_t num_shots, int dev) {
  const uint64_t W = (num_shots + 63) / 64;
  const FrameConfig cfg = choose_config(P.num_qubits, W);
  const uint64_t ntiles = (W + cfg.tile_words - 1) / cfg.tile_words;
  uint64_t bytes = 0;
  if (prepass_enabled(P, ntiles)) {
    std::vector<uint32_t> cap;
    std::vector<uint64_t> base;
    uint32_t max_cap = 1;
    const uint64_t nrec = noise_reservations(P, cfg.tile_words, ntiles, cap, base, max_cap);
    const uint64_t ninst = P.noise_pc.size();
    if (nrec > 0 && nrec * 16 <= kMaxRecordBytes) bytes += ninst * ntiles * sizeof(uint2) + ninst * 12 + nrec * 16;
  }
  if (!cfg.in_lds)
    bytes += global_frame_slots(dev, ntiles) * cfg.tile_words * 16 * (P.num_qubits + 1);
  return bytes;
}

// Detection events formed in the walk (Sec. 5.6), on request
// (STIM_WALK_EVENTS=1): each workgroup keeps its recent flips in a ring of
// max_lookback + max_measure_op rows (at most the record's length) of T
// words, and detector and observable ops write the event tables directly, so
// the flip record is never written out and read back.  Rings are per
// workgroup slot: one workgroup per tile for an LDS-resident frame (capped by
// a memory budget, beyond which workgroups take several tiles in turn), the
// global frame's slots otherwise.  Not the default: the rings live in global
// memory (the LDS holds the frame), and on surface codes from d = 3 to 49
// their traffic through L2 cost the walk as much as the event kernel it
// saves, or more.  STIM_WALK_EVENT_SLOTS caps the slots (workgroups then take
// tiles in turn).
constexpr uint64_t kRingBudget = 512ull << 20;

struct WalkEvents {
  uint64_t *det_out = nullptr, *obs_out = nullptr;
  uint32_t num_obs = 0;
};

// A ring as long as the whole record never wraps: no longer is needed.
uint32_t ring_rows(const Program &P) {
  const uint64_t r = std::min<uint64_t>((uint64_t)P.max_lookback + P.max_measure_op, P.num_measurements);
  return (uint32_t)std::max<uint64_t>(1, r);
}

// Ring slots of a walk with events for num_shots shots (0: not possible).
uint64_t walk_event_slots(const Program &P, uint64_t num_shots, int dev) {
  const char *env = std::getenv("STIM_WALK_EVENTS");
  if (!env || std::strcmp(env, "1") != 0) return 0;
  if (P.num_detectors + P.num_observables == 0) return 0;
  if ((uint64_t)P.max_lookback + P.max_measure_op >= (1ull << 31)) return 0;
  const uint64_t W = (num_shots + 63) / 64;
  const FrameConfig cfg = choose_config(P.num_qubits, W);
  const uint64_t ntiles = (W + cfg.tile_words - 1) / cfg.tile_words;
  const uint64_t slot_bytes = (uint64_t)ring_rows(P) * cfg.tile_words * sizeof(uint64_t);
  uint64_t slots;
  if (cfg.in_lds) {
    const uint64_t fit = kRingBudget / slot_bytes;
    slots = std::min<uint64_t>(ntiles, std::max<uint64_t>(fit, (uint64_t)cu_count(dev)));
  } else {
    slots = global_frame_slots(dev, ntiles);
  }
  if (const char *v = std::getenv("STIM_WALK_EVENT_SLOTS")) slots = std::min<uint64_t>(slots, std::max(1L, atol(v)));
  if (slots == 0 || slots > 0xFFFFFFFFull || slots * slot_bytes > kRingBudget) return 0;
  return slots;
}

uint64_t walk_event_bytes(const Program &P, uint64_t num_shots, int dev) {
  const uint64_t slots = walk_event_slots(P, num_shots, dev);
  const FrameConfig cfg = choose_config(P.num_qubits, (num_shots + 63) / 64);
  return slots * ring_rows(P) * cfg.tile_words * sizeof(uint64_t);
}

// Runs the frame kernel; ref == nullptr writes raw flips.  With `ev`, the walk
// forms detection events and observables instead of writing `out`.
int run_frame(stim_circuit *c, DeviceCopy *d, uint64_t seed, uint64_t shot_offset, uint64_t num_shots,
              const uint64_t *ref, uint64_t *out, hipStream_t s, const WalkEvents *ev = nullptr,
              bool noz = false) {
  const uint64_t W = (num_shots + 63) / 64;
  FrameConfig cfg = choose_config(c->prog.num_qubits, W);
  FrameParams p{};
  // noz: the detector-mode program without Z randomisations (same op list).
  const bool use_noz = noz && d->noz_ops != nullptr;
  p.ops = use_noz ? d->noz_ops : d->ops;
  p.noz = use_noz && ev == nullptr;          // also picks the records table layout below
  p.num_ops = (uint32_t)c->prog.ops.size();
  p.num_qubits = (uint32_t)c->prog.num_qubits;
  p.targets = use_noz ? d->noz_targets : d->targets;
  p.thresholds = d->thresholds;
  p.ref = ref;
  p.seed = seed;
  p.word0 = shot_offset / 64;
  p.num_words = W;
  uint64_t rem = num_shots % 64;
  p.tail_mask = rem ? ((1ull << rem) - 1) : ~0ull;
  p.out = out;
  p.out_stride = W;
  p.scratch = nullptr;
  hipError_t e;
  const uint64_t ntiles = (W + cfg.tile_words - 1) / cfg.tile_words;
  // Noise pre-pass: reserve mean + 6 sigma + 16 records per (noise execution,
  // tile) for the expected number of words whose prefix admits an error; ops
  // whose reservation would exceed one workgroup's queue stay inline.
  const Program &P = c->prog;
  const size_t ninst = P.noise_pc.size();
  bool prepass = prepass_enabled(P, ntiles);
  std::vector<uint64_t> nbase;
  std::vector<uint32_t> ncap;
  uint64_t nrec = 0;
  uint32_t max_cap = 1;
  if (prepass) {
    nrec = noise_reservations(P, cfg.tile_words, ntiles, ncap, nbase, max_cap);
    if (nrec == 0 || nrec * 16 > kMaxRecordBytes) prepass = false;
  }
  uint2 *d_meta = nullptr;
  uint32_t *d_cap = nullptr;
  uint64_t *d_base = nullptr;
  uint4 *d_rec = nullptr;
  auto free_prepass = [&]() {
    void *ptrs[] = {d_meta, d_cap, d_base, d_rec};
    for (void *q : ptrs) if (q) (void)hipFreeAsync(q, s);
  };
  PassEvents tev{};
  bool timed = false;
  {
    std::lock_guard<std::mutex> lock(g_timing_mu);
    if (g_timing_on && g_timing.size() < 4096) {
      timed = hipEventCreate(&tev.start) == hipSuccess;
      if (timed && hipEventCreate(&tev.mid) != hipSuccess) {
        (void)hipEventDestroy(tev.start);
        timed = false;
      }
      if (timed && hipEventCreate(&tev.end) != hipSuccess) {
        (void)hipEventDestroy(tev.start);
        (void)hipEventDestroy(tev.mid);
        timed = false;
      }
    }
  }
  auto drop_events = [&]() {
    if (!timed) return;
    (void)hipEventDestroy(tev.start);
    (void)hipEventDestroy(tev.mid);
    (void)hipEventDestroy(tev.end);
    timed = false;
  };
  if (prepass) {
    if ((e = hipMallocAsync((void **)&d_meta, ninst * ntiles * sizeof(uint2), s)) != hipSuccess ||
        (e = hipMallocAsync((void **)&d_cap, ninst * sizeof(uint32_t), s)) != hipSuccess ||
        (e = hipMallocAsync((void **)&d_base, ninst * sizeof(uint64_t), s)) != hipSuccess ||
        (e = hipMallocAsync((void **)&d_rec, nrec * 16, s)) != hipSuccess) {
      free_prepass();
      drop_events();
      return set_error(STIM_E_OOM, "noise record allocation failed");
    }
    int rc = stage_upload(ncap.data(), ninst * sizeof(uint32_t), d_cap, s);
    if (!rc) rc = stage_upload(nbase.data(), ninst * sizeof(uint64_t), d_base, s);
    if (rc) {
      free_prepass();
      drop_events();
      return rc;
    }
    NoiseGenParams g{};
    g.ops = d->ops;
    g.targets = d->targets;
    g.thresholds = d->thresholds;
    g.inst_pc = d->noise_pc;
    g.inst_instr = d->noise_instr;
    g.base = d_base;
    g.cap = d_cap;
    g.seed = seed;
    g.word0 = p.word0;
    g.num_words = W;
    g.tiles = (uint32_t)ntiles;
    // Tile-major records table for the walk of the program without Z
    // randomisations, execution-major for the others.
    g.tile_stride = p.noz ? (uint32_t)ninst : 1u;
    g.inst_stride = p.noz ? 1u : (uint32_t)ntiles;
    g.meta = d_meta;
    g.rec = d_rec;
    // Each workgroup takes as many tiles of one execution as its LDS queue
    // holds at the largest reservation, so that its lanes stay busy.
    // (STIM_GEN_TILES and STIM_GEN_THREADS override the choice, for tuning.)
    uint32_t want_tiles = kGenTiles, gen_threads = 512;
    if (const char *v = std::getenv("STIM_GEN_TILES")) want_tiles = std::max(1, std::min(atoi(v), (int)kGenTiles));
    if (const char *v = std::getenv("STIM_GEN_THREADS")) {
      const int t = atoi(v);
      if (t >= 64 && t <= 512 && t % 64 == 0) gen_threads = (uint32_t)t;
    }
    g.tiles_per_group = std::max<uint32_t>(1, std::min<uint32_t>(want_tiles, kGenQueue / max_cap));
    g.queue_per_tile = kGenQueue / g.tiles_per_group;
    if (timed) (void)hipEventRecord(tev.start, s);
    if ((e = launch_noise_gen(g, cfg.tile_words, (uint32_t)ninst, gen_threads, s)) != hipSuccess) {
      free_prepass();
      drop_events();
      return hip_error(e, "noise pre-pass launch");
    }
    p.noise_meta = d_meta;
    p.noise_rec = d_rec;
    p.noise_tiles = (uint32_t)ntiles;
    p.noise_instances = (uint32_t)ninst;
  }
  int dev = 0;
  (void)hipGetDevice(&dev);
  if (!cfg.in_lds) {
    // One scratch slot per workgroup in flight: about one workgroup per CU, so
    // that the frames in flight stay within the last-level cache.
    cfg.slots = (uint32_t)global_frame_slots(dev, ntiles);
    const uint64_t tiles = cfg.slots;
    size_t bytes = (size_t)tiles * cfg.tile_words * 16 * (c->prog.num_qubits + 1);     // + the dummy row
    if ((e = hipMallocAsync((void **)&p.scratch, bytes, s)) != hipSuccess) {
      free_prepass();
      drop_events();
      return set_error(STIM_E_OOM, "frame scratch allocation failed");
    }
  }
  if (ev) {
    const uint64_t slots = walk_event_slots(P, num_shots, dev);
    if (slots == 0) {
      if (p.scratch) (void)hipFreeAsync(p.scratch, s);
      free_prepass();
      drop_events();
      return set_error(STIM_E_UNSUPPORTED, "detection events cannot be formed in the walk");
    }
    cfg.slots = (uint32_t)slots;
    p.ops = d->event_ops;
    p.noz = false;
    p.num_ops = (uint32_t)P.event_ops.size();
    p.ring_rows = ring_rows(P);
    p.det_out = ev->det_out;
    p.obs_out = ev->obs_out;
    p.num_obs = ev->obs_out ? ev->num_obs : 0;
    p.out = nullptr;
    if ((e = hipMallocAsync((void **)&p.ring, slots * p.ring_rows * cfg.tile_words * sizeof(uint64_t), s)) !=
        hipSuccess) {
      if (p.scratch) (void)hipFreeAsync(p.scratch, s);
      free_prepass();
      drop_events();
      return set_error(STIM_E_OOM, "flip ring allocation failed");
    }
  }
  if (c->prog.num_measurements > 0 || c->prog.num_qubits > 0) {
    if (timed) {
      if (!prepass) (void)hipEventRecord(tev.start, s);
      (void)hipEventRecord(tev.mid, s);
    }
    if ((e = launch_frame(p, cfg, s)) != hipSuccess) {
      if (p.scratch) (void)hipFreeAsync(p.scratch, s);
      if (p.ring) (void)hipFreeAsync(p.ring, s);
      free_prepass();
      drop_events();
      return hip_error(e, "frame kernel launch");
    }
    if (timed) {
      (void)hipEventRecord(tev.end, s);
      tev.prepass = prepass;
      std::lock_guard<std::mutex> lock(g_timing_mu);
      g_timing.push_back(tev);
      timed = false;
    }
  }
  drop_events();
  free_prepass();
  if (p.scratch && (e = hipFreeAsync(p.scratch, s)) != hipSuccess) return hip_error(e, "hipFreeAsync");
  if (p.ring && (e = hipFreeAsync(p.ring, s)) != hipSuccess) return hip_error(e, "hipFreeAsync");
  return STIM_OK;
}

// ---------------------------------------------------------------------------
// Batched launches.
// ---------------------------------------------------------------------------

// Request set + device tables + captured graph, reused when the same request
// set is submitted again.
struct BatchPlan {
  int device = 0;
  std::vector<stim_request> reqs;
  std::vector<size_t> batched, single;        // request indices inside / outside the persistent launch
  FrameConfig cfg{1, true, 256};
  uint64_t max_n = 0;
  uint32_t blocks = 0, num_items = 0;
  FrameParams *d_params = nullptr;
  BatchItem *d_items = nullptr;
  uint32_t *d_counter = nullptr;
  uint64_t *d_flips = nullptr;
  std::vector<uint64_t *> flips;              // per request (detector mode) or nullptr
  hipGraphExec_t exec = nullptr;
  hipGraph_t graph = nullptr;
  double tuned_ms = 0;
  // Noise pre-pass of each batched noisy request (as in the single-request
  // path): records and meta entries sized for every candidate tile width,
  // reservations per width (index log2 of the width: 1, 2, 4, 8).
  struct Noise {
    uint2 *meta = nullptr;
    uint4 *rec = nullptr;
    uint32_t *cap[4] = {nullptr, nullptr, nullptr, nullptr};
    uint64_t *base[4] = {nullptr, nullptr, nullptr, nullptr};
    uint32_t max_cap[4] = {1, 1, 1, 1};
    uint32_t ninst = 0, stride = 0;
  };
  std::vector<Noise> noise;                   // per request; meta == nullptr: noise drawn inline
};

int width_index(int T) { return T == 1 ? 0 : T == 2 ? 1 : T == 4 ? 2 : 3; }

void free_batch_noise(BatchPlan &pl, hipStream_t s, bool async) {
  for (BatchPlan::Noise &nz : pl.noise) {
    std::vector<void *> ptrs = {nz.meta, nz.rec};
    for (int k = 0; k < 4; k++) {
      ptrs.push_back(nz.cap[k]);
      ptrs.push_back(nz.base[k]);
    }
    for (void *q : ptrs)
      if (q) (void)(async ? hipFreeAsync(q, s) : hipFree(q));
  }
  pl.noise.clear();
}

std::mutex g_batch_mu;
std::vector<std::unique_ptr<BatchPlan>> g_plans;           // most recent last
std::map<std::string, FrameConfig> g_tuned;                // shape class -> config
std::vector<uint64_t> g_seen;                               // signatures of recent one-shot request sets
std::string g_tune_cache_read;                              // cache file last read

// Tuned configurations persist across processes in the text file named by
// STIM_TUNE_CACHE (one "class tile_words threads" line per tuned shape class;
// a later line for a class wins).  Read by the first batched launch that sees
// the variable name that file; each newly tuned class is appended.  Called
// with g_batch_mu held.
void load_tune_cache() {
  const char *path = std::getenv("STIM_TUNE_CACHE");
  if (!path || !*path || g_tune_cache_read == path) return;
  g_tune_cache_read = path;
  FILE *f = std::fopen(path, "r");
  if (!f) return;
  char cls[128];
  int T = 0;
  unsigned threads = 0;
  while (std::fscanf(f, "%127s %d %u", cls, &T, &threads) == 3) {
    // 64 threads names the one-wave-per-tile kernel.
    if ((T == 1 || T == 2 || T == 4 || T == 8) && threads >= 64 && threads <= 1024 && threads % 64 == 0) {
      FrameConfig cfg{T, true, threads};
      cfg.wave = threads == 64;
      g_tuned[cls] = cfg;
    }
  }
  std::fclose(f);
}

void save_tuned(const std::string &cls, const FrameConfig &cfg) {
  g_tuned[cls] = cfg;
  const char *path = std::getenv("STIM_TUNE_CACHE");
  if (!path || !*path) return;
  if (FILE *f = std::fopen(path, "a")) {
    std::fprintf(f, "%s %d %u\n", cls.c_str(), cfg.tile_words, cfg.wave ? 64u : cfg.threads);
    std::fclose(f);
  }
}

void free_plan(BatchPlan *pl) {
  if (pl->exec) (void)hipGraphExecDestroy(pl->exec);
  if (pl->graph) (void)hipGraphDestroy(pl->graph);
  void *ptrs[] = {pl->d_params, pl->d_items, pl->d_counter, pl->d_flips};
  for (void *q : ptrs) if (q) (void)hipFree(q);
  free_batch_noise(*pl, nullptr, false);
}

// Sets up the noise pre-pass of every batched noisy request for the tile
// widths in `widths` (device memory from the stream-ordered pool when
// `async`, else plain allocations kept with the plan).  A request whose
// records would exceed the per-pass limit keeps drawing its noise inline.
int prepare_batch_noise(BatchPlan &pl, const std::vector<int> &widths, hipStream_t s, bool async) {
  pl.noise.assign(pl.reqs.size(), BatchPlan::Noise{});
  const char *pre_env = std::getenv("STIM_NOISE_PREPASS");
  if (pre_env && std::strcmp(pre_env, "0") == 0) return STIM_OK;
  auto alloc = [&](void **ptr, size_t bytes) {
    bytes = std::max<size_t>(bytes, 8);
    return async ? hipMallocAsync(ptr, bytes, s) : hipMalloc(ptr, bytes);
  };
  auto upload = [&](const void *src, size_t bytes, void *dst) -> int {
    if (async) return stage_upload(src, bytes, dst, s);
    const hipError_t e = hipMemcpy(dst, src, bytes, hipMemcpyHostToDevice);
    return e == hipSuccess ? STIM_OK : hip_error(e, "batch noise upload");
  };
  int min_T = 8;
  for (int T : widths) min_T = std::min(min_T, T);
  for (size_t i : pl.batched) {
    const stim_request &r = pl.reqs[i];
    const Program &P = r.c->prog;
    const size_t ninst = P.noise_pc.size();
    if (ninst == 0 || ninst > kMaxGenInstances || P.num_qubits >= (1ull << 27)) continue;
    const uint64_t W = (r.num_shots + 63) / 64;
    std::vector<uint32_t> caps[4];
    std::vector<uint64_t> bases[4];
    uint32_t max_caps[4] = {1, 1, 1, 1};
    uint64_t total = 0;
    for (int T : widths) {
      const int k = width_index(T);
      total = std::max(total, noise_reservations(P, T, (W + T - 1) / T, caps[k], bases[k], max_caps[k]));
    }
    if (total == 0 || total * 16 > kMaxRecordBytes) continue;
    BatchPlan::Noise &nz = pl.noise[i];
    nz.ninst = (uint32_t)ninst;
    nz.stride = (uint32_t)((W + min_T - 1) / min_T);
    hipError_t e;
    if ((e = alloc((void **)&nz.meta, ninst * nz.stride * sizeof(uint2))) != hipSuccess ||
        (e = alloc((void **)&nz.rec, total * 16)) != hipSuccess)
      return set_error(STIM_E_OOM, "batch noise record allocation failed");
    for (int T : widths) {
      const int k = width_index(T);
      nz.max_cap[k] = max_caps[k];
      if ((e = alloc((void **)&nz.cap[k], ninst * sizeof(uint32_t))) != hipSuccess ||
          (e = alloc((void **)&nz.base[k], ninst * sizeof(uint64_t))) != hipSuccess)
        return set_error(STIM_E_OOM, "batch noise table allocation failed");
      int rc = upload(caps[k].data(), ninst * sizeof(uint32_t), nz.cap[k]);
      if (!rc) rc = upload(bases[k].data(), ninst * sizeof(uint64_t), nz.base[k]);
      if (rc) return rc;
    }
  }
  return STIM_OK;
}

void drop_plans_using(const stim_circuit *c) {
  std::lock_guard<std::mutex> lock(g_batch_mu);
  for (size_t i = 0; i < g_plans.size();) {
    bool uses = false;
    for (const stim_request &r : g_plans[i]->reqs) uses |= r.c == c;
    if (uses) {
      free_plan(g_plans[i].get());
      g_plans.erase(g_plans.begin() + (long)i);
    } else {
      i++;
    }
  }
}

bool same_request(const stim_request &a, const stim_request &b) {
  return a.c == b.c && a.seed == b.seed && a.shot_offset == b.shot_offset && a.num_shots == b.num_shots &&
         a.mode == b.mode && a.out0 == b.out0 && a.out1 == b.out1;
}


bool batch_fits(uint64_t n, int T, uint32_t threads) {
  return frame_lds_bytes(n, T, true, threads) + kBatchStaticLds <= kMaxLdsBytes;
}

// Whether a configuration can run a request set whose largest circuit has n
// qubits: a workgroup tile in LDS, or (one wave per tile) at least four waves'
// tiles per workgroup.
bool config_fits(uint64_t n, const FrameConfig &cfg) {
  return cfg.wave ? batch_waves_per_block(n, cfg.tile_words) >= 4 : batch_fits(n, cfg.tile_words, cfg.threads);
}

// The tuned configuration of a plan's shape class, if there is one that fits
// this plan: a class spans a factor of two in qubit count, so a width tuned
// for its smaller circuits may not fit the LDS of its larger ones.
std::string shape_class(const BatchPlan &pl);
int batch_wave_mode();
bool tuned_config(const BatchPlan &pl, FrameConfig *cfg) {
  auto known = g_tuned.find(shape_class(pl));
  if (known == g_tuned.end() || !config_fits(pl.max_n, known->second)) return false;
  const int wave_mode = batch_wave_mode();
  if (wave_mode >= 0 && known->second.wave != (wave_mode == 1)) return false;
  *cfg = known->second;
  return true;
}

std::string shape_class(const BatchPlan &pl) {
  uint64_t words = 0;
  for (size_t i : pl.batched) words += (pl.reqs[i].num_shots + 63) / 64;
  int nb = 0, wb = 0, rb = 0;
  while ((1ull << nb) < pl.max_n) nb++;
  while ((1ull << wb) < words) wb++;
  while ((1ull << rb) < pl.batched.size()) rb++;
  return std::to_string(nb) + "/" + std::to_string(wb) + "/" + std::to_string(rb);
}

hipError_t enqueue_plan(BatchPlan &pl, hipStream_t s) {
  hipError_t e = hipSuccess;
  // Noise pre-passes of the noisy requests, at the plan's tile width.
  const int T = pl.cfg.tile_words, k = width_index(T);
  for (size_t i : pl.batched) {
    if (i >= pl.noise.size() || !pl.noise[i].meta) continue;
    const BatchPlan::Noise &nz = pl.noise[i];
    const stim_request &r = pl.reqs[i];
    DeviceCopy &d = r.c->dev[pl.device];
    const uint64_t W = (r.num_shots + 63) / 64;
    NoiseGenParams g{};
    g.ops = d.ops;
    g.targets = d.targets;
    g.thresholds = d.thresholds;
    g.inst_pc = d.noise_pc;
    g.inst_instr = d.noise_instr;
    g.base = nz.base[k];
    g.cap = nz.cap[k];
    g.seed = r.seed;
    g.word0 = r.shot_offset / 64;
    g.num_words = W;
    g.tiles = (uint32_t)((W + T - 1) / T);
    g.tile_stride = (uint32_t)nz.ninst;       // batched walks read the table tile-major
    g.inst_stride = 1u;
    g.meta = nz.meta;
    g.rec = nz.rec;
    g.tiles_per_group = std::max<uint32_t>(1, std::min<uint32_t>(kGenTiles, kGenQueue / nz.max_cap[k]));
    g.queue_per_tile = kGenQueue / g.tiles_per_group;
    if ((e = launch_noise_gen(g, T, nz.ninst, 512, s)) != hipSuccess) return e;
  }
  if (pl.num_items) {
    e = launch_batch(pl.d_params, pl.d_items, pl.num_items, pl.d_counter, pl.cfg, pl.max_n, pl.blocks, s);
    if (e != hipSuccess) return e;
  }
  for (size_t i : pl.batched) {
    const stim_request &r = pl.reqs[i];
    if (r.mode != 1) continue;
    DeviceCopy &d = r.c->dev[pl.device];
    const uint64_t W = (r.num_shots + 63) / 64;
    e = launch_parity_blocks(pl.flips[i], W, d.det_blocks, r.c->prog.det_blocks.size() / kDetBlockWords, d.det_off,
                             d.det_idx, r.out0, s);
    if (e == hipSuccess && r.out1)
      e = launch_parity(pl.flips[i], W, d.obs_off, d.obs_idx, nullptr, (uint32_t)r.c->prog.num_observables, r.out1,
                        s);
    if (e != hipSuccess) return e;
  }
  return e;
}

// Kernel parameters of every request that runs inside a persistent launch.
void batch_params(BatchPlan &pl, std::vector<FrameParams> &params, uint64_t *flips_base) {
  uint64_t off = 0;
  params.assign(pl.reqs.size(), FrameParams{});
  pl.flips.assign(pl.reqs.size(), nullptr);
  for (size_t i : pl.batched) {
    const stim_request &r = pl.reqs[i];
    DeviceCopy &d = r.c->dev[pl.device];
    FrameParams &p = params[i];
    const uint64_t W = (r.num_shots + 63) / 64;
    p.ops = d.ops;
    p.num_ops = (uint32_t)r.c->prog.ops.size();
    p.num_qubits = (uint32_t)r.c->prog.num_qubits;
    p.targets = d.targets;
    p.thresholds = d.thresholds;
    p.seed = r.seed;
    p.word0 = r.shot_offset / 64;
    p.num_words = W;
    uint64_t rem = r.num_shots % 64;
    p.tail_mask = rem ? ((1ull << rem) - 1) : ~0ull;
    p.out_stride = W;
    p.scratch = nullptr;
    if (r.mode == 1) {
      pl.flips[i] = flips_base + off;
      off += std::max<uint64_t>(r.c->prog.num_measurements, 1) * W;
      p.ref = nullptr;
      p.out = pl.flips[i];
      if (d.noz_ops) {           // the program without Z randomisations (same events)
        p.ops = d.noz_ops;
        p.targets = d.noz_targets;
      }
    } else {
      p.ref = d.ref;
      p.out = r.out0;
    }
    if (i < pl.noise.size() && pl.noise[i].meta) {
      p.noise_meta = pl.noise[i].meta;
      p.noise_rec = pl.noise[i].rec;
      p.noise_tiles = pl.noise[i].stride;
      p.noise_instances = pl.noise[i].ninst;
    }
  }
}

// Splits requests into those that run inside the persistent launch (frames
// fit in LDS) and the rest; returns the flip scratch size in words.
// A noisy request with at least this many shot-gates runs through the
// single-request path: its noise pre-pass outweighs sharing a launch.
constexpr double kSingleWork = 4e9;

uint64_t partition_requests(BatchPlan &pl) {
  uint64_t total_flips = 0;
  for (size_t i = 0; i < pl.reqs.size(); i++) {
    const stim_request &r = pl.reqs[i];
    const double work = (double)r.c->prog.num_gate_targets * (double)r.num_shots;
    const bool big_noisy = r.c->prog.num_noise_targets > 0 && work >= kSingleWork && !r.c->prog.noise_pc.empty();
    if (!big_noisy && batch_fits(r.c->prog.num_qubits, 1, 256)) {
      pl.batched.push_back(i);
      pl.max_n = std::max(pl.max_n, r.c->prog.num_qubits);
      if (r.mode == 1) total_flips += std::max<uint64_t>(r.c->prog.num_measurements, 1) * ((r.num_shots + 63) / 64);
    } else {
      pl.single.push_back(i);
    }
  }
  return total_flips;
}

std::vector<BatchItem> work_list(const BatchPlan &pl, int T) {
  // Longest job first: tiles ordered by the work of their circuit.
  std::vector<std::pair<uint64_t, BatchItem>> v;
  for (size_t i : pl.batched) {
    const stim_request &r = pl.reqs[i];
    uint64_t W = (r.num_shots + 63) / 64, tiles = (W + T - 1) / T;
    uint64_t cost = r.c->prog.num_gate_targets + r.c->prog.num_noise_targets + r.c->prog.num_qubits;
    for (uint64_t t = 0; t < tiles; t++) v.push_back({cost, BatchItem{(uint32_t)i, (uint32_t)t}});
  }
  std::stable_sort(v.begin(), v.end(), [](const auto &a, const auto &b) { return a.first > b.first; });
  std::vector<BatchItem> items;
  items.reserve(v.size());
  for (auto &x : v) items.push_back(x.second);
  return items;
}

// STIM_BATCH_WAVE = 1 / 0 forces the one-wave-per-tile kernel / the
// workgroup kernel for batched launches (default: the tuner chooses).
int batch_wave_mode() {
  const char *v = std::getenv("STIM_BATCH_WAVE");
  return v ? (std::atoi(v) ? 1 : 0) : -1;
}

FrameConfig untuned_batch_config(uint64_t max_n) {
  if (batch_wave_mode() == 1) {
    for (int T : {2, 1}) {
      FrameConfig w{T, true, 64};
      w.wave = true;
      if (config_fits(max_n, w)) return w;
    }
  }
  for (int T : {4, 2, 1})
    if (batch_fits(max_n, T, 256)) return FrameConfig{T, true, 256};
  return FrameConfig{1, true, 256};
}

// One persistent launch with stream-ordered temporaries: nothing is cached and
// nothing blocks the host.
int run_one_shot(BatchPlan &pl, hipStream_t s) {
  uint64_t total_flips = partition_requests(pl);
  if (pl.batched.empty()) return STIM_OK;
  load_tune_cache();
  if (!tuned_config(pl, &pl.cfg)) pl.cfg = untuned_batch_config(pl.max_n);
  std::vector<BatchItem> items = work_list(pl, pl.cfg.tile_words);
  pl.num_items = (uint32_t)items.size();
  pl.blocks = (uint32_t)(cu_count(pl.device) * batch_blocks_per_cu(pl.cfg, pl.max_n));
  hipError_t e;
  int rc = STIM_OK;
  if ((e = hipMallocAsync((void **)&pl.d_params, pl.reqs.size() * sizeof(FrameParams), s)) != hipSuccess ||
      (e = hipMallocAsync((void **)&pl.d_items, std::max<size_t>(items.size(), 1) * sizeof(BatchItem), s)) !=
          hipSuccess ||
      (e = hipMallocAsync((void **)&pl.d_counter, sizeof(uint32_t), s)) != hipSuccess ||
      (total_flips && (e = hipMallocAsync((void **)&pl.d_flips, total_flips * 8, s)) != hipSuccess))
    rc = set_error(STIM_E_OOM, "batch allocation failed");
  if (!rc) rc = prepare_batch_noise(pl, {pl.cfg.tile_words}, s, true);
  std::vector<FrameParams> params;
  batch_params(pl, params, pl.d_flips);
  if (!rc) rc = stage_upload(params.data(), params.size() * sizeof(FrameParams), pl.d_params, s);
  if (!rc) rc = stage_upload(items.data(), items.size() * sizeof(BatchItem), pl.d_items, s);
  if (!rc && (e = enqueue_plan(pl, s)) != hipSuccess) rc = hip_error(e, "batch launch");
  free_batch_noise(pl, s, true);
  void *ptrs[] = {pl.d_params, pl.d_items, pl.d_counter, pl.d_flips};
  for (void *q : ptrs) if (q) (void)hipFreeAsync(q, s);
  pl.d_params = nullptr;
  pl.d_items = nullptr;
  pl.d_counter = nullptr;
  pl.d_flips = nullptr;
  return rc;
}

// Builds the device tables of a plan and picks its configuration: by timing
// each candidate tile width x workgroup size on the real request set (the
// outputs of every trial are complete and identical), unless the shape class
// was tuned before or STIM_TUNE=0.
int build_plan(BatchPlan &pl, hipStream_t s) {
  hipError_t e;
  uint64_t total_flips = partition_requests(pl);
  if (pl.batched.empty()) return STIM_OK;
  if (total_flips && (e = hipMalloc((void **)&pl.d_flips, total_flips * 8)) != hipSuccess)
    return set_error(STIM_E_OOM, "batch flip scratch allocation failed");

  // Candidate configurations; the work list depends on the tile width.
  std::vector<FrameConfig> cands;
  const int wave_mode = batch_wave_mode();
  for (int T : {1, 2, 4, 8}) {
    if (wave_mode != 1)
      for (uint32_t th : {256u, 512u, 1024u})
        if (batch_fits(pl.max_n, T, th)) cands.push_back(FrameConfig{T, true, th});
    FrameConfig w{T, true, 64};
    w.wave = true;
    if (wave_mode != 0 && config_fits(pl.max_n, w)) cands.push_back(w);
  }
  if (cands.empty()) cands.push_back(untuned_batch_config(pl.max_n));
  const char *tune_env = std::getenv("STIM_TUNE");
  const bool tune = !(tune_env && std::strcmp(tune_env, "0") == 0);
  const std::string cls = shape_class(pl);
  load_tune_cache();
  FrameConfig known;
  if (tuned_config(pl, &known)) cands = {known};
  else if (!tune) cands = {untuned_batch_config(pl.max_n)};

  std::vector<int> widths;
  for (const FrameConfig &cfg : cands)
    if (std::find(widths.begin(), widths.end(), cfg.tile_words) == widths.end()) widths.push_back(cfg.tile_words);
  int nrc = prepare_batch_noise(pl, widths, s, false);
  if (nrc) return nrc;
  std::vector<FrameParams> params;
  batch_params(pl, params, pl.d_flips);
  if ((e = hipMalloc((void **)&pl.d_params, params.size() * sizeof(FrameParams))) != hipSuccess ||
      (e = hipMalloc((void **)&pl.d_counter, sizeof(uint32_t))) != hipSuccess)
    return set_error(STIM_E_OOM, "batch table allocation failed");
  if ((e = hipMemcpy(pl.d_params, params.data(), params.size() * sizeof(FrameParams), hipMemcpyHostToDevice)) !=
      hipSuccess)
    return hip_error(e, "batch table upload");

  BatchItem *d_items_by_T[9] = {nullptr};
  auto items_for = [&](int T) -> BatchItem * {
    if (d_items_by_T[T]) return d_items_by_T[T];
    std::vector<BatchItem> items = work_list(pl, T);
    BatchItem *d = nullptr;
    if (hipMalloc((void **)&d, std::max<size_t>(items.size(), 1) * sizeof(BatchItem)) != hipSuccess) return nullptr;
    if (hipMemcpy(d, items.data(), items.size() * sizeof(BatchItem), hipMemcpyHostToDevice) != hipSuccess) {
      (void)hipFree(d);
      return nullptr;
    }
    d_items_by_T[T] = d;
    return d;
  };
  auto num_items_for = [&](int T) {
    uint64_t n = 0;
    for (size_t i : pl.batched) n += ((pl.reqs[i].num_shots + 63) / 64 + T - 1) / T;
    return (uint32_t)n;
  };
  float best = 1e30f;
  FrameConfig best_cfg = cands[0];
  if (cands.size() > 1) {
    hipEvent_t a, b;
    if ((e = hipEventCreate(&a)) != hipSuccess || (e = hipEventCreate(&b)) != hipSuccess)
      return hip_error(e, "hipEventCreate");
    for (const FrameConfig &cfg : cands) {
      pl.cfg = cfg;
      pl.d_items = items_for(cfg.tile_words);
      if (!pl.d_items) return set_error(STIM_E_OOM, "batch work list allocation failed");
      pl.num_items = num_items_for(cfg.tile_words);
      pl.blocks = (uint32_t)(cu_count(pl.device) * batch_blocks_per_cu(cfg, pl.max_n));
      (void)hipEventRecord(a, s);
      if ((e = enqueue_plan(pl, s)) != hipSuccess) return hip_error(e, "batch trial launch");
      (void)hipEventRecord(b, s);
      if ((e = hipEventSynchronize(b)) != hipSuccess) return hip_error(e, "batch trial");
      float ms = 0;
      (void)hipEventElapsedTime(&ms, a, b);
      if (ms < best) { best = ms; best_cfg = cfg; }
    }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    save_tuned(cls, best_cfg);
    pl.tuned_ms = best;
  }
  pl.cfg = best_cfg;
  pl.d_items = items_for(best_cfg.tile_words);
  if (!pl.d_items) return set_error(STIM_E_OOM, "batch work list allocation failed");
  pl.num_items = num_items_for(best_cfg.tile_words);
  pl.blocks = (uint32_t)(cu_count(pl.device) * batch_blocks_per_cu(best_cfg, pl.max_n));
  for (int T = 1; T <= 8; T++)
    if (d_items_by_T[T] && d_items_by_T[T] != pl.d_items) (void)hipFree(d_items_by_T[T]);

  // Capture the launch sequence once; later submissions replay it.
  hipStream_t cap;
  if ((e = hipStreamCreateWithFlags(&cap, hipStreamNonBlocking)) != hipSuccess) return hip_error(e, "stream");
  if ((e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal)) != hipSuccess) {
    (void)hipStreamDestroy(cap);
    return hip_error(e, "hipStreamBeginCapture");
  }
  hipError_t le = enqueue_plan(pl, cap);
  e = hipStreamEndCapture(cap, &pl.graph);
  (void)hipStreamDestroy(cap);
  if (le != hipSuccess) return hip_error(le, "batch capture");
  if (e != hipSuccess) return hip_error(e, "hipStreamEndCapture");
  if ((e = hipGraphInstantiate(&pl.exec, pl.graph, nullptr, nullptr, 0)) != hipSuccess)
    return hip_error(e, "hipGraphInstantiate");
  return STIM_OK;
}

std::mutex g_noalloc_mu;
std::map<int, void *> g_noalloc_ptr;      // device -> address of `scratch` there

// Address of `scratch` on device `dev` (the current device), looked up once.
int noalloc_scratch(int dev, void **out) {
  std::lock_guard<std::mutex> lock(g_noalloc_mu);
  auto it = g_noalloc_ptr.find(dev);
  if (it != g_noalloc_ptr.end()) {
    *out = it->second;
    return STIM_OK;
  }
  void *ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return hip_error(e, "hipGetSymbolAddress(scratch)");
  if (!ptr) return set_error(STIM_E_DEVICE, "hipGetSymbolAddress(scratch) returned no address");
  g_noalloc_ptr[dev] = ptr;
  *out = ptr;
  return STIM_OK;
}

}  // namespace

extern "C" {

const char *stim_last_error(void) { return g_last_error.c_str(); }

int stim_compile(const char *text, size_t len, stim_circuit **out) {
  if (!out || (!text && len)) return set_error(STIM_E_INVALID_ARG, "null argument");
  *out = nullptr;
  try {
    std::unique_ptr<stim_circuit> c(new stim_circuit());
    c->tree = parse_circuit(std::string(text ? text : "", len));
    c->prog = compile_program(c->tree);
    *out = c.release();
    g_last_error.clear();
    return STIM_OK;
  } catch (const CompileError &e) {
    return set_error(e.code, e.msg);
  } catch (const std::bad_alloc &) {
    return set_error(STIM_E_OOM, "out of host memory");
  } catch (const std::exception &e) {
    return set_error(STIM_E_PARSE, e.what());
  }
}

void stim_circuit_free(stim_circuit *c) {
  if (!c) return;
  drop_plans_using(c);
  int cur = 0;
  (void)hipGetDevice(&cur);
  for (auto &kv : c->dev) {
    (void)hipSetDevice(kv.first);
    DeviceCopy &d = kv.second;
    void *ptrs[] = {d.ops,       d.event_ops,   d.noz_ops,     d.noz_targets, d.targets,     d.thresholds, d.ref,     d.det_off,
                    d.det_idx,   d.obs_off,     d.obs_idx,    d.det_order, d.det_blocks, d.noise_pc,
                    d.noise_instr, d.gen_base, d.set_off,    d.set_lanes, d.wb_e0,
                    d.wb_e1,       d.wb_base};
    for (void *p : ptrs) if (p) (void)hipFree(p);
  }
  if (!c->dev.empty()) (void)hipSetDevice(cur);
  delete c;
}

int stim_circuit_shape(const stim_circuit *c, uint64_t *num_qubits, uint64_t *num_measurements,
                       uint64_t *num_detectors, uint64_t *num_observables, uint64_t *num_gate_targets) {
  if (!c) return set_error(STIM_E_INVALID_ARG, "null circuit handle");
  if (num_qubits) *num_qubits = c->prog.num_qubits;
  if (num_measurements) *num_measurements = c->prog.num_measurements;
  if (num_detectors) *num_detectors = c->prog.num_detectors;
  if (num_observables) *num_observables = c->prog.num_observables;
  if (num_gate_targets) *num_gate_targets = c->prog.num_gate_targets;
  return STIM_OK;
}

int stim_reference_sample(stim_circuit *c, uint64_t *ref_out) {
  if (!c) return set_error(STIM_E_INVALID_ARG, "null circuit handle");
  std::lock_guard<std::mutex> lock(c->mu);
  int rc = ensure_reference(c);
  if (rc) return rc;
  if (ref_out && !c->ref.empty()) std::memcpy(ref_out, c->ref.data(), c->ref.size() * sizeof(uint64_t));
  return STIM_OK;
}

int stim_frame_sample(stim_circuit *c, uint64_t seed, uint64_t shot_offset, uint64_t num_shots,
                      uint64_t *out_meas, void *hip_stream) {
  int rc = check_sample_args(c, shot_offset, num_shots);
  if (rc) return rc;
  if (c->prog.num_measurements > 0 && !is_device_pointer(out_meas))
    return set_error(STIM_E_INVALID_ARG, "out_meas is not a device pointer");
  hipStream_t s = (hipStream_t)hip_stream;
  DeviceCopy *d = nullptr;
  {
    std::lock_guard<std::mutex> lock(c->mu);
    if ((rc = ensure_reference(c, s, true))) return rc;
    if ((rc = ensure_device(c, s, &d))) return rc;
  }
  return run_frame(c, d, seed, shot_offset, num_shots, d->ref, out_meas, s);
}

int stim_detector_sample(stim_circuit *c, uint64_t seed, uint64_t shot_offset, uint64_t num_shots,
                         uint64_t *out_det, uint64_t *out_obs, void *hip_stream) {
  int rc = check_sample_args(c, shot_offset, num_shots);
  if (rc) return rc;
  if (c->prog.num_detectors > 0 && !is_device_pointer(out_det))
    return set_error(STIM_E_INVALID_ARG, "out_det is not a device pointer");
  if (out_obs && c->prog.num_observables > 0 && !is_device_pointer(out_obs))
    return set_error(STIM_E_INVALID_ARG, "out_obs is not a device pointer");
  hipStream_t s = (hipStream_t)hip_stream;
  DeviceCopy *d = nullptr;
  {
    std::lock_guard<std::mutex> lock(c->mu);
    if ((rc = ensure_reference(c, s, true))) return rc;
    if ((rc = ensure_device(c, s, &d))) return rc;
    if ((rc = ensure_noz_program(c, d, s))) return rc;
  }
  int dev = 0;
  (void)hipGetDevice(&dev);
  if (walk_event_slots(c->prog, num_shots, dev) > 0) {
    WalkEvents ev;
    ev.det_out = out_det;
    ev.obs_out = c->prog.num_observables > 0 ? out_obs : nullptr;
    ev.num_obs = (uint32_t)c->prog.num_observables;
    return run_frame(c, d, seed, shot_offset, num_shots, nullptr, nullptr, s, &ev);
  }
  const uint64_t W = (num_shots + 63) / 64;
  uint64_t *flips = nullptr;
  size_t bytes = (size_t)std::max<uint64_t>(c->prog.num_measurements, 1) * W * sizeof(uint64_t);
  hipError_t e = hipMallocAsync((void **)&flips, bytes, s);
  if (e != hipSuccess) return set_error(STIM_E_OOM, "flip scratch allocation failed");
  rc = run_frame(c, d, seed, shot_offset, num_shots, nullptr, flips, s, nullptr, true);
  if (!rc && (e = launch_parity_blocks(flips, W, d->det_blocks, c->prog.det_blocks.size() / kDetBlockWords, d->det_off,
                                      d->det_idx, out_det, s)) != hipSuccess)
    rc = hip_error(e, "detector kernel launch");
  if (!rc && out_obs &&
      (e = launch_parity(flips, W, d->obs_off, d->obs_idx, nullptr, (uint32_t)c->prog.num_observables, out_obs, s)) !=
          hipSuccess)
    rc = hip_error(e, "observable kernel launch");
  hipError_t fe = hipFreeAsync(flips, s);
  if (!rc && fe != hipSuccess) rc = hip_error(fe, "hipFreeAsync");
  return rc;
}

int stim_detector_sample_noalloc(stim_circuit *c, uint64_t seed, uint64_t shot_offset, uint64_t num_shots,
                                 uint64_t *out_det, uint64_t *out_obs, void *hip_stream) {
  int rc = check_sample_args(c, shot_offset, num_shots);
  if (rc) return rc;
  if (c->prog.num_detectors > 0 && !is_device_pointer(out_det))
    return set_error(STIM_E_INVALID_ARG, "out_det is not a device pointer");
  if (out_obs && c->prog.num_observables > 0 && !is_device_pointer(out_obs))
    return set_error(STIM_E_INVALID_ARG, "out_obs is not a device pointer");
  hipStream_t s = (hipStream_t)hip_stream;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_error(e, "hipGetDevice");
  DeviceCopy *d = nullptr;
  const DevOp *ops = nullptr;
  const uint32_t *targets = nullptr;
  {
    std::lock_guard<std::mutex> lock(c->mu);
    auto it = c->dev.find(dev);
    if (it == c->dev.end())
      return set_error(STIM_E_INVALID_ARG, "the circuit is not resident on device " + std::to_string(dev) +
                                               ": an allocating sampling call on this device uploads it first");
    d = &it->second;
    // The program without Z randomisations if an earlier detector call built
    // it (this entry point allocates nothing, so it never builds it).
    ops = d->noz_ops ? d->noz_ops : d->ops;
    targets = d->noz_ops ? d->noz_targets : d->targets;
  }
  const Program &P = c->prog;
  const uint64_t W = (num_shots + 63) / 64;
  FrameConfig cfg = choose_config(P.num_qubits, W);
  const uint64_t ntiles = (W + cfg.tile_words - 1) / cfg.tile_words;
  const uint64_t flip_bytes = (std::max<uint64_t>(P.num_measurements, 1) * W * 8 + 255) / 256 * 256;
  uint64_t slot_bytes = 0;
  if (!cfg.in_lds) {
    cfg.slots = (uint32_t)global_frame_slots(dev, ntiles);
    slot_bytes = (uint64_t)cfg.slots * cfg.tile_words * 16 * (P.num_qubits + 1);
  }
  if (flip_bytes + slot_bytes > kNoAllocScratchBytes)
    return set_error(STIM_E_UNSUPPORTED, "this call needs " + std::to_string(flip_bytes + slot_bytes) +
                                             " bytes of device scratch, more than the " +
                                             std::to_string(kNoAllocScratchBytes) +
                                             " this entry point holds: sample fewer shots per call");
  void *base = nullptr;
  if ((rc = noalloc_scratch(dev, &base))) return rc;
  uint64_t *flips = (uint64_t *)base;
  FrameParams p{};
  p.ops = ops;
  p.noz = ops != nullptr && d != nullptr && ops == d->noz_ops;
  p.num_ops = (uint32_t)P.ops.size();
  p.num_qubits = (uint32_t)P.num_qubits;
  p.targets = targets;
  p.thresholds = d->thresholds;
  p.ref = nullptr;                         // raw flips
  p.seed = seed;
  p.word0 = shot_offset / 64;
  p.num_words = W;
  const uint64_t rem = num_shots % 64;
  p.tail_mask = rem ? ((1ull << rem) - 1) : ~0ull;
  p.out = flips;
  p.out_stride = W;
  p.scratch = slot_bytes ? (uint64_t *)((unsigned char *)base + flip_bytes) : nullptr;
  p.noise_meta = nullptr;                  // noise drawn inline: its records would need more scratch
  if (P.num_measurements > 0 || P.num_qubits > 0) {
    if ((e = launch_frame(p, cfg, s)) != hipSuccess) return hip_error(e, "frame kernel launch");
  }
  if ((e = launch_parity_blocks(flips, W, d->det_blocks, P.det_blocks.size() / kDetBlockWords, d->det_off, d->det_idx,
                                out_det, s)) !=
      hipSuccess)
    return hip_error(e, "detector kernel launch");
  if (out_obs &&
      (e = launch_parity(flips, W, d->obs_off, d->obs_idx, nullptr, (uint32_t)P.num_observables, out_obs, s)) !=
          hipSuccess)
    return hip_error(e, "observable kernel launch");
  return STIM_OK;
}

int stim_sparse_detector_sample(stim_circuit *c, uint64_t seed, uint64_t shot_offset, uint64_t num_shots,
                                uint64_t *out_det, uint64_t *out_obs, void *hip_stream) {
  int rc = check_sample_args(c, shot_offset, num_shots);
  if (rc) return rc;
  if (c->prog.num_detectors > 0 && !is_device_pointer(out_det))
    return set_error(STIM_E_INVALID_ARG, "out_det is not a device pointer");
  if (out_obs && c->prog.num_observables > 0 && !is_device_pointer(out_obs))
    return set_error(STIM_E_INVALID_ARG, "out_obs is not a device pointer");
  const uint64_t W = (num_shots + 63) / 64;
  if (W >= (1ull << 32)) return set_error(STIM_E_UNSUPPORTED, "too many shots in one call");
  hipStream_t s = (hipStream_t)hip_stream;
  DeviceCopy *d = nullptr;
  {
    std::lock_guard<std::mutex> lock(c->mu);
    if ((rc = ensure_error_model(c))) return rc;
    if ((rc = ensure_reference(c, s, true))) return rc;
    if ((rc = ensure_device(c, s, &d))) return rc;
    if ((rc = ensure_sparse_device(c, d, s))) return rc;
  }
  const Program &P = c->prog;
  hipError_t e;
  SparseParams sp{};
  sp.ops = d->ops;
  sp.targets = d->targets;
  sp.thresholds = d->thresholds;
  sp.inst_pc = d->noise_pc;
  sp.inst_instr = d->noise_instr;
  sp.gen_base = d->gen_base;
  sp.set_off = d->set_off;
  sp.set_lanes = d->set_lanes;
  sp.seed = seed;
  sp.word0 = shot_offset / 64;
  sp.num_words = W;
  sp.num_shots = num_shots;
  sp.det = out_det;
  sp.obs = P.num_observables ? out_obs : nullptr;
  sp.num_det = (uint32_t)P.num_detectors;
  if (c->win_T) {
    // Windowed kernel: every output word is written exactly once.
    SparseWindowParams wp{};
    wp.s = sp;
    wp.batch_e0 = d->wb_e0;
    wp.batch_e1 = d->wb_e1;
    wp.batch_base = d->wb_base;
    wp.num_batches = (uint32_t)c->wb_e0.size();
    wp.win = c->win_rows;
    wp.num_obs = (uint32_t)P.num_observables;
    if ((e = launch_sparse_window(wp, c->win_T, s)) != hipSuccess) return hip_error(e, "sparse window kernel launch");
    return STIM_OK;
  }
  if (P.num_detectors && (e = hipMemsetAsync(out_det, 0, P.num_detectors * W * sizeof(uint64_t), s)) != hipSuccess)
    return hip_error(e, "hipMemsetAsync");
  if (out_obs && P.num_observables &&
      (e = hipMemsetAsync(out_obs, 0, P.num_observables * W * sizeof(uint64_t), s)) != hipSuccess)
    return hip_error(e, "hipMemsetAsync");
  if ((e = launch_sparse_events(sp, (uint32_t)P.noise_pc.size(), (uint64_t)c->em_max_groups * W, s)) != hipSuccess)
    return hip_error(e, "sparse event kernel launch");
  return STIM_OK;
}

int stim_reference_sample_gpu(stim_circuit *c, uint64_t *ref_out, void *hip_stream) {
  if (!c) return set_error(STIM_E_INVALID_ARG, "null circuit handle");
  if (c->prog.max_loop_depth > 8) return set_error(STIM_E_UNSUPPORTED, "REPEAT nesting deeper than 8");
  std::lock_guard<std::mutex> lock(c->mu);
  std::string err;
  std::vector<uint64_t> bits;
  int rc;
  try {
    rc = gpu_reference_sample(c->tree, c->prog.num_qubits, c->prog.num_measurements, bits, (hipStream_t)hip_stream,
                              err);
  } catch (const std::bad_alloc &) {
    return set_error(STIM_E_OOM, "out of host memory planning the GPU reference sample");
  }
  if (rc) return set_error(rc, err);
  if (ref_out && !bits.empty()) std::memcpy(ref_out, bits.data(), bits.size() * sizeof(uint64_t));
  if (!c->have_ref) {
    c->ref = std::move(bits);
    c->have_ref = true;
  }
  return STIM_OK;
}

int stim_error_sets(stim_circuit *c, uint64_t *num_sets, uint64_t *num_entries, uint32_t *offsets,
                    uint32_t *lanes) {
  if (!c || !num_sets || !num_entries) return set_error(STIM_E_INVALID_ARG, "null argument");
  std::lock_guard<std::mutex> lock(c->mu);
  int rc = ensure_error_model(c);
  if (rc) return rc;
  *num_sets = c->em.num_generators;
  *num_entries = c->em.set_lanes.size();
  if (offsets) std::memcpy(offsets, c->em.set_off.data(), c->em.set_off.size() * sizeof(uint32_t));
  if (lanes && !c->em.set_lanes.empty())
    std::memcpy(lanes, c->em.set_lanes.data(), c->em.set_lanes.size() * sizeof(uint32_t));
  return STIM_OK;
}

int stim_sample_scratch_bytes(stim_circuit *c, uint64_t num_shots, int mode, uint64_t *bytes) {
  if (!c || !bytes) return set_error(STIM_E_INVALID_ARG, "null argument");
  if (mode < 0 || mode > 2) return set_error(STIM_E_INVALID_ARG, "mode must be 0, 1 or 2");
  *bytes = 0;
  if (num_shots == 0 || mode == 2) return STIM_OK;
  int dev = 0;
  (void)hipGetDevice(&dev);
  const Program &P = c->prog;
  uint64_t b = pass_scratch_bytes(P, num_shots, dev);
  if (mode == 1) {
    // The flip rings when the walk forms the events, else the flip record.
    const uint64_t ring = walk_event_bytes(P, num_shots, dev);
    b += ring ? ring : std::max<uint64_t>(P.num_measurements, 1) * ((num_shots + 63) / 64) * sizeof(uint64_t);
  }
  *bytes = b;
  return STIM_OK;
}

int stim_format_shots(const uint64_t *table, uint64_t rows, uint64_t num_shots, int format, uint8_t *out,
                      uint64_t out_cap, uint64_t *out_len, void *hip_stream) {
  if (!out_len) return set_error(STIM_E_INVALID_ARG, "out_len is NULL");
  *out_len = 0;
  if (format < STIM_FORMAT_01 || format > STIM_FORMAT_R8) return set_error(STIM_E_INVALID_ARG, "unknown format");
  if (num_shots == 0) return set_error(STIM_E_INVALID_ARG, "num_shots must be positive");
  if (rows >= (1ull << 31) || num_shots >= (1ull << 40)) return set_error(STIM_E_UNSUPPORTED, "table too large");
  if (rows > 0 && !is_device_pointer(table)) return set_error(STIM_E_INVALID_ARG, "table is not a device pointer");
  if (out_cap > 0 && !is_device_pointer(out)) return set_error(STIM_E_INVALID_ARG, "out is not a device pointer");
  if (out_cap > 0 && (format == STIM_FORMAT_B8 || format == STIM_FORMAT_01) && (uintptr_t)out % 4)
    return set_error(STIM_E_INVALID_ARG, "01 and b8 outputs must be 4-byte aligned");
  hipStream_t s = (hipStream_t)hip_stream;
  const uint64_t W = (num_shots + 63) / 64;
  const bool dense = format == STIM_FORMAT_01 || format == STIM_FORMAT_B8;
  if (dense) {
    const uint64_t per = format == STIM_FORMAT_B8 ? (rows + 7) / 8 : rows + 1;
    *out_len = per * num_shots;
    if (out_cap < *out_len) {
      if (out_cap == 0 && !out) return STIM_OK;          // size query
      return set_error(STIM_E_INVALID_ARG, "output buffer too small");
    }
    if (*out_len == 0) return STIM_OK;
  }
  hipError_t e;
  if (format == STIM_FORMAT_B8 && ((rows + 7) / 8) % 4 == 0) {
    // b8 is the transposed bits with each shot's row cut to ceil(rows / 8)
    // bytes; when that is a multiple of 4, the transpose writes it directly.
    e = launch_transpose_b8(table, rows, W, num_shots, out, s);
    return e == hipSuccess ? STIM_OK : hip_error(e, "b8 launch");
  }
  uint64_t *T = nullptr, *lens = nullptr, *offs = nullptr, *total = nullptr, *sums = nullptr;
  auto release = [&]() {
    void *ptrs[] = {T, lens, offs, total, sums};
    for (void *q : ptrs) if (q) (void)hipFreeAsync(q, s);
  };
  if ((e = hipMallocAsync((void **)&T, std::max<uint64_t>(num_shots * transpose_stride(rows), 1) * 8, s)) !=
      hipSuccess)
    return set_error(STIM_E_OOM, "transpose scratch allocation failed");
  if ((e = launch_transpose(table, rows, W, num_shots, T, s)) != hipSuccess) {
    release();
    return hip_error(e, "transpose launch");
  }
  if (dense) {
    e = launch_dense_format(T, rows, num_shots, format == STIM_FORMAT_B8, out, s);
    release();
    return e == hipSuccess ? STIM_OK : hip_error(e, "format launch");
  }
  const int r8 = format == STIM_FORMAT_R8;
  if ((e = hipMallocAsync((void **)&lens, num_shots * 8, s)) != hipSuccess ||
      (e = hipMallocAsync((void **)&offs, num_shots * 8, s)) != hipSuccess ||
      (e = hipMallocAsync((void **)&total, 8, s)) != hipSuccess ||
      (e = hipMallocAsync((void **)&sums, kScanBlocks * 8, s)) != hipSuccess) {
    release();
    return set_error(STIM_E_OOM, "format scratch allocation failed");
  }
  uint64_t host_total = 0;
  if ((e = launch_sparse_format(T, rows, num_shots, r8, lens, nullptr, nullptr, s)) != hipSuccess ||
      (e = launch_scan(lens, num_shots, offs, sums, total, s)) != hipSuccess ||
      (e = hipMemcpyAsync(&host_total, total, 8, hipMemcpyDeviceToHost, s)) != hipSuccess ||
      (e = hipStreamSynchronize(s)) != hipSuccess) {
    release();
    return hip_error(e, "format size pass");
  }
  *out_len = host_total;
  if (out_cap < host_total) {
    release();
    if (out_cap == 0 && !out) return STIM_OK;            // size query
    return set_error(STIM_E_INVALID_ARG, "output buffer too small");
  }
  e = launch_sparse_format(T, rows, num_shots, r8, lens, offs, out, s);
  release();
  return e == hipSuccess ? STIM_OK : hip_error(e, "format launch");
}

int stim_kernel_timing(int enable) {
  std::lock_guard<std::mutex> lock(g_timing_mu);
  release_timing();
  g_timing_on = enable != 0;
  return STIM_OK;
}

int stim_kernel_times(double *noise_gen_ms, double *frame_ms, uint64_t *passes) {
  std::lock_guard<std::mutex> lock(g_timing_mu);
  double gen = 0, frame = 0;
  for (PassEvents &t : g_timing) {
    hipError_t e = hipEventSynchronize(t.end);
    float a = 0, b = 0;
    if (e == hipSuccess && t.prepass) e = hipEventElapsedTime(&a, t.start, t.mid);
    if (e == hipSuccess) e = hipEventElapsedTime(&b, t.mid, t.end);
    if (e != hipSuccess) {
      release_timing();
      return hip_error(e, "kernel timing events");
    }
    gen += a;
    frame += b;
  }
  if (noise_gen_ms) *noise_gen_ms = gen;
  if (frame_ms) *frame_ms = frame;
  if (passes) *passes = g_timing.size();
  release_timing();
  return STIM_OK;
}

int stim_batch_sample(const stim_request *reqs, size_t n, void *hip_stream) {
  if (!reqs && n) return set_error(STIM_E_INVALID_ARG, "null request array");
  if (n == 0) return STIM_OK;
  if (n > 0xFFFFFFFFull) return set_error(STIM_E_UNSUPPORTED, "too many requests");
  hipStream_t s = (hipStream_t)hip_stream;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_error(e, "hipGetDevice");
  for (size_t i = 0; i < n; i++) {
    const stim_request &r = reqs[i];
    int rc = check_sample_args(r.c, r.shot_offset, r.num_shots);
    if (rc) return rc;
    if (r.mode != 0 && r.mode != 1) return set_error(STIM_E_INVALID_ARG, "request mode must be 0 or 1");
    uint64_t rows = r.mode == 0 ? r.c->prog.num_measurements : r.c->prog.num_detectors;
    if (rows > 0 && !is_device_pointer(r.out0)) return set_error(STIM_E_INVALID_ARG, "out0 is not a device pointer");
    if (r.mode == 1 && r.out1 && r.c->prog.num_observables > 0 && !is_device_pointer(r.out1))
      return set_error(STIM_E_INVALID_ARG, "out1 is not a device pointer");
    if ((r.num_shots + 63) / 64 > 0xFFFFFFFFull) return set_error(STIM_E_UNSUPPORTED, "too many shots in one request");
    std::lock_guard<std::mutex> lock(r.c->mu);
    DeviceCopy *d = nullptr;
    if ((rc = ensure_reference(r.c))) return rc;
    if ((rc = ensure_device(r.c, s, &d))) return rc;
    if (r.mode == 1 && (rc = ensure_noz_program(r.c, d, s))) return rc;
  }
  std::lock_guard<std::mutex> lock(g_batch_mu);
  BatchPlan *plan = nullptr;
  for (size_t k = 0; k < g_plans.size() && !plan; k++) {
    BatchPlan &pl = *g_plans[k];
    if (pl.device != dev || pl.reqs.size() != n) continue;
    bool same = true;
    for (size_t i = 0; i < n && same; i++) same = same_request(pl.reqs[i], reqs[i]);
    if (same) plan = &pl;
  }
  // A request set seen for the first time runs as a one-shot launch; the
  // second submission of the same set builds a tuned, graph-captured plan.
  uint64_t sig = 1469598103934665603ull;
  auto mix = [&sig](uint64_t v) { sig = (sig ^ v) * 1099511628211ull; };
  mix((uint64_t)dev);
  for (size_t i = 0; i < n; i++) {
    const stim_request &r = reqs[i];
    mix((uint64_t)(uintptr_t)r.c); mix(r.seed); mix(r.shot_offset); mix(r.num_shots); mix((uint64_t)r.mode);
    mix((uint64_t)(uintptr_t)r.out0); mix((uint64_t)(uintptr_t)r.out1);
  }
  if (!plan && std::find(g_seen.begin(), g_seen.end(), sig) == g_seen.end()) {
    g_seen.push_back(sig);
    if (g_seen.size() > 64) g_seen.erase(g_seen.begin());
    BatchPlan once;
    once.device = dev;
    once.reqs.assign(reqs, reqs + n);
    int rc = run_one_shot(once, s);
    if (rc) return rc;
    for (size_t i : once.single) {
      const stim_request &r = once.reqs[i];
      rc = r.mode == 0 ? stim_frame_sample(r.c, r.seed, r.shot_offset, r.num_shots, r.out0, hip_stream)
                       : stim_detector_sample(r.c, r.seed, r.shot_offset, r.num_shots, r.out0, r.out1, hip_stream);
      if (rc) return rc;
    }
    return STIM_OK;
  }
  if (!plan) {
    std::unique_ptr<BatchPlan> pl(new BatchPlan());
    pl->device = dev;
    pl->reqs.assign(reqs, reqs + n);
    int rc = build_plan(*pl, s);
    if (rc) {
      free_plan(pl.get());
      return rc;
    }
    if (g_plans.size() >= 8) {
      free_plan(g_plans.front().get());
      g_plans.erase(g_plans.begin());
    }
    g_plans.push_back(std::move(pl));
    plan = g_plans.back().get();
  }
  if (plan->exec && (e = hipGraphLaunch(plan->exec, s)) != hipSuccess) return hip_error(e, "hipGraphLaunch");
  // Requests whose frames do not fit in LDS run through the single-request path.
  for (size_t i : plan->single) {
    const stim_request &r = plan->reqs[i];
    int rc = r.mode == 0 ? stim_frame_sample(r.c, r.seed, r.shot_offset, r.num_shots, r.out0, hip_stream)
                         : stim_detector_sample(r.c, r.seed, r.shot_offset, r.num_shots, r.out0, r.out1, hip_stream);
    if (rc) return rc;
  }
  return STIM_OK;
}

}  // extern "C"
