// Host-side circuit representation of the sampler: parse tree, compiled device
// program and the metadata the kernels need.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

namespace stimgpu {

// Operation vocabulary (Sec. 5.10 format).  Frame rules per Clifford are the
// unsigned xz-linear maps of their tableaus (Sec. 3, Sec. 5.1):
//   swap(x, z): H, SQRT_Y, SQRT_Y_DAG      z ^= x: S, S_DAG, H_XY
//   x ^= z: SQRT_X, SQRT_X_DAG, H_YZ       none: I, X, Y, Z
enum Gate : uint8_t {
  G_I, G_X, G_Y, G_Z, G_H, G_H_XY, G_H_YZ, G_S, G_S_DAG, G_SQRT_X, G_SQRT_X_DAG,
  G_SQRT_Y, G_SQRT_Y_DAG, G_CX, G_CY, G_CZ, G_SWAP, G_R, G_M, G_MR,
  G_X_ERROR, G_Y_ERROR, G_Z_ERROR, G_DEPOLARIZE1, G_DEPOLARIZE2,
  G_DETECTOR, G_OBSERVABLE_INCLUDE, G_TICK, G_QUBIT_COORDS, G_SHIFT_COORDS,
  G_NUM
};

bool gate_is_two_qubit(Gate g);
bool gate_is_noise(Gate g);
bool gate_is_clifford(Gate g);
const char *gate_name(Gate g);

// One line of circuit text, or a REPEAT block.
struct Node {
  bool repeat = false;
  uint64_t reps = 0;
  std::vector<Node> body;
  Gate gate = G_TICK;
  double p = 0;                    // noise probability / observable index
  std::vector<uint32_t> targets;   // qubits, or lookbacks k of rec[-k] (CX/CY/CZ: | TGT_REC)
  int line = 0;
};

// Flag on a CX / CY / CZ target in the parse tree: a measurement-record
// control rec[-k] (k in the low bits) rather than a qubit (Sec. 3, tracking
// corrections).
constexpr uint32_t TGT_REC = 1u << 31;

// Kernel operation codes.
enum OpCode : uint32_t {
  OP_INIT = 0,      // x := 0, z := ZRAND for every qubit (targets = all qubits)
  OP_SWAP_XZ,       // H-like
  OP_Z_XOR_X,       // S-like
  OP_X_XOR_Z,       // SQRT_X-like
  OP_CX, OP_CY, OP_CZ, OP_SWAP,
  OP_R, OP_M, OP_MR,
  OP_NOISE_X, OP_NOISE_Y, OP_NOISE_Z, OP_NOISE_DEP1, OP_NOISE_DEP2,
  OP_LOOP_BEGIN, OP_LOOP_END,
  // Classically controlled Pauli X / Y / Z: pairs (qubit, lookback k); the
  // frame of shots whose result k measurements back differs from the
  // reference's takes the Pauli.
  OP_FB_X, OP_FB_Y, OP_FB_Z,
  // Detection events formed during the walk (Sec. 5.6; used only when the
  // walk keeps recent measurement flips in a ring): DET = op.n consecutive
  // detectors, each the XOR of op.aux lookbacks k (flip of the measurement k
  // back; zero entries pad a detector's list); OBS = observable op.aux takes
  // the XOR of op.n lookbacks.  Neither changes the frame.
  OP_DET, OP_OBS,
  OP_COUNT
};

// Flag in OpCode word: this op starts a new instruction (advance the flat
// index) rather than continuing the previous one after a split.
constexpr uint32_t OPF_NEW_INSTR = 1u << 16;
// Flag in OpCode word of a collapse op (INIT, R, M, MR): every target's ZRAND
// is read later, so the draws need not wait for the target list.
constexpr uint32_t OPF_ZRAND_LIVE = 1u << 17;
// Flag on a target word: the ZRAND of this collapse target is never read
// before it is overwritten, so it need not be drawn.
constexpr uint32_t TGT_DEAD_ZRAND = 1u << 31;
constexpr uint32_t TGT_QUBIT_MASK = ~TGT_DEAD_ZRAND;
// Flag on the qubit word of a classically controlled pair (same bit as
// TGT_DEAD_ZRAND, which only collapse targets carry): the controlling result
// is a Z measurement of this same qubit, and nothing has acted on the qubit
// since, so the result's flip is the qubit's current frame x bit.
constexpr uint32_t TGT_FB_LOCAL = 1u << 31;
// Flag in OpCode word of a classically controlled op: every pair is local.
constexpr uint32_t OPF_FB_LOCAL = 1u << 18;
// Flags of the detector-mode program without Z randomisations: an M whose
// next frame op is an R of the same qubits resets them itself, right after
// measuring (always, or only when its enclosing loop goes round again and the
// R starts the loop body); that R then does nothing when it follows a reset
// M.  With the randomisations gone, M then R is exactly MR.
constexpr uint32_t OPF_M_RESETS = 1u << 19, OPF_M_RESETS_IN_LOOP = 1u << 20, OPF_R_AFTER_M = 1u << 21;
// Flag of the same program on a Clifford op whose qubits are all zero in
// every shot's frame when it runs (a Clifford maps zero to zero): skipped.
constexpr uint32_t OPF_ZERO_SKIP = 1u << 22;

// Device program entry (32 bytes).
struct DevOp {
  uint32_t code;    // OpCode | flags
  uint32_t lead;    // flat instructions (annotations, Pauli gates) skipped before it
  uint32_t n;       // targets (qubits), or pairs for two-qubit ops
  uint32_t toff;    // offset of the first target word in the target array
  uint32_t slot0;   // slot (position in the user instruction) of the first target
  uint32_t aux;     // noise: threshold row; loop begin: repetitions; loop end: begin pc
  uint32_t aux2;    // loop begin: pc of the matching loop end
  uint32_t pad;
};

struct Program {
  // The device program without event ops (DET / OBS), and the same program
  // with them (for walks that form detection events; loop targets renumbered,
  // every other entry equal to its counterpart in `ops`).
  std::vector<DevOp> ops;
  std::vector<DevOp> event_ops;
  std::vector<uint32_t> targets;
  std::vector<uint64_t> thresholds;        // [rows][64]
  std::vector<uint32_t> det_offsets;       // CSR over detectors, size D + 1
  std::vector<uint32_t> det_indices;       // absolute measurement indices
  std::vector<uint32_t> obs_offsets;       // CSR over observables, size L + 1
  std::vector<uint32_t> obs_indices;
  // Order in which the event kernel visits detectors: chains of detectors
  // that share a measurement (each continues from the latest measurement of
  // the previous one), so that a shared flip row is loaded once.
  std::vector<uint32_t> det_order;
  // The same order cut into blocks for the event kernel, kDetBlockWords words
  // each: see DetBlock below.
  std::vector<uint32_t> det_blocks;
  uint64_t num_qubits = 0, num_measurements = 0, num_detectors = 0, num_observables = 0;
  uint64_t num_gate_targets = 0, num_noise_targets = 0, num_instructions = 0;
  uint32_t max_loop_depth = 0;
  // Largest lookback k of a detector, observable or classically controlled
  // pair, and most measurements of one op: a ring of max_lookback +
  // max_measure_op rows holds every flip an event op or feedback reads.
  uint32_t max_lookback = 0, max_measure_op = 0;
  // Every execution of a noise op in walk order: its pc and flat instruction
  // index (empty when there are too many to tabulate).
  std::vector<uint32_t> noise_pc;
  std::vector<uint64_t> noise_instr;
};

// A block of consecutive detectors (in det_order) that together read at most
// kDetBlockRows distinct flip rows, at most kDetBlockDets of them:
//   word 0: detectors | rows << 8 | (1 << 31 when the block is one detector
//           with more rows, read through the CSR lists instead);
//   words 1 .. 20: the rows (measurement indices), or word 1 = that detector;
//   words 21 .. 36: the detectors;
//   words 37 .. 52: per detector, the rows it XORs (bit r = row r; a row named
//           twice cancels).
constexpr uint32_t kDetBlockWords = 64, kDetBlockRows = 20, kDetBlockDets = 16;
constexpr uint32_t kDetBlockCsr = 1u << 31;

struct CompileError {
  int code;          // STIM_E_*
  std::string msg;
};

// Parses text into a tree (throws CompileError).
std::vector<Node> parse_circuit(const std::string &text);
// Lowers a tree into the device program (throws CompileError).
Program compile_program(const std::vector<Node> &tree);
// Canonical reference sample (Sec. 4); bit m of the result = measurement m.
std::vector<uint64_t> reference_sample(const std::vector<Node> &tree, uint64_t num_qubits,
                                       uint64_t num_measurements);
// Detectors and observables flipped by each single-Pauli error (Sec. 5.6),
// for sparse detection-event sampling.  Generators are numbered by noise
// execution (walk order), slot, then X and Z of the slot's first qubit and of
// its second (two-qubit channels); lane d < D is detector d, lane D + o is
// observable o.
struct ErrorModel {
  uint64_t num_generators = 0;
  std::vector<uint64_t> gen_base;     // per noise execution: its first generator
  std::vector<uint32_t> set_off;      // generator g: set_lanes[set_off[g] .. set_off[g + 1])
  std::vector<uint32_t> set_lanes;
};
// Builds the error sets by a backward sensitivity walk (throws CompileError
// with STIM_E_UNSUPPORTED for random detectors or observables, classically
// controlled Paulis, or circuits too long to tabulate).
ErrorModel build_error_model(const Program &P);
// Gap-sampling thresholds t[0..63] of probability p (exact integer recurrence).
void noise_thresholds(double p, uint64_t *t);

}  // namespace stimgpu
