// Circuit text -> parse tree -> device program.
//
// Format (Sec. 5.10): one operation per line; '#' starts a comment; blank
// lines are allowed; an operation broadcasts over its targets (two-qubit
// operations over consecutive pairs); REPEAT N { ... } repeats a block.
//
// The device program keeps REPEAT blocks as loops.  Random bits are keyed by
// the flat instruction index -- the position of a line in the fully unrolled
// instruction list, counting every operation and annotation line but not
// REPEAT headers or braces -- so the kernels recompute that index from a
// running counter and the per-op `lead` (lines skipped since the previous op).
#include "circuit.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <unordered_map>

#include "stim_gpu.h"

namespace stimgpu {

namespace {

struct GateSpec { const char *name; Gate gate; };
const GateSpec kGateNames[] = {
  {"I", G_I}, {"X", G_X}, {"Y", G_Y}, {"Z", G_Z}, {"H", G_H}, {"H_XZ", G_H}, {"H_XY", G_H_XY},
  {"H_YZ", G_H_YZ}, {"S", G_S}, {"SQRT_Z", G_S}, {"S_DAG", G_S_DAG}, {"SQRT_Z_DAG", G_S_DAG},
  {"SQRT_X", G_SQRT_X}, {"SQRT_X_DAG", G_SQRT_X_DAG}, {"SQRT_Y", G_SQRT_Y},
  {"SQRT_Y_DAG", G_SQRT_Y_DAG}, {"CX", G_CX}, {"CNOT", G_CX}, {"ZCX", G_CX}, {"CY", G_CY},
  {"ZCY", G_CY}, {"CZ", G_CZ}, {"ZCZ", G_CZ}, {"SWAP", G_SWAP}, {"R", G_R}, {"RZ", G_R},
  {"M", G_M}, {"MZ", G_M}, {"MR", G_MR}, {"MRZ", G_MR}, {"X_ERROR", G_X_ERROR},
  {"Y_ERROR", G_Y_ERROR}, {"Z_ERROR", G_Z_ERROR}, {"DEPOLARIZE1", G_DEPOLARIZE1},
  {"DEPOLARIZE2", G_DEPOLARIZE2}, {"DETECTOR", G_DETECTOR},
  {"OBSERVABLE_INCLUDE", G_OBSERVABLE_INCLUDE}, {"TICK", G_TICK},
  {"QUBIT_COORDS", G_QUBIT_COORDS}, {"SHIFT_COORDS", G_SHIFT_COORDS},
};

[[noreturn]] void fail(int code, int line, const std::string &msg) {
  throw CompileError{code, (line > 0 ? "line " + std::to_string(line) + ": " : std::string()) + msg};
}

// A small cursor over one line of text.
struct Cursor {
  const char *p, *end;
  int line;
  void skip_ws() { while (p < end && (*p == ' ' || *p == '\t' || *p == '\r')) p++; }
  bool done() { skip_ws(); return p >= end; }
  std::string word() {   // [A-Za-z0-9_]+ upper-cased
    skip_ws();
    std::string s;
    while (p < end && (std::isalnum((unsigned char)*p) || *p == '_')) s += (char)std::toupper((unsigned char)*p++);
    return s;
  }
  uint64_t integer() {
    skip_ws();
    if (p >= end || !std::isdigit((unsigned char)*p)) fail(STIM_E_PARSE, line, "expected an integer");
    uint64_t v = 0;
    while (p < end && std::isdigit((unsigned char)*p)) {
      uint64_t d = (uint64_t)(*p++ - '0');
      if (v > (UINT64_MAX - d) / 10) fail(STIM_E_PARSE, line, "integer too large");
      v = v * 10 + d;
    }
    if (p < end && !(*p == ' ' || *p == '\t' || *p == '\r' || *p == '{' || *p == ']' || *p == ')' || *p == ','))
      fail(STIM_E_PARSE, line, "bad character after integer");
    return v;
  }
};

std::vector<double> parse_args(Cursor &c) {
  std::vector<double> args;
  c.skip_ws();
  if (c.p >= c.end || *c.p != '(') return args;
  c.p++;
  while (true) {
    c.skip_ws();
    const char *start = c.p;
    while (c.p < c.end && *c.p != ',' && *c.p != ')') c.p++;
    if (c.p >= c.end) fail(STIM_E_PARSE, c.line, "unterminated argument list");
    std::string tok(start, c.p);
    while (!tok.empty() && (tok.back() == ' ' || tok.back() == '\t')) tok.pop_back();
    char *e = nullptr;
    double v = std::strtod(tok.c_str(), &e);
    if (tok.empty() || *e != '\0') fail(STIM_E_PARSE, c.line, "bad argument '" + tok + "'");
    args.push_back(v);
    if (*c.p == ')') { c.p++; break; }
    c.p++;
  }
  return args;
}

// Parses lines [pos, ...) into `out` until a closing brace (depth > 0) or EOF.
void parse_block(const std::vector<std::pair<const char *, const char *>> &lines, size_t &pos,
                 std::vector<Node> &out, int depth, int open_line) {
  while (pos < lines.size()) {
    Cursor c{lines[pos].first, lines[pos].second, (int)pos + 1};
    pos++;
    // strip comment
    for (const char *q = c.p; q < c.end; q++) if (*q == '#') { c.end = q; break; }
    if (c.done()) continue;
    if (*c.p == '}') {
      c.p++;
      if (!c.done()) fail(STIM_E_PARSE, c.line, "text after '}'");
      if (depth == 0) fail(STIM_E_PARSE, c.line, "'}' without REPEAT");
      return;
    }
    std::string name = c.word();
    if (name.empty()) fail(STIM_E_PARSE, c.line, "expected an operation name");
    if (name == "REPEAT") {
      Node n;
      n.repeat = true;
      n.line = c.line;
      n.reps = c.integer();
      c.skip_ws();
      if (c.p >= c.end || *c.p != '{') fail(STIM_E_PARSE, c.line, "expected '{' after REPEAT count");
      c.p++;
      if (!c.done()) fail(STIM_E_PARSE, c.line, "text after '{'");
      if (n.reps == 0) fail(STIM_E_PARSE, c.line, "REPEAT 0 is not allowed");
      if (n.reps > 0xFFFFFFFFull) fail(STIM_E_UNSUPPORTED, c.line, "REPEAT count above 2^32 - 1");
      parse_block(lines, pos, n.body, depth + 1, c.line);
      out.push_back(std::move(n));
      continue;
    }
    const GateSpec *spec = nullptr;
    for (const GateSpec &g : kGateNames) if (name == g.name) spec = &g;
    if (!spec) fail(STIM_E_UNSUPPORTED, c.line, "unsupported operation '" + name + "'");
    Node n;
    n.gate = spec->gate;
    n.line = c.line;
    std::vector<double> args = parse_args(c);
    bool recs = n.gate == G_DETECTOR || n.gate == G_OBSERVABLE_INCLUDE;
    bool ann = n.gate == G_TICK || n.gate == G_QUBIT_COORDS || n.gate == G_SHIFT_COORDS;
    if (gate_is_noise(n.gate)) {
      if (args.size() != 1) fail(STIM_E_PARSE, c.line, "noise channel takes one probability");
      if (!(args[0] >= 0.0 && args[0] <= 1.0)) fail(STIM_E_PARSE, c.line, "probability outside [0, 1]");
      n.p = args[0];
    } else if (n.gate == G_OBSERVABLE_INCLUDE) {
      if (args.size() != 1 || args[0] < 0 || args[0] != std::floor(args[0]) || args[0] > 1e9)
        fail(STIM_E_PARSE, c.line, "OBSERVABLE_INCLUDE takes one non-negative integer");
      n.p = args[0];
    } else if (!recs && !ann && !args.empty()) {
      fail(STIM_E_PARSE, c.line, "operation takes no arguments");
    }
    const bool controllable = n.gate == G_CX || n.gate == G_CY || n.gate == G_CZ;
    auto lookback = [&]() -> uint64_t {
      std::string w = c.word();
      if (w != "REC" || c.p + 2 > c.end || c.p[0] != '[' || c.p[1] != '-')
        fail(STIM_E_PARSE, c.line, "expected rec[-k]");
      c.p += 2;
      uint64_t k = c.integer();
      if (c.p >= c.end || *c.p != ']') fail(STIM_E_PARSE, c.line, "expected ']'");
      c.p++;
      if (k == 0) fail(STIM_E_PARSE, c.line, "bad lookback");
      return k;
    };
    while (!c.done()) {
      if (recs) {
        uint64_t k = lookback();
        if (k > 0xFFFFFFFFull) fail(STIM_E_PARSE, c.line, "bad lookback");
        n.targets.push_back((uint32_t)k);
      } else if (controllable && std::isalpha((unsigned char)*c.p)) {
        uint64_t k = lookback();
        if (k >= TGT_REC) fail(STIM_E_UNSUPPORTED, c.line, "lookback too large");
        n.targets.push_back((uint32_t)k | TGT_REC);
      } else if (ann) {
        while (c.p < c.end && *c.p != ' ' && *c.p != '\t') c.p++;   // coordinates etc. ignored
      } else {
        uint64_t q = c.integer();
        if (q >= (1ull << 31)) fail(STIM_E_UNSUPPORTED, c.line, "qubit index too large");
        n.targets.push_back((uint32_t)q);
      }
    }
    if (gate_is_two_qubit(n.gate)) {
      if (n.targets.size() % 2) fail(STIM_E_PARSE, c.line, "two-qubit operation needs pairs of targets");
      for (size_t k = 0; k < n.targets.size(); k += 2) {
        const bool ra = (n.targets[k] & TGT_REC) != 0, rb = (n.targets[k + 1] & TGT_REC) != 0;
        if (ra && rb) fail(STIM_E_PARSE, c.line, "both targets are measurement records");
        if (rb && n.gate != G_CZ) fail(STIM_E_PARSE, c.line, "a measurement record can only be the control");
        if (!ra && !rb && n.targets[k] == n.targets[k + 1])
          fail(STIM_E_PARSE, c.line, "two-qubit operation on one qubit");
      }
    }
    out.push_back(std::move(n));
  }
  if (depth > 0) fail(STIM_E_PARSE, open_line, "REPEAT block is not closed");
}

// --- lowering ------------------------------------------------------------

struct Lowering {
  Program prog;
  uint32_t pending_lead = 0;
  std::map<uint64_t, uint32_t> threshold_rows;          // bits of p -> row
  std::unordered_map<const Node *, std::vector<uint32_t>> slot_targets;  // collapse slots -> target index
  std::unordered_map<const Node *, std::vector<uint32_t>> fb_targets;    // controlled pairs -> qubit word index
  uint32_t depth = 0;
  // Consecutive DETECTOR lines not yet emitted (no op between them).
  std::vector<const Node *> dets;

  // Emits the pending detectors as one DET op: lookback lists padded with
  // zeros to a common even length, starting on an even target index (pairs
  // are read as one 8-byte word).
  void flush_detectors() {
    if (dets.empty()) return;
    size_t c = 2;
    for (const Node *d : dets) c = std::max(c, (d->targets.size() + 1) & ~(size_t)1);
    if (prog.targets.size() % 2) prog.targets.push_back(0);
    DevOp op{};
    op.code = OP_DET;
    op.n = (uint32_t)dets.size();
    op.toff = (uint32_t)prog.targets.size();
    op.aux = (uint32_t)c;
    for (const Node *d : dets)
      for (size_t i = 0; i < c; i++) prog.targets.push_back(i < d->targets.size() ? d->targets[i] : 0u);
    prog.ops.push_back(op);
    dets.clear();
  }

  uint32_t threshold_row(double p) {
    uint64_t bits;
    std::memcpy(&bits, &p, 8);
    auto it = threshold_rows.find(bits);
    if (it != threshold_rows.end()) return it->second;
    uint32_t row = (uint32_t)threshold_rows.size();
    threshold_rows[bits] = row;
    size_t base = prog.thresholds.size();
    prog.thresholds.resize(base + 64);
    noise_thresholds(p, &prog.thresholds[base]);
    return row;
  }

  static OpCode opcode(Gate g) {
    switch (g) {
      case G_H: case G_SQRT_Y: case G_SQRT_Y_DAG: return OP_SWAP_XZ;
      case G_S: case G_S_DAG: case G_H_XY: return OP_Z_XOR_X;
      case G_SQRT_X: case G_SQRT_X_DAG: case G_H_YZ: return OP_X_XOR_Z;
      case G_CX: return OP_CX;
      case G_CY: return OP_CY;
      case G_CZ: return OP_CZ;
      case G_SWAP: return OP_SWAP;
      case G_R: return OP_R;
      case G_M: return OP_M;
      case G_MR: return OP_MR;
      case G_X_ERROR: return OP_NOISE_X;
      case G_Y_ERROR: return OP_NOISE_Y;
      case G_Z_ERROR: return OP_NOISE_Z;
      case G_DEPOLARIZE1: return OP_NOISE_DEP1;
      case G_DEPOLARIZE2: return OP_NOISE_DEP2;
      default: return OP_COUNT;
    }
  }

  // A CX / CY / CZ line with measurement-record controls: runs of ordinary
  // pairs and runs of classically controlled pairs, in line order, each split
  // where a qubit repeats.  Controlled pairs are stored as (qubit, lookback).
  void emit_controlled_line(const Node &n) {
    const OpCode quantum = opcode(n.gate);
    const OpCode fb = n.gate == G_CX ? OP_FB_X : n.gate == G_CY ? OP_FB_Y : OP_FB_Z;
    const size_t pairs = n.targets.size() / 2;
    if (prog.targets.size() % 2) prog.targets.push_back(0);     // pairs start on an even index
    std::vector<uint32_t> &fbt = fb_targets[&n];
    fbt.assign(pairs, 0xFFFFFFFFu);
    std::unordered_map<uint32_t, int> used;
    bool first = true;
    size_t s = 0;
    while (s < pairs) {
      auto is_fb = [&](size_t i) { return ((n.targets[2 * i] | n.targets[2 * i + 1]) & TGT_REC) != 0; };
      const bool kind = is_fb(s);
      used.clear();
      DevOp op{};
      op.code = (uint32_t)(kind ? fb : quantum) | (first ? OPF_NEW_INSTR : 0);
      op.lead = first ? pending_lead : 0;
      op.toff = (uint32_t)prog.targets.size();
      op.slot0 = (uint32_t)s;
      while (s < pairs && is_fb(s) == kind) {
        uint32_t a = n.targets[2 * s], b = n.targets[2 * s + 1];
        if (kind && (a & TGT_REC)) std::swap(a, b);          // (qubit, record)
        if (kind) prog.max_lookback = std::max(prog.max_lookback, b & ~TGT_REC);
        if (used.count(a) || (!kind && used.count(b))) break;
        used[a] = 1;
        if (!kind) used[b] = 1;
        if (kind) fbt[s] = (uint32_t)prog.targets.size();
        prog.targets.push_back(a);
        prog.targets.push_back(kind ? (b & ~TGT_REC) : b);
        s++;
        op.n++;
      }
      prog.ops.push_back(op);
      first = false;
    }
    pending_lead = 0;
  }

  void emit_line(const Node &n) {
    // Event ops take no flat index of their own: the DETECTOR and
    // OBSERVABLE_INCLUDE lines stay counted in the lead of the next op.
    if (n.gate == G_DETECTOR || n.gate == G_OBSERVABLE_INCLUDE) {
      pending_lead++;
      for (uint32_t k : n.targets) prog.max_lookback = std::max(prog.max_lookback, k);
      if (n.gate == G_DETECTOR) {       // an empty one is an event row of zeros
        dets.push_back(&n);
        return;
      }
      if (n.targets.empty()) return;
      flush_detectors();
      DevOp op{};
      op.code = OP_OBS;
      op.n = (uint32_t)n.targets.size();
      op.toff = (uint32_t)prog.targets.size();
      op.aux = (uint32_t)n.p;
      prog.targets.insert(prog.targets.end(), n.targets.begin(), n.targets.end());
      prog.ops.push_back(op);
      return;
    }
    if (n.gate == G_QUBIT_COORDS || n.gate == G_SHIFT_COORDS || n.gate == G_TICK) {
      pending_lead++;
      return;
    }
    flush_detectors();
    if (n.gate == G_CX || n.gate == G_CY || n.gate == G_CZ) {
      bool controlled = false;
      for (uint32_t t : n.targets) controlled |= (t & TGT_REC) != 0;
      if (controlled) {
        emit_controlled_line(n);
        return;
      }
    }
    OpCode code = opcode(n.gate);
    if (code == OP_COUNT || n.targets.empty() || (gate_is_noise(n.gate) && n.p == 0)) {
      pending_lead++;   // annotation, frame no-op or empty: only advances the flat index
      return;
    }
    int k = gate_is_two_qubit(n.gate) ? 2 : 1;
    // Pairs start on an even index, so that a kernel reads a pair as one
    // 8-byte word; the padding word belongs to no op.
    if (k == 2 && prog.targets.size() % 2) prog.targets.push_back(0);
    uint32_t aux = gate_is_noise(n.gate) ? threshold_row(n.p) : 0;
    size_t slots = n.targets.size() / k;
    bool collapse = code == OP_R || code == OP_M || code == OP_MR;
    std::vector<uint32_t> &slot_tidx = slot_targets[&n];
    if (collapse) slot_tidx.resize(slots);
    // Split into segments whose qubits are pairwise distinct, so that a segment
    // can update all of its targets in parallel.
    std::unordered_map<uint32_t, int> used;
    size_t s = 0;
    bool first = true;
    while (s < slots) {
      used.clear();
      DevOp op{};
      op.code = (uint32_t)code | (first ? OPF_NEW_INSTR : 0);
      op.lead = first ? pending_lead : 0;
      op.toff = (uint32_t)prog.targets.size();
      op.slot0 = (uint32_t)s;
      op.aux = aux;
      while (s < slots) {
        bool clash = false;
        for (int j = 0; j < k; j++) clash |= used.count(n.targets[s * k + j]) > 0;
        if (clash) break;
        for (int j = 0; j < k; j++) {
          used[n.targets[s * k + j]] = 1;
          if (collapse) slot_tidx[s] = (uint32_t)prog.targets.size();
          prog.targets.push_back(n.targets[s * k + j]);
        }
        s++;
        op.n++;
      }
      if (code == OP_M || code == OP_MR) prog.max_measure_op = std::max(prog.max_measure_op, op.n);
      prog.ops.push_back(op);
      first = false;
    }
    pending_lead = 0;
  }

  void emit_block(const std::vector<Node> &nodes) {
    for (const Node &n : nodes) {
      if (!n.repeat) {
        emit_line(n);
        continue;
      }
      flush_detectors();
      depth++;
      if (depth > prog.max_loop_depth) prog.max_loop_depth = depth;
      uint32_t begin = (uint32_t)prog.ops.size();
      DevOp b{};
      b.code = OP_LOOP_BEGIN;
      b.lead = pending_lead;
      b.aux = (uint32_t)n.reps;
      pending_lead = 0;
      prog.ops.push_back(b);
      emit_block(n.body);
      flush_detectors();
      DevOp e{};
      e.code = OP_LOOP_END;
      e.lead = pending_lead;
      e.aux = begin;
      pending_lead = 0;
      prog.ops[begin].aux2 = (uint32_t)prog.ops.size();
      prog.ops.push_back(e);
      depth--;
    }
  }
};

// Walks the fully unrolled circuit: measurement numbering, detector sets,
// counts, and which post-collapse Z randomisations are ever read.
struct Walker {
  Lowering &L;
  uint64_t meas = 0, flat = 0;
  std::vector<std::vector<uint32_t>> observables;
  std::vector<uint64_t> pending;      // per qubit: site awaiting a verdict (or NONE)
  std::vector<uint8_t> site_live;     // per target index; then n init sites
  static constexpr uint64_t NONE = ~0ull;
  // Local feedback: per qubit the instruction that last acted on it; per
  // measurement its qubit, instruction and whether it was a plain M; per
  // controlled pair's qubit word whether every execution was local.
  // The last fb_window measurements are kept (a ring; fb_window = the
  // largest lookback of a controlled pair up to a cap, 0 without feedback).
  uint64_t clock = 0, fb_window = 0;
  std::vector<uint64_t> last_touch;
  std::vector<uint32_t> meas_qubit;
  std::vector<uint64_t> meas_clock;
  std::vector<uint8_t> meas_plain;
  std::vector<uint8_t> fb_local;      // per target index (1 until an execution is not local)

  void touch(uint32_t q, bool overwrites_z, uint64_t new_site) {
    if (pending[q] != NONE && !overwrites_z) site_live[pending[q]] = 1;
    pending[q] = new_site;
  }

  void walk(const std::vector<Node> &nodes) {
    for (const Node &n : nodes) {
      if (n.repeat) {
        for (uint64_t r = 0; r < n.reps; r++) walk(n.body);
        continue;
      }
      flat++;
      clock++;
      Program &P = L.prog;
      switch (n.gate) {
        case G_DETECTOR:
        case G_OBSERVABLE_INCLUDE: {
          std::vector<uint32_t> idx;
          for (uint32_t k : n.targets) {
            if (k > meas) fail(STIM_E_PARSE, n.line, "rec[-" + std::to_string(k) + "] reaches before the first measurement");
            idx.push_back((uint32_t)(meas - k));
          }
          if (n.gate == G_DETECTOR) {
            P.det_indices.insert(P.det_indices.end(), idx.begin(), idx.end());
            P.det_offsets.push_back((uint32_t)P.det_indices.size());
            P.num_detectors++;
          } else {
            size_t o = (size_t)n.p;
            if (o >= observables.size()) observables.resize(o + 1);
            observables[o].insert(observables[o].end(), idx.begin(), idx.end());
          }
          break;
        }
        case G_I: case G_X: case G_Y: case G_Z:
          P.num_gate_targets += n.targets.size();
          break;
        case G_R: case G_M: case G_MR: {
          const std::vector<uint32_t> &tid = L.slot_targets.at(&n);
          for (size_t s = 0; s < n.targets.size(); s++) {
            touch(n.targets[s], n.gate != G_M, tid[s]);
            last_touch[n.targets[s]] = clock;
            if (n.gate != G_R && fb_window > 0) {
              const size_t r = (size_t)((meas + s) % (fb_window + 1));
              meas_qubit[r] = n.targets[s];
              meas_clock[r] = clock;
              meas_plain[r] = n.gate == G_M;
            }
          }
          if (n.gate != G_R) meas += n.targets.size();
          P.num_gate_targets += n.targets.size();
          break;
        }
        default:
          if (gate_is_noise(n.gate)) {
            P.num_noise_targets += n.targets.size() / (gate_is_two_qubit(n.gate) ? 2 : 1);
            for (uint32_t q : n.targets) last_touch[q] = clock;
          } else if (gate_is_clifford(n.gate)) {
            for (uint32_t q : n.targets) {
              if (q & TGT_REC) {
                const uint64_t k = q & ~TGT_REC;
                if (k > meas) fail(STIM_E_PARSE, n.line, "rec[-" + std::to_string(k) + "] reaches before the first measurement");
                continue;
              }
              touch(q, false, NONE);
            }
            auto fbt = L.fb_targets.find(&n);
            if (fbt != L.fb_targets.end()) {
              // Pairs in line order (the order the ops run in).  A controlled
              // pair (qubit q, record k) is local when record k is a plain M
              // of q and nothing has acted on q since -- not even an earlier
              // pair of this line.
              for (size_t i = 0; i < fbt->second.size(); i++) {
                uint32_t a = n.targets[2 * i], b = n.targets[2 * i + 1];
                if (fbt->second[i] == 0xFFFFFFFFu) {
                  last_touch[a] = last_touch[b] = clock;
                  continue;
                }
                if (a & TGT_REC) std::swap(a, b);
                const uint64_t k = b & ~TGT_REC;
                bool local = k <= fb_window;
                if (local) {
                  const size_t r = (size_t)((meas - k) % (fb_window + 1));
                  local = meas_qubit[r] == a && meas_plain[r] && last_touch[a] == meas_clock[r];
                }
                if (!local) fb_local[fbt->second[i]] = 0;
                last_touch[a] = clock;
              }
            } else {
              for (uint32_t q : n.targets) last_touch[q] = clock;
            }
            P.num_gate_targets += n.targets.size() / (gate_is_two_qubit(n.gate) ? 2 : 1);
          }
          break;
      }
      if (meas > 0xFFFFFFFFull) fail(STIM_E_UNSUPPORTED, n.line, "more than 2^32 - 1 measurements");
    }
  }
};

uint64_t max_qubit(const std::vector<Node> &nodes) {
  uint64_t m = 0;
  for (const Node &n : nodes) {
    if (n.repeat) { m = std::max(m, max_qubit(n.body)); continue; }
    if (n.gate == G_DETECTOR || n.gate == G_OBSERVABLE_INCLUDE) continue;
    for (uint32_t q : n.targets)
      if (!(q & TGT_REC)) m = std::max(m, (uint64_t)q + 1);
  }
  return m;
}

}  // namespace

bool gate_is_two_qubit(Gate g) {
  return g == G_CX || g == G_CY || g == G_CZ || g == G_SWAP || g == G_DEPOLARIZE2;
}
bool gate_is_noise(Gate g) { return g >= G_X_ERROR && g <= G_DEPOLARIZE2; }
bool gate_is_clifford(Gate g) { return g <= G_SWAP; }
const char *gate_name(Gate g) {
  for (const GateSpec &s : kGateNames) if (s.gate == g) return s.name;
  return "?";
}

// Exact thresholds for gap sampling: a = floor((1 - p) 2^64) computed from the
// binary value of p, t[0] = a, t[g] = floor(t[g-1] a / 2^64).  A uniform 64-bit
// draw u satisfies u < t[g-1] with probability ~(1-p)^g.
void noise_thresholds(double p, uint64_t *t) {
  typedef unsigned __int128 u128;
  // p = m * 2^(e - 53) with m a 53-bit integer.
  int e = 0;
  double frac = std::frexp(p, &e);
  uint64_t m = (uint64_t)std::ldexp(frac, 53);
  int s = e - 53 + 64;          // p * 2^64 = m * 2^s
  u128 up;                      // ceil(p * 2^64)
  if (m == 0) up = 0;
  else if (s >= 0) up = (u128)m << s;
  else if (s > -64) up = ((u128)m >> -s) + ((((u128)m) & ((((u128)1) << -s) - 1)) != 0);
  else up = 1;
  u128 one = (u128)1 << 64;
  uint64_t a = up == 0 ? ~0ull : (uint64_t)(one - up);
  u128 cur = a;
  for (int g = 0; g < 64; g++) {
    t[g] = (uint64_t)cur;
    cur = (cur * (u128)a) >> 64;
  }
}

std::vector<Node> parse_circuit(const std::string &text) {
  std::vector<std::pair<const char *, const char *>> lines;
  const char *b = text.data(), *e = b + text.size();
  while (true) {
    const char *nl = (const char *)std::memchr(b, '\n', (size_t)(e - b));
    lines.push_back({b, nl ? nl : e});
    if (!nl) break;
    b = nl + 1;
  }
  std::vector<Node> tree;
  size_t pos = 0;
  parse_block(lines, pos, tree, 0, 0);
  return tree;
}

Program compile_program(const std::vector<Node> &tree) {
  Lowering L;
  uint64_t n = max_qubit(tree);
  L.prog.num_qubits = n;
  // Initial frame randomisation: one op over every qubit.
  DevOp init{};
  init.code = OP_INIT;
  init.n = (uint32_t)n;
  init.toff = 0;
  for (uint64_t q = 0; q < n; q++) L.prog.targets.push_back((uint32_t)q);
  L.prog.ops.push_back(init);
  L.emit_block(tree);   // trailing annotations need no op: nothing after them draws bits
  L.flush_detectors();
  // Unrolled walk.
  Walker w{L};
  w.pending.assign(n, Walker::NONE);
  size_t ntar = L.prog.targets.size();
  w.site_live.assign(ntar, 0);
  w.last_touch.assign(n, 0);
  w.fb_local.assign(ntar, 1);
  // Largest lookback of a controlled pair (capped: longer ones stay global).
  for (const auto &kv : L.fb_targets)
    for (size_t i = 0; i < kv.second.size(); i++)
      if (kv.second[i] != 0xFFFFFFFFu) {
        const uint32_t a = kv.first->targets[2 * i], b = kv.first->targets[2 * i + 1];
        const uint64_t k = ((a & TGT_REC) ? a : b) & ~TGT_REC;
        w.fb_window = std::max<uint64_t>(w.fb_window, std::min<uint64_t>(k, 1u << 16));
      }
  w.meas_qubit.assign(w.fb_window + 1, 0);
  w.meas_clock.assign(w.fb_window + 1, ~0ull);
  w.meas_plain.assign(w.fb_window + 1, 0);
  for (uint64_t q = 0; q < n; q++) w.pending[q] = q;     // init sites = target slots 0..n-1
  L.prog.det_offsets.push_back(0);
  w.walk(tree);
  L.prog.num_measurements = w.meas;
  L.prog.num_instructions = w.flat;
  L.prog.obs_offsets.push_back(0);
  for (auto &o : w.observables) {
    L.prog.obs_indices.insert(L.prog.obs_indices.end(), o.begin(), o.end());
    L.prog.obs_offsets.push_back((uint32_t)L.prog.obs_indices.size());
  }
  L.prog.num_observables = w.observables.size();
  // Detector visiting order for the event kernel.
  {
    Program &P = L.prog;
    const size_t D = P.det_offsets.size() - 1;
    std::unordered_map<uint32_t, std::vector<uint32_t>> users;   // measurement -> detectors using it
    for (size_t d = 0; d < D; d++)
      for (uint32_t k = P.det_offsets[d]; k < P.det_offsets[d + 1]; k++) users[P.det_indices[k]].push_back((uint32_t)d);
    std::vector<char> seen(D, 0);
    P.det_order.reserve(D);
    for (size_t d0 = 0; d0 < D; d0++) {
      uint32_t cur = (uint32_t)d0;
      while (!seen[cur]) {
        seen[cur] = 1;
        P.det_order.push_back(cur);
        uint32_t last = 0;
        bool any = false;
        for (uint32_t k = P.det_offsets[cur]; k < P.det_offsets[cur + 1]; k++)
          if (!any || P.det_indices[k] > last) { last = P.det_indices[k]; any = true; }
        if (!any) break;
        uint32_t nxt = cur;
        for (uint32_t e : users[last])
          if (!seen[e]) { nxt = e; break; }
        if (nxt == cur) break;
        cur = nxt;
      }
    }
  }
  // Mark dead Z randomisations on init and collapse targets, and flag the
  // collapse ops whose every randomisation is live.
  for (DevOp &op : L.prog.ops) {
    uint32_t code = op.code & 0xFFFF;
    if (code != OP_INIT && code != OP_R && code != OP_M && code != OP_MR) continue;
    bool all_live = true;
    for (uint32_t k = 0; k < op.n; k++)
      if (!w.site_live[op.toff + k]) {
        L.prog.targets[op.toff + k] |= TGT_DEAD_ZRAND;
        all_live = false;
      }
    if (all_live) op.code |= OPF_ZRAND_LIVE;
  }
  // Mark local feedback pairs, and the feedback ops whose pairs all are.
  for (DevOp &op : L.prog.ops) {
    const uint32_t code = op.code & 0xFFFF;
    if (code < OP_FB_X || code > OP_FB_Z) continue;
    bool all_local = true;
    for (uint32_t k = 0; k < op.n; k++) {
      const size_t t = op.toff + 2 * (size_t)k;
      if (w.fb_local[t]) L.prog.targets[t] |= TGT_FB_LOCAL;
      else all_local = false;
    }
    if (all_local && op.n > 0) op.code |= OPF_FB_LOCAL;
  }
  // Detector blocks for the event kernel, cut greedily along det_order.
  {
    Program &P = L.prog;
    const size_t D = P.det_order.size();
    std::vector<uint32_t> rows, dets, masks;
    auto emit = [&]() {
      if (dets.empty()) return;
      const size_t b = P.det_blocks.size();
      P.det_blocks.resize(b + kDetBlockWords, 0);
      uint32_t *w = &P.det_blocks[b];
      w[0] = (uint32_t)dets.size() | (uint32_t)rows.size() << 8;
      for (size_t r = 0; r < rows.size(); r++) w[1 + r] = rows[r];
      for (size_t i = 0; i < dets.size(); i++) {
        w[1 + kDetBlockRows + i] = dets[i];
        w[1 + kDetBlockRows + kDetBlockDets + i] = masks[i];
      }
      rows.clear();
      dets.clear();
      masks.clear();
    };
    for (size_t i = 0; i < D; i++) {
      const uint32_t d = P.det_order[i];
      const uint32_t a0 = P.det_offsets[d], a1 = P.det_offsets[d + 1];
      // Rows this detector adds to the current block.
      std::vector<uint32_t> extra;
      for (uint32_t a = a0; a < a1; a++) {
        const uint32_t m = P.det_indices[a];
        if (std::find(rows.begin(), rows.end(), m) == rows.end() &&
            std::find(extra.begin(), extra.end(), m) == extra.end())
          extra.push_back(m);
      }
      if (dets.size() == kDetBlockDets || rows.size() + extra.size() > kDetBlockRows) {
        emit();
        extra.clear();
        for (uint32_t a = a0; a < a1; a++) {
          const uint32_t m = P.det_indices[a];
          if (std::find(extra.begin(), extra.end(), m) == extra.end()) extra.push_back(m);
        }
      }
      if (extra.size() > kDetBlockRows) {          // one detector with many rows: CSR block
        const size_t b = P.det_blocks.size();
        P.det_blocks.resize(b + kDetBlockWords, 0);
        P.det_blocks[b] = 1u | kDetBlockCsr;
        P.det_blocks[b + 1] = d;
        continue;
      }
      rows.insert(rows.end(), extra.begin(), extra.end());
      uint32_t mask = 0;
      for (uint32_t a = a0; a < a1; a++)
        mask ^= 1u << (uint32_t)(std::find(rows.begin(), rows.end(), P.det_indices[a]) - rows.begin());
      dets.push_back(d);
      masks.push_back(mask);
    }
    emit();
  }
  // Split off the event ops: `ops` keeps everything else, with loop targets
  // renumbered.
  {
    Program &P = L.prog;
    P.event_ops = P.ops;
    std::vector<uint32_t> newpc(P.event_ops.size() + 1, 0);
    P.ops.clear();
    for (size_t pc = 0; pc < P.event_ops.size(); pc++) {
      newpc[pc] = (uint32_t)P.ops.size();
      const uint32_t code = P.event_ops[pc].code & 0xFFFF;
      if (code != OP_DET && code != OP_OBS) P.ops.push_back(P.event_ops[pc]);
    }
    newpc[P.event_ops.size()] = (uint32_t)P.ops.size();
    for (DevOp &op : P.ops) {
      const uint32_t code = op.code & 0xFFFF;
      if (code == OP_LOOP_BEGIN) op.aux2 = newpc[op.aux2];
      if (code == OP_LOOP_END) op.aux = newpc[op.aux];
    }
  }
  // Noise-op executions in walk order (same control flow as the kernels).
  {
    const size_t kMaxInstances = 65535;
    Program &P = L.prog;
    uint64_t flat = 0, steps = 0;
    std::vector<uint32_t> left;
    bool ok = true;
    for (uint32_t pc = 0; pc < P.ops.size() && ok; pc++) {
      if (++steps > 50000000ull) { ok = false; break; }   // very long loops: no table
      const DevOp &op = P.ops[pc];
      uint32_t code = op.code & 0xFFFF;
      if (code == OP_LOOP_BEGIN) { flat += op.lead; left.push_back(op.aux); continue; }
      if (code == OP_LOOP_END) {
        flat += op.lead;
        if (--left.back() > 0) pc = op.aux;
        else left.pop_back();
        continue;
      }
      uint64_t instr = 0;
      if (code == OP_INIT) instr = ~0ull;
      else if (op.code & OPF_NEW_INSTR) { flat += op.lead; instr = flat++; }
      else instr = flat - 1;
      if (code >= OP_NOISE_X && code <= OP_NOISE_DEP2) {
        if (P.noise_pc.size() >= kMaxInstances) { ok = false; break; }
        P.noise_pc.push_back(pc);
        P.noise_instr.push_back(instr);
      }
    }
    if (!ok) { P.noise_pc.clear(); P.noise_instr.clear(); }
  }
  return L.prog;
}

}  // namespace stimgpu
