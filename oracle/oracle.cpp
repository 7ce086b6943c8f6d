// Oracle for batched Pauli-frame sampling of noisy stabilizer circuits.
//
// TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
// benchmark's CPU-baseline leg may load this library.  It shares no code with
// the GPU sampler: its own parser, gate table, tableau simulator, random number
// generator and frame simulator are written here, plainly and slowly, following
// Gidney, "Stim: a fast stabilizer circuit simulator" (arXiv:2103.02202):
//
//   * Sec. 2.1  xz encoding of Paulis; product up to phase is XOR.
//   * Sec. 2.3  stabilizer tableaus; Sec. 2.3.1 conjugating a Pauli product by a
//               tableau; Sec. 2.3.2 prepending / appending operations.
//   * Sec. 3    the Pauli frame simulation algorithm (reference sample, random
//               Z frame at initialisation, Clifford conjugation, reset, Pauli
//               noise, measurement reported as reference XOR x, then Z(0.5)).
//   * Sec. 4    inverse-tableau stabilizer simulation (prepend the inverse of
//               each gate; random measurements resolved by pivot + CNOT appends +
//               a single-qubit collapse + optional X; reset = measure, then force
//               the sign of the Z column to +).
//   * Sec. 5.5  geometric gap sampling of low-probability noise.
//   * Sec. 5.6  detection events = XOR of the detector's measurement results
//               compared with the noiseless value.
//   * Sec. 5.10 the line-oriented circuit format with REPEAT blocks.
//   * Sec. 5.11 LSB-first bit packing with zero padding.
//
// Readings where the paper is silent (each one is listed in the design notes):
//   - Canonical reference sample: every random measurement, including the one
//     hidden inside a reset, takes result 0 (Sec. 3 says any noiseless sample is
//     a valid reference; Sec. 4 says the coin may be arbitrary).
//   - Frame update: the unsigned xz-linear map of the gate's tableau.
//   - Random bits: Philox4x64-10 (Salmon et al., SC'11) keyed by the seed, with
//     counters built from (flat instruction index, target slot, absolute 64-shot
//     word, purpose).  See philox_* and the noise / ZRAND helpers below.
//   - DEPOLARIZE1(p): X, Y, Z each with p/3.  DEPOLARIZE2(p): each of the 15
//     non-identity two-qubit Paulis with p/15.
//   - Classically controlled Paulis (Sec. 3, "Tracking Corrections"): CX, CY
//     and CZ take a measurement-record target rec[-k] in place of the control
//     (CZ on either side); the Pauli X, Y or Z is applied to the qubit when
//     that measurement's result is 1.  The reference run applies it when the
//     reference result is 1, the frame takes the rest: P^(result) =
//     P^(reference) P^(flip), so the frame is multiplied by P where the
//     measurement was flipped.

#include <cstdint>
#include <cstring>
#include <cstdio>
#include <cmath>
#include <string>
#include <vector>
#include <map>
#include <memory>
#include <random>
#include <stdexcept>
#include <algorithm>
#include <cctype>

typedef unsigned __int128 u128;

namespace {

thread_local std::string g_err;

// ---------------------------------------------------------------------------
// Gate table.  Each Clifford is written as its stabilizer tableau (Sec. 2.3):
// the signed Pauli product that the gate's unitary U maps each generator g to,
// U g U^dagger.  One-qubit gates list the images of X and Z; two-qubit gates
// list the images of X1, Z1, X2, Z2.  Terms are written one character per
// qubit ('_' = identity) after a sign character.  The test-suite checks every
// entry against the gate's unitary matrix.  SQRT_Y is the root fixed by the
// identity sqrt(Y) = H_YZ sqrt(Z) H_YZ of Sec. 5.7 (X -> -Z, Z -> +X); the
// tableau printed beside that identity (X -> +Z, Z -> -X) is SQRT_Y_DAG's.
// ---------------------------------------------------------------------------
enum Kind { K_CLIFFORD1, K_CLIFFORD2, K_RESET, K_MEASURE, K_MEASURE_RESET,
            K_NOISE1, K_NOISE2, K_DETECTOR, K_OBSERVABLE, K_ANNOTATION };
enum NoiseType { N_NONE, N_X, N_Y, N_Z, N_DEP1, N_DEP2 };

struct GateInfo {
  const char *name;
  Kind kind;
  NoiseType noise;
  const char *images[4];   // Clifford images (U g U^dagger)
  const char *inverse;     // name of the inverse gate (Cliffords only)
};

const GateInfo GATES[] = {
  {"I",          K_CLIFFORD1, N_NONE, {"+X", "+Z"}, "I"},
  {"X",          K_CLIFFORD1, N_NONE, {"+X", "-Z"}, "X"},
  {"Y",          K_CLIFFORD1, N_NONE, {"-X", "-Z"}, "Y"},
  {"Z",          K_CLIFFORD1, N_NONE, {"-X", "+Z"}, "Z"},
  {"H",          K_CLIFFORD1, N_NONE, {"+Z", "+X"}, "H"},
  {"H_XY",       K_CLIFFORD1, N_NONE, {"+Y", "-Z"}, "H_XY"},
  {"H_YZ",       K_CLIFFORD1, N_NONE, {"-X", "+Y"}, "H_YZ"},
  {"S",          K_CLIFFORD1, N_NONE, {"+Y", "+Z"}, "S_DAG"},
  {"S_DAG",      K_CLIFFORD1, N_NONE, {"-Y", "+Z"}, "S"},
  {"SQRT_X",     K_CLIFFORD1, N_NONE, {"+X", "-Y"}, "SQRT_X_DAG"},
  {"SQRT_X_DAG", K_CLIFFORD1, N_NONE, {"+X", "+Y"}, "SQRT_X"},
  {"SQRT_Y",     K_CLIFFORD1, N_NONE, {"-Z", "+X"}, "SQRT_Y_DAG"},
  {"SQRT_Y_DAG", K_CLIFFORD1, N_NONE, {"+Z", "-X"}, "SQRT_Y"},
  {"CX",         K_CLIFFORD2, N_NONE, {"+XX", "+Z_", "+_X", "+ZZ"}, "CX"},
  {"CY",         K_CLIFFORD2, N_NONE, {"+XY", "+Z_", "+ZX", "+ZZ"}, "CY"},
  {"CZ",         K_CLIFFORD2, N_NONE, {"+XZ", "+Z_", "+ZX", "+_Z"}, "CZ"},
  {"SWAP",       K_CLIFFORD2, N_NONE, {"+_X", "+_Z", "+X_", "+Z_"}, "SWAP"},
  {"R",          K_RESET,         N_NONE, {}, nullptr},
  {"M",          K_MEASURE,       N_NONE, {}, nullptr},
  {"MR",         K_MEASURE_RESET, N_NONE, {}, nullptr},
  {"X_ERROR",    K_NOISE1, N_X,    {}, nullptr},
  {"Y_ERROR",    K_NOISE1, N_Y,    {}, nullptr},
  {"Z_ERROR",    K_NOISE1, N_Z,    {}, nullptr},
  {"DEPOLARIZE1",K_NOISE1, N_DEP1, {}, nullptr},
  {"DEPOLARIZE2",K_NOISE2, N_DEP2, {}, nullptr},
  {"DETECTOR",   K_DETECTOR,   N_NONE, {}, nullptr},
  {"OBSERVABLE_INCLUDE", K_OBSERVABLE, N_NONE, {}, nullptr},
  {"TICK",       K_ANNOTATION, N_NONE, {}, nullptr},
  {"QUBIT_COORDS", K_ANNOTATION, N_NONE, {}, nullptr},
  {"SHIFT_COORDS", K_ANNOTATION, N_NONE, {}, nullptr},
};
const int NUM_GATES = sizeof(GATES) / sizeof(GATES[0]);

struct Alias { const char *alias, *name; };
const Alias ALIASES[] = {
  {"H_XZ", "H"}, {"SQRT_Z", "S"}, {"SQRT_Z_DAG", "S_DAG"}, {"CNOT", "CX"},
  {"ZCX", "CX"}, {"ZCY", "CY"}, {"ZCZ", "CZ"}, {"RZ", "R"}, {"MZ", "M"},
  {"MRZ", "MR"},
};

int find_gate(const std::string &upper) {
  std::string name = upper;
  for (const Alias &a : ALIASES) if (name == a.alias) name = a.name;
  for (int i = 0; i < NUM_GATES; i++) if (name == GATES[i].name) return i;
  return -1;
}

// ---------------------------------------------------------------------------
// Parsing (Sec. 5.10): one operation per line, '#' comments, blank lines,
// broadcasting over targets, REPEAT N { ... } blocks.  The parse result is the
// fully unrolled instruction list; an instruction's position in that list is
// its flat index, which keys its random bits.
// ---------------------------------------------------------------------------
struct Instr {
  int gate;
  double p = 0;                 // noise probability (noise channels)
  std::vector<uint32_t> q;      // qubit targets
  std::vector<uint64_t> rec;    // absolute measurement indices (DETECTOR/OBSERVABLE)
  // CX/CY/CZ: per target, the absolute index of a measurement-record target
  // (classical control), or NO_REC for a qubit.
  std::vector<uint64_t> ctl;
  uint64_t obs = 0;             // observable index
};

const uint64_t NO_REC = ~0ull;

struct Circuit {
  std::vector<Instr> ops;       // unrolled
  uint64_t num_qubits = 0, num_meas = 0, num_det = 0, num_obs = 0, num_gate_targets = 0;
  std::vector<std::vector<uint64_t>> detectors;   // absolute measurement indices
  std::vector<std::vector<uint64_t>> observables; // absolute measurement indices
};

struct ParseError { int line; std::string msg; };

struct Node {             // parse tree: either an instruction line or a REPEAT
  bool is_repeat = false;
  uint64_t reps = 0;
  std::vector<Node> body;
  int gate = -1, line = 0;
  std::vector<double> args;
  std::vector<std::string> targets;
};

std::string upper(std::string s) {
  for (char &c : s) c = (char)std::toupper((unsigned char)c);
  return s;
}

std::string trim(const std::string &s) {
  size_t a = 0, b = s.size();
  while (a < b && std::isspace((unsigned char)s[a])) a++;
  while (b > a && std::isspace((unsigned char)s[b - 1])) b--;
  return s.substr(a, b - a);
}

bool parse_u64(const std::string &s, uint64_t &v) {
  if (s.empty() || s.size() > 19) return false;
  v = 0;
  for (char c : s) { if (c < '0' || c > '9') return false; v = v * 10 + (uint64_t)(c - '0'); }
  return true;
}

void parse_lines(const std::vector<std::string> &lines, size_t &i, std::vector<Node> &out, bool in_block) {
  while (i < lines.size()) {
    int lineno = (int)i + 1;
    std::string s = lines[i];
    size_t hash = s.find('#');
    if (hash != std::string::npos) s = s.substr(0, hash);
    s = trim(s);
    i++;
    if (s.empty()) continue;
    if (s == "}") {
      if (!in_block) throw ParseError{lineno, "unmatched '}'"};
      return;
    }
    // Split off name and optional (args).
    size_t k = 0;
    while (k < s.size() && !std::isspace((unsigned char)s[k]) && s[k] != '(') k++;
    std::string name = upper(s.substr(0, k));
    std::string rest = s.substr(k);
    std::vector<double> args;
    rest = trim(rest);
    if (!rest.empty() && rest[0] == '(') {
      size_t close = rest.find(')');
      if (close == std::string::npos) throw ParseError{lineno, "missing ')'"};
      std::string inner = rest.substr(1, close - 1);
      rest = trim(rest.substr(close + 1));
      size_t start = 0;
      while (start <= inner.size()) {
        size_t comma = inner.find(',', start);
        if (comma == std::string::npos) comma = inner.size();
        std::string tok = trim(inner.substr(start, comma - start));
        if (tok.empty()) throw ParseError{lineno, "empty argument"};
        char *end = nullptr;
        double v = std::strtod(tok.c_str(), &end);
        if (end == tok.c_str() || *end != '\0') throw ParseError{lineno, "bad argument '" + tok + "'"};
        args.push_back(v);
        start = comma + 1;
      }
    }
    if (name == "REPEAT") {
      // REPEAT N {
      std::string t = rest;
      if (t.empty() || t.back() != '{') throw ParseError{lineno, "REPEAT needs '{' on its line"};
      t = trim(t.substr(0, t.size() - 1));
      Node n;
      n.is_repeat = true;
      n.line = lineno;
      if (!parse_u64(t, n.reps) || n.reps == 0) throw ParseError{lineno, "bad REPEAT count"};
      parse_lines(lines, i, n.body, true);
      if (i > lines.size()) throw ParseError{lineno, "unterminated REPEAT"};
      out.push_back(std::move(n));
      continue;
    }
    Node n;
    n.line = lineno;
    n.gate = find_gate(name);
    if (n.gate < 0) throw ParseError{lineno, "unknown gate '" + name + "'"};
    n.args = args;
    size_t a = 0;
    while (a < rest.size()) {
      while (a < rest.size() && std::isspace((unsigned char)rest[a])) a++;
      size_t b = a;
      while (b < rest.size() && !std::isspace((unsigned char)rest[b])) b++;
      if (b > a) n.targets.push_back(rest.substr(a, b - a));
      a = b;
    }
    out.push_back(std::move(n));
  }
  if (in_block) throw ParseError{(int)lines.size(), "unterminated REPEAT block"};
}

bool is_rec(const std::string &t) {
  std::string u = upper(t);
  return u.size() >= 7 && u.compare(0, 5, "REC[-") == 0 && u.back() == ']';
}

// Absolute measurement index of a rec[-k] target, k measurements back.
uint64_t rec_index(const std::string &t, uint64_t num_meas, int line) {
  std::string u = upper(t);
  uint64_t k;
  if (!parse_u64(u.substr(5, u.size() - 6), k) || k == 0) throw ParseError{line, "bad lookback"};
  if (k > num_meas) throw ParseError{line, "lookback reaches before the first measurement"};
  return num_meas - k;
}

// A classically controlled pair of a CX/CY/CZ instruction: the qubit it acts
// on, the controlling measurement and the Pauli (bit 0: X part, bit 1: Z
// part).  Returns false for an ordinary two-qubit pair.
bool controlled_pair(const Instr &ins, size_t k, uint32_t &q, uint64_t &m, int &pauli) {
  if (ins.ctl.empty()) return false;
  const bool ra = ins.ctl[k] != NO_REC, rb = ins.ctl[k + 1] != NO_REC;
  if (!ra && !rb) return false;
  q = ra ? ins.q[k + 1] : ins.q[k];
  m = ra ? ins.ctl[k] : ins.ctl[k + 1];
  const std::string name = GATES[ins.gate].name;
  pauli = name == "CX" ? 1 : name == "CZ" ? 2 : 3;
  return true;
}

const char *pauli_gate_name(int pauli) { return pauli == 1 ? "X" : pauli == 2 ? "Z" : "Y"; }

// Walks the tree and appends unrolled instructions.
void unroll(const std::vector<Node> &nodes, Circuit &c) {
  for (const Node &n : nodes) {
    if (n.is_repeat) {
      for (uint64_t r = 0; r < n.reps; r++) unroll(n.body, c);
      continue;
    }
    const GateInfo &g = GATES[n.gate];
    Instr ins;
    ins.gate = n.gate;
    bool is_noise = g.kind == K_NOISE1 || g.kind == K_NOISE2;
    if (is_noise) {
      if (n.args.size() != 1) throw ParseError{n.line, "noise channel needs one probability"};
      double p = n.args[0];
      if (!(p >= 0.0 && p <= 1.0)) throw ParseError{n.line, "probability outside [0, 1]"};
      ins.p = p;
    } else if (g.kind == K_OBSERVABLE) {
      if (n.args.size() != 1 || n.args[0] < 0 || n.args[0] != std::floor(n.args[0]))
        throw ParseError{n.line, "OBSERVABLE_INCLUDE needs one non-negative integer index"};
      ins.obs = (uint64_t)n.args[0];
    } else if (g.kind != K_DETECTOR && g.kind != K_ANNOTATION && !n.args.empty()) {
      throw ParseError{n.line, "gate takes no arguments"};
    }
    if (g.kind == K_DETECTOR || g.kind == K_OBSERVABLE) {
      for (const std::string &t : n.targets) {
        if (!is_rec(t)) throw ParseError{n.line, "expected rec[-k] target, got '" + t + "'"};
        ins.rec.push_back(rec_index(t, c.num_meas, n.line));
      }
      if (g.kind == K_DETECTOR) {
        c.detectors.push_back(ins.rec);
        c.num_det++;
      } else {
        if (ins.obs >= c.observables.size()) c.observables.resize(ins.obs + 1);
        for (uint64_t m : ins.rec) c.observables[ins.obs].push_back(m);
      }
    } else if (g.kind != K_ANNOTATION) {
      const std::string gname = g.name;
      const bool controllable = gname == "CX" || gname == "CY" || gname == "CZ";
      for (size_t k = 0; k < n.targets.size(); k++) {
        const std::string &t = n.targets[k];
        if (controllable && is_rec(t)) {
          // The record may replace the control (CZ: either qubit), not both.
          if (k % 2 == 1 && gname != "CZ") throw ParseError{n.line, "a record target must be the control"};
          ins.q.push_back(0);
          ins.ctl.push_back(rec_index(t, c.num_meas, n.line));
          continue;
        }
        uint64_t v;
        if (!parse_u64(t, v) || v >= (1ull << 31)) throw ParseError{n.line, "bad qubit target '" + t + "'"};
        ins.q.push_back((uint32_t)v);
        ins.ctl.push_back(NO_REC);
        if (v + 1 > c.num_qubits) c.num_qubits = v + 1;
      }
      if ((g.kind == K_CLIFFORD2 || g.kind == K_NOISE2) && ins.q.size() % 2 != 0)
        throw ParseError{n.line, "two-qubit operation needs an even number of targets"};
      if (g.kind == K_CLIFFORD2 || g.kind == K_NOISE2)
        for (size_t k = 0; k < ins.q.size(); k += 2) {
          const bool ra = ins.ctl[k] != NO_REC, rb = ins.ctl[k + 1] != NO_REC;
          if (ra && rb) throw ParseError{n.line, "both targets are measurement records"};
          if (!ra && !rb && ins.q[k] == ins.q[k + 1]) throw ParseError{n.line, "two-qubit operation on one qubit"};
        }
      if (g.kind == K_MEASURE || g.kind == K_MEASURE_RESET) c.num_meas += ins.q.size();
      if (g.kind == K_CLIFFORD1 || g.kind == K_RESET || g.kind == K_MEASURE || g.kind == K_MEASURE_RESET)
        c.num_gate_targets += ins.q.size();
      if (g.kind == K_CLIFFORD2) c.num_gate_targets += ins.q.size() / 2;
    }
    c.ops.push_back(std::move(ins));
  }
}

// ---------------------------------------------------------------------------
// Pauli strings with phase tracking.  A Hermitian Pauli product is stored as
// sign + xz bits (Sec. 2.1).  For multiplication it is rewritten in the
// "XZ form" i^r * prod_q X_q^x_q Z_q^z_q, where Y = i X Z; then
// (i^a X^x1 Z^z1)(i^b X^x2 Z^z2) = i^(a+b+2 z1.x2) X^(x1^x2) Z^(z1^z2).
// ---------------------------------------------------------------------------
struct Pauli {                  // Hermitian: (-1)^sign * prod P_q
  std::vector<uint64_t> x, z;
  int sign = 0;
  explicit Pauli(size_t n = 0) : x((n + 63) / 64, 0), z((n + 63) / 64, 0) {}
  int getx(size_t q) const { return (int)((x[q >> 6] >> (q & 63)) & 1); }
  int getz(size_t q) const { return (int)((z[q >> 6] >> (q & 63)) & 1); }
  void setx(size_t q, int v) { x[q >> 6] = (x[q >> 6] & ~(1ull << (q & 63))) | ((uint64_t)v << (q & 63)); }
  void setz(size_t q, int v) { z[q >> 6] = (z[q >> 6] & ~(1ull << (q & 63))) | ((uint64_t)v << (q & 63)); }
};

struct PhasedPauli {            // i^r * prod X^x Z^z
  std::vector<uint64_t> x, z;
  int r = 0;
};

int popcount_and(const std::vector<uint64_t> &a, const std::vector<uint64_t> &b) {
  int s = 0;
  for (size_t k = 0; k < a.size(); k++) s += __builtin_popcountll(a[k] & b[k]);
  return s;
}

PhasedPauli to_phased(const Pauli &p) {
  PhasedPauli o;
  o.x = p.x; o.z = p.z;
  o.r = (2 * p.sign + popcount_and(p.x, p.z)) & 3;   // each Y contributes a factor i
  return o;
}

Pauli to_hermitian(const PhasedPauli &p) {
  Pauli o;
  o.x = p.x; o.z = p.z;
  int r = (p.r - popcount_and(p.x, p.z)) & 3;
  if (r & 1) throw std::runtime_error("non-Hermitian Pauli product");
  o.sign = r >> 1;
  return o;
}

void mul_into(PhasedPauli &acc, const PhasedPauli &b) {   // acc = acc * b
  acc.r = (acc.r + b.r + 2 * popcount_and(acc.z, b.x)) & 3;
  for (size_t k = 0; k < acc.x.size(); k++) { acc.x[k] ^= b.x[k]; acc.z[k] ^= b.z[k]; }
}

// A small signed Pauli written as text, e.g. "-XZ" over the gate's qubits.
struct SmallPauli { int sign; std::vector<int> x, z; };

SmallPauli parse_small(const char *s) {
  SmallPauli p;
  p.sign = s[0] == '-';
  for (const char *c = s + 1; *c; c++) {
    p.x.push_back(*c == 'X' || *c == 'Y');
    p.z.push_back(*c == 'Z' || *c == 'Y');
  }
  return p;
}

// ---------------------------------------------------------------------------
// Stabilizer tableau (Sec. 2.3) over n qubits, stored by columns: xs[q] is the
// image of X_q, zs[q] the image of Z_q.  In the simulation of Sec. 4 the
// tableau T maps an observable at the current time to the equivalent
// observable at the start of time.
// ---------------------------------------------------------------------------
struct Tableau {
  size_t n;
  std::vector<Pauli> xs, zs;
  explicit Tableau(size_t n_) : n(n_) {
    for (size_t q = 0; q < n; q++) {
      Pauli a(n), b(n);
      a.setx(q, 1); b.setz(q, 1);
      xs.push_back(a); zs.push_back(b);
    }
  }

  // T(P) for a Pauli P supported on `qs` (Sec. 2.3.1): decompose P into
  // generators (X before Z on each qubit, Y = i X Z), look each one up, and
  // multiply the images together while tracking the phase.
  Pauli image_of(const SmallPauli &p, const std::vector<uint32_t> &qs) const {
    PhasedPauli acc;
    acc.x.assign((n + 63) / 64, 0);
    acc.z.assign((n + 63) / 64, 0);
    int ys = 0;
    for (size_t k = 0; k < qs.size(); k++) ys += p.x[k] & p.z[k];
    acc.r = (2 * p.sign + ys) & 3;
    for (size_t k = 0; k < qs.size(); k++) {
      if (p.x[k]) mul_into(acc, to_phased(xs[qs[k]]));
      if (p.z[k]) mul_into(acc, to_phased(zs[qs[k]]));
    }
    return to_hermitian(acc);
  }

  // Folding a Clifford gate G into T: T'(g) = T(G^dagger g G) for every
  // generator g on G's qubits, i.e. prepend the tableau of G's inverse
  // (Sec. 2.3.2 and Sec. 4).
  void prepend(int gate, const std::vector<uint32_t> &qs) {
    const GateInfo &inv = GATES[find_gate(GATES[gate].inverse)];
    size_t k = qs.size();
    std::vector<Pauli> nx, nz;
    for (size_t j = 0; j < k; j++) {
      nx.push_back(image_of(parse_small(inv.images[2 * j]), qs));
      nz.push_back(image_of(parse_small(inv.images[2 * j + 1]), qs));
    }
    for (size_t j = 0; j < k; j++) { xs[qs[j]] = nx[j]; zs[qs[j]] = nz[j]; }
  }

  // Inserting a self-inverse Clifford B at the start of time (an "append",
  // Sec. 2.3.2): every column P becomes B P B, computed by conjugating the
  // column's terms on B's qubits with B's tableau.
  void append(int gate, const std::vector<uint32_t> &qs) {
    const GateInfo &g = GATES[gate];
    size_t k = qs.size();
    std::vector<SmallPauli> img;
    for (size_t j = 0; j < 2 * k; j++) img.push_back(parse_small(g.images[j]));
    for (int which = 0; which < 2; which++) {
      for (size_t c = 0; c < n; c++) {
        Pauli &col = which ? zs[c] : xs[c];
        // Local part in XZ form: i^ys prod X^x Z^z over B's qubits.
        int r = 0;
        std::vector<int> lx(k), lz(k);
        bool any = false;
        for (size_t j = 0; j < k; j++) {
          lx[j] = col.getx(qs[j]); lz[j] = col.getz(qs[j]);
          r += lx[j] & lz[j];
          any |= lx[j] | lz[j];
        }
        if (!any) continue;
        // Image of the local part: product of the generator images.
        int ar = r & 3;
        std::vector<int> ax(k, 0), az(k, 0);
        for (size_t j = 0; j < k; j++) {
          for (int gz = 0; gz < 2; gz++) {
            if (!(gz ? lz[j] : lx[j])) continue;
            const SmallPauli &m = img[2 * j + gz];
            int mr = 2 * m.sign;
            for (size_t t = 0; t < k; t++) mr += m.x[t] & m.z[t];
            int cross = 0;
            for (size_t t = 0; t < k; t++) cross += az[t] & m.x[t];
            ar = (ar + mr + 2 * cross) & 3;
            for (size_t t = 0; t < k; t++) { ax[t] ^= m.x[t]; az[t] ^= m.z[t]; }
          }
        }
        int ys = 0;
        for (size_t t = 0; t < k; t++) ys += ax[t] & az[t];
        int rr = (ar - ys) & 3;
        if (rr & 1) throw std::runtime_error("non-Hermitian conjugation result");
        col.sign ^= rr >> 1;
        for (size_t t = 0; t < k; t++) { col.setx(qs[t], ax[t]); col.setz(qs[t], az[t]); }
      }
    }
  }

  // Measurement of Z_q (Sec. 4).  If the Z_q column has X or Y terms the
  // result is random: pick the lowest such qubit as pivot, append CNOTs from
  // the pivot to the other X/Y terms, append H (X term) or H_YZ (Y term) on the
  // pivot so that its term becomes Z, then append X on the pivot if that makes
  // the result equal to `coin`.  The result is the sign of the Z_q column.
  int measure(uint32_t q, int coin) {
    Pauli &col = zs[q];
    std::vector<uint32_t> xy;
    for (size_t j = 0; j < n; j++) if (col.getx(j)) xy.push_back((uint32_t)j);
    if (xy.empty()) return col.sign;
    uint32_t pivot = xy[0];
    int cx = find_gate("CX");
    for (size_t j = 1; j < xy.size(); j++) append(cx, {pivot, xy[j]});
    append(find_gate(zs[q].getz(pivot) ? "H_YZ" : "H"), {pivot});
    for (size_t j = 0; j < n; j++)
      if (zs[q].getx(j)) throw std::runtime_error("collapse left an X term");
    if (zs[q].sign != coin) append(find_gate("X"), {pivot});
    return zs[q].sign;
  }
};

// ---------------------------------------------------------------------------
// Random bits.  Philox4x64-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds
// of two 64x64->128 multiplies by fixed constants, a cross-wise xor with the
// round key, and a Weyl increment of the key.
// ---------------------------------------------------------------------------
const uint64_t PHILOX_M0 = 0xD2E7470EE14C6C93ull, PHILOX_M1 = 0xCA5A826395121157ull;
const uint64_t PHILOX_W0 = 0x9E3779B97F4A7C15ull, PHILOX_W1 = 0xBB67AE8584CAA73Bull;
const uint64_t KEY_HI = 0x5354494D5F465241ull;   // second key word: fixed spec constant
const uint64_t PURPOSE_ZRAND = 1, PURPOSE_NOISE_PREFIX = 2, PURPOSE_NOISE_DETAIL = 3;
const uint64_t INIT_INSTRUCTION = ~0ull;

void philox(const uint64_t in[4], uint64_t k0, uint64_t k1, uint64_t out[4]) {
  uint64_t c0 = in[0], c1 = in[1], c2 = in[2], c3 = in[3];
  for (int round = 0; round < 10; round++) {
    u128 p0 = (u128)PHILOX_M0 * c0;
    u128 p1 = (u128)PHILOX_M1 * c2;
    uint64_t hi0 = (uint64_t)(p0 >> 64), lo0 = (uint64_t)p0;
    uint64_t hi1 = (uint64_t)(p1 >> 64), lo1 = (uint64_t)p1;
    c0 = hi1 ^ c1 ^ k0;
    c1 = lo1;
    c2 = hi0 ^ c3 ^ k1;
    c3 = lo0;
    k0 += PHILOX_W0;
    k1 += PHILOX_W1;
  }
  out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

void philox_call(uint64_t seed, uint64_t c0, uint64_t c1, uint64_t c2, uint64_t c3, uint64_t out[4]) {
  uint64_t in[4] = {c0, c1, c2, c3};
  philox(in, seed, KEY_HI, out);
}

// Post-collapse Z randomisation (Sec. 3: Z_ERROR(0.5) after every
// initialisation, reset and measurement): 64 fair bits for one 64-shot word.
// Four consecutive target slots share one Philox call.
uint64_t zrand(uint64_t seed, uint64_t instr, uint64_t slot, uint64_t word) {
  uint64_t o[4];
  philox_call(seed, instr, slot >> 2, word, PURPOSE_ZRAND << 32, o);
  return o[slot & 3];
}

// Thresholds for geometric gap sampling (Sec. 5.5), an exact integer recurrence
// from the bits of p: a = floor((1 - p) 2^64), t[1] = a,
// t[g+1] = floor(t[g] a / 2^64).  u < t[g] for a uniform 64-bit u happens with
// probability t[g] / 2^64 ~ (1-p)^g, i.e. "no error in the next g shots".
void thresholds(double p, uint64_t t[64]) {
  // ceil(p * 2^64) from the exact binary value of p.
  int e;
  double m = std::frexp(p, &e);                 // p = m * 2^e, m in [0.5, 1)
  uint64_t mant = (uint64_t)std::ldexp(m, 53);  // p = mant * 2^(e - 53)
  int shift = e - 53 + 64;                      // p * 2^64 = mant * 2^shift
  u128 ceil_p;
  if (p == 0) ceil_p = 0;
  else if (shift >= 0) ceil_p = (u128)mant << shift;
  else if (shift > -64) ceil_p = ((u128)mant + (((u128)1 << -shift) - 1)) >> -shift;
  else ceil_p = 1;
  u128 a = ((u128)1 << 64) - ceil_p;            // floor((1 - p) * 2^64)
  if (a > ~0ull) a = ~0ull;                     // only for p == 0, never used
  uint64_t av = (uint64_t)a;
  u128 cur = av;
  for (int g = 0; g < 64; g++) {
    t[g] = (uint64_t)cur;
    cur = (cur * av) >> 64;
  }
}

// The sequence of 64-bit draws used by noise on (instruction, slot, word).
// Draw 0 takes its top 8 bits from a call shared by 32 consecutive slots
// (byte slot % 32 of its 256 output bits, lane-major, least significant byte
// first) and its low 56 bits from lane 0 of the slot's own call; draws 1, 2,
// ... are the following lanes of the slot's own calls.
struct NoiseDraws {
  uint64_t seed, instr, slot, word;
  uint64_t buf[4];
  uint64_t next_index = 0;
  uint64_t next() {
    uint64_t j = next_index++;
    if ((j & 3) == 0) philox_call(seed, instr, slot, word, (PURPOSE_NOISE_DETAIL << 32) | (j >> 2), buf);
    uint64_t d = buf[j & 3];
    if (j == 0) {
      uint64_t pre[4];
      philox_call(seed, instr, slot >> 5, word, PURPOSE_NOISE_PREFIX << 32, pre);
      uint64_t k = slot & 31;
      uint64_t v = (pre[k >> 3] >> (8 * (k & 7))) & 0xFF;
      d = (v << 56) | (d & ((1ull << 56) - 1));
    }
    return d;
  }
};

// Error positions within one 64-shot word by geometric gaps (Sec. 5.5).  For
// each hit, `choices` receives floor(u K / 2^64) from the next draw when the
// channel picks among K Paulis (K = 0: no choice).
void sample_hits(uint64_t seed, uint64_t instr, uint64_t slot, uint64_t word, const uint64_t t[64],
                 int K, std::vector<std::pair<int, int>> &hits) {
  hits.clear();
  NoiseDraws d{seed, instr, slot, word, {0, 0, 0, 0}, 0};
  int pos = 0;
  while (true) {
    uint64_t u = d.next();
    int G = 0;
    for (int g = 1; g <= 64; g++) if (u < t[g - 1]) G++;
    pos += G;
    if (pos >= 64) break;
    int choice = 0;
    if (K) choice = (int)(((u128)d.next() * (u128)K) >> 64);
    hits.push_back({pos, choice});
    pos += 1;
    if (pos >= 64) break;
  }
}

// ---------------------------------------------------------------------------
// Reference sample via the inverse tableau (Sec. 4).  coin_mode 0: canonical
// (every random result is 0); otherwise random results come from an mt19937_64
// seeded with coin_seed (used to check that detectors are deterministic).
// ---------------------------------------------------------------------------
std::vector<uint8_t> reference(const Circuit &c, bool canonical, uint64_t coin_seed) {
  Tableau t(c.num_qubits);
  std::mt19937_64 rng(coin_seed);
  std::vector<uint8_t> ref;
  ref.reserve(c.num_meas);
  for (const Instr &ins : c.ops) {
    const GateInfo &g = GATES[ins.gate];
    switch (g.kind) {
      case K_CLIFFORD1:
        for (uint32_t q : ins.q) t.prepend(ins.gate, {q});
        break;
      case K_CLIFFORD2:
        for (size_t k = 0; k < ins.q.size(); k += 2) {
          uint32_t q;
          uint64_t m;
          int pauli;
          if (controlled_pair(ins, k, q, m, pauli)) {
            if (ref[m]) t.prepend(find_gate(pauli_gate_name(pauli)), {q});   // the reference's own result
          } else {
            t.prepend(ins.gate, {ins.q[k], ins.q[k + 1]});
          }
        }
        break;
      case K_MEASURE:
      case K_MEASURE_RESET:
      case K_RESET:
        for (uint32_t q : ins.q) {
          int coin = canonical ? 0 : (int)(rng() & 1);
          int r = t.measure(q, coin);
          if (g.kind != K_RESET) ref.push_back((uint8_t)r);
          if (g.kind != K_MEASURE) t.zs[q].sign = 0;   // force |0>
        }
        break;
      default:
        break;   // noise is disabled for the reference; annotations do nothing
    }
  }
  return ref;
}

// ---------------------------------------------------------------------------
// Pauli frame simulation (Sec. 3) of the 64 shots of one word.  Frame bit
// layout follows Sec. 5.1: for each qubit an x word and a z word, one bit per
// shot.
// ---------------------------------------------------------------------------
struct FrameRule {              // unsigned xz-linear map of a Clifford tableau
  int k;                        // number of qubits
  // new bit (qubit t, x/z) = XOR over old generator bits whose image has it.
  int img[4][4];                // img[generator][out bit], generator/out index = 2*qubit + (0:x,1:z)
};

FrameRule frame_rule(int gate) {
  const GateInfo &g = GATES[gate];
  FrameRule r{};
  r.k = g.kind == K_CLIFFORD2 ? 2 : 1;
  for (int gen = 0; gen < 2 * r.k; gen++) {
    SmallPauli p = parse_small(g.images[gen]);
    for (int t = 0; t < r.k; t++) {
      r.img[gen][2 * t] = p.x[t];
      r.img[gen][2 * t + 1] = p.z[t];
    }
  }
  return r;
}

void simulate_word(const Circuit &c, const std::vector<uint8_t> &ref, const std::vector<FrameRule> &rules,
                   const std::vector<std::vector<uint64_t>> &thr, uint64_t seed, uint64_t word,
                   uint64_t tail_mask, std::vector<uint64_t> &flips) {
  size_t n = c.num_qubits;
  std::vector<uint64_t> x(n, 0), z(n, 0);
  // Step 2: random I or Z on every qubit (initialisation is a collapse).
  for (size_t q = 0; q < n; q++) z[q] = zrand(seed, INIT_INSTRUCTION, q, word);
  flips.assign(c.num_meas, 0);
  uint64_t m = 0;
  std::vector<std::pair<int, int>> hits;
  for (uint64_t i = 0; i < c.ops.size(); i++) {
    const Instr &ins = c.ops[i];
    const GateInfo &g = GATES[ins.gate];
    switch (g.kind) {
      case K_CLIFFORD1:
      case K_CLIFFORD2: {
        const FrameRule &r = rules[ins.gate];
        for (size_t s = 0; s < ins.q.size(); s += r.k) {
          uint32_t fq;
          uint64_t fm;
          int pauli;
          if (r.k == 2 && controlled_pair(ins, s, fq, fm, pauli)) {
            // Shots whose controlling result differs from the reference's get
            // the Pauli in their frame.
            if (pauli & 1) x[fq] ^= flips[fm];
            if (pauli & 2) z[fq] ^= flips[fm];
            continue;
          }
          uint64_t in[4] = {0, 0, 0, 0}, out[4] = {0, 0, 0, 0};
          for (int t = 0; t < r.k; t++) { in[2 * t] = x[ins.q[s + t]]; in[2 * t + 1] = z[ins.q[s + t]]; }
          for (int gen = 0; gen < 2 * r.k; gen++)
            for (int o = 0; o < 2 * r.k; o++)
              if (r.img[gen][o]) out[o] ^= in[gen];
          for (int t = 0; t < r.k; t++) { x[ins.q[s + t]] = out[2 * t]; z[ins.q[s + t]] = out[2 * t + 1]; }
        }
        break;
      }
      case K_RESET:
        for (size_t s = 0; s < ins.q.size(); s++) {
          uint32_t q = ins.q[s];
          x[q] = 0;
          z[q] = zrand(seed, i, s, word);
        }
        break;
      case K_MEASURE:
      case K_MEASURE_RESET:
        for (size_t s = 0; s < ins.q.size(); s++) {
          uint32_t q = ins.q[s];
          flips[m++] = x[q] & tail_mask;            // reported result is ref XOR x
          if (g.kind == K_MEASURE) {
            z[q] ^= zrand(seed, i, s, word);
          } else {
            x[q] = 0;
            z[q] = zrand(seed, i, s, word);
          }
        }
        break;
      case K_NOISE1: {
        if (ins.p == 0) break;
        const uint64_t *t = thr[i].data();
        for (size_t s = 0; s < ins.q.size(); s++) {
          uint32_t q = ins.q[s];
          sample_hits(seed, i, s, word, t, g.noise == N_DEP1 ? 3 : 0, hits);
          for (auto &h : hits) {
            uint64_t bit = 1ull << h.first;
            int px = 0, pz = 0;
            switch (g.noise) {
              case N_X: px = 1; break;
              case N_Y: px = 1; pz = 1; break;
              case N_Z: pz = 1; break;
              case N_DEP1: px = h.second <= 1; pz = h.second >= 1; break;   // 0:X 1:Y 2:Z
              default: break;
            }
            if (px) x[q] ^= bit;
            if (pz) z[q] ^= bit;
          }
        }
        break;
      }
      case K_NOISE2: {
        if (ins.p == 0) break;
        const uint64_t *t = thr[i].data();
        for (size_t s = 0; s < ins.q.size() / 2; s++) {
          uint32_t a = ins.q[2 * s], b = ins.q[2 * s + 1];
          sample_hits(seed, i, s, word, t, 15, hits);
          for (auto &h : hits) {
            uint64_t bit = 1ull << h.first;
            int v = h.second + 1;                    // non-identity two-qubit Pauli
            if (v & 1) x[a] ^= bit;
            if (v & 2) z[a] ^= bit;
            if (v & 4) x[b] ^= bit;
            if (v & 8) z[b] ^= bit;
          }
        }
        break;
      }
      default:
        break;
    }
  }
  (void)ref;
}

// ---------------------------------------------------------------------------
// Sparse detection-event sampling (Sec. 5.6): sample the error events, then
// XOR together the sets of detectors (and observables) each one flips.  A
// set is found by its plain definition: insert the single Pauli into an
// otherwise noiseless frame whose Z randomisations are all zero, run the rest
// of the circuit and see which detectors change.  Errors come from the same
// draws as in the frame simulation, so on circuits whose detectors and
// observables are deterministic both methods give the same events.
// Lanes number the outputs: detector d is lane d, observable o is lane
// num_det + o.
// ---------------------------------------------------------------------------
struct ErrorSets {
  // Generators in order: noise instruction (p > 0, circuit order), slot, then
  // X and Z of the slot's first qubit and (two-qubit channels) of its second.
  std::vector<uint64_t> off{0};   // generator g: lanes[off[g], off[g + 1])
  std::vector<uint32_t> lanes;
  std::vector<uint64_t> first;    // per instruction: its first generator
};

// Lanes flipped by X (xz = 0) or Z (xz = 1) on qubit q right after
// instruction `at`.
void inject(const Circuit &c, const std::vector<FrameRule> &rules, size_t at, uint64_t meas_done, uint32_t q,
            int xz, std::vector<uint32_t> &out) {
  std::vector<uint8_t> x(c.num_qubits, 0), z(c.num_qubits, 0), flips(c.num_meas, 0);
  (xz ? z : x)[q] = 1;
  uint64_t m = meas_done;
  for (size_t i = at + 1; i < c.ops.size(); i++) {
    const Instr &ins = c.ops[i];
    const GateInfo &g = GATES[ins.gate];
    if (g.kind == K_CLIFFORD1 || g.kind == K_CLIFFORD2) {
      const FrameRule &r = rules[ins.gate];
      for (size_t s = 0; s < ins.q.size(); s += r.k) {
        uint32_t fq;
        uint64_t fm;
        int pauli;
        if (r.k == 2 && controlled_pair(ins, s, fq, fm, pauli)) {
          if (pauli & 1) x[fq] ^= flips[fm];
          if (pauli & 2) z[fq] ^= flips[fm];
          continue;
        }
        uint8_t in[4] = {0, 0, 0, 0}, o[4] = {0, 0, 0, 0};
        for (int t = 0; t < r.k; t++) { in[2 * t] = x[ins.q[s + t]]; in[2 * t + 1] = z[ins.q[s + t]]; }
        for (int gen = 0; gen < 2 * r.k; gen++)
          for (int k = 0; k < 2 * r.k; k++)
            if (r.img[gen][k]) o[k] ^= in[gen];
        for (int t = 0; t < r.k; t++) { x[ins.q[s + t]] = o[2 * t]; z[ins.q[s + t]] = o[2 * t + 1]; }
      }
    } else if (g.kind == K_RESET || g.kind == K_MEASURE || g.kind == K_MEASURE_RESET) {
      for (uint32_t t : ins.q) {
        if (g.kind != K_RESET) flips[m++] = x[t];
        if (g.kind != K_MEASURE) { x[t] = 0; z[t] = 0; }
      }
    }
  }
  out.clear();
  for (uint64_t d = 0; d < c.num_det; d++) {
    uint8_t v = 0;
    for (uint64_t mi : c.detectors[d]) v ^= flips[mi];
    if (v) out.push_back((uint32_t)d);
  }
  for (uint64_t o = 0; o < c.num_obs; o++) {
    uint8_t v = 0;
    for (uint64_t mi : c.observables[o]) v ^= flips[mi];
    if (v) out.push_back((uint32_t)(c.num_det + o));
  }
}

std::vector<FrameRule> all_frame_rules() {
  std::vector<FrameRule> rules(NUM_GATES);
  for (int g = 0; g < NUM_GATES; g++)
    if (GATES[g].kind == K_CLIFFORD1 || GATES[g].kind == K_CLIFFORD2) rules[g] = frame_rule(g);
  return rules;
}

ErrorSets error_sets(const Circuit &c) {
  ErrorSets e;
  std::vector<FrameRule> rules = all_frame_rules();
  std::vector<uint32_t> lanes;
  uint64_t meas = 0;
  e.first.assign(c.ops.size(), ~0ull);
  for (size_t i = 0; i < c.ops.size(); i++) {
    const Instr &ins = c.ops[i];
    const GateInfo &g = GATES[ins.gate];
    if ((g.kind == K_NOISE1 || g.kind == K_NOISE2) && ins.p > 0) {
      e.first[i] = e.off.size() - 1;
      for (uint32_t q : ins.q)
        for (int xz = 0; xz < 2; xz++) {
          inject(c, rules, i, meas, q, xz, lanes);
          e.lanes.insert(e.lanes.end(), lanes.begin(), lanes.end());
          e.off.push_back(e.lanes.size());
        }
    }
    if (g.kind == K_MEASURE || g.kind == K_MEASURE_RESET) meas += ins.q.size();
  }
  return e;
}

// True when no detector or observable depends on the random outcomes of the
// noiseless circuit: with noise switched off, a frame run with random Z
// randomisations must leave every detector and observable at zero (a
// dependence escapes with probability 2^-64 per word; two words are run).
bool deterministic(const Circuit &c) {
  Circuit quiet = c;
  for (Instr &ins : quiet.ops) ins.p = 0;
  std::vector<FrameRule> rules = all_frame_rules();
  std::vector<std::vector<uint64_t>> thr(quiet.ops.size());
  std::vector<uint8_t> ref;
  std::vector<uint64_t> flips;
  for (uint64_t word = 0; word < 2; word++) {
    simulate_word(quiet, ref, rules, thr, 0x5eed + word, word, ~0ull, flips);
    for (const auto &d : c.detectors) {
      uint64_t v = 0;
      for (uint64_t mi : d) v ^= flips[mi];
      if (v) return false;
    }
    for (const auto &o : c.observables) {
      uint64_t v = 0;
      for (uint64_t mi : o) v ^= flips[mi];
      if (v) return false;
    }
  }
  return true;
}

struct Handle {
  Circuit c;
  std::unique_ptr<ErrorSets> sets;
  const ErrorSets &error_sets_cached() {
    if (!sets) sets = std::make_unique<ErrorSets>(error_sets(c));
    return *sets;
  }
};

}  // namespace

// ---------------------------------------------------------------------------
// C ABI used by the Python wrapper (oracle/__init__.py).
// ---------------------------------------------------------------------------
extern "C" {

const char *oracle_last_error() { return g_err.c_str(); }

int oracle_parse(const char *text, size_t len, void **out) {
  try {
    std::string s(text, len);
    std::vector<std::string> lines;
    size_t a = 0;
    while (a <= s.size()) {
      size_t b = s.find('\n', a);
      if (b == std::string::npos) b = s.size();
      lines.push_back(s.substr(a, b - a));
      a = b + 1;
    }
    std::vector<Node> tree;
    size_t i = 0;
    parse_lines(lines, i, tree, false);
    auto h = std::make_unique<Handle>();
    unroll(tree, h->c);
    h->c.num_obs = h->c.observables.size();
    *out = h.release();
    return 0;
  } catch (const ParseError &e) {
    g_err = "line " + std::to_string(e.line) + ": " + e.msg;
    return -1;
  } catch (const std::exception &e) {
    g_err = e.what();
    return -1;
  }
}

void oracle_free(void *h) { delete (Handle *)h; }

void oracle_shape(void *hv, uint64_t out[6]) {
  const Circuit &c = ((Handle *)hv)->c;
  out[0] = c.num_qubits; out[1] = c.num_meas; out[2] = c.num_det;
  out[3] = c.num_obs; out[4] = c.num_gate_targets; out[5] = c.ops.size();
}

// Reference sample, one byte per measurement.  canonical != 0: every random
// result is 0; otherwise results come from coin_seed.
int oracle_reference(void *hv, int canonical, uint64_t coin_seed, uint8_t *out) {
  try {
    std::vector<uint8_t> r = reference(((Handle *)hv)->c, canonical != 0, coin_seed);
    std::memcpy(out, r.data(), r.size());
    return 0;
  } catch (const std::exception &e) {
    g_err = e.what();
    return -1;
  }
}

// Frame sampling of shots [shot_offset, shot_offset + num_shots), shot_offset a
// multiple of 64.  Outputs are [rows][W] u64 with W = ceil(num_shots / 64); bit
// j of word w is shot shot_offset + 64 w + j; bits past num_shots are 0.
// ref: one byte per measurement.  meas/det/obs may be null.
int oracle_sample(void *hv, const uint8_t *ref, uint64_t seed, uint64_t shot_offset, uint64_t num_shots,
                  uint64_t *meas, uint64_t *det, uint64_t *obs, int threads) {
  const Circuit &c = ((Handle *)hv)->c;
  if (shot_offset % 64 != 0 || num_shots == 0) { g_err = "bad shot range"; return -2; }
  uint64_t W = (num_shots + 63) / 64;
  std::vector<FrameRule> rules(NUM_GATES);
  for (int g = 0; g < NUM_GATES; g++)
    if (GATES[g].kind == K_CLIFFORD1 || GATES[g].kind == K_CLIFFORD2) rules[g] = frame_rule(g);
  std::vector<std::vector<uint64_t>> thr(c.ops.size());
  for (size_t i = 0; i < c.ops.size(); i++) {
    Kind k = GATES[c.ops[i].gate].kind;
    if ((k == K_NOISE1 || k == K_NOISE2) && c.ops[i].p > 0) {
      thr[i].resize(64);
      thresholds(c.ops[i].p, thr[i].data());
    }
  }
  std::vector<uint8_t> refv(ref, ref + c.num_meas);
#pragma omp parallel for schedule(dynamic, 1) num_threads(threads > 0 ? threads : 1)
  for (uint64_t w = 0; w < W; w++) {
    uint64_t word = shot_offset / 64 + w;
    uint64_t valid = num_shots - 64 * w;
    uint64_t tail = valid >= 64 ? ~0ull : ((1ull << valid) - 1);
    std::vector<uint64_t> flips;
    simulate_word(c, refv, rules, thr, seed, word, tail, flips);
    if (meas)
      for (uint64_t m = 0; m < c.num_meas; m++)
        meas[m * W + w] = (refv[m] ? ~flips[m] : flips[m]) & tail;
    // Detection event (Sec. 5.6): XOR of the detector's results, compared with
    // the XOR of the same reference bits (its noiseless value).
    if (det)
      for (uint64_t d = 0; d < c.num_det; d++) {
        uint64_t acc = 0, expect = 0;
        for (uint64_t mi : c.detectors[d]) {
          acc ^= (refv[mi] ? ~flips[mi] : flips[mi]) & tail;
          expect ^= refv[mi] ? tail : 0;
        }
        det[d * W + w] = acc ^ expect;
      }
    if (obs)
      for (uint64_t o = 0; o < c.num_obs; o++) {
        uint64_t acc = 0, expect = 0;
        for (uint64_t mi : c.observables[o]) {
          acc ^= (refv[mi] ? ~flips[mi] : flips[mi]) & tail;
          expect ^= refv[mi] ? tail : 0;
        }
        obs[o * W + w] = acc ^ expect;
      }
  }
  return 0;
}

// Error sets: *num_sets generators (see ErrorSets) and *num_entries lanes;
// off (num_sets + 1 entries) and lanes are filled when not null.
int oracle_error_sets(void *hv, uint64_t *num_sets, uint64_t *num_entries, uint64_t *off, uint32_t *lanes) {
  try {
    const ErrorSets &e = ((Handle *)hv)->error_sets_cached();
    *num_sets = e.off.size() - 1;
    *num_entries = e.lanes.size();
    if (off) std::memcpy(off, e.off.data(), e.off.size() * sizeof(uint64_t));
    if (lanes && !e.lanes.empty()) std::memcpy(lanes, e.lanes.data(), e.lanes.size() * sizeof(uint32_t));
    return 0;
  } catch (const std::exception &ex) {
    g_err = ex.what();
    return -1;
  }
}

// 1 when every detector and observable is deterministic, else 0.
int oracle_deterministic(void *hv) { return deterministic(((Handle *)hv)->c) ? 1 : 0; }

// Sparse detection-event sampling of shots [shot_offset, shot_offset +
// num_shots): det [D][W], obs [L][W] as in oracle_sample (either may be null).
// Fails (-3) when a detector or observable is not deterministic.
int oracle_sparse_detect(void *hv, uint64_t seed, uint64_t shot_offset, uint64_t num_shots, uint64_t *det,
                         uint64_t *obs, int threads) {
  Handle *h = (Handle *)hv;
  const Circuit &c = h->c;
  if (shot_offset % 64 != 0 || num_shots == 0) { g_err = "bad shot range"; return -2; }
  if (!deterministic(c)) { g_err = "a detector or observable is not deterministic"; return -3; }
  const ErrorSets &e = h->error_sets_cached();
  const uint64_t W = (num_shots + 63) / 64;
  if (det) std::memset(det, 0, c.num_det * W * sizeof(uint64_t));
  if (obs) std::memset(obs, 0, c.num_obs * W * sizeof(uint64_t));
  std::vector<std::vector<uint64_t>> thr(c.ops.size());
  for (size_t i = 0; i < c.ops.size(); i++)
    if (e.first[i] != ~0ull) {
      thr[i].resize(64);
      thresholds(c.ops[i].p, thr[i].data());
    }
#pragma omp parallel for schedule(dynamic, 1) num_threads(threads > 0 ? threads : 1)
  for (uint64_t w = 0; w < W; w++) {
    const uint64_t word = shot_offset / 64 + w;
    std::vector<std::pair<int, int>> hits;
    for (size_t i = 0; i < c.ops.size(); i++) {
      if (e.first[i] == ~0ull) continue;
      const Instr &ins = c.ops[i];
      const NoiseType nt = GATES[ins.gate].noise;
      const int k = nt == N_DEP2 ? 2 : 1;
      for (size_t s = 0; s < ins.q.size() / k; s++) {
        sample_hits(seed, i, s, word, thr[i].data(), nt == N_DEP1 ? 3 : nt == N_DEP2 ? 15 : 0, hits);
        for (auto &hit : hits) {
          if (64 * w + (uint64_t)hit.first >= num_shots) continue;   // past the last shot
          // Generator bits: X_a, Z_a, X_b, Z_b.
          int gens = 0;
          switch (nt) {
            case N_X: gens = 1; break;
            case N_Y: gens = 3; break;
            case N_Z: gens = 2; break;
            case N_DEP1: gens = hit.second == 0 ? 1 : hit.second == 1 ? 3 : 2; break;
            case N_DEP2: gens = hit.second + 1; break;
            default: break;
          }
          const uint64_t bit = 1ull << hit.first;
          for (int gbit = 0; gbit < 2 * k; gbit++) {
            if (!((gens >> gbit) & 1)) continue;
            const uint64_t gid = e.first[i] + s * 2 * k + gbit;
            for (uint64_t a = e.off[gid]; a < e.off[gid + 1]; a++) {
              const uint64_t lane = e.lanes[a];
              if (lane < c.num_det) {
                if (det) det[lane * W + w] ^= bit;
              } else if (obs) {
                obs[(lane - c.num_det) * W + w] ^= bit;
              }
            }
          }
        }
      }
    }
  }
  return 0;
}

// Absolute measurement indices of detector d / observable o.
uint64_t oracle_detector(void *hv, uint64_t d, uint64_t *out, uint64_t cap) {
  const Circuit &c = ((Handle *)hv)->c;
  const std::vector<uint64_t> &v = c.detectors[d];
  for (uint64_t k = 0; k < v.size() && k < cap; k++) out[k] = v[k];
  return v.size();
}

void oracle_philox(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4]) {
  philox(ctr, key[0], key[1], out);
}

uint64_t oracle_key_hi() { return KEY_HI; }

void oracle_thresholds(double p, uint64_t out[64]) { thresholds(p, out); }

uint64_t oracle_zrand(uint64_t seed, uint64_t instr, uint64_t slot, uint64_t word) {
  return zrand(seed, instr, slot, word);
}

// Hit positions/choices of one (instruction, slot, word) noise stream.
int oracle_hits(uint64_t seed, uint64_t instr, uint64_t slot, uint64_t word, double p, int K,
                int *pos, int *choice, int cap) {
  uint64_t t[64];
  thresholds(p, t);
  std::vector<std::pair<int, int>> hits;
  sample_hits(seed, instr, slot, word, t, K, hits);
  int n = (int)hits.size();
  for (int k = 0; k < n && k < cap; k++) { pos[k] = hits[k].first; choice[k] = hits[k].second; }
  return n;
}

// Gate table entry as text "NAME kind img0 img1 ... | inverse".
int oracle_gate(int index, char *out, size_t cap) {
  if (index < 0 || index >= NUM_GATES) return -1;
  const GateInfo &g = GATES[index];
  std::string s = g.name;
  s += " " + std::to_string((int)g.kind);
  int nimg = g.kind == K_CLIFFORD1 ? 2 : g.kind == K_CLIFFORD2 ? 4 : 0;
  for (int k = 0; k < nimg; k++) s += std::string(" ") + g.images[k];
  if (g.inverse) s += std::string(" | ") + g.inverse;
  std::snprintf(out, cap, "%s", s.c_str());
  return 0;
}

// Conjugates a Pauli (text, e.g. "+XY") by a Clifford gate's tableau over the
// same qubits, through the same routine the reference sampler uses to append
// operations.  Writes the image as text.
int oracle_conjugate(const char *gate, const char *pauli, char *out, size_t cap) {
  try {
    int gi = find_gate(upper(gate));
    if (gi < 0) return -1;
    SmallPauli p = parse_small(pauli);
    size_t k = p.x.size();
    // A one-column tableau over k qubits holding p; append the gate.
    Tableau t(k);
    Pauli col(k);
    col.sign = p.sign;
    for (size_t j = 0; j < k; j++) { col.setx(j, p.x[j]); col.setz(j, p.z[j]); }
    t.xs[0] = col;
    std::vector<uint32_t> qs;
    for (size_t j = 0; j < k; j++) qs.push_back((uint32_t)j);
    if (GATES[gi].kind == K_CLIFFORD1) {
      for (size_t j = 0; j < k; j++) t.append(gi, {(uint32_t)j});   // broadcast over qubits
    } else {
      t.append(gi, qs);
    }
    std::string s = t.xs[0].sign ? "-" : "+";
    for (size_t j = 0; j < k; j++) {
      int x = t.xs[0].getx(j), z = t.xs[0].getz(j);
      s += x && z ? 'Y' : x ? 'X' : z ? 'Z' : '_';
    }
    std::snprintf(out, cap, "%s", s.c_str());
    return 0;
  } catch (const std::exception &e) {
    g_err = e.what();
    return -1;
  }
}

// Start-of-time image of Z_q after folding the whole circuit into the inverse
// tableau (canonical resolution of random measurements), as text.
int oracle_z_image(void *hv, uint32_t q, char *out, size_t cap) {
  try {
    const Circuit &c = ((Handle *)hv)->c;
    Tableau t(c.num_qubits);
    std::vector<int> results;
    for (const Instr &ins : c.ops) {
      const GateInfo &g = GATES[ins.gate];
      if (g.kind == K_CLIFFORD1) for (uint32_t qq : ins.q) t.prepend(ins.gate, {qq});
      if (g.kind == K_CLIFFORD2)
        for (size_t k = 0; k < ins.q.size(); k += 2) {
          uint32_t fq;
          uint64_t fm;
          int pauli;
          if (controlled_pair(ins, k, fq, fm, pauli)) {
            if (results[fm]) t.prepend(find_gate(pauli_gate_name(pauli)), {fq});
          } else {
            t.prepend(ins.gate, {ins.q[k], ins.q[k + 1]});
          }
        }
      if (g.kind == K_MEASURE || g.kind == K_MEASURE_RESET || g.kind == K_RESET)
        for (uint32_t qq : ins.q) {
          int r = t.measure(qq, 0);
          if (g.kind != K_RESET) results.push_back(r);
          if (g.kind != K_MEASURE) t.zs[qq].sign = 0;
        }
    }
    std::string s = t.zs[q].sign ? "-" : "+";
    for (size_t j = 0; j < c.num_qubits; j++) {
      int x = t.zs[q].getx(j), z = t.zs[q].getz(j);
      s += x && z ? 'Y' : x ? 'X' : z ? 'Z' : '_';
    }
    std::snprintf(out, cap, "%s", s.c_str());
    return 0;
  } catch (const std::exception &e) {
    g_err = e.what();
    return -1;
  }
}

}  // extern "C"
