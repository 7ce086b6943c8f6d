// Canonical reference sample by inverse-tableau simulation (Sec. 4).
//
// The tableau T maps an observable at the current time to the equivalent
// observable at the start of time, where every qubit is |0>.  Folding a
// Clifford G prepends the tableau of G's inverse: T'(g) = T(G^dagger g G).  A
// Z measurement of qubit q reads column T(Z_q): without X/Y terms its result
// is the column's sign; otherwise the result is random and is resolved by
// inserting operations at the start of time ("appending"): CNOTs from a pivot
// onto the other X/Y terms, then H (X term) or H_YZ (Y term) on the pivot, and
// an X on the pivot when the sign must flip.  Every random measurement resolves
// to 0 here (the canonical reference; Sec. 3 makes any noiseless sample a
// valid reference).  A reset measures without reporting and then forces the
// column's sign to +.
//
// Storage is by columns (Sec. 5.1): for each of the 2n columns, n x bits and n
// z bits packed in 64-bit words, plus a sign.  Column c < n is T(X_c); column
// n + q is T(Z_q).
#include <cstring>
#include <utility>

#include "circuit.h"

namespace stimgpu {

namespace {

class InverseTableau {
 public:
  explicit InverseTableau(size_t n) : n_(n), nw_((n + 63) / 64), xb_(2 * n * nw_, 0), zb_(2 * n * nw_, 0),
                                      sign_(2 * n, 0) {
    for (size_t q = 0; q < n; q++) {
      xb_[q * nw_ + q / 64] |= 1ull << (q % 64);
      zb_[(n + q) * nw_ + q / 64] |= 1ull << (q % 64);
    }
  }

  // ---- prepends: T'(g) = T(G^dagger g G) for the generators g on G's qubits.
  void prepend(Gate g, uint32_t a, uint32_t b) {
    size_t Xa = a, Za = n_ + a, Xb = b, Zb = n_ + b;
    switch (g) {
      case G_I: break;
      case G_X: sign_[Za] ^= 1; break;
      case G_Y: sign_[Xa] ^= 1; sign_[Za] ^= 1; break;
      case G_Z: sign_[Xa] ^= 1; break;
      case G_H: swap_cols(Xa, Za); break;
      case G_S: mul_cols(Xa, Za, 3); break;                     // X -> -Y = -i X Z
      case G_S_DAG: mul_cols(Xa, Za, 1); break;                 // X -> +Y
      case G_SQRT_X: mul_cols(Za, Xa, 3); break;                // Z -> +Y = i X Z = -i Z X
      case G_SQRT_X_DAG: mul_cols(Za, Xa, 1); break;            // Z -> -Y
      case G_SQRT_Y: swap_cols(Xa, Za); sign_[Za] ^= 1; break;  // X -> Z, Z -> -X
      case G_SQRT_Y_DAG: swap_cols(Xa, Za); sign_[Xa] ^= 1; break;
      case G_H_XY: mul_cols(Xa, Za, 1); sign_[Za] ^= 1; break;  // X -> Y, Z -> -Z
      case G_H_YZ: mul_cols(Za, Xa, 3); sign_[Xa] ^= 1; break;  // Z -> Y, X -> -X
      case G_CX: mul_cols(Xa, Xb, 0); mul_cols(Zb, Za, 0); break;
      case G_CZ: mul_cols(Xa, Zb, 0); mul_cols(Xb, Za, 0); break;
      case G_CY:                                                 // X_a -> X_a Y_b
        mul_cols(Xa, Xb, 0); mul_cols(Xa, Zb, 1);
        mul_cols(Xb, Za, 0); mul_cols(Zb, Za, 0);
        break;
      case G_SWAP: swap_cols(Xa, Xb); swap_cols(Za, Zb); break;
      default: break;
    }
  }

  // Canonical Z measurement of qubit q (random results resolve to 0).
  int measure(uint32_t q) {
    size_t c = n_ + q;
    const uint64_t *cx = &xb_[c * nw_];
    size_t pivot = SIZE_MAX;
    for (size_t w = 0; w < nw_ && pivot == SIZE_MAX; w++)
      if (cx[w]) pivot = w * 64 + (size_t)__builtin_ctzll(cx[w]);
    if (pivot == SIZE_MAX) return sign_[c];
    // Collect the other X/Y terms first (appends change the column).
    std::vector<uint32_t> others;
    for (size_t w = pivot / 64; w < nw_; w++) {
      uint64_t v = cx[w];
      if (w == pivot / 64) v &= ~(1ull << (pivot % 64)) & (~0ull << (pivot % 64));
      while (v) {
        others.push_back((uint32_t)(w * 64 + (size_t)__builtin_ctzll(v)));
        v &= v - 1;
      }
    }
    for (uint32_t t : others) append_cx((uint32_t)pivot, t);
    if (bit(zb_, c, pivot)) append_h_yz((uint32_t)pivot);
    else append_h((uint32_t)pivot);
    if (sign_[c]) append_x((uint32_t)pivot);
    return 0;
  }

  void force_zero(uint32_t q) { sign_[n_ + q] = 0; }

 private:
  size_t n_, nw_;
  std::vector<uint64_t> xb_, zb_;
  std::vector<uint8_t> sign_;

  uint64_t bit(const std::vector<uint64_t> &v, size_t col, size_t q) const {
    return (v[col * nw_ + q / 64] >> (q % 64)) & 1;
  }

  void swap_cols(size_t a, size_t b) {
    std::swap_ranges(&xb_[a * nw_], &xb_[a * nw_] + nw_, &xb_[b * nw_]);
    std::swap_ranges(&zb_[a * nw_], &zb_[a * nw_] + nw_, &zb_[b * nw_]);
    std::swap(sign_[a], sign_[b]);
  }

  // Column dst <- i^e * dst * src.  For single-qubit Hermitian Paulis written
  // as P = i^(x z) X^x Z^z, P1 P2 = i^(x1 z1 + x2 z2 + 2 z1 x2 - x3 z3) P3 with
  // x3 = x1 ^ x2, z3 = z1 ^ z2; summing the exponent over all qubits gives the
  // phase of the product, which must be real here.
  void mul_cols(size_t dst, size_t src, int e) {
    uint64_t *x1 = &xb_[dst * nw_], *z1 = &zb_[dst * nw_];
    const uint64_t *x2 = &xb_[src * nw_], *z2 = &zb_[src * nw_];
    int64_t acc = e;
    for (size_t w = 0; w < nw_; w++) {
      uint64_t a = x1[w], b = z1[w], c = x2[w], d = z2[w];
      uint64_t x3 = a ^ c, z3 = b ^ d;
      acc += __builtin_popcountll(a & b) + __builtin_popcountll(c & d) + 2 * __builtin_popcountll(b & c) -
             __builtin_popcountll(x3 & z3);
      x1[w] = x3;
      z1[w] = z3;
    }
    sign_[dst] ^= sign_[src] ^ (uint8_t)((acc >> 1) & 1);
  }

  // ---- appends: every column P becomes B P B for a self-inverse B inserted
  // at the start of time.
  void append_cx(uint32_t c, uint32_t t) {
    size_t wc = c / 64, wt = t / 64;
    int bc = c % 64, bt = t % 64;
    for (size_t col = 0; col < 2 * n_; col++) {
      uint64_t *X = &xb_[col * nw_], *Z = &zb_[col * nw_];
      uint64_t xc = (X[wc] >> bc) & 1, zc = (Z[wc] >> bc) & 1;
      uint64_t xt = (X[wt] >> bt) & 1, zt = (Z[wt] >> bt) & 1;
      sign_[col] ^= (uint8_t)(xc & zt & (xt ^ zc ^ 1));
      X[wt] ^= xc << bt;
      Z[wc] ^= zt << bc;
    }
  }

  void append_h(uint32_t q) {
    size_t w = q / 64;
    int b = q % 64;
    for (size_t col = 0; col < 2 * n_; col++) {
      uint64_t *X = &xb_[col * nw_ + w], *Z = &zb_[col * nw_ + w];
      uint64_t x = (*X >> b) & 1, z = (*Z >> b) & 1;
      sign_[col] ^= (uint8_t)(x & z);
      *X ^= (x ^ z) << b;
      *Z ^= (x ^ z) << b;
    }
  }

  void append_h_yz(uint32_t q) {   // X -> -X, Y -> Z, Z -> Y
    size_t w = q / 64;
    int b = q % 64;
    for (size_t col = 0; col < 2 * n_; col++) {
      uint64_t *X = &xb_[col * nw_ + w], *Z = &zb_[col * nw_ + w];
      uint64_t x = (*X >> b) & 1, z = (*Z >> b) & 1;
      sign_[col] ^= (uint8_t)(x & (z ^ 1));
      *X ^= z << b;
    }
  }

  void append_x(uint32_t q) {
    size_t w = q / 64;
    int b = q % 64;
    for (size_t col = 0; col < 2 * n_; col++) sign_[col] ^= (uint8_t)((zb_[col * nw_ + w] >> b) & 1);
  }
};

struct RefRun {
  InverseTableau t;
  std::vector<uint64_t> bits;
  uint64_t m = 0;

  void run(const std::vector<Node> &nodes) {
    for (const Node &n : nodes) {
      if (n.repeat) {
        for (uint64_t r = 0; r < n.reps; r++) run(n.body);
        continue;
      }
      if (gate_is_clifford(n.gate)) {
        if (gate_is_two_qubit(n.gate)) {
          for (size_t k = 0; k < n.targets.size(); k += 2) {
            uint32_t a = n.targets[k], b = n.targets[k + 1];
            if ((a | b) & TGT_REC) {
              // Classically controlled Pauli: applied when the reference's
              // own result is 1.
              if (a & TGT_REC) std::swap(a, b);
              const uint64_t mi = m - (b & ~TGT_REC);
              if ((bits[mi / 64] >> (mi % 64)) & 1)
                t.prepend(n.gate == G_CX ? G_X : n.gate == G_CY ? G_Y : G_Z, a, a);
              continue;
            }
            t.prepend(n.gate, a, b);
          }
        } else {
          for (uint32_t q : n.targets) t.prepend(n.gate, q, q);
        }
      } else if (n.gate == G_M || n.gate == G_MR || n.gate == G_R) {
        for (uint32_t q : n.targets) {
          int r = t.measure(q);
          if (n.gate != G_R) {
            if (r) bits[m / 64] |= 1ull << (m % 64);
            m++;
          }
          if (n.gate != G_M) t.force_zero(q);
        }
      }
    }
  }
};

}  // namespace

std::vector<uint64_t> reference_sample(const std::vector<Node> &tree, uint64_t num_qubits,
                                       uint64_t num_measurements) {
  RefRun r{InverseTableau(num_qubits), std::vector<uint64_t>((num_measurements + 63) / 64, 0), 0};
  r.run(tree);
  return r.bits;
}

}  // namespace stimgpu
