// Checks the bytewise prefix test of rng.h against a plain per-slot loop
// (host build of the device helpers; run by test_rng_host.py).
#include <cstdio>
#include <cstdint>
#include <random>
#include "rng.h"
using namespace stimgpu;
int main() {
  std::mt19937_64 g(1);
  long bad = 0;
  for (int it = 0; it < 2000000; it++) {
    U64x4 r; for (int i = 0; i < 4; i++) r.v[i] = g();
    if (it % 7 == 0) for (int i = 0; i < 4; i++) r.v[i] &= 0x8080808080808080ull ^ g();
    uint64_t cut = g() % 256; if (it % 11 == 0) cut = 0; if (it % 13 == 0) cut = 255;
    uint32_t lo = g() % 200, hi = lo + g() % 100; uint32_t grp = g() % 10;
    uint32_t want = 0;
    for (uint32_t b = 0; b < 32; b++) {
      uint32_t s = grp * 32 + b;
      uint64_t vp = (r.v[b >> 3] >> (8 * (b & 7))) & 0xFF;
      if (s >= lo && s < hi && vp >= cut) want |= 1u << b;
    }
    uint32_t got = prefix_pass_mask(r, cut) & group_slot_mask(grp, lo, hi);
    if (got != want) { if (bad < 5) printf("mismatch %x %x cut %lu\n", got, want, cut); bad++; }
  }
  printf("bad %ld\n", bad);
  return bad != 0;
}
