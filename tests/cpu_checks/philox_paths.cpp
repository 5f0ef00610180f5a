// Host build of the library's two Philox paths (generic counter, and the
// point-major path with per-lane precomputed first rounds); prints the
// number of mismatching blocks over a seeded set of (seed, g, b) triples.
#include <cstdio>
#include <cstdint>
#include <random>

#include "zmc_device.hpp"

int main() {
  std::mt19937_64 rng(12345);
  long bad = 0, total = 0;
  for (int i = 0; i < 200000; ++i) {
    const uint64_t seed = rng();
    const uint32_t g = (uint32_t)rng();
    const uint32_t b = (i % 3 == 0) ? (uint32_t)(rng() % 4096) : (uint32_t)rng();
    const zmc::Words4 a = zmc::philox_block(b, g, seed);
    const zmc::Words4 c = zmc::philox_block_pm(b, zmc::philox_lane(g, seed));
    for (int k = 0; k < 4; ++k) bad += a.r[k] != c.r[k];
    ++total;
  }
  std::printf("%ld %ld\n", bad, total);
  return bad != 0;
}
