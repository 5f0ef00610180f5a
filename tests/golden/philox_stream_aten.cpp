// Test-only cross-check generator: prints words of the Philox4x32-10 stream
// of PyTorch's open-source ATen engine (ATen/core/PhiloxRNGEngine.h).
// stdin lines: seed subsequence offset_blocks count ; stdout: count hex words.
// The engine keys Philox with the seed, puts the subsequence in counter words
// 2..3 and the 128-bit block offset in counter words 0..1.
#include <ATen/core/PhiloxRNGEngine.h>
#include <cstdio>

int main() {
  unsigned long long seed, subseq, offset;
  long long count;
  while (std::scanf("%llu %llu %llu %lld", &seed, &subseq, &offset, &count) == 4) {
    at::Philox4_32 e(seed, subseq, offset);
    for (long long i = 0; i < count; ++i) std::printf("%08x\n", e());
  }
  return 0;
}
