// Test-only cross-check generator: prints words of the Philox4x32-10 stream
// of the open-source rocRAND device/host header (rocrand_philox4x32_10.h),
// run on the host.  stdin lines: seed subsequence offset_words count.
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>

int main() {
  unsigned long long seed, subseq, offset;
  long long count;
  while (std::scanf("%llu %llu %llu %lld", &seed, &subseq, &offset, &count) == 4) {
    rocrand_state_philox4x32_10 st;
    rocrand_init(seed, subseq, offset, &st);
    for (long long i = 0; i < count; ++i) std::printf("%08x\n", rocrand(&st));
  }
  return 0;
}
