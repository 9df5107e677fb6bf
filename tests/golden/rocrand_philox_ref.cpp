// Reference Philox4x32-10 words from rocRAND's header-only engine (host build).
// Used by the oracle pin tests: prints, for each "seed subsequence offset"
// line on stdin, the four 32-bit words of the first next4() call.
#include <hip/hip_runtime.h>
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>

int main() {
  unsigned long long seed, sub, off;
  while (std::scanf("%llu %llu %llu", &seed, &sub, &off) == 3) {
    rocrand_device::philox4x32_10_engine e(seed, sub, off);
    uint4 v = e.next4();
    std::printf("%u %u %u %u\n", v.x, v.y, v.z, v.w);
  }
  return 0;
}
