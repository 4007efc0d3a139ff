// Test-only glue: prints Philox4x32-10 blocks computed by rocRAND's own
// philox4x32_10 engine (an implementation independent of the oracle), so the
// oracle's generator can be pinned against it bit for bit.
// Usage: philox_rocrand seed level  -> 128 words for ctr = (j, level, 0, 0),
// key = (seed lo, seed hi), j = 0..31, one per line.
#include <hip/hip_runtime.h>
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>
#include <cstdlib>

int main(int argc, char** argv) {
  if (argc != 3) return 2;
  unsigned long long seed = std::strtoull(argv[1], nullptr, 0);
  unsigned long long level = std::strtoull(argv[2], nullptr, 0);
  for (unsigned long long j = 0; j < 32; ++j) {
    // skipping 4*(j + level*2^32) numbers puts the 128-bit counter at
    // (j, level, 0, 0); done as four skips of j + level*2^32 to stay in 64 bits
    rocrand_device::philox4x32_10_engine eng(seed, 0, 0);
    const unsigned long long c = j + (level << 32);
    for (int t = 0; t < 4; ++t) eng.discard(c);
    uint4 r = eng.next4();
    std::printf("%u\n%u\n%u\n%u\n", r.x, r.y, r.z, r.w);
  }
  return 0;
}
